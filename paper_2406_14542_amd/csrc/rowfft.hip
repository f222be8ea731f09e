// Row transforms of the fine grid (the phi direction of N's 2-D FFT, arXiv:2406.14542
// Sec. III) for row lengths n2 = 2 N with N = 2^K or 5 2^K, one workgroup per window row:
//   C2R  x[n] = sum_{k=0}^{n2-1} X[k] e^{+2 pi i k n / n2},  X[n2 - k] = conj X[k],
//        X[k] = 0 for M < k < n2 - M (the band limit), Im X[0] ignored;
//   R2C  X[k] = sum_n x[n] e^{-2 pi i k n / n2}, k = 0 .. M only.
// Both take the half-length route: with N = n2 / 2 and z[n] = x[2n] + i x[2n+1],
//   z = IDFT_N(Z),  Z[k] = E[k] + i O[k],  E[k] = X[k] + X[k + N],
//   O[k] = (X[k] - X[k + N]) e^{2 pi i k / n2},  X[k + N] = conj X[N - k];
// and backwards E = (Z[k] + conj Z[N-k]) / 2, O = (Z[k] - conj Z[N-k]) / (2i),
//   X[k] = E + e^{-2 pi i k / n2} O.
// The theta pass of the same 2-D FFT (n1 = 2^K or 5 2^K, one workgroup per band column mu of
// one map) runs here as well, fused with the deconvolution of N(i) / N^H(iii):
//   synthesis  band[mu][i] = sum_{|k| <= L} C[k][mu] h(k, mu) e^{+2 pi i k i / n1}, window rows i
//   adjoint    C[k][mu] = h(k, mu) sum_{window rows i} band[mu][i] e^{-2 pi i k i / n1}, |k| <= L
// (h = the deconvolution factors d1[|k|] d2[mu]; k of entry t of the length-N_t torus column is
// t or t - N_t): the column is read once from the torus spectrum (synthesis: only its |k| <= L
// entries exist, the padding is zeros in registers) or from the window rows of the band
// (adjoint), transformed in LDS, and written once, so the zero-padded spectrum is never
// stored and no separate deconvolution pass reads or writes it.
// The N-point transform runs in LDS as Stockham radix passes (N = 2^K: a first pass of radix
// 2^(K mod 4) when needed, then radix 16; N = 5 2^K: radix 5, then 2^(K mod 4), then radix
// 16), reading the row straight from HBM in the first pass and writing it in the last: one
// read and one write of each row, and only the M + 1 band columns of the spectrum are read
// (C2R) or written (R2C).
#include "internal.h"

namespace nusht {
namespace {

template <typename T>
struct Cx;
template <>
struct Cx<float> {
    using type = float2;
};
template <>
struct Cx<double> {
    using type = double2;
};

template <typename C>
__device__ inline C cmk(decltype(C::x) re, decltype(C::x) im)
{
    C r;
    r.x = re;
    r.y = im;
    return r;
}
template <typename C>
__device__ inline C cadd(C a, C b)
{
    return cmk<C>(a.x + b.x, a.y + b.y);
}
template <typename C>
__device__ inline C csub(C a, C b)
{
    return cmk<C>(a.x - b.x, a.y - b.y);
}
template <typename C>
__device__ inline C cmul(C a, C b)
{
    return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * (DIR i)
template <int DIR, typename C>
__device__ inline C cmul_i(C a)
{
    return DIR > 0 ? cmk<C>(-a.y, a.x) : cmk<C>(a.y, -a.x);
}

// cos and sin of 2 pi e / 16
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kSin16[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// a * e^{DIR 2 pi i e / 16}; e is a constant once the callers' loops are unrolled, so the
// branches and the table lookups fold away
template <int DIR, typename C>
__device__ __forceinline__ C rot16(C a, int e)
{
    using T = decltype(C::x);
    e &= 15;
    if (e == 0) return a;
    if (e == 4) return cmul_i<DIR>(a);
    if (e == 8) return cmk<C>(-a.x, -a.y);
    if (e == 12) return cmul_i<-DIR>(a);
    return cmul(a, cmk<C>((T)kCos16[e], (T)(DIR * kSin16[e])));
}

// in-place DFT of R = 1, 2, 4, 5, 8 or 16 values, natural order in and out:
// V[k] = sum_n v[n] e^{DIR 2 pi i n k / R}
template <int R, int DIR, typename C>
__device__ inline void dft(C (&v)[R])
{
    if constexpr (R == 2) {
        const C a = v[0];
        v[0] = cadd(a, v[1]);
        v[1] = csub(a, v[1]);
    } else if constexpr (R == 4) {
        const C a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        const C a2 = cadd(v[1], v[3]), a3 = cmul_i<DIR>(csub(v[1], v[3]));
        v[0] = cadd(a0, a2);
        v[2] = csub(a0, a2);
        v[1] = cadd(a1, a3);
        v[3] = csub(a1, a3);
    } else if constexpr (R == 5) {
        // V[k] = sum_n v[n] w^(n k), w = e^{DIR 2 pi i / 5}: pairs (1, 4) and (2, 3) share
        // cos(2 pi / 5), cos(4 pi / 5) and sin(2 pi / 5), sin(4 pi / 5)
        using T = decltype(C::x);
        const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
        const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
        const C t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
        const C t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
        const C a1 = cmk<C>(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
        const C a2 = cmk<C>(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
        const C b1 = cmul_i<DIR>(cmk<C>(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
        const C b2 = cmul_i<DIR>(cmk<C>(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
        v[0] = cadd(v[0], cadd(t1, t2));
        v[1] = cadd(a1, b1);
        v[4] = csub(a1, b1);
        v[2] = cadd(a2, b2);
        v[3] = csub(a2, b2);
    } else if constexpr (R == 8 || R == 16) {
        // R = 4 Q: n = Q n1 + n2, k = k1 + 4 k2; DFT_4 over n1, twiddle e^{DIR 2 pi i n2 k1 / R},
        // DFT_Q over n2
        constexpr int Q = R / 4;
        C u[4][Q];
#pragma unroll
        for (int n2 = 0; n2 < Q; ++n2) {
            C w[4] = {v[n2], v[Q + n2], v[2 * Q + n2], v[3 * Q + n2]};
            dft<4, DIR>(w);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) u[k1][n2] = rot16<DIR>(w[k1], n2 * k1 * (16 / R));
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            dft<Q, DIR>(u[k1]);
#pragma unroll
            for (int k2 = 0; k2 < Q; ++k2) v[k1 + 4 * k2] = u[k1][k2];
        }
    }
}

// LDS index with one pad slot per 16 entries (stride-16 accesses stay off one bank)
__device__ inline int pad16(int i) { return i + (i >> 4); }

// Transform length N = F 2^K, F = 1 or 5.  Passes: radix R0 (from HBM), for F = 5 a radix
// R1 = 2^(K mod 4) pass when K mod 4 > 0, then NPASS16 radix-16 passes (the last one to HBM).
template <int K, int F = 1>
struct RowShape {
    static_assert(F == 1 || F == 5, "length 2^K or 5 2^K");
    static constexpr int N = F << K;                          // complex points
    static constexpr int NB16 = N / 16;                       // radix-16 butterflies per pass
    static constexpr int NT = NB16 < 64 ? 64 : NB16;          // threads
    static constexpr int R0 = F == 5 ? 5 : ((K % 4) ? (1 << (K % 4)) : 16);  // first pass radix
    static constexpr int R1 = (F == 5 && (K % 4)) ? (1 << (K % 4)) : 1;      // second (1: none)
    static constexpr int NPASS16 = F == 5 ? K / 4 : ((K % 4) ? K / 4 : K / 4 - 1);
};

// One Stockham pass (radix R, span Ns) over LDS, in place: every thread loads the inputs of
// its butterflies, the block synchronises, then the outputs are written.
//   butterfly idx: inputs in[idx + r N / R], twiddle e^{DIR 2 pi i j r / (Ns R)} (j = idx mod
//   Ns), DFT_R, outputs out[(idx - j) R + j + r Ns].
// tw[m] = e^{2 pi i m / n2} (n2 = 2 N), so e^{2 pi i a / N} = tw[2 a].
// The twiddles of a butterfly are fetched (global loads, L2-resident table) before the
// pass's LDS reads and barrier, so that their latency overlaps the wait.  A radix-16
// butterfly loads w, w^2, w^4 and w^8 and forms the other powers by at most three complex
// products (the table loads, not the arithmetic, set the time of these passes).
template <int R, int DIR, typename C>
__device__ inline void load_twiddles(C (&w)[R], int j, int Ns, int N, const C* __restrict__ tw)
{
    const int step = 2 * j * (N / (Ns * R));
    if constexpr (R == 16) {
        w[1] = tw[step];
        w[2] = tw[2 * step];
        w[4] = tw[4 * step];
        w[8] = tw[8 * step];
        w[3] = cmul(w[1], w[2]);
        w[5] = cmul(w[4], w[1]);
        w[6] = cmul(w[4], w[2]);
        w[7] = cmul(w[4], w[3]);
#pragma unroll
        for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
    } else {
#pragma unroll
        for (int r = 1; r < R; ++r) w[r] = tw[r * step];
    }
    if (DIR < 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) w[r].y = -w[r].y;
    }
}

// tw[k] read through the constant address space: for a wave-uniform k this is a scalar load
template <typename T>
__device__ inline typename Cx<T>::type tw_uniform(const typename Cx<T>::type* tw, int k)
{
    const __attribute__((address_space(4))) T* p = (const __attribute__((address_space(4))) T*)tw;
    return cmk<typename Cx<T>::type>(p[2 * k], p[2 * k + 1]);
}

template <int R, typename C>
__device__ inline void apply_twiddles(C (&v)[R], const C (&w)[R])
{
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
}

// One in-LDS Stockham pass of radix R and span Ns with N / R butterflies spread over the
// threads (several per thread): the radix-R1 pass of 5 2^K lengths.
template <int R, int DIR, int N, int NT, typename C>
__device__ inline void lds_pass(C* buf, int t, int Ns, const C* __restrict__ tw)
{
    constexpr int NB = N / R;
    constexpr int NBT = (NB + NT - 1) / NT;
    C v[NBT][R], w[NBT][R];
#pragma unroll
    for (int q = 0; q < NBT; ++q) {
        const int b = t + q * NT;
        if (b < NB) {
            load_twiddles<R, DIR>(w[q], b % Ns, Ns, N, tw);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[pad16(b + r * NB)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NBT; ++q) {
        const int b = t + q * NT;
        if (b < NB) {
            apply_twiddles(v[q], w[q]);
            dft<R, DIR>(v[q]);
            const int j = b % Ns;
            const int base = (b - j) * R + j;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[pad16(base + r * Ns)] = v[q][r];
        }
    }
    __syncthreads();
}

template <int K, int DIR, int F = 1, typename C>
__device__ inline void middle_passes(C* buf, int t, const C* __restrict__ tw)
{
    using S = RowShape<K, F>;
    constexpr int N = S::N;
    constexpr int NS0 = S::R0 * S::R1;  // span of the first radix-16 pass
    if constexpr (S::R1 > 1) lds_pass<S::R1, DIR, N, S::NT>(buf, t, S::R0, tw);
    const bool act = t < S::NB16;
#pragma unroll
    for (int p = 0; p < S::NPASS16 - 1; ++p) {
        int Ns = NS0;
        for (int e = 0; e < p; ++e) Ns *= 16;
        const int j = t % Ns;
        C v[16], w[16];
        if (act) {
            load_twiddles<16, DIR>(w, j, Ns, N, tw);
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = buf[pad16(t + r * (N / 16))];
        }
        __syncthreads();
        if (act) {
            apply_twiddles(v, w);
            dft<16, DIR>(v);
            const int base = (t - j) * 16 + j;
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[pad16(base + r * Ns)] = v[r];
        }
        __syncthreads();
    }
}

// C2R of window rows: blockIdx.x = compact window row q, fine row i = q for q < ra, else
// n1 - rb + (q - ra).  rows: [i][rw] spectrum columns 0 .. ncol-1 (ncol = M + 1 <= N);
// fine: real [n1][n2].
template <typename T, int K, int F>
__global__ __launch_bounds__((RowShape<K, F>::NT)) void k_row_c2r(
    const typename Cx<T>::type* __restrict__ rows, int64_t rw, int ncol,
    T* __restrict__ fine, int n1, int ra, int rb, const typename Cx<T>::type* __restrict__ tw)
{
    using C = typename Cx<T>::type;
    using S = RowShape<K, F>;
    constexpr int N = S::N, R0 = S::R0;
    __shared__ C buf[N + N / 16];
    const int q = blockIdx.x, t = threadIdx.x;
    const int i = q < ra ? q : n1 - rb + (q - ra);
    const C* X = rows + (int64_t)i * rw;
    const int M = ncol - 1;
    // first pass (span 1) from HBM: Z[k] built from X[k] and X[N - k].  All of the thread's
    // loads are issued first, then the butterflies are formed; only band columns are loaded
    // (a wave's k lie on one side of the band edge but for one wave, so whole load
    // instructions drop out: 5 % of the fine-FFT stage at lmax 4095).
    constexpr int NU = (N / R0 + S::NT - 1) / S::NT;
    // split twiddles e^{2 pi i k / n2}, k = t + u NT + r N / R0: the thread's tw[t] times a
    // wave-uniform factor
    const C wt = tw[t];
    C xa[NU][R0], xb[NU][R0];
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = t + u * S::NT + r * (N / R0);
            xa[u][r] = k <= M ? X[k] : cmk<C>(0, 0);
            // k < N: threads past the last butterfly (idx >= N / R0) would index below the row
            xb[u][r] = (k > 0 && k < N && N - k <= M) ? X[N - k] : cmk<C>(0, 0);
        }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int idx = t + u * S::NT;
        if (idx < N / R0) {
            C v[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int k = idx + r * (N / R0);
                C xk = k <= M ? xa[u][r] : cmk<C>(0, 0);
                if (k == 0) xk.y = 0;
                const C xm = (k > 0 && N - k <= M) ? xb[u][r] : cmk<C>(0, 0);
                const C xc = cmk<C>(xm.x, -xm.y);
                const C e = cadd(xk, xc);
                const C o = cmul(csub(xk, xc),
                                 cmul(wt, tw_uniform<T>(tw, u * S::NT + r * (N / R0))));
                v[r] = cmk<C>(e.x - o.y, e.y + o.x);
            }
            dft<R0, +1>(v);
#pragma unroll
            for (int r = 0; r < R0; ++r) buf[pad16(idx * R0 + r)] = v[r];
        }
    }
    __syncthreads();
    middle_passes<K, +1, F>(buf, t, tw);
    // last pass (radix 16, span N / 16) into the fine row: z[n] = x[2n] + i x[2n+1]
    if (t < S::NB16) {
        C v[16], w[16];
        load_twiddles<16, +1>(w, t, N / 16, N, tw);
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = buf[pad16(t + r * (N / 16))];
        apply_twiddles(v, w);
        dft<16, +1>(v);
        C* z = reinterpret_cast<C*>(fine + (int64_t)i * (2 * N));
#pragma unroll
        for (int r = 0; r < 16; ++r) z[t + r * (N / 16)] = v[r];
    }
}

// R2C of window rows, columns 0 .. ncol-1 of each row's spectrum into rows[i][.]
template <typename T, int K, int F>
__global__ __launch_bounds__((RowShape<K, F>::NT)) void k_row_r2c(
    const T* __restrict__ fine, int n1, int ra, int rb, typename Cx<T>::type* __restrict__ rows,
    int64_t rw, int ncol, const typename Cx<T>::type* __restrict__ tw)
{
    using C = typename Cx<T>::type;
    using S = RowShape<K, F>;
    constexpr int N = S::N, R0 = S::R0;
    __shared__ C buf[N + N / 16];
    const int q = blockIdx.x, t = threadIdx.x;
    const int i = q < ra ? q : n1 - rb + (q - ra);
    const C* z = reinterpret_cast<const C*>(fine + (int64_t)i * (2 * N));
    constexpr int NU = (N / R0 + S::NT - 1) / S::NT;
    C za[NU][R0];
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int r = 0; r < R0; ++r) za[u][r] = z[min(t + u * S::NT + r * (N / R0), N - 1)];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int idx = t + u * S::NT;
        if (idx < N / R0) {
            dft<R0, -1>(za[u]);
#pragma unroll
            for (int r = 0; r < R0; ++r) buf[pad16(idx * R0 + r)] = za[u][r];
        }
    }
    __syncthreads();
    middle_passes<K, -1, F>(buf, t, tw);
    {
        C v[16], w[16];
        const bool act = t < S::NB16;
        if (act) {
            load_twiddles<16, -1>(w, t, N / 16, N, tw);
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = buf[pad16(t + r * (N / 16))];
            apply_twiddles(v, w);
            dft<16, -1>(v);
        }
        __syncthreads();  // every thread has read its inputs
        if (act) {
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[pad16(t + r * (N / 16))] = v[r];
        }
        __syncthreads();
    }
    C* X = rows + (int64_t)i * rw;
    const C wt = tw[t];  // e^{-2 pi i k / n2} = conj(tw[t] tw[k - t]), k - t wave-uniform
    for (int k = t; k < ncol; k += S::NT) {
        const C zk = buf[pad16(k)];
        const C zm = buf[pad16(k == 0 ? 0 : N - k)];
        const C e = cmk<C>((zk.x + zm.x) / 2, (zk.y - zm.y) / 2);
        // O = (Z[k] - conj Z[N-k]) / (2 i)
        const C d = cmk<C>((zk.x - zm.x) / 2, (zk.y + zm.y) / 2);
        const C o = cmk<C>(d.y, -d.x);
        C w = cmul(wt, tw_uniform<T>(tw, k - t));
        w.y = -w.y;
        X[k] = cadd(e, cmul(o, w));
    }
}


// ---- theta pass (band columns, complex, length n1 = 2^K) ----------------------------------

__device__ inline int kappa_of(int i, int n) { return i <= n / 2 ? i : i - n; }

// synthesis: torus spectrum cs[b][mu][t] (t < nt) -> band[b][mu][i], window rows only
template <typename T, int K, int F>
__global__ __launch_bounds__((RowShape<K, F>::NT)) void k_theta_inv(
    const typename Cx<T>::type* __restrict__ cs, typename Cx<T>::type* __restrict__ band, int nt,
    int lmax, int mmax, const T* __restrict__ d1, const T* __restrict__ d2, int ra, int rb,
    const typename Cx<T>::type* __restrict__ tw)
{
    using C = typename Cx<T>::type;
    using S = RowShape<K, F>;
    constexpr int N = S::N, R0 = S::R0;
    __shared__ C buf[N + N / 16];
    const int mu = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
    const int64_t col = (int64_t)b * (mmax + 1) + mu;
    const C* src = cs + col * nt;
    C* dst = band + col * N;
    const T fm = d2[mu];
    // first pass (span 1) from the torus column: entry i of the padded column has wave number
    // k = kappa_of(i, N); only |k| <= L is loaded (the rest of the column is zero)
    constexpr int NU = (N / R0 + S::NT - 1) / S::NT;
    C x[NU][R0];
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int i = t + u * S::NT + r * (N / R0);
            const int k = kappa_of(i, N);
            const int ak = k < 0 ? -k : k;
            C v = cmk<C>(0, 0);
            if (i < N && ak <= lmax) {
                const C c = src[k < 0 ? k + nt : k];
                const T f = d1[ak] * fm;
                v = cmk<C>(c.x * f, c.y * f);
            }
            x[u][r] = v;
        }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int idx = t + u * S::NT;
        if (idx < N / R0) {
            dft<R0, +1>(x[u]);
#pragma unroll
            for (int r = 0; r < R0; ++r) buf[pad16(idx * R0 + r)] = x[u][r];
        }
    }
    __syncthreads();
    middle_passes<K, +1, F>(buf, t, tw);
    // last pass (radix 16, span N / 16) straight into the band column's window rows
    if (t < S::NB16) {
        C v[16], w[16];
        load_twiddles<16, +1>(w, t, N / 16, N, tw);
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = buf[pad16(t + r * (N / 16))];
        apply_twiddles(v, w);
        dft<16, +1>(v);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = t + r * (N / 16);
            if (i < ra || i >= N - rb) dst[i] = v[r];
        }
    }
}

// adjoint: band[b][mu][i] (window rows; the others are taken as zero) -> torus spectrum
// cs[b][mu][t], deconvolved, zero for |k| > L
template <typename T, int K, int F>
__global__ __launch_bounds__((RowShape<K, F>::NT)) void k_theta_fwd(
    const typename Cx<T>::type* __restrict__ band, typename Cx<T>::type* __restrict__ cs, int nt,
    int lmax, int mmax, const T* __restrict__ d1, const T* __restrict__ d2, int ra, int rb,
    const typename Cx<T>::type* __restrict__ tw)
{
    using C = typename Cx<T>::type;
    using S = RowShape<K, F>;
    constexpr int N = S::N, R0 = S::R0;
    __shared__ C buf[N + N / 16];
    const int mu = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
    const int64_t col = (int64_t)b * (mmax + 1) + mu;
    const C* src = band + col * N;
    C* dst = cs + col * nt;
    const T fm = d2[mu];
    constexpr int NU = (N / R0 + S::NT - 1) / S::NT;
    C x[NU][R0];
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int i = t + u * S::NT + r * (N / R0);
            x[u][r] = (i < N && (i < ra || i >= N - rb)) ? src[i] : cmk<C>(0, 0);
        }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int idx = t + u * S::NT;
        if (idx < N / R0) {
            dft<R0, -1>(x[u]);
#pragma unroll
            for (int r = 0; r < R0; ++r) buf[pad16(idx * R0 + r)] = x[u][r];
        }
    }
    __syncthreads();
    middle_passes<K, -1, F>(buf, t, tw);
    if (t < S::NB16) {
        C v[16], w[16];
        load_twiddles<16, -1>(w, t, N / 16, N, tw);
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = buf[pad16(t + r * (N / 16))];
        apply_twiddles(v, w);
        dft<16, -1>(v);
        // output i carries wave number k = kappa_of(i, N); |k| <= L lands at torus entry t(k)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = t + r * (N / 16);
            const int k = kappa_of(i, N);
            const int ak = k < 0 ? -k : k;
            if (ak <= lmax) {
                const T f = d1[ak] * fm;
                dst[k < 0 ? k + nt : k] = cmk<C>(v[r].x * f, v[r].y * f);
            }
        }
    }
    // torus entries beyond the band limit
    for (int e = t; e < nt; e += S::NT) {
        const int k = kappa_of(e, nt);
        if ((k < 0 ? -k : k) > lmax) dst[e] = cmk<C>(0, 0);
    }
}

// Long columns (16384 FP64 values, 256 KB as complex numbers): the column lives in registers,
// 32 values per thread (two radix-16 butterflies, or 32 / R0 first-pass butterflies), and only
// the exchange between two passes goes through LDS -- the real parts, then the imaginary
// parts, through one array of N reals, half the LDS of a complex column.
template <int K>
struct ThetaHalf {
    static constexpr int N = 1 << K;
    static constexpr int NT = N / 32;
    static constexpr int R0 = RowShape<K>::R0;
    static constexpr int NP16 = RowShape<K>::NPASS16;
};

// one Stockham pass of radix R and span ns on the thread's butterflies idx = t + q NT
template <int R, int DIR, int N, int NT, typename C>
__device__ inline void pass_in_regs(C (&v)[32], int t, int ns, const C* __restrict__ tw)
{
#pragma unroll
    for (int q = 0; q < 32 / R; ++q) {
        C u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[q * R + r];
        if (ns > 1) {
            C w[R];
            load_twiddles<R, DIR>(w, (t + q * NT) & (ns - 1), ns, N, tw);
            apply_twiddles(u, w);
        }
        dft<R, DIR>(u);
#pragma unroll
        for (int r = 0; r < R; ++r) v[q * R + r] = u[r];
    }
}

// part P (0 real, 1 imaginary) of the exchange between a pass of radix RP and span nsp (its
// outputs at (idx - j) RP + j + r nsp) and a pass of radix RN (inputs at idx + r N / RN)
template <int P, int RP, int RN, int N, int NT, typename T, typename C>
__device__ inline void exchange_part(T* lds, C (&v)[32], int t, int nsp)
{
#pragma unroll
    for (int q = 0; q < 32 / RP; ++q) {
        const int idx = t + q * NT;
        const int j = idx & (nsp - 1);
        const int base = (idx - j) * RP + j;
#pragma unroll
        for (int r = 0; r < RP; ++r) lds[pad16(base + r * nsp)] = P ? v[q * RP + r].y : v[q * RP + r].x;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 32 / RN; ++q) {
        const int idx = t + q * NT;
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const T x = lds[pad16(idx + r * (N / RN))];
            if (P)
                v[q * RN + r].y = x;
            else
                v[q * RN + r].x = x;
        }
    }
    __syncthreads();
}

template <int RP, int RN, int N, int NT, typename T, typename C>
__device__ inline void exchange(T* lds, C (&v)[32], int t, int nsp)
{
    exchange_part<0, RP, RN, N, NT>(lds, v, t, nsp);
    exchange_part<1, RP, RN, N, NT>(lds, v, t, nsp);
}

// the passes after the first: radix 16, span R0 16^p; the outputs of the last one are in
// natural order at idx + r N / 16
template <int K, int DIR, typename T, typename C>
__device__ inline void passes_after_first(T* lds, C (&v)[32], int t, const C* __restrict__ tw)
{
    using S = ThetaHalf<K>;
    exchange<S::R0, 16, S::N, S::NT>(lds, v, t, 1);
    int ns = S::R0;
#pragma unroll
    for (int p = 0; p < S::NP16; ++p) {
        pass_in_regs<16, DIR, S::N, S::NT>(v, t, ns, tw);
        if (p < S::NP16 - 1) exchange<16, 16, S::N, S::NT>(lds, v, t, ns);
        ns *= 16;
    }
}

template <typename T, int K>
__global__ __launch_bounds__(ThetaHalf<K>::NT) void k_theta_inv_h(
    const typename Cx<T>::type* __restrict__ cs, typename Cx<T>::type* __restrict__ band, int nt,
    int lmax, int mmax, const T* __restrict__ d1, const T* __restrict__ d2, int ra, int rb,
    const typename Cx<T>::type* __restrict__ tw)
{
    using C = typename Cx<T>::type;
    using S = ThetaHalf<K>;
    constexpr int N = S::N, R0 = S::R0, NT = S::NT;
    __shared__ T lds[N + N / 16];
    const int mu = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
    const int64_t col = (int64_t)b * (mmax + 1) + mu;
    const C* src = cs + col * nt;
    C* dst = band + col * N;
    const T fm = d2[mu];
    C v[32];
#pragma unroll
    for (int q = 0; q < 32 / R0; ++q)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int i = t + q * NT + r * (N / R0);
            const int k = kappa_of(i, N);
            const int ak = k < 0 ? -k : k;
            C x = cmk<C>(0, 0);
            if (ak <= lmax) {
                const C c = src[k < 0 ? k + nt : k];
                const T f = d1[ak] * fm;
                x = cmk<C>(c.x * f, c.y * f);
            }
            v[q * R0 + r] = x;
        }
    pass_in_regs<R0, +1, N, NT>(v, t, 1, tw);
    passes_after_first<K, +1>(lds, v, t, tw);
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = t + q * NT + r * (N / 16);
            if (i < ra || i >= N - rb) dst[i] = v[q * 16 + r];
        }
}

template <typename T, int K>
__global__ __launch_bounds__(ThetaHalf<K>::NT) void k_theta_fwd_h(
    const typename Cx<T>::type* __restrict__ band, typename Cx<T>::type* __restrict__ cs, int nt,
    int lmax, int mmax, const T* __restrict__ d1, const T* __restrict__ d2, int ra, int rb,
    const typename Cx<T>::type* __restrict__ tw)
{
    using C = typename Cx<T>::type;
    using S = ThetaHalf<K>;
    constexpr int N = S::N, R0 = S::R0, NT = S::NT;
    __shared__ T lds[N + N / 16];
    const int mu = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
    const int64_t col = (int64_t)b * (mmax + 1) + mu;
    const C* src = band + col * N;
    C* dst = cs + col * nt;
    const T fm = d2[mu];
    C v[32];
#pragma unroll
    for (int q = 0; q < 32 / R0; ++q)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int i = t + q * NT + r * (N / R0);
            v[q * R0 + r] = (i < ra || i >= N - rb) ? src[i] : cmk<C>(0, 0);
        }
    pass_in_regs<R0, -1, N, NT>(v, t, 1, tw);
    passes_after_first<K, -1>(lds, v, t, tw);
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = t + q * NT + r * (N / 16);
            const int k = kappa_of(i, N);
            const int ak = k < 0 ? -k : k;
            if (ak <= lmax) {
                const T f = d1[ak] * fm;
                dst[k < 0 ? k + nt : k] = cmk<C>(v[q * 16 + r].x * f, v[q * 16 + r].y * f);
            }
        }
    for (int e = t; e < nt; e += NT) {
        const int k = kappa_of(e, nt);
        if ((k < 0 ? -k : k) > lmax) dst[e] = cmk<C>(0, 0);
    }
}

}  // namespace

// n = F 2^K with F = 1 or 5; false otherwise
static bool split_len(int n, int& K, int& F)
{
    F = (n % 5 == 0) ? 5 : 1;
    const int m = n / F;
    if (m < 1 || (m & (m - 1))) return false;
    K = 0;
    while ((1 << K) < m) ++K;
    return true;
}

// one transform of N complex values held in LDS (with the pad slots)
template <typename T>
constexpr bool lds_fits(int N)
{
    return (size_t)(N + N / 16) * 2 * sizeof(T) <= 150 * 1024;
}

// lengths the kernels are built for: 2^K (K = 5 .. 14) and 5 2^K (K = 4 .. 11)
static bool len_supported(int K, int F)
{
    return F == 1 ? (K >= 5 && K <= 14) : (K >= 4 && K <= 11);
}

bool rowfft_supported(const nusht_geometry& g)
{
    const int n2 = g.n2;
    int K, F;
    if (n2 % 2 || !split_len(n2 / 2, K, F) || !len_supported(K, F)) return false;
    if (F == 1 && K > 13) return false;  // rows up to 16384 real values
    const int N = n2 / 2;
    if (!(g.dtype == NUSHT_MIXED ? lds_fits<float>(N) : lds_fits<double>(N))) return false;
    return g.mmax + 1 <= N;
}

#define NUSHT_FK_CASE(FF, KK, ...) \
    case (FF) * 100 + (KK): { constexpr int FV = FF, KV = KK; __VA_ARGS__; } break;
#define NUSHT_FK_SWITCH(F_, K_, ...)                                                             \
    switch ((F_) * 100 + (K_)) {                                                                 \
        NUSHT_FK_CASE(1, 5, __VA_ARGS__) NUSHT_FK_CASE(1, 6, __VA_ARGS__)                        \
        NUSHT_FK_CASE(1, 7, __VA_ARGS__) NUSHT_FK_CASE(1, 8, __VA_ARGS__)                        \
        NUSHT_FK_CASE(1, 9, __VA_ARGS__) NUSHT_FK_CASE(1, 10, __VA_ARGS__)                       \
        NUSHT_FK_CASE(1, 11, __VA_ARGS__) NUSHT_FK_CASE(1, 12, __VA_ARGS__)                      \
        NUSHT_FK_CASE(1, 13, __VA_ARGS__) NUSHT_FK_CASE(1, 14, __VA_ARGS__)                      \
        NUSHT_FK_CASE(5, 4, __VA_ARGS__) NUSHT_FK_CASE(5, 5, __VA_ARGS__)                        \
        NUSHT_FK_CASE(5, 6, __VA_ARGS__) NUSHT_FK_CASE(5, 7, __VA_ARGS__)                        \
        NUSHT_FK_CASE(5, 8, __VA_ARGS__) NUSHT_FK_CASE(5, 9, __VA_ARGS__)                        \
        NUSHT_FK_CASE(5, 10, __VA_ARGS__) NUSHT_FK_CASE(5, 11, __VA_ARGS__)                      \
        default: set_last_error("rowfft", "unsupported transform length"); return NUSHT_EINVAL; \
    }

template <typename T, int KV, int FV, bool C2R>
int launch_row_k(const nusht_plan_s* p, const void* in, void* out, int64_t rw, hipStream_t s)
{
    using C = typename Cx<T>::type;
    const nusht_geometry& g = p->g;
    const int nq = p->fine_ra + p->fine_rb;
    const C* tw = reinterpret_cast<const C*>(p->rowtw);
    if constexpr ((KV <= 13 || FV == 5) && lds_fits<T>(RowShape<KV, FV>::N)) {
        if (C2R)
            hipLaunchKernelGGL((k_row_c2r<T, KV, FV>), dim3(nq), dim3(RowShape<KV, FV>::NT), 0, s,
                               reinterpret_cast<const C*>(in), rw, g.mmax + 1,
                               reinterpret_cast<T*>(out), g.n1, p->fine_ra, p->fine_rb, tw);
        else
            hipLaunchKernelGGL((k_row_r2c<T, KV, FV>), dim3(nq), dim3(RowShape<KV, FV>::NT), 0, s,
                               reinterpret_cast<const T*>(in), g.n1, p->fine_ra, p->fine_rb,
                               reinterpret_cast<C*>(out), rw, g.mmax + 1, tw);
    } else {
        set_last_error("rowfft", "unsupported row length");
        return NUSHT_EINVAL;
    }
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

template <bool C2R>
int launch_row(const nusht_plan_s* p, const void* in, void* out, int64_t rw, hipStream_t s)
{
    int K = 0, F = 1;
    split_len(p->g.n2 / 2, K, F);
    NUSHT_FK_SWITCH(F, K, {
        if (p->g.dtype == NUSHT_MIXED) return launch_row_k<float, KV, FV, C2R>(p, in, out, rw, s);
        return launch_row_k<double, KV, FV, C2R>(p, in, out, rw, s);
    });
    return NUSHT_OK;
}

int launch_row_c2r(const nusht_plan_s* p, const void* rows, int64_t rw, void* fine, hipStream_t s)
{
    return launch_row<true>(p, rows, fine, rw, s);
}

int launch_row_r2c(const nusht_plan_s* p, const void* fine, void* rows, int64_t rw, hipStream_t s)
{
    return launch_row<false>(p, fine, rows, rw, s);
}

bool thetafft_supported(const nusht_geometry& g)
{
    const int n1 = g.n1;
    int K, F;
    if (g.dfs_mode != NUSHT_DFS_FUSED || !rowfft_supported(g)) return false;
    if (!split_len(n1, K, F) || !len_supported(K, F)) return false;
    // a complex column in LDS, or (FP64, 16384) real and imaginary parts in turn
    if (g.dtype == NUSHT_MIXED) return lds_fits<float>(n1);
    return lds_fits<double>(n1) || (F == 1 && K == 14);
}

// columns whose complex values exceed the LDS (FP64, 16384) take the register-resident kernels
// whose passes exchange through half of it.  (For the shorter columns the register-resident
// form needs 200-260 registers per lane and would not run two workgroups per CU after all.)
template <typename T>
constexpr bool theta_half(int K)
{
    return sizeof(T) == 8 && K >= 14;
}

// the theta-pass launch for one precision and length (a template, so that the kernels of the
// other branches are never instantiated)
template <typename T, int KV, int FV, bool INV>
int launch_theta_k(const nusht_plan_s* p, const void* in, void* out, int nmaps, hipStream_t s)
{
    using C = typename Cx<T>::type;
    const nusht_geometry& g = p->g;
    const dim3 grid(g.mmax + 1, nmaps);
    const T* d1 = std::is_same<T, float>::value ? (const T*)p->dec1f : (const T*)p->dec1;
    const T* d2 = std::is_same<T, float>::value ? (const T*)p->dec2f : (const T*)p->dec2;
    const C* tw = reinterpret_cast<const C*>(p->thetatw);
    const C* src = reinterpret_cast<const C*>(in);
    C* dst = reinterpret_cast<C*>(out);
    if constexpr (FV == 1 && theta_half<T>(KV)) {
        if (INV)
            hipLaunchKernelGGL((k_theta_inv_h<T, KV>), grid, dim3(ThetaHalf<KV>::NT), 0, s, src, dst,
                               g.ntorus, g.lmax, g.mmax, d1, d2, p->fine_ra, p->fine_rb, tw);
        else
            hipLaunchKernelGGL((k_theta_fwd_h<T, KV>), grid, dim3(ThetaHalf<KV>::NT), 0, s, src, dst,
                               g.ntorus, g.lmax, g.mmax, d1, d2, p->fine_ra, p->fine_rb, tw);
    } else if constexpr (lds_fits<T>(RowShape<KV, FV>::N)) {
        if (INV)
            hipLaunchKernelGGL((k_theta_inv<T, KV, FV>), grid, dim3(RowShape<KV, FV>::NT), 0, s, src,
                               dst, g.ntorus, g.lmax, g.mmax, d1, d2, p->fine_ra, p->fine_rb, tw);
        else
            hipLaunchKernelGGL((k_theta_fwd<T, KV, FV>), grid, dim3(RowShape<KV, FV>::NT), 0, s, src,
                               dst, g.ntorus, g.lmax, g.mmax, d1, d2, p->fine_ra, p->fine_rb, tw);
    } else {
        set_last_error("thetafft", "unsupported column length");
        return NUSHT_EINVAL;
    }
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

template <bool INV>
int launch_theta(const nusht_plan_s* p, const void* in, void* out, int nmaps, hipStream_t s)
{
    int K = 0, F = 1;
    split_len(p->g.n1, K, F);
    NUSHT_FK_SWITCH(F, K, {
        if (p->g.dtype == NUSHT_MIXED) return launch_theta_k<float, KV, FV, INV>(p, in, out, nmaps, s);
        return launch_theta_k<double, KV, FV, INV>(p, in, out, nmaps, s);
    });
    return NUSHT_OK;
}

int launch_theta_inv(const nusht_plan_s* p, const void* cs, void* band, int nmaps, hipStream_t s)
{
    return launch_theta<true>(p, cs, band, nmaps, s);
}

int launch_theta_fwd(const nusht_plan_s* p, const void* band, void* cs, int nmaps, hipStream_t s)
{
    return launch_theta<false>(p, band, cs, nmaps, s);
}

}  // namespace nusht
