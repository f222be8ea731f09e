// Row transforms of the fine grid (the phi direction of N's 2-D FFT, arXiv:2406.14542
// Sec. III) for power-of-two row lengths n2, one workgroup per window row:
//   C2R  x[n] = sum_{k=0}^{n2-1} X[k] e^{+2 pi i k n / n2},  X[n2 - k] = conj X[k],
//        X[k] = 0 for M < k < n2 - M (the band limit), Im X[0] ignored;
//   R2C  X[k] = sum_n x[n] e^{-2 pi i k n / n2}, k = 0 .. M only.
// Both take the half-length route: with N = n2 / 2 and z[n] = x[2n] + i x[2n+1],
//   z = IDFT_N(Z),  Z[k] = E[k] + i O[k],  E[k] = X[k] + X[k + N],
//   O[k] = (X[k] - X[k + N]) e^{2 pi i k / n2},  X[k + N] = conj X[N - k];
// and backwards E = (Z[k] + conj Z[N-k]) / 2, O = (Z[k] - conj Z[N-k]) / (2i),
//   X[k] = E + e^{-2 pi i k / n2} O.
// The theta pass of the same 2-D FFT (power-of-two n1, one workgroup per band column mu of
// one map) runs here as well, fused with the deconvolution of N(i) / N^H(iii):
//   synthesis  band[mu][i] = sum_{|k| <= L} C[k][mu] h(k, mu) e^{+2 pi i k i / n1}, window rows i
//   adjoint    C[k][mu] = h(k, mu) sum_{window rows i} band[mu][i] e^{-2 pi i k i / n1}, |k| <= L
// (h = the deconvolution factors d1[|k|] d2[mu]; k of entry t of the length-N_t torus column is
// t or t - N_t): the column is read once from the torus spectrum (synthesis: only its |k| <= L
// entries exist, the padding is zeros in registers) or from the window rows of the band
// (adjoint), transformed in LDS, and written once, so the zero-padded spectrum is never
// stored and no separate deconvolution pass reads or writes it.
// The N-point transform runs in LDS as Stockham radix passes (a first pass of radix
// 2^(log2 N mod 4) when needed, then radix 16), reading the row straight from HBM in the
// first pass and writing it in the last: one read and one write of each row, and only the
// M + 1 band columns of the spectrum are read (C2R) or written (R2C).
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

// in-place DFT of R = 1, 2, 4, 8 or 16 values, natural order in and out:
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

template <int K>
struct RowShape {
    static constexpr int N = 1 << K;                          // complex points
    static constexpr int NB16 = N / 16;                       // radix-16 butterflies per pass
    static constexpr int NT = NB16 < 64 ? 64 : NB16;          // threads
    static constexpr int R0 = (K % 4) ? (1 << (K % 4)) : 16;  // first pass radix
    static constexpr int NPASS16 = (K % 4) ? K / 4 : K / 4 - 1;  // radix-16 passes after it
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

template <int K, int DIR, typename C>
__device__ inline void middle_passes(C* buf, int t, const C* __restrict__ tw)
{
    using S = RowShape<K>;
    constexpr int N = S::N;
    const bool act = t < S::NB16;
#pragma unroll
    for (int p = 0; p < S::NPASS16 - 1; ++p) {
        int Ns = S::R0;
        for (int e = 0; e < p; ++e) Ns *= 16;
        const int j = t & (Ns - 1);
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
template <typename T, int K>
__global__ __launch_bounds__(RowShape<K>::NT) void k_row_c2r(
    const typename Cx<T>::type* __restrict__ rows, int64_t rw, int ncol,
    T* __restrict__ fine, int n1, int ra, int rb, const typename Cx<T>::type* __restrict__ tw)
{
    using C = typename Cx<T>::type;
    using S = RowShape<K>;
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
    middle_passes<K, +1>(buf, t, tw);
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
template <typename T, int K>
__global__ __launch_bounds__(RowShape<K>::NT) void k_row_r2c(
    const T* __restrict__ fine, int n1, int ra, int rb, typename Cx<T>::type* __restrict__ rows,
    int64_t rw, int ncol, const typename Cx<T>::type* __restrict__ tw)
{
    using C = typename Cx<T>::type;
    using S = RowShape<K>;
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
    middle_passes<K, -1>(buf, t, tw);
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
        const C zm = buf[pad16((N - k) & (N - 1))];
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
template <typename T, int K>
__global__ __launch_bounds__(RowShape<K>::NT) void k_theta_inv(
    const typename Cx<T>::type* __restrict__ cs, typename Cx<T>::type* __restrict__ band, int nt,
    int lmax, int mmax, const T* __restrict__ d1, const T* __restrict__ d2, int ra, int rb,
    const typename Cx<T>::type* __restrict__ tw)
{
    using C = typename Cx<T>::type;
    using S = RowShape<K>;
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
    middle_passes<K, +1>(buf, t, tw);
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
template <typename T, int K>
__global__ __launch_bounds__(RowShape<K>::NT) void k_theta_fwd(
    const typename Cx<T>::type* __restrict__ band, typename Cx<T>::type* __restrict__ cs, int nt,
    int lmax, int mmax, const T* __restrict__ d1, const T* __restrict__ d2, int ra, int rb,
    const typename Cx<T>::type* __restrict__ tw)
{
    using C = typename Cx<T>::type;
    using S = RowShape<K>;
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
    middle_passes<K, -1>(buf, t, tw);
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

bool rowfft_supported(const nusht_geometry& g)
{
    const int n2 = g.n2;
    if (n2 < 64 || n2 > 16384 || (n2 & (n2 - 1))) return false;
    return g.mmax + 1 <= n2 / 2;
}

#define NUSHT_ROWK_SWITCH(K_, BODY)                    \
    switch (K_) {                                      \
        case 5: { constexpr int KV = 5; BODY; } break;   \
        case 6: { constexpr int KV = 6; BODY; } break;   \
        case 7: { constexpr int KV = 7; BODY; } break;   \
        case 8: { constexpr int KV = 8; BODY; } break;   \
        case 9: { constexpr int KV = 9; BODY; } break;   \
        case 10: { constexpr int KV = 10; BODY; } break; \
        case 11: { constexpr int KV = 11; BODY; } break; \
        case 12: { constexpr int KV = 12; BODY; } break; \
        case 13: { constexpr int KV = 13; BODY; } break; \
        default: set_last_error("rowfft", "unsupported row length"); return NUSHT_EINVAL; \
    }

static int row_log2(int n2)
{
    int k = 0;
    while ((2 << k) < n2) ++k;
    return k;  // n2 / 2 = 2^k
}

int launch_row_c2r(const nusht_plan_s* p, const void* rows, int64_t rw, void* fine, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int nq = p->fine_ra + p->fine_rb;
    const int K = row_log2(g.n2);
    NUSHT_ROWK_SWITCH(K, {
        if (g.dtype == NUSHT_MIXED)
            hipLaunchKernelGGL((k_row_c2r<float, KV>), dim3(nq), dim3(RowShape<KV>::NT), 0, s,
                               reinterpret_cast<const float2*>(rows), rw, g.mmax + 1,
                               reinterpret_cast<float*>(fine), g.n1, p->fine_ra, p->fine_rb,
                               reinterpret_cast<const float2*>(p->rowtw));
        else
            hipLaunchKernelGGL((k_row_c2r<double, KV>), dim3(nq), dim3(RowShape<KV>::NT), 0, s,
                               reinterpret_cast<const double2*>(rows), rw, g.mmax + 1,
                               reinterpret_cast<double*>(fine), g.n1, p->fine_ra, p->fine_rb,
                               reinterpret_cast<const double2*>(p->rowtw));
    });
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int launch_row_r2c(const nusht_plan_s* p, const void* fine, void* rows, int64_t rw, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int nq = p->fine_ra + p->fine_rb;
    const int K = row_log2(g.n2);
    NUSHT_ROWK_SWITCH(K, {
        if (g.dtype == NUSHT_MIXED)
            hipLaunchKernelGGL((k_row_r2c<float, KV>), dim3(nq), dim3(RowShape<KV>::NT), 0, s,
                               reinterpret_cast<const float*>(fine), g.n1, p->fine_ra, p->fine_rb,
                               reinterpret_cast<float2*>(rows), rw, g.mmax + 1,
                               reinterpret_cast<const float2*>(p->rowtw));
        else
            hipLaunchKernelGGL((k_row_r2c<double, KV>), dim3(nq), dim3(RowShape<KV>::NT), 0, s,
                               reinterpret_cast<const double*>(fine), g.n1, p->fine_ra,
                               p->fine_rb, reinterpret_cast<double2*>(rows), rw, g.mmax + 1,
                               reinterpret_cast<const double2*>(p->rowtw));
    });
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

bool thetafft_supported(const nusht_geometry& g)
{
    const int n1 = g.n1;
    if (g.dfs_mode != NUSHT_DFS_FUSED || !rowfft_supported(g)) return false;
    if (n1 < 32 || (n1 & (n1 - 1))) return false;
    // columns up to 16384 values in LDS (complex, or real and imaginary parts in turn)
    return n1 <= 16384;
}

#define NUSHT_THETAK_SWITCH(K_, BODY)                  \
    switch (K_) {                                      \
        case 5: { constexpr int KV = 5; BODY; } break;   \
        case 6: { constexpr int KV = 6; BODY; } break;   \
        case 7: { constexpr int KV = 7; BODY; } break;   \
        case 8: { constexpr int KV = 8; BODY; } break;   \
        case 9: { constexpr int KV = 9; BODY; } break;   \
        case 10: { constexpr int KV = 10; BODY; } break; \
        case 11: { constexpr int KV = 11; BODY; } break; \
        case 12: { constexpr int KV = 12; BODY; } break; \
        case 13: { constexpr int KV = 13; BODY; } break; \
        case 14: { constexpr int KV = 14; BODY; } break; \
        default: set_last_error("thetafft", "unsupported column length"); return NUSHT_EINVAL; \
    }

static int col_log2(int n1)
{
    int k = 0;
    while ((1 << k) < n1) ++k;
    return k;
}

// columns whose complex values exceed the LDS (FP64, 16384) take the register-resident kernels
// whose passes exchange through half of it.  (For the shorter columns the register-resident
// form needs 200-260 registers per lane and would not run two workgroups per CU after all.)
template <typename T>
constexpr bool theta_half(int K)
{
    return sizeof(T) == 8 && K >= 14;
}

int launch_theta_inv(const nusht_plan_s* p, const void* cs, void* band, int nmaps, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int K = col_log2(g.n1);
    const dim3 grid(g.mmax + 1, nmaps);
#define NUSHT_THETA_INV(T, KK, KERN, SHAPE)                                                     \
    hipLaunchKernelGGL((KERN<T, KK>), grid, dim3(SHAPE<KK>::NT), 0, s,                          \
                       reinterpret_cast<const typename Cx<T>::type*>(cs),                       \
                       reinterpret_cast<typename Cx<T>::type*>(band), g.ntorus, g.lmax, g.mmax, \
                       std::is_same<T, float>::value ? (const T*)p->dec1f : (const T*)p->dec1,  \
                       std::is_same<T, float>::value ? (const T*)p->dec2f : (const T*)p->dec2,  \
                       p->fine_ra, p->fine_rb,                                                  \
                       reinterpret_cast<const typename Cx<T>::type*>(p->thetatw))
    NUSHT_THETAK_SWITCH(K, {
        if (g.dtype == NUSHT_MIXED) {
            if constexpr (theta_half<float>(KV))
                NUSHT_THETA_INV(float, KV, k_theta_inv_h, ThetaHalf);
            else
                NUSHT_THETA_INV(float, KV, k_theta_inv, RowShape);
        } else {
            if constexpr (theta_half<double>(KV))
                NUSHT_THETA_INV(double, KV, k_theta_inv_h, ThetaHalf);
            else
                NUSHT_THETA_INV(double, KV, k_theta_inv, RowShape);
        }
    });
#undef NUSHT_THETA_INV
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int launch_theta_fwd(const nusht_plan_s* p, const void* band, void* cs, int nmaps, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int K = col_log2(g.n1);
    const dim3 grid(g.mmax + 1, nmaps);
#define NUSHT_THETA_FWD(T, KK, KERN, SHAPE)                                                     \
    hipLaunchKernelGGL((KERN<T, KK>), grid, dim3(SHAPE<KK>::NT), 0, s,                          \
                       reinterpret_cast<const typename Cx<T>::type*>(band),                     \
                       reinterpret_cast<typename Cx<T>::type*>(cs), g.ntorus, g.lmax, g.mmax,   \
                       std::is_same<T, float>::value ? (const T*)p->dec1f : (const T*)p->dec1,  \
                       std::is_same<T, float>::value ? (const T*)p->dec2f : (const T*)p->dec2,  \
                       p->fine_ra, p->fine_rb,                                                  \
                       reinterpret_cast<const typename Cx<T>::type*>(p->thetatw))
    NUSHT_THETAK_SWITCH(K, {
        if (g.dtype == NUSHT_MIXED) {
            if constexpr (theta_half<float>(KV))
                NUSHT_THETA_FWD(float, KV, k_theta_fwd_h, ThetaHalf);
            else
                NUSHT_THETA_FWD(float, KV, k_theta_fwd, RowShape);
        } else {
            if constexpr (theta_half<double>(KV))
                NUSHT_THETA_FWD(double, KV, k_theta_fwd_h, ThetaHalf);
            else
                NUSHT_THETA_FWD(double, KV, k_theta_fwd, RowShape);
        }
    });
#undef NUSHT_THETA_FWD
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

}  // namespace nusht
