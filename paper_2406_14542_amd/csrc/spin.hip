// Spin-weighted Legendre step: the Wigner-d transform that replaces the Legendre step of S for
// spin-s fields (arXiv:2406.14542, Sec. V names spin-n transforms through Wigner's d as the
// extension of the method).  The rest of the path -- the doubled theta-columns, the torus
// theta-FFT, the nonuniform FFT -- is the spin-0 one run on the two real maps (Q, U) of every
// field; only the sign of the doubling changes: a spin-s quantity in the local (e_theta, e_phi)
// basis continues to theta -> -theta as (-1)^s times its value at phi + pi, so column m
// continues with (-1)^(m+s) instead of (-1)^m.
//
// Definitions (s >= 1, m >= 0, l >= l0 = max(m, s)):
//   slam_lm(theta) = (-1)^s sqrt((2l+1)/4pi) d^l_{m,-s}(theta)   (sY_lm = slam_lm e^{i m phi})
//   W+ = (slam + (-1)^s (-s)lam) / 2,  W- = (slam - (-1)^s (-s)lam) / 2
//   synthesis  Q_m = -sum_l (G_lm W+ + i C_lm W-),  U_m = -sum_l (C_lm W+ - i G_lm W-)
//   adjoint    cG_lm = -sum_j (Q'_m(j) W+ + i U'_m(j) W-),  cC_lm = -sum_j (U'_m(j) W+ - i Q'_m(j) W-)
// with G, C the gradient and curl coefficients (Q + iU = sum sa_lm sY_lm, sa_lm = -(G + iC)).
//
// Both functions p = slam and q = (-s)lam come from the three-term recurrence of Wigner's d in l
// at fixed (m, -+s): y_l = (c - alpha (1 - cos theta)) y_{l-1} - gamma y_{l-2}, where
// c = alpha + b for p and alpha - b for q (b carries m s); the coefficients are a host table in
// long double, rounded once ((alpha, c_p, c_q, gamma) per (l, m), 32 bytes).  The start at l0 is
// a product of half-angle powers, cos^a(theta/2) sin^b(theta/2), formed with an explicit binary
// exponent; the two functions share one count of 2^256 factors per lane, as the spin-0 kernel
// does, and a term enters the sums once the count is zero.
//
// gfx950 mapping (as the spin-0 kernels): a lane takes pairs of mirror rings (j, N_r-1-j)
// -- slam(pi - theta) = (-1)^(l+m) (-s)lam(theta), so W+ has hemisphere parity (-1)^(l+m+s) and
// W- the opposite, and even/odd-l accumulators serve both rings; the lanes of a block share m,
// so the coefficient stream is wave-uniform (scalar loads); blocks of one m sit on one XCD.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <thread>

namespace nusht {
namespace {

constexpr double kSpBig = 0x1p56;     // rescale once a scaled value reaches this
constexpr double kSpUnit = 0x1p-256;  // one scale unit
constexpr int kSpAccumExp = -200;     // terms below 2^-200 are not accumulated
constexpr int kSpLC = 4;              // l values per reduction chunk of the adjoint
constexpr int kSpPf = 32;             // l values between two L2 touches of a coefficient stream

// The coefficient streams of one m (recurrence table, 2 MB coefficient rows) are read through
// the scalar cache, one l at a time, by every wave of that m.  Every kSpPf values of l the wave
// touches the lines holding the next kSpPf coefficients of every stream, kSpPf steps ahead,
// with one LDS-DMA load per line: such a load has no register result, so nothing waits for
// it, and the lines are in L2 by the time the scalar loads reach them.  M0 (the DMA's LDS
// base, pointed at a per-wave sink that nothing reads) is restored after the load; the
// returned value is kept live by the caller, which waits for the DMA before the wave ends.
__device__ inline unsigned l2_touch(const void* src, unsigned lds_sink)
{
    unsigned saved;
    asm("s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %2\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dword %1, off\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(saved)
        : "v"(src), "s"(lds_sink));
    return saved;
}

// lines per stream for kSpPf values of l (one more for an unaligned start)
constexpr int kSpRecLines = kSpPf * 32 / 128 + 1;
constexpr int kSpAlmLines = kSpPf * 16 / 128 + 1;

// lane -> (stream, line); streams: the table, then NA coefficient rows spaced nalm apart
template <int NA>
__device__ inline unsigned spin_touch(const double4* __restrict__ rec,
                                      const double2* __restrict__ alm, int64_t nalm,
                                      int64_t moff, int lmax, int lp, int lane, unsigned sink)
{
    if (lp > lmax) return 0u;
    const void* src;
    if (lane < kSpRecLines) {
        src = rec + moff + min(lp + 4 * lane, lmax);
    } else {
        const int t = lane - kSpRecLines, st = t / kSpAlmLines, line = t - st * kSpAlmLines;
        if (st >= NA) return 0u;
        src = alm + (int64_t)st * nalm + moff + min(lp + 8 * line, lmax);
    }
    return l2_touch(src, sink);
}

// base^n (base >= 0) as mant * 2^e with mant in [0.5, 1); 0^0 = 1, 0^n = 0
__device__ inline void pow_exp(double base, int n, double& mant, int& e)
{
    mant = 0.5;
    e = 1;
    if (n == 0) return;
    if (base == 0.0) {
        mant = 0.0;
        e = 0;
        return;
    }
    int be;
    double b = frexp(base, &be);
    while (n) {
        int t;
        if (n & 1) {
            mant *= b;
            e += be;
            mant = frexp(mant, &t);
            e += t;
        }
        n >>= 1;
        if (n) {
            b *= b;
            be *= 2;
            b = frexp(b, &t);
            be += t;
        }
    }
}

__device__ inline void xcd_place(int b, int nbx, int& m, int& rb)
{
    const int x = b & 7, q = b >> 3;
    m = 8 * (q / nbx) + x;
    rb = q % nbx;
}

// Ring pair j: y = 1 - cos theta_j, and the start values p = slam_{l0 m}, q = (-s)lam_{l0 m}
// as p 2^(-256 k), q 2^(-256 k).
__device__ inline void spin_start(int j, int nr, int m, int spin, double km, int ke, double& y,
                                  double& p, double& q, int& k)
{
    const double a = (double)j / (2.0 * (double)(nr - 1));
    const double s2 = sinpi(a);
    const double c2 = (2 * j == nr - 1) ? s2 : cospi(a);
    y = 2.0 * s2 * s2;
    const int dms = m > spin ? m - spin : spin - m;
    double cu, su, cv, sv;
    int ecu, esu, ecv, esv;
    pow_exp(c2, dms, cu, ecu);
    pow_exp(s2, m + spin, su, esu);
    pow_exp(c2, m + spin, cv, ecv);
    pow_exp(s2, dms, sv, esv);
    // signs: d^{l0}_{m,-s} carries (-1)^(m+s); d^{l0}_{m,+s} carries (-1)^(m+s) when m >= s;
    // both functions carry (-1)^s
    const double sgu = ((m & 1) ? -1.0 : 1.0);
    const double sgv = (m >= spin) ? sgu : ((spin & 1) ? -1.0 : 1.0);
    int t;
    double mu = frexp(km * cu * su, &t);
    int eu = ke + ecu + esu + t;
    double mv = frexp(km * cv * sv, &t);
    int ev = ke + ecv + esv + t;
    int e;
    if (mu == 0.0 && mv == 0.0) {
        p = q = 0.0;
        k = 0;
        return;
    }
    if (mu == 0.0)
        e = ev;
    else if (mv == 0.0)
        e = eu;
    else
        e = max(eu, ev);
    k = e >= kSpAccumExp ? 0 : (kSpAccumExp - e + 255) / 256;
    p = sgu * ldexp(mu, eu + 256 * k);
    q = sgv * ldexp(mv, ev + 256 * k);
}

// one recurrence step of both functions
__device__ inline void spin_step(const double4 c, double y, double& p, double& q, double& pp,
                                 double& qp)
{
    const double tp = fma(-c.x, y, c.y);
    const double tq = fma(-c.x, y, c.z);
    const double pn = fma(tp, p, -(c.w * pp));
    const double qn = fma(tq, q, -(c.w * qp));
    pp = p;
    qp = q;
    p = pn;
    q = qn;
}

// the scaled variant: rescales the lane's pair when it reaches kSpBig while k > 0; returns
// whether the new values are live (k == 0)
__device__ inline bool spin_step_scaled(const double4 c, double y, double& p, double& q,
                                        double& pp, double& qp, int& k)
{
    spin_step(c, y, p, q, pp, qp);
    const bool big = (k > 0) && fmax(fabs(p), fabs(q)) >= kSpBig;
    const double sc = big ? kSpUnit : 1.0;
    p *= sc;
    q *= sc;
    pp *= sc;
    qp *= sc;
    k -= big ? 1 : 0;
    return k == 0;
}

template <typename OutT>
__device__ inline OutT make_pair(double re, double im)
{
    OutT o;
    o.x = re;
    o.y = im;
    return o;
}

// accumulators of one parity class, per field, in the basis of the two functions:
// G p (re, im), C p (re, im), G q (re, im), C q (re, im); W+- are formed from them once, at
// the end (the sums are linear in p and q)
template <int MB>
__device__ inline void spin_accum(double (&A)[MB][8], const double2* __restrict__ alm,
                                  int64_t nalm, int64_t idx, double p, double q)
{
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const double2 G = alm[(int64_t)(2 * b) * nalm + idx];
        const double2 C = alm[(int64_t)(2 * b + 1) * nalm + idx];
        A[b][0] = fma(G.x, p, A[b][0]);
        A[b][1] = fma(G.y, p, A[b][1]);
        A[b][2] = fma(C.x, p, A[b][2]);
        A[b][3] = fma(C.y, p, A[b][3]);
        A[b][4] = fma(G.x, q, A[b][4]);
        A[b][5] = fma(G.y, q, A[b][5]);
        A[b][6] = fma(C.x, q, A[b][6]);
        A[b][7] = fma(C.y, q, A[b][7]);
    }
}

// Synthesis, for maps 2f (Q) and 2f+1 (U) of field f.  FUSED: out[map][m][t] (t < N_t), the
// doubled columns: out(t) = X(t) for t < N_r, (-1)^(m+s) X(N_t - t) for t >= N_r.  Otherwise
// out[map][j][m], the ring rows of the paper composition (its doubling comes later).
template <int MB, typename OutT, bool FUSED>
__global__ __launch_bounds__(256) void k_spin_synth(
    const double2* __restrict__ alm, int64_t nalm, int lmax, int mmax, int spin, int nbx,
    const double4* __restrict__ rec, const double* __restrict__ km, const int* __restrict__ ke,
    const int* __restrict__ jlive, int nr, int nt, OutT* __restrict__ out,
    int64_t out_map_stride, int64_t out_row_stride)
{
    int m, rb;
    xcd_place(blockIdx.x, nbx, m, rb);
    if (m > mmax) return;
    const int npairs = (nr + 1) / 2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wbase = (rb * (blockDim.x >> 6) + wave) * 64;
    if (wbase >= npairs) return;
    alm += (int64_t)blockIdx.y * MB * 2 * nalm;
    out += (int64_t)blockIdx.y * MB * 2 * out_map_stride;
    const int64_t moff = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const int l0 = max(m, spin);
    const double sg = (spin & 1) ? -1.0 : 1.0;

    double E[MB][8], O[MB][8];
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
        for (int i = 0; i < 8; ++i) E[b][i] = O[b][i] = 0.0;

    __shared__ float pf_sink[4][64];
    const int j = min(wbase + lane, npairs - 1);
    // a wave whose ring pairs all lie below the first live pair of this m adds nothing
    if (wbase + 64 > jlive[m]) {
        double y, p, q;
        int k;
        spin_start(j, nr, m, spin, km[m], ke[m], y, p, q, k);
        double pp = 0.0, qp = 0.0;
        bool any_scaled = k > 0;
        if (k == 0) spin_accum<MB>(E, alm, nalm, moff + l0, p, q);
        auto scaled = [&](int l, double (&A)[MB][8]) {
            const bool live = spin_step_scaled(rec[moff + l], y, p, q, pp, qp, k);
            any_scaled = !live;
            spin_accum<MB>(A, alm, nalm, moff + l, live ? p : 0.0, live ? q : 0.0);
        };
        auto plain = [&](int l, double (&A)[MB][8]) {
            spin_step(rec[moff + l], y, p, q, pp, qp);
            spin_accum<MB>(A, alm, nalm, moff + l, p, q);
        };
        int l = l0 + 1;
        int pf_at = l;
        unsigned pf_keep = 0;
        const unsigned sink = __builtin_amdgcn_readfirstlane(
            (unsigned)(uintptr_t)(__attribute__((address_space(3))) float*)pf_sink[wave]);
        auto prefetch = [&]() {
            if (l >= pf_at) {
                pf_keep ^= spin_touch<2 * MB>(rec, alm, nalm, moff, lmax, l + kSpPf, lane, sink);
                pf_at = l + kSpPf;
            }
        };
        // while some lane of the wave still carries a 2^256 factor: the scaled steps (the
        // branch is wave-uniform); then the plain recurrence without further tests
        for (; l + 1 <= lmax && __any(any_scaled); l += 2) {
            prefetch();
            scaled(l, O);
            scaled(l + 1, E);
        }
        for (; l + 1 <= lmax; l += 2) {
            prefetch();
            plain(l, O);
            plain(l + 1, E);
        }
        if (l <= lmax) {
            if (__any(any_scaled))
                scaled(l, O);
            else
                plain(l, O);
        }
        // no LDS-DMA write may be in flight when the workgroup's LDS is released
        asm volatile("s_waitcnt vmcnt(0)" ::"v"(pf_keep) : "memory");
    }

    const int jj = wbase + lane;
    if (jj >= npairs) return;
    const int js = nr - 1 - jj;
    const double dsg = ((m + spin) & 1) ? -1.0 : 1.0;  // doubling sign
    const double tau = ((l0 + m) & 1) ? -1.0 : 1.0;     // (-1)^(l+m) of the even class
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        double S[8], D[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            S[i] = E[b][i] + O[b][i];
            D[i] = tau * (E[b][i] - O[b][i]);
        }
        // With P = sum (G + iC) slam and M = sum (G - iC) (-s)lam:
        //   Q = -(P + (-1)^s M) / 2,  U = i (P - (-1)^s M) / 2.
        // North: P = Gp + i Cp, M = Gq - i Cq.  South, where slam(pi - theta) =
        // (-1)^(l+m) (-s)lam(theta) and vice versa: P = Gq' + i Cq', M = Gp' - i Cp' with the
        // parity-signed sums (').
        const double pnr = S[0] - S[3], pni = S[1] + S[2];
        const double mnr = S[4] + S[7], mni = S[5] - S[6];
        const double psr = D[4] - D[7], psi = D[5] + D[6];
        const double msr = D[0] + D[3], msi = D[1] - D[2];
        double qn_re = -0.5 * fma(sg, mnr, pnr), qn_im = -0.5 * fma(sg, mni, pni);
        double un_re = -0.5 * fma(-sg, mni, pni), un_im = 0.5 * fma(-sg, mnr, pnr);
        double qs_re = -0.5 * fma(sg, msr, psr), qs_im = -0.5 * fma(sg, msi, psi);
        double us_re = -0.5 * fma(-sg, msi, psi), us_im = 0.5 * fma(-sg, msr, psr);
        if (m == 0) qn_im = un_im = qs_im = us_im = 0.0;  // imaginary parts of m = 0 are ignored
        if (!FUSED) {
            OutT* rq = out + (int64_t)(2 * b) * out_map_stride + m;
            OutT* ru = rq + out_map_stride;
            rq[(int64_t)jj * out_row_stride] = make_pair<OutT>(qn_re, qn_im);
            ru[(int64_t)jj * out_row_stride] = make_pair<OutT>(un_re, un_im);
            if (js != jj) {
                rq[(int64_t)js * out_row_stride] = make_pair<OutT>(qs_re, qs_im);
                ru[(int64_t)js * out_row_stride] = make_pair<OutT>(us_re, us_im);
            }
            continue;
        }
        OutT* cq = out + (int64_t)(2 * b) * out_map_stride + (int64_t)m * out_row_stride;
        OutT* cu = cq + out_map_stride;
        cq[jj] = make_pair<OutT>(qn_re, qn_im);
        cu[jj] = make_pair<OutT>(un_re, un_im);
        if (jj >= 1 && jj <= nr - 2) {
            cq[nt - jj] = make_pair<OutT>(dsg * qn_re, dsg * qn_im);
            cu[nt - jj] = make_pair<OutT>(dsg * un_re, dsg * un_im);
        }
        if (js != jj) {
            cq[js] = make_pair<OutT>(qs_re, qs_im);
            cu[js] = make_pair<OutT>(us_re, us_im);
            if (js >= 1 && js <= nr - 2) {
                cq[nt - js] = make_pair<OutT>(dsg * qs_re, dsg * qs_im);
                cu[nt - js] = make_pair<OutT>(dsg * us_re, dsg * us_im);
            }
        }
    }
}

template <typename InT>
__device__ inline double2 load2(const InT* p)
{
    const InT v = *p;
    return make_double2((double)v.x, (double)v.y);
}

// folded ring value of the fused input column: X(j) + [1 <= j <= N_r - 2] sgn X(N_t - j)
template <typename InT>
__device__ inline double2 folded(const InT* col, int j, int nr, int nt, double sgn)
{
    double2 v = load2(col + j);
    if (j >= 1 && j <= nr - 2) {
        const double2 w = load2(col + (nt - j));
        v.x = fma(sgn, w.x, v.x);
        v.y = fma(sgn, w.y, v.y);
    }
    return v;
}

// Adjoint.  Each lane holds kSpAdjR ring pairs (j, j + 64, ...) and multiplies W+- of each
// with its folded ring data, summing them in registers; the sums over the wave's ring pairs
// are then formed per chunk of kSpLC values of l: every lane parks its 4 MB products per l in
// LDS, the wave reads them back transposed (a row per lane group) and sums, and each wave adds
// its sums into the zeroed output with FP64 atomics, with no barrier between the waves (the
// blocks of one m run on one XCD: the atomics resolve in its L2; the order of those additions
// is not fixed, see DET for the fixed-order variant).
constexpr int kSpAdjR = 3;  // ring pairs per lane of the adjoint

// DET: instead of the atomic adds, wave w of the m's waves writes its sums (unscaled) to
// alm + w * part_stride, a zeroed per-wave partial array that k_spin_adj_reduce then adds in
// wave order (bit-identical results from run to run).
template <int MB, typename InT, bool DET, bool FUSED>
__global__ __launch_bounds__(256) void k_spin_adj(
    const InT* __restrict__ in, int64_t in_map_stride, int64_t in_row_stride,
    double* __restrict__ alm, int64_t nalm, int lmax, int mmax, int spin, int nbx,
    const double4* __restrict__ rec, const double* __restrict__ km, const int* __restrict__ ke,
    const int* __restrict__ jlive, int nr, int nt, int64_t part_stride)
{
    constexpr int R = kSpAdjR;
    constexpr int NV = 4 * MB;          // products per l per lane
    constexpr int ROWS = kSpLC * NV;    // rows of one chunk
    constexpr int LPR = 64 / ROWS;      // lanes per row in the transposed read
    constexpr int PER = 64 / LPR;       // entries summed per lane
    static_assert(ROWS * LPR == 64, "chunk shape");
    // rows of 64 lane entries, the upper half shifted by one slot (entry e at e + e / 32):
    // the transposed read's two lanes of a row then fall on different banks
    __shared__ double buf[4][ROWS][66];
    __shared__ float pf_sink[4][64];

    int m, rb;
    xcd_place(blockIdx.x, nbx, m, rb);
    if (m > mmax) return;  // uniform over the block
    const int npairs = (nr + 1) / 2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    const int wbase = (rb * nw + wave) * 64 * R;
    // a wave below the first live pair of this m, or past the last pair, adds nothing
    if (wbase + 64 * R <= jlive[m] || wbase >= npairs) return;
    in += (int64_t)blockIdx.y * MB * 2 * in_map_stride;
    alm += (int64_t)blockIdx.y * MB * 2 * nalm * 2;
    const int64_t moff = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const int l0 = max(m, spin);
    const double sg = (spin & 1) ? -1.0 : 1.0;
    const double dsg = ((m + spin) & 1) ? -1.0 : 1.0;
    const bool even_plus = ((l0 + m + spin) & 1) == 0;

    // Per ring pair and field the four combinations Q+ = Qn + Qs, Q- = Qn - Qs, U+, U- of the
    // folded data.  For hemisphere parity tau = +1 of (l + m + s):
    //   cG <- W+ Q+ + i W- U-,   cC <- W+ U+ - i W- Q-
    // and for tau = -1 the same with + and - exchanged.  X1/Y1 are the Q/U combinations that
    // the even class (l - l0 even) takes as (Q+, U-) roles, X2/Y2 the odd class's.
    double2 X1[R][MB], X2[R][MB], Y1[R][MB], Y2[R][MB];
    double y[R], p[R], q[R], pp[R], qp[R];
    int k[R];
    bool live[R];
    bool any_scaled = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int jraw = wbase + lane + 64 * r;
        const int j = min(jraw, npairs - 1);
        const int js = nr - 1 - j;
        const bool ok = jraw < npairs;
#pragma unroll
        for (int b = 0; b < MB; ++b) {
            double2 qn = make_double2(0.0, 0.0), un = qn, qs = qn, us = qn;
            if (ok && FUSED) {
                const InT* colq = in + (int64_t)(2 * b) * in_map_stride + (int64_t)m * in_row_stride;
                const InT* colu = colq + in_map_stride;
                qn = folded(colq, j, nr, nt, dsg);
                un = folded(colu, j, nr, nt, dsg);
                if (js != j) {
                    qs = folded(colq, js, nr, nt, dsg);
                    us = folded(colu, js, nr, nt, dsg);
                }
            } else if (ok) {
                // ring rows [map][j][m] of the paper composition, already folded
                const InT* rq = in + (int64_t)(2 * b) * in_map_stride + m;
                const InT* ru = rq + in_map_stride;
                qn = load2(rq + (int64_t)j * in_row_stride);
                un = load2(ru + (int64_t)j * in_row_stride);
                if (js != j) {
                    qs = load2(rq + (int64_t)js * in_row_stride);
                    us = load2(ru + (int64_t)js * in_row_stride);
                }
            }
            const double2 qpl = make_double2(qn.x + qs.x, qn.y + qs.y);
            const double2 qmi = make_double2(qn.x - qs.x, qn.y - qs.y);
            const double2 upl = make_double2(un.x + us.x, un.y + us.y);
            const double2 umi = make_double2(un.x - us.x, un.y - us.y);
            X1[r][b] = even_plus ? qpl : qmi;
            X2[r][b] = even_plus ? qmi : qpl;
            Y1[r][b] = even_plus ? umi : upl;
            Y2[r][b] = even_plus ? upl : umi;
        }
        spin_start(j, nr, m, spin, km[m], ke[m], y[r], p[r], q[r], k[r]);
        pp[r] = qp[r] = 0.0;
        live[r] = k[r] == 0;
        any_scaled |= k[r] > 0;
    }

    // the products of one l, summed over the lane's ring pairs, into row li of the chunk:
    // with (A, B, C, D) = (X1, Y1, Y2, X2) for the even class and (X2, Y2, Y1, X1) for the odd
    //   cG.re += W+ A.x - W- B.y,  cG.im += W+ A.y + W- B.x
    //   cC.re += W+ C.x + W- D.y,  cC.im += W+ C.y - W- D.x
    const int slot = lane + (lane >> 5);
    auto put = [&](int li, bool odd, bool gated, const bool (&on)[R]) {
        double v[MB][4];
#pragma unroll
        for (int b = 0; b < MB; ++b) v[b][0] = v[b][1] = v[b][2] = v[b][3] = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double wp = fma(sg, q[r], p[r]);
            double wm = fma(-sg, q[r], p[r]);
            if (gated) {
                wp = on[r] ? wp : 0.0;
                wm = on[r] ? wm : 0.0;
            }
#pragma unroll
            for (int b = 0; b < MB; ++b) {
                const double2 A = odd ? X2[r][b] : X1[r][b];
                const double2 B = odd ? Y2[r][b] : Y1[r][b];
                const double2 C = odd ? Y1[r][b] : Y2[r][b];
                const double2 D = odd ? X1[r][b] : X2[r][b];
                v[b][0] = fma(wp, A.x, fma(-wm, B.y, v[b][0]));
                v[b][1] = fma(wp, A.y, fma(wm, B.x, v[b][1]));
                v[b][2] = fma(wp, C.x, fma(wm, D.y, v[b][2]));
                v[b][3] = fma(wp, C.y, fma(-wm, D.x, v[b][3]));
            }
        }
#pragma unroll
        for (int b = 0; b < MB; ++b)
#pragma unroll
            for (int t = 0; t < 4; ++t) buf[wave][li * NV + 4 * b + t][slot] = v[b][t];
    };

    int pf_at = l0 + 1;
    unsigned pf_keep = 0;
    const unsigned sink = __builtin_amdgcn_readfirstlane(
        (unsigned)(uintptr_t)(__attribute__((address_space(3))) float*)pf_sink[wave]);
    for (int lc = l0; lc <= lmax; lc += kSpLC) {
        if (lc + 1 >= pf_at) {
            pf_keep ^= spin_touch<0>(rec, nullptr, 0, moff, lmax, lc + 1 + kSpPf, lane, sink);
            pf_at = lc + 1 + kSpPf;
        }
        const bool sc = __any(any_scaled);
        // the chunk's coefficients in one go: a scalar load waits on the same counter as
        // the LDS writes of the steps, so none is issued between them
        double4 cc[kSpLC];
#pragma unroll
        for (int li = 0; li < kSpLC; ++li) cc[li] = rec[moff + min(lc + li, lmax)];
        if (sc || lc + kSpLC - 1 > lmax || lc == l0) {
            // some lane still scaled, the last chunk or the first: every step tested
#pragma unroll
            for (int li = 0; li < kSpLC; ++li) {
                const int l = lc + li;
                bool on[R];
#pragma unroll
                for (int r = 0; r < R; ++r) on[r] = false;
                if (l <= lmax) {
                    if (l > l0) {
                        const double4 c = cc[li];
                        if (sc) {
                            any_scaled = false;
#pragma unroll
                            for (int r = 0; r < R; ++r) {
                                live[r] = spin_step_scaled(c, y[r], p[r], q[r], pp[r], qp[r], k[r]);
                                any_scaled |= !live[r];
                            }
                        } else {
#pragma unroll
                            for (int r = 0; r < R; ++r)
                                spin_step(c, y[r], p[r], q[r], pp[r], qp[r]);
                        }
                    }
#pragma unroll
                    for (int r = 0; r < R; ++r) on[r] = live[r];
                }
                put(li, (li & 1) != 0, true, on);
            }
        } else {
            // every lane live, every step in range
            const bool all_on[R] = {};
#pragma unroll
            for (int li = 0; li < kSpLC; ++li) {
#pragma unroll
                for (int r = 0; r < R; ++r) spin_step(cc[li], y[r], p[r], q[r], pp[r], qp[r]);
                put(li, (li & 1) != 0, false, all_on);
            }
        }
        // transposed read of this wave's chunk
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int rr = lane / LPR, h = lane % LPR;
        double acc = 0.0;
#pragma unroll 8
        for (int i = 0; i < PER; ++i) {
            const int e = h * PER + i;
            acc += buf[wave][rr][e + (e >> 5)];
        }
#pragma unroll
        for (int o = 1; o < LPR; o <<= 1) acc += __shfl_xor(acc, o);
        if (h == 0) {
            const int li = rr / NV, v = rr % NV;
            const int l = lc + li;
            // (imaginary parts of m = 0 stay zero: that coefficient is real)
            if (l <= lmax && !(m == 0 && (v & 1))) {
                const int b = v >> 2, t = v & 3;
                const int64_t o = ((int64_t)(2 * b + (t >> 1)) * nalm + moff + l) * 2 + (t & 1);
                if (DET)
                    alm[(int64_t)(rb * nw + wave) * part_stride + o] = acc;
                else
                    atomicAdd(alm + o, -0.5 * acc);
            }
        }
        // this wave's reads of buf are done before its next writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // no LDS-DMA write may be in flight when the workgroup's LDS is released
    asm volatile("s_waitcnt vmcnt(0)" ::"v"(pf_keep) : "memory");
}

__global__ void k_spin_zero(double* __restrict__ a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

// out[i] = -1/2 sum_w part[w * n + i], w = 0..nw-1 in order
__global__ void k_spin_adj_reduce(const double* __restrict__ part, int nw, int64_t n,
                                  double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int w = 0; w < nw; ++w) acc += part[(int64_t)w * n + i];
    out[i] = -0.5 * acc;
}

}  // namespace

// Whether slam or (-s)lam of ring pair j reaches 2^-300 for some l <= L (the kernels add
// nothing below 2^-200): the start value from the closed form in log2, then the recurrence
// with the table's coefficients and an explicit exponent, as in the kernels.
static bool spin_ring_reaches(int L, int m, int spin, int j, int nr, const std::vector<double>& rec,
                              int64_t moff, double km, int ke)
{
    const double a = (double)j / (2.0 * (double)(nr - 1));
    const double s2 = std::sin(M_PI * a);
    const double c2 = (2 * j == nr - 1) ? s2 : std::cos(M_PI * a);
    if (s2 == 0.0) return m == spin;  // at the pole only d^l_{s,s} is nonzero
    const double y = 2.0 * s2 * s2;
    const int dms = std::abs(m - spin), l0 = std::max(m, spin);
    const double lk = std::log2(km) + ke;
    const double lu = lk + dms * std::log2(c2) + (m + spin) * std::log2(s2);
    const double lv = lk + (m + spin) * std::log2(c2) + dms * std::log2(s2);
    const double top = std::max(lu, lv);
    if (top > -300.0) return true;
    int e = (int)std::floor(top);
    double p = std::exp2(lu - e), q = std::exp2(lv - e), pp = 0.0, qp = 0.0;
    for (int l = l0 + 1; l <= L; ++l) {
        const double* c = &rec[4 * (size_t)(moff + l)];
        const double pn = (c[1] - c[0] * y) * p - c[3] * pp;
        const double qn = (c[2] - c[0] * y) * q - c[3] * qp;
        pp = p;
        qp = q;
        p = pn;
        q = qn;
        const double big = std::max(std::max(std::fabs(p), std::fabs(q)),
                                    std::max(std::fabs(pp), std::fabs(qp)));
        if (big > 0x1p200 || (big < 0x1p-200 && big > 0.0)) {
            int t;
            std::frexp(big, &t);
            p = std::ldexp(p, -t);
            q = std::ldexp(q, -t);
            pp = std::ldexp(pp, -t);
            qp = std::ldexp(qp, -t);
            e += t;
        }
        const double cur = std::max(std::fabs(p), std::fabs(q));
        int t2;
        std::frexp(cur, &t2);
        if (cur != 0.0 && e + t2 > -300) return true;
    }
    return false;
}

// (alpha, c_p, c_q, gamma) of the step to every (l, m), l >= l0 + 1, and the start constants
// K_m = sqrt((2 l0 + 1)/4pi) sqrt(binom(2 l0, l0 + min(m, s))) as mantissa * 2^exponent, all
// in long double; rebuilt when the spin changes.
int ensure_spin_tables(nusht_plan_s* p, int spin)
{
    if (p->spin_s == spin && p->spin_rec) return NUSHT_OK;
    const nusht_geometry& g = p->g;
    const int L = g.lmax, M = g.mmax;
    std::vector<double> rec(4 * ((size_t)g.nalm + kRecPad), 0.0);
    std::vector<double> km(M + 1);
    std::vector<int> ke(M + 1);
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nth; ++t)
        pool.emplace_back([&, t] {
            for (int m = (int)t; m <= M; m += (int)nth) {
                const int64_t moff = (int64_t)m * (2 * L + 1 - m) / 2;
                const int l0 = std::max(m, spin), lo = std::min(m, spin);
                const long double mm = m, ss = spin;
                for (int l = l0 + 1; l <= L; ++l) {
                    const long double c = l - 1, c1 = l;  // step from degree c to c + 1
                    const long double dc = sqrtl((c * c - mm * mm) * (c * c - ss * ss));
                    const long double dc1 = sqrtl((c1 * c1 - mm * mm) * (c1 * c1 - ss * ss));
                    const long double r = sqrtl((2 * c + 3) * (2 * c + 1));
                    const long double alpha = r * c1 / dc1;
                    const long double b = (m == 0) ? 0.0L : r * mm * ss / (c * dc1);
                    const long double gam =
                        (l - 1 == l0) ? 0.0L : sqrtl((2 * c + 3) / (2 * c - 1)) * c1 * dc / (c * dc1);
                    double* e = &rec[4 * (size_t)(moff + l)];
                    e[0] = (double)alpha;
                    e[1] = (double)(alpha + b);
                    e[2] = (double)(alpha - b);
                    e[3] = (double)gam;
                }
                long double v = sqrtl((2.0L * l0 + 1.0L) / (4.0L * 3.14159265358979323846264338327950288L));
                int ex = 0, tt;
                v = frexpl(v, &tt);
                ex += tt;
                for (int kk = 1; kk <= l0 - lo; ++kk) {
                    v *= sqrtl((long double)(l0 + lo + kk) / (long double)kk);
                    v = frexpl(v, &tt);
                    ex += tt;
                }
                km[m] = (double)v;
                ke[m] = ex;
            }
        });
    for (auto& th : pool) th.join();
    // first live ring pair of every m (bisection: liveness grows towards the equator)
    std::vector<int> jl(M + 1, 0);
    {
        const int npairs = (g.nrings + 1) / 2;
        std::vector<std::thread> pool2;
        for (unsigned t = 0; t < nth; ++t)
            pool2.emplace_back([&, t] {
                for (int m = (int)t; m <= M; m += (int)nth) {
                    const int64_t moff = (int64_t)m * (2 * L + 1 - m) / 2;
                    int lo = 0, hi = npairs;
                    while (lo < hi) {
                        const int mid = (lo + hi) / 2;
                        if (spin_ring_reaches(L, m, spin, mid, g.nrings, rec, moff, km[m], ke[m]))
                            hi = mid;
                        else
                            lo = mid + 1;
                    }
                    jl[m] = lo;
                }
            });
        for (auto& th : pool2) th.join();
    }
    if (p->spin_rec) {
        NUSHT_HIP(hipDeviceSynchronize());
        hipFree(p->spin_rec);
        hipFree(p->spin_km);
        hipFree(p->spin_ke);
        hipFree(p->spin_jlive);
        p->spin_rec = nullptr;
        p->spin_km = nullptr;
        p->spin_ke = nullptr;
        p->spin_jlive = nullptr;
    }
    p->spin_s = 0;
    NUSHT_HIP(hipMalloc((void**)&p->spin_rec, ((size_t)g.nalm + kRecPad) * sizeof(double4)));
    NUSHT_HIP(hipMalloc((void**)&p->spin_km, (M + 1) * sizeof(double)));
    NUSHT_HIP(hipMalloc((void**)&p->spin_ke, (M + 1) * sizeof(int)));
    NUSHT_HIP(hipMalloc((void**)&p->spin_jlive, (M + 1) * sizeof(int)));
    NUSHT_HIP(hipMemcpy(p->spin_jlive, jl.data(), jl.size() * sizeof(int), hipMemcpyHostToDevice));
    NUSHT_HIP(hipMemcpy(p->spin_rec, rec.data(), rec.size() * sizeof(double), hipMemcpyHostToDevice));
    NUSHT_HIP(hipMemcpy(p->spin_km, km.data(), km.size() * sizeof(double), hipMemcpyHostToDevice));
    NUSHT_HIP(hipMemcpy(p->spin_ke, ke.data(), ke.size() * sizeof(int), hipMemcpyHostToDevice));
    p->spin_s = spin;
    return NUSHT_OK;
}

int launch_spin_synth(nusht_plan_s* p, int spin, const double* alm, void* out, int nfields,
                      int out_f32, hipStream_t s, bool fused)
{
    NUSHT_TRY(ensure_spin_tables(p, spin));
    const nusht_geometry& g = p->g;
    const int npairs = (g.nrings + 1) / 2;
    const int waves_needed = (npairs + 63) / 64;
    const int wpb = waves_needed >= 4 ? 4 : waves_needed;
    const int nbx = (waves_needed + wpb - 1) / wpb;
    const int mpad = (g.mmax + 1 + 7) / 8 * 8;
    const int64_t row_stride = fused ? g.ntorus : g.nphi / 2 + 1;
    const int64_t map_stride = fused ? (int64_t)(g.mmax + 1) * g.ntorus : (int64_t)g.nrings * row_stride;
    const double2* a = reinterpret_cast<const double2*>(alm);
    int f = 0;
    while (f < nfields) {
        const int mb = nfields - f >= 2 ? 2 : 1;
        const int groups = (nfields - f) / mb;
        const double2* af = a + (int64_t)f * 2 * g.nalm;
#define SPS(MBV, OT, FU)                                                                         \
    hipLaunchKernelGGL((k_spin_synth<MBV, OT, FU>), dim3(nbx * mpad, groups), dim3(64 * wpb), 0, \
                       s,                                                                        \
                       af, g.nalm, g.lmax, g.mmax, spin, nbx, p->spin_rec, p->spin_km,           \
                       p->spin_ke, p->spin_jlive, g.nrings, g.ntorus,                            \
                       reinterpret_cast<OT*>(out) + (int64_t)f * 2 * map_stride, map_stride,     \
                       row_stride)
        if (!fused) {
            if (mb == 2) SPS(2, double2, false); else SPS(1, double2, false);
        } else if (out_f32) {
            if (mb == 2) SPS(2, float2, true); else SPS(1, float2, true);
        } else {
            if (mb == 2) SPS(2, double2, true); else SPS(1, double2, true);
        }
#undef SPS
        NUSHT_HIP(hipGetLastError());
        f += groups * mb;
    }
    return NUSHT_OK;
}

int launch_spin_adjoint(nusht_plan_s* p, int spin, const void* in, double* alm, int nfields,
                        int in_f32, hipStream_t s, bool fused)
{
    NUSHT_TRY(ensure_spin_tables(p, spin));
    const nusht_geometry& g = p->g;
    const int npairs = (g.nrings + 1) / 2;
    // four independent waves per block, kSpAdjR ring pairs per lane
    const int nbx = (npairs + 256 * kSpAdjR - 1) / (256 * kSpAdjR);
    const int mpad = (g.mmax + 1 + 7) / 8 * 8;
    const int64_t row_stride = fused ? g.ntorus : g.nphi / 2 + 1;
    const int64_t map_stride = fused ? (int64_t)(g.mmax + 1) * g.ntorus : (int64_t)g.nrings * row_stride;
    const int64_t nz = (int64_t)nfields * 2 * g.nalm * 2;  // doubles of the output
    const int nwm = 4 * nbx;                                // waves per m
    const bool det = p->deterministic != 0;
    double* target = alm;
    if (det) {
        // per-wave partial sums, zeroed (waves below the first live pair write nothing)
        const size_t need = (size_t)nwm * nz * sizeof(double);
        if (need > p->adj_part_bytes) {
            NUSHT_HIP(hipStreamSynchronize(s));
            if (p->adj_part) hipFree(p->adj_part);
            p->adj_part = nullptr;
            p->adj_part_bytes = 0;
            NUSHT_HIP(hipMalloc((void**)&p->adj_part, need));
            p->adj_part_bytes = need;
        }
        target = p->adj_part;
        const int64_t np = (int64_t)nwm * nz;
        hipLaunchKernelGGL(k_spin_zero, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s,
                           target, np);
    } else {
        hipLaunchKernelGGL(k_spin_zero, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s, alm,
                           nz);
    }
    int f = 0;
    while (f < nfields) {
        const int mb = nfields - f >= 2 ? 2 : 1;
        const int groups = (nfields - f) / mb;
        double* af = target + (int64_t)f * 2 * g.nalm * 2;
#define SPA(MBV, IT, D, FU)                                                                      \
    hipLaunchKernelGGL((k_spin_adj<MBV, IT, D, FU>), dim3(nbx * mpad, groups), dim3(256), 0, s,   \
                       reinterpret_cast<const IT*>(in) + (int64_t)f * 2 * map_stride, map_stride, \
                       row_stride, af, g.nalm, g.lmax, g.mmax, spin, nbx, p->spin_rec,           \
                       p->spin_km, p->spin_ke, p->spin_jlive, g.nrings, g.ntorus, nz)
        if (!fused) {
            if (det) {
                if (mb == 2) SPA(2, double2, true, false); else SPA(1, double2, true, false);
            } else {
                if (mb == 2) SPA(2, double2, false, false); else SPA(1, double2, false, false);
            }
        } else if (det) {
            if (in_f32) {
                if (mb == 2) SPA(2, float2, true, true); else SPA(1, float2, true, true);
            } else {
                if (mb == 2) SPA(2, double2, true, true); else SPA(1, double2, true, true);
            }
        } else {
            if (in_f32) {
                if (mb == 2) SPA(2, float2, false, true); else SPA(1, float2, false, true);
            } else {
                if (mb == 2) SPA(2, double2, false, true); else SPA(1, double2, false, true);
            }
        }
#undef SPA
        NUSHT_HIP(hipGetLastError());
        f += groups * mb;
    }
    if (det) {
        hipLaunchKernelGGL(k_spin_adj_reduce, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s,
                           target, nwm, nz, alm);
        NUSHT_HIP(hipGetLastError());
    }
    return NUSHT_OK;
}

}  // namespace nusht
