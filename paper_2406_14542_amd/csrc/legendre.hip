// Legendre step of the iso-latitude transform S (arXiv:2406.14542 Sec. III, "critical part"):
//   synthesis  G_m(theta_j) = sum_{l=m}^{L} a_lm lam_lm(cos theta_j)
//   adjoint    c_lm = sum_j lam_lm(cos theta_j) G'_m(theta_j)
// on the Clenshaw-Curtis rings theta_j = j pi / (N_r - 1).  lam_lm is generated on the fly by
// the three-term recurrence in l (only the O(L^2) coefficient table is stored); the work is
// parallel over rings and m and sequential over l, as the paper describes for SHTns.
//
// gfx950 mapping:
//  * one lane = one pair of mirror rings (j, N_r-1-j): lam_lm(-x) = (-1)^(l+m) lam_lm(x), so
//    one recurrence serves both hemispheres through even/odd-l accumulators;
//  * every lane of a block has the same m, so the recurrence coefficients and a_lm of a step
//    are wave-uniform and are read through the scalar cache;
//  * x * v is formed as v - y v with y = 2 sin^2(theta/2): 1 - cos(theta) keeps full relative
//    precision near the poles, where d lam / d x grows like l^2;
//  * exponent range: lam_mm underflows FP64 for m of a few thousand near the poles.  Each
//    lane carries a count k of 2^256 factors; while any lane of the wave has k > 0 the wave
//    runs a rescaling step, afterwards the plain recurrence.  Terms whose true magnitude is
//    below 2^-200 are dropped (they cannot reach the FP64 result).
#include "internal.h"

namespace nusht {
namespace {

constexpr double kBig = 0x1p56;       // rescale once the scaled value reaches this
constexpr double kUnit = 0x1p-256;    // one scale unit
constexpr int kAccumExp = -200;       // terms below 2^-200 are not accumulated

// lam_mm(theta_j) = c_m sin^m(theta_j), returned as v * 2^(-256 k) with v normal.
__device__ inline void lambda_mm_scaled(double cm, int ce, double s, int m, double& v, int& k)
{
    double mant;
    int e;
    if (m == 0) {
        mant = cm;
        e = ce;
    } else if (s == 0.0) {
        v = 0.0;
        k = 0;
        return;
    } else {
        int be;
        double base = frexp(s, &be);
        double r = 1.0;
        int re = 0;
        int mm = m;
        while (mm) {
            int t;
            if (mm & 1) {
                r *= base;
                re += be;
                r = frexp(r, &t);
                re += t;
            }
            mm >>= 1;
            if (mm) {
                base *= base;
                be *= 2;
                base = frexp(base, &t);
                be += t;
            }
        }
        int t;
        mant = frexp(cm * r, &t);
        e = ce + re + t;
    }
    if (e >= kAccumExp) {
        v = ldexp(mant, e);
        k = 0;
    } else {
        k = (kAccumExp - e + 255) / 256;
        v = ldexp(mant, e + 256 * k);
    }
}

// geometry of ring j of a grid with nr rings: returns (s = sin theta_j, y = 1 - cos theta_j)
__device__ inline void ring_geom(int j, int nr, double& s, double& y)
{
    const double denom = (double)(nr - 1);
    s = sinpi((double)j / denom);
    if (2 * j == nr - 1) {
        y = 1.0;
    } else {
        double h = sinpi((double)j / (2.0 * denom));
        y = 2.0 * h * h;
    }
}

// one recurrence step: returns lam_l from (lam_{l-1} = vc, lam_{l-2} = vp)
__device__ inline double rec_step(double2 c, double y, double vc, double vp)
{
    double xv = fma(-y, vc, vc);
    return fma(c.x, xv, -(c.y * vp));
}

template <int MB>
__device__ inline void accum(double (&acc)[MB][2], const double2* __restrict__ alm, int64_t nalm,
                             int64_t idx, double lam)
{
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        double2 a = alm[b * nalm + idx];
        acc[b][0] = fma(a.x, lam, acc[b][0]);
        acc[b][1] = fma(a.y, lam, acc[b][1]);
    }
}

// ------------------------------------------------------------------------------------
// Synthesis.  FUSED: out[b][m][t], t < N_t, the doubled column of Fig. 1 in (theta, m)
// space: out(t) = G(t) for t < N_r and (-1)^m G(N_t - t) for t >= N_r.  PAPER:
// out[b][j][m], rows of length (N_phi/2 + 1), the input of the per-ring phi-FFT.
// ------------------------------------------------------------------------------------
template <int MB, bool FUSED, typename OutT>
__global__ __launch_bounds__(256) void k_legendre_synth(
    const double2* __restrict__ alm, int64_t nalm, int lmax,
    const double2* __restrict__ rec, const double* __restrict__ cm_mant,
    const int* __restrict__ cm_exp, int nr, int nt, OutT* __restrict__ out,
    int64_t out_map_stride, int64_t out_row_stride)
{
    const int m = blockIdx.y;
    const int npairs = (nr + 1) / 2;
    const int j0 = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = j0 < npairs;
    const int j = active ? j0 : npairs - 1;
    alm += (int64_t)blockIdx.z * MB * nalm;
    out += (int64_t)blockIdx.z * MB * out_map_stride;

    double s, y;
    ring_geom(j, nr, s, y);
    const int64_t moff = (int64_t)m * (2 * lmax + 1 - m) / 2;  // index(l, m) = moff + l

    double E[MB][2], O[MB][2];
#pragma unroll
    for (int b = 0; b < MB; ++b) E[b][0] = E[b][1] = O[b][0] = O[b][1] = 0.0;

    double vc, vp = 0.0;
    int k;
    lambda_mm_scaled(cm_mant[m], cm_exp[m], s, m, vc, k);
    if (k == 0) accum<MB>(E, alm, nalm, moff + m, vc);

    int l = m + 1;
    // scaled phase: some lane of the wave still carries a 2^256 factor
    while (l <= lmax && __any(k > 0)) {
        double vn = rec_step(rec[moff + l], y, vc, vp);
        vp = vc;
        vc = vn;
        const bool big = (k > 0) && (fabs(vc) >= kBig);
        const double sc = big ? kUnit : 1.0;
        vc *= sc;
        vp *= sc;
        k -= big ? 1 : 0;
        const double lam = (k == 0) ? vc : 0.0;
        if ((l - m) & 1)
            accum<MB>(O, alm, nalm, moff + l, lam);
        else
            accum<MB>(E, alm, nalm, moff + l, lam);
        ++l;
    }
    // plain phase, two steps at a time so that the parity of l - m is static
    if (l <= lmax && ((l - m) & 1)) {
        double vn = rec_step(rec[moff + l], y, vc, vp);
        vp = vc;
        vc = vn;
        accum<MB>(O, alm, nalm, moff + l, vc);
        ++l;
    }
    for (; l + 1 <= lmax; l += 2) {
        double vn = rec_step(rec[moff + l], y, vc, vp);
        vp = vc;
        vc = vn;
        accum<MB>(E, alm, nalm, moff + l, vc);
        vn = rec_step(rec[moff + l + 1], y, vc, vp);
        vp = vc;
        vc = vn;
        accum<MB>(O, alm, nalm, moff + l + 1, vc);
    }
    if (l <= lmax) {
        double vn = rec_step(rec[moff + l], y, vc, vp);
        accum<MB>(E, alm, nalm, moff + l, vn);
    }
    if (!active) return;

    const int js = nr - 1 - j;
    const double sgn = (m & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        double nre = E[b][0] + O[b][0], nim = E[b][1] + O[b][1];
        double sre = E[b][0] - O[b][0], sim = E[b][1] - O[b][1];
        if (m == 0) nim = sim = 0.0;  // Im a_l0 is ignored
        OutT* o = out + b * out_map_stride;
        if (FUSED) {
            OutT* col = o + (int64_t)m * out_row_stride;
            col[j] = OutT{nre, nim};
            if (j >= 1 && j <= nr - 2) col[nt - j] = OutT{sgn * nre, sgn * nim};
            if (js != j) {
                col[js] = OutT{sre, sim};
                if (js >= 1 && js <= nr - 2) col[nt - js] = OutT{sgn * sre, sgn * sim};
            }
        } else {
            o[(int64_t)j * out_row_stride + m] = OutT{nre, nim};
            if (js != j) o[(int64_t)js * out_row_stride + m] = OutT{sre, sim};
        }
    }
}

// ------------------------------------------------------------------------------------
// Adjoint.  One block per (m, map); thread t owns ring pairs t, t + T, ..., (R of them).
// Per l the thread forms sum_r lam_lm(x_r) H_r with H = G'(j) + G'(j') for even l - m and
// G'(j) - G'(j') for odd l - m; the block sums these over threads through LDS, CH values
// of l at a time.  FUSED input: Tp[b][m][t] (t < N_t), folded here:
//   G'_m(j) = Tp(j) + [1 <= j <= N_r - 2] (-1)^m Tp(N_t - j)      (D^H of Eq. 6)
// PAPER input: G'[b][j][m] rows of length (N_phi/2 + 1) (output of the per-ring R2C).
// ------------------------------------------------------------------------------------
constexpr int kChunk = 8;
constexpr int kAdjMaxThreads = 640;

template <typename InT>
__device__ inline double2 load_c(const InT* p)
{
    InT v = *p;
    return make_double2((double)v.x, (double)v.y);
}

template <int R, bool FUSED, typename InT>
__global__ __launch_bounds__(kAdjMaxThreads) void k_legendre_adj(
    const InT* __restrict__ in, int64_t in_map_stride, int64_t in_row_stride,
    double2* __restrict__ alm, int64_t nalm, int lmax, const double2* __restrict__ rec,
    const double* __restrict__ cm_mant, const int* __restrict__ cm_exp, int nr, int nt)
{
    __shared__ double red[2 * kChunk][kAdjMaxThreads];
    const int m = blockIdx.x;
    const int map = blockIdx.y;
    const int T = blockDim.x;
    const int tid = threadIdx.x;
    const int npairs = (nr + 1) / 2;
    in += (int64_t)map * in_map_stride;
    alm += (int64_t)map * nalm;
    const int64_t moff = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const double sgn = (m & 1) ? -1.0 : 1.0;

    double y[R], vc[R], vp[R], Sr[R], Si[R], Dr[R], Di[R];
    int k[R];
    bool scaled = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int jr = tid + r * T;
        const bool valid = jr < npairs;
        const int j = valid ? jr : 0;
        const int js = nr - 1 - j;
        double s;
        ring_geom(j, nr, s, y[r]);
        double2 gn, gs;
        if (FUSED) {
            const InT* col = in + (int64_t)m * in_row_stride;
            gn = load_c(col + j);
            if (j >= 1 && j <= nr - 2) {
                double2 t = load_c(col + (nt - j));
                gn.x += sgn * t.x;
                gn.y += sgn * t.y;
            }
            gs = load_c(col + js);
            if (js >= 1 && js <= nr - 2) {
                double2 t = load_c(col + (nt - js));
                gs.x += sgn * t.x;
                gs.y += sgn * t.y;
            }
        } else {
            gn = load_c(in + (int64_t)j * in_row_stride + m);
            gs = load_c(in + (int64_t)js * in_row_stride + m);
        }
        if (!valid) {
            gn = gs = make_double2(0.0, 0.0);
        }
        if (js == j) {  // the equator ring (odd N_r) is its own mirror: count it once
            Sr[r] = gn.x;
            Si[r] = gn.y;
            Dr[r] = gn.x;
            Di[r] = gn.y;
        } else {
            Sr[r] = gn.x + gs.x;
            Si[r] = gn.y + gs.y;
            Dr[r] = gn.x - gs.x;
            Di[r] = gn.y - gs.y;
        }
        vp[r] = 0.0;
        lambda_mm_scaled(cm_mant[m], cm_exp[m], s, m, vc[r], k[r]);
        scaled |= k[r] > 0;
    }

    const int nwaves = (T + 63) / 64;
    const int wave = tid / 64, lane = tid % 64;
    for (int l0 = m; l0 <= lmax; l0 += kChunk) {
        double pr[kChunk], pi[kChunk];
#pragma unroll
        for (int i = 0; i < kChunk; ++i) {
            const int l = l0 + i;
            pr[i] = pi[i] = 0.0;
            if (l > lmax) continue;
            const bool even = ((l - m) & 1) == 0;
            if (l > m) {
                const double2 c = rec[moff + l];
                const bool wscaled = __any(scaled);
                bool still = false;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double vn = rec_step(c, y[r], vc[r], vp[r]);
                    vp[r] = vc[r];
                    vc[r] = vn;
                    if (wscaled) {
                        const bool big = (k[r] > 0) && (fabs(vc[r]) >= kBig);
                        const double sc = big ? kUnit : 1.0;
                        vc[r] *= sc;
                        vp[r] *= sc;
                        k[r] -= big ? 1 : 0;
                        still |= k[r] > 0;
                    }
                }
                if (wscaled) scaled = still;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double lam = (k[r] == 0) ? vc[r] : 0.0;
                pr[i] = fma(lam, even ? Sr[r] : Dr[r], pr[i]);
                pi[i] = fma(lam, even ? Si[r] : Di[r], pi[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < kChunk; ++i) {
            red[2 * i][tid] = pr[i];
            red[2 * i + 1][tid] = pi[i];
        }
        __syncthreads();
        for (int v = wave; v < 2 * kChunk; v += nwaves) {
            double acc = 0.0;
            for (int q = lane; q < T; q += 64) acc += red[v][q];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
            const int l = l0 + v / 2;
            if (lane == 0 && l <= lmax) {
                double* dst = reinterpret_cast<double*>(alm + moff + l);
                dst[v & 1] = (m == 0 && (v & 1)) ? 0.0 : acc;
            }
        }
        __syncthreads();
    }
}

}  // namespace

int launch_legendre_synth(const nusht_plan_s* p, const double* alm, void* out, int nmaps,
                          int fused, int out_f32, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int npairs = (g.nrings + 1) / 2;
    const int threads = npairs >= 256 ? 256 : ((npairs + 63) / 64) * 64;
    const int bx = (npairs + threads - 1) / threads;
    const int64_t nalm = g.nalm;
    const double2* a = reinterpret_cast<const double2*>(alm);
    int64_t map_stride, row_stride;
    if (fused) {
        row_stride = g.ntorus;
        map_stride = (int64_t)(g.mmax + 1) * g.ntorus;
    } else {
        row_stride = g.nphi / 2 + 1;
        map_stride = (int64_t)g.nrings * row_stride;
    }
    int b = 0;
    while (b < nmaps) {
        const int left = nmaps - b;
        const int mb = left >= 4 ? 4 : (left >= 2 ? 2 : 1);
        const int groups = left / mb;
        dim3 grid(bx, g.mmax + 1, groups);
        const double2* ab = a + (int64_t)b * nalm;
#define SYN(MBV, F, OT)                                                                          \
    hipLaunchKernelGGL((k_legendre_synth<MBV, F, OT>), grid, dim3(threads), 0, s, ab, nalm,       \
                       g.lmax, p->rec, p->cm_mant, p->cm_exp, g.nrings, g.ntorus,                \
                       reinterpret_cast<OT*>(out) + (int64_t)b * map_stride, map_stride,          \
                       row_stride)
        if (fused && out_f32) {
            if (mb == 4) SYN(4, true, float2);
            else if (mb == 2) SYN(2, true, float2);
            else SYN(1, true, float2);
        } else if (fused) {
            if (mb == 4) SYN(4, true, double2);
            else if (mb == 2) SYN(2, true, double2);
            else SYN(1, true, double2);
        } else {
            if (mb == 4) SYN(4, false, double2);
            else if (mb == 2) SYN(2, false, double2);
            else SYN(1, false, double2);
        }
#undef SYN
        NUSHT_HIP(hipGetLastError());
        b += groups * mb;
    }
    return NUSHT_OK;
}

int launch_legendre_adjoint(const nusht_plan_s* p, const void* in, double* alm, int nmaps,
                            int fused, int in_f32, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int npairs = (g.nrings + 1) / 2;
    int R = 1;
    while (R < 16 && R * kAdjMaxThreads < npairs) R *= 2;
    if (R * kAdjMaxThreads < npairs) {
        set_last_error("legendre_adjoint", "too many rings for one block");
        return NUSHT_EINVAL;
    }
    int threads = (npairs + R - 1) / R;
    threads = ((threads + 63) / 64) * 64;
    int64_t map_stride, row_stride;
    if (fused) {
        row_stride = g.ntorus;
        map_stride = (int64_t)(g.mmax + 1) * g.ntorus;
    } else {
        row_stride = g.nphi / 2 + 1;
        map_stride = (int64_t)g.nrings * row_stride;
    }
    dim3 grid(g.mmax + 1, nmaps);
    double2* out = reinterpret_cast<double2*>(alm);
#define ADJ(RV, F, IT)                                                                          \
    hipLaunchKernelGGL((k_legendre_adj<RV, F, IT>), grid, dim3(threads), 0, s,                   \
                       reinterpret_cast<const IT*>(in), map_stride, row_stride, out, g.nalm,      \
                       g.lmax, p->rec, p->cm_mant, p->cm_exp, g.nrings, g.ntorus)
#define ADJR(F, IT)                 \
    switch (R) {                    \
        case 1: ADJ(1, F, IT); break; \
        case 2: ADJ(2, F, IT); break; \
        case 4: ADJ(4, F, IT); break; \
        case 8: ADJ(8, F, IT); break; \
        default: ADJ(16, F, IT); break; \
    }
    if (fused && in_f32) {
        ADJR(true, float2);
    } else if (fused) {
        ADJR(true, double2);
    } else {
        ADJR(false, double2);
    }
#undef ADJR
#undef ADJ
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

}  // namespace nusht
