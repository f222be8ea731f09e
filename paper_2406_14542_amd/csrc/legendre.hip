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

// The coefficient stream of one m (recurrence table and MB coefficient rows) is read through
// the scalar cache, one l at a time, by every wave of that m; a miss costs a trip to HBM that
// the few resident waves cannot hide.  Every kPfStep values of l the wave therefore touches
// the next kPfStep coefficients of each stream, kPfStep steps ahead, with one load per
// 128-byte line, so that the scalar loads find them in L2.  The touch is an LDS-DMA load
// (global_load_lds_dword) in inline assembly: it has no register destination, so the
// compiler never waits for it, and the statement is declared free of memory effects, so the
// compiler still knows the coefficients are read-only and keeps their loads scalar.  (It
// does write LDS: a per-wave sink that nothing reads; the wave waits for the DMA once,
// before its LDS is released.)  M0, the DMA's LDS base, is restored afterwards.  The
// statement returns the saved M0 so that it stays live; the caller folds it into a value
// consumed at the end.
constexpr int kPfStep = 32;
constexpr int kPfLines = kPfStep * 16 / 128 + 1;  // lines per stream (unaligned start)

__device__ inline unsigned lds_dma_touch(const void* src, unsigned lds_sink)
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

template <int MB>
__device__ inline unsigned prefetch_coeffs(const double2* __restrict__ rec,
                                           const double2* __restrict__ alm, int64_t nalm,
                                           int64_t moff, int lmax, int lp, int lane,
                                           unsigned lds_sink)
{
    const int stream = lane / kPfLines, line = lane - stream * kPfLines;
    if (stream > MB || lp > lmax) return 0u;
    const int64_t idx = moff + min(lp + 8 * line, lmax);
    const double2* src = (stream == 0 ? rec : alm + (int64_t)(stream - 1) * nalm) + idx;
    return lds_dma_touch(src, lds_sink);
}

// ------------------------------------------------------------------------------------
// Synthesis.  FUSED: out[b][m][t], t < N_t, the doubled column of Fig. 1 in (theta, m)
// space: out(t) = G(t) for t < N_r and (-1)^m G(N_t - t) for t >= N_r.  PAPER:
// out[b][j][m], rows of length (N_phi/2 + 1), the input of the per-ring phi-FFT.
// ------------------------------------------------------------------------------------
template <typename OutT>
__device__ inline OutT make_out(double re, double im)
{
    OutT o;
    o.x = re;
    o.y = im;
    return o;
}

// XCD-aware placement: workgroups are handed to the 8 XCDs round-robin by linear id, and
// every XCD has its own L2.  Block id b = 8 q + x goes to XCD x; the q-th block of XCD x
// gets (m, ring block) = (8 (q / nbx) + x, q % nbx), so all nbx ring blocks of one m run
// on the same XCD at about the same time and fetch that m's coefficient stream into one
// L2 once.  The grid is (nbx * mpad, groups) with mpad = mmax + 1 rounded up to 8.
__device__ inline void xcd_block(int b, int nbx, int& m, int& rb)
{
    const int x = b & 7, q = b >> 3;
    m = 8 * (q / nbx) + x;
    rb = q % nbx;
}

// Each lane owns R ring pairs j = base + lane + 64 r; a wave therefore covers 64 R
// consecutive pairs and loads every coefficient once for all of them.
//
// The kernel comes in two instances.  Ring pairs j >= jscale[m] have lam_mm above 2^-190,
// so none of their lam_lm ever needs the power-of-two scale; their waves run the
// SCALED = false instance, which has no scaled step at all (the scaled step's extra live
// registers would otherwise cost the whole kernel almost half of its occupancy).  The pairs
// below jscale[m] (a multiple of 64 R of both instances, so that their waves partition the
// pairs) run SCALED = true.
template <int MB, int R, bool FUSED, typename OutT, bool SCALED>
__global__ __launch_bounds__(256) void k_legendre_synth(
    const double2* __restrict__ alm, int64_t nalm, int lmax, int mmax, int nbx,
    const double2* __restrict__ rec, const double* __restrict__ cm_mant,
    const int* __restrict__ cm_exp, const int* __restrict__ jlive,
    const int* __restrict__ jscale, int nr, int nt, OutT* __restrict__ out,
    int64_t out_map_stride, int64_t out_row_stride)
{
    int m, rb;
    xcd_block(blockIdx.x, nbx, m, rb);
    if (m > mmax) return;
    const int npairs = (nr + 1) / 2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wbase = (rb * (blockDim.x >> 6) + wave) * 64 * R;
    if (wbase >= npairs) return;
    if (SCALED != (wbase < jscale[m])) return;  // the other instance owns this wave
    alm += (int64_t)blockIdx.y * MB * nalm;
    out += (int64_t)blockIdx.y * MB * out_map_stride;
    const int64_t moff = (int64_t)m * (2 * lmax + 1 - m) / 2;  // index(l, m) = moff + l
    const bool wave_dead = wbase + 64 * R <= jlive[m];
    __shared__ float pf_sink[4][64];

    double E[R][MB][2], O[R][MB][2];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int b = 0; b < MB; ++b) E[r][b][0] = E[r][b][1] = O[r][b][0] = O[r][b][1] = 0.0;

    if (!wave_dead) {
        double y[R], vc[R], vp[R];
        int k[R];
        bool any_scaled = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = min(wbase + lane + 64 * r, npairs - 1);
            double s;
            ring_geom(j, nr, s, y[r]);
            vp[r] = 0.0;
            lambda_mm_scaled(cm_mant[m], cm_exp[m], s, m, vc[r], k[r]);
            if (!SCALED && k[r] != 0) {
                // cannot happen above jscale (10 bits of margin); drop rather than misuse
                vc[r] = 0.0;
                k[r] = 0;
            }
            if (k[r] == 0) accum<MB>(E[r], alm, nalm, moff + m, vc[r]);
            any_scaled |= k[r] > 0;
        }
        // Steps run in (even, odd) pairs of l - m after the first (odd) one, so that the
        // accumulator of every step is static.  While some lane of the wave still carries a
        // 2^256 factor the wave takes the scaled step; the branch is wave-uniform and both
        // sides update the same accumulators in place.
        auto scaled_step = [&](const double2 c, int64_t idx, double (&A)[R][MB][2]) {
            any_scaled = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double vn = rec_step(c, y[r], vc[r], vp[r]);
                vp[r] = vc[r];
                vc[r] = vn;
                const bool big = (k[r] > 0) && (fabs(vc[r]) >= kBig);
                const double sc = big ? kUnit : 1.0;
                vc[r] *= sc;
                vp[r] *= sc;
                k[r] -= big ? 1 : 0;
                any_scaled |= k[r] > 0;
                accum<MB>(A[r], alm, nalm, idx, (k[r] == 0) ? vc[r] : 0.0);
            }
        };
        auto plain_step = [&](const double2 c, int64_t idx, double (&A)[R][MB][2]) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double vn = rec_step(c, y[r], vc[r], vp[r]);
                vp[r] = vc[r];
                vc[r] = vn;
                accum<MB>(A[r], alm, nalm, idx, vc[r]);
            }
        };
        int l = m + 1;
        if (l <= lmax) {
            if (SCALED && __any(any_scaled))
                scaled_step(rec[moff + l], moff + l, O);
            else
                plain_step(rec[moff + l], moff + l, O);
            ++l;
        }
        int pf_at = l;
        unsigned pf_keep = 0;
        const unsigned lds_sink = __builtin_amdgcn_readfirstlane(
            (unsigned)(uintptr_t)(__attribute__((address_space(3))) float*)pf_sink[wave]);
        auto prefetch = [&]() {
            if (l >= pf_at) {
                pf_keep ^= prefetch_coeffs<MB>(rec, alm, nalm, moff, lmax, l + kPfStep, lane,
                                               lds_sink);
                pf_at = l + kPfStep;
            }
        };
        if (SCALED) {
            // Phase 1: no lane has reached the accumulation range (every accumulator is still
            // zero), so the steps run the recurrence and its rescaling only.  The rescale test
            // is made once per pair: one step grows a value by less than 2^7, far from the
            // FP64 range above kBig.  The pair in which some lane reaches k = 0 accumulates
            // both of its values for those lanes (a value one step before k reached 0 is
            // below 2^-200 times its coefficient: kept, not dropped).
            bool reached = false;
#pragma unroll
            for (int r = 0; r < R; ++r) reached |= k[r] == 0;
            if (!__any(reached)) {
                for (; l + 1 <= lmax; l += 2) {
                    const double2 c0 = rec[moff + l], c1 = rec[moff + l + 1];
                    reached = false;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const double v0 = rec_step(c0, y[r], vc[r], vp[r]);
                        const double v1 = rec_step(c1, y[r], v0, vc[r]);
                        const bool big = fmax(fabs(v0), fabs(v1)) >= kBig;
                        const double sc = big ? kUnit : 1.0;
                        vp[r] = v0 * sc;
                        vc[r] = v1 * sc;
                        k[r] -= big ? 1 : 0;
                        reached |= k[r] == 0;
                    }
                    if (__any(reached)) {
                        prefetch();
                        any_scaled = false;
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const bool live = k[r] == 0;
                            any_scaled |= !live;
                            accum<MB>(E[r], alm, nalm, moff + l, live ? vp[r] : 0.0);
                            accum<MB>(O[r], alm, nalm, moff + l + 1, live ? vc[r] : 0.0);
                        }
                        l += 2;
                        break;
                    }
                }
            }
            // Phase 2: some lane still carries a scale factor: the rescale test once per pair
            // of steps, as in phase 1, and the pair's two values accumulated for the lanes
            // whose count is zero after it (scaling by 2^-256 is exact, so the values are the
            // ones a per-step test would give).
            for (; l + 1 <= lmax && __any(any_scaled); l += 2) {
                prefetch();
                const double2 c0 = rec[moff + l], c1 = rec[moff + l + 1];
                any_scaled = false;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double v0 = rec_step(c0, y[r], vc[r], vp[r]);
                    const double v1 = rec_step(c1, y[r], v0, vc[r]);
                    const bool big = (k[r] > 0) && fmax(fabs(v0), fabs(v1)) >= kBig;
                    const double sc = big ? kUnit : 1.0;
                    vp[r] = v0 * sc;
                    vc[r] = v1 * sc;
                    k[r] -= big ? 1 : 0;
                    const bool live = k[r] == 0;
                    any_scaled |= !live;
                    accum<MB>(E[r], alm, nalm, moff + l, live ? vp[r] : 0.0);
                    accum<MB>(O[r], alm, nalm, moff + l + 1, live ? vc[r] : 0.0);
                }
            }
        }
        // Phase 3: every lane is in plain FP64 range.
        for (; l + 1 <= lmax; l += 2) {
            prefetch();
            const double2 c0 = rec[moff + l], c1 = rec[moff + l + 1];
            plain_step(c0, moff + l, E);
            plain_step(c1, moff + l + 1, O);
        }
        if (l <= lmax) {
            if (SCALED && __any(any_scaled))
                scaled_step(rec[moff + l], moff + l, E);
            else
                plain_step(rec[moff + l], moff + l, E);
        }
        // no LDS-DMA write may be in flight when the workgroup's LDS is released
        asm volatile("s_waitcnt vmcnt(0)" ::"v"(pf_keep) : "memory");
    }

    const double sgn = (m & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = wbase + lane + 64 * r;
        if (j >= npairs) continue;
        const int js = nr - 1 - j;
#pragma unroll
        for (int b = 0; b < MB; ++b) {
            double nre = E[r][b][0] + O[r][b][0], nim = E[r][b][1] + O[r][b][1];
            double sre = E[r][b][0] - O[r][b][0], sim = E[r][b][1] - O[r][b][1];
            if (m == 0) nim = sim = 0.0;  // Im a_l0 is ignored
            OutT* o = out + b * out_map_stride;
            if (FUSED) {
                OutT* col = o + (int64_t)m * out_row_stride;
                col[j] = make_out<OutT>(nre, nim);
                if (j >= 1 && j <= nr - 2) col[nt - j] = make_out<OutT>(sgn * nre, sgn * nim);
                if (js != j) {
                    col[js] = make_out<OutT>(sre, sim);
                    if (js >= 1 && js <= nr - 2) col[nt - js] = make_out<OutT>(sgn * sre, sgn * sim);
                }
            } else {
                o[(int64_t)j * out_row_stride + m] = make_out<OutT>(nre, nim);
                if (js != j) o[(int64_t)js * out_row_stride + m] = make_out<OutT>(sre, sim);
            }
        }
    }
}

// ------------------------------------------------------------------------------------
// Adjoint.  c_lm = sum_j lam_lm(x_j) G'_m(theta_j) is, for one m, a product of the
// (L - m + 1) x N_r matrix of lam values (generated by the recurrence) with the N_r x
// (2 B) matrix of ring data, reduced over rings.  gfx950 mapping:
//  * one lane = one ring pair (j, N_r-1-j): lam_lm(-x) = (-1)^(l+m) lam_lm(x), so the pair
//    enters through its even (N + S) and odd (N - S) combinations, chosen by the parity of
//    l - m; the lane runs the recurrence for 16 consecutive l and parks the values in LDS;
//  * the reduction over ring pairs runs on v_mfma_f64_4x4x4_4b: four 4x4x4 products per
//    instruction, one for each (parity, real/imaginary) pair, with rows = the 4 maps,
//    K = 4 ring pairs and columns = 4 values of l of that parity -- every product term is
//    used (the 16x16x4 shape would spend half of its work on the wrong parity) and this
//    shape sustains close to the FP64 peak on gfx950, the 16x16 one about 60 % of it;
//  * the waves of a block (one pair-chunk) are summed without workgroup barriers: each wave
//    adds its D values of a round of kAdjGroup chunks into one of kAdjSlots LDS slots (LDS
//    FP64 atomics) and counts itself in; the last of the block's live waves to arrive adds
//    the slot into the output, clears it and hands it on to the round kAdjSlots later.  The
//    waves therefore run at their own pace (scaled and unscaled lanes, dead waves) instead of
//    meeting at two barriers after every round;
//  * the pair-chunks of one m run on one XCD and add their sums into the zeroed output with
//    FP64 atomics that resolve in that XCD's L2 (the order of the additions is not fixed:
//    results can differ between runs by FP64 rounding).
// Input: FUSED Tp[b][m][t] (t < N_t), folded here:
//   G'_m(j) = Tp(j) + [1 <= j <= N_r - 2] (-1)^m Tp(N_t - j)      (D^H of Eq. 6)
// PAPER G'[b][j][m] rows of length (N_phi/2 + 1) (output of the per-ring R2C).
// ------------------------------------------------------------------------------------
constexpr int kAdjWaves = 4;     // waves per block: one block reduces up to 256 ring pairs
constexpr int kLC = 16;          // l values per chunk = the MFMA N dimension
constexpr int kLS = kLC + 1;     // padded row of the lam staging area
constexpr int kAdjGroup = 2;     // chunks whose sums go through one slot together
constexpr int kAdjSlots = 2;     // slots in flight per block (power of two)
constexpr int kAdjPfAhead = 4;   // chunks between a coefficient line's L2 touch and its use
constexpr int kAdjSpinLimit = 1 << 22;  // sleeps before a slot wait gives up (never reached)


template <typename InT>
__device__ inline double2 load_c(const InT* p)
{
    InT v = *p;
    return make_double2((double)v.x, (double)v.y);
}

template <bool FUSED, typename InT, bool DET>
__global__ __launch_bounds__(kAdjWaves * 64, DET ? 3 : 4) void k_legendre_adj(
    const InT* __restrict__ in, int64_t in_map_stride, int64_t in_row_stride, int nmaps,
    double* __restrict__ alm, int npc, int64_t nalm, int lmax,
    const double2* __restrict__ rec, const double* __restrict__ cm_mant,
    const int* __restrict__ cm_exp, const int* __restrict__ jlive, int nr, int nt,
    int pairs_per_block, int mmax, int* __restrict__ err)
{
    // per wave: the lam values of one chunk (64 pairs x 16 l); per block: the chunk-sum slots
    // (128 D values: 64 lanes x real/imaginary), their arrival counts and hand-on counts
    __shared__ double stage[kAdjWaves][64 * kLS];
    __shared__ float pf_sink[kAdjWaves][64];
    // DET: one region per wave, summed in wave order by the flushing wave (fixed order)
    constexpr int kSlotWaves = DET ? kAdjWaves : 1;
    __shared__ double slot[kAdjSlots][kSlotWaves][kAdjGroup * 128];
    __shared__ unsigned scnt[kAdjSlots], sgen[kAdjSlots];
    static_assert((kAdjSlots & (kAdjSlots - 1)) == 0, "slot count a power of two");
    // all pair-chunks of one m on one XCD, one after the other: they share the m's
    // coefficient stream in that XCD's L2
    int m, pc;
    xcd_block(blockIdx.x, npc, m, pc);
    if (m > mmax) return;
    // DET: alm is the partial-sum array [npc][nmaps][nalm] (complex); this block's part
    if (DET) alm += (int64_t)pc * nmaps * nalm * 2;
    const int grp = blockIdx.y;
    const int nmb = min(4, nmaps - 4 * grp);
    // the wave index read through a scalar register: everything derived from it (dead waves,
    // the slot protocol) is then known to be wave-uniform
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nwaves = blockDim.x >> 6;
    const int npairs = (nr + 1) / 2;
    const int local = wave * 64 + lane;
    const int pair = pc * pairs_per_block + local;
    const bool valid = local < pairs_per_block && pair < npairs;
    const int j = valid ? pair : 0;
    const int js = nr - 1 - j;
    const int64_t moff = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const double msgn = (m & 1) ? -1.0 : 1.0;
    in += (int64_t)(4 * grp) * in_map_stride;
    double* st = stage[wave];
    const int jl = jlive[m];
    // pairs below jl never carry lam above 2^-300 for l <= lmax: a block made only of them
    // writes zero partial sums, a wave made only of them skips its recurrence and MFMAs
    if (pc * pairs_per_block + pairs_per_block <= jl) return;
    // a wave is dead when all its pairs lie below the live-ring bound or beyond the pairs
    const int wfirst = pc * pairs_per_block + wave * 64;
    const bool wave_dead = wfirst + 64 <= jl || wave * 64 >= pairs_per_block || wfirst >= npairs;

    // ring data of this lane's pair: rows 4 b + {N re, N im, S re, S im}.  All loads are
    // issued before any is used (indices clamped into range, unused ones weighted by 0).
    {
        double2 raw[4][4];
        double wgt[4];
        int64_t off[4];
        if (FUSED) {
            // G'(j) = Tp(j) + [1 <= j <= N_r - 2] (-1)^m Tp(N_t - j), likewise for js
            off[0] = j;
            off[1] = (j >= 1 && j <= nr - 2) ? nt - j : j;
            off[2] = js;
            off[3] = (js >= 1 && js <= nr - 2) ? nt - js : js;
            wgt[0] = 1.0;
            wgt[1] = (j >= 1 && j <= nr - 2) ? msgn : 0.0;
            wgt[2] = js != j ? 1.0 : 0.0;
            wgt[3] = (js != j && js >= 1 && js <= nr - 2) ? msgn : 0.0;
            for (int q = 0; q < 4; ++q) off[q] += (int64_t)m * in_row_stride;
        } else {
            off[0] = (int64_t)j * in_row_stride + m;
            off[2] = (int64_t)js * in_row_stride + m;
            off[1] = off[0];
            off[3] = off[2];
            wgt[0] = 1.0;
            wgt[1] = 0.0;
            wgt[2] = js != j ? 1.0 : 0.0;
            wgt[3] = 0.0;
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int bb = b < nmb ? b : 0;
            const InT* im = in + (int64_t)bb * in_map_stride;
#pragma unroll
            for (int q = 0; q < 4; ++q) raw[b][q] = load_c(im + off[q]);
        }
        // hv[(2 h + c) * 4 + map]: h = 0 the even combination N + S, h = 1 the odd one
        // N - S (lam_lm(-x) = (-1)^(l+m) lam_lm(x)); c = 0 real, 1 imaginary part
        double hv[16];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const double use = (valid && b < nmb) ? 1.0 : 0.0;
            const double nre = use * (wgt[0] * raw[b][0].x + wgt[1] * raw[b][1].x);
            const double nim = use * (wgt[0] * raw[b][0].y + wgt[1] * raw[b][1].y);
            const double sre = use * (wgt[2] * raw[b][2].x + wgt[3] * raw[b][3].x);
            const double sim = use * (wgt[2] * raw[b][2].y + wgt[3] * raw[b][3].y);
            hv[0 * 4 + b] = nre + sre;
            hv[1 * 4 + b] = nim + sim;
            hv[2 * 4 + b] = nre - sre;
            hv[3 * 4 + b] = nim - sim;
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) st[lane * kLS + c] = hv[c];
    }
    for (int e = threadIdx.x; e < kAdjSlots * kSlotWaves * kAdjGroup * 128; e += blockDim.x)
        (&slot[0][0][0])[e] = 0.0;
    if (threadIdx.x < kAdjSlots) {
        scnt[threadIdx.x] = 0;
        sgen[threadIdx.x] = 0;
    }
    __syncthreads();
    // D of v_mfma_f64_4x4x4_4b (measured layout: A_b[i][k] in lane i + 4 b + 16 k,
    // B_b[k][j] in lane j + 4 b + 16 k, D_b[i][j] in lane j + 4 b + 16 i).  Here k = ring
    // pair of the group of four, block b = 2 s + h selects l = l0 + 8 s + 2 j + h of the
    // chunk (s: half-chunk, h: parity of l - l0), so that the four blocks of one B operand
    // hold 16 distinct lam values and every lam value is read from LDS once; i = map, and
    // the real and imaginary parts (c) are two MFMAs on the same B.
    const int kk = lane >> 4, bb = (lane >> 2) & 3, jj = lane & 3;
    const int lidx = 8 * (bb >> 1) + 2 * jj + (bb & 1);  // this lane's l - l0 in B
    // A operand of MFMA (q, c): ring data of pair 4 q + k, part c of the combination of
    // parity h, map i
    double aop[2][16];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int q = 0; q < 16; ++q)
            aop[c][q] = st[(4 * q + kk) * kLS + (2 * (bb & 1) + c) * 4 + jj];
    __syncthreads();

    double s, y;
    ring_geom(j, nr, s, y);
    double vc, vp = 0.0;
    int k;
    lambda_mm_scaled(cm_mant[m], cm_exp[m], s, m, vc, k);
    if (!valid) {
        vc = 0.0;
        k = 0;
    }
    bool scaled = k > 0;
    unsigned pf_keep = 0;
    const unsigned lds_sink = __builtin_amdgcn_readfirstlane(
        (unsigned)(uintptr_t)(__attribute__((address_space(3))) float*)pf_sink[wave]);

    // the coefficient lines of chunks 1 .. kAdjPfAhead (later chunks are touched kAdjPfAhead
    // chunks ahead of their use inside the loop)
    if (!wave_dead && lane < 2 * kAdjPfAhead && m + kLC + 8 * lane <= lmax)
        pf_keep ^= lds_dma_touch(rec + moff + m + kLC + 8 * lane, lds_sink);
    const int nchunks = (lmax - m) / kLC + 1;
    // the table is read through the constant address space: it is never written while the
    // kernel runs, so its wave-uniform reads stay scalar loads next to the atomics below
    const __attribute__((address_space(4))) double* crec =
        (const __attribute__((address_space(4))) double*)rec;
    // the block's live waves take part in the chunk sums; the dead ones leave (they issued no
    // LDS-DMA touches)
    int nlive = 0;
    for (int w = 0; w < nwaves; ++w) {
        const int wf = pc * pairs_per_block + w * 64;
        nlive += (wf + 64 <= jl || w * 64 >= pairs_per_block || wf >= npairs) ? 0 : 1;
    }
    if (wave_dead) return;
    // Cross-wave sums: the wave adds its D values of round r (chunks kAdjGroup r ..) into slot
    // r % kAdjSlots and counts itself in; the wave that completes the count adds the slot into
    // the output, clears it and hands it on to round r + kAdjSlots.
    for (int c0 = 0; c0 < nchunks; c0 += kAdjGroup) {
        double dv[kAdjGroup][2];
#pragma unroll
        for (int g = 0; g < kAdjGroup; ++g) {
            double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
            const int l0 = m + (c0 + g) * kLC;
            if (c0 + g < nchunks) {
                // the chunk's recurrence coefficients in one batch of scalar loads (the table
                // is padded past its end), and the lines of the chunk kAdjPfAhead ahead
                // touched into L2
                double2 cc[kLC];
#pragma unroll
                for (int i = 0; i < kLC; ++i)
                    cc[i] = make_double2(crec[2 * (moff + l0 + i)], crec[2 * (moff + l0 + i) + 1]);
                if (lane < 3 && l0 + kAdjPfAhead * kLC <= lmax)
                    pf_keep ^= lds_dma_touch(rec + moff + l0 + kAdjPfAhead * kLC + 8 * lane,
                                             lds_sink);
                double lam[kLC];
                const bool full = l0 > m && l0 + kLC - 1 <= lmax;
                if (full && !__any(scaled)) {
                    // common case: a full chunk past lam_mm with no lane scaled
#pragma unroll
                    for (int i = 0; i < kLC; ++i) {
                        const double vn = rec_step(cc[i], y, vc, vp);
                        vp = vc;
                        vc = vn;
                        lam[i] = vc;
                    }
                } else if (full) {
                    // a full chunk with some lane still scaled: the rescale test once per
                    // pair of steps (a step grows a value by less than 2^7, far from the
                    // FP64 range above kBig); a pair's values count once its lane is in range
#pragma unroll
                    for (int i = 0; i < kLC; i += 2) {
                        const double v0 = rec_step(cc[i], y, vc, vp);
                        const double v1 = rec_step(cc[i + 1], y, v0, vc);
                        const bool big = (k > 0) && fmax(fabs(v0), fabs(v1)) >= kBig;
                        const double sc = big ? kUnit : 1.0;
                        vp = v0 * sc;
                        vc = v1 * sc;
                        k -= big ? 1 : 0;
                        lam[i] = (k == 0) ? vp : 0.0;
                        lam[i + 1] = (k == 0) ? vc : 0.0;
                    }
                    scaled = k > 0;
                } else {
                    // the first chunk (lam_mm) and a partial last one: per-step tests
                    const bool wscaled = __any(scaled);
#pragma unroll
                    for (int i = 0; i < kLC; ++i) {
                        const int l = l0 + i;
                        if (l > lmax) {
                            lam[i] = 0.0;
                            continue;
                        }
                        if (l > m) {
                            const double vn = rec_step(cc[i], y, vc, vp);
                            vp = vc;
                            vc = vn;
                            if (wscaled) {
                                const bool big = (k > 0) && (fabs(vc) >= kBig);
                                const double sc = big ? kUnit : 1.0;
                                vc *= sc;
                                vp *= sc;
                                k -= big ? 1 : 0;
                            }
                        }
                        lam[i] = (k == 0) ? vc : 0.0;
                    }
                    scaled = k > 0;
                }
                // a chunk after which every live lane still carries a scale factor has only
                // zero lam values (k never increases): it adds nothing
                if (!__all(scaled || !valid)) {
#pragma unroll
                    for (int i = 0; i < kLC; ++i) st[lane * kLS + i] = lam[i];
                    // the wave reads back only its own staging rows
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                    for (int q = 0; q < 16; q += 2) {
                        const double b0 = st[(4 * q + kk) * kLS + lidx];
                        const double b1 = st[(4 * (q + 1) + kk) * kLS + lidx];
                        acc0 = __builtin_amdgcn_mfma_f64_4x4x4f64(aop[0][q], b0, acc0, 0, 0, 0);
                        acc2 = __builtin_amdgcn_mfma_f64_4x4x4f64(aop[1][q], b0, acc2, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f64_4x4x4f64(aop[0][q + 1], b1, acc1, 0, 0,
                                                                  0);
                        acc3 = __builtin_amdgcn_mfma_f64_4x4x4f64(aop[1][q + 1], b1, acc3, 0, 0,
                                                                  0);
                    }
                    // the next chunk rewrites the staging rows: all lanes' reads come first
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
            }
            dv[g][0] = acc0 + acc1;
            dv[g][1] = acc2 + acc3;
        }
        // this wave's share of the round into slot r % kAdjSlots, once the round kAdjSlots
        // earlier has been taken out of it.  A slot is handed on as soon as the slowest live
        // wave has added into it, so the slowest wave never waits here and every wait ends; the
        // bound only keeps a broken invariant from hanging the device, and a wave that reaches
        // it sets the error word (the host reports NUSHT_EDEVICE: the sums may be wrong).
        const int rnd = c0 / kAdjGroup;
        const int sl = rnd & (kAdjSlots - 1);
        const unsigned use = (unsigned)(rnd / kAdjSlots);
        bool ready = false;
        for (int it = 0; it < kAdjSpinLimit; ++it) {
            if (__hip_atomic_load(&sgen[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) ==
                use) {
                ready = true;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!ready && lane == 0)
            __hip_atomic_fetch_or(err, kErrAdjWait, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
        for (int g = 0; g < kAdjGroup; ++g) {
            if (DET) {
                slot[sl][DET ? wave : 0][g * 128 + lane] = dv[g][0];
                slot[sl][DET ? wave : 0][g * 128 + 64 + lane] = dv[g][1];
            } else {
                __hip_atomic_fetch_add(&slot[sl][0][g * 128 + lane], dv[g][0], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_fetch_add(&slot[sl][0][g * 128 + 64 + lane], dv[g][1],
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        unsigned arrived = 0;
        if (lane == 0)
            arrived = __hip_atomic_fetch_add(&scnt[sl], 1u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP);
        arrived = __builtin_amdgcn_readfirstlane(arrived);
        if ((int)arrived == nlive - 1) {
            // last arrival: the slot holds the block's sums of this round
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            double v[kAdjGroup][2];
#pragma unroll
            for (int g = 0; g < kAdjGroup; ++g) {
                if (DET) {
                    // waves in order; a dead wave's region stays zero
                    v[g][0] = v[g][1] = 0.0;
                    for (int w = 0; w < nwaves; ++w) {
                        v[g][0] += slot[sl][DET ? w : 0][g * 128 + lane];
                        v[g][1] += slot[sl][DET ? w : 0][g * 128 + 64 + lane];
                    }
                } else {
                    v[g][0] = slot[sl][0][g * 128 + lane];
                    v[g][1] = slot[sl][0][g * 128 + 64 + lane];
                    slot[sl][0][g * 128 + lane] = 0.0;
                    slot[sl][0][g * 128 + 64 + lane] = 0.0;
                }
            }
            // the lane index re-read here (opaque to the compiler), so that the lane's output
            // offset is formed in this branch instead of being held in registers throughout
            unsigned ln;
            asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0"
                         : "=v"(ln));
            const int b = ln >> 4;                // map
            const int blk = (ln >> 2) & 3;        // 2 s + h
            const int dl = 8 * (blk >> 1) + 2 * (ln & 3) + (blk & 1);
#pragma unroll
            for (int g = 0; g < kAdjGroup; ++g) {
                const int l = m + (c0 + g) * kLC + dl;
                if (l <= lmax && b < nmb) {
                    // the lane's map offset in 32 bits (b nalm 2 < 2^32), the rest uniform
                    double* o = alm + ((int64_t)(4 * grp) * nalm + moff + m + (c0 + g) * kLC) * 2 +
                                (unsigned)(b * (unsigned)nalm * 2u + (unsigned)dl * 2u);
                    if (DET) {
                        // this pair-chunk's own partial sums (alm points at them), summed
                        // over the pair-chunks in order afterwards
                        o[0] = v[g][0];
                        o[1] = m > 0 ? v[g][1] : 0.0;
                    } else {
                        if (v[g][0] != 0.0) unsafeAtomicAdd(o, v[g][0]);
                        if (m > 0 && v[g][1] != 0.0) unsafeAtomicAdd(o + 1, v[g][1]);  // c_l0 real
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) {
                // the count is reset before the hand-on becomes visible: a wave that sees the
                // new hand-on count also sees the zero count (release store)
                scnt[sl] = 0;
                __hip_atomic_store(&sgen[sl], use + 1, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
    // no LDS-DMA write may be in flight when the workgroup's LDS is released
    asm volatile("s_waitcnt vmcnt(0)" ::"v"(pf_keep) : "memory");
}

__global__ void k_fill_zero(double* __restrict__ a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

// Deterministic adjoint: alm[b][i] = sum over the pair-chunks pc of part[pc][b][i], in pc order.
// Pair-chunks that wrote nothing for the element's m (all their ring pairs below the live-ring
// bound jlive[m], or past the last pair) are skipped.
__global__ void k_adj_reduce(const double2* __restrict__ part, int npc, int nmaps, int64_t nalm,
                             int lmax, int mmax, const int* __restrict__ jlive, int ppb,
                             int npairs, double2* __restrict__ alm)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nalm) return;
    // m of index i: the largest m <= mmax whose first index first(m) = idx(m, m) =
    // m (2 lmax + 3 - m) / 2 is <= i.  first() grows with m up to lmax, and the discriminant
    // (2 lmax + 3)^2 - 8 i stays positive over the triangle; the estimate is corrected by
    // steps that cannot leave [0, mmax].
    const double bq = 2.0 * lmax + 3.0;
    const double disc = fmax(bq * bq - 8.0 * (double)i, 0.0);
    int m = (int)fmin(fmax(floor(0.5 * (bq - sqrt(disc))), 0.0), (double)mmax);
    while (m > 0 && (int64_t)m * (2 * lmax + 3 - m) / 2 > i) --m;
    while (m < mmax && (int64_t)(m + 1) * (2 * lmax + 2 - m) / 2 <= i) ++m;
    const int pc0 = jlive[m] / ppb;
    for (int b = 0; b < nmaps; ++b) {
        double2 acc = make_double2(0.0, 0.0);
        for (int pc = pc0; pc < npc && pc * ppb < npairs; ++pc) {
            const double2 v = part[((int64_t)pc * nmaps + b) * nalm + i];
            acc.x += v.x;
            acc.y += v.y;
        }
        alm[(int64_t)b * nalm + i] = acc;
    }
}

}  // namespace

int synth_pairs_per_lane(int npairs) { return npairs >= 1024 ? 2 : 1; }
int synth_scaled_pairs_per_lane(int npairs) { return synth_pairs_per_lane(npairs); }

int launch_legendre_synth(const nusht_plan_s* p, const double* alm, void* out, int nmaps,
                          int fused, int out_f32, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int npairs = (g.nrings + 1) / 2;
    // both instances take two ring pairs per lane once there are enough pairs to fill the
    // waves (one pair per lane in the scaled instance, which halves the spread of the scaled
    // phases' lengths across a wave, measured slower at C3: 7.41 against 7.07 ms)
    const int R = synth_pairs_per_lane(npairs);
    const int RS = synth_scaled_pairs_per_lane(npairs);
    auto shape = [&](int r, int& bx, int& threads) {
        const int waves_needed = (npairs + 64 * r - 1) / (64 * r);
        const int wpb = waves_needed >= 4 ? 4 : waves_needed;
        threads = 64 * wpb;
        bx = (waves_needed + wpb - 1) / wpb;
    };
    int bxp, thp, bxs, ths;
    shape(R, bxp, thp);
    shape(RS, bxs, ths);
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
    const int mpad = (g.mmax + 1 + 7) / 8 * 8;
    // the two instances write disjoint ring pairs: the plain one runs on the plan's side
    // stream, forked from and joined back into the call's stream, so that each fills the
    // other's tail
    hipStream_t sp = p->side ? p->side : s;
    if (sp != s) {
        NUSHT_HIP(hipEventRecord(p->fork_ev, s));
        NUSHT_HIP(hipStreamWaitEvent(sp, p->fork_ev, 0));
    }
    int b = 0;
    while (b < nmaps) {
        const int left = nmaps - b;
        const int mb = left >= 4 ? 4 : (left >= 2 ? 2 : 1);
        const int groups = left / mb;
        const double2* ab = a + (int64_t)b * nalm;
#define SYN1(MBV, RV, F, OT, SC, BX, TH)                                                         \
    hipLaunchKernelGGL((k_legendre_synth<MBV, RV, F, OT, SC>), dim3(BX * mpad, groups),          \
                       dim3(TH), 0, SC ? s : sp, ab, nalm, g.lmax, g.mmax, BX, p->rec, p->cm_mant, \
                       p->cm_exp, p->jlive, p->jscale, g.nrings, g.ntorus,                        \
                       reinterpret_cast<OT*>(out) + (int64_t)b * map_stride, map_stride,          \
                       row_stride)
#define SYNR(MBV, F, OT)                              \
    if (R == 2) {                                     \
        SYN1(MBV, 2, F, OT, false, bxp, thp);         \
    } else {                                          \
        SYN1(MBV, 1, F, OT, false, bxp, thp);         \
    }                                                 \
    if (RS == 2) {                                    \
        SYN1(MBV, 2, F, OT, true, bxs, ths);          \
    } else {                                          \
        SYN1(MBV, 1, F, OT, true, bxs, ths);          \
    }
        if (fused && out_f32) {
            if (mb == 4) { SYNR(4, true, float2) }
            else if (mb == 2) { SYNR(2, true, float2) }
            else { SYNR(1, true, float2) }
        } else if (fused) {
            if (mb == 4) { SYNR(4, true, double2) }
            else if (mb == 2) { SYNR(2, true, double2) }
            else { SYNR(1, true, double2) }
        } else {
            if (mb == 4) { SYNR(4, false, double2) }
            else if (mb == 2) { SYNR(2, false, double2) }
            else { SYNR(1, false, double2) }
        }
#undef SYNR
#undef SYN1
        NUSHT_HIP(hipGetLastError());
        b += groups * mb;
    }
    if (sp != s) {
        NUSHT_HIP(hipEventRecord(p->join_ev, sp));
        NUSHT_HIP(hipStreamWaitEvent(s, p->join_ev, 0));
    }
    return NUSHT_OK;
}

int launch_legendre_adjoint(nusht_plan_s* p, const void* in, double* alm, int nmaps,
                            int fused, int in_f32, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int npairs = (g.nrings + 1) / 2;
    const int npc = (npairs + kAdjWaves * 64 - 1) / (kAdjWaves * 64);
    int ppb = (npairs + npc - 1) / npc;
    ppb = ((ppb + 63) / 64) * 64;
    const int threads = ppb < 128 ? 128 : ppb;
    const int groups = (nmaps + 3) / 4;
    int64_t map_stride, row_stride;
    if (fused) {
        row_stride = g.ntorus;
        map_stride = (int64_t)(g.mmax + 1) * g.ntorus;
    } else {
        row_stride = g.nphi / 2 + 1;
        map_stride = (int64_t)g.nrings * row_stride;
    }
    const int mpad = (g.mmax + 1 + 7) / 8 * 8;
    dim3 grid(npc * mpad, groups);
#define ADJ(F, IT, D, OUT)                                                                      \
    hipLaunchKernelGGL((k_legendre_adj<F, IT, D>), grid, dim3(threads), 0, s,                    \
                       reinterpret_cast<const IT*>(in), map_stride, row_stride, nmaps, OUT, npc,  \
                       g.nalm, g.lmax, p->rec, p->cm_mant, p->cm_exp, p->jlive, g.nrings,        \
                       g.ntorus, ppb, g.mmax, p->dstatus)
    if (p->deterministic) {
        // every pair-chunk writes its own partial sums; one pass adds them in pair-chunk order
        const size_t need = (size_t)npc * nmaps * g.nalm * 2 * sizeof(double);
        if (need > p->adj_part_bytes) {
            NUSHT_HIP(hipStreamSynchronize(s));
            if (p->adj_part) hipFree(p->adj_part);
            p->adj_part = nullptr;
            p->adj_part_bytes = 0;
            NUSHT_HIP(hipMalloc((void**)&p->adj_part, need));
            p->adj_part_bytes = need;
        }
        double* part = p->adj_part;
        if (fused && in_f32) {
            ADJ(true, float2, true, part);
        } else if (fused) {
            ADJ(true, double2, true, part);
        } else {
            ADJ(false, double2, true, part);
        }
        NUSHT_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_adj_reduce, dim3((unsigned)((g.nalm + 255) / 256)), dim3(256), 0, s,
                           reinterpret_cast<const double2*>(part), npc, nmaps, g.nalm, g.lmax,
                           g.mmax, p->jlive, ppb, npairs, reinterpret_cast<double2*>(alm));
    } else {
        // the pair-chunk workgroups of one m add their sums into the zeroed output with FP64
        // atomics, which resolve in the L2 of the XCD those workgroups share
        const int64_t nz = (int64_t)nmaps * g.nalm * 2;
        hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s, alm,
                           nz);
        if (fused && in_f32) {
            ADJ(true, float2, false, alm);
        } else if (fused) {
            ADJ(true, double2, false, alm);
        } else {
            ADJ(false, double2, false, alm);
        }
    }
#undef ADJ
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

}  // namespace nusht
