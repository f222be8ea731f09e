// Type-2 interpolation and type-1 spreading of the ES-kernel nuFFT on the fine torus grid
// (arXiv:2406.14542 Sec. III: N and N^H of Eq. 5 / Eq. 6).
//
// Kernel: psi(z) = exp(beta (sqrt(1 - z^2) - 1)) for |z| < 1, z = 2 (x - x_l) / (w h).
// For a coordinate x with t = x / h (grid units) the w taps start at cell
//   ls = ceil(t - w/2),  and tap a has z_a = 2 (t - ls - a) / w  in (-1, 1].
// Points were binned by the plan into kTile x kTile tiles by (ls1 mod n1, ls2 mod n2), inside
// a tile by column band and then by row.
//  * interpolation: a workgroup owns one non-empty tile ("slot") and stages the tile's window
//    of (kTile + w - 1)^2 cells in LDS once; every point of the tile reads its w x w taps from
//    LDS; results are written packed per point;
//  * spreading, FP32 windows, FP64 windows of w <= 8 and deterministic plans: waves sweep
//    column bands row by row and keep the rows a point can reach in registers
//    (k_spread_band): every fine cell is written once, with its points summed in a fixed
//    order, and no atomics or partial grids are involved;
//  * spreading, FP64 windows of w > 8: tile subgrids accumulated with LDS atomics
//    (k_spread_lds) and a halo pass that sums, for every fine cell, the subgrids of the
//    windows covering it (k_halo).
// Offsets are formed in FP64 from FP64 coordinates before any cast to the kernel's type T.
#pragma once

#include "internal.h"

namespace nusht {

struct PointBins {
    const double* sth;
    const double* sph;
    const int* perm;
    const int* slot_off;
    const int* slot_tile;
    int nt2;
    int n1, n2;
    double s1, s2;  // n / (2 pi)
};

// first tap cell and its fractional offset; no fused multiply-add so that the plan and the
// kernels bin every point identically
__device__ inline int first_tap(double x, double scale, int w, double& d)
{
#pragma clang fp contract(off)
    const double t = x * scale;
    const int ls = (int)ceil(t - 0.5 * (double)w);
    d = t - (double)ls;
    return ls;
}

__device__ inline int wrap_index(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

// Slot of a tile workgroup: runs of kSlotRun consecutive slots (neighbouring tiles of a tile
// row) go to one XCD (workgroups go to the 8 XCDs round-robin by linear id), so that the
// 128-byte line a window shares with the next tile of its row comes from that XCD's L2
// instead of a second HBM fetch; the runs themselves alternate over the XCDs, which keeps the
// point load of the XCDs even (points per tile follow sin theta).  The last partial group of
// 8 runs keeps the identity order.
constexpr int kSlotRun = 8;
__device__ inline int xcd_slot(int b, int n)
{
    const int full = n / (8 * kSlotRun) * (8 * kSlotRun);
    if (b >= full) return b;
    const int x = b & 7, i = b >> 3;
    return ((i / kSlotRun) * 8 + x) * kSlotRun + i % kSlotRun;
}

template <typename T>
__device__ inline T es_value(T z, T beta)
{
    const T q = (T(1) - z) * (T(1) + z);
    return q > T(0) ? (T)exp(beta * (sqrt(q) - T(1))) : T(0);
}

template <typename T, int W>
__device__ inline void es_taps(double d, T beta, T (&psi)[W])
{
    const T dd = (T)d;
    const T c = T(2) / T(W);
#pragma unroll
    for (int a = 0; a < W; ++a) psi[a] = es_value<T>((dd - T(a)) * c, beta);
}

// The same taps from the plan's polynomials (degree W in s = 2 d - W + 1, coefficient of s^k
// for tap a at coef[k W + a]): W Horner chains advanced together, one wave-uniform coefficient
// row per step.
template <typename T, int W>
__device__ inline void es_taps_poly(double d, const T* __restrict__ coef, T (&psi)[W])
{
    const T sv = (T)(2.0 * d - (double)(W - 1));
#pragma unroll
    for (int a = 0; a < W; ++a) psi[a] = coef[W * W + a];
#pragma unroll
    for (int k = W - 1; k >= 0; --k)
#pragma unroll
        for (int a = 0; a < W; ++a) psi[a] = psi[a] * sv + coef[k * W + a];
}

// one tap a of one point from the polynomial coefficients creg[k] = coef[k W + a]
template <typename T, int W>
__device__ inline T es_tap_poly(T sv, const T (&creg)[W + 1])
{
    T v = creg[W];
#pragma unroll
    for (int k = W - 1; k >= 0; --k) v = v * sv + creg[k];
    return v;
}

// taps and their derivatives with respect to t (grid units):
// d psi / dt = psi(z) * beta * (-z / sqrt(1 - z^2)) * 2 / w.
// The derivative is singular at the support edge |z| -> 1, where psi itself is only
// e^-beta: a tap within 1 - z^2 < 1e-6 of the edge would add a spike of up to
// e^-beta beta / sqrt(1 - z^2) (and whether 1 - z^2 rounds to 0 or to 1e-16 for a point
// exactly on a grid line depends on FMA contraction).  Such taps get no derivative; what
// is dropped is below e^-beta * beta * 1e3 * 2/w times the grid value (5e-11 at w = 14).
constexpr double kDerivEdgeQ = 1e-6;

template <int W>
__device__ inline void es_taps_d(double d, double beta, double (&psi)[W], double (&dpsi)[W])
{
    const double c = 2.0 / W;
#pragma unroll
    for (int a = 0; a < W; ++a) {
        const double z = (d - a) * c;
        const double q = (1.0 - z) * (1.0 + z);
        if (q > 0.0) {
            const double sq = sqrt(q);
            const double v = exp(beta * (sq - 1.0));
            psi[a] = v;
            dpsi[a] = q > kDerivEdgeQ ? -v * beta * z / sq * c : 0.0;
        } else {
            psi[a] = 0.0;
            dpsi[a] = 0.0;
        }
    }
}

// Stage the tile's P x P window of MB maps into LDS (256 threads).  Each thread issues all
// of its loads before its first LDS write, so the block waits for HBM once rather than once
// per element it stages.
template <typename T, int P, int MB>
__device__ inline void stage_window(const T* __restrict__ fine, int64_t map_stride,
                                    const PointBins& pb, int r0, int c0, T* win)
{
    constexpr int NE = (P * P + 255) / 256;
    T v[NE][MB];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        const int e = (int)threadIdx.x + 256 * i;
        if (e < P * P) {
            const int r = e / P, c = e - r * P;
            int gr = r0 + r;
            if (gr >= pb.n1) gr -= pb.n1;
            int gc = c0 + c;
            if (gc >= pb.n2) gc -= pb.n2;
            const int64_t off = (int64_t)gr * pb.n2 + gc;
#pragma unroll
            for (int b = 0; b < MB; ++b) v[i][b] = fine[b * map_stride + off];
        }
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        const int e = (int)threadIdx.x + 256 * i;
        if (e < P * P) {
#pragma unroll
            for (int b = 0; b < MB; ++b) win[e * MB + b] = v[i][b];
        }
    }
}

// PACKED: one MB * 8-byte row per point, unpacked afterwards by k_unpack_points.  FP32
// windows write the rows in the sorted (tile) order p, coalesced, and the unpack gathers each
// caller point's row through the inverse permutation; FP64 windows (whose taps hide the
// scattered stores) write the rows in the caller's order, out[dst].  Not PACKED:
// out[b][dst] (MB scattered 8-byte stores).
template <typename T, int W, int MB, bool PACKED>
__global__ __launch_bounds__(256) void k_interp(const T* __restrict__ fine, int64_t map_stride,
                                                PointBins pb, T beta,
                                                const T* __restrict__ coef,
                                                double* __restrict__ out, int64_t npts)
{
    constexpr int P = kTile + W - 1;
    constexpr bool kUserRows = !PACKED || sizeof(T) == 8;  // results addressed by caller index
    __shared__ T win[P * P * MB];
    const int slot = xcd_slot(blockIdx.x, gridDim.x);
    const int tile = pb.slot_tile[slot];
    const int r0 = (tile / pb.nt2) * kTile;
    const int c0 = (tile % pb.nt2) * kTile;
    // the first point's coordinates and destination, then the whole window: every load of
    // the thread is in flight before the first one is waited for
    const int p0 = pb.slot_off[slot], p1 = pb.slot_off[slot + 1];
    int p = p0 + threadIdx.x;
    double thn = 0.0, phn = 0.0;
    int dstn = 0;
    if (p < p1) {
        thn = pb.sth[p];
        phn = pb.sph[p];
        if (kUserRows) dstn = pb.perm[p];
    }
    stage_window<T, P, MB>(fine, map_stride, pb, r0, c0, win);
    __syncthreads();
    for (; p < p1; p += 256) {
        const double th = thn, ph = phn;
        const int64_t dst = dstn;
        if (p + 256 < p1) {  // the next point's data, loaded under this point's work
            thn = pb.sth[p + 256];
            phn = pb.sph[p + 256];
            if (kUserRows) dstn = pb.perm[p + 256];
        }
        double d1, d2;
        const int l1 = first_tap(th, pb.s1, W, d1);
        const int l2 = first_tap(ph, pb.s2, W, d2);
        int r = wrap_index(l1, pb.n1) - r0;
        int c = wrap_index(l2, pb.n2) - c0;
        r = min(max(r, 0), kTile - 1);
        c = min(max(c, 0), kTile - 1);
        T p1v[W], p2v[W];
        if (coef) {
            es_taps_poly<T, W>(d1, coef, p1v);
            es_taps_poly<T, W>(d2, coef, p2v);
        } else {
            es_taps<T, W>(d1, beta, p1v);
            es_taps<T, W>(d2, beta, p2v);
        }
        T acc[MB];
#pragma unroll
        for (int b = 0; b < MB; ++b) acc[b] = T(0);
#pragma unroll
        for (int a = 0; a < W; ++a) {
            T row[MB];
#pragma unroll
            for (int b = 0; b < MB; ++b) row[b] = T(0);
            const T* wr = win + ((r + a) * P + c) * MB;
#pragma unroll
            for (int q = 0; q < W; ++q) {
#pragma unroll
                for (int b = 0; b < MB; ++b) row[b] += p2v[q] * wr[q * MB + b];
            }
#pragma unroll
            for (int b = 0; b < MB; ++b) acc[b] += p1v[a] * row[b];
        }
        if (PACKED && !kUserRows) {
            // FP32 rows (the values are FP32 sums): 16 bytes per point
            float* o = reinterpret_cast<float*>(out) + (int64_t)p * MB;
#pragma unroll
            for (int b = 0; b < MB; ++b) o[b] = (float)acc[b];
        } else if (PACKED) {
            double* o = out + dst * MB;
#pragma unroll
            for (int b = 0; b < MB; ++b) o[b] = (double)acc[b];
        } else {
#pragma unroll
            for (int b = 0; b < MB; ++b) out[b * npts + dst] = (double)acc[b];
        }
    }
}

// out[b][i] = packed[src][b].  GATHER: FP32 rows in tile order, src = iperm[i] (one 4 MB-byte
// gather per caller point, writes coalesced; scattered row writes had cost the FP32
// interpolation kernel 1.1 ms at 33.5 M points).  Otherwise FP64 rows in caller order, src = i.
template <int MB, bool GATHER>
__global__ void k_unpack_points(const double* __restrict__ packed,
                                const int* __restrict__ iperm, int64_t npts,
                                double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    double v[MB];
    if (GATHER) {
        const float* pf = reinterpret_cast<const float*>(packed) + (int64_t)iperm[i] * MB;
#pragma unroll
        for (int b = 0; b < MB; ++b) v[b] = (double)pf[b];
    } else {
#pragma unroll
        for (int b = 0; b < MB; ++b) v[b] = packed[i * MB + b];
    }
#pragma unroll
    for (int b = 0; b < MB; ++b) out[b * npts + i] = v[b];
}

// packed[i][b] = (T) in[b][i], the caller's point order kept: both sides coalesced
template <typename T, int MB>
__global__ void k_pack_values(const double* __restrict__ in, int64_t npts, T* __restrict__ packed)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    T v[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) v[b] = (T)in[b * npts + i];
#pragma unroll
    for (int b = 0; b < MB; ++b) packed[i * MB + b] = v[b];
}

template <int W, int MB>
__global__ __launch_bounds__(256) void k_interp_deriv(const double* __restrict__ fine,
                                                      int64_t map_stride, PointBins pb,
                                                      double beta, double* __restrict__ out,
                                                      double* __restrict__ dth,
                                                      double* __restrict__ dph, int64_t npts)
{
    constexpr int P = kTile + W - 1;
    __shared__ double win[P * P * MB];
    const int slot = xcd_slot(blockIdx.x, gridDim.x);
    const int tile = pb.slot_tile[slot];
    const int r0 = (tile / pb.nt2) * kTile;
    const int c0 = (tile % pb.nt2) * kTile;
    // the first point's coordinates and destination, then the whole window: every load of
    // the thread is in flight before the first one is waited for
    const int p0 = pb.slot_off[slot], p1 = pb.slot_off[slot + 1];
    int p = p0 + threadIdx.x;
    double thn = 0.0, phn = 0.0;
    int dstn = 0;
    if (p < p1) {
        thn = pb.sth[p];
        phn = pb.sph[p];
        dstn = pb.perm[p];
    }
    stage_window<double, P, MB>(fine, map_stride, pb, r0, c0, win);
    __syncthreads();
    for (; p < p1; p += 256) {
        const double th = thn, ph = phn;
        const int64_t dst = dstn;
        if (p + 256 < p1) {  // the next point's data, loaded under this point's work
            thn = pb.sth[p + 256];
            phn = pb.sph[p + 256];
            dstn = pb.perm[p + 256];
        }
        double d1, d2;
        const int l1 = first_tap(th, pb.s1, W, d1);
        const int l2 = first_tap(ph, pb.s2, W, d2);
        int r = wrap_index(l1, pb.n1) - r0;
        int c = wrap_index(l2, pb.n2) - c0;
        r = min(max(r, 0), kTile - 1);
        c = min(max(c, 0), kTile - 1);
        double p1v[W], p2v[W], q1v[W], q2v[W];
        es_taps_d<W>(d1, beta, p1v, q1v);
        es_taps_d<W>(d2, beta, p2v, q2v);
        double acc[MB], a1[MB], a2[MB];
#pragma unroll
        for (int b = 0; b < MB; ++b) acc[b] = a1[b] = a2[b] = 0.0;
#pragma unroll
        for (int a = 0; a < W; ++a) {
            double row[MB], rowd[MB];
#pragma unroll
            for (int b = 0; b < MB; ++b) row[b] = rowd[b] = 0.0;
            const double* wr = win + ((r + a) * P + c) * MB;
#pragma unroll
            for (int q = 0; q < W; ++q) {
#pragma unroll
                for (int b = 0; b < MB; ++b) {
                    const double u = wr[q * MB + b];
                    row[b] = fma(p2v[q], u, row[b]);
                    rowd[b] = fma(q2v[q], u, rowd[b]);
                }
            }
#pragma unroll
            for (int b = 0; b < MB; ++b) {
                acc[b] = fma(p1v[a], row[b], acc[b]);
                a1[b] = fma(q1v[a], row[b], a1[b]);
                a2[b] = fma(p1v[a], rowd[b], a2[b]);
            }
        }
#pragma unroll
        for (int b = 0; b < MB; ++b) {
            out[b * npts + dst] = acc[b];
            dth[b * npts + dst] = a1[b] * pb.s1;
            dph[b * npts + dst] = a2[b] * pb.s2;
        }
    }
}

// Spreading of wide FP64 kernels (w > 8), not deterministic: tile subgrids with LDS atomics
// and a halo pass.  (The band sweep below does only 64 / 16 = 4 points per wave step once
// w > 8 and runs FP64 maps one per pass; for FP64 its per-point work then outweighs the
// atomics this kernel pays.)
// Batched: the block stages up to NB of the slot's points (tap
// offsets, first cells relative to the tile, values) in LDS, then every wave takes
// PPW = 64 / LPP points at a time with LPP lanes per point, lane = column tap: each lane forms
// its column tap psi2[col] and the row tap psi1[col], the row taps of the point are exchanged
// through a per-wave LDS row, and lane (point, col) adds f psi1[a] psi2[col] into window
// rows r + a, a < W, of its column.  The window is planar (map-major), so the lanes of one
// point add into consecutive words of one row.  Values come in packed, [point][MB], in the
// caller's order, and are fetched through the permutation.  The window sums in FP64; the order of the additions into a cell is not fixed, so results can
// differ between runs by FP64 rounding (~1e-16 relative) before the cast to T.
template <typename T, int MB>
struct SpreadPoint {
    T d1, d2;  // offsets of the first taps, grid units
    int r, c;  // first tap cell relative to the tile
    T f[MB];
};

template <typename T, int W, int MB>
__global__ __launch_bounds__(256) void k_spread_lds(const T* __restrict__ vals, PointBins pb,
                                                    T beta, T* __restrict__ sub)
{
    constexpr int P = kTile + W - 1;
    constexpr int LPP = W <= 8 ? 8 : 16;
    constexpr int PPW = 64 / LPP;
    constexpr int NB = 128;  // points staged per batch (64 for FP64 measured 0.6 ms slower)
    static_assert(W <= 16, "one lane per column tap");
    // the window accumulates in FP64 for either T: LDS atomic adds of FP64 measured fast on
    // gfx950, those of FP32 an order of magnitude slower than the whole kernel
    __shared__ double win[MB * P * P];
    __shared__ SpreadPoint<T, MB> s_pt[NB];
    __shared__ T s_p1[4][PPW][LPP];
    const int slot = blockIdx.x;
    const int tile = pb.slot_tile[slot];
    const int r0 = (tile / pb.nt2) * kTile;
    const int c0 = (tile % pb.nt2) * kTile;
    const int t = threadIdx.x;
    for (int e = t; e < MB * P * P; e += blockDim.x) win[e] = 0.0;
    const int wave = t >> 6, lane = t & 63;
    const int grp = lane / LPP, col = lane - grp * LPP;
    const int p0 = pb.slot_off[slot], p1 = pb.slot_off[slot + 1];
    const T cw = T(2) / T(W);
    T* p1row = s_p1[wave][grp];
    for (int base = p0; base < p1; base += NB) {
        const int nb = min(NB, p1 - base);
        __syncthreads();  // window cleared, or the previous batch consumed
        if (t < nb) {
            const int p = base + t;
            double d1, d2;
            const int l1 = first_tap(pb.sth[p], pb.s1, W, d1);
            const int l2 = first_tap(pb.sph[p], pb.s2, W, d2);
            int r = wrap_index(l1, pb.n1) - r0;
            int c = wrap_index(l2, pb.n2) - c0;
            const int64_t src = pb.perm[p];
            SpreadPoint<T, MB> sp;
            sp.d1 = (T)d1;
            sp.d2 = (T)d2;
            sp.r = min(max(r, 0), kTile - 1);
            sp.c = min(max(c, 0), kTile - 1);
#pragma unroll
            for (int b = 0; b < MB; ++b) sp.f[b] = vals[src * MB + b];
            s_pt[t] = sp;
        }
        __syncthreads();
        // lane group g takes the points g S + i of the row-sorted batch: the PPW points of one
        // step lie S apart, in different rows, so no two lanes of an atomic add address the
        // same cell (a point adds into rows r + a for the step's common a)
        const int S = (nb + PPW - 1) / PPW;
        for (int i = wave; i < S; i += 4) {
            const int q = grp * S + i;
            const bool live = q < nb;
            const SpreadPoint<T, MB> sp = s_pt[live ? q : 0];
            const bool act = live && col < W;
            const T p2 = act ? es_value<T>((sp.d2 - T(col)) * cw, beta) : T(0);
            p1row[col] = col < W ? es_value<T>((sp.d1 - T(col)) * cw, beta) : T(0);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            T pr[W];
#pragma unroll
            for (int a = 0; a < W; ++a) pr[a] = p1row[a];
            // the next step rewrites the row: every lane's reads come first
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (act) {
                T fb[MB];
#pragma unroll
                for (int b = 0; b < MB; ++b) fb[b] = sp.f[b] * p2;
                double* w0 = win + sp.r * P + sp.c + col;
#pragma unroll
                for (int a = 0; a < W; ++a)
#pragma unroll
                    for (int b = 0; b < MB; ++b)
                        atomicAdd(w0 + (b * P + a) * P, (double)(fb[b] * pr[a]));
            }
        }
    }
    __syncthreads();
    T* dst = sub + (int64_t)slot * (P * P * MB);
    for (int e = t; e < P * P; e += blockDim.x) {
#pragma unroll
        for (int b = 0; b < MB; ++b) dst[e * MB + b] = (T)win[b * P * P + e];
    }
}

// fine[b][i][j] = sum of the subgrids of the windows covering cell (i, j); zero elsewhere
template <typename T, int W, int MB>
__global__ __launch_bounds__(256) void k_halo(const T* __restrict__ sub,
                                              const int* __restrict__ tile_slot, int nt1, int nt2,
                                              int n1, int n2, int ra, int rb,
                                              T* __restrict__ fine, int64_t map_stride)
{
    constexpr int P = kTile + W - 1;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    // rows [0, ra) and [n1 - rb, n1): the only rows any window reaches
    const int i = (int)blockIdx.y < ra ? (int)blockIdx.y : n1 - rb + ((int)blockIdx.y - ra);
    if (j >= n2) return;
    const int tr = i / kTile, rr = i - tr * kTile;
    const int tc = j / kTile, cc = j - tc * kTile;
    const int trp = tr == 0 ? nt1 - 1 : tr - 1;
    const int tcp = tc == 0 ? nt2 - 1 : tc - 1;
    T acc[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) acc[b] = T(0);
    auto add = [&](int t_r, int t_c, int r, int c) {
        const int sl = tile_slot[t_r * nt2 + t_c];
        if (sl < 0) return;
        const T* s = sub + (int64_t)sl * (P * P * MB) + (r * P + c) * MB;
#pragma unroll
        for (int b = 0; b < MB; ++b) acc[b] += s[b];
    };
    add(tr, tc, rr, cc);
    if (rr < W - 1) add(trp, tc, rr + kTile, cc);
    if (cc < W - 1) add(tr, tcp, rr, cc + kTile);
    if (rr < W - 1 && cc < W - 1) add(trp, tcp, rr + kTile, cc + kTile);
    const int64_t off = (int64_t)i * n2 + j;
#pragma unroll
    for (int b = 0; b < MB; ++b) fine[b * map_stride + off] = acc[b];
}

// Spreading (type 1, N^H of Eq. 6): u(l1, l2) = sum_i f_i psi(row taps) psi(column taps), the
// exact adjoint of the interpolation above (same taps).
//
// Band sweep, no atomics.  The fine columns are cut into bands of SW = band_w columns; each
// group of SW lanes of a wave owns one band (lane q = column c0 + q), so a wave sweeps
// K = 64 / SW bands side by side.  The plan keeps, per band, a record of every point whose
// taps reach the band (its own band's points and those of the band to its left), sorted by
// first-tap row.  Every lane keeps the w rows [R, R + w) of its column in registers: a point
// whose first tap is row r (>= R, rows only grow) first pushes rows R .. r-1 out to the fine
// grid, then adds f psi1[a] psi2[q - c] to rows r + a.  Each cell is written once, by the lane
// that owns its column, as the sum of its points in a fixed order: the result does not depend
// on scheduling, and nothing is written twice.
//
// The records stream through LDS in batches of SW (lane j of a group stages record j), with
// the loads two stages ahead: a batch's records are fetched two batches before their turn and
// their point values (gathered through the caller's index) one batch before, so the
// sequential row sweep never waits on a load of its own.
//
// Rows are handled on a virtual axis: physical tile row nt1 - 1 (points near theta = 0 whose
// first tap wraps below row 0) is virtual tile row -1, so a band's rows run on without a wrap
// from -kTile up.  The rows are cut into segments of seg_tiles tile rows (grid.y); a segment
// owns the rows of its tile rows and also sweeps the records of the tile row above it whose
// taps reach its first row (and drops their rows above it), so segments never write the same
// cell either.  The owned rows of all segments are exactly the rows any point window reaches
// ([n1 - kTile, n1) and [0, ra)); when every row is reached, the first segment's overlap row
// is the last tile row shifted by -n1, which carries the wrap.
struct BandBins {
    const int* boff;  // [nbands * nt1 + 1]
    int nt1, n1, n2, nbands;
    int64_t nrec;
    int vt_end;     // virtual tile rows [-1, vt_end) can hold points
    int vrow_hi;    // owned virtual rows are [-kTile, vrow_hi)
    int seg_tiles;  // tile rows per segment
};

// first record of [a, e) whose virtual row (first-tap row + voff) is >= row
template <typename T>
__device__ inline int band_lower_bound(const BandRec<T>* __restrict__ recs, int a, int e,
                                       int voff, int row)
{
    while (a < e) {
        const int mid = (a + e) >> 1;
        if ((recs[mid].rc & 0xffff) + voff < row) a = mid + 1; else e = mid;
    }
    return a;
}

// Row shift of the spreading sweep for one map: r[a] = lane's bit of mk ? r[a + 1] : r[a]
// (a < W - 1), r[W - 1] = lane's bit of mk ? 0 : r[W - 1], as one block of in-place selects
// on the registers themselves, in ascending a (each r[a + 1] is read before it is
// replaced).  One statement for the whole shift leaves the compiler no room to copy the rows.
template <int W>
__device__ inline void shift_rows(uint32_t (&r)[W], uint64_t mk);

#define NUSHT_SEL(i, j) "v_cndmask_b32_e64 %" #i ", %" #i ", %" #j ", %[mk]\n\t"
#define NUSHT_SEL0(i) "v_cndmask_b32_e64 %" #i ", %" #i ", 0, %[mk]"
template <>
__device__ inline void shift_rows<2>(uint32_t (&r)[2], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL0(1)
        : "+v"(r[0]), "+v"(r[1])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<3>(uint32_t (&r)[3], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL0(2)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<4>(uint32_t (&r)[4], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL(2, 3) NUSHT_SEL0(3)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<5>(uint32_t (&r)[5], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL(2, 3) NUSHT_SEL(3, 4) NUSHT_SEL0(4)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<6>(uint32_t (&r)[6], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL(2, 3) NUSHT_SEL(3, 4) NUSHT_SEL(4, 5) NUSHT_SEL0(5)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4]), "+v"(r[5])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<7>(uint32_t (&r)[7], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL(2, 3) NUSHT_SEL(3, 4) NUSHT_SEL(4, 5) NUSHT_SEL(5, 6) NUSHT_SEL0(6)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4]), "+v"(r[5]), "+v"(r[6])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<8>(uint32_t (&r)[8], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL(2, 3) NUSHT_SEL(3, 4) NUSHT_SEL(4, 5) NUSHT_SEL(5, 6) NUSHT_SEL(6, 7) NUSHT_SEL0(7)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4]), "+v"(r[5]), "+v"(r[6]), "+v"(r[7])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<9>(uint32_t (&r)[9], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL(2, 3) NUSHT_SEL(3, 4) NUSHT_SEL(4, 5) NUSHT_SEL(5, 6) NUSHT_SEL(6, 7) NUSHT_SEL(7, 8) NUSHT_SEL0(8)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4]), "+v"(r[5]), "+v"(r[6]), "+v"(r[7]), "+v"(r[8])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<10>(uint32_t (&r)[10], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL(2, 3) NUSHT_SEL(3, 4) NUSHT_SEL(4, 5) NUSHT_SEL(5, 6) NUSHT_SEL(6, 7) NUSHT_SEL(7, 8) NUSHT_SEL(8, 9) NUSHT_SEL0(9)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4]), "+v"(r[5]), "+v"(r[6]), "+v"(r[7]), "+v"(r[8]), "+v"(r[9])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<11>(uint32_t (&r)[11], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL(2, 3) NUSHT_SEL(3, 4) NUSHT_SEL(4, 5) NUSHT_SEL(5, 6) NUSHT_SEL(6, 7) NUSHT_SEL(7, 8) NUSHT_SEL(8, 9) NUSHT_SEL(9, 10) NUSHT_SEL0(10)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4]), "+v"(r[5]), "+v"(r[6]), "+v"(r[7]), "+v"(r[8]), "+v"(r[9]), "+v"(r[10])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<12>(uint32_t (&r)[12], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL(2, 3) NUSHT_SEL(3, 4) NUSHT_SEL(4, 5) NUSHT_SEL(5, 6) NUSHT_SEL(6, 7) NUSHT_SEL(7, 8) NUSHT_SEL(8, 9) NUSHT_SEL(9, 10) NUSHT_SEL(10, 11) NUSHT_SEL0(11)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4]), "+v"(r[5]), "+v"(r[6]), "+v"(r[7]), "+v"(r[8]), "+v"(r[9]), "+v"(r[10]), "+v"(r[11])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<13>(uint32_t (&r)[13], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL(2, 3) NUSHT_SEL(3, 4) NUSHT_SEL(4, 5) NUSHT_SEL(5, 6) NUSHT_SEL(6, 7) NUSHT_SEL(7, 8) NUSHT_SEL(8, 9) NUSHT_SEL(9, 10) NUSHT_SEL(10, 11) NUSHT_SEL(11, 12) NUSHT_SEL0(12)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4]), "+v"(r[5]), "+v"(r[6]), "+v"(r[7]), "+v"(r[8]), "+v"(r[9]), "+v"(r[10]), "+v"(r[11]), "+v"(r[12])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<14>(uint32_t (&r)[14], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL(2, 3) NUSHT_SEL(3, 4) NUSHT_SEL(4, 5) NUSHT_SEL(5, 6) NUSHT_SEL(6, 7) NUSHT_SEL(7, 8) NUSHT_SEL(8, 9) NUSHT_SEL(9, 10) NUSHT_SEL(10, 11) NUSHT_SEL(11, 12) NUSHT_SEL(12, 13) NUSHT_SEL0(13)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4]), "+v"(r[5]), "+v"(r[6]), "+v"(r[7]), "+v"(r[8]), "+v"(r[9]), "+v"(r[10]), "+v"(r[11]), "+v"(r[12]), "+v"(r[13])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<15>(uint32_t (&r)[15], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL(2, 3) NUSHT_SEL(3, 4) NUSHT_SEL(4, 5) NUSHT_SEL(5, 6) NUSHT_SEL(6, 7) NUSHT_SEL(7, 8) NUSHT_SEL(8, 9) NUSHT_SEL(9, 10) NUSHT_SEL(10, 11) NUSHT_SEL(11, 12) NUSHT_SEL(12, 13) NUSHT_SEL(13, 14) NUSHT_SEL0(14)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4]), "+v"(r[5]), "+v"(r[6]), "+v"(r[7]), "+v"(r[8]), "+v"(r[9]), "+v"(r[10]), "+v"(r[11]), "+v"(r[12]), "+v"(r[13]), "+v"(r[14])
        : [mk] "s"(mk));
}
template <>
__device__ inline void shift_rows<16>(uint32_t (&r)[16], uint64_t mk)
{
    asm(NUSHT_SEL(0, 1) NUSHT_SEL(1, 2) NUSHT_SEL(2, 3) NUSHT_SEL(3, 4) NUSHT_SEL(4, 5) NUSHT_SEL(5, 6) NUSHT_SEL(6, 7) NUSHT_SEL(7, 8) NUSHT_SEL(8, 9) NUSHT_SEL(9, 10) NUSHT_SEL(10, 11) NUSHT_SEL(11, 12) NUSHT_SEL(12, 13) NUSHT_SEL(13, 14) NUSHT_SEL(14, 15) NUSHT_SEL0(15)
        : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4]), "+v"(r[5]), "+v"(r[6]), "+v"(r[7]), "+v"(r[8]), "+v"(r[9]), "+v"(r[10]), "+v"(r[11]), "+v"(r[12]), "+v"(r[13]), "+v"(r[14]), "+v"(r[15])
        : [mk] "s"(mk));
}
#undef NUSHT_SEL
#undef NUSHT_SEL0

// N consecutive values from LDS in 16-byte reads (N * sizeof(T) a multiple of 16, or N < that,
// src aligned to the row size)
template <typename T, int N>
__device__ inline void load_row(const T* src, T (&out)[N])
{
    constexpr int kBytes = N * (int)sizeof(T);
    if constexpr (kBytes % 16 == 0) {
        const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
        for (int i = 0; i < kBytes / 16; ++i) {
            const float4 x = s4[i];
            T* o = out + i * (16 / (int)sizeof(T));
            __builtin_memcpy(o, &x, 16);
        }
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = src[i];
    }
}

template <typename T, int W, int MB, int SW>
__global__ __launch_bounds__(256) void k_spread_band(const BandRec<T>* __restrict__ recs,
                                                     const T* __restrict__ vals, int vstride,
                                                     BandBins bb, T beta,
                                                     const T* __restrict__ coef,
                                                     T* __restrict__ fine, int64_t map_stride)
{
    constexpr int K = 64 / SW;
    static_assert(SW >= W && kTile % SW == 0,
                  "one band to the left reaches a band; a group's lanes hold the row taps");
    // staged records (virtual row, column relative to the band, tap offsets) and values
    struct Staged {
        int r, c;
        T s1, s2;
    };
    __shared__ Staged s_rec[4][64];
    __shared__ __align__(16) T s_val[4][64 * MB];
    // the current point's taps: row tap q and column tap q of each group, from its lane q
    __shared__ __align__(16) T s_tap[4][2][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / SW, q = lane - grp * SW;
    const int band = (int)(blockIdx.x * 4 + wave) * K + grp;
    const bool bvalid = band < bb.nbands;
    const int c0 = bvalid ? band * SW : 0;
    const int vt0 = -1 + (int)blockIdx.y * bb.seg_tiles;
    const int vt1 = min(vt0 + bb.seg_tiles, bb.vt_end);
    const int own_lo = vt0 * kTile;
    const int own_hi = vt1 == bb.vt_end ? bb.vrow_hi : vt1 * kTile;
    const int first_row = own_lo - (W - 1);  // the overlap tile row's points from this row on
    const T cw = T(2) / T(W);
    // lane q forms tap q of a point (row tap q, and column tap q for the group): with tap
    // polynomials, its coefficient column in registers for the whole sweep
    const bool poly = coef != nullptr;
    T creg[W + 1];
#pragma unroll
    for (int k = 0; k <= W; ++k) creg[k] = (poly && q < W) ? coef[k * W + q] : T(0);

    // this band's records for the segment: at most two runs [a0, e0) (row offset vo0) and
    // [a1, e1) (vo1) -- the overlap tile row vt0 - 1 (from its first record that reaches
    // first_row on) and the segment's own tile rows, split where virtual tile row -1
    // (physical nt1 - 1) is followed by physical tile row 0
    int a0 = 0, e0 = 0, vo0 = 0, a1 = 0, e1 = 0, vo1 = 0;
    if (bvalid) {
        const int gb = band * bb.nt1;
        const int nt1 = bb.nt1;
        if (vt0 <= 0) {
            // overlap row nt1 - 2 (vt0 = -1) or nt1 - 1 (vt0 = 0), shifted by -n1; for vt0 = -1
            // the virtual tile row -1 (physical nt1 - 1) follows it in the same run
            const int po = vt0 < 0 ? nt1 - 2 : nt1 - 1;
            vo0 = -bb.n1;
            a0 = band_lower_bound(recs, bb.boff[gb + po], bb.boff[gb + po + 1], vo0, first_row);
            e0 = bb.boff[gb + nt1];
            a1 = bb.boff[gb];
            e1 = bb.boff[gb + vt1];
        } else {
            a0 = band_lower_bound(recs, bb.boff[gb + vt0 - 1], bb.boff[gb + vt0], 0, first_row);
            e0 = bb.boff[gb + vt1];
        }
    }
    const int n0 = e0 - a0;
    const int total = n0 + (e1 - a1);
    const int nbatch = (total + SW - 1) / SW;
    // record t of the band's stream, clamped into the array (unused when t >= total)
    auto rec_index = [&](int t, int& voff) {
        voff = t < n0 ? vo0 : vo1;
        int idx = t < n0 ? a0 + t : a1 + (t - n0);
        return (t < total) ? idx : 0;
    };

    T acc[W][MB];
#pragma unroll
    for (int a = 0; a < W; ++a)
#pragma unroll
        for (int m = 0; m < MB; ++m) acc[a][m] = T(0);
    int R = first_row;
    // lanes with adv: push row R out (if this segment owns it) and move the register rows up
    // by one.  Straight-line code with selects, so that the rows stay in place in registers
    // (a branch around the move made the compiler keep copies of all of them).
    auto advance = [&](bool adv) {
        if (adv && bvalid && R >= own_lo && R < own_hi) {
            const int pr = R < 0 ? R + bb.n1 : R;
            T* o = fine + (int64_t)pr * bb.n2 + c0 + q;
#pragma unroll
            for (int m = 0; m < MB; ++m) o[m * map_stride] = acc[0][m];
        }
        const uint64_t mask = __builtin_amdgcn_ballot_w64(adv);
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            if constexpr (sizeof(T) == 4) {
                uint32_t r[W];
#pragma unroll
                for (int a = 0; a < W; ++a) r[a] = __builtin_bit_cast(uint32_t, acc[a][m]);
                shift_rows<W>(r, mask);
#pragma unroll
                for (int a = 0; a < W; ++a) acc[a][m] = __builtin_bit_cast(T, r[a]);
            } else {
                uint32_t lo[W], hi[W];
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    const uint64_t u = __builtin_bit_cast(uint64_t, acc[a][m]);
                    lo[a] = (uint32_t)u;
                    hi[a] = (uint32_t)(u >> 32);
                }
                shift_rows<W>(lo, mask);
                shift_rows<W>(hi, mask);
#pragma unroll
                for (int a = 0; a < W; ++a)
                    acc[a][m] = __builtin_bit_cast(T, ((uint64_t)hi[a] << 32) | lo[a]);
            }
        }
        R += adv ? 1 : 0;
    };

    // push rows R .. tgt - 1 out of the lanes that are behind tgt: up to W row shifts with the
    // rows in registers, unrolled (a loop around the shift made the compiler copy every row
    // into the loop and back), after which a lane still behind has only zero rows left, and
    // its remaining rows are written as zeros
    auto push_to = [&](int tgt) {
#pragma unroll
        for (int i = 0; i < W; ++i) {
            if (!__any(R < tgt)) return;
            advance(R < tgt);
        }
        while (__any(R < tgt)) {
            const bool adv = R < tgt;
            if (adv && bvalid && R >= own_lo && R < own_hi) {
                const int pr = R < 0 ? R + bb.n1 : R;
                T* o = fine + (int64_t)pr * bb.n2 + c0 + q;
#pragma unroll
                for (int m = 0; m < MB; ++m) o[m * map_stride] = T(0);
            }
            R += adv ? 1 : 0;
        }
    };

    // pipeline: recA / valA = batch b (staged at the top of iteration b), recB = batch b + 1
    int voA, voB;
    BandRec<T> recA = recs[rec_index(q, voA)];
    T valA[MB];
    {
        const int64_t src = recA.src;
#pragma unroll
        for (int m = 0; m < MB; ++m) valA[m] = vals[src * vstride + m];
    }
    BandRec<T> recB = recs[rec_index(SW + q, voB)];
    bool okA = q < total;

    for (int b = 0; __any(b < nbatch); ++b) {
        // stage batch b
        {
            Staged st;
            st.r = (recA.rc & 0xffff) + voA;
            st.c = (recA.rc >> 16) - 32;
            st.s1 = recA.s1;
            st.s2 = recA.s2;
            s_rec[wave][lane] = st;
#pragma unroll
            for (int m = 0; m < MB; ++m) s_val[wave][lane * MB + m] = okA ? valA[m] : T(0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // the next stages: values of batch b + 1, records of batch b + 2
        T valB[MB];
        {
            const int64_t src = recB.src;
#pragma unroll
            for (int m = 0; m < MB; ++m) valB[m] = vals[src * vstride + m];
        }
        int voC;
        const BandRec<T> recC = recs[rec_index((b + 2) * SW + q, voC)];
        // the batch's points, one per group and step (not unrolled: the register rows, the tap
        // coefficients and the pipelined loads already fill the register file)
#pragma unroll 1
        for (int jj = 0; jj < SW; ++jj) {
            const int t = b * SW + jj;
            const bool has = bvalid && t < total;
            const Staged h = s_rec[wave][grp * SW + jj];
            // this lane's taps first (row tap q and column tap q of the group's point), so that
            // their latency overlaps the row advance; a group without a point has zero taps
            T t1 = T(0), t2 = T(0);
            if (poly) {
                t1 = es_tap_poly<T, W>(h.s1, creg);
                t2 = es_tap_poly<T, W>(h.s2, creg);
            } else if (q < W) {
                // z of tap a = 2 (d - a) / w = (s + w - 1 - 2 a) / w
                t1 = es_value<T>((h.s1 + T(W - 1 - 2 * q)) * cw * T(0.5), beta);
                t2 = es_value<T>((h.s2 + T(W - 1 - 2 * q)) * cw * T(0.5), beta);
            }
            s_tap[wave][0][lane] = has ? t1 : T(0);
            s_tap[wave][1][lane] = has ? t2 : T(0);
            // push the rows above the point's first row
            const int target = has ? h.r : R;
            push_to(target);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // the group's W row taps (one broadcast read), this lane's column tap (tap q - c,
            // zero outside the point's columns) and the point's MB values
            const int cb = q - h.c;
            const bool act = has && cb >= 0 && cb < W;
            const T p2 = s_tap[wave][1][grp * SW + (act ? cb : 0)];
            T rt[SW];
            load_row<T, SW>(&s_tap[wave][0][grp * SW], rt);
            T v[MB];
            load_row<T, MB>(&s_val[wave][(grp * SW + jj) * MB], v);
            T g[MB];
#pragma unroll
            for (int m = 0; m < MB; ++m) g[m] = act ? v[m] * p2 : T(0);
#pragma unroll
            for (int a = 0; a < W; ++a)
#pragma unroll
                for (int m = 0; m < MB; ++m) acc[a][m] += g[m] * rt[a];
            // the taps are read before the next point writes them
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // every lane's reads of the staged batch come before the next batch is staged
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        recA = recB;
        voA = voB;
#pragma unroll
        for (int m = 0; m < MB; ++m) valA[m] = valB[m];
        okA = (b + 1) * SW + q < total;
        recB = recC;
        voB = voC;
    }
    // the rows after the last point, up to the end of the segment
    push_to(own_hi);
}

// ---- dispatch over the kernel width ---------------------------------------------------

inline PointBins make_bins(const nusht_plan_s* p)
{
    PointBins pb;
    pb.sth = p->sth;
    pb.sph = p->sph;
    pb.perm = p->perm;
    pb.slot_off = p->slot_off;
    pb.slot_tile = p->slot_tile;
    pb.nt2 = p->nt2;
    pb.n1 = p->g.n1;
    pb.n2 = p->g.n2;
    pb.s1 = p->g.n1 / (2.0 * M_PI);
    pb.s2 = p->g.n2 / (2.0 * M_PI);
    return pb;
}

#define NUSHT_WIDTH_SWITCH(W_, BODY) \
    switch (W_) {                    \
        case 2: { constexpr int WV = 2; BODY; } break;   \
        case 3: { constexpr int WV = 3; BODY; } break;   \
        case 4: { constexpr int WV = 4; BODY; } break;   \
        case 5: { constexpr int WV = 5; BODY; } break;   \
        case 6: { constexpr int WV = 6; BODY; } break;   \
        case 7: { constexpr int WV = 7; BODY; } break;   \
        case 8: { constexpr int WV = 8; BODY; } break;   \
        case 9: { constexpr int WV = 9; BODY; } break;   \
        case 10: { constexpr int WV = 10; BODY; } break; \
        case 11: { constexpr int WV = 11; BODY; } break; \
        case 12: { constexpr int WV = 12; BODY; } break; \
        case 13: { constexpr int WV = 13; BODY; } break; \
        case 14: { constexpr int WV = 14; BODY; } break; \
        case 15: { constexpr int WV = 15; BODY; } break; \
        case 16: { constexpr int WV = 16; BODY; } break; \
        default: set_last_error("nufft", "unsupported kernel width"); return NUSHT_EINVAL; \
    }

// Interpolation of maps [0, nmaps): groups of four write packed rows [point][4] into the plan's
// point scratch (one 32-byte store per point instead of four scattered 8-byte ones), unpacked
// into out afterwards; a single map writes straight to out.

// the plan's tap polynomials in the kernels' precision, or null (taps from sqrt and exp)
template <typename T>
inline const T* es_coef_of(const nusht_plan_s* p);
template <>
inline const double* es_coef_of<double>(const nusht_plan_s* p) { return p->es_coef; }
template <>
inline const float* es_coef_of<float>(const nusht_plan_s* p) { return p->es_coeff; }

template <typename T>
int dispatch_interp_impl(const nusht_plan_s* p, const T* fine, double* out, int nmaps, T beta,
                         hipStream_t s)
{
    const T* coef = es_coef_of<T>(p);
    if (p->nslots == 0) return NUSHT_OK;
    const PointBins pb = make_bins(p);
    const int64_t ms = (int64_t)p->g.n1 * p->g.n2;
    const int64_t npts = p->g.npts;
    const unsigned pblocks = (unsigned)((npts + 255) / 256);
    int b = 0;
    while (b < nmaps) {
        const int mb = group_width(nmaps, b);
        NUSHT_WIDTH_SWITCH(p->g.width, {
            if (mb == 4) {
                hipLaunchKernelGGL((k_interp<T, WV, 4, true>), dim3(p->nslots), dim3(256), 0, s,
                                   fine + b * ms, ms, pb, beta, coef, p->V, npts);
                hipLaunchKernelGGL((k_unpack_points<4, sizeof(T) == 4>), dim3(pblocks), dim3(256),
                                   0, s, p->V, p->iperm, npts, out + b * npts);
            } else {
                hipLaunchKernelGGL((k_interp<T, WV, 1, false>), dim3(p->nslots), dim3(256), 0,
                                   s, fine + b * ms, ms, pb, beta, coef, out + b * npts, npts);
            }
        });
        NUSHT_HIP(hipGetLastError());
        b += mb;
    }
    return NUSHT_OK;
}

inline BandBins make_band_bins(const nusht_plan_s* p)
{
    BandBins bb;
    bb.boff = p->boff;
    bb.nt1 = p->g.n1 / kTile;
    bb.n1 = p->g.n1;
    bb.n2 = p->g.n2;
    bb.nbands = p->g.n2 / p->band_w;
    bb.nrec = p->nrec;
    bb.vt_end = p->band_vt_end;
    bb.vrow_hi = p->band_vrow_hi;
    bb.seg_tiles = p->band_seg_tiles;
    return bb;
}

// Spreading of the caller's maps [b, b + mb) (`vals` = its map block [mb][npts]) onto the
// fine grids of those maps: the values are first packed [point][mb] in the caller's order into
// the plan's point scratch, so that the kernels fetch a point's mb values with one load through
// the caller's index.  Kernels of width <= 8 (and every kernel of a deterministic plan) use the
// band sweep; wider ones the tile subgrids (into the plan's scratch Z) and the halo pass.
template <typename T>
int spread_group_impl(const nusht_plan_s* p, const double* vals, T* fine, int mb, T beta,
                      hipStream_t s)
{
    const int64_t npts = p->g.npts;
    const unsigned pblocks = (unsigned)((npts + 255) / 256);
    T* packed = reinterpret_cast<T*>(p->V);
    if (mb == 4)
        hipLaunchKernelGGL((k_pack_values<T, 4>), dim3(pblocks), dim3(256), 0, s, vals, npts,
                           packed);
    else
        hipLaunchKernelGGL((k_pack_values<T, 1>), dim3(pblocks), dim3(256), 0, s, vals, npts,
                           packed);
    NUSHT_HIP(hipGetLastError());
    const int64_t ms = (int64_t)p->g.n1 * p->g.n2;
    if (spread_uses_tiles(p)) {
        if (p->nslots == 0) return NUSHT_OK;
        const PointBins pb = make_bins(p);
        T* sub = reinterpret_cast<T*>(p->Z);
        dim3 hgrid((p->g.n2 + 255) / 256, p->fine_ra + p->fine_rb);
        NUSHT_WIDTH_SWITCH(p->g.width, {
            if (mb == 4) {
                hipLaunchKernelGGL((k_spread_lds<T, WV, 4>), dim3(p->nslots), dim3(256), 0, s,
                                   packed, pb, beta, sub);
                hipLaunchKernelGGL((k_halo<T, WV, 4>), hgrid, dim3(256), 0, s, sub, p->tile_slot,
                                   p->nt1, p->nt2, p->g.n1, p->g.n2, p->fine_ra, p->fine_rb,
                                   fine, ms);
            } else {
                hipLaunchKernelGGL((k_spread_lds<T, WV, 1>), dim3(p->nslots), dim3(256), 0, s,
                                   packed, pb, beta, sub);
                hipLaunchKernelGGL((k_halo<T, WV, 1>), hgrid, dim3(256), 0, s, sub, p->tile_slot,
                                   p->nt1, p->nt2, p->g.n1, p->g.n2, p->fine_ra, p->fine_rb,
                                   fine, ms);
            }
        });
        NUSHT_HIP(hipGetLastError());
        return NUSHT_OK;
    }
    const BandBins bb = make_band_bins(p);
    const T* coef = es_coef_of<T>(p);
    const BandRec<T>* recs = reinterpret_cast<const BandRec<T>*>(p->brec);
    const int K = 64 / p->band_w;
    const dim3 grid((unsigned)((bb.nbands + 4 * K - 1) / (4 * K)),
                    (unsigned)((bb.vt_end + 1 + bb.seg_tiles - 1) / bb.seg_tiles));
    // FP32 sweeps the group's maps together; FP64 one map per pass (four maps' FP64 register
    // rows left one wave per SIMD), reading its values from the packed rows
    NUSHT_WIDTH_SWITCH(p->g.width, {
        constexpr int SWV = WV <= 8 ? 8 : 16;
        bool done = false;
        if constexpr (sizeof(T) == 4) {
            if (mb == 4) {
                hipLaunchKernelGGL((k_spread_band<T, WV, 4, SWV>), grid, dim3(256), 0, s, recs,
                                   packed, 4, bb, beta, coef, fine, ms);
                done = true;
            }
        }
        if (!done) {
            for (int m = 0; m < mb; ++m)
                hipLaunchKernelGGL((k_spread_band<T, WV, 1, SWV>), grid, dim3(256), 0, s, recs,
                                   packed + m, mb, bb, beta, coef, fine + m * ms, ms);
        }
    });
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

}  // namespace nusht
