// Type-2 interpolation and type-1 spreading of the ES-kernel nuFFT on the fine torus grid
// (arXiv:2406.14542 Sec. III: N and N^H, "shared memory" spreading).
//
// Kernel: psi(z) = exp(beta (sqrt(1 - z^2) - 1)) for |z| < 1, z = 2 (x - x_l) / (w h).
// For a coordinate x with t = x / h (grid units) the w taps start at cell
//   ls = ceil(t - w/2),  and tap a has z_a = 2 (t - ls - a) / w  in (-1, 1].
// Points were binned by the plan into kTile x kTile tiles by (ls1 mod n1, ls2 mod n2); a
// workgroup owns one non-empty tile ("slot") and the tile's window of
// (kTile + w - 1)^2 cells, which it stages in LDS.
//  * interpolation: window loaded once from HBM, every point of the tile reads its w x w taps
//    from LDS, results written packed per point in the caller's point order;
//  * spreading: the tile's points (values packed per point, fetched through the permutation)
//    are added into an FP64 LDS copy of the window with LDS atomics; the window is written
//    once to a per-slot subgrid, and a second pass sums, for every fine cell, the subgrids of
//    the (at most four) windows that cover it (no global atomics).
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
                                                PointBins pb, T beta, double* __restrict__ out,
                                                int64_t npts)
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
        es_taps<T, W>(d1, beta, p1v);
        es_taps<T, W>(d2, beta, p2v);
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

// Spreading with LDS atomics, batched.  The block stages up to NB of the slot's points (tap
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

template <typename T>
int dispatch_interp_impl(const nusht_plan_s* p, const T* fine, double* out, int nmaps, T beta,
                         hipStream_t s)
{
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
                                   fine + b * ms, ms, pb, beta, p->V, npts);
                hipLaunchKernelGGL((k_unpack_points<4, sizeof(T) == 4>), dim3(pblocks), dim3(256),
                                   0, s, p->V, p->iperm, npts, out + b * npts);
            } else {
                hipLaunchKernelGGL((k_interp<T, WV, 1, false>), dim3(p->nslots), dim3(256), 0,
                                   s, fine + b * ms, ms, pb, beta, out + b * npts, npts);
            }
        });
        NUSHT_HIP(hipGetLastError());
        b += mb;
    }
    return NUSHT_OK;
}

// Spreading of the caller's maps [b, b + mb) (`vals` = its map block [mb][npts]) into the
// slot subgrids: the values are first packed [point][mb] in the caller's order into the
// plan's point scratch, and the spreading kernel fetches a point's mb values with one load
// through the permutation.
template <typename T>
int spread_group_impl(const nusht_plan_s* p, const double* vals, T* sub, int mb, T beta,
                      hipStream_t s)
{
    if (p->nslots == 0) return NUSHT_OK;
    const PointBins pb = make_bins(p);
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
    NUSHT_WIDTH_SWITCH(p->g.width, {
        if (mb == 4)
            hipLaunchKernelGGL((k_spread_lds<T, WV, 4>), dim3(p->nslots), dim3(256), 0, s,
                               packed, pb, beta, sub);
        else
            hipLaunchKernelGGL((k_spread_lds<T, WV, 1>), dim3(p->nslots), dim3(256), 0, s,
                               packed, pb, beta, sub);
    });
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

// halo reduction of the slot subgrids into fine maps [b, b + mb)
template <typename T>
int halo_group_impl(const nusht_plan_s* p, const T* sub, T* fine, int b, int mb, hipStream_t s)
{
    const int64_t ms = (int64_t)p->g.n1 * p->g.n2;
    dim3 hgrid((p->g.n2 + 255) / 256, p->fine_ra + p->fine_rb);
    NUSHT_WIDTH_SWITCH(p->g.width, {
        if (mb == 4)
            hipLaunchKernelGGL((k_halo<T, WV, 4>), hgrid, dim3(256), 0, s, sub, p->tile_slot,
                               p->nt1, p->nt2, p->g.n1, p->g.n2, p->fine_ra, p->fine_rb,
                               fine + b * ms, ms);
        else
            hipLaunchKernelGGL((k_halo<T, WV, 1>), hgrid, dim3(256), 0, s, sub, p->tile_slot,
                               p->nt1, p->nt2, p->g.n1, p->g.n2, p->fine_ra, p->fine_rb,
                               fine + b * ms, ms);
    });
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

}  // namespace nusht
