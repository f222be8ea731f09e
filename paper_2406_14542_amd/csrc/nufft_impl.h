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
//  * spreading: waves sweep column bands row by row and keep the rows a point can reach in
//    registers (k_spread_band): every fine cell is written once, with its points summed in a
//    fixed order, and no atomics or partial grids are involved.
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

// Spreading (type 1, N^H of Eq. 6): u(l1, l2) = sum_i f_i psi(row taps) psi(column taps), the
// exact adjoint of the interpolation above (same taps).
//
// Band sweep, no atomics.  The fine columns are cut into bands of SW = band_w columns; each
// group of SW lanes of a wave owns one band (lane q = column c0 + q), so a wave sweeps
// K = 64 / SW bands side by side.  A band's points -- its own band's points and those of the
// band to its left whose taps reach it (SW >= w) -- are taken in order of their first-tap
// row, tile row after tile row.  Every lane keeps the w rows [R, R + w) of its column in
// registers: a point whose first tap is row r (>= R, rows only grow) first pushes rows R .. r-1
// out to the fine grid, then adds f psi1[a] psi2[q - c] to rows r + a.  Each cell is written
// once, by the lane that owns its column, as the sum of its points in a fixed order: the
// result does not depend on scheduling, and nothing is written twice.
//
// Rows are handled on a virtual axis: physical tile row nt1 - 1 (points near theta = 0 whose
// first tap wraps below row 0) is virtual tile row -1, so a band's rows run on without a wrap
// from -kTile up.  The rows are cut into segments of seg_tiles tile rows (grid.y); a segment
// owns the rows of its tile rows and also sweeps the points of the tile row above it whose
// taps reach its first row (and drops their rows above it), so segments never write the same
// cell either.  The owned rows of all segments are exactly the rows any point window reaches
// ([n1 - kTile, n1) and [0, ra)); when every row is reached, the first segment's overlap row
// is the last tile row shifted by -n1, which carries the wrap.
struct BandBins {
    const double* sth;
    const double* sph;
    const int* perm;
    const int* band_off;   // [nslots * nsub + 1]
    const int* tile_slot;  // [nt1 * nt2]
    int nt1, nt2, n1, n2, nsub, nbands;
    double s1, s2;
    int vt_end;     // virtual tile rows [-1, vt_end) can hold points
    int vrow_hi;    // owned virtual rows are [-kTile, vrow_hi)
    int seg_tiles;  // tile rows per segment
};

constexpr int kNoRow = 0x7fffffff;

template <typename T, int MB>
struct BandHead {
    int r, c;  // first tap: virtual row, column relative to the band start
    T s1, s2;  // offsets of the first taps as s = 2 d - w + 1 in (-1, 1], formed in FP64
    T f[MB];   // the point's values
};

// first sorted point of band group g of tile (ptr, tcol), or an empty range
__device__ inline void band_range(const BandBins& bb, int ptr, int tcol, int sub, int& p, int& e)
{
    const int sl = bb.tile_slot[ptr * bb.nt2 + tcol];
    if (sl < 0) {
        p = e = 0;
        return;
    }
    const int g = sl * bb.nsub + sub;
    p = bb.band_off[g];
    e = bb.band_off[g + 1];
}

template <typename T, int W, int MB>
__device__ inline int band_row(const BandBins& bb, int p, int voff)
{
    double d;
    return wrap_index(first_tap(bb.sth[p], bb.s1, W, d), bb.n1) + voff;
}

template <typename T, int W, int MB>
__device__ inline void band_decode(const BandBins& bb, const T* __restrict__ vals, int p,
                                   int voff, int cbase, BandHead<T, MB>& h)
{
    double d1, d2;
    const int l1 = first_tap(bb.sth[p], bb.s1, W, d1);
    const int l2 = first_tap(bb.sph[p], bb.s2, W, d2);
    h.r = wrap_index(l1, bb.n1) + voff;
    h.c = wrap_index(l2, bb.n2) - cbase;
    h.s1 = (T)(2.0 * d1 - (double)(W - 1));
    h.s2 = (T)(2.0 * d2 - (double)(W - 1));
    const int64_t src = bb.perm[p];
#pragma unroll
    for (int m = 0; m < MB; ++m) h.f[m] = vals[src * MB + m];
}

template <typename T, int W, int MB, int SW>
__global__ __launch_bounds__(256) void k_spread_band(const T* __restrict__ vals, BandBins bb,
                                                     T beta, const T* __restrict__ coef,
                                                     T* __restrict__ fine, int64_t map_stride)
{
    constexpr int K = 64 / SW;
    static_assert(SW >= W && kTile % SW == 0,
                  "one band to the left reaches a band; a group's lanes hold the row taps");
    const int lane = threadIdx.x & 63;
    const int grp = lane / SW, q = lane - grp * SW;
    const int band = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * K + grp;
    const bool bvalid = band < bb.nbands;
    const int c0 = bvalid ? band * SW : 0;
    const int tcol = c0 / kTile, sub = (c0 % kTile) / SW;
    const int lband = !bvalid ? 0 : band == 0 ? bb.nbands - 1 : band - 1;
    const int lc0 = lband * SW;
    const int ltcol = lc0 / kTile, lsub = (lc0 % kTile) / SW;
    // the left band's columns in this band's frame (band 0: the last band, one period back)
    const int lbase = band == 0 ? c0 + bb.n2 : c0;
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

    T acc[W][MB];
#pragma unroll
    for (int a = 0; a < W; ++a)
#pragma unroll
        for (int m = 0; m < MB; ++m) acc[a][m] = T(0);
    int R = first_row;

    // push row R out (if this segment owns it) and move the register rows up by one
    auto push_row = [&]() {
        if (bvalid && R >= own_lo && R < own_hi) {
            const int pr = R < 0 ? R + bb.n1 : R;
            T* o = fine + (int64_t)pr * bb.n2 + c0 + q;
#pragma unroll
            for (int m = 0; m < MB; ++m) o[m * map_stride] = acc[0][m];
        }
#pragma unroll
        for (int a = 0; a < W - 1; ++a)
#pragma unroll
            for (int m = 0; m < MB; ++m) acc[a][m] = acc[a + 1][m];
#pragma unroll
        for (int m = 0; m < MB; ++m) acc[W - 1][m] = T(0);
        ++R;
    };

    // the lists of the current tile row: own band [po, eo), left band [pl, el); the first
    // row opened is the overlap row vt0 - 1
    int vt = vt0 - 2;
    int po = 0, eo = 0, pl = 0, el = 0, voff = 0;
    BandHead<T, MB> ho, hl;
    ho.r = hl.r = kNoRow;
    ho.c = hl.c = 0;
    ho.s1 = ho.s2 = hl.s1 = hl.s2 = T(0);
#pragma unroll
    for (int m = 0; m < MB; ++m) ho.f[m] = hl.f[m] = T(0);
    bool live = bvalid;
    // open tile row vt: list ranges, and in the overlap row the first point that can reach
    // the segment's rows (rows are sorted along a list: lower bound by bisection)
    auto open_row = [&]() {
        const int ptr = ((vt % bb.nt1) + bb.nt1) % bb.nt1;
        voff = (vt - ptr) * kTile;
        band_range(bb, ptr, tcol, sub, po, eo);
        band_range(bb, ptr, ltcol, lsub, pl, el);
        if (vt < vt0) {
            int lo = po, hi = eo;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (band_row<T, W, MB>(bb, mid, voff) < first_row) lo = mid + 1; else hi = mid;
            }
            po = lo;
            lo = pl;
            hi = el;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (band_row<T, W, MB>(bb, mid, voff) < first_row) lo = mid + 1; else hi = mid;
            }
            pl = lo;
        }
    };
    // next head of the own list / of the left list (skipping points whose taps miss the band)
    auto next_own = [&]() {
        if (po < eo) {
            band_decode<T, W, MB>(bb, vals, po, voff, c0, ho);
            ++po;
        } else {
            ho.r = kNoRow;
        }
    };
    auto next_left = [&]() {
        hl.r = kNoRow;
        while (pl < el) {
            band_decode<T, W, MB>(bb, vals, pl, voff, lbase, hl);
            ++pl;
            if (hl.c > -W) return;
            hl.r = kNoRow;
        }
    };

    while (__any(live)) {
        // the next point of this band, moving on to later tile rows as lists run out
        while (live && ho.r == kNoRow && hl.r == kNoRow) {
            ++vt;
            if (vt >= vt1) {
                live = false;
                break;
            }
            open_row();
            next_own();
            next_left();
        }
        const bool take_own = live && ho.r <= hl.r;
        BandHead<T, MB> h = take_own ? ho : hl;
        const bool has = live && h.r != kNoRow;
        // push the rows above the point's first row
        const int target = has ? h.r : R;
        while (__any(R < target)) {
            if (R < target) push_row();
        }
        // add the point: column tap of this lane, row taps from lanes 0 .. W-1 of the group
        // (a group without a point adds exact zeros: its head's values are not used)
        const int b = q - h.c;
        const bool act = has && b >= 0 && b < W;
        T p1, p2;
        if (poly) {
            // taps q of the point's row and column offsets, then this lane's column tap b
            // from lane b of the group
            const T t1 = (has && q < W) ? es_tap_poly<T, W>(h.s1, creg) : T(0);
            const T t2 = (has && q < W) ? es_tap_poly<T, W>(h.s2, creg) : T(0);
            const T t2b = __shfl(t2, grp * SW + (act ? b : 0), 64);
            p1 = t1;
            p2 = act ? t2b : T(0);
        } else {
            // z of tap a = 2 (d - a) / w = (s + w - 1 - 2 a) / w
            p2 = act ? es_value<T>((h.s2 + T(W - 1 - 2 * b)) * cw * T(0.5), beta) : T(0);
            p1 = (has && q < W) ? es_value<T>((h.s1 + T(W - 1 - 2 * q)) * cw * T(0.5), beta)
                                : T(0);
        }
        T g[MB];
#pragma unroll
        for (int m = 0; m < MB; ++m) g[m] = act ? h.f[m] * p2 : T(0);
#pragma unroll
        for (int a = 0; a < W; ++a) {
            const T pa = __shfl(p1, grp * SW + a, 64);
#pragma unroll
            for (int m = 0; m < MB; ++m) acc[a][m] += g[m] * pa;
        }
        if (has) {
            if (take_own) next_own();
            else next_left();
        }
    }
    // the rows after the last point, up to the end of the segment
    while (__any(R < own_hi)) {
        if (R < own_hi) push_row();
    }
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
    bb.sth = p->sth;
    bb.sph = p->sph;
    bb.perm = p->perm;
    bb.band_off = p->band_off;
    bb.tile_slot = p->tile_slot;
    bb.nt1 = p->nt1;
    bb.nt2 = p->nt2;
    bb.n1 = p->g.n1;
    bb.n2 = p->g.n2;
    bb.nsub = p->nsub;
    bb.nbands = p->g.n2 / p->band_w;
    bb.s1 = p->g.n1 / (2.0 * M_PI);
    bb.s2 = p->g.n2 / (2.0 * M_PI);
    bb.vt_end = p->band_vt_end;
    bb.vrow_hi = p->band_vrow_hi;
    bb.seg_tiles = p->band_seg_tiles;
    return bb;
}

// Spreading of the caller's maps [b, b + mb) (`vals` = its map block [mb][npts]) straight onto
// the fine grids of those maps: the values are first packed [point][mb] in the caller's order
// into the plan's point scratch, so that the band kernel fetches a point's mb values with one
// load through the permutation.
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
    const BandBins bb = make_band_bins(p);
    const T* coef = es_coef_of<T>(p);
    const int64_t ms = (int64_t)p->g.n1 * p->g.n2;
    const int K = 64 / p->band_w;
    const dim3 grid((unsigned)((bb.nbands + 4 * K - 1) / (4 * K)),
                    (unsigned)((bb.vt_end + 1 + bb.seg_tiles - 1) / bb.seg_tiles));
    NUSHT_WIDTH_SWITCH(p->g.width, {
        constexpr int SWV = WV <= 8 ? 8 : 16;
        if (mb == 4)
            hipLaunchKernelGGL((k_spread_band<T, WV, 4, SWV>), grid, dim3(256), 0, s, packed, bb,
                               beta, coef, fine, ms);
        else
            hipLaunchKernelGGL((k_spread_band<T, WV, 1, SWV>), grid, dim3(256), 0, s, packed, bb,
                               beta, coef, fine, ms);
    });
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

}  // namespace nusht
