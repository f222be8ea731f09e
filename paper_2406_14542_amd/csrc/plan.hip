// Plans: sizes, host-computed tables, point binning and scratch (arXiv:2406.14542 Sec. III:
// the nuFFT plans are built once, before the transforms, and reused; planning is excluded
// from the timings).
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <thread>

#include "internal.h"
#include "nufft_impl.h"

namespace nusht {

static thread_local std::string g_last_error;

void set_last_error(const char* what, const char* why)
{
    g_last_error = std::string(what) + ": " + why;
}

namespace {

bool smooth7(long n)
{
    if (n < 1) return false;
    for (long p : {2L, 3L, 5L, 7L})
        while (n % p == 0) n /= p;
    return n == 1;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n in long double).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        long double z = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
        long double dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) {
                p1 = z;
                p0 = 1;
            }
            dp = n * (z * p1 - p0) / (z * z - 1);
            long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        x[i] = (double)z;
        w[i] = (double)(2.0L / ((1 - z * z) * dp * dp));
    }
}

// I(k) = int_{-1}^{1} exp(beta (sqrt(1 - z^2) - 1)) cos(alpha k z) dz, via z = sin(t), so the
// integrand exp(beta (cos t - 1)) cos(alpha k sin t) cos t is analytic on [-pi/2, pi/2].
void es_fourier(double beta, double alpha, int kmax, std::vector<double>& out)
{
    const int nq = 2 * (int)std::ceil(beta + alpha * kmax) + 64;
    std::vector<double> x, w;
    gauss_legendre(nq, x, w);
    out.assign(kmax + 1, 0.0);
    const double half_pi = 0.5 * M_PI;
    for (int q = 0; q < nq; ++q) {
        const double t = half_pi * x[q];
        const double base = w[q] * half_pi * std::exp(beta * (std::cos(t) - 1.0)) * std::cos(t);
        const double st = std::sin(t);
        for (int k = 0; k <= kmax; ++k) out[k] += base * std::cos(alpha * k * st);
    }
}

// ES kernel taps as polynomials.  With t the coordinate in grid units and ls = ceil(t - w/2)
// the first tap, the offset d = t - ls lies in (w/2 - 1, w/2]; tap a has the value
// psi(2 (d - a) / w).  For every tap the value is fitted by a polynomial of degree w in
// s = 2 d - w + 1 in [-1, 1] (interpolation at w + 1 Chebyshev points, long double), so the
// kernels form all taps of a point with w Horner steps instead of a square root and an
// exponential per tap.  coef[k * w + a] holds the coefficient of s^k for tap a.  Returns the
// largest deviation from psi on a fine grid of s.
long double es_psi(long double z, long double beta)
{
    const long double q = (1.0L - z) * (1.0L + z);
    return q > 0.0L ? expl(beta * (sqrtl(q) - 1.0L)) : 0.0L;
}

double es_poly_fit(int w, double beta, std::vector<double>& coef)
{
    const int D = w, n = D + 1;
    coef.assign((size_t)n * w, 0.0);
    std::vector<long double> s(n), A((size_t)n * n), y(n);
    for (int k = 0; k < n; ++k)
        s[k] = cosl(3.14159265358979323846264338327950288L * (k + 0.5L) / n);
    long double worst = 0.0L;
    for (int a = 0; a < w; ++a) {
        // Vandermonde system V c = psi at the nodes, Gaussian elimination with pivoting
        for (int i = 0; i < n; ++i) {
            long double pw = 1.0L;
            for (int k = 0; k < n; ++k) {
                A[(size_t)i * n + k] = pw;
                pw *= s[i];
            }
            const long double d = 0.5L * (s[i] + (long double)w - 1.0L);
            y[i] = es_psi(2.0L * (d - a) / w, beta);
        }
        for (int c = 0; c < n; ++c) {
            int piv = c;
            for (int i = c + 1; i < n; ++i)
                if (fabsl(A[(size_t)i * n + c]) > fabsl(A[(size_t)piv * n + c])) piv = i;
            if (piv != c) {
                for (int k = 0; k < n; ++k) std::swap(A[(size_t)c * n + k], A[(size_t)piv * n + k]);
                std::swap(y[c], y[piv]);
            }
            for (int i = c + 1; i < n; ++i) {
                const long double f = A[(size_t)i * n + c] / A[(size_t)c * n + c];
                for (int k = c; k < n; ++k) A[(size_t)i * n + k] -= f * A[(size_t)c * n + k];
                y[i] -= f * y[c];
            }
        }
        std::vector<long double> cc(n);
        for (int i = n - 1; i >= 0; --i) {
            long double v = y[i];
            for (int k = i + 1; k < n; ++k) v -= A[(size_t)i * n + k] * cc[k];
            cc[i] = v / A[(size_t)i * n + i];
        }
        for (int k = 0; k < n; ++k) coef[(size_t)k * w + a] = (double)cc[k];
        // deviation of the rounded coefficients on a fine grid
        for (int j = 0; j <= 2000; ++j) {
            const long double sj = -1.0L + j / 1000.0L;
            long double pv = 0.0L;
            for (int k = n - 1; k >= 0; --k) pv = pv * sj + (long double)coef[(size_t)k * w + a];
            const long double d = 0.5L * (sj + (long double)w - 1.0L);
            const long double e = fabsl(pv - es_psi(2.0L * (d - a) / w, beta));
            if (e > worst) worst = e;
        }
    }
    return (double)worst;
}

template <typename T>
int dmalloc(T** p, size_t n)
{
    *p = nullptr;
    if (n == 0) return NUSHT_OK;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) {
        set_last_error("hipMalloc", hipGetErrorString(e));
        *p = nullptr;
        return e == hipErrorOutOfMemory ? NUSHT_ENOMEM : NUSHT_EDEVICE;
    }
    return NUSHT_OK;
}

// ---- point binning kernels ----

__global__ void k_bin_keys(const double* __restrict__ theta, const double* __restrict__ phi,
                           int64_t n, int w, double s1, double s2, int n1, int n2, int nt2,
                           double* __restrict__ phw, int* __restrict__ keys,
                           int* __restrict__ idx, int* __restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double th = theta[i];
    double ph = phi[i];
    const bool bad = !(th >= 0.0 && th <= M_PI) || !isfinite(ph);
    if (bad) {
        atomicOr(flag, 1);
        ph = 0.0;
    }
    const double tp = 2.0 * M_PI;
    ph = ph - tp * floor(ph / tp);
    if (ph >= tp) ph -= tp;
    if (ph < 0.0) ph = 0.0;
    const double thc = bad ? 0.0 : th;
    double d;
    const int l1 = wrap_index(first_tap(thc, s1, w, d), n1);
    const int l2 = wrap_index(first_tap(ph, s2, w, d), n2);
    // tile id, then the row inside the tile
    keys[i] = ((l1 / kTile) * nt2 + (l2 / kTile)) * kTile + (l1 % kTile);
    idx[i] = (int)i;
    phw[i] = ph;
}

__global__ void k_gather_sorted(const double* __restrict__ theta, const double* __restrict__ phw,
                                const int* __restrict__ perm, int64_t n, double* __restrict__ sth,
                                double* __restrict__ sph, int* __restrict__ iperm)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int i = perm[k];
    sth[k] = theta[i];
    sph[k] = phw[i];
    iperm[i] = (int)k;
}

__global__ void k_mark(const int* __restrict__ keys, int64_t n, int* __restrict__ first)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    first[k] = (k == 0 || (keys[k] / kTile) != (keys[k - 1] / kTile)) ? 1 : 0;
}

__global__ void k_slots(const int* __restrict__ keys, const int* __restrict__ first,
                        const int* __restrict__ slotidx, int64_t n, int* __restrict__ slot_off,
                        int* __restrict__ slot_tile, int* __restrict__ tile_slot)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (first[k]) {
        const int s = slotidx[k];
        const int t = keys[k] / kTile;
        slot_off[s] = (int)k;
        slot_tile[s] = t;
        tile_slot[t] = s;
    }
}

// ---- band records of the spreading sweep ----
// Every sorted point e gets a record in its own column band (band_w columns) and a second one
// in the next band when its taps reach it.  Records are sorted by (band, tile row, row), and
// boff[band * nt1 + tile row] is the first record of that (band, tile row).

// first taps of sorted point e: wrapped cells and offsets
__device__ inline void rec_taps(const double* __restrict__ sth, const double* __restrict__ sph,
                                int64_t e, int w, double s1, double s2, int n1, int n2, int& l1,
                                int& l2, double& d1, double& d2)
{
    l1 = wrap_index(first_tap(sth[e], s1, w, d1), n1);
    l2 = wrap_index(first_tap(sph[e], s2, w, d2), n2);
}

__global__ void k_rec_count(const double* __restrict__ sth, const double* __restrict__ sph,
                            int64_t n, int w, double s1, double s2, int n1, int n2, int bw,
                            int* __restrict__ cnt)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    int l1, l2;
    double d1, d2;
    rec_taps(sth, sph, e, w, s1, s2, n1, n2, l1, l2, d1, d2);
    cnt[e] = (l2 % bw) + w - 1 >= bw ? 2 : 1;
}

__global__ void k_rec_keys(const double* __restrict__ sth, const double* __restrict__ sph,
                           const int* __restrict__ pos, int64_t n, int w, double s1, double s2,
                           int n1, int n2, int bw, int nt1, int* __restrict__ keys,
                           int* __restrict__ ids, int* __restrict__ ent_e,
                           signed char* __restrict__ ent_c)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    int l1, l2;
    double d1, d2;
    rec_taps(sth, sph, e, w, s1, s2, n1, n2, l1, l2, d1, d2);
    const int nbands = n2 / bw;
    const int band = l2 / bw, cin = l2 % bw;
    const int tr = l1 / kTile, row = l1 % kTile;
    const int j = pos[e];
    keys[j] = (band * nt1 + tr) * kTile + row;
    ids[j] = j;
    ent_e[j] = (int)e;
    ent_c[j] = (signed char)cin;
    if (cin + w - 1 >= bw) {
        const int b2 = band + 1 == nbands ? 0 : band + 1;
        keys[j + 1] = (b2 * nt1 + tr) * kTile + row;
        ids[j + 1] = j + 1;
        ent_e[j + 1] = (int)e;
        ent_c[j + 1] = (signed char)(cin - bw);
    }
}

template <typename T>
__global__ void k_rec_build(const int* __restrict__ ids_s, const int* __restrict__ ent_e,
                            const signed char* __restrict__ ent_c,
                            const double* __restrict__ sth, const double* __restrict__ sph,
                            const int* __restrict__ perm, int64_t nrec, int w, double s1,
                            double s2, int n1, int n2, BandRec<T>* __restrict__ rec)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nrec) return;
    const int j = ids_s[k];
    const int e = ent_e[j];
    int l1, l2;
    double d1, d2;
    rec_taps(sth, sph, e, w, s1, s2, n1, n2, l1, l2, d1, d2);
    BandRec<T> r;
    r.rc = l1 | (((int)ent_c[j] + 32) << 16);
    r.src = perm[e];
    r.s1 = (T)(2.0 * d1 - (double)(w - 1));
    r.s2 = (T)(2.0 * d2 - (double)(w - 1));
    rec[k] = r;
}

// boff[g] = first record of group g = band * nt1 + tile row (records sorted by group): a
// record that starts a group writes the start of every group after its predecessor's up to
// its own; the last record closes the remaining groups
__global__ void k_rec_off(const int* __restrict__ keys_s, int64_t nrec, int ngroups,
                          int* __restrict__ boff)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nrec) return;
    const int g = keys_s[k] / kTile;
    const int gp = k == 0 ? -1 : keys_s[k - 1] / kTile;
    for (int h = gp + 1; h <= g; ++h) boff[h] = (int)k;
    if (k == nrec - 1)
        for (int h = g + 1; h <= ngroups; ++h) boff[h] = (int)nrec;
}

__global__ void k_fill_int(int* p, int64_t n, int v)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

}  // namespace

int compute_geometry(int lmax, int mmax, double eps, int dtype, const nusht_plan_opts* opts,
                     nusht_geometry* g)
{
    if (!g) return NUSHT_EINVAL;
    std::memset(g, 0, sizeof(*g));
    if (lmax < 0 || lmax > 16383 || mmax < 0 || mmax > lmax) {
        set_last_error("geometry", "need 0 <= mmax <= lmax <= 16383");
        return NUSHT_EINVAL;
    }
    if (!(eps >= 1e-14 && eps <= 1e-1)) {
        set_last_error("geometry", "eps must lie in [1e-14, 1e-1]");
        return NUSHT_EINVAL;
    }
    if (dtype != NUSHT_F64 && dtype != NUSHT_MIXED) {
        set_last_error("geometry", "dtype must be NUSHT_F64 or NUSHT_MIXED");
        return NUSHT_EINVAL;
    }
    double sigma = 2.0, bpw = 0.0;
    int width = 0, mode = NUSHT_DFS_FUSED;
    if (opts) {
        for (int r : opts->reserved)
            if (r != 0) {
                set_last_error("geometry", "opts.reserved must be zero");
                return NUSHT_EINVAL;
            }
        if (opts->sigma != 0.0) sigma = opts->sigma;
        width = opts->width;
        bpw = opts->beta_per_w;
        mode = opts->dfs_mode;
    }
    if (!(sigma >= 1.2 && sigma <= 4.0)) {
        set_last_error("geometry", "sigma must lie in [1.2, 4]");
        return NUSHT_EINVAL;
    }
    if (mode != NUSHT_DFS_FUSED && mode != NUSHT_DFS_PAPER) {
        set_last_error("geometry", "unknown dfs_mode");
        return NUSHT_EINVAL;
    }
    // FP32 grid, FFTs and taps reach about 2e-7 at sigma = 2 and about 2e-6 at sigma = 1.25
    // (wider kernel, larger deconvolution factors at the band edge)
    if (dtype == NUSHT_MIXED && eps < (sigma >= 2.0 ? 1e-6 : 1e-5)) {
        set_last_error("geometry", "NUSHT_MIXED needs eps >= 1e-6 (sigma >= 2) or 1e-5 (sigma < 2)");
        return NUSHT_EPRECISION;
    }
    if (opts && opts->kernel_eval != NUSHT_KERNEL_POLY && opts->kernel_eval != NUSHT_KERNEL_EXACT) {
        set_last_error("geometry", "unknown kernel_eval");
        return NUSHT_EINVAL;
    }
    if (width == 0) {
        // ES kernel: error ~ exp(-pi w sqrt(1 - 1/sigma)); one extra cell of margin
        width = (int)std::ceil(std::log(1.0 / eps) / (M_PI * std::sqrt(1.0 - 1.0 / sigma))) + 1;
        if (width < kMinWidth) width = kMinWidth;
    }
    if (width < kMinWidth || width > kMaxWidth) {
        set_last_error("geometry", "kernel width outside [2, 16] (raise sigma or eps)");
        return NUSHT_EINVAL;
    }
    if (bpw == 0.0) bpw = (sigma == 2.0) ? 2.30 : 0.97 * M_PI * (1.0 - 0.5 / sigma);
    if (!(bpw > 0.0 && bpw < 10.0)) {
        set_last_error("geometry", "beta_per_w out of range");
        return NUSHT_EINVAL;
    }
    // CC rings: N_t = 2 (N_r - 1) must carry |kappa| <= lmax without touching the Nyquist bin,
    // so N_r >= lmax + 2 (N_r = lmax + 1 aliases odd-m modes), and N_t should be FFT-friendly.
    int nr = lmax + 2;
    while (!smooth7(2L * (nr - 1))) ++nr;
    int nphi = 2 * mmax + 2;
    while (!smooth7(nphi) || (nphi & 1)) ++nphi;
    auto fine = [&](int band) {
        long n = (long)std::ceil(sigma * (2.0 * band + 1.0));
        if (n < 2 * kTile) n = 2 * kTile;
        n = ((n + kTile - 1) / kTile) * kTile;
        while (!smooth7(n)) n += kTile;
        return (int)n;
    };
    g->lmax = lmax;
    g->mmax = mmax;
    g->nrings = nr;
    g->ntorus = 2 * (nr - 1);
    g->nphi = nphi;
    g->n1 = fine(lmax);
    g->n2 = fine(mmax);
    g->width = width;
    g->beta = bpw * width;
    g->sigma = sigma;
    g->tile = kTile;
    g->dtype = dtype;
    g->dfs_mode = mode;
    g->nalm = (int64_t)(mmax + 1) * (lmax + 1) - (int64_t)mmax * (mmax + 1) / 2;
    return NUSHT_OK;
}

size_t fine_elem_bytes(const nusht_plan_s* p)
{
    return p->g.dtype == NUSHT_MIXED ? sizeof(float) : sizeof(double);
}

// Scratch for up to `nmaps` maps: X and Y each hold the largest per-map intermediate of
// either mode times the batch.
int ensure_capacity(nusht_plan_s* p, int nmaps)
{
    if (nmaps <= p->bcap) return NUSHT_OK;
    const nusht_geometry& g = p->g;
    const size_t e = fine_elem_bytes(p);
    const size_t fine_real = (size_t)g.n1 * g.n2 * e;
    const size_t fine_spec = (size_t)g.n1 * (g.n2 / 2 + 1) * 2 * e;
    const size_t gpaper = (size_t)g.nrings * (g.nphi / 2 + 1) * 16;
    const size_t ring = (size_t)g.nrings * g.nphi * 8;
    const size_t torus = (size_t)g.ntorus * g.nphi * e;
    const size_t tspec = (size_t)g.ntorus * (g.nphi / 2 + 1) * 2 * e;
    const size_t gfused = (size_t)(g.mmax + 1) * g.ntorus * 2 * 8;  // doubled columns, <= c128
    size_t per = fine_real;
    for (size_t v : {fine_spec, gpaper, ring, torus, tspec, gfused}) per = v > per ? v : per;
    NUSHT_HIP(hipDeviceSynchronize());
    if (p->X) hipFree(p->X);
    if (p->Y) hipFree(p->Y);
    p->X = p->Y = nullptr;
    p->bcap = 0;
    NUSHT_TRY(dmalloc((char**)&p->X, per * nmaps));
    NUSHT_TRY(dmalloc((char**)&p->Y, per * nmaps));
    p->Xbytes = p->Ybytes = per * nmaps;
    if (!p->W) {
        NUSHT_TRY(dmalloc((char**)&p->W, fine_spec));
        p->Wbytes = fine_spec;
    }
    if (!p->V) NUSHT_TRY(dmalloc(&p->V, (size_t)g.npts * 4));
    // tile subgrids of the wide-kernel spreading: one group of up to four maps at a time
    if (spread_uses_tiles(p) && !p->Z) {
        const int P = kTile + g.width - 1;
        const size_t zb = (size_t)std::max(p->nslots, 1) * P * P * 4 * e;
        NUSHT_TRY(dmalloc((char**)&p->Z, zb));
        p->Zbytes = zb;
    }
    p->bcap = nmaps;
    return NUSHT_OK;
}

// Records of the spreading sweep (after bin_points: needs the sorted points).  Synchronises.
int build_band_records(nusht_plan_s* p, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int64_t n = g.npts;
    const int w = g.width, bw = band_width_for(w);
    const int nt1 = g.n1 / kTile, nbands = g.n2 / bw;
    const double s1 = g.n1 / (2.0 * M_PI), s2 = g.n2 / (2.0 * M_PI);
    p->band_w = bw;
    const int64_t ngroups = (int64_t)nbands * nt1;
    if (ngroups * kTile >= (1LL << 31) || 2 * n >= (1LL << 31) || g.n1 > 65536) {
        set_last_error("nusht_plan", "fine grid or point count too large for the band records");
        return NUSHT_EINVAL;
    }
    int *cnt = nullptr, *pos = nullptr, *keys = nullptr, *keys_s = nullptr, *ids = nullptr,
        *ids_s = nullptr, *ent_e = nullptr;
    signed char* ent_c = nullptr;
    void* tmp = nullptr;
    int rc = NUSHT_OK;
    const int blocks = (int)((n + 255) / 256);
    do {
        if ((rc = dmalloc(&cnt, n)) || (rc = dmalloc(&pos, n))) break;
        hipLaunchKernelGGL(k_rec_count, dim3(blocks), dim3(256), 0, s, p->sth, p->sph, n, w, s1,
                           s2, g.n1, g.n2, bw, cnt);
        size_t tb = 0, tb2 = 0;
        if (hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, pos, (int)n, s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
        if ((rc = dmalloc((char**)&tmp, tb + 16))) break;
        if (hipcub::DeviceScan::ExclusiveSum(tmp, tb, cnt, pos, (int)n, s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
        int last_pos = 0, last_cnt = 0;
        if (hipMemcpyAsync(&last_pos, pos + n - 1, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&last_cnt, cnt + n - 1, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
        const int64_t nrec = (int64_t)last_pos + last_cnt;
        p->nrec = nrec;
        if ((rc = dmalloc(&keys, nrec)) || (rc = dmalloc(&keys_s, nrec)) || (rc = dmalloc(&ids, nrec)) ||
            (rc = dmalloc(&ids_s, nrec)) || (rc = dmalloc(&ent_e, nrec)) || (rc = dmalloc(&ent_c, nrec)) ||
            (rc = dmalloc(&p->boff, ngroups + 1)))
            break;
        hipLaunchKernelGGL(k_rec_keys, dim3(blocks), dim3(256), 0, s, p->sth, p->sph, pos, n, w, s1,
                           s2, g.n1, g.n2, bw, nt1, keys, ids, ent_e, ent_c);
        int bits = 1;
        while ((1LL << bits) < ngroups * kTile) ++bits;
        if (hipcub::DeviceRadixSort::SortPairs(nullptr, tb2, keys, keys_s, ids, ids_s, (int)nrec, 0,
                                               bits, s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
        if (tb2 > tb) {
            if (hipStreamSynchronize(s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
            hipFree(tmp);
            tmp = nullptr;
            if ((rc = dmalloc((char**)&tmp, tb2 + 16))) break;
            tb = tb2;
        }
        if (hipcub::DeviceRadixSort::SortPairs(tmp, tb, keys, keys_s, ids, ids_s, (int)nrec, 0, bits,
                                               s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
        const int rblocks = (int)((nrec + 255) / 256);
        if (g.dtype == NUSHT_MIXED) {
            if ((rc = dmalloc((BandRec<float>**)&p->brec, nrec))) break;
            hipLaunchKernelGGL(k_rec_build<float>, dim3(rblocks), dim3(256), 0, s, ids_s, ent_e,
                               ent_c, p->sth, p->sph, p->perm, nrec, w, s1, s2, g.n1, g.n2,
                               reinterpret_cast<BandRec<float>*>(p->brec));
        } else {
            if ((rc = dmalloc((BandRec<double>**)&p->brec, nrec))) break;
            hipLaunchKernelGGL(k_rec_build<double>, dim3(rblocks), dim3(256), 0, s, ids_s, ent_e,
                               ent_c, p->sth, p->sph, p->perm, nrec, w, s1, s2, g.n1, g.n2,
                               reinterpret_cast<BandRec<double>*>(p->brec));
        }
        hipLaunchKernelGGL(k_rec_off, dim3(rblocks), dim3(256), 0, s, keys_s, nrec, (int)ngroups,
                           p->boff);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
    } while (0);
    hipFree(cnt);
    hipFree(pos);
    hipFree(keys);
    hipFree(keys_s);
    hipFree(ids);
    hipFree(ids_s);
    hipFree(ent_e);
    hipFree(ent_c);
    hipFree(tmp);
    return rc;
}

int bin_points(nusht_plan_s* p, const double* theta, const double* phi, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int64_t n = g.npts;
    p->nt1 = g.n1 / kTile;
    p->nt2 = g.n2 / kTile;
    const int64_t ntiles = (int64_t)p->nt1 * p->nt2;
    int *keys = nullptr, *keys_s = nullptr, *idx = nullptr, *first = nullptr, *sidx = nullptr;
    double* phw = nullptr;
    void* tmp = nullptr;
    int rc = NUSHT_OK;
    size_t tbytes = 0, t2 = 0;
    const int blocks = (int)((n + 255) / 256);
    int bits = 1;
    while ((1LL << bits) < ntiles * kTile) ++bits;
    if (ntiles * kTile >= (1LL << 31)) {
        set_last_error("nusht_plan", "fine grid too large for 32-bit bin keys");
        return NUSHT_EINVAL;
    }
    do {
        if ((rc = dmalloc(&keys, n)) || (rc = dmalloc(&keys_s, n)) || (rc = dmalloc(&idx, n)) ||
            (rc = dmalloc(&first, n)) || (rc = dmalloc(&sidx, n)) || (rc = dmalloc(&phw, n)) ||
            (rc = dmalloc(&p->perm, n)) || (rc = dmalloc(&p->iperm, n)) ||
            (rc = dmalloc(&p->sth, n)) ||
            (rc = dmalloc(&p->sph, n)) || (rc = dmalloc(&p->tile_slot, ntiles)) ||
            (rc = dmalloc(&p->dflag, 1)) || (rc = dmalloc(&p->dstatus, 1)))
            break;
        if (hipMemsetAsync(p->dflag, 0, sizeof(int), s) != hipSuccess ||
            hipMemsetAsync(p->dstatus, 0, sizeof(int), s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
        hipLaunchKernelGGL(k_bin_keys, dim3(blocks), dim3(256), 0, s, theta, phi, n, g.width,
                           g.n1 / (2.0 * M_PI), g.n2 / (2.0 * M_PI), g.n1, g.n2, p->nt2, phw,
                           keys, idx, p->dflag);
        if (hipcub::DeviceRadixSort::SortPairs(nullptr, tbytes, keys, keys_s, idx, p->perm,
                                               (int)n, 0, bits, s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
        if (hipcub::DeviceScan::ExclusiveSum(nullptr, t2, first, sidx, (int)n, s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
        if (t2 > tbytes) tbytes = t2;
        if ((rc = dmalloc((char**)&tmp, tbytes + 16))) break;
        if (hipcub::DeviceRadixSort::SortPairs(tmp, tbytes, keys, keys_s, idx, p->perm, (int)n, 0,
                                               bits, s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
        hipLaunchKernelGGL(k_gather_sorted, dim3(blocks), dim3(256), 0, s, theta, phw, p->perm, n,
                           p->sth, p->sph, p->iperm);
        hipLaunchKernelGGL(k_mark, dim3(blocks), dim3(256), 0, s, keys_s, n, first);
        if (hipcub::DeviceScan::ExclusiveSum(tmp, tbytes, first, sidx, (int)n, s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
        int last_first = 0, last_idx = 0, flag = 0;
        if (hipMemcpyAsync(&last_first, first + n - 1, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&last_idx, sidx + n - 1, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&flag, p->dflag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
        if (flag) {
            set_last_error("nusht_plan", "theta outside [0, pi] or non-finite coordinate");
            rc = NUSHT_EINVAL;
            break;
        }
        p->nslots = last_idx + last_first;
        if ((rc = dmalloc(&p->slot_off, p->nslots + 1)) || (rc = dmalloc(&p->slot_tile, p->nslots)))
            break;
        hipLaunchKernelGGL(k_fill_int, dim3((int)((ntiles + 255) / 256)), dim3(256), 0, s,
                           p->tile_slot, ntiles, -1);
        hipLaunchKernelGGL(k_slots, dim3(blocks), dim3(256), 0, s, keys_s, first, sidx, n,
                           p->slot_off, p->slot_tile, p->tile_slot);
        const int nn = (int)n;
        if (hipMemcpyAsync(p->slot_off + p->nslots, &nn, sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
        if (hipGetLastError() != hipSuccess) { rc = NUSHT_EDEVICE; break; }
    } while (0);
    hipFree(keys);
    hipFree(keys_s);
    hipFree(idx);
    hipFree(first);
    hipFree(sidx);
    hipFree(phw);
    hipFree(tmp);
    return rc;
}

// Smallest ring index j (0 <= j < ceil(N_r/2)) whose pair (j, N_r-1-j) carries any lam_lm,
// l <= lmax, above 2^-300: rings closer to the poles stay in the evanescent region of every
// l <= lmax for this m and contribute nothing (the kernels accumulate only above 2^-200).
// lam grows with sin(theta) there, so the predicate is monotone in j and bisection applies.
static bool ring_reaches(int lmax, int m, int j, int nr, const std::vector<double>& rec,
                         int64_t moff, double cm, int ce)
{
    const double th = M_PI * (double)j / (double)(nr - 1);
    const double s = std::sin(th);
    if (m > 0 && s == 0.0) return false;
    const double h = std::sin(0.5 * th);
    const double y = (2 * j == nr - 1) ? 1.0 : 2.0 * h * h;
    // log2 |lam_mm| = log2|c_m| + m log2(s), tracked as mantissa * 2^e
    int e = ce;
    double v = std::fabs(cm);
    double ls = m > 0 ? m * std::log2(s) : 0.0;
    const int le = (int)std::floor(ls);
    v *= std::exp2(ls - le);
    e += le;
    if (e > -300) return true;
    double vp = 0.0, vc = v;
    for (int l = m + 1; l <= lmax; ++l) {
        const double a = rec[2 * (moff + l)], b = rec[2 * (moff + l) + 1];
        const double vn = a * (vc - y * vc) - b * vp;
        vp = vc;
        vc = vn;
        const double big = std::fabs(vc) > std::fabs(vp) ? std::fabs(vc) : std::fabs(vp);
        if (big > 0x1p200 || (big < 0x1p-200 && big > 0.0)) {
            int k;
            std::frexp(big, &k);
            vc = std::ldexp(vc, -k);
            vp = std::ldexp(vp, -k);
            e += k;
        }
        int k2;
        std::frexp(vc, &k2);
        if (vc != 0.0 && e + k2 > -300) return true;
    }
    return false;
}

static int build_tables(nusht_plan_s* p)
{
    const nusht_geometry& g = p->g;
    const int L = g.lmax, M = g.mmax;
    // recurrence coefficients (a_lm, a_lm b_lm) in long double, rounded once
    std::vector<double> rec(2 * ((size_t)g.nalm + kRecPad), 0.0);
    for (int m = 0; m <= M; ++m) {
        const int64_t moff = (int64_t)m * (2 * L + 1 - m) / 2;
        for (int l = m + 1; l <= L; ++l) {
            const long double ll = l, mm = m, l1 = l - 1;
            const long double a = sqrtl((4 * ll * ll - 1) / (ll * ll - mm * mm));
            const long double b = sqrtl((l1 * l1 - mm * mm) / (4 * l1 * l1 - 1));
            rec[2 * (moff + l)] = (double)a;
            rec[2 * (moff + l) + 1] = (double)(a * b);
        }
    }
    // lam_mm prefactor (-1)^m sqrt((2m+1)/(4 pi) prod_{k<=m} (2k-1)/(2k)) as mantissa * 2^e
    std::vector<double> cm(M + 1);
    std::vector<int> ce(M + 1);
    {
        long double prod = 1.0L;
        int pe = 0;
        for (int m = 0; m <= M; ++m) {
            if (m > 0) {
                prod *= (2.0L * m - 1.0L) / (2.0L * m);
                int t;
                prod = frexpl(prod, &t);
                pe += t;
            }
            long double v = (2.0L * m + 1.0L) / (4.0L * 3.14159265358979323846264338327950288L) * prod;
            int e2 = pe;
            if (e2 & 1) {
                v *= 2.0L;
                e2 -= 1;
            }
            long double r = sqrtl(v);
            int t;
            r = frexpl(r, &t);
            cm[m] = (double)((m & 1) ? -r : r);
            ce[m] = e2 / 2 + t;
        }
    }
    // first live ring pair of every m
    std::vector<int> jl(M + 1, 0);
    {
        const int npairs = (g.nrings + 1) / 2;
        const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> pool;
        for (unsigned t = 0; t < nth; ++t)
            pool.emplace_back([&, t] {
                for (int m = (int)t; m <= M; m += (int)nth) {
                    const int64_t moff = (int64_t)m * (2 * L + 1 - m) / 2;
                    int lo = 0, hi = npairs;  // first live index in [lo, hi]
                    while (lo < hi) {
                        const int mid = (lo + hi) / 2;
                        if (ring_reaches(L, m, mid, g.nrings, rec, moff, cm[m], ce[m]))
                            hi = mid;
                        else
                            lo = mid + 1;
                    }
                    jl[m] = lo;
                }
            });
        for (auto& th : pool) th.join();
    }
    // first ring pair whose lam_mm = c_m sin^m(theta_j) is at least 2^-190 (sin theta_j grows
    // with j up to the equator); no lam_lm of such a pair needs the power-of-two scale
    std::vector<int> jsc(M + 1, 0);
    {
        const int npairs = (g.nrings + 1) / 2;
        for (int m = 0; m <= M; ++m) {
            const double lc = (double)ce[m] + std::log2(std::fabs(cm[m]));
            int j = 0;
            if (m > 0) {
                // bisection on the monotone log2 lam_mm(theta_j) >= -190
                int lo = 0, hi = npairs;
                while (lo < hi) {
                    const int mid = (lo + hi) / 2;
                    const double sth = std::sin(M_PI * (double)mid / (double)(g.nrings - 1));
                    const bool ok = sth > 0.0 && lc + m * std::log2(sth) >= -190.0;
                    if (ok)
                        hi = mid;
                    else
                        lo = mid + 1;
                }
                j = lo;
            }
            if (j < jl[m]) j = jl[m];
            // the synthesis splits its waves at jsc: a multiple of the spans of both of its
            // instances' waves (powers of two)
            const int span = 64 * std::max(synth_pairs_per_lane(npairs),
                                            synth_scaled_pairs_per_lane(npairs));
            jsc[m] = (j + span - 1) / span * span;
        }
    }
    // deconvolution: h / psi^(k) = 2 / (w I(k)), with the 1/N_t of the theta transform
    std::vector<double> i1, i2;
    es_fourier(g.beta, g.width * M_PI / g.n1, L, i1);
    es_fourier(g.beta, g.width * M_PI / g.n2, M, i2);
    std::vector<double> d1(L + 1), d2(M + 1);
    std::vector<float> d1f(L + 1), d2f(M + 1);
    for (int k = 0; k <= L; ++k) {
        d1[k] = 2.0 / (g.width * i1[k]) / g.ntorus;
        d1f[k] = (float)d1[k];
    }
    for (int k = 0; k <= M; ++k) {
        d2[k] = 2.0 / (g.width * i2[k]);
        d2f[k] = (float)d2[k];
    }
    // tap polynomials, used when their deviation stays well below eps (and, for FP32 taps,
    // above the FP32 rounding of their coefficients); otherwise the kernels form each tap
    // from its square root and exponential
    {
        std::vector<double> coef;
        const double dev = es_poly_fit(g.width, g.beta, coef);
        const double tol = g.dtype == NUSHT_MIXED ? std::max(0.05 * p->eps, 1e-7) : 0.05 * p->eps;
        p->es_poly_dev = dev;
        if (p->es_eval == 0 && dev <= tol) {
            std::vector<float> coeff(coef.begin(), coef.end());
            NUSHT_TRY(dmalloc(&p->es_coef, coef.size()));
            NUSHT_TRY(dmalloc(&p->es_coeff, coeff.size()));
            NUSHT_HIP(hipMemcpy(p->es_coef, coef.data(), coef.size() * sizeof(double),
                                hipMemcpyHostToDevice));
            NUSHT_HIP(hipMemcpy(p->es_coeff, coeff.data(), coeff.size() * sizeof(float),
                                hipMemcpyHostToDevice));
        }
    }
    NUSHT_TRY(dmalloc(&p->rec, (size_t)g.nalm + kRecPad));
    NUSHT_TRY(dmalloc(&p->cm_mant, M + 1));
    NUSHT_TRY(dmalloc(&p->cm_exp, M + 1));
    NUSHT_TRY(dmalloc(&p->dec1, L + 1));
    NUSHT_TRY(dmalloc(&p->dec2, M + 1));
    NUSHT_TRY(dmalloc(&p->dec1f, L + 1));
    NUSHT_TRY(dmalloc(&p->dec2f, M + 1));
    NUSHT_TRY(dmalloc(&p->jlive, M + 1));
    NUSHT_TRY(dmalloc(&p->jscale, M + 1));
    NUSHT_HIP(hipMemcpy(p->jscale, jsc.data(), jsc.size() * sizeof(int), hipMemcpyHostToDevice));
    NUSHT_HIP(hipMemcpy(p->jlive, jl.data(), jl.size() * sizeof(int), hipMemcpyHostToDevice));
    p->jlive_host = jl;
    NUSHT_HIP(hipMemcpy(p->rec, rec.data(), rec.size() * sizeof(double), hipMemcpyHostToDevice));
    NUSHT_HIP(hipMemcpy(p->cm_mant, cm.data(), cm.size() * sizeof(double), hipMemcpyHostToDevice));
    NUSHT_HIP(hipMemcpy(p->cm_exp, ce.data(), ce.size() * sizeof(int), hipMemcpyHostToDevice));
    NUSHT_HIP(hipMemcpy(p->dec1, d1.data(), d1.size() * sizeof(double), hipMemcpyHostToDevice));
    NUSHT_HIP(hipMemcpy(p->dec2, d2.data(), d2.size() * sizeof(double), hipMemcpyHostToDevice));
    NUSHT_HIP(hipMemcpy(p->dec1f, d1f.data(), d1f.size() * sizeof(float), hipMemcpyHostToDevice));
    NUSHT_HIP(hipMemcpy(p->dec2f, d2f.data(), d2f.size() * sizeof(float), hipMemcpyHostToDevice));
    return NUSHT_OK;
}

int create_fft_plans(nusht_plan_s* p);
void destroy_fft_plans(nusht_plan_s* p);

int check_device_status(nusht_plan_s* p)
{
    int cur = 0, word = 0;
    hipGetDevice(&cur);
    if (cur != p->device) hipSetDevice(p->device);
    const hipError_t e = hipDeviceSynchronize();
    const hipError_t e2 = e == hipSuccess
                              ? hipMemcpy(&word, p->dstatus, sizeof(int), hipMemcpyDeviceToHost)
                              : e;
    if (cur != p->device) hipSetDevice(cur);
    if (e2 != hipSuccess) {
        set_last_error("nusht_plan_status", hipGetErrorString(e2));
        return NUSHT_EDEVICE;
    }
    if (word & kErrAdjWait) {
        set_last_error("nusht_plan_status",
                       "a Legendre-adjoint cross-wave wait reached its bound: adjoint sums may be "
                       "wrong");
        return NUSHT_EDEVICE;
    }
    return NUSHT_OK;
}

}  // namespace nusht

using namespace nusht;

extern "C" {

int64_t nusht_nalm(int lmax, int mmax)
{
    if (lmax < 0 || mmax < 0 || mmax > lmax) return -1;
    return (int64_t)(mmax + 1) * (lmax + 1) - (int64_t)mmax * (mmax + 1) / 2;
}

int nusht_geometry_for(int lmax, int mmax, double eps, int dtype, const nusht_plan_opts* opts,
                   nusht_geometry* out)
{
    return compute_geometry(lmax, mmax, eps, dtype, opts, out);
}

const char* nusht_strerror(int status)
{
    switch (status) {
        case NUSHT_OK: return "success";
        case NUSHT_EINVAL: return "invalid argument";
        case NUSHT_ENOMEM: return "device memory allocation failed";
        case NUSHT_EDEVICE: return "HIP or rocFFT call failed";
        case NUSHT_ENOCONV: return "iterative solve did not converge within maxiter";
        case NUSHT_EPRECISION: return "requested accuracy needs NUSHT_F64";
        default: return "unknown status";
    }
}

const char* nusht_last_error(void) { return g_last_error.c_str(); }

void nusht_destroy(nusht_plan_t p)
{
    if (!p) return;
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(p->device);
    hipDeviceSynchronize();
    destroy_fft_plans(p);
    void* bufs[] = {p->rec,  p->cm_mant, p->cm_exp,   p->dec1,      p->dec2,      p->dec1f,
                    p->dec2f, p->sth,    p->sph,      p->perm,      p->iperm,     p->V,
                    p->slot_off,  p->slot_tile,
                    p->tile_slot, p->boff, p->brec, p->dflag, p->dstatus, p->X,     p->Y,         p->W,   p->Z,
                    p->fftwork,   p->rowtw, p->thetatw,
                    p->red,      p->jlive,  p->jscale, p->adj_part, p->es_coef, p->es_coeff,
                    p->spin_rec, p->spin_km, p->spin_ke, p->spin_jlive};
    for (void* b : bufs)
        if (b) hipFree(b);
    for (int c = 0; c < nusht_plan_s::kTimingSlots; ++c)
        for (int i = 0; i < ST_COUNT; ++i) {
            if (p->ev[c][i][0]) hipEventDestroy(p->ev[c][i][0]);
            if (p->ev[c][i][1]) hipEventDestroy(p->ev[c][i][1]);
        }
    if (p->fork_ev) hipEventDestroy(p->fork_ev);
    if (p->join_ev) hipEventDestroy(p->join_ev);
    if (p->side) hipStreamDestroy(p->side);
    hipSetDevice(cur);
    delete p;
}

int nusht_plan_ex(int lmax, int mmax, int64_t npts, const double* theta, const double* phi,
                  double eps, int dtype, const nusht_plan_opts* opts, void* stream,
                  nusht_plan_t* out)
{
    if (!out) return NUSHT_EINVAL;
    *out = nullptr;
    nusht_geometry g;
    NUSHT_TRY(compute_geometry(lmax, mmax, eps, dtype, opts, &g));
    if (npts < 1 || npts >= (int64_t)1 << 31 || !theta || !phi) {
        set_last_error("nusht_plan", "need 1 <= npts < 2^31 and non-null coordinates");
        return NUSHT_EINVAL;
    }
    g.npts = npts;
    nusht_plan_s* p = new nusht_plan_s();
    p->g = g;
    p->eps = eps;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    p->plan_stream = s;
    int rc = NUSHT_OK;
    do {
        if (hipGetDevice(&p->device) != hipSuccess) { rc = NUSHT_EDEVICE; break; }
        p->timing = opts ? opts->timing : 0;
        p->deterministic = opts ? (opts->deterministic != 0) : 0;
        p->es_eval = opts ? opts->kernel_eval : 0;
        if ((rc = build_tables(p))) break;
        if ((rc = bin_points(p, theta, phi, s))) break;
        if ((rc = build_band_records(p, s))) break;
        p->g.ntiles_used = p->nslots;
        if ((rc = create_fft_plans(p))) break;
        if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming) != hipSuccess) {
            rc = NUSHT_EDEVICE;
            break;
        }
        if (p->timing) {
            for (int c = 0; c < nusht_plan_s::kTimingSlots && rc == NUSHT_OK; ++c)
                for (int i = 0; i < ST_COUNT; ++i) {
                    if (hipEventCreate(&p->ev[c][i][0]) != hipSuccess ||
                        hipEventCreate(&p->ev[c][i][1]) != hipSuccess) {
                        rc = NUSHT_EDEVICE;
                        break;
                    }
                }
            if (rc != NUSHT_OK) break;
        }
    } while (0);
    if (rc != NUSHT_OK) {
        nusht_destroy(p);
        return rc;
    }
    *out = p;
    return NUSHT_OK;
}

int nusht_plan(int lmax, int mmax, int64_t npts, const double* theta, const double* phi,
               double eps, int dtype, nusht_plan_t* out)
{
    return nusht_plan_ex(lmax, mmax, npts, theta, phi, eps, dtype, nullptr, nullptr, out);
}

int nusht_plan_info(nusht_plan_t p, nusht_geometry* out)
{
    if (!p || !out) return NUSHT_EINVAL;
    *out = p->g;
    out->kernel_eval = p->es_coef ? NUSHT_KERNEL_POLY : NUSHT_KERNEL_EXACT;
    out->kernel_poly_dev = p->es_poly_dev;
    return NUSHT_OK;
}

int nusht_plan_status(nusht_plan_t p)
{
    if (!p) return NUSHT_EINVAL;
    return check_device_status(p);
}

}  // extern "C"
