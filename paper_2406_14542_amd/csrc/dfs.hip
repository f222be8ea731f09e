// Double-Fourier-sphere glue (arXiv:2406.14542 Sec. II.B, Fig. 1, Eq. 5/6) and the
// deconvolution steps of the nuFFT (Sec. III):
//   D   doubling: extend each meridian over the pole, T(t, k) = g(theta_{N_t - t}, phi_k + pi)
//       for N_r <= t < N_t;
//   D^H folding:  g'(j, k) = T'(j, k) + [1 <= j <= N_r - 2] T'(N_t - j, k + N_phi/2);
//   N step (i)   b(kappa, mu) = C(kappa, mu) h1 h2 / (psi1^(kappa) psi2^(mu)), zero-padded to the
//                fine grid;
//   N^H step (iii) the same factor after truncating the fine spectrum to |kappa| <= L, mu <= M.
// The fine spectrum is kept in two layouts: the band spectrum [mu][i] (mu <= M, all n1 rows
// i = kappa mod n1, the input/output of the theta pass) and the row spectrum [i][mu]
// (mu < n2/2+1, window rows only, the input/output of the phi pass); 32 x 32 LDS-tiled
// transposes link them.  All of these are memory-bound; each thread touches each element
// once and consecutive threads touch consecutive addresses.
#include "internal.h"

namespace nusht {
namespace {

template <typename T>
struct cplx;
template <>
struct cplx<double> {
    using type = double2;
};
template <>
struct cplx<float> {
    using type = float2;
};

// ---- paper mode ----------------------------------------------------------------------

__global__ void k_zero_rows(double2* __restrict__ G, int nr, int row_len, int m_from,
                            int64_t map_stride)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nr) return;
    double2* row = G + (int64_t)blockIdx.y * map_stride + (int64_t)j * row_len;
    for (int m = m_from; m < row_len; ++m) row[m] = make_double2(0.0, 0.0);
}

// D of Fig. 1: torus row t < N_r is ring t, row t >= N_r is ring N_t - t shifted by pi in phi,
// times sgn (1 for spin 0; (-1)^s for the Q, U components of a spin-s field, whose local basis
// turns over with the doubling).  k_fold is its adjoint.
template <typename TO>
__global__ void k_double(const double* __restrict__ ring, TO* __restrict__ torus, int nr, int nt,
                         int nphi, double sgn)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    const int b = blockIdx.z;
    if (k >= nphi) return;
    const double* rg = ring + (int64_t)b * nr * nphi;
    double v;
    if (t < nr) {
        v = rg[(int64_t)t * nphi + k];
    } else {
        int kk = k + nphi / 2;
        if (kk >= nphi) kk -= nphi;
        v = sgn * rg[(int64_t)(nt - t) * nphi + kk];
    }
    torus[(int64_t)b * nt * nphi + (int64_t)t * nphi + k] = (TO)v;
}

template <typename TI>
__global__ void k_fold(const TI* __restrict__ torus, double* __restrict__ ring, int nr, int nt,
                       int nphi, double sgn)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int b = blockIdx.z;
    if (k >= nphi) return;
    const TI* tg = torus + (int64_t)b * nt * nphi;
    double v = (double)tg[(int64_t)j * nphi + k];
    if (j >= 1 && j <= nr - 2) {
        int kk = k + nphi / 2;
        if (kk >= nphi) kk -= nphi;
        v += sgn * (double)tg[(int64_t)(nt - j) * nphi + kk];
    }
    ring[(int64_t)b * nr * nphi + (int64_t)j * nphi + k] = v;
}

// fine row of kappa and back
__device__ inline int kappa_of_row(int i, int n) { return i <= n / 2 ? i : i - n; }

// torus spectrum ts[b][t][mu] (rows of tw) -> band spectrum [b][mu][i], deconvolved and
// zero-padded (paper mode)
template <typename T>
__global__ void k_deconv_pad_paper(const typename cplx<T>::type* __restrict__ ts,
                                   typename cplx<T>::type* __restrict__ band, int nt, int tw,
                                   int n1, int lmax, int mmax, const T* __restrict__ d1,
                                   const T* __restrict__ d2, T scale)
{
    using C = typename cplx<T>::type;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int mu = blockIdx.y;
    const int b = blockIdx.z;
    if (i >= n1) return;
    const int kap = kappa_of_row(i, n1);
    const int ak = kap < 0 ? -kap : kap;
    C v;
    v.x = 0;
    v.y = 0;
    if (ak <= lmax) {
        const int t = kap < 0 ? kap + nt : kap;
        const C c = ts[(int64_t)b * nt * tw + (int64_t)t * tw + mu];
        const T f = d1[ak] * d2[mu] * scale;
        v.x = c.x * f;
        v.y = c.y * f;
    }
    band[((int64_t)b * (mmax + 1) + mu) * n1 + i] = v;
}

// band spectrum [b][mu][i] -> torus spectrum ts[b][t][mu] (zero for mu > M or |kappa| > L)
template <typename T>
__global__ void k_deconv_trunc_paper(const typename cplx<T>::type* __restrict__ band,
                                     typename cplx<T>::type* __restrict__ ts, int nt, int tw,
                                     int n1, int lmax, int mmax, const T* __restrict__ d1,
                                     const T* __restrict__ d2, T scale)
{
    using C = typename cplx<T>::type;
    const int mu = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    const int b = blockIdx.z;
    if (mu >= tw) return;
    const int kap = kappa_of_row(t, nt);
    const int ak = kap < 0 ? -kap : kap;
    C v;
    v.x = 0;
    v.y = 0;
    if (ak <= lmax && mu <= mmax) {
        const int i = kap < 0 ? kap + n1 : kap;
        const C c = band[((int64_t)b * (mmax + 1) + mu) * n1 + i];
        const T f = d1[ak] * d2[mu] * scale;
        v.x = c.x * f;
        v.y = c.y * f;
    }
    ts[(int64_t)b * nt * tw + (int64_t)t * tw + mu] = v;
}

// fused mode: column spectrum Cs[b][m][t] (t < N_t) <-> band spectrum [b][m][i]; both are
// contiguous along the theta frequency, so these are plain gathers
template <typename T>
__global__ void k_deconv_pad_fused(const typename cplx<T>::type* __restrict__ cs,
                                   typename cplx<T>::type* __restrict__ band, int nt, int n1,
                                   int lmax, int mmax, const T* __restrict__ d1,
                                   const T* __restrict__ d2)
{
    using C = typename cplx<T>::type;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    const int b = blockIdx.z;
    if (i >= n1) return;
    const int kap = kappa_of_row(i, n1);
    const int ak = kap < 0 ? -kap : kap;
    C v;
    v.x = 0;
    v.y = 0;
    if (ak <= lmax) {
        const int t = kap < 0 ? kap + nt : kap;
        const C c = cs[((int64_t)b * (mmax + 1) + m) * nt + t];
        const T f = d1[ak] * d2[m];
        v.x = c.x * f;
        v.y = c.y * f;
    }
    band[((int64_t)b * (mmax + 1) + m) * n1 + i] = v;
}

template <typename T>
__global__ void k_deconv_trunc_fused(const typename cplx<T>::type* __restrict__ band,
                                     typename cplx<T>::type* __restrict__ cs, int nt, int n1,
                                     int lmax, int mmax, const T* __restrict__ d1,
                                     const T* __restrict__ d2)
{
    using C = typename cplx<T>::type;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    const int b = blockIdx.z;
    if (t >= nt) return;
    const int kap = kappa_of_row(t, nt);
    const int ak = kap < 0 ? -kap : kap;
    C v;
    v.x = 0;
    v.y = 0;
    if (ak <= lmax) {
        const int i = kap < 0 ? kap + n1 : kap;
        const C c = band[((int64_t)b * (mmax + 1) + m) * n1 + i];
        const T f = d1[ak] * d2[m];
        v.x = c.x * f;
        v.y = c.y * f;
    }
    cs[((int64_t)b * (mmax + 1) + m) * nt + t] = v;
}

// ---- band <-> row spectrum transposes (one map) -----------------------------------------

constexpr int kT = 32;

// window row of compact index q: rows [0, ra) then [n1 - rb, n1)
__device__ inline int window_row(int q, int ra, int rb, int n1) { return q < ra ? q : n1 - rb + (q - ra); }

// rows[i][mu] = band[mu][i] for mu <= M, 0 for mu in (M, fw) (fw = the row width); window
// rows only.
// Block 32 x 8 threads: tile of 32 compact rows x 32 columns.
template <typename C>
__global__ __launch_bounds__(256) void k_band_to_rows(const C* __restrict__ band,
                                                      C* __restrict__ rows, int n1, int fw,
                                                      int ncol, int ra, int rb)
{
    __shared__ C tile[kT][kT + 1];
    const int q0 = blockIdx.y * kT, mu0 = blockIdx.x * kT;
    const int nq = ra + rb;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const bool live = mu0 < ncol;
    if (live) {
        // read along i (contiguous in the band spectrum)
        for (int r = ty; r < kT; r += blockDim.y) {
            const int mu = mu0 + r, q = q0 + tx;
            C v;
            v.x = 0;
            v.y = 0;
            if (mu < ncol && q < nq) v = band[(int64_t)mu * n1 + window_row(q, ra, rb, n1)];
            tile[r][tx] = v;
        }
        __syncthreads();
    }
    for (int r = ty; r < kT; r += blockDim.y) {
        const int q = q0 + r, mu = mu0 + tx;
        if (q >= nq || mu >= fw) continue;
        C v;
        if (live) {
            v = tile[tx][r];
        } else {
            v.x = 0;
            v.y = 0;
        }
        rows[(int64_t)window_row(q, ra, rb, n1) * fw + mu] = v;
    }
}

// band[mu][i] = rows[i][mu] for window rows, 0 for the other rows; mu <= M.  COMPACT: the
// window rows only (tile rows index the compact rows q < ra + rb), nothing else written.
template <typename C, bool COMPACT>
__global__ __launch_bounds__(256) void k_rows_to_band(const C* __restrict__ rows,
                                                      C* __restrict__ band, int n1, int fw,
                                                      int ncol, int ra, int rb)
{
    __shared__ C tile[kT][kT + 1];
    const int i0 = blockIdx.y * kT, mu0 = blockIdx.x * kT;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int nrow = COMPACT ? ra + rb : n1;
    // read along mu (contiguous in the row spectrum)
    for (int r = ty; r < kT; r += blockDim.y) {
        const int q = i0 + r, mu = mu0 + tx;
        const int i = COMPACT ? window_row(q, ra, rb, n1) : q;
        C v;
        v.x = 0;
        v.y = 0;
        if (q < nrow && mu < ncol && (i < ra || i >= n1 - rb)) v = rows[(int64_t)i * fw + mu];
        tile[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < kT; r += blockDim.y) {
        const int mu = mu0 + r, q = i0 + tx;
        if (mu >= ncol || q >= nrow) continue;
        const int i = COMPACT ? window_row(q, ra, rb, n1) : q;
        band[(int64_t)mu * n1 + i] = tile[tx][r];
    }
}

}  // namespace

int launch_zero_nyquist_rows(const nusht_plan_s* p, double* G, int nmaps, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int row = g.nphi / 2 + 1;
    if (g.mmax + 1 >= row) return NUSHT_OK;
    dim3 grid((g.nrings + 255) / 256, nmaps);
    hipLaunchKernelGGL(k_zero_rows, grid, dim3(256), 0, s, reinterpret_cast<double2*>(G),
                       g.nrings, row, g.mmax + 1, (int64_t)g.nrings * row);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int launch_band_to_rows(const nusht_plan_s* p, const void* band, void* rows, int rw,
                        hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int fw = rw, nq = p->fine_ra + p->fine_rb;
    dim3 grid((fw + kT - 1) / kT, (nq + kT - 1) / kT);
    dim3 block(kT, 8);
    if (g.dtype == NUSHT_MIXED)
        hipLaunchKernelGGL(k_band_to_rows<float2>, grid, block, 0, s,
                           reinterpret_cast<const float2*>(band), reinterpret_cast<float2*>(rows),
                           g.n1, fw, g.mmax + 1, p->fine_ra, p->fine_rb);
    else
        hipLaunchKernelGGL(k_band_to_rows<double2>, grid, block, 0, s,
                           reinterpret_cast<const double2*>(band),
                           reinterpret_cast<double2*>(rows), g.n1, fw, g.mmax + 1, p->fine_ra,
                           p->fine_rb);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int launch_rows_to_band(const nusht_plan_s* p, const void* rows, int rw, void* band,
                        hipStream_t s, bool window_only)
{
    const nusht_geometry& g = p->g;
    const int fw = rw;
    const int nrow = window_only ? p->fine_ra + p->fine_rb : g.n1;
    dim3 grid((g.mmax + 1 + kT - 1) / kT, (nrow + kT - 1) / kT);
    dim3 block(kT, 8);
#define NUSHT_R2B(C, COMPACT)                                                                  \
    hipLaunchKernelGGL((k_rows_to_band<C, COMPACT>), grid, block, 0, s,                        \
                       reinterpret_cast<const C*>(rows), reinterpret_cast<C*>(band), g.n1, fw, \
                       g.mmax + 1, p->fine_ra, p->fine_rb)
    if (g.dtype == NUSHT_MIXED) {
        if (window_only) NUSHT_R2B(float2, true);
        else NUSHT_R2B(float2, false);
    } else {
        if (window_only) NUSHT_R2B(double2, true);
        else NUSHT_R2B(double2, false);
    }
#undef NUSHT_R2B
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int launch_double(const nusht_plan_s* p, const double* ring, void* torus, int nmaps, int f32,
                  hipStream_t s, double sgn)
{
    const nusht_geometry& g = p->g;
    dim3 grid((g.nphi + 255) / 256, g.ntorus, nmaps);
    if (f32)
        hipLaunchKernelGGL(k_double<float>, grid, dim3(256), 0, s, ring,
                           reinterpret_cast<float*>(torus), g.nrings, g.ntorus, g.nphi, sgn);
    else
        hipLaunchKernelGGL(k_double<double>, grid, dim3(256), 0, s, ring,
                           reinterpret_cast<double*>(torus), g.nrings, g.ntorus, g.nphi, sgn);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int launch_fold(const nusht_plan_s* p, const void* torus, double* ring, int nmaps, int f32,
                hipStream_t s, double sgn)
{
    const nusht_geometry& g = p->g;
    dim3 grid((g.nphi + 255) / 256, g.nrings, nmaps);
    if (f32)
        hipLaunchKernelGGL(k_fold<float>, grid, dim3(256), 0, s,
                           reinterpret_cast<const float*>(torus), ring, g.nrings, g.ntorus, g.nphi,
                           sgn);
    else
        hipLaunchKernelGGL(k_fold<double>, grid, dim3(256), 0, s,
                           reinterpret_cast<const double*>(torus), ring, g.nrings, g.ntorus,
                           g.nphi, sgn);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int launch_deconv_pad(const nusht_plan_s* p, const void* tspec, void* band, int nmaps, int fused,
                      int f32, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    dim3 grid((g.n1 + 255) / 256, g.mmax + 1, nmaps);
    if (fused) {
        if (f32)
            hipLaunchKernelGGL(k_deconv_pad_fused<float>, grid, dim3(256), 0, s,
                               reinterpret_cast<const float2*>(tspec),
                               reinterpret_cast<float2*>(band), g.ntorus, g.n1, g.lmax, g.mmax,
                               p->dec1f, p->dec2f);
        else
            hipLaunchKernelGGL(k_deconv_pad_fused<double>, grid, dim3(256), 0, s,
                               reinterpret_cast<const double2*>(tspec),
                               reinterpret_cast<double2*>(band), g.ntorus, g.n1, g.lmax, g.mmax,
                               p->dec1, p->dec2);
    } else {
        const int tw = g.nphi / 2 + 1;
        const double sc = 1.0 / g.nphi;
        if (f32)
            hipLaunchKernelGGL(k_deconv_pad_paper<float>, grid, dim3(256), 0, s,
                               reinterpret_cast<const float2*>(tspec),
                               reinterpret_cast<float2*>(band), g.ntorus, tw, g.n1, g.lmax,
                               g.mmax, p->dec1f, p->dec2f, (float)sc);
        else
            hipLaunchKernelGGL(k_deconv_pad_paper<double>, grid, dim3(256), 0, s,
                               reinterpret_cast<const double2*>(tspec),
                               reinterpret_cast<double2*>(band), g.ntorus, tw, g.n1, g.lmax,
                               g.mmax, p->dec1, p->dec2, sc);
    }
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int launch_deconv_trunc(const nusht_plan_s* p, const void* band, void* tspec, int nmaps,
                        int fused, int f32, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    if (fused) {
        dim3 grid((g.ntorus + 255) / 256, g.mmax + 1, nmaps);
        if (f32)
            hipLaunchKernelGGL(k_deconv_trunc_fused<float>, grid, dim3(256), 0, s,
                               reinterpret_cast<const float2*>(band),
                               reinterpret_cast<float2*>(tspec), g.ntorus, g.n1, g.lmax, g.mmax,
                               p->dec1f, p->dec2f);
        else
            hipLaunchKernelGGL(k_deconv_trunc_fused<double>, grid, dim3(256), 0, s,
                               reinterpret_cast<const double2*>(band),
                               reinterpret_cast<double2*>(tspec), g.ntorus, g.n1, g.lmax, g.mmax,
                               p->dec1, p->dec2);
    } else {
        const int tw = g.nphi / 2 + 1;
        dim3 grid((tw + 255) / 256, g.ntorus, nmaps);
        const double sc = 1.0 / g.nphi;
        if (f32)
            hipLaunchKernelGGL(k_deconv_trunc_paper<float>, grid, dim3(256), 0, s,
                               reinterpret_cast<const float2*>(band),
                               reinterpret_cast<float2*>(tspec), g.ntorus, tw, g.n1, g.lmax,
                               g.mmax, p->dec1f, p->dec2f, (float)sc);
        else
            hipLaunchKernelGGL(k_deconv_trunc_paper<double>, grid, dim3(256), 0, s,
                               reinterpret_cast<const double2*>(band),
                               reinterpret_cast<double2*>(tspec), g.ntorus, tw, g.n1, g.lmax,
                               g.mmax, p->dec1, p->dec2, sc);
    }
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

}  // namespace nusht
