// Double-Fourier-sphere glue (arXiv:2406.14542 Sec. II.B, Fig. 1, Eq. 5/6) and the
// deconvolution steps of the nuFFT (Sec. III):
//   D   doubling: extend each meridian over the pole, T(t, k) = g(theta_{N_t - t}, phi_k + pi)
//       for N_r <= t < N_t;
//   D^H folding:  g'(j, k) = T'(j, k) + [1 <= j <= N_r - 2] T'(N_t - j, k + N_phi/2);
//   N step (i)   b(kappa, mu) = C(kappa, mu) h1 h2 / (psi1^(kappa) psi2^(mu)), zero-padded to the
//                fine grid;
//   N^H step (iii) the same factor after truncating the fine spectrum to |kappa| <= L, mu <= M.
// All of these are memory-bound; each thread touches each element once and consecutive
// threads touch consecutive addresses (the fused-mode deconvolutions also transpose
// between the (m, t) and (kappa, mu) layouts through a 32 x 32 LDS tile).
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

template <typename TO>
__global__ void k_double(const double* __restrict__ ring, TO* __restrict__ torus, int nr, int nt,
                         int nphi)
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
        v = rg[(int64_t)(nt - t) * nphi + kk];
    }
    torus[(int64_t)b * nt * nphi + (int64_t)t * nphi + k] = (TO)v;
}

template <typename TI>
__global__ void k_fold(const TI* __restrict__ torus, double* __restrict__ ring, int nr, int nt,
                       int nphi)
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
        v += (double)tg[(int64_t)(nt - j) * nphi + kk];
    }
    ring[(int64_t)b * nr * nphi + (int64_t)j * nphi + k] = v;
}

// torus spectrum [N_t][N_phi/2+1] -> fine spectrum [n1][n2/2+1]
template <typename T>
__global__ void k_deconv_pad_paper(const typename cplx<T>::type* __restrict__ ts,
                                   typename cplx<T>::type* __restrict__ fs, int nt, int tw,
                                   int n1, int fw, int lmax, int mmax,
                                   const T* __restrict__ d1, const T* __restrict__ d2, T scale)
{
    using C = typename cplx<T>::type;
    const int mu = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int b = blockIdx.z;
    if (mu >= fw) return;
    const int kap = (i <= n1 / 2) ? i : i - n1;
    const int ak = kap < 0 ? -kap : kap;
    C v;
    v.x = 0;
    v.y = 0;
    if (ak <= lmax && mu <= mmax) {
        const int t = kap < 0 ? kap + nt : kap;
        const C c = ts[(int64_t)b * nt * tw + (int64_t)t * tw + mu];
        const T f = d1[ak] * d2[mu] * scale;
        v.x = c.x * f;
        v.y = c.y * f;
    }
    fs[(int64_t)b * n1 * fw + (int64_t)i * fw + mu] = v;
}

// fine spectrum [n1][n2/2+1] -> torus spectrum [N_t][N_phi/2+1]
template <typename T>
__global__ void k_deconv_trunc_paper(const typename cplx<T>::type* __restrict__ fs,
                                     typename cplx<T>::type* __restrict__ ts, int nt, int tw,
                                     int n1, int fw, int lmax, int mmax,
                                     const T* __restrict__ d1, const T* __restrict__ d2, T scale)
{
    using C = typename cplx<T>::type;
    const int mu = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    const int b = blockIdx.z;
    if (mu >= tw) return;
    const int kap = (t <= nt / 2) ? t : t - nt;
    const int ak = kap < 0 ? -kap : kap;
    C v;
    v.x = 0;
    v.y = 0;
    if (ak <= lmax && mu <= mmax) {
        const int i = kap < 0 ? kap + n1 : kap;
        const C c = fs[(int64_t)b * n1 * fw + (int64_t)i * fw + mu];
        const T f = d1[ak] * d2[mu] * scale;
        v.x = c.x * f;
        v.y = c.y * f;
    }
    ts[(int64_t)b * nt * tw + (int64_t)t * tw + mu] = v;
}

// ---- fused mode: (m, t) <-> (kappa, mu) transposes --------------------------------------

constexpr int kT = 32;

// column spectrum Cs[b][m][t] (t < N_t, the theta-FFT of the doubled column) -> fine
// spectrum [n1][n2/2+1].  Block (32 x 8 threads) covers fine rows i0..i0+31, columns
// mu0..mu0+31.
template <typename T>
__global__ __launch_bounds__(256) void k_deconv_pad_fused(
    const typename cplx<T>::type* __restrict__ cs, typename cplx<T>::type* __restrict__ fs,
    int nt, int n1, int fw, int lmax, int mmax, const T* __restrict__ d1,
    const T* __restrict__ d2, int ra, int rb)
{
    using C = typename cplx<T>::type;
    __shared__ C tile[kT][kT + 1];
    const int i0 = blockIdx.y * kT, mu0 = blockIdx.x * kT;
    const int b = blockIdx.z;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const C* cb = cs + (int64_t)b * (mmax + 1) * nt;
    // block-level test: does the tile meet |kappa| <= L and mu <= M at all?
    const int ilo = i0, ihi = min(i0 + kT, n1) - 1;
    const bool rows_hit = (ilo <= lmax) || (ihi >= n1 - lmax);
    const bool live = rows_hit && mu0 <= mmax;
    // Columns above mmax are read only by the phi pass, and only in rows [0, ra) and
    // [n1 - rb, n1); elsewhere the tile is never read and need not be written.
    if (mu0 > mmax && ilo >= ra && ihi < n1 - rb) return;
    if (live) {
        // load Cs[mu][kappa(i)] with threads along i (coalesced along t)
        for (int r = ty; r < kT; r += blockDim.y) {
            const int mu = mu0 + r;
            const int i = i0 + tx;
            C v;
            v.x = 0;
            v.y = 0;
            if (mu <= mmax && i < n1) {
                const int kap = (i <= n1 / 2) ? i : i - n1;
                const int ak = kap < 0 ? -kap : kap;
                if (ak <= lmax) {
                    const int t = kap < 0 ? kap + nt : kap;
                    const C c = cb[(int64_t)mu * nt + t];
                    const T f = d1[ak] * d2[mu];
                    v.x = c.x * f;
                    v.y = c.y * f;
                }
            }
            tile[r][tx] = v;
        }
        __syncthreads();
    }
    for (int r = ty; r < kT; r += blockDim.y) {
        const int i = i0 + r;
        const int mu = mu0 + tx;
        if (i >= n1 || mu >= fw) continue;
        C v;
        if (live) {
            v = tile[tx][r];
        } else {
            v.x = 0;
            v.y = 0;
        }
        fs[(int64_t)b * n1 * fw + (int64_t)i * fw + mu] = v;
    }
}

// fine spectrum [n1][n2/2+1] -> column spectrum Cs[b][m][t] for m <= M, t < N_t
template <typename T>
__global__ __launch_bounds__(256) void k_deconv_trunc_fused(
    const typename cplx<T>::type* __restrict__ fs, typename cplx<T>::type* __restrict__ cs,
    int nt, int n1, int fw, int lmax, int mmax, const T* __restrict__ d1,
    const T* __restrict__ d2)
{
    using C = typename cplx<T>::type;
    __shared__ C tile[kT][kT + 1];
    const int t0 = blockIdx.x * kT, m0 = blockIdx.y * kT;
    const int b = blockIdx.z;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const C* fb = fs + (int64_t)b * n1 * fw;
    // load fine[i(t)][m] with threads along m
    for (int r = ty; r < kT; r += blockDim.y) {
        const int t = t0 + r;
        const int m = m0 + tx;
        C v;
        v.x = 0;
        v.y = 0;
        if (t < nt && m <= mmax) {
            const int kap = (t <= nt / 2) ? t : t - nt;
            const int ak = kap < 0 ? -kap : kap;
            if (ak <= lmax) {
                const int i = kap < 0 ? kap + n1 : kap;
                const C c = fb[(int64_t)i * fw + m];
                const T f = d1[ak] * d2[m];
                v.x = c.x * f;
                v.y = c.y * f;
            }
        }
        tile[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < kT; r += blockDim.y) {
        const int m = m0 + r;
        const int t = t0 + tx;
        if (m > mmax || t >= nt) continue;
        cs[(int64_t)b * (mmax + 1) * nt + (int64_t)m * nt + t] = tile[tx][r];
    }
}

// fs[row_lo + blockIdx.y][0 .. ncol) = 0
template <typename C>
__global__ void k_zero_band(C* __restrict__ fs, int row_lo, int fw, int ncol)
{
    const int mu = blockIdx.x * blockDim.x + threadIdx.x;
    if (mu >= ncol) return;
    C z;
    z.x = 0;
    z.y = 0;
    fs[(int64_t)(row_lo + blockIdx.y) * fw + mu] = z;
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

int launch_zero_band_rows(const nusht_plan_s* p, void* fspec, int row_lo, int row_hi,
                          hipStream_t s)
{
    const nusht_geometry& g = p->g;
    if (row_hi <= row_lo) return NUSHT_OK;
    const int fw = g.n2 / 2 + 1;
    dim3 grid((g.mmax + 1 + 255) / 256, row_hi - row_lo);
    if (g.dtype == NUSHT_MIXED)
        hipLaunchKernelGGL(k_zero_band<float2>, grid, dim3(256), 0, s,
                           reinterpret_cast<float2*>(fspec), row_lo, fw, g.mmax + 1);
    else
        hipLaunchKernelGGL(k_zero_band<double2>, grid, dim3(256), 0, s,
                           reinterpret_cast<double2*>(fspec), row_lo, fw, g.mmax + 1);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int launch_double(const nusht_plan_s* p, const double* ring, void* torus, int nmaps, int f32,
                  hipStream_t s)
{
    const nusht_geometry& g = p->g;
    dim3 grid((g.nphi + 255) / 256, g.ntorus, nmaps);
    if (f32)
        hipLaunchKernelGGL(k_double<float>, grid, dim3(256), 0, s, ring,
                           reinterpret_cast<float*>(torus), g.nrings, g.ntorus, g.nphi);
    else
        hipLaunchKernelGGL(k_double<double>, grid, dim3(256), 0, s, ring,
                           reinterpret_cast<double*>(torus), g.nrings, g.ntorus, g.nphi);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int launch_fold(const nusht_plan_s* p, const void* torus, double* ring, int nmaps, int f32,
                hipStream_t s)
{
    const nusht_geometry& g = p->g;
    dim3 grid((g.nphi + 255) / 256, g.nrings, nmaps);
    if (f32)
        hipLaunchKernelGGL(k_fold<float>, grid, dim3(256), 0, s,
                           reinterpret_cast<const float*>(torus), ring, g.nrings, g.ntorus, g.nphi);
    else
        hipLaunchKernelGGL(k_fold<double>, grid, dim3(256), 0, s,
                           reinterpret_cast<const double*>(torus), ring, g.nrings, g.ntorus,
                           g.nphi);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int launch_deconv_pad(const nusht_plan_s* p, const void* tspec, void* fspec, int nmaps, int fused,
                      int f32, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int fw = g.n2 / 2 + 1;
    if (fused) {
        dim3 grid((fw + kT - 1) / kT, (g.n1 + kT - 1) / kT, nmaps);
        dim3 block(kT, 8);
        if (f32)
            hipLaunchKernelGGL(k_deconv_pad_fused<float>, grid, block, 0, s,
                               reinterpret_cast<const float2*>(tspec),
                               reinterpret_cast<float2*>(fspec), g.ntorus, g.n1, fw, g.lmax,
                               g.mmax, p->dec1f, p->dec2f, p->fine_ra, p->fine_rb);
        else
            hipLaunchKernelGGL(k_deconv_pad_fused<double>, grid, block, 0, s,
                               reinterpret_cast<const double2*>(tspec),
                               reinterpret_cast<double2*>(fspec), g.ntorus, g.n1, fw, g.lmax,
                               g.mmax, p->dec1, p->dec2, p->fine_ra, p->fine_rb);
    } else {
        const int tw = g.nphi / 2 + 1;
        dim3 grid((fw + 255) / 256, g.n1, nmaps);
        const double sc = 1.0 / g.nphi;
        if (f32)
            hipLaunchKernelGGL(k_deconv_pad_paper<float>, grid, dim3(256), 0, s,
                               reinterpret_cast<const float2*>(tspec),
                               reinterpret_cast<float2*>(fspec), g.ntorus, tw, g.n1, fw, g.lmax,
                               g.mmax, p->dec1f, p->dec2f, (float)sc);
        else
            hipLaunchKernelGGL(k_deconv_pad_paper<double>, grid, dim3(256), 0, s,
                               reinterpret_cast<const double2*>(tspec),
                               reinterpret_cast<double2*>(fspec), g.ntorus, tw, g.n1, fw, g.lmax,
                               g.mmax, p->dec1, p->dec2, sc);
    }
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int launch_deconv_trunc(const nusht_plan_s* p, const void* fspec, void* tspec, int nmaps,
                        int fused, int f32, hipStream_t s)
{
    const nusht_geometry& g = p->g;
    const int fw = g.n2 / 2 + 1;
    if (fused) {
        dim3 grid((g.ntorus + kT - 1) / kT, (g.mmax + 1 + kT - 1) / kT, nmaps);
        dim3 block(kT, 8);
        if (f32)
            hipLaunchKernelGGL(k_deconv_trunc_fused<float>, grid, block, 0, s,
                               reinterpret_cast<const float2*>(fspec),
                               reinterpret_cast<float2*>(tspec), g.ntorus, g.n1, fw, g.lmax,
                               g.mmax, p->dec1f, p->dec2f);
        else
            hipLaunchKernelGGL(k_deconv_trunc_fused<double>, grid, block, 0, s,
                               reinterpret_cast<const double2*>(fspec),
                               reinterpret_cast<double2*>(tspec), g.ntorus, g.n1, fw, g.lmax,
                               g.mmax, p->dec1, p->dec2);
    } else {
        const int tw = g.nphi / 2 + 1;
        dim3 grid((tw + 255) / 256, g.ntorus, nmaps);
        const double sc = 1.0 / g.nphi;
        if (f32)
            hipLaunchKernelGGL(k_deconv_trunc_paper<float>, grid, dim3(256), 0, s,
                               reinterpret_cast<const float2*>(fspec),
                               reinterpret_cast<float2*>(tspec), g.ntorus, tw, g.n1, fw, g.lmax,
                               g.mmax, p->dec1f, p->dec2f, (float)sc);
        else
            hipLaunchKernelGGL(k_deconv_trunc_paper<double>, grid, dim3(256), 0, s,
                               reinterpret_cast<const double2*>(fspec),
                               reinterpret_cast<double2*>(tspec), g.ntorus, tw, g.n1, fw, g.lmax,
                               g.mmax, p->dec1, p->dec2, sc);
    }
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

}  // namespace nusht
