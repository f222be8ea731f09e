// Learned per-point quadrature weights that precondition the least-squares inverse.
//
// A small multilayer perceptron maps features of a point's neighbourhood in a coarse
// density map to a positive weight w_i; the weights form the row preconditioner W of the
// CGLS solve (nusht_solve) and its initial iterate S^H W d.  Everything here is FP32 except
// the transform calls.
//
//   density:  64 x 128 equal-angle (theta, phi) histogram, normalised to 1 for uniform points
//   features: [log rho bilinear at the point, log rho of the 3 x 3 cells around the point's
//              cell (phi periodic, theta clamped), cos theta, sin theta]      (12 values)
//   network:  12 -> 128 -> 128 -> 128 (tanh) -> 1, w = softplus(z) * scale
//   training: loss = <r, r>_m / <a*, a*>_m with r = S^H (W d) - a*; its gradient with respect
//             to w_i is 2 d_i (S r)_i / <a*, a*>_m (one synthesis), then back through the net.
//
// Parameter layout (FP32, transposed weights so a layer's outputs for one input are
// contiguous): W1t[12][128] b1[128] W2t[128][128] b2[128] W3t[128][128] b3[128] w4[128] b4[1].
#include <mutex>

#include "internal.h"

namespace nusht {
namespace {

constexpr int kIn = 12;
constexpr int kHid = 128;
constexpr int oW1 = 0;
constexpr int oB1 = oW1 + kIn * kHid;
constexpr int oW2 = oB1 + kHid;
constexpr int oB2 = oW2 + kHid * kHid;
constexpr int oW3 = oB2 + kHid;
constexpr int oB3 = oW3 + kHid * kHid;
constexpr int oW4 = oB3 + kHid;
constexpr int oB4 = oW4 + kHid;
constexpr int kParams = oB4 + 1;

constexpr int kTileP = 64;        // points per tile (one per lane)
constexpr int kLd = kHid + 1;     // padded LDS row: lanes read different rows without conflicts
constexpr int kQ = kHid / 4;      // outputs per wave (4 waves split a layer's 128 outputs)

__device__ inline float softplus(float z) { return z > 20.f ? z : log1pf(expf(z)); }
__device__ inline float sigmoid(float z) { return 1.f / (1.f + expf(-z)); }

__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// out[p][32 q .. 32 q + 31] = tanh(W^T in[p] + b) for the tile's 64 points; the weights of
// this wave's quarter are wave-uniform (scalar loads).
template <int NIN, int LDI>
__device__ inline void dense_tanh(const float* __restrict__ Wt, const float* __restrict__ b,
                                  const float* in, float* out)
{
    const int q = wave_id();
    const int lane = threadIdx.x & 63;
    float acc[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) acc[i] = b[q * kQ + i];
    for (int k = 0; k < NIN; ++k) {
        const float a = in[lane * LDI + k];
        const float* wr = Wt + k * kHid + q * kQ;
#pragma unroll
        for (int i = 0; i < kQ; ++i) acc[i] = fmaf(wr[i], a, acc[i]);
    }
#pragma unroll
    for (int i = 0; i < kQ; ++i) out[lane * kLd + q * kQ + i] = tanhf(acc[i]);
}

struct TileBufs {
    float x0[kTileP * kIn];
    float a1[kTileP * kLd];
    float a2[kTileP * kLd];
    float a3[kTileP * kLd];
    float z4[kTileP];
};

// forward pass of one tile into the LDS buffers (256 threads)
__device__ inline void tile_forward(const float* __restrict__ prm, const float* __restrict__ feat,
                                    int64_t p0, int64_t npts, TileBufs& s)
{
    for (int e = threadIdx.x; e < kTileP * kIn; e += blockDim.x) {
        const int64_t p = p0 + e / kIn;
        s.x0[e] = p < npts ? feat[p0 * kIn + e] : 0.f;
    }
    __syncthreads();
    dense_tanh<kIn, kIn>(prm + oW1, prm + oB1, s.x0, s.a1);
    __syncthreads();
    dense_tanh<kHid, kLd>(prm + oW2, prm + oB2, s.a1, s.a2);
    __syncthreads();
    dense_tanh<kHid, kLd>(prm + oW3, prm + oB3, s.a2, s.a3);
    __syncthreads();
    if (threadIdx.x < kTileP) {
        const int lane = threadIdx.x;
        float z = prm[oB4];
        for (int k = 0; k < kHid; ++k) z = fmaf(prm[oW4 + k], s.a3[lane * kLd + k], z);
        s.z4[lane] = z;
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ prm,
                                                     const float* __restrict__ feat, int64_t npts,
                                                     float scale, float* __restrict__ w)
{
    __shared__ TileBufs s;
    const int64_t p0 = (int64_t)blockIdx.x * kTileP;
    tile_forward(prm, feat, p0, npts, s);
    if (threadIdx.x < kTileP && p0 + threadIdx.x < npts)
        w[p0 + threadIdx.x] = softplus(s.z4[threadIdx.x]) * scale;
}

// Backward: grid-stride over tiles; every block accumulates the parameter gradient of its
// tiles in registers (thread t owns output unit j = t % 128 of W2t/W3t for input rows
// k in [64 (t / 128), +64)), then writes one partial vector; k_mlp_reduce sums the partials
// in block order.
__global__ __launch_bounds__(256) void k_mlp_backward(const float* __restrict__ prm,
                                                      const float* __restrict__ feat,
                                                      const float* __restrict__ gw, int64_t npts,
                                                      float scale, float* __restrict__ partial)
{
    __shared__ TileBufs s;
    __shared__ float g4[kTileP];
    __shared__ float dl[kTileP * kLd];  // delta of the current layer
    const int t = threadIdx.x;
    const int j = t & (kHid - 1);
    const int kh = __builtin_amdgcn_readfirstlane(t >> 7);  // which half of the input rows
    float dW2[64], dW3[64];
    float dW1[kIn / 2], db1 = 0.f, db2 = 0.f, db3 = 0.f, dw4 = 0.f, db4 = 0.f;
#pragma unroll
    for (int k = 0; k < 64; ++k) dW2[k] = dW3[k] = 0.f;
#pragma unroll
    for (int k = 0; k < kIn / 2; ++k) dW1[k] = 0.f;

    const int64_t ntiles = (npts + kTileP - 1) / kTileP;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t p0 = tile * kTileP;
        tile_forward(prm, feat, p0, npts, s);
        // output layer: g4 = dL/dz4 = dL/dw * scale * sigmoid(z4)
        if (t < kTileP) {
            const int64_t p = p0 + t;
            g4[t] = p < npts ? gw[p] * scale * sigmoid(s.z4[t]) : 0.f;
        }
        __syncthreads();
        // dw4, db4 and delta3 = g4 w4 (1 - a3^2); threads 0..127 own unit j
        if (t < kHid) {
            float acc = 0.f, accb = 0.f;
            for (int p = 0; p < kTileP; ++p) {
                acc = fmaf(g4[p], s.a3[p * kLd + j], acc);
                accb += g4[p];
            }
            dw4 += acc;
            if (t == 0) db4 += accb;
        }
        for (int e = t; e < kTileP * kHid; e += blockDim.x) {
            const int p = e / kHid, u = e % kHid;
            const float a = s.a3[p * kLd + u];
            dl[p * kLd + u] = g4[p] * prm[oW4 + u] * (1.f - a * a);
        }
        __syncthreads();
        // dW3t[k][j] += sum_p a2[p][k] delta3[p][j];  db3[j] += sum_p delta3[p][j]
        for (int p = 0; p < kTileP; ++p) {
            const float d = dl[p * kLd + j];
            const float* ar = s.a2 + p * kLd + 64 * kh;
#pragma unroll
            for (int k = 0; k < 64; ++k) dW3[k] = fmaf(ar[k], d, dW3[k]);
            if (kh == 0) db3 += d;
        }
        // delta2[p][k] = (sum_j W3t[k][j] delta3[p][j]) (1 - a2^2): thread -> (p = t % 64,
        // k block of 32 = t / 64); computed into registers, then stored over delta3
        float d2[kQ];
        {
            const int p = t & 63;
            const int kb = wave_id();
#pragma unroll
            for (int i = 0; i < kQ; ++i) d2[i] = 0.f;
            for (int jj = 0; jj < kHid; ++jj) {
                const float dv = dl[p * kLd + jj];
#pragma unroll
                for (int i = 0; i < kQ; ++i)
                    d2[i] = fmaf(prm[oW3 + (kb * kQ + i) * kHid + jj], dv, d2[i]);
            }
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const float a = s.a2[p * kLd + kb * kQ + i];
                d2[i] *= (1.f - a * a);
            }
        }
        __syncthreads();
        {
            const int p = t & 63;
            const int kb = wave_id();
#pragma unroll
            for (int i = 0; i < kQ; ++i) dl[p * kLd + kb * kQ + i] = d2[i];
        }
        __syncthreads();
        // dW2t[k][j] += sum_p a1[p][k] delta2[p][j]
        for (int p = 0; p < kTileP; ++p) {
            const float d = dl[p * kLd + j];
            const float* ar = s.a1 + p * kLd + 64 * kh;
#pragma unroll
            for (int k = 0; k < 64; ++k) dW2[k] = fmaf(ar[k], d, dW2[k]);
            if (kh == 0) db2 += d;
        }
        // delta1 = (W2t delta2) (1 - a1^2)
        {
            const int p = t & 63;
            const int kb = wave_id();
#pragma unroll
            for (int i = 0; i < kQ; ++i) d2[i] = 0.f;
            for (int jj = 0; jj < kHid; ++jj) {
                const float dv = dl[p * kLd + jj];
#pragma unroll
                for (int i = 0; i < kQ; ++i)
                    d2[i] = fmaf(prm[oW2 + (kb * kQ + i) * kHid + jj], dv, d2[i]);
            }
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const float a = s.a1[p * kLd + kb * kQ + i];
                d2[i] *= (1.f - a * a);
            }
        }
        __syncthreads();
        {
            const int p = t & 63;
            const int kb = wave_id();
#pragma unroll
            for (int i = 0; i < kQ; ++i) dl[p * kLd + kb * kQ + i] = d2[i];
        }
        __syncthreads();
        // dW1t[k][j] += sum_p x0[p][k] delta1[p][j] (k in this thread's half of the 12 inputs)
        for (int p = 0; p < kTileP; ++p) {
            const float d = dl[p * kLd + j];
#pragma unroll
            for (int k = 0; k < kIn / 2; ++k)
                dW1[k] = fmaf(s.x0[p * kIn + kh * (kIn / 2) + k], d, dW1[k]);
            if (kh == 0) db1 += d;
        }
        __syncthreads();
    }
    float* out = partial + (int64_t)blockIdx.x * kParams;
#pragma unroll
    for (int k = 0; k < 64; ++k) {
        out[oW2 + (64 * kh + k) * kHid + j] = dW2[k];
        out[oW3 + (64 * kh + k) * kHid + j] = dW3[k];
    }
#pragma unroll
    for (int k = 0; k < kIn / 2; ++k) out[oW1 + (kh * (kIn / 2) + k) * kHid + j] = dW1[k];
    if (kh == 0) {
        out[oB1 + j] = db1;
        out[oB2 + j] = db2;
        out[oB3 + j] = db3;
        out[oW4 + j] = dw4;
        if (j == 0) out[oB4] = db4;
    }
}

__global__ void k_mlp_reduce(const float* __restrict__ partial, int nblocks,
                             float* __restrict__ grad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kParams) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * kParams + i];
    grad[i] = s;
}

__global__ void k_adam(float* __restrict__ prm, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    prm[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---- density map and features ----

__global__ void k_density_count(const double* __restrict__ th, const double* __restrict__ ph,
                                int64_t n, int nt, int np, unsigned int* __restrict__ cnt)
{
    // cell decisions are plain products and differences, rounded one at a time
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a = (int)(th[i] * (nt / M_PI));
    a = min(max(a, 0), nt - 1);
    double pw = ph[i] - 2.0 * M_PI * floor(ph[i] / (2.0 * M_PI));
    int b = (int)(pw * (np / (2.0 * M_PI)));
    b = min(max(b, 0), np - 1);
    atomicAdd(&cnt[a * np + b], 1u);
}

__global__ void k_zero_counts(unsigned int* __restrict__ cnt, int n)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) cnt[e] = 0u;
}

// rho = count / (N * area / 4 pi): 1 for uniform points
__global__ void k_density_norm(const unsigned int* __restrict__ cnt, int nt, int np, int64_t n,
                               float* __restrict__ rho)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nt * np) return;
    const int a = e / np;
    const double area = (cos(M_PI * a / nt) - cos(M_PI * (a + 1) / nt)) * (2.0 * M_PI / np);
    rho[e] = (float)((double)cnt[e] / ((double)n * area / (4.0 * M_PI)));
}

__device__ inline float log_rho(const float* rho, int a, int b, int nt, int np)
{
    a = min(max(a, 0), nt - 1);
    b = ((b % np) + np) % np;
    return logf(fmaxf(rho[a * np + b], 1e-3f));
}

__global__ void k_features(const double* __restrict__ th, const double* __restrict__ ph, int64_t n,
                           const float* __restrict__ rho, int nt, int np, float* __restrict__ f)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double t = th[i];
    const double pw = ph[i] - 2.0 * M_PI * floor(ph[i] / (2.0 * M_PI));
    // cell-centre coordinates for the bilinear interpolation
    const double u = t * (nt / M_PI) - 0.5, v = pw * (np / (2.0 * M_PI)) - 0.5;
    const int a0 = (int)floor(u), b0 = (int)floor(v);
    const float fu = (float)(u - a0), fv = (float)(v - b0);
    const float l00 = log_rho(rho, a0, b0, nt, np), l01 = log_rho(rho, a0, b0 + 1, nt, np);
    const float l10 = log_rho(rho, a0 + 1, b0, nt, np), l11 = log_rho(rho, a0 + 1, b0 + 1, nt, np);
    float* o = f + i * kIn;
    o[0] = (1 - fu) * ((1 - fv) * l00 + fv * l01) + fu * ((1 - fv) * l10 + fv * l11);
    const int ac = min(max((int)(t * (nt / M_PI)), 0), nt - 1);
    const int bc = min(max((int)(pw * (np / (2.0 * M_PI))), 0), np - 1);
    int q = 1;
    for (int da = -1; da <= 1; ++da)
        for (int db = -1; db <= 1; ++db) o[q++] = log_rho(rho, ac + da, bc + db, nt, np);
    o[10] = (float)cos(t);
    o[11] = (float)sin(t);
}

// ---- weight loss ----

__global__ void k_weighted_map(const float* __restrict__ w, const double* __restrict__ d,
                               double* __restrict__ out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)w[i] * d[i];
}

__global__ void k_sub_alm(double2* __restrict__ c, const double2* __restrict__ a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 v = c[i];
    const double2 b = a[i];
    v.x -= b.x;
    v.y -= b.y;
    c[i] = v;
}

constexpr int kRB = 1024, kRT = 256;

__global__ __launch_bounds__(kRT) void k_mdot(const double2* __restrict__ a, int64_t n, int lmax,
                                              double* __restrict__ partial)
{
    __shared__ double sh[kRT];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 x = a[i];
        const double v = x.x * x.x + x.y * x.y;
        acc += (i <= lmax) ? v : 2.0 * v;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kRT) void k_sum(const double* __restrict__ partial, int n,
                                             double* __restrict__ out)
{
    __shared__ double sh[kRT];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partial[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_weight_grad(const double* __restrict__ d, const double* __restrict__ q,
                              const double* __restrict__ den, float* __restrict__ g, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) g[i] = (float)(2.0 * d[i] * q[i] / *den);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace
}  // namespace nusht

using namespace nusht;

extern "C" {

int64_t nusht_mlp_param_count(void) { return kParams; }

int nusht_density_map(const double* theta, const double* phi, int64_t npts, int ntheta, int nphi,
                      float* density, void* stream)
{
    if (!theta || !phi || !density || npts < 1 || ntheta < 1 || nphi < 1 ||
        (int64_t)ntheta * nphi > (1 << 24)) {
        set_last_error("nusht_density_map", "bad arguments");
        return NUSHT_EINVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned int* cnt = nullptr;
    const size_t nb = (size_t)ntheta * nphi;
    NUSHT_HIP(hipMallocAsync((void**)&cnt, nb * sizeof(unsigned int), s));
    NUSHT_HIP(hipMemsetAsync(cnt, 0, nb * sizeof(unsigned int), s));
    hipLaunchKernelGGL(k_density_count, dim3(nblk(npts)), dim3(256), 0, s, theta, phi, npts,
                       ntheta, nphi, cnt);
    hipLaunchKernelGGL(k_density_norm, dim3(nblk((int64_t)nb)), dim3(256), 0, s, cnt, ntheta,
                       nphi, npts, density);
    NUSHT_HIP(hipGetLastError());
    NUSHT_HIP(hipFreeAsync(cnt, s));
    return NUSHT_OK;
}

// Fixed device array holding the cell counts of nusht_density_map_noalloc, one copy per GPU
// for the life of the process (kDensityScratchCells counts, 256 KiB).  Host code never passes
// `scratch` itself to a kernel: its device address on each GPU comes from
// hipGetSymbolAddress, looked up once per device on that device's first call.
constexpr int kDensityScratchCells = 1 << 16;
static __device__ __align__(256) unsigned int scratch[kDensityScratchCells];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned int* g_scratch_ptr[kMaxDevices] = {};

int density_scratch(unsigned int** out)
{
    int dev = 0;
    NUSHT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_last_error("nusht_density_map_noalloc", "device index out of range");
        return NUSHT_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        NUSHT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = reinterpret_cast<unsigned int*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return NUSHT_OK;
}
}  // namespace

int nusht_density_map_noalloc(const double* theta, const double* phi, int64_t npts, int ntheta,
                              int nphi, float* density, void* stream)
{
    if (!theta || !phi || !density || npts < 1 || ntheta < 1 || nphi < 1) {
        set_last_error("nusht_density_map_noalloc", "bad arguments");
        return NUSHT_EINVAL;
    }
    if ((int64_t)ntheta * nphi > kDensityScratchCells) {
        set_last_error("nusht_density_map_noalloc",
                       "ntheta * nphi exceeds the fixed count buffer (65536 cells)");
        return NUSHT_EINVAL;
    }
    unsigned int* cnt = nullptr;
    NUSHT_TRY(density_scratch(&cnt));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int nb = ntheta * nphi;
    // the counts are cleared by a kernel (the previous call's counts are still there)
    hipLaunchKernelGGL(k_zero_counts, dim3(nblk(nb)), dim3(256), 0, s, cnt, nb);
    hipLaunchKernelGGL(k_density_count, dim3(nblk(npts)), dim3(256), 0, s, theta, phi, npts,
                       ntheta, nphi, cnt);
    hipLaunchKernelGGL(k_density_norm, dim3(nblk((int64_t)nb)), dim3(256), 0, s, cnt, ntheta,
                       nphi, npts, density);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int nusht_point_features(const double* theta, const double* phi, int64_t npts,
                         const float* density, int ntheta, int nphi, float* features,
                         void* stream)
{
    if (!theta || !phi || !density || !features || npts < 1 || ntheta < 1 || nphi < 1) {
        set_last_error("nusht_point_features", "bad arguments");
        return NUSHT_EINVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_features, dim3(nblk(npts)), dim3(256), 0, s, theta, phi, npts, density,
                       ntheta, nphi, features);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int nusht_mlp_forward(const float* params, const float* features, int64_t npts, float scale,
                      float* weights, void* stream)
{
    if (!params || !features || !weights || npts < 1) return NUSHT_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t tiles = (npts + kTileP - 1) / kTileP;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)tiles), dim3(256), 0, s, params, features,
                       npts, scale, weights);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int nusht_mlp_backward(const float* params, const float* features, const float* grad_weights,
                       int64_t npts, float scale, float* grad_params, void* stream)
{
    if (!params || !features || !grad_weights || !grad_params || npts < 1) return NUSHT_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t tiles = (npts + kTileP - 1) / kTileP;
    const int blocks = (int)(tiles < 512 ? tiles : 512);
    float* partial = nullptr;
    NUSHT_HIP(hipMallocAsync((void**)&partial, (size_t)blocks * kParams * sizeof(float), s));
    hipLaunchKernelGGL(k_mlp_backward, dim3(blocks), dim3(256), 0, s, params, features,
                       grad_weights, npts, scale, partial);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 255) / 256), dim3(256), 0, s, partial, blocks,
                       grad_params);
    NUSHT_HIP(hipGetLastError());
    NUSHT_HIP(hipFreeAsync(partial, s));
    return NUSHT_OK;
}

int nusht_adam_step(float* params, const float* grad, float* m, float* v, int64_t n, float lr,
                    float beta1, float beta2, float eps, int step, void* stream)
{
    if (!params || !grad || !m || !v || n < 1 || step < 1) return NUSHT_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, s, params, grad, m, v, n, lr, beta1,
                       beta2, eps, c1, c2);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int nusht_weighted_adjoint(nusht_plan_t p, const double* d, const float* weights, double* alm,
                           void* stream)
{
    if (!p || !d || !weights || !alm) {
        set_last_error("nusht_weighted_adjoint", "null argument");
        return NUSHT_EINVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = p->g.npts;
    double* wd = nullptr;
    NUSHT_HIP(hipMallocAsync((void**)&wd, n * sizeof(double), s));
    hipLaunchKernelGGL(k_weighted_map, dim3(nblk(n)), dim3(256), 0, s, weights, d, wd, n);
    const int rc = nusht_adjoint(p, wd, alm, 1, stream);
    hipFreeAsync(wd, s);
    NUSHT_HIP(hipGetLastError());
    return rc;
}

int nusht_weight_loss_grad(nusht_plan_t p, const double* d, const double* astar,
                           const float* weights, float* grad_weights, double* loss, void* stream)
{
    if (!p || !d || !astar || !weights || !loss) return NUSHT_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = p->g.npts, na = p->g.nalm;
    double *wd = nullptr, *q = nullptr, *part = nullptr, *sc = nullptr;
    double2* c = nullptr;
    NUSHT_HIP(hipMallocAsync((void**)&wd, n * sizeof(double), s));
    NUSHT_HIP(hipMallocAsync((void**)&q, n * sizeof(double), s));
    NUSHT_HIP(hipMallocAsync((void**)&c, na * sizeof(double2), s));
    NUSHT_HIP(hipMallocAsync((void**)&part, (kRB + 4) * sizeof(double), s));
    sc = part + kRB;
    int rc = NUSHT_OK;
    do {
        hipLaunchKernelGGL(k_weighted_map, dim3(nblk(n)), dim3(256), 0, s, weights, d, wd, n);
        if ((rc = nusht_adjoint(p, wd, reinterpret_cast<double*>(c), 1, stream))) break;
        hipLaunchKernelGGL(k_sub_alm, dim3(nblk(na)), dim3(256), 0, s, c,
                           reinterpret_cast<const double2*>(astar), na);
        hipLaunchKernelGGL(k_mdot, dim3(kRB), dim3(kRT), 0, s, c, na, p->g.lmax, part);
        hipLaunchKernelGGL(k_sum, dim3(1), dim3(kRT), 0, s, part, kRB, sc);
        hipLaunchKernelGGL(k_mdot, dim3(kRB), dim3(kRT), 0, s,
                           reinterpret_cast<const double2*>(astar), na, p->g.lmax, part);
        hipLaunchKernelGGL(k_sum, dim3(1), dim3(kRT), 0, s, part, kRB, sc + 1);
        if (grad_weights) {
            if ((rc = nusht_synthesis(p, reinterpret_cast<const double*>(c), q, 1, stream))) break;
            hipLaunchKernelGGL(k_weight_grad, dim3(nblk(n)), dim3(256), 0, s, d, q, sc + 1,
                               grad_weights, n);
        }
        double h[2];
        if (hipMemcpyAsync(h, sc, 2 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = NUSHT_EDEVICE;
            break;
        }
        *loss = h[1] > 0.0 ? h[0] / h[1] : 0.0;
    } while (0);
    hipFreeAsync(wd, s);
    hipFreeAsync(q, s);
    hipFreeAsync(c, s);
    hipFreeAsync(part, s);
    NUSHT_HIP(hipGetLastError());
    return rc;
}

}  // extern "C"
