// Least-squares inverse of the synthesis by CGLS (the setting in which the transforms are
// called over and over, arXiv:2406.14542 Sec. I): minimise || W^(1/2) (S a - d) ||_2 over
// coefficients a, in the <.,.>_m geometry under which the adjoint of Eq. 2 is S^H.
//
//   u = d - S x;  s = S^H W u;  p = s;  gamma = <s, s>_m
//   repeat:  q = S p;  alpha = gamma / sum(W q^2);  x += alpha p;  u -= alpha q;
//            s = S^H W u;  gamma' = <s, s>_m;  p = s + (gamma'/gamma) p;  gamma = gamma'
//   until ||u|| / ||d|| <= tol   (u is the unweighted residual d - S x, kept by recurrence)
//
// All vectors stay on the device; alpha and beta are formed on the device; every reduction
// is a fixed-shape two-pass sum that adds in a fixed order (the adjoint transform itself adds
// with atomics in no fixed order, so two solves can differ by rounding).  The host reads one 8-byte
// residual per iteration for the stopping test.  When the recurred residual reaches tol, the
// true residual d - S x is formed again; if it is still above tol (the recurrence drifts, more
// so in mixed precision or with weights), CGLS restarts from x with that true residual, at
// most kMaxRestarts times.
//
// The spin-s solve runs the same iteration with S the spin-s synthesis of one field (its
// G, C coefficients to its Q, U maps) and S^H that synthesis's adjoint, which is its
// transpose in the same <.,.>_m product summed over the two coefficient triangles; the
// per-point weight applies to Q and U alike.
#include <cmath>

#include "internal.h"

namespace nusht {
namespace {

constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;
constexpr int kMaxRestarts = 4;

enum { SC_GAMMA = 0, SC_DELTA, SC_RR, SC_DN2, SC_GNEW, SC_ALPHA, SC_BETA, SC_COUNT };

__device__ inline double block_sum(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    return sh[0];
}

// A map-space vector holds one map (spin 0) or the two maps Q, U (spin s) of npts values
// each, and a coefficient vector one or two (G, C) triangles of nalm; the weights and the
// m = 0 test repeat per component.  wrap(i, n) maps an index of either component to its
// position within the component.
__device__ inline int64_t wrap(int64_t i, int64_t n) { return i < n ? i : i - n; }

// partial[blk] = sum over the block's grid-stride range of w_i a_i b_i (w = 1 if null)
__global__ __launch_bounds__(kRedThreads) void k_dot_map(const double* __restrict__ a,
                                                         const double* __restrict__ b,
                                                         const float* __restrict__ w,
                                                         int64_t n, int64_t npts,
                                                         double* __restrict__ partial)
{
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = a[i] * b[i];
        acc += w ? (double)w[wrap(i, npts)] * v : v;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// partial[blk] = sum of the <a, b>_m terms in the block's range (m = 0 block: idx <= lmax)
__global__ __launch_bounds__(kRedThreads) void k_dot_alm(const double2* __restrict__ a,
                                                         const double2* __restrict__ b,
                                                         int64_t n, int64_t nalm, int lmax,
                                                         double* __restrict__ partial)
{
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 x = a[i], y = b[i];
        const double v = x.x * y.x + x.y * y.y;
        acc += (wrap(i, nalm) <= lmax) ? v : 2.0 * v;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedThreads) void k_finish(const double* __restrict__ partial,
                                                        int n, double* __restrict__ out)
{
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partial[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) *out = s;
}

__global__ void k_alpha(double* sc)
{
    const double d = sc[SC_DELTA];
    sc[SC_ALPHA] = d > 0.0 ? sc[SC_GAMMA] / d : 0.0;
}

__global__ void k_beta(double* sc)
{
    const double g = sc[SC_GAMMA];
    sc[SC_BETA] = g > 0.0 ? sc[SC_GNEW] / g : 0.0;
    sc[SC_GAMMA] = sc[SC_GNEW];
}

// x += alpha p (complex, alm space)
__global__ void k_axpy_alm(double2* __restrict__ x, const double2* __restrict__ p,
                           const double* __restrict__ sc, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = sc[SC_ALPHA];
    double2 v = x[i];
    const double2 q = p[i];
    v.x = fma(a, q.x, v.x);
    v.y = fma(a, q.y, v.y);
    x[i] = v;
}

// u -= alpha q; wu = w u (w = 1 if null)
__global__ void k_update_u(double* __restrict__ u, const double* __restrict__ q,
                           const float* __restrict__ w, double* __restrict__ wu,
                           const double* __restrict__ sc, int64_t n, int64_t npts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = fma(-sc[SC_ALPHA], q[i], u[i]);
    u[i] = v;
    wu[i] = w ? (double)w[wrap(i, npts)] * v : v;
}

// u = d - q; wu = w u
__global__ void k_residual(const double* __restrict__ d, const double* __restrict__ q,
                           const float* __restrict__ w, double* __restrict__ u,
                           double* __restrict__ wu, int64_t n, int64_t npts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = d[i] - q[i];
    u[i] = v;
    if (wu) wu[i] = w ? (double)w[wrap(i, npts)] * v : v;
}

// p = s + beta p
__global__ void k_update_p(double2* __restrict__ p, const double2* __restrict__ s,
                           const double* __restrict__ sc, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double b = sc[SC_BETA];
    const double2 v = s[i];
    double2 o = p[i];
    o.x = fma(b, o.x, v.x);
    o.y = fma(b, o.y, v.y);
    p[i] = o;
}

struct SolveBufs {
    double2* s = nullptr;
    double2* p = nullptr;
    double* u = nullptr;
    double* q = nullptr;
    double* wu = nullptr;
    double* partial = nullptr;
    double* sc = nullptr;
};

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace
}  // namespace nusht

using namespace nusht;

namespace {

// The CGLS loop for spin 0 (one map, one coefficient triangle) or spin s >= 1 (the Q, U
// maps of one field and its G, C triangles): the same iteration on vectors of nc = 1 or 2
// components, with S and S^H the transforms of that spin.
int solve_impl(nusht_plan_t p, int spin, const char* who, const double* map, double* alm,
               const float* weights, double tol, int maxiter, int* iters, double* relres,
               double* history, void* stream)
{
    if (!p || !map || !alm || !(tol > 0.0) || maxiter < 0) {
        set_last_error(who, "null plan/buffer, tol <= 0 or maxiter < 0");
        return NUSHT_EINVAL;
    }
    if (spin != 0) NUSHT_TRY(check_spin(p, spin, who));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int nc = spin != 0 ? 2 : 1;
    const int64_t npts = p->g.npts, nalm = p->g.nalm;
    const int64_t n = nc * npts, na = nc * nalm;
    const int lmax = p->g.lmax;
    auto synth = [&](const double* a, double* f) -> int {
        return spin != 0 ? nusht_synthesis_spin(p, spin, a, f, 1, stream)
                         : nusht_synthesis(p, a, f, 1, stream);
    };
    auto adjoint = [&](const double* f, double* a) -> int {
        return spin != 0 ? nusht_adjoint_spin(p, spin, f, a, 1, stream)
                         : nusht_adjoint(p, f, a, 1, stream);
    };
    // solve scratch lives in the plan and is reused by later solves
    const size_t need = (size_t)na * 2 * sizeof(double2) + (size_t)n * 3 * sizeof(double) +
                        (kRedBlocks + SC_COUNT + 8) * sizeof(double);
    if (p->redbytes < need) {
        if (p->red) {
            NUSHT_HIP(hipStreamSynchronize(s));
            hipFree(p->red);
        }
        p->red = nullptr;
        p->redbytes = 0;
        NUSHT_HIP(hipMalloc((void**)&p->red, need));
        p->redbytes = need;
    }
    SolveBufs b;
    char* base = reinterpret_cast<char*>(p->red);
    b.s = reinterpret_cast<double2*>(base);
    b.p = b.s + na;
    b.u = reinterpret_cast<double*>(b.p + na);
    b.q = b.u + n;
    b.wu = b.q + n;
    b.partial = b.wu + n;
    b.sc = b.partial + kRedBlocks;
    double2* x = reinterpret_cast<double2*>(alm);

    auto dot_map = [&](const double* a, const double* c, const float* w, int slot) -> int {
        hipLaunchKernelGGL(k_dot_map, dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, c, w, n, npts,
                           b.partial);
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedThreads), 0, s, b.partial, kRedBlocks,
                           b.sc + slot);
        NUSHT_HIP(hipGetLastError());
        return NUSHT_OK;
    };
    auto dot_alm = [&](const double2* a, const double2* c, int slot) -> int {
        hipLaunchKernelGGL(k_dot_alm, dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, c, na, nalm,
                           lmax, b.partial);
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedThreads), 0, s, b.partial, kRedBlocks,
                           b.sc + slot);
        NUSHT_HIP(hipGetLastError());
        return NUSHT_OK;
    };
    auto read_scalar = [&](int slot, double* out) -> int {
        NUSHT_HIP(hipMemcpyAsync(out, b.sc + slot, sizeof(double), hipMemcpyDeviceToHost, s));
        NUSHT_HIP(hipStreamSynchronize(s));
        return NUSHT_OK;
    };

    // ||d||^2 once
    NUSHT_TRY(dot_map(map, map, nullptr, SC_DN2));
    double dn2 = 0.0, rr = 0.0;
    NUSHT_TRY(read_scalar(SC_DN2, &dn2));
    if (dn2 == 0.0) dn2 = 1.0;  // d = 0: report the absolute residual
    const double tol2 = tol * tol;
    int it = 0;
    for (int restart = 0;; ++restart) {
        // u = d - S x (the true residual), then s = S^H W u, p = s, gamma = <s, s>_m
        NUSHT_TRY(synth(alm, b.q));
        hipLaunchKernelGGL(k_residual, dim3(blocks_for(n)), dim3(256), 0, s, map, b.q, weights,
                           b.u, b.wu, n, npts);
        NUSHT_TRY(dot_map(b.u, b.u, nullptr, SC_RR));
        NUSHT_TRY(read_scalar(SC_RR, &rr));
        if (history && restart == 0) history[0] = std::sqrt(rr / dn2);
        if (rr <= tol2 * dn2 || it >= maxiter || restart > kMaxRestarts) break;
        NUSHT_TRY(adjoint(b.wu, reinterpret_cast<double*>(b.s)));
        NUSHT_HIP(hipMemcpyAsync(b.p, b.s, (size_t)na * sizeof(double2), hipMemcpyDeviceToDevice,
                                 s));
        NUSHT_TRY(dot_alm(b.s, b.s, SC_GAMMA));
        while (rr > tol2 * dn2 && it < maxiter) {
            NUSHT_TRY(synth(reinterpret_cast<const double*>(b.p), b.q));
            NUSHT_TRY(dot_map(b.q, b.q, weights, SC_DELTA));
            hipLaunchKernelGGL(k_alpha, dim3(1), dim3(1), 0, s, b.sc);
            hipLaunchKernelGGL(k_axpy_alm, dim3(blocks_for(na)), dim3(256), 0, s, x, b.p, b.sc,
                               na);
            hipLaunchKernelGGL(k_update_u, dim3(blocks_for(n)), dim3(256), 0, s, b.u, b.q,
                               weights, b.wu, b.sc, n, npts);
            NUSHT_TRY(adjoint(b.wu, reinterpret_cast<double*>(b.s)));
            NUSHT_TRY(dot_alm(b.s, b.s, SC_GNEW));
            hipLaunchKernelGGL(k_beta, dim3(1), dim3(1), 0, s, b.sc);
            hipLaunchKernelGGL(k_update_p, dim3(blocks_for(na)), dim3(256), 0, s, b.p, b.s, b.sc,
                               na);
            NUSHT_TRY(dot_map(b.u, b.u, nullptr, SC_RR));
            NUSHT_HIP(hipGetLastError());
            NUSHT_TRY(read_scalar(SC_RR, &rr));
            ++it;
            if (history) history[it] = std::sqrt(rr / dn2);
        }
    }
    // rr is the true residual of the final iterate
    if (iters) *iters = it;
    if (relres) *relres = std::sqrt(rr / dn2);
    NUSHT_TRY(check_device_status(p));
    return rr <= tol2 * dn2 ? NUSHT_OK : NUSHT_ENOCONV;
}

}  // namespace

extern "C" {

int nusht_solve(nusht_plan_t p, const double* map, double* alm, const float* weights, double tol,
                int maxiter, int* iters, double* relres, void* stream)
{
    return solve_impl(p, 0, "nusht_solve", map, alm, weights, tol, maxiter, iters, relres,
                      nullptr, stream);
}

int nusht_solve_ex(nusht_plan_t p, const double* map, double* alm, const float* weights,
                   double tol, int maxiter, int* iters, double* relres, double* history,
                   void* stream)
{
    return solve_impl(p, 0, "nusht_solve", map, alm, weights, tol, maxiter, iters, relres,
                      history, stream);
}

int nusht_solve_spin(nusht_plan_t p, int spin, const double* map, double* alm,
                     const float* weights, double tol, int maxiter, int* iters, double* relres,
                     double* history, void* stream)
{
    return solve_impl(p, spin, "nusht_solve_spin", map, alm, weights, tol, maxiter, iters,
                      relres, history, stream);
}

}  // extern "C"
