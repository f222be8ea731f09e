// Vector-Jacobian products of the synthesis (gradients for autograd).
//   map[b][i] = sum_lm a_lm Y_lm(theta_i, phi_i) with a real field (Eq. 3, m >= 0 stored).
// For a loss L(map) with g = dL/dmap:
//   dL/dRe a_l0 = c_l0,  dL/d(Re, Im) a_lm = 2 (Re, Im) c_lm  (m > 0),  c = Y^H g  (Eq. 2);
//   the complex gradient in the torch convention is dL/dRe a + i dL/dIm a.
//   dL/dtheta_i = sum_b g[b][i] dmap[b][i]/dtheta_i, and likewise for phi.
#include "internal.h"

namespace nusht {
namespace {

__global__ void k_grad_alm_convention(double2* __restrict__ alm, int64_t nalm, int lmax,
                                      int nmaps)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nalm) return;
    for (int b = 0; b < nmaps; ++b) {
        double2 v = alm[(int64_t)b * nalm + idx];
        if (idx <= lmax) {  // m = 0 block of the m-major triangle
            v.y = 0.0;
        } else {
            v.x *= 2.0;
            v.y *= 2.0;
        }
        alm[(int64_t)b * nalm + idx] = v;
    }
}

__global__ void k_point_vjp(const double* __restrict__ g, const double* __restrict__ dth,
                            const double* __restrict__ dph, double* __restrict__ gth,
                            double* __restrict__ gph, int nmaps, int64_t npts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    double st = 0.0, sp = 0.0;
    for (int b = 0; b < nmaps; ++b) {
        const double gi = g[(int64_t)b * npts + i];
        st = fma(gi, dth[(int64_t)b * npts + i], st);
        sp = fma(gi, dph[(int64_t)b * npts + i], sp);
    }
    if (gth) gth[i] = st;
    if (gph) gph[i] = sp;
}

}  // namespace
}  // namespace nusht

using namespace nusht;

extern "C" {

int nusht_vjp_alm(nusht_plan_t p, const double* grad_map, double* grad_alm, int nmaps,
                  void* stream)
{
    NUSHT_TRY(nusht_adjoint(p, grad_map, grad_alm, nmaps, stream));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t nalm = p->g.nalm;
    hipLaunchKernelGGL(k_grad_alm_convention, dim3((unsigned)((nalm + 255) / 256)), dim3(256), 0,
                       s, reinterpret_cast<double2*>(grad_alm), nalm, p->g.lmax, nmaps);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int nusht_vjp_alm_spin(nusht_plan_t p, int spin, const double* grad_map, double* grad_alm,
                       int nfields, void* stream)
{
    NUSHT_TRY(nusht_adjoint_spin(p, spin, grad_map, grad_alm, nfields, stream));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t nalm = p->g.nalm;
    // G and C of every field are coefficient rows of the same triangle layout
    hipLaunchKernelGGL(k_grad_alm_convention, dim3((unsigned)((nalm + 255) / 256)), dim3(256), 0,
                       s, reinterpret_cast<double2*>(grad_alm), nalm, p->g.lmax, 2 * nfields);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int nusht_vjp_points(const double* grad_map, const double* dtheta, const double* dphi,
                     double* grad_theta, double* grad_phi, int nmaps, int64_t npts, void* stream)
{
    if (!grad_map || !dtheta || !dphi || (!grad_theta && !grad_phi) || nmaps < 1 || npts < 1) {
        set_last_error("nusht_vjp_points", "null buffer or empty shape");
        return NUSHT_EINVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_point_vjp, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, s,
                       grad_map, dtheta, dphi, grad_theta, grad_phi, nmaps, npts);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

}  // extern "C"
