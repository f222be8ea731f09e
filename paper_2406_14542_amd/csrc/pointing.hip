// Lensing pointing (arXiv:2406.14542, App. C): the deflected directions at which a lensed
// field is evaluated.
//
//   Eq. (C2): alpha_theta + i alpha_phi = (d/dtheta + (i / sin theta) d/dphi) Phi
//   Eq. (C1): n' = cos(alpha) n + (sin(alpha) / alpha) (alpha_theta e_theta + alpha_phi e_phi),
//             alpha = |(alpha_theta, alpha_phi)|
//
// with n = (sin t cos p, sin t sin p, cos t), e_theta = (cos t cos p, cos t sin p, -sin t) and
// e_phi = (-sin p, cos p, 0).  The gradient of Phi comes from the derivative synthesis
// (nusht_synthesis_deriv: the same fine grid interpolated with derivative taps); one thread
// per point then forms alpha_phi and moves the point along its great circle in FP64
// (theta' = atan2(|n'_xy|, n'_z), phi' = atan2(n'_y, n'_x) in [0, 2 pi)).  At an exact pole
// (sin theta = 0) alpha_phi is taken as 0.
#include "internal.h"

namespace nusht {
namespace {

__device__ inline void deflect_one(double th, double ph, double ath, double aph, double& th2,
                                   double& ph2)
{
    double st, ct, sp, cp;
    sincos(th, &st, &ct);
    sincos(ph, &sp, &cp);
    const double a = sqrt(ath * ath + aph * aph);
    double sa, ca;
    sincos(a, &sa, &ca);
    const double sinc = a > 0.0 ? sa / a : 1.0;
    const double nx = ca * st * cp + sinc * (ath * ct * cp - aph * sp);
    const double ny = ca * st * sp + sinc * (ath * ct * sp + aph * cp);
    const double nz = ca * ct - sinc * ath * st;
    th2 = atan2(sqrt(nx * nx + ny * ny), nz);
    double p = atan2(ny, nx);
    if (p < 0.0) p += 2.0 * M_PI;
    ph2 = p;
}

// Eq. (C1) for given deflection components, caller's arrays
__global__ void k_deflect(const double* __restrict__ th, const double* __restrict__ ph,
                          const double* __restrict__ ath, const double* __restrict__ aph,
                          int64_t n, double* __restrict__ th2, double* __restrict__ ph2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double t, p;
    deflect_one(th[i], ph[i], ath[i], aph[i], t, p);
    th2[i] = t;
    ph2[i] = p;
}

// Eq. (C2) then Eq. (C1) for the plan's points in the caller's order: the point's angles come
// from the plan's sorted copies through the inverse permutation; dth / dph (dPhi/dtheta,
// dPhi/dphi) may be the output arrays themselves (each thread reads its own entry first).
__global__ void k_pointing(const double* __restrict__ sth, const double* __restrict__ sph,
                           const int* __restrict__ iperm, const double* dth, const double* dph,
                           int64_t n, double* th2, double* ph2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = iperm[i];
    const double th = sth[k], ph = sph[k];
    const double s = sin(th);
    const double ath = dth[i];
    const double aph = s != 0.0 ? dph[i] / s : 0.0;
    double t, p;
    deflect_one(th, ph, ath, aph, t, p);
    th2[i] = t;
    ph2[i] = p;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace
}  // namespace nusht

using namespace nusht;

extern "C" {

int nusht_deflect(const double* theta, const double* phi, const double* alpha_theta,
                  const double* alpha_phi, int64_t npts, double* theta_out, double* phi_out,
                  void* stream)
{
    if (!theta || !phi || !alpha_theta || !alpha_phi || !theta_out || !phi_out || npts < 1) {
        set_last_error("nusht_deflect", "null buffer or npts < 1");
        return NUSHT_EINVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_deflect, dim3(blocks_for(npts)), dim3(256), 0, s, theta, phi,
                       alpha_theta, alpha_phi, npts, theta_out, phi_out);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

int nusht_pointing(nusht_plan_t p, const double* dlm, double* theta_out, double* phi_out,
                   void* stream)
{
    if (!p || !dlm || !theta_out || !phi_out) {
        set_last_error("nusht_pointing", "null plan or buffer");
        return NUSHT_EINVAL;
    }
    if (p->g.dtype != NUSHT_F64) {
        set_last_error("nusht_pointing", "needs an FP64 plan");
        return NUSHT_EPRECISION;
    }
    NUSHT_TRY(ensure_capacity(p, 1));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // Phi at the points goes to the plan's point scratch (unused by a one-map derivative
    // synthesis); its two derivatives straight into the output arrays
    NUSHT_TRY(nusht_synthesis_deriv(p, dlm, p->V, theta_out, phi_out, 1, stream));
    hipLaunchKernelGGL(k_pointing, dim3(blocks_for(p->g.npts)), dim3(256), 0, s, p->sth, p->sph,
                       p->iperm, theta_out, phi_out, p->g.npts, theta_out, phi_out);
    NUSHT_HIP(hipGetLastError());
    return NUSHT_OK;
}

}  // extern "C"
