// FP64 instantiations of the nuFFT point kernels (interpolation, spreading,
// and the derivative interpolation used for gradients with respect to point positions).
#include "nufft_impl.h"

namespace nusht {

int interp_f64(const nusht_plan_s* p, const double* fine, double* out, int nmaps, hipStream_t s)
{
    return dispatch_interp_impl<double>(p, fine, out, nmaps, p->g.beta, s);
}

int spread_group_f64(const nusht_plan_s* p, const double* vals, double* fine, int mb,
                     hipStream_t s)
{
    return spread_group_impl<double>(p, vals, fine, mb, p->g.beta, s);
}

int launch_interp_deriv(const nusht_plan_s* p, const double* fine, double* out, double* dth,
                        double* dph, int nmaps, hipStream_t s)
{
    if (p->nslots == 0) return NUSHT_OK;
    const PointBins pb = make_bins(p);
    const int64_t ms = (int64_t)p->g.n1 * p->g.n2;
    const int64_t npts = p->g.npts;
    int b = 0;
    while (b < nmaps) {
        const int mb = group_width(nmaps, b);
        NUSHT_WIDTH_SWITCH(p->g.width, {
            if (mb == 4)
                hipLaunchKernelGGL((k_interp_deriv<WV, 4>), dim3(p->nslots), dim3(256), 0, s,
                                   fine + b * ms, ms, pb, p->g.beta, out + b * npts,
                                   dth + b * npts, dph + b * npts, npts);
            else
                hipLaunchKernelGGL((k_interp_deriv<WV, 1>), dim3(p->nslots), dim3(256), 0, s,
                                   fine + b * ms, ms, pb, p->g.beta, out + b * npts,
                                   dth + b * npts, dph + b * npts, npts);
        });
        NUSHT_HIP(hipGetLastError());
        b += mb;
    }
    return NUSHT_OK;
}

}  // namespace nusht
