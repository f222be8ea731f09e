// FP32 instantiations of the nuFFT point kernels (mixed precision: FP64 coordinates and
// offsets, FP32 grid values, kernel taps and accumulation).
#include "nufft_impl.h"

namespace nusht {

int interp_f32(const nusht_plan_s* p, const float* fine, double* out, int nmaps, hipStream_t s)
{
    return dispatch_interp_impl<float>(p, fine, out, nmaps, (float)p->g.beta, s);
}

int spread_group_f32(const nusht_plan_s* p, const double* vals, float* fine, int mb,
                     hipStream_t s)
{
    return spread_group_impl<float>(p, vals, fine, mb, (float)p->g.beta, s);
}

}  // namespace nusht
