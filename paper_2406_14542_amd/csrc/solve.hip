// placeholder, replaced below
#include "internal.h"
extern "C" int nusht_solve(nusht_plan_t, const double*, double*, const float*, double, int, int*,
                           double*, void*)
{
    return NUSHT_EINVAL;
}
