// nb_math.h -- the scalar pieces of the FP64 pairwise interaction that every FP64
// evaluation kernel shares (the symmetric kernel includes only this): the position of
// the zero-mass records that pad a tile, and 1/sqrt to about one ulp.
#pragma once

#include <hip/hip_runtime.h>

namespace nb {

constexpr double kFar = 1.0e18;  // position of the zero-mass records that pad a tile

// 1/sqrt(x) to about one ulp: the hardware estimate v_rsq_f64 (relative error
// below 2^-24 measured on gfx950) followed by one third-order correction
// y (1 + e/2 + 3 e^2 / 8) with e = 1 - x y^2, whose truncation error (5/16) e^3 is
// far below the FP64 rounding. (An FP32 estimate is as accurate and measured no
// faster once the conversions are counted.)
__device__ __forceinline__ double rsqrt_f64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = __builtin_fma(-x, y * y, 1.0);
    const double p = __builtin_fma(e, 0.375, 0.5);
    return __builtin_fma(y, e * p, y);
}

}  // namespace nb
