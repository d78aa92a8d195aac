// Device helpers shared by the stencil and transpose kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace nrd {

// Reciprocal and reciprocal square root: the hardware estimate (about 23
// correct bits) refined by two Newton-Raphson steps (quadratic convergence,
// so the result is within about one ulp); valid for the positive, normal
// operands met here.
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double r = __builtin_fma(-(x * y), y, 1.0);     // y <- y (3 - x y^2) / 2
    y = __builtin_fma(0.5 * y, r, y);
    r = __builtin_fma(-(x * y), y, 1.0);
    return __builtin_fma(0.5 * y, r, y);
}

// Interior cell (i, j, k) of the linear (x fastest) interior index lin of
// patch p, and the native (ghosted) index of an interior cell.
__device__ __forceinline__ void cell_coords(const PatchInfo& p, int lin, int& i, int& j,
                                            int& k) {
    i = lin % p.n[0];
    const int r = lin / p.n[0];
    j = r % p.n[1];
    k = r / p.n[1];
}

__device__ __forceinline__ int native_index(const PatchInfo& p, int i, int j, int k) {
    return p.off + (i + 1) + p.sy * (j + 1) + p.sz * (k + 1);
}

}  // namespace nrd
