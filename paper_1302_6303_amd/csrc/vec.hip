// Krylov vector kernels: per-problem inner products (two-stage, fixed
// order, hence bitwise reproducible), vector combinations, positivity
// reductions and the small per-problem FGMRES kernels (Sec. 4.1).
//
// Vectors are native 2-field arrays; only interior cells are read or
// written.  Inner products are volume weighted over composite cells.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "kernels.h"

namespace nrd {

static inline int nblocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum over the workgroup (4 waves), same result on every thread.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}
__device__ __forceinline__ double block_min(double v, double* sh) {
    v = wave_min(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    const double r = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
    __syncthreads();
    return r;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double block_max(double v, double* sh) {
    v = wave_max(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    const double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
    return r;
}

__device__ __forceinline__ int interior_index(const PatchInfo& p, int lin) {
    const int i = lin % p.n[0];
    const int r = lin / p.n[0];
    const int j = r % p.n[1];
    const int k = r / p.n[1];
    return p.off + (i + 1) + p.sy * (j + 1) + p.sz * (k + 1);
}

template <int NV>
__global__ __launch_bounds__(kBlock) void k_multidot(
    const Tile* __restrict__ vt, const PatchInfo* __restrict__ P,
    const uint8_t* __restrict__ ctype, const int32_t* __restrict__ active,
    const double* __restrict__ X, int64_t xs, int nv, const double* __restrict__ xsc,
    const double* __restrict__ y, double* __restrict__ partial, int64_t nl) {
    __shared__ double sh[4];
    const Tile t = vt[blockIdx.x];
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    const bool on = !active || active[t.prob];
    const PatchInfo& p = P[t.patch];
    if (on) {
        const bool cov = p.flags & PF_COVERED;
        const double sc = xsc ? xsc[t.prob] : 1.0;
        for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
            const int c = interior_index(p, lin);
            if (cov && (ctype[c] & CT_COVERED)) continue;
            const double y0 = y[c], y1 = y[c + nl];
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nv) {
                    const double x0 = sc * X[v * xs + c], x1 = sc * X[v * xs + c + nl];
                    acc[v] += x0 * y0 + x1 * y1;
                }
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v < nv) {
            const double s = block_sum(acc[v], sh);
            if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * nv + v] = s * p.vol;
        }
    }
}

// out[p * ostride + v] = sum of the problem's tile partials (fixed order)
__global__ __launch_bounds__(kBlock) void k_sum_partials(
    const int32_t* __restrict__ t0, const double* __restrict__ partial, int nv,
    double* __restrict__ out, int ostride) {
    __shared__ double sh[4];
    const int p = blockIdx.x;
    const int a = t0[p], b = t0[p + 1];
    for (int v = 0; v < nv; ++v) {
        double acc = 0.0;
        for (int i = a + threadIdx.x; i < b; i += kBlock) acc += partial[(int64_t)i * nv + v];
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0) out[p * ostride + v] = s;
    }
}

void multidot(const Dev& D, hipStream_t s, const double* X, int64_t xstride, int nv,
              const double* y, double* partial, double* out, const double* xsc) {
    for (int v0 = 0; v0 < nv; v0 += 16) {
        const int c = std::min(16, nv - v0);
        const double* Xc = X + v0 * xstride;
        if (c == 1)
            k_multidot<1><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active,
                                                       Xc, xstride, c, xsc, y, partial, D.nl);
        else if (c <= 2)
            k_multidot<2><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active,
                                                       Xc, xstride, c, xsc, y, partial, D.nl);
        else if (c <= 4)
            k_multidot<4><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active,
                                                       Xc, xstride, c, xsc, y, partial, D.nl);
        else if (c <= 8)
            k_multidot<8><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active,
                                                       Xc, xstride, c, xsc, y, partial, D.nl);
        else
            k_multidot<16><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype,
                                                        D.active, Xc, xstride, c, xsc, y,
                                                        partial, D.nl);
        k_sum_partials<<<D.nprob, kBlock, 0, s>>>(D.prob_vtile0, partial, c, out + v0, nv);
    }
}

__global__ __launch_bounds__(kBlock) void k_min_pos(
    const Tile* __restrict__ vt, const PatchInfo* __restrict__ P,
    const uint8_t* __restrict__ ctype, const int32_t* __restrict__ active,
    const double* __restrict__ u, const double* __restrict__ du,
    const double* __restrict__ lam, double* __restrict__ partial, int64_t nl) {
    __shared__ double sh[4];
    const Tile t = vt[blockIdx.x];
    double m = DBL_MAX;
    if (!active || active[t.prob]) {
        const PatchInfo& p = P[t.patch];
        const double l = lam[t.prob];
        const bool cov = p.flags & PF_COVERED;
        for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
            const int c = interior_index(p, lin);
            if (cov && (ctype[c] & CT_COVERED)) continue;
            const double e = u[c] + l * du[c];
            const double tt = u[c + nl] + l * du[c + nl];
            // NaN compares false: map it to -1 so that it counts as a failure
            const double v = fmin(e, tt);
            m = fmin(m, (e == e && tt == tt) ? v : -1.0);
        }
    }
    const double r = block_min(m, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ __launch_bounds__(kBlock) void k_min_partials(const int32_t* __restrict__ t0,
                                                         const double* __restrict__ partial,
                                                         double* __restrict__ out) {
    __shared__ double sh[4];
    const int p = blockIdx.x;
    double m = DBL_MAX;
    for (int i = t0[p] + threadIdx.x; i < t0[p + 1]; i += kBlock) m = fmin(m, partial[i]);
    const double r = block_min(m, sh);
    if (threadIdx.x == 0) out[p] = r;
}

void min_positive(const Dev& D, hipStream_t s, const double* u, const double* du,
                  const double* lam, double* partial, double* out) {
    k_min_pos<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active, u, du,
                                           lam, partial, D.nl);
    k_min_partials<<<D.nprob, kBlock, 0, s>>>(D.prob_vtile0, partial, out);
}

template <int NV>
__global__ __launch_bounds__(kBlock) void k_combine(
    const Tile* __restrict__ vt, const PatchInfo* __restrict__ P,
    const int32_t* __restrict__ active, const double* __restrict__ X, int64_t xs, int nv,
    const double* __restrict__ coef, int cs, double* __restrict__ y, int accumulate,
    double alpha, int64_t nl) {
    const Tile t = vt[blockIdx.x];
    if (active && !active[t.prob]) return;
    const PatchInfo& p = P[t.patch];
    double cf[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) cf[v] = (v < nv) ? alpha * coef[t.prob * cs + v] : 0.0;
    for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
        const int c = interior_index(p, lin);
        double a0 = accumulate ? y[c] : 0.0;
        double a1 = accumulate ? y[c + nl] : 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v)
            if (v < nv && cf[v] != 0.0) {     // unused basis vectors may be stale
                a0 += cf[v] * X[v * xs + c];
                a1 += cf[v] * X[v * xs + c + nl];
            }
        y[c] = a0;
        y[c + nl] = a1;
    }
}

void combine(const Dev& D, hipStream_t s, const double* X, int64_t xstride, int nv,
             const double* coef, int cstride, double* y, int accumulate, double alpha) {
    for (int v0 = 0; v0 < nv || (v0 == 0 && nv == 0); v0 += 16) {
        const int c = std::min(16, nv - v0);
        const int acc = (v0 > 0) ? 1 : accumulate;
        const double* Xc = X + v0 * xstride;
        const double* cc = coef + v0;
        if (c <= 1)
            k_combine<1><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.active, Xc,
                                                      xstride, c, cc, cstride, y, acc, alpha,
                                                      D.nl);
        else if (c <= 4)
            k_combine<4><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.active, Xc,
                                                      xstride, c, cc, cstride, y, acc, alpha,
                                                      D.nl);
        else if (c <= 8)
            k_combine<8><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.active, Xc,
                                                      xstride, c, cc, cstride, y, acc, alpha,
                                                      D.nl);
        else
            k_combine<16><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.active, Xc,
                                                       xstride, c, cc, cstride, y, acc, alpha,
                                                       D.nl);
        if (nv == 0) break;
    }
}

// y -= sum_v coef[p][v] x_v (combine with alpha = -1, accumulating) and, in
// the same pass, out[p][v] = x_v . y of the new y (multidot), nv <= 16: the
// first Gram-Schmidt correction of FGMRES followed by the inner products of
// the second, with the expressions of those two kernels.
template <int NV>
__global__ __launch_bounds__(kBlock) void k_combine_dot(
    const Tile* __restrict__ vt, const PatchInfo* __restrict__ P,
    const uint8_t* __restrict__ ctype, const int32_t* __restrict__ active,
    const double* __restrict__ X, int64_t xs, int nv, const double* __restrict__ xsc,
    const double* __restrict__ coef, int cs, double* __restrict__ y,
    double* __restrict__ partial, int64_t nl) {
    __shared__ double sh[4];
    const Tile t = vt[blockIdx.x];
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    const bool on = !active || active[t.prob];
    const PatchInfo& p = P[t.patch];
    if (on) {
        double cf[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) cf[v] = (v < nv) ? -1.0 * coef[t.prob * cs + v] : 0.0;
        const bool cov = p.flags & PF_COVERED;
        const double sc = xsc ? xsc[t.prob] : 1.0;
        for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
            const int c = interior_index(p, lin);
            double a0 = y[c], a1 = y[c + nl];
            double x0[NV], x1[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                x0[v] = (v < nv) ? sc * X[v * xs + c] : 0.0;
                x1[v] = (v < nv) ? sc * X[v * xs + c + nl] : 0.0;
            }
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nv && cf[v] != 0.0) {
                    a0 += cf[v] * x0[v];
                    a1 += cf[v] * x1[v];
                }
            y[c] = a0;
            y[c + nl] = a1;
            if (cov && (ctype[c] & CT_COVERED)) continue;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nv) acc[v] += x0[v] * a0 + x1[v] * a1;
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v < nv) {
            const double sv = block_sum(acc[v], sh);
            if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * nv + v] = sv * p.vol;
        }
    }
}

void combine_dot(const Dev& D, hipStream_t s, const double* X, int64_t xstride, int nv,
                 const double* coef, int cstride, double* y, double* partial, double* out,
                 const double* xsc) {
    if (nv > 16) {            // (never with xsc: scaled bases have one vector)
        combine(D, s, X, xstride, nv, coef, cstride, y, 1, -1.0);
        multidot(D, s, X, xstride, nv, y, partial, out);
        return;
    }
    if (nv <= 1)
        k_combine_dot<1><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active, X,
                                                      xstride, nv, xsc, coef, cstride, y, partial,
                                                      D.nl);
    else if (nv <= 2)
        k_combine_dot<2><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active, X,
                                                      xstride, nv, xsc, coef, cstride, y, partial,
                                                      D.nl);
    else if (nv <= 4)
        k_combine_dot<4><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active, X,
                                                      xstride, nv, xsc, coef, cstride, y, partial,
                                                      D.nl);
    else if (nv <= 8)
        k_combine_dot<8><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active, X,
                                                      xstride, nv, xsc, coef, cstride, y, partial,
                                                      D.nl);
    else
        k_combine_dot<16><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active,
                                                       X, xstride, nv, xsc, coef, cstride, y, partial,
                                                       D.nl);
    k_sum_partials<<<D.nprob, kBlock, 0, s>>>(D.prob_vtile0, partial, nv, out, nv);
}

// y -= sum_v coef[p][v] x_v (accumulating into y) and, in the same pass,
// out[p] = ||y||^2 (volume weighted over composite cells; fixed-order
// two-stage sum).  The second Gram-Schmidt pass of FGMRES ends with the
// norm of the orthogonalised vector, so this saves one pass over it.
template <int NV>
__global__ __launch_bounds__(kBlock) void k_combine_norm(
    const Tile* __restrict__ vt, const PatchInfo* __restrict__ P,
    const uint8_t* __restrict__ ctype, const int32_t* __restrict__ active,
    const double* __restrict__ X, int64_t xs, int nv, const double* __restrict__ xsc,
    const double* __restrict__ coef, int cs, double* __restrict__ y,
    double* __restrict__ partial, int64_t nl) {
    __shared__ double sh[4];
    const Tile t = vt[blockIdx.x];
    double acc = 0.0;
    const bool on = !active || active[t.prob];
    const PatchInfo& p = P[t.patch];
    if (on) {
        double cf[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) cf[v] = (v < nv) ? -coef[t.prob * cs + v] : 0.0;
        const bool cov = p.flags & PF_COVERED;
        const double sc = xsc ? xsc[t.prob] : 1.0;
        for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
            const int c = interior_index(p, lin);
            double a0 = y[c], a1 = y[c + nl];
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nv && cf[v] != 0.0) {
                    a0 += cf[v] * (sc * X[v * xs + c]);
                    a1 += cf[v] * (sc * X[v * xs + c + nl]);
                }
            y[c] = a0;
            y[c + nl] = a1;
            if (!(cov && (ctype[c] & CT_COVERED))) acc += a0 * a0 + a1 * a1;
        }
    }
    const double sblk = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = sblk * p.vol;
}

void combine_norm(const Dev& D, hipStream_t s, const double* X, int64_t xstride, int nv,
                  const double* coef, int cstride, double* y, double* partial, double* out,
                  const double* xsc) {
    // more than 16 basis vectors: plain combines first, the norm with the last 16
    int v0 = 0;
    for (; nv - v0 > 16; v0 += 16)
        combine(D, s, X + v0 * xstride, xstride, 16, coef + v0, cstride, y, 1, -1.0);
    const int c = nv - v0;
    const double* Xc = X + v0 * xstride;
    const double* cc = coef + v0;
    if (c <= 1)
        k_combine_norm<1><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active,
                                                       Xc, xstride, c, xsc, cc, cstride, y, partial,
                                                       D.nl);
    else if (c <= 4)
        k_combine_norm<4><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active,
                                                       Xc, xstride, c, xsc, cc, cstride, y, partial,
                                                       D.nl);
    else if (c <= 8)
        k_combine_norm<8><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active,
                                                       Xc, xstride, c, xsc, cc, cstride, y, partial,
                                                       D.nl);
    else
        k_combine_norm<16><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active,
                                                        Xc, xstride, c, xsc, cc, cstride, y, partial,
                                                        D.nl);
    k_sum_partials<<<D.nprob, kBlock, 0, s>>>(D.prob_vtile0, partial, 1, out, 1);
}

// Newton update from the Krylov basis in one pass: for every active
// problem, keep = x, then x <- x - sum_v coef[p][v] z_v (the values of
// combine into s followed by axpby x <- -1 s + x), and partial = the
// minimum over the tile's composite cells of both fields of the new x (NaN
// counts as -1), as min_positive would report for the step -s.
template <int NV>
__global__ __launch_bounds__(kBlock) void k_update_min(
    const Tile* __restrict__ vt, const PatchInfo* __restrict__ P,
    const uint8_t* __restrict__ ctype, const int32_t* __restrict__ active,
    const double* __restrict__ Z, int64_t zs, int nv, const double* __restrict__ coef, int cs,
    double* __restrict__ x, double* __restrict__ keep, double* __restrict__ partial,
    int64_t nl) {
    __shared__ double sh[4];
    const Tile t = vt[blockIdx.x];
    double m = DBL_MAX;
    if (!active || active[t.prob]) {
        const PatchInfo& p = P[t.patch];
        double cf[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) cf[v] = (v < nv) ? coef[t.prob * cs + v] : 0.0;
        const bool cov = p.flags & PF_COVERED;
        for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
            const int c = interior_index(p, lin);
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nv && cf[v] != 0.0) {
                    s0 += cf[v] * Z[v * zs + c];
                    s1 += cf[v] * Z[v * zs + c + nl];
                }
            const double x0 = x[c], x1 = x[c + nl];
            keep[c] = x0;
            keep[c + nl] = x1;
            const double e = -1.0 * s0 + 1.0 * x0;
            const double tt = -1.0 * s1 + 1.0 * x1;
            x[c] = e;
            x[c + nl] = tt;
            if (cov && (ctype[c] & CT_COVERED)) continue;
            m = fmin(m, (e == e && tt == tt) ? fmin(e, tt) : -1.0);
        }
    }
    const double r = block_min(m, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

void update_min(const Dev& D, hipStream_t s, const double* Z, int64_t zstride, int nv,
                const double* coef, int cstride, double* x, double* keep, double* partial,
                double* out) {
    if (nv <= 1)
        k_update_min<1><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active, Z,
                                                     zstride, nv, coef, cstride, x, keep,
                                                     partial, D.nl);
    else if (nv <= 4)
        k_update_min<4><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active, Z,
                                                     zstride, nv, coef, cstride, x, keep,
                                                     partial, D.nl);
    else if (nv <= 8)
        k_update_min<8><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active, Z,
                                                     zstride, nv, coef, cstride, x, keep,
                                                     partial, D.nl);
    else
        k_update_min<16><<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active, Z,
                                                      zstride, nv, coef, cstride, x, keep,
                                                      partial, D.nl);
    k_min_partials<<<D.nprob, kBlock, 0, s>>>(D.prob_vtile0, partial, out);
}

// Scaled max norm of the BDF2 local error estimate (eq. bdf2le):
// partial = max over the tile's composite cells of |c_p (x - x^p)| / (x + eta)
// for both fields (eta_E, eta_T), a NaN counting as infinity.
__global__ __launch_bounds__(kBlock) void k_err_max(
    const Tile* __restrict__ vt, const PatchInfo* __restrict__ P,
    const uint8_t* __restrict__ ctype, const int32_t* __restrict__ active,
    const double* __restrict__ x, const double* __restrict__ xp,
    const double* __restrict__ coef, double eta_E, double eta_T,
    double* __restrict__ partial, int64_t nl) {
    __shared__ double sh[4];
    const Tile t = vt[blockIdx.x];
    double m = 0.0;
    if (!active || active[t.prob]) {
        const PatchInfo& p = P[t.patch];
        const double cf = coef[t.prob];
        const bool cov = p.flags & PF_COVERED;
        for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
            const int c = interior_index(p, lin);
            if (cov && (ctype[c] & CT_COVERED)) continue;
            const double vE = fabs(cf * (x[c] - xp[c])) / (x[c] + eta_E);
            const double vT = fabs(cf * (x[c + nl] - xp[c + nl])) / (x[c + nl] + eta_T);
            const double v = fmax(vE, vT);
            m = fmax(m, (vE == vE && vT == vT) ? v : HUGE_VAL);
        }
    }
    const double r = block_max(m, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ __launch_bounds__(kBlock) void k_max_partials(const int32_t* __restrict__ t0,
                                                         const double* __restrict__ partial,
                                                         double* __restrict__ out) {
    __shared__ double sh[4];
    const int p = blockIdx.x;
    double m = 0.0;
    for (int i = t0[p] + threadIdx.x; i < t0[p + 1]; i += kBlock) m = fmax(m, partial[i]);
    const double r = block_max(m, sh);
    if (threadIdx.x == 0) out[p] = r;
}

void err_norm(const Dev& D, hipStream_t s, const double* x, const double* xp,
              const double* coef, double eta_E, double eta_T, double* partial, double* out) {
    k_err_max<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, D.active, x, xp, coef,
                                           eta_E, eta_T, partial, D.nl);
    k_max_partials<<<D.nprob, kBlock, 0, s>>>(D.prob_vtile0, partial, out);
}

__global__ __launch_bounds__(kBlock) void k_axpby(const Tile* __restrict__ vt,
                                                  const PatchInfo* __restrict__ P,
                                                  const int32_t* __restrict__ active,
                                                  const double* __restrict__ a,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ b,
                                                  double* __restrict__ y, int64_t nl) {
    const Tile t = vt[blockIdx.x];
    if (active && !active[t.prob]) return;
    const PatchInfo& p = P[t.patch];
    const double aa = a[t.prob], bb = b[t.prob];
    for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
        const int c = interior_index(p, lin);
        y[c] = aa * x[c] + bb * y[c];
        y[c + nl] = aa * x[c + nl] + bb * y[c + nl];
    }
}

void axpby(const Dev& D, hipStream_t s, const double* a, const double* x, const double* b,
           double* y) {
    k_axpby<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.active, a, x, b, y, D.nl);
}

__global__ __launch_bounds__(kBlock) void k_lincomb2(const Tile* __restrict__ vt,
                                                     const PatchInfo* __restrict__ P,
                                                     const int32_t* __restrict__ active,
                                                     const double* __restrict__ a,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ w,
                                                     double* __restrict__ y, int64_t nl) {
    const Tile t = vt[blockIdx.x];
    if (active && !active[t.prob]) return;
    const PatchInfo& p = P[t.patch];
    const double aa = a[t.prob], bb = b[t.prob];
    for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
        const int c = interior_index(p, lin);
        y[c] = bb * w[c] + aa * x[c];
        y[c + nl] = bb * w[c + nl] + aa * x[c + nl];
    }
}

void lincomb2(const Dev& D, hipStream_t s, const double* a, const double* x, const double* b,
              const double* w, double* y) {
    k_lincomb2<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.active, a, x, b, w, y, D.nl);
}

// y = u + A udot + B u_prev + C u, the terms added in that order
__global__ __launch_bounds__(kBlock) void k_bdf2_predict(const Tile* __restrict__ vt,
                                                         const PatchInfo* __restrict__ P,
                                                         const int32_t* __restrict__ active,
                                                         const double* __restrict__ cf,
                                                         const double* __restrict__ u,
                                                         const double* __restrict__ udot,
                                                         const double* __restrict__ uprev,
                                                         double* __restrict__ y,
                                                         double* __restrict__ pred,
                                                         int nprob, int64_t nl) {
    const Tile t = vt[blockIdx.x];
    if (active && !active[t.prob]) return;
    const PatchInfo& p = P[t.patch];
    const double A = cf[t.prob], B = cf[nprob + t.prob], C = cf[2 * nprob + t.prob];
    const bool copy = A == 0.0 && B == 0.0 && C == 0.0;      // a BDF1 step: y = u
    for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
        const int c = interior_index(p, lin);
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const int64_t i = c + f * nl;
            const double uc = u[i];
            double v = uc;
            if (!copy) {
                v = A * udot[i] + v;
                v = B * uprev[i] + v;
                v = C * uc + v;
            }
            y[i] = v;
            if (pred) pred[i] = v;
        }
    }
}

void bdf2_predict(const Dev& D, hipStream_t s, const double* c, const double* u,
                  const double* udot, const double* uprev, double* y, double* pred) {
    k_bdf2_predict<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.active, c, u, udot,
                                                uprev, y, pred, D.nprob, D.nl);
}

__global__ __launch_bounds__(kBlock) void k_scale_copy(const Tile* __restrict__ vt,
                                                       const PatchInfo* __restrict__ P,
                                                       const int32_t* __restrict__ active,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ sc,
                                                       double* __restrict__ y, int64_t nl) {
    const Tile t = vt[blockIdx.x];
    if (active && !active[t.prob]) return;
    const PatchInfo& p = P[t.patch];
    const double a = sc ? sc[t.prob] : 1.0;
    for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
        const int c = interior_index(p, lin);
        y[c] = a * x[c];
        y[c + nl] = a * x[c + nl];
    }
}

void scale_copy(const Dev& D, hipStream_t s, const double* x, const double* sc, double* y) {
    k_scale_copy<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.active, x, sc, y, D.nl);
}
void copy_interior(const Dev& D, hipStream_t s, const double* x, double* y) {
    k_scale_copy<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.active, x, nullptr, y,
                                              D.nl);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T* __restrict__ x, int64_t n, T v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}
void fill_native(hipStream_t s, double* x, int64_t n, double v) {
    if (n > 0) k_fill<double><<<nblocks(n), kBlock, 0, s>>>(x, n, v);
}
void fill_native_f(hipStream_t s, float* x, int64_t n, float v) {
    if (n > 0) k_fill<float><<<nblocks(n), kBlock, 0, s>>>(x, n, v);
}

__global__ __launch_bounds__(kBlock) void k_pack(const Tile* __restrict__ vt,
                                                 const PatchInfo* __restrict__ P,
                                                 const int64_t* __restrict__ coff,
                                                 const double* __restrict__ nat,
                                                 double* __restrict__ cmp, int nf, int dir,
                                                 int64_t nl, int64_t ncells) {
    const Tile t = vt[blockIdx.x];
    const PatchInfo& p = P[t.patch];
    const int64_t base = coff[t.patch];
    for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
        const int c = interior_index(p, lin);
        for (int f = 0; f < nf; ++f) {
            if (dir == 0)
                cmp[f * ncells + base + lin] = nat[f * nl + c];
            else
                const_cast<double*>(nat)[f * nl + c] = cmp[f * ncells + base + lin];
        }
    }
}

void pack(const Dev& D, hipStream_t s, const int64_t* coff, const double* native,
          double* compact, int nf, int64_t ncells) {
    k_pack<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, coff, native, compact, nf, 0,
                                        D.nl, ncells);
}
void unpack(const Dev& D, hipStream_t s, const int64_t* coff, const double* compact,
            double* native, int nf, int64_t ncells) {
    k_pack<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, coff, native,
                                        const_cast<double*>(compact), nf, 1, D.nl, ncells);
}

__global__ __launch_bounds__(kBlock) void k_check_pos(const Tile* __restrict__ vt,
                                                      const PatchInfo* __restrict__ P,
                                                      const double* __restrict__ x, int nf,
                                                      int32_t* __restrict__ flag,
                                                      int64_t nl) {
    const Tile t = vt[blockIdx.x];
    const PatchInfo& p = P[t.patch];
    int bad = 0;
    for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
        const int c = interior_index(p, lin);
        for (int f = 0; f < nf; ++f) {
            const double v = x[f * nl + c];
            if (!(v > 0.0) || !(v < DBL_MAX)) bad = 1;
        }
    }
    if (bad) atomicOr(flag, 1);
}

void check_positive(const Dev& D, hipStream_t s, const double* x, int nf, int32_t* flag) {
    k_check_pos<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, x, nf, flag, D.nl);
}

__global__ __launch_bounds__(kBlock) void k_cube(const double* __restrict__ z,
                                                 double* __restrict__ z3, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double v = z[i];
        z3[i] = v * v * v;
    }
}
void cube(hipStream_t s, const double* z, double* z3, int64_t n) {
    if (n > 0) k_cube<<<nblocks(n), kBlock, 0, s>>>(z, z3, n);
}

__global__ __launch_bounds__(kBlock) void k_to_float(const double* __restrict__ x,
                                                     float* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}
__global__ __launch_bounds__(kBlock) void k_to_double(const float* __restrict__ x,
                                                      double* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (double)x[i];
}
void to_float(hipStream_t s, const double* x, float* y, int64_t n) {
    if (n > 0) k_to_float<<<nblocks(n), kBlock, 0, s>>>(x, y, n);
}
void to_double(hipStream_t s, const float* x, double* y, int64_t n) {
    if (n > 0) k_to_double<<<nblocks(n), kBlock, 0, s>>>(x, y, n);
}

// ---------------------------------------------------------------------------
// Jacobian-free product (Sec. 4.1, eq. Jac-free): per-problem plain sums over
// composite cells of both fields of u.v, |v| and v.v; the differencing step
//   eps = sqrt(eps_mach) <u,v> / ||v||^2                 if |<u,v>| > u_min ||v||_1
//       = sqrt(eps_mach) u_min sign(<u,v>) ||v||_1 / ||v||^2   otherwise,
// u_min = 1e-6, sign(0) = +1, eps = 1 for v = 0; then w = u + eps v and,
// after the residual of w, Jv = (F(w) - F(u)) / eps.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_fd_sums(
    const Tile* __restrict__ vt, const PatchInfo* __restrict__ P,
    const uint8_t* __restrict__ ctype, const double* __restrict__ u,
    const double* __restrict__ v, double* __restrict__ partial, int64_t nl) {
    __shared__ double sh[4];
    const Tile t = vt[blockIdx.x];
    const PatchInfo& p = P[t.patch];
    const bool cov = p.flags & PF_COVERED;
    double uv = 0.0, l1 = 0.0, v2 = 0.0;
    for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
        const int c = interior_index(p, lin);
        if (cov && (ctype[c] & CT_COVERED)) continue;
        const double v0 = v[c], v1 = v[c + nl];
        uv += u[c] * v0 + u[c + nl] * v1;
        l1 += fabs(v0) + fabs(v1);
        v2 += v0 * v0 + v1 * v1;
    }
    uv = block_sum(uv, sh);
    l1 = block_sum(l1, sh);
    v2 = block_sum(v2, sh);
    if (threadIdx.x == 0) {
        partial[(int64_t)blockIdx.x * 3 + 0] = uv;
        partial[(int64_t)blockIdx.x * 3 + 1] = l1;
        partial[(int64_t)blockIdx.x * 3 + 2] = v2;
    }
}

__device__ __forceinline__ double fd_step(const double* __restrict__ S) {
    const double uv = S[0], l1 = S[1], v2 = S[2];
    const double root = 0x1p-26;                 // sqrt(2^-52), exact
    if (!(v2 > 0.0)) return 1.0;
    if (fabs(uv) > 1e-6 * l1) return root * uv / v2;
    const double sg = uv >= 0.0 ? 1.0 : -1.0;
    return root * 1e-6 * sg * l1 / v2;
}

__global__ __launch_bounds__(kBlock) void k_fd_shift(
    const Tile* __restrict__ vt, const PatchInfo* __restrict__ P,
    const double* __restrict__ sums, const double* __restrict__ u,
    const double* __restrict__ v, double* __restrict__ w, int64_t nl) {
    const Tile t = vt[blockIdx.x];
    const PatchInfo& p = P[t.patch];
    const double eps = fd_step(sums + 3 * t.prob);
    for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
        const int c = interior_index(p, lin);
        w[c] = u[c] + eps * v[c];
        w[c + nl] = u[c + nl] + eps * v[c + nl];
    }
}

__global__ __launch_bounds__(kBlock) void k_fd_quotient(
    const Tile* __restrict__ vt, const PatchInfo* __restrict__ P,
    const double* __restrict__ sums, const double* __restrict__ F0,
    double* __restrict__ Jv, int64_t nl) {
    const Tile t = vt[blockIdx.x];
    const PatchInfo& p = P[t.patch];
    const double eps = fd_step(sums + 3 * t.prob);
    for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
        const int c = interior_index(p, lin);
        Jv[c] = (Jv[c] - F0[c]) / eps;
        Jv[c + nl] = (Jv[c + nl] - F0[c + nl]) / eps;
    }
}

void fd_sums(const Dev& D, hipStream_t s, const double* u, const double* v, double* partial,
             double* sums) {
    k_fd_sums<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, u, v, partial, D.nl);
    k_sum_partials<<<D.nprob, kBlock, 0, s>>>(D.prob_vtile0, partial, 3, sums, 3);
}
void fd_shift(const Dev& D, hipStream_t s, const double* sums, const double* u,
              const double* v, double* w) {
    k_fd_shift<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, sums, u, v, w, D.nl);
}
void fd_quotient(const Dev& D, hipStream_t s, const double* sums, const double* F0,
                 double* Jv) {
    k_fd_quotient<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, sums, F0, Jv, D.nl);
}

// ---------------------------------------------------------------------------
// FGMRES per-problem scalars (one thread per problem)
//   H: [nprob][(m+1) * m], column j at H[p][(m+1) j]
// ---------------------------------------------------------------------------

__global__ void k_gmres_column(int nprob, int m, int j, const int32_t* __restrict__ active,
                               const double* __restrict__ h1, const double* __restrict__ h2,
                               const double* __restrict__ hn2, double* __restrict__ H,
                               double* __restrict__ cs, double* __restrict__ sn,
                               double* __restrict__ g, double* __restrict__ rho,
                               double* __restrict__ vscale) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob) return;
    if (active && !active[p]) {
        vscale[p] = 0.0;
        return;
    }
    double* col = H + (int64_t)p * (m + 1) * m + (int64_t)(m + 1) * j;
    double* c = cs + p * m;
    double* s = sn + p * m;
    double* gg = g + p * (m + 1);
    for (int i = 0; i <= j; ++i) col[i] = h1[p * (j + 1) + i] + h2[p * (j + 1) + i];
    const double hn = sqrt(hn2[p]);
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double tmp = c[i] * col[i] + s[i] * col[i + 1];
        col[i + 1] = -s[i] * col[i] + c[i] * col[i + 1];
        col[i] = tmp;
    }
    const double a = col[j], b = col[j + 1];
    double cc, ss, r;
    if (b == 0.0) {
        cc = 1.0;
        ss = 0.0;
        r = a;
    } else {
        r = sqrt(a * a + b * b);
        cc = a / r;
        ss = b / r;
    }
    c[j] = cc;
    s[j] = ss;
    col[j] = r;
    col[j + 1] = 0.0;
    gg[j + 1] = -ss * gg[j];
    gg[j] = cc * gg[j];
    rho[p] = fabs(gg[j + 1]);
    vscale[p] = hn > 0.0 ? 1.0 / hn : 0.0;
}

void gmres_column(hipStream_t s, int nprob, int m, int j, const int32_t* active,
                  const double* h1, const double* h2, const double* hn2, double* H, double* cs,
                  double* sn, double* g, double* rho, double* vscale) {
    k_gmres_column<<<(nprob + 63) / 64, 64, 0, s>>>(nprob, m, j, active, h1, h2, hn2, H, cs,
                                                    sn, g, rho, vscale);
}

__global__ void k_gmres_backsolve(int nprob, int m, const int32_t* __restrict__ kdim,
                                  const double* __restrict__ H, const double* __restrict__ g,
                                  double* __restrict__ y) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob) return;
    const int k = kdim[p];
    const double* Hp = H + (int64_t)p * (m + 1) * m;
    const double* gp = g + p * (m + 1);
    double* yp = y + p * m;
    for (int i = k; i < m; ++i) yp[i] = 0.0;
    for (int i = k - 1; i >= 0; --i) {
        double acc = gp[i];
        for (int l = i + 1; l < k; ++l) acc -= Hp[(m + 1) * l + i] * yp[l];
        yp[i] = acc / Hp[(m + 1) * i + i];
    }
}

void gmres_backsolve(hipStream_t s, int nprob, int m, const int32_t* kdim, const double* H,
                     const double* g, double* y) {
    k_gmres_backsolve<<<(nprob + 63) / 64, 64, 0, s>>>(nprob, m, kdim, H, g, y);
}

}  // namespace nrd
