// Synchronisation of the AMR hierarchy (paper Sec. 3.2.1): covered cells
// take the mean of their eight children (restriction, finest level first);
// ghosts take a sibling patch's value or the coarse-fine interpolation of
// the coarser level (a bilinear tangential stencil of four coarse cells,
// weights 9, 3, 3, 1 over 16, blended 2/3 : 1/3 with the fine cell inside).
// Both are driven by flat host-built tables, one thread per entry.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace nrd {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_ghost_fill(const GhostCopy* __restrict__ cp,
                                                       int ncp,
                                                       const GhostCF* __restrict__ cf,
                                                       int ncf, T* __restrict__ x, int nf,
                                                       int64_t nl) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ncp) {
        const GhostCopy e = cp[t];
        for (int f = 0; f < nf; ++f) x[f * nl + e.dst] = x[f * nl + e.src];
    } else if (t < ncp + ncf) {
        const GhostCF e = cf[t - ncp];
        for (int f = 0; f < nf; ++f) {
            const T* y = x + f * nl;
            const T ci = (T(9) * y[e.src[0]] + T(3) * y[e.src[1]] + T(3) * y[e.src[2]] +
                          y[e.src[3]]) * T(0.0625);
            x[f * nl + e.dst] = T(2.0 / 3.0) * ci + T(1.0 / 3.0) * y[e.src[4]];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(const SyncEntry* __restrict__ se,
                                                     int n, T* __restrict__ x, int nf,
                                                     int64_t nl) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const SyncEntry e = se[t];
    for (int f = 0; f < nf; ++f) {
        const T* y = x + f * nl + e.src;
        T acc = y[0];
        acc += y[1];
        acc += y[e.sy];
        acc += y[e.sy + 1];
        acc += y[e.sz];
        acc += y[e.sz + 1];
        acc += y[e.sz + e.sy];
        acc += y[e.sz + e.sy + 1];
        x[f * nl + e.dst] = acc * T(0.125);
    }
}

static inline int nblocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

void ghost_fill_d(const Dev& D, hipStream_t s, double* x, int nf) {
    const int n = D.ncopy + D.ncf;
    if (n == 0) return;
    k_ghost_fill<double><<<nblocks(n), kBlock, 0, s>>>(D.gcopy, D.ncopy, D.gcf, D.ncf, x,
                                                      nf, D.nl);
}
void ghost_fill_f(const Dev& D, hipStream_t s, float* x, int nf) {
    const int n = D.ncopy + D.ncf;
    if (n == 0) return;
    k_ghost_fill<float><<<nblocks(n), kBlock, 0, s>>>(D.gcopy, D.ncopy, D.gcf, D.ncf, x,
                                                     nf, D.nl);
}

template <typename T>
static void restrict_t(const Dev& D, hipStream_t s, T* x, int nf, int lev_lo) {
    for (int l = D.nlev - 2; l >= lev_lo; --l) {
        if (D.nsync[l] == 0) continue;
        k_restrict<T><<<nblocks(D.nsync[l]), kBlock, 0, s>>>(D.sync[l], D.nsync[l], x, nf,
                                                             D.nl);
    }
}
void restrict_d(const Dev& D, hipStream_t s, double* x, int nf, int lev_lo) {
    restrict_t<double>(D, s, x, nf, lev_lo);
}
void restrict_f(const Dev& D, hipStream_t s, float* x, int nf, int lev_lo) {
    restrict_t<float>(D, s, x, nf, lev_lo);
}

// Adjoint ghost fill of the two fields of a multiplier vector: sibling
// copies; a coarse-fine ghost takes 1/8 of the coarse cell it lies in.
__global__ __launch_bounds__(kBlock) void k_adjoint_ghost(const GhostCopy* __restrict__ cp,
                                                          int ncp,
                                                          const GhostCF* __restrict__ cf,
                                                          int ncf, double* __restrict__ x,
                                                          int64_t nl) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ncp) {
        const GhostCopy e = cp[t];
        x[e.dst] = x[e.src];
        x[nl + e.dst] = x[nl + e.src];
    } else if (t < ncp + ncf) {
        const GhostCF e = cf[t - ncp];
        x[e.dst] = 0.125 * x[e.src[0]];
        x[nl + e.dst] = 0.125 * x[nl + e.src[0]];
    }
}

// Transposed restriction of one level: a covered cell hands 1/8 of its
// value to each child and keeps none.
__global__ __launch_bounds__(kBlock) void k_restrict_t(const SyncEntry* __restrict__ se,
                                                       int n, double* __restrict__ x, int nf,
                                                       int64_t nl) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const SyncEntry e = se[t];
    for (int f = 0; f < nf; ++f) {
        double* y = x + f * nl + e.src;
        const double v = 0.125 * x[f * nl + e.dst];
        y[0] += v;
        y[1] += v;
        y[e.sy] += v;
        y[e.sy + 1] += v;
        y[e.sz] += v;
        y[e.sz + 1] += v;
        y[e.sz + e.sy] += v;
        y[e.sz + e.sy + 1] += v;
        x[f * nl + e.dst] = 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_zero_covered(const SyncEntry* __restrict__ se,
                                                         int n, double* __restrict__ x,
                                                         int nf, int64_t nl) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t c = se[t].dst;
    for (int f = 0; f < nf; ++f) x[f * nl + c] = 0.0;
}

void adjoint_ghost_fill(const Dev& D, hipStream_t s, double* x) {
    const int n = D.ncopy + D.ncf;
    if (n == 0) return;
    k_adjoint_ghost<<<nblocks(n), kBlock, 0, s>>>(D.gcopy, D.ncopy, D.gcf, D.ncf, x, D.nl);
}
void restrict_transpose(const Dev& D, hipStream_t s, double* x, int nf) {
    for (int l = 0; l + 1 < D.nlev; ++l) {
        if (D.nsync[l] == 0) continue;
        k_restrict_t<<<nblocks(D.nsync[l]), kBlock, 0, s>>>(D.sync[l], D.nsync[l], x, nf, D.nl);
    }
}
void zero_covered(const Dev& D, hipStream_t s, double* x, int nf) {
    for (int l = 0; l + 1 < D.nlev; ++l) {
        if (D.nsync[l] == 0) continue;
        k_zero_covered<<<nblocks(D.nsync[l]), kBlock, 0, s>>>(D.sync[l], D.nsync[l], x, nf,
                                                              D.nl);
    }
}

template <typename T>
static void sib_t(const Dev& D, hipStream_t s, T* x, int nf, int lev, int lev_hi) {
    const int a = D.level_sib0[lev], b = D.level_sib0[(lev_hi < 0 ? lev : lev_hi) + 1];
    if (b <= a) return;
    k_ghost_fill<T><<<nblocks(b - a), kBlock, 0, s>>>(D.sib + a, b - a, nullptr, 0, x, nf,
                                                     D.nl);
}
void sibling_exchange_f(const Dev& D, hipStream_t s, float* x, int nf, int lev, int lev_hi) {
    sib_t<float>(D, s, x, nf, lev, lev_hi);
}
void sibling_exchange_d(const Dev& D, hipStream_t s, double* x, int nf, int lev, int lev_hi) {
    sib_t<double>(D, s, x, nf, lev, lev_hi);
}

}  // namespace nrd
