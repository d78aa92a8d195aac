// Dynamic regridding on the device (paper Sec. 5): refinement tags of the
// current state and the transfer of solution data from one hierarchy to
// another by conservative, minmod-limited linear refinement.
//
// Tags are evaluated per interior cell of every patch (covered cells too)
// from the synced, ghost-filled state: centred differences along each axis,
// with the cell itself standing in for a neighbour beyond a physical face.
// The decisions are taken with exactly the operations below, in this order
// and without contraction into fused multiply-adds, so that a CPU
// evaluation of the same formulas reaches the same tags.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "kernels.h"

namespace nrd {

static inline int nblocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------------------
// max |E| over composite cells, per problem (two stages, fixed order)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double rg_wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double rg_block_max(double v, double* sh) {
    v = rg_wave_max(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    const double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kBlock) void k_absmax(const Tile* __restrict__ vt,
                                                   const PatchInfo* __restrict__ P,
                                                   const uint8_t* __restrict__ ctype,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ partial) {
    __shared__ double sh[4];
    const Tile t = vt[blockIdx.x];
    const PatchInfo& p = P[t.patch];
    const bool cov = p.flags & PF_COVERED;
    double m = 0.0;
    for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
        const int i = lin % p.n[0], r = lin / p.n[0];
        const int c = p.off + (i + 1) + p.sy * (r % p.n[1] + 1) + p.sz * (r / p.n[1] + 1);
        if (cov && (ctype[c] & CT_COVERED)) continue;
        m = fmax(m, fabs(x[c]));
    }
    const double r = rg_block_max(m, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ __launch_bounds__(kBlock) void k_absmax_partials(const int32_t* __restrict__ t0,
                                                         const double* __restrict__ partial,
                                                         double* __restrict__ out) {
    __shared__ double sh[4];
    const int p = blockIdx.x;
    double m = 0.0;
    for (int i = t0[p] + threadIdx.x; i < t0[p + 1]; i += kBlock) m = fmax(m, partial[i]);
    const double r = rg_block_max(m, sh);
    if (threadIdx.x == 0) out[p] = r;
}

void abs_max(const Dev& D, hipStream_t s, const double* x, double* partial, double* out) {
    k_absmax<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, D.ctype, x, partial);
    k_absmax_partials<<<D.nprob, kBlock, 0, s>>>(D.prob_vtile0, partial, out);
}

// ---------------------------------------------------------------------------
// tags
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_tag(const Tile* __restrict__ vt,
                                                const PatchInfo* __restrict__ P,
                                                const int64_t* __restrict__ coff,
                                                const double* __restrict__ E,
                                                const double* __restrict__ z,
                                                const double* __restrict__ emax, TagCrit tc,
                                                uint8_t* __restrict__ tags) {
#pragma clang fp contract(off)
    const Tile t = vt[blockIdx.x];
    const PatchInfo& p = P[t.patch];
    const double den = 0.1 * emax[t.prob];
    const int st[3] = {1, p.sy, p.sz};
    for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
        const int i = lin % p.n[0], r = lin / p.n[0];
        const int idx[3] = {i, r % p.n[1], r / p.n[1]};
        const int c = p.off + (idx[0] + 1) + p.sy * (idx[1] + 1) + p.sz * (idx[2] + 1);
        const double e = E[c];
        double g2 = 0.0, ng = 0.0, nc = 0.0;
        bool zt = false;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const bool lo_phys = ((p.phys >> (2 * d)) & 1) && idx[d] == 0;
            const bool hi_phys = ((p.phys >> (2 * d + 1)) & 1) && idx[d] == p.n[d] - 1;
            const int cm = lo_phys ? c : c - st[d];
            const int cp = hi_phys ? c : c + st[d];
            const double em = E[cm], ep = E[cp];
            const double ed = (ep - em) / (2.0 * p.h[d]);
            g2 = g2 + ed * ed;
            ng = ng + 0.5 * fabs(ep - em);
            nc = nc + fabs((ep - e) - (e - em));
            zt = zt || (z[cm] != z[c]) || (z[cp] != z[c]);
        }
        bool tag = false;
        if (tc.grad > 0.0) tag = tag || g2 > (tc.grad * e) * (tc.grad * e);
        if (tc.z_interface) tag = tag || zt;
        if (tc.tau_g > 0.0) tag = tag || (ng / den) > tc.tau_g;
        if (tc.tau_c > 0.0) tag = tag || (nc / den) > tc.tau_c;
        tags[coff[t.patch] + lin] = tag ? 1 : 0;
    }
}

void tag_cells(const Dev& D, hipStream_t s, const int64_t* coff, const double* E,
               const double* z, const double* emax, const TagCrit& tc, uint8_t* tags) {
    k_tag<<<D.nvtiles, kBlock, 0, s>>>(D.vtiles, D.patches, coff, E, z, emax, tc, tags);
}

// Coarse-fine ghosts of x take the value of their coarse parent (the first
// source of the interpolation), sibling ghosts the sibling's: the material
// a ghost cell lies in, for the interface tag.
__global__ __launch_bounds__(kBlock) void k_ghost_parent(const GhostCopy* __restrict__ cp,
                                                         int ncp,
                                                         const GhostCF* __restrict__ cf,
                                                         int ncf, double* __restrict__ x) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ncp) {
        const GhostCopy e = cp[t];
        x[e.dst] = x[e.src];
    } else if (t < ncp + ncf) {
        const GhostCF e = cf[t - ncp];
        x[e.dst] = x[e.src[0]];
    }
}

void ghost_fill_parent(const Dev& D, hipStream_t s, double* x) {
    const int n = D.ncopy + D.ncf;
    if (n == 0) return;
    k_ghost_parent<<<nblocks(n), kBlock, 0, s>>>(D.gcopy, D.ncopy, D.gcf, D.ncf, x);
}

// ---------------------------------------------------------------------------
// transfer
// ---------------------------------------------------------------------------

// dst cells of a fragment box (level index space) <- src cells, nf fields
__global__ __launch_bounds__(kBlock) void k_xfer_copy(
    const XferChunk* __restrict__ chunks, const XferFrag* __restrict__ frags,
    const PatchInfo* __restrict__ dP, const PatchInfo* __restrict__ sP,
    const double* __restrict__ src, double* __restrict__ dst, int64_t snl, int64_t dnl,
    int nf) {
    const XferChunk ch = chunks[blockIdx.x];
    const XferFrag f = frags[ch.frag];
    const PatchInfo& dp = dP[f.dpatch];
    const PatchInfo& sp = sP[f.spatch];
    for (int lin = ch.start + threadIdx.x; lin < ch.start + ch.count; lin += kBlock) {
        const int i = lin % f.n[0], r = lin / f.n[0];
        const int I0 = f.lo[0] + i, I1 = f.lo[1] + r % f.n[1], I2 = f.lo[2] + r / f.n[1];
        const int dc = dp.off + (I0 - dp.lo[0] + 1) + dp.sy * (I1 - dp.lo[1] + 1) +
                       dp.sz * (I2 - dp.lo[2] + 1);
        const int sc = sp.off + (I0 - sp.lo[0] + 1) + sp.sy * (I1 - sp.lo[1] + 1) +
                       sp.sz * (I2 - sp.lo[2] + 1);
        for (int q = 0; q < nf; ++q) dst[q * dnl + dc] = src[q * snl + sc];
    }
}

void xfer_copy(hipStream_t s, int nchunks, const XferChunk* chunks, const XferFrag* frags,
               const PatchInfo* dP, const PatchInfo* sP, const double* src, double* dst,
               int64_t snl, int64_t dnl, int nf) {
    if (nchunks > 0)
        k_xfer_copy<<<nchunks, kBlock, 0, s>>>(chunks, frags, dP, sP, src, dst, snl, dnl, nf);
}

// shadow[q * slen + i] = x[q * nl + src[i]] for the shadow cells [a, b)
__global__ __launch_bounds__(kBlock) void k_shadow_gather(const int32_t* __restrict__ ssrc,
                                                          int a, int b,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ sh,
                                                          int64_t nl, int64_t slen, int nf) {
    const int i = a + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b) return;
    const int c = ssrc[i];
    for (int q = 0; q < nf; ++q) sh[q * slen + i] = x[q * nl + c];
}

__device__ __forceinline__ double rg_minmod(double a, double b) {
    return (a > 0.0 && b > 0.0) ? fmin(a, b) : ((a < 0.0 && b < 0.0) ? fmax(a, b) : 0.0);
}

// every cell of the level's patches <- minmod-limited linear refinement of
// its parent in the shadow block of the coarser level
__global__ __launch_bounds__(kBlock) void k_refine(const Tile* __restrict__ tiles, int t0,
                                                   const PatchInfo* __restrict__ P,
                                                   const ShadowPatch* __restrict__ shp,
                                                   const double* __restrict__ sh,
                                                   double* __restrict__ x, int64_t nl,
                                                   int64_t slen, int nf) {
#pragma clang fp contract(off)
    const Tile t = tiles[t0 + blockIdx.x];
    const PatchInfo& p = P[t.patch];
    const ShadowPatch sp = shp[t.patch];
    const int sst[3] = {1, sp.m0, sp.m0 * sp.m1};
    for (int lin = t.start + threadIdx.x; lin < t.start + t.count; lin += kBlock) {
        const int i = lin % p.n[0], r = lin / p.n[0];
        const int idx[3] = {i, r % p.n[1], r / p.n[1]};
        int s0 = sp.off;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int I = p.lo[d] + idx[d];
            s0 += ((I >> 1) - (p.lo[d] >> 1) + 1) * sst[d];
        }
        const int c = p.off + (idx[0] + 1) + p.sy * (idx[1] + 1) + p.sz * (idx[2] + 1);
        for (int q = 0; q < nf; ++q) {
            const double* S = sh + q * slen;
            const double u = S[s0];
            double v = u;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double s = rg_minmod(S[s0 + sst[d]] - u, u - S[s0 - sst[d]]);
                v = v + (((p.lo[d] + idx[d]) & 1) ? 0.25 * s : -0.25 * s);
            }
            x[q * nl + c] = v;
        }
    }
}

void refine_level(const Dev& D, hipStream_t s, const ShadowPatch* shadows,
                  const int32_t* shadow_src, int lev, double* x, double* sh, int64_t slen,
                  int nf) {
    const int a = D.level_shadow0[lev], b = D.level_shadow0[lev + 1];
    if (b > a)
        k_shadow_gather<<<nblocks(b - a), kBlock, 0, s>>>(shadow_src, a, b, x, sh, D.nl, slen,
                                                          nf);
    const int t0 = D.level_tile0[lev], nt = D.level_tile0[lev + 1] - t0;
    if (nt > 0)
        k_refine<<<nt, kBlock, 0, s>>>(D.tiles, t0, D.patches, shadows, sh, x, D.nl, slen, nf);
}

}  // namespace nrd
