// Launchers of the HIP kernels (defined in sync.hip, stencil.hip, vec.hip, precond.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "nrd_internal.h"

namespace nrd {

constexpr int kMaxLev = 12;
constexpr int kBlock = 256;          // threads per workgroup (4 wave64)

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Tile lists are ordered so that neighbouring tiles share halo data;
// this bijection gives each XCD a contiguous range of tiles instead of every
// 8th one, so a tile's neighbours sit in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int x = b & 7, q = b >> 3;
    const int base = n >> 3, rem = n & 7;
    return x * base + (x < rem ? x : rem) + q;
}

// Flux matching runs four lanes per coarse cell, lane q of a quad taking
// fine face q of each refluxed face.  quad_sum returns, in lane 0 of the
// quad, (((0 + x_0) + x_1) + x_2) + x_3 of the quad's values: the order of a
// sequential loop over the four fine faces.  Every lane of the quad must
// be active.
template <typename V>
__device__ __forceinline__ V quad_sum(V x) {
    const int b = (int)(threadIdx.x & 63) & ~3;
    const V x1 = __shfl(x, b + 1, 64);
    const V x2 = __shfl(x, b + 2, 64);
    const V x3 = __shfl(x, b + 3, 64);
    return (((V(0) + x) + x1) + x2) + x3;
}

// Tile of this workgroup in a launch over tiles [t0, t0 + gridDim.x), or,
// given an index map (the tiles of the problems being solved, in list
// order), over map[0 .. gridDim.x).
__device__ __forceinline__ int tile_index(const int32_t* map, int t0) {
    const int i = xcd_tile(blockIdx.x, gridDim.x);
    return map ? map[i] : t0 + i;
}

// Event timing of operator launches on the library stream (implemented by
// the hierarchy; inactive unless timing is enabled).
struct Clock {
    virtual std::pair<hipEvent_t, hipEvent_t> tic(int which) = 0;
    virtual void toc(int which, std::pair<hipEvent_t, hipEvent_t> p) = 0;
  protected:
    ~Clock() = default;
};

// Device views of the hierarchy tables (pointers into the workspace) plus the
// host-side counts that size the launches.
struct Dev {
    int64_t nl = 0;
    int32_t nprob = 0, nlev = 0, nbox = 0;
    const PatchInfo* patches = nullptr;
    const Tile* tiles = nullptr;
    int32_t level_tile0[kMaxLev + 1] = {};
    const STile* stiles = nullptr;           // z-marching bricks
    int32_t level_stile0[kMaxLev + 1] = {};
    int32_t bricks = 0;                      // stencil variant: 0 flat, 1 bricks
    const Tile* vtiles = nullptr;
    int32_t nvtiles = 0;
    const int32_t* prob_vtile0 = nullptr;    // device [nprob+1]
    const GhostCopy* gcopy = nullptr;
    int32_t ncopy = 0;
    const GhostCF* gcf = nullptr;
    int32_t ncf = 0;
    const GhostCopy* sib = nullptr;
    int32_t level_sib0[kMaxLev + 1] = {};
    const SyncEntry* sync[kMaxLev] = {};
    int32_t nsync[kMaxLev] = {};
    const RefluxFace* rfaces = nullptr;
    const RefluxCell* rcells = nullptr;
    int32_t nrcells = 0;
    const CFRow* cfrows = nullptr;           // transposed coarse-fine interpolation
    const CFSrc* cfsrc = nullptr;
    int32_t ncfrows = 0;
    const uint8_t* ctype = nullptr;
    const ProbScalars* ps = nullptr;         // device [nprob]
    const int32_t* active = nullptr;         // device [nprob], 1 = work on it
    // stencil tiles (plane tiles, or flat tiles for the flat variant) of the
    // problems flagged in active, valid while active is set; NULL when the
    // launches must read the flags instead (captured graphs)
    const int32_t* amap = nullptr;
    int32_t namap = 0;
    const double* z3 = nullptr;              // native, z^3 with ghosts
    const double* z = nullptr;               // native, z with ghosts
    int32_t level_shadow0[kMaxLev + 1] = {}; // prolongation shadow cells per level
};

// ---- sync.hip -----------------------------------------------------------
// x: NF fields of native length nl.  Fills the sibling and coarse-fine
// ghosts of every patch (physical ghosts are never read).
void ghost_fill_d(const Dev& D, hipStream_t s, double* x, int nf);
void ghost_fill_f(const Dev& D, hipStream_t s, float* x, int nf);
// covered cells <- mean of children, finest level first
void restrict_d(const Dev& D, hipStream_t s, double* x, int nf, int lev_lo = 0);
void restrict_f(const Dev& D, hipStream_t s, float* x, int nf, int lev_lo = 0);
// adjoint fill of a multiplier vector's two fields: sibling copies, 1/8 of
// the coarse cell at a coarse-fine ghost
void adjoint_ghost_fill(const Dev& D, hipStream_t s, double* x);
// transposed restriction (coarsest level first): each covered cell adds 1/8
// of its value to its children and is set to 0
void restrict_transpose(const Dev& D, hipStream_t s, double* x, int nf);
// covered cells <- 0
void zero_covered(const Dev& D, hipStream_t s, double* x, int nf);
// sibling ghosts of levels lev .. lev_hi (lev_hi < 0: lev only)
void sibling_exchange_f(const Dev& D, hipStream_t s, float* x, int nf, int lev,
                        int lev_hi = -1);
void sibling_exchange_d(const Dev& D, hipStream_t s, double* x, int nf, int lev,
                        int lev_hi = -1);

// ---- stencil.hip --------------------------------------------------------

// F = c0 u - b - dt f(u) over tiles [t0, t0+nt) (bricks if D.bricks);
// covered cells = 0.  residual_all / jvp_all cover every tile, or only the
// tiles of the active problems when D.amap is set.
void residual(const Dev& D, hipStream_t s, int t0, int nt, const double* u,
              const double* b, double* F);
void residual_all(const Dev& D, hipStream_t s, const double* u, const double* b, double* F);
void residual_reflux(const Dev& D, hipStream_t s, const double* u, double* F);
// Jv
void jvp(const Dev& D, hipStream_t s, int t0, int nt, const double* u,
         const double* v, double* Jv);
void jvp_all(const Dev& D, hipStream_t s, const double* u, const double* v, double* Jv);
void jvp_reflux(const Dev& D, hipStream_t s, const double* u, const double* v,
                double* Jv);
// transpose on any hierarchy: JTl = (dF/du)^T lam (native; covered cells
// 0) and gz = (dF/dz)^T lam (native, every cell).  lam's ghosts are
// overwritten (adjoint fill); the ghost slots of JTl and gz are scratch.
void vjp_full(const Dev& D, hipStream_t s, const double* u, double* lam, double* JTl,
              double* gz);

// ---- vec.hip ------------------------------------------------------------
// Deterministic per-problem reductions over vtiles.
//   out[p * nv + v] = sum over composite cells of problem p of
//                     vol * (x_v . y) (both fields), x_v = X + v * xstride
//   (xsc: optional per-problem factor applied to every x_v as it is read,
//   giving the values a scale_copy of X would hold; also for the next two)
void multidot(const Dev& D, hipStream_t s, const double* X, int64_t xstride,
              int nv, const double* y, double* partial, double* out,
              const double* xsc = nullptr);
// out[p] = min over composite cells of min(E + lam_p dE, T + lam_p dT)
void min_positive(const Dev& D, hipStream_t s, const double* u, const double* du,
                  const double* lam, double* partial, double* out);
// y = sum_v coef[p][v] x_v (+ y if accumulate) on interior cells of active
// problems; coef row stride cstride
void combine(const Dev& D, hipStream_t s, const double* X, int64_t xstride,
             int nv, const double* coef, int cstride, double* y, int accumulate,
             double alpha);
// y -= sum_v coef[p][v] x_v, then out[p * nv + v] = x_v . y (one pass for
// nv <= 16; the values of combine followed by multidot)
void combine_dot(const Dev& D, hipStream_t s, const double* X, int64_t xstride, int nv,
                 const double* coef, int cstride, double* y, double* partial, double* out,
                 const double* xsc = nullptr);
// y -= sum_v coef[p][v] x_v, then out[p] = ||y||^2 (composite, volume
// weighted) in the same pass over y
void combine_norm(const Dev& D, hipStream_t s, const double* X, int64_t xstride,
                  int nv, const double* coef, int cstride, double* y, double* partial,
                  double* out, const double* xsc = nullptr);
// Newton update from a Krylov basis (nv <= 16): keep = x, x -= sum_v
// coef[p][v] z_v on active problems, out[p] = min over composite cells of
// both fields of the new x (-1 for NaN)
void update_min(const Dev& D, hipStream_t s, const double* Z, int64_t zstride, int nv,
                const double* coef, int cstride, double* x, double* keep, double* partial,
                double* out);
// out[p] = max over composite cells of |c_p (x - xp)| / (x + eta) over both
// fields (eta_E, eta_T): the scaled max norm of the BDF2 error estimate
void err_norm(const Dev& D, hipStream_t s, const double* x, const double* xp,
              const double* coef, double eta_E, double eta_T, double* partial, double* out);
// y = a_p x + b_p y elementwise (a, b per problem, host-computed device arrays)
void axpby(const Dev& D, hipStream_t s, const double* a, const double* x,
           const double* b, double* y);
// y = a_p x + b_p w elementwise in one pass (a, b per problem)
void lincomb2(const Dev& D, hipStream_t s, const double* a, const double* x, const double* b,
              const double* w, double* y);
// The leapfrog predictor of a BDF2 step in one pass, coefficients c = (A, B,
// C) per problem: y = u + A udot + B u_prev + C u; pred (may be NULL) gets
// a copy of y
void bdf2_predict(const Dev& D, hipStream_t s, const double* c, const double* u,
                  const double* udot, const double* uprev, double* y, double* pred);
// y = x * scale_p (scale device [nprob])
void scale_copy(const Dev& D, hipStream_t s, const double* x, const double* sc,
                double* y);
void copy_interior(const Dev& D, hipStream_t s, const double* x, double* y);
void fill_native(hipStream_t s, double* x, int64_t n, double v);
void fill_native_f(hipStream_t s, float* x, int64_t n, float v);
void pack(const Dev& D, hipStream_t s, const int64_t* coff, const double* native,
          double* compact, int nf, int64_t ncells);
void unpack(const Dev& D, hipStream_t s, const int64_t* coff,
            const double* compact, double* native, int nf, int64_t ncells);
// flag[0] = 1 if any interior value of the nf fields is <= 0 or not finite
void check_positive(const Dev& D, hipStream_t s, const double* x, int nf,
                    int32_t* flag);
void cube(hipStream_t s, const double* z, double* z3, int64_t n);
void to_float(hipStream_t s, const double* x, float* y, int64_t n);
void to_double(hipStream_t s, const float* x, double* y, int64_t n);

// Jacobian-free product pieces (all problems): sums[3 p..] = plain sums over
// composite cells of u.v, |v|, v.v; w = u + eps_p v; Jv = (Jv - F0) / eps_p.
void fd_sums(const Dev& D, hipStream_t s, const double* u, const double* v,
             double* partial, double* sums);
void fd_shift(const Dev& D, hipStream_t s, const double* sums, const double* u,
              const double* v, double* w);
void fd_quotient(const Dev& D, hipStream_t s, const double* sums, const double* F0,
                 double* Jv);

// ---- regrid.hip ---------------------------------------------------------
// out[p] = max over composite cells of problem p of |x| (field 0)
void abs_max(const Dev& D, hipStream_t s, const double* x, double* partial, double* out);
// tags[coff[b] + lin] = 1 where a criterion holds at interior cell lin of
// patch b (covered cells included); E, z native with ghosts filled (z's
// coarse-fine ghosts by ghost_fill_parent); emax per problem
void tag_cells(const Dev& D, hipStream_t s, const int64_t* coff, const double* E,
               const double* z, const double* emax, const TagCrit& tc, uint8_t* tags);
// sibling ghosts copied, coarse-fine ghosts set to their coarse parent
void ghost_fill_parent(const Dev& D, hipStream_t s, double* x);
// fragment copies from another hierarchy's native vector (src, snl cells
// per field, patch table sP) into this one's (dst, dnl, dP)
void xfer_copy(hipStream_t s, int nchunks, const XferChunk* chunks, const XferFrag* frags,
               const PatchInfo* dP, const PatchInfo* sP, const double* src, double* dst,
               int64_t snl, int64_t dnl, int nf);
// every cell of level lev (>= 1) of x <- conservative minmod-limited linear
// refinement of level lev - 1 of x (sh: shadow scratch of nf * slen values)
void refine_level(const Dev& D, hipStream_t s, const ShadowPatch* shadows,
                  const int32_t* shadow_src, int lev, double* x, double* sh, int64_t slen,
                  int nf);

// Givens / Hessenberg update of FGMRES for every active problem.
//   hcol [nprob][m+1] holds the new column (CGS sums), hn2 [nprob] = ||w||^2
void gmres_column(hipStream_t s, int nprob, int m, int j, const int32_t* active,
                  const double* h1, const double* h2, const double* hn2,
                  double* H, double* cs, double* sn, double* g, double* rho,
                  double* vscale);
void gmres_backsolve(hipStream_t s, int nprob, int m, const int32_t* kdim,
                     const double* H, const double* g, double* y);

}  // namespace nrd
