// Preconditioner state and drivers (see precond.hip).
#pragma once

#include "kernels.h"

namespace nrd {

constexpr int kMaxMG = 12;

// Colour-split storage of the level-0 iterate e and right-hand side f of
// the multigrid V-cycle (hierarchies whose problems have one level and one
// level-0 box, each of even x extent; `split0`).  Within the ghosted block of
// (n0 + 2)(n1 + 2)(n2 + 2) values of a box, the positions of colour 0 come
// first and those of colour 1 after them, each half in native order with
// rows of (n0 + 2) / 2 values.  The colour of ghosted position (x, y, z) is
// the parity of x + y + z + lo_0 + lo_1 + lo_2 + 1: for interior cell
// (x - 1, y - 1, z - 1) its red-black colour.  A half-sweep then reads only
// its own colour's f and the other colour's e, and writes whole lines of e.
__host__ __device__ inline int split_colour(const PatchInfo& p, int x, int y, int z) {
    return (x + y + z + p.lo[0] + p.lo[1] + p.lo[2] + 1) & 1;
}
__host__ __device__ inline int split_index(const PatchInfo& p, int x, int y, int z) {
    const int half = (p.sz >> 1) * (p.n[2] + 2);
    return p.off + split_colour(p, x, y, z) * half + (x >> 1) + (p.sy >> 1) * y +
           (p.sz >> 1) * z;
}
// Interior cell id of a box: its own split index and those of its six face
// neighbours (x-, x+, y-, y+, z-, z+; all of the other colour, so they share
// the other half's base and the neighbour's x >> 1, y and z).
__host__ __device__ inline void split_stencil(const PatchInfo& p, const int id[3], int& own,
                                              int nb[6]) {
    const int x = id[0] + 1, y = id[1] + 1, z = id[2] + 1;
    const int col = split_colour(p, x, y, z);
    const int half = (p.sz >> 1) * (p.n[2] + 2);
    const int R = p.sy >> 1, RZ = p.sz >> 1;
    const int row = R * y + RZ * z;
    own = p.off + col * half + (x >> 1) + row;
    const int ob = p.off + (1 - col) * half + row;
    nb[0] = ob + ((x - 1) >> 1);
    nb[1] = ob + ((x + 1) >> 1);
    nb[2] = ob + (x >> 1) - R;
    nb[3] = ob + (x >> 1) + R;
    nb[4] = ob + (x >> 1) - RZ;
    nb[5] = ob + (x >> 1) + RZ;
}

// Damping of the point Jacobi level smoother: 2d / (2d + 1) for d = 3, the
// weight that damps the upper half of the 7-point Laplacian's spectrum best.
constexpr double kJacobiOmega = 6.0 / 7.0;

// Per multigrid grid: box table, face coefficients, field length (kernel
// argument of the merged bottom-solve setup).
template <typename PT>
struct BottomGrids {
    const PatchInfo* P[kMaxMG] = {};
    const PT* D[kMaxMG] = {};
    int64_t nl[kMaxMG] = {};
    const PT* T0 = nullptr;     // grid 0's T in PT when its D_T arrays are not stored
};

template <typename PT>
struct PcArrays {
    const Dev* D = nullptr;
    PT* Dface = nullptr;        // 6 * nl: (field * 3 + d) * nl
    PT* sigma = nullptr;        // nl
    PT* Tp = nullptr;           // nl: T in PT (written by the snapshot when split0)
    PT* e = nullptr;            // 2 * nl each
    PT* u = nullptr;
    PT* r = nullptr;
    PT* f = nullptr;
    PT* shadow = nullptr;       // 2 * shadow_len
    const int32_t* shadow_src = nullptr;
    const ShadowPatch* shadows = nullptr;
    int64_t shadow_len = 0;
    struct MGArr {
        int G = 0;
        const PatchInfo* box[kMaxMG] = {};
        int64_t len[kMaxMG] = {};
        const Tile* tiles[kMaxMG] = {};
        int ntiles[kMaxMG] = {};
        const int32_t* box_of[kMaxMG] = {};
        const Tile* smooth_tiles[kMaxMG] = {};
        int nsmooth[kMaxMG] = {};
        const int32_t* bottom_probs[kMaxMG] = {};
        const int32_t* bottom_boxes[kMaxMG] = {};
        int nbottom[kMaxMG] = {};
        const int64_t* bottom_off = nullptr;
        double* Lbuf = nullptr;
        double* Xbuf = nullptr;
        // first grid: per native cell, the level-0 patch of its children
        // (a base grid cut into several boxes); multi0: level 0 has siblings
        const int32_t* l0map = nullptr;
        bool multi0 = false;
        // all problems with their coarsest grid (one setup launch)
        const int32_t* bot_probs = nullptr;
        const int32_t* bot_boxes = nullptr;
        const int32_t* bot_grid = nullptr;
        int nbot_all = 0;
        PT* Dg[kMaxMG] = {};
        PT* eg[kMaxMG] = {};
        PT* fg[kMaxMG] = {};
    } mg;
    int p2_mode = 0;
    int nu_pre = 1, nu_post = 1;
    int fac_pre = 1, fac_post = 0;   // FAC V(m, n)
    int fac_smoother = 0;            // NRD_SMOOTH_RBGS, _JACOBI or _LINE
    const Tile* ltiles = nullptr;    // x-line tiles (block Gauss-Seidel), by level
    int32_t level_line0[kMaxLev + 1] = {};
    bool base_smooth = false;        // base level: level sweeps instead of multigrid
    bool split0 = false;             // level-0 e and f in colour-split storage
    int fac_cycle = 0;               // NRD_FAC_MULT (Alg. 1) or NRD_FAC_AFACX
    PT* e2 = nullptr;                // 2 * nl: damped Jacobi with several sweeps,
                                     // line smoother, AFACx coarse approximations
    Clock* clock = nullptr;     // times the base grid's sweeps

    void zero(hipStream_t s) const;
    void setup(hipStream_t s, const double* u_state) const;
    // y = P^-1 (wsc_p w); wsc (per problem, may be NULL) scales the input as
    // it is read
    void apply(hipStream_t s, const double* w, double* y, const double* wsc = nullptr) const;
    void apply_transpose(hipStream_t s, const double* w, double* y) const;
    const PT* fac(hipStream_t s) const;     // returns u or e (one level)
    const PT* afacx(hipStream_t s) const;   // returns e
    const PT* p1(hipStream_t s) const;      // the configured cycle
    void vcycle(hipStream_t s) const;
    void composite_residual(hipStream_t s, int lev) const;
    void smooth_level(hipStream_t s, const PT* rhs, int lev, int sweeps) const;
    void correct_level(hipStream_t s, int lev) const;
    void fill_ghosts(hipStream_t s, PT* x) const;
    void restrict_(hipStream_t s, PT* x, int lev_lo) const;
    // sibling ghosts of levels lev .. lev_hi (lev_hi < 0: lev only)
    void siblings(hipStream_t s, PT* x, int lev, int lev_hi = -1) const;
    // red-black sweeps from x = 0 on A^l x = rhs over levels lo .. hi at once
    // (their patches are independent); region: only covered cells relax,
    // every other cell is set to 0
    void smooth_range(hipStream_t s, const PT* rhs, PT* x, int lo, int hi, int sweeps,
                      bool region) const;
};

}  // namespace nrd
