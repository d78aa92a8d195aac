// Internal types shared by the host table builder, the HIP kernels and the
// solver drivers.  Not part of the ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nrd.h"

namespace nrd {

// Device patch table entry.  A patch's fields live in ghosted blocks of
// (n0+2)(n1+2)(n2+2) values, x fastest, starting at `off` within a field.
struct alignas(16) PatchInfo {
    int32_t off;
    int32_t n[3];
    int32_t sy, sz;          // strides of y and z in the ghosted block
    int32_t lo[3];           // box lo in level index space
    int32_t prob;
    int32_t level;
    int32_t phys;            // bit f = 2d+s: face f lies on the domain boundary
    int32_t robin;           // bit f: E is a Marshak face there
    int32_t flags;           // PF_* below
    double h[3];
    double ih[3];            // 1 / h
    double vol;              // cell volume
    int32_t ncell;           // interior cells
    int32_t pad[3];
};

enum : int32_t {
    PF_CTYPE = 1,            // ctype bytes must be consulted (covered cells,
                             // coarse-fine faces or non-physical patch faces)
    PF_COVERED = 2,          // some interior cells are covered
};

// ctype byte per native cell.
//   interior: bit 0 covered; bit (f+1) face f borders a covered cell
//             (its flux is supplied by flux matching)
//   ghost:    kind: 0 physical, 1 sibling copy, 2 coarse-fine
enum : uint8_t { CT_COVERED = 1 };
enum : uint8_t { GK_PHYS = 0, GK_SIB = 1, GK_CF = 2 };

// A run of interior cells of one patch (x fastest, linear interior index).
struct Tile {
    int32_t patch;
    int32_t start;
    int32_t count;
    int32_t prob;
};

// Plane-marching tile: cells [s0, s0 + cnt) of the (x fastest) linear index
// of one z-plane of a patch, for the planes k0 <= k < k1; one workgroup of
// 256 threads, thread t owns linear index s0 + t.
struct STile {
    int32_t patch, prob;
    int32_t s0, cnt, k0, k1;
    int32_t pad[2];
};

struct GhostCopy { int32_t dst, src; };
struct GhostCF   { int32_t dst, src[5]; };    // 4 coarse (9,3,3,1)/16, fine
struct SyncEntry { int32_t dst, src, sy, sz; };  // src: child (0,0,0)
// One coarse face bordering a finer level: coarse cell c, its face f, the
// four fine cells on the far side and the offset from a fine cell to its
// ghost (which lies inside c).  up = 1 if the face is c's high face.
struct RefluxFace {
    int32_t c;
    int32_t face;            // 2d + s of the coarse cell
    int32_t fine[4];
    int32_t gofs;            // ghost = fine + gofs
    int32_t fpatch;
};
// Coarse cells with refluxed faces, CSR into RefluxFace.
struct RefluxCell { int32_t c, first, count, prob; };
// Transposed coarse-fine interpolation: the coarse cells that feed
// coarse-fine ghosts, CSR into the ghosts they feed with the tangential
// weight (9, 3, 3 or 1) of the bilinear stencil.
struct CFRow { int32_t c, first, count, prob; };
struct CFSrc { int32_t ghost, w; };

// Prolongation source buffers: level m patch p owns a "shadow" block of
// the coarser level over its coarsened box grown by one cell.
struct ShadowPatch { int32_t off, m0, m1, m2; };   // shadow extents (with halo)

// Refinement criteria of the tag kernel (a threshold <= 0 switches one off).
struct TagCrit {
    double grad;             // |grad E| / E
    double tau_g, tau_c;     // the paper's gradient and curvature indicators
    int32_t z_interface;     // a face neighbour of another material
    int32_t pad;
};

// Transfer between hierarchies: a box (level index space) whose cells a
// destination patch takes from a source patch of the same level, cut into
// launch chunks of consecutive cells (x fastest within the box).
struct XferFrag { int32_t dpatch, spatch, lo[3], n[3]; };
struct XferChunk { int32_t frag, start, count; };

struct ProbScalars {         // device per-problem constants of a step
    double dt, c0, beta, alpha;
    double kappa, lam;
    double R[6];
};

// Per-problem multigrid grid (single box) below level 0.
struct MGLevel {
    std::vector<PatchInfo> boxes;   // one per problem that has this grid
    std::vector<int32_t> probs;
    int64_t len = 0;                // ghosted cells
    std::vector<Tile> tiles;
};

struct HostBox { int32_t prob, level, lo[3], hi[3]; };

struct Locator {
    int32_t N[3] = {0, 0, 0};
    int32_t B = 8;
    int32_t nb[3] = {0, 0, 0};
    std::vector<std::vector<int32_t>> buckets;
    const std::vector<HostBox>* boxes = nullptr;
    void build(const std::vector<HostBox>& all, const std::vector<int32_t>& ids,
               const int32_t N_[3]);
    int32_t find(int32_t i, int32_t j, int32_t k) const;
};

struct Tables {
    int32_t nprob = 0, nbox = 0, nlev = 0;
    int64_t nl = 0;                  // native cells per field
    int64_t ncells = 0;              // interior cells (all boxes)
    std::vector<nrd_problem> probs;
    std::vector<HostBox> boxes;
    std::vector<PatchInfo> patches;
    std::vector<int64_t> compact_off;        // per box, start in compact field
    std::vector<std::vector<int32_t>> prob_patches;
    std::vector<std::vector<std::vector<int32_t>>> level_patches; // [prob][lev]
    std::vector<uint8_t> ctype;              // nl bytes

    std::vector<Tile> tiles;                 // flat tiles, all patches
    std::vector<STile> stiles;               // plane-marching tiles, by level
    std::vector<int32_t> level_stile0;       // [nlev+1]
    std::vector<int32_t> patch_stile0;       // [nbox+1] bricks of each patch
    std::vector<int32_t> level_tile0;        // [nlev+1] tiles sorted by level
    std::vector<Tile> vtiles;                // reduction tiles
    std::vector<int32_t> prob_vtile0;        // [nprob+1]
    std::vector<std::vector<Tile>> patch_tiles;   // per patch (per-patch launches)

    std::vector<GhostCopy> gcopy;            // sibling copies (physical ghosts are
                                             // never read: no entries)
    std::vector<GhostCF> gcf;
    std::vector<int32_t> level_sib0;         // sibling copies per level: CSR
    std::vector<GhostCopy> sib;              // sibling copies sorted by level
    std::vector<std::vector<SyncEntry>> sync;        // per level (covered cells)
    std::vector<RefluxFace> rfaces;
    std::vector<RefluxCell> rcells;
    std::vector<int32_t> gcf_prob;           // problem of each gcf entry

    // prolongation: per fine patch a shadow block of the coarser level
    std::vector<ShadowPatch> shadow;         // per patch (level >= 1)
    std::vector<int32_t> shadow_src;         // per shadow cell: native index
    int64_t shadow_len = 0;
    std::vector<int32_t> level_shadow0;      // shadow cells per level (CSR)

    // base multigrid below level 0
    std::vector<MGLevel> mg;                 // grid g = 1..; grid 0 = level 0
    std::vector<int32_t> prob_mgdepth;       // number of grids below level 0
    int32_t bottom_max = 0;                  // max bottom cells per problem
    std::vector<int32_t> bottom_off;         // per problem, in units of
                                             // cells^2 doubles
};

// Band storage per row of the coarsest-grid Cholesky factor (b + 1).
constexpr int32_t kBottomBand = 26;

// Staged-plane stencil tiles: at most kStageCells cells of a plane per tile
// (one per thread: 256-cell runs keep the kernel at 78 registers and 20 KB of
// LDS, six waves per SIMD, faster than two cells per thread at four), whose
// ghosted-plane slice (the run plus its x / y neighbours) holds at most
// kStageLen values.
constexpr int32_t kStageCells = 256;
constexpr int32_t kStageLen = 512;

// Plane-marching tiles: planes per tile (z chunk) of each patch.
int32_t default_zchunk(const int32_t n[3], int32_t variant);
// Length of the ghosted-plane slice that covers cells [s0, s0 + cnt) of a
// plane of patch p and their x / y neighbours.
int32_t staged_len(const PatchInfo& p, int32_t s0, int32_t cnt);
// run: cells of a plane per tile (256 for the plane kernel, 4 x 63 for
// wave runs, kStageCells for staged planes); max_span > 0 shortens a
// patch's runs until every staged slice fits.  False if none fits.
bool build_planes(Tables& t, const std::vector<int32_t>& kc, int32_t run,
                  int32_t max_span = 0);
// Per-patch runs; patch_planes appends one patch's tiles (false: no run fits).
bool build_planes(Tables& t, const std::vector<int32_t>& kc, const std::vector<int32_t>& run,
                  int32_t max_span);
bool patch_planes(const PatchInfo& p, int32_t b, int32_t kc, int32_t run, int32_t max_span,
                  std::vector<STile>& out);

// Berger-Rigoutsos clustering of tags into new boxes (cluster.cpp).
nrd_status cluster_boxes(const nrd_problem* probs, int32_t nprob, const nrd_box* boxes,
                         int32_t nbox, const uint8_t* tags, const nrd_cluster_opt& co,
                         std::vector<nrd_box>& out, std::string& msg);

// CSR of the transposed coarse-fine interpolation (coarse source cell ->
// the ghosts it feeds, with the tangential weight), at most 4 entries and 4
// rows per gcf entry.
void build_cf_transpose(const Tables& t, std::vector<CFRow>& rows, std::vector<CFSrc>& src);

// Builds all tables; returns NRD_OK or an error with msg set.
nrd_status build_tables(const nrd_problem* probs, int32_t nprob,
                        const nrd_box* boxes, int32_t nbox, int32_t tile_cells,
                        int32_t vtile_cells, Tables& t, std::string& msg);

inline bool can_coarsen(const int32_t n[3]) {
    for (int d = 0; d < 3; ++d)
        if (n[d] % 2 != 0 || n[d] <= 5) return false;
    return true;
}

}  // namespace nrd
