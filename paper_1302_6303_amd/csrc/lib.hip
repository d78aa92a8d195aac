// nrd library: workspace, operators, solver drivers and the C ABI.
//
// The host drives one lock-step inexact Newton / FGMRES iteration over all
// problems of the hierarchy; all vector arithmetic, reductions and small
// per-problem FGMRES updates run on the device.  The host reads back one
// small per-problem array per Krylov iteration (the residual estimates)
// and a few per Newton iteration (norms, positivity minima).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>
#include <string>
#include <vector>

#include "kernels.h"
#include "precond.h"

using namespace nrd;

namespace {

thread_local std::string g_err;

nrd_status fail(nrd_status st, const std::string& m) {
    g_err = m;
    return st;
}

#define HIPCHK(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess)                                                       \
            return fail(NRD_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define RCHK(x)                        \
    do {                               \
        nrd_status r_ = (x);           \
        if (r_ != NRD_OK) return r_;   \
    } while (0)

// Partial sums of nrd_dot_noalloc: a fixed device array instead of workspace
// memory, one per GPU for the life of the process.  Host code never uses
// the symbol itself (in host code it is not the device address); it uses the
// address resolved per device by scratch_ptr().
constexpr int32_t kScratchTiles = 32768;
static __device__ __align__(256) double scratch[kScratchTiles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, resolved once per device.
hipError_t scratch_ptr(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

struct Bump {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    }
};

}  // namespace

struct nrd_hierarchy final : public Clock {
    Tables t;
    nrd_options opt;
    hipStream_t stream = nullptr;
    int m = 30;                     // Krylov dimension
    bool bound = false;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Dev D;
    PcArrays<float> pcf;
    PcArrays<double> pcd;
    bool mixed = false;
    bool cf_built = false;          // transposed coarse-fine table uploaded
    std::vector<int32_t> patch_tile0;

    // workspace offsets
    struct Off {
        size_t patches, tiles, stiles, vtiles, prob_vtile0, gcopy, gcf, sib, sync[kMaxLev], rfaces,
            rcells, cfrows, cfsrc, ctype, shadows, shadow_src, coff, ps, active, amap;
        size_t mg_box[kMaxMG], mg_tiles[kMaxMG], mg_box_of[kMaxMG], mg_smooth[kMaxMG],
            mg_bprobs[kMaxMG], mg_bboxes[kMaxMG], bot_probs, bot_boxes, bot_grid, bottom_off,
            Lbuf, Xbuf, mg_l0map, ltiles;
        size_t z, z3, cur, prev, udot, bvec, x, F, s, w, tmp, tmp2, gzn, V, Z, pred;
        size_t pc_D, pc_sigma, pc_T, pc_e, pc_e2, pc_u, pc_r, pc_f, pc_shadow;
        size_t mg_D[kMaxMG], mg_e[kMaxMG], mg_f[kMaxMG];
        size_t partial, dots, h1, h2, hn2, H, cs, sn, g, rho, vscale, y, kdim, coefA, coefB,
            minout, flag, ckpt, fdF, fdw, fdsum;
    } o;
    int32_t adjoint_slots = 0;
    size_t stile_cap = 0;           // plane tiles the workspace holds (tuning scratch incl.)
    bool fields_set = false;
    // host-side per-problem state
    std::vector<double> dt_prev;   // 0: no history (next step BDF1)
    std::vector<double> c0, alpha, beta, dt_cur;
    std::vector<ProbScalars> ps_host;
    bool step_ready = false;
    bool last_valid = false;        // bvec / c0 / alpha / dt_cur hold the last
                                    // accepted step's system
    bool resolve_ready = false;     // a transfer brought that system here
    bool skip_estimate = false;     // next step: no error estimate (regrid)
    // device pointers
    double *z, *z3, *cur, *prev, *udot, *bvec, *x, *F, *s, *w, *tmp, *tmp2, *gzn, *V, *Z, *pred;
    std::vector<double> err_prev;   // per problem: last error norm (-1: none)
    double *partial, *dots, *h1, *h2, *hn2, *H, *cs, *sn, *g, *rho, *vscale, *y, *coefA, *coefB,
        *minout, *ckpt, *fdF, *fdw, *fdsum;
    const double* fd_base = nullptr;   // F at the Newton iterate (Jacobian-free mode)
    int32_t *kdim, *flag, *active;
    int32_t* amap;                  // stencil tiles of the active problems
    std::vector<int32_t> host_amap;
    ProbScalars* ps;
    double* scratch = nullptr;      // device address of the fixed partial-sum array
    // timers
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct Timed {
        int which;
        std::pair<hipEvent_t, hipEvent_t> ev;
        int64_t cells;               // composite cells the launches covered
    };
    std::vector<Timed> ev_pairs;
    std::vector<int64_t> prob_comp;  // composite cells per problem
    std::vector<int32_t> host_active;
    // one FGMRES iteration per direction (0: J, 1: J^T), linearisation
    // point (the iterate's buffer rotates with the time-step history) and
    // Krylov index, captured on first use when use_graph is set
    std::map<std::tuple<int, const void*, int>, hipGraphExec_t> graphs;
    hipStream_t cap_stream = nullptr;  // graphs are captured here (the
                                       // library stream may be the legacy
                                       // null stream) and replayed on the
                                       // library stream
    void drop_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }

    int64_t nl2() const { return 2 * t.nl; }
    // stencil launch ranges for the selected variant
    int ntiles_stencil() const {
        return D.bricks ? D.level_stile0[D.nlev] : D.level_tile0[D.nlev];
    }
    void tile_range(int b, int& a0, int& n0) const {
        if (D.bricks) {
            a0 = t.patch_stile0[b];
            n0 = t.patch_stile0[b + 1] - a0;
        } else {
            a0 = patch_tile0[b];
            n0 = (int)t.patch_tiles[b].size();
        }
    }
    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }

    hipEvent_t ev() {
        if (ev_used == ev_pool.size()) {
            hipEvent_t e;
            (void)hipEventCreate(&e);
            ev_pool.push_back(e);
        }
        return ev_pool[ev_used++];
    }
    std::pair<hipEvent_t, hipEvent_t> tic(int which) override {
        if (!timing) return {nullptr, nullptr};
        hipEvent_t a = ev(), b = ev();
        (void)hipEventRecord(a, stream);
        return {a, b};
    }
    void toc(int which, std::pair<hipEvent_t, hipEvent_t> p) override {
        toc_cells(which, p, 0);
    }
    void toc_cells(int which, std::pair<hipEvent_t, hipEvent_t> p, int64_t cells) {
        if (!timing || !p.first) return;
        (void)hipEventRecord(p.second, stream);
        ev_pairs.push_back({which, p, cells});
    }
    // composite cells of the problems an operator launch covers now
    int64_t covered_cells() const {
        int64_t n = 0;
        for (size_t q = 0; q < prob_comp.size(); ++q)
            if (!D.active || host_active[q]) n += prob_comp[q];
        return n;
    }
};

// ---------------------------------------------------------------------------
// layout
// ---------------------------------------------------------------------------

static void layout(nrd_hierarchy* h) {
    Tables& t = h->t;
    Bump b;
    auto& o = h->o;
    const int64_t nl = t.nl;
    const int nprob = t.nprob;
    const int m = h->m;
    o.patches = b.take(sizeof(PatchInfo) * t.patches.size());
    o.tiles = b.take(sizeof(Tile) * std::max<size_t>(1, t.tiles.size()));
    // room for the current plane tiles plus any candidate shape the tuner
    // times (at least one plane and 64 cells per tile)
    size_t cap = t.stiles.size();
    for (const PatchInfo& p : t.patches)
        cap += (size_t)p.n[2] * (size_t)((p.n[0] * p.n[1] + 63) / 64);
    h->stile_cap = std::max<size_t>(1, cap);
    o.stiles = b.take(sizeof(STile) * h->stile_cap);
    o.vtiles = b.take(sizeof(Tile) * std::max<size_t>(1, t.vtiles.size()));
    o.prob_vtile0 = b.take(sizeof(int32_t) * t.prob_vtile0.size());
    o.gcopy = b.take(sizeof(GhostCopy) * std::max<size_t>(1, t.gcopy.size()));
    o.gcf = b.take(sizeof(GhostCF) * std::max<size_t>(1, t.gcf.size()));
    o.sib = b.take(sizeof(GhostCopy) * std::max<size_t>(1, t.sib.size()));
    for (int l = 0; l < t.nlev; ++l)
        o.sync[l] = b.take(sizeof(SyncEntry) * std::max<size_t>(1, t.sync[l].size()));
    o.rfaces = b.take(sizeof(RefluxFace) * std::max<size_t>(1, t.rfaces.size()));
    o.rcells = b.take(sizeof(RefluxCell) * std::max<size_t>(1, t.rcells.size()));
    // transposed coarse-fine interpolation, built on the first transposed
    // product: at most 4 sources and 4 rows per coarse-fine ghost
    o.cfrows = b.take(sizeof(CFRow) * std::max<size_t>(1, 4 * t.gcf.size()));
    o.cfsrc = b.take(sizeof(CFSrc) * std::max<size_t>(1, 4 * t.gcf.size()));
    o.ctype = b.take(t.ctype.size());
    o.shadows = b.take(sizeof(ShadowPatch) * t.shadow.size());
    o.shadow_src = b.take(sizeof(int32_t) * std::max<int64_t>(1, t.shadow_len));
    o.coff = b.take(sizeof(int64_t) * t.compact_off.size());
    o.ps = b.take(sizeof(ProbScalars) * nprob);
    o.active = b.take(sizeof(int32_t) * nprob);
    o.amap = b.take(sizeof(int32_t) * std::max(h->stile_cap, std::max<size_t>(1, t.tiles.size())));
    const int G = (int)t.mg.size() - 1;
    for (int g = 0; g <= G; ++g) {
        if (g >= 1) {
            o.mg_box[g] = b.take(sizeof(PatchInfo) * t.mg[g].boxes.size());
            o.mg_tiles[g] = b.take(sizeof(Tile) * std::max<size_t>(1, t.mg[g].tiles.size()));
        }
        o.mg_box_of[g] = b.take(sizeof(int32_t) * nprob);
        o.mg_smooth[g] = b.take(sizeof(Tile) * (t.tiles.size() + 1));
        o.mg_bprobs[g] = b.take(sizeof(int32_t) * nprob);
        o.mg_bboxes[g] = b.take(sizeof(int32_t) * nprob);
    }
    // per native cell of the first multigrid grid: the level-0 patch that
    // holds its eight children
    o.mg_l0map = b.take(sizeof(int32_t) * std::max<int64_t>(1, G >= 1 ? t.mg[1].len : 1));
    o.bot_probs = b.take(sizeof(int32_t) * nprob);
    o.bot_boxes = b.take(sizeof(int32_t) * nprob);
    o.bot_grid = b.take(sizeof(int32_t) * nprob);
    o.bottom_off = b.take(sizeof(int64_t) * nprob);
    int64_t bsum = 0;
    for (int p = 0; p < nprob; ++p) {
        int64_t nb = 1;
        for (int d = 0; d < 3; ++d) nb *= t.probs[p].base_n[d] >> t.prob_mgdepth[p];
        bsum += nb * nb;
    }
    o.Lbuf = b.take(8);
    o.Xbuf = b.take(sizeof(double) * 2 * bsum);
    // state and work vectors (double)
    o.z = b.take(8 * nl);
    o.z3 = b.take(8 * nl);
    o.cur = b.take(8 * 2 * nl);
    o.prev = b.take(8 * 2 * nl);
    o.udot = b.take(8 * 2 * nl);
    o.bvec = b.take(8 * 2 * nl);
    o.x = b.take(8 * 2 * nl);
    o.F = b.take(8 * 2 * nl);
    o.s = b.take(8 * 2 * nl);
    o.w = b.take(8 * 2 * nl);
    o.tmp = b.take(8 * 2 * nl);
    o.tmp2 = b.take(8 * 2 * nl);
    o.gzn = b.take(8 * nl);
    o.V = b.take(8 * 2 * nl * (size_t)(m + 1));
    o.Z = b.take(8 * 2 * nl * (size_t)m);
    o.pred = b.take(h->opt.error_estimate ? 8 * 2 * nl : 8);
    // preconditioner (float or double)
    const size_t es = h->mixed ? 4 : 8;
    o.pc_D = b.take(es * 6 * nl);
    o.pc_sigma = b.take(es * nl);
    o.pc_T = b.take(es * nl);
    o.pc_e = b.take(es * 2 * nl);
    o.pc_e2 = b.take(h->opt.fac_smoother != NRD_SMOOTH_RBGS || h->opt.fac_cycle == NRD_FAC_AFACX
                         ? es * 2 * nl
                         : es);
    // x-line tiles of the block Gauss-Seidel smoother (lines of each patch in
    // runs of kBlock lines), by level
    {
        size_t nlt = 0;
        for (const PatchInfo& pi : t.patches) nlt += (pi.n[1] * pi.n[2] + kBlock - 1) / kBlock;
        o.ltiles = b.take(sizeof(Tile) * std::max<size_t>(1, nlt));
    }
    o.pc_u = b.take(es * 2 * nl);
    o.pc_r = b.take(es * 2 * nl);
    o.pc_f = b.take(es * 2 * nl);
    o.pc_shadow = b.take(es * 2 * std::max<int64_t>(1, t.shadow_len));
    for (int g = 1; g <= G; ++g) {
        const int64_t n = t.mg[g].len;
        o.mg_D[g] = b.take(es * 6 * n);
        o.mg_e[g] = b.take(es * 2 * n);
        o.mg_f[g] = b.take(es * 2 * n);
    }
    // reductions and per-problem scalars
    o.partial = b.take(8 * 16 * std::max<size_t>(1, t.vtiles.size()));
    o.dots = b.take(8 * nprob * (m + 2));
    o.h1 = b.take(8 * nprob * (m + 1));
    o.h2 = b.take(8 * nprob * (m + 1));
    o.hn2 = b.take(8 * nprob);
    o.H = b.take(8 * (size_t)nprob * (m + 1) * m);
    o.cs = b.take(8 * nprob * m);
    o.sn = b.take(8 * nprob * m);
    o.g = b.take(8 * nprob * (m + 1));
    o.rho = b.take(8 * nprob);
    o.vscale = b.take(8 * nprob);
    o.y = b.take(8 * nprob * m);
    o.kdim = b.take(4 * nprob);
    o.coefA = b.take(8 * nprob * 4);
    o.coefB = b.take(8 * nprob * 4);
    o.minout = b.take(8 * nprob);
    o.flag = b.take(4 * 4);
    o.ckpt = b.take(8 * 2 * nl * (size_t)std::max(0, h->adjoint_slots));
    const bool fd = h->opt.jvp_mode == NRD_JVP_FD;
    o.fdF = b.take(fd ? 8 * 2 * nl : 8);
    o.fdw = b.take(fd ? 8 * 2 * nl : 8);
    o.fdsum = b.take(8 * 3 * nprob);
    h->ws_bytes = b.off;
}

template <typename T>
static hipError_t up(hipStream_t s, void* dst, const std::vector<T>& v) {
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s);
}

// Colour-split storage of the level-0 V-cycle vectors (split0): problems
// of one level and one level-0 box, even x extents, a multigrid base.  The
// index map is checked here for every box shape: a bijection of the ghosted
// block onto itself, and each interior cell's stencil indices those of its
// neighbours' positions.
static bool split0_ok(const Tables& t, bool base_smooth) {
    if (base_smooth || t.nlev != 1 || t.level_sib0[1] != t.level_sib0[0]) return false;
    std::map<std::tuple<int, int, int, int, int, int>, bool> shapes;
    for (const PatchInfo& p : t.patches) {
        if ((p.n[0] & 1) || (p.sy & 1) || p.sy != p.n[0] + 2) return false;
        shapes[std::make_tuple(p.n[0], p.n[1], p.n[2], p.sy, p.sz,
                               (p.lo[0] + p.lo[1] + p.lo[2]) & 1)] = true;
    }
    // shapes already checked in this process (hierarchies are often rebuilt
    // with the same boxes)
    static std::mutex checked_mu;
    static std::map<std::tuple<int, int, int, int, int, int>, bool> checked;
    for (const auto& kv : shapes) {
        {
            std::lock_guard<std::mutex> lk(checked_mu);
            if (checked.count(kv.first)) continue;
        }
        PatchInfo q;
        std::memset(&q, 0, sizeof(q));
        std::tie(q.n[0], q.n[1], q.n[2], q.sy, q.sz, q.lo[0]) = kv.first;
        const int64_t vol = (int64_t)q.sz * (q.n[2] + 2);
        std::vector<char> seen(vol, 0);
        for (int z = 0; z < q.n[2] + 2; ++z)
            for (int y = 0; y < q.n[1] + 2; ++y)
                for (int x = 0; x < q.sy; ++x) {
                    const int i = split_index(q, x, y, z);
                    if (i < 0 || i >= vol || seen[i]) return false;
                    seen[i] = 1;
                }
        for (int k = 0; k < q.n[2]; ++k)
            for (int j = 0; j < q.n[1]; ++j)
                for (int i = 0; i < q.n[0]; ++i) {
                    const int id[3] = {i, j, k};
                    int own, nb[6];
                    split_stencil(q, id, own, nb);
                    const int x = i + 1, y = j + 1, z = k + 1;
                    if (own != split_index(q, x, y, z) || nb[0] != split_index(q, x - 1, y, z) ||
                        nb[1] != split_index(q, x + 1, y, z) ||
                        nb[2] != split_index(q, x, y - 1, z) ||
                        nb[3] != split_index(q, x, y + 1, z) ||
                        nb[4] != split_index(q, x, y, z - 1) ||
                        nb[5] != split_index(q, x, y, z + 1))
                        return false;
                }
        std::lock_guard<std::mutex> lk(checked_mu);
        checked[kv.first] = true;
    }
    return true;
}

template <typename PT>
static void wire_pc(nrd_hierarchy* h, PcArrays<PT>& pc) {
    auto& o = h->o;
    Tables& t = h->t;
    pc.D = &h->D;
    pc.Dface = h->at<PT>(o.pc_D);
    pc.sigma = h->at<PT>(o.pc_sigma);
    pc.Tp = h->at<PT>(o.pc_T);
    pc.e = h->at<PT>(o.pc_e);
    pc.e2 = h->at<PT>(o.pc_e2);
    pc.u = h->at<PT>(o.pc_u);
    pc.r = h->at<PT>(o.pc_r);
    pc.f = h->at<PT>(o.pc_f);
    pc.shadow = h->at<PT>(o.pc_shadow);
    pc.shadow_src = h->at<int32_t>(o.shadow_src);
    pc.shadows = h->at<ShadowPatch>(o.shadows);
    pc.shadow_len = std::max<int64_t>(1, t.shadow_len);
    const int G = (int)t.mg.size() - 1;
    pc.mg.G = G;
    for (int g = 0; g <= G; ++g) {
        if (g >= 1) {
            pc.mg.box[g] = h->at<PatchInfo>(o.mg_box[g]);
            pc.mg.len[g] = t.mg[g].len;
            pc.mg.tiles[g] = h->at<Tile>(o.mg_tiles[g]);
            pc.mg.ntiles[g] = (int)t.mg[g].tiles.size();
            pc.mg.Dg[g] = h->at<PT>(o.mg_D[g]);
            pc.mg.eg[g] = h->at<PT>(o.mg_e[g]);
            pc.mg.fg[g] = h->at<PT>(o.mg_f[g]);
        }
        pc.mg.box_of[g] = h->at<int32_t>(o.mg_box_of[g]);
        pc.mg.smooth_tiles[g] = h->at<Tile>(o.mg_smooth[g]);
        pc.mg.bottom_probs[g] = h->at<int32_t>(o.mg_bprobs[g]);
        pc.mg.bottom_boxes[g] = h->at<int32_t>(o.mg_bboxes[g]);
    }
    pc.mg.l0map = G >= 1 ? h->at<int32_t>(o.mg_l0map) : nullptr;
    pc.ltiles = h->at<Tile>(o.ltiles);
    pc.mg.multi0 = t.level_sib0[1] > t.level_sib0[0];
    pc.mg.bottom_off = h->at<int64_t>(o.bottom_off);
    pc.mg.bot_probs = h->at<int32_t>(o.bot_probs);
    pc.mg.bot_boxes = h->at<int32_t>(o.bot_boxes);
    pc.mg.bot_grid = h->at<int32_t>(o.bot_grid);
    pc.mg.nbot_all = t.nprob;
    pc.mg.Lbuf = h->at<double>(o.Lbuf);
    pc.mg.Xbuf = h->at<double>(o.Xbuf);
    pc.p2_mode = h->opt.p2_mode;
    pc.nu_pre = std::max(1, h->opt.mg_nu_pre);
    pc.nu_post = std::max(0, h->opt.mg_nu_post);
    pc.fac_pre = h->opt.fac_nu_pre;
    pc.fac_post = h->opt.fac_nu_post;
    pc.fac_smoother = h->opt.fac_smoother;
    pc.base_smooth = h->opt.fac_base == NRD_BASE_SMOOTH;
    pc.split0 = split0_ok(t, pc.base_smooth);
    pc.fac_cycle = h->opt.fac_cycle;
    pc.clock = h;
}

static nrd_status bind(nrd_hierarchy* h, void* ptr, size_t bytes) {
    if (bytes < h->ws_bytes) return fail(NRD_EINVAL, "workspace too small");
    if (reinterpret_cast<uintptr_t>(ptr) % 256) return fail(NRD_EINVAL, "workspace not 256-byte aligned");
    // the fixed partial-sum array of nrd_dot_noalloc, on the device of this
    // workspace (the current device)
    HIPCHK(scratch_ptr(&h->scratch));
    h->ws = static_cast<char*>(ptr);
    Tables& t = h->t;
    auto& o = h->o;
    hipStream_t s = h->stream;
    // zero everything once: ghosts of work vectors stay finite
    fill_native(s, reinterpret_cast<double*>(h->ws), (int64_t)(h->ws_bytes / 8), 0.0);
    HIPCHK(up(s, h->ws + o.patches, t.patches));
    HIPCHK(up(s, h->ws + o.tiles, t.tiles));
    HIPCHK(up(s, h->ws + o.stiles, t.stiles));
    HIPCHK(up(s, h->ws + o.vtiles, t.vtiles));
    HIPCHK(up(s, h->ws + o.prob_vtile0, t.prob_vtile0));
    HIPCHK(up(s, h->ws + o.gcopy, t.gcopy));
    HIPCHK(up(s, h->ws + o.gcf, t.gcf));
    HIPCHK(up(s, h->ws + o.sib, t.sib));
    for (int l = 0; l < t.nlev; ++l) HIPCHK(up(s, h->ws + o.sync[l], t.sync[l]));
    HIPCHK(up(s, h->ws + o.rfaces, t.rfaces));
    HIPCHK(up(s, h->ws + o.rcells, t.rcells));
    HIPCHK(up(s, h->ws + o.ctype, t.ctype));
    HIPCHK(up(s, h->ws + o.shadows, t.shadow));
    HIPCHK(up(s, h->ws + o.shadow_src, t.shadow_src));
    HIPCHK(up(s, h->ws + o.coff, t.compact_off));
    // multigrid tables
    const int G = (int)t.mg.size() - 1;
    std::vector<std::vector<int32_t>> box_of(G + 1, std::vector<int32_t>(t.nprob, -1));
    for (int p = 0; p < t.nprob; ++p) box_of[0][p] = t.level_patches[p][0][0];
    for (int g = 1; g <= G; ++g)
        for (size_t i = 0; i < t.mg[g].probs.size(); ++i) box_of[g][t.mg[g].probs[i]] = (int32_t)i;
    std::vector<int32_t> nsmooth(G + 1, 0), nbottom(G + 1, 0);
    for (int g = 0; g <= G; ++g) {
        if (g >= 1) {
            HIPCHK(up(s, h->ws + o.mg_box[g], t.mg[g].boxes));
            HIPCHK(up(s, h->ws + o.mg_tiles[g], t.mg[g].tiles));
        }
        HIPCHK(up(s, h->ws + o.mg_box_of[g], box_of[g]));
        std::vector<Tile> sm;
        if (g == 0) {
            for (int i = t.level_tile0[0]; i < t.level_tile0[1]; ++i)
                if (t.prob_mgdepth[t.tiles[i].prob] > 0) sm.push_back(t.tiles[i]);
        } else {
            for (const Tile& tl : t.mg[g].tiles)
                if (t.prob_mgdepth[tl.prob] > g) sm.push_back(tl);
        }
        nsmooth[g] = (int)sm.size();
        HIPCHK(up(s, h->ws + o.mg_smooth[g], sm));
        std::vector<int32_t> bp, bb;
        for (int p = 0; p < t.nprob; ++p)
            if (t.prob_mgdepth[p] == g) {
                bp.push_back(p);
                bb.push_back(box_of[g][p]);
            }
        nbottom[g] = (int)bp.size();
        HIPCHK(up(s, h->ws + o.mg_bprobs[g], bp));
        HIPCHK(up(s, h->ws + o.mg_bboxes[g], bb));
    }
    {
        std::vector<Tile> lt;
        std::vector<int32_t> l0(t.nlev + 1, 0);
        for (int l = 0; l < t.nlev; ++l) {
            l0[l] = (int32_t)lt.size();
            for (int b = 0; b < t.nbox; ++b) {
                const PatchInfo& pi = t.patches[b];
                if (pi.level != l) continue;
                const int32_t nlines = pi.n[1] * pi.n[2];
                for (int32_t a = 0; a < nlines; a += kBlock)
                    lt.push_back({b, a, std::min(kBlock, nlines - a), pi.prob});
            }
        }
        l0[t.nlev] = (int32_t)lt.size();
        HIPCHK(up(s, h->ws + o.ltiles, lt));
        for (int l = 0; l <= t.nlev; ++l) {
            h->pcf.level_line0[l] = l0[l];
            h->pcd.level_line0[l] = l0[l];
        }
    }
    if (G >= 1) {
        // children of every first-grid cell: one level-0 patch (level-0 boxes
        // of a tiled base start and end on even planes)
        const MGLevel& M = t.mg[1];
        std::vector<int32_t> l0(M.len, -1);
        for (size_t i = 0; i < M.boxes.size(); ++i) {
            const PatchInfo& g1 = M.boxes[i];
            const int p = M.probs[i];
            for (int32_t b : t.level_patches[p][0]) {
                const HostBox& x = t.boxes[b];
                int32_t lo[3], hi[3];
                for (int d = 0; d < 3; ++d) {
                    lo[d] = x.lo[d] / 2;
                    hi[d] = (x.hi[d] + 1) / 2;
                }
                for (int k = lo[2]; k < hi[2]; ++k)
                    for (int j = lo[1]; j < hi[1]; ++j)
                        for (int ii = lo[0]; ii < hi[0]; ++ii)
                            l0[g1.off + (ii + 1) + (int64_t)g1.sy * (j + 1) +
                               (int64_t)g1.sz * (k + 1)] = b;
            }
        }
        HIPCHK(up(s, h->ws + o.mg_l0map, l0));
    }
    std::vector<int64_t> boff(t.nprob);
    for (int p = 0; p < t.nprob; ++p) boff[p] = t.bottom_off[p];
    HIPCHK(up(s, h->ws + o.bottom_off, boff));
    std::vector<int32_t> bpa, bba, bga;
    for (int g = 0; g <= G; ++g)
        for (int p = 0; p < t.nprob; ++p)
            if (t.prob_mgdepth[p] == g) {
                bpa.push_back(p);
                bba.push_back(box_of[g][p]);
                bga.push_back(g);
            }
    HIPCHK(up(s, h->ws + o.bot_probs, bpa));
    HIPCHK(up(s, h->ws + o.bot_boxes, bba));
    HIPCHK(up(s, h->ws + o.bot_grid, bga));
    // device views
    Dev& D = h->D;
    D.nl = t.nl;
    D.nprob = t.nprob;
    D.nlev = t.nlev;
    D.nbox = t.nbox;
    D.patches = h->at<PatchInfo>(o.patches);
    D.tiles = h->at<Tile>(o.tiles);
    for (int l = 0; l <= t.nlev; ++l) D.level_tile0[l] = t.level_tile0[l];
    D.stiles = h->at<STile>(o.stiles);
    D.bricks = h->opt.stencil;
    for (int l = 0; l <= t.nlev; ++l) D.level_stile0[l] = t.level_stile0[l];
    D.vtiles = h->at<Tile>(o.vtiles);
    D.nvtiles = (int32_t)t.vtiles.size();
    D.prob_vtile0 = h->at<int32_t>(o.prob_vtile0);
    D.gcopy = h->at<GhostCopy>(o.gcopy);
    D.ncopy = (int32_t)t.gcopy.size();
    D.gcf = h->at<GhostCF>(o.gcf);
    D.ncf = (int32_t)t.gcf.size();
    D.sib = h->at<GhostCopy>(o.sib);
    for (int l = 0; l <= t.nlev; ++l) D.level_sib0[l] = t.level_sib0[l];
    for (int l = 0; l <= t.nlev; ++l) D.level_shadow0[l] = t.level_shadow0[l];
    for (int l = 0; l < t.nlev; ++l) {
        D.sync[l] = h->at<SyncEntry>(o.sync[l]);
        D.nsync[l] = (int32_t)t.sync[l].size();
    }
    D.rfaces = h->at<RefluxFace>(o.rfaces);
    D.rcells = h->at<RefluxCell>(o.rcells);
    D.nrcells = (int32_t)t.rcells.size();
    D.cfrows = h->at<CFRow>(o.cfrows);
    D.cfsrc = h->at<CFSrc>(o.cfsrc);
    D.ncfrows = 0;                 // set by ensure_cf_transpose
    h->cf_built = false;
    D.ctype = h->at<uint8_t>(o.ctype);
    D.ps = h->at<ProbScalars>(o.ps);
    D.active = nullptr;
    D.z3 = h->at<double>(o.z3);
    D.z = h->at<double>(o.z);
    h->ps = h->at<ProbScalars>(o.ps);
    h->active = h->at<int32_t>(o.active);
    h->amap = h->at<int32_t>(o.amap);
    h->z = h->at<double>(o.z);
    h->z3 = h->at<double>(o.z3);
    h->cur = h->at<double>(o.cur);
    h->prev = h->at<double>(o.prev);
    h->udot = h->at<double>(o.udot);
    h->bvec = h->at<double>(o.bvec);
    h->x = h->at<double>(o.x);
    h->F = h->at<double>(o.F);
    h->s = h->at<double>(o.s);
    h->w = h->at<double>(o.w);
    h->tmp = h->at<double>(o.tmp);
    h->tmp2 = h->at<double>(o.tmp2);
    h->gzn = h->at<double>(o.gzn);
    h->V = h->at<double>(o.V);
    h->Z = h->at<double>(o.Z);
    h->pred = h->at<double>(o.pred);
    h->err_prev.assign(t.nprob, -1.0);
    h->partial = h->at<double>(o.partial);
    h->dots = h->at<double>(o.dots);
    h->h1 = h->at<double>(o.h1);
    h->h2 = h->at<double>(o.h2);
    h->hn2 = h->at<double>(o.hn2);
    h->H = h->at<double>(o.H);
    h->cs = h->at<double>(o.cs);
    h->sn = h->at<double>(o.sn);
    h->g = h->at<double>(o.g);
    h->rho = h->at<double>(o.rho);
    h->vscale = h->at<double>(o.vscale);
    h->y = h->at<double>(o.y);
    h->kdim = h->at<int32_t>(o.kdim);
    h->coefA = h->at<double>(o.coefA);
    h->coefB = h->at<double>(o.coefB);
    h->minout = h->at<double>(o.minout);
    h->flag = h->at<int32_t>(o.flag);
    h->ckpt = h->at<double>(o.ckpt);
    h->fdF = h->at<double>(o.fdF);
    h->fdw = h->at<double>(o.fdw);
    h->fdsum = h->at<double>(o.fdsum);
    if (h->mixed) {
        wire_pc(h, h->pcf);
        for (int g = 0; g <= G; ++g) {
            h->pcf.mg.nsmooth[g] = nsmooth[g];
            h->pcf.mg.nbottom[g] = nbottom[g];
        }
    } else {
        wire_pc(h, h->pcd);
        for (int g = 0; g <= G; ++g) {
            h->pcd.mg.nsmooth[g] = nsmooth[g];
            h->pcd.mg.nbottom[g] = nbottom[g];
        }
    }
    h->host_active.assign(t.nprob, 1);
    HIPCHK(up(s, h->active, h->host_active));
    // per-problem constants (valid before the first begin_step)
    h->ps_host.assign(t.nprob, ProbScalars());
    for (int p = 0; p < t.nprob; ++p) {
        ProbScalars& q = h->ps_host[p];
        std::memset(&q, 0, sizeof(q));
        q.dt = 0.0;
        q.c0 = 1.0;
        q.beta = 0.0;
        q.kappa = t.probs[p].kappa;
        q.lam = h->opt.limiter;
        for (int f = 0; f < 6; ++f) q.R[f] = t.probs[p].robin_R[f];
    }
    HIPCHK(up(s, h->ps, h->ps_host));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    h->bound = true;
    return NRD_OK;
}

// ---------------------------------------------------------------------------
// operators on native vectors
// ---------------------------------------------------------------------------

static void prepare_state(nrd_hierarchy* h, double* u) {
    restrict_d(h->D, h->stream, u, 2, 0);
    ghost_fill_d(h->D, h->stream, u, 2);
}

static void op_residual(nrd_hierarchy* h, double* u, double* F, bool prepared = false) {
    if (!prepared) prepare_state(h, u);
    const int64_t cells = h->timing ? h->covered_cells() : 0;
    auto tk = h->tic(NRD_TIMER_RESIDUAL);
    const Dev& D = h->D;
    if (h->opt.launch == NRD_PER_PATCH) {
        for (int b = 0; b < h->t.nbox; ++b) {
            int a0, n0;
            h->tile_range(b, a0, n0);
            residual(D, h->stream, a0, n0, u, h->bvec, F);
        }
    } else {
        residual_all(D, h->stream, u, h->bvec, F);
    }
    residual_reflux(D, h->stream, u, F);
    h->toc_cells(NRD_TIMER_RESIDUAL, tk, cells);
}

// Jacobian-free product (Sec. 4.1): Jv = (F(u + eps v) - F(u)) / eps with the
// per-problem step of the Sec. 4.1 formula.  F0 = F(u) if the caller has it
// (the Newton residual at the iterate), else it is evaluated here.
static void op_jvp_fd(nrd_hierarchy* h, double* u, double* v, double* Jv, bool u_prepared,
                      const double* F0) {
    if (!u_prepared) prepare_state(h, u);
    restrict_d(h->D, h->stream, v, 2, 0);
    const int64_t cells = h->timing ? h->covered_cells() : 0;
    auto tk = h->tic(NRD_TIMER_JVP);
    const Dev& D = h->D;
    hipStream_t s = h->stream;
    if (!F0) {
        if (h->opt.launch == NRD_PER_PATCH) {
            for (int b = 0; b < h->t.nbox; ++b) {
                int a0, n0;
                h->tile_range(b, a0, n0);
                residual(D, s, a0, n0, u, h->bvec, h->fdF);
            }
        } else {
            residual_all(D, s, u, h->bvec, h->fdF);
        }
        residual_reflux(D, s, u, h->fdF);
        F0 = h->fdF;
    }
    fd_sums(D, s, u, v, h->partial, h->fdsum);
    fd_shift(D, s, h->fdsum, u, v, h->fdw);
    prepare_state(h, h->fdw);
    if (h->opt.launch == NRD_PER_PATCH) {
        for (int b = 0; b < h->t.nbox; ++b) {
            int a0, n0;
            h->tile_range(b, a0, n0);
            residual(D, s, a0, n0, h->fdw, h->bvec, Jv);
        }
    } else {
        residual_all(D, s, h->fdw, h->bvec, Jv);
    }
    residual_reflux(D, s, h->fdw, Jv);
    fd_quotient(D, s, h->fdsum, F0, Jv);
    h->toc_cells(NRD_TIMER_JVP, tk, cells);
}

static void op_jvp(nrd_hierarchy* h, double* u, double* v, double* Jv, bool u_prepared) {
    if (h->opt.jvp_mode == NRD_JVP_FD) {
        op_jvp_fd(h, u, v, Jv, u_prepared, h->fd_base);
        return;
    }
    if (!u_prepared) prepare_state(h, u);
    prepare_state(h, v);
    const int64_t cells = h->timing ? h->covered_cells() : 0;
    auto tk = h->tic(NRD_TIMER_JVP);
    const Dev& D = h->D;
    if (h->opt.launch == NRD_PER_PATCH) {
        for (int b = 0; b < h->t.nbox; ++b) {
            int a0, n0;
            h->tile_range(b, a0, n0);
            jvp(D, h->stream, a0, n0, u, v, Jv);
        }
    } else {
        jvp_all(D, h->stream, u, v, Jv);
    }
    jvp_reflux(D, h->stream, u, v, Jv);
    h->toc_cells(NRD_TIMER_JVP, tk, cells);
}

static void pc_setup(nrd_hierarchy* h, double* u, bool prepared) {
    if (!prepared) prepare_state(h, u);
    if (h->mixed)
        h->pcf.setup(h->stream, u);
    else
        h->pcd.setup(h->stream, u);
}

static void pc_apply(nrd_hierarchy* h, const double* w, double* y,
                     const double* wsc = nullptr) {
    auto tk = h->tic(NRD_TIMER_PRECOND);
    if (h->mixed)
        h->pcf.apply(h->stream, w, y, wsc);
    else
        h->pcd.apply(h->stream, w, y, wsc);
    h->toc(NRD_TIMER_PRECOND, tk);
}

static void pc_apply_t(nrd_hierarchy* h, const double* w, double* y) {
    if (h->mixed)
        h->pcf.apply_transpose(h->stream, w, y);
    else
        h->pcd.apply_transpose(h->stream, w, y);
}

// Sends the active flags to the device together with the list of stencil
// tiles of the flagged problems, so masked residual and Jacobian launches
// have no workgroups for finished problems (captured graphs keep reading the
// flags: their launch sizes are fixed).
static nrd_status upload_active(nrd_hierarchy* h) {
    HIPCHK(hipMemcpyAsync(h->active, h->host_active.data(), 4 * h->t.nprob,
                          hipMemcpyHostToDevice, h->stream));
    h->D.amap = nullptr;
    h->D.namap = 0;
    if (h->opt.use_graph) return NRD_OK;
    const Tables& t = h->t;
    auto& m = h->host_amap;
    m.clear();
    if (h->D.bricks) {
        for (int32_t i = 0; i < (int32_t)t.stiles.size(); ++i)
            if (h->host_active[t.stiles[i].prob]) m.push_back(i);
    } else {
        for (int32_t i = 0; i < (int32_t)t.tiles.size(); ++i)
            if (h->host_active[t.tiles[i].prob]) m.push_back(i);
    }
    if (!m.empty())
        HIPCHK(hipMemcpyAsync(h->amap, m.data(), 4 * m.size(), hipMemcpyHostToDevice,
                              h->stream));
    h->D.amap = h->amap;
    h->D.namap = (int32_t)m.size();
    return NRD_OK;
}

// masked: only the problems of the current active mask (0 for the others)
static nrd_status dot_host(nrd_hierarchy* h, const double* x, const double* y,
                           std::vector<double>& out, bool masked = false) {
    if (!masked) h->D.active = nullptr;
    multidot(h->D, h->stream, x, 0, 1, y, h->partial, h->dots);
    out.resize(h->t.nprob);
    HIPCHK(hipMemcpyAsync(out.data(), h->dots, 8 * h->t.nprob, hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return NRD_OK;
}

// ---------------------------------------------------------------------------
// BDF coefficients and history combination (eqs. be, bdf2)
// ---------------------------------------------------------------------------

static nrd_status begin_step(nrd_hierarchy* h, const double* dt, bool bdf1_only = false) {
    Tables& t = h->t;
    const int np = t.nprob;
    h->c0.assign(np, 1.0);
    h->alpha.assign(np, 0.0);
    h->beta.assign(np, 0.0);
    h->dt_cur.assign(dt, dt + np);
    std::vector<double> a(np), b(np), one(np, 1.0);
    for (int p = 0; p < np; ++p) {
        if (!(dt[p] > 0.0)) return fail(NRD_EINVAL, "dt must be positive");
        const bool first = !(h->dt_prev[p] > 0.0) || bdf1_only;
        double c0 = 1.0, al = 0.0;
        if (!first) {
            al = dt[p] / h->dt_prev[p];
            c0 = (1.0 + 2.0 * al) / (1.0 + al);
        }
        h->c0[p] = c0;
        h->alpha[p] = al;
        h->beta[p] = dt[p] / c0;
        h->ps_host[p].dt = dt[p];
        h->ps_host[p].c0 = c0;
        h->ps_host[p].alpha = al;
        h->ps_host[p].beta = dt[p] / c0;
        a[p] = first ? 1.0 : 1.0 + al;
        b[p] = first ? 0.0 : -al * al / (1.0 + al);
    }
    hipStream_t s = h->stream;
    HIPCHK(up(s, h->ps, h->ps_host));
    // b = a u_n + b u_{n-1}
    std::vector<double> coef(2 * np);
    for (int p = 0; p < np; ++p) {
        coef[p] = a[p];
        coef[np + p] = b[p];
    }
    HIPCHK(up(s, h->coefA, coef));
    h->D.active = nullptr;
    lincomb2(h->D, s, h->coefA, h->cur, h->coefA + np, h->prev, h->bvec);
    HIPCHK(hipStreamSynchronize(s));
    h->step_ready = true;
    return NRD_OK;
}

// ---------------------------------------------------------------------------
// FGMRES(m), lock-step over the problems with host_active set
// ---------------------------------------------------------------------------

struct GmresOut {
    std::vector<int32_t> its;
};

// Solves J s = rhs (rhs native, s native) for active problems with absolute
// tolerances tol[p].  transpose: use the transposed operators.
// b2_first: ||rhs||^2 per problem if the caller has it (saves that pass).
// pending: if given and the solve ends within its first cycle, sol is not
// formed: *pending returns each problem's Krylov dimension and the caller
// applies the correction Z y (h->Z, h->y) itself; otherwise *pending is
// returned empty and sol holds the solution.
static nrd_status fgmres(nrd_hierarchy* h, double* u, const double* rhs, double* sol,
                         const std::vector<double>& tol, std::vector<int32_t>& its,
                         bool transpose, const std::vector<double>* b2_first = nullptr,
                         std::vector<int32_t>* pending = nullptr) {
    Tables& t = h->t;
    const int np = t.nprob;
    const int m = h->m;
    const int64_t NL = h->nl2();
    hipStream_t s = h->stream;
    std::vector<int32_t> outer = h->host_active;           // problems asked to solve
    its.assign(np, 0);
    std::vector<double> beta0(np), rho(np), inv(np);
    std::vector<int32_t> kd(np);
    if (pending) pending->clear();
    bool sol_set = false;        // sol holds the corrections of earlier cycles
    std::vector<int32_t> todo = outer;
    for (int cycle = 0; cycle <= h->opt.gmres_maxrestarts; ++cycle) {
        // r = rhs - A sol  (first cycle: rhs)
        // r = rhs on the first cycle (read in place), else rhs - A sol in w
        const double* r = rhs;
        h->host_active = todo;
        RCHK(upload_active(h));
        h->D.active = h->active;
        if (cycle > 0) {
            r = h->w;
            copy_interior(h->D, s, sol, h->tmp2);
            if (!transpose) {
                op_jvp(h, u, h->tmp2, h->tmp, true);
            } else {
                vjp_full(h->D, s, u, h->tmp2, h->tmp, h->gzn);
            }
            copy_interior(h->D, s, rhs, h->w);
            std::vector<double> mone(np, -1.0), pone(np, 1.0);
            HIPCHK(up(s, h->coefA, mone));
            HIPCHK(up(s, h->coefB, pone));
            axpby(h->D, s, h->coefA, h->tmp, h->coefB, h->w);
        }
        std::vector<double> b2;
        if (cycle == 0 && b2_first) {
            b2 = *b2_first;
        } else {
            multidot(h->D, s, r, 0, 1, r, h->partial, h->dots);
            b2.resize(np);
            HIPCHK(hipMemcpyAsync(b2.data(), h->dots, 8 * np, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        bool any = false;
        for (int p = 0; p < np; ++p) {
            if (!todo[p]) continue;
            beta0[p] = std::sqrt(std::max(0.0, b2[p]));
            if (beta0[p] <= tol[p]) {
                todo[p] = 0;
                continue;
            }
            inv[p] = 1.0 / beta0[p];
            any = true;
        }
        if (!any) break;
        h->host_active = todo;
        RCHK(upload_active(h));
        HIPCHK(up(s, h->coefA, inv));
        // v_0 = r / beta.  On a forward solve's first cycle r (the right-hand
        // side) stays untouched, so iteration 0 reads r scaled by 1/beta
        // (coefA) in place of v_0 and v_0 is formed only if iteration 1 runs.
        const bool v0_lazy = cycle == 0 && !transpose;
        if (!v0_lazy) scale_copy(h->D, s, r, h->coefA, h->V);
        std::vector<double> g0((size_t)np * (m + 1), 0.0);
        for (int p = 0; p < np; ++p) g0[(size_t)p * (m + 1)] = beta0[p];
        HIPCHK(up(s, h->g, g0));
        std::vector<int32_t> live = todo;
        for (int p = 0; p < np; ++p) kd[p] = 0;
        for (int j = 0; j < m; ++j) {
            // one iteration: v_j = w / ||w|| (the previous iteration's w,
            // scaled only now that another iteration is needed), z_j =
            // P^-1 v_j, w = J z_j, CGS2 against v_0..v_j, Hessenberg column +
            // Givens.  Everything it reads that changes between calls (active
            // mask, scalars, the preconditioner snapshot) is device-resident,
            // so it can be captured once per j and replayed.
            auto iteration = [&]() {
                double* Vj = h->V + j * NL;
                double* Zj = h->Z + j * NL;
                double* wv = h->w;
                if (j > 0) scale_copy(h->D, s, wv, h->vscale, Vj);
                if (j == 1 && v0_lazy) scale_copy(h->D, s, r, h->coefA, h->V);
                // the basis read by this iteration: v_0 .. v_j, or r with 1/beta
                const double* Vb = (j == 0 && v0_lazy) ? r : h->V;
                const double* vsc = (j == 0 && v0_lazy) ? h->coefA : nullptr;
                if (!transpose) {
                    pc_apply(h, (j == 0 && v0_lazy) ? r : Vj, Zj, vsc);
                    op_jvp(h, u, Zj, wv, true);
                } else {
                    pc_apply_t(h, Vj, Zj);
                    vjp_full(h->D, s, u, Zj, wv, h->gzn);
                }
                multidot(h->D, s, Vb, NL, j + 1, wv, h->partial, h->h1, vsc);
                combine_dot(h->D, s, Vb, NL, j + 1, h->h1, j + 1, wv, h->partial, h->h2, vsc);
                combine_norm(h->D, s, Vb, NL, j + 1, h->h2, j + 1, wv, h->partial, h->hn2,
                             vsc);
                gmres_column(s, np, m, j, h->active, h->h1, h->h2, h->hn2, h->H, h->cs, h->sn,
                             h->g, h->rho, h->vscale);
            };
            if (h->opt.use_graph) {
                hipGraphExec_t& ge = h->graphs[std::make_tuple(
                    (transpose ? 1 : 0) + (v0_lazy ? 2 : 0), (const void*)u, j)];
                if (!h->cap_stream) {
                    HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
                }
                if (!ge) {
                    const bool timing = h->timing;
                    h->timing = false;             // no event records inside a graph
                    hipStream_t user = s;
                    hipGraph_t graph = nullptr;
                    hipError_t ec = hipStreamBeginCapture(h->cap_stream,
                                                          hipStreamCaptureModeThreadLocal);
                    if (ec == hipSuccess) {
                        s = h->stream = h->cap_stream;
                        iteration();
                        ec = hipStreamEndCapture(s, &graph);
                        s = h->stream = user;
                    }
                    h->timing = timing;
                    HIPCHK(ec);
                    const hipError_t ei = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(graph);
                    HIPCHK(ei);
                }
                // captured on its own stream, replayed on the library stream
                HIPCHK(hipGraphLaunch(ge, s));
            } else {
                iteration();
            }
            std::vector<double> hn(np);
            HIPCHK(hipMemcpyAsync(rho.data(), h->rho, 8 * np, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(hn.data(), h->hn2, 8 * np, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            bool left = false;
            for (int p = 0; p < np; ++p) {
                if (!live[p]) continue;
                its[p] += 1;
                kd[p] = j + 1;
                if (rho[p] <= tol[p] || hn[p] == 0.0) {
                    live[p] = 0;
                    todo[p] = 0;
                } else {
                    left = true;
                }
            }
            if (!left) break;
            h->host_active = live;
            RCHK(upload_active(h));
        }
        // sol += Z y for every problem that iterated in this cycle
        std::vector<int32_t> did(np, 0);
        for (int p = 0; p < np; ++p) did[p] = kd[p] > 0;
        h->host_active = did;
        RCHK(upload_active(h));
        HIPCHK(up(s, h->kdim, kd));
        gmres_backsolve(s, np, m, h->kdim, h->H, h->g, h->y);
        int kmax = *std::max_element(kd.begin(), kd.end());
        bool rem = false;
        for (int p = 0; p < np; ++p) rem |= todo[p] != 0;
        if (kmax > 0) {
            if (!sol_set && !rem && pending) {
                *pending = kd;               // the caller applies Z y
                break;
            }
            if (!sol_set) {
                // first correction: problems that did not iterate get sol = 0,
                // the others sol = Z y (write-only passes)
                std::vector<int32_t> idle(np, 0);
                bool any_idle = false;
                for (int p = 0; p < np; ++p) {
                    idle[p] = outer[p] && !did[p];
                    any_idle |= idle[p] != 0;
                }
                if (any_idle) {
                    h->host_active = idle;
                    RCHK(upload_active(h));
                    combine(h->D, s, nullptr, 0, 0, h->coefA, 0, sol, 0, 1.0);
                    h->host_active = did;
                    RCHK(upload_active(h));
                }
                combine(h->D, s, h->Z, NL, kmax, h->y, m, sol, 0, 1.0);
                sol_set = true;
            } else {
                combine(h->D, s, h->Z, NL, kmax, h->y, m, sol, 1, 1.0);
            }
        }
        if (!rem) break;
    }
    const bool deferred = pending && !pending->empty();
    if (!sol_set && !deferred) {
        // no correction at all: sol = 0 for every problem asked to solve
        h->host_active = outer;
        RCHK(upload_active(h));
        h->D.active = h->active;
        combine(h->D, s, nullptr, 0, 0, h->coefA, 0, sol, 0, 1.0);
    }
    h->host_active = outer;
    RCHK(upload_active(h));
    HIPCHK(hipStreamSynchronize(s));
    return NRD_OK;
}

// ---------------------------------------------------------------------------
// inexact Newton (lock-step), positivity by step halving
// ---------------------------------------------------------------------------

static nrd_status newton(nrd_hierarchy* h, std::vector<nrd_step_stats>& st) {
    Tables& t = h->t;
    const int np = t.nprob;
    hipStream_t s = h->stream;
    const nrd_options& O = h->opt;
    st.assign(np, nrd_step_stats());
    for (auto& x : st) std::memset(&x, 0, sizeof(x));
    h->host_active.assign(np, 1);
    RCHK(upload_active(h));
    h->D.active = nullptr;
    op_residual(h, h->x, h->F);
    std::vector<double> f2;
    nrd_status rc = dot_host(h, h->F, h->F, f2);
    if (rc) return rc;
    // forcing terms (Eisenstat-Walker): Kelley's choice, or PETSc's choice 2
    const bool petsc = O.newton_forcing == NRD_EW_PETSC;
    const double gamma = petsc ? 1.0 : 0.9, eta_max = 0.9;
    const double ew_a = petsc ? 0.5 * (1.0 + std::sqrt(5.0)) : 2.0;
    std::vector<double> fn(np), fn_old(np), stop(np), eta(np, petsc ? 0.3 : 0.9), tol(np);
    std::vector<int32_t> done(np, 0), failed(np, 0);
    for (int p = 0; p < np; ++p) {
        fn[p] = std::sqrt(f2[p]);
        st[p].fnorm0 = fn[p];
        stop[p] = std::max(O.newton_rtol * fn[p], O.newton_atol);
        fn_old[p] = fn[p];
    }
    for (int k = 0;; ++k) {
        bool any = false;
        for (int p = 0; p < np; ++p) {
            if (done[p] || failed[p]) continue;
            if (!(fn[p] == fn[p])) {
                failed[p] = 1;
                continue;
            }
            if (fn[p] <= stop[p]) {
                done[p] = 1;
                continue;
            }
            if (st[p].newton_iters >= O.newton_maxit) {
                failed[p] = 1;
                continue;
            }
            any = true;
            if (k > 0) {
                const double rat = fn[p] / fn_old[p];
                double en, sg;
                if (petsc) {
                    en = gamma * std::pow(rat, ew_a);
                    sg = gamma * std::pow(eta[p], ew_a);
                } else {
                    en = gamma * rat * rat;
                    sg = gamma * eta[p] * eta[p];
                }
                if (sg > 0.1) en = std::max(en, sg);
                eta[p] = std::min(en, eta_max);
                eta[p] = std::max(eta[p], 0.5 * stop[p] / fn[p]);
            }
            tol[p] = eta[p] * fn[p];
        }
        if (!any) break;
        for (int p = 0; p < np; ++p) h->host_active[p] = !(done[p] || failed[p]);
        RCHK(upload_active(h));
        h->D.active = h->active;              // snapshot only the problems still iterating
        pc_setup(h, h->x, true);              // x was prepared by the residual
        // s = J^-1 F; the Newton step is -s
        h->D.active = h->active;
        std::vector<int32_t> its, pend;
        h->fd_base = h->F;                    // F(x) for Jacobian-free products
        rc = fgmres(h, h->x, h->F, h->s, tol, its, false, &f2, &pend);
        h->fd_base = nullptr;
        if (rc) return rc;
        std::vector<int32_t> act = h->host_active;
        for (int p = 0; p < np; ++p)
            if (act[p]) {
                if (st[p].newton_iters < 24) st[p].krylov_per_newton[st[p].newton_iters] = its[p];
                st[p].krylov_iters += its[p];
            }
        // positivity: halve lambda until E, T > 0 on composite cells
        std::vector<double> lam(np, 1.0), mn(np);
        std::vector<int32_t> ok(np, 0), moved(np, 0);
        for (int p = 0; p < np; ++p) ok[p] = !act[p];
        std::vector<double> mlam(np);
        int cut0 = 0;
        if (!pend.empty()) {
            // the full step -s = -Z y from one FGMRES cycle: applied in place
            // together with its positivity check (the iterate kept in tmp);
            // problems whose step fails go back to the iterate and continue
            // with half the step below
            const int m = h->m;
            const int64_t NL = h->nl2();
            std::vector<int32_t> did(np, 0), bad(np, 0);
            int kmax = 0;
            for (int p = 0; p < np; ++p) {
                did[p] = act[p] && pend[p] > 0;
                kmax = std::max(kmax, did[p] ? pend[p] : 0);
            }
            h->host_active = did;
            RCHK(upload_active(h));
            h->D.active = h->active;
            update_min(h->D, s, h->Z, NL, kmax, h->y, m, h->x, h->tmp, h->partial, h->minout);
            HIPCHK(hipMemcpyAsync(mn.data(), h->minout, 8 * np, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            bool any_bad = false;
            for (int p = 0; p < np; ++p) {
                if (!act[p]) continue;
                if (!did[p] || mn[p] > 0.0) {     // no step (F = 0) or accepted
                    ok[p] = 1;
                    moved[p] = did[p];
                } else {
                    bad[p] = 1;
                    any_bad = true;
                    lam[p] = 0.5;
                    st[p].positivity_cuts += 1;
                }
            }
            if (any_bad) {
                h->host_active = bad;
                RCHK(upload_active(h));
                copy_interior(h->D, s, h->tmp, h->x);
                combine(h->D, s, h->Z, NL, kmax, h->y, m, h->s, 0, 1.0);
            }
            cut0 = 1;
        }
        for (int cut = cut0; cut <= 30; ++cut) {
            // only problems still searching need a pass
            bool searching = false;
            for (int p = 0; p < np; ++p) {
                h->host_active[p] = act[p] && !ok[p] && !failed[p];
                searching |= h->host_active[p] != 0;
            }
            if (!searching) break;
            RCHK(upload_active(h));
            for (int p = 0; p < np; ++p) mlam[p] = -lam[p];      // step = -lam s
            HIPCHK(up(s, h->coefA, mlam));
            h->D.active = h->active;
            min_positive(h->D, s, h->x, h->s, h->coefA, h->partial, h->minout);
            HIPCHK(hipMemcpyAsync(mn.data(), h->minout, 8 * np, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (int p = 0; p < np; ++p) {
                if (!h->host_active[p]) continue;
                if (mn[p] > 0.0) {
                    ok[p] = 1;
                    continue;
                }
                st[p].positivity_cuts += 1;       // every rejected trial step
                if (cut < 30)
                    lam[p] *= 0.5;
                else
                    failed[p] = 1;
            }
        }
        bool step = false;
        for (int p = 0; p < np; ++p) {
            h->host_active[p] = act[p] && !failed[p] && !moved[p];
            step |= h->host_active[p] != 0;
        }
        if (step) {
            RCHK(upload_active(h));
            std::vector<double> one(np, 1.0);
            for (int p = 0; p < np; ++p) mlam[p] = -lam[p];
            HIPCHK(up(s, h->coefA, mlam));
            HIPCHK(up(s, h->coefB, one));
            h->D.active = h->active;
            axpby(h->D, s, h->coefA, h->s, h->coefB, h->x);
        }
        // F and its norm only where x changed (problems still iterating)
        for (int p = 0; p < np; ++p) h->host_active[p] = act[p] && !failed[p];
        RCHK(upload_active(h));
        h->D.active = h->active;
        op_residual(h, h->x, h->F);
        rc = dot_host(h, h->F, h->F, f2, true);
        h->D.active = nullptr;
        if (rc) return rc;
        for (int p = 0; p < np; ++p) {
            if (!act[p] || failed[p]) continue;   // iterations count accepted updates
            fn_old[p] = fn[p];
            fn[p] = std::sqrt(f2[p]);
            st[p].newton_iters += 1;
        }
    }
    bool all_ok = true;
    for (int p = 0; p < np; ++p) {
        st[p].fnorm = fn[p];
        st[p].converged = done[p] && !failed[p];
        all_ok &= st[p].converged != 0;
    }
    h->host_active.assign(np, 1);
    RCHK(upload_active(h));
    h->D.active = nullptr;
    return all_ok ? NRD_OK : NRD_ENOTCONV;
}

static nrd_status implicit_step(nrd_hierarchy* h, const double* dt, nrd_step_stats* stats,
                                bool bdf1_only = false) {
    Tables& t = h->t;
    const int np = t.nprob;
    hipStream_t s = h->stream;
    h->last_valid = false;
    nrd_status rc = begin_step(h, dt, bdf1_only);
    if (rc) return rc;
    // initial guess: leapfrog predictor (BDF2 steps) if positive, else u_n
    h->D.active = nullptr;
    bool any2 = false;
    for (int p = 0; p < np; ++p) any2 |= h->alpha[p] > 0.0;
    if (!any2) {
        copy_interior(h->D, s, h->cur, h->x);
    } else {
        // x = (1 - a^2) u_n + (1 + a) dt u'_n + a^2 u_{n-1}; problems taking a
        // BDF1 step have all three coefficients 0 and get x = u_n
        std::vector<double> buf(3 * np);
        for (int p = 0; p < np; ++p) {
            const double a = h->alpha[p];
            const bool bdf2 = a > 0.0;
            buf[p] = bdf2 ? (1.0 + a) * dt[p] : 0.0;
            buf[np + p] = bdf2 ? a * a : 0.0;
            buf[2 * np + p] = bdf2 ? -a * a : 0.0;
        }
        HIPCHK(up(s, h->coefA, buf));
        // written straight into the Newton iterate, with its copy for the
        // error estimate
        bdf2_predict(h->D, s, h->coefA, h->cur, h->udot, h->prev, h->x,
                     h->opt.error_estimate ? h->pred : nullptr);
        // a BDF2 problem whose predictor is not positive starts from u_n
        std::vector<double> zero(np, 0.0), mn(np);
        HIPCHK(up(s, h->coefB, zero));
        min_positive(h->D, s, h->x, h->x, h->coefB, h->partial, h->minout);
        HIPCHK(hipMemcpyAsync(mn.data(), h->minout, 8 * np, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<int32_t> back(np);
        bool any_back = false;
        for (int p = 0; p < np; ++p) {
            back[p] = (h->alpha[p] > 0.0) && !(mn[p] > 0.0);
            any_back |= back[p] != 0;
        }
        if (any_back) {
            h->host_active = back;
            RCHK(upload_active(h));
            h->D.active = h->active;
            copy_interior(h->D, s, h->cur, h->x);
            h->host_active.assign(np, 1);
            RCHK(upload_active(h));
            h->D.active = nullptr;
        }
    }
    std::vector<nrd_step_stats> st;
    rc = newton(h, st);
    for (int p = 0; p < np; ++p) {
        st[p].dt = dt[p];
        st[p].err_norm = -1.0;
    }
    if (rc == NRD_OK && h->opt.error_estimate && any2 && !h->skip_estimate) {
        // local error estimate of the BDF2 steps (eq. bdf2le), scaled max norm
        std::vector<double> cf(np), en(np);
        for (int p = 0; p < np; ++p) {
            const double a = h->alpha[p];
            cf[p] = (a + 1.0) / (3.0 * a + 2.0);
            h->host_active[p] = a > 0.0;
        }
        RCHK(upload_active(h));
        HIPCHK(up(s, h->coefA, cf));
        h->D.active = h->active;
        err_norm(h->D, s, h->x, h->pred, h->coefA, h->opt.err_eta_E, h->opt.err_eta_T,
                 h->partial, h->minout);
        h->D.active = nullptr;
        HIPCHK(hipMemcpyAsync(en.data(), h->minout, 8 * np, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        h->host_active.assign(np, 1);
        RCHK(upload_active(h));
        for (int p = 0; p < np; ++p)
            if (h->alpha[p] > 0.0) st[p].err_norm = en[p];
    }
    if (stats)
        for (int p = 0; p < np; ++p) stats[p] = st[p];
    if (rc) {
        if (rc == NRD_ENOTCONV) g_err = "Newton did not converge; state rolled back";
        return rc;
    }
    // udot = (c0 x - b) / dt ; rotate history
    std::vector<double> buf(2 * np);
    for (int p = 0; p < np; ++p) {
        buf[p] = h->c0[p] / dt[p];
        buf[np + p] = -1.0 / dt[p];
    }
    HIPCHK(up(s, h->coefA, buf));
    lincomb2(h->D, s, h->coefA, h->x, h->coefA + np, h->bvec, h->udot);
    std::swap(h->prev, h->cur);       // prev <- u_n
    std::swap(h->cur, h->x);          // cur <- u_{n+1}
    // keep ghosts/covered of the new state consistent
    prepare_state(h, h->cur);
    for (int p = 0; p < np; ++p) h->dt_prev[p] = bdf1_only ? 0.0 : dt[p];
    HIPCHK(hipStreamSynchronize(s));
    h->step_ready = false;
    h->last_valid = true;
    h->resolve_ready = false;
    h->skip_estimate = false;
    return NRD_OK;
}

// The transposed coarse-fine interpolation table, built and uploaded on the
// first transposed product (forward work never reads it).
static nrd_status ensure_cf_transpose(nrd_hierarchy* h) {
    if (h->cf_built) return NRD_OK;
    std::vector<CFRow> rows;
    std::vector<CFSrc> src;
    build_cf_transpose(h->t, rows, src);
    HIPCHK(up(h->stream, h->ws + h->o.cfrows, rows));
    HIPCHK(up(h->stream, h->ws + h->o.cfsrc, src));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->D.ncfrows = (int32_t)rows.size();
    h->cf_built = true;
    return NRD_OK;
}

// ---------------------------------------------------------------------------
// discrete adjoint of BDF1 steps with checkpoints
// ---------------------------------------------------------------------------

static nrd_status adjoint_run(nrd_hierarchy* h, const double* dt, int nsteps, int every,
                              const double* dJdE, double* gz) {
    Tables& t = h->t;
    const int np = t.nprob;
    hipStream_t s = h->stream;
    const int64_t NL = h->nl2();
    if (nsteps <= 0 || every <= 0) return fail(NRD_EINVAL, "nsteps and ckpt_every must be > 0");
    RCHK(ensure_cf_transpose(h));
    const int nck = (nsteps + every - 1) / every;
    if (nck + every + 3 > h->adjoint_slots)
        return fail(NRD_EINVAL, "workspace reserved too few adjoint slots "
                                "(need ceil(nsteps / ckpt_every) + ckpt_every + 3)");
    // slots: checkpoints | segment states | rhs | lambda | gradient; the
    // forward recomputation (implicit steps) never touches them
    double* ck = h->ckpt;
    double* seg = ck + (size_t)nck * NL;
    double* rhs = seg + (size_t)every * NL;
    double* lam = rhs + NL;
    double* gacc = lam + NL;
    std::vector<double> dtv(dt, dt + np);
    // forward with checkpoints of u_0, u_every, ...
    for (int n = 0; n < nsteps; ++n) {
        if (n % every == 0) copy_interior(h->D, s, h->cur, ck + (size_t)(n / every) * NL);
        nrd_status rc = implicit_step(h, dtv.data(), nullptr, true);
        if (rc) return rc;
    }
    // lambda_N rhs: (dJ/dE, 0) in the composite unknowns.  A covered cell
    // holds the mean of its children, so a weight given to it passes to them
    // (transposed restriction); the default objective counts composite cells.
    fill_native(s, rhs, NL, 0.0);
    if (dJdE) {
        unpack(h->D, s, h->at<int64_t>(h->o.coff), dJdE, rhs, 1, t.ncells);
        restrict_transpose(h->D, s, rhs, 1);
    } else {
        // a compact vector of ones, built on the device in gz (overwritten below)
        fill_native(s, gz, t.ncells, 1.0);
        unpack(h->D, s, h->at<int64_t>(h->o.coff), gz, rhs, 1, t.ncells);
        zero_covered(h->D, s, rhs, 1);
    }
    fill_native(s, lam, NL, 0.0);
    fill_native(s, gacc, NL, 0.0);              // dJ/dz accumulator (field 0)
    for (int p = 0; p < np; ++p) {
        h->ps_host[p].dt = dt[p];
        h->ps_host[p].c0 = 1.0;
        h->ps_host[p].beta = dt[p];
        h->ps_host[p].alpha = 0.0;
    }
    HIPCHK(up(s, h->ps, h->ps_host));
    for (int segi = nck - 1; segi >= 0; --segi) {
        const int n0 = segi * every;
        const int n1 = std::min(nsteps, n0 + every);
        // recompute u_{n0+1..n1} from the checkpoint
        copy_interior(h->D, s, ck + (size_t)segi * NL, h->cur);
        prepare_state(h, h->cur);
        for (int p = 0; p < np; ++p) h->dt_prev[p] = 0.0;
        for (int n = n0; n < n1; ++n) {
            nrd_status rc = implicit_step(h, dtv.data(), nullptr, true);
            if (rc) return rc;
            copy_interior(h->D, s, h->cur, seg + (size_t)(n - n0) * NL);
        }
        for (int p = 0; p < np; ++p) {
            h->ps_host[p].dt = dt[p];
            h->ps_host[p].c0 = 1.0;
            h->ps_host[p].beta = dt[p];
        }
        HIPCHK(up(s, h->ps, h->ps_host));
        for (int n = n1; n > n0; --n) {
            // the linearisation point goes to the Newton iterate's buffer,
            // which the recomputation no longer needs (and which captured
            // Krylov iterations read)
            h->D.active = nullptr;
            copy_interior(h->D, s, seg + (size_t)(n - n0 - 1) * NL, h->x);
            double* un = h->x;
            prepare_state(h, un);
            pc_setup(h, un, true);
            // A_n^T lam = rhs
            std::vector<double> r2;
            nrd_status rc = dot_host(h, rhs, rhs, r2);
            if (rc) return rc;
            std::vector<double> tol(np);
            for (int p = 0; p < np; ++p) tol[p] = 1e-12 * std::sqrt(r2[p]);
            std::vector<int32_t> its;
            h->host_active.assign(np, 1);
            RCHK(upload_active(h));
            rc = fgmres(h, un, rhs, lam, tol, its, true);
            if (rc) return rc;
            // grad -= lam^T dF/dz ; next rhs = lam
            vjp_full(h->D, s, un, lam, h->w, h->gzn);
            std::vector<double> mone(np, -1.0), one(np, 1.0);
            HIPCHK(up(s, h->coefA, mone));
            HIPCHK(up(s, h->coefB, one));
            // gacc (field 0 only used) += -gz : use a 2-field axpby on (gz | scratch)
            {
                // gz is a single field; place it in tmp field 0, zero field 1
                fill_native(s, h->tmp, NL, 0.0);
                HIPCHK(hipMemcpyAsync(h->tmp, h->gzn, 8 * t.nl, hipMemcpyDeviceToDevice, s));
                axpby(h->D, s, h->coefA, h->tmp, h->coefB, gacc);
            }
            copy_interior(h->D, s, lam, rhs);
        }
    }
    pack(h->D, s, h->at<int64_t>(h->o.coff), gacc, gz, 1, t.ncells);
    // the state ends at u_N: recompute it from the last checkpoint
    copy_interior(h->D, s, ck + (size_t)(nck - 1) * NL, h->cur);
    prepare_state(h, h->cur);
    for (int n = (nck - 1) * every; n < nsteps; ++n) {
        nrd_status rc = implicit_step(h, dtv.data(), nullptr, true);
        if (rc) return rc;
    }
    for (int p = 0; p < np; ++p) h->dt_prev[p] = 0.0;
    HIPCHK(hipStreamSynchronize(s));
    return NRD_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* nrd_last_error(void) { return g_err.c_str(); }

void nrd_default_options(nrd_options* o) {
    std::memset(o, 0, sizeof(*o));
    o->precision = NRD_FP64;
    o->launch = NRD_BATCHED;
    o->use_graph = 0;
    o->jvp_mode = NRD_JVP_ANALYTIC;
    o->limiter = 0.5;
    o->p2_mode = NRD_P2_PAPER;
    o->newton_rtol = 1e-8;
    o->newton_atol = 1e-14;
    o->newton_maxit = 20;
    o->gmres_restart = 30;
    o->gmres_maxrestarts = 10;
    o->mg_nu_pre = 1;
    o->mg_nu_post = 1;
    o->fac_nu_pre = 1;
    o->fac_nu_post = 0;
    o->fac_smoother = NRD_SMOOTH_RBGS;
    o->fac_base = NRD_BASE_MG;
    o->fac_cycle = NRD_FAC_MULT;
    o->newton_forcing = NRD_EW_PETSC;
    o->pad_ = 0;
    o->stencil = 3;
    o->bdf_max_order = 2;
    o->error_estimate = 0;
    o->err_eta_E = 1e-5;
    o->err_eta_T = std::pow(1e-5, 0.25);
}

nrd_status nrd_hierarchy_create(const nrd_problem* probs, int32_t nprob, const nrd_box* boxes,
                                int32_t nbox, const nrd_options* opt, void* hip_stream,
                                nrd_hierarchy** out) {
    if (!out) return fail(NRD_EINVAL, "out is NULL");
    try {
        nrd_hierarchy* h = new nrd_hierarchy();
        if (opt)
            h->opt = *opt;
        else
            nrd_default_options(&h->opt);
        if (h->opt.gmres_restart < 1 || h->opt.gmres_restart > 64) {
            delete h;
            return fail(NRD_EINVAL, "gmres_restart must be in [1, 64]");
        }
        if (h->opt.newton_maxit < 1 || h->opt.newton_maxit > 24) {
            delete h;
            return fail(NRD_EINVAL, "newton_maxit must be in [1, 24]");
        }
        if (h->opt.fac_nu_pre < 1 || h->opt.fac_nu_pre > 8 || h->opt.fac_nu_post < 0 ||
            h->opt.fac_nu_post > 8) {
            delete h;
            return fail(NRD_EINVAL, "fac_nu_pre must be in [1, 8], fac_nu_post in [0, 8]");
        }
        if (h->opt.fac_smoother != NRD_SMOOTH_RBGS && h->opt.fac_smoother != NRD_SMOOTH_JACOBI &&
            h->opt.fac_smoother != NRD_SMOOTH_LINE) {
            delete h;
            return fail(NRD_EINVAL, "fac_smoother must be RBGS, JACOBI or LINE");
        }
        if (h->opt.fac_base != NRD_BASE_MG && h->opt.fac_base != NRD_BASE_SMOOTH) {
            delete h;
            return fail(NRD_EINVAL, "fac_base must be MG or SMOOTH");
        }
        if (h->opt.newton_forcing != NRD_EW_KELLEY && h->opt.newton_forcing != NRD_EW_PETSC) {
            delete h;
            return fail(NRD_EINVAL, "newton_forcing must be KELLEY or PETSC");
        }
        if (h->opt.fac_cycle != NRD_FAC_MULT && h->opt.fac_cycle != NRD_FAC_AFACX) {
            delete h;
            return fail(NRD_EINVAL, "fac_cycle must be MULT or AFACX");
        }
        if (h->opt.fac_cycle == NRD_FAC_AFACX &&
            (h->opt.fac_smoother != NRD_SMOOTH_RBGS || h->opt.fac_nu_post != 0)) {
            delete h;
            return fail(NRD_EINVAL, "AFACx needs the red-black smoother and fac_nu_post = 0");
        }
        if (h->opt.bdf_max_order < 1 || h->opt.bdf_max_order > 2) {
            delete h;
            return fail(NRD_EINVAL, "bdf_max_order must be 1 or 2");
        }
        if (h->opt.error_estimate < 0 || h->opt.error_estimate > 1 ||
            !(h->opt.err_eta_E >= 0.0) || !(h->opt.err_eta_T >= 0.0)) {
            delete h;
            return fail(NRD_EINVAL, "error_estimate must be 0 or 1, err_eta_E/T >= 0");
        }
        if (h->opt.jvp_mode != NRD_JVP_ANALYTIC && h->opt.jvp_mode != NRD_JVP_FD) {
            delete h;
            return fail(NRD_EINVAL, "jvp_mode must be ANALYTIC or FD");
        }
        h->m = h->opt.gmres_restart;
        h->mixed = h->opt.precision == NRD_MIXED;
        h->adjoint_slots = std::max(0, h->opt.adjoint_slots);
        h->stream = static_cast<hipStream_t>(hip_stream);
        std::string msg;
        nrd_status rc = build_tables(probs, nprob, boxes, nbox, kBlock, 8 * kBlock, h->t, msg);
        if (rc) {
            delete h;
            return fail(rc, msg);
        }
        if (h->t.nlev > kMaxLev || (int)h->t.mg.size() > kMaxMG) {
            delete h;
            return fail(NRD_EUNSUPPORTED, "too many levels");
        }
        h->prob_comp.assign(h->t.nprob, 0);
        for (const PatchInfo& pi : h->t.patches) {
            int64_t n = pi.ncell;
            if (pi.flags & PF_COVERED)
                for (int k = 0; k < pi.n[2]; ++k)
                    for (int j = 0; j < pi.n[1]; ++j)
                        for (int i = 0; i < pi.n[0]; ++i) {
                            const int64_t c = pi.off + (i + 1) + (int64_t)pi.sy * (j + 1) +
                                              (int64_t)pi.sz * (k + 1);
                            if (h->t.ctype[c] & CT_COVERED) --n;
                        }
            h->prob_comp[pi.prob] += n;
        }
        h->patch_tile0.assign(h->t.nbox, 0);
        {
            // tiles are grouped per patch in level order
            std::vector<int32_t> first(h->t.nbox, -1);
            for (size_t i = 0; i < h->t.tiles.size(); ++i)
                if (first[h->t.tiles[i].patch] < 0) first[h->t.tiles[i].patch] = (int32_t)i;
            h->patch_tile0 = first;
        }
        if (h->opt.stencil >= 1 || h->opt.zchunk > 0) {
            std::vector<int32_t> kc(h->t.nbox);
            for (int b = 0; b < h->t.nbox; ++b)
                kc[b] = h->opt.zchunk > 0 ? h->opt.zchunk
                                          : default_zchunk(h->t.patches[b].n, h->opt.stencil);
            int st = h->opt.stencil;
            bool ok = build_planes(h->t, kc, st == 2 ? 4 * 63 : (st == 3 ? kStageCells : 256),
                                   st == 3 ? kStageLen : 0);
            if (!ok && st == 3) {
                // rows too wide for the staged slices (x extent above about
                // 250): the plane-marching variant, same values, any width
                st = h->opt.stencil = 1;
                for (int b = 0; b < h->t.nbox; ++b)
                    kc[b] = h->opt.zchunk > 0 ? h->opt.zchunk
                                              : default_zchunk(h->t.patches[b].n, st);
                ok = build_planes(h->t, kc, 256, 0);
            }
            if (!ok) {
                delete h;
                return fail(NRD_EUNSUPPORTED, "a patch plane is too wide for the staged stencil");
            }
        }
        if (h->opt.stencil < 0 || h->opt.stencil > 3) {
            delete h;
            return fail(NRD_EINVAL, "stencil must be 0, 1, 2 or 3");
        }
        h->dt_prev.assign(h->t.nprob, 0.0);
        layout(h);
        *out = h;
        return NRD_OK;
    } catch (const std::exception& e) {
        return fail(NRD_EINVAL, e.what());
    }
}

nrd_status nrd_hierarchy_destroy(nrd_hierarchy* h) {
    if (!h) return NRD_OK;
    h->drop_graphs();
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    delete h;
    return NRD_OK;
}

nrd_status nrd_workspace_size(const nrd_hierarchy* h, size_t* bytes) {
    if (!h || !bytes) return fail(NRD_EINVAL, "NULL argument");
    *bytes = h->ws_bytes;
    return NRD_OK;
}

nrd_status nrd_bind_workspace(nrd_hierarchy* h, void* ptr, size_t bytes) {
    if (!h || !ptr) return fail(NRD_EINVAL, "NULL argument");
    return bind(h, ptr, bytes);
}

nrd_status nrd_layout(const nrd_hierarchy* h, int64_t* ncells, int64_t* native_len) {
    if (!h) return fail(NRD_EINVAL, "NULL hierarchy");
    if (ncells) *ncells = h->t.ncells;
    if (native_len) *native_len = h->t.nl;
    return NRD_OK;
}

#define NEED_BOUND(h)                                                        \
    do {                                                                     \
        if (!(h)) return fail(NRD_EINVAL, "NULL hierarchy");                 \
        if (!(h)->bound) return fail(NRD_ESTATE, "no workspace bound");      \
    } while (0)

nrd_status nrd_pack(nrd_hierarchy* h, const double* native, double* compact) {
    NEED_BOUND(h);
    pack(h->D, h->stream, h->at<int64_t>(h->o.coff), native, compact, 2, h->t.ncells);
    HIPCHK(hipGetLastError());
    return NRD_OK;
}

nrd_status nrd_unpack(nrd_hierarchy* h, const double* compact, double* native) {
    NEED_BOUND(h);
    unpack(h->D, h->stream, h->at<int64_t>(h->o.coff), compact, native, 2, h->t.ncells);
    HIPCHK(hipGetLastError());
    return NRD_OK;
}

nrd_status nrd_set_fields(nrd_hierarchy* h, const double* E, const double* T, const double* z) {
    NEED_BOUND(h);
    if (!E || !T || !z) return fail(NRD_EINVAL, "NULL field");
    hipStream_t s = h->stream;
    const int64_t nc = h->t.ncells;
    const int64_t* coff = h->at<int64_t>(h->o.coff);
    // stage into scratch first so that a rejected input leaves the state intact
    unpack(h->D, s, coff, E, h->tmp, 1, nc);
    unpack(h->D, s, coff, T, h->tmp + h->t.nl, 1, nc);
    unpack(h->D, s, coff, z, h->tmp2, 1, nc);
    fill_native(s, reinterpret_cast<double*>(h->flag), 1, 0.0);
    h->D.active = nullptr;
    check_positive(h->D, s, h->tmp, 2, h->flag);
    check_positive(h->D, s, h->tmp2, 1, h->flag);
    int32_t bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, h->flag, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (bad) return fail(NRD_ENONPOS, "E, T and z must be positive and finite");
    copy_interior(h->D, s, h->tmp, h->cur);
    HIPCHK(hipMemcpyAsync(h->z, h->tmp2, 8 * h->t.nl, hipMemcpyDeviceToDevice, s));
    prepare_state(h, h->cur);
    ghost_fill_d(h->D, s, h->z, 1);
    cube(s, h->z, h->z3, h->t.nl);
    copy_interior(h->D, s, h->cur, h->prev);
    fill_native(s, h->udot, 2 * h->t.nl, 0.0);
    std::fill(h->dt_prev.begin(), h->dt_prev.end(), 0.0);
    std::fill(h->err_prev.begin(), h->err_prev.end(), -1.0);
    h->step_ready = false;
    h->fields_set = true;
    h->last_valid = h->resolve_ready = h->skip_estimate = false;
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    return NRD_OK;
}

nrd_status nrd_get_fields(nrd_hierarchy* h, double* E, double* T) {
    NEED_BOUND(h);
    hipStream_t s = h->stream;
    const int64_t nc = h->t.ncells;
    const int64_t* coff = h->at<int64_t>(h->o.coff);
    if (E) pack(h->D, s, coff, h->cur, E, 1, nc);
    if (T) pack(h->D, s, coff, h->cur + h->t.nl, T, 1, nc);
    HIPCHK(hipStreamSynchronize(s));
    return NRD_OK;
}

nrd_status nrd_begin_step(nrd_hierarchy* h, const double* dt) {
    NEED_BOUND(h);
    if (!dt) return fail(NRD_EINVAL, "NULL dt");
    return begin_step(h, dt);
}

nrd_status nrd_residual(nrd_hierarchy* h, double* u, double* F) {
    NEED_BOUND(h);
    if (!h->step_ready) return fail(NRD_ESTATE, "call nrd_begin_step first");
    h->D.active = nullptr;
    op_residual(h, u, F);
    HIPCHK(hipGetLastError());
    return NRD_OK;
}

nrd_status nrd_jvp(nrd_hierarchy* h, double* u, double* v, double* Jv) {
    NEED_BOUND(h);
    if (!h->step_ready) return fail(NRD_ESTATE, "call nrd_begin_step first");
    h->D.active = nullptr;
    op_jvp(h, u, v, Jv, false);
    HIPCHK(hipGetLastError());
    return NRD_OK;
}

nrd_status nrd_precond_setup(nrd_hierarchy* h, double* u) {
    NEED_BOUND(h);
    if (!h->step_ready) return fail(NRD_ESTATE, "call nrd_begin_step first");
    h->D.active = nullptr;
    pc_setup(h, u, false);
    HIPCHK(hipGetLastError());
    return NRD_OK;
}

nrd_status nrd_precond_apply(nrd_hierarchy* h, const double* w, double* y) {
    NEED_BOUND(h);
    if (!h->step_ready) return fail(NRD_ESTATE, "call nrd_begin_step first");
    h->D.active = nullptr;
    pc_apply(h, w, y);
    HIPCHK(hipGetLastError());
    return NRD_OK;
}

nrd_status nrd_vjp(nrd_hierarchy* h, double* u, double* lam, double* JTl, double* gz) {
    NEED_BOUND(h);
    if (!h->step_ready) return fail(NRD_ESTATE, "call nrd_begin_step first");
    RCHK(ensure_cf_transpose(h));
    hipStream_t s = h->stream;
    h->D.active = nullptr;
    prepare_state(h, u);
    vjp_full(h->D, s, u, lam, JTl, h->gzn);
    if (gz) pack(h->D, s, h->at<int64_t>(h->o.coff), h->gzn, gz, 1, h->t.ncells);
    HIPCHK(hipGetLastError());
    return NRD_OK;
}

nrd_status nrd_implicit_step(nrd_hierarchy* h, const double* dt, nrd_step_stats* stats) {
    NEED_BOUND(h);
    if (!dt) return fail(NRD_EINVAL, "NULL dt");
    nrd_status rc = implicit_step(h, dt, stats, h->opt.bdf_max_order == 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(NRD_EDEVICE, hipGetErrorString(e));
    return rc;
}

nrd_status nrd_adaptive_steps(nrd_hierarchy* h, const nrd_timectl* ctl, int32_t nsteps,
                              double* dt, double* t, nrd_step_stats* stats) {
    NEED_BOUND(h);
    if (!ctl || !dt || nsteps < 0) return fail(NRD_EINVAL, "NULL argument or nsteps < 0");
    if (!h->opt.error_estimate)
        return fail(NRD_EINVAL, "the hierarchy was created without error_estimate");
    if (!(ctl->eps > 0.0) || !(ctl->ratio_min > 0.0) || !(ctl->ratio_max >= ctl->ratio_min) ||
        ctl->max_halvings < 0 || (ctl->controller != NRD_CTL_PC47 && ctl->controller != NRD_CTL_EPS))
        return fail(NRD_EINVAL, "bad time-step controller settings");
    const int np = h->t.nprob;
    for (int p = 0; p < np; ++p)
        if (!(dt[p] > 0.0)) return fail(NRD_EINVAL, "step sizes must be positive");
    std::vector<nrd_step_stats> st(np);
    for (int n = 0; n < nsteps; ++n) {
        std::vector<double> cur(dt, dt + np);
        std::vector<int32_t> halvings(np, 0);
        for (;;) {
            const nrd_status rc = implicit_step(h, cur.data(), st.data(),
                                                h->opt.bdf_max_order == 1);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return fail(NRD_EDEVICE, hipGetErrorString(e));
            if (rc == NRD_OK) break;
            if (rc != NRD_ENOTCONV) return rc;
            // the batch was rolled back: halve the steps that failed
            bool retry = false;
            for (int p = 0; p < np; ++p) {
                if (st[p].converged) continue;
                if (halvings[p] >= ctl->max_halvings)
                    return fail(NRD_ENOTCONV, "a step did not converge after max_halvings "
                                              "halvings; state of the last accepted step");
                cur[p] *= 0.5;
                ++halvings[p];
                retry = true;
            }
            if (!retry) return rc;
        }
        // next step sizes: PC.4.7 (EPS for a problem's first estimate) or EPS,
        // ratio bounded; a BDF1 step keeps its size
        for (int p = 0; p < np; ++p) {
            if (t) t[p] += cur[p];
            double ratio = 1.0;
            const double err = st[p].err_norm;
            if (err >= 0.0) {
                if (err > 0.0) {
                    if (ctl->controller == NRD_CTL_PC47 && h->err_prev[p] >= 0.0)
                        ratio = std::pow(ctl->eps / err, 0.4 / 3.0) *
                                std::pow(h->err_prev[p] / err, 0.7 / 3.0) * h->alpha[p];
                    else
                        ratio = std::pow(ctl->eps / err, 1.0 / 3.0);
                } else {
                    ratio = ctl->ratio_max;
                }
                h->err_prev[p] = err;
            }
            ratio = std::min(std::max(ratio, ctl->ratio_min), ctl->ratio_max);
            dt[p] = ratio * cur[p];
            if (stats) stats[(size_t)n * np + p] = st[p];
        }
    }
    return NRD_OK;
}

nrd_status nrd_adjoint_run(nrd_hierarchy* h, const double* dt, int32_t nsteps, int32_t every,
                           const double* dJdE, double* gz) {
    NEED_BOUND(h);
    if (!dt || !gz) return fail(NRD_EINVAL, "NULL argument");
    return adjoint_run(h, dt, nsteps, every, dJdE, gz);
}

// ---------------------------------------------------------------------------
// tile-shape tuner: per patch-size class, the plane-tile shape (planes per
// tile, cells per plane run) of the plane stencils, chosen by timing the
// residual kernel on that class's patches with every candidate shape
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {

struct ClassKey {
    int32_t n[3];
    bool operator<(const ClassKey& o) const {
        return std::lexicographical_compare(n, n + 3, o.n, o.n + 3);
    }
};

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

}  // namespace

extern "C" {

// Tiles of every patch with the given per-patch shapes, in launch order
// (level by level); false if some patch has no shape that fits.
static bool plane_list(const Tables& t, const std::vector<int32_t>& kc,
                       const std::vector<int32_t>& run, int32_t span, std::vector<STile>& out) {
    out.clear();
    for (int l = 0; l < t.nlev; ++l)
        for (int b = 0; b < t.nbox; ++b)
            if (t.boxes[b].level == l && !patch_planes(t.patches[b], b, kc[b], run[b], span, out))
                return false;
    return true;
}

nrd_status nrd_autotune(nrd_hierarchy* h, const char* cache_path, int32_t* timed_classes) {
    NEED_BOUND(h);
    if (timed_classes) *timed_classes = 0;
    const int var = h->opt.stencil;
    if (var == 0) return NRD_OK;                 // one-cell tiles: nothing to choose
    if (!h->fields_set) return fail(NRD_ESTATE, "nrd_autotune needs nrd_set_fields first");
    Tables& t = h->t;
    hipStream_t s = h->stream;
    const int32_t span = var == 3 ? kStageLen : 0;
    const int32_t run0 = var == 2 ? 4 * 63 : (var == 3 ? kStageCells : 256);
    std::vector<std::pair<int32_t, int32_t>> cand;           // (planes, run)
    if (var == 3) {
        for (int kc : {4, 8, 16, 32}) cand.push_back({kc, kStageCells});
    } else {
        for (int kc : {2, 4, 8, 16}) cand.push_back({kc, run0});
    }
    std::map<ClassKey, std::vector<int32_t>> cls;
    for (int b = 0; b < t.nbox; ++b) {
        ClassKey k;
        std::copy(t.patches[b].n, t.patches[b].n + 3, k.n);
        cls[k].push_back(b);
    }
    const std::string arch = device_arch();
    // cache format tag: the tile constants the cached shapes were chosen with
    const std::string cache_fmt =
        "f" + std::to_string(kStageCells) + "x" + std::to_string(kStageLen) + "b" +
        std::to_string(kBlock);
    std::map<ClassKey, std::pair<int32_t, int32_t>> pick;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string a, v, fmt, dims;
            int32_t kc = 0, run = 0;
            if (!(ls >> a >> v >> fmt >> dims >> kc >> run)) continue;
            ClassKey k;
            if (a != arch || v != "v" + std::to_string(var) || fmt != cache_fmt ||
                std::sscanf(dims.c_str(), "%dx%dx%d", &k.n[0], &k.n[1], &k.n[2]) != 3)
                continue;
            // only shapes this build would itself try: a stale or edited line
            // can never give a tile more cells than a workgroup holds
            bool known = false;
            for (auto [ckc, crun] : cand) known |= (ckc == kc && crun == run);
            if (!known) continue;
            pick[k] = {kc, run};
        }
    }
    // current shapes: cached choices, else the defaults
    std::vector<int32_t> kc(t.nbox), run(t.nbox);
    for (auto& kv : cls) {
        auto it = pick.find(kv.first);
        for (int b : kv.second) {
            kc[b] = it != pick.end() ? it->second.first : default_zchunk(t.patches[b].n, var);
            run[b] = it != pick.end() ? it->second.second : run0;
        }
    }
    // Coordinate descent on the objective that matters: the time of the whole
    // batched residual launch, varying one class's shape with the others held.
    // Trial tile lists go to the tile region beyond the current tiles.
    STile* scratch = h->at<STile>(h->o.stiles) + t.stiles.size();
    const size_t room = h->stile_cap - t.stiles.size();
    h->D.active = nullptr;
    prepare_state(h, h->cur);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    nrd_status rc = NRD_OK;
    std::vector<STile> tl;
    auto time_list = [&](double& ms_out) -> bool {
        if (tl.empty() || tl.size() > room) return false;
        if (hipMemcpyAsync(scratch, tl.data(), sizeof(STile) * tl.size(), hipMemcpyHostToDevice,
                           s) != hipSuccess) {
            rc = fail(NRD_EDEVICE, "tile upload failed");
            return false;
        }
        Dev Dt = h->D;
        Dt.stiles = scratch;
        residual(Dt, s, 0, (int)tl.size(), h->cur, h->bvec, h->tmp);    // warm-up
        double best = 1e300;
        for (int rep = 0; rep < 3; ++rep) {
            (void)hipEventRecord(e0, s);
            residual(Dt, s, 0, (int)tl.size(), h->cur, h->bvec, h->tmp);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, (double)ms);
        }
        ms_out = best;
        return true;
    };
    std::ofstream out;
    if (cache_path) out.open(cache_path, std::ios::app);
    double cur_ms = 1e300;
    if (plane_list(t, kc, run, span, tl)) (void)time_list(cur_ms);
    for (auto& kv : cls) {
        if (rc) break;
        if (pick.count(kv.first)) continue;
        std::pair<int32_t, int32_t> choice{kc[kv.second[0]], run[kv.second[0]]};
        double best = cur_ms;
        for (auto [ckc, crun] : cand) {
            if (ckc == choice.first && crun == choice.second) continue;
            std::vector<int32_t> kc2 = kc, run2 = run;
            for (int b : kv.second) {
                kc2[b] = ckc;
                run2[b] = crun;
            }
            double ms = 0.0;
            if (!plane_list(t, kc2, run2, span, tl) || !time_list(ms)) {
                if (rc) break;
                continue;
            }
            if (ms < 0.98 * best) {                  // keep a change only if it pays
                best = ms;
                choice = {ckc, crun};
            }
        }
        if (rc) break;
        for (int b : kv.second) {
            kc[b] = choice.first;
            run[b] = choice.second;
        }
        cur_ms = best;
        pick[kv.first] = choice;
        if (timed_classes) ++*timed_classes;
        if (out)
            out << arch << " v" << var << " " << cache_fmt << " " << kv.first.n[0] << "x"
                << kv.first.n[1] << "x"
                << kv.first.n[2] << " " << choice.first << " " << choice.second << " "
                << best * 1e3 << "\n";
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    HIPCHK(hipGetLastError());
    // apply the chosen shapes
    Tables trial;
    trial.nlev = t.nlev;
    trial.nbox = t.nbox;
    trial.patches = t.patches;
    trial.boxes = t.boxes;
    if (!build_planes(trial, kc, run, span) || trial.stiles.size() > h->stile_cap)
        return fail(NRD_EINVAL, "tuned tile shapes do not fit");
    t.stiles.swap(trial.stiles);
    t.level_stile0.swap(trial.level_stile0);
    t.patch_stile0.swap(trial.patch_stile0);
    HIPCHK(up(s, h->ws + h->o.stiles, t.stiles));
    for (int l = 0; l <= t.nlev; ++l) h->D.level_stile0[l] = t.level_stile0[l];
    h->drop_graphs();                               // captured launches used the old tiles
    RCHK(upload_active(h));                         // tile map of the new list
    HIPCHK(hipStreamSynchronize(s));
    return NRD_OK;
}

// ---------------------------------------------------------------------------
// dynamic regridding (Sec. 5)
// ---------------------------------------------------------------------------

// udot = (c0 x - b) / dt per problem with the last step's c0, b and dt
static nrd_status set_udot(nrd_hierarchy* h, const double* x) {
    const int np = h->t.nprob;
    hipStream_t s = h->stream;
    std::vector<double> buf(2 * np);
    for (int p = 0; p < np; ++p) {
        buf[p] = h->c0[p] / h->dt_cur[p];
        buf[np + p] = -1.0 / h->dt_cur[p];
    }
    HIPCHK(up(s, h->coefA, buf));
    h->D.active = nullptr;
    lincomb2(h->D, s, h->coefA, x, h->coefA + np, h->bvec, h->udot);
    HIPCHK(hipStreamSynchronize(s));      // the host coefficient buffer ends here
    return NRD_OK;
}

nrd_status nrd_tag(nrd_hierarchy* h, const nrd_tagging* crit, uint8_t* tags) {
    NEED_BOUND(h);
    if (!crit || !tags) return fail(NRD_EINVAL, "NULL argument");
    if (!h->fields_set) return fail(NRD_ESTATE, "nrd_tag needs nrd_set_fields first");
    hipStream_t s = h->stream;
    h->D.active = nullptr;
    prepare_state(h, h->cur);
    abs_max(h->D, s, h->cur, h->partial, h->minout);
    // z with every coarse-fine ghost set to its coarse parent's material
    HIPCHK(hipMemcpyAsync(h->tmp2, h->z, 8 * h->t.nl, hipMemcpyDeviceToDevice, s));
    ghost_fill_parent(h->D, s, h->tmp2);
    TagCrit tc;
    std::memset(&tc, 0, sizeof(tc));
    tc.grad = crit->grad_E;
    tc.tau_g = crit->tau_g;
    tc.tau_c = crit->tau_c;
    tc.z_interface = crit->z_interface != 0;
    tag_cells(h->D, s, h->at<int64_t>(h->o.coff), h->cur, h->tmp2, h->minout, tc, tags);
    HIPCHK(hipGetLastError());
    return NRD_OK;
}

nrd_status nrd_cluster(const nrd_problem* probs, int32_t nprob, const nrd_box* boxes,
                       int32_t nbox, const uint8_t* tags, const nrd_cluster_opt* opt,
                       nrd_box* out, int32_t cap, int32_t* nout) {
    if (!probs || !boxes || !tags || !opt || !nout || nprob <= 0 || nbox <= 0)
        return fail(NRD_EINVAL, "NULL argument or empty input");
    try {
        std::vector<nrd_box> res;
        std::string msg;
        const nrd_status rc = cluster_boxes(probs, nprob, boxes, nbox, tags, *opt, res, msg);
        if (rc) return fail(rc, msg);
        *nout = (int32_t)res.size();
        if ((int32_t)res.size() > cap || !out)
            return fail(NRD_EINVAL, "output holds " + std::to_string(cap) + " boxes, " +
                                        std::to_string(res.size()) + " needed");
        std::copy(res.begin(), res.end(), out);
        return NRD_OK;
    } catch (const std::exception& e) {
        return fail(NRD_EINVAL, e.what());
    }
}

nrd_status nrd_transfer(nrd_hierarchy* src, nrd_hierarchy* dst, const double* z) {
    NEED_BOUND(src);
    NEED_BOUND(dst);
    if (!z) return fail(NRD_EINVAL, "NULL z");
    if (src == dst) return fail(NRD_EINVAL, "source and destination are the same hierarchy");
    if (!src->fields_set) return fail(NRD_ESTATE, "the source has no fields");
    const Tables& ts = src->t;
    Tables& td = dst->t;
    const int np = td.nprob;
    if (ts.nprob != np) return fail(NRD_EINVAL, "the hierarchies hold different problems");
    for (int p = 0; p < np; ++p) {
        const nrd_problem &a = ts.probs[p], &b = td.probs[p];
        for (int d = 0; d < 3; ++d)
            if (a.base_n[d] != b.base_n[d] || a.lo[d] != b.lo[d] || a.hi[d] != b.hi[d])
                return fail(NRD_EINVAL, "problem " + std::to_string(p) +
                                            ": base grid or domain differs");
    }
    HIPCHK(hipStreamSynchronize(src->stream));
    hipStream_t s = dst->stream;
    dst->D.active = nullptr;
    // material field of the new hierarchy (staged: a rejected z changes nothing)
    const int64_t* coff = dst->at<int64_t>(dst->o.coff);
    unpack(dst->D, s, coff, z, dst->tmp2, 1, td.ncells);
    fill_native(s, reinterpret_cast<double*>(dst->flag), 1, 0.0);
    check_positive(dst->D, s, dst->tmp2, 1, dst->flag);
    int32_t bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, dst->flag, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (bad) return fail(NRD_ENONPOS, "z must be positive and finite");
    HIPCHK(hipMemcpyAsync(dst->z, dst->tmp2, 8 * td.nl, hipMemcpyDeviceToDevice, s));
    ghost_fill_d(dst->D, s, dst->z, 1);
    cube(s, dst->z, dst->z3, td.nl);
    // copy fragments: dst patch x src patch of the same problem and level
    std::vector<XferFrag> frags;
    std::vector<XferChunk> chunks;
    std::vector<int32_t> lev_chunk0(td.nlev + 1, 0);
    constexpr int32_t kChunk = 4 * kBlock;
    for (int l = 0; l < td.nlev; ++l) {
        lev_chunk0[l] = (int32_t)chunks.size();
        if (l >= ts.nlev) continue;
        for (int p = 0; p < np; ++p)
            for (int32_t db : td.level_patches[p][l])
                for (int32_t sb : ts.level_patches[p][l]) {
                    const HostBox &a = td.boxes[db], &b = ts.boxes[sb];
                    XferFrag f;
                    f.dpatch = db;
                    f.spatch = sb;
                    int64_t n = 1;
                    for (int d = 0; d < 3; ++d) {
                        f.lo[d] = std::max(a.lo[d], b.lo[d]);
                        f.n[d] = std::min(a.hi[d], b.hi[d]) - f.lo[d];
                        n *= std::max(0, f.n[d]);
                    }
                    if (n <= 0) continue;
                    const int32_t fi = (int32_t)frags.size();
                    frags.push_back(f);
                    for (int64_t c0 = 0; c0 < n; c0 += kChunk)
                        chunks.push_back({fi, (int32_t)c0, (int32_t)std::min<int64_t>(kChunk, n - c0)});
                }
    }
    lev_chunk0[td.nlev] = (int32_t)chunks.size();
    // the tables go to the Krylov basis region of dst, unused until its next solve
    const size_t fbytes = (sizeof(XferFrag) * frags.size() + 255) & ~size_t(255);
    if (fbytes + sizeof(XferChunk) * chunks.size() > 8 * (size_t)dst->nl2() * (dst->m + 1))
        return fail(NRD_EUNSUPPORTED, "transfer tables exceed the scratch region");
    char* base = reinterpret_cast<char*>(dst->V);
    XferFrag* dfr = reinterpret_cast<XferFrag*>(base);
    XferChunk* dch = reinterpret_cast<XferChunk*>(base + fbytes);
    HIPCHK(up(s, dfr, frags));
    HIPCHK(up(s, dch, chunks));
    const PatchInfo* dP = dst->D.patches;
    const PatchInfo* sP = src->D.patches;
    const ShadowPatch* shp = dst->at<ShadowPatch>(dst->o.shadows);
    const int32_t* ssrc = dst->at<int32_t>(dst->o.shadow_src);
    const int64_t slen = std::max<int64_t>(1, td.shadow_len);
    const double* from[3] = {src->cur, src->prev, src->bvec};
    double* to[3] = {dst->cur, dst->prev, dst->bvec};
    for (int v = 0; v < 3; ++v) {
        for (int l = 0; l < td.nlev; ++l) {
            if (l > 0) refine_level(dst->D, s, shp, ssrc, l, to[v], dst->tmp, slen, 2);
            const int a = lev_chunk0[l], n = lev_chunk0[l + 1] - a;
            xfer_copy(s, n, dch + a, dfr, dP, sP, from[v], to[v], ts.nl, td.nl, 2);
        }
        prepare_state(dst, to[v]);
    }
    // time history and the last step's system
    dst->dt_prev = src->dt_prev;
    dst->err_prev.assign(np, -1.0);
    dst->last_valid = src->last_valid;
    dst->resolve_ready = src->last_valid;
    dst->skip_estimate = true;
    if (src->last_valid) {
        dst->c0 = src->c0;
        dst->alpha = src->alpha;
        dst->beta = src->beta;
        dst->dt_cur = src->dt_cur;
        for (int p = 0; p < np; ++p) {
            dst->ps_host[p].dt = src->ps_host[p].dt;
            dst->ps_host[p].c0 = src->ps_host[p].c0;
            dst->ps_host[p].beta = src->ps_host[p].beta;
            dst->ps_host[p].alpha = src->ps_host[p].alpha;
        }
        HIPCHK(up(s, dst->ps, dst->ps_host));
    }
    if (src->last_valid)
        RCHK(set_udot(dst, dst->cur));      // from the interpolated state
    else
        fill_native(s, dst->udot, dst->nl2(), 0.0);
    dst->drop_graphs();
    dst->fields_set = true;
    dst->step_ready = src->last_valid;
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    return NRD_OK;
}

nrd_status nrd_resolve(nrd_hierarchy* h, nrd_step_stats* stats) {
    NEED_BOUND(h);
    const int np = h->t.nprob;
    if (stats)
        for (int p = 0; p < np; ++p) std::memset(&stats[p], 0, sizeof(stats[p]));
    if (!h->resolve_ready) return NRD_OK;
    hipStream_t s = h->stream;
    h->D.active = nullptr;
    HIPCHK(up(s, h->ps, h->ps_host));
    copy_interior(h->D, s, h->cur, h->x);
    std::vector<nrd_step_stats> st;
    const nrd_status rc = newton(h, st);
    for (int p = 0; p < np; ++p) {
        st[p].dt = h->dt_cur[p];
        st[p].err_norm = -1.0;
    }
    if (stats)
        for (int p = 0; p < np; ++p) stats[p] = st[p];
    if (rc) {
        if (rc == NRD_ENOTCONV) g_err = "the re-solve did not converge; transferred state kept";
        return rc;
    }
    // u'_n = (c0 u_n - b) / dt from the re-solved state
    RCHK(set_udot(h, h->x));
    std::swap(h->cur, h->x);
    prepare_state(h, h->cur);
    HIPCHK(hipStreamSynchronize(s));
    h->resolve_ready = false;
    HIPCHK(hipGetLastError());
    return NRD_OK;
}

nrd_status nrd_dot(nrd_hierarchy* h, const double* x, const double* y, double* out) {
    NEED_BOUND(h);
    std::vector<double> v;
    nrd_status rc = dot_host(h, x, y, v);
    if (rc) return rc;
    std::copy(v.begin(), v.end(), out);
    return NRD_OK;
}

nrd_status nrd_dot_noalloc(nrd_hierarchy* h, const double* x, const double* y, double* out) {
    if (!h) return fail(NRD_EINVAL, "NULL hierarchy");
    if (h->t.vtiles.size() > (size_t)kScratchTiles)
        return fail(NRD_EINVAL, "nrd_dot_noalloc: the hierarchy has " +
                                    std::to_string(h->t.vtiles.size()) +
                                    " reduction tiles, more than the " +
                                    std::to_string(kScratchTiles) + " its fixed array holds");
    NEED_BOUND(h);
    if (!x || !y || !out) return fail(NRD_EINVAL, "NULL argument");
    h->D.active = nullptr;
    // same kernels and summation order as nrd_dot; partials in the fixed
    // array, the per-problem sums straight into the caller's device buffer
    multidot(h->D, h->stream, x, 0, 1, y, h->scratch, out);
    HIPCHK(hipGetLastError());
    return NRD_OK;
}

nrd_status nrd_timer_enable(nrd_hierarchy* h, int32_t on) {
    if (!h) return fail(NRD_EINVAL, "NULL hierarchy");
    h->timing = on != 0;
    h->ev_pairs.clear();
    h->ev_used = 0;
    return NRD_OK;
}

nrd_status nrd_timer_read(nrd_hierarchy* h, int32_t which, double* ms, int32_t* count) {
    if (!h) return fail(NRD_EINVAL, "NULL hierarchy");
    if (which < 0 || which >= NRD_TIMER_COUNT) return fail(NRD_EINVAL, "unknown timer");
    HIPCHK(hipStreamSynchronize(h->stream));
    double tot = 0.0;
    int32_t n = 0;
    for (auto& pr : h->ev_pairs) {
        if (pr.which != which) continue;
        float dtm = 0.f;
        HIPCHK(hipEventElapsedTime(&dtm, pr.ev.first, pr.ev.second));
        tot += dtm;
        ++n;
    }
    if (ms) *ms = tot;
    if (count) *count = n;
    return NRD_OK;
}

nrd_status nrd_timer_cells(nrd_hierarchy* h, int32_t which, int64_t* cells) {
    if (!h) return fail(NRD_EINVAL, "NULL hierarchy");
    if (which < 0 || which >= NRD_TIMER_COUNT) return fail(NRD_EINVAL, "unknown timer");
    int64_t n = 0;
    for (auto& pr : h->ev_pairs)
        if (pr.which == which) n += pr.cells;
    if (cells) *cells = n;
    return NRD_OK;
}

}  // extern "C"
