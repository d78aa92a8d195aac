// Physics-based preconditioner kernels (paper Sec. 4.2-4.3, Alg. 1).
//
// P1 = diag(I - beta div D_E grad, I - beta div D_T grad) with D frozen at
// u^k, approximately inverted by one FAC V(m,n) cycle (default V(1,0)):
// red-black Gauss-Seidel (or damped point Jacobi) sweeps per refinement
// level and a multigrid V(1,1) cycle on the base level whose coarsest grid
// is solved with a dense float64 inverse.  P2 is the per-cell 2x2 coupling
// block.  PT is the storage and
// arithmetic type of the V-cycle (float in mixed precision, double
// otherwise); the bottom solve always uses double.
//
// Face coefficient arrays hold D at the LOW face of every cell in the
// native layout, so cell c's high face along d is the low face of c + st_d
// (for the last cell: the ghost slot).  On physical faces they hold the
// unlimited boundary coefficient D_b of E for a Marshak face and 0
// otherwise.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "precond.h"

namespace nrd {

static inline int nblocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

__device__ __forceinline__ void coords(const PatchInfo& p, int lin, int& i, int& j, int& k) {
    i = lin % p.n[0];
    const int r = lin / p.n[0];
    j = r % p.n[1];
    k = r / p.n[1];
}
__device__ __forceinline__ int nat(const PatchInfo& p, int i, int j, int k) {
    return p.off + (i + 1) + p.sy * (j + 1) + p.sz * (k + 1);
}

// ---------------------------------------------------------------------------
// snapshot: D_E, D_T on every face of every patch, sigma per cell
// ---------------------------------------------------------------------------

// D_T = kappa T_f^(5/2) of the face between cells of temperatures Ta, Tb
// (symmetric in Ta, Tb); the sweeps over colour-split storage recompute it
// from T with this same expression, so they see the snapshot's values.
template <typename PT>
__device__ __forceinline__ PT face_DT(PT Ta, PT Tb, PT kappa) {
    const PT Tf = PT(0.5) * (Ta + Tb);
    return kappa * Tf * Tf * sqrt(Tf);
}

// Face coefficients in the preconditioner's precision (the inputs are
// rounded to PT first; in float64 mode this is the float64 formula).
template <typename PT>
__device__ __forceinline__ void face_D(PT Ea, PT Eb, PT Ta, PT Tb, PT za, PT zb, PT h, PT kappa,
                                       PT lam, PT& DE, PT& DT) {
    const PT Tf = PT(0.5) * (Ta + Tb);
    const PT Tf3 = Tf * Tf * Tf;
    const PT S = Ea + Eb;
    // D_h / (1 + lam D_h g) with D_h = 2 Tf^3 / (3 Zf), g = 2|dE| / (h S)
    DE = PT(2) * Tf3 * h * S / (PT(3) * (za + zb) * h * S + PT(4) * lam * Tf3 * fabs(Eb - Ea));
    DT = face_DT(Ta, Tb, kappa);
}

template <typename PT>
__global__ __launch_bounds__(kBlock) void k_snapshot(const int32_t* __restrict__ act, 
    const Tile* __restrict__ tiles, const PatchInfo* __restrict__ P,
    const ProbScalars* __restrict__ ps, const double* __restrict__ u,
    const double* __restrict__ z3, PT* __restrict__ Dface, PT* __restrict__ sigma,
    int64_t nl, PT* __restrict__ Tp) {
    // Tp (may be NULL): T rounded to PT; when given, the three D_T arrays
    // are not written (every reader recomputes D_T from Tp with face_DT)
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    const ProbScalars& q = ps[t.prob];
    int id[3];
    coords(p, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = nat(p, id[0], id[1], id[2]);
    const int st[3] = {1, p.sy, p.sz};
    const PT E = (PT)u[c], T = (PT)u[c + nl], z = (PT)z3[c];
    const PT kappa = (PT)q.kappa, lam = (PT)q.lam;
    sigma[c] = z / (T * T * T);
    if (Tp) Tp[c] = T;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const PT h = (PT)p.h[d];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (s == 1 && id[d] != p.n[d] - 1) continue;     // high face owned by c+st
            const int slot = s ? c + st[d] : c;
            PT DE, DT;
            if ((id[d] == (s ? p.n[d] - 1 : 0)) && ((p.phys >> (2 * d + s)) & 1)) {
                DT = PT(0);
                DE = ((p.robin >> (2 * d + s)) & 1) ? T * T * T / (PT(3) * z) : PT(0);
            } else {
                const int nb = s ? c + st[d] : c - st[d];
                const PT En = (PT)u[nb], Tn = (PT)u[nb + nl], zn = (PT)z3[nb];
                if (s)
                    face_D<PT>(E, En, T, Tn, z, zn, h, kappa, lam, DE, DT);
                else
                    face_D<PT>(En, E, Tn, T, zn, z, h, kappa, lam, DE, DT);
            }
            Dface[(0 * 3 + d) * nl + slot] = DE;
            if (!Tp) Dface[(1 * 3 + d) * nl + slot] = DT;
        }
    }
}

// Coarse face coefficient = mean of the four fine face coefficients
// (grid g+1 from grid g); boundary faces included.
// fmap (may be NULL): per coarse native cell, the fine patch holding its
// children (a base grid cut into several level-0 boxes); else the problem's
// one fine box fbox[prob].  Coarse boxes start at 0, so a coarse cell's
// first child is at 2 id - lo of its fine patch.
template <typename PT>
__global__ __launch_bounds__(kBlock) void k_mg_coarsen(const int32_t* __restrict__ act, 
    const Tile* __restrict__ tiles, const PatchInfo* __restrict__ Pc,
    const PatchInfo* __restrict__ Pf, const int32_t* __restrict__ fbox,
    const int32_t* __restrict__ fmap,
    const PT* __restrict__ Df, int64_t nlf, PT* __restrict__ Dc, int64_t nlc,
    const PT* __restrict__ Tp, const ProbScalars* __restrict__ ps) {
    // Tp (may be NULL; the first grid of a colour-split base, one box
    // covering the domain): the fine D_T recomputed from T with face_DT,
    // 0 on the domain boundary, as the snapshot computes them
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& pc = Pc[t.patch];
    int id[3];
    coords(pc, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = nat(pc, id[0], id[1], id[2]);
    const PatchInfo& pf = Pf[fmap ? fmap[c] : fbox[t.prob]];
    const PT kappa = Tp ? (PT)ps[t.prob].kappa : PT(0);
    const int stc[3] = {1, pc.sy, pc.sz};
    const int stf[3] = {1, pf.sy, pf.sz};
    const int f0 = nat(pf, 2 * id[0] - pf.lo[0], 2 * id[1] - pf.lo[1], 2 * id[2] - pf.lo[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int t1 = d == 0 ? 1 : 0;
        const int t2 = d == 2 ? 1 : 2;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (s == 1 && id[d] != pc.n[d] - 1) continue;
            const int slot = s ? c + stc[d] : c;
            const int fs = s ? f0 + 2 * stf[d] : f0;
            for (int fld = 0; fld < 2; ++fld) {
                PT v;
                if (fld == 1 && Tp) {
                    // the low face of fine cell x lies between x - st and x
                    const bool edge = s ? true : id[d] == 0;
                    const int o = stf[d];
                    auto dt = [&](int x) { return face_DT(Tp[x - o], Tp[x], kappa); };
                    v = edge ? PT(0)
                             : (dt(fs) + dt(fs + stf[t1])) +
                                   (dt(fs + stf[t2]) + dt(fs + stf[t1] + stf[t2]));
                } else {
                    const PT* src = Df + (fld * 3 + d) * nlf;
                    v = (src[fs] + src[fs + stf[t1]]) + (src[fs + stf[t2]] +
                                                          src[fs + stf[t1] + stf[t2]]);
                }
                Dc[(fld * 3 + d) * nlc + slot] = v * PT(0.25);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// level operator: (A e)_c = diag_c e_c - sum w_f e_nb
//   interior / sibling faces: w = a = beta D / h^2, diag += a
//   coarse-fine faces (correction ghost = e_c / 3): diag += 2/3 a
//   Marshak faces (E): diag += 2 beta D_b / ((4 D_b + h) h)
// ---------------------------------------------------------------------------

// Both fields of one cell.  Faces are classified without branching on the
// common path: an interior (or sibling) face contributes a = beta D / h^2 to
// the diagonal and a e_nb to the neighbour sum; a physical face contributes
// nothing (plus the Marshak term for E on a Robin face); a coarse-fine face
// contributes 2/3 a to the diagonal only.  Neighbour values are loaded
// unconditionally (ghost slots always hold finite values).
// Diagonal dg and neighbour sum ns of both fields at cell c = id (ZERO: the
// iterate is taken as zero, ns = 0).
// SPLIT: e in colour-split storage, its neighbours at enb (c indexes the
// face coefficients and cell types, which stay native), and the T-field
// coefficient of each face recomputed from Tp (T in PT, native; kappa) in
// place of reading the three D_T arrays (a box with no siblings or coarse-
// fine faces: every face that enters is between two of its interior cells).
template <typename PT, bool ZERO, bool SPLIT = false>
__device__ __forceinline__ void level_terms(const PatchInfo& p, const int id[3], int c,
                                            double beta, const uint8_t* __restrict__ ctype,
                                            const PT* __restrict__ D, const PT* __restrict__ e,
                                            int64_t nl, PT dgo[2], PT nso[2],
                                            const int* enb = nullptr,
                                            const PT* __restrict__ Tp = nullptr,
                                            PT kappa = PT(0)) {
    const int st[3] = {1, p.sy, p.sz};
    PT bh2[3];
    bool ph[6], cf[6];
    bool any_robin = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        bh2[d] = (PT)(beta * p.ih[d] * p.ih[d]);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int fc = 2 * d + s;
            const bool edge = id[d] == (s ? p.n[d] - 1 : 0);
            ph[fc] = edge && ((p.phys >> fc) & 1);
            cf[fc] = false;
            if (edge && !ph[fc]) cf[fc] = ctype[s ? c + st[d] : c - st[d]] == GK_CF;
            any_robin |= ph[fc] && ((p.robin >> fc) & 1);
        }
    }
#pragma unroll
    for (int fld = 0; fld < 2; ++fld) {
        const PT* ef = e + fld * nl;
        PT dg = PT(1), ns = PT(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const PT* Dd = D + (fld * 3 + d) * nl;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int fc = 2 * d + s;
                const PT a = bh2[d] * ((SPLIT && fld == 1)
                                           ? face_DT(Tp[c], Tp[s ? c + st[d] : c - st[d]], kappa)
                                           : Dd[s ? c + st[d] : c]);
                const PT en = ZERO ? PT(0)
                                   : ef[SPLIT ? enb[fc] : (s ? c + st[d] : c - st[d])];
                const bool open = !(ph[fc] || cf[fc]);
                dg += open ? a : (cf[fc] ? PT(2.0 / 3.0) * a : PT(0));
                ns += open ? a * en : PT(0);
            }
        }
        if (fld == 0 && any_robin) {
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const int fc = 2 * d + s;
                    if (ph[fc] && ((p.robin >> fc) & 1)) {
                        const PT Db = D[d * nl + (s ? c + st[d] : c)];
                        const PT h = (PT)p.h[d];
                        dg += PT(2) * (PT)beta * Db / ((PT(4) * Db + h) * h);
                    }
                }
        }
        dgo[fld] = dg;
        nso[fld] = ns;
    }
}

// SPLIT: e and f in colour-split storage
template <typename PT, int MODE, bool SPLIT>   // MODE 0: RBGS colour (zero start) 1: colour
__device__ __forceinline__ void level_update(const PatchInfo& p, const int id[3], double beta,
                                             const uint8_t* __restrict__ ctype,
                                             const PT* __restrict__ D,
                                             const PT* __restrict__ f, PT* __restrict__ e,
                                             int64_t nl, const PT* __restrict__ Tp, PT kappa) {
    const int c = nat(p, id[0], id[1], id[2]);
    int own = c, enb[6];
    if (SPLIT) split_stencil(p, id, own, enb);
    PT dg[2], ns[2];
    level_terms<PT, MODE == 0, SPLIT>(p, id, c, beta, ctype, D, e, nl, dg, ns, enb, Tp, kappa);
#pragma unroll
    for (int fld = 0; fld < 2; ++fld) {
        const int64_t cfi = fld * nl + own;
        e[cfi] = (f[cfi] + ns[fld]) / dg[fld];
    }
}

// Damped point Jacobi on the level operator (the alternative level smoother
// of Sec. 4.3): every cell from the same old iterate e_in,
// e_out = (1 - omega) e_in + omega (f + ns) / dg; ZERO: e_in = 0.
template <typename PT, bool ZERO>
__global__ __launch_bounds__(kBlock) void k_jacobi(const int32_t* __restrict__ act,
    const Tile* __restrict__ tiles, const PatchInfo* __restrict__ P,
    const ProbScalars* __restrict__ ps, const uint8_t* __restrict__ ctype,
    const PT* __restrict__ D, const PT* __restrict__ f, const PT* __restrict__ e_in,
    PT* __restrict__ e_out, double omega, int64_t nl) {
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    int id[3];
    coords(p, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = nat(p, id[0], id[1], id[2]);
    PT dg[2], ns[2];
    level_terms<PT, ZERO>(p, id, c, ps[t.prob].beta, ctype, D, e_in, nl, dg, ns);
    const PT w = (PT)omega;
#pragma unroll
    for (int fld = 0; fld < 2; ++fld) {
        const int64_t cfi = fld * nl + c;
        const PT x = (f[cfi] + ns[fld]) / dg[fld];
        e_out[cfi] = ZERO ? w * x : (PT(1) - w) * e_in[cfi] + w * x;
    }
}

// Block Gauss-Seidel on x-lines (the third level smoother of Sec. 4.3): one
// thread per line (j, k) of a patch whose colour (j + k in level index space)
// is being swept solves the tridiagonal system of the level operator along
// the line exactly (Thomas algorithm, the elimination factors kept in cp),
// with the y and z neighbours and the sibling ghosts at the line's ends held
// (ZERO: the iterate is zero, the first colour of a sweep from zero; the
// lines of the other colour are then set to zero).
// Faces are classified as in level_terms.
template <typename PT, bool ZERO>
__global__ __launch_bounds__(kBlock) void k_line(const int32_t* __restrict__ act,
    const Tile* __restrict__ ltiles, const PatchInfo* __restrict__ P,
    const ProbScalars* __restrict__ ps, const uint8_t* __restrict__ ctype,
    const PT* __restrict__ D, const PT* __restrict__ f, PT* __restrict__ e,
    PT* __restrict__ cp, int colour, int64_t nl) {
    const Tile t = ltiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    const int q = t.start + threadIdx.x;
    const int j = q % p.n[1], k = q / p.n[1];
    const int n0 = p.n[0];
    if (((j + k + p.lo[1] + p.lo[2]) & 1) != colour) {
        // a sweep from zero: the other colour's lines are zero (their values,
        // and a sibling's through its ghosts, are read by the next colour)
        if (ZERO)
            for (int i = 0; i < n0; ++i) {
                const int c = nat(p, i, j, k);
                e[c] = PT(0);
                e[nl + c] = PT(0);
            }
        return;
    }
    const double beta = ps[t.prob].beta;
    const int st[3] = {1, p.sy, p.sz};
    PT bh2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) bh2[d] = (PT)(beta * p.ih[d] * p.ih[d]);
    for (int fld = 0; fld < 2; ++fld) {
        const PT* Df = D + fld * 3 * nl;
        PT* ef = e + fld * nl;
        PT* cf = cp + fld * nl;
        PT cprev = PT(0), dprev = PT(0);
        for (int i = 0; i < n0; ++i) {
            const int id[3] = {i, j, k};
            const int c = nat(p, i, j, k);
            PT dg = PT(1), b = f[fld * nl + c], alo = PT(0), ahi = PT(0);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const PT* Dd = Df + d * nl;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const int fc = 2 * d + s;
                    const bool edge = id[d] == (s ? p.n[d] - 1 : 0);
                    const bool ph = edge && ((p.phys >> fc) & 1);
                    const bool cfc = edge && !ph && ctype[s ? c + st[d] : c - st[d]] == GK_CF;
                    const PT a = bh2[d] * Dd[s ? c + st[d] : c];
                    const bool open = !(ph || cfc);
                    dg += open ? a : (cfc ? PT(2.0 / 3.0) * a : PT(0));
                    if (ph && fld == 0 && ((p.robin >> fc) & 1)) {
                        const PT Db = Dd[s ? c + st[d] : c];
                        const PT h = (PT)p.h[d];
                        dg += PT(2) * (PT)beta * Db / ((PT(4) * Db + h) * h);
                    }
                    if (!open) continue;
                    if (d == 0 && !edge) {
                        // coupling within the line
                        if (s) ahi = a;
                        else alo = a;
                    } else if (!ZERO) {
                        b += a * ef[s ? c + st[d] : c - st[d]];
                    }
                }
            }
            // Thomas: den = dg - alo cp_{i-1}; cp_i = ahi / den (coupling -ahi);
            // dp_i = (b + alo dp_{i-1}) / den
            const PT den = dg - alo * cprev;
            const PT cpi = ahi / den;
            const PT dpi = (b + alo * dprev) / den;
            cf[c] = cpi;
            ef[c] = dpi;
            cprev = cpi;
            dprev = dpi;
        }
        PT x = PT(0);
        for (int i = n0 - 1; i >= 0; --i) {
            const int c = nat(p, i, j, k);
            x = ef[c] + cf[c] * x;
            ef[c] = x;
        }
    }
}

// One cell of a red-black half-sweep; REGION: only covered cells relax,
// any other cell is set to 0 (the coarse approximation of AFACx lives on
// the region a finer level covers and vanishes outside it).
template <typename PT, int MODE, bool REGION, bool SPLIT>
__device__ __forceinline__ void level_cell(const PatchInfo& p, const int id[3], double beta,
                                           const uint8_t* __restrict__ ctype,
                                           const PT* __restrict__ D, const PT* __restrict__ f,
                                           PT* __restrict__ e, int64_t nl,
                                           const PT* __restrict__ Tp, PT kappa) {
    static_assert(!(REGION && SPLIT), "region sweeps run on native storage");
    if (REGION) {
        const int c = nat(p, id[0], id[1], id[2]);
        if (!(ctype[c] & CT_COVERED)) {
            e[c] = PT(0);
            e[c + nl] = PT(0);
            return;
        }
    }
    level_update<PT, MODE, SPLIT>(p, id, beta, ctype, D, f, e, nl, Tp, kappa);
}

// One colour of a red-black sweep (MODE 0: from e = 0), kBlock / 2 threads
// per tile of kBlock cells.  When the patch's x extent is
// even, rows start at even linear indices, so every pair (2q, 2q + 1) of a
// tile lies in one row and holds exactly one cell of each colour: thread q
// updates that cell and every lane does useful work.  Otherwise each thread
// tests two cells.  SPLIT: e and f in colour-split storage (even x extents).
template <typename PT, int MODE, bool REGION = false, bool SPLIT = false>
__global__ __launch_bounds__(kBlock) void k_level(const int32_t* __restrict__ act, 
    const Tile* __restrict__ tiles, const PatchInfo* __restrict__ P,
    const ProbScalars* __restrict__ ps, const uint8_t* __restrict__ ctype,
    const PT* __restrict__ D, const PT* __restrict__ f, PT* __restrict__ e,
    int colour, int64_t nl, const PT* __restrict__ Tp = nullptr) {
    // Tp: T in PT (SPLIT only; the T-field face coefficients)
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    const PatchInfo& p = P[t.patch];
    const double beta = ps[t.prob].beta;
    const PT kappa = (PT)ps[t.prob].kappa;
    int id[3];
    const int lo = p.lo[0] + p.lo[1] + p.lo[2];
    if ((p.n[0] & 1) == 0) {
        const int a = 2 * (int)threadIdx.x;          // tile starts are even
        if (a >= t.count) return;
        coords(p, t.start + a, id[0], id[1], id[2]);  // id[0] even
        id[0] += (colour + id[1] + id[2] + lo) & 1;
        level_cell<PT, MODE, REGION, SPLIT>(p, id, beta, ctype, D, f, e, nl, Tp, kappa);
    } else if (!SPLIT) {
        for (int q = threadIdx.x; q < t.count; q += kBlock / 2) {
            coords(p, t.start + q, id[0], id[1], id[2]);
            if (((id[0] + id[1] + id[2] + lo) & 1) != colour) continue;
            level_cell<PT, MODE, REGION, false>(p, id, beta, ctype, D, f, e, nl, Tp, kappa);
        }
    }
}

// r -= A^l e on the cells of the tiles (the level operator: coarse-fine
// ghosts with coarse values 0); e's sibling ghosts must be current.
template <typename PT>
__global__ __launch_bounds__(kBlock) void k_level_res(const int32_t* __restrict__ act,
                                                      const Tile* __restrict__ tiles,
                                                      const PatchInfo* __restrict__ P,
                                                      const ProbScalars* __restrict__ ps,
                                                      const uint8_t* __restrict__ ctype,
                                                      const PT* __restrict__ D,
                                                      const PT* __restrict__ e,
                                                      PT* __restrict__ r, int64_t nl) {
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    int id[3];
    coords(p, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = nat(p, id[0], id[1], id[2]);
    PT dg[2], ns[2];
    level_terms<PT, false>(p, id, c, ps[t.prob].beta, ctype, D, e, nl, dg, ns);
#pragma unroll
    for (int fld = 0; fld < 2; ++fld) {
        const int64_t i = fld * nl + c;
        r[i] -= dg[fld] * e[i] - ns[fld];
    }
}

// ---------------------------------------------------------------------------
// composite operator residual r = f - A^c u on composite cells (covered -> 0)
// with flux form on every face; coarse faces bordering a finer level are
// skipped here and supplied by k_comp_reflux.
// ---------------------------------------------------------------------------

template <typename PT>
__global__ __launch_bounds__(kBlock) void k_comp_res(const int32_t* __restrict__ act, 
    const Tile* __restrict__ tiles, const PatchInfo* __restrict__ P,
    const ProbScalars* __restrict__ ps, const uint8_t* __restrict__ ctype,
    const PT* __restrict__ D, const PT* __restrict__ f, const PT* __restrict__ u,
    PT* __restrict__ r, int64_t nl) {
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    int id[3];
    coords(p, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = nat(p, id[0], id[1], id[2]);
    const int ct = (p.flags & PF_CTYPE) ? ctype[c] : 0;
    if (ct & CT_COVERED) {
        r[c] = PT(0);
        r[c + nl] = PT(0);
        return;
    }
    const double beta = ps[t.prob].beta;
    const int st[3] = {1, p.sy, p.sz};
    // faces classified with selects (operands loaded unconditionally; ghost
    // slots are finite): a physical face carries the Marshak flux of E or
    // nothing, a face whose flux comes from flux matching nothing, any other
    // face the flux D (u_b - u_a) / h
    for (int fld = 0; fld < 2; ++fld) {
        const PT* uf = u + fld * nl;
        const PT uc = uf[c];
        PT div = PT(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const PT* Dd = D + (fld * 3 + d) * nl;
            const PT ih = (PT)p.ih[d];
            const int up = c + st[d];
            const PT Dlo = Dd[c], Dhi = Dd[up];
            const PT ulo = uf[c - st[d]], uhi = uf[up];
            const bool plo = id[d] == 0 && ((p.phys >> (2 * d)) & 1);
            const bool phi = id[d] == p.n[d] - 1 && ((p.phys >> (2 * d + 1)) & 1);
            const bool mlo = (ct >> (2 * d + 1)) & 1;
            const bool mhi = (ct >> (2 * d + 2)) & 1;
            PT lo = (plo || mlo) ? PT(0) : Dlo * (uc - ulo) * ih;
            PT hi = (phi || mhi) ? PT(0) : Dhi * (uhi - uc) * ih;
            if (fld == 0 && ((p.robin >> (2 * d)) & 3)) {      // uniform per patch
                if (plo && ((p.robin >> (2 * d)) & 1))
                    lo = PT(2) * Dlo * uc / (PT(4) * Dlo + (PT)p.h[d]);
                if (phi && ((p.robin >> (2 * d + 1)) & 1))
                    hi = -PT(2) * Dhi * uc / (PT(4) * Dhi + (PT)p.h[d]);
            }
            div += (hi - lo) * ih;
        }
        r[fld * nl + c] = f[fld * nl + c] - (uc - (PT)beta * div);
    }
}

template <typename PT>
__global__ __launch_bounds__(kBlock) void k_comp_reflux(
    const RefluxCell* __restrict__ rc, int n, const RefluxFace* __restrict__ rf,
    const PatchInfo* __restrict__ P, const ProbScalars* __restrict__ ps,
    const PT* __restrict__ D, const PT* __restrict__ u, PT* __restrict__ r, int64_t nl) {
    // four lanes per coarse cell (the quad shares the cell's loop bounds)
    const int t = (blockIdx.x * blockDim.x + threadIdx.x) >> 2;
    const int k = threadIdx.x & 3;
    if (t >= n) return;
    const RefluxCell cell = rc[t];
    const double beta = ps[cell.prob].beta;
    for (int fld = 0; fld < 2; ++fld) {
        const PT* uf = u + fld * nl;
        PT acc = PT(0);
        for (int e = cell.first; e < cell.first + cell.count; ++e) {
            const int face = rf[e].face;
            const int d = face >> 1;
            const bool hi = face & 1;
            const PatchInfo& fp = P[rf[e].fpatch];
            const PT* Dd = D + (fld * 3 + d) * nl;
            const PT ih = (PT)fp.ih[d];
            const int fi = rf[e].fine[k];
            const int g = fi + rf[e].gofs;
            // fine face: lower cell a, upper cell b; its D sits at b's slot
            const int a = hi ? g : fi;
            const int b = hi ? fi : g;
            const PT sum = quad_sum(Dd[b] * (uf[b] - uf[a]) * ih);
            acc += (hi ? PT(1) : PT(-1)) * PT(0.25) * sum * (PT(0.5) * ih);
        }
        if (k == 0) r[fld * nl + cell.c] += (PT)beta * acc;
    }
}

// ---------------------------------------------------------------------------
// transfers
// ---------------------------------------------------------------------------

template <typename PT>
__global__ __launch_bounds__(kBlock) void k_gather(const int32_t* __restrict__ src, int n,
                                                   const PT* __restrict__ x, int64_t nlx,
                                                   PT* __restrict__ y, int64_t nly) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int s = src[t];
    y[t] = x[s];
    y[t + nly] = x[s + nlx];
}

// Trilinear prolongation (weights 3/4, 1/4 per axis) of the shadow block of
// each level-m patch onto its cells: e = P e_coarse, u += e.
template <typename PT>
__global__ __launch_bounds__(kBlock) void k_prolong_level(const int32_t* __restrict__ act, 
    const Tile* __restrict__ tiles, const PatchInfo* __restrict__ P,
    const ShadowPatch* __restrict__ SP, const PT* __restrict__ sh, int64_t nls,
    PT* __restrict__ e, PT* __restrict__ u, int64_t nl) {
    // e: the prolonged correction, kept as the source for the next finer
    // level (NULL on the finest level, where only u is updated); u NULL:
    // only e is written
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    const ShadowPatch sp = SP[t.patch];
    int id[3];
    coords(p, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = nat(p, id[0], id[1], id[2]);
    int q[3], o[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int g = p.lo[d] + id[d];
        q[d] = (g >> 1) - (p.lo[d] >> 1) + 1;      // shadow has a one-cell halo
        o[d] = (g & 1) ? 1 : -1;
    }
    const int sy = sp.m0, sz = sp.m0 * sp.m1;
    const int base = sp.off + q[0] + sy * q[1] + sz * q[2];
    const int ox = o[0], oy = o[1] * sy, oz = o[2] * sz;
    for (int fld = 0; fld < 2; ++fld) {
        const PT* s = sh + fld * nls + base;
        const PT v = PT(27.0 / 64) * s[0] +
                     PT(9.0 / 64) * (s[ox] + s[oy] + s[oz]) +
                     PT(3.0 / 64) * (s[ox + oy] + s[ox + oz] + s[oy + oz]) +
                     PT(1.0 / 64) * s[ox + oy + oz];
        if (e) e[fld * nl + c] = v;
        if (u) u[fld * nl + c] += v;
    }
}

template <typename PT>
__global__ __launch_bounds__(kBlock) void k_copy_level(const int32_t* __restrict__ act,
                                                       const Tile* __restrict__ tiles,
                                                       const PatchInfo* __restrict__ P,
                                                       const PT* __restrict__ x,
                                                       PT* __restrict__ y, int64_t nl) {
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    int id[3];
    coords(p, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = nat(p, id[0], id[1], id[2]);
    y[c] = x[c];
    y[c + nl] = x[c + nl];
}

template <typename PT>
__global__ __launch_bounds__(kBlock) void k_add_level(const int32_t* __restrict__ act, const Tile* __restrict__ tiles,
                                                      const PatchInfo* __restrict__ P,
                                                      const PT* __restrict__ e,
                                                      PT* __restrict__ u, int64_t nl) {
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    int id[3];
    coords(p, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = nat(p, id[0], id[1], id[2]);
    u[c] += e[c];
    u[c + nl] += e[c + nl];
}

// multigrid: f_{g+1} = restriction (mean of 8) of the residual f - A e on
// grid g, right after a pre-smoothing sweep whose last half-sweep relaxed
// colour 1.  Relaxing a cell solves its own equation with its neighbours
// (all of the other colour) held, so the residual of every colour-1 cell is
// zero and only the four colour-0 children of each coarse cell are
// evaluated; the residual is never stored.  Four lanes per coarse cell, one
// child each, summed across the lanes in a fixed order.
// fmap: as in k_mg_coarsen.  The children of a coarse cell start at an even
// level index, so its colour-0 children are those with an even offset sum.
template <typename PT, bool SPLIT = false>   // SPLIT: fine grid's e, f colour-split
__global__ __launch_bounds__(kBlock) void k_mg_res_restrict(const int32_t* __restrict__ act,
    const Tile* __restrict__ tiles, const PatchInfo* __restrict__ Pc,
    const PatchInfo* __restrict__ Pf, const int32_t* __restrict__ fbox,
    const int32_t* __restrict__ fmap,
    const ProbScalars* __restrict__ ps, const uint8_t* __restrict__ ctype,
    const PT* __restrict__ D, const PT* __restrict__ f, const PT* __restrict__ e, int64_t nlf,
    PT* __restrict__ fc, int64_t nlc, const PT* __restrict__ Tp = nullptr) {
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // uniform over the workgroup
    const PatchInfo& pc = Pc[t.patch];
    const double beta = ps[t.prob].beta;
    const PT kappa = (PT)ps[t.prob].kappa;
    // colour-0 children (bit 0: x, 1: y, 2: z offset)
    const int lane = threadIdx.x & 3;
    const int child = lane == 0 ? 0 : (lane == 1 ? 3 : (lane == 2 ? 5 : 6));
    for (int q0 = 0; q0 < t.count; q0 += kBlock / 4) {
        const int q = q0 + ((int)threadIdx.x >> 2);
        const bool live = q < t.count;
        int id[3] = {0, 0, 0};
        if (live) coords(pc, t.start + q, id[0], id[1], id[2]);
        PT v0 = PT(0), v1 = PT(0);
        if (live) {
            const PatchInfo& pf = Pf[fmap ? fmap[nat(pc, id[0], id[1], id[2])] : fbox[t.prob]];
            const int fid[3] = {2 * id[0] + (child & 1) - pf.lo[0],
                                2 * id[1] + ((child >> 1) & 1) - pf.lo[1],
                                2 * id[2] + (child >> 2) - pf.lo[2]};
            const int c = nat(pf, fid[0], fid[1], fid[2]);
            int own = c, enb[6];
            if (SPLIT) split_stencil(pf, fid, own, enb);
            PT dg[2], ns[2];
            level_terms<PT, false, SPLIT>(pf, fid, c, beta, ctype, D, e, nlf, dg, ns, enb, Tp,
                                          kappa);
            v0 = f[own] - (dg[0] * e[own] - ns[0]);
            v1 = f[nlf + own] - (dg[1] * e[nlf + own] - ns[1]);
        }
        v0 += __shfl_xor(v0, 1);
        v1 += __shfl_xor(v1, 1);
        v0 += __shfl_xor(v0, 2);
        v1 += __shfl_xor(v1, 2);
        if (live && lane < 2) {
            const int cc = nat(pc, id[0], id[1], id[2]);
            fc[lane * nlc + cc] = (lane ? v1 : v0) * PT(0.125);
        }
    }
}

// The same with one thread per coarse cell (the first grid, where the
// coarse grid is large): the four children's residuals summed in the
// order of the lane reduction above, (r_0 + r_3) + (r_5 + r_6).
template <typename PT, bool SPLIT = false>
__global__ __launch_bounds__(kBlock) void k_mg_res_restrict1(const int32_t* __restrict__ act,
    const Tile* __restrict__ tiles, const PatchInfo* __restrict__ Pc,
    const PatchInfo* __restrict__ Pf, const int32_t* __restrict__ fbox,
    const int32_t* __restrict__ fmap,
    const ProbScalars* __restrict__ ps, const uint8_t* __restrict__ ctype,
    const PT* __restrict__ D, const PT* __restrict__ f, const PT* __restrict__ e, int64_t nlf,
    PT* __restrict__ fc, int64_t nlc, const PT* __restrict__ Tp = nullptr) {
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& pc = Pc[t.patch];
    const double beta = ps[t.prob].beta;
    const PT kappa = (PT)ps[t.prob].kappa;
    int id[3];
    coords(pc, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int cc = nat(pc, id[0], id[1], id[2]);
    const PatchInfo& pf = Pf[fmap ? fmap[cc] : fbox[t.prob]];
    PT r0[4], r1[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int child = k == 0 ? 0 : (k == 1 ? 3 : (k == 2 ? 5 : 6));
        const int fid[3] = {2 * id[0] + (child & 1) - pf.lo[0],
                            2 * id[1] + ((child >> 1) & 1) - pf.lo[1],
                            2 * id[2] + (child >> 2) - pf.lo[2]};
        const int c = nat(pf, fid[0], fid[1], fid[2]);
        int own = c, enb[6];
        if (SPLIT) split_stencil(pf, fid, own, enb);
        PT dg[2], ns[2];
        level_terms<PT, false, SPLIT>(pf, fid, c, beta, ctype, D, e, nlf, dg, ns, enb, Tp,
                                      kappa);
        r0[k] = f[own] - (dg[0] * e[own] - ns[0]);
        r1[k] = f[nlf + own] - (dg[1] * e[nlf + own] - ns[1]);
    }
    fc[cc] = ((r0[0] + r0[1]) + (r0[2] + r0[3])) * PT(0.125);
    fc[nlc + cc] = ((r1[0] + r1[1]) + (r1[2] + r1[3])) * PT(0.125);
}

// multigrid: e_g += trilinear prolongation of e_{g+1} (copy rule at edges)
template <typename PT>
__global__ __launch_bounds__(kBlock) void k_mg_prolong(const int32_t* __restrict__ act, 
    const Tile* __restrict__ tiles, const PatchInfo* __restrict__ Pf,
    const PatchInfo* __restrict__ Pc, const int32_t* __restrict__ cbox,
    const PT* __restrict__ ec, int64_t nlc, PT* __restrict__ ef, int64_t nlf, int split) {
    // split: ef in colour-split storage
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& pf = Pf[t.patch];
    const PatchInfo& pc = Pc[cbox[t.prob]];
    int id[3];
    coords(pf, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = split ? split_index(pf, id[0] + 1, id[1] + 1, id[2] + 1)
                        : nat(pf, id[0], id[1], id[2]);
    int q[3], nbq[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int I = pf.lo[d] + id[d];            // fine level index (coarse box at 0)
        q[d] = I >> 1;
        const int o = (I & 1) ? 1 : -1;
        nbq[d] = min(max(q[d] + o, 0), pc.n[d] - 1);
    }
    for (int fld = 0; fld < 2; ++fld) {
        const PT* s = ec + fld * nlc;
        PT v = PT(0);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int cc = 0; cc < 2; ++cc) {
                    const PT w = (a ? PT(0.25) : PT(0.75)) * (b ? PT(0.25) : PT(0.75)) *
                                 (cc ? PT(0.25) : PT(0.75));
                    v += w * s[nat(pc, a ? nbq[0] : q[0], b ? nbq[1] : q[1],
                                   cc ? nbq[2] : q[2])];
                }
        ef[fld * nlf + c] += v;
    }
}

// The same on the colour-split base grid (even x extents, boxes at even
// level indices), kBlock / 2 threads per tile: thread q takes the cell pair
// (2q, 2q + 1) of a row, which shares its coarse x cell, reads the twelve
// coarse values the two cells use once and updates both cells, each with
// the weights and summation order above.
template <typename PT>
__global__ __launch_bounds__(kBlock) void k_mg_prolong2(const int32_t* __restrict__ act,
    const Tile* __restrict__ tiles, const PatchInfo* __restrict__ Pf,
    const PatchInfo* __restrict__ Pc, const int32_t* __restrict__ cbox,
    const PT* __restrict__ ec, int64_t nlc, PT* __restrict__ ef, int64_t nlf) {
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    const int a0 = 2 * (int)threadIdx.x;       // tile starts are even
    if (a0 >= t.count) return;
    const PatchInfo& pf = Pf[t.patch];
    const PatchInfo& pc = Pc[cbox[t.prob]];
    int id[3];
    coords(pf, t.start + a0, id[0], id[1], id[2]);    // id[0] even
    int q[3], nbq[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int I = pf.lo[d] + id[d];
        q[d] = I >> 1;
        const int o = (I & 1) ? 1 : -1;
        nbq[d] = min(max(q[d] + o, 0), pc.n[d] - 1);
    }
    const int xm = max(q[0] - 1, 0), xp = min(q[0] + 1, pc.n[0] - 1);
    const int c0 = split_index(pf, id[0] + 1, id[1] + 1, id[2] + 1);
    const int c1 = split_index(pf, id[0] + 2, id[1] + 1, id[2] + 1);
    for (int fld = 0; fld < 2; ++fld) {
        const PT* s = ec + fld * nlc;
        PT R[3][2][2];                         // x: q - 1, q, q + 1; y, z: q, neighbour
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                const int y = b ? nbq[1] : q[1], z = cc ? nbq[2] : q[2];
                R[0][b][cc] = s[nat(pc, xm, y, z)];
                R[1][b][cc] = s[nat(pc, q[0], y, z)];
                R[2][b][cc] = s[nat(pc, xp, y, z)];
            }
#pragma unroll
        for (int k = 0; k < 2; ++k) {          // k = 0: even fine x (neighbour q - 1)
            PT v = PT(0);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int cc = 0; cc < 2; ++cc) {
                        const PT w = (a ? PT(0.25) : PT(0.75)) * (b ? PT(0.25) : PT(0.75)) *
                                     (cc ? PT(0.25) : PT(0.75));
                        v += w * R[a ? (k ? 2 : 0) : 1][b][cc];
                    }
            ef[fld * nlf + (k ? c1 : c0)] += v;
        }
    }
}

// ---------------------------------------------------------------------------
// bottom solve (float64).  The coarsest grid's operator is SPD and banded:
// setup factors it as L L^T (band Cholesky; cells numbered with the longest
// axis slowest, so the half-bandwidth b = N / n_max <= N^(2/3) <= 25 for
// N <= 128 cells) and forms the explicit inverse column by column with two
// banded triangular solves (one thread per column); apply is then a dense
// matrix-vector product with one thread per row.  One workgroup per
// (problem, field).
// ---------------------------------------------------------------------------

constexpr int kBottomMax = 128;     // cells of the coarsest grid
constexpr int kBandLd = kBottomBand; // band row stride in LDS (b + 1 <= 26)

struct BottomOrder {
    int a[3];      // axes, fastest first
    int st[3];     // stride of each (original) axis in the band numbering
    int b;         // half-bandwidth
};

// (written with selects only, so that nothing is indexed at run time)
__device__ __forceinline__ BottomOrder bottom_order(const PatchInfo& p) {
    BottomOrder o;
    const int n0 = p.n[0], n1 = p.n[1], n2 = p.n[2];
    const int slow = (n2 > n0 && n2 > n1) ? 2 : ((n1 > n0) ? 1 : 0);
    o.a[0] = slow == 0 ? 1 : 0;
    o.a[1] = slow == 2 ? 1 : 2;
    o.a[2] = slow;
    const int na0 = slow == 0 ? n1 : n0;                  // extent of axis a[0]
    const int na1 = slow == 2 ? n1 : n2;                  // extent of axis a[1]
    o.st[0] = slow == 0 ? na0 * na1 : 1;
    o.st[1] = slow == 1 ? na0 * na1 : (slow == 0 ? 1 : na0);
    o.st[2] = slow == 2 ? na0 * na1 : na0;
    o.b = na0 * na1;
    return o;
}

__device__ __forceinline__ void bottom_coords(const PatchInfo& p, const BottomOrder& o, int lin,
                                              int id[3]) {
    const int n0 = p.n[0], n1 = p.n[1], n2 = p.n[2];
    const int slow = o.a[2];
    const int na0 = slow == 0 ? n1 : n0;
    const int na1 = slow == 2 ? n1 : n2;
    const int c0 = lin % na0;
    const int r = lin / na0;
    const int c1 = r % na1;
    const int c2 = r / na1;
    // axis a[0] gets c0, a[1] gets c1, a[2] (slow) gets c2
    id[0] = slow == 0 ? c2 : c0;
    id[1] = slow == 1 ? c2 : (slow == 0 ? c0 : c1);
    id[2] = slow == 2 ? c2 : c1;
}

// X block of (problem, field): the N x N inverse, row-major, in the band
// numbering.
constexpr int kBottomThreads = 4 * kBottomMax;   // four threads per inverse column

template <typename PT>
__global__ __launch_bounds__(kBottomThreads) void k_bottom_setup(const int32_t* __restrict__ act, 
    const int32_t* __restrict__ probs, const int32_t* __restrict__ boxes,
    const int32_t* __restrict__ grids, const BottomGrids<PT> G,
    const ProbScalars* __restrict__ ps, const int64_t* __restrict__ boff,
    double* __restrict__ X) {
    __shared__ double A[kBottomMax * kBandLd];   // A(i, i - d) at [i kBandLd + d]
    __shared__ double Li[kBottomMax];            // 1 / diagonal of L
    __shared__ double W[kBottomMax * kBottomMax];   // column j of the inverse at [i N + j]
    const int pi = blockIdx.x >> 1;
    const int fld = blockIdx.x & 1;
    const int prob = probs[pi];
    if (act && !act[prob]) return;
    const int g = grids[pi];                    // the problem's coarsest grid
    const PatchInfo& p = G.P[g][boxes[pi]];
    const PT* __restrict__ D = G.D[g];
    const int64_t nl = G.nl[g];
    const double beta = ps[prob].beta;
    // grid 0 without stored D_T: the T-field coefficients from T
    const PT* __restrict__ T0 = (g == 0 && fld == 1) ? G.T0 : nullptr;
    const PT kappa = (PT)ps[prob].kappa;
    const int N = p.ncell;                      // <= kBottomMax (checked on the host)
    const BottomOrder o = bottom_order(p);
    const int b = o.b;                          // < kBandLd (checked on the host)
    const int tid = threadIdx.x;
    for (int i = tid; i < N * kBandLd; i += blockDim.x) A[i] = 0.0;
    __syncthreads();
    const int st[3] = {1, p.sy, p.sz};
    for (int lin = tid; lin < N; lin += blockDim.x) {
        int id[3];
        bottom_coords(p, o, lin, id);
        const int c = nat(p, id[0], id[1], id[2]);
        double dg = 1.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double bh2 = beta * p.ih[d] * p.ih[d];
            const PT* Dd = D + (fld * 3 + d) * nl;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (id[d] == (s ? p.n[d] - 1 : 0)) {        // grid covers the domain
                    if (fld == 0 && ((p.robin >> (2 * d + s)) & 1)) {
                        const double Dv = (double)Dd[s ? c + st[d] : c];
                        dg += 2.0 * beta * Dv / ((4.0 * Dv + p.h[d]) * p.h[d]);
                    }
                    continue;
                }
                const int nb = s ? c + st[d] : c - st[d];
                const double Dv = T0 ? (double)face_DT(T0[c], T0[nb], kappa)
                                     : (double)Dd[s ? c + st[d] : c];
                const double a = bh2 * Dv;
                dg += a;
                // the lower neighbour's entry; the upper one is that
                // neighbour's lower entry (same face, same coefficient)
                if (s == 0) A[lin * kBandLd + o.st[d]] = -a;
            }
        }
        A[lin * kBandLd] = dg;
    }
    // this thread's (r, q) pair of the trailing-update triangle 1 <= q <= r <= b
    // (b (b + 1) / 2 <= 325 < kBottomThreads)
    int pr, pq;
    {
        int r = 1;
        while (r * (r + 1) / 2 <= tid) ++r;
        pr = (tid < b * (b + 1) / 2) ? r : kBottomMax;      // out of range: never used
        pq = tid - r * (r - 1) / 2 + 1;
    }
    __syncthreads();
    // right-looking band Cholesky: scale column k, update the trailing triangle
    for (int k = 0; k < N; ++k) {
        const double dkk = sqrt(A[k * kBandLd]);
        const double inv = 1.0 / dkk;
        const int m = min(b, N - 1 - k);
        if (tid >= 1 && tid <= m) A[(k + tid) * kBandLd + tid] *= inv;
        if (tid == 0) Li[k] = inv;
        __syncthreads();
        if (pr <= m)
            A[(k + pr) * kBandLd + (pr - pq)] -= A[(k + pr) * kBandLd + pr] * A[(k + pq) * kBandLd + pq];
        __syncthreads();
    }
    // inverse: the four threads 4j..4j+3 (one wavefront holds whole groups)
    // solve L L^T x = e_j into column j of W; each sums every fourth band term
    // and the group adds its partial sums with two cross-lane exchanges, so
    // all four hold the row value and write it (same value, same address).
    // Groups run different row counts: no workgroup barrier inside.
    const int j = tid >> 2, q = tid & 3;
    if (j < N) {
        for (int i = q; i < j; i += 4) W[i * N + j] = 0.0;
        for (int i = j; i < N; ++i) {               // L y = e_j
            const int lmax = min(b, i - j);
            double acc = 0.0;
            for (int l = 1 + q; l <= lmax; l += 4) acc -= A[i * kBandLd + l] * W[(i - l) * N + j];
            acc += __shfl_xor(acc, 1, 64);
            acc += __shfl_xor(acc, 2, 64);
            W[i * N + j] = (((i == j) ? 1.0 : 0.0) + acc) * Li[i];
        }
        for (int i = N - 1; i >= 0; --i) {          // L^T x = y
            const int lmax = min(b, N - 1 - i);
            double acc = 0.0;
            for (int l = 1 + q; l <= lmax; l += 4)
                acc -= A[(i + l) * kBandLd + l] * W[(i + l) * N + j];
            acc += __shfl_xor(acc, 1, 64);
            acc += __shfl_xor(acc, 2, 64);
            W[i * N + j] = (W[i * N + j] + acc) * Li[i];
        }
    }
    __syncthreads();
    double* Xi = X + boff[prob] * 2 + (int64_t)fld * N * N;
    for (int i = tid; i < N * N; i += blockDim.x) Xi[i] = W[i];
}

template <typename PT>
__global__ __launch_bounds__(kBlock) void k_bottom_apply(const int32_t* __restrict__ act, 
    const int32_t* __restrict__ probs, const int32_t* __restrict__ boxes,
    const PatchInfo* __restrict__ P, const int64_t* __restrict__ boff,
    const double* __restrict__ X, const PT* __restrict__ f, PT* __restrict__ e,
    int64_t nl, int split) {
    // split: e and f in colour-split storage
    __shared__ double fv[kBottomMax];
    const int pi = blockIdx.x >> 1;
    const int fld = blockIdx.x & 1;
    const int prob = probs[pi];
    if (act && !act[prob]) return;
    const PatchInfo& p = P[boxes[pi]];
    const int N = p.ncell;
    const BottomOrder o = bottom_order(p);
    const double* Xi = X + boff[prob] * 2 + (int64_t)fld * N * N;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        int id[3];
        bottom_coords(p, o, j, id);
        const int c = split ? split_index(p, id[0] + 1, id[1] + 1, id[2] + 1)
                            : nat(p, id[0], id[1], id[2]);
        fv[j] = (double)f[fld * nl + c];
    }
    __syncthreads();
    // X is symmetric: row i = column i, read with consecutive threads on
    // consecutive addresses
    for (int row = threadIdx.x; row < N; row += blockDim.x) {
        double acc = 0.0;
        for (int jj = 0; jj < N; ++jj) acc += Xi[(int64_t)jj * N + row] * fv[jj];
        int id[3];
        bottom_coords(p, o, row, id);
        const int c = split ? split_index(p, id[0] + 1, id[1] + 1, id[2] + 1)
                            : nat(p, id[0], id[1], id[2]);
        e[fld * nl + c] = (PT)acc;
    }
}

// ---------------------------------------------------------------------------
// P2 and precision conversion
// ---------------------------------------------------------------------------

template <typename PT>
__global__ __launch_bounds__(kBlock) void k_p2(const int32_t* __restrict__ act, const Tile* __restrict__ tiles,
                                               const PatchInfo* __restrict__ P,
                                               const ProbScalars* __restrict__ ps,
                                               const PT* __restrict__ sigma,
                                               const double* __restrict__ z3,
                                               const PT* __restrict__ e,
                                               double* __restrict__ y, int mode,
                                               int transpose, int64_t nl, int split) {
    // split: e in colour-split storage
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    int id[3];
    coords(p, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = nat(p, id[0], id[1], id[2]);
    const double beta = ps[t.prob].beta;
    const double sg = (double)sigma[c];
    const double z = z3[c];
    const double k = mode ? 4.0 : 1.0;
    // [[1 + sigma beta, -k beta z^3], [-sigma beta, 1 + k beta z^3]]  (sigma T^3 = z^3)
    const double a = 1.0 + sg * beta, b = -k * beta * z, cc = -sg * beta, d = 1.0 + k * beta * z;
    const double det = a * d - b * cc;
    const int ce = split ? split_index(p, id[0] + 1, id[1] + 1, id[2] + 1) : c;
    const double eE = (double)e[ce], eT = (double)e[ce + nl];
    if (!transpose) {
        y[c] = (d * eE - b * eT) / det;
        y[c + nl] = (a * eT - cc * eE) / det;
    } else {
        y[c] = (d * eE - cc * eT) / det;
        y[c + nl] = (a * eT - b * eE) / det;
    }
}

// P2^-T applied first (transposed preconditioner): double in, PT out
template <typename PT>
__global__ __launch_bounds__(kBlock) void k_p2t_in(const int32_t* __restrict__ act, const Tile* __restrict__ tiles,
                                                   const PatchInfo* __restrict__ P,
                                                   const ProbScalars* __restrict__ ps,
                                                   const PT* __restrict__ sigma,
                                                   const double* __restrict__ z3,
                                                   const double* __restrict__ w,
                                                   PT* __restrict__ x, int mode, int64_t nl,
                                                   int split) {
    // split: x in colour-split storage
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    int id[3];
    coords(p, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = nat(p, id[0], id[1], id[2]);
    const double beta = ps[t.prob].beta;
    const double sg = (double)sigma[c];
    const double z = z3[c];
    const double k = mode ? 4.0 : 1.0;
    const double a = 1.0 + sg * beta, b = -k * beta * z, cc = -sg * beta, d = 1.0 + k * beta * z;
    const double det = a * d - b * cc;
    const double eE = w[c], eT = w[c + nl];
    const int cx = split ? split_index(p, id[0] + 1, id[1] + 1, id[2] + 1) : c;
    x[cx] = (PT)((d * eE - cc * eT) / det);
    x[cx + nl] = (PT)((a * eT - b * eE) / det);
}

template <typename PT>
// x = wsc_p w (wsc may be NULL: factor 1) rounded to PT
__global__ __launch_bounds__(kBlock) void k_in(const int32_t* __restrict__ act, const Tile* __restrict__ tiles,
                                               const PatchInfo* __restrict__ P,
                                               const double* __restrict__ w,
                                               const double* __restrict__ wsc,
                                               PT* __restrict__ x, int64_t nl, int split) {
    // split: x in colour-split storage
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    const double sc = wsc ? wsc[t.prob] : 1.0;
    int id[3];
    coords(p, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = nat(p, id[0], id[1], id[2]);
    const int cx = split ? split_index(p, id[0] + 1, id[1] + 1, id[2] + 1) : c;
    x[cx] = (PT)(sc * w[c]);
    x[cx + nl] = (PT)(sc * w[c + nl]);
}

template <typename PT>
__global__ __launch_bounds__(kBlock) void k_out(const int32_t* __restrict__ act, const Tile* __restrict__ tiles,
                                                const PatchInfo* __restrict__ P,
                                                const PT* __restrict__ x,
                                                double* __restrict__ y, int64_t nl,
                                                int split) {
    // split: x in colour-split storage
    const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    if (act && !act[t.prob]) return;           // problem not being solved
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    int id[3];
    coords(p, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = nat(p, id[0], id[1], id[2]);
    const int cx = split ? split_index(p, id[0] + 1, id[1] + 1, id[2] + 1) : c;
    y[c] = (double)x[cx];
    y[c + nl] = (double)x[cx + nl];
}

template <typename PT>
__global__ __launch_bounds__(kBlock) void k_fill_t(PT* __restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = PT(0);
}

// plain copy (a kernel rather than a runtime copy, so that captured graphs
// hold only kernel nodes)
template <typename PT>
__global__ __launch_bounds__(kBlock) void k_copy_t(const PT* __restrict__ x,
                                                   PT* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

// ---------------------------------------------------------------------------
// drivers
// ---------------------------------------------------------------------------

template <typename PT>
void PcArrays<PT>::zero(hipStream_t s) const {
    k_fill_t<PT><<<nblocks(2 * D->nl), kBlock, 0, s>>>(e, 2 * D->nl);
    k_fill_t<PT><<<nblocks(2 * D->nl), kBlock, 0, s>>>(u, 2 * D->nl);
    k_fill_t<PT><<<nblocks(2 * D->nl), kBlock, 0, s>>>(r, 2 * D->nl);
    k_fill_t<PT><<<nblocks(2 * D->nl), kBlock, 0, s>>>(f, 2 * D->nl);
    k_fill_t<PT><<<nblocks(6 * D->nl), kBlock, 0, s>>>(Dface, 6 * D->nl);
    for (int g = 1; g <= mg.G; ++g) {
        const int64_t n = mg.len[g];
        k_fill_t<PT><<<nblocks(6 * n), kBlock, 0, s>>>(mg.Dg[g], 6 * n);
        k_fill_t<PT><<<nblocks(2 * n), kBlock, 0, s>>>(mg.eg[g], 2 * n);
        k_fill_t<PT><<<nblocks(2 * n), kBlock, 0, s>>>(mg.fg[g], 2 * n);
    }
}

template <typename PT>
void PcArrays<PT>::setup(hipStream_t s, const double* u_state) const {
    const Dev& d = *D;
    const int ntiles = d.level_tile0[d.nlev];
    k_snapshot<PT><<<ntiles, kBlock, 0, s>>>(d.active, d.tiles, d.patches, d.ps, u_state, d.z3, Dface,
                                            sigma, d.nl, split0 ? Tp : nullptr);
    if (base_smooth) return;                   // no multigrid grids to set up
    for (int g = 1; g <= mg.G; ++g) {
        const PT* Df = (g == 1) ? Dface : mg.Dg[g - 1];
        const int64_t nlf = (g == 1) ? d.nl : mg.len[g - 1];
        const PatchInfo* Pf = (g == 1) ? d.patches : mg.box[g - 1];
        k_mg_coarsen<PT><<<mg.ntiles[g], kBlock, 0, s>>>(d.active, mg.tiles[g], mg.box[g], Pf,
                                                         mg.box_of[g - 1],
                                                         g == 1 ? mg.l0map : nullptr, Df, nlf,
                                                         mg.Dg[g], mg.len[g],
                                                         (g == 1 && split0) ? Tp : nullptr,
                                                         d.ps);
    }
    // every problem's coarsest grid in one launch
    BottomGrids<PT> bg;
    for (int g = 0; g <= mg.G; ++g) {
        bg.P[g] = (g == 0) ? d.patches : mg.box[g];
        bg.D[g] = (g == 0) ? Dface : mg.Dg[g];
        bg.nl[g] = (g == 0) ? d.nl : mg.len[g];
        bg.T0 = split0 ? Tp : nullptr;
    }
    if (mg.nbot_all > 0)
        k_bottom_setup<PT><<<2 * mg.nbot_all, kBottomThreads, 0, s>>>(
            d.active, mg.bot_probs, mg.bot_boxes, mg.bot_grid, bg, d.ps, mg.bottom_off,
            mg.Xbuf);
}

template <typename PT>
void PcArrays<PT>::vcycle(hipStream_t s) const {
    // grid 0 = the level-0 patches: rhs in f, result in e (colour-split
    // storage when split0, native otherwise)
    const Dev& d = *D;
    // one colour of a red-black sweep of grid g (zero: from e = 0)
    auto half_sweep = [&](int g, const PatchInfo* Pg, const PT* Dg, const PT* fg, PT* eg,
                          int64_t nlg, bool zero, int colour) {
        const Tile* tl = mg.smooth_tiles[g];
        const int nt = mg.nsmooth[g];
        if (g == 0 && split0) {
            if (zero)
                k_level<PT, 0, false, true><<<nt, kBlock / 2, 0, s>>>(
                    d.active, tl, Pg, d.ps, d.ctype, Dg, fg, eg, colour, nlg, Tp);
            else
                k_level<PT, 1, false, true><<<nt, kBlock / 2, 0, s>>>(
                    d.active, tl, Pg, d.ps, d.ctype, Dg, fg, eg, colour, nlg, Tp);
        } else if (zero) {
            k_level<PT, 0><<<nt, kBlock / 2, 0, s>>>(d.active, tl, Pg, d.ps, d.ctype, Dg, fg, eg,
                                                     colour, nlg);
        } else {
            k_level<PT, 1><<<nt, kBlock / 2, 0, s>>>(d.active, tl, Pg, d.ps, d.ctype, Dg, fg, eg,
                                                     colour, nlg);
        }
    };
    for (int g = 0; g <= mg.G; ++g) {
        const PatchInfo* Pg = (g == 0) ? d.patches : mg.box[g];
        const int64_t nlg = (g == 0) ? d.nl : mg.len[g];
        PT* eg = (g == 0) ? e : mg.eg[g];
        PT* fg = (g == 0) ? f : mg.fg[g];
        const PT* Dg = (g == 0) ? Dface : mg.Dg[g];
        const bool sp = g == 0 && split0;
        if (mg.nsmooth[g] > 0) {
            // a base grid cut into several boxes: sibling ghosts refreshed
            // after every half-sweep that the next one reads
            const bool sib = g == 0 && mg.multi0;
            for (int it = 0; it < nu_pre; ++it) {
                const int which = it == 0 ? NRD_TIMER_SMOOTH_ZERO : NRD_TIMER_SMOOTH;
                std::pair<hipEvent_t, hipEvent_t> tk{nullptr, nullptr};
                if (g == 0 && clock) tk = clock->tic(which);
                if (sib && it > 0) siblings(s, eg, 0);
                half_sweep(g, Pg, Dg, fg, eg, nlg, it == 0, 0);
                if (sib) siblings(s, eg, 0);
                half_sweep(g, Pg, Dg, fg, eg, nlg, false, 1);
                if (g == 0 && clock) clock->toc(which, tk);
            }
            if (sib) siblings(s, eg, 0);
            if (sp)
                k_mg_res_restrict1<PT, true><<<mg.ntiles[g + 1], kBlock, 0, s>>>(d.active,
                    mg.tiles[g + 1], mg.box[g + 1], Pg, mg.box_of[g], mg.l0map, d.ps, d.ctype,
                    Dg, fg, eg, nlg, mg.fg[g + 1], mg.len[g + 1], Tp);
            else if (g == 0)
                k_mg_res_restrict1<PT><<<mg.ntiles[g + 1], kBlock, 0, s>>>(d.active,
                    mg.tiles[g + 1], mg.box[g + 1], Pg, mg.box_of[g], mg.l0map, d.ps, d.ctype,
                    Dg, fg, eg, nlg, mg.fg[g + 1], mg.len[g + 1]);
            else
                k_mg_res_restrict<PT><<<mg.ntiles[g + 1], kBlock, 0, s>>>(d.active,
                    mg.tiles[g + 1], mg.box[g + 1], Pg, mg.box_of[g],
                    g == 0 ? mg.l0map : nullptr, d.ps, d.ctype, Dg, fg, eg, nlg, mg.fg[g + 1],
                    mg.len[g + 1]);
        }
        if (mg.nbottom[g] > 0)
            k_bottom_apply<PT><<<2 * mg.nbottom[g], kBlock, 0, s>>>(d.active, 
                mg.bottom_probs[g], mg.bottom_boxes[g], Pg, mg.bottom_off, mg.Xbuf, fg, eg,
                nlg, sp ? 1 : 0);
    }
    for (int g = mg.G - 1; g >= 0; --g) {
        if (mg.nsmooth[g] == 0) continue;
        const PatchInfo* Pg = (g == 0) ? d.patches : mg.box[g];
        const int64_t nlg = (g == 0) ? d.nl : mg.len[g];
        PT* eg = (g == 0) ? e : mg.eg[g];
        PT* fg = (g == 0) ? f : mg.fg[g];
        const PT* Dg = (g == 0) ? Dface : mg.Dg[g];
        const Tile* tl = mg.smooth_tiles[g];
        const int nt = mg.nsmooth[g];
        if (g == 0 && split0)
            k_mg_prolong2<PT><<<nt, kBlock / 2, 0, s>>>(d.active, tl, Pg, mg.box[1], mg.box_of[1],
                                                        mg.eg[1], mg.len[1], eg, nlg);
        else
            k_mg_prolong<PT><<<nt, kBlock, 0, s>>>(d.active, tl, Pg, mg.box[g + 1],
                                                  mg.box_of[g + 1], mg.eg[g + 1], mg.len[g + 1],
                                                  eg, nlg, 0);
        const bool sib = g == 0 && mg.multi0;
        for (int it = 0; it < nu_post; ++it) {
            std::pair<hipEvent_t, hipEvent_t> tk{nullptr, nullptr};
            if (g == 0 && clock) tk = clock->tic(NRD_TIMER_SMOOTH);
            if (sib) siblings(s, eg, 0);
            half_sweep(g, Pg, Dg, fg, eg, nlg, false, 0);
            if (sib) siblings(s, eg, 0);
            half_sweep(g, Pg, Dg, fg, eg, nlg, false, 1);
            if (g == 0 && clock) clock->toc(NRD_TIMER_SMOOTH, tk);
        }
    }
}

template <>
void PcArrays<float>::fill_ghosts(hipStream_t s, float* x) const {
    ghost_fill_f(*D, s, x, 2);
}
template <>
void PcArrays<double>::fill_ghosts(hipStream_t s, double* x) const {
    ghost_fill_d(*D, s, x, 2);
}
template <>
void PcArrays<float>::restrict_(hipStream_t s, float* x, int lev_lo) const {
    restrict_f(*D, s, x, 2, lev_lo);
}
template <>
void PcArrays<double>::restrict_(hipStream_t s, double* x, int lev_lo) const {
    restrict_d(*D, s, x, 2, lev_lo);
}
template <>
void PcArrays<float>::siblings(hipStream_t s, float* x, int lev, int lev_hi) const {
    sibling_exchange_f(*D, s, x, 2, lev, lev_hi);
}
template <>
void PcArrays<double>::siblings(hipStream_t s, double* x, int lev, int lev_hi) const {
    sibling_exchange_d(*D, s, x, 2, lev, lev_hi);
}

template <typename PT>
void PcArrays<PT>::composite_residual(hipStream_t s, int lev) const {
    // r = f - A^c u on the composite cells of levels lev and finer; covered r
    // <- restriction of finer r on those levels (what the level-lev solve
    // reads).  The covered cells of u already hold the restriction of u.
    const Dev& d = *D;
    fill_ghosts(s, u);
    const int t0 = d.level_tile0[lev], nt = d.level_tile0[d.nlev] - t0;
    k_comp_res<PT><<<nt, kBlock, 0, s>>>(d.active, d.tiles + t0, d.patches, d.ps, d.ctype,
                                         Dface, f, u, r, d.nl);
    if (d.nrcells > 0)
        k_comp_reflux<PT><<<nblocks(4 * (int64_t)d.nrcells), kBlock, 0, s>>>(
            d.rcells, d.nrcells, d.rfaces, d.patches, d.ps, Dface, u, r, d.nl);
    restrict_(s, r, lev);
}

template <typename PT>
void PcArrays<PT>::smooth_level(hipStream_t s, const PT* rhs, int lev, int sweeps) const {
    // smoothing sweeps on A^l e = rhs from e = 0 over the patches of level
    // lev (red-black Gauss-Seidel, or damped point Jacobi alternating between
    // e and e2), sibling ghosts refreshed before every sweep that reads them
    const Dev& d = *D;
    const int t0 = d.level_tile0[lev], nt = d.level_tile0[lev + 1] - t0;
    const Tile* tl = d.tiles + t0;
    if (fac_smoother == NRD_SMOOTH_JACOBI) {
        k_jacobi<PT, true><<<nt, kBlock, 0, s>>>(d.active, tl, d.patches, d.ps, d.ctype, Dface,
                                                 rhs, e, e, kJacobiOmega, d.nl);
        PT* cur = e;
        PT* nxt = e2;
        for (int it = 1; it < sweeps; ++it) {
            siblings(s, cur, lev);
            k_jacobi<PT, false><<<nt, kBlock, 0, s>>>(d.active, tl, d.patches, d.ps, d.ctype,
                                                      Dface, rhs, cur, nxt, kJacobiOmega, d.nl);
            std::swap(cur, nxt);
        }
        if (cur != e)
            k_copy_level<PT><<<nt, kBlock, 0, s>>>(d.active, tl, d.patches, cur, e, d.nl);
        return;
    }
    if (fac_smoother == NRD_SMOOTH_LINE) {
        const int l0 = level_line0[lev], nl0 = level_line0[lev + 1] - l0;
        const Tile* lt = ltiles + l0;
        k_line<PT, true><<<nl0, kBlock, 0, s>>>(d.active, lt, d.patches, d.ps, d.ctype, Dface,
                                                rhs, e, e2, 0, d.nl);
        siblings(s, e, lev);
        k_line<PT, false><<<nl0, kBlock, 0, s>>>(d.active, lt, d.patches, d.ps, d.ctype, Dface,
                                                 rhs, e, e2, 1, d.nl);
        for (int it = 1; it < sweeps; ++it)
            for (int colour = 0; colour < 2; ++colour) {
                siblings(s, e, lev);
                k_line<PT, false><<<nl0, kBlock, 0, s>>>(d.active, lt, d.patches, d.ps, d.ctype,
                                                         Dface, rhs, e, e2, colour, d.nl);
            }
        return;
    }
    k_level<PT, 0><<<nt, kBlock / 2, 0, s>>>(d.active, tl, d.patches, d.ps, d.ctype, Dface, rhs,
                                             e, 0, d.nl);
    siblings(s, e, lev);
    k_level<PT, 1><<<nt, kBlock / 2, 0, s>>>(d.active, tl, d.patches, d.ps, d.ctype, Dface, rhs,
                                             e, 1, d.nl);
    for (int it = 1; it < sweeps; ++it)
        for (int colour = 0; colour < 2; ++colour) {
            siblings(s, e, lev);
            k_level<PT, 1><<<nt, kBlock / 2, 0, s>>>(d.active, tl, d.patches, d.ps, d.ctype,
                                                     Dface, rhs, e, colour, d.nl);
        }
}

template <typename PT>
void PcArrays<PT>::correct_level(hipStream_t s, int lev) const {
    // u += e on level lev and, by trilinear prolongation level by level, on
    // every finer level; then covered cells of u <- mean of their children
    const Dev& d = *D;
    const int L = d.nlev - 1;
    const int t0 = d.level_tile0[lev], nt = d.level_tile0[lev + 1] - t0;
    k_add_level<PT><<<nt, kBlock, 0, s>>>(d.active, d.tiles + t0, d.patches, e, u, d.nl);
    for (int m = lev + 1; m <= L; ++m) {
        const int a = d.level_shadow0[m], b = d.level_shadow0[m + 1];
        k_gather<PT><<<nblocks(b - a), kBlock, 0, s>>>(shadow_src + a, b - a, e, d.nl,
                                                       shadow + a, shadow_len);
        const int m0 = d.level_tile0[m], mt = d.level_tile0[m + 1] - m0;
        k_prolong_level<PT><<<mt, kBlock, 0, s>>>(d.active, d.tiles + m0, d.patches, shadows,
                                                  shadow, shadow_len, m < L ? e : nullptr, u,
                                                  d.nl);
    }
    restrict_(s, u, 0);
}

template <typename PT>
const PT* PcArrays<PT>::fac(hipStream_t s) const {
    // One FAC V(m,n) cycle from u = 0 for A^c u = f (Alg. 1): m = fac_pre
    // sweeps per level on the down-sweep, the base multigrid V-cycle, n =
    // fac_post sweeps per level on the up-sweep with the composite residual
    // refreshed.  Returns the buffer holding the result: u, or e when there
    // is one level (u = 0 plus the base level's correction is that
    // correction).
    const Dev& d = *D;
    const int L = d.nlev - 1;
    if (L == 0) {
        if (base_smooth)
            smooth_level(s, f, 0, fac_pre);
        else
            vcycle(s);
        return e;
    }
    k_fill_t<PT><<<nblocks(2 * d.nl), kBlock, 0, s>>>(u, 2 * d.nl);
    for (int lev = L; lev >= 0; --lev) {
        if (lev == L) {
            // u = 0: r = f (the finest level has no covered cells)
            k_copy_t<PT><<<nblocks(2 * d.nl), kBlock, 0, s>>>(f, r, 2 * d.nl);
        } else {
            composite_residual(s, lev);     // u was restricted by the last correction
        }
        if (lev > 0 || base_smooth) {
            smooth_level(s, r, lev, fac_pre);
        } else {
            // base level: multigrid V-cycle with rhs f^0 = r on level 0 (the
            // V-cycle only reads its level-0 right-hand side)
            PcArrays<PT> v = *this;
            v.f = r;
            v.vcycle(s);
        }
        correct_level(s, lev);
    }
    for (int lev = 1; fac_post > 0 && lev <= L; ++lev) {
        composite_residual(s, lev);
        smooth_level(s, r, lev, fac_post);
        correct_level(s, lev);
    }
    return u;
}

template <typename PT>
void PcArrays<PT>::smooth_range(hipStream_t s, const PT* rhs, PT* x, int lo, int hi,
                                int sweeps, bool region) const {
    const Dev& d = *D;
    const int t0 = d.level_tile0[lo], nt = d.level_tile0[hi + 1] - t0;
    if (nt <= 0) return;
    const Tile* tl = d.tiles + t0;
    for (int it = 0; it < sweeps; ++it)
        for (int colour = 0; colour < 2; ++colour) {
            if (it > 0 || colour > 0) siblings(s, x, lo, hi);
            const bool zero = it == 0 && colour == 0;
            if (region && zero)
                k_level<PT, 0, true><<<nt, kBlock / 2, 0, s>>>(d.active, tl, d.patches, d.ps,
                                                               d.ctype, Dface, rhs, x, 0, d.nl);
            else if (region)
                k_level<PT, 1, true><<<nt, kBlock / 2, 0, s>>>(d.active, tl, d.patches, d.ps,
                                                               d.ctype, Dface, rhs, x, colour,
                                                               d.nl);
            else if (zero)
                k_level<PT, 0><<<nt, kBlock / 2, 0, s>>>(d.active, tl, d.patches, d.ps, d.ctype,
                                                         Dface, rhs, x, 0, d.nl);
            else
                k_level<PT, 1><<<nt, kBlock / 2, 0, s>>>(d.active, tl, d.patches, d.ps, d.ctype,
                                                         Dface, rhs, x, colour, d.nl);
        }
}

template <typename PT>
const PT* PcArrays<PT>::afacx(hipStream_t s) const {
    // AFACx from u = 0 for A^c u = f: r = f with covered cells the mean of
    // their children; the coarse approximations of every pair (l-1, l) at
    // once in e2 (sweeps on the cells level l covers, the rest 0); their
    // trilinear interpolation s onto every refined level in e; the fine
    // right-hand sides r - A^l s; the fine corrections from zero, every
    // refined level at once (sweeps from s minus s, by linearity); the base
    // correction; each level's correction carried to the finer levels.
    const Dev& d = *D;
    const int L = d.nlev - 1;
    k_copy_t<PT><<<nblocks(2 * d.nl), kBlock, 0, s>>>(f, r, 2 * d.nl);
    restrict_(s, r, 0);
    if (L > 0) {
        smooth_range(s, r, e2, 0, L - 1, fac_pre, true);
        const int a = d.level_shadow0[1], b = d.level_shadow0[L + 1];
        k_gather<PT><<<nblocks(b - a), kBlock, 0, s>>>(shadow_src + a, b - a, e2, d.nl,
                                                       shadow + a, shadow_len);
        const int t1 = d.level_tile0[1], nt1 = d.level_tile0[L + 1] - t1;
        k_prolong_level<PT><<<nt1, kBlock, 0, s>>>(d.active, d.tiles + t1, d.patches, shadows,
                                                   shadow, shadow_len, e, nullptr, d.nl);
        siblings(s, e, 1, L);
        k_level_res<PT><<<nt1, kBlock, 0, s>>>(d.active, d.tiles + t1, d.patches, d.ps, d.ctype,
                                               Dface, e, r, d.nl);
        smooth_range(s, r, e, 1, L, fac_pre, false);
    }
    if (base_smooth) {
        smooth_level(s, r, 0, fac_pre);
    } else {
        PcArrays<PT> v = *this;
        v.f = r;
        v.vcycle(s);
    }
    for (int m = 1; m <= L; ++m) {
        const int a = d.level_shadow0[m], b = d.level_shadow0[m + 1];
        k_gather<PT><<<nblocks(b - a), kBlock, 0, s>>>(shadow_src + a, b - a, e, d.nl,
                                                       shadow + a, shadow_len);
        const int m0 = d.level_tile0[m], mt = d.level_tile0[m + 1] - m0;
        k_prolong_level<PT><<<mt, kBlock, 0, s>>>(d.active, d.tiles + m0, d.patches, shadows,
                                                  shadow, shadow_len, nullptr, e, d.nl);
    }
    restrict_(s, e, 0);
    return e;
}

template <typename PT>
const PT* PcArrays<PT>::p1(hipStream_t s) const {
    return fac_cycle == NRD_FAC_AFACX ? afacx(s) : fac(s);
}

template <typename PT>
void PcArrays<PT>::apply(hipStream_t s, const double* w, double* y, const double* wsc) const {
    const Dev& d = *D;
    const int ntiles = d.level_tile0[d.nlev];
    // with split0 the cycle reads f and returns e in colour-split storage
    const int sp = split0 ? 1 : 0;
    k_in<PT><<<ntiles, kBlock, 0, s>>>(d.active, d.tiles, d.patches, w, wsc, f, d.nl, sp);
    const PT* x = p1(s);
    k_p2<PT><<<ntiles, kBlock, 0, s>>>(d.active, d.tiles, d.patches, d.ps, sigma, d.z3, x, y,
                                       p2_mode, 0, d.nl, sp);
}

template <typename PT>
void PcArrays<PT>::apply_transpose(hipStream_t s, const double* w, double* y) const {
    const Dev& d = *D;
    const int ntiles = d.level_tile0[d.nlev];
    const int sp = split0 ? 1 : 0;
    k_p2t_in<PT><<<ntiles, kBlock, 0, s>>>(d.active, d.tiles, d.patches, d.ps, sigma, d.z3, w, f,
                                           p2_mode, d.nl, sp);
    const PT* x = p1(s);
    k_out<PT><<<ntiles, kBlock, 0, s>>>(d.active, d.tiles, d.patches, x, y, d.nl, sp);
}

template struct PcArrays<float>;
template struct PcArrays<double>;

}  // namespace nrd
