// Host construction of the hierarchy tables (paper Sec. 3.2, 3.2.1).
//
// Every kind of ghost region the paper classifies as a coarse-fine boundary
// fragment (face, edge, corner, concave, sibling) reduces here to one entry
// per ghost cell: a copy (physical or sibling) or a coarse-fine
// interpolation with four coarse sources and one fine source.  Sources are
// always interior cells, so one launch fills every ghost of every level.
#include <algorithm>
#include <cstring>
#include <sstream>

#include "nrd_internal.h"

namespace nrd {

void Locator::build(const std::vector<HostBox>& all,
                    const std::vector<int32_t>& ids, const int32_t N_[3]) {
    boxes = &all;
    for (int d = 0; d < 3; ++d) {
        N[d] = N_[d];
        nb[d] = (N[d] + B - 1) / B;
    }
    buckets.assign((size_t)nb[0] * nb[1] * nb[2], {});
    for (int32_t id : ids) {
        const HostBox& b = all[id];
        int32_t a0[3], a1[3];
        for (int d = 0; d < 3; ++d) {
            a0[d] = b.lo[d] / B;
            a1[d] = (b.hi[d] - 1) / B;
        }
        for (int k = a0[2]; k <= a1[2]; ++k)
            for (int j = a0[1]; j <= a1[1]; ++j)
                for (int i = a0[0]; i <= a1[0]; ++i)
                    buckets[((size_t)k * nb[1] + j) * nb[0] + i].push_back(id);
    }
}

int32_t Locator::find(int32_t i, int32_t j, int32_t k) const {
    if (i < 0 || j < 0 || k < 0 || i >= N[0] || j >= N[1] || k >= N[2]) return -1;
    const auto& v = buckets[((size_t)(k / B) * nb[1] + j / B) * nb[0] + i / B];
    for (int32_t id : v) {
        const HostBox& b = (*boxes)[id];
        if (i >= b.lo[0] && i < b.hi[0] && j >= b.lo[1] && j < b.hi[1] &&
            k >= b.lo[2] && k < b.hi[2])
            return id;
    }
    return -1;
}

namespace {

inline int32_t nidx(const PatchInfo& p, int i, int j, int k) {
    return p.off + (i + 1) + p.sy * (j + 1) + p.sz * (k + 1);
}

inline int64_t intersect(const int32_t alo[3], const int32_t ahi[3],
                         const int32_t blo[3], const int32_t bhi[3]) {
    int64_t v = 1;
    for (int d = 0; d < 3; ++d) {
        int32_t l = std::max(alo[d], blo[d]);
        int32_t h = std::min(ahi[d], bhi[d]);
        if (h <= l) return 0;
        v *= (h - l);
    }
    return v;
}

}  // namespace

int32_t default_zchunk(const int32_t n[3], int32_t variant) {
    // staged planes: long runs amortise the first plane's staging and its
    // repeated z face; register-marching: short runs keep enough waves
    // resident to hide load latency
    if (variant == 3) return 16;
    return n[0] * n[1] >= 4096 ? 4 : 8;
}

int32_t staged_len(const PatchInfo& p, int32_t s0, int32_t cnt) {
    const int32_t nx = p.n[0], sy = p.sy;
    const int32_t la = s0, lb = s0 + cnt - 1;
    const int32_t g0 = (la % nx + 1) + sy * (la / nx);
    return (lb % nx + 1) + sy * (lb / nx + 2) - g0 + 1;
}

bool patch_planes(const PatchInfo& p, int32_t b, int32_t kc, int32_t run, int32_t max_span,
                  std::vector<STile>& out) {
    const int32_t plane = p.n[0] * p.n[1];
    const int32_t ch = std::max(1, kc);
    // a tile's cells are owned one per thread of a 256-thread workgroup
    if (run <= 0 || run > kStageCells) return false;
    int32_t r = run;
    if (max_span > 0) {
        // shorten the runs of this patch until every staged slice fits
        for (;; r -= 64) {
            if (r <= 0) return false;
            bool fits = true;
            for (int32_t s0 = 0; s0 < plane && fits; s0 += r)
                fits = staged_len(p, s0, std::min(r, plane - s0)) <= max_span;
            if (fits) break;
        }
    }
    for (int32_t k0 = 0; k0 < p.n[2]; k0 += ch)
        for (int32_t s0 = 0; s0 < plane; s0 += r)
            out.push_back({b, p.prob, s0, std::min(r, plane - s0), k0, std::min(p.n[2], k0 + ch),
                           {0, 0}});
    return true;
}

bool build_planes(Tables& t, const std::vector<int32_t>& kc, int32_t run, int32_t max_span) {
    return build_planes(t, kc, std::vector<int32_t>(t.nbox, run), max_span);
}

bool build_planes(Tables& t, const std::vector<int32_t>& kc, const std::vector<int32_t>& run,
                  int32_t max_span) {
    t.stiles.clear();
    t.level_stile0.assign(t.nlev + 1, 0);
    t.patch_stile0.assign(t.nbox + 1, 0);
    std::vector<std::vector<STile>> per(t.nbox);
    for (int b = 0; b < t.nbox; ++b)
        if (!patch_planes(t.patches[b], b, kc[b], run[b], max_span, per[b])) return false;
    for (int l = 0; l < t.nlev; ++l) {
        t.level_stile0[l] = (int32_t)t.stiles.size();
        for (int b = 0; b < t.nbox; ++b) {
            if (t.boxes[b].level != l) continue;
            t.patch_stile0[b] = (int32_t)t.stiles.size();
            t.stiles.insert(t.stiles.end(), per[b].begin(), per[b].end());
        }
    }
    t.level_stile0[t.nlev] = (int32_t)t.stiles.size();
    t.patch_stile0[t.nbox] = (int32_t)t.stiles.size();
    return true;
}

nrd_status build_tables(const nrd_problem* probs, int32_t nprob,
                        const nrd_box* boxes, int32_t nbox, int32_t tile_cells,
                        int32_t vtile_cells, Tables& t, std::string& msg) {
    std::ostringstream err;
    if (nprob <= 0 || nbox <= 0 || !probs || !boxes) {
        msg = "need at least one problem and one box";
        return NRD_EINVAL;
    }
    t.nprob = nprob;
    t.nbox = nbox;
    t.probs.assign(probs, probs + nprob);
    for (int p = 0; p < nprob; ++p) {
        const nrd_problem& pr = probs[p];
        for (int d = 0; d < 3; ++d) {
            if (pr.base_n[d] <= 0 || !(pr.hi[d] > pr.lo[d])) {
                err << "problem " << p << ": bad base grid or domain";
                msg = err.str();
                return NRD_EINVAL;
            }
        }
        if (!(pr.kappa > 0)) {
            err << "problem " << p << ": kappa must be positive";
            msg = err.str();
            return NRD_EINVAL;
        }
        for (int f = 0; f < 6; ++f)
            if (pr.bc_E[f] != 0 && pr.bc_E[f] != 1) {
                err << "problem " << p << ": bc_E must be 0 or 1";
                msg = err.str();
                return NRD_EINVAL;
            }
    }
    t.boxes.resize(nbox);
    t.nlev = 0;
    for (int b = 0; b < nbox; ++b) {
        const nrd_box& x = boxes[b];
        HostBox& hb = t.boxes[b];
        hb.prob = x.problem;
        hb.level = x.level;
        for (int d = 0; d < 3; ++d) {
            hb.lo[d] = x.lo[d];
            hb.hi[d] = x.hi[d];
        }
        if (x.problem < 0 || x.problem >= nprob || x.level < 0 || x.level > 20) {
            err << "box " << b << ": bad problem or level";
            msg = err.str();
            return NRD_EINVAL;
        }
        for (int d = 0; d < 3; ++d)
            if (x.hi[d] <= x.lo[d]) {
                err << "box " << b << ": empty";
                msg = err.str();
                return NRD_EINVAL;
            }
        if (b > 0) {
            const nrd_box& y = boxes[b - 1];
            if (x.problem < y.problem ||
                (x.problem == y.problem && x.level < y.level)) {
                err << "boxes must be ordered by (problem, level); box " << b;
                msg = err.str();
                return NRD_EINVAL;
            }
        }
        t.nlev = std::max(t.nlev, x.level + 1);
    }
    t.level_patches.assign(nprob, std::vector<std::vector<int32_t>>(t.nlev));
    t.prob_patches.assign(nprob, {});
    for (int b = 0; b < nbox; ++b) {
        t.level_patches[boxes[b].problem][boxes[b].level].push_back(b);
        t.prob_patches[boxes[b].problem].push_back(b);
    }
    auto Nlev = [&](int p, int l, int32_t N[3]) {
        for (int d = 0; d < 3; ++d) N[d] = probs[p].base_n[d] << l;
    };
    // level structure, alignment, bounds, overlap
    for (int p = 0; p < nprob; ++p) {
        const auto& L = t.level_patches[p];
        // level 0: non-overlapping boxes inside the base grid that tile it
        int64_t vol0 = 0, base = 1;
        for (int d = 0; d < 3; ++d) base *= probs[p].base_n[d];
        for (size_t a = 0; a < L[0].size(); ++a) {
            const HostBox& x = t.boxes[L[0][a]];
            int64_t v = 1;
            for (int d = 0; d < 3; ++d) {
                if (x.lo[d] < 0 || x.hi[d] > probs[p].base_n[d]) {
                    err << "box " << L[0][a] << " outside the base grid";
                    msg = err.str();
                    return NRD_ENESTING;
                }
                v *= x.hi[d] - x.lo[d];
            }
            vol0 += v;
            for (size_t c = a + 1; c < L[0].size(); ++c)
                if (intersect(x.lo, x.hi, t.boxes[L[0][c]].lo, t.boxes[L[0][c]].hi) > 0) {
                    err << "boxes " << L[0][a] << " and " << L[0][c] << " overlap";
                    msg = err.str();
                    return NRD_ENESTING;
                }
        }
        if (L[0].empty() || vol0 != base) {
            err << "problem " << p << ": the level-0 boxes must tile the base grid";
            msg = err.str();
            return NRD_ENESTING;
        }
        for (int l = 1; l < t.nlev; ++l) {
            if (!L[l].empty() && L[l - 1].empty()) {
                err << "problem " << p << ": level " << l << " without level " << l - 1;
                msg = err.str();
                return NRD_ENESTING;
            }
            int32_t N[3];
            Nlev(p, l, N);
            for (size_t a = 0; a < L[l].size(); ++a) {
                const HostBox& x = t.boxes[L[l][a]];
                for (int d = 0; d < 3; ++d) {
                    if ((x.lo[d] & 1) || (x.hi[d] & 1)) {
                        err << "box " << L[l][a] << " not aligned to ratio 2";
                        msg = err.str();
                        return NRD_ENESTING;
                    }
                    if (x.lo[d] < 0 || x.hi[d] > N[d]) {
                        err << "box " << L[l][a] << " outside its level";
                        msg = err.str();
                        return NRD_ENESTING;
                    }
                }
                for (size_t c = a + 1; c < L[l].size(); ++c) {
                    const HostBox& y = t.boxes[L[l][c]];
                    if (intersect(x.lo, x.hi, y.lo, y.hi) > 0) {
                        err << "boxes " << L[l][a] << " and " << L[l][c] << " overlap";
                        msg = err.str();
                        return NRD_ENESTING;
                    }
                }
                // proper nesting: coarsened box grown by one coarse cell,
                // clipped to the domain, must be covered by level l-1
                int32_t Nc[3], rlo[3], rhi[3];
                Nlev(p, l - 1, Nc);
                int64_t need = 1;
                for (int d = 0; d < 3; ++d) {
                    rlo[d] = std::max(x.lo[d] / 2 - 1, 0);
                    rhi[d] = std::min(x.hi[d] / 2 + 1, Nc[d]);
                    need *= (rhi[d] - rlo[d]);
                }
                int64_t got = 0;
                for (int32_t cb : L[l - 1]) {
                    const HostBox& y = t.boxes[cb];
                    got += intersect(rlo, rhi, y.lo, y.hi);
                }
                if (got != need) {
                    err << "box " << L[l][a] << " is not properly nested in level " << l - 1;
                    msg = err.str();
                    return NRD_ENESTING;
                }
            }
        }
    }
    // patch table
    t.patches.resize(nbox);
    t.compact_off.resize(nbox);
    int64_t off = 0, coff = 0;
    for (int b = 0; b < nbox; ++b) {
        const HostBox& x = t.boxes[b];
        PatchInfo& pi = t.patches[b];
        std::memset(&pi, 0, sizeof(pi));
        int32_t N[3];
        Nlev(x.prob, x.level, N);
        for (int d = 0; d < 3; ++d) {
            pi.n[d] = x.hi[d] - x.lo[d];
            pi.lo[d] = x.lo[d];
            pi.h[d] = (probs[x.prob].hi[d] - probs[x.prob].lo[d]) / N[d];
            pi.ih[d] = 1.0 / pi.h[d];
        }
        pi.sy = pi.n[0] + 2;
        pi.sz = (pi.n[0] + 2) * (pi.n[1] + 2);
        pi.off = (int32_t)off;
        pi.prob = x.prob;
        pi.level = x.level;
        pi.vol = pi.h[0] * pi.h[1] * pi.h[2];
        pi.ncell = pi.n[0] * pi.n[1] * pi.n[2];
        for (int d = 0; d < 3; ++d) {
            if (x.lo[d] == 0) pi.phys |= 1 << (2 * d);
            if (x.hi[d] == N[d]) pi.phys |= 1 << (2 * d + 1);
        }
        for (int f = 0; f < 6; ++f)
            if ((pi.phys >> f & 1) && probs[x.prob].bc_E[f] == 1) pi.robin |= 1 << f;
        if (pi.phys != 63) pi.flags |= PF_CTYPE;
        off += (int64_t)pi.sz * (pi.n[2] + 2);
        t.compact_off[b] = coff;
        coff += pi.ncell;
    }
    if (2 * off >= (int64_t)INT32_MAX) {
        msg = "hierarchy too large for 32-bit native indices";
        return NRD_EINVAL;
    }
    t.nl = off;
    t.ncells = coff;
    t.ctype.assign(t.nl, 0);
    // locators per (problem, level)
    std::vector<std::vector<Locator>> loc(nprob, std::vector<Locator>(t.nlev));
    for (int p = 0; p < nprob; ++p)
        for (int l = 0; l < t.nlev; ++l) {
            int32_t N[3];
            Nlev(p, l, N);
            loc[p][l].build(t.boxes, t.level_patches[p][l], N);
        }
    auto covered = [&](int p, int l, int32_t i, int32_t j, int32_t k) {
        if (l + 1 >= t.nlev) return false;
        return loc[p][l + 1].find(2 * i, 2 * j, 2 * k) >= 0;
    };
    // covered cells and restriction tables
    t.sync.assign(t.nlev, {});
    for (int b = 0; b < nbox; ++b) {
        const HostBox& x = t.boxes[b];
        if (x.level + 1 >= t.nlev) continue;
        PatchInfo& pi = t.patches[b];
        for (int32_t cb : t.level_patches[x.prob][x.level + 1]) {
            const HostBox& y = t.boxes[cb];
            const PatchInfo& fp = t.patches[cb];
            int32_t clo[3], chi[3];
            for (int d = 0; d < 3; ++d) {
                clo[d] = std::max(y.lo[d] / 2, x.lo[d]);
                chi[d] = std::min(y.hi[d] / 2, x.hi[d]);
            }
            if (clo[0] >= chi[0] || clo[1] >= chi[1] || clo[2] >= chi[2]) continue;
            pi.flags |= PF_COVERED | PF_CTYPE;
            for (int k = clo[2]; k < chi[2]; ++k)
                for (int j = clo[1]; j < chi[1]; ++j)
                    for (int i = clo[0]; i < chi[0]; ++i) {
                        int32_t c = nidx(pi, i - x.lo[0], j - x.lo[1], k - x.lo[2]);
                        t.ctype[c] |= CT_COVERED;
                        SyncEntry e;
                        e.dst = c;
                        e.src = nidx(fp, 2 * i - y.lo[0], 2 * j - y.lo[1], 2 * k - y.lo[2]);
                        e.sy = fp.sy;
                        e.sz = fp.sz;
                        t.sync[x.level].push_back(e);
                    }
        }
    }
    // ghosts
    std::vector<std::vector<GhostCopy>> sib_by_level(t.nlev);
    for (int b = 0; b < nbox; ++b) {
        const HostBox& x = t.boxes[b];
        const PatchInfo& pi = t.patches[b];
        int32_t N[3], Nc[3];
        Nlev(x.prob, x.level, N);
        if (x.level > 0) Nlev(x.prob, x.level - 1, Nc);
        for (int d = 0; d < 3; ++d) {
            int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
            if (t1 > t2) std::swap(t1, t2);
            for (int s = 0; s < 2; ++s) {
                bool phys = pi.phys >> (2 * d + s) & 1;
                for (int b2 = 0; b2 < pi.n[t2]; ++b2)
                    for (int a = 0; a < pi.n[t1]; ++a) {
                        int32_t L[3], G[3];
                        L[d] = s == 0 ? -1 : pi.n[d];
                        L[t1] = a;
                        L[t2] = b2;
                        for (int q = 0; q < 3; ++q) G[q] = x.lo[q] + L[q];
                        int32_t I[3] = {L[0], L[1], L[2]};
                        I[d] = s == 0 ? 0 : pi.n[d] - 1;
                        int32_t gidx = nidx(pi, L[0], L[1], L[2]);
                        int32_t inner = nidx(pi, I[0], I[1], I[2]);
                        if (phys) {
                            // physical faces are evaluated from the cell itself
                            // (zero flux or Marshak); no kernel reads these ghosts
                            t.ctype[gidx] = GK_PHYS;
                            continue;
                        }
                        int32_t o = loc[x.prob][x.level].find(G[0], G[1], G[2]);
                        if (o >= 0) {
                            const PatchInfo& op = t.patches[o];
                            const HostBox& ob = t.boxes[o];
                            int32_t src = nidx(op, G[0] - ob.lo[0], G[1] - ob.lo[1],
                                               G[2] - ob.lo[2]);
                            t.gcopy.push_back({gidx, src});
                            sib_by_level[x.level].push_back({gidx, src});
                            t.ctype[gidx] = GK_SIB;
                            continue;
                        }
                        if (x.level == 0) {
                            err << "box " << b << ": level-0 ghost without owner";
                            msg = err.str();
                            return NRD_ENESTING;
                        }
                        GhostCF e;
                        e.dst = gidx;
                        int32_t P[3] = {G[0] >> 1, G[1] >> 1, G[2] >> 1};
                        int o1 = (G[t1] & 1) ? 1 : -1;
                        int o2 = (G[t2] & 1) ? 1 : -1;
                        for (int q = 0; q < 4; ++q) {
                            int32_t Q[3] = {P[0], P[1], P[2]};
                            if (q & 1) Q[t1] += o1;
                            if (q & 2) Q[t2] += o2;
                            for (int r = 0; r < 3; ++r)
                                Q[r] = std::min(std::max(Q[r], 0), Nc[r] - 1);
                            int32_t co = loc[x.prob][x.level - 1].find(Q[0], Q[1], Q[2]);
                            if (co < 0) {
                                err << "box " << b << ": coarse source outside level "
                                    << x.level - 1 << " (nesting)";
                                msg = err.str();
                                return NRD_ENESTING;
                            }
                            const HostBox& cbx = t.boxes[co];
                            e.src[q] = nidx(t.patches[co], Q[0] - cbx.lo[0],
                                            Q[1] - cbx.lo[1], Q[2] - cbx.lo[2]);
                        }
                        e.src[4] = inner;
                        t.gcf.push_back(e);
                        t.gcf_prob.push_back(x.prob);
                        t.ctype[gidx] = GK_CF;
                    }
            }
        }
    }
    t.level_sib0.assign(t.nlev + 1, 0);
    for (int l = 0; l < t.nlev; ++l) {
        t.level_sib0[l] = (int32_t)t.sib.size();
        t.sib.insert(t.sib.end(), sib_by_level[l].begin(), sib_by_level[l].end());
    }
    t.level_sib0[t.nlev] = (int32_t)t.sib.size();
    // coarse faces bordering a finer level: flux matching entries
    for (int p = 0; p < nprob; ++p)
        for (int l = 0; l + 1 < t.nlev; ++l) {
            int32_t N[3];
            Nlev(p, l, N);
            for (int32_t cb : t.level_patches[p][l + 1]) {
                const HostBox& y = t.boxes[cb];
                int32_t clo[3], chi[3];
                for (int d = 0; d < 3; ++d) {
                    clo[d] = y.lo[d] / 2;
                    chi[d] = y.hi[d] / 2;
                }
                for (int d = 0; d < 3; ++d) {
                    int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
                    if (t1 > t2) std::swap(t1, t2);
                    for (int s = 0; s < 2; ++s) {
                        // coarse cells just outside the coarsened child box
                        int32_t cd = s == 0 ? clo[d] - 1 : chi[d];
                        if (cd < 0 || cd >= N[d]) continue;
                        for (int32_t v = clo[t2]; v < chi[t2]; ++v)
                            for (int32_t u = clo[t1]; u < chi[t1]; ++u) {
                                int32_t C[3];
                                C[d] = cd;
                                C[t1] = u;
                                C[t2] = v;
                                if (covered(p, l, C[0], C[1], C[2])) continue;
                                int32_t o = loc[p][l].find(C[0], C[1], C[2]);
                                if (o < 0) {
                                    msg = "coarse neighbour of a fine box is not on the "
                                          "coarse level (nesting)";
                                    return NRD_ENESTING;
                                }
                                const HostBox& ob = t.boxes[o];
                                const PatchInfo& op = t.patches[o];
                                RefluxFace rf;
                                rf.c = nidx(op, C[0] - ob.lo[0], C[1] - ob.lo[1],
                                            C[2] - ob.lo[2]);
                                // the covered neighbour lies at +d for s == 0
                                int face_s = (s == 0) ? 1 : 0;
                                rf.face = 2 * d + face_s;
                                const PatchInfo& fp = t.patches[cb];
                                int32_t fd = (face_s == 1) ? 2 * (cd + 1) : 2 * (cd - 1) + 1;
                                int q = 0;
                                for (int bb = 0; bb < 2; ++bb)
                                    for (int aa = 0; aa < 2; ++aa) {
                                        int32_t F[3];
                                        F[d] = fd;
                                        F[t1] = 2 * u + aa;
                                        F[t2] = 2 * v + bb;
                                        rf.fine[q++] = nidx(fp, F[0] - y.lo[0], F[1] - y.lo[1],
                                                            F[2] - y.lo[2]);
                                    }
                                int32_t stride = d == 0 ? 1 : (d == 1 ? fp.sy : fp.sz);
                                rf.gofs = (face_s == 1) ? -stride : stride;
                                rf.fpatch = cb;
                                t.rfaces.push_back(rf);
                                t.ctype[rf.c] |= (uint8_t)(1u << (rf.face + 1));
                                t.patches[o].flags |= PF_CTYPE;
                            }
                    }
                }
            }
        }
    std::stable_sort(t.rfaces.begin(), t.rfaces.end(),
                     [](const RefluxFace& a, const RefluxFace& b) { return a.c < b.c; });
    for (size_t i = 0; i < t.rfaces.size();) {
        size_t j = i;
        while (j < t.rfaces.size() && t.rfaces[j].c == t.rfaces[i].c) ++j;
        RefluxCell rc;
        rc.c = t.rfaces[i].c;
        rc.first = (int32_t)i;
        rc.count = (int32_t)(j - i);
        rc.prob = t.patches[t.rfaces[i].fpatch].prob;
        t.rcells.push_back(rc);
        i = j;
    }
    // tiles (stencil, sorted by level) and reduction tiles (by problem)
    t.level_tile0.assign(t.nlev + 1, 0);
    t.patch_tiles.assign(nbox, {});
    for (int l = 0; l < t.nlev; ++l) {
        t.level_tile0[l] = (int32_t)t.tiles.size();
        for (int b = 0; b < nbox; ++b) {
            if (t.boxes[b].level != l) continue;
            const PatchInfo& pi = t.patches[b];
            for (int32_t s0 = 0; s0 < pi.ncell; s0 += tile_cells) {
                Tile tl{b, s0, std::min(tile_cells, pi.ncell - s0), pi.prob};
                t.tiles.push_back(tl);
                t.patch_tiles[b].push_back(tl);
            }
        }
    }
    t.level_tile0[t.nlev] = (int32_t)t.tiles.size();
    {
        std::vector<int32_t> kc(nbox);
        for (int b = 0; b < nbox; ++b) kc[b] = default_zchunk(t.patches[b].n, 1);
        build_planes(t, kc, 256);   // default stencil variant: plane marching
    }
    t.prob_vtile0.assign(nprob + 1, 0);
    for (int p = 0; p < nprob; ++p) {
        t.prob_vtile0[p] = (int32_t)t.vtiles.size();
        for (int32_t b : t.prob_patches[p]) {
            const PatchInfo& pi = t.patches[b];
            for (int32_t s0 = 0; s0 < pi.ncell; s0 += vtile_cells)
                t.vtiles.push_back({b, s0, std::min(vtile_cells, pi.ncell - s0), p});
        }
    }
    t.prob_vtile0[nprob] = (int32_t)t.vtiles.size();
    // shadows for prolongation onto level >= 1 patches, grouped by level
    t.shadow.assign(nbox, ShadowPatch{0, 0, 0, 0});
    t.level_shadow0.assign(t.nlev + 1, 0);
    for (int l = 0; l < t.nlev; ++l) {
        t.level_shadow0[l] = (int32_t)t.shadow_src.size();
        if (l == 0) continue;
        for (int b = 0; b < nbox; ++b) {
            const HostBox& x = t.boxes[b];
            if (x.level != l) continue;
            int32_t Nc[3];
            Nlev(x.prob, l - 1, Nc);
            ShadowPatch sp;
            sp.off = (int32_t)t.shadow_src.size();
            sp.m0 = x.hi[0] / 2 - x.lo[0] / 2 + 2;
            sp.m1 = x.hi[1] / 2 - x.lo[1] / 2 + 2;
            sp.m2 = x.hi[2] / 2 - x.lo[2] / 2 + 2;
            t.shadow[b] = sp;
            for (int k = 0; k < sp.m2; ++k)
                for (int j = 0; j < sp.m1; ++j)
                    for (int i = 0; i < sp.m0; ++i) {
                        int32_t Q[3] = {x.lo[0] / 2 - 1 + i, x.lo[1] / 2 - 1 + j,
                                        x.lo[2] / 2 - 1 + k};
                        for (int r = 0; r < 3; ++r)
                            Q[r] = std::min(std::max(Q[r], 0), Nc[r] - 1);
                        int32_t co = loc[x.prob][l - 1].find(Q[0], Q[1], Q[2]);
                        if (co < 0) {
                            msg = "prolongation source outside the coarser level (nesting)";
                            return NRD_ENESTING;
                        }
                        const HostBox& cbx = t.boxes[co];
                        t.shadow_src.push_back(nidx(t.patches[co], Q[0] - cbx.lo[0],
                                                    Q[1] - cbx.lo[1], Q[2] - cbx.lo[2]));
                    }
        }
    }
    t.level_shadow0[t.nlev] = (int32_t)t.shadow_src.size();
    t.shadow_len = (int64_t)t.shadow_src.size();
    // base multigrid grids below level 0
    t.prob_mgdepth.assign(nprob, 0);
    int32_t maxdepth = 0;
    for (int p = 0; p < nprob; ++p) {
        int32_t n[3] = {probs[p].base_n[0], probs[p].base_n[1], probs[p].base_n[2]};
        int32_t depth = 0;
        while (can_coarsen(n)) {
            for (int d = 0; d < 3; ++d) n[d] /= 2;
            ++depth;
        }
        t.prob_mgdepth[p] = depth;
        maxdepth = std::max(maxdepth, depth);
        // a base grid cut into several boxes: the multigrid below it works on
        // the whole base grid coarsened once, whose cells must each have
        // their eight children in one level-0 box
        if (t.level_patches[p][0].size() > 1) {
            if (depth == 0) {
                msg = "a base grid cut into several level-0 boxes must coarsen at least once "
                      "(even extents above 5)";
                return NRD_EUNSUPPORTED;
            }
            for (int32_t b : t.level_patches[p][0])
                for (int d = 0; d < 3; ++d)
                    if ((t.boxes[b].lo[d] & 1) || (t.boxes[b].hi[d] & 1)) {
                        msg = "level-0 boxes of a base grid cut into several boxes must start "
                              "and end on even planes";
                        return NRD_EUNSUPPORTED;
                    }
        }
    }
    t.mg.assign(maxdepth + 1, MGLevel());
    for (int g = 1; g <= maxdepth; ++g) {
        MGLevel& M = t.mg[g];
        int64_t moff = 0;
        for (int p = 0; p < nprob; ++p) {
            if (t.prob_mgdepth[p] < g) continue;
            PatchInfo pi;
            std::memset(&pi, 0, sizeof(pi));
            for (int d = 0; d < 3; ++d) {
                pi.n[d] = probs[p].base_n[d] >> g;
                pi.h[d] = (probs[p].hi[d] - probs[p].lo[d]) / pi.n[d];
                pi.ih[d] = 1.0 / pi.h[d];
            }
            pi.sy = pi.n[0] + 2;
            pi.sz = (pi.n[0] + 2) * (pi.n[1] + 2);
            pi.off = (int32_t)moff;
            pi.prob = p;
            pi.level = -g;
            pi.phys = 63;
            for (int f = 0; f < 6; ++f)
                if (probs[p].bc_E[f] == 1) pi.robin |= 1 << f;
            pi.vol = pi.h[0] * pi.h[1] * pi.h[2];
            pi.ncell = pi.n[0] * pi.n[1] * pi.n[2];
            int32_t id = (int32_t)M.boxes.size();
            for (int32_t s0 = 0; s0 < pi.ncell; s0 += tile_cells)
                M.tiles.push_back({id, s0, std::min(tile_cells, pi.ncell - s0), p});
            M.boxes.push_back(pi);
            M.probs.push_back(p);
            moff += (int64_t)pi.sz * (pi.n[2] + 2);
        }
        M.len = moff;
    }
    t.bottom_off.assign(nprob, 0);
    int64_t boff = 0;
    t.bottom_max = 0;
    for (int p = 0; p < nprob; ++p) {
        int32_t nb = 1, nmax = 1;
        for (int d = 0; d < 3; ++d) {
            const int32_t e = probs[p].base_n[d] >> t.prob_mgdepth[p];
            nb *= e;
            nmax = std::max(nmax, e);
        }
        t.bottom_off[p] = (int32_t)boff;
        boff += (int64_t)nb * nb;
        t.bottom_max = std::max(t.bottom_max, nb);
        if (nb / nmax + 1 > kBottomBand) {
            msg = "coarsest multigrid grid too wide for the banded bottom solve";
            return NRD_EUNSUPPORTED;
        }
    }
    if (t.bottom_max > 128) {
        msg = "coarsest multigrid grid too large for the bottom solve (> 128 cells); "
              "base grid extents must halve down to at most 128 cells";
        return NRD_EUNSUPPORTED;
    }
    return NRD_OK;
}

// The transposed coarse-fine interpolation gathers, per coarse source cell,
// the ghosts it feeds (a source clipped at the domain edge may appear twice
// for one ghost): CSR rows sorted by the source's native index.  Built on
// the first transposed product only (forward work never reads it).
void build_cf_transpose(const Tables& t, std::vector<CFRow>& rows, std::vector<CFSrc>& src) {
    struct Ent { int32_t c, ghost, w, prob; };
    std::vector<Ent> ents;
    ents.reserve(4 * t.gcf.size());
    static const int32_t wq[4] = {9, 3, 3, 1};
    for (size_t i = 0; i < t.gcf.size(); ++i)
        for (int q = 0; q < 4; ++q)
            ents.push_back({t.gcf[i].src[q], t.gcf[i].dst, wq[q], t.gcf_prob[i]});
    // stable LSD radix sort by source cell (millions of entries on deep
    // hierarchies)
    uint32_t cmax = 0;
    for (const Ent& e : ents) cmax = std::max(cmax, (uint32_t)e.c);
    int bits = 1;
    while (bits < 32 && (cmax >> bits)) ++bits;
    const int npass = (bits + 12) / 13;
    const int dig = (bits + npass - 1) / npass;
    const uint32_t mask = (1u << dig) - 1u;
    std::vector<Ent> tmp(ents.size());
    std::vector<size_t> cnt((size_t)mask + 2);
    for (int shift = 0; shift < npass * dig; shift += dig) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (const Ent& e : ents) ++cnt[((uint32_t)e.c >> shift & mask) + 1];
        for (uint32_t i = 0; i <= mask; ++i) cnt[i + 1] += cnt[i];
        for (const Ent& e : ents) tmp[cnt[(uint32_t)e.c >> shift & mask]++] = e;
        ents.swap(tmp);
    }
    rows.clear();
    src.clear();
    src.reserve(ents.size());
    for (size_t i = 0; i < ents.size();) {
        size_t j = i;
        while (j < ents.size() && ents[j].c == ents[i].c) ++j;
        rows.push_back({ents[i].c, (int32_t)i, (int32_t)(j - i), ents[i].prob});
        for (size_t k = i; k < j; ++k) src.push_back({ents[k].ghost, ents[k].w});
        i = j;
    }
}

}  // namespace nrd
