// Host clustering of refinement tags into a new patch hierarchy (paper
// Sec. 5: tagged cells are grouped into patches by the Berger-Rigoutsos
// algorithm).
//
// Level by level from the base: the tags that decide level l + 1 are taken
// on the cells of the new level l, each from the finest old level at or
// below l that holds the cell (a coarse tag marks all its descendants);
// they are grown by `buffer` cells, kept only where the cell and its 26
// neighbours (clipped to the domain) lie on the new level l (so every box
// built from them is properly nested), and clustered:
//   - a box is shrunk to the bounding box of its tags and accepted when the
//     tagged fraction reaches `efficiency`, no side exceeds `max_side` and
//     the box grown by one cell lies on level l;
//   - otherwise it is cut: at a plane without tags (the one nearest the
//     middle of the longest such axis), else at the strongest inflection of
//     the tag signature (a sign change of its second difference), else in
//     the middle of the longest side; cuts made only for efficiency leave no
//     side below `min_side`;
//   - the accepted boxes, refined by 2, are level l + 1.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "nrd_internal.h"

namespace nrd {
namespace {

struct IBox {
    int32_t lo[3], hi[3];
    int64_t volume() const {
        return (int64_t)(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
    }
};

int64_t overlap(const IBox& a, const IBox& b) {
    int64_t v = 1;
    for (int d = 0; d < 3; ++d) {
        const int32_t l = std::max(a.lo[d], b.lo[d]), h = std::min(a.hi[d], b.hi[d]);
        if (h <= l) return 0;
        v *= h - l;
    }
    return v;
}

struct Pt {
    int32_t x[3];
};

// Union of the non-overlapping boxes of one level, with coarse buckets for
// lookups.
struct Level {
    std::vector<IBox> boxes;
    int32_t N[3];
    static constexpr int32_t B = 16;
    int32_t nb[3];
    std::vector<std::vector<int32_t>> bucket;
    void build(const int32_t N_[3]) {
        for (int d = 0; d < 3; ++d) {
            N[d] = N_[d];
            nb[d] = (N[d] + B - 1) / B;
        }
        bucket.assign((size_t)nb[0] * nb[1] * nb[2], {});
        for (int32_t i = 0; i < (int32_t)boxes.size(); ++i) {
            const IBox& b = boxes[i];
            for (int32_t k = b.lo[2] / B; k <= (b.hi[2] - 1) / B; ++k)
                for (int32_t j = b.lo[1] / B; j <= (b.hi[1] - 1) / B; ++j)
                    for (int32_t a = b.lo[0] / B; a <= (b.hi[0] - 1) / B; ++a)
                        bucket[((size_t)k * nb[1] + j) * nb[0] + a].push_back(i);
        }
    }
    // cells of q (clipped to the level) all on the union
    bool covers(IBox q) const {
        for (int d = 0; d < 3; ++d) {
            q.lo[d] = std::max(q.lo[d], 0);
            q.hi[d] = std::min(q.hi[d], N[d]);
        }
        const int64_t need = q.volume();
        std::vector<int32_t> seen;
        int64_t got = 0;
        for (int32_t k = q.lo[2] / B; k <= (q.hi[2] - 1) / B; ++k)
            for (int32_t j = q.lo[1] / B; j <= (q.hi[1] - 1) / B; ++j)
                for (int32_t a = q.lo[0] / B; a <= (q.hi[0] - 1) / B; ++a)
                    for (int32_t i : bucket[((size_t)k * nb[1] + j) * nb[0] + a]) {
                        if (std::find(seen.begin(), seen.end(), i) != seen.end()) continue;
                        seen.push_back(i);
                        got += overlap(q, boxes[i]);
                    }
        return got == need;
    }
};

struct Opt {
    double eff;
    int32_t min_side, max_side;
};

void bbox(const std::vector<Pt>& p, size_t a, size_t b, IBox& out) {
    for (int d = 0; d < 3; ++d) {
        out.lo[d] = p[a].x[d];
        out.hi[d] = p[a].x[d] + 1;
    }
    for (size_t i = a + 1; i < b; ++i)
        for (int d = 0; d < 3; ++d) {
            out.lo[d] = std::min(out.lo[d], p[i].x[d]);
            out.hi[d] = std::max(out.hi[d], p[i].x[d] + 1);
        }
}

// Berger-Rigoutsos on the tagged points [a, b) (reordered in place).
void br(std::vector<Pt>& p, size_t a, size_t b, const Level& L, const Opt& o,
        std::vector<IBox>& out) {
    if (a >= b) return;
    IBox box;
    bbox(p, a, b, box);
    const int64_t vol = box.volume();
    const double eff = (double)(b - a) / (double)vol;
    int32_t n[3];
    int32_t longest = 0;
    for (int d = 0; d < 3; ++d) {
        n[d] = box.hi[d] - box.lo[d];
        longest = std::max(longest, n[d]);
    }
    IBox grown = box;
    for (int d = 0; d < 3; ++d) {
        grown.lo[d] -= 1;
        grown.hi[d] += 1;
    }
    const bool nested = L.covers(grown);
    const bool fits = longest <= o.max_side;
    if (nested && fits && eff >= o.eff) {
        out.push_back(box);
        return;
    }
    // a box that fails only the efficiency test keeps its sides >= min_side
    const int32_t minside = (nested && fits) ? o.min_side : 1;
    int cut_d = -1, cut_k = 0;
    if (!fits) {
        // too long: halve the longest axis
        for (int d = 0; d < 3; ++d)
            if (n[d] == longest) {
                cut_d = d;
                break;
            }
        cut_k = n[cut_d] / 2;
    } else {
        std::vector<int64_t> sig[3];
        for (int d = 0; d < 3; ++d) sig[d].assign(n[d], 0);
        for (size_t i = a; i < b; ++i)
            for (int d = 0; d < 3; ++d) ++sig[d][p[i].x[d] - box.lo[d]];
        // axes from the longest down
        int ord[3] = {0, 1, 2};
        std::stable_sort(ord, ord + 3, [&](int x, int y) { return n[x] > n[y]; });
        // 1. a plane without tags
        for (int q = 0; q < 3 && cut_d < 0; ++q) {
            const int d = ord[q];
            int best = -1;
            for (int k = minside; k <= n[d] - minside; ++k) {
                if (k >= n[d]) break;
                if (sig[d][k] != 0) continue;
                if (best < 0 || std::abs(2 * k - n[d]) < std::abs(2 * best - n[d])) best = k;
            }
            if (best >= 0) {
                cut_d = d;
                cut_k = best;
            }
        }
        // 2. strongest inflection of the signature
        if (cut_d < 0) {
            int64_t best = 0;
            for (int q = 0; q < 3; ++q) {
                const int d = ord[q];
                if (n[d] < 4) continue;
                std::vector<int64_t> lap(n[d], 0);
                for (int k = 1; k + 1 < n[d]; ++k)
                    lap[k] = sig[d][k + 1] - 2 * sig[d][k] + sig[d][k - 1];
                for (int k = 1; k + 2 < n[d]; ++k) {
                    if (!((lap[k] < 0 && lap[k + 1] > 0) || (lap[k] > 0 && lap[k + 1] < 0)))
                        continue;
                    const int kk = k + 1;                  // cut between k and k + 1
                    if (kk < minside || n[d] - kk < minside) continue;
                    const int64_t s = std::llabs(lap[k + 1] - lap[k]);
                    if (s > best) {
                        best = s;
                        cut_d = d;
                        cut_k = kk;
                    }
                }
            }
        }
        // 3. the middle of the longest side that can be cut
        if (cut_d < 0)
            for (int q = 0; q < 3 && cut_d < 0; ++q) {
                const int d = ord[q];
                if (n[d] >= 2 * minside && n[d] >= 2) {
                    cut_d = d;
                    cut_k = n[d] / 2;
                }
            }
    }
    if (cut_d < 0) {
        // nothing to cut: the box only misses the efficiency target
        // (single cells are always nested: tags lie inside the nest region)
        if (nested) out.push_back(box);
        return;
    }
    const int32_t plane = box.lo[cut_d] + cut_k;
    const size_t mid =
        std::partition(p.begin() + a, p.begin() + b, [&](const Pt& x) { return x.x[cut_d] < plane; }) -
        p.begin();
    br(p, a, mid, L, o, out);
    br(p, mid, b, L, o, out);
}

}  // namespace

nrd_status cluster_boxes(const nrd_problem* probs, int32_t nprob, const nrd_box* boxes,
                         int32_t nbox, const uint8_t* tags, const nrd_cluster_opt& co,
                         std::vector<nrd_box>& out, std::string& msg) {
    out.clear();
    if (co.max_levels < 1 || co.buffer < 0 || !(co.efficiency > 0.0) || co.efficiency > 1.0 ||
        co.min_side < 1 || co.max_side < co.min_side) {
        msg = "bad clustering options";
        return NRD_EINVAL;
    }
    // compact offsets of the old boxes
    std::vector<int64_t> coff(nbox + 1, 0);
    for (int b = 0; b < nbox; ++b) {
        int64_t n = 1;
        for (int d = 0; d < 3; ++d) {
            if (boxes[b].hi[d] <= boxes[b].lo[d]) {
                msg = "empty box";
                return NRD_EINVAL;
            }
            n *= boxes[b].hi[d] - boxes[b].lo[d];
        }
        if (boxes[b].problem < 0 || boxes[b].problem >= nprob || boxes[b].level < 0 ||
            (b > 0 && (boxes[b].problem < boxes[b - 1].problem ||
                       (boxes[b].problem == boxes[b - 1].problem &&
                        boxes[b].level < boxes[b - 1].level)))) {
            msg = "boxes must be ordered by (problem, level)";
            return NRD_EINVAL;
        }
        coff[b + 1] = coff[b] + n;
    }
    const Opt o{co.efficiency, co.min_side, co.max_side};
    for (int p = 0; p < nprob; ++p) {
        std::vector<int32_t> old_ids;
        int32_t old_nlev = 0;
        for (int b = 0; b < nbox; ++b)
            if (boxes[b].problem == p) {
                old_ids.push_back(b);
                old_nlev = std::max(old_nlev, boxes[b].level + 1);
            }
        std::vector<IBox> cur;                          // new level l
        for (int32_t b : old_ids)
            if (boxes[b].level == 0) {
                IBox x;
                std::memcpy(x.lo, boxes[b].lo, sizeof x.lo);
                std::memcpy(x.hi, boxes[b].hi, sizeof x.hi);
                cur.push_back(x);
            }
        if (cur.empty()) {
            msg = "a problem without level-0 boxes";
            return NRD_EINVAL;
        }
        for (const IBox& x : cur)
            out.push_back({p, 0, {x.lo[0], x.lo[1], x.lo[2]}, {x.hi[0], x.hi[1], x.hi[2]}});
        for (int l = 0; l + 1 < co.max_levels && !cur.empty(); ++l) {
            int32_t N[3];
            for (int d = 0; d < 3; ++d) N[d] = probs[p].base_n[d] << l;
            Level L;
            L.boxes = cur;
            L.build(N);
            std::vector<Pt> pts;
            const int32_t g = co.buffer;
            for (const IBox& B : cur) {
                // tags painted on B grown by the buffer (clipped), finest old
                // level at or below l last
                IBox E = B;
                for (int d = 0; d < 3; ++d) {
                    E.lo[d] = std::max(0, B.lo[d] - g);
                    E.hi[d] = std::min(N[d], B.hi[d] + g);
                }
                const int32_t en[3] = {E.hi[0] - E.lo[0], E.hi[1] - E.lo[1], E.hi[2] - E.lo[2]};
                std::vector<uint8_t> t((size_t)en[0] * en[1] * en[2], 0);
                auto at = [&](int32_t i, int32_t j, int32_t k) -> uint8_t& {
                    return t[((size_t)(k - E.lo[2]) * en[1] + (j - E.lo[1])) * en[0] + (i - E.lo[0])];
                };
                for (int32_t lo_l = 0; lo_l <= std::min(l, old_nlev - 1); ++lo_l) {
                    const int sh = l - lo_l;
                    for (int32_t b : old_ids) {
                        if (boxes[b].level != lo_l) continue;
                        const nrd_box& ob = boxes[b];
                        IBox R;
                        for (int d = 0; d < 3; ++d) {
                            R.lo[d] = std::max(E.lo[d], ob.lo[d] << sh);
                            R.hi[d] = std::min(E.hi[d], ob.hi[d] << sh);
                        }
                        if (R.lo[0] >= R.hi[0] || R.lo[1] >= R.hi[1] || R.lo[2] >= R.hi[2])
                            continue;
                        const int32_t on0 = ob.hi[0] - ob.lo[0], on1 = ob.hi[1] - ob.lo[1];
                        for (int32_t k = R.lo[2]; k < R.hi[2]; ++k)
                            for (int32_t j = R.lo[1]; j < R.hi[1]; ++j)
                                for (int32_t i = R.lo[0]; i < R.hi[0]; ++i) {
                                    const int64_t c = coff[b] + ((int64_t)((k >> sh) - ob.lo[2]) * on1 +
                                                                 ((j >> sh) - ob.lo[1])) * on0 +
                                                      ((i >> sh) - ob.lo[0]);
                                    at(i, j, k) = tags[c] ? 1 : 0;
                                }
                    }
                }
                // grow the tags by the buffer, one axis at a time
                for (int d = 0; d < 3 && g > 0; ++d) {
                    std::vector<uint8_t> u(t.size(), 0);
                    const size_t st = d == 0 ? 1 : (d == 1 ? (size_t)en[0] : (size_t)en[0] * en[1]);
                    for (int32_t k = 0; k < en[2]; ++k)
                        for (int32_t j = 0; j < en[1]; ++j)
                            for (int32_t i = 0; i < en[0]; ++i) {
                                const size_t c = ((size_t)k * en[1] + j) * en[0] + i;
                                if (!t[c]) continue;
                                const int32_t pos = d == 0 ? i : (d == 1 ? j : k);
                                for (int32_t s = -g; s <= g; ++s) {
                                    const int32_t q = pos + s;
                                    if (q < 0 || q >= en[d]) continue;
                                    u[c + (ptrdiff_t)s * (ptrdiff_t)st] = 1;
                                }
                            }
                    t.swap(u);
                }
                // keep the tagged cells of B whose neighbourhood lies on level l
                for (int32_t k = B.lo[2]; k < B.hi[2]; ++k)
                    for (int32_t j = B.lo[1]; j < B.hi[1]; ++j)
                        for (int32_t i = B.lo[0]; i < B.hi[0]; ++i) {
                            if (!at(i, j, k)) continue;
                            const bool inside = i > B.lo[0] && i + 1 < B.hi[0] && j > B.lo[1] &&
                                                j + 1 < B.hi[1] && k > B.lo[2] && k + 1 < B.hi[2];
                            if (!inside) {
                                IBox nb{{i - 1, j - 1, k - 1}, {i + 2, j + 2, k + 2}};
                                if (!L.covers(nb)) continue;
                            }
                            pts.push_back({{i, j, k}});
                        }
            }
            std::vector<IBox> fine;
            br(pts, 0, pts.size(), L, o, fine);
            std::vector<IBox> next;
            for (const IBox& x : fine) {
                IBox y;
                for (int d = 0; d < 3; ++d) {
                    y.lo[d] = 2 * x.lo[d];
                    y.hi[d] = 2 * x.hi[d];
                }
                next.push_back(y);
                out.push_back({p, l + 1, {y.lo[0], y.lo[1], y.lo[2]}, {y.hi[0], y.hi[1], y.hi[2]}});
            }
            cur.swap(next);
        }
    }
    return NRD_OK;
}

}  // namespace nrd
