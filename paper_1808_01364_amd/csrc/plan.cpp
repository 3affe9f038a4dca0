// Host planner (integers only). See plan.hpp for the grouping rule.
#include "plan.hpp"

#include <algorithm>
#include <cstring>
#include <stdexcept>
#include <string>

namespace rhif {

namespace {

inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
constexpr int64_t kNarrowTileCells = 16;   // levels with at most this many cells: narrow tiles

// A block family with an interior above kBigApplyMinI is applied panel by panel over many
// workgroups per block, which stages every block's vectors in the global workspace: give the
// blocks that fit LDS a workspace region too.
void big_family_ws(std::vector<ApplyDesc>& fam, int64_t& ws) {
    int mi = 0;
    for (const ApplyDesc& a : fam) mi = std::max(mi, a.nI);
    if (mi <= kBigApplyMinI) return;
    for (ApplyDesc& a : fam)
        if (a.wsoff < 0) {
            a.wsoff = ws;
            ws += align_up(a.nI + a.nB, 32);
        }
}

}  // namespace

void PlanScratch::init(int64_t N) {
    mark_stamp.assign(N, 0);
    stamp = 0;
    keep_ptr.clear();
    keep_t.clear();
}

void PlanScratch::reserve(int64_t N) {
    keep_ptr.clear();
    keep_t.clear();
    if (static_cast<int64_t>(mark_stamp.size()) >= N) return;
    init(N);
}

void LevelPlan::reset() {
    ext_elems = 0;
    level = w = nc1 = 0;
    root = false;
    dofs_on_device = lists_pending = src_on_device = false;
    for (auto* v : {&gptr, &gdofs, &gslot_cnt, &gslot_cell, &gslot_off, &c_nI, &c_nB, &c_nf, &c_ld, &c_dptr,
                    &c_dofs, &c_gptr, &c_g, &c_goff, &seps, &skels, &src, &sep_dofs, &g_g2, &g_t2, &c_g2, &c_t2})
        v->clear();
    gcls.clear();
    c_foff.clear();
    cell_potrf.clear();
    cell_ref.clear();
    tiles.clear();
    sep_desc.clear();
    cell_groups.clear();
    cell_scale.clear();
    skel_desc.clear();
    cell_apply.clear();
    sep_apply.clear();
    gather.clear();
    ncells = 0;
    front_elems = lg_elems = li_elems = skli_elems = m_elems = t_elems = g_elems = y_elems = ws_elems = 0;
    skel_ntotal = max_nf = max_sep_n = max_skel_n = max_cell_groups = 0;
    flops = alg_elim_flops = alg_prec_chol_flops = alg_prec_scale_flops = alg_front_bytes = 0.0;
    alg_apply_cell_bytes = alg_apply_sep_bytes = alg_gather_bytes = 0.0;
}

int num_levels(int s, int leaf) {
    int L = 0;
    while ((static_cast<int64_t>(leaf) << L) <= s) ++L;
    return L;
}

void build_level(const GridInfo& gi, int level, int leaf, bool root, int64_t n_active, const LevelPlan* prev,
                 PlanScratch& scr, int lds_apply_cap, LevelPlan& P) {
    build_cells(gi, level, leaf, root, n_active, prev, scr, lds_apply_cap, P);
    if (!root) build_separators(gi, scr, lds_apply_cap, P);
}

void fill_leaf_lists(const GridInfo& gi, PlanScratch& scr, LevelPlan& P) {
    const int d = gi.d, s = gi.s;
    const int ngroups = static_cast<int>(P.gptr.size()) - 1;
    const int64_t s2 = static_cast<int64_t>(s) * s;
    P.gdofs.resize(gi.N);
    // every group's box in ascending order
    for (int g = 0; g < ngroups; ++g) {
        const int* lo = scr.box_lo.data() + 3 * g;
        const int* nb = scr.box_n.data() + 3 * g;
        int32_t* out = P.gdofs.data() + P.gptr[g];
        for (int x2 = lo[2]; x2 < lo[2] + nb[2]; ++x2)
            for (int x1 = lo[1]; x1 < lo[1] + nb[1]; ++x1) {
                const int64_t base = (d > 2 ? (x2 - 1) * s2 : 0) + (d > 1 ? static_cast<int64_t>(x1 - 1) * s : 0);
                for (int x0 = lo[0]; x0 < lo[0] + nb[0]; ++x0) *out++ = static_cast<int32_t>(base + x0 - 1);
            }
        if (out != P.gdofs.data() + P.gptr[g + 1]) throw std::logic_error("leaf group box size");
    }
    P.lists_pending = false;
}

void build_cells(const GridInfo& gi, int level, int leaf, bool root, int64_t n_active, const LevelPlan* prev,
                 PlanScratch& scr, int lds_apply_cap, LevelPlan& P, bool device_tables) {
    const int d = gi.d, s = gi.s;
    P.reset();
    P.level = level;
    P.root = root;
    const int64_t w = static_cast<int64_t>(leaf) << level;
    P.w = static_cast<int>(w);
    const int nc1 = static_cast<int>((s + w - 1) / w);
    P.nc1 = nc1;
    if (root && nc1 != 1) throw std::logic_error("root level must have a single cell");
    const int KB = 2 * nc1 + 2;
    int64_t nkeys = 1;
    for (int k = 0; k < d; ++k) nkeys *= KB;

    // ---- classify the active unknowns and bucket them by key ----
    int64_t na = 0;
    int ngroups = 0;
    scr.key2g.assign(nkeys, -1);
    if (prev == nullptr) {
        if (n_active != gi.N) throw std::logic_error("the leaf level starts with every unknown active");
        na = gi.N;
        // Every unknown is active (the leaf level): the groups are boxes of the grid,
        // enumerated directly in key order, each in ascending order.
        // per axis and key component kk: the interval's first point and length (0: empty)
        std::vector<int32_t> ax_lo(KB), ax_n(KB);
        for (int kk = 0; kk < KB; ++kk) {
            const int64_t c = kk >> 1;
            int64_t lo, hi;
            if (kk & 1) {
                lo = c * w + 1;
                hi = std::min<int64_t>((c + 1) * w - 1, s);
            } else {
                lo = hi = c * w;
                if (c * w < 1 || c * w > s) hi = lo - 1;
            }
            ax_lo[kk] = static_cast<int32_t>(lo);
            ax_n[kk] = static_cast<int32_t>(std::max<int64_t>(hi - lo + 1, 0));
        }
        const int K1 = d > 1 ? KB : 1, K2 = d > 2 ? KB : 1;
        const int64_t ng_max = nkeys;
        P.gptr.resize(ng_max + 1);
        P.gcls.resize(ng_max);
        scr.box_lo.resize(3 * ng_max);
        scr.box_n.resize(3 * ng_max);
        int64_t at = 0;
        for (int k2 = 0; k2 < K2; ++k2)
            for (int k1 = 0; k1 < K1; ++k1)
                for (int k0 = 0; k0 < KB; ++k0) {
                    const int n0 = ax_n[k0], n1 = d > 1 ? ax_n[k1] : 1, n2 = d > 2 ? ax_n[k2] : 1;
                    if (n0 == 0 || n1 == 0 || n2 == 0) continue;
                    const int64_t K = k0 + static_cast<int64_t>(KB) * (k1 + static_cast<int64_t>(KB) * k2);
                    const int g = ngroups++;
                    scr.key2g[K] = g;
                    P.gptr[g] = static_cast<int32_t>(at);
                    P.gcls[g] = static_cast<int8_t>(((k0 & 1) == 0) + (d > 1 && (k1 & 1) == 0) + (d > 2 && (k2 & 1) == 0));
                    int32_t* bl = scr.box_lo.data() + 3 * g;
                    int32_t* bn = scr.box_n.data() + 3 * g;
                    bl[0] = ax_lo[k0];
                    bl[1] = d > 1 ? ax_lo[k1] : 1;
                    bl[2] = d > 2 ? ax_lo[k2] : 1;
                    bn[0] = n0;
                    bn[1] = n1;
                    bn[2] = n2;
                    at += static_cast<int64_t>(n0) * n1 * n2;
                }
        P.gptr.resize(ngroups + 1);
        P.gcls.resize(ngroups);
        scr.box_lo.resize(3 * static_cast<size_t>(ngroups));
        scr.box_n.resize(3 * static_cast<size_t>(ngroups));
        if (at != na) throw std::logic_error("leaf-level groups do not cover the grid");
        P.gptr[ngroups] = static_cast<int32_t>(na);
        // the groups' unknowns now, or later (fill_leaf_lists) when the device writes the
        // cells' frontal unknowns itself
        P.dofs_on_device = device_tables;
        P.lists_pending = true;
        if (!device_tables) fill_leaf_lists(gi, scr, P);
    } else {
        // Levels >= 1: the kept unknowns of every group of the level below (ascending
        // positions, from next_active_set). The unknowns of one group there share one key
        // here, so groups move as a whole; the parts of a group are then put in ascending
        // order (in 3D the faces below that tile a face here interleave).
        const LevelPlan& Q = *prev;
        const int ng2 = static_cast<int>(Q.gptr.size()) - 1;
        if (static_cast<int>(scr.keep_ptr.size()) != ng2 + 1 || scr.keep_ptr[ng2] != n_active)
            throw std::logic_error("kept unknowns of the level below are missing");
        std::vector<int32_t> keyk(static_cast<size_t>(s) + 1);
        for (int xk = 1; xk <= s; ++xk) keyk[xk] = 2 * (xk / static_cast<int>(w)) + ((xk % w) != 0 ? 1 : 0);
        const int64_t mulk[3] = {1, KB, static_cast<int64_t>(KB) * KB};
        const uint32_t us = static_cast<uint32_t>(s);
        auto key_of = [&](int32_t i) {   // unknowns are int32 indices: 32-bit divisions
            uint32_t r = static_cast<uint32_t>(i);
            int64_t K = 0;
            for (int k = 0; k + 1 < d; ++k) {
                const uint32_t q = r / us;
                K += keyk[r - q * us + 1] * mulk[k];
                r = q;
            }
            return K + keyk[r + 1] * mulk[d - 1];   // the last coordinate is what is left
        };
        std::vector<int32_t>& gkey = scr.akey;
        gkey.assign(ng2, -1);
        scr.count.assign(nkeys + 1, 0);
        for (int g2 = 0; g2 < ng2; ++g2) {
            const int b = scr.keep_ptr[g2], e = scr.keep_ptr[g2 + 1];
            if (e == b) continue;
            const int32_t* gd = Q.gdofs.data() + Q.gptr[g2];
            const int64_t K = key_of(gd[scr.keep_t[b]]);
            if (key_of(gd[scr.keep_t[e - 1]]) != K) throw std::logic_error("a group of the level below spans two groups");
            gkey[g2] = static_cast<int32_t>(K);
            scr.count[K + 1] += e - b;
            na += e - b;
        }
        for (int64_t K = 0; K < nkeys; ++K)
            if (scr.count[K + 1] > 0) scr.key2g[K] = ngroups++;
        for (int64_t K = 0; K < nkeys; ++K) scr.count[K + 1] += scr.count[K];
        P.gptr.assign(ngroups + 1, 0);
        P.gcls.assign(ngroups, 0);
        for (int64_t K = 0; K < nkeys; ++K) {
            const int g = scr.key2g[K];
            if (g < 0) continue;
            P.gptr[g] = scr.count[K];
            int64_t r = K;
            int even = 0;
            for (int k = 0; k < d; ++k) {
                if (((r % KB) & 1) == 0) ++even;
                r /= KB;
            }
            P.gcls[g] = static_cast<int8_t>(even);
        }
        P.gptr[ngroups] = static_cast<int32_t>(na);
        P.gdofs.resize(na);
        P.g_g2.resize(na);
        P.g_t2.resize(na);
        std::vector<int32_t>& pos = scr.pos;
        pos.assign(scr.count.begin(), scr.count.end() - 1);
        for (int g2 = 0; g2 < ng2; ++g2) {
            const int K = gkey[g2];
            if (K < 0) continue;
            const int32_t* gd = Q.gdofs.data() + Q.gptr[g2];
            int at = pos[K];
            for (int e = scr.keep_ptr[g2]; e < scr.keep_ptr[g2 + 1]; ++e) {
                const int t = scr.keep_t[e];
                P.gdofs[at] = gd[t];
                P.g_g2[at] = g2;
                P.g_t2[at] = t;
                ++at;
            }
            pos[K] = at;
        }
        std::vector<int32_t>& ord = scr.ord;
        std::vector<int32_t>& tmp = scr.tmp;
        for (int g = 0; g < ngroups; ++g) {
            const int b = P.gptr[g], e = P.gptr[g + 1];
            bool sorted = true;
            for (int q = b + 1; q < e && sorted; ++q) sorted = P.gdofs[q] > P.gdofs[q - 1];
            if (sorted) continue;
            ord.resize(e - b);
            for (int q = 0; q < e - b; ++q) ord[q] = b + q;
            std::sort(ord.begin(), ord.end(), [&](int32_t u, int32_t v) { return P.gdofs[u] < P.gdofs[v]; });
            tmp.resize(3 * static_cast<size_t>(e - b));
            for (int q = 0; q < e - b; ++q) {
                tmp[3 * q] = P.gdofs[ord[q]];
                tmp[3 * q + 1] = P.g_g2[ord[q]];
                tmp[3 * q + 2] = P.g_t2[ord[q]];
            }
            for (int q = 0; q < e - b; ++q) {
                P.gdofs[b + q] = tmp[3 * q];
                P.g_g2[b + q] = tmp[3 * q + 1];
                P.g_t2[b + q] = tmp[3 * q + 2];
            }
        }
    }

    // ---- cells: every geometric cell; frontal = interior, then boundary groups ----
    int64_t ncells = 1;
    for (int k = 0; k < d; ++k) ncells *= nc1;
    P.ncells = static_cast<int>(ncells);
    P.c_nI.assign(ncells, 0);
    P.c_nB.assign(ncells, 0);
    P.c_nf.assign(ncells, 0);
    P.c_ld.assign(ncells, 0);
    P.c_foff.assign(ncells, 0);
    P.c_dptr.assign(ncells + 1, 0);
    P.c_gptr.assign(ncells + 1, 0);
    P.gslot_cnt.assign(ngroups, 0);
    P.gslot_cell.assign(static_cast<size_t>(ngroups) * kMaxSlots, -1);
    P.gslot_off.assign(static_cast<size_t>(ngroups) * kMaxSlots, -1);
    if (!P.dofs_on_device) P.c_dofs.reserve(na + na / 2);
    int32_t ndofs = 0;
    int n3 = 1;
    for (int k = 0; k < d; ++k) n3 *= 3;
    int64_t foff = 0;
    for (int64_t ci = 0; ci < ncells; ++ci) {
        int c[3];
        int64_t r = ci;
        for (int k = 0; k < d; ++k) {
            c[k] = static_cast<int>(r % nc1);
            r /= nc1;
        }
        P.c_dptr[ci] = ndofs;
        // interior group
        int64_t KI = 0, mul = 1;
        for (int k = 0; k < d; ++k) {
            KI += (2 * c[k] + 1) * mul;
            mul *= KB;
        }
        const int gI = scr.key2g[KI];
        int nI = 0;
        if (gI >= 0) {
            nI = P.gptr[gI + 1] - P.gptr[gI];
            if (!P.dofs_on_device)
                P.c_dofs.insert(P.c_dofs.end(), P.gdofs.begin() + P.gptr[gI], P.gdofs.begin() + P.gptr[gI + 1]);
            if (prev != nullptr) {
                P.c_g2.insert(P.c_g2.end(), P.g_g2.begin() + P.gptr[gI], P.g_g2.begin() + P.gptr[gI + 1]);
                P.c_t2.insert(P.c_t2.end(), P.g_t2.begin() + P.gptr[gI], P.g_t2.begin() + P.gptr[gI + 1]);
            }
        }
        int nf = nI;
        for (int t = 0; t < n3; ++t) {
            int tt = t;
            int64_t K = 0, m2 = 1;
            bool all_one = true;
            for (int k = 0; k < d; ++k) {
                const int dk = tt % 3;
                tt /= 3;
                if (dk != 1) all_one = false;
                K += (2 * c[k] + dk) * m2;
                m2 *= KB;
            }
            if (all_one) continue;
            const int g = scr.key2g[K];
            if (g < 0) continue;
            const int ng = P.gptr[g + 1] - P.gptr[g];
            P.c_g.push_back(g);
            P.c_goff.push_back(nf);
            const int sl = P.gslot_cnt[g]++;
            if (sl >= kMaxSlots) throw std::logic_error("group in too many cells");
            P.gslot_cell[static_cast<size_t>(g) * kMaxSlots + sl] = static_cast<int32_t>(ci);
            P.gslot_off[static_cast<size_t>(g) * kMaxSlots + sl] = nf;
            if (!P.dofs_on_device)
                P.c_dofs.insert(P.c_dofs.end(), P.gdofs.begin() + P.gptr[g], P.gdofs.begin() + P.gptr[g + 1]);
            if (prev != nullptr) {
                P.c_g2.insert(P.c_g2.end(), P.g_g2.begin() + P.gptr[g], P.g_g2.begin() + P.gptr[g + 1]);
                P.c_t2.insert(P.c_t2.end(), P.g_t2.begin() + P.gptr[g], P.g_t2.begin() + P.gptr[g + 1]);
            }
            nf += ng;
        }
        P.c_gptr[ci + 1] = static_cast<int32_t>(P.c_g.size());
        ndofs += nf;
        P.c_nI[ci] = nI;
        P.c_nB[ci] = nf - nI;
        P.c_nf[ci] = nf;
        P.c_ld[ci] = std::max(nf, 1);
        P.c_foff[ci] = foff;
        foff += align_up(static_cast<int64_t>(P.c_ld[ci]) * nf, 32);
        P.max_nf = std::max(P.max_nf, nf);
    }
    P.c_dptr[ncells] = ndofs;
    if (!P.dofs_on_device && static_cast<int64_t>(P.c_dofs.size()) != ndofs)
        throw std::logic_error("cell dof bookkeeping");
    P.front_elems = std::max<int64_t>(foff, 32);

    // ---- batched descriptors of the cells ----
    const bool banded = leaf_interior_banded(d, level, root, P.w);
    // (sums in locals: the table appends below would otherwise force them through memory)
    double front_bytes = 0.0, flops = 0.0, elim_flops = 0.0, apply_bytes = 0.0;
    int64_t ext_elems = P.ext_elems;
    double bw = 1.0, leaf_int = 1.0;
    for (int k = 1; k < d; ++k) bw *= (leaf - 1);
    for (int k = 0; k < d; ++k) leaf_int *= (leaf - 1);
    P.cell_ref.reserve(ncells);
    for (int64_t ci = 0; ci < ncells; ++ci) {
        P.cell_ref.push_back(CellRef{P.c_foff[ci], P.c_ld[ci], P.c_nI[ci], P.c_nf[ci], P.c_dptr[ci]});
        const int nf = P.c_nf[ci];
        const int nI = P.c_nI[ci], nB = P.c_nB[ci];
        const int32_t cc = static_cast<int32_t>(ci);
        if (banded && nI > 0) {
            // the interior band (three 16-wide column blocks per tile), then the boundary rows
            // of the interior columns and the boundary block; the rest is never read
            for (int j0 = 0; j0 < nI; j0 += 48)
                P.tiles.push_back(Tile{cc, j0, j0, tile_shape(std::min(64, nI - j0), std::min(48, nI - j0), true)});
            for (int part = 0; part < 2; ++part) {
                const int cend = part == 0 ? nI : nf;
                for (int c0 = part == 0 ? 0 : nI; c0 < cend; c0 += 64)
                    for (int r0 = nI; r0 < nf; r0 += 64)
                        P.tiles.push_back(
                            Tile{cc, r0, c0, tile_shape(std::min(64, nf - r0), std::min(64, cend - c0), false)});
            }
            double band = 0.0;
            for (int j0 = 0; j0 < nI; j0 += 16) band += std::min(16, nI - j0) * (std::min(32, nI - j0) + 0.0);
            front_bytes += 8.0 * (band + static_cast<double>(nB) * nf);
        } else if (prev != nullptr && ncells <= kNarrowTileCells) {
            // few cells (the upper levels): 64 x 16 extend-add tiles, four times as many
            // workgroups, each with a quarter of the dependent loads
            for (int c0 = 0; c0 < nf; c0 += 16)
                for (int r0 = 0; r0 < nf; r0 += 64)
                    P.tiles.push_back(
                        Tile{cc, r0, c0, tile_shape(std::min(64, nf - r0), std::min(16, nf - c0), false)});
            front_bytes += 8.0 * static_cast<double>(nf) * nf;
        } else {
            for (int c0 = 0; c0 < nf; c0 += 64)
                for (int r0 = 0; r0 < nf; r0 += 64) P.tiles.push_back(Tile{cc, r0, c0, 0});
            front_bytes += 8.0 * static_cast<double>(nf) * nf;
        }
        if (nI > 0) {
            P.cell_potrf.push_back(FrontDesc{P.c_foff[ci], P.c_ld[ci], nf, nI, static_cast<int32_t>(ci),
                                             static_cast<int32_t>(ext_elems), 0});
            ext_elems += (nI + 15) / 16;
            const double a = nI, b = nB;
            flops += a * a * a / 3.0 + a * a * b + a * b * b;
            // a leaf interior (the whole (m-1)^d grid of a leaf cell) is banded with bandwidth
            // (m-1)^(d-1) in natural order: the method needs only the banded work and words
            double lwords;
            if (level == 0 && !root && a == leaf_int && bw < a) {
                elim_flops += a * bw * bw + 2.0 * a * bw * b + b * b * a;
                lwords = a * (bw + 1.0);
            } else {
                elim_flops += a * a * a / 3.0 + a * a * b + a * b * b;
                lwords = a * (a + 1.0) / 2.0;
            }
            apply_bytes += 8.0 * (lwords + a * b) + 8.0 * (2.0 * a + b);
        }
    }
    P.alg_front_bytes += front_bytes;
    P.flops += flops;
    P.alg_elim_flops += elim_flops;
    P.alg_apply_cell_bytes += apply_bytes;
    P.ext_elems = ext_elems;

    // ---- extend-add sources from the children (level >= 1) ----
    const int W = 1 << d;
    P.src_on_device = prev != nullptr && device_tables;
    if (prev != nullptr && !P.src_on_device) {
        const int pnc1 = prev->nc1;
        // parent cell of every cell of the level below
        std::vector<int32_t>& par_of = scr.par_of;
        par_of.resize(prev->ncells);
        for (int64_t cc = 0; cc < prev->ncells; ++cc) {
            int64_t rr = cc, par = 0, mul = 1;
            for (int k = 0; k < d; ++k) {
                par += ((rr % pnc1) / 2) * mul;
                rr /= pnc1;
                mul *= nc1;
            }
            par_of[cc] = static_cast<int32_t>(par);
        }
        P.src.resize(static_cast<size_t>(P.c_dofs.size()) * 2 * W);
        int32_t* srcp = P.src.data();
        for (int64_t ci = 0; ci < ncells; ++ci) {
            int last_g2 = -1, nq = 0;
            int32_t qc[2 * kMaxSlots], qo[2 * kMaxSlots];
            for (int p = P.c_dptr[ci]; p < P.c_dptr[ci + 1]; ++p) {
                const int g2 = P.c_g2[p];
                const int t2 = P.c_t2[p];
                if (g2 < 0 || g2 + 1 >= static_cast<int64_t>(prev->gptr.size()))
                    throw std::logic_error("active unknown missing from the level below");
                if (g2 != last_g2) {
                    // the child cells of ci that hold g2, and where
                    last_g2 = g2;
                    nq = 0;
                    for (int sl = 0; sl < prev->gslot_cnt[g2]; ++sl) {
                        const int cc = prev->gslot_cell[static_cast<size_t>(g2) * kMaxSlots + sl];
                        if (par_of[cc] != ci) continue;
                        qc[nq] = cc;
                        qo[nq] = prev->gslot_off[static_cast<size_t>(g2) * kMaxSlots + sl];
                        ++nq;
                    }
                    if (nq == 0 || nq > W) throw std::logic_error("frontal unknown without a child source");
                }
                int32_t* o = srcp + static_cast<size_t>(p) * W * 2;
                for (int q = 0; q < nq; ++q) {
                    o[2 * q] = qc[q];
                    o[2 * q + 1] = qo[q] + t2;
                }
                for (int q = nq; q < W; ++q) {
                    o[2 * q] = -1;
                    o[2 * q + 1] = -1;
                }
            }
        }
    }

    // ---- cell apply descriptors and the y scratch ----
    int64_t yoff = 0, ws = 0;
    std::vector<int64_t>& cell_y = scr.cell_y;
    cell_y.assign(ncells, -1);
    size_t next_potrf = 0;
    for (int64_t ci = 0; ci < ncells; ++ci) {
        const int nI = P.c_nI[ci], nB = P.c_nB[ci];
        if (nI == 0) continue;
        ApplyDesc ad{};
        ad.ext = P.cell_potrf[next_potrf++].ext;
        ad.li = 256 * ad.ext;
        ad.off = P.c_foff[ci];
        ad.toff = -1;
        ad.yoff = nB > 0 ? yoff : -1;
        cell_y[ci] = yoff;
        ad.wsoff = -1;
        if (nI + nB > lds_apply_cap) {
            ad.wsoff = ws;
            ws += align_up(nI + nB, 32);
        }
        ad.ld = P.c_ld[ci];
        ad.nI = nI;
        ad.nB = nB;
        ad.dofs = P.c_dptr[ci];
        P.cell_apply.push_back(ad);
        yoff += nB;
    }
    big_family_ws(P.cell_apply, ws);
    P.y_elems = std::max<int64_t>(yoff, 1);
    P.ws_elems = ws;
}

void build_separators(const GridInfo& gi, PlanScratch& scr, int lds_apply_cap, LevelPlan& P) {
    if (P.lists_pending) throw std::logic_error("leaf groups without their unknowns");
    (void)gi;
    const int ngroups = static_cast<int>(P.gptr.size()) - 1;
    const int64_t ncells = P.ncells;
    const std::vector<int64_t>& cell_y = scr.cell_y;
    int64_t ws = P.ws_elems;

    // ---- separator groups: block Jacobi and the up-sweep gather ----
    int64_t loff = 0;
    int32_t lioff = 0;
    std::vector<int64_t> g_loff(ngroups, -1);
    std::vector<int32_t> g_lioff(ngroups, -1);
    for (int g = 0; g < ngroups; ++g) {
        if (P.gcls[g] == 0) continue;
        const int n = P.gptr[g + 1] - P.gptr[g];
        P.seps.push_back(g);
        SepDesc sd{};
        sd.n = n;
        sd.nslot = P.gslot_cnt[g];
        for (int sl = 0; sl < kMaxSlots; ++sl) {
            sd.slot_cell[sl] = P.gslot_cell[static_cast<size_t>(g) * kMaxSlots + sl];
            sd.slot_off[sl] = P.gslot_off[static_cast<size_t>(g) * kMaxSlots + sl];
        }
        sd.loff = loff;
        g_loff[g] = loff;
        sd.lioff = lioff;
        g_lioff[g] = lioff;
        lioff += 256 * ((n + 15) / 16);
        sd.dofs = static_cast<int32_t>(P.sep_dofs.size());
        P.sep_dofs.insert(P.sep_dofs.end(), P.gdofs.begin() + P.gptr[g], P.gdofs.begin() + P.gptr[g + 1]);
        P.sep_desc.push_back(sd);
        loff += align_up(static_cast<int64_t>(n) * n, 32);
        P.max_sep_n = std::max(P.max_sep_n, n);
        P.flops += static_cast<double>(n) * n * n / 3.0;
        P.alg_prec_chol_flops += static_cast<double>(n) * n * n / 3.0;
        P.alg_apply_sep_bytes += 8.0 * (static_cast<double>(n) * (n + 1) / 2.0 + 2.0 * n);

        GatherDesc gd{};
        gd.n = n;
        gd.dofs = sd.dofs;
        gd.nslot = 0;
        for (int sl = 0; sl < sd.nslot; ++sl) {
            const int cc = sd.slot_cell[sl];
            if (cell_y[cc] < 0) continue;
            gd.yoff[gd.nslot++] = cell_y[cc] + (sd.slot_off[sl] - P.c_nI[cc]);
        }
        P.alg_gather_bytes += 8.0 * n * (gd.nslot + 2.0);
        P.gather.push_back(gd);

        ApplyDesc ad{};
        ad.ext = -1;
        ad.li = sd.lioff;
        ad.off = sd.loff;
        ad.toff = -1;
        ad.yoff = -1;
        ad.wsoff = -1;
        if (n > lds_apply_cap) {
            ad.wsoff = ws;
            ws += align_up(n, 32);
        }
        ad.ld = n;
        ad.nI = n;
        ad.nB = 0;
        ad.dofs = sd.dofs;
        P.sep_apply.push_back(ad);
    }
    P.lg_elems = std::max<int64_t>(loff, 32);
    P.li_elems = std::max<int64_t>(lioff, 256);
    for (int64_t ci = 0; ci < ncells; ++ci) {
        CellScaleDesc cs{};
        cs.off = P.c_foff[ci];
        cs.ld = P.c_ld[ci];
        cs.nI = P.c_nI[ci];
        cs.nB = P.c_nB[ci];
        cs.g_begin = static_cast<int32_t>(P.cell_groups.size());
        for (int e = P.c_gptr[ci]; e < P.c_gptr[ci + 1]; ++e) {
            const int g = P.c_g[e];
            CellGroup cg{};
            cg.off = P.c_goff[e];
            cg.n = P.gptr[g + 1] - P.gptr[g];
            cg.loff = g_loff[g];
            cg.lioff = g_lioff[g];
            cg.owner = (P.gslot_cell[static_cast<size_t>(g) * kMaxSlots] == ci) ? 1 : 0;
            cg.cell = static_cast<int32_t>(P.cell_scale.size());
            P.cell_groups.push_back(cg);
            const double nb = cs.nB, ng = cg.n;
            P.flops += 2.0 * nb * ng * ng;
            P.alg_prec_scale_flops += 2.0 * nb * ng * ng;
        }
        cs.g_count = static_cast<int32_t>(P.cell_groups.size()) - cs.g_begin;
        if (cs.nB > 0) {
            P.cell_scale.push_back(cs);
            P.max_cell_groups = std::max(P.max_cell_groups, cs.g_count);
        }
    }

    // ---- skeletonized groups: rows of M = A[R_g, g] from the one or two cells ----
    int64_t moff = 0, toff = 0, goff = 0;
    int32_t poff = 0, skli = 0;
    for (int g = 0; g < ngroups; ++g) {
        if (P.gcls[g] != 1) continue;
        const int n = P.gptr[g + 1] - P.gptr[g];
        const int ns = P.gslot_cnt[g];
        if (ns < 1 || ns > 2) throw std::logic_error("an edge/face must touch one or two cells");
        SkelDesc sk{};
        sk.n = n;
        sk.nslot = ns;
        sk.grp = g;
        for (int sl = 0; sl < 2; ++sl) {
            sk.cell[sl] = sl < ns ? P.gslot_cell[static_cast<size_t>(g) * kMaxSlots + sl] : -1;
            sk.off[sl] = sl < ns ? P.gslot_off[static_cast<size_t>(g) * kMaxSlots + sl] : -1;
        }
        // rows of M (built on the device in this order): the other boundary groups of the
        // first cell (with the second cell's share added where the group is shared), then
        // the second cell's remaining groups
        int r = 0;
        const int c1 = sk.cell[0];
        const int c2 = ns == 2 ? sk.cell[1] : -1;
        auto in_cell = [&](int cell, int grp) -> bool {
            for (int e = P.c_gptr[cell]; e < P.c_gptr[cell + 1]; ++e)
                if (P.c_g[e] == grp) return true;
            return false;
        };
        for (int e = P.c_gptr[c1]; e < P.c_gptr[c1 + 1]; ++e) {
            const int h = P.c_g[e];
            if (h != g) r += P.gptr[h + 1] - P.gptr[h];
        }
        if (c2 >= 0) {
            for (int e = P.c_gptr[c2]; e < P.c_gptr[c2 + 1]; ++e) {
                const int h = P.c_g[e];
                if (h != g && !in_cell(c1, h)) r += P.gptr[h + 1] - P.gptr[h];
            }
        }
        sk.r = r;
        sk.moff = moff;
        moff += align_up(static_cast<int64_t>(std::max(r, 1)) * (n | 1), 32);   // row-major, odd stride
        sk.toff = toff;
        toff += align_up(static_cast<int64_t>(n) * n / 4 + 1, 32);
        sk.goff = goff;
        goff += align_up(static_cast<int64_t>(n) * n, 32);
        sk.lioff = skli;
        skli += 256 * ((n + 15) / 16);
        sk.gid = static_cast<int32_t>(P.skels.size());
        sk.poff = poff;
        poff += n;
        P.skels.push_back(g);
        P.skel_desc.push_back(sk);
        P.max_skel_n = std::max(P.max_skel_n, n);
    }
    P.skel_ntotal = poff;
    P.m_elems = std::max<int64_t>(moff, 32);
    P.t_elems = std::max<int64_t>(toff, 32);
    P.g_elems = std::max<int64_t>(goff, 32);
    P.skli_elems = std::max<int64_t>(skli, 256);
    big_family_ws(P.sep_apply, ws);
    P.ws_elems = ws;
}

void skel_apply_tables(const LevelPlan& P, const int32_t* k, const int32_t* perm, int lds_apply_cap,
                       std::vector<ApplyDesc>& skel_apply, std::vector<int32_t>& skel_dofs, int64_t& ws_elems,
                       double& skel_flops, double& skel_apply_bytes) {
    if (P.lists_pending) throw std::logic_error("leaf groups without their unknowns");
    skel_flops = 0.0;
    skel_apply_bytes = 0.0;
    skel_apply.clear();
    skel_apply.reserve(P.skel_desc.size());
    skel_dofs.resize(std::max<int32_t>(P.skel_ntotal, 0));
    size_t ndofs = 0;
    for (size_t e = 0; e < P.skel_desc.size(); ++e) {
        const SkelDesc& sk = P.skel_desc[e];
        const int g = P.skels[e];
        const int n = sk.n;
        const int kk = k[sk.gid];
        const int32_t* pv = perm + sk.poff;
        const int32_t* gd = P.gdofs.data() + P.gptr[g];
        const double nr = n - kk, kd = kk, rr = sk.r, nd = n;
        // ID by pivoted QR of an r x n block to rank k, then the skeleton elimination
        skel_flops += std::max(0.0, 4.0 * rr * nd * kd - 2.0 * kd * kd * (rr + nd) + 4.0 * kd * kd * kd / 3.0) +
                      rr * nd + nr * nr * kd + nr * nr * nr / 3.0 + nr * nr * kd + kd * kd * nr;
        if (kk == n) continue;
        skel_apply_bytes += 8.0 * (nr * (nr + 1.0) / 2.0 + 2.0 * kd * nr) + 8.0 * 2.0 * nd;
        ApplyDesc ad{};
        ad.ext = -1;
        ad.li = sk.lioff;
        ad.off = sk.goff;
        ad.toff = (kk > 0) ? sk.toff : -1;
        ad.yoff = -1;
        ad.wsoff = -1;
        if (n > lds_apply_cap) {
            ad.wsoff = ws_elems;
            ws_elems += align_up(n, 32);
        }
        ad.ld = n;
        ad.nI = n - kk;
        ad.nB = kk;
        ad.dofs = static_cast<int32_t>(ndofs);
        // redundant unknowns first, then the skeleton
        int32_t* o = skel_dofs.data() + ndofs;
        for (int q = kk; q < n; ++q) *o++ = gd[pv[q]];
        for (int q = 0; q < kk; ++q) *o++ = gd[pv[q]];
        ndofs += n;
        skel_apply.push_back(ad);
    }
    big_family_ws(skel_apply, ws_elems);
    skel_dofs.resize(ndofs);
}

int64_t next_active_set(const LevelPlan& P, const int32_t* k, const int32_t* perm, PlanScratch& scr) {
    if (P.lists_pending) throw std::logic_error("leaf groups without their unknowns");
    // the interiors are eliminated; the separator groups keep their unknowns, the skeletonized
    // ones only their skeleton
    const int ng = static_cast<int>(P.gptr.size()) - 1;
    std::vector<int32_t>& kp = scr.keep_ptr;
    kp.assign(ng + 1, 0);
    for (int g = 0; g < ng; ++g) kp[g + 1] = P.gcls[g] != 0 ? P.gptr[g + 1] - P.gptr[g] : 0;
    std::vector<int32_t>& sk_of = scr.skel_of;
    sk_of.assign(ng, -1);
    for (size_t e = 0; e < P.skel_desc.size(); ++e) {
        const int g = P.skels[e];
        const int kk = k[P.skel_desc[e].gid];
        if (kk < 0 || kk > P.skel_desc[e].n) throw std::logic_error("rank out of range");
        sk_of[g] = static_cast<int32_t>(e);
        kp[g + 1] = kk;
    }
    for (int g = 0; g < ng; ++g) kp[g + 1] += kp[g];
    std::vector<int32_t>& kt = scr.keep_t;
    kt.resize(kp[ng] + 1);   // one slack entry for the branch-free compaction below
    // (plain local pointers: the stamps, the output and the counters do not alias)
    int32_t* __restrict__ mark = scr.mark_stamp.data();
    int32_t* __restrict__ out = kt.data();
    const int32_t* __restrict__ kpp = kp.data();
    int32_t stamp = scr.stamp;
    for (int g = 0; g < ng; ++g) {
        int32_t* o = out + kpp[g];
        const int n = kpp[g + 1] - kpp[g];
        const int e = sk_of[g];
        if (e < 0) {
            for (int t = 0; t < n; ++t) o[t] = t;
            continue;
        }
        // skeleton positions in ascending order
        const int nn = P.skel_desc[e].n;
        const int32_t* pv = perm + P.skel_desc[e].poff;
        bool bad = false;
        for (int q = 0; q < n; ++q) bad |= static_cast<uint32_t>(pv[q]) >= static_cast<uint32_t>(nn);
        if (bad) throw std::logic_error("pivot position out of range");
        if (nn <= 64) {
            uint64_t m = 0;
            for (int q = 0; q < n; ++q) m |= uint64_t(1) << pv[q];
            for (; m != 0; m &= m - 1) *o++ = __builtin_ctzll(m);
        } else {
            const int32_t st = ++stamp;
            for (int q = 0; q < n; ++q) mark[pv[q]] = st;
            for (int t = 0; t < nn; ++t) {
                *o = t;
                o += mark[t] == st ? 1 : 0;
            }
        }
        if (o != out + kpp[g + 1]) throw std::logic_error("pivot order is not a permutation");
    }
    scr.stamp = stamp;
    kt.resize(kp[ng]);
    return kp[ng];
}

int64_t finish_level(const LevelPlan& P, const int32_t* k, const int32_t* perm, int lds_apply_cap,
                     std::vector<ApplyDesc>& skel_apply, std::vector<int32_t>& skel_dofs, int64_t& ws_elems,
                     PlanScratch& scr, double& skel_flops, double& skel_apply_bytes) {
    skel_apply_tables(P, k, perm, lds_apply_cap, skel_apply, skel_dofs, ws_elems, skel_flops, skel_apply_bytes);
    return next_active_set(P, k, perm, scr);
}

}  // namespace rhif

namespace rhif {

namespace {
[[noreturn]] void bad(const char* what, int64_t a, int64_t b) {
    throw std::logic_error(std::string("plan check failed: ") + what + " (" + std::to_string(a) + " vs " +
                           std::to_string(b) + ")");
}
inline void need(bool ok, const char* what, int64_t a = 0, int64_t b = 0) {
    if (!ok) bad(what, a, b);
}
}  // namespace

void validate_level(const LevelPlan& P, const LevelPlan* prev, int d) {
    validate_cells(P, prev, d);
    if (!P.root) validate_separators(P);
}

void validate_cells(const LevelPlan& P, const LevelPlan* prev, int d) {
    // every cell's boundary groups follow its interior in list order and cover the frontal
    // (the skeletonization kernel derives group sizes from consecutive offsets)
    for (int64_t c = 0; c < P.ncells; ++c) {
        int at = P.c_nI[c];
        for (int e = P.c_gptr[c]; e < P.c_gptr[c + 1]; ++e) {
            need(P.c_goff[e] == at, "cell group layout", P.c_goff[e], at);
            const int h = P.c_g[e];
            need(h >= 0 && h + 1 < static_cast<int64_t>(P.gptr.size()), "cell group index");
            at += P.gptr[h + 1] - P.gptr[h];
        }
        need(at == P.c_nf[c], "cell groups cover the frontal", at, P.c_nf[c]);
    }
    need(static_cast<int64_t>(P.c_dptr.size()) == P.ncells + 1, "cell dof offsets");
    const int64_t ncd = P.c_dptr[P.ncells];
    need(P.dofs_on_device || static_cast<int64_t>(P.c_dofs.size()) == ncd, "cell dofs", P.c_dofs.size(), ncd);
    for (int c = 0; c < P.ncells; ++c) {
        const CellRef& r = P.cell_ref[c];
        need(r.nf == P.c_nI[c] + P.c_nB[c], "cell nf");
        need(r.ld >= r.nf && r.ld >= 1, "cell ld", r.ld, r.nf);
        need(r.off >= 0 && r.off + static_cast<int64_t>(r.ld) * r.nf <= P.front_elems, "frontal bounds",
             r.off + static_cast<int64_t>(r.ld) * r.nf, P.front_elems);
        need(r.dptr >= 0 && r.dptr + r.nf <= ncd, "cell dofs bounds", r.dptr + r.nf, ncd);
    }
    for (const Tile& t : P.tiles) {
        need(t.cell >= 0 && t.cell < P.ncells, "tile cell", t.cell, P.ncells);
        need(t.r0 >= 0 && t.r0 < P.cell_ref[t.cell].nf && t.c0 >= 0 && t.c0 < P.cell_ref[t.cell].nf, "tile origin");
        if (t.shape != 0) {
            const int rows = (t.shape >> 8) & 0xff, cols = t.shape & 0xff;
            need(rows >= 1 && rows <= 64 && cols >= 1 && cols <= 64 && (t.shape & ~(kTileBand | 0xffff)) == 0,
                 "tile shape", rows, cols);
            need(t.r0 + rows <= P.cell_ref[t.cell].nf && t.c0 + cols <= P.cell_ref[t.cell].nf, "tile extent");
        }
    }
    for (const FrontDesc& f : P.cell_potrf) {
        need(f.id >= 0 && f.id < P.ncells, "potrf id");
        const CellRef& r = P.cell_ref[f.id];
        need(f.off == r.off && f.ld == r.ld && f.n == r.nf && f.p >= 1 && f.p <= f.n, "potrf desc");
        need(f.ext >= 0 && f.ext + (f.p + 15) / 16 <= P.ext_elems, "potrf ext bounds");
    }
    const int W = 1 << d;
    if (prev != nullptr && P.src_on_device) {
        need(static_cast<int64_t>(P.c_g2.size()) == ncd && static_cast<int64_t>(P.c_t2.size()) == ncd,
             "extend-add source lists", P.c_g2.size(), ncd);
    } else if (prev != nullptr) {
        need(static_cast<int64_t>(P.src.size()) == ncd * 2 * W, "src size", P.src.size(), ncd * 2 * W);
        for (int64_t e = 0; e < ncd * W; ++e) {
            const int c = P.src[2 * e], pos = P.src[2 * e + 1];
            if (c < 0) continue;
            need(c < prev->ncells, "src child", c, prev->ncells);
            need(pos >= prev->c_nI[c] && pos < prev->c_nf[c], "src child position", pos, prev->c_nf[c]);
        }
    }
    int64_t ysum = 0;
    for (const ApplyDesc& a : P.cell_apply) {
        need(a.nI >= 1 && a.dofs >= 0 && a.dofs + a.nI + a.nB <= ncd, "cell apply dofs");
        need(a.off >= 0 && a.off + static_cast<int64_t>(a.ld) * (a.nI + a.nB) <= P.front_elems, "cell apply bounds");
        need(a.ld >= a.nI + a.nB, "cell apply ld");
        if (a.yoff >= 0) need(a.yoff + a.nB <= P.y_elems, "cell apply y bounds");
        if (a.wsoff >= 0) need(a.wsoff + a.nI + a.nB <= P.ws_elems, "cell apply ws bounds");
        need(a.ext >= 0 && a.ext + (a.nI + 15) / 16 <= P.ext_elems, "cell apply ext bounds");
        ysum += a.nB;
    }
    need(ysum <= P.y_elems, "y scratch", ysum, P.y_elems);
}

void validate_separators(const LevelPlan& P) {
    for (const SepDesc& s : P.sep_desc) {
        need(s.nslot >= 1 && s.nslot <= kMaxSlots, "sep slots", s.nslot, kMaxSlots);
        need(s.n >= 1 && s.loff >= 0 && s.loff + static_cast<int64_t>(s.n) * s.n <= P.lg_elems, "sep L bounds");
        need(s.lioff >= 0 && s.lioff + 256 * static_cast<int64_t>((s.n + 15) / 16) <= P.li_elems, "sep Li bounds");
        need(s.dofs >= 0 && s.dofs + s.n <= static_cast<int64_t>(P.sep_dofs.size()), "sep dofs");
        for (int q = 0; q < s.nslot; ++q) {
            const int c = s.slot_cell[q];
            need(c >= 0 && c < P.ncells, "sep slot cell", c, P.ncells);
            need(s.slot_off[q] >= P.c_nI[c] && s.slot_off[q] + s.n <= P.c_nf[c], "sep slot offset");
        }
    }
    for (const CellScaleDesc& cs : P.cell_scale) {
        need(cs.g_begin >= 0 && cs.g_begin + cs.g_count <= static_cast<int64_t>(P.cell_groups.size()), "scale groups");
        int64_t tot = 0;
        for (int e = cs.g_begin; e < cs.g_begin + cs.g_count; ++e) {
            const CellGroup& g = P.cell_groups[e];
            need(g.off >= cs.nI && g.off + g.n <= cs.nI + cs.nB, "scale group offset");
            need(g.loff >= 0 && g.loff + static_cast<int64_t>(g.n) * g.n <= P.lg_elems, "scale group L");
            need(g.lioff >= 0 && g.lioff + 256 * static_cast<int64_t>((g.n + 15) / 16) <= P.li_elems,
                 "scale group Li");
            tot += g.n;
        }
        need(tot == cs.nB, "scale groups cover the boundary", tot, cs.nB);
        for (int e = cs.g_begin; e < cs.g_begin + cs.g_count; ++e)
            need(&P.cell_scale[P.cell_groups[e].cell] == &cs, "scale group cell index");
    }
    for (const SkelDesc& k : P.skel_desc) {
        need(k.nslot >= 1 && k.nslot <= 2, "skel slots");
        need(k.grp >= 0 && k.grp + 1 < static_cast<int64_t>(P.gptr.size()) && P.gptr[k.grp + 1] - P.gptr[k.grp] == k.n,
             "skel group");
        for (int q = 0; q < k.nslot; ++q) {
            const int c = k.cell[q];
            need(c >= 0 && c < P.ncells, "skel cell");
            need(k.off[q] >= P.c_nI[c] && k.off[q] + k.n <= P.c_nf[c], "skel group offset");
        }
        need(k.moff >= 0 && k.moff + static_cast<int64_t>(std::max(k.r, 1)) * (k.n | 1) <= P.m_elems, "skel M bounds");
        need(k.toff >= 0 && k.toff + static_cast<int64_t>(k.n) * k.n / 4 + 1 <= P.t_elems, "skel T bounds");
        need(k.goff >= 0 && k.goff + static_cast<int64_t>(k.n) * k.n <= P.g_elems, "skel G bounds");
        need(k.lioff >= 0 && k.lioff + 256 * static_cast<int64_t>((k.n + 15) / 16) <= P.skli_elems, "skel Li bounds");
        need(k.poff >= 0 && k.poff + k.n <= P.skel_ntotal, "skel perm bounds");
        need(k.gid >= 0 && k.gid < static_cast<int>(P.skel_desc.size()), "skel gid");
    }
    for (const GatherDesc& g : P.gather) {
        need(g.dofs >= 0 && g.dofs + g.n <= static_cast<int64_t>(P.sep_dofs.size()), "gather dofs");
        for (int q = 0; q < g.nslot; ++q) need(g.yoff[q] >= 0 && g.yoff[q] + g.n <= P.y_elems, "gather y bounds");
    }
    for (const ApplyDesc& a : P.sep_apply) {
        need(a.nB == 0 && a.nI >= 1 && a.ld == a.nI, "sep apply shape");
        need(a.off >= 0 && a.off + static_cast<int64_t>(a.nI) * a.nI <= P.lg_elems, "sep apply bounds");
        need(a.dofs >= 0 && a.dofs + a.nI <= static_cast<int64_t>(P.sep_dofs.size()), "sep apply dofs");
        if (a.wsoff >= 0) need(a.wsoff + a.nI <= P.ws_elems, "sep apply ws bounds");
    }
}

void validate_skel_apply(const LevelPlan& P, const std::vector<ApplyDesc>& ad, const std::vector<int32_t>& dofs,
                         int64_t N) {
    for (const ApplyDesc& a : ad) {
        need(a.nI >= 1 && a.nB >= 0 && a.ld == a.nI + a.nB, "skel apply shape");
        need(a.off >= 0 && a.off + static_cast<int64_t>(a.ld) * a.ld <= P.g_elems, "skel apply bounds");
        if (a.toff >= 0) need(a.toff + static_cast<int64_t>(a.nB) * a.nI <= P.t_elems, "skel apply T bounds");
        need(a.dofs >= 0 && a.dofs + a.nI + a.nB <= static_cast<int64_t>(dofs.size()), "skel apply dofs");
    }
    for (int32_t i : dofs) need(i >= 0 && i < N, "skel dof range", i, N);
}

}  // namespace rhif
