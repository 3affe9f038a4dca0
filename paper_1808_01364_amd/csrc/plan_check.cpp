// Host-only planner dry run (include/rhif_plan.h).
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/rhif_plan.h"
#include "leafgeom.hpp"
#include "plan.hpp"

namespace {
thread_local std::string g_plan_error;
}

extern "C" const char* rhif_plan_last_error(void) { return g_plan_error.c_str(); }

extern "C" rhif_status rhif_plan_dry_run(const rhif_grid* g, int32_t leaf, rhif_id_choice_fn choose,
                                         void* choose_ctx, rhif_cell_fn cell, void* cell_ctx,
                                         int64_t* root_size) {
    using namespace rhif;
    try {
        if (!g || (g->dim != 2 && g->dim != 3) || g->n[0] < 1 || leaf < 2 || !choose)
            throw std::invalid_argument("bad grid, leaf or callback");
        for (int k = 1; k < g->dim; ++k)
            if (g->n[k] != g->n[0]) throw std::invalid_argument("only cubic grids");
        GridInfo gi;
        gi.d = g->dim;
        gi.s = g->n[0];
        gi.N = 1;
        for (int k = 0; k < gi.d; ++k) gi.N *= gi.s;
        const int L = num_levels(gi.s, leaf);
        PlanScratch scr;
        scr.init(gi.N);
        int64_t n_active = gi.N;
        std::vector<LevelPlan> plans(L + 1);
        int64_t ws = 0;
        for (int lvl = 0; lvl <= L; ++lvl) {
            const bool root = lvl == L;
            LevelPlan& P = plans[lvl];
            build_level(gi, lvl, leaf, root, n_active, lvl ? &plans[lvl - 1] : nullptr, scr, 7000, P);
            validate_level(P, lvl ? &plans[lvl - 1] : nullptr, gi.d);
            if (lvl == 0) {
                // the closed form the device uses for the leaf cells' frontal unknowns
                for (int c = 0; c < P.ncells; ++c) {
                    for (int q = 0; q < P.c_nf[c]; ++q)
                        if (leaf_frontal_dof(gi.d, gi.s, P.w, P.nc1, c, q) != P.c_dofs[P.c_dptr[c] + q])
                            throw std::logic_error("closed-form leaf frontal unknowns differ from the plan");
                    if (leaf_frontal_dof(gi.d, gi.s, P.w, P.nc1, c, P.c_nf[c]) != -1)
                        throw std::logic_error("closed-form leaf frontal is larger than the plan's");
                }
            }
            if (cell)
                for (int c = 0; c < P.ncells; ++c)
                    if (P.c_nI[c] > 0)
                        cell(cell_ctx, lvl, c, P.c_nI[c], P.c_nB[c], P.c_dofs.data() + P.c_dptr[c]);
            if (root) break;
            std::vector<int32_t> ks(P.skel_desc.size()), perm(P.skel_ntotal);
            for (size_t e = 0; e < P.skel_desc.size(); ++e) {
                const SkelDesc& sk = P.skel_desc[e];
                const int gidx = P.skels[e];
                int32_t k = 0;
                if (choose(choose_ctx, lvl, P.gdofs[P.gptr[gidx]], sk.n, &k, perm.data() + sk.poff) != 0)
                    throw std::invalid_argument("choice callback stopped the run");
                if (k < 0 || k > sk.n) throw std::invalid_argument("rank out of range");
                std::vector<char> seen(sk.n, 0);
                for (int q = 0; q < sk.n; ++q) {
                    const int v = perm[sk.poff + q];
                    if (v < 0 || v >= sk.n || seen[v]) throw std::invalid_argument("pivot order is not a permutation");
                    seen[v] = 1;
                }
                ks[sk.gid] = k;
            }
            std::vector<ApplyDesc> sad;
            std::vector<int32_t> sdofs;
            double fl = 0, by = 0;
            ws = std::max(ws, P.ws_elems);
            n_active = finish_level(P, ks.data(), perm.data(), 7000, sad, sdofs, ws, scr, fl, by);
            validate_skel_apply(P, sad, sdofs, gi.N);
        }
        if (root_size) *root_size = n_active;
        g_plan_error.clear();
        return RHIF_OK;
    } catch (const std::exception& e) {
        g_plan_error = e.what();
        return RHIF_EINVAL;
    }
}
