// Host planner: the integer bookkeeping of one level of the factorization.
//
// Level l works at cell width w = 2^l m. An active unknown x is classified by
// key_k = 2 (x_k / w) + (x_k mod w != 0): odd components are the open slab of a cell,
// even ones the separator plane x_k = (key_k / 2) w. Unknowns with equal keys form one
// group; the number of even components is its class (0 cell interior, 1 edge in 2D or
// face in 3D, 2 corner in 2D or edge in 3D, 3 corner in 3D) -- the grouping of Sec. 3.1
// and 3.2 of the paper, extended to any side n by letting the last cell of an axis be
// ragged and the plane x_k = n be a separator with a cell on one side only.
#pragma once
#include <cstdint>
#include <vector>

#include "devstructs.hpp"

namespace rhif {

struct GridInfo {
    int d = 0;
    int s = 0;          // interior points per axis
    int64_t N = 0;
};

struct LevelPlan {
    int level = 0;
    int w = 0;
    int nc1 = 0;        // cells per axis
    bool root = false;  // the last level: one cell, everything interior
    // level 0 only: the cells' frontal unknowns (c_dofs) are written by the device from the
    // closed form of leafgeom.hpp (c_dofs stays empty; c_dptr holds the offsets), and the
    // groups' unknowns and separator lists wait for fill_leaf_lists
    bool dofs_on_device = false;
    bool lists_pending = false;
    // levels >= 1: the extend-add source table (src) is built by the device from c_g2 / c_t2
    // and the level below's slot tables (src stays empty)
    bool src_on_device = false;

    // groups (ascending key), their unknowns ascending
    std::vector<int32_t> gptr;      // ngroups + 1
    std::vector<int32_t> gdofs;
    std::vector<int8_t> gcls;
    std::vector<int32_t> gslot_cnt; // per group, cells containing it
    std::vector<int32_t> gslot_cell;  // ngroups * kMaxSlots
    std::vector<int32_t> gslot_off;

    // cells (every geometric cell of the level)
    int ncells = 0;
    std::vector<int32_t> c_nI, c_nB, c_nf, c_ld, c_dptr;
    std::vector<int64_t> c_foff;
    int64_t front_elems = 0;
    std::vector<int32_t> c_dofs;    // frontal unknowns of every cell
    std::vector<int32_t> c_gptr;    // boundary groups of every cell
    std::vector<int32_t> c_g;
    std::vector<int32_t> c_goff;

    // separator groups (class >= 1) and the skeletonized ones (class 1)
    std::vector<int32_t> seps;
    std::vector<int32_t> g_g2, g_t2;   // sources at the level below, aligned with gdofs
    std::vector<int32_t> c_g2, c_t2;   // and with c_dofs
    std::vector<int32_t> skels;

    // device-ready tables
    std::vector<FrontDesc> cell_potrf;     // cells with interior unknowns
    std::vector<CellRef> cell_ref;         // every cell
    std::vector<Tile> tiles;               // assembly tiles
    std::vector<int32_t> src;              // extend-add sources: per frontal position
                                           // (2^d pairs of child cell, child position)
    std::vector<SepDesc> sep_desc;
    std::vector<CellGroup> cell_groups;
    std::vector<CellScaleDesc> cell_scale;
    std::vector<SkelDesc> skel_desc;
    std::vector<ApplyDesc> cell_apply;
    std::vector<ApplyDesc> sep_apply;
    std::vector<GatherDesc> gather;
    std::vector<int32_t> sep_dofs;         // unknowns of every separator group
    int64_t lg_elems = 0, li_elems = 0, skli_elems = 0, m_elems = 0, t_elems = 0, g_elems = 0, y_elems = 0;
    int64_t ext_elems = 0;                 // per-panel nonzero row ends of the cells' L
    int64_t ws_elems = 0;                  // global workspace for oversized applies
    int32_t skel_ntotal = 0;               // sum of skeletonized group sizes
    int32_t max_nf = 0, max_sep_n = 0, max_skel_n = 0, max_cell_groups = 0;
    double flops = 0.0;                    // algorithmic flops (cells + groups + skeletons)
    // algorithmic work per launch class (what the method must do, not what a kernel does):
    // level-0 cell interiors count as banded matrices of bandwidth (m-1)^(d-1)
    double alg_elim_flops = 0.0;           // cell elimination (potrf + trsm + syrk)
    double alg_prec_chol_flops = 0.0;      // group Cholesky
    double alg_prec_scale_flops = 0.0;     // two-sided scaling
    double alg_front_bytes = 0.0;          // frontal assembly (frontal writes + sources)
    double alg_apply_cell_bytes = 0.0;     // one sweep over the cells (L, W, vectors)
    double alg_apply_sep_bytes = 0.0;      // one sweep over the groups (L_g, vectors)
    double alg_gather_bytes = 0.0;         // one gather

    // Empty every table but keep the allocations (plans are reused across factorizations).
    void reset();
};

// Reusable per-factorization scratch sized by N.
struct PlanScratch {
    std::vector<int32_t> count;            // key buckets
    std::vector<int32_t> key2g;
    // the unknowns that stay active, per group of the level just finished: positions in the
    // group's ascending list (set by next_active_set, read by the next level's build_cells)
    std::vector<int32_t> keep_ptr, keep_t;
    std::vector<int32_t> box_lo, box_n;    // leaf-level group boxes
    std::vector<int32_t> mark_stamp;
    std::vector<int32_t> par_of;
    std::vector<int32_t> akey;             // per group of the level below: its key here
    std::vector<int32_t> pos, ord, tmp, skel_of;
    std::vector<int64_t> cell_y;           // per cell: its offset in the apply scratch
    int32_t stamp = 0;
    void init(int64_t N);
    // Make room for N unknowns without clearing the stamps (they only grow); starts a new
    // factorization (nothing kept from a level below).
    void reserve(int64_t N);
};

// Leaf cells (level 0, not the root) whose interior, in natural order, has bandwidth
// (w - 1)^(d - 1) <= 16: their Cholesky factor is block bidiagonal in 16 x 16 blocks, and
// only those blocks, the boundary rows and the boundary block of the frontal are used.
inline bool leaf_interior_banded(int d, int level, bool root, int w) {
    if (level != 0 || root) return false;
    int bw = 1;
    for (int k = 1; k < d; ++k) bw *= (w - 1);
    return bw <= 16;
}

// Number of skeletonization levels L: all l >= 0 with 2^l m <= s.
int num_levels(int s, int leaf);

// Build the plan of `level` with n_active active unknowns: at level 0 every unknown, above it
// the unknowns next_active_set kept from the level below. `prev` is the plan of the level
// below (nullptr at level 0); its groups and the kept lists in scr give this level's groups,
// and it is used for the extend-add source tables.
// lds_apply_cap: largest nI + nB staged in LDS by the apply kernels.
// The work is split in two halves so that the second can overlap device work:
//   build_cells: groups, cell frontals, assembly tiles, elimination and cell apply tables;
//   build_separators: block-Jacobi, ID / skeleton and gather tables (not at the root).
// device_tables: leave the largest per-unknown table to the device. At level 0 (every unknown
// active) that is c_dofs, and gdofs waits for fill_leaf_lists, which must run before
// build_separators; at levels >= 1 it is the extend-add source table src.
void build_cells(const GridInfo& g, int level, int leaf, bool root, int64_t n_active, const LevelPlan* prev,
                 PlanScratch& scr, int lds_apply_cap, LevelPlan& out, bool device_tables = false);
void fill_leaf_lists(const GridInfo& g, PlanScratch& scr, LevelPlan& out);
void build_separators(const GridInfo& g, PlanScratch& scr, int lds_apply_cap, LevelPlan& out);
// Both halves.
void build_level(const GridInfo& g, int level, int leaf, bool root, int64_t n_active, const LevelPlan* prev,
                 PlanScratch& scr, int lds_apply_cap, LevelPlan& out);

// Check that every offset and size in the device tables of a level stays inside the
// buffers the driver allocates for them (throws std::logic_error otherwise), so that a
// planning mistake becomes an error return instead of an out-of-bounds access on the GPU.
// prev: the plan of the level below (its frontals are read by the extend-add).
void validate_cells(const LevelPlan& lp, const LevelPlan* prev, int d);
void validate_separators(const LevelPlan& lp);
void validate_level(const LevelPlan& lp, const LevelPlan* prev, int d);

// Same for the skeleton apply tables built by finish_level.
void validate_skel_apply(const LevelPlan& lp, const std::vector<ApplyDesc>& ad,
                         const std::vector<int32_t>& dofs, int64_t N);

// After the IDs of a level, given ranks k and pivot orders (positions into each group's
// ascending unknowns): skel_apply_tables builds the apply descriptors of the skeleton blocks
// (and the level's skeletonization flops and apply bytes); next_active_set records, per
// group, which unknowns stay active (all of a separator group, the skeleton of a
// skeletonized one, none of an interior), which is all the next level's plan needs, and
// returns their number; finish_level does both.
void skel_apply_tables(const LevelPlan& lp, const int32_t* k, const int32_t* perm, int lds_apply_cap,
                       std::vector<ApplyDesc>& skel_apply, std::vector<int32_t>& skel_dofs, int64_t& ws_elems,
                       double& skel_flops, double& skel_apply_bytes);
int64_t next_active_set(const LevelPlan& lp, const int32_t* k, const int32_t* perm, PlanScratch& scr);
int64_t finish_level(const LevelPlan& lp, const int32_t* k, const int32_t* perm, int lds_apply_cap,
                     std::vector<ApplyDesc>& skel_apply, std::vector<int32_t>& skel_dofs, int64_t& ws_elems,
                     PlanScratch& scr, double& skel_flops, double& skel_apply_bytes);

}  // namespace rhif
