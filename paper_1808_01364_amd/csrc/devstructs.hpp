// Plain-old-data tables shared by the host planner and the device kernels.
//
// All dense blocks are FP64, column-major. A "frontal" is the dense matrix of one cell of
// the current level over the active unknowns of its closed cell: its interior unknowns
// first, then its boundary groups (edges/corners in 2D, faces/edges/corners in 3D) one
// after another, every group in ascending linear index. A frontal holds the cell's own
// additive share of the current matrix A_l; the shares of all cells sum to A_l.
#pragma once
#include <cstdint>

namespace rhif {

constexpr int kMaxSlots = 8;   // cells whose closure contains one group (2^d, d <= 3)

// One dense matrix of a batch (frontal, group diagonal block, skeleton block).
struct FrontDesc {
    int64_t off;     // element offset into the pool
    int32_t ld;      // leading dimension
    int32_t n;       // order
    int32_t p;       // number of leading pivots to eliminate (p <= n)
    int32_t id;      // block id reported on loss of positive definiteness
    int32_t ext;     // >= 0: offset of ceil(p/16) ints receiving, for every 16-column panel
                     // of L, the end of its nonzero rows below the diagonal (rows < p)
    int32_t pad;
};

// Reference to a cell frontal of some level (for gathers from children / neighbours).
struct CellRef {
    int64_t off;
    int32_t ld;
    int32_t nI;
    int32_t nf;
    int32_t dptr;    // offset of the frontal's unknowns in the level's cell-dof array
};

// A tile of a frontal to be assembled (64 x 64 elements starting at (r0, c0)).
struct Tile {
    int32_t cell;
    int32_t r0;
    int32_t c0;
    int32_t shape;   // 0: 64 x 64; else kTileBand | rows << 8 | cols (rows, cols <= 64)
};
constexpr int32_t kTileBand = 1 << 30;   // write only the diagonal and first subdiagonal 16 x 16 blocks
inline int32_t tile_shape(int rows, int cols, bool band) {
    return (band ? kTileBand : 0) | (rows << 8) | cols;
}

// A separator group for the block-Jacobi step: where its diagonal block sits in every
// cell frontal that contains it, and where its Cholesky factor goes.
struct SepDesc {
    int32_t n;
    int32_t nslot;
    int32_t slot_cell[kMaxSlots];
    int32_t slot_off[kMaxSlots];   // frontal position of the group's first unknown
    int64_t loff;                  // offset of L_g (n x n, ld n) in the group pool
    int32_t dofs;                  // offset of its unknowns in the level's group-dof array
    int32_t lioff;                 // offset of the inverses of L_g's 16 x 16 diagonal blocks
};

// One boundary group of one cell, for the two-sided block-Jacobi scaling of the cell.
struct CellGroup {
    int32_t off;     // frontal position of the group's first unknown
    int32_t n;
    int64_t loff;    // L_g offset in the group pool
    int32_t owner;   // 1 if this cell holds the group's diagonal block after scaling
    int32_t cell;    // index of the cell's CellScaleDesc
    int32_t lioff;   // offset of the inverses of L_g's 16 x 16 diagonal blocks
    int32_t pad;
};

struct CellScaleDesc {
    int64_t off;     // frontal offset
    int32_t ld;
    int32_t nI;
    int32_t nB;
    int32_t g_begin; // first CellGroup of this cell
    int32_t g_count;
    int32_t pad;
};

// One edge (2D) / face (3D) to be skeletonized.
struct SkelDesc {
    int32_t n;           // group size
    int32_t r;           // rows of M = A[R_g, g]
    int32_t nslot;       // cells containing the group (1 or 2)
    int32_t grp;         // group index (its entry in the cells' group lists)
    int32_t cell[2];
    int32_t off[2];      // frontal position of the group's first unknown in each cell
    int64_t moff;        // scratch for M (r x n) and later A_hat,hat T
    int64_t toff;        // T (k x (n-k), ld k), room for floor(n^2/4)+1
    int64_t goff;        // skeleton block G (n x n): [A~_tt, .; A~_ht, A_hh]
    int32_t gid;         // index into the rank / pivot outputs
    int32_t poff;        // offset of this group's pivot order in the pivot output
    int32_t lioff;       // inverses of the 16 x 16 diagonal blocks of L~ (room for n)
    int32_t pad;
};

// State of one group's multi-workgroup interpolative decomposition between the step kernels.
struct BigState {
    double r11;          // |R_11|
    double v0, alpha, beta;   // reflector of the current step: v = (x0 - alpha, x1, ...), beta = 2 / v^T v
    int32_t pc;          // pivot column of the current step
    int32_t active;      // 0 once the rank test failed or every column was taken
    int32_t k;           // steps taken (the rank once inactive)
    int32_t pad;
};

// One block of the factor apply: L in [0,nI)^2 and W^T in rows [nI, nI+nB) of columns
// [0, nI) of the matrix at `off`; optionally an interpolation matrix T (nB x nI, ld nB).
struct ApplyDesc {
    int64_t off;
    int64_t toff;        // -1: no T
    int64_t yoff;        // >= 0: write y = W^T z_I to the scratch; -1: z_B -= y in place
    int64_t wsoff;       // >= 0: stage z_I, z_B in this global workspace instead of LDS
    int32_t ld;
    int32_t nI;
    int32_t nB;
    int32_t dofs;        // offset of nI interior then nB boundary unknowns (global indices)
    int32_t ext;         // >= 0: per-panel nonzero row ends of L (see FrontDesc::ext)
    int32_t li;          // offset of the inverses of L's 16 x 16 diagonal blocks (256 each)
    int64_t zoff;        // offset of the block's problem in the vector (several problems at once)
};

// Apply blocks whose largest interior exceeds kBigApplyMinI are applied panel by panel over
// many workgroups per block (panels of kBigApplyPanel columns); every block of such a family
// stages its vectors in the global workspace.
constexpr int kBigApplyMinI = 272;   // the largest interior of the split apply
constexpr int kBigApplyPanel = 128;

// Gather of the up-sweep boundary contributions of the cells for one separator group.
struct GatherDesc {
    int32_t n;
    int32_t dofs;
    int32_t nslot;
    int32_t pad;
    int64_t yoff[kMaxSlots];  // scratch position of the group's first unknown in each cell
    int64_t zoff;             // offset of the group's problem in the vector
};

// The separator-group part of one level of the factor apply, one workgroup per group: the
// gather of the cells' contributions (up-sweep), the block-Jacobi factor L_g (preconditioned
// levels) and, for a skeletonized group with redundant unknowns, its skeleton elimination.
struct GroupApplyDesc {
    int32_t n;          // group size
    int32_t dofs;       // offset of its unknowns (ascending) in the level's group-dof array
    int32_t nslot;      // cells contributing to the gather
    int32_t precond;    // 1: apply L_g
    int64_t yoff[kMaxSlots];
    int64_t loff;       // L_g (n x n) in the block-Jacobi pool
    int32_t li;         // inverses of L_g's 16 x 16 diagonal blocks
    int32_t nr;         // redundant unknowns of the skeleton elimination (0: none)
    int32_t k;          // skeletons
    int32_t poff;       // group-local pivot order in the level's pivot array
    int64_t goff;       // G (n x n) in the skeleton pool
    int64_t toff;       // T (k x nr, ld k) in the T pool
    int32_t skli;       // inverses of L~'s 16 x 16 diagonal blocks
    int32_t pad;
    int64_t zoff;       // offset of the group's problem in the vector
};

// One problem of a PCG solve over several problems at once: its matrix, its place in the
// concatenated vectors, and its blocks in the grids of the vector kernels (the grid a lone
// solve of the problem uses, so that every sum is formed in the same order).
struct BatchSeg {
    const int32_t* rp;
    const int32_t* ci;
    const double* val;
    int64_t zoff;        // first unknown of the problem in the vectors
    int64_t n;           // its unknowns
    int32_t b0;          // its first block
    int32_t nb;          // its number of blocks
};

}  // namespace rhif
