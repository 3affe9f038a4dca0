// Declarations of the device kernels (defined in kernels.hip) for the host driver.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "devstructs.hpp"

namespace rhif {

__global__ void k_fd_rowptr(int d, int s, int32_t* row_ptr);
__global__ void k_assemble_fd(int d, int s, double inv_h2, const double* a, const double* b,
                              const int32_t* row_ptr, int32_t* col, double* val);
__global__ void k_grad_log_a(int d, int s, double inv_h2, const double* a, const double* u, const double* lam,
                             double* g);
__global__ void k_leaf_dofs(const CellRef* cells, int d, int s, int w, int nc1, int32_t* cdofs);
__global__ void k_front_csr(const Tile* tiles, const CellRef* cells, const int32_t* cdofs, int d, int s, int w,
                            int nc1, const int32_t* row_ptr, const int32_t* col, const double* val, double* F);
__global__ void k_extend_src(const CellRef* cells, const int32_t* g2, const int32_t* t2, int ngroups2,
                             const int32_t* gslot_cnt, const int32_t* gslot_cell, const int32_t* gslot_off,
                             const CellRef* child, int nchild, int d, int pnc1, int nc1, int W, int level,
                             int32_t* src, unsigned long long* err);
__global__ void k_front_extend(const Tile* tiles, const CellRef* cells, const int32_t* src, int W, int d, int pnc1,
                               const CellRef* child, const double* Fc, double* F);
__global__ void k_potrf_batch(const FrontDesc* desc, double* pool, int panel_cap, int level, int step,
                              unsigned long long* err, int32_t* ext, double* linv);
template <bool F32>
__global__ void k_leaf_elim(const FrontDesc* desc, double* pool, double* linv, int tpw, int level,
                            unsigned long long* err, int32_t* ext);
__global__ void k_chol_lead(const FrontDesc* desc, double* pool, double* linv, int lds_pmax, int level, int step,
                            unsigned long long* err, int32_t* ext);
__global__ void k_trsm_rows(const FrontDesc* desc, double* pool, const double* linv, int pstride);
template <bool F32>
__global__ void k_syrk_schur(const FrontDesc* desc, double* pool);
__global__ void k_precond_groups(const SepDesc* sd, const CellRef* cells, const double* F, double* Lg, double* Li,
                                 int panel_cap, int lds_n, int level, unsigned long long* err);
__global__ void k_precond_gather(const SepDesc* sd, const CellRef* cells, const double* F, double* Lg);
__global__ void k_precond_scale(const CellScaleDesc* cd, const CellGroup* cg, const double* Lg, const double* Li,
                                double* F, int pstride, int phase);
// waves per SIMD of the skeletonization form for launches with many groups per CU
constexpr int kSkelWavesMany = 4;
// LDS of k_skeletonize beyond the partials of wg_cpqr_rows that the register ID needs
constexpr int kCpqrRegExtra = 64;
// rows of M per thread of the register forms of the ID compiled into k_skeletonize
constexpr int kSkelRegForms[3] = {16, 32, 96};
template <int STAGED, typename MR, int RMAX>
__global__ void k_skeletonize(const SkelDesc* sd, const int32_t* cgptr, const int32_t* cgl, const int32_t* cgoff,
                              const CellRef* cells, double* F,
                              double* Mpool, double* Tpool, double* Gpool, double* skli, double eps, int32_t* kout,
                              int32_t* pout, int panel_cap, int nmax, int rmax, int level, unsigned long long* err);
// interpolative decompositions of large groups across many workgroups
template <typename MR>
__global__ void k_big_gather(const SkelDesc* sd, const int32_t* cgptr, const int32_t* cgl, const int32_t* cgoff,
                             const CellRef* cells, const double* F, double* Mpool, double* nrm, int32_t* pos,
                             int32_t* pout, BigState* st, int nmax, int nblk, int level, unsigned long long* err);
template <typename MR>
__global__ void k_big_pivot(const SkelDesc* sd, const double* Mpool, const double* nsum, int32_t* pos, int32_t* pout,
                            BigState* st, double eps, int j, int nmax, int32_t* kout);
template <typename MR>
__global__ void k_big_colsum(const SkelDesc* sd, const BigState* st, const double* part, double* sum, int nmax,
                             int nblk);
template <typename MR>
__global__ void k_big_dot(const SkelDesc* sd, const double* Mpool, const int32_t* pos, const BigState* st,
                          double* wpart, int j, int nmax, int nblk);
template <typename MR>
__global__ void k_big_update(const SkelDesc* sd, double* Mpool, double* nrm, const int32_t* pos, const BigState* st,
                             const double* wsum, int j, int nmax, int nblk);
template <typename MR>
__global__ void k_big_trisolve(const SkelDesc* sd, double* Mpool, const int32_t* pout, const BigState* st,
                               double* Tpool, int ncol);
template <typename MR>
__global__ void k_big_elim(const SkelDesc* sd, const CellRef* cells, double* F, const double* Mpool, double* Gpool,
                           const int32_t* kout, const int32_t* pout, int phase);
constexpr int kTrisolveColsHost = 8;   // redundant columns per workgroup of k_big_trisolve
constexpr int kBigRowsHost = 64;    // rows of M per workgroup in the kernels above
__global__ void k_fwd_gt(const ApplyDesc* ad, const double* pool, const double* Tp, const int32_t* dofs,
                         const int32_t* ext, double* z);
__global__ void k_fwd_g(const ApplyDesc* ad, const double* pool, const double* Tp, const int32_t* dofs,
                        const int32_t* ext, double* z, double* ybuf);
__global__ void k_fwd_gather(const GatherDesc* gd, const int32_t* dofs, const double* ybuf, double* z);
__global__ void k_apply_up(const ApplyDesc* ad, const double* pool, const double* Tp, const int32_t* dofs,
                           double* z, double* ybuf, double* ws, const int32_t* ext);
__global__ void k_apply_down(const ApplyDesc* ad, const double* pool, const double* Tp, const int32_t* dofs,
                             double* z, double* ws, const int32_t* ext);
__global__ void k_apply_big_up(const ApplyDesc* ad, int phase, int j, const double* pool, const double* li,
                               const double* Tp, const int32_t* dofs, const int32_t* extp, double* z, double* ybuf,
                               double* ws);
__global__ void k_apply_big_dn(const ApplyDesc* ad, int phase, int j, const double* pool, const double* li,
                               const double* Tp, const int32_t* dofs, const int32_t* extp, double* z, double* ws);
__global__ void k_apply_trsv_up(const ApplyDesc* ad, const double* pool, const double* lip, const double* Tp,
                                const int32_t* dofs, double* z, const int32_t* extp);
__global__ void k_apply_trsv_dn(const ApplyDesc* ad, const double* pool, const double* lip, const double* Tp,
                                const int32_t* dofs, double* z, const int32_t* extp);
template <bool UP>
__global__ void k_apply_band(const ApplyDesc* ad, const double* pool, const double* lip, const int32_t* dofs,
                             double* z);
__global__ void k_apply_gemv_up(const ApplyDesc* ad, const double* pool, const int32_t* dofs, double* z,
                                double* ybuf);
__global__ void k_apply_gemv_dn(const ApplyDesc* ad, const double* pool, const int32_t* dofs, double* z);
__global__ void k_apply_group_up(const GroupApplyDesc* gd, const int32_t* gdofs, const double* ybuf, double* z,
                                 const double* Lg, const double* lig, const double* Gp, const double* Tp,
                                 const double* skli, const int32_t* perm, int tkcap);
__global__ void k_apply_group_dn(const GroupApplyDesc* gd, const int32_t* gdofs, double* z, const double* Lg,
                                 const double* lig, const double* Gp, const double* Tp, const double* skli,
                                 const int32_t* perm, int tkcap);
__global__ void k_sep_gather(const GatherDesc* gd, const int32_t* dofs, const double* ybuf, double* z);
__global__ void k_spmv_dot(int64_t N, const int32_t* rp, const int32_t* ci, const double* v, const double* p,
                           double* q, double* part);
__global__ void k_dot(int64_t N, const double* x, const double* y, double* part);
__global__ void k_finalize(const double* part, int nparts, int mode, double* sc, double* host_out);
__global__ void k_axpy2(int64_t N, const double* sc, const double* p, const double* q, double* u, double* r,
                        double* part, const double* zold, double* part2);
__global__ void k_update_p(int64_t N, const double* sc, const double* z, double* p);
__global__ void k_copy(int64_t N, const double* x, double* y);
__global__ void k_fill(int64_t N, double v, double* y);
__global__ void k_axpby(int64_t N, double a, const double* x, double b, double* y);
__global__ void k_bspmv_dot(const BatchSeg* seg, const int32_t* blk, const double* p, double* q, double* part);
__global__ void k_bdot(const BatchSeg* seg, const int32_t* blk, const double* x, const double* y, double* part);
__global__ void k_bfinalize(const BatchSeg* seg, const double* part, int mode, double* sc, const int32_t* active);
__global__ void k_baxpy2(const BatchSeg* seg, const int32_t* blk, const double* sc, const double* p, const double* q,
                         double* u, double* r, double* part, const double* zold, double* part2);
__global__ void k_bupdate_p(const BatchSeg* seg, const int32_t* blk, const double* sc, const double* z, double* p);
__global__ void k_set_u64(unsigned long long* p, unsigned long long v);

constexpr int kMaxSkelSegs = 64;     // row segments of one skeletonized group (2 x 26 in 3D)
constexpr int kMaxCellGroups = 32;   // boundary groups of one cell (26 in 3D)
constexpr int kSyrkBlock = 64;               // Schur update: rows and columns per workgroup
constexpr int kSplitApplyMaxI = 272;        // split apply: one row / column per thread and panel
constexpr int kApplyDiagDoubles = 32 * 33;   // LDS diagonal block of the apply kernels
constexpr int kApplyExtDoubles = 256;         // LDS panel extents (up to 512 ints, n_I <= 8192)
constexpr int kPotrfMaxTiles = 1024;          // frontal order up to 16384
constexpr int kPotrfSmemFixed = 2 * 16 * 17 + kPotrfMaxTiles / 2;   // doubles before the panel

}  // namespace rhif
