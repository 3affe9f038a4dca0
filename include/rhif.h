/*
 * rhif.h -- C ABI of the MI355X (gfx950) recursively preconditioned hierarchical
 * interpolative factorization (RHIF; "PHIF" in Feliu-Faba, Ho, Ying, "Recursively
 * Preconditioned Hierarchical Interpolative Factorization for Elliptic Partial
 * Differential Equations", arXiv 1808.01364).
 *
 * The library factors the SPD finite-difference matrix A of
 *     -div(a grad u) + b u = f   on (0,1)^d, d = 2 or 3, zero Dirichlet data
 * (the problem of Sec. 1, eqs. (1.1)-(1.2), discretized as in Sec. 3.1 / 3.2) into the
 * generalized Cholesky form F = G G^T of eq. (3.3), and applies F^-1 (eq. (3.2)) as
 * the preconditioner of a CG solve (Sec. 4).
 *
 * Conventions shared by every entry point
 *  - Grid: n interior points per axis, N = n^d unknowns at x in {1..n}^d, h = 1/(n+1).
 *    Unknown (x_1..x_d) has linear index sum_k (x_k-1) n^(k-1)  (x_1 fastest).
 *  - Coefficient a: one value per grid cell, (n+1)^d values, cell (c_1..c_d) with
 *    0 <= c_k <= n at linear index sum_k c_k (n+1)^(k-1). The coefficient of a grid edge
 *    is the mean of the 2^(d-1) cells containing it.
 *  - Pointers marked [device] are device (HBM) pointers owned by the caller; [host] are
 *    host pointers. Device work is enqueued on the given stream (0 = the null stream).
 *  - Every call returns an rhif_status; nothing throws across the ABI. On failure,
 *    rhif_last_error() returns a thread-local message naming the failing step.
 *  - One call in flight per factor handle at a time.
 */
#ifndef RHIF_H
#define RHIF_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RHIF_OK = 0,
    RHIF_EINVAL = 1,    /* invalid argument or matrix structure                          */
    RHIF_ENOTSPD = 2,   /* a Cholesky pivot was <= 0 or not finite (loss of SPD-ness)      */
    RHIF_ENOMEM = 3,    /* device or host allocation failed                              */
    RHIF_EDEVICE = 4,   /* a HIP runtime call failed                                     */
    RHIF_ENOCONV = 5    /* PCG reached maxit before the residual test passed            */
} rhif_status;

/* Regular grid: dim in {2,3}; n[0] = n[1] (= n[2] in 3D) interior points per axis. */
typedef struct {
    int32_t dim;
    int32_t n[3];
} rhif_grid;

/* Factorization options.
 *  leaf      m >= 2: level-l cells span 2^l m grid steps; levels run while 2^l m <= n
 *            (Sec. 3.1: n = 2^L m); what remains after the last level is the root.
 *  eps       relative precision of the interpolative decomposition (Sec. 2.2): the rank
 *            is the number of leading column-pivoted QR steps with |R_jj| > eps |R_11|.
 *            eps = 0 keeps every column (exact nested dissection).
 *  precond   1 = block-Jacobi preconditioning of every separator group before each
 *            skeletonization (the paper's PHIF, Sec. 3.1 step 2); 0 = plain HIF.
 *  precision 0 = FP64 throughout.
 *            1 = FP32-mixed: the interpolative decompositions (the matrix M = A[R_g, g], its
 *            column-pivoted QR and T = R11^-1 R12) in FP32; everything else FP64.
 *            2 = as 1, and the Schur products S = A_BB - W^T W of the cell eliminations
 *            (level 0 and the final product of the upper levels) on the FP32 matrix cores
 *            with FP32 accumulation.
 *            In both, every Cholesky factor (cell interiors, block Jacobi, skeleton
 *            eliminations, root), the stored factor and the apply stay FP64, and
 *            rhif_pcg_solve on such a factor uses the flexible (Polak-Ribiere) CG update
 *            with FP64 residuals and inner products, so that CG refines the solution to the
 *            requested tolerance.
 *  flags     bit 0: record per-phase device times (adds one sync per phase). */
typedef struct {
    int32_t leaf;
    double  eps;
    int32_t precond;
    int32_t precision;
    int32_t flags;
} rhif_opts;

#define RHIF_FLAG_PHASE_TIMES 1
#define RHIF_FLAG_KERNEL_TIMES 2   /* bracket kernel launches with HIP events on the
                                      caller's stream; accumulated in rhif_stats_t        */
#define RHIF_KERNEL_MASK_SHIFT 8   /* flags bits 8..23: if any is set, time only the kernel
                                      classes whose bit (1 << class) is set               */
/* flags bit 2 (value 4) is reserved: rhif_factor rejects it with EINVAL */
#define RHIF_FLAG_SOLVE_GRAPHS 8   /* run the factor applies and PCG iterations of the handle
                                      as HIP graphs, captured at the first rhif_apply /
                                      rhif_pcg_solve call (pays off when the handle serves
                                      many solves); ignored while the solve kernels are
                                      timed with RHIF_FLAG_KERNEL_TIMES                    */
#define RHIF_FLAG_GLOBAL_STAGING 16 /* keep the operands of the block-Jacobi and ID kernels
                                       in global memory even where they fit in LDS: the path
                                       that groups too large for LDS take (same results;
                                       slower); for testing that path on small problems  */
#define RHIF_FLAG_SKEL_MULTI 32     /* take the interpolative decompositions of every level with
                                       the multi-workgroup form (the form for groups whose M is
                                       too large for one workgroup: one launch per pivot step
                                       over row blocks of M); for testing that form on small
                                       problems                                          */
#define RHIF_MAX_LEVELS 32

/* Kernel classes of rhif_stats_t.kernel_* */
enum {
    RHIF_K_FRONT_CSR = 0,     /* level-0 frontal assembly from the CSR matrix            */
    RHIF_K_FRONT_EXTEND = 1,  /* frontal assembly from the children (levels >= 1)        */
    RHIF_K_ELIM_LEAF = 2,     /* cell elimination at level 0                             */
    RHIF_K_ELIM_UPPER = 3,    /* cell elimination at levels >= 1                         */
    RHIF_K_ROOT = 4,          /* root Cholesky                                           */
    RHIF_K_PRECOND_CHOL = 5,  /* block-Jacobi: gather + Cholesky of every group          */
    RHIF_K_PRECOND_SCALE = 6, /* block-Jacobi: two-sided scaling of every cell           */
    RHIF_K_SKELETONIZE = 7,   /* ID + skeleton elimination of every edge / face          */
    RHIF_K_APPLY_UP = 8,      /* apply: up-sweep blocks                                  */
    RHIF_K_APPLY_DOWN = 9,    /* apply: down-sweep blocks                                */
    RHIF_K_APPLY_GATHER = 10, /* apply: gather of the cells' boundary contributions      */
    RHIF_K_SPMV = 11,         /* CG: sparse matrix-vector product (+ p.q)                */
    RHIF_K_VECTOR = 12,       /* CG: dots, axpys, copies                                 */
    RHIF_NUM_KCLASS = 16
};

/* Host-side summary of a factorization. Per-level arrays are indexed by level l = 0..L-1;
 * entry [levels] describes the root. */
typedef struct {
    int32_t levels;                          /* L, the number of levels before the root  */
    int32_t root_size;                       /* |S_L|                                    */
    int64_t factor_bytes;                    /* device bytes held by the factor          */
    int64_t n_active[RHIF_MAX_LEVELS + 1];   /* |S_l| at the start of level l            */
    int32_t n_cells[RHIF_MAX_LEVELS + 1];    /* cell frontal matrices at level l         */
    int32_t max_front[RHIF_MAX_LEVELS + 1];  /* largest frontal order at level l         */
    int32_t n_groups[RHIF_MAX_LEVELS];       /* separator groups preconditioned          */
    int32_t n_skel[RHIF_MAX_LEVELS];         /* edges (2D) / faces (3D) skeletonized     */
    int64_t sum_skel_n[RHIF_MAX_LEVELS];     /* total DOFs in those groups               */
    int64_t sum_rank[RHIF_MAX_LEVELS];       /* total skeleton DOFs kept                 */
    int32_t max_rank[RHIF_MAX_LEVELS];
    double  flops[RHIF_MAX_LEVELS + 1];      /* algorithmic flops of the level's kernels */
    double  t_total_ms;                      /* host wall time of rhif_factor            */
    double  t_phase_ms[8];                   /* with RHIF_FLAG_PHASE_TIMES: assemble,
                                                eliminate, precondition, ID + skeleton
                                                elimination, -, plan+upload, root, -     */
    /* with RHIF_FLAG_KERNEL_TIMES, accumulated over every call on the handle: */
    double  kernel_ms[RHIF_NUM_KCLASS];      /* device time (HIP events)                 */
    int64_t kernel_launches[RHIF_NUM_KCLASS];
    double  kernel_flops[RHIF_NUM_KCLASS];   /* algorithmic flops of those launches      */
    double  kernel_bytes[RHIF_NUM_KCLASS];   /* algorithmic HBM bytes of those launches  */
    int32_t sublevels;                       /* always 0 (reserved)                      */
} rhif_stats_t;

typedef struct rhif_factor_s *rhif_factor_t;

/* Number of nonzeros of the 5-/7-point matrix on grid g: N + 2 d n^(d-1) (n-1).
 * [host] nnz. No device work. Errors: EINVAL for a malformed grid. */
rhif_status rhif_fd_nnz(const rhif_grid *g, int64_t *nnz);

/* Assemble A = h^-2 K(a) + diag(b) in CSR form (eq. (1.1)-(1.2); Sec. 3.1 five-point and
 * Sec. 3.2 seven-point stencils). Columns of every row are ascending.
 *  a_cells [device] (n+1)^d cell coefficients (must be > 0 for an SPD matrix)
 *  b       [device] N reaction values, or NULL for b = 0
 *  row_ptr [device] N+1 int32 (output), col [device] nnz int32 (output),
 *  val     [device] nnz doubles (output); nnz from rhif_fd_nnz.
 * Errors: EINVAL (grid), EDEVICE (launch). */
rhif_status rhif_assemble_fd(const rhif_grid *g, const double *a_cells, const double *b,
                             int32_t *row_ptr, int32_t *col, double *val, hipStream_t s);

/* Factor A ~= F = G G^T level by level (Sec. 3.1 / 3.2): at each level l = 0..L-1 every
 * cell interior is eliminated (Sec. 2.1), every separator group is block-Jacobi
 * preconditioned (Sec. 2.3, when precond = 1), and every edge (2D) / face (3D) is
 * skeletonized with a column-pivoted-QR interpolative decomposition at precision eps
 * (Sec. 2.2, all IDs of a level taken from the same matrix); the rest is factored
 * densely (root, eq. (3.3)).
 *  row_ptr, col, val [device] the CSR of A as produced by rhif_assemble_fd (entries may
 *            only couple grid neighbours); the handle keeps its own copy, so the caller
 *            may free these after the call returns.
 *  out       [host] receives the new handle; NULL on any error (nothing leaks).
 * The call synchronizes the stream once per level (to read the ID ranks back).
 * Errors: EINVAL (grid/options/structure), ENOTSPD (a pivot <= 0 or not finite; the
 * message names level, step E/C/K/root and block), ENOMEM, EDEVICE. */
rhif_status rhif_factor(const rhif_grid *g, const rhif_opts *o, const int32_t *row_ptr,
                        const int32_t *col, const double *val, hipStream_t s,
                        rhif_factor_t *out);

/* Factor `count` independent problems with the same options in one call (the batched form;
 * the cells and groups of different problems are as independent as those of one problem,
 * Sec. 2.1, and their IDs are simultaneous like those of one level, Sec. 2.2). The problems
 * advance level by level together: every elimination, block-Jacobi and skeletonization
 * kernel of a level is ONE launch over the blocks of all problems (only the frontal
 * assembly is launched per problem), and one read-back per level brings the ranks of every
 * problem to the host. Each problem is factored exactly as rhif_factor factors it alone
 * (same choices, same arithmetic order: the results are bitwise those of rhif_factor).
 *  grids   [host] count grids, all with the same dim (the sides may differ)
 *  o       [host] options shared by all problems; flags must not ask for kernel or phase
 *          times when count > 1 (EINVAL)
 *  row_ptr, col, val [host] arrays of count device pointers: problem i's CSR as for
 *          rhif_factor (copied; the caller may free them after the call returns)
 *  out     [host] count handles, used and destroyed like those of rhif_factor and from any
 *          thread; the device memory of the handles of one call is one pool, returned to the
 *          library when the last of them is destroyed. On any error every out[i] is NULL.
 * Synchronizes the stream once per level. Errors: as rhif_factor (an ENOTSPD message numbers
 * blocks over the whole batch). */
rhif_status rhif_factor_batch(int32_t count, const rhif_grid *grids, const rhif_opts *o,
                              const int32_t *const *row_ptr, const int32_t *const *col,
                              const double *const *val, hipStream_t s, rhif_factor_t *out);

/* z = F^-1 r for nrhs right-hand sides stored one after another (column-major N x nrhs):
 * the up-sweep R_l^T = K_l^T C_l^T E_l^T for l = 0..L-1, the root solve, and the
 * down-sweep R_l = E_l C_l K_l for l = L-1..0 (eq. (3.2)).
 *  r [device] input (not modified), z [device] output; r == z is allowed.
 * Stream-ordered, never synchronizes. Errors: EINVAL, EDEVICE. */
rhif_status rhif_apply(rhif_factor_t f, const double *r, double *z, int32_t nrhs,
                       hipStream_t s);

/* Solve A u = rhs by CG preconditioned with F^-1 from u_0 = 0 (Sec. 4), stopping when the
 * recursively updated residual satisfies ||r_k|| <= rtol ||rhs||.
 *  rhs [device] N doubles, u [device] N doubles (output)
 *  iters  [host] number of products A p taken; relres [host] final ||r_k||/||rhs||.
 * Reads one scalar back per iteration. Errors: EINVAL, EDEVICE, ENOCONV (u then holds
 * the last iterate and iters/relres are set). */
rhif_status rhif_pcg_solve(rhif_factor_t f, const double *rhs, double *u, double rtol,
                           int32_t maxit, int32_t *iters, double *relres, hipStream_t s);

/* z_i = F_i^-1 r_i for every problem i of one rhif_factor_batch call (eq. (3.2)), all at
 * once: each level's up- and down-sweep kernels run as one launch over the blocks of all
 * problems. Every block is computed as in its own problem's rhif_apply (the results are
 * bitwise those of rhif_apply).
 *  f     [host] the count (>= 2) handles of ONE rhif_factor_batch call, all of them, in the
 *        call's order (EINVAL otherwise, or once one of them has been destroyed)
 *  r, z  [host] arrays of count device pointers to N_i doubles each (inputs not modified)
 * The first joint call on a batch builds its merged tables (one upload). Calls on one batch
 * are serialized. Stream-ordered, never synchronizes. Errors: EINVAL, EDEVICE. */
rhif_status rhif_apply_batch(int32_t count, const rhif_factor_t *f, const double *const *r,
                             double *const *z, hipStream_t s);

/* rhif_pcg_solve for every problem i of one rhif_factor_batch call at once: the CG vector
 * kernels and the applies each run as one launch over all problems, every problem with its
 * own scalars; a problem stops updating once its own residual test passes, and each takes the
 * iterations of its own rhif_pcg_solve (the same arithmetic: bitwise the same solution). One
 * read-back of every problem's residual norm per iteration.
 *  f              as for rhif_apply_batch
 *  rhs, u         [host] arrays of count device pointers (N_i doubles each; u is output)
 *  iters, relres  [host] arrays of count entries (output), as for rhif_pcg_solve
 * Errors: EINVAL, EDEVICE, ENOCONV (some problem missed rtol within maxit; every u_i, iters_i
 * and relres_i is still set). */
rhif_status rhif_pcg_solve_batch(int32_t count, const rhif_factor_t *f, const double *const *rhs,
                                 double *const *u, double rtol, int32_t maxit, int32_t *iters,
                                 double *relres, hipStream_t s);

/* One half of the factor apply: F^-1 = G^-T G^-1 with F = G G^T (eq. (3.3)).
 *  which = 0: z = G^-1 r (the up-sweep R_0^T .. R_{L-1}^T of eq. (3.2), then the forward
 *             solve with the root factor B_L, A_L = B_L B_L^T);
 *  which = 1: z = G^-T r (the backward solve with B_L^T, then the down-sweep).
 *  r, z [device] N doubles; r == z is allowed. Stream-ordered. Errors: EINVAL, EDEVICE. */
rhif_status rhif_apply_half(rhif_factor_t f, const double *r, double *z, int32_t which, hipStream_t s);

/* The solve error e_s = ||I - G^-1 A G^-T||_2 of the factorization (Sec. 4, the paper's
 * measure of preconditioner quality), by power iteration on the square of the symmetric
 * operator I - G^-1 A G^-T from the start vector v0: each iteration applies the operator
 * twice and normalizes; it stops when the estimate changes by at most rtol (relative) or
 * after maxit iterations.
 *  v0 [device] N doubles (the caller's random start vector; not modified)
 *  es [host] the estimate; iters [host, may be NULL] iterations taken.
 * Synchronizes the stream once per iteration. Errors: EINVAL (zero start, bad maxit/rtol),
 * EDEVICE. */
rhif_status rhif_estimate_es(rhif_factor_t f, const double *v0, int32_t maxit, double rtol, double *es,
                             int32_t *iters, hipStream_t s);

/* y = F x = G G^T x, the forward product of the factorization (eq. (3.3)): every step of
 * the two sweeps of eq. (3.2) undone in reverse order, with products by the stored factors
 * instead of solves. x, y [device] N doubles (x == y allowed). Stream-ordered. */
rhif_status rhif_apply_forward(rhif_factor_t f, const double *x, double *y, hipStream_t s);

/* The apply error e_a = ||A - F||_2 / ||A||_2 of the factorization (Sec. 4), both norms by
 * power iteration from the start vector v0, as for rhif_estimate_es.
 *  ea [host] the estimate; iters [host, may be NULL] the larger of the two iteration counts. */
rhif_status rhif_estimate_ea(rhif_factor_t f, const double *v0, int32_t maxit, double rtol, double *ea,
                             int32_t *iters, hipStream_t s);

/* Largest N that rhif_pcg_solve_noalloc accepts. */
#define RHIF_NOALLOC_MAX_N (1 << 20)

/* rhif_pcg_solve for callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid allocation calls): the same CG iteration (same kernels in the
 * same order, so the same iterates), with its workspace (the vectors r, z, p, q and the
 * reduction scalars, 4 N + 2064 doubles) in a device array of the library sized for
 * N <= RHIF_NOALLOC_MAX_N (32 MiB, held on every GPU the library runs on until the process
 * ends). The call makes no allocation (no hipMalloc / hipFree / pinned host memory / event
 * or graph creation); it reads each scalar back with a copy to the calling thread's host
 * memory and a synchronization of s, and records no kernel timings.
 *  rhs [device] N doubles, u [device] N doubles (output), as for rhif_pcg_solve.
 * Every call on one GPU uses the same workspace: calls that overlap on one GPU (several
 * host threads, or several streams) race and must be serialized by the caller. The handle
 * must belong to the current device.
 * Errors: EINVAL (NULL argument, N > RHIF_NOALLOC_MAX_N, another device), EDEVICE, ENOCONV. */
rhif_status rhif_pcg_solve_noalloc(rhif_factor_t f, const double *rhs, double *u, double rtol,
                                   int32_t maxit, int32_t *iters, double *relres, hipStream_t s);

/* Adjoint of the solve with respect to theta = log a (the adjoint-gradient extension of the
 * solver; the operator is eq. (1.1) with the Sec. 3.1 / 3.2 stencils): for every grid cell c,
 *   grad[c] = -a_c * lambda^T (dA/da_c) u
 *           = -a_c 2^(1-d) h^-2 sum over the cell's grid edges (x, x+e_k) of
 *             (lambda(x+e_k) - lambda(x)) (u(x+e_k) - u(x)),      values at ghosts = 0,
 * which is dL/dtheta_c for a loss L(u) of the solution of A u = f when A lambda = dL/du
 * (A is symmetric, so lambda comes from the same factorization). b does not depend on a.
 *  a_cells [device] (n+1)^d cell coefficients, x_1 fastest (as for rhif_assemble_fd)
 *  u, lam  [device] N values each (solution and adjoint solution)
 *  grad    [device] (n+1)^d outputs, caller-owned
 * Stream-ordered on s. Errors: EINVAL for a malformed grid or a NULL pointer. */
rhif_status rhif_grad_log_a(const rhif_grid *g, const double *a_cells, const double *u, const double *lam,
                            double *grad, hipStream_t s);

/* y = A x with the handle's copy of A (x, y [device] N doubles). */
rhif_status rhif_matvec(rhif_factor_t f, const double *x, double *y, hipStream_t s);

/* Fill [host] *out with the structure, sizes and timings of the factorization. */
rhif_status rhif_stats(rhif_factor_t f, rhif_stats_t *out);

/* Discrete choices of the interpolative decompositions at skeletonization level l, so
 * that a reference implementation can replay them (several pivot orders are valid when
 * column norms tie). With the host arrays NULL, only *ngroups and *total are written.
 *  ngroups [host] number of edges/faces skeletonized at level l
 *  total   [host] sum of their sizes
 *  first_dof [host, ngroups] smallest unknown (linear index) of each group
 *  size, rank [host, ngroups] group size n and kept rank k
 *  perm    [host, total] pivot order of each group, as positions 0..n-1 into the group's
 *          unknowns in ascending linear index, groups one after another. */
rhif_status rhif_skeletons(rhif_factor_t f, int32_t level, int32_t *ngroups, int64_t *total,
                           int32_t *first_dof, int32_t *size, int32_t *rank, int32_t *perm);

/* Release every resource of the handle (synchronizes its device work). NULL is a no-op. */
void rhif_destroy(rhif_factor_t f);

/* Thread-local description of the last error of this thread ("" if none). */
const char *rhif_last_error(void);

/* Library version string. */
const char *rhif_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RHIF_H */
