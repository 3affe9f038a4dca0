/*
 * rhif_plan.h -- host-only diagnostic entry point of librhif: the level planner of the
 * factorization run without any device work, with the interpolative-decomposition
 * choices supplied by the caller. It lets the integer side of the library (the grouping
 * of unknowns into cells, edges, faces and corners of Sec. 3.1 / 3.2 of arXiv 1808.01364,
 * the frontal layouts and every gather table) be checked on a machine without a GPU.
 */
#ifndef RHIF_PLAN_H
#define RHIF_PLAN_H

#include "rhif.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Called once per skeletonized edge/face of a level: the group's smallest unknown and its
 * size n; must write the kept rank k (0..n) and the pivot order perm[0..n) (a permutation
 * of 0..n-1, positions into the group's ascending unknowns). Return 0 to continue. */
typedef int32_t (*rhif_id_choice_fn)(void *ctx, int32_t level, int32_t first_dof, int32_t n,
                                     int32_t *k, int32_t *perm);

/* Called for every cell with interior unknowns: its nI interior unknowns followed by its nB
 * boundary unknowns (linear indices; interior ascending, boundary by group). level == L is
 * the root. */
typedef void (*rhif_cell_fn)(void *ctx, int32_t level, int32_t cell, int32_t nI, int32_t nB,
                             const int32_t *dofs);

/* Run the planner for grid g and leaf m. Every table is bounds-checked against the buffer
 * sizes the factorization would allocate; a violation returns RHIF_EINVAL with a message.
 *  root_size [host] receives |S_L|. Errors: EINVAL (grid, leaf, a bad choice or a failed
 *  check). */
rhif_status rhif_plan_dry_run(const rhif_grid *g, int32_t leaf, rhif_id_choice_fn choose,
                              void *choose_ctx, rhif_cell_fn cell, void *cell_ctx,
                              int64_t *root_size);

#ifdef __cplusplus
}
#endif

#endif /* RHIF_PLAN_H */
