/*
 * mifit.h -- C ABI of the Metaball-Imaging fit on MI355X (gfx950): the
 * genetic algorithm and the gradient search that turn a particle's point
 * hull into a metaball model (arXiv 2209.10411, sec. 2.2).
 *
 * Conventions
 *   - A metaball model is n control points, each (k, x, y, z), FP64, stored
 *     [n][4]; its value at a point h is f(h) = sum_j k_j / |h - p_j|^2
 *     (sec. 2.1, Eq. metaballM).  A population is [P][n][4].
 *   - A point hull is [m][3] FP64, centred at the origin (the paper's
 *     transformation of coordinates); its convex hull is given as half-spaces
 *     [n_pl][4] (n . p + d <= 0 inside), which decides "inside the hull" as
 *     the paper's linear program does.
 *   - Every pointer argument is device memory owned by the caller unless
 *     stated; every call is enqueued on hip_stream (a hipStream_t, NULL = the
 *     default stream).  Calls that run several launches synchronise where
 *     stated.  Random numbers are inputs.
 *   - Limits: 1 <= n <= MI_MAXCP, m >= 1; the GA needs 2 <= N_I and
 *     3 N_I <= 4096; the gradient search takes hulls of up to MI_GS_MAXPTS
 *     points (the slope at every point stays in LDS).
 *   - Errors: LBM_E_INVALID for a NULL pointer or a size out of range,
 *     LBM_E_NOMEM for a workspace smaller than the *_work_bytes figure,
 *     LBM_E_HIP for a failed launch.  lbm_last_error() is not set.
 */
#ifndef MIFIT_H
#define MIFIT_H

#include <stddef.h>
#include <stdint.h>

#include "midelbm.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { MI_MAXCP = 64, MI_GS_MAXPTS = 6144 };

/* Workspace bytes for mi_fitness over P individuals and m hull points (zero
 * when m fits one block's chunk of 2048 points). */
size_t mi_fitness_work_bytes(int64_t m, int32_t P);

/* GA evaluation (sec. 2.2, Evaluation): F[p] = sum_i (f(H_i; pop_p) - 1)^2
 * for each of the P individuals pop [P][n][4] over the hull H [m][3]; F [P]
 * FP64.  A block takes one individual and a chunk of up to 2048 hull points
 * (control points in LDS, one hull point per lane, fixed-order block sums);
 * with several chunks the per-chunk sums go to the workspace (work,
 * work_bytes >= mi_fitness_work_bytes) and a second launch adds them in chunk
 * order.  Asynchronous. */
lbm_status mi_fitness(const double *hull, int64_t m, const double *pop, int32_t P, int32_t n, double *F,
                      void *work, size_t work_bytes, void *hip_stream);

/* Workspace bytes of mi_ga. */
size_t mi_ga_work_bytes(int64_t m, int32_t N_I, int32_t n);

/* Alg. GA (sec. 2.2): from the initial population pop [N_I][n][4] (control
 * points inside the hull, weights > 0), E generations of
 *   mutation   one mutant per individual: gene g of individual a changes
 *              where U[e][a][g] < C_m by Z[e][a][g] * sigma (sigma_k for
 *              the weight, sigma_x for the coordinates); a weight that falls
 *              below zero is set to zero;
 *   crossover  individuals PERM[e][2j] and PERM[e][2j+1] exchange their
 *              control points from c = round(C_c n) on (two children; an odd
 *              last individual is copied);
 *   evaluation F of the mutants and children (mi_fitness);
 *   selection  the N_I individuals of smallest F among parents, mutants and
 *              children (pool in that order; ties to the lower pool index).
 * U, Z: [E][N_I][n][4] FP64; PERM: [E][N_I] int32, each a permutation of
 * 0..N_I-1 (not checked).  On return pop holds the final population, fittest
 * first, and F [N_I] its fitness; pop[0] is the model M^ga.  work:
 * mi_ga_work_bytes bytes.  Synchronises. */
lbm_status mi_ga(const double *hull, int64_t m, int32_t N_I, int32_t n, int32_t E, double C_m, double C_c,
                 double sigma_x, double sigma_k, const double *U, const double *Z, const int32_t *PERM,
                 double *pop, double *F, void *work, size_t work_bytes, void *hip_stream);

/* Alg. GS (sec. 2.2) for B models at once, one workgroup each: E
 * full-batch gradient-descent steps M <- M - eta dL/dM of the piecewise
 * objective of Eq. GSloss summed over the model's hull points (for f < 1 the
 * term (f - 1)^2 + 1/f - 1 with 1/f taken as 1/max(f, 1e-12); for
 * 1 <= f < 2, |f - 1| with slope 1; for f >= 2, (f - 1)^2), then the anomaly
 * cleaning (weight zero for negative weights and for control points outside
 * the convex hull), then E more steps.  Model b fits the hull points
 * hulls[hull_off[b] .. hull_off[b+1]) ([.][3], 1 to MI_GS_MAXPTS of them)
 * with the half-spaces planes[plane_off[b] .. plane_off[b+1]) ([.][4]);
 * hull_off, plane_off: [B + 1] int64 device arrays, read back to the host to
 * check the sizes (the call synchronises for that, then runs
 * asynchronously).  M [B][n][4] is the start (the GA's result) on entry and
 * the fit on return; loss [B][3] receives L before, after the first descent
 * and at the end.  Per step the slope of the objective at every hull point
 * is formed once (one lane per point) and the gradient summed by lanes over
 * (control point, chunk of points), chunks added in a fixed order. */
lbm_status mi_gs(const double *hulls, const int64_t *hull_off, const double *planes, const int64_t *plane_off,
                 int32_t B, int32_t n, int32_t E, double eta, double *M, double *loss, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mi_fitness
 * with its per-chunk sums in a static device array of the library (1 MiB,
 * one copy per GPU, held until the process ends) instead of a workspace;
 * it allocates nothing.  P * ceil(m / 2048) must not exceed 131072, else
 * LBM_E_INVALID (nothing launched).  Every call on one GPU uses the same
 * array: calls that overlap on one GPU (several streams or host threads)
 * race, and the array keeps the last call's sums (every slot read is written
 * first by the same call, so nothing needs clearing).  Asynchronous. */
lbm_status mi_fitness_noalloc(const double *hull, int64_t m, const double *pop, int32_t P, int32_t n, double *F,
                              void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* MIFIT_H */
