/*
 * shape.h -- C ABI of the particle shape descriptors on MI355X (gfx950): the
 * sphericity, nominal diameter, surface-equivalent-sphere diameter and Corey
 * shape factor of a metaball body (arXiv 2209.10411, sec. 4), the parameters
 * the paper steps in its drafting-kissing-tumbling study.
 *
 * Definitions (sec. 4): d_n = (6 V / pi)^(1/3); Phi = pi d_n^2 / S; d_s =
 * sqrt(4 A_p / pi) with A_p the projected area; CSF = d_S / sqrt(d_I d_L)
 * with d_S <= d_I <= d_L the body's dimensions along its principal axes (the
 * paper's CSF numerator, printed as d_s, is read as the shortest dimension,
 * Corey's definition), A_p the projection onto the plane of the two longer
 * axes.
 *
 * Computation on a grid of cell size h over the box [min p - sqrt(sum k) - h,
 * max p + sqrt(sum k) + h] (n_a = ceil(extent / h) + 1 points per axis):
 *   V      h^3 times the cells whose centre has C >= 1 (C = sum k / |x - p|^2,
 *          sec. 2.1, Eq. metaballM, exact quotients in control-point order);
 *   S      area of the C = 1 surface by marching tetrahedra (six tetrahedra per
 *          cube along its main diagonal, linear interpolation on the edges);
 *   axes   eigenvectors of the second moments of the inside cell centres
 *          about their centroid, each signed so that its component of
 *          largest magnitude is positive, ordered by the extent along them;
 *   dims   max - min of the inside centres projected on each axis, plus h;
 *   A_p    h^2 times the columns, on the grid -half + h i (half = dim / 2 +
 *          2 h, i < ceil(2 half / h) + 1) in the plane of the two longer axes
 *          about the centroid, with at least one sample along the shortest
 *          axis (same grid) where C >= 1.
 * One thread per grid cell (or column), block sums in FP64 to per-block slots
 * in the workspace, added on the host in block order; the 3x3 eigenproblem is
 * solved on the host (Jacobi rotations).
 *
 * Memory: cp, k are host arrays (copied); work is caller-owned device memory
 * of mb_shape_work_bytes bytes.  Synchronises.  Errors: LBM_E_INVALID (NULL
 * pointer, n outside 1..64, k <= 0, h <= 0, a grid beyond 2^31 cells),
 * LBM_E_NOMEM (workspace too small), LBM_E_HIP.
 */
#ifndef SHAPE_H
#define SHAPE_H

#include <stddef.h>
#include <stdint.h>

#include "midelbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double V, S, A_p;      /* volume, surface area, projected area          */
    double dims[3];        /* d_S, d_I, d_L                                 */
    double axes[9];        /* principal axes, row a = axis of dims[a]       */
    double centroid[3];    /* of the inside cell centres                    */
    double d_n, d_s, Phi, CSF;
    int64_t cells_inside;  /* V / h^3                                       */
    int64_t columns_hit;   /* A_p / h^2                                     */
} mb_shape;

size_t mb_shape_work_bytes(const double *cp, const double *k, int32_t n, double h);
lbm_status mb_shape_descriptors(const double *cp, const double *k, int32_t n, double h, void *work,
                                size_t work_bytes, void *hip_stream, mb_shape *out);

#ifdef __cplusplus
}
#endif
#endif /* SHAPE_H */
