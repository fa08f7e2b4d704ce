/*
 * Plane-fitting oracle: plain, slow, FP64 brute force on the CPU.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call
 * this library; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the HIP library.
 *
 * For every output pixel (x0, y0) and odd window size k the oracle gathers
 * the k*k depth samples of the window centred there, back-projects each one
 * with the pinhole model (Eq. 1), and fits a plane n.P + d = 0 by brute force:
 *
 *  - PFO_IMPLICIT: the RGBD implicit fit (Sec. II-A).  Every row of the
 *    algebraic fit is divided by Z (Eq. 12), so it minimises
 *    sum_i ((n.P_i + d)/Z_i)^2 subject to |n| = 1.  Written as a weighted
 *    total-least-squares problem with weights 1/Z_i^2: two-pass weighted
 *    centroid and covariance, cyclic Jacobi eigen-decomposition, normal =
 *    eigenvector of the smallest eigenvalue.
 *  - PFO_IMPLICIT_SCATTER: the same fit taken literally from the 4x4 scatter
 *    matrix of the monomials [tan(theta_x), tan(theta_y), 1, 1/Z] (Eq. 14),
 *    with d eliminated in closed form (Schur complement) before the eigen
 *    solve.  A second, independent route used to cross-check the first.
 *  - PFO_EXPLICIT: the RGBD explicit fit (Sec. II-B, Eq. 15): least squares
 *    of 1/Z on (tan(theta_x), tan(theta_y), 1), solved on centred regressors.
 *  - PFO_EXPLICIT_NORMALEQ: Eq. 15 solved literally as (M^T M)^-1 M^T b
 *    (Eq. 16) by Gaussian elimination; cross-check of PFO_EXPLICIT.
 *  - PFO_IMPLICIT_LITERAL: the implicit RGBD fit with the constraint as
 *    Sec. II-A states it, |(a, b, c, d)| = 1: smallest eigenvector of the 4x4
 *    scatter of Eq. 14 (Jacobi), scaled to a unit normal; kappa is
 *    l4 / (l2 - l1) of that 4x4.  Depends on the depth unit.
 *  - PFO_XYZ_IMPLICIT / PFO_XYZ_EXPLICIT: the standard fits of Eq. 3 and
 *    Eq. 7 on the back-projected points (unweighted); cross-checks only.
 *
 * Conventions shared by every mode:
 *  - pixel (x, y) is valid iff mask is NULL or mask[y*W+x] != 0, and the
 *    depth is finite and > 0.  A window is valid iff all k*k pixels lie in
 *    the image and are valid; invalid windows get NaN outputs and status 1.
 *  - the plane is oriented so that d >= 0 (the normal faces the camera).
 *  - the residual is the RMS over the window of (n.P_i + d)/Z_i.
 *  - kappa = l3 / (l2 - l1) for the eigenvalues l1 <= l2 <= l3 of the
 *    implicit problem (NaN for the explicit modes).
 *  - all images are row-major with a pitch of W elements; normals are
 *    channel-planar [3][H][W].
 */
#ifndef PFO_ORACLE_H
#define PFO_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PFO_IMPLICIT = 0,
  PFO_EXPLICIT = 1,
  PFO_IMPLICIT_SCATTER = 2,
  PFO_EXPLICIT_NORMALEQ = 3,
  PFO_XYZ_IMPLICIT = 4,
  PFO_XYZ_EXPLICIT = 5,
  PFO_IMPLICIT_LITERAL = 6
};

/* Returns 0 on success, -1 on a bad argument. threads <= 0 means all cores. */
int pfo_fit_planes(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                   double fx, double fy, double cx, double cy, int32_t k, int32_t mode,
                   int32_t threads, double* normals, double* offsets, double* residuals,
                   double* kappa, uint8_t* status);

/* Same fits from an explicit list of window centres (xs[i], ys[i]), i < count;
 * outputs are [count] (normals [3][count]). */
int pfo_fit_points(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                   double fx, double fy, double cx, double cy, int32_t k, int32_t mode,
                   const int64_t* xs, const int64_t* ys, int64_t count, int32_t threads,
                   double* normals, double* offsets, double* residuals, double* kappa,
                   uint8_t* status);

/* Partial windows: as pfo_fit_planes / pfo_fit_points, but a window is fitted
 * from its valid pixels alone (those inside the image with valid depth) iff
 * there are at least min_valid >= 3 of them and they do not all lie on one
 * line of the pixel grid; the residual is the RMS over those pixels.
 * min_valid >= k*k is the full-window rule.  Returns -1 for min_valid < 3. */
int pfo_fit_planes_partial(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                           double fx, double fy, double cx, double cy, int32_t k, int32_t mode,
                           int32_t min_valid, int32_t threads, double* normals,
                           double* offsets, double* residuals, double* kappa, uint8_t* status);
int pfo_fit_points_partial(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                           double fx, double fy, double cx, double cy, int32_t k, int32_t mode,
                           int32_t min_valid, const int64_t* xs, const int64_t* ys,
                           int64_t count, int32_t threads, double* normals, double* offsets,
                           double* residuals, double* kappa, uint8_t* status);

/* Fits to arbitrary rectangles, the use of integral images the paper makes
 * (Sec. II-C): rects is int32 [count][4] = (x0, y0, w, h), covering columns
 * x0 .. x0+w-1 and rows y0 .. y0+h-1.  A rectangle is valid iff w, h >= 2, it
 * lies in the image and all its pixels are valid; the fit, orientation,
 * residual and kappa follow the window fits.  Outputs are [count]
 * (normals [3][count]). */
int pfo_fit_rects(const double* depth, int64_t H, int64_t W, const uint8_t* mask, double fx,
                  double fy, double cx, double cy, const int32_t* rects, int64_t count,
                  int32_t mode, int32_t threads, double* normals, double* offsets,
                  double* residuals, double* kappa, uint8_t* status);

/* Brute-force window sums of the camera-only monomial products over the
 * window centred at (x0, y0): [sum u^2, sum u v, sum u, sum v^2, sum v, N]
 * with u = (x - cx)/fx, v = (y - cy)/fy (Eq. 10).  No image bounds apply. */
void pfo_camera_moments(double fx, double fy, double cx, double cy, int32_t k,
                        int64_t x0, int64_t y0, double out[6]);

/* Brute-force window sums of the depth-dependent monomials over every window:
 * out[c][H][W] for c = [sum w, sum u w, sum v w, sum w^2, count] with w = 1/Z
 * over the valid pixels of the window (pixels outside the image count as
 * invalid).  Every window gets its sums, valid or not. */
void pfo_window_sums(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                     double fx, double fy, double cx, double cy, int32_t k, double* out);

/* FP64 integral images of the same five integrands (Sec. II-C):
 * out[c][(H+1)][(W+1)], with a zero first row and column. */
void pfo_integral_images(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                         double fx, double fy, double cx, double cy, double* out);

/* The paper's integral-image method in FP64, taken as written: per-frame
 * integral images of the four depth-dependent entries and the count, camera
 * integral images of the five camera-only entries, four-corner box sums,
 * then the 4x4 scatter (implicit, Eq. 14, d eliminated) or the 3x3 normal
 * equations (explicit, Eq. 16).  mode is PFO_IMPLICIT or PFO_EXPLICIT. */
int pfo_fit_planes_integral(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                            double fx, double fy, double cx, double cy, int32_t k,
                            int32_t mode, double* normals, double* offsets,
                            double* residuals, uint8_t* status);

/* Cyclic Jacobi eigen-decomposition of a symmetric 3x3 (row-major a[9]);
 * eigenvalues ascending in evals, eigenvectors as columns of evecs[9]. */
void pfo_jacobi3(const double a[9], double evals[3], double evecs[9]);

#ifdef __cplusplus
}
#endif
#endif
