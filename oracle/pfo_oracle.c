/*
 * Plane-fitting oracle: plain FP64 brute force.  TEST INFRASTRUCTURE ONLY
 * (see pfo_oracle.h).  Every fit gathers its window's samples, back-projects
 * them with Eq. 1 and solves the small least-squares problem directly; there
 * is no blocking, no reuse between windows and no reordering beyond what the
 * definitions state.
 */
#include "pfo_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KMAX 255

/* ---------------------------------------------------------------------------
 * 3x3 symmetric eigen-decomposition: cyclic Jacobi with the symmetric Schur
 * rotation (Golub & Van Loan, Matrix Computations, Sec. 8.5).
 * ------------------------------------------------------------------------- */
static void matmul3(const double a[3][3], const double b[3][3], double c[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int t = 0; t < 3; ++t) s += a[i][t] * b[t][j];
      c[i][j] = s;
    }
}

void pfo_jacobi3(const double a_in[9], double evals[3], double evecs[9]) {
  double A[3][3], V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = 0.5 * (a_in[3 * i + j] + a_in[3 * j + i]);
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off == 0.0 || off <= 1e-36 * dia) break;
    static const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
    for (int r = 0; r < 3; ++r) {
      int p = P[r], q = Q[r];
      if (A[p][q] == 0.0) continue;
      double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
      double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
      double c = 1.0 / hypot(1.0, t), s = t * c;
      double J[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, Jt[3][3], T[3][3];
      J[p][p] = c; J[p][q] = s; J[q][p] = -s; J[q][q] = c;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Jt[i][j] = J[j][i];
      matmul3(Jt, A, T);
      matmul3(T, J, A);
      A[p][q] = A[q][p] = 0.0; /* annihilated by construction */
      matmul3(V, J, T);
      memcpy(V, T, sizeof(V));
    }
  }
  int order[3] = {0, 1, 2};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (A[order[j]][order[j]] < A[order[i]][order[i]]) {
        int t = order[i]; order[i] = order[j]; order[j] = t;
      }
  for (int i = 0; i < 3; ++i) {
    evals[i] = A[order[i]][order[i]];
    for (int r = 0; r < 3; ++r) evecs[3 * r + i] = V[r][order[i]];
  }
}

/* 4x4 symmetric eigen-decomposition by the same cyclic Jacobi method, applying
 * each rotation to rows and columns p, q directly; eigenvalues ascending,
 * eigenvectors in the columns of evecs (row-major 4x4). */
static void jacobi4(const double a_in[16], double evals[4], double evecs[16]) {
  double A[4][4], V[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      A[i][j] = 0.5 * (a_in[4 * i + j] + a_in[4 * j + i]);
      V[i][j] = i == j ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < 4; ++i) {
      dia += A[i][i] * A[i][i];
      for (int j = i + 1; j < 4; ++j) off += A[i][j] * A[i][j];
    }
    if (off == 0.0 || off <= 1e-36 * dia) break;
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 4; ++q) {
        if (A[p][q] == 0.0) continue;
        double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
        double c = 1.0 / hypot(1.0, t), sn = t * c;
        for (int k = 0; k < 4; ++k) { /* columns p, q: A <- A J */
          double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 4; ++k) { /* rows p, q: A <- J^T A */
          double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        A[p][q] = A[q][p] = 0.0;
        for (int k = 0; k < 4; ++k) {
          double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - sn * vkq;
          V[k][q] = sn * vkp + c * vkq;
        }
      }
  }
  int order[4] = {0, 1, 2, 3};
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (A[order[j]][order[j]] < A[order[i]][order[i]]) {
        int t = order[i]; order[i] = order[j]; order[j] = t;
      }
  for (int i = 0; i < 4; ++i) {
    evals[i] = A[order[i]][order[i]];
    for (int r = 0; r < 4; ++r) evecs[4 * r + i] = V[r][order[i]];
  }
}

/* ---------------------------------------------------------------------------
 * Window gathering and back-projection (Eq. 1, delta = 0).
 * ------------------------------------------------------------------------- */
typedef struct {
  double fx, fy, cx, cy;
} cam_t;

static int pixel_valid(const double* depth, const uint8_t* mask, int64_t idx) {
  double z = depth[idx];
  if (mask && mask[idx] == 0) return 0;
  return isfinite(z) && z > 0.0;
}

/* Back-projected points of the window centred at (x0, y0); returns the number
 * of points, or -1 if any window pixel is outside the image or invalid. */
/* Back-projects (Eq. 1) the w x h pixels of columns xa .. xa+w-1 and rows
 * ya .. ya+h-1; -1 if any lies outside the image or is invalid. */
static int gather_rect(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                       const cam_t* cam, int64_t xa, int64_t ya, int64_t w, int64_t h,
                       double* X, double* Y, double* Z) {
  int n = 0;
  for (int64_t y = ya; y < ya + h; ++y)
    for (int64_t x = xa; x < xa + w; ++x) {
      if (x < 0 || y < 0 || x >= W || y >= H) return -1;
      int64_t idx = y * W + x;
      if (!pixel_valid(depth, mask, idx)) return -1;
      double z = depth[idx];
      X[n] = ((double)x - cam->cx) * z / cam->fx;
      Y[n] = ((double)y - cam->cy) * z / cam->fy;
      Z[n] = z;
      ++n;
    }
  return n;
}

/* Partial windows: only the valid pixels of the k x k window (those inside the
 * image with valid depth) are back-projected; the window is fitted iff there are
 * at least max(min_valid, 3) of them and they do not all lie on one line of the
 * pixel grid (else the plane is undetermined); -1 otherwise. */
static int gather_partial(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                          const cam_t* cam, int k, int64_t x0, int64_t y0, int min_valid,
                          double* X, double* Y, double* Z) {
  const int r = k / 2;
  int n = 0, have_a = 0, have_b = 0, spread = 0;
  int64_t ax = 0, ay = 0, bx = 0, by = 0;
  for (int64_t y = y0 - r; y <= y0 + r; ++y)
    for (int64_t x = x0 - r; x <= x0 + r; ++x) {
      if (x < 0 || y < 0 || x >= W || y >= H) continue;
      int64_t idx = y * W + x;
      if (!pixel_valid(depth, mask, idx)) continue;
      if (!have_a) {
        ax = x; ay = y; have_a = 1;
      } else if (!have_b) {
        bx = x; by = y; have_b = 1;
      } else if ((bx - ax) * (y - ay) - (by - ay) * (x - ax) != 0) {
        spread = 1; /* three valid pixels not on one line */
      }
      double z = depth[idx];
      X[n] = ((double)x - cam->cx) * z / cam->fx;
      Y[n] = ((double)y - cam->cy) * z / cam->fy;
      Z[n] = z;
      ++n;
    }
  const int need = min_valid > 3 ? min_valid : 3;
  return (n >= need && spread) ? n : -1;
}

static int gather_window(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                         const cam_t* cam, int k, int64_t x0, int64_t y0, int min_valid,
                         double* X, double* Y, double* Z) {
  const int r = k / 2;
  if (min_valid > 0 && min_valid < k * k)
    return gather_partial(depth, H, W, mask, cam, k, x0, y0, min_valid, X, Y, Z);
  return gather_rect(depth, H, W, mask, cam, x0 - r, y0 - r, k, k, X, Y, Z);
}

typedef struct {
  double n[3], d, residual, kappa;
} fit_t;

/* Orientation.  The smallest eigenvector's sign is free (Sec. I-C), so the
 * plane is made to face the camera: d >= 0.  A plane through the camera centre
 * (d == 0) has no such side; it takes the first non-zero of n_z, n_y, n_x
 * negative.  The offset is never a negative zero. */
static void orient(fit_t* f) {
  int flip;
  if (f->d != 0.0)
    flip = f->d < 0.0;
  else if (f->n[2] != 0.0)
    flip = f->n[2] > 0.0;
  else if (f->n[1] != 0.0)
    flip = f->n[1] > 0.0;
  else
    flip = f->n[0] > 0.0;
  if (flip) {
    f->d = -f->d;
    for (int i = 0; i < 3; ++i) f->n[i] = -f->n[i];
  }
  if (f->d == 0.0) f->d = 0.0;
}

/* RMS over the window of (n.P_i + d)/Z_i: the residual of every mode. */
static double rgbd_rms(const fit_t* f, const double* X, const double* Y, const double* Z,
                       int N) {
  double s = 0.0;
  for (int i = 0; i < N; ++i) {
    double e = (f->n[0] * X[i] + f->n[1] * Y[i] + f->n[2] * Z[i] + f->d) / Z[i];
    s += e * e;
  }
  return sqrt(s / N);
}

static void unit_from(const double v[3], double out[3]) {
  double s = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int i = 0; i < 3; ++i) out[i] = v[i] / s;
}

/* Implicit RGBD fit as weighted total least squares (weights 1/Z^2). */
static void fit_implicit_pca(const double* X, const double* Y, const double* Z, int N,
                             int weighted, fit_t* f) {
  double sw = 0.0, c[3] = {0, 0, 0};
  for (int i = 0; i < N; ++i) {
    double w = weighted ? 1.0 / (Z[i] * Z[i]) : 1.0;
    sw += w;
    c[0] += w * X[i];
    c[1] += w * Y[i];
    c[2] += w * Z[i];
  }
  for (int j = 0; j < 3; ++j) c[j] /= sw;
  double C[9] = {0};
  for (int i = 0; i < N; ++i) {
    double w = weighted ? 1.0 / (Z[i] * Z[i]) : 1.0;
    double p[3] = {X[i] - c[0], Y[i] - c[1], Z[i] - c[2]};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) C[3 * a + b] += w * p[a] * p[b];
  }
  double ev[3], V[9];
  pfo_jacobi3(C, ev, V);
  double n[3] = {V[0], V[3], V[6]};
  unit_from(n, f->n);
  f->d = -(f->n[0] * c[0] + f->n[1] * c[1] + f->n[2] * c[2]);
  f->kappa = (ev[1] > ev[0]) ? ev[2] / (ev[1] - ev[0]) : INFINITY;
}

/* Implicit RGBD fit from the 4x4 scatter of [u, v, 1, w] (Eq. 14), |(a,b,c)| = 1,
 * d eliminated in closed form: S = [[A, b], [b^T, s]] -> A - b b^T / s. */
static void fit_implicit_scatter(const double* X, const double* Y, const double* Z, int N,
                                 fit_t* f) {
  double S[4][4] = {{0}};
  for (int i = 0; i < N; ++i) {
    double m[4] = {X[i] / Z[i], Y[i] / Z[i], 1.0, 1.0 / Z[i]};
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) S[a][b] += m[a] * m[b];
  }
  double C[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) C[3 * a + b] = S[a][b] - S[a][3] * S[b][3] / S[3][3];
  double ev[3], V[9];
  pfo_jacobi3(C, ev, V);
  double n[3] = {V[0], V[3], V[6]};
  unit_from(n, f->n);
  f->d = -(S[0][3] * f->n[0] + S[1][3] * f->n[1] + S[2][3] * f->n[2]) / S[3][3];
  f->kappa = (ev[1] > ev[0]) ? ev[2] / (ev[1] - ev[0]) : INFINITY;
}

/* The implicit fit with the constraint exactly as Sec. II-A states it,
 * |(a, b, c, d)| = 1: the eigenvector of the smallest eigenvalue of the 4x4
 * scatter of [u, v, 1, w] (Eq. 14), then scaled to a unit normal.  Unlike the
 * |(a, b, c)| = 1 fit it depends on the depth unit (d multiplies 1/Z). */
static void fit_implicit_literal(const double* X, const double* Y, const double* Z, int N,
                                 fit_t* f) {
  double S[16] = {0};
  for (int i = 0; i < N; ++i) {
    double m[4] = {X[i] / Z[i], Y[i] / Z[i], 1.0, 1.0 / Z[i]};
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) S[4 * a + b] += m[a] * m[b];
  }
  double ev[4], V[16];
  jacobi4(S, ev, V);
  double s = sqrt(V[0] * V[0] + V[4] * V[4] + V[8] * V[8]);
  f->n[0] = V[0] / s;
  f->n[1] = V[4] / s;
  f->n[2] = V[8] / s;
  f->d = V[12] / s;
  f->kappa = (ev[1] > ev[0]) ? ev[3] / (ev[1] - ev[0]) : INFINITY;
}

/* Explicit plane from coefficients alpha of a u + b v + c = 1/Z: multiplying by Z
 * gives a X + b Y + c Z - 1 = 0, i.e. n = -alpha/|alpha|, d = 1/|alpha|. */
static void explicit_to_plane(const double alpha[3], fit_t* f) {
  double s = sqrt(alpha[0] * alpha[0] + alpha[1] * alpha[1] + alpha[2] * alpha[2]);
  for (int i = 0; i < 3; ++i) f->n[i] = -alpha[i] / s;
  f->d = 1.0 / s;
  f->kappa = NAN;
}

/* Explicit RGBD fit (Eq. 15), least squares on centred regressors. */
static void fit_explicit_centred(const double* X, const double* Y, const double* Z, int N,
                                 fit_t* f) {
  double mu = 0, mv = 0, mw = 0;
  for (int i = 0; i < N; ++i) {
    mu += X[i] / Z[i];
    mv += Y[i] / Z[i];
    mw += 1.0 / Z[i];
  }
  mu /= N; mv /= N; mw /= N;
  double suu = 0, suv = 0, svv = 0, suw = 0, svw = 0;
  for (int i = 0; i < N; ++i) {
    double du = X[i] / Z[i] - mu, dv = Y[i] / Z[i] - mv, dw = 1.0 / Z[i] - mw;
    suu += du * du; suv += du * dv; svv += dv * dv; suw += du * dw; svw += dv * dw;
  }
  double det = suu * svv - suv * suv;
  double alpha[3];
  alpha[0] = (suw * svv - svw * suv) / det;
  alpha[1] = (svw * suu - suw * suv) / det;
  alpha[2] = mw - alpha[0] * mu - alpha[1] * mv;
  explicit_to_plane(alpha, f);
}

/* Solve a 3x3 system by Gaussian elimination with partial pivoting. */
static void solve3(double A[3][3], double b[3], double x[3]) {
  for (int c = 0; c < 3; ++c) {
    int p = c;
    for (int r = c + 1; r < 3; ++r)
      if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
    if (p != c) {
      for (int j = 0; j < 3; ++j) { double t = A[c][j]; A[c][j] = A[p][j]; A[p][j] = t; }
      double t = b[c]; b[c] = b[p]; b[p] = t;
    }
    for (int r = c + 1; r < 3; ++r) {
      double m = A[r][c] / A[c][c];
      for (int j = c; j < 3; ++j) A[r][j] -= m * A[c][j];
      b[r] -= m * b[c];
    }
  }
  for (int r = 2; r >= 0; --r) {
    double s = b[r];
    for (int j = r + 1; j < 3; ++j) s -= A[r][j] * x[j];
    x[r] = s / A[r][r];
  }
}

/* Explicit RGBD fit via the normal equations as written (Eq. 16). */
static void fit_explicit_normaleq(const double* X, const double* Y, const double* Z, int N,
                                  fit_t* f) {
  double A[3][3] = {{0}}, b[3] = {0}, alpha[3];
  for (int i = 0; i < N; ++i) {
    double m[3] = {X[i] / Z[i], Y[i] / Z[i], 1.0}, t = 1.0 / Z[i];
    for (int a = 0; a < 3; ++a) {
      b[a] += m[a] * t;
      for (int c = 0; c < 3; ++c) A[a][c] += m[a] * m[c];
    }
  }
  solve3(A, b, alpha);
  explicit_to_plane(alpha, f);
}

/* Standard explicit XYZ fit (Eq. 7): Z = a X + b Y + c by centred least squares. */
static void fit_xyz_explicit(const double* X, const double* Y, const double* Z, int N,
                             fit_t* f) {
  double mx = 0, my = 0, mz = 0;
  for (int i = 0; i < N; ++i) { mx += X[i]; my += Y[i]; mz += Z[i]; }
  mx /= N; my /= N; mz /= N;
  double sxx = 0, sxy = 0, syy = 0, sxz = 0, syz = 0;
  for (int i = 0; i < N; ++i) {
    double dx = X[i] - mx, dy = Y[i] - my, dz = Z[i] - mz;
    sxx += dx * dx; sxy += dx * dy; syy += dy * dy; sxz += dx * dz; syz += dy * dz;
  }
  double det = sxx * syy - sxy * sxy;
  double a = (sxz * syy - syz * sxy) / det, b = (syz * sxx - sxz * sxy) / det;
  double c = mz - a * mx - b * my;
  double v[3] = {a, b, -1.0};
  double s = sqrt(a * a + b * b + 1.0);
  for (int i = 0; i < 3; ++i) f->n[i] = v[i] / s;
  f->d = c / s;
  f->kappa = NAN;
}

static void nan_out(int64_t o, int64_t plane, double* normals, double* offsets,
                    double* residuals, double* kappa, uint8_t* status) {
  normals[o] = normals[plane + o] = normals[2 * plane + o] = NAN;
  offsets[o] = NAN;
  residuals[o] = NAN;
  if (kappa) kappa[o] = NAN;
  if (status) status[o] = 1;
}

static void fit_gathered(const double* X, const double* Y, const double* Z, int N, int mode,
                         int64_t o, int64_t plane, double* normals, double* offsets,
                         double* residuals, double* kappa, uint8_t* status);

static void fit_one(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                    const cam_t* cam, int k, int mode, int min_valid, int64_t x0, int64_t y0,
                    int64_t o,
                    int64_t plane, double* normals, double* offsets, double* residuals,
                    double* kappa, uint8_t* status, double* buf) {
  double *X = buf, *Y = buf + k * k, *Z = buf + 2 * k * k;
  int N = gather_window(depth, H, W, mask, cam, k, x0, y0, min_valid, X, Y, Z);
  fit_gathered(X, Y, Z, N, mode, o, plane, normals, offsets, residuals, kappa, status);
}

static void fit_gathered(const double* X, const double* Y, const double* Z, int N, int mode,
                         int64_t o, int64_t plane, double* normals, double* offsets,
                         double* residuals, double* kappa, uint8_t* status) {
  if (N < 0) {
    nan_out(o, plane, normals, offsets, residuals, kappa, status);
    return;
  }
  fit_t f;
  switch (mode) {
    case PFO_IMPLICIT: fit_implicit_pca(X, Y, Z, N, 1, &f); break;
    case PFO_IMPLICIT_SCATTER: fit_implicit_scatter(X, Y, Z, N, &f); break;
    case PFO_EXPLICIT: fit_explicit_centred(X, Y, Z, N, &f); break;
    case PFO_EXPLICIT_NORMALEQ: fit_explicit_normaleq(X, Y, Z, N, &f); break;
    case PFO_XYZ_IMPLICIT: fit_implicit_pca(X, Y, Z, N, 0, &f); break;
    case PFO_IMPLICIT_LITERAL: fit_implicit_literal(X, Y, Z, N, &f); break;
    default: fit_xyz_explicit(X, Y, Z, N, &f); break;
  }
  orient(&f);
  f.residual = rgbd_rms(&f, X, Y, Z, N);
  normals[o] = f.n[0];
  normals[plane + o] = f.n[1];
  normals[2 * plane + o] = f.n[2];
  offsets[o] = f.d;
  residuals[o] = f.residual;
  if (kappa) kappa[o] = f.kappa;
  if (status) status[o] = 0;
}

static int bad_args(int64_t H, int64_t W, int k, int mode) {
  return H <= 0 || W <= 0 || k < 1 || k > KMAX || (k % 2) == 0 || mode < 0 || mode > 6;
}

static int fit_planes_impl(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                           double fx, double fy, double cx, double cy, int32_t k, int32_t mode,
                           int32_t min_valid, int32_t threads, double* normals, double* offsets,
                           double* residuals, double* kappa, uint8_t* status) {
  if (!depth || !normals || !offsets || !residuals || bad_args(H, W, k, mode)) return -1;
  cam_t cam = {fx, fy, cx, cy};
  int64_t plane = H * W;
#ifdef _OPENMP
  int nt = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel num_threads(nt)
#endif
  {
    double* buf = (double*)malloc(sizeof(double) * 3 * k * k);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
    for (int64_t y = 0; y < H; ++y)
      for (int64_t x = 0; x < W; ++x)
        fit_one(depth, H, W, mask, &cam, k, mode, min_valid, x, y, y * W + x, plane, normals,
                offsets, residuals, kappa, status, buf);
    free(buf);
  }
  return 0;
}

static int fit_points_impl(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                           double fx, double fy, double cx, double cy, int32_t k, int32_t mode,
                           int32_t min_valid, const int64_t* xs, const int64_t* ys,
                           int64_t count, int32_t threads, double* normals, double* offsets,
                           double* residuals, double* kappa, uint8_t* status) {
  if (!depth || !xs || !ys || !normals || !offsets || !residuals || count < 0 ||
      bad_args(H, W, k, mode))
    return -1;
  cam_t cam = {fx, fy, cx, cy};
#ifdef _OPENMP
  int nt = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel num_threads(nt)
#endif
  {
    double* buf = (double*)malloc(sizeof(double) * 3 * k * k);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < count; ++i)
      fit_one(depth, H, W, mask, &cam, k, mode, min_valid, xs[i], ys[i], i, count, normals,
              offsets, residuals, kappa, status, buf);
    free(buf);
  }
  return 0;
}

int pfo_fit_planes(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                   double fx, double fy, double cx, double cy, int32_t k, int32_t mode,
                   int32_t threads, double* normals, double* offsets, double* residuals,
                   double* kappa, uint8_t* status) {
  return fit_planes_impl(depth, H, W, mask, fx, fy, cx, cy, k, mode, 0, threads, normals,
                         offsets, residuals, kappa, status);
}

int pfo_fit_points(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                   double fx, double fy, double cx, double cy, int32_t k, int32_t mode,
                   const int64_t* xs, const int64_t* ys, int64_t count, int32_t threads,
                   double* normals, double* offsets, double* residuals, double* kappa,
                   uint8_t* status) {
  return fit_points_impl(depth, H, W, mask, fx, fy, cx, cy, k, mode, 0, xs, ys, count, threads,
                         normals, offsets, residuals, kappa, status);
}

int pfo_fit_planes_partial(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                           double fx, double fy, double cx, double cy, int32_t k, int32_t mode,
                           int32_t min_valid, int32_t threads, double* normals,
                           double* offsets, double* residuals, double* kappa, uint8_t* status) {
  if (min_valid < 3) return -1;
  return fit_planes_impl(depth, H, W, mask, fx, fy, cx, cy, k, mode, min_valid, threads,
                         normals, offsets, residuals, kappa, status);
}

int pfo_fit_points_partial(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                           double fx, double fy, double cx, double cy, int32_t k, int32_t mode,
                           int32_t min_valid, const int64_t* xs, const int64_t* ys,
                           int64_t count, int32_t threads, double* normals, double* offsets,
                           double* residuals, double* kappa, uint8_t* status) {
  if (min_valid < 3) return -1;
  return fit_points_impl(depth, H, W, mask, fx, fy, cx, cy, k, mode, min_valid, xs, ys, count,
                         threads, normals, offsets, residuals, kappa, status);
}

int pfo_fit_rects(const double* depth, int64_t H, int64_t W, const uint8_t* mask, double fx,
                  double fy, double cx, double cy, const int32_t* rects, int64_t count,
                  int32_t mode, int32_t threads, double* normals, double* offsets,
                  double* residuals, double* kappa, uint8_t* status) {
  if (!depth || !rects || !normals || !offsets || !residuals || count < 0 || H <= 0 ||
      W <= 0 || mode < 0 || mode > 6)
    return -1;
  cam_t cam = {fx, fy, cx, cy};
#ifdef _OPENMP
  int nt = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel for num_threads(nt) schedule(dynamic, 16)
#endif
  for (int64_t i = 0; i < count; ++i) {
    const int64_t xa = rects[4 * i], ya = rects[4 * i + 1];
    const int64_t w = rects[4 * i + 2], h = rects[4 * i + 3];
    int N = -1;
    double* buf = NULL;
    if (w >= 2 && h >= 2 && xa >= 0 && ya >= 0 && xa + w <= W && ya + h <= H) {
      buf = (double*)malloc(sizeof(double) * 3 * (size_t)(w * h));
      N = gather_rect(depth, H, W, mask, &cam, xa, ya, w, h, buf, buf + w * h,
                      buf + 2 * w * h);
    }
    fit_gathered(buf, buf ? buf + w * h : NULL, buf ? buf + 2 * w * h : NULL, N, mode, i, count,
                 normals, offsets, residuals, kappa, status);
    free(buf);
  }
  return 0;
}

void pfo_camera_moments(double fx, double fy, double cx, double cy, int32_t k, int64_t x0,
                        int64_t y0, double out[6]) {
  int r = k / 2;
  double s[6] = {0};
  for (int dy = -r; dy <= r; ++dy)
    for (int dx = -r; dx <= r; ++dx) {
      double u = ((double)(x0 + dx) - cx) / fx, v = ((double)(y0 + dy) - cy) / fy;
      s[0] += u * u; s[1] += u * v; s[2] += u; s[3] += v * v; s[4] += v; s[5] += 1.0;
    }
  memcpy(out, s, sizeof(s));
}

/* The five depth-dependent integrands at one pixel (zero when invalid). */
static void integrands(const double* depth, const uint8_t* mask, int64_t W, int64_t x,
                       int64_t y, const cam_t* cam, double g[5]) {
  int64_t idx = y * W + x;
  if (!pixel_valid(depth, mask, idx)) {
    g[0] = g[1] = g[2] = g[3] = g[4] = 0.0;
    return;
  }
  double w = 1.0 / depth[idx];
  double u = ((double)x - cam->cx) / cam->fx, v = ((double)y - cam->cy) / cam->fy;
  g[0] = w; g[1] = u * w; g[2] = v * w; g[3] = w * w; g[4] = 1.0;
}

void pfo_window_sums(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                     double fx, double fy, double cx, double cy, int32_t k, double* out) {
  cam_t cam = {fx, fy, cx, cy};
  int r = k / 2;
  int64_t plane = H * W;
  for (int64_t y0 = 0; y0 < H; ++y0)
    for (int64_t x0 = 0; x0 < W; ++x0) {
      double s[5] = {0};
      for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
          int64_t x = x0 + dx, y = y0 + dy;
          if (x < 0 || y < 0 || x >= W || y >= H) continue;
          double g[5];
          integrands(depth, mask, W, x, y, &cam, g);
          for (int c = 0; c < 5; ++c) s[c] += g[c];
        }
      for (int c = 0; c < 5; ++c) out[c * plane + y0 * W + x0] = s[c];
    }
}

void pfo_integral_images(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                         double fx, double fy, double cx, double cy, double* out) {
  cam_t cam = {fx, fy, cx, cy};
  int64_t P = (H + 1) * (W + 1);
  for (int c = 0; c < 5; ++c) {
    double* I = out + c * P;
    for (int64_t x = 0; x <= W; ++x) I[x] = 0.0;
    for (int64_t y = 0; y < H; ++y) {
      double row = 0.0;
      I[(y + 1) * (W + 1)] = 0.0;
      for (int64_t x = 0; x < W; ++x) {
        double g[5];
        integrands(depth, mask, W, x, y, &cam, g);
        row += g[c];
        I[(y + 1) * (W + 1) + x + 1] = I[y * (W + 1) + x + 1] + row;
      }
    }
  }
}

static double box(const double* I, int64_t W, int64_t x0, int64_t y0, int64_t x1, int64_t y1) {
  /* sum over x in [x0, x1), y in [y0, y1) of the image whose integral image is I */
  int64_t p = W + 1;
  return I[y1 * p + x1] - I[y0 * p + x1] - I[y1 * p + x0] + I[y0 * p + x0];
}

int pfo_fit_planes_integral(const double* depth, int64_t H, int64_t W, const uint8_t* mask,
                            double fx, double fy, double cx, double cy, int32_t k,
                            int32_t mode, double* normals, double* offsets,
                            double* residuals, uint8_t* status) {
  if (!depth || !normals || !offsets || !residuals || bad_args(H, W, k, mode) ||
      (mode != PFO_IMPLICIT && mode != PFO_EXPLICIT))
    return -1;
  int64_t P = (H + 1) * (W + 1), plane = H * W;
  double* I = (double*)malloc(sizeof(double) * 5 * P);
  double* J = (double*)malloc(sizeof(double) * 5 * P); /* camera-only images */
  if (!I || !J) { free(I); free(J); return -1; }
  pfo_integral_images(depth, H, W, mask, fx, fy, cx, cy, I);
  /* camera-only integrands u^2, u v, u, v^2, v: fixed for a given calibration */
  for (int c = 0; c < 5; ++c) {
    double* Jc = J + c * P;
    for (int64_t x = 0; x <= W; ++x) Jc[x] = 0.0;
    for (int64_t y = 0; y < H; ++y) {
      double row = 0.0;
      Jc[(y + 1) * (W + 1)] = 0.0;
      for (int64_t x = 0; x < W; ++x) {
        double u = ((double)x - cx) / fx, v = ((double)y - cy) / fy;
        double g[5] = {u * u, u * v, u, v * v, v};
        row += g[c];
        Jc[(y + 1) * (W + 1) + x + 1] = Jc[y * (W + 1) + x + 1] + row;
      }
    }
  }
  int r = k / 2;
  for (int64_t y0 = 0; y0 < H; ++y0)
    for (int64_t x0 = 0; x0 < W; ++x0) {
      int64_t o = y0 * W + x0;
      int64_t xa = x0 - r, xb = x0 + r + 1, ya = y0 - r, yb = y0 + r + 1;
      double cnt = -1.0;
      if (xa >= 0 && ya >= 0 && xb <= W && yb <= H) cnt = box(I + 4 * P, W, xa, ya, xb, yb);
      if (cnt != (double)(k * k)) {
        nan_out(o, plane, normals, offsets, residuals, NULL, status);
        continue;
      }
      double sw = box(I, W, xa, ya, xb, yb), suw = box(I + P, W, xa, ya, xb, yb);
      double svw = box(I + 2 * P, W, xa, ya, xb, yb), sww = box(I + 3 * P, W, xa, ya, xb, yb);
      double suu = box(J, W, xa, ya, xb, yb), suv = box(J + P, W, xa, ya, xb, yb);
      double su = box(J + 2 * P, W, xa, ya, xb, yb), svv = box(J + 3 * P, W, xa, ya, xb, yb);
      double sv = box(J + 4 * P, W, xa, ya, xb, yb), N = (double)(k * k);
      fit_t f;
      if (mode == PFO_IMPLICIT) {
        double S[4][4] = {{suu, suv, su, suw}, {suv, svv, sv, svw}, {su, sv, N, sw},
                          {suw, svw, sw, sww}};
        double C[9];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) C[3 * a + b] = S[a][b] - S[a][3] * S[b][3] / S[3][3];
        double ev[3], V[9];
        pfo_jacobi3(C, ev, V);
        double n[3] = {V[0], V[3], V[6]};
        unit_from(n, f.n);
        f.d = -(suw * f.n[0] + svw * f.n[1] + sw * f.n[2]) / sww;
      } else {
        double A[3][3] = {{suu, suv, su}, {suv, svv, sv}, {su, sv, N}}, b[3] = {suw, svw, sw};
        double alpha[3];
        solve3(A, b, alpha);
        explicit_to_plane(alpha, &f);
      }
      orient(&f);
      /* residual from the moments: sum (n.m + d w)^2 with m = (u, v, 1) */
      double a0 = f.n[0], a1 = f.n[1], a2 = f.n[2], a3 = f.d;
      double q = a0 * a0 * suu + a1 * a1 * svv + a2 * a2 * N + a3 * a3 * sww +
                 2 * (a0 * a1 * suv + a0 * a2 * su + a0 * a3 * suw + a1 * a2 * sv +
                      a1 * a3 * svw + a2 * a3 * sw);
      normals[o] = f.n[0];
      normals[plane + o] = f.n[1];
      normals[2 * plane + o] = f.n[2];
      offsets[o] = f.d;
      residuals[o] = sqrt(fmax(q, 0.0) / N);
      if (status) status[o] = 0;
    }
  free(I);
  free(J);
  return 0;
}
