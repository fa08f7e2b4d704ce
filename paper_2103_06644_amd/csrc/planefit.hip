// planefit: per-pixel RGBD plane fits on MI355X (gfx950).  C-ABI in
// include/planefit.h.
//
// One fused kernel runs the whole per-frame path of the paper's integral-image
// method (Sec. II-A..C) for a tile of output pixels:
//
//   integrands  w = 1/Z (or D * scale for disparity input) and its products
//               with the window coordinates, shifted by a per-tile reference
//               disparity so the sums stay small;
//   2D scan     a transposed integral-image sweep: every thread owns one image
//               column and slides a k-row window sum down the tile (a row
//               enters as the row k above leaves, the leaving sample recomputed
//               with the same operations), then every thread owns a run of
//               output pixels of a row and slides a k-column sum of those
//               column sums along it.  Each slide is the four-corner difference
//               of an integral image (Sec. II-C) up to rounding order, with no
//               k-row history kept anywhere;
//   solve       explicit (Eq. 15-16) in closed form, or implicit (Eq. 14) as a
//               3x3 symmetric eigenproblem after eliminating d (or the literal
//               4x4 with |(a, b, c, d)| = 1; or, for partial windows, with the
//               valid-pixel camera moments carried as extra integer channels);
//   store       normals (channel-planar), offsets, residuals, status.
//
// Only depth comes in and only the five outputs go out: the integral images
// live in registers and LDS.  The camera-only moments (sum u^2 ... N) enter in
// closed form in window-centred coordinates, where the k x k window has
// sum x' = sum y' = sum x'y' = 0 and sum x'^2 = sum y'^2 = k^2 (k^2 - 1)/12.
//
// Also here: the adjoint (a backward instantiation of the same sweep, then a
// box-filter sweep back to the pixels), the standard XYZ formulation for
// comparison (Eq. 3-9, nine channels), and global FP64 integral images with
// fits to arbitrary rectangles (the paper's own use of integral images).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>
#include <atomic>
#include <mutex>

#include "planefit.h"

namespace {

constexpr int kBlock = 256;   // threads per workgroup; also the strip width in input columns
constexpr int kMaxWindow = 63;

// Launch shapes.  Work split of one round: `rows` output rows go through the
// vertical phase together, then every thread fits a run of `run` consecutive
// outputs of one row (kBlock / run runs per row, rows * kBlock / run = kBlock
// threads); `groups` is the number of workgroups per CU the register budget
// is sized for (four: 128 VGPRs; two: 256).
//   shape 0: 4 x 4, register budget of four workgroups per CU (128 VGPRs;
//            37 KB of LDS in FP64);
//   shape 1: 4 x 4, budget of two workgroups per CU (256 VGPRs).  The FP64
//            implicit kernel still fits in 128, so it runs four per CU like
//            shape 0, with the schedule the larger budget allows (the default
//            for FP64 implicit fits);
//   shape 2: 8 x 8, two workgroups per CU (74 KB of LDS; half the per-run
//            warm-up and half the barriers per row).
// Shapes 1 and 2 exist for FP64 implicit and explicit full-window fits (the
// autotuner's candidates); every other path runs shape 0.
//
// LDS layout of one row of window column sums: column i lives at record
// (i % run) * sub + i / run, each record 16 bytes (see ColumnSums).  In the
// horizontal phase, where almost all LDS traffic is (two reads per column
// per output), the runs of a row read the same (i % run) with consecutive
// i / run: consecutive records, no bank conflicts.  The vertical phase writes
// each column once per row, neighbouring threads `sub` records apart; with
// 16 * sub = 32 (mod 128) bytes the eight lanes a 16-byte LDS access serves
// per cycle hit eight different 16-byte bank groups.
template <int SHAPE>
struct Tiling;
template <>
struct Tiling<0> {
  static constexpr int rows = 4, run = 4, sub = 74, groups = 4;
};
template <>
struct Tiling<1> : Tiling<0> {
  static constexpr int groups = 2;
};
template <>
struct Tiling<2> {
  static constexpr int rows = 8, run = 8, sub = 37, groups = 2;
};
constexpr int kShapes = 3;
constexpr int kPitch = 296;  // LDS records per row, >= kBlock for every tiling
static_assert((16 * Tiling<0>::sub) % 128 == 32, "shape 0 write banks");
static_assert((16 * Tiling<2>::sub) % 128 == 80, "shape 2 write banks");
static_assert(Tiling<0>::run * Tiling<0>::sub == kPitch, "pitch");
static_assert(Tiling<2>::run * Tiling<2>::sub == kPitch, "pitch");
static_assert(Tiling<0>::rows * kBlock / Tiling<0>::run == kBlock, "split");
static_assert(Tiling<2>::rows * kBlock / Tiling<2>::run == kBlock, "split");
constexpr int shape_groups(int shape) {
  return shape == 0 ? Tiling<0>::groups : shape == 1 ? Tiling<1>::groups : Tiling<2>::groups;
}
constexpr int shape_rows(int shape) {
  return shape == 2 ? Tiling<2>::rows : Tiling<0>::rows;
}

template <int SHAPE>
__host__ __device__ inline int lds_index(int i) {
  using TL = Tiling<SHAPE>;
  const unsigned u = unsigned(i);  // i >= 0 always
  return int((u % TL::run) * TL::sub + u / TL::run);
}

struct FitArgs {
  const float* depth;
  const uint8_t* mask;
  float* normals;
  float* offsets;
  float* residuals;
  uint8_t* status;
  int64_t depth_pitch;
  int64_t mask_pitch;
  int64_t plane;  // H * W
  int H, W, k, r;
  int tile_w;     // output columns per strip
  int tile_h;     // output rows per band
  int n_strips;
  int n_bands;
  double fx, fy, cx, cy;
  double inv_fx, inv_fy;
  double S2, inv_S2, N, inv_N;
  double kappa_flag;
  double kappa_fp64;  // compensated path: FP64 re-solve above this FP32 kappa
  int vec_store;  // outputs 16-byte aligned, W and tile_w multiples of 4
  double* gws;    // backward: per-window moment gradients [4][H][W]
  double dscale;  // > 0: the input is disparity D with w = D * dscale; 0: depth Z, w = 1/Z
  int min_valid;  // partial windows: fitted from >= min_valid valid pixels
};

// One frame of a launch, passed by value in the kernel arguments.
struct Job {
  const float* depth;
  const uint8_t* mask;
  float* normals;
  float* offsets;
  float* residuals;
  uint8_t* status;
  double fx, fy, cx, cy;
  int32_t depth_pitch, mask_pitch;
  int32_t H, W, k, tile_w, tile_h, n_strips;
  int32_t wg_begin;   // first workgroup of this job in the launch
  int16_t vec_store;  // 1: outputs stored as float4 runs
  int16_t min_valid;  // partial windows: minimum valid pixels per window (< k^2 <= 3969)
};
static_assert(kMaxWindow * kMaxWindow <= INT16_MAX, "min_valid is kept in 16 bits");

// Up to kMaxJobs frames (any sizes and window sizes, one mode and precision)
// per launch; the whole struct stays under the 4 KiB kernel-argument limit.
constexpr int kMaxJobs = 32;
constexpr double kDefaultKappaFp64 = 100.0;
struct LaunchArgs {
  int32_t n_jobs;
  int32_t n_wg;
  double kappa_flag;
  double kappa_fp64;
  double dscale;  // disparity input scale (0: depth input), shared by the launch's jobs
  double* gws;  // backward launches: moment-gradient workspace (one region per job)
  Job jobs[kMaxJobs];
};
static_assert(sizeof(LaunchArgs) <= 4096, "kernel arguments too large");

// ---------------------------------------------------------------------------
// Per-pixel integrand (Sec. II-A: the entries of Eq. 14 that depend on depth).
// ---------------------------------------------------------------------------
__device__ inline bool depth_valid(float z) {
  // finite and strictly positive; written on the bit pattern so no fast-math
  // assumption can drop the test
  const uint32_t b = __float_as_uint(z);
  return ((b & 0x7f800000u) != 0x7f800000u) && z > 0.0f;
}

template <typename T>
struct Cursor {
  T w, yw, ww;  // sums of (w - w_ref), (y - y_ref)(w - w_ref), (w - w_ref)^2
  int n;        // number of valid pixels
  int yn, y2n;  // partial windows: sums of (y - y_ref) and (y - y_ref)^2 over valid pixels
  __device__ void clear() {
    w = yw = ww = T(0);
    n = yn = y2n = 0;
  }
};

// Depth sample of (x, y), with 0 standing for "no valid sample" (outside the
// image, masked out, or `use` false).  Branch-free: the address is clamped into
// the image so every lane loads, and the sample is selected afterwards; a group
// of such loads can then be in flight together before any is consumed.
template <bool MASK>
__device__ inline float load_depth(const FitArgs& a, int x, int y, bool use = true) {
  const bool in = use && x >= 0 && x < a.W && y >= 0 && y < a.H;
  const int xc = min(max(x, 0), a.W - 1), yc = min(max(y, 0), a.H - 1);
  float z = a.depth[(int64_t)yc * a.depth_pitch + xc];
  if (MASK && a.mask) z = a.mask[(int64_t)yc * a.mask_pitch + xc] ? z : 0.0f;
  return in ? z : 0.0f;
}

// Reciprocal of a positive depth: hardware estimate refined by one
// Newton-Raphson step r <- r + r (1 - z r).  Homogeneous under power-of-two
// scaling of z, like the rest of the path.
__device__ inline double recip(float zf, double) {
  const double z = double(depth_valid(zf) ? zf : 1.0f);
  const double r = __builtin_amdgcn_rcp(z);
  return fma(r, fma(-z, r, 1.0), r);
}
__device__ inline float recip(float zf, float) {
  const float z = depth_valid(zf) ? zf : 1.0f;
  float r = __builtin_amdgcn_rcpf(z);
  const float e = fmaf(-z, r, 1.0f);
  return fmaf(r, e, r);
}

// Hardware reciprocal estimate, unrefined.
__device__ inline double rcp_raw(double x) { return __builtin_amdgcn_rcp(x); }
__device__ inline float rcp_raw(float x) { return __builtin_amdgcn_rcpf(x); }

// Reciprocal and reciprocal square root of a positive normal number: hardware
// estimate plus one Newton-Raphson step.  The FP64 estimates are good to about
// 5e-8 (measured on gfx950), so one step leaves about 4e-15 relative error:
// far below what the float outputs carry, and in a depth sample's 1/Z below
// any depth noise (the same value is added and taken out again).
__device__ inline double rcp_nr(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ inline float rcp_nr(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ inline double rsq_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * fma(-0.5 * x * y, y, 1.5);  // y <- y (3 - x y^2) / 2
}
__device__ inline float rsq_nr(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  return y * fmaf(-0.5f * x * y, y, 1.5f);
}

// ---------------------------------------------------------------------------
// Two-float ("double-float") arithmetic for the compensated path: a value is
// the unevaluated sum hi + lo of two FP32 numbers, |lo| <= ulp(hi)/2.  Sums use
// Knuth's TwoSum and Dekker's FastTwoSum error-free transformations, products
// use the FMA-based TwoProduct; about 48 significant bits.  Floating-point
// contraction is switched off inside these functions: fusing the product of
// TwoProduct into the FastTwoSum that follows would use the exact product where
// the error term was taken against the rounded one and double-count it.
// ---------------------------------------------------------------------------
struct df32 {
  float hi, lo;
  df32() = default;
  __host__ __device__ constexpr df32(float h) : hi(h), lo(0.0f) {}
  __host__ __device__ constexpr df32(float h, float l) : hi(h), lo(l) {}
  __host__ __device__ explicit df32(int v) : hi(float(v)), lo(0.0f) {}
};

__device__ inline df32 two_sum(float a, float b) {
#pragma clang fp contract(off)
  const float s = a + b;
  const float bb = s - a;
  return df32(s, (a - (s - bb)) + (b - bb));
}
__device__ inline df32 fast_two_sum(float a, float b) {
#pragma clang fp contract(off)
  const float s = a + b;
  return df32(s, b - (s - a));
}
__device__ inline df32 operator+(df32 a, df32 b) {
#pragma clang fp contract(off)
  df32 s = two_sum(a.hi, b.hi);
  const df32 t = two_sum(a.lo, b.lo);
  s = fast_two_sum(s.hi, s.lo + t.hi);
  return fast_two_sum(s.hi, s.lo + t.lo);
}
__device__ inline df32 operator-(df32 a) { return df32(-a.hi, -a.lo); }
__device__ inline df32 operator-(df32 a, df32 b) { return a + (-b); }
__device__ inline df32& operator+=(df32& a, df32 b) { return a = a + b; }
__device__ inline df32 operator*(df32 a, df32 b) {
#pragma clang fp contract(off)
  const float p = a.hi * b.hi;
  float e = fmaf(a.hi, b.hi, -p);
  e = fmaf(a.hi, b.lo, e);
  e = fmaf(a.lo, b.hi, e);
  return fast_two_sum(p, e);
}
__device__ inline double to_double(df32 a) { return double(a.hi) + double(a.lo); }
__device__ inline df32 to_df32(double d) {
  const float h = float(d);
  return df32(h, float(d - double(h)));
}
// 1/z as a two-float: the FMA residual 1 - z r is exact, so r + r (1 - z r)
// carries the reciprocal to ~2^-46.
__device__ inline df32 recip(float zf, df32) {
#pragma clang fp contract(off)
  const float z = depth_valid(zf) ? zf : 1.0f;
  const float r = rcp_nr(z);
  const float e = fmaf(-z, r, 1.0f);
  return fast_two_sum(r, r * e);
}

// Disparity w of a valid sample: 1/Z for depth input, D * dscale for disparity
// input (one rounding either way: the product is exact to the last bit of T).
__device__ inline double disparity(float z, double dscale, double) {
  return dscale > 0.0 ? double(z) * dscale : recip(z, 0.0);
}
__device__ inline float disparity(float z, double dscale, float) {
  return dscale > 0.0 ? z * float(dscale) : recip(z, 0.0f);
}
__device__ inline df32 disparity(float z, double dscale, df32) {
  return dscale > 0.0 ? df32(z) * to_df32(dscale) : recip(z, df32(0.0f));
}

// The sample's centred disparity w - w_ref, exactly 0 for an invalid sample.
// FP64 takes no branch per sample: w = 1/Z (depth input) and w = D * dscale
// (disparity input) are one blend r m + D s with (m, s) = (1, 0) or
// (0, dscale), exact either way since a valid sample's reciprocal is finite;
// an invalid sample's value, whatever it is, is then replaced by 0.
template <typename T>
__device__ inline T centred_w(float z, bool ok, T w_ref, double dscale) {
  if constexpr (std::is_same<T, double>::value) {
    const double zd = double(z);
    const double m = dscale > 0.0 ? 0.0 : 1.0, s = dscale > 0.0 ? dscale : 0.0;
    const double w = fma(rcp_nr(zd), m, zd * s);
    return ok ? w - w_ref : 0.0;
  } else {
    return ok ? disparity(z, dscale, T(0.0f)) - w_ref : T(0.0f);
  }
}

template <typename T, bool PARTIAL = false>
__device__ inline void add_sample(float z, int y, T w_ref, int y_ref, Cursor<T>& c, double dscale) {
  // branch-free: invalid samples contribute exact zeros
  const bool ok = depth_valid(z);
  const T wh = centred_w(z, ok, w_ref, dscale);
  c.w += wh;
  c.yw += T(y - y_ref) * wh;
  c.ww += wh * wh;
  c.n += ok ? 1 : 0;
  if (PARTIAL) {
    const int dy = ok ? y - y_ref : 0;
    c.yn += dy;
    c.y2n += dy * dy;
  }
}

// The same sample taken out again: recomputed with the same operations, so
// it is the exact value that was added.
template <typename T, bool PARTIAL = false>
__device__ inline void sub_sample(float z, int y, T w_ref, int y_ref, Cursor<T>& c, double dscale) {
  const bool ok = depth_valid(z);
  const T wh = centred_w(z, ok, w_ref, dscale);
  c.w = c.w - wh;
  c.yw = c.yw - T(y - y_ref) * wh;
  c.ww = c.ww - wh * wh;
  c.n -= ok ? 1 : 0;
  if (PARTIAL) {
    const int dy = ok ? y - y_ref : 0;
    c.yn -= dy;
    c.y2n -= dy * dy;
  }
}

// ---------------------------------------------------------------------------
// Symmetric 3x3 smallest eigenpair of a positive semidefinite matrix.
//
// f(l) = det(B - l I) = (l1 - l)(l2 - l)(l3 - l) is convex and decreasing on
// (-inf, l1] and l1 >= 0, so Halley's iteration started at l = 0 climbs to l1
// (cubically once close).  The other two eigenvalues follow by deflating
// the characteristic cubic to a quadratic.  The eigenvector is the
// best-conditioned cross product of two rows of B - l1 I (the approach of
// J. Kopp, "Efficient numerical diagonalization of hermitian 3x3 matrices",
// 2008).  Accuracy of the normal ~ eps * l3 / (l2 - l1).
// ---------------------------------------------------------------------------
template <typename T>
struct Eig3 {
  T l1, l2, l3;  // ascending
  T n[3];        // unit eigenvector of l1
  bool degenerate;
};

template <typename T>
__device__ inline T det3(T a00, T a01, T a02, T a11, T a12, T a22) {
  return a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) +
         a02 * (a01 * a12 - a11 * a02);
}

template <typename T>
__device__ inline Eig3<T> smallest_eig(T c00, T c01, T c02, T c11, T c12, T c22,
                                       bool spectrum = true) {
  Eig3<T> e;
  e.degenerate = false;
  T s = fmax(fabs(c00), fmax(fabs(c11), fabs(c22)));
  if (!(s > T(0)) || !isfinite(s)) {
    e.l1 = e.l2 = e.l3 = T(0);
    e.n[0] = T(0); e.n[1] = T(0); e.n[2] = T(-1);
    e.degenerate = true;
    return e;
  }
  // scale by the power of two nearest below 1/s: exact, keeps every entry <= 1
  const T is = ldexp(T(1), -ilogb(s));
  const T b00 = c00 * is, b01 = c01 * is, b02 = c02 * is;
  const T b11 = c11 * is, b12 = c12 * is, b22 = c22 * is;
  // characteristic polynomial det(B - l I) = -l^3 + c2 l^2 - c1 l + c0
  const T c2 = b00 + b11 + b22;
  const T c1 = (b11 * b22 - b12 * b12) + (b00 * b22 - b02 * b02) + (b00 * b11 - b01 * b01);
  const T c0 = det3(b00, b01, b02, b11, b12, b22);

  // Halley's iteration from the lower bound c0/c1 = 1/(1/l1 + 1/l2 + 1/l3) <= l1:
  // cubic convergence; on (-inf, l1] the polynomial is convex and decreasing
  // and the iterates rise towards l1.  The tolerance (1e-13 of the largest
  // diagonal entry, FP64) keeps the eigenvector error below 1e-13 * kappa.
  T l = T(0);
  if (c0 > T(0) && c1 > T(0)) {
    l = c0 * rcp_nr(c1);
    const T tol = sizeof(T) == 8 ? T(1e-13) : T(1e-8);
    for (int it = 0; it < 24; ++it) {
      const T f = ((c2 - l) * l - c1) * l + c0;
      const T fp = (T(2) * c2 - T(3) * l) * l - c1;
      const T fpp = T(2) * c2 - T(6) * l;
      if (!(f > T(0)) || !(fp < T(0))) break;
      const T den = T(2) * fp * fp - f * fpp;
      if (!(den > T(0))) break;
      // the step's reciprocal needs no refinement: an error of relative size e
      // in a step of size s leaves e s, which the next iteration removes
      const T ln = l - T(2) * f * fp * rcp_raw(den);
      if (!(ln > l)) break;
      const T step = ln - l;
      l = ln;
      if (step <= tol) break;
    }
  }
  // deflate: l2 + l3 = tr - l1, l2 l3 = c1 - l1 (l2 + l3); only when the caller
  // needs the conditioning (a uniform choice: kappa flag, FP64 fallback, adjoint)
  e.l2 = e.l3 = T(0);
  if (spectrum) {
    const T t = c2 - l;
    const T pr = c1 - l * t;
    const T disc = t * t - T(4) * pr;
    const T sq = disc > T(0) ? disc * rsq_nr(disc) : T(0);
    const T l3 = T(0.5) * (t + sq);
    e.l3 = l3;
    e.l2 = l3 > T(0) ? pr * rcp_nr(l3) : T(0);
  }

  // eigenvector: largest cross product of two rows of (B - l I); in FP32 the
  // eigenvalue from the polynomial carries an error ~ eps / f'(l1), so one
  // Rayleigh-quotient step (l <- v^T B v, then the cross product again) brings
  // the eigenvector error back from ~eps kappa^2 to ~eps kappa.
  T vx, vy, vz, nn;
  const int passes = sizeof(T) == 4 ? 2 : 1;
  for (int pass = 0; pass < passes; ++pass) {
    if (pass == 1) {
      const T ux = vx * rsq_nr(nn), uy = vy * rsq_nr(nn), uz = vz * rsq_nr(nn);
      l = ux * (b00 * ux + b01 * uy + b02 * uz) + uy * (b01 * ux + b11 * uy + b12 * uz) +
          uz * (b02 * ux + b12 * uy + b22 * uz);
    }
    const T a00 = b00 - l, a11 = b11 - l, a22 = b22 - l;
    // r0 = (a00, b01, b02), r1 = (b01, a11, b12), r2 = (b02, b12, a22)
    const T x0 = b01 * b12 - b02 * a11, y0 = b02 * b01 - a00 * b12, z0 = a00 * a11 - b01 * b01;
    const T x1 = b01 * a22 - b02 * b12, y1 = b02 * b02 - a00 * a22, z1 = a00 * b12 - b01 * b02;
    const T x2 = a11 * a22 - b12 * b12, y2 = b12 * b02 - b01 * a22, z2 = b01 * b12 - a11 * b02;
    const T n0 = x0 * x0 + y0 * y0 + z0 * z0;
    const T n1 = x1 * x1 + y1 * y1 + z1 * z1;
    const T n2 = x2 * x2 + y2 * y2 + z2 * z2;
    vx = x0; vy = y0; vz = z0; nn = n0;
    if (n1 > nn) { vx = x1; vy = y1; vz = z1; nn = n1; }
    if (n2 > nn) { vx = x2; vy = y2; vz = z2; nn = n2; }
    if (!(nn > T(0)) || !isfinite(nn)) {
      // l1 has multiplicity >= 2: any vector orthogonal to the largest row
      T rx = a00, ry = b01, rz = b02;
      T rn = rx * rx + ry * ry + rz * rz;
      const T r1n = b01 * b01 + a11 * a11 + b12 * b12;
      if (r1n > rn) { rx = b01; ry = a11; rz = b12; rn = r1n; }
      const T r2n = b02 * b02 + b12 * b12 + a22 * a22;
      if (r2n > rn) { rx = b02; ry = b12; rz = a22; rn = r2n; }
      if (rn > T(0)) {
        // cross with the coordinate axis least aligned with r
        if (fabs(rx) <= fabs(ry) && fabs(rx) <= fabs(rz)) { vx = T(0); vy = rz; vz = -ry; }
        else if (fabs(ry) <= fabs(rz)) { vx = -rz; vy = T(0); vz = rx; }
        else { vx = ry; vy = -rx; vz = T(0); }
      } else {
        vx = T(0); vy = T(0); vz = T(1);
      }
      nn = vx * vx + vy * vy + vz * vz;
      e.degenerate = true;
      break;
    }
  }
  const T inv = rsq_nr(nn);
  e.n[0] = vx * inv;
  e.n[1] = vy * inv;
  e.n[2] = vz * inv;
  // undo the power-of-two scaling exactly
  const int ex = ilogb(s);
  e.l1 = ldexp(l, ex);
  e.l2 = ldexp(e.l2, ex);
  e.l3 = ldexp(e.l3, ex);
  return e;
}

// ---------------------------------------------------------------------------
// Per-pixel solve from the window sums.
//   B  = sum (w - w_ref)                 Fx = sum (x - x_c)(w - w_ref)
//   Fy = sum (y - y_c)(w - w_ref)        Q  = sum (w - w_ref)^2
// where x_c, y_c are the window centre's column and row; w = 1/Z.
// ---------------------------------------------------------------------------
// Orientation.  The smallest eigenvector's sign is free (Sec. I-C): the plane
// is made to face the camera, d >= 0.  A plane through the camera centre
// (d == 0) takes the first non-zero of n_z, n_y, n_x negative.  Returns
// whether (n, d) must be negated.
template <typename S>
__device__ inline bool facing_flip(S d, S n0, S n1, S n2) {
  // the first non-zero of (d, -n_z, -n_y, -n_x) decides; selects, no branches
  const S key = d != S(0) ? d : (n2 != S(0) ? -n2 : (n1 != S(0) ? -n1 : -n0));
  return key < S(0);
}

// Square root of a non-negative float output (the residual): the hardware
// instruction, within about 1 ulp, instead of the correctly rounded library
// sequence around it (some fourteen instructions per pixel).
__device__ inline float sqrt_out(float x) { return __builtin_amdgcn_sqrtf(x); }

struct PixelOut {
  float n0, n1, n2, d, res;
  uint8_t st;
  float kappa;  // implicit: l3 / (l2 - l1) of the 3x3 (inf when degenerate)
};

// ---------------------------------------------------------------------------
// Output stores of the horizontal phase through buffer resources.  A wave fits
// ROWS consecutive output rows of one strip (one for runs of 4, two for runs
// of 8); its resources start at the first of them, and a lane's offset is
// replaced by one far past the range when its pixel lies outside the strip,
// the frame or the band, which makes the hardware drop the store.  No branch
// guards a store, so the compiler counts every one of them as issued.
// ---------------------------------------------------------------------------
constexpr int kBufferWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)
constexpr uint32_t kDropOffset = 0x80000000u;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int ROWS>
struct RowOut {
  __amdgpu_buffer_rsrc_t n0, n1, n2, d, r, st;
  int base;  // this lane's row within the wave's rows, times W

  __device__ static __amdgpu_buffer_rsrc_t rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, int(bytes), kBufferWord3);
  }
  // hj: this lane's row of the round; nr: rows of the round inside the band
  __device__ RowOut(const FitArgs& a, int yg, int hj, int nr, int ox0, int& cols) {
    const int h0 = __builtin_amdgcn_readfirstlane(hj);
    const int64_t p = int64_t(min(yg + h0, a.H - 1)) * a.W + ox0;
    const uint32_t n = uint32_t(ROWS) * uint32_t(a.W);
    n0 = rsrc(a.normals + p, 4 * n);
    n1 = rsrc(a.normals + a.plane + p, 4 * n);
    n2 = rsrc(a.normals + 2 * a.plane + p, 4 * n);
    d = rsrc(a.offsets + p, 4 * n);
    r = rsrc(a.residuals + p, 4 * n);
    st = a.status ? rsrc(a.status + p, n) : rsrc(a.offsets, 0u);
    base = (hj - h0) * a.W;
    cols = hj < nr ? min(a.tile_w, a.W - ox0) : 0;
  }
  // element offset of strip column c, or the drop offset
  __device__ uint32_t at(int c, int cols) const { return c < cols ? uint32_t(base + c) : kDropOffset; }
  __device__ void put(uint32_t e, const PixelOut& po) const {
    const uint32_t b = e == kDropOffset ? kDropOffset : 4u * e;
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(po.n0), n0, int(b), 0, 0);
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(po.n1), n1, int(b), 0, 0);
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(po.n2), n2, int(b), 0, 0);
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(po.d), d, int(b), 0, 0);
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(po.res), r, int(b), 0, 0);
    __builtin_amdgcn_raw_buffer_store_b8(po.st, st, int(e), 0, 0);
  }
  __device__ static void put4(__amdgpu_buffer_rsrc_t res, uint32_t e, const float* v) {
    const uint32_t b = e == kDropOffset ? kDropOffset : 4u * e;
    const u32x4 w = {__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                     __float_as_uint(v[3])};
    __builtin_amdgcn_raw_buffer_store_b128(w, res, int(b), 0, 0);
  }
};

__device__ inline PixelOut invalid_pixel() {
  PixelOut o;
  const float nan = __builtin_nanf("");
  o.n0 = o.n1 = o.n2 = o.d = o.res = nan;
  o.st = 1;
  o.kappa = nan;
  return o;
}

// Window moments in window-centred coordinates, from which both solves start:
//   Sxw = sum x' w, Syw = sum y' w, Sw = sum w, Sww = sum w^2,
//   V = N sum w^2 - (sum w)^2, SSR = V/N - (Sxw^2 + Syw^2)/S2 (explicit residual).
template <typename S>
struct Moments {
  S Sxw, Syw, Sw, Sww, V, SSR;
};

// Eq. 14 with |(a, b, c)| = 1: eliminating d leaves G = diag(S2, S2, N) - g g^T / Sww
// over gamma = (n_x/fx, n_y/fy, n . (u_c, v_c, 1)); C = M^T G M is the 3x3 in n.
template <typename S>
struct Implicit3 {
  S c00, c01, c02, c11, c12, c22;  // C
  S ifx, ify, uc, vc, iS, Sxw, Syw, Sw, iN;
};

template <typename S>
__device__ inline Implicit3<S> implicit_matrix(const FitArgs& a, const Moments<S>& m, S uc, S vc) {
  Implicit3<S> c;
  const S S2 = S(a.S2);
  const S iS = rcp_nr(m.Sww);
  const S g11 = S2 - m.Sxw * m.Sxw * iS, g22 = S2 - m.Syw * m.Syw * iS;
  const S g12 = -m.Sxw * m.Syw * iS, g13 = -m.Sxw * m.Sw * iS, g23 = -m.Syw * m.Sw * iS;
  const S g33 = m.V * iS;
  const S ifx = S(a.inv_fx), ify = S(a.inv_fy);
  c.c00 = g11 * ifx * ifx + S(2) * g13 * uc * ifx + g33 * uc * uc;
  c.c01 = g12 * ifx * ify + g13 * vc * ifx + g23 * uc * ify + g33 * uc * vc;
  c.c02 = g13 * ifx + g33 * uc;
  c.c11 = g22 * ify * ify + S(2) * g23 * vc * ify + g33 * vc * vc;
  c.c12 = g23 * ify + g33 * vc;
  c.c22 = g33;
  c.ifx = ifx; c.ify = ify; c.uc = uc; c.vc = vc; c.iS = iS;
  c.Sxw = m.Sxw; c.Syw = m.Syw; c.Sw = m.Sw; c.iN = S(a.inv_N);
  return c;
}

// Orientation (d >= 0), offset, residual sqrt(l1 / N), kappa and its status flag
// from the smallest eigenpair e (computed in E arithmetic) of C (S arithmetic).
template <typename S, typename E>
__device__ inline void finish_implicit(const FitArgs& a, const Implicit3<S>& c, const Eig3<E>& e,
                                       PixelOut& o, bool want_kappa) {
  S n0 = S(e.n[0]), n1 = S(e.n[1]), n2 = S(e.n[2]);
  const S gp = n0 * c.ifx, gq = n1 * c.ify, gt = n0 * c.uc + n1 * c.vc + n2;
  S d = -(gp * c.Sxw + gq * c.Syw + gt * c.Sw) * c.iS;
  if (facing_flip(d, n0, n1, n2)) {
    d = -d; n0 = -n0; n1 = -n1; n2 = -n2;
  }
  d = d + S(0);  // no negative zero
  o.n0 = float(n0);
  o.n1 = float(n1);
  o.n2 = float(n2);
  o.d = float(d);
  o.res = sqrt_out(float(fmax(S(e.l1), S(0)) * c.iN));
  o.kappa = 0.0f;
  if (want_kappa) {
    const E gap = e.l2 - e.l1;
    o.kappa = (e.degenerate || !(gap > E(0))) ? __builtin_inff() : float(e.l3 / gap);
    if (a.kappa_flag > 0.0 && !(o.kappa <= float(a.kappa_flag))) o.st |= 2;
  }
}

// ---------------------------------------------------------------------------
// FP64 implicit solve (Eq. 14 with |(a, b, c)| = 1), the hot path's solve.
//
// G is taken scaled by sum w^2, G' = Sww G = Sww diag(S2, S2, N) - g g^T with
// g = (Sxw, Syw, Sw), so no reciprocal is needed before the offset; eigenvectors
// are unchanged and eigenvalues scale by Sww.  C = M^T G' M in the normal's
// coordinates.  FP64 has the range for these sums at every supported depth
// (1e-3 .. 1e3, k <= 63), so there is no power-of-two scaling.
//
// Smallest eigenvalue: Halley's iteration on det(C - l I), convex and
// decreasing below l1, so iterates started below l1 rise monotonically.  C is
// semidefinite, so 0 lies below l1, and the first iterate is the Halley step
// from 0: c0 c1 / (c1^2 - c0 c2), which is tighter than Newton's c0/c1.
// Halley's error obeys e' ~ e^3 / gap^2 with gap = l2 - l1 >= -f'(l)/(c2 - 3l),
// so the loop stops once a step s has s (c2 - 3l) <= 1e-3 (-f'(l)): the
// remaining error is then below 1e-9 of the gap (measured on the workload
// frames: at most 1.2e-9 rad from the converged eigenvector, against 6e-8 for
// the float rounding of the output), or on a step below 1e-13 c2.
//
// Eigenvector: the column of adj(C - l1 I) with the largest diagonal entry.
// adj(C - l I) = sum_k prod_{j != k} (l_j - l) e_k e_k^T is positive
// semidefinite for l <= l1 and its e_1 weight dominates, so every column is
// parallel to e_1 at l = l1 and the largest diagonal picks a column with
// |e_1j|^2 >= 1/3.  Each column is the cross product of two rows of C - l I
// (the approach of J. Kopp, 2008, for symmetric 3x3 eigenvectors).
// Accuracy of the normal ~ eps * l3 / (l2 - l1).
// ---------------------------------------------------------------------------
__device__ inline PixelOut solve_implicit_fp64(const FitArgs& a, const Moments<double>& m,
                                               double uc, double vc, bool want_kappa) {
  PixelOut o;
  o.st = 0;
  o.kappa = 0.0f;
  const double S2 = a.S2, ifx = a.inv_fx, ify = a.inv_fy;
  const double g11 = fma(S2, m.Sww, -m.Sxw * m.Sxw), g22 = fma(S2, m.Sww, -m.Syw * m.Syw);
  const double g33 = m.V;
  const double g12 = -m.Sxw * m.Syw, g13 = -m.Sxw * m.Sw, g23 = -m.Syw * m.Sw;
  const double c02 = fma(ifx, g13, uc * g33), c12 = fma(ify, g23, vc * g33), c22 = g33;
  const double c00 = fma(ifx, fma(ifx, g11, uc * g13), uc * c02);
  const double c01 = fma(ifx, fma(ify, g12, vc * g13), uc * c12);
  const double c11 = fma(ify, fma(ify, g22, vc * g23), vc * c12);
  // det(C - l I) = -l^3 + c2 l^2 - c1 l + c0
  const double m00 = c11 * c22 - c12 * c12, m11 = c00 * c22 - c02 * c02;
  const double m22 = c00 * c11 - c01 * c01;
  const double c2 = c00 + c11 + c22, c1 = m00 + m11 + m22;
  const double c0 = c00 * m00 + c01 * (c02 * c12 - c01 * c22) + c02 * (c01 * c12 - c02 * c11);
  // One Halley step from l; `done` once a guard fails or the stopping rule
  // holds (then l stays).  Below l1 every factor l_i - l is positive, so
  // f > 0, f' < 0 and 2 f'^2 - f f'' > 0 there and the step rises; from a
  // point that rounding put past l1 (f < 0, f' < 0) it would fall, so the
  // rising-step guard alone stops the iteration there.  The step's
  // reciprocal needs no refinement: an error of relative size e in a step of
  // size s leaves e s, which the next step removes.
  const double tol = 1e-13 * c2;
  auto halley = [&](double& l, bool& done) {
    const double f = fma(fma(c2 - l, l, -c1), l, c0);
    const double fp = fma(fma(-3.0, l, 2.0 * c2), l, -c1);
    const double fpp = fma(-6.0, l, 2.0 * c2);
    const double den = fma(2.0 * fp, fp, -f * fpp);
    const double ln = l - 2.0 * f * fp * rcp_raw(den);
    const bool ok = !done && den > 0.0 && ln > l;
    const double step = ln - l;
    done = !ok || step <= tol || step * (c2 - 3.0 * ln) <= -1e-3 * fp;
    l = ok ? ln : l;
  };
  const double hden = fma(c1, c1, -c0 * c2);  // >= 2 c1^2 / 3 for real roots
  const bool start = c0 > 0.0 && c1 > 0.0 && hden > 0.0;
  double l = start ? c0 * c1 * rcp_nr(hden) : 0.0;
  bool done = !start;
  // almost every window takes two steps: straight-line code, then a loop for
  // the rest
  halley(l, done);
  halley(l, done);
  for (int it = 2; it < 24 && !done; ++it) halley(l, done);
  const double a00 = c00 - l, a11 = c11 - l, a22 = c22 - l;
  const double k00 = a11 * a22 - c12 * c12, k11 = a00 * a22 - c02 * c02, k22 = a00 * a11 - c01 * c01;
  const double q01 = c02 * c12 - c01 * a22, q02 = c01 * c12 - c02 * a11;
  const double q12 = c01 * c02 - a00 * c12;
  double vx = k00, vy = q01, vz = q02, best = k00;
  if (k11 > best) { vx = q01; vy = k11; vz = q12; best = k11; }
  if (k22 > best) { vx = q02; vy = q12; vz = k22; best = k22; }
  double nn = vx * vx + vy * vy + vz * vz;
  bool degenerate = false;
  if (!(best > 0.0) || !(nn > 0.0) || !isfinite(nn)) {
    // l1 has multiplicity >= 2 (or the window is flat in every direction): any
    // vector orthogonal to the largest row of C - l I
    double rx = a00, ry = c01, rz = c02;
    double rn = rx * rx + ry * ry + rz * rz;
    const double r1n = c01 * c01 + a11 * a11 + c12 * c12;
    if (r1n > rn) { rx = c01; ry = a11; rz = c12; rn = r1n; }
    const double r2n = c02 * c02 + c12 * c12 + a22 * a22;
    if (r2n > rn) { rx = c02; ry = c12; rz = a22; rn = r2n; }
    if (rn > 0.0) {
      if (fabs(rx) <= fabs(ry) && fabs(rx) <= fabs(rz)) { vx = 0.0; vy = rz; vz = -ry; }
      else if (fabs(ry) <= fabs(rz)) { vx = -rz; vy = 0.0; vz = rx; }
      else { vx = ry; vy = -rx; vz = 0.0; }
    } else {
      vx = 0.0; vy = 0.0; vz = 1.0;
    }
    nn = vx * vx + vy * vy + vz * vz;
    degenerate = true;
  }
  // one inverse square root gives both 1/|v| and 1/Sww (the uncentred sum of
  // w^2, positive in every valid window): r = 1 / (|v| Sww)
  const double r = rsq_nr(nn * (m.Sww * m.Sww));
  const double inv = r * m.Sww;
  double n0 = vx * inv, n1 = vy * inv, n2 = vz * inv;
  const double iS = (r * r) * (nn * m.Sww);
  double d = -fma(n0 * ifx, m.Sxw, fma(n1 * ify, m.Syw, fma(n0, uc, fma(n1, vc, n2)) * m.Sw)) * iS;
  if (facing_flip(d, n0, n1, n2)) {
    d = -d; n0 = -n0; n1 = -n1; n2 = -n2;
  }
  d = d + 0.0;  // no negative zero
  o.n0 = float(n0);
  o.n1 = float(n1);
  o.n2 = float(n2);
  o.d = float(d);
  o.res = sqrt_out(float(fmax(l, 0.0) * iS * a.inv_N));
  if (want_kappa) {
    // the other two eigenvalues by deflating the characteristic cubic:
    // l2 + l3 = c2 - l1, l2 l3 = c1 - l1 (l2 + l3)
    const double t = c2 - l;
    const double pr = c1 - l * t;
    const double disc = t * t - 4.0 * pr;
    const double l3 = 0.5 * (t + (disc > 0.0 ? sqrt(disc) : 0.0));
    const double l2 = l3 > 0.0 ? pr / l3 : 0.0;
    const double gap = l2 - l;
    o.kappa = (degenerate || !(gap > 0.0)) ? __builtin_inff() : float(l3 / gap);
    if (a.kappa_flag > 0.0 && !(o.kappa <= float(a.kappa_flag))) o.st |= 2;
  }
  return o;
}

// ---------------------------------------------------------------------------
// The implicit fit with the constraint exactly as Sec. II-A states it,
// |(a, b, c, d)| = 1: the eigenvector of the smallest eigenvalue of the 4x4
// scatter of the monomials [u, v, 1, w] (Eq. 14), assembled here from the
// window's centred moments and the closed-form camera block.  FP64.
//   f(l) = det(S - l I) = (l1 - l)(l2 - l)(l3 - l)(l4 - l) is positive,
//   decreasing and convex on (-inf, l1], and c0/c1 = 1/sum(1/li) <= l1, so
//   Halley's iteration from c0/c1 climbs to l1 as for the 3x3.  The eigenvector
//   is the best-conditioned generalised cross product of three rows of S - l1 I
//   (the cofactors of a 3x4 block).
// ---------------------------------------------------------------------------
__device__ inline double det3g(const double* r0, const double* r1, const double* r2, int skip) {
  int c[3], n = 0;
  for (int j = 0; j < 4; ++j)
    if (j != skip) c[n++] = j;
  return r0[c[0]] * (r1[c[1]] * r2[c[2]] - r1[c[2]] * r2[c[1]]) -
         r0[c[1]] * (r1[c[0]] * r2[c[2]] - r1[c[2]] * r2[c[0]]) +
         r0[c[2]] * (r1[c[0]] * r2[c[1]] - r1[c[1]] * r2[c[0]]);
}

__device__ inline PixelOut solve_literal(const FitArgs& a, const Moments<double>& m, double uc,
                                         double vc) {
  PixelOut o;
  o.st = 0;
  o.kappa = 0.0f;
  const double N = a.N, S2 = a.S2, ifx = a.inv_fx, ify = a.inv_fy;
  double S[4][4];
  S[0][0] = N * uc * uc + S2 * ifx * ifx;
  S[0][1] = N * uc * vc;
  S[0][2] = N * uc;
  S[0][3] = uc * m.Sw + m.Sxw * ifx;
  S[1][1] = N * vc * vc + S2 * ify * ify;
  S[1][2] = N * vc;
  S[1][3] = vc * m.Sw + m.Syw * ify;
  S[2][2] = N;
  S[2][3] = m.Sw;
  S[3][3] = m.Sww;
  const double sc = fmax(fmax(S[0][0], S[1][1]), fmax(S[2][2], S[3][3]));
  const double is = ldexp(1.0, -ilogb(sc));
  double B[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = i; j < 4; ++j) B[i][j] = B[j][i] = S[i][j] * is;
  // characteristic polynomial l^4 - c3 l^3 + c2 l^2 - c1 l + c0
  const double c3 = B[0][0] + B[1][1] + B[2][2] + B[3][3];
  double c2 = 0.0;
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j) c2 += B[i][i] * B[j][j] - B[i][j] * B[i][j];
  double c1 = 0.0;
  for (int r = 0; r < 4; ++r) {  // principal 3x3 minors: drop row and column r
    const int i = r == 0 ? 1 : 0, j = r <= 1 ? 2 : 1, k = r <= 2 ? 3 : 2;
    c1 += det3(B[i][i], B[i][j], B[i][k], B[j][j], B[j][k], B[k][k]);
  }
  const double c0 = B[0][0] * det3g(B[1], B[2], B[3], 0) - B[0][1] * det3g(B[1], B[2], B[3], 1) +
                    B[0][2] * det3g(B[1], B[2], B[3], 2) - B[0][3] * det3g(B[1], B[2], B[3], 3);
  double l = 0.0;
  if (c0 > 0.0 && c1 > 0.0) {
    l = c0 * rcp_nr(c1);
    for (int it = 0; it < 32; ++it) {
      const double f = (((l - c3) * l + c2) * l - c1) * l + c0;
      const double fp = ((4.0 * l - 3.0 * c3) * l + 2.0 * c2) * l - c1;
      const double fpp = (12.0 * l - 6.0 * c3) * l + 2.0 * c2;
      if (!(f > 0.0) || !(fp < 0.0)) break;
      const double den = 2.0 * fp * fp - f * fpp;
      if (!(den > 0.0)) break;
      const double ln = l - 2.0 * f * fp * rcp_raw(den);
      if (!(ln > l)) break;
      const double step = ln - l;
      l = ln;
      if (step <= 1e-14) break;
    }
  }
  double A[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) A[i][j] = B[i][j] - (i == j ? l : 0.0);
  double v[4] = {0.0, 0.0, 0.0, 1.0}, best = 0.0;
  for (int r = 0; r < 4; ++r) {  // drop row r, cofactors of the remaining 3x4 block
    const double* q0 = A[r == 0 ? 1 : 0];
    const double* q1 = A[r <= 1 ? 2 : 1];
    const double* q2 = A[r <= 2 ? 3 : 2];
    double t[4];
    double nn = 0.0;
    for (int j = 0; j < 4; ++j) {
      t[j] = ((j & 1) ? -1.0 : 1.0) * det3g(q0, q1, q2, j);
      nn += t[j] * t[j];
    }
    if (nn > best) {
      best = nn;
      for (int j = 0; j < 4; ++j) v[j] = t[j];
    }
  }
  const double sn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  double n0 = v[0] / sn, n1 = v[1] / sn, n2 = v[2] / sn, d = v[3] / sn;
  if (facing_flip(d, n0, n1, n2)) {
    d = -d; n0 = -n0; n1 = -n1; n2 = -n2;
  }
  // residual: S a = l1 a for the unit 4-vector a = v/|v|, so the sum of squares
  // of n.(u, v, 1) + d w is l1 |v|^2 / sn^2
  const double vn2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3];
  const double l1 = ldexp(fmax(l, 0.0), ilogb(sc));
  o.n0 = float(n0);
  o.n1 = float(n1);
  o.n2 = float(n2);
  o.d = float(d);
  o.res = float(sqrt(l1 * vn2 / (sn * sn) * a.inv_N));
  return o;
}

template <typename S, int MODE>
__device__ inline PixelOut solve_moments(const FitArgs& a, const Moments<S>& m, int x0, int y0) {
  PixelOut o;
  o.st = 0;
  o.kappa = 0.0f;
  const S iN = S(a.inv_N), iS2 = S(a.inv_S2);
  const S uc = (S(x0) - S(a.cx)) * S(a.inv_fx);
  const S vc = (S(y0) - S(a.cy)) * S(a.inv_fy);
  if constexpr (MODE == PF_IMPLICIT_LITERAL) {
    return solve_literal(a, m, uc, vc);
  } else if (MODE == PF_EXPLICIT) {
    // Eq. 15 in centred regressors (x', y', 1): a' = Sxw/S2, b' = Syw/S2, c' = Sw/N;
    // with the cancellation-prone differences already formed, single precision suffices.
    const float ap = float(m.Sxw * iS2), bp = float(m.Syw * iS2), cp = float(m.Sw * iN);
    const float aa = float(a.fx) * ap, bb = float(a.fy) * bp;
    const float cc = cp - aa * float(uc) - bb * float(vc);
    const float inv = rsq_nr(aa * aa + bb * bb + cc * cc);
    o.n0 = -aa * inv;
    o.n1 = -bb * inv;
    o.n2 = -cc * inv;
    o.d = inv;
    o.res = inv * sqrt_out(fmaxf(float(m.SSR), 0.0f) * float(a.inv_N));
  } else if constexpr (std::is_same<S, double>::value) {
    return solve_implicit_fp64(a, m, uc, vc, a.kappa_flag > 0.0);
  } else {
    const Implicit3<S> c = implicit_matrix<S>(a, m, uc, vc);
    const bool flag = a.kappa_flag > 0.0;
    finish_implicit<S, S>(a, c, smallest_eig<S>(c.c00, c.c01, c.c02, c.c11, c.c12, c.c22, flag),
                          o, flag);
  }
  return o;
}

// Per-pixel solve from the window sums (FP32 or FP64 arithmetic throughout).
//   B  = sum (w - w_ref)                 Sxw = sum (x - x_c)(w - w_ref)
//   Syw = sum (y - y_c)(w - w_ref)       Q  = sum (w - w_ref)^2
// where x_c, y_c are the window centre's column and row; w = 1/Z.
template <typename T, int MODE>
__device__ inline PixelOut solve_pixel(const FitArgs& a, T B, T Sxw, T Syw, T Q, int cnt,
                                       T w_ref, int x0, int y0) {
  if (cnt != a.k * a.k) return invalid_pixel();
  const T Nt = T(a.N);
  Moments<T> m;
  m.Sxw = Sxw;
  m.Syw = Syw;
  m.V = Nt * Q - B * B;                          // N sum (w - mean w)^2, reference-free
  m.Sw = Nt * w_ref + B;                          // sum w
  m.Sww = Q + w_ref * (T(2) * B + Nt * w_ref);    // sum w^2
  m.SSR = m.V * T(a.inv_N) - (Sxw * Sxw + Syw * Syw) * T(a.inv_S2);
  return solve_moments<T, MODE>(a, m, x0, y0);
}

// Partial windows (FP64): the window is fitted from its Nv valid pixels, whose
// camera-only moments are no longer the closed-form diagonal: with window
// coordinates (x', y') over the valid pixels, P = sum [x' y' 1]^T [x' y' 1] =
// [[Sxx, Sxy, Sx], [Sxy, Syy, Sy], [Sx, Sy, Nv]] (exact integers).  The window
// is valid iff Nv >= max(min_valid, 3) and the valid pixels are not collinear,
// i.e. D = (Nv Sxx - Sx^2)(Nv Syy - Sy^2) - (Nv Sxy - Sx Sy)^2 > 0; D is formed
// from exact integer factors with a fused difference of products (Kahan), so a
// collinear set gives exactly 0.  The data moments carry the hat-disparity
// sums: sum x' w = Sxw^ + w_ref Sx since sum x' no longer vanishes.
struct PartialSums {
  double Nv, Sx, Sy, Sxx, Sxy, Syy;
};

template <int MODE>
__device__ inline PixelOut solve_partial(const FitArgs& a, const PartialSums& c, double B,
                                         double Sxw_h, double Syw_h, double Q, double w_ref,
                                         int x0, int y0) {
  const double Nv = c.Nv;
  if (!(Nv >= double(a.min_valid) && Nv >= 3.0)) return invalid_pixel();
  const double a1 = Nv * c.Sxx - c.Sx * c.Sx, b1 = Nv * c.Syy - c.Sy * c.Sy;
  const double c1 = Nv * c.Sxy - c.Sx * c.Sy;
  const double p = c1 * c1;
  const double D = fma(a1, b1, -p) - fma(c1, c1, -p);
  if (!(D > 0.5)) return invalid_pixel();
  const double uc = (double(x0) - a.cx) * a.inv_fx, vc = (double(y0) - a.cy) * a.inv_fy;
  PixelOut o;
  o.st = 0;
  o.kappa = 0.0f;
  if (MODE == PF_EXPLICIT) {
    // regress w^ = w - w_ref on (x', y', 1): P alpha^ = (Sxw^, Syw^, B); alpha' = alpha^ + w_ref e3
    const double p00 = c.Sxx, p01 = c.Sxy, p02 = c.Sx, p11 = c.Syy, p12 = c.Sy, p22 = Nv;
    const double k00 = p11 * p22 - p12 * p12, k01 = p02 * p12 - p01 * p22, k02 = p01 * p12 - p02 * p11;
    const double k11 = p00 * p22 - p02 * p02, k12 = p01 * p02 - p00 * p12, k22 = p00 * p11 - p01 * p01;
    const double idet = 1.0 / (p00 * k00 + p01 * k01 + p02 * k02);
    const double ah = (k00 * Sxw_h + k01 * Syw_h + k02 * B) * idet;
    const double bh = (k01 * Sxw_h + k11 * Syw_h + k12 * B) * idet;
    const double ch = (k02 * Sxw_h + k12 * Syw_h + k22 * B) * idet;
    const double ax = a.fx * ah, ay = a.fy * bh;
    const double az = (ch + w_ref) - ax * uc - ay * vc;
    const double rho = sqrt(ax * ax + ay * ay + az * az);
    const double ssr = fmax(Q - (ah * Sxw_h + bh * Syw_h + ch * B), 0.0);
    o.n0 = float(-ax / rho);
    o.n1 = float(-ay / rho);
    o.n2 = float(-az / rho);
    o.d = float(1.0 / rho);
    o.res = float(sqrt(ssr / Nv) / rho);
    return o;
  } else {
    const double Sw = Nv * w_ref + B;
    const double Sww = Q + w_ref * (2.0 * B + Nv * w_ref);
    const double Sxw = Sxw_h + w_ref * c.Sx, Syw = Syw_h + w_ref * c.Sy;
    const double iS = rcp_nr(Sww);
    const double g11 = c.Sxx - Sxw * Sxw * iS, g22 = c.Syy - Syw * Syw * iS;
    const double g12 = c.Sxy - Sxw * Syw * iS, g13 = c.Sx - Sxw * Sw * iS;
    const double g23 = c.Sy - Syw * Sw * iS, g33 = (Nv * Q - B * B) * iS;
    const double ifx = a.inv_fx, ify = a.inv_fy;
    Implicit3<double> m;
    m.c00 = g11 * ifx * ifx + 2.0 * g13 * uc * ifx + g33 * uc * uc;
    m.c01 = g12 * ifx * ify + g13 * vc * ifx + g23 * uc * ify + g33 * uc * vc;
    m.c02 = g13 * ifx + g33 * uc;
    m.c11 = g22 * ify * ify + 2.0 * g23 * vc * ify + g33 * vc * vc;
    m.c12 = g23 * ify + g33 * vc;
    m.c22 = g33;
    m.ifx = ifx; m.ify = ify; m.uc = uc; m.vc = vc; m.iS = iS;
    m.Sxw = Sxw; m.Syw = Syw; m.Sw = Sw; m.iN = 1.0 / Nv;
    const bool flag = a.kappa_flag > 0.0;
    finish_implicit<double, double>(
        a, m, smallest_eig<double>(m.c00, m.c01, m.c02, m.c11, m.c12, m.c22, flag), o, flag);
    return o;
  }
}

// Compensated path: moments formed in two-float arithmetic, solved in FP32;
// an implicit window whose FP32 eigen-condition kappa exceeds the plan's
// threshold is solved again in FP64 from the same two-float moments (status
// bit 2 records it).
template <int MODE>
__device__ inline PixelOut solve_pixel_df(const FitArgs& a, df32 B, df32 Sxw, df32 Syw, df32 Q,
                                          int cnt, df32 w_ref, int x0, int y0) {
  if (cnt != a.k * a.k) return invalid_pixel();
  const df32 Nt(float(a.k * a.k));
  const df32 V = Nt * Q - B * B;
  const df32 Sw = Nt * w_ref + B;
  const df32 Sww = Q + w_ref * (B + B + Nt * w_ref);
  const df32 iS2 = to_df32(a.inv_S2), iN = to_df32(a.inv_N);
  const df32 SSR = V * iN - (Sxw * Sxw + Syw * Syw) * iS2;
  if (MODE == PF_EXPLICIT) {
    Moments<float> mf = {Sxw.hi, Syw.hi, Sw.hi, Sww.hi, V.hi, SSR.hi};
    return solve_moments<float, MODE>(a, mf, x0, y0);
  }
  // Implicit: the 3x3 is formed from the two-float moments in FP64 (C = M^T G M
  // cancels terms up to ~f^2 times larger than its entries), its smallest
  // eigenpair is found in FP32, and windows whose FP32 kappa exceeds the
  // threshold are solved again in FP64.
  const Moments<double> md = {to_double(Sxw), to_double(Syw), to_double(Sw), to_double(Sww),
                              to_double(V), to_double(SSR)};
  const double uc = (double(x0) - a.cx) * a.inv_fx, vc = (double(y0) - a.cy) * a.inv_fy;
  const Implicit3<double> c = implicit_matrix<double>(a, md, uc, vc);
  PixelOut o;
  o.st = 0;
  const Eig3<float> ef = smallest_eig<float>(float(c.c00), float(c.c01), float(c.c02),
                                             float(c.c11), float(c.c12), float(c.c22));
  finish_implicit<double, float>(a, c, ef, o, true);
  {
    // residual from the FP64 Rayleigh quotient n^T C n of the final unit
    // eigenvector: its error is quadratic in the eigenvector's, where l1 from
    // the FP32 characteristic polynomial carries an error ~ eps32 * l3
    const double n0 = ef.n[0], n1 = ef.n[1], n2 = ef.n[2];
    const double rq = n0 * (c.c00 * n0 + c.c01 * n1 + c.c02 * n2) +
                      n1 * (c.c01 * n0 + c.c11 * n1 + c.c12 * n2) +
                      n2 * (c.c02 * n0 + c.c12 * n1 + c.c22 * n2);
    const double nn = n0 * n0 + n1 * n1 + n2 * n2;
    o.res = float(sqrt(fmax(rq / nn, 0.0) * c.iN));
  }
  // The FP32 eigenvector's error (~ eps32 kappa) moves the offset by about
  // |P_c| times that angle, |P_c| ~ |(u_c, v_c, 1)| N / sum w the distance of
  // the window's centre point; re-solve in FP64 where kappa max(1, |P_c| / d)
  // exceeds the threshold, which bounds both errors relative to d.
  const double pc = sqrt(1.0 + uc * uc + vc * vc) * a.N / md.Sw;
  const double amp = fmax(1.0, pc / fabs(double(o.d)));
  if (!(double(o.kappa) * amp <= a.kappa_fp64)) {
    o = solve_implicit_fp64(a, md, uc, vc, a.kappa_flag > 0.0);
    o.st |= 4;
  }
  return o;
}

// ---------------------------------------------------------------------------
// Adjoint of the per-pixel solve (FP64).  Given the upstream gradients of one
// window's outputs (normal, offset, residual) it returns the gradients of the
// four window moments the fit depends on,
//   Sw = sum w, Sx = sum x' w, Sy = sum y' w, Sww = sum w^2,
// which the box-sum adjoint then spreads back over the window's pixels.
// ---------------------------------------------------------------------------
struct MomentGrad {
  double Sw, Sx, Sy, Sww;
};

__device__ inline MomentGrad explicit_adjoint(const FitArgs& a, double Sx, double Sy, double Sw,
                                              double V, double uc, double vc, double gnx,
                                              double gny, double gnz, double gd, double gr) {
  // forward: alpha = (fx Sx/S2, fy Sy/S2, Sw/N - ...), n = -alpha/|alpha|, d = 1/|alpha|,
  // r = d sqrt(SSR/N) with SSR = Sww - Sw^2/N - (Sx^2 + Sy^2)/S2
  const double N = a.N, S2 = a.S2;
  const double ax = a.fx * Sx / S2, ay = a.fy * Sy / S2;
  const double az = Sw / N - ax * uc - ay * vc;
  const double rho = sqrt(ax * ax + ay * ay + az * az);
  const double nx = -ax / rho, ny = -ay / rho, nz = -az / rho, d = 1.0 / rho;
  const double ssr = fmax(V / N - (Sx * Sx + Sy * Sy) / S2, 0.0);
  const double sr = sqrt(ssr / N);
  const double gdt = gd + gr * sr;  // d enters r as a factor
  // dn = -(I - n n^T) dalpha / rho, dd = -alpha^T dalpha / rho^3 = n^T dalpha / rho^2
  const double ng = nx * gnx + ny * gny + nz * gnz;
  const double gax = -(gnx - nx * ng) / rho + gdt * nx / (rho * rho);
  const double gay = -(gny - ny * ng) / rho + gdt * ny / (rho * rho);
  const double gaz = -(gnz - nz * ng) / rho + gdt * nz / (rho * rho);
  const double gssr = sr > 0.0 ? gr * d / (2.0 * sr * N) : 0.0;
  MomentGrad g;
  g.Sx = a.fx * (gax - uc * gaz) / S2 - 2.0 * Sx * gssr / S2;
  g.Sy = a.fy * (gay - vc * gaz) / S2 - 2.0 * Sy * gssr / S2;
  g.Sw = gaz / N - 2.0 * Sw * gssr / N;
  g.Sww = gssr;
  return g;
}

__device__ inline MomentGrad implicit_adjoint(const FitArgs& a, const Moments<double>& m,
                                              double uc, double vc, double gnx, double gny,
                                              double gnz, double gd, double gr) {
  MomentGrad g = {0.0, 0.0, 0.0, 0.0};
  const Implicit3<double> c = implicit_matrix<double>(a, m, uc, vc);
  const Eig3<double> e = smallest_eig<double>(c.c00, c.c01, c.c02, c.c11, c.c12, c.c22);
  if (e.degenerate || !(e.l2 > e.l1)) return g;  // the normal is not differentiable here
  double n0 = e.n[0], n1 = e.n[1], n2 = e.n[2];
  const double gv[3] = {m.Sxw, m.Syw, m.Sw};  // g = (Sx, Sy, Sw)
  double gm0 = n0 * c.ifx, gm1 = n1 * c.ify, gm2 = n0 * uc + n1 * vc + n2;  // gamma = M n
  double d = -(gm0 * gv[0] + gm1 * gv[1] + gm2 * gv[2]) * c.iS;
  if (facing_flip(d, n0, n1, n2)) {
    d = -d; n0 = -n0; n1 = -n1; n2 = -n2; gm0 = -gm0; gm1 = -gm1; gm2 = -gm2;
  }
  const double iS = c.iS, N = a.N;
  const double r = sqrt(fmax(e.l1, 0.0) / N);
  // d = -gamma^T g / Sww depends on n through gamma = M n: dd/dn = -M^T g / Sww
  const double mtg0 = c.ifx * gv[0] + uc * gv[2], mtg1 = c.ify * gv[1] + vc * gv[2];
  const double mtg2 = gv[2];
  double bn0 = gnx - gd * mtg0 * iS, bn1 = gny - gd * mtg1 * iS, bn2 = gnz - gd * mtg2 * iS;
  const double glam = r > 0.0 ? gr / (2.0 * N * r) : 0.0;
  // dn = -(C - l1 I)^+ dC n: y = (C - l1 I + mu n n^T)^-1 b for b orthogonal to n
  const double nb = n0 * bn0 + n1 * bn1 + n2 * bn2;
  bn0 -= n0 * nb; bn1 -= n1 * nb; bn2 -= n2 * nb;
  const double mu = e.l3 - e.l1;
  const double a00 = c.c00 - e.l1 + mu * n0 * n0, a01 = c.c01 + mu * n0 * n1;
  const double a02 = c.c02 + mu * n0 * n2, a11 = c.c11 - e.l1 + mu * n1 * n1;
  const double a12 = c.c12 + mu * n1 * n2, a22 = c.c22 - e.l1 + mu * n2 * n2;
  const double k00 = a11 * a22 - a12 * a12, k01 = a02 * a12 - a01 * a22, k02 = a01 * a12 - a02 * a11;
  const double k11 = a00 * a22 - a02 * a02, k12 = a01 * a02 - a00 * a12, k22 = a00 * a11 - a01 * a01;
  const double det = a00 * k00 + a01 * k01 + a02 * k02;
  if (!(fabs(det) > 0.0)) return g;
  const double idet = 1.0 / det;
  const double y0 = (k00 * bn0 + k01 * bn1 + k02 * bn2) * idet;
  const double y1 = (k01 * bn0 + k11 * bn1 + k12 * bn2) * idet;
  const double y2 = (k02 * bn0 + k12 * bn1 + k22 * bn2) * idet;
  // dL/dC = glam n n^T - sym(y n^T)
  const double n[3] = {n0, n1, n2}, y[3] = {y0, y1, y2};
  double GC[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) GC[i][j] = glam * n[i] * n[j] - 0.5 * (y[i] * n[j] + n[i] * y[j]);
  // C = M^T G M  ->  dL/dG = M dL/dC M^T, with M = [[1/fx,0,0],[0,1/fy,0],[uc,vc,1]]
  const double M[3][3] = {{c.ifx, 0.0, 0.0}, {0.0, c.ify, 0.0}, {uc, vc, 1.0}};
  double T1[3][3], GG[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int t = 0; t < 3; ++t) s += M[i][t] * GC[t][j];
      T1[i][j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int t = 0; t < 3; ++t) s += T1[i][t] * M[j][t];
      GG[i][j] = s;
    }
  // G = diag(S2, S2, N) - g g^T / Sww: dL/dg = -2 dL/dG g / Sww, dL/dSww = g^T dL/dG g / Sww^2;
  // plus the offset's direct terms dd/dg = -gamma / Sww, dd/dSww = -d / Sww
  const double gm[3] = {gm0, gm1, gm2};
  double gg[3], qg = 0.0;
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int t = 0; t < 3; ++t) s += GG[i][t] * gv[t];
    gg[i] = -2.0 * s * iS - gd * gm[i] * iS;
    qg += gv[i] * s;
  }
  g.Sx = gg[0];
  g.Sy = gg[1];
  g.Sw = gg[2];
  g.Sww = qg * iS * iS - gd * d * iS;
  return g;
}

// ---------------------------------------------------------------------------
// The fused kernel.  Workgroup = one strip of kBlock input columns (tile_w
// output columns plus k-1 halo) by one band of tile_h output rows.
//
// Row bookkeeping for output row y0: each thread's column sums hold input rows
// y0-r .. y0+r (row y0+r entered, row y0-r-1 left), i.e. the column window of
// output row y0; the warm-up before the first row of the band enters rows
// yb-r .. yb+r-1.
// ---------------------------------------------------------------------------
// Backward launches give every job a region of 4 H W doubles of the workspace,
// in job order (a uniform scan of the job table).
__device__ inline int64_t bwd_ws_offset(const LaunchArgs& la, int jb) {
  int64_t off = 0;
  for (int i = 0; i < jb; ++i) off += 4 * int64_t(la.jobs[i].H) * la.jobs[i].W;
  return off;
}

// Workgroups per CU the register budget is sized for: the forward sweeps
// (32 KB of LDS) are held to 128 VGPRs so that four waves share a SIMD.
// One column's window sums.  In LDS they are 16-byte records: FP32 keeps the
// four values in one record, FP64 and two-float keep (w, yw) and (ww, n) in
// two arrays of records, so that the lanes of a wave read and write
// consecutive 16-byte words (two LDS instructions per column).
template <typename T>
struct ColumnSums {
  T w, yw, ww;  // sums of w - w_ref, (y - y_ref)(w - w_ref), (w - w_ref)^2
  int n;        // valid samples
};
template <typename T>
struct alignas(16) Pair16 {
  T a, b;
};
// (ww, n) as one 12-byte access to a 16-byte record: narrower accesses at a
// 16-byte lane stride would conflict in the LDS banks
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
static_assert(sizeof(u32x3) == 16, "three-word vectors take 16-byte records");
template <typename T>
__device__ inline u32x3 pack_ww_n(T ww, int n) {
  const uint64_t b = __builtin_bit_cast(uint64_t, ww);
  return u32x3{uint32_t(b), uint32_t(b >> 32), uint32_t(n)};
}
template <typename T>
__device__ inline void unpack_ww_n(u32x3 v, T& ww, int& n) {
  ww = __builtin_bit_cast(T, uint64_t(v.x) | (uint64_t(v.y) << 32));
  n = int(v.z);
}
template <typename T>
struct alignas(16) Col16 {
  T w, yw, ww;
  int n;
};
template <typename T>
constexpr bool kWideSums = sizeof(T) > 4;
static_assert(sizeof(Pair16<double>) == 16 && sizeof(Pair16<df32>) == 16, "FP64 records");
static_assert(sizeof(df32) == 8, "two-float values pack into 64 bits");
static_assert(sizeof(Col16<float>) == 16, "FP32 record");

// workgroups per CU each kernel is compiled for; the implicit adjoint sweep
// runs four per CU (as its LDS allows) with a few spilled registers, which is
// faster than three without
template <typename T, int MODE, bool BWD, bool PARTIAL, int SHAPE = 0>
constexpr int kMinGroups =
    (MODE != PF_IMPLICIT_LITERAL && !PARTIAL && (!BWD || MODE == PF_IMPLICIT))
        ? Tiling<SHAPE>::groups
        : 1;

// Launch-wide parameters of a fit (shared by every frame of a launch).
struct LaunchCommon {
  double kappa_flag, kappa_fp64, dscale;
};

// One workgroup tile: strip `wg % n_strips`, band `wg / n_strips` of frame
// `job`.  Called once per workgroup by fit_planes_fused and once per work item
// by the persistent fit_planes_queued, which share every instruction of it.
template <typename T, int MODE, bool MASK, bool BWD = false, bool PARTIAL = false,
          int SHAPE = 0>
__device__ __forceinline__ void fit_tile(const Job& job, int wg, const LaunchCommon& lc,
                                         double* gws) {
  static_assert(!PARTIAL || (std::is_same<T, double>::value && !BWD && MODE != PF_IMPLICIT_LITERAL),
                "partial windows: FP64 forward, implicit or explicit");
  using TL = Tiling<SHAPE>;
  FitArgs a;
  a.depth = job.depth;
  a.mask = job.mask;
  a.normals = job.normals;
  a.offsets = job.offsets;
  a.residuals = job.residuals;
  a.status = job.status;
  a.depth_pitch = job.depth_pitch;
  a.mask_pitch = job.mask_pitch;
  a.H = job.H;
  a.W = job.W;
  a.plane = int64_t(job.H) * job.W;
  a.k = job.k;
  a.r = job.k / 2;
  a.tile_w = job.tile_w;
  a.tile_h = job.tile_h;
  a.n_strips = job.n_strips;
  a.n_bands = (job.H + job.tile_h - 1) / job.tile_h;
  a.fx = job.fx;
  a.fy = job.fy;
  a.cx = job.cx;
  a.cy = job.cy;
  a.inv_fx = 1.0 / job.fx;
  a.inv_fy = 1.0 / job.fy;
  a.N = double(job.k) * job.k;
  a.inv_N = 1.0 / a.N;
  a.S2 = a.N * (a.N - 1.0) / 12.0;
  a.inv_S2 = 1.0 / a.S2;
  a.kappa_flag = lc.kappa_flag;
  a.kappa_fp64 = lc.kappa_fp64;
  a.vec_store = job.vec_store;
  a.gws = gws;
  a.dscale = lc.dscale;
  a.min_valid = job.min_valid;

  // Implicit forward fits with runs of four pack each wave's valid windows
  // before solving them (below), over the wave's own row of column sums.
  constexpr bool PACK =
      !PARTIAL && TL::run == 4 && (BWD ? MODE == PF_IMPLICIT : MODE != PF_EXPLICIT);
  constexpr bool WIDE = kWideSums<T>;
  __shared__ Pair16<T> cs_lo[WIDE ? TL::rows * kPitch : 1];   // (w, yw)
  __shared__ u32x3 cs_hi[WIDE ? TL::rows * kPitch : 1];       // (ww, n)
  __shared__ Col16<T> cs_one[WIDE ? 1 : TL::rows * kPitch];   // FP32: all four
  auto put_col = [&](int idx, const ColumnSums<T>& c) {
    if constexpr (WIDE) {
      Pair16<T> lo;
      lo.a = c.w;
      lo.b = c.yw;
      cs_lo[idx] = lo;
      cs_hi[idx] = pack_ww_n(c.ww, c.n);
    } else {
      Col16<T> r;
      r.w = c.w;
      r.yw = c.yw;
      r.ww = c.ww;
      r.n = c.n;
      cs_one[idx] = r;
    }
  };
  auto get_col = [&](int idx) -> ColumnSums<T> {
    ColumnSums<T> c;
    if constexpr (WIDE) {
      const Pair16<T> lo = cs_lo[idx];
      c.w = lo.a;
      c.yw = lo.b;
      unpack_ww_n(cs_hi[idx], c.ww, c.n);
    } else {
      const Col16<T> r = cs_one[idx];
      c.w = r.w;
      c.yw = r.yw;
      c.ww = r.ww;
      c.n = r.n;
    }
    return c;
  };
  __shared__ int syn[PARTIAL ? TL::rows * kPitch : 1];   // partial windows: sum y~ per column
  __shared__ int sy2n[PARTIAL ? TL::rows * kPitch : 1];  // and sum y~^2
  __shared__ double red[2 * (kBlock / 64)];

  const int tid = threadIdx.x;
  const int strip = wg % a.n_strips;
  const int band = wg / a.n_strips;
  const int ox0 = strip * a.tile_w;        // first output column
  const int ix0 = ox0 - a.r;               // first input column of the strip
  const int x = ix0 + tid;                 // this thread's input column
  const int yb = band * a.tile_h;          // first output row
  const int ye = min(yb + a.tile_h, a.H);  // one past the last output row
  const int y_ref = yb + a.tile_h / 2;
  const bool col_used = tid < a.tile_w + a.k - 1;

  // Every load of the prologue is issued before any is consumed: the reference
  // row, up to kWarm warm-up rows and the first round's rows (the warm-up
  // samples need the reference disparity, whose reduction would otherwise put
  // one memory latency per group of rows on the band's critical path).
  const int nwarm = a.k - 1;  // the column sums first take rows yb-r .. yb+r-1
  constexpr int kWarmGroup = 8, kWarm = 16;
  float zw[kWarm];
  auto issue_warm = [&](int c0) {
#pragma unroll
    for (int g = 0; g < kWarm / kWarmGroup; ++g) {
      if (c0 + g * kWarmGroup < nwarm) {  // uniform
#pragma unroll
        for (int j = 0; j < kWarmGroup; ++j) {
          const int c = c0 + g * kWarmGroup + j;
          zw[g * kWarmGroup + j] = load_depth<MASK>(a, x, yb - a.r + c, col_used && c < nwarm);
        }
      }
    }
  };
  // explicit fits spend a larger share of each band in this prologue (their
  // solve is short): it issues at a raised priority, so its loads go out
  // ahead of the other workgroups' work
  if constexpr (MODE == PF_EXPLICIT) __builtin_amdgcn_s_setprio(2);
  const float zref = load_depth<MASK>(a, x, min(y_ref, a.H - 1), col_used);
  issue_warm(0);
  // depth samples of the current round, loaded one round ahead
  float zl[TL::rows], zg[TL::rows];
#pragma unroll
  for (int j = 0; j < TL::rows; ++j) {
    const int y0 = yb + j;
    zl[j] = load_depth<MASK>(a, x, y0 + a.r, y0 < ye && col_used);
    zg[j] = load_depth<MASK>(a, x, y0 - a.r - 1, y0 < ye && y0 > yb && col_used);
  }

  // Per-tile reference disparity: mean of valid w on the band's middle row.
  double ws = 0.0, wc = 0.0;
  {
    if (depth_valid(zref)) {
      ws = disparity(zref, a.dscale, 0.0);
      wc = 1.0;
    }
    for (int off = 32; off > 0; off >>= 1) {
      ws += __shfl_down(ws, off, 64);
      wc += __shfl_down(wc, off, 64);
    }
    if ((tid & 63) == 0) {
      red[2 * (tid >> 6)] = ws;
      red[2 * (tid >> 6) + 1] = wc;
    }
    __syncthreads();
    ws = 0.0;
    wc = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) {
      ws += red[2 * i];
      wc += red[2 * i + 1];
    }
  }
  T w_ref;
  if constexpr (std::is_same<T, df32>::value)
    w_ref = wc > 0.0 ? to_df32(ws / wc) : df32(0.0f);
  else
    w_ref = wc > 0.0 ? T(ws / wc) : T(0);

  // column window sums, slid down the band: a row enters at the bottom as the
  // row r + 1 above leaves (the four-corner difference of the column integral
  // image, up to rounding order, without carrying its two prefix sums)
  Cursor<T> col;
  col.clear();
  for (int c0 = 0; c0 < nwarm; c0 += kWarm) {
    if (c0 > 0) issue_warm(c0);  // windows above kWarm + 1 rows only
#pragma unroll
    for (int j = 0; j < kWarm; ++j) {
      const int c = c0 + j;
      if (c < nwarm) add_sample<T, PARTIAL>(zw[j], yb - a.r + c, w_ref, y_ref, col, a.dscale);
    }
  }
  if constexpr (MODE == PF_EXPLICIT) __builtin_amdgcn_s_setprio(0);

  const int li = lds_index<SHAPE>(tid);
  // row of the round this thread fits in the horizontal phase (runs of four:
  // one row per wave, so a wave-uniform value)
  const int hj = TL::run == 4 ? __builtin_amdgcn_readfirstlane(tid / (kBlock / TL::run))
                              : tid / (kBlock / TL::run);
  const int run = tid % (kBlock / TL::run);
  const int o0s = run * TL::run;   // first output column (strip-relative) of the run
  // Forward launches run the horizontal phase on every lane: a lane whose run
  // lies past the strip computes the strip's last run again, and its stores
  // land outside the row's buffer range, which the hardware drops.
  const int o0 = (BWD && !PACK) ? o0s : min(o0s, (a.tile_w - 1) / TL::run * TL::run);
  const int o1 = min(o0 + TL::run, a.tile_w);
  const bool vec_store = __builtin_amdgcn_readfirstlane(a.vec_store) != 0;  // uniform per job

  for (int yg = yb; yg < ye; yg += TL::rows) {
    const int nr = min(TL::rows, ye - yg);
    // vertical phase: window column sums for nr output rows.  Rows of the
    // round past the band get empty sums: forward launches run their
    // horizontal phase too (see below), which then sees all-invalid windows
    // rather than stale or never-written LDS.
#pragma unroll
    for (int j = 0; j < TL::rows; ++j) {
      if (j < nr) {
        const int y0 = yg + j;
        if (y0 > yb) sub_sample<T, PARTIAL>(zg[j], y0 - a.r - 1, w_ref, y_ref, col, a.dscale);
        add_sample<T, PARTIAL>(zl[j], y0 + a.r, w_ref, y_ref, col, a.dscale);
        ColumnSums<T> c;
        c.w = col.w;
        c.yw = col.yw;
        c.ww = col.ww;
        c.n = col.n;
        put_col(j * kPitch + li, c);
        if (PARTIAL) {
          syn[j * kPitch + li] = col.yn;
          sy2n[j * kPitch + li] = col.y2n;
        }
      } else if (!BWD || PACK) {
        ColumnSums<T> c;
        c.w = c.yw = c.ww = T(0);
        c.n = 0;
        put_col(j * kPitch + li, c);
        if (PARTIAL) {
          syn[j * kPitch + li] = 0;
          sy2n[j * kPitch + li] = 0;
        }
      }
    }
    // issue the next round's loads now; they land while the horizontal phase runs
    {
      const int yn = yg + TL::rows;
#pragma unroll
      for (int j = 0; j < TL::rows; ++j) {
        const int y0 = yn + j;
        zl[j] = load_depth<MASK>(a, x, y0 + a.r, y0 < ye && col_used);
        zg[j] = load_depth<MASK>(a, x, y0 - a.r - 1, y0 < ye && col_used);
      }
    }
    __syncthreads();
    // horizontal phase: a run of TL::run outputs along one row (forward
    // launches: every lane of every row, see above; a row past the band reads
    // stale column sums and stores nothing)
    if ((BWD && !PACK) ? (hj < nr && o0 < o1) : true) {
      const int y0 = yg + hj;
      const int rc = hj * kPitch;  // first record of this thread's row
      const int base = o0 + a.r;  // x - x_c = (i - base) - (o - o0)
      // window sums slid along the run: column o + k - 1 enters as column o leaves
      T hw = T(0), hx = T(0), hy = T(0), hww = T(0);
      int hn = 0;
      // partial windows: valid-pixel sums of x~, x~^2, y~, x~ y~, y~^2 (x~ = i - base)
      int hxn = 0, hx2n = 0, hyn = 0, hxyn = 0, hy2n = 0;
      auto enter = [&](int i) {
        const int l = lds_index<SHAPE>(i);
        const ColumnSums<T> v = get_col(rc + l);
        hw += v.w;
        hx += T(i - base) * v.w;
        hy += v.yw;
        hww += v.ww;
        hn += v.n;
        if (PARTIAL) {
          const int dx = i - base, n = v.n, yn = syn[hj * kPitch + l];
          hxn += dx * n;
          hx2n += dx * dx * n;
          hyn += yn;
          hxyn += dx * yn;
          hy2n += sy2n[hj * kPitch + l];
        }
      };
      auto leave = [&](int i) {
        const int l = lds_index<SHAPE>(i);
        const ColumnSums<T> v = get_col(rc + l);
        hw = hw - v.w;
        hx = hx - T(i - base) * v.w;
        hy = hy - v.yw;
        hww = hww - v.ww;
        hn -= v.n;
        if (PARTIAL) {
          const int dx = i - base, n = v.n, yn = syn[hj * kPitch + l];
          hxn -= dx * n;
          hx2n -= dx * dx * n;
          hyn -= yn;
          hxyn -= dx * yn;
          hy2n -= sy2n[hj * kPitch + l];
        }
      };
#pragma unroll 4
      for (int i = o0; i < o0 + a.k - 1; ++i) enter(i);
      // one output: column o + k - 1 enters, take the window sums, solve, column o leaves
      auto step = [&](int q) -> PixelOut {
        const int o = o0 + q;
        enter(o + a.k - 1);
        const T B = hw;
        const T Q = hww;
        const int cnt = hn;
        const T Sxw = hx - T(q) * B;
        const T Syw = hy - T(y0 - y_ref) * B;
        PixelOut po;
        if constexpr (PARTIAL) {
          // re-centre the valid-pixel sums to the window: x' = x~ - q, y' = y~ - dy
          const double qd = double(q), dy = double(y0 - y_ref), nv = double(cnt);
          PartialSums ps;
          ps.Nv = nv;
          ps.Sx = double(hxn) - qd * nv;
          ps.Sy = double(hyn) - dy * nv;
          ps.Sxx = double(hx2n) - 2.0 * qd * double(hxn) + qd * qd * nv;
          ps.Syy = double(hy2n) - 2.0 * dy * double(hyn) + dy * dy * nv;
          ps.Sxy = double(hxyn) - dy * double(hxn) - qd * double(hyn) + qd * dy * nv;
          po = solve_partial<MODE>(a, ps, B, Sxw, Syw, Q, w_ref, ox0 + o, y0);
        } else if constexpr (std::is_same<T, df32>::value) {
          po = solve_pixel_df<MODE>(a, B, Sxw, Syw, Q, cnt, w_ref, ox0 + o, y0);
        } else {
          po = solve_pixel<T, MODE>(a, B, Sxw, Syw, Q, cnt, w_ref, ox0 + o, y0);
        }
        leave(o);
        return po;
      };
      if constexpr (BWD && !PACK) {
        // backward: per-window moment gradients from the upstream output gradients
        const int64_t prow = (int64_t)y0 * a.W + ox0;
#pragma unroll 1
        for (int q = 0; q < o1 - o0; ++q) {
          const int o = o0 + q;
          enter(o + a.k - 1);
          const double B = hw, Q = hww;
          const double Sxw = hx - double(q) * B, Syw = hy - double(y0 - y_ref) * B;
          const int cnt = hn;
          leave(o);
          const int x0 = ox0 + o;
          if (x0 >= a.W) continue;
          const int64_t pp = prow + o;
          MomentGrad mg = {0.0, 0.0, 0.0, 0.0};
          if (cnt == a.k * a.k) {
            const double uc = (double(x0) - a.cx) * a.inv_fx, vc = (double(y0) - a.cy) * a.inv_fy;
            const double gnx = a.normals ? a.normals[pp] : 0.0;
            const double gny = a.normals ? a.normals[a.plane + pp] : 0.0;
            const double gnz = a.normals ? a.normals[2 * a.plane + pp] : 0.0;
            const double gd = a.offsets ? a.offsets[pp] : 0.0;
            const double gr = a.residuals ? a.residuals[pp] : 0.0;
            Moments<double> m;
            m.Sxw = Sxw;
            m.Syw = Syw;
            m.V = a.N * Q - B * B;
            m.Sw = a.N * double(w_ref) + B;
            m.Sww = Q + double(w_ref) * (2.0 * B + a.N * double(w_ref));
            m.SSR = 0.0;
            if (MODE == PF_EXPLICIT)
              mg = explicit_adjoint(a, Sxw, Syw, m.Sw, m.V, uc, vc, gnx, gny, gnz, gd, gr);
            else
              mg = implicit_adjoint(a, m, uc, vc, gnx, gny, gnz, gd, gr);
          }
          a.gws[pp] = mg.Sw;
          a.gws[a.plane + pp] = mg.Sx;
          a.gws[2 * a.plane + pp] = mg.Sy;
          a.gws[3 * a.plane + pp] = mg.Sww;
        }
      } else {
        // Forward: stores through per-row buffer ranges: a pixel past the
        // strip, the frame or the band falls outside the range and the
        // hardware drops its store, so no branch guards a store.  The vector memory counter
        // retires in issue order, so the wait for the next round's depth loads
        // (issued before this phase) then counts these stores as issued
        // later and does not wait for them to complete.
        int cols;
        const RowOut<TL::run / 4> ro(a, yg, hj, nr, ox0, cols);
        if constexpr (PACK) {
          // A wave fits one row: 64 lanes x 4 windows.  Solving them lane by
          // lane costs a full solve round per window of the run whenever any
          // lane's window is valid, and near holes most are not.  So the sums
          // of all four windows are taken first; then the wave packs its valid
          // windows into consecutive slots of its own LDS rows (only this wave
          // reads them, and it has read them all: LDS serves a wave's accesses
          // in order), the other pixels after them, and solves 64 slots at a
          // time.  Results are those of the per-lane solve, bit for bit.  The
          // backward sweep packs the same way and runs the adjoint per slot.
          T pB[4], pX[4], pY[4], pQ[4];
          bool fit[4];
          // o0 is a multiple of the run, so column o0 + j sits at record
          // (j % 4) sub + o0 / 4 + j / 4 of the row: the four leaving columns
          // (j = q) at fixed offsets from one per-lane record, the entering
          // ones (j = q + k - 1) at offsets that are the same for every lane,
          // and their x - base (q - r and q + r) too.  The run's first record
          // and the window radius are opaque to the compiler: the LDS
          // addresses and x offsets are then formed here in each round rather
          // than hoisted out of the round loop, where they would hold
          // registers across the solve.
          int rb = rc + o0 / TL::run;
          __asm__ volatile("" : "+v"(rb));
          int kr = a.r;
          __asm__ volatile("" : "+s"(kr));
          auto enter_rec = [&](int l, int dx) {
            const ColumnSums<T> v = get_col(l);
            hw += v.w;
            hx += T(dx) * v.w;
            hy += v.yw;
            hww += v.ww;
            hn += v.n;
          };
          auto leave_rec = [&](int l, int dx) {
            const ColumnSums<T> v = get_col(l);
            hw = hw - v.w;
            hx = hx - T(dx) * v.w;
            hy = hy - v.yw;
            hww = hww - v.ww;
            hn -= v.n;
          };
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const unsigned e = unsigned(q + 2 * kr);  // entering column - o0
            enter_rec(rb + int((e % 4u) * TL::sub + e / 4u), q + kr);
            pB[q] = hw;
            pQ[q] = hww;
            pX[q] = hx - T(q) * hw;
            pY[q] = hy - T(y0 - y_ref) * hw;
            fit[q] = o0s + q < cols && hn == a.k * a.k;
            leave_rec(rb + q * TL::sub, q - kr);
          }
          uint64_t mfit[4];
          int nfit = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            mfit[q] = __builtin_amdgcn_ballot_w64(fit[q]);
            nfit += __builtin_popcountll(mfit[q]);
          }
          // slot s: (B, Q) and (X, Y) as two 16-byte records over the row's
          // records (FP32: one record), at record (s % 4) * kSlotSub + s / 4:
          // a dense row writes its slots lane by lane (consecutive records)
          // and reads them 64 at a time (spread over the bank groups as the
          // vertical phase's writes); the slots' columns as bytes after
          // the slots' records of the first array
          constexpr int kSlotSub = 66;
          static_assert(kSlotSub >= kBlock / 4 && (16 * kSlotSub) % 128 == 32, "slot layout");
          static_assert((kPitch - 4 * kSlotSub) * 16 >= kBlock, "slot columns");
          auto slot_rec = [](int s) { return (s & 3) * kSlotSub + (s >> 2); };
          Pair16<T>* kA = WIDE ? cs_lo + hj * kPitch
                               : reinterpret_cast<Pair16<T>*>(cs_one + hj * kPitch);
          Pair16<T>* kZ = WIDE ? reinterpret_cast<Pair16<T>*>(cs_hi + hj * kPitch) : nullptr;
          uint8_t* kc = reinterpret_cast<uint8_t*>(kA + 4 * kSlotSub);
          __asm__ volatile("" ::: "memory");  // every read of the column sums comes first
          // every window of the wave gets a slot: the valid ones 0 .. nfit-1,
          // the others (a pixel past the strip, the frame or the band among
          // them, whose column then fails the store's range test) the rest,
          // each kind in column order, so that a row's stores go out to
          // consecutive columns; a slot's sums are read only below nfit, so
          // the others are written unconditionally too
          const int lane = tid & 63;
          int below = 0;  // valid windows of the lower lanes
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const uint64_t mf = mfit[q];
            below += int(__builtin_amdgcn_mbcnt_hi(uint32_t(mf >> 32),
                                                   __builtin_amdgcn_mbcnt_lo(uint32_t(mf), 0u)));
          }
          int mine = 0;  // this lane's valid windows before window q
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int s = fit[q] ? below + mine : nfit + (4 * lane - below) + (q - mine);
            mine += fit[q] ? 1 : 0;
            if constexpr (WIDE) {
              Pair16<T> bq, xy;
              bq.a = pB[q];
              bq.b = pQ[q];
              xy.a = pX[q];
              xy.b = pY[q];
              kA[slot_rec(s)] = bq;
              kZ[slot_rec(s)] = xy;
            } else {
              Col16<T> r;  // B, X, Y in the float slots, Q in the last one
              r.w = pB[q];
              r.yw = pX[q];
              r.ww = pY[q];
              r.n = __float_as_int(float(pQ[q]));
              reinterpret_cast<Col16<T>*>(kA)[slot_rec(s)] = r;
            }
            kc[s] = uint8_t(o0s + q);
          }
          __asm__ volatile("" ::: "memory");
          // the loop's later trips run at a raised issue priority: a wave
          // that still has windows to solve there holds up its workgroup at
          // the round's last barrier, so it issues ahead of waves that are in
          // earlier phases of their rounds (a wave with no windows left only
          // issues its stores there)
#pragma unroll 1
          for (int s0 = 0; s0 < kBlock; s0 += 64) {
            if (s0 == 64) __builtin_amdgcn_s_setprio(1);
            const int s = s0 + lane;
            const int c = int(kc[s]);
            if constexpr (BWD) {
              // moment gradients of the window at column c: zero for an
              // invalid window, nothing past the strip, the frame or the band
              if (c < cols) {
                const int64_t pp = int64_t(y0) * a.W + ox0 + c;
                MomentGrad mg = {0.0, 0.0, 0.0, 0.0};
                if (s < nfit) {
                  const Pair16<T> bq = kA[slot_rec(s)], xy = kZ[slot_rec(s)];
                  const double B = bq.a, Q = bq.b;
                  const double uc = (double(ox0 + c) - a.cx) * a.inv_fx;
                  const double vc = (double(y0) - a.cy) * a.inv_fy;
                  const double gnx = a.normals ? a.normals[pp] : 0.0;
                  const double gny = a.normals ? a.normals[a.plane + pp] : 0.0;
                  const double gnz = a.normals ? a.normals[2 * a.plane + pp] : 0.0;
                  const double gd = a.offsets ? a.offsets[pp] : 0.0;
                  const double gr = a.residuals ? a.residuals[pp] : 0.0;
                  Moments<double> m;
                  m.Sxw = xy.a;
                  m.Syw = xy.b;
                  m.V = a.N * Q - B * B;
                  m.Sw = a.N * double(w_ref) + B;
                  m.Sww = Q + double(w_ref) * (2.0 * B + a.N * double(w_ref));
                  m.SSR = 0.0;
                  mg = implicit_adjoint(a, m, uc, vc, gnx, gny, gnz, gd, gr);
                }
                a.gws[pp] = mg.Sw;
                a.gws[a.plane + pp] = mg.Sx;
                a.gws[2 * a.plane + pp] = mg.Sy;
                a.gws[3 * a.plane + pp] = mg.Sww;
              }
            } else {
              PixelOut po = invalid_pixel();
              if (s < nfit) {
                T B, X, Y, Q;
                if constexpr (WIDE) {
                  const Pair16<T> bq = kA[slot_rec(s)], xy = kZ[slot_rec(s)];
                  B = bq.a;
                  Q = bq.b;
                  X = xy.a;
                  Y = xy.b;
                } else {
                  const Col16<T> r = reinterpret_cast<const Col16<T>*>(kA)[slot_rec(s)];
                  B = r.w;
                  X = r.yw;
                  Y = r.ww;
                  Q = T(__int_as_float(r.n));
                }
                if constexpr (std::is_same<T, df32>::value)
                  po = solve_pixel_df<MODE>(a, B, X, Y, Q, a.k * a.k, w_ref, ox0 + c, y0);
                else
                  po = solve_pixel<T, MODE>(a, B, X, Y, Q, a.k * a.k, w_ref, ox0 + c, y0);
              }
              ro.put(ro.at(c, cols), po);
            }
          }
          __builtin_amdgcn_s_setprio(0);
        } else if constexpr (MODE != PF_EXPLICIT) {
          // one pixel at a time, each stored as soon as it is solved (the
          // eigen-solve is large: the loop stays rolled)
#pragma unroll 1
          for (int q = 0; q < TL::run; ++q) {
            const PixelOut po = step(q);
            ro.put(ro.at(o0s + q, cols), po);
          }
        } else {
          float on0[TL::run], on1[TL::run], on2[TL::run], od[TL::run], ores[TL::run];
          uint8_t ost[TL::run];
#pragma unroll
          for (int q = 0; q < TL::run; ++q) {
            const PixelOut po = step(q);
            on0[q] = po.n0; on1[q] = po.n1; on2[q] = po.n2; od[q] = po.d; ores[q] = po.res;
            ost[q] = po.st;
          }
          if (vec_store) {
            // W, tile_w and o0s are multiples of 4, so a group of four is wholly
            // inside the row's range or wholly outside it
            static_assert(TL::run % 4 == 0, "whole 16-byte groups per run");
#pragma unroll
            for (int h = 0; h < TL::run / 4; ++h) {
              const uint32_t e = ro.at(o0s + 4 * h, cols);
              ro.put4(ro.n0, e, on0 + 4 * h);
              ro.put4(ro.n1, e, on1 + 4 * h);
              ro.put4(ro.n2, e, on2 + 4 * h);
              ro.put4(ro.d, e, od + 4 * h);
              ro.put4(ro.r, e, ores + 4 * h);
              uint32_t word = 0;
#pragma unroll
              for (int q = 0; q < 4; ++q) word |= uint32_t(ost[4 * h + q]) << (8 * q);
              __builtin_amdgcn_raw_buffer_store_b32(word, ro.st, int(e), 0, 0);
            }
          } else {
#pragma unroll
            for (int q = 0; q < TL::run; ++q) {
              PixelOut po;
              po.n0 = on0[q]; po.n1 = on1[q]; po.n2 = on2[q]; po.d = od[q]; po.res = ores[q];
              po.st = ost[q];
              ro.put(ro.at(o0s + q, cols), po);
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

template <typename T, int MODE, bool MASK, bool BWD = false, bool PARTIAL = false, int SHAPE = 0>
__global__ __launch_bounds__(kBlock, (kMinGroups<T, MODE, BWD, PARTIAL, SHAPE>)) void fit_planes_fused(LaunchArgs la) {
  // which job and which of its workgroups (the job table is uniform: scalar loop)
  int jb = 0;
  while (jb + 1 < la.n_jobs && int(blockIdx.x) >= la.jobs[jb + 1].wg_begin) ++jb;
  const LaunchCommon lc = {la.kappa_flag, la.kappa_fp64, la.dscale};
  double* gws = nullptr;
  if constexpr (BWD) gws = la.gws + bwd_ws_offset(la, jb);
  fit_tile<T, MODE, MASK, BWD, PARTIAL, SHAPE>(la.jobs[jb], int(blockIdx.x) - la.jobs[jb].wg_begin,
                                               lc, gws);
}

// ---------------------------------------------------------------------------
// Persistent batched launch.  A grid sized to the chip pulls work items (one
// workgroup tile of one frame each, in the job table's dispatch order) from a
// counter in device memory until the queue is drained, so frames of any number,
// size and window run in one launch and no workgroup slot idles while items
// remain.  The job table and the counter live in the caller's workspace; they
// are written by queue_setup launches whose arguments carry the table by value,
// so a batch records into a HIP graph as plain kernel nodes (no memset, no host
// copy) and every replay starts from a fresh counter.
// ---------------------------------------------------------------------------
struct QueueHeader {
  uint32_t next;     // next unclaimed work item
  uint32_t n_items;  // work items of the whole batch
  int32_t n_jobs;
  int32_t reserved;
};
constexpr size_t kQueueHeaderBytes = 256;
constexpr int kQueueSetupJobs = 32;  // jobs written per setup launch

struct QueueSetupArgs {
  QueueHeader* hdr;
  Job* jobs;  // the table in the workspace
  int32_t first, count, n_jobs;
  uint32_t n_items;
  Job chunk[kQueueSetupJobs];
};
static_assert(sizeof(QueueSetupArgs) <= 4096, "kernel arguments too large");
static_assert(sizeof(Job) % 4 == 0, "the job table is copied as 4-byte words");

__global__ __launch_bounds__(kBlock) void queue_setup(QueueSetupArgs qs) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(qs.chunk);
  uint32_t* dst = reinterpret_cast<uint32_t*>(qs.jobs + qs.first);
  const int words = qs.count * int(sizeof(Job) / 4);
  for (int i = int(threadIdx.x); i < words; i += kBlock) dst[i] = src[i];
  if (qs.first == 0 && threadIdx.x == 0) {
    qs.hdr->next = 0u;
    qs.hdr->n_items = qs.n_items;
    qs.hdr->n_jobs = qs.n_jobs;
  }
}

struct QueueArgs {
  QueueHeader* hdr;
  const Job* jobs;
  LaunchCommon lc;
};

// A job of the table read as uniform (scalar) values.
__device__ inline Job load_job_uniform(const Job* p) {
  Job j;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&j);
#pragma unroll
  for (int i = 0; i < int(sizeof(Job) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
  return j;
}

// The job of work item `item`: a forward scan from the job of the workgroup's
// previous item (items only grow), over the jobs' first items held in LDS for
// up to kQueueLdsJobs jobs, else read from the table.
constexpr int kQueueLdsJobs = 256;

// Compiled for four workgroups per CU at the 4 x 4 tiling whatever the shape's
// budget: the persistent loop's extra state would otherwise leave three resident
// (measured about 3 % faster on the 64-frame mixed batch).
template <typename T, int MODE, bool PARTIAL, int SHAPE>
constexpr int kQueuedGroups =
    Tiling<SHAPE>::rows == 4 ? kMinGroups<T, MODE, false, PARTIAL, 0> : kMinGroups<T, MODE, false, PARTIAL, SHAPE>;

template <typename T, int MODE, bool MASK, bool PARTIAL = false, int SHAPE = 0>
__global__ __launch_bounds__(kBlock, (kQueuedGroups<T, MODE, PARTIAL, SHAPE>)) void fit_planes_queued(QueueArgs qa) {
  __shared__ uint32_t s_item;
  __shared__ int32_t s_begin[kQueueLdsJobs];
  const uint32_t n_items = __builtin_amdgcn_readfirstlane(qa.hdr->n_items);
  const int n_jobs = __builtin_amdgcn_readfirstlane(qa.hdr->n_jobs);
  const uint32_t grid = gridDim.x;
  const bool lds_table = n_jobs <= kQueueLdsJobs;
  if (lds_table)
    for (int j = int(threadIdx.x); j < n_jobs; j += kBlock) s_begin[j] = qa.jobs[j].wg_begin;
  __syncthreads();
  // the first item of every workgroup is its own index; later ones come from
  // the counter, offset by the grid size
  uint32_t item = blockIdx.x;
  int jb = 0;
  while (item < n_items) {  // uniform: every wave of the group leaves together
    // While more than two items per workgroup remain, the next item is claimed
    // before this one runs (the atomic's latency overlaps this item's loads);
    // near the end of the queue it is claimed only once this item is done, so
    // the last items go to the workgroups that are free first.
    const bool ahead = item + 2 * grid < n_items;
    uint32_t next = 0;
    if (ahead && threadIdx.x == 0) next = grid + atomicAdd(&qa.hdr->next, 1u);
    while (jb + 1 < n_jobs &&
           int(item) >= (lds_table ? s_begin[jb + 1]
                                   : __builtin_amdgcn_readfirstlane(qa.jobs[jb + 1].wg_begin)))
      ++jb;
    jb = __builtin_amdgcn_readfirstlane(jb);
    const Job job = load_job_uniform(qa.jobs + jb);
    fit_tile<T, MODE, MASK, false, PARTIAL, SHAPE>(job, int(item) - job.wg_begin, qa.lc, nullptr);
    if (!ahead && threadIdx.x == 0) next = grid + atomicAdd(&qa.hdr->next, 1u);
    if (threadIdx.x == 0) s_item = next;
    __syncthreads();
    item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();  // every wave has the item before thread 0 writes the next one
  }
}

// ---------------------------------------------------------------------------
// Backward, second sweep: dL/dZ.  Every window sum S(p) = sum_{i in W_p} f_i
// is adjoint to a box sum over the windows containing pixel i, and for a k x k
// window those are exactly the windows centred in the k x k neighbourhood of i.
// So the same two-cursor integral-image sweep, run over the per-window moment
// gradients instead of the depth integrands, gives
//   dL/dw_i = sum_p [gSw(p) - (x_p - x_i) gSx(p) - (y_p - y_i) gSy(p) + 2 w_i gSww(p)]
// and dL/dZ_i = -dL/dw_i / Z_i^2 (0 for invalid pixels).  FP64 throughout.
// The job's `normals` pointer carries the float dL/dZ output [H][W].
// ---------------------------------------------------------------------------
template <bool MASK>
__global__ __launch_bounds__(kBlock) void grad_depth_fused(LaunchArgs la) {
  using TL = Tiling<0>;  // 4-row rounds, runs of 4: five FP64 channels in 46 KB
  int jb = 0;
  while (jb + 1 < la.n_jobs && int(blockIdx.x) >= la.jobs[jb + 1].wg_begin) ++jb;
  const Job& job = la.jobs[jb];
  const int wg = int(blockIdx.x) - job.wg_begin;
  const int H = job.H, W = job.W, k = job.k, r = job.k / 2;
  const int64_t plane = int64_t(H) * W;
  const double* gws = la.gws + bwd_ws_offset(la, jb);

  __shared__ double s_a[TL::rows * kPitch];
  __shared__ double s_e[TL::rows * kPitch];
  __shared__ double s_gx[TL::rows * kPitch];
  __shared__ double s_gy[TL::rows * kPitch];
  __shared__ double s_ygy[TL::rows * kPitch];

  const int tid = threadIdx.x;
  const int n_strips = job.n_strips;
  const int strip = wg % n_strips, band = wg / n_strips;
  const int ox0 = strip * job.tile_w, ix0 = ox0 - r, x = ix0 + tid;
  const int yb = band * job.tile_h, ye = min(yb + job.tile_h, H);
  const int y_ref = yb + job.tile_h / 2;
  const bool col_used = tid < job.tile_w + k - 1 && x >= 0 && x < W;

  struct C5 {
    double a, e, gx, gy, ygy;
  };
  // branch-free: a sample outside the frame or the strip's columns reads the
  // workspace's first element and is replaced by zero, so the loads of a
  // round all issue before the first is waited for
  auto load = [&](int y, C5& c) {
    const bool ok = col_used && y >= 0 && y < H;
    const int64_t p = ok ? int64_t(y) * W + x : 0;
    const double va = gws[p], vgx = gws[plane + p], vgy = gws[2 * plane + p];
    const double ve = gws[3 * plane + p];
    c.a = ok ? va : 0.0;
    c.gx = ok ? vgx : 0.0;
    c.gy = ok ? vgy : 0.0;
    c.e = ok ? ve : 0.0;
    c.ygy = double(y - y_ref) * c.gy;
  };
  C5 lead = {0, 0, 0, 0, 0}, lag = {0, 0, 0, 0, 0};
  auto add = [](C5& s, const C5& c) {
    s.a += c.a; s.e += c.e; s.gx += c.gx; s.gy += c.gy; s.ygy += c.ygy;
  };
  for (int i = 0; i < k - 1; ++i) {
    C5 c;
    load(yb - r + i, c);
    add(lead, c);
  }
  const int li = lds_index<0>(tid);
  const int hj = tid / (kBlock / TL::run), run = tid % (kBlock / TL::run);
  const int o0 = run * TL::run, o1 = min(o0 + TL::run, job.tile_w);
  for (int yg = yb; yg < ye; yg += TL::rows) {
    const int nr = min(TL::rows, ye - yg);
    // every load of the round is issued before any is used: one memory latency
    // per round instead of one per row and cursor
    C5 cin[TL::rows], cout[TL::rows];
#pragma unroll
    for (int j = 0; j < TL::rows; ++j) {
      const int y0 = yg + j;
      load(j < nr ? y0 + r : -1, cin[j]);
      load(j < nr && y0 > yb ? y0 - r - 1 : -1, cout[j]);
    }
#pragma unroll
    for (int j = 0; j < TL::rows; ++j) {
      if (j < nr) {
        const int y0 = yg + j;
        add(lead, cin[j]);
        if (y0 > yb) add(lag, cout[j]);
        s_a[j * kPitch + li] = lead.a - lag.a;
        s_e[j * kPitch + li] = lead.e - lag.e;
        s_gx[j * kPitch + li] = lead.gx - lag.gx;
        s_gy[j * kPitch + li] = lead.gy - lag.gy;
        s_ygy[j * kPitch + li] = lead.ygy - lag.ygy;
      }
    }
    __syncthreads();
    if (hj < nr && o0 < o1) {
      const int y0 = yg + hj;
      const double* ra = s_a + hj * kPitch;
      const double* re = s_e + hj * kPitch;
      const double* rgx = s_gx + hj * kPitch;
      const double* rgy = s_gy + hj * kPitch;
      const double* rygy = s_ygy + hj * kPitch;
      const int base = o0 + r;
      // the run's depth samples, loaded before the window sums are formed
      float zq[TL::run];
#pragma unroll
      for (int q = 0; q < TL::run; ++q) {
        const int xi = ox0 + o0 + q;
        const bool in = o0 + q < o1 && xi < W;
        const int xs = in ? xi : 0;  // the row's first sample stands in
        const float z = job.depth[int64_t(y0) * job.depth_pitch + xs];
        zq[q] = in ? z : 0.0f;
        if (MASK && job.mask && job.mask[int64_t(y0) * job.mask_pitch + xs] == 0) zq[q] = 0.0f;
      }
      double h[6] = {0, 0, 0, 0, 0, 0}, g[6] = {0, 0, 0, 0, 0, 0};  // a, e, gx, xgx, gy, ygy
      auto acc = [&](double* s6, int i) {
        const int l = lds_index<0>(i);
        const double vx = rgx[l];
        s6[0] += ra[l];
        s6[1] += re[l];
        s6[2] += vx;
        s6[3] += double(i - base) * vx;
        s6[4] += rgy[l];
        s6[5] += rygy[l];
      };
      for (int i = o0; i < o0 + k - 1; ++i) acc(h, i);
#pragma unroll
      for (int q = 0; q < TL::run; ++q) {
        if (q >= o1 - o0) break;
        const int o = o0 + q;
        acc(h, o + k - 1);
        const double A = h[0] - g[0], E = h[1] - g[1];
        const double Bx = (h[3] - g[3]) - double(q) * (h[2] - g[2]);
        const double By = (h[5] - g[5]) - double(y0 - y_ref) * (h[4] - g[4]);
        acc(g, o);
        const int xi = ox0 + o;
        if (xi < W) {
          const float z = zq[q];
          double dz = 0.0;
          if (depth_valid(z)) {
            // dL/dw, then chained to the input: dw/dZ = -w^2, or dw/dD = dscale
            const double w = la.dscale > 0.0 ? double(z) * la.dscale : 1.0 / double(z);
            const double gw = A - Bx - By + 2.0 * w * E;
            dz = la.dscale > 0.0 ? gw * la.dscale : -gw * w * w;
          }
          job.normals[int64_t(y0) * W + xi] = float(dz);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// The standard formulation, for comparison (Sec. II, Eq. 3-9): the same
// sliding-window sweep over the back-projected points P = Z (u, v, 1) instead
// of the disparity integrands.  Every entry of the scatter matrix of Eq. 5
// depends on the depth, so nine channels (sums of X, Y, Z and of their six
// products) plus the count are carried instead of four: the cost the RGBD
// formulation removes.  FP64 throughout; points are taken relative to a
// per-band reference point so that the covariance differences stay small.
//   implicit (Eq. 3-6): n = eigenvector of the smallest eigenvalue of the
//                       window covariance, d = -n . centroid (|n| = 1);
//   explicit (Eq. 7-9): Z = a X + b Y + c by centred least squares, i.e. the
//                       plane (a, b, -1) . P + c = 0, normalised.
// Orientation d >= 0; residual = RMS point-to-plane distance (depth unit);
// status bit 1 (implicit) as in the RGBD fit.  Rounds of 2 rows, runs of 2
// outputs: 10 channels of column sums fit in 44 KB of LDS.
// ---------------------------------------------------------------------------
constexpr int kXyzRows = 2, kXyzRun = 2, kXyzSub = kPitch / kXyzRun;
__device__ inline int xyz_lds_index(int i) { return (i % kXyzRun) * kXyzSub + i / kXyzRun; }

template <int MODE, bool MASK>
__global__ __launch_bounds__(kBlock) void fit_planes_xyz(LaunchArgs la) {
  const Job& job = la.jobs[0];
  const int wg = int(blockIdx.x);
  const int H = job.H, W = job.W, k = job.k, r = job.k / 2;
  const int64_t plane = int64_t(H) * W;
  const int tid = threadIdx.x;
  const int strip = wg % job.n_strips, band = wg / job.n_strips;
  const int ox0 = strip * job.tile_w, ix0 = ox0 - r, x = ix0 + tid;
  const int yb = band * job.tile_h, ye = min(yb + job.tile_h, H);
  const int y_ref = min(yb + job.tile_h / 2, H - 1);
  const bool col_used = tid < job.tile_w + k - 1 && x >= 0 && x < W;
  const double ifx = 1.0 / job.fx, ify = 1.0 / job.fy;
  const double ux = (double(x) - job.cx) * ifx;

  __shared__ double s_c[9][kXyzRows * kPitch];
  __shared__ int s_n[kXyzRows * kPitch];
  __shared__ double red[2 * (kBlock / 64)];

  auto load = [&](int y) -> float {
    if (!col_used || y < 0 || y >= H) return 0.0f;
    float z = job.depth[int64_t(y) * job.depth_pitch + x];
    if (MASK && job.mask && job.mask[int64_t(y) * job.mask_pitch + x] == 0) z = 0.0f;
    return z;
  };

  // reference point: mean depth of the band's middle row on the ray of the strip centre
  double zs = 0.0, zc = 0.0;
  {
    const float z = load(y_ref);
    if (depth_valid(z)) {
      zs = double(z);
      zc = 1.0;
    }
    for (int off = 32; off > 0; off >>= 1) {
      zs += __shfl_down(zs, off, 64);
      zc += __shfl_down(zc, off, 64);
    }
    if ((tid & 63) == 0) {
      red[2 * (tid >> 6)] = zs;
      red[2 * (tid >> 6) + 1] = zc;
    }
    __syncthreads();
    zs = 0.0;
    zc = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) {
      zs += red[2 * i];
      zc += red[2 * i + 1];
    }
  }
  const double Zr = zc > 0.0 ? zs / zc : 1.0;
  const double Xr = Zr * (double(ox0 + job.tile_w / 2) - job.cx) * ifx;
  const double Yr = Zr * (double(y_ref) - job.cy) * ify;

  double c[9];
  int cn = 0;
#pragma unroll
  for (int i = 0; i < 9; ++i) c[i] = 0.0;
  // one sample into (sign +1) or out of (sign -1) the column sums
  auto sample = [&](float z, int y, double sign) {
    const bool ok = depth_valid(z);
    const double zd = ok ? double(z) : 0.0;
    const double px = ok ? zd * ux - Xr : 0.0;
    const double py = ok ? zd * ((double(y) - job.cy) * ify) - Yr : 0.0;
    const double pz = ok ? zd - Zr : 0.0;
    const double sx = sign * px, sy = sign * py, sz = sign * pz;
    c[0] += sx; c[1] += sy; c[2] += sz;
    c[3] += sx * px; c[4] += sx * py; c[5] += sx * pz;
    c[6] += sy * py; c[7] += sy * pz; c[8] += sz * pz;
    cn += ok ? (sign > 0.0 ? 1 : -1) : 0;
  };
  for (int i = 0; i < k - 1; ++i) sample(load(yb - r + i), yb - r + i, 1.0);

  const int li = xyz_lds_index(tid);
  const int hj = tid / (kBlock / kXyzRun), run = tid % (kBlock / kXyzRun);
  const int o0 = run * kXyzRun, o1 = min(o0 + kXyzRun, job.tile_w);
  for (int yg = yb; yg < ye; yg += kXyzRows) {
    const int nr = min(kXyzRows, ye - yg);
    for (int j = 0; j < kXyzRows; ++j) {
      if (j < nr) {
        const int y0 = yg + j;
        if (y0 > yb) sample(load(y0 - r - 1), y0 - r - 1, -1.0);
        sample(load(y0 + r), y0 + r, 1.0);
#pragma unroll
        for (int i = 0; i < 9; ++i) s_c[i][j * kPitch + li] = c[i];
        s_n[j * kPitch + li] = cn;
      }
    }
    __syncthreads();
    if (hj < nr && o0 < o1) {
      const int y0 = yg + hj;
      double h[9];
      int hn = 0;
#pragma unroll
      for (int i = 0; i < 9; ++i) h[i] = 0.0;
      auto move = [&](int i, double sign) {
        const int l = xyz_lds_index(i);
#pragma unroll
        for (int t = 0; t < 9; ++t) h[t] += sign * s_c[t][hj * kPitch + l];
        hn += sign > 0.0 ? s_n[hj * kPitch + l] : -s_n[hj * kPitch + l];
      };
      for (int i = o0; i < o0 + k - 1; ++i) move(i, 1.0);
      for (int q = 0; q < o1 - o0; ++q) {
        const int o = o0 + q;
        move(o + k - 1, 1.0);
        const int xo = ox0 + o;
        float on0 = __builtin_nanf(""), on1 = on0, on2 = on0, od = on0, ores = on0;
        uint8_t st = 1;
        if (hn == k * k && xo < W) {
          const double iN = 1.0 / double(k * k);
          const double mx = h[0] * iN, my = h[1] * iN, mz = h[2] * iN;
          const double cxx = h[3] - h[0] * mx, cxy = h[4] - h[0] * my, cxz = h[5] - h[0] * mz;
          const double cyy = h[6] - h[1] * my, cyz = h[7] - h[1] * mz, czz = h[8] - h[2] * mz;
          const double Mx = mx + Xr, My = my + Yr, Mz = mz + Zr;
          double n0, n1, n2, d, res;
          st = 0;
          if (MODE == PF_IMPLICIT) {
            const Eig3<double> e =
                smallest_eig<double>(cxx, cxy, cxz, cyy, cyz, czz, la.kappa_flag > 0.0);
            n0 = e.n[0]; n1 = e.n[1]; n2 = e.n[2];
            d = -(n0 * Mx + n1 * My + n2 * Mz);
            res = sqrt(fmax(e.l1, 0.0) * iN);
            const double gap = e.l2 - e.l1;
            const double kap = (e.degenerate || !(gap > 0.0)) ? __builtin_inf() : e.l3 / gap;
            if (la.kappa_flag > 0.0 && !(kap <= la.kappa_flag)) st = 2;
          } else {
            const double det = cxx * cyy - cxy * cxy;
            const double idet = 1.0 / det;
            const double aa = (cxz * cyy - cyz * cxy) * idet, bb = (cyz * cxx - cxz * cxy) * idet;
            const double cc = Mz - aa * Mx - bb * My;
            const double is = 1.0 / sqrt(aa * aa + bb * bb + 1.0);
            n0 = aa * is; n1 = bb * is; n2 = -is;
            d = cc * is;
            res = sqrt(fmax(czz - aa * cxz - bb * cyz, 0.0) * iN) * is;
          }
          if (facing_flip(d, n0, n1, n2)) {
            d = -d; n0 = -n0; n1 = -n1; n2 = -n2;
          }
          d = d + 0.0;
          on0 = float(n0); on1 = float(n1); on2 = float(n2); od = float(d); ores = float(res);
        }
        if (xo < W) {
          const int64_t pp = int64_t(y0) * W + xo;
          job.normals[pp] = on0;
          job.normals[plane + pp] = on1;
          job.normals[2 * plane + pp] = on2;
          job.offsets[pp] = od;
          job.residuals[pp] = ores;
          if (job.status) job.status[pp] = st;
        }
        move(o, -1.0);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Global integral images and fits to arbitrary rectangles: the paper's own use
// of integral images (Sec. II-C), for fits to many regions of one frame (tiles,
// segmentation candidates) rather than to every pixel's window.
//
// Workspace (doubles): a 256-byte header (the frame's reference disparity
// w_ref at [0]), then five planes I[c][H+1][W+1] with a zero first row and
// column,
//   c = 0: w^ = w - w_ref,  1: x~ w^,  2: y~ w^,  3: w^2,  4: valid count,
// summed over valid pixels, with x~ = x - W/2 and y~ = y - H/2 (integers; the
// centring halves the magnitude of the prefix sums a corner difference cancels),
// then the tile aggregates the build carries between tiles:
//   CT[c][band][W]   column totals of each band of kIntBand rows, scanned to
//                    the sum of the bands above,
//   RT[c][strip][H]  row totals of each strip of kBlock columns, scanned to the
//                    sum of the strips to the left.
//
// Three launches, each reading the depth at most once and writing each plane
// entry once:
//   integral_tiles  per tile (strip x band): its column totals and row totals;
//   integral_carry  the two exclusive scans of those totals;
//   integral_final  per tile: the tile's own 2D prefix (a running column sum
//                   of row scans) plus its carries.  With Cb[x] the scanned
//                   column total of the tile's band and Rs[y] the scanned row
//                   total of its strip, a pixel (x, y) of the tile at (x0, y0)
//     I[y+1][x+1] = sum_{x' < x0} Cb[x'] + sum_{x0 <= x' <= x} Cb[x']
//                 + sum_{y0 <= y' <= y} Rs[y'] + sum_{y0 <= y' <= y, x0 <= x' <= x} v.
// Every workgroup computes w_ref itself from the middle row (the same
// reduction in the same order, so the same value).
// ---------------------------------------------------------------------------
constexpr int kIntBand = 16;
constexpr int kIntWaves = kBlock / 64;
constexpr int64_t kIntHeader = 32;  // doubles (256 bytes)

struct IntegralArgs {
  const float* depth;
  const uint8_t* mask;
  int64_t depth_pitch, mask_pitch;
  int32_t H, W;
  double* ws;
};

struct IntegralLayout {
  int64_t ld, P;       // plane row length (W + 1) and plane size
  int n_strips, n_bands;
  double* I;           // the five planes
  double* CT;          // [5][n_bands][W]
  double* RT;          // [5][n_strips][H]
  double* WT;          // [n_bands][n_strips][kIntBand][kIntWaves][5]: each wave's row totals
  __device__ explicit IntegralLayout(const IntegralArgs& ia) {
    ld = ia.W + 1;
    P = int64_t(ia.H + 1) * ld;
    n_strips = (ia.W + kBlock - 1) / kBlock;
    n_bands = (ia.H + kIntBand - 1) / kIntBand;
    I = ia.ws + kIntHeader;
    CT = I + 5 * P;
    RT = CT + int64_t(5) * n_bands * ia.W;
    WT = RT + int64_t(5) * n_strips * ia.H;
  }
  __device__ double* tile_wt(int s, int b) const {
    return WT + (int64_t(b) * n_strips + s) * (kIntBand * kIntWaves * 5);
  }
};

// depth of pixel (x, y), clamped into the frame: every load is in bounds and
// none sits behind a branch, so a batch of them is issued back to back
__device__ inline float int_depth(const IntegralArgs& ia, int x, int y) {
  return ia.depth[int64_t(min(y, ia.H - 1)) * ia.depth_pitch + min(x, ia.W - 1)];
}
__device__ inline uint8_t int_mask(const IntegralArgs& ia, int x, int y) {
  return ia.mask[int64_t(min(y, ia.H - 1)) * ia.mask_pitch + min(x, ia.W - 1)];
}

// the frame's reference disparity: mean valid w of the middle row, reduced by
// the whole workgroup in a fixed order
__device__ inline double integral_wref(const IntegralArgs& ia, double* red) {
  const int tid = threadIdx.x, y = ia.H / 2;
  constexpr int kBatch = 8;
  double s = 0.0, c = 0.0;
  for (int x0 = tid; x0 < ia.W; x0 += kBatch * kBlock) {
    float z[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) z[j] = int_depth(ia, x0 + j * kBlock, y);
    if (ia.mask) {
      uint8_t m[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) m[j] = int_mask(ia, x0 + j * kBlock, y);
#pragma unroll
      for (int j = 0; j < kBatch; ++j) z[j] = m[j] ? z[j] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
      if (x0 + j * kBlock < ia.W && depth_valid(z[j])) {
        s += 1.0 / double(z[j]);
        c += 1.0;
      }
  }
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_down(s, off, 64);
    c += __shfl_down(c, off, 64);
  }
  if ((tid & 63) == 0) {
    red[2 * (tid >> 6)] = s;
    red[2 * (tid >> 6) + 1] = c;
  }
  __syncthreads();
  double ts = 0.0, tc = 0.0;
  for (int i = 0; i < kIntWaves; ++i) {
    ts += red[2 * i];
    tc += red[2 * i + 1];
  }
  __syncthreads();
  return tc > 0.0 ? ts / tc : 0.0;
}

// the band's depth samples of column x (0 outside the frame or the band, and
// where masked), all loads issued before any is used
__device__ inline void load_band(const IntegralArgs& ia, int x, int y0, int y1, float z[kIntBand]) {
#pragma unroll
  for (int j = 0; j < kIntBand; ++j) z[j] = int_depth(ia, x, y0 + j);
  if (ia.mask) {
    uint8_t m[kIntBand];
#pragma unroll
    for (int j = 0; j < kIntBand; ++j) m[j] = int_mask(ia, x, y0 + j);
#pragma unroll
    for (int j = 0; j < kIntBand; ++j) z[j] = m[j] ? z[j] : 0.0f;
  }
#pragma unroll
  for (int j = 0; j < kIntBand; ++j) z[j] = (x < ia.W && y0 + j < y1) ? z[j] : 0.0f;
}

// the five integrands of pixel (x, y) with depth z; zero outside the frame and
// where invalid
__device__ inline void integrands(const IntegralArgs& ia, int x, int y, float z, double wref,
                                  double v[5]) {
  for (int c = 0; c < 5; ++c) v[c] = 0.0;
  if (x < ia.W && depth_valid(z)) {
    const double wh = 1.0 / double(z) - wref;
    v[0] = wh;
    v[1] = double(x - ia.W / 2) * wh;
    v[2] = double(y - ia.H / 2) * wh;
    v[3] = wh * wh;
    v[4] = 1.0;
  }
}

// Inclusive prefix sum over the 64 lanes of a wave from DPP lane moves (row
// shifts by 1, 2, 4, 8 within rows of 16 lanes, then the broadcasts of lane
// 15 of each row to the next row and of lane 31 to the upper half): six
// dependent steps with no LDS round trip.  Doubles move as two 32-bit halves.
template <int CTRL>
__device__ inline int dpp_move(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const uint64_t b = uint64_t(__double_as_longlong(v));
  const int lo = dpp_move<CTRL>(int(uint32_t(b)));
  const int hi = dpp_move<CTRL>(int(uint32_t(b >> 32)));
  return __longlong_as_double(int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo)));
}

template <typename V>
__device__ inline V wave_scan_add(V v) {
  const int lane = int(threadIdx.x) & 63, rl = lane & 15;
  V t = dpp_move<0x111>(v);  // row_shr:1
  v = rl >= 1 ? v + t : v;
  t = dpp_move<0x112>(v);    // row_shr:2
  v = rl >= 2 ? v + t : v;
  t = dpp_move<0x114>(v);    // row_shr:4
  v = rl >= 4 ? v + t : v;
  t = dpp_move<0x118>(v);    // row_shr:8
  v = rl >= 8 ? v + t : v;
  t = dpp_move<0x142>(v);    // row_bcast:15
  v = (lane & 31) >= 16 ? v + t : v;
  t = dpp_move<0x143>(v);    // row_bcast:31
  v = lane >= 32 ? v + t : v;
  return v;
}

// Within-wave row prefix of the five integrands.  y~ w^ (channel 2) is y~
// times w^ along a row, so its prefix is y~ times channel 0's and is not
// scanned; the valid count (channel 4) is scanned as an integer.
__device__ inline void wave_row_scan(const double v[5], double yt, double r[5]) {
  r[0] = wave_scan_add(v[0]);
  r[1] = wave_scan_add(v[1]);
  r[3] = wave_scan_add(v[3]);
  r[4] = double(wave_scan_add(int(v[4])));
  r[2] = yt * r[0];
}

// per tile: column totals over the band; row totals over the strip and each
// wave's share of them
__global__ __launch_bounds__(kBlock) void integral_tiles(IntegralArgs ia) {
  __shared__ double red[2 * kIntWaves];
  __shared__ double part[kIntBand][kIntWaves][5];  // per row, per wave
  const IntegralLayout L(ia);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s = int(blockIdx.x), b = int(blockIdx.y);
  const int x = s * kBlock + tid;
  const int y0 = b * kIntBand, y1 = min(y0 + kIntBand, ia.H);
  float z[kIntBand];
  load_band(ia, x, y0, y1, z);
  const double wref = integral_wref(ia, red);
  double cs[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < kIntBand; ++j) {
    const int y = y0 + j;
    if (y >= y1) break;
    double v[5], r[5];
    integrands(ia, x, y, z[j], wref, v);
    for (int c = 0; c < 5; ++c) cs[c] += v[c];
    wave_row_scan(v, double(y - ia.H / 2), r);
    if (lane == 63)
      for (int c = 0; c < 5; ++c) part[j][wave][c] = r[c];
  }
  if (x < ia.W)
    for (int c = 0; c < 5; ++c) L.CT[(int64_t(c) * L.n_bands + b) * ia.W + x] = cs[c];
  __syncthreads();
  double* wt = L.tile_wt(s, b);
  for (int i = tid; i < (y1 - y0) * kIntWaves * 5; i += kBlock) wt[i] = (&part[0][0][0])[i];
  for (int i = tid; i < (y1 - y0) * 5; i += kBlock) {
    const int r = i / 5, c = i % 5;
    double t = 0.0;
    for (int w = 0; w < kIntWaves; ++w) t += part[r][w][c];
    L.RT[(int64_t(c) * L.n_strips + s) * ia.H + y0 + r] = t;
  }
}

// Exclusive scans of the tile totals: column totals down the bands (four
// lanes per column, each over a quarter of the bands, joined by a four-lane
// scan) and row totals across the strips (one thread per row and channel).
constexpr int kCarryLanes = 4;
__global__ __launch_bounds__(kBlock) void integral_carry(IntegralArgs ia) {
  const IntegralLayout L(ia);
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t ncol = int64_t(5) * ia.W * kCarryLanes;
  if (i < ncol) {  // ncol is a multiple of 4, so a group of four lanes is never split
    const int q = int(i % kCarryLanes);
    const int64_t col = i / kCarryLanes;
    const int c = int(col / ia.W), x = int(col % ia.W);
    double* T = L.CT + int64_t(c) * L.n_bands * ia.W + x;
    const int per = (L.n_bands + kCarryLanes - 1) / kCarryLanes;
    const int bb = min(q * per, L.n_bands), be = min(bb + per, L.n_bands);
    double part = 0.0;
    for (int b0 = bb; b0 < be; b0 += 32) {
      double v[32];
#pragma unroll
      for (int j = 0; j < 32; ++j) v[j] = (b0 + j < be) ? T[int64_t(b0 + j) * ia.W] : 0.0;
#pragma unroll
      for (int j = 0; j < 32; ++j) part += v[j];
    }
    // exclusive prefix of the four partial sums (lanes 4g .. 4g+3 share a DPP row)
    const int lane = int(threadIdx.x) & 63;
    double incl = part, t = dpp_move<0x111>(incl);
    incl = (lane & 3) >= 1 ? incl + t : incl;
    t = dpp_move<0x112>(incl);
    incl = (lane & 3) >= 2 ? incl + t : incl;
    double acc = incl - part;
    for (int b0 = bb; b0 < be; b0 += 32) {
      double v[32];
#pragma unroll
      for (int j = 0; j < 32; ++j) v[j] = (b0 + j < be) ? T[int64_t(b0 + j) * ia.W] : 0.0;
#pragma unroll
      for (int j = 0; j < 32; ++j)
        if (b0 + j < be) {
          T[int64_t(b0 + j) * ia.W] = acc;
          acc += v[j];
        }
    }
  } else if (i < ncol + int64_t(5) * ia.H) {
    const int64_t k = i - ncol;
    const int c = int(k / ia.H), y = int(k % ia.H);
    double* T = L.RT + int64_t(c) * L.n_strips * ia.H + y;
    double acc = 0.0;
    for (int s0 = 0; s0 < L.n_strips; s0 += 16) {
      double v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = (s0 + j < L.n_strips) ? T[int64_t(s0 + j) * ia.H] : 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (s0 + j < L.n_strips) {
          T[int64_t(s0 + j) * ia.H] = acc;
          acc += v[j];
        }
    }
  }
}

// inclusive prefix of v over the workgroup's 256 threads (in thread order);
// tot: LDS scratch of 4 x 5 doubles, free on entry and on return
__device__ inline void block_scan5(double v[5], double (*tot)[5]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int c = 0; c < 5; ++c) v[c] = wave_scan_add(v[c]);
  if (lane == 63)
    for (int c = 0; c < 5; ++c) tot[wave][c] = v[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    double before = 0.0;
    for (int w = 0; w < kIntWaves; ++w)
      if (w < wave) before += tot[w][c];
    v[c] += before;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void integral_final(IntegralArgs ia) {
  __shared__ double red[2 * kIntWaves];
  __shared__ double tot[kIntWaves][5];
  __shared__ double wt[kIntBand][kIntWaves][5];  // per row: each wave's total (from the tiles pass)
  __shared__ double rt[kIntBand][5];             // the strip's scanned row totals
  const IntegralLayout L(ia);
  const int tid = threadIdx.x, wave = tid >> 6;
  const int s = int(blockIdx.x), b = int(blockIdx.y);
  const int x = s * kBlock + tid, x0 = s * kBlock;
  const int y0 = b * kIntBand, y1 = min(y0 + kIntBand, ia.H);
  float z[kIntBand];
  load_band(ia, x, y0, y1, z);
  {
    const double* src = L.tile_wt(s, b);
    for (int i = tid; i < (y1 - y0) * kIntWaves * 5; i += kBlock) (&wt[0][0][0])[i] = src[i];
    for (int i = tid; i < (y1 - y0) * 5; i += kBlock)
      rt[i / 5][i % 5] = L.RT[(int64_t(i % 5) * L.n_strips + s) * ia.H + y0 + i / 5];
  }
  const double wref = integral_wref(ia, red);  // its barriers also publish wt and rt
  if (s == 0 && b == 0 && tid == 0) ia.ws[0] = wref;
  // the plane's zero first row (tiles of the first band) and first column
  // (tiles of the first strip)
  if (b == 0)
    for (int c = 0; c < 5; ++c) {
      if (x < ia.W) L.I[c * L.P + x + 1] = 0.0;
      if (s == 0 && tid == 0) L.I[c * L.P] = 0.0;
    }
  if (s == 0)
    for (int i = tid; i < (y1 - y0) * 5; i += kBlock)
      L.I[(i % 5) * L.P + int64_t(y0 + i / 5 + 1) * L.ld] = 0.0;
  // column carries: Pc[x] = sum_{x' <= x} Cb[x'] over the whole row (the part
  // left of the strip, a strided sum reduced over the workgroup, plus the
  // strip's own prefix)
  double pc[5], left[5];
  for (int c = 0; c < 5; ++c) {
    const double* Cb = L.CT + (int64_t(c) * L.n_bands + b) * ia.W;
    pc[c] = x < ia.W ? Cb[x] : 0.0;
    double t = 0.0;
    for (int xx = tid; xx < x0; xx += kBlock) t += Cb[xx];
    left[c] = t;
  }
  block_scan5(pc, tot);
  block_scan5(left, tot);  // thread 255 then holds the total of the strips to the left
  if (tid == kBlock - 1)
    for (int c = 0; c < 5; ++c) tot[0][c] = left[c];
  __syncthreads();
  for (int c = 0; c < 5; ++c) pc[c] += tot[0][c];
  // rows: the strip's row prefix (wave scan plus the totals of the waves to
  // the left), summed down the band, plus the carries
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, rc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < kIntBand; ++j) {
    const int y = y0 + j;
    if (y >= y1) break;
    double v[5], r[5];
    integrands(ia, x, y, z[j], wref, v);
    const double yt = double(y - ia.H / 2);
    wave_row_scan(v, yt, r);
    for (int w = 0; w < kIntWaves; ++w)
      if (w < wave)
        for (int c = 0; c < 5; ++c)
          if (c != 2) r[c] += wt[j][w][c];
    r[2] = yt * r[0];
    const int64_t row = int64_t(y + 1) * L.ld + x + 1;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      rc[c] += rt[j][c];
      acc[c] += r[c];
      if (x < ia.W) L.I[c * L.P + row] = pc[c] + rc[c] + acc[c];
    }
  }
}

struct RectArgs {
  const double* ws;
  const int32_t* rects;  // [n][4] = x0, y0, w, h
  float* normals;        // [3][n]
  float* offsets;
  float* residuals;
  uint8_t* status;
  int64_t n;
  int32_t H, W;
  double fx, fy, cx, cy;
  double kappa_flag;
};

// One fit per rectangle from the four corners of each integral image.  The
// camera-only moments of a w x h rectangle, centred on (xc, yc) =
// (x0 + (w-1)/2, y0 + (h-1)/2), are diagonal: sum x'^2 = h w (w^2-1)/12,
// sum y'^2 = w h (h^2-1)/12, N = w h; the rest is the per-pixel solve with
// unequal x and y second moments.
template <int MODE>
__global__ __launch_bounds__(kBlock) void fit_rects_kernel(RectArgs ra) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= ra.n) return;
  const int x0 = ra.rects[4 * i], y0 = ra.rects[4 * i + 1];
  const int w = ra.rects[4 * i + 2], h = ra.rects[4 * i + 3];
  float on0 = __builtin_nanf(""), on1 = on0, on2 = on0, od = on0, ores = on0;
  uint8_t st = 1;
  const bool inside = w >= 2 && h >= 2 && x0 >= 0 && y0 >= 0 && x0 <= ra.W - w &&
                      y0 <= ra.H - h;
  if (inside) {
    const int64_t ld = ra.W + 1, P = int64_t(ra.H + 1) * ld;
    const double* I = ra.ws + kIntHeader;
    const int64_t a = int64_t(y0) * ld + x0, b = a + w, c = a + int64_t(h) * ld, d = c + w;
    double S[5];
#pragma unroll
    for (int ch = 0; ch < 5; ++ch)
      S[ch] = (I[ch * P + d] - I[ch * P + b]) - (I[ch * P + c] - I[ch * P + a]);
    const double N = double(w) * double(h);
    if (S[4] == N) {
      const double wref = ra.ws[0];
      const double xc = x0 + 0.5 * (w - 1), yc = y0 + 0.5 * (h - 1);
      const double B = S[0], Q = S[3];
      const double Sxw = S[1] - (xc - ra.W / 2) * B, Syw = S[2] - (yc - ra.H / 2) * B;
      const double S2x = N * (double(w) * w - 1.0) / 12.0, S2y = N * (double(h) * h - 1.0) / 12.0;
      const double V = N * Q - B * B;
      const double Sw = N * wref + B;
      const double Sww = Q + wref * (2.0 * B + N * wref);
      const double uc = (xc - ra.cx) / ra.fx, vc = (yc - ra.cy) / ra.fy;
      double n0, n1, n2, dd, res;
      st = 0;
      if (MODE == PF_EXPLICIT) {
        const double ax = ra.fx * Sxw / S2x, ay = ra.fy * Syw / S2y;
        const double az = Sw / N - ax * uc - ay * vc;
        const double rho = sqrt(ax * ax + ay * ay + az * az);
        n0 = -ax / rho; n1 = -ay / rho; n2 = -az / rho;
        dd = 1.0 / rho;
        const double ssr = fmax(V / N - Sxw * Sxw / S2x - Syw * Syw / S2y, 0.0);
        res = dd * sqrt(ssr / N);
      } else {
        // C = M^T G M, G = diag(S2x, S2y, N) - g g^T / Sww (G33 = V / Sww)
        const double iS = 1.0 / Sww, ifx = 1.0 / ra.fx, ify = 1.0 / ra.fy;
        const double g11 = S2x - Sxw * Sxw * iS, g22 = S2y - Syw * Syw * iS;
        const double g12 = -Sxw * Syw * iS, g13 = -Sxw * Sw * iS, g23 = -Syw * Sw * iS;
        const double g33 = V * iS;
        const double c00 = g11 * ifx * ifx + 2.0 * g13 * uc * ifx + g33 * uc * uc;
        const double c01 = g12 * ifx * ify + g13 * vc * ifx + g23 * uc * ify + g33 * uc * vc;
        const double c02 = g13 * ifx + g33 * uc;
        const double c11 = g22 * ify * ify + 2.0 * g23 * vc * ify + g33 * vc * vc;
        const double c12 = g23 * ify + g33 * vc;
        const double c22 = g33;
        const bool flag = ra.kappa_flag > 0.0;
        const Eig3<double> e = smallest_eig<double>(c00, c01, c02, c11, c12, c22, flag);
        n0 = e.n[0]; n1 = e.n[1]; n2 = e.n[2];
        dd = -(n0 * ifx * Sxw + n1 * ify * Syw + (n0 * uc + n1 * vc + n2) * Sw) * iS;
        res = sqrt(fmax(e.l1, 0.0) / N);
        if (flag) {
          const double gap = e.l2 - e.l1;
          const double kap = (e.degenerate || !(gap > 0.0)) ? __builtin_inf() : e.l3 / gap;
          if (!(kap <= ra.kappa_flag)) st = 2;
        }
      }
      if (facing_flip(dd, n0, n1, n2)) {
        dd = -dd; n0 = -n0; n1 = -n1; n2 = -n2;
      }
      dd = dd + 0.0;
      on0 = float(n0); on1 = float(n1); on2 = float(n2); od = float(dd); ores = float(res);
    }
  }
  ra.normals[i] = on0;
  ra.normals[ra.n + i] = on1;
  ra.normals[2 * ra.n + i] = on2;
  ra.offsets[i] = od;
  ra.residuals[i] = ores;
  if (ra.status) ra.status[i] = st;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
thread_local int g_last_hip_error = 0;

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

struct pf_plan {
  pf_intrinsics intr;
  int64_t H, W;
  pf_params params;
  double dscale() const {
    return (params.flags & PF_FLAG_DISPARITY) ? params.disparity_scale : 0.0;
  }
  // partial windows: 3 <= min_valid < k^2 (0 or >= k^2 is the full-window rule)
  bool partial() const { return params.min_valid > 0 && params.min_valid < k * k; }
  int k, r;
  double S2, N;
  int tile_w, tile_h, n_strips, n_bands;
  bool band_auto;  // tile_h is the default rule's: a batch launch may raise it
  int shape;  // launch shape (Tiling<shape>)
  // launch shapes other than 0 exist for FP64 implicit / explicit full-window fits
  bool shapes_allowed() const {
    return params.precision == PF_PREC_FP64 && !partial() &&
           (params.mode == PF_IMPLICIT || params.mode == PF_EXPLICIT);
  }
};

namespace {
// The default band height of a plan for launch shape `shape`: enough
// workgroups for one full round of the chip at four workgroups per CU (two for
// the 8 x 8 shape) on 256 CUs, whatever the shape's occupancy, and at least one
// round of rows.  Rounded up to whole rounds of rows: a band of 4q + 1 rows
// costs as many rounds as one of 4q + 4, whose fewer workgroups then share the
// chip (1920x1080, k = 15: 9 -> 12 rows).
int64_t default_band_height(const pf_plan* p, int shape) {
  const int64_t target_groups = shape_rows(shape) == 4 ? 1024 : 256 * int64_t(shape_groups(shape));
  const int64_t round_rows = shape_rows(shape);
  int64_t th = (p->H * p->n_strips + target_groups - 1) / target_groups;
  th = std::max<int64_t>(th, 4);
  th = (th + round_rows - 1) / round_rows * round_rows;
  return std::min<int64_t>(th, p->H);
}
}  // namespace

extern "C" {

const char* pf_status_string(pf_status s) {
  switch (s) {
    case PF_OK: return "ok";
    case PF_ERR_NULL: return "a required pointer is NULL";
    case PF_ERR_SHAPE: return "bad frame size (need 1 <= H, W <= 65535 and H*W <= 2^31)";
    case PF_ERR_WINDOW: return "bad window (need odd k, 3 <= k <= 63, k <= min(H, W))";
    case PF_ERR_INTRINSICS: return "bad intrinsics (need finite fx, fy > 0 and finite cx, cy)";
    case PF_ERR_PITCH: return "a row pitch is smaller than the frame width";
    case PF_ERR_ALIGNMENT: return "a float pointer is not 4-byte aligned";
    case PF_ERR_WORKSPACE: return "workspace missing or too small";
    case PF_ERR_UNSUPPORTED: return "unsupported mode, precision or flag value";
    case PF_ERR_HIP: return "HIP runtime error (see pf_last_hip_error)";
  }
  return "unknown status";
}

int pf_last_hip_error(void) { return g_last_hip_error; }

pf_status pf_plan_create(const pf_intrinsics* intr, int64_t height, int64_t width,
                         const pf_params* params, pf_plan** out) {
  if (out) *out = nullptr;
  if (!intr || !params || !out) return PF_ERR_NULL;
  if (height < 1 || width < 1 || height > 65535 || width > 65535 ||
      height * width > (int64_t(1) << 31))
    return PF_ERR_SHAPE;
  if (!finite_pos(intr->fx) || !finite_pos(intr->fy) || !std::isfinite(intr->cx) ||
      !std::isfinite(intr->cy))
    return PF_ERR_INTRINSICS;
  const int k = params->window;
  if (k < 3 || k > kMaxWindow || (k % 2) == 0 || k > height || k > width) return PF_ERR_WINDOW;
  if ((params->mode != PF_IMPLICIT && params->mode != PF_EXPLICIT &&
       params->mode != PF_IMPLICIT_LITERAL) ||
      (params->mode == PF_IMPLICIT_LITERAL &&
       (params->precision != PF_PREC_FP64 || params->kappa_flag != 0.0)) ||
      params->min_valid < 0 || (params->min_valid > 0 && params->min_valid < 3) ||
      (params->min_valid > 0 && params->min_valid < k * k &&
       (params->precision != PF_PREC_FP64 || params->mode == PF_IMPLICIT_LITERAL)) ||
      (params->precision != PF_PREC_FP64 && params->precision != PF_PREC_FP32 &&
       params->precision != PF_PREC_COMPENSATED) ||
      (params->flags & ~PF_FLAG_DISPARITY) != 0 ||
      ((params->flags & PF_FLAG_DISPARITY) &&
       !(params->disparity_scale > 0.0 && std::isfinite(params->disparity_scale))) ||
      !(params->kappa_flag >= 0.0) || !std::isfinite(params->kappa_flag) ||
      !(params->kappa_fp64 >= 0.0) || !std::isfinite(params->kappa_fp64))
    return PF_ERR_UNSUPPORTED;
  pf_plan* p = new (std::nothrow) pf_plan;
  if (!p) return PF_ERR_UNSUPPORTED;
  p->intr = *intr;
  p->H = height;
  p->W = width;
  p->params = *params;
  p->k = k;
  p->r = k / 2;
  p->N = double(k) * k;
  p->S2 = double(k) * k * (double(k) * k - 1.0) / 12.0;
  // strips: each workgroup covers kBlock input columns, k - 1 of them halo
  // (tile_w kept a multiple of 4 so rows of a run can be stored as float4)
  const int tw_max = ((kBlock - (k - 1)) / 4) * 4;
  p->n_strips = int((width + tw_max - 1) / tw_max);
  p->tile_w = int(((width + p->n_strips - 1) / p->n_strips + 3) / 4 * 4);
  // launch shape: the FP64 implicit fit is compiled for a budget of two
  // workgroups per CU (same tiles and results as shape 0, and it still fits
  // four per CU; measured 30.3 against 32.4 us on the 640x480 frame at
  // k = 3, 5, 9, 15 in one launch, 47.1 against 48.9 us at 1920x1080, k = 15);
  // everything else runs shape 0
  p->shape = (p->shapes_allowed() && params->mode == PF_IMPLICIT) ? 1 : 0;
  const int64_t th = default_band_height(p, p->shape);  // pf_plan_derive sets others
  p->tile_h = int(th);
  p->n_bands = int((height + th - 1) / th);
  p->band_auto = true;
  *out = p;
  return PF_OK;
}

void pf_plan_destroy(pf_plan* plan) { delete plan; }

size_t pf_plan_workspace_bytes(const pf_plan* plan) {
  (void)plan;
  return 0;
}

pf_status pf_plan_camera_moments(const pf_plan* plan, int64_t x0, int64_t y0, double out[6]) {
  if (!plan || !out) return PF_ERR_NULL;
  // window-centred closed form: sum x' = sum y' = sum x'y' = 0, sum x'^2 = sum y'^2 = S2
  const double uc = (double(x0) - plan->intr.cx) / plan->intr.fx;
  const double vc = (double(y0) - plan->intr.cy) / plan->intr.fy;
  const double N = plan->N, S2 = plan->S2;
  out[0] = N * uc * uc + S2 / (plan->intr.fx * plan->intr.fx);
  out[1] = N * uc * vc;
  out[2] = N * uc;
  out[3] = N * vc * vc + S2 / (plan->intr.fy * plan->intr.fy);
  out[4] = N * vc;
  out[5] = N;
  return PF_OK;
}

}  // extern "C"

namespace {

// Host-side checks of every frame of a batch, before anything is enqueued.
pf_status check_batch(const pf_plan* const* plans, const pf_frame_io* io, int32_t n) {
  if (n < 0) return PF_ERR_SHAPE;
  if (n == 0) return PF_OK;
  if (!plans || !io) return PF_ERR_NULL;
  auto misaligned = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 3u) != 0; };
  for (int32_t i = 0; i < n; ++i) {
    const pf_plan* p = plans[i];
    const pf_frame_io& f = io[i];
    if (!p || !f.depth || !f.normals || !f.offsets || !f.residuals) return PF_ERR_NULL;
    if (f.depth_pitch < p->W || f.depth_pitch > INT32_MAX ||
        (f.mask && (f.mask_pitch < p->W || f.mask_pitch > INT32_MAX)))
      return PF_ERR_PITCH;
    if (misaligned(f.depth) || misaligned(f.normals) || misaligned(f.offsets) ||
        misaligned(f.residuals))
      return PF_ERR_ALIGNMENT;
    if (p->params.mode != plans[0]->params.mode ||
        p->params.precision != plans[0]->params.precision ||
        p->params.kappa_flag != plans[0]->params.kappa_flag ||
        p->params.kappa_fp64 != plans[0]->params.kappa_fp64 ||
        p->dscale() != plans[0]->dscale() || p->partial() != plans[0]->partial() ||
        p->shape != plans[0]->shape)
      return PF_ERR_UNSUPPORTED;
  }
  return PF_OK;
}

// The job of one frame (its workgroups start at wg_begin), in bands of tile_h rows.
Job make_job(const pf_plan* p, const pf_frame_io& f, int32_t wg_begin, int32_t tile_h) {
  auto aligned = [](const void* q, uintptr_t m) { return (reinterpret_cast<uintptr_t>(q) & m) == 0; };
  Job jb;
  std::memset(&jb, 0, sizeof(jb));
  jb.depth = f.depth;
  jb.mask = f.mask;
  jb.normals = f.normals;
  jb.offsets = f.offsets;
  jb.residuals = f.residuals;
  jb.status = f.status;
  jb.fx = p->intr.fx;
  jb.fy = p->intr.fy;
  jb.cx = p->intr.cx;
  jb.cy = p->intr.cy;
  jb.depth_pitch = int32_t(f.depth_pitch);
  jb.mask_pitch = f.mask ? int32_t(f.mask_pitch) : 0;
  jb.H = int32_t(p->H);
  jb.W = int32_t(p->W);
  jb.k = p->k;
  jb.tile_w = p->tile_w;
  jb.tile_h = tile_h;
  jb.n_strips = p->n_strips;
  jb.wg_begin = wg_begin;
  jb.min_valid = int16_t(p->partial() ? p->params.min_valid : 0);
  jb.vec_store = (p->W % 4 == 0) && (p->tile_w % 4 == 0) && aligned(f.normals, 15) &&
                 aligned(f.offsets, 15) && aligned(f.residuals, 15) &&
                 (!f.status || aligned(f.status, 3));
  return jb;
}

int64_t job_groups(const pf_plan* p, int64_t tile_h) {
  return int64_t(p->n_strips) * ((p->H + tile_h - 1) / tile_h);
}

LaunchCommon launch_common(const pf_plan* p) {
  LaunchCommon lc;
  lc.kappa_flag = p->params.kappa_flag;
  lc.kappa_fp64 = p->params.kappa_fp64 > 0.0 ? p->params.kappa_fp64 : kDefaultKappaFp64;
  lc.dscale = p->dscale();
  return lc;
}

// Compute units of the current device (queried once per device).
int device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
  if (dev < 64) {
    const int c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  if (dev < 64) cache[dev].store(cus, std::memory_order_relaxed);
  return cus;
}

// Band heights of a batch's frames (tile_h[i] for plans[i]).  The default
// rule sizes each plan alone, for about one workgroup per resident slot (four
// per CU), so a batch of such frames has several times the chip's slots in
// one-round bands: each band repeats its k - 1 warm-up rows for four output
// rows, and a launch ends on a part-filled round of workgroups.  While the
// batch holds more workgroups than the chip keeps resident, the largest window
// (its warm-up is the longest; on ties the lowest band, then the first frame)
// whose default band height is below 12 rows gets one more round of rows.  Measured on the
// 640x480 frame at k = 3, 5, 9, 15 (1440 -> 1020 workgroups in 4, 4, 8, 12 rows:
// 29.4 -> 28.3 us implicit, 19.1 -> 16.9 us explicit) and on the 64-frame mixed
// batch (12 rows throughout: 336 -> 315 us by value, 398 -> 342 us queued).
// Only FP64 full-window implicit and explicit plans are raised (the FP32 fit
// ran 4 % slower so, its kernels keeping more workgroups resident; the
// compensated one no faster).  Heights set explicitly (pf_plan_derive,
// autotuned plans) are kept, and so are those of the 8-row-round shape.
// Planned over the whole batch, so the by-value and the queued launches of one
// batch run the same bands.
void batch_band_heights(const pf_plan* const* plans, int32_t n, int32_t* tile_h) {
  constexpr int32_t kCap = 12;
  int64_t groups = 0;
  for (int32_t i = 0; i < n; ++i) {
    tile_h[i] = plans[i]->tile_h;
    groups += job_groups(plans[i], tile_h[i]);
  }
  const int64_t slots = 4 * int64_t(device_cus());
  while (groups > slots) {
    int32_t pick = -1;
    for (int32_t i = 0; i < n; ++i) {
      const pf_plan* p = plans[i];
      if (!p->band_auto || !p->shapes_allowed() || shape_rows(p->shape) != 4 ||
          tile_h[i] >= kCap || tile_h[i] >= p->H)
        continue;
      if (pick < 0 || p->k > plans[pick]->k ||
          (p->k == plans[pick]->k && tile_h[i] < tile_h[pick]))
        pick = i;
    }
    if (pick < 0) break;
    groups -= job_groups(plans[pick], tile_h[pick]);
    // capped at the frame, as pf_plan_derive caps it (the height also places
    // the band's reference row)
    tile_h[pick] = int32_t(std::min<int64_t>(tile_h[pick] + 4, plans[pick]->H));
    groups += job_groups(plans[pick], tile_h[pick]);
  }
}


// One persistent launch of the instantiation for (T, MODE, MASK, PARTIAL):
// grid = resident workgroups of the chip (occupancy x compute units), capped
// at the number of work items.
template <typename T, int MODE, bool MASK, bool PARTIAL, int SHAPE = 0>
hipError_t launch_queued(const QueueArgs& qa, uint32_t n_items, hipStream_t s) {
  const void* fn =
      reinterpret_cast<const void*>(&fit_planes_queued<T, MODE, MASK, PARTIAL, SHAPE>);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0) != hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  if (std::getenv("PF_QUEUE_DEBUG"))
    std::fprintf(stderr, "planefit queued launch: %d workgroups per CU x %d CUs, %u items\n",
                 per_cu, device_cus(), n_items);
  const uint32_t grid = std::min<uint32_t>(n_items, uint32_t(per_cu) * uint32_t(device_cus()));
  hipLaunchKernelGGL((fit_planes_queued<T, MODE, MASK, PARTIAL, SHAPE>), dim3(grid), dim3(kBlock),
                     0, s, qa);
  return hipGetLastError();
}

template <int SHAPE>
hipError_t launch_queued_fp64_shape(const QueueArgs& qa, uint32_t n_items, int mode, bool mask,
                                    hipStream_t s) {
  if (mode == PF_EXPLICIT)
    return mask ? launch_queued<double, PF_EXPLICIT, true, false, SHAPE>(qa, n_items, s)
                : launch_queued<double, PF_EXPLICIT, false, false, SHAPE>(qa, n_items, s);
  return mask ? launch_queued<double, PF_IMPLICIT, true, false, SHAPE>(qa, n_items, s)
              : launch_queued<double, PF_IMPLICIT, false, false, SHAPE>(qa, n_items, s);
}

template <typename T>
hipError_t launch_queued_modes(const QueueArgs& qa, uint32_t n_items, int mode, bool mask,
                               hipStream_t s) {
  if (mode == PF_EXPLICIT)
    return mask ? launch_queued<T, PF_EXPLICIT, true, false>(qa, n_items, s)
                : launch_queued<T, PF_EXPLICIT, false, false>(qa, n_items, s);
  if (mode == PF_IMPLICIT_LITERAL) {
    if constexpr (std::is_same<T, double>::value)
      return mask ? launch_queued<T, PF_IMPLICIT_LITERAL, true, false>(qa, n_items, s)
                  : launch_queued<T, PF_IMPLICIT_LITERAL, false, false>(qa, n_items, s);
    return hipErrorInvalidValue;
  }
  return mask ? launch_queued<T, PF_IMPLICIT, true, false>(qa, n_items, s)
              : launch_queued<T, PF_IMPLICIT, false, false>(qa, n_items, s);
}

// The queued batch after the argument checks: dispatch order (frames with the
// costliest work items, the largest windows, first, so the queue ends on the
// cheapest ones; results do not depend on it), job table into `ws` by setup
// launches, then one persistent fit launch.  `jobs`, `order` and `heights` are
// host buffers of n entries (heights: per frame, in the caller's order).
pf_status enqueue_queued(const pf_plan* const* plans, const pf_frame_io* io, int32_t n, void* ws,
                         void* stream, Job* jobs, int32_t* order, int32_t* heights) {
  // up to kMaxJobs frames fit in one launch's arguments: that launch, whose
  // workgroups the hardware dispatches, is already the single launch the
  // queue would give, without the queue's per-item claim and table reads
  if (n <= kMaxJobs) return pf_fit_planes_batch(plans, io, n, stream);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int32_t j = 0; j < n; ++j) order[j] = j;
  std::stable_sort(order, order + n,
                   [&](int32_t x, int32_t y) { return plans[x]->k > plans[y]->k; });
  bool has_mask = false;
  batch_band_heights(plans, n, heights);
  int64_t items = 0;
  for (int32_t j = 0; j < n; ++j) {
    const int32_t i = order[j];
    const int64_t g = job_groups(plans[i], heights[i]);
    if (items + g > INT32_MAX) return PF_ERR_SHAPE;
    jobs[j] = make_job(plans[i], io[i], int32_t(items), heights[i]);
    has_mask = has_mask || io[i].mask != nullptr;
    items += g;
  }
  QueueHeader* hdr = static_cast<QueueHeader*>(ws);
  Job* table = reinterpret_cast<Job*>(static_cast<char*>(ws) + kQueueHeaderBytes);
  for (int32_t first = 0; first < n; first += kQueueSetupJobs) {
    QueueSetupArgs qs;
    std::memset(&qs, 0, sizeof(qs));
    qs.hdr = hdr;
    qs.jobs = table;
    qs.first = first;
    qs.count = std::min<int32_t>(kQueueSetupJobs, n - first);
    qs.n_jobs = n;
    qs.n_items = uint32_t(items);
    std::memcpy(qs.chunk, jobs + first, size_t(qs.count) * sizeof(Job));
    hipLaunchKernelGGL(queue_setup, dim3(1), dim3(kBlock), 0, s, qs);
  }
  hipError_t err = hipGetLastError();
  if (err == hipSuccess) {
    QueueArgs qa;
    qa.hdr = hdr;
    qa.jobs = table;
    qa.lc = launch_common(plans[0]);
    const int prec = plans[0]->params.precision;
    const int mode = plans[0]->params.mode;
    const uint32_t ni = uint32_t(items);
    if (plans[0]->partial())
      err = mode == PF_EXPLICIT
                ? (has_mask ? launch_queued<double, PF_EXPLICIT, true, true>(qa, ni, s)
                            : launch_queued<double, PF_EXPLICIT, false, true>(qa, ni, s))
                : (has_mask ? launch_queued<double, PF_IMPLICIT, true, true>(qa, ni, s)
                            : launch_queued<double, PF_IMPLICIT, false, true>(qa, ni, s));
    else if (prec == PF_PREC_FP64 && plans[0]->shape == 1)
      err = launch_queued_fp64_shape<1>(qa, ni, mode, has_mask, s);
    else if (prec == PF_PREC_FP64 && plans[0]->shape == 2)
      err = launch_queued_fp64_shape<2>(qa, ni, mode, has_mask, s);
    else if (prec == PF_PREC_FP64)
      err = launch_queued_modes<double>(qa, ni, mode, has_mask, s);
    else if (prec == PF_PREC_FP32)
      err = launch_queued_modes<float>(qa, ni, mode, has_mask, s);
    else
      err = launch_queued_modes<df32>(qa, ni, mode, has_mask, s);
  }
  if (err != hipSuccess) {
    g_last_hip_error = int(err);
    return PF_ERR_HIP;
  }
  return PF_OK;
}

// Scratch of the allocation-free queued batch (pf_fit_planes_batch_queued_noalloc):
// the queue header and the job table of up to kNoAllocJobs frames, one copy per
// GPU the library runs on, held until the process ends.  In host code the
// array's name is only a host-side stand-in: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr int kNoAllocJobs = 256;
constexpr size_t kNoAllocScratchBytes =
    (kQueueHeaderBytes + size_t(kNoAllocJobs) * sizeof(Job) + 255) / 256 * 256;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (PF_ERR_HIP if the
// runtime cannot resolve it).
pf_status scratch_for_current_device(void** out) {
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) {
    g_last_hip_error = int(err);
    return PF_ERR_HIP;
  }
  if (dev < 0 || dev >= kMaxDevices) return PF_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess || !p) {
      g_last_hip_error = int(err != hipSuccess ? err : hipErrorInvalidSymbol);
      return PF_ERR_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PF_OK;
}

}  // namespace

extern "C" {

pf_status pf_fit_planes_batch(const pf_plan* const* plans, const pf_frame_io* io, int32_t n,
                              void* stream) {
  const pf_status chk = check_batch(plans, io, n);
  if (chk != PF_OK || n == 0) return chk;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int prec = plans[0]->params.precision;
  const bool expl = plans[0]->params.mode == PF_EXPLICIT;
  int32_t stack_heights[kMaxJobs];
  std::vector<int32_t> heap_heights;
  int32_t* heights = stack_heights;
  if (n > kMaxJobs) {
    heap_heights.resize(static_cast<size_t>(n));
    heights = heap_heights.data();
  }
  batch_band_heights(plans, n, heights);
  for (int32_t first = 0; first < n; first += kMaxJobs) {
    const int32_t cnt = std::min<int32_t>(kMaxJobs, n - first);
    LaunchArgs la;
    std::memset(&la, 0, sizeof(la));
    la.n_jobs = cnt;
    const LaunchCommon lc = launch_common(plans[first]);
    la.kappa_flag = lc.kappa_flag;
    la.dscale = lc.dscale;
    la.kappa_fp64 = lc.kappa_fp64;
    bool has_mask = false;
    int32_t wg = 0;
    // dispatch order: the jobs with the longest workgroups (largest window,
    // whose warm-up is longest, and the tallest bands) first, so that the
    // launch's last, partial round of workgroups holds the shortest ones.
    // Results do not depend on the order.
    int32_t order[kMaxJobs];
    for (int32_t j = 0; j < cnt; ++j) order[j] = first + j;
    std::stable_sort(order, order + cnt,
                     [&](int32_t x, int32_t y) { return plans[x]->k > plans[y]->k; });
    for (int32_t j = 0; j < cnt; ++j) {
      const pf_plan* p = plans[order[j]];
      const pf_frame_io& f = io[order[j]];
      const int32_t th = heights[order[j]];
      la.jobs[j] = make_job(p, f, wg, th);
      has_mask = has_mask || f.mask != nullptr;
      wg += int32_t(job_groups(p, th));
    }
    la.n_wg = wg;
    const dim3 grid(static_cast<unsigned>(wg));
    const dim3 block(kBlock);
#define PF_LAUNCH(T, M, K) \
  hipLaunchKernelGGL((fit_planes_fused<T, M, K>), grid, block, 0, s, la)
#define PF_LAUNCH_MODES(T)                                                     \
  do {                                                                         \
    if (expl) {                                                                \
      if (has_mask) PF_LAUNCH(T, PF_EXPLICIT, true); else PF_LAUNCH(T, PF_EXPLICIT, false); \
    } else {                                                                   \
      if (has_mask) PF_LAUNCH(T, PF_IMPLICIT, true); else PF_LAUNCH(T, PF_IMPLICIT, false); \
    }                                                                          \
  } while (0)
#define PF_LAUNCH_SHAPE(M, K, SH) \
  hipLaunchKernelGGL((fit_planes_fused<double, M, K, false, false, SH>), grid, block, 0, s, la)
#define PF_LAUNCH_FP64_SHAPES(SH)                                              \
  do {                                                                         \
    if (expl) {                                                                \
      if (has_mask) PF_LAUNCH_SHAPE(PF_EXPLICIT, true, SH); else PF_LAUNCH_SHAPE(PF_EXPLICIT, false, SH); \
    } else {                                                                   \
      if (has_mask) PF_LAUNCH_SHAPE(PF_IMPLICIT, true, SH); else PF_LAUNCH_SHAPE(PF_IMPLICIT, false, SH); \
    }                                                                          \
  } while (0)
    if (plans[first]->partial()) {
      if (expl) {
        if (has_mask) hipLaunchKernelGGL((fit_planes_fused<double, PF_EXPLICIT, true, false, true>), grid, block, 0, s, la);
        else hipLaunchKernelGGL((fit_planes_fused<double, PF_EXPLICIT, false, false, true>), grid, block, 0, s, la);
      } else {
        if (has_mask) hipLaunchKernelGGL((fit_planes_fused<double, PF_IMPLICIT, true, false, true>), grid, block, 0, s, la);
        else hipLaunchKernelGGL((fit_planes_fused<double, PF_IMPLICIT, false, false, true>), grid, block, 0, s, la);
      }
    } else if (prec == PF_PREC_FP64 && plans[first]->params.mode == PF_IMPLICIT_LITERAL) {
      if (has_mask) PF_LAUNCH(double, PF_IMPLICIT_LITERAL, true);
      else PF_LAUNCH(double, PF_IMPLICIT_LITERAL, false);
    } else if (prec == PF_PREC_FP64) {
      const int shape = plans[first]->shape;
      if (shape == 1) PF_LAUNCH_FP64_SHAPES(1);
      else if (shape == 2) PF_LAUNCH_FP64_SHAPES(2);
      else PF_LAUNCH_MODES(double);
    } else if (prec == PF_PREC_FP32)
      PF_LAUNCH_MODES(float);
    else
      PF_LAUNCH_MODES(df32);
#undef PF_LAUNCH_FP64_SHAPES
#undef PF_LAUNCH_SHAPE
#undef PF_LAUNCH_MODES
#undef PF_LAUNCH
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
      g_last_hip_error = int(err);
      return PF_ERR_HIP;
    }
  }
  return PF_OK;
}

size_t pf_batch_workspace_bytes(int32_t n) {
  if (n <= 0) return 0;
  const size_t bytes = kQueueHeaderBytes + size_t(n) * sizeof(Job);
  return (bytes + 255) / 256 * 256;
}

pf_status pf_fit_planes_batch_queued(const pf_plan* const* plans, const pf_frame_io* io,
                                     int32_t n, void* workspace, size_t workspace_bytes,
                                     void* stream) {
  const pf_status chk = check_batch(plans, io, n);
  if (chk != PF_OK || n == 0) return chk;
  if (!workspace || workspace_bytes < pf_batch_workspace_bytes(n) ||
      (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return PF_ERR_WORKSPACE;
  std::vector<Job> jobs(static_cast<size_t>(n));
  std::vector<int32_t> order(static_cast<size_t>(n), 0), heights(static_cast<size_t>(n), 0);
  return enqueue_queued(plans, io, n, workspace, stream, jobs.data(), order.data(), heights.data());
}

pf_status pf_fit_planes_batch_queued_noalloc(const pf_plan* const* plans, const pf_frame_io* io,
                                             int32_t n, void* stream) {
  const pf_status chk = check_batch(plans, io, n);
  if (chk != PF_OK || n == 0) return chk;
  if (n > kNoAllocJobs) return PF_ERR_WORKSPACE;
  void* ws = nullptr;
  const pf_status st = scratch_for_current_device(&ws);
  if (st != PF_OK) return st;
  Job jobs[kNoAllocJobs];
  int32_t order[kNoAllocJobs], heights[kNoAllocJobs];
  return enqueue_queued(plans, io, n, ws, stream, jobs, order, heights);
}

int32_t pf_batch_noalloc_max_frames(void) { return kNoAllocJobs; }

pf_status pf_batch_band_heights(const pf_plan* const* plans, int32_t n, int32_t* band_heights) {
  if (n < 0) return PF_ERR_SHAPE;
  if (n == 0) return PF_OK;
  if (!plans || !band_heights) return PF_ERR_NULL;
  for (int32_t i = 0; i < n; ++i)
    if (!plans[i]) return PF_ERR_NULL;
  batch_band_heights(plans, n, band_heights);
  return PF_OK;
}

pf_status pf_fit_planes(const pf_plan* plan, const float* depth, int64_t depth_pitch,
                        const uint8_t* mask, int64_t mask_pitch, float* normals,
                        float* offsets, float* residuals, uint8_t* status, void* workspace,
                        size_t workspace_bytes, void* stream) {
  (void)workspace;
  (void)workspace_bytes;
  if (!plan) return PF_ERR_NULL;
  const pf_frame_io f = {depth, depth_pitch, mask, mask_pitch, normals, offsets, residuals, status};
  return pf_fit_planes_batch(&plan, &f, 1, stream);
}

int32_t pf_plan_band_height(const pf_plan* plan) { return plan ? plan->tile_h : 0; }

pf_status pf_plan_derive(const pf_plan* plan, int32_t band_height, int32_t shape,
                         pf_plan** out) {
  if (out) *out = nullptr;
  if (!plan || !out) return PF_ERR_NULL;
  if (band_height < 0) return PF_ERR_SHAPE;
  if (shape < -1 || shape >= kShapes || (shape > 0 && !plan->shapes_allowed()))
    return PF_ERR_UNSUPPORTED;
  pf_plan* p = new (std::nothrow) pf_plan(*plan);
  if (!p) return PF_ERR_UNSUPPORTED;
  if (shape >= 0) p->shape = shape;
  const int64_t th = band_height > 0 ? band_height : default_band_height(p, p->shape);
  p->tile_h = int(std::min<int64_t>(th, p->H));
  p->n_bands = int((p->H + p->tile_h - 1) / p->tile_h);
  p->band_auto = band_height == 0;
  *out = p;
  return PF_OK;
}

int32_t pf_plan_shape(const pf_plan* plan) { return plan ? plan->shape : -1; }

pf_status pf_plan_autotune(const pf_plan* plan, const float* depth, int64_t depth_pitch,
                           const uint8_t* mask, int64_t mask_pitch, float* normals,
                           float* offsets, float* residuals, uint8_t* status, void* stream,
                           int32_t* chosen_band_height, int32_t* chosen_shape) {
  if (!plan) return PF_ERR_NULL;
  const pf_frame_io f = {depth, depth_pitch, mask, mask_pitch, normals, offsets, residuals, status};
  // validate the buffers once (and warm the code up) with the plan's own shape
  pf_status st = pf_fit_planes_batch(&plan, &f, 1, stream);
  if (st != PF_OK) return st;
  // candidates run on a private copy: the caller's plan is never written
  pf_plan trial(*plan);
  trial.band_auto = false;  // each candidate runs at exactly its own band height
  const pf_plan* tp = &trial;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  static const int kCandidates[] = {4, 6, 8, 12, 16, 20, 24, 32, 48, 64};
  int best_h = plan->tile_h, best_shape = plan->shape;
  float best_ms = 0.0f;
  const int n_shapes = plan->shapes_allowed() ? kShapes : 1;
  for (int shape = 0; shape < n_shapes && err == hipSuccess && st == PF_OK; ++shape) {
    for (int cand : kCandidates) {
      if (err != hipSuccess) break;
      if (cand > plan->H || cand % shape_rows(shape) != 0) continue;
      trial.shape = shape;
      trial.tile_h = cand;
      trial.n_bands = int((plan->H + cand - 1) / cand);
      // two warm-up launches, then the fastest of three timed groups of five
      // back-to-back launches (the minimum filters clock and queue noise)
      for (int rep = 0; rep < 2 && st == PF_OK; ++rep) st = pf_fit_planes_batch(&tp, &f, 1, stream);
      if (st != PF_OK) break;
      float ms = 0.0f;
      for (int grp = 0; grp < 3 && st == PF_OK && err == hipSuccess; ++grp) {
        err = hipEventRecord(e0, s);
        for (int rep = 0; rep < 5 && st == PF_OK && err == hipSuccess; ++rep)
          st = pf_fit_planes_batch(&tp, &f, 1, stream);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float t = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        if (err == hipSuccess && (grp == 0 || t < ms)) ms = t;
      }
      if (st != PF_OK || err != hipSuccess) break;
      if (best_ms == 0.0f || ms < best_ms) {
        best_ms = ms;
        best_h = cand;
        best_shape = shape;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != PF_OK) return st;
  if (err != hipSuccess) {
    g_last_hip_error = int(err);
    return PF_ERR_HIP;
  }
  if (chosen_band_height) *chosen_band_height = best_h;
  if (chosen_shape) *chosen_shape = best_shape;
  return PF_OK;
}

size_t pf_backward_workspace_bytes(const pf_plan* plan) {
  return plan ? size_t(4) * sizeof(double) * size_t(plan->H) * size_t(plan->W) : 0;
}

pf_status pf_fit_planes_backward_batch(const pf_plan* const* plans, const pf_backward_io* io,
                                       int32_t n, void* workspace, size_t workspace_bytes,
                                       void* stream) {
  if (n < 0) return PF_ERR_SHAPE;
  if (n == 0) return PF_OK;
  if (!plans || !io) return PF_ERR_NULL;
  auto misaligned = [](const void* q, uintptr_t m) {
    return (reinterpret_cast<uintptr_t>(q) & m) != 0;
  };
  size_t need = 0;
  for (int32_t i = 0; i < n; ++i) {
    const pf_plan* p = plans[i];
    const pf_backward_io& f = io[i];
    if (!p || !f.depth || !f.grad_depth) return PF_ERR_NULL;
    if (f.depth_pitch < p->W || f.depth_pitch > INT32_MAX ||
        (f.mask && (f.mask_pitch < p->W || f.mask_pitch > INT32_MAX)))
      return PF_ERR_PITCH;
    if (misaligned(f.depth, 3) || misaligned(f.grad_depth, 3) ||
        (f.grad_normals && misaligned(f.grad_normals, 3)) ||
        (f.grad_offsets && misaligned(f.grad_offsets, 3)) ||
        (f.grad_residuals && misaligned(f.grad_residuals, 3)))
      return PF_ERR_ALIGNMENT;
    if (p->params.mode != plans[0]->params.mode || p->dscale() != plans[0]->dscale() ||
        p->params.mode == PF_IMPLICIT_LITERAL || p->partial())
      return PF_ERR_UNSUPPORTED;
    need += pf_backward_workspace_bytes(p);
  }
  if (!workspace || workspace_bytes < need || misaligned(workspace, 7)) return PF_ERR_WORKSPACE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool expl = plans[0]->params.mode == PF_EXPLICIT;
  double* ws = static_cast<double*>(workspace);
  for (int32_t first = 0; first < n; first += kMaxJobs) {
    const int32_t cnt = std::min<int32_t>(kMaxJobs, n - first);
    LaunchArgs la;
    std::memset(&la, 0, sizeof(la));
    la.n_jobs = cnt;
    la.kappa_flag = 0.0;
    la.kappa_fp64 = kDefaultKappaFp64;
    la.dscale = plans[0]->dscale();
    la.gws = ws;
    bool has_mask = false;
    int32_t wg = 0;
    for (int32_t j = 0; j < cnt; ++j) {
      const pf_plan* p = plans[first + j];
      const pf_backward_io& f = io[first + j];
      Job& jb = la.jobs[j];
      jb.depth = f.depth;
      jb.mask = f.mask;
      // the first sweep reads the upstream output gradients through the output slots
      jb.normals = const_cast<float*>(f.grad_normals);
      jb.offsets = const_cast<float*>(f.grad_offsets);
      jb.residuals = const_cast<float*>(f.grad_residuals);
      jb.status = nullptr;
      jb.fx = p->intr.fx;
      jb.fy = p->intr.fy;
      jb.cx = p->intr.cx;
      jb.cy = p->intr.cy;
      jb.depth_pitch = int32_t(f.depth_pitch);
      jb.mask_pitch = f.mask ? int32_t(f.mask_pitch) : 0;
      jb.H = int32_t(p->H);
      jb.W = int32_t(p->W);
      jb.k = p->k;
      jb.tile_w = p->tile_w;
      jb.tile_h = p->tile_h;
      jb.n_strips = p->n_strips;
      jb.wg_begin = wg;
      jb.vec_store = 0;
      has_mask = has_mask || f.mask != nullptr;
      wg += p->n_strips * p->n_bands;
      ws += 4 * int64_t(p->H) * p->W;
    }
    la.n_wg = wg;
    const dim3 grid(static_cast<unsigned>(wg));
    const dim3 block(kBlock);
    if (expl) {
      if (has_mask) hipLaunchKernelGGL((fit_planes_fused<double, PF_EXPLICIT, true, true>), grid, block, 0, s, la);
      else hipLaunchKernelGGL((fit_planes_fused<double, PF_EXPLICIT, false, true>), grid, block, 0, s, la);
    } else {
      if (has_mask) hipLaunchKernelGGL((fit_planes_fused<double, PF_IMPLICIT, true, true>), grid, block, 0, s, la);
      else hipLaunchKernelGGL((fit_planes_fused<double, PF_IMPLICIT, false, true>), grid, block, 0, s, la);
    }
    hipError_t err = hipGetLastError();
    if (err == hipSuccess) {
      // the second sweep writes dL/dZ through the normals slot
      for (int32_t j = 0; j < cnt; ++j) la.jobs[j].normals = io[first + j].grad_depth;
      if (has_mask) hipLaunchKernelGGL((grad_depth_fused<true>), grid, block, 0, s, la);
      else hipLaunchKernelGGL((grad_depth_fused<false>), grid, block, 0, s, la);
      err = hipGetLastError();
    }
    if (err != hipSuccess) {
      g_last_hip_error = int(err);
      return PF_ERR_HIP;
    }
  }
  return PF_OK;
}

pf_status pf_fit_planes_backward(const pf_plan* plan, const float* depth, int64_t depth_pitch,
                                 const uint8_t* mask, int64_t mask_pitch,
                                 const float* grad_normals, const float* grad_offsets,
                                 const float* grad_residuals, float* grad_depth, void* workspace,
                                 size_t workspace_bytes, void* stream) {
  if (!plan) return PF_ERR_NULL;
  const pf_backward_io io = {depth, depth_pitch, mask, mask_pitch, grad_normals, grad_offsets,
                             grad_residuals, grad_depth};
  return pf_fit_planes_backward_batch(&plan, &io, 1, workspace, workspace_bytes, stream);
}

pf_status pf_fit_planes_xyz(const pf_plan* plan, const float* depth, int64_t depth_pitch,
                            const uint8_t* mask, int64_t mask_pitch, float* normals,
                            float* offsets, float* residuals, uint8_t* status, void* stream) {
  if (!plan || !depth || !normals || !offsets || !residuals) return PF_ERR_NULL;
  if (plan->params.precision != PF_PREC_FP64 || plan->dscale() > 0.0 ||
      plan->params.mode == PF_IMPLICIT_LITERAL || plan->partial())
    return PF_ERR_UNSUPPORTED;
  if (depth_pitch < plan->W || depth_pitch > INT32_MAX ||
      (mask && (mask_pitch < plan->W || mask_pitch > INT32_MAX)))
    return PF_ERR_PITCH;
  auto misaligned = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 3) != 0; };
  if (misaligned(depth) || misaligned(normals) || misaligned(offsets) || misaligned(residuals))
    return PF_ERR_ALIGNMENT;
  LaunchArgs la;
  std::memset(&la, 0, sizeof(la));
  la.n_jobs = 1;
  la.kappa_flag = plan->params.kappa_flag;
  Job& jb = la.jobs[0];
  jb.depth = depth;
  jb.mask = mask;
  jb.normals = normals;
  jb.offsets = offsets;
  jb.residuals = residuals;
  jb.status = status;
  jb.fx = plan->intr.fx;
  jb.fy = plan->intr.fy;
  jb.cx = plan->intr.cx;
  jb.cy = plan->intr.cy;
  jb.depth_pitch = int32_t(depth_pitch);
  jb.mask_pitch = mask ? int32_t(mask_pitch) : 0;
  jb.H = int32_t(plan->H);
  jb.W = int32_t(plan->W);
  jb.k = plan->k;
  jb.tile_w = plan->tile_w;
  jb.tile_h = plan->tile_h;
  jb.n_strips = plan->n_strips;
  const int n_wg = plan->n_strips * plan->n_bands;
  la.n_wg = n_wg;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const dim3 grid(static_cast<unsigned>(n_wg));
  const dim3 block(kBlock);
  if (plan->params.mode == PF_EXPLICIT) {
    if (mask) hipLaunchKernelGGL((fit_planes_xyz<PF_EXPLICIT, true>), grid, block, 0, s, la);
    else hipLaunchKernelGGL((fit_planes_xyz<PF_EXPLICIT, false>), grid, block, 0, s, la);
  } else {
    if (mask) hipLaunchKernelGGL((fit_planes_xyz<PF_IMPLICIT, true>), grid, block, 0, s, la);
    else hipLaunchKernelGGL((fit_planes_xyz<PF_IMPLICIT, false>), grid, block, 0, s, la);
  }
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) {
    g_last_hip_error = int(err);
    return PF_ERR_HIP;
  }
  return PF_OK;
}

size_t pf_integral_workspace_bytes(const pf_plan* plan) {
  if (!plan) return 0;
  const size_t ld = size_t(plan->W) + 1, P = (size_t(plan->H) + 1) * ld;
  const size_t bands = (size_t(plan->H) + kIntBand - 1) / kIntBand;
  const size_t strips = (size_t(plan->W) + kBlock - 1) / kBlock;
  return sizeof(double) * (size_t(kIntHeader) + 5 * P + 5 * bands * size_t(plan->W) +
                           5 * strips * size_t(plan->H) +
                           bands * strips * size_t(kIntBand * kIntWaves * 5));
}

pf_status pf_integral_images(const pf_plan* plan, const float* depth, int64_t depth_pitch,
                             const uint8_t* mask, int64_t mask_pitch, void* workspace,
                             size_t workspace_bytes, void* stream) {
  if (!plan || !depth) return PF_ERR_NULL;
  if (plan->dscale() > 0.0 || plan->params.mode == PF_IMPLICIT_LITERAL || plan->partial())
    return PF_ERR_UNSUPPORTED;
  if (depth_pitch < plan->W || (mask && mask_pitch < plan->W)) return PF_ERR_PITCH;
  if ((reinterpret_cast<uintptr_t>(depth) & 3) != 0) return PF_ERR_ALIGNMENT;
  if (!workspace || workspace_bytes < pf_integral_workspace_bytes(plan) ||
      (reinterpret_cast<uintptr_t>(workspace) & 7) != 0)
    return PF_ERR_WORKSPACE;
  IntegralArgs ia;
  ia.depth = depth;
  ia.mask = mask;
  ia.depth_pitch = depth_pitch;
  ia.mask_pitch = mask ? mask_pitch : 0;
  ia.H = int32_t(plan->H);
  ia.W = int32_t(plan->W);
  ia.ws = static_cast<double*>(workspace);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const dim3 block(kBlock);
  const unsigned strips = unsigned((plan->W + kBlock - 1) / kBlock);
  const unsigned bands = unsigned((plan->H + kIntBand - 1) / kIntBand);
  const unsigned carry =
      unsigned((5 * (int64_t(kCarryLanes) * plan->W + plan->H) + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(integral_tiles, dim3(strips, bands), block, 0, s, ia);
  hipLaunchKernelGGL(integral_carry, dim3(carry), block, 0, s, ia);
  hipLaunchKernelGGL(integral_final, dim3(strips, bands), block, 0, s, ia);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) {
    g_last_hip_error = int(err);
    return PF_ERR_HIP;
  }
  return PF_OK;
}

pf_status pf_fit_rects(const pf_plan* plan, const void* workspace, size_t workspace_bytes,
                       const int32_t* rects, int64_t n, float* normals, float* offsets,
                       float* residuals, uint8_t* status, void* stream) {
  if (n < 0) return PF_ERR_SHAPE;
  if (n == 0) return PF_OK;
  if (!plan || !workspace || !rects || !normals || !offsets || !residuals) return PF_ERR_NULL;
  if (workspace_bytes < pf_integral_workspace_bytes(plan)) return PF_ERR_WORKSPACE;
  if (plan->params.mode == PF_IMPLICIT_LITERAL || plan->partial()) return PF_ERR_UNSUPPORTED;
  if (n > int64_t(INT32_MAX) * kBlock / 4) return PF_ERR_SHAPE;
  auto misaligned = [](const void* q, uintptr_t m) { return (reinterpret_cast<uintptr_t>(q) & m) != 0; };
  if (misaligned(rects, 3) || misaligned(normals, 3) || misaligned(offsets, 3) ||
      misaligned(residuals, 3))
    return PF_ERR_ALIGNMENT;
  if (misaligned(workspace, 7)) return PF_ERR_WORKSPACE;
  RectArgs ra;
  ra.ws = static_cast<const double*>(workspace);
  ra.rects = rects;
  ra.normals = normals;
  ra.offsets = offsets;
  ra.residuals = residuals;
  ra.status = status;
  ra.n = n;
  ra.H = int32_t(plan->H);
  ra.W = int32_t(plan->W);
  ra.fx = plan->intr.fx;
  ra.fy = plan->intr.fy;
  ra.cx = plan->intr.cx;
  ra.cy = plan->intr.cy;
  ra.kappa_flag = plan->params.kappa_flag;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const dim3 grid(unsigned((n + kBlock - 1) / kBlock)), block(kBlock);
  if (plan->params.mode == PF_EXPLICIT)
    hipLaunchKernelGGL((fit_rects_kernel<PF_EXPLICIT>), grid, block, 0, s, ra);
  else
    hipLaunchKernelGGL((fit_rects_kernel<PF_IMPLICIT>), grid, block, 0, s, ra);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) {
    g_last_hip_error = int(err);
    return PF_ERR_HIP;
  }
  return PF_OK;
}

}  // extern "C"
