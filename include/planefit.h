/*
 * planefit: dense per-pixel plane fitting to depth images on AMD Instinct
 * MI355X (gfx950), after Papadakis & Willis, "Real-Time Surface Fitting to
 * RGBD Sensor Data" (2017).
 *
 * What is computed (Sec. II).  Each pixel (x, y) of a depth image Z with a
 * pinhole camera (fx, fy, cx, cy) has the ray tangents
 *     u = tan(theta_x) = (x - cx)/fx,   v = tan(theta_y) = (y - cy)/fy   (Eq. 10)
 * and the back-projected point P = Z (u, v, 1) (Eq. 1, Eq. 11).  Dividing the
 * plane equation aX + bY + cZ + d = 0 by Z gives a u + b v + c + d/Z = 0
 * (Eq. 12): the coefficients (a, b, c) multiply camera-only quantities and d
 * multiplies the disparity w = 1/Z.  For every pixel the library fits a plane
 * to the k x k window centred on it:
 *
 *   PF_IMPLICIT  minimises sum_i (a u_i + b v_i + c + d w_i)^2 with
 *                |(a, b, c)| = 1 (Sec. II-A, scatter matrix of Eq. 14).
 *   PF_EXPLICIT  minimises sum_i (a u_i + b v_i + c - w_i)^2 (Sec. II-B,
 *                Eq. 15-16); the plane is a X + b Y + c Z - 1 = 0.
 *
 * The camera-only window moments (sum u^2, sum u v, sum u, sum v^2, sum v,
 * N) are fixed once the calibration and k are known (Sec. II-A/B); per frame
 * only window sums of w, u w, v w, w^2 and a validity count are needed, and
 * they are taken from integral images (Sec. II-C) built on the GPU.
 *
 * Outputs per pixel, for the plane n . P + d = 0 with |n| = 1 and d >= 0
 * (the normal faces the camera):
 *   normals   [3][H][W] float32, channel-planar (n_x plane, n_y plane, n_z plane)
 *   offsets   [H][W]    float32, d in the depth unit
 *   residuals [H][W]    float32, RMS over the window of (n . P_i + d) / Z_i
 *                       (point-to-plane distance over depth: dimensionless)
 *   status    [H][W]    uint8 (optional): bit 0 = invalid window,
 *                       bit 1 = ill-conditioned normal (implicit mode,
 *                       kappa = l3/(l2 - l1) above pf_params.kappa_flag),
 *                       bit 2 = solved in FP64 (compensated precision only).
 * A pixel is valid iff its mask byte (if a mask is given) is non-zero and its
 * depth is finite and > 0.  A window is valid iff all k*k pixels lie inside
 * the image and are valid; invalid windows get NaN outputs and status bit 0.
 * That is a result, not an error.  Results are specified for depths in
 * [1e-3, 1e3] (any unit, consistently used).
 *
 * Memory: every image pointer given to pf_fit_planes is a DEVICE pointer owned
 * by the caller; images are row-major with a pitch in elements.  Calls are
 * enqueue-only on the given HIP stream and return before the GPU finishes;
 * the caller keeps the buffers alive until the stream passes this point.
 * No function aborts or throws; errors come back as pf_status codes.
 */
#ifndef PLANEFIT_H
#define PLANEFIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PF_OK = 0,
  PF_ERR_NULL = 1,        /* a required pointer is NULL */
  PF_ERR_SHAPE = 2,       /* H or W < 1, H or W > 65535, or H*W > 2^31 */
  PF_ERR_WINDOW = 3,      /* k not odd, k < 3, k > 63, or k > min(H, W) */
  PF_ERR_INTRINSICS = 4,  /* fx, fy not finite and > 0, or cx, cy not finite */
  PF_ERR_PITCH = 5,       /* a pitch is smaller than W */
  PF_ERR_ALIGNMENT = 6,   /* a float pointer is not 4-byte aligned */
  PF_ERR_WORKSPACE = 7,   /* workspace missing or smaller than required */
  PF_ERR_UNSUPPORTED = 8, /* mode / precision / flag value not supported */
  PF_ERR_HIP = 9          /* the HIP runtime reported an error (pf_last_hip_error) */
} pf_status;

/* Pinhole intrinsics in pixels (Eq. 1 with the lens correction delta = 0). */
typedef struct {
  double fx, fy, cx, cy;
} pf_intrinsics;

/* PF_IMPLICIT_LITERAL: the implicit fit with the constraint exactly as Sec. II-A
 * states it, |(a, b, c, d)| = 1 (smallest eigenvector of the 4x4 scatter of
 * Eq. 14), scaled to a unit normal afterwards.  It mixes units (d multiplies
 * 1/Z), so its result depends on the depth unit; PF_IMPLICIT constrains
 * |(a, b, c)| = 1 instead.  For comparison: FP64 only, kappa_flag must be 0,
 * and only pf_fit_planes / pf_fit_planes_batch accept it (PF_ERR_UNSUPPORTED
 * elsewhere). */
enum { PF_IMPLICIT = 0, PF_EXPLICIT = 1, PF_IMPLICIT_LITERAL = 2 };

/* Arithmetic of the window moments and the per-pixel solve.
 *  PF_PREC_FP64: disparity integrands, integral-image sums and the solve in
 *                FP64 (MI355X runs FP64 vector FMA at the FP32 rate); the
 *                accurate default.
 *  PF_PREC_FP32: everything in FP32; the throughput reference.  Integral-image
 *                differences lose digits to cancellation, so its errors are
 *                reported, not held to the FP64 oracle's tolerances.
 *  PF_PREC_COMPENSATED: FP32 arithmetic with compensated (two-float, ~48-bit)
 *                integral-image sums and window moments and an FP32 solve;
 *                implicit windows whose FP32 eigen-condition kappa exceeds
 *                pf_params.kappa_fp64 are solved again in FP64 (status bit 2). */
enum { PF_PREC_FP64 = 0, PF_PREC_FP32 = 1, PF_PREC_COMPENSATED = 2 };

/* pf_params.flags.
 *  PF_FLAG_DISPARITY: the input image holds disparity D instead of depth, with
 *    1/Z = D * disparity_scale (a stereo or structured-light sensor reports
 *    D = f b / Z, so disparity_scale = 1 / (f b)).  The integrands of Eq. 14
 *    are then linear in the input: w = D * disparity_scale, no division.
 *    Validity: D finite and > 0.  Offsets are in the unit of 1/disparity_scale.
 *    Supported by pf_fit_planes, pf_fit_planes_batch and the backward pass
 *    (which then returns dL/dD); PF_ERR_UNSUPPORTED for pf_fit_planes_xyz and
 *    the rectangle fits. */
enum { PF_FLAG_DISPARITY = 1 };

typedef struct {
  int32_t window;     /* k: odd, 3 <= k <= 63, k <= min(H, W) */
  int32_t mode;       /* PF_IMPLICIT or PF_EXPLICIT */
  int32_t precision;  /* PF_PREC_FP64 or PF_PREC_FP32 */
  int32_t flags;      /* 0 or PF_FLAG_DISPARITY */
  double kappa_flag;  /* implicit mode: set status bit 1 where kappa > this; 0 = never */
  double kappa_fp64;  /* PF_PREC_COMPENSATED, implicit: FP64 re-solve where the FP32
                         kappa exceeds this (0 = 100); ignored otherwise */
  double disparity_scale;  /* PF_FLAG_DISPARITY: 1/Z = D * disparity_scale (finite, > 0);
                              ignored otherwise */
  int32_t min_valid;  /* partial windows: 0 (or >= k*k) = the full-window rule: every
                         pixel of the window must be valid.  3 <= min_valid < k*k: a
                         window is fitted from its valid pixels alone when there are at
                         least min_valid of them and they do not all lie on one line of
                         the pixel grid (the plane is then determined); the residual is
                         the RMS over those pixels.  The camera-only moments of Sec.
                         II-A/B are then sums over the valid pixels, carried by the sweep
                         as two extra integer channels.  FP64, PF_IMPLICIT/PF_EXPLICIT,
                         pf_fit_planes and pf_fit_planes_batch only (PF_ERR_UNSUPPORTED
                         otherwise); 1, 2 or < 0 is PF_ERR_UNSUPPORTED. */
} pf_params;

typedef struct pf_plan pf_plan;

/* Host only.  Validates the camera, frame size and parameters, precomputes the
 * camera-only window moments for (camera, k) (Sec. II-A/B) and the launch
 * geometry.  Allocates host memory only (no device memory).  The plan is
 * immutable; it may be shared by threads and streams.  *out is set to NULL on
 * error. */
pf_status pf_plan_create(const pf_intrinsics* intr, int64_t height, int64_t width,
                         const pf_params* params, pf_plan** out);

/* Accepts NULL. */
void pf_plan_destroy(pf_plan* plan);

/* Bytes of device workspace pf_fit_planes needs with this plan (0 for the
 * fused path, which keeps its integral images on chip). */
size_t pf_plan_workspace_bytes(const pf_plan* plan);

/* Camera-only moments of the window centred at pixel (x0, y0), in the paper's
 * uncentred form: out = [sum u^2, sum u v, sum u, sum v^2, sum v, N] (the
 * upper-left 3x3 block of Eq. 14, equal to the matrix of Eq. 16).  Host only;
 * evaluated from the plan's closed form, no summation.  Returns PF_ERR_NULL
 * for NULL arguments. */
pf_status pf_plan_camera_moments(const pf_plan* plan, int64_t x0, int64_t y0, double out[6]);

/* Enqueue the per-pixel fits of one frame on `stream` (a hipStream_t; NULL =
 * the default stream).
 *   depth      device float[H][depth_pitch], depth per pixel (0 / NaN = no data)
 *   mask       device uint8[H][mask_pitch] or NULL; 0 marks a pixel invalid
 *   normals    device float[3][H][W]
 *   offsets    device float[H][W]
 *   residuals  device float[H][W]
 *   status     device uint8[H][W] or NULL
 *   workspace  device buffer of at least pf_plan_workspace_bytes() (may be
 *              NULL when that is 0)
 * Argument checks run on the host before anything is enqueued. */
pf_status pf_fit_planes(const pf_plan* plan, const float* depth, int64_t depth_pitch,
                        const uint8_t* mask, int64_t mask_pitch, float* normals,
                        float* offsets, float* residuals, uint8_t* status, void* workspace,
                        size_t workspace_bytes, void* stream);

/* Output rows per workgroup of the plan's launches (its band height); 0 for NULL. */
int32_t pf_plan_band_height(const pf_plan* plan);

/* Launch shapes (tiling of the fused kernel): 0 = rounds of 4 rows and runs of
 * 4 outputs per thread, compiled for four workgroups per compute unit; 1 =
 * the same tiling compiled for two (twice the registers; a kernel that still
 * fits four runs four); 2 = rounds of 8 rows and runs of 8 outputs per thread
 * at two workgroups per compute unit.  Shapes 1 and 2 apply to PF_PREC_FP64 implicit and explicit
 * full-window plans; every other plan runs shape 0.  A new plan runs shape 1
 * when it is a PF_PREC_FP64 full-window PF_IMPLICIT plan and shape 0
 * otherwise.  Shapes 0 and 1 give bit-identical results at the same band
 * height; otherwise results do not depend on the shape beyond the accuracy of
 * the path (the band height moves which pixels share a reference disparity). */
int32_t pf_plan_shape(const pf_plan* plan);  /* -1 for NULL */

/* A new plan equal to `plan` except for its launch shape: `band_height` output
 * rows per workgroup (clamped to H; 0 = the plan's rule for that shape) and
 * launch shape `shape` (-1 = keep).  `plan` is not modified; the new plan is
 * destroyed with pf_plan_destroy.  PF_ERR_NULL for NULL arguments,
 * PF_ERR_SHAPE for band_height < 0, PF_ERR_UNSUPPORTED for a shape the plan's
 * mode and precision do not offer. */
pf_status pf_plan_derive(const pf_plan* plan, int32_t band_height, int32_t shape,
                         pf_plan** out);

/* Autotuning of the launch shape (beside the plan's built-in heuristic): times
 * pf_fit_planes on the caller's frame and buffers with a private copy of the
 * plan for each candidate launch shape (0, 1, 2 where the plan offers them)
 * and band height (output rows per workgroup: 4, 6, 8, 12, 16, 20, 24, 32,
 * 48, 64, up to H, whole rounds of the shape's rows), and returns the fastest
 * in *chosen_band_height and *chosen_shape (each optional, written only on
 * success); apply them with pf_plan_derive.  `plan` itself is never modified,
 * so it stays safe to share between threads and streams.  Arguments as
 * pf_fit_planes; the outputs are overwritten with a valid fit of the frame.
 * Blocks the calling thread until `stream` has run the timing launches (not
 * for use under stream capture). */
pf_status pf_plan_autotune(const pf_plan* plan, const float* depth, int64_t depth_pitch,
                           const uint8_t* mask, int64_t mask_pitch, float* normals,
                           float* offsets, float* residuals, uint8_t* status, void* stream,
                           int32_t* chosen_band_height, int32_t* chosen_shape);

/* Device buffers of one frame for pf_fit_planes_batch (same meaning, layout and
 * ownership as the arguments of pf_fit_planes). */
typedef struct {
  const float* depth;
  int64_t depth_pitch;
  const uint8_t* mask;   /* or NULL */
  int64_t mask_pitch;
  float* normals;        /* [3][H][W] */
  float* offsets;        /* [H][W] */
  float* residuals;      /* [H][W] */
  uint8_t* status;       /* [H][W] or NULL */
} pf_frame_io;

/* Enqueue the fits of n frames (Sec. II-C: many fits from one pass over each
 * frame) in as few launches as possible: up to 32 frames per kernel launch,
 * of any sizes and window sizes, each described by its own plan.  All plans
 * must share mode, precision, kappa_flag, kappa_fp64, the disparity setting and
 * the launch shape, and be all partial-window plans or all full-window ones
 * (else PF_ERR_UNSUPPORTED); partial-window plans may differ in min_valid.  Every
 * frame is checked on the host as in pf_fit_planes before anything is
 * enqueued; n = 0 is a no-op.  No workspace is needed.
 * Band heights are planned for the whole batch (pf_batch_band_heights): a plan
 * whose band height is the default rule's may run taller bands in a batch that
 * holds more workgroups than the chip keeps resident.  A frame's outputs depend
 * on its band height at the rounding level only (well inside the parity bar);
 * fitted alone with the height pf_batch_band_heights reports for it (or with a
 * plan whose height is set, pf_plan_derive), it comes out bit for bit the same
 * as in the batch.  Frames within a launch start in order of decreasing window
 * size, which does not affect results. */
pf_status pf_fit_planes_batch(const pf_plan* const* plans, const pf_frame_io* io, int32_t n,
                              void* stream);

/* The band height (output rows per workgroup) each frame of a batch of n plans
 * runs with in pf_fit_planes_batch and the queued batch calls: band_heights[i]
 * for plans[i] (host array of n entries, written on success).  A plan whose
 * height was set (pf_plan_derive with band_height > 0, an autotuned height),
 * whose launch shape has 8-row rounds, or that is not an FP64 full-window
 * implicit or explicit fit keeps it.  The others start from the default rule
 * (about one workgroup per resident slot for the frame alone,
 * pf_plan_band_height); while the batch would hold more workgroups than four per
 * compute unit of the current device, the plan with the largest window (on
 * ties the lowest height, then the first such plan) whose height is below 12
 * rows and below its frame's gets 4 more rows (at most the frame's height).
 * Host only: no GPU work, nothing enqueued.  PF_ERR_NULL for a NULL pointer,
 * PF_ERR_SHAPE for n < 0; n = 0 is a no-op. */
pf_status pf_batch_band_heights(const pf_plan* const* plans, int32_t n, int32_t* band_heights);

/* Bytes of device workspace pf_fit_planes_batch_queued needs for n frames (a
 * 256-byte queue header and one job record per frame); 0 for n <= 0. */
size_t pf_batch_workspace_bytes(int32_t n);

/* The fits of n frames (any number, sizes and window sizes) in ONE persistent
 * kernel launch (Sec. II-C: many fits from one pass over each frame).  The grid
 * is the chip's resident workgroups; each workgroup pulls its next work item (a
 * band x strip tile of one frame, largest windows first) from a counter in
 * `workspace` until all items are done.  The job table and the counter are
 * written into `workspace` by small setup launches (one per 32 frames) whose
 * arguments carry the table, so the call records into a HIP graph as kernel
 * nodes only and every replay starts from a fresh queue.  Arguments, checks,
 * plan compatibility and results are those of pf_fit_planes_batch (bit for bit
 * the same outputs).  Up to 32 frames fit in one launch's arguments: such a
 * batch is that single launch (the workspace is then not used).  With the
 * environment variable PF_QUEUE_DEBUG set, each persistent launch prints its
 * grid (workgroups per CU x CUs, work items) to stderr.
 *   workspace  device, >= pf_batch_workspace_bytes(n), 256-byte aligned
 *              (else PF_ERR_WORKSPACE); owned by the caller, rewritten by every
 *              call: calls that overlap in time need separate workspaces. */
pf_status pf_fit_planes_batch_queued(const pf_plan* const* plans, const pf_frame_io* io,
                                     int32_t n, void* workspace, size_t workspace_bytes,
                                     void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): pf_fit_planes_batch_queued
 * with its queue header and job table in a scratch array of the library's own
 * static device memory (one array per GPU, about 31 KB, held until the process
 * ends) instead of a caller's workspace.  It calls no hipMalloc, hipFree or
 * other allocating routine; the array's device address is resolved once per
 * device, on the first call with that device current.  n may be at most
 * pf_batch_noalloc_max_frames() (256; larger n returns PF_ERR_WORKSPACE before
 * anything is enqueued).  Every call on a GPU shares that GPU's array, which
 * keeps the last call's table: calls that overlap in time on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 * Arguments, checks and results are otherwise those of
 * pf_fit_planes_batch_queued. */
pf_status pf_fit_planes_batch_queued_noalloc(const pf_plan* const* plans, const pf_frame_io* io,
                                             int32_t n, void* stream);
int32_t pf_batch_noalloc_max_frames(void);

/* Bytes of device workspace pf_fit_planes_backward needs: 32 * H * W (the four
 * per-window moment gradients in FP64). */
size_t pf_backward_workspace_bytes(const pf_plan* plan);

/* Backward pass of pf_fit_planes for one frame: the gradient of a scalar loss
 * with respect to the depth image, given the loss's gradients with respect to
 * the outputs.  The solve of Eq. 14-16 is differentiated per window (FP64,
 * whatever the plan's precision; for the implicit fit through the derivative of
 * the smallest eigenpair, d n = -(C - l1 I)^+ dC n), and the window sums of the
 * integral images (Sec. II-C) are differentiated by the same box-sum sweep run
 * over the per-window gradients; finally w = 1/Z is chained to Z.
 *   depth, mask            as given to pf_fit_planes
 *   grad_normals           device float[3][H][W] or NULL (zero)
 *   grad_offsets           device float[H][W] or NULL (zero)
 *   grad_residuals         device float[H][W] or NULL (zero)
 *   grad_depth             device float[H][W] (written, dense pitch W)
 *   workspace              device buffer >= pf_backward_workspace_bytes(plan),
 *                          8-byte aligned; contents undefined afterwards
 * Invalid windows and windows whose normal is not differentiable (a repeated
 * smallest eigenvalue) contribute nothing; invalid pixels get 0.  Upstream
 * gradients at invalid windows are ignored (their outputs are NaN). */
pf_status pf_fit_planes_backward(const pf_plan* plan, const float* depth, int64_t depth_pitch,
                                 const uint8_t* mask, int64_t mask_pitch,
                                 const float* grad_normals, const float* grad_offsets,
                                 const float* grad_residuals, float* grad_depth, void* workspace,
                                 size_t workspace_bytes, void* stream);

/* Buffers of one frame for pf_fit_planes_backward_batch (same meaning, layout
 * and ownership as the arguments of pf_fit_planes_backward). */
typedef struct {
  const float* depth;
  int64_t depth_pitch;
  const uint8_t* mask;            /* or NULL */
  int64_t mask_pitch;
  const float* grad_normals;      /* [3][H][W] or NULL */
  const float* grad_offsets;      /* [H][W] or NULL */
  const float* grad_residuals;    /* [H][W] or NULL */
  float* grad_depth;              /* [H][W], written */
} pf_backward_io;

/* The backward pass of n frames in as few launches as possible (two launches
 * per group of up to 32 frames of any sizes and window sizes; Sec. II-C: many
 * fits from one pass over each frame).  All plans must share the mode (else
 * PF_ERR_UNSUPPORTED).  The workspace must hold the sum over the frames of
 * pf_backward_workspace_bytes (8-byte aligned); frame i uses its own region,
 * in order.  Each frame is checked on the host as in pf_fit_planes_backward
 * before anything is enqueued; n = 0 is a no-op.  Results are bit-identical to
 * one pf_fit_planes_backward call per frame. */
pf_status pf_fit_planes_backward_batch(const pf_plan* const* plans, const pf_backward_io* io,
                                       int32_t n, void* workspace, size_t workspace_bytes,
                                       void* stream);

/* The standard formulation, for comparison with the RGBD one (Sec. II, Eq. 3-9):
 * the same per-pixel k x k window fits computed from window sums of the
 * back-projected points P = Z (u, v, 1) and their products (nine
 * depth-dependent channels instead of four).
 *   PF_IMPLICIT: unit normal of the smallest eigenvalue of the window's point
 *                covariance (Eq. 3-6, |n| = 1), d = -n . centroid;
 *   PF_EXPLICIT: Z = a X + b Y + c by least squares (Eq. 7-9); the plane
 *                (a, b, -1) . P + c = 0 normalised.
 * Orientation d >= 0.  residuals = RMS point-to-plane distance over the window
 * (in the depth unit, not divided by Z as in pf_fit_planes).  Validity, NaN
 * outputs, status bits 0 and 1 (kappa of the covariance) and the buffer
 * contract are those of pf_fit_planes.  The plan must use PF_PREC_FP64 (else
 * PF_ERR_UNSUPPORTED); its camera, k and mode are used.  No workspace. */
pf_status pf_fit_planes_xyz(const pf_plan* plan, const float* depth, int64_t depth_pitch,
                            const uint8_t* mask, int64_t mask_pitch, float* normals,
                            float* offsets, float* residuals, uint8_t* status, void* stream);

/* Fits to arbitrary rectangles of one frame: the paper's own use of integral
 * images (Sec. II-C), for many fits to regions of a frame (tiles, quadtree
 * cells, segmentation candidates) instead of one per pixel.
 *
 * pf_integral_images builds, in FP64 on the GPU, the integral images of the
 * four depth-dependent moments of Eq. 14 (centred on the frame's reference
 * disparity) and of the valid count into the caller's workspace (three
 * launches over tiles of 256 columns by 16 rows: tile totals, their scans,
 * then each tile's own prefix plus its carries; the depth is read twice and
 * each image entry written once).  pf_fit_rects then fits one plane per rectangle from the four
 * corners of each image; the camera-only moments of a w x h rectangle are in
 * closed form (Sec. II-A/B).  Mode (implicit / explicit), kappa_flag and the
 * camera come from the plan; its window is not used; arithmetic is FP64.
 *   workspace  device, >= pf_integral_workspace_bytes(plan), 8-byte aligned;
 *              written by pf_integral_images, read by pf_fit_rects (both take
 *              its size in bytes and return PF_ERR_WORKSPACE when it is smaller
 *              than the plan's frame needs)
 *   rects      device int32 [n][4] = (x0, y0, w, h): columns x0 .. x0+w-1,
 *              rows y0 .. y0+h-1
 *   normals    device float [3][n]; offsets, residuals float [n]; status
 *              uint8 [n] or NULL
 * A rectangle is valid iff w, h >= 2, it lies in the image and every pixel in
 * it is valid; other rectangles get NaN outputs and status bit 0 (not an
 * error).  Outputs follow pf_fit_planes (orientation, residual, status bit 1). */
size_t pf_integral_workspace_bytes(const pf_plan* plan);
pf_status pf_integral_images(const pf_plan* plan, const float* depth, int64_t depth_pitch,
                             const uint8_t* mask, int64_t mask_pitch, void* workspace,
                             size_t workspace_bytes, void* stream);
pf_status pf_fit_rects(const pf_plan* plan, const void* workspace, size_t workspace_bytes,
                       const int32_t* rects, int64_t n, float* normals, float* offsets,
                       float* residuals, uint8_t* status, void* stream);

/* Static description of a status code. */
const char* pf_status_string(pf_status s);

/* The hipError_t behind the most recent PF_ERR_HIP on this thread (0 if none). */
int pf_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif
