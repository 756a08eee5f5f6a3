/*
 * mpbp.h - C-ABI of the MI355X (gfx950) library for the multi-peak Bragg ptychography
 * (MPBP) objective and its gradient.
 *
 * The operation (Kandel et al., "Imaging extended single crystal lattice distortion
 * fields with multi-peak Bragg ptychography", sections 2-3):
 *
 *   eq. (1), eq. (3)  O_m(r)  = alpha_m * chi(r) * exp(i G_m . u(r))   (G_m in rad/nm)
 *   eq. (2)           I_{m,j} = | F R_m diag(P_m) S_{m,j} O_m |^2 + b_{m,j}
 *   eq. (4)           f       = 1/2 sum_{m,j} || I_{m,j}^{1/2} - y_{m,j}^{1/2} ||^2
 *   eq. (11)          minibatch: f and its gradient summed over a subset of the frames
 *
 * S_{m,j} places the probe support (probe_n x probe_n) at scan position j of peak m's
 * raster.  The probe is constant along the incident beam x3 (section 4), or given per
 * slice under MPBP_PROBE_3D.  R_m projects the illuminated object along the exit beam:
 * slice z is offset laterally by the integer shear s_m(z) = round_half_away((z - nz/2)
 * * t_m), or, under MPBP_SHEAR_LINEAR, by the exact offset (z - nz/2) * t_m with
 * bilinear weights over its four neighbouring pixels; all inside a D_m x D_m exit-wave
 * window whose probe support starts at c_m = (D_m - probe_n) / 2.  F is the
 * orthonormal 2D DFT, kernel exp(-2 pi i k.x / D), DC at index [0][0] (no shift); the
 * measured intensities y and the background b use the same unshifted layout.  b = 0
 * unless set with mpbp_set_background.
 *
 * Layouts (all row-major, x fastest; "(dev)" = device memory of the plan's GPU,
 * "(host)" = host memory).  The caller owns every buffer it passes.
 *   u       (dev) float [3][nz][ny][nx]       displacement components (x, y, z), nm
 *                 ([3][1][ny][nx] under MPBP_Z_TIED)
 *   chi     (dev) float [nz][ny][nx]          amplitude chi >= 0 ([1][ny][nx] under
 *                 MPBP_Z_TIED)
 *   alpha   (dev) float [n_peaks]             per-peak scale alpha_m > 0
 *   probe   (dev) complex64 [n_peaks][probe_n][probe_n], interleaved (re, im) floats
 *                 ([n_peaks][nz][probe_n][probe_n] under MPBP_PROBE_3D)
 *   y       (dev) float, ragged: peaks concatenated, peak m holds
 *                 [frames_m][D_m][D_m]; offsets from mpbp_tables (y_off)
 *   frames  (host) int32 [n_frames]: global frame ids (peak-major, raster order within
 *                 a peak: id = y_off-order index), no duplicates; NULL = all frames
 * Gradients are written (not accumulated) in the layouts of u, chi and alpha.
 *
 * Calls on one plan must be serialised by the caller; work is enqueued on `stream`
 * (a hipStream_t; NULL = the default stream) and returns without waiting, except
 * where stated.  Every argument is validated on the host before anything is enqueued,
 * so a call that returns an error has done no work.  No C++ exception crosses this
 * interface.  mpbp_last_error() describes the last failure of the calling thread.
 */
#ifndef MPBP_H
#define MPBP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpbp_plan_t* mpbp_plan;

typedef enum {
  MPBP_OK = 0,
  MPBP_ERR_INVALID = 1,      /* null pointer, bad option, bad or duplicate frame id     */
  MPBP_ERR_SHAPE = 2,        /* a size is out of range                                  */
  MPBP_ERR_FOOTPRINT = 3,    /* a sheared probe support leaves its detector window      */
  MPBP_ERR_DEVICE = 4,       /* HIP failure, or a compute call on a host-only plan      */
  MPBP_ERR_NOMEM = 5,        /* device or host allocation failed                        */
  MPBP_ERR_UNSUPPORTED = 6,  /* valid but outside what the kernels implement            */
  MPBP_ERR_INTERNAL = 7      /* a device-side consistency check failed                  */
} mpbp_status;

/* One Bragg peak m (sections 2-3; eq. (2) operators S and R). */
typedef struct {
  double  g[3];              /* G_m in rad/nm, lab frame (x1, x2, x3); phase = G_m . u     */
  double  shear[2];          /* t_m = (t_y, t_x): exit-beam lateral offset per slice, voxels*/
  int32_t det;               /* D_m: detector / exit-wave window size (square)             */
  int32_t scan_n[2];         /* raster (rows, cols); local frame j = row * cols + col      */
  int32_t scan_step[2];      /* raster step (rows, cols), voxels                           */
  int32_t scan_origin[2];    /* object voxel of the probe support's top-left, frame 0     */
  double  map[4];            /* with MPBP_DETECTOR_MAP: the 2 x 2 map M (row-major) of the
                                probe window's lateral voxel coordinates (y, x) to exit-
                                wave pixels of this peak's detector frame; ignored otherwise */
} mpbp_peak;

typedef struct {
  int32_t nz, ny, nx;        /* object grid                                                */
  int32_t probe_n;           /* probe support (square)                                     */
  int32_t n_peaks;
  const mpbp_peak* peaks;    /* (host) [n_peaks]; copied by mpbp_plan_create               */
  uint32_t flags;            /* 0, or any of MPBP_Z_TIED, MPBP_PROBE_3D, MPBP_SHEAR_LINEAR,
                                MPBP_DETECTOR_MAP                                          */
} mpbp_problem;

/* Problem flags.
   MPBP_Z_TIED: the membrane parameterisation (sections 3-4: unknowns per lateral pixel,
   constant along the incident beam x3).  u is then (dev) float [3][1][ny][nx] and chi
   [1][ny][nx], both holding for every slice z; grad_u and grad_chi have the same shapes
   and hold the z-sums of the per-voxel gradients. */
enum { MPBP_Z_TIED = 1 };
/* MPBP_PROBE_3D: per-peak 3D illumination volumes (section 2: the probe satisfying each
   Bragg condition is three-dimensional): probe is then (dev) complex64
   [n_peaks][nz][probe_n][probe_n], the probe of every slice z on the same probe_n x
   probe_n support of scan position j, and eq. (2) reads diag(P_m) as P_m[z] on slice z.
   May be combined with MPBP_Z_TIED. */
enum { MPBP_PROBE_3D = 2 };
/* MPBP_SHEAR_LINEAR: the exit-beam operator R interpolates (section 2: R rotates and
   interpolates the illuminated object into the detector frame).  Slice z's lateral
   offset (z - nz/2) * t_m is kept fractional: with s0 = floor and f the fraction per
   axis, the slice lands on offsets s0 + (dy, dx), dy, dx in {0, 1}, with the bilinear
   weights (1 - f_y or f_y) (1 - f_x or f_x) (rounded offsets otherwise).  mpbp_tables
   then reports s0; footprints are one pixel wider per axis. */
enum { MPBP_SHEAR_LINEAR = 4 };
/* MPBP_DETECTOR_MAP: R rotates and scales each slice into the peak's detector frame and
   interpolates it there (section 2: the detector frames differ per Bragg peak, and so may
   the exit-wave pixel size that each detector's sampling dictates).  With M_m = peaks[m].map
   (invertible), slice z's probe-window point (a, b) lands on the exit-wave point
     q = M_m ((a, b) - probe_n/2) + (c_m + probe_n/2) + (z - nz/2) t_m
   (t_m = shear, in exit-wave pixels), and each exit-wave pixel takes the bilinear
   interpolation of the illuminated slice P_z . O_z (zero off the probe support and the
   object) at its pre-image; the slices are summed.  M_m = identity gives the model of
   MPBP_SHEAR_LINEAR.  The footprint is the bounding box of the mapped support widened by
   one sample; MPBP_ERR_FOOTPRINT if it leaves the window.  May be combined with
   MPBP_Z_TIED and MPBP_PROBE_3D, not with MPBP_SHEAR_LINEAR; batched fused path only
   (the plain path returns MPBP_ERR_UNSUPPORTED).  mpbp_tables still reports the rounded
   offsets. */
enum { MPBP_DETECTOR_MAP = 8 };

/* Options of mpbp_set_option / mpbp_get_option. */
enum {
  MPBP_OPT_PATH = 1,         /* 0 = batched fused path (default), 1 = plain path: one
                                launch per stage per peak and scan position              */
  MPBP_OPT_GRAPH = 2,        /* 1 (default): a full-batch fused call (frames = NULL) is
                                captured into a hipGraph on first use for its set of
                                buffer addresses and replayed afterwards; the detector-
                                size classes run as parallel graph branches.  At most 8
                                graphs are kept per plan (least recently used dropped,
                                after a device synchronisation).  Subset calls, the plain
                                path and profiled calls launch directly; direct launches
                                also run the classes side by side on the plan's own
                                streams (joined into the caller's stream).  0 = direct
                                launches always (and drop the plan's graphs).  Results
                                are bitwise those of direct launches.                    */
  MPBP_OPT_XCD_ORDER = 3,    /* 1 = hand each XCD a contiguous band of frames (default) */
  MPBP_OPT_PROFILE = 4,      /* 1 = record HIP events around every kernel stage on the
                                call's stream (read with mpbp_stage_times); 2 = around
                                the frame stage (MPBP_STAGE_FRAMES) only, the least
                                added to the step; default 0.  Profiled calls launch
                                directly (no graph replay)                               */
  MPBP_OPT_GRAD_BATCH = 5,   /* footprint gradients the back-projection kernel reads at
                                once: 1, 2, 4, 8 (default) or 16; the run gather takes
                                at least 4, the per-slice walk at most 4; set by
                                mpbp_autotune                                            */
  MPBP_OPT_GRAD_TILE = 6,    /* back-projection tile: 16 (16 x 4 voxels, default) or 8
                                (8 x 8 voxels on a grid aligned with the first peak's
                                raster); set by mpbp_autotune.  Neither this nor
                                MPBP_OPT_GRAD_BATCH affects MPBP_DETECTOR_MAP plans,
                                whose back-projection walks each frame once per slice */
  MPBP_OPT_RUNS = 7          /* 1 (default): with one probe for all slices and rounded
                                offsets (none of MPBP_PROBE_3D, MPBP_SHEAR_LINEAR and
                                MPBP_DETECTOR_MAP),
                                eq. (2)'s sum over slices is grouped into runs of
                                consecutive slices with equal exit-beam offset: the
                                objects are summed over each run once per call, every
                                frame projects the run sums, and the back-projection sums
                                the frames once per run and applies the chain rule per
                                slice.  0: both per slice.  The back-projection gives
                                bitwise the same results either way; the projection
                                rounds the regrouped sums differently.                   */
};

/* Kernel stages timed under MPBP_OPT_PROFILE. */
enum {
  MPBP_STAGE_OBJECT = 0,     /* per-peak object build, eq. (1)/(3)                        */
  MPBP_STAGE_FRAMES = 1,     /* per-frame transforms, residual and adjoint, eq. (2)-(4)  */
  MPBP_STAGE_GRAD = 2,       /* back-projection gather and chain rule                     */
  MPBP_STAGE_FINALIZE = 3,   /* FP64 reductions                                           */
  MPBP_STAGE_PLAIN = 4,      /* the whole plain path (MPBP_OPT_PATH = 1)                 */
  MPBP_STAGE_PROJECT = 5,    /* per-frame probe product and sheared projection, eq. (2)  */
  MPBP_NUM_STAGES = 6
};

/* Validate `problem`, build the integer tables (scan offsets, shear offsets, ragged y
   offsets) and, for device >= 0, allocate the plan's device workspace on that GPU.
   device = -1 makes a host-only plan: tables and validation only; compute calls then
   return MPBP_ERR_DEVICE.  Errors: MPBP_ERR_INVALID (null pointers, unknown flags),
   MPBP_ERR_SHAPE (non-positive sizes, D outside the supported set), MPBP_ERR_FOOTPRINT,
   MPBP_ERR_DEVICE, MPBP_ERR_NOMEM.  On success *out owns the plan.
   The device workspace holds the per-peak objects (8 n_peaks nz ny nx bytes), two
   footprint slots per frame (its exit wave and that wave's gradient, 8 F_y F_x bytes
   each, F = probe_n plus the peak's shear span per axis), the per-frame losses and the
   per-tile alpha partials: about 0.57 GB for 3 peaks, 32 x 512 x 512 voxels and 12288
   frames with 43 x 43 footprints. */
mpbp_status mpbp_plan_create(const mpbp_problem* problem, int device, mpbp_plan* out);

/* Release the plan and its device workspace (waits for the plan's work to finish).
   NULL is ignored. */
void mpbp_plan_destroy(mpbp_plan plan);

/* Number of frames (sum over peaks of rows * cols); -1 for a NULL plan. */
int64_t mpbp_num_frames(mpbp_plan plan);

/* Length in floats of the ragged intensity array y; -1 for a NULL plan. */
int64_t mpbp_intensity_size(mpbp_plan plan);

/* Copy the plan's integer tables to host memory (each pointer may be NULL):
     scan_yx  (host) int32 [n_frames][2]       (py, px) of each global frame
     shear_yx (host) int32 [n_peaks][nz][2]    s_m(z) = (s_y, s_x)
     y_off    (host) int64 [n_peaks + 1]       element offset of peak m in y
   These are the shift operator S and projection R of eq. (2) in integer form.
   Synchronous, host-only. */
mpbp_status mpbp_tables(mpbp_plan plan, int32_t* scan_yx, int32_t* shear_yx, int64_t* y_off);

/* Forward model and objective, eq. (2) and eq. (4), over the listed frames.
     loss            (dev) double scalar: f summed over the frames, or NULL
     frame_loss      (dev) float [n_frames] per-frame terms in list order, or NULL
     model_intensity (dev) float, ragged like y: I_{m,j} of the listed frames is written
                     (other frames untouched), or NULL
   y may be NULL only when loss and frame_loss are both NULL.
   n_frames is ignored when frames is NULL. */
mpbp_status mpbp_forward(mpbp_plan plan, const float* u, const float* chi,
                         const float* alpha, const void* probe, const float* y,
                         const int32_t* frames, int64_t n_frames,
                         double* loss, float* frame_loss, float* model_intensity,
                         void* stream);

/* Objective and its gradient (the adjoint of eq. (2)-(4)) over the listed frames:
     df/du_c     = sum_m G_m,c Im(g_O,m conj(O_m))
     df/dchi     = sum_m Re(conj(g_O,m) alpha_m exp(i G_m . u))
     df/dalpha_m = sum_voxels Re(conj(g_O,m) chi exp(i G_m . u))
   with g_O,m = df/dO_m.  loss (dev double) and frame_loss (dev float [n_frames]) may be
   NULL; grad_u (dev float [3][nz][ny][nx]), grad_chi (dev float [nz][ny][nx]) and
   grad_alpha (dev float [n_peaks]) are required and overwritten. */
mpbp_status mpbp_loss_grad(mpbp_plan plan, const float* u, const float* chi,
                           const float* alpha, const void* probe, const float* y,
                           const int32_t* frames, int64_t n_frames,
                           double* loss, float* frame_loss,
                           float* grad_u, float* grad_chi, float* grad_alpha,
                           void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc): mpbp_loss_grad with its per-call
   workspace (the per-peak objects, the exit-wave and gradient footprint slots, the
   per-frame losses and the alpha partials) in a fixed device array of the library
   instead of the plan's workspace.  The array holds MPBP_STATIC_SCRATCH_BYTES (64 MiB)
   on every GPU the library creates a plan on; it is set up by mpbp_plan_create and kept
   until the process ends.  This call allocates nothing (no hipMalloc, hipFree or other
   allocating call, host or device).
   Arguments, layouts, ownership and results are those of mpbp_loss_grad, and the
   results are bitwise equal to it (the same kernels with the plan's launch parameters;
   always the batched fused path, launched directly: no graph capture, no stage timing).
   Errors: those of mpbp_loss_grad, and MPBP_ERR_UNSUPPORTED (with the bytes needed in
   mpbp_last_error) when the plan's workspace exceeds the array; 8 n_peaks nz ny nx bytes
   of objects plus 16 bytes per footprint pixel of every frame dominate it (about 23 MB
   for 3 peaks, 16 x 128 x 128 voxels and 768 frames of 37 x 37).
   Every such call on one GPU uses the same array and leaves its contents there (every
   region is written before it is read within a call): calls that overlap in time on one
   GPU, on any streams or plans, race and must be serialised by the caller. */
#define MPBP_STATIC_SCRATCH_BYTES (64ull << 20)
mpbp_status mpbp_loss_grad_static(mpbp_plan plan, const float* u, const float* chi,
                                  const float* alpha, const void* probe, const float* y,
                                  const int32_t* frames, int64_t n_frames,
                                  double* loss, float* frame_loss,
                                  float* grad_u, float* grad_chi, float* grad_alpha,
                                  void* stream);

/* Plain gradient step in place, p <- p - eta_p * g_p, for (u, chi, alpha) with
   eta = (eta_u, eta_chi, eta_alpha) (host float[3]); the update of Algorithm 1 without
   Adam's moments.  All six device pointers are required. */
mpbp_status mpbp_step(mpbp_plan plan, float* u, float* chi, float* alpha,
                      const float* grad_u, const float* grad_chi, const float* grad_alpha,
                      const float* eta, void* stream);

/* Adam settings of mpbp_adam_step. */
typedef struct {
  float lr[3];             /* step sizes for u, chi (or chi~) and alpha (or alpha~)       */
  float beta1, beta2, eps; /* Adam moment decays and denominator offset                   */
  int32_t log_params;      /* 1: optimise chi~ = log chi and alpha~ = log alpha, eq. (8) */
  int32_t fixed_alpha;     /* peak whose alpha is held fixed (the reference peak), or -1 */
} mpbp_adam;

/* One Adam update (Kingma and Ba) of (u, chi, alpha) from the gradients of one
   mpbp_loss_grad call, as in each iteration of Algorithm 1 (minibatch gradients, then
   Adam); the phase-unwrap projection of that algorithm is not applied.
     t         step number, 1 for the first update (bias corrections 1 - beta^t);
               t = 0 initialises instead: zeroes state and, with log_params, writes
               chi = exp(chi_log) and alpha = exp(alpha_log) (gradients not read, may
               be NULL)
     state     (dev) float [2 (4 nf + n_peaks)], zero before t = 1: first moments of u,
               chi, alpha, then second moments; nf = nz ny nx (ny nx under MPBP_Z_TIED)
   With log_params = 1 the optimised variables are chi_log and alpha_log (dev, layouts of
   chi and alpha): the gradients (of f with respect to chi and alpha, at chi =
   exp(chi_log), alpha = exp(alpha_log)) are taken to the log variables by the chain
   rule, and chi and alpha are rewritten as exp of the updated log variables, ready for
   the next mpbp_loss_grad.  With log_params = 0, chi and alpha are updated directly and
   clamped at 0 (chi_log and alpha_log may be NULL).  u is always updated directly. */
mpbp_status mpbp_adam_step(mpbp_plan plan, const mpbp_adam* cfg, int64_t t, float* u, float* chi,
                           float* alpha, float* chi_log, float* alpha_log, float* state,
                           const float* grad_u, const float* grad_chi, const float* grad_alpha,
                           void* stream);

/* *out (dev double) = sum over i < n of a[i]^2 for a (dev) float array (a deterministic
   FP64 sum; used by line searches). */
mpbp_status mpbp_norm2(mpbp_plan plan, const float* a, int64_t n, double* out, void* stream);

/* Set / read a plan option (MPBP_OPT_*).  MPBP_ERR_INVALID for an unknown option or
   value. */
mpbp_status mpbp_set_option(mpbp_plan plan, int option, int64_t value);
mpbp_status mpbp_get_option(mpbp_plan plan, int option, int64_t* value);

/* Accumulated device time of each stage (MPBP_STAGE_*) over the calls enqueued since
   the previous mpbp_stage_times call while MPBP_OPT_PROFILE was 1 (2: the frame stage):
     ms     (host) double [MPBP_NUM_STAGES]  summed milliseconds
     counts (host) int64  [MPBP_NUM_STAGES]  number of launches timed
   Waits for the recorded events, then resets the accumulators.  Either pointer may be
   NULL. */
mpbp_status mpbp_stage_times(mpbp_plan plan, double* ms, int64_t* counts);

/* Autotuner.  Times every compiled launch variant of the per-frame kernel for each
   detector-size class of the plan (footprint bound, projection depth = object slices
   each lane of the projection kernel has in flight, XCD-aware frame order) and of the back-projection kernel
   (frames read per step, tile shape), on the caller's inputs (layouts as in mpbp_loss_grad; y is
   required), and keeps the fastest for later calls.  Every variant computes the same
   result.  Synchronous: waits for `stream`.  Allocates and frees a gradient scratch
   of 16 * nz * ny * nx bytes.  If the environment variable MPBP_TUNE_CACHE names a
   file, the choices are written there (one line per kernel, keyed by GPU architecture
   and shapes) and mpbp_plan_create applies matching lines to later plans.
   Drops the plan's captured graphs. */
mpbp_status mpbp_autotune(mpbp_plan plan, const float* u, const float* chi,
                          const float* alpha, const void* probe, const float* y,
                          void* stream);

/* Select a frame-kernel variant by hand for size class `size_class` (the order of
   the "classes" list of mpbp_tuning): compiled footprint bound (>= the class's
   smallest, see mpbp_tuning "key"), projection depth `slab` (object slices in flight per
   lane: 2, 4 or 8) and XCD order (0 or 1).
   MPBP_ERR_UNSUPPORTED if that variant is not compiled or does not fit in LDS. */
mpbp_status mpbp_set_variant(mpbp_plan plan, int size_class, int footprint_bound, int slab,
                             int xcd_order);

/* The plan's launch parameters as a JSON object: source ("default", "cache",
   "autotune" or "manual"), grad_batch, grad_tile, per size class {D, key, frames, fy, fx, FB, G,
   xcd, us} and the candidates the last mpbp_autotune timed.  Writes at most `cap`
   bytes (NUL-terminated) to buf (may be NULL) and the size needed, NUL included, to
   *len (may be NULL); MPBP_ERR_INVALID if cap is too small for the text. */
mpbp_status mpbp_tuning(mpbp_plan plan, char* buf, int64_t cap, int64_t* len);

/* The background b of eq. (2): the model intensity becomes
     I_{m,j} = | F R_m diag(P_m) S_{m,j} O_m |^2 + b_{m,j}
   in mpbp_forward (model_intensity, loss) and mpbp_loss_grad (eq. (4) compares sqrt(I)
   with sqrt(y); the gradient is (sqrt(I) - sqrt(y)) Psi / sqrt(I) on the far field).
     b  (dev) float, ragged in the layout of y, b >= 0; NULL (the default) = no background.
   The plan keeps the pointer (not a copy): the caller keeps the buffer alive and
   unchanged in size while it is set; its contents may change between calls.  Both paths
   and the autotuner use it; captured graphs are keyed by it. */
mpbp_status mpbp_set_background(mpbp_plan plan, const float* b);

/* The phase-unwrap projector Pi_U of eq. (10) (section 3.3; the last step of every
   iteration of Algorithm 1), applied in place:
     u <- W^{-1}{W{u . H}} . H^T (H H^T)^{-1},
   H the 3 x n_peaks matrix of Bragg vectors (eq. (9)), W the phase wrap, W^{-1} the 2D
   phase unwrapping of every map (one per peak and per z-slice; one per peak under
   MPBP_Z_TIED) by reliability-guided merging (Herraez et al., Appl. Opt. 41, 7437
   (2002)): pixel reliability 1 / sqrt(H^2 + V^2 + D1^2 + D2^2) from the second
   differences of the wrapped phase along the row, the column and both diagonals (0 on
   the map border), edges between 4-neighbours ordered by the summed reliability of
   their pixels (ties by MurmurHash3's fmix32 of the edge index, horizontal edges
   i (nx - 1) + j first, then vertical edges ny (nx - 1) + i nx + j), and groups joined
   from the most reliable edge down.  Every map's free multiple of 2 pi is fixed by
   rounding (halves up) the mean of its wrap counts rint(G_m . u / 2 pi) minus those of
   the unwrapped phase, so that a field without phase jumps is left unchanged.  The
   update is applied as u += 2 pi N . H^+ with the integer maps N below and the
   Moore-Penrose H^+ (equal to eq. (10) for non-coplanar Bragg vectors; for coplanar
   ones the component of u that no peak sees is kept).  Wraps, reliabilities and edge
   keys are computed in float32, each operation rounded in the order written above.
     u      (dev) float, the layout of mpbp_loss_grad; overwritten with Pi_U(u)
     wraps  (dev) int32 [n_peaks][nz][ny][nx] ([n_peaks][1][ny][nx] under MPBP_Z_TIED),
            may be NULL: N, the multiples of 2 pi the projector adds to each phase
            G_m . u (the unwrapped phase is G_m . u + 2 pi N)
   The first call allocates a workspace of about 44 bytes per map pixel, kept until
   mpbp_plan_destroy.  Synchronous: waits for `stream` (it reads back a device-side
   consistency flag; MPBP_ERR_INTERNAL if a merge step found its tree inconsistent). */
mpbp_status mpbp_unwrap_project(mpbp_plan plan, float* u, int32_t* wraps, void* stream);

/* Thread-local description of the last error of this thread ("" if none). */
const char* mpbp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MPBP_H */
