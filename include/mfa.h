/*
 * mfa.h - C ABI of the MI355X (gfx950) MFA evaluator and ray caster.
 *
 * The library evaluates multivariate functional approximation (MFA) models -
 * tensor products of B-spline functions given by knots and control points
 * (paper, Sec. III-A) - for value and analytic gradient at arbitrary points
 * (Sec. III-B; the query interface of Sec. IV-A4), and ray-casts them with
 * transfer-function lookup, gradient shading and front-to-back "over"
 * compositing with early ray termination (Sec. IV-A4, IV-A5, IV-B).  Models
 * are made of blocks from a partition of the volume (Sec. IV-A1), each block
 * an independent model over its own box, and are kept resident in device
 * memory (the "fetched to the memory of each target node" step, Sec. IV-A3).
 *
 * Conventions shared by every entry point
 *  - Every function returns an mfa_status; nothing throws across the ABI.
 *    On a status other than MFA_OK, mfa_last_error() returns a message for
 *    the calling thread.
 *  - Arguments are validated on the host before anything is enqueued; a
 *    rejected call has no effect and returns MFA_E_ARG (or MFA_E_NOMEM /
 *    MFA_E_UNSUPPORTED).
 *  - Buffers named "device" are caller-owned device memory of the device the
 *    model was created on; the library never frees them.  Buffers named
 *    "host" are caller-owned host memory, read or written before the call
 *    returns.
 *  - Work is enqueued on the caller's HIP stream (hipStream_t passed as
 *    void*, NULL = the default stream) and the call returns without
 *    synchronising.  A fault during the kernel surfaces as MFA_E_DEVICE from
 *    a later call that synchronises (or from hipStreamSynchronize).
 *  - Exact FP64 decisions (span, block, ray schedule) follow the readings of
 *    the paper stated at each function; values and gradients are FP32.
 */
#ifndef MFA_H
#define MFA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MFA_OK = 0,
  MFA_E_ARG = -1,          /* invalid argument (message says which)           */
  MFA_E_NOMEM = -2,        /* device or host allocation failed                */
  MFA_E_DEVICE = -3,       /* HIP runtime error or device fault               */
  MFA_E_BUDGET = -4,       /* request exceeds the server's memory budget      */
  MFA_E_BUSY = -5,         /* server queue full                               */
  MFA_E_NOTFOUND = -6,     /* unknown model id / ticket                       */
  MFA_E_UNSUPPORTED = -7   /* valid but not implemented (e.g. degree > 7)     */
} mfa_status;

typedef enum { MFA_F64 = 0, MFA_F32 = 1, MFA_BF16 = 2, MFA_F16 = 3 } mfa_dtype;

typedef struct mfa_model_s* mfa_model;   /* opaque; owns the device copy */

/* ------------------------------------------------------------------ models */

/* World box split into grid[0] x grid[1] x grid[2] blocks (Sec. IV-A1;
 * Table I lists the paper's partitions).
 *  grid   : blocks per axis, each >= 1; {1,1,1} is a single-block model.
 *  lo, hi : world box, lo[a] < hi[a].
 *  edges  : optional host FP64 block edges per axis, grid[a]+1 strictly
 *           increasing values with edges[a][0] == lo[a] and
 *           edges[a][grid[a]] == hi[a]; NULL = lo + (hi-lo) * (i / grid),
 *           computed in FP64.  Copied during create.
 *  voxel  : reference voxel size in world units (> 0); a render step of 0
 *           means half a voxel.                                             */
typedef struct {
  int32_t grid[3];
  double lo[3];
  double hi[3];
  const double* edges[3];
  double voxel;
} mfa_domain_desc;

/* One block: degree and control-point count per axis, knots, coefficients.
 *  degree : 1..7 per axis; all blocks of a model share one degree on all
 *           axes (MFA_E_UNSUPPORTED otherwise).
 *  n_ctrl : control points per axis, n >= degree + 1.
 *  knots  : optional host FP64 knot vectors, n + p + 1 nondecreasing values,
 *           clamped: T[0..p] = 0 and T[n..n+p] = 1, every span inside
 *           [T[p], T[n]] reachable (T[p] < T[p+1] is not required, spans of
 *           zero length are skipped by the span rule).  NULL = clamped
 *           uniform: T[p+j] = j / (n - p), one FP64 division each.
 *  ctrl   : host, C order [n0][n1][n2] (axis 2 fastest), element type
 *           ctrl_dtype (MFA_F64 or MFA_F32), all finite.                    */
typedef struct {
  int32_t degree[3];
  int32_t n_ctrl[3];
  const double* knots[3];
  const void* ctrl;
  mfa_dtype ctrl_dtype;
} mfa_block_desc;

/* Creates a model on the current HIP device (Sec. IV-A2/IV-A3: encoded
 * blocks, fetched once into device memory).
 *  blocks   : host array of nblocks descriptors in C order over the grid
 *             (block (b0,b1,b2) at (b0*grid[1] + b1)*grid[2] + b2);
 *             nblocks must equal grid[0]*grid[1]*grid[2].
 *  storage  : MFA_F32, MFA_BF16 or MFA_F16.  Stored value =
 *             RNE(FP64 -> FP32), then RNE(FP32 -> BF16/FP16).
 *  out      : receives the handle.  Host data are copied; the caller may
 *             free them on return.  The call synchronises the device.
 * Errors: MFA_E_ARG (shape, knots, non-finite data), MFA_E_UNSUPPORTED
 * (degree), MFA_E_NOMEM, MFA_E_DEVICE.                                     */
mfa_status mfa_model_create(const mfa_domain_desc* domain, const mfa_block_desc* blocks,
                            int32_t nblocks, mfa_dtype storage, mfa_model* out);

/* Frees the device copy.  The caller must ensure no enqueued work still
 * uses the model.  NULL is accepted (no-op).                               */
mfa_status mfa_model_destroy(mfa_model model);

typedef struct {
  int64_t device_bytes;    /* bytes of device memory held by the model       */
  int64_t ctrl_bytes;      /* of which stored control points                 */
  int64_t n_ctrl_total;    /* control points over all blocks                 */
  int32_t nblocks;
  int32_t degree;
  mfa_dtype storage;
  float vmin, vmax;        /* min / max of the stored control points         */
  double voxel;
  int32_t device;          /* HIP device ordinal                             */
} mfa_model_info_t;

mfa_status mfa_model_info(mfa_model model, mfa_model_info_t* info);

/* Copies the stored control points of one block back to host memory
 * (stored bits: 4 bytes per point for MFA_F32, 2 for BF16/FP16), C order.
 * dst_bytes must be at least n0*n1*n2*elem_size.  Synchronises the device. */
mfa_status mfa_model_export_ctrl(mfa_model model, int32_t block, void* host_dst, int64_t dst_bytes);

/* ------------------------------------------------------------------ decode */

/* Value and gradient at n world points (the value/gradient query of
 * Sec. IV-A4; analytic derivatives, Sec. III-B; the value-only query of
 * Fig. 8a with MFA_DECODE_VALUE).
 *  xyz   : device FP32, structure of arrays [3][n] (x then y then z); each
 *          coordinate is promoted exactly to FP64.
 *  n     : 0 <= n < 2^31 (n == 0 is a no-op).
 *  flags : a combination of
 *          MFA_DECODE_SORTED: points are first grouped by bucket = (owning
 *          block, tile of 2^k spans per axis, k chosen per model: the
 *          largest whose control-point windows fit 8192 values, larger
 *          while the model has more than 32768 buckets; models of more than
 *          32768 blocks return MFA_E_UNSUPPORTED) and evaluated in that
 *          order, each bucket's control points staged once in on-chip
 *          memory; results are still written in input order and are
 *          identical bit for bit to the unsorted call.  Uses scratch memory
 *          held by the model (16 bytes per point, 36 with more than 1024
 *          buckets, plus about 20 per bucket), allocated on first use and
 *          grown when a larger n arrives (MFA_E_NOMEM if that fails).
 *          Sorted calls on one model are ordered by the library: a call
 *          waits (on its stream) for the previous sorted call's kernels
 *          before it reuses the scratch, and for their completion (on the
 *          host) before it replaces a smaller one.
 *          MFA_DECODE_VALUE: value only, no gradient.
 *  out   : device FP32 [n][4] = (f, df/dx, df/dy, df/dz) in world units;
 *          with MFA_DECODE_VALUE device FP32 [n] = f.
 *  dbg   : NULL, or device int32 [n][4] = (span0, span1, span2, block)
 *          with block = (b0*grid1 + b1)*grid2 + b2.
 * Map: xc = clamp(x, E[0], E[G]); owning block b = max{i : E[i] <= xc};
 * u = clamp((xc - lo_b) * inv_ext_b, 0, 1) with inv_ext_b = 1/(hi_b - lo_b)
 * (FP64, unfused); span s = max{i in [p, n-1] : T[i] <= u}.               */
#define MFA_DECODE_SORTED 1u
#define MFA_DECODE_VALUE 2u
mfa_status mfa_decode_points(mfa_model model, const float* xyz, int64_t n, uint32_t flags,
                             float* out, int32_t* dbg, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that
 * forbid it): the sorted decode of mfa_decode_points (MFA_DECODE_SORTED is
 * implied; MFA_DECODE_VALUE may be given) with its scratch in a file-scope
 * device array of the library, 64 MiB per device, held until the process
 * ends.  No device memory is allocated or freed by the call.  Arguments,
 * outputs and results are those of mfa_decode_points (bit-identical).
 *  n     : the scratch must hold the layout of the sorted decode: 16 bytes
 *          per point (36 with more than 1024 buckets) plus about 20 per
 *          bucket and the decode items, at most 64 MiB (about 4 million
 *          points with up to 1024 buckets, 1.8 million above); a larger n
 *          returns MFA_E_ARG with the largest n accepted for this model.
 * Every call on a device shares that device's scratch, which keeps the last
 * call's contents (the kernels clear what must start at zero): calls whose
 * kernels overlap in time on one device race and give undefined results;
 * order them on one stream or synchronise between them.                   */
mfa_status mfa_decode_points_noalloc(mfa_model model, const float* xyz, int64_t n, uint32_t flags,
                                     float* out, int32_t* dbg, void* stream);

/* Value and gradient on the tensor grid axis_u[0] x axis_u[1] x axis_u[2]
 * of parameters of a single-block model (MFA_E_ARG for multi-block).
 *  axis_u : three device FP64 tables of res[a] parameters (clamped to
 *           [0,1]); any order, nondecreasing tables are fastest.
 *  res    : 1 <= res[a], res0*res1*res2 < 2^40.
 *  flags  : 0, or MFA_DECODE_VALUE (value only).
 *  out    : device FP32 [res0][res1][res2][4] (axis 2 fastest) =
 *           (f, df/dx, df/dy, df/dz), gradient in world units; with
 *           MFA_DECODE_VALUE device FP32 [res0][res1][res2] = f.
 *  spans  : NULL, or device int32 [res0 + res1 + res2]: the span of each
 *           table entry, axis 0 entries first.                             */
mfa_status mfa_decode_grid(mfa_model model, const double* const axis_u[3], const int32_t res[3],
                           uint32_t flags, float* out, int32_t* spans, void* stream);

/* ------------------------------------------------------------------ render */

enum { MFA_ORTHO = 0, MFA_PERSPECTIVE = 1 };

/* Camera (view-dependent parameters, Sec. IV-B).  right, up, forward form
 * an orthonormal right-handed basis built by the caller in FP64.  Pixel
 * (i, j), row j = 0 at the top: px = (2i + 1 - w) * sx,
 * py = (h - 2j - 1) * sy.  Orthographic: origin (eye + px*right) + py*up,
 * direction forward.  Perspective: origin eye, direction
 * (forward + px*right) + py*up, not normalised, so the ray parameter is the
 * depth along forward.                                                     */
typedef struct {
  int32_t kind;
  double eye[3];
  double forward[3];
  double right[3];
  double up[3];
  double sx, sy;
} mfa_camera;

/* Data-dependent parameters (Sec. IV-B: transfer function and shading).
 *  tf_rgba     : device FP32 [256][4], colour not premultiplied, alpha in
 *                [0,1].  s = clamp((f - vmin)/(vmax - vmin), 0, 1) * 255,
 *                linear interpolation between entries floor(s) (<= 254)
 *                and floor(s) + 1.
 *  vmin < vmax : transfer-function domain.
 *  step        : ray-parameter step dt (> 0; 0 = half the model voxel).
 *  max_samples : cap on samples per ray, >= 1.
 *  ert_alpha   : stop after the first sample with accumulated opacity
 *                >= ert_alpha (that sample included); > 1 disables.
 *  ka, kd, ks, shininess : Phong with a headlight, two-sided:
 *                c' = rgb * (ka + kd*diff) + ks * diff^shininess,
 *                diff = |n . L|, n = g / max(|g|, g0), L = -d/|d|.
 *  g0 > 0      : gradient-norm floor of the normal.
 * Schedule: slab test of each ray against the model box (FP64); K =
 * min(floor((t_far - t_near)/dt), max_samples) samples at
 * t_k = t_near + (k + 1/2) dt, x_k = o + t_k d (FP64, unfused).
 * Compositing (front to back, premultiplied): C += (1 - A) * alpha * c',
 * A += (1 - A) * alpha, in FP32 with each operation rounded separately.   */
typedef struct {
  const float* tf_rgba;
  float vmin, vmax;
  double step;
  int32_t max_samples;
  float ert_alpha;
  float ka, kd, ks, g0;
  int32_t shininess;
} mfa_render_params;

/* Optional debug outputs of a render (device memory, NULL = not wanted).
 *  nsamp        : int32 [h][w][2] = (K scheduled samples, samples used).
 *  neval        : int32 [h][w]: samples whose value and gradient were
 *                 evaluated; the others lie where the transfer function is
 *                 zero over the value bounds of the enclosing control points
 *                 (the spline's convex hull), so their opacity is exactly 0
 *                 and they leave the pixel unchanged.
 *  alpha        : FP32 [h][w][alpha_stride]: per-sample opacity after the
 *                 transfer function, for samples 0..used-1 (rest untouched).
 *  alpha_stride : >= max_samples when alpha is given.                      */
typedef struct {
  int32_t* nsamp;
  int32_t* neval;
  float* alpha;
  int32_t alpha_stride;
} mfa_render_debug;

/* Ray-casts the model (MFA-VV, Sec. IV-A4) into a w x h image.
 *  rgba : device FP32 [h][w][4] = (C_r, C_g, C_b, A), premultiplied, no
 *         background.
 *  dbg  : NULL or debug outputs as above.
 *  1 <= w, h <= 16384.                                                     */
mfa_status mfa_render_frame(mfa_model model, const mfa_camera* camera, const mfa_render_params* params,
                            int32_t w, int32_t h, float* rgba, const mfa_render_debug* dbg,
                            void* stream);

/* First-hit isosurface of level iso, from the same value and gradient
 * queries as the volume render (the paper names isosurface rendering as
 * another product of its ray-casting step, Sec. IV-A4, without a method).
 * The rays, their box entry and samples t_k = t_near + (k + 1/2) step are
 * those of mfa_render_frame; a sample is on side 1 where f >= iso; the hit
 * lies between the first two consecutive samples k-1, k of different sides
 * (either direction), at w = (iso - f_{k-1}) / (f_k - f_{k-1}) between them:
 * t* = t_near + (k - 1/2 + w) step.  The pixel is the headlight Phong colour
 * of rgb with the gradient at x* = o + t* d (params ka, kd, ks, g0,
 * shininess), opacity 1; without a hit (0, 0, 0, 0).  params' transfer
 * function, vmin / vmax and ert_alpha are not used (tf_rgba may be NULL).
 *  rgba  : device FP32 [h][w][4].
 *  depth : NULL or device FP64 [h][w]: t* (+inf without a hit), which can
 *          key the image in mfa_composite_over.
 *  dbg   : NULL or nsamp = (K, hit sample k or -1) and neval = values
 *          evaluated; alpha must be NULL.
 * Samples in a macro cell whose value bounds lie wholly on one side of iso
 * are not evaluated: the bounds contain every evaluation in the cell, so
 * the sides, and the image, are those of evaluating every sample.
 * Errors: as mfa_render_frame, and MFA_E_ARG for a non-finite iso or rgb. */
mfa_status mfa_render_iso(mfa_model model, const mfa_camera* camera, const mfa_render_params* params,
                          float iso, const float rgb[3], int32_t w, int32_t h, float* rgba,
                          double* depth, const mfa_render_debug* dbg, void* stream);

/* Local-filter baselines (the reconstruction filters the paper compares MFA
 * queries with, Sec. I and Sec. V) and the analytic Marschner-Lobb field
 * (Sec. V-A1, the ground truth of its quality study), rendered by the same
 * ray caster: rays, schedule, transfer function, shading, compositing and
 * termination are those of mfa_render_frame, with the box [lo, hi] in place
 * of the model box and value + gradient from the volume below.
 *  samples : device FP32 [dims0][dims1][dims2] (axis 2 fastest), sample
 *            (i0, i1, i2) at lo + i * h, h = (hi - lo) / (dims - 1); NULL for
 *            MFA_FIELD_MARSCHNER_LOBB.
 *  kind    : MFA_FILTER_TRILINEAR (cell c = min(floor(g), dims - 2) of the
 *            grid coordinate g = clamp((x - lo) / h, 0, dims - 1), weights
 *            1 - t, t), MFA_FILTER_CATMULL_ROM (cubic interpolation with
 *            tangents (v[c+1] - v[c-1]) / 2, samples c-1 .. c+2),
 *            MFA_FILTER_CUBIC_BSPLINE (the uniform cubic B-spline filter on
 *            the samples, approximating, same stencil), stencil indices
 *            outside the grid repeating the edge sample; gradients are the
 *            analytic derivatives of the filter's polynomial (1 / h per
 *            axis).  MFA_FIELD_MARSCHNER_LOBB: F = (1 - sin(pi z/2) +
 *            a (1 + cos(2 pi f cos(pi r/2)))) / (2 (1 + a)), r = |(x, y)|,
 *            f = 6, a = 0.25, and its analytic gradient, in FP32.
 *  dims    : >= 2 per axis (also for the analytic field: they set the
 *            default step, half the smallest spacing h).
 * The debug outputs are those of mfa_render_frame (every sample up to the
 * termination is evaluated).  Errors: MFA_E_ARG for a bad kind, box or
 * dims, null samples, and as mfa_render_frame.                             */
enum { MFA_FILTER_TRILINEAR = 0, MFA_FILTER_CATMULL_ROM = 1, MFA_FILTER_CUBIC_BSPLINE = 2,
       MFA_FIELD_MARSCHNER_LOBB = 3 };
typedef struct {
  const float* samples;
  int32_t dims[3];
  double lo[3], hi[3];
  int32_t kind;
} mfa_volume_desc;
mfa_status mfa_render_volume(const mfa_volume_desc* volume, const mfa_camera* camera,
                             const mfa_render_params* params, int32_t w, int32_t h, float* rgba,
                             const mfa_render_debug* dbg, void* stream);

/* Object-space split (Sec. IV-A4: each node ray-casts the blocks it holds
 * into a partially rendered image; Sec. IV-A5: the partial images are
 * combined by "over" in depth order).
 *  mfa_render_partial : as mfa_render_frame, but only the samples owned by
 *     blocks with block_lo[a] <= b[a] < block_hi[a] (the block-owner rule)
 *     are composited, on the model's own sample schedule, and early
 *     termination tests the partial's own opacity.  key: device FP64
 *     [h][w] out, the entry parameter of the ray into the region's world box
 *     (+inf when the ray misses that box or the model); the samples of
 *     disjoint regions form runs along a ray in increasing key order.
 *     Errors: MFA_E_ARG for an empty block range or one outside the grid.
 *  mfa_composite_over : per pixel, the g partial images (host array of g
 *     device FP32 [h][w][4] pointers, premultiplied) sorted by their keys
 *     (host array of g device FP64 [h][w] pointers; equal keys keep list
 *     order) and folded front to back, C += (1 - A) c, A += (1 - A) a, into
 *     out (device FP32 [h][w][4]).  1 <= g <= 16.  With termination off and
 *     regions that partition the blocks, the composite equals
 *     mfa_render_frame up to FP32 rounding (associativity of "over").     */
mfa_status mfa_render_partial(mfa_model model, const mfa_camera* camera,
                              const mfa_render_params* params, const int32_t block_lo[3],
                              const int32_t block_hi[3], int32_t w, int32_t h, float* rgba,
                              double* key, const mfa_render_debug* dbg, void* stream);
mfa_status mfa_composite_over(int32_t g, const float* const* images, const double* const* keys,
                              int32_t w, int32_t h, float* out, void* stream);

/* ------------------------------------------------------------------ serving */

/* A request loop for many clients sharing one GPU: the visualisation
 * pipeline re-runs on every change of transfer function, shading or view
 * (Sec. IV-B), here as render and point-query requests against resident
 * models.  A scheduler thread admits requests first come first served
 * while the bytes of their buffers fit the memory budget, splits them into
 * work items (16x16 pixel tiles, 256-point chunks), packs at most
 * max_batch_items items per batch (a large request spans batches) and runs
 * each batch as persistent launches on one of three server-owned streams
 * (up to three batches overlap).  Results equal those of mfa_render_frame and
 * mfa_decode_points (unsorted) bit for bit.                                */
typedef struct mfa_server_s* mfa_server;   /* opaque */

#define MFA_SERVER_FAKE_EXECUTOR 1u   /* no device work: each batch "runs" for
                                         fake_item_us per item (host tests)  */
typedef struct {
  int64_t hbm_budget_bytes;   /* bytes of request buffers admitted at once (> 0)  */
  int32_t queue_cap;          /* requests waiting for a batch (> 0)               */
  int32_t max_batch_items;    /* work items per batch (0 = 8192)                  */
  uint32_t flags;             /* 0 or MFA_SERVER_FAKE_EXECUTOR                    */
  double fake_item_us;        /* modelled time per item with the fake executor    */
  int32_t fake_fail_batch;    /* fake executor only: the batch with this launch
                                 number (1-based) fails as a device error would;
                                 0 = none (host tests of the failure path)       */
} mfa_server_config;

enum { MFA_REQ_RENDER = 0, MFA_REQ_POINTS = 1 };

/* One request.  Render: camera, params, w, h and the device RGBA buffer
 * rgba [h][w][4] as for mfa_render_frame (footprint w*h*16 + 4096 bytes).
 * Points: device SoA xyz [3][n] and device out [n][4] as for
 * mfa_decode_points (footprint 28*n bytes).  The caller keeps the buffers
 * (and the TF table) alive and untouched until the request is done.       */
typedef struct {
  int32_t kind;
  int32_t model_id;
  mfa_camera camera;
  mfa_render_params params;
  int32_t w, h;
  float* rgba;
  const float* xyz;
  int64_t n;
  float* out;
} mfa_request;

/* Host times in seconds since the server was created: submit, admission
 * (memory granted), launch of its first batch, completion noticed by the
 * scheduler.  status is MFA_OK or MFA_E_DEVICE; done is 0 or 1.
 * A failure is per batch: a batch whose launch fails or whose completion
 * event reports an error fails every request with items in it (status
 * MFA_E_DEVICE once the request is done); such a request still releases its
 * budget, and later batches run as usual (after a fault that leaves the
 * device unusable they fail in turn, each with its own status).  Launches
 * run outside the lock that submit, poll and wait take.                    */
typedef struct {
  double t_submit, t_admit, t_start, t_done;
  int32_t status;
  int32_t done;
} mfa_request_stats;

/* Creates a server on the current device (its models must live there).
 * With MFA_SERVER_FAKE_EXECUTOR no device is touched and models may be
 * NULL.                                                                     */
mfa_status mfa_server_create(const mfa_server_config* config, mfa_server* out);

/* Makes a model servable; model_id receives its index.  The model must
 * outlive the server.                                                      */
mfa_status mfa_server_add_model(mfa_server server, mfa_model model, int32_t* model_id);

/* Queues a request without waiting for the GPU.  Errors: MFA_E_ARG (bad
 * request or model id), MFA_E_BUDGET (footprint above the whole budget),
 * MFA_E_BUSY (queue_cap requests waiting).                                 */
mfa_status mfa_server_submit(mfa_server server, const mfa_request* request, uint64_t* ticket);

/* Host-only status read; MFA_E_NOTFOUND for an unknown ticket.            */
mfa_status mfa_server_poll(mfa_server server, uint64_t ticket, mfa_request_stats* stats);

/* Blocks until the request is done; returns its status.                   */
mfa_status mfa_server_wait(mfa_server server, uint64_t ticket, mfa_request_stats* stats);

/* Forgets a finished request (its stats are no longer available).         */
mfa_status mfa_server_release(mfa_server server, uint64_t ticket);

/* Finishes every queued request, then frees the server.  NULL is a no-op. */
mfa_status mfa_server_destroy(mfa_server server);

/* ------------------------------------------------------------------ host utilities */

/* ------------------------------------------------------------------ encoding */

/* Fixed-knot encoding of one block from samples on a tensor grid (Sec. IV-A2
 * "MFA Encoding"; the parameterisation and initial knot distribution of
 * Fig. 1, without the knot insertion that follows it there).  The control
 * points minimise the sum of squared differences between the spline and the
 * samples,
 *     P = argmin sum_i ( f(u0[i0], u1[i1], u2[i2]; P) - F[i0][i1][i2] )^2,
 * which for a tensor grid is P = F x_0 B0+ x_1 B1+ x_2 B2+ with B_a the
 * collocation matrix N_{j,p}(u_a[i]) of axis a and B+ = (B^T B)^-1 B^T.
 * The host factors each Gram matrix B_a^T B_a (banded Cholesky, FP64).  With
 * at least 2^17 fibers along axes 1 and 2 (res1 * res2), and when its bytes
 * take less time than the dense product's work (about n0 > 48 for res0 =
 * 512), the device applies axis 0 without forming B0+: per fiber of the
 * samples, B0^T F (p + 1 non-zeros per sample) and the two banded
 * triangular solves; the other products use the dense B_a+ tables as FP64
 * GEMMs on the matrix cores.
 *  res      : samples per axis, n_ctrl[a] <= res[a] <= 65536.
 *  axis_u   : host FP64 parameters of the samples, res[a] values per axis,
 *             each in [0, 1], any order.
 *  values   : device FP32 [res0][res1][res2] samples, axis 2 fastest.
 *  degree, n_ctrl, knots : as in mfa_block_desc (knots[a] NULL = clamped
 *             uniform); the result can be passed to mfa_model_create as the
 *             block's control points after a copy to the host.
 *  ctrl     : device FP64 [n0][n1][n2] out, axis 2 fastest.
 *  work     : device scratch of at least mfa_encode_workspace() bytes
 *             (caller-owned; not to be shared by calls in flight together).
 * Errors (before any device work): MFA_E_ARG for bad sizes, parameters or
 * knots, and when some B_a^T B_a is not positive definite (a basis function
 * with too few samples in its support: raise res or lower n_ctrl).
 * The call waits for the upload of its tables on the stream (so for the
 * work queued before it); the products are left in flight.
 * mfa_encode_grid = mfa_encode_plan + mfa_encode_apply: blocks of one
 * partition have equal sizes and knots (Sec. IV-A1, IV-A2), so a plan,
 * made once into work, serves every block:
 *  mfa_encode_plan  : validates the arguments, builds the tables (axis 0
 *                     by the banded route: sample order, supports, basis
 *                     values, Cholesky factor and degree; else B_a+) and
 *                     uploads them into work (waits for the upload);
 *  mfa_encode_apply : the three mode products of one block's values into
 *                     ctrl, left in flight; work must hold a plan made for
 *                     the same res and n_ctrl (and the apply of one block
 *                     must finish before another uses the same work).   */
mfa_status mfa_encode_workspace(const int32_t res[3], const int32_t n_ctrl[3], int64_t* bytes);
mfa_status mfa_encode_grid(const int32_t res[3], const double* const axis_u[3], const float* values,
                           const int32_t degree[3], const int32_t n_ctrl[3],
                           const double* const knots[3], double* ctrl, void* work,
                           int64_t work_bytes, void* stream);
mfa_status mfa_encode_plan(const int32_t res[3], const double* const axis_u[3],
                           const int32_t degree[3], const int32_t n_ctrl[3],
                           const double* const knots[3], void* work, int64_t work_bytes,
                           void* stream);
mfa_status mfa_encode_apply(const int32_t res[3], const int32_t n_ctrl[3], const float* values,
                            double* ctrl, void* work, int64_t work_bytes, void* stream);

/* Encoding with knot insertion (Fig. 1: fit, measure the error, add knots
 * where it is too large, refit).  Starting from clamped uniform knots with
 * n_init control points per axis, each pass makes the fixed-knot fit above
 * on the device, reconstructs the spline at every sample (three more mode
 * products with the B_a, the last one taking the errors in its epilogue
 * instead of storing the values), and takes every sample's error relative
 * to the data range, |f - F| / (max F - min F) (range 1 when it is 0).  Per axis,
 * a knot span [t_j, t_j+1) (span rule of mfa_model_create) gets the largest
 * error over the samples whose axis-a parameter falls in it; a span whose
 * error exceeds e_max is halved (a knot at its midpoint) when both halves
 * hold a sample parameter.  When more spans qualify than max_ctrl[a] - n_a
 * leaves room for, the ones of largest error are halved (ties: lower span
 * first).  The loop ends after a pass that halves nothing or after
 * max_fits passes; the result is the last pass's fit and knots.
 *  res, axis_u, values, degree : as in mfa_encode_grid.
 *  n_init   : starting control points per axis, degree + 1 <= n_init <= max_ctrl.
 *  max_ctrl : largest control-point count per axis, max_ctrl[a] <= res[a];
 *             sizes the workspace and ctrl.
 *  e_max    : error bound, finite and > 0.  max_fits >= 1.
 *  knots_out: host FP64 out, knots_out[a] with room for max_ctrl[a] + degree[a] + 1
 *             values; n_out : host out, the final control-point counts.
 *  ctrl     : device FP64 out, room for ctrl_capacity >= the product of
 *             max_ctrl; holds [n_out0][n_out1][n_out2] (axis 2 fastest).
 *  history  : host FP64 out (NULL to skip), max_fits rows of 4 values, per
 *             pass n0, n1, n2 and the largest relative error of that fit;
 *             n_fits : host out, the passes made.
 *  work     : device scratch of mfa_encode_adaptive_workspace(res, max_ctrl)
 *             bytes, caller-owned.
 * res0 * res1 is at most 65535 * 2048.  Errors: as mfa_encode_grid (also
 * from a later pass whose knots leave a basis function without samples); every
 * pass waits for its work on the stream (the knots are chosen on the host),
 * so the call returns with ctrl final.                                     */
mfa_status mfa_encode_adaptive_workspace(const int32_t res[3], const int32_t max_ctrl[3],
                                         int64_t* bytes);
mfa_status mfa_encode_adaptive(const int32_t res[3], const double* const axis_u[3],
                               const float* values, const int32_t degree[3],
                               const int32_t n_init[3], const int32_t max_ctrl[3], double e_max,
                               int32_t max_fits, double* const knots_out[3], int32_t n_out[3],
                               double* ctrl, int64_t ctrl_capacity, double* history,
                               int32_t* n_fits, void* work, int64_t work_bytes, void* stream);

/* Host-only helpers (no device work): the storage rounding and the default
 * knot vector the library uses, exported so they can be checked on a CPU.
 *  mfa_quantize : n FP64 values -> stored bits of dtype (MFA_F32: uint32
 *                 patterns, MFA_BF16 / MFA_F16: uint16 patterns).
 *  mfa_default_knots : clamped uniform knots, n + p + 1 values.            */
mfa_status mfa_quantize(const double* src, int64_t n, mfa_dtype dtype, void* dst);
mfa_status mfa_default_knots(int32_t n, int32_t p, double* dst);

/* Thread-local message of the last non-OK status on this thread. */
const char* mfa_last_error(void);

/* Library version string. */
const char* mfa_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MFA_H */
