/*
 * g4d.h - C ABI of the MI355X (gfx950) deform-then-splat render of
 * 4D Gaussian Splatting ("4D Gaussian Splatting for Real-Time Dynamic Scene
 * Rendering").
 *
 * The library computes  I = S(M, G')  with  G' = G + F(G, t)  (Sec. 4.1):
 *   g4d_deform  evaluates the Gaussian deformation field F (Sec. 4.2: the
 *               multi-resolution HexPlane encoder of Eq. 7, the feature MLP
 *               phi_d and the heads phi_x, phi_r, phi_s) and applies Eq. 8;
 *   g4d_render  splats the deformed Gaussians through a view M (Sec. 3.1:
 *               Eq. 1-4, with the tile rasterizer of 3D Gaussian Splatting).
 * A static render S(M, G) (the warm-up path of Sec. 4.3) is g4d_render on
 * activated canonical Gaussians.
 *
 * Conventions shared by every call
 *   - Every array pointer is a DEVICE pointer, allocated and owned by the
 *     caller; the library never allocates device memory in these calls
 *     (the serving calls at the end are the documented exception: the
 *     server owns what it allocates).
 *   - Per-Gaussian arrays are structure-of-arrays, component-major:
 *     means[3][n] is x[0..n), y[0..n), z[0..n).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls only enqueue work; nothing synchronises unless stated.
 *   - Errors detected on the host are returned synchronously, nothing is
 *     enqueued then.  Device-side conditions (instance overflow) are
 *     recorded in the workspace and read with g4d_read_status.
 *   - No C++ exception crosses the ABI.  Calls on distinct workspaces and
 *     streams may run concurrently.
 */
#ifndef G4D_H
#define G4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    G4D_OK = 0,
    G4D_EINVAL = -1,        /* bad argument (null pointer, size out of range) */
    G4D_EUNSUPPORTED = -2,  /* shape outside the compiled set (feat, scales, hidden) */
    G4D_ECAPACITY = -3,     /* tile instances exceeded the workspace capacity */
    G4D_EHIP = -4,          /* a HIP runtime call failed; see g4d_last_hip_error */
    G4D_EBUSY = -5,         /* serving: no slot or memory free right now */
    G4D_ENOMEM = -6,        /* request larger than the memory budget (serving) or the fixed array (g4d_render_noalloc) */
    G4D_ENOTFOUND = -7,     /* serving: unknown scene or ticket */
    G4D_EDEVICE = -8        /* a device-side consistency check failed */
} g4d_status;

#define G4D_MAX_SCALES 4
#define G4D_TILE 16

/* Canonical 3D Gaussians G (Sec. 3.1): position X, SH colour coefficients,
 * opacity, rotation r and scaling s.  Scales are stored as logarithms and
 * opacity as a logit; g4d_deform applies exp and sigmoid after Eq. 8. */
typedef struct {
    int32_t n;                  /* number of Gaussians, >= 0 */
    int32_t sh_degree;          /* 0..3 */
    const float *means;         /* [3][n] */
    const float *log_scales;    /* [3][n] */
    const float *quats;         /* [4][n], (w, x, y, z), need not be unit */
    const float *opacity_logits;/* [n] */
    const float *sh;            /* [(d+1)^2][3][n]; read by g4d_deform only with a colour head */
} g4d_gaussians;

/* Multi-resolution HexPlane R_l(i, j) (Sec. 4.2, Eq. 7).  For each scale l
 * there are six planes in the order (x,y), (x,z), (y,z), (x,t), (y,t), (z,t);
 * plane (a, b) is stored channels-last as [res_b][res_a][feat] float32.
 * Canonical means are mapped to [-1, 1] through the box [bmin, bmax] and t
 * in [0, 1] to 2t - 1; lookups use align-corners bilinear interpolation
 * with clamping at the border.  Features are multiplied element-wise over
 * the six planes of a scale and concatenated over scales: in_dim = feat *
 * n_scales.  Supported: feat in {16, 32}, n_scales in {1, 2, 3}, every
 * resolution >= 2. */
typedef struct {
    int32_t n_scales;
    int32_t feat;
    float bmin[3];
    float bmax[3];
    int32_t res[G4D_MAX_SCALES][4];            /* (Rx, Ry, Rz, Rt) per scale */
    const float *plane[G4D_MAX_SCALES][6];
} g4d_planes;

typedef enum { G4D_MLP_F32 = 0, G4D_MLP_BF16 = 1 } g4d_mlp_precision;

/* Deformation decoder (Sec. 4.2): h = ReLU(W1 f_h + b1) (the feature
 * merger phi_d), then three linear heads dX = Wx h + bx (3), dr = Wr h + br
 * (4), ds = Ws h + bs (3).  Row-major float32 weights.  precision
 * G4D_MLP_BF16 rounds f_h, the weights and h to bfloat16 for the matrix
 * products (FP32 accumulation, FP32 biases).  Supported hidden: 32, 64,
 * 128.
 *
 * Optional heads of the appendix's colour and opacity deformation (both
 * null, the default, for the method of Sec. 4.2): dC = Wc h + bc, one row
 * per SH coefficient in the [(d+1)^2][3] order of the colour array (so
 * 3 (d+1)^2 rows for the scene's SH degree d), added to the canonical
 * coefficients; dalpha = Wa h + ba (1 row), added to the opacity logit
 * before the sigmoid.  With more than 16 head rows in total (dX dr ds dC
 * dalpha: a colour head at SH degree >= 1) only G4D_MLP_F32 is supported
 * (G4D_EUNSUPPORTED otherwise).  A weight and its bias are given or null
 * together (G4D_EINVAL otherwise). */
typedef struct {
    int32_t in_dim;             /* must equal feat * n_scales */
    int32_t hidden;
    int32_t precision;          /* g4d_mlp_precision */
    const float *w1, *b1;       /* [hidden][in_dim], [hidden] */
    const float *wx, *bx;       /* [3][hidden], [3] */
    const float *wr, *br;       /* [4][hidden], [4] */
    const float *ws, *bs;       /* [3][hidden], [3] */
    const float *wc, *bc;       /* [3 (d+1)^2][hidden], [3 (d+1)^2], or NULL */
    const float *wa, *ba;       /* [1][hidden], [1], or NULL */
} g4d_mlp;

/* Render-ready Gaussians G' (the set after Eq. 8 and activation): linear
 * scales, unit quaternions, opacity in (0, 1).  g4d_deform writes means,
 * scales, quats and opacity, and sh when the decoder has a colour head;
 * g4d_render only reads. */
typedef struct {
    int32_t n;
    int32_t sh_degree;          /* 0..3 */
    float *means;               /* [3][n] */
    float *scales;              /* [3][n] */
    float *quats;               /* [4][n] (w, x, y, z), unit */
    float *opacity;             /* [n] */
    float *sh;                  /* [(d+1)^2][3][n] */
} g4d_splats;

/* Pinhole view M = [R, T] (Sec. 4.1).  Camera axes: x right, y down,
 * z forward.  viewmat is the row-major 3x4 world-to-camera matrix whose
 * 3x3 block is the viewing transform W of Eq. 3.  Pixel (px, py) is
 * sampled at image coordinates (px, py); projection u = fx x/z + cx.
 * Gaussians with camera depth z <= near_plane are culled. */
typedef struct {
    int32_t width, height;      /* 1..4096 */
    float viewmat[12];
    float fx, fy, cx, cy;
    float tan_half_fov_x, tan_half_fov_y;
    float near_plane;
    float campos[3];            /* camera centre in world space (for SH view direction) */
    float bg[3];                /* background colour */
} g4d_camera;

/* Caller-owned device scratch for one render at a time.  `ptr` holds at
 * least g4d_render_workspace_bytes(n_max, width_max, height_max,
 * instance_capacity) bytes, 256-byte aligned.  A workspace may be reused
 * by renders of any size within its maxima; two renders in flight need two
 * workspaces. */
typedef struct {
    void *ptr;
    size_t bytes;
    int32_t n_max;
    int32_t width_max, height_max;
    int64_t instance_capacity;  /* max number of (Gaussian, tile) pairs, < 2^30 */
} g4d_workspace;

/* Gradients with respect to render-ready Gaussians (same layouts as
 * g4d_splats). */
typedef struct {
    float *means;               /* [3][n] */
    float *scales;              /* [3][n] */
    float *quats;               /* [4][n] */
    float *opacity;             /* [n] */
    float *sh;                  /* [(d+1)^2][3][n] */
} g4d_splats_grad;

/* Device-side outcome of the last render on a workspace. */
typedef struct {
    int64_t instances;          /* K: (Gaussian, tile) pairs the frame needed */
    int32_t overflow;           /* 1 if instances > instance_capacity (image invalid) */
    int32_t sort_error;         /* nonzero if a bounded wait in the sort gave up */
    int32_t visible;            /* Gaussians that touched at least one tile */
    int32_t tiles;              /* tiles_x * tiles_y of the frame */
    int64_t blend_evals;        /* list entries the pixels visited up to their stop (-1: not counted) */
    int64_t blend_composited;   /* of those, the ones the blend composited after its per-quadrant
                                   cull (-1: not counted); both are counted by a render that writes
                                   n_contrib or final_T */
} g4d_device_status;

/* ---------------------------------------------------------------- deform */

/* Eq. 7 + Eq. 8 + activations for G->n Gaussians at time t in [0, 1].
 * Writes out->means (X + dX), out->scales (exp(log_s + ds)), out->quats
 * (normalise(r + dr), identity if the sum is zero) and out->opacity
 * (sigmoid(logit [+ dalpha])); out->n must equal G->n.  Without a colour
 * head out->sh and out->sh_degree are not touched (callers point out->sh at
 * G->sh); with one, out->sh_degree must equal G->sh_degree and out->sh
 * (a buffer of its own, not G->sh) receives G->sh + dC.  The output buffers
 * must not alias the inputs. */
g4d_status g4d_deform(const g4d_gaussians *G, const g4d_planes *P, const g4d_mlp *M, float t,
                      g4d_splats *out, void *stream);

/* One deformation job of a batched launch. */
typedef struct {
    const g4d_gaussians *G;
    const g4d_planes *P;
    const g4d_mlp *M;
    float t;
    g4d_splats *out;
} g4d_deform_job;

#define G4D_MAX_BATCH_JOBS 8

/* Several g4d_deform calls in one kernel launch (continuous batching).  All
 * jobs must share feat, n_scales, hidden, precision and the head-tile count
 * (one 16-row tile of head rows, or four); each thread block
 * works on Gaussians of a single job, so every job's output is bitwise the
 * same as a lone g4d_deform call.  1 <= n_jobs <= G4D_MAX_BATCH_JOBS. */
g4d_status g4d_deform_batched(const g4d_deform_job *jobs, int32_t n_jobs, void *stream);

/* Placement of one scene in a composition (the naive rigid edit of the
 * appendix's "Editing with 4D Gaussians"): after Eq. 8 and the activations,
 * mean'' = scale * R(rotation) mean' + translation, quat'' = rotation (x)
 * quat' (Hamilton product, so the Gaussian's rotation matrix becomes
 * R(rotation) R(quat')), scales'' = scale * scales'; opacity and the SH
 * coefficients are kept (view-dependent colour is not rotated). */
typedef struct {
    float rotation[4];          /* (w, x, y, z), nonzero; normalised by the call */
    float scale;                /* uniform, > 0 and finite */
    float translation[3];
} g4d_placement;

/* One scene of a composition: its canonical Gaussians, field, decoder (with
 * or without the colour / opacity heads), time and placement. */
typedef struct {
    const g4d_gaussians *G;
    const g4d_planes *P;
    const g4d_mlp *M;
    float t;
    g4d_placement place;
} g4d_compose_item;

#define G4D_MAX_COMPOSE_ITEMS 64

/* Multi-scene composition (Sec. 5.4, "Composition with 4D Gaussians"): the
 * deformed sets of several trained scenes placed in one space,
 * G' = {G'_1, ..., G'_n}, written into one render-ready set that a single
 * g4d_render call draws.  Item i fills the index range [o_i, o_i + n_i) of
 * every structure-of-arrays row of `out`, o_i = n_0 + ... + n_(i-1);
 * out->n must equal the sum of the n_i.  out->sh holds
 * [(D+1)^2][3][out->n] with D = out->sh_degree >= every item's SH degree:
 * an item's coefficients (C, or C + dC with a colour head) fill its range of
 * its own rows and zeros the rows of higher bands (the same colour).
 * out->sh must be a buffer of its own.  Items whose deform kernels differ
 * (feat, n_scales, hidden, precision, head tiles) run as separate launches
 * on the stream, in order; each item's values are bitwise those of a lone
 * g4d_deform followed by the placement (none at the identity placement).
 * 1 <= n_items <= G4D_MAX_COMPOSE_ITEMS; every argument is checked before
 * the first launch.  Device pointers throughout. */
g4d_status g4d_deform_compose(const g4d_compose_item *items, int32_t n_items, g4d_splats *out,
                              void *stream);

/* A spatial storage order for a Gaussian set: the Gaussians sorted by the
 * 30-bit Morton code of their canonical means, quantised to 1024 cells per
 * axis over the box [bmin, bmax] (means outside are clamped to it; the
 * HexPlane's box is the natural choice), ties in index order.  A set stored
 * in this order (every per-Gaussian array permuted once, e.g. when a scene is
 * loaded) puts Gaussians that query neighbouring plane cells, and that
 * project to neighbouring tiles, in the same deform blocks and near each
 * other in memory.  The set is the same; only its numbering, and so the
 * index tie-break of equal depths, changes.  Uses `ws` (a render workspace
 * with n_max >= G->n) as scratch; writes order[n] (device): order[i] is the
 * index of the i-th Gaussian of the new order.  Asynchronous.  G4D_EINVAL
 * for a null argument, n outside the workspace or an empty box. */
g4d_status g4d_spatial_order(const g4d_gaussians *G, const float bmin[3], const float bmax[3],
                             const g4d_workspace *ws, uint32_t *order, void *stream);

/* The encoder output f_h (Eq. 7) alone, [n][in_dim] float32: exposes the
 * intermediate of g4d_deform for verification.  Same kernel code path. */
g4d_status g4d_deform_features(const g4d_gaussians *G, const g4d_planes *P, float t,
                               float *features, void *stream);

/* ---------------------------------------------------------------- render */

/* Bytes of workspace for renders of up to n Gaussians at up to width x
 * height with up to instance_capacity tile instances.  Returns 0 for
 * arguments out of range. */
size_t g4d_render_workspace_bytes(int32_t n, int32_t width, int32_t height,
                                  int64_t instance_capacity);

/* I = S(M, G') (Sec. 3.1, Eq. 1-4).  Per Gaussian: project (Eq. 2-3 with
 * a 0.3-pixel dilation of the 2D covariance), bound by a square of radius
 * ceil(3 sqrt(lambda_max)), bin into 16x16 tiles.  Instances are keyed
 * (tile_id << 32) | float_bits(depth) and radix-sorted (ties keep Gaussian
 * index order).  Per pixel, Gaussians of its tile are composited front to
 * back: alpha = min(0.99, o exp(-d^T Sigma'^-1 d / 2)), skipped below
 * 1/255, stopping before transmittance would fall below 1e-4; the output
 * is sum c alpha T + T_final bg.
 *   image     [3][height][width] float32 (required)
 *   final_T   [height][width] float32 or NULL
 *   n_contrib [height][width] int32 or NULL: list entries visited up to the
 *             last contributing Gaussian
 * If the frame needs more instances than the workspace holds, the image is
 * left incomplete and g4d_read_status reports overflow with the required
 * count.  Asynchronous; graph-capturable (no host synchronisation, no
 * allocation, fixed launch shapes for fixed arguments). */
g4d_status g4d_render(const g4d_splats *G, const g4d_camera *C, const g4d_workspace *ws,
                      float *image, float *final_T, int32_t *n_contrib, void *stream);

/* Bytes of the library's own device array that g4d_render_noalloc uses as
 * its workspace (128 MiB; one copy per GPU, held until the process ends). */
#define G4D_NOALLOC_SCRATCH_BYTES (128u << 20)

/* g4d_render without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops and harnesses
 * that forbid hipMalloc).  The workspace is a fixed device array of the
 * library, G4D_NOALLOC_SCRATCH_BYTES per GPU; the instance capacity of a call
 * is the largest cap with g4d_render_workspace_bytes(max(n, 1), width, height,
 * cap) <= G4D_NOALLOC_SCRATCH_BYTES (about 7.2 million instances for 100k
 * Gaussians at 800x800).  Same kernels, arguments and outputs as g4d_render.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * call); the first call on a device looks up that device's copy of the
 * array.  Every call on one GPU shares that GPU's array: calls that overlap on
 * one device (other streams or threads) race and must be serialised by the
 * caller.  Nothing carries over between calls (the render clears what it
 * needs at zero).
 *   status  NULL: asynchronous, as g4d_render (an overflowed frame is then
 *           not reported).  Non-NULL: the call waits for `stream` and fills
 *           it (blend_evals and blend_composited are -1, not counted here);
 *           returns G4D_ECAPACITY
 *           if the frame needed more instances than the array holds
 *           (status->instances gives the count; the image is incomplete) and
 *           G4D_EDEVICE if a bounded wait in the sort gave up.
 * G4D_ENOMEM, before any device work, if (n, width, height) leaves no room
 * in the array for even one instance; G4D_EINVAL as g4d_render. */
g4d_status g4d_render_noalloc(const g4d_splats *G, const g4d_camera *C, float *image, float *final_T,
                              int32_t *n_contrib, g4d_device_status *status, void *stream);

/* Copies the device status of the last render on `ws` to the host.  Waits
 * for `stream` to finish. */
g4d_status g4d_read_status(const g4d_workspace *ws, g4d_device_status *out, void *stream);

/* Intermediates of the last render on `ws`, copied device-to-device into
 * `dst` (asynchronous on `stream`); for verification. */
typedef enum {
    G4D_EXPORT_SORTED_KEYS = 0,   /* uint64 [K]: (tile << 32) | depth bits, sorted */
    G4D_EXPORT_SORTED_GIDS = 1,   /* uint32 [K]: Gaussian index per sorted instance */
    G4D_EXPORT_RECT = 2,          /* int32 [n][4]: tile rectangle x0, y0, x1, y1 (empty if culled) */
    G4D_EXPORT_DEPTH_BITS = 3,    /* uint32 [n]: float bits of camera depth, 0xffffffff if culled */
    G4D_EXPORT_RANGES = 4,        /* uint32 [tiles][2]: [start, end) into the sorted list */
    G4D_EXPORT_SPLAT2D = 5,       /* float32 [n][12]: u, v, -A/2, -C/2, -B, opacity, r, g, b, 0,0,0
                                     where (A, B, C) is the conic Sigma'^-1 */
    G4D_EXPORT_DEPTH_ORDER = 6    /* uint32 [n]: Gaussian indices sorted by (depth bits, index) */
} g4d_export_kind;

/* n: Gaussians of the frame; k: instances to copy for the SORTED kinds
 * (at most K, use g4d_read_status), or the frame's tile count for RANGES.
 * dst: device buffer of at least dst_bytes. */
g4d_status g4d_render_export(const g4d_workspace *ws, int32_t kind, int32_t n, int64_t k,
                             void *dst, size_t dst_bytes, void *stream);

/* Stage timing: after this call, every g4d_render on the calling thread
 * records events[i] (a hipEvent_t, or NULL to skip) on its stream at stage
 * boundary i: 0 start, 1 after clearing, 2 preprocess, 3 depth sort,
 * 4 instance offsets, 5 emit, 6 tile sort, 7 ranges, 8 blend.  count must
 * be 9; events == NULL turns recording off.  The caller owns the events. */
g4d_status g4d_set_stage_events(void *const *events, int32_t count);

/* ------------------------------------------------------------- backward */

/* Gradient of a scalar loss L through the last g4d_render on `ws`
 * (Eq. 1-4 and Eq. 2-3): given dL/dimage (grad_image, [3][H][W] like the
 * image), writes dL/d(means, scales, quats, opacity, sh) of the render-ready
 * Gaussians into `grad` (overwritten, not accumulated; zero for Gaussians
 * that touch no pixel).  The render must have been called with these G and C
 * and with final_T and n_contrib outputs, which are passed here unchanged;
 * the workspace must not have been used since.  Per-tile recomputation: each
 * pixel walks its tile's list back to front from its final transmittance and
 * last contributing entry, redoing the forward's binary32 alpha (so skip and
 * stop decisions are the forward's); alpha clamped at 0.99 passes no
 * gradient to opacity or position.  Gradients with respect to the camera are
 * not computed.  A render that overflowed its instance capacity (see
 * g4d_read_status) has truncated lists, and so do these gradients.
 * G4D_EINVAL for a null argument or sizes outside the workspace's maxima.
 * Device pointers; the call allocates nothing. */
g4d_status g4d_render_backward(const g4d_splats *G, const g4d_camera *C, const g4d_workspace *ws,
                               const float *final_T, const int32_t *n_contrib, const float *grad_image,
                               const g4d_splats_grad *grad, void *stream);

/* Gradients with respect to the deformation's inputs: the canonical
 * Gaussians (same layouts as g4d_gaussians), every plane cell (same layouts
 * as g4d_planes) and the decoder weights (same layouts as g4d_mlp; the
 * colour / opacity head entries are used when the decoder has them). */
typedef struct {
    float *means;               /* [3][n] */
    float *log_scales;          /* [3][n] */
    float *quats;               /* [4][n] */
    float *opacity_logits;      /* [n] */
    float *sh;                  /* [(d+1)^2][3][n], or NULL when not wanted */
    float *plane[G4D_MAX_SCALES][6];
    float *w1, *b1, *wx, *bx, *wr, *br, *ws, *bs;
    float *wc, *bc, *wa, *ba;
} g4d_deform_grad;

/* Gradient of a scalar loss L through g4d_deform (Sec. 4.2, Eq. 7-8): given
 * dL/d(render-ready set) in grad_out (e.g. from g4d_render_backward),
 * writes dL/d(canonical Gaussians) and accumulates, from zero, dL/d(plane
 * cells) and dL/d(decoder weights) into `grad` (the call clears them first).
 * The forward is recomputed (nothing from it is kept); plane gradients are
 * an atomic scatter of the bilinear weights; the grid coordinates carry the
 * bilinear slopes, zero for a mean on or outside the box border (where the
 * query is clamped) and for the time axis (t is not a parameter).
 * FP32 decoder only (G4D_EUNSUPPORTED for G4D_MLP_BF16, and for a
 * (feat, n_scales, hidden) outside the compiled set); G4D_EINVAL for a
 * null argument, a head weight without its bias or gradient array, or t
 * outside [0, 1].  Device pointers; the call allocates nothing. */
g4d_status g4d_deform_backward(const g4d_gaussians *G, const g4d_planes *P, const g4d_mlp *M, float t,
                               const g4d_splats_grad *grad_out, const g4d_deform_grad *grad, void *stream);

/* The image term of the training loss (Eq. 9): loss = mean |image - target|
 * over `count` values (a device scalar, cleared by the call; may be NULL)
 * and grad = dloss/dimage = sign(image - target) / count (0 where equal;
 * may be NULL).  G4D_EINVAL for null inputs, count < 1 or both outputs
 * NULL.  Device pointers. */
g4d_status g4d_l1_loss(const float *image, const float *target, int64_t count, float *loss, float *grad,
                       void *stream);

/* The grid total-variation term of Eq. 9 on the HexPlane cells.  The paper
 * names the term without a formula or weight; this is the K-Planes form:
 * for every plane [n_b][n_a][F] of every scale, the mean squared difference
 * of neighbouring cells along a plus the same along b, summed over planes,
 * times `weight` (1 in Eq. 9).  Writes the value into the device scalar
 * `loss` (cleared by the call; may be NULL) and ADDS weight x dtv/dcell to
 * grad->plane (may be NULL), so it follows g4d_deform_backward.
 * G4D_EINVAL for a plane set outside the supported shapes (1-3 scales, F 16
 * or 32, resolutions >= 2), a null plane or gradient plane, or both outputs
 * NULL.  Device pointers. */
g4d_status g4d_tv_loss(const g4d_planes *P, float weight, float *loss, g4d_deform_grad *grad, void *stream);

/* One trainable tensor of an Adam update: count FP32 values of param, their
 * gradient and the two moment buffers (zero before the first step), and the
 * tensor's learning rate. */
typedef struct {
    float *param;
    const float *grad;
    float *m, *v;
    int64_t count;              /* 0 .. 2^32 - 1 */
    float lr;
} g4d_adam_tensor;

/* Adam (the optimiser the method trains with): for step >= 1,
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * param -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps),
 * for 1 <= n <= 64 tensors in one launch.  G4D_EINVAL for a null pointer,
 * n or a count out of range, step < 1 or a beta outside [0, 1).  Device
 * pointers. */
g4d_status g4d_adam_step(const g4d_adam_tensor *tensors, int32_t n, float beta1, float beta2, float eps,
                         int32_t step, void *stream);

/* -------------------------------------------------------------- utilities */

const char *g4d_status_string(int32_t status);
int32_t g4d_last_hip_error(void);   /* hipError_t of the last G4D_EHIP */
const char *g4d_version(void);

/* ------------------------------------------------------------- serving */

/* A request loop that keeps several scenes resident in HBM and renders
 * (scene, camera, t) requests with continuous batching: requests are
 * admitted while render slots and the memory budget allow, the
 * deformations of newly admitted requests run as one batched launch per
 * shape class (on the stream of the first request of the class), and each
 * admitted request renders on its own stream (replaying a captured graph per
 * buffer set and frame size when it overlaps other requests), so requests
 * that arrive while others run overlap on the device.  The server owns all
 * memory it allocates; images are written to caller device buffers. */
typedef struct g4d_server g4d_server;

typedef struct {
    size_t hbm_budget;          /* bytes for per-request memory (workspaces, deformed sets) */
    int32_t max_slots;          /* concurrent requests on the device, 1..64 */
    int32_t use_graphs;         /* replay captured HIP graphs for renders that overlap other
                                   requests (a request alone on the device launches directly) */
    int32_t batch_deform;       /* 1: batched deformation per admission round */
    int32_t max_width, max_height;
    double instance_factor;     /* capacity = factor * n * tiles-per-Gaussian bound; see server.cpp */
} g4d_server_config;

typedef struct {
    int64_t submitted, completed, rejected;
    double p50_ms, p99_ms, mean_ms, max_ms;
    double wall_s;              /* first submit to last completion */
    double frames_per_s;
    int64_t batched_launches, graph_replays, eager_renders, overflow_retries;
    size_t peak_bytes;
} g4d_server_stats;

g4d_status g4d_server_create(const g4d_server_config *cfg, g4d_server **out);
/* Copies the scene into server-owned HBM; the caller's buffers may be
 * freed afterwards.  Device pointers in G, P, M. */
g4d_status g4d_server_add_scene(g4d_server *srv, const g4d_gaussians *G, const g4d_planes *P,
                                const g4d_mlp *M, int32_t *scene_id);
/* Non-blocking.  out_image: device [3][H][W] float32 owned by the caller,
 * valid once g4d_server_wait returns G4D_OK for the ticket. */
g4d_status g4d_server_submit(g4d_server *srv, int32_t scene_id, const g4d_camera *cam, float t,
                             float *out_image, uint64_t *ticket);
/* Blocks until the request completes; latency from submit to completion. */
g4d_status g4d_server_wait(g4d_server *srv, uint64_t ticket, double *latency_ms);
g4d_status g4d_server_drain(g4d_server *srv);
g4d_status g4d_server_stats_get(g4d_server *srv, g4d_server_stats *out);
g4d_status g4d_server_reset_stats(g4d_server *srv);
g4d_status g4d_server_destroy(g4d_server *srv);

/* The scheduler of the serving loop on a simulated device, in virtual time:
 * the same FIFO admission, memory-budget accounting with buffer reuse, slot
 * and batching logic as g4d_server_*, driven by a given arrival trace.  Each
 * request i arrives at arrival_s[i], needs bytes[i] of request memory while
 * it runs (reused by a later request of the same class_id once released) and
 * takes service_s[i] of device time when alone; with m requests on the
 * device each progresses at rate (1 + overlap (m - 1)) / m.  Needs no GPU;
 * used to verify the scheduler. */
typedef struct {
    size_t hbm_budget;
    int32_t max_slots;
    int32_t batch_deform;
    int32_t n_requests;
    const double *arrival_s;    /* [n], non-decreasing */
    const double *service_s;    /* [n] */
    const size_t *bytes;        /* [n] */
    const int32_t *class_id;    /* [n] */
    const int32_t *shape_class; /* [n]: requests of one shape class share a batched deform launch */
    double overlap;             /* 0..1 */
} g4d_sim_config;

typedef struct {
    double p50_ms, p99_ms, mean_ms, max_ms, makespan_s;
    size_t peak_bytes;          /* request memory held at once (in use + kept for reuse) */
    int32_t max_in_flight;
    int32_t rejected;
    int64_t batched_launches;
    int64_t buffer_reuses;
    double *latency_ms;         /* optional [n]: per request, -1 if rejected */
    int32_t *admit_order;       /* optional [n]: request indices in admission order */
} g4d_sim_result;

g4d_status g4d_server_simulate(const g4d_sim_config *cfg, g4d_sim_result *out);

#ifdef __cplusplus
}
#endif
#endif /* G4D_H */
