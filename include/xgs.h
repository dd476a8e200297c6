/*
 * xgs.h -- C ABI of the MI355X (gfx950) hot path of the X-GS Perceiver
 * (arXiv 2603.09632): differentiable tile-based 3D Gaussian splatting of RGB,
 * depth and semantic channels, grid-sampled distillation targets, and
 * EMA-updated vector-quantisation codebook assignment.
 *
 * Conventions shared by every call
 *   - All array arguments are DEVICE pointers unless stated otherwise.  The
 *     caller owns every buffer; the library never allocates device memory and
 *     keeps no mutable global state.  Scratch space is passed in as a
 *     workspace whose size comes from the matching *_workspace() query.  The
 *     one exception is xgs_tile_sort_noalloc, which uses a fixed scratch
 *     array the library holds on each GPU.
 *   - Every call is asynchronous and ordered on the hipStream_t passed in
 *     (NULL = the legacy default stream).  No call synchronises the host, so
 *     every call may be captured into a HIP graph.
 *   - Arguments are validated on the host before any launch.  On failure the
 *     call returns a nonzero xgs_status, launches nothing, and
 *     xgs_last_error() (thread-local) describes the problem.  A failed kernel
 *     launch returns XGS_ERR_HIP.  No C++ exception crosses the ABI.
 *   - Device-side overflow (more (tile, Gaussian) instances than the buffers
 *     hold) sets *status in device memory to a nonzero value; the kernels then
 *     stay within the buffers.  The caller reads the status after its own sync.
 *   - Layouts: per-Gaussian arrays are row-major [n][k] (one row per Gaussian,
 *     as torch stores an (n, k) tensor); images are planar [C][H_s][W_s]; VQ
 *     arrays are row-major [N][D] and [K][D].  All float data is IEEE binary32.
 *   - Calls are re-entrant on distinct buffers and streams.
 *
 * Readings of the paper fixed by this interface (the paper leaves them open):
 *   alpha = min(0.99, o G); pairs with alpha < 1/255 are skipped; a pixel stops
 *   before blending the Gaussian that would take its transmittance below 1e-4;
 *   Sigma' gets a 0.3 I dilation; background is 0; tiles are 16 x 16 sampled
 *   pixels; the depth channel is camera z of the Gaussian mean.
 */
#ifndef XGS_H
#define XGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* xgs_stream_t; /* identical to hipStream_t */

typedef enum {
    XGS_OK = 0,
    XGS_ERR_INVALID_ARG = 1, /* a size, pointer or alignment the call cannot accept */
    XGS_ERR_CAPACITY = 2,    /* a caller-provided buffer or workspace is too small   */
    XGS_ERR_HIP = 3,         /* the HIP runtime reported an error at launch          */
    XGS_ERR_UNSUPPORTED = 4  /* valid request outside what the library implements  */
} xgs_status;

enum { XGS_TILE = 16 };                     /* tile edge in sampled pixels          */
enum { XGS_MAX_C_SEM = 64 };                /* semantic channels per Gaussian        */
enum { XGS_SPLAT_STRIDE = 8 };              /* floats per projected splat record     */
enum { XGS_GRID_BILINEAR = 0, XGS_GRID_NEAREST = 1 };
enum { XGS_VQ_FP32 = 0, XGS_VQ_BF16_RESCORE4 = 1 };
enum { XGS_EMA_PAPER = 0, XGS_EMA_LAPLACE = 1 };

/* Pinhole camera and sampled grid (host struct, passed by pointer).
 * viewmat: world -> camera, row-major 4x4, OpenCV axes (x right, y down,
 * z forward).  The sampled grid is H_s x W_s = ceil(H/stride) x ceil(W/stride);
 * grid pixel (m, n) is image pixel (off_y + m*stride, off_x + n*stride) with its
 * centre at (off_x + n*stride + 0.5, off_y + m*stride + 0.5) -- Eq. (sampled_loc).
 * Gaussians with camera z <= near_plane are culled.  (stride, off_y, off_x) =
 * (1, 0, 0) renders the dense image.  0 <= off_y, off_x < stride. */
typedef struct xgs_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float viewmat[16];
    float near_plane;
    int32_t stride, off_y, off_x;
} xgs_camera;

/* A set of 3D Gaussians Theta_i = {mu, Sigma = R S S^T R^T, o, c} with
 * semantic features f_i (Sec. 3.1, App. A).  Device pointers, row-major:
 *   means [n][3], log_scales [n][3] (S = diag(exp(l))), quats [n][4]
 *   (w, x, y, z; any nonzero length, normalised inside), opacity [n]
 *   (activated, in (0,1]), colors [n][3], features [n][c_sem].
 * features may be NULL when c_sem == 0.  The same struct with writable
 * pointers carries gradients (xgs_gaussians_grad). */
typedef struct xgs_gaussians {
    int64_t n;
    int32_t c_sem;
    int32_t reserved;
    const float* means;
    const float* log_scales;
    const float* quats;
    const float* opacity;
    const float* colors;
    const float* features;
} xgs_gaussians;

typedef struct xgs_gaussians_grad {
    int64_t n;
    int32_t c_sem;
    int32_t reserved;
    float* means;       /* [n][3] */
    float* log_scales;  /* [n][3] */
    float* quats;       /* [n][4] */
    float* opacity;     /* [n]    */
    float* colors;      /* [n][3] */
    float* features;    /* [n][c_sem] */
} xgs_gaussians_grad;

/* Output of xgs_project (device buffers of n rows, caller-allocated):
 *   splat [n][8], 16-byte aligned: mean2d.x, mean2d.y, conic A, B, C (the
 *     quadratic form A dx^2 + 2B dx dy + C dy^2 of Sigma'^-1), opacity,
 *     depth (camera z), 0.
 *   radius [n]: ceil of the larger half-width of the splat's box, 0 = culled.
 *   tile_rect [n][4] u16: tiles [x0, x1) x [y0, y1) stored x0, y0, x1, y1.
 *   tiles_touched [n]: (x1-x0)(y1-y0), 0 when culled. */
typedef struct xgs_projected {
    float* splat;
    int32_t* radius;
    uint16_t* tile_rect;
    uint32_t* tiles_touched;
} xgs_projected;

/* Depth-sorted per-tile instance lists produced by xgs_tile_sort:
 *   keys [max_instances] = (tile_id << 32) | bits(depth) with
 *     tile_id = ty * tiles_x + tx, sorted ascending, ties by Gaussian index;
 *   vals [max_instances] = Gaussian index of each key;
 *   ranges [num_tiles][2] = [first, last+1) of each tile, (0, 0) if empty;
 *   num_instances: device int64 = number of valid keys M;
 *   status: device int32, 0 = ok, 1 = the instances exceeded max_instances;
 *     then num_instances = 0 and every range is empty (nothing is rendered),
 *     and the caller retries with larger buffers;
 *   tile_order [num_tiles] (may be NULL): the order in which the compositing
 *     kernels take the tiles, written by xgs_tile_sort: descending list
 *     length in buckets of 16 instances, ties by tile id (identity above
 *     16384 tiles).  NULL: tiles in id order.  Any permutation gives the same
 *     images and gradients up to the order of the gradient atomics. */
typedef struct xgs_binning {
    uint64_t* keys;
    uint32_t* vals;
    uint32_t* ranges;
    int64_t* num_instances;
    int32_t* status;
    int64_t max_instances;
    uint32_t* tile_order;
} xgs_binning;

/* ------------------------------------------------------------------ info */
const char* xgs_status_string(xgs_status s);
/* Description of the last failure on the calling thread ("" if none). */
const char* xgs_last_error(void);
int32_t xgs_version(void);
/* Sampled-grid geometry of a camera: writes H_s, W_s, tiles_y, tiles_x. */
xgs_status xgs_grid_dims(const xgs_camera* cam, int32_t* hs, int32_t* ws,
                         int32_t* tiles_y, int32_t* tiles_x);

/* ---------------------------------------------------------- a1: project
 * EWA projection (App. A): Sigma = R S S^T R^T, p = W mu + t,
 * Sigma' = J W Sigma W^T J^T + 0.3 I with J the perspective Jacobian at p
 * (x/z, y/z clamped to +-1.3 (W/2)/fx, (H/2)/fy), mean2d = (fx x/z + cx,
 * fy y/z + cy), conic = Sigma'^-1.  The splat's box has half-widths
 * sqrt(2 ln(255 o) Sigma'_xx), sqrt(2 ln(255 o) Sigma'_yy): outside it
 * o G < 1/255.  Culled (radius 0, no tiles): z <= near, o < 1/255, or a box
 * that misses the sampled grid.  One thread per Gaussian; n may be 0. */
xgs_status xgs_project(const xgs_gaussians* g, const xgs_camera* cam, xgs_projected* out,
                       xgs_stream_t stream);
/* Same, with the world->camera matrix read from device memory (d_viewmat,
 * row-major 4x4 floats) instead of cam->viewmat: a captured HIP graph can then
 * be replayed for a new pose by rewriting those 16 floats.  Intrinsics, image
 * size and grid still come from *cam. */
xgs_status xgs_project_posed(const xgs_gaussians* g, const xgs_camera* cam, const float* d_viewmat,
                             xgs_projected* out, xgs_stream_t stream);

/* ------------------------------------------------------- a2: tile sort
 * Binning and depth sort ("depth-sorted Gaussians", Sec. 3.1): exclusive scan
 * of tiles_touched, emission of one key per (tile, Gaussian) in Gaussian
 * order, stable LSD radix sort over the 32 + ceil(log2(tiles)) key bits, and
 * per-tile ranges.  Reads p->tile_rect, p->tiles_touched and the depth of
 * p->splat.  ws must hold xgs_tile_sort_workspace(n, max_instances, tiles)
 * bytes, 256-byte aligned. */
size_t xgs_tile_sort_workspace(int64_t n, int64_t max_instances, int32_t num_tiles);
xgs_status xgs_tile_sort(const xgs_projected* p, const xgs_camera* cam, int64_t n, void* ws,
                         size_t ws_bytes, xgs_binning* b, xgs_stream_t stream);

/* Allocation-free tile sort, for callers that cannot allocate device memory
 * or pass a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * xgs_tile_sort, without ws: the sort runs in a scratch array of
 * xgs_tile_sort_noalloc_max_bytes() bytes (68 MiB: n = 2M Gaussians with
 * max_instances = 4M fit) that the library holds on each GPU it runs on until
 * the process ends.  A call whose xgs_tile_sort_workspace(n, max_instances,
 * tiles) exceeds that size returns XGS_ERR_CAPACITY before any launch.  The
 * entry point calls no hipMalloc, hipFree or allocating library routine.
 * All calls on one GPU share its scratch (later calls overwrite it): calls
 * that overlap on one GPU (different streams or threads without ordering)
 * race and must not be issued. */
size_t xgs_tile_sort_noalloc_max_bytes(void);
xgs_status xgs_tile_sort_noalloc(const xgs_projected* p, const xgs_camera* cam, int64_t n, xgs_binning* b,
                                 xgs_stream_t stream);

/* -------------------------------------------------- a3: render forward
 * Front-to-back alpha blending, Eq. (rendering): for every grid pixel walk its
 * tile's list, alpha = min(0.99, o exp(-q/2)); skip alpha < 1/255; stop
 * before blending when T (1 - alpha) < 1e-4; out += alpha T [rgb, depth, f].
 * out [4 + c_sem][H_s][W_s] (channel order R, G, B, depth, semantic...),
 * final_T [H_s][W_s] (transmittance after the last blended Gaussian),
 * n_last [H_s][W_s] (list position after the last blended Gaussian). */
xgs_status xgs_render_fwd(const xgs_gaussians* g, const xgs_projected* p, const xgs_binning* b,
                          const xgs_camera* cam, float* out, float* final_T, int32_t* n_last,
                          xgs_stream_t stream);

/* ------------------------------------------------- a4: render backward
 * Gradient of L = sum d_out * out with respect to every parameter group: the
 * derivative of Eq. (rendering) (front-to-back blending, App. B Eq.
 * (discrete_render)) with respect to alpha, colour, depth and features,
 * carried through alpha = min(0.99, o G) to opacity, conic and mean2d, then
 * back through the EWA projection of App. A (Sigma' = J W Sigma W^T J^T,
 * Sigma = R S S^T R^T) to mean, log-scale and quaternion.  Per
 * pixel the walk runs back to front from n_last, recovering the transmittance
 * before each Gaussian as T / (1 - alpha) from final_T (nothing per pair is
 * stored); dL/dalpha_k = T_k (g . c_k) - S_k / (1 - alpha_k).  Per-Gaussian
 * sums are reduced across each wavefront before one atomic add per value; a
 * second kernel carries (mean2d, conic, depth) gradients back through the
 * projection.  grads: all six arrays are overwritten (the call zeroes them).
 * flags: XGS_BWD_FEATURES_ONLY computes only d_features (geometry frozen,
 * Sec. 3.2.2 "decouple"); the other gradient pointers may then be NULL.
 * ws must hold xgs_render_bwd_workspace(n) bytes, 256-byte aligned. */
enum { XGS_BWD_ALL = 0, XGS_BWD_FEATURES_ONLY = 1, XGS_BWD_PREZEROED = 2 };
size_t xgs_render_bwd_workspace(int64_t n);
/* The zeroing that xgs_render_bwd does first, as a call of its own: the
 * accumulated gradients (features; with XGS_BWD_ALL also colours and
 * opacity) and the workspace's per-Gaussian rows.  A caller can issue it
 * earlier, on another stream (overlapping the forward pass), and then call
 * xgs_render_bwd with flags | XGS_BWD_PREZEROED on the same grads and ws,
 * which then skips its own zeroing; the caller orders the two (an event). */
xgs_status xgs_render_bwd_zero(const xgs_gaussians* g, int32_t flags, xgs_gaussians_grad* grads, void* ws,
                               size_t ws_bytes, xgs_stream_t stream);
xgs_status xgs_render_bwd(const xgs_gaussians* g, const xgs_projected* p, const xgs_binning* b,
                          const xgs_camera* cam, const float* d_out, const float* final_T,
                          const int32_t* n_last, int32_t flags, xgs_gaussians_grad* grads,
                          void* ws, size_t ws_bytes, xgs_stream_t stream);

/* ------------------------------------------- S3: batched render requests
 * The serving form renders several requests (scene, pose, resolution) in one
 * set of launches, each request a "slot".  Slot s owns a band of rows of a
 * virtual tile grid tiles_x tiles wide: its tile (x, y) is global tile
 * (row_base + y) * tiles_x + x, so one tile sort over the concatenated
 * projections, keyed by (global tile, depth) = (slot, tile, depth), gives
 * every slot's per-tile lists, and one compositing launch takes the tiles of
 * all slots.  Slot s's Gaussians take global indices [gauss_base, gauss_base
 * + g.n) in the batch's projected buffers.  Each slot renders exactly what
 * xgs_project + xgs_tile_sort + xgs_render_fwd give for it alone (same
 * arithmetic, same per-tile order), whatever else is in the batch.
 *
 * The slot table lives in DEVICE memory (n_slots entries), so a HIP graph of
 * the three calls replays for any batch that fits the capacities it was
 * captured with: the caller rewrites the table before each replay.  Launch
 * grids cover the capacities (cap_gaussians, tiles_x * tile_rows); work past
 * the table's content exits at once.  The table's contents cannot be checked
 * on the host: xgs_batch_check validates a host copy of it against the
 * capacities (call it before uploading).  Requirements per slot: 0 <= g.n,
 * gauss_base + g.n <= next slot's gauss_base (slots ascending, disjoint) and
 * the last slot's end <= cap_gaussians; the camera is valid with
 * tiles_x(cam) <= tiles_x; row_base ascending with bands [row_base, row_base
 * + tiles_y(cam)) disjoint and inside [0, tile_rows); g.c_sem equal to the
 * c_sem argument; out [4 + c_sem][H_s][W_s], final_T and n_last [H_s][W_s]
 * of the slot's grid. */
typedef struct xgs_batch_slot {
    xgs_gaussians g;     /* the slot's scene (device pointers), g.n Gaussians */
    xgs_camera cam;      /* the request's camera (viewmat = its pose)         */
    float* out;          /* [4 + c_sem][H_s][W_s]                             */
    float* final_T;      /* [H_s][W_s]                                        */
    int32_t* n_last;     /* [H_s][W_s]                                        */
    int64_t gauss_base;  /* first global Gaussian index of the slot           */
    int32_t row_base;    /* first row of the slot's band in the tile grid     */
    int32_t reserved;
} xgs_batch_slot;
enum { XGS_BATCH_MAX_SLOTS = 16 };

/* Validates a HOST copy of a slot table (see above). */
xgs_status xgs_batch_check(const xgs_batch_slot* h_slots, int32_t n_slots, int64_t cap_gaussians,
                           int32_t tiles_x, int32_t tile_rows, int32_t c_sem);
/* a1 over the batch: projects every slot's Gaussians with its camera into
 * global rows [gauss_base, gauss_base + n) of out (cap_gaussians rows), tile
 * rectangles in the slot's band of the virtual grid.  The batch is then
 * sorted by xgs_tile_sort (or xgs_tile_sort_noalloc) with n = cap_gaussians
 * and a camera whose grid is tiles_x x tile_rows tiles (width 16 tiles_x,
 * height 16 tile_rows, stride 1): the depth keys and rectangles are all it
 * reads.  Rows of no slot get only tiles_touched = 0 (their other fields are
 * left as they were). */
xgs_status xgs_batch_project(const xgs_batch_slot* d_slots, int32_t n_slots, int64_t cap_gaussians,
                             int32_t tiles_x, int32_t tile_rows, xgs_projected* out, xgs_stream_t stream);
/* a3 over the batch: every slot's tiles composited into its own out, final_T
 * and n_last, exactly as xgs_render_fwd does for one request.  b comes from
 * the batch tile sort; c_sem is every slot's channel count (0-4, 8, 16 or
 * 32).  b->tile_order may order the virtual grid's tiles as for one request. */
xgs_status xgs_batch_render_fwd(const xgs_batch_slot* d_slots, int32_t n_slots, int32_t c_sem,
                                int32_t tiles_x, int32_t tile_rows, const xgs_projected* p,
                                const xgs_binning* b, xgs_stream_t stream);

/* -------------------------------------------------- a5: grid-sampled targets
 * App. D, Eq. (target_continuous): for grid pixel (m, n) at image pixel
 * (u, v) = (off_y + m s, off_x + n s), u~ = u (Hf-1)/max(H-1,1),
 * v~ = v (Wf-1)/max(W-1,1).  NEAREST takes P at (round u~, round v~) (round
 * half to even, exact integer arithmetic); BILINEAR interpolates P at
 * (u~, v~).  V = 1 inside the image; V = 0 and G = 0 where u >= H or v >= W.
 * P [D][Hf][Wf], G [D][H_s][W_s], V [H_s][W_s] (V may be NULL). */
xgs_status xgs_grid_sample(const float* P, int32_t D, int32_t Hf, int32_t Wf, int32_t H,
                           int32_t W, int32_t stride, int32_t off_y, int32_t off_x, int32_t mode,
                           float* G, uint8_t* V, xgs_stream_t stream);

/* The targets of every grid offset of one stride in one launch (App. D,
 * Eq. (sampled_loc) over all (off_y, off_x) in [0, stride)^2; the device
 * form of the per-offset target prefetch of Sec. 3.2.2): grid
 * o = off_y * stride + off_x is bitwise what xgs_grid_sample writes for that
 * offset.  G [stride^2][D][H_s][W_s], V [stride^2][H_s][W_s] (V may be NULL),
 * H_s = ceil(H / stride), W_s = ceil(W / stride).  stride <=
 * XGS_GRID_MAX_STRIDE, else XGS_ERR_UNSUPPORTED; other errors as
 * xgs_grid_sample. */
enum { XGS_GRID_MAX_STRIDE = 64 };
xgs_status xgs_grid_sample_offsets(const float* P, int32_t D, int32_t Hf, int32_t Wf, int32_t H,
                                   int32_t W, int32_t stride, int32_t mode, float* G, uint8_t* V,
                                   xgs_stream_t stream);

/* ----------------------------------------- f2: camera-pose gradient (Eq. (tracking))
 * dL/dxi for the left perturbation T(xi) = exp(xi^) T of the world-to-camera
 * pose, xi = (rho, phi) (translation, rotation), at xi = 0:
 *   d_pose[0..2] = sum_i dL/dp_i,
 *   d_pose[3..5] = sum_i [ p_i x dL/dp_i + axial(Sc_i G_i - G_i Sc_i) ],
 * p_i camera-space mean, Sc_i camera covariance, G_i = dL/dSc_i,
 * axial(A) = (A_23 - A_32, A_31 - A_13, A_12 - A_21).
 * Call after xgs_render_bwd (XGS_BWD_ALL) on the same stream with the same
 * g, p, cam and ws: it reads the per-Gaussian image-space adjoints that pass
 * leaves in ws.  d_pose: 6 device floats.  Deterministic (fixed order). */
xgs_status xgs_pose_grad(const xgs_gaussians* g, const xgs_projected* p, const xgs_camera* cam,
                         const void* ws, size_t ws_bytes, float* d_pose, xgs_stream_t stream);

/* Tracking loss (Eq. (loss_track), L_photo read as L1):
 *   loss = (1/(3 P)) sum_x sum_{c<3} |out_c(x) - image_c(x)|
 *        + lambda_d (1/P_D) sum_{x: depth(x) > 0} |out_3(x) - depth(x)|,
 * P = Hs Ws, P_D = #pixels with depth > 0 (no depth term if P_D = 0 or
 * depth == NULL).  out [C][Hs][Ws] (C >= 4: RGB, depth, semantic), image
 * [3][Hs][Ws], depth [Hs][Ws].  Writes *loss (device float) and d_out
 * [C][Hs][Ws] = dL/dout (zero on channels >= 4).  Deterministic.  ws:
 * xgs_tracking_loss_workspace(Hs, Ws) bytes, 256-byte aligned. */
size_t xgs_tracking_loss_workspace(int32_t Hs, int32_t Ws);
xgs_status xgs_tracking_loss(const float* out, int32_t C, int32_t Hs, int32_t Ws, const float* image,
                             const float* depth, float lambda_d, float* d_out, float* loss, void* ws,
                             size_t ws_bytes, xgs_stream_t stream);

/* ------------------------------------------- f1: semantic phase (Sec. 3.2.2, App. D, App. E)
 * Mixture weights w_i = softmax(z_i) over L codewords (Sec. 3.2.2); z, w,
 * dL/dw, dL/dz are [N][L] row-major FP32, 16-byte aligned; L in
 * {4, 8, 16, 32, 64}.  xgs_semantic_softmax_bwd: dL/dz = w (dL/dw - <dL/dw, w>). */
xgs_status xgs_semantic_softmax(const float* z, int64_t N, int32_t L, float* w, xgs_stream_t stream);
xgs_status xgs_semantic_softmax_bwd(const float* w, const float* dw, int64_t N, int32_t L, float* dz,
                                    xgs_stream_t stream);

/* Decode and masked grid loss (App. D Eq. (loss), App. E F(x) = E^T w(x)):
 * wmap [4+L][Hs][Ws] is xgs_render_fwd's output with the mixture weights as
 * the semantic channels (channels 0..3 are not read); E [L][D] codebook
 * (D % 4 == 0, 16-byte aligned);
 * Gstar [D][Hs][Ws] targets; V [Hs][Ws] validity (NULL: all valid).
 *   loss = lambda [ (1/n) sum_valid (1 - cos(G^, G*)) + (1/(n D)) sum_valid |G^ - G*|_1 ],
 *   G^(x) = E^T w(x), cos(a, b) = <a, b> / max(|a| |b|, 1e-8), n = #valid
 *   (n = 0: loss 0, zero gradient).
 * Writes *loss (device float) and d_out [4+L][Hs][Ws] = dL/dwmap with the
 * colour and depth channels zero, ready for xgs_render_bwd with
 * XGS_BWD_FEATURES_ONLY.  Deterministic (fixed reduction order).  ws:
 * xgs_semantic_loss_workspace(Hs, Ws) bytes, 256-byte aligned. */
size_t xgs_semantic_loss_workspace(int32_t Hs, int32_t Ws);
xgs_status xgs_semantic_loss(const float* wmap, int32_t L, int32_t Hs, int32_t Ws, const float* E, int32_t D,
                             const float* Gstar, const uint8_t* V, float lambda, float* d_out, float* loss,
                             void* ws, size_t ws_bytes, xgs_stream_t stream);

/* ------------------------------------------------- f4: region targets, occluders
 * App. D, Eq. (target_discrete): for the grid pixel (m, n) at image pixel
 * (u, v) = (off_y + m s, off_x + n s): V = [0 <= S(u, v) < R] (labels outside
 * [0, R), including -1 = background, count as unannotated) and
 * G[:, m, n] = Phi[S(u, v)], else 0; V = 0 and G = 0 where u >= H or v >= W.
 * S [H][W] int32 (full image), Phi [R][D], G [D][H_s][W_s], V [H_s][W_s]
 * (may be NULL), H_s = ceil(H / s), W_s = ceil(W / s). */
xgs_status xgs_region_targets(const int32_t* S, int32_t H, int32_t W, const float* Phi, int32_t R, int32_t D,
                              int32_t stride, int32_t off_y, int32_t off_x, float* G, uint8_t* V,
                              xgs_stream_t stream);

/* Occluder pruning (Sec. 3.2.1, mapping; relative margin 10% in Sec. 4.1):
 * prune[i] = 1 when Gaussian i is visible (radius > 0), its projected mean
 * lies inside the H x W image, the depth map is positive at the pixel
 * floor(mean2d), and its camera depth is below (1 - margin) times that depth.
 * p: xgs_project's output for the n Gaussians; depth_map [H][W] FP32 (full
 * image); prune [n] u8; *count (device u64) = number pruned.  margin in
 * [0, 1). */
xgs_status xgs_occluder_mask(const xgs_projected* p, int64_t n, const float* depth_map, int32_t H, int32_t W,
                             float margin, uint8_t* prune, uint64_t* count, xgs_stream_t stream);

/* ------------------------------------------------------ a6: VQ assignment
 * a_n = argmin_l ||x_n - E_l||^2 (Sec. 3.2.2), ties to the lowest l.
 * XGS_VQ_FP32: direct FP32 sum of (x - e)^2 over every codeword.
 * XGS_VQ_BF16_RESCORE4: the squared distances of the bf16 roundings x^, e^
 * are formed on MFMA (FP32 accumulation, the norms folded into the product)
 * and each row keeps its 4 best codewords, ranked by half that distance with
 * its lowest b mantissa bits (6 <= b <= 10, set by K) replaced by the
 * codeword's position in its sweep (ties to the lower index); the 4 are rescored
 * with the direct FP32 form and the smallest wins.  E_bf16 [K][D] and
 * e_norm2 [K] must hold xgs_vq_prepare's output for E (xgs_vq_ema_update
 * refreshes them).  BF16 requires D % 8 == 0, K <= 65536, X and E_bf16
 * 16-byte aligned, and ws (256-byte aligned) of xgs_vq_assign_workspace
 * bytes (about N (D + 64) 2 bytes; zero for FP32).  idx [N] int32, dist [N] =
 * FP32 squared distance of the chosen codeword. */
size_t xgs_vq_assign_workspace(int64_t N, int32_t D, int32_t K, int32_t precision);
xgs_status xgs_vq_prepare(const float* E, int32_t K, int32_t D, uint16_t* E_bf16, float* e_norm2,
                          xgs_stream_t stream);
xgs_status xgs_vq_assign(const float* X, int64_t N, int32_t D, const float* E,
                         const uint16_t* E_bf16, const float* e_norm2, int32_t K,
                         int32_t precision, int32_t* idx, float* dist, void* ws, size_t ws_bytes,
                         xgs_stream_t stream);

/* The three stages of the XGS_VQ_BF16_RESCORE4 form, for callers that time
 * or overlap them; xgs_vq_assign runs them in this order on one stream.  All
 * share ws (xgs_vq_assign_workspace bytes, 256-byte aligned, same N, D, K).
 * xgs_vq_stage: writes the bf16 operands of X and of the codebook (E_bf16,
 * e_norm2 as above) into ws.  xgs_vq_candidates: the MFMA distance sweep;
 * writes each row's 4 best codewords into ws.  xgs_vq_rescore: FP32 direct
 * distances of those candidates; writes idx [N] and dist [N]. */
xgs_status xgs_vq_stage(const float* X, int64_t N, int32_t D, const uint16_t* E_bf16,
                        const float* e_norm2, int32_t K, void* ws, size_t ws_bytes, xgs_stream_t stream);
xgs_status xgs_vq_candidates(int64_t N, int32_t D, int32_t K, void* ws, size_t ws_bytes,
                             xgs_stream_t stream);
xgs_status xgs_vq_rescore(const float* X, int64_t N, int32_t D, const float* E, int32_t K,
                          int32_t* idx, float* dist, void* ws, size_t ws_bytes, xgs_stream_t stream);

/* App. C, Eq. (confidence_score): the BF16 form of xgs_vq_assign that also
 * returns conf [N] = max_k p_nk, p_nk = softmax_k(-|x_n - e_k| / tau), from
 * the unsquared distances of the bf16 operands (one log-sum-exp over every
 * codeword, fused in the MFMA sweep; the assignment itself is unchanged).
 * Same arguments and workspace as xgs_vq_assign with precision BF16. */
xgs_status xgs_vq_assign_conf(const float* X, int64_t N, int32_t D, const float* E,
                              const uint16_t* E_bf16, const float* e_norm2, int32_t K, float tau,
                              int32_t* idx, float* dist, float* conf, void* ws, size_t ws_bytes,
                              xgs_stream_t stream);

/* --------------------------------------------------------- a7: EMA update
 * Eq. (ema_update): c_l = #{a_n = l}, s_l = sum_{a_n = l} x_n,
 * N <- decay N + (1-decay) c, M <- decay M + (1-decay) s, then
 * PAPER: E_l = M_l / (N_l + eps); LAPLACE: E_l = M_l / Ntilde_l with
 * Ntilde_l = (N_l + eps) / (n + K eps) * n, n = sum_l N_l.  Sums are formed
 * in a fixed order (rows sorted stably by code), so the result is bitwise
 * reproducible.  Refreshes E_bf16 and e_norm2.  counts [K] (may be NULL)
 * receives c.  ws: xgs_vq_ema_workspace bytes. */
size_t xgs_vq_ema_workspace(int64_t N, int32_t D, int32_t K);
xgs_status xgs_vq_ema_update(const float* X, const int32_t* idx, int64_t N, int32_t D, int32_t K,
                             float* N_ema, float* M_ema, float* E, uint16_t* E_bf16,
                             float* e_norm2, float* counts, float decay, float eps, int32_t mode,
                             void* ws, size_t ws_bytes, xgs_stream_t stream);

/* App. C: the EMA step of xgs_vq_ema_update with the confidence mask
 * (Eq. (mask_confidence): only rows with conf[n] >= gamma update c and s;
 * conf == NULL keeps every row) and the dead-code reset (Eq. (dead_code)):
 * after the decay step every codeword with N_k < delta takes M_k <- reservoir
 * row (offset + j) mod R for the j-th such codeword in index order and
 * N_k <- 1 + eps (delta <= 0: no reset); E, E_bf16, e_norm2 are then
 * recomputed from N and M.  reservoir [R][D] FP32 (recent features);
 * *n_dead (device int32, may be NULL) = number reset.  A warm start is this
 * call with decay 0.  ws: xgs_vq_ema_workspace(N, D, K) bytes. */
xgs_status xgs_vq_ema_update_robust(const float* X, const int32_t* idx, const float* conf, float gamma,
                                    int64_t N, int32_t D, int32_t K, float* N_ema, float* M_ema, float* E,
                                    uint16_t* E_bf16, float* e_norm2, float* counts, float decay, float eps,
                                    int32_t mode, float delta, const float* reservoir, int32_t R,
                                    int64_t offset, int32_t* n_dead, void* ws, size_t ws_bytes,
                                    xgs_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* XGS_H */
