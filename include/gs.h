/*
 * gs.h -- C ABI of the MI355X (gfx950) differentiable Gaussian-splatting hot
 * path of TAMBRIDGE (arXiv 2405.19614): the 3DGS-centred encoder and the
 * online mapping step, batched over the selected keyframes.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array argument is a DEVICE pointer owned by the caller, unless it is
 *   marked "host".  The library owns only its context (a few pinned bytes for
 *   read-backs, the reprojection accumulators and the captured-graph cache).
 * - All work is enqueued on `stream` (a hipStream_t passed as void*; NULL is
 *   the null stream).  Calls return once the work is enqueued, except where a
 *   read-back is stated.
 * - Every call returns an int status (gs_status).  Nothing aborts and no C++
 *   exception crosses the boundary; on failure gs_last_error() describes it.
 * - Gaussian parameters are FP32 structure-of-arrays (see gs_gaussians).
 * - Images of several views are concatenated: view v occupies pixels
 *   [P_v, P_v + H_v W_v) of the depth / alpha buffers and
 *   [3 P_v, 3 P_v + 3 H_v W_v) of the colour buffer, with P_v = sum over u < v
 *   of H_u W_u; each view's colour block is planar [3][H_v][W_v], row-major.
 * - Poses are world-to-camera rigid transforms T_cw, FP32 4x4 row-major,
 *   [V][16] on the device.  A pose gradient is the 6-vector d/dxi at xi = 0
 *   of the left perturbation T_cw <- Exp(xi) T_cw, xi = (v, w) (translation
 *   first, then rotation).
 * - Camera model: pinhole (fx, fy, cx, cy); an integer pixel (x, y) samples
 *   the image point (x, y) itself (OpenCV convention).
 * - The forward model (Sec. 3.4 "Projection", "Differentiable Rasterization",
 *   colour and depth compositing equations; Sec. 3.3 border mask): each
 *   Gaussian is projected by its local affine (EWA) Jacobian, with 0.3 px^2
 *   added to the 2D covariance diagonal; Gaussians with camera-space depth
 *   <= 0.2 are culled; at each pixel the Gaussians whose opacity-aware
 *   support rect contains it are blended front to back in ascending
 *   (depth, index) order with alpha = min(0.99, o exp(-sigma)), fragments with
 *   alpha < 1/255 skipped, and blending stops before the transmittance would
 *   fall below 1e-4.  Outputs: colour C, depth D (not divided by alpha) and
 *   alpha A = 1 - T_final (the border mask M_b).  Background is zero.
 * - Results of the forward pass do not depend on the tile shape.
 */
#ifndef GS_H_
#define GS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_ABI_VERSION 4
#define GS_MAX_VIEWS 64

typedef enum {
    GS_OK = 0,
    GS_EINVAL = -1,     /* bad argument: NULL pointer, size out of range, unsupported shape */
    GS_ENOMEM = -2,     /* a buffer the caller passed is too small, or a library allocation failed */
    GS_ECAPACITY = -3,  /* more (tile, Gaussian) pairs than the pair capacity; see gs_plan.n_pairs */
    GS_EDEVICE = -4,    /* HIP runtime error; text in gs_last_error */
    GS_ECAPTURE = -5    /* graph capture / instantiation failed */
} gs_status;

typedef struct gs_ctx gs_ctx;

/* Gaussian parameters (Sec. 3.4 "Gaussian Representation", Eq. gauss, and
 * its generalisation to an anisotropic covariance).  n Gaussians, FP32, device.
 *   isotropic      0: anisotropic layout; 1: the paper's eight-parameter
 *                  Gaussian f(x) = o exp(-|x - mu|^2 / (2 r^2)) (RGB colours
 *                  give 8 floats per Gaussian; 14 anisotropic)
 *   means          [n][3]  world-space centres
 *   log_scales     anisotropic: [n][3] scale = exp(log_scale) per principal
 *                  axis; isotropic: [n] log radius, r = exp(log_radius)
 *   quats          anisotropic: [n][4] rotation (w, x, y, z), normalised
 *                  inside the forward, 16-byte aligned; isotropic: unused
 *                  (may be NULL)
 *   opacity_logits [n]     opacity = sigmoid(logit)
 *   colors         sh_degree == -1: [n][3] RGB (view independent, as in the paper)
 *                  sh_degree in 0..3: [n][(L+1)^2][3] real orthonormal SH
 *                  coefficients; colour = max(0, sum Y_lm(dir) k_lm + 0.5)
 *                  with dir the unit vector from the camera centre to the mean;
 *                  16-byte aligned for sh_degree 1 and 3 (GS_EINVAL otherwise). */
typedef struct {
    int64_t n;
    int32_t sh_degree;
    int32_t isotropic;
    float* means;
    float* log_scales;
    float* quats;
    float* opacity_logits;
    float* colors;
} gs_gaussians;

/* Gradients with the layout of gs_gaussians (device, FP32; quats unused and
 * may be NULL for an isotropic set; colors 16-byte aligned for sh_degree 1
 * and 3, as the parameters').  Overwritten by gs_render_backward;
 * gs_mapping_step overwrites or accumulates (opts). */
typedef struct {
    float* means;
    float* log_scales;
    float* quats;
    float* opacity_logits;
    float* colors;
} gs_gaussian_grads;

/* Static camera geometry of one view (HOST memory). */
typedef struct {
    int32_t width, height;  /* 1 .. 16384 */
    float fx, fy, cx, cy;
} gs_camera;

/* Tile plan of a forward pass.
 *   tile_w, tile_h : in  compositing tile of the forward; one of 16x16, 16x8,
 *                    8x8, 32x8, 32x16, 32x32, 32x64, 64x32, 64x64 (0, 0 = the
 *                    context's current choice, 16x16 unless gs_autotune
 *                    chose another); out: used
 *   bin_w, bin_h   : in  binning rectangle, multiples of both tiles in
 *                    [8, 2048] (0, 0 = the context's choice, 64x64 by
 *                    default); out: used.  Gaussians are binned per bin; each
 *                    tile composites the entries of its bin's list whose
 *                    support rect meets it.
 *   pair_capacity  : in  (bin, Gaussian) pairs the state buffer was sized for
 *   n_pairs        : out pairs produced (on GS_ECAPACITY: pairs needed)
 *   n_visible      : out visible (view, Gaussian) records
 *   bwd_tile_w, bwd_tile_h : in  compositing tile of the backward (same shapes;
 *                    0, 0 = the context's backward choice, else the forward
 *                    tile); out: the shape gs_render_backward will use.  The
 *                    shapes change only the launch, never a result. */
typedef struct {
    int32_t tile_w, tile_h;
    int32_t bin_w, bin_h;
    int64_t pair_capacity;
    int64_t n_pairs;
    int64_t n_visible;
    int32_t bwd_tile_w, bwd_tile_h;
} gs_plan;

int gs_abi_version(void);

/* Create a context on HIP device `device`.  *out receives the handle. */
int gs_create(gs_ctx** out, int device);
void gs_destroy(gs_ctx* ctx);

/* Text of the last failure on this context (ctx may be NULL: last failure of
 * gs_create on this thread).  Valid until the next call on the context. */
const char* gs_last_error(const gs_ctx* ctx);

/* Bytes of the opaque device state a forward pass writes and the matching
 * backward reads: records of every (view, Gaussian), sort buffers for
 * `pair_capacity` pairs, per-bin ranges and per-pixel final transmittance
 * and stop index, for bins of bin_w x bin_h (0, 0 = 64x64).  cams: HOST [V].
 * Returns 0 on invalid arguments. */
size_t gs_state_bytes(const gs_camera* cams, int32_t V, int64_t n, int64_t pair_capacity, int32_t bin_w,
                      int32_t bin_h);

/* Forward pass (Sec. 3.3 3DGS-centred encoder; Sec. 3.4 projection and
 * rasterisation) over V views in one batched launch sequence.
 *   g      Gaussians (device)          cams  HOST [V] camera geometry
 *   poses  device [V][16] T_cw         V     1 .. GS_MAX_VIEWS
 *   color  device [sum 3 H W]          depth, alpha  device [sum H W]
 *   state  device buffer of state_bytes >= gs_state_bytes(...), 256-byte
 *          aligned (as hipMalloc returns; GS_EINVAL otherwise); written
 *   plan   HOST in/out (see gs_plan)
 * Reads the pair count back once (one stream synchronisation) and returns
 * GS_ECAPACITY with plan->n_pairs = pairs needed when the capacity is too
 * small, or GS_EINVAL when a mean, log-scale, quaternion or opacity logit (or
 * the colour of a visible Gaussian) is not finite; nothing after the count is
 * then enqueued. */
int gs_render_forward(gs_ctx* ctx, const gs_gaussians* g, const gs_camera* cams, const float* poses, int32_t V,
                      float* color, float* depth, float* alpha, void* state, size_t state_bytes, gs_plan* plan,
                      void* stream);

/* gs_render_forward without any host synchronisation (the same kernels; for
 * graph capture and for loops that must not stall on the device).  The pair
 * total stays on the device: plan->pair_capacity is the caller's bound, and
 * plan->n_pairs and plan->n_visible are set to -1.  When the pairs exceed
 * the capacity every per-bin list is left empty, so color, depth and alpha
 * are 0 and a gs_render_backward of this state gives zero gradients; a
 * non-finite parameter makes the results invalid.  Both are flagged in the
 * state's status block: gs_step_status(ctx, state, ...) returns the flags
 * (bit 0 overflow, bit 1 scan time-out, bit 2 non-finite parameter) and the
 * pair and visible-record counts.  Errors returned are those of the
 * arguments only. */
int gs_render_forward_async(gs_ctx* ctx, const gs_gaussians* g, const gs_camera* cams, const float* poses,
                            int32_t V, float* color, float* depth, float* alpha, void* state, size_t state_bytes,
                            gs_plan* plan, void* stream);

/* Reverse mode of gs_render_forward (differentiable rasterisation,
 * Sec. 3.4; pose gradient for the joint optimisation, Sec. 3.3).  Takes the
 * same g, cams, poses, V, state and the plan returned by the forward, and the
 * upstream gradients dL/dcolor [sum 3HW], dL/ddepth [sum HW], dL/dalpha
 * [sum HW] (device; any may be NULL = zero).  Overwrites every array of
 * `grads` (device) and dL_dpose (device [V][6]).  The state is used as
 * scratch and stays valid for further backward calls. */
int gs_render_backward(gs_ctx* ctx, const gs_gaussians* g, const gs_camera* cams, const float* poses, int32_t V,
                       void* state, size_t state_bytes, const gs_plan* plan, const float* dL_dcolor,
                       const float* dL_ddepth, const float* dL_dalpha, gs_gaussian_grads* grads, float* dL_dpose,
                       void* stream);

/* Re-projection residuals of Sec. 3.2 Eq. lba (the tracking-centred encoder
 * of Sec. 3.3): for match m of view k = view_idx[m], r_m = uv_m - pi(K_k,
 * T_k P_m).  Robust loss per view: mean over its matches with camera-space
 * depth > 0.2 of h(|r_m|), h(e) = e^2/2 for e <= huber_delta, else
 * huber_delta (e - huber_delta/2).
 *   points device [M][3], uv device [M][2], view_idx device [M] (int32,
 *   matches with an index outside [0, V) are ignored), M >= 0.
 *   residual device [M][2] (0 for excluded matches), loss device [V]
 *   (overwritten), dL_dpose device [V][6]: ACCUMULATES weight * d loss_k /
 *   d xi_k, so it can be added to the rendering pose gradient.
 *   dL_dpoints device [M][3] or NULL: OVERWRITTEN with d/dP_m of
 *   weight * sum_k loss_k (the point side of the full bundle adjustment of
 *   Sec. 3.2 Eq. for:ba; 0 for excluded matches). */
int gs_reproj_residual(gs_ctx* ctx, const gs_camera* cams, const float* poses, int32_t V, const float* points,
                       const float* uv, const int32_t* view_idx, int64_t M, float huber_delta, float weight,
                       float* residual, float* loss, float* dL_dpose, float* dL_dpoints, void* stream);

/* Allocation-free variant of gs_reproj_residual, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results and error
 * behaviour as gs_reproj_residual; the per-view accumulators live in a static
 * device array of the library (GS_MAX_VIEWS x 8 doubles = 4 KiB per GPU,
 * located once per device by gs_create and held until the process ends)
 * instead of the context's buffer, and the call makes no allocation.
 * V above GS_MAX_VIEWS is rejected (GS_EINVAL).  Every call on one GPU shares
 * that GPU's array, which keeps the last call's sums (each call clears what it
 * uses first): calls that overlap on one GPU (several streams or contexts)
 * race and must be serialised by the caller. */
int gs_reproj_residual_noalloc(gs_ctx* ctx, const gs_camera* cams, const float* poses, int32_t V,
                               const float* points, const float* uv, const int32_t* view_idx, int64_t M,
                               float huber_delta, float weight, float* residual, float* loss, float* dL_dpose,
                               float* dL_dpoints, void* stream);

/* Options of one mapping / pose-refinement step.
 * Loss (Sec. 3.3 joint-loss equation; Sec. 3.4 mapping-loss equation):
 *   L = (1/V) sum_v ( w_color Lc_v + w_depth Ld_v + w_reproj Lr_v + w_ssim Ls_v ),
 *   Lc_v = sum_{p,k} m_p |C - C^| / (3 H_v W_v),  Ld_v = sum_p m_p |D - D^| / (H_v W_v),
 *   Lr_v = the Huber re-projection loss of gs_reproj_residual,
 *   Ls_v = 1 - the mean SSIM of the view's colour render against the target
 *   colour (see gs_ssim; the mask does not apply to it; skipped when
 *   w_ssim = 0).  The paper's mapping loss (1 - zeta)(w4 L1_D + w5 L1_C) +
 *   zeta L_SSIM is w_color = (1 - zeta) w5, w_depth = (1 - zeta) w4, w_ssim = zeta.
 *   m_p = target mask (1 if NULL) times, if use_gate, the filter gate of
 *   Sec. 3.3: target depth > 0, rendered depth > 0, rendered alpha > gate_gamma
 *   (a constant mask, no gradient through it).  sign(0) = 0.
 * Update (the paper's "gradient-based optimization"; Adam with bias
 * correction): update_gaussians applies Adam to every Gaussian parameter
 * with its group's learning rate; update_poses applies Adam to each view's
 * pose tangent and sets T <- Exp(step) T.
 * accumulate_grads: add the Gaussian gradients to `grads` instead of
 * overwriting them.  use_graph: capture the step as a hipGraph on first use
 * of a given (shape, pointers, options) and replay it afterwards. */
typedef struct {
    float w_color, w_depth, w_reproj, huber_delta;
    int32_t use_gate;
    float gate_gamma;
    int32_t update_gaussians, update_poses, accumulate_grads, use_graph;
    float lr_means, lr_log_scales, lr_quats, lr_opacity, lr_colors, lr_pose;
    float adam_b1, adam_b2, adam_eps;
    int32_t tile_w, tile_h;     /* 0, 0 = context choice */
    int32_t bin_w, bin_h;       /* 0, 0 = context choice */
    int64_t pair_capacity;      /* capacity the workspace was sized for */
    float w_ssim;               /* weight of the SSIM term, >= 0 */
    int32_t bwd_tile_w, bwd_tile_h;  /* backward tile; 0, 0 = context choice, else the forward tile */
} gs_step_opts;

/* Targets of the rendering loss (device): color [sum 3HW], depth [sum HW],
 * mask [sum HW] or NULL (per-pixel weight m_p). */
typedef struct {
    const float* color;
    const float* depth;
    const float* mask;
} gs_targets;

/* 2D-3D matches for the re-projection term (device; M may be 0). */
typedef struct {
    const float* points;
    const float* uv;
    const int32_t* view_idx;
    int64_t M;
} gs_matches;

/* Adam state (device): m and v each hold n*(11 + 3K) + 6V floats laid out as
 * means [3n], log_scales [3n], quats [4n], opacity [n], colors [3Kn] (K = 1 for
 * RGB, (L+1)^2 for SH), poses [6V]; isotropic: n*(5 + 3K) + 6V floats, means
 * [3n], log radii [n], opacity [n], colors [3Kn], poses [6V].  step is a
 * device int32[2]: the Gaussian updates done and the pose updates done
 * (incremented on the device).  Each group's bias correction uses its own
 * count, as two optimisers would. */
typedef struct {
    float* m;
    float* v;
    int32_t* step;
} gs_adam;

/* Workspace bytes for gs_mapping_step (device; holds the forward state, the
 * upstream gradients, loss partials and status flags), for bins of
 * bin_w x bin_h (0, 0 = 64x64) and any tile shape.  The workspace must be
 * 256-byte aligned (as hipMalloc returns; GS_EINVAL otherwise). */
size_t gs_step_workspace_bytes(const gs_camera* cams, int32_t V, int64_t n, int32_t sh_degree,
                               int64_t pair_capacity, int32_t bin_w, int32_t bin_h);

/* One mapping / joint-optimisation iteration, entirely on the device with no
 * host synchronisation: forward over V views, fused loss and upstream
 * gradients, re-projection term, backward, optional Adam updates.
 *   params   in (out when update_gaussians)    grads  out (see accumulate_grads)
 *   adam     Adam state (used when an update flag is set; may be NULL otherwise)
 *   cams     HOST [V]                           poses  device [V][16] (out when update_poses)
 *   color, depth, alpha  device render outputs (sum 3HW / sum HW)
 *   loss_out device [1 + 4V]: total L, then (Lc_v, Ld_v, Lr_v, Ls_v) per view
 *   dL_dpose device [V][6]: gradient of L w.r.t. each pose tangent
 * A pair overflow or a non-finite parameter is flagged on the device: the
 * step's results are then invalid and it skips every update (see
 * gs_step_status, which reads the flags). */
int gs_mapping_step(gs_ctx* ctx, gs_gaussians* params, gs_gaussian_grads* grads, const gs_adam* adam,
                    const gs_camera* cams, float* poses, int32_t V, const gs_targets* targets,
                    const gs_matches* matches, const gs_step_opts* opts, void* workspace, size_t workspace_bytes,
                    float* color, float* depth, float* alpha, float* loss_out, float* dL_dpose, void* stream);

/* The optimiser update of gs_mapping_step on its own (Adam with bias
 * correction; the paper's "gradient-based optimization", Sec. 3.4), for
 * gradients the caller computed (e.g. through gs_render_backward):
 * opts->update_gaussians applies Adam to every Gaussian parameter with its
 * group's learning rate (grads device, layout of g); opts->update_poses
 * applies Adam to each view's pose tangent gradient dL_dpose (device [V][6])
 * and sets poses[v] <- Exp(step) poses[v] (device [V][16]).  Uses lr_*,
 * adam_b1, adam_b2, adam_eps of opts and nothing else; the matching
 * counters of adam->step advance by one.  Asynchronous on `stream`. */
int gs_adam_update(gs_ctx* ctx, gs_gaussians* g, const gs_gaussian_grads* grads, const gs_adam* adam, float* poses,
                   const float* dL_dpose, int32_t V, const gs_step_opts* opts, void* stream);

/* Pose retraction for the pose refinement of the joint optimisation
 * (Sec. 3.3): poses_out[v] = Exp(xi[v]) poses[v], with xi = (v, w) the
 * left-perturbation twist (translation first) and Exp the SE(3)
 * exponential.  poses, poses_out device [V][16] (may alias), xi device
 * [V][6].  Asynchronous on `stream`. */
int gs_pose_retract(gs_ctx* ctx, int32_t V, const float* poses, const float* xi, float* poses_out, void* stream);

/* Chain rule through the retraction: given dL_dpose, the left-perturbation
 * gradient at the retracted pose Exp(xi) T (as gs_render_backward returns
 * it), dL_dxi = J_l(xi)^T dL_dpose is the gradient with respect to xi itself
 * (J_l the left Jacobian of SE(3); the identity at xi = 0).  Device [V][6]
 * each.  Asynchronous on `stream`. */
int gs_pose_tangent_grad(gs_ctx* ctx, int32_t V, const float* xi, const float* dL_dpose, float* dL_dxi,
                         void* stream);

/* Synchronous read of the workspace status after gs_mapping_step (or of a
 * forward state after gs_render_forward_async).  *flags is
 * the OR over every step since the previous gs_step_status call on this
 * workspace (the sticky word, which this call then clears) and the last
 * step: bit 0 = pair overflow, bit 1 = a binning scan gave up waiting for
 * another workgroup, bit 2 = a Gaussian parameter the step read was not
 * finite (a mean, log-scale, quaternion or opacity logit of any Gaussian, or
 * the colour of one some view sees).  A step with any bit set has invalid
 * results and makes no update: parameters, poses, Adam moments and the step
 * counter keep their values.  *n_pairs = pairs of the last step (needed ones
 * on overflow), *n_visible = its visible records.  The sticky word of a new
 * workspace must start at zero: zero the first 64 bytes, or call
 * gs_step_status once, before the first step.  Synchronises `stream`. */
int gs_step_status(gs_ctx* ctx, const void* workspace, size_t workspace_bytes, int32_t* flags, int64_t* n_pairs,
                   int64_t* n_visible, void* stream);

/* Diagnostics: one eager mapping step (same arguments and results as
 * gs_mapping_step, never graph-captured) with HIP events recorded on `stream`
 * between its stages.  stage_ms (HOST [gs_num_stages()]) receives each
 * stage's duration in milliseconds; frag_counts (HOST [4], may be NULL)
 * receives the number of (pixel, Gaussian) candidates the forward
 * compositing visited (support rect contains the pixel, up to and including
 * the one that stops the pixel), the number it blended, the list entries
 * the tiles staged before every pixel had stopped, and the total list
 * length.  Synchronises `stream`. */
int gs_num_stages(void);
const char* gs_stage_name(int i);
int gs_step_profile(gs_ctx* ctx, gs_gaussians* params, gs_gaussian_grads* grads, const gs_adam* adam,
                    const gs_camera* cams, float* poses, int32_t V, const gs_targets* targets,
                    const gs_matches* matches, const gs_step_opts* opts, void* workspace, size_t workspace_bytes,
                    float* color, float* depth, float* alpha, float* loss_out, float* dL_dpose, float* stage_ms,
                    int64_t* frag_counts, void* stream);

/* Binning stage on its own (integer; exact): records r = v*n + i carry an
 * inclusive pixel rect rect[r] = (x0 | x1 << 16, y0 | y1 << 16) (empty when
 * x0 > x1 or y0 > y1) and a positive FP32 depth.  For bins of bin_w x bin_h
 * pixels (multiples of 8), produces the record ids of every (bin, record)
 * pair whose rect touches the bin, sorted by (global bin id, depth, record),
 * and per-bin [start, end) ranges ((0, 0) when empty); the global id of bin
 * (bx, by) of view v counts the bins of the views before v, then
 * by * bins_x + bx.
 *   rect device [V*n][2] u32, depth device [V*n] f32, values device
 *   [values_capacity] u32, ranges device [total tiles][2] u32, n_pairs HOST out.
 * Uses `state` (sized by gs_state_bytes with pair_capacity = values_capacity,
 * 256-byte aligned) as scratch; reads the pair count back (one
 * synchronisation). */
int gs_bin_records(gs_ctx* ctx, const gs_camera* cams, int32_t V, int64_t n, int32_t bin_w, int32_t bin_h,
                   const uint32_t* rect, const float* depth, uint32_t* values, int64_t values_capacity,
                   uint32_t* ranges, int64_t* n_pairs, void* state, size_t state_bytes, void* stream);

/* Launch-shape autotuner: times the forward and the backward of the given
 * scene for every supported (tile shape, pixels per thread) pair with 64x64
 * bins and keeps the fastest forward and the fastest backward shape
 * separately, then times every bin size that is a multiple of both, then
 * every shape again at the chosen bins (allocating temporary device
 * buffers).  A tile shape displaces an earlier one only when it is more
 * than 2 % faster, so near-ties resolve the same way from run to run.  Keeps the
 * result as the context's
 * choice for this (V, sizes, n) class and returns the forward tile, the bin
 * and the backward tile (HOST outputs).  Synchronises the device.  No result
 * depends on the choice. */
int gs_autotune(gs_ctx* ctx, const gs_gaussians* g, const gs_camera* cams, const float* poses, int32_t V,
                int32_t iters, int32_t* tile_w, int32_t* tile_h, int32_t* bin_w, int32_t* bin_h, int32_t* bwd_tile_w,
                int32_t* bwd_tile_h, void* stream);

/* Set the context's bin choice explicitly (0, 0 restores 64x64). */
int gs_set_bin(gs_ctx* ctx, int32_t bin_w, int32_t bin_h);

/* Set the context's tile choice explicitly (0, 0 restores 16x16). */
int gs_set_tile(gs_ctx* ctx, int32_t tile_w, int32_t tile_h);

/* Pixels each thread of the compositing kernels owns for a tile shape (1, 2,
 * 4 or 8: 1 and 2 for the shapes up to 32x16 (2 not for 8x8), 4 for 16x16 and
 * the 32-wide shapes, 8 for 32x16, 32x32 and the shapes 64 wide or tall, which
 * take only 8), for the forward and the backward.  Does not change any
 * result, only the launch shape; gs_autotune sets it too. */
int gs_set_pixels_per_thread(gs_ctx* ctx, int32_t tile_w, int32_t tile_h, int32_t ppt);

/* The backward's own tile shape and pixels per thread (0, 0, 0: use the
 * forward's).  Bins must be a multiple of both tiles; where a call's bins are
 * not, the forward tile is used.  Changes no result. */
int gs_set_bwd_shape(gs_ctx* ctx, int32_t tile_w, int32_t tile_h, int32_t ppt);

/* Pixels per thread the compositing kernels use for a tile shape, pass 0 =
 * forward, 1 = backward (the value set by gs_set_pixels_per_thread,
 * gs_set_bwd_shape or gs_autotune, else the default: 2 where a 2-pixel kernel
 * exists, else 1, else 4).  Returns GS_EINVAL for a null context, a bad pass
 * or a tile shape without kernels. */
int gs_get_pixels_per_thread(const gs_ctx* ctx, int32_t pass, int32_t tile_w, int32_t tile_h);

/* SSIM of Sec. 3.4's mapping loss, standalone.  The paper names the term
 * without defining it; this is the usual structural similarity, per colour
 * channel, with an 11 x 11 Gaussian window (standard deviation 1.5 px, taps
 * normalised to sum 1), C1 = 0.01^2, C2 = 0.03^2, and windows clipped at the
 * image border by zero padding (the window mean at a pixel is the weighted sum
 * over the in-image pixels of its window):
 *   s = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)).
 *   img, ref  device planar colour images concatenated over the V views
 *             ([3][H_v][W_v] each, float, values nominally in [0, 1]); x = img.
 *   ssim_out  device [V]: mean of s over each view's pixels and channels.
 *   weights   device [V] or NULL; if not NULL, dL_dimg (device, same layout
 *             as img) ACCUMULATES d/d img of L = sum_v weights[v] (1 - SSIM_v).
 *   workspace device scratch of gs_ssim_workspace_bytes(cams, V) bytes.
 * Returns GS_EINVAL for NULL pointers or bad cameras, GS_ENOMEM for a short
 * workspace; asynchronous on `stream`. */
size_t gs_ssim_workspace_bytes(const gs_camera* cams, int32_t V);
int gs_ssim(gs_ctx* ctx, const gs_camera* cams, int32_t V, const float* img, const float* ref, const float* weights,
            float* ssim_out, float* dL_dimg, void* workspace, size_t workspace_bytes, void* stream);

/* Viewpoint selection of the Fusion Bridge (Sec. 3.3 selection equation), a
 * host-side rule over F keyframes in time order: keyframe 0 is selected;
 * keyframe i > 0 is selected when beta <= M < alpha * T, where M =
 * covis[p * F + i] is the number of feature matches between i and the last
 * selected keyframe p, and T = n_obs[p] is the number of map points the
 * keyframe p observes through its matches (the paper's T, counted for the
 * previously selected keyframe).
 *   covis HOST int32 [F][F], n_obs HOST int32 [F], selected HOST int32 [F]
 *   (out, 1 = selected).  The paper uses alpha = 0.75, beta = 20.
 * Returns GS_EINVAL for F < 0, NULL pointers (F > 0) or a negative or
 * non-finite alpha; needs no context and no device. */
int gs_select_viewpoints(const int32_t* covis, const int32_t* n_obs, int32_t F, float alpha, int32_t beta,
                         int32_t* selected);

/* Map maintenance of the online reconstruction (Sec. 3.4).
 *
 * Pruning (Sec. 3.4 pruning equation; its printed cases and the text
 * disagree on which side is removed, the text is followed): a Gaussian is
 * removed when its opacity sigmoid(opacity_logit) < tau, the others keep their
 * order.  tau <= 0 keeps every Gaussian, tau >= 1 removes every one.  tau is a
 * double and the decision is exact: the FP32 logit is compared with
 * logit(tau) in FP64.
 *   in        device arrays of in->n Gaussians (sh_degree, isotropic as in gs_gaussians).
 *   out       device arrays of in's layout with room for in->n Gaussians, not
 *             overlapping in; out->n, out->sh_degree, out->isotropic are ignored.
 *   adam_in / adam_out  optional (both NULL or both given, not overlapping):
 *             Adam moments laid out for in->n Gaussians and V poses (see
 *             gs_adam) are re-laid out for the kept ones; the step counter is
 *             copied when adam_out->step differs.
 *   n_out     device int64: the number kept.
 *   workspace device scratch of gs_prune_workspace_bytes(in->n) bytes.
 * Asynchronous on `stream`; GS_EINVAL for NULL pointers, GS_ENOMEM for a
 * short workspace. */
size_t gs_prune_workspace_bytes(int64_t n);
int gs_prune(gs_ctx* ctx, const gs_gaussians* in, double tau, gs_gaussians* out, const gs_adam* adam_in,
             gs_adam* adam_out, int32_t V, int64_t* n_out, void* workspace, size_t workspace_bytes, void* stream);

/* Densification (Sec. 3.4 densification, Eq. d): for every pixel of the V
 * views whose rendered alpha (the border mask M_b) is <= gamma (the FP32
 * alpha compared with the double gamma in FP64) -- every pixel
 * when all_pixels is set, as on the first frame -- and whose target depth d
 * is > 0, one Gaussian is appended after the g->n existing ones, in view then
 * row-major pixel order: mean = the pixel's sample point (x, y) back-projected
 * to depth d through the view's pose, log-scale log(d / fx) on every axis (a
 * one-pixel footprint; the log radius of an isotropic set), quaternion
 * (1, 0, 0, 0) (anisotropic), opacity logit 0, colour =
 * the target colour (with SH, the DC coefficient (rgb - 0.5) / Y_00 and the
 * other coefficients 0).
 *   cams HOST [V]; poses device [V][16] world-to-camera; alpha device [sum HW]
 *   (rendered); tgt_color device planar [3][H][W] per view; tgt_depth device [sum HW].
 *   g         device arrays holding g->n Gaussians with room for `capacity`;
 *             the new ones are written in place after them (none past capacity).
 *   adam_in / adam_out  optional (both NULL or both given, not overlapping):
 *             moments for g->n Gaussians re-laid out for the grown set (new
 *             Gaussians start at zero); adam_out must have room for capacity.
 *   counts    device int64[2]: Gaussians now held (<= capacity), Gaussians
 *             the selection asked for (g->n + selected pixels).
 *   workspace device scratch of gs_densify_workspace_bytes(cams, V) bytes.
 * Asynchronous on `stream`. */
size_t gs_densify_workspace_bytes(const gs_camera* cams, int32_t V);
int gs_densify(gs_ctx* ctx, const gs_camera* cams, const float* poses, int32_t V, const float* alpha,
               const float* tgt_color, const float* tgt_depth, double gamma, int32_t all_pixels, gs_gaussians* g,
               int64_t capacity, const gs_adam* adam_in, gs_adam* adam_out, int64_t* counts, void* workspace,
               size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_H_ */
