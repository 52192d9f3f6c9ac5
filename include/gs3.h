/*
 * gs3.h - C-ABI of the MI355X (gfx950) triple-splatting library libgs3.so.
 *
 * The library computes the relit render of GS^3 (Bi et al., "GS^3: Efficient
 * Relighting with Triple Gaussian Splatting", SIGGRAPH Asia 2024) for one
 * camera and one point light, and its adjoint:
 *
 *   gs3_project / gs3_bin / gs3_preprocess   Sec. 3 (Eq. 1-2): EWA projection
 *        of the spatial Gaussians into a view, tile binning, depth sort.
 *   gs3_shadow_splat   Sec. 4.2 and Fig. 3: splat toward the light, per-ray
 *        transmittance with the 0.015 shadow bias, beta-weighted average T.
 *   gs3_render         Sec. 4.1 (Eq. 4-7) shading, Sec. 4.2 (Eq. 8) shadow MLP
 *        Phi, Sec. 4.3 residual MLP Psi, and the camera splat of Sec. 4 /
 *        Fig. 2: final = shading * shadow + residual.
 *   gs3_render_backward  gradients of all of the above (Sec. 4, end-to-end
 *        differentiable training).
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status: GS3_OK (0) or a negative code.
 *    Nothing throws across the ABI and nothing aborts. gs3_status_string()
 *    names a code; gs3_last_error() returns a thread-local message for the
 *    last failure on the calling thread.
 *  - Pointers inside the structs and every array argument are DEVICE
 *    pointers (hipMalloc / torch CUDA tensors) unless stated otherwise.
 *    Inputs are const; the caller owns and allocates every buffer. The
 *    library allocates no device memory on any path.
 *  - All work is enqueued asynchronously on the caller's HIP stream
 *    (`stream`, NULL = the default stream); no call synchronises the host
 *    except gs3_view_pair_count (a workspace's status block, see
 *    gs3_viewbuf, reports the same without a synchronisation).
 *  - Per-Gaussian arrays are float32 structure-of-arrays with the Gaussian
 *    index fastest ([C][n]); images are planar float32 [C][H][W], row-major.
 *  - Calls that share a workspace must be ordered on one stream; distinct
 *    workspaces may be used concurrently.
 */
#ifndef GS3_H
#define GS3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* gs3_stream_t; /* == hipStream_t */

enum {
    GS3_OK = 0,
    GS3_INVALID_ARG = -1,          /* null pointer, bad size, misaligned buffer */
    GS3_WORKSPACE_TOO_SMALL = -2,  /* ws_bytes below gs3_view_workspace_size */
    GS3_PAIR_CAPACITY_EXCEEDED = -3, /* a binning needed more pairs than its capacity:
                                        reported by gs3_view_pair_count, and by the
                                        next call on a workspace with a status block */
    GS3_HIP_ERROR = -4,            /* a HIP runtime call or launch failed */
    GS3_UNSUPPORTED = -5           /* parameter combination not implemented */
};

/* Rasteriser constants. Sec. 4.2 fixes shadow_bias = 0.015; the others are
 * the conventions of vanilla Gaussian splatting the paper builds on (Sec. 3)
 * and are filled in by gs3_consts_default():
 *   near_plane 0.2     cull Gaussians with view-space z <= near_plane
 *   clamp_frac 1.3     x/z, y/z clamped to +-clamp_frac*tan(half fov) in the
 *                      EWA Jacobian only
 *   dilation   0.3     px^2 added to the diagonal of each 2D covariance
 *   cutoff     4.5     a pixel is hit only where power >= -cutoff
 *   alpha_min  1/255   ... and alpha >= alpha_min
 *   alpha_max  0.99    alpha = min(alpha_max, opacity * exp(power))
 *   t_min      1e-4    the camera pass stops before a hit that would take the
 *                      transmittance below t_min
 *   shadow_bias 0.015  Gaussian k shadows j only if dist_k < dist_j - bias
 * cutoff = +inf, alpha_min = 0, alpha_max = 1, t_min = 0, dilation = 0 and
 * shadow_bias = 0 give the threshold-free ("smooth") variant.
 * near_plane, clamp_frac, dilation, cutoff and alpha_min act at projection
 * (gs3_project / gs3_preprocess), which stores the resulting per-splat hit
 * threshold with the view; later calls on the view take it from there and
 * use only alpha_max, t_min and shadow_bias of their own `consts`. */
typedef struct {
    float near_plane;
    float clamp_frac;
    float dilation;
    float cutoff;
    float alpha_min;
    float alpha_max;
    float t_min;
    float shadow_bias;
} gs3_consts;

/* A view looking from `eye` at `target` (host values). Camera axes: x
 * right, y down, z forward; world up +z (+y when the view direction is
 * within acos(0.99) of +-z); square pixels, principal point (width/2,
 * height/2), pixel (i, j) centred at (i + 0.5, j + 0.5).
 *   GS3_PERSPECTIVE   pinhole, focal length (width/2)/tan(fov/2) pixels. A
 *                     point light is such a view whose eye is the light
 *                     (Sec. 4.2: a perspective camera centred at the light).
 *   GS3_ORTHOGRAPHIC  parallel projection, width/ortho_width pixels per world
 *                     unit; x_pixel = scale * x_view + width/2. A directional
 *                     light is such a view (Sec. 4.5: the shadow splat switches
 *                     to an orthographic projection); it shines along
 *                     target - eye, and its distance key is the view-space z
 *                     (depth along the light direction from the eye's plane),
 *                     so the eye must lie outside the scene, on the lit side.
 * The near plane culls Gaussians with view-space z <= near_plane in both. */
enum { GS3_PERSPECTIVE = 0, GS3_ORTHOGRAPHIC = 1 };
typedef struct {
    double eye[3];
    double target[3];
    int32_t width;
    int32_t height;
    double fov;          /* perspective: horizontal field of view, radians, in (0, pi) */
    int32_t projection;  /* GS3_PERSPECTIVE or GS3_ORTHOGRAPHIC */
    double ortho_width;  /* orthographic: world units across the image width, > 0 */
} gs3_view;

/* Appearance model of a scene (gs3_scene.appearance):
 *   GS3_APPEARANCE_LOBES  k isotropic angular lobes per Gaussian, each with
 *       its own axis, sharpness and RGB amplitude (Eq. 7 with sigma_x =
 *       sigma_y), and the MLP inputs [T, feat] / [feat, w_i, w_o] with
 *       3x64 ReLU hidden layers.
 *   GS3_APPEARANCE_BASIS  the paper's own form: k anisotropic basis angular
 *       Gaussians SHARED by all spatial Gaussians (Sec. 4.1, Eq. 6-7 and the
 *       shared-basis paragraph), c = rho_d f_d + rho_s sum_j alpha_j G_j(h');
 *       Phi(T, w_i; mu, l) (Sec. 4.2, Eq. 8) with 3x32 and Psi(w_o; mu, l)
 *       (Sec. 4.3) with 3x128 leaky-ReLU (slope 0.01) hidden layers, inputs
 *       [T, PE(w_i), PE(mu), l] (61) and [PE(w_o), PE(mu), l] (60), where
 *       PE(v) = [v, sin(2^j pi v), cos(2^j pi v) for j = 0..3] (27 values
 *       for a 3-vector, each block ordered x, y, z) and l is the per-Gaussian
 *       6-D latent; w_i, w_o and mu in world space. */
enum { GS3_APPEARANCE_LOBES = 0, GS3_APPEARANCE_BASIS = 1 };

/* Raw (pre-activation) per-Gaussian parameters, device float32 SoA.
 * Activations applied inside the library: scale = exp(log_scale),
 * opacity = sigmoid(opacity_logit), quaternions (w,x,y,z) normalised,
 * lobe axes normalised, lobe sharpness lambda = exp(lobe_log_sharp),
 * basis sigmas = exp(basis_log_sigma). The lobe and feat pointers are read
 * only by GS3_APPEARANCE_LOBES, the fields after `appearance` only by
 * GS3_APPEARANCE_BASIS (zero-initialise the struct for the former). */
typedef struct {
    const float* mean;           /* [3][n] */
    const float* log_scale;      /* [3][n] */
    const float* rot;            /* [4][n]  Sigma = R S S^T R^T (Eq. 1) */
    const float* opacity_logit;  /* [n] */
    const float* shade_rot;      /* [4][n]  world -> shading frame (Sec. 4.1) */
    const float* albedo;         /* [3][n]  rho_d */
    const float* lobe_axis;      /* [k][3][n] in the shading frame */
    const float* lobe_log_sharp; /* [k][n]  log(1/sigma_z) */
    const float* lobe_amp;       /* [k][3][n] RGB weight of each lobe */
    const float* feat;           /* [16][n] per-Gaussian MLP feature */
    int64_t n;                   /* number of Gaussians, >= 0, < 2^31 */
    int32_t k;                   /* lobes per Gaussian (LOBES) or basis angular
                                    Gaussians (BASIS), 0..16 */
    int32_t appearance;          /* GS3_APPEARANCE_LOBES or GS3_APPEARANCE_BASIS */
    const float* spec_albedo;    /* [3][n]  rho_s */
    const float* basis_weight;   /* [k][n]  alpha_j */
    const float* latent;         /* [6][n]  l, input of both MLPs */
    const float* basis_rot;      /* [k][4]  shared: quaternion mapping shading-frame
                                    coordinates to basis j's frame [x_j, y_j, z_j] */
    const float* basis_log_sigma;/* [k][3]  shared: log sigma_x, sigma_y, sigma_z */
} gs3_scene;

/* A dense MLP with three hidden layers and a sigmoid output: w[i] is
 * row-major [out][in] float32, b[i] is [out]. GS3_APPEARANCE_LOBES: 64
 * ReLU units per hidden layer, Phi (shadow refinement, Eq. 8) n_in = 17
 * ([T, feat]), n_out = 1; Psi (residual RGB, Sec. 4.3) n_in = 22 ([feat,
 * w_i, w_o]), n_out = 3. GS3_APPEARANCE_BASIS: leaky ReLU (slope 0.01),
 * Phi 61 -> 32 -> 32 -> 32 -> 1, Psi 60 -> 128 -> 128 -> 128 -> 3. */
typedef struct {
    const float* w[4];
    const float* b[4];
    int32_t n_in;
    int32_t n_out;
} gs3_mlp;

/* A view's device workspace (host struct of plain values, owned by the
 * caller). Its layout is a pure function of (n, width, height,
 * pair_capacity); ws must be 256-byte aligned and hold at least
 * gs3_view_workspace_size(n, width, height, pair_capacity) bytes. */
typedef struct {
    void* ws;
    size_t ws_bytes;
    int64_t n;              /* Gaussians the view was (or will be) built for */
    int32_t width;          /* image size in pixels, 1..16384 */
    int32_t height;
    int64_t pair_capacity;  /* max (tile, Gaussian) pairs, 0..2^31-1 */
    /* Optional (NULL = none) binning status block: two int64 of HOST-PINNED
     * memory (hipHostMalloc / torch pin_memory) owned by the caller and
     * zeroed by it before the first binning. It reports a pair-capacity
     * overflow without synchronising the stream:
     *   status[0]  binning generation, incremented on the host by every
     *              gs3_bin / gs3_sort / gs3_preprocess into this workspace
     *              when it is enqueued;
     *   status[1]  written by the device once that binning's pair count is
     *              known: (generation mod 2^24) << 40 | overflow << 39 |
     *              required pair count (39 bits).
     * gs3_view_poll decodes it. Every call that reads the workspace's lists
     * (gs3_shadow_*, gs3_render*, gs3_render_backward, gs3_view_lists,
     * gs3_view_count_hits) first reads the block on the host and returns
     * GS3_PAIR_CAPACITY_EXCEEDED, enqueueing nothing, when the latest
     * binning has completed with an overflow. A binning call rejects with
     * GS3_INVALID_ARG a block the device cannot address. */
    int64_t* status;
} gs3_viewbuf;

/* Depth key of a view: view-space z (camera) or distance to the eye
 * (light, Sec. 4.2 sorts shadow-ray intersections by distance). */
enum { GS3_DEPTH_Z = 0, GS3_DEPTH_DIST = 1 };

/* Outputs of gs3_render. Images [C][H][W] of the camera view; every
 * pointer is required. n_contrib[p] = one past the position, in the pixel's
 * tile list, of the last Gaussian blended into pixel p (backward state).
 * colour = per-Gaussian [8][n]: c.rgb (Eq. 4), T' (Eq. 8), r.rgb (Sec. 4.3),
 * then 0 - the values splatted into S, Sh and R. */
typedef struct {
    float* final_rgb;  /* [3][H][W]  S * Sh + R */
    float* shading;    /* [3][H][W]  S  */
    float* shadow;     /* [H][W]     Sh */
    float* residual;   /* [3][H][W]  R  */
    float* t_final;    /* [H][W]     transmittance left after the last blend */
    int32_t* n_contrib;/* [H][W] */
    float* colour;     /* [8][n] */
} gs3_images;

/* Gradients written by gs3_render_backward: device pointers with the
 * layouts of gs3_scene (raw parameters) and gs3_mlp. Every call ADDS to
 * them (zero them once per optimisation step; a batch of views accumulates).
 * The MLP pointers of a NULL phi / psi are not used. */
typedef struct gs3_grads {
    float* mean;           /* [3][n] */
    float* log_scale;      /* [3][n] */
    float* rot;            /* [4][n] */
    float* opacity_logit;  /* [n] */
    float* shade_rot;      /* [4][n] */
    float* albedo;         /* [3][n] */
    float* lobe_axis;      /* [k][3][n] */
    float* lobe_log_sharp; /* [k][n] */
    float* lobe_amp;       /* [k][3][n] */
    float* feat;           /* [16][n] */
    float* phi_w[4];       /* like gs3_mlp.w of phi */
    float* phi_b[4];
    float* psi_w[4];
    float* psi_b[4];
    /* GS3_APPEARANCE_BASIS only (the lobe and feat pointers above are then
     * not used): layouts of the gs3_scene fields of the same names */
    float* spec_albedo;
    float* basis_weight;
    float* latent;
    float* basis_rot;
    float* basis_log_sigma;
} gs3_grads;

void gs3_consts_default(gs3_consts* out);
const char* gs3_status_string(int status);
const char* gs3_last_error(void);
/* 1 if the library was built for gfx950 and a gfx950 device is current. */
int gs3_device_ok(void);

/* Bytes of device workspace one view needs: projected splat records, sort
 * buffers for up to `pair_capacity` (tile, Gaussian) pairs, tile ranges.
 * Returns GS3_INVALID_ARG for n < 0, a non-positive image size or
 * pair_capacity < 0. */
int gs3_view_workspace_size(int64_t n, int32_t width, int32_t height,
                            int64_t pair_capacity, size_t* bytes);

/* Sec. 3 / Eq. 1-2 (projection): project the n Gaussians of `scene` into
 * `view` and store the splat records (centre, conic, opacity, depth key,
 * per-axis pixel extent of the hit ellipse) in `ws`. The extent of a splat
 * is rx = ceil(sqrt(2 p Sigma'_xx)), ry = ceil(sqrt(2 p Sigma'_yy)) with
 * p = min(cutoff, ln(opacity / alpha_min)); culled splats get rx = ry = -1.
 * The float32 hit threshold of each splat (q >= thr with q = power log2 e)
 * and its padded bounding box are stored too: every splatting kernel that
 * tests pixels of this view reads them, so all take the same decisions.
 * vb->n must equal scene->n and vb's size the view's. */
int gs3_project(const gs3_scene* scene, const gs3_view* view,
                const gs3_consts* consts, int32_t depth_mode,
                const gs3_viewbuf* vb, gs3_stream_t stream);

/* Sec. 3 ("sorted") and Sec. 4.2 (sorted by distance to the light): tile
 * binning of vb->n splats given explicitly. Splat i covers pixel columns
 * ix[i]-rx[i] .. ix[i]+rx[i] and rows iy[i]-ry[i] .. iy[i]+ry[i] (culled if
 * rx[i] <= 0 or ry[i] <= 0) and is listed in every 16x16 tile of the
 * vb->width x vb->height image those pixels touch. Each tile's list is ordered by
 * (float32 bits of depth[i], i); depth must be >= 0. Results stay in `ws`;
 * gs3_view_lists copies them out. gs3_preprocess calls the same code on the
 * splats gs3_project computed. */
int gs3_bin(const int32_t* ix, const int32_t* iy, const int32_t* rx,
            const int32_t* ry, const float* depth, const gs3_viewbuf* vb,
            gs3_stream_t stream);

/* Sec. 3 (steps a2 / a8): bin and sort the splats the last gs3_project
 * stored in `vb`, exactly as gs3_preprocess does after projecting. Split
 * out so that work that needs only the projected splats (the shadow
 * denominator) can run while the binning does. Errors as gs3_bin. */
int gs3_sort(const gs3_viewbuf* vb, gs3_stream_t stream);

/* gs3_project followed by gs3_sort (steps a1+a2 for the light view, a7+a8
 * for the camera view). */
int gs3_preprocess(const gs3_scene* scene, const gs3_view* view,
                   const gs3_consts* consts, int32_t depth_mode,
                   const gs3_viewbuf* vb, gs3_stream_t stream);

/* Steps a1+a2 / a7+a8 for n_views >= 1 views of one scene in one launch
 * sequence (Sec. 3 projection and sorting; Sec. 4.2 light views sorted by
 * distance): views[v] is projected with depth_modes[v] into vbs[v] and
 * binned there, with the same results as gs3_preprocess on each view alone.
 * The kernels of all views share each launch, so a frame's light and
 * camera views, or the views of many requests, fill the device together
 * and pay the launch sequence once. `views`, `depth_modes` and `vbs` are
 * host arrays of n_views entries; every vbs[v].n equals scene->n, the
 * workspaces must not overlap, and each may have its own size and
 * capacity. Every argument is checked before anything is enqueued
 * (GS3_INVALID_ARG / GS3_WORKSPACE_TOO_SMALL name the offending view);
 * status blocks, overflow and capacity behave per view as for
 * gs3_preprocess. */
int gs3_preprocess_views(const gs3_scene* scene, const gs3_view* views,
                         const int32_t* depth_modes, int32_t n_views,
                         const gs3_consts* consts, const gs3_viewbuf* vbs,
                         gs3_stream_t stream);

/* Number of (tile, Gaussian) pairs of the last binning in `vb` (host
 * value; synchronises `stream`). Returns GS3_PAIR_CAPACITY_EXCEEDED (and
 * the required count) if it exceeded the capacity. An overflowed binning
 * leaves every tile list of the workspace empty; the calls that consume it
 * then write NaN sentinels instead of plausible values: T of
 * gs3_shadow_splat / gs3_shadow_resolve and every image of gs3_render /
 * gs3_render_shaded are NaN. Rebin with a larger capacity. */
int gs3_view_pair_count(const gs3_viewbuf* vb, int64_t* n_pairs, gs3_stream_t stream);

/* Status of the latest binning of `vb` from its status block (vb->status),
 * without touching the device or the stream: *state = 0 while that binning
 * has not completed on the device yet, 1 when it completed within the
 * capacity, 2 when it overflowed; *required_pairs = its unclamped pair count
 * once completed (else -1). GS3_INVALID_ARG when vb->status is NULL. */
enum { GS3_VIEW_PENDING = 0, GS3_VIEW_OK = 1, GS3_VIEW_OVERFLOW = 2 };
int gs3_view_poll(const gs3_viewbuf* vb, int32_t* state, int64_t* required_pairs);

/* Copy the binning of `vb` out: tile_start/tile_end [tiles] (list of tile t
 * is ids[tile_start[t] .. tile_end[t]) ), ids [pair count] Gaussian indices,
 * keys [pair count] (tile << 32 | depth bits). Any pointer may be NULL. */
int gs3_view_lists(const gs3_viewbuf* vb, int32_t* tile_start, int32_t* tile_end,
                   int32_t* ids, uint64_t* keys, gs3_stream_t stream);

/* Copy the projected splats of `vb` out (any pointer may be NULL):
 * mean2d [2][n] (pixel coordinates u, v), conic [3][n] (a, b, c of the
 * inverse 2D covariance, power = -(a dx^2 + 2 b dx dy + c dy^2)/2),
 * opacity [n], depth [n] (the sort key), extent [4][n] int32
 * (floor(u), floor(v), rx, ry). */
int gs3_view_splats(const gs3_viewbuf* vb, float* mean2d, float* conic, float* opacity,
                    float* depth, int32_t* extent, gs3_stream_t stream);

/* Measurement: the number of (pixel, splat) hits of the binned view in
 * `vb` (pixels where power >= -cutoff and alpha >= alpha_min, Sec. 3 Eq. 2)
 * written to *hits (one int64 of device memory). With stop_early != 0 only
 * the hits blended before each pixel's early stop (t_min) are counted, as in
 * the camera pass; with 0 every hit is counted, as the shadow pass evaluates
 * them. This is the work unit the splatting kernels are measured against. */
int gs3_view_count_hits(const gs3_consts* consts, const gs3_viewbuf* vb, int32_t stop_early,
                        int64_t* hits, gs3_stream_t stream);

/* Sec. 4.2, Fig. 3 (step a3): shadow splatting. `light_vb` holds a view
 * preprocessed with GS3_DEPTH_DIST from the light position. For every light
 * pixel m and every Gaussian j hit there, T_m(j) is the product of
 * (1 - alpha_km) over the Gaussians k hit at m with
 * dist_k < dist_j - shadow_bias; num_j = sum_m beta_jm T_m(j) and
 * den_j = sum_m beta_jm (beta = exp(power), the splat density at the pixel
 * centre). Outputs: num_den [2][n] (saved for the backward), T [n] =
 * num/den, or 1 where den = 0. */
int gs3_shadow_splat(const gs3_consts* consts, const gs3_viewbuf* light_vb,
                     float* num_den, float* T, gs3_stream_t stream);

/* The three parts of gs3_shadow_splat (Sec. 4.2), callable one by one so
 * that each can be timed or overlapped on its own; gs3_shadow_splat is
 * exactly gs3_shadow_den, gs3_shadow_num, gs3_shadow_resolve in that order.
 *   gs3_shadow_den      writes den_j = sum_m beta_jm into num_den[n .. 2n).
 *   gs3_shadow_num      accumulates num_j = sum_m beta_jm T_m(j) in the
 *                       view workspace (one kernel; num_den is not touched);
 *                       terms of a pixel whose transmittance in front of j
 *                       is below 2^-20 are left out, which moves
 *                       num_j / den_j by less than 2^-20. The accumulator
 *                       starts at zero after gs3_project and after
 *                       gs3_shadow_resolve, so each gs3_shadow_num must be
 *                       followed by gs3_shadow_resolve before the next one
 *                       on the same workspace.
 *   gs3_shadow_resolve  writes num_j into num_den[0 .. n), T[j] = num_j /
 *                       den_j (1 where den_j = 0), and clears the
 *                       accumulator; reads den from num_den[n .. 2n).
 * Same arguments, layout and errors as gs3_shadow_splat (T is only used by
 * the third). */
int gs3_shadow_den(const gs3_consts* consts, const gs3_viewbuf* light_vb, float* num_den,
                   gs3_stream_t stream);
int gs3_shadow_num(const gs3_consts* consts, const gs3_viewbuf* light_vb, float* num_den,
                   gs3_stream_t stream);
int gs3_shadow_resolve(const gs3_viewbuf* light_vb, float* num_den, float* T, gs3_stream_t stream);

/* Sec. 4.1-4.3 and Fig. 2 (steps a4-a6, a9): shade every Gaussian for the
 * light of view `light` (a perspective view: a point light at light->eye,
 * w_i the unit vector from the Gaussian to it; an orthographic view: a
 * directional light, w_i = (eye - target) / |eye - target| for every
 * Gaussian; Sec. 4.5) seen from the camera `cam`
 * (c = rho_d f_d + sum_k amp_k G_k, Eq. 4-7, isotropic lobes, unit light;
 * or, for a GS3_APPEARANCE_BASIS scene, c = rho_d f_d + rho_s sum_j
 * alpha_j G_j with the shared anisotropic basis),
 * refine T with Phi (T' = T if phi is NULL), evaluate Psi (r = 0 if psi is
 * NULL), then splat c, T' and r toward the camera front to back and write
 * final = S * Sh + R. `cam_vb` holds `cam` preprocessed with GS3_DEPTH_Z.
 * MLP weight pointers may be in any device memory; n_in/n_out must be
 * 17/1 (phi) and 22/3 (psi), or 61/1 and 60/3 for a basis scene. The MLP
 * arithmetic is float32; its hidden layers run as split half-precision
 * products (each operand hi + lo/2048, about 2^-22 relative per product),
 * which assumes layer inputs and weights below the half range (65504). */
int gs3_render(const gs3_scene* scene, const gs3_view* cam,
               const gs3_view* light, const gs3_consts* consts,
               const float* T, const gs3_mlp* phi, const gs3_mlp* psi,
               const gs3_viewbuf* cam_vb, const gs3_images* out,
               gs3_stream_t stream);

/* Steps a3 and a4-a6 + a9 for n_views >= 1 views in one launch sequence
 * (Sec. 4.2 shadow splatting; Sec. 4.1-4.3 and Fig. 2 shading, MLPs and
 * camera splat): the same results as gs3_shadow_splat / gs3_render on each
 * view alone, with the kernels of all views sharing each launch (views of
 * different sizes included), so that the requests of a serving batch pay
 * one launch sequence. Arrays are host arrays of n_views entries:
 *   gs3_shadow_splat_views  light_vbs[v] (preprocessed with GS3_DEPTH_DIST,
 *       every .n equal), num_den[v] / T[v] device outputs of view v.
 *   gs3_render_views        cams[v] / lights[v] views, T[v] the shadow
 *       values of lights[v], cam_vbs[v] (preprocessed with GS3_DEPTH_Z),
 *       outs[v] the images; one scene and one pair of MLPs for all views.
 * Workspaces must not overlap. Every argument is checked before anything is
 * enqueued; errors as for the one-view calls (GS3_PAIR_CAPACITY_EXCEEDED
 * when a status block reports an overflowed binning of any view). */
int gs3_shadow_splat_views(const gs3_consts* consts, const gs3_viewbuf* light_vbs, int32_t n_views,
                           float* const* num_den, float* const* T, gs3_stream_t stream);
int gs3_render_views(const gs3_scene* scene, const gs3_view* cams, const gs3_view* lights, int32_t n_views,
                     const gs3_consts* consts, const float* const* T, const gs3_mlp* phi, const gs3_mlp* psi,
                     const gs3_viewbuf* cam_vbs, const gs3_images* outs, gs3_stream_t stream);

/* The two halves of gs3_render, callable apart so that the part that does
 * not depend on the shadow values can run before (or alongside) the shadow
 * splat; gs3_render is exactly gs3_shade then gs3_render_shaded.
 *   gs3_shade          Sec. 4.1 (Eq. 4-7) and Sec. 4.3: per-Gaussian colour
 *                      c and residual r (Psi, r = 0 if psi is NULL) into
 *                      `cam_vb` and colour rows 0-2 and 4-7.
 *   gs3_render_shaded  Sec. 4.2 (Eq. 8): T' = Phi(T) (T' = T if phi is
 *                      NULL) into cam_vb and colour row 3, then the camera
 *                      splat of Fig. 2 and final = S * Sh + R. Needs the
 *                      gs3_shade of the same camera and light first.
 * Arguments, layouts and errors as in gs3_render. */
int gs3_shade(const gs3_scene* scene, const gs3_view* cam, const gs3_view* light,
              const gs3_mlp* psi, const gs3_viewbuf* cam_vb, float* colour, gs3_stream_t stream);
int gs3_render_shaded(const gs3_scene* scene, const gs3_view* cam, const gs3_view* light,
                      const gs3_consts* consts, const float* T, const gs3_mlp* phi,
                      const gs3_viewbuf* cam_vb, const gs3_images* out, gs3_stream_t stream);

/* Bytes of device workspace gs3_render_backward needs for n Gaussians and
 * a light image of light_width x light_height: per-Gaussian splat and
 * colour gradients, per-light-pixel sums, and the MLP activations kept for
 * the weight gradients (about 3.3 KB per Gaussian with both MLPs). */
int gs3_backward_workspace_size(int64_t n, int32_t light_width, int32_t light_height, size_t* bytes);
/* The same for a scene of appearance `appearance` (gs3_backward_workspace_size
 * is this with GS3_APPEARANCE_LOBES). GS3_APPEARANCE_BASIS keeps about 4.4 KB
 * per Gaussian: both MLPs' layer inputs and pre-activation gradients. */
int gs3_backward_workspace_size_for(int32_t appearance, int64_t n, int32_t light_width, int32_t light_height,
                                    size_t* bytes);

/* Sec. 4.4 (training by gradient descent on an image loss): the adjoint of
 * gs3_shadow_splat followed by gs3_render. Given dL_dfinal [3][H][W] (the
 * gradient of a loss with respect to the camera image `final`), ADDS dL/d
 * of every raw scene parameter and MLP weight to `grads`.
 * Inputs are the forward's, unchanged since it ran: `light` and `cam` the
 * two views (light->eye is the light position), `light_vb` / `cam_vb`
 * their preprocessed buffers (light with GS3_DEPTH_DIST, cam with
 * GS3_DEPTH_Z; cam_vb also holds the per-Gaussian colours gs3_render left
 * there), T and num_den from gs3_shadow_splat, and fwd->shading, ->shadow,
 * ->residual from gs3_render (the other image pointers are not used).
 * Nothing per (pixel, splat) pair is stored by the forward: the splats are
 * recomputed per tile with the forward's arithmetic, so the gradient is that
 * of the function the forward evaluated (threshold decisions fixed). Terms
 * of light rays with transmittance below 2^-20, which the forward numerator
 * leaves out, are left out here as well. `ws` (256-byte aligned,
 * gs3_backward_workspace_size bytes) is scratch. Errors: GS3_INVALID_ARG
 * for NULL or mismatched arguments, GS3_WORKSPACE_TOO_SMALL. */
int gs3_render_backward(const gs3_scene* scene, const gs3_view* cam, const gs3_view* light,
                        const gs3_consts* consts, const float* T, const float* num_den,
                        const gs3_mlp* phi, const gs3_mlp* psi,
                        const gs3_viewbuf* light_vb, const gs3_viewbuf* cam_vb,
                        const gs3_images* fwd, const float* dL_dfinal,
                        const gs3_grads* grads, void* ws, size_t ws_bytes, gs3_stream_t stream);

/* Sec. 4.4, Eq. 9 (the L1 term of the training loss): for `count` float32
 * elements, *loss = scale * sum_i |pred_i - target_i| (one float of device
 * memory) and, unless dL_dpred is NULL, dL_dpred[i] = scale *
 * sign(pred_i - target_i) (0 where the two are equal: the subgradient the
 * oracle uses). scale = 1 / count gives the mean. The sum is formed in a
 * fixed order, float64 partial sums of consecutive 8192-element chunks
 * added in chunk order, so the value is the same on every run. `ws` (256-
 * byte aligned, gs3_l1_loss_workspace_size bytes) holds the partial sums.
 * Errors: GS3_INVALID_ARG (NULL pred/target/loss with count > 0, count < 0,
 * misaligned ws), GS3_WORKSPACE_TOO_SMALL. */
int gs3_l1_loss_workspace_size(int64_t count, size_t* bytes);
int gs3_l1_loss(const float* pred, const float* target, int64_t count, float scale, float* loss,
                float* dL_dpred, void* ws, size_t ws_bytes, gs3_stream_t stream);

/* Sec. 4.4, Eq. 9 (the D-SSIM term; lambda = 0.2 in the paper): SSIM with
 * an 11x11 Gaussian window (sigma 1.5, normalised, zero outside the image),
 * C1 = 0.01^2, C2 = 0.03^2, each of `channels` planes of pred and target
 * ([channels][height][width] float32) on its own:
 *   *loss = scale * sum over channels and pixels of (1 - SSIM)
 * (scale = lambda / (channels height width) gives lambda times the mean
 * D-SSIM), and unless dL_dpred is NULL its gradient with respect to pred,
 * written (accumulate = 0) or added (accumulate != 0) to dL_dpred, so that
 * it can follow gs3_l1_loss into the same buffer. target is not
 * differentiated. The sum is formed in a fixed order (float64 per-tile
 * partial sums added in tile order). `ws` (256-byte aligned,
 * gs3_dssim_loss_workspace_size bytes) holds three per-pixel maps and the
 * partial sums. Errors: GS3_INVALID_ARG (NULL pointer, size out of
 * 1..64 x 1..16384 x 1..16384, misaligned ws), GS3_WORKSPACE_TOO_SMALL. */
int gs3_dssim_loss_workspace_size(int32_t channels, int32_t height, int32_t width, size_t* bytes);
int gs3_dssim_loss(const float* pred, const float* target, int32_t channels, int32_t height, int32_t width,
                   float scale, float* loss, float* dL_dpred, int32_t accumulate, void* ws, size_t ws_bytes,
                   gs3_stream_t stream);

/* Sec. 4.4 (the optimiser: Adam with momentum beta1 = 0.9): one update of
 * `count` float32 parameters in place, step t >= 1 the update's number:
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   param -= lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).
 * m and v (zeroed before step 1) are the caller's moment buffers. Errors:
 * GS3_INVALID_ARG for NULL buffers, step < 1, betas outside [0, 1), eps < 0
 * or a non-finite lr. */
int gs3_adam_step(float* param, const float* grad, float* m, float* v, int64_t count, int32_t step, float lr,
                  float beta1, float beta2, float eps, gs3_stream_t stream);

/* gs3_l1_loss for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels, same arguments without the workspace, same results bit
 * for bit. The partial sums live in a 32 KiB array inside the library, one
 * per device, held until the process ends; nothing is allocated per call.
 * count is limited to 33,554,432 elements (4096 chunks of 8192): larger
 * counts return GS3_INVALID_ARG. Every call on one device shares that
 * array, so calls that overlap on a device (concurrent streams, or threads
 * without ordering) race and must not be issued; calls ordered on one
 * stream are safe, each fully rewriting the partial sums it reads. */
int gs3_l1_loss_noalloc(const float* pred, const float* target, int64_t count, float scale, float* loss,
                        float* dL_dpred, gs3_stream_t stream);

/* Sec. 4.5 (environment lighting as a linear combination of the renders
 * under sampled directional lights): dst[i] += weight * src[i] over `count`
 * float32 of device memory (dst and src must not overlap). Errors:
 * GS3_INVALID_ARG for count < 0, a NULL pointer with count > 0 or a
 * non-finite weight. */
int gs3_image_accumulate(float* dst, const float* src, float weight, int64_t count, gs3_stream_t stream);

/* Gradient-set upkeep of a training step (Sec. 4.4): gs3_render_backward
 * adds into its gradients, so a step clears them first, and views whose
 * gradients were accumulated in separate sets (to run concurrently) are
 * summed afterwards. Both act on `count` float32 of device memory:
 *   gs3_grads_clear       g[i] = 0
 *   gs3_grads_accumulate  dst[i] += src[i]   (dst and src must not overlap)
 * Errors: GS3_INVALID_ARG for count < 0 or a NULL pointer with count > 0. */
int gs3_grads_clear(float* g, int64_t count, gs3_stream_t stream);
int gs3_grads_accumulate(float* dst, const float* src, int64_t count, gs3_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GS3_H */
