/*
 * snx.h -- C ABI of the MI355X (gfx950) surface-normal-from-disparity library.
 *
 * The library implements the per-pixel path of "Robust and Real-time Surface
 * Normal Estimation from Stereo Disparities using Affine Transformations"
 * (Kariko, Faisal, Hajder): a rectified disparity map goes through a denoising
 * filter, per-pixel disparity gradients, the rectified affine transform A, the
 * surface normal from A and the camera, connected surface components, and comes
 * out as a dense oriented point cloud (abstract; Sec. 2-3).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Image buffers are DEVICE pointers (hipMalloc'd or a torch tensor's
 *    data_ptr()), row-major, with row strides given in ELEMENTS (>= width).
 *    The caller owns every buffer; the library never retains or frees one.
 *  - u is the column, v the row (downwards); pixel centres are at integers.
 *  - Disparity is the positive D = u_left - u_right = f_x * b / z.  (The paper's
 *    d is u_right - u_left = -D; every formula below is stated for D.)
 *  - A disparity is valid iff it is finite and > 0.  Invalid pixels are data,
 *    not errors: they produce NaN in float outputs and -1 in labels.  Pixels
 *    outside the image are invalid (no padding, clamping or mirroring).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *    enqueues work; it returns once arguments are validated and kernels are
 *    launched.  Arguments are validated before anything is launched: an invalid
 *    call returns SNX_ERR_ARG / SNX_ERR_UNSUPPORTED / SNX_ERR_WORKSPACE and
 *    writes nothing.  A failed launch returns SNX_ERR_HIP.
 *  - width == 0 or height == 0 is a valid empty call (buffers may be NULL).
 *  - width * height must be < 2^31 (labels are int32 linear indices).
 *  - Results are bit-identical from run to run; the fused and the separate
 *    calls produce bit-identical outputs for the same inputs.
 *  - snx_last_error() returns a message for the calling thread's last failure.
 */
#ifndef SNX_H
#define SNX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum snx_status {
    SNX_OK = 0,
    SNX_ERR_ARG = 1,          /* NULL pointer, bad size, stride, window or camera */
    SNX_ERR_UNSUPPORTED = 2,  /* valid but unsupported (e.g. window too large)   */
    SNX_ERR_WORKSPACE = 3,    /* workspace missing or too small                   */
    SNX_ERR_HIP = 4,          /* a HIP runtime call or kernel launch failed       */
    SNX_ERR_MODEL = 5,        /* learned filter without a complete model, or a
                                 corrupt / incompatible model file               */
    SNX_ERR_IO = 6            /* a model file could not be opened, read or written */
} snx_status;

/* Rectified pin-hole pair (Sec. 2, projections Pi_1 and Pi_2): focal lengths in
 * pixels, baseline in the unit the point cloud is wanted in, principal point in
 * pixels.  fx, fy, baseline must be finite and > 0; u0, v0 finite. */
typedef struct snx_camera {
    float fx, fy, baseline, u0, v0;
} snx_camera;

/* Denoising filter.  window = n_f (odd, 1..63): the output at a valid pixel c is
 * the intercept h of the least-squares plane D_i ~ h + g_u v_ix + g_v v_iy
 * fitted to the valid pixels i of the n_f x n_f window around c (the
 * over-determined LSQ of Sec. 3.2 with a constant column).  On a full window
 * this is the box mean; n_f = 1 is the identity (the paper's unfiltered mode).
 * The centre value passes through unchanged when fewer than
 * max(3, min_support) pixels are valid or the 3x3 normal matrix is singular.
 * mode SNX_FILTER_LSQ: model must be NULL.  mode SNX_FILTER_CNN: the learned
 * denoiser of snx_cnn_denoise replaces the filter (window/min_support unused);
 * model points to an snx_cnn_model. */
#define SNX_FILTER_LSQ 0
#define SNX_FILTER_CNN 1   /* learned residual denoiser; model = const snx_cnn_model* */
typedef struct snx_denoise_params {
    int32_t window;
    int32_t min_support;
    int32_t mode;
    int32_t reserved;
    const void *model;
} snx_denoise_params;

/* Gradient window.  window = n_g (odd, 3..63).  The slope at a valid pixel c is
 * the anchored LSQ of Sec. 3.2-3.3 over the valid pixels i != c of the n_g x n_g
 * window, with alpha, beta, gamma summed over that (possibly masked) support
 * (the two-pass scheme of Sec. 3.4).  It is defined iff at least min_support
 * such pixels exist and alpha*gamma - beta^2 > 0; min_support <= 0 selects the
 * default ceil(n_g^2 / 2). */
typedef struct snx_normal_params {
    int32_t window;
    int32_t min_support;
} snx_normal_params;

/* Component edge predicate: 4-neighbours p, q are joined iff both are valid and
 *   |D_p - D_q| <= max(t_abs, k_rel * min(D_p, D_q))
 * evaluated in binary64 on the float32 inputs (the pairwise form of the
 * covered-depth stopping rule of Sec. 3.4).  k_rel, t_abs finite and >= 0. */
typedef struct snx_component_params {
    float k_rel;   /* default 0.1 */
    float t_abs;   /* default 1.0 px */
} snx_component_params;

/* One point of the dense oriented point cloud, 32 bytes. */
#define SNX_POINT_DEFINED  1u   /* position and normal are defined            */
#define SNX_POINT_LABELLED 2u   /* label >= 0 (the raw disparity was valid)    */
typedef struct snx_point {
    float x, y, z;      /* camera frame, x right, y down, z forward       */
    float nx, ny, nz;   /* unit normal facing the camera                  */
    int32_t label;      /* component label (minimum linear index) or -1    */
    uint32_t flags;     /* SNX_POINT_* bits                                */
} snx_point;

/* ---------------------------------------------------------------------------
 * snx_denoise -- the filter (see snx_denoise_params).
 *   disp [height x disp_stride] float32 in; out [height x out_stride] float32
 *   out (NaN where the input is invalid).  disp and out must not overlap.
 * ------------------------------------------------------------------------- */
snx_status snx_denoise(const float *disp, int64_t disp_stride,
                       float *out, int64_t out_stride,
                       int32_t width, int32_t height,
                       const snx_denoise_params *params, void *stream);

/* ---------------------------------------------------------------------------
 * snx_affine_normals -- gradients, A and normals from a (denoised) disparity.
 * Gradient (g_u, g_v) as in snx_normal_params; then (Sec. 2 eq. affine_mtx and
 * Sec. 3.2) A = [[a1, a2], [0, 1]] with a1 = 1 - g_u, a2 = -g_v; then the normal
 * of Sec. 3.1, computed as n = -m / |m| with
 *   m = (f_x g_u, f_y g_v, D_c - (u - u0) g_u - (v - v0) g_v),
 * which is the cross product of the paper's two constraint vectors divided by
 * b z (the printed closed form has the sign of its b term flipped; m . X =
 * f_x b > 0, so n always faces the camera).
 *   disp_dn [height x stride] float32 in.
 *   affine  NULL or 2 planes (a1 then a2), each [height x out_stride], the second
 *           starting at affine + height * out_stride.
 *   normals NULL or 3 planes (nx, ny, nz) laid out the same way.
 *   Undefined pixels get NaN in every plane.
 * ------------------------------------------------------------------------- */
snx_status snx_affine_normals(const float *disp_dn, int64_t stride,
                              int32_t width, int32_t height,
                              const snx_camera *cam,
                              const snx_normal_params *params,
                              float *affine, float *normals, int64_t out_stride,
                              void *stream);

/* ---------------------------------------------------------------------------
 * snx_affine_normals_labels -- snx_affine_normals with the n_g x n_g window
 * restricted to the centre's surface component: neighbour i is used only if it
 * is valid and labels[i] == labels[c] (so points of a neighbouring surface do
 * not smooth the normal, the concern of Sec. 3.4).  labels: [height x
 * label_stride] int32, e.g. from snx_components on the raw disparity; a centre
 * with a negative label is undefined.  Window, min_support (counted over the
 * restricted support), outputs and layout as in snx_affine_normals; windows
 * above 63 are rejected like there.
 * ------------------------------------------------------------------------- */
snx_status snx_affine_normals_labels(const float *disp_dn, int64_t stride,
                                     const int32_t *labels, int64_t label_stride,
                                     int32_t width, int32_t height,
                                     const snx_camera *cam,
                                     const snx_normal_params *params,
                                     float *affine, float *normals, int64_t out_stride,
                                     void *stream);

/* ---------------------------------------------------------------------------
 * snx_affine_normals_star -- gradients, A and normals over the adaptive
 * star-fill support of Sec. 3.4 (Adaptive Region Estimation) instead of a
 * square window.  From a valid centre c, rays leave in `directions` = 4 (the
 * axes), 8 (axes and diagonals) or 16 directions -- the angles
 * 2 pi m / directions with the step scaled to a unit larger component -- and
 * take c + round(k e_m) (each component rounded to the nearest pixel),
 * k = 1 .. steps (1..32), stopping before the first pixel that is invalid or
 * outside the image or meets the stopping rule:
 *   SNX_STOP_CD  covered depth: with a, b the smallest and largest disparity of
 *                c and of the ray's pixels so far including the new one, stop
 *                when D_c (b - a) > threshold (a b), i.e. when the depth range
 *                f_x B (1/a - 1/b) exceeds `threshold` times the depth of c;
 *   SNX_STOP_ST  simple threshold on the depth Laplacian: stop when
 *                ((z_r + z_l) + (z_d + z_u)) - 4 z, z = f_x B / D, at the new
 *                pixel is undefined (a 4-neighbour invalid or outside) or its
 *                magnitude exceeds `threshold` (baseline units).
 * Both rules are evaluated in binary64 on the float32 disparities.  The slope
 * is the anchored LSQ of snx_normal_params over the pixels the rays take, each
 * pixel once (with 16 directions neighbouring rays share their first pixel;
 * the centre anchors the fit); it is defined iff they number at least min_support
 * (<= 0 selects `directions`) and alpha*gamma - beta^2 > 0.  A and the normal
 * follow as in snx_affine_normals, and the buffers are laid out the same way.
 * Other direction counts return SNX_ERR_UNSUPPORTED; steps outside 1..32, an
 * unknown rule or a negative or non-finite threshold return SNX_ERR_ARG.
 * ------------------------------------------------------------------------- */
#define SNX_STOP_CD 0
#define SNX_STOP_ST 1
typedef struct snx_star_params {
    int32_t directions;   /* 4, 8 or 16 */
    int32_t steps;        /* 1 .. 32 pixels per ray */
    int32_t stop;         /* SNX_STOP_CD or SNX_STOP_ST */
    int32_t min_support;  /* <= 0: directions */
    double threshold;     /* CD: k (e.g. 0.05); ST: t in baseline units */
} snx_star_params;
snx_status snx_affine_normals_star(const float *disp_dn, int64_t stride,
                                   int32_t width, int32_t height,
                                   const snx_camera *cam,
                                   const snx_star_params *params,
                                   float *affine, float *normals, int64_t out_stride,
                                   void *stream);

/* ---------------------------------------------------------------------------
 * snx_components -- connected surface components of the RAW disparity under the
 * predicate of snx_component_params.  labels[v * label_stride + u] receives the
 * smallest linear index v' * width + u' of the pixel's component, or -1 if the
 * pixel is invalid.  num_components: NULL or a device int32 that receives the
 * number of components.  workspace: device memory of at least
 * snx_components_workspace_size(width, height) bytes, owned by the caller; its
 * contents need no initialisation and are scratch after the call.  Concurrent
 * calls need distinct workspaces.
 * ------------------------------------------------------------------------- */
size_t snx_components_workspace_size(int32_t width, int32_t height);
snx_status snx_components(const float *disp_raw, int64_t stride,
                          int32_t width, int32_t height,
                          const snx_component_params *params,
                          int32_t *labels, int64_t label_stride,
                          int32_t *num_components,
                          void *workspace, size_t workspace_bytes,
                          void *stream);

/* snx_components_from_edges -- the labelling of snx_components on a 4-neighbour
 * graph given explicitly instead of by the covered-depth predicate, so that
 * every edge pattern can be posed independently of pixel validity (a test hook
 * for exhaustive checks of the union-find; Sec. 3.4 defines the regions the
 * predicate builds).  edges [height x stride] uint8, one byte per pixel:
 * bit 0 = the pixel is present, bit 1 = edge to its left neighbour (u - 1),
 * bit 2 = edge to its upper neighbour (v - 1); other bits are ignored, and an
 * edge counts only between two present pixels (bits on the image border are
 * ignored).  Labels, count, workspace and errors as in snx_components (absent
 * pixels get -1). */
snx_status snx_components_from_edges(const uint8_t *edges, int64_t stride,
                                     int32_t width, int32_t height,
                                     int32_t *labels, int64_t label_stride,
                                     int32_t *num_components,
                                     void *workspace, size_t workspace_bytes,
                                     void *stream);

/* ---------------------------------------------------------------------------
 * snx_components_creases -- snx_components where every 4-neighbour edge must
 * also pass a normal-crease test: n_p . n_q = ((nx_p nx_q + ny_p ny_q) +
 * nz_p nz_q) >= crease_cos in binary64 on the float32 normals (a pixel whose
 * normal is NaN imposes no test).  Covered depth alone joins surfaces that
 * meet at a depth-continuous crease (Sec. 3.4 says so); this test separates
 * them.  normals: 3 planes [height x normals_stride] (nx, ny, nz, as written
 * by snx_affine_normals), the second starting at normals + height *
 * normals_stride.  crease_cos in [-1, 1].  Labels, count, workspace and
 * errors as in snx_components.
 * ------------------------------------------------------------------------- */
snx_status snx_components_creases(const float *disp_raw, int64_t stride,
                                  const float *normals, int64_t normals_stride,
                                  int32_t width, int32_t height,
                                  const snx_component_params *params, double crease_cos,
                                  int32_t *labels, int64_t label_stride,
                                  int32_t *num_components,
                                  void *workspace, size_t workspace_bytes,
                                  void *stream);

/* ---------------------------------------------------------------------------
 * snx_point_cloud -- dense oriented point cloud (abstract; Sec. 2 projections).
 * Where the normal is defined: z = f_x b / D, x = (u - u0) z / f_x,
 * y = (v - v0) z / f_y with D the denoised disparity, plus the normal; elsewhere
 * NaN coordinates and normal.  label is copied from `labels` (NULL: -1).
 *   disp_dn [height x disp_stride], normals 3 planes [height x normals_stride]
 *   (as written by snx_affine_normals), labels [height x label_stride] or NULL,
 *   out: width * height records, row-major, contiguous.
 * ------------------------------------------------------------------------- */
snx_status snx_point_cloud(const float *disp_dn, int64_t disp_stride,
                           const float *normals, int64_t normals_stride,
                           const int32_t *labels, int64_t label_stride,
                           int32_t width, int32_t height,
                           const snx_camera *cam, snx_point *out, void *stream);

/* ---------------------------------------------------------------------------
 * snx_compact_points -- the compacted oriented point cloud: the records of
 * `points` (width * height contiguous records, as written by snx_point_cloud,
 * snx_oriented_point_cloud or snx_pipeline) whose flags hold
 * SNX_POINT_DEFINED, copied unchanged and contiguously to `out` in raster
 * order; *count (device int32) receives their number.  out must hold
 * width * height records and must not overlap points.  workspace: device
 * memory of at least snx_compact_points_workspace_size(width, height) bytes,
 * owned by the caller, scratch after the call; concurrent calls need distinct
 * workspaces.  width == 0 or height == 0 writes *count = 0.
 * ------------------------------------------------------------------------- */
size_t snx_compact_points_workspace_size(int32_t width, int32_t height);
snx_status snx_compact_points(const snx_point *points, int32_t width, int32_t height,
                              snx_point *out, int32_t *count,
                              void *workspace, size_t workspace_bytes, void *stream);

/* snx_compact_points_noalloc -- snx_compact_points for callers that cannot
 * allocate or pass device memory of their own (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments and
 * output as snx_compact_points without the workspace: the chunk counts live in
 * a static 32 KiB device array of the library (one copy per GPU, held until the
 * process ends; its address is looked up once per device on the first call
 * there).  The call allocates nothing.  Limit: width * height <= 33 554 432
 * records (8192 chunks of 4096); larger frames return
 * SNX_ERR_UNSUPPORTED before anything is launched.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (concurrent streams,
 * host threads) race and must be serialised by the caller. */
snx_status snx_compact_points_noalloc(const snx_point *points, int32_t width, int32_t height,
                                      snx_point *out, int32_t *count, void *stream);

/* ---------------------------------------------------------------------------
 * snx_oriented_point_cloud -- filter, gradients, A, normal and point records in
 * ONE kernel, given component labels already computed by snx_components on the
 * same raw disparity.  Outputs are bit-identical to snx_denoise ->
 * snx_affine_normals -> snx_point_cloud with the same parameters.
 *   disp [height x stride] raw float32; labels [height x label_stride] int32
 *   (input; NULL gives label -1 in every record); disp_dn, affine, normals: NULL
 *   or as in the separate calls (out_stride); points: width * height records.
 * ------------------------------------------------------------------------- */
snx_status snx_oriented_point_cloud(const float *disp, int64_t stride,
                                    int32_t width, int32_t height,
                                    const snx_camera *cam,
                                    const snx_denoise_params *denoise,
                                    const snx_normal_params *normal,
                                    const int32_t *labels, int64_t label_stride,
                                    float *disp_dn, float *affine, float *normals,
                                    int64_t out_stride, snx_point *points,
                                    void *stream);

/* ---------------------------------------------------------------------------
 * snx_pipeline -- the whole path in three kernels: one read of the raw disparity
 * gives the filtered disparity and each tile's local component forest; tile
 * seams are united; one fused kernel then computes gradients, A, normals,
 * resolves the forest into final labels and writes the point records.  Outputs
 * are bit-identical to snx_denoise -> snx_affine_normals -> snx_components ->
 * snx_point_cloud with the same parameters.
 *   disp_dn, affine, normals: NULL or as in the separate calls (out_stride).
 *   labels [height x label_stride] required (final labels on return);
 *   num_components NULL or device int32; points: width * height records.
 *   workspace: at least snx_pipeline_workspace_size(width, height) bytes.
 * ------------------------------------------------------------------------- */
size_t snx_pipeline_workspace_size(int32_t width, int32_t height);
snx_status snx_pipeline(const float *disp, int64_t stride,
                        int32_t width, int32_t height,
                        const snx_camera *cam,
                        const snx_denoise_params *denoise,
                        const snx_normal_params *normal,
                        const snx_component_params *comp,
                        float *disp_dn, float *affine, float *normals,
                        int64_t out_stride,
                        int32_t *labels, int64_t label_stride,
                        int32_t *num_components,
                        snx_point *points,
                        void *workspace, size_t workspace_bytes,
                        void *stream);

/* snx_pipeline split in two parts (for callers that interleave other work or
 * time the parts): parts = SNX_PART_FOREST runs the filter, the local forests
 * and the seam unions; parts = SNX_PART_POINTS runs the fused back kernel.
 * Calling SNX_PART_FOREST then SNX_PART_POINTS on the same stream with the same
 * arguments and workspace equals snx_pipeline (parts = SNX_PART_FOREST |
 * SNX_PART_POINTS).  Between the two calls `labels` (or the workspace) holds a
 * label forest, not final labels. */
#define SNX_PART_FOREST 1
#define SNX_PART_POINTS 2
snx_status snx_pipeline_part(const float *disp, int64_t stride,
                             int32_t width, int32_t height,
                             const snx_camera *cam,
                             const snx_denoise_params *denoise,
                             const snx_normal_params *normal,
                             const snx_component_params *comp,
                             float *disp_dn, float *affine, float *normals,
                             int64_t out_stride,
                             int32_t *labels, int64_t label_stride,
                             int32_t *num_components,
                             snx_point *points,
                             void *workspace, size_t workspace_bytes,
                             int32_t parts, void *stream);

/* ---------------------------------------------------------------------------
 * snx_autotune -- times the compiled tile heights of the stencil kernel for
 * frames of width x height with these windows (the fused filter + gradient
 * kernel, and when the filter window is > 1 also the gradient-only kernel that
 * snx_pipeline's second part and snx_affine_normals use) on `stream`, and
 * records the fastest for later calls in this process (and appends it to the
 * file named by $SNX_AUTOTUNE_CACHE, which later processes read).  A set-up
 * call: it allocates and frees temporary device memory and synchronizes the
 * stream.  chosen: NULL or host int32[2] receiving the tile heights picked
 * (fused, gradient-only); 0 means no compiled candidate (defaults apply).
 * ------------------------------------------------------------------------- */
snx_status snx_autotune(int32_t width, int32_t height,
                        const snx_denoise_params *denoise,
                        const snx_normal_params *normal,
                        int32_t *chosen, void *stream);

/* snx_tune_set -- pins (tile_height > 0) or clears (0) the tile height used for
 * frames of this size class (floor(log2(width*height))) with these windows:
 * filter_window 1 with normal_window n is the gradient-only kernel,
 * normal_window 0 the filter-only kernel.  SNX_ERR_UNSUPPORTED if no kernel is
 * compiled for that tile height.  Outputs never depend on the tile height. */
snx_status snx_tune_set(int32_t width, int32_t height, int32_t filter_window,
                        int32_t normal_window, int32_t tile_height);

/* ===========================================================================
 * Learned residual denoiser (stands in for the LSQ filter; the paper notes the
 * method is differentiable and convolution-like, Sec. 1).
 *   mu = LSQ filter (window 3) as float32; x = [(D - mu)/s, valid], s = 1 px;
 *   six 3x3 convolutions 2->32, 4 x 32->32 (ReLU), 32->1, zero padding;
 *   D~ = mu + s*y at valid pixels, NaN elsewhere.
 * Weights and activations are bfloat16 with float32 accumulation (MFMA).
 * Parameters: snx_cnn_param_count() floats, layer by layer W_k [Cout][Cin][3][3]
 * then b_k.  `packed` holds snx_cnn_packed_bytes() bytes of bf16 weight layouts
 * derived from the parameters by snx_cnn_pack (and by snx_cnn_train_step).
 * ========================================================================= */
typedef struct snx_cnn_model {
    const float *params;    /* device, snx_cnn_param_count() floats, 16-byte aligned */
    const void *packed;     /* device, filled by snx_cnn_pack, 16-byte aligned */
    void *workspace;        /* device, >= snx_cnn_workspace_size(w, h, 1, 0), 16-byte aligned */
    size_t workspace_bytes;
} snx_cnn_model;

int32_t snx_cnn_param_count(void);
size_t snx_cnn_packed_bytes(void);
/* Scratch for a batch of `batch` frames of width x height; training != 0 also
 * keeps every activation and gradient for the backward pass. */
size_t snx_cnn_workspace_size(int32_t width, int32_t height, int32_t batch, int32_t training);
snx_status snx_cnn_pack(const float *params, void *packed, void *stream);

/* Denoise one frame: disp [height x stride] -> out [height x out_stride]. */
snx_status snx_cnn_denoise(const float *disp, int64_t stride, int32_t width, int32_t height,
                           const snx_cnn_model *model, float *out, int64_t out_stride,
                           void *stream);

/* One training step on a batch of equally sized crops:
 *   disp      device, batch x height x width (contiguous)
 *   normals   device, batch x 3 x height x width ground-truth unit normals
 *             (NaN where there is none)
 *   clean     device, batch x height x width noise-free disparity (NaN where
 *             there is none), or NULL for no fidelity term
 *   cams      host, `batch` cameras (principal point relative to each crop);
 *             batch <= 64
 * Loss = L_n + fidelity * L_f with
 *   L_n = mean over pixels with a defined normal (slope window normal_window)
 *         and a ground-truth normal of 1 - n . n_gt,
 *   L_f = mean over pixels with a valid D~ and a finite clean value of
 *         (D~ - clean)^2  (px^2; keeps D~ an unbiased disparity for z and x, y);
 * the gradient flows through the normal, the slope, the residual and the
 * network.  grad receives the parameter gradient.  step >= 1 then applies Adam
 * (moments adam_m, adam_v, bias correction for this step number) to params and
 * repacks `packed`; step == 0 only computes loss and grad.  loss_out: device
 * double[4] = (loss, number of normal pixels, L_n, L_f).  Deterministic:
 * fixed-order reductions only. */
snx_status snx_cnn_train_step(const float *disp, const float *normals, const float *clean,
                              float fidelity, const snx_camera *cams,
                              int32_t width, int32_t height, int32_t batch,
                              int32_t normal_window, float *params, void *packed, float *grad,
                              float *adam_m, float *adam_v, int32_t step, float lr,
                              float beta1, float beta2, float eps, double *loss_out,
                              void *workspace, size_t workspace_bytes, void *stream);

/* ===========================================================================
 * Model files of the learned denoiser.  A model holds the FP32 parameters (the
 * layout of snx_cnn_param_count), optionally the two Adam moments, the
 * optimiser step and a few training facts, on the host; snx_model_bind makes
 * device copies for snx_denoise / snx_pipeline / snx_plan_create.
 *
 * File layout, little-endian, version 1:
 *    0  char[4]   magic "SNXM"
 *    4  uint32    version (1)
 *    8  uint32    parameter count n (must equal snx_cnn_param_count())
 *   12  uint32    flags: bit 0 = the Adam moments follow the parameters
 *   16  int64     optimiser step
 *   24  int32     gradient window the model was trained with (0 = unknown)
 *   28  int32     training seed
 *   32  float32   weight of the fidelity term
 *   36  uint32    reserved (0)
 *   40  float32[n] parameters, then with bit 0 float32[n] first and float32[n]
 *                  second Adam moments
 *  end  uint32    CRC-32 (reflected polynomial 0xEDB88320, as zlib's crc32) of
 *                  every byte before it
 * A file of any other length, magic, version, count, flags or checksum is
 * refused with SNX_ERR_MODEL; open/read/write failures give SNX_ERR_IO.
 * These calls (except snx_model_bind) are host-only: they need no GPU.
 * ========================================================================= */
typedef struct snx_model snx_model;
typedef struct snx_model_info {
    int64_t step;
    int32_t normal_window;
    int32_t seed;
    float fidelity;
    int32_t has_moments;      /* output only: 1 if the model holds Adam moments */
} snx_model_info;

/* New model from host arrays of snx_cnn_param_count() floats (copied); adam_m
 * and adam_v both NULL (no Adam state) or both set; info may be NULL. */
snx_status snx_model_create(const float *params, const float *adam_m, const float *adam_v,
                            const snx_model_info *info, snx_model **model);
/* Reads and checks a model file; *model is NULL on failure. */
snx_status snx_model_load(const char *path, snx_model **model);
/* Writes the model to `path` atomically: to "<path>.tmp", then renamed. */
snx_status snx_model_save(const snx_model *model, const char *path);
/* Copies out the parameters, the moments (SNX_ERR_MODEL if asked for and
 * absent) and the info; each output may be NULL. */
snx_status snx_model_read(const snx_model *model, float *params, float *adam_m, float *adam_v,
                          snx_model_info *info);
/* Device copies of the parameters, packed weights and a workspace for frames up
 * to width x height, owned by the model (kept until snx_model_destroy, grown by
 * later binds); fills *view for the learned filter.  A set-up call: allocates
 * and synchronizes `stream`. */
snx_status snx_model_bind(snx_model *model, int32_t width, int32_t height, void *stream,
                          snx_cnn_model *view);
/* Frees the model and its device copies (NULL is a no-op). */
snx_status snx_model_destroy(snx_model *model);

/* ===========================================================================
 * Batch plans: many frames of uneven size through the whole path (filter or
 * learned filter, gradients, A, normals, components, point records) with one
 * persistent launch per stage over a device-side (frame, tile) work list.  The
 * first snx_plan_run on a (non-NULL) stream captures the launches in a
 * hipGraph; later runs on that stream replay it.  The plan keeps the frame
 * pointers: refill the input buffers in place between runs.  Outputs per frame
 * are bit-identical to snx_pipeline with the same parameters.
 * ========================================================================= */
typedef struct snx_frame {
    const float *disp;          /* raw disparity [height x stride]                  */
    int64_t stride;
    int32_t width, height;
    snx_camera cam;
    float *disp_dn;             /* NULL (plan-owned scratch) or [height x dn_stride]  */
    int64_t dn_stride;
    int32_t *labels;            /* [height x label_stride], final labels after a run */
    int64_t label_stride;
    snx_point *points;          /* width * height records                           */
    int32_t *num_components;    /* NULL or device int32                             */
} snx_frame;

typedef struct snx_plan snx_plan;

/* Validates every frame, picks the tile height (the autotuned one for the
 * largest frame's size class, tuning it now if snx_autotune has not run for
 * that class), allocates the device frame table and any per-frame scratch (a
 * label forest when label_stride != width, the filtered plane when disp_dn is
 * NULL, and with the learned filter the network's input filter plane mu).
 * The filter window must be 1 or 3, or mode SNX_FILTER_CNN with a model whose
 * params and packed weights are set (its workspace is not used: the network
 * runs over the tiles of every frame in one launch).
 * A set-up call (allocates, synchronizes). */
snx_status snx_plan_create(const snx_frame *frames, int32_t n,
                           const snx_denoise_params *denoise,
                           const snx_normal_params *normal,
                           const snx_component_params *comp, snx_plan **plan);
/* Runs every frame; asynchronous on `stream` (NULL: no graph capture). */
snx_status snx_plan_run(snx_plan *plan, void *stream);
snx_status snx_plan_destroy(snx_plan *plan);

/* Status name ("SNX_OK", ...); never NULL. */
const char *snx_status_string(snx_status status);
/* Message describing the calling thread's last failed call ("" if none). */
const char *snx_last_error(void);
/* Library version, major * 10000 + minor * 100 + patch. */
int32_t snx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SNX_H */
