/*
 * ivrgs.h -- C ABI of the MI355X (gfx950) editable-Gaussian rasterizer.
 *
 * The library renders editable 3D Gaussians (iVR-GS, Sec. 4.3: geometry
 * mu, q, s, o, n and shading c_v, k_a, k_d, k_s, beta) with a tile-based
 * pipeline: EWA projection with per-Gaussian Blinn-Phong shading, tile binning
 * with a depth sort, front-to-back alpha compositing, the matching backward
 * pass, and composition of basic models under edits.
 *
 * Conventions shared by every entry point
 *   - Every pointer inside a struct or passed as an array is a DEVICE pointer
 *     owned by the caller, unless the comment says "host".  The library never
 *     allocates device memory; scratch space comes from a caller workspace
 *     whose size ivrgs_workspace_size() returns.
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*).
 *   - The returned status covers host-side validation only (null pointers,
 *     sizes, unsupported settings); on an error nothing is launched.  Errors
 *     found on the device (pair capacity exceeded) are written to the device
 *     status words of ivrgs_bins and make later kernels of the same view skip.
 *   - Gaussian attributes are FP32 planes, component-major ("SoA"):
 *     plane[c * n + i] is component c of Gaussian i.
 *   - Pixel (x, y) has its centre at (x + 0.5, y + 0.5); camera axes follow
 *     OpenCV (x right, y down, z forward).
 *   - Images are planar RGBA, FP32, [job][4][height][width]; RGB is
 *     premultiplied (C + T_final * bg), A = 1 - T_final.
 */
#ifndef IVRGS_H
#define IVRGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IVRGS_OK = 0,
    IVRGS_E_INVALID = 1,     /* null pointer or negative size */
    IVRGS_E_SHAPE = 2,       /* inconsistent sizes (image, tiles, jobs) */
    IVRGS_E_CAPACITY = 3,    /* workspace or pair buffer too small (host-checked) */
    IVRGS_E_HIP = 4,         /* a HIP runtime call failed */
    IVRGS_E_UNSUPPORTED = 5  /* a setting outside the supported range */
} ivrgs_status;

/* Device status bits written by ivrgs_bin_sort into ivrgs_bins.status[1]. */
#define IVRGS_DEV_E_CAPACITY 1u  /* more (tile, Gaussian) pairs than capacity */

/* Parameter flags (ivrgs_params.flags). */
#define IVRGS_FLAG_PERSISTENT 1u  /* render kernels use the persistent (job, tile) queue */
#define IVRGS_FLAG_COUNT_EVAL 2u  /* render_fwd counts evaluated (pixel, Gaussian) pairs into
                                     status[2] and composited ones into status[3] */
#define IVRGS_FLAG_FWD_ONLY 4u    /* nothing will differentiate the render: render_fwd stores no
                                     list checkpoints and needs no workspace (unless
                                     IVRGS_FLAG_PERSISTENT), and a render_bwd with the same flag
                                     walks every tile list whole */
#define IVRGS_FLAG_DETERMINISTIC_BWD 8u
                                  /* render_bwd's gradients are the same bit for bit on every
                                     run: the per-record sums of all waves are added as 64-bit
                                     integers (order-free) at a power-of-two scale that a first
                                     walk over the same lists sets from the largest per-wave sum
                                     of each value kind (its 2^-40 is the quantum), so the
                                     backward walks the lists twice; jobs that share Gaussians
                                     add their gradients in job order (one projection-backward
                                     launch per job; a job lists a Gaussian at most once).  The
                                     workspace grows by 72 bytes per record and 36 per tile. */

/* Editable Gaussians (Sec. 4.3), device SoA planes of length n each:
 *   mean[3][n]       mu
 *   log_scale[3][n]  s = exp(log_scale)
 *   quat[4][n]       q = (w, x, y, z), normalised inside the library
 *   opacity[1][n]    o, used as given (an edit may scale it beyond 1)
 *   normal[3][n]     n, normalised inside the library
 *   color[3][n]      render-ready voxel colour c_v = c_p + delta-c; for
 *                    ivrgs_compose inputs this plane holds delta-c
 *   shade[4][n]      k_a, k_d, k_s, beta
 *   model_id[n]      basic-model index of each Gaussian (selects its light),
 *                    or NULL for model 0 */
typedef struct {
    int64_t n;
    const float *mean, *log_scale, *quat, *opacity, *normal, *color, *shade;
    const int32_t *model_id;
} ivrgs_gaussians;

/* Same layout, writable: outputs of ivrgs_compose and gradients. */
typedef struct {
    int64_t n;
    float *mean, *log_scale, *quat, *opacity, *normal, *color, *shade;
    int32_t *model_id;
} ivrgs_gaussians_mut;

/* Pinhole camera, 16 FP32 words: x_cam = R x_world + t (R row-major,
 * world -> camera); pixel = (fx x/z + cx, fy y/z + cy). */
typedef struct {
    float R[9], t[3];
    float fx, fy, cx, cy;
} ivrgs_camera;

/* Per-basic-model edit row, 16 words (Sec. 4.5 and Sec. 4.6):
 *   palette      new palette colour c_p' (recolour)
 *   opacity_scale  o' = s_o * o
 *   shade_scale, shade_bias   (k_a, k_d, k_s, beta)' = lambda * k + b
 *   light_dir    orbital (directional) light direction, world space, pointing
 *                from the surface toward the light; normalised inside
 *   headlight    nonzero: point light at the camera, l = v (Sec. 3) */
typedef struct {
    float palette[3];
    float opacity_scale;
    float shade_scale[4];
    float shade_bias[4];
    float light_dir[3];
    int32_t headlight;
} ivrgs_model_edit;

/* One render job: one camera over one list of Gaussians.  The Gaussians of
 * job j are g(k) = gauss_index ? gauss_index[gauss_begin + k]
 *                              : gauss_begin + k,  k < gauss_count,
 * and their projected records are rec_begin + k.  Jobs must not overlap in
 * records; records of all jobs form [0, n_records). */
typedef struct {
    int32_t camera;
    int32_t gauss_begin;
    int32_t gauss_count;
    int32_t rec_begin;
} ivrgs_job;

/* A batch of jobs over one Gaussian set. */
typedef struct {
    ivrgs_gaussians g;
    const int32_t *gauss_index;      /* device, or NULL */
    const ivrgs_model_edit *edits;   /* device [n_models]: light per model */
    int32_t n_models;
    const ivrgs_camera *cameras;     /* device */
    const ivrgs_job *jobs;           /* device [n_jobs] */
    int32_t n_jobs;                  /* 0 .. 65535 (a grid dimension) */
    int32_t max_job_count;           /* host-known max gauss_count over jobs */
    int64_t n_records;               /* host-known sum of gauss_count */
} ivrgs_batch;

/* Compositing constants and launch shape.  alpha_min, alpha_max, T_min: an
 * alpha below alpha_min is skipped, alpha is capped at alpha_max and the pass
 * stops before a Gaussian that would drop the transmittance below T_min.
 * lowpass: added to the diagonal of the screen covariance (px^2).  z_near:
 * Gaussians whose depth key is <= z_near are culled.  tile must be 16.
 * fwd_px / bwd_px: pixels per lane of the render kernels (1, 2 or 4; 0 picks
 * the default); they change speed, not results.  With IVRGS_FLAG_PERSISTENT
 * (set for ivrgs_bin_sort and the render calls alike) the render kernels run
 * a fixed grid that takes (job, tile) items, longest lists first, from a
 * queue that ivrgs_bin_sort builds in the workspace. */
typedef struct {
    float alpha_min, alpha_max, T_min, lowpass, z_near;
    float bg[3];
    int32_t width, height;
    int32_t tile;
    uint32_t flags;
    int32_t fwd_px, bwd_px;
    int32_t sort_chunk;              /* records per binning chunk, 0 = automatic (up to 512) */
    int32_t persist_per_cu;          /* IVRGS_FLAG_PERSISTENT: workgroups per CU, 0 = occupancy */
} ivrgs_params;

/* Projected records (device, caller-allocated, n_records entries):
 *   rec[r][16]  x, y, qa, qb, qc, opacity, r, g, b, depth key, alpha cutoff, 0,
 *               rect (two words, as below, stored as their bits), 0, 0:
 *               one 64-byte row (the array 64-byte aligned), where the 2D
 *               Gaussian at offset d = p - (x, y) is
 *               2^(qa dx^2 + qb dx dy + qc dy^2)  (log2 units), alpha =
 *               min(alpha_max, opacity * that), and the depth key is the
 *               FP32 camera-space z of the mean; ivrgs_bin_sort takes each
 *               record's rect from its row
 *   rect[r]     tile rectangle [x0, x1) x [y0, y1) packed as
 *               (x0 | y0 << 16, x1 | y1 << 16); (0, 0) if culled
 *   depth[r]    the depth key's FP32 bits (positive, finite) of a visible
 *               record, 0xFFFFFFFF if culled; ivrgs_bin_sort orders by it
 *   nonfinite   NULL, or one device int64 to which ivrgs_project adds the
 *               number of records it culls because a Gaussian parameter, or
 *               a projected value of a Gaussian with a positive-definite
 *               screen covariance, is NaN or infinite (such a Gaussian is
 *               culled and counted, never propagated); the caller clears it */
typedef struct {
    float *rec;
    uint32_t *rect;
    uint32_t *depth;
    int64_t *nonfinite;
} ivrgs_projected;

/* Tile bins (device, caller-allocated):
 *   tile_start[n_jobs * tiles + 1]  start of each tile's list in `sorted`;
 *                                   the last entry is the pair total
 *   sorted[capacity]                record ids, each tile front to back by
 *                                   (depth key, record id)
 *   status[8]                       written by the library:
 *                                   [0] the pair capacity required (the pair
 *                                   total, or, when the binning's block
 *                                   entries did not fit the workspace sized
 *                                   for the capacity, the capacity whose
 *                                   workspace holds them) and [1]
 *                                   IVRGS_DEV_E_* bits of the last
 *                                   ivrgs_bin_sort,
 *                                   [2] evaluated and [3] composited pixel-
 *                                   Gaussian pairs (IVRGS_FLAG_COUNT_EVAL),
 *                                   [4] the OR of [1] and [5] the largest [0]
 *                                   over every bin sort since the last
 *                                   ivrgs_get_error, which clears them (the
 *                                   caller zeroes [4] and [5] once when it
 *                                   allocates the word), [6] used by the
 *                                   binning, [7] reserved */
typedef struct {
    uint32_t *tile_start;
    uint32_t *sorted;
    int64_t capacity;
    int64_t *status;
} ivrgs_bins;

/* Bytes of workspace needed by ivrgs_bin_sort, ivrgs_render_fwd and
 * ivrgs_render_bwd for this batch: the depth order (two words per record,
 * twice), its digit histograms, the per-chunk block counts, the records'
 * binning fields in depth order (32 bytes per record), the block entries
 * (8 bytes each; capacity / 2, plus 2 per record and 256 per block of 4x4
 * tiles, of them) with, per 256 entries, 68 bytes of tile counts, the record
 * gradients (9 floats per record), the work queue and, with one pixel per
 * lane, no work queue and no IVRGS_FLAG_FWD_ONLY, per-pixel checkpoints at
 * up to 15 cuts of every tile's list (60 KiB per tile, used while they take
 * at most 256 MiB): the backward walks each segment of a long list in its own workgroup from the
 * state the forward stored at the cut.  capacity (>= 0) is the pair capacity
 * of the bins (the block entries grow with it).  Returns 0 for invalid
 * arguments. */
size_t ivrgs_workspace_size(const ivrgs_batch *batch, const ivrgs_params *params,
                            int64_t capacity);

/* Number of tiles per job for the given image size (ceil(W/16) * ceil(H/16)). */
int32_t ivrgs_tiles_per_job(const ivrgs_params *params);

/* Composition and editing (Sec. 4.5; light-magnitude edit in the general
 * lambda * k + b form of Sec. 4.6).  Concatenates `n_models` basic models in
 * order into `out` (out->n must equal the sum of models[m].n) and applies
 * edit row m to model m:
 *   c_v = palette[m] + delta-c,  o' = opacity_scale[m] * o,
 *   (k_a, k_d, k_s, beta)' = shade_scale[m] * (...) + shade_bias[m];
 * mean, log_scale, quat and normal are copied; out->model_id[i] = m.
 * models: HOST array of n_models structs (device planes inside);
 * edits: HOST array of n_models rows. */
ivrgs_status ivrgs_compose(const ivrgs_gaussians *models, int32_t n_models,
                           const ivrgs_model_edit *edits, ivrgs_gaussians_mut *out,
                           void *stream);

/* Projection (Sec. 3: Eq. 1, Sigma = R S S^T R^T, EWA Sigma' = J W Sigma W^T J^T)
 * and Blinn-Phong shading (Eq. 3 with I_a = I_d = c_v, I_s = white, v the unit
 * direction from the Gaussian to the camera, l = v for the headlight or the
 * model's orbital direction; Sec. 4.3) of every (job, Gaussian) into records.
 * A Gaussian is culled (empty rect) if its depth key <= z_near, its screen
 * covariance is not positive definite, opacity < alpha_min, any input is not
 * finite, or its conservative footprint misses the image. */
ivrgs_status ivrgs_project(const ivrgs_batch *batch, const ivrgs_params *params,
                           ivrgs_projected *out, void *stream);

/* Tile binning and depth sort ("sorted by depth", Sec. 3): for each job and
 * 16x16 tile, the list of records whose rect covers the tile and whose
 * footprint {alpha >= alpha_min} can reach one of the tile's pixel centres
 * (a conservative test: the exponent's maximum over the tile's pixel box,
 * with margins for FP32 rounding), ordered by (depth key, record id).  The
 * records are put in depth order first and binned in that order, so the
 * lists need no sort of their own: first into blocks of 4x4 tiles (an
 * entry per overlapped block with the mask of its tiles the footprint
 * reaches), then from each block's entries into its tiles' lists.
 * params->sort_chunk is the number of records per binning chunk (rounded up
 * to a multiple of 64; 0 picks a power of two up to 512 that gives about
 * 1024 chunks per batch); it does not change the result.  Writes
 * bins->tile_start, bins->sorted and bins->status.  Returns IVRGS_E_SHAPE
 * if a job has more blocks than the binning's per-block LDS counters hold
 * (about 4,700 blocks, 4,300 x 4,300 pixels, on a 160 KiB device).  If the
 * pair total exceeds bins->capacity (or the block entries exceed the
 * workspace sized for it), status[1] gets IVRGS_DEV_E_CAPACITY, status[0]
 * the capacity required, and the lists are not written (render calls then
 * leave their outputs untouched). */
ivrgs_status ivrgs_bin_sort(const ivrgs_batch *batch, const ivrgs_params *params,
                            const ivrgs_projected *proj, ivrgs_bins *bins,
                            void *workspace, size_t workspace_bytes, void *stream);

/* Size of the device scratch array behind ivrgs_bin_sort_noalloc (64 MiB).
 * Every device that loads the library holds one until the process ends. */
#define IVRGS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* ivrgs_bin_sort for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result (tile_start, sorted, status), with the
 * binning scratch in a static device array of IVRGS_NOALLOC_SCRATCH_BYTES
 * instead of a caller workspace.  The caller still passes the projection
 * and the bins.  The call allocates nothing; its first call on a device
 * looks up that device's array (do it once outside graph capture).
 * The scratch takes 16 bytes per record for the depth order, 32 per record
 * for the binning fields, the digit histograms, the per-chunk block counts
 * (4 bytes per block of 4x4 tiles per chunk of params->sort_chunk records)
 * and the block entries with their tile counts (about 8.3 bytes per entry;
 * capacity / 2, plus 2 per record and 256 per block, of them);
 * IVRGS_E_CAPACITY if that exceeds IVRGS_NOALLOC_SCRATCH_BYTES (nothing is
 * launched), IVRGS_E_UNSUPPORTED with IVRGS_FLAG_PERSISTENT (the render
 * calls read that launch's work queue from their own workspace).  A render
 * that follows needs no workspace from this call: with
 * IVRGS_FLAG_FWD_ONLY, ivrgs_render_fwd takes none at all.  All calls on
 * one device share the array, which keeps the last call's contents; calls
 * that overlap on one device (concurrent streams or threads) race. */
ivrgs_status ivrgs_bin_sort_noalloc(const ivrgs_batch *batch, const ivrgs_params *params,
                                    const ivrgs_projected *proj, ivrgs_bins *bins, void *stream);

/* Front-to-back alpha compositing (Eq. 2): per pixel C = sum T_i alpha_i c_i,
 * T_i = prod_{j<i} (1 - alpha_j).  out_rgba: [n_jobs][4][H][W].  out_maxw:
 * [n_records] or NULL; if given it must be zeroed by the caller and receives,
 * per record, the largest T*alpha over its composited pixels (culling labels).
 * The workspace is required when the batch uses list checkpoints (see
 * ivrgs_workspace_size) or the persistent launch; the checkpoints it stores
 * there are what a following ivrgs_render_bwd reads. */
ivrgs_status ivrgs_render_fwd(const ivrgs_batch *batch, const ivrgs_params *params,
                              const ivrgs_projected *proj, const ivrgs_bins *bins,
                              float *out_rgba, float *out_maxw,
                              void *workspace, size_t workspace_bytes, void *stream);

/* Backward of ivrgs_project + ivrgs_render_fwd: the gradients of the
 * compositing of Eq. 2 and of the splat projection (Sec. 3) that the
 * gradient-based training of the base and editable Gaussians (Sec. 4.2, 4.3;
 * appendix A, Adam on L1 + SSIM) and the inverse exploration (Sec. 4.6)
 * descend.  Recomputes the per-pixel
 * compositing front to back from out_rgba (nothing per pixel is stored by the
 * forward) and returns dL/d(parameters) for upstream dL/dRGBA (dl_drgba, same
 * layout as out_rgba).  grads: planes of length batch->g.n (model_id unused);
 * the callee zeroes them.  Gaussians shared by several jobs accumulate.
 * Must follow the ivrgs_render_fwd that produced out_rgba with the same
 * batch, params, bins and workspace (it reads the list checkpoints that call
 * stored). */
ivrgs_status ivrgs_render_bwd(const ivrgs_batch *batch, const ivrgs_params *params,
                              const ivrgs_projected *proj, const ivrgs_bins *bins,
                              const float *out_rgba, const float *dl_drgba,
                              ivrgs_gaussians_mut *grads,
                              void *workspace, size_t workspace_bytes, void *stream);

/* Gradients of the edit parameters that inverse volume exploration learns
 * for each basic model (Sec. 4.6): the palette colour c_p, the opacity scale
 * s_o and the light-magnitude transform lambda * (k_a, k_d, k_s, beta) + b
 * of the composition c_v = c_p + delta-c, o' = s_o o, k' = lambda k + b
 * (ivrgs_compose).  grads: the gradients of the composed set (as written by
 * ivrgs_render_bwd, composition order); models: the source models of the
 * composition (device planes; only opacity and shade are read).  Writes
 * out_edit_grad[n_models][12] (device, caller-allocated; overwritten):
 *   [0..2]  dL/dc_p   = sum over the model's Gaussians of dL/dc_v
 *   [3]     dL/ds_o   = sum dL/do' * o
 *   [4..7]  dL/dlambda = sum dL/dk' * k   (per component)
 *   [8..11] dL/db     = sum dL/dk'
 * Sums are accumulated with float atomics (order unspecified). */
ivrgs_status ivrgs_compose_bwd(const ivrgs_gaussians *models, int32_t n_models,
                               const ivrgs_gaussians_mut *grads, float *out_edit_grad, void *stream);

/* Gradient of the loss with respect to each model's orbital light direction
 * (the unnormalised light_dir of its edit row; Sec. 4.6 learns the light
 * direction; Eq. 3 uses it normalised): out_light_grad[n_models][3] (device,
 * caller-allocated; overwritten).  Must follow ivrgs_render_bwd for the same
 * batch, params, projection and workspace: it reads the record gradients
 * that call leaves in the workspace.  Headlight models get zeros. */
ivrgs_status ivrgs_light_bwd(const ivrgs_batch *batch, const ivrgs_params *params,
                             const ivrgs_projected *proj, float *out_light_grad,
                             const void *workspace, size_t workspace_bytes, void *stream);

/* Kernel timing (benchmark instrumentation).  ivrgs_timing_enable(kinds)
 * selects the kernel kinds to time (bit k for kind k, IVRGS_TIMING_ALL for
 * every kind, 0 to stop) and clears the sums.  Every launch of a selected
 * kind is then bracketed by a pair of HIP events recorded on its launch
 * stream (two event records per launch: timing every kind slows a short
 * step measurably, so time only what is needed).  ivrgs_timing_read()
 * waits for those events and returns, per kernel kind, the summed
 * milliseconds and the number of launches since the last enable.  Kinds:
 * 0 project, 1 tile counts (per-chunk counts, column and tile scans, work
 * queue), 2 scatter, 3 depth order, 4 render_fwd, 5 render_bwd,
 * 6 project_bwd, 7 compose, 8 fills, 9 cull, 10 edit and light gradients
 * and the exploration step, 11 VQ (k-means, assignment, quantised compose),
 * 12 SH colour and its backward, 13 auxiliary maps and their backward.
 * Process-wide state; not for concurrent callers. */
#define IVRGS_TIMING_KINDS 14
#define IVRGS_TIMING_ALL 0x3FFFu
void ivrgs_timing_enable(uint32_t kinds);
int32_t ivrgs_timing_read(double *ms, int64_t *launches);

/* Learned culler (device weights): an MLP 16 -> 64 -> 64 -> 1 with ReLU on
 * the features (mean 3, log_scale 3, opacity 1, unit direction from the
 * Gaussian to the camera centre 3, then 6 zeros); any input normalisation is
 * folded into w1/b1.  w1 [64][16] and w2 [64][64] hold BF16 bit patterns
 * (row = output unit; both 8-byte aligned, IVRGS_E_INVALID otherwise); b1,
 * b2, w3 [64] and b3 are FP32.  A Gaussian is kept
 * when its logit >= threshold. */
typedef struct {
    const uint16_t *w1;
    const float *b1;
    const uint16_t *w2;
    const float *b2;
    const float *w3;
    float b3;
    float threshold;
} ivrgs_culler;

/* Evaluates the culler for every Gaussian of g (n of them) seen from
 * cameras[camera], writes the kept ids in ascending order to out_index
 * ([n], device) and their count into jobs[job].gauss_count (device), so
 * that ivrgs_project / ivrgs_bin_sort / ivrgs_render_* over a batch with
 * gauss_index = out_index and that job (gauss_begin = 0, host-side counts
 * set to n as upper bounds) render only the survivors, with no host sync.
 * out_logit: [n] or NULL.  workspace: ivrgs_cull_workspace_size(n) bytes.
 * This is the learned-culling extension of the rasterizer (no paper passage:
 * the label it predicts is the compositing weight of Eq. 2 reaching 1/255). */
size_t ivrgs_cull_workspace_size(int64_t n);
ivrgs_status ivrgs_cull(const ivrgs_gaussians *g, const ivrgs_camera *cameras, int32_t camera,
                        const ivrgs_culler *mlp, int32_t *out_index, ivrgs_job *jobs, int32_t job,
                        float *out_logit, void *workspace, size_t workspace_bytes, void *stream);

/* Same as ivrgs_compose, with the edit table in DEVICE memory (edits:
 * device [n_models]; models: host array as there).  For loops that update the
 * edit rows on the GPU (ivrgs_explore_step) without a host round trip. */
ivrgs_status ivrgs_compose_dev(const ivrgs_gaussians *models, int32_t n_models,
                               const ivrgs_model_edit *edits, ivrgs_gaussians_mut *out, void *stream);

/* Inverse volume exploration (Sec. 4.6): with the Gaussians frozen, learn
 * per basic model the palette colour c_p and the opacity scale s_o, and for
 * the composed model one light-magnitude transform lambda, b (R^4 each,
 * shared by all models) and one orbital light direction given by its polar
 * and azimuthal angles, d = (sin t cos p, sin t sin p, cos t) in world space.
 * The optimiser is Adam (Kingma and Ba, 2015).
 *
 * State (device float array, ivrgs_explore_state_words(n_models) words,
 * caller-allocated and initialised; K = n_models, n = 4K + 10):
 *   [0, n)    parameters: palette[K][3], s_o[K], lambda[4], b[4], t, p
 *   [n, 2n)   Adam first moments (start at 0)
 *   [2n, 3n)  Adam second moments (start at 0)
 *   [3n]      completed steps (starts at 0)
 * learn: bit 0 palette, bit 1 opacity scale, bit 2 lambda and b, bit 3 light
 * angles; parameters of an unset group keep their values. */
typedef struct {
    float lr, beta1, beta2, eps;
    uint32_t learn;
} ivrgs_explore_opts;

int64_t ivrgs_explore_state_words(int32_t n_models);

/* One Adam step of the exploration parameters from the gradients of one
 * backward: edit_grad (device [K][12], ivrgs_compose_bwd) and light_grad
 * (device [K][3], ivrgs_light_bwd, or NULL when no model has an orbital
 * light).  The shared lambda, b and light angles take the sums over the
 * models; the angles chain through d(t, p).  Then rewrites the edit table
 * (device [K]) from the parameters: palette, opacity_scale, shade_scale =
 * lambda, shade_bias = b, and light_dir = d(t, p) for the models whose
 * headlight word is 0 (headlight words and headlight models' light_dir are
 * left as they are).  edit_grad may be NULL when learn has none of bits
 * 0-2.  learn == 0 only rewrites the edit table (no step is counted and the
 * gradients are not read): the way to initialise it.  One
 * workgroup; all arrays on the device. */
ivrgs_status ivrgs_explore_step(const float *edit_grad, const float *light_grad, int32_t n_models,
                                const ivrgs_explore_opts *opts, float *state, ivrgs_model_edit *edits,
                                void *stream);

/* ---- Vector quantisation (Sec. 4.4) ------------------------------------
 * k-means gives one codebook per attribute over all the Gaussians of a basic
 * model; a vector attribute shares one scalar codebook, with one index per
 * component; mean and normal stay exact.  The attributes (Sec. 4.3) are
 * log-scale, rotation, opacity, offset colour delta-c, and the shading terms
 * k_a, k_d, k_s, beta: eight codebooks.  Codebook size k is 1..256 (one byte
 * per index).  The paper gives no sizes or schedule; the readings here:
 * initial centroids at the centres of k equal cells of [min, max] of the
 * finite values (lo + (j + 1/2) * ((hi - lo) / k), FP32); each Lloyd
 * iteration assigns every value to its nearest centroid (|x - c| in FP32,
 * the lowest index on ties), moves each non-empty cluster's centroid to the
 * FP64 mean of its values rounded to FP32 (an empty cluster keeps its
 * centroid) and sorts the codebook ascending; the indices are the assignment
 * to the final codebook.  Non-finite values take index 0 and move no
 * centroid. */

/* A quantised basic model.  Index planes, component-major [15][n] uint8:
 * log_scale 0-2, quat 3-6, opacity 7, delta-c 8-10, k_a 11, k_d 12, k_s 13,
 * beta 14; codebooks [8][k] FP32: log_scale, quat, opacity, delta-c, k_a,
 * k_d, k_s, beta (index plane p reads codebook 0,0,0,1,1,1,1,2,3,3,3,4,5,6,7).
 * An index >= k reads entry k - 1.  All pointers device. */
typedef struct {
    int64_t n;
    const float *mean;      /* [3][n], exact */
    const float *normal;    /* [3][n], exact */
    const uint8_t *index;   /* [15][n] */
    const float *codebook;  /* [8][k] */
    int32_t k;              /* 1..256 */
} ivrgs_vq_model;

/* Workspace bytes of ivrgs_vq_fit for n values and codebook size k (per
 * workgroup FP64 sums and counts of every centroid, and value ranges). */
size_t ivrgs_vq_workspace_size(int64_t n, int32_t k);

/* k-means codebook of one attribute (values: device [n] FP32, all the
 * components of the attribute back to back) with `iters` Lloyd iterations
 * (>= 0) from the cell-centre initialisation, then the index of every value
 * against the final codebook.  Outputs: codebook (device [k], ascending)
 * and index (device [n] uint8).  workspace: device, at least
 * ivrgs_vq_workspace_size(n, k) bytes.  n = 0 writes an all-zero codebook.
 * Returns IVRGS_E_INVALID for k outside 1..256, iters < 0 or a null pointer
 * (values and index may be null when n = 0), IVRGS_E_CAPACITY for a short
 * workspace. */
ivrgs_status ivrgs_vq_fit(const float *values, int64_t n, int32_t k, int32_t iters, float *codebook,
                          uint8_t *index, void *workspace, size_t workspace_bytes, void *stream);

/* One attribute of ivrgs_vq_fit_batch: values device [n] FP32, outputs
 * codebook device [k] and index device [n] uint8, as for ivrgs_vq_fit. */
typedef struct {
    const float *values;
    int64_t n;
    float *codebook;
    uint8_t *index;
} ivrgs_vq_book;

/* Workspace bytes of ivrgs_vq_fit_batch: the sum over the books of
 * ivrgs_vq_workspace_size(n, k). */
size_t ivrgs_vq_fit_batch_workspace_size(const ivrgs_vq_book *books, int32_t count, int32_t k);

/* ivrgs_vq_fit of `count` attributes (books: host array) with one codebook
 * size k and iteration count: each result equals that of ivrgs_vq_fit on
 * the attribute alone, bit for bit.  Up to 8 attributes share each launch
 * (the eight codebooks of a model in one), so a fit costs 2 iters + 3
 * launches per 8 attributes instead of per attribute.  Errors as for
 * ivrgs_vq_fit, checked for every book before any launch. */
ivrgs_status ivrgs_vq_fit_batch(const ivrgs_vq_book *books, int32_t count, int32_t k, int32_t iters,
                                void *workspace, size_t workspace_bytes, void *stream);

/* Nearest-centroid index of each value (the assignment step of the fit):
 * argmin_j |x - c_j| in FP32, the lowest index on ties, 0 for non-finite
 * values.  Any codebook order is accepted (an ascending one takes a binary
 * search, any other a full scan).  values: device [n]; codebook: device
 * [k], k in 1..256; index: device [n] uint8. */
ivrgs_status ivrgs_vq_assign(const float *values, int64_t n, const float *codebook, int32_t k,
                             uint8_t *index, void *stream);

/* Composition and editing of quantised models (Sec. 4.5: each model is
 * decompressed from its indices and codebooks and appended): the same
 * output and edits as ivrgs_compose, with every quantised attribute read
 * through its codebook inside the kernel.  models: HOST array of n_models
 * structs; edits: HOST array of n_models rows; out->n must equal the sum of
 * models[m].n. */
ivrgs_status ivrgs_vq_compose(const ivrgs_vq_model *models, int32_t n_models, const ivrgs_model_edit *edits,
                              ivrgs_gaussians_mut *out, void *stream);

/* ---- Auxiliary maps (Eq. 5; Sec. 4.3) --------------------------------------
 * The training losses of the basic models read, besides the image, maps
 * composited with the image's weights T_i alpha_i: the depth and normal maps
 * of Eq. 5 (normal consistency) and the offset-colour and shading-term maps
 * of Sec. 4.3 (sparsity and bilateral smoothness).  Channel 0 is the
 * camera-space depth of each record (its depth key, row 3 of R applied to
 * the mean plus t); channels 1 .. n_attr composite caller attributes
 * (0 <= n_attr <= 15; for example the unit normal, delta-c, k_a, k_d, k_s,
 * beta).  The attributes are per-Gaussian rows: attr[g * S + c] with the row
 * stride S = n_attr rounded up to a multiple of 4 (the pad entries are not
 * read), 16-byte aligned, so that a record's attributes load as whole
 * vectors.  No background term.  Both calls follow ivrgs_bin_sort of the
 * same batch and params (the composited pairs are exactly the image's). */

/* attr: device [batch->g.n][S]; out_aux: device [n_jobs][1 + n_attr][H][W],
 * written.  IVRGS_E_INVALID if attr is not 16-byte aligned. */
ivrgs_status ivrgs_render_aux_fwd(const ivrgs_batch *batch, const ivrgs_params *params,
                                  const ivrgs_projected *proj, const ivrgs_bins *bins, const float *attr,
                                  int32_t n_attr, float *out_aux, void *stream);

/* Backward for dL/d(maps) grad_aux (same layout as the maps; aux: the
 * forward's maps).  ADDS into grad_attr (device [g.n][S], the rows of attr;
 * the pad entries are left alone) the attribute
 * gradients and into grads the geometry gradients: through alpha (mean,
 * log_scale, quat, opacity, by the projection backward, accumulated) and
 * through the depth (mean).  The caller clears both first.  workspace: the
 * render workspace of this batch (its record-gradient rows are reused). */
ivrgs_status ivrgs_render_aux_bwd(const ivrgs_batch *batch, const ivrgs_params *params,
                                  const ivrgs_projected *proj, const ivrgs_bins *bins, const float *attr,
                                  int32_t n_attr, const float *aux, const float *grad_aux, float *grad_attr,
                                  ivrgs_gaussians_mut *grads, void *workspace, size_t workspace_bytes,
                                  void *stream);

/* ---- Attribute rows of the editable stage (Sec. 4.3; Eq. 5) ---------------
 * The rows that the maps of the editable-stage losses composite: per
 * Gaussian g, attr[g * 12 + c] holds the unit normal (c = 0..2: the normal
 * plane divided by its Euclidean length, the length clamped below at
 * 1e-12), delta-c (c = 3..5: the colour plane of a basic model), k_a, k_d,
 * k_s and beta (c = 6..9: the shade plane), then two zero pad entries; that
 * is the layout ivrgs_render_aux_fwd takes with n_attr = 10.  Planes are
 * device [k][n] (component-major), attr device [n][12], 16-byte aligned.
 * n = 0 is a no-op; IVRGS_E_INVALID for n < 0, a null pointer or an
 * unaligned attr. */
ivrgs_status ivrgs_editable_attr_fwd(const float *normal, const float *color, const float *shade, int64_t n,
                                     float *attr, void *stream);

/* Backward of the rows for dL/d(rows) grad_attr (device [n][12], 16-byte
 * aligned; the pad entries are not read): ADDS into grad_normal [3][n]
 * (the normalisation's derivative, (I - u u^T) / length with u the unit
 * normal, or I / 1e-12 where the length is at the floor), grad_color [3][n]
 * and grad_shade [4][n].  normal: the plane the rows were made from. */
ivrgs_status ivrgs_editable_attr_bwd(const float *normal, int64_t n, const float *grad_attr, float *grad_normal,
                                     float *grad_color, float *grad_shade, void *stream);

/* The image and the maps in one walk over the lists (the forward of a
 * training step that reads both; Eq. 2 and Eq. 5): writes out_rgba exactly as
 * ivrgs_render_fwd with one pixel per lane would (the same image, and the
 * same list checkpoints in the workspace for the backward) and out_aux as
 * ivrgs_render_aux_fwd (same layout and meaning; attr as there).  The
 * workspace is needed when the render workspace holds checkpoints (long
 * lists); IVRGS_E_CAPACITY if it is missing or small then.  IVRGS_E_INVALID
 * for n_attr outside 0..15, a null output or unaligned attr. */
ivrgs_status ivrgs_render_fwd_aux(const ivrgs_batch *batch, const ivrgs_params *params, const ivrgs_projected *proj,
                                  const ivrgs_bins *bins, const float *attr, int32_t n_attr, float *out_rgba,
                                  float *out_aux, void *workspace, size_t workspace_bytes, void *stream);

/* The image's backward and the maps' backward in one call (the training
 * step of the editable stage differentiates both; Eq. 2 and Eq. 5): the
 * result of ivrgs_render_bwd for dl_drgba plus that of ivrgs_render_aux_bwd
 * for grad_aux, from one walk over the lists (the image's colour is three
 * more channels of the maps' walk), summed into one set of record gradients
 * that one projection backward takes to grads.  grads is WRITTEN as by ivrgs_render_bwd (no
 * clearing needed); grad_attr (device [g.n][S], S = n_attr rounded up to a
 * multiple of 4) is cleared, then written, pad entries included.  Arguments
 * as in those two calls, over the same batch, params, bins and workspace;
 * IVRGS_E_UNSUPPORTED with IVRGS_FLAG_DETERMINISTIC_BWD (the maps' sums are
 * float atomics). */
ivrgs_status ivrgs_render_bwd_aux(const ivrgs_batch *batch, const ivrgs_params *params, const ivrgs_projected *proj,
                                  const ivrgs_bins *bins, const float *out_rgba, const float *dl_drgba,
                                  const float *attr, int32_t n_attr, const float *aux, const float *grad_aux,
                                  float *grad_attr, ivrgs_gaussians_mut *grads, void *workspace,
                                  size_t workspace_bytes, void *stream);

/* ---- SSIM term of the photometric loss (Sec. 4.2; appendix weights) -------
 * Structural similarity of an image x against a target y, both device
 * [channels][height][width] float32, contiguous: per channel, every valid
 * 11x11 window (its top-left corner in [0, height - 10) x [0, width - 10))
 * with Gaussian weights of sigma 1.5 normalised to 1, and the constants
 * C1 = 0.01^2, C2 = 0.03^2 (values in [0, 1]); the result is the mean over
 * windows and channels.  height and width must be at least 11
 * (IVRGS_E_SHAPE otherwise).  The forward stores per-window partial
 * derivatives in the workspace, which the backward reads: keep the
 * workspace unchanged between the two calls.  Deterministic. */
size_t ivrgs_ssim_workspace_size(int32_t channels, int32_t height, int32_t width);

/* out_mean: device float, the mean SSIM. */
ivrgs_status ivrgs_ssim_fwd(const float *x, const float *y, int32_t channels, int32_t height, int32_t width,
                            float *out_mean, void *workspace, size_t workspace_bytes, void *stream);

/* grad_mean: device float, dL/d(mean SSIM); grad_x: device, the layout of x,
 * overwritten with dL/dx.  The target gets no gradient. */
ivrgs_status ivrgs_ssim_bwd(const float *x, const float *y, int32_t channels, int32_t height, int32_t width,
                            const float *grad_mean, float *grad_x, const void *workspace, size_t workspace_bytes,
                            void *stream);

/* The L1 term of the photometric loss (Sec. 4.2; the headline training step
 * and the base stage weight it alone or with D-SSIM): mean |x - y| over n
 * values (device float arrays; any layout, the same for both), FP32
 * differences summed in FP64 per workgroup slice, the slices added in a
 * fixed order (deterministic).  out_mean: one device float.  Workspace:
 * ivrgs_l1_workspace_size(n) bytes of device memory (0 for n <= 0).
 * IVRGS_E_SHAPE for n <= 0 or n > 2^40, IVRGS_E_CAPACITY for a small
 * workspace. */
size_t ivrgs_l1_workspace_size(int64_t n);
ivrgs_status ivrgs_l1_fwd(const float *x, const float *y, int64_t n, float *out_mean, void *workspace,
                          size_t workspace_bytes, void *stream);

/* grad_x[i] = sign(x[i] - y[i]) * grad_mean / n (device; grad_mean one device
 * float, dL/d(mean)); sign(0) = 0 and a NaN difference gives NaN.  One
 * launch, no workspace. */
ivrgs_status ivrgs_l1_bwd(const float *x, const float *y, int64_t n, const float *grad_mean, float *grad_x,
                          void *stream);

/* Gradient of the photometric loss L = (1 - lam) mean|x - y| + lam (1 - SSIM)
 * with respect to x (Sec. 4.2 names the L1 + D-SSIM combination, the
 * appendix weights it 0.8 / 0.2; inverse exploration, Sec. 4.6, fits its
 * parameters with the same combination).  mean|x - y| is over all
 * channels x height x width values, with sign(0) = 0; SSIM as above.
 * Needs the workspace of an ivrgs_ssim_fwd call on the same x and y, left
 * unchanged since.  lam in [0, 1] (IVRGS_E_INVALID otherwise); grad_x:
 * device, the layout of x, overwritten.  One launch; deterministic. */
ivrgs_status ivrgs_photometric_grad(const float *x, const float *y, int32_t channels, int32_t height,
                                    int32_t width, float lam, float *grad_x, const void *workspace,
                                    size_t workspace_bytes, void *stream);

/* Both means of the photometric loss in one pass over x and y (Sec. 4.2):
 * out_means (device float[2]) gets the mean SSIM as above and, in [1], the
 * mean |x - y| over all channels x height x width values (per workgroup an
 * FP32 sum over its pixels, the workgroups added in FP64 in a fixed order:
 * deterministic).  Workspace: ivrgs_photometric_workspace_size bytes (that
 * of ivrgs_ssim_fwd plus one float per workgroup; 0 for invalid shapes),
 * laid out so that ivrgs_photometric_grad and ivrgs_photometric_grad_dev
 * take it as an SSIM forward's.  Errors as ivrgs_ssim_fwd. */
size_t ivrgs_photometric_workspace_size(int32_t channels, int32_t height, int32_t width);
ivrgs_status ivrgs_photometric_fwd(const float *x, const float *y, int32_t channels, int32_t height, int32_t width,
                                   float *out_means, void *workspace, size_t workspace_bytes, void *stream);

/* Gradient with respect to x of weights[0] * (mean SSIM) + weights[1] *
 * (mean |x - y|), weights device float[2] (a training loop's upstream
 * gradient times the loss weights, never read on the host): the L1 + D-SSIM
 * photometric loss of Sec. 4.2 (ivrgs_photometric_grad with lam) is weights
 * (-lam, 1 - lam).  Same
 * workspace, layout and error behaviour as ivrgs_photometric_grad; grad_x
 * overwritten.  One launch. */
ivrgs_status ivrgs_photometric_grad_dev(const float *x, const float *y, int32_t channels, int32_t height,
                                        int32_t width, const float *weights, float *grad_x, const void *workspace,
                                        size_t workspace_bytes, void *stream);

/* ---- Training regularisers on the rendered maps (Eq. 5-7, Sec. 4.3) -------
 * The editable stage's regularisers of one view (the appendix weights them
 * 0.01 each, the opacity L1 0.1):
 *   [0] normal consistency (Eq. 6): mean over valid pixels of
 *       || N / max(|N|, 1e-12) - N~ ||_2, N the composited normal map and N~
 *       the pseudo-normal of the depth map under local planarity (Eq. 5; held
 *       fixed, no gradient through it);
 *   [1] sparsity of the offset colour (Sec. 4.3): mean |delta-c map|;
 *   [2] bilateral smoothness (Eq. 7): mean over the four shading-term maps and
 *       pixels of |K(x+1) - K(x)| exp(-mean_c |c(x+1) - c(x)|) plus the same
 *       in y, each averaged over its own (H (W-1) or (H-1) W) differences,
 *       c the target colour;
 *   [3] opacity L1 (Sec. 4.3): mean |o| over the Gaussians.
 * The pseudo-normal: at pixels with alpha > 0.5, d = depth / alpha;
 * P = d ((x + 1/2 - cx) / fx, (y + 1/2 - cy) / fy, 1) in camera space; N~ =
 * the normalised cross product of the central differences of P in x and y,
 * negated if N~ . P > 0 (it faces the camera), then R^T N~ (world space).  A
 * pixel is valid when it and its four neighbours have alpha > 0.5 and it is
 * not on the border.  |x| has the derivative sign(x) (0 at 0).  A NULL map
 * drops its term (0); with no valid pixel term [0] is 0. */
typedef struct {
    const float *depth;    /* [H][W] alpha-weighted depth map (channel 0 of the aux maps) */
    const float *alpha;    /* [H][W] alpha map (channel 3 of the image) */
    const float *normal;   /* [3][H][W] composited normal map, or NULL */
    const float *delta_c;  /* [3][H][W] offset-colour map, or NULL */
    const float *shade;    /* [4][H][W] k_a, k_d, k_s, beta maps, or NULL */
    const float *target;   /* [3][H][W] target colour; required with shade */
    const float *opacity;  /* [n_gauss] opacities, or NULL */
    int64_t n_gauss;
    int32_t height, width; /* each at least 3 */
} ivrgs_reg_maps;

/* Bytes of workspace ivrgs_reg_fwd needs (0 for invalid maps). */
size_t ivrgs_reg_workspace_size(const ivrgs_reg_maps *maps);

/* out_terms: device float[5], written: the four terms above and, in [4], the
 * number of valid pixels.  out_pseudo_normal: device [3][H][W] or NULL,
 * written with N~ (0 at invalid pixels).  camera: HOST struct.  The sums are
 * reduced in a fixed order (deterministic).  Two launches. */
ivrgs_status ivrgs_reg_fwd(const ivrgs_reg_maps *maps, const ivrgs_camera *camera, float *out_terms,
                           float *out_pseudo_normal, void *workspace, size_t workspace_bytes, void *stream);

/* Gradients of sum_k grad_terms[k] * term_k (grad_terms: device float[4];
 * terms: the out_terms of the forward on the same maps) with respect to the
 * normal map, the offset-colour map, the shading maps and the opacities;
 * each output (device, the layout of its input, or NULL to skip) is
 * overwritten.  The depth, alpha and target get no gradient; grad_depth
 * (device [H][W], or NULL) is written with zeros, for a caller whose maps'
 * gradient is one buffer with the depth channel in it.  One launch. */
ivrgs_status ivrgs_reg_bwd(const ivrgs_reg_maps *maps, const ivrgs_camera *camera, const float *terms,
                           const float *grad_terms, float *grad_normal, float *grad_delta_c, float *grad_shade,
                           float *grad_opacity, float *grad_depth, void *stream);

/* ---- SH colour (base 3DGS, Sec. 3 and Sec. 4.2) ---------------------------
 * The base model's view-dependent colour is parameterised by spherical-
 * harmonic coefficients, as in the original 3DGS; the paper gives no degree
 * or convention.  Readings: degree L in 0..3, K = (L + 1)^2 coefficients per
 * channel; the real basis from the complex harmonics with the Condon-Shortley
 * phase (Y_l^0; sqrt(2) Re Y_l^m for m > 0; sqrt(2) Im Y_l^|m| for m < 0),
 * ordered by band l, then m = -l .. l; the direction d = (mean - C) / |mean -
 * C| from the camera centre C = -R^T t (d = 0 for a mean on the centre);
 * colour_c = max(sum_k Y_k(d) sh[k][c] + 1/2, 0) (a NaN passes through).
 * The result is a colour plane for the rest of the path: with shading terms
 * (k_a, k_d, k_s) = (1, 0, 0) projection passes it through unchanged. */

/* sh: device [K][3][n] (coefficient-major planes); mean: device [3][n];
 * camera: HOST struct; color: device [3][n], written.  Returns
 * IVRGS_E_INVALID for a degree outside 0..3, a negative n or a null pointer
 * (none is read when n = 0). */
ivrgs_status ivrgs_sh_color(const float *sh, int32_t degree, const float *mean, int64_t n,
                            const ivrgs_camera *camera, float *color, void *stream);

/* Backward of ivrgs_sh_color for dL/dcolour (device [3][n]): grad_sh
 * (device [K][3][n]) is written with Y_k(d) g_c, where g_c = dL/dcolour_c
 * unless the colour is clamped (raw colour <= 0: g_c = 0); when grad_mean
 * (device [3][n]) is not NULL, the mean's gradient through the direction
 * (tangent to the sphere of directions, over |mean - C|) is ADDED into it,
 * so it can follow the projection backward's mean gradient. */
ivrgs_status ivrgs_sh_color_bwd(const float *sh, int32_t degree, const float *mean, int64_t n,
                                const ivrgs_camera *camera, const float *grad_color, float *grad_sh,
                                float *grad_mean, void *stream);

/* sizeof of the ABI structs, for binding checks: which = 0 gaussians,
 * 1 camera, 2 model_edit, 3 job, 4 batch, 5 params, 6 projected, 7 bins,
 * 8 culler, 9 explore_opts, 10 vq_model, 11 vq_book, 12 reg_maps; -1 for
 * any other value. */
int32_t ivrgs_struct_size(int32_t which);

/* Device-side errors: waits for `stream`, then reads the device status
 * words of every ivrgs_bin_sort on these bins since the previous call: the
 * OR of their IVRGS_DEV_E_* bits (bins->status[4] | status[1]; 0 when none)
 * into *device_error, and the largest pair count any of them required
 * (max of status[5] and status[0]) into *pairs_required when not NULL; then
 * clears status[4] and status[5], so a caller that runs many iterations
 * without reading the pair count back checks them all with one call.  The
 * other entry points return host-side validation only and never wait. */
ivrgs_status ivrgs_get_error(const ivrgs_bins *bins, void *stream, int64_t *device_error,
                             int64_t *pairs_required);

/* Human-readable name of a status code. */
const char *ivrgs_status_string(ivrgs_status s);

#ifdef __cplusplus
}
#endif
#endif /* IVRGS_H */
