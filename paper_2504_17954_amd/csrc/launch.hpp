// Host-side launchers implemented in the kernel translation units.
#pragma once

#include "common.hpp"

namespace ivrgs {

// Kernel-timing hooks (no-ops unless timing is enabled).
enum TimingKind { TK_PROJECT = 0, TK_COUNT, TK_SCATTER, TK_SORT, TK_FWD, TK_BWD, TK_PROJECT_BWD,
                  TK_COMPOSE, TK_FILL, TK_CULL, TK_EDIT_BWD, TK_VQ, TK_SH, TK_AUX, TK_KINDS };
void timing_begin(int kind, hipStream_t s);
void timing_end(int kind, hipStream_t s);

struct TimedScope {
    int kind;
    hipStream_t s;
    TimedScope(int k, hipStream_t st) : kind(k), s(st) { timing_begin(kind, s); }
    ~TimedScope() { timing_end(kind, s); }
};

struct BinWork {
    uint32_t *key[2], *val[2];  // depth-order ping-pong, one word per record each
    uint32_t *hist;             // depth_sort_hist_words
    uint32_t *rng;              // 2 * n_jobs
    uint32_t *counts;           // [job][chunk][block]: block overlaps per chunk
    uint32_t *part;             // col_part_words: per-segment column sums
    uint4 *pay;                 // 2 per record: binning fields in depth order
    uint32_t *sb_len;           // n_jobs * blocks + 1: entries per block
    uint32_t *sb_start;         // n_jobs * blocks + 1: start of each block's (padded) entry list
    uint32_t *part_sb;          // max_parts: block of each part of kPart entries
    uint32_t *pcnt;             // max_parts * 16: per part and tile bit, count then offset
    uint2 *ent;                 // ent_cap block entries (record id, block | tile mask << 16)
    int64_t ent_cap, max_parts;
};
// Level 2 of the binning works on parts of kBinPart entries of one block's
// list (each list padded to whole parts): the parts an entry capacity holds.
constexpr int kBinPart = 256;
inline int64_t bin_max_parts(int64_t ent_cap) { return ent_cap / kBinPart + 1; }
int chunk_rows(const ivrgs_batch &b, int chunk);
size_t depth_sort_hist_words(const ivrgs_batch &b);
// Words of the column-scan partials over chunks for rows of `width` values.
size_t col_part_words(const ivrgs_batch &b, int width, int chunk);
// Blocks of 4x4 tiles per job, and the binning's dynamic LDS per workgroup.
int bin_blocks_per_job(const Consts &k);
size_t bin_dyn_lds_bytes(const Consts &k);

hipError_t launch_project(const ivrgs_batch &b, const Consts &k, float *rec, uint32_t *rect, uint32_t *depth,
                          int64_t *nonfinite, hipStream_t s);
// atomic: several jobs may share a Gaussian; job_order: then add the jobs'
// gradients one launch per job, in job order, instead of with atomics (the
// sums are then reproducible bit for bit).  depth: the record-gradient rows
// carry the auxiliary maps' depth gradient (slot GZ) too.
hipError_t launch_project_bwd(const ivrgs_batch &b, const Consts &k, const uint32_t *rect, const float *grec,
                              const ivrgs_gaussians_mut &out, bool atomic, bool dense, hipStream_t s,
                              bool job_order = false, bool depth = false);
// Models model0 .. model0 + count - 1 (count <= kComposeModels) in one
// launch: src[j] goes to out[offset[j] ...).  host_e != nullptr: edit values
// from the host rows host_e[j]; else from dev_table[model0 + j].
constexpr int kComposeModels = 8;
hipError_t launch_compose(const ivrgs_gaussians *src, const int64_t *offset, int32_t model0, int32_t count,
                          const ivrgs_model_edit *host_e, const ivrgs_model_edit *dev_table,
                          const ivrgs_gaussians_mut &out, hipStream_t s);
struct ExploreOpts {
    float lr, beta1, beta2, eps;
    uint32_t learn;
};
hipError_t launch_explore_step(const float *edit_grad, const float *light_grad, int n_models, const ExploreOpts &o,
                               float *state, ivrgs_model_edit *rows, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill2_u32(uint32_t *p, int64_t n, uint32_t *q, int64_t m, uint32_t v, hipStream_t s);
hipError_t launch_light_bwd(const ivrgs_batch &b, const Consts &k, const uint32_t *rect, const float *grec,
                            float *out, hipStream_t s);
hipError_t launch_compose_bwd(const ivrgs_gaussians &src, int64_t offset, const ivrgs_gaussians_mut &grads,
                              float *out, hipStream_t s);
hipError_t launch_bin_sort(const ivrgs_batch &b, const Consts &k, const float *rec, const uint32_t *rect,
                           const uint32_t *depth, const ivrgs_bins &bins, const BinWork &w, int chunk, size_t bin_lds,
                           int cus, hipStream_t s);
size_t bin_static_lds_bytes();
hipError_t set_bin_lds_limit(size_t bytes);
// ckpt: per-(tile, cut) per-pixel checkpoints [n_tiles][kSplitMax - 1][256]
// float4, or nullptr: the forward writes them and the backward then walks
// each segment of a long list in its own workgroup (one pixel per lane and
// no work queue only; otherwise ignored).
hipError_t launch_render_fwd(const Consts &k, int px, int64_t n_tiles, const float *rec, const uint32_t *starts,
                             const uint32_t *sorted, float *out, float *maxw, int64_t *status, bool count,
                             uint32_t *queue, int per_cu, float *ckpt, hipStream_t s);
// The image and the auxiliary maps (depth and n_attr <= 15 attributes, rows
// of n_attr rounded up to 4 floats) in one walk, one pixel per lane, with the
// list checkpoints of the image's backward when ckpt is given.
hipError_t launch_render_fwd_maps(const Consts &k, int64_t n_tiles, const float *rec, const uint32_t *starts,
                                  const uint32_t *sorted, float *out, float *ckpt, const ivrgs_job *jobs,
                                  const int32_t *gauss_index, const float *attr, int n_attr, float *aux,
                                  hipStream_t s);
// Buffers of the deterministic backward (IVRGS_FLAG_DETERMINISTIC_BWD):
// probe [n_tiles][kGradRec] words, scale 2 * kGradRec floats, gfix
// [n_records][kGradStride] 64-bit integer sums.
struct DetWork {
    uint32_t *probe;
    float *scale;
    unsigned long long *gfix;
};
// det == nullptr: record gradients accumulated with float atomics; else
// bit-reproducible (two walks, 64-bit integer sums; see render.hip).
hipError_t launch_render_bwd(const Consts &k, int px, int64_t n_tiles, const float *rec, const uint32_t *starts,
                             const uint32_t *sorted, const float *rgba, const float *dl, float *grec,
                             uint32_t *queue, int per_cu, const float *ckpt, const DetWork *det,
                             int64_t n_records, hipStream_t s);
hipError_t launch_cull(const ivrgs_gaussians &g, const ivrgs_camera *cams, int camera, const ivrgs_culler &mlp,
                       int32_t *out_index, ivrgs_job *jobs, int job, float *logits, uint8_t *keep,
                       uint32_t *counts, hipStream_t s);
size_t cull_workspace_bytes(int64_t n);
// Vector quantisation: k-means fit of one attribute, assignment against a
// codebook, and the composition of quantised models (count <= kComposeModels
// models in one launch, edits: the host rows of those models).
size_t vq_workspace_bytes(int64_t n, int k);
size_t vq_batch_workspace_bytes(const ivrgs_vq_book *books, int count, int k);
hipError_t launch_vq_fit_batch(const ivrgs_vq_book *books, int count, int k, int iters, void *workspace,
                               hipStream_t s);
hipError_t launch_vq_fit(const float *values, int64_t n, int k, int iters, float *codebook, uint8_t *index,
                         void *workspace, hipStream_t s);
hipError_t launch_vq_assign(const float *values, int64_t n, const float *codebook, int k, uint8_t *index,
                            hipStream_t s);
hipError_t launch_vq_compose(const ivrgs_vq_model *src, const int64_t *offset, int32_t model0, int32_t count,
                             const ivrgs_model_edit *edits, const ivrgs_gaussians_mut &out, hipStream_t s);
// SH colour of base 3DGS and its backward (degree 0..3).
hipError_t launch_sh_color(const float *sh, int degree, const float *mean, int64_t n, const ivrgs_camera &cam,
                           float *color, hipStream_t s);
hipError_t launch_sh_color_bwd(const float *sh, int degree, const float *mean, int64_t n, const ivrgs_camera &cam,
                               const float *grad_color, float *grad_sh, float *grad_mean, hipStream_t s);
// Auxiliary maps: depth plus up to kAuxMax attribute planes composited with
// the image's weights, and their backward (record gradients for the
// projection backward, attribute and depth-to-mean gradients added).
constexpr int kAuxMax = 15;
hipError_t launch_aux_fwd(const ivrgs_batch &b, const Consts &k, int64_t n_tiles, const float *rec,
                          const uint32_t *starts, const uint32_t *sorted, const float *attr, int n_attr, float *aux,
                          hipStream_t s);
hipError_t launch_aux_bwd(const ivrgs_batch &b, const Consts &k, int64_t n_tiles, const float *rec,
                          const uint32_t *starts, const uint32_t *sorted, const float *attr, int n_attr,
                          const float *aux, const float *grad_aux, float *grec, float *grad_attr, hipStream_t s,
                          const float *rgba = nullptr, const float *dl = nullptr);
// (rgba, dl: the image and dL/d(image), or null: with them the image's
// backward runs in the same walk, its colour sums into GCR..GCB.)
// Attribute rows [n][12] of the editable stage from the normal, colour and
// shade planes, and their backward (adds into the plane gradients).
hipError_t launch_edit_attr_fwd(const float *normal, const float *color, const float *shade, int64_t n, float *attr,
                                hipStream_t s);
hipError_t launch_edit_attr_bwd(const float *normal, int64_t n, const float *grad_attr, float *grad_normal,
                                float *grad_color, float *grad_shade, hipStream_t s);

// SSIM of an image against its target over valid 11x11 Gaussian windows
// (sigma 1.5), and its gradient with respect to the image.
constexpr int kSsimWindow = 11;
struct SsimTaps {
    float w[kSsimWindow];
};
SsimTaps ssim_taps();
size_t ssim_workspace_floats(int channels, int H, int W);
hipError_t launch_ssim_fwd(const float *x, const float *y, int channels, int H, int W, float *out, float *ws,
                           hipStream_t s);
hipError_t launch_ssim_bwd(const float *x, const float *y, int channels, int H, int W, const float *grad_mean,
                           float *grad_x, const float *ws, hipStream_t s);
int64_t l1_blocks(int64_t n);
hipError_t launch_l1_fwd(const float *x, const float *y, int64_t n, float *out, double *partial, hipStream_t s);
hipError_t launch_l1_bwd(const float *x, const float *y, int64_t n, const float *grad_mean, float *grad_x,
                         hipStream_t s);
hipError_t launch_photometric_grad(const float *x, const float *y, int channels, int H, int W, float lam,
                                   float *grad_x, const float *ws, hipStream_t s);
// SSIM and L1 means in one pass over x and y (out[0], out[1]); the workspace
// is the SSIM forward's plus one L1 partial per workgroup.
size_t photometric_workspace_floats(int channels, int H, int W);
hipError_t launch_photometric_fwd(const float *x, const float *y, int channels, int H, int W, float *out, float *ws,
                                  hipStream_t s);
// Gradient of weights[0] mean SSIM + weights[1] mean |x - y| (device weights).
hipError_t launch_photometric_grad_dev(const float *x, const float *y, int channels, int H, int W,
                                       const float *weights, float *grad_x, const float *ws, hipStream_t s);
// Training regularisers on the rendered maps of one view (normal
// consistency, offset-colour sparsity, bilateral smoothness, opacity L1).
size_t reg_workspace_bytes(const ivrgs_reg_maps &m);
hipError_t launch_reg_fwd(const ivrgs_reg_maps &m, const ivrgs_camera &cam, float *terms, float *pseudo, void *ws,
                          hipStream_t s);
hipError_t launch_reg_bwd(const ivrgs_reg_maps &m, const ivrgs_camera &cam, const float *terms, const float *gterm,
                          float *g_normal, float *g_dc, float *g_shade, float *g_op, float *g_depth, hipStream_t s);
hipError_t launch_work_queue(const uint32_t *starts, int64_t n_tiles, uint32_t *queue, hipStream_t s);

}  // namespace ivrgs
