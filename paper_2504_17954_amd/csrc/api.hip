// C ABI: host-side validation, workspace layout and launch sequencing.
#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "launch.hpp"

namespace ivrgs {

// --------------------------------------------------------------- timing
namespace {
struct Timing {
    uint32_t mask = 0;  // bit k: kind k is timed
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<std::pair<hipEvent_t, int>> open;  // begun, not yet ended
    double ms[TK_KINDS] = {0};
    long long n[TK_KINDS] = {0};
};
Timing g_timing;
std::mutex g_timing_mu;

hipEvent_t take_event() {
    if (!g_timing.pool.empty()) {
        hipEvent_t e = g_timing.pool.back();
        g_timing.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

void timing_begin(int kind, hipStream_t s) {
    std::lock_guard<std::mutex> lock(g_timing_mu);
    if (!((g_timing.mask >> kind) & 1u)) return;
    hipEvent_t e = take_event();
    if (!e) return;
    hipEventRecord(e, s);
    g_timing.open.push_back({e, kind});
}

void timing_end(int kind, hipStream_t s) {
    std::lock_guard<std::mutex> lock(g_timing_mu);
    if (!((g_timing.mask >> kind) & 1u)) return;
    for (size_t i = g_timing.open.size(); i-- > 0;) {
        if (g_timing.open[i].second != kind) continue;
        hipEvent_t b = g_timing.open[i].first;
        g_timing.open.erase(g_timing.open.begin() + i);
        hipEvent_t e = take_event();
        if (!e) {
            g_timing.pool.push_back(b);
            return;
        }
        hipEventRecord(e, s);
        g_timing.pending.push_back({kind, {b, e}});
        return;
    }
}

namespace {

constexpr size_t kAlign = 256;
constexpr int kDefaultChunk = 512;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Per-device limits queried once per device.
struct DeviceLimits {
    bool ready = false;
    size_t max_lds = 65536;
    size_t bin_lds = 0;  // dynamic LDS the binning kernels may take (per-tile counters)
    int cus = 1;         // compute units
};
std::mutex g_mu;
DeviceLimits g_dev[64];

hipError_t device_limits(DeviceLimits &out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceLimits &d = g_dev[dev];
    if (!d.ready) {
        int lds = 0;
        e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess) return e;
        d.max_lds = (size_t)lds;
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        d.cus = cus > 0 ? cus : 1;
        d.bin_lds = d.max_lds - bin_static_lds_bytes();
        if (d.bin_lds > 65536) {
            e = set_bin_lds_limit(d.bin_lds);
            if (e != hipSuccess) return e;
        }
        d.ready = true;
    }
    out = d;
    return hipSuccess;
}

bool valid_gauss(const ivrgs_gaussians &g) {
    if (g.n < 0) return false;
    if (g.n == 0) return true;
    return g.mean && g.log_scale && g.quat && g.opacity && g.normal && g.color && g.shade;
}

bool valid_gauss_mut(const ivrgs_gaussians_mut &g) {
    if (g.n < 0) return false;
    if (g.n == 0) return true;
    return g.mean && g.log_scale && g.quat && g.opacity && g.normal && g.color && g.shade;
}

ivrgs_status check_params(const ivrgs_params *p) {
    if (!p) return IVRGS_E_INVALID;
    if (p->tile != 0 && p->tile != kTile) return IVRGS_E_UNSUPPORTED;
    if (p->width <= 0 || p->height <= 0) return IVRGS_E_SHAPE;
    const int tx = (p->width + kTile - 1) / kTile, ty = (p->height + kTile - 1) / kTile;
    if (tx > 65535 || ty > 65535) return IVRGS_E_SHAPE;
    if (!(p->alpha_min > 0.f) || !(p->alpha_max > p->alpha_min) || !(p->alpha_max < 1.f)) return IVRGS_E_INVALID;
    if (!(p->T_min > 0.f) || !(p->T_min < 1.f) || !(p->lowpass >= 0.f)) return IVRGS_E_INVALID;
    for (int px : {p->fwd_px, p->bwd_px})
        if (px != 0 && px != 1 && px != 2 && px != 4) return IVRGS_E_UNSUPPORTED;
    if (p->sort_chunk < 0 || p->persist_per_cu < 0) return IVRGS_E_INVALID;
    if ((p->flags & ~(IVRGS_FLAG_PERSISTENT | IVRGS_FLAG_COUNT_EVAL | IVRGS_FLAG_FWD_ONLY |
                      IVRGS_FLAG_DETERMINISTIC_BWD)) != 0u)
        return IVRGS_E_UNSUPPORTED;
    return IVRGS_OK;
}

ivrgs_status check_batch(const ivrgs_batch *b) {
    if (!b) return IVRGS_E_INVALID;
    if (!valid_gauss(b->g)) return IVRGS_E_INVALID;
    if (b->n_jobs < 0 || b->max_job_count < 0 || b->n_records < 0 || b->n_models <= 0) return IVRGS_E_INVALID;
    if (b->n_jobs > 0 && (!b->jobs || !b->cameras || !b->edits)) return IVRGS_E_INVALID;
    if (b->n_jobs > 65535) return IVRGS_E_SHAPE;  // jobs index a grid dimension
    if (b->n_records >= (int64_t)0xFFFFFFF0) return IVRGS_E_SHAPE;
    return IVRGS_OK;
}

// Workspace regions.
struct Layout {
    size_t key0, val0, key1, val1, hist, rng, counts, part, pay, sb_len, sb_start, grec, queue, ckpt, ckpt_bytes,
        det, tail, total;
    int64_t ent_cap, max_parts;
};

// Block entries of the binning (8 bytes each): there are never more than
// tile items (rect tiles), about a sixth of the pairs in practice; the
// region holds capacity / 2 + 2 per record plus each block's padding to
// whole parts, so a larger pair capacity also makes room for more entries.
int64_t ent_capacity(const ivrgs_batch &b, int64_t capacity, int64_t n_blocks) {
    return capacity / 2 + 2 * b.n_records + n_blocks * kBinPart + 64;
}

// The capacity-sized tail of the binning regions: the block entries, then
// the block of each part and the per-part tile counts.
size_t tail_bytes(int64_t ent_cap, int64_t max_parts) {
    return align_up(sizeof(uint2) * (size_t)ent_cap) + align_up(sizeof(uint32_t) * (size_t)max_parts) +
           align_up(sizeof(uint32_t) * 16 * (size_t)max_parts);
}

int pick_px(int requested, int fallback) { return requested == 0 ? fallback : requested; }

// Checkpoints for cutting long tile lists in the backward: (kSplitMax - 1)
// cuts x 256 pixels x 16 B per tile, with one pixel per lane in both render
// kernels and no work queue, while that stays within kCkptBudget (one view or
// a few); otherwise every list is walked whole.
constexpr size_t kCkptBudget = size_t(256) << 20;

size_t ckpt_bytes(const ivrgs_batch &b, const ivrgs_params &p, const Consts &k) {
    if (pick_px(p.fwd_px, 1) != 1 || pick_px(p.bwd_px, 1) != 1) return 0;
    if (p.flags & (IVRGS_FLAG_PERSISTENT | IVRGS_FLAG_FWD_ONLY)) return 0;
    const size_t bytes = (size_t)b.n_jobs * k.tiles_per_job * (kSplitMax - 1) * kCkptPix * sizeof(float) * 4;
    return bytes <= kCkptBudget ? bytes : 0;
}

// Records per binning chunk: the caller's choice rounded up to a multiple of
// 64 (one wave walks a chunk), or by default the largest power of two up to
// kDefaultChunk that still gives about kChunkTarget chunks over the batch, so
// that small or culled scenes keep the GPU's waves busy.
constexpr int64_t kChunkTarget = 1024;

int chunk_of(const ivrgs_params &p, const ivrgs_batch &b) {
    if (p.sort_chunk > 0) return (p.sort_chunk + 63) / 64 * 64;
    const int64_t records = (int64_t)b.max_job_count * b.n_jobs;
    int c = kDefaultChunk;
    while (c > 64 && records / c < kChunkTarget) c /= 2;
    return c;
}

Layout layout(const ivrgs_batch &b, const ivrgs_params &p, int64_t capacity = 0) {
    Layout L;
    const Consts k = make_consts(p);
    const int n_sb = bin_blocks_per_job(k);
    const size_t rec_words = align_up(sizeof(uint32_t) * (size_t)b.n_records);
    size_t off = 0;
    L.key0 = off;
    off += rec_words;
    L.val0 = off;
    off += rec_words;
    L.key1 = off;
    off += rec_words;
    L.val1 = off;
    off += rec_words;
    L.hist = off;
    off += align_up(sizeof(uint32_t) * depth_sort_hist_words(b));
    L.rng = off;
    off += align_up(sizeof(uint32_t) * 2 * (size_t)b.n_jobs);
    L.counts = off;
    off += align_up(sizeof(uint32_t) * (size_t)b.n_jobs * chunk_rows(b, chunk_of(p, b)) * n_sb);
    L.part = off;
    off += align_up(sizeof(uint32_t) * col_part_words(b, n_sb, chunk_of(p, b)));
    L.pay = off;
    off += align_up(2 * sizeof(uint4) * (size_t)b.n_records);
    L.sb_len = off;
    off += align_up(sizeof(uint32_t) * ((size_t)b.n_jobs * n_sb + 1));
    L.sb_start = off;
    off += align_up(sizeof(uint32_t) * ((size_t)b.n_jobs * n_sb + 1));
    L.grec = off;
    off += align_up(sizeof(float) * kGradStride * (size_t)b.n_records);
    L.queue = off;
    off += align_up(sizeof(uint32_t) * (size_t)(2 + (int64_t)b.n_jobs * k.tiles_per_job));
    L.ckpt = off;
    L.ckpt_bytes = ckpt_bytes(b, p, k);
    off += align_up(L.ckpt_bytes);
    // deterministic backward: 64-bit sums per record value, the largest sum
    // per (tile, value kind) and the scales
    L.det = off;
    if (p.flags & IVRGS_FLAG_DETERMINISTIC_BWD)
        off += align_up(sizeof(uint64_t) * kGradStride * (size_t)b.n_records) +
               align_up(sizeof(uint32_t) * kGradRec * (size_t)b.n_jobs * k.tiles_per_job) +
               align_up(sizeof(float) * 2 * kGradRec);
    // last, so that no other region moves with the capacity
    L.ent_cap = ent_capacity(b, capacity, (int64_t)b.n_jobs * n_sb);
    L.max_parts = bin_max_parts(L.ent_cap);
    L.tail = off;
    off += tail_bytes(L.ent_cap, L.max_parts);
    L.total = off;
    return L;
}

ivrgs_status hip_status(hipError_t e) { return e == hipSuccess ? IVRGS_OK : IVRGS_E_HIP; }

}  // namespace
}  // namespace ivrgs

using namespace ivrgs;

extern "C" {

size_t ivrgs_workspace_size(const ivrgs_batch *batch, const ivrgs_params *params, int64_t capacity) {
    if (check_batch(batch) != IVRGS_OK || check_params(params) != IVRGS_OK || capacity < 0) return 0;
    return layout(*batch, *params, capacity).total;
}

int32_t ivrgs_tiles_per_job(const ivrgs_params *params) {
    if (check_params(params) != IVRGS_OK) return 0;
    return make_consts(*params).tiles_per_job;
}

namespace {
ivrgs_status compose_common(const ivrgs_gaussians *models, int32_t n_models, const ivrgs_model_edit *host_edits,
                            const ivrgs_model_edit *dev_edits, ivrgs_gaussians_mut *out, void *stream) {
    if (!models || !out || n_models <= 0) return IVRGS_E_INVALID;
    if (!valid_gauss_mut(*out) || (out->n > 0 && !out->model_id)) return IVRGS_E_INVALID;
    int64_t total = 0;
    for (int m = 0; m < n_models; ++m) {
        if (!valid_gauss(models[m])) return IVRGS_E_INVALID;
        total += models[m].n;
    }
    if (total != out->n) return IVRGS_E_SHAPE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int64_t off = 0;
    for (int m0 = 0; m0 < n_models; m0 += kComposeModels) {
        const int cnt = std::min(kComposeModels, n_models - m0);
        int64_t offs[kComposeModels];
        for (int j = 0; j < cnt; ++j) {
            offs[j] = off;
            off += models[m0 + j].n;
        }
        hipError_t e = launch_compose(models + m0, offs, m0, cnt, host_edits ? host_edits + m0 : nullptr, dev_edits,
                                      *out, s);
        if (e != hipSuccess) return IVRGS_E_HIP;
    }
    return IVRGS_OK;
}
}  // namespace

ivrgs_status ivrgs_compose(const ivrgs_gaussians *models, int32_t n_models, const ivrgs_model_edit *edits,
                           ivrgs_gaussians_mut *out, void *stream) {
    if (!edits) return IVRGS_E_INVALID;
    return compose_common(models, n_models, edits, nullptr, out, stream);
}

ivrgs_status ivrgs_compose_dev(const ivrgs_gaussians *models, int32_t n_models, const ivrgs_model_edit *edits,
                               ivrgs_gaussians_mut *out, void *stream) {
    if (!edits) return IVRGS_E_INVALID;
    return compose_common(models, n_models, nullptr, edits, out, stream);
}

size_t ivrgs_vq_workspace_size(int64_t n, int32_t k) {
    if (n < 0 || k < 1 || k > 256) return 0;
    return vq_workspace_bytes(n, k);
}

ivrgs_status ivrgs_vq_fit(const float *values, int64_t n, int32_t k, int32_t iters, float *codebook,
                          uint8_t *index, void *workspace, size_t workspace_bytes, void *stream) {
    if (n < 0 || k < 1 || k > 256 || iters < 0 || !codebook || !workspace) return IVRGS_E_INVALID;
    if (n > 0 && (!values || !index)) return IVRGS_E_INVALID;
    if (workspace_bytes < vq_workspace_bytes(n, k)) return IVRGS_E_CAPACITY;
    return hip_status(launch_vq_fit(values, n, k, iters, codebook, index, workspace,
                                    reinterpret_cast<hipStream_t>(stream)));
}

size_t ivrgs_vq_fit_batch_workspace_size(const ivrgs_vq_book *books, int32_t count, int32_t k) {
    if (!books || count < 0 || k < 1 || k > 256) return 0;
    for (int i = 0; i < count; ++i)
        if (books[i].n < 0) return 0;
    return vq_batch_workspace_bytes(books, count, k);
}

ivrgs_status ivrgs_vq_fit_batch(const ivrgs_vq_book *books, int32_t count, int32_t k, int32_t iters,
                                void *workspace, size_t workspace_bytes, void *stream) {
    if (count < 0 || k < 1 || k > 256 || iters < 0 || (count > 0 && (!books || !workspace))) return IVRGS_E_INVALID;
    for (int i = 0; i < count; ++i) {
        const ivrgs_vq_book &b = books[i];
        if (b.n < 0 || !b.codebook) return IVRGS_E_INVALID;
        if (b.n > 0 && (!b.values || !b.index)) return IVRGS_E_INVALID;
    }
    if (count == 0) return IVRGS_OK;
    if (workspace_bytes < vq_batch_workspace_bytes(books, count, k)) return IVRGS_E_CAPACITY;
    return hip_status(launch_vq_fit_batch(books, count, k, iters, workspace, reinterpret_cast<hipStream_t>(stream)));
}

ivrgs_status ivrgs_vq_assign(const float *values, int64_t n, const float *codebook, int32_t k, uint8_t *index,
                             void *stream) {
    if (n < 0 || k < 1 || k > 256 || !codebook) return IVRGS_E_INVALID;
    if (n > 0 && (!values || !index)) return IVRGS_E_INVALID;
    return hip_status(launch_vq_assign(values, n, codebook, k, index, reinterpret_cast<hipStream_t>(stream)));
}

ivrgs_status ivrgs_vq_compose(const ivrgs_vq_model *models, int32_t n_models, const ivrgs_model_edit *edits,
                              ivrgs_gaussians_mut *out, void *stream) {
    if (!models || !edits || !out || n_models <= 0) return IVRGS_E_INVALID;
    if (!valid_gauss_mut(*out) || (out->n > 0 && !out->model_id)) return IVRGS_E_INVALID;
    int64_t total = 0;
    for (int m = 0; m < n_models; ++m) {
        const ivrgs_vq_model &q = models[m];
        if (q.n < 0) return IVRGS_E_INVALID;
        if (q.n > 0 && (!q.mean || !q.normal || !q.index || !q.codebook || q.k < 1 || q.k > 256))
            return IVRGS_E_INVALID;
        total += q.n;
    }
    if (total != out->n) return IVRGS_E_SHAPE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int64_t off = 0;
    for (int m0 = 0; m0 < n_models; m0 += kComposeModels) {
        const int cnt = std::min(kComposeModels, n_models - m0);
        int64_t offs[kComposeModels];
        for (int j = 0; j < cnt; ++j) {
            offs[j] = off;
            off += models[m0 + j].n;
        }
        const hipError_t e = launch_vq_compose(models + m0, offs, m0, cnt, edits + m0, *out, s);
        if (e != hipSuccess) return IVRGS_E_HIP;
    }
    return IVRGS_OK;
}

ivrgs_status ivrgs_render_aux_fwd(const ivrgs_batch *batch, const ivrgs_params *params,
                                  const ivrgs_projected *proj, const ivrgs_bins *bins, const float *attr,
                                  int32_t n_attr, float *out_aux, void *stream) {
    ivrgs_status st = check_batch(batch);
    if (st != IVRGS_OK) return st;
    if ((st = check_params(params)) != IVRGS_OK) return st;
    if (!proj || !bins || !bins->tile_start || !out_aux || n_attr < 0 || n_attr > kAuxMax) return IVRGS_E_INVALID;
    if (n_attr > 0 && (!attr || (reinterpret_cast<uintptr_t>(attr) & 15u))) return IVRGS_E_INVALID;
    const Consts k = make_consts(*params);
    const int64_t n_tiles = (int64_t)batch->n_jobs * k.tiles_per_job;
    return hip_status(launch_aux_fwd(*batch, k, n_tiles, proj->rec, bins->tile_start, bins->sorted, attr, n_attr,
                                     out_aux, reinterpret_cast<hipStream_t>(stream)));
}

ivrgs_status ivrgs_render_aux_bwd(const ivrgs_batch *batch, const ivrgs_params *params,
                                  const ivrgs_projected *proj, const ivrgs_bins *bins, const float *attr,
                                  int32_t n_attr, const float *aux, const float *grad_aux, float *grad_attr,
                                  ivrgs_gaussians_mut *grads, void *workspace, size_t workspace_bytes,
                                  void *stream) {
    ivrgs_status st = check_batch(batch);
    if (st != IVRGS_OK) return st;
    if ((st = check_params(params)) != IVRGS_OK) return st;
    if (!proj || !bins || !bins->tile_start || !aux || !grad_aux || !grads || n_attr < 0 || n_attr > kAuxMax)
        return IVRGS_E_INVALID;
    if (n_attr > 0 && (!attr || !grad_attr || (reinterpret_cast<uintptr_t>(attr) & 15u))) return IVRGS_E_INVALID;
    if (!valid_gauss_mut(*grads) || grads->n != batch->g.n) return IVRGS_E_SHAPE;
    const Consts k = make_consts(*params);
    const Layout L = layout(*batch, *params);
    if (!workspace || workspace_bytes < L.total) return IVRGS_E_CAPACITY;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float *grec = reinterpret_cast<float *>(static_cast<char *>(workspace) + L.grec);
    const int64_t n_tiles = (int64_t)batch->n_jobs * k.tiles_per_job;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(grec), kGradStride * batch->n_records, 0u, s);
    if (e == hipSuccess)
        e = launch_aux_bwd(*batch, k, n_tiles, proj->rec, bins->tile_start, bins->sorted, attr, n_attr, aux, grad_aux,
                           grec, grad_attr, s);
    if (e == hipSuccess) e = launch_project_bwd(*batch, k, proj->rect, grec, *grads, true, false, s, false, true);
    return hip_status(e);
}

ivrgs_status ivrgs_editable_attr_fwd(const float *normal, const float *color, const float *shade, int64_t n,
                                     float *attr, void *stream) {
    if (n < 0) return IVRGS_E_INVALID;
    if (n == 0) return IVRGS_OK;
    if (!normal || !color || !shade || !attr || (reinterpret_cast<uintptr_t>(attr) & 15u)) return IVRGS_E_INVALID;
    if ((n + 255) / 256 > (int64_t)UINT32_MAX) return IVRGS_E_SHAPE;
    return hip_status(launch_edit_attr_fwd(normal, color, shade, n, attr, reinterpret_cast<hipStream_t>(stream)));
}

ivrgs_status ivrgs_editable_attr_bwd(const float *normal, int64_t n, const float *grad_attr, float *grad_normal,
                                     float *grad_color, float *grad_shade, void *stream) {
    if (n < 0) return IVRGS_E_INVALID;
    if (n == 0) return IVRGS_OK;
    if (!normal || !grad_attr || !grad_normal || !grad_color || !grad_shade ||
        (reinterpret_cast<uintptr_t>(grad_attr) & 15u))
        return IVRGS_E_INVALID;
    if ((n + 255) / 256 > (int64_t)UINT32_MAX) return IVRGS_E_SHAPE;
    return hip_status(launch_edit_attr_bwd(normal, n, grad_attr, grad_normal, grad_color, grad_shade,
                                           reinterpret_cast<hipStream_t>(stream)));
}

ivrgs_status ivrgs_sh_color(const float *sh, int32_t degree, const float *mean, int64_t n,
                            const ivrgs_camera *camera, float *color, void *stream) {
    if (degree < 0 || degree > 3 || n < 0 || !camera) return IVRGS_E_INVALID;
    if (n > 0 && (!sh || !mean || !color)) return IVRGS_E_INVALID;
    if ((n + 255) / 256 > (int64_t)UINT32_MAX) return IVRGS_E_SHAPE;
    return hip_status(launch_sh_color(sh, degree, mean, n, *camera, color, reinterpret_cast<hipStream_t>(stream)));
}

ivrgs_status ivrgs_sh_color_bwd(const float *sh, int32_t degree, const float *mean, int64_t n,
                                const ivrgs_camera *camera, const float *grad_color, float *grad_sh,
                                float *grad_mean, void *stream) {
    if (degree < 0 || degree > 3 || n < 0 || !camera) return IVRGS_E_INVALID;
    if (n > 0 && (!sh || !mean || !grad_color || !grad_sh)) return IVRGS_E_INVALID;
    if ((n + 255) / 256 > (int64_t)UINT32_MAX) return IVRGS_E_SHAPE;
    return hip_status(launch_sh_color_bwd(sh, degree, mean, n, *camera, grad_color, grad_sh, grad_mean,
                                          reinterpret_cast<hipStream_t>(stream)));
}

static bool ssim_shape_ok(int32_t c, int32_t h, int32_t w) {
    return c >= 1 && h >= kSsimWindow && w >= kSsimWindow && c <= 65535 && (int64_t)h * w <= (int64_t)1 << 31;
}

size_t ivrgs_ssim_workspace_size(int32_t channels, int32_t height, int32_t width) {
    if (!ssim_shape_ok(channels, height, width)) return 0;
    return sizeof(float) * ssim_workspace_floats(channels, height, width);
}

ivrgs_status ivrgs_ssim_fwd(const float *x, const float *y, int32_t channels, int32_t height, int32_t width,
                            float *out_mean, void *workspace, size_t workspace_bytes, void *stream) {
    if (!x || !y || !out_mean || !workspace) return IVRGS_E_INVALID;
    if (!ssim_shape_ok(channels, height, width)) return IVRGS_E_SHAPE;
    if (workspace_bytes < ivrgs_ssim_workspace_size(channels, height, width)) return IVRGS_E_CAPACITY;
    return hip_status(launch_ssim_fwd(x, y, channels, height, width, out_mean, static_cast<float *>(workspace),
                                      reinterpret_cast<hipStream_t>(stream)));
}

ivrgs_status ivrgs_ssim_bwd(const float *x, const float *y, int32_t channels, int32_t height, int32_t width,
                            const float *grad_mean, float *grad_x, const void *workspace, size_t workspace_bytes,
                            void *stream) {
    if (!x || !y || !grad_mean || !grad_x || !workspace) return IVRGS_E_INVALID;
    if (!ssim_shape_ok(channels, height, width)) return IVRGS_E_SHAPE;
    if (workspace_bytes < ivrgs_ssim_workspace_size(channels, height, width)) return IVRGS_E_CAPACITY;
    return hip_status(launch_ssim_bwd(x, y, channels, height, width, grad_mean, grad_x,
                                      static_cast<const float *>(workspace), reinterpret_cast<hipStream_t>(stream)));
}

ivrgs_status ivrgs_photometric_grad(const float *x, const float *y, int32_t channels, int32_t height,
                                    int32_t width, float lam, float *grad_x, const void *workspace,
                                    size_t workspace_bytes, void *stream) {
    if (!x || !y || !grad_x || !workspace) return IVRGS_E_INVALID;
    if (!(lam >= 0.0f && lam <= 1.0f)) return IVRGS_E_INVALID;
    if (!ssim_shape_ok(channels, height, width)) return IVRGS_E_SHAPE;
    if (workspace_bytes < ivrgs_ssim_workspace_size(channels, height, width)) return IVRGS_E_CAPACITY;
    return hip_status(launch_photometric_grad(x, y, channels, height, width, lam, grad_x,
                                              static_cast<const float *>(workspace),
                                              reinterpret_cast<hipStream_t>(stream)));
}

size_t ivrgs_photometric_workspace_size(int32_t channels, int32_t height, int32_t width) {
    if (!ssim_shape_ok(channels, height, width)) return 0;
    return sizeof(float) * photometric_workspace_floats(channels, height, width);
}

ivrgs_status ivrgs_photometric_fwd(const float *x, const float *y, int32_t channels, int32_t height, int32_t width,
                                   float *out_means, void *workspace, size_t workspace_bytes, void *stream) {
    if (!x || !y || !out_means || !workspace) return IVRGS_E_INVALID;
    if (!ssim_shape_ok(channels, height, width)) return IVRGS_E_SHAPE;
    if (workspace_bytes < ivrgs_photometric_workspace_size(channels, height, width)) return IVRGS_E_CAPACITY;
    return hip_status(launch_photometric_fwd(x, y, channels, height, width, out_means,
                                             static_cast<float *>(workspace), reinterpret_cast<hipStream_t>(stream)));
}

ivrgs_status ivrgs_photometric_grad_dev(const float *x, const float *y, int32_t channels, int32_t height,
                                        int32_t width, const float *weights, float *grad_x, const void *workspace,
                                        size_t workspace_bytes, void *stream) {
    if (!x || !y || !weights || !grad_x || !workspace) return IVRGS_E_INVALID;
    if (!ssim_shape_ok(channels, height, width)) return IVRGS_E_SHAPE;
    if (workspace_bytes < ivrgs_ssim_workspace_size(channels, height, width)) return IVRGS_E_CAPACITY;
    return hip_status(launch_photometric_grad_dev(x, y, channels, height, width, weights, grad_x,
                                                  static_cast<const float *>(workspace),
                                                  reinterpret_cast<hipStream_t>(stream)));
}

size_t ivrgs_l1_workspace_size(int64_t n) { return n > 0 ? sizeof(double) * (size_t)l1_blocks(n) : 0; }

ivrgs_status ivrgs_l1_fwd(const float *x, const float *y, int64_t n, float *out_mean, void *workspace,
                          size_t workspace_bytes, void *stream) {
    if (!x || !y || !out_mean || !workspace) return IVRGS_E_INVALID;
    if (n <= 0 || n > ((int64_t)1 << 40)) return IVRGS_E_SHAPE;
    if (workspace_bytes < ivrgs_l1_workspace_size(n)) return IVRGS_E_CAPACITY;
    return hip_status(launch_l1_fwd(x, y, n, out_mean, static_cast<double *>(workspace),
                                    reinterpret_cast<hipStream_t>(stream)));
}

ivrgs_status ivrgs_l1_bwd(const float *x, const float *y, int64_t n, const float *grad_mean, float *grad_x,
                          void *stream) {
    if (!x || !y || !grad_mean || !grad_x) return IVRGS_E_INVALID;
    if (n <= 0 || (n + 255) / 256 > (int64_t)UINT32_MAX) return IVRGS_E_SHAPE;
    return hip_status(launch_l1_bwd(x, y, n, grad_mean, grad_x, reinterpret_cast<hipStream_t>(stream)));
}

int64_t ivrgs_explore_state_words(int32_t n_models) {
    if (n_models <= 0) return 0;
    return 3 * (4 * (int64_t)n_models + 10) + 1;
}

ivrgs_status ivrgs_explore_step(const float *edit_grad, const float *light_grad, int32_t n_models,
                                const ivrgs_explore_opts *opts, float *state, ivrgs_model_edit *edits, void *stream) {
    if (!opts || !state || !edits || n_models <= 0) return IVRGS_E_INVALID;
    if (!edit_grad && (opts->learn & 7u)) return IVRGS_E_INVALID;
    if (n_models > (1 << 20)) return IVRGS_E_SHAPE;
    if (!(opts->lr >= 0.f) || !(opts->beta1 >= 0.f && opts->beta1 < 1.f) || !(opts->beta2 >= 0.f && opts->beta2 < 1.f) ||
        !(opts->eps > 0.f) || (opts->learn & ~15u))
        return IVRGS_E_INVALID;
    ExploreOpts o = {opts->lr, opts->beta1, opts->beta2, opts->eps, opts->learn};
    return hip_status(launch_explore_step(edit_grad, light_grad, n_models, o, state, edits,
                                          reinterpret_cast<hipStream_t>(stream)));
}

ivrgs_status ivrgs_compose_bwd(const ivrgs_gaussians *models, int32_t n_models, const ivrgs_gaussians_mut *grads,
                               float *out_edit_grad, void *stream) {
    if (!models || !grads || !out_edit_grad || n_models <= 0) return IVRGS_E_INVALID;
    if (!valid_gauss_mut(*grads)) return IVRGS_E_INVALID;
    int64_t total = 0;
    for (int m = 0; m < n_models; ++m) {
        if (!valid_gauss(models[m])) return IVRGS_E_INVALID;
        total += models[m].n;
    }
    if (total != grads->n) return IVRGS_E_SHAPE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(out_edit_grad), 12 * (int64_t)n_models, 0u, s);
    int64_t off = 0;
    for (int m = 0; m < n_models && e == hipSuccess; ++m) {
        e = launch_compose_bwd(models[m], off, *grads, out_edit_grad + 12 * m, s);
        off += models[m].n;
    }
    return hip_status(e);
}

ivrgs_status ivrgs_light_bwd(const ivrgs_batch *batch, const ivrgs_params *params, const ivrgs_projected *proj,
                             float *out_light_grad, const void *workspace, size_t workspace_bytes, void *stream) {
    ivrgs_status st = check_batch(batch);
    if (st != IVRGS_OK) return st;
    if ((st = check_params(params)) != IVRGS_OK) return st;
    if (!proj || !out_light_grad) return IVRGS_E_INVALID;
    if (batch->n_records > 0 && (!proj->rec || !proj->rect)) return IVRGS_E_INVALID;
    const Consts k = make_consts(*params);
    const Layout L = layout(*batch, *params);
    if (!workspace || workspace_bytes < L.total) return IVRGS_E_CAPACITY;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const float *grec = reinterpret_cast<const float *>(static_cast<const char *>(workspace) + L.grec);
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(out_light_grad), 3 * (int64_t)batch->n_models, 0u, s);
    if (e == hipSuccess) e = launch_light_bwd(*batch, k, proj->rect, grec, out_light_grad, s);
    return hip_status(e);
}

ivrgs_status ivrgs_project(const ivrgs_batch *batch, const ivrgs_params *params, ivrgs_projected *out,
                           void *stream) {
    ivrgs_status st = check_batch(batch);
    if (st != IVRGS_OK) return st;
    if ((st = check_params(params)) != IVRGS_OK) return st;
    if (!out || (batch->n_records > 0 && (!out->rec || !out->rect || !out->depth))) return IVRGS_E_INVALID;
    const Consts k = make_consts(*params);
    return hip_status(launch_project(*batch, k, out->rec, out->rect, out->depth, out->nonfinite,
                                     reinterpret_cast<hipStream_t>(stream)));
}

namespace {
// Host validation shared by both binning entry points; fills the layout and
// the device limits on success.
ivrgs_status bin_sort_check(const ivrgs_batch *batch, const ivrgs_params *params, const ivrgs_projected *proj,
                            const ivrgs_bins *bins, Layout &L, DeviceLimits &dl) {
    ivrgs_status st = check_batch(batch);
    if (st != IVRGS_OK) return st;
    if ((st = check_params(params)) != IVRGS_OK) return st;
    if (!proj || !bins || !bins->tile_start || !bins->status || bins->capacity < 0) return IVRGS_E_INVALID;
    if (bins->capacity > 0 && !bins->sorted) return IVRGS_E_INVALID;
    if (batch->n_records > 0 && (!proj->rec || !proj->rect || !proj->depth)) return IVRGS_E_INVALID;
    const Consts k = make_consts(*params);
    if (device_limits(dl) != hipSuccess) return IVRGS_E_HIP;
    if (bin_dyn_lds_bytes(k) > dl.bin_lds || bin_blocks_per_job(k) > 65535) return IVRGS_E_SHAPE;
    L = layout(*batch, *params, bins->capacity);
    return IVRGS_OK;
}

// The binning launches over a workspace `ws` laid out by L (the regions
// before L.grec; the work queue too with IVRGS_FLAG_PERSISTENT) and the
// capacity-sized tail at `tail` (tail_bytes of L's sizes).
ivrgs_status bin_sort_run(const ivrgs_batch *batch, const ivrgs_params *params, const ivrgs_projected *proj,
                          ivrgs_bins *bins, const Layout &L, const DeviceLimits &dl, char *ws, char *tail,
                          void *stream) {
    const Consts k = make_consts(*params);
    BinWork w;
    w.key[0] = reinterpret_cast<uint32_t *>(ws + L.key0);
    w.val[0] = reinterpret_cast<uint32_t *>(ws + L.val0);
    w.key[1] = reinterpret_cast<uint32_t *>(ws + L.key1);
    w.val[1] = reinterpret_cast<uint32_t *>(ws + L.val1);
    w.hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    w.rng = reinterpret_cast<uint32_t *>(ws + L.rng);
    w.counts = reinterpret_cast<uint32_t *>(ws + L.counts);
    w.part = reinterpret_cast<uint32_t *>(ws + L.part);
    w.pay = reinterpret_cast<uint4 *>(ws + L.pay);
    w.sb_len = reinterpret_cast<uint32_t *>(ws + L.sb_len);
    w.sb_start = reinterpret_cast<uint32_t *>(ws + L.sb_start);
    w.ent = reinterpret_cast<uint2 *>(tail);
    tail += align_up(sizeof(uint2) * (size_t)L.ent_cap);
    w.part_sb = reinterpret_cast<uint32_t *>(tail);
    tail += align_up(sizeof(uint32_t) * (size_t)L.max_parts);
    w.pcnt = reinterpret_cast<uint32_t *>(tail);
    w.ent_cap = L.ent_cap;
    w.max_parts = L.max_parts;
    const int chunk = chunk_of(*params, *batch);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = launch_bin_sort(*batch, k, proj->rec, proj->rect, proj->depth, *bins, w, chunk, dl.bin_lds, dl.cus, s);
    if (e == hipSuccess && (params->flags & IVRGS_FLAG_PERSISTENT))
        e = launch_work_queue(bins->tile_start, (int64_t)batch->n_jobs * k.tiles_per_job,
                              reinterpret_cast<uint32_t *>(ws + L.queue), s);
    return hip_status(e);
}

}  // namespace

ivrgs_status ivrgs_bin_sort(const ivrgs_batch *batch, const ivrgs_params *params, const ivrgs_projected *proj,
                            ivrgs_bins *bins, void *workspace, size_t workspace_bytes, void *stream) {
    Layout L;
    DeviceLimits dl;
    const ivrgs_status st = bin_sort_check(batch, params, proj, bins, L, dl);
    if (st != IVRGS_OK) return st;
    if (!workspace || workspace_bytes < L.total) return IVRGS_E_CAPACITY;
    char *ws = static_cast<char *>(workspace);
    return bin_sort_run(batch, params, proj, bins, L, dl, ws, ws + L.tail, stream);
}

}  // extern "C"

// ------------------------------------------------ binning without allocation
namespace ivrgs {
namespace {
// Scratch of ivrgs_bin_sort_noalloc: the binning regions of the workspace
// layout (depth order, digit histograms, per-chunk tile counts and the
// records' binning fields in depth order).  Every device that loads the
// library holds its own copy until the process ends, and every call on a
// device shares it.  In host code `scratch` only stands in for the array:
// kernels get the device address that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[IVRGS_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
char *g_scratch[64];  // device address of `scratch`, per device

// The current device's address of `scratch`, looked up on the first call on
// that device (with it current) and kept.
hipError_t scratch_address(char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch[dev] = static_cast<char *>(ptr);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}
}  // namespace
}  // namespace ivrgs

extern "C" {

ivrgs_status ivrgs_bin_sort_noalloc(const ivrgs_batch *batch, const ivrgs_params *params,
                                    const ivrgs_projected *proj, ivrgs_bins *bins, void *stream) {
    Layout L;
    DeviceLimits dl;
    const ivrgs_status st = bin_sort_check(batch, params, proj, bins, L, dl);
    if (st != IVRGS_OK) return st;
    // the work queue of a persistent launch lives in the render calls' workspace
    if (params->flags & IVRGS_FLAG_PERSISTENT) return IVRGS_E_UNSUPPORTED;
    // the binning regions come first in the layout and end where the record
    // gradients begin; the capacity-sized tail follows them here
    if (L.grec + tail_bytes(L.ent_cap, L.max_parts) > (size_t)IVRGS_NOALLOC_SCRATCH_BYTES) return IVRGS_E_CAPACITY;
    char *ws = nullptr;
    if (scratch_address(&ws) != hipSuccess) return IVRGS_E_HIP;
    return bin_sort_run(batch, params, proj, bins, L, dl, ws, ws + L.grec, stream);
}

ivrgs_status ivrgs_render_fwd(const ivrgs_batch *batch, const ivrgs_params *params, const ivrgs_projected *proj,
                              const ivrgs_bins *bins, float *out_rgba, float *out_maxw, void *workspace,
                              size_t workspace_bytes, void *stream) {
    ivrgs_status st = check_batch(batch);
    if (st != IVRGS_OK) return st;
    if ((st = check_params(params)) != IVRGS_OK) return st;
    if (!proj || !bins || !bins->tile_start || !bins->status || !out_rgba) return IVRGS_E_INVALID;
    const Consts k = make_consts(*params);
    const int64_t n_tiles = (int64_t)batch->n_jobs * k.tiles_per_job;
    const bool count = (params->flags & IVRGS_FLAG_COUNT_EVAL) != 0;
    uint32_t *queue = nullptr;
    float *ckpt = nullptr;
    const Layout L = layout(*batch, *params);
    if ((params->flags & IVRGS_FLAG_PERSISTENT) || L.ckpt_bytes) {
        if (!workspace || workspace_bytes < L.total) return IVRGS_E_CAPACITY;
        char *ws = static_cast<char *>(workspace);
        if (params->flags & IVRGS_FLAG_PERSISTENT) queue = reinterpret_cast<uint32_t *>(ws + L.queue);
        if (L.ckpt_bytes) ckpt = reinterpret_cast<float *>(ws + L.ckpt);
    }
    return hip_status(launch_render_fwd(k, pick_px(params->fwd_px, 1), n_tiles, proj->rec, bins->tile_start,
                                        bins->sorted, out_rgba, out_maxw, bins->status, count, queue,
                                        params->persist_per_cu, ckpt, reinterpret_cast<hipStream_t>(stream)));
}

}  // extern "C"

namespace ivrgs {
namespace {
// The maps' part of a combined backward (ivrgs_render_bwd_aux).
struct AuxBwdArgs {
    const float *attr, *aux, *grad_aux;
    float *grad_attr;
    int n_attr;
};

// The image's backward, and with `ax` the maps' too in the same walk: clear
// the record-gradient rows (and the attribute gradients), one walk, one
// projection backward.
ivrgs_status render_bwd_run(const ivrgs_batch *batch, const ivrgs_params *params, const ivrgs_projected *proj,
                            const ivrgs_bins *bins, const float *out_rgba, const float *dl_drgba,
                            ivrgs_gaussians_mut *grads, const AuxBwdArgs *ax, void *workspace, size_t workspace_bytes,
                            void *stream) {
    ivrgs_status st = check_batch(batch);
    if (st != IVRGS_OK) return st;
    if ((st = check_params(params)) != IVRGS_OK) return st;
    if (!proj || !bins || !bins->tile_start || !out_rgba || !dl_drgba || !grads) return IVRGS_E_INVALID;
    if (!valid_gauss_mut(*grads) || grads->n != batch->g.n) return IVRGS_E_SHAPE;
    const Consts k = make_consts(*params);
    const Layout L = layout(*batch, *params);
    if (!workspace || workspace_bytes < L.total) return IVRGS_E_CAPACITY;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float *grec = reinterpret_cast<float *>(static_cast<char *>(workspace) + L.grec);
    const int64_t n_tiles = (int64_t)batch->n_jobs * k.tiles_per_job;
    const bool det = (params->flags & IVRGS_FLAG_DETERMINISTIC_BWD) != 0;
    DetWork dw;
    if (det) {
        char *d = static_cast<char *>(workspace) + L.det;
        dw.gfix = reinterpret_cast<unsigned long long *>(d);
        d += align_up(sizeof(uint64_t) * kGradStride * (size_t)batch->n_records);
        dw.probe = reinterpret_cast<uint32_t *>(d);
        d += align_up(sizeof(uint32_t) * kGradRec * (size_t)n_tiles);
        dw.scale = reinterpret_cast<float *>(d);
    }
    // the deterministic walk writes every record gradient itself
    hipError_t e = hipSuccess;
    const int64_t n_grec = kGradStride * batch->n_records;
    if (ax)
        e = launch_fill2_u32(reinterpret_cast<uint32_t *>(grec), n_grec, reinterpret_cast<uint32_t *>(ax->grad_attr),
                             ax->n_attr > 0 ? batch->g.n * (int64_t)((ax->n_attr + 3) / 4 * 4) : 0, 0u, s);
    else if (!det)
        e = launch_fill_u32(reinterpret_cast<uint32_t *>(grec), n_grec, 0u, s);
    if (e == hipSuccess && !ax)
        e = launch_render_bwd(k, pick_px(params->bwd_px, 1), n_tiles, proj->rec, bins->tile_start, bins->sorted,
                              out_rgba, dl_drgba, grec,
                              (params->flags & IVRGS_FLAG_PERSISTENT)
                                  ? reinterpret_cast<uint32_t *>(static_cast<char *>(workspace) + L.queue)
                                  : nullptr,
                              params->persist_per_cu,
                              L.ckpt_bytes ? reinterpret_cast<const float *>(static_cast<char *>(workspace) + L.ckpt)
                                           : nullptr,
                              det ? &dw : nullptr, batch->n_records, s);
    // with the maps: one walk for both backwards (the image's colour as
    // three more channels of the maps' walk)
    if (e == hipSuccess && ax)
        e = launch_aux_bwd(*batch, k, n_tiles, proj->rec, bins->tile_start, bins->sorted, ax->attr, ax->n_attr,
                           ax->aux, ax->grad_aux, grec, ax->grad_attr, s, out_rgba, dl_drgba);
    // One job over the whole set (its range lies in [0, n) and has n
    // records) writes every Gaussian's gradient, zeros included; otherwise
    // the planes are cleared first and, when several jobs may share a
    // Gaussian, accumulated with atomics.
    const int64_t n = grads->n;
    const bool dense = batch->n_jobs == 1 && !batch->gauss_index && batch->n_records == n;
    const bool shared = batch->n_jobs > 1;
    float *planes[7] = {grads->mean, grads->log_scale, grads->quat, grads->opacity,
                        grads->normal, grads->color, grads->shade};
    const int dims[7] = {3, 3, 4, 1, 3, 3, 4};
    for (int p = 0; p < 7 && e == hipSuccess && !dense; ++p)
        e = launch_fill_u32(reinterpret_cast<uint32_t *>(planes[p]), dims[p] * n, 0u, s);
    if (e == hipSuccess)
        e = launch_project_bwd(*batch, k, proj->rect, grec, *grads, shared, dense, s, det, ax != nullptr);
    return hip_status(e);
}
}  // namespace
}  // namespace ivrgs

extern "C" {

ivrgs_status ivrgs_render_fwd_aux(const ivrgs_batch *batch, const ivrgs_params *params, const ivrgs_projected *proj,
                                  const ivrgs_bins *bins, const float *attr, int32_t n_attr, float *out_rgba,
                                  float *out_aux, void *workspace, size_t workspace_bytes, void *stream) {
    ivrgs_status st = check_batch(batch);
    if (st != IVRGS_OK) return st;
    if ((st = check_params(params)) != IVRGS_OK) return st;
    if (!proj || !bins || !bins->tile_start || !out_rgba || !out_aux || n_attr < 0 || n_attr > kAuxMax)
        return IVRGS_E_INVALID;
    if (n_attr > 0 && (!attr || (reinterpret_cast<uintptr_t>(attr) & 15u))) return IVRGS_E_INVALID;
    const Consts k = make_consts(*params);
    const Layout L = layout(*batch, *params);
    if (L.ckpt_bytes && (!workspace || workspace_bytes < L.total)) return IVRGS_E_CAPACITY;
    float *ckpt = L.ckpt_bytes ? reinterpret_cast<float *>(static_cast<char *>(workspace) + L.ckpt) : nullptr;
    return hip_status(launch_render_fwd_maps(k, (int64_t)batch->n_jobs * k.tiles_per_job, proj->rec,
                                             bins->tile_start, bins->sorted, out_rgba, ckpt, batch->jobs,
                                             batch->gauss_index, attr, n_attr, out_aux,
                                             reinterpret_cast<hipStream_t>(stream)));
}

ivrgs_status ivrgs_render_bwd(const ivrgs_batch *batch, const ivrgs_params *params, const ivrgs_projected *proj,
                              const ivrgs_bins *bins, const float *out_rgba, const float *dl_drgba,
                              ivrgs_gaussians_mut *grads, void *workspace, size_t workspace_bytes, void *stream) {
    return render_bwd_run(batch, params, proj, bins, out_rgba, dl_drgba, grads, nullptr, workspace, workspace_bytes,
                          stream);
}

ivrgs_status ivrgs_render_bwd_aux(const ivrgs_batch *batch, const ivrgs_params *params, const ivrgs_projected *proj,
                                  const ivrgs_bins *bins, const float *out_rgba, const float *dl_drgba,
                                  const float *attr, int32_t n_attr, const float *aux, const float *grad_aux,
                                  float *grad_attr, ivrgs_gaussians_mut *grads, void *workspace,
                                  size_t workspace_bytes, void *stream) {
    if (!params || !aux || !grad_aux || n_attr < 0 || n_attr > kAuxMax) return IVRGS_E_INVALID;
    if (n_attr > 0 && (!attr || !grad_attr || (reinterpret_cast<uintptr_t>(attr) & 15u))) return IVRGS_E_INVALID;
    if (params->flags & IVRGS_FLAG_DETERMINISTIC_BWD) return IVRGS_E_UNSUPPORTED;
    const AuxBwdArgs ax{attr, aux, grad_aux, grad_attr, n_attr};
    return render_bwd_run(batch, params, proj, bins, out_rgba, dl_drgba, grads, &ax, workspace, workspace_bytes,
                          stream);
}

void ivrgs_timing_enable(uint32_t kinds) {
    std::lock_guard<std::mutex> lock(g_timing_mu);
    for (auto &p : g_timing.pending) {
        hipEventSynchronize(p.second.second);
        g_timing.pool.push_back(p.second.first);
        g_timing.pool.push_back(p.second.second);
    }
    g_timing.pending.clear();
    for (auto &o : g_timing.open) g_timing.pool.push_back(o.first);
    g_timing.open.clear();
    for (int k = 0; k < TK_KINDS; ++k) {
        g_timing.ms[k] = 0.0;
        g_timing.n[k] = 0;
    }
    g_timing.mask = kinds & ((1u << TK_KINDS) - 1u);
}

int32_t ivrgs_timing_read(double *ms, int64_t *launches) {
    std::lock_guard<std::mutex> lock(g_timing_mu);
    for (auto &p : g_timing.pending) {
        float t = 0.f;
        if (hipEventSynchronize(p.second.second) == hipSuccess &&
            hipEventElapsedTime(&t, p.second.first, p.second.second) == hipSuccess) {
            g_timing.ms[p.first] += t;
            g_timing.n[p.first] += 1;
        }
        g_timing.pool.push_back(p.second.first);
        g_timing.pool.push_back(p.second.second);
    }
    g_timing.pending.clear();
    for (int k = 0; k < TK_KINDS; ++k) {
        if (ms) ms[k] = g_timing.ms[k];
        if (launches) launches[k] = g_timing.n[k];
    }
    return TK_KINDS;
}

size_t ivrgs_cull_workspace_size(int64_t n) { return n < 0 ? 0 : cull_workspace_bytes(n); }

ivrgs_status ivrgs_cull(const ivrgs_gaussians *g, const ivrgs_camera *cameras, int32_t camera,
                        const ivrgs_culler *mlp, int32_t *out_index, ivrgs_job *jobs, int32_t job,
                        float *out_logit, void *workspace, size_t workspace_bytes, void *stream) {
    if (!g || !valid_gauss(*g) || !cameras || camera < 0 || !mlp || !jobs || job < 0) return IVRGS_E_INVALID;
    if (!mlp->w1 || !mlp->b1 || !mlp->w2 || !mlp->b2 || !mlp->w3) return IVRGS_E_INVALID;
    if ((reinterpret_cast<uintptr_t>(mlp->w1) | reinterpret_cast<uintptr_t>(mlp->w2)) & 7u) return IVRGS_E_INVALID;
    if (g->n > 0 && !out_index) return IVRGS_E_INVALID;
    if (g->n >= (int64_t)0x7FFFFFFF) return IVRGS_E_SHAPE;
    const size_t need = cull_workspace_bytes(g->n);
    if (!workspace || workspace_bytes < need) return IVRGS_E_CAPACITY;
    uint8_t *keep = static_cast<uint8_t *>(workspace);
    uint32_t *counts = reinterpret_cast<uint32_t *>(keep + (g->n + 255) / 256 * 256);
    return hip_status(launch_cull(*g, cameras, camera, *mlp, out_index, jobs, job, out_logit, keep, counts,
                                  reinterpret_cast<hipStream_t>(stream)));
}

namespace {
// Host validation of the regulariser maps: sizes, and the inputs each
// present term needs.
ivrgs_status check_reg_maps(const ivrgs_reg_maps *m) {
    if (!m) return IVRGS_E_INVALID;
    if (m->height < 3 || m->width < 3 || m->n_gauss < 0) return IVRGS_E_SHAPE;
    if (m->normal && (!m->depth || !m->alpha)) return IVRGS_E_INVALID;
    if (m->shade && !m->target) return IVRGS_E_INVALID;
    if ((int64_t)m->height * m->width > ((int64_t)1 << 31)) return IVRGS_E_SHAPE;
    return IVRGS_OK;
}
}  // namespace

size_t ivrgs_reg_workspace_size(const ivrgs_reg_maps *maps) {
    if (check_reg_maps(maps) != IVRGS_OK) return 0;
    return reg_workspace_bytes(*maps);
}

ivrgs_status ivrgs_reg_fwd(const ivrgs_reg_maps *maps, const ivrgs_camera *camera, float *out_terms,
                           float *out_pseudo_normal, void *workspace, size_t workspace_bytes, void *stream) {
    const ivrgs_status st = check_reg_maps(maps);
    if (st != IVRGS_OK) return st;
    if (!camera || !out_terms || !workspace) return IVRGS_E_INVALID;
    if (out_pseudo_normal && (!maps->depth || !maps->alpha)) return IVRGS_E_INVALID;
    if (workspace_bytes < reg_workspace_bytes(*maps)) return IVRGS_E_CAPACITY;
    return hip_status(launch_reg_fwd(*maps, *camera, out_terms, out_pseudo_normal, workspace,
                                     reinterpret_cast<hipStream_t>(stream)));
}

ivrgs_status ivrgs_reg_bwd(const ivrgs_reg_maps *maps, const ivrgs_camera *camera, const float *terms,
                           const float *grad_terms, float *grad_normal, float *grad_delta_c, float *grad_shade,
                           float *grad_opacity, float *grad_depth, void *stream) {
    const ivrgs_status st = check_reg_maps(maps);
    if (st != IVRGS_OK) return st;
    if (!camera || !terms || !grad_terms) return IVRGS_E_INVALID;
    if ((grad_normal && !maps->normal) || (grad_delta_c && !maps->delta_c) || (grad_shade && !maps->shade) ||
        (grad_opacity && !maps->opacity))
        return IVRGS_E_INVALID;
    return hip_status(launch_reg_bwd(*maps, *camera, terms, grad_terms, grad_normal, grad_delta_c, grad_shade,
                                     grad_opacity, grad_depth, reinterpret_cast<hipStream_t>(stream)));
}

int32_t ivrgs_struct_size(int32_t which) {
    switch (which) {
    case 0: return (int32_t)sizeof(ivrgs_gaussians);
    case 1: return (int32_t)sizeof(ivrgs_camera);
    case 2: return (int32_t)sizeof(ivrgs_model_edit);
    case 3: return (int32_t)sizeof(ivrgs_job);
    case 4: return (int32_t)sizeof(ivrgs_batch);
    case 5: return (int32_t)sizeof(ivrgs_params);
    case 6: return (int32_t)sizeof(ivrgs_projected);
    case 7: return (int32_t)sizeof(ivrgs_bins);
    case 8: return (int32_t)sizeof(ivrgs_culler);
    case 9: return (int32_t)sizeof(ivrgs_explore_opts);
    case 10: return (int32_t)sizeof(ivrgs_vq_model);
    case 11: return (int32_t)sizeof(ivrgs_vq_book);
    case 12: return (int32_t)sizeof(ivrgs_reg_maps);
    default: return -1;
    }
}

ivrgs_status ivrgs_get_error(const ivrgs_bins *bins, void *stream, int64_t *device_error,
                             int64_t *pairs_required) {
    if (!bins || !bins->status || !device_error) return IVRGS_E_INVALID;
    if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return IVRGS_E_HIP;
    int64_t st[6] = {0, 0, 0, 0, 0, 0};
    if (hipMemcpy(st, bins->status, sizeof st, hipMemcpyDeviceToHost) != hipSuccess) return IVRGS_E_HIP;
    *device_error = st[1] | st[4];
    if (pairs_required) *pairs_required = st[0] > st[5] ? st[0] : st[5];
    const int64_t zero[2] = {0, 0};
    if (hipMemcpy(bins->status + 4, zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess) return IVRGS_E_HIP;
    return IVRGS_OK;
}

const char *ivrgs_status_string(ivrgs_status s) {
    switch (s) {
    case IVRGS_OK: return "ok";
    case IVRGS_E_INVALID: return "invalid argument";
    case IVRGS_E_SHAPE: return "inconsistent shape";
    case IVRGS_E_CAPACITY: return "workspace or capacity too small";
    case IVRGS_E_HIP: return "HIP runtime error";
    case IVRGS_E_UNSUPPORTED: return "unsupported setting";
    default: return "unknown status";
    }
}

}  // extern "C"
