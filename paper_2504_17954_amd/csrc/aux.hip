// Auxiliary maps composited with the image's weights: the camera-space
// depth and normal maps of Eq. 5, and the offset-colour and shading maps of
// Sec. 4.3 that the training regularisers read; and their backward, to the
// attributes and, through alpha and the depth, to the geometry.
//
// One workgroup per 16x16 tile, one pixel per thread, every pixel walking
// its tile's list in order with the image forward's arithmetic, so the
// composited pairs are exactly those of the image.  The forward runs each
// wave on its own over its 8x8 quadrant with the records in registers.  The
// backward stages the list through LDS 256 records at a time, so that the
// four waves can sum each record's gradients in LDS before one set of global
// atomics per workgroup; each wave takes the staged records 64 at a time
// into registers.
#include "launch.hpp"

namespace ivrgs {

namespace {

constexpr int kAuxChunk = 256;        // records staged per pass
constexpr int kAuxAcc = 7 + kAuxMax;  // per-record sums of the backward: GO, GX, GY, GQA..GQC, depth, attributes
static_assert(kAuxAcc <= 32, "one reduce-scatter of 32 values per record");

struct AuxStage {
    float4 s0[kAuxChunk];  // mean x, mean y, qa, qb
    float4 s1[kAuxChunk];  // qc, opacity, depth, cutoff
    float sa[kAuxMax][kAuxChunk];
    int64_t gid[kAuxChunk];
    uint32_t rid[kAuxChunk];
    uint32_t wmask[kAuxChunk];  // bit w: the record can reach wave w's 16x4 strip of the tile
    int any_alive;
};

// Stage records [base, base + cnt) of the list: fields from the projected
// record, attributes from the record's Gaussian.
__device__ __forceinline__ void stage(AuxStage &S, const ivrgs_batch &b, const ivrgs_job &job,
                                      const float4 *__restrict__ rec, const uint32_t *__restrict__ sorted,
                                      uint32_t base, uint32_t end, const float *__restrict__ attr, int n_attr,
                                      int tx0, int ty0) {
    const uint32_t e = base + threadIdx.x;
    if (e < end) {
        const uint32_t r = sorted[e];
        const float4 r0 = rec[3 * (size_t)r], r1 = rec[3 * (size_t)r + 1], r2 = rec[3 * (size_t)r + 2];
        S.s0[threadIdx.x] = r0;
        S.s1[threadIdx.x] = make_float4(r1.x, r1.y, r2.y, r2.z);
        // the binning's conservative ellipse-box test, per wave strip: a wave
        // skips a record that cannot reach any of its pixels
        const HitTest h = make_hit_test(r0, r1, r2);
        uint32_t m = 0;
#pragma unroll
        for (int w = 0; w < kTilePix / 64; ++w)
            m |= box_hit(h, tx0, ty0 + w * (64 / kTile), kTile, 64 / kTile) ? 1u << w : 0u;
        S.wmask[threadIdx.x] = m;
        const int64_t g = job_gaussian(job, b.gauss_index, (int)((int64_t)r - job.rec_begin));
        S.gid[threadIdx.x] = g;
        S.rid[threadIdx.x] = r;
#pragma unroll
        for (int c = 0; c < kAuxMax; ++c)
            if (c < n_attr) S.sa[c][threadIdx.x] = attr[(int64_t)c * b.g.n + g];
    }
}

// One pixel's step over a staged record, the forward's decisions exactly.
struct Step {
    float dx, dy, G, raw, al, w;
    bool comp;
};

__device__ __forceinline__ Step step(const Consts &k, float4 a, float4 c, float px, float py, float &T,
                                     bool &alive) {
    Step s;
    s.dx = px - a.x;
    s.dy = py - a.y;
    const float p2 = splat_exponent(a.z, a.w, c.x, s.dx, s.dy);
    const bool pass = alive && p2 >= c.w;  // below the cutoff alpha < alpha_min is certain
    s.G = fast_exp2(p2);
    s.raw = c.y * s.G;
    s.al = fminf(k.alpha_max, s.raw);
    const float Tn = T * (1.f - s.al);
    const bool use = pass && s.al >= k.alpha_min;
    const bool stop = use && Tn < k.T_min;
    s.comp = use && !stop;
    s.w = s.comp ? s.al * T : 0.f;
    T = s.comp ? Tn : T;
    alive = alive && !stop;
    return s;
}

// Forward: each wave owns an 8x8 quadrant of the tile and walks the list on
// its own (no LDS, no barrier), 64 records per step: lane l holds record
// base + l in registers (ids loaded two steps ahead, records and attributes
// one step ahead, so the walk does not wait on the gathers), the
// ellipse-box test against the quadrant picks the records to visit, and a
// visited record's fields are broadcast from its lane.
__global__ __launch_bounds__(kTilePix) void k_aux_fwd(ivrgs_batch b, Consts k, const float4 *__restrict__ rec,
                                                      const uint32_t *__restrict__ starts,
                                                      const uint32_t *__restrict__ sorted, int64_t n_tiles,
                                                      const float *__restrict__ attr, int n_attr,
                                                      float *__restrict__ aux) {
    if (starts[n_tiles] == 0xFFFFFFFFu) return;  // pair capacity exceeded: nothing is rendered
    const int64_t tile = blockIdx.x;
    const int ji = (int)(tile / k.tiles_per_job), lt = (int)(tile % k.tiles_per_job);
    const ivrgs_job job = b.jobs[ji];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sx = (lt % k.tiles_x) * kTile + 8 * (wave & 1), sy = (lt / k.tiles_x) * kTile + 8 * (wave >> 1);
    const int x = sx + (lane & 7), y = sy + (lane >> 3);
    const bool inside = x < k.width && y < k.height;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    float T = 1.f, acc[1 + kAuxMax];
#pragma unroll
    for (int c = 0; c < 1 + kAuxMax; ++c) acc[c] = 0.f;
    bool alive = inside;
    const uint32_t start = starts[tile], end = starts[tile + 1];

    float4 n0, n1, n2;
    float na[kAuxMax];
    uint32_t pid = 0;
    auto load_ids = [&](uint32_t base) {
        if (lane < (int)(end - base)) pid = sorted[base + lane];
    };
    auto load_recs = [&](uint32_t base) {
        if (lane < (int)(end - base)) {
            n0 = rec[3 * (size_t)pid];
            n1 = rec[3 * (size_t)pid + 1];
            n2 = rec[3 * (size_t)pid + 2];
            const int64_t g = job_gaussian(job, b.gauss_index, (int)((int64_t)pid - job.rec_begin));
#pragma unroll
            for (int c = 0; c < kAuxMax; ++c)
                if (c < n_attr) na[c] = attr[(int64_t)c * b.g.n + g];
        }
    };
    auto bc = [](float v, int src) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src)); };
    if (start < end) {
        load_ids(start);
        load_recs(start);
        if (end - start > 64) load_ids(start + 64);
    }
    for (uint32_t base = start; base < end; base += 64) {
        if (__ballot(alive) == 0ull) break;  // every pixel of the quadrant is done
        const float4 r0 = n0, r1 = n1, r2 = n2;
        float a[kAuxMax];
#pragma unroll
        for (int c = 0; c < kAuxMax; ++c) a[c] = na[c];
        const bool touch = lane < (int)(end - base) && box_hit(make_hit_test(r0, r1, r2), sx, sy, 8, 8);
        if (end - base > 64) load_recs(base + 64);
        if (end - base > 128) load_ids(base + 128);
        uint64_t m = __ballot(touch);
        while (m) {
            const int src = __builtin_ctzll(m);  // records in list order
            m &= m - 1;
            const float4 fa = make_float4(bc(r0.x, src), bc(r0.y, src), bc(r0.z, src), bc(r0.w, src));
            const float4 fc = make_float4(bc(r1.x, src), bc(r1.y, src), bc(r2.y, src), bc(r2.z, src));
            const Step s = step(k, fa, fc, px, py, T, alive);
            if (__ballot(s.comp) != 0ull) {  // wave-uniform
                acc[0] = fmaf(s.w, fc.z, acc[0]);
#pragma unroll
                for (int c = 0; c < kAuxMax; ++c)
                    if (c < n_attr) acc[1 + c] = fmaf(s.w, bc(a[c], src), acc[1 + c]);
            }
            if (__ballot(alive) == 0ull) break;
        }
    }
    if (!inside) return;
    const int64_t plane = (int64_t)k.width * k.height, pix = (int64_t)y * k.width + x;
    float *out = aux + (int64_t)ji * (1 + n_attr) * plane + pix;
    out[0] = acc[0];
#pragma unroll
    for (int c = 0; c < kAuxMax; ++c)
        if (c < n_attr) out[(1 + c) * plane] = acc[1 + c];
}

// Per pixel: g = dL/d(aux maps), A = the maps from the forward.  For each
// composited pair, with ga = g . (depth, attributes) of the record and the
// prefix P = sum of w ga over the pairs up to this one, dL/dalpha =
// T ga - (g . A - P) / (1 - alpha) (the maps carry no background); then the
// same record-gradient moments as the image backward.  The wave reduces all
// of a record's values in one reduce-scatter and adds them into LDS; the workgroup then adds the record's sums into
// the record gradients (for the projection backward), the attribute
// gradients and, for the depth, the mean gradient (depth = row 3 of R
// applied to the mean, plus t).
__global__ __launch_bounds__(kTilePix) void k_aux_bwd(ivrgs_batch b, Consts k, const float4 *__restrict__ rec,
                                                      const uint32_t *__restrict__ starts,
                                                      const uint32_t *__restrict__ sorted, int64_t n_tiles,
                                                      const float *__restrict__ attr, int n_attr,
                                                      const float *__restrict__ aux, const float *__restrict__ gaux,
                                                      float *__restrict__ grec, float *__restrict__ gattr,
                                                      float *__restrict__ gmean) {
    if (starts[n_tiles] == 0xFFFFFFFFu) return;
    __shared__ AuxStage S;
    __shared__ float acc[kAuxChunk][kAuxAcc];
    const int64_t tile = blockIdx.x;
    const int ji = (int)(tile / k.tiles_per_job), lt = (int)(tile % k.tiles_per_job);
    const ivrgs_job job = b.jobs[ji];
    const int tx0 = (lt % k.tiles_x) * kTile, ty0 = (lt / k.tiles_x) * kTile;
    const int x = tx0 + (threadIdx.x & (kTile - 1));
    const int y = ty0 + threadIdx.x / kTile;
    const uint32_t wave_bit = 1u << (threadIdx.x >> 6);
    const bool inside = x < k.width && y < k.height;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const int nv = 1 + n_attr;
    float g[1 + kAuxMax];
    float gA = 0.f;
    {
        const int64_t plane = (int64_t)k.width * k.height, pix = (int64_t)y * k.width + x;
        const int64_t o = (int64_t)ji * nv * plane + pix;
#pragma unroll
        for (int c = 0; c < 1 + kAuxMax; ++c) {
            const bool on = inside && c < nv;
            g[c] = on ? gaux[o + c * plane] : 0.f;
            gA = fmaf(g[c], on ? aux[o + c * plane] : 0.f, gA);
        }
    }
    const ivrgs_camera &cam = b.cameras[job.camera];
    float T = 1.f, gP = 0.f;
    bool alive = inside;
    const uint32_t beg = starts[tile], end = starts[tile + 1];
    const int lane = threadIdx.x & 63;
    for (uint32_t base = beg; base < end; base += kAuxChunk) {
        __syncthreads();
        if (threadIdx.x == 0) S.any_alive = 0;
        stage(S, b, job, rec, sorted, base, end, attr, n_attr, tx0, ty0);
        for (int v = 0; v < kAuxAcc; ++v) acc[threadIdx.x][v] = 0.f;
        __syncthreads();
        if (alive) S.any_alive = 1;
        __syncthreads();
        if (!S.any_alive) break;
        const int cnt = (int)min((uint32_t)kAuxChunk, end - base);
        auto bc = [](float v, int src) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src)); };
        // 64 staged records at a time into registers (lane l: record
        // sub * 64 + l), one LDS round trip; the records reaching this wave's
        // strip are then visited in order with their fields broadcast
        for (int sub = 0; sub * 64 < cnt; ++sub) {
            if (__ballot(alive) == 0ull) break;  // this wave's pixels are done (it still meets the barriers)
            const int li = sub * 64 + lane;
            const bool have = li < cnt;
            const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
            const float4 q0 = have ? S.s0[li] : z4, q1 = have ? S.s1[li] : z4;
            float qa[kAuxMax];
#pragma unroll
            for (int c = 0; c < kAuxMax; ++c) qa[c] = have && c < n_attr ? S.sa[c][li] : 0.f;
            uint64_t visit = __ballot(have && (S.wmask[have ? li : 0] & wave_bit));
            while (visit) {
                const int src = __builtin_ctzll(visit);  // list order
                visit &= visit - 1;
                const int i = sub * 64 + src;  // position in the staged chunk
                const float4 fa = make_float4(bc(q0.x, src), bc(q0.y, src), bc(q0.z, src), bc(q0.w, src));
                const float4 fc = make_float4(bc(q1.x, src), bc(q1.y, src), bc(q1.z, src), bc(q1.w, src));
                const float T0 = T;  // transmittance in front of this record
                const Step s = step(k, fa, fc, px, py, T, alive);
                if (__ballot(s.comp) != 0ull) {  // wave-uniform: something to add
                    float ga = g[0] * fc.z;
#pragma unroll
                    for (int c = 0; c < kAuxMax; ++c)
                        if (c < n_attr) ga = fmaf(g[1 + c], bc(qa[c], src), ga);
                    gP = fmaf(s.w, ga, gP);
                    const float dA = s.comp ? T0 * ga - (gA - gP) / (1.f - s.al) : 0.f;
                    const float dLdo = s.raw <= k.alpha_max ? dA : 0.f;  // no gradient through alpha where capped
                    const float dp = dLdo * s.raw;
                    float vals[kAuxAcc];
                    vals[0] = dLdo * s.G;        // GO
                    vals[1] = dp * s.dx;         // GX
                    vals[2] = dp * s.dy;         // GY
                    vals[3] = dp * s.dx * s.dx;  // GQA
                    vals[4] = dp * s.dx * s.dy;  // GQB
                    vals[5] = dp * s.dy * s.dy;  // GQC
#pragma unroll
                    for (int c = 0; c < 1 + kAuxMax; ++c) vals[6 + c] = s.w * g[c];  // depth, then attributes
                    // one reduce-scatter for all the values: lanes 2v, 2v + 1
                    // hold the wave total of value v
                    float v32[32];
#pragma unroll
                    for (int v = 0; v < 32; ++v) v32[v] = v < kAuxAcc ? vals[v] : 0.f;
                    const float tot = reduce_scatter32(v32);
                    const int vi = lane >> 1;
                    if ((lane & 1) == 0 && vi < 6 + nv && tot != 0.f) atomicAdd(&acc[i][vi], tot);
                }
                if (__ballot(alive) == 0ull) break;
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const float *a = acc[threadIdx.x];
            const uint32_t r = S.rid[threadIdx.x];
            const int64_t gi = S.gid[threadIdx.x];
            float *gr = grec + (size_t)r * kGradStride;
            if (a[0] != 0.f) atomicAdd(&gr[GO], a[0]);
            if (a[1] != 0.f) atomicAdd(&gr[GX], a[1]);
            if (a[2] != 0.f) atomicAdd(&gr[GY], a[2]);
            if (a[3] != 0.f) atomicAdd(&gr[GQA], a[3]);
            if (a[4] != 0.f) atomicAdd(&gr[GQB], a[4]);
            if (a[5] != 0.f) atomicAdd(&gr[GQC], a[5]);
            if (a[6] != 0.f) {
                atomicAdd(&gmean[gi], a[6] * cam.R[6]);
                atomicAdd(&gmean[b.g.n + gi], a[6] * cam.R[7]);
                atomicAdd(&gmean[2 * b.g.n + gi], a[6] * cam.R[8]);
            }
            for (int c = 0; c < n_attr; ++c)
                if (a[7 + c] != 0.f) atomicAdd(&gattr[(int64_t)c * b.g.n + gi], a[7 + c]);  // LDS row: indexable
        }
    }
}

}  // namespace

hipError_t launch_aux_fwd(const ivrgs_batch &b, const Consts &k, int64_t n_tiles, const float *rec,
                          const uint32_t *starts, const uint32_t *sorted, const float *attr, int n_attr, float *aux,
                          hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    TimedScope ts(TK_AUX, s);
    hipLaunchKernelGGL(k_aux_fwd, dim3((unsigned)n_tiles), dim3(kTilePix), 0, s, b, k,
                       reinterpret_cast<const float4 *>(rec), starts, sorted, n_tiles, attr, n_attr, aux);
    return hipGetLastError();
}

hipError_t launch_aux_bwd(const ivrgs_batch &b, const Consts &k, int64_t n_tiles, const float *rec,
                          const uint32_t *starts, const uint32_t *sorted, const float *attr, int n_attr,
                          const float *aux, const float *grad_aux, float *grec, float *grad_attr, float *grad_mean,
                          hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    TimedScope ts(TK_AUX, s);
    hipLaunchKernelGGL(k_aux_bwd, dim3((unsigned)n_tiles), dim3(kTilePix), 0, s, b, k,
                       reinterpret_cast<const float4 *>(rec), starts, sorted, n_tiles, attr, n_attr, aux, grad_aux,
                       grec, grad_attr, grad_mean);
    return hipGetLastError();
}

}  // namespace ivrgs
