// Auxiliary maps composited with the image's weights: the camera-space
// depth and normal maps of Eq. 5, and the offset-colour and shading maps of
// Sec. 4.3 that the training regularisers read; and their backward, to the
// attributes and, through alpha and the depth, to the geometry.
//
// One workgroup per 16x16 tile; each wave walks the tile's list on its own
// over its 8x8 quadrant, one pixel per lane, with the image forward's
// arithmetic, so the composited pairs are exactly those of the image.  A
// step gathers 64 records (and their attributes) into registers, one step
// ahead of its use; the records whose ellipse reaches the box of the
// quadrant's live pixels are compacted, in list order, into the wave's LDS
// slots, and each is read from there at one address for the whole wave.  No
// workgroup barrier: a wave stops when its own pixels are done.  The
// backward sums each composited record's values over the wave with one
// reduce-scatter and adds them with one atomic per value.
#include "launch.hpp"

namespace ivrgs {

namespace {

constexpr int kAuxAcc = 7 + kAuxMax;  // per-record sums of the backward: GO, GX, GY, GQA..GQC, depth, attributes
static_assert(kAuxAcc <= 32, "one reduce-scatter of 32 values per record");

// Per-wave LDS: the compacted records of one step.
constexpr int kAuxQuads = (kAuxMax + 3) / 4;  // float4s per attribute row

// Row stride of the attributes: n_attr rounded up to a multiple of 4.
__host__ __device__ __forceinline__ int attr_stride(int n_attr) { return (n_attr + 3) & ~3; }

struct AuxSlots {
    float4 f0[64];             // mean x, mean y, qa, qb
    float4 f1[64];             // qc, opacity, depth, cutoff
    float4 sa[kAuxQuads][64];  // attribute row, four at a time
    uint32_t rid[64], gid[64];
};

// The quadrant walk's per-wave state: pixel, gather pipeline (ids two steps
// ahead, records and attributes one step ahead).
struct AuxWalk {
    const ivrgs_batch &b;
    const ivrgs_job &job;
    const float4 *rec;
    const uint32_t *sorted;
    const float *attr;
    int n_attr, lane;
    uint32_t end;
    float4 n0, n1, n2;
    float4 na[kAuxQuads];
    uint32_t nid, pid;

    __device__ __forceinline__ AuxWalk(const ivrgs_batch &b_, const ivrgs_job &j_, const float4 *r_,
                                       const uint32_t *s_, const float *a_, int na_, int lane_, uint32_t end_)
        : b(b_), job(j_), rec(r_), sorted(s_), attr(a_), n_attr(na_), lane(lane_), end(end_), nid(0), pid(0) {
        n0 = n1 = n2 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int q = 0; q < kAuxQuads; ++q) na[q] = n0;
    }
    __device__ __forceinline__ void load_ids(uint32_t base) {
        if (base + lane < end) pid = sorted[base + lane];
    }
    __device__ __forceinline__ void load_recs(uint32_t base) {
        if (base + lane < end) {
            nid = pid;
            n0 = rec[kRecVec * (size_t)nid];
            n1 = rec[kRecVec * (size_t)nid + 1];
            n2 = rec[kRecVec * (size_t)nid + 2];
            const int64_t g = job_gaussian(job, b.gauss_index, (int)((int64_t)nid - job.rec_begin));
            // the record's attribute row, whole vectors
            const float4 *row = reinterpret_cast<const float4 *>(attr + g * attr_stride(n_attr));
#pragma unroll
            for (int q = 0; q < kAuxQuads; ++q)
                if (4 * q < n_attr) na[q] = row[q];
        }
    }
    // Takes the gathered records of the step at base, issues the next
    // gathers and compacts the records that reach the pixel box into the
    // slots; returns their number.
    __device__ __forceinline__ int step(uint32_t base, const PixBox &bx, AuxSlots &S) {
        const float4 r0 = n0, r1 = n1, r2 = n2;
        const uint32_t rid = nid;
        float4 a[kAuxQuads];
#pragma unroll
        for (int q = 0; q < kAuxQuads; ++q) a[q] = na[q];
        const bool touch = base + lane < end && box_hit(make_hit_test(r0, r1, r2), bx.x0, bx.y0, bx.w, bx.h);
        if (base + 64 < end) load_recs(base + 64);
        if (base + 128 < end) load_ids(base + 128);
        const uint64_t m = __ballot(touch);
        if (m == 0ull) return 0;
        wave_lds_sync();  // the previous step's reads are done
        if (touch) {
            const int slot = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            S.f0[slot] = r0;
            S.f1[slot] = make_float4(r1.x, r1.y, r2.y, r2.z);
#pragma unroll
            for (int q = 0; q < kAuxQuads; ++q)
                if (4 * q < n_attr) S.sa[q][slot] = a[q];
            S.rid[slot] = rid;
            S.gid[slot] = (uint32_t)job_gaussian(job, b.gauss_index, (int)((int64_t)rid - job.rec_begin));
        }
        wave_lds_sync();
        return __builtin_popcountll(m);
    }
};

// Forward: maps = sum over composited records of w * (depth, attributes).
__global__ __launch_bounds__(kTilePix) void k_aux_fwd(ivrgs_batch b, Consts k, const float4 *__restrict__ rec,
                                                      const uint32_t *__restrict__ starts,
                                                      const uint32_t *__restrict__ sorted, int64_t n_tiles,
                                                      const float *__restrict__ attr, int n_attr,
                                                      float *__restrict__ aux) {
    if (starts[n_tiles] == 0xFFFFFFFFu) return;  // pair capacity exceeded: nothing is rendered
    __shared__ AuxSlots slots[kTilePix / 64];
    const int64_t tile = blockIdx.x;
    const int ji = (int)(tile / k.tiles_per_job), lt = (int)(tile % k.tiles_per_job);
    const ivrgs_job job = b.jobs[ji];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    AuxSlots &S = slots[wave];
    const int sx = (lt % k.tiles_x) * kTile + 8 * (wave & 1), sy = (lt / k.tiles_x) * kTile + 8 * (wave >> 1);
    const int x = sx + (lane & 7), y = sy + (lane >> 3);
    const bool inside = x < k.width && y < k.height;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    float T = 1.f, acc[1 + kAuxMax];
#pragma unroll
    for (int c = 0; c < 1 + kAuxMax; ++c) acc[c] = 0.f;
    bool alive = inside;
    const uint32_t start = starts[tile], end = starts[tile + 1];
    AuxWalk W(b, job, rec, sorted, attr, n_attr, lane, end);
    if (start < end) {
        W.load_ids(start);
        W.load_recs(start);
        if (start + 64 < end) W.load_ids(start + 64);
    }
    for (uint32_t base = start; base < end; base += 64) {
        const uint64_t live = __ballot(alive);
        if (live == 0ull) break;  // every pixel of the quadrant is done
        const int cnt = W.step(base, alive_box(live, sx, sy), S);
        // records in groups of four: the order-free part (exponent, power,
        // alpha) of the four first, then the chain, then the sums of the
        // group's weighted depth and attributes when a pixel composites
        constexpr int kG = 4;
        for (int sl = 0; sl < cnt; sl += kG) {
            float al[kG], w[kG];
            bool pass[kG];
            int src[kG];
#pragma unroll
            for (int g = 0; g < kG; ++g) {
                const bool valid = sl + g < cnt;  // wave-uniform
                src[g] = valid ? sl + g : sl;
                const float4 fa = S.f0[src[g]], fc = S.f1[src[g]];
                const float p2 = splat_exponent(fa.z, fa.w, fc.x, px - fa.x, py - fa.y);
                pass[g] = valid & (p2 >= fc.w);  // below the cutoff alpha < alpha_min is certain
                al[g] = fminf(k.alpha_max, fc.y * fast_exp2(p2));
            }
            bool any = false;
#pragma unroll
            for (int g = 0; g < kG; ++g) {
                const float Tn = T * (1.f - al[g]);
                const bool use = alive & pass[g] & (al[g] >= k.alpha_min);
                const bool stop = use & (Tn < k.T_min);
                const bool comp = use & !stop;
                w[g] = comp ? al[g] * T : 0.f;
                T = comp ? Tn : T;
                alive = alive & !stop;
                any |= comp;
            }
            if (__ballot(any) != 0ull) {  // wave-uniform
#pragma unroll
                for (int g = 0; g < kG; ++g) {
                    acc[0] = fmaf(w[g], S.f1[src[g]].z, acc[0]);
#pragma unroll
                    for (int q = 0; q < kAuxQuads; ++q) {
                        if (4 * q >= n_attr) break;
                        const float4 a4 = S.sa[q][src[g]];
                        acc[1 + 4 * q] = fmaf(w[g], a4.x, acc[1 + 4 * q]);
                        if (4 * q + 1 < kAuxMax) acc[2 + 4 * q] = fmaf(w[g], a4.y, acc[2 + 4 * q]);
                        if (4 * q + 2 < kAuxMax) acc[3 + 4 * q] = fmaf(w[g], a4.z, acc[3 + 4 * q]);
                        if (4 * q + 3 < kAuxMax) acc[4 + 4 * q] = fmaf(w[g], a4.w, acc[4 + 4 * q]);
                    }
                }
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
// of a record's values in one reduce-scatter; lanes 2v add value v to the
// record gradients (for the projection backward), the attribute gradients
// or, for the depth, the mean gradient (depth = row 3 of R applied to the
// mean, plus t).
__global__ __launch_bounds__(kTilePix) void k_aux_bwd(ivrgs_batch b, Consts k, const float4 *__restrict__ rec,
                                                      const uint32_t *__restrict__ starts,
                                                      const uint32_t *__restrict__ sorted, int64_t n_tiles,
                                                      const float *__restrict__ attr, int n_attr,
                                                      const float *__restrict__ aux, const float *__restrict__ gaux,
                                                      float *__restrict__ grec, float *__restrict__ gattr,
                                                      float *__restrict__ gmean) {
    if (starts[n_tiles] == 0xFFFFFFFFu) return;
    __shared__ AuxSlots slots[kTilePix / 64];
    const int64_t tile = blockIdx.x;
    const int ji = (int)(tile / k.tiles_per_job), lt = (int)(tile % k.tiles_per_job);
    const ivrgs_job job = b.jobs[ji];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    AuxSlots &S = slots[wave];
    const int sx = (lt % k.tiles_x) * kTile + 8 * (wave & 1), sy = (lt / k.tiles_x) * kTile + 8 * (wave >> 1);
    const int x = sx + (lane & 7), y = sy + (lane >> 3);
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
    bool any_g = false;
#pragma unroll
    for (int c = 0; c < 1 + kAuxMax; ++c) any_g |= g[c] != 0.f;
    const ivrgs_camera &cam = b.cameras[job.camera];
    float T = 1.f, gP = 0.f;
    bool alive = inside & any_g;
    const uint32_t start = starts[tile], end = starts[tile + 1];
    const int vi = lane >> 1;
    const bool my_slot = (lane & 1) == 0 && vi < 6 + nv;
    AuxWalk W(b, job, rec, sorted, attr, n_attr, lane, end);
    if (start < end) {
        W.load_ids(start);
        W.load_recs(start);
        if (start + 64 < end) W.load_ids(start + 64);
    }
    for (uint32_t base = start; base < end; base += 64) {
        const uint64_t live = __ballot(alive);
        if (live == 0ull) break;
        const int cnt = W.step(base, alive_box(live, sx, sy), S);
        for (int sl = 0; sl < cnt; ++sl) {
            const float4 fa = S.f0[sl], fc = S.f1[sl];
            const float dx = px - fa.x, dy = py - fa.y;
            const float p2 = splat_exponent(fa.z, fa.w, fc.x, dx, dy);
            const bool pass = alive & (p2 >= fc.w);
            if (__ballot(pass) == 0ull) continue;  // wave-uniform: no live pixel reaches the cutoff
            const float G = fast_exp2(p2);
            const float raw = fc.y * G;
            const float al = fminf(k.alpha_max, raw);
            const float T0 = T;  // transmittance in front of this record
            const float Tn = T * (1.f - al);
            const bool use = pass & (al >= k.alpha_min);
            const bool stop = use & (Tn < k.T_min);
            const bool comp = use & !stop;
            const float w = comp ? al * T : 0.f;
            T = comp ? Tn : T;
            alive = alive & !stop;
            if (__ballot(comp) != 0ull) {  // wave-uniform: something to add
                float ga = g[0] * fc.z;
#pragma unroll
                for (int q = 0; q < kAuxQuads; ++q) {
                    if (4 * q >= n_attr) break;
                    const float4 a4 = S.sa[q][sl];
                    ga = fmaf(g[1 + 4 * q], a4.x, ga);
                    if (4 * q + 1 < kAuxMax) ga = fmaf(g[2 + 4 * q], a4.y, ga);
                    if (4 * q + 2 < kAuxMax) ga = fmaf(g[3 + 4 * q], a4.z, ga);
                    if (4 * q + 3 < kAuxMax) ga = fmaf(g[4 + 4 * q], a4.w, ga);
                }
                gP = fmaf(w, ga, gP);
                const float dA = fmaf(-(gA - gP), __builtin_amdgcn_rcpf(1.f - al), T0 * ga);
                // no gradient through alpha where the cap is active
                const float dLdo = (comp & (raw <= k.alpha_max)) ? dA : 0.f;
                const float dp = dLdo * raw;
                float v32[32];
                v32[0] = dLdo * G;  // GO
                const float dpx = dp * dx, dpy = dp * dy;
                v32[1] = dpx;       // GX
                v32[2] = dpy;       // GY
                v32[3] = dpx * dx;  // GQA
                v32[4] = dpx * dy;  // GQB
                v32[5] = dpy * dy;  // GQC
#pragma unroll
                for (int c = 0; c < 1 + kAuxMax; ++c) v32[6 + c] = c < nv ? w * g[c] : 0.f;  // depth, attributes
#pragma unroll
                for (int v = 7 + kAuxMax; v < 32; ++v) v32[v] = 0.f;
                // lanes 2v, 2v + 1 hold the wave total of value v
                const float tot = reduce_scatter32(v32);
                if (my_slot && tot != 0.f) {
                    const uint32_t r = S.rid[sl];
                    const int64_t gi = S.gid[sl];
                    if (vi < 6) {
                        const int row = vi == 0 ? GO : (vi == 1 ? GX : (vi == 2 ? GY : GQA + (vi - 3)));
                        atomicAdd(&grec[(size_t)r * kGradStride + row], tot);
                    } else if (vi == 6) {
                        atomicAdd(&gmean[gi], tot * cam.R[6]);
                        atomicAdd(&gmean[b.g.n + gi], tot * cam.R[7]);
                        atomicAdd(&gmean[2 * b.g.n + gi], tot * cam.R[8]);
                    } else {
                        atomicAdd(&gattr[gi * attr_stride(n_attr) + (vi - 7)], tot);
                    }
                }
            }
            if (__ballot(alive) == 0ull) break;
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
