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
// backward visits the records a few at a time (their order-free work, then
// the chain), sums the group's values over the wave with one reduce-scatter
// and adds them with one atomic per value.
#include "launch.hpp"

namespace ivrgs {

namespace {

// per-record sums of the backward: GO, GX, GY, GQA..GQC, the image's colour
// (when the image's backward is folded in), depth, attributes
constexpr int kAuxAcc = 7 + 3 + kAuxMax;
static_assert(2 * kAuxAcc <= 64, "at least two records per reduce-scatter of 64 values");

// Per-wave LDS: the compacted records of one step.
constexpr int kAuxQuads = (kAuxMax + 3) / 4;  // float4s per attribute row

// Row stride of the attributes: n_attr rounded up to a multiple of 4.
__host__ __device__ __forceinline__ int attr_stride(int n_attr) { return (n_attr + 3) & ~3; }

// The backward reads a group of up to four records at fixed offsets from
// its first slot, so a group that starts at slot 63 reads three spare slots.
constexpr int kAuxSlots = 64 + 3;
struct AuxSlots {
    float4 f0[kAuxSlots];             // mean x, mean y, qa, qb
    float4 f1[kAuxSlots];             // qc, opacity, depth, cutoff
    float4 sa[kAuxQuads][kAuxSlots];  // attribute row, four at a time
    float4 fc[kAuxSlots];             // the image's colour r, g, b (the backward with the image folded in)
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
            S.fc[slot] = make_float4(r1.z, r1.w, r2.x, 0.f);
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
                pass[g] = valid;  // the alpha test decides (below the cutoff alpha < alpha_min)
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
// same record-gradient moments as the image backward.  Records are visited
// kG at a time (kN attributes: kG = min(4, 64 / (7 + kN)) records of 7 + kN
// values fill one 64-value reduce-scatter): the order-free part (offset,
// exponent, alpha, 1 / (1 - alpha), ga, the alpha-min and cap tests)
// of the group first, then the front-to-back chain, then one reduce-scatter
// of the group's values; lane v adds value v % (7 + kN) of record v / (7 +
// kN) to the record gradients (for the projection backward), the attribute
// gradients or, for the depth, the record's depth slot GZ (the projection
// backward takes it to the mean: depth = row 3 of R applied to the mean,
// plus t).
//
// kImg: the image's backward in the same walk.  Its colour is three more
// channels with gradient dL/d(rgb) of the image (rgba, dl), its alpha
// channel and background enter through g . out - dL/dA T_final, the same
// terms as the image backward's; the moments then come from the summed
// dL/dalpha, and the three colour sums go to the record gradients
// GCR..GCB.
template <int kN, bool kImg>
__global__ __launch_bounds__(kTilePix) void k_aux_bwd(ivrgs_batch b, Consts k, const float4 *__restrict__ rec,
                                                      const uint32_t *__restrict__ starts,
                                                      const uint32_t *__restrict__ sorted, int64_t n_tiles,
                                                      const float *__restrict__ attr,
                                                      const float *__restrict__ aux, const float *__restrict__ gaux,
                                                      const float *__restrict__ rgba, const float *__restrict__ dl,
                                                      float *__restrict__ grec, float *__restrict__ gattr) {
    constexpr int kNi = kImg ? 3 : 0;                        // the image's colour channels
    constexpr int kNv = 1 + kN;                              // depth, attributes
    constexpr int kVpr = 6 + kNi + kNv;                      // values per record
    constexpr int kG = 64 / kVpr < 4 ? 64 / kVpr : 4;        // records per reduce-scatter
    constexpr int kQ = (kN + 3) / 4;                         // float4s of an attribute row
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
    float g[kNv];
    float gA = 0.f;
    {
        const int64_t plane = (int64_t)k.width * k.height, pix = (int64_t)y * k.width + x;
        const int64_t o = (int64_t)ji * kNv * plane + pix;
#pragma unroll
        for (int c = 0; c < kNv; ++c) {
            g[c] = inside ? gaux[o + c * plane] : 0.f;
            gA = fmaf(g[c], inside ? aux[o + c * plane] : 0.f, gA);
        }
    }
    bool any_g = false;
#pragma unroll
    for (int c = 0; c < kNv; ++c) any_g |= g[c] != 0.f;
    // the image: gradient of its colour, and g . out - dL/dA T_final
    float gi0 = 0.f, gi1 = 0.f, gi2 = 0.f;
    if constexpr (kImg) {
        if (inside) {
            const int64_t plane = (int64_t)k.width * k.height;
            const int64_t o = (int64_t)ji * 4 * plane + (int64_t)y * k.width + x;
            gi0 = dl[o];
            gi1 = dl[plane + o];
            gi2 = dl[2 * plane + o];
            const float gAi = dl[3 * plane + o];
            const float go = fmaf(gi2, rgba[2 * plane + o], fmaf(gi1, rgba[plane + o], gi0 * rgba[o]));
            gA += go - gAi * (1.f - rgba[3 * plane + o]);
            any_g |= (gi0 != 0.f) | (gi1 != 0.f) | (gi2 != 0.f) | (gAi != 0.f);
        }
    }
    float T = 1.f, gP = 0.f;
    bool alive = inside & any_g;
    const uint32_t start = starts[tile], end = starts[tile + 1];
    const bool my_slot = lane < kG * kVpr;
    const int my_g = my_slot ? lane / kVpr : 0, my_v = lane % kVpr;
    float acc[64];
#pragma unroll
    for (int q = kG * kVpr; q < 64; ++q) acc[q] = 0.f;  // never written
    AuxWalk W(b, job, rec, sorted, attr, kN, lane, end);
    // every slot starts as the zero record (opacity 0: no power anywhere)
    for (int i = lane; i < kAuxSlots; i += 64) {
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        S.f0[i] = S.f1[i] = S.fc[i] = z;
#pragma unroll
        for (int q = 0; q < kQ; ++q) S.sa[q][i] = z;
    }
    if (start < end) {
        W.load_ids(start);
        W.load_recs(start);
        if (start + 64 < end) W.load_ids(start + 64);
    }
    for (uint32_t base = start; base < end; base += 64) {
        const uint64_t live = __ballot(alive);
        if (live == 0ull) break;
        const int cnt = W.step(base, alive_box(live, sx, sy), S);
        // the compacted records are slots 0 .. cnt - 1, in list order: a group
        // is kG consecutive slots, read at fixed offsets from its first
        for (int sl = 0; sl < cnt; sl += kG) {
            int src[kG];
            bool valid[kG];
#pragma unroll
            for (int gg = 0; gg < kG; ++gg) {
                valid[gg] = sl + gg < cnt;  // wave-uniform
                // a slot past the step's records holds a finite record (an
                // earlier step's, or the zero record): its terms are masked
                src[gg] = sl + gg;
            }
            // order-free part of the group
            float dx[kG], dy[kG], G[kG], raw[kG], al[kG], om[kG], inv[kG], ga[kG];
            bool use[kG], free_a[kG];
#pragma unroll
            for (int gg = 0; gg < kG; ++gg) {
                const float4 fa = S.f0[src[gg]], fc = S.f1[src[gg]];
                dx[gg] = px - fa.x;
                dy[gg] = py - fa.y;
                const float p2 = splat_exponent(fa.z, fa.w, fc.x, dx[gg], dy[gg]);
                G[gg] = fast_exp2(p2);
                raw[gg] = fc.y * G[gg];
                al[gg] = fminf(k.alpha_max, raw[gg]);
                om[gg] = 1.f - al[gg];
                inv[gg] = __builtin_amdgcn_rcpf(om[gg]);
                float d = g[0] * fc.z;
#pragma unroll
                for (int q = 0; q < kQ; ++q) {
                    const float4 a4 = S.sa[q][src[gg]];
                    d = fmaf(g[1 + 4 * q], a4.x, d);
                    if (4 * q + 1 < kN) d = fmaf(g[2 + 4 * q], a4.y, d);
                    if (4 * q + 2 < kN) d = fmaf(g[3 + 4 * q], a4.z, d);
                    if (4 * q + 3 < kN) d = fmaf(g[4 + 4 * q], a4.w, d);
                }
                if constexpr (kImg) {
                    const float4 c4 = S.fc[src[gg]];
                    d = fmaf(gi2, c4.z, fmaf(gi1, c4.y, fmaf(gi0, c4.x, d)));
                }
                ga[gg] = d;
                // the alpha test alone (below the cutoff alpha < alpha_min
                // is certain: the two decide the same)
                use[gg] = valid[gg] & (al[gg] >= k.alpha_min);
                // no gradient through alpha where the cap is active
                free_a[gg] = raw[gg] <= k.alpha_max;
            }
            // the front-to-back chain
            bool any = false;
#pragma unroll
            for (int gg = 0; gg < kG; ++gg) {
                const float Tn = T * om[gg];
                const bool stop = alive & use[gg] & (Tn < k.T_min);
                const bool comp = alive & use[gg] & !stop;
                const float w = comp ? al[gg] * T : 0.f;
                gP = fmaf(w, ga[gg], gP);
                const float dA = fmaf(gP - gA, inv[gg], T * ga[gg]);
                const float dLdo = (comp & free_a[gg]) ? dA : 0.f;
                const float dp = dLdo * G[gg];  // D without the factor o'
                float *v = acc + gg * kVpr;
                v[0] = dp;  // GO
                const float dpx = dp * dx[gg], dpy = dp * dy[gg];
                v[1] = dpx;           // GX
                v[2] = dpy;           // GY
                v[3] = dpx * dx[gg];  // GQA
                v[4] = dpx * dy[gg];  // GQB
                v[5] = dpy * dy[gg];  // GQC
                if constexpr (kImg) {
                    v[6] = w * gi0;  // GCR .. GCB
                    v[7] = w * gi1;
                    v[8] = w * gi2;
                }
#pragma unroll
                for (int c = 0; c < kNv; ++c) v[6 + kNi + c] = w * g[c];  // depth, attributes
                T = comp ? Tn : T;
                alive = alive & !stop;
                any = any | comp;
            }
            if (__ballot(any) != 0ull) {
                const float tot = reduce_scatter64(acc);
                // a record that composites nowhere has all sums exactly 0
                if (my_slot && tot != 0.f) {
                    int sl = src[0];
#pragma unroll
                    for (int gg = 1; gg < kG; ++gg) sl = my_g == gg ? src[gg] : sl;
                    const uint32_t r = S.rid[sl];
                    const int64_t gi = S.gid[sl];
                    if (my_v < 6) {
                        const int row = my_v == 0 ? GO : (my_v == 1 ? GX : (my_v == 2 ? GY : GQA + (my_v - 3)));
                        atomicAdd(&grec[(size_t)r * kGradStride + row], tot);
                    } else if (my_v < 6 + kNi) {
                        atomicAdd(&grec[(size_t)r * kGradStride + GCR + (my_v - 6)], tot);
                    } else if (my_v == 6 + kNi) {
                        atomicAdd(&grec[(size_t)r * kGradStride + GZ], tot);
                    } else {
                        atomicAdd(&gattr[gi * attr_stride(kN) + (my_v - 7 - kNi)], tot);
                    }
                }
            }
            if (__ballot(alive) == 0ull) break;  // every pixel of the wave is done
        }
    }
}

// Attribute rows of the editable stage, one thread per Gaussian: the unit
// normal (the length clamped below at kNormalFloor), delta-c, k_a, k_d,
// k_s, beta and two zero pad entries, as three 16-byte stores.
constexpr float kNormalFloor = 1e-12f;
constexpr int kEditAttrStride = 12;

__global__ __launch_bounds__(256) void k_edit_attr_fwd(const float *__restrict__ normal,
                                                       const float *__restrict__ color,
                                                       const float *__restrict__ shade, int64_t n,
                                                       float4 *__restrict__ attr) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float nx = normal[i], ny = normal[n + i], nz = normal[2 * n + i];
    const float inv = 1.f / fmaxf(sqrtf(fmaf(nz, nz, fmaf(ny, ny, nx * nx))), kNormalFloor);
    float4 *row = attr + 3 * i;
    row[0] = make_float4(nx * inv, ny * inv, nz * inv, color[i]);
    row[1] = make_float4(color[n + i], color[2 * n + i], shade[i], shade[n + i]);
    row[2] = make_float4(shade[2 * n + i], shade[3 * n + i], 0.f, 0.f);
}

// Backward of the rows: with u the unit normal and L the (clamped) length,
// d u / d normal = (I - u u^T) / L above the floor and I / floor at it.
// Adds into the plane gradients (each Gaussian once).
__global__ __launch_bounds__(256) void k_edit_attr_bwd(const float *__restrict__ normal, int64_t n,
                                                       const float4 *__restrict__ grad_attr,
                                                       float *__restrict__ gnormal, float *__restrict__ gcolor,
                                                       float *__restrict__ gshade) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float nx = normal[i], ny = normal[n + i], nz = normal[2 * n + i];
    const float len = sqrtf(fmaf(nz, nz, fmaf(ny, ny, nx * nx)));
    const bool above = len > kNormalFloor;
    const float inv = 1.f / (above ? len : kNormalFloor);
    const float4 a = grad_attr[3 * i], b = grad_attr[3 * i + 1], c = grad_attr[3 * i + 2];
    float gx = a.x, gy = a.y, gz = a.z;
    if (above) {
        const float ux = nx * inv, uy = ny * inv, uz = nz * inv;
        const float dot = fmaf(uz, gz, fmaf(uy, gy, ux * gx));
        gx = fmaf(-ux, dot, gx);
        gy = fmaf(-uy, dot, gy);
        gz = fmaf(-uz, dot, gz);
    }
    gnormal[i] += gx * inv;
    gnormal[n + i] += gy * inv;
    gnormal[2 * n + i] += gz * inv;
    gcolor[i] += a.w;
    gcolor[n + i] += b.x;
    gcolor[2 * n + i] += b.y;
    gshade[i] += b.z;
    gshade[n + i] += b.w;
    gshade[2 * n + i] += c.x;
    gshade[3 * n + i] += c.y;
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
                          const float *aux, const float *grad_aux, float *grec, float *grad_attr,
                          hipStream_t s, const float *rgba, const float *dl) {
    if (n_tiles == 0) return hipSuccess;
    TimedScope ts(TK_AUX, s);
    const float4 *rec4 = reinterpret_cast<const float4 *>(rec);
    const bool img = rgba != nullptr;
    switch (n_attr) {
#define IVRGS_AUX_BWD(N)                                                                                       \
    case N:                                                                                                    \
        if (img)                                                                                               \
            hipLaunchKernelGGL((k_aux_bwd<N, true>), dim3((unsigned)n_tiles), dim3(kTilePix), 0, s, b, k, rec4,  \
                               starts, sorted, n_tiles, attr, aux, grad_aux, rgba, dl, grec, grad_attr);         \
        else                                                                                                   \
            hipLaunchKernelGGL((k_aux_bwd<N, false>), dim3((unsigned)n_tiles), dim3(kTilePix), 0, s, b, k, rec4, \
                               starts, sorted, n_tiles, attr, aux, grad_aux, nullptr, nullptr, grec, grad_attr); \
        break;
        IVRGS_AUX_BWD(0) IVRGS_AUX_BWD(1) IVRGS_AUX_BWD(2) IVRGS_AUX_BWD(3) IVRGS_AUX_BWD(4) IVRGS_AUX_BWD(5)
        IVRGS_AUX_BWD(6) IVRGS_AUX_BWD(7) IVRGS_AUX_BWD(8) IVRGS_AUX_BWD(9) IVRGS_AUX_BWD(10) IVRGS_AUX_BWD(11)
        IVRGS_AUX_BWD(12) IVRGS_AUX_BWD(13) IVRGS_AUX_BWD(14) IVRGS_AUX_BWD(15)
#undef IVRGS_AUX_BWD
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_edit_attr_fwd(const float *normal, const float *color, const float *shade, int64_t n, float *attr,
                                hipStream_t s) {
    if (n == 0) return hipSuccess;
    TimedScope ts(TK_AUX, s);
    hipLaunchKernelGGL(k_edit_attr_fwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, normal, color, shade, n,
                       reinterpret_cast<float4 *>(attr));
    return hipGetLastError();
}

hipError_t launch_edit_attr_bwd(const float *normal, int64_t n, const float *grad_attr, float *grad_normal,
                                float *grad_color, float *grad_shade, hipStream_t s) {
    if (n == 0) return hipSuccess;
    TimedScope ts(TK_AUX, s);
    hipLaunchKernelGGL(k_edit_attr_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, normal, n,
                       reinterpret_cast<const float4 *>(grad_attr), grad_normal, grad_color, grad_shade);
    return hipGetLastError();
}

}  // namespace ivrgs
