// Front-to-back compositing (forward) and its recompute-based backward.
//
// One workgroup per 16x16 tile; each lane owns PX pixels (PX = 1, 2, 4, so a
// workgroup has 256/PX threads).  With one pixel per lane the forward and the
// backward run each wave on its own 8x8 quadrant of the tile: the wave
// gathers 64 records at a time into registers, tests them against the
// quadrant, and visits only the records that can reach it, broadcast lane by
// lane into scalar registers (the backward with PX > 1 pixels per lane does
// the same on a 16 x 4PX strip).  The
// forward with more pixels per lane gathers each batch of records into LDS
// for the whole workgroup and walks it by broadcast reads, skipping per wave
// the records that cannot reach the wave's pixels; a workgroup-wide OR ends
// the walk once every pixel has terminated.
// Compositing is plain FP32 VALU work (not a dense contraction), so no matrix
// cores are involved.
//
// The backward walks the same list front to back and recomputes alpha and T
// with the same instruction sequence as the forward.  Nothing per pixel is
// stored by the forward: the colour behind Gaussian i is out_rgb - P_i with
// P_i the recomputed prefix sum, and T_final = 1 - A.  Per-Gaussian partial
// gradients of three Gaussians are summed over the wave with one
// reduce-scatter and added to the records' gradients with one atomic per
// value.
#include <algorithm>

#include "launch.hpp"

namespace ivrgs {

struct TileGeom {
    int job, tx, ty;
};

__device__ __forceinline__ TileGeom tile_geom(const Consts &k, int64_t tile) {
    TileGeom g;
    g.job = (int)(tile / k.tiles_per_job);
    const int lt = (int)(tile % k.tiles_per_job);
    g.tx = lt % k.tiles_x;
    g.ty = lt / k.tiles_x;
    return g;
}

template <int PX>
__device__ __forceinline__ void pixel_of(const TileGeom &g, int j, int &x, int &y) {
    constexpr int NT = kTilePix / PX;
    const int p = threadIdx.x + j * NT;
    x = g.tx * kTile + (p & (kTile - 1));
    y = g.ty * kTile + p / kTile;
}

// Which waves of the workgroup own pixels the record can reach.  With one
// pixel per lane wave w owns rows 4w .. 4w+3 of the tile; with more pixels
// per lane a wave's pixels are spread over the tile and every wave is marked.
template <int PX>
__device__ __forceinline__ uint32_t wave_mask(const TileGeom &tg, float4 r0, float4 r1, float4 r2) {
    if (PX != 1) return 0xFu;
    const HitTest h = make_hit_test(r0, r1, r2);
    uint32_t m = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w)
        if (box_hit(h, tg.tx * kTile, tg.ty * kTile + 4 * w, kTile, 4)) m |= 1u << w;
    return m;
}

// Issue priority of a wave from the length of its tile's list.  All waves
// of a view start together, most finish within a few microseconds, and the
// view ends with the few tiles whose walks are longest; raising their
// priority lets them run at nearly the speed of a wave alone on its SIMD
// while the short walks fill the remaining issue slots.
__device__ __forceinline__ void walk_priority(uint32_t list_len) {
    if (list_len >= 2048u) __builtin_amdgcn_s_setprio(3);
    else if (list_len >= 1024u) __builtin_amdgcn_s_setprio(2);
    else if (list_len >= 512u) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);  // a persistent wave's next tile may be shorter
}

__device__ __forceinline__ float wave_max_to_lane63(float v) {
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false)));
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false)));
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false)));
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false)));
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xA, 0xF, false)));
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xC, 0xF, false)));
    return v;
}


// ----------------------------------------------------------------------------
// Forward of one tile (the whole workgroup takes part).
template <int PX, bool kMaxw, bool kCount>
__device__ __forceinline__ void fwd_tile(const Consts &k, const float4 *__restrict__ rec,
                                         const uint32_t *__restrict__ starts, const uint32_t *__restrict__ sorted,
                                         float *__restrict__ out, float *__restrict__ maxw,
                                         int64_t *__restrict__ status, int64_t tile) {
    constexpr int NT = kTilePix / PX;
    __shared__ float4 s0[NT], s1[NT];
    __shared__ float2 s2[NT];
    __shared__ uint32_t sid[NT];
    __shared__ uint32_t smask[NT];  // bit w: the record can reach wave w's pixels
    const TileGeom tg = tile_geom(k, tile);
    const uint32_t start = starts[tile], end = starts[tile + 1];

    float px[PX], py[PX], T[PX], C0[PX], C1[PX], C2[PX];
    bool alive[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        int x, y;
        pixel_of<PX>(tg, j, x, y);
        alive[j] = x < k.width && y < k.height;
        px[j] = (float)x + 0.5f;
        py[j] = (float)y + 0.5f;
        T[j] = 1.f;
        C0[j] = C1[j] = C2[j] = 0.f;
    }
    uint32_t evaluated = 0, composited = 0;
    for (uint32_t base = start; base < end; base += NT) {
        bool mine = false;
#pragma unroll
        for (int j = 0; j < PX; ++j) mine |= alive[j];
        if (!__syncthreads_or(mine)) break;
        const uint32_t idx = base + threadIdx.x;
        if (idx < end) {
            const uint32_t r = sorted[idx];
            const float4 r0 = rec[kRecVec * (size_t)r], r1 = rec[kRecVec * (size_t)r + 1], r2 = rec[kRecVec * (size_t)r + 2];
            s0[threadIdx.x] = r0;
            s1[threadIdx.x] = r1;
            s2[threadIdx.x] = make_float2(r2.x, r2.z);
            if (kMaxw) sid[threadIdx.x] = r;
            smask[threadIdx.x] = wave_mask<PX>(tg, r0, r1, r2);
        }
        __syncthreads();
        const int cnt = min((uint32_t)NT, end - base);
        const uint32_t my_bit = __builtin_amdgcn_readfirstlane(1u << (threadIdx.x >> 6));  // wave-uniform
        for (int i = 0; i < cnt; ++i) {
            if (__ballot(mine) == 0ull) break;
            if (!(__builtin_amdgcn_readfirstlane(smask[i]) & my_bit)) {  // wave-uniform
                // the record cannot reach this wave's pixels; the evaluations
                // the plain walk would make are still counted
                if (kCount)
                    for (int j = 0; j < PX; ++j) evaluated += alive[j] ? 1u : 0u;
                continue;
            }
            const float4 a = s0[i];
            const float4 c = s1[i];
            const float2 cc = s2[i];
            const float cb = cc.x;
            float wmax = 0.f;
#pragma unroll
            for (int j = 0; j < PX; ++j) {
                if (kCount) evaluated += alive[j] ? 1u : 0u;
                const float dx = px[j] - a.x, dy = py[j] - a.y;
                const float p2 = splat_exponent(a.z, a.w, c.x, dx, dy);
                // below the cutoff alpha < alpha_min is certain
                const bool pass = alive[j] && p2 >= cc.y;
                if (__ballot(pass) == 0ull) continue;  // wave-uniform
                // branch-free from here: a lane that does not composite adds
                // w = 0 times a finite colour, which leaves its sums unchanged
                const float G = fast_exp2(p2);
                const float al = fminf(k.alpha_max, c.y * G);
                const float Tn = T[j] * (1.f - al);
                const bool use = pass && al >= k.alpha_min;
                const bool stop = use && Tn < k.T_min;
                const bool comp = use && !stop;
                const float w = comp ? al * T[j] : 0.f;
                C0[j] = fmaf(w, c.z, C0[j]);
                C1[j] = fmaf(w, c.w, C1[j]);
                C2[j] = fmaf(w, cb, C2[j]);
                T[j] = comp ? Tn : T[j];
                alive[j] = alive[j] && !stop;
                if (kCount) composited += comp ? 1u : 0u;
                if (kMaxw) wmax = fmaxf(wmax, w);
            }
            if (kMaxw) {
                const uint64_t hit = __ballot(wmax > 0.f);
                if (hit) {
                    const float m = wave_max_to_lane63(wmax);
                    if (lane_id() == 63) atomicMax(reinterpret_cast<int *>(&maxw[sid[i]]), __float_as_int(m));
                }
            }
            mine = false;
#pragma unroll
            for (int j = 0; j < PX; ++j) mine |= alive[j];
        }
    }
    const size_t plane = (size_t)k.width * k.height;
    float *img = out + (size_t)tg.job * 4 * plane;
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        int x, y;
        pixel_of<PX>(tg, j, x, y);
        if (x >= k.width || y >= k.height) continue;
        const size_t o = (size_t)y * k.width + x;
        img[o] = C0[j] + T[j] * k.bg0;
        img[plane + o] = C1[j] + T[j] * k.bg1;
        img[2 * plane + o] = C2[j] + T[j] * k.bg2;
        img[3 * plane + o] = 1.f - T[j];
    }
    if (kCount && evaluated) {
        atomicAdd(reinterpret_cast<unsigned long long *>(&status[2]), (unsigned long long)evaluated);
        atomicAdd(reinterpret_cast<unsigned long long *>(&status[3]), (unsigned long long)composited);
    }
}

// Per-wave LDS of the one-pixel-per-lane walks: the records of one step of
// 64 that can reach the wave's pixels, compacted in list order, three float4
// each: (x, y, qa, qb), (qc, cutoff, opacity, r), (g, b, id, lane of the
// record in its step).
// The backward reads its groups of three at fixed offsets from the group's
// first slot, so a group that starts at slot 63 reads two spare slots.
struct WaveSlots {
    float4 f[64 + 2][3];
};

// The auxiliary maps composited in the image's walk: per compacted record up
// to four float4 of its attribute row (the depth rides in the record's third
// float4, in place of the lane index that only the counting walk reads).
struct MapSlots {
    float4 a[64][4];
};
struct MapsArgs {
    const ivrgs_job *jobs;
    const int32_t *gauss_index;
    const float4 *attr;  // rows of 4 kA floats per Gaussian
    float *aux;          // [n_jobs][1 + n_attr][H][W]
    int n_attr;
};

// Compacts the records of lanes with `touch` (ballot m) into the wave's
// slots, in lane order; returns their number.
__device__ __forceinline__ int compact_records(WaveSlots &slots, uint64_t m, bool touch, float4 r0, float4 r1,
                                               float4 r2, uint32_t rid, int lane) {
    wave_lds_sync();  // the previous step's reads are done
    if (touch) {
        const int slot = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        slots.f[slot][0] = r0;
        slots.f[slot][1] = make_float4(r1.x, r2.z, r1.y, r1.z);
        slots.f[slot][2] = make_float4(r1.w, r2.x, __uint_as_float(rid), __int_as_float(lane));
    }
    wave_lds_sync();
    return __builtin_popcountll(m);
}

// Forward of one tile with one pixel per lane, each wave on its own.  Wave
// w owns the 8x8 quadrant (w % 2, w / 2) of the tile and walks the tile's
// list 64 records at a time: every lane gathers one record into registers
// and tests it against the quadrant (the conservative ellipse-box test of the
// binning), a ballot gives the records that can reach it, and the wave visits
// only those, in list order, broadcasting each record's fields from its
// lane into scalar registers.  The next 64 records are gathered, and the ids
// of the 64 after them loaded, while the current ones are composited.  No LDS and no workgroup barrier: a wave
// stops as soon as its own 64 pixels are done.
//
// ckpt != nullptr: at every cut of the tile's list (split_of) the wave stores
// each pixel's state before the cut, (T, C) with T = -1 for a pixel that has
// already terminated, for the backward's segments.
//
// kA >= 0: the walk also composites the auxiliary maps with the same weights:
// the record's depth and the kA float4 of its attribute row (the first
// mp.n_attr values), written to mp.aux; no background term for the maps.
template <bool kMaxw, bool kCount, int kA = -1>
__device__ __forceinline__ void fwd_tile_wave(const Consts &k, const float4 *__restrict__ rec,
                                              const uint32_t *__restrict__ starts,
                                              const uint32_t *__restrict__ sorted, float *__restrict__ out,
                                              float *__restrict__ maxw, int64_t *__restrict__ status, int64_t tile,
                                              float4 *__restrict__ ckpt, WaveSlots &slots,
                                              const MapsArgs *mp = nullptr, MapSlots *ms = nullptr) {
    static_assert(kA < 0 || !kCount, "the maps take the lane-index field of the counting walk");
    const TileGeom tg = tile_geom(k, tile);
    const uint32_t start = starts[tile], end = starts[tile + 1];
    walk_priority(end - start);
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sx = tg.tx * kTile + 8 * (wave & 1), sy = tg.ty * kTile + 8 * (wave >> 1);
    const int x = sx + (lane & 7), y = sy + (lane >> 3);
    bool alive = x < k.width && y < k.height;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    uint32_t stop_at = end;  // list position of this pixel's terminating record
    uint32_t composited = 0;
    // the maps: depth, then the attributes
    constexpr int kAq = kA > 0 ? kA : 1;
    float Dm = 0.f, Mv[4 * kAq];
#pragma unroll
    for (int c = 0; c < 4 * kAq; ++c) Mv[c] = 0.f;
    float4 na[kAq], ca[kAq];
    ivrgs_job job_m{};
    if constexpr (kA >= 0) job_m = mp->jobs[tg.job];

    // Two-stage software pipeline over steps of 64 records: while one step
    // is composited, the records of the next are gathered with ids loaded a
    // step earlier, and the ids of the step after are loaded, so neither the
    // id load nor the gather that depends on it is waited for in the walk.
    float4 n0, n1, n2;
    uint32_t nid = 0, pid = 0;  // ids of the next step's records / of the step after
    auto load_ids = [&](uint32_t base) {
        if (base + lane < end) pid = sorted[base + lane];
    };
    auto load_recs = [&](uint32_t base) {
        if (base + lane < end) {
            nid = pid;
            n0 = rec[kRecVec * (size_t)nid];
            n1 = rec[kRecVec * (size_t)nid + 1];
            n2 = rec[kRecVec * (size_t)nid + 2];
            if constexpr (kA > 0) {
                const int64_t gid = job_gaussian(job_m, mp->gauss_index, (int)(nid - job_m.rec_begin));
#pragma unroll
                for (int q = 0; q < kA; ++q) na[q] = mp->attr[(size_t)gid * kA + q];
            }
        }
    };
    if (start < end) {
        load_ids(start);
        load_recs(start);
        if (start + 64 < end) load_ids(start + 64);
    }
    int nseg = 1, next_cut = 1;
    uint32_t seg_len = end - start;
    if (ckpt) split_of(end - start, nseg, seg_len);
    auto store_cut = [&](int cut, bool live_px) {
        ckpt[((size_t)tile * (kSplitMax - 1) + (cut - 1)) * kCkptPix + wave * 64 + lane] =
            make_float4(live_px ? T : -1.f, C0, C1, C2);
    };
    for (uint32_t base = start; base < end; base += 64) {
        if (next_cut < nseg && base - start == (uint32_t)next_cut * seg_len) store_cut(next_cut++, alive);
        const uint64_t live = __ballot(alive);
        if (live == 0ull) break;
        const PixBox bx = alive_box(live, sx, sy);
        const float4 r0 = n0, r1 = n1, r2 = n2;
        const uint32_t rid = nid;
        if constexpr (kA > 0) {
#pragma unroll
            for (int q = 0; q < kA; ++q) ca[q] = na[q];
        }
        bool touch = false;
        if (base + lane < end) touch = box_hit(make_hit_test(r0, r1, r2), bx.x0, bx.y0, bx.w, bx.h);
        if (base + 64 < end) load_recs(base + 64);
        if (base + 128 < end) load_ids(base + 128);
        const uint64_t m = __ballot(touch);
        if (m == 0ull) continue;
        const int cnt = compact_records(slots, m, touch, r0, r1, r2, rid, lane);
        if constexpr (kA >= 0) {
            // the record's depth in place of its lane, and its attribute row
            if (touch) {
                const int slot =
                    __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                slots.f[slot][2].w = r2.y;
#pragma unroll
                for (int q = 0; q < kA; ++q) ms->a[slot][q] = ca[q];
            }
            wave_lds_sync();
        }
        // Records are visited in groups of kGroupFwd.  Phase 1 computes, with
        // no branch, everything that does not depend on the compositing
        // order (fields read from LDS at one address for the whole wave,
        // exponent, cutoff test, power, alpha); the records are independent,
        // so their instructions interleave.  Phase 2 is the front-to-back
        // chain in list order, a few instructions per record.  The
        // arithmetic of each record is the same as on every other path.
        constexpr int kGroupFwd = 4;
        for (int sl = 0; sl < cnt; sl += kGroupFwd) {
            float al[kGroupFwd], cr[kGroupFwd], cg[kGroupFwd], cb[kGroupFwd];
            bool pass[kGroupFwd];
            int src[kGroupFwd];
#pragma unroll
            for (int g = 0; g < kGroupFwd; ++g) {
                const bool valid = sl + g < cnt;  // wave-uniform
                src[g] = valid ? sl + g : sl;
                const float4 a = slots.f[src[g]][0], b = slots.f[src[g]][1], c = slots.f[src[g]][2];
                const float p2 = splat_exponent(a.z, a.w, b.x, px - a.x, py - a.y);
                // no separate cutoff test: below the cutoff (1e-3 under
                // log2(alpha_min / o')) alpha < alpha_min is certain, so the
                // alpha test below decides the same
                pass[g] = valid;
                al[g] = fminf(k.alpha_max, b.z * fast_exp2(p2));
                cr[g] = b.w;
                cg[g] = c.x;
                cb[g] = c.y;
            }
#pragma unroll
            for (int g = 0; g < kGroupFwd; ++g) {
                const float Tn = T * (1.f - al[g]);
                // alive as it stands after the records before this one
                const bool use = alive & pass[g] & (al[g] >= k.alpha_min);
                const bool stop = use & (Tn < k.T_min);
                const bool comp = use & !stop;
                const float w = comp ? al[g] * T : 0.f;
                C0 = fmaf(w, cr[g], C0);
                C1 = fmaf(w, cg[g], C1);
                C2 = fmaf(w, cb[g], C2);
                if constexpr (kA >= 0) {
                    Dm = fmaf(w, slots.f[src[g]][2].w, Dm);
#pragma unroll
                    for (int q = 0; q < kA; ++q) {
                        const float4 a4 = ms->a[src[g]][q];
                        Mv[4 * q] = fmaf(w, a4.x, Mv[4 * q]);
                        Mv[4 * q + 1] = fmaf(w, a4.y, Mv[4 * q + 1]);
                        Mv[4 * q + 2] = fmaf(w, a4.z, Mv[4 * q + 2]);
                        Mv[4 * q + 3] = fmaf(w, a4.w, Mv[4 * q + 3]);
                    }
                }
                T = comp ? Tn : T;
                if (kCount) {
                    composited += comp ? 1u : 0u;
                    if (stop) stop_at = base + (uint32_t)__float_as_int(slots.f[src[g]][2].w);
                }
                alive = alive & !stop;
                if (kMaxw) {
                    if (__ballot(w > 0.f)) {
                        const float wm = wave_max_to_lane63(w);
                        const uint32_t id = __float_as_uint(slots.f[src[g]][2].z);
                        if (lane == 63) atomicMax(reinterpret_cast<int *>(&maxw[id]), __float_as_int(wm));
                    }
                }
            }
            if (__ballot(alive) == 0ull) break;
        }
    }
    while (next_cut < nseg) store_cut(next_cut++, false);  // the walk ended before these cuts
    if (x < k.width && y < k.height) {
        const size_t plane = (size_t)k.width * k.height;
        float *img = out + (size_t)tg.job * 4 * plane;
        const size_t o = (size_t)y * k.width + x;
        img[o] = C0 + T * k.bg0;
        img[plane + o] = C1 + T * k.bg1;
        img[2 * plane + o] = C2 + T * k.bg2;
        img[3 * plane + o] = 1.f - T;
        if constexpr (kA >= 0) {
            const int nc = 1 + mp->n_attr;
            float *am = mp->aux + (size_t)tg.job * nc * plane + o;
            am[0] = Dm;
#pragma unroll
            for (int c = 0; c < 4 * kAq; ++c)
                if (kA > 0 && c < mp->n_attr) am[(size_t)(1 + c) * plane] = Mv[c];
        }
        if (kCount) {
            // every list entry up to and including the terminating one is an
            // evaluation of the plain walk, skipped or not
            const uint32_t ev = stop_at < end ? stop_at - start + 1u : end - start;
            const uint64_t e = ev, c = composited;
            atomicAdd(reinterpret_cast<unsigned long long *>(&status[2]), (unsigned long long)e);
            atomicAdd(reinterpret_cast<unsigned long long *>(&status[3]), (unsigned long long)c);
        }
    }
}

template <int PX, bool kMaxw, bool kCount>
__global__ __launch_bounds__(kTilePix / PX) void k_render_fwd(Consts k, const float4 *__restrict__ rec,
                                                             const uint32_t *__restrict__ starts,
                                                             const uint32_t *__restrict__ sorted, int64_t n_tiles,
                                                             float *__restrict__ out, float *__restrict__ maxw,
                                                             int64_t *__restrict__ status, float4 *__restrict__ ckpt) {
    if (starts[n_tiles] == 0xFFFFFFFFu) return;
    if constexpr (PX == 1) {
        __shared__ WaveSlots slots[kTilePix / 64];
        fwd_tile_wave<kMaxw, kCount>(k, rec, starts, sorted, out, maxw, status, blockIdx.x, ckpt,
                                     slots[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)]);
    }
    else fwd_tile<PX, kMaxw, kCount>(k, rec, starts, sorted, out, maxw, status, blockIdx.x);
}

// The image and the auxiliary maps in one walk (one pixel per lane).
template <int kA>
__global__ __launch_bounds__(kTilePix) void k_render_fwd_maps(Consts k, const float4 *__restrict__ rec,
                                                              const uint32_t *__restrict__ starts,
                                                              const uint32_t *__restrict__ sorted, int64_t n_tiles,
                                                              float *__restrict__ out, float4 *__restrict__ ckpt,
                                                              MapsArgs mp) {
    if (starts[n_tiles] == 0xFFFFFFFFu) return;
    __shared__ WaveSlots slots[kTilePix / 64];
    __shared__ MapSlots mslots[kA > 0 ? kTilePix / 64 : 1];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    fwd_tile_wave<false, false, kA>(k, rec, starts, sorted, out, nullptr, nullptr, blockIdx.x, ckpt, slots[wave], &mp,
                                    &mslots[kA > 0 ? wave : 0]);
}

// Persistent variant: a fixed grid pops tiles from queue[2 ..] (heaviest
// first) through the counter queue[0] until queue[1] items are taken.
__device__ __forceinline__ bool next_item(uint32_t *queue, uint32_t n_items, uint32_t &item) {
    __shared__ uint32_t s_item;
    if (threadIdx.x == 0) s_item = atomicAdd(&queue[0], 1u);
    __syncthreads();
    item = s_item;
    __syncthreads();
    return item < n_items;
}

template <int PX, bool kMaxw, bool kCount>
__global__ __launch_bounds__(kTilePix / PX) void k_render_fwd_persistent(
    Consts k, const float4 *__restrict__ rec, const uint32_t *__restrict__ starts,
    const uint32_t *__restrict__ sorted, int64_t n_tiles, float *__restrict__ out, float *__restrict__ maxw,
    int64_t *__restrict__ status, uint32_t *__restrict__ queue) {
    if (starts[n_tiles] == 0xFFFFFFFFu) return;
    const uint32_t n_items = queue[1];
    uint32_t item;
    while (next_item(queue, n_items, item)) {
        if constexpr (PX == 1) {
            __shared__ WaveSlots slots[kTilePix / 64];
            fwd_tile_wave<kMaxw, kCount>(k, rec, starts, sorted, out, maxw, status, queue[2 + item], nullptr,
                                         slots[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)]);
        } else {
            fwd_tile<PX, kMaxw, kCount>(k, rec, starts, sorted, out, maxw, status, queue[2 + item]);
        }
    }
}

// ----------------------------------------------------------------------------
// Where a backward walk puts each record's per-wave sums (one value kind per
// lane, my_v).  kSinkFloat: float atomics into grec.  The deterministic mode
// runs the walk twice: kSinkProbe keeps the largest |sum| of each value kind
// over the tile (a lane-local running maximum, then one atomicMax of its FP32
// bits per lane into probe[tile][9]); kSinkFixed adds each sum to gfix as a
// 64-bit integer, sum * scale[v] rounded, where the power of two scale[v] puts
// the largest |sum| below 2^40.  The integer sums do not depend on the order
// in which waves add them.
enum { kSinkFloat = 0, kSinkProbe = 1, kSinkFixed = 2 };
struct GradSink {
    float *grec;
    uint32_t *probe;
    unsigned long long *gfix;
    const float *scale;
};

template <int kMode>
struct SinkLane {
    float scale = 0.f, vmax = 0.f;
    __device__ __forceinline__ void init(const GradSink &s, int my_v) {
        if (kMode == kSinkFixed) scale = s.scale[my_v];
    }
    // tot: the wave's sum of value my_v for record id
    __device__ __forceinline__ void add(const GradSink &s, uint32_t id, int my_v, float tot) {
        if constexpr (kMode == kSinkFloat) {
            atomicAdd(&s.grec[(size_t)id * kGradStride + my_v], tot);
        } else if constexpr (kMode == kSinkProbe) {
            vmax = fmaxf(vmax, fabsf(tot));
        } else {
            const long long q = (long long)rintf(tot * scale);
            atomicAdd(&s.gfix[(size_t)id * kGradStride + my_v], (unsigned long long)q);
        }
    }
    __device__ __forceinline__ void flush(const GradSink &s, int64_t tile, int my_v, bool my_slot) {
        if (kMode == kSinkProbe && my_slot && vmax > 0.f)
            atomicMax(&s.probe[tile * kGradRec + my_v], __float_as_uint(vmax));
    }
};

// ----------------------------------------------------------------------------
// Backward of one tile, each wave on its own region (the walk of
// fwd_tile_wave: 64 records gathered per step into registers, a ballot of the
// records that can reach the region, fields broadcast from the record's
// lane).  With one pixel per lane the region is the 8x8 quadrant of the
// forward; with PX > 1, wave w owns the 16 x 4PX strip of rows 4PX w ..
// 4PX (w+1) - 1 and lane l its pixels (l % 16, l / 16 + 4j), j < PX, so every
// broadcast, test and reduce-scatter serves PX pixels.  No LDS
// and no workgroup barrier, so a wave never waits for the other regions of
// its tile.  Records that composite somewhere in the region fill the three
// slots of one reduce-scatter; their ids are kept in scalar registers for
// the atomics.
//
// ckpt != nullptr (one pixel per lane): the workgroup walks segment `seg` of
// the tile's list (split_of), starting from the forward's checkpoint at its
// cut: T exactly as the forward had it, and the colour prefix as g . C.
template <int PX, int kMode>
__device__ __forceinline__ void bwd_tile_wave(const Consts &k, const float4 *__restrict__ rec,
                                              const uint32_t *__restrict__ starts,
                                              const uint32_t *__restrict__ sorted, const float *__restrict__ rgba,
                                              const float *__restrict__ dl, const GradSink &sink, int64_t tile,
                                              int seg, const float4 *__restrict__ ckpt) {
    const TileGeom tg = tile_geom(k, tile);
    uint32_t start = starts[tile], end = starts[tile + 1];
    if (PX == 1 && ckpt) {
        int nseg;
        uint32_t seg_len;
        split_of(end - start, nseg, seg_len);
        if (seg >= nseg) return;  // the whole workgroup
        start += (uint32_t)seg * seg_len;
        end = min(end, start + seg_len);
    } else if (seg > 0) {
        return;
    }
    walk_priority(end - start);
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the wave's region: with one pixel per lane the 8x8 quadrant w of the
    // tile (the most compact shape, so the fewest records reach it), else the
    // 16 x 4PX strip w
    constexpr int RW = PX == 1 ? 8 : kTile, RH = PX == 1 ? 8 : 4 * PX;
    const int sx = tg.tx * kTile + (PX == 1 ? 8 * (wave & 1) : 0);
    const int sy = tg.ty * kTile + (PX == 1 ? 8 * (wave >> 1) : RH * wave);
    const size_t plane = (size_t)k.width * k.height;
    // per pixel: upstream colour gradient g, g . out, gA T_final and the
    // running g . P_i of the composited prefix (as in bwd_tile)
    float px[PX], py[PX], T[PX], gP[PX], go[PX], gATf[PX], g0[PX], g1[PX], g2[PX];
    bool alive[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        const int x = sx + lane % RW, y = sy + lane / RW + (64 / RW) * j;
        px[j] = (float)x + 0.5f;
        py[j] = (float)y + 0.5f;
        T[j] = 1.f;
        gP[j] = go[j] = gATf[j] = g0[j] = g1[j] = g2[j] = 0.f;
        alive[j] = x < k.width && y < k.height;
        if (alive[j]) {
            const float *img = rgba + (size_t)tg.job * 4 * plane;
            const float *gimg = dl + (size_t)tg.job * 4 * plane;
            const size_t o = (size_t)y * k.width + x;
            const float Tf = 1.f - img[3 * plane + o];
            g0[j] = gimg[o];
            g1[j] = gimg[plane + o];
            g2[j] = gimg[2 * plane + o];
            const float gA = gimg[3 * plane + o];
            go[j] = fmaf(g2[j], img[2 * plane + o], fmaf(g1[j], img[plane + o], g0[j] * img[o]));
            gATf[j] = gA * Tf;
            alive[j] = (g0[j] != 0.f) | (g1[j] != 0.f) | (g2[j] != 0.f) | (gA != 0.f);
        }
        if (PX == 1 && ckpt && seg > 0) {
            const float4 c = ckpt[((size_t)tile * (kSplitMax - 1) + (seg - 1)) * kCkptPix + wave * 64 + lane];
            if (c.x < 0.f) {
                alive[j] = false;  // terminated before the cut
            } else {
                T[j] = c.x;
                gP[j] = fmaf(g2[j], c.w, fmaf(g1[j], c.z, g0[j] * c.y));
            }
        }
    }
    auto any_alive = [&]() {
        bool a = false;
#pragma unroll
        for (int j = 0; j < PX; ++j) a |= alive[j];
        return __ballot(a) != 0ull;
    };
    constexpr int kGroup = 3;
    const int my_m = lane >> 1;
    const bool my_slot = ((lane & 1) == 0) && my_m < kGroup * kGradRec;
    const int my_g = my_m / kGradRec, my_v = my_m % kGradRec;
    SinkLane<kMode> out;
    out.init(sink, my_v);

    // records of the current step (r*, rid) and of the next one (n*, nid),
    // ids of the step after (pid): the two-stage pipeline of fwd_tile_wave
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0, n0 = r0, n1 = r0, n2 = r0;
    uint32_t rid = 0, nid = 0, pid = 0;
    uint32_t nbase = start;  // list position of the records held in n*
    auto load_ids = [&](uint32_t base) {
        if (base + lane < end) pid = sorted[base + lane];
    };
    auto load_recs = [&](uint32_t base) {
        if (base + lane < end) {
            nid = pid;
            n0 = rec[kRecVec * (size_t)nid];
            n1 = rec[kRecVec * (size_t)nid + 1];
            n2 = rec[kRecVec * (size_t)nid + 2];
        }
    };
    if (start < end) {
        load_ids(start);
        load_recs(start);
        if (start + 64 < end) load_ids(start + 64);
    }
    uint64_t m = 0;
    // the next record that can reach the region (its lane in r*), moving on to
    // the next 64 records when the current ones are used up; false at the end
    auto next = [&](int &src) -> bool {
        while (m == 0ull) {
            if (nbase >= end) return false;
            r0 = n0;
            r1 = n1;
            r2 = n2;
            rid = nid;
            PixBox bx = {sx, sy, RW, RH};
            if constexpr (PX == 1) {
                const uint64_t live = __ballot(alive[0]);
                if (live != 0ull) bx = alive_box(live, sx, sy);
            }
            const bool touch =
                nbase + lane < end && box_hit(make_hit_test(r0, r1, r2), bx.x0, bx.y0, bx.w, bx.h);
            nbase += 64;
            if (nbase < end) load_recs(nbase);
            if (nbase + 64 < end) load_ids(nbase + 64);
            m = __ballot(touch);
        }
        src = (int)__builtin_ctzll(m);
        m &= m - 1;
        return true;
    };
    auto bcast = [&](float v, int src) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src)); };

    bool more = any_alive();
    while (more) {
        float acc[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) acc[q] = 0.f;
        uint32_t ids[kGroup];
        bool filled[kGroup];
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
            filled[g] = false;
            ids[g] = 0;
            while (more) {
                int src;
                if (!next(src)) {
                    more = false;
                    break;
                }
                const float mx = bcast(r0.x, src), my = bcast(r0.y, src);
                const float qa = bcast(r0.z, src), qb = bcast(r0.w, src), qc = bcast(r1.x, src);
                const float cut = bcast(r2.z, src);
                float dx[PX], dy[PX], p2[PX];
                bool pass[PX], anyp = false;
#pragma unroll
                for (int j = 0; j < PX; ++j) {
                    dx[j] = px[j] - mx;
                    dy[j] = py[j] - my;
                    p2[j] = splat_exponent(qa, qb, qc, dx[j], dy[j]);
                    // below the cutoff alpha < alpha_min is certain
                    pass[j] = alive[j] && p2[j] >= cut;
                    anyp |= pass[j];
                }
                if (__ballot(anyp) == 0ull) continue;  // wave-uniform
                const float o = bcast(r1.y, src), cr = bcast(r1.z, src), cg = bcast(r1.w, src);
                const float cb = bcast(r2.x, src);
                bool anyc = false;
                float *ag = acc + g * kGradRec;
#pragma unroll
                for (int j = 0; j < PX; ++j) {
                    // branch-free, with the same arithmetic as the forward: a
                    // pixel that does not composite adds zero-weight terms
                    // (all operands finite)
                    const float G = fast_exp2(p2[j]);
                    const float raw = o * G;
                    const float al = fminf(k.alpha_max, raw);
                    const float Tn = T[j] * (1.f - al);
                    const bool use = pass[j] && al >= k.alpha_min;
                    const bool stop = use && Tn < k.T_min;
                    const bool comp = use && !stop;
                    const float w = comp ? al * T[j] : 0.f;
                    const float gc = fmaf(g2[j], cb, fmaf(g1[j], cg, g0[j] * cr));
                    gP[j] = fmaf(w, gc, gP[j]);
                    // g . (colour behind this Gaussian, background included)
                    const float gb = go[j] - gP[j];
                    const float inv = __builtin_amdgcn_rcpf(1.f - al);
                    const float dLda = comp ? T[j] * gc - (gb - gATf[j]) * inv : 0.f;
                    // no gradient through alpha where the cap is active
                    const float dLdo = raw <= k.alpha_max ? dLda : 0.f;
                    ag[GCR] = fmaf(w, g0[j], ag[GCR]);
                    ag[GCG] = fmaf(w, g1[j], ag[GCG]);
                    ag[GCB] = fmaf(w, g2[j], ag[GCB]);
                    // moments of dL/do' G about the mean (see GX .. GQC)
                    const float dp = dLdo * G;
                    ag[GO] += dp;
                    ag[GQA] = fmaf(dp, dx[j] * dx[j], ag[GQA]);
                    ag[GQB] = fmaf(dp, dx[j] * dy[j], ag[GQB]);
                    ag[GQC] = fmaf(dp, dy[j] * dy[j], ag[GQC]);
                    ag[GX] = fmaf(dp, dx[j], ag[GX]);
                    ag[GY] = fmaf(dp, dy[j], ag[GY]);
                    T[j] = comp ? Tn : T[j];
                    alive[j] = alive[j] && !stop;
                    anyc |= comp;
                }
                const bool hit = __ballot(anyc) != 0ull;
                if (!any_alive()) more = false;  // every pixel of the wave is done
                if (hit) {
                    filled[g] = true;
                    ids[g] = __builtin_amdgcn_readlane(rid, src);
                    break;
                }
            }
        }
        if (filled[0]) {
            const float tot = reduce_scatter32(acc);
            const bool ok = my_g == 0 ? filled[0] : (my_g == 1 ? filled[1] : filled[2]);
            const uint32_t id = my_g == 0 ? ids[0] : (my_g == 1 ? ids[1] : ids[2]);
            if (my_slot && ok && tot != 0.f) out.add(sink, id, my_v, tot);
        }
    }
    out.flush(sink, tile, my_v, my_slot);
}

// Backward of one tile with one pixel per lane, each wave on its own 8x8
// quadrant (the walk of fwd_tile_wave: 64 records gathered per step into
// registers and tested against the box of the quadrant's live pixels).  The
// records of a step that can reach the box are compacted, in list order,
// into the wave's LDS slots; one pass over them keeps those whose exponent
// passes the cutoff at a live pixel (a bit mask); the rest are visited in
// groups of three.  Each record's fields are read from LDS with one address
// for the whole wave (a broadcast).  A group first computes, without
// branches, everything that does not depend on the compositing order (offset,
// exponent, power, alpha, 1 / (1 - alpha), g . colour) for its three records,
// then runs the front-to-back chain and writes each record's nine per-pixel
// gradient terms into its slots of one reduce-scatter; records that
// composite somewhere get one atomic per value.
//
// ckpt != nullptr: the workgroup walks segment `seg` of the tile's list
// (split_of), starting from the forward's checkpoint at its cut: T exactly as
// the forward had it, and the colour prefix as g . C.
template <int kMode>
__device__ __forceinline__ void bwd_tile_quad(const Consts &k, const float4 *__restrict__ rec,
                                              const uint32_t *__restrict__ starts,
                                              const uint32_t *__restrict__ sorted, const float *__restrict__ rgba,
                                              const float *__restrict__ dl, const GradSink &sink, int64_t tile,
                                              int seg, const float4 *__restrict__ ckpt, WaveSlots &slots) {
    const TileGeom tg = tile_geom(k, tile);
    uint32_t start = starts[tile], end = starts[tile + 1];
    if (ckpt) {
        int nseg;
        uint32_t seg_len;
        split_of(end - start, nseg, seg_len);
        if (seg >= nseg) return;  // the whole workgroup
        start += (uint32_t)seg * seg_len;
        end = min(end, start + seg_len);
    } else if (seg > 0) {
        return;
    }
    walk_priority(end - start);
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sx = tg.tx * kTile + 8 * (wave & 1), sy = tg.ty * kTile + 8 * (wave >> 1);
    const int x = sx + (lane & 7), y = sy + (lane >> 3);
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const size_t plane = (size_t)k.width * k.height;
    // per pixel: upstream colour gradient g, g . out, gA T_final and the
    // running g . P_i of the composited prefix
    float T = 1.f, gP = 0.f, go = 0.f, gATf = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
    bool alive = x < k.width && y < k.height;
    if (alive) {
        const float *img = rgba + (size_t)tg.job * 4 * plane;
        const float *gimg = dl + (size_t)tg.job * 4 * plane;
        const size_t o = (size_t)y * k.width + x;
        const float Tf = 1.f - img[3 * plane + o];
        g0 = gimg[o];
        g1 = gimg[plane + o];
        g2 = gimg[2 * plane + o];
        const float gA = gimg[3 * plane + o];
        go = fmaf(g2, img[2 * plane + o], fmaf(g1, img[plane + o], g0 * img[o]));
        gATf = gA * Tf;
        alive = (g0 != 0.f) | (g1 != 0.f) | (g2 != 0.f) | (gA != 0.f);
    }
    if (ckpt && seg > 0) {
        const float4 c = ckpt[((size_t)tile * (kSplitMax - 1) + (seg - 1)) * kCkptPix + wave * 64 + lane];
        if (c.x < 0.f) {
            alive = false;  // terminated before the cut
        } else {
            T = c.x;
            gP = fmaf(g2, c.w, fmaf(g1, c.z, g0 * c.y));
        }
    }
    // g . (colour behind a Gaussian) - gA T_final is goA - gP
    const float goA = go - gATf;
    constexpr int kGroup = 3;
    const int my_m = lane >> 1;
    const bool my_slot = ((lane & 1) == 0) && my_m < kGroup * kGradRec;
    const int my_g = my_m < kGroup * kGradRec ? my_m / kGradRec : 0, my_v = my_m % kGradRec;
    SinkLane<kMode> out;
    out.init(sink, my_v);
    float acc[32];
    // every slot starts as the zero record (opacity 0: no power anywhere)
    {
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        slots.f[lane][0] = slots.f[lane][1] = slots.f[lane][2] = z;
        if (lane < 2) slots.f[64 + lane][0] = slots.f[64 + lane][1] = slots.f[64 + lane][2] = z;
    }

    // the two-stage gather pipeline of fwd_tile_wave
    float4 n0 = make_float4(0.f, 0.f, 0.f, 0.f), n1 = n0, n2 = n0;
    uint32_t nid = 0, pid = 0;
    auto load_ids = [&](uint32_t base) {
        if (base + lane < end) pid = sorted[base + lane];
    };
    auto load_recs = [&](uint32_t base) {
        if (base + lane < end) {
            nid = pid;
            n0 = rec[kRecVec * (size_t)nid];
            n1 = rec[kRecVec * (size_t)nid + 1];
            n2 = rec[kRecVec * (size_t)nid + 2];
        }
    };
    if (start < end) {
        load_ids(start);
        load_recs(start);
        if (start + 64 < end) load_ids(start + 64);
    }
    for (uint32_t base = start; base < end; base += 64) {
        const uint64_t live = __ballot(alive);
        if (live == 0ull) break;
        const PixBox bx = alive_box(live, sx, sy);
        const float4 r0 = n0, r1 = n1, r2 = n2;
        const uint32_t rid = nid;
        const bool touch = base + lane < end && box_hit(make_hit_test(r0, r1, r2), bx.x0, bx.y0, bx.w, bx.h);
        if (base + 64 < end) load_recs(base + 64);
        if (base + 128 < end) load_ids(base + 128);
        const uint64_t m = __ballot(touch);
        if (m == 0ull) continue;
        const int cnt = compact_records(slots, m, touch, r0, r1, r2, rid, lane);
        // every compacted record is visited: the cutoff test is part of its
        // order-free work (a separate pass to drop the records that pass at no
        // live pixel costs more than it saves)
        // the compacted records are slots 0 .. cnt - 1, in list order: a group
        // is kGroup consecutive slots (one address for the group, the records
        // at fixed offsets from it)
        for (int sl = 0; sl < cnt; sl += kGroup) {
            int src[kGroup];
            bool valid[kGroup];
#pragma unroll
            for (int g = 0; g < kGroup; ++g) {
                valid[g] = sl + g < cnt;  // wave-uniform
                // a slot past the step's records holds a finite record (an
                // earlier step's, or the zero record): its terms are masked
                src[g] = sl + g;
            }
            // order-free part of the three records: everything but T
            float dx[kGroup], dy[kGroup], G[kGroup], raw[kGroup], al[kGroup], om[kGroup], inv[kGroup], gc[kGroup];
            float idf[kGroup];
            bool use[kGroup], free_a[kGroup];
#pragma unroll
            for (int g = 0; g < kGroup; ++g) {
                const float4 a = slots.f[src[g]][0], b = slots.f[src[g]][1], c = slots.f[src[g]][2];
                dx[g] = px - a.x;
                dy[g] = py - a.y;
                const float p2 = splat_exponent(a.z, a.w, b.x, dx[g], dy[g]);
                G[g] = fast_exp2(p2);
                raw[g] = b.z * G[g];
                al[g] = fminf(k.alpha_max, raw[g]);
                om[g] = 1.f - al[g];
                inv[g] = __builtin_amdgcn_rcpf(om[g]);
                gc[g] = fmaf(g2, c.y, fmaf(g1, c.x, g0 * b.w));
                // the alpha test alone (below the cutoff alpha < alpha_min
                // is certain: the two decide the same)
                use[g] = valid[g] & (al[g] >= k.alpha_min);
                // no gradient through alpha where the cap is active
                free_a[g] = raw[g] <= k.alpha_max;
                idf[g] = c.z;
            }
            // the front-to-back chain, the arithmetic of the forward
            bool any = false;
#pragma unroll
            for (int g = 0; g < kGroup; ++g) {
                // bitwise logic: no short-circuit branches in the chain
                const float Tn = T * om[g];
                const bool stop = alive & use[g] & (Tn < k.T_min);
                const bool comp = alive & use[g] & !stop;
                const float w = comp ? al[g] * T : 0.f;
                gP = fmaf(w, gc[g], gP);
                const float dLda = fmaf(gP - goA, inv[g], T * gc[g]);
                const float dLdo = (comp & free_a[g]) ? dLda : 0.f;
                // D without the factor o' (the projection backward applies it)
                const float dp = dLdo * G[g];
                float *ag = acc + g * kGradRec;
                ag[GCR] = w * g0;
                ag[GCG] = w * g1;
                ag[GCB] = w * g2;
                ag[GO] = dp;
                // moments of dL/dG G about the mean (see GX .. GQC)
                const float dpx = dp * dx[g], dpy = dp * dy[g];
                ag[GX] = dpx;
                ag[GY] = dpy;
                ag[GQA] = dpx * dx[g];
                ag[GQB] = dpx * dy[g];
                ag[GQC] = dpy * dy[g];
                T = comp ? Tn : T;
                alive = alive & !stop;
                any = any | comp;
            }
            // the five spare slots of the reduce-scatter carry values that
            // are dead by now: their sums land on lanes that add nothing
            acc[27] = dx[0];
            acc[28] = dy[0];
            acc[29] = dx[1];
            acc[30] = dy[1];
            acc[31] = dx[2];
            if (__ballot(any) != 0ull) {
                const float tot = reduce_scatter32(acc);
                // a record that composites nowhere has all sums exactly 0
                if (my_slot && tot != 0.f) {
                    const float id = my_g == 0 ? idf[0] : (my_g == 1 ? idf[1] : idf[2]);
                    out.add(sink, kMode == kSinkProbe ? 0u : __float_as_uint(id), my_v, tot);
                }
            }
            if (__ballot(alive) == 0ull) break;  // every pixel of the wave is done
        }
    }
    out.flush(sink, tile, my_v, my_slot);
}

template <int PX, int kMode>
__global__ __launch_bounds__(kTilePix / PX) void k_render_bwd(Consts k, const float4 *__restrict__ rec,
                                                             const uint32_t *__restrict__ starts,
                                                             const uint32_t *__restrict__ sorted, int64_t n_tiles,
                                                             const float *__restrict__ rgba,
                                                             const float *__restrict__ dl, GradSink sink,
                                                             const float4 *__restrict__ ckpt) {
    if (starts[n_tiles] == 0xFFFFFFFFu) return;
    if constexpr (PX == 1) {
        __shared__ WaveSlots slots[kTilePix / 64];
        bwd_tile_quad<kMode>(k, rec, starts, sorted, rgba, dl, sink, blockIdx.x, blockIdx.y, ckpt,
                             slots[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)]);
    } else {
        bwd_tile_wave<PX, kMode>(k, rec, starts, sorted, rgba, dl, sink, blockIdx.x, blockIdx.y, ckpt);
    }
}

template <int PX, int kMode>
__global__ __launch_bounds__(kTilePix / PX) void k_render_bwd_persistent(
    Consts k, const float4 *__restrict__ rec, const uint32_t *__restrict__ starts,
    const uint32_t *__restrict__ sorted, int64_t n_tiles, const float *__restrict__ rgba,
    const float *__restrict__ dl, GradSink sink, uint32_t *__restrict__ queue) {
    if (starts[n_tiles] == 0xFFFFFFFFu) return;
    const uint32_t n_items = queue[1];
    uint32_t item;
    while (next_item(queue, n_items, item)) {
        if constexpr (PX == 1) {
            __shared__ WaveSlots slots[kTilePix / 64];
            bwd_tile_quad<kMode>(k, rec, starts, sorted, rgba, dl, sink, queue[2 + item], 0, nullptr,
                                 slots[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)]);
        } else {
            bwd_tile_wave<PX, kMode>(k, rec, starts, sorted, rgba, dl, sink, queue[2 + item], 0, nullptr);
        }
    }
}

// Deterministic mode, between the two walks: scale[v] = 2^(40 - e) with
// 2^(e-1) <= max over tiles of probe[tile][v] < 2^e (1 if nothing was
// added), and its inverse.  One workgroup of kGradRec * 64 threads.
__global__ __launch_bounds__(kGradRec * 64) void k_det_scale(const uint32_t *__restrict__ probe, int64_t n_tiles,
                                                             float *__restrict__ scale) {
    const int v = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t m = 0;
    for (int64_t t = lane; t < n_tiles; t += 64) m = max(m, probe[t * kGradRec + v]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, 64));
    if (lane == 0) {
        int e = 0;
        if (m != 0u) {
            frexpf(__uint_as_float(m), &e);
            e = max(e, -80);
        }
        scale[v] = m ? ldexpf(1.f, 40 - e) : 1.f;
        scale[kGradRec + v] = m ? ldexpf(1.f, e - 40) : 1.f;
    }
}

// Deterministic mode, after the second walk: the FP32 record gradients from
// their integer sums (the slots past the image's components are cleared).
__global__ void k_det_finish(const unsigned long long *__restrict__ gfix, const float *__restrict__ scale,
                             int64_t n, float *__restrict__ grec) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int v = (int)(i % kGradStride);
        grec[i] = v < kGradRec ? (float)((double)(long long)gfix[i] * (double)scale[kGradRec + v]) : 0.f;
    }
}

// ----------------------------------------------------------------------------
template <int PX>
static void fwd_variant(bool maxw, bool count, dim3 grid, hipStream_t s, const Consts &k, const float4 *rec,
                        const uint32_t *starts, const uint32_t *sorted, int64_t n_tiles, float *out, float *mw,
                        int64_t *status, uint32_t *queue, float4 *ckpt) {
    constexpr int NT = kTilePix / PX;
    if (queue) {
#define IVRGS_FWD_P(M, C)                                                                                          \
    hipLaunchKernelGGL((k_render_fwd_persistent<PX, M, C>), grid, dim3(NT), 0, s, k, rec, starts, sorted, n_tiles, \
                       out, mw, status, queue)
        if (maxw && count) IVRGS_FWD_P(true, true);
        else if (maxw) IVRGS_FWD_P(true, false);
        else if (count) IVRGS_FWD_P(false, true);
        else IVRGS_FWD_P(false, false);
#undef IVRGS_FWD_P
        return;
    }
#define IVRGS_FWD(M, C) \
    hipLaunchKernelGGL((k_render_fwd<PX, M, C>), grid, dim3(NT), 0, s, k, rec, starts, sorted, n_tiles, out, mw, status, \
                       ckpt)
    if (maxw && count) IVRGS_FWD(true, true);
    else if (maxw) IVRGS_FWD(true, false);
    else if (count) IVRGS_FWD(false, true);
    else IVRGS_FWD(false, false);
#undef IVRGS_FWD
}

// Workgroups per CU that the persistent variants keep resident.
template <typename K>
static int resident_blocks(K kernel, int threads) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) nb = 1;
    return nb;
}

static int cu_count() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
    }
    return cus;
}

template <int PX>
static dim3 persistent_grid_fwd(bool maxw, bool count, int per_cu) {
    constexpr int NT = kTilePix / PX;
    static int occ[4] = {0, 0, 0, 0};  // per (maxw, count) variant, queried once
    const int v = (maxw ? 2 : 0) + (count ? 1 : 0);
    if (occ[v] == 0) {
        if (maxw && count) occ[v] = resident_blocks(k_render_fwd_persistent<PX, true, true>, NT);
        else if (maxw) occ[v] = resident_blocks(k_render_fwd_persistent<PX, true, false>, NT);
        else if (count) occ[v] = resident_blocks(k_render_fwd_persistent<PX, false, true>, NT);
        else occ[v] = resident_blocks(k_render_fwd_persistent<PX, false, false>, NT);
    }
    const int nb = per_cu > 0 ? per_cu : occ[v];
    return dim3((unsigned)(nb * cu_count()));
}

hipError_t launch_render_fwd(const Consts &k, int px, int64_t n_tiles, const float *rec, const uint32_t *starts,
                             const uint32_t *sorted, float *out, float *maxw, int64_t *status, bool count,
                             uint32_t *queue, int per_cu, float *ckpt, hipStream_t s) {
    float4 *ck = px == 1 && !queue ? reinterpret_cast<float4 *>(ckpt) : nullptr;
    if (n_tiles == 0) return hipSuccess;
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const bool mw = maxw != nullptr;
    if (queue) {
        hipError_t e = launch_fill_u32(queue, 1, 0u, s);  // reset the work counter
        if (e != hipSuccess) return e;
    }
    TimedScope ts(TK_FWD, s);
    switch (px) {
    case 1: fwd_variant<1>(mw, count, queue ? persistent_grid_fwd<1>(mw, count, per_cu) : dim3((unsigned)n_tiles), s, k, r4, starts, sorted, n_tiles, out, maxw, status, queue, ck); break;
    case 2: fwd_variant<2>(mw, count, queue ? persistent_grid_fwd<2>(mw, count, per_cu) : dim3((unsigned)n_tiles), s, k, r4, starts, sorted, n_tiles, out, maxw, status, queue, nullptr); break;
    default: fwd_variant<4>(mw, count, queue ? persistent_grid_fwd<4>(mw, count, per_cu) : dim3((unsigned)n_tiles), s, k, r4, starts, sorted, n_tiles, out, maxw, status, queue, nullptr); break;
    }
    return hipGetLastError();
}

hipError_t launch_render_fwd_maps(const Consts &k, int64_t n_tiles, const float *rec, const uint32_t *starts,
                                  const uint32_t *sorted, float *out, float *ckpt, const ivrgs_job *jobs,
                                  const int32_t *gauss_index, const float *attr, int n_attr, float *aux,
                                  hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    float4 *ck = reinterpret_cast<float4 *>(ckpt);
    const MapsArgs mp{jobs, gauss_index, reinterpret_cast<const float4 *>(attr), aux, n_attr};
    const dim3 grid((unsigned)n_tiles), block(kTilePix);
    TimedScope ts(TK_FWD, s);
    switch ((n_attr + 3) / 4) {
    case 0: hipLaunchKernelGGL(k_render_fwd_maps<0>, grid, block, 0, s, k, r4, starts, sorted, n_tiles, out, ck, mp); break;
    case 1: hipLaunchKernelGGL(k_render_fwd_maps<1>, grid, block, 0, s, k, r4, starts, sorted, n_tiles, out, ck, mp); break;
    case 2: hipLaunchKernelGGL(k_render_fwd_maps<2>, grid, block, 0, s, k, r4, starts, sorted, n_tiles, out, ck, mp); break;
    case 3: hipLaunchKernelGGL(k_render_fwd_maps<3>, grid, block, 0, s, k, r4, starts, sorted, n_tiles, out, ck, mp); break;
    case 4: hipLaunchKernelGGL(k_render_fwd_maps<4>, grid, block, 0, s, k, r4, starts, sorted, n_tiles, out, ck, mp); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int PX, int kMode>
static void bwd_variant(hipStream_t s, const Consts &k, const float4 *rec, const uint32_t *starts,
                        const uint32_t *sorted, int64_t n_tiles, const float *rgba, const float *dl,
                        const GradSink &sink, uint32_t *queue, int per_cu, const float4 *ckpt) {
    constexpr int NT = kTilePix / PX;
    if (queue) {
        static int occ = 0;  // queried once
        if (occ == 0) occ = resident_blocks(k_render_bwd_persistent<PX, kMode>, NT);
        const int nb = per_cu > 0 ? per_cu : occ;
        hipLaunchKernelGGL((k_render_bwd_persistent<PX, kMode>), dim3((unsigned)(nb * cu_count())), dim3(NT), 0, s,
                           k, rec, starts, sorted, n_tiles, rgba, dl, sink, queue);
    } else {
        // one workgroup per (tile, segment of its list)
        hipLaunchKernelGGL((k_render_bwd<PX, kMode>), dim3((unsigned)n_tiles, ckpt ? kSplitMax : 1), dim3(NT), 0, s,
                           k, rec, starts, sorted, n_tiles, rgba, dl, sink, ckpt);
    }
}

template <int kMode>
static hipError_t bwd_walk(const Consts &k, int px, int64_t n_tiles, const float4 *r4, const uint32_t *starts,
                           const uint32_t *sorted, const float *rgba, const float *dl, const GradSink &sink,
                           uint32_t *queue, int per_cu, const float4 *ck, hipStream_t s) {
    if (queue) {
        hipError_t e = launch_fill_u32(queue, 1, 0u, s);  // reset the work counter
        if (e != hipSuccess) return e;
    }
    TimedScope ts(TK_BWD, s);
    switch (px) {
    case 1: bwd_variant<1, kMode>(s, k, r4, starts, sorted, n_tiles, rgba, dl, sink, queue, per_cu, ck); break;
    case 2: bwd_variant<2, kMode>(s, k, r4, starts, sorted, n_tiles, rgba, dl, sink, queue, per_cu, nullptr); break;
    default: bwd_variant<4, kMode>(s, k, r4, starts, sorted, n_tiles, rgba, dl, sink, queue, per_cu, nullptr); break;
    }
    return hipGetLastError();
}

hipError_t launch_render_bwd(const Consts &k, int px, int64_t n_tiles, const float *rec, const uint32_t *starts,
                             const uint32_t *sorted, const float *rgba, const float *dl, float *grec,
                             uint32_t *queue, int per_cu, const float *ckpt, const DetWork *det,
                             int64_t n_records, hipStream_t s) {
    const float4 *ck = px == 1 && !queue ? reinterpret_cast<const float4 *>(ckpt) : nullptr;
    if (n_tiles == 0) return hipSuccess;
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    GradSink sink = {grec, nullptr, nullptr, nullptr};
    if (!det) return bwd_walk<kSinkFloat>(k, px, n_tiles, r4, starts, sorted, rgba, dl, sink, queue, per_cu, ck, s);
    // deterministic: the largest |sum| per value kind, its scale, then the
    // integer sums and their FP32 values
    sink.probe = det->probe;
    sink.gfix = det->gfix;
    sink.scale = det->scale;
    hipError_t e = launch_fill_u32(det->probe, n_tiles * kGradRec, 0u, s);
    if (e == hipSuccess)
        e = bwd_walk<kSinkProbe>(k, px, n_tiles, r4, starts, sorted, rgba, dl, sink, queue, per_cu, ck, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_det_scale, dim3(1), dim3(kGradRec * 64), 0, s, det->probe, n_tiles, det->scale);
    e = hipGetLastError();
    if (e == hipSuccess)
        e = launch_fill_u32(reinterpret_cast<uint32_t *>(det->gfix), 2 * kGradStride * n_records, 0u, s);
    if (e == hipSuccess)
        e = bwd_walk<kSinkFixed>(k, px, n_tiles, r4, starts, sorted, rgba, dl, sink, queue, per_cu, ck, s);
    if (e != hipSuccess) return e;
    const int64_t nv = kGradStride * n_records;
    const unsigned blocks = (unsigned)std::min<int64_t>((nv + 255) / 256, 65535);
    if (nv > 0) hipLaunchKernelGGL(k_det_finish, dim3(blocks), dim3(256), 0, s, det->gfix, det->scale, nv, grec);
    return hipGetLastError();
}

}  // namespace ivrgs
