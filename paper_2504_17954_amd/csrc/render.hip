// Front-to-back compositing (forward) and its recompute-based backward.
//
// One workgroup per 16x16 tile; each lane owns PX pixels (PX = 1, 2, 4, so a
// workgroup has 256/PX threads).  The tile's sorted list is consumed in
// batches: every thread gathers one projected record into LDS, then all lanes
// walk the batch reading the record by broadcast.  A workgroup-wide OR ends
// the walk once every pixel has terminated; inside a batch a wave leaves as
// soon as its own pixels are done.  Compositing is plain FP32 VALU work (not a
// dense contraction), so no matrix cores are involved.
//
// The backward walks the same list front to back and recomputes alpha and T
// with the same instruction sequence as the forward.  Nothing per pixel is
// stored by the forward: the colour behind Gaussian i is out_rgb - P_i with
// P_i the recomputed prefix sum, and T_final = 1 - A.  Per-Gaussian partial
// gradients are summed over the wave with DPP and added to the record's
// gradient with one atomic per value.
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
template <int PX, bool kMaxw, bool kCount>
__global__ __launch_bounds__(kTilePix / PX) void k_render_fwd(Consts k, const float4 *__restrict__ rec,
                                                             const uint32_t *__restrict__ starts,
                                                             const uint32_t *__restrict__ sorted, int64_t n_tiles,
                                                             float *__restrict__ out, float *__restrict__ maxw,
                                                             int64_t *__restrict__ status) {
    constexpr int NT = kTilePix / PX;
    __shared__ float4 s0[NT], s1[NT];
    __shared__ float2 s2[NT];
    __shared__ uint32_t sid[NT];
    if (starts[n_tiles] == 0xFFFFFFFFu) return;
    const int64_t tile = blockIdx.x;
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
            s0[threadIdx.x] = rec[3 * (size_t)r];
            s1[threadIdx.x] = rec[3 * (size_t)r + 1];
            const float4 r2 = rec[3 * (size_t)r + 2];
            s2[threadIdx.x] = make_float2(r2.x, r2.z);
            if (kMaxw) sid[threadIdx.x] = r;
        }
        __syncthreads();
        const int cnt = min((uint32_t)NT, end - base);
        for (int i = 0; i < cnt; ++i) {
            if (__ballot(mine) == 0ull) break;
            const float4 a = s0[i];
            const float4 c = s1[i];
            const float2 cc = s2[i];
            const float cb = cc.x;
            float wmax = 0.f;
#pragma unroll
            for (int j = 0; j < PX; ++j) {
                if (!alive[j]) continue;
                if (kCount) ++evaluated;
                const float dx = px[j] - a.x, dy = py[j] - a.y;
                const float p2 = splat_exponent(a.z, a.w, c.x, dx, dy);
                if (p2 < cc.y) continue;  // implies alpha < alpha_min
                const float G = fast_exp2(p2);
                const float al = fminf(k.alpha_max, c.y * G);
                if (al < k.alpha_min) continue;
                const float Tn = T[j] * (1.f - al);
                if (Tn < k.T_min) {
                    alive[j] = false;
                    continue;
                }
                const float w = al * T[j];
                C0[j] = fmaf(w, c.z, C0[j]);
                C1[j] = fmaf(w, c.w, C1[j]);
                C2[j] = fmaf(w, cb, C2[j]);
                T[j] = Tn;
                if (kCount) ++composited;
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

// ----------------------------------------------------------------------------
template <int PX>
__global__ __launch_bounds__(kTilePix / PX) void k_render_bwd(Consts k, const float4 *__restrict__ rec,
                                                             const uint32_t *__restrict__ starts,
                                                             const uint32_t *__restrict__ sorted, int64_t n_tiles,
                                                             const float *__restrict__ rgba,
                                                             const float *__restrict__ dl, float *__restrict__ grec,
                                                             int64_t n_rec) {
    constexpr int NT = kTilePix / PX;
    __shared__ float4 s0[NT], s1[NT];
    __shared__ float2 s2[NT];
    __shared__ uint32_t sid[NT];
    if (starts[n_tiles] == 0xFFFFFFFFu) return;
    const int64_t tile = blockIdx.x;
    const TileGeom tg = tile_geom(k, tile);
    const uint32_t start = starts[tile], end = starts[tile + 1];
    const size_t plane = (size_t)k.width * k.height;
    const float *img = rgba + (size_t)tg.job * 4 * plane;
    const float *gimg = dl + (size_t)tg.job * 4 * plane;

    float px[PX], py[PX], T[PX], P0[PX], P1[PX], P2[PX];
    float o0[PX], o1[PX], o2[PX], Tf[PX], g0[PX], g1[PX], g2[PX], gA[PX];
    bool alive[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        int x, y;
        pixel_of<PX>(tg, j, x, y);
        alive[j] = x < k.width && y < k.height;
        px[j] = (float)x + 0.5f;
        py[j] = (float)y + 0.5f;
        T[j] = 1.f;
        P0[j] = P1[j] = P2[j] = 0.f;
        o0[j] = o1[j] = o2[j] = Tf[j] = g0[j] = g1[j] = g2[j] = gA[j] = 0.f;
        if (alive[j]) {
            const size_t o = (size_t)y * k.width + x;
            o0[j] = img[o];
            o1[j] = img[plane + o];
            o2[j] = img[2 * plane + o];
            Tf[j] = 1.f - img[3 * plane + o];
            g0[j] = gimg[o];
            g1[j] = gimg[plane + o];
            g2[j] = gimg[2 * plane + o];
            gA[j] = gimg[3 * plane + o];
            // a pixel with no upstream gradient contributes nothing
            alive[j] = (g0[j] != 0.f) | (g1[j] != 0.f) | (g2[j] != 0.f) | (gA[j] != 0.f);
        }
    }
    for (uint32_t base = start; base < end; base += NT) {
        bool mine = false;
#pragma unroll
        for (int j = 0; j < PX; ++j) mine |= alive[j];
        if (!__syncthreads_or(mine)) break;
        const uint32_t idx = base + threadIdx.x;
        if (idx < end) {
            const uint32_t r = sorted[idx];
            s0[threadIdx.x] = rec[3 * (size_t)r];
            s1[threadIdx.x] = rec[3 * (size_t)r + 1];
            const float4 r2 = rec[3 * (size_t)r + 2];
            s2[threadIdx.x] = make_float2(r2.x, r2.z);
            sid[threadIdx.x] = r;
        }
        __syncthreads();
        const int cnt = min((uint32_t)NT, end - base);
        for (int i = 0; i < cnt; ++i) {
            if (__ballot(mine) == 0ull) break;
            const float4 a = s0[i];
            const float4 c = s1[i];
            const float2 cc = s2[i];
            const float cb = cc.x;
            float ax = 0.f, ay = 0.f, aqa = 0.f, aqb = 0.f, aqc = 0.f, ao = 0.f, ar = 0.f, ag = 0.f, ab = 0.f;
            bool hit = false;
#pragma unroll
            for (int j = 0; j < PX; ++j) {
                if (!alive[j]) continue;
                const float dx = px[j] - a.x, dy = py[j] - a.y;
                const float p2 = splat_exponent(a.z, a.w, c.x, dx, dy);
                if (p2 < cc.y) continue;  // implies alpha < alpha_min
                const float G = fast_exp2(p2);
                const float raw = c.y * G;
                const float al = fminf(k.alpha_max, raw);
                if (al < k.alpha_min) continue;
                const float Tn = T[j] * (1.f - al);
                if (Tn < k.T_min) {
                    alive[j] = false;
                    continue;
                }
                const float w = al * T[j];
                P0[j] = fmaf(w, c.z, P0[j]);
                P1[j] = fmaf(w, c.w, P1[j]);
                P2[j] = fmaf(w, cb, P2[j]);
                // colour behind this Gaussian, background included
                const float b0 = o0[j] - P0[j], b1 = o1[j] - P1[j], b2 = o2[j] - P2[j];
                const float gc = g0[j] * c.z + g1[j] * c.w + g2[j] * cb;
                const float gb = g0[j] * b0 + g1[j] * b1 + g2[j] * b2;
                const float inv = __builtin_amdgcn_rcpf(1.f - al);
                const float dLda = T[j] * gc - (gb - gA[j] * Tf[j]) * inv;
                ar = fmaf(w, g0[j], ar);
                ag = fmaf(w, g1[j], ag);
                ab = fmaf(w, g2[j], ab);
                if (raw <= k.alpha_max) {
                    ao = fmaf(dLda, G, ao);
                    const float dp = dLda * raw * kLn2;
                    aqa = fmaf(dp, dx * dx, aqa);
                    aqb = fmaf(dp, dx * dy, aqb);
                    aqc = fmaf(dp, dy * dy, aqc);
                    ax = fmaf(-dp, fmaf(2.f * a.z, dx, a.w * dy), ax);
                    ay = fmaf(-dp, fmaf(a.w, dx, 2.f * c.x * dy), ay);
                }
                hit = true;
                T[j] = Tn;
            }
            if (__ballot(hit)) {
                const float sx = wave_sum_to_lane63(ax);
                const float sy = wave_sum_to_lane63(ay);
                const float sqa = wave_sum_to_lane63(aqa);
                const float sqb = wave_sum_to_lane63(aqb);
                const float sqc = wave_sum_to_lane63(aqc);
                const float so = wave_sum_to_lane63(ao);
                const float sr = wave_sum_to_lane63(ar);
                const float sg = wave_sum_to_lane63(ag);
                const float sb = wave_sum_to_lane63(ab);
                if (lane_id() == 63) {
                    const size_t r = sid[i];
                    atomicAdd(&grec[GX * n_rec + r], sx);
                    atomicAdd(&grec[GY * n_rec + r], sy);
                    atomicAdd(&grec[GQA * n_rec + r], sqa);
                    atomicAdd(&grec[GQB * n_rec + r], sqb);
                    atomicAdd(&grec[GQC * n_rec + r], sqc);
                    atomicAdd(&grec[GO * n_rec + r], so);
                    atomicAdd(&grec[GCR * n_rec + r], sr);
                    atomicAdd(&grec[GCG * n_rec + r], sg);
                    atomicAdd(&grec[GCB * n_rec + r], sb);
                }
            }
            mine = false;
#pragma unroll
            for (int j = 0; j < PX; ++j) mine |= alive[j];
        }
    }
}

// ----------------------------------------------------------------------------
template <int PX>
static void fwd_variant(bool maxw, bool count, dim3 grid, hipStream_t s, const Consts &k, const float4 *rec,
                        const uint32_t *starts, const uint32_t *sorted, int64_t n_tiles, float *out, float *mw,
                        int64_t *status) {
    constexpr int NT = kTilePix / PX;
    if (maxw && count)
        hipLaunchKernelGGL((k_render_fwd<PX, true, true>), grid, dim3(NT), 0, s, k, rec, starts, sorted, n_tiles, out, mw, status);
    else if (maxw)
        hipLaunchKernelGGL((k_render_fwd<PX, true, false>), grid, dim3(NT), 0, s, k, rec, starts, sorted, n_tiles, out, mw, status);
    else if (count)
        hipLaunchKernelGGL((k_render_fwd<PX, false, true>), grid, dim3(NT), 0, s, k, rec, starts, sorted, n_tiles, out, mw, status);
    else
        hipLaunchKernelGGL((k_render_fwd<PX, false, false>), grid, dim3(NT), 0, s, k, rec, starts, sorted, n_tiles, out, mw, status);
}

hipError_t launch_render_fwd(const Consts &k, int px, int64_t n_tiles, const float *rec, const uint32_t *starts,
                             const uint32_t *sorted, float *out, float *maxw, int64_t *status, bool count,
                             hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    dim3 grid((unsigned)n_tiles);
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const bool mw = maxw != nullptr;
    TimedScope ts(TK_FWD, s);
    switch (px) {
    case 1: fwd_variant<1>(mw, count, grid, s, k, r4, starts, sorted, n_tiles, out, maxw, status); break;
    case 2: fwd_variant<2>(mw, count, grid, s, k, r4, starts, sorted, n_tiles, out, maxw, status); break;
    default: fwd_variant<4>(mw, count, grid, s, k, r4, starts, sorted, n_tiles, out, maxw, status); break;
    }
    return hipGetLastError();
}

hipError_t launch_render_bwd(const Consts &k, int px, int64_t n_tiles, const float *rec, const uint32_t *starts,
                             const uint32_t *sorted, const float *rgba, const float *dl, float *grec,
                             int64_t n_rec, hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    dim3 grid((unsigned)n_tiles);
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    TimedScope ts(TK_BWD, s);
    switch (px) {
    case 1: hipLaunchKernelGGL(k_render_bwd<1>, grid, dim3(256), 0, s, k, r4, starts, sorted, n_tiles, rgba, dl, grec, n_rec); break;
    case 2: hipLaunchKernelGGL(k_render_bwd<2>, grid, dim3(128), 0, s, k, r4, starts, sorted, n_tiles, rgba, dl, grec, n_rec); break;
    default: hipLaunchKernelGGL(k_render_bwd<4>, grid, dim3(64), 0, s, k, r4, starts, sorted, n_tiles, rgba, dl, grec, n_rec); break;
    }
    return hipGetLastError();
}

}  // namespace ivrgs
