// Device-side helpers shared by the rasterizer kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ivrgs.h"

namespace ivrgs {

constexpr int kTile = 16;             // tile edge in pixels
constexpr int kTilePix = kTile * kTile;
constexpr int kRecWords = 16;         // floats per projected record: one 64-byte row
constexpr int kRecVec = kRecWords / 4;  // float4 per record
constexpr int kGradRec = 9;           // record-gradient components of the image
constexpr int kGradStride = 10;       // floats between the gradient rows of consecutive records

// Long tile lists are cut for the backward: a list of more than kSplitMin
// records becomes up to kSplitMax segments of equal length (a multiple of 64
// records, the step of the walks), each walked by its own workgroup from a
// per-pixel checkpoint (T, C) that the forward stores at the cut.
constexpr int kSplitMax = 16;
constexpr uint32_t kSplitMin = 128;
constexpr int kCkptPix = 256;  // checkpoint floats4 per (tile, cut): one per pixel

__host__ __device__ __forceinline__ void split_of(uint32_t len, int &nseg, uint32_t &seg_len) {
    if (len <= kSplitMin) {
        nseg = 1;
        seg_len = len;
        return;
    }
    uint32_t n = (len + kSplitMin - 1) / kSplitMin;
    if (n > (uint32_t)kSplitMax) n = kSplitMax;
    seg_len = (len + 64u * n - 1) / (64u * n) * 64u;
    nseg = (int)((len + seg_len - 1) / seg_len);  // every segment nonempty
}
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// Record word indices.
enum { RX = 0, RY, RQA, RQB, RQC, RO, RCR, RCG, RCB, RZ, RCUT, RPAD, RRECT0, RRECT1, RPAD1, RPAD2 };
// Record-gradient rows (kGradStride floats per record).  With d = pixel
// centre - screen mean and D = dL/do'' * G (o'' = o' G the record's power at
// the pixel, o' its opacity) summed over the record's composited pixels:
// GX, GY = sum D dx, sum D dy; GQA, GQB, GQC = sum D dx^2, D dx dy, D dy^2
// (moments; the opacity o', the conic and ln 2 are applied once per record
// by the projection backward); GO = dL/do' = sum D; GCR..GCB = dL/d(rgb).  GZ, past
// the image's components, is dL/d(depth) of the auxiliary maps (their depth
// channel composites each record's camera-space depth).
enum { GX = 0, GY, GQA, GQB, GQC, GO, GCR, GCG, GCB, GZ };
static_assert(GZ == kGradRec && GZ < kGradStride, "the depth slot follows the image's components");

// Compositing constants passed by value to kernels.
struct Consts {
    float alpha_min, alpha_max, T_min, lowpass, z_near;
    float bg0, bg1, bg2;
    int width, height, tiles_x, tiles_y, tiles_per_job;
};

inline Consts make_consts(const ivrgs_params &p) {
    Consts c;
    c.alpha_min = p.alpha_min;
    c.alpha_max = p.alpha_max;
    c.T_min = p.T_min;
    c.lowpass = p.lowpass;
    c.z_near = p.z_near;
    c.bg0 = p.bg[0];
    c.bg1 = p.bg[1];
    c.bg2 = p.bg[2];
    c.width = p.width;
    c.height = p.height;
    c.tiles_x = (p.width + kTile - 1) / kTile;
    c.tiles_y = (p.height + kTile - 1) / kTile;
    c.tiles_per_job = c.tiles_x * c.tiles_y;
    return c;
}

// The Gaussian id of local entry k of a job.
__device__ __forceinline__ int64_t job_gaussian(const ivrgs_job &j, const int32_t *index, int k) {
    return index ? (int64_t)index[j.gauss_begin + k] : (int64_t)j.gauss_begin + k;
}

// 2D Gaussian exponent in log2 units at offset d = p - mean; the exact same
// instruction sequence is used by the forward and the backward recompute.
__device__ __forceinline__ float splat_exponent(float qa, float qb, float qc, float dx, float dy) {
    float t = qa * dx;
    t = fmaf(qb, dy, t);
    float u = qc * dy;
    return fmaf(t, dx, u * dy);
}

// Whether a box of pixels can hold a pixel where a record reaches
// alpha >= alpha_min: the largest exponent qa dx^2 + qb dx dy + qc dy^2 over
// the box of pixel centres (offsets from the mean) is compared with the
// record's cutoff.  The exponent is a concave quadratic, so over a box that
// misses the mean its maximum lies on an edge, where it is a 1D quadratic
// maximised by clamping its vertex.  The test is conservative against FP32
// rounding: a relative margin on the cutoff plus a bound on the rounding of
// the per-pixel evaluation (a few units in the last place of the largest
// term magnitude |qa| X^2 + |qb| X Y + |qc| Y^2 over the box), so a box that
// fails has no pixel whose evaluation would pass the cutoff.
struct HitTest {
    float mx, my, qa, qb, qc, i2qa, i2qc, tol;
};

__device__ __forceinline__ HitTest make_hit_test(const float4 r0, const float4 r1, const float4 r2) {
    HitTest h;
    h.mx = r0.x;
    h.my = r0.y;
    h.qa = r0.z;
    h.qb = r0.w;
    h.qc = r1.x;
    h.i2qa = 0.5f * __builtin_amdgcn_rcpf(h.qa);  // locates a vertex; an error there is second order
    h.i2qc = 0.5f * __builtin_amdgcn_rcpf(h.qc);
    h.tol = r2.z - 1.0e-3f * (1.f + fabsf(r2.z));
    return h;
}

// Box of pixels [px0, px0 + w) x [py0, py0 + h).
__device__ __forceinline__ bool box_hit(const HitTest &h, int px0, int py0, int w, int hgt) {
    const float x0 = (float)px0 + 0.5f - h.mx, x1 = x0 + (float)(w - 1);
    const float y0 = (float)py0 + 0.5f - h.my, y1 = y0 + (float)(hgt - 1);
    if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return true;
    auto q = [&](float dx, float dy) { return fmaf(fmaf(h.qa, dx, h.qb * dy), dx, h.qc * dy * dy); };
    // on the edge x = xe the exponent is maximal at dy = -qb xe / (2 qc), clamped
    const float ya = fminf(fmaxf(-h.qb * x0 * h.i2qc, y0), y1);
    const float yb = fminf(fmaxf(-h.qb * x1 * h.i2qc, y0), y1);
    const float xa = fminf(fmaxf(-h.qb * y0 * h.i2qa, x0), x1);
    const float xb = fminf(fmaxf(-h.qb * y1 * h.i2qa, x0), x1);
    const float best = fmaxf(fmaxf(q(x0, ya), q(x1, yb)), fmaxf(q(xa, y0), q(xb, y1)));
    const float X = fmaxf(fabsf(x0), fabsf(x1)), Y = fmaxf(fabsf(y0), fabsf(y1));
    const float mag = fmaf(fabsf(h.qa) * X, X, fmaf(fabsf(h.qb) * X, Y, fabsf(h.qc) * Y * Y));
    return fmaf(1.0e-6f, mag, best) >= h.tol;
}

// Bounding box, within the wave's 8x8 quadrant at (sx, sy), of the pixels
// whose lanes are set in `alive` (lane l owns pixel (l % 8, l / 8)); `alive`
// must be nonzero.  Scalar bit operations only.  A record that cannot reach
// this box cannot reach a pixel still compositing, and a pixel that has
// terminated ignores every later record, so testing the records of each step
// of the walk against this box instead of the whole quadrant changes no
// result while the walks of the last pixels of a quadrant shrink.
struct PixBox {
    int x0, y0, w, h;
};
__device__ __forceinline__ PixBox alive_box(uint64_t alive, int sx, int sy) {
    uint64_t c = alive | (alive >> 32);
    c |= c >> 16;
    c |= c >> 8;
    const uint32_t cols = (uint32_t)c & 0xFFu;
    const int xa = __builtin_ctz(cols), xb = 31 - __builtin_clz(cols);
    const int ya = __builtin_ctzll(alive) >> 3, yb = (63 - __builtin_clzll(alive)) >> 3;
    return {sx + xa, sy + ya, xb - xa + 1, yb - ya + 1};
}

// Orders this wave's LDS stores before its later loads (and the loads before
// later stores): the lanes of one wave exchange records through LDS.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Sum over the 64 lanes of a wave; the total lands in lane 63.  DPP row
// butterflies give every lane its row sum, then row_bcast15 / row_bcast31
// fold the four rows.
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));  // quad_perm [1,0,3,2]
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));  // quad_perm [2,3,0,1]
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false)); // row_half_mirror
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false)); // row_mirror
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xA, 0xF, false)); // row_bcast15
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xC, 0xF, false)); // row_bcast31
    return v;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Reduce-scatter of 32 per-lane values over the 64 lanes of a wave.  On
// return, lanes 2m and 2m+1 both hold the wave total of value m.  Each
// butterfly level pairs every lane with a partner that holds the same set of
// value indices, keeps one half of the set and adds the partner's copy of it.
// The levels at lane distance 32 and 16 use the permlane swaps: swapping the
// upper half-wave (odd 16-lane rows) of v[k] with the lower half-wave (even
// rows) of v[k + half] leaves in the two registers exactly the pair of
// copies each lane must add, with no select and no trip through LDS.  The
// rest come from DPP (row rotate by 8, half-row mirror, quad permutes).
#define IVRGS_DPP(v, ctrl) __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, (v)), (ctrl), 0xF, 0xF, false))

__device__ __forceinline__ float reduce_scatter32(float v[32]) {
    const int lane = lane_id();
    float a[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[k]), __float_as_uint(v[k + 16]), false,
                                                        false);
        a[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    float b[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a[k]), __float_as_uint(a[k + 8]), false,
                                                        false);
        b[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const bool hi3 = (lane >> 3) & 1, hi2 = (lane >> 2) & 1, hi1 = (lane >> 1) & 1;
    float c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float keep = hi3 ? b[k + 4] : b[k], send = hi3 ? b[k] : b[k + 4];
        c[k] = keep + IVRGS_DPP(send, 0x128);  // row_ror:8, partner lane ^ 8
    }
    float d[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float keep = hi2 ? c[k + 2] : c[k], send = hi2 ? c[k] : c[k + 2];
        d[k] = keep + IVRGS_DPP(send, 0x141);  // row_half_mirror, partner 7 - i
    }
    const float keep = hi1 ? d[1] : d[0], send = hi1 ? d[0] : d[1];
    float e = keep + IVRGS_DPP(send, 0x4E);  // quad_perm [2,3,0,1], partner lane ^ 2
    return e + IVRGS_DPP(e, 0xB1);           // quad_perm [1,0,3,2], partner lane ^ 1
}

// The same butterfly over 64 values, one more level: lane l returns the
// wave's total of v[l].
__device__ __forceinline__ float reduce_scatter64(float v[64]) {
    const int lane = lane_id();
    float a[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[k]), __float_as_uint(v[k + 32]), false,
                                                        false);
        a[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    float b[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a[k]), __float_as_uint(a[k + 16]), false,
                                                        false);
        b[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const bool hi3 = (lane >> 3) & 1, hi2 = (lane >> 2) & 1, hi1 = (lane >> 1) & 1, hi0 = lane & 1;
    float c[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float keep = hi3 ? b[k + 8] : b[k], send = hi3 ? b[k] : b[k + 8];
        c[k] = keep + IVRGS_DPP(send, 0x128);  // row_ror:8, partner lane ^ 8
    }
    float d[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float keep = hi2 ? c[k + 4] : c[k], send = hi2 ? c[k] : c[k + 4];
        d[k] = keep + IVRGS_DPP(send, 0x141);  // row_half_mirror, partner 7 - i
    }
    float e[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float keep = hi1 ? d[k + 2] : d[k], send = hi1 ? d[k] : d[k + 2];
        e[k] = keep + IVRGS_DPP(send, 0x4E);  // quad_perm [2,3,0,1], partner lane ^ 2
    }
    const float keep = hi0 ? e[1] : e[0], send = hi0 ? e[0] : e[1];
    return keep + IVRGS_DPP(send, 0xB1);  // quad_perm [1,0,3,2], partner lane ^ 1
}

}  // namespace ivrgs
