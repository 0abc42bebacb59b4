// Projection of editable Gaussians (EWA + Blinn-Phong), its backward chain,
// and the composition/edit pass.  One thread per (job, Gaussian); attribute
// planes are read component-major so each load instruction is coalesced.
#include "launch.hpp"

namespace ivrgs {

struct Cam {
    float R[9], t[3], fx, fy, cx, cy;
};

__device__ __forceinline__ Cam load_cam(const ivrgs_camera *c) {
    Cam k;
#pragma unroll
    for (int i = 0; i < 9; ++i) k.R[i] = c->R[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) k.t[i] = c->t[i];
    k.fx = c->fx; k.fy = c->fy; k.cx = c->cx; k.cy = c->cy;
    return k;
}

// Camera-space depth of the mean rounded step by step in FP32, in the order
// ((R20 x + R21 y) + R22 z) + t2; this is the sort key.
__device__ __forceinline__ float depth_key(const Cam &c, float x, float y, float z) {
    float s = __fadd_rn(__fmul_rn(c.R[6], x), __fmul_rn(c.R[7], y));
    s = __fadd_rn(s, __fmul_rn(c.R[8], z));
    return __fadd_rn(s, c.t[2]);
}

// Double-float ("hi + lo") helpers for the screen-space mean: the mean is
// an absolute pixel coordinate (hundreds of px), so plain FP32 would put its
// error near 1e-4 px; carrying the camera-space mean and the perspective
// quotient in double-float leaves only the final rounding of the coordinate.
struct DF {
    float hi, lo;
};
__device__ __forceinline__ DF two_prod(float a, float b) {
    const float p = a * b;
    return {p, fmaf(a, b, -p)};
}
__device__ __forceinline__ DF two_sum(float a, float b) {
    const float s = a + b;
    const float bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ DF df_add(DF x, DF y) {
    const DF s = two_sum(x.hi, y.hi);
    const float lo = s.lo + (x.lo + y.lo);
    const float hi = s.hi + lo;
    return {hi, lo - (hi - s.hi)};
}
// fx * (num / den) + cx, rounded once at the end.
__device__ __forceinline__ float df_screen(DF num, DF den, float f, float c) {
    const float q = num.hi / den.hi;
    const float r = (fmaf(-q, den.hi, num.hi) + num.lo) - q * den.lo;
    const float ql = r / den.hi;
    DF m = two_prod(f, q);
    m.lo = fmaf(f, ql, m.lo);
    const DF s = two_sum(m.hi, c);
    return s.hi + (s.lo + m.lo);
}
__device__ __forceinline__ DF df_cam(const float R[3], float t, const float mu[3]) {
    DF s = two_prod(R[0], mu[0]);
    s = df_add(s, two_prod(R[1], mu[1]));
    s = df_add(s, two_prod(R[2], mu[2]));
    return df_add(s, DF{t, 0.f});
}

// Inputs of one Gaussian.
struct GIn {
    float mu[3], ls[3], q[4], o, n[3], c[3], k[4];
};

__device__ __forceinline__ GIn load_gaussian(const ivrgs_gaussians &g, int64_t i) {
    GIn a;
    const int64_t n = g.n;
#pragma unroll
    for (int c = 0; c < 3; ++c) a.mu[c] = g.mean[c * n + i];
#pragma unroll
    for (int c = 0; c < 3; ++c) a.ls[c] = g.log_scale[c * n + i];
#pragma unroll
    for (int c = 0; c < 4; ++c) a.q[c] = g.quat[c * n + i];
    a.o = g.opacity[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) a.n[c] = g.normal[c * n + i];
#pragma unroll
    for (int c = 0; c < 3; ++c) a.c[c] = g.color[c * n + i];
#pragma unroll
    for (int c = 0; c < 4; ++c) a.k[c] = g.shade[c * n + i];
    return a;
}

__device__ __forceinline__ bool all_finite(const GIn &a) {
    bool ok = isfinite(a.o);
#pragma unroll
    for (int c = 0; c < 3; ++c) ok = ok && isfinite(a.mu[c]) && isfinite(a.ls[c]) && isfinite(a.n[c]) && isfinite(a.c[c]);
#pragma unroll
    for (int c = 0; c < 4; ++c) ok = ok && isfinite(a.q[c]) && isfinite(a.k[c]);
    return ok;
}

// Forward intermediates kept for the backward recompute.
struct Fwd {
    float s[3];          // scales
    float qlen, qu[4];   // |q| and unit quaternion
    float Rq[9];         // rotation
    float Sig[6];        // 3D covariance (00 01 02 11 12 22)
    float t[3];          // camera-space mean
    float T[6];          // J W (2x3)
    float a, b, c, det;  // screen covariance [[a,b],[b,c]] incl. low-pass
    float Q00, Q01, Q11;
    float mx, my;
    // shading
    float vlen, v[3], l[3], nlen, nu[3], nl, hlen, h[3], nh, spec_pow;
    bool spec_on;
    float rgb[3];
};

__device__ __forceinline__ void quat_rot(const float q[4], float R[9]) {
    const float w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.f - 2.f * (y * y + z * z);
    R[1] = 2.f * (x * y - w * z);
    R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z);
    R[4] = 1.f - 2.f * (x * x + z * z);
    R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y);
    R[7] = 2.f * (y * z + w * x);
    R[8] = 1.f - 2.f * (x * x + y * y);
}

__device__ __forceinline__ void forward_gaussian(const GIn &a, const Cam &cam, const float cpos[3],
                                                 const ivrgs_model_edit &e, float lowpass, Fwd &f) {
#pragma unroll
    for (int i = 0; i < 3; ++i) f.s[i] = expf(a.ls[i]);
    f.qlen = sqrtf(a.q[0] * a.q[0] + a.q[1] * a.q[1] + a.q[2] * a.q[2] + a.q[3] * a.q[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) f.qu[i] = a.q[i] / f.qlen;
    quat_rot(f.qu, f.Rq);
    float M[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) M[i * 3 + j] = f.Rq[i * 3 + j] * f.s[j];
    f.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    f.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    f.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    f.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    f.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    f.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        f.t[i] = cam.R[i * 3 + 0] * a.mu[0] + cam.R[i * 3 + 1] * a.mu[1] + cam.R[i * 3 + 2] * a.mu[2] + cam.t[i];
    const float iz = 1.f / f.t[2];
    const float j00 = cam.fx * iz, j02 = -cam.fx * f.t[0] * iz * iz;
    const float j11 = cam.fy * iz, j12 = -cam.fy * f.t[1] * iz * iz;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        f.T[j] = j00 * cam.R[j] + j02 * cam.R[6 + j];
        f.T[3 + j] = j11 * cam.R[3 + j] + j12 * cam.R[6 + j];
    }
    // Sigma' = T Sigma T^T
    float S0[3], S1[3];  // Sigma T0^T, Sigma T1^T
    const float *Sg = f.Sig;
    S0[0] = Sg[0] * f.T[0] + Sg[1] * f.T[1] + Sg[2] * f.T[2];
    S0[1] = Sg[1] * f.T[0] + Sg[3] * f.T[1] + Sg[4] * f.T[2];
    S0[2] = Sg[2] * f.T[0] + Sg[4] * f.T[1] + Sg[5] * f.T[2];
    S1[0] = Sg[0] * f.T[3] + Sg[1] * f.T[4] + Sg[2] * f.T[5];
    S1[1] = Sg[1] * f.T[3] + Sg[3] * f.T[4] + Sg[4] * f.T[5];
    S1[2] = Sg[2] * f.T[3] + Sg[4] * f.T[4] + Sg[5] * f.T[5];
    f.a = f.T[0] * S0[0] + f.T[1] * S0[1] + f.T[2] * S0[2] + lowpass;
    f.b = f.T[3] * S0[0] + f.T[4] * S0[1] + f.T[5] * S0[2];
    f.c = f.T[3] * S1[0] + f.T[4] * S1[1] + f.T[5] * S1[2] + lowpass;
    {
        // 2x2 determinant with one rounding on b^2 recovered (Kahan)
        const float bb = f.b * f.b;
        const float bb_lo = fmaf(f.b, f.b, -bb);
        f.det = fmaf(f.a, f.c, -bb) - bb_lo;
    }
    const float idet = 1.f / f.det;
    f.Q00 = f.c * idet;
    f.Q01 = -f.b * idet;
    f.Q11 = f.a * idet;
    {
        const DF tx = df_cam(&cam.R[0], cam.t[0], a.mu), ty = df_cam(&cam.R[3], cam.t[1], a.mu);
        const DF tz = df_cam(&cam.R[6], cam.t[2], a.mu);
        f.mx = df_screen(tx, tz, cam.fx, cam.cx);
        f.my = df_screen(ty, tz, cam.fy, cam.cy);
    }

    // Blinn-Phong (Eq. 3), I_a = I_d = c_v, I_s = white
    float vd[3] = {cpos[0] - a.mu[0], cpos[1] - a.mu[1], cpos[2] - a.mu[2]};
    f.vlen = sqrtf(vd[0] * vd[0] + vd[1] * vd[1] + vd[2] * vd[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) f.v[i] = vd[i] / f.vlen;
    if (e.headlight) {
#pragma unroll
        for (int i = 0; i < 3; ++i) f.l[i] = f.v[i];
    } else {
        const float ll = sqrtf(e.light_dir[0] * e.light_dir[0] + e.light_dir[1] * e.light_dir[1] +
                               e.light_dir[2] * e.light_dir[2]);
#pragma unroll
        for (int i = 0; i < 3; ++i) f.l[i] = e.light_dir[i] / ll;
    }
    f.nlen = sqrtf(a.n[0] * a.n[0] + a.n[1] * a.n[1] + a.n[2] * a.n[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) f.nu[i] = a.n[i] / f.nlen;
    f.nl = f.nu[0] * f.l[0] + f.nu[1] * f.l[1] + f.nu[2] * f.l[2];
    float hv[3] = {f.v[0] + f.l[0], f.v[1] + f.l[1], f.v[2] + f.l[2]};
    f.hlen = sqrtf(hv[0] * hv[0] + hv[1] * hv[1] + hv[2] * hv[2]);
    f.nh = 0.f;
    f.spec_on = false;
    f.spec_pow = 0.f;
    if (f.hlen > 0.f) {
#pragma unroll
        for (int i = 0; i < 3; ++i) f.h[i] = hv[i] / f.hlen;
        f.nh = f.nu[0] * f.h[0] + f.nu[1] * f.h[1] + f.nu[2] * f.h[2];
        const float ah = fabsf(f.nh);
        if (fabsf(f.nl) > 0.f && ah > 0.f) {
            f.spec_on = true;
            f.spec_pow = exp2f(a.k[3] * log2f(ah));  // |n.h|^beta
        }
    } else {
        f.h[0] = f.h[1] = f.h[2] = 0.f;
    }
    const float anl = fabsf(f.nl);
    const float spec = f.spec_on ? a.k[2] * f.spec_pow : 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i) f.rgb[i] = a.k[0] * a.c[i] + a.k[1] * a.c[i] * anl + spec;
}

__device__ __forceinline__ void camera_center(const Cam &c, float p[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] = -(c.R[0 * 3 + i] * c.t[0] + c.R[1 * 3 + i] * c.t[1] + c.R[2 * 3 + i] * c.t[2]);
}

// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_project(ivrgs_batch b, Consts k, float4 *__restrict__ rec,
                                                 uint2 *__restrict__ rect, uint32_t *__restrict__ depth,
                                                 unsigned long long *__restrict__ nonfinite) {
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int local = blockIdx.x * blockDim.x + threadIdx.x;
    if (local >= job.gauss_count) return;
    const int64_t r = (int64_t)job.rec_begin + local;
    const int64_t gi = job_gaussian(job, b.gauss_index, local);
    const Cam cam = load_cam(&b.cameras[job.camera]);
    const GIn a = load_gaussian(b.g, gi);
    int m = b.g.model_id ? b.g.model_id[gi] : 0;
    m = (m >= 0 && m < b.n_models) ? m : 0;
    const ivrgs_model_edit e = b.edits[m];

    const float z32 = depth_key(cam, a.mu[0], a.mu[1], a.mu[2]);
    const bool finite_in = all_finite(a);
    bool bad = !finite_in;  // culled for a value that is not finite
    bool valid = finite_in && z32 > k.z_near && a.o >= k.alpha_min;
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
    uint2 rc = make_uint2(0u, 0u);
    if (valid) {
        float cpos[3];
        camera_center(cam, cpos);
        Fwd f;
        forward_gaussian(a, cam, cpos, e, k.lowpass, f);
        const bool finite_out = isfinite(f.Q00) && isfinite(f.Q01) && isfinite(f.Q11) && isfinite(f.mx) &&
                                isfinite(f.my) && isfinite(f.rgb[0]) && isfinite(f.rgb[1]) && isfinite(f.rgb[2]);
        bad = f.det > 0.f && !finite_out;
        valid = f.det > 0.f && finite_out;
        if (valid) {
            // conservative footprint of {alpha >= alpha_min}: the ellipse
            // d^T Q d <= 2 ln(o / alpha_min) has half-widths k sqrt(a), k sqrt(c)
            const float k2 = fmaxf(2.f * logf(a.o / k.alpha_min), 0.f);
            const float ex = sqrtf(k2 * f.a) * 1.001f + 0.05f;
            const float ey = sqrtf(k2 * f.c) * 1.001f + 0.05f;
            // pixel columns whose centres i + 0.5 lie in [mx - ex, mx + ex]
            const float lim = 1.0e7f;
            const float fx0 = fminf(fmaxf(ceilf(f.mx - ex - 0.5f), -lim), lim);
            const float fx1 = fminf(fmaxf(floorf(f.mx + ex - 0.5f), -lim), lim);
            const float fy0 = fminf(fmaxf(ceilf(f.my - ey - 0.5f), -lim), lim);
            const float fy1 = fminf(fmaxf(floorf(f.my + ey - 0.5f), -lim), lim);
            const int px0 = max((int)fx0, 0), px1 = min((int)fx1, k.width - 1);
            const int py0 = max((int)fy0, 0), py1 = min((int)fy1, k.height - 1);
            if (px0 <= px1 && py0 <= py1) {
                const uint32_t tx0 = px0 / kTile, tx1 = px1 / kTile + 1;
                const uint32_t ty0 = py0 / kTile, ty1 = py1 / kTile + 1;
                rc = make_uint2(tx0 | (ty0 << 16), tx1 | (ty1 << 16));
                r0 = make_float4(f.mx, f.my, -0.5f * kLog2e * f.Q00, -kLog2e * f.Q01);
                r1 = make_float4(-0.5f * kLog2e * f.Q11, a.o, f.rgb[0], f.rgb[1]);
                // exponent below which alpha < alpha_min for sure
                const float cut = log2f(k.alpha_min / a.o) - 1.0e-3f;
                r2 = make_float4(f.rgb[2], z32, cut, 0.f);
            }
        }
    }
    rec[kRecVec * r + 0] = r0;
    rec[kRecVec * r + 1] = r1;
    rec[kRecVec * r + 2] = r2;
    // the tile rectangle also in the row, so that the binning's gather of a
    // record in depth order reads one 64-byte row
    rec[kRecVec * r + 3] = make_float4(__uint_as_float(rc.x), __uint_as_float(rc.y), 0.f, 0.f);
    rect[r] = rc;
    depth[r] = (rc.x | rc.y) ? __float_as_uint(z32) : 0xFFFFFFFFu;
    if (nonfinite) {
        const uint64_t nb = __ballot(bad);
        if (nb && lane_id() == (int)__builtin_ctzll(nb)) atomicAdd(nonfinite, (unsigned long long)__popcll(nb));
    }
}

// Shading backward (Eq. 3): from the record's colour gradient gr[GCR..GCB],
// the gradients with respect to the colour c_v, the coefficients (k_a, k_d,
// k_s, beta), the unit normal, the unit light direction and (through the
// half vector only) the unit view direction.
__device__ __forceinline__ void shade_bwd(const GIn &a, const Fwd &f, const float gr[kGradRec], float g_c[3],
                                          float g_k[4], float g_nu[3], float g_l[3], float g_v[3]) {
    // ---- shading: rgb = k_a c + k_d c |n.l| + k_s |n.h|^beta [..]
    const float anl = fabsf(f.nl);
    const float gsum = gr[GCR] + gr[GCG] + gr[GCB];
    const float gcdot = gr[GCR] * a.c[0] + gr[GCG] * a.c[1] + gr[GCB] * a.c[2];
    g_c[0] = gr[GCR] * (a.k[0] + a.k[1] * anl);
    g_c[1] = gr[GCG] * (a.k[0] + a.k[1] * anl);
    g_c[2] = gr[GCB] * (a.k[0] + a.k[1] * anl);
    g_k[0] = gcdot;
    g_k[1] = gcdot * anl;
    g_k[2] = 0.f;
    g_k[3] = 0.f;
    float g_h[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 3; ++i) g_nu[i] = g_l[i] = g_v[i] = 0.f;
    const float sgn_nl = f.nl > 0.f ? 1.f : (f.nl < 0.f ? -1.f : 0.f);
    const float g_nl = a.k[1] * gcdot * sgn_nl;
    if (f.spec_on) {
        const float ah = fabsf(f.nh);
        g_k[2] = gsum * f.spec_pow;
        g_k[3] = gsum * a.k[2] * f.spec_pow * logf(ah);
        const float g_ah = gsum * a.k[2] * a.k[3] * f.spec_pow / ah;  // beta a^(beta-1)
        const float g_nh = g_ah * (f.nh > 0.f ? 1.f : -1.f);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            g_nu[i] += g_nh * f.h[i];
            g_h[i] = g_nh * f.nu[i];
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        g_nu[i] += g_nl * f.l[i];
        g_l[i] += g_nl * f.nu[i];
    }
    if (f.hlen > 0.f) {
        const float hd = f.h[0] * g_h[0] + f.h[1] * g_h[1] + f.h[2] * g_h[2];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float ghv = (g_h[i] - f.h[i] * hd) / f.hlen;
            g_v[i] += ghv;
            g_l[i] += ghv;
        }
    }
}

// ----------------------------------------------------------------------------
// Backward: record gradients (dL/d mx, my, qa, qb, qc, o, r, g, b) -> the 21
// parameter gradients, by the chain rule through the forward above.
// kDense (one job over every Gaussian, no index list): each Gaussian is
// written exactly once, zeros included, so the output needs no clearing.
// kOut: how a Gaussian's gradient reaches `out`: stored (kOutStore), added
// with float atomics (kOutAtomic: several jobs of one launch may share it) or
// added without atomics (kOutAccum: one launch per job, in job order, so the
// sums do not depend on the order of the atomics).  kDepth: the rows also
// carry dL/d(depth) of the auxiliary maps (slot GZ), which reaches the mean
// through the camera-space depth.
enum { kOutStore = 0, kOutAtomic = 1, kOutAccum = 2 };
template <int kOut, bool kDense, bool kDepth>
__global__ __launch_bounds__(256) void k_project_bwd(ivrgs_batch b, Consts k, const uint2 *__restrict__ rect,
                                                     const float *__restrict__ grec, ivrgs_gaussians_mut out) {
    static_assert(!(kOut != kOutStore && kDense), "dense output is written, not accumulated");
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int local = blockIdx.x * blockDim.x + threadIdx.x;
    if (local >= job.gauss_count) return;
    const int64_t r = (int64_t)job.rec_begin + local;
    auto zero = [&]() {
        if constexpr (kDense) {
            const int64_t gi = (int64_t)job.gauss_begin + local, n = out.n;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                out.mean[c * n + gi] = 0.f;
                out.log_scale[c * n + gi] = 0.f;
                out.normal[c * n + gi] = 0.f;
                out.color[c * n + gi] = 0.f;
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                out.quat[c * n + gi] = 0.f;
                out.shade[c * n + gi] = 0.f;
            }
            out.opacity[gi] = 0.f;
        }
    };
    const uint2 rc = rect[r];
    if (rc.x == 0u && rc.y == 0u) {  // culled
        zero();
        return;
    }
    float gr[kGradRec];
#pragma unroll
    for (int i = 0; i < kGradRec; ++i) gr[i] = grec[r * kGradStride + i];
    const float gz = kDepth ? grec[r * kGradStride + GZ] : 0.f;
    bool any = gz != 0.f;
#pragma unroll
    for (int i = 0; i < kGradRec; ++i) any |= gr[i] != 0.f;
    if (!any) {
        zero();
        return;
    }

    const int64_t gi = job_gaussian(job, b.gauss_index, local);
    const Cam cam = load_cam(&b.cameras[job.camera]);
    const GIn a = load_gaussian(b.g, gi);
    int m = b.g.model_id ? b.g.model_id[gi] : 0;
    m = (m >= 0 && m < b.n_models) ? m : 0;
    const ivrgs_model_edit e = b.edits[m];
    float cpos[3];
    camera_center(cam, cpos);
    Fwd f;
    forward_gaussian(a, cam, cpos, e, k.lowpass, f);
    // the moments were summed without the record's opacity factor
#pragma unroll
    for (int i = GX; i <= GQC; ++i) gr[i] *= a.o;

    float g_mu[3] = {0.f, 0.f, 0.f}, g_ls[3], g_q[4], g_n[3], g_c[3], g_k[4];
    const float g_o = gr[GO];
    float g_nu[3], g_l[3], g_v[3];
    shade_bwd(a, f, gr, g_c, g_k, g_nu, g_l, g_v);
    if (e.headlight) {
#pragma unroll
        for (int i = 0; i < 3; ++i) g_v[i] += g_l[i];
    }
    {
        const float vd = f.v[0] * g_v[0] + f.v[1] * g_v[1] + f.v[2] * g_v[2];
#pragma unroll
        for (int i = 0; i < 3; ++i) g_mu[i] -= (g_v[i] - f.v[i] * vd) / f.vlen;  // v = (c - mu)/|c - mu|
        const float nd = f.nu[0] * g_nu[0] + f.nu[1] * g_nu[1] + f.nu[2] * g_nu[2];
#pragma unroll
        for (int i = 0; i < 3; ++i) g_n[i] = (g_nu[i] - f.nu[i] * nd) / f.nlen;
    }

    // ---- conic: the exponent is -(Q00 dx^2 + 2 Q01 dx dy + Q11 dy^2) / 2
    // (base e), so from the moments D dx^2, D dx dy, D dy^2:
    const float gQ00 = -0.5f * gr[GQA];
    const float gQ01 = -gr[GQB];
    const float gQ11 = -0.5f * gr[GQC];
    // and the screen mean (d = pixel - mean): dL/dm = Q (sum D d)
    const float gmx = f.Q00 * gr[GX] + f.Q01 * gr[GY];
    const float gmy = f.Q01 * gr[GX] + f.Q11 * gr[GY];
    // dL/dSigma' (full symmetric) = -Q G Q, G = [[gQ00, gQ01/2], [gQ01/2, gQ11]]
    const float G01 = 0.5f * gQ01;
    const float A00 = f.Q00 * gQ00 + f.Q01 * G01, A01 = f.Q00 * G01 + f.Q01 * gQ11;
    const float A10 = f.Q01 * gQ00 + f.Q11 * G01, A11 = f.Q01 * G01 + f.Q11 * gQ11;
    const float S00 = -(A00 * f.Q00 + A01 * f.Q01);
    const float S01 = -(A00 * f.Q01 + A01 * f.Q11);
    const float S11 = -(A10 * f.Q01 + A11 * f.Q11);
    // Sigma' = T Sigma T^T: dSigma = T^T S T, dT = 2 S T Sigma
    float TS[6];  // T Sigma (2x3)
    {
        const float *Sg = f.Sig;
        const float Sfull[9] = {Sg[0], Sg[1], Sg[2], Sg[1], Sg[3], Sg[4], Sg[2], Sg[4], Sg[5]};
#pragma unroll
        for (int r2 = 0; r2 < 2; ++r2)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                TS[r2 * 3 + j] = f.T[r2 * 3 + 0] * Sfull[0 * 3 + j] + f.T[r2 * 3 + 1] * Sfull[1 * 3 + j] +
                                 f.T[r2 * 3 + 2] * Sfull[2 * 3 + j];
    }
    float gT[6];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        gT[j] = 2.f * (S00 * TS[j] + S01 * TS[3 + j]);
        gT[3 + j] = 2.f * (S01 * TS[j] + S11 * TS[3 + j]);
    }
    float gSig[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            gSig[i * 3 + j] = f.T[i] * (S00 * f.T[j] + S01 * f.T[3 + j]) +
                              f.T[3 + i] * (S01 * f.T[j] + S11 * f.T[3 + j]);
    // T = J W -> dJ = dT W^T; only J00, J02, J11, J12 are variable
    float gJ[6];
#pragma unroll
    for (int r2 = 0; r2 < 2; ++r2)
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
            gJ[r2 * 3 + kk] = gT[r2 * 3 + 0] * cam.R[kk * 3 + 0] + gT[r2 * 3 + 1] * cam.R[kk * 3 + 1] +
                              gT[r2 * 3 + 2] * cam.R[kk * 3 + 2];
    const float iz = 1.f / f.t[2], iz2 = iz * iz, iz3 = iz2 * iz;
    float gt[3];
    gt[0] = gJ[2] * (-cam.fx * iz2) + gmx * cam.fx * iz;
    gt[1] = gJ[5] * (-cam.fy * iz2) + gmy * cam.fy * iz;
    gt[2] = gJ[0] * (-cam.fx * iz2) + gJ[2] * (2.f * cam.fx * f.t[0] * iz3) + gJ[4] * (-cam.fy * iz2) +
            gJ[5] * (2.f * cam.fy * f.t[1] * iz3) - gmx * cam.fx * f.t[0] * iz2 -
            gmy * cam.fy * f.t[1] * iz2 + gz;
#pragma unroll
    for (int i = 0; i < 3; ++i) g_mu[i] += cam.R[0 * 3 + i] * gt[0] + cam.R[1 * 3 + i] * gt[1] + cam.R[2 * 3 + i] * gt[2];

    // ---- Sigma = M M^T, M = R diag(s): dM = 2 dSigma M (dSigma symmetric)
    float gM[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float acc = 0.f;
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) acc += (gSig[i * 3 + kk] + gSig[kk * 3 + i]) * f.Rq[kk * 3 + j] * f.s[j];
            gM[i * 3 + j] = acc;
        }
    float gR[9];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        float gs = 0.f;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            gR[i * 3 + j] = gM[i * 3 + j] * f.s[j];
            gs += gM[i * 3 + j] * f.Rq[i * 3 + j];
        }
        g_ls[j] = gs * f.s[j];
    }
    // rotation matrix -> unit quaternion -> raw quaternion
    {
        const float w = f.qu[0], x = f.qu[1], y = f.qu[2], z = f.qu[3];
        float gu[4];
        gu[0] = 2.f * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
        gu[1] = 2.f * (y * gR[1] + z * gR[2] + y * gR[3] - 2.f * x * gR[4] - w * gR[5] + z * gR[6] + w * gR[7] -
                       2.f * x * gR[8]);
        gu[2] = 2.f * (-2.f * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] + z * gR[7] -
                       2.f * y * gR[8]);
        gu[3] = 2.f * (-2.f * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.f * z * gR[4] + y * gR[5] +
                       x * gR[6] + y * gR[7]);
        const float dd = w * gu[0] + x * gu[1] + y * gu[2] + z * gu[3];
#pragma unroll
        for (int i = 0; i < 4; ++i) g_q[i] = (gu[i] - f.qu[i] * dd) / f.qlen;
    }

    const int64_t n = out.n;
    if (kOut == kOutAtomic) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            atomicAdd(&out.mean[c * n + gi], g_mu[c]);
            atomicAdd(&out.log_scale[c * n + gi], g_ls[c]);
            atomicAdd(&out.normal[c * n + gi], g_n[c]);
            atomicAdd(&out.color[c * n + gi], g_c[c]);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            atomicAdd(&out.quat[c * n + gi], g_q[c]);
            atomicAdd(&out.shade[c * n + gi], g_k[c]);
        }
        atomicAdd(&out.opacity[gi], g_o);
    } else if (kOut == kOutAccum) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            out.mean[c * n + gi] += g_mu[c];
            out.log_scale[c * n + gi] += g_ls[c];
            out.normal[c * n + gi] += g_n[c];
            out.color[c * n + gi] += g_c[c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            out.quat[c * n + gi] += g_q[c];
            out.shade[c * n + gi] += g_k[c];
        }
        out.opacity[gi] += g_o;
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            out.mean[c * n + gi] = g_mu[c];
            out.log_scale[c * n + gi] = g_ls[c];
            out.normal[c * n + gi] = g_n[c];
            out.color[c * n + gi] = g_c[c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            out.quat[c * n + gi] = g_q[c];
            out.shade[c * n + gi] = g_k[c];
        }
        out.opacity[gi] = g_o;
    }
}

// ----------------------------------------------------------------------------
// Composition: one launch covers up to kComposeModels basic models; a thread
// writes 4 consecutive Gaussians of one model, as float4 loads and stores
// where the model's source planes and its output slice are 16-byte aligned.
struct ComposeArgs {
    ivrgs_gaussians src[kComposeModels];
    int64_t offset[kComposeModels];  // first output index of each model
    int64_t quad[kComposeModels + 1];  // first thread of each model (4 Gaussians per thread)
    int32_t model0;                  // model number of src[0]
    int32_t count;
    float edit[kComposeModels][12];  // palette 3, opacity scale, shade scale 4, shade bias 4 (host rows)
};

__device__ __forceinline__ bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0u; }

// table != nullptr: the edit values come from the device rows table[model]
// (the same for every thread of the model); else from the host rows in `a`.
__global__ __launch_bounds__(256) void k_compose(ComposeArgs a, const ivrgs_model_edit *__restrict__ table,
                                                 ivrgs_gaussians_mut out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.quad[a.count]) return;
    int j = 0;
    while (j + 1 < a.count && t >= a.quad[j + 1]) ++j;
    const ivrgs_gaussians &src = a.src[j];
    const int64_t n = src.n, N = out.n, i0 = 4 * (t - a.quad[j]), o0 = a.offset[j] + i0;
    const int model = a.model0 + j;
    float e[12];
    if (table) {
        const ivrgs_model_edit &r = table[model];
#pragma unroll
        for (int c = 0; c < 3; ++c) e[c] = r.palette[c];
        e[3] = r.opacity_scale;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            e[4 + c] = r.shade_scale[c];
            e[8 + c] = r.shade_bias[c];
        }
    } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) e[c] = a.edit[j][c];
    }
    // the whole quad in range, the model's planes (n % 4 == 0) and its output
    // slice (N % 4 == 0, offset % 4 == 0) on 16-byte boundaries
    const bool vec = i0 + 4 <= n && (n & 3) == 0 && (N & 3) == 0 && (a.offset[j] & 3) == 0 &&
                     aligned16(src.mean) && aligned16(src.log_scale) && aligned16(src.quat) &&
                     aligned16(src.opacity) && aligned16(src.normal) && aligned16(src.color) &&
                     aligned16(src.shade) && aligned16(out.mean) && aligned16(out.log_scale) &&
                     aligned16(out.quat) && aligned16(out.opacity) && aligned16(out.normal) &&
                     aligned16(out.color) && aligned16(out.shade) && aligned16(out.model_id);
    if (vec) {
        auto ld = [](const float *p) { return *reinterpret_cast<const float4 *>(p); };
        // streaming stores: the composed planes are not read again by this kernel
        auto st = [](float *p, float4 v) {
            typedef float f4v __attribute__((ext_vector_type(4)));
            __builtin_nontemporal_store(f4v{v.x, v.y, v.z, v.w}, reinterpret_cast<f4v *>(p));
        };
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            st(out.mean + c * N + o0, ld(src.mean + c * n + i0));
            st(out.log_scale + c * N + o0, ld(src.log_scale + c * n + i0));
            st(out.normal + c * N + o0, ld(src.normal + c * n + i0));
            const float4 v = ld(src.color + c * n + i0);
            st(out.color + c * N + o0, make_float4(e[c] + v.x, e[c] + v.y, e[c] + v.z, e[c] + v.w));
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            st(out.quat + c * N + o0, ld(src.quat + c * n + i0));
            const float4 v = ld(src.shade + c * n + i0);
            const float ks = e[4 + c], kb = e[8 + c];
            st(out.shade + c * N + o0, make_float4(fmaf(ks, v.x, kb), fmaf(ks, v.y, kb), fmaf(ks, v.z, kb),
                                                   fmaf(ks, v.w, kb)));
        }
        const float4 v = ld(src.opacity + i0);
        st(out.opacity + o0, make_float4(e[3] * v.x, e[3] * v.y, e[3] * v.z, e[3] * v.w));
        typedef int i4v __attribute__((ext_vector_type(4)));
        __builtin_nontemporal_store(i4v{model, model, model, model}, reinterpret_cast<i4v *>(out.model_id + o0));
        return;
    }
    for (int64_t i = i0; i < i0 + 4 && i < n; ++i) {
        const int64_t o = a.offset[j] + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            out.mean[c * N + o] = src.mean[c * n + i];
            out.log_scale[c * N + o] = src.log_scale[c * n + i];
            out.normal[c * N + o] = src.normal[c * n + i];
            out.color[c * N + o] = e[c] + src.color[c * n + i];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            out.quat[c * N + o] = src.quat[c * n + i];
            out.shade[c * N + o] = fmaf(e[4 + c], src.shade[c * n + i], e[8 + c]);
        }
        out.opacity[o] = e[3] * src.opacity[i];
        out.model_id[o] = model;
    }
}

// ----------------------------------------------------------------------------
// Inverse volume exploration (Sec. 4.6) learns, per basic model, the palette
// colour, the opacity scale and the light-magnitude transform lambda * k + b,
// and the orbital light direction.  Their gradients are reductions of the
// per-Gaussian gradients over each model's Gaussians.

// Sum of v over the wave, in every lane.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// dL/d(light direction of the record's model), the unnormalised vector of
// the edit row: with l = d / |d|, dL/dd = (dL/dl - l (l . dL/dl)) / |d|.
// Headlight models get nothing (their light is the view direction).  Waves
// whose records all belong to one model add one sum per component.
__global__ __launch_bounds__(256) void k_light_bwd(ivrgs_batch b, Consts k, const uint2 *__restrict__ rect,
                                                   const float *__restrict__ grec, float *__restrict__ out) {
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int local = blockIdx.x * blockDim.x + threadIdx.x;
    float g[3] = {0.f, 0.f, 0.f};
    int m = -1;
    if (local < job.gauss_count) {
        const int64_t r = (int64_t)job.rec_begin + local;
        const uint2 rc = rect[r];
        if (rc.x | rc.y) {
            float gr[kGradRec];
            bool any = false;
#pragma unroll
            for (int i = 0; i < kGradRec; ++i) {
                gr[i] = grec[r * kGradStride + i];
                any |= gr[i] != 0.f;
            }
            const int64_t gi = job_gaussian(job, b.gauss_index, local);
            int mm = b.g.model_id ? b.g.model_id[gi] : 0;
            mm = (mm >= 0 && mm < b.n_models) ? mm : 0;
            const ivrgs_model_edit e = b.edits[mm];
            if (any && !e.headlight) {
                const Cam cam = load_cam(&b.cameras[job.camera]);
                const GIn a = load_gaussian(b.g, gi);
                float cpos[3];
                camera_center(cam, cpos);
                Fwd f;
                forward_gaussian(a, cam, cpos, e, k.lowpass, f);
                float g_c[3], g_k[4], g_nu[3], g_l[3], g_v[3];
                shade_bwd(a, f, gr, g_c, g_k, g_nu, g_l, g_v);
                const float dlen = sqrtf(e.light_dir[0] * e.light_dir[0] + e.light_dir[1] * e.light_dir[1] +
                                         e.light_dir[2] * e.light_dir[2]);
                const float ld = f.l[0] * g_l[0] + f.l[1] * g_l[1] + f.l[2] * g_l[2];
#pragma unroll
                for (int i = 0; i < 3; ++i) g[i] = (g_l[i] - f.l[i] * ld) / dlen;
                m = mm;
            }
        }
    }
    const uint64_t act = __ballot(m >= 0);
    if (act == 0ull) return;
    const int m0 = __shfl(m, (int)__builtin_ctzll(act), 64);
    if (__ballot(m >= 0 && m != m0) == 0ull) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float s = wave_sum(g[i]);
            if ((threadIdx.x & 63) == 0) atomicAdd(&out[3 * m0 + i], s);
        }
    } else if (m >= 0) {
#pragma unroll
        for (int i = 0; i < 3; ++i) atomicAdd(&out[3 * m + i], g[i]);
    }
}

// One model's 12 edit-parameter gradients (palette 3, opacity scale, shade
// scale 4, shade bias 4) from the gradients of its slice [offset, offset + n)
// of the composed set: a grid-stride sum per thread, then the wave, then the
// workgroup, then one atomic per value per workgroup.
__global__ __launch_bounds__(256) void k_compose_bwd(ivrgs_gaussians src, int64_t offset,
                                                     const ivrgs_gaussians_mut grads, float *__restrict__ out) {
    __shared__ float part[4][12];
    const int64_t n = src.n, N = grads.n;
    float v[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) v[j] = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = offset + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] += grads.color[c * N + o];
        v[3] = fmaf(grads.opacity[o], src.opacity[i], v[3]);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float gk = grads.shade[c * N + o];
            v[4 + c] = fmaf(gk, src.shade[c * n + i], v[4 + c]);
            v[8 + c] += gk;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        const float s = wave_sum(v[j]);
        if (lane == 0) part[wave][j] = s;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        const float s = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] + part[3][threadIdx.x];
        atomicAdd(&out[threadIdx.x], s);
    }
}

// One Adam step (Kingma and Ba, 2015) of the exploration parameters
// [palette K*3 | s_o K | lambda 4 | b 4 | polar, azimuth], then the edit rows
// rebuilt from them.  The shared lambda, b and angles sum the per-model
// gradients; d(t, p) = (sin t cos p, sin t sin p, cos t) gives
// dL/dt = g.(cos t cos p, cos t sin p, -sin t), dL/dp = g.(-sin t sin p, sin t cos p, 0).
__global__ __launch_bounds__(256) void k_explore_step(const float *__restrict__ eg, const float *__restrict__ lg,
                                                      int K, ExploreOpts o, float *__restrict__ st,
                                                      ivrgs_model_edit *__restrict__ rows) {
    const int n = 4 * K + 10;
    float *p = st, *m = st + n, *v = st + 2 * n;
    const float t = st[3 * n] + 1.f;
    const float c1 = 1.f - powf(o.beta1, t), c2 = 1.f - powf(o.beta2, t);
    const float th = p[4 * K + 8], ph = p[4 * K + 9];
    __syncthreads();  // every wave has read the angles before any update
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const uint32_t group = j < 3 * K ? 1u : j < 4 * K ? 2u : j < 4 * K + 8 ? 4u : 8u;
        if (!(o.learn & group) || (group == 8u && lg == nullptr)) continue;
        float g = 0.f;
        if (group == 1u) {
            g = eg[(j / 3) * 12 + j % 3];
        } else if (group == 2u) {
            g = eg[(j - 3 * K) * 12 + 3];
        } else if (group == 4u) {
            const int c = 4 + (j - 4 * K);  // lambda: columns 4..7, b: 8..11
            for (int k = 0; k < K; ++k) g += eg[k * 12 + c];
        } else {
            float gd[3] = {0.f, 0.f, 0.f};
            for (int k = 0; k < K; ++k)
                for (int i = 0; i < 3; ++i) gd[i] += lg[k * 3 + i];
            const float sth = sinf(th), cth = cosf(th), sph = sinf(ph), cph = cosf(ph);
            g = (j == 4 * K + 8) ? gd[0] * cth * cph + gd[1] * cth * sph - gd[2] * sth
                                 : -gd[0] * sth * sph + gd[1] * sth * cph;
        }
        const float mj = o.beta1 * m[j] + (1.f - o.beta1) * g;
        const float vj = o.beta2 * v[j] + (1.f - o.beta2) * g * g;
        m[j] = mj;
        v[j] = vj;
        p[j] -= o.lr * (mj / c1) / (sqrtf(vj / c2) + o.eps);
    }
    __syncthreads();
    if (threadIdx.x == 0 && o.learn != 0u) st[3 * n] = t;
    const float nth = p[4 * K + 8], nph = p[4 * K + 9];
    const float d[3] = {sinf(nth) * cosf(nph), sinf(nth) * sinf(nph), cosf(nth)};
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        ivrgs_model_edit &e = rows[k];
        for (int c = 0; c < 3; ++c) e.palette[c] = p[3 * k + c];
        e.opacity_scale = p[3 * K + k];
        for (int c = 0; c < 4; ++c) {
            e.shade_scale[c] = p[4 * K + c];
            e.shade_bias[c] = p[4 * K + 4 + c];
        }
        if (e.headlight == 0)
            for (int c = 0; c < 3; ++c) e.light_dir[c] = d[c];
    }
}

// ----------------------------------------------------------------------------
// host launchers
hipError_t launch_project(const ivrgs_batch &b, const Consts &k, float *rec, uint32_t *rect, uint32_t *depth,
                          int64_t *nonfinite, hipStream_t s) {
    if (b.n_jobs == 0 || b.max_job_count == 0) return hipSuccess;
    dim3 grid((b.max_job_count + 255) / 256, b.n_jobs);
    TimedScope ts(TK_PROJECT, s);
    hipLaunchKernelGGL(k_project, grid, dim3(256), 0, s, b, k, reinterpret_cast<float4 *>(rec),
                       reinterpret_cast<uint2 *>(rect), depth, reinterpret_cast<unsigned long long *>(nonfinite));
    return hipGetLastError();
}

template <bool kDepth>
static void project_bwd_variant(const ivrgs_batch &b, const Consts &k, const uint2 *rc, const float *grec,
                                const ivrgs_gaussians_mut &out, bool atomic, bool dense, hipStream_t s,
                                bool job_order) {
    dim3 grid((b.max_job_count + 255) / 256, b.n_jobs);
    if (atomic && job_order) {
        // one launch per job, in job order, each adding its Gaussians'
        // gradients (a job lists a Gaussian at most once)
        for (int j = 0; j < b.n_jobs; ++j) {
            ivrgs_batch bj = b;
            bj.jobs = b.jobs + j;
            bj.n_jobs = 1;
            hipLaunchKernelGGL((k_project_bwd<kOutAccum, false, kDepth>), dim3(grid.x, 1), dim3(256), 0, s, bj, k,
                               rc, grec, out);
        }
    } else if (atomic) {
        hipLaunchKernelGGL((k_project_bwd<kOutAtomic, false, kDepth>), grid, dim3(256), 0, s, b, k, rc, grec, out);
    } else if (dense) {
        hipLaunchKernelGGL((k_project_bwd<kOutStore, true, kDepth>), grid, dim3(256), 0, s, b, k, rc, grec, out);
    } else {
        hipLaunchKernelGGL((k_project_bwd<kOutStore, false, kDepth>), grid, dim3(256), 0, s, b, k, rc, grec, out);
    }
}

hipError_t launch_project_bwd(const ivrgs_batch &b, const Consts &k, const uint32_t *rect, const float *grec,
                              const ivrgs_gaussians_mut &out, bool atomic, bool dense, hipStream_t s,
                              bool job_order, bool depth) {
    if (b.n_jobs == 0 || b.max_job_count == 0) return hipSuccess;
    const uint2 *rc = reinterpret_cast<const uint2 *>(rect);
    TimedScope ts(TK_PROJECT_BWD, s);
    if (depth)
        project_bwd_variant<true>(b, k, rc, grec, out, atomic, dense, s, job_order);
    else
        project_bwd_variant<false>(b, k, rc, grec, out, atomic, dense, s, job_order);
    return hipGetLastError();
}

hipError_t launch_compose(const ivrgs_gaussians *src, const int64_t *offset, int32_t model0, int32_t count,
                          const ivrgs_model_edit *host_e, const ivrgs_model_edit *dev_table,
                          const ivrgs_gaussians_mut &out, hipStream_t s) {
    if (count <= 0 || count > kComposeModels) return hipErrorInvalidValue;
    ComposeArgs a = {};
    a.model0 = model0;
    a.count = count;
    a.quad[0] = 0;
    for (int j = 0; j < count; ++j) {
        a.src[j] = src[j];
        a.offset[j] = offset[j];
        a.quad[j + 1] = a.quad[j] + (src[j].n + 3) / 4;
        if (host_e) {
            const ivrgs_model_edit &r = host_e[j];
            for (int c = 0; c < 3; ++c) a.edit[j][c] = r.palette[c];
            a.edit[j][3] = r.opacity_scale;
            for (int c = 0; c < 4; ++c) {
                a.edit[j][4 + c] = r.shade_scale[c];
                a.edit[j][8 + c] = r.shade_bias[c];
            }
        }
    }
    if (a.quad[count] == 0) return hipSuccess;
    dim3 grid((unsigned)((a.quad[count] + 255) / 256));
    TimedScope ts(TK_COMPOSE, s);
    hipLaunchKernelGGL(k_compose, grid, dim3(256), 0, s, a, host_e ? nullptr : dev_table, out);
    return hipGetLastError();
}

hipError_t launch_light_bwd(const ivrgs_batch &b, const Consts &k, const uint32_t *rect, const float *grec,
                            float *out, hipStream_t s) {
    if (b.n_jobs == 0 || b.max_job_count == 0) return hipSuccess;
    dim3 grid((b.max_job_count + 255) / 256, b.n_jobs);
    TimedScope ts(TK_EDIT_BWD, s);
    hipLaunchKernelGGL(k_light_bwd, grid, dim3(256), 0, s, b, k, reinterpret_cast<const uint2 *>(rect), grec, out);
    return hipGetLastError();
}

hipError_t launch_explore_step(const float *edit_grad, const float *light_grad, int n_models, const ExploreOpts &o,
                               float *state, ivrgs_model_edit *rows, hipStream_t s) {
    TimedScope ts(TK_EDIT_BWD, s);
    hipLaunchKernelGGL(k_explore_step, dim3(1), dim3(256), 0, s, edit_grad, light_grad, n_models, o, state, rows);
    return hipGetLastError();
}

hipError_t launch_compose_bwd(const ivrgs_gaussians &src, int64_t offset, const ivrgs_gaussians_mut &grads,
                              float *out, hipStream_t s) {
    if (src.n == 0) return hipSuccess;
    const int64_t want = (src.n + 255) / 256;
    const unsigned blocks = (unsigned)(want < 1024 ? want : 1024);
    TimedScope ts(TK_EDIT_BWD, s);
    hipLaunchKernelGGL(k_compose_bwd, dim3(blocks), dim3(256), 0, s, src, offset, grads, out);
    return hipGetLastError();
}

}  // namespace ivrgs
