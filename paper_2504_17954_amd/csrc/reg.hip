// Training regularisers of the editable Gaussians on the rendered maps of
// one view, and their gradients:
//   - normal consistency (Eq. 6): the mean over valid pixels of
//     || N / |N| - N~ ||, N the composited normal map (Eq. 5) and N~ the
//     pseudo-normal of the rendered depth under local planarity (held fixed);
//   - sparsity of the offset-colour map (Sec. 4.3): mean |delta-c|;
//   - bilateral smoothness of the shading-term maps (Eq. 7): mean of
//     |grad K| exp(-|grad c_gt|), x and y forward differences averaged over
//     their own entries and summed;
//   - opacity L1 (Sec. 4.3): mean |o| over the Gaussians.
//
// The pseudo-normal back-projects the pixel centres, P = d r with d =
// depth / alpha and r = ((x + 1/2 - cx) / fx, (y + 1/2 - cy) / fy, 1), and
// crosses the central differences.  A central difference is written as
// P[x+1] - P[x-1] = (d[x+1] - d[x-1]) r[x+1] + d[x-1] (2 / fx, 0, 0) (the
// rays differ by exactly that), and d[x+1] - d[x-1] as one quotient whose
// numerator is a 2x2 determinant in Kahan's form, so in FP32 the difference
// is accurate relative to itself: on a flat, fronto-parallel patch it does
// not lose the factor f (the focal length in pixels) that subtracting two
// rounded depths would.
//
// The forward is one pass over pixels (and Gaussians, in the trailing
// workgroups) writing one row of partial sums per workgroup, and one
// workgroup that adds the rows in a fixed order in FP64, so the result does
// not depend on scheduling.  The backward is one elementwise pass.  Bound:
// HBM (about 60 bytes of maps read per pixel; a few flops each).
#include <cmath>

#include "launch.hpp"

namespace ivrgs {

namespace {

constexpr int kRegBlock = 256;
constexpr float kNormFloor = 1e-12f;
constexpr float kAlphaValid = 0.5f;

struct RegView {
    const float *depth, *alpha, *normal, *delta_c, *shade, *target, *opacity;
    int64_t n_gauss;
    int H, W;
    float fx, fy, cx, cy;
    float R[9];
};

__device__ __forceinline__ bool opaque(const RegView &v, int x, int y) {
    return v.alpha[(int64_t)y * v.W + x] > kAlphaValid;
}

__device__ __forceinline__ bool valid_px(const RegView &v, int x, int y) {
    if (x < 1 || y < 1 || x >= v.W - 1 || y >= v.H - 1) return false;
    return opaque(v, x, y) && opaque(v, x - 1, y) && opaque(v, x + 1, y) && opaque(v, x, y - 1) &&
           opaque(v, x, y + 1);
}

// d[b] - d[a] for d = depth / alpha, as (dep_b al_a - dep_a al_b) / (al_a al_b)
// with the numerator in Kahan's form (fused products).
__device__ __forceinline__ float depth_diff(float dep_a, float al_a, float dep_b, float al_b) {
    const float w = dep_a * al_b;
    const float e = fmaf(-dep_a, al_b, w);
    const float f = fmaf(dep_b, al_a, -w);
    return (f + e) / (al_a * al_b);
}

// The world-space pseudo-normal at a valid pixel.
__device__ __forceinline__ void pseudo_normal_at(const RegView &v, int x, int y, float n[3]) {
    const int64_t p = (int64_t)y * v.W + x;
    const float *dp = v.depth, *al = v.alpha;
    const float rx0 = ((float)x + 0.5f - v.cx) / v.fx, ry0 = ((float)y + 0.5f - v.cy) / v.fy;
    const float rx1 = ((float)x + 1.5f - v.cx) / v.fx, ry1 = ((float)y + 1.5f - v.cy) / v.fy;
    // along x: (d_r - d_l) r(x+1, y) + d_l (2 / fx, 0, 0)
    const float dx = depth_diff(dp[p - 1], al[p - 1], dp[p + 1], al[p + 1]);
    const float dl = dp[p - 1] / al[p - 1];
    const float tx0 = fmaf(dx, rx1, 2.f * dl / v.fx), tx1 = dx * ry0, tx2 = dx;
    // along y: (d_d - d_u) r(x, y+1) + d_u (0, 2 / fy, 0)
    const float dy = depth_diff(dp[p - v.W], al[p - v.W], dp[p + v.W], al[p + v.W]);
    const float du = dp[p - v.W] / al[p - v.W];
    const float ty0 = dy * rx0, ty1 = fmaf(dy, ry1, 2.f * du / v.fy), ty2 = dy;
    float c0 = tx1 * ty2 - tx2 * ty1;
    float c1 = tx2 * ty0 - tx0 * ty2;
    float c2 = tx0 * ty1 - tx1 * ty0;
    const float len = sqrtf(c0 * c0 + c1 * c1 + c2 * c2);
    const float inv = len > 0.f ? 1.f / len : 0.f;
    c0 *= inv;
    c1 *= inv;
    c2 *= inv;
    // face the camera: N~ . P <= 0 with P = d r at the pixel
    const float d = dp[p] / al[p];
    if ((c0 * rx0 + c1 * ry0 + c2) * d > 0.f) {
        c0 = -c0;
        c1 = -c1;
        c2 = -c2;
    }
    // camera to world: R^T n
#pragma unroll
    for (int i = 0; i < 3; ++i) n[i] = v.R[i] * c0 + v.R[3 + i] * c1 + v.R[6 + i] * c2;
}

__device__ __forceinline__ float sgn(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

// exp(-mean_c |c_gt(b) - c_gt(a)|), the weight of one difference of Eq. 7
__device__ __forceinline__ float edge_weight(const RegView &v, int64_t a, int64_t b, int64_t plane) {
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) s += fabsf(v.target[c * plane + b] - v.target[c * plane + a]);
    return expf(-s / 3.f);
}

// wave sum to every lane (xor butterfly)
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Partial sums per workgroup: [0] normal consistency, [1] valid pixels,
// [2] |delta-c|, [3] x smoothness, [4] y smoothness, [5] |opacity|.
constexpr int kRegSums = 6;

__global__ __launch_bounds__(kRegBlock) void k_reg_fwd(RegView v, int64_t pix_blocks, float *__restrict__ partial,
                                                       float *__restrict__ pseudo) {
    float s[kRegSums] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int64_t plane = (int64_t)v.H * v.W;
    if ((int64_t)blockIdx.x < pix_blocks) {
        const int64_t p = (int64_t)blockIdx.x * kRegBlock + threadIdx.x;
        if (p < plane) {
            const int y = (int)(p / v.W), x = (int)(p - (int64_t)y * v.W);
            if (v.normal || pseudo) {
                float pn[3] = {0.f, 0.f, 0.f};
                const bool ok = valid_px(v, x, y);
                if (ok) pseudo_normal_at(v, x, y, pn);
                if (pseudo)
                    for (int c = 0; c < 3; ++c) pseudo[c * plane + p] = pn[c];
                if (ok && v.normal) {
                    const float N0 = v.normal[p], N1 = v.normal[plane + p], N2 = v.normal[2 * plane + p];
                    const float nn = fmaxf(sqrtf(N0 * N0 + N1 * N1 + N2 * N2), kNormFloor);
                    const float e0 = N0 / nn - pn[0], e1 = N1 / nn - pn[1], e2 = N2 / nn - pn[2];
                    s[0] = sqrtf(e0 * e0 + e1 * e1 + e2 * e2);
                    s[1] = 1.f;
                }
            }
            if (v.delta_c)
                for (int c = 0; c < 3; ++c) s[2] += fabsf(v.delta_c[c * plane + p]);
            if (v.shade) {
                if (x + 1 < v.W) {
                    const float w = edge_weight(v, p, p + 1, plane);
                    float a = 0.f;
                    for (int c = 0; c < 4; ++c) a += fabsf(v.shade[c * plane + p + 1] - v.shade[c * plane + p]);
                    s[3] = a * w;
                }
                if (y + 1 < v.H) {
                    const float w = edge_weight(v, p, p + v.W, plane);
                    float a = 0.f;
                    for (int c = 0; c < 4; ++c) a += fabsf(v.shade[c * plane + p + v.W] - v.shade[c * plane + p]);
                    s[4] = a * w;
                }
            }
        }
    } else {
        const int64_t i = ((int64_t)blockIdx.x - pix_blocks) * kRegBlock + threadIdx.x;
        if (i < v.n_gauss) s[5] = fabsf(v.opacity[i]);
    }
    __shared__ float red[kRegSums][kRegBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kRegSums; ++k) {
        const float t = wave_sum(s[k]);
        if (lane == 0) red[k][wave] = t;
    }
    __syncthreads();
    if (threadIdx.x < kRegSums) {
        const int k = threadIdx.x;
        partial[(int64_t)blockIdx.x * kRegSums + k] = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
    }
}

// One workgroup: the rows of partial sums added in a fixed order in FP64,
// then the four terms and the valid pixel count.
__global__ __launch_bounds__(kRegBlock) void k_reg_reduce(const float *__restrict__ partial, int64_t blocks,
                                                          int H, int W, int64_t n_gauss, int has_normal,
                                                          int has_dc, int has_shade, float *__restrict__ terms) {
    __shared__ double red[kRegSums][kRegBlock];
    double s[kRegSums] = {0, 0, 0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < blocks; b += kRegBlock)
        for (int k = 0; k < kRegSums; ++k) s[k] += (double)partial[b * kRegSums + k];
    for (int k = 0; k < kRegSums; ++k) red[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int w = kRegBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < kRegSums; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double cnt = red[1][0];
        terms[0] = has_normal && cnt > 0 ? (float)(red[0][0] / cnt) : 0.f;
        terms[1] = has_dc ? (float)(red[2][0] / (3.0 * H * W)) : 0.f;
        terms[2] = has_shade ? (float)(red[3][0] / (4.0 * H * (W - 1)) + red[4][0] / (4.0 * (H - 1) * W)) : 0.f;
        terms[3] = n_gauss > 0 ? (float)(red[5][0] / (double)n_gauss) : 0.f;
        terms[4] = (float)cnt;
    }
}

// Gradients of sum_k g[k] term_k (g = grad_terms, device) with respect to the
// normal, offset-colour and shading maps and the opacities; the valid pixel
// count is the forward's terms[4].  Outputs are overwritten; g_depth (the
// depth map gets no gradient) with zeros.
__global__ __launch_bounds__(kRegBlock) void k_reg_bwd(RegView v, int64_t pix_blocks, const float *__restrict__ terms,
                                                       const float *__restrict__ gterm, float *__restrict__ g_normal,
                                                       float *__restrict__ g_dc, float *__restrict__ g_shade,
                                                       float *__restrict__ g_op, float *__restrict__ g_depth) {
    const int64_t plane = (int64_t)v.H * v.W;
    if ((int64_t)blockIdx.x >= pix_blocks) {
        const int64_t i = ((int64_t)blockIdx.x - pix_blocks) * kRegBlock + threadIdx.x;
        if (i < v.n_gauss && g_op) g_op[i] = gterm[3] * sgn(v.opacity[i]) / (float)v.n_gauss;
        return;
    }
    const int64_t p = (int64_t)blockIdx.x * kRegBlock + threadIdx.x;
    if (p >= plane) return;
    const int y = (int)(p / v.W), x = (int)(p - (int64_t)y * v.W);
    if (g_depth) g_depth[p] = 0.f;
    if (g_normal) {
        float g[3] = {0.f, 0.f, 0.f};
        const float cnt = terms[4];
        if (cnt > 0.f && valid_px(v, x, y)) {
            float pn[3];
            pseudo_normal_at(v, x, y, pn);
            const float N0 = v.normal[p], N1 = v.normal[plane + p], N2 = v.normal[2 * plane + p];
            const float len = sqrtf(N0 * N0 + N1 * N1 + N2 * N2);
            const float nn = fmaxf(len, kNormFloor);
            const float m0 = N0 / nn, m1 = N1 / nn, m2 = N2 / nn;
            const float e0 = m0 - pn[0], e1 = m1 - pn[1], e2 = m2 - pn[2];
            const float L = sqrtf(e0 * e0 + e1 * e1 + e2 * e2);
            if (L > 0.f) {
                const float sc = gterm[0] / cnt / (L * nn);
                if (len >= kNormFloor) {
                    // (m (m . N~) - N~) / (L |N|): the tangential part of m - N~
                    const float mp = m0 * pn[0] + m1 * pn[1] + m2 * pn[2];
                    g[0] = sc * (m0 * mp - pn[0]);
                    g[1] = sc * (m1 * mp - pn[1]);
                    g[2] = sc * (m2 * mp - pn[2]);
                } else {  // below the floor the normalisation is a constant scale
                    g[0] = sc * e0;
                    g[1] = sc * e1;
                    g[2] = sc * e2;
                }
            }
        }
        for (int c = 0; c < 3; ++c) g_normal[c * plane + p] = g[c];
    }
    if (g_dc) {
        const float sc = gterm[1] / (3.f * (float)plane);
        for (int c = 0; c < 3; ++c) g_dc[c * plane + p] = sc * sgn(v.delta_c[c * plane + p]);
    }
    if (g_shade) {
        const float sx = gterm[2] / (4.f * (float)v.H * (float)(v.W - 1));
        const float sy = gterm[2] / (4.f * (float)(v.H - 1) * (float)v.W);
        const float wl = x > 0 ? edge_weight(v, p - 1, p, plane) : 0.f;
        const float wr = x + 1 < v.W ? edge_weight(v, p, p + 1, plane) : 0.f;
        const float wu = y > 0 ? edge_weight(v, p - v.W, p, plane) : 0.f;
        const float wd = y + 1 < v.H ? edge_weight(v, p, p + v.W, plane) : 0.f;
        for (int c = 0; c < 4; ++c) {
            const float *k = v.shade + c * plane;
            const float kc = k[p];
            float gx = 0.f, gy = 0.f;
            if (x > 0) gx += sgn(kc - k[p - 1]) * wl;
            if (x + 1 < v.W) gx -= sgn(k[p + 1] - kc) * wr;
            if (y > 0) gy += sgn(kc - k[p - v.W]) * wu;
            if (y + 1 < v.H) gy -= sgn(k[p + v.W] - kc) * wd;
            g_shade[c * plane + p] = sx * gx + sy * gy;
        }
    }
}

RegView make_view(const ivrgs_reg_maps &m, const ivrgs_camera &cam) {
    RegView v;
    v.depth = m.depth;
    v.alpha = m.alpha;
    v.normal = m.normal;
    v.delta_c = m.delta_c;
    v.shade = m.shade;
    v.target = m.target;
    v.opacity = m.opacity;
    v.n_gauss = m.opacity ? m.n_gauss : 0;
    v.H = m.height;
    v.W = m.width;
    v.fx = cam.fx;
    v.fy = cam.fy;
    v.cx = cam.cx;
    v.cy = cam.cy;
    for (int i = 0; i < 9; ++i) v.R[i] = cam.R[i];
    return v;
}

int64_t pixel_blocks(const ivrgs_reg_maps &m) {
    return ((int64_t)m.height * m.width + kRegBlock - 1) / kRegBlock;
}

int64_t gauss_blocks(const ivrgs_reg_maps &m) {
    return m.opacity ? (m.n_gauss + kRegBlock - 1) / kRegBlock : 0;
}

}  // namespace

size_t reg_workspace_bytes(const ivrgs_reg_maps &m) {
    return sizeof(float) * kRegSums * (size_t)(pixel_blocks(m) + gauss_blocks(m));
}

hipError_t launch_reg_fwd(const ivrgs_reg_maps &m, const ivrgs_camera &cam, float *terms, float *pseudo, void *ws,
                          hipStream_t s) {
    const RegView v = make_view(m, cam);
    const int64_t pb = pixel_blocks(m), blocks = pb + gauss_blocks(m);
    float *partial = static_cast<float *>(ws);
    hipLaunchKernelGGL(k_reg_fwd, dim3((unsigned)blocks), dim3(kRegBlock), 0, s, v, pb, partial, pseudo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reg_reduce, dim3(1), dim3(kRegBlock), 0, s, partial, blocks, m.height, m.width, v.n_gauss,
                       m.normal ? 1 : 0, m.delta_c ? 1 : 0, m.shade ? 1 : 0, terms);
    return hipGetLastError();
}

hipError_t launch_reg_bwd(const ivrgs_reg_maps &m, const ivrgs_camera &cam, const float *terms, const float *gterm,
                          float *g_normal, float *g_dc, float *g_shade, float *g_op, float *g_depth, hipStream_t s) {
    const RegView v = make_view(m, cam);
    const int64_t pb = pixel_blocks(m), blocks = pb + gauss_blocks(m);
    hipLaunchKernelGGL(k_reg_bwd, dim3((unsigned)blocks), dim3(kRegBlock), 0, s, v, pb, terms, gterm, g_normal,
                       g_dc, g_shade, g_op, g_depth);
    return hipGetLastError();
}

}  // namespace ivrgs
