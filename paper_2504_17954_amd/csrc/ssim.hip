// Structural similarity of a rendered image against its target, the second
// term of the photometric loss (Sec. 4.2; weights in the appendix), and its
// gradient with respect to the rendered image.
//
// Per channel, every valid 11x11 window p (top-left corner, Ho x Wo of them)
// carries Gaussian-weighted moments mx, my, Exx, Eyy, Exy (weights
// g[i] g[j], sigma 1.5, normalised).  With sxx = Exx - mx^2 and likewise
//   S(p) = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sxx + syy + C2)),
// and the loss term is the mean of S over windows and channels.  Writing
// N1, N2, D1, D2 for the four factors, the partial derivatives of S(p) are
//   dS/dmx  = (2 my (N2 - N1)) / (D1 D2) + 2 mx S (1/D2 - 1/D1)   (= A),
//   dS/dExx = -S / D2                                              (= B),
//   dS/dExy = 2 N1 / (D1 D2)                                       (= C),
// so the gradient at pixel q is the transposed window sum
//   dmean/dx_q = (sum_p w(q - p) [A(p) + 2 x_q B(p) + y_q C(p)]) / (channels Ho Wo).
// No factor divides by N1 or N2, which may vanish.
//
// Both kernels are separable stencils over 16x16 output tiles: the 26x26
// input region (the tile plus the window's 10-pixel halo) is staged in LDS,
// a horizontal 11-tap pass writes 26 x 16 row sums to LDS, and each thread
// finishes one output with the vertical pass.  The forward keeps A, B, C per
// window in the workspace for the backward and one partial sum of S per
// workgroup; a single workgroup adds the partials in a fixed order (FP64),
// so the result does not depend on scheduling.  Bound: HBM (the image and
// target read once, 12 B per window written, read back once).
#include <algorithm>
#include <cmath>

#include "launch.hpp"

namespace ivrgs {

namespace {

constexpr int kSsimTile = 16;
constexpr int kWin = kSsimWindow;          // 11
constexpr int kReg = kSsimTile + kWin - 1;     // 26: tile plus halo
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

__global__ __launch_bounds__(256) void k_ssim_fwd(const float *__restrict__ x, const float *__restrict__ y, int H,
                                                  int W, SsimTaps taps, float *__restrict__ abc,
                                                  float *__restrict__ partial, float *__restrict__ partial_l1) {
    __shared__ float sx[kReg][kReg + 1], sy[kReg][kReg + 1];
    __shared__ float hs[5][kReg][kSsimTile];
    __shared__ float wsum[4], wl1[4];
    const int Ho = H - kWin + 1, Wo = W - kWin + 1;
    const int ox0 = blockIdx.x * kSsimTile, oy0 = blockIdx.y * kSsimTile, c = blockIdx.z;
    const int64_t plane = (int64_t)H * W;
    const float *xc = x + c * plane, *yc = y + c * plane;
    const int t = threadIdx.x;
    for (int i = t; i < kReg * kReg; i += 256) {
        const int r = i / kReg, q = i - r * kReg;
        const int gy = oy0 + r, gx = ox0 + q;
        const bool ok = gy < H && gx < W;
        sx[r][q] = ok ? xc[(int64_t)gy * W + gx] : 0.0f;
        sy[r][q] = ok ? yc[(int64_t)gy * W + gx] : 0.0f;
    }
    __syncthreads();
    for (int i = t; i < kReg * kSsimTile; i += 256) {
        const int r = i / kSsimTile, q = i - r * kSsimTile;
        float a = 0, b = 0, aa = 0, bb = 0, ab = 0;
#pragma unroll
        for (int k = 0; k < kWin; ++k) {
            const float u = sx[r][q + k], v = sy[r][q + k], g = taps.w[k];
            a = fmaf(g, u, a);
            b = fmaf(g, v, b);
            aa = fmaf(g, u * u, aa);
            bb = fmaf(g, v * v, bb);
            ab = fmaf(g, u * v, ab);
        }
        hs[0][r][q] = a;
        hs[1][r][q] = b;
        hs[2][r][q] = aa;
        hs[3][r][q] = bb;
        hs[4][r][q] = ab;
    }
    __syncthreads();
    const int ty = t / kSsimTile, tx = t - ty * kSsimTile;
    const int oy = oy0 + ty, ox = ox0 + tx;
    float m[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kWin; ++k) {
        const float g = taps.w[k];
#pragma unroll
        for (int s = 0; s < 5; ++s) m[s] = fmaf(g, hs[s][ty + k][tx], m[s]);
    }
    float S = 0.0f;
    if (oy < Ho && ox < Wo) {
        const float mx = m[0], my = m[1];
        const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
        const float N1 = 2.0f * mx * my + kC1, N2 = 2.0f * sxy + kC2;
        const float D1 = mx * mx + my * my + kC1, D2 = sxx + syy + kC2;
        const float D = D1 * D2;
        S = N1 * N2 / D;
        const float A = 2.0f * my * (N2 - N1) / D + 2.0f * mx * S * (1.0f / D2 - 1.0f / D1);
        const float B = -S / D2;
        const float C = 2.0f * N1 / D;
        const int64_t wp = (int64_t)Ho * Wo, at = (int64_t)oy * Wo + ox;
        float *o = abc + (int64_t)c * 3 * wp;
        o[at] = A;
        o[wp + at] = B;
        o[2 * wp + at] = C;
    }
    // the L1 term over the pixels this workgroup owns: its 16x16 tile, and
    // for the last tile of a row or column also the pixels past it (at most
    // 26 in all, inside the staged region)
    float l1 = 0.0f;
    if (partial_l1) {
        const int nx = (blockIdx.x + 1 == gridDim.x) ? W - ox0 : kSsimTile;
        const int ny = (blockIdx.y + 1 == gridDim.y) ? H - oy0 : kSsimTile;
        for (int i = t; i < nx * ny; i += 256) {
            const int r = i / nx, q = i - r * nx;
            l1 += fabsf(sx[r][q] - sy[r][q]);
        }
    }
    // workgroup sums of S and of |x - y|, lanes then waves in a fixed order
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        S += __shfl_xor(S, d, 64);
        l1 += __shfl_xor(l1, d, 64);
    }
    if ((t & 63) == 0) {
        wsum[t >> 6] = S;
        wl1[t >> 6] = l1;
    }
    __syncthreads();
    if (t == 0) {
        const int64_t b = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        partial[b] = ((wsum[0] + wsum[1]) + (wsum[2] + wsum[3]));
        if (partial_l1) partial_l1[b] = ((wl1[0] + wl1[1]) + (wl1[2] + wl1[3]));
    }
}

// One workgroup: the partials in a fixed order (FP64), divided by the
// number of windows; with partial_l1, also the L1 partials divided by the
// number of values, into out[1].
__global__ __launch_bounds__(256) void k_ssim_reduce(const float *__restrict__ partial,
                                                     const float *__restrict__ partial_l1, int64_t n, double inv,
                                                     double inv_n, float *__restrict__ out) {
    __shared__ double red[256], red1[256];
    double s = 0.0, s1 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        s += (double)partial[i];
        if (partial_l1) s1 += (double)partial_l1[i];
    }
    red[threadIdx.x] = s;
    red1[threadIdx.x] = s1;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[threadIdx.x] += red[threadIdx.x + w];
            red1[threadIdx.x] += red1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (float)(red[0] * inv);
        if (partial_l1) out[1] = (float)(red1[0] * inv_n);
    }
}

// Pixel tile [qy0, qy0 + 16) x [qx0, qx0 + 16): the windows that cover it
// have corners in [q0 - 10, q0 + 15]; corners outside [0, Ho) x [0, Wo)
// contribute zero.  The taps are symmetric (g[k] = g[10 - k]), so the
// transposed sum over corners p = q - k with weight g[k] is the same
// forward 11-tap sum over the staged region.
__global__ __launch_bounds__(256) void k_ssim_bwd(const float *__restrict__ x, const float *__restrict__ y, int H,
                                                  int W, SsimTaps taps, const float *__restrict__ abc,
                                                  const float *__restrict__ grad_mean, double inv,
                                                  float ssim_w, float l1_w, const float *__restrict__ dev_w,
                                                  double inv_n, float *__restrict__ grad_x) {
    __shared__ float sa[3][kReg][kReg + 1];
    __shared__ float hs[3][kReg][kSsimTile];
    const int Ho = H - kWin + 1, Wo = W - kWin + 1;
    const int qx0 = blockIdx.x * kSsimTile, qy0 = blockIdx.y * kSsimTile, c = blockIdx.z;
    const int64_t wp = (int64_t)Ho * Wo;
    const float *ac = abc + (int64_t)c * 3 * wp;
    const int t = threadIdx.x;
    for (int i = t; i < kReg * kReg; i += 256) {
        const int r = i / kReg, q = i - r * kReg;
        const int py = qy0 - (kWin - 1) + r, px = qx0 - (kWin - 1) + q;
        const bool ok = py >= 0 && py < Ho && px >= 0 && px < Wo;
        const int64_t at = (int64_t)py * Wo + px;
        sa[0][r][q] = ok ? ac[at] : 0.0f;
        sa[1][r][q] = ok ? ac[wp + at] : 0.0f;
        sa[2][r][q] = ok ? ac[2 * wp + at] : 0.0f;
    }
    __syncthreads();
    for (int i = t; i < kReg * kSsimTile; i += 256) {
        const int r = i / kSsimTile, q = i - r * kSsimTile;
        float s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int k = 0; k < kWin; ++k) {
            const float g = taps.w[k];
            s0 = fmaf(g, sa[0][r][q + k], s0);
            s1 = fmaf(g, sa[1][r][q + k], s1);
            s2 = fmaf(g, sa[2][r][q + k], s2);
        }
        hs[0][r][q] = s0;
        hs[1][r][q] = s1;
        hs[2][r][q] = s2;
    }
    __syncthreads();
    const int ty = t / kSsimTile, tx = t - ty * kSsimTile;
    const int qy = qy0 + ty, qx = qx0 + tx;
    if (qy >= H || qx >= W) return;
    float bA = 0, bB = 0, bC = 0;
#pragma unroll
    for (int k = 0; k < kWin; ++k) {
        const float g = taps.w[k];
        bA = fmaf(g, hs[0][ty + k][tx], bA);
        bB = fmaf(g, hs[1][ty + k][tx], bB);
        bC = fmaf(g, hs[2][ty + k][tx], bC);
    }
    const int64_t at = (int64_t)c * H * W + (int64_t)qy * W + qx;
    const float xq = x[at], yq = y[at];
    // dL/d(mean SSIM) from the device (ivrgs_ssim_bwd; dev_w[0] of
    // ivrgs_photometric_grad_dev) or the host weight; the L1 weight per value
    // from the host or dev_w[1]
    const float scale =
        (float)((grad_mean ? (double)grad_mean[0] : (dev_w ? (double)dev_w[0] : (double)ssim_w)) * inv);
    if (dev_w) l1_w = (float)((double)dev_w[1] * inv_n);
    float gq = scale * (bA + 2.0f * xq * bB + yq * bC);
    // the L1 term: l1_w sign(x - y), with sign(0) = 0
    if (l1_w != 0.0f) gq = fmaf(l1_w, (float)((xq > yq) - (xq < yq)), gq);
    grad_x[at] = gq;
}

}  // namespace

SsimTaps ssim_taps() {
    // g[k] = exp(-(k - 5)^2 / (2 * 1.5^2)), normalised in FP64, then rounded
    SsimTaps t;
    double g[kWin], s = 0.0;
    for (int k = 0; k < kWin; ++k) {
        const double d = k - (kWin - 1) / 2;
        g[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
        s += g[k];
    }
    for (int k = 0; k < kWin; ++k) t.w[k] = (float)(g[k] / s);
    return t;
}

size_t ssim_workspace_floats(int channels, int H, int W) {
    const int64_t Ho = H - kWin + 1, Wo = W - kWin + 1;
    const int64_t blocks = (int64_t)channels * ((Ho + kSsimTile - 1) / kSsimTile) * ((Wo + kSsimTile - 1) / kSsimTile);
    return (size_t)(3 * channels * Ho * Wo + blocks);
}

hipError_t launch_ssim_fwd(const float *x, const float *y, int channels, int H, int W, float *out, float *ws,
                           hipStream_t s) {
    const int Ho = H - kWin + 1, Wo = W - kWin + 1;
    const dim3 grid((Wo + kSsimTile - 1) / kSsimTile, (Ho + kSsimTile - 1) / kSsimTile, channels);
    float *abc = ws, *partial = ws + (size_t)3 * channels * Ho * Wo;
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, s, x, y, H, W, ssim_taps(), abc, partial, nullptr);
    const int64_t n = (int64_t)grid.x * grid.y * grid.z;
    hipLaunchKernelGGL(k_ssim_reduce, dim3(1), dim3(256), 0, s, partial, nullptr, n,
                       1.0 / ((double)channels * Ho * Wo), 0.0, out);
    return hipGetLastError();
}

size_t photometric_workspace_floats(int channels, int H, int W) {
    const int64_t Ho = H - kWin + 1, Wo = W - kWin + 1;
    const int64_t blocks = (int64_t)channels * ((Ho + kSsimTile - 1) / kSsimTile) * ((Wo + kSsimTile - 1) / kSsimTile);
    return ssim_workspace_floats(channels, H, W) + (size_t)blocks;
}

hipError_t launch_photometric_fwd(const float *x, const float *y, int channels, int H, int W, float *out, float *ws,
                                  hipStream_t s) {
    const int Ho = H - kWin + 1, Wo = W - kWin + 1;
    const dim3 grid((Wo + kSsimTile - 1) / kSsimTile, (Ho + kSsimTile - 1) / kSsimTile, channels);
    const int64_t n = (int64_t)grid.x * grid.y * grid.z;
    float *abc = ws, *partial = ws + (size_t)3 * channels * Ho * Wo, *partial_l1 = partial + n;
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, s, x, y, H, W, ssim_taps(), abc, partial, partial_l1);
    hipLaunchKernelGGL(k_ssim_reduce, dim3(1), dim3(256), 0, s, partial, partial_l1, n,
                       1.0 / ((double)channels * Ho * Wo), 1.0 / ((double)channels * H * W), out);
    return hipGetLastError();
}

hipError_t launch_ssim_bwd(const float *x, const float *y, int channels, int H, int W, const float *grad_mean,
                           float *grad_x, const float *ws, hipStream_t s) {
    const int Ho = H - kWin + 1, Wo = W - kWin + 1;
    const dim3 grid((W + kSsimTile - 1) / kSsimTile, (H + kSsimTile - 1) / kSsimTile, channels);
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, s, x, y, H, W, ssim_taps(), ws, grad_mean,
                       1.0 / ((double)channels * Ho * Wo), 0.0f, 0.0f, nullptr, 0.0, grad_x);
    return hipGetLastError();
}

hipError_t launch_photometric_grad_dev(const float *x, const float *y, int channels, int H, int W,
                                       const float *weights, float *grad_x, const float *ws, hipStream_t s) {
    const int Ho = H - kWin + 1, Wo = W - kWin + 1;
    const dim3 grid((W + kSsimTile - 1) / kSsimTile, (H + kSsimTile - 1) / kSsimTile, channels);
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, s, x, y, H, W, ssim_taps(), ws, nullptr,
                       1.0 / ((double)channels * Ho * Wo), 0.0f, 0.0f, weights, 1.0 / ((double)channels * H * W),
                       grad_x);
    return hipGetLastError();
}

hipError_t launch_photometric_grad(const float *x, const float *y, int channels, int H, int W, float lam,
                                   float *grad_x, const float *ws, hipStream_t s) {
    const int Ho = H - kWin + 1, Wo = W - kWin + 1;
    const dim3 grid((W + kSsimTile - 1) / kSsimTile, (H + kSsimTile - 1) / kSsimTile, channels);
    // L = (1 - lam) mean |x - y| + lam (1 - mean SSIM): the SSIM mean enters
    // with weight -lam, each |x - y| with (1 - lam) / (channels H W)
    const float l1_w = (float)((1.0 - (double)lam) / ((double)channels * H * W));
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, s, x, y, H, W, ssim_taps(), ws, nullptr,
                       1.0 / ((double)channels * Ho * Wo), -lam, l1_w, nullptr, 0.0, grad_x);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The L1 term of the photometric loss, mean |x - y| over n values, and its
// gradient sign(x - y) g / n.  Forward: each workgroup sums |x - y| over a
// fixed slice (the FP32 difference, accumulated in FP64) into one partial;
// one workgroup adds the partials in a fixed order, so the result does not
// depend on scheduling.  Both bound by HBM (x and y read once; the backward
// writes the gradient once).
constexpr int kL1MaxBlocks = 1024;
constexpr int64_t kL1Quantum = 4 * 256;  // values per workgroup step (float4 per thread)

int64_t l1_blocks(int64_t n) { return std::min<int64_t>(kL1MaxBlocks, (n + 4095) / 4096); }

namespace {

__device__ __forceinline__ double block_sum_256(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

// Workgroup b sums values [b per, min((b + 1) per, n)); per is a multiple of
// kL1Quantum, so with 16-byte aligned x and y (vec) every float4 of a slice
// is aligned and only the last slice has a scalar tail.
__global__ __launch_bounds__(256) void k_l1_partial(const float *__restrict__ x, const float *__restrict__ y,
                                                    int64_t n, int64_t per, bool vec, double *__restrict__ partial) {
    __shared__ double red[256];
    const int64_t b0 = (int64_t)blockIdx.x * per, b1 = min(b0 + per, n);
    double s = 0.0;
    int64_t tail = b0;
    if (vec) {
        const int64_t v1 = b0 + (b1 - b0) / 4 * 4;
        const float4 *x4 = reinterpret_cast<const float4 *>(x), *y4 = reinterpret_cast<const float4 *>(y);
        for (int64_t i = b0 / 4 + threadIdx.x; i < v1 / 4; i += 256) {
            const float4 a = x4[i], c = y4[i];
            s += (double)fabsf(a.x - c.x) + (double)fabsf(a.y - c.y) + (double)fabsf(a.z - c.z) +
                 (double)fabsf(a.w - c.w);
        }
        tail = v1;
    }
    for (int64_t i = tail + threadIdx.x; i < b1; i += 256) s += (double)fabsf(x[i] - y[i]);
    const double t = block_sum_256(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_l1_final(const double *__restrict__ partial, int64_t m, double inv_n,
                                                  float *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += 256) s += partial[i];
    const double t = block_sum_256(s, red);
    if (threadIdx.x == 0) out[0] = (float)(t * inv_n);
}

// d = x - y: g / n with the sign of d, 0 where d = 0, NaN where d is NaN.
__global__ __launch_bounds__(256) void k_l1_bwd(const float *__restrict__ x, const float *__restrict__ y, int64_t n,
                                                const float *__restrict__ grad_mean, double inv_n,
                                                float *__restrict__ gx) {
    const float g = (float)((double)grad_mean[0] * inv_n);
    auto one = [g](float d) { return d > 0.f ? g : (d < 0.f ? -g : (d == 0.f ? 0.f : d)); };
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) gx[i] = one(x[i] - y[i]);
}

}  // namespace

hipError_t launch_l1_fwd(const float *x, const float *y, int64_t n, float *out, double *partial, hipStream_t s) {
    const int64_t m = l1_blocks(n);
    const int64_t per = ((n + m - 1) / m + kL1Quantum - 1) / kL1Quantum * kL1Quantum;
    const int64_t blocks = (n + per - 1) / per;
    const bool vec = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15u) == 0;
    hipLaunchKernelGGL(k_l1_partial, dim3((unsigned)blocks), dim3(256), 0, s, x, y, n, per, vec, partial);
    hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(256), 0, s, partial, blocks, 1.0 / (double)n, out);
    return hipGetLastError();
}

hipError_t launch_l1_bwd(const float *x, const float *y, int64_t n, const float *grad_mean, float *grad_x,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_l1_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n, grad_mean,
                       1.0 / (double)n, grad_x);
    return hipGetLastError();
}

}  // namespace ivrgs
