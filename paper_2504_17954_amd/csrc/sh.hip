// View-dependent colour from spherical-harmonic coefficients, the colour
// model of base 3DGS (Sec. 3; Sec. 4.2), and its backward.
//
// One thread per Gaussian; the coefficients are planes [K][3][n], so every
// load and store is coalesced across the wave.  The work is a short
// polynomial per Gaussian: both kernels are bound by HBM.
#include "launch.hpp"

namespace ivrgs {

namespace {

// Normalisations of the real basis (Condon-Shortley phase), band by band:
// 1/(2 sqrt(pi)); sqrt(3/(4 pi)); sqrt(15/pi)/2, sqrt(5/pi)/4, sqrt(15/pi)/4;
// sqrt(35/(2 pi))/4, sqrt(105/pi)/2, sqrt(21/(2 pi))/4, sqrt(7/pi)/4,
// sqrt(105/pi)/4.
constexpr float kN0 = 0.28209479177387814f;
constexpr float kN1 = 0.4886025119029199f;
constexpr float kN2a = 1.0925484305920792f, kN2b = 0.31539156525252005f, kN2c = 0.5462742152960396f;
constexpr float kN3e = 0.5900435899266435f, kN3f = 2.890611442640554f, kN3g = 0.4570457994644658f,
                kN3h = 0.3731763325901154f, kN3j = 1.445305721320277f;

template <int L>
constexpr int sh_count() {
    return (L + 1) * (L + 1);
}

// Y[0 .. K) at the unit direction (x, y, z): ordered by band l, then
// m = -l .. l; Y_l^0, sqrt(2) Re Y_l^m (m > 0), sqrt(2) Im Y_l^|m| (m < 0).
template <int L>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *Y) {
    Y[0] = kN0;
    if constexpr (L >= 1) {
        Y[1] = -kN1 * y;
        Y[2] = kN1 * z;
        Y[3] = -kN1 * x;
    }
    if constexpr (L >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = kN2a * x * y;
        Y[5] = -kN2a * y * z;
        Y[6] = kN2b * (2.f * zz - xx - yy);
        Y[7] = -kN2a * x * z;
        Y[8] = kN2c * (xx - yy);
    }
    if constexpr (L >= 3) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[9] = -kN3e * y * (3.f * xx - yy);
        Y[10] = kN3f * x * y * z;
        Y[11] = -kN3g * y * (4.f * zz - xx - yy);
        Y[12] = kN3h * z * (2.f * zz - 3.f * xx - 3.f * yy);
        Y[13] = -kN3g * x * (4.f * zz - xx - yy);
        Y[14] = kN3j * z * (xx - yy);
        Y[15] = -kN3e * x * (xx - 3.f * yy);
    }
}

// Gradient of sum_k w_k Y_k with respect to (x, y, z) taken as independent
// variables (the caller projects it onto the sphere).
template <int L>
__device__ __forceinline__ float3 sh_basis_grad(float x, float y, float z, const float *w) {
    float gx = 0.f, gy = 0.f, gz = 0.f;
    if constexpr (L >= 1) {
        gx -= kN1 * w[3];
        gy -= kN1 * w[1];
        gz += kN1 * w[2];
    }
    if constexpr (L >= 2) {
        gx += kN2a * y * w[4] - 2.f * kN2b * x * w[6] - kN2a * z * w[7] + 2.f * kN2c * x * w[8];
        gy += kN2a * x * w[4] - kN2a * z * w[5] - 2.f * kN2b * y * w[6] - 2.f * kN2c * y * w[8];
        gz += -kN2a * y * w[5] + 4.f * kN2b * z * w[6] - kN2a * x * w[7];
    }
    if constexpr (L >= 3) {
        const float xx = x * x, yy = y * y, zz = z * z;
        const float E = -kN3e, F = kN3f, G = -kN3g, H = kN3h, J = kN3j;  // signed band-3 factors
        // Y9 = E y(3xx - yy)
        gx += 6.f * E * x * y * w[9];
        gy += E * (3.f * xx - 3.f * yy) * w[9];
        // Y10 = F xyz
        gx += F * y * z * w[10];
        gy += F * x * z * w[10];
        gz += F * x * y * w[10];
        // Y11 = G y(4zz - xx - yy)
        gx += -2.f * G * x * y * w[11];
        gy += G * (4.f * zz - xx - 3.f * yy) * w[11];
        gz += 8.f * G * y * z * w[11];
        // Y12 = H z(2zz - 3xx - 3yy)
        gx += -6.f * H * x * z * w[12];
        gy += -6.f * H * y * z * w[12];
        gz += H * (6.f * zz - 3.f * xx - 3.f * yy) * w[12];
        // Y13 = G x(4zz - xx - yy)
        gx += G * (4.f * zz - 3.f * xx - yy) * w[13];
        gy += -2.f * G * x * y * w[13];
        gz += 8.f * G * x * z * w[13];
        // Y14 = J z(xx - yy)
        gx += 2.f * J * x * z * w[14];
        gy += -2.f * J * y * z * w[14];
        gz += J * (xx - yy) * w[14];
        // Y15 = E x(xx - 3yy)
        gx += E * (3.f * xx - 3.f * yy) * w[15];
        gy += -6.f * E * x * y * w[15];
    }
    return make_float3(gx, gy, gz);
}

// Unit direction from the camera centre to the mean, and 1/|mean - C|
// (both zero when the mean sits on the centre).
struct Dir {
    float x, y, z, inv_r;
};

__device__ __forceinline__ Dir direction(const float *__restrict__ mean, int64_t n, int64_t i, float3 C) {
    const float vx = mean[i] - C.x, vy = mean[n + i] - C.y, vz = mean[2 * n + i] - C.z;
    const float r2 = vx * vx + vy * vy + vz * vz;
    const float inv = r2 > 0.f ? 1.f / sqrtf(r2) : 0.f;
    return {vx * inv, vy * inv, vz * inv, inv};
}

template <int L>
__global__ __launch_bounds__(256) void k_sh_color(const float *__restrict__ sh, const float *__restrict__ mean,
                                                  int64_t n, float3 C, float *__restrict__ color) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int K = sh_count<L>();
    const Dir d = direction(mean, n, i, C);
    float Y[K];
    sh_basis<L>(d.x, d.y, d.z, Y);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < K; ++k) acc += Y[k] * sh[(int64_t)(3 * k + c) * n + i];
        const float raw = acc + 0.5f;
        color[c * n + i] = raw < 0.f ? 0.f : raw;  // a NaN passes through
    }
}

// dL/dsh = Y_k g_c with g_c = dL/dcolour_c where the colour is not clamped;
// dL/dmean (added into grad_mean when given) = the tangential part of
// d(sum_k w_k Y_k)/dd over |mean - C|, w_k = sum_c g_c sh_kc.
template <int L>
__global__ __launch_bounds__(256) void k_sh_color_bwd(const float *__restrict__ sh, const float *__restrict__ mean,
                                                      int64_t n, float3 C, const float *__restrict__ grad_color,
                                                      float *__restrict__ grad_sh, float *__restrict__ grad_mean) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int K = sh_count<L>();
    const Dir d = direction(mean, n, i, C);
    float Y[K];
    sh_basis<L>(d.x, d.y, d.z, Y);
    float f[K][3], g[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            f[k][c] = sh[(int64_t)(3 * k + c) * n + i];
            acc += Y[k] * f[k][c];
        }
        g[c] = acc + 0.5f > 0.f ? grad_color[c * n + i] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) grad_sh[(int64_t)(3 * k + c) * n + i] = Y[k] * g[c];
    if constexpr (L >= 1) {
        if (grad_mean && d.inv_r > 0.f) {
            float w[K];
#pragma unroll
            for (int k = 0; k < K; ++k) w[k] = g[0] * f[k][0] + g[1] * f[k][1] + g[2] * f[k][2];
            const float3 gd = sh_basis_grad<L>(d.x, d.y, d.z, w);
            const float dot = d.x * gd.x + d.y * gd.y + d.z * gd.z;
            grad_mean[i] += (gd.x - d.x * dot) * d.inv_r;
            grad_mean[n + i] += (gd.y - d.y * dot) * d.inv_r;
            grad_mean[2 * n + i] += (gd.z - d.z * dot) * d.inv_r;
        }
    }
}

float3 camera_centre(const ivrgs_camera &c) {
    // x_cam = R x + t, so the centre is -R^T t
    double C[3];
    for (int a = 0; a < 3; ++a)
        C[a] = -((double)c.R[0 * 3 + a] * c.t[0] + (double)c.R[1 * 3 + a] * c.t[1] + (double)c.R[2 * 3 + a] * c.t[2]);
    return make_float3((float)C[0], (float)C[1], (float)C[2]);
}

template <int L>
void launch_fwd(const float *sh, const float *mean, int64_t n, float3 C, float *color, hipStream_t s) {
    hipLaunchKernelGGL(k_sh_color<L>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, sh, mean, n, C, color);
}

template <int L>
void launch_bwd(const float *sh, const float *mean, int64_t n, float3 C, const float *gc, float *gs, float *gm,
                hipStream_t s) {
    hipLaunchKernelGGL(k_sh_color_bwd<L>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, sh, mean, n, C, gc, gs,
                       gm);
}

}  // namespace

hipError_t launch_sh_color(const float *sh, int degree, const float *mean, int64_t n, const ivrgs_camera &cam,
                           float *color, hipStream_t s) {
    if (n == 0) return hipSuccess;
    TimedScope ts(TK_SH, s);
    const float3 C = camera_centre(cam);
    switch (degree) {
    case 0: launch_fwd<0>(sh, mean, n, C, color, s); break;
    case 1: launch_fwd<1>(sh, mean, n, C, color, s); break;
    case 2: launch_fwd<2>(sh, mean, n, C, color, s); break;
    default: launch_fwd<3>(sh, mean, n, C, color, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_sh_color_bwd(const float *sh, int degree, const float *mean, int64_t n, const ivrgs_camera &cam,
                               const float *grad_color, float *grad_sh, float *grad_mean, hipStream_t s) {
    if (n == 0) return hipSuccess;
    TimedScope ts(TK_SH, s);
    const float3 C = camera_centre(cam);
    switch (degree) {
    case 0: launch_bwd<0>(sh, mean, n, C, grad_color, grad_sh, grad_mean, s); break;
    case 1: launch_bwd<1>(sh, mean, n, C, grad_color, grad_sh, grad_mean, s); break;
    case 2: launch_bwd<2>(sh, mean, n, C, grad_color, grad_sh, grad_mean, s); break;
    default: launch_bwd<3>(sh, mean, n, C, grad_color, grad_sh, grad_mean, s); break;
    }
    return hipGetLastError();
}

}  // namespace ivrgs
