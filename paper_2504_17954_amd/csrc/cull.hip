// Learned culling: an MLP (16 -> 64 -> 64 -> 1, ReLU) predicts per
// Gaussian and view whether the Gaussian's largest compositing weight reaches
// 1/255; the kept ids are compacted, in ascending order, into an index list
// and their count is written into the job table on the device, so the
// following projection, binning and rendering run on the survivors with no
// host round trip.
//
// The MLP is a dense contraction, so it runs on the matrix cores: BF16
// operands, FP32 accumulation, v_mfma_f32_16x16x16_bf16.  Hidden units are
// the M dimension and Gaussians the N dimension (16 per MFMA), so the
// accumulator layout of one layer (lane l: column l % 16, rows 4 (l / 16) + i)
// is exactly the B-operand layout the next layer needs (lane l: column
// l % 16, k = 4 (l / 16) + i); activations never leave registers.
#include "launch.hpp"

namespace ivrgs {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kHidden = 64;
constexpr int kFeat = 16;         // 10 features padded with zeros
constexpr int kCullBlock = 256;   // Gaussians per workgroup (4 waves x 4 groups of 16)

// float -> bf16 bits, round to nearest even (inputs are finite here).
__device__ __forceinline__ short to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
    bf16x4 v;
    v[0] = to_bf16(a);
    v[1] = to_bf16(b);
    v[2] = to_bf16(c);
    v[3] = to_bf16(d);
    return v;
}

// Four consecutive BF16 weights in one 8-byte load (the weight arrays are
// 8-byte aligned and every fragment starts at a multiple of 4 elements).
__device__ __forceinline__ bf16x4 load4(const uint16_t *p) {
    const uint2 u = *reinterpret_cast<const uint2 *>(p);
    bf16x4 v;
    v[0] = (short)(u.x & 0xFFFFu);
    v[1] = (short)(u.x >> 16);
    v[2] = (short)(u.y & 0xFFFFu);
    v[3] = (short)(u.y >> 16);
    return v;
}

__global__ __launch_bounds__(kCullBlock) void k_cull_mlp(ivrgs_gaussians g, const ivrgs_camera *__restrict__ cams,
                                                        int camera, ivrgs_culler mlp, uint8_t *__restrict__ keep,
                                                        uint32_t *__restrict__ block_count,
                                                        float *__restrict__ logit_out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kg = lane >> 4;
    // weights of this lane's fragments
    bf16x4 a1[4], a2[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) a1[t] = load4(mlp.w1 + (16 * t + col) * kFeat + 4 * kg);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) a2[u][t] = load4(mlp.w2 + (16 * u + col) * kHidden + 16 * t + 4 * kg);
    // camera centre c = -R^T t
    const ivrgs_camera &cm = cams[camera];
    float cpos[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) cpos[i] = -(cm.R[i] * cm.t[0] + cm.R[3 + i] * cm.t[1] + cm.R[6 + i] * cm.t[2]);

    // biases and output weights staged once (global reads inside the loop
    // could not be hoisted past the stores below)
    __shared__ float sb1[kHidden], sb2[kHidden], sw3[kHidden];
    __shared__ uint32_t wave_cnt[4];
    if (threadIdx.x < kHidden) {
        sb1[threadIdx.x] = mlp.b1[threadIdx.x];
        sb2[threadIdx.x] = mlp.b2[threadIdx.x];
        sw3[threadIdx.x] = mlp.w3[threadIdx.x];
    }
    uint32_t kept_by_wave = 0;
    const int64_t n = g.n;
    // the features of the wave's four groups of 16 Gaussians, all loads
    // issued before the first product
    float fe[4][4];
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
        const int64_t gi = (int64_t)blockIdx.x * kCullBlock + wave * 64 + grp * 16 + col;
        float *f = fe[grp];
        f[0] = f[1] = f[2] = f[3] = 0.f;
        if (gi < n) {
            const float mx = g.mean[gi], my = g.mean[n + gi], mz = g.mean[2 * n + gi];
            const float vx = cpos[0] - mx, vy = cpos[1] - my, vz = cpos[2] - mz;
            const float inv = 1.f / sqrtf(vx * vx + vy * vy + vz * vz);
            if (kg == 0) {
                f[0] = mx; f[1] = my; f[2] = mz; f[3] = g.log_scale[gi];
            } else if (kg == 1) {
                f[0] = g.log_scale[n + gi]; f[1] = g.log_scale[2 * n + gi]; f[2] = g.opacity[gi]; f[3] = vx * inv;
            } else if (kg == 2) {
                f[0] = vy * inv; f[1] = vz * inv;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
        const int64_t gi = (int64_t)blockIdx.x * kCullBlock + wave * 64 + grp * 16 + col;
        const bool valid = gi < n;
        float f[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) f[i] = fe[grp][i];
        const bf16x4 x = pack4(f[0], f[1], f[2], f[3]);
        bf16x4 h1[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[t], x, acc, 0, 0, 0);
            float h[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) h[i] = fmaxf(acc[i] + sb1[16 * t + 4 * kg + i], 0.f);
            h1[t] = pack4(h[0], h[1], h[2], h[3]);
        }
        float part = 0.f;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[u][t], h1[t], acc, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int h = 16 * u + 4 * kg + i;
                part = fmaf(sw3[h], fmaxf(acc[i] + sb2[h], 0.f), part);
            }
        }
        // lanes col, col + 16, col + 32, col + 48 hold partial sums of one Gaussian
        part += __shfl_xor(part, 16, 64);
        part += __shfl_xor(part, 32, 64);
        const float logit = part + mlp.b3;
        const bool k = valid && logit >= mlp.threshold;
        if (kg == 0 && valid) {
            keep[gi] = k ? 1 : 0;
            if (logit_out) logit_out[gi] = logit;
        }
        kept_by_wave += __popcll(__ballot(k && kg == 0));
    }
    if (lane == 0) wave_cnt[wave] = kept_by_wave;
    __syncthreads();
    if (threadIdx.x == 0) block_count[blockIdx.x] = wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
}

// Ordered compaction: each workgroup sums the survivor counts of the blocks
// before its own (at most a few thousand words, read by all its threads at
// once) for its base; the last workgroup also writes the survivor total into
// the job table.
__global__ __launch_bounds__(kCullBlock) void k_cull_compact(const uint8_t *__restrict__ keep, int64_t n,
                                                            const uint32_t *__restrict__ counts, int n_blocks,
                                                            ivrgs_job *__restrict__ jobs, int job,
                                                            int32_t *__restrict__ out_index) {
    __shared__ uint32_t wave_before[4], wave_off[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t part = 0;
    for (int i = threadIdx.x; i < (int)blockIdx.x; i += kCullBlock) part += counts[i];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) part += __shfl_xor(part, d, 64);
    const int64_t gi = (int64_t)blockIdx.x * kCullBlock + threadIdx.x;
    const bool k = gi < n && keep[gi];
    const uint64_t m = __ballot(k);
    if (lane == 0) {
        wave_before[wave] = part;
        wave_off[wave] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    const uint32_t before = wave_before[0] + wave_before[1] + wave_before[2] + wave_before[3];
    if ((int)blockIdx.x == n_blocks - 1 && threadIdx.x == 0)
        jobs[job].gauss_count = (int32_t)(before + wave_off[0] + wave_off[1] + wave_off[2] + wave_off[3]);
    uint32_t off = before;
    for (int w = 0; w < wave; ++w) off += wave_off[w];
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (k) out_index[off + below] = (int32_t)gi;
}

__global__ void k_cull_empty(ivrgs_job *__restrict__ jobs, int job) {
    if (threadIdx.x == 0) jobs[job].gauss_count = 0;
}

hipError_t launch_cull(const ivrgs_gaussians &g, const ivrgs_camera *cams, int camera, const ivrgs_culler &mlp,
                       int32_t *out_index, ivrgs_job *jobs, int job, float *logits, uint8_t *keep,
                       uint32_t *counts, hipStream_t s) {
    const int n_blocks = (int)((g.n + kCullBlock - 1) / kCullBlock);
    TimedScope ts(TK_CULL, s);
    if (n_blocks > 0)
        hipLaunchKernelGGL(k_cull_mlp, dim3(n_blocks), dim3(kCullBlock), 0, s, g, cams, camera, mlp, keep, counts,
                           logits);
    if (n_blocks > 0)
        hipLaunchKernelGGL(k_cull_compact, dim3(n_blocks), dim3(kCullBlock), 0, s, keep, g.n, counts, n_blocks,
                           jobs, job, out_index);
    else
        hipLaunchKernelGGL(k_cull_empty, dim3(1), dim3(64), 0, s, jobs, job);
    return hipGetLastError();
}

size_t cull_workspace_bytes(int64_t n) {
    const int64_t n_blocks = (n + kCullBlock - 1) / kCullBlock;
    return (size_t)((n + 255) / 256 * 256) + sizeof(uint32_t) * (size_t)(n_blocks + 64);
}

}  // namespace ivrgs
