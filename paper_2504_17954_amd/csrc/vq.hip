// Vector quantisation of editable Gaussians (Sec. 4.4): scalar k-means
// codebooks per attribute, and the composition of quantised models with the
// codebook reads fused into the compose kernel (Sec. 4.5).
//
// The fit is memory-bound over the attribute's values: each Lloyd iteration
// streams them once, assigns each by binary search over the codebook held
// in LDS, and accumulates per-centroid FP64 sums and counts in LDS; one
// small workgroup then folds the per-workgroup partials in a fixed order,
// forms the means and re-sorts the codebook.
#include <algorithm>

#include "launch.hpp"

namespace ivrgs {

namespace {

constexpr int kVqThreads = 256;
constexpr int kVqItems = 16;                    // values per thread per tile
constexpr int kVqTile = kVqThreads * kVqItems;  // values per tile
constexpr int kVqMaxGroups = 1024;              // workgroups of the streaming kernels
constexpr int kVqMaxK = 256;
constexpr int kUpdateThreads = 1024;            // 4 threads per centroid in the update

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

int vq_groups(int64_t n) {
    const int64_t tiles = (n + kVqTile - 1) / kVqTile;
    return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, kVqMaxGroups));
}

struct VqWork {
    double *sum;     // [groups][k]
    uint32_t *cnt;   // [groups][k]
    float *range;    // [groups][2]: min, max of the finite values
};

VqWork vq_work(void *ws, int64_t n, int k) {
    const int g = vq_groups(n);
    char *p = static_cast<char *>(ws);
    VqWork w;
    w.sum = reinterpret_cast<double *>(p);
    p += align256(sizeof(double) * (size_t)g * k);
    w.cnt = reinterpret_cast<uint32_t *>(p);
    p += align256(sizeof(uint32_t) * (size_t)g * k);
    w.range = reinterpret_cast<float *>(p);
    return w;
}

// Nearest centroid of a finite x in an ascending codebook c[0, k): the
// index that a scan for the least |x - c_j| (FP32 difference, the lowest
// index on ties) returns.  Rounding is monotonic, so left of x the
// difference x - c_j only grows as j falls and right of x c_j - x only grows
// as j rises: the candidates are the last centroid at or below x, moved down
// over centroids whose difference rounds to the same value, and the first
// centroid above x.
__device__ __forceinline__ int nearest_sorted(float x, const float *c, int k) {
    int lo = 0, hi = k;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (c[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    const int q = lo;  // first centroid above x (k if none)
    if (q == 0) return 0;
    int p = q - 1;
    const float dl = x - c[p];
    while (p > 0 && x - c[p - 1] == dl) --p;
    if (q == k) return p;
    return dl <= c[q] - x ? p : q;
}

__device__ __forceinline__ int nearest_scan(float x, const float *c, int k) {
    int best = 0;
    float bd = fabsf(x - c[0]);
    for (int j = 1; j < k; ++j) {
        const float d = fabsf(x - c[j]);
        if (d < bd) {
            bd = d;
            best = j;
        }
    }
    return best;
}

__device__ __forceinline__ bool is_finite32(float x) { return (__float_as_uint(x) & 0x7F800000u) != 0x7F800000u; }

// The fits of one launch: codebook blockIdx.y takes its values, outputs and
// workspace rows from its entry, and its streaming kernels run on `groups`
// workgroups (a workgroup past them returns), so one codebook alone or
// several side by side decompose their values identically.
constexpr int kVqFitBatch = 8;
struct VqBook {
    const float *v;
    int64_t n;
    float *cb;
    uint8_t *index;
    double *psum;    // [groups][k]
    uint32_t *pcnt;  // [groups][k]
    float *part;     // [groups][2]
    int groups;
};
struct VqBooks {
    VqBook b[kVqFitBatch];
};

// Per workgroup: min and max of the finite values of its tiles.
__global__ __launch_bounds__(kVqThreads) void k_vq_range(VqBooks books) {
    const VqBook &bk = books.b[blockIdx.y];
    const int bid = blockIdx.x, nb = bk.groups;
    if (bid >= nb) return;
    const float *__restrict__ v = bk.v;
    const int64_t n = bk.n;
    float *__restrict__ part = bk.part;
    __shared__ float slo[kVqThreads / 64], shi[kVqThreads / 64];
    float lo = __builtin_inff(), hi = -__builtin_inff();
    for (int64_t t0 = (int64_t)bid * kVqTile; t0 < n; t0 += (int64_t)nb * kVqTile) {
        float x[kVqItems];
#pragma unroll
        for (int u = 0; u < kVqItems; ++u) {
            const int64_t i = t0 + u * kVqThreads + threadIdx.x;
            x[u] = i < n ? v[i] : __builtin_nanf("");
        }
#pragma unroll
        for (int u = 0; u < kVqItems; ++u)
            if (is_finite32(x[u])) {
                lo = fminf(lo, x[u]);
                hi = fmaxf(hi, x[u]);
            }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, d, 64));
        hi = fmaxf(hi, __shfl_xor(hi, d, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        slo[threadIdx.x >> 6] = lo;
        shi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kVqThreads / 64; ++w) {
            lo = fminf(lo, slo[w]);
            hi = fmaxf(hi, shi[w]);
        }
        part[2 * bid] = lo;
        part[2 * bid + 1] = hi;
    }
}

// One workgroup: the range over the `groups` partials, then centroid j at
// lo + (j + 1/2) * ((hi - lo) / k); all zero without a finite value.
__global__ __launch_bounds__(kVqThreads) void k_vq_init(VqBooks books, int k) {
    const VqBook &bk = books.b[blockIdx.y];
    const float *__restrict__ part = bk.part;
    const int groups = bk.n > 0 ? bk.groups : 0;
    float *__restrict__ cb = bk.cb;
    __shared__ float slo[kVqThreads / 64], shi[kVqThreads / 64];
    float lo = __builtin_inff(), hi = -__builtin_inff();
    for (int g = threadIdx.x; g < groups; g += kVqThreads) {
        lo = fminf(lo, part[2 * g]);
        hi = fmaxf(hi, part[2 * g + 1]);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, d, 64));
        hi = fmaxf(hi, __shfl_xor(hi, d, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        slo[threadIdx.x >> 6] = lo;
        shi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    lo = fminf(fminf(slo[0], slo[1]), fminf(slo[2], slo[3]));
    hi = fmaxf(fmaxf(shi[0], shi[1]), fmaxf(shi[2], shi[3]));
    const bool any = lo <= hi;
    const float w = (hi - lo) / (float)k;
    for (int j = threadIdx.x; j < k; j += kVqThreads) cb[j] = any ? lo + ((float)j + 0.5f) * w : 0.f;
}

// Assignment and accumulation of one Lloyd iteration: per workgroup, the
// FP64 sum and the count of the finite values nearest each centroid (the
// codebook is ascending throughout the fit).
__global__ __launch_bounds__(kVqThreads) void k_vq_lloyd(VqBooks books, int k) {
    const VqBook &bk = books.b[blockIdx.y];
    const int bid = blockIdx.x, nb = bk.groups;
    if (bid >= nb) return;
    const float *__restrict__ v = bk.v;
    const int64_t n = bk.n;
    const float *__restrict__ cb = bk.cb;
    double *__restrict__ psum = bk.psum;
    uint32_t *__restrict__ pcnt = bk.pcnt;
    __shared__ float c[kVqMaxK];
    __shared__ double sum[kVqMaxK];
    __shared__ uint32_t cnt[kVqMaxK];
    for (int j = threadIdx.x; j < k; j += kVqThreads) {
        c[j] = cb[j];
        sum[j] = 0.0;
        cnt[j] = 0u;
    }
    __syncthreads();
    for (int64_t t0 = (int64_t)bid * kVqTile; t0 < n; t0 += (int64_t)nb * kVqTile) {
        float x[kVqItems];
#pragma unroll
        for (int u = 0; u < kVqItems; ++u) {
            const int64_t i = t0 + u * kVqThreads + threadIdx.x;
            x[u] = i < n ? v[i] : __builtin_nanf("");
        }
#pragma unroll
        for (int u = 0; u < kVqItems; ++u)
            if (is_finite32(x[u])) {
                const int j = nearest_sorted(x[u], c, k);
                atomicAdd(&sum[j], (double)x[u]);
                atomicAdd(&cnt[j], 1u);
            }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += kVqThreads) {
        psum[(size_t)bid * k + j] = sum[j];
        pcnt[(size_t)bid * k + j] = cnt[j];
    }
}

// One workgroup of kUpdateThreads: thread (quarter q, centroid j) adds the
// partials of workgroups q, q + 4, ... in order; the quarters combine in a
// fixed order; each non-empty centroid becomes its mean, rounded to FP32;
// then a bitonic sort of the padded codebook in LDS.
__global__ __launch_bounds__(kUpdateThreads) void k_vq_update(VqBooks books, int k) {
    const VqBook &bk = books.b[blockIdx.y];
    const double *__restrict__ psum = bk.psum;
    const uint32_t *__restrict__ pcnt = bk.pcnt;
    const int groups = bk.groups;
    float *__restrict__ cb = bk.cb;
    __shared__ double qs[4][kVqMaxK];
    __shared__ uint32_t qc[4][kVqMaxK];
    __shared__ float key[kVqMaxK];
    const int j = threadIdx.x & (kVqMaxK - 1), q = threadIdx.x / kVqMaxK;
    double s = 0.0;
    uint32_t cn = 0u;
    if (j < k) {
#pragma unroll 8
        for (int g = q; g < groups; g += 4) {
            s += psum[(size_t)g * k + j];
            cn += pcnt[(size_t)g * k + j];
        }
    }
    qs[q][j] = s;
    qc[q][j] = cn;
    __syncthreads();
    if (q == 0) {
        float v = __builtin_inff();  // padding sorts last
        if (j < k) {
            const double S = (qs[0][j] + qs[1][j]) + (qs[2][j] + qs[3][j]);
            const uint32_t C = (qc[0][j] + qc[1][j]) + (qc[2][j] + qc[3][j]);
            v = C ? (float)(S / (double)C) : cb[j];
        }
        key[j] = v;
    }
    for (int size = 2; size <= kVqMaxK; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            const int t = threadIdx.x;
            if (t < kVqMaxK / 2) {
                const int i = 2 * stride * (t / stride) + (t % stride), l = i + stride;
                const bool up = (i & size) == 0;
                const float a = key[i], b = key[l];
                if ((a > b) == up) {
                    key[i] = b;
                    key[l] = a;
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < k) cb[threadIdx.x] = key[threadIdx.x];
}

// Index of every value: binary search when the codebook is ascending, a
// full scan otherwise (both give the least FP32 |x - c_j|, lowest index on
// ties); 0 for non-finite values.
__device__ __forceinline__ void vq_assign_body(const float *__restrict__ v, int64_t n, const float *__restrict__ cb,
                                               int k, uint8_t *__restrict__ index, int bid, int nb) {
    __shared__ float c[kVqMaxK];
    __shared__ int unsorted;
    if (threadIdx.x == 0) unsorted = 0;
    for (int j = threadIdx.x; j < k; j += kVqThreads) c[j] = cb[j];
    __syncthreads();
    for (int j = threadIdx.x; j + 1 < k; j += kVqThreads)
        if (!(c[j] <= c[j + 1])) unsorted = 1;
    __syncthreads();
    const bool sorted = unsorted == 0;
    for (int64_t t0 = (int64_t)bid * kVqTile; t0 < n; t0 += (int64_t)nb * kVqTile) {
        float x[kVqItems];
#pragma unroll
        for (int u = 0; u < kVqItems; ++u) {
            const int64_t i = t0 + u * kVqThreads + threadIdx.x;
            x[u] = i < n ? v[i] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < kVqItems; ++u) {
            const int64_t i = t0 + u * kVqThreads + threadIdx.x;
            if (i < n) {
                const int j = !is_finite32(x[u]) ? 0 : sorted ? nearest_sorted(x[u], c, k) : nearest_scan(x[u], c, k);
                index[i] = (uint8_t)j;
            }
        }
    }
}

__global__ __launch_bounds__(kVqThreads) void k_vq_assign(const float *__restrict__ v, int64_t n,
                                                          const float *__restrict__ cb, int k,
                                                          uint8_t *__restrict__ index) {
    vq_assign_body(v, n, cb, k, index, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kVqThreads) void k_vq_assign_books(VqBooks books, int k) {
    const VqBook &bk = books.b[blockIdx.y];
    if ((int)blockIdx.x >= bk.groups) return;
    vq_assign_body(bk.v, bk.n, bk.cb, k, bk.index, blockIdx.x, bk.groups);
}

constexpr int kVqBooks = 8;

struct VqComposeArgs {
    ivrgs_vq_model src[kComposeModels];
    int64_t offset[kComposeModels];    // first output index of each model
    int64_t quad[kComposeModels + 1];  // first thread of each model (4 Gaussians per thread)
    int32_t model0;                    // model number of src[0]
    int32_t count;
    float edit[kComposeModels][12];    // palette 3, opacity scale, shade scale 4, shade bias 4
};

__device__ __forceinline__ bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

// Decode and compose, four Gaussians per thread: mean and normal copied,
// every other attribute read through its codebook (index clamped to k - 1),
// then the edits of ivrgs_compose.  A workgroup inside one model stages that
// model's codebooks (at most 8 KiB) in LDS; one that straddles models reads
// them from global memory.  Planes move as float4 and the indices as four
// bytes when the model's slices are aligned.
__global__ __launch_bounds__(256) void k_vq_compose(VqComposeArgs a, ivrgs_gaussians_mut out) {
    __shared__ float book[kVqBooks * kVqMaxK];
    auto model_of = [&](int64_t t) {
        int j = 0;
        while (j + 1 < a.count && t >= a.quad[j + 1]) ++j;
        return j;
    };
    const int64_t nq = a.quad[a.count];
    const int64_t q0 = (int64_t)blockIdx.x * blockDim.x, q1 = min(q0 + (int64_t)blockDim.x, nq) - 1;
    const int jb = model_of(q0);
    const bool staged = jb == model_of(q1);
    if (staged) {
        const ivrgs_vq_model &m = a.src[jb];
        for (int e = threadIdx.x; e < kVqBooks * m.k; e += blockDim.x) book[e] = m.codebook[e];
    }
    __syncthreads();
    const int64_t t = q0 + threadIdx.x;
    if (t >= nq) return;
    const int j = model_of(t);
    const ivrgs_vq_model &m = a.src[j];
    const int64_t n = m.n, N = out.n, i0 = 4 * (t - a.quad[j]), o0 = a.offset[j] + i0;
    const int kk = m.k, last = kk - 1;
    const float *e = a.edit[j];
    // the body is instantiated once per codebook location, so that each keeps
    // its address space (LDS reads, or global loads)
    auto body = [&](auto look) {
        const bool vec = i0 + 4 <= n && (n & 3) == 0 && (N & 3) == 0 && (a.offset[j] & 3) == 0 &&
                         aligned(m.mean, 16) && aligned(m.normal, 16) && aligned(m.index, 4) && aligned(out.mean, 16) &&
                         aligned(out.log_scale, 16) && aligned(out.quat, 16) && aligned(out.opacity, 16) &&
                         aligned(out.normal, 16) && aligned(out.color, 16) && aligned(out.shade, 16) &&
                         aligned(out.model_id, 16);
        if (vec) {
            auto ld = [](const float *p) { return *reinterpret_cast<const float4 *>(p); };
            // streaming stores: the composed planes are not read again by this kernel
            auto st = [](float *p, float4 v) {
                typedef float f4v __attribute__((ext_vector_type(4)));
                __builtin_nontemporal_store(f4v{v.x, v.y, v.z, v.w}, reinterpret_cast<f4v *>(p));
            };
            auto idx4 = [&](int plane) { return *reinterpret_cast<const uint32_t *>(m.index + plane * n + i0); };
            // the four Gaussians' entries of codebook bk, then f applied to each
            auto dec4 = [&](int bk, int plane, auto f) {
                const uint32_t w = idx4(plane);
                return make_float4(f(look(bk, w & 255u)), f(look(bk, (w >> 8) & 255u)), f(look(bk, (w >> 16) & 255u)),
                                   f(look(bk, w >> 24)));
            };
            auto id = [](float v) { return v; };
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                st(out.mean + c * N + o0, ld(m.mean + c * n + i0));
                st(out.normal + c * N + o0, ld(m.normal + c * n + i0));
                st(out.log_scale + c * N + o0, dec4(0, c, id));
                const float pc = e[c];
                st(out.color + c * N + o0, dec4(3, 8 + c, [pc](float v) { return pc + v; }));
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                st(out.quat + c * N + o0, dec4(1, 3 + c, id));
                const float ks = e[4 + c], kb = e[8 + c];
                st(out.shade + c * N + o0, dec4(4 + c, 11 + c, [ks, kb](float v) { return fmaf(ks, v, kb); }));
            }
            const float so = e[3];
            st(out.opacity + o0, dec4(2, 7, [so](float v) { return so * v; }));
            const int model = a.model0 + j;
            typedef int i4v __attribute__((ext_vector_type(4)));
            __builtin_nontemporal_store(i4v{model, model, model, model}, reinterpret_cast<i4v *>(out.model_id + o0));
            return;
        }
        for (int64_t i = i0; i < i0 + 4 && i < n; ++i) {
            const int64_t o = a.offset[j] + i;
            auto dec = [&](int bk, int plane) { return look(bk, m.index[plane * n + i]); };
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                out.mean[c * N + o] = m.mean[c * n + i];
                out.normal[c * N + o] = m.normal[c * n + i];
                out.log_scale[c * N + o] = dec(0, c);
                out.color[c * N + o] = e[c] + dec(3, 8 + c);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                out.quat[c * N + o] = dec(1, 3 + c);
                out.shade[c * N + o] = fmaf(e[4 + c], dec(4 + c, 11 + c), e[8 + c]);
            }
            out.opacity[o] = e[3] * dec(2, 7);
            out.model_id[o] = a.model0 + j;
        }
    };
    if (staged) body([&](int bk, uint32_t idx) { return book[bk * kk + min((int)idx, last)]; });
    else body([&](int bk, uint32_t idx) { return m.codebook[bk * kk + min((int)idx, last)]; });
}

}  // namespace

size_t vq_workspace_bytes(int64_t n, int k) {
    const int g = vq_groups(n);
    return align256(sizeof(double) * (size_t)g * k) + align256(sizeof(uint32_t) * (size_t)g * k) +
           align256(sizeof(float) * 2 * (size_t)g);
}

static VqBook vq_book(const float *values, int64_t n, float *codebook, uint8_t *index, void *workspace, int k) {
    const VqWork w = vq_work(workspace, n, k);
    return VqBook{values, n, codebook, index, w.sum, w.cnt, w.range, vq_groups(n)};
}

// Up to kVqFitBatch fits side by side: one launch per step for all of them.
static hipError_t launch_vq_books(const VqBooks &bs, int count, int k, int iters, bool any_values, hipStream_t s) {
    int g = 1;
    for (int i = 0; i < count; ++i) g = std::max(g, bs.b[i].groups);
    const dim3 grid(g, count);
    if (any_values) hipLaunchKernelGGL(k_vq_range, grid, dim3(kVqThreads), 0, s, bs);
    hipLaunchKernelGGL(k_vq_init, dim3(1, count), dim3(kVqThreads), 0, s, bs, k);
    if (any_values) {
        for (int it = 0; it < iters; ++it) {
            hipLaunchKernelGGL(k_vq_lloyd, grid, dim3(kVqThreads), 0, s, bs, k);
            hipLaunchKernelGGL(k_vq_update, dim3(1, count), dim3(kUpdateThreads), 0, s, bs, k);
        }
        hipLaunchKernelGGL(k_vq_assign_books, grid, dim3(kVqThreads), 0, s, bs, k);
    }
    return hipGetLastError();
}

hipError_t launch_vq_fit(const float *values, int64_t n, int k, int iters, float *codebook, uint8_t *index,
                         void *workspace, hipStream_t s) {
    TimedScope ts(TK_VQ, s);
    VqBooks bs = {};
    bs.b[0] = vq_book(values, n, codebook, index, workspace, k);
    return launch_vq_books(bs, 1, k, iters, n > 0, s);
}

size_t vq_batch_workspace_bytes(const ivrgs_vq_book *books, int count, int k) {
    size_t b = 0;
    for (int i = 0; i < count; ++i) b += vq_workspace_bytes(books[i].n, k);
    return b;
}

hipError_t launch_vq_fit_batch(const ivrgs_vq_book *books, int count, int k, int iters, void *workspace,
                               hipStream_t s) {
    TimedScope ts(TK_VQ, s);
    char *ws = static_cast<char *>(workspace);
    for (int c0 = 0; c0 < count; c0 += kVqFitBatch) {
        const int m = std::min(kVqFitBatch, count - c0);
        VqBooks bs = {};
        bool any = false;
        for (int i = 0; i < m; ++i) {
            const ivrgs_vq_book &src = books[c0 + i];
            bs.b[i] = vq_book(src.values, src.n, src.codebook, src.index, ws, k);
            ws += vq_workspace_bytes(src.n, k);
            any = any || src.n > 0;
        }
        const hipError_t e = launch_vq_books(bs, m, k, iters, any, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_vq_assign(const float *values, int64_t n, const float *codebook, int k, uint8_t *index,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    TimedScope ts(TK_VQ, s);
    hipLaunchKernelGGL(k_vq_assign, dim3(vq_groups(n)), dim3(kVqThreads), 0, s, values, n, codebook, k, index);
    return hipGetLastError();
}

hipError_t launch_vq_compose(const ivrgs_vq_model *src, const int64_t *offset, int32_t model0, int32_t count,
                             const ivrgs_model_edit *edits, const ivrgs_gaussians_mut &out, hipStream_t s) {
    VqComposeArgs a = {};
    a.model0 = model0;
    a.count = count;
    int64_t quads = 0;
    for (int j = 0; j < count; ++j) {
        a.src[j] = src[j];
        a.offset[j] = offset[j];
        a.quad[j] = quads;
        quads += (src[j].n + 3) / 4;
        const ivrgs_model_edit &r = edits[j];
        for (int c = 0; c < 3; ++c) a.edit[j][c] = r.palette[c];
        a.edit[j][3] = r.opacity_scale;
        for (int c = 0; c < 4; ++c) {
            a.edit[j][4 + c] = r.shade_scale[c];
            a.edit[j][8 + c] = r.shade_bias[c];
        }
    }
    a.quad[count] = quads;
    if (quads == 0) return hipSuccess;
    TimedScope ts(TK_VQ, s);
    hipLaunchKernelGGL(k_vq_compose, dim3((unsigned)((quads + 255) / 256)), dim3(256), 0, s, a, out);
    return hipGetLastError();
}

}  // namespace ivrgs
