// Tile binning and per-tile depth sort.
//
// 1. Count: each workgroup owns a chunk of a job's records and counts, in LDS,
//    the pairs each tile of the job receives from it; the counts form a
//    [job][chunk][tile] matrix.
// 2. A column scan over chunks gives every (chunk, tile) its offset inside
//    the tile's list and each tile its total; one exclusive scan over all
//    (job, tile) totals gives the list starts, and the pair total is checked
//    against the capacity on the device.
// 3. Scatter: each chunk workgroup writes its (depth key, record id) pairs
//    from per-tile LDS cursors; no global atomics.
// 4. Per-tile stable LSD radix sort of the depth keys (8-bit digits, only the
//    digits that vary inside the tile), in LDS when the tile fits, otherwise
//    through global memory; equal keys are then ordered by record id, so the
//    result is the unique (depth key, record id) order whatever order the
//    scatter produced.
#include "launch.hpp"

namespace ivrgs {

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__device__ __forceinline__ void unpack_rect(uint2 rc, int &x0, int &y0, int &x1, int &y1) {
    x0 = rc.x & 0xFFFF;
    y0 = rc.x >> 16;
    x1 = rc.y & 0xFFFF;
    y1 = rc.y >> 16;
}

// Visits every (record, tile) pair of records [begin, end) of a job whose
// tile the record's ellipse reaches.  The work of 64 consecutive records is
// spread evenly over the lanes of one wave: the lanes scan the records' rect
// areas, then take the flattened (record, tile) items 64 at a time and find
// each item's record by binary search over the scanned offsets (a lane per
// record would leave most lanes idle behind the largest rect of the wave).
// f(record, tile x, tile y, depth key bits) is called once per hit pair; the
// order of the calls is unspecified.
constexpr int kBinWaves = 4;  // 256 threads per binning workgroup

struct ExpandLds {
    float4 h0[kBinWaves][64], h1[kBinWaves][64];  // hit tests of the wave's records
    uint32_t off[kBinWaves][64];                  // exclusive prefix of rect areas
    uint32_t org[kBinWaves][64];                  // rect origin, x0 | y0 << 16
    uint32_t wid[kBinWaves][64];                  // rect width in tiles
    uint32_t zb[kBinWaves][64];                   // depth key bits
};

// Orders a wave's LDS writes before its other lanes' reads.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename F>
__device__ __forceinline__ void for_each_pair(const ivrgs_job &job, int begin, int end, const float4 *rec4,
                                              const uint2 *rect, ExpandLds &L, F &&f) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int g0 = begin + wave * 64; g0 < end; g0 += kBinWaves * 64) {
        const int l = g0 + lane;
        uint32_t n = 0;
        if (l < end) {
            const int64_t r = (int64_t)job.rec_begin + l;
            const uint2 rc = rect[r];
            if (rc.x | rc.y) {
                int x0, y0, x1, y1;
                unpack_rect(rc, x0, y0, x1, y1);
                n = (uint32_t)((x1 - x0) * (y1 - y0));
                const float4 r2 = rec4[3 * r + 2];
                const HitTest h = make_hit_test(rec4[3 * r], rec4[3 * r + 1], r2);
                L.h0[wave][lane] = make_float4(h.mx, h.my, h.qa, h.qb);
                L.h1[wave][lane] = make_float4(h.qc, h.i2qa, h.i2qc, h.tol);
                L.org[wave][lane] = rc.x;
                L.wid[wave][lane] = (uint32_t)(x1 - x0);
                L.zb[wave][lane] = __float_as_uint(r2.y);
            }
        }
        uint32_t incl = n;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        L.off[wave][lane] = incl - n;
        const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
        wave_lds_sync();
        for (uint32_t base = 0; base < total; base += 64) {
            const uint32_t idx = base + lane;
            if (idx < total) {
                // the last record whose offset is <= idx; it has a nonempty rect
                int j = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1)
                    if (L.off[wave][j + step] <= idx) j += step;
                const uint32_t t = idx - L.off[wave][j];
                const uint32_t w = L.wid[wave][j];
                const uint32_t dy = t / w, dx = t - dy * w;
                const uint32_t o = L.org[wave][j];
                const int x = (int)((o & 0xFFFFu) + dx), y = (int)((o >> 16) + dy);
                const float4 a = L.h0[wave][j], c = L.h1[wave][j];
                const HitTest h = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
                if (box_hit(h, x * kTile, y * kTile, kTile, kTile))
                    f((int64_t)job.rec_begin + g0 + j, x, y, L.zb[wave][j]);
            }
        }
        wave_lds_sync();  // every lane is done with the tables before they are rewritten
    }
}

// Pass 1 of the binning: per (job, chunk of records) the number of pairs each
// tile receives, counted with LDS atomics and written into the count matrix
// [job][tile][chunk].
__global__ __launch_bounds__(256) void k_chunk_count(ivrgs_batch b, Consts k, const float *__restrict__ rec,
                                                     const uint2 *__restrict__ rect,
                                                     uint32_t *__restrict__ counts, int chunk, int n_chunks) {
    extern __shared__ uint32_t cnt[];
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int begin = blockIdx.x * chunk;
    if (begin >= job.gauss_count) return;
    const int end = min(begin + chunk, job.gauss_count);
    const int tpj = k.tiles_per_job, tx_n = k.tiles_x;
    for (int t = threadIdx.x; t < tpj; t += blockDim.x) cnt[t] = 0;
    __syncthreads();
    __shared__ ExpandLds L;
    for_each_pair(job, begin, end, reinterpret_cast<const float4 *>(rec), rect, L,
                  [&](int64_t, int x, int y, uint32_t) { atomicAdd(&cnt[y * tx_n + x], 1u); });
    __syncthreads();
    uint32_t *col = counts + (int64_t)blockIdx.y * tpj * n_chunks + blockIdx.x;
    for (int t = threadIdx.x; t < tpj; t += blockDim.x) col[(int64_t)t * n_chunks] = cnt[t];
}

// Per (job, tile), one wave: exclusive scan of the tile's counts over the
// job's chunks (contiguous in memory, in place) and the tile's total.
__global__ __launch_bounds__(256) void k_col_scan(ivrgs_batch b, Consts k, uint32_t *__restrict__ counts, int chunk,
                                                  int n_chunks, uint32_t *__restrict__ tile_counts) {
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= k.tiles_per_job) return;
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int rows = (job.gauss_count + chunk - 1) / chunk;
    uint32_t *col = counts + ((int64_t)blockIdx.y * k.tiles_per_job + t) * n_chunks;
    uint32_t carry = 0;
    for (int base = 0; base < rows; base += 64) {
        const int c = base + lane;
        const uint32_t v = c < rows ? col[c] : 0u;
        uint32_t incl = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        if (c < rows) col[c] = carry + incl - v;
        carry += __shfl(incl, 63, 64);
    }
    if (lane == 0) tile_counts[(int64_t)blockIdx.y * k.tiles_per_job + t] = carry;
}

// Exclusive prefix of 64-bit values over a workgroup of 1024 threads.
__device__ uint64_t block_exclusive_scan_1024(uint64_t v, uint64_t *tmp /* >= 16 */, uint64_t &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) tmp[wave] = incl;
    __syncthreads();
    uint64_t wave_off = 0, all = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        const uint64_t t = tmp[w];
        if (w < wave) wave_off += t;
        all += t;
    }
    total = all;
    __syncthreads();
    return wave_off + incl - v;
}

// Single workgroup: tile counts -> exclusive starts (in place) and the total,
// checked against the capacity.
__global__ __launch_bounds__(1024) void k_scan_tiles(uint32_t *__restrict__ starts, int64_t n_tiles,
                                                     int64_t *__restrict__ status, int64_t capacity) {
    __shared__ uint64_t tmp[16];
    const int64_t per = (n_tiles + blockDim.x - 1) / blockDim.x;
    const int64_t lo = threadIdx.x * per, hi = min(lo + per, n_tiles);
    uint64_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += starts[i];
    uint64_t total;
    uint64_t run = block_exclusive_scan_1024(sum, tmp, total);
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t c = starts[i];
        starts[i] = (uint32_t)run;
        run += c;
    }
    if (threadIdx.x == 0) {
        const bool over = total > (uint64_t)capacity || total > 0xFFFFFFF0ull;
        starts[n_tiles] = over ? 0xFFFFFFFFu : (uint32_t)total;
        status[0] = (int64_t)total;
        status[1] = over ? (int64_t)IVRGS_DEV_E_CAPACITY : 0;
        status[2] = 0;
        status[3] = 0;
    }
}

// Pass 2: each (job, chunk) workgroup starts its per-tile cursors at the
// tile's list start plus the chunk's exclusive column prefix and writes its
// (depth key, record id) pairs.  No global atomics.
__global__ __launch_bounds__(256) void k_scatter(ivrgs_batch b, Consts k, const float *__restrict__ rec,
                                                 const uint2 *__restrict__ rect, const uint32_t *__restrict__ counts,
                                                 uint32_t *__restrict__ keys, uint32_t *__restrict__ vals, int chunk,
                                                 int n_chunks, const uint32_t *__restrict__ starts, int64_t n_tiles) {
    extern __shared__ uint32_t cur[];
    if (starts[n_tiles] == 0xFFFFFFFFu) return;  // capacity exceeded
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int begin = blockIdx.x * chunk;
    if (begin >= job.gauss_count) return;
    const int end = min(begin + chunk, job.gauss_count);
    const int tpj = k.tiles_per_job, tx_n = k.tiles_x;
    const uint32_t *col = counts + (int64_t)blockIdx.y * tpj * n_chunks + blockIdx.x;
    const uint32_t *st = starts + (int64_t)blockIdx.y * tpj;
    for (int t = threadIdx.x; t < tpj; t += blockDim.x) cur[t] = st[t] + col[(int64_t)t * n_chunks];
    __syncthreads();
    __shared__ ExpandLds L;
    for_each_pair(job, begin, end, reinterpret_cast<const float4 *>(rec), rect, L,
                  [&](int64_t r, int x, int y, uint32_t z) {
                      const uint32_t slot = atomicAdd(&cur[y * tx_n + x], 1u);
                      keys[slot] = z;
                      vals[slot] = (uint32_t)r;
                  });
}

// ---------------------------------------------------------------------------
// Per-tile sort: wave w of a block owns the contiguous segment
// [w * seg, (w + 1) * seg) of the tile's list (seg a multiple of 64), so
// processing (wave, sub-batch of 64, lane) in order visits the list in order
// and each counting pass is stable.  Buffers ping-pong between an LDS pair
// (lists up to half the staging capacity), LDS and global memory (up to the
// capacity: the list lives in LDS and each pass stages through global
// memory), or two global arrays (larger lists).  A pass prefetches kU
// sub-batches per round so that a global source costs one latency per round.
constexpr int kBigWaves = 16;       // 1024 threads for lists above kSmallCap
constexpr int kSmallWaves = 4;      // 256 threads for lists up to kSmallCap
constexpr int kSmallCap = 4096;     // both ping-pong buffers in LDS
constexpr int kU = 8;

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lanes of the active mask whose digit equals this lane's digit.
__device__ __forceinline__ uint64_t match_digit(uint32_t dg, uint64_t active) {
    uint64_t m = active;
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        const uint64_t bb = __ballot((dg >> bit) & 1u);
        m &= ((dg >> bit) & 1u) ? bb : ~bb;
    }
    return m;
}

// Exclusive scan over threads 0..255 (others pass 0); every thread calls it.
__device__ uint32_t scan256(uint32_t v, uint32_t *tmp /* >= waves per block */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) tmp[wave] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (int w = 0; w < wave; ++w) off += tmp[w];
    __syncthreads();
    return off + incl - v;
}

// Turn per-wave digit histograms into per-wave starting offsets.
template <int NW>
__device__ void hist_to_offsets(uint32_t *hist, uint32_t *tmp) {
    uint32_t c[NW];
    uint32_t tot = 0;
    if (threadIdx.x < 256) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            c[w] = hist[w * 256 + threadIdx.x];
            tot += c[w];
        }
    }
    const uint32_t pre = scan256(threadIdx.x < 256 ? tot : 0u, tmp);
    if (threadIdx.x < 256) {
        uint32_t run = pre;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            hist[w * 256 + threadIdx.x] = run;
            run += c[w];
        }
    }
    __syncthreads();
}

// One stable counting pass on digit (key >> shift) & 255, src -> dst.
template <int NW>
__device__ void radix_pass(const uint32_t *sk, const uint32_t *sv, uint32_t *dk, uint32_t *dv, int n, int shift,
                           uint32_t *hist, uint32_t *tmp) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int seg = ((n + NW - 1) / NW + 63) / 64 * 64;
    const int s0 = min(wave * seg, n), s1 = min(s0 + seg, n);
    uint32_t *h = hist + wave * 256;
    for (int d = lane; d < 256; d += 64) h[d] = 0;
    __syncthreads();
    for (int i = s0 + lane; i < s1; i += 64) atomicAdd(&h[(sk[i] >> shift) & 255u], 1u);
    __syncthreads();
    hist_to_offsets<NW>(hist, tmp);
    for (int base = s0; base < s1; base += 64 * kU) {
        uint32_t kk[kU], vv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int i = base + u * 64 + lane;
            kk[u] = i < s1 ? sk[i] : 0u;
            vv[u] = i < s1 ? sv[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (base + u * 64 < s1) {  // wave-uniform
                const bool act = base + u * 64 + lane < s1;
                const uint32_t dg = (kk[u] >> shift) & 255u;
                const uint64_t m = match_digit(dg, __ballot(act));
                const uint32_t rank = lanes_below(m);
                const uint32_t pos = h[dg] + rank;
                if (act) {
                    dk[pos] = kk[u];
                    dv[pos] = vv[u];
                }
                if (act && rank == 0) h[dg] += (uint32_t)__popcll(m);
            }
        }
    }
    __syncthreads();
}

// Order runs of equal keys by value (record id).  Runs of equal FP32 depth
// keys are rare and short; each is insertion-sorted by one thread.
__device__ void fix_ties(const uint32_t *key, uint32_t *val, int n) {
    int tie = 0;
    for (int i = threadIdx.x + 1; i < n; i += blockDim.x) tie |= key[i] == key[i - 1];
    if (!__syncthreads_or(tie)) return;
    for (int i = threadIdx.x; i + 1 < n; i += blockDim.x) {
        if (key[i + 1] != key[i] || (i > 0 && key[i - 1] == key[i])) continue;
        int e = i + 1;
        while (e < n && key[e] == key[i]) ++e;
        for (int a = i + 1; a < e; ++a) {
            const uint32_t v = val[a];
            int c = a - 1;
            while (c >= i && val[c] > v) {
                val[c + 1] = val[c];
                --c;
            }
            val[c + 1] = v;
        }
    }
    __syncthreads();
}

// NW waves per block.  The small class takes lists of 2..kSmallCap pairs and
// keeps both buffers in LDS; the big class takes the longer lists.
template <int NW, bool kSmall>
__global__ __launch_bounds__(NW * 64) void k_tile_sort(const uint32_t *__restrict__ starts, int64_t n_tiles,
                                                       uint32_t *keys, uint32_t *vals, uint32_t *keys2,
                                                       uint32_t *vals2, int lds_cap) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t red_and[NW], red_or[NW], tmp[NW];
    if (starts[n_tiles] == 0xFFFFFFFFu) return;
    const uint32_t start = starts[blockIdx.x], end = starts[blockIdx.x + 1];
    const int n = (int)(end - start);
    if (n <= 1 || (kSmall ? n > kSmallCap : n <= kSmallCap)) return;
    uint32_t *hist = lds;
    uint32_t *buf = lds + NW * 256;  // keys [lds_cap] then values [lds_cap]
    const int half = lds_cap / 2;
    uint32_t *ka, *va, *kb, *vb;
    bool copy_back = false;  // list in LDS, staging in global memory
    if (n <= half) {
        ka = buf;
        va = buf + lds_cap;
        kb = buf + half;
        vb = buf + lds_cap + half;
    } else if (n <= lds_cap) {
        ka = buf;
        va = buf + lds_cap;
        kb = keys2 + start;
        vb = vals2 + start;
        copy_back = true;
    } else {
        ka = keys + start;
        va = vals + start;
        kb = keys2 + start;
        vb = vals2 + start;
    }
    const bool in_lds = n <= lds_cap;
    uint32_t a = 0xFFFFFFFFu, o = 0u;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t key = keys[start + i];
        if (in_lds) {
            ka[i] = key;
            va[i] = vals[start + i];
        }
        a &= key;
        o |= key;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        a &= __shfl_xor(a, d, 64);
        o |= __shfl_xor(o, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red_and[threadIdx.x >> 6] = a;
        red_or[threadIdx.x >> 6] = o;
    }
    __syncthreads();
    a = 0xFFFFFFFFu;
    o = 0u;
    for (int w = 0; w < NW; ++w) {
        a &= red_and[w];
        o |= red_or[w];
    }
    const uint32_t varying = a ^ o;
    for (int d = 0; d < 4; ++d) {
        if (((varying >> (8 * d)) & 255u) == 0u) continue;
        radix_pass<NW>(ka, va, kb, vb, n, 8 * d, hist, tmp);
        if (copy_back) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                ka[i] = kb[i];
                va[i] = vb[i];
            }
            __syncthreads();
        } else {
            uint32_t *t0 = ka, *t1 = va;
            ka = kb;
            va = vb;
            kb = t0;
            vb = t1;
        }
    }
    fix_ties(ka, va, n);
    if (va != vals + start)
        for (int i = threadIdx.x; i < n; i += blockDim.x) vals[start + i] = va[i];
}

// Work queue for the persistent render kernels: nonempty tiles ordered by
// floor(log2(pairs)) descending, so the longest lists start first.
// queue[1] = number of items, queue[2 + i] = tile of item i; queue[0] is the
// counter the render kernels advance (reset before each launch).
__global__ __launch_bounds__(1024) void k_work_queue(const uint32_t *__restrict__ starts, int64_t n_tiles,
                                                     uint32_t *__restrict__ queue) {
    __shared__ uint32_t hist[32], base[32];
    if (starts[n_tiles] == 0xFFFFFFFFu) {
        if (threadIdx.x == 0) queue[1] = 0;
        return;
    }
    if (threadIdx.x < 32) hist[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < n_tiles; t += blockDim.x) {
        const uint32_t c = starts[t + 1] - starts[t];
        if (c) atomicAdd(&hist[31 - __clz(c)], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int b = 31; b >= 0; --b) {
            base[b] = run;
            run += hist[b];
        }
        queue[1] = run;
    }
    __syncthreads();
    for (int64_t t = threadIdx.x; t < n_tiles; t += blockDim.x) {
        const uint32_t c = starts[t + 1] - starts[t];
        if (c) queue[2 + atomicAdd(&base[31 - __clz(c)], 1u)] = (uint32_t)t;
    }
}

hipError_t launch_work_queue(const uint32_t *starts, int64_t n_tiles, uint32_t *queue, hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    TimedScope ts(TK_COUNT, s);
    hipLaunchKernelGGL(k_work_queue, dim3(1), dim3(1024), 0, s, starts, n_tiles, queue);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + 255) / 256;
    const int64_t blocks = want < 4096 ? want : 4096;
    TimedScope ts(TK_FILL, s);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

int chunk_rows(const ivrgs_batch &b, int chunk) { return (b.max_job_count + chunk - 1) / chunk; }

hipError_t launch_bin_sort(const ivrgs_batch &b, const Consts &k, const float *rec, const uint32_t *rect,
                           const ivrgs_bins &bins, const BinWork &w, int chunk, int lds_cap, size_t sort_lds,
                           hipStream_t s) {
    const int64_t n_tiles = (int64_t)b.n_jobs * k.tiles_per_job;
    const int n_chunks = chunk_rows(b, chunk);
    const size_t cnt_lds = sizeof(uint32_t) * k.tiles_per_job;
    {
        TimedScope ts(TK_COUNT, s);
        if (n_chunks > 0) {
            hipLaunchKernelGGL(k_chunk_count, dim3(n_chunks, b.n_jobs), dim3(256), cnt_lds, s, b, k, rec,
                               reinterpret_cast<const uint2 *>(rect), w.counts, chunk, n_chunks);
            hipLaunchKernelGGL(k_col_scan, dim3((k.tiles_per_job + 3) / 4, b.n_jobs), dim3(256), 0, s, b, k,
                               w.counts, chunk, n_chunks, bins.tile_start);
        } else if (n_tiles > 0) {
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, bins.tile_start, n_tiles, 0u);
        }
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, bins.tile_start, n_tiles, bins.status,
                           bins.capacity);
    }
    if (n_chunks > 0) {
        TimedScope ts(TK_SCATTER, s);
        hipLaunchKernelGGL(k_scatter, dim3(n_chunks, b.n_jobs), dim3(256), cnt_lds, s, b, k, rec,
                           reinterpret_cast<const uint2 *>(rect), w.counts, w.keys, bins.sorted, chunk, n_chunks,
                           bins.tile_start, n_tiles);
    }
    if (n_tiles > 0) {
        TimedScope ts(TK_SORT, s);
        hipLaunchKernelGGL((k_tile_sort<kSmallWaves, true>), dim3((unsigned)n_tiles), dim3(kSmallWaves * 64),
                           small_sort_lds_bytes(), s, bins.tile_start, n_tiles, w.keys, bins.sorted, w.keys2,
                           w.vals2, 2 * kSmallCap);
        hipLaunchKernelGGL((k_tile_sort<kBigWaves, false>), dim3((unsigned)n_tiles), dim3(kBigWaves * 64), sort_lds,
                           s, bins.tile_start, n_tiles, w.keys, bins.sorted, w.keys2, w.vals2, lds_cap);
    }
    return hipGetLastError();
}

// Static LDS of the binning kernels (their per-tile counters are dynamic).
size_t bin_static_lds_bytes() { return sizeof(ExpandLds); }

hipError_t set_bin_lds_limit(size_t bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_chunk_count),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k_scatter), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

// LDS bytes of the big-list sort for a staging capacity (elements).
size_t sort_lds_bytes(int lds_cap) { return sizeof(uint32_t) * (kBigWaves * 256 + 2 * (size_t)lds_cap); }

size_t small_sort_lds_bytes() { return sizeof(uint32_t) * (kSmallWaves * 256 + 4 * (size_t)kSmallCap); }

hipError_t set_sort_lds_limit(size_t bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_tile_sort<kBigWaves, false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k_tile_sort<kSmallWaves, true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)small_sort_lds_bytes());
}

}  // namespace ivrgs
