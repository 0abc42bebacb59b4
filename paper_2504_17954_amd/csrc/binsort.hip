// Tile binning in depth order.
//
// 1. Depth order: each job's records are sorted by (FP32 depth key bits,
//    record id) with a segmented LSD radix sort: 8-bit digits, segments of
//    4096 records per workgroup, every pass stable, the initial order by id.
//    A digit that is constant over the job's visible records is skipped.
// 2. Count: one wave per chunk of consecutive records of the depth order
//    counts, in LDS, the pairs each tile of the job receives from it; the
//    counts form a [job][tile][chunk] matrix.
// 3. A column scan over chunks gives every (chunk, tile) its offset inside
//    the tile's list and each tile its total; one exclusive scan over all
//    (job, tile) totals gives the list starts, and the pair total is checked
//    against the capacity on the device.
// 4. Scatter: each chunk walks its records in depth order and appends every
//    pair to its tile from a per-tile LDS cursor.  Lanes of one step that
//    append to the same tile hold different records, in depth order by
//    lane, and are ranked by lane, so each tile's list comes out in
//    (depth key, record id) order: no per-tile sort.
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

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Active lanes whose value v (bits < nbits) equals this lane's.
__device__ __forceinline__ uint64_t match_bits(uint32_t v, int nbits, uint64_t active) {
    uint64_t m = active;
    for (int bit = 0; bit < nbits; ++bit) {
        const uint64_t bb = __ballot((v >> bit) & 1u);
        m &= ((v >> bit) & 1u) ? bb : ~bb;
    }
    return m;
}

// ---------------------------------------------------------------------------
// Depth order.
constexpr int kSegThreads = 256;
constexpr int kSegItems = 16;                         // per thread
constexpr int kSeg = kSegThreads * kSegItems;         // records per segment
constexpr int kSegWaveItems = kSeg / (kSegThreads / 64);  // contiguous per wave

int seg_rows(const ivrgs_batch &b) { return (b.max_job_count + kSeg - 1) / kSeg; }

// AND and OR of the depth keys of each job's visible records (rng[j] and
// rng[n_jobs + j], preset to ~0 and 0).  Culled records carry the key ~0.
__global__ __launch_bounds__(kSegThreads) void k_dkey_range(ivrgs_batch b, const uint32_t *__restrict__ depth,
                                                            uint32_t *__restrict__ rng) {
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int64_t base = (int64_t)blockIdx.x * kSeg;
    if (base >= job.gauss_count) return;
    uint32_t a = 0xFFFFFFFFu, o = 0u;
    for (int i = threadIdx.x; i < kSeg && base + i < job.gauss_count; i += kSegThreads) {
        const uint32_t z = depth[(int64_t)job.rec_begin + base + i];
        if (z != 0xFFFFFFFFu) {
            a &= z;
            o |= z;
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        a &= __shfl_xor(a, d, 64);
        o |= __shfl_xor(o, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAnd(&rng[blockIdx.y], a);
        atomicOr(&rng[b.n_jobs + blockIdx.y], o);
    }
}

__device__ __forceinline__ bool digit_varies(const uint32_t *rng, int n_jobs, int job, int shift) {
    return (((rng[job] ^ rng[n_jobs + job]) >> shift) & 255u) != 0u;
}

// Passes on varying digits below digit `shift` (only those move the data).
// The first such pass reads the keys from the projection's depth array with
// the record ids implicit; pass i (from 0) writes buffer i & 1.
__device__ __forceinline__ int passes_before(const uint32_t *rng, int n_jobs, int job, int shift) {
    const uint32_t v = rng[job] ^ rng[n_jobs + job];
    int p = 0;
    for (int sh = 0; sh < shift; sh += 8) p += ((v >> sh) & 255u) != 0u;
    return p;
}

// The job's records in depth order (absolute record indices), or nullptr if
// no digit varies: then the order is the record order itself.
__device__ __forceinline__ const uint32_t *depth_order(const uint32_t *rng, int n_jobs, int job,
                                                      const uint32_t *val0, const uint32_t *val1) {
    const int p = passes_before(rng, n_jobs, job, 32);
    return p == 0 ? nullptr : ((p - 1) & 1 ? val1 : val0);
}

// Per (job, segment): digit histogram into hist[job][digit][segment].
__global__ __launch_bounds__(kSegThreads) void k_dsort_hist(ivrgs_batch b, const uint32_t *__restrict__ depth,
                                                            const uint32_t *__restrict__ key0,
                                                            const uint32_t *__restrict__ key1,
                                                            const uint32_t *__restrict__ rng, int shift,
                                                            uint32_t *__restrict__ hist, int n_seg) {
    __shared__ uint32_t h[256];
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int64_t base = (int64_t)blockIdx.x * kSeg;
    if (base >= job.gauss_count || !digit_varies(rng, b.n_jobs, blockIdx.y, shift)) return;
    h[threadIdx.x] = 0;
    __syncthreads();
    const int before = passes_before(rng, b.n_jobs, blockIdx.y, shift);
    const uint32_t *k = (before == 0 ? depth : ((before - 1) & 1 ? key1 : key0)) + job.rec_begin + base;
    const int n = (int)min((int64_t)kSeg, job.gauss_count - base);
    for (int i = threadIdx.x; i < n; i += kSegThreads) atomicAdd(&h[(k[i] >> shift) & 255u], 1u);
    __syncthreads();
    hist[((int64_t)blockIdx.y * 256 + threadIdx.x) * n_seg + blockIdx.x] = h[threadIdx.x];
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
    uint64_t off = 0;
    total = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        if (w < wave) off += tmp[w];
        total += tmp[w];
    }
    __syncthreads();
    return off + incl - v;
}

// Per (job, digit), one wave: exclusive scan of the digit's counts over the
// job's segments (contiguous, in place) and the digit's total into
// tot[job][digit].
__global__ __launch_bounds__(256) void k_dsort_colscan(ivrgs_batch b, const uint32_t *__restrict__ rng, int shift,
                                                       uint32_t *__restrict__ hist, uint32_t *__restrict__ tot,
                                                       int n_seg) {
    const int d = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int rows = (job.gauss_count + kSeg - 1) / kSeg;
    if (rows == 0 || !digit_varies(rng, b.n_jobs, blockIdx.y, shift)) return;
    uint32_t *col = hist + ((int64_t)blockIdx.y * 256 + d) * n_seg;
    uint32_t carry = 0;
    for (int base = 0; base < rows; base += 64) {
        const int c = base + lane;
        const uint32_t v = c < rows ? col[c] : 0u;
        uint32_t incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (c < rows) col[c] = carry + incl - v;
        carry += __shfl(incl, 63, 64);
    }
    if (lane == 0) tot[(int64_t)blockIdx.y * 256 + d] = carry;
}

// Per (job, segment): stable scatter of the segment's (key, id) pairs by
// digit.  Wave w owns the contiguous part [w * kSegWaveItems, ...) of the
// segment and ranks equal digits by lane inside each step of 64, so the
// order within a digit is the input order.  A digit that is constant over
// the job leaves the pairs where they are (see passes_before).
__global__ __launch_bounds__(kSegThreads) void k_dsort_scatter(ivrgs_batch b, const uint32_t *__restrict__ depth,
                                                               uint32_t *__restrict__ key0,
                                                               uint32_t *__restrict__ val0,
                                                               uint32_t *__restrict__ key1,
                                                               uint32_t *__restrict__ val1,
                                                               const uint32_t *__restrict__ rng, int shift,
                                                               const uint32_t *__restrict__ hist,
                                                               const uint32_t *__restrict__ tot, int n_seg) {
    __shared__ uint32_t wh[kSegThreads / 64][256];  // per wave: count, then start, per digit
    __shared__ uint32_t wsum[kSegThreads / 64];
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int64_t base = (int64_t)blockIdx.x * kSeg;
    if (base >= job.gauss_count) return;
    const int n = (int)min((int64_t)kSeg, job.gauss_count - base);
    const int64_t off = job.rec_begin + base;
    if (!digit_varies(rng, b.n_jobs, blockIdx.y, shift)) return;
    const int before = passes_before(rng, b.n_jobs, blockIdx.y, shift);
    const bool first = before == 0, to1 = (before & 1) != 0;
    const uint32_t *sk = first ? depth : (to1 ? key0 : key1), *sv = to1 ? val0 : val1;
    uint32_t *dk = to1 ? key1 : key0, *dv = to1 ? val1 : val0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int w0 = wave * kSegWaveItems;
    uint32_t kk[kSegItems], vv[kSegItems];
#pragma unroll
    for (int u = 0; u < kSegItems; ++u) {
        const int i = w0 + u * 64 + lane;
        kk[u] = i < n ? sk[off + i] : 0u;
        vv[u] = i < n ? (first ? (uint32_t)(off + i) : sv[off + i]) : 0u;
    }
    for (int d = lane; d < 256; d += 64) wh[wave][d] = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kSegItems; ++u)
        if (w0 + u * 64 + lane < n) atomicAdd(&wh[wave][(kk[u] >> shift) & 255u], 1u);
    __syncthreads();
    {
        // thread d: start of digit d in the job (exclusive scan of the digit
        // totals), plus this segment's offset inside the digit, plus the
        // counts of the waves before
        const int d = threadIdx.x;
        const uint32_t t = tot[(int64_t)blockIdx.y * 256 + d];
        uint32_t incl = t;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t digit_start = incl - t;
        for (int w = 0; w < wave; ++w) digit_start += wsum[w];
        uint32_t run = digit_start + hist[((int64_t)blockIdx.y * 256 + d) * n_seg + blockIdx.x];
#pragma unroll
        for (int w = 0; w < kSegThreads / 64; ++w) {
            const uint32_t c = wh[w][d];
            wh[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
    uint32_t *dkj = dk + job.rec_begin, *dvj = dv + job.rec_begin;
#pragma unroll
    for (int u = 0; u < kSegItems; ++u) {
        if (w0 + u * 64 < n) {  // wave-uniform
            const bool act = w0 + u * 64 + lane < n;
            const uint32_t dg = (kk[u] >> shift) & 255u;
            const uint64_t m = match_bits(dg, 8, __ballot(act));
            const uint32_t rank = lanes_below(m);
            const uint32_t pos = wh[wave][dg] + rank;
            if (act) {
                dkj[pos] = kk[u];
                dvj[pos] = vv[u];
            }
            if (act && rank == 0) wh[wave][dg] += (uint32_t)__popcll(m);
        }
    }
}

// ---------------------------------------------------------------------------
// Binning over the depth order.
//
// Visits every (record, tile) pair of the chunk [begin, end) of a job's depth
// order whose tile the record's ellipse reaches, in depth order.  The work of
// 64 consecutive records is spread evenly over the lanes: the lanes scan the
// records' rect areas, then take the flattened (record, tile) items 64 at a
// time (record-major, so in depth order) and find each item's record by
// binary search over the scanned offsets.  f(record, tile x, tile y) is
// called by the lanes of a hit, all lanes of one step together.
struct ExpandLds {
    float4 h0[64], h1[64];  // hit tests of the step's records
    uint32_t off[64];       // exclusive prefix of rect areas
    uint32_t org[64];       // rect origin, x0 | y0 << 16
    uint32_t wid[64];       // rect width in tiles
    uint32_t rid[64];       // record index
};
constexpr int kBinWaves = 4;  // waves (chunks) per binning workgroup at most

// Orders a wave's LDS writes before its other lanes' reads.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename F>
__device__ __forceinline__ void for_each_pair(const ivrgs_job &job, int begin, int end, const uint32_t *order,
                                              const float4 *rec4, const uint2 *rect, ExpandLds &L, F &&f) {
    const int lane = threadIdx.x & 63;
    for (int g0 = begin; g0 < end; g0 += 64) {
        const int l = g0 + lane;
        uint32_t n = 0;
        if (l < end) {
            const int64_t r = order ? (int64_t)order[(int64_t)job.rec_begin + l] : (int64_t)job.rec_begin + l;
            const uint2 rc = rect[r];
            if (rc.x | rc.y) {
                int x0, y0, x1, y1;
                unpack_rect(rc, x0, y0, x1, y1);
                n = (uint32_t)((x1 - x0) * (y1 - y0));
                const HitTest h = make_hit_test(rec4[3 * r], rec4[3 * r + 1], rec4[3 * r + 2]);
                L.h0[lane] = make_float4(h.mx, h.my, h.qa, h.qb);
                L.h1[lane] = make_float4(h.qc, h.i2qa, h.i2qc, h.tol);
                L.org[lane] = rc.x;
                L.wid[lane] = (uint32_t)(x1 - x0);
                L.rid[lane] = (uint32_t)r;
            }
        }
        uint32_t incl = n;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        L.off[lane] = incl - n;
        const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
        wave_lds_sync();
        for (uint32_t base = 0; base < total; base += 64) {
            const uint32_t idx = base + lane;
            if (idx < total) {
                // the last record whose offset is <= idx; it has a nonempty rect
                int j = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1)
                    if (L.off[j + step] <= idx) j += step;
                const uint32_t t = idx - L.off[j];
                const uint32_t w = L.wid[j];
                const uint32_t dy = t / w, dx = t - dy * w;
                const uint32_t o = L.org[j];
                const int x = (int)((o & 0xFFFFu) + dx), y = (int)((o >> 16) + dy);
                const float4 a = L.h0[j], c = L.h1[j];
                const HitTest h = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
                if (box_hit(h, x * kTile, y * kTile, kTile, kTile)) f(L.rid[j], x, y);
            }
        }
        wave_lds_sync();  // every lane is done with the tables before they are rewritten
    }
}

// Pairs per tile from each (job, chunk), into counts[job][tile][chunk].  A
// workgroup of NW waves takes NW consecutive chunks, one per wave, each with
// its own LDS counters; the NW counts of a tile are adjacent in the matrix.
template <int NW>
__global__ __launch_bounds__(NW * 64) void k_chunk_count(ivrgs_batch b, Consts k, const float *__restrict__ rec,
                                                         const uint2 *__restrict__ rect,
                                                         const uint32_t *__restrict__ val0,
                                                         const uint32_t *__restrict__ val1,
                                                         const uint32_t *__restrict__ rng,
                                                         uint32_t *__restrict__ counts, int chunk, int n_chunks) {
    extern __shared__ uint32_t cnt[];  // [NW][tiles]
    __shared__ ExpandLds L[NW];
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int first = blockIdx.x * NW * chunk;
    if (first >= job.gauss_count) return;
    const int tpj = k.tiles_per_job, tx_n = k.tiles_x;
    const int wave = threadIdx.x >> 6;
    for (int t = threadIdx.x; t < NW * tpj; t += NW * 64) cnt[t] = 0;
    __syncthreads();
    const int begin = first + wave * chunk;
    const int end = min(begin + chunk, job.gauss_count);
    const uint32_t *order = depth_order(rng, b.n_jobs, blockIdx.y, val0, val1);
    uint32_t *c = cnt + wave * tpj;
    for_each_pair(job, begin, end, order, reinterpret_cast<const float4 *>(rec), rect, L[wave],
                  [&](uint32_t, int x, int y) { atomicAdd(&c[y * tx_n + x], 1u); });
    __syncthreads();
    uint32_t *col = counts + (int64_t)blockIdx.y * tpj * n_chunks + blockIdx.x * NW;
    for (int t = threadIdx.x; t < tpj; t += NW * 64)
#pragma unroll
        for (int w = 0; w < NW; ++w) col[(int64_t)t * n_chunks + w] = cnt[w * tpj + t];
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

// Each (job, chunk) wave starts its per-tile cursors at the tile's list start
// plus the chunk's exclusive column prefix and appends its record ids in
// depth order.  No global atomics.
template <int NW>
__global__ __launch_bounds__(NW * 64) void k_scatter(ivrgs_batch b, Consts k, const float *__restrict__ rec,
                                                     const uint2 *__restrict__ rect,
                                                     const uint32_t *__restrict__ val0,
                                                     const uint32_t *__restrict__ val1,
                                                     const uint32_t *__restrict__ rng,
                                                     const uint32_t *__restrict__ counts,
                                                     uint32_t *__restrict__ sorted, int chunk, int n_chunks,
                                                     const uint32_t *__restrict__ starts, int64_t n_tiles) {
    extern __shared__ uint32_t cur[];  // [NW][tiles]
    __shared__ ExpandLds L[NW];
    if (starts[n_tiles] == 0xFFFFFFFFu) return;  // capacity exceeded
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int first = blockIdx.x * NW * chunk;
    if (first >= job.gauss_count) return;
    const int tpj = k.tiles_per_job, tx_n = k.tiles_x;
    const int tile_bits = 32 - __clz(max(tpj - 1, 1));
    const int wave = threadIdx.x >> 6;
    const uint32_t *col = counts + (int64_t)blockIdx.y * tpj * n_chunks + blockIdx.x * NW;
    const uint32_t *st = starts + (int64_t)blockIdx.y * tpj;
    for (int t = threadIdx.x; t < tpj; t += NW * 64) {
        const uint32_t s0 = st[t];
#pragma unroll
        for (int w = 0; w < NW; ++w) cur[w * tpj + t] = s0 + col[(int64_t)t * n_chunks + w];
    }
    __syncthreads();
    const int begin = first + wave * chunk;
    const int end = min(begin + chunk, job.gauss_count);
    const uint32_t *order = depth_order(rng, b.n_jobs, blockIdx.y, val0, val1);
    uint32_t *c = cur + wave * tpj;
    for_each_pair(job, begin, end, order, reinterpret_cast<const float4 *>(rec), rect, L[wave],
                  [&](uint32_t r, int x, int y) {
                      const uint32_t t = (uint32_t)(y * tx_n + x);
                      const uint64_t m = match_bits(t, tile_bits, __ballot(true));
                      const uint32_t rank = lanes_below(m);
                      const uint32_t at = c[t];
                      sorted[at + rank] = r;
                      if (rank == 0) c[t] = at + (uint32_t)__popcll(m);
                  });
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

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + 255) / 256;
    const int64_t blocks = want < 4096 ? want : 4096;
    TimedScope ts(TK_FILL, s);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Chunks per job, padded to a multiple of kBinWaves (a workgroup takes up
// to kBinWaves consecutive chunks).
int chunk_rows(const ivrgs_batch &b, int chunk) {
    const int rows = (b.max_job_count + chunk - 1) / chunk;
    return (rows + kBinWaves - 1) / kBinWaves * kBinWaves;
}

size_t depth_sort_hist_words(const ivrgs_batch &b) { return (size_t)b.n_jobs * 256 * ((size_t)seg_rows(b) + 1); }

template <int NW>
static void launch_binning(const ivrgs_batch &b, const Consts &k, const float *rec, const uint2 *rect2,
                           const ivrgs_bins &bins, const BinWork &w, int chunk, int n_chunks,
                           int64_t n_tiles, hipStream_t s) {
    const size_t lds = sizeof(uint32_t) * NW * (size_t)k.tiles_per_job;
    const dim3 grid((unsigned)(n_chunks / NW), (unsigned)b.n_jobs);
    {
        TimedScope ts(TK_COUNT, s);
        hipLaunchKernelGGL(k_chunk_count<NW>, grid, dim3(NW * 64), lds, s, b, k, rec, rect2, w.val[0], w.val[1],
                           w.rng, w.counts, chunk, n_chunks);
        hipLaunchKernelGGL(k_col_scan, dim3((k.tiles_per_job + 3) / 4, b.n_jobs), dim3(256), 0, s, b, k, w.counts,
                           chunk, n_chunks, bins.tile_start);
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, bins.tile_start, n_tiles, bins.status,
                           bins.capacity);
    }
    TimedScope ts(TK_SCATTER, s);
    hipLaunchKernelGGL(k_scatter<NW>, grid, dim3(NW * 64), lds, s, b, k, rec, rect2, w.val[0], w.val[1], w.rng,
                       w.counts, bins.sorted, chunk, n_chunks, bins.tile_start, n_tiles);
}

hipError_t launch_bin_sort(const ivrgs_batch &b, const Consts &k, const float *rec, const uint32_t *rect,
                           const uint32_t *depth, const ivrgs_bins &bins, const BinWork &w, int chunk,
                           size_t bin_lds, hipStream_t s) {
    const int64_t n_tiles = (int64_t)b.n_jobs * k.tiles_per_job;
    const int n_chunks = chunk_rows(b, chunk);
    const int n_seg = seg_rows(b);
    const uint2 *rect2 = reinterpret_cast<const uint2 *>(rect);
    uint32_t *tot = w.hist + (size_t)b.n_jobs * 256 * n_seg;
    if (n_seg > 0) {
        TimedScope ts(TK_SORT, s);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, w.rng, (int64_t)b.n_jobs, 0xFFFFFFFFu);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, w.rng + b.n_jobs, (int64_t)b.n_jobs, 0u);
        hipLaunchKernelGGL(k_dkey_range, dim3(n_seg, b.n_jobs), dim3(kSegThreads), 0, s, b, depth, w.rng);
        for (int pass = 0; pass < 4; ++pass) {
            const int shift = 8 * pass;
            hipLaunchKernelGGL(k_dsort_hist, dim3(n_seg, b.n_jobs), dim3(kSegThreads), 0, s, b, depth, w.key[0],
                               w.key[1], w.rng, shift, w.hist, n_seg);
            hipLaunchKernelGGL(k_dsort_colscan, dim3(64, b.n_jobs), dim3(256), 0, s, b, w.rng, shift, w.hist, tot,
                               n_seg);
            hipLaunchKernelGGL(k_dsort_scatter, dim3(n_seg, b.n_jobs), dim3(kSegThreads), 0, s, b, depth, w.key[0],
                               w.val[0], w.key[1], w.val[1], w.rng, shift, w.hist, tot, n_seg);
        }
    }
    if (n_chunks == 0) {
        TimedScope ts(TK_COUNT, s);
        if (n_tiles > 0) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, bins.tile_start, n_tiles, 0u);
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, bins.tile_start, n_tiles, bins.status,
                           bins.capacity);
        return hipGetLastError();
    }
    // as many chunks per workgroup as the per-tile counters allow
    const size_t per_wave = sizeof(uint32_t) * (size_t)k.tiles_per_job;
    if (4 * per_wave <= bin_lds) launch_binning<4>(b, k, rec, rect2, bins, w, chunk, n_chunks, n_tiles, s);
    else if (2 * per_wave <= bin_lds) launch_binning<2>(b, k, rec, rect2, bins, w, chunk, n_chunks, n_tiles, s);
    else launch_binning<1>(b, k, rec, rect2, bins, w, chunk, n_chunks, n_tiles, s);
    return hipGetLastError();
}

// Static LDS of the binning kernels (their per-tile counters are dynamic).
size_t bin_static_lds_bytes() { return kBinWaves * sizeof(ExpandLds); }

template <int NW>
static hipError_t set_lds(size_t bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_chunk_count<NW>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k_scatter<NW>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t set_bin_lds_limit(size_t bytes) {
    hipError_t e = set_lds<4>(bytes);
    if (e == hipSuccess) e = set_lds<2>(bytes);
    if (e == hipSuccess) e = set_lds<1>(bytes);
    return e;
}

}  // namespace ivrgs
