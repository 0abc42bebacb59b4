// Tile binning in depth order.
//
// 1. Depth order: each job's records are sorted by (FP32 depth key bits,
//    record id) with a segmented LSD radix sort: 8-bit digits, segments of
//    4096 records per workgroup, every pass stable, the initial order by id.
//    A digit that is constant over the job's visible records is skipped.
// 2. Count: each workgroup counts, in LDS, the pairs each tile of the job
//    receives from one chunk of consecutive records of the depth order; the
//    counts form a [job][chunk][tile] matrix (a chunk's row is contiguous).
// 3. A column scan over chunks gives every (chunk, tile) its offset inside
//    the tile's list and each tile its total; one exclusive scan over all
//    (job, tile) totals gives the list starts, and the pair total is checked
//    against the capacity on the device.
// 4. Scatter: each chunk's workgroup appends its record ids in depth order
//    from per-tile LDS cursors (one set per wave, each wave taking a quarter
//    of the chunk).  Lanes of one step that append to the same tile hold
//    different records, in depth order by lane, and are ranked by lane, so
//    each tile's list comes out in (depth key, record id) order: no per-tile
//    sort.
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

// Active lanes whose value v (bits < nbits <= kMaxBits) equals this lane's.
// Per bit: the lane's bit sign-extended to a full word x (0 or ~0) gives
// the ballot of set bits b, and the lanes that agree with this lane are
// ~b ^ x (b where the bit is set, ~b where it is clear); nbits is uniform.
template <int kMaxBits>
__device__ __forceinline__ uint64_t match_bits(uint32_t v, int nbits, uint64_t active) {
    uint32_t lo = (uint32_t)active, hi = (uint32_t)(active >> 32);
#pragma unroll
    for (int bit = 0; bit < kMaxBits; ++bit) {
        if (bit < nbits) {
            const uint32_t x = (uint32_t)__builtin_amdgcn_sbfe((int)v, bit, 1);
            const uint64_t bb = __ballot(x != 0u);
            lo &= ~(uint32_t)bb ^ x;
            hi &= ~(uint32_t)(bb >> 32) ^ x;
        }
    }
    return (uint64_t)hi << 32 | lo;
}

// Inclusive prefix maximum over the lanes of a wave, for values >= -1 (a lane
// with no source in a step takes -1): DPP shifts within each row of 16,
// then row_bcast15 / row_bcast31 carry the row maxima into the later rows.
__device__ __forceinline__ int wave_prefix_max(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x111, 0xF, 0xF, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x112, 0xF, 0xF, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x114, 0xF, 0xF, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x118, 0xF, 0xF, false));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x142, 0xA, 0xF, false));  // row_bcast15 -> rows 1, 3
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x143, 0xC, 0xF, false));  // row_bcast31 -> rows 2, 3
    return v;
}

// Inclusive prefix sum over the lanes of a wave, with the same DPP steps.
__device__ __forceinline__ uint32_t wave_prefix_sum(uint32_t u) {
    int v = (int)u;
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);
    return (uint32_t)v;
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
__global__ void k_rng_init(uint32_t *__restrict__ rng, int n_jobs) {
    for (int i = threadIdx.x; i < 2 * n_jobs; i += blockDim.x) rng[i] = i < n_jobs ? 0xFFFFFFFFu : 0u;
}

// One workgroup per segment of kSeg keys, kSegItems loads per thread issued
// together; the four waves combine in LDS so each workgroup adds one AND and
// one OR (same-address atomics serialise in L2: one pair per segment).
__global__ __launch_bounds__(kSegThreads) void k_dkey_range(ivrgs_batch b, const uint32_t *__restrict__ depth,
                                                            uint32_t *__restrict__ rng) {
    __shared__ uint32_t sa[kSegThreads / 64], so[kSegThreads / 64];
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int64_t base = (int64_t)blockIdx.x * kSeg;
    if (base >= job.gauss_count) return;
    const int n = (int)min((int64_t)kSeg, job.gauss_count - base);
    const uint32_t *z = depth + job.rec_begin + base;
    uint32_t a = 0xFFFFFFFFu, o = 0u;
    uint32_t v[kSegItems];
#pragma unroll
    for (int u = 0; u < kSegItems; ++u) {
        const int i = u * kSegThreads + threadIdx.x;
        v[u] = i < n ? z[i] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int u = 0; u < kSegItems; ++u)
        if (v[u] != 0xFFFFFFFFu) {
            a &= v[u];
            o |= v[u];
        }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        a &= __shfl_xor(a, d, 64);
        o |= __shfl_xor(o, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sa[threadIdx.x >> 6] = a;
        so[threadIdx.x >> 6] = o;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kSegThreads / 64; ++w) {
            a &= sa[w];
            o |= so[w];
        }
        if (a != 0xFFFFFFFFu) atomicAnd(&rng[blockIdx.y], a);
        if (o != 0u) atomicOr(&rng[b.n_jobs + blockIdx.y], o);
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
    uint32_t v[kSegItems];
#pragma unroll
    for (int u = 0; u < kSegItems; ++u) {
        const int i = u * kSegThreads + threadIdx.x;
        v[u] = i < n ? k[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kSegItems; ++u)
        if (u * kSegThreads + (int)threadIdx.x < n) atomicAdd(&h[(v[u] >> shift) & 255u], 1u);
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
// tot[job][digit].  The counts of up to kColBlock x 64 segments are loaded
// before any is scanned, so a column pays one load latency per block.
constexpr int kColBlock = 16;
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
    for (int base = 0; base < rows; base += 64 * kColBlock) {
        uint32_t v[kColBlock];
#pragma unroll
        for (int u = 0; u < kColBlock; ++u) {
            const int c = base + u * 64 + lane;
            v[u] = c < rows ? col[c] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kColBlock; ++u) {
            if (base + u * 64 >= rows) break;  // wave-uniform
            const uint32_t incl = wave_prefix_sum(v[u]);
            const int c = base + u * 64 + lane;
            if (c < rows) col[c] = carry + incl - v[u];
            carry += __builtin_amdgcn_readlane(incl, 63);
        }
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
            const uint64_t m = match_bits<8>(dg, 8, __ballot(act));
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
// Visits every (record, tile) pair of the range [begin, end) of a job's depth
// order whose tile the record's ellipse reaches, in depth order.  The work of
// 64 consecutive records is spread evenly over the lanes: the lanes scan the
// records' rect areas, then take the flattened (record, tile) items 64 at a
// time (record-major, so in depth order).  Each record that starts inside
// the current window of 64 items marks its first position in LDS; an item's
// record is the last mark at or before it (a ballot finds its position), or
// the record still running from the previous window.  f(record, tile x,
// tile y) is called by the lanes of a hit, all lanes of one step together.
struct ExpandLds {
    float4 h0[64], h1[64];  // hit tests of the step's records
    uint32_t off[64];       // exclusive prefix of rect areas
    uint32_t org[64];       // rect origin, x0 | y0 << 16
    uint32_t wid[64];       // rect width in tiles
    float iwid[64];         // 1 / wid
    uint32_t rid[64];       // record index
    int32_t mark[64];       // record starting at each position of the current item window, or -1
};
constexpr int kBinWaves = 4;  // waves per binning workgroup (sharing one chunk)

// Groups of 64 records start at begin, begin + stride, ... (stride 64: the
// whole range in order; stride 64 * waves: the waves of a workgroup share it).
// In depth order (order != nullptr) the records' binning fields are
// gathered once, by the counting pass, which also stores them in depth order
// (kPayWrite: 32 bytes per record, its rect and the fields of the ellipse-box
// test), so the scatter reads them coalesced beside the ids (kPayRead).
enum { kPayNone = 0, kPayWrite = 1, kPayRead = 2 };

template <int kPay, typename F>
__device__ __forceinline__ void for_each_pair(const ivrgs_job &job, int begin, int end, int stride,
                                              const uint32_t *order, uint4 *pay, const float4 *rec4,
                                              const uint2 *rect, ExpandLds &L, F &&f) {
    const int lane = threadIdx.x & 63;
    for (int g0 = begin; g0 < end; g0 += stride) {
        const int l = g0 + lane;
        uint32_t n = 0;
        if (l < end) {
            const int64_t at = (int64_t)job.rec_begin + l;
            const int64_t r = order ? (int64_t)order[at] : at;
            uint2 rc;
            float4 r0, r1, r2;
            if (kPay == kPayRead && order) {
                const uint4 pa = pay[2 * at], pb = pay[2 * at + 1];
                rc = make_uint2(pa.x, pa.y);
                r0 = make_float4(__uint_as_float(pa.z), __uint_as_float(pa.w), __uint_as_float(pb.x),
                                 __uint_as_float(pb.y));
                r1 = make_float4(__uint_as_float(pb.z), 0.f, 0.f, 0.f);
                r2 = make_float4(0.f, 0.f, __uint_as_float(pb.w), 0.f);
            } else {
                rc = rect[r];
                r0 = rec4[3 * r];
                r1 = rec4[3 * r + 1];
                r2 = rec4[3 * r + 2];
                if (kPay == kPayWrite && order) {
                    pay[2 * at] = make_uint4(rc.x, rc.y, __float_as_uint(r0.x), __float_as_uint(r0.y));
                    pay[2 * at + 1] = make_uint4(__float_as_uint(r0.z), __float_as_uint(r0.w), __float_as_uint(r1.x),
                                                 __float_as_uint(r2.z));
                }
            }
            if (rc.x | rc.y) {
                int x0, y0, x1, y1;
                unpack_rect(rc, x0, y0, x1, y1);
                n = (uint32_t)((x1 - x0) * (y1 - y0));
                const HitTest h = make_hit_test(r0, r1, r2);
                L.h0[lane] = make_float4(h.mx, h.my, h.qa, h.qb);
                L.h1[lane] = make_float4(h.qc, h.i2qa, h.i2qc, h.tol);
                L.org[lane] = rc.x;
                L.wid[lane] = (uint32_t)(x1 - x0);
                L.iwid[lane] = __builtin_amdgcn_rcpf((float)(x1 - x0));
                L.rid[lane] = (uint32_t)r;
            }
        }
        const uint32_t incl = wave_prefix_sum(n);
        const uint32_t my_off = incl - n;
        L.off[lane] = my_off;
        const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
        int carry = 0;  // record covering the first item of the window
        for (uint32_t base = 0; base < total; base += 64) {
            L.mark[lane] = -1;
            wave_lds_sync();
            if (n != 0u && my_off >= base && my_off < base + 64u) L.mark[my_off - base] = lane;
            wave_lds_sync();
            // marks rise with the position, so the last one at or before
            // this item is the prefix maximum
            const int pm = wave_prefix_max(L.mark[lane]);
            const int j = pm >= 0 ? pm : carry;
            carry = __builtin_amdgcn_readlane(j, 63);
            const uint32_t idx = base + lane;
            if (idx < total) {
                // every field of the item's record in one LDS round trip
                const uint32_t offj = L.off[j], w = L.wid[j], o = L.org[j], rid = L.rid[j];
                const float iw = L.iwid[j];
                const float4 a = L.h0[j], c = L.h1[j];
                asm volatile("" ::"v"(offj), "v"(w), "v"(o), "v"(rid), "v"(iw), "v"(a.x), "v"(a.y), "v"(a.z),
                             "v"(a.w), "v"(c.x), "v"(c.y), "v"(c.z), "v"(c.w));
                const uint32_t t = idx - offj;
                // t / w from the reciprocal, corrected to the exact value:
                // t is below the tiles of one job (at most 2^16, as the
                // per-tile LDS counters require), where the estimate is
                // within one of the quotient
                int q = (int)((float)t * iw);
                q -= (int)((uint32_t)q * w > t);
                q += (int)((uint32_t)(q + 1) * w <= t);
                const uint32_t dy = (uint32_t)q, dx = t - dy * w;
                const int x = (int)((o & 0xFFFFu) + dx), y = (int)((o >> 16) + dy);
                const HitTest h = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
                if (box_hit(h, x * kTile, y * kTile, kTile, kTile)) f(rid, x, y);
            }
        }
        wave_lds_sync();  // every lane is done with the tables before they are rewritten
    }
}

// Pairs per tile from each (job, chunk), into counts[job][chunk][tile].  The
// four waves of a workgroup share the chunk (the order of counting does not
// matter) and one set of LDS counters.
__global__ __launch_bounds__(kBinWaves * 64) void k_chunk_count(ivrgs_batch b, Consts k, const float *__restrict__ rec,
                                                                const uint2 *__restrict__ rect,
                                                                const uint32_t *__restrict__ val0,
                                                                const uint32_t *__restrict__ val1,
                                                                const uint32_t *__restrict__ rng,
                                                                uint4 *__restrict__ pay,
                                                                uint32_t *__restrict__ counts, int chunk,
                                                                int n_chunks) {
    extern __shared__ uint32_t cnt[];  // [tiles]
    __shared__ ExpandLds L[kBinWaves];
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int begin = blockIdx.x * chunk;
    if (begin >= job.gauss_count) return;
    const int end = min(begin + chunk, job.gauss_count);
    const int tpj = k.tiles_per_job, tx_n = k.tiles_x;
    const int wave = threadIdx.x >> 6;
    for (int t = threadIdx.x; t < tpj; t += kBinWaves * 64) cnt[t] = 0;
    __syncthreads();
    const uint32_t *order = depth_order(rng, b.n_jobs, blockIdx.y, val0, val1);
    for_each_pair<kPayWrite>(job, begin + wave * 64, end, kBinWaves * 64, order, pay, reinterpret_cast<const float4 *>(rec), rect,
                  L[wave], [&](uint32_t, int x, int y) { atomicAdd(&cnt[y * tx_n + x], 1u); });
    __syncthreads();
    uint32_t *row = counts + ((int64_t)blockIdx.y * n_chunks + blockIdx.x) * tpj;
    for (int t = threadIdx.x; t < tpj; t += kBinWaves * 64) row[t] = cnt[t];
}

// Exclusive scan of every tile's counts down the chunks (a column of the
// [chunk][tile] matrix), in place, in three steps over segments of `seg`
// chunks so that the column reads stay coalesced across tiles: the sum of
// each segment, the scan of the segment sums (giving the tile totals), and
// the segment-local scan from the segment's start.  Thread = tile.
constexpr int kColUnroll = 8;

__global__ __launch_bounds__(256) void k_col_sum(ivrgs_batch b, Consts k, const uint32_t *__restrict__ counts,
                                                 int chunk, int n_chunks, int seg, uint32_t *__restrict__ part,
                                                 int n_part) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= k.tiles_per_job) return;
    const ivrgs_job job = b.jobs[blockIdx.z];
    const int rows = (job.gauss_count + chunk - 1) / chunk;
    const int r0 = blockIdx.y * seg, r1 = min(r0 + seg, rows);
    const uint32_t *col = counts + (int64_t)blockIdx.z * n_chunks * k.tiles_per_job + t;
    uint32_t sum = 0;
    int r = r0;
    for (; r + kColUnroll <= r1; r += kColUnroll) {
        uint32_t v[kColUnroll];
#pragma unroll
        for (int u = 0; u < kColUnroll; ++u) v[u] = col[(int64_t)(r + u) * k.tiles_per_job];
#pragma unroll
        for (int u = 0; u < kColUnroll; ++u) sum += v[u];
    }
    for (; r < r1; ++r) sum += col[(int64_t)r * k.tiles_per_job];
    part[((int64_t)blockIdx.z * n_part + blockIdx.y) * k.tiles_per_job + t] = sum;
}

constexpr int kPartUnroll = 16;

__global__ __launch_bounds__(256) void k_col_part_scan(ivrgs_batch b, Consts k, uint32_t *__restrict__ part,
                                                       int n_part, uint32_t *__restrict__ tile_counts) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= k.tiles_per_job) return;
    uint32_t *p = part + (int64_t)blockIdx.y * n_part * k.tiles_per_job + t;
    uint32_t run = 0;
    int i = 0;
    // loads issued kPartUnroll at a time: one memory round trip per batch
    for (; i + kPartUnroll <= n_part; i += kPartUnroll) {
        uint32_t v[kPartUnroll];
#pragma unroll
        for (int u = 0; u < kPartUnroll; ++u) v[u] = p[(int64_t)(i + u) * k.tiles_per_job];
#pragma unroll
        for (int u = 0; u < kPartUnroll; ++u) {
            p[(int64_t)(i + u) * k.tiles_per_job] = run;
            run += v[u];
        }
    }
    for (; i < n_part; ++i) {
        const uint32_t v = p[(int64_t)i * k.tiles_per_job];
        p[(int64_t)i * k.tiles_per_job] = run;
        run += v;
    }
    tile_counts[(int64_t)blockIdx.y * k.tiles_per_job + t] = run;
}

__global__ __launch_bounds__(256) void k_col_apply(ivrgs_batch b, Consts k, uint32_t *__restrict__ counts, int chunk,
                                                   int n_chunks, int seg, const uint32_t *__restrict__ part,
                                                   int n_part) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= k.tiles_per_job) return;
    const ivrgs_job job = b.jobs[blockIdx.z];
    const int rows = (job.gauss_count + chunk - 1) / chunk;
    const int r0 = blockIdx.y * seg, r1 = min(r0 + seg, rows);
    uint32_t *col = counts + (int64_t)blockIdx.z * n_chunks * k.tiles_per_job + t;
    uint32_t run = part[((int64_t)blockIdx.z * n_part + blockIdx.y) * k.tiles_per_job + t];
    int r = r0;
    for (; r + kColUnroll <= r1; r += kColUnroll) {
        uint32_t v[kColUnroll];
#pragma unroll
        for (int u = 0; u < kColUnroll; ++u) v[u] = col[(int64_t)(r + u) * k.tiles_per_job];
#pragma unroll
        for (int u = 0; u < kColUnroll; ++u) {
            col[(int64_t)(r + u) * k.tiles_per_job] = run;
            run += v[u];
        }
    }
    for (; r < r1; ++r) {
        const uint32_t v = col[(int64_t)r * k.tiles_per_job];
        col[(int64_t)r * k.tiles_per_job] = run;
        run += v;
    }
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
        const int64_t bits = over ? (int64_t)IVRGS_DEV_E_CAPACITY : 0;
        status[0] = (int64_t)total;
        status[1] = bits;
        status[2] = 0;
        status[3] = 0;
        // sticky until ivrgs_get_error reads them: the bits of every sort
        // since, and the largest requirement
        status[4] |= bits;
        status[5] = max(status[5], (int64_t)total);
    }
}

// Appends each chunk's record ids in depth order.  Two shapes:
//  - kSplit: one chunk per workgroup; wave w takes the w-th part of the chunk
//    (whole groups of 64 records), first counts its own pairs per tile, and
//    the waves' per-tile cursors start at the tile's list start plus the
//    chunk's column prefix plus the counts of the earlier parts.  Four times
//    the parallelism for an extra counting pass: for few chunks.
//  - otherwise: NW consecutive chunks per workgroup, one per wave, each
//    cursor at the tile's list start plus the chunk's column prefix.
// Each wave appends its records in order.  No global atomics.
template <int NW, bool kSplit>
__global__ __launch_bounds__(NW * 64) void k_scatter(ivrgs_batch b, Consts k, const float *__restrict__ rec,
                                                     const uint2 *__restrict__ rect,
                                                     const uint32_t *__restrict__ val0,
                                                     const uint32_t *__restrict__ val1,
                                                     const uint32_t *__restrict__ rng,
                                                     uint4 *__restrict__ pay,
                                                     const uint32_t *__restrict__ counts,
                                                     uint32_t *__restrict__ sorted, int chunk, int n_chunks,
                                                     const uint32_t *__restrict__ starts, int64_t n_tiles,
                                                     int whole_min) {
    extern __shared__ uint32_t cur[];  // [NW][tiles]: counts, then cursors
    __shared__ ExpandLds L[NW];
    if (starts[n_tiles] == 0xFFFFFFFFu) return;  // capacity exceeded
    const ivrgs_job job = b.jobs[blockIdx.y];
    // Both shapes are launched; the job's record count on the device picks
    // the one that works: whole chunks per wave once there are at least
    // whole_min such workgroups over the batch (estimated from this job).
    const int rows = (job.gauss_count + chunk - 1) / chunk;
    const bool whole = NW == 1 || (int64_t)(rows + NW - 1) / NW * b.n_jobs >= whole_min;
    if (whole == kSplit) return;
    const int begin = blockIdx.x * (kSplit ? 1 : NW) * chunk;
    if (begin >= job.gauss_count) return;
    const int end = min(begin + chunk, job.gauss_count);
    const int tpj = k.tiles_per_job, tx_n = k.tiles_x;
    const int tile_bits = __builtin_amdgcn_readfirstlane(32 - __clz(max(tpj - 1, 1)));
    const int wave = threadIdx.x >> 6;
    const uint32_t *order = depth_order(rng, b.n_jobs, blockIdx.y, val0, val1);
    const float4 *rec4 = reinterpret_cast<const float4 *>(rec);
    uint32_t *c = cur + wave * tpj;
    const uint32_t *st = starts + (int64_t)blockIdx.y * tpj;
    int qb, qe;
    if (kSplit) {
        const int part = (chunk / 64 + NW - 1) / NW * 64;
        qb = min(begin + wave * part, end);
        qe = min(qb + part, end);
        for (int t = threadIdx.x; t < NW * tpj; t += NW * 64) cur[t] = 0;
        __syncthreads();
        for_each_pair<kPayRead>(job, qb, qe, 64, order, pay, rec4, rect, L[wave],
                      [&](uint32_t, int x, int y) { atomicAdd(&c[y * tx_n + x], 1u); });
        __syncthreads();
        const uint32_t *row = counts + ((int64_t)blockIdx.y * n_chunks + blockIdx.x) * tpj;
        for (int t = threadIdx.x; t < tpj; t += NW * 64) {
            uint32_t run = st[t] + row[t];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint32_t n = cur[w * tpj + t];
                cur[w * tpj + t] = run;
                run += n;
            }
        }
    } else {
        const int ch = blockIdx.x * NW + wave;  // this wave's chunk
        qb = min(ch * chunk, job.gauss_count);
        qe = min(qb + chunk, job.gauss_count);
        const uint32_t *row = counts + ((int64_t)blockIdx.y * n_chunks + blockIdx.x * NW) * tpj;
        for (int t = threadIdx.x; t < tpj; t += NW * 64) {
            const uint32_t s0 = st[t];
#pragma unroll
            for (int w = 0; w < NW; ++w)
                if (blockIdx.x * NW + w < n_chunks) cur[w * tpj + t] = s0 + row[(int64_t)w * tpj + t];
        }
    }
    __syncthreads();
    for_each_pair<kPayRead>(job, qb, qe, 64, order, pay, rec4, rect, L[wave], [&](uint32_t r, int x, int y) {
        const uint32_t t = (uint32_t)(y * tx_n + x);
        const uint32_t at = c[t];  // read ahead of the match, which hides its latency
        const uint64_t m = match_bits<16>(t, tile_bits, __ballot(true));
        const uint32_t rank = lanes_below(m);
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

int chunk_rows(const ivrgs_batch &b, int chunk) { return (b.max_job_count + chunk - 1) / chunk; }

// Chunks per segment of the column scan: about 32, and at most 64 segments.
int col_segment(int n_chunks) {
    const int by_count = (n_chunks + 63) / 64;
    return by_count > 32 ? by_count : 32;
}

size_t col_part_words(const ivrgs_batch &b, const Consts &k, int chunk) {
    const int n_chunks = chunk_rows(b, chunk);
    const int seg = col_segment(n_chunks);
    return (size_t)b.n_jobs * ((n_chunks + seg - 1) / seg) * (size_t)k.tiles_per_job;
}

size_t depth_sort_hist_words(const ivrgs_batch &b) { return (size_t)b.n_jobs * 256 * ((size_t)seg_rows(b) + 1); }

template <int NW>
static void launch_scatter(const ivrgs_batch &b, const Consts &k, const float *rec, const uint2 *rect2,
                           const ivrgs_bins &bins, const BinWork &w, int chunk, int n_chunks, int64_t n_tiles,
                           int cus, hipStream_t s) {
    const size_t lds = sizeof(uint32_t) * NW * (size_t)k.tiles_per_job;
    // the shape is chosen on the device from the job's record count (a
    // culled job may hold far fewer records than the host's bound), so both
    // are launched unless even the bound is too small for whole chunks
    const int whole_min = cus;
    const int64_t whole_bound = (int64_t)(n_chunks + NW - 1) / NW * b.n_jobs;
    if (NW > 1)
        hipLaunchKernelGGL((k_scatter<NW, true>), dim3((unsigned)n_chunks, (unsigned)b.n_jobs), dim3(NW * 64), lds, s,
                           b, k, rec, rect2, w.val[0], w.val[1], w.rng, w.pay, w.counts, bins.sorted, chunk,
                           n_chunks, bins.tile_start, n_tiles, whole_min);
    if (NW == 1 || whole_bound >= whole_min)
        hipLaunchKernelGGL((k_scatter<NW, false>), dim3((unsigned)((n_chunks + NW - 1) / NW), (unsigned)b.n_jobs),
                           dim3(NW * 64), lds, s, b, k, rec, rect2, w.val[0], w.val[1], w.rng, w.pay, w.counts,
                           bins.sorted, chunk, n_chunks, bins.tile_start, n_tiles, whole_min);
}

hipError_t launch_bin_sort(const ivrgs_batch &b, const Consts &k, const float *rec, const uint32_t *rect,
                           const uint32_t *depth, const ivrgs_bins &bins, const BinWork &w, int chunk,
                           size_t bin_lds, int cus, hipStream_t s) {
    const int64_t n_tiles = (int64_t)b.n_jobs * k.tiles_per_job;
    const int n_chunks = chunk_rows(b, chunk);
    const int n_seg = seg_rows(b);
    const uint2 *rect2 = reinterpret_cast<const uint2 *>(rect);
    uint32_t *tot = w.hist + (size_t)b.n_jobs * 256 * n_seg;
    if (n_seg > 0) {
        TimedScope ts(TK_SORT, s);
        hipLaunchKernelGGL(k_rng_init, dim3(1), dim3(256), 0, s, w.rng, b.n_jobs);
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
    {
        TimedScope ts(TK_COUNT, s);
        if (n_chunks > 0) {
            hipLaunchKernelGGL(k_chunk_count, dim3((unsigned)n_chunks, (unsigned)b.n_jobs), dim3(kBinWaves * 64),
                               sizeof(uint32_t) * (size_t)k.tiles_per_job, s, b, k, rec, rect2, w.val[0], w.val[1],
                               w.rng, w.pay, w.counts, chunk, n_chunks);
            const int seg = col_segment(n_chunks), n_part = (n_chunks + seg - 1) / seg;
            const unsigned tg = (unsigned)((k.tiles_per_job + 255) / 256);
            hipLaunchKernelGGL(k_col_sum, dim3(tg, (unsigned)n_part, (unsigned)b.n_jobs), dim3(256), 0, s, b, k,
                               w.counts, chunk, n_chunks, seg, w.part, n_part);
            hipLaunchKernelGGL(k_col_part_scan, dim3(tg, (unsigned)b.n_jobs), dim3(256), 0, s, b, k, w.part, n_part,
                               bins.tile_start);
            hipLaunchKernelGGL(k_col_apply, dim3(tg, (unsigned)n_part, (unsigned)b.n_jobs), dim3(256), 0, s, b, k,
                               w.counts, chunk, n_chunks, seg, w.part, n_part);
        } else if (n_tiles > 0) {
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, bins.tile_start, n_tiles, 0u);
        }
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, bins.tile_start, n_tiles, bins.status,
                           bins.capacity);
    }
    if (n_chunks == 0) return hipGetLastError();
    // as many waves per chunk as the per-wave tile counters allow
    TimedScope ts(TK_SCATTER, s);
    const size_t per_wave = sizeof(uint32_t) * (size_t)k.tiles_per_job;
    if (4 * per_wave <= bin_lds) launch_scatter<4>(b, k, rec, rect2, bins, w, chunk, n_chunks, n_tiles, cus, s);
    else if (2 * per_wave <= bin_lds) launch_scatter<2>(b, k, rec, rect2, bins, w, chunk, n_chunks, n_tiles, cus, s);
    else launch_scatter<1>(b, k, rec, rect2, bins, w, chunk, n_chunks, n_tiles, cus, s);
    return hipGetLastError();
}

// Static LDS of the binning kernels (their per-tile counters are dynamic).
size_t bin_static_lds_bytes() { return kBinWaves * sizeof(ExpandLds); }

template <int NW>
static hipError_t set_scatter_lds(size_t bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_scatter<NW, true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k_scatter<NW, false>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t set_bin_lds_limit(size_t bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_chunk_count),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) e = set_scatter_lds<4>(bytes);
    if (e == hipSuccess) e = set_scatter_lds<2>(bytes);
    if (e == hipSuccess) e = set_scatter_lds<1>(bytes);
    return e;
}

}  // namespace ivrgs
