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
#include <algorithm>

#include "launch.hpp"

namespace ivrgs {

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Two buffers in one launch: p[0, n) and q[0, m).
__global__ void k_fill2_u32(uint32_t *__restrict__ p, int64_t n, uint32_t *__restrict__ q, int64_t m, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n + m; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < n)
            p[i] = v;
        else
            q[i - n] = v;
    }
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
static_assert(kSegThreads == 256, "the depth sort's scans give every digit one thread");
// Keys per thread (kItems) of the depth sort's segments: 16, segments of
// 4096 keys, for large jobs; 4, segments of 1024, for jobs of at most
// kSmallSegJob records, where four times the workgroups hide more of each
// one's load and LDS latency (at a million records the longer column scans
// over the segments cost more than that gains).
constexpr int64_t kSmallSegJob = int64_t(1) << 19;
template <int kItems>
struct Seg {
    static constexpr int kSeg = kSegThreads * kItems;               // records per segment
    static constexpr int kWaveItems = kSeg / (kSegThreads / 64);   // contiguous per wave
};
int seg_items(const ivrgs_batch &b) { return b.max_job_count <= kSmallSegJob ? 4 : 16; }

int seg_rows(const ivrgs_batch &b) {
    const int seg = kSegThreads * seg_items(b);
    return (b.max_job_count + seg - 1) / seg;
}

// The key range: the AND and the OR of each job's visible depth keys (rng[j]
// and rng[n_jobs + j]; culled records carry the key ~0 and are left out).
// A digit on which they agree is the same for every visible key.  The first
// histogram pass also takes each segment's AND and OR (prng[j][segment] and
// prng[n_jobs + j][segment]); the first column scan combines them.
template <int kItems>
__device__ __forceinline__ void seg_range(const uint32_t (&v)[kItems], int n, uint32_t &a, uint32_t &o) {
    a = 0xFFFFFFFFu;
    o = 0u;
#pragma unroll
    for (int u = 0; u < kItems; ++u)
        if (u * kSegThreads + (int)threadIdx.x < n && v[u] != 0xFFFFFFFFu) {
            a &= v[u];
            o |= v[u];
        }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        a &= __shfl_xor(a, d, 64);
        o |= __shfl_xor(o, d, 64);
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

// Per (job, segment): digit histogram into hist[job][digit][segment].  The
// first pass (shift 0) runs before the key range is known: it counts every
// segment and stores the segment's part of the range.
template <int kItems>
__global__ __launch_bounds__(kSegThreads) void k_dsort_hist(ivrgs_batch b, const uint32_t *__restrict__ depth,
                                                            const uint32_t *__restrict__ key0,
                                                            const uint32_t *__restrict__ key1,
                                                            const uint32_t *__restrict__ rng, int shift,
                                                            uint32_t *__restrict__ hist, uint32_t *__restrict__ prng,
                                                            int n_seg) {
    __shared__ uint32_t h[256];
    __shared__ uint32_t sa[kSegThreads / 64], so[kSegThreads / 64];
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int64_t base = (int64_t)blockIdx.x * Seg<kItems>::kSeg;
    const bool first = shift == 0;
    if (base >= job.gauss_count || (!first && !digit_varies(rng, b.n_jobs, blockIdx.y, shift))) return;
    h[threadIdx.x] = 0;
    __syncthreads();
    const int before = first ? 0 : passes_before(rng, b.n_jobs, blockIdx.y, shift);
    const uint32_t *k = (before == 0 ? depth : ((before - 1) & 1 ? key1 : key0)) + job.rec_begin + base;
    const int n = (int)min((int64_t)Seg<kItems>::kSeg, job.gauss_count - base);
    uint32_t v[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int i = u * kSegThreads + threadIdx.x;
        v[u] = i < n ? k[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kItems; ++u)
        if (u * kSegThreads + (int)threadIdx.x < n) atomicAdd(&h[(v[u] >> shift) & 255u], 1u);
    if (first) {
        uint32_t a, o;
        seg_range<kItems>(v, n, a, o);
        if ((threadIdx.x & 63) == 0) {
            sa[threadIdx.x >> 6] = a;
            so[threadIdx.x >> 6] = o;
        }
    }
    __syncthreads();
    hist[((int64_t)blockIdx.y * 256 + threadIdx.x) * n_seg + blockIdx.x] = h[threadIdx.x];
    if (first && threadIdx.x == 0) {
        uint32_t a = sa[0], o = so[0];
        for (int w = 1; w < kSegThreads / 64; ++w) {
            a &= sa[w];
            o |= so[w];
        }
        prng[(int64_t)blockIdx.y * n_seg + blockIdx.x] = a;
        prng[((int64_t)b.n_jobs + blockIdx.y) * n_seg + blockIdx.x] = o;
    }
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
// before any is scanned, so a column pays one load latency per block.  The
// first pass combines the segments' key ranges first (every wave for
// itself; workgroup 0 of the job stores the range for the later launches).
constexpr int kColBlock = 16;
template <int kItems>
__global__ __launch_bounds__(256) void k_dsort_colscan(ivrgs_batch b, uint32_t *__restrict__ rng, int shift,
                                                       uint32_t *__restrict__ hist, uint32_t *__restrict__ tot,
                                                       const uint32_t *__restrict__ prng, int n_seg) {
    const int d = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int rows = (job.gauss_count + Seg<kItems>::kSeg - 1) / Seg<kItems>::kSeg;
    bool varies;
    if (shift == 0) {
        uint32_t a = 0xFFFFFFFFu, o = 0u;
        for (int c = lane; c < rows; c += 64) {
            a &= prng[(int64_t)blockIdx.y * n_seg + c];
            o |= prng[((int64_t)b.n_jobs + blockIdx.y) * n_seg + c];
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            a &= __shfl_xor(a, m, 64);
            o |= __shfl_xor(o, m, 64);
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            rng[blockIdx.y] = a;
            rng[b.n_jobs + blockIdx.y] = o;
        }
        varies = ((a ^ o) & 255u) != 0u;
    } else {
        varies = digit_varies(rng, b.n_jobs, blockIdx.y, shift);
    }
    if (rows == 0 || !varies) return;
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
// digit.  Wave w owns the contiguous part [w * Seg<kItems>::kWaveItems, ...)
// of the segment and ranks equal digits by lane inside each step of 64, so
// the order within a digit is the input order.  The pairs are first placed
// in LDS in the segment's digit order; the workgroup then writes them out
// in that order, so consecutive lanes store to consecutive addresses inside
// each digit's run.  A digit that is constant over the job leaves the pairs
// where they are (see passes_before).
template <int kItems>
__global__ __launch_bounds__(kSegThreads) void k_dsort_scatter(ivrgs_batch b, const uint32_t *__restrict__ depth,
                                                               uint32_t *__restrict__ key0,
                                                               uint32_t *__restrict__ val0,
                                                               uint32_t *__restrict__ key1,
                                                               uint32_t *__restrict__ val1,
                                                               const uint32_t *__restrict__ rng, int shift,
                                                               const uint32_t *__restrict__ hist,
                                                               const uint32_t *__restrict__ tot, int n_seg) {
    constexpr int kWaves = kSegThreads / 64;
    __shared__ uint32_t wh[kWaves][256];    // per wave: count, then place in the segment, per digit
    __shared__ uint32_t delta[256];         // per digit: place in the job minus place in the segment
    __shared__ uint32_t wsum[kWaves], wcnt[kWaves];
    __shared__ uint2 kv[Seg<kItems>::kSeg];  // the segment in digit order
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int64_t base = (int64_t)blockIdx.x * Seg<kItems>::kSeg;
    if (base >= job.gauss_count) return;
    const int n = (int)min((int64_t)Seg<kItems>::kSeg, job.gauss_count - base);
    const int64_t off = job.rec_begin + base;
    if (!digit_varies(rng, b.n_jobs, blockIdx.y, shift)) return;
    const int before = passes_before(rng, b.n_jobs, blockIdx.y, shift);
    const bool first = before == 0, to1 = (before & 1) != 0;
    const uint32_t *sk = first ? depth : (to1 ? key0 : key1), *sv = to1 ? val0 : val1;
    uint32_t *dk = to1 ? key1 : key0, *dv = to1 ? val1 : val0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int w0 = wave * Seg<kItems>::kWaveItems;
    // thread d: digit d's total in the job and this segment's offset inside
    // the digit (loaded together with the keys)
    const int d = threadIdx.x;
    const uint32_t t = tot[(int64_t)blockIdx.y * 256 + d];
    const uint32_t seg_off = hist[((int64_t)blockIdx.y * 256 + d) * n_seg + blockIdx.x];
    uint32_t kk[kItems], vv[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int i = w0 + u * 64 + lane;
        kk[u] = i < n ? sk[off + i] : 0u;
        vv[u] = i < n ? (first ? (uint32_t)(off + i) : sv[off + i]) : 0u;
    }
    for (int q = lane; q < 256; q += 64) wh[wave][q] = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kItems; ++u)
        if (w0 + u * 64 + lane < n) atomicAdd(&wh[wave][(kk[u] >> shift) & 255u], 1u);
    __syncthreads();
    {
        // thread d: digit d's place in the segment (scan of the segment's
        // digit counts) and in the job (scan of the digit totals, plus the
        // segment's offset), then each wave's first place
        uint32_t c[kWaves], cs = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            c[w] = wh[w][d];
            cs += c[w];
        }
        uint32_t it = t, ic = cs;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t ut = __shfl_up(it, o, 64), uc = __shfl_up(ic, o, 64);
            if (lane >= o) {
                it += ut;
                ic += uc;
            }
        }
        if (lane == 63) {
            wsum[wave] = it;
            wcnt[wave] = ic;
        }
        __syncthreads();
        uint32_t gstart = it - t + seg_off, lstart = ic - cs;
        for (int w = 0; w < wave; ++w) {
            gstart += wsum[w];
            lstart += wcnt[w];
        }
        delta[d] = gstart - lstart;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            wh[w][d] = lstart;
            lstart += c[w];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        if (w0 + u * 64 < n) {  // wave-uniform
            const bool act = w0 + u * 64 + lane < n;
            const uint32_t dg = (kk[u] >> shift) & 255u;
            const uint64_t m = match_bits<8>(dg, 8, __ballot(act));
            const uint32_t rank = lanes_below(m);
            const uint32_t pos = wh[wave][dg] + rank;
            if (act) kv[pos] = make_uint2(kk[u], vv[u]);
            if (act && rank == 0) wh[wave][dg] += (uint32_t)__popcll(m);
        }
    }
    __syncthreads();
    uint32_t *dkj = dk + job.rec_begin, *dvj = dv + job.rec_begin;
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int i = u * kSegThreads + threadIdx.x;
        if (i < n) {
            const uint2 p = kv[i];
            const uint32_t g = delta[(p.x >> shift) & 255u] + (uint32_t)i;
            dkj[g] = p.x;
            dvj[g] = p.y;
        }
    }
}

// ---------------------------------------------------------------------------
// Binning over the depth order, in two levels.
//
// Level 1 bins the records, in depth order, into blocks of 4x4 tiles (64x64
// pixels): an entry per (record, block) that the record's tile rect
// overlaps, with a 16-bit mask of the block's tiles that the record's
// ellipse reaches (the ellipse-box test of each (record, tile) item).  Each
// entry contains at least one tile of its record's rect, so there are never
// more entries than rect tiles (about 1.8 per record at 1M Gaussians,
// 800x800, against 11 tile items).  A counting pass per chunk of records
// (block overlaps only, no ellipse tests), a column scan over chunks and a
// scan over blocks give every (chunk, block) its place in the block's entry
// list; the scatter then computes the masks (one ellipse-box test per tile
// item, load-balanced over the wave) and appends the entries from per-block
// cursors, so each block's list is in (depth key, record id) order.
// Level 2 gives every tile one wave: it counts the entries of its block
// that carry its bit (the tile totals, then one scan for the list starts),
// and a second launch copies those entries' record ids in order into the
// tile's list, which one wave writes contiguously.
constexpr int kSbEdge = 4;  // tiles per block edge
constexpr int kBinWaves = 4;  // waves per binning workgroup

struct SbGeom {
    int sbx, sby, n_sb;  // blocks per row, per column, per job
};
inline SbGeom sb_geom(const Consts &k) {
    SbGeom g;
    g.sbx = (k.tiles_x + kSbEdge - 1) / kSbEdge;
    g.sby = (k.tiles_y + kSbEdge - 1) / kSbEdge;
    g.n_sb = g.sbx * g.sby;
    return g;
}

// Entry slots of one group of records in a scatter wave: at least every
// block of a job, so that any single record fits.
__host__ __device__ inline int sb_ent_cap(int n_sb) { return (n_sb > 256 ? n_sb + 63 : 256 + 63) / 64 * 64; }

// A record's fields for binning: from its 64-byte row of the projection
// (gathered through the depth order), or from the 32-byte copy the counting
// pass stored in depth order.  In depth order (order != nullptr) the counting pass gathers them
// once and stores them (kPayWrite: the rect and the fields of the
// ellipse-box test), so the scatter reads them coalesced (kPayRead).
enum { kPayNone = 0, kPayWrite = 1, kPayRead = 2 };

template <int kPay>
__device__ __forceinline__ void load_bin_record(const ivrgs_job &job, int l, const uint32_t *order, uint4 *pay,
                                                const float4 *rec4, uint32_t &r, uint2 &rc,
                                                float4 &r0, float4 &r1, float4 &r2) {
    const int64_t at = (int64_t)job.rec_begin + l;
    r = order ? order[at] : (uint32_t)at;
    if (kPay == kPayRead && order) {
        const uint4 pa = pay[2 * at], pb = pay[2 * at + 1];
        rc = make_uint2(pa.x, pa.y);
        r0 = make_float4(__uint_as_float(pa.z), __uint_as_float(pa.w), __uint_as_float(pb.x), __uint_as_float(pb.y));
        r1 = make_float4(__uint_as_float(pb.z), 0.f, 0.f, 0.f);
        r2 = make_float4(0.f, 0.f, __uint_as_float(pb.w), 0.f);
    } else {
        // one 64-byte row: the fields and, in its last float4, the rect
        const float4 r3 = rec4[kRecVec * (size_t)r + 3];
        rc = make_uint2(__float_as_uint(r3.x), __float_as_uint(r3.y));
        r0 = rec4[kRecVec * (size_t)r];
        r1 = rec4[kRecVec * (size_t)r + 1];
        r2 = rec4[kRecVec * (size_t)r + 2];
        if (kPay == kPayWrite && order) {
            pay[2 * at] = make_uint4(rc.x, rc.y, __float_as_uint(r0.x), __float_as_uint(r0.y));
            pay[2 * at + 1] = make_uint4(__float_as_uint(r0.z), __float_as_uint(r0.w), __float_as_uint(r1.x),
                                         __float_as_uint(r2.z));
        }
    }
}

// Level-1 counting: block overlaps per (job, chunk), into
// counts[job][chunk][block]; one record per thread, the workgroup's
// counters in LDS.
__global__ __launch_bounds__(kBinWaves * 64) void k_sb_count(ivrgs_batch b, SbGeom sg, const float *__restrict__ rec,
                                                             const uint32_t *__restrict__ val0,
                                                             const uint32_t *__restrict__ val1,
                                                             const uint32_t *__restrict__ rng,
                                                             uint4 *__restrict__ pay,
                                                             uint32_t *__restrict__ counts, int chunk,
                                                             int n_chunks) {
    extern __shared__ uint32_t cnt[];  // [n_sb]
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int begin = blockIdx.x * chunk;
    if (begin >= job.gauss_count) return;
    const int end = min(begin + chunk, job.gauss_count);
    for (int t = threadIdx.x; t < sg.n_sb; t += kBinWaves * 64) cnt[t] = 0;
    __syncthreads();
    const uint32_t *order = depth_order(rng, b.n_jobs, blockIdx.y, val0, val1);
    const float4 *rec4 = reinterpret_cast<const float4 *>(rec);
    for (int l = begin + (int)threadIdx.x; l < end; l += kBinWaves * 64) {
        uint32_t r;
        uint2 rc;
        float4 r0, r1, r2;
        load_bin_record<kPayWrite>(job, l, order, pay, rec4, r, rc, r0, r1, r2);
        if (rc.x | rc.y) {
            int x0, y0, x1, y1;
            unpack_rect(rc, x0, y0, x1, y1);
            const int bx0 = x0 / kSbEdge, bx1 = (x1 - 1) / kSbEdge, by0 = y0 / kSbEdge, by1 = (y1 - 1) / kSbEdge;
            for (int by = by0; by <= by1; ++by)
                for (int bx = bx0; bx <= bx1; ++bx) atomicAdd(&cnt[by * sg.sbx + bx], 1u);
        }
    }
    __syncthreads();
    uint32_t *row = counts + ((int64_t)blockIdx.y * n_chunks + blockIdx.x) * sg.n_sb;
    for (int t = threadIdx.x; t < sg.n_sb; t += kBinWaves * 64) row[t] = cnt[t];
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

// Per column (block of the job) and segment of chunks: the segment's start
// is the sum of the column's partials of the segments before it (at most 64,
// loaded together); the last segment also writes the column's total.  Then
// the counts of the segment's chunks become their exclusive starts.
__global__ __launch_bounds__(256) void k_col_apply(ivrgs_batch b, Consts k, uint32_t *__restrict__ counts, int chunk,
                                                   int n_chunks, int seg, const uint32_t *__restrict__ part,
                                                   int n_part, uint32_t *__restrict__ tile_counts) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= k.tiles_per_job) return;
    const ivrgs_job job = b.jobs[blockIdx.z];
    const int rows = (job.gauss_count + chunk - 1) / chunk;
    const int r0 = blockIdx.y * seg, r1 = min(r0 + seg, rows);
    uint32_t *col = counts + (int64_t)blockIdx.z * n_chunks * k.tiles_per_job + t;
    const uint32_t *pp = part + (int64_t)blockIdx.z * n_part * k.tiles_per_job + t;
    uint32_t run = 0;
    {
        uint32_t v[kColUnroll];
        int q = 0;
        for (; q + kColUnroll <= (int)blockIdx.y; q += kColUnroll) {
#pragma unroll
            for (int u = 0; u < kColUnroll; ++u) v[u] = pp[(int64_t)(q + u) * k.tiles_per_job];
#pragma unroll
            for (int u = 0; u < kColUnroll; ++u) run += v[u];
        }
        for (; q < (int)blockIdx.y; ++q) run += pp[(int64_t)q * k.tiles_per_job];
    }
    if ((int)blockIdx.y == n_part - 1)
        tile_counts[(int64_t)blockIdx.z * k.tiles_per_job + t] = run + pp[(int64_t)blockIdx.y * k.tiles_per_job];
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
                                                     int64_t *__restrict__ status, int64_t capacity,
                                                     const uint32_t *__restrict__ ent_total) {
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
        // the block entries did not fit: no pair was counted, and status[6]
        // holds the capacity whose workspace would hold them
        const bool ent_over = ent_total && *ent_total == 0xFFFFFFFFu;
        const bool over = ent_over || total > (uint64_t)capacity || total > 0xFFFFFFF0ull;
        starts[n_tiles] = over ? 0xFFFFFFFFu : (uint32_t)total;
        const int64_t bits = over ? (int64_t)IVRGS_DEV_E_CAPACITY : 0;
        if (ent_over) total = (uint64_t)status[6];
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

constexpr int kPart = kBinPart;

// Exclusive scan over (job, block) of the blocks' entry totals len[] padded
// to whole parts (one workgroup): start[], with the padded total in
// start[n], checked against the entry capacity (beyond it start[n] =
// 0xFFFFFFFF, the later binning kernels do nothing, and status[6] gets the
// pair capacity whose workspace holds the entries: capacity / 2 + 2 per
// record of them); and part_sb[g], the block of each part.
__global__ __launch_bounds__(1024) void k_scan_sb(const uint32_t *__restrict__ len, uint32_t *__restrict__ start,
                                                  uint32_t *__restrict__ part_sb, int64_t n, int64_t ent_cap,
                                                  int64_t n_records, int64_t *__restrict__ status) {
    __shared__ uint64_t tmp[16];
    __shared__ uint32_t first_part[1024];  // each thread's first part
    const int64_t per = (n + blockDim.x - 1) / blockDim.x;
    const int64_t lo = threadIdx.x * per, hi = min(lo + per, n);
    auto padded = [](uint32_t c) { return (uint64_t)(c + kPart - 1) / kPart * kPart; };
    uint64_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += padded(len[i]);
    uint64_t total;
    const uint64_t run0 = block_exclusive_scan_1024(sum, tmp, total);
    const bool over = total > (uint64_t)ent_cap;
    if (threadIdx.x == 0) {
        start[n] = over ? 0xFFFFFFFFu : (uint32_t)total;
        status[6] = over ? 2 * ((int64_t)total - 2 * n_records) + 1024 : 0;
    }
    uint64_t run = run0;
    for (int64_t i = lo; i < hi; ++i) {
        start[i] = (uint32_t)run;
        run += padded(len[i]);
    }
    if (over) return;
    // the block of each part, spread over the threads: the thread whose
    // blocks hold the part (the last one whose first part is at or before
    // it), then the block among that thread's
    first_part[threadIdx.x] = (uint32_t)(run0 / kPart);
    __syncthreads();
    const uint32_t n_parts = (uint32_t)(total / kPart);
    for (uint32_t g = threadIdx.x; g < n_parts; g += blockDim.x) {
        int t = 0;
        for (int step = 512; step > 0; step >>= 1)
            if (t + step < (int)blockDim.x && first_part[t + step] <= g) t += step;
        int64_t i = (int64_t)t * per;
        uint32_t p = first_part[t];
        while (p + padded(len[i]) / kPart <= g) p += (uint32_t)(padded(len[i++]) / kPart);
        part_sb[g] = (uint32_t)i;
    }
}

// The tiles of one tile row that a record's footprint reaches, as one
// interval.  The footprint E = {q(d) >= tol}, q(d) = qa dx^2 + qb dx dy +
// qc dy^2 (negative definite, log2 units) and tol the cutoff with the box
// test's margin, is convex, so the pixel centres of a row band
// Y0 <= dy <= Y1 that it reaches span one interval [L, R] in dx: the
// projection of E and the band onto x.  With det4 = 4 qa qc - qb^2 > 0 the
// extreme points of E in x are (-Xe, yL) and (Xe, -yL), Xe^2 = 4 qc tol /
// det4, yL = qb Xe / (2 qc); if the band holds yL then L = -Xe, else L is
// the smaller root in x of q(x, y) = tol at the band edge nearest yL,
// (sqrt(4 qa tol - det4 y^2) - qb y) / (2 qa), and R likewise.  The band
// and the interval are widened by (1e-4 + 2e-7 kappa) of the footprint's
// half-extent plus 0.05 pixel, kappa = 4 qa qc / det4 >= 1: several times
// the FP32 error of these formulas, which grows with kappa through det4,
// for the footprints they are used on (kappa below 1e5); any other record
// (a degenerate or extremely elongated form) reaches its whole rect row.
// The result is a superset of the tiles whose pixels can reach the cutoff,
// which is all the lists need.
struct RowIv {
    float mx, my, xe, yl;         // mean, half-extent in x (+inf: whole rows), y of the leftmost point
    float det4, a4, inv2qa, qb;   // 4 qa qc - qb^2, 4 qa tol, 1 / (2 qa), qb
    float marg;                   // widening of the band and the interval
};

__device__ __forceinline__ RowIv make_row_iv(float4 r0, float qc, float cut) {
    RowIv v;
    v.mx = r0.x;
    v.my = r0.y;
    const float qa = r0.z, qb = r0.w;
    const float tol = cut - 1.0e-3f * (1.f + fabsf(cut));
    const float det4 = 4.f * qa * qc - qb * qb;
    const float a4 = 4.f * qa * tol;
    const float xe = sqrtf(4.f * qc * tol / det4), ye = sqrtf(a4 / det4);
    const bool ok = qa < 0.f && qc < 0.f && tol < 0.f && det4 > 1.0e-5f * (4.f * qa * qc) && xe < 1.0e30f &&
                    ye < 1.0e30f;
    v.xe = ok ? xe : INFINITY;
    v.yl = ok ? qb * xe / (2.f * qc) : 0.f;
    v.det4 = ok ? det4 : 0.f;
    v.a4 = ok ? a4 : INFINITY;
    v.inv2qa = ok ? 0.5f / qa : -1.f;
    v.qb = ok ? qb : 0.f;
    const float kappa = 4.f * qa * qc / det4;  // >= 1; the FP32 error of det4 grows with it
    v.marg = ok ? fmaf(fmaf(2.0e-7f, kappa, 1.0e-4f), fmaxf(xe, ye), 0.05f) : 0.f;
    return v;
}

// Tiles [lo, hi] of tile row ty that the record reaches (lo > hi: none),
// within the rect columns [x0, x1).
__device__ __forceinline__ void row_tiles(const float4 a, const float4 c, float marg, int ty, int x0, int x1,
                                          int &lo, int &hi) {
    const float mx = a.x, my = a.y, xe = a.z, yl = a.w;
    const float det4 = c.x, a4 = c.y, inv2qa = c.z, qb = c.w;
    const float Y0 = (float)(ty * kTile) + 0.5f - my - marg, Y1 = Y0 + (float)(kTile - 1) + 2.f * marg;
    const float ya = fminf(fmaxf(yl, Y0), Y1), yb = fminf(fmaxf(-yl, Y0), Y1);
    const float da = fmaf(-det4 * ya, ya, a4), db = fmaf(-det4 * yb, yb, a4);
    const float L = ya == yl ? -xe : (sqrtf(fmaxf(da, 0.f)) - qb * ya) * inv2qa;
    const float R = yb == -yl ? xe : (-sqrtf(fmaxf(db, 0.f)) - qb * yb) * inv2qa;
    const bool meets = (da >= 0.f) & (db >= 0.f);
    // tile t holds the pixel centres [16 t + 0.5, 16 t + 15.5] - mx
    const float flo = ceilf((L - marg + mx - (float)(kTile - 1) - 0.5f) * (1.f / kTile));
    const float fhi = floorf((R + marg + mx - 0.5f) * (1.f / kTile));
    lo = (int)fmaxf(flo, (float)x0);
    hi = meets ? (int)fminf(fhi, (float)(x1 - 1)) : lo - 1;
}

// Per-wave LDS of the level-1 scatter: the records of one group (at most
// 64, in depth order) and their row-item and entry offsets.
struct SbLds {
    float4 h0[64], h1[64];  // row intervals: (mx, my, Xe, yL), (det4, 4 qa tol, 1 / (2 qa), qb)
    float marg[64];         // their widening
    uint32_t off[64];       // exclusive prefix of rect heights (row items)
    uint32_t org[64];       // rect origin, x0 | y0 << 16
    uint32_t xend[64];      // rect end column x1
    uint32_t rid[64];       // record index
    uint32_t eoff[64];      // exclusive prefix of block overlaps (entries)
    uint32_t borg[64];      // first block, bx0 | by0 << 16
    uint32_t bcol[64];      // blocks per row of the overlap
    float ibcol[64];        // 1 / bcol
    int32_t mark[64];       // record starting at each position of the current window, or -1
};

// q = t / w for t < 2^24, w >= 1, from the reciprocal iw = 1 / w corrected to
// the exact quotient (the estimate is within one of it).
__device__ __forceinline__ uint32_t div_small(uint32_t t, uint32_t w, float iw) {
    int q = (int)((float)t * iw);
    q -= (int)((uint32_t)q * w > t);
    q += (int)((uint32_t)(q + 1) * w <= t);
    return (uint32_t)q;
}

// Window over flattened items of the group: the record of each position
// (the last record starting at or before it, by a prefix maximum of the
// marks, or the one carried from the previous window).
__device__ __forceinline__ int window_record(SbLds &L, const uint32_t *off, bool starts_here, uint32_t my_off,
                                             uint32_t base, int lane, int &carry) {
    L.mark[lane] = -1;
    wave_lds_sync();
    if (starts_here && my_off >= base && my_off < base + 64u) L.mark[my_off - base] = lane;
    wave_lds_sync();
    const int pm = wave_prefix_max(L.mark[lane]);
    const int j = pm >= 0 ? pm : carry;
    carry = __builtin_amdgcn_readlane(j, 63);
    (void)off;
    return j;
}

// Level-1 scatter: one chunk per wave.  Records are taken in groups of up to
// 64 whose block overlaps fit the wave's entry slots; the group's row items
// (record, tile row of its rect) are spread evenly over the lanes (64 at a
// time, record-major), each sets the bits of the row's reached tiles
// (row_tiles) in the entries of (record, block) with LDS ORs; then the
// entries, 64 at a time in (record, block) order, are
// appended to their blocks' lists from the wave's cursors (lanes appending
// to one block hold different records, ranked by lane).  Entries are
// (record id, block | tile mask << 16).
__global__ __launch_bounds__(kBinWaves * 64) void k_sb_scatter(ivrgs_batch b, SbGeom sg,
                                                               const float *__restrict__ rec,
                                                               const uint32_t *__restrict__ val0,
                                                               const uint32_t *__restrict__ val1,
                                                               const uint32_t *__restrict__ rng,
                                                               const uint4 *__restrict__ pay,
                                                               const uint32_t *__restrict__ counts,
                                                               const uint32_t *__restrict__ sb_start,
                                                               uint2 *__restrict__ ent, int chunk, int n_chunks) {
    extern __shared__ uint32_t dyn[];  // per wave: [n_sb] cursors, then [ent_cap] masks
    __shared__ SbLds Ls[kBinWaves];
    const int n_all = b.n_jobs * sg.n_sb;
    if (sb_start[n_all] == 0xFFFFFFFFu) return;  // the entries do not fit
    const ivrgs_job job = b.jobs[blockIdx.y];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int ch = blockIdx.x * kBinWaves + wave;  // this wave's chunk
    const int cap = sb_ent_cap(sg.n_sb);
    uint32_t *cur = dyn + wave * (sg.n_sb + cap);
    uint32_t *emask = cur + sg.n_sb;
    SbLds &L = Ls[wave];
    const int qb = min(ch * chunk, job.gauss_count), qe = min(qb + chunk, job.gauss_count);
    if (qb >= qe) return;  // no barrier below: each wave works alone
    {
        const uint32_t *row = counts + ((int64_t)blockIdx.y * n_chunks + ch) * sg.n_sb;
        const uint32_t *st = sb_start + (int64_t)blockIdx.y * sg.n_sb;
        for (int t = lane; t < sg.n_sb; t += 64) cur[t] = st[t] + row[t];
    }
    const uint32_t *order = depth_order(rng, b.n_jobs, blockIdx.y, val0, val1);
    const float4 *rec4 = reinterpret_cast<const float4 *>(rec);
    const int sb_bits = __builtin_amdgcn_readfirstlane(32 - __clz(max(sg.n_sb - 1, 1)));
    int g0 = qb;
    while (g0 < qe) {
        // the group's records and their item and entry counts
        const int l = g0 + lane;
        uint32_t n_it = 0, n_en = 0;
        RowIv h = {};
        int x0 = 0, y0 = 0, x1 = 0, y1 = 0, bx0 = 0, by0 = 0, bcols = 1;
        uint32_t r = 0;
        if (l < qe) {
            uint2 rc;
            float4 r0, r1, r2;
            load_bin_record<kPayRead>(job, l, order, const_cast<uint4 *>(pay), rec4, r, rc, r0, r1, r2);
            if (rc.x | rc.y) {
                unpack_rect(rc, x0, y0, x1, y1);
                n_it = (uint32_t)(y1 - y0);
                bx0 = x0 / kSbEdge;
                by0 = y0 / kSbEdge;
                bcols = (x1 - 1) / kSbEdge - bx0 + 1;
                n_en = (uint32_t)(bcols * ((y1 - 1) / kSbEdge - by0 + 1));
                h = make_row_iv(r0, r1.x, r2.z);
            }
        }
        // the longest prefix of records whose entries fit the slots (the
        // first always does: a record overlaps at most every block)
        const uint32_t e_incl = wave_prefix_sum(n_en);
        const bool take = l < qe && e_incl <= (uint32_t)cap;
        const uint64_t tk = __ballot(take);
        const int ng = __popcll(tk);
        if (!take) n_it = n_en = 0;
        const uint32_t e_off = e_incl - n_en;
        const uint32_t n_ent = __builtin_amdgcn_readlane(e_incl, ng - 1);
        const uint32_t i_incl = wave_prefix_sum(n_it);
        const uint32_t i_off = i_incl - n_it;
        const uint32_t n_items = __builtin_amdgcn_readlane(i_incl, 63);
        wave_lds_sync();  // the previous group's tables are no longer read
        L.h0[lane] = make_float4(h.mx, h.my, h.xe, h.yl);
        L.h1[lane] = make_float4(h.det4, h.a4, h.inv2qa, h.qb);
        L.marg[lane] = h.marg;
        L.off[lane] = i_off;
        L.org[lane] = (uint32_t)x0 | ((uint32_t)y0 << 16);
        L.xend[lane] = (uint32_t)x1;
        L.rid[lane] = r;
        L.eoff[lane] = e_off;
        L.borg[lane] = (uint32_t)bx0 | ((uint32_t)by0 << 16);
        L.bcol[lane] = (uint32_t)bcols;
        L.ibcol[lane] = __builtin_amdgcn_rcpf((float)bcols);
        for (uint32_t e = lane; e < n_ent; e += 64) emask[e] = 0u;
        wave_lds_sync();
        // row items: the row's reached tiles, bits into the (record, block)
        // entries they fall in
        int carry = 0;
        for (uint32_t base = 0; base < n_items; base += 64) {
            const int j = window_record(L, L.off, n_it != 0u, i_off, base, lane, carry);
            const uint32_t idx = base + lane;
            if (idx < n_items) {
                const uint32_t o = L.org[j];
                const int ty = (int)((o >> 16) + (idx - L.off[j]));
                int lo, hi;
                row_tiles(L.h0[j], L.h1[j], L.marg[j], ty, (int)(o & 0xFFFFu), (int)L.xend[j], lo, hi);
                const uint32_t eoj = L.eoff[j], bo = L.borg[j], bc = L.bcol[j];
                const uint32_t erow = eoj + (uint32_t)(ty / kSbEdge - (int)(bo >> 16)) * bc;
                const int shift = (ty % kSbEdge) * kSbEdge;
                for (int bx = lo / kSbEdge; bx <= hi / kSbEdge && lo <= hi; ++bx) {
                    const int c0 = max(lo, bx * kSbEdge) - bx * kSbEdge, c1 = min(hi, bx * kSbEdge + 3) - bx * kSbEdge;
                    atomicOr(&emask[erow + (uint32_t)(bx - (int)(bo & 0xFFFFu))], ((2u << c1) - (1u << c0)) << shift);
                }
            }
        }
        wave_lds_sync();
        // entries, in (record, block) order, onto their blocks' lists
        carry = 0;
        for (uint32_t base = 0; base < n_ent; base += 64) {
            const int j = window_record(L, L.eoff, n_en != 0u, e_off, base, lane, carry);
            const uint32_t idx = base + lane;
            const bool act = idx < n_ent;
            uint32_t sb = 0, mask = 0, rid = 0;
            if (act) {
                const uint32_t k = idx - L.eoff[j], bc = L.bcol[j], bo = L.borg[j];
                const uint32_t ry = div_small(k, bc, L.ibcol[j]), rx = k - ry * bc;
                sb = ((bo >> 16) + ry) * (uint32_t)sg.sbx + (bo & 0xFFFFu) + rx;
                mask = emask[idx];
                rid = L.rid[j];
            }
            const uint32_t at = act ? cur[sb] : 0u;  // read ahead of the match
            const uint64_t m = match_bits<16>(sb, sb_bits, __ballot(act));
            const uint32_t rank = lanes_below(m);
            if (act) {
                ent[at + rank] = make_uint2(rid, sb | (mask << 16));
                if (rank == 0) cur[sb] = at + (uint32_t)__popcll(m);
            }
            wave_lds_sync();  // cursor updates before the next window reads them
        }
        g0 += ng;
    }
}

// The tile of bit `bit` of block `sbl` of a job, or -1 past the image.
__device__ __forceinline__ int block_tile(const Consts &k, const SbGeom &sg, int sbl, int bit) {
    const int tx = (sbl % sg.sbx) * kSbEdge + bit % kSbEdge, ty = (sbl / sg.sbx) * kSbEdge + bit / kSbEdge;
    return tx < k.tiles_x && ty < k.tiles_y ? ty * k.tiles_x + tx : -1;
}

// Level 2a, one wave per part (grid-stride over the parts): the part's
// entries per tile bit into pcnt[part][16].  Entries past the block's length
// (the padding) are not read.
__global__ __launch_bounds__(256) void k_part_count(int64_t n_all, const uint32_t *__restrict__ len,
                                                    const uint32_t *__restrict__ start,
                                                    const uint32_t *__restrict__ part_sb,
                                                    const uint2 *__restrict__ ent, uint32_t *__restrict__ pcnt) {
    const uint32_t tot = start[n_all];
    if (tot == 0xFFFFFFFFu) return;
    const int64_t n_parts = tot / kPart;
    const int lane = threadIdx.x & 63;
    for (int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); g < n_parts; g += (int64_t)gridDim.x * 4) {
        const uint32_t sb = part_sb[g];
        const uint32_t e1 = start[sb] + len[sb];
        uint32_t mask[kPart / 64];
#pragma unroll
        for (int u = 0; u < kPart / 64; ++u) {
            const uint32_t e = (uint32_t)g * kPart + u * 64 + lane;
            mask[u] = e < e1 ? ent[e].y >> 16 : 0u;
        }
        uint32_t my = 0;  // lane b < 16: the count of bit b
#pragma unroll
        for (int bit = 0; bit < 16; ++bit) {
            uint32_t c = 0;
#pragma unroll
            for (int u = 0; u < kPart / 64; ++u) c += (uint32_t)__popcll(__ballot((mask[u] >> bit) & 1u));
            if (lane == bit) my = c;
        }
        if (lane < 16) pcnt[g * 16 + lane] = my;
    }
}

// Level 2b, one wave per (job, block, tile bit): exclusive scan of the
// bit's part counts over the block's parts (in place), and the total into
// tile_count[job * tiles + tile].
__global__ __launch_bounds__(256) void k_part_scan(Consts k, SbGeom sg, int64_t n_all,
                                                   const uint32_t *__restrict__ len,
                                                   const uint32_t *__restrict__ start,
                                                   uint32_t *__restrict__ pcnt, uint32_t *__restrict__ tile_count) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= n_all * 16) return;
    const int lane = threadIdx.x & 63;
    const int64_t sb = w >> 4;
    const int bit = (int)(w & 15);
    const int job = (int)(sb / sg.n_sb), sbl = (int)(sb % sg.n_sb);
    const int tile = block_tile(k, sg, sbl, bit);
    if (tile < 0) return;
    uint32_t run = 0;
    if (start[n_all] != 0xFFFFFFFFu) {
        const int64_t g0 = start[sb] / kPart, g1 = g0 + (len[sb] + kPart - 1) / kPart;
        for (int64_t g = g0; g < g1; g += 64) {
            const int64_t gi = g + lane;
            const uint32_t c = gi < g1 ? pcnt[gi * 16 + bit] : 0u;
            const uint32_t incl = wave_prefix_sum(c);
            if (gi < g1) pcnt[gi * 16 + bit] = run + incl - c;
            run += __builtin_amdgcn_readlane(incl, 63);
        }
    }
    if (lane == 0) tile_count[(int64_t)job * k.tiles_per_job + tile] = run;
}

// Level 2c, one wave per part (grid-stride): the record ids of the part's
// entries, per tile bit in entry order, at the tile's start plus the part's
// offset (ranked by lane within each step of 64).
__global__ __launch_bounds__(256) void k_part_extract(Consts k, SbGeom sg, int64_t n_all,
                                                      const uint32_t *__restrict__ len,
                                                      const uint32_t *__restrict__ start,
                                                      const uint32_t *__restrict__ part_sb,
                                                      const uint2 *__restrict__ ent, const uint32_t *__restrict__ pcnt,
                                                      const uint32_t *__restrict__ starts, int64_t n_tiles,
                                                      uint32_t *__restrict__ sorted) {
    if (starts[n_tiles] == 0xFFFFFFFFu) return;  // capacity exceeded
    const uint32_t tot = start[n_all];
    if (tot == 0xFFFFFFFFu) return;
    const int64_t n_parts = tot / kPart;
    const int lane = threadIdx.x & 63;
    for (int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); g < n_parts; g += (int64_t)gridDim.x * 4) {
        const uint32_t sb = part_sb[g];
        const uint32_t e1 = start[sb] + len[sb];
        const int job = (int)(sb / sg.n_sb), sbl = (int)(sb % sg.n_sb);
        // lane b < 16: where bit b's ids of this part start
        uint32_t my_pos = 0;
        if (lane < 16) {
            const int tile = block_tile(k, sg, sbl, lane);
            if (tile >= 0) my_pos = starts[(int64_t)job * k.tiles_per_job + tile] + pcnt[g * 16 + lane];
        }
        uint2 v[kPart / 64];
#pragma unroll
        for (int u = 0; u < kPart / 64; ++u) {
            const uint32_t e = (uint32_t)g * kPart + u * 64 + lane;
            v[u] = e < e1 ? ent[e] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int bit = 0; bit < 16; ++bit) {
            uint32_t pos = __builtin_amdgcn_readlane(my_pos, bit);
#pragma unroll
            for (int u = 0; u < kPart / 64; ++u) {
                const bool hit = (v[u].y >> (16 + bit)) & 1u;
                const uint64_t m = __ballot(hit);
                if (hit) sorted[pos + lanes_below(m)] = v[u].x;
                pos += (uint32_t)__popcll(m);
            }
        }
    }
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

hipError_t launch_fill2_u32(uint32_t *p, int64_t n, uint32_t *q, int64_t m, uint32_t v, hipStream_t s) {
    if (n <= 0 && m <= 0) return hipSuccess;
    n = n > 0 ? n : 0;
    m = m > 0 ? m : 0;
    const int64_t want = (n + m + 255) / 256;
    const int64_t blocks = want < 4096 ? want : 4096;
    TimedScope ts(TK_FILL, s);
    hipLaunchKernelGGL(k_fill2_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, q, m, v);
    return hipGetLastError();
}

int chunk_rows(const ivrgs_batch &b, int chunk) { return (b.max_job_count + chunk - 1) / chunk; }

// Chunks per segment of the column scan: about 32, and at most 64 segments.
int col_segment(int n_chunks) {
    const int by_count = (n_chunks + 63) / 64;
    return by_count > 32 ? by_count : 32;
}

size_t col_part_words(const ivrgs_batch &b, int width, int chunk) {
    const int n_chunks = chunk_rows(b, chunk);
    const int seg = col_segment(n_chunks);
    return (size_t)b.n_jobs * ((n_chunks + seg - 1) / seg) * (size_t)width;
}

// Per job: 256 digit counts per segment, the 256 digit totals, and the
// segments' key ranges (two words each).
size_t depth_sort_hist_words(const ivrgs_batch &b) {
    return (size_t)b.n_jobs * (256 * ((size_t)seg_rows(b) + 1) + 2 * (size_t)seg_rows(b));
}

// The passes of the depth sort (the first also takes the key range; a later
// pass on a constant digit returns at once).
template <int kItems>
void launch_depth_sort(const ivrgs_batch &b, const uint32_t *depth, const BinWork &w, uint32_t *tot, int n_seg,
                       hipStream_t s) {
    uint32_t *prng = tot + (size_t)b.n_jobs * 256;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_dsort_hist<kItems>, dim3(n_seg, b.n_jobs), dim3(kSegThreads), 0, s, b, depth, w.key[0],
                           w.key[1], w.rng, shift, w.hist, prng, n_seg);
        hipLaunchKernelGGL(k_dsort_colscan<kItems>, dim3(64, b.n_jobs), dim3(256), 0, s, b, w.rng, shift, w.hist,
                           tot, prng, n_seg);
        hipLaunchKernelGGL(k_dsort_scatter<kItems>, dim3(n_seg, b.n_jobs), dim3(kSegThreads), 0, s, b, depth,
                           w.key[0], w.val[0], w.key[1], w.val[1], w.rng, shift, w.hist, tot, n_seg);
    }
}

hipError_t launch_bin_sort(const ivrgs_batch &b, const Consts &k, const float *rec, const uint32_t *rect,
                           const uint32_t *depth, const ivrgs_bins &bins, const BinWork &w, int chunk,
                           size_t bin_lds, int cus, hipStream_t s) {
    (void)bin_lds;
    (void)cus;
    const int64_t n_tiles = (int64_t)b.n_jobs * k.tiles_per_job;
    const int n_chunks = chunk_rows(b, chunk);
    const int n_seg = seg_rows(b);
    (void)rect;  // the binning reads each record's rect from its row in rec
    uint32_t *tot = w.hist + (size_t)b.n_jobs * 256 * n_seg;
    if (n_seg > 0) {
        TimedScope ts(TK_SORT, s);
        if (seg_items(b) == 4)
            launch_depth_sort<4>(b, depth, w, tot, n_seg, s);
        else
            launch_depth_sort<16>(b, depth, w, tot, n_seg, s);
    }
    const SbGeom sg = sb_geom(k);
    const int64_t n_all = (int64_t)b.n_jobs * sg.n_sb;
    {
        // level 1: block overlaps per chunk, their column scan (the
        // per-chunk places and block totals) and the scan over blocks
        TimedScope ts(TK_COUNT, s);
        if (n_chunks > 0) {
            hipLaunchKernelGGL(k_sb_count, dim3((unsigned)n_chunks, (unsigned)b.n_jobs), dim3(kBinWaves * 64),
                               sizeof(uint32_t) * (size_t)sg.n_sb, s, b, sg, rec, w.val[0], w.val[1], w.rng,
                               w.pay, w.counts, chunk, n_chunks);
            Consts kb = k;  // the column scan over blocks instead of tiles
            kb.tiles_per_job = sg.n_sb;
            const int seg = col_segment(n_chunks), n_part = (n_chunks + seg - 1) / seg;
            const unsigned tg = (unsigned)((sg.n_sb + 255) / 256);
            hipLaunchKernelGGL(k_col_sum, dim3(tg, (unsigned)n_part, (unsigned)b.n_jobs), dim3(256), 0, s, b, kb,
                               w.counts, chunk, n_chunks, seg, w.part, n_part);
            hipLaunchKernelGGL(k_col_apply, dim3(tg, (unsigned)n_part, (unsigned)b.n_jobs), dim3(256), 0, s, b, kb,
                               w.counts, chunk, n_chunks, seg, w.part, n_part, w.sb_len);
        } else {
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, w.sb_len, n_all, 0u);
        }
        hipLaunchKernelGGL(k_scan_sb, dim3(1), dim3(1024), 0, s, w.sb_len, w.sb_start, w.part_sb, n_all, w.ent_cap,
                           b.n_records, bins.status);
    }
    {
        // the block entries, then level 2: the tiles' pair totals, their
        // scan (list starts, checked against the capacity), the lists
        TimedScope ts(TK_SCATTER, s);
        if (n_chunks > 0) {
            const size_t lds = sizeof(uint32_t) * kBinWaves * (size_t)(sg.n_sb + sb_ent_cap(sg.n_sb));
            hipLaunchKernelGGL(k_sb_scatter,
                               dim3((unsigned)((n_chunks + kBinWaves - 1) / kBinWaves), (unsigned)b.n_jobs),
                               dim3(kBinWaves * 64), lds, s, b, sg, rec, w.val[0], w.val[1], w.rng, w.pay,
                               w.counts, w.sb_start, w.ent, chunk, n_chunks);
        }
        const unsigned pgrid = (unsigned)std::min<int64_t>((w.max_parts + 3) / 4, 4096);
        if (n_chunks > 0)
            hipLaunchKernelGGL(k_part_count, dim3(pgrid), dim3(256), 0, s, n_all, w.sb_len, w.sb_start, w.part_sb,
                               w.ent, w.pcnt);
        if (n_tiles > 0)
            hipLaunchKernelGGL(k_part_scan, dim3((unsigned)((n_all * 16 + 3) / 4)), dim3(256), 0, s, k, sg, n_all,
                               w.sb_len, w.sb_start, w.pcnt, bins.tile_start);
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, bins.tile_start, n_tiles, bins.status,
                           bins.capacity, w.sb_start + n_all);
        if (n_chunks > 0 && n_tiles > 0)
            hipLaunchKernelGGL(k_part_extract, dim3(pgrid), dim3(256), 0, s, k, sg, n_all, w.sb_len, w.sb_start,
                               w.part_sb, w.ent, w.pcnt, bins.tile_start, n_tiles, bins.sorted);
    }
    return hipGetLastError();
}

// Static LDS of the binning kernels (their block counters are dynamic).
size_t bin_static_lds_bytes() { return kBinWaves * sizeof(SbLds); }

// Dynamic LDS the binning needs for this job size (the scatter's per-wave
// block cursors and entry slots).
size_t bin_dyn_lds_bytes(const Consts &k) {
    const SbGeom sg = sb_geom(k);
    return sizeof(uint32_t) * kBinWaves * (size_t)(sg.n_sb + sb_ent_cap(sg.n_sb));
}

int bin_blocks_per_job(const Consts &k) { return sb_geom(k).n_sb; }

hipError_t set_bin_lds_limit(size_t bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_sb_count),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_sb_scatter), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes);
    return e;
}

}  // namespace ivrgs
