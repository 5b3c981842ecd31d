// Binning: visible records -> (bin, depth, record)-ordered pair list and
// per-bin ranges (the front-to-back order of the Sec. 3.4 rasteriser).  A bin
// is a rectangle of pixels (a multiple of the compositing tile); each
// compositing tile reads its bin's list.
//
// Two-stage design instead of one 64-bit-key sort of all pairs:
//   1. compact the visible records and sort them by the bit pattern of their
//      positive FP32 depth (stable LSD radix sort, so equal depths keep
//      ascending record order);
//   2. emit one pair (global bin id, record) per touched bin in that depth
//      order and sort the pairs stably by bin id only (ceil(log2 bins)
//      bits).  Stability makes the result the (bin, depth, record) order.
// Stage 1 sorts records (millions), stage 2 sorts only 8-18 key bits of the
// pairs, instead of ~50 bits.
//
// Kernel launches, not bandwidth, dominate binning at these sizes (about
// 4.5 us per small kernel), so the short scans (per-chunk sums of visible
// records and of pairs, radix histograms) are chained across workgroups
// (decoupled look-back): each workgroup publishes its tile's total, then
// reads its predecessors' totals or running prefixes, so one launch does what
// a reduce / scan / down-sweep triple does.  A workgroup takes its tile index
// in arrival order, so every tile it waits for belongs to a workgroup that is
// already running, and every wait is bounded.  The long passes (compaction,
// pair emission) rank within 2048-record chunks and take the chunk offsets
// from such a scan; chaining them directly measured slower (every status
// poll crosses the XCDs).
//
// The compaction also writes each visible record's (record, bin count, rect)
// into a dense array at its compaction slot, and the depth sort carries the
// slot, so the pair kernels read that small array instead of gathering from
// the record lines.  Radix blocks take contiguous ranges of the keys, at most
// 512 of them, so the histogram table does not grow with the key bound.
//
// All kernels read element counts from the device (scalars block), so the
// whole sequence needs no host synchronisation; grids are sized from host
// upper bounds.
#include <algorithm>
#include <type_traits>

#include "gs_device.h"

namespace gs {

namespace {

// ------------------------------------------------------------------ fills
__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_f32_kernel(float* p, float v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

inline int fill_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

// ------------------------------------------------------------------ scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

struct LoadBits {   // 1 if padded record i is visible (the projection's bitmap)
    const uint64_t* vis;
    int64_t words;
    __device__ uint32_t operator()(int64_t i) const {
        return (i >> 6) < words ? (uint32_t)((vis[i >> 6] >> (i & 63)) & 1ull) : 0u;
    }
};
struct LoadArr {
    const uint32_t* a;
    int64_t n;
    __device__ uint32_t operator()(int64_t i) const { return i < n ? a[i] : 0u; }
};

// a[base .. base + N) into v, zeros past n.  Every array read this way is a
// workspace array (256-byte aligned) and base is a multiple of N (N a
// multiple of 4), so a full group is N / 4 16-byte loads.
template <int N>
__device__ __forceinline__ void loadN(const uint32_t* a, int64_t base, int64_t n, uint32_t (&v)[N]) {
    static_assert(N % 4 == 0, "whole 16-byte loads");
    if (base + N <= n) {
#pragma unroll
        for (int i = 0; i < N / 4; i++) {
            const uint4 x = *reinterpret_cast<const uint4*>(a + base + 4 * i);
            v[4 * i] = x.x; v[4 * i + 1] = x.y; v[4 * i + 2] = x.z; v[4 * i + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < N; k++) v[k] = base + k < n ? a[base + k] : 0u;
    }
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// exclusive scan of one value per thread over the block; returns the block total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t& excl) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan(x, lane);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / 64; i++) {
        const uint32_t s = wsum[i];
        if (i < w) off += s;
        tot += s;
    }
    excl = off + incl - x;
    __syncthreads();
    return tot;
}

template <class Ld>
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(Ld ld, int64_t n, uint32_t* bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
    if constexpr (std::is_same<Ld, LoadBits>::value) {
        // eight records per thread: one byte of a visibility word
        static_assert(kScanItems == 8, "a byte of bits per thread");
        const int64_t wi = base >> 6;
        const uint64_t wd = wi < ld.words ? ld.vis[wi] : 0ull;
        s = (uint32_t)__popc((uint32_t)(wd >> (base & 63)) & 0xffu);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; k++)
            if (base + k < n) s += ld(base + k);
    }
    uint32_t ex;
    const uint32_t tot = block_excl_scan(s, ex);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// single block: exclusive scan of a[0..n) in place, in chunks; writes the
// 64-bit total to total64[0..1] (lo, hi) and, if total32 != null, the u32 total
__global__ __launch_bounds__(kScanThreads) void scan_single_kernel(uint32_t* a, int64_t n, uint32_t* total64,
                                                                   uint32_t* total32) {
    __shared__ uint64_t carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int64_t c = 0; c < n; c += kScanTile) {
        const int64_t base = c + (int64_t)threadIdx.x * kScanItems;
        uint32_t v[kScanItems];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; k++) {
            v[k] = (base + k < n) ? a[base + k] : 0u;
            s += v[k];
        }
        uint32_t ex;
        const uint32_t tot = block_excl_scan(s, ex);
        const uint64_t carry = carry_s;
        uint32_t run = (uint32_t)carry + ex;
#pragma unroll
        for (int k = 0; k < kScanItems; k++) {
            if (base + k < n) a[base + k] = run;
            run += v[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (total64) {
            total64[0] = (uint32_t)(carry_s & 0xffffffffu);
            total64[1] = (uint32_t)(carry_s >> 32);
        }
        if (total32) total32[0] = (uint32_t)carry_s;
    }
}

template <class Ld>
__global__ __launch_bounds__(kScanThreads) void scan_down_kernel(Ld ld, int64_t n, const uint32_t* boff, uint32_t* out) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        v[k] = (base + k < n) ? ld(base + k) : 0u;
        s += v[k];
    }
    uint32_t ex;
    block_excl_scan(s, ex);
    uint32_t run = boff[blockIdx.x] + ex;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

// exclusive scan of ld(0..n) into out; bsum needs ceil(n / kScanTile) entries
template <class Ld>
hipError_t device_scan(Ld ld, int64_t n, uint32_t* out, uint32_t* bsum, uint32_t* total64, uint32_t* total32,
                       hipStream_t s) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        scan_single_kernel<<<1, kScanThreads, 0, s>>>(bsum, 0, total64, total32);
        return hipGetLastError();
    }
    scan_reduce_kernel<Ld><<<(unsigned)nb, kScanThreads, 0, s>>>(ld, n, bsum);
    scan_single_kernel<<<1, kScanThreads, 0, s>>>(bsum, nb, total64, total32);
    scan_down_kernel<Ld><<<(unsigned)nb, kScanThreads, 0, s>>>(ld, n, bsum, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ chained scans
// Tile status word: bits 62-63 the state (0 not yet published, 1 the tile's
// own total, 2 the running total through this tile), bits 0-61 the value.
constexpr uint64_t kLbAgg = 1ull << 62, kLbPrefix = 2ull << 62, kLbValue = (1ull << 62) - 1ull;
// about 4 s of polling before a workgroup gives up (flagging kFlagLookback)
constexpr uint32_t kLbMaxPolls = 1u << 22;

// The value travels inside the status word, so relaxed device-scope atomics
// suffice: no other memory is published through it (acquire / release here
// would write back and invalidate the XCD's L2 on every poll).
__device__ __forceinline__ uint64_t lb_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lb_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// this workgroup's tile, in arrival order
__device__ __forceinline__ uint32_t lb_tile(uint32_t* counter) {
    __shared__ uint32_t s_t;
    if (threadIdx.x == 0) s_t = atomicAdd(counter, 1u);
    __syncthreads();
    return s_t;
}

// Exclusive prefix of `agg` (this tile's total) over the tiles before it.
// Called by every thread; wavefront 0 publishes and looks back 64 tiles at a
// time, summing back to the nearest running total.
__device__ uint64_t lb_exclusive(uint64_t* status, uint32_t tile, uint64_t agg, uint32_t* flags) {
    __shared__ uint64_t s_excl;
    if (threadIdx.x < 64) {
        const int lane = (int)threadIdx.x;
        if (lane == 0) lb_store(&status[tile], (tile == 0 ? kLbPrefix : kLbAgg) | agg);
        uint64_t excl = 0;
        if (tile > 0) {
            int64_t p = (int64_t)tile - 1;
            uint32_t polls = 0;
            while (true) {
                const int64_t q = p - lane;
                const uint64_t w = q >= 0 ? lb_load(&status[q]) : kLbPrefix;   // before tile 0: prefix 0
                const uint32_t st = (uint32_t)(w >> 62);
                const uint64_t pre = __ballot(st == 2u);
                const int fp = pre ? __ffsll((long long)pre) - 1 : 64;
                const uint64_t need = fp >= 63 ? ~0ull : ((2ull << fp) - 1ull);
                if (__ballot(st == 0u) & need) {
                    if (++polls > kLbMaxPolls) {
                        if (lane == 0) atomicOr(flags, kFlagLookback);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                    continue;
                }
                uint64_t v = lane <= fp ? (w & kLbValue) : 0ull;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
                excl += v;
                if (fp < 64) break;
                p -= 64;
            }
            if (lane == 0) lb_store(&status[tile], kLbPrefix | (excl + agg));
        }
        if (lane == 0) s_excl = excl;
    }
    __syncthreads();
    return s_excl;
}

// exclusive scan of one 64-bit value per thread over the block of NT
// threads; returns the total
template <int NT = kScanThreads>
__device__ __forceinline__ uint64_t block_excl_scan64(uint64_t x, uint64_t& excl) {
    __shared__ uint64_t wsum[NT / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint64_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; i++) {
        const uint64_t s = wsum[i];
        if (i < w) off += s;
        tot += s;
    }
    excl = off + incl - x;
    __syncthreads();
    return tot;
}

// In-place exclusive scan of a[0..n), one chained launch (radix histograms,
// visible records per chunk).
__global__ __launch_bounds__(kScanThreads) void scan_chained_kernel(uint32_t* a, int64_t n, uint64_t* status,
                                                                    uint32_t* counter, uint32_t* flags) {
    const uint32_t t = lb_tile(counter);
    const int64_t base = (int64_t)t * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    loadN(a, base, n, v);
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) sum += v[k];
    uint32_t ex;
    const uint32_t agg = block_excl_scan(sum, ex);
    uint32_t run = (uint32_t)lb_exclusive(status, t, agg, flags) + ex;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        if (base + k < n) a[base + k] = run;
        run += v[k];
    }
}

// info[o].y = bin count | view << kInfoViewShift (a record's bins number at
// most (16384 / 8)^2 < 2^22; views are at most 64)
constexpr uint32_t kInfoViewShift = 24, kInfoCountMask = (1u << kInfoViewShift) - 1u;
static_assert(kMaxViews <= 256, "the view fits above the bin count");

// Visible records (nt != 0) of chunk blockIdx.x (kScanTile records), in
// record order from the chunk's offset o: sort key = depth bits, sort value =
// o, and info[o] = (record, bin count, pixel rect), so that the passes after
// the depth sort read one 16-byte entry of a dense array per record instead
// of gathering from the record lines.  The last chunk stores the visible
// count.  Depth from `depth` when given, else from the records' colour w.
// Visible records of one 2048-record chunk of the padded index, in index
// order: depth key, compaction slot, and the dense entry (record, bin count,
// rect).  The bin count comes from the rect and the bin size, as the pair
// kernels divide it.
__global__ __launch_bounds__(kScanThreads) void compact_kernel(const uint64_t* vis, int64_t words, int64_t n,
                                                               int bw, int bh, const RecLine* lines,
                                                               const float* depth, const uint32_t* chunk_off,
                                                               uint32_t* keys, uint32_t* vals, uint4* info,
                                                               uint32_t* n_visible) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    const int64_t wi = base >> 6;
    const uint32_t vis8 = wi < words ? (uint32_t)(vis[wi] >> (base & 63)) & 0xffu : 0u;
    const uint32_t cnt = (uint32_t)__popc(vis8);
    // a word never straddles two views (rows are padded to whole words): the
    // thread's eight records are Gaussians g0 .. g0 + 7 of view v
    // (32-bit division: the word count stays below 2^31, and a 64-bit
    // division is a long software sequence)
    const uint32_t row = (uint32_t)vis_words(n);
    const uint32_t v = (uint32_t)wi / row;
    const int64_t r0 = (int64_t)v * n + (int64_t)((uint32_t)wi - v * row) * 64 + (base & 63);
    // depths and rects are gathered before any store, so they are in flight at once
    float dz[kScanItems];
    uint2 rc[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const bool f = (vis8 >> k) & 1u;
        const int64_t r = r0 + k;
        dz[k] = f ? (depth ? depth[r] : lines[r].col.w) : 0.f;
        rc[k] = f ? lines[r].rect : make_uint2(0u, 0u);
    }
    uint32_t ex;
    const uint32_t tot = block_excl_scan(cnt, ex);
    uint32_t o = chunk_off[blockIdx.x] + ex;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        if ((vis8 >> k) & 1u) {
            const uint32_t x0 = rc[k].x & 0xffffu, x1 = rc[k].x >> 16, y0 = rc[k].y & 0xffffu, y1 = rc[k].y >> 16;
            const uint32_t nt =
                (x1 / (uint32_t)bw - x0 / (uint32_t)bw + 1u) * (y1 / (uint32_t)bh - y0 / (uint32_t)bh + 1u);
            keys[o] = __float_as_uint(dz[k]);
            vals[o] = o;
            info[o] = make_uint4((uint32_t)(r0 + k), nt | (v << kInfoViewShift), rc[k].x, rc[k].y);
            o++;
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *n_visible = chunk_off[blockIdx.x] + tot;
}

// The forward projection's per-block lists (block b: qcount[b] entries at
// stage[b * kProjBlock * V ...], one per queued pair in queue order) moved to
// the compacted order of the visible records: block b's records start at
// boff[b] (the exclusive scan of the blocks' visible counts, whose last entry
// boff[nb] is the total) and follow in (view, Gaussian) order, the rank of
// record (v, thread t) being the visible records of the block's earlier
// bitmap words (views before v, then wavefronts before t's) plus those of its
// own word below t.  Within a view this is record order, as the bitmap
// compaction gives; records of different views never share a bin, so the
// (bin, depth, record) order of the pairs is the same either way.
__global__ __launch_bounds__(kScanThreads) void stage_copy_kernel(const uint4* stage, const uint32_t* qcount,
                                                                  const uint32_t* boff, const uint64_t* vis,
                                                                  int64_t n, int V, int64_t nb, int bw, int bh,
                                                                  uint32_t* keys, uint32_t* vals, uint4* info,
                                                                  uint32_t* pre, float* g2, uint32_t* n_visible) {
    constexpr int kW = kProjBlock / 64;   // bitmap words per view of one projection block
    static_assert(kMaxViews * kW <= kScanThreads, "one thread per bitmap word of the block");
    __shared__ uint64_t s_w[kMaxViews * kW];
    __shared__ uint32_t s_pre[kMaxViews * kW];
    const int64_t b = blockIdx.x;
    const int64_t vrow = vis_words(n);
    const int k = threadIdx.x;
    uint64_t wd = 0ull;
    if (k < V * kW && b * kW + k % kW < vrow) wd = vis[(int64_t)(k / kW) * vrow + b * kW + k % kW];
    if (k < V * kW) s_w[k] = wd;
    uint32_t ex;
    block_excl_scan((uint32_t)__popcll(wd), ex);
    if (k < V * kW) s_pre[k] = ex;
    const uint32_t o0 = boff[b];
    // the slot bases for the projection backward
    if (k < V * kW) pre[b * V * kW + k] = o0 + ex;
    __syncthreads();
    if (b == nb - 1 && threadIdx.x == 0) *n_visible = boff[nb];
    const uint4* src = stage + b * kProjBlock * (int64_t)V;
    const uint32_t nq = qcount[b];
    for (uint32_t i = threadIdx.x; i < nq; i += kScanThreads) {
        const uint4 e = src[i];
        if (e.x == kStageNone) continue;
        const int v = (int)(e.x >> 8), t = (int)(e.x & 255u);
        const int wk = v * kW + (t >> 6);
        const uint32_t o = o0 + s_pre[wk] + (uint32_t)__popcll(s_w[wk] & ((1ull << (t & 63)) - 1ull));
        const uint32_t x0 = e.z & 0xffffu, x1 = e.z >> 16, y0 = e.w & 0xffffu, y1 = e.w >> 16;
        const uint32_t nt = (x1 / (uint32_t)bw - x0 / (uint32_t)bw + 1u) * (y1 / (uint32_t)bh - y0 / (uint32_t)bh + 1u);
        keys[o] = e.y;
        vals[o] = o;
        info[o] = make_uint4((uint32_t)((int64_t)v * n + b * kProjBlock + t), nt | ((uint32_t)v << kInfoViewShift),
                             e.z, e.w);
        if (g2) {
            float4* z = reinterpret_cast<float4*>(g2 + (int64_t)o * kG2Floats);
            z[0] = z[1] = z[2] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
}

// The pair kernels walk the depth-sorted visible records: 512 threads per
// 2048-record chunk (four records each), so that the few chunks there are
// run as many wavefronts.
constexpr int kPairThreads = 512;
constexpr int kPairItems = kScanTile / kPairThreads;
constexpr int kPairGrid = 1024;   // blocks of the pair counting (four per CU, 32 wavefronts)

// pairs (touched bins) of the depth-sorted visible records of one chunk
// (their entries in depth order: sinfo[i] = (slot, bin count | view << 24, rect))
__global__ __launch_bounds__(kPairThreads) void pair_count_kernel(const uint4* sinfo, const uint32_t* nvis_p,
                                                                  uint64_t* chunk, int64_t nc) {
    const int64_t nvis = (int64_t)*nvis_p;
    for (int64_t c = blockIdx.x; c < nc; c += gridDim.x) {   // (c is uniform over the block)
        if (c * kScanTile >= nvis) {   // the whole chunk is past the records
            if (threadIdx.x == 0) chunk[c] = 0ull;
            continue;
        }
        const int64_t base = c * kScanTile + (int64_t)threadIdx.x * kPairItems;
        uint64_t sum = 0;
#pragma unroll
        for (int k = 0; k < kPairItems; k++)
            if (base + k < nvis) sum += sinfo[base + k].y & kInfoCountMask;
        uint64_t ex;
        const uint64_t tot = block_excl_scan64<kPairThreads>(sum, ex);
        if (threadIdx.x == 0) chunk[c] = tot;
    }
}

// In-place exclusive scan of the chunks' pair counts (64-bit), chained; the
// last tile stores the total (kPairsLo/Hi) and the pair count for the sort
// (kNPairs, 0 with kFlagCapacity when the total exceeds the capacity).
__global__ __launch_bounds__(kScanThreads) void pair_offsets_kernel(uint64_t* a, int64_t n, int64_t cap,
                                                                    uint64_t* status, uint32_t* scal) {
    const uint32_t t = lb_tile(scal + kLbPairs);
    const int64_t base = (int64_t)t * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint64_t v[kScanItems];
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        v[k] = base + k < n ? a[base + k] : 0ull;
        sum += v[k];
    }
    uint64_t ex;
    const uint64_t agg = block_excl_scan64(sum, ex);
    const uint64_t excl = lb_exclusive(status, t, agg, scal + kFlags);
    uint64_t run = excl + ex;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        if (base + k < n) a[base + k] = run;
        run += v[k];
    }
    if (t == gridDim.x - 1 && threadIdx.x == 0) {
        const uint64_t total = excl + agg;
        scal[kPairsLo] = (uint32_t)(total & 0xffffffffu);
        scal[kPairsHi] = (uint32_t)(total >> 32);
        if (total > (uint64_t)cap) {
            atomicOr(&scal[kFlags], kFlagCapacity);
            scal[kNPairs] = 0u;
        } else {
            scal[kNPairs] = (uint32_t)total;
        }
    }
}

// One (global bin id, compaction slot) pair per bin each depth-sorted visible record
// of the chunk touches, at the chunk's offset plus the rank within it; pairs
// past the capacity are not written.  Also clears the per-bin ranges.
__global__ __launch_bounds__(kPairThreads) void emit_kernel(ViewTable vt, const uint4* sinfo,
                                                            const uint32_t* nvis_p,
                                                            const uint64_t* chunk_off, int64_t cap, uint32_t* pk,
                                                            uint32_t* pv, uint2* ranges, int64_t n_bins) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n_bins; b += (int64_t)gridDim.x * blockDim.x)
        ranges[b] = make_uint2(0u, 0u);
    const int64_t nvis = (int64_t)*nvis_p;
    if ((int64_t)blockIdx.x * kScanTile >= nvis) return;   // uniform: the whole chunk is past the records
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kPairItems;
    uint4 inf[kPairItems];   // (slot, bin count | view << 24, rect) of each depth-ordered record
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kPairItems; k++) {
        inf[k] = base + k < nvis ? sinfo[base + k] : make_uint4(0u, 0u, 0u, 0u);
        sum += inf[k].y & kInfoCountMask;
    }
    uint64_t ex;
    block_excl_scan64<kPairThreads>(sum, ex);
    uint64_t o = chunk_off[blockIdx.x] + ex;
#pragma unroll
    for (int k = 0; k < kPairItems; k++) {
        if ((inf[k].y & kInfoCountMask) == 0u) continue;
        const uint32_t r = inf[k].x;   // the record's compaction slot
        const ViewInfo& vi = vt.v[(int)(inf[k].y >> kInfoViewShift)];
        const uint2 rc = make_uint2(inf[k].z, inf[k].w);
        const uint32_t tx0 = (rc.x & 0xffffu) / vt.bw, tx1 = (rc.x >> 16) / vt.bw;
        const uint32_t ty0 = (rc.y & 0xffffu) / vt.bh, ty1 = (rc.y >> 16) / vt.bh;
        for (uint32_t ty = ty0; ty <= ty1; ty++) {
            const uint32_t row = (uint32_t)vi.bin_off + ty * (uint32_t)vi.bins_x;
            for (uint32_t tx = tx0; tx <= tx1; tx++, o++) {
                if (o < (uint64_t)cap) {
                    pk[o] = row + tx;
                    pv[o] = r;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ radix sort
constexpr int kRsThreads = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsThreads * kRsItems;   // 2048
static_assert(kRsTile == kRsTileKeys, "the layout sizes the histogram table with kRsTileKeys");
constexpr int kRsWaves = kRsThreads / 64;
constexpr int kRsPerWave = 64 * kRsItems;        // 512

// element count: the device count, never more than the bound the launch was sized for
__device__ __forceinline__ uint32_t load_count(const uint32_t* n_dev, uint32_t n_host) {
    return n_dev ? min(*n_dev, n_host) : n_host;
}

// Items [lo, hi) of this block: the n items are split into gridDim.x
// contiguous ranges whose length is a multiple of one wavefront's share of a
// tile, so block b's items all precede block b + 1's (what makes the
// digit-major histogram scan give stable positions).  A block walks its range
// one 2048-item tile at a time.
__device__ __forceinline__ void rs_range(uint32_t n, uint64_t& lo, uint64_t& hi) {
    const uint64_t per = ((uint64_t)n + gridDim.x - 1) / gridDim.x;
    const uint64_t S = (per + kRsPerWave - 1) / kRsPerWave * kRsPerWave;
    lo = (uint64_t)blockIdx.x * S < n ? (uint64_t)blockIdx.x * S : (uint64_t)n;
    hi = lo + S < n ? lo + S : (uint64_t)n;
}

__global__ __launch_bounds__(kRsThreads) void rs_upsweep_kernel(const uint32_t* keys, const uint32_t* n_dev,
                                                                uint32_t n_host, int shift, uint32_t* hist) {
    __shared__ uint32_t h[kRsWaves][256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kRsWaves * 256; i += kRsThreads) (&h[0][0])[i] = 0u;
    __syncthreads();
    uint64_t lo, hi;
    rs_range(load_count(n_dev, n_host), lo, hi);
    for (uint64_t t0 = lo; t0 < hi; t0 += kRsTile) {
        const uint64_t base = t0 + (uint64_t)w * kRsPerWave;
#pragma unroll 4
        for (int k = 0; k < kRsItems; k++) {
            const uint64_t e = base + (uint64_t)k * 64 + lane;
            if (e < hi) atomicAdd(&h[w][(keys[e] >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    const int d = threadIdx.x;
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < kRsWaves; i++) c += h[i][d];
    hist[(uint64_t)d * gridDim.x + blockIdx.x] = c;
}

// Per tile: rank every key among the tile's keys of its digit (ballots over
// the 8 digit bits within a wavefront, per-wavefront digit counters across
// them), place the tile in LDS in digit order, then write it out with
// consecutive threads on consecutive positions of each digit's run.
// pin / pout (nullable): instead of the keys and values, write pout[pos] =
// pin[value] (the sort's last pass carries a payload in key order)
__global__ __launch_bounds__(kRsThreads) void rs_downsweep_kernel(const uint32_t* kin, const uint32_t* vin,
                                                                  uint32_t* kout, uint32_t* vout,
                                                                  const uint32_t* n_dev, uint32_t n_host, int shift,
                                                                  const uint32_t* hist, const uint4* pin,
                                                                  uint4* pout) {
    static_assert(kRsThreads == kScanThreads && kRsThreads == 256, "one thread per digit");
    __shared__ uint32_t cnt[kRsWaves][256];
    __shared__ uint32_t goff[256];   // global position of the block's next key of each digit
    __shared__ uint32_t toff[256];   // first LDS slot of each digit in the current tile
    __shared__ uint32_t sk[kRsTile], sv[kRsTile];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    goff[threadIdx.x] = hist[(uint64_t)threadIdx.x * gridDim.x + blockIdx.x];
    uint64_t lo, hi;
    rs_range(load_count(n_dev, n_host), lo, hi);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (uint64_t t0 = lo; t0 < hi; t0 += kRsTile) {
        for (int i = threadIdx.x; i < kRsWaves * 256; i += kRsThreads) (&cnt[0][0])[i] = 0u;
        __syncthreads();
        const uint64_t base = t0 + (uint64_t)w * kRsPerWave;
        uint32_t key[kRsItems], val[kRsItems], rank[kRsItems];
#pragma unroll
        for (int k = 0; k < kRsItems; k++) {
            const uint64_t e = base + (uint64_t)k * 64 + lane;
            const bool act = e < hi;
            key[k] = act ? kin[e] : 0u;
            val[k] = act ? vin[e] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kRsItems; k++) {
            const uint64_t e = base + (uint64_t)k * 64 + lane;
            const bool act = e < hi;
            const uint32_t d = (key[k] >> shift) & 255u;
            uint64_t peers = __ballot(act);
#pragma unroll
            for (int b = 0; b < 8; b++) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                peers &= bit ? bb : ~bb;
            }
            rank[k] = 0;
            if (act) {
                const uint32_t before = cnt[w][d];
                rank[k] = before + (uint32_t)__popcll(peers & lt);
                if ((peers >> lane) == 1ull) cnt[w][d] = before + (uint32_t)__popcll(peers);
            }
        }
        __syncthreads();
        uint32_t tile_total;
        {
            const int d = threadIdx.x;
            uint32_t run = 0;
#pragma unroll
            for (int i = 0; i < kRsWaves; i++) {
                const uint32_t c = cnt[i][d];
                cnt[i][d] = run;
                run += c;
            }
            tile_total = run;
        }
        uint32_t tex;
        const uint32_t tile_n = block_excl_scan(tile_total, tex);   // (its barriers order cnt as well)
        toff[threadIdx.x] = tex;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kRsItems; k++) {
            const uint64_t e = base + (uint64_t)k * 64 + lane;
            if (e < hi) {
                const uint32_t d = (key[k] >> shift) & 255u;
                const uint32_t loc = toff[d] + cnt[w][d] + rank[k];
                sk[loc] = key[k];
                sv[loc] = val[k];
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < tile_n; i += kRsThreads) {
            const uint32_t kk = sk[i];
            const uint32_t d = (kk >> shift) & 255u;
            const uint32_t pos = goff[d] + (i - toff[d]);
            if (pout) {
                // the entry in key order, its record replaced by its slot
                const uint4 e = pin[sv[i]];
                pout[pos] = make_uint4(sv[i], e.y, e.z, e.w);
            } else {
                kout[pos] = kk;
                vout[pos] = sv[i];
            }
        }
        __syncthreads();   // goff, cnt and the staging arrays are reused by the next tile
        goff[threadIdx.x] += tile_total;
    }
}

// Stable LSD sort of (key, value) pairs on key bits [0, bits).  Element count
// from n_dev (or n_host when n_dev is null), at most n_bound.  Ping-pongs
// between (k0, v0) and (k1, v1); *in_second tells where the result is.  The
// histogram of pass i is scanned by one chained launch using status[i] and
// counters[i] (cleared beforehand).
// pay_in / pay_out (nullable): the last pass writes pay_out[i] = pay_in[value]
// in key order instead of the sorted keys and values
hipError_t radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* n_dev,
                      int64_t n_bound, int bits, uint32_t* hist, uint64_t* const* status, uint32_t* counters,
                      uint32_t* flags, int max_passes, hipStream_t s, bool* in_second,
                      const uint4* pay_in = nullptr, uint4* pay_out = nullptr) {
    *in_second = false;
    const int64_t nb = std::min<int64_t>((n_bound + kRsTile - 1) / kRsTile, kRsMaxGrid);
    if (nb == 0 || bits <= 0) return hipSuccess;
    if ((bits + 7) / 8 > max_passes) return hipErrorInvalidValue;
    const uint32_t n_host = (uint32_t)n_bound;
    const int64_t nh = 256 * nb;
    const unsigned scan_grid = (unsigned)((nh + kScanTile - 1) / kScanTile);
    bool second = false;
    for (int shift = 0, pass = 0; shift < bits; shift += 8, pass++) {
        const uint32_t* ki = second ? k1 : k0;
        const uint32_t* vi = second ? v1 : v0;
        uint32_t* ko = second ? k0 : k1;
        uint32_t* vo = second ? v0 : v1;
        rs_upsweep_kernel<<<(unsigned)nb, kRsThreads, 0, s>>>(ki, n_dev, n_host, shift, hist);
        scan_chained_kernel<<<scan_grid, kScanThreads, 0, s>>>(hist, nh, status[pass], counters + pass, flags);
        const bool last = shift + 8 >= bits;
        rs_downsweep_kernel<<<(unsigned)nb, kRsThreads, 0, s>>>(ki, vi, ko, vo, n_dev, n_host, shift, hist,
                                                                last ? pay_in : nullptr, last ? pay_out : nullptr);
        second = !second;
    }
    *in_second = second;
    return hipGetLastError();
}

// ------------------------------------------------------------------ ranges
__global__ void ranges_kernel(const uint32_t* keys, const uint32_t* np, uint2* ranges) {
    const uint32_t P = *np;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)P) return;
    const uint32_t k = keys[i];
    if (i == 0 || keys[i - 1] != k) ranges[k].x = (uint32_t)i;
    if (i == (int64_t)P - 1 || keys[i + 1] != k) ranges[k].y = (uint32_t)(i + 1);
}

// Per-bin ranges when the pairs were sorted in one 8-bit pass: the pass's
// scanned histogram table (digit-major, nb blocks) holds at hist[d * nb] the
// number of pairs whose bin is below d, i.e. where bin d's range starts.
// Empty bins get (0, 0), as ranges_kernel leaves them.
__global__ void ranges_from_hist_kernel(const uint32_t* hist, int64_t nb, const uint32_t* np, int n_bins,
                                        uint2* ranges) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n_bins) return;
    const uint32_t b = hist[(int64_t)d * nb];
    const uint32_t e = d + 1 < 256 ? hist[(int64_t)(d + 1) * nb] : *np;
    ranges[d] = e > b ? make_uint2(b, e) : make_uint2(0u, 0u);
}

__global__ void slots_to_records_kernel(const uint32_t* slots, const uint4* info, const uint32_t* np, uint32_t* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (int64_t)*np) out[i] = info[slots[i]].x;
}

// each record's pixel rect (binning entry point) clipped to its image into
// its line, and the visibility bitmap of the non-empty ones; the clipped rect
// is what pairs are emitted from, so a caller's out-of-image rect cannot
// address a tile of another view.  One thread per padded record.
__global__ void rect_tiles_kernel(ViewTable vt, const uint2* rect, RecLine* lines, uint64_t* vis, int64_t n) {
    const int64_t n64 = 64 * vis_words(n), words = (int64_t)vt.V * vis_words(n);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t v = p / n64, g = p - v * n64;
    bool valid = false;
    if (v < vt.V && g < n) {
        const ViewInfo& vi = vt.v[v];
        const int64_t i = v * n + g;
        const uint2 rc = rect[i];
        const uint32_t x0 = rc.x & 0xffffu, y0 = rc.y & 0xffffu;
        const uint32_t x1 = min(rc.x >> 16, (uint32_t)vi.W - 1u), y1 = min(rc.y >> 16, (uint32_t)vi.H - 1u);
        valid = !(x0 > x1 || y0 > y1);
        lines[i].rect = valid ? make_uint2(x0 | (x1 << 16), y0 | (y1 << 16)) : make_uint2(1u, 1u);
    }
    const uint64_t bm = __ballot(valid);
    if ((threadIdx.x & 63) == 0 && (p >> 6) < words) vis[p >> 6] = bm;
}

inline int ceil_log2(int64_t x) {
    int b = 0;
    while (((int64_t)1 << b) < x) b++;
    return b;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    fill_u32_kernel<<<fill_grid(n), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    fill_f32_kernel<<<fill_grid(n), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_rect_tiles(const ViewTable& vt, const uint2* rect, RecLine* lines, uint64_t* vis, int64_t n,
                             hipStream_t s) {
    const int64_t Rp = 64 * vis_words(n) * vt.V;
    if (Rp <= 0) return hipSuccess;
    rect_tiles_kernel<<<(unsigned)((Rp + 255) / 256), 256, 0, s>>>(vt, rect, lines, vis, n);
    return hipGetLastError();
}

#define GS_AT(T, off) reinterpret_cast<T*>(base + (off))

namespace {
// zero p[0, n) except the sticky status word
__global__ void status_clear_kernel(uint32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (i != kSticky) p[i] = 0u;
}
}  // namespace

hipError_t launch_status_clear(const Layout& L, char* base, hipStream_t s) {
    uint32_t* scal = GS_AT(uint32_t, L.off_scalars);
    const int64_t n = (int64_t)((L.off_lb - L.off_scalars) / 4) + 2 * lb_words(L);
    int64_t b = (n + 255) / 256;
    if (b > 1024) b = 1024;
    status_clear_kernel<<<(unsigned)b, 256, 0, s>>>(scal, n);
    return hipGetLastError();
}

hipError_t launch_binning_count(const ViewTable& vt, const Layout& L, char* base, const uint64_t* vis,
                                const RecLine* lines, const float* depth_src, bool staged, float* zero_g2,
                                hipStream_t s) {
    uint32_t* scal = GS_AT(uint32_t, L.off_scalars);
    uint64_t* lb = GS_AT(uint64_t, L.off_lb);
    uint32_t* k0 = GS_AT(uint32_t, L.off_k0);
    uint32_t* v0 = GS_AT(uint32_t, L.off_v0);
    uint32_t* k1 = GS_AT(uint32_t, L.off_k1);
    uint32_t* v1 = GS_AT(uint32_t, L.off_v1);
    uint32_t* csum = GS_AT(uint32_t, L.off_chunk);
    uint64_t* psum = GS_AT(uint64_t, L.off_chunk);
    const int64_t R = L.R, words = L.Rp / 64;
    const int64_t nc = L.n_chunks;
    const unsigned g = (unsigned)nc, gs = (unsigned)L.lb_tiles_chunk;
    hipError_t e;
    // (the scalars and every chained-scan status word were cleared by
    // launch_status_clear before the projection)
    // 1. visible records -> compacted (depth bits, record), in record order
    //    within each view
    uint4* info = GS_AT(uint4, L.off_info);
    if (staged) {
        // from the forward projection's per-block lists (none when n = 0:
        // the visible count stays at its cleared 0)
        const int64_t nb = proj_blocks(vt.n);
        if (nb > 0) {
            uint32_t* bcount = GS_AT(uint32_t, L.off_bcount);
            uint64_t* lbp = lb + 2 * L.lb_tiles_chunk + (int64_t)kLbHistUses * L.lb_tiles_hist;
            scan_chained_kernel<<<(unsigned)L.lb_tiles_proj, kScanThreads, 0, s>>>(bcount, nb + 1, lbp,
                                                                                  scal + kLbProj, scal + kFlags);
            stage_copy_kernel<<<(unsigned)nb, kScanThreads, 0, s>>>(
                GS_AT(uint4, L.off_sinfo), GS_AT(uint32_t, L.off_qcount), bcount, vis, vt.n, vt.V, nb, vt.bw,
                vt.bh, k0, v0, info, GS_AT(uint32_t, L.off_pre), zero_g2, scal + kNVis);
        }
    } else {
        scan_reduce_kernel<LoadBits><<<g, kScanThreads, 0, s>>>(LoadBits{vis, words}, L.Rp, csum);
        scan_chained_kernel<<<gs, kScanThreads, 0, s>>>(csum, nc, lb, scal + kLbVis, scal + kFlags);
        compact_kernel<<<g, kScanThreads, 0, s>>>(vis, words, vt.n, vt.bw, vt.bh, lines, depth_src, csum, k0,
                                                  v0, info, scal + kNVis);
    }
    // 2. stable sort by depth bits (4 passes: the result is back in (k0, v0))
    uint64_t* hs[kLbHistUses];
    for (int i = 0; i < kLbHistUses; i++) hs[i] = lb + 2 * L.lb_tiles_chunk + (int64_t)i * L.lb_tiles_hist;
    // the last pass writes the dense entries themselves in depth order
    uint4* sinfo = GS_AT(uint4, L.off_sinfo);
    bool second;
    e = radix_sort(k0, v0, k1, v1, scal + kNVis, R, 32, GS_AT(uint32_t, L.off_hist), hs, scal + kLbHist0,
                   scal + kFlags, 4, s, &second, info, sinfo);
    if (e != hipSuccess) return e;
    // 3. pairs in depth order: per-chunk counts, chained offsets (the total
    //    stays on the device), emission
    // (the visible count is on the device: a capped grid loops over the
    // chunks for the counts; emission keeps one block per chunk, which
    // measured faster than the loop)
    const unsigned gp = (unsigned)std::min<int64_t>(nc, kPairGrid);
    pair_count_kernel<<<gp, kPairThreads, 0, s>>>(sinfo, scal + kNVis, psum, nc);
    pair_offsets_kernel<<<gs, kScanThreads, 0, s>>>(psum, nc, L.cap, lb + L.lb_tiles_chunk, scal);
    emit_kernel<<<g, kPairThreads, 0, s>>>(vt, sinfo, scal + kNVis, psum, L.cap,
                                           GS_AT(uint32_t, L.off_pk0), GS_AT(uint32_t, L.off_pv0),
                                           GS_AT(uint2, L.off_ranges), L.n_bins);
    return hipGetLastError();
}

hipError_t launch_binning_sort(const ViewTable& vt, const Layout& L, char* base, int64_t pair_bound, hipStream_t s,
                               uint32_t** sorted_vals_out) {
    uint32_t* scal = GS_AT(uint32_t, L.off_scalars);
    uint64_t* lb = GS_AT(uint64_t, L.off_lb);
    uint32_t* pk0 = GS_AT(uint32_t, L.off_pk0);
    uint32_t* pv0 = GS_AT(uint32_t, L.off_pv0);
    uint32_t* pk1 = GS_AT(uint32_t, L.off_pk1);
    uint32_t* pv1 = GS_AT(uint32_t, L.off_pv1);
    // the pair sort's histogram scans follow the record sort's four
    uint64_t* hs[kLbHistUses - 4];
    for (int i = 0; i < kLbHistUses - 4; i++) hs[i] = lb + 2 * L.lb_tiles_chunk + (int64_t)(4 + i) * L.lb_tiles_hist;
    bool second;
    hipError_t e = radix_sort(pk0, pv0, pk1, pv1, scal + kNPairs, pair_bound, ceil_log2(L.n_bins),
                              GS_AT(uint32_t, L.off_hist), hs, scal + kLbHist0 + 4, scal + kFlags, kLbHistUses - 4,
                              s, &second);
    if (e != hipSuccess) return e;
    const uint32_t* keys = second ? pk1 : pk0;
    uint2* ranges = GS_AT(uint2, L.off_ranges);
    const int bits = ceil_log2(L.n_bins);
    if (pair_bound > 0 && bits >= 1 && bits <= 8) {
        // one pass: the ranges are the scanned histogram's digit offsets
        const int64_t nb = std::min<int64_t>((pair_bound + kRsTile - 1) / kRsTile, kRsMaxGrid);
        ranges_from_hist_kernel<<<(unsigned)((L.n_bins + 255) / 256), 256, 0, s>>>(
            GS_AT(uint32_t, L.off_hist), nb, scal + kNPairs, (int)L.n_bins, ranges);
    } else if (pair_bound > 0) {
        const int64_t g = (pair_bound + 255) / 256;
        ranges_kernel<<<(unsigned)g, 256, 0, s>>>(keys, scal + kNPairs, ranges);
    }
    *sorted_vals_out = second ? pv1 : pv0;
    return hipGetLastError();
}

hipError_t launch_binning(const ViewTable& vt, const Layout& L, char* base, const uint64_t* vis,
                          const RecLine* lines, const float* depth_src, bool staged, float* zero_g2,
                          int64_t pair_bound, hipStream_t s, uint32_t** sorted_vals_out) {
    hipError_t e = launch_binning_count(vt, L, base, vis, lines, depth_src, staged, zero_g2, s);
    if (e != hipSuccess) return e;
    return launch_binning_sort(vt, L, base, pair_bound, s, sorted_vals_out);
}

#undef GS_AT

hipError_t launch_slots_to_records(const uint32_t* slots, const uint4* info, const uint32_t* n, int64_t bound,
                                   uint32_t* out, hipStream_t s) {
    if (bound <= 0) return hipSuccess;
    slots_to_records_kernel<<<(unsigned)((bound + 255) / 256), 256, 0, s>>>(slots, info, n, out);
    return hipGetLastError();
}

hipError_t launch_scan_u32(const uint32_t* a, int64_t n, uint32_t* out, uint32_t* bsum, uint32_t* total32,
                           hipStream_t s) {
    return device_scan(LoadArr{a, n}, n, out, bsum, nullptr, total32, s);
}

}  // namespace gs
