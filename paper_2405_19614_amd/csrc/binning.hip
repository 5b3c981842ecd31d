// Binning: visible records -> (bin, depth, record)-ordered pair list and
// per-bin ranges (the front-to-back order of the Sec. 3.4 rasteriser).  A bin
// is a rectangle of pixels (a multiple of the compositing tile); each
// compositing tile reads its bin's list.
//
// Two-stage design instead of one 64-bit-key sort of all pairs:
//   1. compact the visible records (scan of a 0/1 flag) and sort them by the
//      bit pattern of their positive FP32 depth (stable LSD radix sort, so
//      equal depths keep ascending record order);
//   2. emit one pair (global bin id, record) per touched bin in that depth
//      order and sort the pairs stably by bin id only (ceil(log2 bins)
//      bits).  Stability makes the result the (bin, depth, record) order.
// Stage 1 sorts records (millions), stage 2 sorts only 8-18 key bits of the
// pairs, instead of ~50 bits.
//
// All kernels read element counts from the device (scalars block), so the
// whole sequence needs no host synchronisation; grids are sized from host
// upper bounds.
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

struct LoadVis {   // 1 if the record is visible
    const uint32_t* nt;
    int64_t n;
    __device__ uint32_t operator()(int64_t i) const { return (i < n && nt[i] != 0u) ? 1u : 0u; }
};
struct LoadCnt {   // tile count of the i-th depth-sorted visible record
    const uint32_t* nt;
    const uint32_t* ids;
    const uint32_t* nvis;
    __device__ uint32_t operator()(int64_t i) const { return i < (int64_t)*nvis ? nt[ids[i]] : 0u; }
};
struct LoadArr {
    const uint32_t* a;
    int64_t n;
    __device__ uint32_t operator()(int64_t i) const { return i < n ? a[i] : 0u; }
};

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
#pragma unroll
    for (int k = 0; k < kScanItems; k++)
        if (base + k < n) s += ld(base + k);
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

// ------------------------------------------------------------------ compaction
__global__ void compact_kernel(const uint32_t* nt, const float4* col, const uint32_t* off, int64_t R, uint32_t* keys,
                               uint32_t* vals) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R || nt[r] == 0u) return;
    const uint32_t o = off[r];
    keys[o] = __float_as_uint(col[r].w);
    vals[o] = (uint32_t)r;
}
__global__ void compact_depth_kernel(const uint32_t* nt, const float* depth, const uint32_t* off, int64_t R,
                                     uint32_t* keys, uint32_t* vals) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R || nt[r] == 0u) return;
    const uint32_t o = off[r];
    keys[o] = __float_as_uint(depth[r]);
    vals[o] = (uint32_t)r;
}

// ------------------------------------------------------------------ radix sort
constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;   // 4096
constexpr int kRsWaves = kRsThreads / 64;
constexpr int kRsPerWave = 64 * kRsItems;        // 1024

__device__ __forceinline__ uint32_t load_count(const uint32_t* n_dev, uint32_t n_host) {
    return n_dev ? *n_dev : n_host;
}

__global__ __launch_bounds__(kRsThreads) void rs_upsweep_kernel(const uint32_t* keys, const uint32_t* n_dev,
                                                                uint32_t n_host, int shift, uint32_t* hist) {
    __shared__ uint32_t h[kRsWaves][256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kRsWaves * 256; i += kRsThreads) (&h[0][0])[i] = 0u;
    __syncthreads();
    const uint32_t n = load_count(n_dev, n_host);
    const uint64_t base = (uint64_t)blockIdx.x * kRsTile + (uint64_t)w * kRsPerWave;
#pragma unroll 4
    for (int k = 0; k < kRsItems; k++) {
        const uint64_t e = base + (uint64_t)k * 64 + lane;
        if (e < n) atomicAdd(&h[w][(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    const int d = threadIdx.x;
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < kRsWaves; i++) c += h[i][d];
    hist[(uint64_t)d * gridDim.x + blockIdx.x] = c;
}

__global__ __launch_bounds__(kRsThreads) void rs_downsweep_kernel(const uint32_t* kin, const uint32_t* vin,
                                                                  uint32_t* kout, uint32_t* vout,
                                                                  const uint32_t* n_dev, uint32_t n_host, int shift,
                                                                  const uint32_t* hist) {
    __shared__ uint32_t cnt[kRsWaves][256];
    __shared__ uint32_t goff[256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kRsWaves * 256; i += kRsThreads) (&cnt[0][0])[i] = 0u;
    goff[threadIdx.x] = hist[(uint64_t)threadIdx.x * gridDim.x + blockIdx.x];
    __syncthreads();
    const uint32_t n = load_count(n_dev, n_host);
    const uint64_t base = (uint64_t)blockIdx.x * kRsTile + (uint64_t)w * kRsPerWave;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t key[kRsItems], val[kRsItems], rank[kRsItems];
#pragma unroll
    for (int k = 0; k < kRsItems; k++) {
        const uint64_t e = base + (uint64_t)k * 64 + lane;
        const bool act = e < n;
        key[k] = act ? kin[e] : 0u;
        val[k] = act ? vin[e] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kRsItems; k++) {
        const uint64_t e = base + (uint64_t)k * 64 + lane;
        const bool act = e < n;
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
    {
        const int d = threadIdx.x;
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < kRsWaves; i++) {
            const uint32_t c = cnt[i][d];
            cnt[i][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRsItems; k++) {
        const uint64_t e = base + (uint64_t)k * 64 + lane;
        if (e < n) {
            const uint32_t d = (key[k] >> shift) & 255u;
            const uint32_t pos = goff[d] + cnt[w][d] + rank[k];
            kout[pos] = key[k];
            vout[pos] = val[k];
        }
    }
}

// Stable LSD sort of (key, value) pairs on key bits [0, bits).  Element count
// from n_dev (or n_host when n_dev is null), at most n_bound.  Ping-pongs
// between (k0, v0) and (k1, v1); *in_second tells where the result is.
hipError_t radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* n_dev,
                      int64_t n_bound, int bits, uint32_t* hist, uint32_t* scan_bsum, hipStream_t s,
                      bool* in_second) {
    *in_second = false;
    const int64_t nb = (n_bound + kRsTile - 1) / kRsTile;
    if (nb == 0 || bits <= 0) return hipSuccess;
    const uint32_t n_host = (uint32_t)n_bound;
    bool second = false;
    for (int shift = 0; shift < bits; shift += 8) {
        const uint32_t* ki = second ? k1 : k0;
        const uint32_t* vi = second ? v1 : v0;
        uint32_t* ko = second ? k0 : k1;
        uint32_t* vo = second ? v0 : v1;
        rs_upsweep_kernel<<<(unsigned)nb, kRsThreads, 0, s>>>(ki, n_dev, n_host, shift, hist);
        hipError_t e = device_scan(LoadArr{hist, 256 * nb}, 256 * nb, hist, scan_bsum, nullptr, nullptr, s);
        if (e != hipSuccess) return e;
        rs_downsweep_kernel<<<(unsigned)nb, kRsThreads, 0, s>>>(ki, vi, ko, vo, n_dev, n_host, shift, hist);
        second = !second;
    }
    *in_second = second;
    return hipGetLastError();
}

// ------------------------------------------------------------------ pairs
__global__ void emit_kernel(ViewTable vt, const uint32_t* ids, const uint32_t* nvis, const uint2* rect,
                            const uint32_t* off, const uint32_t* total64, int64_t cap, uint32_t* pk, uint32_t* pv,
                            uint32_t* scal) {
    const uint64_t total = (uint64_t)total64[0] | ((uint64_t)total64[1] << 32);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (total > (uint64_t)cap) {
        if (i == 0) {
            atomicOr(&scal[kFlags], 1u);
            scal[kNPairs] = 0u;
        }
        return;
    }
    if (i == 0) scal[kNPairs] = (uint32_t)total;
    if (i >= (int64_t)*nvis) return;
    const uint32_t r = ids[i];
    const int v = (int)(r / (uint32_t)vt.n);
    const ViewInfo& vi = vt.v[v];
    const uint2 rc = rect[r];
    const uint32_t tx0 = (rc.x & 0xffffu) / vt.bw, tx1 = (rc.x >> 16) / vt.bw;
    const uint32_t ty0 = (rc.y & 0xffffu) / vt.bh, ty1 = (rc.y >> 16) / vt.bh;
    uint32_t o = off[i];
    for (uint32_t ty = ty0; ty <= ty1; ty++) {
        const uint32_t row = (uint32_t)vi.bin_off + ty * (uint32_t)vi.bins_x;
        for (uint32_t tx = tx0; tx <= tx1; tx++, o++) {
            pk[o] = row + tx;
            pv[o] = r;
        }
    }
}

__global__ void ranges_kernel(const uint32_t* keys, const uint32_t* np, uint2* ranges) {
    const uint32_t P = *np;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)P) return;
    const uint32_t k = keys[i];
    if (i == 0 || keys[i - 1] != k) ranges[k].x = (uint32_t)i;
    if (i == (int64_t)P - 1 || keys[i + 1] != k) ranges[k].y = (uint32_t)(i + 1);
}

// tile count of each record from its pixel rect (binning entry point); the
// rect is clipped to its image and the clipped copy is what pairs are emitted
// from, so a caller's out-of-image rect cannot address a tile of another view
__global__ void rect_tiles_kernel(ViewTable vt, const uint2* rect, uint2* rect_out, uint32_t* nt, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * vt.V) return;
    const ViewInfo& vi = vt.v[i / n];
    const uint2 rc = rect[i];
    const uint32_t x0 = rc.x & 0xffffu, y0 = rc.y & 0xffffu;
    const uint32_t x1 = min(rc.x >> 16, (uint32_t)vi.W - 1u), y1 = min(rc.y >> 16, (uint32_t)vi.H - 1u);
    const bool empty = x0 > x1 || y0 > y1;
    rect_out[i] = empty ? make_uint2(1u, 1u) : make_uint2(x0 | (x1 << 16), y0 | (y1 << 16));
    nt[i] = empty ? 0u : (x1 / vt.bw - x0 / vt.bw + 1) * (y1 / vt.bh - y0 / vt.bh + 1);
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

hipError_t launch_rect_tiles(const ViewTable& vt, const uint2* rect, uint2* rect_out, uint32_t* nt, int64_t n,
                             hipStream_t s) {
    const int64_t R = n * vt.V;
    if (R <= 0) return hipSuccess;
    rect_tiles_kernel<<<(unsigned)((R + 255) / 256), 256, 0, s>>>(vt, rect, rect_out, nt, n);
    return hipGetLastError();
}

#define GS_AT(T, off) reinterpret_cast<T*>(base + (off))

hipError_t launch_binning_count(const ViewTable& vt, const Layout& L, char* base, const uint32_t* nt_src,
                                const float* depth_src, hipStream_t s) {
    uint32_t* scal = GS_AT(uint32_t, L.off_scalars);
    uint32_t* cnt = GS_AT(uint32_t, L.off_cnt);
    uint32_t* bsum = GS_AT(uint32_t, L.off_scan);
    uint32_t* k0 = GS_AT(uint32_t, L.off_k0);
    uint32_t* v0 = GS_AT(uint32_t, L.off_v0);
    uint32_t* k1 = GS_AT(uint32_t, L.off_k1);
    uint32_t* v1 = GS_AT(uint32_t, L.off_v1);
    const int64_t R = L.R;
    hipError_t e = launch_fill_u32(scal, 0u, kNumScalars, s);
    if (e != hipSuccess) return e;
    // 1. visible records -> compacted (depth bits, record) in record order
    e = device_scan(LoadVis{nt_src, R}, R, cnt, bsum, nullptr, scal + kNVis, s);
    if (e != hipSuccess) return e;
    if (R > 0) {
        const unsigned g = (unsigned)((R + 255) / 256);
        if (depth_src)
            compact_depth_kernel<<<g, 256, 0, s>>>(nt_src, depth_src, cnt, R, k0, v0);
        else
            compact_kernel<<<g, 256, 0, s>>>(nt_src, GS_AT(float4, L.off_col), cnt, R, k0, v0);
    }
    // 2. stable sort by depth bits
    bool second;
    e = radix_sort(k0, v0, k1, v1, scal + kNVis, R, 32, GS_AT(uint32_t, L.off_hist), bsum, s, &second);
    if (e != hipSuccess) return e;
    const uint32_t* ids = second ? v1 : v0;
    // 3. pair offsets of the sorted records, 64-bit total in the scalars
    e = device_scan(LoadCnt{nt_src, ids, scal + kNVis}, R, cnt, bsum, scal + kPairsLo, nullptr, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_binning_emit(const ViewTable& vt, const Layout& L, char* base, const uint2* rect_src,
                               int64_t pair_bound, hipStream_t s, uint32_t** sorted_vals_out) {
    uint32_t* scal = GS_AT(uint32_t, L.off_scalars);
    uint32_t* cnt = GS_AT(uint32_t, L.off_cnt);
    uint32_t* bsum = GS_AT(uint32_t, L.off_scan);
    // the record sort always runs 4 passes (32 bits): result back in (k0, v0)
    const uint32_t* ids = GS_AT(uint32_t, L.off_v0);
    uint32_t* pk0 = GS_AT(uint32_t, L.off_pk0);
    uint32_t* pv0 = GS_AT(uint32_t, L.off_pv0);
    uint32_t* pk1 = GS_AT(uint32_t, L.off_pk1);
    uint32_t* pv1 = GS_AT(uint32_t, L.off_pv1);
    const int64_t R = L.R;
    hipError_t e;
    {
        const int64_t g = R > 0 ? (R + 255) / 256 : 1;
        emit_kernel<<<(unsigned)g, 256, 0, s>>>(vt, ids, scal + kNVis, rect_src, cnt, scal + kPairsLo, L.cap, pk0,
                                                 pv0, scal);
    }
    bool second;
    e = radix_sort(pk0, pv0, pk1, pv1, scal + kNPairs, pair_bound, ceil_log2(L.n_bins),
                   GS_AT(uint32_t, L.off_hist), bsum, s, &second);
    if (e != hipSuccess) return e;
    const uint32_t* keys = second ? pk1 : pk0;
    uint2* ranges = GS_AT(uint2, L.off_ranges);
    e = launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2 * L.n_bins, s);
    if (e != hipSuccess) return e;
    if (pair_bound > 0) {
        const int64_t g = (pair_bound + 255) / 256;
        ranges_kernel<<<(unsigned)g, 256, 0, s>>>(keys, scal + kNPairs, ranges);
    }
    *sorted_vals_out = second ? pv1 : pv0;
    return hipGetLastError();
}

hipError_t launch_binning(const ViewTable& vt, const Layout& L, char* base, const uint32_t* nt_src,
                          const uint2* rect_src, const float* depth_src, int64_t pair_bound, hipStream_t s,
                          uint32_t** sorted_vals_out) {
    hipError_t e = launch_binning_count(vt, L, base, nt_src, depth_src, s);
    if (e != hipSuccess) return e;
    return launch_binning_emit(vt, L, base, rect_src, pair_bound, s, sorted_vals_out);
}

#undef GS_AT

hipError_t launch_scan_u32(const uint32_t* a, int64_t n, uint32_t* out, uint32_t* bsum, uint32_t* total32,
                           hipStream_t s) {
    return device_scan(LoadArr{a, n}, n, out, bsum, nullptr, total32, s);
}

}  // namespace gs
