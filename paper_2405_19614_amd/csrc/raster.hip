// Tile compositing, forward and backward (Sec. 3.4 "Differentiable
// Rasterization": colour and depth compositing; Sec. 3.3 border mask).
//
// One workgroup per (view, tile) of every view in one launch, tiles taken
// heaviest first (order_tiles_kernel).  Each thread
// owns PPT vertically adjacent pixels of the tile, so one LDS read of a list
// entry and one wavefront reduction serve PPT pixels.  The tile's
// depth-ordered list is staged through LDS in batches of one record per
// thread.
// Forward: front to back per pixel, workgroup-wide early exit once every
// pixel has stopped; an optional fused epilogue writes the L1 loss's upstream
// gradients and per-tile loss partials.
// Backward: the list walked back to front from each pixel's stop index,
// transmittance recovered by division, per-Gaussian gradients summed over the
// thread's pixels, then over each 16-lane row by a DPP reduce-scatter that
// leaves the ten values in ten distinct lanes, then across rows and waves with
// one LDS atomic instruction per entry, then one global atomic per (tile,
// Gaussian, value).
#include <type_traits>

#include "gs_device.h"

namespace gs {

namespace {

__device__ __forceinline__ float sgnf(float e) { return (float)((e > 0.f) - (e < 0.f)); }

template <int NT>
__device__ __forceinline__ double2 block_sum2(float a, float b) {
    __shared__ double red[NT / 64][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if (lane == 0) { red[w][0] = (double)a; red[w][1] = (double)b; }
    __syncthreads();
    double2 r = make_double2(0.0, 0.0);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / 64; i++) { r.x += red[i][0]; r.y += red[i][1]; }
    }
    __syncthreads();   // red[] may be reused by a following call
    return r;
}

// Lane exchange inside a 16-lane DPP row: row_mirror pairs lane i with 15 - i,
// row_half_mirror i with i ^ 7 (inside each half row), the two quad_perm
// patterns i with i ^ 2 and i ^ 1.
template <int CTRL>
__device__ __forceinline__ float dpp_x(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// Reduce-scatter of ten per-lane values over each 16-lane row: four
// butterfly exchanges (lane pairs differing in bit 3, 2, 1, 0) in which each
// lane keeps the half of its values that its bit selects and adds the
// partner's copy of that half.  Afterwards lane i of a row holds the row total
// of value kRsSlot[i] (-1: nothing).  33 VALU operations against 60 for ten
// separate lane-63 reductions, and the results land in distinct lanes, so
// one LDS atomic instruction stores all ten.
__device__ __forceinline__ float row_reduce_scatter10(const float (&v)[10], int lane) {
    const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0, b1 = (lane & 2) != 0, b0 = (lane & 1) != 0;
    float u[5];
#pragma unroll
    for (int i = 0; i < 5; i++) {
        const float snd = b3 ? v[i] : v[i + 5];
        const float kp = b3 ? v[i + 5] : v[i];
        u[i] = kp + dpp_x<0x140>(snd);   // row_mirror
    }
    float w[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const float hi = (i < 2) ? u[i + 3] : 0.f;
        const float snd = b2 ? u[i] : hi;
        const float kp = b2 ? hi : u[i];
        w[i] = kp + dpp_x<0x141>(snd);   // row_half_mirror
    }
    float x[2];
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const float hi = (i < 1) ? w[i + 2] : 0.f;
        const float snd = b1 ? w[i] : hi;
        const float kp = b1 ? hi : w[i];
        x[i] = kp + dpp_x<0x4E>(snd);    // quad_perm [2, 3, 0, 1]
    }
    const float snd = b0 ? x[0] : x[1];
    const float kp = b0 ? x[1] : x[0];
    return kp + dpp_x<0xB1>(snd);        // quad_perm [1, 0, 3, 2]
}

// value held by lane (i mod 16) after row_reduce_scatter10, -1 for none
__device__ __forceinline__ int rs_slot(int lane) {
    const int l = lane & 15;
    const int w = (l & 3) == 3 ? -1 : (l & 3);         // bits 1, 0 -> index among three
    if (w < 0) return -1;
    const int u = (l & 4) ? (w + 3 < 5 ? w + 3 : -1) : w;   // bit 2 -> index among five
    if (u < 0) return -1;
    return ((l & 8) ? 5 : 0) + u;                      // bit 3 -> index among ten
}

// Block-wide stream compaction: the rank of this thread's flagged item among
// the flagged items of the workgroup (in thread order); *total = their count.
template <int NT>
__device__ __forceinline__ int block_compact(bool flag, int* total) {
    __shared__ int wcnt[NT / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t m = __ballot(flag);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[w] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; i++) {
        const int c = wcnt[i];
        off += (i < w) ? c : 0;
        tot += c;
    }
    *total = tot;
    __syncthreads();   // wcnt[] may be reused by the next call
    return off + before;
}

// rect (x0 | x1 << 16, y0 | y1 << 16) meets the pixel box [bx0, bx1] x [by0, by1]
__device__ __forceinline__ bool rect_meets(uint2 rc, int bx0, int bx1, int by0, int by1) {
    return (int)(rc.x & 0xffffu) <= bx1 && (int)(rc.x >> 16) >= bx0 && (int)(rc.y & 0xffffu) <= by1 &&
           (int)(rc.y >> 16) >= by0;
}

// Whether any pixel of the box [x0, x1] x [y0, y1] (a compositing tile clipped
// to the entry's rect) can reach alpha >= 1/255: the smallest exponent
// t = A'dx^2 + B'dx dy + C'dy^2 - log2 o over the box (a convex quadratic, so
// at the mean if the box holds it, else on an edge, where it is a parabola
// minimised in closed form and clamped to the edge) against log2(255).  The
// rect is the box of the alpha ellipse, but a tile inside it can still miss
// the ellipse (thin, tilted Gaussians); such entries are not staged.  The
// 0.1 margin (7 % in alpha) keeps the test conservative under FP32 rounding,
// so no entry that blends a pixel of the tile is dropped.
__device__ __forceinline__ bool ellipse_meets(float2 xy, float4 co, int x0, int x1, int y0, int y1) {
    const float X0 = (float)x0 - xy.x, X1 = (float)x1 - xy.x;
    const float Y0 = (float)y0 - xy.y, Y1 = (float)y1 - xy.y;
    if (X0 <= 0.f && X1 >= 0.f && Y0 <= 0.f && Y1 >= 0.f) return true;
    const auto q = [&](float dx, float dy) { return (co.x * dx + co.y * dy) * dx + co.z * dy * dy; };
    // vertical edges dx = X: minimum at dy = -B' X / (2 C'); horizontal edges likewise
    const float iA = 0.5f / co.x, iC = 0.5f / co.z;
    const float m0 = q(X0, fminf(fmaxf(-co.y * X0 * iC, Y0), Y1));
    const float m1 = q(X1, fminf(fmaxf(-co.y * X1 * iC, Y0), Y1));
    const float m2 = q(fminf(fmaxf(-co.y * Y0 * iA, X0), X1), Y0);
    const float m3 = q(fminf(fmaxf(-co.y * Y1 * iA, X0), X1), Y1);
    const float tmin = fminf(fminf(m0, m1), fminf(m2, m3)) - co.w;
    return tmin <= kLog2AlphaMinInv + 0.1f;
}

// Rect of a staged entry.  Every lane reads the entry from the same LDS
// address, so the packed words are moved to scalar registers and unpacked on
// the scalar unit.
struct RectS {
    int x0, x1, y0, y1;
};
__device__ __forceinline__ RectS rect_scalar(uint2 rc) {
    const uint32_t rx = __builtin_amdgcn_readfirstlane(rc.x), ry = __builtin_amdgcn_readfirstlane(rc.y);
    return RectS{(int)(rx & 0xffffu), (int)(rx >> 16), (int)(ry & 0xffffu), (int)(ry >> 16)};
}

// bin of compositing tile (txi, tyi) of view vi
__device__ __forceinline__ int bin_of_tile(const ViewTable& vt, const ViewInfo& vi, int txi, int tyi, int TW, int TH) {
    return vi.bin_off + ((tyi * TH) / vt.bh) * vi.bins_x + (txi * TW) / vt.bw;
}

// At most six waves per SIMD: the compiler otherwise keeps 64 VGPRs for
// eight and recomputes the pixel coordinates in the inner loop.
template <int TW, int TH, int PPT, bool LOSS, bool COUNT>
__global__ __launch_bounds__(TW* TH / PPT) __attribute__((amdgpu_waves_per_eu(1, 6))) void composite_fwd_kernel(ViewTable vt, const uint2* __restrict__ ranges,
                                                                     const uint32_t* __restrict__ vals, Records rec,
                                                                     float* color, float* depth, float* alpha,
                                                                     float* tfin, uint32_t* last, LossArgs la,
                                                                     const uint32_t* __restrict__ order,
                                                                     uint32_t* __restrict__ work,
                                                                     unsigned long long* counts) {
    constexpr int NT = TW * TH / PPT;
    static_assert(64 % TW == 0 && NT % 64 == 0, "a wavefront spans whole rows of the tile");
    // the staged entries, one 64-byte record each, so that the inner loop
    // reads all of an entry's fields from one LDS address register
    struct alignas(16) Staged {
        float4 co, cz;
        float2 xy;
        uint2 rc;
        uint32_t j, pad[3];
    };
    __shared__ Staged s_e[NT];
    const int t = order ? (int)order[blockIdx.x] : (int)blockIdx.x;   // heaviest tiles first when ordered
    const int v = view_of_tile(vt, t);
    const ViewInfo& vi = vt.v[v];
    const int lt = t - vi.tile_off;
    const int tyi = lt / vi.tiles_x, txi = lt - tyi * vi.tiles_x;
    const int px = txi * TW + (int)(threadIdx.x % TW);
    const int py0 = tyi * TH + (int)(threadIdx.x / TW) * PPT;
    const float fpx = (float)px;
    const uint2 rg = ranges[bin_of_tile(vt, vi, txi, tyi, TW, TH)];
    const int bx0 = txi * TW, bx1 = bx0 + TW - 1, by0 = tyi * TH, by1 = by0 + TH - 1;

    // T[q] < 0 marks a pixel that has stopped (or lies outside the image);
    // its transmittance is then -T[q]
    float T[PPT], C0[PPT], C1[PPT], C2[PPT], D[PPT];
    uint32_t lastp[PPT];
    uint32_t n_visit = 0u, n_blend = 0u, n_entries = 0u;
    // rows of this wavefront: (64 / TW) row groups of PPT rows
    const int wy0 = __builtin_amdgcn_readfirstlane(py0), wy1 = wy0 + (64 / TW) * PPT - 1;
    bool all_done = true;
#pragma unroll
    for (int q = 0; q < PPT; q++) {
        T[q] = (px < vi.W && py0 + q < vi.H) ? 1.f : -1.f;
        C0[q] = C1[q] = C2[q] = D[q] = 0.f;
        lastp[q] = 0u;
        all_done = all_done && T[q] < 0.f;
    }
    for (uint32_t b = rg.x; b < rg.y; b += NT) {
        if (__syncthreads_count(all_done) == NT) break;
        // stage the bin-list entries whose rect meets this tile, in list order
        const uint32_t j = b + threadIdx.x;
        uint32_t r = 0u;
        uint2 rc = make_uint2(1u, 1u);
        bool pass = false;
        float2 exy;
        float4 eco;
        if (j < rg.y) {
            r = rec.info[vals[j]].x;   // the pair carries the record's compaction slot
            const float4 xr = reinterpret_cast<const float4*>(rec.line + r)[2];   // (x, y, rect)
            rc = make_uint2(__float_as_uint(xr.z), __float_as_uint(xr.w));
            pass = rect_meets(rc, bx0, bx1, by0, by1);
            if (pass) {
                exy = make_float2(xr.x, xr.y);
                eco = rec.line[r].conic;
                pass = ellipse_meets(exy, eco, max(bx0, (int)(rc.x & 0xffffu)), min(bx1, (int)(rc.x >> 16)),
                                     max(by0, (int)(rc.y & 0xffffu)), min(by1, (int)(rc.y >> 16)));
            }
        }
        int cnt;
        const int pos = block_compact<NT>(pass, &cnt);
        if (pass) {
            s_e[pos].xy = exy;
            s_e[pos].co = eco;
            s_e[pos].cz = rec.line[r].col;
            s_e[pos].rc = rc;
            s_e[pos].j = j;
        }
        __syncthreads();
        n_entries += (uint32_t)cnt;
        // every owned pixel is evaluated with predicated selects, no branch
        for (int k = 0; k < cnt; k++) {
            const uint2 rc = s_e[k].rc;
            const float2 xy = s_e[k].xy;
            const float4 co = s_e[k].co;
            const float4 cz = s_e[k].cz;
            const uint32_t jk = __builtin_amdgcn_readfirstlane(s_e[k].j) + 1u;
            // predicates combine with & (not &&): no per-pixel exec-mask branches
            const RectS rs = rect_scalar(rc);
            const bool colok = (px >= rs.x0) & (px <= rs.x1);   // counters only
            const FragCol fc = frag_col(fpx, xy, co);
            // rows known to lie inside the rect skip the counters' per-row compares
            const auto blend = [&](auto rows_in) {
#pragma unroll
                for (int q = 0; q < PPT; q++) {
                    const float raw = frag_raw(fc, co, (float)(py0 + q) - xy.y);
                    const float a = fminf(kAlphaMax, raw);
                    // the rect needs no test: outside it the exact alpha is at
                    // least 2.5 % below 1/255 (the projection's margins), so the
                    // alpha test rejects those pixels by itself; the counters
                    // still count candidates inside the rect
                    bool inr = colok;
                    if constexpr (COUNT && !decltype(rows_in)::value)
                        inr = inr & (py0 + q >= rs.y0) & (py0 + q <= rs.y1);
                    const bool ok = a >= kAlphaMin;
                    // T (1 - alpha), negative once stopped, so a stopped pixel
                    // never blends again
                    const float aT = a * T[q];
                    const float Tn = T[q] - aT;
                    const bool stop = ok & (Tn < kTMin);
                    const bool bl = ok & !stop;
                    if (COUNT) {
                        n_visit += (inr & (T[q] > 0.f)) ? 1u : 0u;
                        n_blend += bl ? 1u : 0u;
                    }
                    const float w = bl ? aT : 0.f;
                    T[q] = bl ? Tn : (stop ? -fabsf(T[q]) : T[q]);
                    lastp[q] = bl ? jk : lastp[q];
                    C0[q] += cz.x * w;
                    C1[q] += cz.y * w;
                    C2[q] += cz.z * w;
                    D[q] += cz.w * w;
                }
            };
            if (!COUNT || (rs.y0 <= wy0 && rs.y1 >= wy1)) blend(std::true_type{});
            else blend(std::false_type{});
        }
        all_done = true;
#pragma unroll
        for (int q = 0; q < PPT; q++) all_done = all_done && T[q] < 0.f;
    }
    const int64_t hw = (int64_t)vi.W * vi.H;
    float lc = 0.f, ld = 0.f;
#pragma unroll
    for (int q = 0; q < PPT; q++) {
        const int py = py0 + q;
        if (!(px < vi.W && py < vi.H)) continue;
        T[q] = fabsf(T[q]);
        const int64_t pl = (int64_t)py * vi.W + px;
        const int64_t pi = (int64_t)vi.pix_off + pl;
        const int64_t ci = 3 * (int64_t)vi.pix_off + pl;
        color[ci] = C0[q];
        color[ci + hw] = C1[q];
        color[ci + 2 * hw] = C2[q];
        depth[pi] = D[q];
        alpha[pi] = 1.f - T[q];
        tfin[pi] = T[q];
        last[pi] = lastp[q];
        if (LOSS) {
            const float t0 = la.tc[ci], t1 = la.tc[ci + hw], t2 = la.tc[ci + 2 * hw], td = la.td[pi];
            float m = la.mask ? la.mask[pi] : 1.f;
            if (la.use_gate && !(td > 0.f && D[q] > 0.f && (1.f - T[q]) > la.gamma)) m = 0.f;
            const float e0 = C0[q] - t0, e1 = C1[q] - t1, e2 = C2[q] - t2, ed = D[q] - td;
            la.dC[ci] = vi.lsc * m * sgnf(e0);
            la.dC[ci + hw] = vi.lsc * m * sgnf(e1);
            la.dC[ci + 2 * hw] = vi.lsc * m * sgnf(e2);
            la.dD[pi] = vi.lsd * m * sgnf(ed);
            lc += m * (fabsf(e0) + fabsf(e1) + fabsf(e2));
            ld += m * fabsf(ed);
        }
    }
    if (threadIdx.x == 0) work[t] = n_entries;   // orders the backward
    if (LOSS && la.g2) {
        const int64_t m = (int64_t)*la.nvis * (kG2Floats / 4);
        for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < m; i += (int64_t)gridDim.x * NT)
            reinterpret_cast<float4*>(la.g2)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (LOSS) {
        const double2 s = block_sum2<NT>(lc, ld);
        if (threadIdx.x == 0) la.tile_part[t] = s;
    }
    if (COUNT) {
        const double2 s = block_sum2<NT>((float)n_visit, (float)n_blend);
        if (threadIdx.x == 0) {
            atomicAdd(counts, (unsigned long long)s.x);
            atomicAdd(counts + 1, (unsigned long long)s.y);
            atomicAdd(counts + 2, (unsigned long long)n_entries);   // entries this tile composited
            atomicAdd(counts + 3, (unsigned long long)(rg.y - rg.x));  // its bin's list length
        }
    }
}

// At most 128 VGPRs (four waves per SIMD): left to itself the compiler takes
// 140 for the 8-pixel shapes, which leaves room for three, and the kernel
// fits in 128 without spilling.
template <int TW, int TH, int PPT>
__global__ __launch_bounds__(TW* TH / PPT) __attribute__((amdgpu_waves_per_eu(4))) void composite_bwd_kernel(ViewTable vt, const uint2* __restrict__ ranges,
                                                                     const uint32_t* __restrict__ vals, Records rec,
                                                                     const float* __restrict__ tfin,
                                                                     const uint32_t* __restrict__ last,
                                                                     const float* __restrict__ dC,
                                                                     const float* __restrict__ dD,
                                                                     const float* __restrict__ dA, float* g2,
                                                                     const uint32_t* __restrict__ order) {
    constexpr int NT = TW * TH / PPT;
    static_assert(64 % TW == 0 && NT % 64 == 0, "a wavefront spans whole rows of the tile");
    constexpr int NG = 10;
    __shared__ float2 s_xy[NT];
    __shared__ float4 s_co[NT];
    __shared__ float4 s_cz[NT];
    __shared__ uint32_t s_id[NT];
    __shared__ float s_g[NT][NG];
    __shared__ uint32_t s_hi;
    const int t = order ? (int)order[blockIdx.x] : (int)blockIdx.x;   // heaviest tiles first when ordered
    const int v = view_of_tile(vt, t);
    const ViewInfo& vi = vt.v[v];
    const int lt = t - vi.tile_off;
    const int tyi = lt / vi.tiles_x, txi = lt - tyi * vi.tiles_x;
    const int px = txi * TW + (int)(threadIdx.x % TW);
    const int py0 = tyi * TH + (int)(threadIdx.x / TW) * PPT;
    const float fpx = (float)px;
    const uint2 rg = ranges[bin_of_tile(vt, vi, txi, tyi, TW, TH)];
    const int bx0 = txi * TW, bx1 = bx0 + TW - 1, by0 = tyi * TH, by1 = by0 + TH - 1;
    __shared__ uint32_t s_j[NT];
    const int lane = threadIdx.x & 63;
    const int slot = rs_slot(lane);
    const int64_t hw = (int64_t)vi.W * vi.H;

    // per pixel: transmittance, upstream gradients, and Q = sum over the
    // fragments behind the current one of (dL/dC . colour + dL/dD z) w,
    // started at -dL/dA T_final (dA/dalpha_i = T_final / (1 - alpha_i)), so
    // that T_{i+1} gcol_i - Q is the numerator of dL/dalpha_i
    float T[PPT], g0[PPT], g1[PPT], g2c[PPT], gd[PPT], Q[PPT];
    uint32_t lastp[PPT];
    uint32_t mylast = 0u;
#pragma unroll
    for (int q = 0; q < PPT; q++) {
        T[q] = 1.f;
        g0[q] = g1[q] = g2c[q] = gd[q] = 0.f;
        Q[q] = 0.f;
        lastp[q] = 0u;
        const int py = py0 + q;
        if (px < vi.W && py < vi.H) {
            const int64_t pl = (int64_t)py * vi.W + px;
            const int64_t pi = (int64_t)vi.pix_off + pl;
            const int64_t ci = 3 * (int64_t)vi.pix_off + pl;
            T[q] = tfin[pi];
            lastp[q] = last[pi];
            if (dC) { g0[q] = dC[ci]; g1[q] = dC[ci + hw]; g2c[q] = dC[ci + 2 * hw]; }
            if (dD) gd[q] = dD[pi];
            if (dA) Q[q] = -(dA[pi] * T[q]);
            mylast = max(mylast, lastp[q]);
        }
        // a pixel that blended nothing (or lies outside the image) carries
        // zero transmittance and zero upstream gradients, so evaluating it
        // adds exact zeros
        if (lastp[q] == 0u) T[q] = g0[q] = g1[q] = g2c[q] = gd[q] = Q[q] = 0.f;
    }
    // the smallest stop index among this wavefront's pixels that blended
    // something: entries before it need no per-pixel stop test
    uint32_t wmin = 0xffffffffu;
#pragma unroll
    for (int q = 0; q < PPT; q++) wmin = min(wmin, lastp[q] ? lastp[q] : 0xffffffffu);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wmin = min(wmin, (uint32_t)__shfl_xor((int)wmin, o, 64));
    wmin = __builtin_amdgcn_readfirstlane(wmin);
    if (threadIdx.x == 0) s_hi = rg.x;
    for (int i = threadIdx.x; i < NT * NG; i += NT) (&s_g[0][0])[i] = 0.f;
    __syncthreads();
    if (mylast > rg.x) atomicMax(&s_hi, mylast);
    __syncthreads();
    const uint32_t hi0 = s_hi;

    for (uint32_t hi = hi0; hi > rg.x;) {
        const uint32_t lo = (hi - rg.x > (uint32_t)NT) ? hi - NT : rg.x;
        const int span = (int)(hi - lo);
        // stage, back to front, the entries whose rect meets this tile
        const uint32_t jj = hi - 1u - threadIdx.x;
        uint32_t r = 0u, o = 0u;
        uint2 rc0 = make_uint2(1u, 1u);
        bool pass = false;
        float2 exy;
        float4 eco;
        if ((int)threadIdx.x < span) {
            o = vals[jj];              // the record's compaction slot (its gradient sums')
            r = rec.info[o].x;
            const float4 xr = reinterpret_cast<const float4*>(rec.line + r)[2];   // (x, y, rect)
            rc0 = make_uint2(__float_as_uint(xr.z), __float_as_uint(xr.w));
            pass = rect_meets(rc0, bx0, bx1, by0, by1);
            if (pass) {
                exy = make_float2(xr.x, xr.y);
                eco = rec.line[r].conic;
                pass = ellipse_meets(exy, eco, max(bx0, (int)(rc0.x & 0xffffu)), min(bx1, (int)(rc0.x >> 16)),
                                     max(by0, (int)(rc0.y & 0xffffu)), min(by1, (int)(rc0.y >> 16)));
            }
        }
        int cnt;
        const int pos = block_compact<NT>(pass, &cnt);
        if (pass) {
            s_id[pos] = o;
            s_j[pos] = jj;
            s_xy[pos] = exy;
            s_co[pos] = eco;
            s_cz[pos] = rec.line[r].col;
        }
        __syncthreads();
        // the wavefront reduction of an entry's gradients runs one blended
        // entry late, beside the next one's arithmetic (they are independent,
        // so the cross-lane steps no longer wait on each other alone); the
        // first reduction of a chunk adds zeros to entry 0
        float gp[NG];
#pragma unroll
        for (int e = 0; e < NG; e++) gp[e] = 0.f;
        int kp = 0;
        for (int k = 0; k < cnt; k++) {
            const uint32_t j = __builtin_amdgcn_readfirstlane(s_j[k]);
            const float2 xy = s_xy[k];
            const float4 co = s_co[k];
            const float4 cz = s_cz[k];
            // past every stop index of this thread the column gets an infinite
            // exponent, so its alpha is exactly zero
            FragCol fc = frag_col(fpx, xy, co);
            if (!(j < mylast)) fc.a0 = __builtin_inff();
            // pass 1: the alpha of every owned pixel, zeroed past the pixel's
            // stop index (where the forward did not blend it); min(0.99, raw)
            // >= 1/255 exactly when raw >= 1/255.  The rect needs no test, as
            // in the forward: outside it raw < 1/255 by the projection's
            // margins.  Entries before every pixel's stop index need no
            // per-pixel test at all.
            float raw[PPT];
            if (j < wmin) {
#pragma unroll
                for (int q = 0; q < PPT; q++) raw[q] = frag_raw(fc, co, (float)(py0 + q) - xy.y);
            } else {
#pragma unroll
                for (int q = 0; q < PPT; q++) {
                    const float r = frag_raw(fc, co, (float)(py0 + q) - xy.y);
                    raw[q] = (j < lastp[q]) ? r : 0.f;
                }
            }
            float rmax = raw[0];
#pragma unroll
            for (int q = 1; q < PPT; q++) rmax = fmaxf(rmax, raw[q]);
            if (__ballot(rmax >= kAlphaMin) == 0ull) continue;   // no pixel of the wavefront blended it
            // pass 2: gradients.  A pixel that did not blend the entry gets
            // alpha 0, so its transmittance is divided by exactly 1 and its
            // weight is 0; a clamped alpha (0.99) does not depend on opacity
            // or sigma, so its raw value is zeroed for the sigma gradient.
            // Sums over this thread's pixels (the column, dx, is shared) of
            // dL/dsigma times 1, q and q^2, with dy = dy0 + q.
            float s0 = 0.f, s1 = 0.f, s2 = 0.f;
            float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f, gcd = 0.f;
#pragma unroll
            for (int q = 0; q < PPT; q++) {
                const bool ok = raw[q] >= kAlphaMin;
                const float a = ok ? __builtin_amdgcn_fmed3f(raw[q], 0.f, kAlphaMax) : 0.f;
                const float rsig = (ok & (raw[q] <= kAlphaMax)) ? raw[q] : 0.f;
                const float inv = __builtin_amdgcn_rcpf(1.f - a);
                const float Ti = T[q] * inv;
                const float gcol = g0[q] * cz.x + g1[q] * cz.y + g2c[q] * cz.z + gd[q] * cz.w;
                // dL/dalpha_i = (T_{i+1} gcol - Q) / (1 - alpha_i)
                const float dal = inv * (T[q] * gcol - Q[q]);
                const float wk = a * Ti;
                gc0 += wk * g0[q];
                gc1 += wk * g1[q];
                gc2 += wk * g2c[q];
                gcd += wk * gd[q];
                Q[q] += wk * gcol;
                T[q] = Ti;
                const float dsig = -dal * rsig;   // dL/dsigma
                s0 += dsig;
                if (q > 0) {
                    s1 += (float)q * dsig;
                    s2 += (float)(q * q) * dsig;
                }
            }
            const float dy0 = (float)py0 - xy.y;
            const float s_ds = s0;
            const float s_dsdy = dy0 * s0 + s1;
            const float s_dsdy2 = dy0 * (dy0 * s0 + 2.f * s1) + s2;
            // moments of dL/dsigma over the pixels; the conic factors, the
            // same for every pixel, are applied once per entry at write-back
            const float dx = fc.dx;
            float gv[NG];
            gv[0] = dx * s_ds;
            gv[1] = s_dsdy;
            gv[2] = dx * gv[0];
            gv[3] = dx * s_dsdy;
            gv[4] = s_dsdy2;
            gv[5] = s_ds;
            gv[6] = gc0;
            gv[7] = gc1;
            gv[8] = gc2;
            gv[9] = gcd;
            const float s = row_reduce_scatter10(gp, lane);
            if (slot >= 0) atomicAdd(&s_g[kp][slot], s);
#pragma unroll
            for (int e = 0; e < NG; e++) gp[e] = gv[e];
            kp = k;
        }
        {
            const float s = row_reduce_scatter10(gp, lane);
            if (slot >= 0) atomicAdd(&s_g[kp][slot], s);
        }
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            float* dst = g2 + (int64_t)s_id[threadIdx.x] * kG2Floats;
            // d sigma / d mean is linear in (dx, dy) with the entry's conic
            // coefficients, which every pixel shares, so the mean gradient is
            // those coefficients applied to the two summed moments; slot 5
            // holds the plain sum of dL/dsigma, whose negative is the opacity
            // term.  Constant factors are applied by the projection backward.
            const float4 co = s_co[threadIdx.x];
            const float hb = 0.5f * co.y;
            const float m_dx = s_g[threadIdx.x][0], m_dy = s_g[threadIdx.x][1];
            s_g[threadIdx.x][0] = -(co.x * m_dx + hb * m_dy);
            s_g[threadIdx.x][1] = -(co.z * m_dy + hb * m_dx);
            s_g[threadIdx.x][5] = -s_g[threadIdx.x][5];
#pragma unroll
            for (int e = 0; e < NG; e++) {
                const float s = s_g[threadIdx.x][e];
                if (s != 0.f) atomicAdd(dst + e, s);
                s_g[threadIdx.x][e] = 0.f;
            }
        }
        __syncthreads();
        hi = lo;
    }
}

// Heaviest tiles first (longest-processing-time order).  Workgroups start in
// blockIdx order, so a tile with a long list that started late would finish
// long after the rest of the grid.  One workgroup buckets the tiles by a work
// estimate in quarter octaves, descending, with LDS counters: the bin's list
// length before the forward, the entries the forward staged before the
// backward.  Order inside a bucket is arbitrary; no result depends on it.
constexpr int kOrderBuckets = 128;
constexpr int kOrderThreads = 1024;

// Per-view tile geometry of the ordering kernel, staged in LDS once so that
// the per-tile lookups (a binary search over the views, the tile grids) do
// not each wait on loads of the kernel arguments.
struct OrderViews {
    int toff[kMaxViews], tx[kMaxViews];                 // tiles being ordered
    int ftoff[kMaxViews], ftx[kMaxViews], fty[kMaxViews];   // forward tiles (work counts)
    int boff[kMaxViews], bx[kMaxViews];                 // bins
};

// work estimate of tile t of vt: with `work` (per tile of vtf, the forward's
// tiling), the sum over the forward tiles that overlap it; else its bin's
// list length
__device__ __forceinline__ int order_bucket(const ViewTable& vt, const TileGrid& vtf, const OrderViews& ov,
                                            const uint2* ranges, const uint32_t* work, int t) {
    int lo = 0, hi = vt.V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ov.toff[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int v = lo;
    const int lt = t - ov.toff[v];
    const int tyi = lt / ov.tx[v], txi = lt - tyi * ov.tx[v];
    uint32_t w = 0u;
    if (work) {
        const int x0 = txi * vt.tw, y0 = tyi * vt.th;
        const int fx0 = x0 / vtf.tw, fy0 = y0 / vtf.th;
        const int fx1 = min((x0 + vt.tw - 1) / vtf.tw, ov.ftx[v] - 1);
        const int fy1 = min((y0 + vt.th - 1) / vtf.th, ov.fty[v] - 1);
        for (int fy = fy0; fy <= fy1; fy++)
            for (int fx = fx0; fx <= fx1; fx++) w += work[ov.ftoff[v] + fy * ov.ftx[v] + fx];
    } else {
        const uint2 rg = ranges[ov.boff[v] + ((tyi * vt.th) / vt.bh) * ov.bx[v] + (txi * vt.tw) / vt.bw];
        w = rg.y - rg.x;
    }
    // 4 log2(w + 1) in whole steps: exponent and top two mantissa bits
    const uint32_t b = (__float_as_uint((float)w + 1.f) >> 21) - (127u << 2);
    return kOrderBuckets - 1 - (int)min(b, (uint32_t)(kOrderBuckets - 1));
}

// Per-view tile geometry of the ordering, staged in LDS by each block
__device__ __forceinline__ void stage_order_views(const ViewTable& vt, const TileGrid& vtf, OrderViews& ov,
                                                  int nthreads) {
    for (int v = threadIdx.x; v < vt.V; v += nthreads) {
        ov.toff[v] = vt.v[v].tile_off; ov.tx[v] = vt.v[v].tiles_x;
        ov.ftoff[v] = vtf.tile_off[v]; ov.ftx[v] = vtf.tiles_x[v]; ov.fty[v] = vtf.tiles_y[v];
        ov.boff[v] = vt.v[v].bin_off; ov.bx[v] = vt.v[v].bins_x;
    }
}

// the work bucket of every tile, one thread per tile over many workgroups (a
// tile's estimate sums several forward tiles' counts: one workgroup issuing
// them in sequence was the ordering's whole cost)
constexpr int kBucketThreads = 256;
__global__ __launch_bounds__(kBucketThreads) void tile_bucket_kernel(ViewTable vt, TileGrid vtf,
                                                                     const uint2* __restrict__ ranges,
                                                                     const uint32_t* __restrict__ work,
                                                                     uint8_t* __restrict__ bucket) {
    __shared__ OrderViews ov;
    stage_order_views(vt, vtf, ov, kBucketThreads);
    __syncthreads();
    const int t = blockIdx.x * kBucketThreads + threadIdx.x;
    if (t < vt.n_tiles) bucket[t] = (uint8_t)order_bucket(vt, vtf, ov, ranges, work, t);
}

// a counting sort of the tiles by bucket, in one workgroup
__global__ __launch_bounds__(kOrderThreads) void order_tiles_kernel(int n, const uint8_t* __restrict__ bucket,
                                                                    uint32_t* __restrict__ order) {
    __shared__ uint32_t cnt[kOrderBuckets];
    constexpr int kKeep = 8;   // buckets a thread keeps for the second pass
    for (int i = threadIdx.x; i < kOrderBuckets; i += kOrderThreads) cnt[i] = 0u;
    __syncthreads();
    int keep[kKeep];
#pragma unroll
    for (int k = 0; k < kKeep; k++) {
        const int t = threadIdx.x + k * kOrderThreads;
        keep[k] = t < n ? (int)bucket[t] : 0;
    }
#pragma unroll
    for (int k = 0; k < kKeep; k++)
        if (threadIdx.x + k * kOrderThreads < n) atomicAdd(&cnt[keep[k]], 1u);
    for (int t = threadIdx.x + kKeep * kOrderThreads; t < n; t += kOrderThreads) atomicAdd(&cnt[bucket[t]], 1u);
    __syncthreads();
    static_assert(kOrderBuckets == 128, "two buckets per lane of one wavefront");
    if (threadIdx.x < 64) {
        // exclusive scan of the bucket counts by the first wavefront
        const int l = threadIdx.x;
        const uint32_t a = cnt[2 * l], b = cnt[2 * l + 1];
        uint32_t x = a + b;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (l >= o) x += y;
        }
        const uint32_t ex = x - (a + b);
        cnt[2 * l] = ex;
        cnt[2 * l + 1] = ex + a;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kKeep; k++) {
        const int t = threadIdx.x + k * kOrderThreads;
        if (t < n) order[atomicAdd(&cnt[keep[k]], 1u)] = (uint32_t)t;
    }
    for (int t = threadIdx.x + kKeep * kOrderThreads; t < n; t += kOrderThreads)
        order[atomicAdd(&cnt[bucket[t]], 1u)] = (uint32_t)t;
}

template <int TW, int TH, int PPT>
hipError_t fwd_t(const ViewTable& vt, const uint2* ranges, const uint32_t* vals, const Records& rec, float* color,
                 float* depth, float* alpha, float* tfin, uint32_t* last, const LossArgs* loss, const TileSched& ts,
                 unsigned long long* counts, hipStream_t s) {
    if (vt.n_tiles == 0) return hipSuccess;
    constexpr int NT = TW * TH / PPT;
    const LossArgs la = loss ? *loss : LossArgs{};
    if (loss && counts)
        composite_fwd_kernel<TW, TH, PPT, true, true><<<vt.n_tiles, NT, 0, s>>>(
            vt, ranges, vals, rec, color, depth, alpha, tfin, last, la, nullptr, ts.work, counts);
    else if (loss)
        composite_fwd_kernel<TW, TH, PPT, true, false><<<vt.n_tiles, NT, 0, s>>>(
            vt, ranges, vals, rec, color, depth, alpha, tfin, last, la, nullptr, ts.work, counts);
    else if (counts)
        composite_fwd_kernel<TW, TH, PPT, false, true><<<vt.n_tiles, NT, 0, s>>>(
            vt, ranges, vals, rec, color, depth, alpha, tfin, last, la, nullptr, ts.work, counts);
    else
        composite_fwd_kernel<TW, TH, PPT, false, false><<<vt.n_tiles, NT, 0, s>>>(
            vt, ranges, vals, rec, color, depth, alpha, tfin, last, la, nullptr, ts.work, counts);
    return hipGetLastError();
}

template <int TW, int TH, int PPT>
hipError_t bwd_t(const ViewTable& vt, const uint2* ranges, const uint32_t* vals, const Records& rec,
                 const float* tfin, const uint32_t* last, const float* dC, const float* dD, const float* dA,
                 float* g2, const TileSched& ts, const ViewTable& vtf, bool ordered, hipStream_t s) {
    if (vt.n_tiles == 0) return hipSuccess;
    constexpr int NT = TW * TH / PPT;
    if (!ordered) {
        const hipError_t e = launch_order_tiles(vt, vtf, ranges, ts, s);
        if (e != hipSuccess) return e;
    }
    composite_bwd_kernel<TW, TH, PPT><<<vt.n_tiles, NT, 0, s>>>(vt, ranges, vals, rec, tfin, last, dC, dD, dA, g2,
                                                                 ts.order);
    return hipGetLastError();
}

}  // namespace

// (tile width, tile height, pixels per thread) combinations with whole
// wavefronts per workgroup
#define GS_TILE_DISPATCH(FN, ...)                                                   \
    if (vt.tw == 16 && vt.th == 16 && vt.ppt == 1) return FN<16, 16, 1>(__VA_ARGS__); \
    if (vt.tw == 16 && vt.th == 16 && vt.ppt == 2) return FN<16, 16, 2>(__VA_ARGS__); \
    if (vt.tw == 16 && vt.th == 16 && vt.ppt == 4) return FN<16, 16, 4>(__VA_ARGS__); \
    if (vt.tw == 16 && vt.th == 8 && vt.ppt == 1) return FN<16, 8, 1>(__VA_ARGS__);   \
    if (vt.tw == 16 && vt.th == 8 && vt.ppt == 2) return FN<16, 8, 2>(__VA_ARGS__);   \
    if (vt.tw == 8 && vt.th == 8 && vt.ppt == 1) return FN<8, 8, 1>(__VA_ARGS__);     \
    if (vt.tw == 32 && vt.th == 8 && vt.ppt == 1) return FN<32, 8, 1>(__VA_ARGS__);   \
    if (vt.tw == 32 && vt.th == 8 && vt.ppt == 2) return FN<32, 8, 2>(__VA_ARGS__);   \
    if (vt.tw == 32 && vt.th == 8 && vt.ppt == 4) return FN<32, 8, 4>(__VA_ARGS__);   \
    if (vt.tw == 32 && vt.th == 16 && vt.ppt == 1) return FN<32, 16, 1>(__VA_ARGS__); \
    if (vt.tw == 32 && vt.th == 16 && vt.ppt == 2) return FN<32, 16, 2>(__VA_ARGS__); \
    if (vt.tw == 32 && vt.th == 16 && vt.ppt == 4) return FN<32, 16, 4>(__VA_ARGS__); \
    if (vt.tw == 32 && vt.th == 16 && vt.ppt == 8) return FN<32, 16, 8>(__VA_ARGS__); \
    if (vt.tw == 32 && vt.th == 32 && vt.ppt == 4) return FN<32, 32, 4>(__VA_ARGS__); \
    if (vt.tw == 32 && vt.th == 32 && vt.ppt == 8) return FN<32, 32, 8>(__VA_ARGS__); \
    if (vt.tw == 32 && vt.th == 64 && vt.ppt == 8) return FN<32, 64, 8>(__VA_ARGS__); \
    if (vt.tw == 64 && vt.th == 32 && vt.ppt == 8) return FN<64, 32, 8>(__VA_ARGS__); \
    if (vt.tw == 64 && vt.th == 64 && vt.ppt == 8) return FN<64, 64, 8>(__VA_ARGS__); \
    return hipErrorInvalidValue;

hipError_t launch_composite_fwd(const ViewTable& vt, const uint2* ranges, const uint32_t* vals, const Records& rec,
                                float* color, float* depth, float* alpha, float* tfin, uint32_t* last,
                                const LossArgs* loss, const TileSched& ts, hipStream_t s,
                                unsigned long long* counts) {
    GS_TILE_DISPATCH(fwd_t, vt, ranges, vals, rec, color, depth, alpha, tfin, last, loss, ts, counts, s)
}

hipError_t launch_composite_bwd(const ViewTable& vt, const uint2* ranges, const uint32_t* vals, const Records& rec,
                                const float* tfin, const uint32_t* last, const float* dC, const float* dD,
                                const float* dA, float* g2, const TileSched& ts, const ViewTable& vtf,
                                bool ordered, hipStream_t s) {
    GS_TILE_DISPATCH(bwd_t, vt, ranges, vals, rec, tfin, last, dC, dD, dA, g2, ts, vtf, ordered, s)
}

hipError_t launch_order_tiles(const ViewTable& vt, const ViewTable& vtf, const uint2* ranges, const TileSched& ts,
                              hipStream_t s) {
    if (vt.n_tiles == 0) return hipSuccess;
    tile_bucket_kernel<<<(unsigned)((vt.n_tiles + kBucketThreads - 1) / kBucketThreads), kBucketThreads, 0, s>>>(
        vt, tile_grid(vtf), ranges, ts.work, ts.bucket);
    order_tiles_kernel<<<1, kOrderThreads, 0, s>>>(vt.n_tiles, ts.bucket, ts.order);
    return hipGetLastError();
}

#undef GS_TILE_DISPATCH

}  // namespace gs
