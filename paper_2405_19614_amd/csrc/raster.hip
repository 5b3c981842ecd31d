// Tile compositing, forward and backward (Sec. 3.4 "Differentiable
// Rasterization": colour and depth compositing; Sec. 3.3 border mask).
//
// One workgroup per (view, tile) of every view in one launch; the tile's
// depth-ordered list is staged through LDS in batches of one record per
// thread.  Forward: front to back per pixel with a workgroup-wide early exit
// once every pixel has stopped; an optional fused epilogue writes the L1
// loss's upstream gradients and per-tile loss partials.  Backward: the same
// lists walked back to front from each pixel's stop index, transmittance
// recovered by division, per-Gaussian gradients reduced across the wavefront
// (64 lanes) and then across the workgroup in LDS before one global atomic
// per (tile, Gaussian, value).
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

template <int TW, int TH, bool LOSS, bool COUNT>
__global__ __launch_bounds__(TW* TH) void composite_fwd_kernel(ViewTable vt, const uint2* __restrict__ ranges,
                                                               const uint32_t* __restrict__ vals, Records rec,
                                                               float* color, float* depth, float* alpha,
                                                               float* tfin, uint32_t* last, LossArgs la,
                                                               unsigned long long* counts) {
    constexpr int NT = TW * TH;
    __shared__ float2 s_xy[NT];
    __shared__ float4 s_co[NT];
    __shared__ float4 s_cz[NT];
    __shared__ uint2 s_rc[NT];
    const int t = blockIdx.x;
    const int v = view_of_tile(vt, t);
    const ViewInfo& vi = vt.v[v];
    const int lt = t - vi.tile_off;
    const int tyi = lt / vi.tiles_x, txi = lt - tyi * vi.tiles_x;
    const int px = txi * TW + (int)(threadIdx.x % TW);
    const int py = tyi * TH + (int)(threadIdx.x / TW);
    const bool inside = px < vi.W && py < vi.H;
    const float fpx = (float)px, fpy = (float)py;
    const uint2 rg = ranges[t];

    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
    uint32_t lastp = 0u;
    uint32_t n_visit = 0u, n_blend = 0u;
    bool done = !inside;
    for (uint32_t b = rg.x; b < rg.y; b += NT) {
        if (__syncthreads_count(done) == NT) break;
        const uint32_t j = b + threadIdx.x;
        if (j < rg.y) {
            const uint32_t r = vals[j];
            s_xy[threadIdx.x] = rec.xy[r];
            s_co[threadIdx.x] = rec.conic[r];
            s_cz[threadIdx.x] = rec.col[r];
            s_rc[threadIdx.x] = rec.rect[r];
        }
        __syncthreads();
        const int cnt = (int)min((uint32_t)NT, rg.y - b);
        if (!done) {
            for (int k = 0; k < cnt; k++) {
                if (!rect_has(s_rc[k], px, py)) continue;
                if (COUNT) n_visit++;
                Frag f;
                if (!frag_eval(fpx, fpy, s_xy[k], s_co[k], f)) continue;
                const float Tn = T * (1.f - f.alpha);
                if (Tn < kTMin) { done = true; break; }
                if (COUNT) n_blend++;
                const float w = f.alpha * T;
                const float4 cz = s_cz[k];
                C0 += cz.x * w;
                C1 += cz.y * w;
                C2 += cz.z * w;
                D += cz.w * w;
                T = Tn;
                lastp = b + (uint32_t)k + 1u;
            }
        }
    }
    const int64_t hw = (int64_t)vi.W * vi.H;
    const int64_t pl = (int64_t)py * vi.W + px;
    const int64_t pi = (int64_t)vi.pix_off + pl;
    const int64_t ci = 3 * (int64_t)vi.pix_off + pl;
    float lc = 0.f, ld = 0.f;
    if (inside) {
        color[ci] = C0;
        color[ci + hw] = C1;
        color[ci + 2 * hw] = C2;
        depth[pi] = D;
        alpha[pi] = 1.f - T;
        tfin[pi] = T;
        last[pi] = lastp;
        if (LOSS) {
            const float t0 = la.tc[ci], t1 = la.tc[ci + hw], t2 = la.tc[ci + 2 * hw], td = la.td[pi];
            float m = la.mask ? la.mask[pi] : 1.f;
            if (la.use_gate && !(td > 0.f && D > 0.f && (1.f - T) > la.gamma)) m = 0.f;
            const float e0 = C0 - t0, e1 = C1 - t1, e2 = C2 - t2, ed = D - td;
            la.dC[ci] = vi.lsc * m * sgnf(e0);
            la.dC[ci + hw] = vi.lsc * m * sgnf(e1);
            la.dC[ci + 2 * hw] = vi.lsc * m * sgnf(e2);
            la.dD[pi] = vi.lsd * m * sgnf(ed);
            lc = m * (fabsf(e0) + fabsf(e1) + fabsf(e2));
            ld = m * fabsf(ed);
        }
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
        }
    }
}

__device__ __forceinline__ float wsum(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void composite_bwd_kernel(ViewTable vt, const uint2* __restrict__ ranges,
                                                               const uint32_t* __restrict__ vals, Records rec,
                                                               const float* __restrict__ tfin,
                                                               const uint32_t* __restrict__ last,
                                                               const float* __restrict__ dC,
                                                               const float* __restrict__ dD,
                                                               const float* __restrict__ dA, float* g2) {
    constexpr int NT = TW * TH;
    constexpr int NG = 10;
    __shared__ float2 s_xy[NT];
    __shared__ float4 s_co[NT];
    __shared__ float4 s_cz[NT];
    __shared__ uint2 s_rc[NT];
    __shared__ uint32_t s_id[NT];
    __shared__ float s_g[NT][NG];
    __shared__ uint32_t s_hi;
    const int t = blockIdx.x;
    const int v = view_of_tile(vt, t);
    const ViewInfo& vi = vt.v[v];
    const int lt = t - vi.tile_off;
    const int tyi = lt / vi.tiles_x, txi = lt - tyi * vi.tiles_x;
    const int px = txi * TW + (int)(threadIdx.x % TW);
    const int py = tyi * TH + (int)(threadIdx.x / TW);
    const bool inside = px < vi.W && py < vi.H;
    const float fpx = (float)px, fpy = (float)py;
    const uint2 rg = ranges[t];
    const int lane = threadIdx.x & 63;

    const int64_t hw = (int64_t)vi.W * vi.H;
    const int64_t pl = (int64_t)py * vi.W + px;
    const int64_t pi = (int64_t)vi.pix_off + pl;
    const int64_t ci = 3 * (int64_t)vi.pix_off + pl;
    float T = 1.f, Tf = 1.f, g0 = 0.f, g1 = 0.f, g2c = 0.f, gd = 0.f, ga = 0.f;
    uint32_t lastp = 0u;
    if (inside) {
        Tf = tfin[pi];
        T = Tf;
        lastp = last[pi];
        if (dC) { g0 = dC[ci]; g1 = dC[ci + hw]; g2c = dC[ci + 2 * hw]; }
        if (dD) gd = dD[pi];
        if (dA) ga = dA[pi];
    }
    if (threadIdx.x == 0) s_hi = rg.x;
    for (int i = threadIdx.x; i < NT * NG; i += NT) (&s_g[0][0])[i] = 0.f;
    __syncthreads();
    if (lastp > rg.x) atomicMax(&s_hi, lastp);
    __syncthreads();
    const uint32_t hi0 = s_hi;
    float S0 = 0.f, S1 = 0.f, S2 = 0.f, SD = 0.f;

    for (uint32_t hi = hi0; hi > rg.x;) {
        const uint32_t lo = (hi - rg.x > (uint32_t)NT) ? hi - NT : rg.x;
        const int cnt = (int)(hi - lo);
        // slot k holds list entry hi - 1 - k (back to front)
        if ((int)threadIdx.x < cnt) {
            const uint32_t r = vals[hi - 1u - threadIdx.x];
            s_id[threadIdx.x] = r;
            s_xy[threadIdx.x] = rec.xy[r];
            s_co[threadIdx.x] = rec.conic[r];
            s_cz[threadIdx.x] = rec.col[r];
            s_rc[threadIdx.x] = rec.rect[r];
        }
        __syncthreads();
        for (int k = 0; k < cnt; k++) {
            const uint32_t j = hi - 1u - (uint32_t)k;
            float gv[NG];
            bool any = false;
#pragma unroll
            for (int q = 0; q < NG; q++) gv[q] = 0.f;
            Frag f;
            if (j < lastp && rect_has(s_rc[k], px, py) && frag_eval(fpx, fpy, s_xy[k], s_co[k], f)) {
                const float4 co = s_co[k];
                const float4 cz = s_cz[k];
                const float inv = 1.f / (1.f - f.alpha);
                const float Ti = T * inv;
                const float w = f.alpha * Ti;
                gv[6] = w * g0;
                gv[7] = w * g1;
                gv[8] = w * g2c;
                gv[9] = w * gd;
                const float dal = inv * (g0 * (cz.x * T - S0) + g1 * (cz.y * T - S1) + g2c * (cz.z * T - S2) +
                                         gd * (cz.w * T - SD) + ga * Tf);
                S0 += cz.x * w;
                S1 += cz.y * w;
                S2 += cz.z * w;
                SD += cz.w * w;
                T = Ti;
                if (f.raw <= kAlphaMax) {
                    gv[5] = dal * f.G;
                    const float ds = -dal * f.raw;
                    gv[2] = 0.5f * ds * f.dx * f.dx;
                    gv[3] = ds * f.dx * f.dy;
                    gv[4] = 0.5f * ds * f.dy * f.dy;
                    gv[0] = -ds * (co.x * f.dx + co.y * f.dy);
                    gv[1] = -ds * (co.z * f.dy + co.y * f.dx);
                }
                any = true;
            }
            if (__ballot(any) != 0ull) {
#pragma unroll
                for (int q = 0; q < NG; q++) {
                    const float s = wsum(gv[q]);
                    if (lane == 0 && s != 0.f) atomicAdd(&s_g[k][q], s);
                }
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            float* dst = g2 + (int64_t)s_id[threadIdx.x] * kG2Stride;
#pragma unroll
            for (int q = 0; q < NG; q++) {
                const float s = s_g[threadIdx.x][q];
                if (s != 0.f) atomicAdd(dst + q, s);
                s_g[threadIdx.x][q] = 0.f;
            }
        }
        __syncthreads();
        hi = lo;
    }
}

template <int TW, int TH>
hipError_t fwd_t(const ViewTable& vt, const uint2* ranges, const uint32_t* vals, const Records& rec, float* color,
                 float* depth, float* alpha, float* tfin, uint32_t* last, const LossArgs* loss,
                 unsigned long long* counts, hipStream_t s) {
    if (vt.n_tiles == 0) return hipSuccess;
    const LossArgs la = loss ? *loss : LossArgs{};
    if (loss && counts)
        composite_fwd_kernel<TW, TH, true, true><<<vt.n_tiles, TW * TH, 0, s>>>(vt, ranges, vals, rec, color, depth,
                                                                                 alpha, tfin, last, la, counts);
    else if (loss)
        composite_fwd_kernel<TW, TH, true, false><<<vt.n_tiles, TW * TH, 0, s>>>(vt, ranges, vals, rec, color,
                                                                                  depth, alpha, tfin, last, la, counts);
    else if (counts)
        composite_fwd_kernel<TW, TH, false, true><<<vt.n_tiles, TW * TH, 0, s>>>(vt, ranges, vals, rec, color,
                                                                                  depth, alpha, tfin, last, la, counts);
    else
        composite_fwd_kernel<TW, TH, false, false><<<vt.n_tiles, TW * TH, 0, s>>>(vt, ranges, vals, rec, color,
                                                                                   depth, alpha, tfin, last, la, counts);
    return hipGetLastError();
}

template <int TW, int TH>
hipError_t bwd_t(const ViewTable& vt, const uint2* ranges, const uint32_t* vals, const Records& rec,
                 const float* tfin, const uint32_t* last, const float* dC, const float* dD, const float* dA,
                 float* g2, hipStream_t s) {
    if (vt.n_tiles == 0) return hipSuccess;
    composite_bwd_kernel<TW, TH><<<vt.n_tiles, TW * TH, 0, s>>>(vt, ranges, vals, rec, tfin, last, dC, dD, dA, g2);
    return hipGetLastError();
}

}  // namespace

#define GS_TILE_DISPATCH(FN, ...)                                        \
    if (vt.tw == 16 && vt.th == 16) return FN<16, 16>(__VA_ARGS__);      \
    if (vt.tw == 16 && vt.th == 8) return FN<16, 8>(__VA_ARGS__);        \
    if (vt.tw == 8 && vt.th == 8) return FN<8, 8>(__VA_ARGS__);          \
    if (vt.tw == 32 && vt.th == 8) return FN<32, 8>(__VA_ARGS__);        \
    if (vt.tw == 32 && vt.th == 16) return FN<32, 16>(__VA_ARGS__);      \
    return hipErrorInvalidValue;

hipError_t launch_composite_fwd(const ViewTable& vt, const uint2* ranges, const uint32_t* vals, const Records& rec,
                                float* color, float* depth, float* alpha, float* tfin, uint32_t* last,
                                const LossArgs* loss, hipStream_t s, unsigned long long* counts) {
    GS_TILE_DISPATCH(fwd_t, vt, ranges, vals, rec, color, depth, alpha, tfin, last, loss, counts, s)
}

hipError_t launch_composite_bwd(const ViewTable& vt, const uint2* ranges, const uint32_t* vals, const Records& rec,
                                const float* tfin, const uint32_t* last, const float* dC, const float* dD,
                                const float* dA, float* g2, hipStream_t s) {
    GS_TILE_DISPATCH(bwd_t, vt, ranges, vals, rec, tfin, last, dC, dD, dA, g2, s)
}

#undef GS_TILE_DISPATCH

}  // namespace gs
