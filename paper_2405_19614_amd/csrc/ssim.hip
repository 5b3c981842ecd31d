// SSIM term of the mapping loss (Sec. 3.4, mapping-loss equation) on the RGB
// render.  The paper names the term without defining it; the kernels compute
// the usual structural similarity per colour channel with an 11 x 11 Gaussian
// window (standard deviation 1.5 px), C1 = 0.01^2, C2 = 0.03^2, and windows
// clipped at the image border by zero padding.  L_SSIM of a view is 1 - the
// mean over its pixels and channels.
//
// Two launches, each one workgroup per (32 x 16 output tile, colour channel)
// of every view:
// the forward stages the tile and a 5-pixel halo of both images in LDS, forms
// the five window means (x, y, x^2, y^2, xy) with a separable pass (rows, then
// columns), and writes per pixel the SSIM map's partial derivatives with
// respect to the three window means that depend on x; the backward applies
// the same separable window to those partials (the zero-padded window
// correlation is its own transpose) and adds the gradient to dL/dimg.
// Their HBM traffic is the minimum (each input read once, the partials
// written and read once); neither cutting their LDS reads to a third nor
// overlapping one item's staging with the previous item's arithmetic sped
// them up.  Vector issue, at about half the peak over six workgroups per CU,
// is what they spend their time on.
#include <cmath>

#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kR = 5;                       // window radius
constexpr int kW = 2 * kR + 1;              // taps
constexpr int kTW = kSsimTW, kTH = kSsimTH; // outputs per workgroup
constexpr int kRW = kTW + 2 * kR;           // staged region width
constexpr int kRH = kTH + 2 * kR;           // staged region height
constexpr int kNT = 256;
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Window {
    float g[kW];
};

Window make_window() {
    double g[kW], sum = 0.0;
    for (int i = 0; i < kW; i++) {
        const double x = i - kR;
        g[i] = std::exp(-x * x / (2.0 * 1.5 * 1.5));
        sum += g[i];
    }
    Window w;
    for (int i = 0; i < kW; i++) w.g[i] = (float)(g[i] / sum);
    return w;
}

__device__ __forceinline__ int view_of_ssim_tile(const ViewTable& vt, int t) {
    int lo = 0, hi = vt.V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (vt.v[mid].ssim_off <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

struct TileGeom {
    int v, tx, ty;
    int64_t hw;
};

__device__ __forceinline__ TileGeom tile_geom(const ViewTable& vt, int t) {
    TileGeom g;
    g.v = view_of_ssim_tile(vt, t);
    const ViewInfo& vi = vt.v[g.v];
    const int lt = t - vi.ssim_off;
    const int tiles_x = (vi.W + kTW - 1) / kTW;
    g.ty = lt / tiles_x;
    g.tx = lt - g.ty * tiles_x;
    g.hw = (int64_t)vi.W * vi.H;
    return g;
}

// Stage rows [ty*TH - R, ...) x cols [tx*TW - R, ...) of NP image planes
// (zero outside the image).  Every load of a thread is issued before the
// first LDS store, so the staging costs one memory latency, not one per
// element.
constexpr int kStageIters = (kRH * kRW + kNT - 1) / kNT;

template <int NP>
__device__ __forceinline__ void stage(float (*const (&dst)[NP])[kRW], const float* const (&src)[NP],
                                      const ViewInfo& vi, const TileGeom& g) {
    const int x0 = g.tx * kTW - kR, y0 = g.ty * kTH - kR;
    float val[NP][kStageIters];
#pragma unroll
    for (int it = 0; it < kStageIters; it++) {
        const int i = threadIdx.x + it * kNT;
        const int r = i / kRW, c = i - r * kRW;
        const int gx = x0 + c, gy = y0 + r;
        const bool in = i < kRH * kRW && gx >= 0 && gx < vi.W && gy >= 0 && gy < vi.H;
        const int64_t o = in ? (int64_t)gy * vi.W + gx : 0;
#pragma unroll
        for (int q = 0; q < NP; q++) val[q][it] = in ? src[q][o] : 0.f;
    }
#pragma unroll
    for (int it = 0; it < kStageIters; it++) {
        const int i = threadIdx.x + it * kNT;
        if (i < kRH * kRW) {
            const int r = i / kRW, c = i - r * kRW;
#pragma unroll
            for (int q = 0; q < NP; q++) dst[q][r][c] = val[q][it];
        }
    }
}

__global__ __launch_bounds__(kNT) void ssim_fwd_kernel(ViewTable vt, Window w, const float* __restrict__ img,
                                                       const float* __restrict__ ref, float* __restrict__ part,
                                                       double* __restrict__ tile_sum) {
    __shared__ float sx[kRH][kRW], sy[kRH][kRW];
    __shared__ float hm[5][kRH][kTW];
    __shared__ double red[kNT / 64];
    // (channel, tile) of this workgroup, contiguous per XCD
    const int item = (int)xcd_slot((int64_t)blockIdx.y * gridDim.x + blockIdx.x, 3 * (int64_t)vt.n_ssim_tiles);
    const int k = item / vt.n_ssim_tiles, tile = item - k * vt.n_ssim_tiles;
    const TileGeom g = tile_geom(vt, tile);
    const ViewInfo& vi = vt.v[g.v];
    const int64_t np = vt.n_pix;
    const int64_t plane = 3 * (int64_t)vi.pix_off + k * g.hw;
    {
        float (*const dst[2])[kRW] = {sx, sy};
        const float* const src[2] = {img + plane, ref + plane};
        stage<2>(dst, src, vi, g);
    }
    __syncthreads();
    // window means along rows
    for (int i = threadIdx.x; i < kRH * kTW; i += kNT) {
        const int r = i / kTW, c = i - r * kTW;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
        for (int j = 0; j < kW; j++) {
            const float wj = w.g[j], xv = sx[r][c + j], yv = sy[r][c + j];
            const float wx = wj * xv, wy = wj * yv;
            a0 += wx;
            a1 += wy;
            a2 += wx * xv;
            a3 += wy * yv;
            a4 += wx * yv;
        }
        hm[0][r][c] = a0; hm[1][r][c] = a1; hm[2][r][c] = a2; hm[3][r][c] = a3; hm[4][r][c] = a4;
    }
    __syncthreads();
    // then along columns, and the SSIM map with its partials
    float ssum = 0.f;
    for (int i = threadIdx.x; i < kTH * kTW; i += kNT) {
        const int r = i / kTW, c = i - r * kTW;
        const int gx = g.tx * kTW + c, gy = g.ty * kTH + r;
        if (gx >= vi.W || gy >= vi.H) continue;
        float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < kW; j++) {
            const float wj = w.g[j];
#pragma unroll
            for (int q = 0; q < 5; q++) m[q] += wj * hm[q][r + j][c];
        }
        const float mx = m[0], my = m[1];
        const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
        const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
        const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
        const float iD = 1.f / (B1 * B2);
        const float sv = A1 * A2 * iD;
        const int64_t o = plane + (int64_t)gy * vi.W + gx;
        part[o] = (2.f * my * (A2 - A1) - sv * 2.f * mx * (B2 - B1)) * iD;   // d s / d mean(x)
        part[o + 3 * np] = -sv * B1 * iD;                                    // d s / d mean(x^2)
        part[o + 6 * np] = 2.f * A1 * iD;                                     // d s / d mean(xy)
        ssum += sv;
    }
    // workgroup sum in FP64, one slot per (channel, tile)
    double d = (double)ssum;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < kNT / 64; i++) t += red[i];
        tile_sum[(int64_t)k * vt.n_ssim_tiles + tile] = t;
    }
}

__global__ __launch_bounds__(kNT) void ssim_bwd_kernel(ViewTable vt, Window w, const float* __restrict__ img,
                                                       const float* __restrict__ ref, const float* __restrict__ part,
                                                       const float* __restrict__ wdev, float wconst,
                                                       float* __restrict__ dimg) {
    __shared__ float sp[3][kRH][kRW];
    __shared__ float hm[3][kRH][kTW];
    // (channel, tile) of this workgroup, contiguous per XCD
    const int item = (int)xcd_slot((int64_t)blockIdx.y * gridDim.x + blockIdx.x, 3 * (int64_t)vt.n_ssim_tiles);
    const int k = item / vt.n_ssim_tiles, tile = item - k * vt.n_ssim_tiles;
    const TileGeom g = tile_geom(vt, tile);
    const ViewInfo& vi = vt.v[g.v];
    const int64_t np = vt.n_pix;
    const float wv = wdev ? wdev[g.v] : wconst;
    const float scale = -wv / (3.f * (float)g.hw);
    const int64_t plane = 3 * (int64_t)vi.pix_off + k * g.hw;
    {
        float (*const dst[3])[kRW] = {sp[0], sp[1], sp[2]};
        const float* const src[3] = {part + plane, part + 3 * np + plane, part + 6 * np + plane};
        stage<3>(dst, src, vi, g);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kRH * kTW; i += kNT) {
        const int r = i / kTW, c = i - r * kTW;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int j = 0; j < kW; j++) {
            const float wj = w.g[j];
            a0 += wj * sp[0][r][c + j];
            a1 += wj * sp[1][r][c + j];
            a2 += wj * sp[2][r][c + j];
        }
        hm[0][r][c] = a0; hm[1][r][c] = a1; hm[2][r][c] = a2;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTH * kTW; i += kNT) {
        const int r = i / kTW, c = i - r * kTW;
        const int gx = g.tx * kTW + c, gy = g.ty * kTH + r;
        if (gx >= vi.W || gy >= vi.H) continue;
        float b0 = 0.f, b1 = 0.f, b2 = 0.f;
#pragma unroll
        for (int j = 0; j < kW; j++) {
            const float wj = w.g[j];
            b0 += wj * hm[0][r + j][c];
            b1 += wj * hm[1][r + j][c];
            b2 += wj * hm[2][r + j][c];
        }
        const int64_t o = plane + (int64_t)gy * vi.W + gx;
        dimg[o] += scale * (b0 + 2.f * img[o] * b1 + ref[o] * b2);
    }
}

__global__ __launch_bounds__(256) void ssim_reduce_kernel(ViewTable vt, const double* __restrict__ tile_sum,
                                                          float* __restrict__ out) {
    __shared__ double red[256];
    for (int v = 0; v < vt.V; v++) {
        const ViewInfo& vi = vt.v[v];
        const int nt = ((vi.W + kTW - 1) / kTW) * ((vi.H + kTH - 1) / kTH);
        double a = 0.0;
        for (int i = threadIdx.x; i < 3 * nt; i += 256) {
            const int k = i / nt;
            a += tile_sum[(int64_t)k * vt.n_ssim_tiles + vi.ssim_off + (i - k * nt)];
        }
        red[threadIdx.x] = a;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[v] = (float)(red[0] / (3.0 * (double)vi.W * vi.H));
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_ssim_fwd(const ViewTable& vt, const float* img, const float* ref, float* part, double* tile_sum,
                           hipStream_t s) {
    if (vt.n_ssim_tiles == 0) return hipSuccess;
    static const Window w = make_window();
    ssim_fwd_kernel<<<dim3(vt.n_ssim_tiles, 3), kNT, 0, s>>>(vt, w, img, ref, part, tile_sum);
    return hipGetLastError();
}

hipError_t launch_ssim_bwd(const ViewTable& vt, const float* img, const float* ref, const float* part,
                           const float* wdev, float wconst, float* dimg, hipStream_t s) {
    if (vt.n_ssim_tiles == 0) return hipSuccess;
    static const Window w = make_window();
    ssim_bwd_kernel<<<dim3(vt.n_ssim_tiles, 3), kNT, 0, s>>>(vt, w, img, ref, part, wdev, wconst, dimg);
    return hipGetLastError();
}

hipError_t launch_ssim_reduce(const ViewTable& vt, const double* tile_sum, float* ssim_out, hipStream_t s) {
    ssim_reduce_kernel<<<1, 256, 0, s>>>(vt, tile_sum, ssim_out);
    return hipGetLastError();
}

}  // namespace gs
