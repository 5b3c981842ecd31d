// Map maintenance of the online reconstruction (Sec. 3.4): Gaussian pruning
// and densification, with the re-layout of the Adam moments both imply.
//
// Pruning removes the Gaussians whose opacity sigmoid(logit) is below tau
// (compared as logit < logit(tau)), keeping the order of the others: a flag
// per Gaussian, an exclusive scan, one scatter.  Densification appends one
// isotropic Gaussian for every pixel outside the border mask (rendered alpha
// <= gamma; every pixel on the first frame) that has a sensor depth: the
// pixel's sample point back-projected to that depth, radius depth / fx (a
// one-pixel footprint, Eq. d; every axis, or the one radius of the isotropic
// layout), identity rotation, opacity 1/2, the target
// colour (with SH, in the DC coefficient).  New Gaussians follow the existing
// ones in view, then row-major pixel order.
#include "gs_internal.h"

namespace gs {

namespace {

constexpr float kShC0 = 0.28209479177387814f;   // Y_00 of the real orthonormal SH basis

// sigmoid(logit) < tau  <=>  logit < logit(tau) (sigmoid is increasing); the
// FP32 logit is compared with logit(tau) in FP64, so the decision is that of
// the real numbers for every FP32 logit (none lies within FP64 rounding of
// logit(tau) unless it equals it)
__global__ void prune_flags_kernel(const float* __restrict__ opl, int64_t n, double logit_tau,
                                   uint32_t* __restrict__ flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = ((double)opl[i] >= logit_tau) ? 1u : 0u;
}

__global__ void prune_scatter_kernel(Params in, int K3, GaussOut out, const uint32_t* __restrict__ flag,
                                     const uint32_t* __restrict__ off) {
    const int64_t n = in.n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[i]) continue;
        const int64_t j = off[i];
#pragma unroll
        for (int e = 0; e < 3; e++) out.means[3 * j + e] = in.means[3 * i + e];
        if (in.iso) {
            out.ls[j] = in.ls[i];
        } else {
#pragma unroll
            for (int e = 0; e < 3; e++) out.ls[3 * j + e] = in.ls[3 * i + e];
#pragma unroll
            for (int e = 0; e < 4; e++) out.q[4 * j + e] = in.q[4 * i + e];
        }
        out.opl[j] = in.opl[i];
        for (int e = 0; e < K3; e++) out.col[K3 * j + e] = in.col[K3 * i + e];
    }
}

// moments of a kept Gaussian i -> new slot off[i]; the new count is *total
__global__ void prune_adam_kernel(AdamIO a, int64_t n, int K3, int iso, int V, const uint32_t* __restrict__ flag,
                                  const uint32_t* __restrict__ off, const uint32_t* __restrict__ total) {
    const int64_t nn = *total;
    const int w[5] = {3, iso ? 1 : 3, iso ? 0 : 4, 1, K3};
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid == 0) {
        const int64_t po = floats_per_gaussian(K3, iso) * n, pn = floats_per_gaussian(K3, iso) * nn;
        for (int e = 0; e < 6 * V; e++) {
            a.m_out[pn + e] = a.m_in[po + e];
            a.v_out[pn + e] = a.v_in[po + e];
        }
        if (a.step_out != a.step_in) {
            a.step_out[0] = a.step_in[0];   // both update counters (Gaussians, poses)
            a.step_out[1] = a.step_in[1];
        }
    }
    for (int64_t i = gid; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[i]) continue;
        const int64_t j = off[i];
        int64_t oo = 0, on = 0;
        for (int g = 0; g < 5; g++) {
            for (int e = 0; e < w[g]; e++) {
                a.m_out[on + w[g] * j + e] = a.m_in[oo + w[g] * i + e];
                a.v_out[on + w[g] * j + e] = a.v_in[oo + w[g] * i + e];
            }
            oo += (int64_t)w[g] * n;
            on += (int64_t)w[g] * nn;
        }
    }
}

__global__ void store_count_kernel(const uint32_t* __restrict__ total, int64_t base, int64_t capacity,
                                   int64_t* __restrict__ out, int two) {
    const int64_t want = base + (int64_t)*total;
    out[0] = want < capacity ? want : capacity;
    if (two) out[1] = want;
}

__device__ __forceinline__ int view_of_pixel(const ViewTable& vt, int64_t p) {
    int lo = 0, hi = vt.V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (vt.v[mid].pix_off <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// alpha <= gamma with the FP32 alpha compared against gamma in FP64 (gamma is
// the caller's double, e.g. 0.99 itself rather than its FP32 rounding)
__global__ void densify_flags_kernel(ViewTable vt, const float* __restrict__ alpha, const float* __restrict__ td,
                                     double gamma, int all_pixels, uint32_t* __restrict__ flag) {
    const int64_t np = vt.n_pix;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x)
        flag[p] = (td[p] > 0.f && (all_pixels || (double)alpha[p] <= gamma)) ? 1u : 0u;
}

__global__ void densify_write_kernel(ViewTable vt, const float* __restrict__ poses, const float* __restrict__ tc,
                                     const float* __restrict__ td, GaussOut g, int n, int K, int iso,
                                     int64_t capacity, const uint32_t* __restrict__ flag,
                                     const uint32_t* __restrict__ off) {
    const int64_t np = vt.n_pix;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[p]) continue;
        const int64_t j = (int64_t)n + off[p];
        if (j >= capacity) continue;
        const int v = view_of_pixel(vt, p);
        const ViewInfo& vi = vt.v[v];
        const int64_t pl = p - vi.pix_off;
        const int y = (int)(pl / vi.W), x = (int)(pl - (int64_t)y * vi.W);
        const float d = td[p];
        // camera point of the pixel's sample, then p_w = R^T (p_c - t)
        const float pc0 = ((float)x - vi.cx) / vi.fx * d - poses[16 * v + 3];
        const float pc1 = ((float)y - vi.cy) / vi.fy * d - poses[16 * v + 7];
        const float pc2 = d - poses[16 * v + 11];
        const float* R = poses + 16 * v;
#pragma unroll
        for (int e = 0; e < 3; e++) g.means[3 * j + e] = R[e] * pc0 + R[4 + e] * pc1 + R[8 + e] * pc2;
        const float lsv = logf(d / vi.fx);
        if (iso) {
            g.ls[j] = lsv;
        } else {
#pragma unroll
            for (int e = 0; e < 3; e++) g.ls[3 * j + e] = lsv;
            g.q[4 * j] = 1.f;
            g.q[4 * j + 1] = 0.f;
            g.q[4 * j + 2] = 0.f;
            g.q[4 * j + 3] = 0.f;
        }
        g.opl[j] = 0.f;
        const int64_t hw = (int64_t)vi.W * vi.H;
        const int64_t ci = 3 * (int64_t)vi.pix_off + pl;
        for (int k = 0; k < 3; k++) {
            const float rgb = tc[ci + k * hw];
            if (K == 1) {
                g.col[3 * j + k] = rgb;
            } else {
                g.col[3 * K * j + k] = (rgb - 0.5f) / kShC0;
                for (int l = 1; l < K; l++) g.col[3 * K * j + 3 * l + k] = 0.f;
            }
        }
    }
}

// moments for the grown layout: existing Gaussians keep theirs, new ones
// start at zero; the new count is counts[0]
__global__ void densify_adam_kernel(AdamIO a, int64_t n, int K3, int iso, int V, const int64_t* __restrict__ counts,
                                    int64_t capacity) {
    const int64_t nn = counts[0];
    const int w[5] = {3, iso ? 1 : 3, iso ? 0 : 4, 1, K3};
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid == 0) {
        const int64_t po = floats_per_gaussian(K3, iso) * n, pn = floats_per_gaussian(K3, iso) * nn;
        for (int e = 0; e < 6 * V; e++) {
            a.m_out[pn + e] = a.m_in[po + e];
            a.v_out[pn + e] = a.v_in[po + e];
        }
        if (a.step_out != a.step_in) {
            a.step_out[0] = a.step_in[0];   // both update counters (Gaussians, poses)
            a.step_out[1] = a.step_in[1];
        }
    }
    for (int64_t j = gid; j < capacity; j += (int64_t)gridDim.x * blockDim.x) {
        if (j >= nn) break;
        int64_t oo = 0, on = 0;
        for (int g = 0; g < 5; g++) {
            for (int e = 0; e < w[g]; e++) {
                const bool old = j < n;
                a.m_out[on + w[g] * j + e] = old ? a.m_in[oo + w[g] * j + e] : 0.f;
                a.v_out[on + w[g] * j + e] = old ? a.v_in[oo + w[g] * j + e] : 0.f;
            }
            oo += (int64_t)w[g] * n;
            on += (int64_t)w[g] * nn;
        }
    }
}

unsigned grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

hipError_t launch_prune(const Params& in, int K3, double logit_tau, GaussOut out, const AdamIO* adam, int V,
                        uint32_t* flag, uint32_t* off, uint32_t* bsum, uint32_t* total, int64_t* n_out,
                        hipStream_t s) {
    const int64_t n = in.n;
    if (n > 0) prune_flags_kernel<<<grid_for(n), 256, 0, s>>>(in.opl, n, logit_tau, flag);
    hipError_t e = launch_scan_u32(flag, n, off, bsum, total, s);
    if (e != hipSuccess) return e;
    if (n > 0) prune_scatter_kernel<<<grid_for(n), 256, 0, s>>>(in, K3, out, flag, off);
    if (adam) prune_adam_kernel<<<grid_for(n), 256, 0, s>>>(*adam, n, K3, in.iso, V, flag, off, total);
    store_count_kernel<<<1, 1, 0, s>>>(total, 0, (int64_t)1 << 62, n_out, 0);
    return hipGetLastError();
}

hipError_t launch_densify(const ViewTable& vt, const float* poses, const float* alpha, const float* tc,
                          const float* td, double gamma, int all_pixels, GaussOut g, int n, int K, int iso,
                          int64_t capacity, const AdamIO* adam, uint32_t* flag, uint32_t* off, uint32_t* bsum,
                          uint32_t* total, int64_t* counts, hipStream_t s) {
    const int64_t np = vt.n_pix;
    densify_flags_kernel<<<grid_for(np), 256, 0, s>>>(vt, alpha, td, gamma, all_pixels, flag);
    hipError_t e = launch_scan_u32(flag, np, off, bsum, total, s);
    if (e != hipSuccess) return e;
    densify_write_kernel<<<grid_for(np), 256, 0, s>>>(vt, poses, tc, td, g, n, K, iso, capacity, flag, off);
    store_count_kernel<<<1, 1, 0, s>>>(total, n, capacity, counts, 1);
    if (adam)
        densify_adam_kernel<<<grid_for(capacity), 256, 0, s>>>(*adam, n, 3 * K, iso, vt.V, counts, capacity);
    return hipGetLastError();
}

}  // namespace gs
