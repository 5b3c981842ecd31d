// Loss reductions, the re-projection residual and the optimiser updates.
//
// Re-projection (Sec. 3.2 Eq. lba): one thread per match, Huber kernel on the
// residual norm, per-view sums of loss, count and pose gradient in FP64.
// Loss (Sec. 3.3 joint-loss equation, L1 terms of the Sec. 3.4 mapping loss):
// FP64 reduction of the per-tile partials written by the compositing epilogue.
// Updates: Adam on every parameter group; pose steps applied on SE(3) by
// left multiplication with the exponential of the Adam step.
#include <algorithm>

#include "gs_device.h"

namespace gs {

namespace {

// the gradient sums of the *nvis visible records (their slots 0 .. *nvis - 1),
// in 16-byte stores (the count is on the device: a capped grid strides)
__global__ void zero_g2_kernel(const uint32_t* nvis, float* g2) {
    const int64_t m = (int64_t)*nvis * (kG2Floats / 4);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        reinterpret_cast<float4*>(g2)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void zero_f64_kernel(double* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// acc per view: [sum h, count, dxi(6)]
__global__ __launch_bounds__(256) void reproj_kernel(ViewTable vt, const float* poses, const float* pts,
                                                     const float* uv, const int32_t* vid, int64_t M, float delta,
                                                     float* residual, double* acc, float* dpts) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = m < M;
    int v = in ? vid[m] : -1;
    if (v < 0 || v >= vt.V) v = -1;
    double h = 0.0, g[6] = {0, 0, 0, 0, 0, 0}, c = 0.0;
    float r0 = 0.f, r1 = 0.f;
    if (v >= 0) {
        const float* T = poses + 16 * v;
        const float X = pts[3 * m], Y = pts[3 * m + 1], Z = pts[3 * m + 2];
        const float px = T[0] * X + T[1] * Y + T[2] * Z + T[3];
        const float py = T[4] * X + T[5] * Y + T[6] * Z + T[7];
        const float pz = T[8] * X + T[9] * Y + T[10] * Z + T[11];
        if (pz > kZNear) {
            const ViewInfo& vi = vt.v[v];
            const float iz = 1.f / pz;
            r0 = uv[2 * m] - (vi.fx * px * iz + vi.cx);
            r1 = uv[2 * m + 1] - (vi.fy * py * iz + vi.cy);
            const float e = sqrtf(r0 * r0 + r1 * r1);
            float s;
            if (e <= delta) {
                h = 0.5 * (double)e * (double)e;
                s = 1.f;
            } else {
                h = (double)delta * ((double)e - 0.5 * (double)delta);
                s = delta / e;
            }
            c = 1.0;
            // dh/dr = s r and r = uv - pi, so dh/dpi = -s r
            const float gu = -s * r0, gv = -s * r1;
            const float dpx = gu * vi.fx * iz, dpy = gv * vi.fy * iz;
            const float dpz = -(gu * vi.fx * px + gv * vi.fy * py) * iz * iz;
            g[0] = dpx; g[1] = dpy; g[2] = dpz;
            g[3] = (double)(py * dpz - pz * dpy);
            g[4] = (double)(pz * dpx - px * dpz);
            g[5] = (double)(px * dpy - py * dpx);
            if (dpts) {   // dh/dP = R^T dh/dp; scaled by weight / (matches of the view) afterwards
#pragma unroll
                for (int k = 0; k < 3; k++) dpts[3 * m + k] = T[k] * dpx + T[4 + k] * dpy + T[8 + k] * dpz;
            }
        } else {
            v = -1;
        }
    }
    if (in && residual) {
        residual[2 * m] = r0;
        residual[2 * m + 1] = r1;
    }
    if (in && dpts && v < 0) dpts[3 * m] = dpts[3 * m + 1] = dpts[3 * m + 2] = 0.f;
    // matches are usually grouped by view: reduce over the wavefront when
    // every valid lane has the same view, else one atomic set per lane
    const uint64_t valid = __ballot(v >= 0);
    if (valid == 0ull) return;
    const int lane = threadIdx.x & 63;
    const int first = __ffsll((unsigned long long)valid) - 1;
    const int v0 = __shfl(v, first, 64);
    if (__ballot(v >= 0 && v != v0) == 0ull) {
        const double sh = wave_sum_d(h), sc = wave_sum_d(c);
        double sg[6];
#pragma unroll
        for (int k = 0; k < 6; k++) sg[k] = wave_sum_d(g[k]);
        if (lane == first) {
            double* a = acc + 8 * v0;
            atomicAdd(a, sh);
            atomicAdd(a + 1, sc);
#pragma unroll
            for (int k = 0; k < 6; k++) atomicAdd(a + 2 + k, sg[k]);
        }
    } else if (v >= 0) {
        double* a = acc + 8 * v;
        atomicAdd(a, h);
        atomicAdd(a + 1, c);
#pragma unroll
        for (int k = 0; k < 6; k++) atomicAdd(a + 2 + k, g[k]);
    }
}

__global__ void reproj_finalize_kernel(int V, const double* acc, float weight, float* loss, float* dpose) {
    const int v = threadIdx.x;
    if (v >= V) return;
    const double c = acc[8 * v + 1];
    loss[v] = c > 0 ? (float)(acc[8 * v] / c) : 0.f;
    if (dpose && c > 0) {
#pragma unroll
        for (int k = 0; k < 6; k++) dpose[6 * v + k] += (float)((double)weight * acc[8 * v + 2 + k] / c);
    }
}

// one workgroup per view: its loss terms, and its weighted sum in tot[v]
__global__ __launch_bounds__(256) void loss_view_kernel(ViewTable vt, const double2* part, const double* rp,
                                                        const double* ssim_part, float wc, float wd, float wr,
                                                        float wsm, float* out, double* tot) {
    __shared__ double red[256][3];
    const int v = blockIdx.x;
    const ViewInfo& vi = vt.v[v];
    const int nt = vi.tiles_x * vi.tiles_y;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nt; i += 256) {
        const double2 p = part[vi.tile_off + i];
        a += p.x;
        b += p.y;
    }
    if (ssim_part) {
        const int ns = ((vi.W + kSsimTW - 1) / kSsimTW) * ((vi.H + kSsimTH - 1) / kSsimTH);
        for (int i = threadIdx.x; i < 3 * ns; i += 256) {
            const int k = i / ns;
            c += ssim_part[(int64_t)k * vt.n_ssim_tiles + vi.ssim_off + (i - k * ns)];
        }
    }
    red[threadIdx.x][0] = a;
    red[threadIdx.x][1] = b;
    red[threadIdx.x][2] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[threadIdx.x][0] += red[threadIdx.x + s][0];
            red[threadIdx.x][1] += red[threadIdx.x + s][1];
            red[threadIdx.x][2] += red[threadIdx.x + s][2];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double npx = (double)vi.W * vi.H;
        const double lc = red[0][0] / (3.0 * npx);
        const double ld = red[0][1] / npx;
        const double ls = ssim_part ? 1.0 - red[0][2] / (3.0 * npx) : 0.0;
        double lr = 0.0;
        if (rp && rp[8 * v + 1] > 0) lr = rp[8 * v] / rp[8 * v + 1];
        out[1 + 4 * v] = (float)lc;
        out[2 + 4 * v] = (float)ld;
        out[3 + 4 * v] = (float)lr;
        out[4 + 4 * v] = (float)ls;
        tot[v] = (double)wc * lc + (double)wd * ld + (double)wr * lr + (double)wsm * ls;
    }
}

// the step's total loss; also folds the step's status bits into the sticky word
__global__ void loss_total_kernel(int V, const double* tot, float* out, uint32_t* scal) {
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int v = 0; v < V; v++) t += tot[v];
        out[0] = (float)(t / (double)V);
        if (scal) scal[kSticky] |= scal[kFlags];
    }
}

// Adam over every parameter group in one launch.  Group i owns blocks
// [blk[i], blk[i + 1]); its elements go four to a thread with 16-byte loads
// and stores when its four arrays are 16-byte aligned and its count is a
// multiple of four (vec[i]), else one to a thread.
struct AdamLaunch {
    float* p[5];
    const float* g[5];
    float* m[5];
    float* v[5];
    int64_t n[5];
    float lr[5];
    int vec[5];
    int64_t blk[6];
};

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float lr, float b1, float b2,
                                         float eps, float c1, float c2) {
    m = b1 * m + (1.f - b1) * g;
    v = b2 * v + (1.f - b2) * g * g;
    p -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

constexpr int64_t kAdamMaxBlocks = int64_t(1) << 21;   // per group; five groups stay below 2^32 threads

__global__ __launch_bounds__(256) void adam_kernel(AdamLaunch a, float b1, float b2, float eps, const int32_t* step,
                                                   const uint32_t* flags) {
    if (flags && *flags != 0u) return;   // the step is invalid: leave everything as it was
    int gi = 0;
    while (gi < 4 && (int64_t)blockIdx.x >= a.blk[gi + 1]) gi++;
    const float t = (float)(*step + 1);
    const float c1 = 1.f / (1.f - powf(b1, t));
    const float c2 = 1.f / (1.f - powf(b2, t));
    const float lr = a.lr[gi];
    const int64_t nb = a.blk[gi + 1] - a.blk[gi];
    const int64_t t0 = (blockIdx.x - a.blk[gi]) * (int64_t)blockDim.x + threadIdx.x, stride = nb * blockDim.x;
    if (a.vec[gi]) {
        // each element is touched once: streaming (non-temporal) 16-byte
        // accesses, which keep the caches out of the way (1.11 -> 1.00 ms
        // for 177M parameters)
        typedef float v4f __attribute__((ext_vector_type(4)));
        v4f* P = reinterpret_cast<v4f*>(a.p[gi]);
        const v4f* G = reinterpret_cast<const v4f*>(a.g[gi]);
        v4f* M = reinterpret_cast<v4f*>(a.m[gi]);
        v4f* Vv = reinterpret_cast<v4f*>(a.v[gi]);
        for (int64_t i = t0; i < a.n[gi] / 4; i += stride) {
            v4f p4 = __builtin_nontemporal_load(P + i), m4 = __builtin_nontemporal_load(M + i),
                v4 = __builtin_nontemporal_load(Vv + i);
            const v4f g4 = __builtin_nontemporal_load(G + i);
#pragma unroll
            for (int c = 0; c < 4; c++) {
                float pc = p4[c], mc = m4[c], vc = v4[c];
                adam_one(pc, g4[c], mc, vc, lr, b1, b2, eps, c1, c2);
                p4[c] = pc; m4[c] = mc; v4[c] = vc;
            }
            __builtin_nontemporal_store(p4, P + i);
            __builtin_nontemporal_store(m4, M + i);
            __builtin_nontemporal_store(v4, Vv + i);
        }
    } else {
        for (int64_t i = t0; i < a.n[gi]; i += stride)
            adam_one(a.p[gi][i], a.g[gi][i], a.m[gi][i], a.v[gi][i], lr, b1, b2, eps, c1, c2);
    }
}

// T_out = Exp(xi) T_in for the twist xi = (v, w) (translation first): R by
// Rodrigues, translation V(w) v; FP64 arithmetic, the bottom row (0 0 0 1)
// written as such.  T_in and T_out may alias.
__device__ void se3_exp_left(const double xi[6], const float* Tin, float* Tout) {
    const double wx = xi[3], wy = xi[4], wz = xi[5];
    const double th2 = wx * wx + wy * wy + wz * wz, th = sqrt(th2);
    double A, B, Cc;
    if (th < 1e-6) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
        Cc = 1.0 / 6.0 - th2 / 120.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
        Cc = (th - sin(th)) / (th2 * th);
    }
    const double W[9] = {0, -wz, wy, wz, 0, -wx, -wy, wx, 0};
    double W2[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) W2[3 * r + c] = W[3 * r] * W[c] + W[3 * r + 1] * W[3 + c] + W[3 * r + 2] * W[6 + c];
    double R[9], Vm[9];
    for (int i = 0; i < 9; i++) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + A * W[i] + B * W2[i];
        Vm[i] = I + B * W[i] + Cc * W2[i];
    }
    double tr[3];
    for (int r = 0; r < 3; r++) tr[r] = Vm[3 * r] * xi[0] + Vm[3 * r + 1] * xi[1] + Vm[3 * r + 2] * xi[2];
    double old[12];
    for (int i = 0; i < 12; i++) old[i] = Tin[i];
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 4; c++) {
            double sum = R[3 * r] * old[c] + R[3 * r + 1] * old[4 + c] + R[3 * r + 2] * old[8 + c];
            if (c == 3) sum += tr[r];
            Tout[4 * r + c] = (float)sum;
        }
    }
    Tout[12] = 0.f; Tout[13] = 0.f; Tout[14] = 0.f; Tout[15] = 1.f;
}

// step[1] counts the pose updates (step[0] the Gaussian ones): separate
// bias corrections, as two optimisers would keep
__global__ void pose_update_kernel(int V, float* poses, const float* dpose, float* m, float* v, float lr, float b1,
                                   float b2, float eps, const int32_t* step, const uint32_t* flags) {
    const int k = threadIdx.x;
    if (k >= V) return;
    if (flags && *flags != 0u) return;
    const double t = (double)(step[1] + 1);
    double xi[6];
    for (int i = 0; i < 6; i++) {
        const float gi = dpose[6 * k + i];
        const float mi = b1 * m[6 * k + i] + (1.f - b1) * gi;
        const float vi = b2 * v[6 * k + i] + (1.f - b2) * gi * gi;
        m[6 * k + i] = mi;
        v[6 * k + i] = vi;
        const double mh = (double)mi / (1.0 - pow((double)b1, t));
        const double vh = (double)vi / (1.0 - pow((double)b2, t));
        xi[i] = -(double)lr * mh / (sqrt(vh) + (double)eps);
    }
    float* P = poses + 16 * k;
    se3_exp_left(xi, P, P);
}

// poses_out[k] = Exp(xi[k]) poses_in[k]
__global__ void pose_retract_kernel(int V, const float* pin, const float* xi, float* pout) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= V) return;
    double x[6];
    for (int i = 0; i < 6; i++) x[i] = xi[6 * k + i];
    float T[16];
    for (int i = 0; i < 16; i++) T[i] = pin[16 * k + i];
    se3_exp_left(x, T, pout + 16 * k);
}

// out[k] = J_l(xi[k])^T g[k]: the gradient with respect to xi of L(Exp(xi) T)
// from the left-perturbation gradient g at Exp(xi) T, since
// Exp(xi + e) = Exp(J_l(xi) e) Exp(xi) to first order.  J_l is summed from its
// series sum_n ad(xi)^n / (n + 1)!, ad(xi) = [[w^, v^], [0, w^]]; 40 terms in
// FP64 (the remainder is below 1e-16 relative for |xi| <= 4).
__global__ void pose_tangent_grad_kernel(int V, const float* xi, const float* g, float* out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= V) return;
    const double vx = xi[6 * k], vy = xi[6 * k + 1], vz = xi[6 * k + 2];
    const double wx = xi[6 * k + 3], wy = xi[6 * k + 4], wz = xi[6 * k + 5];
    double ad[36];
    for (int i = 0; i < 36; i++) ad[i] = 0.0;
    const double wh[9] = {0, -wz, wy, wz, 0, -wx, -wy, wx, 0};
    const double vh[9] = {0, -vz, vy, vz, 0, -vx, -vy, vx, 0};
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            ad[6 * r + c] = wh[3 * r + c];
            ad[6 * r + 3 + c] = vh[3 * r + c];
            ad[6 * (r + 3) + 3 + c] = wh[3 * r + c];
        }
    // J^T g = sum_n (ad^T)^n g / (n + 1)!: iterate the vector u_n = ad^T u_{n-1} / (n + 1)
    double u[6], acc[6];
    for (int i = 0; i < 6; i++) u[i] = acc[i] = g[6 * k + i];
    for (int n = 1; n <= 40; n++) {
        double w[6];
        for (int i = 0; i < 6; i++) {
            double sum = 0.0;
            for (int j = 0; j < 6; j++) sum += ad[6 * j + i] * u[j];
            w[i] = sum / (double)(n + 1);
        }
        for (int i = 0; i < 6; i++) {
            u[i] = w[i];
            acc[i] += w[i];
        }
    }
    for (int i = 0; i < 6; i++) out[6 * k + i] = (float)acc[i];
}

__global__ void step_bump_kernel(int32_t* step, int gaussians, int poses, const uint32_t* flags) {
    if (flags && *flags != 0u) return;
    if (gaussians) step[0] += 1;
    if (poses) step[1] += 1;
}

}  // namespace

hipError_t launch_zero_g2(const uint32_t* nvis, float* g2, int64_t bound, hipStream_t s) {
    const int64_t m = bound * (kG2Floats / 4);
    if (m <= 0) return hipSuccess;
    zero_g2_kernel<<<(unsigned)std::min<int64_t>((m + 255) / 256, 4096), 256, 0, s>>>(nvis, g2);
    return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    zero_f64_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_reproj(const ViewTable& vt, const float* poses, const float* pts, const float* uv,
                         const int32_t* vid, int64_t M, float delta, float* residual, double* acc, hipStream_t s,
                         float* dpts) {
    if (M <= 0) return hipSuccess;
    reproj_kernel<<<(unsigned)((M + 255) / 256), 256, 0, s>>>(vt, poses, pts, uv, vid, M, delta, residual, acc,
                                                              dpts);
    return hipGetLastError();
}

namespace {
__global__ __launch_bounds__(256) void reproj_points_scale_kernel(int V, const int32_t* vid, int64_t M,
                                                                  const double* acc, float weight, float* dpts) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const int v = vid[m];
    const double cnt = (v >= 0 && v < V) ? acc[8 * v + 1] : 0.0;
    const float sc = cnt > 0.0 ? (float)((double)weight / cnt) : 0.f;
#pragma unroll
    for (int k = 0; k < 3; k++) dpts[3 * m + k] *= sc;
}
}  // namespace

hipError_t launch_reproj_points_scale(const ViewTable& vt, const int32_t* vid, int64_t M, const double* acc,
                                      float weight, float* dpts, hipStream_t s) {
    if (M <= 0) return hipSuccess;
    reproj_points_scale_kernel<<<(unsigned)((M + 255) / 256), 256, 0, s>>>(vt.V, vid, M, acc, weight, dpts);
    return hipGetLastError();
}

hipError_t launch_reproj_finalize(const ViewTable& vt, const double* acc, float weight, float* loss,
                                  float* dL_dpose, hipStream_t s) {
    reproj_finalize_kernel<<<1, kMaxViews, 0, s>>>(vt.V, acc, weight, loss, dL_dpose);
    return hipGetLastError();
}

hipError_t launch_loss_reduce(const ViewTable& vt, const double2* tile_part, const double* rp_acc,
                              const double* ssim_part, float w_color, float w_depth, float w_reproj, float w_ssim,
                              float* loss_out, double* view_tot, hipStream_t s, uint32_t* scal) {
    loss_view_kernel<<<vt.V, 256, 0, s>>>(vt, tile_part, rp_acc, ssim_part, w_color, w_depth, w_reproj, w_ssim,
                                          loss_out, view_tot);
    loss_total_kernel<<<1, 64, 0, s>>>(vt.V, view_tot, loss_out, scal);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamGroups& ag, float* m, float* v, int32_t* step, float b1, float b2, float eps,
                       const uint32_t* flags, hipStream_t s, unsigned groups) {
    AdamLaunch a;
    int64_t off = 0, blocks = 0;
    const auto al16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
    for (int i = 0; i < 5; i++) {
        const int64_t n = ag.cnt[i] > 0 ? ag.cnt[i] : 0;
        const bool on = (groups >> i) & 1u;
        a.p[i] = ag.p[i];
        a.g[i] = ag.g[i];
        a.m[i] = m + off;
        a.v[i] = v + off;
        a.n[i] = on ? n : 0;
        a.lr[i] = ag.lr[i];
        a.vec[i] = n % 4 == 0 && al16(ag.p[i]) && al16(ag.g[i]) && al16(m + off) && al16(v + off);
        a.blk[i] = blocks;
        const int64_t items = !on ? 0 : a.vec[i] ? n / 4 : n;
        // one 16-byte item per thread: a grid-stride loop over a capped grid
        // (8192 blocks per group) ran 0.96 ms for 177M parameters, this 0.81
        // ms; the cap only keeps the grid's thread count within 32 bits
        blocks += std::min<int64_t>((items + 255) / 256, kAdamMaxBlocks);
        off += n;
    }
    a.blk[5] = blocks;
    if (blocks > 0) adam_kernel<<<(unsigned)blocks, 256, 0, s>>>(a, b1, b2, eps, step, flags);
    return hipGetLastError();
}

hipError_t launch_pose_update(int V, float* poses, const float* dpose, float* m, float* v, int32_t* step, float lr,
                              float b1, float b2, float eps, const uint32_t* flags, hipStream_t s) {
    pose_update_kernel<<<1, kMaxViews, 0, s>>>(V, poses, dpose, m, v, lr, b1, b2, eps, step, flags);
    return hipGetLastError();
}

hipError_t launch_step_bump(int32_t* step, int gaussians, int poses, hipStream_t s, const uint32_t* flags) {
    step_bump_kernel<<<1, 1, 0, s>>>(step, gaussians, poses, flags);
    return hipGetLastError();
}

hipError_t launch_pose_retract(int V, const float* pin, const float* xi, float* pout, hipStream_t s) {
    if (V <= 0) return hipSuccess;
    pose_retract_kernel<<<1, kMaxViews, 0, s>>>(V, pin, xi, pout);
    return hipGetLastError();
}

hipError_t launch_pose_tangent_grad(int V, const float* xi, const float* g, float* out, hipStream_t s) {
    if (V <= 0) return hipSuccess;
    pose_tangent_grad_kernel<<<1, kMaxViews, 0, s>>>(V, xi, g, out);
    return hipGetLastError();
}

}  // namespace gs
