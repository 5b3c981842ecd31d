// Projection of every (view, Gaussian) pair and its reverse mode.
//
// Forward (Sec. 3.4 "Projection"): one thread per Gaussian looping over the
// views, writes each visible (view, Gaussian) record line (conic + opacity,
// colour + depth, mean, pixel rect), every record's bin count, and each
// Gaussian's view mask.
// Backward: per block of Gaussians, the ones some view sees are packed into a
// list and one thread per listed Gaussian loops over its views, so each
// Gaussian's parameter gradient is summed in registers (no atomics) and the
// per-view pose 6-vector is reduced in a fixed order in FP64 (deterministic).
#include "gs_device.h"

namespace gs {

namespace {

constexpr int kProjBlock = 256;

// One thread per Gaussian, looping over the views: the parameters come from
// HBM once and stay in the thread's cache lines for the other views.
__global__ __launch_bounds__(kProjBlock) void preprocess_fwd_kernel(ViewTable vt, Params P, const float* poses,
                                                                    Records rec, bool zero_g2, uint32_t* flags) {
    const int g = blockIdx.x * kProjBlock + threadIdx.x;
    if (g >= P.n) return;
    GPrep gp;
    gauss_prep(P, g, gp);
    bool bad = !gp.finite;
    uint64_t vm = 0;
    for (int v = 0; v < vt.V; v++) {
        const ViewInfo& vi = vt.v[v];
        float T[12];
#pragma unroll
        for (int k = 0; k < 12; k++) T[k] = poses[16 * v + k];
        Proj pr;
        project_view<true>(P, g, gp, vi, T, pr);
        const int64_t r = (int64_t)v * P.n + g;
        if (!pr.valid) {
            rec.nt[r] = 0u;
            continue;
        }
        const uint32_t tx0 = (uint32_t)pr.x0 / vt.bw, tx1 = (uint32_t)pr.x1 / vt.bw;
        const uint32_t ty0 = (uint32_t)pr.y0 / vt.bh, ty1 = (uint32_t)pr.y1 / vt.bh;
        // the record line in 16-byte stores: base-2 conic with log2(opacity)
        // (the compositing kernels' form), colour and depth, mean and rect,
        // then (mapping step) the zeroed gradient sums
        float4* q = reinterpret_cast<float4*>(rec.line + r);
        const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
        q[0] = make_float4(kHalfLog2e * pr.A, 2.f * kHalfLog2e * pr.B, kHalfLog2e * pr.C, log2f(pr.o));
        q[1] = make_float4(pr.col[0], pr.col[1], pr.col[2], pr.p[2]);
        q[2] = make_float4(pr.u, pr.v, __uint_as_float((uint32_t)pr.x0 | ((uint32_t)pr.x1 << 16)),
                           __uint_as_float((uint32_t)pr.y0 | ((uint32_t)pr.y1 << 16)));
        q[3] = zero;
        if (zero_g2) {
            q[4] = zero; q[5] = zero; q[6] = zero; q[7] = zero;
        }
        rec.nt[r] = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
        vm |= 1ull << v;
        bad |= pr.colbad;
    }
    rec.vmask[g] = vm;
    // one atomic per wavefront that read a non-finite parameter, from its
    // first active lane
    const uint64_t bad_lanes = __ballot(bad);
    const int first = __ffsll((unsigned long long)__ballot(true)) - 1;
    if (flags && bad_lanes != 0ull && (int)(threadIdx.x & 63) == first) atomicOr(flags, kFlagNonFinite);
}

template <int CTRL, int ROWM, int BANKM>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWM, BANKM, true));
}

// Sum over the wavefront, left in lane 63, without LDS: three row shifts give
// each lane the sum of itself and up to three lanes below it in its 16-lane
// row, shifts by 4 and 8 (on the upper banks) complete each row's total in
// its lane 15, and the two row broadcasts add row 0 into row 1, row 2 into
// row 3 and then lane 31 into rows 2 and 3.
__device__ __forceinline__ float wave_sum_to_last(float x) {
    float t = x + dpp_mov<0x111, 0xf, 0xf>(x);   // row_shr:1
    t += dpp_mov<0x112, 0xf, 0xf>(x);            // row_shr:2
    t += dpp_mov<0x113, 0xf, 0xf>(x);            // row_shr:3
    t += dpp_mov<0x114, 0xf, 0xe>(t);            // row_shr:4, lanes 4..15 of each row
    t += dpp_mov<0x118, 0xf, 0xc>(t);            // row_shr:8, lanes 8..15
    t += dpp_mov<0x142, 0xa, 0xf>(t);            // row_bcast:15 into rows 1 and 3
    t += dpp_mov<0x143, 0xc, 0xf>(t);            // row_bcast:31 into rows 2 and 3
    return t;
}

// Zero p[e0, e1) with the block's threads, in 16-byte stores when p + e0 is
// 16-byte aligned.
__device__ __forceinline__ void block_zero(float* p, int64_t e0, int64_t e1) {
    if (e0 >= e1) return;
    int64_t i0 = e0;
    if ((reinterpret_cast<uintptr_t>(p + e0) & 15) == 0) {
        const int64_t nv = (e1 - e0) >> 2;
        float4* q = reinterpret_cast<float4*>(p + e0);
        for (int64_t i = threadIdx.x; i < nv; i += kProjBlock) q[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        i0 = e0 + 4 * nv;
    }
    for (int64_t i = i0 + threadIdx.x; i < e1; i += kProjBlock) p[i] = 0.f;
}

constexpr int kBwdPer = kProjBwdSpan / kProjBlock;   // Gaussians each thread scans
static_assert(kProjBwdSpan % kProjBlock == 0 && kProjBwdSpan <= 65536, "span of a backward block");

// One block per span of kProjBwdSpan Gaussians.  The block first reads the
// view masks the forward projection left (bit v: visible in view v); the
// Gaussians visible in none get a zero gradient (or nothing, when
// accumulating) and the others are packed, in increasing index order,
// into a list that the block then walks 256 at a time.  Every lane of that
// walk holds a Gaussian some view sees, so the per-view recomputation runs on
// full wavefronts instead of on the few lanes a random 64 Gaussians leave
// visible.  The per-Gaussian gradient is summed over views in registers; the
// per-view pose 6-vector is summed over each wavefront (FP32), added to that
// wavefront's FP64 slot, and the four slots are added at the end: a fixed
// order, with no barrier inside the walk.
// RGB colours: at most 128 VGPRs (four waves per SIMD; it fits without
// spilling).  The SH variants keep the compiler's choice: capped, they spill.
template <int SH>
__global__ __launch_bounds__(kProjBlock, SH < 0 ? 4 : 1) void preprocess_bwd_kernel(ViewTable vt, Params P, const float* poses,
                                                                    const uint64_t* vmask, const float* g2, Grads G,
                                                                    int accumulate, double* pose_part,
                                                                    int pose_blocks) {
    constexpr int K = SH < 0 ? 1 : (SH + 1) * (SH + 1);
    __shared__ uint16_t s_loc[kProjBwdSpan];
    __shared__ uint64_t s_mask[kProjBwdSpan];
    __shared__ int s_cnt[kBwdPer][kProjBlock / 64];
    __shared__ double s_pose[kProjBlock / 64][kMaxViews][6];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t g0 = (int64_t)blockIdx.x * kProjBwdSpan;
    const int V = vt.V;

    // view mask of Gaussian g0 + threadIdx.x + kProjBlock * j
    uint64_t m[kBwdPer];
#pragma unroll
    for (int j = 0; j < kBwdPer; j++) {
        const int64_t g = g0 + threadIdx.x + kProjBlock * j;
        m[j] = g < P.n ? vmask[g] : 0ull;
    }
    uint64_t ball[kBwdPer];
#pragma unroll
    for (int j = 0; j < kBwdPer; j++) ball[j] = __ballot(m[j] != 0);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < kBwdPer; j++) s_cnt[j][w] = __popcll(ball[j]);
    }
    for (int k = threadIdx.x; k < (kProjBlock / 64) * V * 6; k += kProjBlock)
        s_pose[k / (V * 6)][(k / 6) % V][k % 6] = 0.0;
    __syncthreads();
    // list position: (j, wave, lane) order, which is increasing Gaussian order
    int total = 0, off[kBwdPer];
#pragma unroll
    for (int j = 0; j < kBwdPer; j++)
#pragma unroll
        for (int i = 0; i < kProjBlock / 64; i++) {
            if (i == w) off[j] = total;
            total += s_cnt[j][i];
        }
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int j = 0; j < kBwdPer; j++) {
        const int loc = threadIdx.x + kProjBlock * j;
        if (m[j] != 0) {
            const int e = off[j] + __popcll(ball[j] & lt);
            s_loc[e] = (uint16_t)loc;
            s_mask[e] = m[j];
        }
    }
    if (!accumulate) {
        // the whole span's gradient starts at zero; the walk below overwrites
        // the visible Gaussians' entries after the barrier
        const int64_t g1 = g0 + kProjBwdSpan < (int64_t)P.n ? g0 + kProjBwdSpan : (int64_t)P.n;
        block_zero(G.means, 3 * g0, 3 * g1);
        block_zero(G.ls, 3 * g0, 3 * g1);
        block_zero(G.q, 4 * g0, 4 * g1);
        block_zero(G.opl, g0, g1);
        block_zero(G.col, 3 * K * g0, 3 * K * g1);
    }
    __syncthreads();

    for (int base = 0; base < total; base += kProjBlock) {
        if (base + 64 * w >= total) break;   // nothing left for this wavefront
        const int e = base + (int)threadIdx.x;
        const bool live = e < total;
        const int g = live ? (int)(g0 + s_loc[e]) : 0;
        const uint64_t vmask = live ? s_mask[e] : 0ull;
        float gm[3] = {0.f, 0.f, 0.f}, gl[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f}, go = 0.f;
        float gc[3 * K];
#pragma unroll
        for (int k = 0; k < 3 * K; k++) gc[k] = 0.f;
        GPrep gp;
        gp.ok = false;
        if (live) gauss_prep(P, g, gp);

        for (int v = 0; v < V; v++) {
            float pose[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            const int64_t r = (int64_t)v * P.n + g;
            const bool on = (vmask >> v) & 1ull;
            if (__ballot(on) == 0) continue;
            if (on) {
                const ViewInfo& vi = vt.v[v];
                float T[12];
#pragma unroll
                for (int k = 0; k < 12; k++) T[k] = poses[16 * v + k];
                Proj pr;
                project_view<true>(P, g, gp, vi, T, pr);
                const float4* a4 = reinterpret_cast<const float4*>(g2 + r * kG2Stride);
                const float4 a0 = a4[0], a1 = a4[1], a2 = a4[2];
                // undo the compositing kernel's constant factors (g2 layout)
                const float du = a0.x * (1.f / kHalfLog2e), dv = a0.y * (1.f / kHalfLog2e);
                const float dA = 0.5f * a0.z, dB = a0.w, dC = 0.5f * a1.x;
                const float odo = a1.y;   // o dL/do
                const float dcol[3] = {a1.z, a1.w, a2.x};
                const float dz = a2.y;
                float dmu[3] = {0.f, 0.f, 0.f};
                float dcam[3] = {0.f, 0.f, 0.f};   // gradient w.r.t. the camera centre (SH path)

                // colour
                if (SH < 0) {
                    gc[0] += dcol[0]; gc[1] += dcol[1]; gc[2] += dcol[2];
                } else {
                    float Y[16], dY[16][3];
                    sh_basis<true>(SH, pr.dir[0], pr.dir[1], pr.dir[2], Y, dY);
                    const float* sh = P.col + (int64_t)g * K * 3;
                    float dd[3] = {0.f, 0.f, 0.f};
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        if (pr.cclamp[k]) continue;
#pragma unroll
                        for (int l = 0; l < K; l++) {
                            gc[3 * l + k] += Y[l] * dcol[k];
                            const float w = dcol[k] * sh[3 * l + k];
                            dd[0] += w * dY[l][0]; dd[1] += w * dY[l][1]; dd[2] += w * dY[l][2];
                        }
                    }
                    const float proj = dd[0] * pr.dir[0] + dd[1] * pr.dir[1] + dd[2] * pr.dir[2];
                    const float idn = 1.f / pr.dirn;
#pragma unroll
                    for (int j = 0; j < 3; j++) {
                        const float t = (dd[j] - pr.dir[j] * proj) * idn;
                        dmu[j] += t;
                        dcam[j] -= t;
                    }
                }
                // opacity
                go += odo * (1.f - pr.o);   // dL/do o (1 - o)

                // camera-space mean from depth and projected mean
                const float px = pr.p[0], py = pr.p[1], pz = pr.p[2];
                const float iz = 1.f / pz, iz2 = iz * iz;
                float dpx = du * vi.fx * iz;
                float dpy = dv * vi.fy * iz;
                float dpz = dz - (du * vi.fx * px + dv * vi.fy * py) * iz2;

                // conic -> dilated 2D covariance: G = -Q Gq Q, Gq = [[dA, dB/2], [dB/2, dC]]
                const float hb = 0.5f * dB;
                const float q00 = pr.A * dA + pr.B * hb, q01 = pr.A * hb + pr.B * dC;
                const float q10 = pr.B * dA + pr.C * hb, q11 = pr.B * hb + pr.C * dC;
                const float ga = -(q00 * pr.A + q01 * pr.B);
                const float gb = -0.5f * ((q00 * pr.B + q01 * pr.C) + (q10 * pr.A + q11 * pr.B));
                const float gcc = -(q10 * pr.B + q11 * pr.C);

                // Sigma_2D = J Sc J^T
                const float* S = pr.Sc;  // xx xy xz yy yz zz
                const float j00 = pr.j00, j02 = pr.j02, j11 = pr.j11, j12 = pr.j12;
                const float r00 = j00 * S[0] + j02 * S[2], r01 = j00 * S[1] + j02 * S[4], r02 = j00 * S[2] + j02 * S[5];
                const float r10 = j11 * S[1] + j12 * S[2], r11 = j11 * S[3] + j12 * S[4], r12 = j11 * S[4] + j12 * S[5];
                const float dJ00 = 2.f * (ga * r00 + gb * r10);
                const float dJ02 = 2.f * (ga * r02 + gb * r12);
                const float dJ11 = 2.f * (gb * r01 + gcc * r11);
                const float dJ12 = 2.f * (gb * r02 + gcc * r12);
                // gradient w.r.t. Sc (symmetric, full-matrix convention)
                const float gj02 = ga * j02 + gb * j12, gj12 = gb * j02 + gcc * j12;
                float Gs[9];
                Gs[0] = j00 * j00 * ga;
                Gs[1] = j00 * j11 * gb;
                Gs[2] = j00 * gj02;
                Gs[4] = j11 * j11 * gcc;
                Gs[5] = j11 * gj12;
                Gs[8] = j02 * gj02 + j12 * gj12;
                Gs[3] = Gs[1]; Gs[6] = Gs[2]; Gs[7] = Gs[5];

                // J -> camera-space mean
                dpz -= (dJ00 * vi.fx + dJ11 * vi.fy) * iz2;
                if (!pr.clx) {
                    dpx -= dJ02 * vi.fx * iz2;
                    dpz += dJ02 * 2.f * vi.fx * px * iz2 * iz;
                } else {
                    dpz += dJ02 * vi.fx * (pr.tx * iz) * iz2;
                }
                if (!pr.cly) {
                    dpy -= dJ12 * vi.fy * iz2;
                    dpz += dJ12 * 2.f * vi.fy * py * iz2 * iz;
                } else {
                    dpz += dJ12 * vi.fy * (pr.ty * iz) * iz2;
                }

                // world covariance gradient: GS = W^T Gs W
                float t1[9], GS[9];
#pragma unroll
                for (int r_ = 0; r_ < 3; r_++)
#pragma unroll
                    for (int c = 0; c < 3; c++)
                        t1[3 * r_ + c] = T[r_] * Gs[c] + T[4 + r_] * Gs[3 + c] + T[8 + r_] * Gs[6 + c];
#pragma unroll
                for (int r_ = 0; r_ < 3; r_++)
#pragma unroll
                    for (int c = 0; c < 3; c++)
                        GS[3 * r_ + c] = t1[3 * r_] * T[c] + t1[3 * r_ + 1] * T[4 + c] + t1[3 * r_ + 2] * T[8 + c];

                // Sigma = R diag(s^2) R^T
                float GR[9];
#pragma unroll
                for (int r_ = 0; r_ < 3; r_++)
#pragma unroll
                    for (int c = 0; c < 3; c++)
                        GR[3 * r_ + c] = GS[3 * r_] * pr.R[c] + GS[3 * r_ + 1] * pr.R[3 + c] + GS[3 * r_ + 2] * pr.R[6 + c];
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    // (R^T GS R)_kk = sum_r R[r][k] GR[r][k]
                    const float rgr = pr.R[k] * GR[k] + pr.R[3 + k] * GR[3 + k] + pr.R[6 + k] * GR[6 + k];
                    gl[k] += 2.f * pr.s[k] * pr.s[k] * rgr;
                }
                float dR[9];
#pragma unroll
                for (int r_ = 0; r_ < 3; r_++)
#pragma unroll
                    for (int c = 0; c < 3; c++) dR[3 * r_ + c] = 2.f * GR[3 * r_ + c] * pr.s[c] * pr.s[c];
                const float w = pr.qh[0], x = pr.qh[1], y = pr.qh[2], z = pr.qh[3];
                float dq[4];
                dq[0] = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
                dq[1] = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                               2.f * x * dR[8]);
                dq[2] = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                               2.f * y * dR[8]);
                dq[3] = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] + y * dR[5] +
                               x * dR[6] + y * dR[7]);
                const float qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
                const float iqn = 1.f / pr.qn;
#pragma unroll
                for (int k = 0; k < 4; k++) gq[k] += (dq[k] - pr.qh[k] * qd) * iqn;

                // p = W mu + t
                dmu[0] += T[0] * dpx + T[4] * dpy + T[8] * dpz;
                dmu[1] += T[1] * dpx + T[5] * dpy + T[9] * dpz;
                dmu[2] += T[2] * dpx + T[6] * dpy + T[10] * dpz;
                gm[0] += dmu[0]; gm[1] += dmu[1]; gm[2] += dmu[2];

                // pose (left perturbation): dp/dv = I, dp/dw = -[p]x, the camera
                // centre moves by -W^T v, and Sc picks up [w]x Sc - Sc [w]x
                pose[0] = dpx - (T[0] * dcam[0] + T[1] * dcam[1] + T[2] * dcam[2]);
                pose[1] = dpy - (T[4] * dcam[0] + T[5] * dcam[1] + T[6] * dcam[2]);
                pose[2] = dpz - (T[8] * dcam[0] + T[9] * dcam[1] + T[10] * dcam[2]);
                const float Sf[9] = {S[0], S[1], S[2], S[1], S[3], S[4], S[2], S[4], S[5]};
                // N = Sc Gs - Gs Sc (antisymmetric); d/dw = 2 (N12, N20, N01)
                auto Nij = [&](int i, int j) {
                    return Sf[3 * i] * Gs[j] + Sf[3 * i + 1] * Gs[3 + j] + Sf[3 * i + 2] * Gs[6 + j] -
                           (Gs[3 * i] * Sf[j] + Gs[3 * i + 1] * Sf[3 + j] + Gs[3 * i + 2] * Sf[6 + j]);
                };
                pose[3] = py * dpz - pz * dpy + 2.f * Nij(1, 2);
                pose[4] = pz * dpx - px * dpz + 2.f * Nij(2, 0);
                pose[5] = px * dpy - py * dpx + 2.f * Nij(0, 1);
            }
            float ps[6];
#pragma unroll
            for (int k = 0; k < 6; k++) ps[k] = wave_sum_to_last(pose[k]);
            if (lane == 63) {
#pragma unroll
                for (int k = 0; k < 6; k++) s_pose[w][v][k] += (double)ps[k];
            }
        }
        if (live) {
            float* om = G.means + 3 * (int64_t)g;
            float* ol = G.ls + 3 * (int64_t)g;
            float* oq = G.q + 4 * (int64_t)g;
            float* oc = G.col + (int64_t)g * 3 * K;
            if (accumulate) {
#pragma unroll
                for (int k = 0; k < 3; k++) { om[k] += gm[k]; ol[k] += gl[k]; }
#pragma unroll
                for (int k = 0; k < 4; k++) oq[k] += gq[k];
                G.opl[g] += go;
#pragma unroll
                for (int k = 0; k < 3 * K; k++) oc[k] += gc[k];
            } else {
#pragma unroll
                for (int k = 0; k < 3; k++) { om[k] = gm[k]; ol[k] = gl[k]; }
#pragma unroll
                for (int k = 0; k < 4; k++) oq[k] = gq[k];
                G.opl[g] = go;
#pragma unroll
                for (int k = 0; k < 3 * K; k++) oc[k] = gc[k];
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < V * 6; k += kProjBlock) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < kProjBlock / 64; i++) t += s_pose[i][k / 6][k % 6];
        pose_part[((int64_t)(k / 6) * pose_blocks + blockIdx.x) * 6 + k % 6] = t;
    }
}

// one block per view: FP64 sum of the per-block pose partials, plus the
// re-projection term (acc = [sum h, count, sum dh/dxi (6)] per view)
__global__ __launch_bounds__(256) void pose_finalize_kernel(const double* part, int pose_blocks, const double* rp,
                                                            float rp_w, float* out) {
    const int v = blockIdx.x;
    __shared__ double red[256][6];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < pose_blocks; b += 256)
#pragma unroll
        for (int k = 0; k < 6; k++) acc[k] += part[((int64_t)v * pose_blocks + b) * 6 + k];
#pragma unroll
    for (int k = 0; k < 6; k++) red[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < 6; k++) red[threadIdx.x][k] += red[threadIdx.x + s][k];
        __syncthreads();
    }
    if (threadIdx.x < 6) {
        double r = red[0][threadIdx.x];
        if (rp) {
            const double cnt = rp[8 * v + 1];
            if (cnt > 0) r += (double)rp_w * rp[8 * v + 2 + threadIdx.x] / cnt;
        }
        out[6 * v + threadIdx.x] = (float)r;
    }
}

}  // namespace

hipError_t launch_preprocess_fwd(const ViewTable& vt, const Params& P, const float* poses, Records rec,
                                 bool zero_g2, hipStream_t s, uint32_t* flags) {
    if (P.n == 0) return hipSuccess;
    preprocess_fwd_kernel<<<(P.n + kProjBlock - 1) / kProjBlock, kProjBlock, 0, s>>>(vt, P, poses, rec, zero_g2,
                                                                                       flags);
    return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const ViewTable& vt, const Params& P, const float* poses, const Records& rec,
                                 const float* g2, Grads G, int accumulate, double* pose_part, int64_t pose_blocks,
                                 hipStream_t s) {
    if (P.n == 0) return hipSuccess;
    const int nb = (P.n + kProjBwdSpan - 1) / kProjBwdSpan;
    if (nb != pose_blocks) return hipErrorInvalidValue;
    switch (P.sh) {
        case -1: preprocess_bwd_kernel<-1><<<nb, kProjBlock, 0, s>>>(vt, P, poses, rec.vmask, g2, G, accumulate, pose_part, nb); break;
        case 0: preprocess_bwd_kernel<0><<<nb, kProjBlock, 0, s>>>(vt, P, poses, rec.vmask, g2, G, accumulate, pose_part, nb); break;
        case 1: preprocess_bwd_kernel<1><<<nb, kProjBlock, 0, s>>>(vt, P, poses, rec.vmask, g2, G, accumulate, pose_part, nb); break;
        case 2: preprocess_bwd_kernel<2><<<nb, kProjBlock, 0, s>>>(vt, P, poses, rec.vmask, g2, G, accumulate, pose_part, nb); break;
        case 3: preprocess_bwd_kernel<3><<<nb, kProjBlock, 0, s>>>(vt, P, poses, rec.vmask, g2, G, accumulate, pose_part, nb); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pose_finalize(const ViewTable& vt, const double* pose_part, int64_t pose_blocks,
                                const double* rp_acc, float rp_weight, float* dL_dpose, hipStream_t s) {
    pose_finalize_kernel<<<vt.V, 256, 0, s>>>(pose_part, (int)pose_blocks, rp_acc, rp_weight, dL_dpose);
    return hipGetLastError();
}

}  // namespace gs
