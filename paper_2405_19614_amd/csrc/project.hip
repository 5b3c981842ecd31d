// Projection of every (view, Gaussian) pair and its reverse mode.
//
// Forward (Sec. 3.4 "Projection"): one thread per Gaussian looping over the
// views, writes each visible (view, Gaussian) record line (conic + opacity,
// colour + depth, mean, pixel rect), each wavefront's visibility word per view
// (its ballot), and each Gaussian's view mask.
// Backward: per block of Gaussians, the ones some view sees are packed into a
// list and one thread per listed Gaussian loops over the views that see it,
// so each Gaussian's parameter gradient is summed in registers (no atomics);
// the per-view pose 6-vector is summed in FP64 in LDS.
#include "gs_device.h"

namespace gs {

namespace {

// Views per round of the forward's queue (kProjBlock x kProjChunk entries of
// 4 bytes in LDS).
constexpr int kProjChunk = 16;

// One thread per Gaussian prepares it (activations, world covariance) once;
// then, per round of kProjChunk views, two phases:
//  A. each thread tests its Gaussian against each view of the round with the
//     conservative may_be_visible (a few dozen instructions) and queues the
//     (thread, view) pairs that pass in LDS;
//  B. the block's threads take the queued pairs, every lane busy, and run the
//     full projection (and the SH colour), writing each visible record's
//     line, its visibility bit and its view-mask bit;
//     With rec.stage set, phase B also writes every queued pair's entry
//     (view and thread, depth, rect; or a mark for a pair the projection
//     rejects) to the block's list, densely in queue order: the binning's
//     compaction then reads these lists instead of gathering depth and rect
//     from HBM, one record line per visible record.
// About a tenth of the (view, Gaussian) pairs are visible and they are
// scattered over the Gaussians, so a thread looping over its own views would
// run the full projection on nearly every wavefront for every view.  The
// prepared Gaussians wait in LDS for phase B; the records' contents do not
// depend on which lane projects them.
template <int SH, bool ISO>
__global__ __launch_bounds__(kProjBlock) void preprocess_fwd_kernel(ViewTable vt, Params P, const float* poses,
                                                                    Records rec, uint32_t* flags) {
    constexpr int kW = kProjBlock / 64;
    constexpr int K3 = SH < 0 ? 3 : 3 * (SH + 1) * (SH + 1);   // colour floats per Gaussian
    // SH coefficients of the Gaussians with queued pairs, staged in LDS per
    // round (coefficient-major, kShSlots Gaussians; the others read theirs
    // from HBM in phase B): a visible Gaussian is seen by several views, and
    // per-pair reads would fetch its row once per view, 16 bytes per lane
    constexpr bool kStageSh = SH >= 1;
    constexpr int kShSlots = 80;
    constexpr int kShVec = K3 % 4 == 0 ? 4 : 1;   // floats per load (a row starts 16-byte aligned)
    __shared__ uint16_t s_ent[kProjBlock * kProjChunk];   // (thread << 6) | view
    __shared__ int s_n;
    __shared__ float s_gp[10][kProjBlock];                // mu (3), M (6), o
    __shared__ float s_sh[kStageSh ? K3 * kShSlots : 1];
    __shared__ int16_t s_slot[kProjBlock];                // the thread's staging slot, -1 for none
    __shared__ uint8_t s_own[kShSlots];                   // the thread owning a slot
    __shared__ int s_wq[kW];                              // threads with queued pairs, per wavefront
    __shared__ unsigned long long s_vis[kProjChunk][kW];  // visibility words of the round
    __shared__ unsigned long long s_vm[kProjBlock];       // view masks
    __shared__ float s_T[kProjChunk][12];                 // the round's poses
    __shared__ float2 s_lim[kProjChunk];                  // their views' Jacobian clamp limits
    __shared__ uint32_t s_qrun;                           // pairs queued in earlier rounds
    __shared__ uint32_t s_nvis;                           // visible records of the block
    const int lane = threadIdx.x & 63;
    const int g = blockIdx.x * kProjBlock + threadIdx.x;
    const bool live = g < P.n;
    GPrep gp;
    gp.ok = false;
    gp.finite = true;
    if (live) gauss_prep<ISO>(P, g, gp);
    bool bad = !gp.finite;
    // inputs of the conservative test
    const float smax2 = fmaxf(fmaxf(gp.s[0] * gp.s[0], gp.s[1] * gp.s[1]), gp.s[2] * gp.s[2]);
    const float qbox = (gp.ok && gp.o >= kAlphaMin) ? 2.f * logf(255.f * gp.o) + 0.05f : -1.f;
#pragma unroll
    for (int k = 0; k < 3; k++) s_gp[k][threadIdx.x] = gp.mu[k];
#pragma unroll
    for (int k = 0; k < 6; k++) s_gp[3 + k][threadIdx.x] = gp.M[k];
    s_gp[9][threadIdx.x] = gp.o;
    s_vm[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) {
        s_qrun = 0u;
        s_nvis = 0u;
    }
    const int64_t vrow = vis_words(P.n);
    for (int v0 = 0; v0 < vt.V; v0 += kProjChunk) {
        const int v1 = v0 + kProjChunk < vt.V ? v0 + kProjChunk : vt.V;
        if (threadIdx.x == 0) s_n = 0;
        for (int k = threadIdx.x; k < (v1 - v0) * kW; k += kProjBlock) s_vis[k / kW][k % kW] = 0ull;
        for (int k = threadIdx.x; k < (v1 - v0) * 12; k += kProjBlock) s_T[k / 12][k % 12] = poses[16 * (v0 + k / 12) + k % 12];
        for (int k = threadIdx.x; k < v1 - v0; k += kProjBlock) {
            const ViewInfo& vk = vt.v[v0 + k];
            s_lim[k] = make_float2(kJClamp * (float)vk.W / (2.f * vk.fx), kJClamp * (float)vk.H / (2.f * vk.fy));
        }
        __syncthreads();
        // phase A: the pairs that may be visible, queued (one LDS atomic per wavefront and view)
        bool queued = false;
        for (int v = v0; v < v1; v++) {
            const ViewInfo& vi = vt.v[v];
            float T[12];
#pragma unroll
            for (int k = 0; k < 12; k++) T[k] = s_T[v - v0][k];
            const float2 lim = s_lim[v - v0];
            const bool pass = gp.ok && may_be_visible(gp.mu, smax2, qbox, vi, T, lim.x, lim.y);
            const uint64_t bm = __ballot(pass);
            if (bm != 0ull) {
                const int leader = __ffsll((unsigned long long)bm) - 1;
                int base = 0;
                if (lane == leader) base = atomicAdd(&s_n, __popcll(bm));
                base = __shfl(base, leader, 64);
                if (pass) s_ent[base + __popcll(bm & ((1ull << lane) - 1ull))] = (uint16_t)((threadIdx.x << 6) | v);
            }
            queued |= pass;
        }
        const uint64_t qm = __ballot(queued);
        if (kStageSh && lane == 0) s_wq[threadIdx.x >> 6] = __popcll(qm);
        __syncthreads();
        if (kStageSh) {
            // slots in thread order, then the coefficient rows of the first
            // kShSlots, slot-fastest so that a store instruction's lanes hit
            // distinct LDS banks
            int before = 0, m = 0;
#pragma unroll
            for (int w = 0; w < kW; w++) {
                before += w < (int)(threadIdx.x >> 6) ? s_wq[w] : 0;
                m += s_wq[w];
            }
            const int slot = queued ? before + __popcll(qm & ((1ull << lane) - 1ull)) : -1;
            s_slot[threadIdx.x] = (int16_t)(slot < kShSlots ? slot : -1);
            if (slot >= 0 && slot < kShSlots) s_own[slot] = (uint8_t)threadIdx.x;
            m = m < kShSlots ? m : kShSlots;
            __syncthreads();
            for (int idx = threadIdx.x; idx < kShSlots * (K3 / kShVec); idx += kProjBlock) {
                const int j = idx % kShSlots, q = idx / kShSlots;
                if (j >= m) continue;
                const float* src = P.col + (int64_t)(blockIdx.x * kProjBlock + s_own[j]) * K3;
                if (kShVec == 4) {
                    const float4 c = reinterpret_cast<const float4*>(src)[q];
                    s_sh[(4 * q) * kShSlots + j] = c.x;
                    s_sh[(4 * q + 1) * kShSlots + j] = c.y;
                    s_sh[(4 * q + 2) * kShSlots + j] = c.z;
                    s_sh[(4 * q + 3) * kShSlots + j] = c.w;
                } else {
                    s_sh[q * kShSlots + j] = src[q];
                }
            }
            __syncthreads();
        }
        // phase B: the full projection of the queued pairs
        const int nq = s_n;
        const uint32_t qb = s_qrun;
        for (int i = threadIdx.x; i < nq; i += kProjBlock) {
            const uint32_t e = s_ent[i];
            const int v = (int)(e & 63u), t = (int)(e >> 6);
            const int gg = blockIdx.x * kProjBlock + t;
            GPrep q;
            q.ok = true;   // (only prepared Gaussians pass the test of phase A)
            q.finite = true;
            q.qn = 1.f;
            q.qh[0] = 1.f; q.qh[1] = q.qh[2] = q.qh[3] = 0.f;
#pragma unroll
            for (int k = 0; k < 9; k++) q.R[k] = (k % 4 == 0) ? 1.f : 0.f;
            q.s[0] = q.s[1] = q.s[2] = 0.f;
#pragma unroll
            for (int k = 0; k < 3; k++) q.mu[k] = s_gp[k][t];
#pragma unroll
            for (int k = 0; k < 6; k++) q.M[k] = s_gp[3 + k][t];
            q.o = s_gp[9][t];
            float T[12];
#pragma unroll
            for (int k = 0; k < 12; k++) T[k] = s_T[v - v0][k];
            const ViewInfo& vi = vt.v[v];
            Proj pr;
            project_view<SH < 0, ISO>(P, gg, q, vi, T, pr);
            if (rec.stage) {
                // the pair's entry in the block's list for the binning, in
                // queue order (an invisible pair is marked as such)
                rec.stage[(int64_t)blockIdx.x * kProjBlock * vt.V + qb + i] =
                    pr.valid ? make_uint4(((uint32_t)v << 8) | (uint32_t)t, __float_as_uint(pr.p[2]),
                                          (uint32_t)pr.x0 | ((uint32_t)pr.x1 << 16),
                                          (uint32_t)pr.y0 | ((uint32_t)pr.y1 << 16))
                             : make_uint4(kStageNone, 0u, 0u, 0u);
            }
            if (!pr.valid) continue;
            float col[3];
            if (SH < 0) {
                col[0] = pr.col[0]; col[1] = pr.col[1]; col[2] = pr.col[2];
                bad |= pr.colbad;
            } else {
                float dir[3], dirn;
                bool cclamp[3], cb;
                const int slot = kStageSh ? (int)s_slot[t] : -1;
                if (slot >= 0) {
                    sh_colour_of(SH, CoefStrided<kShSlots>{s_sh + slot}, q.mu[0], q.mu[1], q.mu[2], T, dir, dirn,
                                 col, cclamp, cb);
                } else {
                    const CoefRegs<K3> sh(P.col + (int64_t)gg * K3);
                    sh_colour_of(SH, sh, q.mu[0], q.mu[1], q.mu[2], T, dir, dirn, col, cclamp, cb);
                }
                bad |= cb;
            }
            // the record line in 16-byte stores: base-2 conic with
            // log2(opacity) (the compositing kernels' form), colour and
            // depth, mean and rect (the pad is never read)
            float4* ql = reinterpret_cast<float4*>(rec.line + ((int64_t)v * P.n + gg));
            ql[0] = make_float4(kHalfLog2e * pr.A, 2.f * kHalfLog2e * pr.B, kHalfLog2e * pr.C, log2f(pr.o));
            ql[1] = make_float4(col[0], col[1], col[2], pr.p[2]);
            ql[2] = make_float4(pr.u, pr.v, __uint_as_float((uint32_t)pr.x0 | ((uint32_t)pr.x1 << 16)),
                                __uint_as_float((uint32_t)pr.y0 | ((uint32_t)pr.y1 << 16)));
            atomicOr(&s_vis[v - v0][t >> 6], 1ull << (t & 63));
            atomicOr(&s_vm[t], 1ull << v);
        }
        __syncthreads();
        // the round's visibility words (a wavefront wholly past the Gaussians has none)
        for (int k = threadIdx.x; k < (v1 - v0) * kW; k += kProjBlock) {
            const int64_t word = (int64_t)blockIdx.x * kW + k % kW;
            if (word < vrow) rec.vis[(int64_t)(v0 + k / kW) * vrow + word] = s_vis[k / kW][k % kW];
        }
        if (threadIdx.x == 0) s_qrun = qb + (uint32_t)nq;
        __syncthreads();   // s_vis, s_T, s_ent and s_n are rewritten by the next round
    }
    if (live) rec.vmask[g] = s_vm[threadIdx.x];
    if (rec.stage) {
        // the block's visible records (the bits of its view masks) and its
        // queued pairs
        uint32_t c = (uint32_t)__popcll(s_vm[threadIdx.x]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += (uint32_t)__shfl_xor((int)c, o, 64);
        if (lane == 0) atomicAdd(&s_nvis, c);
        __syncthreads();
        if (threadIdx.x == 0) {
            rec.bcount[blockIdx.x] = s_nvis;
            rec.qcount[blockIdx.x] = s_qrun;
            if (blockIdx.x == 0) rec.bcount[gridDim.x] = 0u;
        }
    }
    // one atomic per wavefront that read a non-finite parameter, from its
    // first active lane
    const uint64_t bad_lanes = __ballot(bad);
    const int first = __ffsll((unsigned long long)__ballot(true)) - 1;
    if (flags && bad_lanes != 0ull && lane == first) atomicOr(flags, kFlagNonFinite);
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

// In-place exclusive prefix sum of a[0, ne), ne <= 4 kProjBlock, by the
// block's threads; returns the total.  Starts and ends with a barrier.
__device__ __forceinline__ int block_scan_excl(int* a, int ne, int* s_wsum) {
    constexpr int kPer = 4;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    int loc[kPer], sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; k++) {
        const int i = kPer * (int)threadIdx.x + k;
        loc[k] = i < ne ? a[i] : 0;
        sum += loc[k];
    }
    int x = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_wsum[w] = x;
    __syncthreads();
    int run = x - sum, total = 0;
#pragma unroll
    for (int i = 0; i < kProjBlock / 64; i++) {
        if (i < w) run += s_wsum[i];
        total += s_wsum[i];
    }
#pragma unroll
    for (int k = 0; k < kPer; k++) {
        const int i = kPer * (int)threadIdx.x + k;
        if (i < ne) a[i] = run;
        run += loc[k];
    }
    __syncthreads();
    return total;
}

// Pack the Gaussians of the span [g0, g0 + kProjBwdSpan) that some view sees
// into s_loc (offset in the span) and s_mask (their view masks), ordered by
// decreasing number of views that see them and, within one count, by
// increasing index.  The backward walks the packed list 64 Gaussians per
// wavefront, each lane looping over its own Gaussian's views: with the list
// sorted by count, the lanes of a wavefront run nearly the same number of
// iterations.  s_hist: ints [V][kBwdPer][kProjBlock / 64].  s_mask may be
// NULL (the caller re-reads the masks).  Returns the number packed (the same
// in every thread).  Ends with a barrier.
__device__ __forceinline__ int pack_by_views(const uint64_t* vmask, int n, int64_t g0, int V, uint16_t* s_loc,
                                             uint64_t* s_mask, int* s_hist, int* s_wsum) {
    constexpr int NW = kProjBlock / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t m[kBwdPer];
    int c[kBwdPer];
#pragma unroll
    for (int j = 0; j < kBwdPer; j++) {
        const int64_t g = g0 + threadIdx.x + kProjBlock * j;
        m[j] = g < n ? vmask[g] : 0ull;
        c[j] = __popcll(m[j]);
    }
    // entry (b, j, w) counts the wavefront's Gaussians of slot j seen by
    // exactly V - b views
    for (int b = 0; b < V; b++)
#pragma unroll
        for (int j = 0; j < kBwdPer; j++) {
            const uint64_t bl = __ballot(c[j] == V - b);
            if (lane == 0) s_hist[(b * kBwdPer + j) * NW + w] = __popcll(bl);
        }
    const int total = block_scan_excl(s_hist, V * kBwdPer * NW, s_wsum);
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int b = 0; b < V; b++)
#pragma unroll
        for (int j = 0; j < kBwdPer; j++) {
            const bool mine = c[j] == V - b;
            const uint64_t bl = __ballot(mine);
            if (mine) {
                const int e = s_hist[(b * kBwdPer + j) * NW + w] + __popcll(bl & lt);
                s_loc[e] = (uint16_t)(threadIdx.x + kProjBlock * j);
                if (s_mask) s_mask[e] = m[j];
            }
        }
    __syncthreads();
    return total;
}

// Colour part of the projection backward for SH colours, one block per span
// of kProjBwdSpan Gaussians, one thread per Gaussian some view sees looping
// over the views that see it (as preprocess_bwd_kernel): the SH coefficient gradient
// sum_v Y(dir_v) dL/dcolour_v over the unclamped channels, the direction's
// gradient mapped to the mean and to the camera centre (the pose tangent's
// translation; the centre does not move under a rotation about itself).
// Compaction slot of the visible record (v, g): the slot base of g's bitmap
// word (its projection block's wavefront, in view v) plus the visible records
// below g in that word (Records::pre)
__device__ __forceinline__ uint32_t record_slot(const Records& rec, int64_t n, int V, int v, int64_t g) {
    const uint64_t wd = rec.vis[(int64_t)v * vis_words(n) + (g >> 6)];
    const int64_t b = g / kProjBlock;
    const int w = (int)((g % kProjBlock) >> 6);
    return rec.pre[(b * V + v) * (kProjBlock / 64) + w] + (uint32_t)__popcll(wd & ((1ull << (g & 63)) - 1ull));
}

// Runs before preprocess_bwd_kernel<SH>, which adds the geometric gradients
// to the means and to the pose partials written here.  Kept apart because the
// coefficient gradients (3K floats per Gaussian) and the geometric chain rule
// together need twice the registers (two wavefronts per SIMD instead of four).
// Each lane copies its Gaussian's coefficients once into LDS (its own
// column, lane-contiguous, so no barrier and no bank conflicts) and reads
// them from there for every view: reading them from the parameter array per
// view made one L2 request per lane and coefficient once the block's
// working set outgrew L1 (70M requests per launch at 16 views of 3M SH3
// Gaussians).
template <int SH>
__global__ __launch_bounds__(kProjBlock, SH >= 3 ? 3 : 4) void sh_bwd_kernel(ViewTable vt, Params P, const float* poses,
                                                            Records rec, const float* g2, Grads G,
                                                            int accumulate, double* pose_part, int pose_blocks) {
    constexpr int K = (SH + 1) * (SH + 1);
    constexpr bool VEC = (3 * K) % 4 == 0;   // a Gaussian's coefficients start 16-byte aligned
    constexpr int kHist = kMaxViews * kBwdPer * (kProjBlock / 64);
    // the packing's histogram lives in the coefficient buffer, which is
    // written only after the packing's last barrier
    __shared__ float s_sh[3 * K * kProjBlock > kHist ? 3 * K * kProjBlock : kHist];
    __shared__ uint16_t s_loc[kProjBwdSpan];
    __shared__ int s_wsum[kProjBlock / 64];
    // dynamic: FP64 pose translation sums [V][3], then the poses' top rows [V][12]
    extern __shared__ double s_dyn[];
    int* s_hist = reinterpret_cast<int*>(s_sh);
    const int w = threadIdx.x >> 6;
    const int64_t g0 = (int64_t)blockIdx.x * kProjBwdSpan;
    const int V = vt.V;
    double* s_pose = s_dyn;
    float* s_T = reinterpret_cast<float*>(s_dyn + 3 * V);
    for (int k = threadIdx.x; k < V * 3; k += kProjBlock) s_pose[k] = 0.0;
    for (int k = threadIdx.x; k < V * 12; k += kProjBlock) s_T[k] = poses[16 * (k / 12) + k % 12];
    if (!accumulate) {
        const int64_t g1 = g0 + kProjBwdSpan < (int64_t)P.n ? g0 + kProjBwdSpan : (int64_t)P.n;
        block_zero(G.means, 3 * g0, 3 * g1);
        block_zero(G.col, 3 * K * g0, 3 * K * g1);
    }
    const int total = pack_by_views(rec.vmask, P.n, g0, V, s_loc, nullptr, s_hist, s_wsum);

    for (int base = 0; base < total; base += kProjBlock) {
        if (base + 64 * w >= total) break;   // nothing left for this wavefront
        const int e = base + (int)threadIdx.x;
        const bool live = e < total;
        const int g = live ? (int)(g0 + s_loc[e]) : 0;
        const uint64_t vm = live ? rec.vmask[g] : 0ull;
        float mx = 0.f, my = 0.f, mz = 0.f;
        if (live) {
            const float* mu = P.means + 3 * (int64_t)g;
            mx = mu[0]; my = mu[1]; mz = mu[2];
        }
        float* my_sh = s_sh + threadIdx.x;
        if (live) {
            const float* src = P.col + (int64_t)g * K * 3;
            if (VEC) {
#pragma unroll
                for (int q = 0; q < 3 * K / 4; q++) {
                    const float4 c4 = reinterpret_cast<const float4*>(src)[q];
                    my_sh[(4 * q) * kProjBlock] = c4.x;
                    my_sh[(4 * q + 1) * kProjBlock] = c4.y;
                    my_sh[(4 * q + 2) * kProjBlock] = c4.z;
                    my_sh[(4 * q + 3) * kProjBlock] = c4.w;
                }
            } else {
#pragma unroll
                for (int k = 0; k < 3 * K; k++) my_sh[k * kProjBlock] = src[k];
            }
        }
        const CoefStrided<kProjBlock> sh{my_sh};
        float gc[3 * K];
#pragma unroll
        for (int k = 0; k < 3 * K; k++) gc[k] = 0.f;
        float dmu[3] = {0.f, 0.f, 0.f};
        // the lane's own views, lowest first
        for (uint64_t rem = vm; rem != 0ull; rem &= rem - 1ull) {
            const int v = __ffsll((unsigned long long)rem) - 1;
            {
                float T[12];
#pragma unroll
                for (int k = 0; k < 12; k++) T[k] = s_T[12 * v + k];
                float dir[3], dirn, col[3];
                bool cclamp[3], cb;
                sh_colour_of(SH, sh, mx, my, mz, T, dir, dirn, col, cclamp, cb);
                const float* a = g2 + (int64_t)record_slot(rec, P.n, V, v, g) * kG2Floats;
                const float dcol[3] = {cclamp[0] ? 0.f : a[6], cclamp[1] ? 0.f : a[7], cclamp[2] ? 0.f : a[8]};
                float Y[16];
                sh_basis<false>(SH, dir[0], dir[1], dir[2], Y, nullptr);
                float sl[K];
#pragma unroll
                for (int l = 0; l < K; l++) {
                    gc[3 * l] += Y[l] * dcol[0];
                    gc[3 * l + 1] += Y[l] * dcol[1];
                    gc[3 * l + 2] += Y[l] * dcol[2];
                    sl[l] = dcol[0] * sh[3 * l] + dcol[1] * sh[3 * l + 1] + dcol[2] * sh[3 * l + 2];
                }
                float dd[3];
                sh_grad_dot<SH>(dir[0], dir[1], dir[2], sl, dd);
                // dir = (mu - C) / |mu - C|
                const float pj = dd[0] * dir[0] + dd[1] * dir[1] + dd[2] * dir[2];
                const float idn = 1.f / dirn;
                float t[3];
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    t[j] = (dd[j] - dir[j] * pj) * idn;
                    dmu[j] += t[j];
                }
                // the centre C = -W^T t moves by -W^T v: dL/dv = -W dL/dC = W t
#pragma unroll
                for (int i = 0; i < 3; i++)
                    atomicAdd(&s_pose[3 * v + i], (double)(T[4 * i] * t[0] + T[4 * i + 1] * t[1] + T[4 * i + 2] * t[2]));
            }
        }
        if (live) {
            float* om = G.means + 3 * (int64_t)g;
            float* oc = G.col + (int64_t)g * 3 * K;
            if (accumulate) {
#pragma unroll
                for (int k = 0; k < 3; k++) om[k] += dmu[k];
#pragma unroll
                for (int k = 0; k < 3 * K; k++) oc[k] += gc[k];
            } else {
#pragma unroll
                for (int k = 0; k < 3; k++) om[k] = dmu[k];
                if (VEC) {
#pragma unroll
                    for (int q = 0; q < 3 * K / 4; q++)
                        reinterpret_cast<float4*>(oc)[q] =
                            make_float4(gc[4 * q], gc[4 * q + 1], gc[4 * q + 2], gc[4 * q + 3]);
                } else {
#pragma unroll
                    for (int k = 0; k < 3 * K; k++) oc[k] = gc[k];
                }
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < V * 6; k += kProjBlock)
        pose_part[((int64_t)(k / 6) * pose_blocks + blockIdx.x) * 6 + k % 6] = k % 6 < 3 ? s_pose[3 * (k / 6) + k % 6] : 0.0;
}

// One block per span of kProjBwdSpan Gaussians.  The block first reads the
// view masks the forward projection left (bit v: visible in view v); the
// Gaussians visible in none get a zero gradient (or nothing, when
// accumulating) and the others are packed, most-seen first, into a list that
// the block then walks 256 at a time.  Each lane loops over the views that
// see its Gaussian only, and the sort by view count gives the lanes of a
// wavefront nearly equal trip counts, so the per-view recomputation runs on
// nearly full wavefronts (a loop over all views, skipping a view only when
// no lane sees it, keeps about one lane in ten busy at 16 views).  The
// per-Gaussian gradient is summed over views in registers; the per-view pose
// 6-vector is added into the block's FP64 slots in LDS (atomically: the
// summation order is not fixed, as for the compositing backward's sums).
// With SH colours the colour part runs in sh_bwd_kernel first: this kernel
// then adds its mean and pose gradients to what that one wrote.  At most 128
// VGPRs (four waves per SIMD; it fits without spilling).  ISO: the camera
// covariance r^2 I does not turn with the camera, so the covariance gradient
// reaches only the log radius (2 r^2 trace of dL/dSigma_c) and the pose only
// through the mean.
template <int SH, bool ISO>
__global__ __launch_bounds__(kProjBlock, 4) void preprocess_bwd_kernel(ViewTable vt, Params P, const float* poses,
                                                                    Records rec, const float* g2, Grads G,
                                                                    int accumulate, double* pose_part,
                                                                    int pose_blocks) {
    constexpr int K = SH < 0 ? 1 : (SH + 1) * (SH + 1);
    __shared__ uint16_t s_loc[kProjBwdSpan];
    __shared__ uint64_t s_mask[kProjBwdSpan];
    __shared__ int s_hist[kMaxViews * kBwdPer * (kProjBlock / 64)];
    __shared__ int s_wsum[kProjBlock / 64];
    // dynamic: FP64 pose sums [V][6], the poses' top rows [V][12], and the
    // cameras [V][6] (fx, fy, cx, cy, W, H)
    extern __shared__ double s_dyn[];
    const int w = threadIdx.x >> 6;
    const int64_t g0 = (int64_t)blockIdx.x * kProjBwdSpan;
    const int V = vt.V;
    double* s_pose = s_dyn;
    float* s_T = reinterpret_cast<float*>(s_dyn + 6 * V);
    float* s_cam = s_T + 12 * V;
    for (int k = threadIdx.x; k < V * 6; k += kProjBlock) s_pose[k] = 0.0;
    for (int k = threadIdx.x; k < V * 12; k += kProjBlock) s_T[k] = poses[16 * (k / 12) + k % 12];
    for (int k = threadIdx.x; k < V; k += kProjBlock) {
        const ViewInfo& c = vt.v[k];
        s_cam[6 * k] = c.fx; s_cam[6 * k + 1] = c.fy; s_cam[6 * k + 2] = c.cx; s_cam[6 * k + 3] = c.cy;
        s_cam[6 * k + 4] = (float)c.W; s_cam[6 * k + 5] = (float)c.H;
    }
    if (!accumulate) {
        // the whole span's gradient starts at zero; the walk below overwrites
        // the visible Gaussians' entries after the barrier (with SH colours
        // sh_bwd_kernel has already written the colour and mean gradients)
        const int64_t g1 = g0 + kProjBwdSpan < (int64_t)P.n ? g0 + kProjBwdSpan : (int64_t)P.n;
        if (SH < 0) {
            block_zero(G.means, 3 * g0, 3 * g1);
            block_zero(G.col, 3 * g0, 3 * g1);
        }
        if (ISO) {
            block_zero(G.ls, g0, g1);
        } else {
            block_zero(G.ls, 3 * g0, 3 * g1);
            block_zero(G.q, 4 * g0, 4 * g1);
        }
        block_zero(G.opl, g0, g1);
    }
    const int total = pack_by_views(rec.vmask, P.n, g0, V, s_loc, s_mask, s_hist, s_wsum);

    for (int base = 0; base < total; base += kProjBlock) {
        if (base + 64 * w >= total) break;   // nothing left for this wavefront
        const int e = base + (int)threadIdx.x;
        const bool live = e < total;
        const int g = live ? (int)(g0 + s_loc[e]) : 0;
        const uint64_t vmask = live ? s_mask[e] : 0ull;
        float gm[3] = {0.f, 0.f, 0.f}, gl[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f}, go = 0.f;
        float gc[3] = {0.f, 0.f, 0.f};   // RGB only
        GPrep gp;
        gp.ok = false;
        if (live) gauss_prep<ISO>(P, g, gp);

        // the lane's own views, lowest first
        for (uint64_t rem = vmask; rem != 0ull; rem &= rem - 1ull) {
            const int v = __ffsll((unsigned long long)rem) - 1;
            float pose[6];
            {
                ViewInfo vi;
                vi.fx = s_cam[6 * v]; vi.fy = s_cam[6 * v + 1]; vi.cx = s_cam[6 * v + 2]; vi.cy = s_cam[6 * v + 3];
                vi.W = (int)s_cam[6 * v + 4]; vi.H = (int)s_cam[6 * v + 5];
                float T[12];
#pragma unroll
                for (int k = 0; k < 12; k++) T[k] = s_T[12 * v + k];
                Proj pr;
                project_view<false, ISO>(P, g, gp, vi, T, pr);
                const float4* a4 =
                    reinterpret_cast<const float4*>(g2 + (int64_t)record_slot(rec, P.n, V, v, g) * kG2Floats);
                const float4 a0 = a4[0], a1 = a4[1], a2 = a4[2];
                // undo the compositing kernel's constant factors (g2 layout)
                const float du = a0.x * (1.f / kHalfLog2e), dv = a0.y * (1.f / kHalfLog2e);
                const float dA = 0.5f * a0.z, dB = a0.w, dC = 0.5f * a1.x;
                const float odo = a1.y;   // o dL/do
                const float dcol[3] = {a1.z, a1.w, a2.x};
                const float dz = a2.y;
                float dmu[3] = {0.f, 0.f, 0.f};

                // colour (RGB: the gradient is dL/dcolour itself; SH: sh_bwd_kernel)
                if (SH < 0) {
                    gc[0] += dcol[0]; gc[1] += dcol[1]; gc[2] += dcol[2];
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

                if (ISO) {
                    // Sc = r^2 I: dL/dlog r = 2 r^2 (Gs_xx + Gs_yy + Gs_zz)
                    gl[0] += 2.f * pr.s[0] * pr.s[0] * (Gs[0] + Gs[4] + Gs[8]);
                } else {
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
                            GR[3 * r_ + c] =
                                GS[3 * r_] * pr.R[c] + GS[3 * r_ + 1] * pr.R[3 + c] + GS[3 * r_ + 2] * pr.R[6 + c];
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
                    dq[1] = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] +
                                   w * dR[7] - 2.f * x * dR[8]);
                    dq[2] = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                                   z * dR[7] - 2.f * y * dR[8]);
                    dq[3] = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] + y * dR[5] +
                                   x * dR[6] + y * dR[7]);
                    const float qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
                    const float iqn = 1.f / pr.qn;
#pragma unroll
                    for (int k = 0; k < 4; k++) gq[k] += (dq[k] - pr.qh[k] * qd) * iqn;
                }

                // p = W mu + t
                dmu[0] += T[0] * dpx + T[4] * dpy + T[8] * dpz;
                dmu[1] += T[1] * dpx + T[5] * dpy + T[9] * dpz;
                dmu[2] += T[2] * dpx + T[6] * dpy + T[10] * dpz;
                gm[0] += dmu[0]; gm[1] += dmu[1]; gm[2] += dmu[2];

                // pose (left perturbation): dp/dv = I, dp/dw = -[p]x, and Sc picks
                // up [w]x Sc - Sc [w]x (the camera centre's share: sh_bwd_kernel)
                pose[0] = dpx;
                pose[1] = dpy;
                pose[2] = dpz;
                const float Sf[9] = {S[0], S[1], S[2], S[1], S[3], S[4], S[2], S[4], S[5]};
                // N = Sc Gs - Gs Sc (antisymmetric); d/dw = 2 (N12, N20, N01)
                auto Nij = [&](int i, int j) {
                    return Sf[3 * i] * Gs[j] + Sf[3 * i + 1] * Gs[3 + j] + Sf[3 * i + 2] * Gs[6 + j] -
                           (Gs[3 * i] * Sf[j] + Gs[3 * i + 1] * Sf[3 + j] + Gs[3 * i + 2] * Sf[6 + j]);
                };
                pose[3] = py * dpz - pz * dpy + (ISO ? 0.f : 2.f * Nij(1, 2));
                pose[4] = pz * dpx - px * dpz + (ISO ? 0.f : 2.f * Nij(2, 0));
                pose[5] = px * dpy - py * dpx + (ISO ? 0.f : 2.f * Nij(0, 1));
            }
#pragma unroll
            for (int k = 0; k < 6; k++) atomicAdd(&s_pose[6 * v + k], (double)pose[k]);
        }
        if (live) {
            float* om = G.means + 3 * (int64_t)g;
            if (accumulate) {
#pragma unroll
                for (int k = 0; k < 3; k++) om[k] += gm[k];
                if (ISO) {
                    G.ls[g] += gl[0];
                } else {
#pragma unroll
                    for (int k = 0; k < 3; k++) G.ls[3 * (int64_t)g + k] += gl[k];
#pragma unroll
                    for (int k = 0; k < 4; k++) G.q[4 * (int64_t)g + k] += gq[k];
                }
                G.opl[g] += go;
            } else {
#pragma unroll
                for (int k = 0; k < 3; k++) om[k] = SH < 0 ? gm[k] : om[k] + gm[k];   // SH: add to the colour share
                if (ISO) {
                    G.ls[g] = gl[0];
                } else {
#pragma unroll
                    for (int k = 0; k < 3; k++) G.ls[3 * (int64_t)g + k] = gl[k];
#pragma unroll
                    for (int k = 0; k < 4; k++) G.q[4 * (int64_t)g + k] = gq[k];
                }
                G.opl[g] = go;
            }
            if (SH < 0) {
                float* oc = G.col + 3 * (int64_t)g;
#pragma unroll
                for (int k = 0; k < 3; k++) oc[k] = accumulate ? oc[k] + gc[k] : gc[k];
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < V * 6; k += kProjBlock) {
        const double t = s_pose[k];
        double* dst = pose_part + ((int64_t)(k / 6) * pose_blocks + blockIdx.x) * 6 + k % 6;
        if (SH < 0) *dst = t; else *dst += t;   // SH: the colour path's partial is there already
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

template <int SH, bool ISO>
void fwd_one(const ViewTable& vt, const Params& P, const float* poses, Records rec, hipStream_t s,
             uint32_t* flags) {
    const unsigned nb = (unsigned)((P.n + kProjBlock - 1) / kProjBlock);
    preprocess_fwd_kernel<SH, ISO><<<nb, kProjBlock, 0, s>>>(vt, P, poses, rec, flags);
}

template <bool ISO>
hipError_t fwd_sh(const ViewTable& vt, const Params& P, const float* poses, Records rec, hipStream_t s,
                  uint32_t* flags) {
    switch (P.sh) {
        case -1: fwd_one<-1, ISO>(vt, P, poses, rec, s, flags); break;
        case 0: fwd_one<0, ISO>(vt, P, poses, rec, s, flags); break;
        case 1: fwd_one<1, ISO>(vt, P, poses, rec, s, flags); break;
        case 2: fwd_one<2, ISO>(vt, P, poses, rec, s, flags); break;
        case 3: fwd_one<3, ISO>(vt, P, poses, rec, s, flags); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int SH, bool ISO>
void bwd_one(const ViewTable& vt, const Params& P, const float* poses, const Records& rec, const float* g2, Grads G,
             int accumulate, double* pose_part, int nb, hipStream_t s, hipEvent_t colour_done) {
    const size_t dyn_sh = (size_t)vt.V * (3 * sizeof(double) + 12 * sizeof(float));
    const size_t dyn_geo = (size_t)vt.V * (6 * sizeof(double) + 18 * sizeof(float));
    if constexpr (SH >= 0) {
        sh_bwd_kernel<SH><<<nb, kProjBlock, dyn_sh, s>>>(vt, P, poses, rec, g2, G, accumulate, pose_part, nb);
        if (colour_done) (void)hipEventRecord(colour_done, s);
    }
    preprocess_bwd_kernel<SH, ISO><<<nb, kProjBlock, dyn_geo, s>>>(vt, P, poses, rec, g2, G, accumulate, pose_part,
                                                                  nb);
}

template <bool ISO>
hipError_t bwd_sh(const ViewTable& vt, const Params& P, const float* poses, const Records& rec, const float* g2,
                  Grads G, int accumulate, double* pose_part, int nb, hipStream_t s, hipEvent_t cd) {
    switch (P.sh) {
        case -1: bwd_one<-1, ISO>(vt, P, poses, rec, g2, G, accumulate, pose_part, nb, s, cd); break;
        case 0: bwd_one<0, ISO>(vt, P, poses, rec, g2, G, accumulate, pose_part, nb, s, cd); break;
        case 1: bwd_one<1, ISO>(vt, P, poses, rec, g2, G, accumulate, pose_part, nb, s, cd); break;
        case 2: bwd_one<2, ISO>(vt, P, poses, rec, g2, G, accumulate, pose_part, nb, s, cd); break;
        case 3: bwd_one<3, ISO>(vt, P, poses, rec, g2, G, accumulate, pose_part, nb, s, cd); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_preprocess_fwd(const ViewTable& vt, const Params& P, const float* poses, Records rec,
                                 hipStream_t s, uint32_t* flags) {
    if (P.n == 0) return hipSuccess;
    return P.iso ? fwd_sh<true>(vt, P, poses, rec, s, flags) : fwd_sh<false>(vt, P, poses, rec, s, flags);
}

hipError_t launch_preprocess_bwd(const ViewTable& vt, const Params& P, const float* poses, const Records& rec,
                                 const float* g2, Grads G, int accumulate, double* pose_part, int64_t pose_blocks,
                                 hipStream_t s, hipEvent_t colour_done) {
    if (P.n == 0) {
        if (colour_done) (void)hipEventRecord(colour_done, s);
        return hipSuccess;
    }
    const int nb = (P.n + kProjBwdSpan - 1) / kProjBwdSpan;
    if (nb != pose_blocks) return hipErrorInvalidValue;
    return P.iso ? bwd_sh<true>(vt, P, poses, rec, g2, G, accumulate, pose_part, nb, s, colour_done)
                 : bwd_sh<false>(vt, P, poses, rec, g2, G, accumulate, pose_part, nb, s, colour_done);
}

hipError_t launch_pose_finalize(const ViewTable& vt, const double* pose_part, int64_t pose_blocks,
                                const double* rp_acc, float rp_weight, float* dL_dpose, hipStream_t s) {
    pose_finalize_kernel<<<vt.V, 256, 0, s>>>(pose_part, (int)pose_blocks, rp_acc, rp_weight, dL_dpose);
    return hipGetLastError();
}

}  // namespace gs
