// Internal declarations shared by the HIP kernels and the host runtime.
// Not part of the public ABI (include/gs.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gs {

constexpr int kMaxViews = 64;

// Forward-model constants (Sec. 3.4 rasterisation; the paper gives none, these
// are the thresholds the ABI documents).
constexpr float kZNear = 0.2f;
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr float kLog2AlphaMinInv = 7.99435343685885793f;   // log2(255)
constexpr float kDilate = 0.3f;
constexpr float kJClamp = 1.3f;

// SSIM term of the mapping loss: outputs per workgroup of the SSIM kernels
constexpr int kSsimTW = 32;
constexpr int kSsimTH = 16;

// Per-view constants, passed by value in every launch (no upload, graph safe).
struct ViewInfo {
    int W, H;
    int tiles_x, tiles_y;
    int tile_off;   // global id of this view's first compositing tile
    int bins_x, bins_y;
    int bin_off;    // global id of this view's first bin
    int pix_off;    // first pixel of this view in the concatenated images
    int ssim_off;   // global id of this view's first SSIM tile
    float fx, fy, cx, cy;
    float lsc;      // dL/dC scale: w_color / (V * 3 * H * W)
    float lsd;      // dL/dD scale: w_depth / (V * H * W)
};

// Binning works on bins of bw x bh pixels; compositing on tiles of tw x th
// pixels (bw, bh multiples of tw, th), each tile reading its bin's list and
// keeping the entries whose support rect meets the tile.
struct ViewTable {
    int V;
    int tw, th;
    int bw, bh;
    int ppt;        // pixels per thread in the compositing kernels (1, 2 or 4)
    int n_bins;
    int n_tiles;
    int n_pix;
    int n_ssim_tiles;
    int n;          // Gaussians
    ViewInfo v[kMaxViews];
};

// Workgroups of a launch are dealt round-robin to the 8 XCDs (each with its
// own L2).  xcd_slot maps the linear workgroup id to an item index so that
// every XCD processes one contiguous range of items: neighbouring tiles then
// share their halos and lists in one L2.
constexpr int kNumXcd = 8;
__host__ __device__ inline int64_t xcd_slot(int64_t wg, int64_t n) {
    const int64_t q = n / kNumXcd, r = n % kNumXcd;
    const int64_t k = wg % kNumXcd, slot = wg / kNumXcd;
    return k * q + (k < r ? k : r) + slot;
}

// The compositing tiles of a ViewTable, compact enough to pass beside one.
struct TileGrid {
    int tw, th;
    int tile_off[kMaxViews];
    int tiles_x[kMaxViews];
    int tiles_y[kMaxViews];
};

inline TileGrid tile_grid(const ViewTable& vt) {
    TileGrid g{};
    g.tw = vt.tw;
    g.th = vt.th;
    for (int v = 0; v < vt.V; v++) {
        g.tile_off[v] = vt.v[v].tile_off;
        g.tiles_x[v] = vt.v[v].tiles_x;
        g.tiles_y[v] = vt.v[v].tiles_y;
    }
    return g;
}

// Gaussian parameters (device, FP32 SoA).  Anisotropic: ls [n][3] log-scales,
// q [n][4] quaternions.  Isotropic (iso = 1, the paper's eight-parameter
// Gaussian): ls [n] log radii, q unused.
struct Params {
    const float* means;
    const float* ls;
    const float* q;
    const float* opl;
    const float* col;
    int n;
    int sh;         // -1 = RGB
    int iso;
};

// floats per Gaussian in the parameter (and Adam moment) layout
__host__ __device__ inline int64_t floats_per_gaussian(int K3, int iso) { return (iso ? 5 : 11) + (int64_t)K3; }

struct Grads {
    float* means;
    float* ls;
    float* q;
    float* opl;
    float* col;
};

// Per-record 2D gradients summed by the compositing backward (twelve floats,
// ten used): with c = log2(e)/2, sd = dL/dsigma per pixel and (dx, dy) the
// pixel offset from the projected mean,
//   [0] c dL/du = -sum sd (A' dx + B' dy / 2)   [1] c dL/dv = -sum sd (C' dy + B' dx / 2)
//   [2] 2 dL/dA = sum sd dx^2   [3] dL/dB = sum sd dx dy   [4] 2 dL/dC = sum sd dy^2
//   [5] o dL/do = -sum sd       [6..8] dL/dcolour          [9] dL/dz
// The projection backward undoes the constant factors once per record.
// They sit in a dense array indexed by the record's compaction slot o (its
// rank among the visible records, Records::pre), kG2Floats floats each, so
// that the backward kernels read 48 bytes per visible record from a few
// hundred MB rather than a line each from the whole record array.
constexpr int kG2Floats = 12;

// One (view, Gaussian) record, r = v*n + g, in one 64-byte line: what the
// projection leaves for binning and compositing.  The projection of a
// visible record writes its first 48 bytes; compositing reads them per
// staged entry, instead of partial lines of several separate arrays.
struct alignas(64) RecLine {
    float4 conic;   // (A', B', C', log2 opacity): conic in base-2 units, see frag_col
    float4 col;     // (r, g, b, depth)
    float2 xy;      // projected mean
    uint2 rect;     // inclusive pixel rect (x0 | x1 << 16, y0 | y1 << 16)
    float4 pad0;
};
static_assert(sizeof(RecLine) == 64, "one record per 64-byte line");

// Visibility bitmap of the records: word v * vis_words(n) + g / 64, bit g % 64
// set when record (v, g) is visible.  Each view's row is padded to whole
// words, so one projection wavefront (64 consecutive Gaussians, a multiple
// of 64 apart) writes one word per view from its ballot.  Binning scans the
// padded index p = v * 64 vis_words(n) + g.
__host__ __device__ inline int64_t vis_words(int64_t n) { return (n + 63) / 64; }

struct Records {
    RecLine* line;    // R record lines
    uint64_t* vis;    // V * vis_words(n) visibility words
    uint64_t* vmask;  // per Gaussian (n entries): bit v set when its record in view v is visible
    // The projection's lists for the binning (stage NULL: none): block b of
    // the forward projection writes one entry per pair it queued, qcount[b]
    // in all, at stage[b * kProjBlock * V ...]: (view << 8 | thread, depth
    // bits, rect) for a visible record, kStageNone in .x for a rejected pair;
    // bcount[b] = its visible records, and block 0 zeroes bcount[blocks], so
    // that an exclusive scan of the blocks + 1 counts ends with the total.
    uint4* stage;
    uint32_t* bcount;
    uint32_t* qcount;
    // After binning: info[o] = (record, bin count | view << 24, rect) of the
    // visible record in compaction slot o, and for projection block b,
    // pre[(b * V + v) * 4 + w] = the slot of the first visible record of its
    // wavefront w in view v; record (v, g) of block b's wavefront w then has
    // slot pre[...] + (the visible records below g in its bitmap word).
    // The sorted pairs carry slots, not records.
    const uint4* info;
    uint32_t* pre;
};
constexpr uint32_t kStageNone = 0xffffffffu;

// Gaussians per block of the forward projection
constexpr int kProjBlock = 256;
inline int64_t proj_blocks(int64_t n) { return (n + kProjBlock - 1) / kProjBlock; }

// Gaussians per block of the projection backward; the per-view pose partial
// sums are kept per such block (Layout::pose_blocks = ceil(n / kProjBwdSpan)).
constexpr int kProjBwdSpan = 1024;

// Largest radix-sort grid: each block sorts a contiguous range of the keys,
// so the digit histograms (256 x grid words) and their scans stay small
// however large the key-count bound is.
constexpr int kRsMaxGrid = 512;
// Keys one radix-sort block ranks per tile (the layout sizes the histogram
// table as 256 x min(ceil(bound / kRsTileKeys), kRsMaxGrid)).
constexpr int kRsTileKeys = 2048;

// Device layout of the forward state / mapping workspace (byte offsets).
struct Layout {
    int64_t R;            // V * n records
    int64_t Rp;           // V * 64 vis_words(n): records in the padded index of the visibility bitmap
    int64_t cap;          // pair capacity
    int64_t n_bins, n_tiles, n_pix;
    int64_t sort_blocks;  // radix-sort grid for max(R, cap), at most kRsMaxGrid
    size_t off_line, off_vis;                     // R record lines (gradient sums inside), visibility bitmap
    size_t off_vmask;                             // n uint64 (last, so it moves no other array)
    size_t off_info;                              // R uint4: (record, bin count, rect) per visible record (binning)
    size_t off_sinfo;                             // R uint4: the same entries in depth order; before the
                                                  // depth sort, the projection's per-block lists (stage)
    size_t off_k0, off_v0, off_k1, off_v1;        // record sort (R)
    size_t off_pk0, off_pv0, off_pk1, off_pv1;    // pair sort (cap)
    size_t off_hist;                              // 256 * sort_blocks
    size_t off_ranges;                            // n_bins uint2
    size_t off_tfin, off_last;                    // n_pix
    size_t off_torder, off_twork;                 // tile order and work, sized for the smallest tile
    size_t off_tbucket;                           // per-tile work bucket (u8), same size
    size_t off_posepart;                          // V * pose_blocks * 6 doubles
    size_t off_scalars;                           // counters and flags
    size_t off_lb;                                // chained-scan tile status words (u64), right after the scalars
    int64_t n_chunks;                             // 2048-record chunks of the padded records (binning)
    int64_t lb_tiles_chunk, lb_tiles_hist;        // tiles of a chunk-sum scan and of a radix histogram scan
    int64_t lb_tiles_proj;                        // tiles of the scan of the projection blocks' counts
    size_t off_chunk;                             // n_chunks u64 chunk sums / offsets
    size_t off_bcount;                            // proj_blocks(n) + 1 u32 visible counts / offsets
    size_t off_qcount;                            // proj_blocks(n) u32 queued pairs
    size_t off_pre;                               // proj_blocks(n) * V * 4 u32 slot bases (Records::pre)
    size_t off_g2;                                // R * kG2Floats floats: gradient sums by compaction slot
    // mapping workspace only
    size_t off_dC, off_dD;                        // upstream gradients
    size_t off_tilepart;                          // tile partials (sized for the smallest tile)
    size_t off_rpacc;                             // V * 9 doubles (accumulators, per-view loss)
    size_t off_ssim_part;                         // 9 * n_pix floats (SSIM partials)
    size_t off_ssim_tiles;                        // 3 * n_ssim_tiles doubles
    size_t bytes;
    int64_t pose_blocks;
};

// scalars block (u32 unless noted), at off_scalars.  kFlags: this step's
// status bits (cleared when a step starts); kSticky: the OR of kFlags over the
// steps since gs_step_status last read it (never cleared by a step).  kLb*:
// arrival counters of the chained scans (visible counts and pair counts per
// chunk, radix histograms: up to kLbHistUses passes per step).
enum ScalarSlot {
    kNVis = 0, kNPairs = 1, kFlags = 2, kSticky = 3, kPairsLo = 4, kPairsHi = 5,
    kLbVis = 6, kLbPairs = 7, kLbHist0 = 8, kLbProj = 16, kNumScalars = 17
};
constexpr int kLbHistUses = kLbProj - kLbHist0;
// kFlags bits: pair capacity exceeded; a chained scan gave up waiting; a
// Gaussian parameter the step read is not finite
constexpr uint32_t kFlagCapacity = 1u, kFlagLookback = 2u, kFlagNonFinite = 4u;
// status words of the chained scans: two chunk-sum scans (visible records,
// pairs), then kLbHistUses histogram scans, then the projection blocks' counts
inline int64_t lb_words(const Layout& L) {
    return 2 * L.lb_tiles_chunk + (int64_t)kLbHistUses * L.lb_tiles_hist + L.lb_tiles_proj;
}

// tiles_bound: per-tile buffers (workspace) are sized for max(tiles_bound, n_tiles) tiles
Layout make_layout(const ViewTable& vt, int64_t n, int64_t cap, bool workspace, int64_t tiles_bound = 0);

// ---------------------------------------------------------------------------
// launchers (each enqueues kernels on `s` and returns hipGetLastError())
// ---------------------------------------------------------------------------
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);
// zero the gradient sums of the visible records (device count *nvis, at most bound)
hipError_t launch_zero_g2(const uint32_t* nvis, float* g2, int64_t bound, hipStream_t s);
hipError_t launch_zero_f64(double* p, int n, hipStream_t s);
// step[0] += gaussians, step[1] += poses (the two update counters)
hipError_t launch_step_bump(int32_t* step, int gaussians, int poses, hipStream_t s, const uint32_t* flags = nullptr);
// pout = Exp(xi) pin per view (device [V][16], [V][6]; may alias)
hipError_t launch_pose_retract(int V, const float* pin, const float* xi, float* pout, hipStream_t s);
// out = J_l(xi)^T g per view (device [V][6] each)
hipError_t launch_pose_tangent_grad(int V, const float* xi, const float* g, float* out, hipStream_t s);
// binning entry point: each record's caller-given rect clipped into its line,
// and the visibility bitmap of the non-empty ones
hipError_t launch_rect_tiles(const ViewTable& vt, const uint2* rect, RecLine* lines, uint64_t* vis, int64_t n,
                             hipStream_t s);

// flags (nullable, device u32): OR-ed with kFlagNonFinite when a mean,
// log-scale, quaternion or opacity logit, or the colour of a visible record,
// is not finite
hipError_t launch_preprocess_fwd(const ViewTable& vt, const Params& P, const float* poses, Records rec,
                                 hipStream_t s, uint32_t* flags = nullptr);
// colour_done (nullable): with SH colours, recorded on s once the colour
// gradients are complete (after the colour kernel, before the geometric one)
hipError_t launch_preprocess_bwd(const ViewTable& vt, const Params& P, const float* poses, const Records& rec,
                                 const float* g2, Grads G, int accumulate, double* pose_part, int64_t pose_blocks,
                                 hipStream_t s, hipEvent_t colour_done = nullptr);
hipError_t launch_pose_finalize(const ViewTable& vt, const double* pose_part, int64_t pose_blocks,
                                const double* rp_acc, float rp_weight, float* dL_dpose, hipStream_t s);

// Clears the scalars block (all but kSticky) and the chained-scan status
// words; enqueued first in every pass that bins, before the projection, whose
// non-finite check already writes kFlags.
hipError_t launch_status_clear(const Layout& L, char* base, hipStream_t s);

// Binning: records -> sorted pair values (compaction slots) and tile ranges.
// All sizes bounded by the layout; counts live on the device in the scalars
// block.  staged: the forward projection listed the visible records per block
// (Records::stage), so the compaction moves those lists instead of reading the
// bitmap, and writes the slot bases (Records::pre); zero_g2 (nullable): the
// gradient sums of the visible records are zeroed on the way.
hipError_t launch_binning(const ViewTable& vt, const Layout& L, char* base, const uint64_t* vis,
                          const RecLine* lines, const float* depth_src, bool staged, float* zero_g2,
                          int64_t pair_bound, hipStream_t s, uint32_t** sorted_vals_out);
// first half of binning (visibility, depth sort, pair emission); leaves the
// pair total on the device (kPairsLo/Hi) and flags an exceeded capacity
hipError_t launch_binning_count(const ViewTable& vt, const Layout& L, char* base, const uint64_t* vis,
                                const RecLine* lines, const float* depth_src, bool staged, float* zero_g2,
                                hipStream_t s);
// the record of each of the n (device count) sorted pair slots, for callers
// that take records: out[i] = info[slots[i]].x
hipError_t launch_slots_to_records(const uint32_t* slots, const uint4* info, const uint32_t* n, int64_t bound,
                                   uint32_t* out, hipStream_t s);
// second half: the pairs' sort by bin (pair_bound: an upper bound of the
// pair count, which is read on the device) and the per-bin ranges
hipError_t launch_binning_sort(const ViewTable& vt, const Layout& L, char* base, int64_t pair_bound, hipStream_t s,
                               uint32_t** sorted_vals_out);

struct LossArgs {
    const float* tc;
    const float* td;
    const float* mask;
    int use_gate;
    float gamma;
    float* dC;
    float* dD;
    double2* tile_part;
    // (nullable) the gradient sums of the *nvis visible records, zeroed by
    // the compositing blocks after their tiles (a grid-stride fill that the
    // compute-bound forward hides)
    float* g2;
    const uint32_t* nvis;
};

// Order in which the compositing launches take their tiles (device, n_tiles
// each): `order` is filled by the launchers themselves, heaviest first;
// `work` receives, per tile, the list entries the forward staged, which
// orders the backward.
struct TileSched {
    uint32_t* order;
    uint32_t* work;
    uint8_t* bucket;   // per tile being ordered: its work bucket (scratch of the ordering)
};

// counts (nullable, device u64[4]): += candidates visited (rect contains the
// pixel, up to and including the terminating one), fragments blended, list
// entries staged, bin-list entries scanned
hipError_t launch_composite_fwd(const ViewTable& vt, const uint2* ranges, const uint32_t* vals, const Records& rec,
                                float* color, float* depth, float* alpha, float* tfin, uint32_t* last,
                                const LossArgs* loss, const TileSched& ts, hipStream_t s,
                                unsigned long long* counts = nullptr);
// vt: the backward's own tiling (same bins); vtf: the forward's tiling, whose
// per-tile work orders the backward's tiles.  ordered: ts.order already holds
// that order (launch_order_tiles ran after the forward); else it is computed
// first.
hipError_t launch_composite_bwd(const ViewTable& vt, const uint2* ranges, const uint32_t* vals, const Records& rec,
                                const float* tfin, const uint32_t* last, const float* dC, const float* dD,
                                const float* dA, float* g2, const TileSched& ts, const ViewTable& vtf,
                                bool ordered, hipStream_t s);
// the backward's tile order (heaviest first) from the forward's per-tile work
hipError_t launch_order_tiles(const ViewTable& vt, const ViewTable& vtf, const uint2* ranges, const TileSched& ts,
                              hipStream_t s);

// loss_out [1 + 4V]: total, then (Lc, Ld, Lr, Ls) per view; ssim_part (nullable)
// holds per-(channel, SSIM tile) sums of the SSIM map, channel-major
// view_tot: device double [V] scratch
// scal (nullable): the scalars block; kFlags is then OR-ed into kSticky
hipError_t launch_loss_reduce(const ViewTable& vt, const double2* tile_part, const double* rp_acc,
                              const double* ssim_part, float w_color, float w_depth, float w_reproj, float w_ssim,
                              float* loss_out, double* view_tot, hipStream_t s, uint32_t* scal = nullptr);

// SSIM (mapping loss, Sec. 3.4) of planar colour images img against ref.
// part: device float [9 * n_pix] scratch (per pixel and channel: the SSIM map's
// partials with respect to the window means of x, x^2 and xy); tile_sum:
// device double [3 * n_ssim_tiles] (channel-major).  The forward fills both; the backward adds
// -w_v / (3 H W) * d(sum of the view's SSIM map)/d img into dimg, with w_v =
// wdev[v] if wdev is not null, else wconst.
hipError_t launch_ssim_fwd(const ViewTable& vt, const float* img, const float* ref, float* part, double* tile_sum,
                           hipStream_t s);
hipError_t launch_ssim_bwd(const ViewTable& vt, const float* img, const float* ref, const float* part,
                           const float* wdev, float wconst, float* dimg, hipStream_t s);
// per-view mean SSIM from the tile sums
hipError_t launch_ssim_reduce(const ViewTable& vt, const double* tile_sum, float* ssim_out, hipStream_t s);
// dpts (nullable, device [M][3]): dh/dP per match, unscaled (0 for excluded
// matches); launch_reproj_points_scale then multiplies by weight / matches of
// the view, once acc holds the counts
hipError_t launch_reproj(const ViewTable& vt, const float* poses, const float* pts, const float* uv,
                         const int32_t* vid, int64_t M, float delta, float* residual, double* acc, hipStream_t s,
                         float* dpts = nullptr);
hipError_t launch_reproj_points_scale(const ViewTable& vt, const int32_t* vid, int64_t M, const double* acc,
                                      float weight, float* dpts, hipStream_t s);
hipError_t launch_reproj_finalize(const ViewTable& vt, const double* acc, float weight, float* loss,
                                  float* dL_dpose, hipStream_t s);

// exclusive scan of a[0..n) into out (u32), *total32 = sum; bsum needs
// max(1, ceil(n / 2048)) entries
hipError_t launch_scan_u32(const uint32_t* a, int64_t n, uint32_t* out, uint32_t* bsum, uint32_t* total32,
                           hipStream_t s);
inline int64_t scan_bsum_entries(int64_t n) { return n <= 0 ? 1 : (n + 2047) / 2048; }

// Map maintenance (Sec. 3.4).  Gaussian arrays as in Params, `col` with 3K
// floats per Gaussian.
struct GaussOut {
    float* means;
    float* ls;
    float* q;
    float* opl;
    float* col;
};
// Adam moments (m, v) of a layout for n Gaussians: groups of width 3, 3, 4,
// 1, 3K floats per Gaussian (isotropic: 3, 1, 0, 1, 3K), then 6V pose floats
struct AdamIO {
    const float* m_in;
    const float* v_in;
    float* m_out;
    float* v_out;
    const int32_t* step_in;
    int32_t* step_out;
};
// pruning: keep Gaussians with opacity logit >= logit_tau (compared in FP64), in order; scratch
// u32 flag[n], off[n], bsum[scan_bsum_entries(n)], total[1]; n_out device
// int64 = kept count; adam (nullable m_in) re-laid out for the kept ones
hipError_t launch_prune(const Params& in, int K3, double logit_tau, GaussOut out, const AdamIO* adam, int V,
                        uint32_t* flag, uint32_t* off, uint32_t* bsum, uint32_t* total, int64_t* n_out,
                        hipStream_t s);
// densification: append a Gaussian for every selected pixel after the n
// existing ones (at most capacity in all); counts device int64[2] = (Gaussians
// now held, Gaussians the selection asked for); scratch as for pruning over
// the n_pix pixels
hipError_t launch_densify(const ViewTable& vt, const float* poses, const float* alpha, const float* tc,
                          const float* td, double gamma, int all_pixels, GaussOut g, int n, int K, int iso,
                          int64_t capacity, const AdamIO* adam, uint32_t* flag, uint32_t* off, uint32_t* bsum,
                          uint32_t* total, int64_t* counts, hipStream_t s);

struct AdamGroups {
    float* p[5];
    const float* g[5];
    int64_t cnt[5];
    float lr[5];
};
// The updates (and launch_step_bump) do nothing when *flags (the step's
// kFlags word; nullable = always update) is non-zero: a step whose binning
// overflowed or read a non-finite parameter leaves parameters, poses, moments
// and the step counter as they were.
// groups: bit i updates group i (the moments keep the layout of all five)
hipError_t launch_adam(const AdamGroups& ag, float* m, float* v, int32_t* step, float b1, float b2, float eps,
                       const uint32_t* flags, hipStream_t s, unsigned groups = 0x1fu);
hipError_t launch_pose_update(int V, float* poses, const float* dpose, float* m, float* v, int32_t* step, float lr,
                              float b1, float b2, float eps, const uint32_t* flags, hipStream_t s);

}  // namespace gs
