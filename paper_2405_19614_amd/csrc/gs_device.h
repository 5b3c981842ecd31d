// Device-side math of the forward model and its derivatives (FP32).
//
// Projection (Sec. 3.4 "Projection"): camera transform, pinhole mean, local
// affine (EWA) footprint J Sigma_c J^T + 0.3 I, conic, opacity-aware support.
// Compositing weight of one fragment (Sec. 3.4 colour / depth equations).
#pragma once

#include "gs_internal.h"

namespace gs {

// rotation of a unit quaternion (w, x, y, z), row-major
__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float* R) {
    const float xx = x * x, yy = y * y, zz = z * z;
    const float xy = x * y, xz = x * z, yz = y * z, wx = w * x, wy = w * y, wz = w * z;
    R[0] = 1.f - 2.f * (yy + zz); R[1] = 2.f * (xy - wz);       R[2] = 2.f * (xz + wy);
    R[3] = 2.f * (xy + wz);       R[4] = 1.f - 2.f * (xx + zz); R[5] = 2.f * (yz - wx);
    R[6] = 2.f * (xz - wy);       R[7] = 2.f * (yz + wx);       R[8] = 1.f - 2.f * (xx + yy);
}

// Real orthonormal SH basis up to degree 3 at unit direction d, index
// l*l + l + m; optionally the gradient of each polynomial w.r.t. (x, y, z).
template <bool GRAD>
__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float* Y, float (*dY)[3]) {
    constexpr float PI = 3.14159265358979323846f;
    const float c0 = 0.28209479177387814f;            // 1/(2 sqrt(pi))
    const float c1 = 0.48860251190291992f;            // sqrt(3/(4 pi))
    const float c2a = 1.0925484305920792f;            // sqrt(15/pi)/2
    const float c2b = 0.31539156525252005f;           // sqrt(5/pi)/4
    const float c2c = 0.54627421529603959f;           // sqrt(15/pi)/4
    const float c3a = 0.59004358992664352f;           // sqrt(35/(2 pi))/4
    const float c3b = 2.8906114426405538f;            // sqrt(105/pi)/2
    const float c3c = 0.45704579946446572f;           // sqrt(21/(2 pi))/4
    const float c3d = 0.37317633259011546f;           // sqrt(7/pi)/4
    const float c3e = 1.4453057213202769f;            // sqrt(105/pi)/4
    (void)PI;
    Y[0] = c0;
    if (GRAD) { dY[0][0] = dY[0][1] = dY[0][2] = 0.f; }
    if (deg < 1) return;
    Y[1] = -c1 * y; Y[2] = c1 * z; Y[3] = -c1 * x;
    if (GRAD) {
        dY[1][0] = 0.f; dY[1][1] = -c1; dY[1][2] = 0.f;
        dY[2][0] = 0.f; dY[2][1] = 0.f; dY[2][2] = c1;
        dY[3][0] = -c1; dY[3][1] = 0.f; dY[3][2] = 0.f;
    }
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c2b * (2.f * zz - xx - yy);
    Y[7] = -c2a * x * z;
    Y[8] = c2c * (xx - yy);
    if (GRAD) {
        dY[4][0] = c2a * y;         dY[4][1] = c2a * x;         dY[4][2] = 0.f;
        dY[5][0] = 0.f;             dY[5][1] = -c2a * z;        dY[5][2] = -c2a * y;
        dY[6][0] = -2.f * c2b * x;  dY[6][1] = -2.f * c2b * y;  dY[6][2] = 4.f * c2b * z;
        dY[7][0] = -c2a * z;        dY[7][1] = 0.f;             dY[7][2] = -c2a * x;
        dY[8][0] = 2.f * c2c * x;   dY[8][1] = -2.f * c2c * y;  dY[8][2] = 0.f;
    }
    if (deg < 3) return;
    Y[9] = -c3a * y * (3.f * xx - yy);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (4.f * zz - xx - yy);
    Y[12] = c3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = -c3c * x * (4.f * zz - xx - yy);
    Y[14] = c3e * z * (xx - yy);
    Y[15] = -c3a * x * (xx - 3.f * yy);
    if (GRAD) {
        dY[9][0] = -6.f * c3a * x * y;  dY[9][1] = -3.f * c3a * (xx - yy);  dY[9][2] = 0.f;
        dY[10][0] = c3b * y * z;        dY[10][1] = c3b * x * z;            dY[10][2] = c3b * x * y;
        dY[11][0] = 2.f * c3c * x * y;  dY[11][1] = -c3c * (4.f * zz - xx - 3.f * yy);
        dY[11][2] = -8.f * c3c * y * z;
        dY[12][0] = -6.f * c3d * x * z; dY[12][1] = -6.f * c3d * y * z;
        dY[12][2] = c3d * (6.f * zz - 3.f * xx - 3.f * yy);
        dY[13][0] = -c3c * (4.f * zz - 3.f * xx - yy); dY[13][1] = 2.f * c3c * x * y;
        dY[13][2] = -8.f * c3c * x * z;
        dY[14][0] = 2.f * c3e * x * z;  dY[14][1] = -2.f * c3e * y * z;     dY[14][2] = c3e * (xx - yy);
        dY[15][0] = -3.f * c3a * (xx - yy); dY[15][1] = 6.f * c3a * x * y;  dY[15][2] = 0.f;
    }
}

// sum_l s[l] grad Y_l(x, y, z) for the basis of sh_basis (the gradient of each
// polynomial with respect to (x, y, z) as free variables), without storing
// the per-function gradients.
template <int DEG>
__device__ __forceinline__ void sh_grad_dot(float x, float y, float z, const float* s, float* g) {
    const float c1 = 0.48860251190291992f;
    const float c2a = 1.0925484305920792f;
    const float c2b = 0.31539156525252005f;
    const float c2c = 0.54627421529603959f;
    const float c3a = 0.59004358992664352f;
    const float c3b = 2.8906114426405538f;
    const float c3c = 0.45704579946446572f;
    const float c3d = 0.37317633259011546f;
    const float c3e = 1.4453057213202769f;
    float gx = 0.f, gy = 0.f, gz = 0.f;
    if (DEG >= 1) {
        gy -= c1 * s[1];
        gz += c1 * s[2];
        gx -= c1 * s[3];
    }
    if (DEG >= 2) {
        gx += c2a * y * s[4];                gy += c2a * x * s[4];
        gy -= c2a * z * s[5];                gz -= c2a * y * s[5];
        gx -= 2.f * c2b * x * s[6];          gy -= 2.f * c2b * y * s[6];   gz += 4.f * c2b * z * s[6];
        gx -= c2a * z * s[7];                gz -= c2a * x * s[7];
        gx += 2.f * c2c * x * s[8];          gy -= 2.f * c2c * y * s[8];
    }
    if (DEG >= 3) {
        const float xx = x * x, yy = y * y, zz = z * z;
        gx += -6.f * c3a * x * y * s[9];     gy += -3.f * c3a * (xx - yy) * s[9];
        gx += c3b * y * z * s[10];           gy += c3b * x * z * s[10];    gz += c3b * x * y * s[10];
        gx += 2.f * c3c * x * y * s[11];     gy += -c3c * (4.f * zz - xx - 3.f * yy) * s[11];
        gz += -8.f * c3c * y * z * s[11];
        gx += -6.f * c3d * x * z * s[12];    gy += -6.f * c3d * y * z * s[12];
        gz += c3d * (6.f * zz - 3.f * xx - 3.f * yy) * s[12];
        gx += -c3c * (4.f * zz - 3.f * xx - yy) * s[13];                   gy += 2.f * c3c * x * y * s[13];
        gz += -8.f * c3c * x * z * s[13];
        gx += 2.f * c3e * x * z * s[14];     gy += -2.f * c3e * y * z * s[14];   gz += c3e * (xx - yy) * s[14];
        gx += -3.f * c3a * (xx - yy) * s[15];                              gy += 6.f * c3a * x * y * s[15];
    }
    g[0] = gx; g[1] = gy; g[2] = gz;
}

// Coefficient k = 3 l + channel of one Gaussian's SH colour, read from its
// parameter array (CoefPtr), from a copy strided S floats apart (CoefStrided,
// the colour backward's LDS copy: lane t's coefficient k at t + S k), or from
// registers loaded up front (CoefRegs: all N coefficients in flight at once,
// in 16-byte loads when N is a multiple of four, where the row starts 16-byte
// aligned).
struct CoefPtr {
    const float* p;
    __device__ __forceinline__ float operator[](int k) const { return p[k]; }
};
template <int S>
struct CoefStrided {
    const float* p;
    __device__ __forceinline__ float operator[](int k) const { return p[k * S]; }
};
template <int N>
struct CoefRegs {
    float c[N];
    __device__ __forceinline__ explicit CoefRegs(const float* p) {
        if (N % 4 == 0) {
#pragma unroll
            for (int q = 0; q < N / 4; q++) {
                const float4 t = reinterpret_cast<const float4*>(p)[q];
                c[4 * q] = t.x; c[4 * q + 1] = t.y; c[4 * q + 2] = t.z; c[4 * q + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < N; k++) c[k] = p[k];
        }
    }
    __device__ __forceinline__ float operator[](int k) const { return c[k]; }
};

// View-dependent colour (SH of degree deg >= 0, coefficients sh) of a
// Gaussian with mean (mx, my, mz) seen from the camera of world-to-camera pose
// T: dir = unit vector from the camera centre C = -R^T t to the mean, colour =
// max(0, sum Y_lm(dir) k_lm + 0.5) per channel.  The projection, its deferred
// colour pass and the backward all evaluate the colour through this one
// function on the same coefficient values, so they agree bit for bit (the
// clamp decisions included).
template <class Coef>
__device__ __forceinline__ void sh_colour_of(int deg, const Coef& sh, float mx, float my, float mz, const float* T,
                                             float* dir, float& dirn, float* col, bool* cclamp, bool& colbad) {
    // camera centre C = -R_cw^T t_cw
    const float Cx = -(T[0] * T[3] + T[4] * T[7] + T[8] * T[11]);
    const float Cy = -(T[1] * T[3] + T[5] * T[7] + T[9] * T[11]);
    const float Cz = -(T[2] * T[3] + T[6] * T[7] + T[10] * T[11]);
    const float dx = mx - Cx, dy = my - Cy, dz = mz - Cz;
    dirn = sqrtf(dx * dx + dy * dy + dz * dz);
    const float idn = 1.f / dirn;
    dir[0] = dx * idn; dir[1] = dy * idn; dir[2] = dz * idn;
    float Y[16];
    sh_basis<false>(deg, dir[0], dir[1], dir[2], Y, nullptr);
    const int K = (deg + 1) * (deg + 1);
    float acc[3] = {0.5f, 0.5f, 0.5f};
    for (int l = 0; l < K; l++) {
        acc[0] += Y[l] * sh[3 * l];
        acc[1] += Y[l] * sh[3 * l + 1];
        acc[2] += Y[l] * sh[3 * l + 2];
    }
#pragma unroll
    for (int k = 0; k < 3; k++) {
        cclamp[k] = acc[k] < 0.f;
        col[k] = fmaxf(acc[k], 0.f);
    }
    colbad = !__builtin_isfinite(acc[0] + acc[1] + acc[2]);
}

// sh_colour_of for Gaussian g of P (degree P.sh), coefficients from P.col
__device__ __forceinline__ void sh_colour(const Params& P, int g, float mx, float my, float mz, const float* T,
                                          float* dir, float& dirn, float* col, bool* cclamp, bool& colbad) {
    const int K = (P.sh + 1) * (P.sh + 1);
    sh_colour_of(P.sh, CoefPtr{P.col + (int64_t)g * K * 3}, mx, my, mz, T, dir, dirn, col, cclamp, colbad);
}

// Everything the projection of one Gaussian into one view computes; the
// backward recomputes it instead of storing it.
struct Proj {
    bool valid;
    float qn;           // |q|
    float qh[4];        // unit quaternion
    float R[9];         // Gaussian rotation
    float s[3];         // scales
    float Sc[6];        // camera covariance (xx, xy, xz, yy, yz, zz)
    float p[3];         // camera-space mean
    bool clx, cly;      // Jacobian clamp active
    float tx, ty;       // clamped x, y used in J
    float j00, j02, j11, j12;
    float a, b, c, det; // dilated 2D covariance
    float u, v;
    float A, B, C;      // conic
    float o;
    float col[3];
    bool cclamp[3];     // SH colour clamped at 0
    bool colbad;        // the colour (RGB, or the SH sum before its clamp) is not finite
    float dir[3], dirn; // unit view direction, |mu - camera centre|
    float radius;
    int x0, x1, y0, y1;
};

// View-independent part of a Gaussian's projection: activations and the
// world covariance M = R diag(s^2) R^T (isotropic: r^2 I, no rotation).
struct GPrep {
    bool ok;
    bool finite;        // mean, log-scales (radius), quaternion and opacity logit all finite
    float qn, qh[4], R[9], s[3], o;
    float mu[3];
    float M[6];
};

template <bool ISO>
__device__ __forceinline__ void gauss_prep(const Params& P, int g, GPrep& gp) {
    gp.ok = false;
    if (ISO) {
        // the paper's Gaussian: one radius r = exp(log r), covariance r^2 I
        const float l = P.ls[g];
        const float* mp = P.means + 3 * (int64_t)g;
        gp.finite = __builtin_isfinite((mp[0] + mp[1] + mp[2]) + l + P.opl[g]);
        gp.ok = true;
        const float r = expf(l);
        gp.s[0] = gp.s[1] = gp.s[2] = r;
        gp.o = 1.f / (1.f + expf(-P.opl[g]));
        gp.mu[0] = mp[0]; gp.mu[1] = mp[1]; gp.mu[2] = mp[2];
        const float r2 = r * r;
        gp.M[0] = r2; gp.M[1] = 0.f; gp.M[2] = 0.f; gp.M[3] = r2; gp.M[4] = 0.f; gp.M[5] = r2;
        return;
    }
    const float4 q = reinterpret_cast<const float4*>(P.q)[g];
    {
        const float* lp = P.ls + 3 * (int64_t)g;
        const float* mp = P.means + 3 * (int64_t)g;
        // one non-finite value makes the sum non-finite (finite values of this
        // size do not overflow the sum)
        const float sum = (q.x + q.y + q.z + q.w) + (lp[0] + lp[1] + lp[2]) + (mp[0] + mp[1] + mp[2]) + P.opl[g];
        gp.finite = __builtin_isfinite(sum);
    }
    const float qn2 = q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w;
    if (!(qn2 > 0.f)) return;
    gp.ok = true;
    gp.qn = sqrtf(qn2);
    const float iq = 1.f / gp.qn;
    gp.qh[0] = q.x * iq; gp.qh[1] = q.y * iq; gp.qh[2] = q.z * iq; gp.qh[3] = q.w * iq;
    quat_rot(gp.qh[0], gp.qh[1], gp.qh[2], gp.qh[3], gp.R);
    const float* lsp = P.ls + 3 * (int64_t)g;
    gp.s[0] = expf(lsp[0]); gp.s[1] = expf(lsp[1]); gp.s[2] = expf(lsp[2]);
    gp.o = 1.f / (1.f + expf(-P.opl[g]));
    const float* mu = P.means + 3 * (int64_t)g;
    gp.mu[0] = mu[0]; gp.mu[1] = mu[1]; gp.mu[2] = mu[2];
    const float s0 = gp.s[0] * gp.s[0], s1 = gp.s[1] * gp.s[1], s2 = gp.s[2] * gp.s[2];
    const float* R = gp.R;
    gp.M[0] = R[0] * R[0] * s0 + R[1] * R[1] * s1 + R[2] * R[2] * s2;
    gp.M[1] = R[0] * R[3] * s0 + R[1] * R[4] * s1 + R[2] * R[5] * s2;
    gp.M[2] = R[0] * R[6] * s0 + R[1] * R[7] * s1 + R[2] * R[8] * s2;
    gp.M[3] = R[3] * R[3] * s0 + R[4] * R[4] * s1 + R[5] * R[5] * s2;
    gp.M[4] = R[3] * R[6] * s0 + R[4] * R[7] * s1 + R[5] * R[8] * s2;
    gp.M[5] = R[6] * R[6] * s0 + R[7] * R[7] * s1 + R[8] * R[8] * s2;
}

// Project a prepared Gaussian g into view vi with pose T (row-major 4x4,
// world->camera).  COL: also evaluate the colour (RGB or SH).  ISO: the
// camera covariance of r^2 I is r^2 I (a rigid motion keeps it), so the 2D
// covariance is r^2 J J^T + 0.3 I; on the optical axis r2D = f r / d.
template <bool COL, bool ISO>
__device__ __forceinline__ void project_view(const Params& P, int g, const GPrep& gp, const ViewInfo& vi,
                                             const float* T, Proj& o) {
    o.valid = false;
    if (!gp.ok) return;
    if (!ISO) {
        o.qn = gp.qn;
#pragma unroll
        for (int k = 0; k < 4; k++) o.qh[k] = gp.qh[k];
#pragma unroll
        for (int k = 0; k < 9; k++) o.R[k] = gp.R[k];
    }
    o.s[0] = gp.s[0]; o.s[1] = gp.s[1]; o.s[2] = gp.s[2];
    o.o = gp.o;

    const float mx = gp.mu[0], my = gp.mu[1], mz = gp.mu[2];
    o.p[0] = T[0] * mx + T[1] * my + T[2] * mz + T[3];
    o.p[1] = T[4] * mx + T[5] * my + T[6] * mz + T[7];
    o.p[2] = T[8] * mx + T[9] * my + T[10] * mz + T[11];
    const float pz = o.p[2];
    if (!(pz > kZNear)) return;
    const float iz = 1.f / pz;
    o.u = vi.fx * o.p[0] * iz + vi.cx;
    o.v = vi.fy * o.p[1] * iz + vi.cy;

    // EWA Jacobian with x/z, y/z clamped at 1.3x the half field of view
    const float limx = kJClamp * (float)vi.W / (2.f * vi.fx);
    const float limy = kJClamp * (float)vi.H / (2.f * vi.fy);
    const float xz = o.p[0] * iz, yz = o.p[1] * iz;
    o.clx = (xz < -limx) || (xz > limx);
    o.cly = (yz < -limy) || (yz > limy);
    o.tx = fminf(fmaxf(xz, -limx), limx) * pz;
    o.ty = fminf(fmaxf(yz, -limy), limy) * pz;
    o.j00 = vi.fx * iz;
    o.j11 = vi.fy * iz;
    o.j02 = -vi.fx * o.tx * iz * iz;
    o.j12 = -vi.fy * o.ty * iz * iz;

    // Sigma_c = W M W^T with the world covariance M of gauss_prep
    const float* M = gp.M;
    if (ISO) {
        o.Sc[0] = M[0]; o.Sc[1] = 0.f; o.Sc[2] = 0.f; o.Sc[3] = M[0]; o.Sc[4] = 0.f; o.Sc[5] = M[0];
        const float r2 = M[0];
        o.a = r2 * (o.j00 * o.j00 + o.j02 * o.j02) + kDilate;
        o.b = r2 * (o.j02 * o.j12);
        o.c = r2 * (o.j11 * o.j11 + o.j12 * o.j12) + kDilate;
    } else {
        // WM = W * M (full 3x3), Sc = WM * W^T (symmetric)
        float Mf[9] = {M[0], M[1], M[2], M[1], M[3], M[4], M[2], M[4], M[5]};
        float WM[9];
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
            for (int c = 0; c < 3; c++)
                WM[3 * r + c] = T[4 * r] * Mf[c] + T[4 * r + 1] * Mf[3 + c] + T[4 * r + 2] * Mf[6 + c];
        o.Sc[0] = WM[0] * T[0] + WM[1] * T[1] + WM[2] * T[2];
        o.Sc[1] = WM[0] * T[4] + WM[1] * T[5] + WM[2] * T[6];
        o.Sc[2] = WM[0] * T[8] + WM[1] * T[9] + WM[2] * T[10];
        o.Sc[3] = WM[3] * T[4] + WM[4] * T[5] + WM[5] * T[6];
        o.Sc[4] = WM[3] * T[8] + WM[4] * T[9] + WM[5] * T[10];
        o.Sc[5] = WM[6] * T[8] + WM[7] * T[9] + WM[8] * T[10];
    }
    // Sigma_2D = J Sc J^T with J = [[j00, 0, j02], [0, j11, j12]]
    if (!ISO) {
        const float* S = o.Sc;
        const float r00 = o.j00 * S[0] + o.j02 * S[2], r01 = o.j00 * S[1] + o.j02 * S[4],
                    r02 = o.j00 * S[2] + o.j02 * S[5];
        const float r11 = o.j11 * S[3] + o.j12 * S[4], r12 = o.j11 * S[4] + o.j12 * S[5];
        o.a = r00 * o.j00 + r02 * o.j02 + kDilate;
        o.b = r01 * o.j11 + r02 * o.j12;
        o.c = r11 * o.j11 + r12 * o.j12 + kDilate;
    }
    o.det = o.a * o.c - o.b * o.b;
    if (!(o.det > 0.f)) return;
    const float idet = 1.f / o.det;
    o.A = o.c * idet;
    o.B = -o.b * idet;
    o.C = o.a * idet;

    if (COL) {
        if (P.sh < 0) {
            const float* cp = P.col + 3 * (int64_t)g;
            o.col[0] = cp[0]; o.col[1] = cp[1]; o.col[2] = cp[2];
            o.cclamp[0] = o.cclamp[1] = o.cclamp[2] = false;
            o.colbad = !__builtin_isfinite(cp[0] + cp[1] + cp[2]);
        } else {
            sh_colour(P, g, mx, my, mz, T, o.dir, o.dirn, o.col, o.cclamp, o.colbad);
        }
    }

    // opacity-aware support radius: alpha >= 1/255 only where
    // |d|^2 <= 2 ln(255 o) lambda_max
    if (o.o < kAlphaMin) return;
    const float qmax = 2.f * logf(255.f * o.o);
    const float m = 0.5f * (o.a + o.c);
    const float lmax = m + sqrtf(fmaxf(m * m - o.det, 0.f));
    o.radius = ceilf(sqrtf(qmax * lmax));
    // The pixel rect is the bounding box of that ellipse, which is tighter
    // than the square of the radius unless the ellipse is round or
    // axis-aligned: for a fixed dx the smallest sigma over dy is
    // dx^2 / (2 Sigma_xx), so alpha >= 1/255 needs |dx| <= sqrt(qmax Sigma_xx)
    // (and |dy| <= sqrt(qmax Sigma_yy)).  The widened qmax and the extra
    // hundredth of a pixel keep the box conservative under FP32 rounding: a
    // pixel outside it has an exact alpha at least 2.5 % below 1/255.  The
    // cap by the radius is taken at the widened qmax too, so the bound holds
    // where the cap binds; the compositing kernels rely on it (they test no
    // rect per pixel and let the alpha test reject pixels outside it).
    const float qbox = qmax + 0.05f;
    const float rbox = ceilf(sqrtf(qbox * lmax));
    const float hx = fminf(rbox, sqrtf(qbox * o.a) + 0.01f);
    const float hy = fminf(rbox, sqrtf(qbox * o.c) + 0.01f);
    const float fx0 = fmaxf(ceilf(o.u - hx), 0.f);
    const float fx1 = fminf(floorf(o.u + hx), (float)(vi.W - 1));
    const float fy0 = fmaxf(ceilf(o.v - hy), 0.f);
    const float fy1 = fminf(floorf(o.v + hy), (float)(vi.H - 1));
    if (!(fx0 <= fx1) || !(fy0 <= fy1)) return;
    o.x0 = (int)fx0; o.x1 = (int)fx1; o.y0 = (int)fy0; o.y1 = (int)fy1;
    o.valid = true;
}

// Conservative visibility test of a prepared Gaussian in view vi: false only
// when project_view would find no pixel rect.  It takes project_view's
// camera-space mean and, up to the hardware reciprocal's and square root's
// rounding (a few ulps: below 1e-3 px at any image coordinate, far inside the
// margins below), its projected mean, and bounds the rect's half-widths from
// above.  limx, limy are project_view's Jacobian clamp limits of the view
// (the caller computes them once per view, with the same expression).  With W the pose's linear part, the 2D covariance's diagonal entry
// a = w^T M w + 0.3 for w = j00 W_0 + j02 W_2 (rows of W), and
// w^T M w <= s_max^2 |w|^2 with s_max^2 the world covariance's largest
// eigenvalue (the largest scale squared); likewise c with
// w = j11 W_1 + j12 W_2.  This holds for any linear W, rigid or not.  Against
// rounding, a and c are widened by 1 % plus 0.01 px^2, the half-width
// sqrt(qbox a) + 0.01 by 0.1 % plus 0.01 px, the near plane by 0.1 % and the
// image bounds by one pixel.  qbox = 2 ln(255 o) + 0.05, as project_view's;
// it is negative (no visibility) for o < 1/255.
__device__ __forceinline__ bool may_be_visible(const float* mu, float smax2, float qbox, const ViewInfo& vi,
                                               const float* T, float limx, float limy) {
    const float mx = mu[0], my = mu[1], mz = mu[2];
    const float p0 = T[0] * mx + T[1] * my + T[2] * mz + T[3];
    const float p1 = T[4] * mx + T[5] * my + T[6] * mz + T[7];
    const float pz = T[8] * mx + T[9] * my + T[10] * mz + T[11];
    if (!(pz > 0.999f * kZNear) || !(qbox > 0.f)) return false;
    const float iz = __builtin_amdgcn_rcpf(pz);
    const float u = vi.fx * p0 * iz + vi.cx;
    const float v = vi.fy * p1 * iz + vi.cy;
    const float tx = fminf(fmaxf(p0 * iz, -limx), limx) * pz;
    const float ty = fminf(fmaxf(p1 * iz, -limy), limy) * pz;
    const float j00 = vi.fx * iz, j11 = vi.fy * iz;
    const float j02 = -vi.fx * tx * iz * iz, j12 = -vi.fy * ty * iz * iz;
    const float wx0 = j00 * T[0] + j02 * T[8], wx1 = j00 * T[1] + j02 * T[9], wx2 = j00 * T[2] + j02 * T[10];
    const float wy0 = j11 * T[4] + j12 * T[8], wy1 = j11 * T[5] + j12 * T[9], wy2 = j11 * T[6] + j12 * T[10];
    const float a = 1.01f * (wx0 * wx0 + wx1 * wx1 + wx2 * wx2) * smax2 + (kDilate + 0.01f);
    const float c = 1.01f * (wy0 * wy0 + wy1 * wy1 + wy2 * wy2) * smax2 + (kDilate + 0.01f);
    const float hx = 1.001f * __builtin_amdgcn_sqrtf(qbox * a) + 0.02f;
    const float hy = 1.001f * __builtin_amdgcn_sqrtf(qbox * c) + 0.02f;
    return (u + hx >= -1.f) && (u - hx <= (float)vi.W) && (v + hy >= -1.f) && (v - hy <= (float)vi.H);
}

// Records keep the conic in base-2 units with the opacity folded in:
// co = (A', B', C', log2 o) with A' = c A, B' = 2 c B, C' = c C and
// c = log2(e) / 2, so o exp(-sigma) = exp2(log2 o - (A' dx^2 + B' dx dy +
// C' dy^2)).  For a thread's fixed pixel column the exponent is a quadratic
// in dy, t(dy) = (C' dy + a1) dy + a0, evaluated with two FMAs per pixel.
constexpr float kHalfLog2e = 0.72134752044448170368f;   // log2(e) / 2

struct FragCol {
    float dx, a0, a1;
};

// Per-column part of the exponent.  No contraction, and the per-pixel part
// uses explicit FMAs, so forward and backward take the same skip and clamp
// decisions bit for bit whatever code surrounds the inlined copies.
__device__ __forceinline__ FragCol frag_col(float px, float2 xy, float4 co) {
#pragma clang fp contract(off)
    FragCol f;
    f.dx = px - xy.x;
    f.a0 = co.x * f.dx * f.dx - co.w;
    f.a1 = co.y * f.dx;
    return f;
}

// o exp(-sigma) at pixel row py (dy = py - v)
__device__ __forceinline__ float frag_raw(const FragCol& f, float4 co, float dy) {
    const float t = fmaf(fmaf(co.z, dy, f.a1), dy, f.a0);
    return __builtin_amdgcn_exp2f(-t);
}

__device__ __forceinline__ bool rect_has(uint2 r, int x, int y) {
    const int x0 = (int)(r.x & 0xffffu), x1 = (int)(r.x >> 16);
    const int y0 = (int)(r.y & 0xffffu), y1 = (int)(r.y >> 16);
    return x >= x0 && x <= x1 && y >= y0 && y <= y1;
}

// view of a global tile id (V is small; scalar binary search over tile_off)
__device__ __forceinline__ int view_of_tile(const ViewTable& vt, int t) {
    int lo = 0, hi = vt.V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (vt.v[mid].tile_off <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace gs
