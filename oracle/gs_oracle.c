/*
 * gs_oracle.c -- plain FP64 CPU definition of the Gaussian-splatting forward
 * model and its reverse mode.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the HIP path.
 *
 * What it follows (TAMBRIDGE, arXiv 2405.19614):
 *   - Sec. 3.4 "Gaussian Representation" (Eq. gauss): a Gaussian has a
 *     colour, a centre, a footprint and an opacity.  Generalised here to an
 *     anisotropic covariance R diag(s^2) R^T from log-scales and a quaternion;
 *     equal log-scales give the paper's isotropic model.
 *   - Sec. 3.4 "Projection" (projection equation): mean projected by K E_t mu / d,
 *     footprint by a local affine (EWA) transform, whose on-axis isotropic limit
 *     is r2D = f r / d.
 *   - Sec. 3.4 colour and depth compositing equations and Sec. 3.3 border-mask
 *     equation: front-to-back alpha blending of C, D and M_b = 1 - T_final.
 *   - Sec. 3.2 Eq. lba: re-projection residual u - pi(C_j, P_i), robustified
 *     by a Huber kernel on its Euclidean norm.
 *   - Sec. 3.3 joint-loss equation and Sec. 3.4 mapping-loss equation: the
 *     weighted L1 terms (the weighting is done by the Python wrapper).
 *
 * Readings of points the paper leaves open (alpha clamp 0.99, skip below
 * 1/255, stop when T would fall below 1e-4, +0.3 px^2 dilation, near plane
 * 0.2, Jacobian clamp 1.3x the half field of view, opacity-aware support
 * radius, integer pixel-centre convention, ascending-index tie break) are
 * stated beside the code that uses them.
 *
 * Everything is double precision; inputs are FP32 values promoted by the
 * caller.  Per-pixel fragment lists are stored in the backward pass (no
 * transmittance recovery by division).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ZNEAR 0.2            /* cull if camera-space z <= 0.2 */
#define ALPHA_MAX 0.99       /* alpha clamp */
#define ALPHA_MIN (1.0 / 255.0) /* skip if alpha < 1/255 */
#define T_MIN 1e-4           /* stop before T would fall below 1e-4 */
#define DILATE 0.3           /* low-pass dilation added to the 2D covariance diagonal, px^2 */
#define JCLAMP 1.3           /* Jacobian clamp, in units of the half field of view */
#define BUCKET 8             /* the oracle's own coarse pixel buckets */

typedef struct {
    int W, H;
    double fx, fy, cx, cy;
    double Rw[9]; /* world->camera rotation, row-major */
    double tw[3]; /* world->camera translation */
} cam_t;

typedef struct {
    int64_t n;
    int sh_degree; /* -1 = direct RGB */
    const double *means, *log_scales, *quats, *opl, *colors;
} gs_t;

/* one projected Gaussian (one view) with every intermediate the reverse mode needs */
typedef struct {
    int valid;
    double qn;         /* |q| */
    double qh[4];      /* unit quaternion (w,x,y,z) */
    double R[9];       /* rotation of the Gaussian */
    double s[3];       /* scales */
    double Sig[9];     /* world covariance */
    double Sc[9];      /* camera covariance */
    double p[3];       /* camera-space mean */
    int clx, cly;      /* Jacobian clamp active */
    double cxv, cyv;   /* clamped x/z, y/z */
    double J[6];       /* 2x3 Jacobian, row-major */
    double a, b, c;    /* dilated 2D covariance [[a b][b c]] */
    double det;
    double u, v;       /* projected mean, px */
    double A, B, C;    /* conic = inverse 2D covariance [[A B][B C]] */
    double o;          /* opacity */
    double col[3];
    int colclamp[3];   /* SH colour clamped at 0 */
    double dir[3];     /* unit view direction (SH) */
    double dirn;       /* |mu - camera centre| */
    double Y[16];      /* SH basis at dir */
    double z;
    double zsc;        /* sum of |terms| of the depth dot product (its rounding scale) */
    double radius;
    int x0, x1, y0, y1;
} proj_t;

static void make_cam(cam_t* c, int W, int H, double fx, double fy, double cx, double cy,
                     const double* T) {
    c->W = W; c->H = H; c->fx = fx; c->fy = fy; c->cx = cx; c->cy = cy;
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) c->Rw[3 * i + j] = T[4 * i + j];
        c->tw[i] = T[4 * i + 3];
    }
}

/* ---------------- small dense linear algebra ---------------- */
static void mat3_mul(const double* A, const double* B, double* C) {
    double t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += A[3 * i + k] * B[3 * k + j];
            t[3 * i + j] = s;
        }
    memcpy(C, t, sizeof t);
}
static void mat3_mul_bt(const double* A, const double* B, double* C) { /* A B^T */
    double t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += A[3 * i + k] * B[3 * j + k];
            t[3 * i + j] = s;
        }
    memcpy(C, t, sizeof t);
}
static void mat3_mul_at(const double* A, const double* B, double* C) { /* A^T B */
    double t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += A[3 * k + i] * B[3 * k + j];
            t[3 * i + j] = s;
        }
    memcpy(C, t, sizeof t);
}

/* rotation matrix of a unit quaternion (w, x, y, z) */
static void quat_rot(const double* q, double* R) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* ---------------- real orthonormal spherical harmonics, degree <= 3 ----------------
 * Y_lm of a unit direction (x, y, z), written as the standard real polynomials with
 * normalisation sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (times sqrt 2 for m != 0), signed
 * so that index l*l + l + m runs m = -l..l.  The gradient is of the polynomial in
 * (x, y, z) taken as free variables; the caller projects it onto the sphere. */
static void sh_eval(int deg, const double* d, double* Y, double (*dY)[3]) {
    const double x = d[0], y = d[1], z = d[2];
    const double k0 = 0.5 * sqrt(1.0 / M_PI);
    const double k1 = sqrt(3.0 / (4.0 * M_PI));
    const double k2a = 0.5 * sqrt(15.0 / M_PI);
    const double k2b = 0.25 * sqrt(5.0 / M_PI);
    const double k2c = 0.25 * sqrt(15.0 / M_PI);
    const double k3a = 0.25 * sqrt(35.0 / (2.0 * M_PI));
    const double k3b = 0.5 * sqrt(105.0 / M_PI);
    const double k3c = 0.25 * sqrt(21.0 / (2.0 * M_PI));
    const double k3d = 0.25 * sqrt(7.0 / M_PI);
    const double k3e = 0.25 * sqrt(105.0 / M_PI);
    double g[16][3];
    memset(g, 0, sizeof g);
    Y[0] = k0;
    if (deg >= 1) {
        Y[1] = -k1 * y; g[1][1] = -k1;
        Y[2] = k1 * z;  g[2][2] = k1;
        Y[3] = -k1 * x; g[3][0] = -k1;
    }
    if (deg >= 2) {
        Y[4] = k2a * x * y;                 g[4][0] = k2a * y; g[4][1] = k2a * x;
        Y[5] = -k2a * y * z;                g[5][1] = -k2a * z; g[5][2] = -k2a * y;
        Y[6] = k2b * (2 * z * z - x * x - y * y);
        g[6][0] = -2 * k2b * x; g[6][1] = -2 * k2b * y; g[6][2] = 4 * k2b * z;
        Y[7] = -k2a * x * z;                g[7][0] = -k2a * z; g[7][2] = -k2a * x;
        Y[8] = k2c * (x * x - y * y);       g[8][0] = 2 * k2c * x; g[8][1] = -2 * k2c * y;
    }
    if (deg >= 3) {
        Y[9] = -k3a * y * (3 * x * x - y * y);
        g[9][0] = -k3a * 6 * x * y; g[9][1] = -k3a * (3 * x * x - 3 * y * y);
        Y[10] = k3b * x * y * z;
        g[10][0] = k3b * y * z; g[10][1] = k3b * x * z; g[10][2] = k3b * x * y;
        Y[11] = -k3c * y * (4 * z * z - x * x - y * y);
        g[11][0] = -k3c * (-2 * x * y); g[11][1] = -k3c * (4 * z * z - x * x - 3 * y * y);
        g[11][2] = -k3c * 8 * y * z;
        Y[12] = k3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
        g[12][0] = k3d * (-6 * x * z); g[12][1] = k3d * (-6 * y * z);
        g[12][2] = k3d * (6 * z * z - 3 * x * x - 3 * y * y);
        Y[13] = -k3c * x * (4 * z * z - x * x - y * y);
        g[13][0] = -k3c * (4 * z * z - 3 * x * x - y * y); g[13][1] = -k3c * (-2 * x * y);
        g[13][2] = -k3c * 8 * x * z;
        Y[14] = k3e * z * (x * x - y * y);
        g[14][0] = k3e * 2 * x * z; g[14][1] = -k3e * 2 * y * z; g[14][2] = k3e * (x * x - y * y);
        Y[15] = -k3a * x * (x * x - 3 * y * y);
        g[15][0] = -k3a * (3 * x * x - 3 * y * y); g[15][1] = -k3a * (-6 * x * y);
    }
    if (dY) {
        int K = (deg + 1) * (deg + 1);
        for (int i = 0; i < K; i++)
            for (int j = 0; j < 3; j++) dY[i][j] = g[i][j];
    }
}

/* ---------------- forward projection of one Gaussian into one view ---------------- */
static void project(const gs_t* g, int64_t i, const cam_t* cam, proj_t* P) {
    memset(P, 0, sizeof *P);
    const double* q = g->quats + 4 * i;
    /* activations: scale = exp(log-scale), unit quaternion, opacity = sigmoid(logit) */
    P->qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(P->qn > 0)) return;
    for (int k = 0; k < 4; k++) P->qh[k] = q[k] / P->qn;
    quat_rot(P->qh, P->R);
    for (int k = 0; k < 3; k++) P->s[k] = exp(g->log_scales[3 * i + k]);
    double RS[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) RS[3 * r + c] = P->R[3 * r + c] * P->s[c] * P->s[c];
    mat3_mul_bt(RS, P->R, P->Sig); /* R diag(s^2) R^T */
    P->o = 1.0 / (1.0 + exp(-g->opl[i]));

    /* camera transform: p = R_cw mu + t_cw */
    const double* mu = g->means + 3 * i;
    for (int r = 0; r < 3; r++)
        P->p[r] = cam->Rw[3 * r] * mu[0] + cam->Rw[3 * r + 1] * mu[1] + cam->Rw[3 * r + 2] * mu[2] +
                  cam->tw[r];
    if (P->p[2] <= ZNEAR) return;
    const double px = P->p[0], py = P->p[1], pz = P->p[2];
    P->zsc = fabs(cam->Rw[6] * mu[0]) + fabs(cam->Rw[7] * mu[1]) + fabs(cam->Rw[8] * mu[2]) + fabs(cam->tw[2]);

    /* pinhole projection of the mean (integer pixel coordinates sample the
       point itself: OpenCV convention) */
    P->u = cam->fx * px / pz + cam->cx;
    P->v = cam->fy * py / pz + cam->cy;

    /* local affine (EWA) Jacobian, with x/z and y/z clamped at 1.3x the half
       field of view (the clamp only enters J, never the projected mean) */
    double limx = JCLAMP * cam->W / (2.0 * cam->fx);
    double limy = JCLAMP * cam->H / (2.0 * cam->fy);
    double xz = px / pz, yz = py / pz;
    P->clx = (xz < -limx || xz > limx);
    P->cly = (yz < -limy || yz > limy);
    P->cxv = xz < -limx ? -limx : (xz > limx ? limx : xz);
    P->cyv = yz < -limy ? -limy : (yz > limy ? limy : yz);
    double tx = P->cxv * pz, ty = P->cyv * pz;
    P->J[0] = cam->fx / pz; P->J[1] = 0; P->J[2] = -cam->fx * tx / (pz * pz);
    P->J[3] = 0; P->J[4] = cam->fy / pz; P->J[5] = -cam->fy * ty / (pz * pz);

    /* Sigma_c = R_cw Sigma R_cw^T ; Sigma_2D = J Sigma_c J^T ; dilation */
    double tmp[9];
    mat3_mul(cam->Rw, P->Sig, tmp);
    mat3_mul_bt(tmp, cam->Rw, P->Sc);
    double JS[6];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++)
            JS[3 * r + c] = P->J[3 * r] * P->Sc[c] + P->J[3 * r + 1] * P->Sc[3 + c] +
                            P->J[3 * r + 2] * P->Sc[6 + c];
    double s00 = JS[0] * P->J[0] + JS[1] * P->J[1] + JS[2] * P->J[2];
    double s01 = JS[0] * P->J[3] + JS[1] * P->J[4] + JS[2] * P->J[5];
    double s11 = JS[3] * P->J[3] + JS[4] * P->J[4] + JS[5] * P->J[5];
    P->a = s00 + DILATE;
    P->b = s01;
    P->c = s11 + DILATE;
    P->det = P->a * P->c - P->b * P->b;
    if (!(P->det > 0)) return;
    P->A = P->c / P->det;
    P->B = -P->b / P->det;
    P->C = P->a / P->det;

    /* colour: direct RGB, or SH evaluated along the unit direction from the
       camera centre to the mean, plus 0.5, clamped at 0 */
    if (g->sh_degree < 0) {
        for (int k = 0; k < 3; k++) P->col[k] = g->colors[3 * i + k];
    } else {
        double Cc[3];
        for (int r = 0; r < 3; r++)
            Cc[r] = -(cam->Rw[r] * cam->tw[0] + cam->Rw[3 + r] * cam->tw[1] + cam->Rw[6 + r] * cam->tw[2]);
        double d[3] = {mu[0] - Cc[0], mu[1] - Cc[1], mu[2] - Cc[2]};
        P->dirn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int k = 0; k < 3; k++) P->dir[k] = d[k] / P->dirn;
        sh_eval(g->sh_degree, P->dir, P->Y, NULL);
        int K = (g->sh_degree + 1) * (g->sh_degree + 1);
        const double* sh = g->colors + (int64_t)K * 3 * i;
        for (int k = 0; k < 3; k++) {
            double acc = 0;
            for (int l = 0; l < K; l++) acc += P->Y[l] * sh[3 * l + k];
            acc += 0.5;
            P->colclamp[k] = acc < 0;
            P->col[k] = acc < 0 ? 0 : acc;
        }
    }
    P->z = pz;

    /* opacity-aware support: alpha >= 1/255 needs o exp(-sigma) >= 1/255, i.e.
       sigma <= ln(255 o); with sigma >= |d|^2 / (2 lambda_max) this bounds
       |d| <= sqrt(2 ln(255 o) lambda_max).  Rounded up to whole pixels. */
    if (P->o < ALPHA_MIN) return;
    double qmax = 2.0 * log(255.0 * P->o);
    double m = 0.5 * (P->a + P->c);
    double disc = m * m - P->det;
    double lmax = m + sqrt(disc > 0 ? disc : 0);
    P->radius = ceil(sqrt(qmax * lmax));
    double fx0 = ceil(P->u - P->radius), fx1 = floor(P->u + P->radius);
    double fy0 = ceil(P->v - P->radius), fy1 = floor(P->v + P->radius);
    if (fx0 < 0) fx0 = 0;
    if (fy0 < 0) fy0 = 0;
    if (fx1 > cam->W - 1) fx1 = cam->W - 1;
    if (fy1 > cam->H - 1) fy1 = cam->H - 1;
    if (fx0 > fx1 || fy0 > fy1) return;
    P->x0 = (int)fx0; P->x1 = (int)fx1; P->y0 = (int)fy0; P->y1 = (int)fy1;
    P->valid = 1;
}

/* ---------------- per-view candidate lists ---------------- */
typedef struct {
    int64_t nvis;
    int64_t* order;      /* visible Gaussian ids in ascending (depth, id) order */
    int bx, by;          /* bucket grid */
    int64_t* bstart;     /* [bx*by+1] */
    int64_t* blist;      /* ids, each bucket in ascending (depth, id) order */
    proj_t* P;           /* [n] */
} view_t;

static const proj_t* g_sort_P;
static int cmp_depth_id(const void* x, const void* y) {
    int64_t i = *(const int64_t*)x, j = *(const int64_t*)y;
    double zi = g_sort_P[i].z, zj = g_sort_P[j].z;
    if (zi < zj) return -1;
    if (zi > zj) return 1;
    return (i < j) ? -1 : (i > j);
}

static int build_view(const gs_t* g, const cam_t* cam, view_t* V) {
    memset(V, 0, sizeof *V);
    V->P = (proj_t*)malloc(sizeof(proj_t) * (g->n > 0 ? g->n : 1));
    if (!V->P) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->n; i++) project(g, i, cam, &V->P[i]);
    int64_t nv = 0;
    for (int64_t i = 0; i < g->n; i++) nv += V->P[i].valid;
    V->nvis = nv;
    V->order = (int64_t*)malloc(sizeof(int64_t) * (nv > 0 ? nv : 1));
    nv = 0;
    for (int64_t i = 0; i < g->n; i++)
        if (V->P[i].valid) V->order[nv++] = i;
    g_sort_P = V->P; /* qsort has no context argument; build_view is not re-entrant */
    qsort(V->order, (size_t)nv, sizeof(int64_t), cmp_depth_id);
    V->bx = (cam->W + BUCKET - 1) / BUCKET;
    V->by = (cam->H + BUCKET - 1) / BUCKET;
    int64_t nb = (int64_t)V->bx * V->by;
    V->bstart = (int64_t*)calloc((size_t)nb + 1, sizeof(int64_t));
    for (int64_t k = 0; k < nv; k++) {
        const proj_t* p = &V->P[V->order[k]];
        for (int yb = p->y0 / BUCKET; yb <= p->y1 / BUCKET; yb++)
            for (int xb = p->x0 / BUCKET; xb <= p->x1 / BUCKET; xb++) V->bstart[yb * V->bx + xb + 1]++;
    }
    for (int64_t b = 0; b < nb; b++) V->bstart[b + 1] += V->bstart[b];
    V->blist = (int64_t*)malloc(sizeof(int64_t) * (V->bstart[nb] > 0 ? V->bstart[nb] : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (nb > 0 ? nb : 1));
    memcpy(fill, V->bstart, sizeof(int64_t) * nb);
    for (int64_t k = 0; k < nv; k++) {
        int64_t id = V->order[k];
        const proj_t* p = &V->P[id];
        for (int yb = p->y0 / BUCKET; yb <= p->y1 / BUCKET; yb++)
            for (int xb = p->x0 / BUCKET; xb <= p->x1 / BUCKET; xb++) V->blist[fill[yb * V->bx + xb]++] = id;
    }
    free(fill);
    return 0;
}

static void free_view(view_t* V) {
    free(V->P); free(V->order); free(V->bstart); free(V->blist);
}

/* one blended fragment */
typedef struct {
    int64_t id;
    double alpha, raw, G, dx, dy, T; /* T = transmittance before this fragment */
} frag_t;

/* Tie groups of blended fragments whose depths a single-precision renderer
 * may order either way (consecutive in depth order, each within the order
 * band of the previous one).  Reordering a group that starts at transmittance
 * T0 leaves the product of its (1 - alpha) and everything behind it unchanged
 * and changes the colour by at most T0 sum_{i<j} a_i a_j |c_i - c_j| (any
 * order is reached by swapping each inverted pair once, each swap at a
 * transmittance <= T0 changing the colour by a_i a_j T |c_i - c_j|); depth the
 * same with z, alpha not at all.  Where the order also decides where the pixel
 * stops (a tie with the stopping candidate), or the group is longer than
 * GROUP_MAX, the coarser bound holds: whatever blends from T0 on contributes
 * between 0 and T0 max c (a weighted sum with weights summing to at most 1),
 * T0 max z to the depth, and leaves T_final in [0, T0]. */
#define GROUP_MAX 32
typedef struct {
    double T0;
    int n;
    int coarse;
    double cmax[3], zmax;
    double a[GROUP_MAX], c[GROUP_MAX][3], z[GROUP_MAX];
} group_t;

static void group_open(group_t* g, double T0) {
    g->T0 = T0;
    g->n = 0;
    g->coarse = 0;
    g->cmax[0] = g->cmax[1] = g->cmax[2] = 0.0;
    g->zmax = 0.0;
}

static void group_add(group_t* g, double a, const double* c, double z) {
    for (int k = 0; k < 3; k++) g->cmax[k] = c[k] > g->cmax[k] ? c[k] : g->cmax[k];
    g->zmax = z > g->zmax ? z : g->zmax;
    if (g->n < GROUP_MAX) {
        g->a[g->n] = a;
        g->c[g->n][0] = c[0]; g->c[g->n][1] = c[1]; g->c[g->n][2] = c[2];
        g->z[g->n] = z;
        g->n++;
    } else {
        g->coarse = 1;
    }
}

/* bound[0..2] colour, [3] depth, [4] alpha */
static void group_close(group_t* g, double* bound) {
    if (g->coarse) {
        for (int k = 0; k < 3; k++) bound[k] += g->T0 * g->cmax[k];
        bound[3] += g->T0 * g->zmax;
        bound[4] += g->T0;
    } else {
        for (int i = 0; i < g->n; i++)
            for (int j = i + 1; j < g->n; j++) {
                const double w = g->T0 * g->a[i] * g->a[j];
                for (int k = 0; k < 3; k++) bound[k] += w * fabs(g->c[i][k] - g->c[j][k]);
                bound[3] += w * fabs(g->z[i] - g->z[j]);
            }
    }
    g->n = 0;
    g->coarse = 0;
}

/* Composite one pixel front to back (colour / depth compositing equations,
 * border-mask equation).  Candidates are the visible Gaussians whose pixel
 * rect contains (x, y), in ascending (depth, id) order.  Fills the outputs and,
 * if frags != NULL, the blended fragments; if bound != NULL, bound[0..4] =
 * the largest change of C (per channel), D and A that reordering the tie
 * groups can make.  Returns the number of blended fragments. */
static int composite_pixel(const view_t* V, int x, int y, double band_skip, double band_clamp,
                           double band_term, double band_order, double* col, double* dep, double* Tfin,
                           int* amb, int64_t* nvisit, frag_t** frags, int* fcap, double* bound) {
    const int64_t b = (int64_t)(y / BUCKET) * V->bx + x / BUCKET;
    double T = 1.0, C0 = 0, C1 = 0, C2 = 0, D = 0;
    double zprev = -1.0, zscprev = 0.0;
    int nb = 0;
    int64_t visits = 0;
    group_t grp;
    group_open(&grp, 1.0);
    if (bound) bound[0] = bound[1] = bound[2] = bound[3] = bound[4] = 0.0;
    *amb = 0;
    for (int64_t k = V->bstart[b]; k < V->bstart[b + 1]; k++) {
        const int64_t id = V->blist[k];
        const proj_t* p = &V->P[id];
        if (x < p->x0 || x > p->x1 || y < p->y0 || y > p->y1) continue;
        visits++;
        const double dx = x - p->u, dy = y - p->v;
        const double sigma = 0.5 * (p->A * dx * dx + p->C * dy * dy) + p->B * dx * dy;
        if (sigma < 0) continue;
        const double G = exp(-sigma);
        const double raw = p->o * G;
        if (fabs(raw - ALPHA_MIN) < band_skip * ALPHA_MIN) *amb |= 1;
        if (fabs(raw - ALPHA_MAX) < band_clamp) *amb |= 2;
        const double alpha = raw < ALPHA_MAX ? raw : ALPHA_MAX;
        if (alpha < ALPHA_MIN) continue;
        const double Tn = T * (1.0 - alpha);
        if (fabs(Tn - T_MIN) < band_term * T_MIN) *amb |= 4;
        /* two blended Gaussians whose depths a single-precision renderer
           cannot order reliably: the blend order there is a rounding decision */
        const int tied = zprev >= 0 && fabs(p->z - zprev) <= band_order * (p->zsc > zscprev ? p->zsc : zscprev);
        if (Tn < T_MIN) {
            /* a tie at the stop: the order decides which fragments blend */
            if (tied) {
                *amb |= 16;
                if (bound) {
                    group_add(&grp, alpha, p->col, p->z);
                    grp.coarse = 1;
                }
            }
            break;
        }
        if (tied) *amb |= 8;
        if (bound) {
            if (!tied) {
                group_close(&grp, bound);
                group_open(&grp, T);
            }
            group_add(&grp, alpha, p->col, p->z);
        }
        zprev = p->z;
        zscprev = p->zsc;
        const double w = alpha * T;
        C0 += p->col[0] * w;
        C1 += p->col[1] * w;
        C2 += p->col[2] * w;
        D += p->z * w;
        if (frags) {
            if (nb == *fcap) {
                *fcap = *fcap ? 2 * *fcap : 64;
                *frags = (frag_t*)realloc(*frags, sizeof(frag_t) * (size_t)*fcap);
            }
            frag_t* f = &(*frags)[nb];
            f->id = id; f->alpha = alpha; f->raw = raw; f->G = G; f->dx = dx; f->dy = dy; f->T = T;
        }
        nb++;
        T = Tn;
    }
    if (bound) group_close(&grp, bound);
    col[0] = C0; col[1] = C1; col[2] = C2;
    *dep = D;
    *Tfin = T;
    *nvisit = visits;
    return nb;
}

static void unpack_gs(gs_t* g, int64_t n, int sh, const double* means, const double* ls, const double* q,
                      const double* opl, const double* col) {
    g->n = n; g->sh_degree = sh; g->means = means; g->log_scales = ls; g->quats = q; g->opl = opl;
    g->colors = col;
}

/* ============================ exported API ============================ */

int or_abi_version(void) { return 1; }

/* Per-Gaussian projection records of one view: out[n, 20] =
 * valid, u, v, A, B, C, o, r, g, b, z, radius, x0, x1, y0, y1, a, b, c, det */
int or_project(int64_t n, int sh, const double* means, const double* ls, const double* q, const double* opl,
               const double* col, int W, int H, double fx, double fy, double cx, double cy, const double* T,
               double* out) {
    gs_t g; cam_t cam;
    unpack_gs(&g, n, sh, means, ls, q, opl, col);
    make_cam(&cam, W, H, fx, fy, cx, cy, T);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        proj_t P;
        project(&g, i, &cam, &P);
        double* o = out + 20 * i;
        o[0] = P.valid; o[1] = P.u; o[2] = P.v; o[3] = P.A; o[4] = P.B; o[5] = P.C; o[6] = P.o;
        o[7] = P.col[0]; o[8] = P.col[1]; o[9] = P.col[2]; o[10] = P.z; o[11] = P.radius;
        o[12] = P.x0; o[13] = P.x1; o[14] = P.y0; o[15] = P.y1; o[16] = P.a; o[17] = P.b; o[18] = P.c;
        o[19] = P.det;
    }
    return 0;
}

/* Render one view.  npix < 0: the whole image, outputs planar [3,H,W] / [H,W];
 * otherwise the listed pixels pix[npix,2] (x, y), outputs [3,npix] / [npix].
 * ambiguous[k] flags decisions near their thresholds: bit 0 the 1/255 skip
 * (relative band), bit 1 the 0.99 clamp (absolute band; changes gradients
 * only), bit 2 the 1e-4 termination (relative band), bit 3 two blended
 * Gaussians whose depths differ by at most band_order times the magnitude of
 * the terms their depths are summed from (the order a single-precision sort
 * may swap), bit 4 such a tie at the candidate that stops the pixel (the
 * order decides which fragments blend).  order_bound (nullable, [5, np]): the
 * largest change of C (per channel), D and A that reordering the tie groups
 * can make.  nfrag_alg returns the number of
 * candidates visited up to and including the terminating one. */
int or_render(int64_t n, int sh, const double* means, const double* ls, const double* q, const double* opl,
              const double* col, int W, int H, double fx, double fy, double cx, double cy, const double* T,
              int64_t npix, const int32_t* pix, double band_skip, double band_clamp, double band_term,
              double band_order, double* color, double* depth, double* alpha, double* tfinal, int32_t* nblend,
              int8_t* ambiguous, int64_t* nfrag_alg, double* order_bound) {
    gs_t g; cam_t cam; view_t V;
    unpack_gs(&g, n, sh, means, ls, q, opl, col);
    make_cam(&cam, W, H, fx, fy, cx, cy, T);
    if (build_view(&g, &cam, &V)) return -1;
    const int64_t np = npix < 0 ? (int64_t)W * H : npix;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (int64_t k = 0; k < np; k++) {
        int x = npix < 0 ? (int)(k % W) : pix[2 * k];
        int y = npix < 0 ? (int)(k / W) : pix[2 * k + 1];
        double c3[3], d, t;
        int amb;
        int64_t visits;
        double bd[5];
        int nb = composite_pixel(&V, x, y, band_skip, band_clamp, band_term, band_order, c3, &d, &t, &amb, &visits,
                                 NULL, NULL, order_bound ? bd : NULL);
        if (order_bound)
            for (int q = 0; q < 5; q++) order_bound[(int64_t)q * np + k] = bd[q];
        /* the terminating candidate counts as visited (it was evaluated) */
        total += visits;
        color[k] = c3[0]; color[np + k] = c3[1]; color[2 * np + k] = c3[2];
        depth[k] = d;
        alpha[k] = 1.0 - t;
        if (tfinal) tfinal[k] = t;
        if (nblend) nblend[k] = nb;
        if (ambiguous) ambiguous[k] = (int8_t)amb;
    }
    if (nfrag_alg) *nfrag_alg = total;
    free_view(&V);
    return 0;
}

/* Reverse mode of or_render for one view.  dC [3,np], dD [np], dA [np] are the
 * upstream gradients of the rendered colour, depth and alpha at the listed
 * pixels (any may be NULL = zero).  Gradients are ACCUMULATED (+=) into
 * g_means [n,3], g_ls [n,3], g_q [n,4], g_opl [n], g_col [n,3] or [n,K,3], and
 * into g_pose [6] = d/dxi at xi = 0 of the left perturbation
 * T_cw <- Exp(xi) T_cw, xi = (v, w). */
int or_backward(int64_t n, int sh, const double* means, const double* ls, const double* q, const double* opl,
                const double* col, int W, int H, double fx, double fy, double cx, double cy, const double* T,
                int64_t npix, const int32_t* pix, const double* dC, const double* dD, const double* dA,
                double* g_means, double* g_ls, double* g_q, double* g_opl, double* g_col, double* g_pose) {
    gs_t g; cam_t cam; view_t V;
    unpack_gs(&g, n, sh, means, ls, q, opl, col);
    make_cam(&cam, W, H, fx, fy, cx, cy, T);
    if (build_view(&g, &cam, &V)) return -1;
    const int64_t np = npix < 0 ? (int64_t)W * H : npix;
    const int nth = omp_get_max_threads();
    /* per-thread accumulators of the gradient w.r.t. each Gaussian's 2D record:
       du, dv, dA, dB, dC, dopacity, dcolour[3], ddepth */
    double* g2 = (double*)calloc((size_t)nth * (size_t)(n > 0 ? n : 1) * 10, sizeof(double));
    if (!g2) { free_view(&V); return -1; }
#pragma omp parallel
    {
        const int tid = omp_get_thread_num();
        double* acc = g2 + (size_t)tid * (size_t)n * 10;
        frag_t* fr = NULL;
        int fcap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < np; k++) {
            int x = npix < 0 ? (int)(k % W) : pix[2 * k];
            int y = npix < 0 ? (int)(k / W) : pix[2 * k + 1];
            double c3[3], d, Tf;
            int amb;
            int64_t visits;
            int nb = composite_pixel(&V, x, y, 0, 0, 0, -1.0, c3, &d, &Tf, &amb, &visits, &fr, &fcap, NULL);
            const double gC0 = dC ? dC[k] : 0, gC1 = dC ? dC[np + k] : 0, gC2 = dC ? dC[2 * np + k] : 0;
            const double gD = dD ? dD[k] : 0, gA = dA ? dA[k] : 0;
            /* suffix sums S of later weighted colours / depths */
            double S0 = 0, S1 = 0, S2 = 0, SD = 0;
            for (int i = nb - 1; i >= 0; i--) {
                const frag_t* f = &fr[i];
                const proj_t* p = &V.P[f->id];
                const double w = f->alpha * f->T;
                const double om = 1.0 - f->alpha;
                double* a = acc + 10 * f->id;
                /* colour and depth of the fragment */
                a[6] += gC0 * w; a[7] += gC1 * w; a[8] += gC2 * w;
                a[9] += gD * w;
                /* alpha of the fragment */
                double dal = gC0 * (p->col[0] * f->T - S0 / om) + gC1 * (p->col[1] * f->T - S1 / om) +
                             gC2 * (p->col[2] * f->T - S2 / om) + gD * (p->z * f->T - SD / om) +
                             gA * Tf / om;
                S0 += p->col[0] * w; S1 += p->col[1] * w; S2 += p->col[2] * w; SD += p->z * w;
                if (f->raw > ALPHA_MAX) continue; /* clamped: alpha does not depend on o, sigma */
                a[5] += dal * f->G;               /* d alpha / d o */
                const double dsig = -dal * f->raw; /* d alpha / d sigma = -o G */
                a[2] += dsig * 0.5 * f->dx * f->dx;
                a[3] += dsig * f->dx * f->dy;
                a[4] += dsig * 0.5 * f->dy * f->dy;
                /* delta = pixel - mean, so d/du = -d/d(dx) */
                a[0] += -dsig * (p->A * f->dx + p->B * f->dy);
                a[1] += -dsig * (p->C * f->dy + p->B * f->dx);
            }
        }
        free(fr);
    }
    /* reduce the per-thread accumulators in a fixed order */
    for (int t = 1; t < nth; t++) {
        const double* src = g2 + (size_t)t * (size_t)n * 10;
        for (int64_t i = 0; i < n * 10; i++) g2[i] += src[i];
    }

    /* chain rule from each Gaussian's 2D record to its parameters and to the pose */
    const int K = sh >= 0 ? (sh + 1) * (sh + 1) : 0;
    double pose[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < n; i++) {
        const proj_t* P = &V.P[i];
        if (!P->valid) continue;
        const double* a = g2 + 10 * i;
        const double px = P->p[0], py = P->p[1], pz = P->p[2];
        double dp[3] = {0, 0, 0};
        double dmu[3] = {0, 0, 0};
        /* colour */
        double dCc[3] = {0, 0, 0};
        if (sh < 0) {
            for (int k = 0; k < 3; k++) g_col[3 * i + k] += a[6 + k];
        } else {
            double Y[16], dY[16][3];
            sh_eval(sh, P->dir, Y, dY);
            const double* shc = col + (int64_t)K * 3 * i;
            double ddir[3] = {0, 0, 0};
            for (int k = 0; k < 3; k++) {
                if (P->colclamp[k]) continue;
                for (int l = 0; l < K; l++) {
                    g_col[(int64_t)K * 3 * i + 3 * l + k] += Y[l] * a[6 + k];
                    for (int j = 0; j < 3; j++) ddir[j] += a[6 + k] * shc[3 * l + k] * dY[l][j];
                }
            }
            /* unit direction = (mu - C_cam) / |mu - C_cam| */
            double dd = ddir[0] * P->dir[0] + ddir[1] * P->dir[1] + ddir[2] * P->dir[2];
            for (int j = 0; j < 3; j++) {
                double gdj = (ddir[j] - P->dir[j] * dd) / P->dirn;
                dmu[j] += gdj;
                dCc[j] -= gdj;
            }
        }
        /* opacity = sigmoid(logit) */
        g_opl[i] += a[5] * P->o * (1.0 - P->o);
        /* depth */
        dp[2] += a[9];
        /* projected mean */
        dp[0] += a[0] * cam.fx / pz;
        dp[2] += -a[0] * cam.fx * px / (pz * pz);
        dp[1] += a[1] * cam.fy / pz;
        dp[2] += -a[1] * cam.fy * py / (pz * pz);
        /* conic -> dilated 2D covariance: G_S = -Q G_Q Q with Q the conic matrix */
        double Q[4] = {P->A, P->B, P->B, P->C};
        double GQ[4] = {a[2], 0.5 * a[3], 0.5 * a[3], a[4]};
        double QG[4] = {Q[0] * GQ[0] + Q[1] * GQ[2], Q[0] * GQ[1] + Q[1] * GQ[3], Q[2] * GQ[0] + Q[3] * GQ[2],
                        Q[2] * GQ[1] + Q[3] * GQ[3]};
        double G2[4] = {-(QG[0] * Q[0] + QG[1] * Q[2]), -(QG[0] * Q[1] + QG[1] * Q[3]),
                        -(QG[2] * Q[0] + QG[3] * Q[2]), -(QG[2] * Q[1] + QG[3] * Q[3])};
        /* Sigma_2D = J Sigma_c J^T (dilation is a constant) */
        double GSc[9], dJ[6];
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) {
                double s = 0;
                for (int u = 0; u < 2; u++)
                    for (int v = 0; v < 2; v++) s += P->J[3 * u + r] * G2[2 * u + v] * P->J[3 * v + c];
                GSc[3 * r + c] = s;
            }
        for (int u = 0; u < 2; u++)
            for (int c = 0; c < 3; c++) {
                double s = 0;
                for (int v = 0; v < 2; v++)
                    for (int k = 0; k < 3; k++) s += G2[2 * u + v] * P->J[3 * v + k] * P->Sc[3 * k + c];
                dJ[3 * u + c] = 2.0 * s;
            }
        /* J -> camera-space mean */
        dp[2] += dJ[0] * (-cam.fx / (pz * pz));
        dp[2] += dJ[4] * (-cam.fy / (pz * pz));
        if (!P->clx) {
            dp[0] += dJ[2] * (-cam.fx / (pz * pz));
            dp[2] += dJ[2] * (2.0 * cam.fx * px / (pz * pz * pz));
        } else {
            dp[2] += dJ[2] * (cam.fx * P->cxv / (pz * pz));
        }
        if (!P->cly) {
            dp[1] += dJ[5] * (-cam.fy / (pz * pz));
            dp[2] += dJ[5] * (2.0 * cam.fy * py / (pz * pz * pz));
        } else {
            dp[2] += dJ[5] * (cam.fy * P->cyv / (pz * pz));
        }
        /* Sigma_c = R_cw Sigma R_cw^T -> dSigma = R_cw^T GSc R_cw */
        double t1[9], GS[9];
        mat3_mul_at(cam.Rw, GSc, t1);
        mat3_mul(t1, cam.Rw, GS);
        /* Sigma = R diag(s^2) R^T: dR = 2 GS R diag(s^2); ds_k = 2 s_k (R^T GS R)_kk */
        double RtGR[9], t2[9];
        mat3_mul_at(P->R, GS, t2);
        mat3_mul(t2, P->R, RtGR);
        for (int k = 0; k < 3; k++) g_ls[3 * i + k] += 2.0 * P->s[k] * RtGR[4 * k] * P->s[k];
        double GR[9], dR[9];
        mat3_mul(GS, P->R, GR);
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) dR[3 * r + c] = 2.0 * GR[3 * r + c] * P->s[c] * P->s[c];
        /* R(q) -> unit quaternion */
        const double w = P->qh[0], x = P->qh[1], y = P->qh[2], z = P->qh[3];
        double dq[4];
        dq[0] = dR[1] * (-2 * z) + dR[2] * (2 * y) + dR[3] * (2 * z) + dR[5] * (-2 * x) + dR[6] * (-2 * y) +
                dR[7] * (2 * x);
        dq[1] = dR[1] * (2 * y) + dR[2] * (2 * z) + dR[3] * (2 * y) + dR[4] * (-4 * x) + dR[5] * (-2 * w) +
                dR[6] * (2 * z) + dR[7] * (2 * w) + dR[8] * (-4 * x);
        dq[2] = dR[0] * (-4 * y) + dR[1] * (2 * x) + dR[2] * (2 * w) + dR[3] * (2 * x) + dR[5] * (2 * z) +
                dR[6] * (-2 * w) + dR[7] * (2 * z) + dR[8] * (-4 * y);
        dq[3] = dR[0] * (-4 * z) + dR[1] * (-2 * w) + dR[2] * (2 * x) + dR[3] * (2 * w) + dR[4] * (-4 * z) +
                dR[5] * (2 * y) + dR[6] * (2 * x) + dR[7] * (2 * y);
        /* normalisation q -> q / |q| */
        double qd = dq[0] * P->qh[0] + dq[1] * P->qh[1] + dq[2] * P->qh[2] + dq[3] * P->qh[3];
        for (int k = 0; k < 4; k++) g_q[4 * i + k] += (dq[k] - P->qh[k] * qd) / P->qn;
        /* p = R_cw mu + t_cw */
        for (int c = 0; c < 3; c++)
            dmu[c] += cam.Rw[c] * dp[0] + cam.Rw[3 + c] * dp[1] + cam.Rw[6 + c] * dp[2];
        for (int c = 0; c < 3; c++) g_means[3 * i + c] += dmu[c];
        /* pose, left perturbation: dp/dv = I, dp/dw = -[p]x; Sigma_c picks up
           [w]x Sigma_c - Sigma_c [w]x; the camera centre moves by -R_cw^T v */
        pose[0] += dp[0]; pose[1] += dp[1]; pose[2] += dp[2];
        for (int r = 0; r < 3; r++)
            pose[r] -= cam.Rw[3 * r] * dCc[0] + cam.Rw[3 * r + 1] * dCc[1] + cam.Rw[3 * r + 2] * dCc[2];
        pose[3] += py * dp[2] - pz * dp[1];
        pose[4] += pz * dp[0] - px * dp[2];
        pose[5] += px * dp[1] - py * dp[0];
        for (int k = 0; k < 3; k++) {
            double E[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            /* hat(e_k) */
            if (k == 0) { E[5] = -1; E[7] = 1; }
            if (k == 1) { E[2] = 1; E[6] = -1; }
            if (k == 2) { E[1] = -1; E[3] = 1; }
            double M1[9], M2[9];
            mat3_mul(E, P->Sc, M1);
            mat3_mul(P->Sc, E, M2);
            double s = 0;
            for (int e = 0; e < 9; e++) s += GSc[e] * (M1[e] - M2[e]);
            pose[3 + k] += s;
        }
    }
    for (int k = 0; k < 6; k++) g_pose[k] += pose[k];
    free(g2);
    free_view(&V);
    return 0;
}

/* Re-projection residuals (Sec. 3.2, Eq. lba) with a Huber kernel on the
 * Euclidean norm.  residual[M,2] = uv - pi(T_v P) (0 for matches with
 * camera-space z <= 0.2, which are excluded).  loss[V] = mean over valid
 * matches of h(|r|); dpose[V,6] = d loss[v] / d xi_v (overwritten). */
int or_reproj(int V, const int32_t* W, const int32_t* H, const double* intr /*[V,4] fx fy cx cy*/,
              const double* T /*[V,16]*/, int64_t M, const double* P, const double* uv, const int32_t* vid,
              double delta, double* residual, double* loss, double* dpose, int64_t* nvalid) {
    (void)W; (void)H;
    for (int v = 0; v < V; v++) {
        loss[v] = 0;
        nvalid[v] = 0;
        for (int k = 0; k < 6; k++) dpose[6 * v + k] = 0;
    }
    for (int64_t m = 0; m < M; m++) {
        int v = vid[m];
        residual[2 * m] = 0;
        residual[2 * m + 1] = 0;
        if (v < 0 || v >= V) continue;
        const double* Tv = T + 16 * v;
        double p[3];
        for (int r = 0; r < 3; r++)
            p[r] = Tv[4 * r] * P[3 * m] + Tv[4 * r + 1] * P[3 * m + 1] + Tv[4 * r + 2] * P[3 * m + 2] + Tv[4 * r + 3];
        if (p[2] <= ZNEAR) continue;
        const double fx = intr[4 * v], fy = intr[4 * v + 1], cx = intr[4 * v + 2], cy = intr[4 * v + 3];
        double r0 = uv[2 * m] - (fx * p[0] / p[2] + cx);
        double r1 = uv[2 * m + 1] - (fy * p[1] / p[2] + cy);
        residual[2 * m] = r0;
        residual[2 * m + 1] = r1;
        double e = sqrt(r0 * r0 + r1 * r1);
        double h, s;
        if (e <= delta) { h = 0.5 * e * e; s = 1.0; }
        else { h = delta * (e - 0.5 * delta); s = delta / e; }
        loss[v] += h;
        nvalid[v]++;
        /* dh/dr = s r;  r = uv - pi  =>  dh/dpi = -s r */
        double gu = -s * r0, gv = -s * r1;
        double dp[3] = {gu * fx / p[2], gv * fy / p[2], -(gu * fx * p[0] + gv * fy * p[1]) / (p[2] * p[2])};
        double* g = dpose + 6 * v;
        g[0] += dp[0]; g[1] += dp[1]; g[2] += dp[2];
        g[3] += p[1] * dp[2] - p[2] * dp[1];
        g[4] += p[2] * dp[0] - p[0] * dp[2];
        g[5] += p[0] * dp[1] - p[1] * dp[0];
    }
    for (int v = 0; v < V; v++) {
        if (nvalid[v] > 0) {
            loss[v] /= (double)nvalid[v];
            for (int k = 0; k < 6; k++) dpose[6 * v + k] /= (double)nvalid[v];
        }
    }
    return 0;
}

/* ---------------- binning (integer stage) ----------------
 * Records r = v*n + i carry an inclusive pixel rect, packed
 * rect[2r] = x0 | x1 << 16, rect[2r+1] = y0 | y1 << 16 (clipped to its view's
 * image: x1 <= W - 1, y1 <= H - 1; empty if then x0 > x1 or y0 > y1), and an
 * FP32 depth whose bit pattern orders positive depths.  The
 * global id of tile (tx, ty) of view v is tile_off[v] + ty * tiles_x[v] + tx.
 * Output: every (tile, record) pair with the record's rect touching the tile,
 * sorted by (tile, depth bits, record); ranges[2t], ranges[2t+1] = [start,
 * end) of tile t in that order, (0, 0) for a tile with no pair. */
typedef struct { uint32_t tile, dbits, rec; } trip_t;
static int cmp_trip(const void* a, const void* b) {
    const trip_t* x = (const trip_t*)a;
    const trip_t* y = (const trip_t*)b;
    if (x->tile != y->tile) return x->tile < y->tile ? -1 : 1;
    if (x->dbits != y->dbits) return x->dbits < y->dbits ? -1 : 1;
    if (x->rec != y->rec) return x->rec < y->rec ? -1 : 1;
    return 0;
}

/* record r's rect clipped to its view's image (W x H); 0 when empty */
static int clip_rect(const uint32_t* rect, int64_t r, int32_t W, int32_t H, uint32_t* x0, uint32_t* x1,
                     uint32_t* y0, uint32_t* y1) {
    *x0 = rect[2 * r] & 0xffff;
    *x1 = rect[2 * r] >> 16;
    *y0 = rect[2 * r + 1] & 0xffff;
    *y1 = rect[2 * r + 1] >> 16;
    if (*x1 > (uint32_t)W - 1) *x1 = (uint32_t)W - 1;
    if (*y1 > (uint32_t)H - 1) *y1 = (uint32_t)H - 1;
    return !(*x0 > *x1 || *y0 > *y1);
}

int64_t or_binning_count(int V, int64_t n, const int32_t* W, const int32_t* H, int tw, int th,
                         const uint32_t* rect) {
    int64_t total = 0;
    for (int v = 0; v < V; v++)
        for (int64_t i = 0; i < n; i++) {
            uint32_t x0, x1, y0, y1;
            if (!clip_rect(rect, (int64_t)v * n + i, W[v], H[v], &x0, &x1, &y0, &y1)) continue;
            total += (int64_t)(x1 / tw - x0 / tw + 1) * (y1 / th - y0 / th + 1);
        }
    return total;
}

int or_binning(int V, int64_t n, const int32_t* W, const int32_t* H, int tw, int th, const uint32_t* rect,
               const float* depth, uint32_t* values, uint32_t* ranges, int64_t ntiles_total) {
    int64_t total = or_binning_count(V, n, W, H, tw, th, rect);
    trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)(total > 0 ? total : 1));
    int64_t k = 0;
    uint32_t toff = 0;
    for (int v = 0; v < V; v++) {
        uint32_t tx = (uint32_t)((W[v] + tw - 1) / tw), ty = (uint32_t)((H[v] + th - 1) / th);
        for (int64_t i = 0; i < n; i++) {
            int64_t r = (int64_t)v * n + i;
            uint32_t x0, x1, y0, y1;
            if (!clip_rect(rect, r, W[v], H[v], &x0, &x1, &y0, &y1)) continue;
            uint32_t bits;
            memcpy(&bits, &depth[r], 4);
            for (uint32_t b = y0 / th; b <= y1 / th; b++)
                for (uint32_t a = x0 / tw; a <= x1 / tw; a++) {
                    t[k].tile = toff + b * tx + a;
                    t[k].dbits = bits;
                    t[k].rec = (uint32_t)r;
                    k++;
                }
        }
        toff += tx * ty;
    }
    qsort(t, (size_t)total, sizeof(trip_t), cmp_trip);
    for (int64_t i = 0; i < 2 * ntiles_total; i++) ranges[i] = 0;
    for (int64_t i = 0; i < total; i++) {
        values[i] = t[i].rec;
        if (i == 0 || t[i].tile != t[i - 1].tile) ranges[2 * (int64_t)t[i].tile] = (uint32_t)i;
        if (i == total - 1 || t[i].tile != t[i + 1].tile) ranges[2 * (int64_t)t[i].tile + 1] = (uint32_t)(i + 1);
    }
    free(t);
    return 0;
}

/* SH basis values (and polynomial gradients) at unit directions, for pins. */
int or_sh_basis(int deg, int64_t m, const double* dirs, double* Y, double* dY) {
    int K = (deg + 1) * (deg + 1);
    for (int64_t i = 0; i < m; i++) {
        double y[16], g[16][3];
        sh_eval(deg, dirs + 3 * i, y, g);
        for (int l = 0; l < K; l++) {
            Y[K * i + l] = y[l];
            if (dY)
                for (int j = 0; j < 3; j++) dY[(K * i + l) * 3 + j] = g[l][j];
        }
    }
    return 0;
}

int or_num_threads(void) { return omp_get_max_threads(); }

/* thread count of the OpenMP loops (the benchmark's 1-thread baseline) */
void or_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
