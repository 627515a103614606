/*
 * CPU oracle for the 3D-Gaussian rasterizer: TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct reference for one render call and its
 * adjoint.  Only tests, the smoke check and the benchmark's CPU-baseline leg
 * may load it; the product path never does.  It shares no code with the HIP
 * library.
 *
 * What it computes (paper, Sec. 3 and Sec. 4.1):
 *   - transformed Gaussians: mu' = mu + dmu, q' = norm(q) x norm(dq)
 *     (Sec. 4.1, "Mean" and "Rotation"); view-dependent colour evaluated at
 *     the direction rotated back by the delta rotation (Sec. 4.1 "SH
 *     Coefficients" and Suppl. Sec. B: rotating the SH coefficients equals
 *     evaluating the original SH at the inversely rotated direction);
 *   - covariance Sigma = R S S^T R^T (Eq. 2);
 *   - EWA projection Sigma' = J W Sigma W^T J^T, keep the upper-left 2x2
 *     (Eq. 3), plus a 0.3 px^2 low-pass on the diagonal;
 *   - per-pixel front-to-back alpha blending of the depth-ordered Gaussians
 *     that cover the pixel (Eq. 4), untiled;
 *   - the exact FP64 adjoint of all of the above.
 * Continuous arithmetic is double precision.  The discrete decisions
 * (culling, 3-sigma pixel box, tile rectangle, depth key bits) are taken by
 * spec_preprocess() in single precision with a fixed operation order and no
 * contraction, which the GPU path reproduces, so that sort keys and tile
 * ranges can be compared bit for bit.
 *
 * Readings where the paper is silent: quaternions are (w, x, y, z) with the
 * Hamilton product; pixel (x, y) is evaluated at integer coordinates; a
 * Gaussian covers pixel p when p lies in its 3-sigma pixel box; alpha is
 * clamped to 0.99, candidates with alpha < 1/255 are skipped, and the walk
 * stops before a Gaussian that would drive transmittance below 1e-4; colour
 * = max(0, SH + 0.5); background added with the final transmittance.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t n;
    int32_t sh_degree;
    int32_t pad_;
    const float *means, *quats, *log_scales, *opacity_logits, *sh, *dmu, *dq;
} orc_gaussians;

typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy, near_z;
    float w2c[12];
    float cam_pos[3];
    float bg[3];
} orc_camera;

typedef struct {
    /* per-Gaussian gradients, double, caller-zeroed, accumulated; any may be NULL */
    double *d_means, *d_quats, *d_log_scales, *d_opacity_logits, *d_sh, *d_dmu, *d_dq;
    /* 2D intermediates: (u, v), (A, B, C) conic, opacity, rgb */
    double *d_uv, *d_conic, *d_opacity, *d_rgb;
} orc_grads;

/* ------------------------------------------------------------------------ */
/* Single-precision decision procedure                                       */
/* ------------------------------------------------------------------------ */

/* exp for the scale activation in the decision procedure: Cody-Waite
 * reduction x = k ln2 + r (ln2 split into a 16-bit head and a tail), then
 * the degree-7 Taylor polynomial of e^r by Horner's rule, scaled by 2^k. */
float orc_spec_exp(float x) {
    x = fminf(fmaxf(x, -87.0f), 88.0f);
    float k = rintf(x * 0x1.715476p+0f);
    float r = x - k * 0x1.62e4p-1f;
    r = r - k * 0x1.7f7d1cp-20f;
    float p = 1.0f / 5040.0f;
    p = p * r + 1.0f / 720.0f;
    p = p * r + 1.0f / 120.0f;
    p = p * r + 1.0f / 24.0f;
    p = p * r + 1.0f / 6.0f;
    p = p * r + 0.5f;
    p = p * r + 1.0f;
    p = p * r + 1.0f;
    return ldexpf(p, (int)k);
}

typedef struct {
    int visible;
    uint32_t key;      /* bit pattern of view-space z */
    int32_t box[4];    /* x0, y0, x1, y1 inclusive pixel box */
    int32_t rect[4];   /* tile rectangle, inclusive */
    int64_t ntiles;
    float u, v, radius;
    float A, B, C;     /* conic: inverse of the dilated 2D covariance */
    float opacity;     /* sigmoid of the logit */
} spec_t;

static void spec_preprocess(const orc_gaussians* g, const orc_camera* c, int64_t i,
                            int tile, spec_t* o) {
    o->visible = 0;
    o->ntiles = 0;
    const float* W = c->w2c;
    float m0 = g->means[3 * i + 0], m1 = g->means[3 * i + 1], m2 = g->means[3 * i + 2];
    if (g->dmu) {
        m0 = m0 + g->dmu[3 * i + 0];
        m1 = m1 + g->dmu[3 * i + 1];
        m2 = m2 + g->dmu[3 * i + 2];
    }
    float tx = ((W[0] * m0 + W[1] * m1) + W[2] * m2) + W[3];
    float ty = ((W[4] * m0 + W[5] * m1) + W[6] * m2) + W[7];
    float tz = ((W[8] * m0 + W[9] * m1) + W[10] * m2) + W[11];
    if (!(tz > c->near_z)) return;

    const float* q = g->quats + 4 * i;
    float qn = sqrtf(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
    float aw = 1.0f, ax = 0.0f, ay = 0.0f, az = 0.0f;
    if (qn > 0.0f) { aw = q[0] / qn; ax = q[1] / qn; ay = q[2] / qn; az = q[3] / qn; }
    float w = aw, x = ax, y = ay, z = az;
    if (g->dq) {
        const float* d = g->dq + 4 * i;
        float dn = sqrtf(((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]) + d[3] * d[3]);
        dn = fmaxf(dn, 1e-12f);
        float bw = d[0] / dn, bx = d[1] / dn, by = d[2] / dn, bz = d[3] / dn;
        w = ((aw * bw - ax * bx) - ay * by) - az * bz;
        x = ((aw * bx + ax * bw) + ay * bz) - az * by;
        y = ((aw * by - ax * bz) + ay * bw) + az * bx;
        z = ((aw * bz + ax * by) - ay * bx) + az * bw;
    }
    float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
    float wx = w * x, wy = w * y, wz = w * z;
    float r00 = 1.0f - 2.0f * (yy + zz), r01 = 2.0f * (xy - wz), r02 = 2.0f * (xz + wy);
    float r10 = 2.0f * (xy + wz), r11 = 1.0f - 2.0f * (xx + zz), r12 = 2.0f * (yz - wx);
    float r20 = 2.0f * (xz - wy), r21 = 2.0f * (yz + wx), r22 = 1.0f - 2.0f * (xx + yy);
    float s0 = orc_spec_exp(g->log_scales[3 * i + 0]);
    float s1 = orc_spec_exp(g->log_scales[3 * i + 1]);
    float s2 = orc_spec_exp(g->log_scales[3 * i + 2]);
    float M00 = r00 * s0, M01 = r01 * s1, M02 = r02 * s2;
    float M10 = r10 * s0, M11 = r11 * s1, M12 = r12 * s2;
    float M20 = r20 * s0, M21 = r21 * s1, M22 = r22 * s2;
    float S00 = (M00 * M00 + M01 * M01) + M02 * M02;
    float S01 = (M00 * M10 + M01 * M11) + M02 * M12;
    float S02 = (M00 * M20 + M01 * M21) + M02 * M22;
    float S11 = (M10 * M10 + M11 * M11) + M12 * M12;
    float S12 = (M10 * M20 + M11 * M21) + M12 * M22;
    float S22 = (M20 * M20 + M21 * M21) + M22 * M22;

    float limx = (1.3f * (0.5f * (float)c->width)) / c->fx;
    float limy = (1.3f * (0.5f * (float)c->height)) / c->fy;
    float txz = tx / tz, tyz = ty / tz;
    float txc = fminf(fmaxf(txz, -limx), limx);
    float tyc = fminf(fmaxf(tyz, -limy), limy);
    float j00 = c->fx / tz, j02 = -(c->fx * txc) / tz;
    float j11 = c->fy / tz, j12 = -(c->fy * tyc) / tz;
    float T00 = j00 * W[0] + j02 * W[8], T01 = j00 * W[1] + j02 * W[9], T02 = j00 * W[2] + j02 * W[10];
    float T10 = j11 * W[4] + j12 * W[8], T11 = j11 * W[5] + j12 * W[9], T12 = j11 * W[6] + j12 * W[10];
    float U00 = (T00 * S00 + T01 * S01) + T02 * S02;
    float U01 = (T00 * S01 + T01 * S11) + T02 * S12;
    float U02 = (T00 * S02 + T01 * S12) + T02 * S22;
    float U10 = (T10 * S00 + T11 * S01) + T12 * S02;
    float U11 = (T10 * S01 + T11 * S11) + T12 * S12;
    float U12 = (T10 * S02 + T11 * S12) + T12 * S22;
    float a = ((U00 * T00 + U01 * T01) + U02 * T02) + 0.3f;
    float b = (U00 * T10 + U01 * T11) + U02 * T12;
    float cc = ((U10 * T10 + U11 * T11) + U12 * T12) + 0.3f;
    float det = a * cc - b * b;
    if (!(det > 0.0f)) return;
    float mid = 0.5f * (a + cc);
    float disc = mid * mid - det;
    float lam = mid + sqrtf(fmaxf(disc, 0.0f));
    float r = ceilf(3.0f * sqrtf(lam));
    float u = c->fx * txz + c->cx;
    float v = c->fy * tyz + c->cy;
    if (!(fabsf(u) <= 1e7f && fabsf(v) <= 1e7f && r <= 1e7f)) return;
    float x0 = fmaxf(ceilf(u - r), 0.0f), x1 = fminf(floorf(u + r), (float)(c->width - 1));
    float y0 = fmaxf(ceilf(v - r), 0.0f), y1 = fminf(floorf(v + r), (float)(c->height - 1));
    if (x0 > x1 || y0 > y1) return;
    o->box[0] = (int32_t)x0; o->box[1] = (int32_t)y0;
    o->box[2] = (int32_t)x1; o->box[3] = (int32_t)y1;
    for (int k = 0; k < 4; k++) o->rect[k] = o->box[k] / tile;
    o->ntiles = (int64_t)(o->rect[2] - o->rect[0] + 1) * (int64_t)(o->rect[3] - o->rect[1] + 1);
    uint32_t bits;
    memcpy(&bits, &tz, 4);
    o->key = bits;
    o->u = u; o->v = v; o->radius = r;
    o->A = cc / det;
    o->B = -b / det;
    o->C = a / det;
    o->opacity = 1.0f / (1.0f + orc_spec_exp(-g->opacity_logits[i]));
    o->visible = 1;
}

/* Contributor decision of the blend (Eq. 4 with the 1/255 cut-off), taken in
 * single precision: dx, dy and the exponent from the single-precision image
 * position and conic with a fixed operation order, alpha from the
 * decision-procedure exponential.  Returns 1 when the Gaussian contributes
 * and stores the single-precision exponent. */
static int spec_contributes(const spec_t* p, int x, int y, float* power_out) {
    float dx = (float)x - p->u, dy = (float)y - p->v;
    float power = -0.5f * (p->A * dx * dx + p->C * dy * dy) - p->B * dx * dy;
    *power_out = power;
    if (power > 0.0f) return 0;
    return p->opacity * orc_spec_exp(power) >= 1.0f / 255.0f;
}

/* ------------------------------------------------------------------------ */
/* Double-precision geometry                                                 */
/* ------------------------------------------------------------------------ */

static void quat_mul(const double a[4], const double b[4], double p[4]) {
    p[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    p[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    p[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    p[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

/* rotation matrix of a unit quaternion, row-major */
static void quat_rot(const double q[4], double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* adjoint of quat_rot: dq += (dR/dq)^T gR */
static void quat_rot_adj(const double q[4], const double g[9], double dq[4]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    dq[0] += 2 * (-z * g[1] + y * g[2] + z * g[3] - x * g[5] - y * g[6] + x * g[7]);
    dq[1] += 2 * (y * g[1] + z * g[2] + y * g[3] - 2 * x * g[4] - w * g[5] + z * g[6] + w * g[7] - 2 * x * g[8]);
    dq[2] += 2 * (-2 * y * g[0] + x * g[1] + w * g[2] + x * g[3] + z * g[5] - w * g[6] + z * g[7] - 2 * y * g[8]);
    dq[3] += 2 * (-2 * z * g[0] - w * g[1] + x * g[2] + w * g[3] - 2 * z * g[4] + y * g[5] + x * g[6] + y * g[7]);
}

static void mat3_mul(const double A[9], const double B[9], double C[9]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}

static void mat3_transpose(const double A[9], double B[9]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) B[3 * j + i] = A[3 * i + j];
}

/* Real orthonormal spherical harmonics up to degree 3 (Condon-Shortley
 * phase), index k = l*l + l + m, m = -l..l; Y[k] and its gradient with
 * respect to the (not renormalised) direction components. */
void orc_sh_basis(int deg, const double d[3], double Y[16], double dY[48]) {
    double x = d[0], y = d[1], z = d[2];
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < 16; k++) { Y[k] = 0; dY[3 * k] = dY[3 * k + 1] = dY[3 * k + 2] = 0; }
    Y[0] = 0.5 * sqrt(1.0 / pi);
    if (deg < 1) return;
    double c1 = sqrt(3.0 / (4.0 * pi));
    Y[1] = -c1 * y; dY[3 * 1 + 1] = -c1;
    Y[2] = c1 * z;  dY[3 * 2 + 2] = c1;
    Y[3] = -c1 * x; dY[3 * 3 + 0] = -c1;
    if (deg < 2) return;
    double a = 0.5 * sqrt(15.0 / pi), b = 0.25 * sqrt(5.0 / pi), e = 0.25 * sqrt(15.0 / pi);
    Y[4] = a * x * y;       dY[12] = a * y;      dY[13] = a * x;      dY[14] = 0;
    Y[5] = -a * y * z;      dY[15] = 0;          dY[16] = -a * z;     dY[17] = -a * y;
    Y[6] = b * (2 * z * z - x * x - y * y); dY[18] = -2 * b * x; dY[19] = -2 * b * y; dY[20] = 4 * b * z;
    Y[7] = -a * x * z;      dY[21] = -a * z;     dY[22] = 0;          dY[23] = -a * x;
    Y[8] = e * (x * x - y * y); dY[24] = 2 * e * x; dY[25] = -2 * e * y; dY[26] = 0;
    if (deg < 3) return;
    double f = 0.25 * sqrt(35.0 / (2.0 * pi)), h = 0.5 * sqrt(105.0 / pi);
    double s = 0.25 * sqrt(21.0 / (2.0 * pi)), t = 0.25 * sqrt(7.0 / pi), u = 0.25 * sqrt(105.0 / pi);
    Y[9] = -f * y * (3 * x * x - y * y);
    dY[27] = -f * 6 * x * y; dY[28] = -f * (3 * x * x - 3 * y * y); dY[29] = 0;
    Y[10] = h * x * y * z;
    dY[30] = h * y * z; dY[31] = h * x * z; dY[32] = h * x * y;
    Y[11] = -s * y * (4 * z * z - x * x - y * y);
    dY[33] = -s * y * (-2 * x); dY[34] = -s * (4 * z * z - x * x - 3 * y * y); dY[35] = -s * y * 8 * z;
    Y[12] = t * z * (2 * z * z - 3 * x * x - 3 * y * y);
    dY[36] = t * z * (-6 * x); dY[37] = t * z * (-6 * y); dY[38] = t * (6 * z * z - 3 * x * x - 3 * y * y);
    Y[13] = -s * x * (4 * z * z - x * x - y * y);
    dY[39] = -s * (4 * z * z - 3 * x * x - y * y); dY[40] = -s * x * (-2 * y); dY[41] = -s * x * 8 * z;
    Y[14] = u * z * (x * x - y * y);
    dY[42] = u * z * 2 * x; dY[43] = -u * z * 2 * y; dY[44] = u * (x * x - y * y);
    Y[15] = -f * x * (x * x - 3 * y * y);
    dY[45] = -f * (3 * x * x - 3 * y * y); dY[46] = -f * x * (-6 * y); dY[47] = 0;
}

/* all double-precision per-Gaussian quantities of the forward pass */
typedef struct {
    double m[3];
    double q_in_norm, qh[4];
    int has_dq;
    double dq_norm, dh[4];
    double qp[4];
    double Rp[9], Rh[9];
    double s[3];
    double Sig[9];
    double t[3];
    double txz, tyz;
    int clamp_x, clamp_y;
    double J00, J02, J11, J12;
    double T[6];
    double a, b, c, det;
    double A, B, C;
    double u, v;
    double opacity;
    double wvec[3], wnorm, dir[3];
    double Mloc[9];
    double dloc[3];
    double Y[16], dY[48];
    double rgb_raw[3], rgb[3];
} g64_t;

static void pre64(const orc_gaussians* g, const orc_camera* c, int64_t i, g64_t* o) {
    const float* W = c->w2c;
    for (int k = 0; k < 3; k++) o->m[k] = (double)g->means[3 * i + k] + (g->dmu ? (double)g->dmu[3 * i + k] : 0.0);
    double q[4];
    for (int k = 0; k < 4; k++) q[k] = g->quats[4 * i + k];
    o->q_in_norm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (o->q_in_norm > 0) for (int k = 0; k < 4; k++) o->qh[k] = q[k] / o->q_in_norm;
    else { o->qh[0] = 1; o->qh[1] = o->qh[2] = o->qh[3] = 0; }
    o->has_dq = g->dq != NULL;
    if (o->has_dq) {
        double d[4];
        for (int k = 0; k < 4; k++) d[k] = g->dq[4 * i + k];
        double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + d[3] * d[3]);
        o->dq_norm = n;
        double nn = n > 1e-12 ? n : 1e-12;
        for (int k = 0; k < 4; k++) o->dh[k] = d[k] / nn;
        quat_mul(o->qh, o->dh, o->qp);
    } else {
        for (int k = 0; k < 4; k++) o->qp[k] = o->qh[k];
    }
    quat_rot(o->qp, o->Rp);
    quat_rot(o->qh, o->Rh);
    for (int k = 0; k < 3; k++) o->s[k] = exp((double)g->log_scales[3 * i + k]);
    double M[9];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) M[3 * r + k] = o->Rp[3 * r + k] * o->s[k];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) {
            double acc = 0;
            for (int j = 0; j < 3; j++) acc += M[3 * r + j] * M[3 * k + j];
            o->Sig[3 * r + k] = acc;
        }
    for (int r = 0; r < 3; r++)
        o->t[r] = W[4 * r + 0] * o->m[0] + W[4 * r + 1] * o->m[1] + W[4 * r + 2] * o->m[2] + W[4 * r + 3];
    double fx = c->fx, fy = c->fy;
    double limx = 1.3 * 0.5 * c->width / fx, limy = 1.3 * 0.5 * c->height / fy;
    double tz = o->t[2];
    o->txz = o->t[0] / tz;
    o->tyz = o->t[1] / tz;
    double txc = o->txz, tyc = o->tyz;
    o->clamp_x = 0; o->clamp_y = 0;
    if (txc < -limx) { txc = -limx; o->clamp_x = 1; }
    if (txc > limx) { txc = limx; o->clamp_x = 1; }
    if (tyc < -limy) { tyc = -limy; o->clamp_y = 1; }
    if (tyc > limy) { tyc = limy; o->clamp_y = 1; }
    o->J00 = fx / tz; o->J02 = -fx * txc / tz;
    o->J11 = fy / tz; o->J12 = -fy * tyc / tz;
    for (int k = 0; k < 3; k++) {
        o->T[k] = o->J00 * W[k] + o->J02 * W[8 + k];
        o->T[3 + k] = o->J11 * W[4 + k] + o->J12 * W[8 + k];
    }
    double S2[4] = {0, 0, 0, 0};
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 2; k++) {
            double acc = 0;
            for (int p = 0; p < 3; p++)
                for (int qq = 0; qq < 3; qq++) acc += o->T[3 * r + p] * o->Sig[3 * p + qq] * o->T[3 * k + qq];
            S2[2 * r + k] = acc;
        }
    o->a = S2[0] + 0.3;
    o->b = S2[1];
    o->c = S2[3] + 0.3;
    o->det = o->a * o->c - o->b * o->b;
    o->A = o->c / o->det;
    o->B = -o->b / o->det;
    o->C = o->a / o->det;
    o->u = fx * o->txz + c->cx;
    o->v = fy * o->tyz + c->cy;
    o->opacity = 1.0 / (1.0 + exp(-(double)g->opacity_logits[i]));
    for (int k = 0; k < 3; k++) o->wvec[k] = o->m[k] - (double)c->cam_pos[k];
    o->wnorm = sqrt(o->wvec[0] * o->wvec[0] + o->wvec[1] * o->wvec[1] + o->wvec[2] * o->wvec[2]);
    for (int k = 0; k < 3; k++) o->dir[k] = o->wvec[k] / o->wnorm;
    if (o->has_dq) {
        double RpT[9];
        mat3_transpose(o->Rp, RpT);
        mat3_mul(o->Rh, RpT, o->Mloc); /* delta-R transposed = R(q^) R(q')^T */
    } else {
        for (int k = 0; k < 9; k++) o->Mloc[k] = (k % 4 == 0) ? 1.0 : 0.0;
    }
    for (int r = 0; r < 3; r++)
        o->dloc[r] = o->Mloc[3 * r] * o->dir[0] + o->Mloc[3 * r + 1] * o->dir[1] + o->Mloc[3 * r + 2] * o->dir[2];
    orc_sh_basis(g->sh_degree, o->dloc, o->Y, o->dY);
    int K = (g->sh_degree + 1) * (g->sh_degree + 1);
    const float* sh = g->sh + (int64_t)i * K * 3;
    for (int ch = 0; ch < 3; ch++) {
        double acc = 0;
        for (int k = 0; k < K; k++) acc += (double)sh[3 * k + ch] * o->Y[k];
        o->rgb_raw[ch] = acc + 0.5;
        o->rgb[ch] = o->rgb_raw[ch] > 0 ? o->rgb_raw[ch] : 0.0;
    }
}

/* Adjoint of pre64 given gradients on (u, v), (A, B, C), opacity and rgb. */
static void pre64_adj(const orc_gaussians* g, const orc_camera* c, int64_t i, const g64_t* o,
                      const double duv[2], const double dcon[3], double dop, const double drgb[3],
                      const orc_grads* out) {
    const float* W = c->w2c;
    double fx = c->fx, fy = c->fy;
    int K = (g->sh_degree + 1) * (g->sh_degree + 1);
    const float* sh = g->sh + (int64_t)i * K * 3;
    double dm[3] = {0, 0, 0};
    double dqp[4] = {0, 0, 0, 0};   /* gradient on q' */
    double dqh[4] = {0, 0, 0, 0};   /* gradient on normalised q */
    double dRp[9] = {0}, dRh[9] = {0};

    /* opacity = sigmoid(logit) */
    if (out->d_opacity_logits) out->d_opacity_logits[i] += dop * o->opacity * (1.0 - o->opacity);

    /* colour = max(0, sum sh * Y(dloc) + 0.5) */
    double gch[3];
    for (int ch = 0; ch < 3; ch++) gch[ch] = o->rgb_raw[ch] > 0 ? drgb[ch] : 0.0;
    double ddloc[3] = {0, 0, 0};
    for (int k = 0; k < K; k++)
        for (int ch = 0; ch < 3; ch++) {
            if (out->d_sh) out->d_sh[(int64_t)i * K * 3 + 3 * k + ch] += gch[ch] * o->Y[k];
            for (int r = 0; r < 3; r++) ddloc[r] += gch[ch] * (double)sh[3 * k + ch] * o->dY[3 * k + r];
        }
    /* dloc = Mloc dir */
    double ddir[3] = {0, 0, 0}, dMloc[9];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) {
            dMloc[3 * r + k] = ddloc[r] * o->dir[k];
            ddir[k] += o->Mloc[3 * r + k] * ddloc[r];
        }
    if (o->has_dq) {
        /* Mloc = Rh Rp^T: dRh = dMloc Rp ; dRp = dMloc^T Rh */
        double t1[9], dMT[9];
        mat3_mul(dMloc, o->Rp, t1);
        for (int k = 0; k < 9; k++) dRh[k] += t1[k];
        mat3_transpose(dMloc, dMT);
        mat3_mul(dMT, o->Rh, t1);
        for (int k = 0; k < 9; k++) dRp[k] += t1[k];
    }
    /* dir = w / |w|, w = m - cam_pos */
    double dd = ddir[0] * o->dir[0] + ddir[1] * o->dir[1] + ddir[2] * o->dir[2];
    for (int k = 0; k < 3; k++) dm[k] += (ddir[k] - o->dir[k] * dd) / o->wnorm;

    /* conic = inverse of [[a, b], [b, c]] stored as (A, B, C) */
    double a = o->a, b = o->b, cc = o->c, det = o->det, det2 = det * det;
    double dA = dcon[0], dB = dcon[1], dC = dcon[2];
    double da = dA * (-cc * cc / det2) + dB * (b * cc / det2) + dC * (1.0 / det - a * cc / det2);
    double db = dA * (2.0 * b * cc / det2) + dB * (-1.0 / det - 2.0 * b * b / det2) + dC * (2.0 * a * b / det2);
    double dc = dA * (1.0 / det - a * cc / det2) + dB * (a * b / det2) + dC * (-a * a / det2);
    /* Sigma2 = T Sigma T^T (+0.3 I): symmetric gradient G2 */
    double G2[4] = {da, 0.5 * db, 0.5 * db, dc};
    double dSig[9], dT[6];
    for (int p = 0; p < 3; p++)
        for (int qq = 0; qq < 3; qq++) {
            double acc = 0;
            for (int r = 0; r < 2; r++)
                for (int k = 0; k < 2; k++) acc += o->T[3 * r + p] * G2[2 * r + k] * o->T[3 * k + qq];
            dSig[3 * p + qq] = acc;
        }
    for (int r = 0; r < 2; r++)
        for (int p = 0; p < 3; p++) {
            double acc = 0;
            for (int k = 0; k < 2; k++)
                for (int qq = 0; qq < 3; qq++) acc += G2[2 * r + k] * o->T[3 * k + qq] * o->Sig[3 * qq + p];
            dT[3 * r + p] = 2.0 * acc;
        }
    /* T = J Wrot */
    double dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
    for (int k = 0; k < 3; k++) {
        dJ00 += dT[k] * W[k];
        dJ02 += dT[k] * W[8 + k];
        dJ11 += dT[3 + k] * W[4 + k];
        dJ12 += dT[3 + k] * W[8 + k];
    }
    double tx = o->t[0], ty = o->t[1], tz = o->t[2];
    double txc = o->clamp_x ? (o->txz < 0 ? -1.3 * 0.5 * c->width / fx : 1.3 * 0.5 * c->width / fx) : o->txz;
    double tyc = o->clamp_y ? (o->tyz < 0 ? -1.3 * 0.5 * c->height / fy : 1.3 * 0.5 * c->height / fy) : o->tyz;
    double dt[3] = {0, 0, 0};
    dt[2] += dJ00 * (-fx / (tz * tz)) + dJ11 * (-fy / (tz * tz));
    dt[2] += dJ02 * (fx * txc / (tz * tz)) + dJ12 * (fy * tyc / (tz * tz));
    double dtxc = dJ02 * (-fx / tz), dtyc = dJ12 * (-fy / tz);
    if (!o->clamp_x) { dt[0] += dtxc / tz; dt[2] += -dtxc * tx / (tz * tz); }
    if (!o->clamp_y) { dt[1] += dtyc / tz; dt[2] += -dtyc * ty / (tz * tz); }
    /* u = fx tx/tz + cx, v = fy ty/tz + cy */
    dt[0] += duv[0] * fx / tz;
    dt[1] += duv[1] * fy / tz;
    dt[2] += -duv[0] * fx * tx / (tz * tz) - duv[1] * fy * ty / (tz * tz);
    for (int k = 0; k < 3; k++) dm[k] += W[k] * dt[0] + W[4 + k] * dt[1] + W[8 + k] * dt[2];

    /* Sigma = M M^T, M = Rp diag(s) */
    double M[9], dM[9];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) M[3 * r + k] = o->Rp[3 * r + k] * o->s[k];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) {
            double acc = 0;
            for (int j = 0; j < 3; j++) acc += (dSig[3 * r + j] + dSig[3 * j + r]) * M[3 * j + k];
            dM[3 * r + k] = acc;
        }
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) dRp[3 * r + k] += dM[3 * r + k] * o->s[k];
    for (int k = 0; k < 3; k++) {
        double ds = 0;
        for (int r = 0; r < 3; r++) ds += dM[3 * r + k] * o->Rp[3 * r + k];
        if (out->d_log_scales) out->d_log_scales[3 * i + k] += ds * o->s[k];
    }
    /* rotation matrices -> quaternions */
    quat_rot_adj(o->qp, dRp, dqp);
    quat_rot_adj(o->qh, dRh, dqh);
    if (o->has_dq) {
        /* q' = qh (x) dh: bilinear */
        const double* bq = o->dh;
        const double* aq = o->qh;
        double Rb[16] = {bq[0], -bq[1], -bq[2], -bq[3],
                         bq[1], bq[0], bq[3], -bq[2],
                         bq[2], -bq[3], bq[0], bq[1],
                         bq[3], bq[2], -bq[1], bq[0]};
        double La[16] = {aq[0], -aq[1], -aq[2], -aq[3],
                         aq[1], aq[0], -aq[3], aq[2],
                         aq[2], aq[3], aq[0], -aq[1],
                         aq[3], -aq[2], aq[1], aq[0]};
        double ddh[4] = {0, 0, 0, 0};
        for (int r = 0; r < 4; r++)
            for (int k = 0; k < 4; k++) {
                dqh[k] += Rb[4 * r + k] * dqp[r];
                ddh[k] += La[4 * r + k] * dqp[r];
            }
        /* dh = dq / max(|dq|, 1e-12) */
        if (out->d_dq) {
            if (o->dq_norm > 1e-12) {
                double p = 0;
                for (int k = 0; k < 4; k++) p += o->dh[k] * ddh[k];
                for (int k = 0; k < 4; k++) out->d_dq[4 * i + k] += (ddh[k] - o->dh[k] * p) / o->dq_norm;
            } else {
                for (int k = 0; k < 4; k++) out->d_dq[4 * i + k] += ddh[k] / 1e-12;
            }
        }
    } else {
        for (int k = 0; k < 4; k++) dqh[k] += dqp[k];
    }
    if (out->d_quats && o->q_in_norm > 0) {
        double p = 0;
        for (int k = 0; k < 4; k++) p += o->qh[k] * dqh[k];
        for (int k = 0; k < 4; k++) out->d_quats[4 * i + k] += (dqh[k] - o->qh[k] * p) / o->q_in_norm;
    }
    for (int k = 0; k < 3; k++) {
        if (out->d_means) out->d_means[3 * i + k] += dm[k];
        if (out->d_dmu) out->d_dmu[3 * i + k] += dm[k];
    }
}

/* ------------------------------------------------------------------------ */
/* Ordering and per-pixel candidate lists                                    */
/* ------------------------------------------------------------------------ */

typedef struct { uint32_t key; int64_t id; } kid_t;

static int cmp_kid(const void* pa, const void* pb) {
    const kid_t* a = pa;
    const kid_t* b = pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

typedef struct {
    int64_t n;
    spec_t* sp;
    g64_t* gp;
    int64_t* order;       /* visible ids sorted by (key, id) */
    int64_t nvis;
    int64_t* row_start;   /* H+1 */
    int64_t* row_ids;     /* per row: ids in depth order whose box covers the row */
} scene_t;

static void scene_free(scene_t* s) {
    free(s->sp); free(s->gp); free(s->order); free(s->row_start); free(s->row_ids);
}

static int scene_build(const orc_gaussians* g, const orc_camera* c, scene_t* s) {
    memset(s, 0, sizeof(*s));
    s->n = g->n;
    s->sp = calloc((size_t)(g->n > 0 ? g->n : 1), sizeof(spec_t));
    s->gp = calloc((size_t)(g->n > 0 ? g->n : 1), sizeof(g64_t));
    if (!s->sp || !s->gp) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->n; i++) {
        spec_preprocess(g, c, i, 16, &s->sp[i]);
        if (s->sp[i].visible) pre64(g, c, i, &s->gp[i]);
    }
    int64_t nvis = 0;
    for (int64_t i = 0; i < g->n; i++) nvis += s->sp[i].visible;
    kid_t* tmp = malloc((size_t)(nvis > 0 ? nvis : 1) * sizeof(kid_t));
    s->order = malloc((size_t)(nvis > 0 ? nvis : 1) * sizeof(int64_t));
    if (!tmp || !s->order) { free(tmp); return -2; }
    int64_t j = 0;
    for (int64_t i = 0; i < g->n; i++)
        if (s->sp[i].visible) { tmp[j].key = s->sp[i].key; tmp[j].id = i; j++; }
    qsort(tmp, (size_t)nvis, sizeof(kid_t), cmp_kid);
    for (int64_t k = 0; k < nvis; k++) s->order[k] = tmp[k].id;
    free(tmp);
    s->nvis = nvis;
    int H = c->height;
    s->row_start = calloc((size_t)H + 1, sizeof(int64_t));
    if (!s->row_start) return -2;
    for (int64_t k = 0; k < nvis; k++) {
        const spec_t* p = &s->sp[s->order[k]];
        for (int y = p->box[1]; y <= p->box[3]; y++) s->row_start[y + 1]++;
    }
    for (int y = 0; y < H; y++) s->row_start[y + 1] += s->row_start[y];
    s->row_ids = malloc((size_t)(s->row_start[H] > 0 ? s->row_start[H] : 1) * sizeof(int64_t));
    int64_t* fill = malloc((size_t)H * sizeof(int64_t) + 1);
    if (!s->row_ids || !fill) { free(fill); return -2; }
    for (int y = 0; y < H; y++) fill[y] = s->row_start[y];
    for (int64_t k = 0; k < nvis; k++) {
        int64_t id = s->order[k];
        const spec_t* p = &s->sp[id];
        for (int y = p->box[1]; y <= p->box[3]; y++) s->row_ids[fill[y]++] = id;
    }
    free(fill);
    return 0;
}

/* one contributor of a pixel's front-to-back walk */
typedef struct { int64_t id; double alpha, raw, G, T, dx, dy; } contrib_t;

/* Walk the candidates of pixel (x, y) (Eq. 4).  Returns the number of
 * contributors; fills list[] when list != NULL (capacity cap).  Which
 * Gaussians contribute is decided in single precision (spec_contributes);
 * their weights are double.  Two decisions still depend on values each side
 * computes in its own precision; *ambig gets bit 0 when the 0.99 clamp of
 * alpha is within reach of going the other way, bit 1 when the
 * transmittance cut-off is, and bit 2 when a second cut-off decision of the
 * same walk is.  The margins follow from the difference between the single-
 * and double-precision exponents (which moves alpha by the same relative
 * amount), the error of a hardware exponential (taken as 2e-6 relative) and
 * rounding of the transmittance product.  *stop_k receives the candidate
 * position of the first cut-off decision within reach (-1 if none); the
 * walk takes the other outcome of the cut-off at candidate position flip_k
 * (-1: none), which gives the pixel's alternative value. */
static int64_t walk_pixel(const scene_t* s, int x, int y, double* T_out, double col[3],
                          contrib_t* list, int64_t cap, int* ambig, int64_t flip_k, int64_t* stop_k) {
    double T = 1.0;
    double relT = 0.0;   /* bound on the relative error of a single-precision T */
    col[0] = col[1] = col[2] = 0;
    int64_t n = 0;
    *ambig = 0;
    if (stop_k) *stop_k = -1;
    for (int64_t k = s->row_start[y]; k < s->row_start[y + 1]; k++) {
        int64_t id = s->row_ids[k];
        const spec_t* p = &s->sp[id];
        if (x < p->box[0] || x > p->box[2]) continue;
        float power32;
        if (!spec_contributes(p, x, y, &power32)) continue;
        const g64_t* q = &s->gp[id];
        double dx = (double)x - q->u, dy = (double)y - q->v;
        double power = -0.5 * (q->A * dx * dx + q->C * dy * dy) - q->B * dx * dy;
        double G = exp(power);
        double raw = q->opacity * G;
        double alpha = raw < 0.99 ? raw : 0.99;
        double e = fabs((double)power32 - power) + fabs((double)p->opacity - q->opacity) / q->opacity + 2e-6;
        if (fabs(raw - 0.99) < 2.0 * e * 0.99) *ambig |= 1;
        double Tn = T * (1.0 - alpha);
        relT += (raw < 0.99 ? alpha / (1.0 - alpha) : 0.0) * e + 3.0e-7;
        if (fabs(Tn - 1e-4) < 2.0 * relT * 1e-4 + 1e-9) {
            if (*ambig & 2) *ambig |= 4;
            *ambig |= 2;
            if (stop_k && *stop_k < 0) *stop_k = k;
        }
        int stop = Tn < 1e-4;
        if (k == flip_k) stop = !stop;
        if (stop) break;
        for (int ch = 0; ch < 3; ch++) col[ch] += alpha * T * q->rgb[ch];
        if (list && n < cap) {
            list[n].id = id; list[n].alpha = alpha; list[n].raw = raw; list[n].G = G;
            list[n].T = T; list[n].dx = dx; list[n].dy = dy;
        }
        n++;
        T = Tn;
    }
    *T_out = T;
    return n;
}

/* ------------------------------------------------------------------------ */
/* Exported calls                                                            */
/* ------------------------------------------------------------------------ */

/* Per-Gaussian decisions and double-precision 2D quantities.  Any output may
 * be NULL.  box/rect are n x 4 (x0, y0, x1, y1); invisible Gaussians get
 * visible[i] = 0 and zero elsewhere. */
int orc_preprocess(const orc_gaussians* g, const orc_camera* c, int tile,
                   uint8_t* visible, uint32_t* key, int32_t* box, int32_t* rect, int64_t* ntiles,
                   double* uv, double* conic, double* opacity, double* rgb, double* depth) {
    if (!g || !c || tile <= 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->n; i++) {
        spec_t sp;
        spec_preprocess(g, c, i, tile, &sp);
        if (visible) visible[i] = (uint8_t)sp.visible;
        if (key) key[i] = sp.visible ? sp.key : 0;
        for (int k = 0; k < 4; k++) {
            if (box) box[4 * i + k] = sp.visible ? sp.box[k] : 0;
            if (rect) rect[4 * i + k] = sp.visible ? sp.rect[k] : 0;
        }
        if (ntiles) ntiles[i] = sp.ntiles;
        g64_t q;
        if (sp.visible) pre64(g, c, i, &q);
        else memset(&q, 0, sizeof(q));
        if (uv) { uv[2 * i] = q.u; uv[2 * i + 1] = q.v; }
        if (conic) { conic[3 * i] = q.A; conic[3 * i + 1] = q.B; conic[3 * i + 2] = q.C; }
        if (opacity) opacity[i] = q.opacity;
        if (rgb) for (int k = 0; k < 3; k++) rgb[3 * i + k] = q.rgb[k];
        if (depth) depth[i] = q.t[2];
    }
    return 0;
}

typedef struct { uint32_t tile; uint32_t key; uint32_t id; } pair_t;

static int cmp_pair(const void* pa, const void* pb) {
    const pair_t* a = pa;
    const pair_t* b = pb;
    if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

/* Sorted (tile, depth, id) pairs: keys = tile << 32 | depth bits, vals = id,
 * ranges[2 t], ranges[2 t + 1] = [start, end) of tile t (tiles numbered
 * row-major, ceil(W/tile) per row).  Writes min(K, cap) pairs; returns K,
 * or a negative value on error. */
int64_t orc_sorted_pairs(const orc_gaussians* g, const orc_camera* c, int tile,
                         uint64_t* keys, uint32_t* vals, int64_t cap, uint32_t* ranges) {
    if (!g || !c || tile <= 0) return -1;
    int tw = (c->width + tile - 1) / tile, th = (c->height + tile - 1) / tile;
    spec_t* sp = malloc((size_t)(g->n > 0 ? g->n : 1) * sizeof(spec_t));
    if (!sp) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->n; i++) spec_preprocess(g, c, i, tile, &sp[i]);
    int64_t K = 0;
    for (int64_t i = 0; i < g->n; i++) K += sp[i].visible ? sp[i].ntiles : 0;
    pair_t* pr = malloc((size_t)(K > 0 ? K : 1) * sizeof(pair_t));
    if (!pr) { free(sp); return -2; }
    int64_t j = 0;
    for (int64_t i = 0; i < g->n; i++) {
        if (!sp[i].visible) continue;
        for (int ty = sp[i].rect[1]; ty <= sp[i].rect[3]; ty++)
            for (int tx = sp[i].rect[0]; tx <= sp[i].rect[2]; tx++) {
                pr[j].tile = (uint32_t)(ty * tw + tx);
                pr[j].key = sp[i].key;
                pr[j].id = (uint32_t)i;
                j++;
            }
    }
    qsort(pr, (size_t)K, sizeof(pair_t), cmp_pair);
    for (int64_t k = 0; k < K && k < cap; k++) {
        if (keys) keys[k] = ((uint64_t)pr[k].tile << 32) | pr[k].key;
        if (vals) vals[k] = pr[k].id;
    }
    if (ranges) {
        memset(ranges, 0, sizeof(uint32_t) * 2 * (size_t)tw * th);
        for (int64_t k = 0; k < K; k++) {
            uint32_t t = pr[k].tile;
            if (k == 0 || pr[k - 1].tile != t) ranges[2 * t] = (uint32_t)k;
            if (k == K - 1 || pr[k + 1].tile != t) ranges[2 * t + 1] = (uint32_t)(k + 1);
        }
    }
    free(pr);
    free(sp);
    return K;
}

/* Forward render: image 3 x H x W (planar), final transmittance H x W,
 * contributor count H x W, ambiguity flags H x W (bits as in walk_pixel).
 * image_alt / T_alt hold, where the transmittance cut-off is within reach of
 * going the other way (bit 1), the pixel rendered with the other outcome of
 * that decision, and the primary value elsewhere; when the alternative walk
 * meets a further cut-off decision within reach, bit 2 is set (the two
 * values do not cover every outcome).  Any output may be NULL. */
int orc_render(const orc_gaussians* g, const orc_camera* c, double* image, double* T_final,
               int32_t* n_contrib, uint8_t* ambiguous, double* image_alt, double* T_alt) {
    if (!g || !c || c->width <= 0 || c->height <= 0) return -1;
    scene_t s;
    int rc = scene_build(g, c, &s);
    if (rc) { scene_free(&s); return rc; }
    int Wd = c->width, H = c->height;
    int64_t P = (int64_t)Wd * H;
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < Wd; x++) {
            double T, col[3];
            int amb;
            int64_t stop_k;
            int64_t n = walk_pixel(&s, x, y, &T, col, NULL, 0, &amb, -1, &stop_k);
            int64_t p = (int64_t)y * Wd + x;
            double Ta = T, cola[3] = {col[0], col[1], col[2]};
            if ((amb & 2) && (image_alt || T_alt)) {
                int amb2;
                walk_pixel(&s, x, y, &Ta, cola, NULL, 0, &amb2, stop_k, NULL);
                if (amb2 & 4) amb |= 4;
            }
            for (int ch = 0; ch < 3; ch++) {
                if (image) image[ch * P + p] = col[ch] + T * (double)c->bg[ch];
                if (image_alt) image_alt[ch * P + p] = cola[ch] + Ta * (double)c->bg[ch];
            }
            if (T_final) T_final[p] = T;
            if (T_alt) T_alt[p] = Ta;
            if (n_contrib) n_contrib[p] = (int32_t)n;
            if (ambiguous) ambiguous[p] = (uint8_t)amb;
        }
    }
    scene_free(&s);
    return 0;
}

/* Adjoint of orc_render for dL/dimage (3 x H x W).  Gradients accumulate
 * into the caller's zeroed double arrays; ambiguous pixels, when the mask is
 * given, are reported through touched[i] = 1 for every Gaussian they reach. */
int orc_render_backward(const orc_gaussians* g, const orc_camera* c, const double* dl_dimg,
                        const orc_grads* out, uint8_t* touched_ambiguous) {
    if (!g || !c || !dl_dimg || !out) return -1;
    scene_t s;
    int rc = scene_build(g, c, &s);
    if (rc) { scene_free(&s); return rc; }
    int Wd = c->width, H = c->height;
    int64_t P = (int64_t)Wd * H, n = g->n;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    /* per-thread accumulators: du, dv, dA, dB, dC, dop, dr, dg, db */
    double* acc = calloc((size_t)nthr * (size_t)(n > 0 ? n : 1) * 9, sizeof(double));
    if (!acc) { scene_free(&s); return -2; }
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* A = acc + (size_t)tid * (size_t)n * 9;
        int64_t cap = 1024;
        contrib_t* list = malloc((size_t)cap * sizeof(contrib_t));
#pragma omp for schedule(dynamic, 1)
        for (int y = 0; y < H; y++) {
            for (int x = 0; x < Wd; x++) {
                double T, col[3];
                int amb;
                int64_t cnt = walk_pixel(&s, x, y, &T, col, list, cap, &amb, -1, NULL);
                if (cnt > cap) {
                    free(list);
                    cap = cnt;
                    list = malloc((size_t)cap * sizeof(contrib_t));
                    walk_pixel(&s, x, y, &T, col, list, cap, &amb, -1, NULL);
                }
                int64_t p = (int64_t)y * Wd + x;
                double gc[3] = {dl_dimg[p], dl_dimg[P + p], dl_dimg[2 * P + p]};
                double behind[3] = {c->bg[0], c->bg[1], c->bg[2]};
                for (int64_t j = cnt - 1; j >= 0; j--) {
                    const contrib_t* e = &list[j];
                    const g64_t* q = &s.gp[e->id];
                    double* a = A + 9 * e->id;
                    double dalpha = 0;
                    for (int ch = 0; ch < 3; ch++) {
                        a[6 + ch] += gc[ch] * e->alpha * e->T;
                        dalpha += gc[ch] * e->T * (q->rgb[ch] - behind[ch]);
                    }
                    for (int ch = 0; ch < 3; ch++) behind[ch] = e->alpha * q->rgb[ch] + (1.0 - e->alpha) * behind[ch];
                    if (e->raw < 0.99) {
                        a[5] += dalpha * e->G;
                        double dp = dalpha * e->raw;
                        a[0] += dp * (q->A * e->dx + q->B * e->dy);
                        a[1] += dp * (q->B * e->dx + q->C * e->dy);
                        a[2] += dp * (-0.5 * e->dx * e->dx);
                        a[3] += dp * (-e->dx * e->dy);
                        a[4] += dp * (-0.5 * e->dy * e->dy);
                    }
                    if (amb && touched_ambiguous) touched_ambiguous[e->id] = 1;
                }
            }
        }
        free(list);
    }
    for (int t = 1; t < nthr; t++)
        for (int64_t k = 0; k < n * 9; k++) acc[k] += acc[(size_t)t * (size_t)n * 9 + (size_t)k];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        if (!s.sp[i].visible) continue;
        const double* a = acc + 9 * i;
        if (out->d_uv) { out->d_uv[2 * i] += a[0]; out->d_uv[2 * i + 1] += a[1]; }
        if (out->d_conic) for (int k = 0; k < 3; k++) out->d_conic[3 * i + k] += a[2 + k];
        if (out->d_opacity) out->d_opacity[i] += a[5];
        if (out->d_rgb) for (int k = 0; k < 3; k++) out->d_rgb[3 * i + k] += a[6 + k];
        pre64_adj(g, c, i, &s.gp[i], a, a + 2, a[5], a + 6, out);
    }
    free(acc);
    scene_free(&s);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Hooks for the oracle's own pins                                           */
/* ------------------------------------------------------------------------ */

void orc_quat_mul(const double* a, const double* b, double* p) { quat_mul(a, b, p); }
void orc_quat_rot(const double* q, double* R) { quat_rot(q, R); }
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
