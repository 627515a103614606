// Device-side building blocks shared by the gs3 kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs3 {

constexpr int kTile = 16;
constexpr int kBlendThreads = kTile * kTile;   // one thread per pixel of a tile

// Camera constants passed by value to kernels.
struct CamDev {
    int W, H, tiles_x, tiles_y;
    float fx, fy, cx, cy, near_z;
    float R[9];     // world_to_cam rotation, row-major
    float t[3];     // world_to_cam translation
    float cpos[3];  // camera centre
    float bg[3];
};

// Gaussian inputs of one render.
struct GaussDev {
    const float* means;
    const float* quats;
    const float* log_scales;
    const float* opac;
    const float* sh;
    const float* dmu;   // may be null
    const float* dq;    // may be null
    int64_t n;
    int sh_degree;
};

// Blend record of one Gaussian, three 16-byte words:
//   w0 = (u, v, A, B), w1 = (C, opacity, r, g), w2 = (b, box x0|y0<<16, box x1|y1<<16, ln(1/(255 opacity)))
// with the conic stored so that power = -(A dx^2 + C dy^2)/2 - B dx dy.

// exp used for the scale activation.  It is part of the single-precision
// decision procedure (the 3-sigma radius depends on it), so its result is
// fixed bit for bit: Cody-Waite reduction x = k ln2 + r with ln2 split into
// a 16-bit head and a tail, degree-7 Taylor polynomial of e^r by Horner's
// rule, then scaling by 2^k.
__device__ __forceinline__ float spec_exp(float x) {
#pragma clang fp contract(off)
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

// Forward geometry of one Gaussian in single precision.  Every quantity
// that feeds a discrete decision (view depth, 2D covariance, radius, pixel
// box) is evaluated with a fixed operation order and no contraction; the
// same values are then used as the continuous forward values.
struct Geo {
    float m[3];          // translated mean
    float t[3];          // camera-space mean
    float qn;            // |q|
    float qh[4];         // q / |q|
    float dn;            // max(|dq|, 1e-12)
    float dh[4];         // dq / dn
    float qp[4];         // q' = qh (x) dh
    float Rp[9];         // R(q')
    float s[3];          // exp(log-scale)
    float S00, S01, S02, S11, S12, S22;   // 3D covariance
    float txz, tyz;      // t_x / t_z, t_y / t_z
    float txc, tyc;      // clamped for J
    bool clx, cly;       // clamp active
    float j00, j02, j11, j12;
    float T00, T01, T02, T10, T11, T12;   // J W
    float a, b, c, det;  // 2D covariance (+0.3 I) and its determinant
    float u, v, r;       // image-space mean and 3-sigma radius (pixels)
    int x0, y0, x1, y1;  // inclusive pixel box
};

// Returns false when the Gaussian is culled.
__device__ __forceinline__ bool geo_forward(const GaussDev& g, const CamDev& cam, int64_t i, Geo& o) {
#pragma clang fp contract(off)
    const float* R = cam.R;
    float m0 = g.means[3 * i + 0], m1 = g.means[3 * i + 1], m2 = g.means[3 * i + 2];
    if (g.dmu) {
        m0 = m0 + g.dmu[3 * i + 0];
        m1 = m1 + g.dmu[3 * i + 1];
        m2 = m2 + g.dmu[3 * i + 2];
    }
    o.m[0] = m0; o.m[1] = m1; o.m[2] = m2;
    float tx = ((R[0] * m0 + R[1] * m1) + R[2] * m2) + cam.t[0];
    float ty = ((R[3] * m0 + R[4] * m1) + R[5] * m2) + cam.t[1];
    float tz = ((R[6] * m0 + R[7] * m1) + R[8] * m2) + cam.t[2];
    o.t[0] = tx; o.t[1] = ty; o.t[2] = tz;
    if (!(tz > cam.near_z)) return false;

    float q0 = g.quats[4 * i + 0], q1 = g.quats[4 * i + 1], q2 = g.quats[4 * i + 2], q3 = g.quats[4 * i + 3];
    float qn = sqrtf(((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3);
    o.qn = qn;
    float aw = 1.0f, ax = 0.0f, ay = 0.0f, az = 0.0f;
    if (qn > 0.0f) { aw = q0 / qn; ax = q1 / qn; ay = q2 / qn; az = q3 / qn; }
    o.qh[0] = aw; o.qh[1] = ax; o.qh[2] = ay; o.qh[3] = az;
    float w = aw, x = ax, y = ay, z = az;
    if (g.dq) {
        float d0 = g.dq[4 * i + 0], d1 = g.dq[4 * i + 1], d2 = g.dq[4 * i + 2], d3 = g.dq[4 * i + 3];
        float dn = sqrtf(((d0 * d0 + d1 * d1) + d2 * d2) + d3 * d3);
        dn = fmaxf(dn, 1e-12f);
        float bw = d0 / dn, bx = d1 / dn, by = d2 / dn, bz = d3 / dn;
        o.dn = dn;
        o.dh[0] = bw; o.dh[1] = bx; o.dh[2] = by; o.dh[3] = bz;
        w = ((aw * bw - ax * bx) - ay * by) - az * bz;
        x = ((aw * bx + ax * bw) + ay * bz) - az * by;
        y = ((aw * by - ax * bz) + ay * bw) + az * bx;
        z = ((aw * bz + ax * by) - ay * bx) + az * bw;
    }
    o.qp[0] = w; o.qp[1] = x; o.qp[2] = y; o.qp[3] = z;
    float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
    float wx = w * x, wy = w * y, wz = w * z;
    float r00 = 1.0f - 2.0f * (yy + zz), r01 = 2.0f * (xy - wz), r02 = 2.0f * (xz + wy);
    float r10 = 2.0f * (xy + wz), r11 = 1.0f - 2.0f * (xx + zz), r12 = 2.0f * (yz - wx);
    float r20 = 2.0f * (xz - wy), r21 = 2.0f * (yz + wx), r22 = 1.0f - 2.0f * (xx + yy);
    o.Rp[0] = r00; o.Rp[1] = r01; o.Rp[2] = r02;
    o.Rp[3] = r10; o.Rp[4] = r11; o.Rp[5] = r12;
    o.Rp[6] = r20; o.Rp[7] = r21; o.Rp[8] = r22;
    float s0 = spec_exp(g.log_scales[3 * i + 0]);
    float s1 = spec_exp(g.log_scales[3 * i + 1]);
    float s2 = spec_exp(g.log_scales[3 * i + 2]);
    o.s[0] = s0; o.s[1] = s1; o.s[2] = s2;
    float M00 = r00 * s0, M01 = r01 * s1, M02 = r02 * s2;
    float M10 = r10 * s0, M11 = r11 * s1, M12 = r12 * s2;
    float M20 = r20 * s0, M21 = r21 * s1, M22 = r22 * s2;
    o.S00 = (M00 * M00 + M01 * M01) + M02 * M02;
    o.S01 = (M00 * M10 + M01 * M11) + M02 * M12;
    o.S02 = (M00 * M20 + M01 * M21) + M02 * M22;
    o.S11 = (M10 * M10 + M11 * M11) + M12 * M12;
    o.S12 = (M10 * M20 + M11 * M21) + M12 * M22;
    o.S22 = (M20 * M20 + M21 * M21) + M22 * M22;

    float limx = (1.3f * (0.5f * (float)cam.W)) / cam.fx;
    float limy = (1.3f * (0.5f * (float)cam.H)) / cam.fy;
    float txz = tx / tz, tyz = ty / tz;
    o.txz = txz; o.tyz = tyz;
    float txc = fminf(fmaxf(txz, -limx), limx);
    float tyc = fminf(fmaxf(tyz, -limy), limy);
    o.txc = txc; o.tyc = tyc;
    o.clx = (txz < -limx) || (txz > limx);
    o.cly = (tyz < -limy) || (tyz > limy);
    float j00 = cam.fx / tz, j02 = -(cam.fx * txc) / tz;
    float j11 = cam.fy / tz, j12 = -(cam.fy * tyc) / tz;
    o.j00 = j00; o.j02 = j02; o.j11 = j11; o.j12 = j12;
    float T00 = j00 * R[0] + j02 * R[6], T01 = j00 * R[1] + j02 * R[7], T02 = j00 * R[2] + j02 * R[8];
    float T10 = j11 * R[3] + j12 * R[6], T11 = j11 * R[4] + j12 * R[7], T12 = j11 * R[5] + j12 * R[8];
    o.T00 = T00; o.T01 = T01; o.T02 = T02; o.T10 = T10; o.T11 = T11; o.T12 = T12;
    float U00 = (T00 * o.S00 + T01 * o.S01) + T02 * o.S02;
    float U01 = (T00 * o.S01 + T01 * o.S11) + T02 * o.S12;
    float U02 = (T00 * o.S02 + T01 * o.S12) + T02 * o.S22;
    float U10 = (T10 * o.S00 + T11 * o.S01) + T12 * o.S02;
    float U11 = (T10 * o.S01 + T11 * o.S11) + T12 * o.S12;
    float U12 = (T10 * o.S02 + T11 * o.S12) + T12 * o.S22;
    float a = ((U00 * T00 + U01 * T01) + U02 * T02) + 0.3f;
    float b = (U00 * T10 + U01 * T11) + U02 * T12;
    float c = ((U10 * T10 + U11 * T11) + U12 * T12) + 0.3f;
    float det = a * c - b * b;
    o.a = a; o.b = b; o.c = c; o.det = det;
    if (!(det > 0.0f)) return false;
    float mid = 0.5f * (a + c);
    float disc = mid * mid - det;
    float lam = mid + sqrtf(fmaxf(disc, 0.0f));
    float r = ceilf(3.0f * sqrtf(lam));
    float u = cam.fx * txz + cam.cx;
    float v = cam.fy * tyz + cam.cy;
    o.u = u; o.v = v; o.r = r;
    if (!(fabsf(u) <= 1e7f && fabsf(v) <= 1e7f && r <= 1e7f)) return false;
    float x0 = fmaxf(ceilf(u - r), 0.0f), x1 = fminf(floorf(u + r), (float)(cam.W - 1));
    float y0 = fmaxf(ceilf(v - r), 0.0f), y1 = fminf(floorf(v + r), (float)(cam.H - 1));
    if (x0 > x1 || y0 > y1) return false;
    o.x0 = (int)x0; o.y0 = (int)y0; o.x1 = (int)x1; o.y1 = (int)y1;
    return true;
}

// Real orthonormal SH (Condon-Shortley phase), k = l^2 + l + m.
namespace shc {
constexpr float c0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float c1 = 0.4886025119029199f;    // sqrt(3 / (4 pi))
constexpr float c2a = 1.0925484305920792f;   // sqrt(15 / pi) / 2
constexpr float c2b = 0.31539156525252005f;  // sqrt(5 / pi) / 4
constexpr float c2c = 0.5462742152960396f;   // sqrt(15 / pi) / 4
constexpr float c3a = 0.5900435899266435f;   // sqrt(35 / (2 pi)) / 4
constexpr float c3b = 2.890611442640554f;    // sqrt(105 / pi) / 2
constexpr float c3c = 0.4570457994644658f;   // sqrt(21 / (2 pi)) / 4
constexpr float c3d = 0.3731763325901154f;   // sqrt(7 / pi) / 4
constexpr float c3e = 1.445305721320277f;    // sqrt(105 / pi) / 4
}  // namespace shc

template <typename F>
__host__ __device__ __forceinline__ void sh_basis_t(int deg, F x, F y, F z, F Y[16]) {
    using namespace shc;
    Y[0] = (F)c0;
    if (deg < 1) return;
    Y[1] = -(F)c1 * y; Y[2] = (F)c1 * z; Y[3] = -(F)c1 * x;
    if (deg < 2) return;
    const F xx = x * x, yy = y * y, zz = z * z;
    Y[4] = (F)c2a * x * y;
    Y[5] = -(F)c2a * y * z;
    Y[6] = (F)c2b * (2 * zz - xx - yy);
    Y[7] = -(F)c2a * x * z;
    Y[8] = (F)c2c * (xx - yy);
    if (deg < 3) return;
    Y[9] = -(F)c3a * y * (3 * xx - yy);
    Y[10] = (F)c3b * x * y * z;
    Y[11] = -(F)c3c * y * (4 * zz - xx - yy);
    Y[12] = (F)c3d * z * (2 * zz - 3 * xx - 3 * yy);
    Y[13] = -(F)c3c * x * (4 * zz - xx - yy);
    Y[14] = (F)c3e * z * (xx - yy);
    Y[15] = -(F)c3a * x * (xx - 3 * yy);
}

__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float Y[16]) {
    using namespace shc;
    Y[0] = c0;
    if (deg < 1) return;
    Y[1] = -c1 * y; Y[2] = c1 * z; Y[3] = -c1 * x;
    if (deg < 2) return;
    float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c2b * (2.0f * zz - xx - yy);
    Y[7] = -c2a * x * z;
    Y[8] = c2c * (xx - yy);
    if (deg < 3) return;
    Y[9] = -c3a * y * (3.0f * xx - yy);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (4.0f * zz - xx - yy);
    Y[12] = c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -c3c * x * (4.0f * zz - xx - yy);
    Y[14] = c3e * z * (xx - yy);
    Y[15] = -c3a * x * (xx - 3.0f * yy);
}

// sum_k w_k grad Y_k(x, y, z) (gradient with respect to the raw components)
__device__ __forceinline__ void sh_grad(int deg, float x, float y, float z, const float w[16],
                                        float& gx, float& gy, float& gz) {
    using namespace shc;
    gx = 0.0f; gy = 0.0f; gz = 0.0f;
    if (deg < 1) return;
    gy += -c1 * w[1]; gz += c1 * w[2]; gx += -c1 * w[3];
    if (deg < 2) return;
    float xx = x * x, yy = y * y, zz = z * z;
    gx += c2a * y * w[4];               gy += c2a * x * w[4];
    gy += -c2a * z * w[5];              gz += -c2a * y * w[5];
    gx += -2.0f * c2b * x * w[6];       gy += -2.0f * c2b * y * w[6];   gz += 4.0f * c2b * z * w[6];
    gx += -c2a * z * w[7];              gz += -c2a * x * w[7];
    gx += 2.0f * c2c * x * w[8];        gy += -2.0f * c2c * y * w[8];
    if (deg < 3) return;
    gx += -c3a * 6.0f * x * y * w[9];   gy += -c3a * (3.0f * xx - 3.0f * yy) * w[9];
    gx += c3b * y * z * w[10];          gy += c3b * x * z * w[10];      gz += c3b * x * y * w[10];
    gx += 2.0f * c3c * x * y * w[11];   gy += -c3c * (4.0f * zz - xx - 3.0f * yy) * w[11];
    gz += -8.0f * c3c * y * z * w[11];
    gx += -6.0f * c3d * x * z * w[12];  gy += -6.0f * c3d * y * z * w[12];
    gz += c3d * (6.0f * zz - 3.0f * xx - 3.0f * yy) * w[12];
    gx += -c3c * (4.0f * zz - 3.0f * xx - yy) * w[13];
    gy += 2.0f * c3c * x * y * w[13];   gz += -8.0f * c3c * x * z * w[13];
    gx += 2.0f * c3e * x * z * w[14];   gy += -2.0f * c3e * y * z * w[14];  gz += c3e * (xx - yy) * w[14];
    gx += -c3a * (3.0f * xx - 3.0f * yy) * w[15];  gy += 6.0f * c3a * x * y * w[15];
}

// rotation matrix of a unit quaternion (w, x, y, z), row-major
__device__ __forceinline__ void quat_to_rot(const float q[4], float R[9]) {
    float w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0f - 2.0f * (y * y + z * z); R[1] = 2.0f * (x * y - w * z); R[2] = 2.0f * (x * z + w * y);
    R[3] = 2.0f * (x * y + w * z); R[4] = 1.0f - 2.0f * (x * x + z * z); R[5] = 2.0f * (y * z - w * x);
    R[6] = 2.0f * (x * z - w * y); R[7] = 2.0f * (y * z + w * x); R[8] = 1.0f - 2.0f * (x * x + y * y);
}

// Colour of a Gaussian: direction from the camera centre to the translated
// mean, rotated back into the frame of the untransformed Gaussian
// (d_loc = R(qh) R(q')^T d), then max(0, SH(d_loc) + 0.5).
// 0.5 + sum_k Y_k c_k for one Gaussian's K x 3 SH row; rows of 12 or 48
// floats are 16-byte aligned and read as float4 (12 loads instead of 48).
template <int K>
__device__ __forceinline__ void sh_colour(const float* __restrict__ sh, const float Y[16], float raw[3]) {
    float v[3 * K];
    if constexpr ((3 * K) % 4 == 0) {
#pragma unroll
        for (int q = 0; q < 3 * K / 4; q++) {
            const float4 t = reinterpret_cast<const float4*>(sh)[q];
            v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 3 * K; q++) v[q] = sh[q];
    }
    float c0 = 0.5f, c1 = 0.5f, c2 = 0.5f;
#pragma unroll
    for (int k = 0; k < K; k++) {
        c0 += Y[k] * v[3 * k + 0];
        c1 += Y[k] * v[3 * k + 1];
        c2 += Y[k] * v[3 * k + 2];
    }
    raw[0] = c0; raw[1] = c1; raw[2] = c2;
}

// wk_k = sum_c gch_c SH_{k,c} (the colour gradient pulled back onto the
// basis values), with the same row loads as sh_colour.
template <int K>
__device__ __forceinline__ void sh_weights(const float* __restrict__ sh, const float gch[3], float wk[16]) {
    float v[3 * K];
    if constexpr ((3 * K) % 4 == 0) {
#pragma unroll
        for (int q = 0; q < 3 * K / 4; q++) {
            const float4 t = reinterpret_cast<const float4*>(sh)[q];
            v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 3 * K; q++) v[q] = sh[q];
    }
#pragma unroll
    for (int k = 0; k < K; k++) wk[k] = gch[0] * v[3 * k] + gch[1] * v[3 * k + 1] + gch[2] * v[3 * k + 2];
}

struct ColourCtx {
    float dir[3], wn;     // unit direction and |mu' - c|
    float Rh[9];          // R(qh) (only with a rotation delta)
    float Ml[9];          // R(qh) R(q')^T
    float dl[3];          // d_loc
    float raw[3];         // SH + 0.5 before the clamp
};

__device__ __forceinline__ void colour_forward(const GaussDev& g, const CamDev& cam, int64_t i, const Geo& o,
                                               ColourCtx& cc) {
    float w0 = o.m[0] - cam.cpos[0], w1 = o.m[1] - cam.cpos[1], w2 = o.m[2] - cam.cpos[2];
    float wn = sqrtf(w0 * w0 + w1 * w1 + w2 * w2);
    cc.wn = wn;
    float inv = 1.0f / wn;
    cc.dir[0] = w0 * inv; cc.dir[1] = w1 * inv; cc.dir[2] = w2 * inv;
    if (g.dq) {
        quat_to_rot(o.qh, cc.Rh);
        // Ml = Rh Rp^T
        for (int r = 0; r < 3; r++)
            for (int k = 0; k < 3; k++)
                cc.Ml[3 * r + k] = cc.Rh[3 * r + 0] * o.Rp[3 * k + 0] + cc.Rh[3 * r + 1] * o.Rp[3 * k + 1] +
                                   cc.Rh[3 * r + 2] * o.Rp[3 * k + 2];
        for (int r = 0; r < 3; r++)
            cc.dl[r] = cc.Ml[3 * r] * cc.dir[0] + cc.Ml[3 * r + 1] * cc.dir[1] + cc.Ml[3 * r + 2] * cc.dir[2];
    } else {
        cc.dl[0] = cc.dir[0]; cc.dl[1] = cc.dir[1]; cc.dl[2] = cc.dir[2];
    }
    float Y[16];
    sh_basis(g.sh_degree, cc.dl[0], cc.dl[1], cc.dl[2], Y);
    switch (g.sh_degree) {
        case 3: sh_colour<16>(g.sh + i * 48, Y, cc.raw); break;
        case 1: sh_colour<4>(g.sh + i * 12, Y, cc.raw); break;
        case 2: sh_colour<9>(g.sh + i * 27, Y, cc.raw); break;
        default: sh_colour<1>(g.sh + i * 3, Y, cc.raw); break;
    }
}

// alpha of a Gaussian record at pixel (px, py); false when the candidate is
// skipped (power > 0 or alpha < 1/255).  Used identically by the forward and
// backward blend so that both walk the same contributors.
// pthr = ln(1 / (255 opacity)) (record word w2.w): a candidate with power
// below it has alpha < 1/255 and is rejected without the exp; the exact
// alpha test below stays the deciding one for the rest.
// Opacity activation, in the decision procedure's arithmetic (the opacity
// takes part in the contributor decision below).
__device__ __forceinline__ float opacity_of(float logit) {
#pragma clang fp contract(off)
    return 1.0f / (1.0f + spec_exp(-logit));
}

// Contributor test and alpha of one (pixel, Gaussian) evaluation (Eq. 4).
// A Gaussian contributes when its exponent
//     power = -0.5 ((A dx) dx + (C dy) dy) - (B dx) dy
// is <= 0 and opacity * exp(power) >= 1/255, both evaluated in single
// precision in exactly this order and with the decision-procedure
// exponential.  The per-Gaussian threshold pthr = ln(1 / (255 opacity))
// settles every case more than 1e-4 away from it (the exponential and logf
// errors are below 2e-6 there); only the rest evaluate the exact test.  alpha
// itself uses the hardware exponential.  The pixel-column products (A dx) dx
// and B dx are shared by the rows a thread walks (blend_dx_terms).
__device__ __forceinline__ void blend_dx_terms(float dx, const float4& w0, float& adx2, float& bdx) {
#pragma clang fp contract(off)
    adx2 = w0.z * dx * dx;
    bdx = w0.w * dx;
}

// The exponent in the decision procedure's order; the blend loops compare
// it with 0 and with the band edges pthr -/+ 1e-4 themselves.
__device__ __forceinline__ float blend_power(float adx2, float bdx, float dy, float C) {
#pragma clang fp contract(off)
    return -0.5f * (adx2 + C * dy * dy) - bdx * dy;
}

// the exact opacity test, for exponents inside the band
__device__ __forceinline__ bool blend_exact_test(float power, float opacity) {
#pragma clang fp contract(off)
    return opacity * spec_exp(power) >= 1.0f / 255.0f;
}

// bits lo..hi of a 16-bit span, clipped to 0..15 (0 when empty)
__device__ __forceinline__ uint32_t span_mask16(int lo, int hi) {
    lo = lo > 0 ? lo : 0;
    hi = hi < 15 ? hi : 15;
    return lo <= hi ? (0xFFFFu >> (15 - hi + lo)) << lo : 0u;
}

// The LDS form of a record's third quad in the blend loops of the tile whose
// first pixel is (tx0p, ty0p): colour b, the lower and upper edge of the
// exponent band around the opacity threshold (pthr -/+ 1e-4, the same
// single-precision operations the per-pixel test used), and a pixel box as
// a mask of the tile columns (bits 0-15) and rows (bits 16-31) it covers.  A
// pixel at (lx, ly) of the tile is inside the box iff both of its bits
// (1 << lx) | (1 << (16 + ly)) are set.  kTight: the record's pixel box is
// cut to the bounding box of the ellipse where the exponent can reach the
// band's lower edge: with M = [[A, B], [B, C]] (the conic), -power / 2 =
// d^T M d / 2 <= -(pthr - 1e-4) bounds |dx| by sqrt(k (M^-1)_xx) and |dy| by
// sqrt(k (M^-1)_yy), k = -2 (pthr - 1e-4), here widened by 0.1% and a pixel.
// It only drops pixels whose exponent is below the band (their opacity test
// fails), so every pixel that takes the entry is still inside.  The pixel
// margin is worth about 2 k / h of the quadratic form at half-width h; the
// single-precision exponent of a pixel in the record's box can be off by a
// few ulps of 9 cond(M), so the box is only cut where cond(M) h stays well
// below what the margin covers (cond(M) <= (A + C)^2 / det M).
template <bool kTight = true>
__device__ __forceinline__ float4 blend_stage_w2(const float4& w0, const float4& w1, const float4& w2, int tx0p,
                                                 int ty0p) {
    const uint32_t b0 = __float_as_uint(w2.y), b1 = __float_as_uint(w2.z);
    int x0 = (int)(b0 & 0xFFFFu), y0 = (int)(b0 >> 16), x1 = (int)(b1 & 0xFFFFu), y1 = (int)(b1 >> 16);
    const float A = w0.z, B = w0.w, C = w1.x;
    const float k = fmaxf(-2.0f * (w2.w - 1e-4f), 0.0f) * 1.001f;
    const float det = A * C - B * B;
    const float hx = sqrtf(k * C / det) + 1.0f, hy = sqrtf(k * A / det) + 1.0f;
    const float cond = (A + C) * (A + C) / det;
    if (kTight && det > 0.0f && hx <= 1e6f && hy <= 1e6f && fabsf(w0.x) <= 1e6f && fabsf(w0.y) <= 1e6f &&
        cond * fmaxf(hx, hy) <= 4e4f * k) {
        x0 = max(x0, (int)floorf(w0.x - hx));
        x1 = min(x1, (int)ceilf(w0.x + hx));
        y0 = max(y0, (int)floorf(w0.y - hy));
        y1 = min(y1, (int)ceilf(w0.y + hy));
    }
    const uint32_t cm = span_mask16(x0 - tx0p, x1 - tx0p);
    const uint32_t rm = span_mask16(y0 - ty0p, y1 - ty0p);
    return make_float4(w2.x, w2.w - 1e-4f, w2.w + 1e-4f, __uint_as_float(cm | (rm << 16)));
}

// Rows of the tile that wave wv of a blend workgroup covers (16 columns x R
// rows per 16 threads), as bits 16-31 of a box mask.
template <int R>
__device__ __forceinline__ uint32_t wave_row_bits(int wv) {
    return (R * 4 >= 16 ? 0xFFFFu : ((1u << (4 * R)) - 1u) << (4 * R * wv)) << 16;
}

// Whether a staged box mask reaches a pixel of the wave's rows.
__device__ __forceinline__ bool box_meets_rows(float w2w, uint32_t rows) {
    const uint32_t m = __float_as_uint(w2w);
    return (m & rows) != 0u && (m & 0xFFFFu) != 0u;
}

// wave64 helpers

template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_add(float x) {
    const int moved = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kCtrl, kRowMask, 0xF, false);
    return x + __builtin_bit_cast(float, moved);
}

// Lane exchanges of gfx950: v_permlane32_swap exchanges the upper 32 lanes
// of its first operand with the lower 32 lanes of its second, so afterwards
// x + y holds, in lanes 0-31, x[l] + x[l + 32] and, in lanes 32-63,
// y[l - 32] + y[l]; v_permlane16_swap does the same between the odd 16-lane
// rows of x and the even rows of y.  Written as inline assembly with both
// operands read and written (the compiler's two-result builtin for these
// instructions dropped the second result); the s_nop keeps the VALU write
// of the operands apart from the exchange.
__device__ __forceinline__ float swap_add32(float x, float y) {
    asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1" : "+v"(x), "+v"(y));
    return x + y;
}

__device__ __forceinline__ float swap_add16(float x, float y) {
    asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1" : "+v"(x), "+v"(y));
    return x + y;
}

// Eight per-lane values -> their eight wave sums, spread over lane groups:
// after the call, every lane of the 8-lane group g (lanes 8g..8g+7) holds
// the total of term g.  Two exchanges halve the set (permlane32: terms 0-3
// stay in the lower half, 4-7 in the upper; permlane16: two terms per 16-lane
// row), a third (^8, DPP row_ror:8) leaves one term per lane, then DPP sums
// the 8-lane group.
__device__ __forceinline__ float wave_reduce_scatter8(const float v[8], int lane) {
    float a[4], b[2], c;
#pragma unroll
    for (int k = 0; k < 4; k++) a[k] = swap_add32(v[k], v[4 + k]);
#pragma unroll
    for (int k = 0; k < 2; k++) b[k] = swap_add16(a[k], a[2 + k]);
    {
        const bool hi8 = lane & 8;
        const float send = hi8 ? b[0] : b[1];
        const float keep = hi8 ? b[1] : b[0];
        const int moved = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, send), 0x128, 0xF, 0xF, false);
        c = keep + __builtin_bit_cast(float, moved);   // row_ror:8 pairs lane i with lane i ^ 8
    }
    c = dpp_add<0xB1, 0xF>(c);    // quad_perm [1,0,3,2]
    c = dpp_add<0x4E, 0xF>(c);    // quad_perm [2,3,0,1]
    c = dpp_add<0x141, 0xF>(c);   // row_half_mirror: the 8-lane group total in every lane
    return c;                     // term index: lane >> 3
}

// The same for two independent sets of eight values (two tile entries):
// the eight permlane32 and four permlane16 exchanges are issued back to
// back after a single wait (the operands were all written before it), and
// the two DPP chains interleave, so their read-after-write waits overlap.
__device__ __forceinline__ void wave_reduce_scatter8x2(const float v[8], const float u[8], int lane, float& rv,
                                                       float& ru) {
    float va[8], ua[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        va[k] = v[k];
        ua[k] = u[k];
    }
    asm volatile(
        "s_nop 1\n\t"
        "v_permlane32_swap_b32 %0, %4\n\t"
        "v_permlane32_swap_b32 %1, %5\n\t"
        "v_permlane32_swap_b32 %2, %6\n\t"
        "v_permlane32_swap_b32 %3, %7\n\t"
        "v_permlane32_swap_b32 %8, %12\n\t"
        "v_permlane32_swap_b32 %9, %13\n\t"
        "v_permlane32_swap_b32 %10, %14\n\t"
        "v_permlane32_swap_b32 %11, %15"
        : "+v"(va[0]), "+v"(va[1]), "+v"(va[2]), "+v"(va[3]), "+v"(va[4]), "+v"(va[5]), "+v"(va[6]), "+v"(va[7]),
          "+v"(ua[0]), "+v"(ua[1]), "+v"(ua[2]), "+v"(ua[3]), "+v"(ua[4]), "+v"(ua[5]), "+v"(ua[6]), "+v"(ua[7]));
    float a[4], b[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        a[k] = va[k] + va[4 + k];
        b[k] = ua[k] + ua[4 + k];
    }
    asm volatile(
        "s_nop 1\n\t"
        "v_permlane16_swap_b32 %0, %2\n\t"
        "v_permlane16_swap_b32 %1, %3\n\t"
        "v_permlane16_swap_b32 %4, %6\n\t"
        "v_permlane16_swap_b32 %5, %7"
        : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(b[0]), "+v"(b[1]), "+v"(b[2]), "+v"(b[3]));
    const float a0 = a[0] + a[2], a1 = a[1] + a[3], b0 = b[0] + b[2], b1 = b[1] + b[3];
    const bool hi8 = lane & 8;
    const int mv = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, hi8 ? a0 : a1), 0x128, 0xF, 0xF, false);
    const int mu = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, hi8 ? b0 : b1), 0x128, 0xF, 0xF, false);
    float c = (hi8 ? a1 : a0) + __builtin_bit_cast(float, mv);
    float d = (hi8 ? b1 : b0) + __builtin_bit_cast(float, mu);
    c = dpp_add<0xB1, 0xF>(c);
    d = dpp_add<0xB1, 0xF>(d);
    c = dpp_add<0x4E, 0xF>(c);
    d = dpp_add<0x4E, 0xF>(d);
    rv = dpp_add<0x141, 0xF>(c);
    ru = dpp_add<0x141, 0xF>(d);
}

// Inclusive prefix sum over the 64 lanes with DPP moves: shifts by 1, 2, 4
// and 8 lanes within each 16-lane row (lanes that would read before the row
// start add nothing), then the last lane of row 0 into row 1 and of row 2
// into row 3 (row_bcast:15), then the last lane of row 1 into rows 2 and 3
// (row_bcast:31).  No LDS traffic, unlike a permute-based scan.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);   // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return x;
}

// The value of lane 63 (a wave-uniform scalar read).
__device__ __forceinline__ uint32_t lane63_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Sum over the 64 lanes with DPP moves (no LDS traffic); the result is
// returned uniformly (read from lane 63).  Steps: pairs and quads
// (quad_perm), 8 and 16 lanes (row_half_mirror, row_mirror), then rows
// (row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3).
__device__ __forceinline__ float wave_sum_dpp(float x) {
    x = dpp_add<0xB1, 0xF>(x);    // quad_perm [1,0,3,2]
    x = dpp_add<0x4E, 0xF>(x);    // quad_perm [2,3,0,1]
    x = dpp_add<0x141, 0xF>(x);   // row_half_mirror
    x = dpp_add<0x140, 0xF>(x);   // row_mirror
    x = dpp_add<0x142, 0xA>(x);   // row_bcast:15
    x = dpp_add<0x143, 0xC>(x);   // row_bcast:31
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 63));
}

}  // namespace gs3
