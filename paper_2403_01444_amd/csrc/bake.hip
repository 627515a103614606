// Per-frame transform bake (Sec. 4.1 "Mean", "Rotation", "SH Coefficients";
// Suppl. Sec. B): the transformed Gaussians written out so the next frame
// starts from them.  mu' = mu + dmu, q' = norm(q) x norm(dq), and each SH band
// l >= 1 turned by M_l(dR), dR = R(q') R(norm q)^T, with
// M_l = [P_l(dR N_0), ..., P_l(dR N_2l)] A_l^{-1}, A_l = [P_l(N_0), ...]: the
// paper's construction (band 1 with N = e_x, e_y, e_z) applied to bands 2-3
// with 2l+1 fixed directions.
#include <math.h>

#include "kernels.h"

namespace gs3 {

namespace {

__global__ __launch_bounds__(128) void k_bake(GaussDev g, ShRotConst rc, float* __restrict__ mu_out,
                                              float* __restrict__ q_out, float* __restrict__ sh_out) {
    const int64_t i = (int64_t)blockIdx.x * 128 + threadIdx.x;
    if (i >= g.n) return;
    for (int k = 0; k < 3; k++) mu_out[3 * i + k] = g.means[3 * i + k] + (g.dmu ? g.dmu[3 * i + k] : 0.f);
    float q[4] = {g.quats[4 * i], g.quats[4 * i + 1], g.quats[4 * i + 2], g.quats[4 * i + 3]};
    const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    float qh[4] = {1.f, 0.f, 0.f, 0.f};
    if (qn > 0.f)
        for (int k = 0; k < 4; k++) qh[k] = q[k] / qn;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    const float* sh = g.sh + i * (int64_t)K * 3;
    float* so = sh_out + i * (int64_t)K * 3;
    if (!g.dq) {
        for (int k = 0; k < 4; k++) q_out[4 * i + k] = qh[k];
        for (int k = 0; k < 3 * K; k++) so[k] = sh[k];
        return;
    }
    const float d0 = g.dq[4 * i], d1 = g.dq[4 * i + 1], d2 = g.dq[4 * i + 2], d3 = g.dq[4 * i + 3];
    const float dn = fmaxf(sqrtf(d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3), 1e-12f);
    const float b[4] = {d0 / dn, d1 / dn, d2 / dn, d3 / dn};
    const float qp[4] = {qh[0] * b[0] - qh[1] * b[1] - qh[2] * b[2] - qh[3] * b[3],
                         qh[0] * b[1] + qh[1] * b[0] + qh[2] * b[3] - qh[3] * b[2],
                         qh[0] * b[2] - qh[1] * b[3] + qh[2] * b[0] + qh[3] * b[1],
                         qh[0] * b[3] + qh[1] * b[2] - qh[2] * b[1] + qh[3] * b[0]};
    for (int k = 0; k < 4; k++) q_out[4 * i + k] = qp[k];
    float Rp[9], Rh[9], dR[9];
    quat_to_rot(qp, Rp);
    quat_to_rot(qh, Rh);
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++)
            dR[3 * r + c] = Rp[3 * r] * Rh[3 * c] + Rp[3 * r + 1] * Rh[3 * c + 1] + Rp[3 * r + 2] * Rh[3 * c + 2];
    for (int k = 0; k < 3; k++) so[k] = sh[k];   // band 0 does not turn
    int dir0 = 0, a0 = 0;
    for (int l = 1; l <= g.sh_degree; l++) {
        const int m = 2 * l + 1, base = l * l;
        float B[7][7];   // B[row = basis function][col = direction]
        for (int k = 0; k < m; k++) {
            const float* N = rc.dirs + 3 * (dir0 + k);
            const float x = dR[0] * N[0] + dR[1] * N[1] + dR[2] * N[2];
            const float y = dR[3] * N[0] + dR[4] * N[1] + dR[5] * N[2];
            const float z = dR[6] * N[0] + dR[7] * N[1] + dR[8] * N[2];
            float Y[16];
            sh_basis(l, x, y, z, Y);
            for (int r = 0; r < m; r++) B[r][k] = Y[base + r];
        }
        const float* Ainv = rc.ainv + a0;   // m x m, row-major
        for (int r = 0; r < m; r++) {
            float Mr[7];
            for (int c = 0; c < m; c++) {
                float acc = 0.f;
                for (int k = 0; k < m; k++) acc += B[r][k] * Ainv[k * m + c];
                Mr[c] = acc;
            }
            for (int ch = 0; ch < 3; ch++) {
                float acc = 0.f;
                for (int c = 0; c < m; c++) acc += Mr[c] * sh[3 * (base + c) + ch];
                so[3 * (base + r) + ch] = acc;
            }
        }
        dir0 += m;
        a0 += m * m;
    }
}

}  // namespace

// Directions and A_l^{-1} for bands 1..3 (double on the host, then float).
ShRotConst make_shrot_const() {
    ShRotConst rc{};
    int dir0 = 0, a0 = 0;
    for (int l = 1; l <= 3; l++) {
        const int m = 2 * l + 1;
        double N[7][3];
        for (int k = 0; k < m; k++) {
            if (l == 1) {
                for (int c = 0; c < 3; c++) N[k][c] = k == c ? 1.0 : 0.0;
            } else {
                // golden-angle spiral started at 0.2 (a symmetric start makes A singular for band 3)
                const double ii = k + 0.2, z = 1.0 - 2.0 * ii / m, phi = M_PI * (1.0 + sqrt(5.0)) * ii;
                const double r = sqrt(1.0 - z * z);
                N[k][0] = r * cos(phi);
                N[k][1] = r * sin(phi);
                N[k][2] = z;
            }
            for (int c = 0; c < 3; c++) rc.dirs[3 * (dir0 + k) + c] = (float)N[k][c];
        }
        // A[r][k] = Y_{l, r}(N_k); invert by Gauss-Jordan with partial pivoting
        double A[7][14];
        for (int k = 0; k < m; k++) {
            double Y[16];
            sh_basis_t<double>(l, N[k][0], N[k][1], N[k][2], Y);
            for (int r = 0; r < m; r++) A[r][k] = Y[l * l + r];
        }
        for (int r = 0; r < m; r++)
            for (int c = 0; c < m; c++) A[r][m + c] = r == c ? 1.0 : 0.0;
        for (int c = 0; c < m; c++) {
            int piv = c;
            for (int r = c + 1; r < m; r++)
                if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
            for (int k = 0; k < 2 * m; k++) {
                const double t = A[c][k];
                A[c][k] = A[piv][k];
                A[piv][k] = t;
            }
            const double inv = 1.0 / A[c][c];
            for (int k = 0; k < 2 * m; k++) A[c][k] *= inv;
            for (int r = 0; r < m; r++) {
                if (r == c) continue;
                const double f = A[r][c];
                for (int k = 0; k < 2 * m; k++) A[r][k] -= f * A[c][k];
            }
        }
        for (int r = 0; r < m; r++)
            for (int c = 0; c < m; c++) rc.ainv[a0 + r * m + c] = (float)A[r][m + c];
        dir0 += m;
        a0 += m * m;
    }
    return rc;
}

void transform_bake(const Launch& L, const GaussDev& g, const ShRotConst& rc, float* mu_out, float* q_out,
                    float* sh_out) {
    if (g.n <= 0) return;
    if (L.prof) L.prof->begin("transform_bake", L.st);
    hipLaunchKernelGGL(k_bake, dim3((unsigned)((g.n + 127) / 128)), dim3(128), 0, L.st, g, rc, mu_out, q_out, sh_out);
    if (L.prof) L.prof->end(L.st);
}

}  // namespace gs3
