// Stage 2, adaptive 3DG addition (Sec. 4.2): selection of Gaussians by a
// threshold (view-space gradient average, or opacity for pruning) and the
// spawning of additional Gaussians around the selected ones.
#include <math.h>

#include "kernels.h"

namespace gs3 {

namespace {

// flag[i] = den ? (den[i] > 0 && num[i] / den[i] > thr) : num[i] >= thr
__global__ __launch_bounds__(256) void k_select_flags(const float* __restrict__ num, const float* __restrict__ den,
                                                      int64_t n, float thr, uint32_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    bool keep;
    if (den) {
        const float d = den[i];
        keep = d > 0.f && num[i] / d > thr;
    } else {
        keep = num[i] >= thr;
    }
    flag[i] = keep ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_select_compact(const uint32_t* __restrict__ flag,
                                                        const uint32_t* __restrict__ pos, int64_t n,
                                                        uint32_t* __restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if (flag[i]) idx[pos[i]] = (uint32_t)i;
}

// X = mu + sqrt(2) R(q^) diag(exp(log s)) z, i.e. a draw of N(mu, 2 Sigma).
__global__ __launch_bounds__(256) void k_spawn(GaussDev g, const uint32_t* __restrict__ idx, int64_t m,
                                               const float* __restrict__ z, int mode, float logit0, float log_shrink,
                                               float* __restrict__ mu_out, float* __restrict__ q_out,
                                               float* __restrict__ ls_out, float* __restrict__ lo_out,
                                               float* __restrict__ sh_out) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= m) return;
    const int64_t i = idx[k];
    float q[4] = {g.quats[4 * i], g.quats[4 * i + 1], g.quats[4 * i + 2], g.quats[4 * i + 3]};
    const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    float qh[4] = {1.f, 0.f, 0.f, 0.f};
    if (qn > 0.f)
        for (int c = 0; c < 4; c++) qh[c] = q[c] / qn;
    float R[9];
    quat_to_rot(qh, R);
    float sz[3];
    for (int c = 0; c < 3; c++) sz[c] = expf(g.log_scales[3 * i + c]) * z[3 * k + c];
    for (int r = 0; r < 3; r++)
        mu_out[3 * k + r] = g.means[3 * i + r] + 1.41421356237f * (R[3 * r] * sz[0] + R[3 * r + 1] * sz[1] +
                                                                    R[3 * r + 2] * sz[2]);
    for (int c = 0; c < 4; c++) q_out[4 * k + c] = mode == 0 ? (c == 0 ? 1.f : 0.f) : q[c];
    for (int c = 0; c < 3; c++) ls_out[3 * k + c] = g.log_scales[3 * i + c] + (mode == 0 ? 0.f : log_shrink);
    lo_out[k] = mode == 0 ? logit0 : g.opac[i];
    const int K3 = 3 * (g.sh_degree + 1) * (g.sh_degree + 1);
    for (int c = 0; c < K3; c++) sh_out[k * K3 + c] = g.sh[i * K3 + c];
}

}  // namespace

void select_indices(const Launch& L, const float* num, const float* den, int64_t n, float thr, uint32_t* flag,
                    uint32_t* pos, uint64_t* total, uint64_t* tmp, uint32_t* idx) {
    if (n <= 0) return;
    if (L.prof) L.prof->begin("select", L.st);
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_select_flags, dim3(nb), dim3(256), 0, L.st, num, den, n, thr, flag);
    scan_u32_to_u32(L, flag, n, pos, total, tmp);
    hipLaunchKernelGGL(k_select_compact, dim3(nb), dim3(256), 0, L.st, flag, pos, n, idx);
    if (L.prof) L.prof->end(L.st);
}

void spawn(const Launch& L, const GaussDev& g, const uint32_t* idx, int64_t m, const float* z, int mode,
           float logit0, float log_shrink, float* mu, float* q, float* ls, float* lo, float* sh) {
    if (m <= 0) return;
    if (L.prof) L.prof->begin("spawn", L.st);
    hipLaunchKernelGGL(k_spawn, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, L.st, g, idx, m, z, mode, logit0,
                       log_shrink, mu, q, ls, lo, sh);
    if (L.prof) L.prof->end(L.st);
}

}  // namespace gs3
