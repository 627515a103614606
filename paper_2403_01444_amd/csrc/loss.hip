// Stage-1 loss (Eq. 6): L = (1 - lambda) L1 + lambda (1 - SSIM), and dL/dx.
//
// SSIM uses an 11 x 11 Gaussian window (sigma 1.5) with zero padding, per
// channel, means over 3 x H x W.  The window is separable, so each 16 x 16
// output tile loads a 26 x 26 halo tile into LDS and filters rows then
// columns.  Forward: five filtered maps -> SSIM and its partial derivatives
// with respect to the filtered mean, E[x^2] and E[xy] at each pixel.
// Backward: the adjoint of a zero-padded correlation with a symmetric window
// is the same correlation, so the three partial maps are filtered again and
// combined with x and y.
#include "kernels.h"

namespace gs3 {

namespace {

constexpr int kT = 16;          // output tile edge
constexpr int kR = 5;           // window radius
constexpr int kH = kT + 2 * kR; // halo tile edge (26)
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Win {
    float g[11];
};

__device__ __forceinline__ float sgnf(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

__device__ __forceinline__ void block_sum2(double a, double b, double* out) {
    __shared__ double s[2][4];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s[0][w] = a;
        s[1][w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = s[0][0] + s[0][1] + s[0][2] + s[0][3];
        out[1] = s[1][0] + s[1][1] + s[1][2] + s[1][3];
    }
}

__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ x, const float* __restrict__ y, int64_t N,
                                            float scale, float* __restrict__ d, double* __restrict__ bsum) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double l1 = 0.0;
    if (i < N) {
        const float df = x[i] - y[i];
        l1 = fabsf(df);
        d[i] = scale * sgnf(df);
    }
    block_sum2(l1, 0.0, bsum + 2 * (int64_t)blockIdx.x);
}

__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ x, const float* __restrict__ y, int H,
                                                  int W, Win win, float* __restrict__ maps, double* __restrict__ bsum) {
    __shared__ float sx[kH][kH + 1];
    __shared__ float sy[kH][kH + 1];
    __shared__ float sh[5][kH][kT + 1];
    const int ch = blockIdx.z;
    const int bx = blockIdx.x, by = blockIdx.y;
    const int64_t P = (int64_t)H * W;
    const float* xc = x + ch * P;
    const float* yc = y + ch * P;
    for (int k = threadIdx.x; k < kH * kH; k += 256) {
        const int r = k / kH, c = k % kH;
        const int gy = by * kT + r - kR, gx = bx * kT + c - kR;
        const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
        sx[r][c] = in ? xc[(int64_t)gy * W + gx] : 0.f;
        sy[r][c] = in ? yc[(int64_t)gy * W + gx] : 0.f;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kH * kT; k += 256) {
        const int r = k / kT, c = k % kT;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
        for (int j = 0; j < 11; j++) {
            const float u = sx[r][c + j], v = sy[r][c + j], wj = win.g[j];
            a0 += wj * u;
            a1 += wj * v;
            a2 += wj * u * u;
            a3 += wj * v * v;
            a4 += wj * u * v;
        }
        sh[0][r][c] = a0; sh[1][r][c] = a1; sh[2][r][c] = a2; sh[3][r][c] = a3; sh[4][r][c] = a4;
    }
    __syncthreads();
    const int r = threadIdx.x / kT, c = threadIdx.x % kT;
    float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
    for (int j = 0; j < 11; j++) {
        const float wj = win.g[j];
        mx += wj * sh[0][r + j][c];
        my += wj * sh[1][r + j][c];
        exx += wj * sh[2][r + j][c];
        eyy += wj * sh[3][r + j][c];
        exy += wj * sh[4][r + j][c];
    }
    const int gy = by * kT + r, gx = bx * kT + c;
    double s_sum = 0.0, l1 = 0.0;
    if (gy < H && gx < W) {
        const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
        const float a1 = 2.f * mx * my + kC1, a2 = 2.f * sxy + kC2;
        const float b1 = mx * mx + my * my + kC1, b2 = sxx + syy + kC2;
        const float ib = 1.0f / (b1 * b2);
        const float S = a1 * a2 * ib;
        const float dS_da1 = a2 * ib, dS_da2 = a1 * ib, dS_db1 = -S / b1, dS_db2 = -S / b2;
        const float d_mx = 2.f * my * (dS_da1 - dS_da2) + 2.f * mx * (dS_db1 - dS_db2);
        const int64_t p = ch * P + (int64_t)gy * W + gx;
        const int64_t N = 3 * P;
        maps[p] = d_mx;
        maps[N + p] = dS_db2;
        maps[2 * N + p] = 2.f * dS_da2;
        s_sum = S;
        l1 = fabsf(sx[r + kR][c + kR] - sy[r + kR][c + kR]);
    }
    const int64_t blk = ((int64_t)ch * gridDim.y + by) * gridDim.x + bx;
    block_sum2(l1, s_sum, bsum + 2 * blk);
}

__global__ __launch_bounds__(256) void k_ssim_bwd(const float* __restrict__ x, const float* __restrict__ y, int H,
                                                  int W, Win win, float lam, const float* __restrict__ maps,
                                                  float* __restrict__ d) {
    __shared__ float sm[3][kH][kH + 1];
    __shared__ float sh[3][kH][kT + 1];
    const int ch = blockIdx.z;
    const int bx = blockIdx.x, by = blockIdx.y;
    const int64_t P = (int64_t)H * W, N = 3 * P;
    for (int k = threadIdx.x; k < kH * kH; k += 256) {
        const int r = k / kH, c = k % kH;
        const int gy = by * kT + r - kR, gx = bx * kT + c - kR;
        const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
        const int64_t p = ch * P + (int64_t)gy * W + gx;
        sm[0][r][c] = in ? maps[p] : 0.f;
        sm[1][r][c] = in ? maps[N + p] : 0.f;
        sm[2][r][c] = in ? maps[2 * N + p] : 0.f;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kH * kT; k += 256) {
        const int r = k / kT, c = k % kT;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int j = 0; j < 11; j++) {
            const float wj = win.g[j];
            a0 += wj * sm[0][r][c + j];
            a1 += wj * sm[1][r][c + j];
            a2 += wj * sm[2][r][c + j];
        }
        sh[0][r][c] = a0; sh[1][r][c] = a1; sh[2][r][c] = a2;
    }
    __syncthreads();
    const int r = threadIdx.x / kT, c = threadIdx.x % kT;
    const int gy = by * kT + r, gx = bx * kT + c;
    if (gy >= H || gx >= W) return;
    float fm = 0.f, fe = 0.f, ff = 0.f;
#pragma unroll
    for (int j = 0; j < 11; j++) {
        const float wj = win.g[j];
        fm += wj * sh[0][r + j][c];
        fe += wj * sh[1][r + j][c];
        ff += wj * sh[2][r + j][c];
    }
    const int64_t p = ch * P + (int64_t)gy * W + gx;
    const float xv = x[p], yv = y[p];
    const float invN = 1.0f / (float)N;
    d[p] = (1.f - lam) * sgnf(xv - yv) * invN - lam * invN * (fm + 2.f * xv * fe + yv * ff);
}

__global__ __launch_bounds__(256) void k_loss_finalize(const double* __restrict__ bsum, int64_t nblk, int64_t N,
                                                       float lam, float* __restrict__ loss, int* __restrict__ nonfinite) {
    __shared__ double s[2][4];
    // four independent partial sums per thread (fixed order), then combined
    double a4[4] = {0.0, 0.0, 0.0, 0.0}, b4[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t k = threadIdx.x;
    for (; k + 768 < nblk; k += 1024) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const double2 v = reinterpret_cast<const double2*>(bsum)[k + 256 * u];
            a4[u] += v.x;
            b4[u] += v.y;
        }
    }
    for (; k < nblk; k += 256) {
        a4[0] += bsum[2 * k];
        b4[0] += bsum[2 * k + 1];
    }
    double a = (a4[0] + a4[1]) + (a4[2] + a4[3]), b = (b4[0] + b4[1]) + (b4[2] + b4[3]);
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s[0][w] = a;
        s[1][w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double l1 = (s[0][0] + s[0][1] + s[0][2] + s[0][3]) / (double)N;
        const double ss = (s[1][0] + s[1][1] + s[1][2] + s[1][3]) / (double)N;
        const double L = lam == 0.f ? l1 : (1.0 - lam) * l1 + lam * (1.0 - ss);
        loss[0] = (float)L;
        if (!isfinite(L)) atomicOr(nonfinite, 1);
    }
}

Win make_window() {
    Win w;
    double g[11], s = 0.0;
    for (int k = 0; k < 11; k++) {
        g[k] = exp(-((k - 5) * (k - 5)) / (2.0 * 1.5 * 1.5));
        s += g[k];
    }
    for (int k = 0; k < 11; k++) w.g[k] = (float)(g[k] / s);
    return w;
}

}  // namespace

int64_t loss_map_floats(int H, int W) { return 3 * 3 * (int64_t)H * W; }

int loss_blocks(int H, int W) {
    const int a = 3 * ((W + kT - 1) / kT) * ((H + kT - 1) / kT);
    const int b = (int)((3 * (int64_t)H * W + 255) / 256);
    return a > b ? a : b;
}

void loss_forward_backward(const Launch& L, const float* x, const float* y, int H, int W, float lambda,
                           const LossWork& w, float* loss_dev, float* d_image, int* nonfinite) {
    const int64_t N = 3 * (int64_t)H * W;
    if (L.prof) L.prof->begin("loss", L.st);
    if (lambda == 0.f) {
        const unsigned nb = (unsigned)((N + 255) / 256);
        hipLaunchKernelGGL(k_l1, dim3(nb), dim3(256), 0, L.st, x, y, N, 1.0f / (float)N, d_image, w.block_sums);
        hipLaunchKernelGGL(k_loss_finalize, dim3(1), dim3(256), 0, L.st, w.block_sums, (int64_t)nb, N, 0.f, loss_dev,
                           nonfinite);
    } else {
        const Win win = make_window();
        dim3 grid((W + kT - 1) / kT, (H + kT - 1) / kT, 3);
        hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, L.st, x, y, H, W, win, w.partial_maps, w.block_sums);
        hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, L.st, x, y, H, W, win, lambda, w.partial_maps, d_image);
        const int64_t nblk = (int64_t)grid.x * grid.y * grid.z;
        hipLaunchKernelGGL(k_loss_finalize, dim3(1), dim3(256), 0, L.st, w.block_sums, nblk, N, lambda, loss_dev,
                           nonfinite);
    }
    if (L.prof) L.prof->end(L.st);
}

}  // namespace gs3
