// Stage-1 loss (Eq. 6): L = (1 - lambda) L1 + lambda (1 - SSIM), and dL/dx.
//
// SSIM uses an 11 x 11 Gaussian window (sigma 1.5) with zero padding, per
// channel, means over 3 x H x W.  The window is separable: each workgroup
// loads a 42 x 42 halo tile for a 32 x 32 output tile into LDS, filters the
// rows (a thread takes four adjacent outputs of a halo row, so it reads 14
// inputs and forms their products once), then the columns (a thread takes
// four outputs of one column from 14 row-filtered values).  Forward: five
// filtered maps (the two means, then the three second moments, through the
// same LDS) -> SSIM and its partial derivatives with respect to the
// filtered mean, E[x^2] and E[xy] at each pixel.  Backward: the adjoint of a
// zero-padded correlation with a symmetric window is the same correlation,
// so the three partial maps are filtered again (one at a time) and combined
// with x and y.  Keeping few row-filtered maps in LDS at once lets five
// workgroups share a CU.
#include <mutex>

#include "../../include/gs3.h"
#include "kernels.h"

namespace gs3 {

namespace {

constexpr int kTW = 32;              // output tile width
constexpr int kTH = 32;              // output tile height
constexpr int kR = 5;                // window radius
constexpr int kHW = kTW + 2 * kR;    // halo tile width (42)
constexpr int kHH = kTH + 2 * kR;    // halo tile height (42)
constexpr int kQ = 4;                // outputs per thread in each filter pass
constexpr int kIn = kQ + 2 * kR;     // inputs per thread in each filter pass (14)
constexpr int kQR = 8;               // outputs per task of the row filters: 42 x 4 tasks, one round of 256 threads
constexpr int kInR = kQR + 2 * kR;   // their inputs (18)
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

// The loss from the per-block (L1, SSIM) sums: one block of 256 threads, a
// fixed summation order.
__device__ __forceinline__ void finalize_sums(const double* __restrict__ bsum, int64_t nblk, int64_t N, float lam,
                                              float* __restrict__ loss, int* __restrict__ nonfinite) {
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

// Row filter: for the tasks t = threadIdx.x, threadIdx.x + 256, ... of the
// 42 x 4 (halo row r, column octet q) tasks, outputs at columns 8 q .. 8 q + 7
// of the NM maps src[m] -> dst[m] (one round of tasks: 168 of the 256
// threads, each reading 18 inputs per map).
template <int NM>
__device__ __forceinline__ void row_filter(const Win& win, const float (*src)[kHH][kHW + 1],
                                           float (*dst)[kHH][kTW + 1]) {
    for (int t = threadIdx.x; t < kHH * (kTW / kQR); t += 256) {
        const int r = t / (kTW / kQR), c0 = (t % (kTW / kQR)) * kQR;
#pragma unroll
        for (int m = 0; m < NM; m++) {
            float u[kInR];
#pragma unroll
            for (int i = 0; i < kInR; i++) u[i] = src[m][r][c0 + i];
#pragma unroll
            for (int o = 0; o < kQR; o++) {
                float a = 0.f;
#pragma unroll
                for (int j = 0; j < 11; j++) a += win.g[j] * u[o + j];
                dst[m][r][c0 + o] = a;
            }
        }
    }
}

// Row filter of the three second moments x^2, y^2, x y of src[0] = x and
// src[1] = y (same task layout as row_filter).
__device__ __forceinline__ void row_filter_second(const Win& win, const float (*src)[kHH][kHW + 1],
                                                  float (*dst)[kHH][kTW + 1]) {
    for (int t = threadIdx.x; t < kHH * (kTW / kQR); t += 256) {
        const int r = t / (kTW / kQR), c0 = (t % (kTW / kQR)) * kQR;
        float u[kInR], v[kInR];
#pragma unroll
        for (int i = 0; i < kInR; i++) {
            u[i] = src[0][r][c0 + i];
            v[i] = src[1][r][c0 + i];
        }
#pragma unroll
        for (int o = 0; o < kQR; o++) {
            float a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
            for (int j = 0; j < 11; j++) {
                const float uj = u[o + j], vj = v[o + j], wj = win.g[j];
                a2 += wj * uj * uj;
                a3 += wj * vj * vj;
                a4 += wj * uj * vj;
            }
            dst[0][r][c0 + o] = a2;
            dst[1][r][c0 + o] = a3;
            dst[2][r][c0 + o] = a4;
        }
    }
}

// column filter of map m: outputs rows 4 g .. 4 g + 3 of column c
__device__ __forceinline__ void col_filter(const Win& win, const float (*src)[kTW + 1], int g, int c, float out[kQ]) {
    float u[kIn];
#pragma unroll
    for (int i = 0; i < kIn; i++) u[i] = src[kQ * g + i][c];
#pragma unroll
    for (int o = 0; o < kQ; o++) {
        float a = 0.f;
#pragma unroll
        for (int j = 0; j < 11; j++) a += win.g[j] * u[o + j];
        out[o] = a;
    }
}

__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ x, const float* __restrict__ y, int H,
                                                  int W, Win win, float* __restrict__ maps, double* __restrict__ bsum) {
    __shared__ float s_img[2][kHH][kHW + 1];   // x, y halo tiles
    __shared__ float sh[3][kHH][kTW + 1];      // row-filtered maps, three at a time
    __shared__ float s_w[2][4];
    const int ch = blockIdx.z;
    const int bx = blockIdx.x, by = blockIdx.y;
    const int64_t P = (int64_t)H * W;
    const float* xc = x + ch * P;
    const float* yc = y + ch * P;
    for (int k = threadIdx.x; k < kHH * kHW; k += 256) {
        const int r = k / kHW, c = k % kHW;
        const int gy = by * kTH + r - kR, gx = bx * kTW + c - kR;
        const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
        s_img[0][r][c] = in ? xc[(int64_t)gy * W + gx] : 0.f;
        s_img[1][r][c] = in ? yc[(int64_t)gy * W + gx] : 0.f;
    }
    __syncthreads();
    // the means first, then the second moments through the same LDS maps
    // (their products formed in the second row pass): three maps of LDS
    // instead of five leave room for five workgroups per CU
    const int c = threadIdx.x % kTW, g = threadIdx.x / kTW;
    float mx[kQ], my[kQ], exx[kQ], eyy[kQ], exy[kQ];
    row_filter<2>(win, s_img, sh);
    __syncthreads();
    col_filter(win, sh[0], g, c, mx);
    col_filter(win, sh[1], g, c, my);
    __syncthreads();
    row_filter_second(win, s_img, sh);
    __syncthreads();
    col_filter(win, sh[0], g, c, exx);
    col_filter(win, sh[1], g, c, eyy);
    col_filter(win, sh[2], g, c, exy);
    const int gx = bx * kTW + c;
    const int64_t N = 3 * P;
    float s_sum = 0.f, l1 = 0.f;
#pragma unroll
    for (int o = 0; o < kQ; o++) {
        const int r = kQ * g + o;
        const int gy = by * kTH + r;
        if (gy < H && gx < W) {
            const float sxx = exx[o] - mx[o] * mx[o], syy = eyy[o] - my[o] * my[o], sxy = exy[o] - mx[o] * my[o];
            const float a1 = 2.f * mx[o] * my[o] + kC1, a2 = 2.f * sxy + kC2;
            const float b1 = mx[o] * mx[o] + my[o] * my[o] + kC1, b2 = sxx + syy + kC2;
            // hardware reciprocal (1 ulp; b1 b2 >= C1 C2 is a normal number);
            // 1 / b1 = b2 ib and 1 / b2 = b1 ib
            const float ib = __builtin_amdgcn_rcpf(b1 * b2);
            const float S = a1 * a2 * ib;
            const float dS_da1 = a2 * ib, dS_da2 = a1 * ib, dS_db1 = -S * (b2 * ib), dS_db2 = -S * (b1 * ib);
            const float d_mx = 2.f * my[o] * (dS_da1 - dS_da2) + 2.f * mx[o] * (dS_db1 - dS_db2);
            const int64_t p = ch * P + (int64_t)gy * W + gx;
            maps[p] = d_mx;
            maps[N + p] = dS_db2;
            maps[2 * N + p] = 2.f * dS_da2;
            s_sum += S;
            l1 += fabsf(s_img[0][r + kR][c + kR] - s_img[1][r + kR][c + kR]);
        }
    }
    // block sums: float within a wave, double across the four waves
    for (int off = 32; off > 0; off >>= 1) {
        l1 += __shfl_xor(l1, off, 64);
        s_sum += __shfl_xor(s_sum, off, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_w[0][w] = l1;
        s_w[1][w] = s_sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t blk = ((int64_t)ch * gridDim.y + by) * gridDim.x + bx;
        bsum[2 * blk] = ((double)s_w[0][0] + (double)s_w[0][1]) + ((double)s_w[0][2] + (double)s_w[0][3]);
        bsum[2 * blk + 1] = ((double)s_w[1][0] + (double)s_w[1][1]) + ((double)s_w[1][2] + (double)s_w[1][3]);
    }
}

__global__ __launch_bounds__(256) void k_ssim_bwd(const float* __restrict__ x, const float* __restrict__ y, int H,
                                                  int W, Win win, float lam, const float* __restrict__ maps,
                                                  float* __restrict__ d, const double* __restrict__ bsum,
                                                  int64_t nblk, float* __restrict__ loss, int* __restrict__ nonfinite) {
    __shared__ float sm[3][kHH][kHW + 1];
    __shared__ float sh[1][kHH][kTW + 1];   // one row-filtered map at a time
    const int ch = blockIdx.z;
    const int bx = blockIdx.x, by = blockIdx.y;
    const int64_t P = (int64_t)H * W, N = 3 * P;
    for (int k = threadIdx.x; k < kHH * kHW; k += 256) {
        const int r = k / kHW, c = k % kHW;
        const int gy = by * kTH + r - kR, gx = bx * kTW + c - kR;
        const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
        const int64_t p = ch * P + (int64_t)gy * W + gx;
        sm[0][r][c] = in ? maps[p] : 0.f;
        sm[1][r][c] = in ? maps[N + p] : 0.f;
        sm[2][r][c] = in ? maps[2 * N + p] : 0.f;
    }
    const int c = threadIdx.x % kTW, g = threadIdx.x / kTW;
    float fm[kQ], fe[kQ], ff[kQ];
    float* const fout[3] = {fm, fe, ff};
#pragma unroll
    for (int m = 0; m < 3; m++) {
        __syncthreads();
        row_filter<1>(win, sm + m, sh);
        __syncthreads();
        col_filter(win, sh[0], g, c, fout[m]);
    }
    const int gx = bx * kTW + c;
    const float invN = 1.0f / (float)N;
#pragma unroll
    for (int o = 0; o < kQ; o++) {
        const int gy = by * kTH + kQ * g + o;
        if (gy < H && gx < W) {
            const int64_t p = ch * P + (int64_t)gy * W + gx;
            const float xv = x[p], yv = y[p];
            d[p] = (1.f - lam) * sgnf(xv - yv) * invN - lam * invN * (fm[o] + 2.f * xv * fe[o] + yv * ff[o]);
        }
    }
    // the loss value: the forward wrote every block's sums before this
    // launch, so one block adds them up here instead of a launch of its own
    if (bx == 0 && by == 0 && ch == 0) finalize_sums(bsum, nblk, N, lam, loss, nonfinite);
}


__global__ __launch_bounds__(256) void k_loss_finalize(const double* __restrict__ bsum, int64_t nblk, int64_t N,
                                                       float lam, float* __restrict__ loss, int* __restrict__ nonfinite) {
    finalize_sums(bsum, nblk, N, lam, loss, nonfinite);
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
    const int a = 3 * ((W + kTW - 1) / kTW) * ((H + kTH - 1) / kTH);
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
        dim3 grid((W + kTW - 1) / kTW, (H + kTH - 1) / kTH, 3);
        hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, L.st, x, y, H, W, win, w.partial_maps, w.block_sums);
        const int64_t nblk = (int64_t)grid.x * grid.y * grid.z;
        hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, L.st, x, y, H, W, win, lambda, w.partial_maps, d_image,
                           (const double*)w.block_sums, nblk, loss_dev, nonfinite);
    }
    if (L.prof) L.prof->end(L.st);
}

}  // namespace gs3

// ---- Eq. 6 without allocation ---------------------------------------------
// gs3_loss_noalloc runs the kernels of gs3_loss with their scratch (the SSIM
// partial maps, the per-block partial sums and a flag word) in `scratch`, a
// file-scope device array: every GPU the library runs on holds its own copy
// until the process ends, and every call on that GPU shares it.  Host code
// never passes the array's name to a kernel (on the host it only stands for
// the symbol): the device address comes from hipGetSymbolAddress, taken once
// per device with that device current.
namespace gs3 {
namespace {
constexpr int64_t kNaMaxPixels = int64_t(1) << 21;   // 2,097,152: 1920 x 1080 fits
constexpr int kNaMaxSide = 4096;
constexpr int64_t kNaMapFloats = 9 * kNaMaxPixels;   // loss_map_floats at the largest size
// loss_blocks(H, W) <= max(3 ceil(W/32) ceil(H/32), ceil(3 H W / 256)); with
// H W <= 2^21 and both sides <= 4096 the second term dominates: 24,576
constexpr int64_t kNaMaxBlocks = 3 * kNaMaxPixels / 256;
constexpr int64_t kNaFloats = kNaMapFloats + 2 * (2 * kNaMaxBlocks) + 64;
constexpr int kNaMaxDevices = 64;

static __device__ __align__(256) float scratch[kNaFloats];

std::once_flag g_na_once[kNaMaxDevices];
float* g_na_ptr[kNaMaxDevices];
hipError_t g_na_err[kNaMaxDevices];
}  // namespace
}  // namespace gs3

extern "C" gs3_status gs3_loss_noalloc(const float* image, const float* target, int32_t height, int32_t width,
                                       float lambda_dssim, float* loss_dev, float* d_image, void* hip_stream) {
    using namespace gs3;
    if (!image || !target || !loss_dev || !d_image) return GS3_EINVAL;
    if (height < 1 || width < 1 || height > kNaMaxSide || width > kNaMaxSide ||
        (int64_t)height * width > kNaMaxPixels)
        return GS3_EINVAL;
    if (!(lambda_dssim >= 0.f && lambda_dssim <= 1.f)) return GS3_EINVAL;
    if ((int64_t)loss_blocks(height, width) > kNaMaxBlocks) return GS3_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNaMaxDevices) return GS3_EHIP;
    std::call_once(g_na_once[dev], [dev] {
        void* ptr = nullptr;
        g_na_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_na_ptr[dev] = g_na_err[dev] == hipSuccess ? static_cast<float*>(ptr) : nullptr;
    });
    if (g_na_err[dev] != hipSuccess || !g_na_ptr[dev]) return GS3_EHIP;
    float* base = g_na_ptr[dev];
    // every word the kernels read is written earlier in the same call (maps
    // by the forward SSIM pass, block sums by each block), so nothing needs
    // clearing; the flag word is only ever set and is not reported here
    LossWork w{base, reinterpret_cast<double*>(base + kNaMapFloats), (int)kNaMaxBlocks};
    int* flag = reinterpret_cast<int*>(base + kNaMapFloats + 4 * kNaMaxBlocks);
    Launch L{static_cast<hipStream_t>(hip_stream), nullptr};
    loss_forward_backward(L, image, target, height, width, lambda_dssim, w, loss_dev, d_image, flag);
    return hipGetLastError() == hipSuccess ? GS3_OK : GS3_EHIP;
}
