// Neural Transformation Cache on gfx950 (Sec. 4.1, Eq. 5):
//   (dmu, dq) = MLP(h(mu)),  h = multi-resolution hash encoding,
//   MLP = 32 -> 64 (ReLU) -> 64 (ReLU) -> 7, no biases.
//
// Work unit: a batch of 16 points per wave.  Lane l owns point l % 16 and
// levels 4 (l / 16) .. 4 (l / 16) + 3 of the encoding, so the 64 lanes cover
// the 16 x 16 (point, level) pairs of a batch.  Activations go through LDS in
// [point][feature] layout; every layer is a 16 x 16 MFMA tile product
// (v_mfma_f32_16x16x16 f16 / bf16, or 16x16x4 f32), weights staged once per
// workgroup in LDS.  The backward pass recomputes the forward and
// propagates the output gradient through the three layers, each wave on its
// own batch; then the four waves accumulate the weight gradients of the
// four batches with MFMA (contraction over each batch's 16 points) in FP32
// registers, each wave a quarter of the weight tiles; the encoding gradient
// goes to the per-entry gather of the table gradient, or is scatter-added
// into it with global atomics.
//
// Half-precision backward: each activation-gradient stage is rescaled by a
// power of two so that its largest magnitude in the batch sits near 2^13
// before it is rounded to FP16/BF16; the FP32 results are unscaled exactly.
#include <algorithm>

#include "kernels.h"
#include "ntc.h"

namespace gs3 {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef __bf16 b4v __attribute__((ext_vector_type(4)));

struct PF32 {
    using S = float;
    using AF = float;
    static constexpr int KPL = 1;
    static constexpr int KSTEP = 4;
    __device__ static f4v mfma(AF a, AF b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static S cvt(float x) { return x; }
    __device__ static float tof(S x) { return x; }
    static constexpr bool kScaled = false;
};
struct PF16 {
    using S = _Float16;
    using AF = h4v;
    static constexpr int KPL = 4;
    static constexpr int KSTEP = 16;
    __device__ static f4v mfma(AF a, AF b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0); }
    __device__ static S cvt(float x) { return (S)x; }
    __device__ static float tof(S x) { return (float)x; }
    static constexpr bool kScaled = true;
};
struct PBF16 {
    using S = __bf16;
    using AF = b4v;
    static constexpr int KPL = 4;
    static constexpr int KSTEP = 16;
    __device__ static f4v mfma(AF a, AF b, f4v c) {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
    __device__ static S cvt(float x) { return (S)x; }
    __device__ static float tof(S x) { return (float)x; }
    static constexpr bool kScaled = true;
};

// A or B fragment, elements base[row * ld + k0 + i] (contiguous in k)
template <class P>
__device__ __forceinline__ typename P::AF frag_k_contig(const typename P::S* base, int ld, int row, int k0) {
    typename P::AF f;
    if constexpr (P::KPL == 1) {
        f = base[row * ld + k0];
    } else {
#pragma unroll
        for (int i = 0; i < P::KPL; i++) f[i] = base[row * ld + k0 + i];
    }
    return f;
}
// fragment with elements base[(k0 + i) * ld + col] (strided in k)
template <class P>
__device__ __forceinline__ typename P::AF frag_k_strided(const typename P::S* base, int ld, int col, int k0) {
    typename P::AF f;
    if constexpr (P::KPL == 1) {
        f = base[k0 * ld + col];
    } else {
#pragma unroll
        for (int i = 0; i < P::KPL; i++) f[i] = base[(k0 + i) * ld + col];
    }
    return f;
}

// Inside the batch loops each wave works on its own activation arrays in LDS
// (the staged weights are read-only there), so the waves of a workgroup only
// order their own LDS accesses: a wave-level barrier that keeps the compiler
// from moving LDS accesses across it (a wave's LDS operations complete in
// issue order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row strides (elements) of the LDS arrays; +4 breaks bank regularity.
constexpr int kMlpParams = 64 * 32 + 64 * 64 + 7 * 64;
constexpr int LD32 = 32 + 4;
constexpr int LD64 = 64 + 4;
constexpr int LD16 = 16 + 4;
constexpr int kWaves = 4;
constexpr int kPts = 16;

// the two features of a table entry; the entry's byte offset fits in 32 bits
// (at most 2^26 entries), so the load takes a scalar base and a 32-bit offset
template <class P>
__device__ __forceinline__ float2 load2(const typename P::S* table, uint32_t entry) {
    const unsigned char* base = reinterpret_cast<const unsigned char*>(table);
    const uint32_t off = entry * (uint32_t)(2 * sizeof(typename P::S));
    if constexpr (sizeof(typename P::S) == 4) {
        return *reinterpret_cast<const float2*>(base + off);
    } else {
        typedef typename P::S s2v __attribute__((ext_vector_type(2)));
        const s2v v = *reinterpret_cast<const s2v*>(base + off);
        return make_float2(P::tof(v.x), P::tof(v.y));
    }
}

// normalised position; false when outside [0, 1]^3 (the point is discarded)
__device__ __forceinline__ bool ntc_normalise(const NtcDev& nd, const float* mu, float x[3]) {
#pragma clang fp contract(off)
    bool in = true;
    for (int k = 0; k < 3; k++) {
        x[k] = (mu[k] - nd.aabb_min[k]) * nd.inv_ext[k];
        in = in && (x[k] >= 0.0f) && (x[k] <= 1.0f);
    }
    return in;
}

// corner entries and trilinear weights of level lv
__device__ __forceinline__ void ntc_corners(const NtcDev& nd, int lv, const float x[3], uint32_t ent[8], float wt[8]) {
    float w[3];
    uint32_t i0[3];
    {
#pragma clang fp contract(off)
        const int N = nd.res[lv];
        const float fN = (float)N;
        for (int k = 0; k < 3; k++) {
            const float p = x[k] * fN;
            int c = (int)floorf(p);
            c = c > N - 1 ? N - 1 : c;
            c = c < 0 ? 0 : c;
            i0[k] = (uint32_t)c;
            w[k] = p - (float)c;
        }
    }
    const int N1 = nd.res[lv] + 1;
    const bool dense = (nd.dense_mask >> lv) & 1u;
#pragma unroll
    for (int c = 0; c < 8; c++) {
        const uint32_t vx = i0[0] + (c & 1), vy = i0[1] + ((c >> 1) & 1), vz = i0[2] + ((c >> 2) & 1);
        uint32_t idx;
        if (dense)
            idx = vx + (uint32_t)N1 * (vy + (uint32_t)N1 * vz);
        else
            idx = ((vx * 1u) ^ (vy * 2654435761u) ^ (vz * 805459861u)) & nd.T_mask;
        ent[c] = (uint32_t)nd.off[lv] + idx;
        wt[c] = ((c & 1) ? w[0] : 1.0f - w[0]) * (((c >> 1) & 1) ? w[1] : 1.0f - w[1]) *
                (((c >> 2) & 1) ? w[2] : 1.0f - w[2]);
    }
}

template <class P>
__device__ __forceinline__ void load_weights(const typename P::S* __restrict__ mlp, typename P::S* sW1,
                                             typename P::S* sW2, typename P::S* sW3, typename P::S* sW1t,
                                             typename P::S* sW2t, typename P::S* sW3t) {
    using S = typename P::S;
    const S* W1 = mlp;
    const S* W2 = mlp + 64 * 32;
    const S* W3 = mlp + 64 * 32 + 64 * 64;
    for (int k = threadIdx.x; k < 64 * 32; k += blockDim.x) {
        const int r = k / 32, c = k % 32;
        if (sW1) sW1[r * LD32 + c] = W1[k];
        if (sW1t) sW1t[c * LD64 + r] = W1[k];
    }
    for (int k = threadIdx.x; k < 64 * 64; k += blockDim.x) {
        const int r = k / 64, c = k % 64;
        if (sW2) sW2[r * LD64 + c] = W2[k];
        if (sW2t) sW2t[c * LD64 + r] = W2[k];
    }
    for (int k = threadIdx.x; k < 16 * 64; k += blockDim.x) {
        const int r = k / 64, c = k % 64;
        const S v = r < 7 ? W3[r * 64 + c] : P::cvt(0.0f);
        if (sW3) sW3[r * LD64 + c] = v;
        if (sW3t) sW3t[c * LD16 + r] = v;
    }
}

// D (16 x 16, rows m0.., cols = points) += W[m0..m0+15][0..K) X[p][0..K)
template <class P, int K>
__device__ __forceinline__ f4v layer_tile(const typename P::S* W, int ldw, int m0, const typename P::S* X, int ldx,
                                          int lane) {
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    const int row = lane & 15, g = lane >> 4;
#pragma unroll
    for (int ks = 0; ks < K / P::KSTEP; ks++) {
        const int k0 = ks * P::KSTEP + P::KPL * g;
        acc = P::mfma(frag_k_contig<P>(W, ldw, m0 + row, k0), frag_k_contig<P>(X, ldx, row, k0), acc);
    }
    return acc;
}

// encode this lane's 4 levels of its point into X[p][8 g .. 8 g + 7]
template <class P>
__device__ __forceinline__ void encode_lane(const NtcDev& nd, const typename P::S* __restrict__ table,
                                            const float x[3], int g, typename P::S* X, int p) {
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int lv = 4 * g + j;
        uint32_t ent[8];
        float wt[8];
        ntc_corners(nd, lv, x, ent, wt);
        float e0 = 0.f, e1 = 0.f;
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const float2 v = load2<P>(table, ent[c]);
            e0 += wt[c] * v.x;
            e1 += wt[c] * v.y;
        }
        X[p * LD32 + 2 * lv] = P::cvt(e0);
        X[p * LD32 + 2 * lv + 1] = P::cvt(e1);
    }
}

// A lane's eight encoding values (levels 4 g .. 4 g + 3) of point pt:
// LDS row X[p] <-> the cached encoding enc[pt][8 g .. 8 g + 7].
template <class P>
__device__ __forceinline__ void enc_to_cache(const typename P::S* X, int p, int g, typename P::S* enc, int64_t pt) {
#pragma unroll
    for (int j = 0; j < 8; j++) enc[pt * 32 + 8 * g + j] = X[p * LD32 + 8 * g + j];
}
template <class P>
__device__ __forceinline__ void enc_from_cache(typename P::S* X, int p, int g, const typename P::S* enc, int64_t pt) {
#pragma unroll
    for (int j = 0; j < 8; j++) X[p * LD32 + 8 * g + j] = enc[pt * 32 + 8 * g + j];
}

template <class P>
__global__ __launch_bounds__(256) void k_ntc_fwd(NtcDev nd, const typename P::S* __restrict__ table,
                                                 const typename P::S* __restrict__ mlp, const float* __restrict__ means,
                                                 int64_t n, float* __restrict__ dmu, float* __restrict__ dq,
                                                 typename P::S* __restrict__ enc_out) {
    using S = typename P::S;
    __shared__ S sW1[64 * LD32], sW2[64 * LD64], sW3[16 * LD64];
    __shared__ S sX[kWaves][kPts * LD32], sH1[kWaves][kPts * LD64], sH2[kWaves][kPts * LD64];
    load_weights<P>(mlp, sW1, sW2, sW3, nullptr, nullptr, nullptr);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = lane & 15, g = lane >> 4;
    S* X = sX[w];
    S* H1 = sH1[w];
    S* H2 = sH2[w];
    const int64_t nb = (n + kPts - 1) / kPts;
    // each batch's means are loaded one round ahead
    float nmu[3] = {0.f, 0.f, 0.f};
    auto prefetch = [&](int64_t bb) {
        const int64_t q = (bb + w) * kPts + p;
        if (bb < nb && q < n) {
            nmu[0] = means[3 * q];
            nmu[1] = means[3 * q + 1];
            nmu[2] = means[3 * q + 2];
        }
    };
    prefetch((int64_t)blockIdx.x * kWaves);
    for (int64_t b0 = (int64_t)blockIdx.x * kWaves; b0 < nb; b0 += (int64_t)gridDim.x * kWaves) {
        const int64_t pt = (b0 + w) * kPts + p;
        const bool valid = pt < n;
        float x[3] = {0.f, 0.f, 0.f};
        bool in = false;
        if (valid) in = ntc_normalise(nd, nmu, x);
        prefetch(b0 + (int64_t)gridDim.x * kWaves);
        wave_sync();   // previous batch's reads of X done
        if (in) {
            encode_lane<P>(nd, table, x, g, X, p);
        } else {
            for (int j = 0; j < 8; j++) X[p * LD32 + 8 * g + j] = P::cvt(0.f);
        }
        wave_sync();
        if (enc_out && valid) enc_to_cache<P>(X, p, g, enc_out, pt);   // kept for the backward
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            const f4v a = layer_tile<P, 32>(sW1, LD32, mt * 16, X, LD32, lane);
            for (int r = 0; r < 4; r++) H1[p * LD64 + mt * 16 + 4 * g + r] = P::cvt(fmaxf(a[r], 0.f));
        }
        wave_sync();
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            const f4v a = layer_tile<P, 64>(sW2, LD64, mt * 16, H1, LD64, lane);
            for (int r = 0; r < 4; r++) H2[p * LD64 + mt * 16 + 4 * g + r] = P::cvt(fmaxf(a[r], 0.f));
        }
        wave_sync();
        const f4v o = layer_tile<P, 64>(sW3, LD64, 0, H2, LD64, lane);
        if (valid && g < 2) {
            if (g == 0) {
                dmu[3 * pt + 0] = in ? o[0] : 0.f;
                dmu[3 * pt + 1] = in ? o[1] : 0.f;
                dmu[3 * pt + 2] = in ? o[2] : 0.f;
                dq[4 * pt + 0] = in ? o[3] : 1.f;
            } else {
                dq[4 * pt + 1] = in ? o[0] : 0.f;
                dq[4 * pt + 2] = in ? o[1] : 0.f;
                dq[4 * pt + 3] = in ? o[2] : 0.f;
            }
        }
    }
}

__device__ __forceinline__ float wave_max(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// exponent k of the power of two 2^k with max * 2^k in [2^12, 2^13); 0 when
// max is 0 or not finite
__device__ __forceinline__ int pow2_exp(float mx) {
    if (!(mx > 0.f) || !isfinite(mx)) return 0;
    int e;
    frexpf(mx, &e);   // mx = f 2^e, f in [0.5, 1)
    return 13 - e;
}

// the scale exponents stay inside the normal range of float, so 2^k and
// 2^-k are exact
__device__ __forceinline__ int clamp_exp(int k) { return k < -126 ? -126 : (k > 126 ? 126 : k); }

// kCSR: write the encoding gradient (n x 32 floats) to `denc` for the
// per-entry gather of the prepared contribution lists; otherwise scatter-add
// it into the table gradient with atomics.
//
// Each iteration takes four batches, one per wave.  Phase A (each wave on its
// own batch): the encoding, the forward layers, the output gradient and the
// activation gradients of the three layers, all kept in the wave's LDS
// arrays (activations and gradients side by side), and the encoding
// gradient.  Phase B (after a workgroup barrier): the weight gradients of
// all four batches, split between the waves by output rows (wave w: the 16
// rows 16 w.. of dW1 and dW2 and the 16 columns 16 w.. of dW3), so a wave
// holds 7 accumulator tiles instead of 28 and the register file leaves room
// for more than one wave per SIMD.
template <class P, bool kCSR>
__global__ __launch_bounds__(256) void k_ntc_bwd(NtcDev nd, const typename P::S* __restrict__ table,
                                                 const typename P::S* __restrict__ mlp, const float* __restrict__ means,
                                                 int64_t n, const float* __restrict__ d_dmu,
                                                 const float* __restrict__ d_dq, float* __restrict__ g_table,
                                                 float* __restrict__ g_part, float* __restrict__ denc,
                                                 const typename P::S* __restrict__ enc_in) {
    using S = typename P::S;
    constexpr int kWElems = 64 * LD32 + 64 * LD64 + 32 * LD64 + 64 * LD64 + 64 * LD16;
    __shared__ __align__(16) S sWraw[kWElems];
    S* sW1 = sWraw;
    S* sW2 = sW1 + 64 * LD32;
    S* sW1t = sW2 + 64 * LD64;
    S* sW2t = sW1t + 32 * LD64;
    S* sW3t = sW2t + 64 * LD64;
    // per wave: encoding, activations, their gradients, output gradient
    __shared__ S sX[kWaves][kPts * LD32], sH1[kWaves][kPts * LD64], sH2[kWaves][kPts * LD64];
    __shared__ S sD1[kWaves][kPts * LD64], sD2[kWaves][kPts * LD64];
    __shared__ S sO[kWaves][kPts * LD16];
    __shared__ float sE[kCSR ? 1 : kWaves][kPts * 33];
    __shared__ int sK[kWaves][3];   // each batch's scale exponents k0, k1, k2
    load_weights<P>(mlp, sW1, sW2, nullptr, sW1t, sW2t, sW3t);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = lane & 15, g = lane >> 4, col = lane & 15;
    S* X = sX[w];
    S* H1 = sH1[w];
    S* H2 = sH2[w];
    S* D1 = sD1[w];
    S* D2 = sD2[w];
    S* O = sO[w];
    float* E = sE[kCSR ? 0 : w];
    // this wave's weight-gradient tiles: dW1 rows 16 w.. (2 column tiles),
    // dW2 rows 16 w.. (4 column tiles), dW3 columns 16 w..
    f4v gW1[2], gW2[4], gW3;
    for (int a = 0; a < 2; a++) gW1[a] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int a = 0; a < 4; a++) gW2[a] = f4v{0.f, 0.f, 0.f, 0.f};
    gW3 = f4v{0.f, 0.f, 0.f, 0.f};
    // the level slices this lane writes in the level-major encoding gradient:
    // levels 2 g and 8 + 2 g (and the level after each)
    float2* dlev[2] = {nullptr, nullptr};
    if (kCSR) {
        dlev[0] = reinterpret_cast<float2*>(denc) + (int64_t)(2 * g) * n;
        dlev[1] = reinterpret_cast<float2*>(denc) + (int64_t)(8 + 2 * g) * n;
    }
    const int64_t nb = (n + kPts - 1) / kPts;
    // the inputs of this wave's batch are loaded one round ahead, so that
    // their latency overlaps the previous round's work
    float nmu[3] = {0.f, 0.f, 0.f}, ndv[4] = {0.f, 0.f, 0.f, 0.f};
    S nenc[8];
    auto prefetch = [&](int64_t bb) {
        const int64_t q = (bb + w) * kPts + p;
        if (bb < nb && q < n) {
            nmu[0] = means[3 * q];
            nmu[1] = means[3 * q + 1];
            nmu[2] = means[3 * q + 2];
            if (enc_in) {
#pragma unroll
                for (int j = 0; j < 8; j++) nenc[j] = enc_in[q * 32 + 8 * g + j];
            }
            if (g == 0) {
                ndv[0] = d_dmu[3 * q];
                ndv[1] = d_dmu[3 * q + 1];
                ndv[2] = d_dmu[3 * q + 2];
                ndv[3] = d_dq[4 * q];
            } else if (g == 1) {
                ndv[0] = d_dq[4 * q + 1];
                ndv[1] = d_dq[4 * q + 2];
                ndv[2] = d_dq[4 * q + 3];
            }
        }
    };
    prefetch((int64_t)blockIdx.x * kWaves);
    for (int64_t b0 = (int64_t)blockIdx.x * kWaves; b0 < nb; b0 += (int64_t)gridDim.x * kWaves) {
        // ---------------- phase A: this wave's batch ----------------
        const int64_t pt = (b0 + w) * kPts + p;
        const bool valid = pt < n;   // false for every lane of a wave past the last batch
        float x[3] = {0.f, 0.f, 0.f};
        bool in = false;
        if (valid) in = ntc_normalise(nd, nmu, x);
        // 1. encoding: the forward's, when it kept it, else recomputed
        if (enc_in && valid) {
#pragma unroll
            for (int j = 0; j < 8; j++) X[p * LD32 + 8 * g + j] = nenc[j];
        } else if (in) {
            encode_lane<P>(nd, table, x, g, X, p);
        } else {
            for (int j = 0; j < 8; j++) X[p * LD32 + 8 * g + j] = P::cvt(0.f);
        }
        // output gradient (lanes of group 0 own the 7 outputs of their point)
        float dv[4] = {0.f, 0.f, 0.f, 0.f};
        if (in && g <= 1) {
#pragma unroll
            for (int r = 0; r < 4; r++) dv[r] = ndv[r];
        }
        prefetch(b0 + (int64_t)gridDim.x * kWaves);
        // the activation gradients of this batch are held scaled by 2^k0,
        // 2^k1, 2^k2 (exact powers of two; the weight gradients unscale them)
        int k0 = 0;
        if (P::kScaled)
            k0 = clamp_exp(pow2_exp(wave_max(fmaxf(fmaxf(fabsf(dv[0]), fabsf(dv[1])), fmaxf(fabsf(dv[2]), fabsf(dv[3]))))));
        const float s0 = ldexpf(1.0f, k0);
        for (int r = 0; r < 4; r++) O[p * LD16 + 4 * g + r] = P::cvt(dv[r] * s0);   // rows 8..15 stay zero
        wave_sync();
        // 2. forward recompute
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            const f4v a = layer_tile<P, 32>(sW1, LD32, mt * 16, X, LD32, lane);
            for (int r = 0; r < 4; r++) H1[p * LD64 + mt * 16 + 4 * g + r] = P::cvt(fmaxf(a[r], 0.f));
        }
        wave_sync();
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            const f4v a = layer_tile<P, 64>(sW2, LD64, mt * 16, H1, LD64, lane);
            for (int r = 0; r < 4; r++) H2[p * LD64 + mt * 16 + 4 * g + r] = P::cvt(fmaxf(a[r], 0.f));
        }
        wave_sync();
        // 3. dH2 = (W3^T dO) * [H2 > 0]
        f4v d2[4];
        float m2 = 0.f;
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            d2[mt] = layer_tile<P, 16>(sW3t, LD16, mt * 16, O, LD16, lane);
            for (int r = 0; r < 4; r++) {
                const bool on = P::tof(H2[p * LD64 + mt * 16 + 4 * g + r]) > 0.f;
                d2[mt][r] = on ? d2[mt][r] : 0.f;
                m2 = fmaxf(m2, fabsf(d2[mt][r]));
            }
        }
        int k1 = k0;
        if (P::kScaled) k1 = clamp_exp(k0 + pow2_exp(wave_max(m2)));
        {
            const float f = ldexpf(1.0f, k1 - k0);
            for (int mt = 0; mt < 4; mt++)
                for (int r = 0; r < 4; r++) D2[p * LD64 + mt * 16 + 4 * g + r] = P::cvt(d2[mt][r] * f);
        }
        wave_sync();
        // 4. dH1 = (W2^T dH2) * [H1 > 0]
        f4v d1[4];
        float m1 = 0.f;
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            d1[mt] = layer_tile<P, 64>(sW2t, LD64, mt * 16, D2, LD64, lane);
            for (int r = 0; r < 4; r++) {
                const bool on = P::tof(H1[p * LD64 + mt * 16 + 4 * g + r]) > 0.f;
                d1[mt][r] = on ? d1[mt][r] : 0.f;
                m1 = fmaxf(m1, fabsf(d1[mt][r]));
            }
        }
        int k2 = k1;
        if (P::kScaled) k2 = clamp_exp(k1 + pow2_exp(wave_max(m1)));
        {
            const float f = ldexpf(1.0f, k2 - k1);
            for (int mt = 0; mt < 4; mt++)
                for (int r = 0; r < 4; r++) D1[p * LD64 + mt * 16 + 4 * g + r] = P::cvt(d1[mt][r] * f);
        }
        if (lane == 0) {
            sK[w][0] = k0;
            sK[w][1] = k1;
            sK[w][2] = k2;
        }
        wave_sync();
        // 5. dX = W1^T dH1: the encoding gradient
        {
            const float inv = ldexpf(1.0f, -k2);
#pragma unroll
            for (int mt = 0; mt < 2; mt++) {
                const f4v e = layer_tile<P, 64>(sW1t, LD64, mt * 16, D1, LD64, lane);
                if (kCSR) {
                    // level-major [level][point][2]: one level's slice (8 n bytes)
                    // stays cache-resident while the gather walks that level
                    if (valid) {
                        float2* d = dlev[mt] + pt;
                        d[0] = make_float2(e[0] * inv, e[1] * inv);
                        d[n] = make_float2(e[2] * inv, e[3] * inv);   // level lv + 1
                    }
                } else {
                    for (int r = 0; r < 4; r++) E[p * 33 + mt * 16 + 4 * g + r] = e[r] * inv;
                }
            }
        }
        if (!kCSR) {
            wave_sync();
            // 6. scatter-add the encoding gradient into the table gradient
            if (in) {
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int lv = 4 * g + j;
                    uint32_t ent[8];
                    float wt[8];
                    ntc_corners(nd, lv, x, ent, wt);
                    const float e0 = E[p * 33 + 2 * lv], e1 = E[p * 33 + 2 * lv + 1];
#pragma unroll
                    for (int c = 0; c < 8; c++) {
                        atomicAdd(g_table + 2 * (int64_t)ent[c], wt[c] * e0);
                        atomicAdd(g_table + 2 * (int64_t)ent[c] + 1, wt[c] * e1);
                    }
                }
            }
        }
        __syncthreads();
        // ---------------- phase B: weight gradients of the four batches ----------------
#pragma unroll
        for (int b = 0; b < kWaves; b++) {
            const float inv0 = ldexpf(1.0f, -sK[b][0]);
            const float inv1 = ldexpf(1.0f, -sK[b][1]);
            const float inv2 = ldexpf(1.0f, -sK[b][2]);
            // dW3[o][m] += sum_p dO[p][o] H2[p][m], columns m = 16 w..
            {
                f4v t = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < kPts / P::KSTEP; ks++) {
                    const int kk = ks * P::KSTEP + P::KPL * g;
                    t = P::mfma(frag_k_strided<P>(sO[b], LD16, col, kk),
                                frag_k_strided<P>(sH2[b], LD64, w * 16 + col, kk), t);
                }
                gW3 += t * inv0;
            }
            // dW2[m][k] += sum_p dH2[p][m] H1[p][k], rows m = 16 w..
#pragma unroll
            for (int nt = 0; nt < 4; nt++) {
                f4v t = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < kPts / P::KSTEP; ks++) {
                    const int kk = ks * P::KSTEP + P::KPL * g;
                    t = P::mfma(frag_k_strided<P>(sD2[b], LD64, w * 16 + col, kk),
                                frag_k_strided<P>(sH1[b], LD64, nt * 16 + col, kk), t);
                }
                gW2[nt] += t * inv1;
            }
            // dW1[m][k] += sum_p dH1[p][m] X[p][k], rows m = 16 w..
#pragma unroll
            for (int nt = 0; nt < 2; nt++) {
                f4v t = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < kPts / P::KSTEP; ks++) {
                    const int kk = ks * P::KSTEP + P::KPL * g;
                    t = P::mfma(frag_k_strided<P>(sD1[b], LD64, w * 16 + col, kk),
                                frag_k_strided<P>(sX[b], LD32, nt * 16 + col, kk), t);
                }
                gW1[nt] += t * inv2;
            }
        }
        __syncthreads();   // phase B's reads done before the next batches are written
    }
    // weight-gradient partials of this workgroup: every wave writes its own
    // tiles (they are disjoint and cover the MLP's parameters once)
    float* out = g_part + (int64_t)blockIdx.x * kMlpParams;
    for (int nt = 0; nt < 2; nt++)
        for (int r = 0; r < 4; r++) out[(w * 16 + 4 * g + r) * 32 + nt * 16 + col] = gW1[nt][r];
    for (int nt = 0; nt < 4; nt++)
        for (int r = 0; r < 4; r++) out[64 * 32 + (w * 16 + 4 * g + r) * 64 + nt * 16 + col] = gW2[nt][r];
    for (int r = 0; r < 4; r++)
        if (4 * g + r < 7) out[64 * 32 + 64 * 64 + (4 * g + r) * 64 + w * 16 + col] = gW3[r];
}

// ---------------------------------------------------------------------------
// Per-frame contribution lists.  The means are frozen during Stage 1, so
// every (point, level, corner) contribution to the table gradient has a fixed
// entry and a fixed trilinear weight for the whole frame.  They are sorted
// by entry once; each iteration then sums, per entry, weight x encoding
// gradient of the contributing points (no atomics, fixed summation order).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_csr_contrib(NtcDev nd, const float* __restrict__ means, int64_t n,
                                                     uint32_t sentinel, uint32_t* __restrict__ key,
                                                     uint32_t* __restrict__ pid) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;   // (point, level)
    if (t >= n * 16) return;
    const int64_t pt = t >> 4;
    const int lv = (int)(t & 15);
    const float mu[3] = {means[3 * pt], means[3 * pt + 1], means[3 * pt + 2]};
    float x[3];
    const bool in = ntc_normalise(nd, mu, x);
    uint32_t ent[8];
    float wt[8];
    ntc_corners(nd, lv, x, ent, wt);
    for (int c = 0; c < 8; c++) {
        key[8 * t + c] = in ? (uint32_t)ent[c] : sentinel;
        pid[8 * t + c] = ((uint32_t)pt << 7) | ((uint32_t)lv << 3) | (uint32_t)c;
    }
}

__global__ __launch_bounds__(256) void k_csr_rows(const uint32_t* __restrict__ key, int64_t m, uint32_t sentinel,
                                                  uint2* __restrict__ rows) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= m) return;
    const uint32_t e = key[k];
    if (e == sentinel) return;
    if (k == 0 || key[k - 1] != e) rows[e].x = (uint32_t)k;
    if (k == m - 1 || key[k + 1] != e) rows[e].y = (uint32_t)(k + 1);
}

__global__ __launch_bounds__(256) void k_csr_weights(NtcDev nd, const float* __restrict__ means,
                                                     const uint32_t* __restrict__ key, const uint32_t* __restrict__ pid,
                                                     int64_t m, uint32_t sentinel, uint2* __restrict__ pw) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= m) return;
    const uint32_t c = pid[k];
    if (key[k] == sentinel) {
        pw[k] = make_uint2(c, 0u);
        return;
    }
    const int64_t pt = c >> 7;
    const int lv = (c >> 3) & 15, corner = c & 7;
    const float mu[3] = {means[3 * pt], means[3 * pt + 1], means[3 * pt + 2]};
    float x[3];
    ntc_normalise(nd, mu, x);
    uint32_t ent[8];
    float wt[8];
    ntc_corners(nd, lv, x, ent, wt);
    pw[k] = make_uint2(c, __float_as_uint(wt[corner]));
}

// 16 lanes per table entry: the entry's (point, weight) contributions are
// read 16 at a time (coalesced, one 8-byte load each), each lane gathers its
// point's encoding gradient, and the group sums with DPP (pairs, quads,
// half-row and row mirror): fixed order.
//
// Every level takes the same number of contributions (8 per point) and reads
// only its own slice of the encoding gradient (n x 8 bytes).  Workgroups are
// handed to the 8 XCDs in turn, so workgroup b runs on XCD b mod 8; the grid
// gives XCD x the entries of levels x and 15 - x (a coarse level with few,
// long rows and a fine one with many short rows), one level after the other.
// Each XCD then fetches two slices of the encoding gradient into its own L2
// instead of all sixteen.  The placement is a performance choice only: the
// result does not depend on where a workgroup runs.
constexpr int kGatherLanes = 16;
constexpr int kGatherEntries = 256 / kGatherLanes;   // entries per workgroup
constexpr int kXcds = 8;

struct GatherLevels {
    int64_t begin[16];   // first entry of each level
    int64_t end[16];     // one past its last entry
};

static int64_t gather_blocks(const GatherLevels& gl, int lv) {
    return (gl.end[lv] - gl.begin[lv] + kGatherEntries - 1) / kGatherEntries;
}

__global__ __launch_bounds__(256) void k_csr_gather(GatherLevels gl, const uint2* __restrict__ rows,
                                                    const uint2* __restrict__ pw, const float* __restrict__ denc,
                                                    int64_t n, float* __restrict__ g_table) {
    const int x = (int)(blockIdx.x % kXcds);
    int64_t j = blockIdx.x / kXcds;   // this workgroup's place among its XCD's
    int lv = x;
    const int64_t na = (gl.end[lv] - gl.begin[lv] + kGatherEntries - 1) / kGatherEntries;
    if (j >= na) {
        j -= na;
        lv = 15 - x;
    }
    const int64_t e = gl.begin[lv] + j * kGatherEntries + threadIdx.x / kGatherLanes;
    const bool valid = e < gl.end[lv];
    const int sub = threadIdx.x % kGatherLanes;
    uint2 r = make_uint2(0u, 0u);
    if (valid) r = rows[e];
    float a0 = 0.f, a1 = 0.f;
    auto enc = [&](uint32_t c) {
        return *reinterpret_cast<const float2*>(denc + 2 * ((int64_t)((c >> 3) & 15) * n + (c >> 7)));
    };
    uint32_t k = r.x + sub;
    // four independent contribution loads in flight per lane; the sum keeps
    // the order k, k + 16, k + 32, ...
    constexpr int G = kGatherLanes;
    for (; k + 3 * G < r.y; k += 4 * G) {
        const uint2 c0 = pw[k], c1 = pw[k + G], c2 = pw[k + 2 * G], c3 = pw[k + 3 * G];
        const float2 d0 = enc(c0.x), d1 = enc(c1.x), d2 = enc(c2.x), d3 = enc(c3.x);
        const float w0 = __uint_as_float(c0.y), w1 = __uint_as_float(c1.y);
        const float w2 = __uint_as_float(c2.y), w3 = __uint_as_float(c3.y);
        a0 += w0 * d0.x;
        a1 += w0 * d0.y;
        a0 += w1 * d1.x;
        a1 += w1 * d1.y;
        a0 += w2 * d2.x;
        a1 += w2 * d2.y;
        a0 += w3 * d3.x;
        a1 += w3 * d3.y;
    }
    for (; k < r.y; k += G) {
        const uint2 c = pw[k];
        const float2 d = enc(c.x);
        const float wk = __uint_as_float(c.y);
        a0 += wk * d.x;
        a1 += wk * d.y;
    }
    a0 = dpp_add<0xB1, 0xF>(a0);    // quad_perm [1,0,3,2]
    a0 = dpp_add<0x4E, 0xF>(a0);    // quad_perm [2,3,0,1]
    a0 = dpp_add<0x141, 0xF>(a0);   // row_half_mirror
    a0 = dpp_add<0x140, 0xF>(a0);   // row_mirror: lane 0 of the row holds the sum
    a1 = dpp_add<0xB1, 0xF>(a1);
    a1 = dpp_add<0x4E, 0xF>(a1);
    a1 = dpp_add<0x141, 0xF>(a1);
    a1 = dpp_add<0x140, 0xF>(a1);
    if (sub == 0 && valid && r.y > r.x) {
        g_table[2 * e] += a0;
        g_table[2 * e + 1] += a1;
    }
}

// Sum the per-workgroup weight-gradient rows: blockIdx.y takes a slice of
// the rows, blockIdx.x a range of columns; one atomic per (slice, column).
constexpr int kPartSlice = 32;
__global__ __launch_bounds__(256) void k_reduce_parts(const float* __restrict__ part, int nparts, int len,
                                                      float* __restrict__ dst) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= len) return;
    const int b0 = blockIdx.y * kPartSlice;
    const int b1 = min(b0 + kPartSlice, nparts);
    // eight loads in flight, summed in order
    float s = 0.f;
    int b = b0;
    for (; b + 8 <= b1; b += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = part[(int64_t)(b + u) * len + k];
#pragma unroll
        for (int u = 0; u < 8; u++) s += v[u];
    }
    for (; b < b1; b++) s += part[(int64_t)b * len + k];
    atomicAdd(dst + k, s);
}

template <class P>
__global__ __launch_bounds__(256) void k_ntc_adam(float* __restrict__ p, float* __restrict__ gr, float* __restrict__ m,
                                                  float* __restrict__ v, typename P::S* __restrict__ work, int64_t n,
                                                  float lr, float b1, float b2, float eps, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    gr[i] = 0.f;
    if (work) work[i] = P::cvt(pi);
}

template <class P>
__global__ __launch_bounds__(256) void k_to_work(const float* __restrict__ p, typename P::S* __restrict__ work,
                                                 int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) work[i] = P::cvt(p[i]);
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ gr,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                              float b1, float b2, float eps, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Eq. 7 per point, plus per-block partial sums of the loss
__global__ __launch_bounds__(256) void k_warmup(const float* __restrict__ dmu, const float* __restrict__ dq, int64_t n,
                                                float* __restrict__ gmu, float* __restrict__ gq,
                                                double* __restrict__ bsum) {
    __shared__ double s[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double L = 0.0;
    if (i < n) {
        const float invn = 1.0f / (float)n;
        float a = 0.f;
        for (int k = 0; k < 3; k++) {
            const float d = dmu[3 * i + k];
            a += fabsf(d);
            gmu[3 * i + k] = (d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f)) * invn;
        }
        const float w = dq[4 * i], x = dq[4 * i + 1], y = dq[4 * i + 2], z = dq[4 * i + 3];
        const float n2 = w * w + x * x + y * y + z * z;
        float c2 = 0.f;
        if (n2 > 0.f) {
            c2 = w * w / n2;
            const float i4 = 1.0f / (n2 * n2);
            gq[4 * i] = -(2.f * w * (n2 - w * w) * i4) * invn;
            gq[4 * i + 1] = (2.f * w * w * x * i4) * invn;
            gq[4 * i + 2] = (2.f * w * w * y * i4) * invn;
            gq[4 * i + 3] = (2.f * w * w * z * i4) * invn;
        } else {
            for (int k = 0; k < 4; k++) gq[4 * i + k] = 0.f;
        }
        L = (double)a - (double)c2;
    }
    for (int off = 32; off > 0; off >>= 1) L += __shfl_xor(L, off, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = L;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

__global__ __launch_bounds__(256) void k_warmup_finalize(const double* __restrict__ bsum, int64_t nb, int64_t n,
                                                         float* __restrict__ loss) {
    __shared__ double s[4];
    double a = 0.0;
    for (int64_t k = threadIdx.x; k < nb; k += 256) a += bsum[k];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) loss[0] = (float)((s[0] + s[1] + s[2] + s[3]) / (double)n);
}

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

template <class P>
void fwd_impl(const Launch& L, const NtcDev& nd, const void* table, const void* mlp, const float* means, int64_t n,
              float* dmu, float* dq, void* enc_out) {
    const int64_t nb = (n + kPts - 1) / kPts;
    // four workgroups per CU are resident (LDS-bound) on 256 CUs: one round of
    // workgroups, each looping over its share of the batches
    const unsigned grid = (unsigned)std::min<int64_t>((nb + kWaves - 1) / kWaves, 1024);
    hipLaunchKernelGGL((k_ntc_fwd<P>), dim3(grid), dim3(256), 0, L.st, nd, (const typename P::S*)table,
                       (const typename P::S*)mlp, means, n, dmu, dq, (typename P::S*)enc_out);
}

template <class P>
void bwd_impl(const Launch& L, const NtcDev& nd, const void* table, const void* mlp, const float* means, int64_t n,
              const float* d_dmu, const float* d_dq, float* g_table, float* g_mlp, float* g_part, int max_parts,
              const NtcCsr* csr, const void* enc_in) {
    const int64_t nb = (n + kPts - 1) / kPts;
    // max_parts is two per CU: the half-precision kernels fit two workgroups
    // on a CU, the float32 one (twice the LDS) one
    const int parts = sizeof(typename P::S) == 4 ? max_parts / 2 : max_parts;
    const unsigned grid = (unsigned)std::min<int64_t>((nb + kWaves - 1) / kWaves, parts);
    if (csr) {
        hipLaunchKernelGGL((k_ntc_bwd<P, true>), dim3(grid), dim3(256), 0, L.st, nd, (const typename P::S*)table,
                           (const typename P::S*)mlp, means, n, d_dmu, d_dq, g_table, g_part, csr->denc,
                           (const typename P::S*)enc_in);
        if (L.prof) L.prof->end(L.st);
        if (L.prof) L.prof->begin("ntc_scatter", L.st);
        GatherLevels gl;
        for (int lv = 0; lv < 16; lv++) {
            gl.begin[lv] = nd.off[lv];
            gl.end[lv] = lv < 15 ? nd.off[lv + 1] : csr->entries;
        }
        int64_t per_xcd = 0;
        for (int x = 0; x < kXcds; x++)
            per_xcd = std::max(per_xcd, gather_blocks(gl, x) + gather_blocks(gl, 15 - x));
        hipLaunchKernelGGL(k_csr_gather, dim3((unsigned)(per_xcd * kXcds)), dim3(256), 0, L.st, gl, csr->rows,
                           csr->pw, csr->denc, n, g_table);
    } else {
        hipLaunchKernelGGL((k_ntc_bwd<P, false>), dim3(grid), dim3(256), 0, L.st, nd, (const typename P::S*)table,
                           (const typename P::S*)mlp, means, n, d_dmu, d_dq, g_table, g_part, (float*)nullptr,
                           (const typename P::S*)enc_in);
    }
    hipLaunchKernelGGL(k_reduce_parts, dim3(nblk(kMlpParams, 256), (grid + kPartSlice - 1) / kPartSlice), dim3(256), 0,
                       L.st, g_part, (int)grid, kMlpParams, g_mlp);
}

}  // namespace

int ntc_mlp_params() { return kMlpParams; }

void ntc_forward(const Launch& L, int precision, const NtcDev& nd, const void* table, const void* mlp,
                 const float* means, int64_t n, float* dmu, float* dq, void* enc_out) {
    if (n <= 0) return;
    if (L.prof) L.prof->begin("ntc_fwd", L.st);
    if (precision == 1)
        fwd_impl<PF16>(L, nd, table, mlp, means, n, dmu, dq, enc_out);
    else if (precision == 2)
        fwd_impl<PBF16>(L, nd, table, mlp, means, n, dmu, dq, enc_out);
    else
        fwd_impl<PF32>(L, nd, table, mlp, means, n, dmu, dq, enc_out);
    if (L.prof) L.prof->end(L.st);
}

void ntc_backward(const Launch& L, int precision, const NtcDev& nd, const void* table, const void* mlp,
                  const float* means, int64_t n, const float* d_dmu, const float* d_dq, float* g_table, float* g_mlp,
                  float* g_part, int max_parts, const NtcCsr* csr, const void* enc_in) {
    if (n <= 0) return;
    if (L.prof) L.prof->begin("ntc_bwd", L.st);
    if (precision == 1)
        bwd_impl<PF16>(L, nd, table, mlp, means, n, d_dmu, d_dq, g_table, g_mlp, g_part, max_parts, csr, enc_in);
    else if (precision == 2)
        bwd_impl<PBF16>(L, nd, table, mlp, means, n, d_dmu, d_dq, g_table, g_mlp, g_part, max_parts, csr, enc_in);
    else
        bwd_impl<PF32>(L, nd, table, mlp, means, n, d_dmu, d_dq, g_table, g_mlp, g_part, max_parts, csr, enc_in);
    if (L.prof) L.prof->end(L.st);
}

void ntc_csr_build(const Launch& L, const NtcDev& nd, const float* means, int64_t n, NtcCsr& csr, uint32_t* keys[2],
                   uint32_t* vals[2], uint32_t* hist, uint64_t* tmp) {
    const int64_t m = n * 128;
    const uint32_t sentinel = (uint32_t)csr.entries;
    int bits = 1;
    while (((int64_t)1 << bits) <= csr.entries) bits++;
    if (L.prof) L.prof->begin("ntc_prepare", L.st);
    hipLaunchKernelGGL(k_csr_contrib, dim3(nblk(n * 16, 256)), dim3(256), 0, L.st, nd, means, n, sentinel, keys[0],
                       vals[0]);
    Launch inner{L.st, nullptr};
    const int r = radix_sort_u32(inner, keys, vals, m, bits, hist, tmp);
    csr.pid = vals[r];
    fill_u32(inner, reinterpret_cast<uint32_t*>(csr.rows), 0u, 2 * csr.entries);
    hipLaunchKernelGGL(k_csr_rows, dim3(nblk(m, 256)), dim3(256), 0, L.st, keys[r], m, sentinel, csr.rows);
    hipLaunchKernelGGL(k_csr_weights, dim3(nblk(m, 256)), dim3(256), 0, L.st, nd, means, keys[r], csr.pid, m, sentinel,
                       csr.pw);
    if (L.prof) L.prof->end(L.st);
}

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) used as a counter-based generator: output i of
// the stream seeded with `seed` is the generator's mixing function applied to
// seed + (i + 1) * 0x9E3779B97F4A7C15.
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Parameter i = bound * (2u - 1) with u the top 24 bits of output i over
// 2^24 (exact in float32, so 2u - 1 is exact and the product rounds once).
// bound: b_table for the table, then b_w1 / b_w2 / b_w3 for the three
// weight matrices (n_w1, n_w2 entries; the rest W3).
__global__ __launch_bounds__(256) void k_ntc_init(float* __restrict__ p, int64_t n, int64_t n_table, int64_t n_w1,
                                                  int64_t n_w2, float b_table, float b_w1, float b_w2, float b_w3,
                                                  uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t j = i - n_table;
    const float b = j < 0 ? b_table : j < n_w1 ? b_w1 : j < n_w1 + n_w2 ? b_w2 : b_w3;
    const float u = (float)(uint32_t)(splitmix64_at(seed, (uint64_t)i) >> 40) * 0x1p-24f;
    p[i] = b * (2.0f * u - 1.0f);
}

void ntc_init(const Launch& L, float* p, int64_t n, int64_t n_table, uint64_t seed) {
    // U(-1e-4, 1e-4) for the table (instant-NGP's), Kaiming-uniform
    // U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)) for W1 (fan-in 32), W2, W3 (64)
    const float b_table = 1e-4f, b_w1 = (float)sqrt(6.0 / 32.0), b_w2 = (float)sqrt(6.0 / 64.0);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_ntc_init, dim3(nblk(n, 256)), dim3(256), 0, L.st, p, n, n_table, (int64_t)64 * 32,
                       (int64_t)64 * 64, b_table, b_w1, b_w2, b_w2, seed);
}

void ntc_adam(const Launch& L, int precision, float* p, float* g, float* m, float* v, void* work, int64_t n, float lr,
              float b1, float b2, float eps, float bc1, float bc2) {
    if (L.prof) L.prof->begin("ntc_adam", L.st);
    if (precision == 1)
        hipLaunchKernelGGL((k_ntc_adam<PF16>), dim3(nblk(n, 256)), dim3(256), 0, L.st, p, g, m, v, (_Float16*)work, n,
                           lr, b1, b2, eps, bc1, bc2);
    else if (precision == 2)
        hipLaunchKernelGGL((k_ntc_adam<PBF16>), dim3(nblk(n, 256)), dim3(256), 0, L.st, p, g, m, v, (__bf16*)work, n,
                           lr, b1, b2, eps, bc1, bc2);
    else
        hipLaunchKernelGGL((k_ntc_adam<PF32>), dim3(nblk(n, 256)), dim3(256), 0, L.st, p, g, m, v, (float*)nullptr, n,
                           lr, b1, b2, eps, bc1, bc2);
    if (L.prof) L.prof->end(L.st);
}

void ntc_refresh_work(const Launch& L, int precision, const float* p, void* work, int64_t n) {
    if (precision == 1)
        hipLaunchKernelGGL((k_to_work<PF16>), dim3(nblk(n, 256)), dim3(256), 0, L.st, p, (_Float16*)work, n);
    else if (precision == 2)
        hipLaunchKernelGGL((k_to_work<PBF16>), dim3(nblk(n, 256)), dim3(256), 0, L.st, p, (__bf16*)work, n);
}

void adam(const Launch& L, float* p, const float* g, float* m, float* v, int64_t n, int step, float lr, float b1,
          float b2, float eps) {
    if (n <= 0) return;
    const float bc1 = (float)(1.0 - pow((double)b1, (double)step));
    const float bc2 = (float)(1.0 - pow((double)b2, (double)step));
    if (L.prof) L.prof->begin("adam", L.st);
    hipLaunchKernelGGL(k_adam, dim3(nblk(n, 256)), dim3(256), 0, L.st, p, g, m, v, n, lr, b1, b2, eps, bc1, bc2);
    if (L.prof) L.prof->end(L.st);
}

void warmup_loss(const Launch& L, const float* dmu, const float* dq, int64_t n, float* loss, float* gmu, float* gq,
                 double* bsum) {
    if (n <= 0) return;
    if (L.prof) L.prof->begin("warmup_loss", L.st);
    const unsigned nb = nblk(n, 256);
    hipLaunchKernelGGL(k_warmup, dim3(nb), dim3(256), 0, L.st, dmu, dq, n, gmu, gq, bsum);
    hipLaunchKernelGGL(k_warmup_finalize, dim3(1), dim3(256), 0, L.st, bsum, (int64_t)nb, n, loss);
    if (L.prof) L.prof->end(L.st);
}

}  // namespace gs3
