// NTC launchers (internal to libgs3.so).
#pragma once
#include "kernels.h"

namespace gs3 {

// Shape of the hash encoding, passed by value to kernels.
struct NtcDev {
    int res[16];           // grid resolution per level
    int64_t off[16];       // first table entry of each level
    uint32_t dense_mask;   // bit l set: level l is stored densely
    uint32_t T_mask;       // 2^log2_T - 1
    float aabb_min[3];
    float inv_ext[3];
};

// Per-frame contribution lists of the table gradient (see ntc.hip).
struct NtcCsr {
    int64_t entries = 0;      // table entries
    uint2* rows = nullptr;    // [entries]: [start, end) into pw
    uint32_t* pid = nullptr;  // point << 7 | level << 3 | corner, sorted by entry
    uint2* pw = nullptr;      // (pid, float bits of the trilinear weight) of each contribution
    float* denc = nullptr;    // [16 levels][n][2] encoding gradient of the current backward
};

int ntc_mlp_params();
// keys/vals: two ping-pong buffers of n * 128 u32 each; hist: radix_hist_words(n * 128)
void ntc_csr_build(const Launch& L, const NtcDev& nd, const float* means, int64_t n, NtcCsr& csr, uint32_t* keys[2],
                   uint32_t* vals[2], uint32_t* hist, uint64_t* tmp);
// enc_out (optional, n x 32 values of the working precision): the forward
// also stores each point's encoding there
void ntc_forward(const Launch& L, int precision, const NtcDev& nd, const void* table, const void* mlp,
                 const float* means, int64_t n, float* dmu, float* dq, void* enc_out);
// g_part holds max_parts x ntc_mlp_params() floats; enc_in (optional): the
// encoding a forward with the same parameters and means stored, used instead
// of recomputing it
void ntc_backward(const Launch& L, int precision, const NtcDev& nd, const void* table, const void* mlp,
                  const float* means, int64_t n, const float* d_dmu, const float* d_dq, float* g_table, float* g_mlp,
                  float* g_part, int max_parts, const NtcCsr* csr, const void* enc_in);
void ntc_adam(const Launch& L, int precision, float* p, float* g, float* m, float* v, void* work, int64_t n, float lr,
              float b1, float b2, float eps, float bc1, float bc2);
// float32 master parameters [table | W1 | W2 | W3] from a counter-based
// generator (SplitMix64) seeded with `seed`
void ntc_init(const Launch& L, float* p, int64_t n, int64_t n_table, uint64_t seed);
void ntc_refresh_work(const Launch& L, int precision, const float* p, void* work, int64_t n);
void warmup_loss(const Launch& L, const float* dmu, const float* dq, int64_t n, float* loss, float* gmu, float* gq,
                 double* bsum);

}  // namespace gs3
