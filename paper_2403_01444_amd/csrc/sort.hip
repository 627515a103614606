// Prefix sums and a stable LSD radix sort for gfx950 (wave64).
//
// Scan: per-block reduce, then a per-block rescan with the block prefix;
// each block of the rescan adds up the sums of the blocks before it (up to
// 2048 blocks; above that a single-block scan of the block sums runs in
// between).  Each block owns 2048 consecutive items (256 threads x 8).  Up
// to eight blocks' worth of items (the per-tile totals of a view, for
// instance) take one kernel: a single block walks them 2048 at a time with
// a running carry.
//
// Radix sort: 8-bit digits, one histogram kernel and one scatter kernel per
// pass.  A block owns 256 x I consecutive items (I = 8, or 4 for inputs
// under kSmallSort items so that the launch still covers the chip); wave w
// takes the 64 I items starting at w 64 I in I rounds of 64.  Inside a round the lanes that
// share a digit are found with eight ballots (one per digit bit); a lane's
// rank is the number of earlier lanes with its digit plus the wave's running
// count for that digit.  Items keep their order (block, wave, round, lane),
// so each pass is stable and the sort orders ties by their input position.
#include "kernels.h"

namespace gs3 {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTileItems = kThreads * kItems;

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t x, int lane) {
    for (int off = 1; off < 64; off <<= 1) {
        uint64_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// A thread's kItems consecutive inputs: two 16-byte loads when they are all
// in range and the array is 16-byte aligned, else one by one.
__device__ __forceinline__ void load8(const uint32_t* __restrict__ in, int64_t base, int64_t n, uint32_t v[kItems]) {
    if (base + kItems <= n && ((reinterpret_cast<uintptr_t>(in) & 15u) == 0)) {
        const uint4 a = *reinterpret_cast<const uint4*>(in + base);
        const uint4 b = *reinterpret_cast<const uint4*>(in + base + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < kItems; k++) v[k] = base + k < n ? in[base + k] : 0u;
    }
}

template <typename Tin>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const Tin* __restrict__ in, int64_t n,
                                                          uint64_t* __restrict__ bsum) {
    __shared__ uint64_t s_w[kThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kTileItems + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    load8(in, base, n, v);
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; k++) s += (uint64_t)v[k];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kThreads / 64; w++) t += s_w[w];
        bsum[blockIdx.x] = t;
    }
}

// One block: exclusive scan of nb block sums in place; total to *total.
__global__ __launch_bounds__(kThreads) void k_scan_bsums(uint64_t* __restrict__ bsum, int64_t nb,
                                                         uint64_t* __restrict__ total) {
    __shared__ uint64_t s_w[kThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kThreads) {
        int64_t i = b0 + threadIdx.x;
        uint64_t v = i < nb ? bsum[i] : 0;
        uint64_t x = wave_incl_scan(v, lane);
        if (lane == 63) s_w[w] = x;
        __syncthreads();
        uint64_t pre = 0, tot = 0;
        for (int k = 0; k < kThreads / 64; k++) {
            if (k < w) pre += s_w[k];
            tot += s_w[k];
        }
        if (i < nb) bsum[i] = carry + pre + x - v;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// bpre: the exclusive prefix of the block sums (k_scan_bsums), or, with
// kSelf, the raw block sums (k_scan_reduce): the block then adds up those of
// the blocks before it itself (nb of them at most kSelfPrefixBlocks) and the
// last block writes the total, one launch fewer than k_scan_bsums.
constexpr int64_t kSelfPrefixBlocks = 2048;

template <typename Tin, typename Tout, bool kSelf>
__global__ __launch_bounds__(kThreads) void k_scan_down(const Tin* __restrict__ in, int64_t n,
                                                        const uint64_t* __restrict__ bpre, Tout* __restrict__ out,
                                                        uint64_t* __restrict__ total) {
    __shared__ uint64_t s_w[kThreads / 64];
    __shared__ uint64_t s_p[kThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kTileItems + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    load8(in, base, n, v);
    uint64_t bp = 0;
    if (kSelf) {
        for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += kThreads) bp += bpre[b];
        for (int off = 32; off > 0; off >>= 1) bp += __shfl_xor(bp, off, 64);
        if (lane == 0) s_p[w] = bp;
    }
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; k++) s += (uint64_t)v[k];
    uint64_t x = wave_incl_scan(s, lane);
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint64_t pre;
    if (kSelf) {
        pre = 0;
        for (int k = 0; k < kThreads / 64; k++) pre += s_p[k];
        if (threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) {
            uint64_t t = pre;
            for (int k = 0; k < kThreads / 64; k++) t += s_w[k];
            *total = t;
        }
    } else {
        pre = bpre[blockIdx.x];
    }
    for (int k = 0; k < w; k++) pre += s_w[k];
    uint64_t run = pre + x - s;
    Tout o[kItems];
#pragma unroll
    for (int k = 0; k < kItems; k++) {
        o[k] = (Tout)run;
        run += v[k];
    }
    if (base + kItems <= n && ((reinterpret_cast<uintptr_t>(out) & 15u) == 0)) {
        // 16-byte stores of the thread's consecutive outputs
        constexpr int kPer = 16 / (int)sizeof(Tout);
#pragma unroll
        for (int k = 0; k < kItems; k += kPer) {
            if constexpr (sizeof(Tout) == 8)
                *reinterpret_cast<ulonglong2*>(out + base + k) = make_ulonglong2(o[k], o[k + 1]);
            else
                *reinterpret_cast<uint4*>(out + base + k) = make_uint4(o[k], o[k + 1], o[k + 2], o[k + 3]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < kItems; k++)
            if (base + k < n) out[base + k] = o[k];
    }
}

// Inputs of at most kSmallScan items: one block walks them kTileItems at a
// time with a running carry (one launch instead of three).
constexpr int64_t kSmallScan = 8 * kTileItems;

template <typename Tout>
__global__ __launch_bounds__(kThreads) void k_scan_single(const uint32_t* __restrict__ in, int64_t n,
                                                          Tout* __restrict__ out, uint64_t* __restrict__ total) {
    __shared__ uint64_t s_w[kThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t carry = 0;
    for (int64_t b0 = 0; b0 < n; b0 += kTileItems) {
        const int64_t base = b0 + (int64_t)threadIdx.x * kItems;
        uint32_t v[kItems];
        load8(in, base, n, v);
        uint64_t s = 0;
#pragma unroll
        for (int k = 0; k < kItems; k++) s += (uint64_t)v[k];
        const uint64_t x = wave_incl_scan(s, lane);
        if (lane == 63) s_w[w] = x;
        __syncthreads();
        uint64_t pre = carry, tot = 0;
        for (int k = 0; k < kThreads / 64; k++) {
            if (k < w) pre += s_w[k];
            tot += s_w[k];
        }
        uint64_t run = pre + x - s;
#pragma unroll
        for (int k = 0; k < kItems; k++) {
            if (base + k < n) out[base + k] = (Tout)run;
            run += v[k];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// Tile ranges of the chunk-major pair list from the pairs per tile: one
// block walks the counts with a running carry (as k_scan_single) and writes
// ranges[t] = [start, start + len[t]) clamped to cap; the first thread also
// flags an overflow when the list's total exceeds cap.
__global__ __launch_bounds__(kThreads) void k_scan_ranges(const uint32_t* __restrict__ len, int64_t n, uint64_t cap,
                                                          const uint64_t* __restrict__ total,
                                                          uint2* __restrict__ ranges, int* __restrict__ overflow) {
    __shared__ uint64_t s_w[kThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0 && *total > cap) atomicOr(overflow, 1);
    uint64_t carry = 0;
    for (int64_t b0 = 0; b0 < n; b0 += kTileItems) {
        const int64_t base = b0 + (int64_t)threadIdx.x * kItems;
        uint32_t v[kItems];
        load8(len, base, n, v);
        uint64_t s = 0;
#pragma unroll
        for (int k = 0; k < kItems; k++) s += (uint64_t)v[k];
        const uint64_t x = wave_incl_scan(s, lane);
        if (lane == 63) s_w[w] = x;
        __syncthreads();
        uint64_t pre = carry, tot = 0;
        for (int k = 0; k < kThreads / 64; k++) {
            if (k < w) pre += s_w[k];
            tot += s_w[k];
        }
        uint64_t run = pre + x - s;
#pragma unroll
        for (int k = 0; k < kItems; k++) {
            const uint64_t e = run + v[k];
            if (base + k < n) ranges[base + k] = make_uint2((uint32_t)(run < cap ? run : cap), (uint32_t)(e < cap ? e : cap));
            run = e;
        }
        carry += tot;
        __syncthreads();
    }
}

template <typename Tout>
void scan_impl(const Launch& L, const uint32_t* in, int64_t n, Tout* out, uint64_t* total, uint64_t* tmp) {
    int64_t nb = (n + kTileItems - 1) / kTileItems;
    if (nb == 0) {
        hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(kThreads), 0, L.st, tmp, (int64_t)0, total);
        return;
    }
    if (L.prof) L.prof->begin("scan", L.st);
    if (n <= kSmallScan) {
        hipLaunchKernelGGL((k_scan_single<Tout>), dim3(1), dim3(kThreads), 0, L.st, in, n, out, total);
        if (L.prof) L.prof->end(L.st);
        return;
    }
    hipLaunchKernelGGL((k_scan_reduce<uint32_t>), dim3((unsigned)nb), dim3(kThreads), 0, L.st, in, n, tmp);
    if (nb <= kSelfPrefixBlocks) {
        hipLaunchKernelGGL((k_scan_down<uint32_t, Tout, true>), dim3((unsigned)nb), dim3(kThreads), 0, L.st, in, n,
                           tmp, out, total);
    } else {
        hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(kThreads), 0, L.st, tmp, nb, total);
        hipLaunchKernelGGL((k_scan_down<uint32_t, Tout, false>), dim3((unsigned)nb), dim3(kThreads), 0, L.st, in, n,
                           tmp, out, total);
    }
    if (L.prof) L.prof->end(L.st);
}

__device__ __forceinline__ uint64_t match_digit(uint32_t d) {
    uint64_t m = ~0ull;
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

template <typename K, int I>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const K* __restrict__ keys, int64_t n, int shift,
                                                         uint32_t* __restrict__ hist, int64_t nblocks) {
    __shared__ uint32_t s_h[256];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * (kThreads * I) + w * (64 * I);
    for (int r = 0; r < I; r++) {
        const int64_t idx = base + r * 64 + lane;
        const bool valid = idx < n;
        const uint32_t d = valid ? (uint32_t)(keys[idx] >> shift) & 0xFFu : 0u;
        const uint64_t peers = match_digit(d) & __ballot(valid);
        if (valid && __popcll(peers & ((1ull << lane) - 1ull)) == 0) atomicAdd(&s_h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = s_h[threadIdx.x];
}

// offs: per (digit, block) output offsets; with dtotal (per-digit scan) they
// are relative to the digit's base, which the block adds from the totals.
template <typename K, int I>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                            K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                            int64_t n, int shift, const uint32_t* __restrict__ offs,
                                                            int64_t nblocks, const uint32_t* __restrict__ dtotal) {
    __shared__ uint32_t s_cnt[4][256];
    __shared__ uint32_t s_base[4][256];
    __shared__ uint32_t s_dw[4];
    for (int k = threadIdx.x; k < 4 * 256; k += kThreads) (&s_cnt[0][0])[k] = 0;
    uint32_t dbase = 0;   // exclusive prefix of the digit totals at digit threadIdx.x
    if (dtotal) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const uint32_t v = dtotal[threadIdx.x];
        const uint32_t x = wave_incl_scan_u32(v);
        if (lane == 63) s_dw[w] = x;
        __syncthreads();
        dbase = x - v;
        for (int k = 0; k < w; k++) dbase += s_dw[k];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * (kThreads * I) + w * (64 * I);
    K key[I];
    uint32_t val[I], rank[I], dig[I];
#pragma unroll
    for (int r = 0; r < I; r++) {
        const int64_t idx = base + r * 64 + lane;
        const bool valid = idx < n;
        key[r] = valid ? kin[idx] : (K)0;
        val[r] = valid ? (vin ? vin[idx] : (uint32_t)idx) : 0u;   // no values: the input positions
        const uint32_t d = (uint32_t)(key[r] >> shift) & 0xFFu;
        dig[r] = d;
        const uint64_t peers = match_digit(d) & __ballot(valid);
        const uint32_t before = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
        const uint32_t cur = s_cnt[w][d];
        rank[r] = cur + before;
        if (valid && before == 0) s_cnt[w][d] = cur + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        uint32_t run = dbase + offs[(int64_t)d * nblocks + blockIdx.x];
        for (int k = 0; k < 4; k++) {
            s_base[k][d] = run;
            run += s_cnt[k][d];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < I; r++) {
        const int64_t idx = base + r * 64 + lane;
        const uint32_t pos = s_base[w][dig[r]] + rank[r];
        if (idx < n && pos < (uint64_t)n) {   // pos < n always holds for consistent counts
            kout[pos] = key[r];
            vout[pos] = val[r];
        }
    }
}

// One wave per digit d: exclusive scan over the blocks of hist[d][0..nb) in
// place, the digit's total to dtotal[d].  With the totals, the scatter adds
// the digit's base (the totals of the smaller digits) itself.
__global__ __launch_bounds__(64) void k_radix_digit_scan(uint32_t* __restrict__ hist, int64_t nb,
                                                         uint32_t* __restrict__ dtotal) {
    uint32_t* h = hist + (int64_t)blockIdx.x * nb;
    const int lane = threadIdx.x;
    uint32_t carry = 0;
    for (int64_t i0 = 0; i0 < nb; i0 += 64) {
        const int64_t i = i0 + lane;
        const uint32_t v = i < nb ? h[i] : 0u;
        const uint32_t x = wave_incl_scan_u32(v);
        if (i < nb) h[i] = carry + x - v;
        carry += lane63_u32(x);
    }
    if (lane == 0) dtotal[blockIdx.x] = carry;
}

// blocks per pass up to which the per-digit scan is used
constexpr int64_t kDigitScanBlocks = 4096;

// first: the keys the first pass reads (left unchanged; its output goes to
// keys[1] as usual), or null to start from keys[0].  iota: the first pass
// takes the input positions as values instead of reading vals[0].
template <typename K, int I>
int radix_passes(const Launch& L, const K* first, bool iota, K* keys[2], uint32_t* vals[2], int64_t n, int bits,
                 uint32_t* hist, uint64_t* tmp) {
    int cur = 0;
    const int64_t nb = (n + kThreads * I - 1) / (kThreads * I);
    const int64_t hn = nb * 256;
    for (int shift = 0; shift < bits; shift += 8) {
        if (L.prof) L.prof->begin("radix_pass", L.st);
        const K* kin = shift == 0 && first ? first : keys[cur];
        const uint32_t* vin = shift == 0 && iota ? nullptr : vals[cur];
        hipLaunchKernelGGL((k_radix_hist<K, I>), dim3((unsigned)nb), dim3(kThreads), 0, L.st, kin, n, shift, hist, nb);
        Launch inner{L.st, nullptr};
        uint32_t* dtotal = nullptr;
        if (nb <= kDigitScanBlocks) {
            dtotal = hist + hn;   // radix_hist_words leaves 256 words after the histogram
            hipLaunchKernelGGL(k_radix_digit_scan, dim3(256), dim3(64), 0, L.st, hist, nb, dtotal);
        } else {
            scan_impl<uint32_t>(inner, hist, hn, hist, (uint64_t*)(tmp), tmp + 1);
        }
        hipLaunchKernelGGL((k_radix_scatter<K, I>), dim3((unsigned)nb), dim3(kThreads), 0, L.st, kin, vin,
                           keys[cur ^ 1], vals[cur ^ 1], n, shift, hist, nb, dtotal);
        if (L.prof) L.prof->end(L.st);
        cur ^= 1;
    }
    return cur;
}

// inputs below this size take four items per thread (twice the workgroups)
constexpr int64_t kSmallSort = (int64_t)1 << 21;

template <typename K>
int radix_impl(const Launch& L, const K* first, bool iota, K* keys[2], uint32_t* vals[2], int64_t n, int bits,
               uint32_t* hist, uint64_t* tmp) {
    if (n <= 1 || bits <= 0) {
        // nothing to order: the result is the input, in buffer 0
        if (n > 0 && first) (void)hipMemcpyAsync(keys[0], first, (size_t)n * sizeof(K), hipMemcpyDeviceToDevice, L.st);
        if (iota) iota_u32(L, vals[0], n);
        return 0;
    }
    if (n < kSmallSort) return radix_passes<K, 4>(L, first, iota, keys, vals, n, bits, hist, tmp);
    return radix_passes<K, 8>(L, first, iota, keys, vals, n, bits, hist, tmp);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_f32(float* p, float v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
// Sum of n u32 values into *out (u64, zeroed by the caller): a wave sum per
// 64 values, one atomic per wave.
__global__ __launch_bounds__(256) void k_sum_u32(const uint32_t* __restrict__ a, int64_t n,
                                                 unsigned long long* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned long long v = i < n ? (unsigned long long)a[i] : 0ull;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(out, v);
}
__global__ void k_iota_u32(uint32_t* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (uint32_t)i;
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ means, int64_t n, float3 lo, float3 inv,
                                                uint32_t* __restrict__ code, uint32_t* __restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float x = fminf(fmaxf((means[3 * i] - lo.x) * inv.x, 0.f), 1.f);
    const float y = fminf(fmaxf((means[3 * i + 1] - lo.y) * inv.y, 0.f), 1.f);
    const float z = fminf(fmaxf((means[3 * i + 2] - lo.z) * inv.z, 0.f), 1.f);
    const uint32_t qx = min((uint32_t)(x * 1024.f), 1023u), qy = min((uint32_t)(y * 1024.f), 1023u),
                   qz = min((uint32_t)(z * 1024.f), 1023u);
    code[i] = spread10(qx) | (spread10(qy) << 1) | (spread10(qz) << 2);
    idx[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_gather_rows(const float* __restrict__ src, const uint32_t* __restrict__ perm,
                                                     int64_t n, int rf, float* __restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n * rf) return;
    const int64_t i = t / rf;
    const int c = (int)(t - i * rf);
    dst[t] = src[(int64_t)perm[i] * rf + c];
}

}  // namespace

void morton_codes(const Launch& L, const float* means, int64_t n, const float lo[3], const float inv[3],
                  uint32_t* code, uint32_t* idx) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_morton, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.st, means, n,
                       make_float3(lo[0], lo[1], lo[2]), make_float3(inv[0], inv[1], inv[2]), code, idx);
}

void gather_rows(const Launch& L, const float* src, const uint32_t* perm, int64_t n, int rf, float* dst) {
    if (n <= 0 || rf <= 0) return;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((n * rf + 255) / 256)), dim3(256), 0, L.st, src, perm, n, rf,
                       dst);
}

int64_t scan_tmp_words(int64_t n) { return (n + kTileItems - 1) / kTileItems + 2; }

void scan_u32_to_u64(const Launch& L, const uint32_t* in, int64_t n, uint64_t* out, uint64_t* total, uint64_t* tmp) {
    scan_impl<uint64_t>(L, in, n, out, total, tmp);
}

void tile_ranges_from_counts(const Launch& L, const uint32_t* len, int64_t ntiles, uint64_t cap, const uint64_t* total,
                             uint2* ranges, int* overflow) {
    if (L.prof) L.prof->begin("tile_ranges", L.st);
    hipLaunchKernelGGL(k_scan_ranges, dim3(1), dim3(kThreads), 0, L.st, len, ntiles, cap, total, ranges, overflow);
    if (L.prof) L.prof->end(L.st);
}

void scan_u32_to_u32(const Launch& L, const uint32_t* in, int64_t n, uint32_t* out, uint64_t* total, uint64_t* tmp) {
    scan_impl<uint32_t>(L, in, n, out, total, tmp);
}

// histogram words for sorting any number of items up to n (the smaller,
// 1024-item tiles bound both pass layouts), plus 256 for the digit totals
int64_t radix_hist_words(int64_t n) { return ((n + kThreads * 4 - 1) / (kThreads * 4)) * 256 + 256; }

int radix_sort_u32(const Launch& L, uint32_t* keys[2], uint32_t* vals[2], int64_t n, int bits, uint32_t* hist,
                   uint64_t* tmp) {
    return radix_impl<uint32_t>(L, nullptr, false, keys, vals, n, bits, hist, tmp);
}

int radix_order_u32(const Launch& L, const uint32_t* keys_in, uint32_t* keys[2], uint32_t* vals[2], int64_t n,
                    int bits, uint32_t* hist, uint64_t* tmp) {
    return radix_impl<uint32_t>(L, keys_in, true, keys, vals, n, bits, hist, tmp);
}

int radix_sort_u64(const Launch& L, uint64_t* keys[2], uint32_t* vals[2], int64_t n, int bits, uint32_t* hist,
                   uint64_t* tmp) {
    return radix_impl<uint64_t>(L, nullptr, false, keys, vals, n, bits, hist, tmp);
}

void fill_u32(const Launch& L, uint32_t* p, uint32_t v, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.st, p, v, n);
}
void fill_f32(const Launch& L, float* p, float v, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.st, p, v, n);
}
void sum_u32(const Launch& L, const uint32_t* a, int64_t n, uint64_t* out) {
    fill_u32(L, (uint32_t*)out, 0u, 2);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_sum_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.st, a, n,
                       (unsigned long long*)out);
}
void iota_u32(const Launch& L, uint32_t* p, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_iota_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.st, p, n);
}

}  // namespace gs3
