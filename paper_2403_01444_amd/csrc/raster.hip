// Tile rasterizer of 3D Gaussians for gfx950 (Sec. 3.2: Eq. 2-4), forward
// and adjoint, plus the Gaussian transform of Sec. 4.1 fused into the
// per-Gaussian kernels.
#include "kernels.h"

#ifndef GS3_BLEND_ROWS_FWD
#define GS3_BLEND_ROWS_FWD 1
#endif
#ifndef GS3_BLEND_ROWS_BWD
#define GS3_BLEND_ROWS_BWD 1
#endif

namespace gs3 {

namespace {

__device__ __forceinline__ uint32_t pack16(int lo, int hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }

// ---------------------------------------------------------------------------
// preprocess: transform, covariance (Eq. 2), EWA projection (Eq. 3), conic,
// pixel box, tile rectangle, depth key, SH colour, tile count.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_preprocess(GaussDev g, CamDev cam, float4* __restrict__ rec,
                                                    uint32_t* __restrict__ key, uint2* __restrict__ rect,
                                                    uint32_t* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.n) return;
    Geo o;
    if (!geo_forward(g, cam, i, o)) {
        key[i] = 0xFFFFFFFFu;
        count[i] = 0;
        rect[i] = make_uint2(1u, 0u);
        rec[3 * i + 0] = make_float4(0.f, 0.f, 0.f, 0.f);
        rec[3 * i + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
        rec[3 * i + 2] = make_float4(0.f, __uint_as_float(pack16(1, 1)), __uint_as_float(0u), 0.f);
        return;
    }
    ColourCtx cc;
    colour_forward(g, cam, i, o, cc);
    const float A = o.c / o.det, B = -o.b / o.det, C = o.a / o.det;
    const float op = opacity_of(g.opac[i]);
    rec[3 * i + 0] = make_float4(o.u, o.v, A, B);
    rec[3 * i + 1] = make_float4(C, op, fmaxf(cc.raw[0], 0.f), fmaxf(cc.raw[1], 0.f));
    rec[3 * i + 2] = make_float4(fmaxf(cc.raw[2], 0.f), __uint_as_float(pack16(o.x0, o.y0)),
                                 __uint_as_float(pack16(o.x1, o.y1)), -logf(255.0f * op));
    const int tx0 = o.x0 / kTile, ty0 = o.y0 / kTile, tx1 = o.x1 / kTile, ty1 = o.y1 / kTile;
    rect[i] = make_uint2(pack16(tx0, ty0), pack16(tx1, ty1));
    count[i] = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
    key[i] = __float_as_uint(o.t[2]);
}

// ---------------------------------------------------------------------------
// radix64 ordering: one (tile << 32 | depth bits, index) pair per covered
// tile, in Gaussian order, then a 64-bit LSD sort and a boundary scan.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_emit(int64_t n, const uint32_t* __restrict__ key,
                                              const uint2* __restrict__ rect, const uint64_t* __restrict__ offs,
                                              int tiles_x, uint64_t cap, uint64_t* __restrict__ keys,
                                              uint32_t* __restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = key[i];
    if (k == 0xFFFFFFFFu) return;
    const uint2 r = rect[i];
    const int tx0 = r.x & 0xFFFF, ty0 = r.x >> 16, tx1 = r.y & 0xFFFF, ty1 = r.y >> 16;
    uint64_t off = offs[i];
    for (int ty = ty0; ty <= ty1; ty++)
        for (int tx = tx0; tx <= tx1; tx++) {
            if (off < cap) {
                keys[off] = ((uint64_t)(ty * tiles_x + tx) << 32) | k;
                vals[off] = (uint32_t)i;
            }
            off++;
        }
}

__global__ __launch_bounds__(256) void k_gpos_from_pairs(const uint64_t* __restrict__ keys,
                                                         const uint32_t* __restrict__ vals, int64_t K,
                                                         const uint2* __restrict__ rect,
                                                         const uint64_t* __restrict__ goff, int tiles_x, uint64_t cap,
                                                         uint32_t* __restrict__ gpos) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= K) return;
    const uint32_t id = vals[p];
    const uint32_t t = (uint32_t)(keys[p] >> 32);
    const int tx = (int)(t % (uint32_t)tiles_x), ty = (int)(t / (uint32_t)tiles_x);
    const uint2 r = rect[id];
    const int tx0 = r.x & 0xFFFF, ty0 = r.x >> 16, tx1 = r.y & 0xFFFF;
    const uint64_t k = goff[id] + (uint64_t)((ty - ty0) * (tx1 - tx0 + 1) + (tx - tx0));
    if (k < cap) gpos[k] = (uint32_t)p;
}

__global__ __launch_bounds__(256) void k_zero_ranges(uint2* ranges, int ntiles) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < ntiles) ranges[t] = make_uint2(0u, 0u);
}

__global__ __launch_bounds__(256) void k_ranges_from_keys(const uint64_t* __restrict__ keys, int64_t K,
                                                          uint2* __restrict__ ranges) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= K) return;
    const uint32_t t = (uint32_t)(keys[k] >> 32);
    if (k == 0 || (uint32_t)(keys[k - 1] >> 32) != t) ranges[t].x = (uint32_t)k;
    if (k == K - 1 || (uint32_t)(keys[k + 1] >> 32) != t) ranges[t].y = (uint32_t)(k + 1);
}

// ---------------------------------------------------------------------------
// depth-first ordering.  The Gaussians are first sorted by (depth bits,
// index) and their tile rectangles gathered into that order.  The sorted
// sequence is cut into chunks of kBinChunk.  A workgroup stages one chunk's
// rectangles in LDS; each of its waves owns one tile row.  Pass 1 counts
// pairs per (chunk, tile); an exclusive scan of the counts gives each
// (chunk, tile) segment its first slot; pass 2 lists the chunk's Gaussians
// spanning the row in depth order and writes, column by column, the indices
// of those covering the column at consecutive slots of the segment.  Inside
// a tile the result is ordered by (chunk, position in chunk), i.e. by
// (depth bits, index): the order a stable (tile, depth) sort gives.
// ---------------------------------------------------------------------------
#ifndef GS3_BIN_ROWS
#define GS3_BIN_ROWS 8
#endif
constexpr int kBinRowsPerBlock = GS3_BIN_ROWS;   // one wave per tile row
constexpr int kBinThreads = 64 * kBinRowsPerBlock;

// Workgroups are dealt round-robin to the eight XCDs (linear id mod 8), each
// with its own L2.  The binning passes give each XCD a contiguous eighth of
// the chunks of every row block, so the (tile, chunk) segments that follow
// each other in a tile's list (about a dozen entries each) are written
// through the same L2 and merge into whole lines there, instead of eight L2s
// writing back partial lines of each other's segments.  nchunks is a
// multiple of 8 (bin_chunks); the padding chunks are empty.
__device__ __forceinline__ void bin_block(int64_t nchunks, int& rowblock, int64_t& chunk) {
    const int64_t per = nchunks >> 3;
    const int64_t b = blockIdx.x;
    const int64_t k = b >> 3;
    rowblock = (int)(k / per);
    chunk = (b & 7) * per + k % per;
}

__global__ __launch_bounds__(256) void k_bin_gather(const uint32_t* __restrict__ order, int64_t n,
                                                    const uint2* __restrict__ rect, const uint32_t* __restrict__ count,
                                                    const uint64_t* __restrict__ goff, uint32_t cap,
                                                    uint2* __restrict__ srect, uint32_t* __restrict__ sgoff,
                                                    uint32_t* __restrict__ zero, int64_t nzero) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < nzero) zero[e] = 0u;
    if (e >= n) return;
    const uint32_t id = order[e];
    srect[e] = count[id] ? rect[id] : make_uint2(0xFFFF0000u, 0u);   // empty: no row spans
    if (sgoff) {
        const uint64_t go = goff[id];
        sgoff[e] = go < (uint64_t)cap ? (uint32_t)go : cap;
    }
}

// Counting pass of the depth-first binning: for a tile row (one wave) and a
// chunk of depth-ordered Gaussians, how many of the chunk's Gaussians have a
// tile rectangle covering each tile of the row.  Every covering Gaussian
// adds +1 at its first column and -1 past its last to an LDS difference
// array; a prefix sum over the row's columns gives the counts (the same
// coverage test the scatter applies tile by tile).  The counts are stored
// chunk-major, so a wave writes its row as consecutive words.  A workgroup
// takes kCountGroup consecutive chunks of one row block and, when ttot is
// set, adds each tile's count over them to ttot (one atomic per tile and
// group).
constexpr int kCountGroup = 8;   // bin_chunks is a multiple of 8

__global__ __launch_bounds__(kBinThreads) void k_bin_count(const uint2* __restrict__ srect, int64_t n, int tiles_x,
                                                           int tiles_y, int64_t nchunks, uint32_t* __restrict__ hist,
                                                           uint32_t* __restrict__ ttot) {
    const int64_t ntiles = (int64_t)tiles_x * tiles_y;
    __shared__ uint2 s_rect[kBinChunk];
    __shared__ int s_diff[kBinRowsPerBlock][kMaxTilesX + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t ngroups = nchunks / kCountGroup;
    const int64_t group = (int64_t)blockIdx.x % ngroups;
    const int rowblock = (int)((int64_t)blockIdx.x / ngroups);
    const int row = rowblock * kBinRowsPerBlock + w;
    uint32_t tot[4] = {0u, 0u, 0u, 0u};
    for (int64_t chunk = group * kCountGroup; chunk < (group + 1) * kCountGroup; chunk++) {
        const int64_t e0 = chunk * kBinChunk;
        const int m = (int)min((int64_t)kBinChunk, n - e0);   // <= 0 for the padding chunks
        __syncthreads();   // the previous chunk's rectangles are no longer read
        for (int e = threadIdx.x; e < m; e += kBinThreads) s_rect[e] = srect[e0 + e];
        for (int k = lane; k <= kMaxTilesX; k += 64) s_diff[w][k] = 0;
        __syncthreads();
        if (row >= tiles_y) continue;
        for (int e = lane; e < m; e += 64) {
            const uint2 r = s_rect[e];
            if ((int)(r.x >> 16) <= row && row <= (int)(r.y >> 16)) {
                atomicAdd(&s_diff[w][r.x & 0xFFFFu], 1);
                atomicAdd(&s_diff[w][(r.y & 0xFFFFu) + 1u], -1);
            }
        }
        // the wave's atomics are done before its reads below (LDS operations of
        // one wave complete in order); lane l takes columns 4 l .. 4 l + 3
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int a[4];
        int t = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            t += s_diff[w][4 * lane + k];
            a[k] = t;
        }
        const int x = (int)wave_incl_scan_u32((uint32_t)t);   // inclusive scan of the lane totals
        const int pre = x - t;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int tx = 4 * lane + k;
            const uint32_t v = (uint32_t)(pre + a[k]);
            tot[k] += v;
            if (tx < tiles_x) hist[chunk * ntiles + (int64_t)row * tiles_x + tx] = v;
        }
    }
    if (ttot && row < tiles_y) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int tx = 4 * lane + k;
            if (tx < tiles_x && tot[k]) atomicAdd(&ttot[(int64_t)row * tiles_x + tx], tot[k]);
        }
    }
}

// Start slots of the tiles in the tile-major list: ranges[t] = [s, s + len)
// from the exclusive scan of the tile totals, clamped to cap.
// Tile-major exclusive prefix of the chunk-major counts.  A thread owns one
// tile and a segment of kBinScanSeg chunks, so every load and store of a
// warp-wide step touches consecutive tiles of one chunk: (1) segment sums,
// (2) per tile, the exclusive prefix over its segments and its total,
// (3) an exclusive scan of the tile totals (scan_u32_to_u64), (4) each
// segment's chunks walked again from the tile's and the segment's offset.
constexpr int kBinScanSeg = 32;

__global__ __launch_bounds__(256) void k_bin_scan_part(const uint32_t* __restrict__ hist, int64_t nchunks, int ntiles,
                                                       int64_t nseg, uint32_t* __restrict__ part) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= ntiles) return;
    for (int64_t sg = blockIdx.y; sg < nseg; sg += gridDim.y) {
        const int64_t c0 = sg * kBinScanSeg;
        const int64_t c1 = min(c0 + kBinScanSeg, nchunks);
        uint32_t s = 0u;
        for (int64_t c = c0; c < c1; c++) s += hist[c * ntiles + t];
        part[sg * ntiles + t] = s;
    }
}

__global__ __launch_bounds__(256) void k_bin_scan_tiles(uint32_t* __restrict__ part, int64_t nseg, int ntiles,
                                                        uint32_t* __restrict__ ttot) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= ntiles) return;
    uint32_t run = 0u;   // a tile holds at most one pair per Gaussian (< 2^31)
    for (int64_t sg = 0; sg < nseg; sg++) {
        const uint32_t v = part[sg * ntiles + t];
        part[sg * ntiles + t] = run;
        run += v;
    }
    ttot[t] = run;
}

__global__ __launch_bounds__(256) void k_bin_scan_base(const uint32_t* __restrict__ hist, int64_t nchunks, int ntiles,
                                                       int64_t nseg, const uint32_t* __restrict__ part,
                                                       const uint64_t* __restrict__ toff, uint32_t cap,
                                                       uint32_t* __restrict__ base) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= ntiles) return;
    for (int64_t sg = blockIdx.y; sg < nseg; sg += gridDim.y) {
        const int64_t c0 = sg * kBinScanSeg;
        const int64_t c1 = min(c0 + kBinScanSeg, nchunks);
        uint64_t run = toff[t] + part[sg * ntiles + t];
        for (int64_t c = c0; c < c1; c++) {
            base[c * ntiles + t] = run < (uint64_t)cap ? (uint32_t)run : cap;
            run += hist[c * ntiles + t];
        }
    }
}

// Scatter pass, one wave per (tile row, chunk of depth-ordered Gaussians):
// the wave lists the chunk's Gaussians whose rectangle spans its row, in
// depth order, and holds that list in registers, 64 Gaussians per group
// (lane = position in the group).  It then walks the row's columns: at
// column tx the Gaussians covering tx find their rank among the covering
// ones by a ballot and a masked bit count, and write their indices at
// consecutive slots from the (chunk, tile) segment's first slot.  One store
// instruction therefore fills one segment (about a dozen consecutive
// words) instead of touching a dozen tiles' lists, and every tile's entries
// keep the depth order.  The first slot of each (chunk, tile) segment comes
// from `base` in [chunk][tile] layout: the tile-major list's slots (u32,
// already clamped to cap) or the chunk-major list's (u64).
constexpr int kBinGroups = kBinChunk / 64;   // register groups of the covering list
static_assert(kBinChunk % 64 == 0, "the covering list is held in groups of 64");

template <typename B, bool kRec>
__global__ __launch_bounds__(kBinThreads) void k_bin_rows(const uint32_t* __restrict__ order, int64_t n,
                                                  const uint2* __restrict__ srect, const uint32_t* __restrict__ sgoff,
                                                  int tiles_x, int tiles_y, int64_t nchunks,
                                                  const B* __restrict__ base, uint32_t cap,
                                                  uint32_t* __restrict__ vals, uint32_t* __restrict__ gpos) {
    // A segment's slots start at min(first slot, cap) and run at most
    // kBinChunk past it, so with cap < 2^31 they never wrap; slots at or
    // past cap are not written.
    __shared__ uint2 s_rect[kBinChunk];
    __shared__ uint32_t s_id[kBinChunk];
    __shared__ uint32_t s_goff[kBinChunk];
    __shared__ uint32_t s_cov[kBinRowsPerBlock][kBinChunk];   // chunk positions of the row's covering Gaussians
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int rowblock;
    int64_t chunk;
    bin_block(nchunks, rowblock, chunk);
    const int row = rowblock * kBinRowsPerBlock + w;
    const int64_t e0 = chunk * kBinChunk;
    const int m = (int)min((int64_t)kBinChunk, n - e0);
    for (int e = threadIdx.x; e < m; e += kBinThreads) {
        s_id[e] = order[e0 + e];
        s_rect[e] = srect[e0 + e];
        s_goff[e] = kRec ? sgoff[e0 + e] : 0u;
    }
    __syncthreads();
    if (row >= tiles_y) return;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;   // lanes under this one
    // 1. the chunk's Gaussians spanning this row, in depth order
    int G = 0;
    for (int eb = 0; eb < m; eb += 64) {
        const int e = eb + lane;
        bool cov = false;
        if (e < m) {
            const uint2 r = s_rect[e];
            cov = (int)(r.x >> 16) <= row && row <= (int)(r.y >> 16);
        }
        const uint64_t bal = __ballot(cov);
        if (cov) s_cov[w][G + __popcll(bal & below)] = (uint32_t)e;
        G += __popcll(bal);
    }
    if (G == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // 2. the list in registers: column span, index and (record mode) the
    // slot of column 0 of this row in the Gaussian's own pair range
    int lo[kBinGroups], hi[kBinGroups];
    uint32_t gid[kBinGroups], gk[kBinGroups];
    int cmin = 1 << 30, cmax = -1;
#pragma unroll
    for (int gi = 0; gi < kBinGroups; gi++) {
        lo[gi] = 1 << 30;
        hi[gi] = -1;
        gid[gi] = 0u;
        gk[gi] = 0u;
        const int k = 64 * gi + lane;
        if (64 * gi < G && k < G) {
            const uint32_t e = s_cov[w][k];
            const uint2 r = s_rect[e];
            lo[gi] = (int)(r.x & 0xFFFFu);
            hi[gi] = (int)(r.y & 0xFFFFu);   // < tiles_x
            gid[gi] = s_id[e];
            if (kRec)
                gk[gi] = s_goff[e] + (uint32_t)(row - (int)(r.x >> 16)) * (uint32_t)(hi[gi] - lo[gi] + 1) -
                         (uint32_t)lo[gi];
            cmin = min(cmin, lo[gi]);
            cmax = max(cmax, hi[gi]);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        cmin = min(cmin, __shfl_xor(cmin, off));
        cmax = max(cmax, __shfl_xor(cmax, off));
    }
    cmin = __builtin_amdgcn_readfirstlane(cmin);
    cmax = __builtin_amdgcn_readfirstlane(cmax);
    const int ngr = (G + 63) >> 6;
    // 3. the columns the list covers; lane l of colb[cg] holds the first
    // slot of column 64 cg + l
    const B* brow = base + chunk * ((int64_t)tiles_x * tiles_y) + (int64_t)row * tiles_x;
    uint32_t colb[kMaxTilesX / 64];
#pragma unroll
    for (int cg = 0; cg < kMaxTilesX / 64; cg++) {
        const int tx = 64 * cg + lane;
        const uint64_t b = (tx < tiles_x && cg * 64 <= cmax) ? (uint64_t)brow[tx] : (uint64_t)cap;
        colb[cg] = b < (uint64_t)cap ? (uint32_t)b : cap;
    }
#pragma unroll
    for (int cg = 0; cg < kMaxTilesX / 64; cg++) {
        if (64 * cg > cmax) break;
        const int t0 = max(cmin, 64 * cg), t1 = min(cmax, 64 * cg + 63);
        for (int tx = t0; tx <= t1; tx++) {
            uint32_t pos = (uint32_t)__builtin_amdgcn_readlane((int)colb[cg], tx - 64 * cg);
#pragma unroll
            for (int gi = 0; gi < kBinGroups; gi++) {
                if (gi >= ngr) break;
                const uint64_t bal =
                    __builtin_amdgcn_ballot_w64(lo[gi] <= tx) & __builtin_amdgcn_ballot_w64(tx <= hi[gi]);
                // rank among the covering lanes below this one
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                const uint32_t slot = pos + rank;
                if (__builtin_amdgcn_inverse_ballot_w64(bal) && slot < cap) {
                    vals[slot] = gid[gi];
                    if (kRec) {
                        const uint32_t kk = gk[gi] + (uint32_t)tx;
                        if (kk < cap) gpos[kk] = slot;
                    }
                }
                pos += (uint32_t)__popcll(bal);
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_ranges_from_hist(const uint32_t* __restrict__ base,
                                                          const uint64_t* __restrict__ total, int ntiles, uint64_t cap,
                                                          uint2* __restrict__ ranges, int* __restrict__ overflow) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    const uint64_t K = *total;
    if (t == 0 && K > cap) atomicOr(overflow, 1);
    if (t >= ntiles) return;
    // chunk 0's row of the bases: the first slot of every tile (clamped to cap)
    const uint32_t s = base[t];
    const uint32_t e = t + 1 < ntiles ? base[t + 1] : (uint32_t)(K < cap ? K : cap);
    ranges[t] = make_uint2(s, e);
}

// XCD-aware tile order: consecutive workgroups are dealt round-robin to the
// eight XCDs, so give each XCD a contiguous band of tiles (neighbouring tiles
// share most of their Gaussians and hit the same L2).
__device__ __forceinline__ int tile_of_block(int b, int ntiles) {
    const int per = (ntiles + 7) / 8;
    const int xcd = b & 7, k = b >> 3;
    const int t = xcd * per + k;
    return t;
}

// Longest-first tile schedule: tiles bucketed by the work they carry (list
// length for the forward, walked entries for the backward) on a half-octave
// scale, heaviest bucket first, so the long tiles start in the first wave of
// workgroups instead of trailing the launch.  One workgroup; the order inside
// a bucket is whatever the atomics give (it only affects scheduling).
constexpr int kOrderBuckets = 66;
__device__ __forceinline__ int work_bucket(uint32_t w) {
    if (w == 0u) return 0;
    const int lz = 31 - __clz(w);
    const int half = lz >= 1 ? (int)((w >> (lz - 1)) & 1u) : 0;
    return 1 + 2 * lz + half;
}

__global__ __launch_bounds__(1024) void k_tile_order(const uint2* __restrict__ ranges,
                                                     const uint32_t* __restrict__ walk, int ntiles,
                                                     int* __restrict__ order) {
    __shared__ uint32_t cnt[kOrderBuckets], off[kOrderBuckets];
    for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) cnt[b] = 0u;
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
        const uint32_t w = walk ? walk[t] : ranges[t].y - ranges[t].x;
        atomicAdd(&cnt[work_bucket(w)], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0u;
        for (int b = kOrderBuckets - 1; b >= 0; b--) {
            off[b] = acc;
            acc += cnt[b];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
        const uint32_t w = walk ? walk[t] : ranges[t].y - ranges[t].x;
        order[atomicAdd(&off[work_bucket(w)], 1u)] = t;
    }
}

// ---------------------------------------------------------------------------
// blend forward (Eq. 4): one workgroup per 16x16 tile; each thread owns R
// vertically adjacent pixels of one column, so a staged record is read from
// LDS once per R evaluations and the column terms of the exponent are shared.
// The tile's Gaussian records are staged through LDS 256/R at a time.
//
// kChunked: the pairs are in the chunk-major list of the depth-first
// binning (ChunkDev): the tile's entries are its segments of successive
// depth chunks.  A cursor (chunk, offset) walks them: per batch, the first
// wave reads the lengths and starts of the tile's segments in the next 64
// chunks and scans the lengths, and each thread finds its entry's segment
// by binary search.  Every staged entry's Gaussian index is also written to
// the tile-major list at the tile's slot (ranges[tile].x + entry), which
// the backward walks.  The result equals the walk of the tile-major list.
// ---------------------------------------------------------------------------
template <int R, bool kChunked>
__global__ __launch_bounds__(kTile * kTile / R) void k_blend_fwd(CamDev cam, int ntiles,
                                                                 const uint2* __restrict__ ranges,
                                                                 const uint32_t* __restrict__ vals,
                                                                 const float4* __restrict__ rec,
                                                                 float* __restrict__ image, float* __restrict__ T_final,
                                                                 uint32_t* __restrict__ last_out,
                                                                 uint32_t* __restrict__ tile_walk,
                                                                 const int* __restrict__ order, ChunkDev cl) {
    constexpr int NT = kTile * kTile / R;
    static_assert(!kChunked || NT >= 64, "the chunk window needs a full wave");
    __shared__ uint32_t s_walk;
    __shared__ uint32_t s_pre[65];   // chunk window: exclusive prefix of the segment lengths
    __shared__ uint32_t s_sb[64];    // and the slot of each segment's next entry
    __shared__ int64_t s_cc;         // cursor: first chunk of the window
    __shared__ uint32_t s_co;        // and the entries of it already staged
    const int tile = order ? order[blockIdx.x] : tile_of_block(blockIdx.x, ntiles);
    __shared__ float4 s_w0[NT];
    __shared__ float4 s_w1[NT];
    __shared__ float4 s_w2[NT];   // blend_stage_w2 form
    if (tile >= ntiles) return;
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int tx0p = tx * kTile, ty0p = ty * kTile;
    const int px = tx0p + (threadIdx.x & 15), py0 = ty0p + (threadIdx.x >> 4) * R;
    const float fpx = (float)px;
    uint32_t sel[R];   // this thread's column and row bits in the box masks
#pragma unroll
    for (int k = 0; k < R; k++) sel[k] = (1u << (threadIdx.x & 15)) | (1u << (16 + (threadIdx.x >> 4) * R + k));
    const uint2 rg = ranges[tile];
    const uint32_t start = rg.x, end = rg.y;
    float T[R], c0[R], c1[R], c2[R];
    uint32_t last[R];
    // pixel row coordinate, NaN once the pixel has stopped (and for pixels
    // outside the image): every comparison of its exponent is then false, so
    // a stopped pixel takes no further contribution without a flag test
    const float kStopped = __int_as_float(0x7FC00000);
    float fpy[R];
#pragma unroll
    for (int k = 0; k < R; k++) {
        T[k] = 1.0f;
        c0[k] = c1[k] = c2[k] = 0.f;
        last[k] = 0u;
        fpy[k] = (px < cam.W && py0 + k < cam.H) ? (float)(py0 + k) : kStopped;
    }
    if (threadIdx.x == 0) {
        s_walk = 0u;
        s_cc = 0;
        s_co = 0u;
    }
    const uint32_t total = end - start;
    for (uint32_t eb = 0; eb < total;) {   // eb: entries staged so far
        bool all = true;
#pragma unroll
        for (int k = 0; k < R; k++) all = all && (fpy[k] != fpy[k]);
        if (__syncthreads_count(all) == NT) break;
        uint32_t cnt_u;
        if (kChunked) {
            const int64_t ntl = (int64_t)ntiles;
            if (threadIdx.x < 64) {
                const int l = threadIdx.x;
                const int64_t c = s_cc + l;
                uint32_t len = 0u, sb = 0u;
                if (c < cl.nchunks) {
                    len = cl.hist[c * ntl + tile];
                    const uint64_t b = cl.cmb[c * ntl + tile];
                    sb = b < (uint64_t)cl.cap ? (uint32_t)b : cl.cap;
                }
                if (l == 0) {
                    len -= s_co;
                    sb += s_co;
                }
                const uint32_t x = wave_incl_scan_u32(len);   // inclusive scan of the lengths
                s_pre[l + 1] = x;
                if (l == 0) s_pre[0] = 0u;
                s_sb[l] = sb;
            }
            __syncthreads();
            const uint32_t avail = s_pre[64];
            // (avail exceeds the rest of the tile's range only when the pair
            // list overflowed and the ranges were clamped to cap)
            cnt_u = min(min((uint32_t)NT, avail), total - eb);
            const uint32_t e = threadIdx.x;
            if (e < cnt_u) {
                int lo = 0, hi = 63;   // the last segment starting at or before entry e
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_pre[mid] <= e) lo = mid; else hi = mid - 1;
                }
                const uint32_t idx = s_sb[lo] + (e - s_pre[lo]);
                if (idx < cl.cap) {
                    const uint32_t id = vals[idx];
                    const float4 r0 = rec[3 * (int64_t)id + 0], r1 = rec[3 * (int64_t)id + 1];
                    s_w0[threadIdx.x] = r0;
                    s_w1[threadIdx.x] = r1;
                    s_w2[threadIdx.x] = blend_stage_w2<false>(r0, r1, rec[3 * (int64_t)id + 2], tx0p, ty0p);
                    const uint32_t slot = start + eb + e;
                    if (slot < cl.cap) cl.walked[slot] = id;
                } else {
                    // past the pair capacity (the render reports the overflow):
                    // an entry no pixel takes
                    s_w0[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
                    s_w1[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
                    s_w2[threadIdx.x] = make_float4(0.f, 0.f, 0.f, __uint_as_float(0u));
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                // advance past the cnt_u staged entries
                if (cnt_u == avail) {
                    s_cc += 64;
                    s_co = 0u;
                } else {
                    int lo = 0, hi = 63;   // the segment holding the next entry
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_pre[mid] <= cnt_u) lo = mid; else hi = mid - 1;
                    }
                    s_co = (lo == 0 ? s_co : 0u) + (cnt_u - s_pre[lo]);
                    s_cc += lo;
                }
            }
        } else {
            const uint32_t e = start + eb + threadIdx.x;
            if (e < end) {
                const uint32_t id = vals[e];
                const float4 r0 = rec[3 * (int64_t)id + 0], r1 = rec[3 * (int64_t)id + 1];
                s_w0[threadIdx.x] = r0;
                s_w1[threadIdx.x] = r1;
                s_w2[threadIdx.x] = blend_stage_w2<false>(r0, r1, rec[3 * (int64_t)id + 2], tx0p, ty0p);
            }
            __syncthreads();
            cnt_u = min((uint32_t)NT, total - eb);
        }
        const int cnt = (int)cnt_u;
        if (!all) {
            // branch-free per-pixel body: every lane evaluates, selects keep
            // the state of pixels that do not take the contribution
            auto eval = [&](int j) {
                const float4 w0 = s_w0[j], w1 = s_w1[j], w2 = s_w2[j];
                const uint32_t box = __float_as_uint(w2.w);
                float adx2, bdx;
                blend_dx_terms(fpx - w0.x, w0, adx2, bdx);
                // lane masks (wave-uniform): okm[k] the lanes whose pixel k
                // takes the entry, bm[k] those whose exponent lies in the
                // band where the exact test decides
                float power[R];
                uint64_t okm[R], bm[R];
                uint64_t any_band = 0ull;
#pragma unroll
                for (int k = 0; k < R; k++) {
                    power[k] = blend_power(adx2, bdx, fpy[k] - w0.y, w1.x);
                    const uint64_t pm = __builtin_amdgcn_ballot_w64((box & sel[k]) == sel[k]) &
                                        __builtin_amdgcn_ballot_w64(power[k] <= 0.0f) &
                                        __builtin_amdgcn_ballot_w64(power[k] >= w2.y);
                    bm[k] = pm & __builtin_amdgcn_ballot_w64(power[k] < w2.z);
                    okm[k] = pm & ~bm[k];
                    any_band |= bm[k];
                }
                if (any_band) {
#pragma unroll
                    for (int k = 0; k < R; k++)
                        okm[k] |= bm[k] & __builtin_amdgcn_ballot_w64(blend_exact_test(power[k], w1.y));
                }
                uint64_t any_ok = 0ull;   // no pixel of the wave takes the entry: nothing changes
#pragma unroll
                for (int k = 0; k < R; k++) any_ok |= okm[k];
                if (!any_ok) return;
#pragma unroll
                for (int k = 0; k < R; k++) {
                    const bool ok = __builtin_amdgcn_inverse_ballot_w64(okm[k]);
                    const float alpha = fminf(0.99f, w1.y * __expf(power[k]));
                    const float Tn = T[k] * (1.0f - alpha);
                    const bool stop = ok & (Tn < 1e-4f);
                    const bool take = ok & !stop;
                    const float wgt = take ? alpha * T[k] : 0.0f;
                    c0[k] += wgt * w1.z;
                    c1[k] += wgt * w1.w;
                    c2[k] += wgt * w2.x;
                    T[k] = take ? Tn : T[k];
                    last[k] = take ? eb + (uint32_t)j + 1u : last[k];
                    fpy[k] = stop ? kStopped : fpy[k];
                }
            };
            // two entries per trip; the wave leaves once all its pixels have stopped
            int j = 0;
            for (; j + 1 < cnt; j += 2) {
                eval(j);
                eval(j + 1);
                bool active = false;
#pragma unroll
                for (int k = 0; k < R; k++) active = active | (fpy[k] == fpy[k]);
                if (!__builtin_amdgcn_ballot_w64(active)) break;
            }
            if (j + 1 == cnt) eval(j);
        }
        eb += cnt_u;
        __syncthreads();
    }
    const int64_t P = (int64_t)cam.W * cam.H;
    uint32_t mx = 0u;
#pragma unroll
    for (int k = 0; k < R; k++) {
        if (px < cam.W && py0 + k < cam.H) {
            const int64_t p = (int64_t)(py0 + k) * cam.W + px;
            image[p] = c0[k] + T[k] * cam.bg[0];
            image[P + p] = c1[k] + T[k] * cam.bg[1];
            image[2 * P + p] = c2[k] + T[k] * cam.bg[2];
            T_final[p] = T[k];
            last_out[p] = last[k];
        }
        mx = max(mx, last[k]);
    }
    if (mx) atomicMax(&s_walk, mx);
    __syncthreads();
    if (threadIdx.x == 0) tile_walk[tile] = s_walk;
}

// ---------------------------------------------------------------------------
// blend backward: walk the tile list from the last contributor of any pixel
// down to the first, recover T_i = T_{i+1} / (1 - alpha_i), keep the colour
// accumulated behind each contributor, sum each Gaussian's nine gradient
// terms over a thread's R pixels, then across the wave (reduce-scatter) and
// the tile's waves in LDS, before one global atomic per term and tile.
// ---------------------------------------------------------------------------
// kRecords: write each walked entry's nine sums to the compact record buffer
// (fixed summation order; gathered per Gaussian by the preprocess backward),
// atomics only past its capacity; otherwise one global atomic per term and
// (tile, Gaussian).  kOpacity: also reduce the opacity term.
// factors of the nine reduced terms: the conic terms are summed as dx^2,
// dx dy and dy^2 (powers of two: the scaling is exact)
#ifndef GS3_BWD_BATCH
#define GS3_BWD_BATCH 128
#endif
constexpr int kBwdBatch = GS3_BWD_BATCH;   // backward blend: entries staged per batch (LDS: about 200 B each)
__constant__ float kConicScale[9] = {1.f, 1.f, -0.5f, -1.f, -0.5f, 1.f, 1.f, 1.f, 1.f};

template <int R, bool kRecords, bool kOpacity>
__global__ __launch_bounds__(kTile * kTile / R) void k_blend_bwd(CamDev cam, int ntiles,
                                                                 const uint2* __restrict__ ranges,
                                                                 const uint32_t* __restrict__ vals,
                                                                 const float4* __restrict__ rec,
                                                                 const float* __restrict__ d_image,
                                                                 const float* __restrict__ T_final,
                                                                 const uint32_t* __restrict__ last_in,
                                                                 const uint32_t* __restrict__ tile_walk,
                                                                 const uint32_t* __restrict__ walk_off,
                                                                 float* __restrict__ grec, uint32_t grec_cap,
                                                                 float* __restrict__ accum,
                                                                 const int* __restrict__ order) {
    constexpr int NT = kTile * kTile / R, NW = NT / 64;
    constexpr int KB = kBwdBatch < NT ? kBwdBatch : NT;   // entries staged per batch
    static_assert(KB <= 128, "the wave entry masks hold two words");
    __shared__ float4 s_w0[KB];
    __shared__ float4 s_w1[KB];
    __shared__ float4 s_w2[KB];   // blend_stage_w2 form
    __shared__ uint32_t s_id[KB];
    __shared__ float s_g[NW][9][KB + 1];   // per-wave sums, [wave][term][entry] (padded: term rows on distinct banks)
    const int tile = order ? order[blockIdx.x] : tile_of_block(blockIdx.x, ntiles);
    if (tile >= ntiles) return;
    const uint32_t maxlast = tile_walk[tile];
    if (maxlast == 0) return;
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int tx0p = tx * kTile, ty0p = ty * kTile;
    const int px = tx0p + (threadIdx.x & 15), py0 = ty0p + (threadIdx.x >> 4) * R;
    const float fpx = (float)px;
    uint32_t sel[R];   // this thread's column and row bits in the box masks
#pragma unroll
    for (int k = 0; k < R; k++) sel[k] = (1u << (threadIdx.x & 15)) | (1u << (16 + (threadIdx.x >> 4) * R + k));
    const uint32_t start = ranges[tile].x;
    const uint32_t woff = kRecords ? walk_off[tile] : 0u;
    const int64_t P = (int64_t)cam.W * cam.H;
    // gb: dL/dC . (colour behind the current contributor), the only use of
    // that colour (dL/dalpha_i = T_i (dL/dC . c_i - gb)); it starts at the
    // background and moves to alpha c + (1 - alpha) b past each contributor
    float T[R], g0[R], g1[R], g2[R], gb[R];
    uint32_t last[R];
#pragma unroll
    for (int k = 0; k < R; k++) {
        T[k] = 1.0f;
        last[k] = 0u;
        g0[k] = g1[k] = g2[k] = 0.f;
        if (px < cam.W && py0 + k < cam.H) {
            const int64_t p = (int64_t)(py0 + k) * cam.W + px;
            T[k] = T_final[p];
            last[k] = last_in[p];
            g0[k] = d_image[p];
            g1[k] = d_image[P + p];
            g2[k] = d_image[2 * P + p];
        }
        gb[k] = g0[k] * cam.bg[0] + g1[k] * cam.bg[1] + g2[k] * cam.bg[2];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // reduce-scatter terms: the image-space mean terms summed as dp dx and
    // dp dy (the conic is applied to the sums per entry), the conic terms,
    // r, g, b; lane group (lane >> 3) holds term (lane >> 3)
    const int my_term = lane >> 3;
    // the wave's last contributor: entries past it reach none of its pixels
    uint32_t wlast = 0u;
#pragma unroll
    for (int k = 0; k < R; k++) wlast = max(wlast, last[k]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) wlast = max(wlast, (uint32_t)__shfl_xor((int)wlast, off));
    wlast = __builtin_amdgcn_readfirstlane(wlast);
    const uint32_t wrows = wave_row_bits<R>(wv);
    const int my_slot = my_term < 5 ? my_term : my_term + 1;   // index in the nine-term layout
    for (int64_t jb = ((int64_t)(maxlast - 1) / KB) * KB; jb >= 0; jb -= KB) {
        const uint32_t e = (uint32_t)jb + threadIdx.x;
        if ((int)threadIdx.x < KB && e < maxlast) {
            const uint32_t id = vals[start + e];
            const float4 r0 = rec[3 * (int64_t)id + 0], r1 = rec[3 * (int64_t)id + 1];
            s_id[threadIdx.x] = id;
            s_w0[threadIdx.x] = r0;
            s_w1[threadIdx.x] = r1;
            s_w2[threadIdx.x] = blend_stage_w2(r0, r1, rec[3 * (int64_t)id + 2], tx0p, ty0p);
        }
        __syncthreads();
        const int cnt = (int)min((int64_t)KB, (int64_t)maxlast - jb);
        // the staged entries that can reach a pixel of this wave: box on its
        // rows, before its last contributor (bit j % 64 of wm0 for j < 64,
        // of wm1 above)
        auto bword = [&](int q) -> uint64_t {
            const int jq = 64 * q + lane;
            return __builtin_amdgcn_ballot_w64(jq < cnt && (uint32_t)jb + (uint32_t)jq < wlast &&
                                               box_meets_rows(s_w2[jq].w, wrows));
        };
        const uint64_t wm0 = bword(0), wm1 = KB > 64 ? bword(1) : 0ull;
        // one entry: this thread's R pixels walk back past entry j (their
        // transmittance and behind-colour state), and gr receives the eight
        // terms summed over them; returns whether any pixel of the wave
        // takes the entry (gr and gop are left unset when none does)
        auto entry = [&](int j, float gr[8], float& gop) -> bool {
            const uint32_t ej = (uint32_t)jb + (uint32_t)j;
            gop = 0.f;
            {
                const uint64_t mw = (j >> 6) == 0 ? wm0 : wm1;
                if (!((mw >> (j & 63)) & 1ull)) return false;
            }
            uint64_t act = 0ull;
            const float4 w0 = s_w0[j], w1 = s_w1[j], w2 = s_w2[j];
            const uint32_t box = __float_as_uint(w2.w);
            const float cr = w1.z, cg = w1.w, cb = w2.x;
            const float dx = fpx - w0.x;
            float adx2, bdx;
            blend_dx_terms(dx, w0, adx2, bdx);
            float power[R], dy[R];
            // lane masks (wave-uniform): okm[k] the lanes whose pixel k takes
            // the entry, bm[k] those whose exponent lies in the band where
            // the exact test decides
            uint64_t okm[R], bm[R];
            uint64_t any_band = 0ull;
#pragma unroll
            for (int k = 0; k < R; k++) {
                dy[k] = (float)(py0 + k) - w0.y;
                power[k] = blend_power(adx2, bdx, dy[k], w1.x);
                const uint64_t pm =
                    __builtin_amdgcn_ballot_w64(ej < last[k]) & __builtin_amdgcn_ballot_w64((box & sel[k]) == sel[k]) &
                    __builtin_amdgcn_ballot_w64(power[k] <= 0.0f) & __builtin_amdgcn_ballot_w64(power[k] >= w2.y);
                bm[k] = pm & __builtin_amdgcn_ballot_w64(power[k] < w2.z);
                okm[k] = pm & ~bm[k];
                any_band |= bm[k];
            }
            if (any_band) {
#pragma unroll
                for (int k = 0; k < R; k++)
                    okm[k] |= bm[k] & __builtin_amdgcn_ballot_w64(blend_exact_test(power[k], w1.y));
            }
#pragma unroll
            for (int k = 0; k < R; k++) act |= okm[k];
            // no pixel of the wave takes the entry: its state and sums stay
            if (!act) return false;
            // branch-free per-pixel body: selects keep the state of pixels
            // that this Gaussian does not reach
            bool ok[R];
#pragma unroll
            for (int k = 0; k < R; k++) ok[k] = __builtin_amdgcn_inverse_ballot_w64(okm[k]);
#pragma unroll
            for (int k = 0; k < R; k++) {
                const float G = __expf(power[k]);
                const float raw = w1.y * G;
                const float alpha = fminf(0.99f, raw);
                // T recovery T_i = T_{i+1} / (1 - alpha_i), with the hardware reciprocal (1 ulp)
                const float Tk = ok[k] ? T[k] * __builtin_amdgcn_rcpf(1.0f - alpha) : T[k];
                T[k] = Tk;
                const float aok = ok[k] ? alpha : 0.0f;   // zero: the pixel's state is kept
                const float wgt = aok * Tk;
                const float e = (g0[k] * cr + g1[k] * cg + g2[k] * cb) - gb[k];
                const float dal = Tk * e;
                gb[k] += aok * e;
                const bool unclamped = ok[k] && raw < 0.99f;
                const float dp = unclamped ? dal * raw : 0.0f;
                gop += unclamped ? dal * G : 0.0f;
                // d power / d(u, v) = (A dx + B dy, B dx + C dy): the sums of
                // dp dx and dp dy take A, B, C after the reduction; the conic
                // terms -dx^2 / 2, -dx dy, -dy^2 / 2 get their constant
                // factors there too (kConicScale)
                const float tx = dp * dx, ty = dp * dy[k];
                const float t8[8] = {tx, ty, tx * dx, tx * dy[k], ty * dy[k], g0[k] * wgt, g1[k] * wgt, g2[k] * wgt};
#pragma unroll
                for (int c = 0; c < 8; c++) gr[c] = k == 0 ? t8[c] : gr[c] + t8[c];
            }
            return act != 0ull;
        };
        // two entries per reduction: their exchanges and DPP chains overlap
        int j = cnt - 1;
        for (; j >= 1; j -= 2) {
            float ga[8], gc[8], opa, opc;
            const bool anya = entry(j, ga, opa);
            const bool anyc = entry(j - 1, gc, opc);
            float ra = 0.f, rc = 0.f;
            if (anya && anyc)
                wave_reduce_scatter8x2(ga, gc, lane, ra, rc);
            else if (anya)
                ra = wave_reduce_scatter8(ga, lane);
            else if (anyc)
                rc = wave_reduce_scatter8(gc, lane);
            if ((lane & 7) == 0) {
                s_g[wv][my_slot][j] = ra;
                s_g[wv][my_slot][j - 1] = rc;
            }
            if (kOpacity) {
                const float oa = anya ? wave_sum_dpp(opa) : 0.f;
                const float oc = anyc ? wave_sum_dpp(opc) : 0.f;
                if (lane == 8) {
                    s_g[wv][5][j] = oa;
                    s_g[wv][5][j - 1] = oc;
                }
            }
        }
        if (j == 0) {
            float ga[8], opa;
            const bool any = entry(0, ga, opa);
            float red = 0.f, redop = 0.f;
            if (any) {
                red = wave_reduce_scatter8(ga, lane);
                if (kOpacity) redop = wave_sum_dpp(opa);
            }
            if ((lane & 7) == 0) s_g[wv][my_slot][0] = red;
            if (kOpacity && lane == 8) s_g[wv][5][0] = redop;
        }
        __syncthreads();
        // term k of entry e summed over the waves: the mean terms from the
        // sums of dp dx and dp dy and the entry's conic (A, B, C)
        auto entry_term = [&](int k, int e) -> float {
            float v = s_g[0][k][e];
#pragma unroll
            for (int w = 1; w < NW; w++) v += s_g[w][k][e];
            if (k <= 1) {
                float o = s_g[0][1 - k][e];
#pragma unroll
                for (int w = 1; w < NW; w++) o += s_g[w][1 - k][e];
                const float4 w0 = s_w0[e];
                const float C = s_w1[e].x;
                return k == 0 ? w0.z * v + w0.w * o : w0.w * o + C * v;
            }
            return v * kConicScale[k];
        };
        if (kRecords) {
            if ((int)threadIdx.x < cnt) {
                const uint32_t widx = woff + (uint32_t)jb + threadIdx.x;   // compact index of this walked entry
                const bool fits = widx < grec_cap;
#pragma unroll
                for (int k = 0; k < 9; k++) {
                    if (!kOpacity && k == 5) {
                        if (fits) grec[(int64_t)k * grec_cap + widx] = 0.f;
                        continue;
                    }
                    const float v = entry_term(k, threadIdx.x);
                    if (fits)
                        grec[(int64_t)k * grec_cap + widx] = v;
                    else if (v != 0.f)
                        atomicAdd(accum + 9 * (int64_t)s_id[threadIdx.x] + k, v);
                }
            }
        } else {
            // lane = (entry, term): the atomics of one entry's terms are
            // adjacent lanes on adjacent addresses (one or two cache lines)
            for (int q = threadIdx.x; q < 9 * cnt; q += NT) {
                const int e = q / 9, k = q - 9 * e;
                if (!kOpacity && k == 5) continue;
                const float v = entry_term(k, e);
                if (v != 0.f) atomicAdd(accum + 9 * (int64_t)s_id[e] + k, v);
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void quat_rot_adj(const float q[4], const float g[9], float d[4]) {
    const float w = q[0], x = q[1], y = q[2], z = q[3];
    d[0] += 2.f * (-z * g[1] + y * g[2] + z * g[3] - x * g[5] - y * g[6] + x * g[7]);
    d[1] += 2.f * (y * g[1] + z * g[2] + y * g[3] - 2.f * x * g[4] - w * g[5] + z * g[6] + w * g[7] - 2.f * x * g[8]);
    d[2] += 2.f * (-2.f * y * g[0] + x * g[1] + w * g[2] + x * g[3] + z * g[5] - w * g[6] + z * g[7] - 2.f * y * g[8]);
    d[3] += 2.f * (-2.f * z * g[0] - w * g[1] + x * g[2] + w * g[3] - 2.f * z * g[4] + y * g[5] + x * g[6] + y * g[7]);
}

// ---------------------------------------------------------------------------
// preprocess backward: chain the per-Gaussian 2D gradients through the conic
// inverse, EWA (with J depending on the camera-space mean), the covariance,
// the colour (SH and its view direction) and the transform.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_preprocess_bwd(GaussDev g, CamDev cam, const float* __restrict__ accum,
                                                        GatherDev ga, GradsDev out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.n) return;
    Geo o;
    if (!geo_forward(g, cam, i, o)) return;
    ColourCtx cc;
    colour_forward(g, cam, i, o, cc);
    // the nine 2D gradient terms: fallback atomics plus this Gaussian's walked
    // entries, visited in its tile-rectangle order
    float a9[9];
    for (int k = 0; k < 9; k++) a9[k] = accum[9 * i + k];
    if (ga.grec_cap > 0) {
        const uint2 r = ga.rect[i];
        const int tx0 = r.x & 0xFFFF, ty0 = r.x >> 16, tx1 = r.y & 0xFFFF, ty1 = r.y >> 16;
        uint64_t k = ga.goff[i];
        for (int ty = ty0; ty <= ty1; ty++)
            for (int tx = tx0; tx <= tx1; tx++, k++) {
                if (k >= ga.cap) continue;
                const int t = ty * cam.tiles_x + tx;
                const uint32_t rel = ga.gpos[k] - ga.ranges[t].x;
                if (rel >= ga.tile_walk[t]) continue;
                const uint32_t widx = ga.walk_off[t] + rel;
                if (widx >= ga.grec_cap) continue;
                for (int c = 0; c < 9; c++) a9[c] += ga.grec[(int64_t)c * ga.grec_cap + widx];
            }
    }
    const float du = a9[0], dv = a9[1], dA = a9[2], dB = a9[3], dC = a9[4], dop = a9[5];
    const float drgb[3] = {a9[6], a9[7], a9[8]};
    if (out.d_uv) { out.d_uv[2 * i] += du; out.d_uv[2 * i + 1] += dv; }
    if (out.vgrad) {
        // gradient with respect to the normalised-device-coordinate mean
        const float gx = du * (0.5f * (float)cam.W), gy = dv * (0.5f * (float)cam.H);
        out.vgrad[i] += sqrtf(gx * gx + gy * gy);
        out.vcount[i] += 1.0f;
    }
    if (out.d_conic) { out.d_conic[3 * i] += dA; out.d_conic[3 * i + 1] += dB; out.d_conic[3 * i + 2] += dC; }
    if (out.d_opacity) out.d_opacity[i] += dop;
    if (out.d_rgb) for (int k = 0; k < 3; k++) out.d_rgb[3 * i + k] += drgb[k];
    if (out.d_opac) {
        const float op = opacity_of(g.opac[i]);
        out.d_opac[i] += dop * op * (1.0f - op);
    }
    float dm[3] = {0.f, 0.f, 0.f};
    float dRp[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float dRh[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

    // colour
    float gch[3];
    for (int k = 0; k < 3; k++) gch[k] = cc.raw[k] > 0.f ? drgb[k] : 0.f;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    float wk[16];
    switch (g.sh_degree) {
        case 3: sh_weights<16>(g.sh + i * 48, gch, wk); break;
        case 1: sh_weights<4>(g.sh + i * 12, gch, wk); break;
        case 2: sh_weights<9>(g.sh + i * 27, gch, wk); break;
        default: sh_weights<1>(g.sh + i * 3, gch, wk); break;
    }
    if (out.d_sh) {
        float Y[16];
        sh_basis(g.sh_degree, cc.dl[0], cc.dl[1], cc.dl[2], Y);
        for (int k = 0; k < K; k++) {
            float* ds = out.d_sh + i * (int64_t)K * 3 + 3 * k;
            ds[0] += gch[0] * Y[k];
            ds[1] += gch[1] * Y[k];
            ds[2] += gch[2] * Y[k];
        }
    }
    float gdl[3];
    sh_grad(g.sh_degree, cc.dl[0], cc.dl[1], cc.dl[2], wk, gdl[0], gdl[1], gdl[2]);
    float ddir[3];
    if (g.dq) {
        for (int k = 0; k < 3; k++) ddir[k] = cc.Ml[k] * gdl[0] + cc.Ml[3 + k] * gdl[1] + cc.Ml[6 + k] * gdl[2];
        // Ml = Rh Rp^T, dMl = gdl dir^T:  dRh = dMl Rp, dRp = dMl^T Rh
        for (int r = 0; r < 3; r++)
            for (int k = 0; k < 3; k++) {
                dRh[3 * r + k] += gdl[r] * (cc.dir[0] * o.Rp[k] + cc.dir[1] * o.Rp[3 + k] + cc.dir[2] * o.Rp[6 + k]);
                dRp[3 * r + k] += cc.dir[r] * (gdl[0] * cc.Rh[k] + gdl[1] * cc.Rh[3 + k] + gdl[2] * cc.Rh[6 + k]);
            }
    } else {
        ddir[0] = gdl[0]; ddir[1] = gdl[1]; ddir[2] = gdl[2];
    }
    {
        const float pd = ddir[0] * cc.dir[0] + ddir[1] * cc.dir[1] + ddir[2] * cc.dir[2];
        for (int k = 0; k < 3; k++) dm[k] += (ddir[k] - cc.dir[k] * pd) / cc.wn;
    }

    // conic (A, B, C) = (c, -b, a) / det
    const float a = o.a, b = o.b, c = o.c, det = o.det, id2 = 1.0f / (det * det), idt = 1.0f / det;
    const float da = dA * (-c * c * id2) + dB * (b * c * id2) + dC * (idt - a * c * id2);
    const float db = dA * (2.f * b * c * id2) + dB * (-idt - 2.f * b * b * id2) + dC * (2.f * a * b * id2);
    const float dc = dA * (idt - a * c * id2) + dB * (a * b * id2) + dC * (-a * a * id2);
    // Sigma2 = T Sigma T^T: G2 = [[da, db/2], [db/2, dc]]
    const float G00 = da, G01 = 0.5f * db, G11 = dc;
    const float T0[3] = {o.T00, o.T01, o.T02}, T1[3] = {o.T10, o.T11, o.T12};
    const float S[9] = {o.S00, o.S01, o.S02, o.S01, o.S11, o.S12, o.S02, o.S12, o.S22};
    float dS[9];
    for (int p = 0; p < 3; p++)
        for (int q = 0; q < 3; q++)
            dS[3 * p + q] = T0[p] * (G00 * T0[q] + G01 * T1[q]) + T1[p] * (G01 * T0[q] + G11 * T1[q]);
    // dT = 2 G2 T Sigma
    float TS0[3], TS1[3];
    for (int q = 0; q < 3; q++) {
        TS0[q] = T0[0] * S[q] + T0[1] * S[3 + q] + T0[2] * S[6 + q];
        TS1[q] = T1[0] * S[q] + T1[1] * S[3 + q] + T1[2] * S[6 + q];
    }
    float dT0[3], dT1[3];
    for (int q = 0; q < 3; q++) {
        dT0[q] = 2.f * (G00 * TS0[q] + G01 * TS1[q]);
        dT1[q] = 2.f * (G01 * TS0[q] + G11 * TS1[q]);
    }
    const float* R = cam.R;
    const float dj00 = dT0[0] * R[0] + dT0[1] * R[1] + dT0[2] * R[2];
    const float dj02 = dT0[0] * R[6] + dT0[1] * R[7] + dT0[2] * R[8];
    const float dj11 = dT1[0] * R[3] + dT1[1] * R[4] + dT1[2] * R[5];
    const float dj12 = dT1[0] * R[6] + dT1[1] * R[7] + dT1[2] * R[8];
    const float tx = o.t[0], ty = o.t[1], tz = o.t[2], itz = 1.0f / tz, itz2 = itz * itz;
    const float fx = cam.fx, fy = cam.fy;
    float dtx = 0.f, dty = 0.f, dtz = 0.f;
    dtz += dj00 * (-fx * itz2) + dj11 * (-fy * itz2) + dj02 * (fx * o.txc * itz2) + dj12 * (fy * o.tyc * itz2);
    const float dtxc = dj02 * (-fx * itz), dtyc = dj12 * (-fy * itz);
    if (!o.clx) { dtx += dtxc * itz; dtz += -dtxc * tx * itz2; }
    if (!o.cly) { dty += dtyc * itz; dtz += -dtyc * ty * itz2; }
    dtx += du * fx * itz;
    dty += dv * fy * itz;
    dtz += -du * fx * tx * itz2 - dv * fy * ty * itz2;
    for (int k = 0; k < 3; k++) dm[k] += R[k] * dtx + R[3 + k] * dty + R[6 + k] * dtz;

    // Sigma = M M^T with M = Rp diag(s): dM = 2 dS M
    float M[9];
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) M[3 * r + k] = o.Rp[3 * r + k] * o.s[k];
    float ds[3] = {0.f, 0.f, 0.f};
    for (int r = 0; r < 3; r++)
        for (int k = 0; k < 3; k++) {
            const float dMrk = 2.f * (dS[3 * r] * M[k] + dS[3 * r + 1] * M[3 + k] + dS[3 * r + 2] * M[6 + k]);
            dRp[3 * r + k] += dMrk * o.s[k];
            ds[k] += dMrk * o.Rp[3 * r + k];
        }
    if (out.d_log_scales)
        for (int k = 0; k < 3; k++) out.d_log_scales[3 * i + k] += ds[k] * o.s[k];

    // rotations -> quaternions
    float dqp[4] = {0.f, 0.f, 0.f, 0.f}, dqh[4] = {0.f, 0.f, 0.f, 0.f};
    quat_rot_adj(o.qp, dRp, dqp);
    if (g.dq) {
        quat_rot_adj(o.qh, dRh, dqh);
        const float bw = o.dh[0], bx = o.dh[1], by = o.dh[2], bz = o.dh[3];
        const float aw = o.qh[0], ax = o.qh[1], ay = o.qh[2], az = o.qh[3];
        // q' = qh (x) dh; gradient with respect to qh is Rb^T dqp, to dh is La^T dqp
        dqh[0] += bw * dqp[0] + bx * dqp[1] + by * dqp[2] + bz * dqp[3];
        dqh[1] += -bx * dqp[0] + bw * dqp[1] - bz * dqp[2] + by * dqp[3];
        dqh[2] += -by * dqp[0] + bz * dqp[1] + bw * dqp[2] - bx * dqp[3];
        dqh[3] += -bz * dqp[0] - by * dqp[1] + bx * dqp[2] + bw * dqp[3];
        float ddh[4];
        ddh[0] = aw * dqp[0] + ax * dqp[1] + ay * dqp[2] + az * dqp[3];
        ddh[1] = -ax * dqp[0] + aw * dqp[1] + az * dqp[2] - ay * dqp[3];
        ddh[2] = -ay * dqp[0] - az * dqp[1] + aw * dqp[2] + ax * dqp[3];
        ddh[3] = -az * dqp[0] + ay * dqp[1] - ax * dqp[2] + aw * dqp[3];
        if (out.d_dq) {
            const float pd = o.dh[0] * ddh[0] + o.dh[1] * ddh[1] + o.dh[2] * ddh[2] + o.dh[3] * ddh[3];
            const bool nz = o.dn > 1e-12f;
            for (int k = 0; k < 4; k++)
                out.d_dq[4 * i + k] += nz ? (ddh[k] - o.dh[k] * pd) / o.dn : ddh[k] / o.dn;
        }
    } else {
        for (int k = 0; k < 4; k++) dqh[k] += dqp[k];
    }
    if (out.d_quats && o.qn > 0.f) {
        const float pd = o.qh[0] * dqh[0] + o.qh[1] * dqh[1] + o.qh[2] * dqh[2] + o.qh[3] * dqh[3];
        for (int k = 0; k < 4; k++) out.d_quats[4 * i + k] += (dqh[k] - o.qh[k] * pd) / o.qn;
    }
    for (int k = 0; k < 3; k++) {
        if (out.d_means) out.d_means[3 * i + k] += dm[k];
        if (out.d_dmu) out.d_dmu[3 * i + k] += dm[k];
    }
}

__global__ __launch_bounds__(256) void k_debug_keys(const uint2* __restrict__ ranges, const uint32_t* __restrict__ vals,
                                                    const uint32_t* __restrict__ key, int ntiles,
                                                    uint64_t* __restrict__ keys_out) {
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const uint2 r = ranges[t];
    for (uint32_t e = r.x + threadIdx.x; e < r.y; e += 256) keys_out[e] = ((uint64_t)t << 32) | key[vals[e]];
}

__global__ __launch_bounds__(256) void k_debug_records(int64_t n, const float4* __restrict__ rec,
                                                       int32_t* __restrict__ box, float* __restrict__ rec9) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float4 a = rec[3 * i], b = rec[3 * i + 1], c = rec[3 * i + 2];
    if (box) {
        const uint32_t b0 = __float_as_uint(c.y), b1 = __float_as_uint(c.z);
        box[4 * i + 0] = b0 & 0xFFFF; box[4 * i + 1] = b0 >> 16;
        box[4 * i + 2] = b1 & 0xFFFF; box[4 * i + 3] = b1 >> 16;
    }
    if (rec9) {
        float v[9] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x};
        for (int k = 0; k < 9; k++) rec9[9 * i + k] = v[k];
    }
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

void preprocess(const Launch& L, const GaussDev& g, const CamDev& cam, float4* rec, uint32_t* key, uint2* rect,
                uint32_t* count) {
    if (g.n <= 0) return;
    if (L.prof) L.prof->begin("preprocess_fwd", L.st);
    hipLaunchKernelGGL(k_preprocess, dim3(blocks_for(g.n, 256)), dim3(256), 0, L.st, g, cam, rec, key, rect, count);
    if (L.prof) L.prof->end(L.st);
}

void emit_pairs(const Launch& L, int64_t n, const uint32_t* key, const uint2* rect, const uint64_t* offs, int tiles_x,
                uint64_t cap, uint64_t* keys, uint32_t* vals) {
    if (n <= 0) return;
    if (L.prof) L.prof->begin("emit_keys", L.st);
    hipLaunchKernelGGL(k_emit, dim3(blocks_for(n, 256)), dim3(256), 0, L.st, n, key, rect, offs, tiles_x, cap, keys,
                       vals);
    if (L.prof) L.prof->end(L.st);
}

void ranges_from_keys(const Launch& L, const uint64_t* keys, int64_t K, int ntiles, uint2* ranges) {
    if (L.prof) L.prof->begin("tile_ranges", L.st);
    hipLaunchKernelGGL(k_zero_ranges, dim3(blocks_for(ntiles, 256)), dim3(256), 0, L.st, ranges, ntiles);
    if (K > 0)
        hipLaunchKernelGGL(k_ranges_from_keys, dim3(blocks_for(K, 256)), dim3(256), 0, L.st, keys, K, ranges);
    if (L.prof) L.prof->end(L.st);
}

void bin_gather(const Launch& L, const uint32_t* order, int64_t n, const uint2* rect, const uint32_t* count,
                const uint64_t* goff, uint64_t cap, uint2* srect, uint32_t* sgoff, uint32_t* zero, int64_t nzero) {
    if (n <= 0) return;
    if (L.prof) L.prof->begin("bin_gather", L.st);
    hipLaunchKernelGGL(k_bin_gather, dim3(blocks_for(std::max(n, nzero), 256)), dim3(256), 0, L.st, order, n, rect,
                       count, goff, (uint32_t)std::min<uint64_t>(cap, 0xFFFFFFFFull), srect, sgoff, zero, nzero);
    if (L.prof) L.prof->end(L.st);
}

int64_t bin_chunks(int64_t n) { return (((n + kBinChunk - 1) / kBinChunk) + 7) / 8 * 8; }

static dim3 bin_grid(int64_t nchunks, int tiles_y) {
    return dim3((unsigned)(nchunks * ((tiles_y + kBinRowsPerBlock - 1) / kBinRowsPerBlock)));
}

void bin_count(const Launch& L, const uint32_t* order, int64_t n, const uint2* srect, int tiles_x, int tiles_y,
               uint32_t* hist, uint32_t* ttot) {
    const int64_t nchunks = n > 0 ? bin_chunks(n) : 0;
    if (nchunks == 0) return;
    if (L.prof) L.prof->begin("bin_count", L.st);
    const unsigned grid = (unsigned)((nchunks / kCountGroup) * ((tiles_y + kBinRowsPerBlock - 1) / kBinRowsPerBlock));
    hipLaunchKernelGGL(k_bin_count, dim3(grid), dim3(kBinThreads), 0, L.st, srect, n, tiles_x, tiles_y, nchunks, hist,
                       ttot);
    if (L.prof) L.prof->end(L.st);
}


int64_t bin_scan_part_words(int64_t nchunks, int ntiles) {
    return ((nchunks + kBinScanSeg - 1) / kBinScanSeg) * (int64_t)ntiles;
}

void bin_scan(const Launch& L, const uint32_t* hist, int64_t nchunks, int ntiles, uint32_t cap, uint32_t* base,
              uint64_t* total, uint32_t* part, uint32_t* ttot, uint64_t* toff, uint64_t* tmp) {
    if (nchunks <= 0 || ntiles <= 0) return;
    if (L.prof) L.prof->begin("scan", L.st);
    const int64_t nseg = (nchunks + kBinScanSeg - 1) / kBinScanSeg;
    const dim3 grid((unsigned)((ntiles + 255) / 256), (unsigned)std::min<int64_t>(nseg, 65535));
    hipLaunchKernelGGL(k_bin_scan_part, grid, dim3(256), 0, L.st, hist, nchunks, ntiles, nseg, part);
    hipLaunchKernelGGL(k_bin_scan_tiles, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, L.st, part, nseg,
                       ntiles, ttot);
    if (L.prof) L.prof->end(L.st);
    scan_u32_to_u64(L, ttot, ntiles, toff, total, tmp);
    if (L.prof) L.prof->begin("scan", L.st);
    hipLaunchKernelGGL(k_bin_scan_base, grid, dim3(256), 0, L.st, hist, nchunks, ntiles, nseg, part, toff, cap, base);
    if (L.prof) L.prof->end(L.st);
}

template <typename B>
static void bin_scatter_impl(const Launch& L, const uint32_t* order, int64_t n, const uint2* srect,
                             const uint32_t* sgoff, int tiles_x, int tiles_y, const B* base, uint64_t cap,
                             uint32_t* vals, uint32_t* gpos) {
    const int64_t nchunks = n > 0 ? bin_chunks(n) : 0;
    if (nchunks == 0) return;
    if (L.prof) L.prof->begin("bin_scatter", L.st);
    if (gpos)
        hipLaunchKernelGGL((k_bin_rows<B, true>), bin_grid(nchunks, tiles_y), dim3(kBinThreads), 0, L.st, order, n,
                           srect, sgoff, tiles_x, tiles_y, nchunks, base, (uint32_t)cap, vals, gpos);
    else
        hipLaunchKernelGGL((k_bin_rows<B, false>), bin_grid(nchunks, tiles_y), dim3(kBinThreads), 0, L.st, order, n,
                           srect, sgoff, tiles_x, tiles_y, nchunks, base, (uint32_t)cap, vals, gpos);
    if (L.prof) L.prof->end(L.st);
}

void bin_scatter(const Launch& L, const uint32_t* order, int64_t n, const uint2* srect, const uint32_t* sgoff,
                 int tiles_x, int tiles_y, const uint32_t* base, uint64_t cap, uint32_t* vals, uint32_t* gpos) {
    bin_scatter_impl(L, order, n, srect, sgoff, tiles_x, tiles_y, base, cap, vals, gpos);
}

void bin_scatter_chunked(const Launch& L, const uint32_t* order, int64_t n, const uint2* srect, int tiles_x,
                         int tiles_y, const uint64_t* cmb, uint64_t cap, uint32_t* vals) {
    bin_scatter_impl(L, order, n, srect, (const uint32_t*)nullptr, tiles_x, tiles_y, cmb, cap, vals,
                     (uint32_t*)nullptr);
}

__global__ __launch_bounds__(256) void k_chunked_to_tile_major(const uint32_t* __restrict__ hist,
                                                               const uint64_t* __restrict__ cmb,
                                                               const uint32_t* __restrict__ base_tm, int64_t m,
                                                               uint64_t cap, const uint32_t* __restrict__ vals_cm,
                                                               uint32_t* __restrict__ vals_tm) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;   // (chunk, tile) in [chunk][tile] order
    if (i >= m) return;
    const uint32_t len = hist[i];
    const uint64_t src = cmb[i], dst = base_tm[i];
    for (uint32_t k = 0; k < len; k++)
        if (src + k < cap && dst + k < cap) vals_tm[dst + k] = vals_cm[src + k];
}

void chunked_to_tile_major(const Launch& L, const uint32_t* hist, const uint64_t* cmb, const uint32_t* base_tm,
                           int64_t nchunks, int ntiles, uint64_t cap, const uint32_t* vals_cm, uint32_t* vals_tm) {
    const int64_t m = nchunks * ntiles;
    if (m <= 0) return;
    hipLaunchKernelGGL(k_chunked_to_tile_major, dim3(blocks_for(m, 256)), dim3(256), 0, L.st, hist, cmb, base_tm, m, cap,
                       vals_cm, vals_tm);
}

void gpos_from_pairs(const Launch& L, const uint64_t* keys, const uint32_t* vals, int64_t K, const uint2* rect,
                     const uint64_t* goff, int tiles_x, uint64_t cap, uint32_t* gpos) {
    if (K <= 0) return;
    hipLaunchKernelGGL(k_gpos_from_pairs, dim3(blocks_for(K, 256)), dim3(256), 0, L.st, keys, vals, K, rect, goff,
                       tiles_x, cap, gpos);
}

void ranges_from_hist(const Launch& L, const uint32_t* base, const uint64_t* total, int ntiles, uint64_t cap,
                      uint2* ranges, int* overflow) {
    if (L.prof) L.prof->begin("tile_ranges", L.st);
    hipLaunchKernelGGL(k_ranges_from_hist, dim3(blocks_for(ntiles, 256)), dim3(256), 0, L.st, base, total, ntiles, cap,
                       ranges, overflow);
    if (L.prof) L.prof->end(L.st);
}


static unsigned blend_grid(int ntiles) { return (unsigned)(((ntiles + 7) / 8) * 8); }

// pixels per thread of the blend kernels
constexpr int kBlendRows = GS3_BLEND_ROWS_FWD;
constexpr int kBlendRowsBwd = GS3_BLEND_ROWS_BWD;

void tile_order(const Launch& L, const uint2* ranges, const uint32_t* walk, int ntiles, int* order) {
    if (L.prof) L.prof->begin("tile_order", L.st);
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, L.st, ranges, walk, ntiles, order);
    if (L.prof) L.prof->end(L.st);
}

void blend_forward(const Launch& L, const CamDev& cam, const uint2* ranges, const uint32_t* vals, const float4* rec,
                   float* image, float* T_final, uint32_t* last, uint32_t* tile_walk, const int* order,
                   const ChunkDev* chunks) {
    const int ntiles = cam.tiles_x * cam.tiles_y;
    if (L.prof) L.prof->begin("blend_fwd", L.st);
    const dim3 grid(order ? (unsigned)ntiles : blend_grid(ntiles));
    const ChunkDev cl = chunks ? *chunks : ChunkDev{};
    if (chunks)
        hipLaunchKernelGGL((k_blend_fwd<kBlendRows, true>), grid, dim3(kTile * kTile / kBlendRows), 0, L.st, cam, ntiles,
                           ranges, vals, rec, image, T_final, last, tile_walk, order, cl);
    else
        hipLaunchKernelGGL((k_blend_fwd<kBlendRows, false>), grid, dim3(kTile * kTile / kBlendRows), 0, L.st, cam,
                           ntiles, ranges, vals, rec, image, T_final, last, tile_walk, order, cl);
    if (L.prof) L.prof->end(L.st);
}

void blend_backward(const Launch& L, const CamDev& cam, const uint2* ranges, const uint32_t* vals, const float4* rec,
                    const float* d_image, const float* T_final, const uint32_t* last, const GatherDev& ga,
                    float* accum, bool want_opacity, const int* order) {
    const int ntiles = cam.tiles_x * cam.tiles_y;
    if (L.prof) L.prof->begin("blend_bwd", L.st);
    const bool records = ga.grec_cap > 0;
    constexpr int R = kBlendRowsBwd;
    auto kern = records ? (want_opacity ? k_blend_bwd<R, true, true> : k_blend_bwd<R, true, false>)
                        : (want_opacity ? k_blend_bwd<R, false, true> : k_blend_bwd<R, false, false>);
    hipLaunchKernelGGL(kern, dim3(order ? (unsigned)ntiles : blend_grid(ntiles)), dim3(kTile * kTile / R), 0, L.st,
                       cam, ntiles, ranges, vals, rec, d_image, T_final, last, ga.tile_walk, ga.walk_off, ga.grec,
                       (uint32_t)ga.grec_cap, accum, order);
    if (L.prof) L.prof->end(L.st);
}

void preprocess_backward(const Launch& L, const GaussDev& g, const CamDev& cam, const float* accum,
                         const GatherDev& ga, const GradsDev& out) {
    if (g.n <= 0) return;
    if (L.prof) L.prof->begin("preprocess_bwd", L.st);
    hipLaunchKernelGGL(k_preprocess_bwd, dim3(blocks_for(g.n, 256)), dim3(256), 0, L.st, g, cam, accum, ga, out);
    if (L.prof) L.prof->end(L.st);
}

void debug_keys(const Launch& L, const uint2* ranges, const uint32_t* vals, const uint32_t* key, int ntiles,
                uint64_t* keys_out) {
    hipLaunchKernelGGL(k_debug_keys, dim3((unsigned)ntiles), dim3(256), 0, L.st, ranges, vals, key, ntiles, keys_out);
}

void debug_records(const Launch& L, int64_t n, const float4* rec, int32_t* box, float* rec9) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_debug_records, dim3(blocks_for(n, 256)), dim3(256), 0, L.st, n, rec, box, rec9);
}

}  // namespace gs3
