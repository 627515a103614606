// Host-side launchers of the gs3 kernels (internal to libgs3.so).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace gs3 {

// Optional per-kernel timing: when `prof` is set, every launch is bracketed
// by events recorded on the launch stream.
struct Profiler {
    virtual ~Profiler() = default;
    virtual void begin(const char* name, hipStream_t st) = 0;
    virtual void end(hipStream_t st) = 0;
};

struct Launch {
    hipStream_t st;
    Profiler* prof;
};

// ---- scan / sort (sort.hip) ------------------------------------------------
// Exclusive prefix sum of n u32 values into u32 or u64 outputs; the grand
// total goes to *total (device).  `tmp` holds scan_tmp_words(n) u64.
int64_t scan_tmp_words(int64_t n);
void scan_u32_to_u64(const Launch& L, const uint32_t* in, int64_t n, uint64_t* out, uint64_t* total, uint64_t* tmp);
void scan_u32_to_u32(const Launch& L, const uint32_t* in, int64_t n, uint32_t* out, uint64_t* total, uint64_t* tmp);

// Stable LSD radix sort of (key, value) pairs over the low `bits` key bits.
// Buffers ping-pong; returns the index (0 or 1) holding the result.
// `hist` holds radix_hist_words(n) u32, `tmp` scan_tmp_words(radix_hist_words(n)) u64.
int64_t radix_hist_words(int64_t n);
int radix_sort_u32(const Launch& L, uint32_t* keys[2], uint32_t* vals[2], int64_t n, int bits, uint32_t* hist,
                   uint64_t* tmp);
int radix_sort_u64(const Launch& L, uint64_t* keys[2], uint32_t* vals[2], int64_t n, int bits, uint32_t* hist,
                   uint64_t* tmp);
// The same sort of keys_in (left unchanged) with the positions 0..n-1 as
// values: the order that sorts keys_in, without copying the keys first.
int radix_order_u32(const Launch& L, const uint32_t* keys_in, uint32_t* keys[2], uint32_t* vals[2], int64_t n,
                    int bits, uint32_t* hist, uint64_t* tmp);

void morton_codes(const Launch& L, const float* means, int64_t n, const float lo[3], const float inv[3],
                  uint32_t* code, uint32_t* idx);
void gather_rows(const Launch& L, const float* src, const uint32_t* perm, int64_t n, int rf, float* dst);

void fill_u32(const Launch& L, uint32_t* p, uint32_t v, int64_t n);
void fill_f32(const Launch& L, float* p, float v, int64_t n);
void iota_u32(const Launch& L, uint32_t* p, int64_t n);
// *out (one u64, device) = sum of the n values
void sum_u32(const Launch& L, const uint32_t* a, int64_t n, uint64_t* out);

// ---- rasterizer (raster.hip) -------------------------------------------------
void preprocess(const Launch& L, const GaussDev& g, const CamDev& cam, float4* rec, uint32_t* key, uint2* rect,
                uint32_t* count);
// radix64 path: keys/vals of every pair in Gaussian order from exclusive offsets
void emit_pairs(const Launch& L, int64_t n, const uint32_t* key, const uint2* rect, const uint64_t* offs,
                int tiles_x, uint64_t cap, uint64_t* keys, uint32_t* vals);
void ranges_from_keys(const Launch& L, const uint64_t* keys, int64_t K, int ntiles, uint2* ranges);
// depth-first path: per-chunk tile histograms of depth-ordered Gaussians,
// then an order-preserving scatter of Gaussian indices.
#ifndef GS3_BIN_CHUNK
#define GS3_BIN_CHUNK 512
#endif
constexpr int kBinChunk = GS3_BIN_CHUNK;
constexpr int kMaxTilesX = 256;   // widest image: 4096 pixels
// chunks of kBinChunk depth-ordered Gaussians for n Gaussians, rounded up to
// a multiple of 8 (the passes give each XCD an eighth; padding chunks are empty)
int64_t bin_chunks(int64_t n);
// tile rectangles (empty for culled Gaussians) and, when sgoff is set, the
// first pair slots goff, gathered into depth order; also zeroes zero[0,
// nzero) (the per-tile totals bin_count adds to; null with nzero 0)
void bin_gather(const Launch& L, const uint32_t* order, int64_t n, const uint2* rect, const uint32_t* count,
                const uint64_t* goff, uint64_t cap, uint2* srect, uint32_t* sgoff, uint32_t* zero, int64_t nzero);
// Pairs per (chunk, tile), chunk-major: hist[chunk * ntiles + tile] with
// ntiles = tiles_x * tiles_y, so each pass writes and reads a tile row of one
// chunk as consecutive words; ttot (optional, zeroed by the caller) receives
// the pairs per tile.
void bin_count(const Launch& L, const uint32_t* order, int64_t n, const uint2* srect, int tiles_x, int tiles_y,
               uint32_t* hist, uint32_t* ttot);
// ranges[t] = [start, start + len[t]) clamped to cap, start the exclusive
// prefix of len; sets *overflow when *total (the list's length) exceeds cap
void tile_ranges_from_counts(const Launch& L, const uint32_t* len, int64_t ntiles, uint64_t cap, const uint64_t* total,
                             uint2* ranges, int* overflow);
// First slot of every (tile, chunk) segment in the tile-major pair list:
// base[chunk * ntiles + tile] = (pairs of earlier tiles) + (pairs of the
// tile in earlier chunks), clamped to cap; the grand total goes to *total.
// Scratch: part (bin_scan_part_words u32), ttot (ntiles u32), toff (ntiles
// u64) and the scan's tmp.
int64_t bin_scan_part_words(int64_t nchunks, int ntiles);
void bin_scan(const Launch& L, const uint32_t* hist, int64_t nchunks, int ntiles, uint32_t cap, uint32_t* base,
              uint64_t* total, uint32_t* part, uint32_t* ttot, uint64_t* toff, uint64_t* tmp);
// also records, for each Gaussian's k-th rectangle tile, the slot of that
// pair: gpos[goff[id] + k] (goff = exclusive scan of the tile counts)
void bin_scatter(const Launch& L, const uint32_t* order, int64_t n, const uint2* srect, const uint32_t* sgoff,
                 int tiles_x, int tiles_y, const uint32_t* base, uint64_t cap, uint32_t* vals, uint32_t* gpos);
// The chunk-major pair list of the depth-first binning, as the forward
// blend reads it: segment lengths hist[chunk][tile], segment starts
// cmb[chunk][tile] (the exclusive scan of hist in that order), and the
// tile-major list `walked`, into which the forward writes each entry it
// stages at its tile-major slot (the backward walks that list).
struct ChunkDev {
    const uint32_t* hist;
    const uint64_t* cmb;
    int64_t nchunks;
    uint32_t cap;
    uint32_t* walked;
};
// The same into the chunk-major list: cmb = exclusive scan of hist in its
// [chunk][tile] order (the start of every (chunk, tile) segment).
void bin_scatter_chunked(const Launch& L, const uint32_t* order, int64_t n, const uint2* srect, int tiles_x,
                         int tiles_y, const uint64_t* cmb, uint64_t cap, uint32_t* vals);
// Copy every (chunk, tile) segment of the chunk-major list to its slot in
// the tile-major list (base_tm: the tile-major first slot of each segment,
// from bin_scan); slots at or past cap are skipped.
void chunked_to_tile_major(const Launch& L, const uint32_t* hist, const uint64_t* cmb, const uint32_t* base_tm,
                           int64_t nchunks, int ntiles, uint64_t cap, const uint32_t* vals_cm, uint32_t* vals_tm);
void gpos_from_pairs(const Launch& L, const uint64_t* keys, const uint32_t* vals, int64_t K, const uint2* rect,
                     const uint64_t* goff, int tiles_x, uint64_t cap, uint32_t* gpos);
void ranges_from_hist(const Launch& L, const uint32_t* base, const uint64_t* total, int ntiles, uint64_t cap,
                      uint2* ranges, int* overflow);

// Per-pair gradient records of the backward blend: walked entries of tile t
// (list positions [start_t, start_t + tile_walk[t])) get compact indices
// walk_off[t] + (position - start_t); term c of entry w lives at
// grec[c * grec_cap + w].  Entries past grec_cap fall back to atomics.
struct GatherDev {
    const uint2* rect;
    const uint64_t* goff;
    const uint32_t* gpos;
    const uint2* ranges;
    const uint32_t* tile_walk;
    const uint32_t* walk_off;
    float* grec;
    uint64_t grec_cap;
    uint64_t cap;   // pair capacity (gpos length)
};

// Longest-first launch order of the tiles: by list length (walk == nullptr)
// or by walked entries.  `order` holds ntiles ints.
void tile_order(const Launch& L, const uint2* ranges, const uint32_t* walk, int ntiles, int* order);
// `order` (optional) maps workgroups to tiles
// chunks: the chunk-major list (vals is then that list), or NULL for a
// tile-major list read through ranges.
void blend_forward(const Launch& L, const CamDev& cam, const uint2* ranges, const uint32_t* vals, const float4* rec,
                   float* image, float* T_final, uint32_t* last, uint32_t* tile_walk, const int* order,
                   const ChunkDev* chunks);
void blend_backward(const Launch& L, const CamDev& cam, const uint2* ranges, const uint32_t* vals,
                    const float4* rec, const float* d_image, const float* T_final, const uint32_t* last,
                    const GatherDev& ga, float* accum, bool want_opacity, const int* order);

struct GradsDev {
    float *d_means, *d_quats, *d_log_scales, *d_opac, *d_sh, *d_dmu, *d_dq;
    float *d_uv, *d_conic, *d_opacity, *d_rgb;
    float *vgrad, *vcount;   // view-space gradient norm and visibility count (accumulated)
};
void preprocess_backward(const Launch& L, const GaussDev& g, const CamDev& cam, const float* accum,
                         const GatherDev& ga, const GradsDev& out);
void debug_keys(const Launch& L, const uint2* ranges, const uint32_t* vals, const uint32_t* key, int ntiles,
                uint64_t* keys_out);
void debug_records(const Launch& L, int64_t n, const float4* rec, int32_t* box, float* rec9);

// ---- transform bake (bake.hip) -------------------------------------------------
struct ShRotConst {
    float dirs[3 * 15];       // bands 1..3: 3 + 5 + 7 directions
    float ainv[9 + 25 + 49];  // A_l^{-1}, row-major, bands 1..3
};
ShRotConst make_shrot_const();
void transform_bake(const Launch& L, const GaussDev& g, const ShRotConst& rc, float* mu_out, float* q_out,
                    float* sh_out);

// ---- Stage 2 (stage2.hip) -------------------------------------------------------
// idx <- ascending indices i with den ? (den[i] > 0 && num[i]/den[i] > thr)
// : num[i] >= thr; the count lands in *total.  flag, pos: n u32 scratch.
void select_indices(const Launch& L, const float* num, const float* den, int64_t n, float thr, uint32_t* flag,
                    uint32_t* pos, uint64_t* total, uint64_t* tmp, uint32_t* idx);
// mode 0: spawn (identity rotation, opacity logit0); mode 1: split (rotation
// and opacity kept, log-scale + log_shrink).  Position mu + sqrt(2) R S z.
void spawn(const Launch& L, const GaussDev& g, const uint32_t* idx, int64_t m, const float* z, int mode,
           float logit0, float log_shrink, float* mu, float* q, float* ls, float* lo, float* sh);

// ---- loss (loss.hip) ---------------------------------------------------------
struct LossWork {
    float* partial_maps;   // 3 x (3 H W) SSIM partial derivatives
    double* block_sums;    // 2 x blocks
    int max_blocks;
};
int64_t loss_map_floats(int H, int W);
int loss_blocks(int H, int W);
void loss_forward_backward(const Launch& L, const float* x, const float* y, int H, int W, float lambda,
                           const LossWork& w, float* loss_dev, float* d_image, int* nonfinite);

// ---- optimiser ---------------------------------------------------------------
void adam(const Launch& L, float* p, const float* g, float* m, float* v, int64_t n, int step, float lr, float b1,
          float b2, float eps);

}  // namespace gs3
