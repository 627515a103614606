// C ABI of libgs3.so (declared in include/gs3.h).
#include <math.h>
#include <string.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/gs3.h"
#include "kernels.h"
#include "ntc.h"

using namespace gs3;

namespace {

struct EventProfiler : Profiler {
    struct Rec {
        std::string name;
        hipEvent_t a, b;   // null when the launch is not timed
    };
    std::string only;                 // time only this kernel (empty: every kernel)
    std::vector<hipEvent_t> pool;     // created events, reused across launches
    std::vector<Rec> pending;
    std::vector<Rec> open;
    std::map<std::string, std::pair<double, int64_t>> totals;
    // profiling is best effort: a launch whose events cannot be created or
    // recorded is simply not timed
    hipEvent_t take() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
    void give(hipEvent_t e) {
        if (e) pool.push_back(e);
    }
    void begin(const char* name, hipStream_t st) override {
        Rec r{name, nullptr, nullptr};
        if (only.empty() || only == name) {
            r.a = take();
            r.b = take();
            if (!r.a || !r.b || hipEventRecord(r.a, st) != hipSuccess) {
                give(r.a);
                give(r.b);
                r.a = r.b = nullptr;
            }
        }
        open.push_back(r);
    }
    void end(hipStream_t st) override {
        if (open.empty()) return;
        Rec r = open.back();
        open.pop_back();
        if (!r.a) return;
        if (hipEventRecord(r.b, st) != hipSuccess) {
            give(r.a);
            give(r.b);
            return;
        }
        pending.push_back(r);
    }
    void collect() {
        for (auto& r : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                auto& t = totals[r.name];
                t.first += ms;
                t.second += 1;
            }
            give(r.a);
            give(r.b);
        }
        pending.clear();
    }
    ~EventProfiler() override {
        collect();
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

struct Slot {
    float4* rec = nullptr;
    uint32_t* key = nullptr;
    uint2* rect = nullptr;
    uint32_t* count = nullptr;
    uint32_t* vals[2] = {nullptr, nullptr};
    uint64_t* pkeys[2] = {nullptr, nullptr};
    int cur = 0;
    uint2* ranges = nullptr;
    float* T_final = nullptr;
    uint32_t* last = nullptr;
    uint64_t* total = nullptr;
    uint64_t* goff = nullptr;        // exclusive scan of the tile counts
    uint32_t* gpos = nullptr;        // per Gaussian and rectangle tile: slot of that pair
    uint32_t* tile_walk = nullptr;   // list entries walked per tile by the forward blend
    int* order_fwd = nullptr;        // longest-first tile order of the forward blend
    int* order_bwd = nullptr;        // and of the backward blend
    // chunk-major list of the depth-first binning (without gradient records):
    // vals[0] holds the (chunk, tile) segments; `walked` the tile-major list,
    // filled by the forward up to each tile's last staged entry (and in full
    // by materialise_tile_major for the inspection calls)
    uint32_t* chist = nullptr;       // [chunk][tile] pairs
    uint64_t* cmb = nullptr;         // [chunk][tile] first slot in vals[0]
    uint32_t* ttot = nullptr;        // pairs per tile
    uint32_t* walked = nullptr;
    bool chunked = false;
    bool tile_major_full = false;    // walked holds the whole tile-major list
    int64_t nchunks = 0;
    bool valid = false;
    GaussDev g{};
    CamDev cam{};
    int64_t K_host = -1;
};

}  // namespace

struct gs3_ctx {
    gs3_config cfg{};
    hipStream_t st = nullptr;
    std::string err;
    std::vector<Slot> slots;
    std::vector<void*> allocs;
    int max_tiles = 0;
    // depth sort and binning
    uint32_t* dkeys[2] = {nullptr, nullptr};
    uint32_t* dvals[2] = {nullptr, nullptr};
    uint32_t* radix_hist = nullptr;
    uint64_t* scan_tmp = nullptr;
    uint32_t* bin_hist = nullptr;
    uint32_t* bin_base = nullptr;
    uint32_t* bin_part = nullptr;    // segment sums of the tile-major scan of bin_hist
    uint32_t* bin_ttot = nullptr;    // pairs per tile
    uint64_t* bin_toff = nullptr;    // first pair of each tile
    uint32_t* sel_flag = nullptr;    // selection scratch (max_gaussians each)
    uint32_t* sel_pos = nullptr;
    uint64_t* sel_total = nullptr;
    uint2* bin_rect = nullptr;       // tile rectangles in depth order
    uint32_t* bin_goff = nullptr;    // first pair slots in depth order (record mode)
    float* accum = nullptr;
    uint32_t* walk_off = nullptr;
    uint64_t* walk_total = nullptr;
    uint64_t* goff_total = nullptr;
    float* grec = nullptr;
    int64_t grec_cap = 0;
    int* flags = nullptr;   // [0] pair overflow, [1] non-finite loss
    uint64_t* sums = nullptr;        // two u64 sums of the inspection calls
    float* loss_maps = nullptr;
    double* loss_bsum = nullptr;
    // NTC
    NtcDev nd{};
    int64_t n_table_floats = 0, n_params = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    void* work = nullptr;
    int step = 0;
    float* g_part = nullptr;
    int max_parts = 0;
    double* warm_bsum = nullptr;
    // per-frame contribution lists of the table gradient
    void* enc_cache = nullptr;   // encoding of the prepared means from the last forward (n x 32)
    bool enc_valid = false;      // it matches the current parameters
    NtcCsr csr;
    const float* csr_means = nullptr;
    int64_t csr_n = -1, csr_cap = 0;
    uint64_t csr_token = 0;          // token of the current preparation (0: none)
    uint64_t last_token = 0;         // last token handed out
    std::vector<void*> csr_allocs;
    uint32_t* csr_keys[2] = {nullptr, nullptr};
    uint32_t* csr_vals[2] = {nullptr, nullptr};
    uint32_t* csr_hist = nullptr;
    uint64_t* csr_tmp = nullptr;
    EventProfiler prof;
    bool prof_on = false;

    Launch L() { return Launch{st, prof_on ? &prof : nullptr}; }

    int64_t bytes = 0;       // device memory held by the context (fixed workspaces)
    int64_t csr_bytes = 0;   // and by the per-frame contribution lists
    template <typename T>
    bool alloc(T** out, int64_t count) {
        *out = nullptr;
        if (count <= 0) count = 1;
        void* ptr = nullptr;
        if (hipMalloc(&ptr, (size_t)count * sizeof(T)) != hipSuccess) {
            err = "hipMalloc of " + std::to_string((long long)count * (long long)sizeof(T)) + " bytes failed";
            return false;
        }
        allocs.push_back(ptr);
        bytes += (int64_t)count * (int64_t)sizeof(T);
        *out = (T*)ptr;
        return true;
    }
    gs3_status fail(gs3_status s, const std::string& msg) {
        err = msg;
        return s;
    }
    gs3_status check_launch(const char* what) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(GS3_EHIP, std::string(what) + ": " + hipGetErrorString(e));
        return GS3_OK;
    }
};

static const char* kNullCtx = "null context";

static int tiles_of(int w, int h) { return ((w + kTile - 1) / kTile) * ((h + kTile - 1) / kTile); }

extern "C" {

gs3_status gs3_create(const gs3_config* cfg, gs3_ctx** out) {
    if (!cfg || !out) return GS3_EINVAL;
    *out = nullptr;
    if (cfg->max_gaussians < 1 || cfg->max_gaussians > (int64_t)1 << 31 || cfg->max_pairs < 1 ||
        cfg->max_pairs >= (int64_t)1 << 31 || cfg->max_width < 1 || cfg->max_height < 1 ||
        cfg->max_width > 32767 || cfg->max_height > 32767 || cfg->num_slots < 1 || cfg->num_slots > 8 ||
        (cfg->sort_mode != GS3_SORT_DEPTH_FIRST && cfg->sort_mode != GS3_SORT_RADIX64))
        return GS3_EINVAL;
    if (tiles_of(cfg->max_width, cfg->max_height) > GS3_MAX_TILES) return GS3_EINVAL;
    if ((cfg->max_width + 15) / 16 > kMaxTilesX) return GS3_EINVAL;
    if ((cfg->max_width + kTile - 1) / kTile > 2048) return GS3_EINVAL;
    // the binning passes launch bin_chunks(N) x ceil(tile rows / 8) workgroups
    // of 512 threads on a 1-D grid: keep that below 2^32 work-items
    if (bin_chunks(cfg->max_gaussians) * (((cfg->max_height + kTile - 1) / kTile + 7) / 8) * 512 >= ((int64_t)1 << 32))
        return GS3_EINVAL;
    gs3_ctx* c = new gs3_ctx();
    c->cfg = *cfg;
    c->max_tiles = tiles_of(cfg->max_width, cfg->max_height);
    const int64_t N = cfg->max_gaussians, PK = cfg->max_pairs, PX = (int64_t)cfg->max_width * cfg->max_height;
    const int64_t nchunks = bin_chunks(N);
    bool ok = true;
    c->slots.resize(cfg->num_slots);
    for (auto& s : c->slots) {
        ok = ok && c->alloc(&s.rec, 3 * N) && c->alloc(&s.key, N) && c->alloc(&s.rect, N) && c->alloc(&s.count, N) &&
             c->alloc(&s.vals[0], PK) && c->alloc(&s.ranges, c->max_tiles) && c->alloc(&s.T_final, PX) &&
             c->alloc(&s.last, PX) && c->alloc(&s.total, 1) && c->alloc(&s.goff, N) &&
             c->alloc(&s.gpos, cfg->grad_record_log2 > 0 ? PK : 1) && c->alloc(&s.tile_walk, c->max_tiles) &&
             c->alloc(&s.order_fwd, c->max_tiles) && c->alloc(&s.order_bwd, c->max_tiles);
        if (ok && cfg->sort_mode == GS3_SORT_RADIX64)
            ok = c->alloc(&s.vals[1], PK) && c->alloc(&s.pkeys[0], PK) && c->alloc(&s.pkeys[1], PK);
        if (ok && cfg->sort_mode == GS3_SORT_DEPTH_FIRST && cfg->grad_record_log2 <= 0)
            ok = c->alloc(&s.chist, (int64_t)c->max_tiles * nchunks) && c->alloc(&s.cmb, (int64_t)c->max_tiles * nchunks) &&
                 c->alloc(&s.ttot, c->max_tiles) && c->alloc(&s.walked, PK);
    }
    const int64_t sort_items = cfg->sort_mode == GS3_SORT_RADIX64 ? std::max(N, PK) : N;
    const int64_t hist_words = radix_hist_words(sort_items);
    const int64_t bin_words = (int64_t)c->max_tiles * nchunks;
    const int64_t scan_items = std::max(std::max(hist_words, bin_words), N);
    ok = ok && c->alloc(&c->dkeys[0], N) && c->alloc(&c->dkeys[1], N) && c->alloc(&c->dvals[0], N) &&
         c->alloc(&c->dvals[1], N) && c->alloc(&c->radix_hist, hist_words) &&
         c->alloc(&c->scan_tmp, scan_tmp_words(scan_items) + 4) && c->alloc(&c->accum, 9 * N) &&
         c->alloc(&c->flags, 4) && c->alloc(&c->sums, 2) && c->alloc(&c->loss_maps, loss_map_floats(cfg->max_height, cfg->max_width)) &&
         c->alloc(&c->walk_off, c->max_tiles) && c->alloc(&c->walk_total, 1) && c->alloc(&c->goff_total, 1) &&
         c->alloc(&c->sel_flag, N) && c->alloc(&c->sel_pos, N) && c->alloc(&c->sel_total, 1) &&
         c->alloc(&c->loss_bsum, 2 * (int64_t)loss_blocks(cfg->max_height, cfg->max_width));
    if (cfg->grad_record_log2 > 0) {
        c->grec_cap = std::min<int64_t>(PK, (int64_t)1 << std::min(cfg->grad_record_log2, 30));
        ok = ok && c->alloc(&c->grec, 9 * c->grec_cap);
    }
    if (ok && cfg->sort_mode == GS3_SORT_DEPTH_FIRST)
        ok = c->alloc(&c->bin_hist, bin_words) && c->alloc(&c->bin_base, bin_words) &&
             c->alloc(&c->bin_part, bin_scan_part_words(nchunks, c->max_tiles)) &&
             c->alloc(&c->bin_ttot, c->max_tiles) && c->alloc(&c->bin_toff, c->max_tiles) && c->alloc(&c->bin_rect, N) &&
             c->alloc(&c->bin_goff, cfg->grad_record_log2 > 0 ? N : 1);
    if (ok && cfg->enable_ntc) {
        const gs3_ntc_config& nc = cfg->ntc;
        if (nc.levels != 16 || nc.feats != 2 || nc.hidden != 64 || nc.log2_T < 10 || nc.log2_T > 22 ||
            nc.precision < GS3_F32 || nc.precision > GS3_BF16) {
            gs3_destroy(c);
            return GS3_EINVAL;
        }
        const int64_t T = (int64_t)1 << nc.log2_T;
        int64_t off = 0;
        c->nd.dense_mask = 0;
        for (int l = 0; l < 16; l++) {
            if (nc.res[l] < 1 || nc.res[l] > 65535) {
                gs3_destroy(c);
                return GS3_EINVAL;
            }
            const int64_t r1 = (int64_t)nc.res[l] + 1;
            const int64_t full = r1 * r1 * r1;
            c->nd.res[l] = nc.res[l];
            c->nd.off[l] = off;
            if (full <= T) c->nd.dense_mask |= 1u << l;
            off += full <= T ? full : T;
        }
        c->nd.T_mask = (uint32_t)(T - 1);
        for (int k = 0; k < 3; k++) {
            c->nd.aabb_min[k] = nc.aabb_min[k];
            c->nd.inv_ext[k] = nc.inv_extent[k];
        }
        c->n_table_floats = off * 2;
        c->n_params = c->n_table_floats + ntc_mlp_params();
        // up to two NTC-backward workgroups per CU (their LDS allows two in
        // half precision, one in float32); each loops over its share of the
        // point batches in a single round
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        c->max_parts = 2 * cus;
        ok = c->alloc(&c->p, c->n_params) && c->alloc(&c->g, c->n_params) && c->alloc(&c->m, c->n_params) &&
             c->alloc(&c->v, c->n_params) && c->alloc((float**)&c->work, c->n_params) &&
             c->alloc(&c->g_part, (int64_t)c->max_parts * ntc_mlp_params()) && c->alloc(&c->warm_bsum, (N + 255) / 256);
    }
    if (!ok) {
        gs3_destroy(c);
        return GS3_ENOMEM;
    }
    Launch L{nullptr, nullptr};
    fill_u32(L, (uint32_t*)c->flags, 0u, 4);
    if (c->n_params) {
        fill_f32(L, c->p, 0.f, c->n_params);
        fill_f32(L, c->g, 0.f, c->n_params);
        fill_f32(L, c->m, 0.f, c->n_params);
        fill_f32(L, c->v, 0.f, c->n_params);
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        gs3_destroy(c);
        return GS3_EHIP;
    }
    *out = c;
    return GS3_OK;
}

void gs3_destroy(gs3_ctx* ctx) {
    if (!ctx) return;
    // teardown has no caller to report to: errors here are dropped
    (void)hipStreamSynchronize(ctx->st);
    for (void* p : ctx->allocs) (void)hipFree(p);
    for (void* p : ctx->csr_allocs) (void)hipFree(p);
    delete ctx;
}

const char* gs3_last_error(const gs3_ctx* ctx) { return ctx ? ctx->err.c_str() : kNullCtx; }

gs3_status gs3_set_stream(gs3_ctx* ctx, void* hip_stream) {
    if (!ctx) return GS3_EINVAL;
    ctx->st = (hipStream_t)hip_stream;
    return GS3_OK;
}

/* ---- per-frame setup ------------------------------------------------------ */

gs3_status gs3_morton_order(gs3_ctx* c, const float* means, int64_t n, const float aabb_min[3],
                            const float inv_extent[3], uint32_t* perm) {
    if (!c) return GS3_EINVAL;
    if (n < 0 || n > c->cfg.max_gaussians || (n > 0 && (!means || !perm)) || !aabb_min || !inv_extent)
        return c->fail(GS3_EINVAL, "morton_order: bad arguments");
    if (n == 0) return GS3_OK;
    Launch L = c->L();
    morton_codes(L, means, n, aabb_min, inv_extent, c->dkeys[0], c->dvals[0]);
    const int r = radix_sort_u32(L, c->dkeys, c->dvals, n, 30, c->radix_hist, c->scan_tmp);
    if (hipMemcpyAsync(perm, c->dvals[r], (size_t)n * 4, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "morton_order: copy failed");
    return c->check_launch("morton_order");
}

gs3_status gs3_gather_rows(gs3_ctx* c, const float* src, const uint32_t* perm, int64_t n, int32_t row_floats,
                           float* dst) {
    if (!c) return GS3_EINVAL;
    if (n < 0 || row_floats < 1 || (n > 0 && (!src || !perm || !dst || src == dst)))
        return c->fail(GS3_EINVAL, "gather_rows: bad arguments");
    gather_rows(c->L(), src, perm, n, row_floats, dst);
    return c->check_launch("gather_rows");
}

/* ---- NTC ---------------------------------------------------------------- */

gs3_status gs3_ntc_num_params(const gs3_ctx* ctx, int64_t* n) {
    if (!ctx || !n) return GS3_EINVAL;
    *n = ctx->n_params;
    return ctx->n_params ? GS3_OK : GS3_ESTATE;
}

gs3_status gs3_ntc_load(gs3_ctx* c, const float* host_params, int64_t n) {
    if (!c || !host_params) return GS3_EINVAL;
    if (!c->n_params) return c->fail(GS3_ESTATE, "context created without an NTC");
    if (n != c->n_params) return c->fail(GS3_EINVAL, "ntc_load: wrong parameter count");
    if (hipMemcpyAsync(c->p, host_params, (size_t)n * 4, hipMemcpyHostToDevice, c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "ntc_load: copy failed");
    Launch L = c->L();
    fill_f32(L, c->g, 0.f, n);
    fill_f32(L, c->m, 0.f, n);
    fill_f32(L, c->v, 0.f, n);
    ntc_refresh_work(L, c->cfg.ntc.precision, c->p, c->work, n);
    c->step = 0;
    c->enc_valid = false;
    if (hipStreamSynchronize(c->st) != hipSuccess) return c->fail(GS3_EHIP, "ntc_load: sync failed");
    return c->check_launch("ntc_load");
}

gs3_status gs3_ntc_save(gs3_ctx* c, float* host_params, int64_t cap) {
    if (!c || !host_params) return GS3_EINVAL;
    if (!c->n_params) return c->fail(GS3_ESTATE, "context created without an NTC");
    if (cap < c->n_params) return c->fail(GS3_EINVAL, "ntc_save: buffer too small");
    if (hipMemcpyAsync(host_params, c->p, (size_t)c->n_params * 4, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "ntc_save: copy failed");
    return GS3_OK;
}

// Reset everything that follows the parameters: gradients, Adam moments,
// step counter, the working copy and the kept encoding.
static void ntc_reset_state(gs3_ctx* c, bool keep_moments) {
    Launch L = c->L();
    fill_f32(L, c->g, 0.f, c->n_params);
    if (!keep_moments) {
        fill_f32(L, c->m, 0.f, c->n_params);
        fill_f32(L, c->v, 0.f, c->n_params);
        c->step = 0;
    }
    ntc_refresh_work(L, c->cfg.ntc.precision, c->p, c->work, c->n_params);
    c->enc_valid = false;
}

gs3_status gs3_ntc_init(gs3_ctx* c, uint64_t seed) {
    if (!c) return GS3_EINVAL;
    if (!c->n_params) return c->fail(GS3_ESTATE, "context created without an NTC");
    ntc_init(c->L(), c->p, c->n_params, c->n_table_floats, seed);
    ntc_reset_state(c, false);
    if (hipStreamSynchronize(c->st) != hipSuccess) return c->fail(GS3_EHIP, "ntc_init: sync failed");
    return c->check_launch("ntc_init");
}

namespace {
// Fixed-layout header of a saved NTC state, followed by the float32
// parameters, first and second Adam moments (n_params each).
struct NtcStateHeader {
    char magic[8];
    int64_t n_params;
    int64_t step;
    int32_t levels, feats, log2_T, hidden, precision, reserved;
    int32_t res[16];
    float aabb_min[3], inv_extent[3];
};
const char kStateMagic[8] = {'G', 'S', '3', 'N', 'T', 'C', '1', '\0'};
}  // namespace

gs3_status gs3_ntc_state_bytes(const gs3_ctx* c, size_t* bytes) {
    if (!c || !bytes) return GS3_EINVAL;
    if (!c->n_params) return GS3_ESTATE;
    *bytes = sizeof(NtcStateHeader) + 3 * (size_t)c->n_params * 4;
    return GS3_OK;
}

gs3_status gs3_ntc_save_state(gs3_ctx* c, void* host, size_t cap, size_t* used) {
    if (!c || !host) return GS3_EINVAL;
    if (!c->n_params) return c->fail(GS3_ESTATE, "context created without an NTC");
    size_t need = 0;
    gs3_ntc_state_bytes(c, &need);
    if (used) *used = need;
    if (cap < need) return c->fail(GS3_EINVAL, "ntc_save_state: buffer too small");
    NtcStateHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, kStateMagic, 8);
    const gs3_ntc_config& nc = c->cfg.ntc;
    h.n_params = c->n_params; h.step = c->step;
    h.levels = nc.levels; h.feats = nc.feats; h.log2_T = nc.log2_T; h.hidden = nc.hidden; h.precision = nc.precision;
    for (int l = 0; l < 16; l++) h.res[l] = nc.res[l];
    for (int k = 0; k < 3; k++) { h.aabb_min[k] = nc.aabb_min[k]; h.inv_extent[k] = nc.inv_extent[k]; }
    memcpy(host, &h, sizeof(h));
    char* dst = (char*)host + sizeof(h);
    const size_t b = (size_t)c->n_params * 4;
    if (hipMemcpyAsync(dst, c->p, b, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipMemcpyAsync(dst + b, c->m, b, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipMemcpyAsync(dst + 2 * b, c->v, b, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "ntc_save_state: copy failed");
    return GS3_OK;
}

gs3_status gs3_ntc_load_state(gs3_ctx* c, const void* host, size_t n) {
    if (!c || !host) return GS3_EINVAL;
    if (!c->n_params) return c->fail(GS3_ESTATE, "context created without an NTC");
    size_t need = 0;
    gs3_ntc_state_bytes(c, &need);
    if (n != need) return c->fail(GS3_EINVAL, "ntc_load_state: size does not match this context's NTC");
    NtcStateHeader h;
    memcpy(&h, host, sizeof(h));
    const gs3_ntc_config& nc = c->cfg.ntc;
    bool same = memcmp(h.magic, kStateMagic, 8) == 0 && h.n_params == c->n_params && h.step >= 0 &&
                h.levels == nc.levels && h.feats == nc.feats && h.log2_T == nc.log2_T && h.hidden == nc.hidden;
    for (int l = 0; l < 16 && same; l++) same = h.res[l] == nc.res[l];
    for (int k = 0; k < 3 && same; k++) same = h.aabb_min[k] == nc.aabb_min[k] && h.inv_extent[k] == nc.inv_extent[k];
    if (!same) return c->fail(GS3_EINVAL, "ntc_load_state: the saved NTC has another shape or AABB");
    const char* src = (const char*)host + sizeof(h);
    const size_t b = (size_t)c->n_params * 4;
    if (hipMemcpyAsync(c->p, src, b, hipMemcpyHostToDevice, c->st) != hipSuccess ||
        hipMemcpyAsync(c->m, src + b, b, hipMemcpyHostToDevice, c->st) != hipSuccess ||
        hipMemcpyAsync(c->v, src + 2 * b, b, hipMemcpyHostToDevice, c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "ntc_load_state: copy failed");
    c->step = (int)h.step;
    ntc_reset_state(c, true);
    if (hipStreamSynchronize(c->st) != hipSuccess) return c->fail(GS3_EHIP, "ntc_load_state: sync failed");
    return c->check_launch("ntc_load_state");
}

static void ntc_ptrs(gs3_ctx* c, const void** table, const void** mlp) {
    if (c->cfg.ntc.precision == GS3_F32) {
        *table = c->p;
        *mlp = c->p + c->n_table_floats;
    } else {
        *table = c->work;
        *mlp = (const char*)c->work + 2 * c->n_table_floats;
    }
}

// A nonzero token must be the one the last gs3_ntc_prepare returned, for
// the same means and n.
static gs3_status check_token(gs3_ctx* c, const float* means, int64_t n, uint64_t token, const char* what) {
    if (token == 0) return GS3_OK;
    if (token != c->csr_token || c->csr_token == 0)
        return c->fail(GS3_ESTATE, std::string(what) + ": the token is not the last ntc_prepare's");
    if (means != c->csr_means || n != c->csr_n)
        return c->fail(GS3_EINVAL, std::string(what) + ": means or n differ from the prepared ones");
    return GS3_OK;
}

gs3_status gs3_ntc_forward(gs3_ctx* c, const float* means, int64_t n, uint64_t token, float* dmu, float* dq) {
    if (!c) return GS3_EINVAL;
    if (!c->n_params) return c->fail(GS3_ESTATE, "context created without an NTC");
    if (n < 0 || n > c->cfg.max_gaussians || (n > 0 && (!means || !dmu || !dq)))
        return c->fail(GS3_EINVAL, "ntc_forward: bad arguments");
    gs3_status s = check_token(c, means, n, token, "ntc_forward");
    if (s != GS3_OK) return s;
    const void *table, *mlp;
    ntc_ptrs(c, &table, &mlp);
    // on the prepared means the forward keeps the encoding for the backward
    const bool prepared = token != 0 && n > 0;
    ntc_forward(c->L(), c->cfg.ntc.precision, c->nd, table, mlp, means, n, dmu, dq,
                prepared ? c->enc_cache : nullptr);
    if (prepared) c->enc_valid = true;
    return c->check_launch("ntc_forward");
}

gs3_status gs3_ntc_backward(gs3_ctx* c, const float* means, int64_t n, uint64_t token, const float* d_dmu,
                            const float* d_dq) {
    if (!c) return GS3_EINVAL;
    if (!c->n_params) return c->fail(GS3_ESTATE, "context created without an NTC");
    if (n < 0 || n > c->cfg.max_gaussians || (n > 0 && (!means || !d_dmu || !d_dq)))
        return c->fail(GS3_EINVAL, "ntc_backward: bad arguments");
    gs3_status s = check_token(c, means, n, token, "ntc_backward");
    if (s != GS3_OK) return s;
    const void *table, *mlp;
    ntc_ptrs(c, &table, &mlp);
    const bool prepared = token != 0;
    ntc_backward(c->L(), c->cfg.ntc.precision, c->nd, table, mlp, means, n, d_dmu, d_dq, c->g,
                 c->g + c->n_table_floats, c->g_part, c->max_parts, prepared ? &c->csr : nullptr,
                 prepared && c->enc_valid ? c->enc_cache : nullptr);
    return c->check_launch("ntc_backward");
}

gs3_status gs3_ntc_prepare(gs3_ctx* c, const float* means, int64_t n, uint64_t* token) {
    if (!c) return GS3_EINVAL;
    if (token) *token = 0;
    if (!c->n_params) return c->fail(GS3_ESTATE, "context created without an NTC");
    if (n < 1 || n > c->cfg.max_gaussians || n >= ((int64_t)1 << 25) || !means)
        return c->fail(GS3_EINVAL, "ntc_prepare: bad arguments");
    c->csr_means = nullptr;
    c->csr_n = -1;
    c->csr_token = 0;
    c->enc_valid = false;
    const int64_t m = n * 128;
    if (n > c->csr_cap) {
        if (hipStreamSynchronize(c->st) != hipSuccess) return c->fail(GS3_EHIP, "ntc_prepare: sync failed");
        for (void* p : c->csr_allocs) (void)hipFree(p);
        c->csr_bytes = 0;
        c->csr_allocs.clear();
        auto get = [&](void** out, size_t bytes) {
            *out = nullptr;
            if (hipMalloc(out, bytes) != hipSuccess) return false;
            c->csr_allocs.push_back(*out);
            c->csr_bytes += (int64_t)bytes;
            return true;
        };
        const int64_t entries = c->n_table_floats / 2;
        bool ok = get((void**)&c->csr_keys[0], m * 4) && get((void**)&c->csr_keys[1], m * 4) &&
                  get((void**)&c->csr_vals[0], m * 4) && get((void**)&c->csr_vals[1], m * 4) &&
                  get((void**)&c->csr_hist, radix_hist_words(m) * 4) &&
                  get((void**)&c->csr_tmp, (scan_tmp_words(radix_hist_words(m)) + 4) * 8) &&
                  get((void**)&c->csr.rows, entries * 8) && get((void**)&c->csr.pw, m * 8) &&
                  get((void**)&c->csr.denc, n * 32 * 4) && get(&c->enc_cache, n * 32 * 4);
        if (!ok) {
            for (void* p : c->csr_allocs) (void)hipFree(p);
            c->csr_allocs.clear();
            c->csr_cap = 0;
            return c->fail(GS3_ENOMEM, "ntc_prepare: allocation failed");
        }
        c->csr_cap = n;
        c->csr.entries = entries;
    }
    ntc_csr_build(c->L(), c->nd, means, n, c->csr, c->csr_keys, c->csr_vals, c->csr_hist, c->csr_tmp);
    if (hipStreamSynchronize(c->st) != hipSuccess) return c->fail(GS3_EHIP, "ntc_prepare: sync failed");
    gs3_status s = c->check_launch("ntc_prepare");
    if (s != GS3_OK) return s;
    c->csr_means = means;
    c->csr_n = n;
    c->csr_token = ++c->last_token;
    if (token) *token = c->csr_token;
    return GS3_OK;
}

gs3_status gs3_ntc_step(gs3_ctx* c, float lr, float beta1, float beta2, float eps) {
    if (!c) return GS3_EINVAL;
    if (!c->n_params) return c->fail(GS3_ESTATE, "context created without an NTC");
    c->step += 1;
    c->enc_valid = false;
    const float bc1 = (float)(1.0 - pow((double)beta1, (double)c->step));
    const float bc2 = (float)(1.0 - pow((double)beta2, (double)c->step));
    ntc_adam(c->L(), c->cfg.ntc.precision, c->p, c->g, c->m, c->v, c->work, c->n_params, lr, beta1, beta2, eps, bc1,
             bc2);
    return c->check_launch("ntc_step");
}

gs3_status gs3_ntc_grads(gs3_ctx* c, float* dev_out, int64_t cap) {
    if (!c || !dev_out) return GS3_EINVAL;
    if (!c->n_params) return c->fail(GS3_ESTATE, "context created without an NTC");
    if (cap < c->n_params) return c->fail(GS3_EINVAL, "ntc_grads: buffer too small");
    if (hipMemcpyAsync(dev_out, c->g, (size_t)c->n_params * 4, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "ntc_grads: copy failed");
    return GS3_OK;
}

gs3_status gs3_ntc_zero_grads(gs3_ctx* c) {
    if (!c) return GS3_EINVAL;
    if (!c->n_params) return c->fail(GS3_ESTATE, "context created without an NTC");
    fill_f32(c->L(), c->g, 0.f, c->n_params);
    return c->check_launch("ntc_zero_grads");
}

gs3_status gs3_warmup_loss(gs3_ctx* c, const float* dmu, const float* dq, int64_t n, float* loss_dev, float* d_dmu,
                           float* d_dq) {
    if (!c) return GS3_EINVAL;
    if (!c->n_params) return c->fail(GS3_ESTATE, "context created without an NTC");
    if (n < 1 || n > c->cfg.max_gaussians || !dmu || !dq || !loss_dev || !d_dmu || !d_dq)
        return c->fail(GS3_EINVAL, "warmup_loss: bad arguments");
    warmup_loss(c->L(), dmu, dq, n, loss_dev, d_dmu, d_dq, c->warm_bsum);
    return c->check_launch("warmup_loss");
}

/* ---- render ------------------------------------------------------------- */

static gs3_status make_cam(gs3_ctx* c, const gs3_camera* cam, CamDev* out) {
    if (!cam) return c->fail(GS3_EINVAL, "null camera");
    if (cam->width < 1 || cam->height < 1 || cam->width > c->cfg.max_width || cam->height > c->cfg.max_height)
        return c->fail(GS3_EINVAL, "camera size outside the context's maximum");
    if (!(cam->fx > 0.f) || !(cam->fy > 0.f) || !(cam->near_z > 0.f)) return c->fail(GS3_EINVAL, "bad intrinsics");
    CamDev d;
    d.W = cam->width;
    d.H = cam->height;
    d.tiles_x = (cam->width + kTile - 1) / kTile;
    d.tiles_y = (cam->height + kTile - 1) / kTile;
    d.fx = cam->fx; d.fy = cam->fy; d.cx = cam->cx; d.cy = cam->cy; d.near_z = cam->near_z;
    for (int r = 0; r < 3; r++) {
        for (int k = 0; k < 3; k++) d.R[3 * r + k] = cam->world_to_cam[4 * r + k];
        d.t[r] = cam->world_to_cam[4 * r + 3];
        d.cpos[r] = cam->cam_pos[r];
        d.bg[r] = cam->bg[r];
    }
    *out = d;
    return GS3_OK;
}

gs3_status gs3_render(gs3_ctx* c, int32_t slot, const gs3_gaussians* g, const float* dmu, const float* dq,
                      const gs3_camera* cam, float* image) {
    if (!c) return GS3_EINVAL;
    if (slot < 0 || slot >= (int)c->slots.size()) return c->fail(GS3_EINVAL, "bad slot");
    if (!g || !image) return c->fail(GS3_EINVAL, "null argument");
    if (g->n < 0 || g->n > c->cfg.max_gaussians) return c->fail(GS3_EINVAL, "Gaussian count outside [0, max]");
    if (g->sh_degree < 0 || g->sh_degree > 3) return c->fail(GS3_EINVAL, "sh_degree must be 0..3");
    if (g->n > 0 && (!g->means || !g->quats || !g->log_scales || !g->opacity_logits || !g->sh))
        return c->fail(GS3_EINVAL, "null Gaussian array");
    CamDev cd;
    gs3_status s = make_cam(c, cam, &cd);
    if (s != GS3_OK) return s;
    Slot& sl = c->slots[slot];
    sl.valid = false;
    GaussDev gd;
    gd.means = g->means; gd.quats = g->quats; gd.log_scales = g->log_scales; gd.opac = g->opacity_logits;
    gd.sh = g->sh; gd.dmu = dmu; gd.dq = dq; gd.n = g->n; gd.sh_degree = g->sh_degree;
    const int ntiles = cd.tiles_x * cd.tiles_y;
    const uint64_t cap = (uint64_t)c->cfg.max_pairs;
    Launch L = c->L();
    const int64_t n = g->n;
    preprocess(L, gd, cd, sl.rec, sl.key, sl.rect, sl.count);
    if (c->cfg.sort_mode == GS3_SORT_DEPTH_FIRST) {
        sl.cur = 0;
        if (n > 0) {
            const int r = radix_order_u32(L, sl.key, c->dkeys, c->dvals, n, 32, c->radix_hist, c->scan_tmp);
            const uint32_t* order = c->dvals[r];
            const int64_t nchunks = bin_chunks(n);
            const bool rec_mode = c->grec_cap > 0;
            // first pair slot of each Gaussian: only the record mode's
            // gradient gather needs it
            if (rec_mode) scan_u32_to_u64(L, sl.count, n, sl.goff, c->goff_total, c->scan_tmp);
            bin_gather(L, order, n, sl.rect, sl.count, sl.goff, cap, c->bin_rect, rec_mode ? c->bin_goff : nullptr,
                       rec_mode ? nullptr : sl.ttot, rec_mode ? 0 : (int64_t)ntiles);
            if (rec_mode) {
                // tile-major list (the record gather needs every pair's slot)
                bin_count(L, order, n, c->bin_rect, cd.tiles_x, cd.tiles_y, c->bin_hist, nullptr);
                bin_scan(L, c->bin_hist, nchunks, ntiles, (uint32_t)cap, c->bin_base, sl.total, c->bin_part,
                         c->bin_ttot, c->bin_toff, c->scan_tmp);
                // gpos (and the first slots bin_gather stored) exist only in
                // record mode; without it the buffers hold one element
                bin_scatter(L, order, n, c->bin_rect, rec_mode ? c->bin_goff : nullptr, cd.tiles_x, cd.tiles_y,
                            c->bin_base, cap, sl.vals[0], rec_mode ? sl.gpos : nullptr);
                ranges_from_hist(L, c->bin_base, sl.total, ntiles, cap, sl.ranges, c->flags);
            } else {
                // chunk-major list: every wave writes one run of consecutive
                // slots; the forward walks each tile's segments
                bin_count(L, order, n, c->bin_rect, cd.tiles_x, cd.tiles_y, sl.chist, sl.ttot);
                scan_u32_to_u64(L, sl.chist, (int64_t)ntiles * nchunks, sl.cmb, sl.total, c->scan_tmp);
                tile_ranges_from_counts(L, sl.ttot, ntiles, cap, sl.total, sl.ranges, c->flags);
                bin_scatter_chunked(L, order, n, c->bin_rect, cd.tiles_x, cd.tiles_y, sl.cmb, cap, sl.vals[0]);
            }
            sl.chunked = !rec_mode;
            sl.nchunks = nchunks;
        } else {
            fill_u32(L, (uint32_t*)sl.ranges, 0u, 2 * (int64_t)ntiles);
            fill_u32(L, (uint32_t*)sl.total, 0u, 2);
            sl.chunked = false;
            sl.nchunks = 0;
        }
        sl.K_host = -1;
    } else {
        scan_u32_to_u64(L, sl.count, n, sl.goff, sl.total, c->scan_tmp);
        emit_pairs(L, n, sl.key, sl.rect, sl.goff, cd.tiles_x, cap, sl.pkeys[0], sl.vals[0]);
        uint64_t K = 0;
        if (hipMemcpyAsync(&K, sl.total, 8, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
            hipStreamSynchronize(c->st) != hipSuccess)
            return c->fail(GS3_EHIP, "render: reading the pair count failed");
        sl.K_host = (int64_t)K;
        if (K > cap) {
            fill_u32(L, (uint32_t*)c->flags, 1u, 1);
            return c->fail(GS3_ECAPACITY, "render: more pairs than max_pairs");
        }
        int tb = 0;
        while ((1 << tb) < ntiles) tb++;
        sl.cur = radix_sort_u64(L, sl.pkeys, sl.vals, (int64_t)K, 32 + tb, c->radix_hist, c->scan_tmp);
        ranges_from_keys(L, sl.pkeys[sl.cur], (int64_t)K, ntiles, sl.ranges);
        if (c->grec_cap > 0)
            gpos_from_pairs(L, sl.pkeys[sl.cur], sl.vals[sl.cur], (int64_t)K, sl.rect, sl.goff, cd.tiles_x, cap,
                            sl.gpos);
    }
    tile_order(L, sl.ranges, nullptr, ntiles, sl.order_fwd);
    sl.tile_major_full = false;
    if (sl.chunked) {
        const ChunkDev cl{sl.chist, sl.cmb, sl.nchunks, (uint32_t)cap, sl.walked};
        blend_forward(L, cd, sl.ranges, sl.vals[0], sl.rec, image, sl.T_final, sl.last, sl.tile_walk, sl.order_fwd, &cl);
    } else {
        blend_forward(L, cd, sl.ranges, sl.vals[sl.cur], sl.rec, image, sl.T_final, sl.last, sl.tile_walk, sl.order_fwd,
                      nullptr);
    }
    gs3_status st = c->check_launch("render");
    if (st != GS3_OK) return st;
    sl.g = gd;
    sl.cam = cd;
    sl.valid = true;
    return GS3_OK;
}

gs3_status gs3_render_backward(gs3_ctx* c, int32_t slot, const float* d_image, const gs3_grads* out) {
    if (!c) return GS3_EINVAL;
    if (slot < 0 || slot >= (int)c->slots.size()) return c->fail(GS3_EINVAL, "bad slot");
    if (!d_image || !out) return c->fail(GS3_EINVAL, "null argument");
    Slot& sl = c->slots[slot];
    if (!sl.valid) return c->fail(GS3_ESTATE, "render_backward before a successful render on this slot");
    Launch L = c->L();
    const int64_t n = sl.g.n;
    const int ntiles = sl.cam.tiles_x * sl.cam.tiles_y;
    fill_f32(L, c->accum, 0.f, 9 * n);
    if (c->grec_cap > 0) scan_u32_to_u32(L, sl.tile_walk, ntiles, c->walk_off, c->walk_total, c->scan_tmp);
    GatherDev ga;
    ga.rect = sl.rect; ga.goff = sl.goff; ga.gpos = sl.gpos; ga.ranges = sl.ranges; ga.tile_walk = sl.tile_walk;
    ga.walk_off = c->walk_off; ga.grec = c->grec; ga.grec_cap = (uint64_t)c->grec_cap;
    ga.cap = (uint64_t)c->cfg.max_pairs;
    tile_order(L, sl.ranges, sl.tile_walk, ntiles, sl.order_bwd);
    blend_backward(L, sl.cam, sl.ranges, sl.chunked ? sl.walked : sl.vals[sl.cur], sl.rec, d_image, sl.T_final,
                   sl.last, ga, c->accum, out->d_opacity != nullptr || out->d_opacity_logits != nullptr, sl.order_bwd);
    GradsDev gd;
    gd.d_means = out->d_means; gd.d_quats = out->d_quats; gd.d_log_scales = out->d_log_scales;
    gd.d_opac = out->d_opacity_logits; gd.d_sh = out->d_sh; gd.d_dmu = sl.g.dmu ? out->d_dmu : nullptr;
    gd.d_dq = sl.g.dq ? out->d_dq : nullptr; gd.d_uv = out->d_uv; gd.d_conic = out->d_conic;
    gd.d_opacity = out->d_opacity; gd.d_rgb = out->d_rgb;
    if ((out->vspace_grad == nullptr) != (out->vspace_count == nullptr))
        return c->fail(GS3_EINVAL, "render_backward: vspace_grad and vspace_count go together");
    gd.vgrad = out->vspace_grad; gd.vcount = out->vspace_count;
    preprocess_backward(L, sl.g, sl.cam, c->accum, ga, gd);
    return c->check_launch("render_backward");
}

gs3_status gs3_transform_bake(gs3_ctx* c, const gs3_gaussians* g, const float* dmu, const float* dq,
                              float* means_out, float* quats_out, float* sh_out) {
    if (!c) return GS3_EINVAL;
    if (!g || g->n < 0 || g->sh_degree < 0 || g->sh_degree > 3)
        return c->fail(GS3_EINVAL, "transform_bake: bad Gaussians");
    if (g->n > 0 && (!g->means || !g->quats || !g->sh || !means_out || !quats_out || !sh_out))
        return c->fail(GS3_EINVAL, "transform_bake: null array");
    if (g->n > 0 && (means_out == g->means || quats_out == g->quats || sh_out == g->sh))
        return c->fail(GS3_EINVAL, "transform_bake: outputs alias inputs");
    GaussDev gd{};
    gd.means = g->means; gd.quats = g->quats; gd.log_scales = g->log_scales; gd.opac = g->opacity_logits;
    gd.sh = g->sh; gd.dmu = dmu; gd.dq = dq; gd.n = g->n; gd.sh_degree = g->sh_degree;
    static const ShRotConst rc = make_shrot_const();
    transform_bake(c->L(), gd, rc, means_out, quats_out, sh_out);
    return c->check_launch("transform_bake");
}

gs3_status gs3_select(gs3_ctx* c, const float* num, const float* den, int64_t n, float threshold, uint32_t* idx,
                      int64_t* count) {
    if (!c) return GS3_EINVAL;
    if (!count || n < 0) return c->fail(GS3_EINVAL, "select: bad arguments");
    if (n > c->cfg.max_gaussians) return c->fail(GS3_ECAPACITY, "select: n exceeds max_gaussians");
    if (n > 0 && (!num || !idx)) return c->fail(GS3_EINVAL, "select: null array");
    *count = 0;
    if (n == 0) return GS3_OK;
    select_indices(c->L(), num, den, n, threshold, c->sel_flag, c->sel_pos, c->sel_total, c->scan_tmp, idx);
    uint64_t total = 0;
    if (hipMemcpyAsync(&total, c->sel_total, sizeof(total), hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "select: copy of the count failed");
    *count = (int64_t)total;
    return c->check_launch("select");
}

gs3_status gs3_spawn(gs3_ctx* c, const gs3_gaussians* src, const uint32_t* idx, int64_t m, const float* z,
                     int32_t mode, float* means, float* quats, float* log_scales, float* opacity_logits, float* sh) {
    if (!c) return GS3_EINVAL;
    if (!src || src->n < 0 || src->sh_degree < 0 || src->sh_degree > 3 || m < 0)
        return c->fail(GS3_EINVAL, "spawn: bad arguments");
    if (mode != GS3_SPAWN && mode != GS3_SPLIT) return c->fail(GS3_EINVAL, "spawn: unknown mode");
    if (m == 0) return GS3_OK;
    if (!idx || !z || !means || !quats || !log_scales || !opacity_logits || !sh || !src->means || !src->quats ||
        !src->log_scales || !src->opacity_logits || !src->sh)
        return c->fail(GS3_EINVAL, "spawn: null array");
    if (means == src->means || quats == src->quats || log_scales == src->log_scales ||
        opacity_logits == src->opacity_logits || sh == src->sh)
        return c->fail(GS3_EINVAL, "spawn: outputs alias the sources");
    GaussDev gd{};
    gd.means = src->means; gd.quats = src->quats; gd.log_scales = src->log_scales; gd.opac = src->opacity_logits;
    gd.sh = src->sh; gd.n = src->n; gd.sh_degree = src->sh_degree;
    const float logit0 = (float)log(0.1 / 0.9), shrink = (float)log(0.8);
    spawn(c->L(), gd, idx, m, z, mode, logit0, shrink, means, quats, log_scales, opacity_logits, sh);
    return c->check_launch("spawn");
}

/* ---- loss / optimiser ----------------------------------------------------- */

gs3_status gs3_loss(gs3_ctx* c, const float* image, const float* target, int32_t height, int32_t width,
                    float lambda_dssim, float* loss_dev, float* d_image) {
    if (!c) return GS3_EINVAL;
    if (!image || !target || !loss_dev || !d_image) return c->fail(GS3_EINVAL, "loss: null argument");
    if (height < 1 || width < 1 || height > c->cfg.max_height || width > c->cfg.max_width)
        return c->fail(GS3_EINVAL, "loss: image size outside the context's maximum");
    if (!(lambda_dssim >= 0.f && lambda_dssim <= 1.f)) return c->fail(GS3_EINVAL, "loss: lambda outside [0, 1]");
    LossWork w{c->loss_maps, c->loss_bsum, loss_blocks(height, width)};
    loss_forward_backward(c->L(), image, target, height, width, lambda_dssim, w, loss_dev, d_image, c->flags + 1);
    return c->check_launch("loss");
}

gs3_status gs3_adam(gs3_ctx* c, float* param, const float* grad, float* m, float* v, int64_t n, int32_t step,
                    float lr, float beta1, float beta2, float eps) {
    if (!c) return GS3_EINVAL;
    if (n < 0 || step < 1 || (n > 0 && (!param || !grad || !m || !v))) return c->fail(GS3_EINVAL, "adam: bad arguments");
    adam(c->L(), param, grad, m, v, n, step, lr, beta1, beta2, eps);
    return c->check_launch("adam");
}

gs3_status gs3_zero(gs3_ctx* c, float* dev, int64_t n) {
    if (!c) return GS3_EINVAL;
    if (n < 0 || (n > 0 && !dev)) return c->fail(GS3_EINVAL, "zero: bad arguments");
    fill_f32(c->L(), dev, 0.f, n);
    return c->check_launch("zero");
}

/* ---- inspection ----------------------------------------------------------- */

gs3_status gs3_debug_counts(gs3_ctx* c, int32_t slot, int64_t* num_pairs, int64_t* sum_contrib,
                            int64_t* walked, int32_t* overflow) {
    if (!c) return GS3_EINVAL;
    if (slot < 0 || slot >= (int)c->slots.size()) return c->fail(GS3_EINVAL, "bad slot");
    Slot& sl = c->slots[slot];
    uint64_t K = 0, sums[2] = {0, 0};
    const bool need_sums = sl.valid && (sum_contrib || walked);
    if (need_sums) {
        Launch L = c->L();
        sum_u32(L, sl.last, (int64_t)sl.cam.W * sl.cam.H, c->sums);
        sum_u32(L, sl.tile_walk, (int64_t)sl.cam.tiles_x * sl.cam.tiles_y, c->sums + 1);
    }
    if (hipMemcpyAsync(&K, sl.total, 8, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        (need_sums && hipMemcpyAsync(sums, c->sums, 16, hipMemcpyDeviceToHost, c->st) != hipSuccess) ||
        hipStreamSynchronize(c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "debug_counts: copy failed");
    if (num_pairs) *num_pairs = (int64_t)K;
    if (sum_contrib) *sum_contrib = sl.valid ? (int64_t)sums[0] : -1;
    if (walked) *walked = sl.valid ? (int64_t)sums[1] : -1;
    const int ov = K > (uint64_t)c->cfg.max_pairs;
    if (overflow) *overflow = ov;
    return ov ? c->fail(GS3_ECAPACITY, "pair list overflowed") : GS3_OK;
}

gs3_status gs3_debug_pairs(gs3_ctx* c, int32_t slot, uint64_t* keys, uint32_t* vals, int64_t cap) {
    if (!c) return GS3_EINVAL;
    if (slot < 0 || slot >= (int)c->slots.size()) return c->fail(GS3_EINVAL, "bad slot");
    Slot& sl = c->slots[slot];
    if (!sl.valid) return c->fail(GS3_ESTATE, "no render on this slot");
    int64_t K = 0;
    int32_t ov = 0;
    gs3_status s = gs3_debug_counts(c, slot, &K, nullptr, nullptr, &ov);
    if (s != GS3_OK) return s;
    if (cap < K) return c->fail(GS3_EINVAL, "debug_pairs: buffer too small");
    if (K == 0) return GS3_OK;
    const int ntiles = sl.cam.tiles_x * sl.cam.tiles_y;
    const uint32_t* tm = sl.vals[sl.cur];
    if (sl.chunked) {
        // the whole tile-major list from the chunk-major one (its prefix
        // walked by the forward is unchanged by this)
        if (!sl.tile_major_full) {
            Launch L = c->L();
            bin_scan(L, sl.chist, sl.nchunks, ntiles, (uint32_t)c->cfg.max_pairs, c->bin_base, c->walk_total,
                     c->bin_part, c->bin_ttot, c->bin_toff, c->scan_tmp);
            chunked_to_tile_major(L, sl.chist, sl.cmb, c->bin_base, sl.nchunks, ntiles, (uint64_t)c->cfg.max_pairs,
                                  sl.vals[0], sl.walked);
            sl.tile_major_full = true;
        }
        tm = sl.walked;
    }
    if (vals && hipMemcpyAsync(vals, tm, (size_t)K * 4, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "debug_pairs: copy failed");
    if (keys) {
        if (c->cfg.sort_mode == GS3_SORT_RADIX64) {
            if (hipMemcpyAsync(keys, sl.pkeys[sl.cur], (size_t)K * 8, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
                return c->fail(GS3_EHIP, "debug_pairs: copy failed");
        } else {
            debug_keys(c->L(), sl.ranges, tm, sl.key, ntiles, keys);
        }
    }
    return c->check_launch("debug_pairs");
}

gs3_status gs3_debug_ranges(gs3_ctx* c, int32_t slot, uint32_t* ranges) {
    if (!c || !ranges) return GS3_EINVAL;
    if (slot < 0 || slot >= (int)c->slots.size()) return c->fail(GS3_EINVAL, "bad slot");
    Slot& sl = c->slots[slot];
    if (!sl.valid) return c->fail(GS3_ESTATE, "no render on this slot");
    const int ntiles = sl.cam.tiles_x * sl.cam.tiles_y;
    if (hipMemcpyAsync(ranges, sl.ranges, (size_t)ntiles * 8, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "debug_ranges: copy failed");
    return GS3_OK;
}

gs3_status gs3_debug_gaussians(gs3_ctx* c, int32_t slot, uint32_t* key, int32_t* box, float* rec) {
    if (!c) return GS3_EINVAL;
    if (slot < 0 || slot >= (int)c->slots.size()) return c->fail(GS3_EINVAL, "bad slot");
    Slot& sl = c->slots[slot];
    if (!sl.valid) return c->fail(GS3_ESTATE, "no render on this slot");
    const int64_t n = sl.g.n;
    if (key && n && hipMemcpyAsync(key, sl.key, (size_t)n * 4, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "debug_gaussians: copy failed");
    if (box || rec) debug_records(c->L(), n, sl.rec, box, rec);
    return c->check_launch("debug_gaussians");
}

gs3_status gs3_debug_pixels(gs3_ctx* c, int32_t slot, float* T_final, int32_t* last) {
    if (!c) return GS3_EINVAL;
    if (slot < 0 || slot >= (int)c->slots.size()) return c->fail(GS3_EINVAL, "bad slot");
    Slot& sl = c->slots[slot];
    if (!sl.valid) return c->fail(GS3_ESTATE, "no render on this slot");
    const size_t P = (size_t)sl.cam.W * sl.cam.H;
    if (T_final && hipMemcpyAsync(T_final, sl.T_final, P * 4, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "debug_pixels: copy failed");
    if (last && hipMemcpyAsync(last, sl.last, P * 4, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "debug_pixels: copy failed");
    return GS3_OK;
}

gs3_status gs3_workspace_bytes(const gs3_ctx* c, int64_t* bytes) {
    if (!c || !bytes) return GS3_EINVAL;
    *bytes = c->bytes + c->csr_bytes;
    return GS3_OK;
}

gs3_status gs3_check_flags(gs3_ctx* c) {
    if (!c) return GS3_EINVAL;
    int flags[4] = {0, 0, 0, 0};
    if (hipMemcpyAsync(flags, c->flags, 16, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess)
        return c->fail(GS3_EHIP, "check_flags: copy failed");
    fill_u32(c->L(), (uint32_t*)c->flags, 0u, 4);
    if (flags[0]) return c->fail(GS3_ECAPACITY, "a pair list overflowed");
    if (flags[1]) return c->fail(GS3_ENONFINITE, "a loss was not finite");
    return GS3_OK;
}

/* ---- profiling ------------------------------------------------------------- */

gs3_status gs3_profile_enable(gs3_ctx* c, int32_t on) {
    if (!c) return GS3_EINVAL;
    c->prof_on = on != 0;
    return GS3_OK;
}

gs3_status gs3_profile_only(gs3_ctx* c, const char* kernel) {
    if (!c) return GS3_EINVAL;
    c->prof.only = kernel ? kernel : "";
    return GS3_OK;
}

gs3_status gs3_profile_reset(gs3_ctx* c) {
    if (!c) return GS3_EINVAL;
    c->prof.collect();
    c->prof.totals.clear();
    return GS3_OK;
}

gs3_status gs3_profile_query(gs3_ctx* c, const char* kernel, double* total_ms, int64_t* launches) {
    if (!c || !kernel) return GS3_EINVAL;
    c->prof.collect();
    auto it = c->prof.totals.find(kernel);
    if (total_ms) *total_ms = it == c->prof.totals.end() ? 0.0 : it->second.first;
    if (launches) *launches = it == c->prof.totals.end() ? 0 : it->second.second;
    return GS3_OK;
}

}  // extern "C"
