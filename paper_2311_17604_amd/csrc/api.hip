// C ABI of libpdd: argument checks, context, scratch pool and entry points.
#include <new>
#include <string>
#include <vector>

#include "predictor.h"

namespace pdd {

int decimate(Ctx* c, const Grid& grid, int k, int K, float frac, int check, const int64_t* h_off,
             const int64_t* h_keep, int nseg, int32_t* kept, int32_t* order, uint64_t* order_cost);

int hip_fail(Ctx* c, hipError_t e, const char* what) {
    if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return PDD_ENOMEM;
    return PDD_EHIP;
}

void* scratch(Ctx* c, int slot, size_t bytes) {
    if (slot < 0 || slot >= kScratchSlots) return nullptr;
    Ctx::Buf& b = c->bufs[slot];
    if (b.bytes >= bytes && b.p) return b.p;
    if (b.p) {
        // work already queued may still use the old buffer
        if (hipStreamSynchronize(c->stream) != hipSuccess) return nullptr;
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes < 256 ? 256 : bytes;
    want = (want + 255) & ~(size_t)255;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        c->err = "hipMalloc of scratch failed (" + std::to_string(want) + " bytes)";
        return nullptr;
    }
    b.bytes = want;
    return b.p;
}

// Buffer width of the neighbour lists: k + b rounded up to a compiled size.
static int list_width(int kb) {
    if (kb <= 8) return 8;
    if (kb <= 16) return 16;
    if (kb <= 24) return 24;
    return 32;
}

}  // namespace pdd

struct pdd_ctx {
    pdd::Ctx c;
};

struct pdd_grid {
    pdd::Grid g;
};

using pdd::Ctx;

extern "C" {

const char* pdd_strerror(int status) {
    switch (status) {
        case PDD_OK: return "ok";
        case PDD_EINVAL: return "invalid argument";
        case PDD_ERANGE: return "coordinate extent too large (>= 2^21 mm on an axis)";
        case PDD_ENOMEM: return "out of device memory";
        case PDD_EHIP: return "HIP runtime error";
        case PDD_EINTERNAL: return "internal error";
        default: return "unknown status";
    }
}

const char* pdd_last_error(const pdd_ctx* ctx) { return ctx ? ctx->c.err.c_str() : ""; }

int pdd_ctx_create(pdd_ctx** out, int hip_device, void* hip_stream) {
    if (!out) return PDD_EINVAL;
    *out = nullptr;
    pdd_ctx* x = new (std::nothrow) pdd_ctx();
    if (!x) return PDD_ENOMEM;
    Ctx* c = &x->c;
    c->device = hip_device;
    c->stream = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(hip_device);
    if (e == hipSuccess) e = hipHostMalloc(&c->pinned, 4096, hipHostMallocDefault);
    // a stream to capture the round graph on (capture needs a stream other
    // than the default one; nothing ever runs on it)
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (c->pinned) (void)hipHostFree(c->pinned);
        delete x;
        return PDD_EHIP;
    }
    *out = x;
    return PDD_OK;
}

void pdd_ctx_destroy(pdd_ctx* ctx) {
    if (!ctx) return;
    Ctx* c = &ctx->c;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto& b : c->bufs)
        if (b.p) (void)hipFree(b.p);
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->pred_P) (void)hipFree(c->pred_P);
    if (c->pred_M) (void)hipFree(c->pred_M);
    if (c->pred_V) (void)hipFree(c->pred_V);
    delete ctx;
}

int pdd_build_grid(pdd_ctx* ctx, const int32_t* d_xyz, int64_t n, int32_t stride, int32_t voxel_log2,
                   pdd_grid** out) {
    if (!ctx || !d_xyz || !out || n < 2 || (stride != 12 && stride != 16)) return PDD_EINVAL;
    *out = nullptr;
    Ctx* c = &ctx->c;
    if (hipSetDevice(c->device) != hipSuccess) return PDD_EHIP;
    pdd_grid* g = new (std::nothrow) pdd_grid();
    if (!g) return PDD_ENOMEM;
    int rc = pdd::build_grid(c, d_xyz, n, stride, voxel_log2, &g->g);
    if (rc) {
        (void)hipStreamSynchronize(c->stream);
        pdd::free_grid(&g->g);
        delete g;
        return rc;
    }
    *out = g;
    return PDD_OK;
}

void pdd_grid_free(pdd_ctx* ctx, pdd_grid* grid) {
    if (!grid) return;
    if (ctx) {
        (void)hipSetDevice(ctx->c.device);
        (void)hipStreamSynchronize(ctx->c.stream);
    }
    pdd::free_grid(&grid->g);
    delete grid;
}

int pdd_grid_info(const pdd_grid* grid, int64_t* ncells, int32_t* voxel_log2) {
    if (!grid) return PDD_EINVAL;
    if (ncells) *ncells = grid->g.v.lv[0].ncells;
    if (voxel_log2) *voxel_log2 = grid->g.v.lv[0].s;
    return PDD_OK;
}

int pdd_knn_cost(pdd_ctx* ctx, const pdd_grid* grid, int32_t k, int32_t b, int32_t* d_nbr, int64_t* d_r2k,
                 uint64_t* d_cost) {
    if (!ctx || !grid || !d_cost || k < 1 || b < 0 || k + b > pdd::kMaxK) return PDD_EINVAL;
    Ctx* c = &ctx->c;
    if (hipSetDevice(c->device) != hipSuccess) return PDD_EHIP;
    const pdd::GridView& g = grid->g.v;
    const int K = pdd::list_width(k + b);
    pdd::KnnOut ko;
    ko.nbr = (int32_t*)pdd::scratch(c, 56, (size_t)g.n * K * 4);
    ko.cnt = (uint8_t*)pdd::scratch(c, 57, (size_t)g.n);
    ko.cost = (uint64_t*)pdd::scratch(c, 58, (size_t)g.n * 8);
    ko.r2k = (int64_t*)pdd::scratch(c, 59, (size_t)g.n * 8);
    if (!ko.nbr || !ko.cnt || !ko.cost || !ko.r2k) return PDD_ENOMEM;
    int rc = pdd::knn_all(c, g, k, K, ko, nullptr);
    if (rc) return rc;
    return pdd::knn_to_original(c, g, K, k + b, ko, d_nbr, d_r2k, d_cost);
}

// largest group of clouds one batched decimation takes at once (points)
constexpr int64_t kBatchGroup = (int64_t)1 << 28;

}  // extern "C"

namespace pdd {
int quality(Ctx* c, const int32_t* d_xyz, int64_t m, int stride, const int64_t* h_r2, int R, uint32_t* d_counts,
            int64_t* d_nn2, pdd_quality* out);
int autotune_batch(Ctx* c, const int32_t* d_xyz, const int64_t* h_off, int nscan, const int64_t* h_keep,
                   const pdd_opts* base, int64_t sample, pdd_opts* out, float* best_ms);
int decimate_entry(Ctx* c, const int32_t* d_xyz, int64_t n, const int64_t* h_off, const int64_t* h_keep, int nseg,
                   const pdd_opts* opts, int32_t* d_kept, int32_t* d_order, uint64_t* d_order_cost);
int autotune(Ctx* c, const int32_t* d_xyz, int64_t n, int64_t keep, const pdd_opts* base, int64_t sample,
             pdd_opts* out, float* best_ms);
}  // namespace pdd

static int decimate_common(pdd_ctx* ctx, const int32_t* d_xyz, int64_t n, const int64_t* h_off, const int64_t* h_keep,
                           int nseg, const pdd_opts* opts, int32_t* d_kept, int32_t* d_order, uint64_t* d_order_cost) {
    return pdd::decimate_entry(&ctx->c, d_xyz, n, h_off, h_keep, nseg, opts, d_kept, d_order, d_order_cost);
}

int pdd::decimate_entry(Ctx* c, const int32_t* d_xyz, int64_t n, const int64_t* h_off, const int64_t* h_keep, int nseg,
                        const pdd_opts* opts, int32_t* d_kept, int32_t* d_order, uint64_t* d_order_cost) {
    const int k = opts->k;
    if (k < 1 || k > pdd::kMaxK) return PDD_EINVAL;
    int b = opts->b;
    if (b < 0) return PDD_EINVAL;
    if (b == 0) b = (pdd::kMaxK - k) < 8 ? (pdd::kMaxK - k) : 8;
    if (k + b > pdd::kMaxK) return PDD_EINVAL;
    float frac = opts->round_frac == 0.0f ? 0.01f : opts->round_frac;
    if (!(frac > 0.0f && frac <= 1.0f)) return PDD_EINVAL;
    const int stride = opts->point_stride == 0 ? 12 : opts->point_stride;
    if (stride != 12 && stride != 16) return PDD_EINVAL;
    if (opts->voxel_log2 != 0 && (opts->voxel_log2 < 2 || opts->voxel_log2 > 20)) return PDD_EINVAL;
    if (opts->round_blocks != 0 && (opts->round_blocks < 64 || opts->round_blocks > 65535)) return PDD_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return PDD_EHIP;
    c->round_blocks = opts->round_blocks == 0 ? 1024u : (unsigned)opts->round_blocks;
    for (auto& s : c->stats) s = 0;
    for (auto& t : c->phase_ms) t = 0.0f;
    c->timing = (opts->flags & PDD_F_TIMING) != 0;
    c->progress = (opts->flags & PDD_F_PROGRESS) != 0;
    c->eager = (opts->flags & PDD_F_EAGER) != 0;
    if (c->timing && !c->ev[0])
        for (auto& e : c->ev)
            if (hipEventCreate(&e) != hipSuccess) return PDD_EHIP;
    pdd::mark(c, pdd::kPhStart);
    pdd::Grid grid;
    int rc = pdd::build_grid_seg(c, d_xyz, n, stride, opts->voxel_log2, h_off, nseg, &grid);
    if (rc == PDD_OK) {
        const int K = pdd::list_width(k + b);
        c->stats[5] = grid.v.lv[0].s;
        c->stats[6] = K;
        rc = pdd::decimate(c, grid, k, K, frac, (opts->flags & PDD_F_CHECK) ? 1 : 0, h_off, h_keep, nseg, d_kept,
                           d_order, d_order_cost);
    }
    (void)hipStreamSynchronize(c->stream);
    size_t held = 0;
    for (const auto& buf : c->bufs) held += buf.bytes;
    c->stats[4] = (int64_t)held;
    if (rc == PDD_OK && c->timing)
        for (int i = 1; i < pdd::kPhCount; i++) (void)hipEventElapsedTime(&c->phase_ms[i - 1], c->ev[i - 1], c->ev[i]);
    pdd::free_grid(&grid);
    return rc;
}

extern "C" {

int pdd_decimate(pdd_ctx* ctx, const int32_t* d_xyz, int64_t n, int64_t keep_count, const pdd_opts* opts,
                 int32_t* d_kept, int32_t* d_order, uint64_t* d_order_cost) {
    if (!ctx || !d_xyz || !opts || !d_kept || n < 2 || n >= (int64_t)0x7FFFFFFF) return PDD_EINVAL;
    if (keep_count < 1 || keep_count > n) return PDD_EINVAL;
    const int64_t off[2] = {0, n};
    return decimate_common(ctx, d_xyz, n, off, &keep_count, 1, opts, d_kept, d_order, d_order_cost);
}

int pdd_decimate_batch(pdd_ctx* ctx, const int32_t* d_xyz, const int64_t* h_offsets, int32_t nscan,
                       const int64_t* h_keep, const pdd_opts* opts, int32_t* d_kept, int32_t* d_order,
                       uint64_t* d_order_cost) {
    if (!ctx || !d_xyz || !h_offsets || !h_keep || !opts || !d_kept || nscan < 1 || nscan > (1 << 20))
        return PDD_EINVAL;
    if (h_offsets[0] != 0) return PDD_EINVAL;
    for (int s = 0; s < nscan; s++) {
        const int64_t ns = h_offsets[s + 1] - h_offsets[s];
        if (ns < 2 || ns >= (int64_t)0x7FFFFFFF || h_keep[s] < 1 || h_keep[s] > ns) return PDD_EINVAL;
    }
    const int stride = opts->point_stride == 0 ? 12 : opts->point_stride;
    if (stride != 12 && stride != 16) return PDD_EINVAL;
    // consecutive groups of clouds of at most kBatchGroup points, each one
    // segmented decimation; the outputs of a group go after the previous ones
    int64_t kept_at = 0, order_at = 0;
    int first = 0;
    // counters and phase times of the whole call: summed over the groups
    // (scratch held and the levels/list width: the last group's)
    int64_t stats[pdd::kNumStats] = {0};
    float phase[pdd::kPhCount] = {0};
    while (first < nscan) {
        int last = first + 1;
        while (last < nscan && h_offsets[last + 1] - h_offsets[first] <= kBatchGroup) last++;
        const int ng = last - first;
        std::vector<int64_t> off((size_t)ng + 1), keep((size_t)ng);
        int64_t gkeep = 0;
        for (int s = 0; s < ng; s++) {
            off[s] = h_offsets[first + s] - h_offsets[first];
            keep[s] = h_keep[first + s];
            gkeep += keep[s];
        }
        off[ng] = h_offsets[last] - h_offsets[first];
        const int32_t* xyz = (const int32_t*)((const char*)d_xyz + h_offsets[first] * stride);
        int rc = decimate_common(ctx, xyz, off[ng], off.data(), keep.data(), ng, opts, d_kept + kept_at,
                                 d_order ? d_order + order_at : nullptr, d_order_cost ? d_order_cost + order_at : nullptr);
        if (rc) return rc;
        for (int i = 0; i < pdd::kNumStats; i++) stats[i] = (i == 4 || i == 5 || i == 6) ? ctx->c.stats[i] : stats[i] + ctx->c.stats[i];
        for (int i = 0; i < pdd::kPhCount; i++) phase[i] += ctx->c.phase_ms[i];
        kept_at += gkeep;
        order_at += off[ng] - gkeep;
        first = last;
    }
    for (int i = 0; i < pdd::kNumStats; i++) ctx->c.stats[i] = stats[i];
    for (int i = 0; i < pdd::kPhCount; i++) ctx->c.phase_ms[i] = phase[i];
    return PDD_OK;
}

int pdd_last_stats(const pdd_ctx* ctx, int64_t* stats, int n) {
    if (!ctx || !stats || n < 0) return 0;
    int m = n < pdd::kNumStats ? n : pdd::kNumStats;
    for (int i = 0; i < m; i++) stats[i] = ctx->c.stats[i];
    return m;
}

int pdd_last_timing(const pdd_ctx* ctx, float* ms, int n) {
    if (!ctx || !ms || n < 0) return 0;
    int m = n < pdd::kPhCount - 1 ? n : pdd::kPhCount - 1;
    for (int i = 0; i < m; i++) ms[i] = ctx->c.phase_ms[i];
    return m;
}

int pdd_autotune(pdd_ctx* ctx, const int32_t* d_xyz, int64_t n, int64_t keep, const pdd_opts* base, int64_t sample,
                 pdd_opts* out, float* best_ms) {
    if (!ctx || !d_xyz || !base || !out || n >= (int64_t)0x7FFFFFFF) return PDD_EINVAL;
    Ctx* c = &ctx->c;
    if (hipSetDevice(c->device) != hipSuccess) return PDD_EHIP;
    return pdd::autotune(c, d_xyz, n, keep, base, sample, out, best_ms);
}

int pdd_quality_measure(pdd_ctx* ctx, const int32_t* d_xyz, int64_t m, int32_t stride_bytes, const int64_t* h_r2,
                        int32_t R, uint32_t* d_counts, int64_t* d_nn2, pdd_quality* out) {
    if (!ctx || !d_xyz || !h_r2 || !out || m < 2 || m >= (int64_t)0x7FFFFFFF) return PDD_EINVAL;
    Ctx* c = &ctx->c;
    if (hipSetDevice(c->device) != hipSuccess) return PDD_EHIP;
    return pdd::quality(c, d_xyz, m, stride_bytes == 0 ? 12 : stride_bytes, h_r2, R, d_counts, d_nn2, out);
}

int pdd_autotune_batch(pdd_ctx* ctx, const int32_t* d_xyz, const int64_t* h_offsets, int32_t nscan,
                       const int64_t* h_keep, const pdd_opts* base, int64_t sample, pdd_opts* out, float* best_ms) {
    if (!ctx || !d_xyz || !h_offsets || !h_keep || !base || !out || nscan < 1 || nscan > (1 << 20))
        return PDD_EINVAL;
    if (h_offsets[0] != 0) return PDD_EINVAL;
    Ctx* c = &ctx->c;
    if (hipSetDevice(c->device) != hipSuccess) return PDD_EHIP;
    return pdd::autotune_batch(c, d_xyz, h_offsets, nscan, h_keep, base, sample, out, best_ms);
}

// ---------------------------------------------------------------------------
// search-radius predictor
// ---------------------------------------------------------------------------

int pdd_pred_set_weights(pdd_ctx* ctx, const float* params, int64_t n) {
    if (!ctx) return PDD_EINVAL;
    if (hipSetDevice(ctx->c.device) != hipSuccess) return PDD_EHIP;
    return pdd::pred_set(&ctx->c, params, n);
}

int pdd_pred_get_weights(pdd_ctx* ctx, float* params, int64_t n) {
    if (!ctx) return PDD_EINVAL;
    if (hipSetDevice(ctx->c.device) != hipSuccess) return PDD_EHIP;
    return pdd::pred_get(&ctx->c, params, n);
}

int pdd_pred_enable(pdd_ctx* ctx, int32_t on, float margin_log2) {
    if (!ctx || !(margin_log2 >= 0.0f && margin_log2 <= 8.0f)) return PDD_EINVAL;
    if (on && !ctx->c.pred_ready) return PDD_EINVAL;
    ctx->c.pred_on = on != 0;
    ctx->c.pred_margin = margin_log2;
    return PDD_OK;
}

int pdd_pred_samples(pdd_ctx* ctx, const pdd_grid* grid, int32_t k, int32_t b, uint16_t* d_feat, float* d_target,
                     int64_t cap, int64_t* count) {
    if (!ctx || !grid || !count || k < 1 || b < 0 || k + b > pdd::kMaxK || cap < 0) return PDD_EINVAL;
    if (cap > 0 && (!d_feat || !d_target)) return PDD_EINVAL;
    Ctx* c = &ctx->c;
    if (hipSetDevice(c->device) != hipSuccess) return PDD_EHIP;
    return pdd::pred_samples(c, grid->g.v, k, pdd::list_width(k + b), d_feat, d_target, cap, count);
}

int pdd_pred_forward(pdd_ctx* ctx, const uint16_t* d_feat, int64_t n, float* d_out) {
    if (!ctx || n < 0 || (n > 0 && (!d_feat || !d_out))) return PDD_EINVAL;
    Ctx* c = &ctx->c;
    if (hipSetDevice(c->device) != hipSuccess) return PDD_EHIP;
    int rc = pdd::pred_forward(c, d_feat, n, d_out);
    if (rc) return rc;
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    return PDD_OK;
}

int pdd_pred_grad(pdd_ctx* ctx, const uint16_t* d_feat, const float* d_target, int64_t n, float tau, float* d_grad,
                  float* d_loss) {
    if (!ctx || !d_feat || !d_target || !d_grad || !(tau > 0.0f && tau < 1.0f)) return PDD_EINVAL;
    Ctx* c = &ctx->c;
    if (hipSetDevice(c->device) != hipSuccess) return PDD_EHIP;
    int rc = pdd::pred_grad(c, d_feat, d_target, n, tau, d_grad, d_loss);
    if (rc) return rc;
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    return PDD_OK;
}

int pdd_pred_train(pdd_ctx* ctx, const uint16_t* d_feat, const float* d_target, int64_t n, int32_t steps,
                   int32_t batch, float lr, float tau, uint64_t seed, float* d_loss) {
    if (!ctx || !d_feat || !d_target) return PDD_EINVAL;
    Ctx* c = &ctx->c;
    if (hipSetDevice(c->device) != hipSuccess) return PDD_EHIP;
    return pdd::pred_train(c, d_feat, d_target, n, steps, batch, lr, tau, seed, d_loss);
}

}  // extern "C"
