// Autotuner: picks the finest cell level, the list width (k + b) and the
// initial round share for a cloud by timing trial decimations of a strided
// sample.  None of the three can change a result (the grid, the buffer and
// the rounds are exact for every setting), so the tuner trades only time.
#include <algorithm>
#include <vector>

#include "common.h"

namespace pdd {

int decimate_entry(Ctx* c, const int32_t* d_xyz, int64_t n, const int64_t* h_off, const int64_t* h_keep, int nseg,
                   const pdd_opts* opts, int32_t* d_kept, int32_t* d_order, uint64_t* d_order_cost);

namespace {

// every step-th point (a sparser copy of the cloud with the same structure)
__global__ void __launch_bounds__(kBlock) gather_k(const int32_t* __restrict__ xyz, int sw, uint64_t step, uint32_t m,
                                                   int32_t* __restrict__ out) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const int32_t* p = xyz + (size_t)(i * step) * sw;
        out[3 * (size_t)i] = p[0];
        out[3 * (size_t)i + 1] = p[1];
        out[3 * (size_t)i + 2] = p[2];
    }
}

enum { kTuneXyz = 120, kTuneKept, kTuneOrder, kTuneCost };

}  // namespace

int autotune(Ctx* c, const int32_t* d_xyz, int64_t n, int64_t keep, const pdd_opts* base, int64_t sample,
             pdd_opts* out, float* best_ms) {
    const int stride = base->point_stride == 0 ? 12 : base->point_stride;
    if (n < 2 || keep < 1 || keep > n || (stride != 12 && stride != 16) || base->k < 1 || base->k > kMaxK)
        return PDD_EINVAL;
    if (sample <= 0) sample = 2000000;
    const uint64_t step = (uint64_t)std::max<int64_t>(1, (n + sample - 1) / sample);
    const uint32_t m = (uint32_t)((n + (int64_t)step - 1) / (int64_t)step);
    if (m < 2) return PDD_EINVAL;
    const int64_t mkeep = std::max<int64_t>(1, std::min<int64_t>(m, (int64_t)((double)keep * m / n + 0.5)));
    int32_t* xs = (int32_t*)scratch(c, kTuneXyz, (size_t)m * 12);
    int32_t* kept = (int32_t*)scratch(c, kTuneKept, (size_t)mkeep * 4);
    int32_t* order = (int32_t*)scratch(c, kTuneOrder, (size_t)(m - mkeep + 1) * 4);
    uint64_t* oc = (uint64_t*)scratch(c, kTuneCost, (size_t)(m - mkeep + 1) * 8);
    if (!xs || !kept || !order || !oc) return PDD_ENOMEM;
    hipLaunchKernelGGL(gather_k, dim3(std::min<uint32_t>((m + kBlock - 1) / kBlock, 16384u)), dim3(kBlock), 0,
                       c->stream, d_xyz, stride / 4, step, m, xs);
    PDD_HIP(c, hipGetLastError());
    hipEvent_t e0, e1;
    PDD_HIP(c, hipEventCreate(&e0));
    PDD_HIP(c, hipEventCreate(&e1));
    const int64_t off[2] = {0, (int64_t)m};
    auto trial = [&](const pdd_opts& o, float* ms) -> int {
        pdd_opts t = o;
        t.point_stride = 12;
        t.flags = 0;
        PDD_HIP(c, hipEventRecord(e0, c->stream));
        int rc = decimate_entry(c, xs, m, off, &mkeep, 1, &t, kept, order, oc);
        if (rc) return rc;
        PDD_HIP(c, hipEventRecord(e1, c->stream));
        PDD_HIP(c, hipEventSynchronize(e1));
        PDD_HIP(c, hipEventElapsedTime(ms, e0, e1));
        return PDD_OK;
    };
    pdd_opts best = *base;
    best.flags = base->flags;
    if (best.round_frac == 0.0f) best.round_frac = 0.01f;
    float tbest = 0.f;
    int rc = trial(best, &tbest);
    // the sample's automatic finest level, to tune an offset from it
    const int s_auto_sample = (int)c->stats[5];
    int dvox = 0;
    // coordinate descent: round share, list width, finest level
    for (float f : {0.005f, 0.0025f, 0.00175f, 0.00125f, 0.02f, 0.04f}) {
        pdd_opts o = best;
        o.round_frac = f;
        float ms;
        if (!rc && !(rc = trial(o, &ms)) && ms < tbest) {
            tbest = ms;
            best = o;
        }
    }
    for (int b : {4, 12, 16}) {
        if (base->k + b > kMaxK) continue;
        pdd_opts o = best;
        o.b = b;
        float ms;
        if (!rc && !(rc = trial(o, &ms)) && ms < tbest) {
            tbest = ms;
            best = o;
        }
    }
    for (int d : {-1, 1}) {
        const int v = s_auto_sample + d;
        if (v < 2 || v > 20) continue;
        pdd_opts o = best;
        o.voxel_log2 = v;
        float ms;
        if (!rc && !(rc = trial(o, &ms)) && ms < tbest) {
            tbest = ms;
            best = o;
            dvox = d;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    // the finest level for the whole cloud: its own automatic level moved by
    // the offset that won on the sample
    if (dvox != 0) {
        Grid g;
        rc = build_grid(c, d_xyz, n, stride, 0, &g);
        const int s_full = g.v.lv[0].s;
        (void)hipStreamSynchronize(c->stream);
        free_grid(&g);
        if (rc) return rc;
        best.voxel_log2 = std::min(20, std::max(2, s_full + dvox));
    } else {
        best.voxel_log2 = base->voxel_log2;
    }
    best.point_stride = base->point_stride;
    *out = best;
    if (best_ms) *best_ms = tbest;
    return PDD_OK;
}

// Batches: trial batched decimations of every step-th cloud (whole clouds,
// about `sample` points in all), gathered into one smaller batch with its
// own offsets; coordinate descent over the round share and the list width.
// The finest level stays automatic (each group of a batch picks its own).
int autotune_batch(Ctx* c, const int32_t* d_xyz, const int64_t* h_off, int nscan, const int64_t* h_keep,
                   const pdd_opts* base, int64_t sample, pdd_opts* out, float* best_ms) {
    const int stride = base->point_stride == 0 ? 12 : base->point_stride;
    if (nscan < 1 || (stride != 12 && stride != 16) || base->k < 1 || base->k > kMaxK) return PDD_EINVAL;
    if (sample <= 0) sample = 8000000;
    const int64_t total = h_off[nscan] - h_off[0];
    const int step = (int)std::max<int64_t>(1, std::min<int64_t>(nscan, (total + sample - 1) / sample));
    std::vector<int64_t> off(1, 0), keep;
    int64_t m = 0, mkeep = 0;
    for (int s = 0; s < nscan; s += step) {
        const int64_t ns = h_off[s + 1] - h_off[s];
        if (ns < 2 || h_keep[s] < 1 || h_keep[s] > ns) return PDD_EINVAL;
        if (m + ns > ((int64_t)1 << 28)) break;
        m += ns;
        mkeep += h_keep[s];
        off.push_back(m);
        keep.push_back(h_keep[s]);
    }
    const int nsub = (int)keep.size();
    if (nsub < 1) return PDD_EINVAL;
    int32_t* xs = (int32_t*)scratch(c, kTuneXyz, (size_t)m * 12);
    int32_t* kept = (int32_t*)scratch(c, kTuneKept, (size_t)mkeep * 4);
    int32_t* order = (int32_t*)scratch(c, kTuneOrder, (size_t)(m - mkeep + 1) * 4);
    uint64_t* oc = (uint64_t*)scratch(c, kTuneCost, (size_t)(m - mkeep + 1) * 8);
    if (!xs || !kept || !order || !oc) return PDD_ENOMEM;
    for (int i = 0; i < nsub; i++) {
        const int s = i * step;
        const int64_t ns = h_off[s + 1] - h_off[s];
        hipLaunchKernelGGL(gather_k, dim3(std::min<uint32_t>((uint32_t)((ns + kBlock - 1) / kBlock), 16384u)),
                           dim3(kBlock), 0, c->stream, d_xyz + (size_t)h_off[s] * (stride / 4), stride / 4, 1ull,
                           (uint32_t)ns, xs + (size_t)off[i] * 3);
    }
    PDD_HIP(c, hipGetLastError());
    hipEvent_t e0, e1;
    PDD_HIP(c, hipEventCreate(&e0));
    PDD_HIP(c, hipEventCreate(&e1));
    auto trial = [&](const pdd_opts& o, float* ms) -> int {
        pdd_opts t = o;
        t.point_stride = 12;
        t.flags = 0;
        PDD_HIP(c, hipEventRecord(e0, c->stream));
        int rc = decimate_entry(c, xs, m, off.data(), keep.data(), nsub, &t, kept, order, oc);
        if (rc) return rc;
        PDD_HIP(c, hipEventRecord(e1, c->stream));
        PDD_HIP(c, hipEventSynchronize(e1));
        PDD_HIP(c, hipEventElapsedTime(ms, e0, e1));
        return PDD_OK;
    };
    pdd_opts best = *base;
    if (best.round_frac == 0.0f) best.round_frac = 0.01f;
    float tbest = 0.f;
    int rc = trial(best, &tbest);
    for (float f : {0.005f, 0.0025f, 0.00125f, 0.000625f, 0.02f}) {
        pdd_opts o = best;
        o.round_frac = f;
        float ms;
        if (!rc && !(rc = trial(o, &ms)) && ms < tbest) {
            tbest = ms;
            best = o;
        }
    }
    for (int b : {4, 16, 24}) {
        if (base->k + b > kMaxK) continue;
        pdd_opts o = best;
        o.b = b;
        float ms;
        if (!rc && !(rc = trial(o, &ms)) && ms < tbest) {
            tbest = ms;
            best = o;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    best.voxel_log2 = base->voxel_log2;
    best.point_stride = base->point_stride;
    *out = best;
    if (best_ms) *best_ms = tbest;
    return PDD_OK;
}

}  // namespace pdd
