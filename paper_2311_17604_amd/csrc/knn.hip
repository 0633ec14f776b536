// Initial k-nearest-neighbour lists and costs of every point (Eq. 12).
#include <algorithm>

#include "predictor.h"

namespace pdd {

namespace {

constexpr int kSlotKnnStat = 88;

// One wavefront per query (see wave_knn).  With rhat2 (squared radius per
// anchor cell, 0 = none) the search first tests the predicted ball and
// falls back to the shell search when that does not certify the list.
// stat: points tested, ball hits, ball misses (one atomic each per wave).
template <int K>
__global__ void __launch_bounds__(kBlock) knn_wave_k(GridView g, int k, int32_t* __restrict__ nbr,
                                                     uint8_t* __restrict__ cnt, uint64_t* __restrict__ cost,
                                                     int64_t* __restrict__ r2k, const uint64_t* __restrict__ rhat2,
                                                     unsigned long long* __restrict__ stat) {
    __shared__ uint32_t lds[kBlock / kWave][2][kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t tested = 0, hits = 0, misses = 0;
    // Waves stride over the queries in Morton order, so the waves resident
    // at one time read overlapping cells.
    const uint32_t nw = gridDim.x * (kBlock / kWave);
    for (uint32_t q = blockIdx.x * (kBlock / kWave) + w; q < g.n; q += nw) {
        const int4 qp = g.pts[q];
        SearchCtx sc{nullptr};
        uint64_t d;
        int32_t id;
        int La;
        uint32_t ca;
        anchor_cell(g, q, K + 1, nullptr, &La, &ca);
        bool done = false;
        if (rhat2 && La >= 1) {
            const uint64_t r2 = rhat2[g.lv[La].base + ca];
            if (r2) {
                done = wave_knn_ball<K, kAll>(g, q, qp, sc, K, r2, d, id, lds[w][0], lds[w][1], &tested);
                if (done) hits++;
                else misses++;
            }
        }
        if (!done) wave_knn<K, kAll>(g, q, qp, sc, K, La > 0 ? La - 1 : 0, d, id, lds[w][0], lds[w][1], &tested);
        const int c = __popcll(__ballot(lane < K && d != ~0ull));
        const int use = c < k ? c : k;
        const uint64_t wsum = wave_sum64(lane < use ? cost_term(d) : 0ull);
        if (lane < K) nbr[(size_t)q * K + lane] = id;
        if (lane == use - 1 && r2k) r2k[q] = (int64_t)d;
        if (lane == 0) {
            cnt[q] = (uint8_t)c;
            cost[q] = wsum;
        }
    }
    if (lane == 0) {
        atomicAdd(&stat[0], (unsigned long long)tested);
        if (hits) atomicAdd(&stat[1], (unsigned long long)hits);
        if (misses) atomicAdd(&stat[2], (unsigned long long)misses);
    }
}

__global__ void __launch_bounds__(kBlock) to_original_k(const int4* __restrict__ pts, uint32_t n, int K, int Kout,
                                                        const int32_t* __restrict__ nbr_s,
                                                        const uint64_t* __restrict__ cost_s,
                                                        const int64_t* __restrict__ r2k_s, int32_t* __restrict__ nbr,
                                                        int64_t* __restrict__ r2k, uint64_t* __restrict__ cost) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const uint32_t o = (uint32_t)pts[q].w;
    if (nbr)
        for (int j = 0; j < Kout; j++) {
            int32_t id = nbr_s[(size_t)q * K + j];
            nbr[(size_t)o * Kout + j] = id >= 0 ? pts[id].w : -1;
        }
    if (r2k) r2k[o] = r2k_s[q];
    cost[o] = cost_s[q];
}

}  // namespace

int knn_all(Ctx* c, const GridView& g, int k, int K, KnnOut out, int64_t* fallbacks) {
    if (fallbacks) *fallbacks = 0;
    unsigned long long* stat = (unsigned long long*)scratch(c, kSlotKnnStat, 4 * sizeof(unsigned long long));
    if (!stat) return PDD_ENOMEM;
    int rc = fill_u32(c, (uint32_t*)stat, 0, 8);
    if (rc) return rc;
    const uint64_t* r2 = nullptr;
    if (c->pred_on && c->pred_ready && (rc = pred_radii(c, g, K, &r2))) return rc;
    const dim3 wg(std::min<uint32_t>((g.n + 3) / 4, 16384u)), block(kBlock);
    switch (K) {
        case 8: hipLaunchKernelGGL(knn_wave_k<8>, wg, block, 0, c->stream, g, k, out.nbr, out.cnt, out.cost, out.r2k, r2, stat); break;
        case 16: hipLaunchKernelGGL(knn_wave_k<16>, wg, block, 0, c->stream, g, k, out.nbr, out.cnt, out.cost, out.r2k, r2, stat); break;
        case 24: hipLaunchKernelGGL(knn_wave_k<24>, wg, block, 0, c->stream, g, k, out.nbr, out.cnt, out.cost, out.r2k, r2, stat); break;
        case 32: hipLaunchKernelGGL(knn_wave_k<32>, wg, block, 0, c->stream, g, k, out.nbr, out.cnt, out.cost, out.r2k, r2, stat); break;
        default: return PDD_EINVAL;
    }
    PDD_HIP(c, hipGetLastError());
    // counters: points tested, predicted balls that certified, that did not
    unsigned long long* h = (unsigned long long*)c->pinned;
    PDD_HIP(c, hipMemcpyAsync(h, stat, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    c->stats[8] = (int64_t)h[0];
    c->stats[9] = (int64_t)h[1];
    c->stats[10] = (int64_t)h[2];
    return PDD_OK;
}

int knn_to_original(Ctx* c, const GridView& g, int K, int Kout, const KnnOut& in, int32_t* nbr, int64_t* r2k,
                    uint64_t* cost) {
    hipLaunchKernelGGL(to_original_k, dim3((g.n + kBlock - 1) / kBlock), dim3(kBlock), 0, c->stream, g.pts, g.n, K,
                       Kout, in.nbr, in.cost, in.r2k, nbr, r2k, cost);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

}  // namespace pdd
