// Initial k-nearest-neighbour lists and costs of every point (Eq. 12).
#include <algorithm>

#include "search.h"

namespace pdd {

namespace {

// One wavefront per query (see wave_knn).
template <int K>
__global__ void __launch_bounds__(kBlock) knn_wave_k(GridView g, int k, int32_t* __restrict__ nbr,
                                                     uint8_t* __restrict__ cnt, uint64_t* __restrict__ cost,
                                                     int64_t* __restrict__ r2k) {
    __shared__ uint32_t lds[kBlock / kWave][2][kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    // Waves stride over the queries in Morton order, so the waves resident
    // at one time read overlapping cells.
    const uint32_t nw = gridDim.x * (kBlock / kWave);
    for (uint32_t q = blockIdx.x * (kBlock / kWave) + w; q < g.n; q += nw) {
        const int4 qp = g.pts[q];
        SearchCtx sc{nullptr};
        uint64_t d;
        int32_t id;
        const int L0 = start_level(g, q, K + 1, nullptr);
        wave_knn<K, kAll>(g, q, qp, sc, K, L0, d, id, lds[w][0], lds[w][1]);
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
    const dim3 wg(std::min<uint32_t>((g.n + 3) / 4, 16384u)), block(kBlock);
    switch (K) {
        case 8: hipLaunchKernelGGL(knn_wave_k<8>, wg, block, 0, c->stream, g, k, out.nbr, out.cnt, out.cost, out.r2k); break;
        case 16: hipLaunchKernelGGL(knn_wave_k<16>, wg, block, 0, c->stream, g, k, out.nbr, out.cnt, out.cost, out.r2k); break;
        case 24: hipLaunchKernelGGL(knn_wave_k<24>, wg, block, 0, c->stream, g, k, out.nbr, out.cnt, out.cost, out.r2k); break;
        case 32: hipLaunchKernelGGL(knn_wave_k<32>, wg, block, 0, c->stream, g, k, out.nbr, out.cnt, out.cost, out.r2k); break;
        default: return PDD_EINVAL;
    }
    PDD_HIP(c, hipGetLastError());
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
