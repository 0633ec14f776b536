// Quality measures of a decimated cloud (Sec. 6): for every point the number
// of other points within each of several radii, exact in integers; from them
// the fractiles and mean per radius and the least-squares line of count
// against area with its R^2 and RMSE; and the squared distance from every
// point to its nearest other point (Eq. 2 maximises the smallest of them).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace pdd {

namespace {

constexpr int kQHist = 4096;  // count histogram bins per radius (the last one holds every larger count)

struct Radii {
    uint64_t r2[PDD_QUALITY_MAX_R];
};

constexpr double kQFractiles[PDD_QUALITY_NFRAC] = {0.01, 0.1, 0.25, 0.5, 0.75, 0.9, 0.99};

// One thread per point.  At level Ls the cell edge is at least the largest
// radius, so the 3x3x3 cells around the point hold every point within it.
// counts[orig * R + r]; sums[2r] += count, sums[2r+1] += count^2; the count
// histogram of each radius.
__global__ void __launch_bounds__(kBlock) nc_count_k(GridView g, int Ls, Radii rad, int R,
                                                     uint32_t* __restrict__ counts,
                                                     unsigned long long* __restrict__ sums,
                                                     uint32_t* __restrict__ hist) {
    const LevelView& lv = g.lv[Ls];
    const int s = lv.s;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += gridDim.x * blockDim.x) {
        const int4 p = g.pts[i];
        const int cx = (p.x - g.minx) >> s, cy = (p.y - g.miny) >> s, cz = (p.z - g.minz) >> s;
        const uint32_t sg = seg_at(g, i);
        uint32_t cnt[PDD_QUALITY_MAX_R];
#pragma unroll
        for (int r = 0; r < PDD_QUALITY_MAX_R; r++) cnt[r] = 0;
        for (int b = 0; b < 27; b++) {
            const int x = cx + b % 3 - 1, y = cy + (b / 3) % 3 - 1, z = cz + b / 9 - 1;
            if (x < 0 || y < 0 || z < 0 || x > lv.cmax[0] || y > lv.cmax[1] || z > lv.cmax[2]) continue;
            const uint32_t c = hash_find(lv.hkeys, lv.hvals, lv.hmask, cell_code(lv, sg, x, y, z));
            if (c == kNone) continue;
            const uint32_t j1 = lv.start[c + 1];
            for (uint32_t j = lv.start[c]; j < j1; j++) {
                if (j == i) continue;
                const int4 q = g.pts[j];
                const uint64_t d = dist2(p.x, p.y, p.z, q.x, q.y, q.z);
#pragma unroll
                for (int r = 0; r < PDD_QUALITY_MAX_R; r++) cnt[r] += (r < R && d <= rad.r2[r]) ? 1u : 0u;
            }
        }
        const size_t o = (size_t)(uint32_t)p.w;
#pragma unroll
        for (int r = 0; r < PDD_QUALITY_MAX_R; r++) {
            if (r >= R) break;
            if (counts) counts[o * R + r] = cnt[r];
            atomicAdd(&sums[2 * r], (unsigned long long)cnt[r]);
            atomicAdd(&sums[2 * r + 1], (unsigned long long)cnt[r] * cnt[r]);
            atomicAdd(&hist[(size_t)r * kQHist + (cnt[r] < (uint32_t)kQHist ? cnt[r] : kQHist - 1)], 1u);
        }
    }
}

__global__ void __launch_bounds__(kBlock) nn_min_k(const int64_t* __restrict__ nn2, uint32_t m,
                                                   unsigned long long* __restrict__ out) {
    unsigned long long best = ~0ull;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
        best = std::min(best, (unsigned long long)nn2[i]);
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)best, o, kWave);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(best >> 32), o, kWave);
        const unsigned long long v = ((unsigned long long)hi << 32) | lo;
        if (v < best) best = v;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMin(out, best);
}

enum { kSlotQSums = 106, kSlotQHist = 107, kSlotQNbr = 108, kSlotQCnt = 109, kSlotQCost = 110, kSlotQR2k = 111,
       kSlotQNN = 112, kSlotQMin = 113, kSlotQCostO = 114 };

constexpr double kPi = 3.14159265358979323846;

}  // namespace

int quality(Ctx* c, const int32_t* d_xyz, int64_t m, int stride, const int64_t* h_r2, int R, uint32_t* d_counts,
            int64_t* d_nn2, pdd_quality* out) {
    if (m < 2 || R < 1 || R > PDD_QUALITY_MAX_R || (stride != 12 && stride != 16) || !out) return PDD_EINVAL;
    for (int r = 0; r < R; r++)
        if (h_r2[r] < 0 || (r > 0 && h_r2[r] <= h_r2[r - 1])) return PDD_EINVAL;
    Grid grid;
    int rc = build_grid(c, d_xyz, m, stride, 0, &grid);
    if (rc) {
        free_grid(&grid);
        return rc;
    }
    const GridView& g = grid.v;
    const uint32_t n = g.n;
    unsigned long long* sums = (unsigned long long*)scratch(c, kSlotQSums, (size_t)2 * R * 8);
    uint32_t* hist = (uint32_t*)scratch(c, kSlotQHist, (size_t)R * kQHist * 4);
    unsigned long long* dmin = (unsigned long long*)scratch(c, kSlotQMin, 8);
    KnnOut ko;
    ko.nbr = (int32_t*)scratch(c, kSlotQNbr, (size_t)n * 8 * 4);
    ko.cnt = (uint8_t*)scratch(c, kSlotQCnt, (size_t)n);
    ko.cost = (uint64_t*)scratch(c, kSlotQCost, (size_t)n * 8);
    ko.r2k = (int64_t*)scratch(c, kSlotQR2k, (size_t)n * 8);
    int64_t* nn2 = d_nn2 ? d_nn2 : (int64_t*)scratch(c, kSlotQNN, (size_t)n * 8);
    uint64_t* cost_o = (uint64_t*)scratch(c, kSlotQCostO, (size_t)n * 8);  // the k = 1 costs (not reported)
    if (!sums || !hist || !dmin || !ko.nbr || !ko.cnt || !ko.cost || !ko.r2k || !nn2 || !cost_o) {
        free_grid(&grid);
        return PDD_ENOMEM;
    }
    do {
        if ((rc = fill_u32(c, (uint32_t*)sums, 0, (size_t)4 * R))) break;
        if ((rc = fill_u32(c, hist, 0, (size_t)R * kQHist))) break;
        if ((rc = fill_u32(c, (uint32_t*)dmin, 0xFFFFFFFFu, 2))) break;
        // the finest level whose cell edge reaches the largest radius
        const double rmax = std::sqrt((double)h_r2[R - 1]);
        int sn = 0;
        while (sn < 30 && (double)(1ll << sn) < rmax) sn++;
        const int Ls = std::min(std::max(sn - g.lv[0].s, 0), g.nlev - 1);
        // the 3x3x3 block must hold every point within the largest radius:
        // the cell edge reaches it, or the level's cells cover the cloud in
        // at most two per axis
        const LevelView& ls = g.lv[Ls];
        if (!((double)(1ll << ls.s) >= rmax || (ls.cmax[0] <= 1 && ls.cmax[1] <= 1 && ls.cmax[2] <= 1))) {
            c->err = "largest radius beyond the grid's levels";
            rc = PDD_EINVAL;
            break;
        }
        Radii rad{};
        for (int r = 0; r < R; r++) rad.r2[r] = (uint64_t)h_r2[r];
        hipLaunchKernelGGL(nc_count_k, dim3(std::min<uint32_t>((n + kBlock - 1) / kBlock, 16384u)), dim3(kBlock), 0,
                           c->stream, g, Ls, rad, R, d_counts, sums, hist);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            rc = hip_fail(c, e, "nc_count_k");
            break;
        }
        // nearest other point: the k-NN with k = 1 (list width 8)
        if ((rc = knn_all(c, g, 1, 8, ko, nullptr))) break;
        if ((rc = knn_to_original(c, g, 8, 1, ko, nullptr, nn2, cost_o))) break;
        hipLaunchKernelGGL(nn_min_k, dim3(std::min<uint32_t>((n + kBlock - 1) / kBlock, 1024u)), dim3(kBlock), 0,
                           c->stream, nn2, n, dmin);
        e = hipGetLastError();
        if (e != hipSuccess) rc = hip_fail(c, e, "nn_min_k");
    } while (0);
    std::vector<unsigned long long> hs((size_t)2 * R);
    std::vector<uint32_t> hh((size_t)R * kQHist);
    unsigned long long hmin = 0;
    if (!rc) {
        hipError_t e = hipMemcpyAsync(hs.data(), sums, hs.size() * 8, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(hh.data(), hist, hh.size() * 4, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&hmin, dmin, 8, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = hip_fail(c, e, "quality read-back");
    }
    (void)hipStreamSynchronize(c->stream);
    free_grid(&grid);
    if (rc) return rc;

    // the summary, from the exact sums and histograms
    *out = pdd_quality{};
    out->R = R;
    out->m = m;
    double sx = 0, sxx = 0, sy = 0, syy = 0, sxy = 0;
    for (int r = 0; r < R; r++) {
        const double area = kPi * (double)h_r2[r] / 1e6;
        out->area_m2[r] = area;
        out->sum[r] = hs[2 * r];
        out->sum_sq[r] = hs[2 * r + 1];
        out->mean[r] = (double)hs[2 * r] / (double)m;
        for (int f = 0; f < PDD_QUALITY_NFRAC; f++) {
            const uint64_t k = (uint64_t)std::floor(kQFractiles[f] * (double)(m - 1));
            uint64_t cum = 0;
            int v = kQHist - 1;
            for (int b = 0; b < kQHist; b++) {
                cum += hh[(size_t)r * kQHist + b];
                if (cum > k) {
                    v = b;
                    break;
                }
            }
            out->fractile[r][f] = (uint32_t)v;
            if (v == kQHist - 1) out->fractile_capped = 1;
        }
        sx += area;
        sxx += area * area;
        sy += (double)hs[2 * r];
        syy += (double)hs[2 * r + 1];
        sxy += area * (double)hs[2 * r];
    }
    const double nn = (double)m * (double)R;
    sx *= (double)m;
    sxx *= (double)m;
    const double den = nn * sxx - sx * sx;
    const double slope = den != 0 ? (nn * sxy - sx * sy) / den : 0.0;
    const double icpt = (sy - slope * sx) / nn;
    const double ss_res = syy - 2.0 * icpt * sy - 2.0 * slope * sxy + nn * icpt * icpt + 2.0 * icpt * slope * sx +
                          slope * slope * sxx;
    const double ss_tot = syy - sy * sy / nn;
    out->slope = slope;
    out->intercept = icpt;
    out->r_squared = ss_tot > 0 ? 1.0 - ss_res / ss_tot : 1.0;
    out->rmse = std::sqrt(std::max(ss_res, 0.0) / nn);
    out->nn2_min = (int64_t)hmin;
    return PDD_OK;
}

}  // namespace pdd
