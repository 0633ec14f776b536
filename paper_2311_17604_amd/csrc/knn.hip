// Initial k-nearest-neighbour lists and costs of every point (Eq. 12).
#include <algorithm>

#include "predictor.h"

namespace pdd {

namespace {

constexpr int kSlotKnnStat = 88;
constexpr int kSlotTileAnc = 124, kSlotTileFlag = 125, kSlotTilePos = 126, kSlotTileList = 127,
              kSlotTileFB = 100, kSlotTileSorted = 104;
constexpr int kTileCap = 2048;  // candidates of one tile held in LDS (11-bit index)
constexpr int kTileCells = kBlock; // cells of one tile's region, at most

// Anchor cell of every point (global cell id), and a flag per anchor cell.
__global__ void __launch_bounds__(kBlock) tile_mark_k(GridView g, uint32_t need, uint32_t* __restrict__ anc_of,
                                                      uint32_t* __restrict__ flag) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < g.n; j += gridDim.x * blockDim.x) {
        int L;
        uint32_t c;
        anchor_cell(g, j, need, nullptr, &L, &c);
        const uint32_t gid = g.lv[L].base + c;
        anc_of[j] = gid;
        flag[gid] = 1u;
    }
}

__global__ void __launch_bounds__(kBlock) tile_list_k(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                                                      uint32_t total, uint32_t* __restrict__ tiles) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x)
        if (flag[t]) tiles[pos[t]] = t;
}

// Packs the threads with pred set onto slots 0.. in thread order (block
// wide; every thread must call it).  Returns the thread's slot; *count gets
// the total after the call.
__device__ inline uint32_t block_pack(bool pred, uint32_t* s_w, uint32_t* count) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint64_t m = __ballot(pred);
    if (lane == 0) s_w[w] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int i = 0; i < kBlock / kWave; i++) {
            const uint32_t v = s_w[i];
            s_w[i] = acc;
            acc += v;
        }
        *count = acc;
    }
    __syncthreads();
    return s_w[w] + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// Squared distance from u to the nearest coordinate outside cells
// [r0, r0 + w) (edge 2^s) along one axis, ignoring a side with no cell
// beyond it; ~0 when neither side has one.
__device__ inline uint64_t region_gap2(int u, int r0, int w, int s, int cmax) {
    uint64_t g = ~0ull;
    if (r0 - 1 >= 0) {
        const uint64_t lo = (uint64_t)(u - (r0 << s) + 1);
        g = lo * lo;
    }
    if (r0 + w <= cmax) {
        const uint64_t hi = (uint64_t)(((r0 + w) << s) - u);
        if (hi * hi < g) g = hi * hi;
    }
    return g;
}

// The region searched for the points anchored in one cell (global cell id
// gid): cells of level rl, per axis from r0 over w cells.  By default the
// cells of level L-1 from half an edge below the anchor cell to half an edge
// above it (level 0: the 3x3x3 block); with a predicted radius r, the cells
// of the finest level at which the anchor cell grown by r spans at most 6
// cells per axis, when they cover less than the default region.
struct TileRegion {
    int L;           // anchor level
    uint32_t c;      // anchor cell at level L
    uint32_t sg;     // segment of the anchor cell
    int ac[3];       // anchor cell coordinates at level L
    int rl;          // level of the region's cells
    int r0[3], w[3];
    bool pred;       // a predicted radius was given for this anchor
};

__device__ inline TileRegion tile_region(const GridView& g, uint32_t gid, const uint64_t* __restrict__ rhat2) {
    TileRegion R;
    int L = 0;
    while (L + 1 < g.nlev && gid >= g.lv[L + 1].base) L++;
    const LevelView& lv = g.lv[L];
    R.L = L;
    R.c = gid - lv.base;
    const uint64_t code = lv.key[R.c];
    R.sg = (uint32_t)(code >> lv.segshift);
    const uint64_t mc = code & ((1ull << lv.segshift) - 1ull);
    R.ac[0] = (int)compact21(mc);
    R.ac[1] = (int)compact21(mc >> 1);
    R.ac[2] = (int)compact21(mc >> 2);
    R.rl = L >= 1 ? L - 1 : 0;
    for (int a = 0; a < 3; a++) {
        R.r0[a] = L >= 1 ? 2 * R.ac[a] - 1 : R.ac[a] - 1;
        R.w[a] = L >= 1 ? 4 : 3;
    }
    const uint64_t rp2 = (rhat2 && L >= 1) ? rhat2[gid] : 0ull;
    R.pred = rp2 != 0;
    if (rp2) {
        const int r = (int)sqrt((double)rp2) + 1;
        for (int l = 0; l <= L; l++) {
            const int sl = g.lv[l].s;
            bool ok = true;
            int q0[3], qw[3];
            for (int a = 0; a < 3; a++) {
                const int lo = max((R.ac[a] << lv.s) - r, 0), hi = (((R.ac[a] + 1) << lv.s) - 1) + r;
                q0[a] = lo >> sl;
                qw[a] = min(hi >> sl, g.lv[l].cmax[a]) - q0[a] + 1;
                if (qw[a] > 6) ok = false;
            }
            if (ok) {
                // taken only when smaller than the default region
                const int64_t vol = (int64_t)qw[0] * qw[1] * qw[2] << (3 * sl);
                const int64_t vdef = (int64_t)R.w[0] * R.w[1] * R.w[2] << (3 * g.lv[R.rl].s);
                if (vol < vdef) {
                    R.rl = l;
                    for (int a = 0; a < 3; a++) {
                        R.r0[a] = q0[a];
                        R.w[a] = qw[a];
                    }
                }
                break;
            }
        }
    }
    return R;
}

// Largest region edge (mm) for which every squared distance between two of
// its points is below 2^21 (3 * 835^2 < 2^21), so that a candidate key
// (d2 << 11 | slot) fits 32 bits.
constexpr int kKey32Edge = 836;

// Splits the tiles by key width: regions within kKey32Edge per axis go to
// the front of `sorted` (count cnt[0]), the others to the back (cnt[1]).
__global__ void __launch_bounds__(kBlock) tile_class_k(GridView g, const uint32_t* __restrict__ tiles, uint32_t ntiles,
                                                       const uint64_t* __restrict__ rhat2,
                                                       uint32_t* __restrict__ sorted, uint32_t* __restrict__ cnt) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += gridDim.x * blockDim.x) {
        const uint32_t gid = tiles[t];
        const TileRegion R = tile_region(g, gid, rhat2);
        const int s = g.lv[R.rl].s;
        bool small = true;
        for (int a = 0; a < 3; a++)
            if (((int64_t)R.w[a] << s) > kKey32Edge) small = false;
        if (small) sorted[atomicAdd(&cnt[0], 1u)] = gid;
        else sorted[ntiles - 1u - atomicAdd(&cnt[1], 1u)] = gid;
    }
}

template <typename KT>
__device__ inline KT tile_d2(int ax, int ay, int az, int bx, int by, int bz);
template <>
__device__ inline uint32_t tile_d2<uint32_t>(int ax, int ay, int az, int bx, int by, int bz) {
    const uint32_t dx = (uint32_t)abs(ax - bx), dy = (uint32_t)abs(ay - by), dz = (uint32_t)abs(az - bz);
    return __umul24(dx, dx) + __umul24(dy, dy) + __umul24(dz, dz);
}
template <>
__device__ inline uint64_t tile_d2<uint64_t>(int ax, int ay, int az, int bx, int by, int bz) {
    return dist2(ax, ay, az, bx, by, bz);
}

// squared distance from a point at offset u (relative to the region's
// corner) to the cell at offset o (cells of edge 2^s) along one axis
template <typename KT>
__device__ inline KT box_gap2(int u, int o, int s) {
    const int lo = o << s, hi = lo + (1 << s) - 1;
    const int d = max(max(lo - u, u - hi), 0);
    return (KT)d * (KT)d;
}

// LDS-tiled k-NN: one block per anchor cell (the finest cell holding K + 1
// points).  The block loads the points of the cell's region (tile_region)
// into LDS once, ordered by cell: cells that overlap the anchor cell first,
// then cells beside it across a face, an edge, a corner.  Each thread takes
// one point anchored there and walks the cells, keeping its K smallest
// (d2, slot) keys in registers; a wave passes over a cell when no lane's
// K-th distance reaches beyond the cell's distance from that lane's point.
// KT is the key type: 32 bits for tiles whose region fits kKey32Edge, else
// 64.  The list is exact when its K-th distance is within the region's
// distance to the nearest cell outside it; other points (and tiles whose
// region holds more than kTileCap points) go to the fallback list for the
// wave search.  part 0 takes tiles[0, tcnt[0]), part 1 tiles[ntiles -
// tcnt[1], ntiles).
template <int K, typename KT>
__global__ void __launch_bounds__(kBlock) knn_tile_k(GridView g, int k, const uint32_t* __restrict__ tiles,
                                                     const uint32_t* __restrict__ tcnt, uint32_t ntiles, int part,
                                                     const uint32_t* __restrict__ anc_of,
                                                     const uint64_t* __restrict__ rhat2, int32_t* __restrict__ nbr,
                                                     uint8_t* __restrict__ cnt, uint64_t* __restrict__ cost,
                                                     int64_t* __restrict__ r2k, uint32_t* __restrict__ fb,
                                                     unsigned long long* __restrict__ stat) {
    constexpr KT kEmpty = (KT)~(KT)0;
    __shared__ int4 cand[kTileCap];
    __shared__ uint32_t cst[kTileCells], cex[kTileCells + 1], coff[kTileCells];
    __shared__ uint32_t s_q[kBlock], s_pack[kBlock / kWave + 1], s_npack;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const uint32_t tb = part == 0 ? 0u : ntiles - tcnt[1];
    const uint32_t te = part == 0 ? tcnt[0] : ntiles;
    uint32_t tested = 0, hits = 0, misses = 0;
    for (uint32_t t = tb + blockIdx.x; t < te; t += gridDim.x) {
        const uint32_t gid = tiles[t];
        const TileRegion R = tile_region(g, gid, rhat2);
        const LevelView& lv = g.lv[R.L];
        const LevelView& rv = g.lv[R.rl];
        const int s = rv.s;
        const int ncell = R.w[0] * R.w[1] * R.w[2];
        // look the cells up (one per thread); rank = axes along which the
        // cell lies outside the anchor cell
        uint32_t st = 0, n = 0, off = 0;
        int rank = 4;
        if (tid < ncell) {
            const int ix = tid % R.w[0], iy = (tid / R.w[0]) % R.w[1], iz = tid / (R.w[0] * R.w[1]);
            const int x = R.r0[0] + ix, y = R.r0[1] + iy, z = R.r0[2] + iz;
            const int sh = lv.s - rv.s;
            rank = ((x >> sh) != R.ac[0]) + ((y >> sh) != R.ac[1]) + ((z >> sh) != R.ac[2]);
            off = (uint32_t)ix | ((uint32_t)iy << 8) | ((uint32_t)iz << 16);
            if (x >= 0 && y >= 0 && z >= 0 && x <= rv.cmax[0] && y <= rv.cmax[1] && z <= rv.cmax[2]) {
                const uint32_t cc = hash_find(rv.hkeys, rv.hvals, rv.hmask, cell_code(rv, R.sg, x, y, z));
                if (cc != kNone) {
                    st = rv.start[cc];
                    n = rv.start[cc + 1] - st;
                }
            }
        }
        uint32_t slot = 0, acc = 0;
        for (int r = 0; r < 4; r++) {
            const uint32_t sr = block_pack(rank == r, s_pack, &s_npack);
            if (rank == r) slot = acc + sr;
            acc += s_npack;
        }
        if (tid < ncell) {
            cst[slot] = st;
            cex[slot] = n;
            coff[slot] = off;
        }
        __syncthreads();
        // exclusive scan of the ordered counts (up to kTileCells = kBlock)
        {
            const uint32_t v = tid < ncell ? cex[tid] : 0u;
            uint32_t incl = v;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const uint32_t u = (uint32_t)__shfl_up((int)incl, o, kWave);
                if (lane >= o) incl += u;
            }
            if (lane == kWave - 1) s_pack[wv] = incl;
            __syncthreads();
            uint32_t base = 0;
            for (int i = 0; i < wv; i++) base += s_pack[i];
            uint32_t tot = 0;
            for (int i = 0; i < kBlock / kWave; i++) tot += s_pack[i];
            // cex[l] = first slot of cell l; cex[l] = total past the last cell
            cex[tid] = tid < ncell ? base + incl - v : tot;
            if (tid == kBlock - 1) cex[kTileCells] = tot;
        }
        __syncthreads();
        const uint32_t total = cex[kTileCells];
        const bool fits = total <= (uint32_t)kTileCap;
        if (fits)
            for (uint32_t u = tid; u < total; u += blockDim.x) {
                int l = 0;
#pragma unroll
                for (int step = kTileCells / 2; step > 0; step >>= 1)
                    if (l + step < ncell && cex[l + step] <= u) l += step;
                const uint32_t j = cst[l] + (u - cex[l]);
                const int4 p = g.pts[j];
                cand[u] = make_int4(p.x, p.y, p.z, (int)j);
            }
        __syncthreads();
        // the points anchored here, packed onto the first threads (waves
        // past the last query skip the scan)
        const uint32_t q0 = lv.start[R.c], q1 = lv.start[R.c + 1];
        for (uint32_t qb = q0; qb < q1; qb += blockDim.x) {
            const uint32_t qq = qb + tid;
            const bool anch = qq < q1 && anc_of[qq] == gid;
            const uint32_t qslot = block_pack(anch, s_pack, &s_npack);
            if (anch) s_q[qslot] = qq;
            __syncthreads();
            const uint32_t nq = s_npack;
            const bool mine = (uint32_t)tid < nq;
            const uint32_t q = mine ? s_q[tid] : 0u;
            __syncthreads();
            if (!fits) {
                if (mine) fb[atomicAdd(&stat[3], 1ull)] = q;
                if (mine && R.pred) misses++;
                continue;
            }
            if ((uint32_t)(tid & ~(kWave - 1)) >= nq) continue;  // whole wave without a query
            int4 qp = make_int4(0, 0, 0, 0);
            if (mine) qp = g.pts[q];
            // the point relative to the region's corner
            const int ux = qp.x - g.minx - R.r0[0] * (1 << s), uy = qp.y - g.miny - R.r0[1] * (1 << s),
                      uz = qp.z - g.minz - R.r0[2] * (1 << s);
            KT top[K];
#pragma unroll
            for (int e = 0; e < K; e++) top[e] = kEmpty;
            // candidates below the lane's K-th key wait in a 4-entry buffer;
            // the (wave-wide) sorted insertion runs when some lane's buffer
            // is full, and at the end
            KT b0 = kEmpty, b1 = kEmpty, b2 = kEmpty, b3 = kEmpty;
            int nb = 0;
            auto insert = [&](KT key) {
                if (key < top[K - 1]) {
#pragma unroll
                    for (int e = K - 1; e > 0; e--) {
                        if (key < top[e - 1]) top[e] = top[e - 1];
                        else if (key < top[e]) top[e] = key;
                    }
                    if (key < top[0]) top[0] = key;
                }
            };
            auto flush = [&]() {
                if (nb > 0) insert(b0);
                if (nb > 1) insert(b1);
                if (nb > 2) insert(b2);
                if (nb > 3) insert(b3);
                nb = 0;
            };
            for (int l = 0; l < ncell; l++) {
                const uint32_t u0 = cex[l], u1 = cex[l + 1];
                if (u0 == u1) continue;
                // no candidate of a cell at box distance >= the lane's K-th
                // distance can change the lane's distances (a tie at the
                // K-th distance leaves their multiset as it is)
                const uint32_t o = coff[l];
                const KT bd = box_gap2<KT>(ux, (int)(o & 255u), s) + box_gap2<KT>(uy, (int)((o >> 8) & 255u), s) +
                              box_gap2<KT>(uz, (int)(o >> 16), s);
                if (!__any(mine && bd < (KT)(top[K - 1] >> 11))) continue;
                if (mine) tested += u1 - u0;
                for (uint32_t u = u0; u < u1; u++) {
                    const int4 p = cand[u];
                    const KT key = (tile_d2<KT>(qp.x, qp.y, qp.z, p.x, p.y, p.z) << 11) | (KT)u;
                    if (mine && (uint32_t)p.w != q && key < top[K - 1]) {
                        b3 = nb == 3 ? key : b3;
                        b2 = nb == 2 ? key : b2;
                        b1 = nb == 1 ? key : b1;
                        b0 = nb == 0 ? key : b0;
                        nb++;
                    }
                    if (__any(nb == 4)) flush();
                }
            }
            flush();
            if (!mine) continue;
            int filled = 0;
#pragma unroll
            for (int e = 0; e < K; e++) filled += top[e] != kEmpty;
            uint64_t gap = region_gap2(qp.x - g.minx, R.r0[0], R.w[0], s, rv.cmax[0]);
            const uint64_t gy = region_gap2(qp.y - g.miny, R.r0[1], R.w[1], s, rv.cmax[1]);
            const uint64_t gz = region_gap2(qp.z - g.minz, R.r0[2], R.w[2], s, rv.cmax[2]);
            if (gy < gap) gap = gy;
            if (gz < gap) gap = gz;
            const bool ok = gap == ~0ull || (filled == K && (uint64_t)(top[K - 1] >> 11) <= gap);
            if (R.pred) {
                if (ok) hits++;
                else misses++;
            }
            if (!ok) {
                fb[atomicAdd(&stat[3], 1ull)] = q;
                continue;
            }
            const int use = filled < k ? filled : k;
            uint64_t wsum = 0, dk = 0;
#pragma unroll
            for (int e = 0; e < K; e++) {
                const uint64_t d = (uint64_t)(top[e] >> 11);
                if (e < use) wsum += cost_term(d);
                if (e == use - 1) dk = d;
                nbr[(size_t)q * K + e] = e < filled ? cand[(uint32_t)(top[e] & (KT)2047)].w : -1;
            }
            cnt[q] = (uint8_t)filled;
            cost[q] = wsum;
            if (r2k) r2k[q] = (int64_t)dk;
        }
        __syncthreads();
    }
    if (tested) atomicAdd(&stat[0], (unsigned long long)tested);
    if (hits) atomicAdd(&stat[1], (unsigned long long)hits);
    if (misses) atomicAdd(&stat[2], (unsigned long long)misses);
}

// The wave search for a list of points (the tiles' fallbacks).
template <int K>
__global__ void __launch_bounds__(kBlock) knn_list_k(GridView g, int k, const uint32_t* __restrict__ list,
                                                     const unsigned long long* __restrict__ nlist,
                                                     int32_t* __restrict__ nbr, uint8_t* __restrict__ cnt,
                                                     uint64_t* __restrict__ cost, int64_t* __restrict__ r2k,
                                                     unsigned long long* __restrict__ stat) {
    __shared__ uint32_t lds[kBlock / kWave][2][kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t tested = 0;
    const uint32_t m = (uint32_t)*nlist;
    const uint32_t nw = gridDim.x * (kBlock / kWave);
    for (uint32_t t = blockIdx.x * (kBlock / kWave) + w; t < m; t += nw) {
        const uint32_t q = list[t];
        const int4 qp = g.pts[q];
        SearchCtx sc{nullptr};
        uint64_t d;
        int32_t id;
        int La;
        uint32_t ca;
        anchor_cell(g, q, K + 1, nullptr, &La, &ca);
        wave_knn<K, kAll>(g, q, qp, sc, K, La > 0 ? La - 1 : 0, d, id, lds[w][0], lds[w][1], &tested);
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
    if (lane == 0 && tested) atomicAdd(&stat[0], (unsigned long long)tested);
}

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

// tiled search with wave-search fallbacks (no predictor)
template <int K>
int knn_tiled(Ctx* c, const GridView& g, int k, KnnOut out, const uint64_t* rhat2, unsigned long long* stat) {
    const uint32_t total = g.total_cells;
    uint32_t* anc_of = (uint32_t*)scratch(c, kSlotTileAnc, (size_t)g.n * 4);
    uint32_t* flag = (uint32_t*)scratch(c, kSlotTileFlag, (size_t)(total + 1) * 4);
    uint32_t* pos = (uint32_t*)scratch(c, kSlotTilePos, (size_t)(total + 1) * 4);
    uint32_t* tiles = (uint32_t*)scratch(c, kSlotTileList, (size_t)std::max<uint32_t>(total, g.n) * 4);
    if (!anc_of || !flag || !pos || !tiles) return PDD_ENOMEM;
    int rc = fill_u32(c, flag, 0, total + 1);
    if (rc) return rc;
    const dim3 block(kBlock);
    const unsigned gp = std::min<uint32_t>((g.n + kBlock - 1) / kBlock, 16384u);
    hipLaunchKernelGGL(tile_mark_k, dim3(gp), block, 0, c->stream, g, (uint32_t)K + 1, anc_of, flag);
    PDD_HIP(c, hipGetLastError());
    if ((rc = exclusive_scan_u32(c, flag, pos, total, pos + total))) return rc;
    hipLaunchKernelGGL(tile_list_k, dim3(std::min<uint32_t>((total + kBlock - 1) / kBlock, 16384u)), block, 0,
                       c->stream, flag, pos, total, tiles);
    PDD_HIP(c, hipGetLastError());
    uint32_t* h = (uint32_t*)((char*)c->pinned + 3072);
    PDD_HIP(c, hipMemcpyAsync(h, pos + total, 4, hipMemcpyDeviceToHost, c->stream));
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    const uint32_t ntiles = h[0];
    uint32_t* fb = (uint32_t*)scratch(c, kSlotTileFB, (size_t)g.n * 4);
    if (!fb) return PDD_ENOMEM;
    uint32_t* sorted = (uint32_t*)scratch(c, kSlotTileSorted, (size_t)std::max<uint32_t>(ntiles, 1u) * 4);
    if (!sorted) return PDD_ENOMEM;
    uint32_t* tcnt = (uint32_t*)(stat + 4);
    hipLaunchKernelGGL(tile_class_k, dim3(std::min<uint32_t>((ntiles + kBlock - 1) / kBlock + 1, 16384u)), block, 0,
                       c->stream, g, tiles, ntiles, rhat2, sorted, tcnt);
    PDD_HIP(c, hipGetLastError());
    const dim3 tgrid(std::min<uint32_t>(std::max<uint32_t>(ntiles, 1u), 65535u));
    hipLaunchKernelGGL((knn_tile_k<K, uint32_t>), tgrid, block, 0, c->stream, g, k, sorted, tcnt, ntiles, 0, anc_of,
                       rhat2, out.nbr, out.cnt, out.cost, out.r2k, fb, stat);
    PDD_HIP(c, hipGetLastError());
    hipLaunchKernelGGL((knn_tile_k<K, uint64_t>), tgrid, block, 0, c->stream, g, k, sorted, tcnt, ntiles, 1, anc_of,
                       rhat2, out.nbr, out.cnt, out.cost, out.r2k, fb, stat);
    PDD_HIP(c, hipGetLastError());
    hipLaunchKernelGGL(knn_list_k<K>, dim3(2048), block, 0, c->stream, g, k, fb, stat + 3, out.nbr, out.cnt, out.cost,
                       out.r2k, stat);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

int knn_all(Ctx* c, const GridView& g, int k, int K, KnnOut out, int64_t* fallbacks) {
    if (fallbacks) *fallbacks = 0;
    // 4 counters, then the two tile counts of knn_tiled
    unsigned long long* stat = (unsigned long long*)scratch(c, kSlotKnnStat, 5 * sizeof(unsigned long long));
    if (!stat) return PDD_ENOMEM;
    int rc = fill_u32(c, (uint32_t*)stat, 0, 10);
    if (rc) return rc;
    const uint64_t* r2 = nullptr;
    if (c->pred_on && c->pred_ready && (rc = pred_radii(c, g, K, &r2))) return rc;
    switch (K) {
        case 8: rc = knn_tiled<8>(c, g, k, out, r2, stat); break;
        case 16: rc = knn_tiled<16>(c, g, k, out, r2, stat); break;
        case 24: rc = knn_tiled<24>(c, g, k, out, r2, stat); break;
        case 32: rc = knn_tiled<32>(c, g, k, out, r2, stat); break;
        default: return PDD_EINVAL;
    }
    if (rc) return rc;
    // counters: points tested, predicted balls that certified, that did
    // not, tile points that fell back to the wave search
    unsigned long long* h = (unsigned long long*)c->pinned;
    PDD_HIP(c, hipMemcpyAsync(h, stat, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    c->stats[8] = (int64_t)h[0];
    c->stats[9] = (int64_t)h[1];
    c->stats[10] = (int64_t)h[2];
    c->stats[11] = (int64_t)h[3];
    if (fallbacks) *fallbacks = (int64_t)h[3];
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
