// Exact k-nearest-neighbour search over the voxel grid (device code).
//
// Sec. 5 searches a point's neighbourhood in its voxel and the 26 adjacent
// ones.  That is exact only while the k-th neighbour is closer than the
// nearest face of the searched block, so the search here grows the block
// one shell of cells at a time and stops once the k-th distance is certified
// (no unsearched point can be nearer), or the block covers the whole grid.
#pragma once

#include "common.h"

namespace pdd {

// Top-K by squared distance, ascending, in registers.  A candidate at the
// same distance as the current K-th is not inserted: among equal distances
// the first one seen stays, which leaves the multiset of distances exact.
template <int K>
struct TopK {
    uint64_t d[K];
    int32_t id[K];

    __device__ inline void init() {
#pragma unroll
        for (int j = 0; j < K; j++) {
            d[j] = ~0ull;
            id[j] = -1;
        }
    }

    __device__ inline void push(uint64_t dd, int32_t ii) {
        if (dd >= d[K - 1]) return;
#pragma unroll
        for (int j = K - 1; j > 0; --j) {
            if (dd < d[j - 1]) {
                d[j] = d[j - 1];
                id[j] = id[j - 1];
            } else if (dd < d[j]) {
                d[j] = dd;
                id[j] = ii;
            }
        }
        if (dd < d[0]) {
            d[0] = dd;
            id[0] = ii;
        }
    }

    __device__ inline int count() const {
        int c = 0;
#pragma unroll
        for (int j = 0; j < K; j++) c += d[j] != ~0ull;
        return c;
    }
};

// Which points a search may return besides excluding the query itself.
enum SearchMode { kAll = 0, kAlive = 1, kAliveNotA = 2 };

struct SearchCtx {
    const uint8_t* alive;   // [n] 1 = alive (modes kAlive, kAliveNotA)
    const uint32_t* inA;    // [n] round stamp of the current threshold set (kAliveNotA)
    uint32_t round;
};

// Squared distance from relative coordinate u (cell cu) to the nearest point
// outside the cell block [cu - r, cu + r] along one axis; ~0 if no cell exists
// beyond that face on either side.
__device__ inline uint64_t face_gap2(int u, int cu, int r, int s, int cmax) {
    uint64_t g = ~0ull;
    if (cu - r - 1 >= 0) {
        uint64_t lo = (uint64_t)(u - ((cu - r) << s) + 1);
        g = lo * lo;
    }
    if (cu + r + 1 <= cmax) {
        uint64_t hi = (uint64_t)(((cu + r + 1) << s) - u);
        uint64_t h2 = hi * hi;
        if (h2 < g) g = h2;
    }
    return g;
}

template <int K, int MODE>
__device__ inline void scan_cell(const GridView& g, const LevelView& lv, uint32_t c, uint32_t q, int qx, int qy,
                                 int qz, const SearchCtx& sc, TopK<K>& t) {
    const uint32_t b = lv.start[c], e = lv.start[c + 1];
    for (uint32_t j = b; j < e; j++) {
        if (j == q) continue;
        if (MODE != kAll) {
            if (!sc.alive[j]) continue;
            if (MODE == kAliveNotA && sc.inA[j] == sc.round) continue;
        }
        int4 p = g.pts[j];
        t.push(dist2(qx, qy, qz, p.x, p.y, p.z), (int32_t)j);
    }
}

template <int K, int MODE>
__device__ inline void scan_cell_at(const GridView& g, const LevelView& lv, int x, int y, int z, uint32_t q, int qx,
                                    int qy, int qz, const SearchCtx& sc, TopK<K>& t) {
    uint32_t c = hash_find(lv.hkeys, lv.hvals, lv.hmask, morton3((uint32_t)x, (uint32_t)y, (uint32_t)z));
    if (c != kNone) scan_cell<K, MODE>(g, lv, c, q, qx, qy, qz, sc, t);
}

// Grows shells of cells around the query at the finest level, at most two
// shells per level before moving one level up (edge x8, search restarted),
// until entry kcert-1 is certified (no unsearched point can be nearer) or
// the block covers the grid.  Returns the level that ended the search.
template <int K, int MODE>
__device__ int ring_search(const GridView& g, uint32_t q, int4 qp, const SearchCtx& sc, TopK<K>& t, int kcert) {
    const int ux = qp.x - g.minx, uy = qp.y - g.miny, uz = qp.z - g.minz;
    for (int L = 0; L < g.nlev; L++) {
        const LevelView& lv = g.lv[L];
        const int s = lv.s;
        const int cx = ux >> s, cy = uy >> s, cz = uz >> s;
        const int rmax = (L == g.nlev - 1) ? (1 << 22) : 2;
        if (L > 0) t.init();
        for (int r = 0; r <= rmax; r++) {
            if (r == 0) {
                scan_cell_at<K, MODE>(g, lv, cx, cy, cz, q, qp.x, qp.y, qp.z, sc, t);
            } else {
                const int z0 = max(cz - r, 0), z1 = min(cz + r, lv.cmax[2]);
                const int y0 = max(cy - r, 0), y1 = min(cy + r, lv.cmax[1]);
                const int x0 = max(cx - r, 0), x1 = min(cx + r, lv.cmax[0]);
                for (int z = z0; z <= z1; z++) {
                    const bool zface = (z == cz - r) || (z == cz + r);
                    for (int y = y0; y <= y1; y++) {
                        const bool yface = (y == cy - r) || (y == cy + r);
                        if (zface || yface) {
                            for (int x = x0; x <= x1; x++)
                                scan_cell_at<K, MODE>(g, lv, x, y, z, q, qp.x, qp.y, qp.z, sc, t);
                        } else {
                            if (cx - r >= 0) scan_cell_at<K, MODE>(g, lv, cx - r, y, z, q, qp.x, qp.y, qp.z, sc, t);
                            if (cx + r <= lv.cmax[0])
                                scan_cell_at<K, MODE>(g, lv, cx + r, y, z, q, qp.x, qp.y, qp.z, sc, t);
                        }
                    }
                }
            }
            uint64_t g2 = face_gap2(ux, cx, r, s, lv.cmax[0]);
            uint64_t gy = face_gap2(uy, cy, r, s, lv.cmax[1]);
            uint64_t gz = face_gap2(uz, cz, r, s, lv.cmax[2]);
            if (gy < g2) g2 = gy;
            if (gz < g2) g2 = gz;
            if (g2 == ~0ull) return L;  // the block covers the grid
            if (t.d[kcert - 1] != ~0ull && t.d[kcert - 1] <= g2) return L;
        }
    }
    return g.nlev;  // not reached: the top level's block grows until it covers the grid
}

// ---------------------------------------------------------------------------
// One wavefront per query.  The 64 lanes look up the cells of a shell at
// once, pack the points of the found cells into chunks of 64 (a wave prefix
// sum over the cell sizes, then a binary search per lane), and test one
// point each.  The top-K list is spread over the lanes (lane j holds the
// j-th nearest); a candidate below the K-th distance is inserted with one
// ballot (its rank) and one lane shift.  Same levels, shells and
// certification as ring_search, same tie rule as TopK.
// ---------------------------------------------------------------------------

__device__ inline uint64_t readlane64(uint64_t v, int l) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t shfl_up64(uint64_t v) {
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, 1, kWave);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), 1, kWave);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// lds_start / lds_excl: 64 entries of wave-private LDS each.  On return lane
// j < K holds the j-th nearest (my_d = ~0 past the end).
template <int K, int MODE>
__device__ void wave_knn(const GridView& g, uint32_t q, int4 qp, const SearchCtx& sc, int kcert, uint64_t& my_d,
                         int32_t& my_id, uint32_t* lds_start, uint32_t* lds_excl) {
    const int lane = (int)lane_id();
    const int ux = qp.x - g.minx, uy = qp.y - g.miny, uz = qp.z - g.minz;
    my_d = ~0ull;
    my_id = -1;
    for (int L = 0; L < g.nlev; L++) {
        const LevelView& lv = g.lv[L];
        const int s = lv.s;
        const int cx = ux >> s, cy = uy >> s, cz = uz >> s;
        const int rmax = (L == g.nlev - 1) ? (1 << 22) : 2;
        if (L > 0) {
            my_d = ~0ull;
            my_id = -1;
        }
        for (int r = 0; r <= rmax; r++) {
            const int side = 2 * r + 1;
            const int ncube = side * side * side;
            for (int base = 0; base < ncube; base += kWave) {
                const int idx = base + lane;
                uint32_t st = 0, cnt = 0;
                if (idx < ncube) {
                    const int dz = idx / (side * side) - r;
                    const int rem = idx % (side * side);
                    const int dy = rem / side - r, dx = rem % side - r;
                    const int m = max(abs(dx), max(abs(dy), abs(dz)));
                    const int x = cx + dx, y = cy + dy, z = cz + dz;
                    if (m == r && x >= 0 && y >= 0 && z >= 0 && x <= lv.cmax[0] && y <= lv.cmax[1] &&
                        z <= lv.cmax[2]) {
                        const uint32_t c =
                            hash_find(lv.hkeys, lv.hvals, lv.hmask, morton3((uint32_t)x, (uint32_t)y, (uint32_t)z));
                        if (c != kNone) {
                            st = lv.start[c];
                            cnt = lv.start[c + 1] - st;
                        }
                    }
                }
                uint32_t incl = cnt;
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) {
                    const uint32_t v = (uint32_t)__shfl_up((int)incl, o, kWave);
                    if (lane >= o) incl += v;
                }
                const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
                if (total == 0) continue;
                lds_start[lane] = st;
                lds_excl[lane] = incl - cnt;
                wave_sync_lds();
                for (uint32_t t0 = 0; t0 < total; t0 += kWave) {
                    const uint32_t t = t0 + (uint32_t)lane;
                    uint64_t d = ~0ull;
                    uint32_t j = 0;
                    if (t < total) {
                        int l = 0;
#pragma unroll
                        for (int step = 32; step > 0; step >>= 1)
                            if (lds_excl[l + step] <= t) l += step;
                        j = lds_start[l] + (t - lds_excl[l]);
                        bool ok = j != q;
                        if (MODE != kAll && ok) {
                            ok = sc.alive[j] != 0;
                            if (MODE == kAliveNotA && ok) ok = sc.inA[j] != sc.round;
                        }
                        if (ok) {
                            const int4 p = g.pts[j];
                            d = dist2(qp.x, qp.y, qp.z, p.x, p.y, p.z);
                        }
                    }
                    uint64_t thr = readlane64(my_d, K - 1);
                    uint64_t m = __ballot(d < thr);
                    while (m) {
                        const int l2 = __ffsll((unsigned long long)m) - 1;
                        m &= m - 1;
                        const uint64_t dv = readlane64(d, l2);
                        const int32_t iv = __builtin_amdgcn_readlane((int)j, l2);
                        const int p = __popcll(__ballot(lane < K && my_d <= dv));
                        if (p < K) {
                            const uint64_t upd = shfl_up64(my_d);
                            const int32_t upi = __shfl_up(my_id, 1, kWave);
                            if (lane == p) {
                                my_d = dv;
                                my_id = iv;
                            } else if (lane > p && lane < K) {
                                my_d = upd;
                                my_id = upi;
                            }
                            thr = readlane64(my_d, K - 1);
                            m &= __ballot(d < thr);
                        }
                    }
                }
                wave_sync_lds();
            }
            uint64_t g2 = face_gap2(ux, cx, r, s, lv.cmax[0]);
            const uint64_t gy = face_gap2(uy, cy, r, s, lv.cmax[1]);
            const uint64_t gz = face_gap2(uz, cz, r, s, lv.cmax[2]);
            if (gy < g2) g2 = gy;
            if (gz < g2) g2 = gz;
            if (g2 == ~0ull) return;
            const uint64_t kth = readlane64(my_d, kcert - 1);
            if (kth != ~0ull && kth <= g2) return;
        }
    }
}

// Sum over lanes of v (wave-uniform result).
__device__ inline uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o, kWave);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o, kWave);
        v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

// Cost of a sorted neighbour list: sum of cost_term over its first `use` entries.
template <int K>
__device__ inline uint64_t list_cost(const TopK<K>& t, int use) {
    uint64_t w = 0;
#pragma unroll
    for (int j = 0; j < K; j++)
        if (j < use) w += cost_term(t.d[j]);
    return w;
}

}  // namespace pdd
