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

// Which points a search may return besides excluding the query itself.
//   kAll    every point; the grid's points are the sorted points and a
//           point's id is its position
//   kAlive  alive points; the grid view holds a compacted copy of the points
//           that were alive when it was built (same cells, same Morton
//           order), each with its sorted position in .w, set to -1 when the
//           point is removed
enum SearchMode { kAll = 0, kAlive = 1 };

struct SearchCtx {
    const uint8_t* alive;   // [n] 1 = alive (mode kAlive)
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

// Anchor cell of sorted point j: the finest level L whose cell c around j
// holds at least `need` points (alive points when alive_cnt, indexed by
// level base + cell, is given), or the top level.
__device__ inline void anchor_cell(const GridView& g, uint32_t j, uint32_t need, const uint32_t* alive_cnt, int* Lout,
                                   uint32_t* cout) {
    uint32_t c = g.of0[j];
    int L = 0;
    for (;;) {
        const LevelView& lv = g.lv[L];
        const uint32_t cnt = alive_cnt ? alive_cnt[lv.base + c] : lv.start[c + 1] - lv.start[c];
        if (cnt >= need || L + 1 >= g.nlev) break;
        c = lv.parent[c];
        L++;
    }
    *Lout = L;
    *cout = c;
}

// ---------------------------------------------------------------------------
// One wavefront per query.  The search starts at level L0 and grows the
// block of cells around the query one shell at a time: shells 0 and 1 at
// each level, then one level up (edge x2), whose 3x3x3 block contains the
// previous one; points of the previous block are skipped there, so every
// point is tested once.  It stops once entry kcert-1 is certified (every
// point not yet tested lies at least that far) or the block covers the grid;
// at the top level the shells keep growing.
//
// Per shell, the 64 lanes look up its cells at once, pack the points of the
// found cells into chunks of 64 (a wave prefix sum over the cell sizes, then
// a binary search per lane) and test one point each.  The list is spread
// over the lanes (lane j holds the j-th nearest); a candidate below the K-th
// distance is inserted with one ballot (its rank) and one lane shift.  A
// candidate at the same distance as the current K-th is not inserted: among
// equal distances the first one seen stays, which leaves the multiset of
// distances exact.
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

__device__ inline uint64_t shfl_xor64(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, kWave);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t shfl64(uint64_t v, int l) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, l, kWave);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), l, kWave);
    return ((uint64_t)hi << 32) | lo;
}

// More candidates than this below the K-th distance in one batch are merged
// into the list at once (wave_merge) instead of one by one.
constexpr int kBulkInsert = 8;

// Merges one candidate per lane (distance cd, ~0 for none, id cj) into the
// wave's sorted list (lane j < K holds the j-th nearest, ~0 past the end):
// a bitonic sort of the 64 candidates across the lanes, the elementwise
// minimum of the list and the reversed candidates (the 64 smallest of both,
// a bitonic sequence), then a bitonic merge.  Among equal distances the
// choice is arbitrary, which leaves the list exact as a multiset.
template <int K>
__device__ inline void wave_merge(uint64_t cd, int32_t cj, uint64_t& my_d, int32_t& my_id) {
    const int lane = (int)lane_id();
#pragma unroll
    for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
        for (int stride = size / 2; stride > 0; stride >>= 1) {
            const uint64_t od = shfl_xor64(cd, stride);
            const int32_t oj = __shfl_xor(cj, stride, kWave);
            const bool up = (lane & size) == 0 || size == kWave;
            const bool lower = (lane & stride) == 0;
            const bool take = (lower == up) ? od < cd : od > cd;
            if (take) {
                cd = od;
                cj = oj;
            }
        }
    }
    const uint64_t rd = shfl64(cd, kWave - 1 - lane);
    const int32_t rj = __shfl(cj, kWave - 1 - lane, kWave);
    if (rd < my_d) {
        my_d = rd;
        my_id = rj;
    }
#pragma unroll
    for (int stride = kWave / 2; stride > 0; stride >>= 1) {
        const uint64_t od = shfl_xor64(my_d, stride);
        const int32_t oj = __shfl_xor(my_id, stride, kWave);
        const bool lower = (lane & stride) == 0;
        const bool take = lower ? od < my_d : od > my_d;
        if (take) {
            my_d = od;
            my_id = oj;
        }
    }
    if (lane >= K) {
        my_d = ~0ull;
        my_id = -1;
    }
}

__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tests the points of up to 64 cells, one cell range [st, st + cnt) per lane,
// against the wave's top-K list (lane j < K holds the j-th nearest).  Points
// inside the previous level's block (skip; cell coordinates at shift ps
// within 1 of (px, py, pz)) were tested already and are passed over.
// Returns the number of points looked at (wave-uniform).
template <int K, int MODE>
__device__ inline uint32_t wave_scan(const GridView& g, uint32_t q, int4 qp, const SearchCtx& sc, uint32_t st,
                                     uint32_t cnt, bool skip, int ps, int px, int py, int pz, uint64_t& my_d,
                                     int32_t& my_id, uint32_t* lds_start, uint32_t* lds_excl) {
    const int lane = (int)lane_id();
    uint32_t incl = cnt;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)incl, o, kWave);
        if (lane >= o) incl += v;
    }
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    if (total == 0) return 0;
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
            const uint32_t pos = lds_start[l] + (t - lds_excl[l]);
            const int4 p = g.pts[pos];
            j = MODE == kAll ? pos : (uint32_t)p.w;
            bool ok = j != q;
            if (MODE != kAll && ok) ok = p.w >= 0;
            if (ok && skip && abs(((p.x - g.minx) >> ps) - px) <= 1 && abs(((p.y - g.miny) >> ps) - py) <= 1 &&
                abs(((p.z - g.minz) >> ps) - pz) <= 1)
                ok = false;
            if (ok) d = dist2(qp.x, qp.y, qp.z, p.x, p.y, p.z);
        }
        uint64_t thr = readlane64(my_d, K - 1);
        uint64_t m = __ballot(d < thr);
        if (__popcll(m) > kBulkInsert) {
            wave_merge<K>(d < thr ? d : ~0ull, (int32_t)j, my_d, my_id);
            m = 0;
        }
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
    return total;
}

// lds_start / lds_excl: 64 entries of wave-private LDS each.  On return lane
// j < K holds the j-th nearest (my_d = ~0 past the end).  *tested (if not
// null) is increased by the number of points looked at.
template <int K, int MODE>
__device__ void wave_knn(const GridView& g, uint32_t q, int4 qp, const SearchCtx& sc, int kcert, int L0,
                         uint64_t& my_d, int32_t& my_id, uint32_t* lds_start, uint32_t* lds_excl,
                         uint32_t* tested = nullptr) {
    const int lane = (int)lane_id();
    const int ux = qp.x - g.minx, uy = qp.y - g.miny, uz = qp.z - g.minz;
    const uint32_t qs = seg_at(g, q);
    my_d = ~0ull;
    my_id = -1;
    uint64_t cert = 0;  // squared radius around the query within which every point was tested
    for (int L = L0; L < g.nlev; L++) {
        const LevelView& lv = g.lv[L];
        const int s = lv.s;
        const int cx = ux >> s, cy = uy >> s, cz = uz >> s;
        const int rmax = (L == g.nlev - 1) ? (1 << 22) : 1;
        // below the top level the 3x3x3 block is scanned in one pass (the
        // centre cell alone almost never certifies k neighbours)
        const bool whole = rmax == 1;
        // the previous level's block, already tested
        const bool skip = L > L0;
        const int ps = s - 1, px = ux >> ps, py = uy >> ps, pz = uz >> ps;
        for (int r = whole ? 1 : 0; r <= rmax; r++) {
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
                    if ((m == r || whole) && x >= 0 && y >= 0 && z >= 0 && x <= lv.cmax[0] && y <= lv.cmax[1] &&
                        z <= lv.cmax[2]) {
                        const uint32_t c = hash_find(lv.hkeys, lv.hvals, lv.hmask, cell_code(lv, qs, x, y, z));
                        if (c != kNone) {
                            st = lv.start[c];
                            cnt = lv.start[c + 1] - st;
                        }
                    }
                }
                const uint32_t n = wave_scan<K, MODE>(g, q, qp, sc, st, cnt, skip, ps, px, py, pz, my_d, my_id,
                                                      lds_start, lds_excl);
                if (tested) *tested += n;
            }
            uint64_t g2 = face_gap2(ux, cx, r, s, lv.cmax[0]);
            const uint64_t gy = face_gap2(uy, cy, r, s, lv.cmax[1]);
            const uint64_t gz = face_gap2(uz, cz, r, s, lv.cmax[2]);
            if (gy < g2) g2 = gy;
            if (gz < g2) g2 = gz;
            if (g2 == ~0ull) return;
            if (g2 > cert) cert = g2;
            const uint64_t kth = readlane64(my_d, kcert - 1);
            if (kth != ~0ull && kth <= cert) return;
        }
    }
}

// Distance along one axis from coordinate u to the cell [c << s, (c+1) << s).
__device__ inline uint64_t cell_gap(int u, int c, int s) {
    const int lo = c << s, hi = ((c + 1) << s) - 1;
    return (uint64_t)(u < lo ? lo - u : (u > hi ? u - hi : 0));
}

// Search bounded by a predicted ball: tests every point of the cells (at the
// finest level whose edge is at least half the radius) that meet the ball of
// squared radius r2 around the query.  True when the result is certified: the
// kcert-th distance is within r2, so no untested point (all beyond r2) can be
// nearer.  Otherwise the caller falls back to wave_knn.
template <int K, int MODE>
__device__ bool wave_knn_ball(const GridView& g, uint32_t q, int4 qp, const SearchCtx& sc, int kcert, uint64_t r2,
                              uint64_t& my_d, int32_t& my_id, uint32_t* lds_start, uint32_t* lds_excl,
                              uint32_t* tested = nullptr) {
    const int lane = (int)lane_id();
    const int ux = qp.x - g.minx, uy = qp.y - g.miny, uz = qp.z - g.minz;
    const uint32_t qs = seg_at(g, q);
    my_d = ~0ull;
    my_id = -1;
    const int ri = (int)sqrt((double)r2) + 1;
    int L = 0;
    while (L + 1 < g.nlev && (2 << g.lv[L].s) < ri) L++;
    const LevelView& lv = g.lv[L];
    const int s = lv.s;
    const int x0 = max((ux - ri) >> s, 0), x1 = min((ux + ri) >> s, lv.cmax[0]);
    const int y0 = max((uy - ri) >> s, 0), y1 = min((uy + ri) >> s, lv.cmax[1]);
    const int z0 = max((uz - ri) >> s, 0), z1 = min((uz + ri) >> s, lv.cmax[2]);
    const int nx = x1 - x0 + 1, ny = y1 - y0 + 1, nz = z1 - z0 + 1;
    const int nbox = nx * ny * nz;
    for (int base = 0; base < nbox; base += kWave) {
        const int idx = base + lane;
        uint32_t st = 0, cnt = 0;
        if (idx < nbox) {
            const int x = x0 + idx % nx, y = y0 + (idx / nx) % ny, z = z0 + idx / (nx * ny);
            const uint64_t gx = cell_gap(ux, x, s), gy = cell_gap(uy, y, s), gz = cell_gap(uz, z, s);
            if (gx * gx + gy * gy + gz * gz <= r2) {
                const uint32_t c = hash_find(lv.hkeys, lv.hvals, lv.hmask, cell_code(lv, qs, x, y, z));
                if (c != kNone) {
                    st = lv.start[c];
                    cnt = lv.start[c + 1] - st;
                }
            }
        }
        const uint32_t n =
            wave_scan<K, MODE>(g, q, qp, sc, st, cnt, false, 0, 0, 0, 0, my_d, my_id, lds_start, lds_excl);
        if (tested) *tested += n;
    }
    const uint64_t kth = readlane64(my_d, kcert - 1);
    return kth != ~0ull && kth <= r2;
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

}  // namespace pdd
