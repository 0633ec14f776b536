// Which points of A are removed this round (the conditions are stated at the
// top of rounds.hip).  The kernels here give one wavefront (rb_pair: half
// a wavefront) to one point.
#include "rounds.h"

namespace pdd {

namespace {

// y in A: its list entries, one per lane of a half wavefront (two points of
// A per wavefront; lane j < K of a half holds entry j).
//  - blocks y when an entry of H(y) is nearer than rho'(y);
//  - blocks every lower A entry x with fewer than k alive entries not in
//    H(x) (other than x) within d(x, y) of y, or whose distance the list
//    does not cover;
//  - puts y on the danger list (with threshold key and list radius) when
//    its list is full and holds fewer than k entries outside A.
template <int K>
__global__ void __launch_bounds__(kBlock) rb_pair(RoundArrays a) {
    static_assert(K <= kWave / 2, "a list fits half a wavefront");
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    constexpr int W = kBlock / kWave, H = kWave / 2;
    __shared__ int s_cls[W][kWave];
    __shared__ uint64_t s_d[W][kWave], s_c[W][kWave];
    __shared__ int32_t s_o[W][kWave];
    const uint32_t nA = st->nA, round = st->round;
    const int k = a.k;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int half = lane / H, sub = lane % H, hb = half * H;
    const uint64_t hmask = 0xFFFFFFFFull << hb;
    // the half's bits of a ballot, as entry bits
    auto hballot = [&](bool p) { return (uint32_t)((__ballot(p) & hmask) >> hb); };
    const uint32_t below_sub = (1u << sub) - 1u;
    const uint32_t nw = gridDim.x * W;
    uint32_t ndanger = 0;  // danger entries of this half (kept by its first lane)
    for (uint32_t t0 = (blockIdx.x * W + w) * 2; t0 < nA; t0 += nw * 2) {
        const uint32_t t = t0 + (uint32_t)half;
        const bool act = t < nA;
        uint32_t y = 0;
        int4 py = make_int4(0, 0, 0, 0);
        uint64_t cy = 0;
        int c = 0;
        if (act) {
            y = a.A[t];
            py = a.pts[y];
            cy = a.cost[y];
            c = a.cnt[y];
        }
        const int32_t oy = py.w;
        int cls = 0;
        uint64_t d = ~0ull, draw = 0, cj = 0;
        int32_t oj = 0;
        uint32_t z = 0;
        if (sub < c) {
            z = (uint32_t)a.nbr[(size_t)y * K + sub];
            const int4 pz = a.pts[z];
            draw = dist2(py.x, py.y, py.z, pz.x, pz.y, pz.z);
            if (a.alive[z]) {
                d = draw;
                if (a.inA[z] == round) {
                    cls = 2;
                    cj = a.cost[z];
                    oj = pz.w;
                } else {
                    cls = 1;
                }
            }
        }
        // cross-lane reads are made by every lane, outside the branches
        const uint64_t dl = shfl64(draw, hb + (c > 0 ? c - 1 : 0));
        const uint64_t dlast = c > 0 ? dl : 0ull;
        const bool complete = c < K;
        const bool higher = cls == 2 && key_above(cj, oj, cy, oy);
        const bool low = cls != 0 && !higher;
        const uint32_t lowm = hballot(low), highm = hballot(higher);
        const uint32_t km = hballot(low && __popc(lowm & below_sub) == k - 1);
        const uint64_t rho = shfl64(d, hb + (km ? __ffs(km) - 1 : 0));
        const uint64_t dhigh = shfl64(d, hb + (highm ? __ffs(highm) - 1 : 0));
        // y itself
        bool blocked_self;
        if (__popc(lowm) >= k) blocked_self = highm && dhigh < rho;
        else blocked_self = complete ? highm != 0 : true;
        if (act && sub == 0 && blocked_self) a.blocked[y] = round;
        // rank counts over the other entries of the half (entries from LDS)
        s_cls[w][lane] = cls;
        s_d[w][lane] = d;
        s_c[w][lane] = cj;
        s_o[w][lane] = oj;
        wave_sync_lds();
        int q = 0, rankA = 0;
        for (int i = 0; i < K; i++) {
            const int ci = s_cls[w][hb + i];
            if (ci == 0) continue;
            const uint64_t di = s_d[w][hb + i];
            const uint64_t ki = s_c[w][hb + i];
            const int32_t oi = s_o[w][hb + i];
            if (i != sub && di <= d && (ci == 1 || key_above(cj, oj, ki, oi))) q++;
            if (ci == 2 && i != sub && key_above(cj, oj, ki, oi)) rankA++;
        }
        const bool lower = cls == 2 && !higher;
        const bool covered = complete || d < dlast;
        if (lower && (q < k || !covered)) a.blocked[z] = round;
        // lower points beyond the list
        const int nL = __popc(hballot(cls == 1)), nAe = __popc(hballot(cls == 2));
        const int need = k - nL;
        const uint32_t mm = hballot(cls == 2 && rankA == need - 1);
        const int ml = hb + (mm ? __ffs(mm) - 1 : 0);
        const uint64_t tcm = shfl64(cj, ml);
        const int32_t tom = __shfl(oj, ml, kWave);
        const bool danger = act && !complete && nL < k;
        if (act && sub == 0) {
            if (!danger) {
                a.dg_y[t] = kNone;
            } else {
                ndanger++;
                // the need-th lowest key among the alive A entries, else y's
                const bool from_list = nAe >= need;
                // the danger entry sits at y's position in A (no shared counter)
                a.dg_y[t] = y;
                a.dg_tc[t] = from_list ? tcm : cy;
                a.dg_to[t] = from_list ? tom : oy;
                a.dg_dlast[t] = dlast;
            }
        }
        wave_sync_lds();
    }
    const uint32_t nd = (uint32_t)__builtin_amdgcn_readlane((int)ndanger, 0) +
                        (uint32_t)__builtin_amdgcn_readlane((int)ndanger, H);
    if (lane == 0 && nd) atomicAdd(&st->nDanger, nd);
}

// x in A with at least k alive points of identical coordinates ranked below
// it (same cost, larger original index) is removed this round whatever
// happens around it: those points keep rho'(x) = 0 and rho(x | y) <= d2(x, y)
// for every y.  Marks such x in gsafe.
__global__ void __launch_bounds__(kBlock) rb_group(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t nA = st->nA, round = st->round;
    const uint32_t k = (uint32_t)a.k;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nA; t += gridDim.x * blockDim.x) {
        const uint32_t x = a.A[t];
        const uint32_t lo = a.grp_lo[x], hi = a.grp_hi[x];
        if (hi - lo <= k) continue;
        const int32_t ox = a.pts[x].w;
        uint32_t below = 0;
        for (uint32_t z = lo; z < hi && below < k; z++)
            if (z != x && a.alive[z] && a.pts[z].w > ox) below++;
        if (below >= k) a.gsafe[x] = round;
    }
}

__global__ void __launch_bounds__(kBlock) rb_survive(RoundArrays a, GridView g) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t nA = st->nA, round = st->round;
    const uint32_t n_it = (nA + blockDim.x - 1) / blockDim.x * blockDim.x;
    uint64_t smin[kLev];
#pragma unroll
    for (int j = 0; j < kLev; j++) smin[j] = ~0ull;
    uint32_t top_seg = kNone;
    uint64_t top_cost = 0;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_it; t += gridDim.x * blockDim.x) {
        bool sv = false;
        uint32_t x = 0;
        uint64_t cmax = 0;
        int lev = 0;
        const bool act = t < nA;
        if (act) {
            x = a.A[t];
            cmax = a.cost[x];
            lev = level_of(st, cmax);
        }
        // A counts of x's cells at every level; where the whole wave's A
        // points share a cell (coarse levels: A arrives in index order, so
        // a wave's points are neighbours) one lane adds the wave's counts
        {
            uint32_t c = act ? a.of0[x] : 0u;
            const uint64_t am = __ballot(act);
            const int leader = am ? __ffsll((unsigned long long)am) - 1 : 0;
            for (int L = 0; L < a.lc && am; L++) {
                const uint32_t gc = g.lv[L].base + c;
                const uint32_t g0 = (uint32_t)__shfl((int)gc, leader, kWave);
                if (__all(!act || gc == g0)) {
#pragma unroll
                    for (int j = 0; j < kLev; j++) {
                        const uint32_t cnt = (uint32_t)__popcll(__ballot(act && lev == j));
                        if ((int)(threadIdx.x & (kWave - 1)) == leader && cnt)
                            atomicAdd(&a.cellAlev[(size_t)g0 * kLev + j], cnt);
                    }
                } else if (act) {
                    atomicAdd(&a.cellAlev[(size_t)gc * kLev + lev], 1u);
                }
                if (act && L + 1 < a.lc) c = g.lv[L].parent[c];
            }
        }
        if (act) {
            if (a.blocked[x] != round && a.gsafe[x] != round) {
                sv = true;
                a.surv[x] = round;
                atomicOr(&a.sbits[x >> 6], 1ull << (x & 63u));
            }
        }
        // the block's survivors: one shared-counter atomic per block
        // (the loop bound is uniform over the block)
        const uint32_t p = block_reserve(&st->nSurv, sv ? 1u : 0u);
        if (sv) a.surv_list[p] = x;
        // lowest survivor cost per key level, kept per thread
#pragma unroll
        for (int j = 0; j < kLev; j++)
            if (sv && lev == j && cmax < smin[j]) smin[j] = cmax;
        // highest cost of each segment's A: kept per thread while the
        // thread's points share one segment
        if (act && cmax) {
            const uint32_t sx = seg_of_pt(a, x);
            if (top_seg == kNone || top_seg == sx) {
                top_seg = sx;
                if (cmax > top_cost) top_cost = cmax;
            } else {
                atomicMax((unsigned long long*)&a.seg_top_cost[sx], (unsigned long long)cmax);
            }
        }
    }
    // block minima / maxima: one atomic per block (and level)
    __shared__ unsigned long long s_min[kLev];
    if (threadIdx.x < kLev) s_min[threadIdx.x] = ~0ull;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kLev; j++)
        if (smin[j] != ~0ull) atomicMin(&s_min[j], (unsigned long long)smin[j]);
    block_seg_max64(a.seg_top_cost, top_seg, top_cost);
    if (threadIdx.x < kLev && s_min[threadIdx.x] != ~0ull)
        atomicMin((unsigned long long*)&st->surv_min[threadIdx.x], s_min[threadIdx.x]);
}

// Puts every survivor's record (point, cost, index) at its rank among the
// survivors by sorted index, so that the survivors of any cell of any level
// (a run of sorted indices) are one run of surv_rec.
// Survivors per 64-point word of the survivor bits (0 past the last word).
__global__ void __launch_bounds__(kBlock) rb_wcount(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w <= a.nwords; w += gridDim.x * blockDim.x)
        a.swcnt[w] = w < a.nwords ? (uint32_t)__popcll(a.sbits[w]) : 0u;
}

__global__ void __launch_bounds__(kBlock) rb_bucket(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t ns = st->nSurv;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < ns; t += gridDim.x * blockDim.x) {
        const uint32_t x = a.surv_list[t];
        const uint32_t pos = surv_rank(a, x);
        if (pos < a.rec_cap) {
            SurvRec r;
            r.p = a.pts[x];
            r.cost = a.cost[x];
            r.x = x;
            r.pad = 0;
            a.surv_rec[pos] = r;
        } else {
            st->err = 8;
        }
    }
    // the highest key of each segment's A survives every condition; find
    // its index
    const uint32_t nA = st->nA;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nA; t += gridDim.x * blockDim.x) {
        const uint32_t x = a.A[t];
        const uint32_t sx = seg_of_pt(a, x);
        if (a.cost[x] == a.seg_top_cost[sx]) atomicMin(&a.seg_top_orig[sx], a.pts[x].w);
    }
}

// Largest squared distance from relative coordinate u to an integer point of
// cells [c - r, c + r] (edge 2^s) along one axis.
__device__ inline uint64_t block_reach2(int u, int c, int r, int s) {
    const int lo = (c - r) << s, hi = ((c + r + 1) << s) - 1;
    const uint64_t m = (uint64_t)max(u - lo, hi - u);
    return m * m;
}

// For each key level j in `want`, an upper bound R2[j] on the squared
// distance from y (relative coordinates u) to its k-th nearest alive point
// ranked below level j (outside A, or in A at a lower level): the reach of
// the first block, over shells 0 and 1 of the levels from L1 up, whose cells
// hold k such points by the per-cell counts.  0 where even the top block
// (the whole cloud) holds fewer.
__device__ void level_bounds(const GridView& g, const RoundArrays& a, uint32_t ys, int ux, int uy, int uz, int L1,
                             uint32_t want, int k, uint64_t* R2) {
    const int lane = (int)lane_id();
#pragma unroll
    for (int j = 0; j < kLev; j++) R2[j] = 0;
    for (int L = L1; L < g.nlev && want; L++) {
        const LevelView& lv = g.lv[L];
        const int s = lv.s;
        const int cx = ux >> s, cy = uy >> s, cz = uz >> s;
        uint32_t b1[kLev];
#pragma unroll
        for (int j = 0; j < kLev; j++) b1[j] = 0;
        if (lane < 27) {
            const int x = cx + lane % 3 - 1, y = cy + (lane / 3) % 3 - 1, z = cz + lane / 9 - 1;
            if (x >= 0 && y >= 0 && z >= 0 && x <= lv.cmax[0] && y <= lv.cmax[1] && z <= lv.cmax[2]) {
                const uint32_t c = hash_find(lv.hkeys, lv.hvals, lv.hmask, cell_code(lv, ys, x, y, z));
                if (c != kNone) {
                    const size_t gc = lv.base + c;
                    uint32_t la[kLev], inA = 0;
#pragma unroll
                    for (int j = 0; j < kLev; j++) {
                        la[j] = a.cellAlev[gc * kLev + j];
                        inA += la[j];
                    }
                    uint32_t below = a.cell_alive[gc] - inA;
#pragma unroll
                    for (int j = 0; j < kLev; j++) {
                        b1[j] = below;
                        below += la[j];
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kLev; j++) {
            if (!((want >> j) & 1u)) continue;
            const uint32_t own = (uint32_t)__builtin_amdgcn_readlane((int)b1[j], 13);
            uint32_t v = b1[j];
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, kWave);
            if (own >= (uint32_t)k) {
                R2[j] = block_reach2(ux, cx, 0, s) + block_reach2(uy, cy, 0, s) + block_reach2(uz, cz, 0, s);
                want &= ~(1u << j);
            } else if (v >= (uint32_t)k) {
                R2[j] = block_reach2(ux, cx, 1, s) + block_reach2(uy, cy, 1, s) + block_reach2(uz, cz, 1, s);
                want &= ~(1u << j);
            }
        }
    }
}

// Distance along one axis from coordinate u to cell index c of size 2^s.
__device__ inline uint64_t axis_gap(int u, int c, int s) {
    const int lo = c << s, hi = ((c + 1) << s) - 1;
    return (uint64_t)(u < lo ? lo - u : (u > hi ? u - hi : 0));
}

// A dangerous y may hold a surviving lower x beyond its list within
// rho(x | y) only if key(x) <= its threshold.  For x of key level j,
// rho(x | y) is at most R_j (level_bounds).  Such an x stays unless a count
// of alive points not above x within d(x, y) of y reaches k: the entries of
// y's list not above x, plus entries of x's own list that lie beyond y's
// list radius and within d(x, y).  When no R_j is found, every survivor of
// level j at or below min(key(y), threshold) in y's segment waits (cost
// bound in seg_glob, applied at removal).
template <int K>
__global__ void __launch_bounds__(kBlock) rb_danger(RoundArrays a, GridView g) {
    RoundDev* st = a.st;
    if (st->done || st->err || st->nSurv == 0) return;
    constexpr int W = kBlock / kWave;
    __shared__ uint32_t s_start[W][kWave], s_excl[W][kWave];
    __shared__ uint64_t s_yc[W][K];
    __shared__ int32_t s_yo[W][K];
    __shared__ int s_ycls[W][K];
    // the danger entries are at their points' positions in A; kNone elsewhere
    const uint32_t nd = st->nA, round = st->round, ns = st->nSurv;
    const int k = a.k, Kb = a.K;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t nw = gridDim.x * W;
    uint32_t enumerated = 0;  // survivors this wave enumerated (wave-uniform)
    for (uint32_t t = blockIdx.x * W + w; t < nd; t += nw) {
        const uint32_t y = a.dg_y[t];
        if (y == kNone) continue;
        const uint64_t tc = a.dg_tc[t], dlast = a.dg_dlast[t];
        const int32_t to = a.dg_to[t];
        const uint64_t cy = a.cost[y];
        // key levels with a survivor that y could hold back: at or below
        // the threshold's level, with some survivor cost <= min(cost y, threshold)
        const int lth = level_of(st, tc);
        const uint64_t cmin = cy < tc ? cy : tc;
        uint32_t risk = 0;
#pragma unroll
        for (int j = 0; j < kLev; j++)
            if (j <= lth && st->surv_min[j] <= cmin) risk |= 1u << j;
        if (!risk) continue;
        const int4 py = a.pts[y];
        const int32_t oy = py.w;
        // y's list: class and key of every entry
        int lcls = 0, llev = kLev;
        if (lane < K) {
            uint64_t cc = 0;
            int32_t oo = 0;
            if (lane < a.cnt[y]) {
                const uint32_t z = (uint32_t)a.nbr[(size_t)y * Kb + lane];
                if (a.alive[z]) {
                    if (a.inA[z] == round) {
                        lcls = 2;
                        cc = a.cost[z];
                        oo = a.pts[z].w;
                        llev = level_of(st, cc);
                    } else {
                        lcls = 1;
                        llev = -1;
                    }
                }
            }
            s_ycls[w][lane] = lcls;
            s_yc[w][lane] = cc;
            s_yo[w][lane] = oo;
        }
        wave_sync_lds();
        // a level whose survivors have k entries of y's list ranked below
        // them (all within y's list radius) is safe
#pragma unroll
        for (int j = 0; j < kLev; j++)
            if (__popcll(__ballot(lcls != 0 && llev < j)) >= k) risk &= ~(1u << j);
        if (!risk) continue;
        const int ux = py.x - g.minx, uy = py.y - g.miny, uz = py.z - g.minz;
        const uint32_t ys = seg_at(g, y);
        // R2[j] (0 = none found) for the key levels at risk, from the finest
        // level whose 3x3x3 block can reach beyond y's list radius (the
        // list holds every alive point nearer than dlast, fewer than k of
        // them below a risky level)
        uint64_t R2[kLev];
        uint64_t rbox = 0;
        {
            int sneed = 0;
            while (sneed < 21 && (12ull << (2 * sneed)) < dlast) sneed++;
            const int L1 = min(max(sneed - g.lv[0].s, 0), g.nlev - 1);
            level_bounds(g, a, ys, ux, uy, uz, L1, risk, k, R2);
            const uint64_t cb = (cy < tc ? cy : tc) + 1;
#pragma unroll
            for (int j = 0; j < kLev; j++) {
                if (!((risk >> j) & 1u)) continue;
                if (R2[j] == 0) {
                    if (lane == 0) atomicMax((unsigned long long*)&a.seg_glob[ys * kLev + j], (unsigned long long)cb);
                } else if (R2[j] > rbox) {
                    rbox = R2[j];
                }
            }
        }
        // (gsafe points are not survivors; a survivor another check has
        // blocked already is passed over once it clears the filters)
        auto consider = [&](const SurvRec& r) {
            const uint32_t x = r.x;
            if (x == y) return;
            const uint64_t cx = r.cost;
            const int lx = level_of(st, cx);
            if (!((risk >> lx) & 1u) || R2[lx] == 0) return;  // safe level, or waiting on glob_block
            const int4 px = r.p;
            const uint64_t dxy = dist2(px.x, px.y, px.z, py.x, py.y, py.z);
            if (dxy < dlast || dxy >= R2[lx]) return;
            const int32_t ox = px.w;
            if (key_above(cx, ox, cy, oy) || key_above(cx, ox, tc, to)) return;
            if (a.blocked[x] == round) return;
            // witnesses not above x within d(x, y) of y
            int q = 0;
            for (int i = 0; i < K; i++) {
                const int ci = s_ycls[w][i];
                if (ci == 1 || (ci == 2 && key_above(cx, ox, s_yc[w][i], s_yo[w][i]))) q++;
            }
            // x's entries four at a time (ids, then alive flags, then
            // points, each batch of gathers in flight together); q only
            // grows, so finishing a chunk after q reaches k changes nothing
            const int cxn = a.cnt[x];
            const int32_t* nbx = a.nbr + (size_t)x * Kb;
            for (int j0 = 0; j0 < cxn && q < k; j0 += 4) {
                const int4 v = *(const int4*)(nbx + j0);
                const uint32_t zs[4] = {(uint32_t)v.x, (uint32_t)v.y, (uint32_t)v.z, (uint32_t)v.w};
                bool ok[4];
#pragma unroll
                for (int i = 0; i < 4; i++) ok[i] = j0 + i < cxn && zs[i] != y && a.alive[zs[i]];
                int4 pz[4];
#pragma unroll
                for (int i = 0; i < 4; i++) pz[i] = ok[i] ? a.pts[zs[i]] : py;
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    if (!ok[i]) continue;
                    const uint64_t dyz = dist2(pz[i].x, pz[i].y, pz[i].z, py.x, py.y, py.z);
                    if (dyz <= dlast || dyz > dxy) continue;
                    if (a.inA[zs[i]] == round && key_above(a.cost[zs[i]], pz[i].w, cx, ox)) continue;
                    q++;
                }
            }
            if (q < k) a.blocked[x] = round;
        };
        (void)ns;
        if (rbox != 0) {
            // survivors within sqrt(rbox) of y, from the cells of the level
            // where the box spans at most 4 cells per axis; the survivors of
            // a cell are the records ranked between its first point's rank
            // and the next cell's
            const int ri = (int)sqrt((double)rbox) + 1;
            int se = 0;
            while (se < 21 && (3 << se) < 2 * ri) se++;
            const int Le = min(max(se - g.lv[0].s, 0), g.nlev - 1);
            const LevelView& lv = g.lv[Le];
            const int sc = lv.s;
            const int x0 = max((ux - ri) >> sc, 0), x1 = min((ux + ri) >> sc, lv.cmax[0]);
            const int y0 = max((uy - ri) >> sc, 0), y1 = min((uy + ri) >> sc, lv.cmax[1]);
            const int z0 = max((uz - ri) >> sc, 0), z1 = min((uz + ri) >> sc, lv.cmax[2]);
            const int nx = x1 - x0 + 1, nyy = y1 - y0 + 1, nz = z1 - z0 + 1;
            const int nbox = nx * nyy * nz;
            for (int base = 0; base < nbox; base += kWave) {
                const int idx = base + lane;
                uint32_t st0 = 0, cnt = 0;
                if (idx < nbox) {
                    const int xx = x0 + idx % nx, yy = y0 + (idx / nx) % nyy, zz = z0 + idx / (nx * nyy);
                    // skip cells wholly at squared distance >= rbox
                    const uint64_t gx = axis_gap(ux, xx, sc), gy = axis_gap(uy, yy, sc), gz = axis_gap(uz, zz, sc);
                    if (gx * gx + gy * gy + gz * gz < rbox) {
                        const uint32_t c = hash_find(lv.hkeys, lv.hvals, lv.hmask, cell_code(lv, ys, xx, yy, zz));
                        if (c != kNone) {
                            st0 = surv_rank(a, lv.start[c]);
                            cnt = surv_rank(a, lv.start[c + 1]) - st0;
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
                enumerated += total;
                s_start[w][lane] = st0;
                s_excl[w][lane] = incl - cnt;
                wave_sync_lds();
                for (uint32_t t0 = 0; t0 < total; t0 += kWave) {
                    const uint32_t u = t0 + (uint32_t)lane;
                    if (u < total) {
                        int l = 0;
#pragma unroll
                        for (int step = 32; step > 0; step >>= 1)
                            if (s_excl[w][l + step] <= u) l += step;
                        const uint32_t ri = s_start[w][l] + (u - s_excl[w][l]);
                        if (ri < a.rec_cap) consider(a.surv_rec[ri]);
                    }
                }
                wave_sync_lds();
            }
        }
        wave_sync_lds();
    }
    if (lane == 0 && enumerated) {
        atomicAdd(&st->work, enumerated);
        atomicAdd(&st->stat_enum, (unsigned long long)enumerated);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&st->stat_danger, st->nDanger);
}

template <int K>
int launch_k(Ctx* c, const RoundArrays& a, const GridView& g) {
    const unsigned G = c->round_blocks;
    hipLaunchKernelGGL(rb_group, dim3(G), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_pair<K>, dim3(G), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_survive, dim3(G), dim3(kBlock), 0, c->stream, a, g);
    launch_coarse(c, a, g, 0);
    PDD_HIP(c, hipGetLastError());
    hipLaunchKernelGGL(rb_wcount, dim3(std::min((a.nwords + kBlock) / kBlock, 1024u)), dim3(kBlock), 0, c->stream, a);
    // slots of its own: a captured round keeps their addresses while the
    // budget cut of a batch sorts between its two graphs
    int rc = exclusive_scan_u32_at(c, a.swcnt, a.swpre, a.nwords + 1, nullptr, kSlotSurvScan, 4);
    if (rc) return rc;
    hipLaunchKernelGGL(rb_bucket, dim3(G), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_danger<K>, dim3(G), dim3(kBlock), 0, c->stream, a, g);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

}  // namespace

int launch_blocking(Ctx* c, const RoundArrays& a, const GridView& g, int K) {
    switch (K) {
        case 8: return launch_k<8>(c, a, g);
        case 16: return launch_k<16>(c, a, g);
        case 24: return launch_k<24>(c, a, g);
        case 32: return launch_k<32>(c, a, g);
        default: return PDD_EINVAL;
    }
}

}  // namespace pdd
