// Greedy removal in exact parallel rounds.
//
// The method removes the remaining point of highest cost and re-costs the
// points whose neighbourhood contained it (Sec. 4, Sec. 4.2), with stored
// k+b neighbour lists and reverse lists N(p) (Sec. 5).  Removing a point
// never raises a cost (Sec. 5, step 2).  That monotonicity makes the
// following round rule exact: it yields the sequential greedy's removals,
// each with the cost the greedy removes it at.
//
//   B     removals still to do
//   A     an upper set of the alive keys (key = cost desc, original index
//         asc) with |A| <= min(B, ceil(frac * alive))
//   H(x)  the points of A above x
//   rho'(x)      k-th smallest d2 from x to alive points not in H(x), not x
//   rho(x | y)   k-th smallest d2 from y to alive points not in H(x), not x, y
//   x in A is removed now, with its current cost, unless some y in H(x) has
//        d2(x, y) < rho'(x)        (y could change x's cost before x's turn)
//     or d2(x, y) < rho(x | y)     (x could be in y's neighbourhood when y goes)
//
// Why: while x keeps its key, only points of H(x) can be removed before it
// and every point not in H(x) stays; so x's k-neighbourhood cannot change,
// and removing x first changes no earlier removal's cost.  Induction over
// the removed points in key order extends this to all of them at once.
// The sequential removal order is the removals sorted by key, because the
// greedy's removal keys strictly decrease.
//
// Both conditions are decided from the stored lists, which hold the nearest
// alive points up to their last distance.  Where a list cannot decide, the
// point is blocked (it waits for a later round), which keeps the result
// exact.  The one case that needs a spatial query is a higher y whose list
// holds fewer than k points outside A: lower points beyond its list may then
// be inside rho(x | y) <= the k-th distance from y to alive points outside
// A, which is bounded from per-cell counts and scanned for surviving lower
// points.
#include <type_traits>

#include "search.h"

namespace pdd {

struct RoundDev {
    uint32_t n_alive, n_alive_new, removed, target, m, round, done, err;
    uint32_t nA, nCand, nDanger, nSurv, nTouch, nResearch, nR, mode;
    uint32_t sel_need, sel_bin, pad0, pad1;
    int32_t sel_rem;  // key bits below the first-level prefix
    uint32_t pool_count, pool_cap, overflow;
    uint32_t stat_research, stat_danger, stat_touch, stat_surv;
};

struct RoundArrays {
    const int4* pts;
    const uint32_t* cell_of;
    const uint32_t* coarse_of;
    uint8_t* alive;
    uint64_t* cost;
    int32_t* nbr;       // [n*K]
    uint8_t* cnt;       // [n]
    uint32_t* inA;      // round stamps
    uint32_t* blocked;
    uint32_t* touched;
    uint32_t* surv;
    uint32_t* alive_list[2];
    uint32_t* A;
    uint32_t* cand[2];
    uint32_t* dg_y;      // danger list
    uint64_t* dg_tc;
    int32_t* dg_to;
    uint64_t* dg_dlast;
    uint32_t* touch_list;
    uint32_t* research_list;
    uint32_t* R;
    uint64_t* ev_cost;
    int32_t* ev_orig;
    uint32_t* hist;      // [kSelBins0]
    uint32_t* rev_off;   // [n+1]
    int32_t* rev_src;    // [n*K]
    int32_t* head;       // [n] pool chains
    int32_t* pool_src;
    int32_t* pool_next;
    uint32_t* cell_alive;   // [ncells]
    uint32_t* cellA;        // [ncells] A points per cell, this round
    uint32_t* ccell_alive;  // [nccells]
    uint32_t* ccellA;       // [nccells]
    uint32_t* ccS;          // [nccells] survivors per coarse cell, this round
    RoundDev* st;
    int k, K;
    float frac;
    int check;
};

namespace {

__device__ inline uint32_t wave_append(uint32_t* counter, bool pred) {
    const uint64_t m = __ballot(pred);
    const uint32_t lane = lane_id();
    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1u;
    uint32_t base = 0;
    if (m && lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, (int)leader, kWave);
    return base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// First-level bucket of a cost: 0 for 0, else (msb + 1) * 64 + next 6 bits.
__device__ inline uint32_t bin0(uint64_t c) {
    if (c == 0) return 0;
    const int e = 63 - __clzll(c);
    const uint32_t mant = e >= 6 ? (uint32_t)(c >> (e - 6)) & 63u : (uint32_t)(c << (6 - e)) & 63u;
    return (uint32_t)(e + 1) * 64u + mant;
}

// Bits [lo, lo + w) of the 95-bit key (cost << 31 | (2^31 - 1 - orig)).
__device__ inline uint32_t key_digit(uint64_t c, int32_t orig, int lo, int w) {
    const uint64_t inv = (uint64_t)(0x7FFFFFFF - orig);
    const uint64_t mask = (1ull << w) - 1ull;
    if (lo >= 31) return (uint32_t)((c >> (lo - 31)) & mask);
    if (lo + w <= 31) return (uint32_t)((inv >> lo) & mask);
    return (uint32_t)(((inv >> lo) | (c << (31 - lo))) & mask);
}

// Calls f(x, y, z) for every cell of Chebyshev shell r around (cx, cy, cz)
// inside [0, cm]; returns true when the block of radius r covers [0, cm].
template <class F>
__device__ inline bool for_shell(int cx, int cy, int cz, int r, const int32_t* cm, F f) {
    const int z0 = max(cz - r, 0), z1 = min(cz + r, cm[2]);
    const int y0 = max(cy - r, 0), y1 = min(cy + r, cm[1]);
    const int x0 = max(cx - r, 0), x1 = min(cx + r, cm[0]);
    if (r == 0) {
        f(cx, cy, cz);
    } else {
        for (int z = z0; z <= z1; z++) {
            const bool zf = (z == cz - r) || (z == cz + r);
            for (int y = y0; y <= y1; y++) {
                const bool yf = (y == cy - r) || (y == cy + r);
                if (zf || yf) {
                    for (int x = x0; x <= x1; x++) f(x, y, z);
                } else {
                    if (cx - r >= 0) f(cx - r, y, z);
                    if (cx + r <= cm[0]) f(cx + r, y, z);
                }
            }
        }
    }
    return cx - r <= 0 && cy - r <= 0 && cz - r <= 0 && cx + r >= cm[0] && cy + r >= cm[1] && cz + r >= cm[2];
}

// ---------------------------------------------------------------------------
// selection of A
// ---------------------------------------------------------------------------

__global__ void rb_begin(RoundArrays a) {
    RoundDev* st = a.st;
    __shared__ int skip;
    if (threadIdx.x == 0) {
        skip = 0;
        if (st->done || st->err) {
            skip = 1;
        } else {
            if (st->round > 0) st->n_alive = st->n_alive_new;
            st->n_alive_new = 0;
            if (st->removed >= st->target) {
                st->done = 1;
                skip = 1;
            } else {
                const uint32_t B = st->target - st->removed;
                double want = ceil((double)a.frac * (double)st->n_alive);
                uint32_t m = want < 1.0 ? 1u : (want > (double)B ? B : (uint32_t)want);
                st->m = m;
                st->round++;
                st->nA = st->nCand = st->nDanger = st->nSurv = st->nTouch = st->nResearch = st->nR = 0;
                st->mode = 0;
            }
        }
    }
    __syncthreads();
    if (skip) return;
    for (int i = threadIdx.x; i < kSelBins0; i += blockDim.x) a.hist[i] = 0;
}

__global__ void __launch_bounds__(kBlock) rb_hist0(RoundArrays a, int par) {
    const RoundDev* st = a.st;
    if (st->done || st->err) return;
    __shared__ uint32_t h[kSelBins0];
    for (int i = threadIdx.x; i < kSelBins0; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint32_t na = st->n_alive;
    const uint32_t* L = a.alive_list[par];
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < na; t += gridDim.x * blockDim.x)
        atomicAdd(&h[bin0(a.cost[L[t]])], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < kSelBins0; i += blockDim.x)
        if (h[i]) atomicAdd(&a.hist[i], h[i]);
}

// Bin holding the `need`-th largest key (bins counted from the top) and how
// many of that bin are still needed.  Any block size.
__device__ void find_bin(const uint32_t* hist, int nbins, uint32_t need, uint32_t* bin_out, uint32_t* need_out) {
    __shared__ uint32_t part[1024];
    const int nt = blockDim.x;
    const int per = (nbins + nt - 1) / nt;
    const int t = threadIdx.x;
    uint32_t s = 0;
    for (int r = t * per; r < (t + 1) * per && r < nbins; r++) s += hist[nbins - 1 - r];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        uint32_t cum = 0;
        bool done = false;
        for (int u = 0; u < nt && !done; u++) {
            if (cum + part[u] >= need) {
                for (int r = u * per; r < (u + 1) * per && r < nbins; r++) {
                    const uint32_t h = hist[nbins - 1 - r];
                    if (cum + h >= need) {
                        *bin_out = (uint32_t)(nbins - 1 - r);
                        *need_out = need - cum;
                        done = true;
                        break;
                    }
                    cum += h;
                }
            } else {
                cum += part[u];
            }
        }
        if (!done) {
            *bin_out = 0;
            *need_out = 0;
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kBlock) rb_find0(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    __shared__ uint32_t b, need;
    find_bin(a.hist, kSelBins0, st->m, &b, &need);
    if (threadIdx.x == 0) {
        st->sel_bin = b;
        // A = every bin above b when that is not empty; else the exact top m
        // out of bin b (all of the top m lie in it)
        st->mode = (st->m - need) >= 1 ? 0u : 1u;
        st->sel_need = st->m;
        const int e = (int)(b / 64u) - 1;
        st->sel_rem = (e >= 6 ? e - 6 : 0) + 31;
    }
}

__global__ void __launch_bounds__(kBlock) rb_collect0(RoundArrays a, int par) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t na = st->n_alive, bsel = st->sel_bin, round = st->round, mode = st->mode;
    const uint32_t* L = a.alive_list[par];
    const uint32_t n_it = (na + blockDim.x - 1) / blockDim.x * blockDim.x;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_it; t += gridDim.x * blockDim.x) {
        uint32_t i = 0, bb = 0;
        const bool ok = t < na;
        if (ok) {
            i = L[t];
            bb = bin0(a.cost[i]);
        }
        const bool toA = ok && mode == 0 && bb > bsel;
        const bool toC = ok && mode == 1 && bb == bsel;
        const uint32_t pa = wave_append(&st->nA, toA);
        const uint32_t pc = wave_append(&st->nCand, toC);
        if (toA) {
            a.A[pa] = i;
            a.inA[i] = round;
        }
        if (toC) a.cand[0][pc] = i;
    }
}

// Exact top sel_need of the candidate bin, in one block: 12-bit digits of
// the key below the first-level prefix until at most kSelFinal remain, then
// a bitonic sort.
__global__ void __launch_bounds__(1024) rb_refine(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err || st->mode != 1) return;
    __shared__ uint32_t h[kSelBins];
    __shared__ uint32_t s_nc, s_bin, s_need, s_out;
    __shared__ uint64_t sc[kSelFinal];
    __shared__ int32_t so[kSelFinal];
    __shared__ uint32_t si[kSelFinal];
    const uint32_t round = st->round;
    uint32_t nc = st->nCand, need = st->sel_need;
    int par = 0;
    int hi = st->sel_rem;
    while (nc > (uint32_t)kSelFinal) {
        if (hi <= 0) {
            if (threadIdx.x == 0) st->err = 2;  // keys are unique: cannot happen
            return;
        }
        const int w = hi < 12 ? hi : 12, lo = hi - w;
        const uint32_t* C = a.cand[par];
        uint32_t* D = a.cand[par ^ 1];
        for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) h[i] = 0;
        if (threadIdx.x == 0) s_out = 0;
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < nc; t += blockDim.x) {
            const uint32_t i = C[t];
            atomicAdd(&h[key_digit(a.cost[i], a.pts[i].w, lo, w)], 1u);
        }
        __syncthreads();
        find_bin(h, 1 << w, need, &s_bin, &s_need);
        const uint32_t dsel = s_bin;
        for (uint32_t t = threadIdx.x; t < nc; t += blockDim.x) {
            const uint32_t i = C[t];
            const uint32_t d = key_digit(a.cost[i], a.pts[i].w, lo, w);
            if (d > dsel) {
                const uint32_t p = atomicAdd(&st->nA, 1u);
                a.A[p] = i;
                a.inA[i] = round;
            } else if (d == dsel) {
                D[atomicAdd(&s_out, 1u)] = i;
            }
        }
        __syncthreads();
        nc = s_out;
        need = s_need;
        par ^= 1;
        hi = lo;
        __syncthreads();
    }
    const uint32_t* C = a.cand[par];
    for (int t = threadIdx.x; t < kSelFinal; t += blockDim.x) {
        if ((uint32_t)t < nc) {
            const uint32_t i = C[t];
            si[t] = i;
            sc[t] = a.cost[i];
            so[t] = a.pts[i].w;
        } else {
            si[t] = kNone;
            sc[t] = 0;
            so[t] = 0x7FFFFFFF;
        }
    }
    __syncthreads();
    // bitonic sort, descending by key, padding last
    for (int size = 2; size <= kSelFinal; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < kSelFinal; t += blockDim.x) {
                const int u = t ^ stride;
                if (u > t) {
                    const bool desc = (t & size) == 0;
                    const bool pad_t = si[t] == kNone, pad_u = si[u] == kNone;
                    const bool t_first = pad_u ? true : (pad_t ? false : key_above(sc[t], so[t], sc[u], so[u]));
                    if (t_first != desc) {
                        const uint64_t c0 = sc[t]; sc[t] = sc[u]; sc[u] = c0;
                        const int32_t o0 = so[t]; so[t] = so[u]; so[u] = o0;
                        const uint32_t i0 = si[t]; si[t] = si[u]; si[u] = i0;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) s_out = atomicAdd(&st->nA, need);
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < need; t += blockDim.x) {
        const uint32_t i = si[t];
        a.A[s_out + t] = i;
        a.inA[i] = round;
    }
}

// ---------------------------------------------------------------------------
// blocking
// ---------------------------------------------------------------------------

// One A point y per lane; its list (ascending distance) staged in LDS with
// each entry's class: 0 dead, 1 alive outside A, 2 alive in A.
//  - blocks y when an entry of H(y) is nearer than rho'(y);
//  - blocks every lower A entry x with fewer than k alive entries not in
//    H(x) (other than x) within d(x, y) of y;
//  - puts y on the danger list, with the lowest key a lower point beyond
//    its list must exceed to be safe, when its list is full and holds fewer
//    than k entries outside A.
constexpr int kPairBlock = 64;

template <int K>
__global__ void __launch_bounds__(kPairBlock) rb_pair(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    __shared__ uint64_t sd[K][kPairBlock];
    __shared__ uint64_t sc[K][kPairBlock];
    __shared__ int32_t so[K][kPairBlock];
    __shared__ uint32_t sz[K][kPairBlock];
    __shared__ uint8_t scls[K][kPairBlock];
    const uint32_t nA = st->nA, round = st->round;
    const int k = a.k;
    const int l = threadIdx.x;
    const uint32_t n_it = (nA + kPairBlock - 1) / kPairBlock * kPairBlock;
    for (uint32_t t = blockIdx.x * kPairBlock + l; t < n_it; t += gridDim.x * kPairBlock) {
        bool danger = false;
        uint32_t y = 0;
        uint64_t tc = 0, dlast = 0;
        int32_t to = 0;
        if (t < nA) {
            y = a.A[t];
            const int4 py = a.pts[y];
            const uint64_t cy = a.cost[y];
            const int32_t oy = py.w;
            const int c = a.cnt[y];
            const int32_t* nb = a.nbr + (size_t)y * K;
            int nL = 0, nAe = 0;
            for (int j = 0; j < K; j++) {
                uint8_t cls = 0;
                uint64_t d = ~0ull;
                uint32_t z = 0;
                if (j < c) {
                    z = (uint32_t)nb[j];
                    const int4 pz = a.pts[z];
                    const uint64_t dz = dist2(py.x, py.y, py.z, pz.x, pz.y, pz.z);
                    dlast = dz;
                    if (a.alive[z]) {
                        d = dz;
                        if (a.inA[z] == round) {
                            cls = 2;
                            nAe++;
                            sc[j][l] = a.cost[z];
                            so[j][l] = pz.w;
                        } else {
                            cls = 1;
                            nL++;
                        }
                    }
                }
                sd[j][l] = d;
                scls[j][l] = cls;
                sz[j][l] = z;
            }
            const bool complete = c < K;
            // y itself
            int low = 0;
            uint64_t dH = ~0ull, rho = ~0ull;
            for (int j = 0; j < K; j++) {
                const uint8_t cls = scls[j][l];
                if (cls == 0) continue;
                if (cls == 2 && key_above(sc[j][l], so[j][l], cy, oy)) {
                    if (dH == ~0ull) dH = sd[j][l];
                } else if (++low == k) {
                    rho = sd[j][l];
                    break;
                }
            }
            bool blocked_self;
            if (low >= k) blocked_self = dH < rho;
            else if (complete) blocked_self = dH != ~0ull;
            else blocked_self = true;  // implies higher entries at or before the list's end
            if (blocked_self) a.blocked[y] = round;
            // lower A entries of the list
            for (int j = 0; j < K; j++) {
                if (scls[j][l] != 2) continue;
                const uint64_t cj = sc[j][l];
                const int32_t oj = so[j][l];
                if (key_above(cj, oj, cy, oy)) continue;
                const uint64_t dj = sd[j][l];
                int q = 0;
                for (int i = 0; i < K; i++) {
                    if (i == j) continue;
                    const uint8_t ci = scls[i][l];
                    if (ci == 0) continue;
                    if (sd[i][l] > dj) break;
                    if (ci == 1 || key_above(cj, oj, sc[i][l], so[i][l])) q++;
                }
                const bool covered = complete || dj < dlast;
                if (q < k || !covered) a.blocked[sz[j][l]] = round;
            }
            // lower points beyond the list
            if (!complete && nL < k) {
                danger = true;
                const int need = k - nL;
                if (nAe < need) {
                    tc = cy;
                    to = oy;
                } else {
                    // need-th lowest key among the alive A entries
                    bool have = false;
                    uint64_t pc = 0;
                    int32_t po = 0;
                    for (int r = 0; r < need; r++) {
                        bool found = false;
                        uint64_t bc = 0;
                        int32_t bo = 0;
                        for (int j = 0; j < K; j++) {
                            if (scls[j][l] != 2) continue;
                            const uint64_t cz = sc[j][l];
                            const int32_t oz = so[j][l];
                            if (have && !key_above(cz, oz, pc, po)) continue;
                            if (!found || key_above(bc, bo, cz, oz)) {
                                bc = cz;
                                bo = oz;
                                found = true;
                            }
                        }
                        pc = bc;
                        po = bo;
                        have = true;
                    }
                    tc = pc;
                    to = po;
                }
            }
        }
        const uint32_t p = wave_append(&st->nDanger, danger);
        if (danger) {
            a.dg_y[p] = y;
            a.dg_tc[p] = tc;
            a.dg_to[p] = to;
            a.dg_dlast[p] = dlast;
        }
    }
}

__global__ void __launch_bounds__(kBlock) rb_survive(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t nA = st->nA, round = st->round;
    const uint32_t n_it = (nA + blockDim.x - 1) / blockDim.x * blockDim.x;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_it; t += gridDim.x * blockDim.x) {
        bool sv = false;
        if (t < nA) {
            const uint32_t x = a.A[t];
            atomicAdd(&a.cellA[a.cell_of[x]], 1u);
            atomicAdd(&a.ccellA[a.coarse_of[x]], 1u);
            if (a.blocked[x] != round) {
                sv = true;
                a.surv[x] = round;
                atomicAdd(&a.ccS[a.coarse_of[x]], 1u);
            }
        }
        wave_append(&st->nSurv, sv);
    }
}

// A dangerous y blocks every surviving lower x with key <= its threshold,
// at or beyond its list's last distance and nearer than R, where R bounds
// the k-th distance from y to alive points outside A: the smallest cell
// block around y holding k such points (per-cell counts) gives it.
__global__ void __launch_bounds__(kBlock) rb_danger(RoundArrays a, GridView g) {
    RoundDev* st = a.st;
    if (st->done || st->err || st->nSurv == 0) return;
    const uint32_t nd = st->nDanger, round = st->round;
    const int k = a.k;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nd; t += gridDim.x * blockDim.x) {
        const uint32_t y = a.dg_y[t];
        const uint64_t tc = a.dg_tc[t], dlast = a.dg_dlast[t];
        const int32_t to = a.dg_to[t];
        const int4 py = a.pts[y];
        const uint64_t cy = a.cost[y];
        const int32_t oy = py.w;
        const int ux = py.x - g.minx, uy = py.y - g.miny, uz = py.z - g.minz;
        uint64_t R2 = 0;
        bool inf = false, found = false;
        {
            uint32_t cntL = 0;
            const LevelView& l0 = g.lv[0];
            const int fx = ux >> l0.s, fy = uy >> l0.s, fz = uz >> l0.s;
            for (int r = 0; r <= 2 && !found && !inf; r++) {
                const bool cover = for_shell(fx, fy, fz, r, l0.cmax, [&](int x, int yy, int z) {
                    const uint32_t c =
                        hash_find(l0.hkeys, l0.hvals, l0.hmask, morton3((uint32_t)x, (uint32_t)yy, (uint32_t)z));
                    if (c != kNone) cntL += a.cell_alive[c] - a.cellA[c];
                });
                if (cntL >= (uint32_t)k) {
                    const uint64_t e = (uint64_t)(r + 1) << l0.s;
                    R2 = 3 * e * e;
                    found = true;
                } else if (cover) {
                    inf = true;
                }
            }
            cntL = 0;
            const LevelView& l1 = g.lv[1];
            const int qx = ux >> l1.s, qy = uy >> l1.s, qz = uz >> l1.s;
            for (int r = 0; !found && !inf; r++) {
                const bool cover = for_shell(qx, qy, qz, r, l1.cmax, [&](int x, int yy, int z) {
                    const uint32_t c =
                        hash_find(l1.hkeys, l1.hvals, l1.hmask, morton3((uint32_t)x, (uint32_t)yy, (uint32_t)z));
                    if (c != kNone) cntL += a.ccell_alive[c] - a.ccellA[c];
                });
                if (cntL >= (uint32_t)k) {
                    const uint64_t e = (uint64_t)(r + 1) << l1.s;
                    R2 = 3 * e * e;
                    found = true;
                } else if (cover || r >= 4) {
                    inf = true;  // far or unbounded: every surviving lower point is checked
                }
            }
        }
        auto consider = [&](uint32_t x) {
            if (x == y || a.surv[x] != round) return;
            const int4 px = a.pts[x];
            const uint64_t d = dist2(px.x, px.y, px.z, py.x, py.y, py.z);
            if (d < dlast || (!inf && d >= R2)) return;
            const uint64_t cx = a.cost[x];
            if (key_above(cx, px.w, cy, oy) || key_above(cx, px.w, tc, to)) return;
            a.blocked[x] = round;
        };
        if (inf) {
            const uint32_t nA = st->nA;
            for (uint32_t u = 0; u < nA; u++) consider(a.A[u]);
            continue;
        }
        const int ri = (int)sqrt((double)R2) + 1;
        const LevelView& l1 = g.lv[1];
        const int sc = l1.s;
        const int x0 = max((ux - ri) >> sc, 0), x1 = min((ux + ri) >> sc, l1.cmax[0]);
        const int y0 = max((uy - ri) >> sc, 0), y1 = min((uy + ri) >> sc, l1.cmax[1]);
        const int z0 = max((uz - ri) >> sc, 0), z1 = min((uz + ri) >> sc, l1.cmax[2]);
        for (int zz = z0; zz <= z1; zz++)
            for (int yy = y0; yy <= y1; yy++)
                for (int xx = x0; xx <= x1; xx++) {
                    const uint32_t c =
                        hash_find(l1.hkeys, l1.hvals, l1.hmask, morton3((uint32_t)xx, (uint32_t)yy, (uint32_t)zz));
                    if (c == kNone || a.ccS[c] == 0) continue;
                    for (uint32_t j = l1.start[c]; j < l1.start[c + 1]; j++) consider(j);
                }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&st->stat_danger, nd);
}

// ---------------------------------------------------------------------------
// removal and re-costing
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) rb_remove(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t nA = st->nA, round = st->round;
    const uint32_t n_it = (nA + blockDim.x - 1) / blockDim.x * blockDim.x;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_it; t += gridDim.x * blockDim.x) {
        uint32_t x = 0;
        bool rm = false;
        if (t < nA) {
            x = a.A[t];
            rm = a.blocked[x] != round;
            a.cellA[a.cell_of[x]] = 0;
            a.ccellA[a.coarse_of[x]] = 0;
            a.ccS[a.coarse_of[x]] = 0;
        }
        const uint32_t p = wave_append(&st->nR, rm);
        if (rm) {
            a.R[p] = x;
            a.ev_cost[st->removed + p] = a.cost[x];
            a.ev_orig[st->removed + p] = a.pts[x].w;
            a.alive[x] = 0;
            atomicSub(&a.cell_alive[a.cell_of[x]], 1u);
            atomicSub(&a.ccell_alive[a.coarse_of[x]], 1u);
        }
    }
}

__global__ void rb_remove_end(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    if (st->nR == 0) st->err = 5;  // the top key is never blocked
    st->removed += st->nR;
    st->stat_surv += st->nSurv;
}

__device__ inline void touch(const RoundArrays& a, RoundDev* st, uint32_t z, uint32_t round) {
    if (!a.alive[z]) return;
    if (atomicExch(&a.touched[z], round) == round) return;
    const uint32_t p = atomicAdd(&st->nTouch, 1u);
    a.touch_list[p] = z;
}

__global__ void __launch_bounds__(kBlock) rb_touch(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t nR = st->nR, round = st->round;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nR; t += gridDim.x * blockDim.x) {
        const uint32_t x = a.R[t];
        for (uint32_t e = a.rev_off[x]; e < a.rev_off[x + 1]; e++) touch(a, st, (uint32_t)a.rev_src[e], round);
        for (int32_t p = a.head[x]; p >= 0; p = a.pool_next[p]) touch(a, st, (uint32_t)a.pool_src[p], round);
    }
}

// Cost from the list's first k alive entries; a list with fewer alive
// entries than k that did not hold every alive point is searched again.
__global__ void __launch_bounds__(kBlock) rb_recost(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t nt = st->nTouch;
    const int K = a.K, k = a.k;
    const uint32_t n_it = (nt + blockDim.x - 1) / blockDim.x * blockDim.x;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_it; t += gridDim.x * blockDim.x) {
        bool rs = false;
        uint32_t z = 0;
        if (t < nt) {
            z = a.touch_list[t];
            const int4 pz = a.pts[z];
            const int c = a.cnt[z];
            const int32_t* nb = a.nbr + (size_t)z * K;
            int valid = 0;
            uint64_t w = 0;
            for (int j = 0; j < c && valid < k; j++) {
                const uint32_t y = (uint32_t)nb[j];
                if (!a.alive[y]) continue;
                const int4 py = a.pts[y];
                w += cost_term(dist2(pz.x, pz.y, pz.z, py.x, py.y, py.z));
                valid++;
            }
            if (valid < k && c == K) {
                rs = true;
            } else {
                if (a.check && w > a.cost[z]) st->err = 6;
                a.cost[z] = w;
            }
        }
        const uint32_t p = wave_append(&st->nResearch, rs);
        if (rs) a.research_list[p] = z;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&st->stat_touch, nt);
}

template <int K>
__global__ void __launch_bounds__(kBlock) rb_research(RoundArrays a, GridView g) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t nr = st->nResearch;
    const int k = a.k;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nr; t += gridDim.x * blockDim.x) {
        const uint32_t z = a.research_list[t];
        const int4 pz = a.pts[z];
        TopK<K> tk;
        tk.init();
        SearchCtx sc{a.alive, nullptr, 0};
        ring_search<K, kAlive>(g, z, pz, sc, tk, K);
        const int c = tk.count();
        int32_t* nb = a.nbr + (size_t)z * K;
#pragma unroll
        for (int j = 0; j < K; j++) nb[j] = tk.id[j];
        a.cnt[z] = (uint8_t)c;
        const uint64_t w = list_cost<K>(tk, c < k ? c : k);
        if (a.check && w > a.cost[z]) st->err = 7;
        a.cost[z] = w;
        // reverse edges of the new members
        for (int j = 0; j < c; j++) {
            const uint32_t node = atomicAdd(&st->pool_count, 1u);
            if (node < st->pool_cap) {
                a.pool_src[node] = (int32_t)z;
                a.pool_next[node] = atomicExch(&a.head[nb[j]], (int32_t)node);
            } else {
                st->overflow = 1;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&st->stat_research, nr);
}

__global__ void __launch_bounds__(kBlock) rb_compact(RoundArrays a, int par) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t na = st->n_alive;
    const uint32_t* L = a.alive_list[par];
    uint32_t* M = a.alive_list[par ^ 1];
    const uint32_t n_it = (na + blockDim.x - 1) / blockDim.x * blockDim.x;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_it; t += gridDim.x * blockDim.x) {
        uint32_t i = 0;
        bool keep = false;
        if (t < na) {
            i = L[t];
            keep = a.alive[i] != 0;
        }
        const uint32_t p = wave_append(&st->n_alive_new, keep);
        if (keep) M[p] = i;
    }
}

// ---------------------------------------------------------------------------
// reverse lists
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) rev_count_k(RoundArrays a, uint32_t n, uint32_t* deg) {
    for (uint32_t z = blockIdx.x * blockDim.x + threadIdx.x; z < n; z += gridDim.x * blockDim.x) {
        if (!a.alive[z]) continue;
        const int c = a.cnt[z];
        for (int j = 0; j < c; j++) atomicAdd(&deg[a.nbr[(size_t)z * a.K + j]], 1u);
    }
}

__global__ void __launch_bounds__(kBlock) rev_fill_k(RoundArrays a, uint32_t n, uint32_t* cursor) {
    for (uint32_t z = blockIdx.x * blockDim.x + threadIdx.x; z < n; z += gridDim.x * blockDim.x) {
        if (!a.alive[z]) continue;
        const int c = a.cnt[z];
        for (int j = 0; j < c; j++) {
            const uint32_t slot = atomicAdd(&cursor[a.nbr[(size_t)z * a.K + j]], 1u);
            a.rev_src[slot] = (int32_t)z;
        }
    }
}

__global__ void rev_reset_k(RoundArrays a) {
    a.st->pool_count = 0;
    a.st->overflow = 0;
}

// ---------------------------------------------------------------------------
// setup and finalisation
// ---------------------------------------------------------------------------

__global__ void rd_init(RoundDev* st, uint32_t n, uint32_t target, uint32_t pool_cap) {
    RoundDev z = {};
    z.n_alive = n;
    z.target = target;
    z.pool_cap = pool_cap;
    *st = z;
}

__global__ void __launch_bounds__(kBlock) cell_count_k(const uint32_t* __restrict__ start, uint32_t ncells,
                                                       uint32_t* __restrict__ count) {
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncells; c += gridDim.x * blockDim.x)
        count[c] = start[c + 1] - start[c];
}

__global__ void __launch_bounds__(kBlock) kept_flag_k(const int4* __restrict__ pts, const uint8_t* __restrict__ alive,
                                                      uint32_t n, uint32_t* __restrict__ flag_o) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        flag_o[pts[j].w] = alive[j];
}

__global__ void __launch_bounds__(kBlock) kept_write_k(const uint32_t* __restrict__ flag_o,
                                                       const uint32_t* __restrict__ pos, uint32_t n,
                                                       uint32_t keep, int32_t* __restrict__ kept) {
    for (uint32_t o = blockIdx.x * blockDim.x + threadIdx.x; o < n; o += gridDim.x * blockDim.x)
        if (flag_o[o] && pos[o] < keep) kept[pos[o]] = (int32_t)o;
}

__global__ void __launch_bounds__(kBlock) ev_keys1_k(const int32_t* __restrict__ ev_orig, uint32_t m,
                                                     uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        keys[t] = (uint64_t)(uint32_t)ev_orig[t];
        vals[t] = t;
    }
}

__global__ void __launch_bounds__(kBlock) ev_keys2_k(const uint64_t* __restrict__ k1, const uint32_t* __restrict__ v1,
                                                     const uint64_t* __restrict__ ev_cost, uint32_t m,
                                                     uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        keys[t] = ~ev_cost[v1[t]];
        vals[t] = (uint32_t)k1[t];
    }
}

__global__ void __launch_bounds__(kBlock) ev_out_k(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                                   uint32_t m, int32_t* __restrict__ order,
                                                   uint64_t* __restrict__ order_cost) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        if (order) order[t] = (int32_t)vals[t];
        if (order_cost) order_cost[t] = ~keys[t];
    }
}

inline unsigned gfor(size_t count, unsigned maxg = 4096) {
    size_t g = (count + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > maxg) g = maxg;
    return (unsigned)g;
}

// scratch slots of the decimation state
enum {
    // 0..5 grid build, 40..47 scan partials, 48..50 radix sort, 52..55 order sort, 56..59 k-NN output
    kSAlive = 10, kSCost, kSNbr, kSCnt, kSInA, kSBlocked, kSTouched, kSAl0, kSAl1, kSA, kSC0, kSC1, kSDgY,
    kSTouch, kSResearch, kSR, kSEvC, kSEvO, kSHist, kSRevOff, kSRevSrc, kSHead, kSPoolS, kSPoolN, kSSt, kSTmp,
    kSFin1, kSFin2, kSSurv,
    kSCellAlive = 60, kSCellA, kSCCellAlive, kSCCellA, kSCCS, kSDgC, kSDgO, kSDgD
};
static_assert(kSSurv < 40, "scratch slots overlap the scan's");

int build_reverse(Ctx* c, RoundArrays& a, uint32_t n) {
    uint32_t* deg = (uint32_t*)scratch(c, kSTmp, (size_t)(n + 1) * 4);
    if (!deg) return PDD_ENOMEM;
    int rc;
    if ((rc = fill_u32(c, deg, 0, n + 1))) return rc;
    hipLaunchKernelGGL(rev_count_k, dim3(gfor(n)), dim3(kBlock), 0, c->stream, a, n, deg);
    PDD_HIP(c, hipGetLastError());
    if ((rc = exclusive_scan_u32(c, deg, a.rev_off, n + 1, nullptr))) return rc;
    PDD_HIP(c, hipMemcpyAsync(deg, a.rev_off, (size_t)(n + 1) * 4, hipMemcpyDeviceToDevice, c->stream));
    hipLaunchKernelGGL(rev_fill_k, dim3(gfor(n)), dim3(kBlock), 0, c->stream, a, n, deg);
    PDD_HIP(c, hipGetLastError());
    if ((rc = fill_u32(c, (uint32_t*)a.head, 0xFFFFFFFFu, n))) return rc;
    hipLaunchKernelGGL(rev_reset_k, dim3(1), dim3(1), 0, c->stream, a);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

template <int K>
int launch_round(Ctx* c, RoundArrays& a, const GridView& g, int par) {
    const unsigned G = 1024;
    hipLaunchKernelGGL(rb_begin, dim3(1), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_hist0, dim3(G), dim3(kBlock), 0, c->stream, a, par);
    hipLaunchKernelGGL(rb_find0, dim3(1), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_collect0, dim3(G), dim3(kBlock), 0, c->stream, a, par);
    hipLaunchKernelGGL(rb_refine, dim3(1), dim3(1024), 0, c->stream, a);
    hipLaunchKernelGGL(rb_pair<K>, dim3(2048), dim3(kPairBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_survive, dim3(G), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_danger, dim3(G), dim3(kBlock), 0, c->stream, a, g);
    hipLaunchKernelGGL(rb_remove, dim3(G), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_remove_end, dim3(1), dim3(1), 0, c->stream, a);
    hipLaunchKernelGGL(rb_touch, dim3(G), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_recost, dim3(G), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_research<K>, dim3(G), dim3(kBlock), 0, c->stream, a, g);
    hipLaunchKernelGGL(rb_compact, dim3(G), dim3(kBlock), 0, c->stream, a, par);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

template <int K>
int run_rounds(Ctx* c, RoundArrays& a, const GridView& g, uint32_t n) {
    RoundDev* hst = (RoundDev*)c->pinned;
    int par = 0;
    for (uint64_t it = 0;; it++) {
        int rc = launch_round<K>(c, a, g, par);
        if (rc) return rc;
        par ^= 1;
        PDD_HIP(c, hipMemcpyAsync(hst, a.st, sizeof(RoundDev), hipMemcpyDeviceToHost, c->stream));
        PDD_HIP(c, hipStreamSynchronize(c->stream));
        if (hst->err) {
            c->err = "round invariant violated (code " + std::to_string(hst->err) + ")";
            return PDD_EINTERNAL;
        }
        if (hst->done) {
            c->stats[0] = hst->round;
            c->stats[1] = hst->stat_research;
            c->stats[2] = hst->stat_danger;
            c->stats[7] = hst->stat_touch;
            return PDD_OK;
        }
        if (hst->overflow) {
            if ((rc = build_reverse(c, a, n))) return rc;
            c->stats[3]++;
        }
        if (it > (uint64_t)n + 16) {
            c->err = "round loop made no progress";
            return PDD_EINTERNAL;
        }
    }
}

}  // namespace

int decimate(Ctx* c, const Grid& grid, int k, int K, float frac, int check, int64_t keep, int32_t* kept,
             int32_t* order, uint64_t* order_cost) {
    const GridView& g = grid.v;
    const uint32_t n = g.n;
    const uint32_t target = (uint32_t)(n - keep);
    RoundArrays a{};
    a.pts = g.pts;
    a.cell_of = g.lv[0].of;
    a.coarse_of = g.lv[1].of;
    const uint32_t ncells = g.lv[0].ncells, nccells = g.lv[1].ncells;
    a.k = k;
    a.K = K;
    a.frac = frac;
    a.check = check;
    const size_t pool_cap = (size_t)n * K;
#define ALLOC(field, slot, bytes)                                                         \
    do {                                                                                  \
        a.field = (std::remove_reference<decltype(a.field)>::type)scratch(c, slot, bytes); \
        if (!a.field) return PDD_ENOMEM;                                                  \
    } while (0)
    ALLOC(alive, kSAlive, n);
    ALLOC(cost, kSCost, (size_t)n * 8);
    ALLOC(nbr, kSNbr, (size_t)n * K * 4);
    ALLOC(cnt, kSCnt, n);
    ALLOC(inA, kSInA, (size_t)n * 4);
    ALLOC(blocked, kSBlocked, (size_t)n * 4);
    ALLOC(touched, kSTouched, (size_t)n * 4);
    ALLOC(surv, kSSurv, (size_t)n * 4);
    ALLOC(alive_list[0], kSAl0, (size_t)n * 4);
    ALLOC(alive_list[1], kSAl1, (size_t)n * 4);
    ALLOC(A, kSA, (size_t)n * 4);
    ALLOC(cand[0], kSC0, (size_t)n * 4);
    ALLOC(cand[1], kSC1, (size_t)n * 4);
    ALLOC(dg_y, kSDgY, (size_t)n * 4);
    ALLOC(dg_tc, kSDgC, (size_t)n * 8);
    ALLOC(dg_to, kSDgO, (size_t)n * 4);
    ALLOC(dg_dlast, kSDgD, (size_t)n * 8);
    ALLOC(touch_list, kSTouch, (size_t)n * 4);
    ALLOC(research_list, kSResearch, (size_t)n * 4);
    ALLOC(R, kSR, (size_t)n * 4);
    ALLOC(ev_cost, kSEvC, (size_t)n * 8);
    ALLOC(ev_orig, kSEvO, (size_t)n * 4);
    ALLOC(hist, kSHist, (size_t)kSelBins0 * 4);
    ALLOC(rev_off, kSRevOff, (size_t)(n + 1) * 4);
    ALLOC(rev_src, kSRevSrc, (size_t)n * K * 4);
    ALLOC(head, kSHead, (size_t)n * 4);
    ALLOC(pool_src, kSPoolS, pool_cap * 4);
    ALLOC(pool_next, kSPoolN, pool_cap * 4);
    ALLOC(cell_alive, kSCellAlive, (size_t)ncells * 4);
    ALLOC(cellA, kSCellA, (size_t)ncells * 4);
    ALLOC(ccell_alive, kSCCellAlive, (size_t)nccells * 4);
    ALLOC(ccellA, kSCCellA, (size_t)nccells * 4);
    ALLOC(ccS, kSCCS, (size_t)nccells * 4);
    ALLOC(st, kSSt, sizeof(RoundDev));
#undef ALLOC
    int rc;
    if ((rc = fill_u8(c, a.alive, 1, n))) return rc;
    if ((rc = fill_u32(c, a.inA, 0, n))) return rc;
    if ((rc = fill_u32(c, a.blocked, 0, n))) return rc;
    if ((rc = fill_u32(c, a.touched, 0, n))) return rc;
    if ((rc = fill_u32(c, a.surv, 0, n))) return rc;
    if ((rc = fill_u32(c, a.cellA, 0, ncells))) return rc;
    if ((rc = fill_u32(c, a.ccellA, 0, nccells))) return rc;
    if ((rc = fill_u32(c, a.ccS, 0, nccells))) return rc;
    if ((rc = iota_u32(c, a.alive_list[0], n))) return rc;
    hipLaunchKernelGGL(cell_count_k, dim3(gfor(ncells)), dim3(kBlock), 0, c->stream, g.lv[0].start, ncells,
                       a.cell_alive);
    hipLaunchKernelGGL(cell_count_k, dim3(gfor(nccells)), dim3(kBlock), 0, c->stream, g.lv[1].start, nccells,
                       a.ccell_alive);
    hipLaunchKernelGGL(rd_init, dim3(1), dim3(1), 0, c->stream, a.st, n, target, (uint32_t)pool_cap);
    PDD_HIP(c, hipGetLastError());

    KnnOut ko{a.nbr, a.cnt, a.cost, nullptr};
    mark(c, kPhGrid);
    if ((rc = knn_all(c, g, k, K, ko, &c->stats[4]))) return rc;
    mark(c, kPhKnn);
    if ((rc = build_reverse(c, a, n))) return rc;
    mark(c, kPhReverse);
    c->stats[3] = 0;

    switch (K) {
        case 8: rc = run_rounds<8>(c, a, g, n); break;
        case 16: rc = run_rounds<16>(c, a, g, n); break;
        case 24: rc = run_rounds<24>(c, a, g, n); break;
        case 32: rc = run_rounds<32>(c, a, g, n); break;
        default: return PDD_EINVAL;
    }
    if (rc) return rc;
    mark(c, kPhRounds);

    // kept: ascending original indices of the alive points
    uint32_t* flag_o = (uint32_t*)scratch(c, kSFin1, (size_t)(n + 1) * 4);
    uint32_t* pos = (uint32_t*)scratch(c, kSFin2, (size_t)(n + 1) * 4);
    if (!flag_o || !pos) return PDD_ENOMEM;
    hipLaunchKernelGGL(kept_flag_k, dim3(gfor(n)), dim3(kBlock), 0, c->stream, g.pts, a.alive, n, flag_o);
    PDD_HIP(c, hipGetLastError());
    if ((rc = exclusive_scan_u32(c, flag_o, pos, n, nullptr))) return rc;
    hipLaunchKernelGGL(kept_write_k, dim3(gfor(n)), dim3(kBlock), 0, c->stream, flag_o, pos, n, (uint32_t)keep, kept);
    PDD_HIP(c, hipGetLastError());

    // order: removals sorted by (cost desc, original index asc)
    if ((order || order_cost) && target > 0) {
        uint64_t* keys = (uint64_t*)scratch(c, 52, (size_t)target * 8);
        uint32_t* vals = (uint32_t*)scratch(c, 53, (size_t)target * 4);
        uint64_t* keys2 = (uint64_t*)scratch(c, 54, (size_t)target * 8);
        uint32_t* vals2 = (uint32_t*)scratch(c, 55, (size_t)target * 4);
        if (!keys || !vals || !keys2 || !vals2) return PDD_ENOMEM;
        hipLaunchKernelGGL(ev_keys1_k, dim3(gfor(target)), dim3(kBlock), 0, c->stream, a.ev_orig, target, keys, vals);
        PDD_HIP(c, hipGetLastError());
        int obits = 1;
        while (obits < 31 && (1u << obits) < n) obits++;
        uint64_t* sk;
        uint32_t* sv;
        if ((rc = radix_sort_pairs(c, keys, vals, target, obits, &sk, &sv))) return rc;
        hipLaunchKernelGGL(ev_keys2_k, dim3(gfor(target)), dim3(kBlock), 0, c->stream, sk, sv, a.ev_cost, target,
                           keys2, vals2);
        PDD_HIP(c, hipGetLastError());
        if ((rc = radix_sort_pairs(c, keys2, vals2, target, 64, &sk, &sv))) return rc;
        hipLaunchKernelGGL(ev_out_k, dim3(gfor(target)), dim3(kBlock), 0, c->stream, sk, sv, target, order,
                           order_cost);
        PDD_HIP(c, hipGetLastError());
    }
    mark(c, kPhFinal);
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    return PDD_OK;
}

}  // namespace pdd
