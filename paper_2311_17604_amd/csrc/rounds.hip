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
#include <stdio.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "rounds.h"

namespace pdd {

namespace {

// Bits [lo, lo + w) of the 95-bit key (cost << 31 | (2^31 - 1 - orig)).
__device__ inline uint32_t key_digit(uint64_t c, int32_t orig, int lo, int w) {
    const uint64_t inv = (uint64_t)(0x7FFFFFFF - orig);
    const uint64_t mask = (1ull << w) - 1ull;
    if (lo >= 31) return (uint32_t)((c >> (lo - 31)) & mask);
    if (lo + w <= 31) return (uint32_t)((inv >> lo) & mask);
    return (uint32_t)(((inv >> lo) | (c << (31 - lo))) & mask);
}

// ---------------------------------------------------------------------------
// selection of A
// ---------------------------------------------------------------------------

// candidate pool size: kPoolFactor * m points (at least kPoolMin) when built
constexpr uint32_t kPoolFactor = 16, kPoolMin = 1u << 16;

__global__ void rb_begin(RoundArrays a) {
    RoundDev* st = a.st;
    __shared__ int skip;
    if (threadIdx.x == 0) {
        skip = 0;
        if (st->done || st->err) {
            skip = 1;
        } else {
            if (st->round > 0) st->n_alive = st->n_alive_new;
            if (st->removed >= st->target) {
                st->done = 1;
                skip = 1;
            } else {
                const uint32_t B = st->target - st->removed;
                double want = ceil((double)st->frac * (double)st->n_alive);
                uint32_t m = want < 1.0 ? 1u : (want > (double)B ? B : (uint32_t)want);
                st->m = m;
                st->round++;
                st->nA = st->nCand = st->nDanger = st->nSurv = st->nTouch = st->nResearch = st->nR = 0;
                st->mode = 0;
                st->nOvf = 0;
                st->nA2 = 0;
                st->work = 0;
                for (int j = 0; j < kLev; j++) st->surv_min[j] = ~0ull;
                st->full = st->p_valid ? 0u : 1u;
                st->nP_next = 0;
                st->n_list_new = 0;
            }
        }
    }
    __syncthreads();
    if (skip) return;
    for (int i = threadIdx.x; i < kSelBins0; i += blockDim.x) a.hist[i] = 0;
}

// Key histogram of the ranked points: in a full round every alive point
// (the alive list still holds points removed since its last compaction), in
// a pool round the pool members with bin0(cost) >= p_lo, which this pass
// also compacts into the other pool buffer.  st->full: 0 pool round, 1 full
// round, 2 full round decided by rb_pool_check after the pool pass; pass 0
// runs before that check, pass 1 after it (full rounds of kind 2 only).
__global__ void __launch_bounds__(kBlock) rb_hist0(RoundArrays a, int pass) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    if (pass == 1 && st->full != 2) return;
    __shared__ uint32_t h[kSelBins0];
    for (int i = threadIdx.x; i < kSelBins0; i += blockDim.x) h[i] = 0;
    __syncthreads();
    if (st->full) {
        const uint32_t na = st->n_list;
        const uint32_t* L = a.alive_list[st->apar];
        for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < na; t += gridDim.x * blockDim.x) {
            const uint32_t x = L[t];
            if (!a.alive[x]) continue;
            if (a.seg && a.seg_left[a.seg[x]] == 0) continue;  // segment done: not ranked
            atomicAdd(&h[bin0(a.cost[x])], 1u);
        }
    } else {
        const uint32_t np = st->nP, lo = st->p_lo;
        const uint32_t* P = a.pool_list[st->pcur];
        uint32_t* Q = a.pool_list[st->pcur ^ 1u];
        constexpr int IPT = 8;
        for (uint32_t base = blockIdx.x * kBlock * IPT; base < np; base += gridDim.x * kBlock * IPT) {
            uint32_t item[IPT];
            uint32_t sel = 0, nsel = 0;
#pragma unroll
            for (int e = 0; e < IPT; e++) {
                const uint32_t t = base + e * kBlock + threadIdx.x;
                item[e] = 0;
                if (t < np) {
                    const uint32_t x = P[t];
                    item[e] = x;
                    if (a.alive[x] && !(a.seg && a.seg_left[a.seg[x]] == 0)) {
                        const uint32_t bb = bin0(a.cost[x]);
                        if (bb >= lo) {
                            atomicAdd(&h[bb], 1u);
                            sel |= 1u << e;
                            nsel++;
                        }
                    }
                }
            }
            uint32_t p = block_reserve(&st->nP_next, nsel);
#pragma unroll
            for (int e = 0; e < IPT; e++)
                if ((sel >> e) & 1u) Q[p++] = item[e];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSelBins0; i += blockDim.x)
        if (h[i]) atomicAdd(&a.hist[i], h[i]);
}

// Pool round: the compacted pool becomes current when it holds at least half
// of m (it is an upper set, so its top is the top of all alive points);
// otherwise the round is a full one.
__global__ void rb_pool_check(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err || st->full) return;
    __shared__ uint32_t total;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    uint32_t part = 0;
    for (int i = threadIdx.x; i < kSelBins0; i += blockDim.x) part += a.hist[i];
    atomicAdd(&total, part);
    __syncthreads();
    const bool full = 2ull * total < (uint64_t)st->m;
    if (full) {
        for (int i = threadIdx.x; i < kSelBins0; i += blockDim.x) a.hist[i] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (full) {
            st->full = 2;
        } else {
            st->pcur ^= 1u;
            st->nP = st->nP_next;
        }
    }
}

// Bin holding the `need`-th largest key (bins counted from the top) and how
// many of that bin are still needed (bin 0 and none when the bins hold fewer
// than `need`; the top bin and none when `need` is 0).  Block sizes that are
// multiples of the wavefront, up to 1024: each thread sums a run of bins, a
// block scan of the sums finds the one thread whose run holds the
// need-th key, and that thread walks its run.
__device__ void find_bin(const uint32_t* hist, int nbins, uint32_t need, uint32_t* bin_out, uint32_t* need_out) {
    __shared__ uint32_t wsum[1024 / kWave];
    __shared__ int found;
    const int nt = blockDim.x, t = threadIdx.x;
    const int lane = t & (kWave - 1), wid = t / kWave;
    const int per = (nbins + nt - 1) / nt;
    uint32_t s = 0;
    for (int r = t * per; r < (t + 1) * per && r < nbins; r++) s += hist[nbins - 1 - r];
    uint32_t x = s;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[wid] = x;
    if (t == 0) found = 0;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wid; w++) base += wsum[w];
    const uint32_t incl = base + x, excl = incl - s;
    if (need == 0) {
        if (t == 0) {
            *bin_out = (uint32_t)(nbins - 1);
            *need_out = 0;
            found = 1;
        }
    } else if (excl < need && incl >= need) {
        uint32_t cum = excl;
        for (int r = t * per; r < (t + 1) * per && r < nbins; r++) {
            const uint32_t h = hist[nbins - 1 - r];
            if (cum + h >= need) {
                *bin_out = (uint32_t)(nbins - 1 - r);
                *need_out = need - cum;
                break;
            }
            cum += h;
        }
        found = 1;
    }
    __syncthreads();
    if (t == 0 && !found) {
        *bin_out = 0;
        *need_out = 0;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kBlock) rb_find0(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    __shared__ uint32_t b, need, total;
    // the m of this round, at most the ranked (eligible) points
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    uint32_t part = 0;
    for (int i = threadIdx.x; i < kSelBins0; i += blockDim.x) part += a.hist[i];
    atomicAdd(&total, part);
    __syncthreads();
    if (threadIdx.x == 0 && total < st->m) st->m = total > 0 ? total : 1u;
    __syncthreads();
    find_bin(a.hist, kSelBins0, st->m, &b, &need);
    if (st->full) {
        // the new pool: the bins from the one holding the M-th largest key up
        __shared__ uint32_t pb, pneed;
        const uint64_t want = std::max<uint64_t>((uint64_t)kPoolFactor * st->m, (uint64_t)kPoolMin);
        const uint32_t M = (uint32_t)std::min<uint64_t>(want, (uint64_t)total);
        find_bin(a.hist, kSelBins0, M, &pb, &pneed);
        if (threadIdx.x == 0) {
            st->p_lo = pb;
            st->nP = 0;
        }
    }
    if (threadIdx.x == 0) {
        st->sel_bin = b;
        // A = the bins above b, plus (mode 1) the exact top `need` of bin b
        // when the bins above hold less than half of m
        const uint32_t above = st->m - need;
        const uint32_t mode = 2 * above >= st->m ? 0u : 1u;
        st->mode = mode;
        st->sel_need = need;
        const int e = (int)(b / 64u) - 1;
        st->sel_rem = (e >= 6 ? e - 6 : 0) + 31;
        // key levels: split A into kLev parts of about equal count by bin
        // (the part taken from bin b is in level 0)
        st->lev_t[0] = 0;
        for (int j = 1; j < kLev; j++) st->lev_t[j] = 0xFFFFFFFFu;
        const uint64_t total = mode == 0 ? above : st->m;
        uint64_t cum = mode == 0 ? 0 : need;
        int j = 1;
        while (j < kLev && cum * kLev >= total * j && total > cum) {
            st->lev_t[j] = b + 1;
            j++;
        }
        for (uint32_t bb = b + 1; bb < (uint32_t)kSelBins0 && j < kLev; bb++) {
            cum += a.hist[bb];
            while (j < kLev && cum * kLev >= total * j) {
                st->lev_t[j] = bb + 1;
                j++;
            }
        }
    }
}

// A (bins above sel_bin) and, in mode 1, the candidates of bin sel_bin.  A
// full round collects them from the alive list, which it compacts, and
// builds the pool (bins >= p_lo); a pool round collects them from the pool
// that rb_hist0 compacted.
__global__ void __launch_bounds__(kBlock) rb_collect0(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t bsel = st->sel_bin, round = st->round, mode = st->mode, full = st->full, lo = st->p_lo;
    const uint32_t na = full ? st->n_list : st->nP;
    const uint32_t* L = full ? a.alive_list[st->apar] : a.pool_list[st->pcur];
    uint32_t* Lc = a.alive_list[st->apar ^ 1u];
    uint32_t* P = a.pool_list[st->pcur];
    constexpr int IPT = 8;
    for (uint32_t base = blockIdx.x * kBlock * IPT; base < na; base += gridDim.x * kBlock * IPT) {
        uint32_t item[IPT];
        uint32_t selA = 0, selC = 0, selL = 0, selP = 0, nA = 0, nC = 0, nL = 0, nP = 0;
#pragma unroll
        for (int e = 0; e < IPT; e++) {
            const uint32_t t = base + e * kBlock + threadIdx.x;
            item[e] = 0;
            if (t < na) {
                const uint32_t i = L[t];
                item[e] = i;
                bool elig = true;
                if (full) {
                    const bool al = a.alive[i] != 0;
                    if (al) {
                        selL |= 1u << e;
                        nL++;
                    }
                    elig = al && !(a.seg && a.seg_left[a.seg[i]] == 0);  // segment done: not ranked
                }
                const uint32_t bb = elig ? bin0(a.cost[i]) : 0u;
                if (full && elig && bb >= lo) {
                    selP |= 1u << e;
                    nP++;
                }
                if (elig && bb > bsel) {
                    selA |= 1u << e;
                    nA++;
                } else if (elig && mode == 1 && bb == bsel) {
                    selC |= 1u << e;
                    nC++;
                }
            }
        }
        uint32_t pA = block_reserve(&st->nA, nA);
        uint32_t pC = mode == 1 ? block_reserve(&st->nCand, nC) : 0u;
        uint32_t pL = full ? block_reserve(&st->n_list_new, nL) : 0u;
        uint32_t pP = full ? block_reserve(&st->nP, nP) : 0u;
#pragma unroll
        for (int e = 0; e < IPT; e++) {
            if ((selA >> e) & 1u) {
                a.A[pA++] = item[e];
                a.inA[item[e]] = round;
            } else if ((selC >> e) & 1u) {
                a.cand[0][pC++] = item[e];
            }
            if ((selL >> e) & 1u) Lc[pL++] = item[e];
            if ((selP >> e) & 1u) P[pP++] = item[e];
        }
    }
}

// candidates per thread and step of rb_refine's passes
constexpr int kRefineIPT = 8;

// Exact top sel_need of the candidate bin, in one block: 12-bit digits of
// the key below the first-level prefix until at most kSelFinal remain, then
// a bitonic sort.

__global__ void __launch_bounds__(1024) rb_refine(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err || st->mode != 1) return;
    __shared__ uint32_t h[kSelBins];
    __shared__ uint32_t s_bin, s_need, s_out;
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
        // kRefineIPT candidates per thread at a time: their indices, then
        // their keys, each batch of loads in flight together
        for (uint32_t t0 = threadIdx.x; t0 < nc; t0 += blockDim.x * kRefineIPT) {
            uint32_t ii[kRefineIPT];
            uint32_t dd[kRefineIPT];
#pragma unroll
            for (int e = 0; e < kRefineIPT; e++) {
                const uint32_t t = t0 + e * blockDim.x;
                ii[e] = t < nc ? C[t] : kNone;
            }
#pragma unroll
            for (int e = 0; e < kRefineIPT; e++)
                dd[e] = ii[e] != kNone ? key_digit(a.cost[ii[e]], a.pts[ii[e]].w, lo, w) : 0u;
#pragma unroll
            for (int e = 0; e < kRefineIPT; e++)
                if (ii[e] != kNone) atomicAdd(&h[dd[e]], 1u);
        }
        __syncthreads();
        find_bin(h, 1 << w, need, &s_bin, &s_need);
        const uint32_t dsel = s_bin;
        for (uint32_t t0 = threadIdx.x; t0 < nc; t0 += blockDim.x * kRefineIPT) {
            uint32_t ii[kRefineIPT];
            uint32_t dd[kRefineIPT];
#pragma unroll
            for (int e = 0; e < kRefineIPT; e++) {
                const uint32_t t = t0 + e * blockDim.x;
                ii[e] = t < nc ? C[t] : kNone;
            }
#pragma unroll
            for (int e = 0; e < kRefineIPT; e++)
                dd[e] = ii[e] != kNone ? key_digit(a.cost[ii[e]], a.pts[ii[e]].w, lo, w) : 0u;
#pragma unroll
            for (int e = 0; e < kRefineIPT; e++) {
                if (ii[e] == kNone) continue;
                const uint32_t i = ii[e];
                if (dd[e] > dsel) {
                    const uint32_t p = atomicAdd(&st->nA, 1u);
                    a.A[p] = i;
                    a.inA[i] = round;
                } else if (dd[e] == dsel) {
                    D[atomicAdd(&s_out, 1u)] = i;
                }
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
// per-segment budgets (a batch of independent clouds)
// ---------------------------------------------------------------------------

// this round's per-segment counters and bounds back to their start values
__global__ void __launch_bounds__(kBlock) rb_seg_reset(RoundArrays a) {
    if (a.st->done || a.st->err) return;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < a.nseg; s += gridDim.x * blockDim.x) {
        a.seg_cntA[s] = 0;
        a.seg_top_cost[s] = 0;
        a.seg_top_orig[s] = 0x7FFFFFFF;
#pragma unroll
        for (int j = 0; j < kLev; j++) a.seg_glob[(size_t)s * kLev + j] = 0;
    }
}

// A points per segment, then the A points of the segments whose A holds
// more than their remaining budget (those keep only their top keys)
__global__ void __launch_bounds__(kBlock) rb_seg_count(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t nA = st->nA;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nA; t += gridDim.x * blockDim.x)
        atomicAdd(&a.seg_cntA[a.seg[a.A[t]]], 1u);
}

__global__ void __launch_bounds__(kBlock) rb_seg_over(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t nA = st->nA;
    const uint32_t n_it = (nA + blockDim.x - 1) / blockDim.x * blockDim.x;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_it; t += gridDim.x * blockDim.x) {
        uint32_t x = 0;
        bool over = false;
        if (t < nA) {
            x = a.A[t];
            const uint32_t sx = a.seg[x];
            over = a.seg_cntA[sx] > a.seg_left[sx];
        }
        const uint32_t p = wave_append(&st->nOvf, over);
        if (over) a.ovf[p] = x;
    }
}

// sort keys of the over-budget A points: original index, then the
// complement of the cost, then the segment (three stable passes give
// segment ascending, key descending)
__global__ void __launch_bounds__(kBlock) ovf_keys_k(RoundArrays a, int pass, const uint32_t* __restrict__ src,
                                                     uint32_t m, uint64_t* __restrict__ keys,
                                                     uint32_t* __restrict__ vals) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        const uint32_t x = src[t];
        keys[t] = pass == 0 ? (uint64_t)(uint32_t)a.pts[x].w : (pass == 1 ? ~a.cost[x] : (uint64_t)a.seg[x]);
        vals[t] = x;
    }
}

// first sorted position of each segment, then drop the points ranked at or
// beyond their segment's budget from A
__global__ void __launch_bounds__(kBlock) ovf_first_k(RoundArrays a, const uint32_t* __restrict__ sorted, uint32_t m,
                                                      uint32_t* __restrict__ first) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        const uint32_t sx = a.seg[sorted[t]];
        if (t == 0 || a.seg[sorted[t - 1]] != sx) first[sx] = t;
    }
}

__global__ void __launch_bounds__(kBlock) ovf_drop_k(RoundArrays a, const uint32_t* __restrict__ sorted, uint32_t m,
                                                     const uint32_t* __restrict__ first) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        const uint32_t x = sorted[t], sx = a.seg[x];
        if (t - first[sx] >= a.seg_left[sx]) a.inA[x] = 0;
    }
}

// A without the dropped points (into cand[1], then back)
__global__ void __launch_bounds__(kBlock) ovf_compact_k(RoundArrays a) {
    RoundDev* st = a.st;
    const uint32_t nA = st->nA, round = st->round;
    const uint32_t n_it = (nA + blockDim.x - 1) / blockDim.x * blockDim.x;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_it; t += gridDim.x * blockDim.x) {
        uint32_t x = 0;
        bool keep = false;
        if (t < nA) {
            x = a.A[t];
            keep = a.inA[x] == round;
        }
        const uint32_t p = wave_append(&st->nA2, keep);
        if (keep) a.cand[1][p] = x;
    }
}

// (nA2 is cleared by rb_begin: a block of this kernel that cleared it could
// run before another block has read it)
__global__ void __launch_bounds__(kBlock) ovf_copy_k(RoundArrays a) {
    RoundDev* st = a.st;
    const uint32_t m = st->nA2;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) a.A[t] = a.cand[1][t];
    if (blockIdx.x == 0 && threadIdx.x == 0) st->nA = m;
}

// ---------------------------------------------------------------------------
// removal and re-costing
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) rb_remove(RoundArrays a, GridView g) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint32_t nA = st->nA, round = st->round;
    const uint32_t n_it = (nA + blockDim.x - 1) / blockDim.x * blockDim.x;
    uint32_t run_seg = 0, run_cnt = 0;  // removals of the thread's current segment
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_it; t += gridDim.x * blockDim.x) {
        uint32_t x = 0;
        bool rm = false;
        if (t < nA) {
            x = a.A[t];
            // the survivor bits of this round are read no more (every
            // survivor is in A)
            a.sbits[x >> 6] = 0ull;
            // an identical point ranked below is a witness for everything:
            // with k of them x is removed whatever its neighbours do
            rm = a.gsafe[x] == round;
            if (!rm && a.blocked[x] != round) {
                // a dangerous point with no bound for this level makes every
                // survivor of the level at or below its cost wait (except the
                // round's highest key, which no point can precede)
                const uint64_t cx = a.cost[x];
                const uint32_t sx = seg_of_pt(a, x);
                const bool top = cx == a.seg_top_cost[sx] && a.pts[x].w == a.seg_top_orig[sx];
                rm = top || cx >= a.seg_glob[sx * kLev + level_of(st, cx)];
            }
        }
        // clear this round's A counts of x's cells at every level, and take
        // the removed points off the alive counts (one lane per wave where
        // the wave's points share the cell)
        {
            const bool act = t < nA;
            uint32_t c = act ? a.of0[x] : 0u;
            const uint64_t am = __ballot(act);
            const int leader = am ? __ffsll((unsigned long long)am) - 1 : 0;
            const int lane = (int)(threadIdx.x & (kWave - 1));
            for (int L = 0; L < a.lc && am; L++) {
                const uint32_t gc = g.lv[L].base + c;
                const uint32_t g0 = (uint32_t)__shfl((int)gc, leader, kWave);
                const bool uni = __all(!act || gc == g0);
                if (act && (!uni || lane == leader)) {
#pragma unroll
                    for (int j = 0; j < kLev; j++) a.cellAlev[(size_t)gc * kLev + j] = 0;
                }
                if (uni) {
                    const uint32_t cnt = (uint32_t)__popcll(__ballot(rm));
                    if (lane == leader && cnt) atomicSub(&a.cell_alive[g0], cnt);
                } else if (rm) {
                    atomicSub(&a.cell_alive[gc], 1u);
                }
                if (act && L + 1 < a.lc) c = g.lv[L].parent[c];
            }
        }
        // one shared-counter atomic per block (the loop bound is uniform over
        // the block)
        const uint32_t p = block_reserve(&st->nR, rm ? 1u : 0u);
        if (rm) {
            a.R[p] = x;
            a.ev_cost[st->removed + p] = a.cost[x];
            a.ev_orig[st->removed + p] = a.pts[x].w;
            a.alive[x] = 0;
            a.apts[a.vpos[x]].w = -1;  // dead in the search view
            const uint32_t sx = seg_of_pt(a, x);
            if (run_cnt && sx != run_seg) {
                atomicSub(&a.seg_left[run_seg], run_cnt);
                run_cnt = 0;
            }
            run_seg = sx;
            run_cnt++;
        }
    }
    block_seg_sub(a.seg_left, run_seg, run_cnt);
}

__global__ void rb_remove_end(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    if (st->nR == 0) st->err = 5;  // the top key is never blocked
    st->removed += st->nR;
    st->n_alive_new = st->n_alive - st->nR;
    if (st->full) {
        // the compacted alive list and the new pool take over
        st->apar ^= 1u;
        st->n_list = st->n_list_new;
        st->p_valid = 1;
    }
    st->stat_surv += st->nSurv;
    // adapt the ranked share: a round that frees few of A (a dense region
    // filling A), or whose danger checks enumerate many survivors (their
    // number grows faster than A), ranks fewer points next time; a
    // productive and cheap one more
    const float yield = (float)st->nR / (float)(st->nA ? st->nA : 1);
    if (yield < 0.05f || st->work > (4u << 20)) st->frac = fmaxf(st->frac * 0.5f, 1e-5f);
    else if (yield > 0.2f && st->work < (1u << 20)) st->frac = fminf(st->frac * 1.5f, st->frac_max);
}

// removed points per wavefront in rb_touch_recost, and chain nodes each of
// them collects per step (kTouchGroup * kChainStep = one wavefront)
constexpr int kTouchGroup = 4, kChainStep = kWave / kTouchGroup;

// Re-costs every alive point whose list held a removed point (the removed
// points' reverse lists): kTouchGroup removed points per wavefront, one lane
// per reverse entry.  The lane that touches a point first this round re-costs
// it from its list's first k alive entries; a list with fewer alive entries
// than k that did not hold every alive point is queued for the re-search
// (staged in the wave's LDS: one shared-counter atomic per 64 entries).
__global__ void __launch_bounds__(kBlock) rb_touch_recost(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    constexpr int W = kBlock / kWave;
    __shared__ uint32_t s_rs[W][2 * kWave], s_chain[W][kWave], s_cnt[W];
    const uint32_t nR = st->nR, round = st->round;
    const int K = a.K, k = a.k;
    const int lane = (int)lane_id(), w = threadIdx.x / kWave;
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t nrs = 0, ntouched = 0;  // wave-uniform
    // touch z (if valid) and re-cost it when this lane touched it first;
    // every lane of the wave calls it
    auto visit = [&](bool valid, uint32_t z) {
        // z's alive flag, touch stamp, point, list length and window in one
        // batch of gathers (a dead z takes the stamp too; nothing reads it)
        bool fresh = false;
        int4 pz = make_int4(0, 0, 0, 0);
        int c = 0;
        uint32_t win = 0;
        if (valid) {
            const uint8_t az = a.alive[z];
            const uint32_t was = atomicExch(&a.touched[z], round);
            pz = a.pts[z];
            c = a.cnt[z];
            win = a.win[z];
            fresh = az && was != round;
        }
        bool rs = false;
        if (fresh) {
            // z's cost is the exact sum of the terms of the entries that
            // win[z] marks: the first k of its list that were alive before
            // this round.  The new cost takes off the terms of the marked
            // entries removed this round and adds those of the next alive
            // entries past the marked ones, so only their points are read.
            const int wend = win ? 32 - __builtin_clz(win) : 0;  // positions [0, wend) hold every marked entry
            const int32_t* nb = a.nbr + (size_t)z * K;
            int nnew = 0;       // alive entries of the new window
            uint32_t nwin = 0;  // and their positions
            uint64_t sub = 0, add = 0;
            // eight entries at a time (K is a multiple of 8 and every list
            // starts 32-byte aligned): their ids in two loads, then their
            // alive flags, then the points whose terms change, each batch of
            // gathers in flight together
            for (int j0 = 0; j0 < c && (j0 < wend || nnew < k); j0 += 8) {
                const int4 v0 = *(const int4*)(nb + j0), v1 = *(const int4*)(nb + j0 + 4);
                const uint32_t ys[8] = {(uint32_t)v0.x, (uint32_t)v0.y, (uint32_t)v0.z, (uint32_t)v0.w,
                                        (uint32_t)v1.x, (uint32_t)v1.y, (uint32_t)v1.z, (uint32_t)v1.w};
                bool al[8], chg[8];
#pragma unroll
                for (int i = 0; i < 8; i++) al[i] = j0 + i < c && a.alive[ys[i]];
                // an alive entry outside the window lies past it (every
                // entry alive now was alive before, and the window holds the
                // first k of those)
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    const bool marked = (win >> (j0 + i)) & 1u;
                    chg[i] = marked ? !al[i] : (al[i] && nnew < k);
                    if (al[i] && (marked || nnew < k)) {
                        nnew++;
                        nwin |= 1u << (j0 + i);
                    }
                }
                int4 py[8];
#pragma unroll
                for (int i = 0; i < 8; i++) py[i] = chg[i] ? a.pts[ys[i]] : pz;
#pragma unroll
                for (int i = 0; i < 8; i++)
                    if (chg[i]) {
                        const uint64_t t = cost_term(dist2(pz.x, pz.y, pz.z, py[i].x, py[i].y, py[i].z));
                        if (al[i]) add += t;
                        else sub += t;
                    }
            }
            if (nnew < k && c == K) {
                rs = true;
            } else if (nwin != win) {
                const uint64_t old = a.cost[z];
                const uint64_t wsum = old - sub + add;
                if (a.check) {
                    // the full sum over the first k alive entries
                    uint64_t full = 0;
                    uint32_t fwin = 0;
                    int nv = 0;
                    for (int j = 0; j < c && nv < k; j++) {
                        const uint32_t y = (uint32_t)nb[j];
                        if (!a.alive[y]) continue;
                        const int4 q = a.pts[y];
                        full += cost_term(dist2(pz.x, pz.y, pz.z, q.x, q.y, q.z));
                        fwin |= 1u << j;
                        nv++;
                    }
                    if (sub > old || wsum > old || full != wsum || fwin != nwin) st->err = 6;
                }
                a.cost[z] = wsum;
                a.win[z] = nwin;
            }
        }
        ntouched += (uint32_t)__popcll(__ballot(fresh));
        const uint64_t bm = __ballot(rs);
        if (rs) s_rs[w][nrs + (uint32_t)__popcll(bm & below)] = z;
        nrs += (uint32_t)__popcll(bm);
        wave_sync_lds();
        if (nrs >= (uint32_t)kWave) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&st->nResearch, (uint32_t)kWave);
            base = (uint32_t)__shfl((int)base, 0, kWave);
            a.research_list[base + lane] = s_rs[w][lane];
            const uint32_t rem = nrs - kWave;
            const uint32_t v = (uint32_t)lane < rem ? s_rs[w][kWave + lane] : 0u;
            wave_sync_lds();
            if ((uint32_t)lane < rem) s_rs[w][lane] = v;
            nrs = rem;
            wave_sync_lds();
        }
    };
    // kTouchGroup removed points per wave: their CSR entries packed into
    // chunks of 64, their chains walked side by side
    const uint32_t nw = gridDim.x * W;
    for (uint32_t g0 = (blockIdx.x * W + w) * kTouchGroup; g0 < nR; g0 += nw * kTouchGroup) {
        const bool mine = lane < kTouchGroup && g0 + (uint32_t)lane < nR;
        const uint32_t x = mine ? a.R[g0 + lane] : 0u;
        const uint64_t e0 = mine ? a.rev_off[x] : 0ull;
        const uint32_t len = mine ? (uint32_t)(a.rev_off[x + 1] - e0) : 0u;
        // exclusive prefix of the lengths over the group's lanes
        uint32_t incl = len;
#pragma unroll
        for (int o = 1; o < kTouchGroup; o <<= 1) {
            const uint32_t v = (uint32_t)__shfl_up((int)incl, o, kWave);
            if (lane >= o) incl += v;
        }
        uint32_t ex[kTouchGroup];
        uint64_t st0[kTouchGroup];
#pragma unroll
        for (int i = 0; i < kTouchGroup; i++) {
            ex[i] = (uint32_t)__shfl((int)(incl - len), i, kWave);
            st0[i] = readlane64(e0, i);
        }
        const uint32_t total = (uint32_t)__shfl((int)incl, kTouchGroup - 1, kWave);
        for (uint32_t c0 = 0; c0 < total; c0 += kWave) {
            const uint32_t u = c0 + (uint32_t)lane;
            const bool valid = u < total;
            int i = 0;
#pragma unroll
            for (int j = 1; j < kTouchGroup; j++)
                if (u >= ex[j]) i = j;
            uint64_t src = st0[0] + u;
#pragma unroll
            for (int j = 1; j < kTouchGroup; j++)
                if (i == j) src = st0[j] + (u - ex[j]);
            visit(valid, valid ? (uint32_t)a.rev_src[src] : 0u);
        }
        // the appended chains: lane j < kTouchGroup walks up to kChainStep
        // nodes of its point's chain into its LDS segment, then the lanes
        // visit the collected nodes
        int32_t p = mine ? a.head[x] : -1;
        while (__any(p >= 0)) {
            uint32_t m = 0;
            if (lane < kTouchGroup) {
                while (p >= 0 && m < (uint32_t)kChainStep) {
                    s_chain[w][lane * kChainStep + m++] = (uint32_t)a.pool_src[p];
                    p = a.pool_next[p];
                }
            }
            const uint32_t mj = (uint32_t)__shfl((int)m, lane / kChainStep, kWave);
            wave_sync_lds();
            const bool valid = (uint32_t)(lane % kChainStep) < mj;
            visit(valid, valid ? s_chain[w][lane] : 0u);
            wave_sync_lds();
        }
    }
    if (nrs) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&st->nResearch, nrs);
        base = (uint32_t)__shfl((int)base, 0, kWave);
        if ((uint32_t)lane < nrs) a.research_list[base + lane] = s_rs[w][lane];
    }
    // touched count: one atomic per block
    if (lane == 0) s_cnt[w] = ntouched;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sum = 0;
        for (int i = 0; i < W; i++) sum += s_cnt[i];
        if (sum) {
            atomicAdd(&st->nTouch, sum);
            atomicAdd(&st->stat_touch, sum);
        }
    }
}

// New list of z over the alive points: one wavefront per point.
template <int K>
__global__ void __launch_bounds__(kBlock) rb_research(RoundArrays a, GridView g) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    __shared__ uint32_t lds[kBlock / kWave][2][kWave];
    const uint32_t nr = st->nResearch;
    const int k = a.k;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t nw = gridDim.x * (kBlock / kWave);
    const uint32_t pool_base = st->pool_count;
    uint32_t tested = 0;
    for (uint32_t t = blockIdx.x * (kBlock / kWave) + w; t < nr; t += nw) {
        const uint32_t z = a.research_list[t];
        const int4 pz = a.pts[z];
        SearchCtx sc{a.alive};
        uint64_t d;
        int32_t id;
        // z's list was full (a re-search follows only a full list), and its
        // K-th distance can only have grown since: start at the finest level
        // whose cell edge reaches the old K-th distance
        const int32_t last = a.nbr[(size_t)z * K + K - 1];
        const int4 pl = a.pts[(uint32_t)last];
        const uint64_t dold = dist2(pz.x, pz.y, pz.z, pl.x, pl.y, pl.z);
        int sn = 0;
        while (sn < 21 && (1ull << (2 * sn)) < dold) sn++;
        const int L0 = min(max(sn - g.lv[0].s, 0), g.nlev - 1);
        wave_knn<K, kAlive>(g, z, pz, sc, K, L0, d, id, lds[w][0], lds[w][1], &tested);
        const int c = __popcll(__ballot(lane < K && d != ~0ull));
        const int use = c < k ? c : k;
        const uint64_t wsum = wave_sum64(lane < use ? cost_term(d) : 0ull);
        if (lane < K) a.nbr[(size_t)z * K + lane] = id;
        if (lane == 0) {
            a.cnt[z] = (uint8_t)c;
            if (a.check && wsum > a.cost[z]) st->err = 7;
            a.cost[z] = wsum;
            a.win[z] = (uint32_t)((1ull << use) - 1ull);
        }
        // reverse edges of the new members, in pool nodes at fixed slots
        // (K per re-search; rb_pool_end advances the pool past them)
        if (lane < c) {
            const uint64_t node64 = (uint64_t)pool_base + (uint64_t)t * K + (uint64_t)lane;
            const uint32_t node = (uint32_t)node64;
            if (node64 < st->pool_cap) {
                a.pool_src[node] = (int32_t)z;
                a.pool_next[node] = atomicExch(&a.head[id], (int32_t)node);
            } else {
                st->overflow = 1;
            }
        }
    }
    if (lane == 0 && tested) atomicAdd(&st->stat_rtested, (unsigned long long)tested);
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&st->stat_research, nr);
}

__global__ void __launch_bounds__(1024) rb_coarse(RoundArrays a, GridView g, int what) {
    const RoundDev* st = a.st;
    if (st->done || st->err) return;
    for (int L = a.lc; L < g.nlev; L++) {
        const LevelView& lv = g.lv[L];
        const uint32_t b = lv.base, bc = g.lv[L - 1].base, nc = lv.ncells, ncc = g.lv[L - 1].ncells;
        for (uint32_t c = threadIdx.x; c < nc; c += blockDim.x) {
            const uint32_t c0 = a.clo[b + c], c1 = c + 1 < nc ? a.clo[b + c + 1] : ncc;
            if (what == 0) {
                uint32_t s[kLev] = {};
                for (uint32_t u = c0; u < c1; u++)
#pragma unroll
                    for (int j = 0; j < kLev; j++) s[j] += a.cellAlev[(size_t)(bc + u) * kLev + j];
#pragma unroll
                for (int j = 0; j < kLev; j++) a.cellAlev[(size_t)(b + c) * kLev + j] = s[j];
            } else {
                uint32_t s = 0;
                for (uint32_t u = c0; u < c1; u++) s += a.cell_alive[bc + u];
                a.cell_alive[b + c] = s;
            }
        }
        __syncthreads();
    }
}

// First child (index at the level below) of every cell of the levels >= lc.
__global__ void __launch_bounds__(kBlock) coarse_clo_k(const uint32_t* __restrict__ parent, uint32_t nchild,
                                                      uint32_t* __restrict__ clo) {
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < nchild; u += gridDim.x * blockDim.x)
        if (u == 0 || parent[u] != parent[u - 1]) clo[parent[u]] = u;
}

// Advances the reverse-list pool past the re-searches' nodes.
__global__ void rb_pool_end(RoundArrays a) {
    RoundDev* st = a.st;
    if (st->done || st->err) return;
    const uint64_t used = (uint64_t)st->pool_count + (uint64_t)st->nResearch * (uint64_t)a.K;
    if (used > st->pool_cap) st->overflow = 1;
    st->pool_count = (uint32_t)(used < st->pool_cap ? used : st->pool_cap);
}


// ---------------------------------------------------------------------------
// reverse lists
// ---------------------------------------------------------------------------

// Reverse lists of the alive points' list entries that are alive (a removed
// entry is never removed again, so nothing needs to find it): one thread per
// (point of the list L, entry).  fill = 0 counts, fill = 1 places.
__global__ void __launch_bounds__(kBlock) rev_k(RoundArrays a, const uint32_t* __restrict__ L, uint32_t m,
                                                uint32_t* deg, int fill) {
    const int K = a.K;
    const uint64_t total = (uint64_t)m * (uint64_t)K;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t z = L[t / (uint32_t)K];
        const int j = (int)(t % (uint32_t)K);
        if (!a.alive[z] || j >= a.cnt[z]) continue;
        const uint32_t y = (uint32_t)a.nbr[(size_t)z * K + j];
        if (!a.alive[y]) continue;
        if (fill) a.rev_src[a.rev_off[y] + atomicAdd(&deg[y], 1u)] = (int32_t)z;
        else atomicAdd(&deg[y], 1u);
    }
}

__global__ void rev_reset_k(RoundArrays a) {
    a.st->pool_count = 0;
    a.st->overflow = 0;
}

// ---------------------------------------------------------------------------
// setup and finalisation
// ---------------------------------------------------------------------------

__global__ void rd_init(RoundDev* st, uint32_t n, uint32_t target, uint32_t pool_cap, float frac) {
    RoundDev z = {};
    z.n_alive = n;
    z.n_alive_new = n;
    z.n_list = n;
    z.target = target;
    z.pool_cap = pool_cap;
    z.frac = frac;
    z.frac_max = fminf(4.0f * frac, 1.0f);
    *st = z;
}

// Search view over the alive points: a compacted copy of the sorted points
// that are alive (Morton order kept, sorted position in .w) and, for every
// cell of every level, its range in that copy.  Re-searches scan it instead
// of the full point array, whose cells fill up with removed points.
__global__ void __launch_bounds__(kBlock) av_flag_k(const uint8_t* __restrict__ alive, uint32_t n,
                                                    uint32_t* __restrict__ flag) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) flag[j] = alive[j];
}

__global__ void __launch_bounds__(kBlock) av_pack_k(const int4* __restrict__ pts, const uint8_t* __restrict__ alive,
                                                    const uint32_t* __restrict__ pos, uint32_t n,
                                                    int4* __restrict__ apts) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        if (alive[j]) {
            const int4 p = pts[j];
            apts[pos[j]] = make_int4(p.x, p.y, p.z, (int)j);
        }
}

__global__ void __launch_bounds__(kBlock) av_start_k(const uint32_t* __restrict__ start, uint32_t nc,
                                                     const uint32_t* __restrict__ pos, uint32_t* __restrict__ astart) {
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c <= nc; c += gridDim.x * blockDim.x)
        astart[c] = pos[start[c]];
}

// The cost of a fresh list sums its first min(k, cnt) entries.
__global__ void __launch_bounds__(kBlock) win_init_k(const uint8_t* __restrict__ cnt, uint32_t n, int k,
                                                     uint32_t* __restrict__ win) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const int c = cnt[j] < k ? cnt[j] : k;
        win[j] = (uint32_t)((1ull << c) - 1ull);
    }
}

// Runs of identical coordinates (equal Morton codes, hence adjacent in the
// sorted order): the first point of a run writes the run to all its points.
__global__ void __launch_bounds__(kBlock) grp_init_k(const int4* __restrict__ pts, const uint32_t* __restrict__ seg,
                                                     uint32_t n, uint32_t* __restrict__ lo, uint32_t* __restrict__ hi) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const int4 p = pts[j];
        const uint32_t sj = seg ? seg[j] : 0u;
        if (j > 0) {
            const int4 q = pts[j - 1];
            if (q.x == p.x && q.y == p.y && q.z == p.z && (seg ? seg[j - 1] : 0u) == sj) continue;
        }
        uint32_t e = j + 1;
        while (e < n) {
            const int4 q = pts[e];
            if (q.x != p.x || q.y != p.y || q.z != p.z || (seg ? seg[e] : 0u) != sj) break;
            e++;
        }
        for (uint32_t i = j; i < e; i++) {
            lo[i] = j;
            hi[i] = e;
        }
    }
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

// segment of original index o (device offsets, nseg + 1 entries)
__device__ inline uint32_t seg_of_orig(const int64_t* __restrict__ off, int nseg, uint32_t o) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int m = (lo + hi + 1) >> 1;
        if ((uint64_t)off[m] <= o) lo = m; else hi = m - 1;
    }
    return (uint32_t)lo;
}

// kept indices from global to per-cloud (the global order is already
// cloud-major because the clouds are contiguous in the input)
__global__ void __launch_bounds__(kBlock) kept_local_k(int32_t* __restrict__ kept, uint32_t m,
                                                       const int64_t* __restrict__ off, int nseg) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        const uint32_t o = (uint32_t)kept[t];
        kept[t] = (int32_t)(o - (uint32_t)off[seg_of_orig(off, nseg, o)]);
    }
}

// third pass of the removal order of a batch: by cloud (stable)
__global__ void __launch_bounds__(kBlock) ev_keys3_k(const uint32_t* __restrict__ v2, uint32_t m,
                                                     const int64_t* __restrict__ off, int nseg,
                                                     uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        keys[t] = seg_of_orig(off, nseg, v2[t]);
        vals[t] = t;
    }
}

__global__ void __launch_bounds__(kBlock) ev_out3_k(const uint64_t* __restrict__ k2, const uint32_t* __restrict__ v2,
                                                    const uint32_t* __restrict__ v3, uint32_t m,
                                                    const int64_t* __restrict__ off, int nseg,
                                                    int32_t* __restrict__ order, uint64_t* __restrict__ order_cost) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        const uint32_t i = v3[t], o = v2[i];
        if (order) order[t] = (int32_t)(o - (uint32_t)off[seg_of_orig(off, nseg, o)]);
        if (order_cost) order_cost[t] = ~k2[i];
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
    kSWin, kSResearch, kSR, kSEvC, kSEvO, kSHist, kSRevOff, kSRevSrc, kSHead, kSPoolS, kSPoolN, kSSt, kSTmp,
    kSFin1, kSFin2, kSSurv,
    kSCellAlive = 60, kSCellA, kSDgC, kSDgO, kSDgD, kSSurvOff, kSSurvList, kSSurvBucket, kSCS, kSGrpLo, kSGrpHi,
    kSGSafe, kSAPts, kSAStart, kSAFlag, kSAPos,
    kSOvfK0 = 89, kSOvfV0, kSOvfK1, kSOvfV1, kSSegFirst, kSSeg, kSOff, kSSegCnt, kSSegGlob, kSSegTopC, kSSegTopO,
    kSPool0 = 101, kSPool1, kSClo, kSSwCnt = 105
};
// levels with at most this many cells are counted by rb_coarse
constexpr uint32_t kCoarseCells = 4096;
static_assert(kSSurv < 40, "scratch slots overlap the scan's");
static_assert(kSAPos < 76 && kSSegTopO < kScratchSlots, "scratch slots beyond the context's table");

// L, m: a list holding every alive point (dead entries are skipped)
int build_reverse(Ctx* c, RoundArrays& a, uint32_t n, const uint32_t* L, uint32_t m) {
    uint32_t* deg = (uint32_t*)scratch(c, kSTmp, (size_t)(n + 1) * 4);
    if (!deg) return PDD_ENOMEM;
    int rc;
    if ((rc = fill_u32(c, deg, 0, n + 1))) return rc;
    const unsigned gr = (unsigned)std::min<uint64_t>(((uint64_t)m * a.K + kBlock - 1) / kBlock, 16384u);
    hipLaunchKernelGGL(rev_k, dim3(std::max(gr, 1u)), dim3(kBlock), 0, c->stream, a, L, m, deg, 0);
    PDD_HIP(c, hipGetLastError());
    if ((rc = exclusive_scan_u32_u64(c, deg, a.rev_off, n + 1))) return rc;
    // the fill pass counts again from zero within each point's run
    if ((rc = fill_u32(c, deg, 0, n + 1))) return rc;
    hipLaunchKernelGGL(rev_k, dim3(std::max(gr, 1u)), dim3(kBlock), 0, c->stream, a, L, m, deg, 1);
    PDD_HIP(c, hipGetLastError());
    if ((rc = fill_u32(c, (uint32_t*)a.head, 0xFFFFFFFFu, n))) return rc;
    hipLaunchKernelGGL(rev_reset_k, dim3(1), dim3(1), 0, c->stream, a);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

// (Re)builds the alive search view gs of grid g.
int build_alive_view(Ctx* c, RoundArrays& a, const GridView& g, GridView* gs) {
    const uint32_t n = g.n;
    int4* apts = (int4*)scratch(c, kSAPts, (size_t)n * sizeof(int4));
    uint32_t* astart = (uint32_t*)scratch(c, kSAStart, ((size_t)g.total_cells + g.nlev) * 4);
    uint32_t* flag = (uint32_t*)scratch(c, kSAFlag, (size_t)n * 4);
    uint32_t* pos = (uint32_t*)scratch(c, kSAPos, (size_t)(n + 1) * 4);
    if (!apts || !astart || !flag || !pos) return PDD_ENOMEM;
    hipLaunchKernelGGL(av_flag_k, dim3(gfor(n)), dim3(kBlock), 0, c->stream, a.alive, n, flag);
    PDD_HIP(c, hipGetLastError());
    int rc = exclusive_scan_u32(c, flag, pos, n, pos + n);
    if (rc) return rc;
    hipLaunchKernelGGL(av_pack_k, dim3(gfor(n)), dim3(kBlock), 0, c->stream, g.pts, a.alive, pos, n, apts);
    a.apts = apts;
    a.vpos = pos;
    *gs = g;
    gs->pts = apts;
    size_t off = 0;
    for (int L = 0; L < g.nlev; L++) {
        hipLaunchKernelGGL(av_start_k, dim3(gfor(g.lv[L].ncells + 1)), dim3(kBlock), 0, c->stream, g.lv[L].start,
                           g.lv[L].ncells, pos, astart + off);
        gs->lv[L].start = astart + off;
        off += g.lv[L].ncells + 1;
    }
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

// A batch: keep, in each segment whose A exceeds its remaining budget B_s,
// only its top B_s keys (A stays an upper set of every segment's keys).
// Reads the count of such A points back to size the sort.
// A batch's budget cut after the A counts per segment (rb_seg_count,
// rb_seg_over): reads back how many A points lie in segments over budget
// and sorts them, by a sort that this count sizes.
int segment_budgets(Ctx* c, RoundArrays& a) {
    uint32_t* h = (uint32_t*)((char*)c->pinned + 2048);
    PDD_HIP(c, hipMemcpyAsync(h, &a.st->nOvf, 4, hipMemcpyDeviceToHost, c->stream));
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    const uint32_t m = h[0];
    if (m == 0) return PDD_OK;
    uint64_t* k0 = (uint64_t*)scratch(c, kSOvfK0, (size_t)m * 8);
    uint32_t* v0 = (uint32_t*)scratch(c, kSOvfV0, (size_t)m * 4);
    uint64_t* k1 = (uint64_t*)scratch(c, kSOvfK1, (size_t)m * 8);
    uint32_t* v1 = (uint32_t*)scratch(c, kSOvfV1, (size_t)m * 4);
    uint32_t* first = (uint32_t*)scratch(c, kSSegFirst, (size_t)a.nseg * 4);
    if (!k0 || !v0 || !k1 || !v1 || !first) return PDD_ENOMEM;
    int seg_bits = 1;
    while ((1ll << seg_bits) < a.nseg) seg_bits++;
    const int passes[3] = {31, 64, seg_bits};
    const uint32_t* src = a.ovf;
    uint64_t* sk;
    uint32_t* sv = nullptr;
    for (int p = 0; p < 3; p++) {
        uint64_t* kk = (p & 1) ? k1 : k0;
        uint32_t* vv = (p & 1) ? v1 : v0;
        hipLaunchKernelGGL(ovf_keys_k, dim3(gfor(m)), dim3(kBlock), 0, c->stream, a, p, src, m, kk, vv);
        PDD_HIP(c, hipGetLastError());
        int rc = radix_sort_pairs(c, kk, vv, m, passes[p], &sk, &sv);
        if (rc) return rc;
        src = sv;
    }
    hipLaunchKernelGGL(ovf_first_k, dim3(gfor(m)), dim3(kBlock), 0, c->stream, a, sv, m, first);
    hipLaunchKernelGGL(ovf_drop_k, dim3(gfor(m)), dim3(kBlock), 0, c->stream, a, sv, m, first);
    hipLaunchKernelGGL(ovf_compact_k, dim3(1024), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(ovf_copy_k, dim3(1024), dim3(kBlock), 0, c->stream, a);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

// A round in two parts, with a batch's budget cut (sized on the host)
// between them: the selection of A, then the round rule, the removals and
// the re-costing.
void launch_round_a(Ctx* c, RoundArrays& a) {
    const unsigned GS = 1024;  // passes over the alive points or the pool
    hipLaunchKernelGGL(rb_begin, dim3(1), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_seg_reset, dim3(gfor(a.nseg)), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_hist0, dim3(GS), dim3(kBlock), 0, c->stream, a, 0);
    hipLaunchKernelGGL(rb_pool_check, dim3(1), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_hist0, dim3(GS), dim3(kBlock), 0, c->stream, a, 1);
    hipLaunchKernelGGL(rb_find0, dim3(1), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_collect0, dim3(GS), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_refine, dim3(1), dim3(1024), 0, c->stream, a);
    if (a.nseg > 1) {
        hipLaunchKernelGGL(rb_seg_count, dim3(1024), dim3(kBlock), 0, c->stream, a);
        hipLaunchKernelGGL(rb_seg_over, dim3(1024), dim3(kBlock), 0, c->stream, a);
    }
}

template <int K>
int launch_round_b(Ctx* c, RoundArrays& a, const GridView& g, const GridView& gs) {
    // per-item kernels take the configured launch size
    const unsigned G = c->round_blocks;
    int rc = launch_blocking(c, a, g, K);
    if (rc) return rc;
    hipLaunchKernelGGL(rb_remove, dim3(G), dim3(kBlock), 0, c->stream, a, g);
    hipLaunchKernelGGL(rb_remove_end, dim3(1), dim3(1), 0, c->stream, a);
    launch_coarse(c, a, g, 1);
    hipLaunchKernelGGL(rb_touch_recost, dim3(G), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(rb_research<K>, dim3(G), dim3(kBlock), 0, c->stream, a, gs);
    hipLaunchKernelGGL(rb_pool_end, dim3(1), dim3(1), 0, c->stream, a);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

template <int K>
int launch_round(Ctx* c, RoundArrays& a, const GridView& g, const GridView& gs) {
    launch_round_a(c, a);
    PDD_HIP(c, hipGetLastError());
    int rc;
    if (a.nseg > 1 && (rc = segment_budgets(c, a))) return rc;
    return launch_round_b<K>(c, a, g, gs);
}

// A round's kernels as hipGraphs.  Every kernel of a round reads its sizes
// and decisions from the device state, so one capture serves every round
// with the same arguments.  It is taken once the first round has allocated
// every buffer the round uses, on the context's private capture stream
// (nothing runs there), and again after a rebuild between rounds; the graphs
// are launched on the context's stream.  A single cloud's round is one
// graph.  A batch's round is two, one for each part around the budget cut,
// which sizes its sort on the host and runs eagerly between them (its
// scratch slots are not among those the graphs hold).  A failed capture
// leaves that part eager.
struct RoundGraph {
    hipGraphExec_t exec = nullptr;
    ~RoundGraph() { reset(); }
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
    }
};

template <class Launch>
void capture(Ctx* c, RoundGraph* rg, Launch launch) {
    rg->reset();
    hipStream_t run = c->stream;
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    c->stream = c->cap_stream;
    const int rc = launch();
    c->stream = run;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
    if (rc == PDD_OK && e == hipSuccess && graph) {
        if (hipGraphInstantiate(&rg->exec, graph, nullptr, nullptr, 0) != hipSuccess) rg->exec = nullptr;
    }
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    c->err.clear();
}

template <int K>
int run_rounds(Ctx* c, RoundArrays& a, const GridView& g, uint32_t n) {
    RoundDev* hst = (RoundDev*)c->pinned;
    GridView gs;
    int rc = build_alive_view(c, a, g, &gs);
    if (rc) return rc;
    uint32_t view_alive = n;
    RoundGraph rg, rgb;  // the round (a batch: its part before the budget cut) and a batch's part after it
    const bool graphs = !c->eager && c->cap_stream;
    const bool split = a.nseg > 1;
    for (uint64_t it = 0;; it++) {
        if (!split) {
            if (rg.exec) {
                PDD_HIP(c, hipGraphLaunch(rg.exec, c->stream));
                c->stats[14]++;
            } else if ((rc = launch_round<K>(c, a, g, gs))) {
                return rc;
            }
        } else {
            if (rg.exec) {
                PDD_HIP(c, hipGraphLaunch(rg.exec, c->stream));
                c->stats[14]++;
            } else {
                launch_round_a(c, a);
                PDD_HIP(c, hipGetLastError());
            }
            if ((rc = segment_budgets(c, a))) return rc;
            if (rgb.exec) {
                PDD_HIP(c, hipGraphLaunch(rgb.exec, c->stream));
            } else if ((rc = launch_round_b<K>(c, a, g, gs))) {
                return rc;
            }
        }
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
            c->stats[12] = (int64_t)hst->stat_rtested;
            c->stats[13] = (int64_t)hst->stat_enum;
            return PDD_OK;
        }
        if (c->progress && hst->round % 50 == 0) {
            fprintf(stderr, "pdd: round %u removed %u/%u alive %u A %u removed-now %u danger %u survivors %u "
                    "researched %u enumerated %u frac %g research-tested-total %llu\n", hst->round, hst->removed, hst->target,
                    hst->n_alive_new, hst->nA, hst->nR, hst->nDanger, hst->nSurv, hst->nResearch, hst->work, hst->frac,
                    hst->stat_rtested);
            fflush(stderr);
        }
        // rebuild the reverse lists when the appended chains overflowed or
        // grew longer than twenty nodes per alive point on average
        if (hst->overflow || (uint64_t)hst->pool_count > 20ull * hst->n_alive_new) {
            if ((rc = build_reverse(c, a, n, a.alive_list[hst->apar], hst->n_list))) return rc;
            c->stats[3]++;
            rg.reset();
            rgb.reset();
        }
        // re-pack the alive search view once a fifth of its points are gone
        if ((uint64_t)hst->n_alive_new * 5 < (uint64_t)view_alive * 4) {
            if ((rc = build_alive_view(c, a, g, &gs))) return rc;
            view_alive = hst->n_alive_new;
            rg.reset();
            rgb.reset();
        }
        if (graphs && !rg.exec) {
            if (!split) {
                capture(c, &rg, [&] { return launch_round<K>(c, a, g, gs); });
            } else {
                capture(c, &rg, [&] {
                    launch_round_a(c, a);
                    return PDD_OK;
                });
                capture(c, &rgb, [&] { return launch_round_b<K>(c, a, g, gs); });
            }
        }
        if (it > (uint64_t)n + 16) {
            c->err = "round loop made no progress";
            return PDD_EINTERNAL;
        }
    }
}

}  // namespace

void launch_coarse(Ctx* c, const RoundArrays& a, const GridView& g, int what) {
    if (a.lc < g.nlev) hipLaunchKernelGGL(rb_coarse, dim3(1), dim3(1024), 0, c->stream, a, g, what);
}

int decimate(Ctx* c, const Grid& grid, int k, int K, float frac, int check, const int64_t* h_off,
             const int64_t* h_keep, int nseg, int32_t* kept, int32_t* order, uint64_t* order_cost) {
    const GridView& g = grid.v;
    const uint32_t n = g.n;
    int64_t keep = 0;
    std::vector<uint32_t> left((size_t)nseg);
    for (int s = 0; s < nseg; s++) {
        keep += h_keep[s];
        left[s] = (uint32_t)(h_off[s + 1] - h_off[s] - h_keep[s]);
    }
    const uint32_t target = (uint32_t)(n - keep);
    RoundArrays a{};
    a.pts = g.pts;
    a.of0 = g.of0;
    const uint32_t tcells = g.total_cells;
    a.k = k;
    a.K = K;
    a.frac = frac;
    a.check = check;
    // pool nodes are int32 indices; a full pool only triggers a rebuild
    const size_t pool_cap = std::min<size_t>((size_t)n * K, (size_t)0x7FFFFFFF);
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
    ALLOC(win, kSWin, (size_t)n * 4);
    ALLOC(surv, kSSurv, (size_t)n * 4);
    ALLOC(alive_list[0], kSAl0, (size_t)n * 4);
    ALLOC(alive_list[1], kSAl1, (size_t)n * 4);
    ALLOC(pool_list[0], kSPool0, (size_t)n * 4);
    ALLOC(pool_list[1], kSPool1, (size_t)n * 4);
    ALLOC(A, kSA, (size_t)n * 4);
    ALLOC(cand[0], kSC0, (size_t)n * 4);
    ALLOC(cand[1], kSC1, (size_t)n * 4);
    ALLOC(dg_y, kSDgY, (size_t)n * 4);
    ALLOC(dg_tc, kSDgC, (size_t)n * 8);
    ALLOC(dg_to, kSDgO, (size_t)n * 4);
    ALLOC(dg_dlast, kSDgD, (size_t)n * 8);
    ALLOC(research_list, kSResearch, (size_t)n * 4);
    ALLOC(R, kSR, (size_t)n * 4);
    ALLOC(ev_cost, kSEvC, (size_t)n * 8);
    ALLOC(ev_orig, kSEvO, (size_t)n * 4);
    ALLOC(hist, kSHist, (size_t)kSelBins0 * 4);
    ALLOC(rev_off, kSRevOff, (size_t)(n + 1) * 8);
    ALLOC(rev_src, kSRevSrc, (size_t)n * K * 4);
    ALLOC(head, kSHead, (size_t)n * 4);
    ALLOC(pool_src, kSPoolS, pool_cap * 4);
    ALLOC(pool_next, kSPoolN, pool_cap * 4);
    ALLOC(cell_alive, kSCellAlive, (size_t)tcells * 4);
    ALLOC(cellAlev, kSCellA, (size_t)tcells * kLev * 4);
    ALLOC(clo, kSClo, (size_t)tcells * 4);
    a.lc = g.nlev;
    for (int L = 1; L < g.nlev; L++)
        if (g.lv[L].ncells <= kCoarseCells) {
            a.lc = L;
            break;
        }
    a.nwords = (n + 63) / 64;
    ALLOC(sbits, kSCS, (size_t)a.nwords * 8);
    ALLOC(swcnt, kSSwCnt, (size_t)(a.nwords + 1) * 4);
    ALLOC(swpre, kSSurvOff, (size_t)(a.nwords + 1) * 4);
    ALLOC(surv_list, kSSurvList, (size_t)n * 4);
    // a round's A holds at most ceil(frac_max * alive) points (rb_begin),
    // frac_max = min(4 frac, 1) as rd_init sets it
    {
        const float fmax = std::fmin(4.0f * frac, 1.0f);
        const double cap = std::ceil((double)fmax * (double)n) + 1.0;
        a.rec_cap = cap >= (double)n ? n : (uint32_t)cap;
    }
    ALLOC(surv_rec, kSSurvBucket, (size_t)a.rec_cap * sizeof(SurvRec));
    uint32_t *glo, *ghi;
    if (!(glo = (uint32_t*)scratch(c, kSGrpLo, (size_t)n * 4)) || !(ghi = (uint32_t*)scratch(c, kSGrpHi, (size_t)n * 4)))
        return PDD_ENOMEM;
    a.grp_lo = glo;
    a.grp_hi = ghi;
    ALLOC(gsafe, kSGSafe, (size_t)n * 4);
    a.nseg = nseg;
    a.seg = g.seg;
    ALLOC(seg_left, kSSeg, (size_t)nseg * 4);
    ALLOC(seg_cntA, kSSegCnt, (size_t)nseg * 4);
    ALLOC(seg_glob, kSSegGlob, (size_t)nseg * kLev * 8);
    ALLOC(seg_top_cost, kSSegTopC, (size_t)nseg * 8);
    ALLOC(seg_top_orig, kSSegTopO, (size_t)nseg * 4);
    a.ovf = a.R;  // the removal list is free while A is selected
    ALLOC(st, kSSt, sizeof(RoundDev));
#undef ALLOC
    int rc;
    if ((rc = fill_u8(c, a.alive, 1, n))) return rc;
    if ((rc = fill_u32(c, a.inA, 0, n))) return rc;
    if ((rc = fill_u32(c, a.blocked, 0, n))) return rc;
    if ((rc = fill_u32(c, a.touched, 0, n))) return rc;
    if ((rc = fill_u32(c, a.surv, 0, n))) return rc;
    if ((rc = fill_u32(c, a.cellAlev, 0, (size_t)tcells * kLev))) return rc;
    if ((rc = fill_u32(c, (uint32_t*)a.sbits, 0, (size_t)a.nwords * 2))) return rc;
    if ((rc = fill_u32(c, a.gsafe, 0, n))) return rc;
    PDD_HIP(c, hipMemcpyAsync(a.seg_left, left.data(), (size_t)nseg * 4, hipMemcpyHostToDevice, c->stream));
    int64_t* doff = (int64_t*)scratch(c, kSOff, (size_t)(nseg + 1) * 8);
    if (!doff) return PDD_ENOMEM;
    PDD_HIP(c, hipMemcpyAsync(doff, h_off, (size_t)(nseg + 1) * 8, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(grp_init_k, dim3(gfor(n)), dim3(kBlock), 0, c->stream, g.pts, g.seg, n, glo, ghi);
    if ((rc = iota_u32(c, a.alive_list[0], n))) return rc;
    for (int L = 0; L < g.nlev; L++)
        hipLaunchKernelGGL(cell_count_k, dim3(gfor(g.lv[L].ncells)), dim3(kBlock), 0, c->stream, g.lv[L].start,
                           g.lv[L].ncells, a.cell_alive + g.lv[L].base);
    for (int L = a.lc; L < g.nlev; L++)
        hipLaunchKernelGGL(coarse_clo_k, dim3(gfor(g.lv[L - 1].ncells)), dim3(kBlock), 0, c->stream, g.lv[L - 1].parent,
                           g.lv[L - 1].ncells, a.clo + g.lv[L].base);
    hipLaunchKernelGGL(rd_init, dim3(1), dim3(1), 0, c->stream, a.st, n, target, (uint32_t)pool_cap, frac);
    PDD_HIP(c, hipGetLastError());

    KnnOut ko{a.nbr, a.cnt, a.cost, nullptr};
    mark(c, kPhGrid);
    if ((rc = knn_all(c, g, k, K, ko, nullptr))) return rc;
    hipLaunchKernelGGL(win_init_k, dim3(gfor(n)), dim3(kBlock), 0, c->stream, a.cnt, n, k, a.win);
    PDD_HIP(c, hipGetLastError());
    mark(c, kPhKnn);
    if ((rc = build_reverse(c, a, n, a.alive_list[0], n))) return rc;
    mark(c, kPhReverse);
    c->stats[3] = 0;
    c->stats[14] = 0;

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
    if (nseg > 1)
        hipLaunchKernelGGL(kept_local_k, dim3(gfor(keep)), dim3(kBlock), 0, c->stream, kept, (uint32_t)keep, doff, nseg);
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
        if (nseg == 1) {
            hipLaunchKernelGGL(ev_out_k, dim3(gfor(target)), dim3(kBlock), 0, c->stream, sk, sv, target, order,
                               order_cost);
        } else {
            // cloud-major: a stable third pass by cloud, indices made per-cloud
            uint64_t* k3 = (uint64_t*)scratch(c, kSOvfK0, (size_t)target * 8);
            uint32_t* v3 = (uint32_t*)scratch(c, kSOvfV0, (size_t)target * 4);
            uint64_t* k2s = (uint64_t*)scratch(c, kSOvfK1, (size_t)target * 8);
            uint32_t* v2s = (uint32_t*)scratch(c, kSOvfV1, (size_t)target * 4);
            if (!k3 || !v3 || !k2s || !v2s) return PDD_ENOMEM;
            PDD_HIP(c, hipMemcpyAsync(k2s, sk, (size_t)target * 8, hipMemcpyDeviceToDevice, c->stream));
            PDD_HIP(c, hipMemcpyAsync(v2s, sv, (size_t)target * 4, hipMemcpyDeviceToDevice, c->stream));
            hipLaunchKernelGGL(ev_keys3_k, dim3(gfor(target)), dim3(kBlock), 0, c->stream, v2s, target, doff, nseg, k3,
                               v3);
            PDD_HIP(c, hipGetLastError());
            int sbits = 1;
            while ((1ll << sbits) < nseg) sbits++;
            uint64_t* sk3;
            uint32_t* sv3;
            if ((rc = radix_sort_pairs(c, k3, v3, target, sbits, &sk3, &sv3))) return rc;
            hipLaunchKernelGGL(ev_out3_k, dim3(gfor(target)), dim3(kBlock), 0, c->stream, k2s, v2s, sv3, target, doff,
                               nseg, order, order_cost);
        }
        PDD_HIP(c, hipGetLastError());
    }
    mark(c, kPhFinal);
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    return PDD_OK;
}

}  // namespace pdd
