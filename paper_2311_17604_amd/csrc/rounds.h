// Device state of the removal rounds, shared by rounds.hip and blocking.hip.
#pragma once

#include "search.h"

namespace pdd {

// A is split into kLev key levels per round (equal shares of A by
// first-level bucket); points of a lower level rank below every point of a
// higher one.
constexpr int kLev = 4;

struct RoundDev {
    uint32_t n_alive, n_alive_new, removed, target, m, round, done, err;
    uint32_t nA, nCand, nDanger, nSurv, nTouch, nResearch, nR, mode;
    uint32_t sel_need, sel_bin, pad0, pad1;
    int32_t sel_rem;  // key bits below the first-level prefix
    uint32_t pool_count, pool_cap, overflow;
    uint32_t stat_research, stat_danger, stat_touch, stat_surv;
    uint32_t lev_t[kLev];         // level(x) = #{j >= 1 : bin0(cost x) >= lev_t[j]}
    uint32_t nOvf;                // A points of segments whose A exceeds their budget
    uint32_t nA2;                 // A after the per-segment budget cut
    float frac;                   // share of alive points ranked this round (adapted)
    float frac_max;
    uint32_t work;                // survivors enumerated by the danger checks, this round
    uint32_t pad3;
    // candidate pool: every alive point outside it has bin0(cost) < p_lo, so
    // its members with bin0(cost) >= p_lo are an upper set of the keys
    uint32_t n_list;              // entries of the alive list (dead ones included)
    uint32_t n_list_new;          // its length after this round's compaction (full rounds)
    uint32_t apar;                // which alive-list buffer is current
    uint32_t full;                // this round ranks all alive points (and rebuilds the pool)
    uint32_t pcur, nP, nP_next;   // current pool buffer and its length; length after compaction
    uint32_t p_lo, p_valid;
    uint32_t pad4;
    unsigned long long stat_rtested;  // points looked at by the re-searches, all rounds
    unsigned long long stat_enum;     // survivors enumerated by the danger checks, all rounds
    uint64_t surv_min[kLev];      // lowest survivor cost per key level, this round
};

// A survivor of the round as the danger checks read it: its point (.w the
// original index), cost and sorted index, in one 32-byte record.
struct alignas(16) SurvRec {
    int4 p;
    uint64_t cost;
    uint32_t x;
    uint32_t pad;
};

// scratch slots of the survivor-word scan inside a round (116 .. 119)
constexpr int kSlotSurvScan = 116;

struct RoundArrays {
    const int4* pts;
    const uint32_t* of0;    // [n] level-0 cell of each point
    uint8_t* alive;
    uint64_t* cost;
    int32_t* nbr;       // [n*K]
    uint8_t* cnt;       // [n]
    uint32_t* inA;      // round stamps
    uint32_t* blocked;
    uint32_t* touched;
    uint32_t* win;      // [n] bit j set: entry j of the list is summed in the cost
    uint32_t* surv;
    uint32_t* alive_list[2];
    int4* apts;              // alive search view (.w = -1 once removed)
    const uint32_t* vpos;    // [n] view position of each point alive when it was built
    uint32_t* pool_list[2];  // candidate pool (see RoundDev)
    uint32_t* A;
    uint32_t* cand[2];
    uint32_t* dg_y;      // danger list
    uint64_t* dg_tc;
    int32_t* dg_to;
    uint64_t* dg_dlast;
    uint32_t* research_list;
    uint32_t* R;
    uint64_t* ev_cost;
    int32_t* ev_orig;
    uint32_t* hist;      // [kSelBins0]
    uint64_t* rev_off;   // [n+1] (64-bit: n * K may pass 2^32)
    int32_t* rev_src;    // [n*K]
    int32_t* head;       // [n] pool chains
    int32_t* pool_src;
    int32_t* pool_next;
    uint32_t* cell_alive;   // [total cells] alive points per cell, all levels (index base + cell)
    uint32_t* cellAlev;     // [total cells * kLev] A points per cell and key level, this round
    // Levels >= lc (few, large cells) are not updated point by point, which
    // would make many waves add to the same counters; rb_coarse recomputes
    // them from their children (clo: first child of each cell, by global id)
    int lc;
    uint32_t* clo;
    uint32_t* surv_list;    // [n] survivors of this round
    const uint32_t* grp_lo; // [n] run of points with identical coordinates around each
    const uint32_t* grp_hi; //     point in Morton order: [grp_lo, grp_hi)
    uint32_t* gsafe;        // [n] round stamp: at least k alive identical points rank below
    // segments (independent clouds of one batch; one segment otherwise)
    const uint32_t* seg;    // [n] segment of each point (nullptr: one segment)
    uint32_t* seg_left;     // [nseg] removals still to do
    uint32_t* seg_cntA;     // [nseg] A points, this round
    uint64_t* seg_glob;     // [nseg * kLev] survivors of level j with cost below this wait, this round
    uint64_t* seg_top_cost; // [nseg] highest key of the segment's A (never waits), this round
    int32_t* seg_top_orig;  // [nseg]
    uint32_t* ovf;          // [n] A points of over-budget segments
    // survivors of this round by sorted index: one bit per point, the
    // survivors in each 64-point word and their exclusive scan; a survivor's
    // rank among them places its record (cleared by rb_remove)
    unsigned long long* sbits;  // [nwords]
    uint32_t* swcnt;            // [nwords + 1]
    uint32_t* swpre;            // [nwords + 1]
    uint32_t nwords;
    SurvRec* surv_rec;      // [rec_cap] survivors grouped by level-0 cell, in cell order
    uint32_t rec_cap;       // at least the largest A of any round
    RoundDev* st;
    int k, K;
    float frac;
    int check;
    int nseg;
};

__device__ inline uint32_t seg_of_pt(const RoundArrays& a, uint32_t x) { return a.seg ? a.seg[x] : 0u; }

__device__ inline uint32_t wave_append(uint32_t* counter, bool pred) {
    const uint64_t m = __ballot(pred);
    const uint32_t lane = lane_id();
    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1u;
    uint32_t base = 0;
    if (m && lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, (int)leader, kWave);
    return base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// arr[seg] -= cnt for every thread with cnt > 0; the threads of the block
// that share the first such thread's seg add up in LDS and make one global
// atomic.  Every thread of the block must call it.
__device__ inline void block_seg_sub(uint32_t* arr, uint32_t seg, uint32_t cnt) {
    __shared__ uint32_t s_seg, s_sum;
    if (threadIdx.x == 0) {
        s_seg = 0xFFFFFFFFu;
        s_sum = 0;
    }
    __syncthreads();
    if (cnt) atomicCAS(&s_seg, 0xFFFFFFFFu, seg);
    __syncthreads();
    if (cnt) {
        if (s_seg == seg) atomicAdd(&s_sum, cnt);
        else atomicSub(&arr[seg], cnt);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_sum) atomicSub(&arr[s_seg], s_sum);
}

// arr[seg] = max(arr[seg], v) for every thread with seg != 0xFFFFFFFF, in
// the same way (one global atomic for the block's first segment).
__device__ inline void block_seg_max64(uint64_t* arr, uint32_t seg, uint64_t v) {
    __shared__ uint32_t s_seg;
    __shared__ unsigned long long s_max;
    if (threadIdx.x == 0) {
        s_seg = 0xFFFFFFFFu;
        s_max = 0;
    }
    __syncthreads();
    const bool has = seg != 0xFFFFFFFFu;
    if (has) atomicCAS(&s_seg, 0xFFFFFFFFu, seg);
    __syncthreads();
    if (has) {
        if (s_seg == seg) atomicMax(&s_max, (unsigned long long)v);
        else atomicMax((unsigned long long*)&arr[seg], (unsigned long long)v);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_max) atomicMax((unsigned long long*)&arr[s_seg], s_max);
}

// Space for `cnt` items per thread of a kBlock-thread block: returns the
// thread's first slot; one atomic on `counter` per block.  Every thread of
// the block must call it.
__device__ inline uint32_t block_reserve(uint32_t* counter, uint32_t cnt) {
    constexpr int W = kBlock / kWave;
    __shared__ uint32_t s_w[W + 1];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    uint32_t incl = cnt;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)incl, o, kWave);
        if (lane >= o) incl += v;
    }
    if (lane == kWave - 1) s_w[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < W; w++) {
            const uint32_t t = s_w[w];
            s_w[w] = tot;
            tot += t;
        }
        s_w[W] = tot ? atomicAdd(counter, tot) : 0u;
    }
    __syncthreads();
    const uint32_t r = s_w[W] + s_w[wid] + incl - cnt;
    __syncthreads();
    return r;
}

// First-level bucket of a cost: 0 for 0, else (msb + 1) * 64 + next 6 bits.
// Monotone in the cost.
__device__ inline uint32_t bin0(uint64_t c) {
    if (c == 0) return 0;
    const int e = 63 - __clzll(c);
    const uint32_t mant = e >= 6 ? (uint32_t)(c >> (e - 6)) & 63u : (uint32_t)(c << (6 - e)) & 63u;
    return (uint32_t)(e + 1) * 64u + mant;
}

__device__ inline int level_of(const RoundDev* st, uint64_t cost) {
    const uint32_t b = bin0(cost);
    int l = 0;
#pragma unroll
    for (int j = 1; j < kLev; j++) l += b >= st->lev_t[j];
    return l;
}

// Survivors of this round with sorted index below p (p <= n).
__device__ inline uint32_t surv_rank(const RoundArrays& a, uint32_t p) {
    const uint32_t w = p >> 6, b = p & 63u;
    uint32_t r = a.swpre[w];
    if (b) r += (uint32_t)__popcll(a.sbits[w] & ((1ull << b) - 1ull));
    return r;
}

// Per-cell counts of the levels >= a.lc from the level below, level by
// level, in one block: A points per key level (what = 0) or alive points
// (what = 1).  Children of a cell are a run of the level below (Morton order).
void launch_coarse(Ctx* c, const RoundArrays& a, const GridView& g, int what);

// blocking kernels (blocking.hip), enqueued on the context's stream
int launch_blocking(Ctx* c, const RoundArrays& a, const GridView& g, int K);

}  // namespace pdd
