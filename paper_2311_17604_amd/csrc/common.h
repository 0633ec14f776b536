// Internal declarations shared by the HIP translation units of libpdd.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/pdd.h"

namespace pdd {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kMaxK = 32;           // k + b <= 32
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint64_t kEmptyKey = ~0ull;
constexpr int kSelBins0 = 4160;     // first-level bins of the threshold select (65 * 64)
constexpr int kSelBins = 4096;      // refinement bins (12-bit digits)
constexpr int kSelFinal = 2048;     // candidates resolved by one block sort
constexpr int kScratchSlots = 128;  // scratch buffers of a context
constexpr int kNumStats = 15;       // counters reported by pdd_last_stats

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

// 21-bit spread for 3-D Morton codes
__host__ __device__ inline uint64_t spread21(uint32_t v) {
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__host__ __device__ inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return spread21(x) | (spread21(y) << 1) | (spread21(z) << 2);
}

// inverse of spread21
__host__ __device__ inline uint32_t compact21(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10C30C30C30C30C3ull;
    x = (x ^ (x >> 4)) & 0x100F00F00F00F00Full;
    x = (x ^ (x >> 8)) & 0x1F0000FF0000FFull;
    x = (x ^ (x >> 16)) & 0x1F00000000FFFFull;
    x = (x ^ (x >> 32)) & 0x1FFFFFull;
    return (uint32_t)x;
}

// exact squared distance of two int32 points whose per-axis difference is
// below 2^21 in magnitude (extent check at grid build)
__device__ inline uint64_t dist2(int ax, int ay, int az, int bx, int by, int bz) {
    uint32_t dx = (uint32_t)abs(ax - bx), dy = (uint32_t)abs(ay - by), dz = (uint32_t)abs(az - bz);
    return (uint64_t)dx * dx + (uint64_t)dy * dy + (uint64_t)dz * dz;
}

// floor(2^56 / D) for D >= 1, 2^58 for D = 0: a double quotient corrected by
// exact integer remainders.
__device__ inline uint64_t cost_term(uint64_t D) {
    if (D == 0) return 1ull << 58;
    const uint64_t num = 1ull << 56;
    double q = 72057594037927936.0 / (double)D;
    uint64_t t = (uint64_t)q;
    int64_t r = (int64_t)(num - t * D);
    while (r < 0) { t--; r += (int64_t)D; }
    while (r >= (int64_t)D) { t++; r -= (int64_t)D; }
    return t;
}

__device__ inline uint32_t hash_slot(uint64_t key, uint32_t mask) {
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 32) & mask;
}

// cell index of a Morton cell key, or kNone
__device__ inline uint32_t hash_find(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                     uint32_t mask, uint64_t key) {
    uint32_t s = hash_slot(key, mask);
    for (;;) {
        uint64_t k = keys[s];
        if (k == key) return vals[s];
        if (k == kEmptyKey) return kNone;
        s = (s + 1) & mask;
    }
}

// key order of the greedy: true when (ca, ia) ranks above (cb, ib)
__device__ inline bool key_above(uint64_t ca, int32_t ia, uint64_t cb, int32_t ib) {
    return ca > cb || (ca == cb && ia < ib);
}

__device__ inline uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// ---------------------------------------------------------------------------
// device views
// ---------------------------------------------------------------------------

constexpr int kMaxLevels = 22;

// Cells of one level: cubes of edge 2^s mm, i.e. runs of equal Morton code
// >> 3s in the sorted points.  Level l has s = s0 + l: each cell is the union
// of the (at most 8) cells below it, and its descendants at every finer
// level are a contiguous run of that level's cells.
struct LevelView {
    const uint32_t* start;    // [ncells + 1] first sorted point of each cell
    const uint64_t* hkeys;    // [hmask + 1] Morton cell codes (kEmptyKey = empty slot)
    const uint32_t* hvals;    // [hmask + 1] cell index
    const uint32_t* parent;   // [ncells] cell one level up (nullptr at the top level)
    const uint64_t* key;      // [ncells] Morton code of each cell (coordinates at this level)
    uint32_t hmask;
    uint32_t ncells;
    uint32_t base;            // index of the level's first cell in the numbering of all levels' cells
    int32_t cmax[3];          // largest cell coordinate per axis (over all segments)
    int32_t s;
    int32_t segshift;         // cell code = segment << segshift | Morton code of the cell coordinates
};

// hash key of cell (x, y, z) of segment sg at a level
__device__ inline uint64_t cell_code(const LevelView& lv, uint32_t sg, int x, int y, int z) {
    return ((uint64_t)sg << lv.segshift) | morton3((uint32_t)x, (uint32_t)y, (uint32_t)z);
}

// The grid: points in Morton order with their original index, and a stack
// of cell levels with edges 2^s0, 2^(s0+1), ... up to one whose 3x3x3 block
// covers the cloud.  A grid may hold several independent clouds
// (segments): the segment is the top of the sort key, so each segment's
// points are contiguous and cells never span two segments; coordinates are
// relative to the segment's minimum corner.
struct GridView {
    const int4* pts;          // [n] x, y, z (relative to the segment's corner), original index
    const uint32_t* of0;      // [n] level-0 cell of each sorted point
    const uint32_t* seg;      // [n] segment of each sorted point (nullptr: one segment)
    uint32_t n;
    uint32_t total_cells;     // cells over all levels
    int32_t minx, miny, minz; // 0: coordinates are already relative
    int32_t nlev;             // >= 1
    int32_t nseg;
    int32_t bits_axis;        // bits per axis of the Morton codes
    LevelView lv[kMaxLevels];
};

__device__ inline uint32_t seg_at(const GridView& g, uint32_t j) { return g.seg ? g.seg[j] : 0u; }

// level-l cell of a level-0 cell
__device__ inline uint32_t cell_up(const GridView& g, uint32_t c0, int l) {
    for (int i = 0; i < l; i++) c0 = g.lv[i].parent[c0];
    return c0;
}

struct Level {
    uint32_t* start = nullptr;
    uint64_t* key = nullptr;
    uint64_t* hkeys = nullptr;
    uint32_t* hvals = nullptr;
    uint32_t* parent = nullptr;
    uint64_t hcap = 0;
    uint32_t ncells = 0;
};

struct Grid {
    GridView v;
    int4* pts = nullptr;
    uint32_t* of0 = nullptr;
    uint32_t* seg = nullptr;
    Level lev[kMaxLevels];
};

// ---------------------------------------------------------------------------
// host side: context and launchers
// ---------------------------------------------------------------------------

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int64_t stats[kNumStats] = {0};
    // scratch pool: grow-only buffers keyed by slot
    struct Buf { void* p = nullptr; size_t bytes = 0; };
    Buf bufs[kScratchSlots];
    void* pinned = nullptr;   // small pinned host buffer for status read-back
    // phase timing (PDD_F_TIMING): events recorded on the context's stream
    bool timing = false;
    bool progress = false;    // PDD_F_PROGRESS: a line to stderr every 50 rounds
    bool eager = false;       // PDD_F_EAGER: no hipGraph replay of the rounds
    hipStream_t cap_stream = nullptr;  // private stream the round graph is captured on (never run)
    unsigned round_blocks = 1024;  // workgroups per launch of the round kernels
    hipEvent_t ev[8] = {};
    float phase_ms[8] = {0};
    // search-radius predictor: fp32 parameters and Adam moments (device)
    float* pred_P = nullptr;
    float* pred_M = nullptr;
    float* pred_V = nullptr;
    int64_t pred_step = 0;
    bool pred_ready = false;   // parameters set or trained
    bool pred_on = false;      // the initial k-NN uses the predicted radius
    float pred_margin = 0.25f; // added to the predicted log2 radius
};

// phase boundaries of a decimation, timed when PDD_F_TIMING is set
enum Phase { kPhStart = 0, kPhGrid, kPhKnn, kPhReverse, kPhRounds, kPhFinal, kPhCount };
inline void mark(Ctx* c, int i) {
    if (c->timing && c->ev[i]) (void)hipEventRecord(c->ev[i], c->stream);
}

// scratch buffer `slot` of at least `bytes` (contents undefined); nullptr on failure
void* scratch(Ctx* c, int slot, size_t bytes);

int hip_fail(Ctx* c, hipError_t e, const char* what);
#define PDD_HIP(c, call)                                            \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return ::pdd::hip_fail((c), e_, #call); \
    } while (0)

// scan / sort (scan_sort.hip)
int exclusive_scan_u32(Ctx* c, const uint32_t* in, uint32_t* out, uint32_t count, uint32_t* total_dev);
// the same with its partial sums in scratch slots slot0 .. slot0 + levels - 1
int exclusive_scan_u32_at(Ctx* c, const uint32_t* in, uint32_t* out, uint32_t count, uint32_t* total_dev,
                          int slot0, int levels);
int exclusive_scan_u32_u64(Ctx* c, const uint32_t* in, uint64_t* out, uint32_t count);
int radix_sort_pairs(Ctx* c, uint64_t* keys, uint32_t* vals, uint32_t n, int bits, uint64_t** keys_out,
                     uint32_t** vals_out);
int fill_u32(Ctx* c, uint32_t* p, uint32_t value, size_t count);
int fill_u8(Ctx* c, uint8_t* p, uint8_t value, size_t count);
int iota_u32(Ctx* c, uint32_t* p, uint32_t count);

// grid (grid.hip)
int build_grid(Ctx* c, const int32_t* xyz, int64_t n, int stride, int voxel_log2, Grid* g);
// several clouds at once: cloud s is points [h_off[s], h_off[s + 1]) (host array)
int build_grid_seg(Ctx* c, const int32_t* xyz, int64_t n, int stride, int voxel_log2, const int64_t* h_off, int nseg,
                   Grid* g);
void free_grid(Grid* g);

// k-NN (knn.hip)
struct KnnOut {
    int32_t* nbr;      // [n * K] sorted-space neighbour positions (-1 pad)
    uint8_t* cnt;      // [n] entries found
    uint64_t* cost;    // [n]
    int64_t* r2k;      // [n] or nullptr
};
int knn_all(Ctx* c, const GridView& g, int k, int K, KnnOut out, int64_t* fallbacks);
// rows of the sorted-space lists (width K) to original order (width Kout <= K)
int knn_to_original(Ctx* c, const GridView& g, int K, int Kout, const KnnOut& in, int32_t* nbr, int64_t* r2k,
                    uint64_t* cost);

}  // namespace pdd
