// Voxel grid: bounds, Morton order, cell table and cell hash.
//
// Sec. 5 voxelises the cloud and searches the k-neighbourhood in a point's
// voxel and its 26 neighbours.  Here voxels are cubes of 2^s mm; points are
// sorted by the Morton code of their coordinates relative to the minimum
// corner, so every voxel (and every coarser Morton cell) is a contiguous run
// of the sorted array.
#include "common.h"

namespace pdd {

namespace {

__global__ void bounds_init(int32_t* b) {
    if (threadIdx.x < 3) b[threadIdx.x] = INT32_MAX;
    else if (threadIdx.x < 6) b[threadIdx.x] = INT32_MIN;
}

__global__ void __launch_bounds__(kBlock) bounds_k(const int32_t* __restrict__ xyz, uint32_t n, int sw,
                                                   int32_t* __restrict__ b) {
    int32_t mn[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, mx[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int32_t* p = xyz + i * sw;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            int32_t v = p[a];
            mn[a] = min(mn[a], v);
            mx[a] = max(mx[a], v);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; a++) {
        for (int o = kWave / 2; o > 0; o >>= 1) {
            mn[a] = min(mn[a], __shfl_xor(mn[a], o, kWave));
            mx[a] = max(mx[a], __shfl_xor(mx[a], o, kWave));
        }
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            atomicMin(&b[a], mn[a]);
            atomicMax(&b[3 + a], mx[a]);
        }
    }
}

__global__ void __launch_bounds__(kBlock) morton_k(const int32_t* __restrict__ xyz, uint32_t n, int sw, int32_t mx,
                                                   int32_t my, int32_t mz, uint64_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int32_t* p = xyz + i * sw;
        keys[i] = morton3((uint32_t)(p[0] - mx), (uint32_t)(p[1] - my), (uint32_t)(p[2] - mz));
        vals[i] = (uint32_t)i;
    }
}

__global__ void __launch_bounds__(kBlock) permute_k(const int32_t* __restrict__ xyz, int sw,
                                                    const uint32_t* __restrict__ vals, uint32_t n,
                                                    int4* __restrict__ pts) {
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (size_t)gridDim.x * blockDim.x) {
        uint32_t o = vals[j];
        const int32_t* p = xyz + (size_t)o * sw;
        pts[j] = make_int4(p[0], p[1], p[2], (int)o);
    }
}

// lev_hist[L] += 1 for each sorted neighbour pair whose codes first differ at
// level L (bit position / 3): that pair is a cell boundary for every s <= L.
__global__ void __launch_bounds__(kBlock) level_hist_k(const uint64_t* __restrict__ keys, uint32_t n,
                                                       uint32_t* __restrict__ lev_hist) {
    __shared__ uint32_t h[22];
    if (threadIdx.x < 22) h[threadIdx.x] = 0;
    __syncthreads();
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x + 1; j < n; j += (size_t)gridDim.x * blockDim.x) {
        uint64_t x = keys[j] ^ keys[j - 1];
        if (x) atomicAdd(&h[(63 - __clzll(x)) / 3], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 22 && h[threadIdx.x]) atomicAdd(&lev_hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void zero22(uint32_t* p) {
    if (threadIdx.x < 22) p[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(kBlock) cell_flag_k(const uint64_t* __restrict__ keys, uint32_t n, int s,
                                                      uint32_t* __restrict__ flag) {
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (size_t)gridDim.x * blockDim.x)
        flag[j] = (j == 0 || (keys[j] >> (3 * s)) != (keys[j - 1] >> (3 * s))) ? 1u : 0u;
}

__global__ void __launch_bounds__(kBlock) cell_write_k(const uint64_t* __restrict__ keys, uint32_t n, int s,
                                                       const uint32_t* __restrict__ flag,
                                                       const uint32_t* __restrict__ pos, uint32_t* __restrict__ start,
                                                       uint64_t* __restrict__ ckey, uint32_t ncells,
                                                       uint32_t* __restrict__ of) {
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (size_t)gridDim.x * blockDim.x) {
        if (of) of[j] = pos[j] + flag[j] - 1u;
        if (flag[j]) {
            uint32_t c = pos[j];
            start[c] = (uint32_t)j;
            ckey[c] = keys[j] >> (3 * s);
        }
        if (j == 0) start[ncells] = n;
    }
}

__global__ void __launch_bounds__(kBlock) hash_clear_k(uint64_t* __restrict__ hk, uint64_t cap) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (size_t)gridDim.x * blockDim.x)
        hk[i] = kEmptyKey;
}

__global__ void __launch_bounds__(kBlock) hash_insert_k(const uint64_t* __restrict__ ckey, uint32_t ncells,
                                                        uint64_t* hk, uint32_t* hv, uint32_t mask) {
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncells; c += (size_t)gridDim.x * blockDim.x) {
        uint64_t key = ckey[c];
        uint32_t s = hash_slot(key, mask);
        for (;;) {
            unsigned long long prev =
                atomicCAS((unsigned long long*)&hk[s], (unsigned long long)kEmptyKey, (unsigned long long)key);
            if (prev == kEmptyKey || prev == key) {
                hv[s] = (uint32_t)c;
                break;
            }
            s = (s + 1) & mask;
        }
    }
}

inline unsigned grid_for(size_t count, unsigned maxg = 16384) {
    size_t g = (count + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > maxg) g = maxg;
    return (unsigned)g;
}

// scratch slots used while building a grid
enum { kSlotBounds = 0, kSlotKeys = 1, kSlotVals = 2, kSlotFlag = 3, kSlotPos = 4, kSlotLev = 5 };

}  // namespace

static void free_level(Level* l) {
    if (l->start) (void)hipFree(l->start);
    if (l->key) (void)hipFree(l->key);
    if (l->hkeys) (void)hipFree(l->hkeys);
    if (l->hvals) (void)hipFree(l->hvals);
    if (l->of) (void)hipFree(l->of);
    *l = Level();
}

void free_grid(Grid* g) {
    if (g->pts) (void)hipFree(g->pts);
    for (auto& l : g->lev) free_level(&l);
    *g = Grid();
}

static int alloc_dev(Ctx* c, void** p, size_t bytes);

// Cells at level s: runs of equal code >> 3s in the sorted keys, their
// starts, a hash table from cell code to cell index, and the cell of every
// sorted point.
static int build_level(Ctx* c, const uint64_t* sk, uint32_t n, int s, uint32_t* flag, uint32_t* pos, Level* l,
                       bool with_of) {
    int rc;
    hipLaunchKernelGGL(cell_flag_k, dim3(grid_for(n)), dim3(kBlock), 0, c->stream, sk, n, s, flag);
    PDD_HIP(c, hipGetLastError());
    if ((rc = exclusive_scan_u32(c, flag, pos, n, pos + n))) return rc;
    uint32_t* hn = (uint32_t*)c->pinned;
    PDD_HIP(c, hipMemcpyAsync(hn, pos + n, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    const uint32_t ncells = hn[0];
    l->ncells = ncells;
    if ((rc = alloc_dev(c, (void**)&l->start, (size_t)(ncells + 1) * 4))) return rc;
    if ((rc = alloc_dev(c, (void**)&l->key, (size_t)ncells * 8))) return rc;
    if (with_of && (rc = alloc_dev(c, (void**)&l->of, (size_t)n * 4))) return rc;
    hipLaunchKernelGGL(cell_write_k, dim3(grid_for(n)), dim3(kBlock), 0, c->stream, sk, n, s, flag, pos, l->start,
                       l->key, ncells, l->of);
    PDD_HIP(c, hipGetLastError());
    uint64_t cap = 1024;
    while (cap < 2ull * ncells) cap <<= 1;
    if ((rc = alloc_dev(c, (void**)&l->hkeys, cap * 8))) return rc;
    if ((rc = alloc_dev(c, (void**)&l->hvals, cap * 4))) return rc;
    l->hcap = cap;
    hipLaunchKernelGGL(hash_clear_k, dim3(grid_for(cap)), dim3(kBlock), 0, c->stream, l->hkeys, cap);
    hipLaunchKernelGGL(hash_insert_k, dim3(grid_for(ncells)), dim3(kBlock), 0, c->stream, l->key, ncells, l->hkeys,
                       l->hvals, (uint32_t)(cap - 1));
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

static int alloc_dev(Ctx* c, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        c->err = "hipMalloc: out of memory";
        return PDD_ENOMEM;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipMalloc");
    return PDD_OK;
}

// Chooses the voxel so that a cell holds about `target` points on average.
static int choose_level(const uint32_t* lev_hist, uint32_t n, int min_s, int max_s, double target) {
    int best = min_s;
    double bestd = 1e300;
    for (int s = min_s; s <= max_s; s++) {
        uint64_t cells = 1;
        for (int L = s; L < 22; L++) cells += lev_hist[L];
        double occ = (double)n / (double)cells;
        double d = occ > target ? occ / target : target / occ;
        if (d < bestd) { bestd = d; best = s; }
    }
    return best;
}

int build_grid(Ctx* c, const int32_t* xyz, int64_t n64, int stride, int voxel_log2, Grid* g) {
    *g = Grid();
    if (n64 < 2 || n64 >= (int64_t)0x7FFFFFFF || (stride != 12 && stride != 16)) return PDD_EINVAL;
    if (voxel_log2 != 0 && (voxel_log2 < 2 || voxel_log2 > 20)) return PDD_EINVAL;
    const uint32_t n = (uint32_t)n64;
    const int sw = stride / 4;
    int32_t* bnd = (int32_t*)scratch(c, kSlotBounds, 64);
    uint64_t* keys = (uint64_t*)scratch(c, kSlotKeys, (size_t)n * 8);
    uint32_t* vals = (uint32_t*)scratch(c, kSlotVals, (size_t)n * 4);
    uint32_t* flag = (uint32_t*)scratch(c, kSlotFlag, (size_t)n * 4);
    uint32_t* pos = (uint32_t*)scratch(c, kSlotPos, (size_t)(n + 1) * 4);
    uint32_t* lev = (uint32_t*)scratch(c, kSlotLev, 32 * 4);
    if (!bnd || !keys || !vals || !flag || !pos || !lev) return PDD_ENOMEM;
    int32_t* hb = (int32_t*)c->pinned;

    hipLaunchKernelGGL(bounds_init, dim3(1), dim3(64), 0, c->stream, bnd);
    hipLaunchKernelGGL(bounds_k, dim3(grid_for(n, 2048)), dim3(kBlock), 0, c->stream, xyz, n, sw, bnd);
    PDD_HIP(c, hipGetLastError());
    PDD_HIP(c, hipMemcpyAsync(hb, bnd, 6 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    int32_t mn[3] = {hb[0], hb[1], hb[2]}, mx[3] = {hb[3], hb[4], hb[5]};
    int64_t ext = 0;
    for (int a = 0; a < 3; a++) {
        int64_t e = (int64_t)mx[a] - mn[a];
        if (e >= (1 << 21)) return PDD_ERANGE;
        if (e > ext) ext = e;
    }
    int bits_axis = 0;
    while (bits_axis < 21 && ((int64_t)1 << bits_axis) <= ext) bits_axis++;
    if (bits_axis == 0) bits_axis = 1;

    hipLaunchKernelGGL(morton_k, dim3(grid_for(n)), dim3(kBlock), 0, c->stream, xyz, n, sw, mn[0], mn[1], mn[2],
                       keys, vals);
    PDD_HIP(c, hipGetLastError());
    uint64_t* sk;
    uint32_t* sv;
    int rc = radix_sort_pairs(c, keys, vals, n, 3 * bits_axis, &sk, &sv);
    if (rc) return rc;

    if ((rc = alloc_dev(c, (void**)&g->pts, (size_t)n * sizeof(int4)))) return rc;
    hipLaunchKernelGGL(permute_k, dim3(grid_for(n)), dim3(kBlock), 0, c->stream, xyz, sw, sv, n, g->pts);
    PDD_HIP(c, hipGetLastError());

    int s = voxel_log2;
    if (s == 0) {
        hipLaunchKernelGGL(zero22, dim3(1), dim3(64), 0, c->stream, lev);
        hipLaunchKernelGGL(level_hist_k, dim3(grid_for(n, 2048)), dim3(kBlock), 0, c->stream, sk, n, lev);
        PDD_HIP(c, hipGetLastError());
        uint32_t* hl = (uint32_t*)c->pinned;
        PDD_HIP(c, hipMemcpyAsync(hl, lev, 22 * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
        PDD_HIP(c, hipStreamSynchronize(c->stream));
        uint32_t lh[22];
        for (int i = 0; i < 22; i++) lh[i] = hl[i];
        s = choose_level(lh, n, 4, 12, 4.0);
    }

    GridView& v = g->v;
    v.pts = g->pts;
    v.n = n;
    v.minx = mn[0];
    v.miny = mn[1];
    v.minz = mn[2];
    // levels s, s+3, ... until one cell per axis covers the cloud (at least two)
    int nlev = 0;
    for (int sl = s;; sl += 3) {
        if (sl > 21) sl = 21;
        Level* l = &g->lev[nlev];
        if ((rc = build_level(c, sk, n, sl, flag, pos, l, nlev < 2))) return rc;
        LevelView& lv = v.lv[nlev];
        lv.start = l->start;
        lv.hkeys = l->hkeys;
        lv.hvals = l->hvals;
        lv.of = l->of;
        lv.hmask = (uint32_t)(l->hcap - 1);
        lv.ncells = l->ncells;
        lv.s = sl;
        bool top = true;
        for (int a = 0; a < 3; a++) {
            lv.cmax[a] = (int32_t)(((int64_t)mx[a] - mn[a]) >> sl);
            if (lv.cmax[a] > 1) top = false;
        }
        nlev++;
        if ((top && nlev >= 2) || sl == 21 || nlev == kMaxLevels) break;
    }
    v.nlev = nlev;
    return PDD_OK;
}

}  // namespace pdd
