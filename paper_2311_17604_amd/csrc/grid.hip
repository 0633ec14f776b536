// Voxel grid: bounds, Morton order, cell table and cell hash.
//
// Sec. 5 voxelises the cloud and searches the k-neighbourhood in a point's
// voxel and its 26 neighbours.  Here voxels are cubes of 2^s mm; points are
// sorted by the Morton code of their coordinates relative to the minimum
// corner, so every voxel (and every coarser Morton cell) is a contiguous run
// of the sorted array.
#include <vector>

#include "common.h"

namespace pdd {

namespace {

__global__ void __launch_bounds__(kBlock) bounds_init(int32_t* b, int nseg) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 6 * nseg; i += gridDim.x * blockDim.x)
        b[i] = (i % 6) < 3 ? INT32_MAX : INT32_MIN;
}

// segment of input point i: the last s with off[s] <= i
__device__ inline uint32_t seg_of(const int64_t* __restrict__ off, int nseg, uint64_t i) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int m = (lo + hi + 1) >> 1;
        if ((uint64_t)off[m] <= i) lo = m; else hi = m - 1;
    }
    return (uint32_t)lo;
}

// per-segment minimum and maximum of each axis, b[6 s + a]: each thread
// takes a run of kBoundsRun points, keeps running bounds while the segment
// stays the same, and flushes them with atomics (wave-reduced when the whole
// wave ends in one segment)
constexpr int kBoundsRun = 256;

__device__ inline void bounds_flush(int32_t* b, uint32_t sg, const int32_t* mn, const int32_t* mx) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        atomicMin(&b[6 * sg + a], mn[a]);
        atomicMax(&b[6 * sg + 3 + a], mx[a]);
    }
}

__global__ void __launch_bounds__(kBlock) bounds_k(const int32_t* __restrict__ xyz, uint32_t n, int sw,
                                                   const int64_t* __restrict__ off, int nseg, int32_t* __restrict__ b) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t i0 = t * kBoundsRun, i1 = min(i0 + kBoundsRun, (uint64_t)n);
    int32_t mn[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, mx[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    uint32_t sg = 0;
    uint64_t seg_end = ~0ull;
    if (i0 < i1 && nseg > 1) {
        sg = seg_of(off, nseg, i0);
        seg_end = (uint64_t)off[sg + 1];
    }
    for (uint64_t i = i0; i < i1; i++) {
        if (i >= seg_end) {
            bounds_flush(b, sg, mn, mx);
#pragma unroll
            for (int a = 0; a < 3; a++) {
                mn[a] = INT32_MAX;
                mx[a] = INT32_MIN;
            }
            while (i >= (uint64_t)off[sg + 1]) sg++;
            seg_end = (uint64_t)off[sg + 1];
        }
        const int32_t* p = xyz + i * sw;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            mn[a] = min(mn[a], p[a]);
            mx[a] = max(mx[a], p[a]);
        }
    }
    // threads without points hold the identities; they join any segment
    const bool has = i0 < i1;
    const uint32_t s0 = (uint32_t)__shfl((int)sg, 0, kWave);
    if (__all(!has || sg == s0)) {
#pragma unroll
        for (int a = 0; a < 3; a++)
            for (int o = kWave / 2; o > 0; o >>= 1) {
                mn[a] = min(mn[a], __shfl_xor(mn[a], o, kWave));
                mx[a] = max(mx[a], __shfl_xor(mx[a], o, kWave));
            }
        if ((threadIdx.x & (kWave - 1)) == 0 && __shfl((int)has, 0, kWave)) bounds_flush(b, s0, mn, mx);
    } else if (has) {
        bounds_flush(b, sg, mn, mx);
    }
}

// key = segment << 3 bits_axis | Morton code of the coordinates relative to
// the segment's minimum corner
__global__ void __launch_bounds__(kBlock) morton_k(const int32_t* __restrict__ xyz, uint32_t n, int sw,
                                                   const int64_t* __restrict__ off, int nseg,
                                                   const int32_t* __restrict__ b, int bits_axis,
                                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int32_t* p = xyz + i * sw;
        const uint32_t sg = nseg > 1 ? seg_of(off, nseg, i) : 0u;
        const int32_t* m = b + 6 * sg;
        keys[i] = ((uint64_t)sg << (3 * bits_axis)) |
                  morton3((uint32_t)(p[0] - m[0]), (uint32_t)(p[1] - m[1]), (uint32_t)(p[2] - m[2]));
        vals[i] = (uint32_t)i;
    }
}

// sorted points in coordinates relative to their segment's minimum corner
__global__ void __launch_bounds__(kBlock) permute_k(const int32_t* __restrict__ xyz, int sw,
                                                    const uint64_t* __restrict__ sk, const uint32_t* __restrict__ vals,
                                                    uint32_t n, int bits_axis, const int32_t* __restrict__ b,
                                                    int4* __restrict__ pts, uint32_t* __restrict__ seg) {
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (size_t)gridDim.x * blockDim.x) {
        const uint32_t o = vals[j];
        const uint32_t sg = (uint32_t)(sk[j] >> (3 * bits_axis));
        const int32_t* p = xyz + (size_t)o * sw;
        const int32_t* m = b + 6 * sg;
        pts[j] = make_int4(p[0] - m[0], p[1] - m[1], p[2] - m[2], (int)o);
        if (seg) seg[j] = sg;
    }
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
        of[j] = pos[j] + flag[j] - 1u;
        if (flag[j]) {
            uint32_t c = pos[j];
            start[c] = (uint32_t)j;
            ckey[c] = keys[j] >> (3 * s);
        }
        if (j == 0) start[ncells] = n;
    }
}

// Level l+1 from level l: a new cell starts where the parent code
// (cell code >> 3) changes.
__global__ void __launch_bounds__(kBlock) up_flag_k(const uint64_t* __restrict__ key, uint32_t nc,
                                                    uint32_t* __restrict__ flag) {
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (size_t)gridDim.x * blockDim.x)
        flag[c] = (c == 0 || (key[c] >> 3) != (key[c - 1] >> 3)) ? 1u : 0u;
}

__global__ void __launch_bounds__(kBlock) up_write_k(const uint64_t* __restrict__ key, const uint32_t* __restrict__ start,
                                                     uint32_t nc, uint32_t n, const uint32_t* __restrict__ flag,
                                                     const uint32_t* __restrict__ pos, uint32_t* __restrict__ parent,
                                                     uint32_t* __restrict__ ustart, uint64_t* __restrict__ ukey,
                                                     uint32_t unc) {
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (size_t)gridDim.x * blockDim.x) {
        parent[c] = pos[c] + flag[c] - 1u;
        if (flag[c]) {
            const uint32_t u = pos[c];
            ustart[u] = start[c];
            ukey[u] = key[c] >> 3;
        }
        if (c == 0) ustart[unc] = n;
    }
}

// Occupancy sample for the choice of the finest level: for `ns` points
// spread evenly over the sorted order and every s in [0, 21], the number of
// points sharing the point's cell of edge 2^s, binned by floor(log2) into
// hist[s * 32 + bin].
__global__ void __launch_bounds__(kBlock) occ_sample_k(const uint64_t* __restrict__ keys, uint32_t n, uint32_t ns,
                                                       uint32_t* __restrict__ hist) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    const uint32_t j = (uint32_t)((uint64_t)i * n / ns);
    const uint64_t key = keys[j];
    for (int s = 0; s < 22; s++) {
        const uint64_t p = key >> (3 * s);
        // first index with prefix >= p, first index with prefix > p
        uint32_t lo = 0, hi = j;
        while (lo < hi) {
            const uint32_t m = (lo + hi) >> 1;
            if ((keys[m] >> (3 * s)) < p) lo = m + 1; else hi = m;
        }
        const uint32_t b = lo;
        lo = j + 1;
        hi = n;
        while (lo < hi) {
            const uint32_t m = (lo + hi) >> 1;
            if ((keys[m] >> (3 * s)) <= p) lo = m + 1; else hi = m;
        }
        const uint32_t cnt = lo - b;
        atomicAdd(&hist[s * 32 + (31 - __clz(cnt))], 1u);
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
enum { kSlotBounds = 0, kSlotKeys = 1, kSlotVals = 2, kSlotFlag = 3, kSlotPos = 4, kSlotOff = 5, kSlotOcc = 6 };

}  // namespace

static void free_level(Level* l) {
    if (l->start) (void)hipFree(l->start);
    if (l->key) (void)hipFree(l->key);
    if (l->hkeys) (void)hipFree(l->hkeys);
    if (l->hvals) (void)hipFree(l->hvals);
    if (l->parent) (void)hipFree(l->parent);
    *l = Level();
}

void free_grid(Grid* g) {
    if (g->pts) (void)hipFree(g->pts);
    if (g->of0) (void)hipFree(g->of0);
    if (g->seg) (void)hipFree(g->seg);
    for (auto& l : g->lev) free_level(&l);
    *g = Grid();
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

// number of cells (the scan total), read back
static int read_count(Ctx* c, const uint32_t* dev, uint32_t* out) {
    uint32_t* h = (uint32_t*)c->pinned;
    PDD_HIP(c, hipMemcpyAsync(h, dev, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    *out = h[0];
    return PDD_OK;
}

// hash table from cell code to cell index, capacity >= 2 * ncells
static int build_hash(Ctx* c, Level* l) {
    int rc;
    uint64_t cap = 1024;
    while (cap < 2ull * l->ncells) cap <<= 1;
    if ((rc = alloc_dev(c, (void**)&l->hkeys, cap * 8))) return rc;
    if ((rc = alloc_dev(c, (void**)&l->hvals, cap * 4))) return rc;
    l->hcap = cap;
    hipLaunchKernelGGL(hash_clear_k, dim3(grid_for(cap)), dim3(kBlock), 0, c->stream, l->hkeys, cap);
    hipLaunchKernelGGL(hash_insert_k, dim3(grid_for(l->ncells)), dim3(kBlock), 0, c->stream, l->key, l->ncells,
                       l->hkeys, l->hvals, (uint32_t)(cap - 1));
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

// The finest level: the largest s whose cells hold fewer than 32 points for 90%
// of the points (occupancy seen from the points, which is what a search
// pays), so that the densest regions still get small cells; coarser regions
// use the levels above.
static int choose_finest(Ctx* c, const uint64_t* sk, uint32_t n, int smax, int* s_out) {
    uint32_t* hist = (uint32_t*)scratch(c, kSlotOcc, 22 * 32 * 4);
    if (!hist) return PDD_ENOMEM;
    int rc;
    if ((rc = fill_u32(c, hist, 0, 22 * 32))) return rc;
    const uint32_t ns = n < 4096 ? n : 4096;
    hipLaunchKernelGGL(occ_sample_k, dim3((ns + kBlock - 1) / kBlock), dim3(kBlock), 0, c->stream, sk, n, ns, hist);
    PDD_HIP(c, hipGetLastError());
    uint32_t* h = (uint32_t*)c->pinned;
    PDD_HIP(c, hipMemcpyAsync(h, hist, 22 * 32 * 4, hipMemcpyDeviceToHost, c->stream));
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    int best = 0;
    for (int s = 0; s <= smax; s++) {
        // 90th percentile bin of the counts
        uint32_t acc = 0;
        int p90 = 31;
        for (int b = 0; b < 32; b++) {
            acc += h[s * 32 + b];
            if ((uint64_t)acc * 10 >= (uint64_t)ns * 9) {
                p90 = b;
                break;
            }
        }
        if (p90 <= 4) best = s;  // counts below 32
        else break;
    }
    *s_out = best > 16 ? 16 : best;
    return PDD_OK;
}

int build_grid(Ctx* c, const int32_t* xyz, int64_t n64, int stride, int voxel_log2, Grid* g) {
    const int64_t off[2] = {0, n64};
    return build_grid_seg(c, xyz, n64, stride, voxel_log2, off, 1, g);
}

int build_grid_seg(Ctx* c, const int32_t* xyz, int64_t n64, int stride, int voxel_log2, const int64_t* h_off, int nseg,
                   Grid* g) {
    *g = Grid();
    if (n64 < 2 || n64 >= (int64_t)0x7FFFFFFF || (stride != 12 && stride != 16) || nseg < 1) return PDD_EINVAL;
    if (voxel_log2 != 0 && (voxel_log2 < 2 || voxel_log2 > 20)) return PDD_EINVAL;
    const uint32_t n = (uint32_t)n64;
    const int sw = stride / 4;
    int32_t* bnd = (int32_t*)scratch(c, kSlotBounds, (size_t)nseg * 6 * 4);
    int64_t* doff = (int64_t*)scratch(c, kSlotOff, (size_t)(nseg + 1) * 8);
    uint64_t* keys = (uint64_t*)scratch(c, kSlotKeys, (size_t)n * 8);
    uint32_t* vals = (uint32_t*)scratch(c, kSlotVals, (size_t)n * 4);
    uint32_t* flag = (uint32_t*)scratch(c, kSlotFlag, (size_t)n * 4);
    uint32_t* pos = (uint32_t*)scratch(c, kSlotPos, (size_t)(n + 1) * 4);
    if (!bnd || !doff || !keys || !vals || !flag || !pos) return PDD_ENOMEM;

    PDD_HIP(c, hipMemcpyAsync(doff, h_off, (size_t)(nseg + 1) * 8, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(bounds_init, dim3(grid_for((size_t)nseg * 6)), dim3(kBlock), 0, c->stream, bnd, nseg);
    const size_t nthreads = ((size_t)n + kBoundsRun - 1) / kBoundsRun;
    hipLaunchKernelGGL(bounds_k, dim3((unsigned)((nthreads + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, xyz, n,
                       sw, doff, nseg, bnd);
    PDD_HIP(c, hipGetLastError());
    std::vector<int32_t> hb((size_t)nseg * 6);
    PDD_HIP(c, hipMemcpyAsync(hb.data(), bnd, hb.size() * 4, hipMemcpyDeviceToHost, c->stream));
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    int64_t ext = 0;
    int64_t ext_axis[3] = {0, 0, 0};
    for (int sg = 0; sg < nseg; sg++)
        for (int a = 0; a < 3; a++) {
            const int64_t e = (int64_t)hb[6 * sg + 3 + a] - hb[6 * sg + a];
            if (e >= (1 << 21)) return PDD_ERANGE;
            if (e > ext) ext = e;
            if (e > ext_axis[a]) ext_axis[a] = e;
        }
    int bits_axis = 0;
    while (bits_axis < 21 && ((int64_t)1 << bits_axis) <= ext) bits_axis++;
    if (bits_axis == 0) bits_axis = 1;
    int seg_bits = 0;
    while ((1ll << seg_bits) < nseg) seg_bits++;
    if (3 * bits_axis + seg_bits > 63) return PDD_ERANGE;

    hipLaunchKernelGGL(morton_k, dim3(grid_for(n)), dim3(kBlock), 0, c->stream, xyz, n, sw, doff, nseg, bnd, bits_axis,
                       keys, vals);
    PDD_HIP(c, hipGetLastError());
    uint64_t* sk;
    uint32_t* sv;
    int rc = radix_sort_pairs(c, keys, vals, n, 3 * bits_axis + seg_bits, &sk, &sv);
    if (rc) return rc;

    if ((rc = alloc_dev(c, (void**)&g->pts, (size_t)n * sizeof(int4)))) return rc;
    if (nseg > 1 && (rc = alloc_dev(c, (void**)&g->seg, (size_t)n * 4))) return rc;
    hipLaunchKernelGGL(permute_k, dim3(grid_for(n)), dim3(kBlock), 0, c->stream, xyz, sw, sk, sv, n, bits_axis, bnd,
                       g->pts, g->seg);
    PDD_HIP(c, hipGetLastError());

    int s0 = voxel_log2;
    if (s0 == 0 && (rc = choose_finest(c, sk, n, bits_axis, &s0))) return rc;
    if (s0 > bits_axis) s0 = bits_axis;

    GridView& v = g->v;
    v.pts = g->pts;
    v.n = n;
    v.minx = v.miny = v.minz = 0;  // points are relative to their segment's corner
    v.seg = g->seg;
    v.nseg = nseg;
    v.bits_axis = bits_axis;

    // level 0 from the sorted point codes
    Level* l0 = &g->lev[0];
    hipLaunchKernelGGL(cell_flag_k, dim3(grid_for(n)), dim3(kBlock), 0, c->stream, sk, n, s0, flag);
    PDD_HIP(c, hipGetLastError());
    if ((rc = exclusive_scan_u32(c, flag, pos, n, pos + n))) return rc;
    if ((rc = read_count(c, pos + n, &l0->ncells))) return rc;
    if ((rc = alloc_dev(c, (void**)&l0->start, (size_t)(l0->ncells + 1) * 4))) return rc;
    if ((rc = alloc_dev(c, (void**)&l0->key, (size_t)l0->ncells * 8))) return rc;
    if ((rc = alloc_dev(c, (void**)&g->of0, (size_t)n * 4))) return rc;
    hipLaunchKernelGGL(cell_write_k, dim3(grid_for(n)), dim3(kBlock), 0, c->stream, sk, n, s0, flag, pos, l0->start,
                       l0->key, l0->ncells, g->of0);
    PDD_HIP(c, hipGetLastError());
    if ((rc = build_hash(c, l0))) return rc;
    v.of0 = g->of0;

    // coarser levels from the cells below, until the 3x3x3 block around any
    // cell covers the cloud (cmax <= 1 per axis), at least two levels
    int nlev = 1;
    uint32_t total = l0->ncells;
    for (int l = 0;; l++) {
        const int sl = s0 + l;
        LevelView& lv = v.lv[l];
        Level* L = &g->lev[l];
        bool top = true;
        for (int a = 0; a < 3; a++) {
            lv.cmax[a] = (int32_t)(ext_axis[a] >> sl);
            if (lv.cmax[a] > 1) top = false;
        }
        lv.segshift = 3 * (bits_axis - sl);
        lv.start = L->start;
        lv.hkeys = L->hkeys;
        lv.hvals = L->hvals;
        lv.key = L->key;
        lv.hmask = (uint32_t)(L->hcap - 1);
        lv.ncells = L->ncells;
        lv.s = sl;
        lv.parent = nullptr;
        if ((top && nlev >= 2) || sl >= bits_axis || nlev == kMaxLevels) break;
        // level l + 1
        Level* U = &g->lev[l + 1];
        const uint32_t nc = L->ncells;
        hipLaunchKernelGGL(up_flag_k, dim3(grid_for(nc)), dim3(kBlock), 0, c->stream, L->key, nc, flag);
        PDD_HIP(c, hipGetLastError());
        if ((rc = exclusive_scan_u32(c, flag, pos, nc, pos + nc))) return rc;
        if ((rc = read_count(c, pos + nc, &U->ncells))) return rc;
        if ((rc = alloc_dev(c, (void**)&L->parent, (size_t)nc * 4))) return rc;
        if ((rc = alloc_dev(c, (void**)&U->start, (size_t)(U->ncells + 1) * 4))) return rc;
        if ((rc = alloc_dev(c, (void**)&U->key, (size_t)U->ncells * 8))) return rc;
        hipLaunchKernelGGL(up_write_k, dim3(grid_for(nc)), dim3(kBlock), 0, c->stream, L->key, L->start, nc, n, flag,
                           pos, L->parent, U->start, U->key, U->ncells);
        PDD_HIP(c, hipGetLastError());
        if ((rc = build_hash(c, U))) return rc;
        lv.parent = L->parent;
        v.lv[l + 1].base = total;
        total += U->ncells;
        nlev++;
    }
    v.lv[0].base = 0;
    v.nlev = nlev;
    v.total_cells = total;
    return PDD_OK;
}

}  // namespace pdd
