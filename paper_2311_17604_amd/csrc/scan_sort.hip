// Device-wide exclusive scan and stable LSD radix sort of (uint64 key, uint32 value).
#include "common.h"

namespace pdd {

namespace {

constexpr int kScanIpt = 16;
constexpr int kScanTile = kBlock * kScanIpt;  // 4096

// exclusive scan of one value per thread over a 256-thread block
__device__ uint32_t block_exscan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t wsum[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[wid] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; w++) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

__global__ void __launch_bounds__(kBlock) scan_partials(const uint32_t* __restrict__ in, uint32_t count,
                                                        uint32_t* __restrict__ partial) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (int i = 0; i < kScanIpt; i++) {
        uint64_t e = base + (uint64_t)i * kBlock + threadIdx.x;
        if (e < count) s += in[e];
    }
    uint32_t tot;
    block_exscan(s, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) scan_tiles(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                     uint32_t count, const uint32_t* __restrict__ partial_ex,
                                                     uint32_t* __restrict__ total_dev) {
    __shared__ uint32_t tile[kScanTile + kScanTile / 32];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    // coalesced load into LDS (padded every 32 words against bank conflicts)
    for (int i = 0; i < kScanIpt; i++) {
        uint32_t l = i * kBlock + threadIdx.x;
        uint64_t e = base + l;
        tile[l + (l >> 5)] = e < count ? in[e] : 0u;
    }
    __syncthreads();
    uint32_t v[kScanIpt];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanIpt; i++) {
        uint32_t l = threadIdx.x * kScanIpt + i;
        v[i] = tile[l + (l >> 5)];
        s += v[i];
    }
    uint32_t tot;
    uint32_t run = block_exscan(s, &tot) + (partial_ex ? partial_ex[blockIdx.x] : 0u);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kScanIpt; i++) {
        uint32_t l = threadIdx.x * kScanIpt + i;
        tile[l + (l >> 5)] = run;
        run += v[i];
    }
    __syncthreads();
    for (int i = 0; i < kScanIpt; i++) {
        uint32_t l = i * kBlock + threadIdx.x;
        uint64_t e = base + l;
        if (e < count) out[e] = tile[l + (l >> 5)];
        if (total_dev && e == (uint64_t)count - 1) *total_dev = tile[l + (l >> 5)] + in[e];
    }
}

// 64-bit exclusive scan of 32-bit counts (sums that may pass 2^32): the
// sum of each tile of kScanTile counts, one block's scan of the tile sums,
// then the scan inside each tile on top of its tile's base.
__device__ uint64_t block_exscan64(uint64_t v, uint64_t* total) {
    __shared__ uint64_t wsum[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    uint64_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)x, o, kWave);
        const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(x >> 32), o, kWave);
        if (lane >= o) x += ((uint64_t)hi << 32) | lo;
    }
    if (lane == kWave - 1) wsum[wid] = x;
    __syncthreads();
    uint64_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; w++) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

__global__ void __launch_bounds__(kBlock) scan64_partials(const uint32_t* __restrict__ in, uint32_t count,
                                                          uint64_t* __restrict__ partial) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint64_t s = 0;
    for (int i = 0; i < kScanIpt; i++) {
        const uint64_t e = base + (uint64_t)i * kBlock + threadIdx.x;
        if (e < count) s += in[e];
    }
    uint64_t tot;
    block_exscan64(s, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// one block: partial[0, nb) becomes its exclusive scan
__global__ void __launch_bounds__(kBlock) scan64_bases(uint64_t* __restrict__ partial, uint32_t nb) {
    uint64_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += kBlock) {
        const uint32_t i = b0 + threadIdx.x;
        const uint64_t v = i < nb ? partial[i] : 0ull;
        uint64_t tot;
        const uint64_t ex = block_exscan64(v, &tot);
        if (i < nb) partial[i] = carry + ex;
        carry += tot;
    }
}

__global__ void __launch_bounds__(kBlock) scan64_tiles(const uint32_t* __restrict__ in, uint64_t* __restrict__ out,
                                                       uint32_t count, const uint64_t* __restrict__ base_ex) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    // each thread scans kScanIpt consecutive counts
    const uint64_t e0 = base + (uint64_t)threadIdx.x * kScanIpt;
    uint32_t v[kScanIpt];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanIpt; i++) {
        v[i] = e0 + i < count ? in[e0 + i] : 0u;
        s += v[i];
    }
    uint64_t tot;
    uint64_t run = block_exscan64(s, &tot) + base_ex[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanIpt; i++) {
        if (e0 + i < count) out[e0 + i] = run;
        run += v[i];
    }
}

__global__ void fill_u32_k(uint32_t* p, uint32_t v, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_u8_k(uint8_t* p, uint8_t v, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void iota_u32_k(uint32_t* p, uint32_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)i;
}

__global__ void set_zero_k(uint32_t* p) { *p = 0; }

// ---------------------------------------------------------------------------
// radix sort: 8-bit digits, tiles of 2048 (256 threads x 8 rounds)
// ---------------------------------------------------------------------------
constexpr int kRsIpt = 8;
constexpr int kRsTile = kBlock * kRsIpt;

__global__ void __launch_bounds__(kBlock) rs_hist(const uint64_t* __restrict__ keys, uint32_t n, int shift,
                                                  uint32_t* __restrict__ hist, uint32_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRsTile;
    for (int i = 0; i < kRsIpt; i++) {
        uint64_t e = base + (uint64_t)i * kBlock + threadIdx.x;
        if (e < n) atomicAdd(&h[(uint32_t)(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: within a tile, element order is (round, wave, lane); ranks
// among equal digits come from ballot-matched peers inside a wave and
// per-wave digit counts accumulated over rounds.
__global__ void __launch_bounds__(kBlock) rs_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                     uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                     uint32_t n, int shift, const uint32_t* __restrict__ offs,
                                                     uint32_t nblocks) {
    constexpr int W = kBlock / kWave;
    __shared__ uint32_t whist[W][256];
    __shared__ uint32_t wbase[W][256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t goff[256];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    run[tid] = 0;
    goff[tid] = offs[(uint64_t)tid * nblocks + blockIdx.x];
#pragma unroll
    for (int w = 0; w < W; w++) whist[w][tid] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRsTile;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int i = 0; i < kRsIpt; i++) {
        uint64_t e = base + (uint64_t)i * kBlock + tid;
        bool valid = e < n;
        uint64_t k = valid ? kin[e] : ~0ull;
        uint32_t v = valid ? vin[e] : 0u;
        uint32_t d = (uint32_t)(k >> shift) & 255u;
        uint64_t peers = ~0ull;
#pragma unroll
        for (int b = 0; b < 8; b++) {
            uint32_t bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t rank = __popcll(peers & lt);
        if (rank == 0) whist[wid][d] = __popcll(peers);
        __syncthreads();
        {
            uint32_t r = run[tid];
#pragma unroll
            for (int w = 0; w < W; w++) {
                wbase[w][tid] = r;
                r += whist[w][tid];
                whist[w][tid] = 0;
            }
            run[tid] = r;
        }
        __syncthreads();
        if (valid) {
            uint32_t pos = goff[d] + wbase[wid][d] + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
    }
}

inline unsigned grid_for(size_t count, unsigned maxg = 8192) {
    size_t g = (count + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > maxg) g = maxg;
    return (unsigned)g;
}

}  // namespace

int fill_u32(Ctx* c, uint32_t* p, uint32_t value, size_t count) {
    if (!count) return PDD_OK;
    hipLaunchKernelGGL(fill_u32_k, dim3(grid_for(count)), dim3(kBlock), 0, c->stream, p, value, count);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

int fill_u8(Ctx* c, uint8_t* p, uint8_t value, size_t count) {
    if (!count) return PDD_OK;
    hipLaunchKernelGGL(fill_u8_k, dim3(grid_for(count)), dim3(kBlock), 0, c->stream, p, value, count);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

int iota_u32(Ctx* c, uint32_t* p, uint32_t count) {
    if (!count) return PDD_OK;
    hipLaunchKernelGGL(iota_u32_k, dim3(grid_for(count)), dim3(kBlock), 0, c->stream, p, count);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

// The scan's partial sums take scratch slots slot0, slot0 + 1, ... (one
// per recursion level, at most `levels`): 40..47 by default.
static int scan_level(Ctx* c, const uint32_t* in, uint32_t* out, uint32_t count, uint32_t* total_dev, int level,
                      int slot0, int levels) {
    if (count == 0) {
        if (total_dev) {
            hipLaunchKernelGGL(set_zero_k, dim3(1), dim3(1), 0, c->stream, total_dev);
            PDD_HIP(c, hipGetLastError());
        }
        return PDD_OK;
    }
    uint32_t nb = (count + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        hipLaunchKernelGGL(scan_tiles, dim3(1), dim3(kBlock), 0, c->stream, in, out, count, nullptr, total_dev);
        PDD_HIP(c, hipGetLastError());
        return PDD_OK;
    }
    if (level >= levels) return PDD_EINTERNAL;
    uint32_t* part = (uint32_t*)scratch(c, slot0 + level, (size_t)nb * 2 * sizeof(uint32_t));
    if (!part) return PDD_ENOMEM;
    uint32_t* part_ex = part + nb;
    hipLaunchKernelGGL(scan_partials, dim3(nb), dim3(kBlock), 0, c->stream, in, count, part);
    PDD_HIP(c, hipGetLastError());
    int rc = scan_level(c, part, part_ex, nb, nullptr, level + 1, slot0, levels);
    if (rc) return rc;
    hipLaunchKernelGGL(scan_tiles, dim3(nb), dim3(kBlock), 0, c->stream, in, out, count, part_ex, total_dev);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

int exclusive_scan_u32(Ctx* c, const uint32_t* in, uint32_t* out, uint32_t count, uint32_t* total_dev) {
    return scan_level(c, in, out, count, total_dev, 0, 40, 8);
}

int exclusive_scan_u32_at(Ctx* c, const uint32_t* in, uint32_t* out, uint32_t count, uint32_t* total_dev,
                          int slot0, int levels) {
    return scan_level(c, in, out, count, total_dev, 0, slot0, levels);
}

// out[i] = in[0] + ... + in[i-1] in 64 bits, for i < count.  Scratch slot 51
// holds the tile sums.
int exclusive_scan_u32_u64(Ctx* c, const uint32_t* in, uint64_t* out, uint32_t count) {
    if (count == 0) return PDD_OK;
    const uint32_t nb = (count + kScanTile - 1) / kScanTile;
    uint64_t* part = (uint64_t*)scratch(c, 51, (size_t)nb * sizeof(uint64_t));
    if (!part) return PDD_ENOMEM;
    hipLaunchKernelGGL(scan64_partials, dim3(nb), dim3(kBlock), 0, c->stream, in, count, part);
    hipLaunchKernelGGL(scan64_bases, dim3(1), dim3(kBlock), 0, c->stream, part, nb);
    hipLaunchKernelGGL(scan64_tiles, dim3(nb), dim3(kBlock), 0, c->stream, in, out, count, part);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

// Sorts by the low `bits` bits of the keys (stable).  The result lands in
// either the input buffers or scratch slots 48/49; *keys_out / *vals_out
// point at it.
int radix_sort_pairs(Ctx* c, uint64_t* keys, uint32_t* vals, uint32_t n, int bits, uint64_t** keys_out,
                     uint32_t** vals_out) {
    *keys_out = keys;
    *vals_out = vals;
    if (n <= 1 || bits <= 0) return PDD_OK;
    uint32_t nb = (n + kRsTile - 1) / kRsTile;
    uint64_t* k2 = (uint64_t*)scratch(c, 48, (size_t)n * sizeof(uint64_t));
    uint32_t* v2 = (uint32_t*)scratch(c, 49, (size_t)n * sizeof(uint32_t));
    uint32_t* hist = (uint32_t*)scratch(c, 50, (size_t)nb * 256 * 2 * sizeof(uint32_t));
    if (!k2 || !v2 || !hist) return PDD_ENOMEM;
    uint32_t* offs = hist + (size_t)nb * 256;
    uint64_t* ka = keys;
    uint32_t* va = vals;
    uint64_t* kb = k2;
    uint32_t* vb = v2;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(rs_hist, dim3(nb), dim3(kBlock), 0, c->stream, ka, n, shift, hist, nb);
        PDD_HIP(c, hipGetLastError());
        int rc = exclusive_scan_u32(c, hist, offs, nb * 256, nullptr);
        if (rc) return rc;
        hipLaunchKernelGGL(rs_scatter, dim3(nb), dim3(kBlock), 0, c->stream, ka, va, kb, vb, n, shift, offs, nb);
        PDD_HIP(c, hipGetLastError());
        uint64_t* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
    }
    *keys_out = ka;
    *vals_out = va;
    return PDD_OK;
}

}  // namespace pdd
