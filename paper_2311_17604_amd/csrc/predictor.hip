// Learned bound on the k-NN search radius.
//
// Sec. 5 searches a point's k+b neighbourhood in a fixed block of voxels
// around it.  Here the k-NN runs in tiles, one per anchor cell (the finest
// cell around a point that holds K+1 points), over a region of cells around
// it; a small network predicts, from the occupancy of the 4x4x4 half-size
// cells around the anchor, by how much the anchor cell must be grown for the
// region to hold every anchored point's K nearest.  The tile then loads only
// that region (when it is smaller than the default one) and keeps a list
// when its K-th distance lies inside the region (then it is exact: every
// nearer point was tested); other points fall back to the shell search.
// The prediction can cost time but never changes a result.
//
// Network: 64 -> 64 -> 64 -> 1 with ReLU, parameters flat in fp32
// (W1 [64 in][64 out], b1, W2, b2, w3, b3); the two 64x64 products run on
// MFMA in bf16 with fp32 accumulation (v_mfma_f32_16x16x16_bf16: lane l holds
// A row l%16 and B/D column l%16, k or row 4*(l/16)+v).  Features are
// log1p(count) in bf16; the output is log2(radius / cell edge).  Training
// minimises the pinball loss at level tau (predictions above the targets for
// tau > 1/2) with Adam, one fused forward+backward+update kernel per step.
#include <math.h>

#include <algorithm>

#include "predictor.h"

namespace pdd {

namespace {

constexpr int kF = 64;
constexpr int oW1 = 0, oB1 = 4096, oW2 = 4160, oB2 = 8256, oW3 = 8320, oB3 = 8384;
static_assert(oB3 + 1 == kPredParams, "parameter layout");
constexpr int kTB = 128;  // largest training minibatch

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline f4 mfma16(bf4 a, bf4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }

// A operand: rows r0 + l%16, columns 16ks + 4(l/16) + v of a row-major
// [*, 64] bf16 matrix.
__device__ inline bf4 frag_rows(const uint16_t* M, int r0, int ks, int lane) {
    const uint16_t* p = M + (size_t)(r0 + (lane & 15)) * kF + 16 * ks + 4 * (lane >> 4);
    bf4 a;
#pragma unroll
    for (int v = 0; v < 4; v++) a[v] = (short)p[v];
    return a;
}

// B operand: rows 16ks + 4(l/16) + v, column 16nb + l%16 of a row-major
// [*, 64] bf16 matrix.  (Also the A operand of the transpose: A[i][k] =
// M[k][i] with i = 16nb + l%16.)
__device__ inline bf4 frag_cols(const uint16_t* M, int ks, int nb, int lane) {
    bf4 b;
#pragma unroll
    for (int v = 0; v < 4; v++) b[v] = (short)M[(size_t)(16 * ks + 4 * (lane >> 4) + v) * kF + 16 * nb + (lane & 15)];
    return b;
}

// sum over the 16 lanes that share lane / 16 (one D row group)
__device__ inline float row_sum16(float v) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// sum over the 4 lanes that share lane % 16 (one D column)
__device__ inline float col_sum4(float v) {
    v += __shfl_xor(v, 16, kWave);
    v += __shfl_xor(v, 32, kWave);
    return v;
}

// ---------------------------------------------------------------------------
// anchors, features, targets
// ---------------------------------------------------------------------------

// Marks the anchor cell (level >= 1) of every point.  With dK (squared
// distance to the point's K-th neighbour), also the expansion of the anchor
// cell that the point needs: its K-th distance (rounded up) less its
// distance to the nearest coordinate outside the cell, maximised over the
// cell's points into tmax (non-negative; 0 when every point's list lies
// inside the cell).  A tile whose region is the anchor cell grown by that
// much certifies all its points.
__global__ void __launch_bounds__(kBlock) pr_mark_k(GridView g, uint32_t need, uint32_t* __restrict__ flag,
                                                    const uint64_t* __restrict__ dK, int64_t* __restrict__ tmax) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < g.n; j += gridDim.x * blockDim.x) {
        int L;
        uint32_t c;
        anchor_cell(g, j, need, nullptr, &L, &c);
        if (L < 1) continue;
        const uint32_t gid = g.lv[L].base + c;
        flag[gid] = 1u;
        if (dK) {
            const uint64_t d2 = dK[j];
            uint64_t r = (uint64_t)sqrt((double)d2);
            while (r * r < d2) r++;
            while (r > 0 && (r - 1) * (r - 1) >= d2) r--;
            const int4 p = g.pts[j];
            const int s = g.lv[L].s;
            const int u[3] = {p.x - g.minx, p.y - g.miny, p.z - g.minz};
            int64_t face = INT64_MAX;
            for (int a = 0; a < 3; a++) {
                const int cc = u[a] >> s;
                const int64_t lo = (int64_t)u[a] - ((int64_t)cc << s) + 1, hi = ((int64_t)(cc + 1) << s) - u[a];
                face = min(face, min(lo, hi));
            }
            const int64_t e = (int64_t)r - face;
            if (e > 0) atomicMax((long long*)&tmax[gid], (long long)e);
        }
    }
}

__global__ void __launch_bounds__(kBlock) pr_compact_k(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                                                       uint32_t total, uint32_t* __restrict__ anc) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x)
        if (flag[t]) anc[pos[t]] = t;
}

__device__ inline int level_of_gid(const GridView& g, uint32_t gid) {
    int L = 0;
    while (L + 1 < g.nlev && gid >= g.lv[L + 1].base) L++;
    return L;
}

// One wavefront per anchor cell (level L >= 1, coordinates c): lane
// (dx, dy, dz) in 0..3 counts the points of the level L-1 cell
// 2c + (dx, dy, dz) - 1; feature = log1p(count) in bf16.  With tmax, also
// the target log2(expansion / 2^s_L) (-8 when no expansion is needed).
__global__ void __launch_bounds__(kBlock) pr_feat_k(GridView g, const uint32_t* __restrict__ anc, uint32_t nanc,
                                                    uint16_t* __restrict__ feat, const int64_t* __restrict__ tmax,
                                                    float* __restrict__ target) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (uint32_t t = blockIdx.x * (kBlock / kWave) + w; t < nanc; t += gridDim.x * (kBlock / kWave)) {
        const uint32_t gid = anc[t];
        const int L = level_of_gid(g, gid);
        const LevelView& lv = g.lv[L];
        const uint64_t code = lv.key[gid - lv.base];
        const uint32_t sg = (uint32_t)(code >> lv.segshift);
        const uint64_t mc = code & ((1ull << lv.segshift) - 1ull);
        const int cx = (int)compact21(mc), cy = (int)compact21(mc >> 1), cz = (int)compact21(mc >> 2);
        const LevelView& ls = g.lv[L - 1];
        const int x = 2 * cx + (lane & 3) - 1, y = 2 * cy + ((lane >> 2) & 3) - 1, z = 2 * cz + (lane >> 4) - 1;
        uint32_t cnt = 0;
        if (x >= 0 && y >= 0 && z >= 0 && x <= ls.cmax[0] && y <= ls.cmax[1] && z <= ls.cmax[2]) {
            const uint32_t c = hash_find(ls.hkeys, ls.hvals, ls.hmask, cell_code(ls, sg, x, y, z));
            if (c != kNone) cnt = ls.start[c + 1] - ls.start[c];
        }
        feat[(size_t)t * kF + lane] = to_bf16(log1pf((float)cnt));
        if (tmax && lane == 0) {
            const int64_t m = tmax[gid];
            target[t] = m <= 0 ? -8.0f : fmaxf(log2f((float)m) - (float)lv.s, -8.0f);
        }
    }
}

// K-th list distance of every point (0 when its list is empty)
template <int K>
__global__ void __launch_bounds__(kBlock) pr_dk_k(GridView g, const int32_t* __restrict__ nbr,
                                                  const uint8_t* __restrict__ cnt, uint64_t* __restrict__ dK) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < g.n; j += gridDim.x * blockDim.x) {
        const int c = cnt[j];
        uint64_t d = 0;
        if (c > 0) {
            const int4 p = g.pts[j], q = g.pts[nbr[(size_t)j * K + c - 1]];
            d = dist2(p.x, p.y, p.z, q.x, q.y, q.z);
        }
        dK[j] = d;
    }
}

// ---------------------------------------------------------------------------
// network
// ---------------------------------------------------------------------------

// Outputs of n feature rows, 16 rows per wavefront.
__global__ void __launch_bounds__(kBlock) pr_forward_k(const uint16_t* __restrict__ X, uint32_t n,
                                                       const float* __restrict__ P, float* __restrict__ out) {
    __shared__ uint16_t w1[kF * kF], w2[kF * kF];
    __shared__ float b1[kF], b2[kF], w3[kF];
    __shared__ uint16_t h1[kBlock / kWave][16 * kF];
    for (int i = threadIdx.x; i < kF * kF; i += blockDim.x) {
        w1[i] = to_bf16(P[oW1 + i]);
        w2[i] = to_bf16(P[oW2 + i]);
    }
    if (threadIdx.x < kF) {
        b1[threadIdx.x] = P[oB1 + threadIdx.x];
        b2[threadIdx.x] = P[oB2 + threadIdx.x];
        w3[threadIdx.x] = P[oW3 + threadIdx.x];
    }
    __syncthreads();
    const float b3 = P[oB3];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t ntiles = (n + 15) / 16;
    for (uint32_t tile = blockIdx.x * (kBlock / kWave) + w; tile < ntiles; tile += gridDim.x * (kBlock / kWave)) {
        const uint32_t r0 = tile * 16;
        const bool row_ok = r0 + (lane & 15) < n;
        f4 acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; nb++) acc[nb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ks++) {
            bf4 a = bf4{0, 0, 0, 0};
            if (row_ok) a = frag_rows(X, (int)r0, ks, lane);
#pragma unroll
            for (int nb = 0; nb < 4; nb++) acc[nb] = mfma16(a, frag_cols(w1, ks, nb, lane), acc[nb]);
        }
#pragma unroll
        for (int nb = 0; nb < 4; nb++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int col = 16 * nb + (lane & 15);
                h1[w][(4 * (lane >> 4) + v) * kF + col] = to_bf16(fmaxf(acc[nb][v] + b1[col], 0.f));
            }
        wave_sync_lds();
#pragma unroll
        for (int nb = 0; nb < 4; nb++) acc[nb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ks++) {
            const bf4 a = frag_rows(h1[w], 0, ks, lane);
#pragma unroll
            for (int nb = 0; nb < 4; nb++) acc[nb] = mfma16(a, frag_cols(w2, ks, nb, lane), acc[nb]);
        }
        float part[4];
#pragma unroll
        for (int v = 0; v < 4; v++) {
            part[v] = 0.f;
#pragma unroll
            for (int nb = 0; nb < 4; nb++) {
                const int col = 16 * nb + (lane & 15);
                part[v] += fmaxf(acc[nb][v] + b2[col], 0.f) * w3[col];
            }
            part[v] = row_sum16(part[v]);
        }
        if ((lane & 15) == 0)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const uint32_t row = r0 + 4 * (lane >> 4) + v;
                if (row < n) out[row] = part[v] + b3;
            }
        wave_sync_lds();
    }
}

__device__ inline uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// One training step in one block of 256 threads.  mode 0: gradient of the
// mean pinball loss over rows 0..n-1 (n <= kTB) into grad, no update.
// mode 1: a minibatch of B rows drawn with replacement (splitmix64 of seed,
// step and row), gradient into grad, then an Adam step (beta 0.9 / 0.999,
// eps 1e-8, bias-corrected, step t >= 1) on P with moments M, V.
__global__ void __launch_bounds__(kBlock) pr_train_k(const uint16_t* __restrict__ X, const float* __restrict__ Y,
                                                     uint32_t n, float* __restrict__ P, float* __restrict__ M,
                                                     float* __restrict__ V, float* __restrict__ grad, int B, int t,
                                                     float lr, float tau, uint64_t seed, int mode,
                                                     float* __restrict__ loss_out) {
    __shared__ uint16_t xs[kTB * kF], h1s[kTB * kF], gs[kTB * kF];
    __shared__ uint16_t w1s[kF * kF], w2s[kF * kF];
    __shared__ float b1[kF], b2[kF], w3[kF], ys[kTB];
    __shared__ float red_w3[kBlock / kWave][kF], red_b2[kBlock / kWave][kF], red_b1[kBlock / kWave][kF];
    __shared__ float red_b3[kBlock / kWave], red_loss[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int rows = mode == 0 ? (int)n : B;            // rows that count
    const int BT = (rows + 15) / 16 * 16;               // rows in tiles
    // minibatch rows and targets
    for (int r = w; r < BT; r += kBlock / kWave) {
        uint32_t src = 0;
        bool ok = r < rows;
        if (ok) src = mode == 0 ? (uint32_t)r : (uint32_t)(splitmix64(seed ^ ((uint64_t)t << 32) ^ (uint64_t)r) % n);
        xs[r * kF + lane] = ok ? X[(size_t)src * kF + lane] : (uint16_t)0;
        if (lane == 0) ys[r] = ok ? Y[src] : 0.f;
    }
    for (int i = threadIdx.x; i < kF * kF; i += blockDim.x) {
        w1s[i] = to_bf16(P[oW1 + i]);
        w2s[i] = to_bf16(P[oW2 + i]);
    }
    if (threadIdx.x < kF) {
        b1[threadIdx.x] = P[oB1 + threadIdx.x];
        b2[threadIdx.x] = P[oB2 + threadIdx.x];
        w3[threadIdx.x] = P[oW3 + threadIdx.x];
    }
    __syncthreads();
    const float b3 = P[oB3];
    const float inv = 1.0f / (float)rows;
    const int ntile = BT / 16;

    // forward, output gradient, dZ2 (gs), and the sums for w3, b2, b3
    float gw3[4] = {0.f, 0.f, 0.f, 0.f}, gb2[4] = {0.f, 0.f, 0.f, 0.f}, gb3 = 0.f, lsum = 0.f;
    for (int tile = w; tile < ntile; tile += kBlock / kWave) {
        const int r0 = tile * 16;
        f4 acc[4];
#pragma unroll
        for (int nb = 0; nb < 4; nb++) acc[nb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ks++) {
            const bf4 a = frag_rows(xs, r0, ks, lane);
#pragma unroll
            for (int nb = 0; nb < 4; nb++) acc[nb] = mfma16(a, frag_cols(w1s, ks, nb, lane), acc[nb]);
        }
#pragma unroll
        for (int nb = 0; nb < 4; nb++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int col = 16 * nb + (lane & 15);
                h1s[(r0 + 4 * (lane >> 4) + v) * kF + col] = to_bf16(fmaxf(acc[nb][v] + b1[col], 0.f));
            }
        wave_sync_lds();
#pragma unroll
        for (int nb = 0; nb < 4; nb++) acc[nb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ks++) {
            const bf4 a = frag_rows(h1s, r0, ks, lane);
#pragma unroll
            for (int nb = 0; nb < 4; nb++) acc[nb] = mfma16(a, frag_cols(w2s, ks, nb, lane), acc[nb]);
        }
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int row = r0 + 4 * (lane >> 4) + v;
            float h2[4], part = 0.f;
#pragma unroll
            for (int nb = 0; nb < 4; nb++) {
                const int col = 16 * nb + (lane & 15);
                h2[nb] = fmaxf(acc[nb][v] + b2[col], 0.f);
                part += h2[nb] * w3[col];
            }
            const float yhat = row_sum16(part) + b3;
            const float r = ys[row] - yhat;
            float dy = r > 0.f ? -tau : (r < 0.f ? 1.0f - tau : 0.f);
            const bool live = row < rows;
            dy = live ? dy * inv : 0.f;
            if ((lane & 15) == 0 && live) {
                lsum += (r > 0.f ? tau * r : (tau - 1.0f) * r) * inv;
                gb3 += dy;
            }
#pragma unroll
            for (int nb = 0; nb < 4; nb++) {
                const int col = 16 * nb + (lane & 15);
                const float dz = h2[nb] > 0.f ? dy * w3[col] : 0.f;
                gw3[nb] += dy * h2[nb];
                gb2[nb] += dz;
                gs[row * kF + col] = to_bf16(dz);
            }
        }
    }
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
        gw3[nb] = col_sum4(gw3[nb]);
        gb2[nb] = col_sum4(gb2[nb]);
        if (lane < 16) {
            red_w3[w][16 * nb + lane] = gw3[nb];
            red_b2[w][16 * nb + lane] = gb2[nb];
        }
    }
    // lanes 0, 16, 32, 48 hold the b3 and loss sums of their row groups
    gb3 += __shfl_xor(gb3, 16, kWave);
    gb3 += __shfl_xor(gb3, 32, kWave);
    lsum += __shfl_xor(lsum, 16, kWave);
    lsum += __shfl_xor(lsum, 32, kWave);
    if (lane == 0) {
        red_b3[w] = gb3;
        red_loss[w] = lsum;
    }
    __syncthreads();

    // dW2 = H1^T dZ2: wave w takes output tiles (w, 0..3)
    {
        const int ti = w;
        for (int tj = 0; tj < 4; tj++) {
            f4 acc = f4{0.f, 0.f, 0.f, 0.f};
            for (int ks = 0; ks < ntile; ks++) acc = mfma16(frag_cols(h1s, ks, ti, lane), frag_cols(gs, ks, tj, lane), acc);
#pragma unroll
            for (int v = 0; v < 4; v++)
                grad[oW2 + (16 * ti + 4 * (lane >> 4) + v) * kF + 16 * tj + (lane & 15)] = acc[v];
        }
    }
    // dH1 = dZ2 W2^T, masked by H1 > 0, for this wave's row tiles (kept in
    // registers until every wave has finished reading H1)
    constexpr int kMaxT = kTB / 16 / (kBlock / kWave);
    f4 dz1[kMaxT][4];
    float gb1[4] = {0.f, 0.f, 0.f, 0.f};
    {
        int q = 0;
        for (int tile = w; tile < ntile; tile += kBlock / kWave, q++) {
            const int r0 = tile * 16;
#pragma unroll
            for (int nb = 0; nb < 4; nb++) dz1[q][nb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ks++) {
                const bf4 a = frag_rows(gs, r0, ks, lane);
#pragma unroll
                for (int nb = 0; nb < 4; nb++) dz1[q][nb] = mfma16(a, frag_rows(w2s, 16 * nb, ks, lane), dz1[q][nb]);
            }
#pragma unroll
            for (int nb = 0; nb < 4; nb++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int col = 16 * nb + (lane & 15);
                    if (h1s[(r0 + 4 * (lane >> 4) + v) * kF + col] == 0) dz1[q][nb][v] = 0.f;
                    gb1[nb] += dz1[q][nb][v];
                }
        }
    }
    __syncthreads();
    {
        int q = 0;
        for (int tile = w; tile < ntile; tile += kBlock / kWave, q++) {
            const int r0 = tile * 16;
#pragma unroll
            for (int nb = 0; nb < 4; nb++)
#pragma unroll
                for (int v = 0; v < 4; v++)
                    h1s[(r0 + 4 * (lane >> 4) + v) * kF + 16 * nb + (lane & 15)] = to_bf16(dz1[q][nb][v]);
        }
    }
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
        gb1[nb] = col_sum4(gb1[nb]);
        if (lane < 16) red_b1[w][16 * nb + lane] = gb1[nb];
    }
    __syncthreads();
    // dW1 = X^T dZ1
    {
        const int ti = w;
        for (int tj = 0; tj < 4; tj++) {
            f4 acc = f4{0.f, 0.f, 0.f, 0.f};
            for (int ks = 0; ks < ntile; ks++) acc = mfma16(frag_cols(xs, ks, ti, lane), frag_cols(h1s, ks, tj, lane), acc);
#pragma unroll
            for (int v = 0; v < 4; v++)
                grad[oW1 + (16 * ti + 4 * (lane >> 4) + v) * kF + 16 * tj + (lane & 15)] = acc[v];
        }
    }
    if (threadIdx.x < kF) {
        float s1 = 0.f, s2 = 0.f, s3 = 0.f;
        for (int q = 0; q < kBlock / kWave; q++) {
            s1 += red_b1[q][threadIdx.x];
            s2 += red_b2[q][threadIdx.x];
            s3 += red_w3[q][threadIdx.x];
        }
        grad[oB1 + threadIdx.x] = s1;
        grad[oB2 + threadIdx.x] = s2;
        grad[oW3 + threadIdx.x] = s3;
    }
    if (threadIdx.x == 0) {
        float s = 0.f, l = 0.f;
        for (int q = 0; q < kBlock / kWave; q++) {
            s += red_b3[q];
            l += red_loss[q];
        }
        grad[oB3] = s;
        if (loss_out) loss_out[0] = l;
    }
    if (mode == 0) return;
    __syncthreads();
    const float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
    for (int i = threadIdx.x; i < kPredParams; i += blockDim.x) {
        const float gi = grad[i];
        const float m = 0.9f * M[i] + 0.1f * gi;
        const float v = 0.999f * V[i] + 0.001f * gi * gi;
        M[i] = m;
        V[i] = v;
        P[i] -= lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
    }
}

// squared expansion per anchor cell: (2^(yhat + margin) * 2^s)^2, rounded up
__global__ void __launch_bounds__(kBlock) pr_radius_k(GridView g, const uint32_t* __restrict__ anc, uint32_t nanc,
                                                      const float* __restrict__ yhat, float margin,
                                                      uint64_t* __restrict__ r2) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nanc; t += gridDim.x * blockDim.x) {
        const uint32_t gid = anc[t];
        const int L = level_of_gid(g, gid);
        const float e = fminf(fmaxf(yhat[t] + margin, -20.f), 2.f) + (float)g.lv[L].s;
        const double rr = exp2((double)e);
        r2[gid] = (uint64_t)ceil(rr * rr) + 1;
    }
}

inline unsigned gfor(size_t count) {
    size_t g = (count + kBlock - 1) / kBlock;
    return (unsigned)std::max<size_t>(1, std::min<size_t>(g, 16384));
}

// scratch slots of the predictor
enum { kPrFlag = 76, kPrPos, kPrAnc, kPrFeat, kPrY, kPrR2, kPrTmax, kPrDK, kPrNbr, kPrCnt, kPrCost, kPrGrad };

// anchor cells of every point, compacted; returns their count in *nanc
int anchors(Ctx* c, const GridView& g, uint32_t need, const uint64_t* dK, int64_t* tmax, uint32_t** anc_out,
            uint32_t* nanc) {
    const uint32_t total = g.total_cells;
    uint32_t* flag = (uint32_t*)scratch(c, kPrFlag, (size_t)(total + 1) * 4);
    uint32_t* pos = (uint32_t*)scratch(c, kPrPos, (size_t)(total + 1) * 4);
    uint32_t* anc = (uint32_t*)scratch(c, kPrAnc, (size_t)(total + 1) * 4);
    if (!flag || !pos || !anc) return PDD_ENOMEM;
    int rc;
    if ((rc = fill_u32(c, flag, 0, total + 1))) return rc;
    if (tmax && (rc = fill_u32(c, (uint32_t*)tmax, 0, (size_t)total * 2))) return rc;
    hipLaunchKernelGGL(pr_mark_k, dim3(gfor(g.n)), dim3(kBlock), 0, c->stream, g, need, flag, dK, tmax);
    PDD_HIP(c, hipGetLastError());
    if ((rc = exclusive_scan_u32(c, flag, pos, total, pos + total))) return rc;
    hipLaunchKernelGGL(pr_compact_k, dim3(gfor(total)), dim3(kBlock), 0, c->stream, flag, pos, total, anc);
    PDD_HIP(c, hipGetLastError());
    uint32_t* h = (uint32_t*)c->pinned;
    PDD_HIP(c, hipMemcpyAsync(h, pos + total, 4, hipMemcpyDeviceToHost, c->stream));
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    *nanc = h[0];
    *anc_out = anc;
    return PDD_OK;
}

int ensure_params(Ctx* c) {
    if (c->pred_P) return PDD_OK;
    const size_t bytes = (size_t)kPredParams * 4;
    if (hipMalloc(&c->pred_P, bytes) != hipSuccess || hipMalloc(&c->pred_M, bytes) != hipSuccess ||
        hipMalloc(&c->pred_V, bytes) != hipSuccess) {
        (void)hipGetLastError();
        c->err = "hipMalloc: out of memory";
        return PDD_ENOMEM;
    }
    int rc;
    if ((rc = fill_u32(c, (uint32_t*)c->pred_P, 0, kPredParams))) return rc;
    if ((rc = fill_u32(c, (uint32_t*)c->pred_M, 0, kPredParams))) return rc;
    if ((rc = fill_u32(c, (uint32_t*)c->pred_V, 0, kPredParams))) return rc;
    c->pred_step = 0;
    return PDD_OK;
}

}  // namespace

int pred_set(Ctx* c, const float* host, int64_t n) {
    if (n != kPredParams || !host) return PDD_EINVAL;
    int rc = ensure_params(c);
    if (rc) return rc;
    PDD_HIP(c, hipMemcpyAsync(c->pred_P, host, (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
    if ((rc = fill_u32(c, (uint32_t*)c->pred_M, 0, kPredParams))) return rc;
    if ((rc = fill_u32(c, (uint32_t*)c->pred_V, 0, kPredParams))) return rc;
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    c->pred_step = 0;
    c->pred_ready = true;
    return PDD_OK;
}

int pred_get(Ctx* c, float* host, int64_t n) {
    if (n != kPredParams || !host) return PDD_EINVAL;
    if (!c->pred_ready) return PDD_EINVAL;
    PDD_HIP(c, hipMemcpyAsync(host, c->pred_P, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream));
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    return PDD_OK;
}

int pred_forward(Ctx* c, const uint16_t* feat, int64_t n, float* out) {
    if (!c->pred_ready || n < 0 || n > 0x7FFFFFFF) return PDD_EINVAL;
    if (n == 0) return PDD_OK;
    const uint32_t tiles = (uint32_t)((n + 15) / 16);
    const unsigned blocks = std::max(1u, std::min((tiles + 3) / 4, 4096u));
    hipLaunchKernelGGL(pr_forward_k, dim3(blocks), dim3(kBlock), 0, c->stream, feat, (uint32_t)n, c->pred_P, out);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

int pred_grad(Ctx* c, const uint16_t* feat, const float* target, int64_t n, float tau, float* grad, float* loss) {
    if (!c->pred_ready || n < 1 || n > kTB) return PDD_EINVAL;
    hipLaunchKernelGGL(pr_train_k, dim3(1), dim3(kBlock), 0, c->stream, feat, target, (uint32_t)n, c->pred_P,
                       c->pred_M, c->pred_V, grad, (int)n, 1, 0.f, tau, 0ull, 0, loss);
    PDD_HIP(c, hipGetLastError());
    return PDD_OK;
}

int pred_train(Ctx* c, const uint16_t* feat, const float* target, int64_t n, int steps, int batch, float lr, float tau,
               uint64_t seed, float* loss) {
    if (!c->pred_ready || n < 1 || n > 0x7FFFFFFF || steps < 0 || batch < 16 || batch > kTB || batch % 16 ||
        !(lr > 0.f) || !(tau > 0.f && tau < 1.f))
        return PDD_EINVAL;
    float* grad = (float*)scratch(c, kPrGrad, (size_t)kPredParams * 4);
    if (!grad) return PDD_ENOMEM;
    for (int s = 0; s < steps; s++) {
        const int t = (int)(++c->pred_step);
        hipLaunchKernelGGL(pr_train_k, dim3(1), dim3(kBlock), 0, c->stream, feat, target, (uint32_t)n, c->pred_P,
                           c->pred_M, c->pred_V, grad, batch, t, lr, tau, seed, 1, loss ? loss + s : nullptr);
    }
    PDD_HIP(c, hipGetLastError());
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    return PDD_OK;
}

int pred_samples(Ctx* c, const GridView& g, int k, int K, uint16_t* feat, float* target, int64_t cap, int64_t* count) {
    if (cap < 0 || !count) return PDD_EINVAL;
    KnnOut ko;
    ko.nbr = (int32_t*)scratch(c, kPrNbr, (size_t)g.n * K * 4);
    ko.cnt = (uint8_t*)scratch(c, kPrCnt, (size_t)g.n);
    ko.cost = (uint64_t*)scratch(c, kPrCost, (size_t)g.n * 8);
    ko.r2k = nullptr;
    uint64_t* dK = (uint64_t*)scratch(c, kPrDK, (size_t)g.n * 8);
    int64_t* tmax = (int64_t*)scratch(c, kPrTmax, (size_t)(g.total_cells + 1) * 8);
    if (!ko.nbr || !ko.cnt || !ko.cost || !dK || !tmax) return PDD_ENOMEM;
    const bool on = c->pred_on;
    c->pred_on = false;  // samples come from the plain search
    int rc = knn_all(c, g, k, K, ko, nullptr);
    c->pred_on = on;
    if (rc) return rc;
    switch (K) {
        case 8: hipLaunchKernelGGL(pr_dk_k<8>, dim3(gfor(g.n)), dim3(kBlock), 0, c->stream, g, ko.nbr, ko.cnt, dK); break;
        case 16: hipLaunchKernelGGL(pr_dk_k<16>, dim3(gfor(g.n)), dim3(kBlock), 0, c->stream, g, ko.nbr, ko.cnt, dK); break;
        case 24: hipLaunchKernelGGL(pr_dk_k<24>, dim3(gfor(g.n)), dim3(kBlock), 0, c->stream, g, ko.nbr, ko.cnt, dK); break;
        case 32: hipLaunchKernelGGL(pr_dk_k<32>, dim3(gfor(g.n)), dim3(kBlock), 0, c->stream, g, ko.nbr, ko.cnt, dK); break;
        default: return PDD_EINVAL;
    }
    PDD_HIP(c, hipGetLastError());
    uint32_t* anc;
    uint32_t nanc;
    if ((rc = anchors(c, g, (uint32_t)K + 1, dK, tmax, &anc, &nanc))) return rc;
    *count = nanc;
    const uint32_t m = (uint32_t)std::min<int64_t>(cap, nanc);
    if (m > 0 && feat && target) {
        hipLaunchKernelGGL(pr_feat_k, dim3(std::min<uint32_t>((m + 3) / 4, 16384u)), dim3(kBlock), 0, c->stream, g, anc,
                           m, feat, tmax, target);
        PDD_HIP(c, hipGetLastError());
    }
    PDD_HIP(c, hipStreamSynchronize(c->stream));
    return PDD_OK;
}

int pred_radii(Ctx* c, const GridView& g, int K, const uint64_t** r2_out) {
    *r2_out = nullptr;
    uint32_t* anc;
    uint32_t nanc;
    int rc = anchors(c, g, (uint32_t)K + 1, nullptr, nullptr, &anc, &nanc);
    if (rc) return rc;
    uint64_t* r2 = (uint64_t*)scratch(c, kPrR2, (size_t)(g.total_cells + 1) * 8);
    uint16_t* feat = (uint16_t*)scratch(c, kPrFeat, (size_t)std::max<uint32_t>(nanc, 1) * kF * 2);
    float* y = (float*)scratch(c, kPrY, (size_t)std::max<uint32_t>(nanc, 1) * 4);
    if (!r2 || !feat || !y) return PDD_ENOMEM;
    if ((rc = fill_u32(c, (uint32_t*)r2, 0, (size_t)(g.total_cells + 1) * 2))) return rc;
    if (nanc > 0) {
        hipLaunchKernelGGL(pr_feat_k, dim3(std::min<uint32_t>((nanc + 3) / 4, 16384u)), dim3(kBlock), 0, c->stream, g,
                           anc, nanc, feat, nullptr, nullptr);
        PDD_HIP(c, hipGetLastError());
        if ((rc = pred_forward(c, feat, nanc, y))) return rc;
        hipLaunchKernelGGL(pr_radius_k, dim3(gfor(nanc)), dim3(kBlock), 0, c->stream, g, anc, nanc, y, c->pred_margin,
                           r2);
        PDD_HIP(c, hipGetLastError());
    }
    *r2_out = r2;
    return PDD_OK;
}

}  // namespace pdd
