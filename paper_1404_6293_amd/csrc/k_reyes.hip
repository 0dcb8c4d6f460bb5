// k_reyes.hip -- the Reyes front end of libpk (include/pk_reyes.h): Split
// and Dice of bicubic Bezier patches.
//
// Split is the self-loop stage of the Reyes pipeline (Sec. 7.1), run as in
// Sec. 5.1 by launching it once per round; every round is two kernels over
// the round's queue, whose length they read from device memory:
//   k_split_decide  one thread per patch: the split test (drop, dice, split
//                   in u or v), a decision byte, and per-workgroup counts of
//                   children and leaves over a contiguous chunk;
//   k_split_write   every workgroup sums the counts of the chunks before its
//                   own (prefix sums instead of atomically appended queues,
//                   as the bins of Sec. 6), scans its chunk tile by tile and
//                   writes the halves of split patches to the next round's
//                   queue and the leaves to the leaf list, both in queue
//                   order; workgroup 0 also publishes the next round's queue
//                   length and the running leaf count.
// The queue order therefore equals a breadth-first traversal with halves in
// parameter order, independent of timing, and all rounds are enqueued at
// once (a round whose queue is empty exits at once).
//
// Dice (Sec. 7.1) evaluates an (n+1) x (n+1) grid per leaf in LDS (one
// workgroup of one wave per leaf) and writes SoA vertex planes, normals from
// central differences, and the grid's triangles, ready for the rasterizer.
#include <cmath>
#include <cstring>

#include "pk_internal.h"
#include "../../include/pk_reyes.h"

namespace pk {
namespace {

constexpr int kRT = 256;           // threads of a Split workgroup
constexpr int kRGroups = 1024;     // Split workgroups (contiguous chunks) per round
constexpr int kPatch = 48;         // floats per patch: 16 points x 3
constexpr int kMaxDepth = 30;
constexpr int kDiceMaxN = 16;
// int64 words at the head of the workspace
constexpr int kCtlN = 0;           // [32] patches queued for round r
constexpr int kCtlLeaf = 32;       // [32] leaves emitted before round r
constexpr int kCtlWords = 64;

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct SplitWs {
    int64_t *ctl;
    int32_t *agg;                  // [kRGroups][2]: children, leaves of each chunk
    uint8_t *dec;                  // decision of each patch of the round
    float *q[2];                   // queues [cap][48]
    int32_t *qsrc[2];              // their source patch numbers
};

// byte layout of the workspace; also its size
size_t split_layout(int64_t np, int64_t cap, char *base, SplitWs *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += align_up(bytes); return base ? base + o : nullptr; };
    char *ctl = take(sizeof(int64_t) * kCtlWords);
    char *agg = take(sizeof(int32_t) * 2 * kRGroups);
    char *dec = take((size_t)std::max(np, cap));
    char *q0 = take(sizeof(float) * kPatch * (size_t)cap);
    char *q1 = take(sizeof(float) * kPatch * (size_t)cap);
    char *s0 = take(sizeof(int32_t) * (size_t)cap);
    char *s1 = take(sizeof(int32_t) * (size_t)cap);
    if (w) {
        w->ctl = (int64_t *)ctl;
        w->agg = (int32_t *)agg;
        w->dec = (uint8_t *)dec;
        w->q[0] = (float *)q0;
        w->q[1] = (float *)q1;
        w->qsrc[0] = (int32_t *)s0;
        w->qsrc[1] = (int32_t *)s1;
    }
    return off;
}

struct SplitArgs {
    SplitWs w;
    const float *mvp;              // [16] or null (identity)
    float W, H, hw, hh, dice;
    int max_depth;
    int64_t cap;
    float *leaves;
    int32_t *leaf_src;
    int64_t leaf_cap;
    int64_t *counts;
};

__device__ inline void load_patch(const float *p, float (&cp)[kPatch]) {
    const float4 *v = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int k = 0; k < kPatch / 4; ++k) {
        const float4 t = v[k];
        cp[4 * k] = t.x; cp[4 * k + 1] = t.y; cp[4 * k + 2] = t.z; cp[4 * k + 3] = t.w;
    }
}

__device__ inline void store_patch(float *p, const float (&cp)[kPatch]) {
    float4 *v = reinterpret_cast<float4 *>(p);
#pragma unroll
    for (int k = 0; k < kPatch / 4; ++k)
        v[k] = make_float4(cp[4 * k], cp[4 * k + 1], cp[4 * k + 2], cp[4 * k + 3]);
}

// The vertex transform of pk.h without snapping: products rounded, sums
// left to right, one correctly rounded reciprocal of w.
__device__ inline bool ctrl_screen(const float (&m)[16], bool has_m, float hw, float hh,
                                   float x, float y, float z, float &xs, float &ys) {
    float c0 = x, c1 = y, c3 = 1.0f;
    if (has_m) {
        c0 = m[0] * x; c0 = c0 + m[1] * y; c0 = c0 + m[2] * z; c0 = c0 + m[3];
        c1 = m[4] * x; c1 = c1 + m[5] * y; c1 = c1 + m[6] * z; c1 = c1 + m[7];
        c3 = m[12] * x; c3 = c3 + m[13] * y; c3 = c3 + m[14] * z; c3 = c3 + m[15];
    }
    if (!(isfinite(c0) && isfinite(c1) && isfinite(c3) && c3 > 0.0f)) return false;
    const float iw = 1.0f / c3;
    xs = (c0 * iw + 1.0f) * hw;
    ys = (c1 * iw + 1.0f) * hh;
    return isfinite(xs) && isfinite(ys);
}

// 0 drop, 1 dice, 2 split in u, 3 split in v (include/pk_reyes.h).
__device__ inline int split_decide(const float (&cp)[kPatch], const float (&m)[16], bool has_m,
                                   const SplitArgs &a, bool last) {
    float xs[16], ys[16];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 16; ++k)
        ok = ctrl_screen(m, has_m, a.hw, a.hh, cp[3 * k], cp[3 * k + 1], cp[3 * k + 2], xs[k], ys[k]) && ok;
    if (!ok) return 0;
    float x0 = xs[0], x1 = xs[0], y0 = ys[0], y1 = ys[0];
#pragma unroll
    for (int k = 1; k < 16; ++k) {
        x0 = fminf(x0, xs[k]); x1 = fmaxf(x1, xs[k]);
        y0 = fminf(y0, ys[k]); y1 = fmaxf(y1, ys[k]);
    }
    if (x1 < 0.0f || x0 > a.W || y1 < 0.0f || y0 > a.H) return 0;
    if ((x1 - x0 <= a.dice && y1 - y0 <= a.dice) || last) return 1;
    float du = 0.0f, dv = 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float ux = xs[4 * r + 3] - xs[4 * r], uy = ys[4 * r + 3] - ys[4 * r];
        const float vx = xs[12 + r] - xs[r], vy = ys[12 + r] - ys[r];
        du = fmaxf(du, ux * ux + uy * uy);
        dv = fmaxf(dv, vx * vx + vy * vy);
    }
    return du >= dv ? 2 : 3;
}

__device__ inline float lerp_rn(float x, float y, float t) { return x + t * (y - x); }

// de Casteljau of one cubic at t: the point, and optionally both halves.
__device__ inline float cubic_at(float a, float b, float c, float d, float t) {
    const float ab = lerp_rn(a, b, t), bc = lerp_rn(b, c, t), cd = lerp_rn(c, d, t);
    const float abc = lerp_rn(ab, bc, t), bcd = lerp_rn(bc, cd, t);
    return lerp_rn(abc, bcd, t);
}

// Halves of a patch at u = 1/2 (DIR 0: every row is a cubic in u) or
// v = 1/2 (DIR 1: every column is a cubic in v).
template <int DIR>
__device__ inline void halve(const float (&cp)[kPatch], float (&lo)[kPatch], float (&hi)[kPatch]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int p0 = DIR == 0 ? 4 * r : r, st = DIR == 0 ? 1 : 4;
            const float a = cp[3 * p0 + c], b = cp[3 * (p0 + st) + c];
            const float cc = cp[3 * (p0 + 2 * st) + c], d = cp[3 * (p0 + 3 * st) + c];
            const float ab = lerp_rn(a, b, 0.5f), bc = lerp_rn(b, cc, 0.5f), cd = lerp_rn(cc, d, 0.5f);
            const float abc = lerp_rn(ab, bc, 0.5f), bcd = lerp_rn(bc, cd, 0.5f);
            const float p = lerp_rn(abc, bcd, 0.5f);
            lo[3 * p0 + c] = a;                lo[3 * (p0 + st) + c] = ab;
            lo[3 * (p0 + 2 * st) + c] = abc;   lo[3 * (p0 + 3 * st) + c] = p;
            hi[3 * p0 + c] = p;                hi[3 * (p0 + st) + c] = bcd;
            hi[3 * (p0 + 2 * st) + c] = cd;    hi[3 * (p0 + 3 * st) + c] = d;
        }
    }
}

__device__ inline void load_matrix(const float *mvp, float (&m)[16]) {
#pragma unroll
    for (int k = 0; k < 16; ++k) m[k] = mvp ? mvp[k] : 0.0f;
}

// Patches of round r and the chunk [begin, end) of this workgroup.
__device__ inline int64_t round_size(const SplitArgs &a, int r) {
    const int64_t n = a.w.ctl[kCtlN + r];
    return r == 0 ? n : (n < a.cap ? n : a.cap);
}

__device__ inline void chunk_of(int64_t n, int64_t &begin, int64_t &end) {
    int64_t chunk = (n + kRGroups - 1) / kRGroups;
    chunk = (chunk + kRT - 1) / kRT * kRT;
    begin = (int64_t)blockIdx.x * chunk;
    end = begin + chunk < n ? begin + chunk : n;
    if (begin > n) begin = n;
}

__global__ void k_split_init(SplitArgs a, int64_t np) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        a.w.ctl[kCtlN] = np;
        a.w.ctl[kCtlLeaf] = 0;
        a.counts[0] = 0;
        a.counts[1] = 0;
        a.counts[2] = 0;
        a.counts[3] = 0;
    }
}

__global__ __launch_bounds__(kRT) void k_split_decide(SplitArgs a, int r, const float *in) {
    __shared__ int s_wave[kRT / kWave];
    const int64_t n = round_size(a, r);
    int64_t begin, end;
    chunk_of(n, begin, end);
    float m[16];
    load_matrix(a.mvp, m);
    const bool has_m = a.mvp != nullptr, last = r == a.max_depth;
    int kids = 0, lv = 0;
    for (int64_t b = begin; b < end; b += kRT) {
        const int64_t i = b + threadIdx.x;
        if (i < end) {
            float cp[kPatch];
            load_patch(in + kPatch * i, cp);
            const int d = split_decide(cp, m, has_m, a, last);
            a.w.dec[i] = (uint8_t)d;
            kids += d >= 2 ? 2 : 0;
            lv += d == 1 ? 1 : 0;
        }
    }
    int tk, tl;
    block_exclusive_scan<kRT>(kids, s_wave, tk);
    block_exclusive_scan<kRT>(lv, s_wave, tl);
    if (threadIdx.x == 0) {
        a.w.agg[2 * blockIdx.x] = tk;
        a.w.agg[2 * blockIdx.x + 1] = tl;
    }
}

__global__ __launch_bounds__(kRT) void k_split_write(SplitArgs a, int r, const float *in,
                                                      const int32_t *in_src, float *out,
                                                      int32_t *out_src) {
    __shared__ int s_wave[kRT / kWave];
    const int64_t n = round_size(a, r);
    int64_t begin, end;
    chunk_of(n, begin, end);
    if (begin >= end && blockIdx.x != 0) return;          // uniform per workgroup
    // children and leaves of the chunks before this one (and of all chunks)
    int kb = 0, lb = 0, kt = 0, lt = 0;
    for (int g = threadIdx.x; g < kRGroups; g += kRT) {
        const int c = a.w.agg[2 * g], l = a.w.agg[2 * g + 1];
        if (g < (int)blockIdx.x) { kb += c; lb += l; }
        kt += c;
        lt += l;
    }
    int t;
    block_exclusive_scan<kRT>(kb, s_wave, t); kb = t;
    block_exclusive_scan<kRT>(lb, s_wave, t); lb = t;
    block_exclusive_scan<kRT>(kt, s_wave, t); kt = t;
    block_exclusive_scan<kRT>(lt, s_wave, t); lt = t;
    const int64_t leaf0 = a.w.ctl[kCtlLeaf + r];
    int64_t kid_run = kb, leaf_run = leaf0 + lb;
    for (int64_t b = begin; b < end; b += kRT) {
        const int64_t i = b + threadIdx.x;
        const int d = i < end ? (int)a.w.dec[i] : 0;
        int tk, tl;
        const int ek = block_exclusive_scan<kRT>(d >= 2 ? 2 : 0, s_wave, tk);
        const int el = block_exclusive_scan<kRT>(d == 1 ? 1 : 0, s_wave, tl);
        if (d != 0) {
            float cp[kPatch];
            load_patch(in + kPatch * i, cp);
            const int32_t src = in_src ? in_src[i] : (int32_t)i;
            if (d == 1) {
                const int64_t slot = leaf_run + el;
                if (slot < a.leaf_cap) {
                    store_patch(a.leaves + kPatch * slot, cp);
                    a.leaf_src[slot] = src;
                }
            } else {
                float lo[kPatch], hi[kPatch];
                if (d == 2) halve<0>(cp, lo, hi); else halve<1>(cp, lo, hi);
                const int64_t slot = kid_run + ek;
                if (slot < a.cap) { store_patch(out + kPatch * slot, lo); out_src[slot] = src; }
                if (slot + 1 < a.cap) { store_patch(out + kPatch * (slot + 1), hi); out_src[slot + 1] = src; }
            }
        }
        kid_run += tk;
        leaf_run += tl;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.w.ctl[kCtlN + r + 1] = kt;
        a.w.ctl[kCtlLeaf + r + 1] = leaf0 + lt;
        a.counts[0] = leaf0 + lt;
        if (kt > a.counts[1]) a.counts[1] = kt;
        a.counts[2] += n;
        if (kt > a.cap) a.counts[3] = 1;
    }
}

// One wave per leaf: the grid in LDS, then vertices, normals and triangles.
__global__ __launch_bounds__(kWave) void k_dice(const float *leaves, const int32_t *leaf_src,
                                                int64_t nl, const float *pcol, int64_t np, int n,
                                                float *pos, float *col, float *nrm, int32_t *idx,
                                                int64_t V) {
    __shared__ float s_cp[kPatch];
    __shared__ float s_g[3][(kDiceMaxN + 1) * (kDiceMaxN + 1)];
    const int m = n + 1, mm = m * m, nf = 6 * n * n;
    const float fn = (float)n;
    const int lane = threadIdx.x;
    for (int64_t l = blockIdx.x; l < nl; l += gridDim.x) {
        if (lane < kPatch) s_cp[lane] = leaves[kPatch * l + lane];
        __syncthreads();
        for (int v = lane; v < mm; v += kWave) {
            const int i = v / m, j = v - i * m;
            const float u = (float)j / fn, w = (float)i / fn;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float cv[4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    cv[r] = cubic_at(s_cp[3 * (4 * r) + c], s_cp[3 * (4 * r + 1) + c],
                                     s_cp[3 * (4 * r + 2) + c], s_cp[3 * (4 * r + 3) + c], u);
                s_g[c][v] = cubic_at(cv[0], cv[1], cv[2], cv[3], w);
            }
        }
        __syncthreads();
        const int32_t s = leaf_src[l];
        const bool sv = s >= 0 && (int64_t)s < np;
        const float pc0 = sv ? pcol[3 * (int64_t)s] : 0.0f;
        const float pc1 = sv ? pcol[3 * (int64_t)s + 1] : 0.0f;
        const float pc2 = sv ? pcol[3 * (int64_t)s + 2] : 0.0f;
        const int64_t vb = l * mm;
        for (int v = lane; v < mm; v += kWave) {
            const int i = v / m, j = v - i * m;
            const int jp = j < n ? j + 1 : n, jm = j > 0 ? j - 1 : 0;
            const int ip = i < n ? i + 1 : n, im = i > 0 ? i - 1 : 0;
            float pu[3], pv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pu[c] = s_g[c][i * m + jp] - s_g[c][i * m + jm];
                pv[c] = s_g[c][ip * m + j] - s_g[c][im * m + j];
                pos[c * V + vb + v] = s_g[c][v];
            }
            col[vb + v] = pc0;
            col[V + vb + v] = pc1;
            col[2 * V + vb + v] = pc2;
            nrm[vb + v] = pu[1] * pv[2] - pu[2] * pv[1];
            nrm[V + vb + v] = pu[2] * pv[0] - pu[0] * pv[2];
            nrm[2 * V + vb + v] = pu[0] * pv[1] - pu[1] * pv[0];
        }
        const int64_t fb = l * nf;
        for (int f = lane; f < nf; f += kWave) {
            const int t = f / 3, k = f - 3 * t, q = t >> 1;
            const int i = q / n, j = q - i * n;
            const int32_t v00 = (int32_t)(vb + i * m + j), v10 = v00 + 1, v01 = v00 + m, v11 = v01 + 1;
            const int32_t val = (t & 1) ? (k == 0 ? v00 : k == 1 ? v11 : v01)
                                        : (k == 0 ? v00 : k == 1 ? v10 : v11);
            idx[fb + f] = val;
        }
        __syncthreads();
    }
}

bool params_ok(const pk_reyes_params *p) {
    return p && p->width >= 1 && p->width <= 8192 && p->height >= 1 && p->height <= 8192 &&
           std::isfinite(p->dice_px) && p->dice_px > 0.0f && p->max_depth >= 0 &&
           p->max_depth <= kMaxDepth && p->dice_n >= 1 && p->dice_n <= kDiceMaxN;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace
}  // namespace pk

using namespace pk;

extern "C" size_t pk_reyes_workspace_bytes(const pk_reyes_params *p, int64_t num_patches,
                                           int64_t queue_capacity) {
    if (!params_ok(p) || num_patches < 0 || num_patches > PK_REYES_MAX_QUEUE ||
        queue_capacity < 0 || queue_capacity > PK_REYES_MAX_QUEUE)
        return 0;
    return split_layout(num_patches, queue_capacity, nullptr, nullptr);
}

extern "C" pk_status pk_reyes_split(const pk_reyes_params *p, const float *patches,
                                    int64_t num_patches, const float *mvp, void *ws,
                                    int64_t queue_capacity, float *leaves, int32_t *leaf_src,
                                    int64_t leaf_capacity, int64_t *counts, void *stream) {
    if (!params_ok(p) || num_patches < 0 || num_patches > PK_REYES_MAX_QUEUE ||
        queue_capacity < 0 || queue_capacity > PK_REYES_MAX_QUEUE || leaf_capacity < 0 ||
        !ws || !aligned(ws, kAlign) || !counts || (num_patches > 0 && !patches) ||
        !aligned(patches, 16) || (leaf_capacity > 0 && (!leaves || !leaf_src)) ||
        !aligned(leaves, 16))
        return PK_ERR_INVALID_ARGUMENT;
    SplitArgs a;
    std::memset(&a, 0, sizeof a);
    split_layout(num_patches, queue_capacity, (char *)ws, &a.w);
    a.mvp = mvp;
    a.W = (float)p->width;
    a.H = (float)p->height;
    a.hw = 0.5f * (float)p->width;
    a.hh = 0.5f * (float)p->height;
    a.dice = p->dice_px;
    a.max_depth = p->max_depth;
    a.cap = queue_capacity;
    a.leaves = leaves;
    a.leaf_src = leaf_src;
    a.leaf_cap = leaf_capacity;
    a.counts = counts;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_split_init, dim3(1), dim3(64), 0, st, a, num_patches);
    for (int r = 0; r <= p->max_depth; ++r) {
        const float *in = r == 0 ? patches : a.w.q[(r - 1) & 1];
        const int32_t *in_src = r == 0 ? nullptr : a.w.qsrc[(r - 1) & 1];
        hipLaunchKernelGGL(k_split_decide, dim3(kRGroups), dim3(kRT), 0, st, a, r, in);
        hipLaunchKernelGGL(k_split_write, dim3(kRGroups), dim3(kRT), 0, st, a, r, in, in_src,
                           a.w.q[r & 1], a.w.qsrc[r & 1]);
    }
    return hipGetLastError() == hipSuccess ? PK_OK : PK_ERR_HIP;
}

extern "C" pk_status pk_reyes_dice(const pk_reyes_params *p, const float *leaves,
                                   const int32_t *leaf_src, int64_t num_leaves,
                                   const float *patch_color, int64_t num_patches, float *pos,
                                   float *color, float *normal, int32_t *indices, void *stream) {
    if (!params_ok(p) || num_leaves < 0 || num_patches < 0)
        return PK_ERR_INVALID_ARGUMENT;
    const int64_t m = p->dice_n + 1;
    const int64_t V = num_leaves * m * m, T = 2 * (int64_t)p->dice_n * p->dice_n * num_leaves;
    if (V >= (1ll << 31) || T >= (1ll << 31)) return PK_ERR_INVALID_ARGUMENT;
    if (num_leaves == 0) return PK_OK;
    if (!leaves || !leaf_src || (num_patches > 0 && !patch_color) || !pos || !color || !normal ||
        !indices)
        return PK_ERR_INVALID_ARGUMENT;
    const int64_t blocks = num_leaves < 32768 ? num_leaves : 32768;
    hipLaunchKernelGGL(k_dice, dim3((unsigned)blocks), dim3(kWave), 0, (hipStream_t)stream,
                       leaves, leaf_src, num_leaves, patch_color, num_patches, p->dice_n, pos,
                       color, normal, indices, V);
    return hipGetLastError() == hipSuccess ? PK_OK : PK_ERR_HIP;
}
