// k_reyes.hip -- the Reyes front end of libpk (include/pk_reyes.h): Split
// and Dice of bicubic Bezier patches.
//
// Split is the self-loop stage of the Reyes pipeline (Sec. 7.1), run as in
// Sec. 5.1 by launching it once per round.  A round's queue is cut into
// fixed chunks; one workgroup per chunk.  The decision of every queued patch
// (drop, dice, split in u or v) and the per-chunk counts of children and
// leaves are known before the round's kernel starts: the kernel that wrote a
// patch into the queue also decided it.  k_split_round then
//   - sums the counts of the chunks before its own (prefix sums instead of
//     atomically appended queues, as the bins of Sec. 6),
//   - scans its chunk tile by tile and writes the two halves of each split
//     patch to the next queue and each diced patch to the leaf list, both
//     in queue order,
//   - decides the halves it wrote (for the next round) and adds their
//     counts to the next round's per-chunk counts,
//   - (workgroup 0) publishes the next queue length and the leaf count.
// k_split_first decides the input patches.  The queue order is therefore a
// breadth-first traversal with halves in parameter order, independent of
// timing; every round is one kernel, all enqueued at once, reading the
// round's length from device memory (a round whose queue is empty exits at
// once).
//
// Dice (Sec. 7.1) evaluates an (n+1) x (n+1) grid per leaf in LDS (one
// workgroup of one wave per leaf): the four rows of control points at each
// u once, then each vertex's column at its v; it writes SoA vertex planes,
// normals from central differences, and the grid's triangles, ready for
// the rasterizer.
#include <cmath>
#include <cstring>

#include "pk_internal.h"
#include "../../include/pk_reyes.h"

namespace pk {
namespace {

constexpr int kRT = 256;           // threads of a Split workgroup
constexpr int kMaxChunks = 1024;   // chunks (workgroups) of one round at most
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
    int32_t *agg[3];               // [kMaxChunks][2]: children, leaves decided per chunk
    uint8_t *dec[2];               // decision of each patch of a round
    float *q[2];                   // queues [cap][48]
    int32_t *qsrc[2];              // their source patch numbers
};

// byte layout of the workspace; also its size
size_t split_layout(int64_t np, int64_t cap, char *base, SplitWs *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += align_up(bytes); return base ? base + o : nullptr; };
    const size_t nd = (size_t)std::max(np, cap);
    char *ctl = take(sizeof(int64_t) * kCtlWords);
    char *agg[3], *dec[2], *q[2], *qs[2];
    for (auto &x : agg) x = take(sizeof(int32_t) * 2 * kMaxChunks);
    for (auto &x : dec) x = take(nd);
    for (auto &x : q) x = take(sizeof(float) * kPatch * (size_t)cap);
    for (auto &x : qs) x = take(sizeof(int32_t) * (size_t)cap);
    if (w) {
        w->ctl = (int64_t *)ctl;
        for (int k = 0; k < 3; ++k) w->agg[k] = (int32_t *)agg[k];
        for (int k = 0; k < 2; ++k) {
            w->dec[k] = (uint8_t *)dec[k];
            w->q[k] = (float *)q[k];
            w->qsrc[k] = (int32_t *)qs[k];
        }
    }
    return off;
}

// Patches per chunk: a whole number of 64-patch tiles, and few enough
// chunks for the largest round (the input or a full queue).
int64_t chunk_size(int64_t np, int64_t cap) {
    const int64_t n = std::max<int64_t>(std::max(np, cap), 1);
    const int64_t c = (n + kMaxChunks - 1) / kMaxChunks;
    return std::max<int64_t>(64, (c + 63) / 64 * 64);
}

struct SplitArgs {
    SplitWs w;
    const float *mvp;              // [16] or null (identity)
    float W, H, hw, hh, dice;
    int max_depth;
    int64_t cap;
    int64_t chunk;
    float *leaves;
    int32_t *leaf_src;
    int64_t leaf_cap;
    int64_t *counts;
};

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

__device__ inline float lerp_rn(float x, float y, float t) { return x + t * (y - x); }

// de Casteljau of one cubic at t.
__device__ inline float cubic_at(float a, float b, float c, float d, float t) {
    const float ab = lerp_rn(a, b, t), bc = lerp_rn(b, c, t), cd = lerp_rn(c, d, t);
    const float abc = lerp_rn(ab, bc, t), bcd = lerp_rn(bc, cd, t);
    return lerp_rn(abc, bcd, t);
}

__device__ inline void load_matrix(const float *mvp, float (&m)[16]) {
#pragma unroll
    for (int k = 0; k < 16; ++k) m[k] = mvp ? mvp[k] : 0.0f;
}

// Patches of round r (rounds after the first never exceed the queue).
__device__ inline int64_t round_size(const SplitArgs &a, int r) {
    const int64_t n = a.w.ctl[kCtlN + r];
    return r == 0 ? n : (n < a.cap ? n : a.cap);
}

__global__ __launch_bounds__(kRT) void k_split_init(SplitArgs a, int64_t np) {
    if (threadIdx.x == 0) {
        a.w.ctl[kCtlN] = np;
        a.w.ctl[kCtlLeaf] = 0;
        for (int k = 0; k < 6; ++k) a.counts[k] = 0;
    }
    // round 0 adds the counts of the halves it decides into agg[1]
    for (int k = threadIdx.x; k < 2 * kMaxChunks; k += kRT) a.w.agg[1][k] = 0;
}

// ---- quads: four lanes per patch, lane a holding row a -------------------
constexpr int kTile = 64;          // patches per tile of a Split workgroup (kRT / 4)

__device__ inline float quad_min(float v) {
    v = fminf(v, __shfl_xor(v, 1));
    return fminf(v, __shfl_xor(v, 2));
}

__device__ inline float quad_max(float v) {
    v = fmaxf(v, __shfl_xor(v, 1));
    return fmaxf(v, __shfl_xor(v, 2));
}

// What Split does with the patch at s (48 floats in LDS): 0 drop, 1 dice,
// 2 split in u, 3 split in v (include/pk_reyes.h).  Computed by the four
// lanes of a quad: lane a transforms row a and the two end points of column
// a; the box and the row and column spans are reduced over the quad.  Every
// lane of the quad returns the same decision; the four lanes must be active
// together.
__device__ inline int quad_decide(const float *s, int a, const float (&m)[16], bool has_m,
                                  const SplitArgs &A, bool last) {
    float xs[4], ys[4], cx0, cy0, cx3, cy3;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float *q = s + 3 * (4 * a + k);
        ok = ctrl_screen(m, has_m, A.hw, A.hh, q[0], q[1], q[2], xs[k], ys[k]) && ok;
    }
    ok = ctrl_screen(m, has_m, A.hw, A.hh, s[3 * a], s[3 * a + 1], s[3 * a + 2], cx0, cy0) && ok;
    ok = ctrl_screen(m, has_m, A.hw, A.hh, s[3 * (12 + a)], s[3 * (12 + a) + 1],
                     s[3 * (12 + a) + 2], cx3, cy3) && ok;
    int okq = ok ? 1 : 0;
    okq &= __shfl_xor(okq, 1);
    okq &= __shfl_xor(okq, 2);
    if (!okq) return 0;
    float x0 = fminf(fminf(xs[0], xs[1]), fminf(xs[2], xs[3]));
    float x1 = fmaxf(fmaxf(xs[0], xs[1]), fmaxf(xs[2], xs[3]));
    float y0 = fminf(fminf(ys[0], ys[1]), fminf(ys[2], ys[3]));
    float y1 = fmaxf(fmaxf(ys[0], ys[1]), fmaxf(ys[2], ys[3]));
    x0 = quad_min(x0); y0 = quad_min(y0);
    x1 = quad_max(x1); y1 = quad_max(y1);
    if (x1 < 0.0f || x0 > A.W || y1 < 0.0f || y0 > A.H) return 0;
    if ((x1 - x0 <= A.dice && y1 - y0 <= A.dice) || last) return 1;
    const float ux = xs[3] - xs[0], uy = ys[3] - ys[0];
    const float vx = cx3 - cx0, vy = cy3 - cy0;
    const float du = quad_max(ux * ux + uy * uy), dv = quad_max(vx * vx + vy * vy);
    return du >= dv ? 2 : 3;
}

// Copy `cnt` consecutive patches starting at `first` into LDS, coalesced.
__device__ inline void stage_tile(float4 *dst, const float *src, int64_t first, int cnt) {
    const float4 *s4 = reinterpret_cast<const float4 *>(src) + first * (kPatch / 4);
    for (int f = threadIdx.x; f < cnt * (kPatch / 4); f += kRT) dst[f] = s4[f];
}

// Decisions and per-chunk counts of the input patches (round 0).
__global__ __launch_bounds__(kRT) void k_split_first(SplitArgs a, const float *in, int64_t np) {
    __shared__ int s_wave[kRT / kWave];
    __shared__ float4 s_in4[kTile * kPatch / 4];
    const float *s_in = reinterpret_cast<const float *>(s_in4);
    const int64_t begin = (int64_t)blockIdx.x * a.chunk;
    const int64_t end = begin + a.chunk < np ? begin + a.chunk : np;
    float m[16];
    load_matrix(a.mvp, m);
    const bool has_m = a.mvp != nullptr, last = a.max_depth == 0;
    const int p = threadIdx.x >> 2, row = threadIdx.x & 3;
    int kids = 0, lv = 0;
    for (int64_t b = begin; b < end; b += kTile) {
        const int cnt = (int)(end - b < kTile ? end - b : kTile);
        stage_tile(s_in4, in, b, cnt);
        __syncthreads();
        if (p < cnt) {
            const int d = quad_decide(s_in + kPatch * p, row, m, has_m, a, last);
            if (row == 0) {
                a.w.dec[0][b + p] = (uint8_t)d;
                kids += d >= 2 ? 2 : 0;
                lv += d == 1 ? 1 : 0;
            }
        }
        __syncthreads();
    }
    int tk, tl;
    block_exclusive_scan<kRT>(kids, s_wave, tk);
    block_exclusive_scan<kRT>(lv, s_wave, tl);
    if (threadIdx.x == 0) {
        a.w.agg[0][2 * blockIdx.x] = tk;
        a.w.agg[0][2 * blockIdx.x + 1] = tl;
    }
}

// One round: leaves and halves of the round's patches written in queue
// order (staged in LDS, stored coalesced), the halves decided for the next
// round.  Tiles of 64 patches, four lanes per patch.
__global__ __launch_bounds__(kRT) void k_split_round(SplitArgs a, int r, const float *in,
                                                      const int32_t *in_src, const uint8_t *dec_in,
                                                      const int32_t *agg_in, float *out,
                                                      int32_t *out_src, uint8_t *dec_out,
                                                      int32_t *agg_out, int32_t *agg_clear) {
    __shared__ int s_wave[kRT / kWave];
    __shared__ int s_next[4][2];   // counts of the next round's chunks this tile touches
    __shared__ float4 s_in4[kTile * kPatch / 4];
    __shared__ float4 s_out4[2 * kTile * kPatch / 4];
    __shared__ int s_leaf[kTile];  // tile patch of each leaf of the tile
    __shared__ int32_t s_ksrc[2 * kTile];
    float *s_in = reinterpret_cast<float *>(s_in4);
    float *s_out = reinterpret_cast<float *>(s_out4);
    // the next round but one accumulates into agg_clear
    if (threadIdx.x < 2) agg_clear[2 * blockIdx.x + threadIdx.x] = 0;
    // Every load that does not depend on another is issued before the first
    // wait: a round is a short chain of dependent memory round trips, and
    // each one removed shortens it.
    // children and leaves of the chunks before this one (and of all chunks)
    int kb = 0, lb = 0, kt = 0, lt = 0;
    for (int g = threadIdx.x; g < (int)gridDim.x; g += kRT) {
        const int2 cl = reinterpret_cast<const int2 *>(agg_in)[g];
        if (g < (int)blockIdx.x) { kb += cl.x; lb += cl.y; }
        kt += cl.x;
        lt += cl.y;
    }
    const int64_t n = round_size(a, r);
    const int64_t leaf0 = a.w.ctl[kCtlLeaf + r];
    const int64_t CH = a.chunk;
    const int64_t begin = (int64_t)blockIdx.x * CH;
    const int64_t end = begin + CH < n ? begin + CH : n;
    if (begin >= end && blockIdx.x != 0) return;          // uniform per workgroup
    int t;
    block_exclusive_scan<kRT>(kb, s_wave, t); kb = t;
    block_exclusive_scan<kRT>(lb, s_wave, t); lb = t;
    block_exclusive_scan<kRT>(kt, s_wave, t); kt = t;
    block_exclusive_scan<kRT>(lt, s_wave, t); lt = t;
    float m[16];
    load_matrix(a.mvp, m);
    const bool has_m = a.mvp != nullptr, last_next = r + 1 == a.max_depth;
    int64_t kid_run = kb, leaf_run = leaf0 + lb;
    const int p = threadIdx.x >> 2, row = threadIdx.x & 3;
    const int lane = threadIdx.x & (kWave - 1), lead_lane = lane & ~3;
    float4 *out4 = reinterpret_cast<float4 *>(out);
    float4 *leaves4 = reinterpret_cast<float4 *>(a.leaves);
    const float4 *in4 = reinterpret_cast<const float4 *>(in);
    for (int64_t b = begin; b < end; b += kTile) {
        const int cnt = (int)(end - b < kTile ? end - b : kTile);
        // the tile (3 float4 per thread), its decisions and sources, all in flight at once
        float4 v4[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int f = threadIdx.x + k * kRT;
            v4[k] = f < cnt * (kPatch / 4) ? in4[b * (kPatch / 4) + f] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        const int d = p < cnt ? (int)dec_in[b + p] : 0;
        const int32_t src_l = (row == 0 && p < cnt) ? (in_src ? in_src[b + p] : (int32_t)(b + p)) : 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) s_in4[threadIdx.x + k * kRT] = v4[k];
        const bool lead = row == 0;
        int tk, tl;
        int ek = block_exclusive_scan<kRT>(lead && d >= 2 ? 2 : 0, s_wave, tk);
        int el = block_exclusive_scan<kRT>(lead && d == 1 ? 1 : 0, s_wave, tl);
        ek = __shfl(ek, lead_lane);
        el = __shfl(el, lead_lane);
        if (lead && d != 0) {
            const int32_t src = src_l;
            if (d == 1) {
                s_leaf[el] = p;
                if (leaf_run + el < a.leaf_cap) a.leaf_src[leaf_run + el] = src;
            } else {
                s_ksrc[ek] = src;
                s_ksrc[ek + 1] = src;
            }
        }
        if (threadIdx.x < 8) (&s_next[0][0])[threadIdx.x] = 0;
        __syncthreads();                                   // tile, maps in LDS
        if (d >= 2) {
            // lane `row` halves line `row`: a row (split in u) or a column (in v)
            const float *cp = s_in + kPatch * p;
            float *lo = s_out + kPatch * ek, *hi = s_out + kPatch * (ek + 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                int pt[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) pt[k] = d == 2 ? 4 * row + k : 4 * k + row;
                const float x0 = cp[3 * pt[0] + c], x1 = cp[3 * pt[1] + c];
                const float x2 = cp[3 * pt[2] + c], x3 = cp[3 * pt[3] + c];
                const float ab = lerp_rn(x0, x1, 0.5f), bc = lerp_rn(x1, x2, 0.5f);
                const float cd = lerp_rn(x2, x3, 0.5f);
                const float abc = lerp_rn(ab, bc, 0.5f), bcd = lerp_rn(bc, cd, 0.5f);
                const float mid = lerp_rn(abc, bcd, 0.5f);
                lo[3 * pt[0] + c] = x0;   lo[3 * pt[1] + c] = ab;
                lo[3 * pt[2] + c] = abc;  lo[3 * pt[3] + c] = mid;
                hi[3 * pt[0] + c] = mid;  hi[3 * pt[1] + c] = bcd;
                hi[3 * pt[2] + c] = cd;   hi[3 * pt[3] + c] = x3;
            }
        }
        __syncthreads();                                   // halves in LDS
        for (int f = threadIdx.x; f < tl * (kPatch / 4); f += kRT) {
            const int j = f / (kPatch / 4), k = f - j * (kPatch / 4);
            const int64_t slot = leaf_run + j;
            if (slot < a.leaf_cap) leaves4[slot * (kPatch / 4) + k] = s_in4[s_leaf[j] * (kPatch / 4) + k];
        }
        for (int f = threadIdx.x; f < tk * (kPatch / 4); f += kRT) {
            const int64_t slot = kid_run + f / (kPatch / 4);
            if (slot < a.cap) out4[kid_run * (kPatch / 4) + f] = s_out4[f];
        }
        for (int j = threadIdx.x; j < tk; j += kRT)
            if (kid_run + j < a.cap) out_src[kid_run + j] = s_ksrc[j];
        // decide the halves for the next round: quad p takes halves p, p + 64
        const int64_t c0 = kid_run / CH;
        for (int j = p; j < tk; j += kTile) {
            const int64_t slot = kid_run + j;
            if (slot < a.cap) {
                const int dh = quad_decide(s_out + kPatch * j, row, m, has_m, a, last_next);
                if (row == 0) {
                    dec_out[slot] = (uint8_t)dh;
                    const int c = (int)(slot / CH - c0);
                    if (dh >= 2) atomicAdd(&s_next[c][0], 2);
                    if (dh == 1) atomicAdd(&s_next[c][1], 1);
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < 8) {
            const int c = threadIdx.x >> 1, v = (&s_next[0][0])[threadIdx.x];
            if (v) atomicAdd(&agg_out[2 * (c0 + c) + (threadIdx.x & 1)], v);
        }
        kid_run += tk;
        leaf_run += tl;
        __syncthreads();                                   // LDS reused by the next tile
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.w.ctl[kCtlN + r + 1] = kt;
        a.w.ctl[kCtlLeaf + r + 1] = leaf0 + lt;
        a.counts[0] = leaf0 + lt;
        if (kt > a.counts[1]) a.counts[1] = kt;
        a.counts[2] += n;
        if (kt > a.cap) a.counts[3] = 1;
        a.counts[4] = kt;
        if (n > 0) a.counts[5] = r + 1;
    }
}

// One wave per leaf: the grid in LDS, then vertices, normals and triangles.
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(8))) void k_dice(const float *leaves, const int32_t *leaf_src,
                                                int64_t nl, const float *pcol, int64_t np, int n,
                                                float *pos, float *col, float *nrm, int32_t *idx,
                                                int64_t V) {
    __shared__ float s_cp[kPatch];
    // rows of control points evaluated at each u_j: [j][row][coordinate]
    __shared__ float s_col[(kDiceMaxN + 1) * 12];
    __shared__ float s_g[3][(kDiceMaxN + 1) * (kDiceMaxN + 1)];
    const int m = n + 1, mm = m * m, nf = 6 * n * n;
    const float fn = (float)n;
    const int lane = threadIdx.x;
    for (int64_t l = blockIdx.x; l < nl; l += gridDim.x) {
        if (lane < kPatch) s_cp[lane] = leaves[kPatch * l + lane];
        __syncthreads();
        // every row of control points at u_j = j / n, once per j (each
        // vertex of column j uses the same values)
        for (int e = lane; e < m * 12; e += kWave) {
            const int j = e / 12, rc = e - 12 * j, r = rc / 3, c = rc - 3 * r;
            const float u = (float)j / fn;
            s_col[e] = cubic_at(s_cp[3 * (4 * r) + c], s_cp[3 * (4 * r + 1) + c],
                                s_cp[3 * (4 * r + 2) + c], s_cp[3 * (4 * r + 3) + c], u);
        }
        __syncthreads();
        // then the resulting column at v_i = i / n
        for (int v = lane; v < mm; v += kWave) {
            const int i = v / m, j = v - i * m;
            const float w = (float)i / fn;
            const float *cv = s_col + 12 * j;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                s_g[c][v] = cubic_at(cv[c], cv[3 + c], cv[6 + c], cv[9 + c], w);
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
                                    int64_t leaf_capacity, int32_t round_begin,
                                    int32_t round_end, int64_t *counts, void *stream) {
    if (!params_ok(p) || num_patches < 0 || num_patches > PK_REYES_MAX_QUEUE ||
        round_begin < 0 || round_end < round_begin ||
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
    const int64_t n_max = std::max<int64_t>(std::max(num_patches, queue_capacity), 1);
    a.chunk = chunk_size(num_patches, queue_capacity);
    const unsigned groups = (unsigned)((n_max + a.chunk - 1) / a.chunk);
    if (round_begin == 0 && round_end > 0) {
        hipLaunchKernelGGL(k_split_init, dim3(1), dim3(kRT), 0, st, a, num_patches);
        hipLaunchKernelGGL(k_split_first, dim3(groups), dim3(kRT), 0, st, a, patches, num_patches);
    }
    const int r_end = std::min(round_end, p->max_depth + 1);
    for (int r = round_begin; r < r_end; ++r) {
        const float *in = r == 0 ? patches : a.w.q[(r - 1) & 1];
        const int32_t *in_src = r == 0 ? nullptr : a.w.qsrc[(r - 1) & 1];
        hipLaunchKernelGGL(k_split_round, dim3(groups), dim3(kRT), 0, st, a, r, in, in_src,
                           a.w.dec[r & 1], a.w.agg[r % 3], a.w.q[r & 1], a.w.qsrc[r & 1],
                           a.w.dec[(r + 1) & 1], a.w.agg[(r + 1) % 3], a.w.agg[(r + 2) % 3]);
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
