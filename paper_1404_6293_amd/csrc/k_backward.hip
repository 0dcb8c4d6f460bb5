// k_backward.hip -- gradients of an image loss with respect to per-vertex
// colours and texels for Gouraud and textured shading.  For each covered
// pixel with upstream gradient G (alpha ignored) and saved perspective
// barycentrics (b0, b1, b2):
//   untextured: dC[v_k][c] += b_k G_c
//   textured:   dC[v_k][c] += b_k G_c T_c ,  dTex[j][c] += w_j G_c Cint_c
// Coverage is not differentiated.
//
// Device-scope float atomics are slow on this part at spread addresses
// (about 20 G/s, against about 2 T/s for LDS atomics), and neighbouring
// pixels scatter to the same vertices (shared by neighbouring triangles) and
// the same texels (overlapping bilinear footprints).  So each workgroup takes
// a 64 x 16 pixel tile and sums its contributions per vertex and per texel
// in LDS hash tables (open addressing, keys claimed by compare-and-swap,
// values added with LDS float atomics), then adds each distinct entry to the
// gradient buffers with one global atomic per channel, in runs of
// neighbouring addresses (below).
#include "pk_internal.h"

#pragma clang fp contract(off)

namespace pk {

// Pixels per workgroup tile.  Wide tiles pre-reduce best here (measured on
// 64 views of the textured grid: 64 x 16 2.50 ms, 32 x 32 2.55, 32 x 16
// 2.70, 128 x 8 2.72, 256 x 4 2.87, 16 x 16 3.83): fewer tile borders split
// a vertex's or a texel's sum, and a tile row's texels are neighbours in
// memory.
constexpr int kBwdTW = 64, kBwdTH = 16;
constexpr int kBwdThreads = kBwdTW * kBwdTH;
// A tile has at most 1024 x 3 distinct vertices and 1024 x 4 distinct
// texels: the vertex table is never more than 3/4 full and the texel table
// never over-full, so an insert always finds its key or a free slot
// (128 KiB of LDS, one workgroup per CU).
constexpr int kVtxSlots = 4096;
constexpr int kTexSlots = 4096;
constexpr int32_t kNoKey = -1;

// Device-scope float atomics are executed at the memory side, one request
// per cache line that a wave's instruction touches: measured on this GPU
// with one atomic per lane into a 9 MB buffer, 322 G/s when a wave's
// addresses are consecutive (318 G/s for random runs of 16), 21 G/s when
// they are random.  So the tables keep neighbouring keys in neighbouring
// slots: a key's home slot keeps its position within its run of
// 2^kRunLog2 consecutive keys, and the run goes to a randomly placed group
// of as many slots.  The flush walks the slots in order, so a wave's
// atomics fall on a few runs of neighbouring addresses.  On 64 textured
// views at 512 x 512 this took the pass from 4.12 ms (a plain multiplicative
// hash of the key) to 2.49 ms; runs of 4 and 16 measured the same within
// 1%, runs of 32 were slower (4.48 ms: long probe chains).
constexpr int kRunLog2 = 3;

template <int N>
__device__ inline uint32_t slot_of(int32_t key) {
    constexpr int LB = kRunLog2;
    const uint32_t run = (uint32_t)key >> LB;
    const uint32_t g = (run * 2654435761u) >> (32 - __builtin_ctz(N) + LB);
    return (g << LB) | ((uint32_t)key & ((1u << LB) - 1));
}

// Slot of `key` (>= 0) from slot h on, claiming a free one if needed, or -1
// when the table is full.  Linear probing over at most N slots.
template <int N>
__device__ inline int lds_claim_from(int32_t *keys, int32_t key, uint32_t h) {
#pragma unroll 1
    for (int probe = 0; probe < N; ++probe) {
        const int32_t k = atomicCAS(&keys[h], kNoKey, key);
        if (k == kNoKey || k == key) return (int)h;
        h = (h + 1) & (N - 1);
    }
    return -1;
}

// Add (v0, v1, v2) to slot h, or straight to the global buffer at `gbase`
// (channel stride `gstride`) when the key found no slot (h < 0; the tables
// never fill, see above).
template <int N>
__device__ inline void lds_add(float *vals, int h, float v0, float v1, float v2, float *gbase,
                               int64_t gstride) {
    if (h >= 0) {
        atomicAdd(&vals[h], v0);
        atomicAdd(&vals[N + h], v1);
        atomicAdd(&vals[2 * N + h], v2);
    } else {
        atomicAdd(gbase, v0);
        atomicAdd(gbase + gstride, v1);
        atomicAdd(gbase + 2 * gstride, v2);
    }
}

// Lanes of a wave hold one tile row's pixels in order, and a triangle (and
// a magnified texel) covers a contiguous span of a row: lanes with the same
// key form runs.  Same-address LDS atomics of one instruction serialize, so
// when the wave has runs, each run's values are summed across its lanes
// first (segmented doubling over shuffles, stopping once no run is longer
// than the distance reached) and only the run's first lane keeps its key
// (the others get kNoKey).  On 64 textured views at 512 x 512 this took the
// pass from 2.50 to 2.11 ms; summing only in waves with at most 32 runs
// kept 2.44.  Call from uniform control flow.
__device__ inline void wave_run_sum(int32_t &key, float &a, float &b, float &c) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t prev = __shfl_up(key, 1, kWave);
    const bool head = lane == 0 || prev != key;
    const uint64_t heads = __ballot(head);
    if (heads == ~0ull) return;   // no two neighbours share a key
    const uint64_t le = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1);
    const int run = __popcll(heads & le);
#pragma unroll 1
    for (int d = 1; d < kWave; d <<= 1) {
        const int r2 = __shfl_down(run, d, kWave);
        const bool same = lane + d < kWave && r2 == run;
        if (!__ballot(same)) break;   // every run is at most d lanes long
        const float a2 = __shfl_down(a, d, kWave), b2 = __shfl_down(b, d, kWave),
                    c2 = __shfl_down(c, d, kWave);
        if (same) { a = a + a2; b = b + b2; c = c + c2; }
    }
    if (!head) key = kNoKey;
}

template <bool TEX>
__global__ __launch_bounds__(kBwdThreads) void k_backward(Geom G, Shade sh, const int32_t *primid,
                                                          const float *bary, const float *grad,
                                                          float *gv, float *gt) {
    __shared__ int32_t s_vkey[kVtxSlots];
    __shared__ float s_vval[3 * kVtxSlots];
    __shared__ int32_t s_tkey[TEX ? kTexSlots : 1];
    __shared__ float s_tval[TEX ? 3 * kTexSlots : 1];
    const int tid = threadIdx.x;
    for (int i = tid; i < kVtxSlots; i += kBwdThreads) {
        s_vkey[i] = kNoKey;
        s_vval[i] = s_vval[kVtxSlots + i] = s_vval[2 * kVtxSlots + i] = 0.0f;
    }
    if (TEX) {
        for (int i = tid; i < kTexSlots; i += kBwdThreads) {
            s_tkey[i] = kNoKey;
            s_tval[i] = s_tval[kTexSlots + i] = s_tval[2 * kTexSlots + i] = 0.0f;
        }
    }
    __syncthreads();

    // this thread's pixel: tile (scene, tx, ty), position (lx, ly) in it
    const uint32_t ntx = (uint32_t)((G.W + kBwdTW - 1) / kBwdTW);
    const uint32_t nty = (uint32_t)((G.H + kBwdTH - 1) / kBwdTH);
    const uint32_t per_scene = ntx * nty;
    const uint32_t s = blockIdx.x / per_scene;
    const uint32_t ts = blockIdx.x - s * per_scene;
    const uint32_t ty = ts / ntx, tx = ts - ty * ntx;
    const int px = (int)(tx * kBwdTW) + tid % kBwdTW;
    const int py = (int)(ty * kBwdTH) + tid / kBwdTW;
    const int64_t V = G.V;
    const int64_t p = ((int64_t)s * G.H + py) * G.W + px;
    const int32_t t = (px < G.W && py < G.H) ? primid[p] : -1;
    // this pixel's entries: its triangle's three vertices and (textured) its
    // four texel taps, kNoKey where there is none, with what each adds per
    // channel
    int32_t vkey[3] = {kNoKey, kNoKey, kNoKey};
    float vval[3][3] = {};
    int32_t tkey[4] = {kNoKey, kNoKey, kNoKey, kNoKey};
    float tval[4][3] = {};
    if (t >= 0) {
        int64_t g, vb;
        if (G.S == 1 || G.instanced) { g = t; vb = 0; }
        else { g = (int64_t)G.tri_off[s] + t; vb = G.vtx_off[s]; }
        // the pixel's own inputs and the triangle's three indices (one
        // load) are issued together
        const float2 bb = reinterpret_cast<const float2 *>(bary)[p];
        const float4 Gc = reinterpret_cast<const float4 *>(grad)[p];
        int32_t v[3];
        if (G.idx) {
            const int32_t *ip = G.idx + 3 * g;
            const int32_t i0 = ip[0], i1 = ip[1], i2 = ip[2];
            v[0] = (int32_t)(vb + i0);
            v[1] = (int32_t)(vb + i1);
            v[2] = (int32_t)(vb + i2);
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) v[k] = (int32_t)(vb + 3 * (int64_t)t + k);
        }
        const float b1 = bb.x, b2 = bb.y, b0 = (1.0f - b1) - b2;
        const float bw[3] = {b0, b1, b2};
        float gvc[3] = {Gc.x, Gc.y, Gc.z};     // what multiplies b_k per channel
        if (TEX) {
            float rgb[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float *pl = sh.color + c * V;
                float acc = b0 * pl[v[0]];
                acc = acc + b1 * pl[v[1]];
                acc = acc + b2 * pl[v[2]];
                rgb[c] = acc;
            }
            float u = b0 * sh.uv[v[0]];
            u = u + b1 * sh.uv[v[1]];
            u = u + b2 * sh.uv[v[2]];
            float vv = b0 * sh.uv[V + v[0]];
            vv = vv + b1 * sh.uv[V + v[1]];
            vv = vv + b2 * sh.uv[V + v[2]];
            const float su = u * (float)sh.tex_w - 0.5f, sv = vv * (float)sh.tex_h - 0.5f;
            const float fi = floorf(su), fj = floorf(sv);
            const float fs = su - fi, ft = sv - fj;
            const float ci = fminf(fmaxf(fi, -1.0f), (float)sh.tex_w);
            const float cj = fminf(fmaxf(fj, -1.0f), (float)sh.tex_h);
            const int i0 = min(max((int)ci, 0), sh.tex_w - 1), i1 = min(max((int)ci + 1, 0), sh.tex_w - 1);
            const int j0 = min(max((int)cj, 0), sh.tex_h - 1), j1 = min(max((int)cj + 1, 0), sh.tex_h - 1);
            const float w[4] = {(1.0f - fs) * (1.0f - ft), fs * (1.0f - ft), (1.0f - fs) * ft, fs * ft};
            const int32_t txl[4] = {j0 * sh.tex_w + i0, j0 * sh.tex_w + i1,
                                    j1 * sh.tex_w + i0, j1 * sh.tex_w + i1};
            float gC[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float T = w[0] * sh.texture[3 * (int64_t)txl[0] + c];
                T = T + w[1] * sh.texture[3 * (int64_t)txl[1] + c];
                T = T + w[2] * sh.texture[3 * (int64_t)txl[2] + c];
                T = T + w[3] * sh.texture[3 * (int64_t)txl[3] + c];
                gvc[c] = gvc[c] * T;
                gC[c] = (c == 0 ? Gc.x : c == 1 ? Gc.y : Gc.z) * rgb[c];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                tkey[j] = txl[j];
#pragma unroll
                for (int c = 0; c < 3; ++c) tval[j][c] = w[j] * gC[c];
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            vkey[k] = v[k];
#pragma unroll
            for (int c = 0; c < 3; ++c) vval[k][c] = bw[k] * gvc[c];
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) wave_run_sum(vkey[k], vval[k][0], vval[k][1], vval[k][2]);
    if (TEX) {
#pragma unroll
        for (int j = 0; j < 4; ++j) wave_run_sum(tkey[j], tval[j][0], tval[j][1], tval[j][2]);
    }
    // the slots of all entries: every claim is issued at its home slot
    // before any result is needed (one LDS round trip), and only a key whose
    // home slot holds another key probes on
    int hv[3] = {0, 0, 0}, ht[4] = {0, 0, 0, 0};
    int32_t gotv[3] = {0, 0, 0}, gott[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (vkey[k] == kNoKey) continue;
        hv[k] = (int)slot_of<kVtxSlots>(vkey[k]);
        gotv[k] = atomicCAS(&s_vkey[hv[k]], kNoKey, vkey[k]);
    }
    if (TEX) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (tkey[j] == kNoKey) continue;
            ht[j] = (int)slot_of<kTexSlots>(tkey[j]);
            gott[j] = atomicCAS(&s_tkey[ht[j]], kNoKey, tkey[j]);
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (vkey[k] != kNoKey && gotv[k] != kNoKey && gotv[k] != vkey[k])
            hv[k] = lds_claim_from<kVtxSlots>(s_vkey, vkey[k], (hv[k] + 1) & (kVtxSlots - 1));
    if (TEX) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (tkey[j] != kNoKey && gott[j] != kNoKey && gott[j] != tkey[j])
                ht[j] = lds_claim_from<kTexSlots>(s_tkey, tkey[j], (ht[j] + 1) & (kTexSlots - 1));
        for (int j = 0; j < 4; ++j)
            if (tkey[j] != kNoKey)
                lds_add<kTexSlots>(s_tval, ht[j], tval[j][0], tval[j][1], tval[j][2],
                                   gt + 3 * (int64_t)tkey[j], 1);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (vkey[k] != kNoKey)
            lds_add<kVtxSlots>(s_vval, hv[k], vval[k][0], vval[k][1], vval[k][2],
                               gv + vkey[k], V);
    __syncthreads();
    // one global atomic per channel of every distinct vertex and texel
    for (int i = tid; i < kVtxSlots; i += kBwdThreads) {
        const int32_t k = s_vkey[i];
        if (k == kNoKey) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) atomicAdd(gv + c * V + k, s_vval[c * kVtxSlots + i]);
    }
    if (TEX) {
        for (int i = tid; i < kTexSlots; i += kBwdThreads) {
            const int32_t k = s_tkey[i];
            if (k == kNoKey) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) atomicAdd(gt + 3 * (int64_t)k + c, s_tval[c * kTexSlots + i]);
        }
    }
}

hipError_t launch_backward(const Geom &G, const Shade &sh, const int32_t *primid,
                           const float *bary, const float *grad, float *grad_vcolor,
                           float *grad_tex, hipStream_t st) {
    const int64_t ntiles = (int64_t)G.S * ((G.W + kBwdTW - 1) / kBwdTW) *
                           ((G.H + kBwdTH - 1) / kBwdTH);
    if (ntiles == 0) return hipSuccess;
    if (ntiles >= (int64_t)INT32_MAX || G.V >= (int64_t)INT32_MAX) return hipErrorInvalidValue;
    if (sh.shading == PK_SHADE_TEXTURED) {
        if ((int64_t)sh.tex_w * sh.tex_h >= (int64_t)INT32_MAX / 3) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_backward<true>, dim3((unsigned)ntiles), dim3(kBwdThreads), 0, st, G,
                           sh, primid, bary, grad, grad_vcolor, grad_tex);
    } else {
        hipLaunchKernelGGL(k_backward<false>, dim3((unsigned)ntiles), dim3(kBwdThreads), 0, st, G,
                           sh, primid, bary, grad, grad_vcolor, grad_tex);
    }
    return hipGetLastError();
}

}  // namespace pk
