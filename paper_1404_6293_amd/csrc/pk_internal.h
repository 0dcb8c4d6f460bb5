// pk_internal.h -- device-side data layout and helpers shared by the HIP
// kernels of libpk (never installed; the public ABI is include/pk.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pk.h"

#pragma clang fp contract(off)

namespace pk {

constexpr int kWave = 64;
constexpr int kXcd = 8;       // accelerator complex dies of an MI355X
constexpr unsigned long long kEmptyKey = ~0ull;
// Fragment counts are summed per workgroup into kFragSlots partial counters
// (workgroup w adds to slot w mod kFragSlots) and then reduced by one small
// kernel: device-scope atomics on a single address serialize, thousands of
// them cost more than the kernel they count in.
constexpr int kFragSlots = 256;
constexpr int kMiscWords = 64 + 2 * kFragSlots;

// Per-triangle setup record, 32 bytes (a quarter of a 128-byte cache line,
// two dwordx4 loads): the six fixed-point screen coordinates X0 Y0 X1 Y1 X2
// Y2 as 24-bit two's-complement fields packed end to end into xy[0..4]
// (vertex_stage bounds them by 2^22 in magnitude), then the three NDC depths.
// The pixel bbox and 1/|A2| are recomputed from the coordinates where they
// are needed, with the same expressions as setup, so they are the same bits.
struct __align__(16) TriRec {
    uint32_t xy[5];
    float z0, z1, z2;
};
static_assert(sizeof(TriRec) == 32, "setup record must stay 32 bytes");

__device__ inline void pack_xy(const int32_t X[3], const int32_t Y[3], uint32_t w[5]) {
    const uint32_t f0 = (uint32_t)X[0] & 0xffffffu, f1 = (uint32_t)Y[0] & 0xffffffu;
    const uint32_t f2 = (uint32_t)X[1] & 0xffffffu, f3 = (uint32_t)Y[1] & 0xffffffu;
    const uint32_t f4 = (uint32_t)X[2] & 0xffffffu, f5 = (uint32_t)Y[2] & 0xffffffu;
    w[0] = f0 | (f1 << 24);
    w[1] = (f1 >> 8) | (f2 << 16);
    w[2] = (f2 >> 16) | (f3 << 8);
    w[3] = f4 | (f5 << 24);
    w[4] = f5 >> 8;
}

__device__ inline int32_t sext24(uint32_t v) { return ((int32_t)(v << 8)) >> 8; }

__device__ inline void unpack_xy(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                 uint32_t w4, int32_t X[3], int32_t Y[3]) {
    X[0] = sext24(w0);
    Y[0] = sext24((w0 >> 24) | (w1 << 8));
    X[1] = sext24((w1 >> 16) | (w2 << 16));
    Y[1] = sext24(w2 >> 8);
    X[2] = sext24(w3);
    Y[2] = sext24((w3 >> 24) | (w4 << 8));
}

// Twice the signed area of the snapped triangle (exact in int64) and the
// float64 1/|A2| with the sign of A2 (a correctly rounded division).
__device__ inline int64_t area2(const int32_t X[3], const int32_t Y[3]) {
    return (int64_t)(X[1] - X[0]) * (Y[2] - Y[0]) - (int64_t)(X[2] - X[0]) * (Y[1] - Y[0]);
}

__device__ inline double signed_inv_area(int64_t A2) {
    const int64_t a = A2 > 0 ? A2 : -A2;
    const double inv = 1.0 / (double)a;
    return A2 > 0 ? inv : -inv;
}

// Inclusive pixel bbox of the samples (pixel p is sampled at 256 p + 128) a
// snapped triangle can cover, clipped to the W x H screen; x0 > x1 or y0 > y1
// when there is none.  Arithmetic shifts floor.
__device__ inline void sample_bbox(const int32_t X[3], const int32_t Y[3], int32_t W, int32_t H,
                                   int32_t &x0, int32_t &x1, int32_t &y0, int32_t &y1) {
    const int32_t mnx = min(X[0], min(X[1], X[2])), mxx = max(X[0], max(X[1], X[2]));
    const int32_t mny = min(Y[0], min(Y[1], Y[2])), mxy = max(Y[0], max(Y[1], Y[2]));
    x0 = max((mnx + 127) >> 8, 0);
    x1 = min((mxx - 128) >> 8, W - 1);
    y0 = max((mny + 127) >> 8, 0);
    y1 = min((mxy - 128) >> 8, H - 1);
}

// Everything the geometry kernels need about the mesh and the bin grid.
struct Geom {
    const float *pos;
    int64_t V;
    const int32_t *idx;
    int32_t T;                 // triangles of the mesh (instanced) or of all scenes
    const float *mvp;
    const int32_t *tri_off;
    const int32_t *vtx_off;
    int32_t W, H, B, log2B;
    int32_t nbx, nby, nbins_scene;
    int32_t S, instanced;
    int64_t items;             // instanced ? S*T : T
    int64_t nbins_total;       // S * nbins_scene
};

// Snapped vertex of an indexed mesh (the Vertex Shader stage's output),
// 16 bytes; X == kBadVertex marks a vertex that drops its triangles.
struct __align__(16) VtxRec {
    int32_t X, Y;
    float z, iw;
};
constexpr int32_t kBadVertex = (int32_t)0x80000000;

// Workspace slices (device pointers carved out of the caller's buffer).
struct Ws {
    VtxRec *vtx;               // [S or 1][V] for indexed meshes, else unused
    TriRec *rec;               // [items]
    float4 *iw;                // [items] 1/w0, 1/w1, 1/w2 (unindexed meshes with a
                               // matrix; indexed ones read 1/w from the vertex
                               // records, and without a matrix it is 1)
    uint64_t *bbox;            // [items], kEmptyKey for culled triangles
    uint32_t *bin_count;       // [nbins_total]
    int32_t *bin_off;          // [nbins_total + 1]
    int32_t *vbin_off;         // [nbins_total + 1] first work item of each bin
                               // (PK_SCHED_SPLIT only, else NULL)
    int32_t *cursor;           // [nbins_total], between bin_count and misc: next
                               // free slot of each bin (set by the scan)
    uint32_t *misc;            // [kMiscWords], right after bin_count: [1] pair
                               // overflow flag, [8..15] DYNAMIC queue heads,
                               // [64..) kFragSlots 64-bit fragment partial sums;
                               // zeroed by pk_setup, heads and sums re-zeroed
                               // after each bin kernel that used them
    unsigned long long *keys;  // [S][H][W] winning (depth, primitive) keys
    int32_t *pairs;            // [pair_capacity]
    int64_t pair_capacity;
    int32_t split;             // PK_SCHED_SPLIT: pairs per work item; 0 otherwise
};

struct Shade {
    const float *color, *uv, *normal, *texture, *lights;
    int32_t tex_w, tex_h, num_lights, shading;
    float *out_color, *out_depth, *out_bary, *gbuf_n, *gbuf_a;
    int32_t *out_primid;
    unsigned long long *frag_count;
    int32_t flags;
    const float *alpha;        // [V] per-vertex opacity (layers > 0)
    int32_t layers;            // 0 = opaque, else layers composited per pixel
};

// Which scene an item belongs to and which triangle of the mesh it is.
struct ItemRef {
    int32_t s;       // scene
    int32_t t;       // scene-local triangle index (the primitive ID)
    int64_t g;       // index into the index buffer
    int64_t vbase;   // added to scene-local vertex numbers
};

__device__ inline ItemRef item_ref(const Geom &G, int64_t item) {
    ItemRef r;
    if (G.S == 1) {
        r.s = 0; r.t = (int32_t)item; r.g = item; r.vbase = 0;
    } else if (G.instanced) {
        // items < 2^31: a 32-bit divide instead of the 64-bit routine
        r.s = (int32_t)((uint32_t)item / (uint32_t)G.T);
        r.t = (int32_t)(item - (int64_t)r.s * G.T);
        r.g = r.t; r.vbase = 0;
    } else {
        int lo = 0, hi = G.S - 1;          // last scene with tri_off[s] <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (G.tri_off[mid] <= item) lo = mid; else hi = mid - 1;
        }
        r.s = lo;
        r.t = (int32_t)(item - G.tri_off[lo]);
        r.g = item;
        r.vbase = G.vtx_off[lo];
    }
    return r;
}

__device__ inline int64_t vertex_of(const Geom &G, const ItemRef &r, int k) {
    const int64_t local = G.idx ? (int64_t)G.idx[3 * r.g + k] : 3 * (int64_t)r.t + k;
    return r.vbase + local;
}

// Vertex shader stage: clip = MVP (x,y,z,1) with every product rounded and
// the sums taken left to right, NDC = clip * (1/w) with one correctly
// rounded reciprocal, viewport, 8-bit sub-pixel snap (round half to even).  Returns false for a vertex that drops its triangle.
__device__ inline bool vertex_stage_xyz(const Geom &G, float x, float y, float zz,
                                        const float *m, int32_t &X, int32_t &Y, float &z,
                                        float &iw) {
    float c0, c1, c2, c3;
    if (m) {
        float t;
        t = m[0] * x;  t = t + m[1] * y;  t = t + m[2] * zz;  t = t + m[3];  c0 = t;
        t = m[4] * x;  t = t + m[5] * y;  t = t + m[6] * zz;  t = t + m[7];  c1 = t;
        t = m[8] * x;  t = t + m[9] * y;  t = t + m[10] * zz; t = t + m[11]; c2 = t;
        t = m[12] * x; t = t + m[13] * y; t = t + m[14] * zz; t = t + m[15]; c3 = t;
    } else {
        c0 = x; c1 = y; c2 = zz; c3 = 1.0f;
    }
    bool ok = __builtin_isfinite(c0) && __builtin_isfinite(c1) && __builtin_isfinite(c2) &&
              __builtin_isfinite(c3) && c3 > 0.0f;
    const float w1 = 1.0f / c3;     // correctly rounded; NDC = clip * (1/w)
    const float xn = c0 * w1;
    const float yn = c1 * w1;
    const float zn = c2 * w1;
    const float xs = (xn + 1.0f) * (0.5f * (float)G.W);
    const float ys = (yn + 1.0f) * (0.5f * (float)G.H);
    ok = ok && __builtin_isfinite(zn) && __builtin_isfinite(w1);
    ok = ok && fabsf(xs) < 16384.0f && fabsf(ys) < 16384.0f;
    if (!ok) return false;
    X = (int32_t)rintf(xs * 256.0f);
    Y = (int32_t)rintf(ys * 256.0f);
    z = zn;
    iw = w1;
    return true;
}

__device__ inline bool vertex_stage(const Geom &G, int64_t v, const float *m, int32_t &X,
                                    int32_t &Y, float &z, float &iw) {
    return vertex_stage_xyz(G, G.pos[v], G.pos[G.V + v], G.pos[2 * G.V + v], m, X, Y, z, iw);
}

__device__ inline uint32_t bb_x0(uint64_t b) { return (uint32_t)(b & 0xffff); }
__device__ inline uint32_t bb_x1(uint64_t b) { return (uint32_t)((b >> 16) & 0xffff); }
__device__ inline uint32_t bb_y0(uint64_t b) { return (uint32_t)((b >> 32) & 0xffff); }
__device__ inline uint32_t bb_y1(uint64_t b) { return (uint32_t)(b >> 48); }

// Exclusive scan of one int per thread over a workgroup of TPB threads.
// s_wave needs TPB/64 ints.  Contains barriers: call from uniform control flow.
template <int TPB>
__device__ inline int block_exclusive_scan(int v, int *s_wave, int &total) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) s_wave[wid] = x;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < TPB / kWave; ++w) {
        const int t = s_wave[w];
        before += (w < wid) ? t : 0;
        tot += t;
    }
    total = tot;
    __syncthreads();
    return before + x - v;
}

// ---- wave-level aggregation of atomics on per-bin counters -------------
// Lanes of a wave often target the same bin (consecutive triangles of a
// mesh are neighbours on screen).  When the wave's keys change at most
// kCoherent times between neighbouring lanes, lanes are grouped by key and
// one lane per group issues a single atomic for the whole group; otherwise
// every lane issues its own.  key < 0 means "no update".  Must be called by
// every active lane of the wave (uniform control flow).
constexpr int kCoherent = 16;

__device__ inline uint64_t lanemask_lt() {
    const int lane = threadIdx.x & (kWave - 1);
    return lane ? (~0ull >> (kWave - lane)) : 0ull;
}

__device__ inline bool wave_keys_coherent(int key) {
    const int prev = __shfl_up(key, 1, kWave);
    const int lane = threadIdx.x & (kWave - 1);
    const bool boundary = key >= 0 && (lane == 0 || key != prev);
    return __popcll(__ballot(boundary)) <= kCoherent;
}

// counter[key] += 1 for every lane with key >= 0.
__device__ inline void agg_count(uint32_t *counter, int key) {
    if (wave_keys_coherent(key)) {
        uint64_t active = __ballot(key >= 0);
        const int lane = threadIdx.x & (kWave - 1);
        while (active) {
            const int leader = __ffsll((unsigned long long)active) - 1;
            const int k = __shfl(key, leader, kWave);
            const uint64_t same = __ballot(key == k) & active;
            if (lane == leader) atomicAdd(counter + k, (uint32_t)__popcll(same));
            active &= ~same;
        }
    } else if (key >= 0) {
        atomicAdd(counter + key, 1u);
    }
}

// slot = counter[key]++ for every lane with key >= 0 (distinct slots per
// lane; lanes with the same key get consecutive slots in lane order).
__device__ inline int32_t agg_slot(int32_t *counter, int key) {
    if (wave_keys_coherent(key)) {
        uint64_t active = __ballot(key >= 0);
        const int lane = threadIdx.x & (kWave - 1);
        int my_leader = lane, my_rank = 0, group = 0;
        while (active) {
            const int leader = __ffsll((unsigned long long)active) - 1;
            const int k = __shfl(key, leader, kWave);
            const uint64_t same = __ballot(key == k) & active;
            if (key == k) {
                my_leader = leader;
                my_rank = __popcll(same & lanemask_lt());
            }
            if (lane == leader) group = __popcll(same);
            active &= ~same;
        }
        int32_t base = 0;
        if (group) base = atomicAdd(counter + key, group);   // leaders, all at once
        base = __shfl(base, my_leader, kWave);
        return base + my_rank;
    }
    return key >= 0 ? atomicAdd(counter + key, 1) : 0;
}

__device__ inline int wave_max(int v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d, kWave));
    return v;
}

// Host launchers (defined in the .hip files).
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);
hipError_t launch_setup(const Geom &G, const Ws &w, hipStream_t st);
hipError_t launch_scan(const Geom &G, const Ws &w, int64_t *pairs_needed, hipStream_t st);
hipError_t launch_scatter(const Geom &G, const Ws &w, hipStream_t st);
hipError_t launch_assign(const Geom &G, const Ws &w, int64_t *pairs_needed, hipStream_t st);
// What a pk_raster_shade call launches after the bin kernel's depth test.
enum RasterMode : int {
    kRasterSplit = 0,      // keys to the workspace, then the per-pixel resolve pass
    kRasterFused = 1,      // resolve and shade inside the bin kernel
    kRasterKeysOnly = 2    // keys to the workspace only (pk_shade resolves later)
};
hipError_t launch_raster(const Geom &G, const Ws &w, const Shade &sh, int schedule, int tpb,
                         int groups, RasterMode mode, hipStream_t st);
hipError_t launch_resolve_pass(const Geom &G, const Ws &w, const Shade &sh, hipStream_t st);
hipError_t launch_deferred(const Geom &G, const Shade &sh, hipStream_t st);
hipError_t launch_backward(const Geom &G, const Shade &sh, const int32_t *primid,
                           const float *bary, const float *grad, float *grad_vcolor,
                           float *grad_tex, hipStream_t st);

}  // namespace pk
