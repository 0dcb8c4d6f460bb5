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
// DYNAMIC queue heads: kSubQueues per die, each on a 256-byte line of its
// own (atomics on words of one line serialize at the memory side as if on
// one address): head q at misc[kQueueBase + kQueueStride * q]
constexpr int kSubQueues = 8;
constexpr int kQueueBase = 64 + 2 * kFragSlots;
constexpr int kQueueStride = 64;
constexpr int kMiscWords = kQueueBase + kXcd * kSubQueues * kQueueStride;

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

// One staged triangle of a bin, in registers: edge functions normalised so
// that a sample is covered iff all three are > 0 (the top-left ownership bit
// is folded into the constant), clipped candidate rectangle, depth inputs.
// Edge values are integers below 2^48 held in float64: every product, sum and
// step below stays an integer below 2^53, so the float64 arithmetic is exact
// and equals the integer definition bit for bit (and feeds the float64
// barycentrics without conversions).
struct EdgeTri {
    int32_t A[3], Bc[3];   // e_k(P) = A_k Px + B_k Py + C_k   (P in 1/256 px)
    double C[3];
    float z[3];
    double inv;            // 1 / |A2|
    int32_t x0, y0, wdt, cnt, own, prim;
};

// Edge functions, ownership bits, depth inputs and the candidate rectangle
// (the sample bbox clipped to the pw x ph pixel window at (px0, py0)) of a
// snapped triangle; prim is the primitive number carried into the keys.
__device__ inline void edge_setup(const int32_t X[3], const int32_t Y[3], float z0, float z1,
                                  float z2, int32_t prim, int32_t px0, int32_t py0, int32_t pw,
                                  int32_t ph, int32_t W, int32_t H, EdgeTri &t) {
    const int64_t A2 = area2(X, Y);
    const double sinv = signed_inv_area(A2);
    const int sgn = A2 > 0 ? 1 : -1;
    t.own = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int ka = (k + 1) % 3, kb = (k + 2) % 3;   // edge v_ka -> v_kb, opposite v_k
        const int32_t dx = X[kb] - X[ka], dy = Y[kb] - Y[ka];
        const int32_t Ak = -sgn * dy, Bk = sgn * dx;
        const int own = (Ak > 0) || (Ak == 0 && Bk < 0);
        t.own |= own << k;
        t.A[k] = Ak;
        t.Bc[k] = Bk;
        t.C[k] = (double)(-((int64_t)Ak * X[ka] + (int64_t)Bk * Y[ka]) + own);
    }
    t.z[0] = z0;
    t.z[1] = z1;
    t.z[2] = z2;
    t.inv = sinv > 0.0 ? sinv : -sinv;
    int32_t bx0, bx1, by0, by1;
    sample_bbox(X, Y, W, H, bx0, bx1, by0, by1);
    t.x0 = max(bx0, px0);
    t.y0 = max(by0, py0);
    const int32_t x1 = min(bx1, px0 + pw - 1);
    const int32_t y1 = min(by1, py0 + ph - 1);
    t.wdt = x1 - t.x0 + 1;
    const int32_t hgt = y1 - t.y0 + 1;
    t.cnt = (t.wdt > 0 && hgt > 0) ? t.wdt * hgt : 0;
    t.prim = prim;
}

// Depth of a covered sample from its biased edge values: the float64
// barycentric form, then the (depth, primitive) key.  Returns false when the
// fragment is outside [0, 1).
__device__ inline bool depth_key(double e0, double e1, double e2, int own, double inv,
                                 float z0, float z1, float z2, uint32_t prim,
                                 unsigned long long &key) {
    const double be0 = (e0 - (double)(own & 1)) * inv;
    const double be1 = (e1 - (double)((own >> 1) & 1)) * inv;
    const double be2 = (e2 - (double)((own >> 2) & 1)) * inv;
    double zd = be0 * (double)z0;
    zd = zd + be1 * (double)z1;
    zd = zd + be2 * (double)z2;
    float z = (float)zd;
    z = z + 0.0f;
    key = ((unsigned long long)__float_as_uint(z) << 32) | prim;
    return 0.0f <= z && z < 1.0f;
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
    // PK_FLAG_TWO_LEVEL_BINS: a scene's bins are its nbins_f fine bins (B px)
    // followed by its coarse bins (4B px, nbx_c wide); nbins_scene counts both
    int32_t two_level, nbins_f, nbx_c, nby_c;
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
    int32_t *order;            // [nbins_total] DYNAMIC only (else NULL): each die's
                               // range of bins, heaviest first
    int32_t *vbin_off;         // [nbins_total + 1] first work item of each bin
                               // (PK_SCHED_SPLIT only, else NULL)
    int32_t *cursor;           // [nbins_total], between bin_count and misc: next
                               // free slot of each bin (set by the scan)
    uint32_t *misc;            // [kMiscWords], right after bin_count: [1] pair
                               // overflow flag, [64..) kFragSlots 64-bit fragment
                               // partial sums, [kQueueBase..) DYNAMIC queue heads;
                               // zeroed by pk_setup, heads and sums re-zeroed
                               // after each bin kernel that used them
    unsigned long long *keys;  // [S][H][W] winning (depth, primitive) keys
    int32_t *pairs;            // [pair_capacity]
    int64_t pair_capacity;
    int32_t split;             // PK_SCHED_SPLIT: pairs per work item; 0 otherwise
    // PK_SCHED_FRAGMENT_BINS: `pairs` holds the fragments instead, as
    // kFbPlanes planes of pair_capacity 16-byte entries; fb_mat [fb_groups]
    // [nbins] the per-workgroup fragment counts of each bin
    uint32_t *fb_mat;
    int32_t fb_groups;         // 0 = not this schedule
    int32_t fb_rounds;         // rounds of 1024 triangles per workgroup
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

// Lighting of the deferred pass: sum over the lights of max(0, n . l), in
// the lights' order.
__device__ inline float light_sum(const Shade &sh, float n0, float n1, float n2) {
    float lit = 0.0f;
    for (int l = 0; l < sh.num_lights; ++l) {
        const float *L = sh.lights + 3 * l;
        float d = n0 * L[0];
        d = d + n1 * L[1];
        d = d + n2 * L[2];
        d = d < 0.0f ? 0.0f : d;
        lit = (l == 0) ? d : lit + d;
    }
    return lit;
}

// Fragment shader of one covered sample from its float32 screen-space
// barycentrics bs_k and the three vertices' 1/w: perspective-correct b1, b2
// (b0 = 1 - b1 - b2), then the interpolated colour (modulated by the bilinear
// texture for TEXTURED), for DEFERRED the interpolated albedo and the unit
// interpolated normal, and for LIT that albedo times the sum over the lights
// of max(0, n . l).  c[k][ch] are vertex colours, ex[k][ch] the uv
// (TEXTURED) or normal (DEFERRED) of vertex k.
struct FragOut {
    float b1, b2;
    float rgb[3];
    float n[3];
};

template <int SHADE>
__device__ inline void shade_fragment(const Shade &sh, float bs0, float bs1, float bs2, float iw0,
                                      float iw1, float iw2, const float c[3][3],
                                      const float ex[3][3], FragOut &o) {
    const float qq0 = bs0 * iw0, qq1 = bs1 * iw1, qq2 = bs2 * iw2;
    const float Q = (qq0 + qq1) + qq2;
    const float b1 = qq1 / Q, b2 = qq2 / Q;
    const float b0 = (1.0f - b1) - b2;
    o.b1 = b1;
    o.b2 = b2;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float acc = b0 * c[0][ch];
        acc = acc + b1 * c[1][ch];
        acc = acc + b2 * c[2][ch];
        o.rgb[ch] = acc;
    }
    if (SHADE == PK_SHADE_TEXTURED) {
        float u = b0 * ex[0][0];
        u = u + b1 * ex[1][0];
        u = u + b2 * ex[2][0];
        float vv = b0 * ex[0][1];
        vv = vv + b1 * ex[1][1];
        vv = vv + b2 * ex[2][1];
        const float su = u * (float)sh.tex_w - 0.5f, sv = vv * (float)sh.tex_h - 0.5f;
        const float fi = floorf(su), fj = floorf(sv);
        const float fs = su - fi, ft = sv - fj;
        const float ci = fminf(fmaxf(fi, -1.0f), (float)sh.tex_w);
        const float cj = fminf(fmaxf(fj, -1.0f), (float)sh.tex_h);
        const int i0 = min(max((int)ci, 0), sh.tex_w - 1), i1 = min(max((int)ci + 1, 0), sh.tex_w - 1);
        const int j0 = min(max((int)cj, 0), sh.tex_h - 1), j1 = min(max((int)cj + 1, 0), sh.tex_h - 1);
        const float w00 = (1.0f - fs) * (1.0f - ft), w10 = fs * (1.0f - ft);
        const float w01 = (1.0f - fs) * ft, w11 = fs * ft;
        const float *t00 = sh.texture + 3 * ((int64_t)j0 * sh.tex_w + i0);
        const float *t10 = sh.texture + 3 * ((int64_t)j0 * sh.tex_w + i1);
        const float *t01 = sh.texture + 3 * ((int64_t)j1 * sh.tex_w + i0);
        const float *t11 = sh.texture + 3 * ((int64_t)j1 * sh.tex_w + i1);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float tc = w00 * t00[ch];
            tc = tc + w10 * t10[ch];
            tc = tc + w01 * t01[ch];
            tc = tc + w11 * t11[ch];
            o.rgb[ch] = o.rgb[ch] * tc;
        }
    }
    if (SHADE == PK_SHADE_DEFERRED || SHADE == PK_SHADE_LIT) {
        float n[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float acc = b0 * ex[0][ch];
            acc = acc + b1 * ex[1][ch];
            acc = acc + b2 * ex[2][ch];
            n[ch] = acc;
        }
        float nn = n[0] * n[0];
        nn = nn + n[1] * n[1];
        nn = nn + n[2] * n[2];
        o.n[0] = o.n[1] = o.n[2] = 0.0f;
        if (nn != 0.0f) {
            const float len = sqrtf(nn);
            o.n[0] = n[0] / len; o.n[1] = n[1] / len; o.n[2] = n[2] / len;
        }
    }
    if (SHADE == PK_SHADE_LIT) {
        const float lit = light_sum(sh, o.n[0], o.n[1], o.n[2]);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) o.rgb[ch] = o.rgb[ch] * lit;
    }
}

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
    // correctly rounded; NDC = clip * (1/w).  Without a matrix w is 1 and so
    // is its reciprocal: the division is skipped, the value is the same
    const float w1 = m ? 1.0f / c3 : 1.0f;
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

// Setup of one triangle in three steps, so that a thread can issue the loads
// of all its triangles before it waits for any: (1) the vertex numbers (the
// index buffer's three entries issued together, checked only in the next
// step), (2) the vertices (snapped records of k_vertex, or raw positions),
// (3) transform if needed, snap, cull and write the record.
struct TriIn {
    int64_t v[3];          // vertex numbers (valid after setup_fetch)
    int4 q[3];             // indexed: snapped X, Y, z, 1/w; else raw x, y, z
    int64_t vbase;         // added to scene-local vertex numbers
    int64_t vlo, vhi;      // the vertices the triangle's scene owns
    int64_t g;             // indexed: the triangle's entry in the index buffer
    int32_t iv[3];         // indexed: the index buffer's entries (in flight)
    int32_t tloc;          // scene-local triangle number
    int32_t s;             // scene
    bool ok;
};

__device__ inline void setup_indices(const Geom &G, int64_t item, TriIn &t) {
    t.s = 0;
    t.g = 0;
    t.ok = item < G.items;
    if (!t.ok) return;
    const ItemRef r = item_ref(G, item);
    t.s = r.s;
    t.tloc = r.t;
    t.vbase = r.vbase;
    // a triangle may only use the vertices of its own scene
    const bool own_range = G.S > 1 && !G.instanced;
    t.vlo = own_range ? (int64_t)G.vtx_off[r.s] : 0;
    t.vhi = own_range ? (int64_t)G.vtx_off[r.s + 1] : G.V;
    t.g = r.g;
}

// Indexed meshes: the index buffer's three entries, one load.  A caller with
// several triangles issues these for all of them in one branch on G.idx, so
// that no wait for one triangle's entries comes before the next one's load.
// A lane without a triangle loads entry 0 instead (it exists whenever the
// kernel runs: items > 0 means at least one triangle) and ignores it, so the
// loads need no branch of their own.
__device__ inline void setup_index_load(const Geom &G, TriIn &t) {
    const int32_t *ip = G.idx + 3 * (t.ok ? t.g : 0);
    t.iv[0] = ip[0];
    t.iv[1] = ip[1];
    t.iv[2] = ip[2];
}

// WHOLE: keep each loaded vertex record's four words live in the indexed
// branch, so that the compiler issues one 16-byte load per record instead of
// merging the branch with the unindexed one into separate 4-byte loads.  It
// also waits for the records there: for callers that use them right away.
template <bool WHOLE = false>
__device__ inline void setup_fetch(const Geom &G, const Ws &w, TriIn &t) {
    if (!t.ok) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t local = G.idx ? (int64_t)t.iv[k] : 3 * (int64_t)t.tloc + k;
        t.v[k] = t.vbase + local;
        if (t.v[k] < t.vlo || t.v[k] >= t.vhi || t.v[k] >= G.V) t.ok = false;
    }
    if (!t.ok) return;
    if (G.idx) {
        const int64_t vb = G.instanced ? (int64_t)t.s * G.V : 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) t.q[k] = reinterpret_cast<const int4 *>(w.vtx)[vb + t.v[k]];
        if (WHOLE) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                __asm__ volatile("" : : "v"(t.q[k].x), "v"(t.q[k].y), "v"(t.q[k].z), "v"(t.q[k].w));
        }
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            t.q[k] = make_int4(__float_as_int(G.pos[t.v[k]]), __float_as_int(G.pos[G.V + t.v[k]]),
                               __float_as_int(G.pos[2 * G.V + t.v[k]]), 0);
    }
}

// Snapped vertices, depth and 1/w of a triangle from its fetched inputs
// (indexed: the Vertex Shader's records; else the vertex transform here);
// returns the packed pixel bbox, or kEmptyKey when the triangle is culled
// (a dropped vertex, zero area, or no sample centre in its box).
__device__ inline uint64_t setup_snap(const Geom &G, const TriIn &t, int32_t X[3], int32_t Y[3],
                                      float z[3], float iw[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { X[k] = 0; Y[k] = 0; z[k] = 0.0f; iw[k] = 0.0f; }
    bool ok = t.ok;
    if (ok) {
        if (G.idx) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ok = ok && t.q[k].x != kBadVertex;
                X[k] = t.q[k].x; Y[k] = t.q[k].y;
                z[k] = __int_as_float(t.q[k].z); iw[k] = __int_as_float(t.q[k].w);
            }
        } else {
            const float *m = G.mvp ? G.mvp + 16 * (int64_t)t.s : nullptr;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                ok = vertex_stage_xyz(G, __int_as_float(t.q[k].x), __int_as_float(t.q[k].y),
                                      __int_as_float(t.q[k].z), m, X[k], Y[k], z[k], iw[k]) && ok;
        }
    }
    if (!ok) return kEmptyKey;
    const int64_t A2 = area2(X, Y);
    int32_t x0, x1, y0, y1;
    sample_bbox(X, Y, G.W, G.H, x0, x1, y0, y1);
    if (A2 == 0 || x0 > x1 || y0 > y1) return kEmptyKey;
    return (uint64_t)x0 | ((uint64_t)x1 << 16) | ((uint64_t)y0 << 32) | ((uint64_t)y1 << 48);
}

// The 32-byte setup record of a live triangle (and its 1/w entry when an
// unindexed mesh has a matrix: without one 1/w is exactly 1).
__device__ inline void store_record(const Geom &G, const Ws &w, int64_t item, const int32_t X[3],
                                    const int32_t Y[3], const float z[3], const float iw[3]) {
    uint32_t xy[5];
    pack_xy(X, Y, xy);
    uint4 *dst = reinterpret_cast<uint4 *>(w.rec + item);
    dst[0] = make_uint4(xy[0], xy[1], xy[2], xy[3]);
    dst[1] = make_uint4(xy[4], __float_as_uint(z[0]), __float_as_uint(z[1]), __float_as_uint(z[2]));
    if (!G.idx && G.mvp) w.iw[item] = make_float4(iw[0], iw[1], iw[2], 0.0f);
}

// Whole-screen bins, unindexed meshes: the per-pixel resolve is the only
// reader of the setup record there, and it reads the packed snapped vertices
// only, so the depth-test kernel stores just those five words per triangle
// (20 bytes at 20-byte stride, in the record buffer), not the 32-byte record.
__device__ inline uint32_t *xy20_of(const Ws &w, int64_t item) {
    return reinterpret_cast<uint32_t *>(w.rec) + 5 * item;
}

__device__ inline void store_xy20(const Ws &w, int64_t item, const int32_t X[3],
                                  const int32_t Y[3]) {
    uint32_t xy[5];
    pack_xy(X, Y, xy);
    uint32_t *dst = xy20_of(w, item);
#pragma unroll
    for (int k = 0; k < 5; ++k) dst[k] = xy[k];
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
// PK_SCHED_FRAGMENT_BINS (k_fragbin.hip): fragment counts per bin (pk_setup),
// the prefix sum (pk_assign_bin), fragment shading and scatter, then the
// per-bin depth test and composite (pk_raster_shade).
hipError_t launch_epilogue(const Ws &w, unsigned long long *frag_count, int rewind,
                           hipStream_t st);
hipError_t launch_fb_count(const Geom &G, const Ws &w, hipStream_t st);
hipError_t launch_fb_assign(const Geom &G, const Ws &w, int64_t *pairs_needed, hipStream_t st);
hipError_t launch_fb_raster(const Geom &G, const Ws &w, const Shade &sh, bool light,
                            hipStream_t st);
constexpr int kFbThreads = 256;        // threads of a fragment workgroup
constexpr int kFbRoundTris = 1024;     // triangles per round (4 per thread)
constexpr int kFbMaxBins = 8192;       // LDS counters of a fragment workgroup
hipError_t launch_backward(const Geom &G, const Shade &sh, const int32_t *primid,
                           const float *bary, const float *grad, float *grad_vcolor,
                           float *grad_tex, hipStream_t st);

}  // namespace pk
