// k_fragbin.hip -- PK_SCHED_FRAGMENT_BINS: bins of shaded fragments instead
// of bins of triangles.
//
// The Rasterizer and the Fragment Shader form one stage with whole-screen
// bins (Sec. 4.4: 0x0 bins are the screen; the two stages fused as in
// Sec. 5.2.1), scheduled over the input triangles in submission order, so
// every triangle's vertices and attributes are read once, coalesced.  Each
// covered sample is shaded where it is found and goes to the bin of its
// pixel; the Depth Test and Composite stage then runs per bin, its key tile
// in LDS.  The bins are built by counting, a prefix sum and a scatter, with
// the counts of a workgroup's many triangles summed in LDS first: the only
// device-scope atomics are one per (workgroup, bin), on consecutive
// addresses.  Nothing is gathered at random: no triangle record is re-read
// per bin and no winner's attributes are fetched per pixel, which is what
// bounds the triangle-binned pipeline on many tiny triangles.
//
//   k_fb_count     (pk_setup) workgroup g takes fb_rounds rounds of 1024
//                  consecutive triangles, counts the fragments of every bin
//                  in LDS, writes its row of the count matrix and adds each
//                  count to the bin's total
//   k_scan         (pk_assign_bin) exclusive prefix sum of the totals
//   k_fb_scatter   (pk_raster_shade) the same triangles again: workgroup g
//                  reserves its run of each bin, rasterizes and shades every
//                  fragment and writes it to its slot
//   k_fb_composite (pk_raster_shade) one workgroup per bin: depth test of
//                  every fragment into the LDS key tile, then the winner of
//                  each pixel writes its shaded values, and empty pixels
//                  their empty values
//
// A fragment is kFbPlanes 16-byte entries in separate planes, so that the
// depth test reads only the first: (pixel in bin, primitive, depth bits,
// b1), (b2, colour or albedo), (unit normal) for deferred shading.  The
// fragment shader is the one of the per-pixel resolve (shade_fragment), fed
// the same float32 barycentrics, so the image is the same bit for bit.
#include "pk_internal.h"

#pragma clang fp contract(off)

namespace pk {

namespace {

struct F3 {
    float x, y, z;
};

// Boxes of up to kFbExpandMax pixels are covered by the lane-balanced
// expansion, larger ones by a whole-wave sweep.  Start marks carry a block
// tag in their upper bits (below kFbNoTag).
constexpr uint32_t kFbExpandMax = 1u << 18;
constexpr uint32_t kFbNoTag = 0xffffffffu >> 6;

// One triangle of a fragment workgroup: edges and candidate box (the sample
// bbox on the screen), 1/w and vertex numbers.
struct FbTri {
    EdgeTri e;
    float iw[3];
    int32_t v[3];
};

// Transform, snap and set up triangle `item` of the (single) scene; e.cnt
// is 0 when it is culled (a bad vertex, zero area, or no sample in its box).
__device__ inline void fb_load(const Geom &G, const Ws &w, int64_t item, FbTri &t) {
    t.e.cnt = 0;
    if (item >= G.items) return;
    int32_t X[3], Y[3];
    float z[3];
    bool ok = true;
    if (G.idx) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int32_t v = G.idx[3 * item + k];
            ok = ok && v >= 0 && (int64_t)v < G.V;
            t.v[k] = ok ? v : 0;
        }
        if (!ok) return;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int4 q = reinterpret_cast<const int4 *>(w.vtx)[t.v[k]];
            ok = ok && q.x != kBadVertex;
            X[k] = q.x;
            Y[k] = q.y;
            z[k] = __int_as_float(q.z);
            t.iw[k] = __int_as_float(q.w);
        }
    } else {
        const int64_t v0 = 3 * item;
        if (v0 + 2 >= G.V) return;
        t.v[0] = (int32_t)v0; t.v[1] = (int32_t)v0 + 1; t.v[2] = (int32_t)v0 + 2;
        // the three vertices are consecutive in every plane: one 12-byte load each
        const F3 px = *reinterpret_cast<const F3 *>(G.pos + v0);
        const F3 py = *reinterpret_cast<const F3 *>(G.pos + G.V + v0);
        const F3 pz = *reinterpret_cast<const F3 *>(G.pos + 2 * G.V + v0);
        const float xs[3] = {px.x, px.y, px.z}, ys[3] = {py.x, py.y, py.z}, zs[3] = {pz.x, pz.y, pz.z};
#pragma unroll
        for (int k = 0; k < 3; ++k)
            ok = vertex_stage_xyz(G, xs[k], ys[k], zs[k], G.mvp, X[k], Y[k], z[k], t.iw[k]) && ok;
    }
    if (!ok || area2(X, Y) == 0) return;
    edge_setup(X, Y, z[0], z[1], z[2], (int32_t)item, 0, 0, G.W, G.H, G.W, G.H, t.e);
}

// The vertex attributes the fragment shader needs: colours, and uv
// (TEXTURED) or normals (DEFERRED), as [vertex][channel].
template <int SHADE>
__device__ inline void fb_attribs(const Geom &G, const Shade &sh, const FbTri &t, float c[3][3],
                                  float ex[3][3]) {
    const int64_t V = G.V;
    if (!G.idx) {
        const int64_t v0 = t.v[0];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const F3 a = *reinterpret_cast<const F3 *>(sh.color + ch * V + v0);
            c[0][ch] = a.x; c[1][ch] = a.y; c[2][ch] = a.z;
        }
        if (SHADE == PK_SHADE_TEXTURED) {
#pragma unroll
            for (int ch = 0; ch < 2; ++ch) {
                const F3 a = *reinterpret_cast<const F3 *>(sh.uv + ch * V + v0);
                ex[0][ch] = a.x; ex[1][ch] = a.y; ex[2][ch] = a.z;
            }
        }
        if (SHADE == PK_SHADE_DEFERRED || SHADE == PK_SHADE_LIT) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const F3 a = *reinterpret_cast<const F3 *>(sh.normal + ch * V + v0);
                ex[0][ch] = a.x; ex[1][ch] = a.y; ex[2][ch] = a.z;
            }
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) c[k][ch] = sh.color[ch * V + t.v[k]];
        if (SHADE == PK_SHADE_TEXTURED) {
            ex[k][0] = sh.uv[t.v[k]];
            ex[k][1] = sh.uv[V + t.v[k]];
        }
        if (SHADE == PK_SHADE_DEFERRED || SHADE == PK_SHADE_LIT) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) ex[k][ch] = sh.normal[ch * V + t.v[k]];
        }
    }
}

// Fragment i's entry in plane j: blocks of 64 fragments hold each plane's 64
// entries in turn ([block][plane][64] x 16 bytes), so that one plane of
// consecutive fragments is read in 1-KB runs whatever the capacity.
template <int SHADE>
__device__ inline int4 &fb_at(const Ws &w, int64_t i, int j) {
    constexpr int P = SHADE == PK_SHADE_DEFERRED ? 3 : 2;
    return reinterpret_cast<int4 *>(w.pairs)[((i >> 6) * P + j) * 64 + (i & 63)];
}

// One covered sample (px, py) with biased edge values e_k: COUNT adds it to
// its bin's LDS counter, else it takes the next slot of the bin's run and is
// shaded and stored there.  Returns 1 (it counts as a fragment whatever its
// depth).
template <bool COUNT, int SHADE>
__device__ inline uint32_t fb_emit(const Geom &G, const Ws &w, const Shade &sh, uint32_t *s_cnt,
                                   uint32_t total, int px, int py, double e0, double e1,
                                   double e2, int own,
                                   double inv, float z0, float z1, float z2, uint32_t prim,
                                   const float iw[3], const float c[3][3], const float ex[3][3]) {
    unsigned long long key;
    if (!depth_key(e0, e1, e2, own, inv, z0, z1, z2, prim, key)) return 1;
    const int bin = (py >> G.log2B) * G.nbx + (px >> G.log2B);
    if (COUNT) {
        atomicAdd(&s_cnt[bin], 1u);
        return 1;
    }
    const uint32_t slot = atomicAdd(&s_cnt[bin], 1u);
    // the runs were sized by the counting pass over the same arithmetic; the
    // bound only keeps a stray slot inside the frame's fragments
    if (slot >= total) return 1;
    // the resolve's float32 barycentrics: (E_k / |A2|) with the winding's sign
    const float bs0 = (float)((e0 - (double)(own & 1)) * inv);
    const float bs1 = (float)((e1 - (double)((own >> 1) & 1)) * inv);
    const float bs2 = (float)((e2 - (double)((own >> 2) & 1)) * inv);
    FragOut o;
    shade_fragment<SHADE>(sh, bs0, bs1, bs2, iw[0], iw[1], iw[2], c, ex, o);
    const int lp = (py & (G.B - 1)) * G.B + (px & (G.B - 1));
    fb_at<SHADE>(w, slot, 0) = make_int4(lp, (int)prim, (int)(uint32_t)(key >> 32), __float_as_int(o.b1));
    fb_at<SHADE>(w, slot, 1) = make_int4(__float_as_int(o.b2), __float_as_int(o.rgb[0]),
                                         __float_as_int(o.rgb[1]), __float_as_int(o.rgb[2]));
    if (SHADE == PK_SHADE_DEFERRED)
        fb_at<SHADE>(w, slot, 2) = make_int4(__float_as_int(o.n[0]), __float_as_int(o.n[1]),
                                             __float_as_int(o.n[2]), 0);
    return 1;
}

// The counting pass (COUNT) and the scatter pass over the same triangles:
// workgroup g takes rounds r = 0..fb_rounds-1 of 1024 triangles, a thread
// one triangle of each quarter.  The candidate pixels of a wave's triangles
// are shared out evenly over its lanes (below); boxes beyond kFbExpandMax
// pixels are swept by the whole wave.  s_cnt (dynamic LDS, one word per
// bin): the counts, or the next free slot of each of the workgroup's runs.
template <bool COUNT, int SHADE>
__global__ __launch_bounds__(kFbThreads) void k_fb_pass(Geom G, Ws w, Shade sh) {
    extern __shared__ uint32_t s_cnt[];
    __shared__ unsigned long long s_frag[kFbThreads / kWave];
    __shared__ uint32_t s_mark[kFbThreads];
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int64_t nbins = G.nbins_total;
    const int64_t g = blockIdx.x;
    uint32_t *row = w.fb_mat + g * nbins;
    uint32_t total_frags = 0;
    uint32_t *mark = s_mark + (tid & ~(kWave - 1));   // this wave's start marks
    mark[lane] = 0xffffffffu;
    uint32_t tag = 0;
    if (COUNT) {
        for (int64_t b = tid; b < nbins; b += kFbThreads) s_cnt[b] = 0u;
    } else {
        if (w.misc[1]) return;   // fragment capacity exceeded: nothing is written
        total_frags = (uint32_t)w.bin_off[nbins];
        // reserve this workgroup's run of every bin it has fragments in
        for (int64_t b = tid; b < nbins; b += kFbThreads) {
            const uint32_t cnt = row[b];
            s_cnt[b] = cnt ? (uint32_t)atomicAdd(&w.cursor[b], (int32_t)cnt) : 0u;
        }
    }
    __syncthreads();
    uint32_t frags = 0;
    const int64_t first = g * (int64_t)kFbRoundTris * w.fb_rounds;
#pragma unroll 1
    for (int r = 0; r < w.fb_rounds * (kFbRoundTris / kFbThreads); ++r) {
        const int64_t item = first + (int64_t)r * kFbThreads + tid;
        FbTri t;
        fb_load(G, w, item, t);
        float c[3][3], ex[3][3];
        if (!COUNT && t.e.cnt > 0) fb_attribs<SHADE>(G, sh, t, c, ex);
        const EdgeTri &e = t.e;
        // Candidates (box pixels) of the wave's 64 triangles laid end to end
        // and handed out 64 at a time, one per lane, so that the lanes stay
        // busy whatever the boxes' sizes (micropolygon boxes range from one
        // pixel to dozens).  The owner of candidate j is the last triangle
        // whose run starts at or before j: every triangle starting inside
        // the block marks its start with its lane number (marks carry the
        // block's tag, so the plane is never cleared); a ballot of the live
        // marks and a leading-zero count find the nearest mark at or below
        // j.  The owner's edge data reach the lane by lane shuffles.
        const uint32_t n = (e.cnt > 0 && (uint32_t)e.cnt <= kFbExpandMax) ? (uint32_t)e.cnt : 0u;
        uint32_t incl = n;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += y;
        }
        const uint32_t start = incl - n;
        const uint32_t total = __shfl(incl, kWave - 1, kWave);
        int carry = 0;
#pragma unroll 1
        for (uint32_t b0 = 0; b0 < total; b0 += kWave) {
            if (tag + 1 >= kFbNoTag) {      // (never in practice) recycle the tags
                mark[lane] = 0xffffffffu;
                tag = 0;
            }
            if (n > 0 && start >= b0 && start < b0 + kWave)
                mark[start - b0] = (tag << 6) | (uint32_t)lane;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const uint32_t mk = mark[lane];
            const uint64_t live = __ballot((mk >> 6) == tag);
            const uint64_t upto = live & ((2ull << lane) - 1ull);
            const int from = upto ? 63 - __clzll((long long)upto) : 0;
            const int marked = __shfl((int)(mk & (kWave - 1)), from, kWave);
            const int o = upto ? marked : carry;
            carry = __shfl(o, kWave - 1, kWave);
            ++tag;
            const uint32_t j = b0 + (uint32_t)lane;
            const uint32_t o_start = __shfl(start, o, kWave);
            const int o_x0 = __shfl(e.x0, o, kWave), o_y0 = __shfl(e.y0, o, kWave);
            const int32_t o_wdt = __shfl(e.wdt, o, kWave);
            double A[3], Bv[3], C[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                A[k] = (double)__shfl(e.A[k], o, kWave);
                Bv[k] = (double)__shfl(e.Bc[k], o, kWave);
                C[k] = __shfl(e.C[k], o, kWave);
            }
            // row and column of the candidate in the owner's box: a float
            // quotient (error below one for runs under 2^18) and one correction
            const int32_t local = (int32_t)(j - o_start);
            int32_t row = (int32_t)((float)local * __builtin_amdgcn_rcpf((float)o_wdt));
            int32_t col = local - row * o_wdt;
            if (col < 0) { --row; col += o_wdt; }
            else if (col >= o_wdt) { ++row; col -= o_wdt; }
            const int px = o_x0 + col, py = o_y0 + row;
            const double Px = (double)(256 * px + 128), Py = (double)(256 * py + 128);
            const double e0 = A[0] * Px + Bv[0] * Py + C[0];
            const double e1 = A[1] * Px + Bv[1] * Py + C[1];
            const double e2 = A[2] * Px + Bv[2] * Py + C[2];
            const bool cov = j < total && e0 > 0.0 && e1 > 0.0 && e2 > 0.0;
            if (!__ballot(cov)) continue;
            float z[3], iw[3], cc[3][3], ee[3][3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                z[k] = __shfl(e.z[k], o, kWave);
                if (!COUNT) {
                    iw[k] = __shfl(t.iw[k], o, kWave);
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) {
                        cc[k][ch] = __shfl(c[k][ch], o, kWave);
                        if (SHADE != PK_SHADE_GOURAUD) ee[k][ch] = __shfl(ex[k][ch], o, kWave);
                    }
                }
            }
            const double inv = __shfl(e.inv, o, kWave);
            const int own = __shfl(e.own, o, kWave);
            const uint32_t prim = (uint32_t)__shfl(e.prim, o, kWave);
            if (cov)
                frags += fb_emit<COUNT, SHADE>(G, w, sh, s_cnt, total_frags, px, py, e0, e1, e2, own,
                                               inv, z[0], z[1], z[2], prim, iw, cc, ee);
        }
        // boxes beyond the expansion's run limit: the wave sweeps each in
        // turn, one pixel per lane; the edge values are evaluated directly
        // (integers below 2^53, exact)
        uint64_t big = __ballot((uint32_t)e.cnt > kFbExpandMax);
        while (big) {
            const int l = __ffsll((unsigned long long)big) - 1;
            big &= big - 1;
            double A[3], Bv[3], C[3];
            float z[3], iw[3], cc[3][3], ee[3][3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                A[k] = (double)__shfl(e.A[k], l, kWave);
                Bv[k] = (double)__shfl(e.Bc[k], l, kWave);
                C[k] = __shfl(e.C[k], l, kWave);
                z[k] = __shfl(e.z[k], l, kWave);
                iw[k] = __shfl(t.iw[k], l, kWave);
                if (!COUNT) {
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) {
                        cc[k][ch] = __shfl(c[k][ch], l, kWave);
                        ee[k][ch] = __shfl(ex[k][ch], l, kWave);
                    }
                }
            }
            const double inv = __shfl(e.inv, l, kWave);
            const int x0 = __shfl(e.x0, l, kWave), y0 = __shfl(e.y0, l, kWave);
            const uint32_t wdt = (uint32_t)__shfl(e.wdt, l, kWave);
            const int cnt = __shfl(e.cnt, l, kWave), own = __shfl(e.own, l, kWave);
            const uint32_t prim = (uint32_t)__shfl(e.prim, l, kWave);
#pragma unroll 1
            for (int i = lane; i < cnt; i += kWave) {
                const uint32_t rr = (uint32_t)i / wdt, cl = (uint32_t)i - rr * wdt;
                const int px = x0 + (int)cl, py = y0 + (int)rr;
                const double Px = (double)(256 * px + 128), Py = (double)(256 * py + 128);
                const double e0 = A[0] * Px + Bv[0] * Py + C[0];
                const double e1 = A[1] * Px + Bv[1] * Py + C[1];
                const double e2 = A[2] * Px + Bv[2] * Py + C[2];
                if (e0 > 0.0 && e1 > 0.0 && e2 > 0.0)
                    frags += fb_emit<COUNT, SHADE>(G, w, sh, s_cnt, total_frags, px, py, e0, e1, e2, own, inv,
                                                   z[0], z[1], z[2], prim, iw, cc, ee);
            }
        }
    }
    if (!COUNT) return;
    __syncthreads();
    // this workgroup's row of the count matrix, and the bins' totals (one
    // atomic per bin with fragments, on consecutive addresses)
    for (int64_t b = tid; b < nbins; b += kFbThreads) {
        const uint32_t cnt = s_cnt[b];
        row[b] = cnt;
        if (cnt) atomicAdd(&w.bin_count[b], cnt);
    }
    // covered samples: wave sums, then one atomic on this workgroup's partial slot
    unsigned long long f = frags;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) f += __shfl_down(f, d, kWave);
    if (lane == 0) s_frag[tid / kWave] = f;
    __syncthreads();
    if (tid == 0) {
        unsigned long long tot = 0;
        for (int i = 0; i < kFbThreads / kWave; ++i) tot += s_frag[i];
        unsigned long long *slots = reinterpret_cast<unsigned long long *>(w.misc + 64);
        if (tot) atomicAdd(&slots[blockIdx.x % kFragSlots], tot);
    }
}

// Depth Test and Composite of one bin: the bin's fragments' keys into the
// LDS tile, then each pixel's winner (the fragment whose key is the tile's:
// keys are unique per pixel, a triangle covering a sample once) writes its
// targets, and empty pixels theirs.  LIGHT: also the deferred lighting.
template <int B, int TPB, int SHADE, bool LIGHT>
__global__ __launch_bounds__(TPB) void k_fb_composite(Geom G, Ws w, Shade sh) {
    __shared__ unsigned long long s_key[B * B];
    const int tid = threadIdx.x;
    const int32_t bin = (int32_t)blockIdx.x;
    const int32_t by = bin / G.nbx, bx = bin - by * G.nbx;
    const int32_t px0 = bx * B, py0 = by * B;
    const int32_t pw = min(B, G.W - px0), ph = min(B, G.H - py0);
    const bool overflow = w.misc[1] != 0;
    const int32_t beg = overflow ? 0 : w.bin_off[bin];
    const int32_t end = overflow ? 0 : w.bin_off[bin + 1];
    for (int i = tid; i < B * B; i += TPB) s_key[i] = kEmptyKey;
    __syncthreads();
#pragma unroll 1
    for (int32_t i = beg + tid; i < end; i += TPB) {
        const int4 q = fb_at<SHADE>(w, i, 0);
        atomicMin(&s_key[q.x & (B * B - 1)], ((unsigned long long)(uint32_t)q.z << 32) | (uint32_t)q.y);
    }
    __syncthreads();
#pragma unroll 1
    for (int32_t i = beg + tid; i < end; i += TPB) {
        const int4 q = fb_at<SHADE>(w, i, 0);
        const unsigned long long key = ((unsigned long long)(uint32_t)q.z << 32) | (uint32_t)q.y;
        const int lp = q.x & (B * B - 1);
        if (s_key[lp] != key) continue;
        const int lx = lp & (B - 1), ly = lp / B;
        if (lx >= pw || ly >= ph) continue;
        const int64_t p = (int64_t)(py0 + ly) * G.W + px0 + lx;
        const int4 a = fb_at<SHADE>(w, i, 1);
        if (sh.out_depth) sh.out_depth[p] = __int_as_float(q.z);
        if (sh.out_primid) sh.out_primid[p] = q.y;
        if (sh.out_bary)
            reinterpret_cast<float2 *>(sh.out_bary)[p] = make_float2(__int_as_float(q.w), __int_as_float(a.x));
        const float r = __int_as_float(a.y), gg = __int_as_float(a.z), bb = __int_as_float(a.w);
        if (SHADE == PK_SHADE_DEFERRED) {
            const int4 nq = fb_at<SHADE>(w, i, 2);
            const float n0 = __int_as_float(nq.x), n1 = __int_as_float(nq.y), n2 = __int_as_float(nq.z);
            *reinterpret_cast<F3 *>(sh.gbuf_n + 3 * p) = F3{n0, n1, n2};
            *reinterpret_cast<F3 *>(sh.gbuf_a + 3 * p) = F3{r, gg, bb};
            if (LIGHT) {
                const float lit = light_sum(sh, n0, n1, n2);
                reinterpret_cast<float4 *>(sh.out_color)[p] = make_float4(r * lit, gg * lit, bb * lit, 1.0f);
            }
        } else if (sh.out_color) {
            reinterpret_cast<float4 *>(sh.out_color)[p] = make_float4(r, gg, bb, 1.0f);
        }
    }
    // empty pixels (the key tile is final since the barrier above)
#pragma unroll 1
    for (int i = tid; i < B * B; i += TPB) {
        const int lx = i & (B - 1), ly = i / B;
        if (lx >= pw || ly >= ph || s_key[i] != kEmptyKey) continue;
        const int64_t p = (int64_t)(py0 + ly) * G.W + px0 + lx;
        if (sh.out_depth) sh.out_depth[p] = 1.0f;
        if (sh.out_primid) sh.out_primid[p] = -1;
        if (sh.out_bary) reinterpret_cast<float2 *>(sh.out_bary)[p] = make_float2(0.0f, 0.0f);
        if (SHADE == PK_SHADE_DEFERRED) {
            *reinterpret_cast<F3 *>(sh.gbuf_n + 3 * p) = F3{0.0f, 0.0f, 0.0f};
            *reinterpret_cast<F3 *>(sh.gbuf_a + 3 * p) = F3{0.0f, 0.0f, 0.0f};
            if (LIGHT) reinterpret_cast<float4 *>(sh.out_color)[p] = make_float4(0, 0, 0, 0);
        } else if (sh.out_color) {
            reinterpret_cast<float4 *>(sh.out_color)[p] = make_float4(0, 0, 0, 0);
        }
    }
}

template <bool COUNT, int SHADE>
hipError_t launch_pass(const Geom &G, const Ws &w, const Shade &sh, hipStream_t st) {
    hipLaunchKernelGGL((k_fb_pass<COUNT, SHADE>), dim3((unsigned)w.fb_groups), dim3(kFbThreads),
                       sizeof(uint32_t) * (size_t)G.nbins_total, st, G, w, sh);
    return hipGetLastError();
}

template <int SHADE, bool LIGHT>
hipError_t launch_composite(const Geom &G, const Ws &w, const Shade &sh, hipStream_t st) {
    const dim3 grid((unsigned)G.nbins_total);
    switch (G.B) {
    case 16: hipLaunchKernelGGL((k_fb_composite<16, 256, SHADE, LIGHT>), grid, dim3(256), 0, st, G, w, sh); break;
    case 32: hipLaunchKernelGGL((k_fb_composite<32, 256, SHADE, LIGHT>), grid, dim3(256), 0, st, G, w, sh); break;
    case 64: hipLaunchKernelGGL((k_fb_composite<64, 1024, SHADE, LIGHT>), grid, dim3(1024), 0, st, G, w, sh); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fb_count(const Geom &G, const Ws &w, hipStream_t st) {
    if (G.items == 0) return hipSuccess;
    return launch_pass<true, PK_SHADE_GOURAUD>(G, w, Shade{}, st);
}

hipError_t launch_fb_assign(const Geom &G, const Ws &w, int64_t *pairs_needed, hipStream_t st) {
    return launch_scan(G, w, pairs_needed, st);
}

hipError_t launch_fb_raster(const Geom &G, const Ws &w, const Shade &sh, bool light,
                            hipStream_t st) {
    hipError_t e = hipSuccess;
    if (G.items > 0) {
        switch (sh.shading) {
        case PK_SHADE_GOURAUD:  e = launch_pass<false, PK_SHADE_GOURAUD>(G, w, sh, st); break;
        case PK_SHADE_TEXTURED: e = launch_pass<false, PK_SHADE_TEXTURED>(G, w, sh, st); break;
        case PK_SHADE_DEFERRED: e = launch_pass<false, PK_SHADE_DEFERRED>(G, w, sh, st); break;
        case PK_SHADE_LIT:      e = launch_pass<false, PK_SHADE_LIT>(G, w, sh, st); break;
        default:                e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    switch (sh.shading) {
    case PK_SHADE_GOURAUD:  e = launch_composite<PK_SHADE_GOURAUD, false>(G, w, sh, st); break;
    case PK_SHADE_TEXTURED: e = launch_composite<PK_SHADE_TEXTURED, false>(G, w, sh, st); break;
    case PK_SHADE_LIT:      e = launch_composite<PK_SHADE_LIT, false>(G, w, sh, st); break;
    case PK_SHADE_DEFERRED:
        e = light ? launch_composite<PK_SHADE_DEFERRED, true>(G, w, sh, st)
                  : launch_composite<PK_SHADE_DEFERRED, false>(G, w, sh, st);
        break;
    default: e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (sh.frag_count) e = launch_epilogue(w, sh.frag_count, 0, st);
    return e;
}

}  // namespace pk
