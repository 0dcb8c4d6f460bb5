// k_raster.hip -- Schedule + Process of the screen-space stage (Piko Sec. 4.4
// sort-middle renderer): for every bin, coverage, depth test, resolve and
// shading in one kernel.  The paper's Rasterizer, Fragment Shader, Depth
// Test and Composite stages share bin size and bin mapping, so they fuse
// (Sec. 5.2.1); the depth buffer of a bin stays on chip (the on-chip depth
// buffer of Sec. 5.2.4), here as 64-bit (depth, primitive) keys in LDS
// updated with ds_min_u64, which makes the test order-independent.
//
// Work inside a bin: each wave takes its own chunks of 64 triangles of the
// bin list (no workgroup barrier until EndBin).  When every box of a chunk,
// clipped to the bin, holds at most 12 pixels, each lane walks its own
// triangle's candidates with incrementally stepped edge functions; otherwise
// the wave covers the boxes with 2x2 pixel quads laid end to end and hands
// them out 64 at a time, finding each quad's triangle from start marks in
// LDS, so large and small triangles share the lanes evenly.
//
// Schedules (Sec. 4.3 directives; Sec. 6 work-group organization):
//   LOAD_BALANCE  one workgroup per bin (the hardware dispatcher balances)
//   DIRECT_MAP    G persistent workgroups, bins pre-assigned in contiguous
//                 ranges per die (pre-scheduling, Sec. 5.2.2), with the
//                 records and pair numbers of the next chunks prefetched
//   DYNAMIC       G persistent workgroups pop batches of bins from per-die
//                 device counters
// Whole-screen bins (bin size 0) skip the bin lists: k_direct rasterizes
// every triangle on its own with a device-scope depth test, and k_resolve
// reads the keys from the workspace.
#include "pk_internal.h"

#pragma clang fp contract(off)

namespace pk {

// Three consecutive floats with 4-byte alignment: one dwordx3 access.
struct Float3 {
    float x, y, z;
};

struct RasterArgs {
    Geom G;
    Ws w;
    Shade sh;
    int32_t schedule;
    // Two bin levels: this launch's bins are one level of each scene's CSR
    // block (csr_stride bins per scene, this level's first at csr_base;
    // csr_stride 0: the launch's bins are the CSR bins).  init_keys: the key
    // tile starts from the workspace keys (the finer level's result)
    // instead of empty.
    int32_t csr_stride, csr_base, init_keys;
};

// CSR number of bin b of the launch's bin grid.
__device__ inline int64_t csr_bin(const RasterArgs &a, int64_t b) {
    if (a.csr_stride == 0) return b;
    const uint32_t s = (uint32_t)b / (uint32_t)a.G.nbins_scene;
    return (int64_t)s * a.csr_stride + a.csr_base + (b - (int64_t)s * a.G.nbins_scene);
}

// Resolve of one pixel in three phases so that the loads of several pixels
// can be in flight together: (1) unpack the winning key and load the
// winner's setup record and vertex numbers, (2) load the vertex attributes
// the shading needs, (3) recompute the barycentrics at the pixel centre,
// shade, and write every requested target.
struct Resolve {
    uint32_t t;         // winner (scene-local), or ~0u for an empty pixel
    float depth;
    uint4 xy;           // X0 Y0 X1 Y1 of the winner's setup record
    uint2 xy2;          // X2 Y2
    float iw[3];
    double sinv;
    int32_t v[3];       // vertex numbers
    float c[3][3];      // vertex colours [vertex][channel]
    float ex[3][3];     // uv (2 channels) or normal (3 channels) [vertex][channel]
};

template <int SHADE>
__device__ inline void resolve_fetch(const RasterArgs &a, int32_t s, int64_t item_base,
                                     int64_t vbase_scene, int px, int py,
                                     unsigned long long key, Resolve &r) {
    const Geom &G = a.G;
    r.t = key == kEmptyKey ? ~0u : (uint32_t)(key & 0xffffffffu);
    r.depth = __uint_as_float((uint32_t)(key >> 32));
    if (r.t == ~0u) return;
    if (G.idx) {
        // indexed: the snapped vertices come with the attributes (next
        // phase), from the per-vertex records shared by neighbouring
        // triangles, instead of from the 64-byte setup record
        const int64_t g = G.instanced ? (int64_t)r.t : item_base + r.t;
#pragma unroll
        for (int k = 0; k < 3; ++k) r.v[k] = (int32_t)(vbase_scene + (int64_t)G.idx[3 * g + k]);
        return;
    }
    const int64_t item = item_base + r.t;
    uint32_t q[5];
    if (G.B == 0) {
        // whole-screen bins: the five-word record of the depth-test kernel
        const uint32_t *src = xy20_of(a.w, item);
#pragma unroll
        for (int k = 0; k < 5; ++k) q[k] = src[k];
    } else {
        const uint4 q0 = reinterpret_cast<const uint4 *>(a.w.rec + item)[0];
        q[0] = q0.x; q[1] = q0.y; q[2] = q0.z; q[3] = q0.w;
        q[4] = a.w.rec[item].xy[4];
    }
    int32_t X[3], Y[3];
    unpack_xy(q[0], q[1], q[2], q[3], q[4], X, Y);
    r.xy = make_uint4((uint32_t)X[0], (uint32_t)Y[0], (uint32_t)X[1], (uint32_t)Y[1]);
    r.xy2 = make_uint2((uint32_t)X[2], (uint32_t)Y[2]);
    if (G.mvp) {
        const float4 iw = a.w.iw[item];
        r.iw[0] = iw.x; r.iw[1] = iw.y; r.iw[2] = iw.z;
    } else {
        r.iw[0] = r.iw[1] = r.iw[2] = 1.0f;   // w = 1 exactly without a matrix
    }
    r.sinv = signed_inv_area(area2(X, Y));
#pragma unroll
    for (int k = 0; k < 3; ++k) r.v[k] = (int32_t)(vbase_scene + 3 * (int64_t)r.t + k);
}

template <int SHADE>
__device__ inline void resolve_attribs(const RasterArgs &a, int32_t s, Resolve &r) {
    if (r.t == ~0u) return;
    const Shade &sh = a.sh;
    const int64_t V = a.G.V;
    if (a.G.idx) {
        const int64_t vb = a.G.instanced ? (int64_t)s * V : 0;
        // the three vertex records and every attribute gather are issued
        // before any of them is used
        int4 q[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) q[k] = reinterpret_cast<const int4 *>(a.w.vtx)[vb + r.v[k]];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) r.c[k][ch] = sh.color[ch * V + r.v[k]];
            if (SHADE == PK_SHADE_TEXTURED) {
                r.ex[k][0] = sh.uv[r.v[k]];
                r.ex[k][1] = sh.uv[V + r.v[k]];
            }
            if (SHADE == PK_SHADE_DEFERRED || SHADE == PK_SHADE_LIT) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) r.ex[k][ch] = sh.normal[ch * V + r.v[k]];
            }
        }
        // (z is not needed here; keeping it nominally live makes each record
        // one 16-byte gather instead of an 8-byte and a 4-byte one)
#pragma unroll
        for (int k = 0; k < 3; ++k) __asm__ volatile("" : : "v"(q[k].z));
        r.xy = make_uint4((uint32_t)q[0].x, (uint32_t)q[0].y, (uint32_t)q[1].x, (uint32_t)q[1].y);
        r.xy2 = make_uint2((uint32_t)q[2].x, (uint32_t)q[2].y);
#pragma unroll
        for (int k = 0; k < 3; ++k) r.iw[k] = __int_as_float(q[k].w);
        // 1 / |2 area| with the sign of the winding, computed exactly as setup does
        const int32_t X[3] = {q[0].x, q[1].x, q[2].x}, Y[3] = {q[0].y, q[1].y, q[2].y};
        r.sinv = signed_inv_area(area2(X, Y));
        return;
    }
    // unindexed: the three vertices are consecutive in every plane, one
    // 12-byte load per plane instead of three
    const int64_t v0 = r.v[0];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const Float3 c = *reinterpret_cast<const Float3 *>(sh.color + ch * V + v0);
        r.c[0][ch] = c.x; r.c[1][ch] = c.y; r.c[2][ch] = c.z;
    }
    if (SHADE == PK_SHADE_TEXTURED) {
#pragma unroll
        for (int ch = 0; ch < 2; ++ch) {
            const Float3 u = *reinterpret_cast<const Float3 *>(sh.uv + ch * V + v0);
            r.ex[0][ch] = u.x; r.ex[1][ch] = u.y; r.ex[2][ch] = u.z;
        }
    }
    if (SHADE == PK_SHADE_DEFERRED || SHADE == PK_SHADE_LIT) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const Float3 n = *reinterpret_cast<const Float3 *>(sh.normal + ch * V + v0);
            r.ex[0][ch] = n.x; r.ex[1][ch] = n.y; r.ex[2][ch] = n.z;
        }
    }
}

template <int SHADE>
__device__ inline void resolve_finish(const RasterArgs &a, int32_t s, int px, int py,
                                      const Resolve &r, bool write_dp = true) {
    const Shade &sh = a.sh;
    const int64_t p = ((int64_t)s * a.G.H + py) * a.G.W + px;
    if (r.t == ~0u) {
        if (sh.out_color) reinterpret_cast<float4 *>(sh.out_color)[p] = make_float4(0, 0, 0, 0);
        if (write_dp && sh.out_depth) sh.out_depth[p] = 1.0f;
        if (write_dp && sh.out_primid) sh.out_primid[p] = -1;
        if (sh.out_bary) reinterpret_cast<float2 *>(sh.out_bary)[p] = make_float2(0, 0);
        if (SHADE == PK_SHADE_DEFERRED) {
            *reinterpret_cast<Float3 *>(sh.gbuf_n + 3 * p) = Float3{0.0f, 0.0f, 0.0f};
            *reinterpret_cast<Float3 *>(sh.gbuf_a + 3 * p) = Float3{0.0f, 0.0f, 0.0f};
        }
        return;
    }
    const int32_t X0 = (int32_t)r.xy.x, Y0 = (int32_t)r.xy.y, X1 = (int32_t)r.xy.z,
                  Y1 = (int32_t)r.xy.w;
    const int32_t X2 = (int32_t)r.xy2.x, Y2 = (int32_t)r.xy2.y;
    const float iw0 = r.iw[0], iw1 = r.iw[1], iw2 = r.iw[2];
    const double sinv = r.sinv;
    const int64_t Px = 256 * (int64_t)px + 128, Py = 256 * (int64_t)py + 128;
    const int64_t E0 = (int64_t)(X2 - X1) * (Py - Y1) - (int64_t)(Y2 - Y1) * (Px - X1);
    const int64_t E1 = (int64_t)(X0 - X2) * (Py - Y2) - (int64_t)(Y0 - Y2) * (Px - X2);
    const int64_t E2 = (int64_t)(X1 - X0) * (Py - Y0) - (int64_t)(Y1 - Y0) * (Px - X0);
    const float bs0 = (float)((double)E0 * sinv);
    const float bs1 = (float)((double)E1 * sinv);
    const float bs2 = (float)((double)E2 * sinv);
    FragOut o;
    shade_fragment<SHADE>(sh, bs0, bs1, bs2, iw0, iw1, iw2, r.c, r.ex, o);
    const float b1 = o.b1, b2 = o.b2;
    if (SHADE == PK_SHADE_DEFERRED) {
        *reinterpret_cast<Float3 *>(sh.gbuf_n + 3 * p) = Float3{o.n[0], o.n[1], o.n[2]};
        *reinterpret_cast<Float3 *>(sh.gbuf_a + 3 * p) = Float3{o.rgb[0], o.rgb[1], o.rgb[2]};
    } else if (sh.out_color) {
        reinterpret_cast<float4 *>(sh.out_color)[p] = make_float4(o.rgb[0], o.rgb[1], o.rgb[2], 1.0f);
    }
    if (write_dp && sh.out_depth) sh.out_depth[p] = r.depth;
    if (write_dp && sh.out_primid) sh.out_primid[p] = (int32_t)r.t;
    if (sh.out_bary) reinterpret_cast<float2 *>(sh.out_bary)[p] = make_float2(b1, b2);
}

struct RawTri {
    uint4 q0, q1;   // the 32-byte setup record
};

__device__ inline void fetch_tri(const Ws &w, int32_t item, RawTri &r) {
    const uint4 *rp = reinterpret_cast<const uint4 *>(w.rec + item);
    r.q0 = rp[0];
    r.q1 = rp[1];
}

// The software pipeline below prefetches into loop-carried registers.  A
// prefetch load under a lane condition makes those registers a merge of the
// loaded and the old value, and the compiler then waits for the load right
// after issuing it in order to copy it.  So every lane issues the load: lanes
// without an entry read a dummy address inside the workspace (the misc words,
// 2304 bytes, 256-byte aligned) and discard the value.
__device__ inline void prefetch_tri(const Ws &w, int32_t item, RawTri &r) {
    const uint4 *rp = item >= 0 ? reinterpret_cast<const uint4 *>(w.rec + item)
                                : reinterpret_cast<const uint4 *>(w.misc);
    r.q0 = rp[0];
    r.q1 = rp[1];
}

// The raw value: the caller applies `valid` when it uses it (a select right
// after the load would wait for it).
__device__ inline int32_t prefetch_pair(const Ws &w, bool valid, int32_t j) {
    return *(valid ? w.pairs + j : reinterpret_cast<const int32_t *>(w.misc));
}

// The CSR offsets are read-only in the bin kernel and the bin is uniform
// across the wave: read them through the constant address space so that
// they are scalar loads, whose waits do not hold up the vector prefetches.
typedef const __attribute__((address_space(4))) int32_t ConstI32;
__device__ inline void bin_range(const Ws &w, int64_t b, int32_t &beg, int32_t &end) {
    const ConstI32 *off = (const ConstI32 *)w.bin_off;
    beg = off[b];
    end = off[b + 1];
}

__device__ inline void decode_tri(const RawTri &r, int32_t item, int64_t item_base, int32_t px0,
                                  int32_t py0, int32_t pw, int32_t ph, int32_t W, int32_t H,
                                  EdgeTri &t) {
    int32_t X[3], Y[3];
    unpack_xy(r.q0.x, r.q0.y, r.q0.z, r.q0.w, r.q1.x, X, Y);
    edge_setup(X, Y, __uint_as_float(r.q1.y), __uint_as_float(r.q1.z), __uint_as_float(r.q1.w),
               (int32_t)(item - item_base), px0, py0, pw, ph, W, H, t);
}

// SHADE value of a bin kernel that ends by storing its tile of winning keys
// for the per-pixel resolve kernel instead of resolving in place
constexpr int kKeysOnly = -1;

// Per-triangle staging record of the expansion mode, in 32-bit words, read
// with 128-bit LDS loads: [0..3] first quad, width | height << 8 | own << 16 |
// quads per row << 19, divide magic, origin x | y << 16; [4..9] 256 A_k as float64 (the edge step per
// pixel in x); [10..15] 256 B_k (in y); [16..21] the edge values e_k at the
// origin pixel centre (float64, own bias included); [22..23] 1/|A2|;
// [24..26] z_k; [27] primitive.  With a stride of 28 words the 128-bit
// reads of up to eight consecutive triangles' records touch disjoint LDS
// banks, and a one-wave workgroup with 16x16 bins fits 16 per CU.
constexpr int kStRec = 28;
// Start marks of the expansion mode carry a block tag in their upper bits so
// that the plane never needs clearing; kNoTag is never a live tag.
constexpr uint32_t kTagShift = 6, kNoTag = 0xffffffffu >> kTagShift;

// PIPED: the DIRECT_MAP schedule with its prefetching chunk stream (its own
// instantiation keeps the loop simple enough for the prefetches to land in
// their loop-carried registers); otherwise LOAD_BALANCE or DYNAMIC.
// OIT: transparency layers by depth peeling (one pass per layer).  KBUF:
// transparency layers in one pass, each pixel keeping its K smallest keys in
// LDS by an atomic-min cascade (a key that displaces a larger one carries that
// one on to the next slot): the value left in slot j is the minimum of all
// keys that reached it, i.e. the (j+1)-th smallest, whatever the order.
// Slot 0 is the opaque test's key tile; slots 1..K-1 live in the dynamic LDS
// ((K-1) * B*B * 8 bytes, sized at launch).
template <int TPB, int B, int SHADE, bool PIPED, bool OIT = false, bool KBUF = false>
__global__ __launch_bounds__(TPB)
__attribute__((amdgpu_waves_per_eu(SHADE == kKeysOnly ? 4 : 1))) void k_raster(RasterArgs a) {
    constexpr int NPIX = B * B;
    constexpr int NW = TPB / kWave;
    constexpr int kLoopMax = 12;   // wave-max candidates for the per-lane loop
    __shared__ unsigned long long s_key[NPIX];
    // transparency layers: the previous pass's nearest keys (depth peeling)
    __shared__ unsigned long long s_prev[OIT ? NPIX : 1];
    extern __shared__ unsigned long long s_kbuf[];
    // per-wave staging for the expansion mode (large triangles): one record
    // per lane's triangle, and a plane of start marks
    __shared__ __align__(16) uint32_t s_rec[NW][kWave * kStRec];
    __shared__ uint32_t s_mark[NW][kWave];
    __shared__ int64_t s_bin, s_bin_end;
    __shared__ unsigned long long s_frag[NW];

    const Geom &G = a.G;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wv = tid / kWave;
    uint32_t frags = 0;   // covered samples seen by this thread
    const bool overflow = a.w.misc[1] != 0;   // pair capacity exceeded: no lists
    // expansion-mode start marks: no live tag yet
    uint32_t tag = 0;
    s_mark[wv][lane] = 0xffffffffu;
    // Bins are split into kXcd contiguous ranges; workgroup w works in range
    // w mod kXcd (workgroups are dealt to the dies round-robin), so each die's
    // L2 sees a compact screen region.  The mapping is a bijection whatever
    // the real placement is; only locality depends on it.
    const int64_t nb = G.nbins_total;
    const int64_t q = nb / kXcd, rem = nb % kXcd;
    const int xcd = blockIdx.x % kXcd;
    const int64_t r_beg = xcd * q + min<int64_t>(xcd, rem);
    const int64_t r_len = q + (xcd < rem ? 1 : 0);
    const int64_t lane_in_xcd = blockIdx.x / kXcd;
    const int64_t groups_in_xcd = (gridDim.x - xcd + kXcd - 1) / kXcd;
    // DIRECT_MAP: the bin of iteration i is known in advance (-1: none)
    auto dm_bin = [&](int64_t i) -> int64_t {
        if (gridDim.x < kXcd) {            // too few groups to give every die a range
            const int64_t b = blockIdx.x + i * (int64_t)gridDim.x;
            return b < nb ? b : -1;
        }
        const int64_t l = lane_in_xcd + i * groups_in_xcd;
        return l < r_len ? r_beg + l : -1;
    };
    // Software pipeline (DIRECT_MAP).  A wave's work is a stream of chunks
    // (64 consecutive entries of a bin list) in bin order, known in advance.
    // While chunk n is tested, the setup records of chunk n+1 and the pair
    // numbers of chunk n+2 are in flight, and the CSR offsets of the bin
    // after chunk n+2's bin are loaded, so no chunk waits for memory unless a
    // bin without chunks for this wave is skipped.
    constexpr bool piped = PIPED;
    const int32_t wbase = __builtin_amdgcn_readfirstlane(wv) * kWave;
    int64_t n_it = -1;                 // chunk n+1: iteration (bin) of the stream, -1 = none
    int32_t id_n = -1;                 //   this lane's pair number (-1 = past the list end)
    RawTri raw_n;                      //   its setup record (in flight)
    int64_t nn_it = -1;                // chunk n+2: iteration, first entry, list end
    int32_t nn_c0 = 0, nn_end = 0;
    int32_t id_nn = -1;                //   this lane's pair number (in flight; valid iff ok_nn)
    bool ok_nn = false;
    int64_t pre_it = -1;               // offsets of bin dm_bin(pre_it) (pre_it = nn_it + 1)
    int32_t pre_beg = 0, pre_end = 0;
    auto load_offsets = [&](int64_t it, int64_t &o_it, int32_t &o_beg, int32_t &o_end) {
        const int64_t b = dm_bin(it);
        o_it = b >= 0 ? it : -1;
        o_beg = 0;
        o_end = 0;
        if (b >= 0 && !overflow) bin_range(a.w, csr_bin(a, b), o_beg, o_end);
    };
    // move chunk n+2 one chunk on, and start loading its pair numbers
    auto advance_nn = [&]() {
        if (nn_it >= 0) {
            nn_c0 += TPB;
            while (nn_c0 >= nn_end) {
                if (pre_it < 0) { nn_it = -1; break; }
                nn_it = pre_it;
                nn_c0 = pre_beg + wbase;
                nn_end = pre_end;
                load_offsets(nn_it + 1, pre_it, pre_beg, pre_end);
            }
        }
        const int32_t j = nn_c0 + lane;
        ok_nn = nn_it >= 0 && j < nn_end;
        id_nn = prefetch_pair(a.w, ok_nn, j);
    };
    if (piped) {
        // prologue: chunk 0 becomes "n+1", chunk 1 "n+2"
        load_offsets(0, pre_it, pre_beg, pre_end);
        nn_it = 0;                       // just before the stream's first chunk
        nn_c0 = -TPB;
        nn_end = -TPB;
        advance_nn();
        n_it = nn_it;
        id_n = ok_nn ? id_nn : -1;
        prefetch_tri(a.w, id_n, raw_n);
        advance_nn();
    }
    // PK_SCHED_SPLIT: work-item numbers of the bins (read-only here: scalar
    // loads) and their count
    const ConstI32 *voff = (const ConstI32 *)a.w.vbin_off;
    const int64_t nwork = (!piped && a.w.split && !overflow) ? (int64_t)voff[nb] : 0;
    int32_t piece = 0;
    // DYNAMIC: current queue (range) and the bins of the last batch taken
    int64_t batch_beg = 0, batch_end = 0;
    for (int64_t it = 0;; ++it) {
        int64_t bin;
        if (!piped && a.schedule == PK_SCHED_DYNAMIC) {
            // Each die's bins, heaviest first (the order the scan built):
            // the first min(groups, bins) of a die's order go one to each of
            // its workgroups without any atomic.  The rest (the tail) are
            // dealt round-robin to kSubQueues queues per die and popped one
            // at a time: a workgroup starts at queue (its number mod
            // kSubQueues) of its die, then tries the die's other queues,
            // then the other dies'.
            if (it == 0) {
                const int64_t nstat = min<int64_t>(groups_in_xcd, r_len);
                if (lane_in_xcd < nstat) {
                    batch_beg = r_beg + lane_in_xcd;
                    batch_end = batch_beg + 1;
                }
            }
            if (batch_beg >= batch_end) {
                if (tid < kWave) {
                    // the first wave looks at the heads at once, lane l at
                    // this workgroup's l-th choice, and pops the first
                    // non-empty one; a queue found drained by a pop is never
                    // chosen again, so this ends
                    int64_t b0 = 0, b1 = 0;
                    const int s0 = (int)(lane_in_xcd % kSubQueues);
                    const int qd = (xcd + lane / kSubQueues) % kXcd;
                    const int qsub = (s0 + lane) % kSubQueues;
                    const int64_t qb = qd * q + min<int64_t>(qd, rem);
                    const int64_t ql = q + (qd < rem ? 1 : 0);
                    const int64_t qg = ((int64_t)gridDim.x - qd + kXcd - 1) / kXcd;
                    const int64_t tail = ql - min<int64_t>(qg, ql);   // after the static part
                    uint32_t *head = &a.w.misc[kQueueBase + kQueueStride * (qd * kSubQueues + qsub)];
                    // first the die's own queues (lanes 0..kSubQueues-1), and
                    // only when they are drained all of them
                    int nq = kSubQueues;
#pragma unroll 1
                    for (int tries = 0; tries < kSubQueues + kXcd * kSubQueues; ++tries) {
                        uint32_t seen = 0xffffffffu;
                        if (lane < nq)
                            seen = __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const uint64_t avail = __ballot(lane < nq &&
                                                        qsub + (int64_t)kSubQueues * seen < tail);
                        if (!avail) {
                            if (nq == kWave) break;
                            nq = kWave;
                            continue;
                        }
                        const int f = __ffsll((unsigned long long)avail) - 1;
                        int64_t got = -1;
                        if (lane == f) {
                            const int64_t i = qsub + (int64_t)kSubQueues * (int64_t)atomicAdd(head, 1u);
                            if (i < tail) got = qb + (ql - tail) + i;
                        }
                        got = __shfl(got, f, kWave);
                        if (got >= 0) { b0 = got; b1 = got + 1; break; }
                    }
                    if (tid == 0) {
                        s_bin = b0;
                        s_bin_end = b1;
                    }
                }
                __syncthreads();
                batch_beg = __builtin_amdgcn_readfirstlane((int)s_bin);
                batch_end = __builtin_amdgcn_readfirstlane((int)s_bin_end);
                __syncthreads();
                if (batch_beg >= batch_end) break;
            }
            // a position in the order; the bin itself is the order's entry
            bin = a.w.order[batch_beg++];
        } else if (piped) {
            bin = dm_bin(it);
            if (bin < 0) break;
        } else if (a.w.split) {
            // PK_SCHED_SPLIT: work item v is piece `piece` of the last bin
            // whose first work item is at or before v (bins without pairs
            // have none and share the next bin's first number)
            if (overflow) break;
            const int64_t v = blockIdx.x + it * (int64_t)gridDim.x;
            if (v >= nwork) break;
            // each wave searches with 64 probes per step (every wave finds the
            // same bin): the answer stays in [lo, hi] and voff[lo] <= v
            int64_t lo = 0, hi = nb - 1;
            while (lo < hi) {
                const int64_t step = (hi - lo + kWave) / kWave;
                const int64_t probe = lo + (int64_t)lane * step;
                const uint64_t m = __ballot(probe <= hi && (int64_t)a.w.vbin_off[probe] <= v);
                lo += (int64_t)(63 - __clzll((long long)m)) * step;
                hi = min(hi, lo + step - 1);
            }
            bin = lo;
            piece = (int32_t)(v - voff[lo]);
        } else {
            if (it > 0 || lane_in_xcd >= r_len) break;
            bin = r_beg + lane_in_xcd;
        }
        // bin numbers are below 2^31: 32-bit divides (the 64-bit routine is
        // a long scalar sequence)
        const uint32_t ub = (uint32_t)bin;
        const int32_t s = G.S == 1 ? 0 : (int32_t)(ub / (uint32_t)G.nbins_scene);
        const int32_t lb = (int32_t)(ub - (uint32_t)s * (uint32_t)G.nbins_scene);
        const int32_t by = (int32_t)((uint32_t)lb / (uint32_t)G.nbx), bx = lb - by * G.nbx;
        const int32_t px0 = bx * B, py0 = by * B;
        const int32_t pw = min(B, G.W - px0), ph = min(B, G.H - py0);
        const int64_t item_base = G.instanced ? (int64_t)s * G.T : (G.S > 1 ? G.tri_off[s] : 0);
        const int64_t vbase = (G.S > 1 && !G.instanced) ? G.vtx_off[s] : 0;

        // One pass per transparency layer (one pass when opaque): pass l keeps,
        // per pixel, the smallest key above pass l-1's, so the passes find the
        // nearest fragments in order.
        const int nlayers = OIT ? a.sh.layers : 1;
#pragma unroll 1
        for (int layer = 0; layer < nlayers; ++layer) {
        auto zmin = [&](uint32_t sl, unsigned long long key) {
            if (KBUF) {
                // slot-major, so that neighbouring pixels use neighbouring
                // banks; the last slot's minimum needs no old value
                unsigned long long *slot = &s_key[sl];
                for (int j = 1;; ++j) {
                    if (j == a.sh.layers) {
                        atomicMin(slot, key);
                        break;
                    }
                    const unsigned long long old = atomicMin(slot, key);
                    if (old == kEmptyKey) break;
                    key = old > key ? old : key;
                    slot = &s_kbuf[(j - 1) * NPIX + sl];
                }
            } else if (!OIT || layer == 0 || key > s_prev[sl]) {
                atomicMin(&s_key[sl], key);
            }
        };
        int32_t lbeg = 0, lend = 0;
        bool shared = false;   // PK_SCHED_SPLIT: the bin has several pieces
        if (!overflow && !piped) {
            const int64_t cb = csr_bin(a, bin);
            lbeg = a.w.bin_off[cb];
            lend = a.w.bin_off[cb + 1];
            if (a.w.split) {
                shared = lend - lbeg > a.w.split;
                lbeg += piece * a.w.split;
                lend = min(lend, lbeg + a.w.split);
            }
        }
        // a coarse bin without triangles leaves the fine level's keys, which
        // are already in the workspace, as they are
        if (a.init_keys && lbeg >= lend) continue;
        if (a.init_keys) {
            // the coarse level starts from the fine level's keys: split into
            // the depth and primitive-ID targets when the caller gave both
            // (the two halves of a key; primitive ID -1 marks an empty
            // pixel), else in the workspace
            const int64_t sb = (int64_t)s * G.W * G.H;
            const bool halves = a.sh.out_depth && a.sh.out_primid;
            for (int i = tid; i < NPIX; i += TPB) {
                const int lx = i % B, ly = i / B;
                unsigned long long k = kEmptyKey;
                if (lx < pw && ly < ph) {
                    const int64_t p = sb + (int64_t)(py0 + ly) * G.W + px0 + lx;
                    if (halves) {
                        const int32_t pid = a.sh.out_primid[p];
                        if (pid != -1)
                            k = ((unsigned long long)__float_as_uint(a.sh.out_depth[p]) << 32) |
                                (uint32_t)pid;
                    } else {
                        k = a.w.keys[p];
                    }
                }
                s_key[i] = k;
            }
        } else {
            for (int i = tid; i < NPIX; i += TPB) s_key[i] = kEmptyKey;
        }
        if (KBUF)
            for (int i = tid; i < (a.sh.layers - 1) * NPIX; i += TPB) s_kbuf[i] = kEmptyKey;
        __syncthreads();

        // Process: every wave takes chunks of 64 triangles of the bin list
        // (without the pipeline, each chunk's pair numbers are loaded while
        // the chunk before it is tested)
        int32_t id_next = 0;
        bool ok_next = false;
        if (!piped) {
            ok_next = lbeg + wbase + lane < lend;
            id_next = prefetch_pair(a.w, ok_next, lbeg + wbase + lane);
        }
#pragma unroll 1
        for (int32_t c0 = lbeg + wbase;; c0 += TPB) {
            RawTri raw;
            int32_t item;
            if (piped) {
                if (n_it != it) break;          // the stream has left this bin
                raw = raw_n;
                item = id_n;
                // chunk n+2 becomes n+1: fetch its records; load the next pair numbers
                n_it = nn_it;
                id_n = ok_nn ? id_nn : -1;
                prefetch_tri(a.w, id_n, raw_n);
                advance_nn();
            } else {
                if (c0 >= lend) break;
                item = ok_next ? id_next : -1;
                if (item >= 0) fetch_tri(a.w, item, raw);
                ok_next = c0 + TPB + lane < lend;
                id_next = prefetch_pair(a.w, ok_next, c0 + TPB + lane);
            }
            EdgeTri t;
            t.cnt = 0;
            if (item >= 0) decode_tri(raw, item, item_base, px0, py0, pw, ph, G.W, G.H, t);
            const int mx = wave_max(t.cnt);
            if (mx <= kLoopMax) {
                // small triangles: each lane walks its own candidates with
                // incrementally stepped edge functions
                double e0 = 0.0, e1 = 0.0, e2 = 0.0;
                // the candidate's key slot in the tile, stepped with the edges
                int col = 0;
                uint32_t slot = (uint32_t)((t.y0 - py0) * B + (t.x0 - px0));
                const uint32_t row_skip = (uint32_t)(B - t.wdt + 1);
                const double Px = (double)(256 * t.x0 + 128), Py = (double)(256 * t.y0 + 128);
                e0 = (double)t.A[0] * Px + (double)t.Bc[0] * Py + t.C[0];
                e1 = (double)t.A[1] * Px + (double)t.Bc[1] * Py + t.C[1];
                e2 = (double)t.A[2] * Px + (double)t.Bc[2] * Py + t.C[2];
                const double sx0 = (double)(256 * t.A[0]), sx1 = (double)(256 * t.A[1]),
                             sx2 = (double)(256 * t.A[2]);
                // to the next row start: +256 B, minus the (width-1) x steps taken
                const double back = (double)(256 * (t.wdt - 1));
                const double sy0 = (double)(256 * t.Bc[0]) - back * (double)t.A[0];
                const double sy1 = (double)(256 * t.Bc[1]) - back * (double)t.A[1];
                const double sy2 = (double)(256 * t.Bc[2]) - back * (double)t.A[2];
#pragma unroll 1
                for (int j = 0; j < mx; ++j) {
                    if (j < t.cnt) {
                        if (e0 > 0.0 && e1 > 0.0 && e2 > 0.0) {
                            frags += (!OIT || layer == 0);
                            unsigned long long key;
                            if (depth_key(e0, e1, e2, t.own, t.inv, t.z[0], t.z[1], t.z[2],
                                          (uint32_t)t.prim, key))
                                zmin(slot, key);
                        }
                        if (++col < t.wdt) {
                            e0 += sx0; e1 += sx1; e2 += sx2;
                            ++slot;
                        } else {
                            col = 0;
                            slot += row_skip;
                            e0 += sy0; e1 += sy1; e2 += sy2;
                        }
                    }
                }
            } else {
                // large triangles: cover each clipped bbox with 2x2 pixel
                // quads, lay the wave's quads end to end and hand them out in
                // blocks of 64, one per lane.  A quad pays the owner lookup,
                // the record reads and the divide once for four pixels.
                const int hgt = t.cnt > 0 ? t.cnt / t.wdt : 0;
                const int qw = (t.wdt + 1) >> 1, qh = (hgt + 1) >> 1;
                const int qcnt = t.cnt > 0 ? qw * qh : 0;
                int total = qcnt;
#pragma unroll
                for (int d = 1; d < kWave; d <<= 1) {
                    const int y = __shfl_up(total, d, kWave);
                    if (lane >= d) total += y;
                }
                const int start = total - qcnt;
                total = __shfl(total, kWave - 1, kWave);
                uint32_t *rec = s_rec[wv];
                uint32_t *mark = s_mark[wv];
                {
                    // stage this lane's triangle
                    uint32_t *r = rec + lane * kStRec;
                    // m = ceil(2^18 / qw) makes (c * m) >> 18 an exact divide
                    // for quad numbers c < 2^12 (c * (m * qw - 2^18) < 2^12 * qw
                    // <= 2^18), all in full-rate 24-bit multiplies
                    const uint32_t q1 = (uint32_t)max(qw, 1);
                    const uint32_t mag = ((1u << 18) + q1 - 1u) / q1;
                    *reinterpret_cast<uint4 *>(r) =
                        make_uint4((uint32_t)start,
                                   (uint32_t)(max(t.wdt, 1) | (hgt << 8) | (t.own << 16) | (q1 << 19)),
                                   mag, (uint32_t)(t.x0 | (t.y0 << 16)));
                    const double Px = (double)(256 * t.x0 + 128), Py = (double)(256 * t.y0 + 128);
                    double st[12];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        st[k] = (double)(256 * t.A[k]);
                        st[3 + k] = (double)(256 * t.Bc[k]);
                        // exact: integers below 2^53
                        st[6 + k] = (double)t.A[k] * Px + (double)t.Bc[k] * Py + t.C[k];
                    }
                    st[9] = t.inv;
                    st[10] = __hiloint2double((int)__float_as_uint(t.z[1]), (int)__float_as_uint(t.z[0]));
                    st[11] = __hiloint2double((int)t.prim, (int)__float_as_uint(t.z[2]));
                    double2 *r2 = reinterpret_cast<double2 *>(r + 4);
#pragma unroll
                    for (int k = 0; k < 6; ++k) r2[k] = make_double2(st[2 * k], st[2 * k + 1]);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                int carry = 0;   // triangle of the last quad of the previous block
                if (tag + (uint32_t)(total / kWave + 1) >= kNoTag) {
                    // (never in practice) recycle the tags before they run out
                    mark[lane] = 0xffffffffu;
                    tag = 0;
                }
#pragma unroll 1
                for (int b = 0; b < total; b += kWave) {
                    // Which triangle owns quad j = b + lane: the last non-empty
                    // triangle starting at or before j.  Each one starting inside
                    // this block marks its start position with its lane; a ballot
                    // of the live marks and a leading-zero count find the nearest
                    // mark at or below j, a lane shuffle fetches it, and a block
                    // position before any mark belongs to the previous block's
                    // last triangle.
                    if (qcnt > 0 && start >= b && start < b + kWave)
                        mark[start - b] = (tag << kTagShift) | (uint32_t)lane;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    const uint32_t mk = mark[lane];
                    const uint64_t live = __ballot((mk >> kTagShift) == tag);
                    const uint64_t upto = live & ((2ull << lane) - 1ull);
                    const int from = upto ? 63 - __clzll(upto) : 0;
                    const int marked = __shfl((int)(mk & (kWave - 1)), from, kWave);
                    const int lo = upto ? marked : carry;
                    carry = __shfl(lo, kWave - 1, kWave);
                    ++tag;
                    const int j = b + lane;
                    if (j >= total) continue;
                    const uint32_t *r = rec + __umul24((uint32_t)lo, (uint32_t)kStRec);
                    const uint4 hd = *reinterpret_cast<const uint4 *>(r);
                    const double2 *r2 = reinterpret_cast<const double2 *>(r + 4);
                    const double2 a01 = r2[0], a2b0 = r2[1], b12 = r2[2];
                    const double2 e01 = r2[3], e2i = r2[4];
                    const uint32_t local = (uint32_t)j - hd.x;
                    const uint32_t wi = hd.y;
                    const uint32_t wdt = wi & 0xff, hh = (wi >> 8) & 0xff, own = (wi >> 16) & 7;
                    const uint32_t qwl = wi >> 19;
                    const uint32_t qr = __umul24(local, hd.z) >> 18;
                    const uint32_t qc = local - __umul24(qr, qwl);
                    const uint32_t col = 2 * qc, row = 2 * qr;
                    const double dc = (double)col, dr = (double)row;
                    // e_k at the quad's first pixel from the origin value and the
                    // steps, then one step right, down, and both: every product
                    // and sum is an integer below 2^53, so all are exact
                    double ea[3], eb[3], ec[3], ed[3];
                    ea[0] = fma(dr, a2b0.y, fma(dc, a01.x, e01.x));
                    ea[1] = fma(dr, b12.x, fma(dc, a01.y, e01.y));
                    ea[2] = fma(dr, b12.y, fma(dc, a2b0.x, e2i.x));
                    const double sxk[3] = {a01.x, a01.y, a2b0.x}, syk[3] = {a2b0.y, b12.x, b12.y};
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        eb[k] = ea[k] + sxk[k];
                        ec[k] = ea[k] + syk[k];
                        ed[k] = eb[k] + syk[k];
                    }
                    const bool right = col + 1 < wdt, down = row + 1 < hh;
                    const bool ca = ea[0] > 0.0 && ea[1] > 0.0 && ea[2] > 0.0;
                    const bool cb = right && eb[0] > 0.0 && eb[1] > 0.0 && eb[2] > 0.0;
                    const bool cc = down && ec[0] > 0.0 && ec[1] > 0.0 && ec[2] > 0.0;
                    const bool cd = right && down && ed[0] > 0.0 && ed[1] > 0.0 && ed[2] > 0.0;
                    if (!(ca || cb || cc || cd)) continue;
                    const double2 zz = r2[5];
                    const float z0 = __uint_as_float((uint32_t)__double2loint(zz.x));
                    const float z1 = __uint_as_float((uint32_t)__double2hiint(zz.x));
                    const float z2 = __uint_as_float((uint32_t)__double2loint(zz.y));
                    const uint32_t prim = (uint32_t)__double2hiint(zz.y);
                    const int32_t org = (int32_t)hd.w;
                    const uint32_t slot = (uint32_t)(((org >> 16) + (int32_t)row - py0) * B +
                                                     (org & 0xffff) + (int32_t)col - px0);
                    unsigned long long key;
                    if (ca) {
                        frags += (!OIT || layer == 0);
                        if (depth_key(ea[0], ea[1], ea[2], own, e2i.y, z0, z1, z2, prim, key))
                            zmin(slot, key);
                    }
                    if (cb) {
                        frags += (!OIT || layer == 0);
                        if (depth_key(eb[0], eb[1], eb[2], own, e2i.y, z0, z1, z2, prim, key))
                            zmin(slot + 1, key);
                    }
                    if (cc) {
                        frags += (!OIT || layer == 0);
                        if (depth_key(ec[0], ec[1], ec[2], own, e2i.y, z0, z1, z2, prim, key))
                            zmin(slot + B, key);
                    }
                    if (cd) {
                        frags += (!OIT || layer == 0);
                        if (depth_key(ed[0], ed[1], ed[2], own, e2i.y, z0, z1, z2, prim, key))
                            zmin(slot + B + 1, key);
                    }
                }
                // the staging slots are rewritten by this wave's next chunk
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        __syncthreads();
        // EndBin: every fragment of this bin has been tested
        if (SHADE == kKeysOnly) {
            // hand the tile's winning keys to the per-pixel resolve kernel:
            // as the final depth and primitive-ID targets when the caller
            // has both (the two halves of the key), else as keys
            const int64_t sb = (int64_t)s * G.W * G.H;
            const bool split = !OIT && !KBUF && !a.w.split && a.sh.out_depth && a.sh.out_primid;
            // layer l's keys follow the whole key buffer of layers 0..l-1
            const int64_t lofs = OIT ? (int64_t)layer * G.S * G.W * G.H : 0;
#pragma unroll 1
            for (int i = tid; i < NPIX; i += TPB) {
                const int lx = i % B, ly = i / B;
                if (lx < pw && ly < ph) {
                    const int64_t p = sb + (int64_t)(py0 + ly) * G.W + px0 + lx;
                    const unsigned long long k = s_key[i];
                    if (split) {
                        a.sh.out_depth[p] = k == kEmptyKey ? 1.0f : __uint_as_float((uint32_t)(k >> 32));
                        a.sh.out_primid[p] = k == kEmptyKey ? -1 : (int32_t)(uint32_t)k;
                    } else if (shared) {
                        // pieces of one bin merge in the cleared key buffer
                        if (k != kEmptyKey) atomicMin(&a.w.keys[p], k);
                    } else if (KBUF) {
                        const int64_t stride = (int64_t)G.S * G.W * G.H;
                        a.w.keys[p] = k;
                        for (int l = 1; l < a.sh.layers; ++l)
                            a.w.keys[p + l * stride] = s_kbuf[(l - 1) * NPIX + i];
                    } else {
                        a.w.keys[p + lofs] = k;
                    }
                }
            }
        } else {
            // resolve in place, two pixels per thread at a time so their
            // gathers overlap
            constexpr int PPT = NPIX / TPB >= 2 ? 2 : 1;
#pragma unroll 1
            for (int i0 = tid; i0 < NPIX; i0 += PPT * TPB) {
                Resolve rs[PPT];
                int lx[PPT], ly[PPT];
                bool on[PPT];
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const int i = i0 + k * TPB;
                    lx[k] = i % B;
                    ly[k] = i / B;
                    on[k] = i < NPIX && lx[k] < pw && ly[k] < ph;
                    if (on[k])
                        resolve_fetch<SHADE>(a, s, item_base, vbase, px0 + lx[k], py0 + ly[k],
                                             s_key[i], rs[k]);
                }
#pragma unroll
                for (int k = 0; k < PPT; ++k)
                    if (on[k]) resolve_attribs<SHADE>(a, s, rs[k]);
#pragma unroll
                for (int k = 0; k < PPT; ++k)
                    if (on[k]) resolve_finish<SHADE>(a, s, px0 + lx[k], py0 + ly[k], rs[k]);
            }
        }
        if (OIT) {
            // each thread copies the pixels it stored; the next pass reads
            // them only after the barrier that follows its key reset
            for (int i = tid; i < NPIX; i += TPB) s_prev[i] = s_key[i];
        }
        }   // layer
        __syncthreads();
    }
    if (a.sh.frag_count) {
        // wave reduction, then one atomic per workgroup on its partial slot
        unsigned long long f = (unsigned long long)frags;
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) f += __shfl_down(f, d, kWave);
        if (lane == 0) s_frag[wv] = f;
        __syncthreads();
        if (tid == 0) {
            unsigned long long tot = 0;
            for (int i = 0; i < NW; ++i) tot += s_frag[i];
            unsigned long long *slots = reinterpret_cast<unsigned long long *>(a.w.misc + 64);
            if (tot) atomicAdd(&slots[blockIdx.x % kFragSlots], tot);
        }
    }
}

// Runs after a bin kernel that used the misc words (one workgroup): adds the
// partial fragment counts to the caller's counter and clears them, and
// rewinds the DYNAMIC queue heads, so the words are zero again for another
// pk_raster_shade on the same workspace (pk_setup also clears them).
__global__ __launch_bounds__(kFragSlots) void k_raster_epilogue(uint32_t *misc,
                                                                unsigned long long *frag_count,
                                                                int rewind) {
    __shared__ unsigned long long s_part[kFragSlots / kWave];
    if (frag_count) {
        unsigned long long *slots = reinterpret_cast<unsigned long long *>(misc + 64);
        unsigned long long v = slots[threadIdx.x];
        slots[threadIdx.x] = 0ull;
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_down(v, d, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0) s_part[threadIdx.x / kWave] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long tot = 0;
            for (int i = 0; i < kFragSlots / kWave; ++i) tot += s_part[i];
            *frag_count += tot;
        }
    }
    if (rewind && threadIdx.x < kXcd * kSubQueues) misc[kQueueBase + kQueueStride * threadIdx.x] = 0u;
}

hipError_t launch_epilogue(const Ws &w, unsigned long long *frag_count, int rewind,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_raster_epilogue, dim3(1), dim3(kFragSlots), 0, st, w.misc, frag_count,
                       rewind);
    return hipGetLastError();
}

// Whole-screen bins (bin size 0, the unbinned pipeline of Sec. 4.4 and the
// paper's full-screen-bin baseline of Sec. 7): no bin lists, one thread per
// triangle over its sample bounding box on the screen, and the depth test as
// a device-scope 64-bit atomic min into the workspace key buffer (cleared to
// all ones beforehand).  The keys are the same (depth, primitive) keys as in
// the bin kernel, so the image is the same.  The candidates of triangles
// whose box holds at most kDirectLoopMax samples are dealt over the wave's
// lanes as (triangle, sample) pairs; larger boxes are swept by the whole
// wave, one triangle at a time, one pixel per lane.  Measured on
// micro8m and on the 1080p grid (k_direct per frame): each lane walking its
// own box of up to 16 samples took 256 and 50 us (lanes idled while the
// wave's largest box was walked: 5.3 times the useful iterations on
// micro8m); dealing pairs up to 16, 32, 64 and 128 samples 271/41, 247/41,
// 244/42 and 246/42 us.  Reading a pixel's key before the atomic min, to
// skip atomics that cannot win, was slower (291 and 48 us).  One-wave
// workgroups measured fastest.
constexpr int kDirectThreads = 64;
constexpr int kDirectLoopMax = 64;

// The small-box triangles of a k_direct wave as its lanes read them from
// LDS: one array per field, so that lanes reading different triangles hit
// neighbouring words.
struct DirTris {
    double C[3][kDirectThreads];
    double inv[kDirectThreads];
    int64_t kbase[kDirectThreads];
    int32_t A[3][kDirectThreads], Bc[3][kDirectThreads];
    float z[3][kDirectThreads];
    int32_t x0[kDirectThreads], y0[kDirectThreads], wdt[kDirectThreads], own[kDirectThreads],
        prim[kDirectThreads];
};

__global__ __launch_bounds__(kDirectThreads) void k_direct(RasterArgs a) {
    const Geom &G = a.G;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t item = blockIdx.x * (int64_t)kDirectThreads + threadIdx.x;
    EdgeTri t;
    t.cnt = 0;
    int64_t kbase = 0;   // first key of the triangle's scene
    // Triangle setup happens here, not in pk_setup: the kernel reads the
    // triangle's vertices (the Vertex Shader's records, or raw positions),
    // snaps and culls it and keeps the result in registers; only an
    // unindexed mesh's packed snapped vertices are stored, for the per-pixel
    // resolve.
    TriIn tin;
    setup_indices(G, item, tin);
    if (G.idx) setup_index_load(G, tin);
    setup_fetch<true>(G, a.w, tin);
    if (item < G.items) {
        int32_t X[3], Y[3];
        float z[3], iw[3];
        if (setup_snap(G, tin, X, Y, z, iw) != kEmptyKey) {
            if (!G.idx) {
                store_xy20(a.w, item, X, Y);
                if (G.mvp) a.w.iw[item] = make_float4(iw[0], iw[1], iw[2], 0.0f);
            }
            const ItemRef r = item_ref(G, item);
            edge_setup(X, Y, z[0], z[1], z[2], (int32_t)r.t, 0, 0, G.W, G.H, G.W, G.H, t);
            kbase = (int64_t)r.s * G.W * G.H;
        }
    }
    uint32_t frags = 0;
    unsigned long long *keys = a.w.keys;
    // Small boxes: the wave's (triangle, candidate) pairs are laid end to end
    // in lane order and dealt 64 at a time, one per lane, so that no lane
    // idles while a neighbour walks a longer box.  Pair j belongs to the
    // last lane whose first pair is at or before j; that lane's triangle is
    // read from LDS.
    const int small = t.cnt <= kDirectLoopMax ? t.cnt : 0;
    int incl = small;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += y;
    }
    const int total = __shfl(incl, kWave - 1, kWave);
    const int start = incl - small;
    if (total > 0) {
        // (one-wave workgroups: the barrier orders the wave's LDS stores
        // before its loads)
        static_assert(kDirectThreads == kWave, "k_direct deals pairs within one wave");
        __shared__ DirTris s_tri;
        if (small > 0) {
            const int i = threadIdx.x;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                s_tri.C[k][i] = t.C[k];
                s_tri.A[k][i] = t.A[k];
                s_tri.Bc[k][i] = t.Bc[k];
                s_tri.z[k][i] = t.z[k];
            }
            s_tri.inv[i] = t.inv;
            s_tri.kbase[i] = kbase;
            s_tri.x0[i] = t.x0;
            s_tri.y0[i] = t.y0;
            s_tri.wdt[i] = t.wdt;
            s_tri.own[i] = t.own;
            s_tri.prim[i] = t.prim;
        }
        __syncthreads();
#pragma unroll 1
        for (int b0 = 0; b0 < total; b0 += kWave) {
            const int j = b0 + lane;
            int o = 0;
#pragma unroll
            for (int step = kWave / 2; step >= 1; step >>= 1) {
                const int c = o + step;
                const int sc = __shfl(start, c, kWave);
                if (sc <= j) o = c;
            }
            const int o_start = __shfl(start, o, kWave);
            if (j < total) {
                const uint32_t local = (uint32_t)(j - o_start);
                const uint32_t wdt = (uint32_t)s_tri.wdt[o];
                const uint32_t row = local / wdt, col = local - row * wdt;
                const int px = s_tri.x0[o] + (int)col, py = s_tri.y0[o] + (int)row;
                const double Px = (double)(256 * px + 128), Py = (double)(256 * py + 128);
                double e[3];
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    e[k] = (double)s_tri.A[k][o] * Px + (double)s_tri.Bc[k][o] * Py + s_tri.C[k][o];
                if (e[0] > 0.0 && e[1] > 0.0 && e[2] > 0.0) {
                    ++frags;
                    unsigned long long key;
                    if (depth_key(e[0], e[1], e[2], s_tri.own[o], s_tri.inv[o], s_tri.z[0][o],
                                  s_tri.z[1][o], s_tri.z[2][o], (uint32_t)s_tri.prim[o], key))
                        atomicMin(keys + s_tri.kbase[o] + (int64_t)py * G.W + px, key);
                }
            }
        }
    }
    // large boxes: the wave sweeps each in turn, one pixel per lane.  Edge
    // values are evaluated directly: every product and sum is an integer
    // below 2^53, so the float64 arithmetic is exact.
    uint64_t big = __ballot(t.cnt > kDirectLoopMax);
    while (big) {
        const int l = __ffsll((unsigned long long)big) - 1;
        big &= big - 1;
        double A[3], Bv[3], C[3];
        float z[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            A[k] = (double)__shfl(t.A[k], l, kWave);
            Bv[k] = (double)__shfl(t.Bc[k], l, kWave);
            C[k] = __shfl(t.C[k], l, kWave);
            z[k] = __shfl(t.z[k], l, kWave);
        }
        const double inv = __shfl(t.inv, l, kWave);
        const int x0 = __shfl(t.x0, l, kWave), y0 = __shfl(t.y0, l, kWave);
        const uint32_t wdt = (uint32_t)__shfl(t.wdt, l, kWave);
        const int cnt = __shfl(t.cnt, l, kWave), own = __shfl(t.own, l, kWave);
        const uint32_t prim = (uint32_t)__shfl(t.prim, l, kWave);
        const int64_t kb = __shfl(kbase, l, kWave);
#pragma unroll 1
        for (int i = lane; i < cnt; i += kWave) {
            const uint32_t row = (uint32_t)i / wdt, col = (uint32_t)i - row * wdt;
            const int px = x0 + (int)col, py = y0 + (int)row;
            const double Px = (double)(256 * px + 128), Py = (double)(256 * py + 128);
            const double e0 = A[0] * Px + Bv[0] * Py + C[0];
            const double e1 = A[1] * Px + Bv[1] * Py + C[1];
            const double e2 = A[2] * Px + Bv[2] * Py + C[2];
            if (e0 > 0.0 && e1 > 0.0 && e2 > 0.0) {
                ++frags;
                unsigned long long key;
                if (depth_key(e0, e1, e2, own, inv, z[0], z[1], z[2], prim, key))
                    atomicMin(keys + kb + (int64_t)py * G.W + px, key);
            }
        }
    }
    if (a.sh.frag_count) {
        // wave reduction, then one atomic per workgroup on its partial slot
        __shared__ unsigned long long s_frag[kDirectThreads / kWave];
        unsigned long long f = (unsigned long long)frags;
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) f += __shfl_down(f, d, kWave);
        if (lane == 0) s_frag[threadIdx.x / kWave] = f;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long tot = 0;
            for (int i = 0; i < kDirectThreads / kWave; ++i) tot += s_frag[i];
            unsigned long long *slots = reinterpret_cast<unsigned long long *>(a.w.misc + 64);
            if (tot) atomicAdd(&slots[blockIdx.x % kFragSlots], tot);
        }
    }
}

hipError_t launch_direct(const Geom &G, const Ws &w, const Shade &sh, RasterMode mode,
                         hipStream_t st) {
    const int64_t npix = (int64_t)G.S * G.W * G.H;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(w.keys), 2 * npix, 0xffffffffu, st);
    if (e != hipSuccess) return e;
    RasterArgs a{G, w, sh, 0};
    if (G.items > 0) {
        const int64_t blocks = (G.items + kDirectThreads - 1) / kDirectThreads;
        hipLaunchKernelGGL(k_direct, dim3((unsigned)blocks), dim3(kDirectThreads), 0, st, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (sh.frag_count) {
        hipLaunchKernelGGL(k_raster_epilogue, dim3(1), dim3(kFragSlots), 0, st, w.misc,
                           sh.frag_count, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // no EndBin inside a bin here: the per-pixel pass follows unless deferred
    if (mode != kRasterKeysOnly) return launch_resolve_pass(G, w, sh, st);
    return hipSuccess;
}

// Resolve of every pixel of every scene from the key buffer: one thread per
// pixel, TW x TH pixel tiles per workgroup (64 x 4 on wide screens, 16 x 16
// on screens at most 512 pixels wide: measured on batch256's 256 x 256
// scenes 264 against 309 us, on the 1080p grid 24.1 against 23.9 us; the
// order-independent transparency resolve keeps 64 x 4).  Tiles are numbered row-major
// (scene by scene) and split into kXcd contiguous ranges like the bins, and
// workgroup w takes a tile from range w mod kXcd, so a die resolves the same
// screen band whose triangles its bin kernel just read into its L2.
constexpr int kResW = 64, kResH = 4;
// Pixels per thread: each thread resolves kResPPT pixels of one column
// (kResH rows apart) phase by phase, so that the dependent gathers of all of
// them are in flight together.  One is fastest on the grid and batched
// workloads (measured 25.2 / 27.8 / 33.0 us at 1 / 2 / 4 on the 1080p grid):
// the gathers are bound by address processing, not by latency.
constexpr int kResPPT = 1;
constexpr int kResRows = kResH * kResPPT;   // rows of a tile

template <int SHADE, int TW, int TH>
__global__ __launch_bounds__(TW * TH) void k_resolve(RasterArgs a) {
    constexpr int TR = TH * kResPPT;   // rows of a tile
    const Geom &G = a.G;
    const int ntx = (G.W + TW - 1) / TW, nty = (G.H + TR - 1) / TR;
    const int64_t per_scene = (int64_t)ntx * nty;
    const int64_t ntiles = per_scene * G.S;
    const int64_t q = ntiles / kXcd, rem = ntiles % kXcd;
    const int xcd = blockIdx.x % kXcd;
    // one workgroup per tile, so tile numbers fit the 32-bit grid size
    const uint32_t tile = (uint32_t)(xcd * q + min<int64_t>(xcd, rem) + blockIdx.x / kXcd);
    const int32_t s = G.S == 1 ? 0 : (int32_t)(tile / (uint32_t)per_scene);
    const uint32_t ts = tile - (uint32_t)s * (uint32_t)per_scene;
    const int ty = (int)(ts / (uint32_t)ntx), tx = (int)(ts - (uint32_t)ty * (uint32_t)ntx);
    const int px = tx * TW + (int)(threadIdx.x % TW);
    const int py0 = ty * TR + (int)(threadIdx.x / TW);
    if (px >= G.W || py0 >= G.H) return;
    const int64_t item_base = G.instanced ? (int64_t)s * G.T : (G.S > 1 ? G.tri_off[s] : 0);
    const int64_t vbase = (G.S > 1 && !G.instanced) ? G.vtx_off[s] : 0;
    // keys in the workspace: whole-screen bins and split bins always, other
    // bins when a depth or primitive-ID target is missing
    const bool split = G.B != 0 && !a.w.split && a.sh.out_depth && a.sh.out_primid;
    Resolve r[kResPPT];
    bool on[kResPPT];
#pragma unroll
    for (int k = 0; k < kResPPT; ++k) {
        const int py = py0 + k * TH;
        on[k] = py < G.H;
        if (!on[k]) continue;
        const int64_t p = ((int64_t)s * G.H + py) * G.W + px;
        unsigned long long key;
        if (split) {
            // the bin kernel already wrote the depth and primitive-ID targets;
            // shading needs the winner only (the depth half stays unused)
            const int32_t prim = a.sh.out_primid[p];
            key = prim < 0 ? kEmptyKey : (unsigned long long)(uint32_t)prim;
        } else {
            key = a.w.keys[p];
        }
        resolve_fetch<SHADE>(a, s, item_base, vbase, px, py, key, r[k]);
    }
#pragma unroll
    for (int k = 0; k < kResPPT; ++k)
        if (on[k]) resolve_attribs<SHADE>(a, s, r[k]);
#pragma unroll
    for (int k = 0; k < kResPPT; ++k)
        if (on[k]) resolve_finish<SHADE>(a, s, px, py0 + k * TH, r[k], !split);
}

// Order-independent transparency, per pixel: the layers' keys (nearest
// first, as the bin kernel left them) are
// resolved one after another and composited with the interpolated per-vertex
// opacity a:  T = 1, C = 0;  w = T*a, C += w*c, T = T*(1 - a);  colour =
// (C, 1 - T).  Depth, primitive ID and barycentrics are the nearest layer's.
// Gouraud colours; same tiles as k_resolve.
__global__ __launch_bounds__(kResW * kResH) void k_resolve_oit(RasterArgs a) {
    const Geom &G = a.G;
    const Shade &sh = a.sh;
    const int ntx = (G.W + kResW - 1) / kResW, nty = (G.H + kResRows - 1) / kResRows;
    const int64_t per_scene = (int64_t)ntx * nty;
    const int64_t ntiles = per_scene * G.S;
    const int64_t q = ntiles / kXcd, rem = ntiles % kXcd;
    const int xcd = blockIdx.x % kXcd;
    const uint32_t tile = (uint32_t)(xcd * q + min<int64_t>(xcd, rem) + blockIdx.x / kXcd);
    const int32_t s = G.S == 1 ? 0 : (int32_t)(tile / (uint32_t)per_scene);
    const uint32_t ts = tile - (uint32_t)s * (uint32_t)per_scene;
    const int ty = (int)(ts / (uint32_t)ntx), tx = (int)(ts - (uint32_t)ty * (uint32_t)ntx);
    const int px = tx * kResW + (int)(threadIdx.x % kResW);
    const int64_t item_base = G.instanced ? (int64_t)s * G.T : (G.S > 1 ? G.tri_off[s] : 0);
    const int64_t vbase = (G.S > 1 && !G.instanced) ? G.vtx_off[s] : 0;
    const int64_t layer_stride = (int64_t)G.S * G.W * G.H;
#pragma unroll 1
    for (int k = 0; k < kResPPT; ++k) {
        const int py = ty * kResRows + (int)(threadIdx.x / kResW) + k * kResH;
        if (px >= G.W || py >= G.H) continue;
        const int64_t p = ((int64_t)s * G.H + py) * G.W + px;
        float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, T = 1.0f;
        bool any = false;
        // composite one resolved fragment behind the ones before it
        auto composite = [&](const Resolve &r) {
            const int32_t X0 = (int32_t)r.xy.x, Y0 = (int32_t)r.xy.y, X1 = (int32_t)r.xy.z,
                          Y1 = (int32_t)r.xy.w;
            const int32_t X2 = (int32_t)r.xy2.x, Y2 = (int32_t)r.xy2.y;
            const int64_t Px = 256 * (int64_t)px + 128, Py = 256 * (int64_t)py + 128;
            const int64_t E0 = (int64_t)(X2 - X1) * (Py - Y1) - (int64_t)(Y2 - Y1) * (Px - X1);
            const int64_t E1 = (int64_t)(X0 - X2) * (Py - Y2) - (int64_t)(Y0 - Y2) * (Px - X2);
            const int64_t E2 = (int64_t)(X1 - X0) * (Py - Y0) - (int64_t)(Y1 - Y0) * (Px - X0);
            const float bs0 = (float)((double)E0 * r.sinv);
            const float bs1 = (float)((double)E1 * r.sinv);
            const float bs2 = (float)((double)E2 * r.sinv);
            const float qq0 = bs0 * r.iw[0], qq1 = bs1 * r.iw[1], qq2 = bs2 * r.iw[2];
            const float Q = (qq0 + qq1) + qq2;
            const float b1 = qq1 / Q, b2 = qq2 / Q;
            const float b0 = (1.0f - b1) - b2;
            float al = b0 * sh.alpha[r.v[0]];
            al = al + b1 * sh.alpha[r.v[1]];
            al = al + b2 * sh.alpha[r.v[2]];
            float rgb[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = b0 * r.c[0][ch];
                acc = acc + b1 * r.c[1][ch];
                acc = acc + b2 * r.c[2][ch];
                rgb[ch] = acc;
            }
            const float w = T * al;
            C0 = C0 + w * rgb[0];
            C1 = C1 + w * rgb[1];
            C2 = C2 + w * rgb[2];
            T = T * (1.0f - al);
            if (!any) {
                any = true;
                if (sh.out_depth) sh.out_depth[p] = r.depth;
                if (sh.out_primid) sh.out_primid[p] = (int32_t)r.t;
                if (sh.out_bary) reinterpret_cast<float2 *>(sh.out_bary)[p] = make_float2(b1, b2);
            }
        };
        // two layers at a time, so that their gathers overlap
#pragma unroll 1
        for (int l = 0; l < sh.layers; l += 2) {
            const unsigned long long k0 = a.w.keys[p + l * layer_stride];
            const unsigned long long k1 =
                l + 1 < sh.layers ? a.w.keys[p + (l + 1) * layer_stride] : kEmptyKey;
            if (k0 == kEmptyKey) break;
            Resolve r0, r1;
            resolve_fetch<PK_SHADE_GOURAUD>(a, s, item_base, vbase, px, py, k0, r0);
            resolve_fetch<PK_SHADE_GOURAUD>(a, s, item_base, vbase, px, py, k1, r1);
            resolve_attribs<PK_SHADE_GOURAUD>(a, s, r0);
            resolve_attribs<PK_SHADE_GOURAUD>(a, s, r1);
            composite(r0);
            if (k1 == kEmptyKey) break;
            composite(r1);
        }
        if (!any) {
            if (sh.out_depth) sh.out_depth[p] = 1.0f;
            if (sh.out_primid) sh.out_primid[p] = -1;
            if (sh.out_bary) reinterpret_cast<float2 *>(sh.out_bary)[p] = make_float2(0, 0);
        }
        if (sh.out_color)
            reinterpret_cast<float4 *>(sh.out_color)[p] =
                make_float4(C0, C1, C2, any ? 1.0f - T : 0.0f);
    }
}

// 32-px bins keep transparency slots in LDS for up to this many layers
// ((K-1) * 8 KB); beyond, they peel
constexpr int kSlotLayers32 = 3;

template <int TPB, int B, int SHADE>
static hipError_t launch_b(const RasterArgs &a, dim3 grid, hipStream_t st) {
    if constexpr (SHADE == kKeysOnly && B <= 32) {
        if (a.sh.layers > 0 && (B <= 16 || a.sh.layers <= kSlotLayers32)) {
            // K slots per pixel fit the LDS: one pass
            const size_t slots = (size_t)(a.sh.layers - 1) * B * B * sizeof(unsigned long long);
            hipLaunchKernelGGL((k_raster<TPB, B, SHADE, false, false, true>), grid, dim3(TPB),
                               slots, st, a);
            return hipGetLastError();
        }
    }
    if constexpr (SHADE == kKeysOnly && B == 32) {
        if (a.sh.layers > kSlotLayers32) {
            hipLaunchKernelGGL((k_raster<TPB, B, SHADE, false, true>), grid, dim3(TPB), 0, st, a);
            return hipGetLastError();
        }
    }
    if (a.schedule == PK_SCHED_DIRECT_MAP)
        hipLaunchKernelGGL((k_raster<TPB, B, SHADE, true>), grid, dim3(TPB), 0, st, a);
    else
        hipLaunchKernelGGL((k_raster<TPB, B, SHADE, false>), grid, dim3(TPB), 0, st, a);
    return hipGetLastError();
}

template <int TPB, int SHADE>
static hipError_t launch_tpb(const RasterArgs &a, dim3 grid, hipStream_t st) {
    switch (a.G.B) {
    case 8:  return launch_b<TPB, 8, SHADE>(a, grid, st);
    case 16: return launch_b<TPB, 16, SHADE>(a, grid, st);
    case 32: return launch_b<TPB, 32, SHADE>(a, grid, st);
    case 64: return launch_b<TPB, 64, SHADE>(a, grid, st);
    default: return hipErrorInvalidValue;
    }
}

template <int SHADE>
static hipError_t launch_shade(const RasterArgs &a, int tpb, dim3 grid, hipStream_t st) {
    switch (tpb) {
    case 64:  return launch_tpb<64, SHADE>(a, grid, st);
    case 128: return launch_tpb<128, SHADE>(a, grid, st);
    case 256: return launch_tpb<256, SHADE>(a, grid, st);
    default:  return hipErrorInvalidValue;
    }
}

template <int SHADE>
static hipError_t launch_resolve(const RasterArgs &a, hipStream_t st) {
    // one workgroup per tile; the tile count is a multiple of nothing in
    // particular, so ranges differ by at most one tile between dies
    if (a.G.W <= 512) {
        const int64_t ntiles = (int64_t)((a.G.W + 15) / 16) * ((a.G.H + 16 * kResPPT - 1) /
                                                            (16 * kResPPT)) * a.G.S;
        hipLaunchKernelGGL((k_resolve<SHADE, 16, 16>), dim3((unsigned)ntiles), dim3(256), 0, st, a);
        return hipGetLastError();
    }
    const int64_t ntiles = (int64_t)((a.G.W + kResW - 1) / kResW) *
                           ((a.G.H + kResRows - 1) / kResRows) * a.G.S;
    hipLaunchKernelGGL((k_resolve<SHADE, kResW, kResH>), dim3((unsigned)ntiles), dim3(kResW * kResH),
                       0, st, a);
    return hipGetLastError();
}

hipError_t launch_resolve_pass(const Geom &G, const Ws &w, const Shade &sh, hipStream_t st) {
    if (G.nbins_total == 0) return hipSuccess;
    RasterArgs a{G, w, sh, 0};
    if (sh.layers > 0) {
        const int64_t ntiles = (int64_t)((G.W + kResW - 1) / kResW) *
                               ((G.H + kResRows - 1) / kResRows) * G.S;
        hipLaunchKernelGGL(k_resolve_oit, dim3((unsigned)ntiles), dim3(kResW * kResH), 0, st, a);
        return hipGetLastError();
    }
    switch (sh.shading) {
    case PK_SHADE_GOURAUD:  return launch_resolve<PK_SHADE_GOURAUD>(a, st);
    case PK_SHADE_TEXTURED: return launch_resolve<PK_SHADE_TEXTURED>(a, st);
    case PK_SHADE_DEFERRED: return launch_resolve<PK_SHADE_DEFERRED>(a, st);
    case PK_SHADE_LIT:      return launch_resolve<PK_SHADE_LIT>(a, st);
    default:                return hipErrorInvalidValue;
    }
}

hipError_t launch_raster(const Geom &G, const Ws &w, const Shade &sh, int schedule, int tpb,
                         int groups, RasterMode mode, hipStream_t st) {
    if (G.nbins_total == 0) return hipSuccess;
    if (G.B == 0) return launch_direct(G, w, sh, mode, st);
    if (G.two_level) {
        // fine bins (keys to the workspace), then coarse bins starting from
        // those keys, then the per-pixel resolve
        Geom Gf = G, Gc = G;
        Gf.nbins_scene = G.nbins_f;
        Gf.nbins_total = (int64_t)G.S * G.nbins_f;
        Gc.B = 4 * G.B;
        Gc.log2B = G.log2B + 2;
        Gc.nbx = G.nbx_c;
        Gc.nby = G.nby_c;
        Gc.nbins_scene = G.nbx_c * G.nby_c;
        Gc.nbins_total = (int64_t)G.S * Gc.nbins_scene;
        hipError_t e = hipSuccess;
        for (int level = 0; level < 2 && e == hipSuccess; ++level) {
            const Geom &Gl = level ? Gc : Gf;
            const int tl = level ? 256 : tpb;
            // the coarse level: one workgroup per coarse bin (LOAD_BALANCE),
            // so that a bin without triangles costs nothing but its launch
            const int sl = level ? PK_SCHED_LOAD_BALANCE : schedule;
            RasterArgs al{Gl, w, sh, sl, G.nbins_scene, level ? G.nbins_f : 0, level};
            const int64_t nb = sl == PK_SCHED_LOAD_BALANCE ? Gl.nbins_total
                               : (groups < Gl.nbins_total ? groups : Gl.nbins_total);
            e = launch_shade<kKeysOnly>(al, tl, dim3((unsigned)nb), st);
        }
        if (e != hipSuccess) return e;
        if (sh.frag_count) {
            hipLaunchKernelGGL(k_raster_epilogue, dim3(1), dim3(kFragSlots), 0, st, w.misc,
                               sh.frag_count, 0);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (mode == kRasterSplit) return launch_resolve_pass(G, w, sh, st);
        return hipSuccess;
    }
    RasterArgs a{G, w, sh, schedule};
    int64_t nblk = G.nbins_total;
    if (schedule != PK_SCHED_LOAD_BALANCE) nblk = groups < G.nbins_total ? groups : G.nbins_total;
    const dim3 grid((unsigned)nblk);
    hipError_t e = hipSuccess;
    if (w.split) {
        // pieces of a bin merge by atomic min, bins without pairs have no
        // work item: start from empty keys
        e = launch_fill_u32(reinterpret_cast<uint32_t *>(w.keys), 2 * (int64_t)G.S * G.W * G.H,
                            0xffffffffu, st);
        if (e != hipSuccess) return e;
    }
    if (mode != kRasterFused) {
        e = launch_shade<kKeysOnly>(a, tpb, grid, st);
    } else {
        switch (sh.shading) {
        case PK_SHADE_GOURAUD:  e = launch_shade<PK_SHADE_GOURAUD>(a, tpb, grid, st); break;
        case PK_SHADE_TEXTURED: e = launch_shade<PK_SHADE_TEXTURED>(a, tpb, grid, st); break;
        case PK_SHADE_DEFERRED: e = launch_shade<PK_SHADE_DEFERRED>(a, tpb, grid, st); break;
        case PK_SHADE_LIT:      e = launch_shade<PK_SHADE_LIT>(a, tpb, grid, st); break;
        default:                e = hipErrorInvalidValue;
        }
    }
    if (e != hipSuccess) return e;
    const int rewind = schedule == PK_SCHED_DYNAMIC;
    if (sh.frag_count || rewind) {
        hipLaunchKernelGGL(k_raster_epilogue, dim3(1), dim3(kFragSlots), 0, st, w.misc,
                           sh.frag_count, rewind);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (mode == kRasterSplit) return launch_resolve_pass(G, w, sh, st);
    return hipSuccess;
}

// Deferred shading pass over the G-buffer: colour = albedo * sum_l max(0, n.l).
__global__ __launch_bounds__(256) void k_deferred(Shade sh, int64_t npix) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= npix) return;
    if (sh.out_primid[p] < 0) {
        reinterpret_cast<float4 *>(sh.out_color)[p] = make_float4(0, 0, 0, 0);
        return;
    }
    const Float3 nn = *reinterpret_cast<const Float3 *>(sh.gbuf_n + 3 * p);
    const float lit = light_sum(sh, nn.x, nn.y, nn.z);
    const Float3 al = *reinterpret_cast<const Float3 *>(sh.gbuf_a + 3 * p);
    reinterpret_cast<float4 *>(sh.out_color)[p] = make_float4(al.x * lit, al.y * lit, al.z * lit, 1.0f);
}

hipError_t launch_deferred(const Geom &G, const Shade &sh, hipStream_t st) {
    const int64_t npix = (int64_t)G.S * G.W * G.H;
    if (npix == 0) return hipSuccess;
    hipLaunchKernelGGL(k_deferred, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, sh,
                       npix);
    return hipGetLastError();
}

}  // namespace pk
