// k_setup.hip -- geometry phase of the sort-middle renderer and AssignBin of
// the screen-space stage (Piko Sec. 4.4; AssignToBoundingBox, Sec. 4.3;
// bin management by prefix sums, Sec. 6).
//
//   k_setup    one thread per triangle: gather three vertices, transform and
//              snap them, compute the setup record, cull, and count the
//              triangle into every bin its sample bounding box overlaps.
//   k_scan     exclusive prefix sum of the per-bin counts into CSR offsets.
//   k_scatter  one thread per triangle: append the triangle to each of its
//              bins' lists at a slot taken from the bin's cursor.
#include <climits>

#include "pk_internal.h"

#pragma clang fp contract(off)

namespace pk {

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// A setup/scatter workgroup covers kGroupItems consecutive triangles.  When
// the bins those triangles touch span at most kHist consecutive bin numbers
// (counted over the scenes they belong to), the per-bin counts are first
// accumulated in LDS over that span and flushed with one global atomic per
// touched bin (and the scatter reserves one contiguous slot range per
// touched bin); otherwise lanes fall back to wave-aggregated global atomics.
// Device-scope atomics are slow on this part, LDS atomics are not.
// 512 threads with two triangles each measured fastest on the batched
// scenes and as fast as any on the 1080p grid (batch256 frame 1.40 ms,
// against 1.45 with 256 threads and four; grid1080 0.093 either way): more
// waves share each LDS histogram.
constexpr int kGroupThreads = 512;
constexpr int kItemsPerThread = 2;
constexpr int kGroupItems = kGroupThreads * kItemsPerThread;
// (with the reduction words, one workgroup takes exactly 32 KiB of LDS).
// k_setup takes its histogram as dynamic LDS, launched without it for
// whole-screen bins, which count nothing: there the occupancy is not
// capped by LDS.
constexpr int kHist = 8192 - 2 * kGroupThreads / 64;

__device__ inline int32_t scene_of(const Geom &G, int64_t item) {
    if (G.S == 1) return 0;
    if (G.instanced) return (int32_t)((uint32_t)item / (uint32_t)G.T);   // items < 2^31
    return item_ref(G, item).s;
}

// First scene of this workgroup's items: bin numbers inside the workgroup
// count from that scene's first bin.
__device__ inline int32_t group_scene(const Geom &G, int64_t first) {
    return scene_of(G, first);
}

// Vertex Shader stage for indexed meshes: each vertex (of each view when
// instanced) is transformed and snapped once, instead of once per triangle
// that uses it.  The same vertex_stage function as the per-triangle path, so
// the results are identical.
// It also clears the nzero words at `zero` (the bin counters and misc words
// that k_setup accumulates into), which saves a fill launch.
__global__ __launch_bounds__(256) void k_vertex(Geom G, Ws w, uint32_t *zero, int64_t nzero) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t j = i; j < nzero; j += (int64_t)gridDim.x * blockDim.x) zero[j] = 0u;
    const int64_t nv = G.V * (G.instanced ? G.S : 1);
    if (i >= nv) return;
    int32_t s = 0;
    int64_t v = i;
    if (G.instanced) {
        s = (int32_t)((uint64_t)i / (uint64_t)G.V);
        v = i - (int64_t)s * G.V;
    } else if (G.S > 1) {
        int lo = 0, hi = G.S - 1;           // last scene with vtx_off[s] <= v
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (G.vtx_off[mid] <= v) lo = mid; else hi = mid - 1;
        }
        s = lo;
    }
    const float *m = G.mvp ? G.mvp + 16 * (int64_t)s : nullptr;
    VtxRec r;
    if (!vertex_stage(G, v, m, r.X, r.Y, r.z, r.iw)) { r.X = kBadVertex; r.Y = 0; r.z = 0; r.iw = 0; }
    reinterpret_cast<int4 *>(w.vtx)[i] = make_int4(r.X, r.Y, __float_as_int(r.z), __float_as_int(r.iw));
}

// Returns the packed pixel bbox (kEmptyKey when culled).
__device__ inline uint64_t setup_finish(const Geom &G, const Ws &w, int64_t item,
                                        const TriIn &t) {
    if (item >= G.items) return kEmptyKey;
    int32_t X[3], Y[3];
    float z[3], iw[3];
    const uint64_t bb = setup_snap(G, t, X, Y, z, iw);
    if (bb != kEmptyKey) store_record(G, w, item, X, Y, z, iw);
    w.bbox[item] = bb;
    return bb;
}

// Bin rectangle of a packed bbox: nb bins starting at (bx0, by0), nbx_t wide,
// numbered base + by * stride + bx within the scene.  With two bin levels a
// triangle whose box spans more than 2 x 2 fine bins goes to the coarse bins
// (four times the size) instead.
struct BinRect {
    int bx0, by0, nbx_t, nb, base, stride;
};

__device__ inline BinRect bin_rect(const Geom &G, uint64_t bb) {
    BinRect r;
    r.base = 0;
    r.stride = G.nbx;
    if (bb == kEmptyKey) { r.bx0 = r.by0 = 0; r.nbx_t = 1; r.nb = 0; return r; }
    int sh = G.log2B;
    r.bx0 = bb_x0(bb) >> sh;
    r.by0 = bb_y0(bb) >> sh;
    r.nbx_t = (bb_x1(bb) >> sh) - r.bx0 + 1;
    int rows = (bb_y1(bb) >> sh) - r.by0 + 1;
    if (G.two_level && (r.nbx_t > 2 || rows > 2)) {
        sh += 2;
        r.bx0 = bb_x0(bb) >> sh;
        r.by0 = bb_y0(bb) >> sh;
        r.nbx_t = (bb_x1(bb) >> sh) - r.bx0 + 1;
        rows = (bb_y1(bb) >> sh) - r.by0 + 1;
        r.base = G.nbins_f;
        r.stride = G.nbx_c;
    }
    r.nb = r.nbx_t * rows;
    return r;
}

__device__ inline int bin_of(const BinRect &br, int cx, int cy) { return br.base + cy * br.stride + cx; }

// The device-atomic path for a wave whose items have bin rectangles of very
// different sizes (a large triangle among small ones): instead of one round
// per bin of the largest rectangle, with the other lanes idle, the wave's
// (item, bin) pairs are laid end to end in lane order and dealt 64 at a time,
// one per lane.  Pair j belongs to the last lane whose first pair is at or
// before j (a binary search over the lanes' exclusive prefix of counts); its
// rectangle, scene and item come from that lane by shuffles.  fn(key, item)
// runs on every lane once per round, key = scene * bins per scene + bin, or
// -1 for no pair.  Call from uniform control flow.
template <class F>
__device__ inline void spread_pairs(const Geom &G, const BinRect &br, int32_t s, int64_t item, F fn) {
    const int lane = threadIdx.x & (kWave - 1);
    int incl = br.nb;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += y;
    }
    const int total = __shfl(incl, kWave - 1, kWave);
    const int start = incl - br.nb;
    const int ilo = (int)(uint32_t)item, ihi = (int)(item >> 32);
    for (int b = 0; b < total; b += kWave) {
        const int j = b + lane;
        // the largest lane whose first pair is at or before j (starts never
        // decrease over the lanes, and the owner found has pairs: a lane with
        // none starts where the next one does)
        int o = 0;
#pragma unroll
        for (int step = kWave / 2; step >= 1; step >>= 1) {
            const int c = o + step;
            const int sc = __shfl(start, c, kWave);
            if (sc <= j) o = c;
        }
        const int o_start = __shfl(start, o, kWave);
        const int bx0 = __shfl(br.bx0, o, kWave), by0 = __shfl(br.by0, o, kWave);
        const int nbx = __shfl(br.nbx_t, o, kWave);
        const int base = __shfl(br.base, o, kWave), stride = __shfl(br.stride, o, kWave);
        const int so = __shfl(s, o, kWave);
        const int64_t it = ((int64_t)__shfl(ihi, o, kWave) << 32) |
                           (uint32_t)__shfl(ilo, o, kWave);
        int key = -1;
        if (j < total) {
            const int local = j - o_start;
            const int ry = (int)((uint32_t)local / (uint32_t)nbx), rx = local - ry * nbx;
            key = so * G.nbins_scene + base + (by0 + ry) * stride + bx0 + rx;
        }
        fn(key, it);
    }
}

// Whether spreading the wave's pairs over the lanes saves rounds: the
// largest rectangle needs wave_max(nb) rounds one bin at a time, the spread
// needs ceil(total / 64) plus the cost of its searches.
__device__ inline bool spread_pays(int nb) {
    const int mx = wave_max(nb);
    int total = nb;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) total += __shfl_xor(total, d, kWave);
    return mx > (total + kWave - 1) / kWave + 4;
}

// Range [lo, hi] of LDS window indices ((scene - s_lo) * bins per scene +
// bin) that a triangle's bin rectangle touches; lo > hi when it touches none.
__device__ inline void window_span(const Geom &G, const BinRect &br, int32_t s, int32_t s_lo,
                                   int &lo, int &hi) {
    if (br.nb == 0) { lo = INT_MAX; hi = INT_MIN; return; }
    const int base = (s - s_lo) * G.nbins_scene;
    const int rows = br.nb / br.nbx_t;
    lo = base + bin_of(br, br.bx0, br.by0);
    hi = base + bin_of(br, br.bx0 + br.nbx_t - 1, br.by0 + rows - 1);
}

// Smallest lo and largest hi over the workgroup.  Contains barriers: call
// from uniform control flow.  s_red holds 2 ints per wave.
__device__ inline void group_span(int lo, int hi, int *s_red, int &glo, int &ghi) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        lo = min(lo, __shfl_xor(lo, d, kWave));
        hi = max(hi, __shfl_xor(hi, d, kWave));
    }
    const int wid = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) { s_red[2 * wid] = lo; s_red[2 * wid + 1] = hi; }
    __syncthreads();
    glo = INT_MAX;
    ghi = INT_MIN;
#pragma unroll
    for (int i = 0; i < kGroupThreads / kWave; ++i) {
        glo = min(glo, s_red[2 * i]);
        ghi = max(ghi, s_red[2 * i + 1]);
    }
}

__global__ __launch_bounds__(kGroupThreads) void k_setup(Geom G, Ws w) {
    extern __shared__ uint32_t s_hist[];   // kHist words, binned screens only
    __shared__ int s_red[2 * kGroupThreads / kWave];
    const int tid = threadIdx.x;
    const int64_t first = blockIdx.x * (int64_t)kGroupItems;
    const int32_t s_lo = group_scene(G, first);
    TriIn tin[kItemsPerThread];
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k)
        setup_indices(G, first + k * kGroupThreads + tid, tin[k]);
    if (G.idx) {
#pragma unroll
        for (int k = 0; k < kItemsPerThread; ++k) setup_index_load(G, tin[k]);
    }
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) setup_fetch(G, w, tin[k]);
    if (G.B == 0) {
        // whole-screen bins: records and boxes only, no per-bin counts
#pragma unroll
        for (int k = 0; k < kItemsPerThread; ++k)
            setup_finish(G, w, first + k * kGroupThreads + tid, tin[k]);
        return;
    }
    // (unrolled: tin and the rectangles must stay in registers)
    BinRect br[kItemsPerThread];
    int lo = INT_MAX, hi = INT_MIN;
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
        const int64_t item = first + k * kGroupThreads + tid;
        br[k] = bin_rect(G, setup_finish(G, w, item, tin[k]));
        int l, h;
        window_span(G, br[k], tin[k].s, s_lo, l, h);
        lo = min(lo, l);
        hi = max(hi, h);
    }
    // AssignBin counts of the screen-space stage.  In LDS, only over the
    // span of bins this workgroup touches (a row strip for coherent meshes)
    int glo, ghi;
    group_span(lo, hi, s_red, glo, ghi);
    // (a workgroup touching no bin has glo > ghi and takes the other path,
    // which then does nothing)
    const bool lds = glo <= ghi && (int64_t)ghi - glo + 1 <= kHist;
    if (lds) {
        for (int i = glo + tid; i <= ghi; i += kGroupThreads) s_hist[i - glo] = 0;
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
        const int32_t s = tin[k].s;
        if (lds) {
            // LDS atomics are cheap enough per lane
            const int hb = (s - s_lo) * G.nbins_scene - glo;   // histogram index of bin 0
            int cx = br[k].bx0, cy = br[k].by0;
            for (int r = 0; r < br[k].nb; ++r) {
                atomicAdd(s_hist + (hb + bin_of(br[k], cx, cy)), 1u);
                if (++cx >= br[k].bx0 + br[k].nbx_t) { cx = br[k].bx0; ++cy; }
            }
        } else if (spread_pays(br[k].nb)) {
            spread_pairs(G, br[k], s, 0, [&](int key, int64_t) { agg_count(w.bin_count, key); });
        } else {
            // one round per bin of the largest bin rectangle in the wave
            const int rounds = wave_max(br[k].nb);
            const int base = s * G.nbins_scene;
            int cx = br[k].bx0, cy = br[k].by0;
            for (int r = 0; r < rounds; ++r) {
                agg_count(w.bin_count, r < br[k].nb ? base + bin_of(br[k], cx, cy) : -1);
                if (++cx >= br[k].bx0 + br[k].nbx_t) { cx = br[k].bx0; ++cy; }
            }
        }
    }
    if (lds) {
        __syncthreads();
        uint32_t *dst = w.bin_count + (int64_t)s_lo * G.nbins_scene;
        for (int i = glo + tid; i <= ghi; i += kGroupThreads) {
            const uint32_t c = s_hist[i - glo];
            if (c) atomicAdd(dst + i, c);
        }
    }
}

hipError_t launch_setup(const Geom &G, const Ws &w, hipStream_t st) {
    // bin_count and misc are adjacent: one fill clears both (and the padding)
    const int64_t words = (reinterpret_cast<char *>(w.misc) - reinterpret_cast<char *>(w.bin_count)) / 4 + kMiscWords;
    hipError_t e = hipSuccess;
    if (G.idx && G.items > 0) {
        // the vertex kernel clears them on its way (grid-stride)
        const int64_t nv = G.V * (G.instanced ? G.S : 1);
        int64_t blocks = (nv + 255) / 256;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(k_vertex, dim3((unsigned)blocks), dim3(256), 0, st, G, w, w.bin_count,
                           words);
        e = hipGetLastError();
    } else {
        e = launch_fill_u32(w.bin_count, words, 0u, st);
    }
    if (e != hipSuccess || G.items == 0) return e;
    if (w.fb_groups) return launch_fb_count(G, w, st);
    // whole-screen bins: the triangle setup runs inside the depth-test
    // kernel (k_direct), which needs no record or box from here
    if (G.B == 0) return hipSuccess;
    const int64_t blocks = (G.items + kGroupItems - 1) / kGroupItems;
    const size_t hist = G.B ? kHist * sizeof(uint32_t) : 0;
    hipLaunchKernelGGL(k_setup, dim3((unsigned)blocks), dim3(kGroupThreads), hist, st, G, w);
    return hipGetLastError();
}

// Single-workgroup exclusive scan over the bin counts, in tiles of
// kScanThreads * kScanPer counts: coalesced loads into LDS, a contiguous run
// of kScanPer counts per thread, a workgroup scan of the run sums, and
// coalesced stores of offsets and cursors.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;

// Exclusive prefix sum of get(0..n-1) by the whole (single) workgroup, tile
// by tile; put(i, prefix) stores each result.  Returns the total.
template <class Get, class Put>
__device__ inline int64_t block_scan(int64_t n, Get get, Put put, uint32_t *s_v, int64_t *s_part) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    int64_t carry = 0;
    for (int64_t t0 = 0; t0 < n; t0 += kScanTile) {
        // all of a thread's loads first (past the end from entry n - 1, which
        // exists here, and ignored), then the stores: no load waits for another
        uint32_t g[kScanPer];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int64_t i = t0 + k * kScanThreads + tid;
            g[k] = get(i < n ? i : n - 1);
        }
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int64_t i = t0 + k * kScanThreads + tid;
            s_v[k * kScanThreads + tid] = i < n ? g[k] : 0u;
        }
        __syncthreads();
        uint32_t v[kScanPer];
        int64_t sum = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) { v[k] = s_v[tid * kScanPer + k]; sum += v[k]; }
        int64_t x = sum;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int64_t y = __shfl_up(x, d, kWave);
            if (lane >= d) x += y;
        }
        if (lane == kWave - 1) s_part[wid] = x;
        __syncthreads();
        int64_t before = 0, total = 0;
#pragma unroll
        for (int i = 0; i < kScanThreads / kWave; ++i) {
            before += (i < wid) ? s_part[i] : 0;
            total += s_part[i];
        }
        int64_t run = carry + before + x - sum;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            s_v[tid * kScanPer + k] = (uint32_t)run;   // wraps only when it overflows,
            run += v[k];                                // which the caller reports
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int64_t i = t0 + k * kScanThreads + tid;
            if (i < n) put(i, (int32_t)s_v[k * kScanThreads + tid]);
        }
        carry += total;
        __syncthreads();
    }
    return carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan(Ws w, int64_t n, int64_t *pairs_needed) {
    __shared__ uint32_t s_v[kScanTile];
    __shared__ int64_t s_part[kScanThreads / kWave];
    __shared__ int s_hist[33];
    const int64_t carry = block_scan(
        n, [&](int64_t i) { return w.bin_count[i]; },
        [&](int64_t i, int32_t o) { w.bin_off[i] = o; w.cursor[i] = o; }, s_v, s_part);
    const bool fits = carry <= w.pair_capacity;
    if (threadIdx.x == 0) {
        w.bin_off[n] = fits ? (int32_t)carry : 0;
        w.misc[1] = fits ? 0u : 1u;
        if (pairs_needed) *pairs_needed = carry;
    }
    if (w.order) {
        // DYNAMIC: each die's range of bins (the bin kernel's ranges) ordered
        // by descending pair count, in buckets of equal bit length (empty
        // bins last), by a counting sort per range
        const int64_t q = n / kXcd, rem = n % kXcd;
        for (int d = 0; d < kXcd; ++d) {
            const int64_t beg = d * q + min<int64_t>(d, rem), len = q + (d < rem ? 1 : 0);
            if (threadIdx.x < 33) s_hist[threadIdx.x] = 0;
            __syncthreads();
            for (int64_t i = threadIdx.x; i < len; i += kScanThreads) {
                const uint32_t c = w.bin_count[beg + i];
                atomicAdd(&s_hist[c ? 32 - __clz((int)c) : 0], 1);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int run = 0;
                for (int bk = 32; bk >= 0; --bk) {
                    const int t = s_hist[bk];
                    s_hist[bk] = run;
                    run += t;
                }
            }
            __syncthreads();
            for (int64_t i = threadIdx.x; i < len; i += kScanThreads) {
                const uint32_t c = w.bin_count[beg + i];
                const int pos = atomicAdd(&s_hist[c ? 32 - __clz((int)c) : 0], 1);
                w.order[beg + pos] = (int32_t)(beg + i);
            }
            __syncthreads();
        }
    }
    if (w.split && fits) {
        // PK_SCHED_SPLIT: bin b is ceil(count / split) work items (none when
        // empty); vbin_off numbers them
        const uint32_t sp = (uint32_t)w.split;
        const int64_t works = block_scan(
            n, [&](int64_t i) { return (w.bin_count[i] + sp - 1u) / sp; },
            [&](int64_t i, int32_t o) { w.vbin_off[i] = o; }, s_v, s_part);
        if (threadIdx.x == 0) w.vbin_off[n] = (int32_t)works;
    }
}

hipError_t launch_scan(const Geom &G, const Ws &w, int64_t *pairs_needed, hipStream_t st) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, st, w, G.nbins_total,
                       pairs_needed);
    return hipGetLastError();
}

__global__ __launch_bounds__(kGroupThreads) void k_scatter(Geom G, Ws w) {
    __shared__ uint32_t s_hist[kHist];
    __shared__ int s_red[2 * kGroupThreads / kWave];
    if (w.misc[1]) return;   // pair capacity exceeded: lists stay unwritten
    const int tid = threadIdx.x;
    const int64_t first = blockIdx.x * (int64_t)kGroupItems;
    const int32_t s_lo = group_scene(G, first);
    uint64_t bb[kItemsPerThread];
    int32_t sc[kItemsPerThread];
    // (both boxes loaded before either is used; an item past the end reads
    // box items - 1, which exists whenever this kernel runs, and ignores it)
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
        const int64_t item = first + k * kGroupThreads + tid;
        bb[k] = w.bbox[item < G.items ? item : G.items - 1];
    }
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
        const int64_t item = first + k * kGroupThreads + tid;
        if (item >= G.items) bb[k] = kEmptyKey;
        sc[k] = bb[k] != kEmptyKey ? scene_of(G, item) : 0;
    }
    // the span of bins this workgroup touches
    int lo = INT_MAX, hi = INT_MIN;
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
        int l, h;
        window_span(G, bin_rect(G, bb[k]), sc[k], s_lo, l, h);
        lo = min(lo, l);
        hi = max(hi, h);
    }
    int glo, ghi;
    group_span(lo, hi, s_red, glo, ghi);
    // (a workgroup touching no bin has glo > ghi and takes the other path,
    // which then does nothing)
    const bool lds = glo <= ghi && (int64_t)ghi - glo + 1 <= kHist;
    if (lds) {
        for (int i = glo + tid; i <= ghi; i += kGroupThreads) s_hist[i - glo] = 0;
        __syncthreads();
        // count this workgroup's pairs per bin
#pragma unroll
        for (int k = 0; k < kItemsPerThread; ++k) {
            const BinRect br = bin_rect(G, bb[k]);
            const int hb = (sc[k] - s_lo) * G.nbins_scene - glo;
            int cx = br.bx0, cy = br.by0;
            for (int r = 0; r < br.nb; ++r) {
                atomicAdd(s_hist + (hb + bin_of(br, cx, cy)), 1u);
                if (++cx >= br.bx0 + br.nbx_t) { cx = br.bx0; ++cy; }
            }
        }
        __syncthreads();
        // reserve one contiguous range per touched bin
        int32_t *cur = w.cursor + (int64_t)s_lo * G.nbins_scene;
        for (int i = glo + tid; i <= ghi; i += kGroupThreads) {
            const uint32_t c = s_hist[i - glo];
            if (c) s_hist[i - glo] = (uint32_t)atomicAdd(cur + i, (int32_t)c);
        }
        __syncthreads();
        // hand out the slots
#pragma unroll
        for (int k = 0; k < kItemsPerThread; ++k) {
            const int64_t item = first + k * kGroupThreads + tid;
            const BinRect br = bin_rect(G, bb[k]);
            const int hb = (sc[k] - s_lo) * G.nbins_scene - glo;
            int cx = br.bx0, cy = br.by0;
            for (int r = 0; r < br.nb; ++r) {
                const uint32_t slot = atomicAdd(s_hist + (hb + bin_of(br, cx, cy)), 1u);
                w.pairs[slot] = (int32_t)item;
                if (++cx >= br.bx0 + br.nbx_t) { cx = br.bx0; ++cy; }
            }
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
        const int64_t item = first + k * kGroupThreads + tid;
        const BinRect br = bin_rect(G, bb[k]);
        if (spread_pays(br.nb)) {
            spread_pairs(G, br, sc[k], item, [&](int key, int64_t it) {
                const int32_t slot = agg_slot(w.cursor, key);
                if (key >= 0) w.pairs[slot] = (int32_t)it;
            });
            continue;
        }
        const int rounds = wave_max(br.nb);
        const int base = sc[k] * G.nbins_scene;
        int cx = br.bx0, cy = br.by0;
        for (int r = 0; r < rounds; ++r) {
            const int key = r < br.nb ? base + bin_of(br, cx, cy) : -1;
            const int32_t slot = agg_slot(w.cursor, key);
            if (key >= 0) w.pairs[slot] = (int32_t)item;
            if (++cx >= br.bx0 + br.nbx_t) { cx = br.bx0; ++cy; }
        }
    }
}

hipError_t launch_scatter(const Geom &G, const Ws &w, hipStream_t st) {
    if (G.items == 0) return hipSuccess;
    const int64_t blocks = (G.items + kGroupItems - 1) / kGroupItems;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(kGroupThreads), 0, st, G, w);
    return hipGetLastError();
}

// (A variant that folded the prefix sum into the scatter, every workgroup
// scanning all counts with each thread owning consecutive bins, measured 2x
// slower on the 1080p grid: the per-thread runs make the count loads
// uncoalesced.  The one-workgroup scan stays.)
hipError_t launch_assign(const Geom &G, const Ws &w, int64_t *pairs_needed, hipStream_t st) {
    if (G.B == 0) {
        // whole-screen bins: every scene is one bin holding all its
        // triangles, and no list is built
        return pairs_needed ? launch_fill_u32(reinterpret_cast<uint32_t *>(pairs_needed), 2, 0u, st)
                            : hipSuccess;
    }
    hipError_t e = launch_scan(G, w, pairs_needed, st);
    if (e == hipSuccess) e = launch_scatter(G, w, st);
    return e;
}

}  // namespace pk
