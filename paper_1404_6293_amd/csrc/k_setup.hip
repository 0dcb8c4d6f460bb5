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

__global__ __launch_bounds__(256) void k_setup(Geom G, Ws w) {
    const int64_t item = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    // lanes past the end stay in the wave (culled) so that the per-bin
    // counting below runs with the whole wave
    const bool in_range = item < G.items;
    int32_t X[3] = {0, 0, 0}, Y[3] = {0, 0, 0};
    float z[3] = {0, 0, 0}, iw[3] = {0, 0, 0};
    bool ok = in_range;
    int32_t s = 0;
    if (in_range) {
        const ItemRef r = item_ref(G, item);
        s = r.s;
        const float *m = G.mvp ? G.mvp + 16 * (int64_t)r.s : nullptr;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t v = vertex_of(G, r, k);
            if (v < 0 || v >= G.V) { ok = false; continue; }
            ok = vertex_stage(G, v, m, X[k], Y[k], z[k], iw[k]) && ok;
        }
    }
    uint64_t bb = kEmptyKey;
    int32_t x0 = 0, x1 = -1, y0 = 0, y1 = -1;
    if (ok) {
        const int64_t A2 = (int64_t)(X[1] - X[0]) * (Y[2] - Y[0]) -
                           (int64_t)(X[2] - X[0]) * (Y[1] - Y[0]);
        if (A2 != 0) {
            const int32_t mnx = min(X[0], min(X[1], X[2])), mxx = max(X[0], max(X[1], X[2]));
            const int32_t mny = min(Y[0], min(Y[1], Y[2])), mxy = max(Y[0], max(Y[1], Y[2]));
            // pixel p is sampled at 256 p + 128 (arithmetic shifts floor)
            x0 = max((mnx + 127) >> 8, 0); x1 = min((mxx - 128) >> 8, G.W - 1);
            y0 = max((mny + 127) >> 8, 0); y1 = min((mxy - 128) >> 8, G.H - 1);
            if (x0 <= x1 && y0 <= y1) {
                bb = (uint64_t)x0 | ((uint64_t)x1 << 16) | ((uint64_t)y0 << 32) |
                     ((uint64_t)y1 << 48);
                TriRec rec;
                rec.X0 = X[0]; rec.Y0 = Y[0]; rec.X1 = X[1]; rec.Y1 = Y[1];
                rec.X2 = X[2]; rec.Y2 = Y[2];
                rec.z0 = z[0]; rec.z1 = z[1]; rec.z2 = z[2];
                rec.iw0 = iw[0]; rec.iw1 = iw[1]; rec.iw2 = iw[2];
                rec.bbox = bb;
                const int64_t a = A2 > 0 ? A2 : -A2;
                const double inv = 1.0 / (double)a;
                rec.sinv = A2 > 0 ? inv : -inv;
                const uint4 *src = reinterpret_cast<const uint4 *>(&rec);
                uint4 *dst = reinterpret_cast<uint4 *>(w.rec + item);
                dst[0] = src[0]; dst[1] = src[1]; dst[2] = src[2]; dst[3] = src[3];
            }
        }
    }
    if (in_range) w.bbox[item] = bb;
    // AssignBin counts of the screen-space stage, one round per bin of the
    // largest bin rectangle in the wave
    const bool live = bb != kEmptyKey;
    const int bx0 = x0 >> G.log2B, bx1 = x1 >> G.log2B;
    const int by0 = y0 >> G.log2B;
    const int nbx_t = bx1 - bx0 + 1;
    const int nb = live ? nbx_t * ((y1 >> G.log2B) - by0 + 1) : 0;
    const int rounds = wave_max(nb);
    const int base = s * G.nbins_scene;
    int cx = bx0, cy = by0;
    for (int r = 0; r < rounds; ++r) {
        agg_count(w.bin_count, r < nb ? base + cy * G.nbx + cx : -1);
        if (++cx > bx1) { cx = bx0; ++cy; }
    }
}

hipError_t launch_setup(const Geom &G, const Ws &w, hipStream_t st) {
    // bin_count and misc are adjacent: one fill clears both (and the padding)
    const int64_t words = (reinterpret_cast<char *>(w.misc) - reinterpret_cast<char *>(w.bin_count)) / 4 + 64;
    hipError_t e = launch_fill_u32(w.bin_count, words, 0u, st);
    if (e != hipSuccess || G.items == 0) return e;
    const int64_t blocks = (G.items + 255) / 256;
    hipLaunchKernelGGL(k_setup, dim3((unsigned)blocks), dim3(256), 0, st, G, w);
    return hipGetLastError();
}

// Single-workgroup exclusive scan over the bin counts, in tiles of
// kScanThreads * kScanPer counts: coalesced loads into LDS, a contiguous run
// of kScanPer counts per thread, a workgroup scan of the run sums, and
// coalesced stores of offsets and cursors.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;

__global__ __launch_bounds__(kScanThreads) void k_scan(Ws w, int64_t n, int64_t *pairs_needed) {
    __shared__ uint32_t s_v[kScanTile];
    __shared__ int64_t s_part[kScanThreads / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    int64_t carry = 0;
    for (int64_t t0 = 0; t0 < n; t0 += kScanTile) {
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int64_t i = t0 + k * kScanThreads + tid;
            s_v[k * kScanThreads + tid] = i < n ? w.bin_count[i] : 0u;
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
            run += v[k];                                // which the flag below reports
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int64_t i = t0 + k * kScanThreads + tid;
            if (i < n) {
                const int32_t o = (int32_t)s_v[k * kScanThreads + tid];
                w.bin_off[i] = o;
                w.cursor[i] = o;
            }
        }
        carry += total;
        __syncthreads();
    }
    if (tid == 0) {
        const bool fits = carry <= w.pair_capacity;
        w.bin_off[n] = fits ? (int32_t)carry : 0;
        w.misc[1] = fits ? 0u : 1u;
        if (pairs_needed) *pairs_needed = carry;
    }
}

hipError_t launch_scan(const Geom &G, const Ws &w, int64_t *pairs_needed, hipStream_t st) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, st, w, G.nbins_total,
                       pairs_needed);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_scatter(Geom G, Ws w) {
    const int64_t item = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (w.misc[1]) return;   // pair capacity exceeded: lists stay unwritten
    const uint64_t bb = item < G.items ? w.bbox[item] : kEmptyKey;
    const bool live = bb != kEmptyKey;
    int32_t s = 0;
    if (live && G.S > 1) s = G.instanced ? (int32_t)(item / G.T) : item_ref(G, item).s;
    const int bx0 = bb_x0(bb) >> G.log2B, bx1 = bb_x1(bb) >> G.log2B;
    const int by0 = bb_y0(bb) >> G.log2B, by1 = bb_y1(bb) >> G.log2B;
    const int nb = live ? (bx1 - bx0 + 1) * (by1 - by0 + 1) : 0;
    const int rounds = wave_max(nb);
    const int base = s * G.nbins_scene;
    int cx = bx0, cy = by0;
    for (int r = 0; r < rounds; ++r) {
        const int key = r < nb ? base + cy * G.nbx + cx : -1;
        const int32_t slot = agg_slot(w.cursor, key);
        if (key >= 0) w.pairs[slot] = (int32_t)item;
        if (++cx > bx1) { cx = bx0; ++cy; }
    }
}

hipError_t launch_scatter(const Geom &G, const Ws &w, hipStream_t st) {
    if (G.items == 0) return hipSuccess;
    const int64_t blocks = (G.items + 255) / 256;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(256), 0, st, G, w);
    return hipGetLastError();
}

}  // namespace pk
