// k_raster.hip -- Schedule + Process of the screen-space stage (Piko Sec. 4.4
// sort-middle renderer): for every bin, coverage, depth test, resolve and
// shading in one kernel.  The paper's Rasterizer, Fragment Shader, Depth
// Test and Composite stages share bin size and bin mapping, so they fuse
// (Sec. 5.2.2); the depth buffer of a bin stays on chip (the on-chip depth
// buffer of Sec. 5.2.4), here as 64-bit (depth, primitive) keys in LDS
// updated with ds_min_u64, which makes the test order-independent.
//
// Work inside a bin is balanced per fragment candidate, not per triangle:
// a chunk of TPB triangles is staged in LDS, each contributes the pixels of
// its bounding box clipped to the bin, a workgroup prefix sum lays those
// candidates end to end, and every thread tests candidates j, j+TPB, ...,
// finding its triangle by binary search over the prefix sums.  Tiny and
// large triangles therefore cost the same per candidate.
//
// Schedules (Sec. 4.3 directives; Sec. 6 work-group organization):
//   LOAD_BALANCE  one workgroup per bin (hardware dispatcher balances)
//   DIRECT_MAP    G workgroups, bin b on workgroup b mod G (pre-scheduled)
//   DYNAMIC       G workgroups pop bins from a device counter
#include "pk_internal.h"

#pragma clang fp contract(off)

namespace pk {

constexpr int kDynBatch = 4;   // bins taken per pop of a DYNAMIC queue

struct RasterArgs {
    Geom G;
    Ws w;
    Shade sh;
    int32_t schedule;
};

// Per-pixel resolve: unpack the winning key, recompute barycentrics at the
// pixel centre, shade and write every requested target.
__device__ inline void resolve_pixel(const RasterArgs &a, int32_t s, int64_t item_base,
                                     int64_t vbase_scene, int px, int py,
                                     unsigned long long key) {
    const Geom &G = a.G;
    const Shade &sh = a.sh;
    const int64_t p = ((int64_t)s * G.H + py) * G.W + px;
    if (key == kEmptyKey) {
        if (sh.out_color) reinterpret_cast<float4 *>(sh.out_color)[p] = make_float4(0, 0, 0, 0);
        if (sh.out_depth) sh.out_depth[p] = 1.0f;
        if (sh.out_primid) sh.out_primid[p] = -1;
        if (sh.out_bary) reinterpret_cast<float2 *>(sh.out_bary)[p] = make_float2(0, 0);
        if (sh.gbuf_n) { sh.gbuf_n[3 * p] = 0; sh.gbuf_n[3 * p + 1] = 0; sh.gbuf_n[3 * p + 2] = 0; }
        if (sh.gbuf_a) { sh.gbuf_a[3 * p] = 0; sh.gbuf_a[3 * p + 1] = 0; sh.gbuf_a[3 * p + 2] = 0; }
        return;
    }
    const int32_t t = (int32_t)(key & 0xffffffffu);
    const float depth = __uint_as_float((uint32_t)(key >> 32));
    const TriRec *rp = a.w.rec + (item_base + t);
    const uint4 q0 = reinterpret_cast<const uint4 *>(rp)[0];
    const uint4 q1 = reinterpret_cast<const uint4 *>(rp)[1];
    const uint4 q2 = reinterpret_cast<const uint4 *>(rp)[2];
    const uint4 q3 = reinterpret_cast<const uint4 *>(rp)[3];
    const int32_t X0 = (int32_t)q0.x, Y0 = (int32_t)q0.y, X1 = (int32_t)q0.z, Y1 = (int32_t)q0.w;
    const int32_t X2 = (int32_t)q1.x, Y2 = (int32_t)q1.y;
    const float iw0 = __uint_as_float(q2.y), iw1 = __uint_as_float(q2.z),
                iw2 = __uint_as_float(q2.w);
    const double sinv = __hiloint2double((int)q3.w, (int)q3.z);
    const int64_t Px = 256 * (int64_t)px + 128, Py = 256 * (int64_t)py + 128;
    const int64_t E0 = (int64_t)(X2 - X1) * (Py - Y1) - (int64_t)(Y2 - Y1) * (Px - X1);
    const int64_t E1 = (int64_t)(X0 - X2) * (Py - Y2) - (int64_t)(Y0 - Y2) * (Px - X2);
    const int64_t E2 = (int64_t)(X1 - X0) * (Py - Y0) - (int64_t)(Y1 - Y0) * (Px - X0);
    const float bs0 = (float)((double)E0 * sinv);
    const float bs1 = (float)((double)E1 * sinv);
    const float bs2 = (float)((double)E2 * sinv);
    const float qq0 = bs0 * iw0, qq1 = bs1 * iw1, qq2 = bs2 * iw2;
    const float Q = (qq0 + qq1) + qq2;
    const float b1 = qq1 / Q, b2 = qq2 / Q;
    const float b0 = (1.0f - b1) - b2;
    // vertices of the winner
    const int64_t g = item_base + t - (G.instanced ? item_base : 0);
    int64_t v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        v[k] = vbase_scene + (G.idx ? (int64_t)G.idx[3 * g + k] : 3 * (int64_t)t + k);
    const int64_t V = G.V;
    float rgb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float *pl = sh.color + c * V;
        float acc = b0 * pl[v[0]];
        acc = acc + b1 * pl[v[1]];
        acc = acc + b2 * pl[v[2]];
        rgb[c] = acc;
    }
    if (sh.shading == PK_SHADE_TEXTURED) {
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
        const float w00 = (1.0f - fs) * (1.0f - ft), w10 = fs * (1.0f - ft);
        const float w01 = (1.0f - fs) * ft, w11 = fs * ft;
        const float *t00 = sh.texture + 3 * ((int64_t)j0 * sh.tex_w + i0);
        const float *t10 = sh.texture + 3 * ((int64_t)j0 * sh.tex_w + i1);
        const float *t01 = sh.texture + 3 * ((int64_t)j1 * sh.tex_w + i0);
        const float *t11 = sh.texture + 3 * ((int64_t)j1 * sh.tex_w + i1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float tc = w00 * t00[c];
            tc = tc + w10 * t10[c];
            tc = tc + w01 * t01[c];
            tc = tc + w11 * t11[c];
            rgb[c] = rgb[c] * tc;
        }
    }
    if (sh.shading == PK_SHADE_DEFERRED) {
        float n[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float *pl = sh.normal + c * V;
            float acc = b0 * pl[v[0]];
            acc = acc + b1 * pl[v[1]];
            acc = acc + b2 * pl[v[2]];
            n[c] = acc;
        }
        float nn = n[0] * n[0];
        nn = nn + n[1] * n[1];
        nn = nn + n[2] * n[2];
        float nh0 = 0.0f, nh1 = 0.0f, nh2 = 0.0f;
        if (nn != 0.0f) {
            const float len = sqrtf(nn);
            nh0 = n[0] / len; nh1 = n[1] / len; nh2 = n[2] / len;
        }
        sh.gbuf_n[3 * p] = nh0; sh.gbuf_n[3 * p + 1] = nh1; sh.gbuf_n[3 * p + 2] = nh2;
        sh.gbuf_a[3 * p] = rgb[0]; sh.gbuf_a[3 * p + 1] = rgb[1]; sh.gbuf_a[3 * p + 2] = rgb[2];
    } else if (sh.out_color) {
        reinterpret_cast<float4 *>(sh.out_color)[p] = make_float4(rgb[0], rgb[1], rgb[2], 1.0f);
    }
    if (sh.out_depth) sh.out_depth[p] = depth;
    if (sh.out_primid) sh.out_primid[p] = t;
    if (sh.out_bary) reinterpret_cast<float2 *>(sh.out_bary)[p] = make_float2(b1, b2);
}

template <int TPB, int B>
__global__ __launch_bounds__(TPB) void k_raster(RasterArgs a) {
    constexpr int NPIX = B * B;
    __shared__ unsigned long long s_key[NPIX];
    // staged chunk of triangles (SoA to keep LDS accesses conflict-free)
    __shared__ int32_t s_A[3][TPB], s_B[3][TPB];
    __shared__ int64_t s_C[3][TPB];
    __shared__ float s_z[3][TPB];
    __shared__ double s_inv[TPB];
    __shared__ int32_t s_org[TPB];    // x0 | y0 << 16 (absolute pixels)
    __shared__ int32_t s_wid[TPB];    // width | owned mask << 8
    __shared__ uint32_t s_mag[TPB];   // ceil(2^32 / width), 0 for width 1
    __shared__ int32_t s_prim[TPB];   // scene-local triangle index
    __shared__ int32_t s_start[TPB];  // exclusive prefix sum of candidate counts
    __shared__ int32_t s_wave[TPB / kWave];
    __shared__ int64_t s_bin, s_bin_end;
    __shared__ unsigned long long s_frag[TPB / kWave];

    const Geom &G = a.G;
    const int tid = threadIdx.x;
    unsigned long long frags = 0;
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
    // DYNAMIC: current queue (range) and the bins of the last batch taken
    int qx = xcd, q_tried = 0;
    int64_t batch_beg = 0, batch_end = 0;
    int64_t iter = 0;
    for (;;) {
        int64_t bin;
        if (a.schedule == PK_SCHED_DYNAMIC) {
            if (batch_beg >= batch_end) {
                // take kDynBatch bins from this die's queue; when it is empty,
                // move on to the other dies' queues
                if (tid == 0) {
                    int64_t b0 = 0, b1 = 0;
                    while (q_tried < kXcd) {
                        const int64_t qb = qx * q + min<int64_t>(qx, rem);
                        const int64_t ql = q + (qx < rem ? 1 : 0);
                        const int64_t t = (int64_t)atomicAdd(&a.w.misc[8 + qx], (uint32_t)kDynBatch);
                        if (t < ql) { b0 = qb + t; b1 = qb + min<int64_t>(t + kDynBatch, ql); break; }
                        qx = (qx + 1) % kXcd;
                        ++q_tried;
                    }
                    s_bin = b0;
                    s_bin_end = b1;
                }
                __syncthreads();
                batch_beg = s_bin;
                batch_end = s_bin_end;
                __syncthreads();
                if (batch_beg >= batch_end) break;
            }
            bin = batch_beg++;
        } else if (a.schedule == PK_SCHED_DIRECT_MAP) {
            if (gridDim.x < kXcd) {            // too few groups to give every die a range
                bin = blockIdx.x + iter * (int64_t)gridDim.x;
                if (bin >= nb) break;
            } else {
                const int64_t l = lane_in_xcd + iter * groups_in_xcd;
                if (l >= r_len) break;
                bin = r_beg + l;
            }
        } else {
            if (iter > 0 || lane_in_xcd >= r_len) break;
            bin = r_beg + lane_in_xcd;
        }
        ++iter;
        const int32_t s = (int32_t)(bin / G.nbins_scene);
        const int32_t lb = (int32_t)(bin - (int64_t)s * G.nbins_scene);
        const int32_t by = lb / G.nbx, bx = lb - by * G.nbx;
        const int32_t px0 = bx * B, py0 = by * B;
        const int32_t pw = min(B, G.W - px0), ph = min(B, G.H - py0);
        const int64_t item_base = G.instanced ? (int64_t)s * G.T : (G.S > 1 ? G.tri_off[s] : 0);
        const int64_t vbase = (G.S > 1 && !G.instanced) ? G.vtx_off[s] : 0;

        for (int i = tid; i < NPIX; i += TPB) s_key[i] = kEmptyKey;
        const bool overflow = a.w.misc[1] != 0;
        const int32_t lbeg = overflow ? 0 : a.w.bin_off[bin];
        const int32_t lend = overflow ? 0 : a.w.bin_off[bin + 1];
        __syncthreads();

        for (int32_t c0 = lbeg; c0 < lend; c0 += TPB) {
            const int32_t nv = min(TPB, lend - c0);
            int cnt = 0;
            if (tid < nv) {
                const int32_t item = a.w.pairs[c0 + tid];
                const TriRec *rp = a.w.rec + item;
                const uint4 q0 = reinterpret_cast<const uint4 *>(rp)[0];
                const uint4 q1 = reinterpret_cast<const uint4 *>(rp)[1];
                const uint4 q2 = reinterpret_cast<const uint4 *>(rp)[2];
                const uint4 q3 = reinterpret_cast<const uint4 *>(rp)[3];
                const int32_t X[3] = {(int32_t)q0.x, (int32_t)q0.z, (int32_t)q1.x};
                const int32_t Y[3] = {(int32_t)q0.y, (int32_t)q0.w, (int32_t)q1.y};
                const uint64_t bb = ((uint64_t)q3.y << 32) | q3.x;
                const double sinv = __hiloint2double((int)q3.w, (int)q3.z);
                const int sgn = sinv > 0.0 ? 1 : -1;
                int owned = 0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int ka = (k + 1) % 3, kb = (k + 2) % 3;   // edge v_ka -> v_kb
                    const int32_t dx = X[kb] - X[ka], dy = Y[kb] - Y[ka];
                    const int32_t Ak = -sgn * dy, Bk = sgn * dx;
                    const int own = (Ak > 0) || (Ak == 0 && Bk < 0);
                    owned |= own << k;
                    s_A[k][tid] = Ak;
                    s_B[k][tid] = Bk;
                    s_C[k][tid] = -((int64_t)Ak * X[ka] + (int64_t)Bk * Y[ka]) + own;
                }
                s_z[0][tid] = __uint_as_float(q1.z);
                s_z[1][tid] = __uint_as_float(q1.w);
                s_z[2][tid] = __uint_as_float(q2.x);
                s_inv[tid] = sinv > 0.0 ? sinv : -sinv;
                const int32_t x0 = max((int32_t)bb_x0(bb), px0), x1 = min((int32_t)bb_x1(bb), px0 + pw - 1);
                const int32_t y0 = max((int32_t)bb_y0(bb), py0), y1 = min((int32_t)bb_y1(bb), py0 + ph - 1);
                const int32_t wdt = x1 - x0 + 1, hgt = y1 - y0 + 1;
                cnt = (wdt > 0 && hgt > 0) ? wdt * hgt : 0;
                s_org[tid] = x0 | (y0 << 16);
                s_wid[tid] = max(wdt, 1) | (owned << 8);
                // ceil(2^32 / width) makes umulhi an exact divide for the
                // candidate counts of one bin (< 2^12); width 1 needs no divide
                s_mag[tid] = wdt > 1 ? 0xffffffffu / (uint32_t)wdt + 1u : 0u;
                s_prim[tid] = (int32_t)(item - item_base);
            }
            int total;
            const int start = block_exclusive_scan<TPB>(cnt, s_wave, total);
            s_start[tid] = start;
            __syncthreads();
            for (int j = tid; j < total; j += TPB) {
                int lo = 0, hi = nv - 1;     // last staged triangle with start <= j
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_start[mid] <= j) lo = mid; else hi = mid - 1;
                }
                const uint32_t local = (uint32_t)(j - s_start[lo]);
                const int32_t wi = s_wid[lo];
                const uint32_t wdt = (uint32_t)(wi & 0xff);
                const uint32_t mag = s_mag[lo];
                const uint32_t row = mag ? __umulhi(local, mag) : local;
                const uint32_t col = local - row * wdt;
                const int32_t org = s_org[lo];
                const int32_t px = (org & 0xffff) + (int32_t)col;
                const int32_t py = (org >> 16) + (int32_t)row;
                const int32_t Px = 256 * px + 128, Py = 256 * py + 128;
                const int64_t e0 = (int64_t)s_A[0][lo] * Px + (int64_t)s_B[0][lo] * Py + s_C[0][lo];
                const int64_t e1 = (int64_t)s_A[1][lo] * Px + (int64_t)s_B[1][lo] * Py + s_C[1][lo];
                const int64_t e2 = (int64_t)s_A[2][lo] * Px + (int64_t)s_B[2][lo] * Py + s_C[2][lo];
                if (e0 > 0 && e1 > 0 && e2 > 0) {
                    ++frags;
                    const int own = wi >> 8;
                    const double inv = s_inv[lo];
                    const double be0 = (double)(e0 - (own & 1)) * inv;
                    const double be1 = (double)(e1 - ((own >> 1) & 1)) * inv;
                    const double be2 = (double)(e2 - ((own >> 2) & 1)) * inv;
                    double zd = be0 * (double)s_z[0][lo];
                    zd = zd + be1 * (double)s_z[1][lo];
                    zd = zd + be2 * (double)s_z[2][lo];
                    float z = (float)zd;
                    z = z + 0.0f;
                    if (0.0f <= z && z < 1.0f) {
                        const unsigned long long key =
                            ((unsigned long long)__float_as_uint(z) << 32) | (uint32_t)s_prim[lo];
                        atomicMin(&s_key[(py - py0) * B + (px - px0)], key);
                    }
                }
            }
            __syncthreads();
        }
        // EndBin: every fragment of this bin has been tested; resolve
        for (int i = tid; i < NPIX; i += TPB) {
            const int lx = i % B, ly = i / B;
            if (lx < pw && ly < ph)
                resolve_pixel(a, s, item_base, vbase, px0 + lx, py0 + ly, s_key[i]);
        }
        __syncthreads();
    }
    if (a.sh.frag_count) {
        // wave reduction, then one atomic per workgroup
        unsigned long long f = frags;
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) f += __shfl_down(f, d, kWave);
        if ((tid & (kWave - 1)) == 0) s_frag[tid / kWave] = f;
        __syncthreads();
        if (tid == 0) {
            unsigned long long tot = 0;
            for (int i = 0; i < TPB / kWave; ++i) tot += s_frag[i];
            if (tot) atomicAdd(a.sh.frag_count, tot);
        }
    }
    if (a.schedule == PK_SCHED_DYNAMIC && tid == 0) {
        // the last workgroup out rewinds the queue for the next launch
        __threadfence();
        const uint32_t done = atomicAdd(&a.w.misc[2], 1u);
        if (done == gridDim.x - 1) {
            for (int i = 0; i < kXcd; ++i) atomicExch(&a.w.misc[8 + i], 0u);
            atomicExch(&a.w.misc[2], 0u);
        }
    }
}

template <int TPB>
static hipError_t launch_tpb(const RasterArgs &a, dim3 grid, hipStream_t st) {
    switch (a.G.B) {
    case 8:  hipLaunchKernelGGL((k_raster<TPB, 8>), grid, dim3(TPB), 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_raster<TPB, 16>), grid, dim3(TPB), 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_raster<TPB, 32>), grid, dim3(TPB), 0, st, a); break;
    case 64: hipLaunchKernelGGL((k_raster<TPB, 64>), grid, dim3(TPB), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_raster(const Geom &G, const Ws &w, const Shade &sh, int schedule, int tpb,
                         int groups, hipStream_t st) {
    if (G.nbins_total == 0) return hipSuccess;
    RasterArgs a{G, w, sh, schedule};
    int64_t nblk = G.nbins_total;
    if (schedule != PK_SCHED_LOAD_BALANCE) nblk = groups < G.nbins_total ? groups : G.nbins_total;
    const dim3 grid((unsigned)nblk);
    switch (tpb) {
    case 64:  return launch_tpb<64>(a, grid, st);
    case 128: return launch_tpb<128>(a, grid, st);
    case 256: return launch_tpb<256>(a, grid, st);
    default:  return hipErrorInvalidValue;
    }
}

// Deferred shading pass over the G-buffer: colour = albedo * sum_l max(0, n.l).
__global__ __launch_bounds__(256) void k_deferred(Shade sh, int64_t npix) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= npix) return;
    if (sh.out_primid[p] < 0) {
        reinterpret_cast<float4 *>(sh.out_color)[p] = make_float4(0, 0, 0, 0);
        return;
    }
    const float n0 = sh.gbuf_n[3 * p], n1 = sh.gbuf_n[3 * p + 1], n2 = sh.gbuf_n[3 * p + 2];
    float lit = 0.0f;
    for (int l = 0; l < sh.num_lights; ++l) {
        const float *L = sh.lights + 3 * l;
        float d = n0 * L[0];
        d = d + n1 * L[1];
        d = d + n2 * L[2];
        d = d < 0.0f ? 0.0f : d;
        lit = (l == 0) ? d : lit + d;
    }
    reinterpret_cast<float4 *>(sh.out_color)[p] =
        make_float4(sh.gbuf_a[3 * p] * lit, sh.gbuf_a[3 * p + 1] * lit,
                    sh.gbuf_a[3 * p + 2] * lit, 1.0f);
}

hipError_t launch_deferred(const Geom &G, const Shade &sh, hipStream_t st) {
    const int64_t npix = (int64_t)G.S * G.W * G.H;
    if (npix == 0) return hipSuccess;
    hipLaunchKernelGGL(k_deferred, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, sh,
                       npix);
    return hipGetLastError();
}

}  // namespace pk
