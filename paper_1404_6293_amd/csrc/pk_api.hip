// pk_api.hip -- the C ABI of libpk (include/pk.h): host-side validation,
// workspace layout and kernel launches.  No allocation, no synchronization.
#include <algorithm>
#include <mutex>
#include <new>

#include "pk_internal.h"

namespace pk {

// The workspace of pk_render_static: one array per GPU, placed by the code
// object loader (no allocation call), held until the process ends.  In host
// code `scratch` names a host-side shadow, not device memory: its device
// address is taken once per device with hipGetSymbolAddress (with that
// device current) and only that address is ever handed to kernels.
__device__ __align__(256) unsigned char scratch[PK_STATIC_WORKSPACE_BYTES];

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool is_pow2_bin(int b) { return b == 8 || b == 16 || b == 32 || b == 64; }

int ilog2(int b) { int l = 0; while ((1 << l) < b) ++l; return l; }

// Host-side view of the parameters that every entry point shares.
struct Frame {
    int64_t items = 0;
    int64_t vrecs = 0;     // snapped vertex records (indexed meshes)
    bool indexed = false;
    int32_t layers = 0;    // order-independent transparency: key tiles per pixel
    int32_t split = 0;     // PK_SCHED_SPLIT with bins: pairs per work item
    int64_t npix = 0;      // S * W * H
    int64_t nbins_scene = 0;
    int64_t nbins_total = 0;
    int nbx = 0, nby = 0;
    bool fragbins = false; // PK_SCHED_FRAGMENT_BINS
    bool dynamic = false;  // PK_SCHED_DYNAMIC with bins: the bins' order
    bool two_level = false;                 // PK_FLAG_TWO_LEVEL_BINS
    int64_t nbins_f = 0;
    int nbx_c = 0, nby_c = 0;
    int32_t fb_groups = 0, fb_rounds = 0, fb_planes = 0;
};

pk_status check_params(const pk_params *p, Frame &f) {
    if (!p) return PK_ERR_INVALID_ARGUMENT;
    if (p->width < 1 || p->width > 8192 || p->height < 1 || p->height > 8192)
        return PK_ERR_INVALID_ARGUMENT;
    if (p->bin_size != 0 && !is_pow2_bin(p->bin_size)) return PK_ERR_INVALID_ARGUMENT;
    if (p->schedule < PK_SCHED_LOAD_BALANCE || p->schedule > PK_SCHED_FRAGMENT_BINS)
        return PK_ERR_INVALID_ARGUMENT;
    if (p->split_size < 0) return PK_ERR_INVALID_ARGUMENT;
    if (p->layers < 0 || p->layers > 8) return PK_ERR_INVALID_ARGUMENT;
    if (p->layers > 0) {
        if (p->flags & PK_FLAG_FUSE_RESOLVE) return PK_ERR_INVALID_ARGUMENT;
        if (p->shading != PK_SHADE_GOURAUD || p->bin_size == 0 || p->bin_size == 64 ||
            p->schedule == PK_SCHED_SPLIT)
            return PK_ERR_UNSUPPORTED;
    }
    // pieces of a bin merge in the workspace: no resolve inside the bin kernel
    if (p->schedule == PK_SCHED_SPLIT && (p->flags & PK_FLAG_FUSE_RESOLVE))
        return PK_ERR_INVALID_ARGUMENT;
    f.layers = p->layers;
    f.dynamic = p->schedule == PK_SCHED_DYNAMIC && p->bin_size != 0 && p->layers == 0;
    f.split = (p->schedule == PK_SCHED_SPLIT && p->bin_size != 0)
                  ? (p->split_size ? p->split_size : 256) : 0;
    if (p->threads_per_bin != 0 && p->threads_per_bin != 64 && p->threads_per_bin != 128 &&
        p->threads_per_bin != 256)
        return PK_ERR_INVALID_ARGUMENT;
    if (p->shading < PK_SHADE_GOURAUD || p->shading > PK_SHADE_LIT)
        return PK_ERR_INVALID_ARGUMENT;
    if (p->flags & ~(PK_FLAG_COUNT_FRAGS | PK_FLAG_FUSE_RESOLVE | PK_FLAG_DEFER_SHADE |
                     PK_FLAG_TWO_LEVEL_BINS))
        return PK_ERR_INVALID_ARGUMENT;
    if ((p->flags & PK_FLAG_TWO_LEVEL_BINS) &&
        ((p->bin_size != 8 && p->bin_size != 16) || p->layers != 0 ||
         (p->flags & PK_FLAG_FUSE_RESOLVE) ||
         (p->schedule != PK_SCHED_LOAD_BALANCE && p->schedule != PK_SCHED_DIRECT_MAP)))
        return PK_ERR_UNSUPPORTED;
    if ((p->flags & PK_FLAG_FUSE_RESOLVE) && (p->flags & PK_FLAG_DEFER_SHADE))
        return PK_ERR_INVALID_ARGUMENT;
    if (p->num_scenes < 1 || p->num_scenes > 65535) return PK_ERR_INVALID_ARGUMENT;
    if (p->instanced != 0 && p->instanced != 1) return PK_ERR_INVALID_ARGUMENT;
    if (p->persistent_groups < 0) return PK_ERR_INVALID_ARGUMENT;
    // bin size 0: one whole-screen bin per scene (Sec. 4.4)
    f.nbx = p->bin_size ? (p->width + p->bin_size - 1) / p->bin_size : 1;
    f.nby = p->bin_size ? (p->height + p->bin_size - 1) / p->bin_size : 1;
    f.nbins_scene = (int64_t)f.nbx * f.nby;
    if (p->flags & PK_FLAG_TWO_LEVEL_BINS) {
        // the coarse bins follow each scene's fine bins
        f.two_level = true;
        f.nbins_f = f.nbins_scene;
        f.nbx_c = (p->width + 4 * p->bin_size - 1) / (4 * p->bin_size);
        f.nby_c = (p->height + 4 * p->bin_size - 1) / (4 * p->bin_size);
        f.nbins_scene += (int64_t)f.nbx_c * f.nby_c;
    }
    f.nbins_total = f.nbins_scene * p->num_scenes;
    if (f.nbins_total >= (int64_t)INT32_MAX) return PK_ERR_INVALID_ARGUMENT;
    f.npix = (int64_t)p->num_scenes * p->width * p->height;
    if (f.npix > (int64_t)1 << 40) return PK_ERR_INVALID_ARGUMENT;
    if (p->schedule == PK_SCHED_FRAGMENT_BINS) {
        // one scene, opaque, the bins' counters in one workgroup's LDS
        if (p->bin_size < 16 || p->num_scenes != 1 || p->layers != 0 ||
            f.nbins_total > kFbMaxBins)
            return PK_ERR_UNSUPPORTED;
        f.fragbins = true;
        f.fb_planes = p->shading == PK_SHADE_DEFERRED ? 3 : 2;
    }
    // the per-pixel pass runs one workgroup per 64 x 4 tile
    if ((int64_t)p->num_scenes * ((p->width + 63) / 64) * ((p->height + 3) / 4) >=
        (int64_t)INT32_MAX)
        return PK_ERR_INVALID_ARGUMENT;
    return PK_OK;
}

pk_status check_mesh(const pk_params *p, const pk_mesh *m, Frame &f) {
    if (!m) return PK_ERR_INVALID_ARGUMENT;
    if (m->num_tris < 0 || m->num_vertices < 0) return PK_ERR_INVALID_ARGUMENT;
    if (m->num_tris > 0 && (!m->pos || m->num_vertices == 0)) return PK_ERR_INVALID_ARGUMENT;
    if (p->num_scenes > 1 && !p->instanced && (!m->scene_tri_off || !m->scene_vtx_off))
        return PK_ERR_INVALID_ARGUMENT;
    f.items = p->instanced ? (int64_t)m->num_tris * p->num_scenes : m->num_tris;
    if (f.items >= (int64_t)INT32_MAX) return PK_ERR_INVALID_ARGUMENT;
    f.indexed = m->indices != nullptr;
    f.vrecs = m->indices ? (int64_t)m->num_vertices * (p->instanced ? p->num_scenes : 1) : 0;
    if (f.fragbins) {
        // workgroups of fb_rounds rounds of 1024 triangles: about 1024 of
        // them (at least 256 when the scene allows), fewer when the bins are
        // many, so that the count matrix stays near 2^22 words
        const int64_t target = std::max<int64_t>(256, std::min<int64_t>(1024, ((int64_t)1 << 22) / f.nbins_total));
        const int64_t rounds = (f.items + kFbRoundTris * target - 1) / (kFbRoundTris * target);
        f.fb_rounds = (int32_t)std::max<int64_t>(1, rounds);
        const int64_t per = (int64_t)kFbRoundTris * f.fb_rounds;
        f.fb_groups = (int32_t)std::max<int64_t>(1, (f.items + per - 1) / per);
    }
    return PK_OK;
}

struct Layout {
    size_t vtx, rec, iw, bbox, fb_mat, bin_count, bin_off, vbin_off, order, cursor, misc, keys,
        pairs, total;
};

Layout layout(const Frame &f, int64_t pair_capacity) {
    Layout L;
    size_t o = 0;
    // fragment bins keep no per-triangle records, boxes or keys; their "pairs"
    // are fragments of fb_planes 16-byte planes
    const size_t tri = f.fragbins ? 0 : (size_t)f.items;
    L.vtx = o;       o = align_up(o + sizeof(VtxRec) * (size_t)f.vrecs);
    L.rec = o;       o = align_up(o + sizeof(TriRec) * tri);
    L.iw = o;        o = align_up(o + sizeof(float4) * (f.indexed ? 0 : tri));
    L.bbox = o;      o = align_up(o + sizeof(uint64_t) * tri);
    L.fb_mat = o;    o = align_up(o + sizeof(uint32_t) * (size_t)f.fb_groups * (size_t)(f.fragbins ? f.nbins_total : 0));
    // counters, cursors and misc words are adjacent so one clear covers them
    L.bin_count = o; o = align_up(o + sizeof(uint32_t) * (size_t)f.nbins_total);
    L.cursor = o;    o = align_up(o + sizeof(int32_t) * (size_t)f.nbins_total);
    L.misc = o;      o = align_up(o + sizeof(uint32_t) * kMiscWords);
    L.bin_off = o;   o = align_up(o + sizeof(int32_t) * (size_t)(f.nbins_total + 1));
    L.vbin_off = o;  o = align_up(o + sizeof(int32_t) * (size_t)(f.split ? f.nbins_total + 1 : 0));
    L.order = o;     o = align_up(o + sizeof(int32_t) * (size_t)(f.dynamic ? f.nbins_total : 0));
    L.keys = o;      o = align_up(o + sizeof(uint64_t) * (f.fragbins ? 0 : (size_t)f.npix * (size_t)(f.layers > 0 ? f.layers : 1)));
    L.pairs = o;     o = align_up(o + (f.fragbins ? 16 * (size_t)f.fb_planes * (size_t)((pair_capacity + 63) / 64 * 64)
                                                 : sizeof(int32_t) * (size_t)pair_capacity));
    L.total = o;
    return L;
}

// The pair list is the last slice: pair_capacity changes the total size
// only, so every call carves the same addresses.
Ws carve(void *ws, const Frame &f, int64_t pair_capacity) {
    const Layout L = layout(f, pair_capacity);
    char *b = static_cast<char *>(ws);
    Ws w;
    w.vtx = reinterpret_cast<VtxRec *>(b + L.vtx);
    w.rec = reinterpret_cast<TriRec *>(b + L.rec);
    w.iw = reinterpret_cast<float4 *>(b + L.iw);
    w.bbox = reinterpret_cast<uint64_t *>(b + L.bbox);
    w.bin_count = reinterpret_cast<uint32_t *>(b + L.bin_count);
    w.bin_off = reinterpret_cast<int32_t *>(b + L.bin_off);
    w.vbin_off = f.split ? reinterpret_cast<int32_t *>(b + L.vbin_off) : nullptr;
    w.order = f.dynamic ? reinterpret_cast<int32_t *>(b + L.order) : nullptr;
    w.split = f.split;
    w.cursor = reinterpret_cast<int32_t *>(b + L.cursor);
    w.keys = reinterpret_cast<unsigned long long *>(b + L.keys);
    w.misc = reinterpret_cast<uint32_t *>(b + L.misc);
    w.pairs = reinterpret_cast<int32_t *>(b + L.pairs);
    w.pair_capacity = pair_capacity;
    w.fb_mat = reinterpret_cast<uint32_t *>(b + L.fb_mat);
    w.fb_groups = f.fragbins ? f.fb_groups : 0;
    w.fb_rounds = f.fb_rounds;
    return w;
}

Geom geom(const pk_params *p, const pk_mesh *m, const Frame &f) {
    Geom G;
    G.pos = m->pos;
    G.V = m->num_vertices;
    G.idx = m->indices;
    G.T = m->num_tris;
    G.mvp = m->mvp;
    G.tri_off = m->scene_tri_off;
    G.vtx_off = m->scene_vtx_off;
    G.W = p->width;
    G.H = p->height;
    G.B = p->bin_size;
    G.log2B = ilog2(p->bin_size);
    G.nbx = f.nbx;
    G.nby = f.nby;
    G.nbins_scene = (int32_t)f.nbins_scene;
    G.S = p->num_scenes;
    G.instanced = (p->num_scenes > 1) ? p->instanced : 0;
    G.items = f.items;
    G.nbins_total = f.nbins_total;
    G.two_level = f.two_level ? 1 : 0;
    G.nbins_f = (int32_t)f.nbins_f;
    G.nbx_c = f.nbx_c;
    G.nby_c = f.nby_c;
    return G;
}

pk_status hip_status(hipError_t e) { return e == hipSuccess ? PK_OK : PK_ERR_HIP; }

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's array (nullptr on failure).
void *static_workspace(hipError_t &err) {
    int dev = -1;
    err = hipGetDevice(&dev);
    if (err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) { err = hipErrorInvalidDevice; return nullptr; }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (err != hipSuccess || !ptr) {
            if (err == hipSuccess) err = hipErrorInvalidSymbol;
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

// Validation shared by pk_raster_shade and pk_shade, and the kernels' view of
// the attributes and targets.
pk_status shade_args(const pk_params *p, const pk_attribs *a, const pk_targets *out,
                     const Frame &f, Shade &sh) {
    if (!a || !out) return PK_ERR_INVALID_ARGUMENT;
    if (f.items > 0 && !a->color) return PK_ERR_INVALID_ARGUMENT;
    if (p->shading == PK_SHADE_TEXTURED &&
        (!a->uv || !a->texture || a->tex_w < 1 || a->tex_h < 1))
        return PK_ERR_INVALID_ARGUMENT;
    if (p->shading == PK_SHADE_DEFERRED &&
        (!a->normal || !out->gbuf_normal || !out->gbuf_albedo || !out->primid || !out->color ||
         a->num_lights < 0 || (a->num_lights > 0 && !a->lights)))
        return PK_ERR_INVALID_ARGUMENT;
    if (p->shading == PK_SHADE_LIT &&
        (!a->normal || a->num_lights < 0 || (a->num_lights > 0 && !a->lights)))
        return PK_ERR_INVALID_ARGUMENT;
    if ((p->flags & PK_FLAG_COUNT_FRAGS) && !out->frag_count) return PK_ERR_INVALID_ARGUMENT;
    if (p->layers > 0 && !a->alpha) return PK_ERR_INVALID_ARGUMENT;
    sh = Shade{};
    sh.color = a->color; sh.uv = a->uv; sh.normal = a->normal; sh.texture = a->texture;
    sh.lights = a->lights; sh.tex_w = a->tex_w; sh.tex_h = a->tex_h;
    sh.num_lights = a->num_lights; sh.shading = p->shading;
    sh.out_color = out->color; sh.out_depth = out->depth; sh.out_bary = out->bary;
    sh.gbuf_n = p->shading == PK_SHADE_DEFERRED ? out->gbuf_normal : nullptr;
    sh.gbuf_a = p->shading == PK_SHADE_DEFERRED ? out->gbuf_albedo : nullptr;
    sh.out_primid = out->primid;
    sh.flags = p->flags;
    sh.frag_count = (p->flags & PK_FLAG_COUNT_FRAGS) ? out->frag_count : nullptr;
    sh.alpha = p->layers > 0 ? a->alpha : nullptr;
    sh.layers = p->layers;
    return PK_OK;
}

}  // namespace
}  // namespace pk

using namespace pk;

extern "C" {

size_t pk_workspace_bytes(const pk_params *p, const pk_mesh *m, int64_t pair_capacity) {
    Frame f;
    if (check_params(p, f) != PK_OK || check_mesh(p, m, f) != PK_OK || pair_capacity < 0 ||
        pair_capacity >= (int64_t)INT32_MAX)
        return 0;
    return layout(f, pair_capacity).total;
}

pk_status pk_setup(const pk_params *p, const pk_mesh *m, void *ws, void *stream) {
    Frame f;
    pk_status st = check_params(p, f);
    if (st != PK_OK) return st;
    if ((st = check_mesh(p, m, f)) != PK_OK) return st;
    if (!ws) return PK_ERR_INVALID_ARGUMENT;
    const Geom G = geom(p, m, f);
    return hip_status(launch_setup(G, carve(ws, f, 0), (hipStream_t)stream));
}

pk_status pk_assign_bin(const pk_params *p, const pk_mesh *m, void *ws, int64_t pair_capacity,
                        int64_t *pairs_needed, void *stream) {
    Frame f;
    pk_status st = check_params(p, f);
    if (st != PK_OK) return st;
    if ((st = check_mesh(p, m, f)) != PK_OK) return st;
    if (!ws || pair_capacity < 0 || pair_capacity >= (int64_t)INT32_MAX)
        return PK_ERR_INVALID_ARGUMENT;
    const Geom G = geom(p, m, f);
    const Ws w = carve(ws, f, pair_capacity);
    if (f.fragbins) return hip_status(launch_fb_assign(G, w, pairs_needed, (hipStream_t)stream));
    return hip_status(launch_assign(G, w, pairs_needed, (hipStream_t)stream));
}

pk_status pk_raster_shade(const pk_params *p, const pk_mesh *m, const pk_attribs *a, void *ws,
                          const pk_targets *out, void *stream) {
    Frame f;
    pk_status st = check_params(p, f);
    if (st != PK_OK) return st;
    if ((st = check_mesh(p, m, f)) != PK_OK) return st;
    if (!ws) return PK_ERR_INVALID_ARGUMENT;
    Shade sh;
    if ((st = shade_args(p, a, out, f, sh)) != PK_OK) return st;
    const Geom G = geom(p, m, f);
    // defaults: one wave per bin up to 16x16 bins (no cross-wave barriers),
    // and 16 resident waves per compute unit for the persistent schedules.
    // Transparency slots take LDS per workgroup: with 16x16 bins and more
    // layers, more waves share one bin's slots (measured on batches of
    // random triangles)
    int tpb = p->threads_per_bin;
    if (tpb == 0) tpb = p->bin_size <= 16 ? 64 : 256;
    if (p->threads_per_bin == 0 && p->bin_size == 16 && p->layers > 1)
        tpb = p->layers == 2 ? 128 : 256;
    int groups = p->persistent_groups;
    // persistent workgroups: 64 one-wave groups per CU (fewer measured
    // slower: 1080p grid bin kernel 31.5 us at 16,384 or 8,192, 32.5 at
    // 4,096, 45 at 2,048; batch256 with 16-px bins 0.74 / 0.75 / 0.78 ms)
    if (groups == 0) groups = 256 * 64 * kWave / tpb;
    const RasterMode mode = (p->flags & PK_FLAG_FUSE_RESOLVE) ? kRasterFused
                            : (p->flags & PK_FLAG_DEFER_SHADE) ? kRasterKeysOnly
                                                               : kRasterSplit;
    // the pair list is the last slice, so its address does not depend on the
    // capacity; the lists are read through bin_off only
    const Ws w = carve(ws, f, 0);
    if (f.fragbins) {
        const bool light = p->shading == PK_SHADE_DEFERRED && mode != kRasterKeysOnly;
        return hip_status(launch_fb_raster(G, w, sh, light, (hipStream_t)stream));
    }
    // transparency layers keep per-pixel LDS state for a whole bin (slots or
    // peeling passes): one workgroup per bin
    const int sched = p->layers > 0 ? PK_SCHED_LOAD_BALANCE : p->schedule;
    hipError_t e = launch_raster(G, w, sh, sched, tpb, groups, mode, (hipStream_t)stream);
    if (e == hipSuccess && mode != kRasterKeysOnly && p->shading == PK_SHADE_DEFERRED)
        e = launch_deferred(G, sh, (hipStream_t)stream);
    return hip_status(e);
}

pk_status pk_shade(const pk_params *p, const pk_mesh *m, const pk_attribs *a, void *ws,
                   const pk_targets *out, void *stream) {
    Frame f;
    pk_status st = check_params(p, f);
    if (st != PK_OK) return st;
    if ((st = check_mesh(p, m, f)) != PK_OK) return st;
    if (!ws || !(p->flags & PK_FLAG_DEFER_SHADE)) return PK_ERR_INVALID_ARGUMENT;
    Shade sh;
    if ((st = shade_args(p, a, out, f, sh)) != PK_OK) return st;
    sh.frag_count = nullptr;
    const Geom G = geom(p, m, f);
    const Ws w = carve(ws, f, 0);
    if (f.fragbins) {
        // the fragments were shaded before the depth test: only the
        // lighting of the deferred pass is left
        return hip_status(p->shading == PK_SHADE_DEFERRED ? launch_deferred(G, sh, (hipStream_t)stream)
                                                          : hipSuccess);
    }
    hipError_t e = launch_resolve_pass(G, w, sh, (hipStream_t)stream);
    if (e == hipSuccess && p->shading == PK_SHADE_DEFERRED)
        e = launch_deferred(G, sh, (hipStream_t)stream);
    return hip_status(e);
}

pk_status pk_backward(const pk_params *p, const pk_mesh *m, const pk_attribs *a,
                      const int32_t *primid, const float *bary, const float *grad_color,
                      float *grad_vcolor, float *grad_tex, void *stream) {
    Frame f;
    pk_status st = check_params(p, f);
    if (st != PK_OK) return st;
    if ((st = check_mesh(p, m, f)) != PK_OK) return st;
    if (p->shading == PK_SHADE_DEFERRED || p->shading == PK_SHADE_LIT || p->layers > 0)
        return PK_ERR_UNSUPPORTED;
    if (!a || !primid || !bary || !grad_color || !grad_vcolor || !a->color)
        return PK_ERR_INVALID_ARGUMENT;
    if (p->shading == PK_SHADE_TEXTURED &&
        (!a->uv || !a->texture || !grad_tex || a->tex_w < 1 || a->tex_h < 1))
        return PK_ERR_INVALID_ARGUMENT;
    const Geom G = geom(p, m, f);
    Shade sh{};
    sh.color = a->color; sh.uv = a->uv; sh.texture = a->texture;
    sh.tex_w = a->tex_w; sh.tex_h = a->tex_h; sh.shading = p->shading;
    return hip_status(launch_backward(G, sh, primid, bary, grad_color, grad_vcolor, grad_tex,
                                      (hipStream_t)stream));
}

pk_status pk_render_static(const pk_params *p, const pk_mesh *m, const pk_attribs *a,
                           const pk_targets *out, int64_t *pairs_needed, void *stream) {
    Frame f;
    pk_status st = check_params(p, f);
    if (st != PK_OK) return st;
    if ((st = check_mesh(p, m, f)) != PK_OK) return st;
    Shade sh;
    if ((st = shade_args(p, a, out, f, sh)) != PK_OK) return st;
    // every slice but the pair list must fit; the pairs take what is left
    const size_t fixed = layout(f, 0).total;
    if (fixed + kAlign > (size_t)PK_STATIC_WORKSPACE_BYTES) return PK_ERR_CAPACITY;
    int64_t cap = (int64_t)(((size_t)PK_STATIC_WORKSPACE_BYTES - fixed - kAlign) / sizeof(int32_t));
    if (cap >= (int64_t)INT32_MAX) cap = (int64_t)INT32_MAX - 1;
    hipError_t err = hipSuccess;
    void *ws = static_workspace(err);
    if (!ws) return PK_ERR_HIP;
    if ((st = pk_setup(p, m, ws, stream)) != PK_OK) return st;
    if ((st = pk_assign_bin(p, m, ws, cap, pairs_needed, stream)) != PK_OK) return st;
    if ((st = pk_raster_shade(p, m, a, ws, out, stream)) != PK_OK) return st;
    if (p->flags & PK_FLAG_DEFER_SHADE) st = pk_shade(p, m, a, ws, out, stream);
    return st;
}

pk_status pk_bin_lists(const pk_params *p, const pk_mesh *m, void *ws, pk_bin_view *out) {
    Frame f;
    pk_status st = check_params(p, f);
    if (st != PK_OK) return st;
    if ((st = check_mesh(p, m, f)) != PK_OK) return st;
    if (!ws || !out) return PK_ERR_INVALID_ARGUMENT;
    // whole-screen bins keep no lists; fragment bins hold fragments
    if (p->bin_size == 0 || p->schedule == PK_SCHED_FRAGMENT_BINS) return PK_ERR_UNSUPPORTED;
    const Ws w = carve(ws, f, 0);
    out->bin_offsets = w.bin_off;
    out->bin_tris = w.pairs;
    out->num_bins = f.nbins_total;
    return PK_OK;
}

const char *pk_status_string(pk_status s) {
    switch (s) {
    case PK_OK: return "ok";
    case PK_ERR_INVALID_ARGUMENT: return "invalid argument";
    case PK_ERR_CAPACITY: return "frame does not fit the static workspace";
    case PK_ERR_HIP: return "HIP runtime error";
    case PK_ERR_UNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

}  // extern "C"
