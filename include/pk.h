/*
 * pk.h -- C ABI of an MI355X (gfx950) spatially-binned software rasterizer.
 *
 * The library implements the sort-middle tiled renderer of Piko (Patney,
 * Tzeng, Seitz, Owens; Sec. 4.4 "Sort-Middle Tiled Renderer"): a geometry
 * phase with screen-sized bins (vertex transform and triangle setup), then a
 * screen-space phase with small square bins.  Each stage is split into the
 * paper's three phases (Sec. 4.1, Table "phases"):
 *
 *   pk_setup        vertex shader + rasterizer setup; the next stage's
 *                   AssignBin counts are produced in the same kernel
 *                   (Sec. 5.2, opening text: a kernel holds Schedule + Process of one
 *                   stage and AssignBin of the next).
 *   pk_assign_bin   AssignToBoundingBox (Sec. 4.3, directive table): a prefix
 *                   sum over the per-bin counts and a scatter into CSR bin
 *                   lists (Sec. 6, "Bin Management": prefix sums instead of
 *                   atomically appended lists).
 *   pk_raster_shade Schedule + Process of the per-bin stage: rasterizer and
 *                   depth test in one kernel per bin (the on-chip depth
 *                   buffer of Sec. 5.2.4 lives in LDS), then composite and
 *                   fragment shader either in a per-pixel pass over the
 *                   bins' winning keys or fused into the bin kernel
 *                   (Sec. 5.2.1 kernel fusion), then the deferred shading
 *                   pass when requested.
 *   pk_shade        the per-pixel composite + shading pass on its own, for
 *                   callers that split the frame (PK_FLAG_DEFER_SHADE).
 *
 * Variants selected by parameters: whole-screen bins (bin_size 0, the
 * unbinned pipeline), heavy bins split across workgroups (PK_SCHED_SPLIT)
 * and order-independent transparency (layers > 0: one pass keeping every
 * pixel's nearest keys in LDS, or depth peeling for 32-px bins beyond 3
 * layers).
 *   pk_backward     gradients of an image loss with respect to per-vertex
 *                   colours and texels (not in the paper).
 *
 * Calls follow the paper's statement of the problem: vertices, indices and
 * attributes in; colour, depth and primitive-ID buffers out; bin size and
 * schedule as parameters (Sec. 4.1 listing "kernels": Stage<binSizeX,
 * binSizeY, threadsPerBin, ...>; Sec. 4.3 Schedule directives).
 *
 * Conventions that hold for every entry point:
 *  - Pointers inside pk_mesh, pk_attribs and pk_targets, the workspace and
 *    every array argument are DEVICE pointers unless marked [host].  The
 *    pk_params / pk_mesh / pk_attribs / pk_targets structs themselves are
 *    [host] and read during the call only.
 *  - The caller owns all memory.  The library never allocates or frees
 *    device memory, keeps no device state between calls and never
 *    synchronizes: every call only enqueues kernels on `stream` (a
 *    hipStream_t; NULL is the default stream) and may be captured into a
 *    HIP graph.  Results are valid once the stream reaches them.
 *  - Arguments are validated on the host before anything is enqueued; an
 *    invalid call returns PK_ERR_INVALID_ARGUMENT (or PK_ERR_UNSUPPORTED)
 *    and leaves every buffer untouched.  A failed launch returns PK_ERR_HIP.
 *    No C++ exception crosses the ABI.
 *  - Pixels are row-major [H][W], row 0 at the bottom of the screen
 *    (NDC y = -1).  Batched outputs are [S][H][W].
 *
 * Fixed numeric conventions (the paper fixes none):
 *  - A vertex is transformed as clip = MVP * (x, y, z, 1) in float32 with
 *    each product rounded and the sums taken left to right (no fused
 *    multiply-add); NDC = clip * (1/w) with one correctly rounded reciprocal; screen = (ndc + 1) * (W/2, H/2); snapped
 *    to fixed point with 8 fractional bits, rounding half to even.  A
 *    triangle is dropped when a vertex has w <= 0, a non-finite value, or a
 *    screen coordinate outside (-16384, 16384) px, when its area is zero, or
 *    when no pixel centre lies inside its bounding box.  Both windings draw.
 *  - Pixel (x, y) is sampled at its centre.  Coverage uses exact integer
 *    edge functions with a top-left fill rule in y-up coordinates (an edge
 *    owns its samples when the interior lies to its right in +x, or below
 *    it for horizontal edges), so triangles sharing edges never double-cover.
 *  - Depth is z_ndc interpolated with float64 screen-space barycentrics and
 *    rounded to float32; fragments with z outside [0, 1) are discarded; the
 *    visible fragment is the one with the smallest (depth, triangle index)
 *    pair, i.e. a less-than test in submission order.  Results are therefore
 *    independent of bin size, schedule and batching, bit for bit.
 *  - Colours, UVs and normals are interpolated perspective-correctly in
 *    float32.  Empty pixels: colour 0, depth 1, primid -1, bary 0.
 */
#ifndef PK_H
#define PK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PK_OK = 0,
    PK_ERR_INVALID_ARGUMENT = 1, /* bad parameter; nothing was enqueued */
    PK_ERR_CAPACITY = 2,         /* pk_render_static only: the frame does not fit the
                                    library's static workspace (nothing was enqueued);
                                    pair overflow is reported on the device instead */
    PK_ERR_HIP = 3,              /* a HIP runtime call or launch failed */
    PK_ERR_UNSUPPORTED = 4       /* valid request this build does not implement */
} pk_status;

/* Schedule directives of the paper (Sec. 4.3 directive table; Sec. 6
 * "Work-Group Organization"). */
typedef enum {
    PK_SCHED_LOAD_BALANCE = 0, /* one workgroup per bin, hardware dispatcher balances */
    PK_SCHED_DIRECT_MAP = 1,   /* G persistent workgroups, bins pre-assigned to them */
    PK_SCHED_DYNAMIC = 2,      /* G persistent workgroups pop bins from device counters */
    PK_SCHED_SPLIT = 3,        /* heavy bins split (the All directive with a tile split
                                  size, Sec. 4.3): a bin with more than split_size pairs
                                  becomes several work items on different workgroups,
                                  whose depth tiles merge by device-scope 64-bit atomic
                                  min; G persistent workgroups take the work items */
    PK_SCHED_FRAGMENT_BINS = 4 /* bin fragments, not triangles: the Rasterizer and
                                  Fragment Shader run per triangle before any bin
                                  (one stage with whole-screen bins, fused as in
                                  Sec. 5.2.1), each shaded fragment goes to the bin
                                  of its pixel, and Depth Test + Composite run per
                                  bin in LDS.  For one scene (num_scenes 1), opaque,
                                  bins of 16, 32 or 64 px and at most 8192 bins per
                                  frame (else PK_ERR_UNSUPPORTED).  pk_setup counts
                                  each bin's fragments, pk_assign_bin takes their
                                  prefix sum (*pairs_needed receives the number of
                                  fragments, which pair_capacity bounds), and
                                  pk_raster_shade shades and scatters the fragments
                                  and then tests and composites every bin, writing
                                  every target; under PK_FLAG_DEFER_SHADE it leaves
                                  only the lighting of DEFERRED to pk_shade.
                                  threads_per_bin, persistent_groups and
                                  PK_FLAG_FUSE_RESOLVE are ignored */
} pk_schedule;

typedef enum {
    PK_SHADE_GOURAUD = 0,  /* colour = perspective-correct vertex colour */
    PK_SHADE_TEXTURED = 1, /* colour = Gouraud colour * bilinear texture(uv) */
    PK_SHADE_DEFERRED = 2, /* write G-buffer (unit normal, albedo), then
                              colour = albedo * sum_l max(0, n . l_l) */
    PK_SHADE_LIT = 3       /* forward lighting in the fragment shader itself:
                              colour = vertex colour * sum_l max(0, n . l_l) with
                              the unit interpolated normal n (the same value as
                              DEFERRED, without a G-buffer); needs normals and
                              lights, no G-buffer targets */
} pk_shading;

enum {
    PK_FLAG_COUNT_FRAGS = 1,  /* add the number of covered samples (before the
                                 depth test) to *targets.frag_count */
    PK_FLAG_FUSE_RESOLVE = 2, /* resolve and shade inside the per-bin kernel
                                 (Rasterizer and Fragment Shader fused, Sec. 7.2)
                                 instead of in a separate per-pixel pass over the
                                 bins' winning keys; the image is the same */
    PK_FLAG_DEFER_SHADE = 4,  /* pk_raster_shade stops after the depth test:
                                 every pixel's winning (depth, primitive) key
                                 goes to the depth and primid targets when both
                                 are given (they are then final), else to the
                                 workspace; pk_shade then resolves and shades.
                                 Excludes PK_FLAG_FUSE_RESOLVE. */
    PK_FLAG_TWO_LEVEL_BINS = 8 /* two bin sizes (hierarchical bins, the paper's
                                 non-uniform bins of Sec. 8): a triangle whose box
                                 spans more than 2 x 2 bins is assigned to coarse
                                 bins of four times bin_size instead of to the fine
                                 ones.  The fine bins are tested first, then each
                                 coarse bin starts from its pixels' keys and tests
                                 its own triangles; the per-pixel resolve follows.
                                 bin_size 8 or 16, LOAD_BALANCE or DIRECT_MAP,
                                 opaque, not fused (else PK_ERR_UNSUPPORTED).  The
                                 lists of pk_bin_lists then number each scene's
                                 fine bins first, then its coarse bins (row-major,
                                 ceil(W / (4 bin_size)) wide).  The image is the
                                 same */
};

typedef struct {               /* [host] */
    int32_t width, height;     /* 1..8192 pixels */
    int32_t bin_size;          /* screen-space bin edge: 8, 16, 32 or 64 pixels, or
                                  0 = one whole-screen bin per scene (the unbinned
                                  pipeline: no bin lists; each triangle is
                                  rasterized on its own with a device-scope
                                  depth test; schedule, threads_per_bin and
                                  persistent_groups are ignored) */
    int32_t schedule;          /* pk_schedule */
    int32_t threads_per_bin;   /* workgroup size for a bin: 64, 128, 256; 0 = auto
                                  (64 up to 16-px bins, else 256; with 16-px bins
                                  and 2 / 3+ transparency layers 128 / 256) */
    int32_t shading;           /* pk_shading */
    int32_t flags;             /* PK_FLAG_* */
    int32_t num_scenes;        /* S, 1..65535; S*W*H <= 2^40 pixels and
                                  S*ceil(W/64)*ceil(H/4) < 2^31 */
    int32_t instanced;         /* S > 1 only: 1 = S views (one MVP each) of the same
                                  mesh; 0 = S concatenated scenes (scene_*_off) */
    int32_t persistent_groups; /* DIRECT_MAP / DYNAMIC / SPLIT workgroup count; 0 = auto */
    int32_t split_size;        /* PK_SCHED_SPLIT: most (bin, triangle) pairs per work
                                  item, >= 1; 0 = 256.  Ignored by other schedules */
    int32_t layers;            /* 0 = opaque.  1..8 = order-independent transparency:
                                  every pixel composites its `layers` nearest fragments
                                  (smallest (depth, triangle) keys, the opaque test's
                                  keys), nearest first, with the per-vertex opacity
                                  pk_attribs.alpha:  T = 1, C = 0;  per fragment
                                  w = T*a, C += w*c, T = T*(1 - a);  colour = (C, 1 - T).
                                  Depth, primid and bary are the nearest fragment's.
                                  The paper's example of an EndBin between Depth Test
                                  and Composite (Sec. 5.2.3); the compositing rule is
                                  this library's.  Gouraud shading, 8/16/32-px bins,
                                  not SPLIT (else PK_ERR_UNSUPPORTED), not fused; the
                                  bins run one workgroup each (LOAD_BALANCE).  The bin
                                  kernel keeps each pixel's `layers` nearest keys in
                                  LDS in one pass, except 32-px bins with more than 3
                                  layers, which take one pass per layer */
} pk_params;

typedef struct {                 /* [host] struct of device pointers */
    const float *pos;            /* SoA [3][V] float32: x plane, y plane, z plane */
    int32_t num_vertices;        /* V over all scenes */
    const int32_t *indices;      /* [T][3] int32 (scene-local vertex numbers), or NULL:
                                    triangle t of a scene uses its vertices 3t, 3t+1, 3t+2 */
    int32_t num_tris;            /* T: all scenes (concatenated) or the one mesh (instanced) */
    const float *mvp;            /* [S][16] float32 row-major acting on column vectors
                                    (clip_r = sum_c m[4r+c] v_c), or NULL = identity */
    const int32_t *scene_tri_off;/* [S+1] first triangle of each scene; concatenated S > 1 only */
    const int32_t *scene_vtx_off;/* [S+1] first vertex of each scene;   concatenated S > 1 only */
} pk_mesh;

typedef struct {                 /* [host] struct of device pointers */
    const float *color;          /* [3][V] per-vertex RGB (albedo for DEFERRED) */
    const float *uv;             /* [2][V] texture coordinates, TEXTURED only */
    const float *normal;         /* [3][V] per-vertex normals, DEFERRED and LIT only */
    const float *texture;        /* [tex_h][tex_w][3] float32, TEXTURED only; texel
                                    centres at ((i+1/2)/tex_w, (j+1/2)/tex_h), clamp to edge */
    int32_t tex_w, tex_h;
    const float *lights;         /* [num_lights][3] unit directions, DEFERRED and LIT only */
    int32_t num_lights;
    const float *alpha;          /* [V] per-vertex opacity in [0, 1]; pk_params.layers > 0 only */
} pk_attribs;

typedef struct {                 /* [host] struct of device pointers; outputs [S][H][W](...) */
    float *color;                /* [..][4] RGBA float32, alpha 1 where covered */
    float *depth;                /* [..] float32 */
    int32_t *primid;             /* [..] scene-local triangle index, -1 where empty */
    float *bary;                 /* [..][2] perspective-correct (b1, b2), or NULL */
    float *gbuf_normal;          /* [..][3] unit normal; required for DEFERRED */
    float *gbuf_albedo;          /* [..][3] albedo;      required for DEFERRED */
    unsigned long long *frag_count; /* one counter (PK_FLAG_COUNT_FRAGS), accumulated */
} pk_targets;

/* Size in bytes of the workspace that pk_setup / pk_assign_bin /
 * pk_raster_shade share for one frame: snapped vertex records (indexed
 * meshes: V per view), per-triangle setup records and bounding boxes
 * (num_tris triangles, times S when instanced), per-bin counters and
 * offsets, one 64-bit key per output pixel, and room for pair_capacity
 * (bin, triangle) pairs.  Reads only the sizes and the indices pointer of
 * `m` [host struct].  Returns 0 for invalid parameters.  Host-only; no HIP
 * call. */
size_t pk_workspace_bytes(const pk_params *p, const pk_mesh *m, int64_t pair_capacity);

/* Vertex transform and triangle setup of every triangle (of every scene),
 * plus the per-bin triangle counts of AssignToBoundingBox.  Indexed meshes
 * first run the Vertex Shader once per vertex (per view), then setup gathers
 * the snapped vertices; unindexed ones transform in setup.  Writes the
 * workspace only.  With bin_size 0 there is nothing to count, and triangle
 * setup runs inside pk_raster_shade's per-triangle kernel instead (no setup
 * result goes through memory): this call then only runs the Vertex Shader
 * of indexed meshes and clears counters.  Sec. 7.1 stage list (Vertex
 * Shader, Rasterizer setup); Sec. 5.2 opening text, basic kernel mapping,
 * with setup fused into the next stage's kernel for whole-screen bins
 * (Sec. 5.2.1). */
pk_status pk_setup(const pk_params *p, const pk_mesh *m, void *ws, void *stream);

/* AssignToBoundingBox (Sec. 4.3): exclusive prefix sum of the per-bin counts
 * and scatter of triangle indices into CSR bin lists inside the workspace.
 * *pairs_needed (device, one int64) receives the total number of (bin,
 * triangle) pairs.  If it exceeds pair_capacity, no list is written and the
 * following pk_raster_shade writes empty pixels (colour 0, depth 1, primid -1,
 * bary 0) to every given target; call again with a larger workspace.  The order of triangles inside one bin is unspecified.
 * With PK_SCHED_SPLIT it also numbers the work items (each bin's list cut
 * into pieces of at most split_size pairs) for pk_raster_shade.
 * With bin_size 0 every scene is one bin that holds all of its triangles
 * (Sec. 4.4: full-screen bins need no assignment): nothing is built and
 * *pairs_needed receives 0. */
pk_status pk_assign_bin(const pk_params *p, const pk_mesh *m, void *ws, int64_t pair_capacity,
                        int64_t *pairs_needed, void *stream);

/* Schedule + Process of the screen-space stage for every bin of every scene:
 * coverage, depth test in an LDS-resident tile, resolve and shading, writing
 * every pixel of every target that is non-NULL (Sec. 4.4 sort-middle renderer;
 * Sec. 5.2.1 fusion of Rasterizer, Fragment Shader, Depth Test, Composite).
 * With PK_SHADE_DEFERRED the colour comes from a second pass over the
 * G-buffer.  Requires pk_setup and pk_assign_bin on the same workspace.
 * With bin_size 0 (whole-screen bins) one thread per triangle sets the
 * triangle up, covers its bounding box on the screen, and the depth test is
 * a device-scope 64-bit
 * atomic min into the workspace's key buffer (the paper's baseline with
 * full-screen bins, Sec. 7); the per-pixel resolve then always runs as its
 * own pass (also under PK_FLAG_FUSE_RESOLVE, since there is no per-bin EndBin),
 * and under PK_FLAG_DEFER_SHADE the keys stay in the workspace.  The image
 * is the same as with any bin size.  PK_SCHED_SPLIT likewise keeps the keys
 * in the workspace (pieces of one bin merge there) and resolves in a
 * per-pixel pass; it excludes PK_FLAG_FUSE_RESOLVE. */
pk_status pk_raster_shade(const pk_params *p, const pk_mesh *m, const pk_attribs *a, void *ws,
                          const pk_targets *out, void *stream);

/* Second half of a frame rendered with PK_FLAG_DEFER_SHADE: the Composite and
 * Fragment Shader stages as their own per-pixel pass (Sec. 7.1 stage list;
 * Sec. 5.2.1 discusses running them fused or apart).  Reads the winning keys
 * that pk_raster_shade left (in the depth and primid targets, or in `ws`),
 * resolves and shades every pixel, and
 * writes every non-NULL target exactly as a pk_raster_shade without the flag
 * would (frag_count is not touched).  `p` must carry PK_FLAG_DEFER_SHADE and
 * equal the parameters of the pk_raster_shade call; `m`, `a`, `ws` and the
 * depth and primid targets of `out` (or their absence) are the same.
 * Arguments are validated as for pk_raster_shade. */
pk_status pk_shade(const pk_params *p, const pk_mesh *m, const pk_attribs *a, void *ws,
                   const pk_targets *out, void *stream);

/* Backward pass of Gouraud (or textured) shading: from the forward's saved
 * primid and bary buffers and the upstream gradient grad_color [S][H][W][4]
 * (alpha ignored), ACCUMULATE dL/d(vertex colour) into grad_vcolor [3][V] and,
 * for TEXTURED, dL/d(texel) into grad_tex [tex_h][tex_w][3] (may be NULL
 * otherwise).  Coverage is not differentiated: nothing flows to positions,
 * UVs or alpha.  Summation order is unspecified (float32 atomics). */
pk_status pk_backward(const pk_params *p, const pk_mesh *m, const pk_attribs *a,
                      const int32_t *primid, const float *bary, const float *grad_color,
                      float *grad_vcolor, float *grad_tex, void *stream);

/* Where the CSR bin lists written by pk_assign_bin live inside `ws`, for
 * callers that consume or check them (AssignToBoundingBox, Sec. 4.3).
 * bin_offsets has num_bins + 1 entries (bins of scene s are numbered
 * s * bins_per_scene + by * ceil(W/bin_size) + bx); bin_tris holds the
 * triangle numbers (s * T + t for instanced views, the concatenated index
 * otherwise).  Host-only: computes addresses, launches nothing.  Returns
 * PK_ERR_UNSUPPORTED for bin_size 0 (whole-screen bins keep no lists). */
typedef struct {
    const int32_t *bin_offsets;  /* device */
    const int32_t *bin_tris;     /* device */
    int64_t num_bins;
} pk_bin_view;

pk_status pk_bin_lists(const pk_params *p, const pk_mesh *m, void *ws, pk_bin_view *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one whole
 * frame -- pk_setup, pk_assign_bin, pk_raster_shade and, with
 * PK_FLAG_DEFER_SHADE, pk_shade -- on a workspace the library owns instead
 * of a caller's `ws`.  That workspace is a static device array of
 * PK_STATIC_WORKSPACE_BYTES on every GPU the library runs on, placed when
 * the library's code is loaded there and held until the process ends; the
 * call itself allocates nothing (no hipMalloc, no allocating library
 * routine).  Every slice of the workspace but the bin-pair list must fit in
 * it, else PK_ERR_CAPACITY is returned and nothing is enqueued (see
 * pk_workspace_bytes with pair_capacity 0); the pair list takes the rest.
 * *pairs_needed (device, one int64, or NULL) receives the frame's pair count
 * as from pk_assign_bin; when the pairs outgrow the room left, the frame
 * writes empty pixels (colour 0, depth 1, primid -1, bary 0) to every given
 * target.  Arguments and results are otherwise those of the four calls.
 * All calls on one GPU share its array and it keeps the last frame's
 * contents (every frame clears what it needs): calls that overlap on one GPU
 * (several streams or host threads) race, and the caller must serialize
 * them. */
#define PK_STATIC_WORKSPACE_BYTES (64ull << 20)
pk_status pk_render_static(const pk_params *p, const pk_mesh *m, const pk_attribs *a,
                           const pk_targets *out, int64_t *pairs_needed, void *stream);

/* Static description of a status code.  Host-only. */
const char *pk_status_string(pk_status s);

#ifdef __cplusplus
}
#endif
#endif /* PK_H */
