/*
 * oracle.c -- plain, slow, single-threaded CPU reference of what the binned
 * raster pipeline computes.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) may include, link, import or call this file; only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg use it.  It
 * shares no code, header, table or constant with the HIP path.
 *
 * What it computes (Piko, Sec. 4.1 "AssignBin/Schedule/Process" and Sec. 4.4
 * "Sort-Middle Tiled Renderer"; stage list of the Baseline rasterizer in
 * Sec. 7.1): vertex transform, triangle setup, coverage, depth test and
 * Gouraud / textured / deferred shading.  The binning and scheduling phases of
 * the paper only regroup and reorder work (Sec. 4.1: AssignBin decides how
 * work is grouped, Schedule when and where it runs, Process what is computed),
 * so the image has a plain definition that uses no bins at all: for every
 * pixel sample, the nearest covering triangle.  This file is that definition.
 * The bin lists are produced separately (orc_assign_bin) only so the
 * AssignBin stage of the HIP path can be checked.
 *
 * The paper fixes none of the numeric conventions; the readings used here
 * (sample position, 8 sub-pixel bits with round-half-even snapping, the
 * top-left fill rule, the float64 barycentric depth, the (depth, primID)
 * tie-break, perspective-correct attributes, bilinear clamp-to-edge texturing,
 * the clamped Lambert deferred pass) are listed in the design notes.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC.  Contraction
 * must stay off: every float operation below is one IEEE-rounded operation,
 * evaluated in the order written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Inputs and outputs (plain arrays; all float planes are SoA [c][V]).      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t width, height;
    const float *pos;        /* [3][V] */
    int64_t num_vertices;    /* V */
    const int32_t *idx;      /* [T][3] or NULL (vertex 3t+k) */
    int64_t num_tris;        /* T */
    const float *mvp;        /* [16] row-major, or NULL (identity) */
    const float *color;      /* [3][V] */
    const float *uv;         /* [2][V] or NULL */
    const float *normal;     /* [3][V] or NULL */
    const float *texture;    /* [th][tw][3] or NULL */
    int32_t tex_w, tex_h;
    const float *lights;     /* [L][3] */
    int32_t num_lights;
    int32_t shading;         /* 0 gouraud, 1 textured, 2 deferred, 3 forward-lit */
} orc_scene;

typedef struct {
    float *color;            /* [H][W][4] */
    float *depth;            /* [H][W] */
    int32_t *primid;         /* [H][W] */
    float *bary;             /* [H][W][2] or NULL */
    float *gbuf_normal;      /* [H][W][3] or NULL */
    float *gbuf_albedo;      /* [H][W][3] or NULL */
    int32_t *cover_count;    /* [H][W] or NULL: samples covered, before z test */
    uint64_t *frag_count;    /* one value or NULL */
} orc_targets;

/* ------------------------------------------------------------------------ */
/* Step 1: per-vertex transform, perspective divide, viewport, snap.        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int valid;
    int32_t X, Y;            /* fixed point, 8 fractional bits */
    float z, iw;             /* NDC depth, 1/w */
} ovtx;

static ovtx vertex_stage(const orc_scene *s, int64_t v)
{
    const int64_t V = s->num_vertices;
    const float x = s->pos[v], y = s->pos[V + v], z = s->pos[2 * V + v];
    float c[4];
    if (s->mvp) {
        const float *m = s->mvp;
        for (int r = 0; r < 4; ++r) {
            float t = m[4 * r + 0] * x;
            t = t + m[4 * r + 1] * y;
            t = t + m[4 * r + 2] * z;
            t = t + m[4 * r + 3];
            c[r] = t;
        }
    } else {
        c[0] = x; c[1] = y; c[2] = z; c[3] = 1.0f;
    }
    ovtx o;
    memset(&o, 0, sizeof o);
    int ok = isfinite(c[0]) && isfinite(c[1]) && isfinite(c[2]) && isfinite(c[3]) && c[3] > 0.0f;
    /* one correctly rounded reciprocal of w, then products */
    const float iw = 1.0f / c[3];
    const float xn = c[0] * iw;
    const float yn = c[1] * iw;
    const float zn = c[2] * iw;
    const float xs = (xn + 1.0f) * (0.5f * (float)s->width);
    const float ys = (yn + 1.0f) * (0.5f * (float)s->height);
    ok = ok && isfinite(zn) && isfinite(iw);
    ok = ok && fabsf(xs) < 16384.0f && fabsf(ys) < 16384.0f;
    o.valid = ok;
    if (ok) {
        o.X = (int32_t)rintf(xs * 256.0f);   /* round half to even */
        o.Y = (int32_t)rintf(ys * 256.0f);
        o.z = zn;
        o.iw = iw;
    }
    return o;
}

/* ------------------------------------------------------------------------ */
/* Step 2: triangle setup.                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int live;
    int32_t X[3], Y[3];
    float z[3], iw[3];
    int64_t A2;              /* twice the signed area, 1/256 px units squared */
    int s;                   /* orientation sign */
    int32_t bx0, bx1, by0, by1; /* inclusive pixel bbox of covered-candidate samples */
    int64_t vid[3];
} otri;

static int64_t floor_div256(int64_t a)
{
    return (a >= 0) ? (a / 256) : -((-a + 255) / 256);
}

static int64_t vertex_id(const orc_scene *s, int64_t t, int k)
{
    return s->idx ? (int64_t)s->idx[3 * t + k] : 3 * t + k;
}

static otri setup_stage(const orc_scene *s, int64_t t)
{
    otri r;
    memset(&r, 0, sizeof r);
    int valid = 1;
    for (int k = 0; k < 3; ++k) {
        r.vid[k] = vertex_id(s, t, k);
        if (r.vid[k] < 0 || r.vid[k] >= s->num_vertices) { valid = 0; continue; }
        ovtx v = vertex_stage(s, r.vid[k]);
        valid = valid && v.valid;
        r.X[k] = v.X; r.Y[k] = v.Y; r.z[k] = v.z; r.iw[k] = v.iw;
    }
    if (!valid) return r;
    r.A2 = (int64_t)(r.X[1] - r.X[0]) * (int64_t)(r.Y[2] - r.Y[0])
         - (int64_t)(r.X[2] - r.X[0]) * (int64_t)(r.Y[1] - r.Y[0]);
    if (r.A2 == 0) return r;
    r.s = r.A2 > 0 ? 1 : -1;
    int32_t mnx = r.X[0], mxx = r.X[0], mny = r.Y[0], mxy = r.Y[0];
    for (int k = 1; k < 3; ++k) {
        if (r.X[k] < mnx) mnx = r.X[k];
        if (r.X[k] > mxx) mxx = r.X[k];
        if (r.Y[k] < mny) mny = r.Y[k];
        if (r.Y[k] > mxy) mxy = r.Y[k];
    }
    /* pixel p is sampled at 256p+128: smallest p with 256p+128 >= min,
     * largest p with 256p+128 <= max */
    int64_t x0 = floor_div256((int64_t)mnx - 128 + 255);
    int64_t x1 = floor_div256((int64_t)mxx - 128);
    int64_t y0 = floor_div256((int64_t)mny - 128 + 255);
    int64_t y1 = floor_div256((int64_t)mxy - 128);
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > s->width - 1) x1 = s->width - 1;
    if (y1 > s->height - 1) y1 = s->height - 1;
    if (x0 > x1 || y0 > y1) return r;   /* no sample inside the bbox */
    r.bx0 = (int32_t)x0; r.bx1 = (int32_t)x1; r.by0 = (int32_t)y0; r.by1 = (int32_t)y1;
    r.live = 1;
    return r;
}

/* ------------------------------------------------------------------------ */
/* Step 4: coverage with the top-left rule (y up: top = larger y).          */
/* Edge k is the edge opposite vertex k, directed v1->v2, v2->v0, v0->v1.   */
/* ------------------------------------------------------------------------ */
static void edge_values(const otri *r, int64_t Px, int64_t Py, int64_t E[3])
{
    static const int a_of[3] = {1, 2, 0};
    static const int b_of[3] = {2, 0, 1};
    for (int k = 0; k < 3; ++k) {
        const int a = a_of[k], b = b_of[k];
        const int64_t dx = (int64_t)r->X[b] - r->X[a];
        const int64_t dy = (int64_t)r->Y[b] - r->Y[a];
        E[k] = dx * (Py - r->Y[a]) - dy * (Px - r->X[a]);
    }
}

static int covers(const otri *r, const int64_t E[3])
{
    static const int a_of[3] = {1, 2, 0};
    static const int b_of[3] = {2, 0, 1};
    for (int k = 0; k < 3; ++k) {
        const int64_t e = r->s * E[k];
        if (e > 0) continue;
        if (e < 0) return 0;
        const int64_t dx = (int64_t)r->X[b_of[k]] - r->X[a_of[k]];
        const int64_t dy = (int64_t)r->Y[b_of[k]] - r->Y[a_of[k]];
        const int owned = (r->s * dy < 0) || (dy == 0 && r->s * dx < 0);
        if (!owned) return 0;
    }
    return 1;
}

/* Step 5: screen-linear depth through float64 barycentrics. */
static void barycentrics64(const otri *r, const int64_t E[3], double beta[3])
{
    const int64_t a = r->s * r->A2;          /* > 0 */
    const double inv = 1.0 / (double)a;
    for (int k = 0; k < 3; ++k) beta[k] = (double)(r->s * E[k]) * inv;
}

static float depth_of(const otri *r, const double beta[3])
{
    double zd = beta[0] * (double)r->z[0];
    zd = zd + beta[1] * (double)r->z[1];
    zd = zd + beta[2] * (double)r->z[2];
    float z = (float)zd;
    z = z + 0.0f;                            /* -0 -> +0 */
    return z;
}

static uint32_t float_bits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float bits_float(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* ------------------------------------------------------------------------ */
/* Shading helpers (step 7).                                                */
/* ------------------------------------------------------------------------ */
static void persp_bary(const otri *r, const double beta[3], float bp[3])
{
    const float bs0 = (float)beta[0], bs1 = (float)beta[1], bs2 = (float)beta[2];
    const float q0 = bs0 * r->iw[0];
    const float q1 = bs1 * r->iw[1];
    const float q2 = bs2 * r->iw[2];
    const float Q = (q0 + q1) + q2;
    bp[1] = q1 / Q;
    bp[2] = q2 / Q;
    bp[0] = (1.0f - bp[1]) - bp[2];
}

static float interp(const float *plane, const int64_t vid[3], const float bp[3])
{
    float t = bp[0] * plane[vid[0]];
    t = t + bp[1] * plane[vid[1]];
    t = t + bp[2] * plane[vid[2]];
    return t;
}

/* Bilinear, texel centres at (i+1/2)/N, clamp to edge; row j follows v. */
typedef struct { int64_t texel[4]; float w[4]; } otap;

static otap bilinear_taps(const orc_scene *s, float u, float v)
{
    otap o;
    const float su = u * (float)s->tex_w - 0.5f;
    const float sv = v * (float)s->tex_h - 0.5f;
    const float fi = floorf(su), fj = floorf(sv);
    const float fs = su - fi, ft = sv - fj;
    /* clamping the float index first only avoids an out-of-range conversion;
     * every tap beyond an edge lands on that edge either way */
    const float ci = fminf(fmaxf(fi, -1.0f), (float)s->tex_w);
    const float cj = fminf(fmaxf(fj, -1.0f), (float)s->tex_h);
    int64_t i0 = (int64_t)ci, j0 = (int64_t)cj;
    int64_t i1 = i0 + 1, j1 = j0 + 1;
    const int64_t wmax = s->tex_w - 1, hmax = s->tex_h - 1;
    if (i0 < 0) i0 = 0; if (i0 > wmax) i0 = wmax;
    if (i1 < 0) i1 = 0; if (i1 > wmax) i1 = wmax;
    if (j0 < 0) j0 = 0; if (j0 > hmax) j0 = hmax;
    if (j1 < 0) j1 = 0; if (j1 > hmax) j1 = hmax;
    o.texel[0] = j0 * s->tex_w + i0;
    o.texel[1] = j0 * s->tex_w + i1;
    o.texel[2] = j1 * s->tex_w + i0;
    o.texel[3] = j1 * s->tex_w + i1;
    o.w[0] = (1.0f - fs) * (1.0f - ft);
    o.w[1] = fs * (1.0f - ft);
    o.w[2] = (1.0f - fs) * ft;
    o.w[3] = fs * ft;
    return o;
}

static float sample_channel(const orc_scene *s, const otap *tp, int c)
{
    float t = tp->w[0] * s->texture[3 * tp->texel[0] + c];
    t = t + tp->w[1] * s->texture[3 * tp->texel[1] + c];
    t = t + tp->w[2] * s->texture[3 * tp->texel[2] + c];
    t = t + tp->w[3] * s->texture[3 * tp->texel[3] + c];
    return t;
}

/* ------------------------------------------------------------------------ */
/* Public entry points                                                      */
/* ------------------------------------------------------------------------ */

/* Per-vertex stage, for checking the snap against closed forms. */
int orc_vertices(const orc_scene *s, int32_t *X, int32_t *Y, float *z, float *iw, uint8_t *valid)
{
    for (int64_t v = 0; v < s->num_vertices; ++v) {
        ovtx o = vertex_stage(s, v);
        X[v] = o.X; Y[v] = o.Y; z[v] = o.z; iw[v] = o.iw; valid[v] = (uint8_t)o.valid;
    }
    return 0;
}

/* Per-triangle setup: live flag, inclusive pixel bbox [T][4] = x0,x1,y0,y1, A2. */
int orc_setup(const orc_scene *s, uint8_t *live, int32_t *bbox, int64_t *A2)
{
    for (int64_t t = 0; t < s->num_tris; ++t) {
        otri r = setup_stage(s, t);
        live[t] = (uint8_t)r.live;
        bbox[4 * t + 0] = r.bx0; bbox[4 * t + 1] = r.bx1;
        bbox[4 * t + 2] = r.by0; bbox[4 * t + 3] = r.by1;
        A2[t] = r.A2;
    }
    return 0;
}

/*
 * AssignToBoundingBox (Sec. 4.3, directive table): every bin that the
 * triangle's sample bbox overlaps.  Bins are bin_size x bin_size pixels,
 * numbered row-major, ceil(W/B) per row; bin_size 0 means one bin covering
 * the whole screen (Sec. 4.4 "No Tiling").  Lists are ascending in t.
 * Writes bin_off[nbins+1]; writes bin_tris when it is non-NULL and the total
 * fits in cap.  Returns the total number of (bin, triangle) pairs.
 */
int64_t orc_assign_bin(const orc_scene *s, int32_t bin_size, int32_t *bin_off,
                       int32_t *bin_tris, int64_t cap)
{
    const int W = s->width, H = s->height;
    const int bw = bin_size > 0 ? bin_size : W;
    const int bh = bin_size > 0 ? bin_size : H;
    const int nbx = (W + bw - 1) / bw, nby = (H + bh - 1) / bh;
    const int64_t nbins = (int64_t)nbx * nby;
    int64_t *cnt = calloc((size_t)nbins, sizeof(int64_t));
    otri *tr = malloc(sizeof(otri) * (size_t)(s->num_tris > 0 ? s->num_tris : 1));
    if (!cnt || !tr) { free(cnt); free(tr); return -1; }
    for (int64_t t = 0; t < s->num_tris; ++t) {
        tr[t] = setup_stage(s, t);
        if (!tr[t].live) continue;
        for (int by = tr[t].by0 / bh; by <= tr[t].by1 / bh; ++by)
            for (int bx = tr[t].bx0 / bw; bx <= tr[t].bx1 / bw; ++bx)
                cnt[(int64_t)by * nbx + bx] += 1;
    }
    int64_t total = 0;
    for (int64_t b = 0; b < nbins; ++b) { bin_off[b] = (int32_t)total; total += cnt[b]; }
    bin_off[nbins] = (int32_t)total;
    if (bin_tris && total <= cap) {
        for (int64_t b = 0; b < nbins; ++b) cnt[b] = bin_off[b];
        for (int64_t t = 0; t < s->num_tris; ++t) {
            if (!tr[t].live) continue;
            for (int by = tr[t].by0 / bh; by <= tr[t].by1 / bh; ++by)
                for (int bx = tr[t].bx0 / bw; bx <= tr[t].bx1 / bw; ++bx)
                    bin_tris[cnt[(int64_t)by * nbx + bx]++] = (int32_t)t;
        }
    }
    free(cnt);
    free(tr);
    return total;
}

/*
 * The image: for every pixel sample the covering triangle with the smallest
 * 64-bit key (depth bits << 32 | triangle index) among fragments with
 * 0 <= z < 1, then the shading of that winner.
 */
/*
 * Steps 2, 4, 5 and 6 for the triangles [t0, t1) and the pixel rows
 * [row0, row1): every sample of every such triangle's bbox in those rows,
 * its key min-ed into zbuf (pixel p at zbuf[p - row0 * W], which the caller
 * fills with all ones), covered samples added to *frags and, when given,
 * cover_count (pixel p at cover_count[p]).
 */
static void depth_keys(const orc_scene *s, int64_t t0, int64_t t1, int32_t row0, int32_t row1,
                       uint64_t *zbuf, int32_t *cover_count, uint64_t *frags)
{
    const int W = s->width;
    const int64_t base = (int64_t)row0 * W;
    uint64_t n = 0;
    for (int64_t t = t0; t < t1; ++t) {
        otri r = setup_stage(s, t);
        if (!r.live) continue;
        const int y0 = r.by0 > row0 ? r.by0 : row0;
        const int y1 = r.by1 < row1 - 1 ? r.by1 : row1 - 1;
        for (int py = y0; py <= y1; ++py) {
            for (int px = r.bx0; px <= r.bx1; ++px) {
                const int64_t Px = 256 * (int64_t)px + 128, Py = 256 * (int64_t)py + 128;
                int64_t E[3];
                edge_values(&r, Px, Py, E);
                if (!covers(&r, E)) continue;
                const int64_t p = (int64_t)py * W + px;
                n += 1;
                if (cover_count) cover_count[p] += 1;
                double beta[3];
                barycentrics64(&r, E, beta);
                const float z = depth_of(&r, beta);
                if (!(0.0f <= z && z < 1.0f)) continue;
                const uint64_t key = ((uint64_t)float_bits(z) << 32) | (uint32_t)t;
                if (key < zbuf[p - base]) zbuf[p - base] = key;
            }
        }
    }
    *frags += n;
}

/*
 * Step 7 for the pixel rows [row0, row1) from their finished keys (pixel p
 * at zbuf[p - row0 * W]): resolve and shade every pixel, writing every
 * target of o.
 */
static void resolve_rows(const orc_scene *s, const uint64_t *zbuf, const orc_targets *o,
                         int32_t row0, int32_t row1)
{
    const int W = s->width;
    const int64_t base = (int64_t)row0 * W;
    /* step 7: resolve and shade every pixel */
    for (int py = row0; py < row1; ++py) {
        for (int px = 0; px < W; ++px) {
            const int64_t p = (int64_t)py * W + px;
            const uint64_t kp = zbuf[p - base];
            float *col = o->color ? o->color + 4 * p : NULL;
            if (kp == ~0ull) {
                if (col) col[0] = col[1] = col[2] = col[3] = 0.0f;
                if (o->depth) o->depth[p] = 1.0f;
                if (o->primid) o->primid[p] = -1;
                if (o->bary) o->bary[2 * p] = o->bary[2 * p + 1] = 0.0f;
                if (o->gbuf_normal) o->gbuf_normal[3 * p] = o->gbuf_normal[3 * p + 1] = o->gbuf_normal[3 * p + 2] = 0.0f;
                if (o->gbuf_albedo) o->gbuf_albedo[3 * p] = o->gbuf_albedo[3 * p + 1] = o->gbuf_albedo[3 * p + 2] = 0.0f;
                continue;
            }
            const int64_t t = (int64_t)(kp & 0xffffffffull);
            const float z = bits_float((uint32_t)(kp >> 32));
            otri r = setup_stage(s, t);
            int64_t E[3];
            edge_values(&r, 256 * (int64_t)px + 128, 256 * (int64_t)py + 128, E);
            double beta[3];
            barycentrics64(&r, E, beta);
            float bp[3];
            persp_bary(&r, beta, bp);
            const int64_t V = s->num_vertices;
            float rgb[3];
            for (int c = 0; c < 3; ++c) rgb[c] = interp(s->color + c * V, r.vid, bp);
            if (s->shading == 1) {
                const float u = interp(s->uv, r.vid, bp);
                const float v = interp(s->uv + V, r.vid, bp);
                otap tp = bilinear_taps(s, u, v);
                for (int c = 0; c < 3; ++c) rgb[c] = rgb[c] * sample_channel(s, &tp, c);
            }
            if (s->shading == 2 || s->shading == 3) {
                /* deferred (2) writes the G-buffer and lights it in a second
                 * pass; forward-lit (3) lights the same unit normal and albedo
                 * in the fragment shader itself.  Either way the colour is
                 * albedo * sum over the lights of max(0, n.l). */
                float n[3];
                for (int c = 0; c < 3; ++c) n[c] = interp(s->normal + c * V, r.vid, bp);
                float nn = n[0] * n[0];
                nn = nn + n[1] * n[1];
                nn = nn + n[2] * n[2];
                float nh[3] = {0.0f, 0.0f, 0.0f};
                if (nn != 0.0f) {
                    const float len = sqrtf(nn);
                    for (int c = 0; c < 3; ++c) nh[c] = n[c] / len;
                }
                if (o->gbuf_normal) for (int c = 0; c < 3; ++c) o->gbuf_normal[3 * p + c] = nh[c];
                if (o->gbuf_albedo) for (int c = 0; c < 3; ++c) o->gbuf_albedo[3 * p + c] = rgb[c];
                /* lighting: albedo * sum_l max(0, n.l), lights in the given order */
                float lit = 0.0f;
                for (int l = 0; l < s->num_lights; ++l) {
                    const float *L = s->lights + 3 * l;
                    float d = nh[0] * L[0];
                    d = d + nh[1] * L[1];
                    d = d + nh[2] * L[2];
                    if (d < 0.0f) d = 0.0f;
                    lit = (l == 0) ? d : lit + d;
                }
                for (int c = 0; c < 3; ++c) rgb[c] = rgb[c] * lit;
            }
            if (col) { col[0] = rgb[0]; col[1] = rgb[1]; col[2] = rgb[2]; col[3] = 1.0f; }
            if (o->depth) o->depth[p] = z;
            if (o->primid) o->primid[p] = (int32_t)t;
            if (o->bary) { o->bary[2 * p] = bp[1]; o->bary[2 * p + 1] = bp[2]; }
        }
    }
}

/*
 * The same definition for the pixel rows [row0, row1) only: every pixel is
 * computed on its own, so rendering the rows in disjoint bands (for instance
 * one band per host thread) gives the whole image bit for bit.  Writes the
 * band's rows of every target; *frag_count receives the band's covered
 * samples.
 */
int orc_render_rows(const orc_scene *s, const orc_targets *o, int32_t row0, int32_t row1)
{
    const int W = s->width, H = s->height;
    if (row0 < 0) row0 = 0;
    if (row1 > H) row1 = H;
    if (row1 < row0) row1 = row0;
    const int64_t base = (int64_t)row0 * W;           /* first pixel of the band */
    const int64_t npx = (int64_t)(row1 - row0) * W;
    uint64_t *zbuf = malloc(sizeof(uint64_t) * (size_t)(npx > 0 ? npx : 1));
    if (!zbuf) return -1;
    for (int64_t p = 0; p < npx; ++p) zbuf[p] = ~0ull;
    if (o->cover_count) memset(o->cover_count + base, 0, sizeof(int32_t) * (size_t)npx);
    uint64_t frags = 0;
    depth_keys(s, 0, s->num_tris, row0, row1, zbuf, o->cover_count, &frags);
    if (o->frag_count) *o->frag_count = frags;
    resolve_rows(s, zbuf, o, row0, row1);
    free(zbuf);
    return 0;
}

/*
 * The depth test is a minimum over keys, so it can be split over the
 * triangles as well: orc_depth_keys takes the triangles [t0, t1) over the
 * whole screen into zbuf [H][W] (all ones beforehand), adding their covered
 * samples to *frag_count and cover_count [H][W] (either may be NULL); the
 * element-wise minimum of several ranges' buffers is the whole scene's, and
 * orc_resolve_rows then shades any band of rows from it.  Together they
 * give orc_render's image bit for bit.
 */
int orc_depth_keys(const orc_scene *s, int64_t t0, int64_t t1, uint64_t *zbuf,
                   int32_t *cover_count, uint64_t *frag_count)
{
    if (t0 < 0) t0 = 0;
    if (t1 > s->num_tris) t1 = s->num_tris;
    uint64_t frags = 0;
    depth_keys(s, t0, t1, 0, s->height, zbuf, cover_count, &frags);
    if (frag_count) *frag_count += frags;
    return 0;
}

int orc_resolve_rows(const orc_scene *s, const uint64_t *zbuf, const orc_targets *o,
                     int32_t row0, int32_t row1)
{
    if (row0 < 0) row0 = 0;
    if (row1 > s->height) row1 = s->height;
    if (row1 <= row0) return 0;
    resolve_rows(s, zbuf + (int64_t)row0 * s->width, o, row0, row1);
    return 0;
}

int orc_render(const orc_scene *s, const orc_targets *o)
{
    return orc_render_rows(s, o, 0, s->height);
}

/*
 * Order-independent transparency (the paper's example of an EndBin between
 * Depth Test and Composite; the compositing rule is this project's reading):
 * every pixel keeps the K fragments with the smallest (depth, triangle) keys
 * -- the same keys and range test as the opaque depth test -- and composites
 * them nearest first with per-vertex opacity `alpha` [V], interpolated like
 * the colours:
 *   T = 1, C = 0;  for each kept fragment j, nearest first:
 *     a = alpha_j;  w = T * a;  C_c = C_c + w * c_jc;  T = T * (1 - a)
 *   colour = (C_0, C_1, C_2, 1 - T).
 * Depth, primid and bary are those of the nearest fragment; an empty pixel is
 * as in orc_render.  Gouraud colours only.  color [H][W][4]; depth, primid,
 * bary may be NULL.
 */
int orc_render_oit(const orc_scene *s, const float *alpha, int32_t K, float *color, float *depth,
                   int32_t *primid, float *bary)
{
    const int W = s->width, H = s->height;
    const int64_t npx = (int64_t)W * H;
    if (K < 1) return -1;
    uint64_t *keys = malloc(sizeof(uint64_t) * (size_t)(npx > 0 ? npx : 1) * (size_t)K);
    if (!keys) return -1;
    for (int64_t i = 0; i < npx * K; ++i) keys[i] = ~0ull;

    /* every triangle in submission order, every sample of its bbox: insert
     * the key into the pixel's ascending list of the K smallest */
    for (int64_t t = 0; t < s->num_tris; ++t) {
        otri r = setup_stage(s, t);
        if (!r.live) continue;
        for (int py = r.by0; py <= r.by1; ++py) {
            for (int px = r.bx0; px <= r.bx1; ++px) {
                int64_t E[3];
                edge_values(&r, 256 * (int64_t)px + 128, 256 * (int64_t)py + 128, E);
                if (!covers(&r, E)) continue;
                double beta[3];
                barycentrics64(&r, E, beta);
                const float z = depth_of(&r, beta);
                if (!(0.0f <= z && z < 1.0f)) continue;
                uint64_t key = ((uint64_t)float_bits(z) << 32) | (uint32_t)t;
                uint64_t *list = keys + ((int64_t)py * W + px) * K;
                for (int j = 0; j < K; ++j) {
                    if (key < list[j]) { const uint64_t tmp = list[j]; list[j] = key; key = tmp; }
                }
            }
        }
    }

    const int64_t V = s->num_vertices;
    for (int py = 0; py < H; ++py) {
        for (int px = 0; px < W; ++px) {
            const int64_t p = (int64_t)py * W + px;
            const uint64_t *list = keys + p * K;
            float C[3] = {0.0f, 0.0f, 0.0f};
            float T = 1.0f;
            if (list[0] == ~0ull) {
                if (depth) depth[p] = 1.0f;
                if (primid) primid[p] = -1;
                if (bary) bary[2 * p] = bary[2 * p + 1] = 0.0f;
            }
            for (int j = 0; j < K && list[j] != ~0ull; ++j) {
                const int64_t t = (int64_t)(list[j] & 0xffffffffull);
                otri r = setup_stage(s, t);
                int64_t E[3];
                edge_values(&r, 256 * (int64_t)px + 128, 256 * (int64_t)py + 128, E);
                double beta[3];
                barycentrics64(&r, E, beta);
                float bp[3];
                persp_bary(&r, beta, bp);
                const float a = interp(alpha, r.vid, bp);
                const float w = T * a;
                for (int c = 0; c < 3; ++c) C[c] = C[c] + w * interp(s->color + c * V, r.vid, bp);
                T = T * (1.0f - a);
                if (j == 0) {
                    if (depth) depth[p] = bits_float((uint32_t)(list[0] >> 32));
                    if (primid) primid[p] = (int32_t)t;
                    if (bary) { bary[2 * p] = bp[1]; bary[2 * p + 1] = bp[2]; }
                }
            }
            float *col = color + 4 * p;
            col[0] = C[0]; col[1] = C[1]; col[2] = C[2];
            col[3] = list[0] == ~0ull ? 0.0f : 1.0f - T;
        }
    }
    free(keys);
    return 0;
}

/*
 * Reference gradient of an image loss with respect to the per-vertex colours
 * and the texels, given the forward's primid and bary buffers and the
 * upstream gradient G[H][W][4] (alpha ignored).  float64 accumulation in
 * pixel-major order.  Coverage is not differentiated: nothing flows to
 * positions, UVs or alpha.
 *   untextured: dC[v_k][c] += b'_k G_c
 *   textured:   dC[v_k][c] += b'_k G_c T_c ;  dTex[j][c] += w_j G_c Cint_c
 * grad_vcolor is [3][V] and grad_tex [th][tw][3]; both are accumulated.
 */
int orc_backward(const orc_scene *s, const int32_t *primid, const float *bary,
                 const float *grad, double *grad_vcolor, double *grad_tex)
{
    const int W = s->width, H = s->height;
    const int64_t V = s->num_vertices;
    for (int64_t p = 0; p < (int64_t)W * H; ++p) {
        const int32_t t = primid[p];
        if (t < 0) continue;
        int64_t vid[3];
        for (int k = 0; k < 3; ++k) vid[k] = vertex_id(s, t, k);
        float bp[3];
        bp[1] = bary[2 * p];
        bp[2] = bary[2 * p + 1];
        bp[0] = (1.0f - bp[1]) - bp[2];
        const float *G = grad + 4 * p;
        if (s->shading == 1) {
            float rgb[3];
            for (int c = 0; c < 3; ++c) rgb[c] = interp(s->color + c * V, vid, bp);
            const float u = interp(s->uv, vid, bp);
            const float v = interp(s->uv + V, vid, bp);
            otap tp = bilinear_taps(s, u, v);
            for (int c = 0; c < 3; ++c) {
                const double Tc = (double)sample_channel(s, &tp, c);
                for (int k = 0; k < 3; ++k)
                    grad_vcolor[c * V + vid[k]] += (double)bp[k] * (double)G[c] * Tc;
                for (int j = 0; j < 4; ++j)
                    grad_tex[3 * tp.texel[j] + c] += (double)tp.w[j] * (double)G[c] * (double)rgb[c];
            }
        } else {
            for (int c = 0; c < 3; ++c)
                for (int k = 0; k < 3; ++k)
                    grad_vcolor[c * V + vid[k]] += (double)bp[k] * (double)G[c];
        }
    }
    return 0;
}

/* ======================================================================== */
/* Reyes front end: Split and Dice of bicubic Bezier patches.  The Reyes    */
/* pipeline of Sec. 7.1 has Split as a self-loop stage with one output back  */
/* to itself and one to Dice, and Dice turns a patch into micropolygons for  */
/* Sample and Shade; Sec. 5.1 runs such a self-loop by launching the stage   */
/* again until nothing is left.  The paper fixes no split test, split        */
/* direction or dice rate.  Readings used here: breadth-first rounds; a      */
/* patch is diced once the screen box of its control points is at most      */
/* dice_px on both axes; otherwise it is halved by de Casteljau at 1/2 along */
/* the parameter whose control polygon is longer on screen; an n x n dice    */
/* grid with central-difference normals.                                     */
/* ======================================================================== */

/* a patch: 16 control points, row-major over (v, u): point 4*i + j has u
 * index j and v index i; 3 float32 coordinates each (48 floats) */
enum { ORC_CP = 48 };

/* x + t (y - x), three rounded operations in this order */
static float lerpf(float x, float y, float t) { return x + t * (y - x); }

/* one cubic (a, b, c, d) at t by de Casteljau; also its two halves when
 * asked (left = a, ab, abc, p; right = p, bcd, cd, d) */
static float casteljau(float a, float b, float c, float d, float t, float *left, float *right)
{
    const float ab = lerpf(a, b, t), bc = lerpf(b, c, t), cd = lerpf(c, d, t);
    const float abc = lerpf(ab, bc, t), bcd = lerpf(bc, cd, t);
    const float p = lerpf(abc, bcd, t);
    if (left) { left[0] = a; left[1] = ab; left[2] = abc; left[3] = p; }
    if (right) { right[0] = p; right[1] = bcd; right[2] = cd; right[3] = d; }
    return p;
}

/* Halve a patch at u = 1/2 (dir 0: every row is a cubic in u) or v = 1/2
 * (dir 1: every column is a cubic in v). */
void orc_reyes_halve(const float *cp, int dir, float *lo, float *hi)
{
    for (int a = 0; a < 4; ++a) {
        for (int c = 0; c < 3; ++c) {
            float in[4], l[4], h[4];
            for (int k = 0; k < 4; ++k)
                in[k] = dir == 0 ? cp[3 * (4 * a + k) + c] : cp[3 * (4 * k + a) + c];
            casteljau(in[0], in[1], in[2], in[3], 0.5f, l, h);
            for (int k = 0; k < 4; ++k) {
                const int pt = dir == 0 ? 4 * a + k : 4 * k + a;
                lo[3 * pt + c] = l[k];
                hi[3 * pt + c] = h[k];
            }
        }
    }
}

/* Screen position of a control point through the same transform as the
 * vertex stage (each product rounded, sums left to right, one reciprocal of
 * w; no matrix: the identity), without snapping; 0 when w <= 0 or a value
 * is not finite. */
static int screen_point(const float *mvp, int W, int H, const float *p, float *xs, float *ys)
{
    float c[4] = {p[0], p[1], p[2], 1.0f};
    if (mvp) {
        for (int r = 0; r < 4; ++r) {
            float t = mvp[4 * r + 0] * p[0];
            t = t + mvp[4 * r + 1] * p[1];
            t = t + mvp[4 * r + 2] * p[2];
            t = t + mvp[4 * r + 3];
            c[r] = t;
        }
    }
    if (!(isfinite(c[0]) && isfinite(c[1]) && isfinite(c[3]) && c[3] > 0.0f)) return 0;
    const float iw = 1.0f / c[3];
    *xs = (c[0] * iw + 1.0f) * (0.5f * (float)W);
    *ys = (c[1] * iw + 1.0f) * (0.5f * (float)H);
    return isfinite(*xs) && isfinite(*ys);
}

/* What Split does with one patch: 0 drop (a control point behind the eye or
 * not finite, or the control points' screen bound outside the screen),
 * 1 dice (bound at most dice_px on both axes, or the last round), 2 split in u,
 * 3 split in v (the direction whose control polygon is longer on screen:
 * the largest squared screen distance between the end points of a row,
 * against that of a column; u on ties). */
int orc_reyes_decide(const float *cp, const float *mvp, int W, int H, float dice_px, int last)
{
    float xs[16], ys[16];
    for (int k = 0; k < 16; ++k)
        if (!screen_point(mvp, W, H, cp + 3 * k, &xs[k], &ys[k])) return 0;
    float x0 = xs[0], x1 = xs[0], y0 = ys[0], y1 = ys[0];
    for (int k = 1; k < 16; ++k) {
        x0 = fminf(x0, xs[k]); x1 = fmaxf(x1, xs[k]);
        y0 = fminf(y0, ys[k]); y1 = fmaxf(y1, ys[k]);
    }
    if (x1 < 0.0f || x0 > (float)W || y1 < 0.0f || y0 > (float)H) return 0;
    if ((x1 - x0 <= dice_px && y1 - y0 <= dice_px) || last) return 1;
    float du = 0.0f, dv = 0.0f;
    for (int a = 0; a < 4; ++a) {
        const float ux = xs[4 * a + 3] - xs[4 * a], uy = ys[4 * a + 3] - ys[4 * a];
        const float vx = xs[12 + a] - xs[a], vy = ys[12 + a] - ys[a];
        du = fmaxf(du, ux * ux + uy * uy);
        dv = fmaxf(dv, vx * vx + vy * vy);
    }
    return du >= dv ? 2 : 3;
}

/* Split: breadth-first rounds r = 0..max_depth.  Round 0 takes the input
 * patches in order; every patch of round r is dropped, kept for Dice
 * (appended to the leaves, in order) or halved, its two halves (lower
 * parameter first) going in order to round r + 1; round max_depth dices
 * whatever it holds.  Writes up to cap leaves (48 floats each) and their
 * input patch numbers; returns the number of leaves (-1 when out of memory). */
int64_t orc_reyes_split(const float *patches, int64_t np, const float *mvp, int W, int H,
                        float dice_px, int max_depth, float *leaf_cp, int32_t *leaf_src,
                        int64_t cap)
{
    int64_t qn = np, nleaf = 0;
    float *q = malloc(sizeof(float) * ORC_CP * (size_t)(np > 0 ? np : 1));
    int32_t *qs = malloc(sizeof(int32_t) * (size_t)(np > 0 ? np : 1));
    if (!q || !qs) { free(q); free(qs); return -1; }
    memcpy(q, patches, sizeof(float) * ORC_CP * (size_t)np);
    for (int64_t i = 0; i < np; ++i) qs[i] = (int32_t)i;
    for (int r = 0; r <= max_depth && qn > 0; ++r) {
        int64_t nn = 0;
        for (int64_t i = 0; i < qn; ++i)
            if (orc_reyes_decide(q + ORC_CP * i, mvp, W, H, dice_px, r == max_depth) >= 2) nn += 2;
        float *q2 = malloc(sizeof(float) * ORC_CP * (size_t)(nn > 0 ? nn : 1));
        int32_t *qs2 = malloc(sizeof(int32_t) * (size_t)(nn > 0 ? nn : 1));
        if (!q2 || !qs2) { free(q); free(qs); free(q2); free(qs2); return -1; }
        int64_t k = 0;
        for (int64_t i = 0; i < qn; ++i) {
            const float *cp = q + ORC_CP * i;
            const int d = orc_reyes_decide(cp, mvp, W, H, dice_px, r == max_depth);
            if (d == 1) {
                if (nleaf < cap) {
                    memcpy(leaf_cp + ORC_CP * nleaf, cp, sizeof(float) * ORC_CP);
                    leaf_src[nleaf] = qs[i];
                }
                ++nleaf;
            } else if (d >= 2) {
                orc_reyes_halve(cp, d - 2, q2 + ORC_CP * k, q2 + ORC_CP * (k + 1));
                qs2[k] = qs2[k + 1] = qs[i];
                k += 2;
            }
        }
        free(q); free(qs);
        q = q2; qs = qs2; qn = nn;
    }
    free(q); free(qs);
    return nleaf;
}

/* Dice: leaf l becomes an (n+1) x (n+1) grid of vertices at u = j/n, v = i/n
 * (every row of control points evaluated at u by de Casteljau, then the
 * resulting column at v), vertex l (n+1)^2 + i (n+1) + j, with the patch's
 * colour and the normal cross(Pu, Pv) of central differences of the grid
 * (one-sided at the border); and 2 n^2 triangles, quad (i, j) giving
 * (v00, v10, v11) and (v00, v11, v01) with v10 one step in u and v01 one in
 * v, triangle l 2n^2 + 2(i n + j) + {0, 1}.  Planes are [3][V] with
 * V = nl (n+1)^2. */
void orc_reyes_dice(const float *leaf_cp, const int32_t *leaf_src, const float *patch_color,
                    int64_t nl, int n, float *pos, float *color, float *normal, int32_t *idx)
{
    const int m = n + 1;
    const int64_t V = nl * (int64_t)m * m;
    float *g = malloc(sizeof(float) * 3 * (size_t)m * (size_t)m);
    if (!g) return;
    for (int64_t l = 0; l < nl; ++l) {
        const float *cp = leaf_cp + ORC_CP * l;
        for (int i = 0; i < m; ++i) {
            const float v = (float)i / (float)n;
            for (int j = 0; j < m; ++j) {
                const float u = (float)j / (float)n;
                for (int c = 0; c < 3; ++c) {
                    float col[4];
                    for (int a = 0; a < 4; ++a)
                        col[a] = casteljau(cp[3 * (4 * a) + c], cp[3 * (4 * a + 1) + c],
                                           cp[3 * (4 * a + 2) + c], cp[3 * (4 * a + 3) + c], u,
                                           NULL, NULL);
                    g[3 * (i * m + j) + c] = casteljau(col[0], col[1], col[2], col[3], v, NULL, NULL);
                }
            }
        }
        const int64_t vb = l * (int64_t)m * m;
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < m; ++j) {
                const int jp = j < n ? j + 1 : n, jm = j > 0 ? j - 1 : 0;
                const int ip = i < n ? i + 1 : n, im = i > 0 ? i - 1 : 0;
                float pu[3], pv[3];
                for (int c = 0; c < 3; ++c) {
                    pu[c] = g[3 * (i * m + jp) + c] - g[3 * (i * m + jm) + c];
                    pv[c] = g[3 * (ip * m + j) + c] - g[3 * (im * m + j) + c];
                }
                const int64_t vtx = vb + i * m + j;
                for (int c = 0; c < 3; ++c) {
                    pos[c * V + vtx] = g[3 * (i * m + j) + c];
                    color[c * V + vtx] = patch_color[3 * leaf_src[l] + c];
                }
                normal[vtx] = pu[1] * pv[2] - pu[2] * pv[1];
                normal[V + vtx] = pu[2] * pv[0] - pu[0] * pv[2];
                normal[2 * V + vtx] = pu[0] * pv[1] - pu[1] * pv[0];
            }
        }
        const int64_t tb = l * 2 * (int64_t)n * n;
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) {
                const int32_t v00 = (int32_t)(vb + i * m + j), v10 = v00 + 1;
                const int32_t v01 = v00 + m, v11 = v01 + 1;
                int32_t *t = idx + 3 * (tb + 2 * (i * n + j));
                t[0] = v00; t[1] = v10; t[2] = v11;
                t[3] = v00; t[4] = v11; t[5] = v01;
            }
        }
    }
    free(g);
}
