/*
 * pk_reyes.h -- C ABI of the Reyes front end of libpk: Split and Dice of
 * bicubic Bezier patches on an MI355X (gfx950).
 *
 * The Reyes pipeline of Piko (Sec. 7.1, "Reyes") has four stages: Split,
 * Dice, Sample and Shade.  Split is a self-loop stage with two output
 * channels, one back to itself and one to Dice; Dice turns each patch it
 * receives into a grid of micropolygons; Sample tests them for screen
 * coverage in small bins and Shade colours the fragments with a diffuse
 * model.  Sample and Shade are the binned rasterizer of pk.h drawing the
 * diced mesh with PK_SHADE_LIT; this header adds the two stages in front of
 * it.  A self-loop stage runs by launching it again until its queue is
 * empty (Sec. 5.1, stage ordering with cycles); here each round of Split is
 * one kernel that reads the round's queue length from device memory, so
 * rounds are enqueued in batches and no round waits for the host.
 *
 * The paper fixes neither the split test nor the dice rate.  This library
 * reads them as follows (every rule is exact and deterministic, so results
 * are bit-identical run to run):
 *  - A patch is 16 float32 control points of 3 coordinates, row-major over
 *    (v, u): point 4i + j has u index j and v index i (48 floats per patch,
 *    [P][16][3]).
 *  - Screen position of a control point: the vertex transform of pk.h
 *    (clip = MVP * (x, y, z, 1), products rounded, sums left to right, no
 *    fused multiply-add, one correctly rounded 1/w, screen = (ndc + 1) *
 *    (W/2, H/2)), without snapping.
 *  - Split visits patches in breadth-first rounds r = 0 .. max_depth.
 *    Round 0 holds the input patches in order.  A patch is dropped when a
 *    control point has w <= 0 or a non-finite value, or when the screen box
 *    of its control points lies outside [0, W] x [0, H]; it goes to Dice
 *    when that box is at most dice_px wide and high, or in round max_depth;
 *    otherwise it is halved at u = 1/2 or v = 1/2 (de Casteljau, each
 *    interpolation a + t (b - a) rounded as written) along the direction
 *    whose control polygon is longer on screen (the largest squared screen
 *    distance between the end points of a row, against that of a column;
 *    u on ties), and both halves, the lower parameter first, go to round
 *    r + 1 in the order of their parents.  Leaves are numbered in the order
 *    the rounds emit them (round by round, in queue order).
 *  - Dice: leaf l becomes (n+1)^2 vertices, vertex l (n+1)^2 + i (n+1) + j
 *    at (u, v) = (j/n, i/n) (each row of control points evaluated at u by
 *    de Casteljau, then the resulting column at v), with the colour of its
 *    source patch and the unnormalised normal cross(Pu, Pv) of central
 *    differences of the grid (one-sided on the border); and 2 n^2
 *    triangles, quad (i, j) giving (v00, v10, v11) and (v00, v11, v01)
 *    with v10 one step in u and v01 one step in v, triangle
 *    l 2n^2 + 2 (i n + j) + {0, 1}.
 *
 * Conventions are those of pk.h: pointers in argument lists are DEVICE
 * pointers unless marked [host]; the caller owns all memory; the library
 * never allocates and never synchronizes (calls only enqueue on `stream`, a
 * hipStream_t, NULL = the default stream); arguments are validated on the
 * host before anything is enqueued (PK_ERR_INVALID_ARGUMENT, nothing
 * enqueued); a failed launch returns PK_ERR_HIP.
 */
#ifndef PK_REYES_H
#define PK_REYES_H

#include "pk.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {             /* [host] */
    int32_t width, height;   /* screen, 1..8192 pixels */
    float dice_px;           /* dice test: screen box at most this on both axes;
                                finite, > 0 */
    int32_t max_depth;       /* last round (0..30): whatever it holds is diced */
    int32_t dice_n;          /* dice grid: n x n quads per leaf, 1..16 */
} pk_reyes_params;

/* Most patches one round's queue may hold (queue_capacity) and most input
 * patches of one call. */
#define PK_REYES_MAX_QUEUE (1ll << 28)

/* Bytes of the workspace of pk_reyes_split for num_patches input patches
 * and a queue of queue_capacity patches: two queues of patches and source
 * numbers (one round reads one, writes the other), a decision byte per
 * patch of a round, per-workgroup counts and the rounds' counters.  0 for
 * invalid arguments.  Host-only. */
size_t pk_reyes_workspace_bytes(const pk_reyes_params *p, int64_t num_patches,
                                int64_t queue_capacity);

/* Split (Sec. 7.1 Reyes; self-loop of Sec. 5.1) of num_patches patches
 * [P][16][3] seen through `mvp` ([16] float32 row-major acting on column
 * vectors, or NULL = identity).  `patches` and `leaves` are 16-byte
 * aligned.  Enqueues rounds round_begin .. min(round_end, max_depth + 1) - 1:
 * a whole Split is rounds 0 .. max_depth, in one call or in several calls on
 * the same workspace and buffers, each starting where the previous one
 * stopped (a call with round_begin 0 starts afresh).  The leaves, in the
 * order above, go to leaves [leaf_capacity][16][3] and their input patch
 * numbers to leaf_src [leaf_capacity]; leaves beyond leaf_capacity are
 * counted, not written.  counts (device, int64[6]) receives, over the
 * rounds run so far:
 *   [0] the number of leaves,
 *   [1] the most patches any round had to queue,
 *   [2] the patches visited (Split's work),
 *   [3] 1 when a round's queue outgrew queue_capacity, else 0,
 *   [4] the patches queued for the round after the last one run (0: Split
 *       has drained, and further rounds would do nothing),
 *   [5] the number of rounds that had patches to visit.
 * A caller that knows roughly how deep a scene splits (say [5] of the
 * previous frame) enqueues that many rounds, reads [4] (the paper's check
 * that the self-loop has drained) and enqueues the rest only if it is not
 * 0: empty rounds cost a launch each.  When [3] is 1 the rounds after the
 * overflow saw a truncated queue and [0] is not the true count: split again
 * from round 0 with queue_capacity >= [1] (which may grow again in later
 * rounds).  `ws` (256-byte aligned) holds pk_reyes_workspace_bytes(p,
 * num_patches, queue_capacity) bytes; it needs no initialisation, and keeps
 * the state between the calls of one Split.  num_patches
 * 0..PK_REYES_MAX_QUEUE, queue_capacity 0..PK_REYES_MAX_QUEUE,
 * leaf_capacity >= 0, 0 <= round_begin <= round_end. */
pk_status pk_reyes_split(const pk_reyes_params *p, const float *patches, int64_t num_patches,
                         const float *mvp, void *ws, int64_t queue_capacity, float *leaves,
                         int32_t *leaf_src, int64_t leaf_capacity, int32_t round_begin,
                         int32_t round_end, int64_t *counts, void *stream);

/* Dice (Sec. 7.1 Reyes) of num_leaves leaves [L][16][3] with source patch
 * numbers leaf_src [L] into a one-scene indexed mesh for pk.h: pos, color
 * and normal are SoA planes [3][V] with V = L (n+1)^2, indices [2 n^2 L][3]
 * (the layout of pk_mesh and pk_attribs).  patch_color [num_patches][3]
 * gives each vertex its source patch's colour; a source number outside
 * [0, num_patches) gives colour 0.  V and 2 n^2 L must be below 2^31. */
pk_status pk_reyes_dice(const pk_reyes_params *p, const float *leaves, const int32_t *leaf_src,
                        int64_t num_leaves, const float *patch_color, int64_t num_patches,
                        float *pos, float *color, float *normal, int32_t *indices,
                        void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PK_REYES_H */
