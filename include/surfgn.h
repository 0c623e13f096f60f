/*
 * surfgn.h -- C ABI of the MI355X (gfx950) surfel Gauss-Newton library.
 *
 * Method: "Dense monocular SLAM by direct surfel optimization" (Trabes,
 * Dondo Gazzano, Sosa Paez).  A keyframe is covered by surfels, each an
 * inverse depth id_s along its centre ray r_s and a unit normal n_s
 * (Surfel Parameterization section, Eq. 1).  Every Gauss-Newton iteration
 * warps each surfel into every neighbour frame by its plane-induced
 * homography (Eq. 6), samples the frame bilinearly with its gradient, forms
 * Huber-weighted photometric residuals (Eq. 5) and their Jacobians with
 * respect to the surfel's three parameters (Eq. 7-9), reduces J^T W J and
 * J^T W r, solves the 3x3 system and updates id_s and the renormalised
 * normal (Surfel Optimization section).  New surfels are initialised from
 * their neighbours' planes (Surfel Initialization section) and the per-pixel
 * inverse depth is rendered from the surfel planes (Eq. 3).
 *
 * Conventions
 *   - Camera frame x right, y down, z forward.  Pixel (x, y) has its centre
 *     at integer coordinates.  K = [[fx, 0, cx], [0, fy, cy], [0, 0, 1]].
 *   - A pose P_kf^fn maps keyframe coordinates to frame n: X_n = R X_kf + t,
 *     R row-major (Eq. 6).
 *   - Surfels are S x S pixel tiles (S = patch, 4, 8 or 16): tile (tx, ty) owns
 *     pixels [S tx, S tx + S) x [S ty, S ty + S); its centre pixel is
 *     (S tx + (S-1)/2, S ty + (S-1)/2).  The grid is gw x gh with
 *     gw = width / S, gh = height / S (floor; the ragged right/bottom border
 *     has no surfel).  Surfel arrays are indexed ty * gw + tx.
 *   - Images are row-major with a pitch in elements.  The sampled value is
 *     stored_value * scale (f32: scale is normally 1; u8: e.g. 1/255).
 *
 * Memory and ownership
 *   - Every buffer is allocated and owned by the caller; the library never
 *     frees caller memory.  Pointers inside sgn_image / sgn_surfels and the
 *     output arrays are DEVICE pointers (on the context's device).  The
 *     descriptor arrays themselves (sgn_keyframe.nbr, .pose, sgn_batch_item
 *     arrays) are HOST memory, read during the call only.
 *   - The context owns a descriptor table of fixed capacity (SGN_MAX_BATCH
 *     keyframes or keyframe pairs and SGN_MAX_BATCH_FRAMES neighbour frames
 *     per call; about 2 MB on the device and four times that in pinned host
 *     staging memory), the work-queue counters, timing events and captured
 *     HIP graphs.  sgn_create allocates all of it; no other call allocates
 *     device or pinned memory.
 *   - Calls that need scratch memory (re-gridding, disc render and
 *     placement, the autotuner's state snapshot) take a caller-provided
 *     workspace `ws` of `ws_bytes` bytes: device memory, 256-byte aligned, at
 *     least the size the matching sgn_*_workspace_bytes function returns for
 *     the same arguments.  Its contents need not be initialised and are
 *     undefined afterwards; it must stay allocated until the call's work on
 *     the context's stream has completed.  A missing, misaligned or
 *     undersized workspace is an argument error (SGN_E_INVALID, nothing
 *     enqueued).
 *   - All work is enqueued asynchronously on the context's stream; the caller
 *     synchronises that stream before reading results.  Calls on one context
 *     must come from one host thread at a time.
 *
 * Errors
 *   - Invalid arguments and shapes are reported synchronously
 *     (SGN_E_INVALID, SGN_E_UNSUPPORTED) and nothing is enqueued.
 *   - HIP runtime failures return SGN_E_DEVICE (on the call or on a later one).
 *   - sgn_last_error() returns a thread-local description of the last failure.
 *   - Numerical failures of single surfels are NOT API errors: they set bits
 *     of the surfel's flags word (SGN_FLAG_*), and its state is kept.
 */
#ifndef SURFGN_H
#define SURFGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sgn_ctx sgn_ctx;

typedef enum {
    SGN_OK = 0,
    SGN_E_INVALID = -1,      /* bad argument, shape or pointer */
    SGN_E_NOMEM = -2,        /* the context could not grow its own tables */
    SGN_E_DEVICE = -3,       /* HIP runtime error */
    SGN_E_UNSUPPORTED = -4,  /* valid but not implemented (e.g. patch size) */
    SGN_E_BUSY = -5
} sgn_status;

typedef enum { SGN_F32 = 0, SGN_F16 = 1, SGN_U8 = 2 } sgn_dtype;

/* Per-surfel flag bits. */
enum {
    SGN_FLAG_DEGENERATE = 1u << 0,   /* |n_s . r_s| < 1e-6: Eq. 3 undefined */
    SGN_FLAG_FEW_SAMPLES = 1u << 1,  /* fewer than 3 valid (pixel, frame) samples */
    SGN_FLAG_SOLVE_FAIL = 1u << 2,   /* J^T W J not positive definite */
    SGN_FLAG_REJECTED = 1u << 3,     /* update gave id_s <= 0 or a non-finite value */
    SGN_FLAG_FP64_SOLVE = 1u << 4,   /* 3x3 solved in double (ill-conditioned) */
    SGN_FLAG_UNINIT = 1u << 5        /* new surfel without usable neighbours */
};

typedef struct { double fx, fy, cx, cy; } sgn_intrinsics;

/* P_kf^fn of Eq. 6: X_n = R X_kf + t, R row-major. */
typedef struct { double R[9]; double t[3]; } sgn_pose;

typedef struct {
    const void* data;      /* device pointer to pixel (0, 0) */
    int32_t width, height;
    int32_t pitch;         /* elements between rows, >= width */
    int32_t dtype;         /* sgn_dtype */
    float scale;           /* sampled value = stored * scale (> 0) */
} sgn_image;

/* One keyframe and its group Omega of neighbour frames (Eq. 5).  All images
 * share the keyframe's width, height and dtype. */
typedef struct {
    sgn_image kf;               /* I_kf */
    const sgn_image* nbr;       /* host array [n_nbr]: I_fn */
    const sgn_pose* pose;       /* host array [n_nbr]: P_kf^fn */
    int32_t n_nbr;              /* 1 .. SGN_MAX_NBR */
    sgn_intrinsics K;
    int32_t patch;              /* S: 4, 8 or 16 */
} sgn_keyframe;

#define SGN_MAX_NBR 16
#define SGN_MAX_BATCH 1024          /* keyframes (or keyframe pairs) per call */
#define SGN_MAX_BATCH_FRAMES 8192   /* neighbour frames per call, all keyframes together */
#define SGN_STATIC_SCRATCH_BYTES (4u << 20)  /* static device scratch of sgn_transfer_surfels_static */

/* Surfel state, structure of arrays of length gw * gh (device pointers).
 * inv_depth, nx, ny, nz, flags are read and written; cost, nvalid and
 * last_update are written (last_update only when a step was accepted). */
typedef struct {
    float* inv_depth;           /* id_s (1/m along the centre ray, z = 1) */
    float* nx; float* ny; float* nz;  /* unit normal n_s (sign is preserved) */
    uint32_t* flags;            /* SGN_FLAG_* */
    float* cost;                /* Huber cost (Eq. 5) at the last linearisation point */
    uint32_t* nvalid;           /* valid samples at that point */
    uint32_t* last_update;      /* params.stamp of the last accepted update */
} sgn_surfels;

typedef struct {
    int32_t iters;              /* Gauss-Newton iterations (>= 0) */
    float huber_k;              /* Huber threshold in sampled-value units (> 0) */
    float kappa_fp64;           /* solve in double when the equilibrated condition
                                   estimate exceeds this (e.g. 1e6) */
    int32_t depth_only;         /* 1: d id_u / d n_s := 0 (ablation), only id_s moves */
    float beta_r;               /* init neighbour radius in pixels (<= 0: S) */
    uint32_t stamp;             /* written to last_update */
    float lm_lambda;            /* 0: Gauss-Newton.  > 0: Levenberg-Marquardt (the method
                                   names it; the paper gives no schedule): each iteration
                                   solves (H + lambda diag H) d = -b, evaluates the Huber cost
                                   at the candidate and accepts it when the mean cost per
                                   valid sample does not rise (then lambda /= 10, floor 1e-9),
                                   else keeps the state (lambda *= 10); a candidate plane
                                   containing the centre ray is refused.  lm_lambda is the
                                   starting lambda of every surfel. */
} sgn_params;

/* Launch plan for the fused Gauss-Newton kernel (chosen by sgn_autotune or
 * by the caller; all-zero means "library default"). */
typedef struct {
    int32_t tiles_x, tiles_y;   /* surfels per wavefront as a tiles_x x tiles_y block
                                   (S = 4: 4x1, 2x2 or 1x4, one pixel per lane; 4x2 or
                                   2x4, two pixels per lane; 4x4, four pixels per lane;
                                   S = 8 and 16: 1x1, an S = 16 surfel giving each lane
                                   four pixels).  Plans with the same pixels per lane
                                   give bitwise-equal results */
    int32_t persistent;         /* 1: persistent grid pulling work items from a
                                   device queue; 0: one wavefront per work item */
    int32_t waves_per_cu;       /* persistent grid size per compute unit (0: occupancy) */
    int32_t lds_stage;          /* 1: stage neighbour-frame footprints in LDS */
    int32_t xcd_queues;         /* 1: keyframes bound to an XCD, balanced by work: with
                                   persistent, one device queue per XCD; without, the
                                   workgroups the hardware gives XCD x (every eighth,
                                   from x) take XCD x's share of the work items in
                                   order (batches of eight keyframes or more; fewer
                                   run as with 0) */
    int32_t groups;             /* tiles_x x tiles_y groups per work item: 1, 2 or 4; 1 or
                                   2 for the 4x2 and 2x4 blocks; 1 for 4x4 and S = 16 (0:
                                   as many as fit, at most four).  A work item lies in one
                                   aligned 16 x 16-pixel block; its per-surfel solves run
                                   together, one lane each */
} sgn_plan;

/* One keyframe of a batch with its surfels and optional outputs. */
typedef struct {
    sgn_keyframe kf;
    sgn_surfels surfels;
    const uint8_t* is_new;      /* device [gw*gh] or NULL: surfels to initialise from
                                   their neighbours before the first iteration */
    float* inv_depth_out;       /* device [height * width] or NULL: rendered id_u
                                   (0 = no measurement), row-major, pitch = width */
    int32_t* index_out;         /* device [height * width] or NULL: owning surfel or -1 */
} sgn_batch_item;

typedef struct {
    int32_t device;
    int32_t compute_units;
    int32_t xcds;
    int32_t clock_khz;
    int32_t memory_clock_khz;
    int32_t memory_bus_bits;
    int64_t total_global_mem;
    int32_t lds_per_cu;
    char name[64];
    char arch[32];
} sgn_device_props;

/* Create a context on `device` whose work goes to `hip_stream` (a hipStream_t;
 * NULL = the device's null stream).  The stream stays owned by the caller. */
sgn_status sgn_create(sgn_ctx** out, int32_t device, void* hip_stream);
sgn_status sgn_destroy(sgn_ctx* ctx);
sgn_status sgn_set_stream(sgn_ctx* ctx, void* hip_stream);

/* Surfel Initialization section: every surfel with is_new[i] != 0 gets
 *   id_s = mean_j id_j (n_j . r_s) / (n_j . r_j)   (Eq. 3 of neighbour j at r_s)
 *   n_s  = normalise(sum_j sign(n_j . n_ref) n_j)    (n_ref: first neighbour)
 * over the surfels j that are not new, not flagged DEGENERATE/UNINIT, have
 * |n_j . r_j| >= 1e-6 and own a pixel closer than beta_r to the new surfel's
 * centre pixel.  Without such neighbours the surfel is flagged UNINIT and
 * left unchanged.  is_new: device [gw*gh]. */
sgn_status sgn_init_from_neighbours(sgn_ctx* ctx, const sgn_keyframe* kf,
                                    const sgn_surfels* surfels, const uint8_t* is_new,
                                    const sgn_params* params);

/* Surfel Optimization section: params->iters Gauss-Newton iterations on every
 * surfel of the keyframe (Eq. 5-9), in place.  Per iteration and surfel:
 * Huber IRLS normal equations over all (pixel, frame) samples, 3x3 solve
 * (float; double above kappa_fp64), id_s += d0 and
 * n_s = normalise(n_s + d1 b1 + d2 b2) on a fixed tangent basis. */
sgn_status sgn_optimize_keyframe(sgn_ctx* ctx, const sgn_keyframe* kf,
                                 const sgn_surfels* surfels, const sgn_params* params,
                                 const sgn_plan* plan /* NULL: default */);

/* Inverse Depth Calculation section: per-pixel id_u of the owning surfel by
 * Eq. 3 (0 where there is no measurement: pixel outside the grid, surfel
 * flagged DEGENERATE or UNINIT, or id_u <= 0).  inv_depth_out: device
 * [height * width]; index_out: device [height * width] or NULL. */
sgn_status sgn_render_inverse_depth(sgn_ctx* ctx, const sgn_keyframe* kf,
                                    const sgn_surfels* surfels, float* inv_depth_out,
                                    int32_t* index_out);

/* The whole per-keyframe update for many keyframes at once: initialisation
 * of new surfels, the Gauss-Newton iterations in one fused kernel launch
 * (persistent, or one wavefront per work item as the plan says), and the
 * inverse-depth render; the setup + initialisation and render parts (and a
 * persistent GN launch) are replayed from captured HIP graphs.  All
 * items must share patch and image dtype.  Results equal those of the
 * per-keyframe calls for the same plan (each surfel is reduced in a fixed
 * order that does not depend on the batch). */
sgn_status sgn_optimize_batch(sgn_ctx* ctx, const sgn_batch_item* items, int32_t n_items,
                              const sgn_params* params, const sgn_plan* plan /* NULL: default */);

/* Time candidate plans on a sample batch and return the fastest in *out
 * (host): every tile layout with its group counts, persistent or not, XCD
 * queues or shares or not; each timed as the fastest of three runs after a warm-up
 * run.  When the default plan is within 1 % of the fastest it is returned
 * instead (a tie at the timer's resolution), so a batch gets the same plan
 * from run to run.  The surfel state is snapshotted into the workspace
 * before the first trial and restored from it after every trial, so the
 * items' state is unchanged on return.  Synchronous (waits for the trials).
 * ws: see sgn_autotune_workspace_bytes. */
sgn_status sgn_autotune(sgn_ctx* ctx, const sgn_batch_item* sample, int32_t n_items,
                        const sgn_params* params, sgn_plan* out, void* ws, size_t ws_bytes);

/* Workspace bytes of sgn_autotune for these items: 256-byte aligned copies of
 * the eight state arrays of every item (about 32 bytes per surfel).  0 when
 * the items are invalid (n_items outside [1, SGN_MAX_BATCH], null array, bad
 * patch or size). */
size_t sgn_autotune_workspace_bytes(int32_t n_items, const sgn_batch_item* sample);

/* A keyframe's surfel grid for re-gridding: intrinsics, image size and tile
 * edge S (4, 8 or 16); the grid is (width / S) x (height / S) tiles. */
typedef struct {
    sgn_intrinsics K;
    int32_t width, height, patch;
} sgn_grid;

/* Surfel reference-frame change (Eq. 10) and re-gridding into the tiles of
 * another keyframe whose pose is X_dst = R X_src + t (pose, host memory).
 * A usable source surfel (no DEGENERATE or UNINIT flag, inv_depth > 0) moves
 * to p' = R (r_s / id_s) + t with normal n' = R n and lands in the
 * destination pixel nearest to pi(K_dst p'), hence in that pixel's tile.  In
 * each destination tile the closest landed surfel wins (largest 1/p'_z; ties
 * to the lower source index) and its plane is re-expressed at the tile's
 * centre ray by Eq. 3.  Tiles that receive nothing get id 0, n (0, 0, -1),
 * the UNINIT flag and dst_is_new = 1, ready for sgn_init_from_neighbours.
 * Landing decisions are taken in double.  src, dst: device surfel arrays of
 * the two grids (all fields written for dst; cost and nvalid are zeroed,
 * last_update is the winner's).  dst_is_new: device [dst tiles];
 * dst_src_index: device [dst tiles] or NULL (winning source index or -1).
 * src and dst must not overlap.  ws: see sgn_transfer_workspace_bytes. */
sgn_status sgn_transfer_surfels(sgn_ctx* ctx, const sgn_grid* src_grid, const sgn_surfels* src,
                                const sgn_pose* pose, const sgn_grid* dst_grid, sgn_surfels* dst,
                                uint8_t* dst_is_new, int32_t* dst_src_index, void* ws,
                                size_t ws_bytes);

/* Workspace bytes of re-gridding into the n destination grids dst_grids
 * (host array): a 64-bit landing key and a 32-bit winner index per
 * destination tile, 12 bytes per tile plus alignment.  0 when n is outside
 * [1, SGN_MAX_BATCH], dst_grids is null or a grid is invalid. */
size_t sgn_transfer_workspace_bytes(int32_t n, const sgn_grid* dst_grids);

/* sgn_transfer_surfels without a workspace argument, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same operation, the same results bitwise.  The
 * re-gridding scratch (a landing key and a winner index per destination
 * tile) is a static device array of SGN_STATIC_SCRATCH_BYTES that every GPU
 * the library runs on holds until the process ends; its address on the
 * context's device is looked up once, by sgn_create.  The call allocates no
 * memory, device or host, and clears the part of the scratch it uses on the
 * device before use (a kernel, not a memset).  All calls on one GPU share
 * that GPU's array and it keeps the last call's contents: calls that
 * overlap on one GPU (several streams, contexts or threads) race, and the
 * caller must order them.  Errors: as sgn_transfer_surfels (nothing
 * enqueued); SGN_E_INVALID when the destination grid needs more scratch
 * than SGN_STATIC_SCRATCH_BYTES (12 bytes per destination tile plus
 * alignment: about 349,000 tiles). */
sgn_status sgn_transfer_surfels_static(sgn_ctx* ctx, const sgn_grid* src_grid, const sgn_surfels* src,
                                       const sgn_pose* pose, const sgn_grid* dst_grid, sgn_surfels* dst,
                                       uint8_t* dst_is_new, int32_t* dst_src_index);

/* sgn_transfer_surfels for n keyframe pairs at once (Eq. 10, Surfel
 * reference frame change): four launches for the whole batch, the same
 * results as n calls (pairs share nothing).  Pair k takes src_grids[k],
 * srcs[k], poses[k], dst_grids[k], dsts[k], dst_is_new[k] and
 * dst_src_index[k] (dst_src_index itself may be NULL, as may its entries);
 * all arrays are host memory read during the call.  ws: see
 * sgn_transfer_workspace_bytes(n, dst_grids).  Errors: as
 * sgn_transfer_surfels for any pair (nothing enqueued), SGN_E_INVALID for
 * n < 1 or a null array, SGN_E_UNSUPPORTED for n > SGN_MAX_BATCH. */
sgn_status sgn_transfer_surfels_batch(sgn_ctx* ctx, int32_t n, const sgn_grid* src_grids,
                                      const sgn_surfels* srcs, const sgn_pose* poses,
                                      const sgn_grid* dst_grids, const sgn_surfels* dsts,
                                      uint8_t* const* dst_is_new, int32_t* const* dst_src_index,
                                      void* ws, size_t ws_bytes);

/* ------------------------------------------------------------ disc surfels
 *
 * Disc surfels (Eq. 4): surfel i is centred at u_s = (ux[i], uy[i]) in
 * keyframe pixels and covers the pixels u inside the image with
 * |u - u_s| < r.  The radius r is the same for every surfel of a keyframe
 * (the paper sizes it so that every surfel covers the same screen area).
 * Membership is decided as dx^2 + dy^2 < r^2 in double.  A disc item's
 * kf.patch is not used; its surfel arrays (sgn_surfels fields plus ux, uy)
 * hold `count` surfels, or more for sgn_disc_place. */
typedef struct {
    sgn_keyframe kf;
    sgn_surfels surfels;        /* device arrays, [count] or more */
    float* ux;                  /* device: centre x of each surfel (pixels) */
    float* uy;                  /* device: centre y */
    int32_t count;              /* surfels 0 .. count-1 */
    float radius;               /* r in pixels, 0 < r <= 12 */
} sgn_disc_item;

/* Gauss-Newton over the disc surfels of n_items keyframes (Proposed
 * Approach section, Eq. 5-9): as sgn_optimize_batch, with each surfel's
 * cost summed over the pixels of its disc (Eq. 5 with u in s read as Eq. 4).
 * Two surfels per wavefront for f16 and u8 images, one for f32; per-surfel
 * results do not depend on the batch.
 * params as for tiles (beta_r unused).  Asynchronous on the context's
 * stream; sgn_last_kernel_ms times the Gauss-Newton kernel.  Errors: invalid
 * items or params (SGN_E_INVALID, nothing enqueued). */
sgn_status sgn_disc_optimize(sgn_ctx* ctx, const sgn_disc_item* items, int32_t n_items,
                             const sgn_params* params);

/* Inverse Depth Calculation section with disc surfels: every surfel without
 * the DEGENERATE or UNINIT flag whose plane does not contain its centre ray
 * (|n . r_s| >= 1e-6) writes Eq. 3 into the pixels of its disc; the depth
 * buffer keeps the closest (largest id_u > 0; equal values go to the lower
 * index).  id_u is evaluated in double and rounded to float.
 * inv_depth_out: device float [height * width] (row-major, width per row,
 * 0 = no measurement); index_out: device int32 of the same shape (winning
 * surfel, -1 = none) or NULL.  Reads only the item's surfels, intrinsics and
 * image size.  ws: see sgn_disc_render_workspace_bytes(1, item). */
sgn_status sgn_disc_render(sgn_ctx* ctx, const sgn_disc_item* item, float* inv_depth_out,
                           int32_t* index_out, void* ws, size_t ws_bytes);

/* sgn_disc_render for n_items keyframes in one pass (seven launches in all):
 * inv_depth_outs and index_outs are host arrays of n_items device pointers
 * (index_outs, or any of its entries, may be NULL).  ws: see
 * sgn_disc_render_workspace_bytes(n_items, items). */
sgn_status sgn_disc_render_batch(sgn_ctx* ctx, const sgn_disc_item* items, int32_t n_items,
                                 float* const* inv_depth_outs, int32_t* const* index_outs, void* ws,
                                 size_t ws_bytes);

/* Workspace bytes of a disc render of these items (host array): a raster
 * record (48 bytes) and up to nine tile-list entries (36 bytes) per surfel,
 * and 8 bytes per 16 x 16-pixel render tile, plus alignment.  Depends only
 * on the items' image sizes and counts.  0 when the items are invalid. */
size_t sgn_disc_render_workspace_bytes(int32_t n_items, const sgn_disc_item* items);

/* Parameters of the empty-area search (the paper leaves alpha and beta open). */
typedef struct {
    float alpha;                /* a candidate needs no measurement within alpha r: (0, 4] */
    float beta;                 /* neighbours own a pixel closer than beta r: (0, 4] */
    int32_t spacing;            /* candidate lattice step in pixels: [1, 1024] */
} sgn_disc_place_params;

/* Surfel Initialization section with disc surfels.  Candidates are the
 * pixels (spacing/2 + i spacing, spacing/2 + j spacing) of the keyframe; a
 * candidate u_ns qualifies when every non-empty pixel of index_map lies
 * farther than alpha r from it (integer squared distance against
 * (alpha r)^2 in double).  The qualifying candidates, in row-by-row lattice
 * order, become surfels count, count + 1, ... up to capacity - 1 (their
 * centres are written to ux, uy).  Each new surfel is initialised from its
 * neighbours: the surfels below `count` that own a pixel of index_map closer
 * than beta r to u_ns (skipping DEGENERATE / UNINIT ones and planes through
 * the camera centre), visited in index order; id_s = the mean of Eq. 3 of
 * their planes at r_ns, n_s = the mean of their normals sign-aligned to the
 * first, renormalised; with no usable neighbour the surfel gets id 0,
 * n = (0, 0, -1) and UNINIT.  cost, nvalid and last_update of new surfels
 * are zeroed.  index_map: device int32 [height * width], normally
 * sgn_disc_render's index_out for surfels 0 .. count-1.  capacity: entries
 * the surfel arrays and ux, uy hold (>= count).  counts_out: device int32[2]
 * receiving the number placed and the number that qualified (which may
 * exceed the room).  Asynchronous: read counts_out after synchronising to
 * learn the new count. */
sgn_status sgn_disc_place(sgn_ctx* ctx, const sgn_disc_item* item, const int32_t* index_map,
                          int32_t capacity, const sgn_disc_place_params* params,
                          int32_t* counts_out, void* ws, size_t ws_bytes);

/* Workspace bytes of a placement of these items with this lattice spacing:
 * one byte per lattice candidate, plus alignment.  Depends only on the
 * items' image sizes.  0 when the items or the spacing are invalid. */
size_t sgn_disc_place_workspace_bytes(int32_t n_items, const sgn_disc_item* items, int32_t spacing);

/* sgn_disc_place for n keyframes at once (Surfel Initialization section):
 * three launches for the whole batch instead of three per keyframe, with
 * the same results as n calls in any order (keyframes share nothing).
 * items[i], index_maps[i] (device int32 [height * width]), capacities[i] and
 * counts_outs[i] (device int32[2]) are keyframe i's arguments of
 * sgn_disc_place; the three arrays of pointers and counts are host memory
 * read during the call; params apply to every keyframe.  ws: see
 * sgn_disc_place_workspace_bytes(n, items, params->spacing).  Errors: as
 * sgn_disc_place for any keyframe (nothing enqueued), SGN_E_INVALID for
 * n < 1 or a null array. */
sgn_status sgn_disc_place_batch(sgn_ctx* ctx, const sgn_disc_item* items, int32_t n,
                                const int32_t* const* index_maps, const int32_t* capacities,
                                const sgn_disc_place_params* params, int32_t* const* counts_outs,
                                void* ws, size_t ws_bytes);

/* Surfel reference-frame change (Eq. 10) for disc surfels, which stay discs:
 * a usable surfel of src (no DEGENERATE or UNINIT flag, id_s > 0) moves to
 * p' = R (r_s / id_s) + t with n' = R n (pose: X_dst = R X_src + t, host
 * memory) and is centred in the destination keyframe at u' = K_dst pi(p')
 * with inverse depth 1/p'_z.  Those with p'_z > 0 whose u' lies in
 * [0, W-1] x [0, H-1] of dst's image are written in source order to dst's
 * surfels 0, 1, ... up to capacity - 1: id, n, centre, flags 0, cost 0,
 * nvalid 0 and the source's last_update.  Landing decisions are taken in
 * double.  dst supplies the destination intrinsics, image size and arrays
 * (dst->count is not read).  counts_out: device int32[2] receiving the number
 * written and the number that landed; src_index_out: device int32
 * [capacity] (source index of each written surfel) or NULL.  src and dst
 * arrays must not overlap.  Asynchronous. */
sgn_status sgn_disc_transfer(sgn_ctx* ctx, const sgn_disc_item* src, const sgn_pose* pose,
                             const sgn_disc_item* dst, int32_t capacity, int32_t* counts_out,
                             int32_t* src_index_out);

/* sgn_disc_transfer for n keyframe pairs in one launch (one workgroup per
 * pair), the same results as n calls (pairs share nothing).  Pair k takes
 * srcs[k], poses[k], dsts[k], capacities[k], counts_outs[k] and
 * src_index_outs[k] (src_index_outs itself may be NULL, as may its entries);
 * all arrays are host memory read during the call.  Errors: as
 * sgn_disc_transfer for any pair (nothing enqueued), SGN_E_INVALID for
 * n < 1 or a null array. */
sgn_status sgn_disc_transfer_batch(sgn_ctx* ctx, int32_t n, const sgn_disc_item* srcs,
                                   const sgn_pose* poses, const sgn_disc_item* dsts,
                                   const int32_t* capacities, int32_t* const* counts_outs,
                                   int32_t* const* src_index_outs);

/* Convert a float image (device, src_pitch elements per row) to dst->dtype
 * storage at dst->data: F16 with round-to-nearest-even, or U8 as
 * round(clamp(v / dst->scale, 0, 255)). */
sgn_status sgn_quantize(sgn_ctx* ctx, const float* src, int32_t src_pitch, const sgn_image* dst);

/* Milliseconds of the last fused Gauss-Newton kernel launched by this context
 * (HIP events on the context's stream around that kernel alone; waits for it). */
sgn_status sgn_last_kernel_ms(sgn_ctx* ctx, float* ms_out);

/* Milliseconds of the last n fused Gauss-Newton kernels of this context
 * (tile or disc), oldest first, into ms_out (host, n floats): the same HIP
 * events as sgn_last_kernel_ms, kept for the last 64 launches, so a caller
 * can time many launches without waiting between them.  Waits for the
 * kernels.  Errors: n outside [1, min(launches, 64)] (SGN_E_INVALID). */
sgn_status sgn_recent_kernel_ms(sgn_ctx* ctx, int32_t n, float* ms_out);

sgn_status sgn_device_info(int32_t device, sgn_device_props* out);
const char* sgn_status_str(sgn_status status);
const char* sgn_last_error(void);
const char* sgn_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SURFGN_H */
