/*
 * sgo.h -- plain FP64 CPU oracle of the per-surfel Gauss-Newton update.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this code; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source with the HIP path.
 *
 * Paper: "Dense monocular SLAM by direct surfel optimization" (Trabes,
 * Dondo Gazzano, Sosa Paez).  Section and equation numbers below are the
 * paper's.  All arithmetic is IEEE double, no fast-math, no reordering
 * beyond what the equations state.
 *
 * Conventions (where the paper is silent; each is a stated reading):
 *   - camera x right, y down, z forward; pixel (x, y) has its centre at
 *     integer coordinates and homogeneous form u~ = (x, y, 1);
 *   - a keyframe is tiled into S x S surfels; tile (tx, ty) owns pixels
 *     [S tx, S tx + S) x [S ty, S ty + S) and its centre pixel is
 *     u_s = (S tx + (S-1)/2, S ty + (S-1)/2); r_s = K^-1 u~_s (z = 1);
 *   - a pose P_kf^fn is stored as X_n = R X_kf + t with R row-major;
 *   - images are row-major doubles, width entries per row.
 */
#ifndef SGO_H
#define SGO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double fx, fy, cx, cy; } sgo_intrinsics;
typedef struct { double R[9]; double t[3]; } sgo_pose;
typedef struct { const double* pix; int32_t width, height; } sgo_image;

typedef struct {
    sgo_image kf;             /* I_kf */
    const sgo_image* nbr;     /* I_fn, n = 0 .. n_nbr-1 (the group Omega) */
    const sgo_pose* pose;     /* P_kf^fn */
    int32_t n_nbr;
    sgo_intrinsics K;
    int32_t patch;            /* S */
} sgo_keyframe;

/* Surfel grid, structure of arrays, length gw*gh, index ty*gw + tx. */
typedef struct {
    double* inv_depth;        /* id_s */
    double* nx; double* ny; double* nz;  /* n_s */
    uint32_t* flags;
    double* cost;             /* Huber cost at the last linearisation point */
    int32_t* nvalid;          /* valid (pixel, frame) samples at that point */
    uint32_t* last_update;
    double* kappa;            /* optional (may be NULL): cond_2 of the equilibrated J^T J */
    double* margin;           /* optional test probe (may be NULL): smallest distance, over
                                 all samples and iterations, of a warped point from the edge
                                 of the valid sampling window (pixels) */
} sgo_surfels;

typedef struct {
    int32_t iters;            /* Gauss-Newton iterations */
    double huber_k;           /* Huber threshold (intensity units) */
    int32_t depth_only;       /* ablation: d id_u / d n_s := 0 */
    double beta_r;            /* neighbour radius for initialisation (pixels) */
    uint32_t stamp;           /* written to last_update */
    double lm_lambda;         /* 0: pure Gauss-Newton; >0: Levenberg-Marquardt start damping */
    double perturb;           /* test probe, 0 = off: scale each entry of the normal equations
                                 and, after every accepted step, id_s and each normal component
                                 by (1 + perturb * u), u in [-1, 1) from a counter hash of
                                 (perturb_seed, surfel, iteration, component) */
    uint32_t perturb_seed;
    int32_t perturb_parts;    /* which parts the probe perturbs, a bit set: 1 = the normal
                                 equations, 2 = the state after accepted steps, 4 = the damped
                                 variant's acceptance threshold (cost / nvalid scaled by
                                 (1 + tie_window * u)); 0 = all three */
    double tie_window;        /* test probe: the acceptance threshold's relative noise (bit 4 of
                                 perturb_parts); 0 = perturb */
} sgo_params;

enum {
    SGO_DEGENERATE  = 1u << 0,  /* |n_s . r_s| < 1e-6: plane through the camera centre */
    SGO_FEW_SAMPLES = 1u << 1,  /* fewer than 3 valid samples */
    SGO_SOLVE_FAIL  = 1u << 2,  /* J^T J not positive definite */
    SGO_REJECTED    = 1u << 3,  /* update non-finite or id_s <= 0 */
    SGO_FP64_SOLVE  = 1u << 4,  /* (device only) solved in double */
    SGO_UNINIT      = 1u << 5   /* no neighbour available for initialisation */
};

/* Eq. 2 ray r_u = K^-1 pi^-1(u) for pixel (x, y). */
void sgo_ray(const sgo_intrinsics* K, double x, double y, double r[3]);

/* Eq. 3: inverse depth of pixel u on the plane of a surfel (centre pixel us,
 * inverse depth id_s, normal n). */
double sgo_pixel_inverse_depth(const sgo_intrinsics* K, double usx, double usy,
                               double id_s, const double n[3], double ux, double uy);

/* Eq. 6: coordinates u_p in frame n of keyframe pixel u at inverse depth id_u.
 * Returns 0 when the point is not in front of the frame's camera. */
int sgo_warp(const sgo_intrinsics* K, const sgo_pose* P, double ux, double uy,
             double id_u, double uv[2]);

/* Bilinear interpolant of an image and its exact gradient at (x, y).
 * out = {value, d/dx, d/dy}.  Returns 0 outside 0 <= x < w-1, 0 <= y < h-1. */
int sgo_bilinear(const sgo_image* I, double x, double y, double out[3]);

/* Orthonormal tangent basis of a unit normal. */
void sgo_tangent_basis(const double n[3], double b1[3], double b2[3]);

/* One sample: residual r = I_fn(u_p) - I_kf(u) and its Jacobian row with
 * respect to (id_s, alpha_1, alpha_2), where n(alpha) = normalise(n + a1 b1 +
 * a2 b2).  Returns 1 when the sample is valid. */
int sgo_eval_sample(const sgo_intrinsics* K, const sgo_pose* P, const sgo_image* In,
                    double kf_value, double usx, double usy, double ux, double uy,
                    double id_s, const double n[3], int depth_only,
                    double* r, double J[3]);

/* Huber IRLS normal equations of one surfel at its current state.
 * H is 3x3 row-major.  Returns the number of valid samples. */
int32_t sgo_linearize(const sgo_keyframe* kf, int32_t tx, int32_t ty, double id_s,
                      const double n[3], double huber_k, int depth_only,
                      double H[9], double b[3], double* cost);

/* Cholesky solve of H delta = -b; returns 0 on success, SGO_SOLVE_FAIL when a
 * pivot is <= 1e-12 * max diag (or not finite). */
uint32_t sgo_solve3(const double H[9], const double b[3], double delta[3]);

/* 2-norm condition number of D^-1/2 H D^-1/2, D = diag(H) (inf if singular). */
double sgo_kappa_eq(const double H[9]);

/* Gauss-Newton over all surfels (subset == NULL) or the listed surfel indices. */
int sgo_optimize_keyframe(const sgo_keyframe* kf, sgo_surfels* s, const sgo_params* p,
                          const int32_t* subset, int32_t n_subset);

/* Huber cost and valid-sample count of the surfels idx[0 .. n-1] at the
 * states (id_s[i], n[i]) (arrays indexed by surfel): tiles, or discs of the
 * given radius centred at (disc_ux[i], disc_uy[i]) when disc_ux is not NULL.
 * Test use: judging the end points of different optimisation runs. */
int sgo_costs_at(const sgo_keyframe* kf, const double* id_s, const double* nx, const double* ny,
                 const double* nz, const int32_t* idx, int32_t n, double huber_k,
                 const double* disc_ux, const double* disc_uy, double radius, double* cost_out,
                 int32_t* nvalid_out);

/* Neighbour-plane initialisation of surfels with is_new[i] != 0. */
int sgo_init_from_neighbours(const sgo_keyframe* kf, sgo_surfels* s, const uint8_t* is_new,
                             const sgo_params* p, const int32_t* subset, int32_t n_subset);

/* Per-pixel inverse depth (0 = no measurement) and owning surfel (-1 = none). */
int sgo_render_inverse_depth(const sgo_keyframe* kf, const sgo_surfels* s,
                             double* inv_depth, int32_t* surfel_index);

/* Eq. 10: move surfels of keyframe kf0 into keyframe kf1 (pose X1 = R X0 + t).
 * For each input surfel (ray r_s, id_s, n) returns the transformed point's
 * pixel (x, y), inverse depth and rotated normal.  Returns count of surfels in
 * front of the new camera (others get id = 0). */
int sgo_transfer_surfels(const sgo_intrinsics* K, const sgo_pose* P, int32_t count,
                         const double* usx, const double* usy, const double* id_s,
                         const double* n, double* ux_out, double* uy_out,
                         double* id_out, double* n_out);

/* A keyframe's surfel grid: intrinsics, image size and tile edge S. */
typedef struct { sgo_intrinsics K; int32_t width, height, patch; } sgo_grid;

/* Surfel reference-frame change (Eq. 10) and re-gridding into the tiles of
 * another keyframe (pose X_dst = R X_src + t).  A usable source surfel (no
 * DEGENERATE or UNINIT flag, id_s > 0) moves to p' = R (r_s / id_s) + t with
 * normal n' = R n, and lands in the destination pixel nearest to
 * pi(K_dst p'), hence in that pixel's tile.  In each destination tile the
 * closest landed surfel wins (largest 1/p'_z, ties to the lower source
 * index); its plane is re-expressed at the tile's centre ray r_t by Eq. 3:
 * id_t = (1/p'_z) (n'.r_t) / (n'.r'), r' = p'/p'_z, n_t = n' normalised.
 * Tiles that receive nothing, or whose plane cannot be evaluated at r_t, get
 * id 0, n (0, 0, -1), the UNINIT flag and is_new = 1 (for neighbour
 * initialisation).  dst_src_index (may be NULL) receives the winning source
 * index or -1.  Returns the number of filled destination tiles. */
int sgo_transfer_regrid(const sgo_grid* src_grid, const sgo_surfels* src, const sgo_pose* P,
                        const sgo_grid* dst_grid, sgo_surfels* dst, uint8_t* dst_is_new,
                        int32_t* dst_src_index);

/* Disc surfels (Eq. 4).  Surfel i is centred at pixel (ux[i], uy[i]) of the
 * keyframe and covers the pixels u (integer coordinates, inside the image)
 * with |u - u_s| < r; r (pixels) is the same for every surfel.  The state
 * arrays are indexed by surfel, length count.  kf->patch is not used. */

/* Pixels of one disc, row by row: writes the first `capacity`, returns the count. */
int32_t sgo_disc_support(int32_t width, int32_t height, double usx, double usy, double radius,
                         int32_t* xs, int32_t* ys, int32_t capacity);

/* Huber IRLS normal equations of one disc surfel (as sgo_linearize). */
int32_t sgo_disc_linearize(const sgo_keyframe* kf, double usx, double usy, double radius,
                           double id_s, const double n[3], double huber_k, int depth_only,
                           double H[9], double b[3], double* cost);

/* Gauss-Newton over all disc surfels (subset == NULL) or the listed ones. */
int sgo_disc_optimize(const sgo_keyframe* kf, sgo_surfels* s, const double* ux, const double* uy,
                      int32_t count, double radius, const sgo_params* p,
                      const int32_t* subset, int32_t n_subset);

/* Depth-buffered render: per pixel the largest Eq. 3 inverse depth over the
 * discs that contain it (ties to the lower index), 0 and -1 where none. */
int sgo_disc_render(const sgo_keyframe* kf, const sgo_surfels* s, const double* ux,
                    const double* uy, int32_t count, double radius, double* inv_depth,
                    int32_t* surfel_index);

/* Empty-area search on the lattice (spacing/2 + i spacing, spacing/2 + j
 * spacing): candidates farther than alpha r from every non-empty pixel of
 * the index map.  Writes the first `capacity`, returns how many qualify. */
int32_t sgo_disc_search(int32_t width, int32_t height, const int32_t* surfel_index,
                        double radius, double alpha, int32_t spacing, int32_t* out_x,
                        int32_t* out_y, int32_t capacity);

/* Neighbour initialisation of disc surfels first .. first + n_new - 1 from
 * the surfels below `first` that own a pixel of the index map closer than
 * beta r to the new centre. */
int sgo_disc_init(const sgo_keyframe* kf, sgo_surfels* s, const double* ux, const double* uy,
                  const int32_t* surfel_index, int32_t first, int32_t n_new, double radius,
                  double beta);

/* Eq. 10 for disc surfels: usable surfels move to p' = R p + t, n' = R n and
 * are re-centred at K_dst pi(p'); those landing in the destination image are
 * written in source order (first `capacity`).  Returns the number written. */
int32_t sgo_disc_transfer(const sgo_intrinsics* Ks, const sgo_intrinsics* Kd, int32_t dst_w,
                          int32_t dst_h, const sgo_pose* P, const sgo_surfels* src,
                          const double* ux, const double* uy, int32_t count, sgo_surfels* dst,
                          double* dux, double* duy, int32_t capacity, int32_t* src_index,
                          int32_t* landed_out);

void sgo_set_threads(int32_t n);
int32_t sgo_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
