/*
 * sgo.c -- plain FP64 CPU oracle of the per-surfel Gauss-Newton update.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing).  It
 * shares no code with the HIP path.  See sgo.h for conventions.
 *
 * Structure follows the paper's Proposed Approach section:
 *   Eq. 1  p_s = r_s / id_s                       (surfel point)
 *   Eq. 2  r_u = K^-1 pi^-1(u)                    (pixel ray, z = 1)
 *   Eq. 3  id_u = (r_u . n_s) / ((r_s / id_s) . n_s)
 *   Eq. 5  C = sum_n sum_u huber(I_fn(u_p) - I_kf(u))
 *   Eq. 6  u_p = pi(K P_kf^fn (K^-1 u~ / id_u))   (printed with pi / pi^-1
 *          swapped; read as the projection of the back-projected point)
 *   Eq. 7-9 chain rule J = dC/did_u * did_u/d[n_s, id_s]
 *   normal updated with three components then renormalised (Surfel
 *   Optimization section, last paragraph)
 *   Surfel Initialization section: mean of neighbours' Eq. 3 inverse depths
 *   at the new ray, mean of their normals.
 *   Eq. 10 reference-frame change.
 *   Eq. 4 disc surfels: support |u_s - u| < r, depth-buffered render with a
 *   surfel-index map, the search for empty areas and neighbour
 *   initialisation from that map (Inverse Depth Calculation and Surfel
 *   Initialization sections).
 * Nothing is blocked, fused or hoisted: every (pixel, frame) sample forms its
 * own full Jacobian row and is added to J^T W J and J^T W r directly.
 */
#include "sgo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static int normalize3(double v[3]) {
    double l = sqrt(dot3(v, v));
    if (!(l > 0.0) || !isfinite(l)) return 0;
    v[0] /= l; v[1] /= l; v[2] /= l;
    return 1;
}

/* Eq. 2: r_u = K^-1 [x, y, 1]^T. */
void sgo_ray(const sgo_intrinsics* K, double x, double y, double r[3]) {
    r[0] = (x - K->cx) / K->fx;
    r[1] = (y - K->cy) / K->fy;
    r[2] = 1.0;
}

/* Eq. 3 as printed: id_u = (r_u . n_s) / ((r_s / id_s) . n_s). */
double sgo_pixel_inverse_depth(const sgo_intrinsics* K, double usx, double usy,
                               double id_s, const double n[3], double ux, double uy) {
    double rs[3], ru[3], ps[3];
    sgo_ray(K, usx, usy, rs);
    sgo_ray(K, ux, uy, ru);
    ps[0] = rs[0] / id_s; ps[1] = rs[1] / id_s; ps[2] = rs[2] / id_s;  /* Eq. 1 */
    return dot3(ru, n) / dot3(ps, n);
}

/* Eq. 6: X = r_u / id_u, X_n = R X + t, u_p = pi(K X_n). */
static int warp_point(const sgo_intrinsics* K, const sgo_pose* P, const double ru[3],
                      double id_u, double Xn[3], double uv[2]) {
    double X[3] = {ru[0] / id_u, ru[1] / id_u, ru[2] / id_u};
    for (int i = 0; i < 3; ++i)
        Xn[i] = P->R[3 * i] * X[0] + P->R[3 * i + 1] * X[1] + P->R[3 * i + 2] * X[2] + P->t[i];
    if (!(Xn[2] > 0.0)) return 0;
    uv[0] = K->fx * Xn[0] / Xn[2] + K->cx;
    uv[1] = K->fy * Xn[1] / Xn[2] + K->cy;
    return 1;
}

int sgo_warp(const sgo_intrinsics* K, const sgo_pose* P, double ux, double uy,
             double id_u, double uv[2]) {
    double ru[3], Xn[3];
    sgo_ray(K, ux, uy, ru);
    return warp_point(K, P, ru, id_u, Xn, uv);
}

/* Bilinear interpolation of the four pixels around (x, y) and the exact
 * derivative of that interpolant (the image gradient nabla I_fn of Eq. 8). */
int sgo_bilinear(const sgo_image* I, double x, double y, double out[3]) {
    if (!(x >= 0.0 && y >= 0.0 && x < (double)(I->width - 1) && y < (double)(I->height - 1)))
        return 0;
    int x0 = (int)floor(x), y0 = (int)floor(y);
    double ax = x - x0, ay = y - y0;
    const double* row0 = I->pix + (size_t)y0 * I->width;
    const double* row1 = row0 + I->width;
    double i00 = row0[x0], i01 = row0[x0 + 1], i10 = row1[x0], i11 = row1[x0 + 1];
    double top = i00 + ax * (i01 - i00);
    double bot = i10 + ax * (i11 - i10);
    out[0] = top + ay * (bot - top);
    out[1] = (i01 - i00) + ay * ((i11 - i10) - (i01 - i00));
    out[2] = bot - top;
    return 1;
}

void sgo_tangent_basis(const double n[3], double b1[3], double b2[3]) {
    double e[3] = {0.0, 0.0, 0.0};
    if (fabs(n[0]) < 0.9) e[0] = 1.0; else e[1] = 1.0;
    double en = dot3(e, n);
    b1[0] = e[0] - en * n[0]; b1[1] = e[1] - en * n[1]; b1[2] = e[2] - en * n[2];
    normalize3(b1);
    cross3(n, b1, b2);
}

/* Huber norm of Eq. 5 and its IRLS weight w (Eq. 8: dC/dI_f = w r). */
static double huber_rho(double r, double k) {
    double a = fabs(r);
    return a <= k ? 0.5 * r * r : k * a - 0.5 * k * k;
}
/* w = min(1, k/|r|), the minimum taken as IEEE minNum: a residual that is
 * not a number gets weight 1, so its term of J^T W r and its cost stay not a
 * number while J^T W J keeps its finite value. */
static double huber_w(double r, double k) {
    double a = fabs(r);
    return fmin(1.0, k / a);
}

/* Residual and Jacobian row of one (pixel, frame) sample, by the chain rule
 * of Eq. 7-9:
 *   dr/dtheta = nabla I_fn(u_p) * dpi/dq * dq/did_u * did_u/dtheta
 * with did_u/did_s from Eq. 9 (correct as printed) and did_u/dn_s the exact
 * derivative of Eq. 3 (the printed form collapses to zero; reading:
 * id_s (r_u (n.r_s) - r_s (n.r_u)) / (n.r_s)^2), projected on the tangent
 * basis because the normal is updated and then renormalised. */
static int eval_sample(const sgo_intrinsics* K, const sgo_pose* P, const sgo_image* In,
                       double kf_value, double usx, double usy, double ux, double uy,
                       double id_s, const double n[3], int depth_only, double* r, double J[3],
                       double* margin);

int sgo_eval_sample(const sgo_intrinsics* K, const sgo_pose* P, const sgo_image* In,
                    double kf_value, double usx, double usy, double ux, double uy,
                    double id_s, const double n[3], int depth_only,
                    double* r, double J[3]) {
    return eval_sample(K, P, In, kf_value, usx, usy, ux, uy, id_s, n, depth_only, r, J, NULL);
}

/* margin (test probe, may be NULL): lowered to the distance of the warped
 * point from the nearest edge of the valid sampling window, so that a caller
 * can tell which validity decisions are close calls. */
static int eval_sample(const sgo_intrinsics* K, const sgo_pose* P, const sgo_image* In,
                       double kf_value, double usx, double usy, double ux, double uy,
                       double id_s, const double n[3], int depth_only, double* r, double J[3],
                       double* margin) {
    double rs[3], ru[3];
    sgo_ray(K, usx, usy, rs);
    sgo_ray(K, ux, uy, ru);
    double ps[3] = {rs[0] / id_s, rs[1] / id_s, rs[2] / id_s};  /* Eq. 1 */
    double ru_n = dot3(ru, n), rs_n = dot3(rs, n);
    double id_u = ru_n / dot3(ps, n);                            /* Eq. 3 */
    if (!(id_u > 0.0) || !isfinite(id_u)) return 0;
    double Xn[3], uv[2];
    if (!warp_point(K, P, ru, id_u, Xn, uv)) return 0;           /* Eq. 6 */
    if (margin) {
        double m = fmin(fmin(fabs(uv[0]), fabs(uv[0] - (In->width - 1))),
                        fmin(fabs(uv[1]), fabs(uv[1] - (In->height - 1))));
        if (m < *margin) *margin = m;
    }
    double s[3];
    if (!sgo_bilinear(In, uv[0], uv[1], s)) return 0;
    *r = s[0] - kf_value;
    /* Eq. 8 chain with the projection read as pi(q), where q is the point's
     * homogeneous pixel K X_n scaled by id_u (pi is scale invariant):
     *   q = id_u K X_n = K R r_u + id_u K t,   so  dq/did_u = K t
     * (the printed du_p/did_u is the derivative with respect to depth, not
     * inverse depth), and dpi/dq = (1/q_z) [[1, 0, -u_x], [0, 1, -u_y]]
     * (the printed matrix repeats -u_y and drops 1/q_z). */
    double Kt[3] = {K->fx * P->t[0] + K->cx * P->t[2], K->fy * P->t[1] + K->cy * P->t[2], P->t[2]};
    double qz = id_u * Xn[2];
    double du[2];
    du[0] = (Kt[0] - uv[0] * Kt[2]) / qz;
    du[1] = (Kt[1] - uv[1] * Kt[2]) / qz;
    double dr_did_u = s[1] * du[0] + s[2] * du[1];               /* Eq. 8 */
    /* Eq. 9 */
    double did_dids = ru_n / rs_n;
    double dn[3];
    for (int i = 0; i < 3; ++i)
        dn[i] = id_s * (ru[i] * rs_n - rs[i] * ru_n) / (rs_n * rs_n);
    double b1[3], b2[3];
    sgo_tangent_basis(n, b1, b2);
    J[0] = dr_did_u * did_dids;
    if (depth_only) {
        J[1] = 0.0;
        J[2] = 0.0;
    } else {
        J[1] = dr_did_u * dot3(dn, b1);
        J[2] = dr_did_u * dot3(dn, b2);
    }
    return 1;
}

static void tile_centre(const sgo_keyframe* kf, int32_t tx, int32_t ty, double* x, double* y) {
    int S = kf->patch;
    *x = S * tx + 0.5 * (S - 1);
    *y = S * ty + 0.5 * (S - 1);
}

/* Pixel support of one surfel (the pixels u of "u in s" in Eq. 5): the
 * candidate pixels are the box [x0, x1] x [y0, y1] (inclusive, inside the
 * image).  For a tile every box pixel belongs; for a disc (Eq. 4) a box
 * pixel u belongs when |u - u_s| < r, decided as dx^2 + dy^2 < r^2 in
 * double. */
typedef struct {
    double usx, usy;          /* centre pixel u_s */
    int x0, y0, x1, y1;
    double r2;                /* disc: r^2; tile: negative */
} support;

static support tile_support(const sgo_keyframe* kf, int32_t tx, int32_t ty) {
    support sp;
    int S = kf->patch;
    tile_centre(kf, tx, ty, &sp.usx, &sp.usy);
    sp.x0 = S * tx; sp.x1 = S * tx + S - 1;
    sp.y0 = S * ty; sp.y1 = S * ty + S - 1;
    sp.r2 = -1.0;
    return sp;
}

static support disc_support(int32_t width, int32_t height, double usx, double usy, double r) {
    support sp;
    sp.usx = usx; sp.usy = usy;
    sp.r2 = r * r;
    sp.x0 = (int)fmax(0.0, ceil(usx - r));
    sp.x1 = (int)fmin((double)(width - 1), floor(usx + r));
    sp.y0 = (int)fmax(0.0, ceil(usy - r));
    sp.y1 = (int)fmin((double)(height - 1), floor(usy + r));
    return sp;
}

static int in_support(const support* sp, int x, int y) {
    if (sp->r2 < 0.0) return 1;
    double dx = (double)x - sp->usx, dy = (double)y - sp->usy;
    return dx * dx + dy * dy < sp->r2;
}

static int32_t linearize(const sgo_keyframe* kf, const support* sp, double id_s,
                         const double n[3], double huber_k, int depth_only, double H[9],
                         double b[3], double* cost, double* margin);

int32_t sgo_linearize(const sgo_keyframe* kf, int32_t tx, int32_t ty, double id_s,
                      const double n[3], double huber_k, int depth_only,
                      double H[9], double b[3], double* cost) {
    support sp = tile_support(kf, tx, ty);
    return linearize(kf, &sp, id_s, n, huber_k, depth_only, H, b, cost, NULL);
}

int32_t sgo_disc_linearize(const sgo_keyframe* kf, double usx, double usy, double radius,
                           double id_s, const double n[3], double huber_k, int depth_only,
                           double H[9], double b[3], double* cost) {
    support sp = disc_support(kf->kf.width, kf->kf.height, usx, usy, radius);
    return linearize(kf, &sp, id_s, n, huber_k, depth_only, H, b, cost, NULL);
}

int32_t sgo_disc_support(int32_t width, int32_t height, double usx, double usy, double radius,
                         int32_t* xs, int32_t* ys, int32_t capacity) {
    support sp = disc_support(width, height, usx, usy, radius);
    int32_t count = 0;
    for (int y = sp.y0; y <= sp.y1; ++y)
        for (int x = sp.x0; x <= sp.x1; ++x) {
            if (!in_support(&sp, x, y)) continue;
            if (count < capacity) { xs[count] = x; ys[count] = y; }
            ++count;
        }
    return count;
}

static int32_t linearize(const sgo_keyframe* kf, const support* sp, double id_s,
                         const double n[3], double huber_k, int depth_only, double H[9],
                         double b[3], double* cost, double* margin) {
    memset(H, 0, 9 * sizeof(double));
    memset(b, 0, 3 * sizeof(double));
    *cost = 0.0;
    int32_t nvalid = 0;
    for (int uy = sp->y0; uy <= sp->y1; ++uy) {
        for (int ux = sp->x0; ux <= sp->x1; ++ux) {
            if (!in_support(sp, ux, uy)) continue;
            double ikf = kf->kf.pix[(size_t)uy * kf->kf.width + ux];
            for (int f = 0; f < kf->n_nbr; ++f) {               /* sum over Omega */
                double r, J[3];
                if (!eval_sample(&kf->K, &kf->pose[f], &kf->nbr[f], ikf, sp->usx, sp->usy,
                                 (double)ux, (double)uy, id_s, n, depth_only, &r, J, margin))
                    continue;
                double w = huber_w(r, huber_k);
                for (int i = 0; i < 3; ++i) {
                    for (int j = 0; j < 3; ++j) H[3 * i + j] += w * J[i] * J[j];
                    b[i] += w * J[i] * r;
                }
                *cost += huber_rho(r, huber_k);
                ++nvalid;
            }
        }
    }
    return nvalid;
}

/* Textbook Cholesky H = L L^T, then forward/back substitution for
 * H delta = -b.  A pivot <= 1e-12 * max diag(H) means "not positive
 * definite". */
uint32_t sgo_solve3(const double H[9], const double b[3], double delta[3]) {
    double L[3][3] = {{0}};
    double maxd = fmax(H[0], fmax(H[4], H[8]));
    if (!(maxd > 0.0) || !isfinite(maxd)) return SGO_SOLVE_FAIL;
    double tol = 1e-12 * maxd;
    for (int j = 0; j < 3; ++j) {
        double d = H[3 * j + j];
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        if (!(d > tol) || !isfinite(d)) return SGO_SOLVE_FAIL;
        L[j][j] = sqrt(d);
        for (int i = j + 1; i < 3; ++i) {
            double v = H[3 * i + j];
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            L[i][j] = v / L[j][j];
        }
    }
    double y[3];
    for (int i = 0; i < 3; ++i) {
        double v = -b[i];
        for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
        y[i] = v / L[i][i];
    }
    for (int i = 2; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < 3; ++k) v -= L[k][i] * delta[k];
        delta[i] = v / L[i][i];
    }
    return 0;
}

/* Eigenvalues of a symmetric 3x3 matrix by cyclic Jacobi rotations. */
static void sym_eig3(const double A_in[9], double ev[3]) {
    double A[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = A_in[3 * i + j];
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        double diag = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-34 * diag || off == 0.0) break;
        for (int p = 0; p < 2; ++p) {
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) {   /* A <- A J */
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {   /* A <- J^T A */
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
            }
        }
    }
    ev[0] = A[0][0]; ev[1] = A[1][1]; ev[2] = A[2][2];
}

double sgo_kappa_eq(const double H[9]) {
    double d[3];
    for (int i = 0; i < 3; ++i) {
        if (!(H[4 * i] > 0.0) || !isfinite(H[4 * i])) return INFINITY;
        d[i] = 1.0 / sqrt(H[4 * i]);
    }
    double E[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) E[3 * i + j] = d[i] * H[3 * i + j] * d[j];
    double ev[3];
    sym_eig3(E, ev);
    double lo = fmin(ev[0], fmin(ev[1], ev[2])), hi = fmax(ev[0], fmax(ev[1], ev[2]));
    if (!(lo > 0.0)) return INFINITY;
    return hi / lo;
}

/* Normal update with three components then renormalisation (Surfel
 * Optimization section): the tangent step (alpha_1, alpha_2) is the 3-DOF
 * step n + a1 b1 + a2 b2, renormalised. */
static int apply_update(double id_s, const double n[3], const double b1[3], const double b2[3],
                        const double delta[3], int depth_only, double* id_new, double n_new[3]) {
    *id_new = id_s + delta[0];
    if (depth_only) {          /* only id_s is a parameter of the ablation */
        n_new[0] = n[0]; n_new[1] = n[1]; n_new[2] = n[2];
        return *id_new > 0.0 && isfinite(*id_new);
    }
    for (int i = 0; i < 3; ++i) n_new[i] = n[i] + delta[1] * b1[i] + delta[2] * b2[i];
    if (!normalize3(n_new)) return 0;
    if (!(*id_new > 0.0) || !isfinite(*id_new)) return 0;
    return 1;
}

/* Conditioning probe (test use only): a uniform number in [-1, 1) from a
 * 64-bit mix of (seed, surfel, iteration, component) (splitmix64 finaliser). */
static double probe_uniform(uint32_t seed, int32_t surfel, int it, int comp) {
    uint64_t z = ((uint64_t)seed << 40) ^ ((uint64_t)(uint32_t)surfel << 12) ^ ((uint64_t)it << 3) ^
                 (uint64_t)comp;
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static void optimize_one(const sgo_keyframe* kf, sgo_surfels* s, const sgo_params* p, int32_t i,
                         const support* sp) {
    double rs[3];
    sgo_ray(&kf->K, sp->usx, sp->usy, rs);
    double id_s = s->inv_depth[i];
    double n[3] = {s->nx[i], s->ny[i], s->nz[i]};
    uint32_t flags = s->flags[i] & ~(uint32_t)(SGO_DEGENERATE | SGO_FEW_SAMPLES | SGO_SOLVE_FAIL |
                                              SGO_REJECTED | SGO_FP64_SOLVE);
    double cost = 0.0, kappa = 0.0;
    int32_t nvalid = 0;
    int updated = 0;
    double lambda = p->lm_lambda;
    double margin = INFINITY;
    for (int it = 0; it < p->iters; ++it) {
        if (fabs(dot3(n, rs)) < 1e-6) {           /* Eq. 3 undefined */
            flags |= SGO_DEGENERATE;
            cost = 0.0;
            nvalid = 0;
            break;
        }
        double b1[3], b2[3];
        sgo_tangent_basis(n, b1, b2);
        double H[9], b[3];
        nvalid = linearize(kf, sp, id_s, n, p->huber_k, p->depth_only, H, b, &cost,
                           s->margin ? &margin : NULL);
        kappa = p->depth_only ? 1.0 : sgo_kappa_eq(H);
        double delta[3] = {0.0, 0.0, 0.0};
        if (nvalid < 3) {
            flags |= SGO_FEW_SAMPLES;
            continue;
        }
        const int probe_ne = p->perturb > 0.0 && (p->perturb_parts & 1 || p->perturb_parts == 0);
        const int probe_state = p->perturb > 0.0 && (p->perturb_parts & 2 || p->perturb_parts == 0);
        const int probe_decision = p->perturb > 0.0 && (p->perturb_parts & 4 || p->perturb_parts == 0);
        if (probe_ne) {
            /* probe: relative noise on the normal equations as well (float
             * accumulation of J^T W J and J^T W r reaches the step scaled by
             * the condition number, which state noise alone does not model) */
            int comp = 4;
            for (int a = 0; a < 3; ++a)
                for (int c = a; c < 3; ++c) {
                    H[3 * a + c] *= 1.0 + p->perturb * probe_uniform(p->perturb_seed, i, it, comp++);
                    H[3 * c + a] = H[3 * a + c];
                }
            for (int a = 0; a < 3; ++a)
                b[a] *= 1.0 + p->perturb * probe_uniform(p->perturb_seed, i, it, comp++);
        }
        double Hs[9];
        memcpy(Hs, H, sizeof(Hs));
        if (lambda > 0.0)                          /* Levenberg-Marquardt damping */
            for (int k = 0; k < 3; ++k) Hs[4 * k] *= 1.0 + lambda;
        if (p->depth_only) {
            if (!(Hs[0] > 0.0) || !isfinite(Hs[0])) {
                flags |= SGO_SOLVE_FAIL;
                continue;
            }
            delta[0] = -b[0] / Hs[0];
        } else {
            uint32_t st = sgo_solve3(Hs, b, delta);
            if (st) {
                flags |= st;
                continue;
            }
        }
        double id_new, n_new[3];
        if (!apply_update(id_s, n, b1, b2, delta, p->depth_only, &id_new, n_new)) {
            flags |= SGO_REJECTED;
            if (lambda > 0.0) lambda *= 10.0;
            continue;
        }
        if (lambda > 0.0) {
            /* Levenberg-Marquardt acceptance: the candidate is taken when
             * the mean Huber cost per valid sample does not rise (a rise of
             * any size is refused); a candidate plane that contains the
             * centre ray is refused as well */
            if (fabs(dot3(n_new, rs)) < 1e-6) {
                flags |= SGO_REJECTED;
                lambda *= 10.0;
                continue;
            }
            double H2[9], b2v[3], cost2;
            int32_t nv2 = linearize(kf, sp, id_new, n_new, p->huber_k, p->depth_only, H2,
                                    b2v, &cost2, s->margin ? &margin : NULL);
            /* probe: a relative tie window on the comparison (a float cost
             * sum decides near-ties either way) */
            double bar = cost / nvalid;
            if (probe_decision)
                bar *= 1.0 + (p->tie_window > 0.0 ? p->tie_window : p->perturb) *
                                 probe_uniform(p->perturb_seed, i, it, 16);
            if (nv2 < 3 || !(cost2 / nv2 <= bar)) {
                lambda *= 10.0;
                continue;
            }
            lambda = fmax(lambda * 0.1, 1e-9);
        }
        if (probe_state) {
            id_new *= 1.0 + p->perturb * probe_uniform(p->perturb_seed, i, it, 0);
            if (!p->depth_only) {
                for (int k = 0; k < 3; ++k)
                    n_new[k] *= 1.0 + p->perturb * probe_uniform(p->perturb_seed, i, it, 1 + k);
                normalize3(n_new);
            }
        }
        id_s = id_new;
        n[0] = n_new[0]; n[1] = n_new[1]; n[2] = n_new[2];
        updated = 1;
    }
    s->inv_depth[i] = id_s;
    s->nx[i] = n[0]; s->ny[i] = n[1]; s->nz[i] = n[2];
    s->flags[i] = flags;
    s->cost[i] = cost;
    s->nvalid[i] = nvalid;
    if (s->kappa) s->kappa[i] = kappa;
    if (s->margin) s->margin[i] = margin;
    if (updated) s->last_update[i] = p->stamp;
}

int sgo_optimize_keyframe(const sgo_keyframe* kf, sgo_surfels* s, const sgo_params* p,
                          const int32_t* subset, int32_t n_subset) {
    if (!kf || !s || !p || kf->patch <= 0) return -1;
    int S = kf->patch;
    int32_t total = (kf->kf.width / S) * (kf->kf.height / S);
    int32_t count = subset ? n_subset : total;
    int gw = kf->kf.width / S;
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t k = 0; k < count; ++k) {
        int32_t i = subset ? subset[k] : k;
        if (i >= 0 && i < total) {
            support sp = tile_support(kf, i % gw, i / gw);
            optimize_one(kf, s, p, i, &sp);
        }
    }
    return 0;
}

/* Gauss-Newton over disc surfels (Eq. 4 support, centres ux, uy). */
int sgo_disc_optimize(const sgo_keyframe* kf, sgo_surfels* s, const double* ux, const double* uy,
                      int32_t count, double radius, const sgo_params* p,
                      const int32_t* subset, int32_t n_subset) {
    if (!kf || !s || !ux || !uy || !p || !(radius > 0.0)) return -1;
    int32_t m = subset ? n_subset : count;
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t k = 0; k < m; ++k) {
        int32_t i = subset ? subset[k] : k;
        if (i >= 0 && i < count) {
            support sp = disc_support(kf->kf.width, kf->kf.height, ux[i], uy[i], radius);
            optimize_one(kf, s, p, i, &sp);
        }
    }
    return 0;
}

/* Huber cost (Eq. 5) and valid-sample count of listed surfels at given
 * states (test use: judging where an optimisation ended). */
int sgo_costs_at(const sgo_keyframe* kf, const double* id_s, const double* nx, const double* ny,
                 const double* nz, const int32_t* idx, int32_t n, double huber_k,
                 const double* disc_ux, const double* disc_uy, double radius, double* cost_out,
                 int32_t* nvalid_out) {
    if (!kf || !id_s || !nx || !ny || !nz || !idx || !cost_out || !nvalid_out) return -1;
    if (!disc_ux && kf->patch <= 0) return -1;
    const int gw = disc_ux ? 1 : kf->kf.width / kf->patch;
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t k = 0; k < n; ++k) {
        const int32_t i = idx[k];
        support sp = disc_ux ? disc_support(kf->kf.width, kf->kf.height, disc_ux[i], disc_uy[i], radius)
                             : tile_support(kf, i % gw, i / gw);
        double nn[3] = {nx[i], ny[i], nz[i]};
        double H[9], b[3], c;
        nvalid_out[k] = linearize(kf, &sp, id_s[i], nn, huber_k, 0, H, b, &c, NULL);
        cost_out[k] = c;
    }
    return 0;
}

/* Surfel Initialization section.  Neighbours of a new surfel at centre u_ns
 * are the surfels (not new, not flagged unusable) that own at least one pixel
 * closer than beta r to u_ns.  The new inverse depth is the mean over them of
 * Eq. 3 evaluated with the neighbour's plane at the new surfel's ray; the new
 * normal is the mean of their normals (sign-aligned to the first neighbour in
 * index order), renormalised. */
static void init_one(const sgo_keyframe* kf, sgo_surfels* s, const uint8_t* is_new,
                     const sgo_params* p, int32_t i) {
    int S = kf->patch;
    int gw = kf->kf.width / S, gh = kf->kf.height / S;
    int tx = i % gw, ty = i / gw;
    double ux, uy;
    tile_centre(kf, tx, ty, &ux, &uy);
    double br = p->beta_r;
    int reach = (int)ceil(br / S) + 1;
    double id_sum = 0.0, nsum[3] = {0.0, 0.0, 0.0}, nref[3] = {0.0, 0.0, 0.0};
    int count = 0;
    for (int ny = ty - reach; ny <= ty + reach; ++ny) {
        for (int nx = tx - reach; nx <= tx + reach; ++nx) {
            if (nx < 0 || ny < 0 || nx >= gw || ny >= gh) continue;
            int32_t j = ny * gw + nx;
            if (j == i || is_new[j]) continue;
            if (s->flags[j] & (SGO_UNINIT | SGO_DEGENERATE)) continue;
            /* does surfel j own a pixel within beta r of u_ns? */
            int near = 0;
            for (int py = 0; py < S && !near; ++py)
                for (int px = 0; px < S && !near; ++px) {
                    double dx = (S * nx + px) - ux, dy = (S * ny + py) - uy;
                    if (sqrt(dx * dx + dy * dy) < br) near = 1;
                }
            if (!near) continue;
            double nj[3] = {s->nx[j], s->ny[j], s->nz[j]};
            double jx, jy, rj[3];
            tile_centre(kf, nx, ny, &jx, &jy);
            sgo_ray(&kf->K, jx, jy, rj);
            if (fabs(dot3(nj, rj)) < 1e-6) continue;
            /* Eq. 3 with the neighbour's plane, at the new surfel's pixel */
            double id = sgo_pixel_inverse_depth(&kf->K, jx, jy, s->inv_depth[j], nj, ux, uy);
            if (count == 0) { nref[0] = nj[0]; nref[1] = nj[1]; nref[2] = nj[2]; }
            double sg = dot3(nj, nref) < 0.0 ? -1.0 : 1.0;
            id_sum += id;
            for (int k = 0; k < 3; ++k) nsum[k] += sg * nj[k];
            ++count;
        }
    }
    if (count == 0) {
        s->flags[i] |= SGO_UNINIT;
        return;
    }
    double id_new = id_sum / count;
    double n_new[3] = {nsum[0] / count, nsum[1] / count, nsum[2] / count};
    if (!normalize3(n_new) || !(id_new > 0.0) || !isfinite(id_new)) {
        s->flags[i] |= SGO_UNINIT;
        return;
    }
    s->inv_depth[i] = id_new;
    s->nx[i] = n_new[0]; s->ny[i] = n_new[1]; s->nz[i] = n_new[2];
    s->flags[i] &= ~(uint32_t)SGO_UNINIT;
}

int sgo_init_from_neighbours(const sgo_keyframe* kf, sgo_surfels* s, const uint8_t* is_new,
                             const sgo_params* p, const int32_t* subset, int32_t n_subset) {
    if (!kf || !s || !is_new || !p || kf->patch <= 0) return -1;
    int S = kf->patch;
    int32_t total = (kf->kf.width / S) * (kf->kf.height / S);
    int32_t count = subset ? n_subset : total;
    /* New surfels read only non-new ones, so the order does not matter. */
#pragma omp parallel for schedule(dynamic, 64)
    for (int32_t k = 0; k < count; ++k) {
        int32_t i = subset ? subset[k] : k;
        if (i >= 0 && i < total && is_new[i]) init_one(kf, s, is_new, p, i);
    }
    return 0;
}

/* Inverse Depth Calculation section: each pixel takes Eq. 3 of the surfel
 * that owns it (tiles do not overlap, so no depth test is needed). */
int sgo_render_inverse_depth(const sgo_keyframe* kf, const sgo_surfels* s,
                             double* inv_depth, int32_t* surfel_index) {
    int W = kf->kf.width, H = kf->kf.height, S = kf->patch;
    int gw = W / S, gh = H / S;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            size_t o = (size_t)y * W + x;
            inv_depth[o] = 0.0;
            if (surfel_index) surfel_index[o] = -1;
            int tx = x / S, ty = y / S;
            if (tx >= gw || ty >= gh) continue;
            int32_t i = ty * gw + tx;
            if (s->flags[i] & (SGO_DEGENERATE | SGO_UNINIT)) continue;
            double n[3] = {s->nx[i], s->ny[i], s->nz[i]};
            double usx, usy, rs[3];
            tile_centre(kf, tx, ty, &usx, &usy);
            sgo_ray(&kf->K, usx, usy, rs);
            if (fabs(dot3(n, rs)) < 1e-6) continue;
            double id = sgo_pixel_inverse_depth(&kf->K, usx, usy, s->inv_depth[i], n, x, y);
            if (!(id > 0.0) || !isfinite(id)) continue;
            inv_depth[o] = id;
            if (surfel_index) surfel_index[o] = i;
        }
    }
    return 0;
}

/* Inverse Depth Calculation section with disc surfels: pixel u takes Eq. 3
 * of every surfel whose disc (Eq. 4) contains it, and the depth buffer keeps
 * the closest one (the largest id_u; equal values go to the lower surfel
 * index).  Surfels flagged DEGENERATE or UNINIT, planes through the camera
 * centre (|n . r_s| < 1e-6) and non-positive or non-finite id_u give no
 * measurement. */
int sgo_disc_render(const sgo_keyframe* kf, const sgo_surfels* s, const double* ux,
                    const double* uy, int32_t count, double radius, double* inv_depth,
                    int32_t* surfel_index) {
    int W = kf->kf.width, H = kf->kf.height;
    for (size_t o = 0; o < (size_t)W * H; ++o) {
        inv_depth[o] = 0.0;
        surfel_index[o] = -1;
    }
    for (int32_t i = 0; i < count; ++i) {
        if (s->flags[i] & (SGO_DEGENERATE | SGO_UNINIT)) continue;
        double n[3] = {s->nx[i], s->ny[i], s->nz[i]}, rs[3];
        sgo_ray(&kf->K, ux[i], uy[i], rs);
        if (fabs(dot3(n, rs)) < 1e-6) continue;
        support sp = disc_support(W, H, ux[i], uy[i], radius);
        for (int y = sp.y0; y <= sp.y1; ++y)
            for (int x = sp.x0; x <= sp.x1; ++x) {
                if (!in_support(&sp, x, y)) continue;
                double id = sgo_pixel_inverse_depth(&kf->K, ux[i], uy[i], s->inv_depth[i], n, x, y);
                if (!(id > 0.0) || !isfinite(id)) continue;
                size_t o = (size_t)y * W + x;
                if (id > inv_depth[o]) {          /* depth test; ties keep the lower index */
                    inv_depth[o] = id;
                    surfel_index[o] = i;
                }
            }
    }
    return 0;
}

/* Surfel Initialization section, the search for an empty area: a candidate
 * pixel u_ns qualifies when every non-empty pixel u_nn of the surfel-index
 * map (index >= 0) lies farther than alpha r from it, decided on the
 * integer squared distance against (alpha r)^2 in double.  The candidates
 * are the pixels (spacing/2 + i spacing, spacing/2 + j spacing) of a fixed
 * lattice, visited row by row.  Writes the first `capacity` qualifying
 * candidates and returns how many qualify. */
int32_t sgo_disc_search(int32_t width, int32_t height, const int32_t* surfel_index,
                        double radius, double alpha, int32_t spacing, int32_t* out_x,
                        int32_t* out_y, int32_t capacity) {
    if (spacing < 1) return -1;
    double ar = alpha * radius;
    double ar2 = ar * ar;
    int reach = (int)floor(ar);
    int32_t found = 0;
    for (int cy = spacing / 2; cy < height; cy += spacing) {
        for (int cx = spacing / 2; cx < width; cx += spacing) {
            int empty = 1;
            for (int y = cy - reach; y <= cy + reach && empty; ++y) {
                if (y < 0 || y >= height) continue;
                for (int x = cx - reach; x <= cx + reach; ++x) {
                    if (x < 0 || x >= width) continue;
                    if (surfel_index[(size_t)y * width + x] < 0) continue;
                    int dx = x - cx, dy = y - cy;
                    if ((double)(dx * dx + dy * dy) <= ar2) { empty = 0; break; }
                }
            }
            if (!empty) continue;
            if (found < capacity) { out_x[found] = cx; out_y[found] = cy; }
            ++found;
        }
    }
    return found;
}

/* Surfel Initialization section with disc surfels: the neighbours of a new
 * surfel at u_ns are the surfels that own, in the surfel-index map, a pixel
 * u with |u_ns - u| < beta r (integer squared distance against (beta r)^2 in
 * double), skipping those flagged DEGENERATE or UNINIT and planes through
 * the camera centre.  The new inverse depth is the mean over them, in index
 * order, of Eq. 3 of the neighbour's plane at u_ns; the new normal the mean
 * of their normals sign-aligned to the first, renormalised.  Surfels
 * first .. first + n_new - 1 (centres ux, uy) are written: id, n, flags (0,
 * or UNINIT with id 0 and n = (0, 0, -1) when nothing qualifies), cost 0,
 * nvalid 0, last_update 0.  Only surfels below `first` are neighbours. */
int sgo_disc_init(const sgo_keyframe* kf, sgo_surfels* s, const double* ux, const double* uy,
                  const int32_t* surfel_index, int32_t first, int32_t n_new, double radius,
                  double beta) {
    int W = kf->kf.width, H = kf->kf.height;
    double br = beta * radius;
    double br2 = br * br;
    int reach = (int)ceil(br);
    uint8_t* seen = (uint8_t*)calloc(first > 0 ? (size_t)first : 1, 1);
    if (!seen) return -1;
    for (int32_t i = first; i < first + n_new; ++i) {
        double cx = ux[i], cy = uy[i];
        int icx = (int)cx, icy = (int)cy;        /* new centres are lattice pixels */
        memset(seen, 0, first > 0 ? (size_t)first : 1);
        for (int y = icy - reach; y <= icy + reach; ++y) {
            if (y < 0 || y >= H) continue;
            for (int x = icx - reach; x <= icx + reach; ++x) {
                if (x < 0 || x >= W) continue;
                int32_t j = surfel_index[(size_t)y * W + x];
                if (j < 0 || j >= first) continue;
                int dx = x - icx, dy = y - icy;
                if ((double)(dx * dx + dy * dy) < br2) seen[j] = 1;
            }
        }
        double id_sum = 0.0, nsum[3] = {0.0, 0.0, 0.0}, nref[3] = {0.0, 0.0, 0.0};
        int count = 0;
        for (int32_t j = 0; j < first; ++j) {
            if (!seen[j]) continue;
            if (s->flags[j] & (SGO_UNINIT | SGO_DEGENERATE)) continue;
            double nj[3] = {s->nx[j], s->ny[j], s->nz[j]}, rj[3];
            sgo_ray(&kf->K, ux[j], uy[j], rj);
            if (fabs(dot3(nj, rj)) < 1e-6) continue;
            /* Eq. 3 with the neighbour's plane, at the new surfel's pixel */
            double id = sgo_pixel_inverse_depth(&kf->K, ux[j], uy[j], s->inv_depth[j], nj, cx, cy);
            if (count == 0) { nref[0] = nj[0]; nref[1] = nj[1]; nref[2] = nj[2]; }
            double sg = dot3(nj, nref) < 0.0 ? -1.0 : 1.0;
            id_sum += id;
            for (int k = 0; k < 3; ++k) nsum[k] += sg * nj[k];
            ++count;
        }
        double id_new = count ? id_sum / count : 0.0;
        double n_new[3] = {0.0, 0.0, 0.0};
        int ok = count > 0;
        if (ok) {
            for (int k = 0; k < 3; ++k) n_new[k] = nsum[k] / count;
            ok = normalize3(n_new) && id_new > 0.0 && isfinite(id_new);
        }
        if (ok) {
            s->inv_depth[i] = id_new;
            s->nx[i] = n_new[0]; s->ny[i] = n_new[1]; s->nz[i] = n_new[2];
            s->flags[i] = 0;
        } else {
            s->inv_depth[i] = 0.0;
            s->nx[i] = 0.0; s->ny[i] = 0.0; s->nz[i] = -1.0;
            s->flags[i] = SGO_UNINIT;
        }
        s->cost[i] = 0.0;
        s->nvalid[i] = 0;
        s->last_update[i] = 0;
    }
    free(seen);
    return 0;
}

/* Eq. 10: p' = P p (p = r_s / id_s by Eq. 1), n' = R n, r' = pi(p'). */
int sgo_transfer_surfels(const sgo_intrinsics* K, const sgo_pose* P, int32_t count,
                         const double* usx, const double* usy, const double* id_s,
                         const double* n, double* ux_out, double* uy_out,
                         double* id_out, double* n_out) {
    int ok = 0;
    for (int32_t k = 0; k < count; ++k) {
        double rs[3], p0[3], p1[3];
        sgo_ray(K, usx[k], usy[k], rs);
        for (int i = 0; i < 3; ++i) p0[i] = rs[i] / id_s[k];
        for (int i = 0; i < 3; ++i)
            p1[i] = P->R[3 * i] * p0[0] + P->R[3 * i + 1] * p0[1] + P->R[3 * i + 2] * p0[2] + P->t[i];
        for (int i = 0; i < 3; ++i)
            n_out[3 * k + i] = P->R[3 * i] * n[3 * k] + P->R[3 * i + 1] * n[3 * k + 1] +
                               P->R[3 * i + 2] * n[3 * k + 2];
        if (!(p1[2] > 0.0)) {
            ux_out[k] = uy_out[k] = 0.0;
            id_out[k] = 0.0;
            continue;
        }
        double r1[3] = {p1[0] / p1[2], p1[1] / p1[2], 1.0};   /* pi(p') */
        ux_out[k] = K->fx * r1[0] + K->cx;
        uy_out[k] = K->fy * r1[1] + K->cy;
        id_out[k] = 1.0 / p1[2];
        ++ok;
    }
    return ok;
}

/* Eq. 10 for disc surfels.  Reading: a disc surfel stays a disc; a usable
 * source surfel (no DEGENERATE or UNINIT flag, id_s > 0) moves to
 * p' = R (r_s / id_s) + t with n' = R n, and in the destination keyframe it is
 * centred at u' = K_dst pi(p') with inverse depth 1/p'_z (Eq. 1 with
 * r' = pi(p')).  Those with p'_z > 0 and u' inside [0, W-1] x [0, H-1] are
 * written in source order to destination surfels 0, 1, ... (the first
 * `capacity`): id, n, centre, flags 0, cost 0, nvalid 0 and the source's
 * last_update; src_index (may be NULL) receives the source index.  Returns
 * the number written; *landed_out the number that landed. */
int32_t sgo_disc_transfer(const sgo_intrinsics* Ks, const sgo_intrinsics* Kd, int32_t dst_w,
                          int32_t dst_h, const sgo_pose* P, const sgo_surfels* src,
                          const double* ux, const double* uy, int32_t count, sgo_surfels* dst,
                          double* dux, double* duy, int32_t capacity, int32_t* src_index,
                          int32_t* landed_out) {
    int32_t landed = 0;
    for (int32_t k = 0; k < count; ++k) {
        if (src->flags[k] & (SGO_DEGENERATE | SGO_UNINIT)) continue;
        if (!(src->inv_depth[k] > 0.0)) continue;
        double rs[3], p0[3], p1[3], n1[3];
        double n0[3] = {src->nx[k], src->ny[k], src->nz[k]};
        sgo_ray(Ks, ux[k], uy[k], rs);
        for (int i = 0; i < 3; ++i) p0[i] = rs[i] / src->inv_depth[k];          /* Eq. 1 */
        for (int i = 0; i < 3; ++i) {                                            /* Eq. 10 */
            p1[i] = P->R[3 * i] * p0[0] + P->R[3 * i + 1] * p0[1] + P->R[3 * i + 2] * p0[2] + P->t[i];
            n1[i] = P->R[3 * i] * n0[0] + P->R[3 * i + 1] * n0[1] + P->R[3 * i + 2] * n0[2];
        }
        if (!(p1[2] > 0.0)) continue;
        double r1[2] = {p1[0] / p1[2], p1[1] / p1[2]};                          /* pi(p') */
        double u = Kd->fx * r1[0] + Kd->cx, v = Kd->fy * r1[1] + Kd->cy;
        if (!(u >= 0.0 && u <= (double)(dst_w - 1) && v >= 0.0 && v <= (double)(dst_h - 1))) continue;
        if (landed < capacity) {
            int32_t j = landed;
            dst->inv_depth[j] = 1.0 / p1[2];
            dst->nx[j] = n1[0]; dst->ny[j] = n1[1]; dst->nz[j] = n1[2];
            dst->flags[j] = 0;
            dst->cost[j] = 0.0;
            dst->nvalid[j] = 0;
            dst->last_update[j] = src->last_update[k];
            dux[j] = u;
            duy[j] = v;
            if (src_index) src_index[j] = k;
        }
        ++landed;
    }
    if (landed_out) *landed_out = landed;
    return landed < capacity ? landed : capacity;
}

/* Landing of one source surfel in the destination keyframe (Eq. 10):
 * returns 0 when the surfel is unusable, behind the destination camera or
 * outside its tiles; else the tile index, 1/p'_z, r' = p'/p'_z and n'. */
static int regrid_land(const sgo_grid* sg, const sgo_surfels* src, const sgo_pose* P,
                       const sgo_grid* dg, int32_t i, int32_t* tile, double* idp, double rp[3],
                       double np[3]) {
    const int S0 = sg->patch, gw0 = sg->width / S0;
    if (src->flags[i] & (SGO_DEGENERATE | SGO_UNINIT)) return 0;
    const double id = src->inv_depth[i];
    if (!(id > 0.0) || !isfinite(id)) return 0;
    double usx = S0 * (i % gw0) + 0.5 * (S0 - 1), usy = S0 * (i / gw0) + 0.5 * (S0 - 1);
    double rs[3], p0[3], p1[3];
    const double n0[3] = {src->nx[i], src->ny[i], src->nz[i]};
    sgo_ray(&sg->K, usx, usy, rs);
    for (int k = 0; k < 3; ++k) p0[k] = rs[k] / id;
    for (int k = 0; k < 3; ++k) {
        p1[k] = P->R[3 * k] * p0[0] + P->R[3 * k + 1] * p0[1] + P->R[3 * k + 2] * p0[2] + P->t[k];
        np[k] = P->R[3 * k] * n0[0] + P->R[3 * k + 1] * n0[1] + P->R[3 * k + 2] * n0[2];
    }
    if (!(p1[2] > 0.0)) return 0;
    rp[0] = p1[0] / p1[2];
    rp[1] = p1[1] / p1[2];
    rp[2] = 1.0;
    const double ux = dg->K.fx * rp[0] + dg->K.cx, uy = dg->K.fy * rp[1] + dg->K.cy;
    const double px = floor(ux + 0.5), py = floor(uy + 0.5);      /* nearest pixel */
    const int S1 = dg->patch, gw1 = dg->width / S1, gh1 = dg->height / S1;
    if (!(px >= 0.0 && px < (double)(gw1 * S1) && py >= 0.0 && py < (double)(gh1 * S1))) return 0;
    *tile = ((int32_t)py / S1) * gw1 + (int32_t)px / S1;
    *idp = 1.0 / p1[2];
    return 1;
}

int sgo_transfer_regrid(const sgo_grid* src_grid, const sgo_surfels* src, const sgo_pose* P,
                        const sgo_grid* dst_grid, sgo_surfels* dst, uint8_t* dst_is_new,
                        int32_t* dst_src_index) {
    const int32_t n_src = (src_grid->width / src_grid->patch) * (src_grid->height / src_grid->patch);
    const int S1 = dst_grid->patch, gw1 = dst_grid->width / S1, gh1 = dst_grid->height / S1;
    const int32_t n_dst = gw1 * gh1;
    int32_t* win = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_dst > 0 ? n_dst : 1));
    double* best = (double*)malloc(sizeof(double) * (size_t)(n_dst > 0 ? n_dst : 1));
    for (int32_t j = 0; j < n_dst; ++j) { win[j] = -1; best[j] = 0.0; }
    /* z-test: closest landed surfel per destination tile, in index order */
    for (int32_t i = 0; i < n_src; ++i) {
        int32_t j;
        double idp, rp[3], np[3];
        if (!regrid_land(src_grid, src, P, dst_grid, i, &j, &idp, rp, np)) continue;
        if (win[j] < 0 || idp > best[j]) { win[j] = i; best[j] = idp; }
    }
    int filled = 0;
    for (int32_t j = 0; j < n_dst; ++j) {
        int ok = 0;
        double idt = 0.0, nt[3] = {0.0, 0.0, -1.0};
        if (win[j] >= 0) {
            int32_t jj;
            double idp, rp[3], np[3], rt[3];
            regrid_land(src_grid, src, P, dst_grid, win[j], &jj, &idp, rp, np);
            sgo_ray(&dst_grid->K, S1 * (j % gw1) + 0.5 * (S1 - 1), S1 * (j / gw1) + 0.5 * (S1 - 1), rt);
            const double c1 = dot3(np, rp), ct = dot3(np, rt);
            if (fabs(c1) >= 1e-6 && fabs(ct) >= 1e-6) {
                idt = idp * ct / c1;                      /* Eq. 3 of the moved plane at r_t */
                double nn[3] = {np[0], np[1], np[2]};
                if (idt > 0.0 && isfinite(idt) && normalize3(nn)) {
                    nt[0] = nn[0]; nt[1] = nn[1]; nt[2] = nn[2];
                    ok = 1;
                }
            }
            if (!ok) idt = 0.0;
        }
        dst->inv_depth[j] = ok ? idt : 0.0;
        dst->nx[j] = ok ? nt[0] : 0.0;
        dst->ny[j] = ok ? nt[1] : 0.0;
        dst->nz[j] = ok ? nt[2] : -1.0;
        dst->flags[j] = ok ? 0u : SGO_UNINIT;
        dst->cost[j] = 0.0;
        dst->nvalid[j] = 0;
        dst->last_update[j] = ok ? src->last_update[win[j]] : 0u;
        if (dst->kappa) dst->kappa[j] = 0.0;
        if (dst->margin) dst->margin[j] = INFINITY;
        dst_is_new[j] = ok ? 0 : 1;
        if (dst_src_index) dst_src_index[j] = ok ? win[j] : -1;
        filled += ok;
    }
    free(win);
    free(best);
    return filled;
}

void sgo_set_threads(int32_t n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t sgo_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
