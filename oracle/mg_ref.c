/*
 * Serial FP64 reference implementation of the method of Oo & Vogel,
 * "Accelerating Geometric Multigrid Preconditioning with Half-Precision
 * Arithmetic on GPUs" (arXiv 2007.07539).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no source, header, table or helper
 * with the GPU library, and the GPU library never calls it.
 *
 * Everything is computed in IEEE double precision, in physical units, with
 * the plainest loops that state the definitions:
 *
 *   Model problem (Section 5): -Laplace(u) = f on the unit square (D = 2) or
 *   unit cube (D = 3), u = 0 on the boundary, on n^D interior points of a
 *   uniform mesh of width h = 1/(n+1), in one of two discretisations:
 *
 *   FD (disc 0): the standard (2D+1)-point finite-difference stencil,
 *       (A v)_i = (2D v_i - sum_{j face neighbour of i} v_j) / h^2,
 *   with v_j = 0 for neighbours on the boundary (homogeneous Dirichlet).
 *
 *   Q1 (disc 1): the bilinear (2-D) / trilinear (3-D) finite elements that
 *   the paper uses (Section 5): A_ij = integral of grad(phi_i) . grad(phi_j)
 *   over the domain, phi_i the nodal basis, assembled cell by cell.
 *
 *   Grid hierarchy (Section 4.2): level sizes n, (n-1)/2, ... down to the
 *   base level; with n = 2^m - 1 the base can be a single point.  Coarse
 *   operators are the same discretisation on the coarser mesh (for Q1 this is
 *   also the Galerkin product R A P, which the tests check).
 *
 *   Smoother (Section 4.2): damped Jacobi,  c <- c + omega * D^-1 (b - A c),
 *   with D = diag(A) (2D/h^2 for FD).
 *
 *   Transfers: linear (bi-/tri-linear) interpolation P for prolongation.
 *   Restriction: FD uses full weighting (tensor product of the 1-D weights
 *   1/4, 1/2, 1/4 centred on the coarse point's fine twin), Q1 the transpose
 *   R = P^T of the interpolation (2^D times full weighting), so that
 *   R A_h P = A_2h.
 *
 *   V-cycle: the two-grid method of Algorithm 1 applied recursively, with an
 *   exact solve on a one-point base level or CG on a larger one.
 *
 *   Outer solver: mixed-precision iterative refinement with residuum scaling,
 *   Algorithm 2 (Section 4.3), run here entirely in FP64.
 *
 * Array layout: dense n^D, x fastest: index (k*n + j)*n + i in 3-D, j*n + i in
 * 2-D.  All arrays are caller-owned.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define REF_OK 0
#define REF_ERR_ARG -1
#define REF_ERR_SHAPE -2
#define REF_ERR_NOT_CONVERGED -6
#define REF_ERR_NONFINITE -7
#define REF_ERR_NOMEM -9

#define REF_DISC_FD 0
#define REF_DISC_Q1 1

/* n must be 2^m - 1 with m >= 1 so that coarsening by two ends on one point. */
static int ref_valid_n(int n) { return n >= 1 && (((long)n + 1) & (long)n) == 0; }

/* The hierarchy n, (n-1)/2, ... reaches n_base through odd sizes only
 * (every coarse point has a fine twin and two fine neighbours). */
static int ref_chain_ok(int n, int n_base) {
    if (n_base < 1 || n < n_base) return 0;
    while (n > n_base) {
        if (n % 2 == 0) return 0;
        n = (n - 1) / 2;
    }
    return n == n_base;
}

long ref_points(int dim, int n) {
    return dim == 2 ? (long)n * n : (long)n * n * n;
}

/* Number of levels of the full hierarchy n, (n-1)/2, ...: down to the
 * 1-point base for n = 2^m - 1, otherwise down to the first even size. */
int ref_levels(int n) {
    int L = 0;
    while (n > 1 && n % 2 == 1) { n = (n - 1) / 2; L++; }
    return L + 1;
}

static double ref_h(int n) { return 1.0 / (double)(n + 1); }

/* v at interior coordinates (i, j, k); zero outside: homogeneous Dirichlet. */
static double ref_get(int dim, int n, const double *v, int i, int j, int k) {
    if (i < 0 || i >= n || j < 0 || j >= n) return 0.0;
    if (dim == 2) return v[(long)j * n + i];
    if (k < 0 || k >= n) return 0.0;
    return v[((long)k * n + j) * n + i];
}

/* out = A v  (Section 5, finite-difference discretisation of -Laplace). */
void ref_apply_A(int dim, int n, const double *v, double *out) {
    double h = ref_h(n);
    double inv_h2 = 1.0 / (h * h);
    int nk = dim == 2 ? 1 : n;
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                double centre = ref_get(dim, n, v, i, j, k);
                double nb = ref_get(dim, n, v, i - 1, j, k) + ref_get(dim, n, v, i + 1, j, k) +
                            ref_get(dim, n, v, i, j - 1, k) + ref_get(dim, n, v, i, j + 1, k);
                if (dim == 3)
                    nb += ref_get(dim, n, v, i, j, k - 1) + ref_get(dim, n, v, i, j, k + 1);
                long idx = dim == 2 ? (long)j * n + i : ((long)k * n + j) * n + i;
                out[idx] = (2.0 * dim * centre - nb) * inv_h2;
            }
}

/* The Q1 element matrix of one cell of side h (Section 5): with the 1-D
 * element stiffness k = [1 -1; -1 1] / h and mass m = h [1/3 1/6; 1/6 1/3]
 * of the linear hat functions, the tensor-product basis gives
 *   K_e[a][b] = sum_d k[a_d][b_d] * prod_{d' != d} m[a_d'][b_d'],
 * a, b in {0,1}^D the local vertex numbers (bit d of a = offset along axis d). */
static void ref_q1_element(int dim, double h, double Ke[8][8]) {
    const double k1[2][2] = {{1.0 / h, -1.0 / h}, {-1.0 / h, 1.0 / h}};
    const double m1[2][2] = {{h / 3.0, h / 6.0}, {h / 6.0, h / 3.0}};
    int nv = 1 << dim;
    for (int a = 0; a < nv; a++)
        for (int b = 0; b < nv; b++) {
            double s = 0.0;
            for (int d = 0; d < dim; d++) {
                double t = k1[(a >> d) & 1][(b >> d) & 1];
                for (int e = 0; e < dim; e++)
                    if (e != d) t *= m1[(a >> e) & 1][(b >> e) & 1];
                s += t;
            }
            Ke[a][b] = s;
        }
}

/* out = A v for Q1: the sum of the element matrices over the (n+1)^D cells,
 * cell (cx, cy, cz) spanning interior indices cx-1 .. cx (0-based, -1 and n on
 * the boundary).  Boundary vertices hold v = 0 and have no row. */
static void ref_apply_q1(int dim, int n, const double *v, double *out) {
    double Ke[8][8];
    ref_q1_element(dim, ref_h(n), Ke);
    int nv = 1 << dim;
    long N = ref_points(dim, n);
    for (long p = 0; p < N; p++) out[p] = 0.0;
    int ncz = dim == 3 ? n + 1 : 1;
    for (int cz = 0; cz < ncz; cz++)
        for (int cy = 0; cy <= n; cy++)
            for (int cx = 0; cx <= n; cx++)
                for (int a = 0; a < nv; a++) {
                    int i = cx - 1 + (a & 1), j = cy - 1 + ((a >> 1) & 1);
                    int k = dim == 3 ? cz - 1 + ((a >> 2) & 1) : 0;
                    if (i < 0 || i >= n || j < 0 || j >= n || k < 0 || (dim == 3 && k >= n)) continue;
                    double s = 0.0;
                    for (int b = 0; b < nv; b++) {
                        int bi = cx - 1 + (b & 1), bj = cy - 1 + ((b >> 1) & 1);
                        int bk = dim == 3 ? cz - 1 + ((b >> 2) & 1) : 0;
                        s += Ke[a][b] * ref_get(dim, n, v, bi, bj, bk);
                    }
                    long idx = dim == 2 ? (long)j * n + i : ((long)k * n + j) * n + i;
                    out[idx] += s;
                }
}

/* diag(A): 2D/h^2 for FD; for Q1 the 2^D cells around a vertex each add
 * K_e[0][0] = D h^(D-2) / 3^(D-1). */
static double ref_diag(int dim, int n, int disc) {
    double h = ref_h(n);
    if (disc == REF_DISC_Q1) return (double)(1 << dim) * dim * pow(h, dim - 2) / pow(3.0, dim - 1);
    return 2.0 * dim / (h * h);
}

void ref_apply_A_disc(int dim, int n, int disc, const double *v, double *out) {
    if (disc == REF_DISC_Q1) ref_apply_q1(dim, n, v, out);
    else ref_apply_A(dim, n, v, out);
}

/* r = b - A c  (the residual of Algorithms 1 and 2). */
static void ref_residual_d(int dim, int n, int disc, const double *b, const double *c, double *r) {
    long N = ref_points(dim, n);
    ref_apply_A_disc(dim, n, disc, c, r);
    for (long p = 0; p < N; p++) r[p] = b[p] - r[p];
}

void ref_residual(int dim, int n, const double *b, const double *c, double *r) {
    ref_residual_d(dim, n, REF_DISC_FD, b, c, r);
}

void ref_residual_disc(int dim, int n, int disc, const double *b, const double *c, double *r) {
    ref_residual_d(dim, n, disc, b, c, r);
}

/* One damped-Jacobi sweep (Section 4.2): out = c + omega * (b - A c) / diag(A).
 * The update is simultaneous, so out must not alias c. */
void ref_jacobi_disc(int dim, int n, int disc, double omega, const double *b, const double *c, double *out) {
    long N = ref_points(dim, n);
    double diag = ref_diag(dim, n, disc);
    double *r = (double *)malloc(sizeof(double) * N);
    ref_residual_d(dim, n, disc, b, c, r);
    for (long p = 0; p < N; p++) out[p] = c[p] + omega * r[p] / diag;
    free(r);
}

void ref_jacobi(int dim, int n, double omega, const double *b, const double *c, double *out) {
    ref_jacobi_disc(dim, n, REF_DISC_FD, omega, b, c, out);
}

/* Restriction from a fine grid of n_f points per dimension to the coarse grid
 * of n_c = (n_f - 1)/2 points.  Coarse point I sits on fine point 2I+1
 * (0-based).  FD: full weighting, 1-D weights 1/4, 1/2, 1/4.  Q1: the
 * transpose of linear interpolation, 1-D weights 1/2, 1, 1/2. */
void ref_restrict_disc(int dim, int n_f, int disc, const double *r_f, double *b_c) {
    int n_c = (n_f - 1) / 2;
    const double g = disc == REF_DISC_Q1 ? 2.0 : 1.0;
    const double w[3] = {0.25 * g, 0.5 * g, 0.25 * g};
    int nK = dim == 2 ? 1 : n_c;
    for (int K = 0; K < nK; K++)
        for (int J = 0; J < n_c; J++)
            for (int I = 0; I < n_c; I++) {
                double s = 0.0;
                int oz_lo = dim == 2 ? 1 : 0, oz_hi = dim == 2 ? 1 : 2;
                for (int oz = oz_lo; oz <= oz_hi; oz++)
                    for (int oy = 0; oy < 3; oy++)
                        for (int ox = 0; ox < 3; ox++) {
                            double wt = w[ox] * w[oy] * (dim == 3 ? w[oz] : 1.0);
                            int fi = 2 * I + ox, fj = 2 * J + oy, fk = 2 * K + oz;
                            s += wt * ref_get(dim, n_f, r_f, fi, fj, dim == 3 ? fk : 0);
                        }
                long idx = dim == 2 ? (long)J * n_c + I : ((long)K * n_c + J) * n_c + I;
                b_c[idx] = s;
            }
}

void ref_restrict(int dim, int n_f, const double *r_f, double *b_c) {
    ref_restrict_disc(dim, n_f, REF_DISC_FD, r_f, b_c);
}

/* Linear interpolation weight of coarse point I for fine point i (0-based):
 * the fine twin of I is 2I+1; distance 0 -> 1, distance 1 -> 1/2. */
static double ref_lin_w(int i, int I) {
    int d = i - (2 * I + 1);
    if (d == 0) return 1.0;
    if (d == 1 || d == -1) return 0.5;
    return 0.0;
}

/* Prolongation by bi-/tri-linear interpolation from n_c to n_f = 2 n_c + 1:
 * e_f = P e_c, with coarse values outside the grid taken as zero. */
void ref_prolong(int dim, int n_c, const double *e_c, double *e_f) {
    int n_f = 2 * n_c + 1;
    int nk = dim == 2 ? 1 : n_f;
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < n_f; j++)
            for (int i = 0; i < n_f; i++) {
                /* The coarse points that can touch fine index i are
                 * floor((i-1)/2) and floor((i-1)/2) + 1 in each dimension. */
                int I0 = (i + 1) / 2 - 1, J0 = (j + 1) / 2 - 1, K0 = (k + 1) / 2 - 1;
                double s = 0.0;
                for (int dz = 0; dz < (dim == 3 ? 2 : 1); dz++)
                    for (int dy = 0; dy < 2; dy++)
                        for (int dx = 0; dx < 2; dx++) {
                            int I = I0 + dx, J = J0 + dy, K = K0 + dz;
                            double wt = ref_lin_w(i, I) * ref_lin_w(j, J);
                            if (dim == 3) wt *= ref_lin_w(k, K);
                            if (wt == 0.0) continue;
                            s += wt * ref_get(dim, n_c, e_c, I, J, dim == 3 ? K : 0);
                        }
                long idx = dim == 2 ? (long)j * n_f + i : ((long)k * n_f + j) * n_f + i;
                e_f[idx] = s;
            }
}

/* Exact solve on the one-point base level: A_0 = diag(A_0) is 1x1. */
static void ref_base_solve(int dim, int n, int disc, const double *b, double *c) {
    long N = ref_points(dim, n);
    if (N != 1) return;
    c[0] = b[0] / ref_diag(dim, n, disc);
}

/* Conjugate gradients for A x = b on the level with n points per dimension
 * (the paper's base solver, Section 4.2), from x = 0: with r = b, p = r,
 *   q = A p,  a = (r.r)/(p.q),  x += a p,  r -= a q,
 *   p = r + ((r.r)_new/(r.r)) p,
 * until ||r||_2 <= tol ||b||_2 or max_iter steps (the paper's 1e-4 is an
 * absolute bound on residuals that the scaling has brought to norm one; taken
 * relative to the base right-hand side, the test means the same there and does
 * not switch the base solve off once an unscaled residual is small).
 * Returns the steps taken. */
int ref_cg_disc(int dim, int n, int disc, const double *b, double *x, double tol, int max_iter) {
    long N = ref_points(dim, n);
    double *r = (double *)malloc(sizeof(double) * N);
    double *p = (double *)malloc(sizeof(double) * N);
    double *q = (double *)malloc(sizeof(double) * N);
    if (!r || !p || !q) { free(r); free(p); free(q); return REF_ERR_NOMEM; }
    memset(x, 0, sizeof(double) * N);
    memcpy(r, b, sizeof(double) * N);
    memcpy(p, b, sizeof(double) * N);
    double rr = 0.0;
    for (long i = 0; i < N; i++) rr += r[i] * r[i];
    const double stop = tol * sqrt(rr);
    int k = 0;
    while (k < max_iter && sqrt(rr) > stop) {
        ref_apply_A_disc(dim, n, disc, p, q);
        double pq = 0.0;
        for (long i = 0; i < N; i++) pq += p[i] * q[i];
        if (!(pq > 0.0)) break;                      /* p = 0 (or breakdown) */
        double a = rr / pq;
        for (long i = 0; i < N; i++) { x[i] += a * p[i]; r[i] -= a * q[i]; }
        double rr_new = 0.0;
        for (long i = 0; i < N; i++) rr_new += r[i] * r[i];
        double beta = rr_new / rr;
        for (long i = 0; i < N; i++) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        k++;
    }
    free(r); free(p); free(q);
    return k;
}

int ref_cg(int dim, int n, const double *b, double *x, double tol, int max_iter) {
    return ref_cg_disc(dim, n, REF_DISC_FD, b, x, tol, max_iter);
}

/* One V-cycle for A_l c = b on the level with n points per dimension
 * (Algorithm 1 applied recursively, Section 4.2), starting from c = 0, down
 * to the base level of n_base points per dimension (n_base = 1: the exact
 * one-point solve; otherwise CG to base_tol, at most base_max_iter steps):
 *   1. pre-smooth nu1 times,
 *   2. residual, restrict to the coarse grid,
 *   3. coarse correction by the same cycle one level down (exact on 1 point),
 *   4. prolongate and add,
 *   5. post-smooth nu2 times.
 * Returns REF_OK or an error code. */
int ref_vcycle_disc(int dim, int n, int disc, int n_base, int nu1, int nu2, double omega, double base_tol,
                    int base_max_iter, const double *b, double *c) {
    if ((dim != 2 && dim != 3) || (disc != REF_DISC_FD && disc != REF_DISC_Q1) || !ref_chain_ok(n, n_base) ||
        nu1 < 0 || nu2 < 0)
        return REF_ERR_ARG;
    long N = ref_points(dim, n);
    if (n == n_base) {
        if (n == 1) {
            ref_base_solve(dim, n, disc, b, c);
        } else {
            int k = ref_cg_disc(dim, n, disc, b, c, base_tol, base_max_iter);
            if (k < 0) return k;
        }
        return REF_OK;
    }
    int n_c = (n - 1) / 2;
    long Nc = ref_points(dim, n_c);
    double *tmp = (double *)malloc(sizeof(double) * N);
    double *bc = (double *)malloc(sizeof(double) * Nc);
    double *ec = (double *)malloc(sizeof(double) * Nc);
    if (!tmp || !bc || !ec) { free(tmp); free(bc); free(ec); return REF_ERR_NOMEM; }

    memset(c, 0, sizeof(double) * N);
    for (int s = 0; s < nu1; s++) {                 /* pre-smooth */
        ref_jacobi_disc(dim, n, disc, omega, b, c, tmp);
        memcpy(c, tmp, sizeof(double) * N);
    }
    ref_residual_d(dim, n, disc, b, c, tmp);        /* residual, restrict */
    ref_restrict_disc(dim, n, disc, tmp, bc);
    int st = ref_vcycle_disc(dim, n_c, disc, n_base, nu1, nu2, omega, base_tol, base_max_iter, bc, ec);
    if (st == REF_OK) {
        ref_prolong(dim, n_c, ec, tmp);             /* prolongate, add */
        for (long p = 0; p < N; p++) c[p] += tmp[p];
        for (int s = 0; s < nu2; s++) {             /* post-smooth */
            ref_jacobi_disc(dim, n, disc, omega, b, c, tmp);
            memcpy(c, tmp, sizeof(double) * N);
        }
    }
    free(tmp); free(bc); free(ec);
    return st;
}

int ref_vcycle_base(int dim, int n, int n_base, int nu1, int nu2, double omega, double base_tol,
                    int base_max_iter, const double *b, double *c) {
    if (!ref_valid_n(n) || !ref_valid_n(n_base)) return REF_ERR_ARG;
    return ref_vcycle_disc(dim, n, REF_DISC_FD, n_base, nu1, nu2, omega, base_tol, base_max_iter, b, c);
}

int ref_vcycle(int dim, int n, int nu1, int nu2, double omega, const double *b, double *c) {
    return ref_vcycle_base(dim, n, 1, nu1, nu2, omega, 0.0, 0, b, c);
}

/* Pairwise sum of squares (accurate Euclidean norm). */
static double ref_sumsq(const double *v, long N) {
    if (N <= 8) {
        double s = 0.0;
        for (long p = 0; p < N; p++) s += v[p] * v[p];
        return s;
    }
    long m = N / 2;
    return ref_sumsq(v, m) + ref_sumsq(v + m, N - m);
}

double ref_norm2(const double *v, long N) { return sqrt(ref_sumsq(v, N)); }

double ref_norminf(const double *v, long N) {
    double m = 0.0;
    for (long p = 0; p < N; p++) {
        double a = fabs(v[p]);
        if (a > m || a != a) m = a;          /* NaN propagates */
    }
    return m;
}

/* Options and result of the iterative-refinement solve. */
typedef struct {
    int nu1, nu2;
    double omega;
    int residual_scaling;      /* 1: alpha = ||r||_inf (residuum scaling, Algorithm 2); 0: alpha = 1 */
    int recursive_residual;    /* 1: r -= alpha A c as in Algorithm 2; 0: r = b - A u */
    int max_iter;
    double rtol;               /* stop when ||r||_2 <= rtol ||b||_2 */
    int use_initial_guess;     /* 0: u starts at zero */
    int cycles;                /* V-cycles per refinement step (<= 1: one, as in Algorithm 2);
                                  each further cycle continues from the correction so far:
                                  c <- c + V(r/alpha - A c) */
    int base_n;                /* points per dimension of the base level (<= 1: one point) */
    double base_tol;           /* CG on a base of more than one point: ||r||_2 <= base_tol */
    int base_max_iter;         /* ... at most this many steps */
    int disc;                  /* REF_DISC_FD or REF_DISC_Q1 */
} ref_ir_opts;

typedef struct {
    int iterations;            /* V-cycles applied */
    double rel_residual;       /* ||r||_2 / ||b||_2 of the returned iterate (as tracked) */
    double true_rel_residual;  /* ||b - A u||_2 / ||b||_2 recomputed at the end */
} ref_ir_result;

/* Iterative refinement with residuum scaling (Algorithm 2, Section 4.3), with
 * every quantity in FP64.  The solution u is improved by corrections from the
 * correction equation A c = r / alpha, whose right-hand side is the current
 * residual divided by its largest entry (alpha = 1 without scaling); one
 * V-cycle from zero (or several, each continuing from the correction so far)
 * approximates c, u moves by alpha c, and r is brought up to date either by
 * subtracting alpha A c or by recomputing b - A u.  The loop ends when
 * ||r||_2 <= rtol ||b||_2.  history (optional, length hist_cap) receives
 * ||r||_2/||b||_2 before each V-cycle and after the last one. */
int ref_ir_solve(int dim, int n, const double *b, double *u, const ref_ir_opts *o,
                 ref_ir_result *res, double *history, int hist_cap) {
    if ((dim != 2 && dim != 3) || !o || !res) return REF_ERR_ARG;
    const int disc = o->disc;
    if (disc != REF_DISC_FD && disc != REF_DISC_Q1) return REF_ERR_ARG;
    const int nbase = o->base_n > 1 ? o->base_n : 1;
    if (n < 1) return REF_ERR_SHAPE;
    if (!ref_chain_ok(n, nbase)) return nbase == 1 ? REF_ERR_SHAPE : REF_ERR_ARG;
    long N = ref_points(dim, n);
    memset(res, 0, sizeof(*res));
    double nb = ref_norm2(b, N);
    if (nb != nb || isinf(nb)) return REF_ERR_NONFINITE;
    if (nb == 0.0) {                      /* A u = 0 has the solution u = 0 */
        memset(u, 0, sizeof(double) * N);
        if (history && hist_cap > 0) history[0] = 0.0;
        return REF_OK;
    }
    const int cycles = o->cycles > 1 ? o->cycles : 1;
    double *r = (double *)malloc(sizeof(double) * N);
    double *rl = (double *)malloc(sizeof(double) * N);
    double *c = (double *)malloc(sizeof(double) * N);
    double *ac = (double *)malloc(sizeof(double) * N);
    double *t = cycles > 1 ? (double *)malloc(sizeof(double) * N) : NULL;
    double *e = cycles > 1 ? (double *)malloc(sizeof(double) * N) : NULL;
    if (!r || !rl || !c || !ac || (cycles > 1 && (!t || !e))) {
        free(r); free(rl); free(c); free(ac); free(t); free(e);
        return REF_ERR_NOMEM;
    }

    if (!o->use_initial_guess) memset(u, 0, sizeof(double) * N);
    ref_residual_d(dim, n, disc, b, u, r);
    int st = REF_OK;
    int k = 0;
    for (;;) {
        double rn = ref_norm2(r, N);
        if (history && k < hist_cap) history[k] = rn / nb;
        res->rel_residual = rn / nb;
        if (rn != rn || isinf(rn)) { st = REF_ERR_NONFINITE; break; }
        if (rn <= o->rtol * nb) break;
        if (k >= o->max_iter) { st = REF_ERR_NOT_CONVERGED; break; }
        double alpha = o->residual_scaling ? ref_norminf(r, N) : 1.0;
        double inv_alpha = 1.0 / alpha;
        for (long p = 0; p < N; p++) rl[p] = inv_alpha * r[p];
        int vs = ref_vcycle_disc(dim, n, disc, nbase, o->nu1, o->nu2, o->omega, o->base_tol, o->base_max_iter,
                                 rl, c);
        for (int j = 1; j < cycles && vs == REF_OK; j++) {
            ref_residual_d(dim, n, disc, rl, c, t);
            vs = ref_vcycle_disc(dim, n, disc, nbase, o->nu1, o->nu2, o->omega, o->base_tol, o->base_max_iter,
                                 t, e);
            for (long p = 0; p < N; p++) c[p] += e[p];
        }
        if (vs != REF_OK) { st = vs; break; }
        for (long p = 0; p < N; p++) u[p] += alpha * c[p];
        if (o->recursive_residual) {
            ref_apply_A_disc(dim, n, disc, c, ac);
            for (long p = 0; p < N; p++) r[p] -= alpha * ac[p];
        } else {
            ref_residual_d(dim, n, disc, b, u, r);
        }
        k++;
    }
    res->iterations = k;
    ref_residual_d(dim, n, disc, b, u, ac);
    res->true_rel_residual = ref_norm2(ac, N) / nb;
    free(r); free(rl); free(c); free(ac); free(t); free(e);
    return st;
}
