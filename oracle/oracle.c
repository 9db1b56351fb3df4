/*
 * oracle.c -- plain, slow, FP64 CPU oracle of the consistent-SPH
 * advection-dispersion step (Klapp, Sigalotti, Alvarado-Rodriguez & Rendon,
 * "Consistent SPH simulations of the anisotropic dispersion of a contaminant
 * plume", arXiv:2108.09488).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or constant with
 * the HIP implementation.
 *
 * Everything is written straight from the paper's equations, in FP64, with no
 * blocking, fusion or reordering beyond what the equations state:
 *   Eq. (1)-(2)   Lagrangian advection-dispersion equation
 *   Eq. (3)       dispersion tensor D(v; alpha_L, alpha_T, D_m)
 *   Eq. (4)-(5)   SPH form of d C / d t (dispersion part and convective part)
 *   Eq. (7)       Wendland C4 kernel (and the Wendland C2 kernel, same family)
 *   Eq. (8)-(9)   predictor-corrector update; explicit Euler as the one-stage case
 *   Eq. (10)      time-step rule
 *   Eq. (11)-(13) Gaussian plume and its closed-form solution under uniform flow
 *                 (with the typo of the printed denominator corrected, see below)
 *
 * Readings of points the paper leaves open (each also listed in the design notes):
 *   R1  W(q) vanishes for q = r/H > 1: H is the support radius of the kernel.
 *   R2  Gamma = 4 in 2D (Eq. 5); in d dimensions Gamma = d + 2.
 *   R3  The elementwise harmonic mean 4 D_a D_b / (D_a + D_b) of Eq. (5) is taken
 *       as 0 when D_ij,a * D_ij,b <= 0 (covers the 0/0 of a vanishing entry).
 *   R4  The pair sum runs over b != a with 0 < |x_ab| <= H (inclusive support).
 *   R5  The box is periodic; x_ab is the minimum-image separation.
 *   R6  Predictor-corrector: x^{1/2} = x^l + dt/2 v, C^{1/2} = C^l + dt/2 rhs(C^l, x^l),
 *       then C^{l+1} = C^l + dt rhs(C^{1/2}, x^{1/2}), x^{l+1} = x^l + dt v.
 *   R7  Eq. (12): the denominator term 2 w^2 is read 2 w^4 (dimensional check;
 *       it is then the Green's-function convolution) and the centre is advected,
 *       x0 -> x0 + v t.
 *   R8  Shepard interpolation C_s = sum_b W_sb C_b / sum_b W_sb at sensor points
 *       (equal particle volumes cancel), J = sum_s (C_s - d_s)^2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Problem description                                                        */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t dim;      /* 2 or 3 */
    int32_t kernel;   /* 2 = Wendland C2, 4 = Wendland C4 (Eq. 7) */
    double H;         /* support radius (R1) */
    double L;         /* side of the periodic box (R5) */
    double alpha_L;   /* longitudinal dispersivity, Eq. (3) */
    double alpha_T;   /* transverse dispersivity, Eq. (3) */
    double D_m;       /* molecular diffusion, Eq. (3) */
    double gamma;     /* Gamma of Eq. (5); R2 */
} or_model;

/* ------------------------------------------------------------------------- */
/* Kernel, Eq. (7): W(q) = B (1-q)^6 (1 + 6 q + 35 q^2 / 3), q = r / H <= 1.   */
/* Wendland C2: W(q) = B (1-q)^4 (1 + 4 q).                                    */
/* B normalises the integral of W over the support to 1: B = 9/(pi H^2) for    */
/* C4 in 2D (as printed in the paper); the others follow from the same         */
/* normalisation: C4 3D 495/(32 pi H^3), C2 2D 7/(pi H^2), C2 3D 21/(2 pi H^3).*/
/* ------------------------------------------------------------------------- */
double or_kernel_B(int kernel, int dim, double H)
{
    if (kernel == 4 && dim == 2) return 9.0 / (OR_PI * H * H);
    if (kernel == 4 && dim == 3) return 495.0 / (32.0 * OR_PI * H * H * H);
    if (kernel == 2 && dim == 2) return 7.0 / (OR_PI * H * H);
    if (kernel == 2 && dim == 3) return 21.0 / (2.0 * OR_PI * H * H * H);
    return NAN;
}

double or_kernel_W(int kernel, int dim, double H, double r)
{
    double q = r / H;
    if (q > 1.0) return 0.0;
    double B = or_kernel_B(kernel, dim, H);
    double omq = 1.0 - q;
    if (kernel == 4)
        return B * pow(omq, 6) * (1.0 + 6.0 * q + 35.0 / 3.0 * q * q);
    return B * pow(omq, 4) * (1.0 + 4.0 * q);
}

/* dW/dr, by differentiating the polynomials above with respect to q and
 * multiplying by dq/dr = 1/H:
 *   C4: d/dq = -(56/3) q (1-q)^5 (1 + 5q)
 *   C2: d/dq = -20 q (1-q)^3                                                 */
double or_kernel_dWdr(int kernel, int dim, double H, double r)
{
    double q = r / H;
    if (q > 1.0) return 0.0;
    double B = or_kernel_B(kernel, dim, H);
    double omq = 1.0 - q;
    if (kernel == 4)
        return B / H * (-56.0 / 3.0) * q * pow(omq, 5) * (1.0 + 5.0 * q);
    return B / H * (-20.0) * q * pow(omq, 3);
}

/* ------------------------------------------------------------------------- */
/* Eq. (3): D_ij = (alpha_T |v| + D_m) delta_ij + (alpha_L - alpha_T) v_i v_j / |v| */
/* For |v| = 0 the second term is taken as 0.                                 */
/* ------------------------------------------------------------------------- */
void or_dispersion(int dim, double aL, double aT, double Dm, const double *v, double *D)
{
    double speed2 = 0.0;
    for (int i = 0; i < dim; ++i) speed2 += v[i] * v[i];
    double speed = sqrt(speed2);
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            double d = (i == j) ? (aT * speed + Dm) : 0.0;
            if (speed > 0.0) d += (aL - aT) * v[i] * v[j] / speed;
            D[i * dim + j] = d;
        }
}

/* Eq. (5) prefactor: elementwise 4 D_ij,a D_ij,b / (D_ij,a + D_ij,b)  (R3). */
void or_harmonic(int dim, const double *Da, const double *Db, double *h)
{
    for (int k = 0; k < dim * dim; ++k) {
        double p = Da[k] * Db[k];
        h[k] = (p > 0.0) ? 4.0 * p / (Da[k] + Db[k]) : 0.0;
    }
}

/* ------------------------------------------------------------------------- */
/* Geometry                                                                   */
/* ------------------------------------------------------------------------- */
static double min_image(double d, double L)
{
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

static double wrap_pos(double x, double L)
{
    if (x >= L) x -= L;
    if (x < 0.0) x += L;
    if (x >= L) x = 0.0;
    return x;
}

/* Separation x_ab (minimum image) and |x_ab|^2 for SoA positions x[c*n + a]. */
static double separation(const or_model *m, int64_t n, const double *x, int64_t a, int64_t b,
                         double *xab)
{
    double r2 = 0.0;
    for (int c = 0; c < m->dim; ++c) {
        xab[c] = min_image(x[c * n + a] - x[c * n + b], m->L);
        r2 += xab[c] * xab[c];
    }
    return r2;
}

/* ------------------------------------------------------------------------- */
/* Cell-linked list (Hockney & Eastwood style head / next chains) on cells of  */
/* side >= H; neighbours of a are searched in the 3^d surrounding cells.       */
/* When fewer than 3 cells fit along a side the search falls back to all       */
/* particles (brute force), which is always correct.                           */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t nc;         /* cells per side */
    int64_t ncell;      /* nc^dim */
    int64_t *head;      /* first particle in each cell, -1 = empty */
    int64_t *next;      /* next particle in the same cell */
} or_cells;

static int64_t cell_coord(double x, double L, int64_t nc)
{
    int64_t c = (int64_t)floor(x / L * (double)nc);
    if (c < 0) c = 0;
    if (c >= nc) c = nc - 1;
    return c;
}

static void cells_build(const or_model *m, int64_t n, const double *x, or_cells *cl)
{
    /* cells a little wider than H, so that a pair two cells apart is farther
     * than H even after rounding of the separation */
    int64_t nc = (int64_t)floor(m->L / (m->H * (1.0 + 1e-6)));
    int64_t cap = (m->dim == 2) ? 4096 : 256;
    if (nc > cap) nc = cap;
    cl->nc = nc;
    cl->ncell = 1;
    for (int c = 0; c < m->dim; ++c) cl->ncell *= nc;
    cl->head = NULL;
    cl->next = NULL;
    if (nc < 3) return;
    cl->head = (int64_t *)malloc(sizeof(int64_t) * cl->ncell);
    cl->next = (int64_t *)malloc(sizeof(int64_t) * n);
    for (int64_t k = 0; k < cl->ncell; ++k) cl->head[k] = -1;
    /* insert in reverse index order so each chain lists particles ascending */
    for (int64_t a = n - 1; a >= 0; --a) {
        int64_t key = 0;
        for (int c = m->dim - 1; c >= 0; --c) key = key * nc + cell_coord(x[c * n + a], m->L, nc);
        cl->next[a] = cl->head[key];
        cl->head[key] = a;
    }
}

static void cells_free(or_cells *cl)
{
    free(cl->head);
    free(cl->next);
}

/* Visit every b with 0 < |x_ab| <= H (R4, R5); calls fn(b, xab, r2, ctx). */
typedef void (*or_visit_fn)(int64_t b, const double *xab, double r2, void *ctx);

static void for_neighbours(const or_model *m, int64_t n, const double *x, const or_cells *cl,
                           const double *xa_pos, int64_t a, or_visit_fn fn, void *ctx)
{
    double H2 = m->H * m->H;
    double xab[3];
    if (cl->head == NULL) {
        for (int64_t b = 0; b < n; ++b) {
            if (b == a) continue;
            double r2 = 0.0;
            for (int c = 0; c < m->dim; ++c) {
                xab[c] = min_image(xa_pos[c] - x[c * n + b], m->L);
                r2 += xab[c] * xab[c];
            }
            if (r2 > 0.0 && r2 <= H2) fn(b, xab, r2, ctx);
        }
        return;
    }
    int64_t nc = cl->nc, ca[3] = {0, 0, 0};
    for (int c = 0; c < m->dim; ++c) ca[c] = cell_coord(xa_pos[c], m->L, nc);
    int oz_lo = (m->dim == 3) ? -1 : 0, oz_hi = (m->dim == 3) ? 1 : 0;
    for (int oz = oz_lo; oz <= oz_hi; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                int64_t cx = (ca[0] + ox + nc) % nc, cy = (ca[1] + oy + nc) % nc;
                int64_t cz = (m->dim == 3) ? (ca[2] + oz + nc) % nc : 0;
                int64_t key = (cz * nc + cy) * nc + cx;
                for (int64_t b = cl->head[key]; b >= 0; b = cl->next[b]) {
                    if (b == a) continue;
                    double r2 = 0.0;
                    for (int c = 0; c < m->dim; ++c) {
                        xab[c] = min_image(xa_pos[c] - x[c * n + b], m->L);
                        r2 += xab[c] * xab[c];
                    }
                    if (r2 > 0.0 && r2 <= H2) fn(b, xab, r2, ctx);
                }
            }
}

/* ------------------------------------------------------------------------- */
/* Neighbour sets                                                             */
/* ------------------------------------------------------------------------- */
/* FP64 predicate, brute force over all pairs (O(N^2)); writes counts[a]. If ids
 * is non-NULL, offsets (n+1) must be filled by the caller from the counts and
 * the ids of a's neighbours are written in ascending order. */
void or_neighbours_brute(const or_model *m, int64_t n, const double *x, int64_t *counts,
                         const int64_t *offsets, int32_t *ids)
{
    double H2 = m->H * m->H;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < n; ++a) {
        int64_t k = 0;
        double xab[3];
        for (int64_t b = 0; b < n; ++b) {
            if (b == a) continue;
            double r2 = separation(m, n, x, a, b, xab);
            if (r2 > 0.0 && r2 <= H2) {
                if (ids) ids[offsets[a] + k] = (int32_t)b;
                ++k;
            }
        }
        counts[a] = k;
    }
}

typedef struct {
    int32_t *out;
    int64_t k;
} collect_ctx;

static void collect_visit(int64_t b, const double *xab, double r2, void *vctx)
{
    (void)xab; (void)r2;
    collect_ctx *c = (collect_ctx *)vctx;
    if (c->out) c->out[c->k] = (int32_t)b;
    c->k++;
}

static int cmp_i32(const void *p, const void *q)
{
    int32_t a = *(const int32_t *)p, b = *(const int32_t *)q;
    return (a > b) - (a < b);
}

/* Same sets as or_neighbours_brute, found through the cell-linked list. */
void or_neighbours_cells(const or_model *m, int64_t n, const double *x, int64_t *counts,
                         const int64_t *offsets, int32_t *ids)
{
    or_cells cl;
    cells_build(m, n, x, &cl);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < n; ++a) {
        double xa[3];
        for (int c = 0; c < m->dim; ++c) xa[c] = x[c * n + a];
        collect_ctx cc = {ids ? ids + offsets[a] : NULL, 0};
        for_neighbours(m, n, x, &cl, xa, a, collect_visit, &cc);
        counts[a] = cc.k;
        if (ids) qsort(ids + offsets[a], (size_t)cc.k, sizeof(int32_t), cmp_i32);
    }
    cells_free(&cl);
}

/* Neighbour predicate evaluated the way a program holding positions as 32-bit
 * fixed-point fractions of the box decides it: u = x / L * 2^32 (uint32),
 * separation in grid units d = (int32)(u_a - u_b) (two's-complement wrap gives
 * the minimum image), converted to the working precision (real_bytes 4: float,
 * 8: double), r2 = d_x*d_x, then r2 = fma(d_y, d_y, r2) [, r2 = fma(d_z, d_z, r2)],
 * pair iff 0 < r2 <= H_u^2 with H_u = H / L * 2^32 and H_u^2 formed in double
 * and rounded to the working precision.
 * Candidates come from a cell list on the fixed-point grid with cells wider
 * than H_u (1 + 2^-16), so that a pair two cells apart fails the predicate even
 * after the rounding of d; brute force when fewer than 3 cells fit. */
static int fixed_keep(int dim, int real_bytes, const uint32_t *ua, const uint32_t *ub,
                      float H2f, double H2d)
{
    if (real_bytes == 4) {
        float d[3] = {0.0f, 0.0f, 0.0f};
        for (int c = 0; c < dim; ++c) d[c] = (float)(int32_t)(ua[c] - ub[c]);
        float r2 = d[0] * d[0];
        r2 = fmaf(d[1], d[1], r2);
        if (dim == 3) r2 = fmaf(d[2], d[2], r2);
        return (r2 > 0.0f) && (r2 <= H2f);
    }
    double d[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < dim; ++c) d[c] = (double)(int32_t)(ua[c] - ub[c]);
    double r2 = d[0] * d[0];
    r2 = fma(d[1], d[1], r2);
    if (dim == 3) r2 = fma(d[2], d[2], r2);
    return (r2 > 0.0) && (r2 <= H2d);
}

void or_neighbours_fixed(int dim, int64_t n, const uint32_t *u, double L, double H,
                         int real_bytes, int force_brute, int64_t *counts, const int64_t *offsets, int32_t *ids)
{
    double Hu = H / L * 4294967296.0;
    double H2d = Hu * Hu;
    float H2f = (float)H2d;
    int64_t nc = (int64_t)floor(4294967296.0 / (Hu * (1.0 + 1.0 / 65536.0)));
    int64_t cap = (dim == 2) ? 4096 : 256;
    if (nc > cap) nc = cap;
    int64_t ncell = 1;
    for (int c = 0; c < dim; ++c) ncell *= nc;
    int64_t *head = NULL, *next = NULL;
    if (nc >= 3 && !force_brute) {
        head = (int64_t *)malloc(sizeof(int64_t) * ncell);
        next = (int64_t *)malloc(sizeof(int64_t) * n);
        for (int64_t k = 0; k < ncell; ++k) head[k] = -1;
        for (int64_t a = n - 1; a >= 0; --a) {
            int64_t key = 0;
            for (int c = dim - 1; c >= 0; --c)
                key = key * nc + (int64_t)(((uint64_t)u[c * n + a] * (uint64_t)nc) >> 32);
            next[a] = head[key];
            head[key] = a;
        }
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < n; ++a) {
        uint32_t ua[3], ub[3];
        for (int c = 0; c < dim; ++c) ua[c] = u[c * n + a];
        int64_t k = 0;
        int32_t *out = ids ? ids + offsets[a] : NULL;
        if (head == NULL) {
            for (int64_t b = 0; b < n; ++b) {
                if (b == a) continue;
                for (int c = 0; c < dim; ++c) ub[c] = u[c * n + b];
                if (fixed_keep(dim, real_bytes, ua, ub, H2f, H2d)) {
                    if (out) out[k] = (int32_t)b;
                    ++k;
                }
            }
        } else {
            int64_t ca[3] = {0, 0, 0};
            for (int c = 0; c < dim; ++c) ca[c] = (int64_t)(((uint64_t)ua[c] * (uint64_t)nc) >> 32);
            int oz_lo = (dim == 3) ? -1 : 0, oz_hi = (dim == 3) ? 1 : 0;
            for (int oz = oz_lo; oz <= oz_hi; ++oz)
                for (int oy = -1; oy <= 1; ++oy)
                    for (int ox = -1; ox <= 1; ++ox) {
                        int64_t cx = (ca[0] + ox + nc) % nc, cy = (ca[1] + oy + nc) % nc;
                        int64_t cz = (dim == 3) ? (ca[2] + oz + nc) % nc : 0;
                        for (int64_t b = head[(cz * nc + cy) * nc + cx]; b >= 0; b = next[b]) {
                            if (b == a) continue;
                            for (int c = 0; c < dim; ++c) ub[c] = u[c * n + b];
                            if (fixed_keep(dim, real_bytes, ua, ub, H2f, H2d)) {
                                if (out) out[k] = (int32_t)b;
                                ++k;
                            }
                        }
                    }
            if (out) qsort(out, (size_t)k, sizeof(int32_t), cmp_i32);
        }
        counts[a] = k;
    }
    free(head);
    free(next);
}

/* ------------------------------------------------------------------------- */
/* Right-hand side, Eq. (4) with Eq. (5):                                      */
/*   (dC/dt)_a = 1/2 sum_b (m_b / rhobar_ab) Dcal_ab (C_a - C_b) / |x_ab|^2     */
/*                        x_ab . grad_a W_ab                                    */
/*             + C_a sum_b (m_b / rhobar_ab) sum_i (v_i,a - v_i,b) dW_ab/dx_i,a */
/*   Dcal_ab = sum_ij h_ij [Gamma x_i x_j / |x_ab|^2 - delta_ij],               */
/*   h_ij = 4 D_ij,a D_ij,b / (D_ij,a + D_ij,b),  rhobar_ab = (rho_a+rho_b)/2.  */
/* grad_a W_ab = dW/dr (x_ab / r).                                             */
/* v is per particle (SoA, dim x n); m and rho are per particle.              */
/* ------------------------------------------------------------------------- */
typedef struct {
    const or_model *m;
    int64_t n, a;
    const double *x, *C, *v, *mass, *rho, *D; /* D: per-particle tensors, n x dim*dim */
    const double *Dfix;  /* if non-NULL: h_ij replaced by this tensor for every pair */
    double disp, conv;
    int dk;              /* 0: Eq. (4); k = 1..3: the derivative of its dispersion part with
                            respect to theta_k = (alpha_L, alpha_T, D_m) for per-particle
                            tensors (h_ij replaced by dh_ij/dtheta_k, no convective part) */
} rhs_ctx;

/* dD/dtheta_k of Eq. (3) at velocity v (k = 0: alpha_L, 1: alpha_T, 2: D_m):
 * v v^T/|v|, |v| I - v v^T/|v|, I (the v v^T/|v| parts taken as 0 for v = 0). */
static void dispersion_deriv(int dim, int k, const double *v, double *dD)
{
    double speed2 = 0.0;
    for (int i = 0; i < dim; ++i) speed2 += v[i] * v[i];
    double speed = sqrt(speed2);
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            double vv = speed > 0.0 ? v[i] * v[j] / speed : 0.0;
            double id = (i == j) ? 1.0 : 0.0;
            dD[i * dim + j] = (k == 0) ? vv : (k == 1) ? speed * id - vv : id;
        }
}

/* dh/dtheta of the harmonic mean h = 4 p q / (p + q) of Eq. (5), elementwise:
 * 4 (q^2 dp + p^2 dq) / (p + q)^2, and 0 where p q <= 0 (R3). */
static void harmonic_deriv(int dim, const double *Da, const double *Db, const double *dDa,
                           const double *dDb, double *dh)
{
    for (int k = 0; k < dim * dim; ++k) {
        double p = Da[k], q = Db[k];
        dh[k] = (p * q > 0.0) ? 4.0 * (q * q * dDa[k] + p * p * dDb[k]) / ((p + q) * (p + q)) : 0.0;
    }
}

static void rhs_visit(int64_t b, const double *xab, double r2, void *vctx)
{
    rhs_ctx *c = (rhs_ctx *)vctx;
    const or_model *m = c->m;
    int dim = m->dim;
    int64_t a = c->a, n = c->n;
    double r = sqrt(r2);
    double dWdr = or_kernel_dWdr(m->kernel, dim, m->H, r);
    double gradW[3];
    for (int i = 0; i < dim; ++i) gradW[i] = dWdr * xab[i] / r;
    double rhobar = 0.5 * (c->rho[a] + c->rho[b]);
    double vol = c->mass[b] / rhobar;
    double h[9];
    if (c->Dfix) memcpy(h, c->Dfix, sizeof(double) * dim * dim);
    else if (c->dk > 0) {
        double va[3] = {0, 0, 0}, vb[3] = {0, 0, 0}, dDa[9], dDb[9];
        for (int i = 0; i < dim; ++i) {
            va[i] = c->v[i * n + a];
            vb[i] = c->v[i * n + b];
        }
        dispersion_deriv(dim, c->dk - 1, va, dDa);
        dispersion_deriv(dim, c->dk - 1, vb, dDb);
        harmonic_deriv(dim, c->D + a * dim * dim, c->D + b * dim * dim, dDa, dDb, h);
    } else or_harmonic(dim, c->D + a * dim * dim, c->D + b * dim * dim, h);
    double Dcal = 0.0;
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j)
            Dcal += h[i * dim + j] * (m->gamma * xab[i] * xab[j] / r2 - (i == j ? 1.0 : 0.0));
    double xdotgrad = 0.0;
    for (int i = 0; i < dim; ++i) xdotgrad += xab[i] * gradW[i];
    c->disp += 0.5 * vol * Dcal * (c->C[a] - c->C[b]) / r2 * xdotgrad;
    if (c->v && c->dk == 0) {
        double s = 0.0;
        for (int i = 0; i < dim; ++i) s += (c->v[i * n + a] - c->v[i * n + b]) * gradW[i];
        c->conv += vol * s;
    }
}

static double *tensors_per_particle(const or_model *m, int64_t n, const double *v, const double *vu)
{
    int dim = m->dim;
    double *D = (double *)malloc(sizeof(double) * n * dim * dim);
    for (int64_t a = 0; a < n; ++a) {
        double va[3] = {0, 0, 0};
        for (int c = 0; c < dim; ++c) va[c] = v ? v[c * n + a] : vu[c];
        or_dispersion(dim, m->alpha_L, m->alpha_T, m->D_m, va, D + a * dim * dim);
    }
    return D;
}

/* rhs for the particles idx[0..nidx) (idx NULL: all, nidx = n).
 *   v     per-particle velocity (dim x n) or NULL for the uniform velocity vu
 *   mass, rho per particle
 *   Dfix  NULL, or a dim x dim tensor used in place of the harmonic mean h_ij
 *         (used for the derivative operators of the adjoint)
 *   out   rhs of Eq. (4) per listed particle                                  */
void or_rhs(const or_model *m, int64_t n, const double *x, const double *C, const double *v,
            const double *vu, const double *mass, const double *rho, const double *Dfix,
            int64_t nidx, const int64_t *idx, double *out)
{
    or_cells cl;
    cells_build(m, n, x, &cl);
    double *D = tensors_per_particle(m, n, v, vu);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < nidx; ++k) {
        int64_t a = idx ? idx[k] : k;
        rhs_ctx c = {m, n, a, x, C, v, mass, rho, D, Dfix, 0.0, 0.0};
        double xa[3];
        for (int i = 0; i < m->dim; ++i) xa[i] = x[i * n + a];
        for_neighbours(m, n, x, &cl, xa, a, rhs_visit, &c);
        out[k] = c.disp + C[a] * c.conv;
    }
    free(D);
    cells_free(&cl);
}

/* Same sums by brute force over all b (O(N^2)), for checking the cell list. */
void or_rhs_brute(const or_model *m, int64_t n, const double *x, const double *C,
                  const double *v, const double *vu, const double *mass, const double *rho,
                  double *out)
{
    double *D = tensors_per_particle(m, n, v, vu);
    or_cells none = {0, 0, NULL, NULL};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < n; ++a) {
        rhs_ctx c = {m, n, a, x, C, v, mass, rho, D, NULL, 0.0, 0.0};
        double xa[3];
        for (int i = 0; i < m->dim; ++i) xa[i] = x[i * n + a];
        for_neighbours(m, n, x, &none, xa, a, rhs_visit, &c);
        out[a] = c.disp + C[a] * c.conv;
    }
    free(D);
}

/* ------------------------------------------------------------------------- */
/* Time integration.  integrator 1: explicit Euler                             */
/*   C^{l+1} = C^l + dt rhs(C^l, x^l),  x^{l+1} = x^l + dt v;                  */
/* integrator 2: predictor-corrector of Eqs. (8)-(9) with reading R6.          */
/* Positions are wrapped into [0, L).  mass_hist (nsteps+1 entries, or NULL)   */
/* receives sum_a m_a C_a before the first and after every step.             */
/* ------------------------------------------------------------------------- */
double or_mass(int64_t n, const double *mass, const double *C)
{
    double s = 0.0;
    for (int64_t a = 0; a < n; ++a) s += mass[a] * C[a];
    return s;
}

static void advect(const or_model *m, int64_t n, const double *x, const double *v,
                   const double *vu, double tau, double *out)
{
    for (int c = 0; c < m->dim; ++c)
        for (int64_t a = 0; a < n; ++a)
            out[c * n + a] = wrap_pos(x[c * n + a] + tau * (v ? v[c * n + a] : vu[c]), m->L);
}

void or_run(const or_model *m, int64_t n, double *x, double *C, const double *v,
            const double *vu, const double *mass, const double *rho, double dt,
            int64_t nsteps, int integrator, double *mass_hist)
{
    int dim = m->dim;
    double *rhs = (double *)malloc(sizeof(double) * n);
    double *Ch = (double *)malloc(sizeof(double) * n);
    double *xh = (double *)malloc(sizeof(double) * n * dim);
    if (mass_hist) mass_hist[0] = or_mass(n, mass, C);
    for (int64_t s = 0; s < nsteps; ++s) {
        if (integrator == 2) {
            or_rhs(m, n, x, C, v, vu, mass, rho, NULL, n, NULL, rhs);
            for (int64_t a = 0; a < n; ++a) Ch[a] = C[a] + 0.5 * dt * rhs[a];
            advect(m, n, x, v, vu, 0.5 * dt, xh);
            or_rhs(m, n, xh, Ch, v, vu, mass, rho, NULL, n, NULL, rhs);
        } else {
            or_rhs(m, n, x, C, v, vu, mass, rho, NULL, n, NULL, rhs);
        }
        for (int64_t a = 0; a < n; ++a) C[a] += dt * rhs[a];
        advect(m, n, x, v, vu, dt, xh);
        memcpy(x, xh, sizeof(double) * n * dim);
        if (mass_hist) mass_hist[s + 1] = or_mass(n, mass, C);
    }
    free(rhs);
    free(Ch);
    free(xh);
}

/* Eq. (10): dt = C min_a H_s^2 / (sum_i D_ii,a) with C = 0.1, for a uniform
 * velocity; hs is the length used in the rule. */
double or_dt_rule(const or_model *m, const double *vu, double hs)
{
    double D[9];
    or_dispersion(m->dim, m->alpha_L, m->alpha_T, m->D_m, vu, D);
    double tr = 0.0;
    for (int i = 0; i < m->dim; ++i) tr += D[i * m->dim + i];
    return 0.1 * hs * hs / tr;
}

/* ------------------------------------------------------------------------- */
/* Closed-form plume under uniform flow, Eqs. (12)-(13) with reading R7.       */
/* 2D: C/C0 = w^2 / C4 exp[(-X^2 A1 - Y^2 A2 + 4 X Y A3) / (8 t^2 C2 +         */
/*     4 w^2 t C3 + 2 w^4)], X, Y measured from the advected centre.           */
/* 3D: the same Gaussian law, amplitude w^3 / sqrt(det S) and exponent         */
/*     -1/2 X^T S^{-1} X with S = w^2 I + 2 D t.                               */
/* Summed over the 3^d periodic images.                                        */
/* ------------------------------------------------------------------------- */
void or_analytic(const or_model *m, const double *vu, const double *x0, double w, double C0,
                 double t, int64_t n, const double *x, double *out)
{
    int dim = m->dim;
    double D[9];
    or_dispersion(dim, m->alpha_L, m->alpha_T, m->D_m, vu, D);
    double centre[3];
    for (int c = 0; c < dim; ++c) centre[c] = x0[c] + vu[c] * t;
    double w2 = w * w;
    double A1 = 0, A2 = 0, A3 = 0, C2 = 0, C3 = 0, C4 = 0, Sinv[9], amp3 = 0;
    if (dim == 2) {
        double Dxx = D[0], Dxy = D[1], Dyy = D[3];
        A1 = 2.0 * t * Dyy + w2;
        A2 = 2.0 * t * Dxx + w2;
        A3 = t * Dxy;
        C2 = Dxx * Dyy - Dxy * Dxy;
        C3 = Dxx + Dyy;
        C4 = sqrt(4.0 * t * t * C2 + 2.0 * t * w2 * C3 + w2 * w2);
    } else {
        double S[9];
        for (int i = 0; i < 9; ++i) S[i] = 2.0 * t * D[i] + ((i % 4) == 0 ? w2 : 0.0);
        double det = S[0] * (S[4] * S[8] - S[5] * S[7]) - S[1] * (S[3] * S[8] - S[5] * S[6]) +
                     S[2] * (S[3] * S[7] - S[4] * S[6]);
        Sinv[0] = (S[4] * S[8] - S[5] * S[7]) / det;
        Sinv[1] = (S[2] * S[7] - S[1] * S[8]) / det;
        Sinv[2] = (S[1] * S[5] - S[2] * S[4]) / det;
        Sinv[3] = (S[5] * S[6] - S[3] * S[8]) / det;
        Sinv[4] = (S[0] * S[8] - S[2] * S[6]) / det;
        Sinv[5] = (S[2] * S[3] - S[0] * S[5]) / det;
        Sinv[6] = (S[3] * S[7] - S[4] * S[6]) / det;
        Sinv[7] = (S[1] * S[6] - S[0] * S[7]) / det;
        Sinv[8] = (S[0] * S[4] - S[1] * S[3]) / det;
        amp3 = w2 * w / sqrt(det);
    }
    for (int64_t a = 0; a < n; ++a) {
        double acc = 0.0;
        int iz_lo = (dim == 3) ? -1 : 0, iz_hi = (dim == 3) ? 1 : 0;
        for (int iz = iz_lo; iz <= iz_hi; ++iz)
            for (int iy = -1; iy <= 1; ++iy)
                for (int ix = -1; ix <= 1; ++ix) {
                    int img[3] = {ix, iy, iz};
                    double X[3] = {0.0, 0.0, 0.0};
                    for (int c = 0; c < dim; ++c) {
                        double d = x[c * n + a] - centre[c];
                        d -= m->L * floor(d / m->L + 0.5); /* nearest image of the centre */
                        X[c] = d + img[c] * m->L;
                    }
                    if (dim == 2) {
                        double num = -X[0] * X[0] * A1 - X[1] * X[1] * A2 + 4.0 * X[0] * X[1] * A3;
                        double den = 8.0 * t * t * C2 + 4.0 * w2 * t * C3 + 2.0 * w2 * w2;
                        acc += w2 / C4 * exp(num / den);
                    } else {
                        double q = 0.0;
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j) q += X[i] * Sinv[i * 3 + j] * X[j];
                        acc += amp3 * exp(-0.5 * q);
                    }
                }
        out[a] = C0 * acc;
    }
}

/* ------------------------------------------------------------------------- */
/* Sensors (R8): Shepard interpolation with the same kernel and support.       */
/* Pc[s*n + b] = W_sb / sum_b' W_sb' is the interpolation matrix row s        */
/* (dense; only for small problems), or NULL.                                 */
/* ------------------------------------------------------------------------- */
void or_sensor_interp(const or_model *m, int64_t n, const double *x, const double *C,
                      int64_t ns, const double *xs, double *Cs, double *wsum_out)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t s = 0; s < ns; ++s) {
        double num = 0.0, den = 0.0;
        for (int64_t b = 0; b < n; ++b) {
            double r2 = 0.0;
            for (int c = 0; c < m->dim; ++c) {
                double d = min_image(xs[c * ns + s] - x[c * n + b], m->L);
                r2 += d * d;
            }
            if (r2 <= m->H * m->H) {
                double w = or_kernel_W(m->kernel, m->dim, m->H, sqrt(r2));
                num += w * C[b];
                den += w;
            }
        }
        Cs[s] = (den > 0.0) ? num / den : 0.0;
        if (wsum_out) wsum_out[s] = den;
    }
}

/* Transpose of the interpolation applied to a sensor vector g: out_b =
 * sum_s g_s W_sb / sum_b' W_sb'. */
static void sensor_interp_T(const or_model *m, int64_t n, const double *x, int64_t ns,
                            const double *xs, const double *g, double *out)
{
    double *den = (double *)calloc((size_t)ns, sizeof(double));
    for (int64_t s = 0; s < ns; ++s)
        for (int64_t b = 0; b < n; ++b) {
            double r2 = 0.0;
            for (int c = 0; c < m->dim; ++c) {
                double d = min_image(xs[c * ns + s] - x[c * n + b], m->L);
                r2 += d * d;
            }
            if (r2 <= m->H * m->H) den[s] += or_kernel_W(m->kernel, m->dim, m->H, sqrt(r2));
        }
    memset(out, 0, sizeof(double) * n);
    for (int64_t s = 0; s < ns; ++s) {
        if (den[s] <= 0.0) continue;
        for (int64_t b = 0; b < n; ++b) {
            double r2 = 0.0;
            for (int c = 0; c < m->dim; ++c) {
                double d = min_image(xs[c * ns + s] - x[c * n + b], m->L);
                r2 += d * d;
            }
            if (r2 <= m->H * m->H)
                out[b] += g[s] * or_kernel_W(m->kernel, m->dim, m->H, sqrt(r2)) / den[s];
        }
    }
    free(den);
}

/* ------------------------------------------------------------------------- */
/* Transposed operator: with rhs = L C written as rhs_a = sum_b w_ab (C_a - C_b) */
/* (+ the convective part, zero for uniform v), returns y = L^T lam, evaluated */
/* entry by entry (row b of L^T at a time).  Uniform velocity only.            */
/* ------------------------------------------------------------------------- */
/* Weight w_ij of the pair (i, j) in row i of the operator, for the separation
 * x_ij (r2 = |x_ij|^2): the dispersion term of Eq. (4) for particle i reads
 * sum_j w_ij (C_i - C_j) with
 *   w_ij = 1/2 (m_j / rhobar_ij) Dcal_ij x_ij . grad_i W_ij / |x_ij|^2. */
static double pair_weight(const or_model *m, const double *mass, const double *rho,
                          const double *h, int64_t i, int64_t j, const double *xij, double r2)
{
    int dim = m->dim;
    double r = sqrt(r2);
    double dWdr = or_kernel_dWdr(m->kernel, dim, m->H, r);
    double xdotgrad = 0.0;
    for (int k = 0; k < dim; ++k) xdotgrad += xij[k] * dWdr * xij[k] / r;
    double rhobar = 0.5 * (rho[i] + rho[j]);
    double Dcal = 0.0;
    for (int k = 0; k < dim; ++k)
        for (int l = 0; l < dim; ++l)
            Dcal += h[k * dim + l] * (m->gamma * xij[k] * xij[l] / r2 - (k == l ? 1.0 : 0.0));
    return 0.5 * mass[j] / rhobar * Dcal / r2 * xdotgrad;
}

typedef struct {
    const or_model *m;
    int64_t b;
    const double *mass, *rho, *h, *lam;
    double y;
} lt_ctx;

/* For row b of L^T: with L_aa = sum_j w_aj and L_ab = -w_ab (a != b),
 * (L^T lam)_b = sum_a L_ab lam_a = (sum_a w_ba) lam_b - sum_{a != b} w_ab lam_a,
 * visiting every neighbour a of b. */
static void lt_visit(int64_t a, const double *xba, double r2, void *vctx)
{
    lt_ctx *c = (lt_ctx *)vctx;
    double xab[3];
    for (int k = 0; k < c->m->dim; ++k) xab[k] = -xba[k];
    double w_ba = pair_weight(c->m, c->mass, c->rho, c->h, c->b, a, xba, r2);
    double w_ab = pair_weight(c->m, c->mass, c->rho, c->h, a, c->b, xab, r2);
    c->y += w_ba * c->lam[c->b] - w_ab * c->lam[a];
}

static void apply_LT(const or_model *m, int64_t n, const double *x, const double *mass,
                     const double *rho, const double *h, const double *lam, double *y)
{
    or_cells cl;
    cells_build(m, n, x, &cl);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < n; ++b) {
        lt_ctx c = {m, b, mass, rho, h, lam, 0.0};
        double xb[3];
        for (int i = 0; i < m->dim; ++i) xb[i] = x[i * n + b];
        for_neighbours(m, n, x, &cl, xb, b, lt_visit, &c);
        y[b] = c.y;
    }
    cells_free(&cl);
}

/* y = L^T lam with the harmonic-mean tensor of the model at uniform velocity. */
void or_apply_LT(const or_model *m, int64_t n, const double *x, const double *vu,
                 const double *mass, const double *rho, const double *lam, double *y)
{
    double D[9], h[9];
    or_dispersion(m->dim, m->alpha_L, m->alpha_T, m->D_m, vu, D);
    or_harmonic(m->dim, D, D, h);
    apply_LT(m, n, x, mass, rho, h, lam, y);
}

/* ------------------------------------------------------------------------- */
/* Discrete adjoint of the explicit run (uniform velocity), J = sum_s         */
/* (P C^N - d)_s^2 with P the sensor interpolation at the final positions:    */
/*   lam^N = P^T 2 (P C^N - d).                                                */
/* Euler (integrator 1): C^{n+1} = C^n + dt L1 C^n, L1 = L(x^n):               */
/*   lam^n = lam^{n+1} + dt L1^T lam^{n+1},                                    */
/*   dJ/dtheta_k += dt lam^{n+1} . L1_k C^n.                                   */
/* Predictor-corrector (integrator 2, Eqs. 8-9): C^h = C^n + dt/2 L1 C^n and   */
/* C^{n+1} = C^n + dt L2 C^h with L2 = L(x^n + dt/2 v), i.e. C^{n+1} =        */
/* (I + dt L2 + dt^2/2 L2 L1) C^n, so with y = L2^T lam^{n+1}:                 */
/*   lam^n = lam^{n+1} + dt y + dt^2/2 L1^T y,                                 */
/*   dJ/dtheta_k += dt lam^{n+1} . L2_k C^h + dt^2/2 y . L1_k C^n.             */
/* L_k is the operator with the tensor replaced by its derivative: theta =    */
/* (alpha_L, alpha_T, D_m); for a uniform tensor the harmonic mean of Eq. (5) */
/* is h = 2 D (entries with D_ij = 0 stay 0), so dh/dtheta_k = 2 dD/dtheta_k  */
/* with dD/dalpha_L = v v^T/|v|, dD/dalpha_T = |v| I - v v^T/|v|, dD/dD_m = I. */
/* All states are kept in memory (plain reverse sweep).                        */
/* ------------------------------------------------------------------------- */
void or_adjoint(const or_model *m, int64_t n, const double *x0, const double *C0,
                const double *vu, const double *mass, const double *rho, double dt,
                int64_t nsteps, int64_t ns, const double *xs, const double *obs,
                int integrator, double *J_out, double *grad_out, double *Cfinal_out)
{
    int dim = m->dim;
    double *X = (double *)malloc(sizeof(double) * dim * n * (nsteps + 1));
    double *Cs = (double *)malloc(sizeof(double) * n * (nsteps + 1));
    double *rhs = (double *)malloc(sizeof(double) * n);
    memcpy(X, x0, sizeof(double) * dim * n);
    memcpy(Cs, C0, sizeof(double) * n);
    double *Ch = (double *)malloc(sizeof(double) * n);
    double *xh = (double *)malloc(sizeof(double) * n * dim);
    /* C^h and x^h of step s: the predictor stage */
    #define HALF_STAGE(xs_n, C_n)                                                   \
        do {                                                                        \
            or_rhs(m, n, xs_n, C_n, NULL, vu, mass, rho, NULL, n, NULL, rhs);       \
            for (int64_t a = 0; a < n; ++a) Ch[a] = (C_n)[a] + 0.5 * dt * rhs[a];   \
            advect(m, n, xs_n, NULL, vu, 0.5 * dt, xh);                             \
        } while (0)
    for (int64_t s = 0; s < nsteps; ++s) {
        const double *xs_n = X + (size_t)s * dim * n;
        const double *C_n = Cs + (size_t)s * n;
        if (integrator == 2) {
            HALF_STAGE(xs_n, C_n);
            or_rhs(m, n, xh, Ch, NULL, vu, mass, rho, NULL, n, NULL, rhs);
        } else {
            or_rhs(m, n, xs_n, C_n, NULL, vu, mass, rho, NULL, n, NULL, rhs);
        }
        for (int64_t a = 0; a < n; ++a) Cs[(size_t)(s + 1) * n + a] = C_n[a] + dt * rhs[a];
        advect(m, n, xs_n, NULL, vu, dt, X + (size_t)(s + 1) * dim * n);
    }
    const double *xN = X + (size_t)nsteps * dim * n, *CN = Cs + (size_t)nsteps * n;
    double *pred = (double *)malloc(sizeof(double) * (ns > 0 ? ns : 1));
    double *g = (double *)malloc(sizeof(double) * (ns > 0 ? ns : 1));
    or_sensor_interp(m, n, xN, CN, ns, xs, pred, NULL);
    double J = 0.0;
    for (int64_t s = 0; s < ns; ++s) {
        double r = pred[s] - obs[s];
        J += r * r;
        g[s] = 2.0 * r;
    }
    double *lam = (double *)malloc(sizeof(double) * n);
    double *y = (double *)malloc(sizeof(double) * n);
    sensor_interp_T(m, n, xN, ns, xs, g, lam);

    double speed = 0.0;
    for (int c = 0; c < dim; ++c) speed += vu[c] * vu[c];
    speed = sqrt(speed);
    double dD[3][9], D[9], h[9];
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            double vv = speed > 0.0 ? vu[i] * vu[j] / speed : 0.0;
            double id = (i == j) ? 1.0 : 0.0;
            dD[0][i * dim + j] = 2.0 * vv;
            dD[1][i * dim + j] = 2.0 * (speed * id - vv);
            dD[2][i * dim + j] = 2.0 * id;
        }
    or_dispersion(dim, m->alpha_L, m->alpha_T, m->D_m, vu, D);
    or_harmonic(dim, D, D, h);
    double grad[3] = {0.0, 0.0, 0.0};
    double *z = (double *)malloc(sizeof(double) * n);
    for (int64_t s = nsteps - 1; s >= 0; --s) {
        const double *xs_n = X + (size_t)s * dim * n;
        const double *C_n = Cs + (size_t)s * n;
        if (integrator == 2) {
            HALF_STAGE(xs_n, C_n);
            apply_LT(m, n, xh, mass, rho, h, lam, y);  /* y = L2^T lam */
            for (int k = 0; k < 3; ++k) {
                double acc = 0.0;
                or_rhs(m, n, xh, Ch, NULL, vu, mass, rho, dD[k], n, NULL, rhs);
                for (int64_t a = 0; a < n; ++a) acc += dt * lam[a] * rhs[a];
                or_rhs(m, n, xs_n, C_n, NULL, vu, mass, rho, dD[k], n, NULL, rhs);
                for (int64_t a = 0; a < n; ++a) acc += 0.5 * dt * dt * y[a] * rhs[a];
                grad[k] += acc;
            }
            apply_LT(m, n, xs_n, mass, rho, h, y, z);   /* z = L1^T y */
            for (int64_t a = 0; a < n; ++a) lam[a] += dt * y[a] + 0.5 * dt * dt * z[a];
        } else {
            for (int k = 0; k < 3; ++k) {
                or_rhs(m, n, xs_n, C_n, NULL, vu, mass, rho, dD[k], n, NULL, rhs);
                double acc = 0.0;
                for (int64_t a = 0; a < n; ++a) acc += lam[a] * rhs[a];
                grad[k] += dt * acc;
            }
            apply_LT(m, n, xs_n, mass, rho, h, lam, y);
            for (int64_t a = 0; a < n; ++a) lam[a] += dt * y[a];
        }
    }
    #undef HALF_STAGE
    *J_out = J;
    for (int k = 0; k < 3; ++k) grad_out[k] = grad[k];
    if (Cfinal_out) memcpy(Cfinal_out, CN, sizeof(double) * n);
    free(X); free(Cs); free(rhs); free(pred); free(g); free(lam); free(y); free(z); free(Ch); free(xh);
}

/* Forward run (Euler or predictor-corrector) followed by the misfit J only
 * (for finite differences). */
double or_misfit(const or_model *m, int64_t n, const double *x0, const double *C0,
                 const double *vu, const double *mass, const double *rho, double dt,
                 int64_t nsteps, int64_t ns, const double *xs, const double *obs, int integrator,
                 double *pred_out)
{
    int dim = m->dim;
    double *x = (double *)malloc(sizeof(double) * dim * n);
    double *C = (double *)malloc(sizeof(double) * n);
    memcpy(x, x0, sizeof(double) * dim * n);
    memcpy(C, C0, sizeof(double) * n);
    or_run(m, n, x, C, NULL, vu, mass, rho, dt, nsteps, integrator, NULL);
    double *pred = (double *)malloc(sizeof(double) * (ns > 0 ? ns : 1));
    or_sensor_interp(m, n, x, C, ns, xs, pred, NULL);
    double J = 0.0;
    for (int64_t s = 0; s < ns; ++s) {
        double r = pred[s] - (obs ? obs[s] : 0.0);
        J += r * r;
    }
    if (pred_out) memcpy(pred_out, pred, sizeof(double) * ns);
    free(x); free(C); free(pred);
    return J;
}

/* ------------------------------------------------------------------------- */
/* Velocity field (per-particle v, explicit Euler)                            */
/* ------------------------------------------------------------------------- */
/* L_k C: the derivative of rhs = L C with respect to theta_k (k = 0, 1, 2 for */
/* alpha_L, alpha_T, D_m) with per-particle tensors; the convective part of   */
/* Eq. (4) does not depend on theta.                                           */
void or_rhs_deriv(const or_model *m, int64_t n, const double *x, const double *C, const double *v,
                  const double *mass, const double *rho, int k, double *out)
{
    or_cells cl;
    cells_build(m, n, x, &cl);
    double *D = tensors_per_particle(m, n, v, NULL);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < n; ++a) {
        rhs_ctx c = {m, n, a, x, C, v, mass, rho, D, NULL, 0.0, 0.0, k + 1};
        double xa[3];
        for (int i = 0; i < m->dim; ++i) xa[i] = x[i * n + a];
        for_neighbours(m, n, x, &cl, xa, a, rhs_visit, &c);
        out[a] = c.disp;
    }
    free(D);
    cells_free(&cl);
}

typedef struct {
    const or_model *m;
    int64_t n, b;
    const double *v, *mass, *rho, *D, *lam;
    double y, conv;
} ltf_ctx;

/* Row b of L^T for per-particle tensors: with L_bb = sum_j w_bj + c_b (c_b the
 * convective factor of Eq. 4, multiplying C_b) and L_ab = -w_ab,
 * (L^T lam)_b = (sum_a w_ba + c_b) lam_b - sum_{a != b} w_ab lam_a. */
static void ltf_visit(int64_t a, const double *xba, double r2, void *vctx)
{
    ltf_ctx *c = (ltf_ctx *)vctx;
    const or_model *m = c->m;
    int dim = m->dim;
    int64_t b = c->b, n = c->n;
    double xab[3], h[9];
    for (int k = 0; k < dim; ++k) xab[k] = -xba[k];
    or_harmonic(dim, c->D + b * dim * dim, c->D + a * dim * dim, h);
    double w_ba = pair_weight(m, c->mass, c->rho, h, b, a, xba, r2);
    double w_ab = pair_weight(m, c->mass, c->rho, h, a, b, xab, r2);
    c->y += w_ba * c->lam[b] - w_ab * c->lam[a];
    double r = sqrt(r2);
    double dWdr = or_kernel_dWdr(m->kernel, dim, m->H, r);
    double s = 0.0;
    for (int i = 0; i < dim; ++i) s += (c->v[i * n + b] - c->v[i * n + a]) * dWdr * xba[i] / r;
    c->conv += c->mass[a] / (0.5 * (c->rho[a] + c->rho[b])) * s;
}

void or_apply_LT_field(const or_model *m, int64_t n, const double *x, const double *v,
                       const double *mass, const double *rho, const double *lam, double *y)
{
    or_cells cl;
    cells_build(m, n, x, &cl);
    double *D = tensors_per_particle(m, n, v, NULL);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < n; ++b) {
        ltf_ctx c = {m, n, b, v, mass, rho, D, lam, 0.0, 0.0};
        double xb[3];
        for (int i = 0; i < m->dim; ++i) xb[i] = x[i * n + b];
        for_neighbours(m, n, x, &cl, xb, b, ltf_visit, &c);
        y[b] = c.y + c.conv * lam[b];
    }
    free(D);
    cells_free(&cl);
}

/* Discrete adjoint of the run with per-particle velocities, J = sum_s
 * (P C^N - d)_s^2, lam^N = P^T 2 (P C^N - d).
 * Euler (integrator 1): C^{n+1} = C^n + dt L^n C^n, x^{n+1} = x^n + dt v;
 *   lam^n = lam^{n+1} + dt (L^n)^T lam^{n+1},  dJ/dtheta_k += dt lam^{n+1} . L^n_k C^n.
 * Predictor-corrector (integrator 2, R6 with each particle's velocity):
 * C^h = C^n + dt/2 L1 C^n with L1 = L(x^n), C^{n+1} = C^n + dt L2 C^h with
 * L2 = L(x^n + dt/2 v); with y = L2^T lam^{n+1}:
 *   lam^n = lam^{n+1} + dt y + dt^2/2 L1^T y,
 *   dJ/dtheta_k += dt lam^{n+1} . L2_k C^h + dt^2/2 y . L1_k C^n.
 * All states are kept in memory (plain reverse sweep). */
void or_adjoint_field(const or_model *m, int64_t n, const double *x0, const double *C0,
                      const double *v, const double *mass, const double *rho, double dt,
                      int64_t nsteps, int64_t ns, const double *xs, const double *obs, int integrator,
                      double *J_out, double *grad_out, double *Cfinal_out)
{
    int dim = m->dim;
    double *X = (double *)malloc(sizeof(double) * dim * n * (nsteps + 1));
    double *Cs = (double *)malloc(sizeof(double) * n * (nsteps + 1));
    double *rhs = (double *)malloc(sizeof(double) * n);
    double *Ch = (double *)malloc(sizeof(double) * n);
    double *xh = (double *)malloc(sizeof(double) * n * dim);
    memcpy(X, x0, sizeof(double) * dim * n);
    memcpy(Cs, C0, sizeof(double) * n);
    /* C^h and x^h of step s: the predictor stage */
    #define FIELD_HALF(xs_n, C_n)                                                   \
        do {                                                                        \
            or_rhs(m, n, xs_n, C_n, v, NULL, mass, rho, NULL, n, NULL, rhs);        \
            for (int64_t a = 0; a < n; ++a) Ch[a] = (C_n)[a] + 0.5 * dt * rhs[a];   \
            advect(m, n, xs_n, v, NULL, 0.5 * dt, xh);                              \
        } while (0)
    for (int64_t s = 0; s < nsteps; ++s) {
        const double *xs_n = X + (size_t)s * dim * n;
        const double *C_n = Cs + (size_t)s * n;
        if (integrator == 2) {
            FIELD_HALF(xs_n, C_n);
            or_rhs(m, n, xh, Ch, v, NULL, mass, rho, NULL, n, NULL, rhs);
        } else {
            or_rhs(m, n, xs_n, C_n, v, NULL, mass, rho, NULL, n, NULL, rhs);
        }
        for (int64_t a = 0; a < n; ++a) Cs[(size_t)(s + 1) * n + a] = C_n[a] + dt * rhs[a];
        advect(m, n, xs_n, v, NULL, dt, X + (size_t)(s + 1) * dim * n);
    }
    const double *xN = X + (size_t)nsteps * dim * n, *CN = Cs + (size_t)nsteps * n;
    double *pred = (double *)malloc(sizeof(double) * (ns > 0 ? ns : 1));
    double *g = (double *)malloc(sizeof(double) * (ns > 0 ? ns : 1));
    or_sensor_interp(m, n, xN, CN, ns, xs, pred, NULL);
    double J = 0.0;
    for (int64_t s = 0; s < ns; ++s) {
        double r = pred[s] - obs[s];
        J += r * r;
        g[s] = 2.0 * r;
    }
    double *lam = (double *)malloc(sizeof(double) * n);
    double *y = (double *)malloc(sizeof(double) * n);
    sensor_interp_T(m, n, xN, ns, xs, g, lam);
    double grad[3] = {0.0, 0.0, 0.0};
    double *z = (double *)malloc(sizeof(double) * n);
    for (int64_t s = nsteps - 1; s >= 0; --s) {
        const double *xs_n = X + (size_t)s * dim * n;
        const double *C_n = Cs + (size_t)s * n;
        if (integrator == 2) {
            FIELD_HALF(xs_n, C_n);
            or_apply_LT_field(m, n, xh, v, mass, rho, lam, y); /* y = L2^T lam */
            for (int k = 0; k < 3; ++k) {
                double acc = 0.0;
                or_rhs_deriv(m, n, xh, Ch, v, mass, rho, k, rhs);
                for (int64_t a = 0; a < n; ++a) acc += dt * lam[a] * rhs[a];
                or_rhs_deriv(m, n, xs_n, C_n, v, mass, rho, k, rhs);
                for (int64_t a = 0; a < n; ++a) acc += 0.5 * dt * dt * y[a] * rhs[a];
                grad[k] += acc;
            }
            or_apply_LT_field(m, n, xs_n, v, mass, rho, y, z); /* z = L1^T y */
            for (int64_t a = 0; a < n; ++a) lam[a] += dt * y[a] + 0.5 * dt * dt * z[a];
        } else {
            for (int k = 0; k < 3; ++k) {
                or_rhs_deriv(m, n, xs_n, C_n, v, mass, rho, k, rhs);
                double acc = 0.0;
                for (int64_t a = 0; a < n; ++a) acc += lam[a] * rhs[a];
                grad[k] += dt * acc;
            }
            or_apply_LT_field(m, n, xs_n, v, mass, rho, lam, y);
            for (int64_t a = 0; a < n; ++a) lam[a] += dt * y[a];
        }
    }
    #undef FIELD_HALF
    *J_out = J;
    for (int k = 0; k < 3; ++k) grad_out[k] = grad[k];
    if (Cfinal_out) memcpy(Cfinal_out, CN, sizeof(double) * n);
    free(X); free(Cs); free(rhs); free(pred); free(g); free(lam); free(y); free(z); free(Ch); free(xh);
}

/* Forward run with per-particle velocities (Euler 1, predictor-corrector 2)
 * and J only. */
double or_misfit_field(const or_model *m, int64_t n, const double *x0, const double *C0,
                       const double *v, const double *mass, const double *rho, double dt,
                       int64_t nsteps, int64_t ns, const double *xs, const double *obs, int integrator)
{
    int dim = m->dim;
    double *x = (double *)malloc(sizeof(double) * dim * n);
    double *C = (double *)malloc(sizeof(double) * n);
    memcpy(x, x0, sizeof(double) * dim * n);
    memcpy(C, C0, sizeof(double) * n);
    or_run(m, n, x, C, v, NULL, mass, rho, dt, nsteps, integrator, NULL);
    double *pred = (double *)malloc(sizeof(double) * (ns > 0 ? ns : 1));
    or_sensor_interp(m, n, x, C, ns, xs, pred, NULL);
    double J = 0.0;
    for (int64_t s = 0; s < ns; ++s) {
        double r = pred[s] - obs[s];
        J += r * r;
    }
    free(x); free(C); free(pred);
    return J;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
