/*
 * CPU oracle for the immersed-boundary interaction operators (spreading S(X)F and
 * interpolation J(X)u) of Kassen, Shankar & Fogelson, "A fine-grained parallelization
 * of the immersed boundary method" (arXiv 2012.06646).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls this
 * file; only the test suite, the smoke check and the benchmark's CPU-baseline leg do.
 * It shares no code, header, table or constant with the HIP path.
 *
 * Everything here is written straight from the definitions, in double precision with
 * long-double accumulators, without blocking, fusion or reordering:
 *
 *   - grid points of one velocity component: x = h (i + xi), i in Z^d taken modulo N
 *     (Sec. 3.1, "Preliminaries");
 *   - regularized delta: delta_h(x) = prod_k h_k^-1 phi(x_k / h_k) (Sec. 2, the
 *     paragraph introducing the regularized kernel);
 *   - discrete interpolation and spreading, eqs. (disc-interp) and (disc-spread) of
 *     Sec. 2: U_j = sum_i delta_h(x_i - X_j) u_i h^d and f_i = sum_j delta_h(x_i - X_j) F_j,
 *     where F_j already carries the Lagrangian weight dtheta_j;
 *   - sort keys and the stable key/index sort of Alg. 4 (Sec. 3.4), keys numbered
 *     x-fastest as in Fig. 2, counted from 0;
 *   - the position update X + dt U of the IB time step (Sec. 2), rounded once and wrapped
 *     into the periodic box;
 *   - non-periodic ("walled") dimensions (Sec. 3.1, the grid indexing function #): a grid
 *     index outside 0..n_k-1 of such a dimension is no grid point, so it takes no part in
 *     spreading or interpolation, and distances along it are not folded to a periodic
 *     image.  walls is a bit mask over dimensions (bit k set: dimension k is walled).
 *
 * phi is evaluated from its piecewise closed form (Peskin 2002, the kernel reference of
 * Sec. 2): the 4-point kernel, or the cosine kernel the paper itself uses, or the 3-point
 * kernel of Roma, Peskin & Berger (J. Comput. Phys. 153, 1999), the odd-support (s = 3)
 * case of Fig. 1(b).
 *
 * Two independent evaluation orders are provided for the operators:
 *   tier A ("all pairs")  loops every (point, grid point) pair with the nearest periodic image;
 *   tier B ("candidate stencil") loops 6 candidate indices per dimension around the point
 *   (a deliberate superset of the 4-point support), so it does not depend on any cell or
 *   shift convention.  Spreading visits points in input order, as the serial Alg. 2 does.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (see oracle/build.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PESKIN4 0
#define OR_COSINE4 1
#define OR_ROMA3 2

/* ---- the one-dimensional kernel phi and its derivative ------------------------- */

/* Peskin's 4-point kernel, piecewise closed form, evaluated at |r|. */
static double phi_peskin4(double r)
{
    double a = fabs(r);
    if (a <= 1.0)
        return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
    if (a <= 2.0)
        return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
    return 0.0;
}

/* d phi / d r for the 4-point kernel; odd in r. */
static double dphi_peskin4(double r)
{
    double a = fabs(r), g;
    if (a <= 1.0)
        g = (-1.0 + (1.0 - 2.0 * a) / sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 4.0;
    else if (a < 2.0)
        g = (-1.0 - (3.0 - 2.0 * a) / sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 4.0;
    else
        g = 0.0;
    return r < 0.0 ? -g : g;
}

/* The cosine kernel of Peskin 2002: phi(r) = (1 + cos(pi r / 2)) / 4 on |r| <= 2. */
static double phi_cosine4(double r)
{
    double a = fabs(r);
    if (a <= 2.0)
        return 0.25 * (1.0 + cos(M_PI * a / 2.0));
    return 0.0;
}

static double dphi_cosine4(double r)
{
    if (fabs(r) <= 2.0)
        return -(M_PI / 8.0) * sin(M_PI * r / 2.0);
    return 0.0;
}

/* The 3-point kernel of Roma, Peskin & Berger 1999, piecewise closed form at |r|:
 * (1 + sqrt(1 - 3 r^2)) / 3 on |r| <= 1/2, (5 - 3|r| - sqrt(1 - 3 (1 - |r|)^2)) / 6 on
 * 1/2 <= |r| <= 3/2, zero beyond. */
static double phi_roma3(double r)
{
    double a = fabs(r);
    if (a <= 0.5)
        return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
    if (a <= 1.5)
        return (5.0 - 3.0 * a - sqrt(1.0 - 3.0 * (1.0 - a) * (1.0 - a))) / 6.0;
    return 0.0;
}

static double dphi_roma3(double r)
{
    double a = fabs(r), g;
    if (a <= 0.5)
        g = -a / sqrt(1.0 - 3.0 * a * a);
    else if (a < 1.5)
        g = -0.5 - (1.0 - a) / (2.0 * sqrt(1.0 - 3.0 * (1.0 - a) * (1.0 - a)));
    else
        g = 0.0;
    return r < 0.0 ? -g : g;
}

double or_phi(int kernel, double r)
{
    if (kernel == OR_ROMA3) return phi_roma3(r);
    return kernel == OR_COSINE4 ? phi_cosine4(r) : phi_peskin4(r);
}

double or_dphi(int kernel, double r)
{
    if (kernel == OR_ROMA3) return dphi_roma3(r);
    return kernel == OR_COSINE4 ? dphi_cosine4(r) : dphi_peskin4(r);
}

/* ---- cell keys (Alg. 4 key step; Fig. 2 numbering, 0-based) ------------------------
 * For one grid staggering xi: t_k = X_k * (N_k / L_k), rounded once in the job precision
 * (prec 0 = double, 1 = float, never fused), y_k = t_k - xi_k.  The cell (Sec. 3.1, Fig. 1)
 * is the region of points sharing one set of support points, named by its grid point: for
 * an even support size (odd == 0) the cell whose lower corner is the node floor(y_k); for
 * an odd support size (odd == 1, Fig. 1(b)) the cell centred on the nearest node,
 * floor(y_k + 1/2), a point exactly half-way going to the upper node.  cell_k is taken
 * modulo N_k (Euclidean), key = cell_0 + N_0 * (cell_1 + N_1 * cell_2).
 * Returns the number of points whose scaled coordinate is not finite or too large
 * (|t| >= 2^30); their key is set to -1. */
long or_keys(int dim, const int *n, const double *length, const double *xi, int prec, int odd,
             long np, const double *X, int32_t *keys)
{
    long bad = 0;
    for (long j = 0; j < np; ++j) {
        long long key = 0, stride = 1;
        int ok = 1;
        for (int k = 0; k < dim; ++k) {
            double y;
            if (prec == 1) {
                volatile float inv_h = (float)n[k] / (float)length[k];
                volatile float t = (float)X[j * dim + k] * inv_h;
                volatile float yf = t - (float)xi[k];
                y = (double)yf;
            } else {
                volatile double inv_h = (double)n[k] / length[k];
                volatile double t = X[j * dim + k] * inv_h;
                y = t - xi[k];
            }
            if (!isfinite(y) || fabs(y) >= 1073741824.0) { ok = 0; break; }
            long long c = (long long)floor(y);
            /* y - floor(y) is exact; the nearest node is the upper one from 1/2 on */
            if (odd && y - floor(y) >= 0.5) c += 1;
            c %= n[k];
            if (c < 0) c += n[k];
            key += c * stride;
            stride *= n[k];
        }
        if (ok) keys[j] = (int32_t)key;
        else { keys[j] = -1; ++bad; }
    }
    return bad;
}

/* ---- stable key/index sort, unique count and segment offsets (Alg. 4, Fig. 2) ------- */

static const int32_t *cmp_keys;

static int cmp_key_then_index(const void *a, const void *b)
{
    int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
    if (cmp_keys[i] != cmp_keys[j]) return cmp_keys[i] < cmp_keys[j] ? -1 : 1;
    return i < j ? -1 : (i > j ? 1 : 0);
}

/* perm = indices ordered by (key, index): the unique stable ascending order.
 * sorted_keys[i] = keys[perm[i]]; seg_off[0..q] = first sorted position of each run of
 * equal keys, with seg_off[q] = np; returns q, the number of distinct keys. */
long or_plan(long np, const int32_t *keys, int32_t *sorted_keys, int32_t *perm,
             int32_t *seg_off)
{
    for (long i = 0; i < np; ++i) perm[i] = (int32_t)i;
    cmp_keys = keys;
    qsort(perm, (size_t)np, sizeof(int32_t), cmp_key_then_index);
    long q = 0;
    for (long i = 0; i < np; ++i) {
        sorted_keys[i] = keys[perm[i]];
        if (i == 0 || sorted_keys[i] != sorted_keys[i - 1]) seg_off[q++] = (int32_t)i;
    }
    seg_off[q] = (int32_t)np;
    return q;
}

/* ---- operators ------------------------------------------------------------------- */

typedef struct {
    int dim, ncomp, kernel, walls;
    int n[3];
    double length[3];
    double xi[3][3];
} grid_t;

static grid_t make_grid(int dim, const int *n, const double *length, int ncomp,
                        const double *stagger, int kernel, int walls)
{
    grid_t g;
    memset(&g, 0, sizeof g);
    g.dim = dim; g.ncomp = ncomp; g.kernel = kernel; g.walls = walls;
    for (int k = 0; k < 3; ++k) { g.n[k] = 1; g.length[k] = 1.0; }
    for (int k = 0; k < dim; ++k) { g.n[k] = n[k]; g.length[k] = length[k]; }
    for (int c = 0; c < ncomp; ++c)
        for (int k = 0; k < dim; ++k) g.xi[c][k] = stagger[c * 3 + k];
    return g;
}

static long grid_size(const grid_t *g)
{
    long G = 1;
    for (int k = 0; k < g->dim; ++k) G *= g->n[k];
    return G;
}

/* X_k / h_k in long double. */
static long double scaled(const grid_t *g, int k, double Xk)
{
    return (long double)Xk * (long double)g->n[k] / (long double)g->length[k];
}

static int walled(const grid_t *g, int k) { return (g->walls >> k) & 1; }

/* Tier A weight: rho_k = (i_k + xi_k) - X_k / h_k, folded to the nearest periodic image
 * along periodic dimensions. */
static double weight_allpairs(const grid_t *g, int c, const long *idx, const double *Xj)
{
    double w = 1.0;
    for (int k = 0; k < g->dim; ++k) {
        long double rho = ((long double)idx[k] + g->xi[c][k]) - scaled(g, k, Xj[k]);
        long double N = g->n[k];
        if (!walled(g, k)) rho -= N * roundl(rho / N);
        if (fabsl(rho) >= 2.0L) return 0.0;
        w *= or_phi(g->kernel, (double)rho);
    }
    return w;
}

static void unflatten(const grid_t *g, long m, long *idx)
{
    for (int k = 0; k < 3; ++k) idx[k] = 0;
    for (int k = 0; k < g->dim; ++k) { idx[k] = m % g->n[k]; m /= g->n[k]; }
}

static long flatten(const grid_t *g, const long *idx)
{
    long m = 0, stride = 1;
    for (int k = 0; k < g->dim; ++k) { m += idx[k] * stride; stride *= g->n[k]; }
    return m;
}

/* Tier B: enumerate the 6^d candidate indices i_k = floor(X_k/h_k - xi_k) + {-2..3}
 * around point Xj, calling back with the (wrapped) flat grid index and the weight; along a
 * walled dimension an index outside 0..n_k-1 is skipped. */
typedef void (*visit_fn)(void *ctx, long m, double w);

static void visit_stencil(const grid_t *g, int c, const double *Xj, visit_fn fn, void *ctx)
{
    long base[3] = {0, 0, 0};
    long double s[3] = {0, 0, 0};
    for (int k = 0; k < g->dim; ++k) {
        s[k] = scaled(g, k, Xj[k]);
        base[k] = (long)floorl(s[k] - g->xi[c][k]);
    }
    int reach[3] = {1, 1, 1};
    for (int k = 0; k < g->dim; ++k) reach[k] = 6;
    for (int a2 = 0; a2 < reach[2]; ++a2)
        for (int a1 = 0; a1 < reach[1]; ++a1)
            for (int a0 = 0; a0 < reach[0]; ++a0) {
                int a[3] = {a0, a1, a2};
                double w = 1.0;
                long idx[3] = {0, 0, 0};
                for (int k = 0; k < g->dim && w != 0.0; ++k) {
                    long i = base[k] - 2 + a[k];
                    long double rho = ((long double)i + g->xi[c][k]) - s[k];
                    if (fabsl(rho) >= 2.0L) { w = 0.0; break; }
                    if (walled(g, k) && (i < 0 || i >= g->n[k])) { w = 0.0; break; }
                    w *= or_phi(g->kernel, (double)rho);
                    long im = i % g->n[k];
                    if (im < 0) im += g->n[k];
                    idx[k] = im;
                }
                if (w != 0.0) fn(ctx, flatten(g, idx), w);
            }
}

typedef struct { long double *acc; long double val; } spread_ctx;
static void spread_visit(void *vctx, long m, double w)
{
    spread_ctx *ctx = (spread_ctx *)vctx;
    ctx->acc[m] += (long double)w * ctx->val;
}

typedef struct { const double *u; long double sum; } interp_ctx;
static void interp_visit(void *vctx, long m, double w)
{
    interp_ctx *ctx = (interp_ctx *)vctx;
    ctx->sum += (long double)w * ctx->u[m];
}

/* Spreading, eq. (disc-spread): f_{c,i} = (prod_k h_k)^-1 sum_j W_{c,i,j} F_{j,c}.
 * X: np x dim row-major; F: np x ncomp row-major; f: ncomp x G (x fastest), overwritten.
 * tier 0 = all pairs, 1 = candidate stencil.  Returns 0, or -1 on allocation failure. */
int or_spread(int dim, const int *n, const double *length, int ncomp, const double *stagger,
              int kernel, int walls, int tier, long np, const double *X, const double *F,
              double *f)
{
    grid_t g = make_grid(dim, n, length, ncomp, stagger, kernel, walls);
    long G = grid_size(&g);
    long double hd = 1.0L;
    for (int k = 0; k < dim; ++k) hd *= (long double)length[k] / (long double)n[k];
    long double *acc = (long double *)calloc((size_t)G, sizeof(long double));
    if (!acc) return -1;
    for (int c = 0; c < ncomp; ++c) {
        memset(acc, 0, (size_t)G * sizeof(long double));
        for (long j = 0; j < np; ++j) {
            const double *Xj = X + j * dim;
            long double Fj = F[j * ncomp + c];
            if (tier == 0) {
                long idx[3];
                for (long m = 0; m < G; ++m) {
                    unflatten(&g, m, idx);
                    double w = weight_allpairs(&g, c, idx, Xj);
                    if (w != 0.0) acc[m] += (long double)w * Fj;
                }
            } else {
                spread_ctx ctx = {acc, Fj};
                visit_stencil(&g, c, Xj, spread_visit, &ctx);
            }
        }
        for (long m = 0; m < G; ++m) f[(long)c * G + m] = (double)(acc[m] / hd);
    }
    free(acc);
    return 0;
}

/* Interpolation, eq. (disc-interp) with delta_h h^d = prod phi:
 * U_{j,c} = sum_i W_{c,i,j} u_{c,i}.  u: ncomp x G; U: np x ncomp, overwritten. */
int or_interp(int dim, const int *n, const double *length, int ncomp, const double *stagger,
              int kernel, int walls, int tier, long np, const double *X, const double *u,
              double *U)
{
    grid_t g = make_grid(dim, n, length, ncomp, stagger, kernel, walls);
    long G = grid_size(&g);
    for (long j = 0; j < np; ++j) {
        const double *Xj = X + j * dim;
        for (int c = 0; c < ncomp; ++c) {
            const double *uc = u + (long)c * G;
            long double sum = 0.0L;
            if (tier == 0) {
                long idx[3];
                for (long m = 0; m < G; ++m) {
                    unflatten(&g, m, idx);
                    double w = weight_allpairs(&g, c, idx, Xj);
                    if (w != 0.0) sum += (long double)w * uc[m];
                }
            } else {
                interp_ctx ctx = {uc, 0.0L};
                visit_stencil(&g, c, Xj, interp_visit, &ctx);
                sum = ctx.sum;
            }
            U[j * ncomp + c] = (double)sum;
        }
    }
    return 0;
}

/* Spreading evaluated only at the listed targets: out[t] = f_{comp[t], idx[t]}, each by a
 * plain loop over all points (used to check large problems at sampled grid points). */
int or_spread_at(int dim, const int *n, const double *length, int ncomp,
                 const double *stagger, int kernel, int walls, long np, const double *X,
                 const double *F, long nt, const int32_t *comp, const int64_t *target,
                 double *out)
{
    grid_t g = make_grid(dim, n, length, ncomp, stagger, kernel, walls);
    long double hd = 1.0L;
    for (int k = 0; k < dim; ++k) hd *= (long double)length[k] / (long double)n[k];
    for (long t = 0; t < nt; ++t) {
        int c = comp[t];
        long idx[3];
        unflatten(&g, (long)target[t], idx);
        long double sum = 0.0L;
        for (long j = 0; j < np; ++j) {
            double w = weight_allpairs(&g, c, idx, X + j * dim);
            if (w != 0.0) sum += (long double)w * F[j * ncomp + c];
        }
        out[t] = (double)(sum / hd);
    }
    return 0;
}

/* Position gradient of interpolation, contracted with W (np x ncomp):
 * dX_{j,k} = sum_c W_{j,c} dU_{j,c}/dX_{j,k}, with
 * dW/dX_k = -(1/h_k) phi'(rho_k) prod_{l != k} phi(rho_l), rho = (x - X)/h.
 * The same routine gives the position gradient of <S(X)F, g>_h with u = g and W = F.
 * dX: np x dim, overwritten.  Candidate-stencil order. */
int or_interp_grad(int dim, const int *n, const double *length, int ncomp,
                   const double *stagger, int kernel, int walls, long np, const double *X,
                   const double *u, const double *W, double *dX)
{
    grid_t g = make_grid(dim, n, length, ncomp, stagger, kernel, walls);
    long G = grid_size(&g);
    for (long j = 0; j < np; ++j) {
        const double *Xj = X + j * dim;
        long double grad[3] = {0, 0, 0};
        for (int c = 0; c < ncomp; ++c) {
            const double *uc = u + (long)c * G;
            long double s[3] = {0, 0, 0};
            long base[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) {
                s[k] = scaled(&g, k, Xj[k]);
                base[k] = (long)floorl(s[k] - g.xi[c][k]);
            }
            int reach[3] = {1, 1, 1};
            for (int k = 0; k < dim; ++k) reach[k] = 6;
            for (int a2 = 0; a2 < reach[2]; ++a2)
                for (int a1 = 0; a1 < reach[1]; ++a1)
                    for (int a0 = 0; a0 < reach[0]; ++a0) {
                        int a[3] = {a0, a1, a2};
                        double ph[3] = {1, 1, 1}, dph[3] = {0, 0, 0};
                        long idx[3] = {0, 0, 0};
                        int inside = 1;
                        for (int k = 0; k < dim; ++k) {
                            long i = base[k] - 2 + a[k];
                            long double rho = ((long double)i + g.xi[c][k]) - s[k];
                            if (fabsl(rho) >= 2.0L) { inside = 0; break; }
                            if (walled(&g, k) && (i < 0 || i >= g.n[k])) { inside = 0; break; }
                            ph[k] = or_phi(kernel, (double)rho);
                            dph[k] = or_dphi(kernel, (double)rho);
                            long im = i % g.n[k];
                            if (im < 0) im += g.n[k];
                            idx[k] = im;
                        }
                        if (!inside) continue;
                        long double um = uc[flatten(&g, idx)] * (long double)W[j * ncomp + c];
                        for (int k = 0; k < dim; ++k) {
                            long double d = -(long double)dph[k] * (long double)n[k] / length[k];
                            for (int l = 0; l < dim; ++l)
                                if (l != k) d *= ph[l];
                            grad[k] += d * um;
                        }
                    }
        }
        for (int k = 0; k < dim; ++k) dX[j * dim + k] = (double)grad[k];
    }
    return 0;
}

/* ---- position update ------------------------------------------------------------ */

/* Position update of the IB time step (Sec. 2, steps (b) and (g)): y = X + dt U per
 * coordinate, the exact value rounded once (C99 fma), then wrapped into [0, L_k) along
 * periodic dimensions: y - L_k floor(y / L_k); a result that rounds to L_k or falls below
 * 0 is set to 0.  Along walled dimensions y is left as it is.  out: np x dim (may alias X). */
void or_advect(int dim, const double *length, int walls, long np, const double *X,
               const double *U, double dt, double *out)
{
    for (long j = 0; j < np; ++j)
        for (int k = 0; k < dim; ++k) {
            const double L = length[k];
            double y = fma(dt, U[j * dim + k], X[j * dim + k]);
            if ((walls >> k) & 1) {
                out[j * dim + k] = y;
                continue;
            }
            y = y - L * floor(y / L);
            if (y >= L || y < 0.0) y = 0.0;
            out[j * dim + k] = y;
        }
}
