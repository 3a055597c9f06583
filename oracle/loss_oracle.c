/*
 * loss_oracle.c -- plain FP64 CPU oracle of the local spline simulator (LOSS),
 * arXiv 2301.05127.  TEST INFRASTRUCTURE ONLY (see loss_oracle.h).
 *
 * Parity unpinned: none of the routines below lacks a pin; the pins live in
 * tests/test_oracle_pins.py (dense brute force, closed forms, invariants,
 * analytic plane-wave dispersion, finite differences of the adjoint) and
 * tests/test_oracle_pml*.py (the layer: ODE integration, no-damping limit,
 * absorption, wider domains, elastic plane waves against the acoustic layer).
 *
 * Method, in the paper's order (Sec. 3):
 *   1. cubic B-spline coefficients v~_{-1..N+1} of a line from the collocation rows
 *      (v~_{i-1} + 4 v~_i + v~_{i+1})/6 = v_i and two end rows  (Sec. 3.1);
 *   2. the line is cut into patches of M intervals sharing their junction nodes;
 *      each patch solves its own bordered system with Hermite end rows
 *      (v~_1 - v~_{-1})/(2h) = phi  (eq. spline_cofficient_eq_piece);
 *   3. the junction slope phi is the truncated row of the global inverse b = A^{-1}
 *      (eq. truncated_solution, truncation, PMBC, PMBC_coeffcients);
 *   4. the derivative is the centred difference of the coefficients
 *      (eq. derivative_approximation); the second derivative is the second
 *      difference of the coefficients divided by h^2 (second derivative of B_i);
 *   5. time: Strang splitting, half step of the velocity sub-flow, full step of the
 *      stress sub-flow, half step of the velocity sub-flow (Sec. 3.3);
 *   6. optional absorbing layer: the ADE-PML memory variables, each sub-flow solved
 *      exactly with the driving derivative frozen (Sec. 3.3); written out in the paper
 *      for the 2-D acoustic system, applied here to every derivative of the elastic
 *      system as well.
 */
#include "loss_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Bordered spline system.                                                   */
/* Unknowns x_{-1..K+1} stored as xs[0..K+2].  Rows:                         */
/*   L[0] x_{-1} + L[1] x_0 + L[2] x_1 = rl                                  */
/*   (x_{i-1} + 4 x_i + x_{i+1}) / 6   = r_i        i = 0..K                 */
/*   R[0] x_{K-1} + R[1] x_K + R[2] x_{K+1} = rr                             */
/* Solved by substituting the two ghost unknowns from the border rows into   */
/* rows 0 and K, Gaussian elimination of the remaining (K+1) tridiagonal     */
/* system (diagonally dominant: no pivoting), and back-substitution.         */
/* ------------------------------------------------------------------------ */
static void bordered_solve(int K, const double L[3], double rl, const double *r,
                           const double R[3], double rr, double *xs)
{
    int n = K + 1, i;
    double *a = (double *)malloc(sizeof(double) * 4 * n);
    double *b = a + n, *c = b + n, *d = c + n;
    for (i = 0; i < n; ++i) { a[i] = 1.0; b[i] = 4.0; c[i] = 1.0; d[i] = 6.0 * r[i]; }
    a[0] = 0.0;
    c[n - 1] = 0.0;
    /* row 0 with x_{-1} = (rl - L1 x_0 - L2 x_1) / L0 */
    b[0] -= L[1] / L[0];
    c[0] = (n > 1 ? 1.0 : 0.0) - L[2] / L[0];
    d[0] -= rl / L[0];
    /* row K with x_{K+1} = (rr - R0 x_{K-1} - R1 x_K) / R2 */
    if (n > 1) a[n - 1] = 1.0 - R[0] / R[2];
    b[n - 1] -= R[1] / R[2];
    d[n - 1] -= rr / R[2];
    /* forward elimination */
    for (i = 1; i < n; ++i) {
        double m = a[i] / b[i - 1];
        b[i] -= m * c[i - 1];
        d[i] -= m * d[i - 1];
    }
    /* back substitution into xs[1..K+1] = x_0..x_K */
    xs[n] = d[n - 1] / b[n - 1];
    for (i = n - 2; i >= 0; --i) xs[i + 1] = (d[i] - c[i] * xs[i + 2]) / b[i];
    /* ghosts */
    xs[0] = (rl - L[1] * xs[1] - L[2] * xs[2]) / L[0];
    xs[K + 2] = (rr - R[0] * xs[K] - R[1] * xs[K + 1]) / R[2];
    free(a);
}

static void natural_row(double h, double row[3])
{
    row[0] = 1.0 / (h * h); row[1] = -2.0 / (h * h); row[2] = 1.0 / (h * h);
}

static void hermite_row(double h, double row[3])
{
    row[0] = -1.0 / (2.0 * h); row[1] = 0.0; row[2] = 1.0 / (2.0 * h);
}

void or_global_spline(int N, double h, const double *v, double *vt)
{
    double L[3], R[3];
    natural_row(h, L);
    natural_row(h, R);
    bordered_solve(N, L, 0.0, v, R, 0.0, vt);
}

void or_global_inverse_column(int N, double h, int k, double *out)
{
    double *e = (double *)calloc((size_t)N + 1, sizeof(double));
    e[k] = 1.0;
    or_global_spline(N, h, e, out);
    free(e);
}

void or_patch_lu(int M, double *d, double *l)
{
    int i;
    d[1] = 4.0;
    l[1] = 0.25;
    d[2] = 4.0 - 2.0 * l[1];
    for (i = 2; i <= M; ++i) {
        l[i] = 1.0 / d[i];
        d[i + 1] = 4.0 - l[i];
    }
    l[M + 1] = 1.0 / (d[M] * d[M + 1]);
    d[M + 2] = 1.0 - l[M + 1];
}

/* ------------------------------------------------------------------------ */
/* Periodic line: circulant collocation system on N distinct nodes           */
/* (node N is node 0).  First column g of its inverse, by dense Gaussian      */
/* elimination with partial pivoting (obviously correct, O(N^3), small N).    */
/* ------------------------------------------------------------------------ */
static int periodic_inverse_column0(int N, double *g)
{
    double *A = (double *)calloc((size_t)N * N, sizeof(double));
    int i, j, k;
    if (!A) return -1;
    for (i = 0; i < N; ++i) {
        A[(size_t)i * N + i] += 4.0 / 6.0;
        A[(size_t)i * N + (i + 1) % N] += 1.0 / 6.0;
        A[(size_t)i * N + (i + N - 1) % N] += 1.0 / 6.0;
        g[i] = (i == 0) ? 1.0 : 0.0;
    }
    for (k = 0; k < N; ++k) {
        int p = k;
        for (i = k + 1; i < N; ++i)
            if (fabs(A[(size_t)i * N + k]) > fabs(A[(size_t)p * N + k])) p = i;
        if (p != k) {
            for (j = 0; j < N; ++j) {
                double t = A[(size_t)k * N + j];
                A[(size_t)k * N + j] = A[(size_t)p * N + j];
                A[(size_t)p * N + j] = t;
            }
            { double t = g[k]; g[k] = g[p]; g[p] = t; }
        }
        for (i = k + 1; i < N; ++i) {
            double m = A[(size_t)i * N + k] / A[(size_t)k * N + k];
            if (m == 0.0) continue;
            for (j = k; j < N; ++j) A[(size_t)i * N + j] -= m * A[(size_t)k * N + j];
            g[i] -= m * g[k];
        }
    }
    for (i = N - 1; i >= 0; --i) {
        double s = g[i];
        for (j = i + 1; j < N; ++j) s -= A[(size_t)i * N + j] * g[j];
        g[i] = s / A[(size_t)i * N + i];
    }
    free(A);
    return 0;
}

static int num_patches(int N, int M) { return (N + M - 1) / M; }

static int node_has_row(int N, int M, int end_mode, int J)
{
    if (J < 0 || J > N) return 0;
    if (J == 0 || J == N) return end_mode != OR_END_NATURAL;
    return (J % M) == 0;
}

int or_pmbc_row(int N, double h, int M, int halo, int end_mode, int J, double *c, int *idx)
{
    int n = halo, t;
    for (t = 0; t <= 2 * n; ++t) { c[t] = 0.0; idx[t] = -1; }
    if (!node_has_row(N, M, end_mode, J)) return 0;
    if (end_mode == OR_END_PERIODIC) {
        /* b_{i,k} = g[(i - k) mod N] for the circulant system */
        double *g = (double *)malloc(sizeof(double) * N);
        periodic_inverse_column0(N, g);
        for (t = 0; t <= 2 * n; ++t) {
            int k = (((J - n + t) % N) + N) % N;
            int ip = (((J + 1 - k) % N) + N) % N, im = (((J - 1 - k) % N) + N) % N;
            c[t] = (g[ip] - g[im]) / (2.0 * h);
            idx[t] = k;
        }
        free(g);
        return 1;
    }
    {
        /* phi_J = sum_k (b_{J+1,k} - b_{J-1,k}) / (2h) v_k over |k - J| <= n, k in [0,N]
         * (eq. PMBC with the coefficients of eq. PMBC_coeffcients; at J = 0 and J = N
         * the same window clipped to the line is the paper's one-sided end stencil). */
        double *col = (double *)malloc(sizeof(double) * ((size_t)N + 3));
        for (t = 0; t <= 2 * n; ++t) {
            int k = J - n + t;
            if (k < 0 || k > N) continue;
            or_global_inverse_column(N, h, k, col);
            /* col[i+1] = b_{i,k} */
            c[t] = (col[J + 2] - col[J]) / (2.0 * h);
            idx[t] = k;
        }
        free(col);
        return 1;
    }
}

/* Per-axis table: the PMBC row of every node that carries one. */
typedef struct {
    int N, M, n, mode;
    double h;
    unsigned char *has;
    double *c;
    int *idx;
} axis_tab;

static void axis_tab_build(axis_tab *T, int N, double h, int M, int halo, int mode)
{
    int J, w = 2 * halo + 1;
    T->N = N; T->M = M; T->n = halo; T->mode = mode; T->h = h;
    T->has = (unsigned char *)calloc((size_t)N + 1, 1);
    T->c = (double *)calloc((size_t)(N + 1) * w, sizeof(double));
    T->idx = (int *)calloc((size_t)(N + 1) * w, sizeof(int));
    for (J = 0; J <= N; ++J)
        T->has[J] = (unsigned char)or_pmbc_row(N, h, M, halo, mode, J, T->c + (size_t)J * w,
                                               T->idx + (size_t)J * w);
}

static void axis_tab_free(axis_tab *T)
{
    free(T->has); free(T->c); free(T->idx);
}

static double axis_phi(const axis_tab *T, int J, const double *u)
{
    int w = 2 * T->n + 1, t;
    double s = 0.0;
    for (t = 0; t < w; ++t) {
        int k = T->idx[(size_t)J * w + t];
        if (k >= 0) s += T->c[(size_t)J * w + t] * u[k];
    }
    return s;
}

/* Derivative of one line with a prebuilt table; xs is scratch of M+3 doubles. */
static void line_deriv_tab(const axis_tab *T, const double *u, double *d1, double *d2, double *xs)
{
    int N = T->N, M = T->M, p = num_patches(N, M), l, i;
    double h = T->h;
    for (l = 0; l < p; ++l) {
        int s = l * M, e = s + M < N ? s + M : N, K = e - s;
        double L[3], R[3], rl = 0.0, rr = 0.0;
        if (s == 0 && T->mode == OR_END_NATURAL) natural_row(h, L);
        else { hermite_row(h, L); rl = axis_phi(T, s, u); }
        if (e == N && T->mode == OR_END_NATURAL) natural_row(h, R);
        else { hermite_row(h, R); rr = axis_phi(T, e, u); }
        bordered_solve(K, L, rl, u + s, R, rr, xs);
        for (i = 0; i <= K; ++i) {
            if (i == K && e != N) break;  /* junction node e is owned by patch l+1 */
            if (d1) d1[s + i] = (xs[i + 2] - xs[i]) / (2.0 * h);
            if (d2) d2[s + i] = (xs[i] - 2.0 * xs[i + 1] + xs[i + 2]) / (h * h);
        }
    }
}

void or_line_deriv(int N, double h, int M, int halo, int end_mode, const double *u, double *d1,
                   double *d2)
{
    axis_tab T;
    double *xs = (double *)malloc(sizeof(double) * ((size_t)M + 3));
    axis_tab_build(&T, N, h, M, halo, end_mode);
    line_deriv_tab(&T, u, d1, d2, xs);
    axis_tab_free(&T);
    free(xs);
}

void or_line_deriv_matrix(int N, double h, int M, int halo, int end_mode, double *D)
{
    axis_tab T;
    int j, i;
    double *e = (double *)calloc((size_t)N + 1, sizeof(double));
    double *col = (double *)malloc(sizeof(double) * ((size_t)N + 1));
    double *xs = (double *)malloc(sizeof(double) * ((size_t)M + 3));
    axis_tab_build(&T, N, h, M, halo, end_mode);
    for (j = 0; j <= N; ++j) {
        e[j] = 1.0;
        line_deriv_tab(&T, e, col, NULL, xs);
        for (i = 0; i <= N; ++i) D[(size_t)i * (N + 1) + j] = col[i];
        e[j] = 0.0;
    }
    axis_tab_free(&T);
    free(e); free(col); free(xs);
}

/* ------------------------------------------------------------------------ */
/* Fields                                                                    */
/* ------------------------------------------------------------------------ */
static void grid_nodes(const or_grid *g, long nn[3])
{
    nn[0] = g->n[0] + 1;
    nn[1] = g->ndim == 3 ? g->n[1] + 1 : 1;
    nn[2] = g->n[2] + 1;
}

static long grid_total(const or_grid *g)
{
    long nn[3];
    grid_nodes(g, nn);
    return nn[0] * nn[1] * nn[2];
}

/* Apply a line operator along `axis` to every line.  op(ctx, in_line, out_line). */
typedef void (*line_op)(const void *ctx, const double *in, double *out, double *scratch);

static void apply_lines(const or_grid *g, int axis, const double *in, double *out, line_op op,
                        const void *ctx, int scratch_len)
{
    long nn[3], stride[3], nlines, L;
    int len;
    grid_nodes(g, nn);
    stride[0] = 1; stride[1] = nn[0]; stride[2] = nn[0] * nn[1];
    len = (int)nn[axis];
    nlines = grid_total(g) / len;
#pragma omp parallel
    {
        double *a = (double *)malloc(sizeof(double) * (size_t)(2 * len + scratch_len));
        double *b = a + len, *s = b + len;
#pragma omp for schedule(static)
        for (L = 0; L < nlines; ++L) {
            /* decompose the line index into the two other coordinates */
            long base, o0, o1;
            int ax0 = axis == 0 ? 1 : 0, ax1 = axis == 2 ? 1 : 2, i;
            o0 = L % nn[ax0];
            o1 = L / nn[ax0];
            base = o0 * stride[ax0] + o1 * stride[ax1];
            for (i = 0; i < len; ++i) a[i] = in[base + i * stride[axis]];
            op(ctx, a, b, s);
            for (i = 0; i < len; ++i) out[base + i * stride[axis]] = b[i];
        }
        free(a);
    }
}

typedef struct { const axis_tab *T; int order; } deriv_ctx;

static void deriv_op(const void *ctx, const double *in, double *out, double *scratch)
{
    const deriv_ctx *c = (const deriv_ctx *)ctx;
    if (c->order == 2) line_deriv_tab(c->T, in, NULL, out, scratch);
    else line_deriv_tab(c->T, in, out, NULL, scratch);
}

typedef struct { const double *D; int n; int transpose; } dense_ctx;

static void dense_op(const void *ctx, const double *in, double *out, double *scratch)
{
    const dense_ctx *c = (const dense_ctx *)ctx;
    int i, j, n = c->n;
    (void)scratch;
    for (i = 0; i < n; ++i) {
        double s = 0.0;
        if (c->transpose)
            for (j = 0; j < n; ++j) s += c->D[(size_t)j * n + i] * in[j];
        else
            for (j = 0; j < n; ++j) s += c->D[(size_t)i * n + j] * in[j];
        out[i] = s;
    }
}

static void tab_for_axis(const or_grid *g, int axis, axis_tab *T)
{
    axis_tab_build(T, g->n[axis], g->h[axis], g->M[axis], g->halo, g->end_mode);
}

void or_field_deriv(const or_grid *g, int axis, int order, const double *in, double *out)
{
    axis_tab T;
    deriv_ctx c;
    tab_for_axis(g, axis, &T);
    c.T = &T; c.order = order;
    apply_lines(g, axis, in, out, deriv_op, &c, g->M[axis] + 3);
    axis_tab_free(&T);
}

/* ------------------------------------------------------------------------ */
/* Sources                                                                   */
/* ------------------------------------------------------------------------ */
void or_source_weights(const or_grid *g, const double pos[3], double spread, double *w)
{
    long nn[3], tot = grid_total(g), i;
    int a, ax[3], lo[3], hi[3], cnode[3], x, y, z, nax = g->ndim == 3 ? 3 : 2;
    double hd = 1.0, sum = 0.0;
    grid_nodes(g, nn);
    ax[0] = 0; ax[1] = g->ndim == 3 ? 1 : 2; ax[2] = 2;
    for (i = 0; i < tot; ++i) w[i] = 0.0;
    for (a = 0; a < 3; ++a) {
        lo[a] = hi[a] = cnode[a] = 0;
    }
    for (a = 0; a < nax; ++a) {
        int d = ax[a];
        hd *= g->h[d];
        cnode[d] = (int)floor(pos[d] / g->h[d] + 0.5);
        if (cnode[d] < 0) cnode[d] = 0;
        if (cnode[d] > g->n[d]) cnode[d] = g->n[d];
        if (spread > 0.0) {
            int r = (int)ceil(4.0 * spread / g->h[d]);
            lo[d] = cnode[d] - r < 0 ? 0 : cnode[d] - r;
            hi[d] = cnode[d] + r > g->n[d] ? g->n[d] : cnode[d] + r;
        } else {
            lo[d] = hi[d] = cnode[d];
        }
    }
    for (z = lo[2]; z <= hi[2]; ++z)
        for (y = lo[1]; y <= hi[1]; ++y)
            for (x = lo[0]; x <= hi[0]; ++x) {
                double q = 1.0;
                if (spread > 0.0) {
                    double dx = x * g->h[0] - pos[0], dz = z * g->h[2] - pos[2], dy = 0.0;
                    if (g->ndim == 3) dy = y * g->h[1] - pos[1];
                    q = exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * spread * spread));
                }
                w[((long)z * nn[1] + y) * nn[0] + x] = q;
                sum += q;
            }
    for (z = lo[2]; z <= hi[2]; ++z)
        for (y = lo[1]; y <= hi[1]; ++y)
            for (x = lo[0]; x <= hi[0]; ++x)
                w[((long)z * nn[1] + y) * nn[0] + x] /= sum * hd;
}

int or_num_fields(int physics) { return physics == OR_ACOUSTIC ? 3 : 9; }

static double sample(const or_source *s, long k)
{
    return (k >= 0 && k < s->nt) ? s->wavelet[k] : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Strang stepper                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    const or_grid *g;
    axis_tab T[3];
    deriv_ctx c[3];
    long tot;
    double *tmp;     /* one field of scratch */
} stepper;

static void deriv_into(stepper *S, int axis, const double *in, double *out)
{
    apply_lines(S->g, axis, in, out, deriv_op, &S->c[axis], S->g->M[axis] + 3);
}

static int check_grid(const or_grid *g, int physics)
{
    int a;
    if (physics == OR_ACOUSTIC && g->ndim != 2) return -1;
    if (physics == OR_ELASTIC && g->ndim != 3) return -1;
    for (a = 0; a < 3; ++a) {
        if (a == 1 && g->ndim == 2) continue;
        if (g->n[a] < 2 || g->M[a] < 1 || g->h[a] <= 0) return -1;
        if (g->end_mode == OR_END_PERIODIC && 2 * g->halo + 1 > g->n[a]) return -1;
    }
    if (g->halo < 1) return -1;
    return 0;
}

int or_run_from(const or_grid *g, int physics, double dt, int step0, int nsteps,
                const double *vp, const double *vs, const double *rho,
                int nsrc, const or_source *src,
                int nrec, const int *rec_idx, int rec_comp,
                const double *fields_in, double *fields, double *traces)
{
    stepper S;
    long nn[3], tot, i;
    int nf = or_num_fields(physics), a, k, n, r;
    double *F, *K1, *K2, *b, *d[9], **W;
    if (check_grid(g, physics)) return -1;
    grid_nodes(g, nn);
    tot = grid_total(g);
    S.g = g; S.tot = tot;
    for (a = 0; a < 3; ++a) {
        if (a == 1 && g->ndim == 2) { memset(&S.T[a], 0, sizeof(axis_tab)); continue; }
        tab_for_axis(g, a, &S.T[a]);
        S.c[a].T = &S.T[a];
        S.c[a].order = 1;
    }
    F = (double *)calloc((size_t)tot * (nf + 3 + 9), sizeof(double));
    K1 = F + (size_t)tot * nf;   /* acoustic: K = rho c^2 ; elastic: lambda */
    K2 = K1 + tot;               /* elastic: mu */
    b = K2 + tot;                /* 1 / rho */
    for (k = 0; k < 9; ++k) d[k] = b + tot + (size_t)k * tot;
    if (fields_in) memcpy(F, fields_in, sizeof(double) * (size_t)tot * nf);
    for (i = 0; i < tot; ++i) {
        b[i] = 1.0 / rho[i];
        if (physics == OR_ACOUSTIC) {
            K1[i] = rho[i] * vp[i] * vp[i];
        } else {
            K2[i] = rho[i] * vs[i] * vs[i];
            K1[i] = rho[i] * vp[i] * vp[i] - 2.0 * K2[i];
        }
    }
    W = (double **)malloc(sizeof(double *) * (nsrc > 0 ? nsrc : 1));
    for (k = 0; k < nsrc; ++k) {
        W[k] = (double *)malloc(sizeof(double) * tot);
        or_source_weights(g, src[k].pos, src[k].spread, W[k]);
    }

    for (n = 0; n < nsteps; ++n) {
        long sn = (long)step0 + n;
        int half;
        for (half = 0; half < 3; ++half) {
            if (half == 0 || half == 2) {
                /* (A) velocity sub-flow over dt/2 with the stress frozen */
                long fk = half == 0 ? sn : sn + 1;   /* force sample time index */
                double hdt = 0.5 * dt;
                if (physics == OR_ACOUSTIC) {
                    deriv_into(&S, 0, F + OR_A_SIGMA * tot, d[0]);
                    deriv_into(&S, 2, F + OR_A_SIGMA * tot, d[1]);
                    for (i = 0; i < tot; ++i) {
                        F[OR_A_V1 * tot + i] -= hdt * b[i] * d[0][i];
                        F[OR_A_V3 * tot + i] -= hdt * b[i] * d[1][i];
                    }
                    for (k = 0; k < nsrc; ++k) {
                        int fld = src[k].kind == OR_SRC_FORCE_X ? OR_A_V1
                                : src[k].kind == OR_SRC_FORCE_Z ? OR_A_V3 : -1;
                        double s = sample(&src[k], fk);
                        if (fld < 0) continue;
                        for (i = 0; i < tot; ++i) F[fld * tot + i] += hdt * b[i] * s * W[k][i];
                    }
                } else {
                    /* v_i += dt/2 * b * (d_j sigma_ij + f_i) */
                    deriv_into(&S, 0, F + OR_E_S11 * tot, d[0]);
                    deriv_into(&S, 1, F + OR_E_S12 * tot, d[1]);
                    deriv_into(&S, 2, F + OR_E_S13 * tot, d[2]);
                    deriv_into(&S, 0, F + OR_E_S12 * tot, d[3]);
                    deriv_into(&S, 1, F + OR_E_S22 * tot, d[4]);
                    deriv_into(&S, 2, F + OR_E_S23 * tot, d[5]);
                    deriv_into(&S, 0, F + OR_E_S13 * tot, d[6]);
                    deriv_into(&S, 1, F + OR_E_S23 * tot, d[7]);
                    deriv_into(&S, 2, F + OR_E_S33 * tot, d[8]);
                    for (i = 0; i < tot; ++i) {
                        F[OR_E_V1 * tot + i] += hdt * b[i] * (d[0][i] + d[1][i] + d[2][i]);
                        F[OR_E_V2 * tot + i] += hdt * b[i] * (d[3][i] + d[4][i] + d[5][i]);
                        F[OR_E_V3 * tot + i] += hdt * b[i] * (d[6][i] + d[7][i] + d[8][i]);
                    }
                    for (k = 0; k < nsrc; ++k) {
                        int fld = src[k].kind == OR_SRC_FORCE_X ? OR_E_V1
                                : src[k].kind == OR_SRC_FORCE_Y ? OR_E_V2
                                : src[k].kind == OR_SRC_FORCE_Z ? OR_E_V3 : -1;
                        double s = sample(&src[k], fk);
                        if (fld < 0) continue;
                        for (i = 0; i < tot; ++i) F[fld * tot + i] += hdt * b[i] * s * W[k][i];
                    }
                }
            } else {
                /* (B) stress sub-flow over dt with the velocity frozen */
                if (physics == OR_ACOUSTIC) {
                    deriv_into(&S, 0, F + OR_A_V1 * tot, d[0]);
                    deriv_into(&S, 2, F + OR_A_V3 * tot, d[1]);
                    for (i = 0; i < tot; ++i)
                        F[OR_A_SIGMA * tot + i] -= dt * K1[i] * (d[0][i] + d[1][i]);
                    for (k = 0; k < nsrc; ++k) {
                        double s = sample(&src[k], sn);
                        if (src[k].kind != OR_SRC_PRESSURE && src[k].kind != OR_SRC_EXPLOSIVE) continue;
                        for (i = 0; i < tot; ++i) F[OR_A_SIGMA * tot + i] += dt * s * W[k][i];
                    }
                } else {
                    deriv_into(&S, 0, F + OR_E_V1 * tot, d[0]);  /* d1 v1 */
                    deriv_into(&S, 1, F + OR_E_V2 * tot, d[1]);  /* d2 v2 */
                    deriv_into(&S, 2, F + OR_E_V3 * tot, d[2]);  /* d3 v3 */
                    deriv_into(&S, 1, F + OR_E_V1 * tot, d[3]);  /* d2 v1 */
                    deriv_into(&S, 0, F + OR_E_V2 * tot, d[4]);  /* d1 v2 */
                    deriv_into(&S, 2, F + OR_E_V1 * tot, d[5]);  /* d3 v1 */
                    deriv_into(&S, 0, F + OR_E_V3 * tot, d[6]);  /* d1 v3 */
                    deriv_into(&S, 2, F + OR_E_V2 * tot, d[7]);  /* d3 v2 */
                    deriv_into(&S, 1, F + OR_E_V3 * tot, d[8]);  /* d2 v3 */
                    for (i = 0; i < tot; ++i) {
                        double div = d[0][i] + d[1][i] + d[2][i];
                        double lam = K1[i], mu = K2[i];
                        F[OR_E_S11 * tot + i] += dt * (lam * div + 2.0 * mu * d[0][i]);
                        F[OR_E_S22 * tot + i] += dt * (lam * div + 2.0 * mu * d[1][i]);
                        F[OR_E_S33 * tot + i] += dt * (lam * div + 2.0 * mu * d[2][i]);
                        F[OR_E_S12 * tot + i] += dt * mu * (d[3][i] + d[4][i]);
                        F[OR_E_S13 * tot + i] += dt * mu * (d[5][i] + d[6][i]);
                        F[OR_E_S23 * tot + i] += dt * mu * (d[7][i] + d[8][i]);
                    }
                    for (k = 0; k < nsrc; ++k) {
                        double s = sample(&src[k], sn);
                        if (src[k].kind != OR_SRC_PRESSURE && src[k].kind != OR_SRC_EXPLOSIVE) continue;
                        for (i = 0; i < tot; ++i) {
                            F[OR_E_S11 * tot + i] += dt * s * W[k][i];
                            F[OR_E_S22 * tot + i] += dt * s * W[k][i];
                            F[OR_E_S33 * tot + i] += dt * s * W[k][i];
                        }
                    }
                }
            }
        }
        if (traces) {
            int comp = physics == OR_ACOUSTIC ? OR_A_SIGMA : rec_comp;
            for (r = 0; r < nrec; ++r) {
                long ix = rec_idx[3 * r], iy = rec_idx[3 * r + 1], iz = rec_idx[3 * r + 2];
                traces[(size_t)r * nsteps + n] = F[(size_t)comp * tot + (iz * nn[1] + iy) * nn[0] + ix];
            }
        }
    }
    if (fields) memcpy(fields, F, sizeof(double) * (size_t)tot * nf);
    for (k = 0; k < nsrc; ++k) free(W[k]);
    free(W);
    free(F);
    for (a = 0; a < 3; ++a)
        if (!(a == 1 && g->ndim == 2)) axis_tab_free(&S.T[a]);
    return 0;
}

int or_run(const or_grid *g, int physics, double dt, int nsteps,
           const double *vp, const double *vs, const double *rho,
           int nsrc, const or_source *src,
           int nrec, const int *rec_idx, int rec_comp,
           double *fields, double *traces)
{
    return or_run_from(g, physics, dt, 0, nsteps, vp, vs, rho, nsrc, src, nrec, rec_idx,
                       rec_comp, NULL, fields, traces);
}

/* ------------------------------------------------------------------------ */
/* ADE-PML (Sec. 3.3)                                                        */
/* ------------------------------------------------------------------------ */
void or_pml_flow(double d, double k, double alpha, double tau, double D, double psi,
                 double *psi_out, double *dv_over_b)
{
    /* With D frozen, psi' = -beta psi - (d/k^2) D (beta = d/k + alpha) has the exact
     * solution psi(t) = e^{-beta t} psi0 - (d/k^2) t phi1(beta t) D, and
     * int_0^tau psi = tau phi1(x) psi0 - (d/k^2) tau^2 phi2(x) D  (x = beta tau) with
     * the exponential-integrator functions phi1(x) = (1 - e^{-x}) / x and
     * phi2(x) = (x - 1 + e^{-x}) / x^2 (Taylor series near x = 0, where the closed
     * forms cancel).  Then v(tau) - v(0) = -b (tau D / k + int psi). */
    double beta = d / k + alpha, x = beta * tau, phi1, phi2;
    if (fabs(x) < 1e-3) {
        phi1 = 1.0 - x / 2.0 + x * x / 6.0 - x * x * x / 24.0 + x * x * x * x / 120.0;
        phi2 = 0.5 - x / 6.0 + x * x / 24.0 - x * x * x / 120.0 + x * x * x * x / 720.0;
    } else {
        phi1 = -expm1(-x) / x;
        phi2 = (x + expm1(-x)) / (x * x);
    }
    double dk2 = d / (k * k);
    *psi_out = exp(-x) * psi - dk2 * tau * phi1 * D;
    *dv_over_b = -(tau * D / k + tau * phi1 * psi - dk2 * tau * tau * phi2 * D);
}

/* depth fraction into the layer of node j of an axis with N intervals */
static double pml_delta(int j, int N, int width)
{
    int dist = 0;
    if (j < width) dist = width - j;
    if (j > N - width && j - (N - width) > dist) dist = j - (N - width);
    return (double)dist / (double)width;
}

int or_run_pml(const or_grid *g, const or_pml *pml, double dt, int step0, int nsteps,
               const double *vp, const double *rho, int nsrc, const or_source *src,
               int nrec, const int *rec_idx, const double *fields_in, double *fields, double *traces)
{
    stepper S;
    long nn[3], tot, i;
    int a, k, n, r;
    const int nf = 7;
    double *F, *K, *b, *dx, *dz, **W, *pd[3], *pk[3], *pa[3];
    if (check_grid(g, OR_ACOUSTIC) || pml->width < 1 || pml->width > g->n[0] / 2 ||
        pml->width > g->n[2] / 2 || !(pml->R > 0.0 && pml->R < 1.0) || pml->kmax < 1.0 || pml->f0 <= 0.0)
        return -1;
    grid_nodes(g, nn);
    tot = grid_total(g);
    S.g = g; S.tot = tot;
    for (a = 0; a < 3; ++a) {
        if (a == 1) { memset(&S.T[a], 0, sizeof(axis_tab)); continue; }
        tab_for_axis(g, a, &S.T[a]);
        S.c[a].T = &S.T[a];
        S.c[a].order = 1;
    }
    /* profiles d, k, alpha per node of the x and z axes */
    for (a = 0; a < 3; a += 2) {
        int j, N = g->n[a];
        double d0 = -3.0 * pml->cmax * log(pml->R) / (2.0 * pml->width * g->h[a]);
        pd[a] = (double *)malloc(sizeof(double) * 3 * (N + 1));
        pk[a] = pd[a] + N + 1;
        pa[a] = pk[a] + N + 1;
        for (j = 0; j <= N; ++j) {
            double del = pml_delta(j, N, pml->width);
            pd[a][j] = d0 * del * del;
            pk[a][j] = 1.0 + (pml->kmax - 1.0) * del;
            pa[a][j] = 3.14159265358979323846 * pml->f0 * (1.0 - del);
        }
    }
    F = (double *)calloc((size_t)tot * (nf + 4), sizeof(double));
    K = F + (size_t)tot * nf;
    b = K + tot;
    dx = b + tot;
    dz = dx + tot;
    if (fields_in) memcpy(F, fields_in, sizeof(double) * (size_t)tot * nf);
    for (i = 0; i < tot; ++i) {
        b[i] = 1.0 / rho[i];
        K[i] = rho[i] * vp[i] * vp[i];
    }
    W = (double **)malloc(sizeof(double *) * (nsrc > 0 ? nsrc : 1));
    for (k = 0; k < nsrc; ++k) {
        W[k] = (double *)malloc(sizeof(double) * tot);
        or_source_weights(g, src[k].pos, src[k].spread, W[k]);
    }
    double *sig = F, *v1 = F + tot, *v3 = F + 2 * tot;
    double *psx = F + 3 * tot, *psz = F + 4 * tot, *phx = F + 5 * tot, *phz = F + 6 * tot;
    for (n = 0; n < nsteps; ++n) {
        long sn = (long)step0 + n;
        int half;
        for (half = 0; half < 3; ++half) {
            if (half != 1) {
                /* (A) over dt/2 with sigma frozen (eq. ADE_PML_A) */
                long fk = half == 0 ? sn : sn + 1;
                double tau = 0.5 * dt;
                deriv_into(&S, 0, sig, dx);
                deriv_into(&S, 2, sig, dz);
#pragma omp parallel for
                for (i = 0; i < tot; ++i) {
                    int x = (int)(i % nn[0]), z = (int)(i / nn[0]);
                    double p1, dvb;
                    or_pml_flow(pd[0][x], pk[0][x], pa[0][x], tau, dx[i], psx[i], &p1, &dvb);
                    psx[i] = p1;
                    v1[i] += b[i] * dvb;
                    or_pml_flow(pd[2][z], pk[2][z], pa[2][z], tau, dz[i], psz[i], &p1, &dvb);
                    psz[i] = p1;
                    v3[i] += b[i] * dvb;
                }
                for (k = 0; k < nsrc; ++k) {
                    int fld = src[k].kind == OR_SRC_FORCE_X ? OR_A_V1
                            : src[k].kind == OR_SRC_FORCE_Z ? OR_A_V3 : -1;
                    double s = sample(&src[k], fk);
                    if (fld < 0) continue;
                    for (i = 0; i < tot; ++i) F[fld * tot + i] += tau * b[i] * s * W[k][i];
                }
            } else {
                /* (B) over dt with the velocities frozen (eq. ADE_PML_B): the same
                 * exact flow, with K in place of b */
                deriv_into(&S, 0, v1, dx);
                deriv_into(&S, 2, v3, dz);
#pragma omp parallel for
                for (i = 0; i < tot; ++i) {
                    int x = (int)(i % nn[0]), z = (int)(i / nn[0]);
                    double p1, dsk;
                    or_pml_flow(pd[0][x], pk[0][x], pa[0][x], dt, dx[i], phx[i], &p1, &dsk);
                    phx[i] = p1;
                    sig[i] += K[i] * dsk;
                    or_pml_flow(pd[2][z], pk[2][z], pa[2][z], dt, dz[i], phz[i], &p1, &dsk);
                    phz[i] = p1;
                    sig[i] += K[i] * dsk;
                }
                for (k = 0; k < nsrc; ++k) {
                    double s = sample(&src[k], sn);
                    if (src[k].kind != OR_SRC_PRESSURE && src[k].kind != OR_SRC_EXPLOSIVE) continue;
                    for (i = 0; i < tot; ++i) sig[i] += dt * s * W[k][i];
                }
            }
        }
        if (traces)
            for (r = 0; r < nrec; ++r) {
                long ix = rec_idx[3 * r], iz = rec_idx[3 * r + 2];
                traces[(size_t)r * nsteps + n] = sig[iz * nn[0] + ix];
            }
    }
    if (fields) memcpy(fields, F, sizeof(double) * (size_t)tot * nf);
    for (k = 0; k < nsrc; ++k) free(W[k]);
    free(W);
    free(F);
    for (a = 0; a < 3; a += 2) {
        free(pd[a]);
        axis_tab_free(&S.T[a]);
    }
    return 0;
}

/* Elastic 3-D run with the layer on all three axes.  The paper writes the layer out
 * for the 2-D acoustic system only; the same stretching applies to every spatial
 * derivative of the elastic system: each derivative d_j f met in a sub-flow gets a
 * memory variable driven by the profile of axis j, and its sub-flow with d_j f
 * frozen is the exact flow of or_pml_flow.  The elastic signs are +b d_j sigma_ij and
 * +lambda div + 2 mu eps, so each field moves by +(tau D / k + int psi) per derivative.
 * State: the 9 elastic fields (OR_E_* order), then psi[3i + j] of d_j sigma_ij (velocity
 * sub-flow), then phi[3i + j] of d_j v_i (stress sub-flow). */
int or_run_pml_elastic(const or_grid *g, const or_pml *pml, double dt, int step0, int nsteps,
                       const double *vp, const double *vs, const double *rho, int nsrc, const or_source *src,
                       int nrec, const int *rec_idx, int rec_comp,
                       const double *fields_in, double *fields, double *traces)
{
    /* sigma_ij as an index into the elastic fields */
    static const int sig_of[3][3] = {{OR_E_S11, OR_E_S12, OR_E_S13},
                                     {OR_E_S12, OR_E_S22, OR_E_S23},
                                     {OR_E_S13, OR_E_S23, OR_E_S33}};
    stepper S;
    long nn[3], tot, i;
    int a, k, n, r, ci, cj;
    const int nf = 9 + 18;
    double *F, *lam, *mu, *b, *d[9], **W, *pd[3], *pk[3], *pa[3], *psi, *phi;
    if (check_grid(g, OR_ELASTIC) || pml->width < 1 || !(pml->R > 0.0 && pml->R < 1.0) || pml->kmax < 1.0 ||
        pml->f0 <= 0.0 || rec_comp < 0 || rec_comp >= 9)
        return -1;
    for (a = 0; a < 3; ++a)
        if (pml->width > g->n[a] / 2) return -1;
    grid_nodes(g, nn);
    tot = grid_total(g);
    S.g = g; S.tot = tot;
    for (a = 0; a < 3; ++a) {
        tab_for_axis(g, a, &S.T[a]);
        S.c[a].T = &S.T[a];
        S.c[a].order = 1;
    }
    /* the acoustic profiles, on every axis */
    for (a = 0; a < 3; ++a) {
        int j, N = g->n[a];
        double d0 = -3.0 * pml->cmax * log(pml->R) / (2.0 * pml->width * g->h[a]);
        pd[a] = (double *)malloc(sizeof(double) * 3 * (N + 1));
        pk[a] = pd[a] + N + 1;
        pa[a] = pk[a] + N + 1;
        for (j = 0; j <= N; ++j) {
            double del = pml_delta(j, N, pml->width);
            pd[a][j] = d0 * del * del;
            pk[a][j] = 1.0 + (pml->kmax - 1.0) * del;
            pa[a][j] = 3.14159265358979323846 * pml->f0 * (1.0 - del);
        }
    }
    F = (double *)calloc((size_t)tot * (nf + 3 + 9), sizeof(double));
    lam = F + (size_t)tot * nf;
    mu = lam + tot;
    b = mu + tot;
    for (k = 0; k < 9; ++k) d[k] = b + tot + (size_t)k * tot;
    psi = F + (size_t)9 * tot;
    phi = F + (size_t)18 * tot;
    if (fields_in) memcpy(F, fields_in, sizeof(double) * (size_t)tot * nf);
    for (i = 0; i < tot; ++i) {
        b[i] = 1.0 / rho[i];
        mu[i] = rho[i] * vs[i] * vs[i];
        lam[i] = rho[i] * vp[i] * vp[i] - 2.0 * mu[i];
    }
    W = (double **)malloc(sizeof(double *) * (nsrc > 0 ? nsrc : 1));
    for (k = 0; k < nsrc; ++k) {
        W[k] = (double *)malloc(sizeof(double) * tot);
        or_source_weights(g, src[k].pos, src[k].spread, W[k]);
    }
    for (n = 0; n < nsteps; ++n) {
        long sn = (long)step0 + n;
        int half;
        for (half = 0; half < 3; ++half) {
            if (half != 1) {
                /* (A) over dt/2 with the stress frozen: v_i += b sum_j (d_j sigma_ij)_stretched */
                long fk = half == 0 ? sn : sn + 1;
                double tau = 0.5 * dt;
                for (ci = 0; ci < 3; ++ci) {
                    double *v = F + (size_t)(OR_E_V1 + ci) * tot;
                    for (cj = 0; cj < 3; ++cj) deriv_into(&S, cj, F + (size_t)sig_of[ci][cj] * tot, d[cj]);
#pragma omp parallel for
                    for (i = 0; i < tot; ++i) {
                        const int c[3] = {(int)(i % nn[0]), (int)(i / nn[0] % nn[1]), (int)(i / (nn[0] * nn[1]))};
                        int j;
                        for (j = 0; j < 3; ++j) {
                            double p1, dvb, *m = psi + (size_t)(3 * ci + j) * tot;
                            or_pml_flow(pd[j][c[j]], pk[j][c[j]], pa[j][c[j]], tau, d[j][i], m[i], &p1, &dvb);
                            m[i] = p1;
                            v[i] -= b[i] * dvb;
                        }
                    }
                }
                for (k = 0; k < nsrc; ++k) {
                    int fld = src[k].kind == OR_SRC_FORCE_X ? OR_E_V1
                            : src[k].kind == OR_SRC_FORCE_Y ? OR_E_V2
                            : src[k].kind == OR_SRC_FORCE_Z ? OR_E_V3 : -1;
                    double s = sample(&src[k], fk);
                    if (fld < 0) continue;
                    for (i = 0; i < tot; ++i) F[fld * tot + i] += tau * b[i] * s * W[k][i];
                }
            } else {
                /* (B) over dt with the velocity frozen: every d_j v_i stretched, then the
                 * stress-strain law applied to the stretched increments */
                for (ci = 0; ci < 3; ++ci)
                    for (cj = 0; cj < 3; ++cj) deriv_into(&S, cj, F + (size_t)(OR_E_V1 + ci) * tot, d[3 * ci + cj]);
#pragma omp parallel for
                for (i = 0; i < tot; ++i) {
                    const int c[3] = {(int)(i % nn[0]), (int)(i / nn[0] % nn[1]), (int)(i / (nn[0] * nn[1]))};
                    double e[9], div;
                    int q;
                    for (q = 0; q < 9; ++q) {
                        const int j = q % 3;
                        double p1, dvb, *m = phi + (size_t)q * tot;
                        or_pml_flow(pd[j][c[j]], pk[j][c[j]], pa[j][c[j]], dt, d[q][i], m[i], &p1, &dvb);
                        m[i] = p1;
                        e[q] = -dvb;   /* tau D / k + int phi */
                    }
                    div = e[0] + e[4] + e[8];
                    F[OR_E_S11 * tot + i] += lam[i] * div + 2.0 * mu[i] * e[0];
                    F[OR_E_S22 * tot + i] += lam[i] * div + 2.0 * mu[i] * e[4];
                    F[OR_E_S33 * tot + i] += lam[i] * div + 2.0 * mu[i] * e[8];
                    F[OR_E_S12 * tot + i] += mu[i] * (e[1] + e[3]);
                    F[OR_E_S13 * tot + i] += mu[i] * (e[2] + e[6]);
                    F[OR_E_S23 * tot + i] += mu[i] * (e[5] + e[7]);
                }
                for (k = 0; k < nsrc; ++k) {
                    double s = sample(&src[k], sn);
                    if (src[k].kind != OR_SRC_PRESSURE && src[k].kind != OR_SRC_EXPLOSIVE) continue;
                    for (i = 0; i < tot; ++i) {
                        F[OR_E_S11 * tot + i] += dt * s * W[k][i];
                        F[OR_E_S22 * tot + i] += dt * s * W[k][i];
                        F[OR_E_S33 * tot + i] += dt * s * W[k][i];
                    }
                }
            }
        }
        if (traces)
            for (r = 0; r < nrec; ++r) {
                long ix = rec_idx[3 * r], iy = rec_idx[3 * r + 1], iz = rec_idx[3 * r + 2];
                traces[(size_t)r * nsteps + n] = F[(size_t)rec_comp * tot + (iz * nn[1] + iy) * nn[0] + ix];
            }
    }
    if (fields) memcpy(fields, F, sizeof(double) * (size_t)tot * nf);
    for (k = 0; k < nsrc; ++k) free(W[k]);
    free(W);
    free(F);
    for (a = 0; a < 3; ++a) {
        free(pd[a]);
        axis_tab_free(&S.T[a]);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint of the acoustic 2-D Strang scheme                        */
/* ------------------------------------------------------------------------ */
int or_acoustic_adjoint(const or_grid *g, double dt, int nsteps,
                        const double *vp, const double *rho,
                        int nsrc, const or_source *src,
                        int nrec, const int *rec_idx,
                        const double *res, double *grad_K)
{
    long nn[3], tot, i;
    int n, r, k, ax[2] = {0, 2};
    double *Dm[2];
    dense_ctx dc[2];
    double *sig, *v1, *v3, *K, *b, *t0, *t1, *divA, **W;
    double *ls, *m1, *m3, *gs;
    if (check_grid(g, OR_ACOUSTIC)) return -1;
    grid_nodes(g, nn);
    tot = grid_total(g);
    for (k = 0; k < 2; ++k) {
        int N = g->n[ax[k]];
        Dm[k] = (double *)malloc(sizeof(double) * (size_t)(N + 1) * (N + 1));
        or_line_deriv_matrix(N, g->h[ax[k]], g->M[ax[k]], g->halo, g->end_mode, Dm[k]);
        dc[k].D = Dm[k]; dc[k].n = N + 1; dc[k].transpose = 0;
    }
    sig = (double *)calloc((size_t)tot * 11, sizeof(double));
    v1 = sig + tot; v3 = v1 + tot; K = v3 + tot; b = K + tot; t0 = b + tot; t1 = t0 + tot;
    ls = t1 + tot; m1 = ls + tot; m3 = m1 + tot; gs = m3 + tot;
    divA = (double *)malloc(sizeof(double) * (size_t)tot * nsteps);
    if (!divA) { free(sig); return -2; }
    for (i = 0; i < tot; ++i) { K[i] = rho[i] * vp[i] * vp[i]; b[i] = 1.0 / rho[i]; }
    W = (double **)malloc(sizeof(double *) * (nsrc > 0 ? nsrc : 1));
    for (k = 0; k < nsrc; ++k) {
        W[k] = (double *)malloc(sizeof(double) * tot);
        or_source_weights(g, src[k].pos, src[k].spread, W[k]);
    }
    /* forward, same canonical sequence as or_run, keeping div v at the half step */
    for (n = 0; n < nsteps; ++n) {
        int half;
        for (half = 0; half < 2; ++half) {
            long fk = half == 0 ? n : n + 1;
            dc[0].transpose = dc[1].transpose = 0;
            apply_lines(g, 0, sig, t0, dense_op, &dc[0], 0);
            apply_lines(g, 2, sig, t1, dense_op, &dc[1], 0);
            for (i = 0; i < tot; ++i) { v1[i] -= 0.5 * dt * b[i] * t0[i]; v3[i] -= 0.5 * dt * b[i] * t1[i]; }
            for (k = 0; k < nsrc; ++k) {
                double *f = src[k].kind == OR_SRC_FORCE_X ? v1 : src[k].kind == OR_SRC_FORCE_Z ? v3 : NULL;
                double s = sample(&src[k], fk);
                if (!f) continue;
                for (i = 0; i < tot; ++i) f[i] += 0.5 * dt * b[i] * s * W[k][i];
            }
            if (half == 1) break;
            apply_lines(g, 0, v1, t0, dense_op, &dc[0], 0);
            apply_lines(g, 2, v3, t1, dense_op, &dc[1], 0);
            for (i = 0; i < tot; ++i) {
                divA[(size_t)n * tot + i] = t0[i] + t1[i];
                sig[i] -= dt * K[i] * (t0[i] + t1[i]);
            }
            for (k = 0; k < nsrc; ++k) {
                double s = sample(&src[k], n);
                if (src[k].kind != OR_SRC_PRESSURE && src[k].kind != OR_SRC_EXPLOSIVE) continue;
                for (i = 0; i < tot; ++i) sig[i] += dt * s * W[k][i];
            }
        }
    }
    /* reverse sweep: ls = adjoint of sigma^{n+1}; m1, m3 = adjoint of v^{n+1} */
    for (i = 0; i < tot; ++i) { ls[i] = m1[i] = m3[i] = 0.0; grad_K[i] = 0.0; }
    dc[0].transpose = dc[1].transpose = 1;
    for (n = nsteps - 1; n >= 0; --n) {
        /* trace injection and the second velocity half step */
        for (r = 0; r < nrec; ++r) {
            long ix = rec_idx[3 * r], iz = rec_idx[3 * r + 2];
            ls[iz * nn[0] + ix] += res[(size_t)r * nsteps + n];
        }
        for (i = 0; i < tot; ++i) { t0[i] = b[i] * m1[i]; t1[i] = b[i] * m3[i]; }
        apply_lines(g, 0, t0, gs, dense_op, &dc[0], 0);
        for (i = 0; i < tot; ++i) ls[i] -= 0.5 * dt * gs[i];
        apply_lines(g, 2, t1, gs, dense_op, &dc[1], 0);
        for (i = 0; i < tot; ++i) ls[i] -= 0.5 * dt * gs[i];
        /* stress sub-flow: gradient, then the velocity adjoint */
        for (i = 0; i < tot; ++i) {
            grad_K[i] -= dt * ls[i] * divA[(size_t)n * tot + i];
            t0[i] = K[i] * ls[i];
        }
        apply_lines(g, 0, t0, gs, dense_op, &dc[0], 0);
        for (i = 0; i < tot; ++i) m1[i] -= dt * gs[i];
        apply_lines(g, 2, t0, gs, dense_op, &dc[1], 0);
        for (i = 0; i < tot; ++i) m3[i] -= dt * gs[i];
        /* first velocity half step */
        for (i = 0; i < tot; ++i) { t0[i] = b[i] * m1[i]; t1[i] = b[i] * m3[i]; }
        apply_lines(g, 0, t0, gs, dense_op, &dc[0], 0);
        for (i = 0; i < tot; ++i) ls[i] -= 0.5 * dt * gs[i];
        apply_lines(g, 2, t1, gs, dense_op, &dc[1], 0);
        for (i = 0; i < tot; ++i) ls[i] -= 0.5 * dt * gs[i];
    }
    for (k = 0; k < nsrc; ++k) free(W[k]);
    free(W);
    free(divA);
    free(sig);
    free(Dm[0]); free(Dm[1]);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint of the elastic 3-D Strang scheme                         */
/* ------------------------------------------------------------------------ */
/* Plain transposes, one operation at a time, of the canonical sequence of or_run_from:
 *   A(dt/2): v_i += (dt/2) b sum_j D_j sigma_ij (+ forces)
 *   B(dt):   sigma_kk += dt (lambda tr(e) + 2 mu e_kk), sigma_ij += dt mu g_ij (i < j)
 *            with e_kk = D_k v_k, g_ij = D_j v_i + D_i v_j
 *   A(dt/2) again; trace n samples field rec_comp after the step.
 * Adjoints (bars) in the same field order as the state.  Transposing A: each
 * sigma_ij-bar gains (dt/2) D_j^T (b v_i-bar) from every velocity it drives.
 * Transposing B: v_k-bar gains dt D_k^T (lambda S + 2 mu sigma_kk-bar) with S the sum of
 * the normal stress bars, and v_i-bar, v_j-bar gain dt D_j^T (mu sigma_ij-bar),
 * dt D_i^T (mu sigma_ij-bar).  Lambda and mu enter B only:
 *   dJ/dlambda += dt tr(e) S,  dJ/dmu += dt (2 sum_k e_kk sigma_kk-bar + sum g_ij sigma_ij-bar),
 * with the strains of the state B was applied to; b = 1/rho enters A only:
 *   dJ/db += (dt/2) sum_i (sum_j D_j sigma_ij + f_i W) v_i-bar per velocity half step. */
int or_elastic_adjoint(const or_grid *g, double dt, int nsteps,
                       const double *vp, const double *vs, const double *rho,
                       int nsrc, const or_source *src,
                       int nrec, const int *rec_idx, int rec_comp,
                       const double *res, double *grad_lam, double *grad_mu, double *grad_b)
{
    /* sigma_ij as an index into the fields; shear pairs (i, j) */
    static const int sig_of[3][3] = {{OR_E_S11, OR_E_S12, OR_E_S13},
                                     {OR_E_S12, OR_E_S22, OR_E_S23},
                                     {OR_E_S13, OR_E_S23, OR_E_S33}};
    static const int shear[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    long nn[3], tot, i;
    int n, r, k, a, ci, cj, half;
    double *Dm[3];
    dense_ctx dc[3];
    double *F, *Fb, *lam, *mu, *b, *t0, *t1, *strain, *gsig, **W;
    if (check_grid(g, OR_ELASTIC) || rec_comp < 0 || rec_comp >= 9) return -1;
    grid_nodes(g, nn);
    tot = grid_total(g);
    for (a = 0; a < 3; ++a) {
        int N = g->n[a];
        Dm[a] = (double *)malloc(sizeof(double) * (size_t)(N + 1) * (N + 1));
        or_line_deriv_matrix(N, g->h[a], g->M[a], g->halo, g->end_mode, Dm[a]);
        dc[a].D = Dm[a]; dc[a].n = N + 1; dc[a].transpose = 0;
    }
    F = (double *)calloc((size_t)tot * 23, sizeof(double));
    Fb = F + (size_t)9 * tot;
    lam = Fb + (size_t)9 * tot; mu = lam + tot; b = mu + tot; t0 = b + tot; t1 = t0 + tot;
    strain = (double *)malloc(sizeof(double) * (size_t)tot * 6 * nsteps);
    /* per velocity half step (2n + h): sum_j D_j sigma_ij + f_i W, what b multiplies */
    gsig = (double *)calloc((size_t)tot * 3 * 2 * nsteps, sizeof(double));
    if (!strain || !gsig) { free(strain); free(gsig); free(F); return -2; }
    for (i = 0; i < tot; ++i) {
        b[i] = 1.0 / rho[i];
        mu[i] = rho[i] * vs[i] * vs[i];
        lam[i] = rho[i] * vp[i] * vp[i] - 2.0 * mu[i];
    }
    W = (double **)malloc(sizeof(double *) * (nsrc > 0 ? nsrc : 1));
    for (k = 0; k < nsrc; ++k) {
        W[k] = (double *)malloc(sizeof(double) * tot);
        or_source_weights(g, src[k].pos, src[k].spread, W[k]);
    }
    /* forward, keeping e_11, e_22, e_33, g_12, g_13, g_23 of the state B sees */
    for (n = 0; n < nsteps; ++n) {
        for (half = 0; half < 2; ++half) {
            long fk = half == 0 ? n : n + 1;
            double *gh = gsig + (size_t)(2 * n + half) * 3 * tot;
            for (ci = 0; ci < 3; ++ci)
                for (cj = 0; cj < 3; ++cj) {
                    apply_lines(g, cj, F + (size_t)sig_of[ci][cj] * tot, t0, dense_op, &dc[cj], 0);
                    for (i = 0; i < tot; ++i) {
                        F[(size_t)(OR_E_V1 + ci) * tot + i] += 0.5 * dt * b[i] * t0[i];
                        gh[(size_t)ci * tot + i] += t0[i];
                    }
                }
            for (k = 0; k < nsrc; ++k) {
                int fld = src[k].kind == OR_SRC_FORCE_X ? OR_E_V1
                        : src[k].kind == OR_SRC_FORCE_Y ? OR_E_V2
                        : src[k].kind == OR_SRC_FORCE_Z ? OR_E_V3 : -1;
                double s = sample(&src[k], fk);
                if (fld < 0) continue;
                for (i = 0; i < tot; ++i) {
                    F[(size_t)fld * tot + i] += 0.5 * dt * b[i] * s * W[k][i];
                    gh[(size_t)(fld - OR_E_V1) * tot + i] += s * W[k][i];
                }
            }
            if (half == 1) break;
            {
                double *e = strain + (size_t)n * 6 * tot;
                for (k = 0; k < 3; ++k)
                    apply_lines(g, k, F + (size_t)(OR_E_V1 + k) * tot, e + (size_t)k * tot, dense_op, &dc[k], 0);
                for (k = 0; k < 3; ++k) {
                    int p = shear[k][0], q = shear[k][1];
                    double *gk = e + (size_t)(3 + k) * tot;
                    apply_lines(g, q, F + (size_t)(OR_E_V1 + p) * tot, gk, dense_op, &dc[q], 0);
                    apply_lines(g, p, F + (size_t)(OR_E_V1 + q) * tot, t0, dense_op, &dc[p], 0);
                    for (i = 0; i < tot; ++i) gk[i] += t0[i];
                }
                for (i = 0; i < tot; ++i) {
                    double tr = e[i] + e[tot + i] + e[2 * tot + i];
                    for (k = 0; k < 3; ++k)
                        F[(size_t)(OR_E_S11 + k) * tot + i] += dt * (lam[i] * tr + 2.0 * mu[i] * e[(size_t)k * tot + i]);
                    F[(size_t)OR_E_S12 * tot + i] += dt * mu[i] * e[3 * (size_t)tot + i];
                    F[(size_t)OR_E_S13 * tot + i] += dt * mu[i] * e[4 * (size_t)tot + i];
                    F[(size_t)OR_E_S23 * tot + i] += dt * mu[i] * e[5 * (size_t)tot + i];
                }
            }
            for (k = 0; k < nsrc; ++k) {
                double s = sample(&src[k], n);
                if (src[k].kind != OR_SRC_PRESSURE && src[k].kind != OR_SRC_EXPLOSIVE) continue;
                for (i = 0; i < tot; ++i)
                    for (a = 0; a < 3; ++a) F[(size_t)(OR_E_S11 + a) * tot + i] += dt * s * W[k][i];
            }
        }
    }
    /* reverse sweep */
    for (i = 0; i < tot; ++i) {
        grad_lam[i] = 0.0;
        grad_mu[i] = 0.0;
        if (grad_b) grad_b[i] = 0.0;
    }
    dc[0].transpose = dc[1].transpose = dc[2].transpose = 1;
    for (n = nsteps - 1; n >= 0; --n) {
        const double *e = strain + (size_t)n * 6 * tot;
        for (r = 0; r < nrec; ++r) {
            long ix = rec_idx[3 * r], iy = rec_idx[3 * r + 1], iz = rec_idx[3 * r + 2];
            Fb[(size_t)rec_comp * tot + (iz * nn[1] + iy) * nn[0] + ix] += res[(size_t)r * nsteps + n];
        }
        for (half = 0; half < 2; ++half) {
            /* dJ/db: (dt/2) (sum_j D_j sigma_ij + f_i W) against v_i-bar, which the
             * transpose of A leaves unchanged (reverse half 0 undoes the step's second
             * velocity half step) */
            if (grad_b) {
                const double *gh = gsig + (size_t)(2 * n + 1 - half) * 3 * tot;
                for (ci = 0; ci < 3; ++ci)
                    for (i = 0; i < tot; ++i)
                        grad_b[i] += 0.5 * dt * gh[(size_t)ci * tot + i] * Fb[(size_t)(OR_E_V1 + ci) * tot + i];
            }
            /* transpose of A(dt/2) */
            for (ci = 0; ci < 3; ++ci) {
                for (i = 0; i < tot; ++i) t1[i] = b[i] * Fb[(size_t)(OR_E_V1 + ci) * tot + i];
                for (cj = 0; cj < 3; ++cj) {
                    apply_lines(g, cj, t1, t0, dense_op, &dc[cj], 0);
                    for (i = 0; i < tot; ++i) Fb[(size_t)sig_of[ci][cj] * tot + i] += 0.5 * dt * t0[i];
                }
            }
            if (half == 1) break;
            /* gradient with the strains B used, then the transpose of B */
            for (i = 0; i < tot; ++i) {
                double S = Fb[(size_t)OR_E_S11 * tot + i] + Fb[(size_t)OR_E_S22 * tot + i] + Fb[(size_t)OR_E_S33 * tot + i];
                double tr = e[i] + e[tot + i] + e[2 * tot + i], m = 0.0;
                for (k = 0; k < 3; ++k) m += 2.0 * e[(size_t)k * tot + i] * Fb[(size_t)(OR_E_S11 + k) * tot + i];
                m += e[3 * (size_t)tot + i] * Fb[(size_t)OR_E_S12 * tot + i] + e[4 * (size_t)tot + i] * Fb[(size_t)OR_E_S13 * tot + i]
                   + e[5 * (size_t)tot + i] * Fb[(size_t)OR_E_S23 * tot + i];
                grad_lam[i] += dt * tr * S;
                grad_mu[i] += dt * m;
            }
            for (k = 0; k < 3; ++k) {
                for (i = 0; i < tot; ++i) {
                    double S = Fb[(size_t)OR_E_S11 * tot + i] + Fb[(size_t)OR_E_S22 * tot + i] + Fb[(size_t)OR_E_S33 * tot + i];
                    t1[i] = lam[i] * S + 2.0 * mu[i] * Fb[(size_t)(OR_E_S11 + k) * tot + i];
                }
                apply_lines(g, k, t1, t0, dense_op, &dc[k], 0);
                for (i = 0; i < tot; ++i) Fb[(size_t)(OR_E_V1 + k) * tot + i] += dt * t0[i];
            }
            for (k = 0; k < 3; ++k) {
                int p = shear[k][0], q = shear[k][1];
                for (i = 0; i < tot; ++i) t1[i] = mu[i] * Fb[(size_t)sig_of[p][q] * tot + i];
                apply_lines(g, q, t1, t0, dense_op, &dc[q], 0);
                for (i = 0; i < tot; ++i) Fb[(size_t)(OR_E_V1 + p) * tot + i] += dt * t0[i];
                apply_lines(g, p, t1, t0, dense_op, &dc[p], 0);
                for (i = 0; i < tot; ++i) Fb[(size_t)(OR_E_V1 + q) * tot + i] += dt * t0[i];
            }
        }
    }
    for (k = 0; k < nsrc; ++k) free(W[k]);
    free(W);
    free(strain);
    free(gsig);
    free(F);
    for (a = 0; a < 3; ++a) free(Dm[a]);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint of the acoustic 2-D scheme with the absorbing layer      */
/* ------------------------------------------------------------------------ */
/* Every sub-flow of or_run_pml is linear in (D, psi): with the flow's own outputs for
 * unit inputs, psi' = Ep psi + Dp D and field += c (Dv D + Pv psi) (c = b or K).  Its
 * transpose, given the field's bar fb (unchanged) and psi'-bar mb:
 *   D-bar = c Dv fb + Dp mb,  psi-bar = c Pv fb + Ep mb,  input-bar += D^T (D-bar).
 * dJ/dK gathers sigma-bar times the stress sub-flow's drive (Dv D + Pv phi, both axes). */
typedef struct { double *Ep, *Dp, *Dv, *Pv; } flow_lin;

static void flow_lin_build(const or_pml *pml, const or_grid *g, int a, double tau, flow_lin *L)
{
    int j, N = g->n[a];
    double d0 = -3.0 * pml->cmax * log(pml->R) / (2.0 * pml->width * g->h[a]);
    L->Ep = (double *)malloc(sizeof(double) * 4 * (N + 1));
    L->Dp = L->Ep + N + 1; L->Dv = L->Dp + N + 1; L->Pv = L->Dv + N + 1;
    for (j = 0; j <= N; ++j) {
        double del = pml_delta(j, N, pml->width);
        double d = d0 * del * del, k = 1.0 + (pml->kmax - 1.0) * del;
        double al = 3.14159265358979323846 * pml->f0 * (1.0 - del);
        or_pml_flow(d, k, al, tau, 1.0, 0.0, &L->Dp[j], &L->Dv[j]);
        or_pml_flow(d, k, al, tau, 0.0, 1.0, &L->Ep[j], &L->Pv[j]);
    }
}

int or_acoustic_adjoint_pml(const or_grid *g, const or_pml *pml, double dt, int nsteps,
                            const double *vp, const double *rho, int nsrc, const or_source *src,
                            int nrec, const int *rec_idx, const double *res, double *grad_K)
{
    long nn[3], tot, i;
    int n, r, k, half, ax[2] = {0, 2};
    double *Dm[2];
    dense_ctx dc[2];
    flow_lin Lh[2], Lf[2];        /* tau = dt/2 (velocity), dt (stress), per axis x, z */
    double *F, *K, *b, *t0, *t1, *drive, **W;
    double *sig, *v1, *v3, *psx, *psz, *phx, *phz;
    double *sb, *m1, *m3, *bpsx, *bpsz, *bphx, *bphz;
    if (check_grid(g, OR_ACOUSTIC) || pml->width < 1 || pml->width > g->n[0] / 2 ||
        pml->width > g->n[2] / 2 || !(pml->R > 0.0 && pml->R < 1.0) || pml->kmax < 1.0 || pml->f0 <= 0.0)
        return -1;
    grid_nodes(g, nn);
    tot = grid_total(g);
    for (k = 0; k < 2; ++k) {
        int N = g->n[ax[k]];
        Dm[k] = (double *)malloc(sizeof(double) * (size_t)(N + 1) * (N + 1));
        or_line_deriv_matrix(N, g->h[ax[k]], g->M[ax[k]], g->halo, g->end_mode, Dm[k]);
        dc[k].D = Dm[k]; dc[k].n = N + 1; dc[k].transpose = 0;
        flow_lin_build(pml, g, ax[k], 0.5 * dt, &Lh[k]);
        flow_lin_build(pml, g, ax[k], dt, &Lf[k]);
    }
    F = (double *)calloc((size_t)tot * 18, sizeof(double));
    sig = F; v1 = F + tot; v3 = F + 2 * tot; psx = F + 3 * tot; psz = F + 4 * tot; phx = F + 5 * tot;
    phz = F + 6 * tot; K = F + 7 * tot; b = F + 8 * tot; t0 = F + 9 * tot; t1 = F + 10 * tot;
    sb = F + 11 * tot; m1 = F + 12 * tot; m3 = F + 13 * tot; bpsx = F + 14 * tot; bpsz = F + 15 * tot;
    bphx = F + 16 * tot; bphz = F + 17 * tot;
    drive = (double *)malloc(sizeof(double) * (size_t)tot * nsteps);
    if (!drive) { free(F); return -2; }
    for (i = 0; i < tot; ++i) { K[i] = rho[i] * vp[i] * vp[i]; b[i] = 1.0 / rho[i]; }
    W = (double **)malloc(sizeof(double *) * (nsrc > 0 ? nsrc : 1));
    for (k = 0; k < nsrc; ++k) {
        W[k] = (double *)malloc(sizeof(double) * tot);
        or_source_weights(g, src[k].pos, src[k].spread, W[k]);
    }
    /* forward: the sequence of or_run_pml through the linear forms, keeping the stress
     * sub-flow's drive per step */
    for (n = 0; n < nsteps; ++n) {
        for (half = 0; half < 2; ++half) {
            long fk = half == 0 ? n : n + 1;
            apply_lines(g, 0, sig, t0, dense_op, &dc[0], 0);
            apply_lines(g, 2, sig, t1, dense_op, &dc[1], 0);
            for (i = 0; i < tot; ++i) {
                int x = (int)(i % nn[0]), z = (int)(i / nn[0]);
                double px = psx[i], pz = psz[i];
                psx[i] = Lh[0].Ep[x] * px + Lh[0].Dp[x] * t0[i];
                v1[i] += b[i] * (Lh[0].Dv[x] * t0[i] + Lh[0].Pv[x] * px);
                psz[i] = Lh[1].Ep[z] * pz + Lh[1].Dp[z] * t1[i];
                v3[i] += b[i] * (Lh[1].Dv[z] * t1[i] + Lh[1].Pv[z] * pz);
            }
            for (k = 0; k < nsrc; ++k) {
                double *f = src[k].kind == OR_SRC_FORCE_X ? v1 : src[k].kind == OR_SRC_FORCE_Z ? v3 : NULL;
                double s = sample(&src[k], fk);
                if (!f) continue;
                for (i = 0; i < tot; ++i) f[i] += 0.5 * dt * b[i] * s * W[k][i];
            }
            if (half == 1) break;
            apply_lines(g, 0, v1, t0, dense_op, &dc[0], 0);
            apply_lines(g, 2, v3, t1, dense_op, &dc[1], 0);
            for (i = 0; i < tot; ++i) {
                int x = (int)(i % nn[0]), z = (int)(i / nn[0]);
                double fx = phx[i], fz = phz[i];
                double dr = Lf[0].Dv[x] * t0[i] + Lf[0].Pv[x] * fx + Lf[1].Dv[z] * t1[i] + Lf[1].Pv[z] * fz;
                phx[i] = Lf[0].Ep[x] * fx + Lf[0].Dp[x] * t0[i];
                phz[i] = Lf[1].Ep[z] * fz + Lf[1].Dp[z] * t1[i];
                drive[(size_t)n * tot + i] = dr;
                sig[i] += K[i] * dr;
            }
            for (k = 0; k < nsrc; ++k) {
                double s = sample(&src[k], n);
                if (src[k].kind != OR_SRC_PRESSURE && src[k].kind != OR_SRC_EXPLOSIVE) continue;
                for (i = 0; i < tot; ++i) sig[i] += dt * s * W[k][i];
            }
        }
    }
    /* reverse sweep */
    for (i = 0; i < tot; ++i) grad_K[i] = 0.0;
    dc[0].transpose = dc[1].transpose = 1;
    for (n = nsteps - 1; n >= 0; --n) {
        for (r = 0; r < nrec; ++r) {
            long ix = rec_idx[3 * r], iz = rec_idx[3 * r + 2];
            sb[iz * nn[0] + ix] += res[(size_t)r * nsteps + n];
        }
        for (half = 0; half < 2; ++half) {
            /* transpose of a velocity half step: (v1, psi_x) from sigma along x, (v3, psi_z)
             * along z */
            for (i = 0; i < tot; ++i) {
                int x = (int)(i % nn[0]), z = (int)(i / nn[0]);
                double mx = bpsx[i], mz = bpsz[i];
                t0[i] = b[i] * Lh[0].Dv[x] * m1[i] + Lh[0].Dp[x] * mx;
                bpsx[i] = b[i] * Lh[0].Pv[x] * m1[i] + Lh[0].Ep[x] * mx;
                t1[i] = b[i] * Lh[1].Dv[z] * m3[i] + Lh[1].Dp[z] * mz;
                bpsz[i] = b[i] * Lh[1].Pv[z] * m3[i] + Lh[1].Ep[z] * mz;
            }
            apply_lines(g, 0, t0, t0, dense_op, &dc[0], 0);
            for (i = 0; i < tot; ++i) sb[i] += t0[i];
            apply_lines(g, 2, t1, t1, dense_op, &dc[1], 0);
            for (i = 0; i < tot; ++i) sb[i] += t1[i];
            if (half == 1) break;
            /* dJ/dK, then the transpose of the stress sub-flow */
            for (i = 0; i < tot; ++i) {
                int x = (int)(i % nn[0]), z = (int)(i / nn[0]);
                double fx = bphx[i], fz = bphz[i];
                grad_K[i] += sb[i] * drive[(size_t)n * tot + i];
                t0[i] = K[i] * Lf[0].Dv[x] * sb[i] + Lf[0].Dp[x] * fx;
                bphx[i] = K[i] * Lf[0].Pv[x] * sb[i] + Lf[0].Ep[x] * fx;
                t1[i] = K[i] * Lf[1].Dv[z] * sb[i] + Lf[1].Dp[z] * fz;
                bphz[i] = K[i] * Lf[1].Pv[z] * sb[i] + Lf[1].Ep[z] * fz;
            }
            apply_lines(g, 0, t0, t0, dense_op, &dc[0], 0);
            for (i = 0; i < tot; ++i) m1[i] += t0[i];
            apply_lines(g, 2, t1, t1, dense_op, &dc[1], 0);
            for (i = 0; i < tot; ++i) m3[i] += t1[i];
        }
    }
    for (k = 0; k < nsrc; ++k) free(W[k]);
    free(W);
    free(drive);
    free(F);
    for (k = 0; k < 2; ++k) { free(Dm[k]); free(Lh[k].Ep); free(Lf[k].Ep); }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint of the elastic 3-D scheme with the absorbing layer       */
/* ------------------------------------------------------------------------ */
/* The canonical sequence of or_run_pml_elastic written through the flows' linear forms
 * (flow_lin: with L = the form of the pass's axis and time span, the pass maps
 * (D, psi) to psi' = Ep psi + Dp D and the drive Dv D + Pv psi):
 *   A(dt/2): v_i += -b (Dv D_j sigma_ij + Pv psi_ij) for every j, psi_ij advanced (+ forces);
 *   B(dt):   e_ij = -(Dv D_j v_i + Pv phi_ij) (stretched increments, dt included),
 *            phi_ij advanced; sigma_kk += lambda tr(e) + 2 mu e_kk,
 *            sigma_ij += mu (e_ij + e_ji) (i < j).
 * Transposes, given the field bars and the memory-variable bars (of psi', phi'):
 *   A: for each pass, t = -b v_i-bar; D-bar = Dv t + Dp psi-bar, psi-bar <- Pv t + Ep psi-bar,
 *      sigma_ij-bar += D_j^T D-bar;
 *   B: e-bar_kk = lambda S + 2 mu sigma_kk-bar (S the sum of the normal bars),
 *      e-bar_ij = e-bar_ji = mu sigma_ij-bar; t = -e-bar_ij; D-bar = Dv t + Dp phi-bar,
 *      phi-bar <- Pv t + Ep phi-bar, v_i-bar += D_j^T D-bar.
 * Gradients as in or_elastic_adjoint with the stretched increments: dJ/dlambda += tr(e) S,
 * dJ/dmu += 2 sum_k e_kk sigma_kk-bar + sum_{i<j} (e_ij + e_ji) sigma_ij-bar, and
 * dJ/db += the drive of each velocity half step (-(Dv D + Pv psi) summed over j, plus
 * (dt/2) f_i W) times v_i-bar. */
int or_elastic_adjoint_pml(const or_grid *g, const or_pml *pml, double dt, int nsteps,
                           const double *vp, const double *vs, const double *rho,
                           int nsrc, const or_source *src,
                           int nrec, const int *rec_idx, int rec_comp,
                           const double *res, double *grad_lam, double *grad_mu, double *grad_b)
{
    static const int sig_of[3][3] = {{OR_E_S11, OR_E_S12, OR_E_S13},
                                     {OR_E_S12, OR_E_S22, OR_E_S23},
                                     {OR_E_S13, OR_E_S23, OR_E_S33}};
    static const int shear[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    long nn[3], tot, i;
    int n, r, k, a, ci, cj, half;
    double *Dm[3];
    dense_ctx dc[3];
    flow_lin Lh[3], Lf[3];        /* tau = dt/2 (velocity half steps), dt (stress), per axis */
    double *F, *Fb, *psi, *phi, *bpsi, *bphi, *lam, *mu, *b, *t0, *t1, *strain, *drive, **W;
    if (check_grid(g, OR_ELASTIC) || rec_comp < 0 || rec_comp >= 9) return -1;
    for (a = 0; a < 3; ++a)
        if (pml->width < 1 || pml->width > g->n[a] / 2) return -1;
    if (!(pml->R > 0.0 && pml->R < 1.0) || pml->kmax < 1.0 || pml->f0 <= 0.0) return -1;
    grid_nodes(g, nn);
    tot = grid_total(g);
    for (a = 0; a < 3; ++a) {
        int N = g->n[a];
        Dm[a] = (double *)malloc(sizeof(double) * (size_t)(N + 1) * (N + 1));
        or_line_deriv_matrix(N, g->h[a], g->M[a], g->halo, g->end_mode, Dm[a]);
        dc[a].D = Dm[a]; dc[a].n = N + 1; dc[a].transpose = 0;
        flow_lin_build(pml, g, a, 0.5 * dt, &Lh[a]);
        flow_lin_build(pml, g, a, dt, &Lf[a]);
    }
    F = (double *)calloc((size_t)tot * 59, sizeof(double));
    Fb = F + (size_t)9 * tot;
    psi = Fb + (size_t)9 * tot; phi = psi + (size_t)9 * tot;
    bpsi = phi + (size_t)9 * tot; bphi = bpsi + (size_t)9 * tot;
    lam = bphi + (size_t)9 * tot; mu = lam + tot; b = mu + tot; t0 = b + tot; t1 = t0 + tot;
    /* per step: the stretched e_11, e_22, e_33, e_12 + e_21, e_13 + e_31, e_23 + e_32;
     * per velocity half step (2n + h): each component's drive, what b multiplies */
    strain = (double *)malloc(sizeof(double) * (size_t)tot * 6 * nsteps);
    drive = (double *)calloc((size_t)tot * 3 * 2 * nsteps, sizeof(double));
    if (!F || !strain || !drive) { free(strain); free(drive); free(F); return -2; }
    for (i = 0; i < tot; ++i) {
        b[i] = 1.0 / rho[i];
        mu[i] = rho[i] * vs[i] * vs[i];
        lam[i] = rho[i] * vp[i] * vp[i] - 2.0 * mu[i];
    }
    W = (double **)malloc(sizeof(double *) * (nsrc > 0 ? nsrc : 1));
    for (k = 0; k < nsrc; ++k) {
        W[k] = (double *)malloc(sizeof(double) * tot);
        or_source_weights(g, src[k].pos, src[k].spread, W[k]);
    }
    for (n = 0; n < nsteps; ++n) {
        for (half = 0; half < 2; ++half) {
            long fk = half == 0 ? n : n + 1;
            double *dr = drive + (size_t)(2 * n + half) * 3 * tot;
            for (ci = 0; ci < 3; ++ci)
                for (cj = 0; cj < 3; ++cj) {
                    const flow_lin *L = &Lh[cj];
                    double *m = psi + (size_t)(3 * ci + cj) * tot;
                    apply_lines(g, cj, F + (size_t)sig_of[ci][cj] * tot, t0, dense_op, &dc[cj], 0);
                    for (i = 0; i < tot; ++i) {
                        const long c[3] = {i % nn[0], i / nn[0] % nn[1], i / (nn[0] * nn[1])};
                        const long jj = c[cj];
                        const double m0 = m[i], inc = -(L->Dv[jj] * t0[i] + L->Pv[jj] * m0);
                        m[i] = L->Ep[jj] * m0 + L->Dp[jj] * t0[i];
                        F[(size_t)(OR_E_V1 + ci) * tot + i] += b[i] * inc;
                        dr[(size_t)ci * tot + i] += inc;
                    }
                }
            for (k = 0; k < nsrc; ++k) {
                int fld = src[k].kind == OR_SRC_FORCE_X ? OR_E_V1
                        : src[k].kind == OR_SRC_FORCE_Y ? OR_E_V2
                        : src[k].kind == OR_SRC_FORCE_Z ? OR_E_V3 : -1;
                double sv = sample(&src[k], fk);
                if (fld < 0) continue;
                for (i = 0; i < tot; ++i) {
                    F[(size_t)fld * tot + i] += 0.5 * dt * b[i] * sv * W[k][i];
                    dr[(size_t)(fld - OR_E_V1) * tot + i] += 0.5 * dt * sv * W[k][i];
                }
            }
            if (half == 1) break;
            {
                double *e = strain + (size_t)n * 6 * tot;
                double *inc = (double *)malloc(sizeof(double) * (size_t)tot * 9);
                int q;
                for (q = 0; q < 9; ++q) {
                    const int vi = q / 3, j = q % 3;
                    const flow_lin *L = &Lf[j];
                    double *m = phi + (size_t)q * tot;
                    apply_lines(g, j, F + (size_t)(OR_E_V1 + vi) * tot, t0, dense_op, &dc[j], 0);
                    for (i = 0; i < tot; ++i) {
                        const long c[3] = {i % nn[0], i / nn[0] % nn[1], i / (nn[0] * nn[1])};
                        const long jj = c[j];
                        const double m0 = m[i];
                        inc[(size_t)q * tot + i] = -(L->Dv[jj] * t0[i] + L->Pv[jj] * m0);
                        m[i] = L->Ep[jj] * m0 + L->Dp[jj] * t0[i];
                    }
                }
                for (i = 0; i < tot; ++i) {
                    double tr;
                    e[i] = inc[i];
                    e[tot + i] = inc[4 * (size_t)tot + i];
                    e[2 * (size_t)tot + i] = inc[8 * (size_t)tot + i];
                    e[3 * (size_t)tot + i] = inc[1 * (size_t)tot + i] + inc[3 * (size_t)tot + i];
                    e[4 * (size_t)tot + i] = inc[2 * (size_t)tot + i] + inc[6 * (size_t)tot + i];
                    e[5 * (size_t)tot + i] = inc[5 * (size_t)tot + i] + inc[7 * (size_t)tot + i];
                    tr = e[i] + e[tot + i] + e[2 * (size_t)tot + i];
                    for (k = 0; k < 3; ++k)
                        F[(size_t)(OR_E_S11 + k) * tot + i] += lam[i] * tr + 2.0 * mu[i] * e[(size_t)k * tot + i];
                    F[(size_t)OR_E_S12 * tot + i] += mu[i] * e[3 * (size_t)tot + i];
                    F[(size_t)OR_E_S13 * tot + i] += mu[i] * e[4 * (size_t)tot + i];
                    F[(size_t)OR_E_S23 * tot + i] += mu[i] * e[5 * (size_t)tot + i];
                }
                free(inc);
            }
            for (k = 0; k < nsrc; ++k) {
                double sv = sample(&src[k], n);
                if (src[k].kind != OR_SRC_PRESSURE && src[k].kind != OR_SRC_EXPLOSIVE) continue;
                for (i = 0; i < tot; ++i)
                    for (a = 0; a < 3; ++a) F[(size_t)(OR_E_S11 + a) * tot + i] += dt * sv * W[k][i];
            }
        }
    }
    /* reverse sweep (bars of the memory variables start at zero with the fields') */
    for (i = 0; i < tot; ++i) {
        grad_lam[i] = 0.0;
        grad_mu[i] = 0.0;
        if (grad_b) grad_b[i] = 0.0;
    }
    dc[0].transpose = dc[1].transpose = dc[2].transpose = 1;
    for (n = nsteps - 1; n >= 0; --n) {
        const double *e = strain + (size_t)n * 6 * tot;
        for (r = 0; r < nrec; ++r) {
            long ix = rec_idx[3 * r], iy = rec_idx[3 * r + 1], iz = rec_idx[3 * r + 2];
            Fb[(size_t)rec_comp * tot + (iz * nn[1] + iy) * nn[0] + ix] += res[(size_t)r * nsteps + n];
        }
        for (half = 0; half < 2; ++half) {
            if (grad_b) {
                const double *dr = drive + (size_t)(2 * n + 1 - half) * 3 * tot;
                for (ci = 0; ci < 3; ++ci)
                    for (i = 0; i < tot; ++i)
                        grad_b[i] += dr[(size_t)ci * tot + i] * Fb[(size_t)(OR_E_V1 + ci) * tot + i];
            }
            /* transpose of a velocity half step */
            for (ci = 0; ci < 3; ++ci)
                for (cj = 0; cj < 3; ++cj) {
                    const flow_lin *L = &Lh[cj];
                    double *mb = bpsi + (size_t)(3 * ci + cj) * tot;
                    for (i = 0; i < tot; ++i) {
                        const long c[3] = {i % nn[0], i / nn[0] % nn[1], i / (nn[0] * nn[1])};
                        const long jj = c[cj];
                        const double t = -b[i] * Fb[(size_t)(OR_E_V1 + ci) * tot + i], m0 = mb[i];
                        t1[i] = L->Dv[jj] * t + L->Dp[jj] * m0;
                        mb[i] = L->Pv[jj] * t + L->Ep[jj] * m0;
                    }
                    apply_lines(g, cj, t1, t0, dense_op, &dc[cj], 0);
                    for (i = 0; i < tot; ++i) Fb[(size_t)sig_of[ci][cj] * tot + i] += t0[i];
                }
            if (half == 1) break;
            /* gradient with the stretched increments, then the transpose of the stress
             * sub-flow (increment bars from the stress bars, then each pass) */
            for (i = 0; i < tot; ++i) {
                double S = Fb[(size_t)OR_E_S11 * tot + i] + Fb[(size_t)OR_E_S22 * tot + i] + Fb[(size_t)OR_E_S33 * tot + i];
                double tr = e[i] + e[tot + i] + e[2 * (size_t)tot + i], m = 0.0;
                for (k = 0; k < 3; ++k) m += 2.0 * e[(size_t)k * tot + i] * Fb[(size_t)(OR_E_S11 + k) * tot + i];
                m += e[3 * (size_t)tot + i] * Fb[(size_t)OR_E_S12 * tot + i] + e[4 * (size_t)tot + i] * Fb[(size_t)OR_E_S13 * tot + i]
                   + e[5 * (size_t)tot + i] * Fb[(size_t)OR_E_S23 * tot + i];
                grad_lam[i] += tr * S;
                grad_mu[i] += m;
            }
            {
                int q;
                for (q = 0; q < 9; ++q) {
                    const int vi = q / 3, j = q % 3;
                    const flow_lin *L = &Lf[j];
                    double *mb = bphi + (size_t)q * tot;
                    for (i = 0; i < tot; ++i) {
                        const long c[3] = {i % nn[0], i / nn[0] % nn[1], i / (nn[0] * nn[1])};
                        const long jj = c[j];
                        double eb, t, m0 = mb[i];
                        if (vi == j) {
                            double S = Fb[(size_t)OR_E_S11 * tot + i] + Fb[(size_t)OR_E_S22 * tot + i]
                                     + Fb[(size_t)OR_E_S33 * tot + i];
                            eb = lam[i] * S + 2.0 * mu[i] * Fb[(size_t)(OR_E_S11 + vi) * tot + i];
                        } else {
                            eb = mu[i] * Fb[(size_t)sig_of[vi][j] * tot + i];
                        }
                        t = -eb;
                        t1[i] = L->Dv[jj] * t + L->Dp[jj] * m0;
                        mb[i] = L->Pv[jj] * t + L->Ep[jj] * m0;
                    }
                    apply_lines(g, j, t1, t0, dense_op, &dc[j], 0);
                    for (i = 0; i < tot; ++i) Fb[(size_t)(OR_E_V1 + vi) * tot + i] += t0[i];
                }
            }
        }
    }
    (void)shear;
    for (k = 0; k < nsrc; ++k) free(W[k]);
    free(W);
    free(strain);
    free(drive);
    free(F);
    for (a = 0; a < 3; ++a) { free(Dm[a]); free(Lh[a].Ep); free(Lf[a].Ep); }
    return 0;
}
