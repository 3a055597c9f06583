/*
 * loss_oracle.h -- plain FP64 CPU oracle of the local spline simulator (LOSS),
 * arXiv 2301.05127 (Guo, Li, Xiong), "Distributed local spline simulator for
 * wave propagation".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this code: only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no source with the HIP library.
 *
 * Every routine is a direct, unblocked, unfused transcription of what the paper
 * computes, in double precision, with plain loops.  Where the paper is garbled or
 * silent, the reading taken is stated at the routine.
 *
 * Layout of every field: nodes [z][y][x], x fastest, dense (no padding);
 * a 2-D grid uses axes x and z (n[1] == 0, one y node).
 */
#ifndef LOSS_ORACLE_H
#define LOSS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_END_NATURAL = 0, OR_END_PAPER_STENCIL = 1, OR_END_PERIODIC = 2 };
enum { OR_ACOUSTIC = 0, OR_ELASTIC = 1 };
/* acoustic fields: sigma (pressure), v1 (x velocity), v3 (z velocity) */
enum { OR_A_SIGMA = 0, OR_A_V1 = 1, OR_A_V3 = 2 };
/* elastic fields */
enum { OR_E_V1 = 0, OR_E_V2, OR_E_V3, OR_E_S11, OR_E_S22, OR_E_S33, OR_E_S12, OR_E_S13, OR_E_S23 };
/* source kinds */
enum { OR_SRC_PRESSURE = 0, OR_SRC_EXPLOSIVE = 1, OR_SRC_FORCE_X = 2, OR_SRC_FORCE_Y = 3,
       OR_SRC_FORCE_Z = 4 };

typedef struct {
    int ndim;        /* 2 (axes x,z) or 3 (x,y,z) */
    int n[3];        /* intervals per axis; nodes = n+1; n[1] = 0 for ndim == 2 */
    double h[3];     /* spacing [m] */
    int M[3];        /* patch length in intervals (last patch takes the remainder) */
    int halo;        /* n_nb of the perfectly matched boundary condition */
    int end_mode;    /* OR_END_* */
} or_grid;

typedef struct {
    int kind;              /* OR_SRC_* */
    double pos[3];         /* metres from node 0 along x, y, z */
    double spread;         /* Gaussian std [m]; 0 = point source at the nearest node */
    const double *wavelet; /* samples, see or_run */
    int nt;                /* number of samples */
} or_source;

/* ---- 1-D building blocks ------------------------------------------------ */

/* Solve the global cubic-spline system with natural end rows (paper, Sec. 3.1,
 * eq. spline_cofficient_eq): v[0..N] -> coefficients vt[0..N+2] = (v~_{-1}..v~_{N+1}). */
void or_global_spline(int N, double h, const double *v, double *vt);

/* Column k (0 <= k <= N) of b = A^{-1} of the global natural system, restricted to the
 * coefficient rows: out[i+1] = b_{i,k}, i = -1..N+1 (N+3 values). */
void or_global_inverse_column(int N, double h, int k, double *out);

/* Explicit LU factors of the local bordered matrix A_M (paper, eq. explicit_L/U):
 * d[1..M+2], l[1..M+1] (index 0 unused). Reading: the recursion l_i = 1/d_i,
 * d_{i+1} = 4 - l_i runs over i = 2..M (the printed upper limit M+1 contradicts the
 * closing formulas for l_{M+1}, d_{M+2}). */
void or_patch_lu(int M, double *d, double *l);

/* Coefficient row of the perfectly matched boundary condition for the derivative
 * at node J of an axis (paper, eq. PMBC / PMBC_coeffcients, and the global-end
 * stencils that follow them). Writes 2*halo+1 coefficients c[t] for tap node
 * idx[t] (t = 0..2n, offset t-n from J); taps outside the line get c = 0, idx = -1.
 * Returns 1 if node J carries such a row for the given end mode, else 0. */
int or_pmbc_row(int N, double h, int M, int halo, int end_mode, int J, double *c, int *idx);

/* Patched first and second derivative of one line u[0..N] (paper, Sec. 3.2):
 * per patch, the Hermite-bordered local system eq. spline_cofficient_eq_piece with
 * junction slopes from the truncated PMBC rows, then eq. derivative_approximation
 * for D1 and the second difference of the coefficients for D2.  d2 may be NULL. */
void or_line_deriv(int N, double h, int M, int halo, int end_mode, const double *u,
                   double *d1, double *d2);

/* Same, for every line of a field along axis a (0 = x, 1 = y, 2 = z). */
void or_field_deriv(const or_grid *g, int axis, int order, const double *in, double *out);

/* ---- time stepping ------------------------------------------------------ */

/* Source amplitude weights on the node grid (Gaussian of std `spread`, normalised to
 * unit integral, or a point weight 1/h^d): writes the full node field. */
void or_source_weights(const or_grid *g, const double pos[3], double spread, double *w);

/* Run one shot for nsteps Strang steps (paper, Sec. 3.3: half step of the velocity
 * sub-flow (A), full step of the stress sub-flow (B), half step of (A)), starting
 * from rest.  Media per node: vp, vs (elastic only; may be NULL for acoustic), rho.
 * Source time samples: pressure / explosive wavelet[n] is injected in step n
 * (sampled by the caller at t_n + dt/2); force wavelet[k] = f(t_k) is used by the
 * velocity half steps at t_n (first half) and t_{n+1} (second half).
 * Receivers: rec_idx[3*r + a] node index along axis a; after step n, trace[r*nsteps+n]
 * = the receiver component (acoustic: sigma; elastic: field id) at t_{n+1}.
 * fields (output, may be NULL): nfields x nodes, the state at t_nsteps.
 * Returns 0 on success. */
int or_run(const or_grid *g, int physics, double dt, int nsteps,
           const double *vp, const double *vs, const double *rho,
           int nsrc, const or_source *src,
           int nrec, const int *rec_idx, int rec_comp,
           double *fields, double *traces);

/* Same as or_run but starting from a given state (fields_in, nfields x nodes) at
 * step `step0` (the source sample index offset). */
int or_run_from(const or_grid *g, int physics, double dt, int step0, int nsteps,
                const double *vp, const double *vs, const double *rho,
                int nsrc, const or_source *src,
                int nrec, const int *rec_idx, int rec_comp,
                const double *fields_in, double *fields, double *traces);

/* ---- absorbing layer (paper, Sec. 3.3: ADE-PML with exponential splitting) -- */

/* Layer of `width` nodes at both ends of every axis.  At a node whose distance into
 * the layer is delta * width nodes (delta in (0, 1]; 0 outside the layer):
 *   d = d0 delta^2, k = 1 + (kmax - 1) delta, alpha = amax (1 - delta),
 *   d0 = -3 cmax ln(R) / (2 width h), amax = pi f0
 * (reading of the profile formulas after eq. ADE_PML_1: the exponent m = p = 1 applies
 * to delta, and L is the layer thickness in metres). */
typedef struct {
    int width;       /* nodes */
    double R;        /* target reflection coefficient */
    double kmax;     /* coordinate stretching at the outer edge */
    double f0;       /* dominant source frequency [Hz] */
    double cmax;     /* largest P velocity [m/s] */
} or_pml;

/* Exact flow over tau of one memory variable and its field with the driving
 * derivative D frozen (the sub-flow solutions of Sec. 3.3):
 *   psi' = -(d/k + alpha) psi - (d/k^2) D,   v' = -b (D/k + psi)
 * psi_out = psi(tau); dv_over_b = (v(tau) - v(0)) / b. */
void or_pml_flow(double d, double k, double alpha, double tau, double D, double psi,
                 double *psi_out, double *dv_over_b);

/* Acoustic 2-D run with the layer on both axes: like or_run_from, with the state
 * extended by the memory variables, fields (7 x nodes) = sigma, v1, v3, psi_x, psi_z,
 * phi_x, phi_z (psi: velocity sub-flow, phi: stress sub-flow; zero outside the layer).
 * Receivers record sigma.  Returns 0 on success. */
int or_run_pml(const or_grid *g, const or_pml *pml, double dt, int step0, int nsteps,
               const double *vp, const double *rho, int nsrc, const or_source *src,
               int nrec, const int *rec_idx, const double *fields_in, double *fields, double *traces);

/* Elastic 3-D run with the layer on all three axes: every derivative d_j f of the
 * elastic sub-flows is stretched with the profile of axis j.  fields (27 x nodes) =
 * the 9 elastic fields (OR_E_* order), psi[3i + j] (memory of d_j sigma_ij, velocity
 * sub-flow), phi[3i + j] (memory of d_j v_i, stress sub-flow).  Receivers record field
 * rec_comp.  Returns 0 on success. */
int or_run_pml_elastic(const or_grid *g, const or_pml *pml, double dt, int step0, int nsteps,
                       const double *vp, const double *vs, const double *rho, int nsrc, const or_source *src,
                       int nrec, const int *rec_idx, int rec_comp,
                       const double *fields_in, double *fields, double *traces);

/* Gradient of J = 1/2 sum_n sum_r (trace - obs)^2 of one acoustic 2-D shot with
 * respect to the bulk modulus K = rho c^2 at every node, given the residual
 * res[r*nsteps+n] = trace - obs.  Exact transpose of the discrete canonical Strang
 * scheme (every derivative operator transposed as a dense line matrix); the
 * forward states are kept in memory.  grad_K: nodes.  Returns 0 on success. */
int or_acoustic_adjoint(const or_grid *g, double dt, int nsteps,
                        const double *vp, const double *rho,
                        int nsrc, const or_source *src,
                        int nrec, const int *rec_idx,
                        const double *res, double *grad_K);

/* Dense matrix (N+1)x(N+1) of the patched first-derivative operator of one line
 * (column j = derivative of the unit vector e_j). */
void or_line_deriv_matrix(int N, double h, int M, int halo, int end_mode, double *D);

int or_num_fields(int physics);

/* Gradient of J = 1/2 sum_n sum_r (trace - obs)^2 of one elastic 3-D shot with respect to
 * the Lame parameters lambda and mu and (grad_b, if not null) the buoyancy b = 1/rho at
 * every node, given res[r*nsteps+n] = trace - obs for receivers of field rec_comp.
 * Exact transpose of the canonical Strang scheme (dense line matrices); forward
 * strains and velocity drives kept in memory.  Returns 0 on success. */
int or_elastic_adjoint(const or_grid *g, double dt, int nsteps,
                       const double *vp, const double *vs, const double *rho,
                       int nsrc, const or_source *src,
                       int nrec, const int *rec_idx, int rec_comp,
                       const double *res, double *grad_lam, double *grad_mu, double *grad_b);

/* Gradient dJ/dK of one acoustic 2-D shot run with the absorbing layer (or_run_pml's
 * sequence, memory variables starting at zero), J = 1/2 sum residual^2: the exact
 * transpose of every sub-flow, each linear in its frozen derivative and memory variable.
 * grad_K: nodes.  Returns 0 on success. */
/* Elastic Lame-parameter (and optionally buoyancy) gradients with the absorbing layer on
 * every axis: the transpose of or_run_pml_elastic's sequence, every pass through its
 * flow's linear form (Sec. 3.3).  grad_b may be NULL. */
int or_elastic_adjoint_pml(const or_grid *g, const or_pml *pml, double dt, int nsteps,
                           const double *vp, const double *vs, const double *rho,
                           int nsrc, const or_source *src,
                           int nrec, const int *rec_idx, int rec_comp,
                           const double *res, double *grad_lam, double *grad_mu, double *grad_b);

int or_acoustic_adjoint_pml(const or_grid *g, const or_pml *pml, double dt, int nsteps,
                            const double *vp, const double *rho, int nsrc, const or_source *src,
                            int nrec, const int *rec_idx, const double *res, double *grad_K);

#ifdef __cplusplus
}
#endif

#endif
