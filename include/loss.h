/*
 * loss.h -- C ABI of the MI355X local spline simulator (LOSS) of arXiv 2301.05127,
 * "Distributed local spline simulator for wave propagation" (Guo, Li, Xiong).
 *
 * The library (libloss.so, HIP for gfx950) owns all device memory.  Plain pointers
 * and sizes only; no C++ or framework types cross this boundary.  Every function
 * returns a status (0 = LOSS_OK, < 0 = error) and never throws; loss_last_error()
 * gives a thread-local message for the last failure.  A handle is not thread safe:
 * use one handle per thread / HIP stream.
 *
 * Memory arguments: `mem` = LOSS_MEM_HOST for host pointers (copied synchronously),
 * LOSS_MEM_DEVICE for device pointers on the simulation's device (used in stream
 * order on the simulation's stream; the caller keeps them alive until loss_sync).
 *
 * Field layout at the boundary: dense node arrays [z][y][x], x fastest, float32;
 * a 2-D grid uses axes x and z (n[1] = 0, one y node).  Internally rows are padded.
 *
 * Physics (paper Sec. 2):
 *   acoustic, eq. acoustic_wave:  dv1/dt = -b dsigma/dx, dv3/dt = -b dsigma/dz,
 *                                 dsigma/dt = -K (dv1/dx + dv3/dz),  K = rho c^2, b = 1/rho;
 *   elastic velocity-stress (Sec. 2): rho dv_i/dt = d_j sigma_ij + f_i,
 *                                 dsigma/dt = lambda tr(e) I + 2 mu e,  e = sym grad v,
 *                                 lambda = rho (Vp^2 - 2 Vs^2), mu = rho Vs^2.
 * Spatial derivatives (Sec. 3.1-3.2): patched cubic B-splines with the perfectly
 * matched boundary condition at patch junctions; time (Sec. 3.3): Strang splitting
 * of the velocity sub-flow (A) and the stress sub-flow (B), A(dt/2) B(dt) A(dt/2).
 * Outer ends: the end rows below (LOSS_END_*), optionally with the absorbing layer of
 * Sec. 3.3 on the outermost nodes (loss_set_pml).
 */
#ifndef LOSS_H
#define LOSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct loss_sim loss_sim;   /* opaque, library owned */
typedef int32_t loss_status;

#define LOSS_OK            0
#define LOSS_EINVAL       -1   /* bad argument (size, index, null pointer, kind) */
#define LOSS_ENOMEM       -2   /* device or host allocation failed */
#define LOSS_EHIP         -3   /* a HIP runtime call failed */
#define LOSS_ESTATE       -4   /* call out of order (e.g. step before set_media) */
#define LOSS_EUNSUPPORTED -5   /* valid request this build does not implement */
#define LOSS_EUNSTABLE    -6   /* dt above the stability bound, or a non-finite field */

/* physics */
#define LOSS_ACOUSTIC 0        /* 2-D (x, z) */
#define LOSS_ELASTIC  1        /* 3-D (x, y, z) */

/* End rows of the outermost patches:
 *  NATURAL       the global spline's natural row v~_{-1} - 2 v~_0 + v~_1 = 0 (Sec. 3.1,
 *                eq. natural_boundary), applied exactly;
 *  PAPER_STENCIL the truncated one-sided slope stencil that closes the first and last
 *                patch in Sec. 3.2 (the formulas after eq. PMBC_coeffcients);
 *  PERIODIC      node N is node 0; every junction, 0 = N included, uses the PMBC built
 *                from the circulant collocation matrix. */
#define LOSS_END_NATURAL       0
#define LOSS_END_PAPER_STENCIL 1
#define LOSS_END_PERIODIC      2

#define LOSS_MEM_HOST   0
#define LOSS_MEM_DEVICE 1

/* field ids: acoustic */
#define LOSS_F_SIGMA 0
#define LOSS_F_V1    1
#define LOSS_F_V3    2
/* field ids: elastic */
#define LOSS_F_EV1  0
#define LOSS_F_EV2  1
#define LOSS_F_EV3  2
#define LOSS_F_S11  3
#define LOSS_F_S22  4
#define LOSS_F_S33  5
#define LOSS_F_S12  6
#define LOSS_F_S13  7
#define LOSS_F_S23  8

/* source kinds (spatial amplitude A(x) times a time function, paper Sec. 4.3) */
#define LOSS_SRC_PRESSURE  0   /* rate added to sigma (acoustic) or sigma_ii (elastic) */
#define LOSS_SRC_EXPLOSIVE 1   /* same as PRESSURE */
#define LOSS_SRC_FORCE_X   2   /* body force f_1: dv1/dt += b f */
#define LOSS_SRC_FORCE_Y   3
#define LOSS_SRC_FORCE_Z   4

/* desc.flags */
#define LOSS_FLAG_NO_GRAPH 1   /* launch every step eagerly instead of replaying a hipGraph */
#define LOSS_FLAG_NO_FUSE_X 2  /* acoustic: keep the x velocity pass and the next step's x
                                  stress pass in separate kernels (by default one kernel
                                  runs both when a whole x line fits one workgroup and
                                  there are no body forces or velocity receivers) */
#define LOSS_FLAG_LINE_PASSES 4 /* elastic: one kernel per derivative along one axis (18 per
                                  step) instead of the plane schedule (per sub-flow: the z
                                  derivatives of its inputs, then one pass that solves the x
                                  and y lines of each patch tile of a plane from LDS and
                                  updates every output once); the plane schedule applies to
                                  x and y patches of at most 64 intervals without the
                                  absorbing layer */

typedef struct {
    int32_t physics;      /* LOSS_ACOUSTIC (ndim 2) or LOSS_ELASTIC (ndim 3) */
    int32_t ndim;         /* 2 or 3 */
    int64_t n[3];         /* intervals along x, y, z (nodes = n + 1); n[1] = 0 in 2-D */
    double h[3];          /* node spacing [m] per axis */
    double dt;            /* time step [s] */
    int32_t patch[3];     /* patch length M in intervals per axis; the last patch of an
                             axis takes the remainder n mod M */
    int32_t halo;         /* n_nb of the PMBC: taps j = -n_nb..n_nb around a junction */
    int32_t end_mode;     /* LOSS_END_* */
    int32_t nshots;       /* independent shots stepped together (same grid and media) */
    int32_t flags;        /* LOSS_FLAG_* */
    int64_t trace_len;    /* samples kept per receiver trace (0 = no traces) */
} loss_desc;

/* Create a simulation on the current HIP device.  `hip_stream` is a hipStream_t to
 * run on (NULL: the library creates its own).  Builds the per-axis PMBC and
 * tridiagonal factor tables in FP64 on the host (Sec. 3.2: truncated rows of the
 * inverse of the global collocation matrix) and stores them as float32.
 * Errors: LOSS_EINVAL for an inconsistent desc (ndim/physics mismatch, M < 1,
 * n < 2, halo < 1 or > 64, periodic with 2*halo+1 > n), LOSS_EUNSUPPORTED for a
 * patch length above 1024 or a per-shot field of 2^31 or more elements (the x extent
 * padded to a multiple of 4), LOSS_ENOMEM, LOSS_EHIP. */
loss_status loss_create(const loss_desc *desc, void *hip_stream, loss_sim **out);

/* Free every resource of the handle (NULL is accepted). */
loss_status loss_destroy(loss_sim *sim);

/* Media per node (dense [z][y][x]): vp (c_P), vs (c_S; NULL for acoustic), rho.
 * Derived on the device: acoustic K = rho vp^2, b = 1/rho; elastic lambda, mu, b.
 * Returns LOSS_EUNSTABLE (media kept) if dt exceeds the bound
 * 2 h_min / (sqrt(3) sqrt(ndim) max vp) of the Strang scheme with the spline symbol. */
loss_status loss_set_media(loss_sim *sim, const float *vp, const float *vs, const float *rho,
                           int32_t mem);

/* Add a source to `shot`.  pos: metres from node 0 along x, y, z.  spread_m > 0: a
 * Gaussian exp(-d^2 / (2 spread^2)) over nodes within 4 spread, normalised to unit
 * integral; spread_m == 0: weight 1/h^d at the nearest node.  wavelet (host, nt
 * samples): stress kinds use wavelet[n] in step n (sample it at t_n + dt/2); forces
 * use wavelet[k] = f(t_k) in the velocity half steps at t_n and t_{n+1}.  Samples
 * past nt are zero.  At most 16 sources per shot. */
loss_status loss_add_source(loss_sim *sim, int32_t shot, const double pos[3], int32_t kind,
                            const float *wavelet, int64_t nt, double spread_m);

/* Receivers (Sec. 4.3: the synthetic traces are the time series of a field sampled at
 * fixed nodes, there v_3 along a vertical line; Sec. 2 lists the wavefields and traces as
 * the outputs of the forward problem).
 * Add receivers to `shot`: node_idx (host) = nrec triples (ix, iy, iz).  After every
 * step n (counted from the last reset) sample n of each trace receives the field
 * `component` at t_{n+1} (acoustic: LOSS_F_SIGMA only; elastic: any field id),
 * accumulated in float64.  A velocity at t_{n+1} is the mean of the half-step-ahead
 * states on either side (exact for the Strang scheme, whose velocity sub-flow is linear
 * in its step; inside an absorbing layer the exact sub-flow is not, and a velocity
 * receiver there is off by the layer's second-order term, about 1e-4 relative).
 * Replaces earlier receivers of the shot. */
loss_status loss_add_receivers(loss_sim *sim, int32_t shot, int64_t nrec, const int32_t *node_idx,
                               int32_t component);

/* Zero every wavefield, trace, memory variable, the step counter and the non-finite
 * sentinel (media and sources are kept). */
loss_status loss_reset(loss_sim *sim);

/* Absorbing layer (paper Sec. 3.3: ADE-PML with the exponential operator splitting):
 * the outermost `width` nodes at both ends of every axis carry memory variables that
 * damp outgoing waves, one per spatial derivative of a sub-flow (acoustic: psi_x,
 * psi_z of the velocity sub-flow, phi_x, phi_z of the stress sub-flow; elastic, where
 * the paper's acoustic construction is applied to every derivative: 9 for the
 * d_j sigma_ij and 9 for the d_j v_i), each stretched by the profile of its own axis.
 * At depth fraction delta in (0, 1] into the layer:
 *   d = d0 delta^2, k = 1 + (kmax - 1) delta, alpha = pi f0 (1 - delta),
 *   d0 = -3 cmax ln(reflection) / (2 width h), cmax = the largest velocity of the
 * media set (call after loss_set_media; setting media again does not update d0).
 * Each sub-flow is solved exactly with its driving derivative frozen.  width = 0
 * removes the layer.  The memory variables (4 or 18 fields of device memory) start at
 * zero (and return to zero on loss_reset); the acoustic adjoint runs through the layer
 * (checkpoints carry the memory variables), the elastic one refuses it
 * (LOSS_EUNSUPPORTED).  Errors: LOSS_EINVAL (width < 0 or
 * > n/2 on an axis, reflection outside (0, 1), kmax < 1, f0 <= 0), LOSS_ESTATE (no
 * media yet). */
loss_status loss_set_pml(loss_sim *sim, int32_t width, double reflection, double kmax, double f0);

/* Advance all shots by nsteps Strang steps (Sec. 3.3), asynchronously on the sim stream.
 * Per step: stress sub-flow B(dt) then the velocity sub-flow, the two velocity half
 * steps of consecutive steps fused into one (the state holds the velocity half a
 * step ahead; loss_get_field returns it at the integer time).  Steps are replayed from
 * hipGraphs of 1, 2, 4, ..., 32 steps captured on the first call after a change of
 * configuration (LOSS_FLAG_NO_GRAPH: eager launches).
 * Non-finite sentinel: every 32 steps and at the end of each call, field 0 of every
 * shot (sigma; v1 when elastic) is checked for NaN or infinity on the device; the
 * result reaches the host without a wait, and once a check has seen one, loss_step and
 * loss_sync return LOSS_EUNSTABLE until loss_reset. */
loss_status loss_step(loss_sim *sim, int64_t nsteps);

/* Wavefields (the outputs of the forward problem, Sec. 2).
 * Copy one field of one shot at the current integer time into dst (nodes floats). */
loss_status loss_get_field(loss_sim *sim, int32_t shot, int32_t field, float *dst, int32_t mem);

/* Overwrite one field of one shot at the current integer time. */
loss_status loss_set_field(loss_sim *sim, int32_t shot, int32_t field, const float *src,
                           int32_t mem);

/* Receiver traces of one shot (Sec. 4.3): dst = nrec x trace_len doubles,
 * receiver-major; sample n holds the field at t_{n+1}. */
loss_status loss_get_traces(loss_sim *sim, int32_t shot, double *dst, int32_t mem);

/* Hot-path primitive: the patched spline derivative of order 1 (eq.
 * derivative_approximation) or 2 (second difference of the coefficients) along
 * axis 0 (x), 1 (y) or 2 (z) of `batch` dense fields in[batch][nodes] -> out.
 * The PMBC junction slopes come from a halo of n_nb nodes on each side.
 * order = -1 applies the transpose of the order-1 operator (used by the adjoint).
 * Any fused step state is converted back to integer time first. */
loss_status loss_deriv(loss_sim *sim, int32_t axis, int32_t order, const float *in, float *out,
                       int64_t batch, int32_t mem);

/* For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): loss_deriv on device arrays
 * (in, out: batch dense fields on the simulation's device, x fastest) that allocates
 * nothing.  Instead of the handle's temporaries its kernels stage the padded fields
 * in a library-static device array of LOSS_STATIC_SCRATCH_FLOATS floats (3 slots;
 * each GPU the library runs on holds its copy until the process ends), a slot's worth
 * of fields per pass (loss_create looks up the array's address on its device, which
 * is when the runtime sets the array up).  The work is queued on the simulation's stream (call loss_sync
 * before reading out).  The array is shared by every call on that GPU and keeps the
 * last call's contents: calls that overlap on one GPU (several handles, several
 * streams or threads) race; serialise them.  The handle's state is not touched.
 * Errors: LOSS_EINVAL (null pointer, axis, order, batch < 1, or one padded field of the
 * grid above the slot size LOSS_STATIC_SCRATCH_FLOATS / 3), LOSS_ESTATE (the current
 * device is not the simulation's), LOSS_EHIP. */
#define LOSS_STATIC_SCRATCH_FLOATS (3 * 18 * 1024 * 1024)
loss_status loss_deriv_static(loss_sim *sim, int32_t axis, int32_t order, const float *in, float *out,
                              int64_t batch);

/* Adjoint-state gradient (the discrete transpose of the Strang scheme of Sec. 3.3 applied
 * to the systems of Sec. 2; the paper states the forward problem only, the gradient is
 * the standard adjoint-state one).  loss_forward_ckpt resets, runs nsteps (<= trace_len) steps
 * from rest recording traces and keeping the state every ckpt_every steps in device
 * memory (3 fields per checkpoint acoustic, 9 elastic; with the absorbing layer the
 * checkpoint also carries its 4 (acoustic) or 18 (elastic) memory variables, and the
 * adjoint allocates 5 resp. 19 more fields for their bars and its operand: every pass
 * is transposed through its layer's exact sub-flow).  loss_adjoint then takes the trace
 * residual of J = 1/2 sum residual^2, laid out like the traces of all shots concatenated (residual[shot][rec][t], t < trace_len,
 * float64; samples t >= nsteps are ignored) and returns dJ/dparam summed over shots
 * (float64).  Acoustic: param = LOSS_GRAD_K (bulk modulus K) or LOSS_GRAD_VP (c with rho
 * fixed: 2 rho c dJ/dK), grad = nodes values.  Elastic: param = LOSS_GRAD_LAME
 * (grad = dJ/dlambda then dJ/dmu, 2 x nodes) or LOSS_GRAD_VPVS (dJ/dvp then dJ/dvs with
 * rho fixed, 2 x nodes); LOSS_GRAD_LAME_RHO / LOSS_GRAD_VPVS_RHO append dJ/drho (with
 * lambda, mu resp. vp, vs fixed; 3 x nodes).  The segment recompute keeps six strain
 * fields per step, nine with the density (6 or 9 x ckpt_every fields of device memory).  The adjoint applies the exact transpose
 * of every discrete operator of the time-stepping scheme; forward states are
 * recomputed from the checkpoints segment by segment.  Afterwards the wavefields hold
 * an intermediate state (call loss_reset).  Errors: LOSS_EUNSUPPORTED (patches shorter
 * than 2 intervals), LOSS_EINVAL (param not of the physics),
 * LOSS_ESTATE (no loss_forward_ckpt since the last loss_set_media or loss_set_pml: the
 * checkpoints must belong to the media and layer the adjoint runs with). */
#define LOSS_GRAD_K    0
#define LOSS_GRAD_VP   1
#define LOSS_GRAD_LAME 2
#define LOSS_GRAD_VPVS 3
#define LOSS_GRAD_LAME_RHO 4
#define LOSS_GRAD_VPVS_RHO 5
loss_status loss_forward_ckpt(loss_sim *sim, int64_t nsteps, int64_t ckpt_every);
loss_status loss_adjoint(loss_sim *sim, const double *residual, int32_t param, double *grad,
                         int32_t mem);

/* Autotune the launch shape of the line kernels: along x the nodes per lane (4, 8 or
 * 16) and, where every patch fills 16 lanes and the patches of a line come in fours, the
 * lines a wave solves in turn (1, 4, 8 or automatic); along y and z the columns per
 * wave (16, 32 or 64 x-columns; the rest of the wave's lanes take further chunks of the
 * same lines) and the nodes per lane (8 or 16), and for elastic grids the shape of the y
 * store passes apart (the axis's own, 64 or 32 columns with 8 nodes per lane); each
 * candidate timed over `trial_steps` steps, the fastest kept.  Elastic grids
 * that admit the plane schedule (LOSS_FLAG_LINE_PASSES) have it timed against the line
 * passes and the faster one kept.  A shape or schedule changes only how the carries of
 * the scan are grouped and the order in which derivative terms are summed
 * (rounding-level differences).  Wavefields, traces and the step counter are restored
 * afterwards. */
loss_status loss_autotune(loss_sim *sim, int32_t trial_steps);

/* The launch shape in use along `axis`: for x, 100 * lines per wave + nodes per lane
 * (lines per wave 0 = automatic: 16, 8, 4 or 2 where the kernel applies, as long as
 * that leaves 8192 waves; 1 = one unit per lane group); for y and z,
 * 100 * columns per wave + nodes per lane (0 = automatic choice); axis 3: the elastic
 * schedule in use (0 plane passes, 1 line passes); axes 4 and 5: the shape of the y and
 * z store passes (passes that only store a derivative), 0 when they take the axis's. */
loss_status loss_autotune_choice(loss_sim *sim, int32_t axis, int32_t *cw);

/* Set the launch shape along `axis` in the encoding of loss_autotune_choice
 * (x: 100 * {0, 1, 2, 4, 8, 16} + {4, 8, 16}; y/z: 100 * {8, 16, 32, 64} + {8, 16};
 * 0 = automatic; axis 3: 0 plane schedule where it applies, 1 line passes; axes 4, 5:
 * the y / z store passes, 100 * {8, 16, 32, 64} + {8, 16}, 0 = the axis's shape).
 * LOSS_EINVAL for any other value. */
loss_status loss_set_shape(loss_sim *sim, int32_t axis, int32_t shape);

/* Energy of the wavefield of every shot at the state's time (velocities at the same
 * integer time as loss_get_field returns them): the kinetic energy 1/2 rho |v|^2 plus the
 * strain energy 1/2 sigma : C^-1 : sigma of the velocity-stress system (Sec. 2; elastic,
 * isotropic: s:s / (4 mu) + (tr sigma)^2 / (18 K) with s the stress deviator and
 * K = lambda + 2 mu / 3; acoustic: sigma^2 / (2 K)), summed over the nodes times the cell
 * volume (h_x h_y h_z, or h_x h_z in 2-D).  Reduced on the device in FP64 in a fixed order
 * (repeated calls give the same bits).  energy: host array of nshots doubles.  Blocks until
 * done.  Errors: LOSS_EINVAL (null argument), LOSS_ESTATE (no media yet), LOSS_EHIP. */
loss_status loss_energy(loss_sim *sim, double *energy);

/* Wait for all work queued on the sim stream; LOSS_EUNSTABLE if the non-finite sentinel
 * (see loss_step) has fired. */
loss_status loss_sync(loss_sim *sim);

/* Per-kernel timing (for roofline accounting): when on, loss_step launches every
 * kernel eagerly between HIP events on the sim stream and accumulates each kernel
 * class's duration.  loss_kernel_timing returns the accumulated milliseconds and
 * launch count of class `id` and its name; LOSS_EINVAL past the last class. */
loss_status loss_set_timing(loss_sim *sim, int32_t on);
loss_status loss_kernel_timing(loss_sim *sim, int32_t id, double *ms, int64_t *launches,
                               const char **name);

/* Steps taken since the last reset. */
int64_t loss_current_step(const loss_sim *sim);

const char *loss_status_str(loss_status s);
const char *loss_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
