// C ABI of include/loss.h: buffer ownership, table upload, step orchestration,
// hipGraph capture and replay, sources, receivers, the adjoint driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/loss.h"
#include "loss_internal.h"

using namespace loss;

namespace {

thread_local std::string g_err;

loss_status fail(loss_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess)                                                          \
            return fail(LOSS_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

struct SrcHost {
    int kind;
    double pos[3];
    double spread;
    std::vector<float> wavelet;
};

struct RecHost {
    std::vector<int32_t> idx;  // nrec * 3
    int comp = 0;
};

// Kernel classes reported by loss_kernel_timing.
enum KClass {
    KC_STRESS_X, KC_STRESS_Y, KC_STRESS_Z, KC_VEL_X, KC_VEL_Y, KC_VEL_Z, KC_SOURCE, KC_RECEIVER,
    KC_ADVANCE, KC_ADJ_SOLVE, KC_ADJ_GATHER, KC_GRAD, KC_VEL_STRESS_X, KC_ADJ_X, KC_ADJ_XX, KC_STRESS_XY,
    KC_VEL_XY, KC_COUNT
};
const char *kKClassName[KC_COUNT] = {
    "stress_line_x", "stress_line_y", "stress_line_z", "velocity_line_x", "velocity_line_y",
    "velocity_line_z", "source_inject", "receiver_record", "step_advance", "adjoint_line_solve",
    "adjoint_gather", "gradient_accumulate", "velocity_stress_x", "adjoint_line_x", "adjoint_line_x_pair",
    "stress_plane_xy", "velocity_plane_xy"};

}  // namespace

struct loss_sim {
    loss_desc d{};
    hipStream_t st = nullptr;
    bool own_stream = false;
    int device = 0;
    int nf = 0, S = 0;
    int nx = 0, ny = 0, nz = 0;
    int64_t pitch = 0, plane = 0, shot_stride = 0, nodes = 0;
    std::vector<void *> allocs;
    std::vector<float *> f;        // nf fields [S][nz][ny][pitch]
    std::vector<float *> med;      // times dt: acoustic K, b; elastic lambda, mu, lambda+2mu, b
    float *tmp[3] = {nullptr, nullptr, nullptr};
    float **d_fields = nullptr;    // device copy of f
    float **d_tmpfields = nullptr; // device pointer table used for unfused velocity output
    AxisHost axh[3];
    AxisDev axd[3]{};
    bool media_set = false;
    bool fused = false;
    // sources
    std::vector<std::vector<SrcHost>> src;
    bool src_dirty = true;
    SrcDev *d_src = nullptr;
    int *d_src_begin = nullptr;    // [S+1]
    int cw[3] = {0, 0, 0};         // strided-kernel columns per wave per axis (0 = automatic)
    int cx = 0;                    // x-kernel nodes per lane (0 = automatic)
    int xl = 0;                    // x-kernel lines per wave over whole units (1: one; 0 = automatic)
    int cws[3] = {0, 0, 0};        // y/z store passes: columns per wave (0: the axis's shape)
    int css[3] = {0, 0, 0};        // y/z store passes: nodes per lane
    int cs[3] = {0, 0, 0};         // strided-kernel nodes per lane per axis (0 = automatic)
    int nsrc = 0;
    bool pending_inc = false;      // next line kernel advances the step counter
    float *d_wpool = nullptr, *d_wavpool = nullptr;
    // receivers
    std::vector<RecHost> rec;
    bool rec_dirty = true;
    RecDev *d_rec = nullptr;
    int nrec_total = 0;
    bool rec_has_vel = false, rec_has_stress = false;
    RecDev *d_rec_vel = nullptr, *d_rec_str = nullptr;
    int nrec_vel = 0, nrec_str = 0;
    // the same receivers grouped by target node for the adjoint's residual injection
    RecTarget *d_tgt_vel = nullptr, *d_tgt_str = nullptr;
    int64_t *d_toff_vel = nullptr, *d_toff_str = nullptr;
    int ntgt_vel = 0, ntgt_str = 0;
    // box [x0, x1) x [y0, y1) x [z0, z1) covering every force source's footprint
    int force_box[6] = {0, 0, 0, 0, 0, 0};
    std::vector<int64_t> rec_off;  // per shot trace offset
    double *traces = nullptr;
    int64_t trace_total = 0;
    // step counter
    int64_t *d_step = nullptr;
    int64_t step = 0;
    // non-finite sentinel: a device flag set when the checked field holds a NaN or an
    // infinity, copied in stream order into pinned host memory that the host reads
    // without waiting
    int *d_bad = nullptr;
    int *h_bad = nullptr;
    // graphs: gexec[k] replays 2^k steps (k = 0 .. kGraphLevels - 1), all built together
    static constexpr int kGraphLevels = 6;
    hipGraphExec_t gexec[kGraphLevels] = {};
    bool graphs_built = false;
    // timing
    bool timing = false;
    double kms[KC_COUNT] = {0};
    int64_t kcount[KC_COUNT] = {0};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // acoustic pressure receivers recorded by the z stress kernel: per flattened z
    // column {first, count, min row, max row}, then rows and trace offsets
    int4 *d_rcol = nullptr;
    int *d_rrow = nullptr;
    int64_t *d_rtoff = nullptr;
    // elastic schedule: 0 plane passes where they apply, 1 line passes (autotune's choice)
    int elastic_schedule = 0;
    // adjoint
    float *ckpt = nullptr;         // [nseg][nf fields][S][shot_stride] fused states
    int64_t ck_every = 0, ck_steps = 0, ck_nseg = 0;
    // per recomputed step, acoustic: div u; elastic: e11, e22, e33, g12, g13, g23
    float *divstore = nullptr;     // [ck_every][1, 6 or 9][S][shot_stride]
    int strain_slots = 6;          // elastic: strains, then the three velocity drives if 9
    int divstore_slots = 0;        // slots per step divstore was allocated with
    float *adj[4] = {nullptr, nullptr, nullptr, nullptr};   // lambda, mu1, mu3, Y scratch
    float *adj_el[11] = {};        // elastic: the 9 field bars (field order), Y scratch, operand
    float *adj_pml[5] = {};        // acoustic with the layer: the 4 memory-variable bars, operand
    float *adj_pml_el[19] = {};    // elastic with the layer: the 18 memory-variable bars, operand
    int ck_fields = 0;             // fields per checkpoint (the state, and the layer's variables)
    float **d_adjtab = nullptr;    // device copy of adj_el[0..8]
    double *grad_pad = nullptr, *grad_dense = nullptr, *res_dev = nullptr;
    float *d_vp = nullptr, *d_rho = nullptr;   // dense copies of the media for the gradient map
    float *d_vs = nullptr;
    double *energy_buf = nullptr;  // loss_energy: block partials [S][1024], then one value per shot
    double cmax = 0.0;                         // largest velocity of the media
    // absorbing layer: memory variables, each laid out like a field (acoustic: psi_x,
    // psi_z of the velocity sub-flow, phi_x, phi_z of the stress sub-flow; elastic:
    // 3i + j of d_j sigma_ij, then 9 + 3i + j of d_j v_i); per-axis coefficient tables
    float *pml_mem = nullptr;
    int npml = 0;
    float4 *pml_tab[3] = {nullptr, nullptr, nullptr};
    int pml_w = 0;

    template <class T>
    loss_status alloc(T **p, size_t count)
    {
        void *q = nullptr;
        if (count == 0) count = 1;
        hipError_t e = hipMalloc(&q, count * sizeof(T));
        if (e != hipSuccess) return fail(LOSS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        allocs.push_back(q);
        *p = (T *)q;
        return LOSS_OK;
    }
    void release(void *p)
    {
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) {
            (void)hipFree(p);
            allocs.erase(it);
        }
    }
};

namespace {

int64_t field_elems(const loss_sim *s) { return (int64_t)s->S * s->shot_stride; }

LineArgs base_args(const loss_sim *s, int axis)
{
    LineArgs a{};
    a.S = s->S;
    a.nx = s->nx; a.ny = s->ny; a.nz = s->nz;
    a.pitch = s->pitch; a.plane = s->plane; a.shot_stride = s->shot_stride;
    a.ax = s->axd[axis];
    a.nout = 1;
    a.cw = s->cw[axis];
    a.cx = s->cx;
    a.xl = s->xl;
    a.cs = s->cs[axis];
    return a;
}

// Memory variables of the absorbing layer: 0 psi_x, 1 psi_z (velocity sub-flow),
// 2 phi_x, 3 phi_z (stress sub-flow).
float *pml_var(const loss_sim *s, int k)
{
    return s->pml_mem ? s->pml_mem + (size_t)k * field_elems(s) : nullptr;
}

// Fractions of dt over which a pass advances the layer: full steps, the half step that
// opens the fused schedule, the half step back to the integer time.
constexpr float kPmlFrac[3] = {1.f, 0.5f, -0.5f};

// Point a pass along `axis` at memory variable k, advancing it over frac * dt (one of
// kPmlFrac; any other value is a programming error of this file).
void set_pml(const loss_sim *s, LineArgs &a, int axis, int k, float frac, bool store)
{
    a.pml_mem = pml_var(s, k);
    a.pml_tab = nullptr;
    a.pml_store = store ? 1 : 0;
    if (!a.pml_mem) return;
    int fi = -1;
    for (int i = 0; i < 3; ++i)
        if (frac == kPmlFrac[i]) fi = i;
    if (fi < 0) {
        std::fprintf(stderr, "loss: absorbing layer asked for an untabulated step fraction %g\n", (double)frac);
        std::abort();
    }
    a.pml_tab = s->pml_tab[axis] + (size_t)fi * (s->d.n[axis] + 1);
}

// 3-D axis index of the grid axis for a 2-D acoustic grid: (x, z) -> (0, 2).
int grid_axis_count(const loss_sim *s) { return s->d.ndim; }

loss_status timed_begin(loss_sim *s)
{
    if (s->timing) HIPCHK(hipEventRecord(s->ev0, s->st));
    return LOSS_OK;
}

loss_status timed_end(loss_sim *s, int kc)
{
    if (!s->timing) return LOSS_OK;
    HIPCHK(hipEventRecord(s->ev1, s->st));
    HIPCHK(hipEventSynchronize(s->ev1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    s->kms[kc] += ms;
    s->kcount[kc] += 1;
    return LOSS_OK;
}

loss_status run_line(loss_sim *s, int kc, int axis, int solve, int epi, const LineArgs &a0)
{
    LineArgs a = a0;
    if (s->pending_inc) {
        a.step_inc = s->d_step;
        s->pending_inc = false;
    }
    if (epi == EPI_STORE && axis > 0 && s->cws[axis]) {   // the store passes' own shape
        a.cw = s->cws[axis];
        a.cs = s->css[axis];
    }
    loss_status r = timed_begin(s);
    if (r) return r;
    hipError_t e = launch_line(axis, solve, epi, a, s->st);
    if (e != hipSuccess) return fail(LOSS_EHIP, std::string("line kernel launch: ") + hipGetErrorString(e));
    return timed_end(s, kc);
}

// Let the epilogue of a line kernel add the sources whose fields are among out_field.
// Stress sources are added as dt * s(t) * weight; body forces as (dt b) * f(t) * weight
// with dt b taken from the media array, so their scale is 1.
void attach_sources(const loss_sim *s, LineArgs &a, int time_offset, const int *out_field, int nout,
                    bool forces)
{
    if (s->nsrc == 0) return;
    a.src = s->d_src;
    a.src_begin = s->d_src_begin;
    a.wpool = s->d_wpool;
    a.wavpool = s->d_wavpool;
    a.bcoef = s->med.back();
    a.d_step = s->d_step;
    a.src_time_offset = time_offset;
    a.src_scale = forces ? 1.f : (float)s->d.dt;
    for (int j = 0; j < 3; ++j) a.out_field[j] = j < nout ? out_field[j] : -1;
}

// out (+)= alpha * D^T (in_coef * in) along axis: the transposed solve y = T^{-T} z on
// the patch interiors into Y, then G^T y (stencil, junction rows, transposed PMBC).
loss_status adj_deriv(loss_sim *s, int axis, const float *in, const float *in_coef, float *out,
                      float alpha, int epi, float *Y, int nshots)
{
    LineArgs x = base_args(s, 0);
    x.S = nshots;
    if (axis == 0 && !(s->d.flags & LOSS_FLAG_NO_FUSE_X) && line_xx_threads(x) > 0 &&
        (epi == EPI_STORE || epi == EPI_AXPY)) {
        // the whole line in one block: solve, junction rows and gather share y in LDS
        x.in = in;
        x.in_coef = in_coef;
        x.out[0] = out;
        x.alpha = alpha;
        loss_status r = timed_begin(s);
        if (r) return r;
        const hipError_t e = launch_adj_x(epi, x, s->st);
        if (e != hipSuccess) return fail(LOSS_EHIP, std::string("adjoint x: ") + hipGetErrorString(e));
        return timed_end(s, KC_ADJ_X);
    }
    LineArgs a = base_args(s, axis);
    a.S = nshots;
    a.in = in;
    a.in_coef = in_coef;
    a.out[0] = Y;
    loss_status r = run_line(s, KC_ADJ_SOLVE, axis, SOLVE_T1, EPI_STORE, a);
    if (r) return r;
    LineArgs g = base_args(s, axis);
    g.S = nshots;
    g.in = in;
    g.in_coef = in_coef;
    g.out[0] = out;
    g.alpha = alpha;
    if ((r = timed_begin(s))) return r;
    hipError_t e = launch_adj_junctions(axis, g, Y, s->st);
    if (e == hipSuccess) e = launch_adj_gather(axis, epi, g, Y, s->st);
    if (e != hipSuccess) return fail(LOSS_EHIP, std::string("adjoint gather: ") + hipGetErrorString(e));
    return timed_end(s, KC_ADJ_GATHER);
}

// mu1 += -Dx^T(K lam), then lam += -Dx^T(b mu1) with the updated mu1: one kernel when a
// whole x line fits a workgroup, else the two passes in that order (same arithmetic).
loss_status adj_x_pair(loss_sim *s, float *lam, const float *K, float *mu1, const float *b, float *Y, int nshots)
{
    LineArgs x = base_args(s, 0);
    x.S = nshots;
    x.in = lam;
    x.in_coef = K;
    x.out[0] = mu1;
    x.alpha = -1.f;
    if (!(s->d.flags & LOSS_FLAG_NO_FUSE_X) && line_xx_threads(x) > 0) {
        loss_status r = timed_begin(s);
        if (r) return r;
        const hipError_t e = launch_adj_xx(x, b, lam, -1.f, s->st);
        if (e != hipSuccess) return fail(LOSS_EHIP, std::string("adjoint x pair: ") + hipGetErrorString(e));
        return timed_end(s, KC_ADJ_XX);
    }
    loss_status r = adj_deriv(s, 0, lam, K, mu1, -1.f, EPI_AXPY, Y, nshots);
    if (r) return r;
    return adj_deriv(s, 0, mu1, b, lam, -1.f, EPI_AXPY, Y, nshots);
}

loss_status inject(loss_sim *s, float **fields_dev, int time_offset, float scale, int want_force)
{
    if (s->nsrc == 0) return LOSS_OK;
    loss_status r = timed_begin(s);
    if (r) return r;
    const float *b = s->med.back();
    hipError_t e = launch_inject(s->d_src, s->nsrc, fields_dev, b, s->d_wpool, s->d_wavpool, s->shot_stride,
                                 s->pitch, s->plane, s->d_step, time_offset, scale,
                                 want_force, s->st);
    if (e != hipSuccess) return fail(LOSS_EHIP, std::string("inject: ") + hipGetErrorString(e));
    return timed_end(s, KC_SOURCE);
}

// record one or two receiver lists into trace sample (*d_step - 1) (inside a step)
loss_status record(loss_sim *s, const RecDev *rec0, int nrec0, float w0, int acc0,
                   const RecDev *rec1 = nullptr, int nrec1 = 0, float w1 = 0.f, int acc1 = 0)
{
    if (nrec0 + nrec1 == 0 || s->d.trace_len == 0) return LOSS_OK;
    loss_status r = timed_begin(s);
    if (r) return r;
    hipError_t e = launch_record2(rec0, nrec0, w0, acc0, rec1, nrec1, w1, acc1, s->d_fields, s->shot_stride,
                                  s->traces, s->d_step, -1, s->d.trace_len, s->st);
    if (e != hipSuccess) return fail(LOSS_EHIP, std::string("record: ") + hipGetErrorString(e));
    return timed_end(s, KC_RECEIVER);
}

// ---- elastic plane schedule ------------------------------------------------------
// Per stage: three z passes store the z derivatives T of the stage's inputs, then the
// plane kernel adds the x and y derivatives from LDS tiles and updates every output
// once (see plane_xy.hip).  Used for elastic runs without the absorbing layer whose x
// and y patches are at most kPlaneMaxM long, unless the line-pass schedule is asked for.
bool plane_ok(const loss_sim *s)
{
    return s->d.physics == LOSS_ELASTIC && !s->pml_mem && !(s->d.flags & LOSS_FLAG_LINE_PASSES) &&
           s->elastic_schedule != 1 && s->d.patch[0] <= kPlaneMaxM && s->d.patch[1] <= kPlaneMaxM &&
           s->d.halo <= kPlaneMaxHalo;
}

PlaneArgs plane_args(const loss_sim *s)
{
    PlaneArgs p{};
    p.S = s->S;
    p.nx = s->nx; p.ny = s->ny; p.nz = s->nz;
    p.pitch = s->pitch; p.plane = s->plane; p.shot_stride = s->shot_stride;
    p.ax = s->axd[0];
    p.ay = s->axd[1];
    p.lam = s->med[0]; p.mu = s->med[1]; p.l2m = s->med[2]; p.b = s->med[3];
    for (int i = 0; i < 3; ++i) p.T[i] = s->tmp[i];
    return p;
}

loss_status run_plane(loss_sim *s, int kc, int mode, const PlaneArgs &p)
{
    loss_status r = timed_begin(s);
    if (r) return r;
    const hipError_t e = launch_plane_xy(mode, p, s->st);
    if (e != hipSuccess) return fail(LOSS_EHIP, std::string("plane kernel launch: ") + hipGetErrorString(e));
    return timed_end(s, kc);
}

// z derivatives of three fields into tmp[0..2] (the first kernel of a step when pending)
loss_status z_stores(loss_sim *s, int kc, const float *const *in)
{
    for (int i = 0; i < 3; ++i) {
        LineArgs z = base_args(s, 2);
        z.in = in[i];
        z.out[0] = s->tmp[i];
        loss_status r = run_line(s, kc, 2, SOLVE_D1, EPI_STORE, z);
        if (r) return r;
    }
    return LOSS_OK;
}

// stress sub-flow B(dt): T_i = d3 v_i, then the plane pass over the six stresses
loss_status stress_stage_planes(loss_sim *s)
{
    float *const *F = s->f.data();
    const float *v[3] = {F[LOSS_F_EV1], F[LOSS_F_EV2], F[LOSS_F_EV3]};
    loss_status r = z_stores(s, KC_STRESS_Z, v);
    if (r) return r;
    PlaneArgs p = plane_args(s);
    for (int i = 0; i < 3; ++i) p.in[i] = v[i];
    const int outs[6] = {LOSS_F_S11, LOSS_F_S22, LOSS_F_S33, LOSS_F_S12, LOSS_F_S13, LOSS_F_S23};
    for (int i = 0; i < 6; ++i) p.out[i] = F[outs[i]];
    p.alpha = 1.f;
    p.src = base_args(s, 0);
    const int fid[3] = {LOSS_F_S11, LOSS_F_S22, LOSS_F_S33};
    attach_sources(s, p.src, -1, fid, 3, false);
    return run_plane(s, KC_STRESS_XY, 0, p);
}

// velocity sub-flow over frac * dt: T_i = d3 sigma_i3, then the plane pass over v
loss_status velocity_stage_planes(loss_sim *s, float frac, float *const *vel, bool with_forces)
{
    float *const *F = s->f.data();
    const float *t3[3] = {F[LOSS_F_S13], F[LOSS_F_S23], F[LOSS_F_S33]};
    loss_status r = z_stores(s, KC_VEL_Z, t3);
    if (r) return r;
    PlaneArgs p = plane_args(s);
    const int ins[5] = {LOSS_F_S11, LOSS_F_S12, LOSS_F_S22, LOSS_F_S13, LOSS_F_S23};
    for (int i = 0; i < 5; ++i) p.in[i] = F[ins[i]];
    for (int i = 0; i < 3; ++i) p.out[i] = vel[i];
    p.alpha = frac;
    p.src = base_args(s, 0);
    if (with_forces) {
        const int fid[3] = {LOSS_F_EV1, LOSS_F_EV2, LOSS_F_EV3};
        attach_sources(s, p.src, 0, fid, 3, true);
    }
    return run_plane(s, KC_VEL_XY, 1, p);
}

// ---- velocity sub-flow (A) over frac * dt with the stress frozen -------------
// acoustic: v1 -= a b dsigma/dx, v3 -= a b dsigma/dz ; elastic: v_i += a b d_j sigma_ij
// `vel` are the velocity destinations (state or a temporary), `base` optional source
// for EPI_BASE on the first pass of each component.
loss_status velocity_stage(loss_sim *s, float frac, float *const *vel, const float *const *base,
                           bool with_forces = false, float *div_store = nullptr, int64_t div_shot_stride = 0)
{
    const float *b = s->med.back();
    loss_status r;
    if (s->d.physics == LOSS_ACOUSTIC) {
        const float *sig = s->f[LOSS_F_SIGMA];
        for (int c = 0; c < 2; ++c) {
            const int axis = c == 0 ? 0 : 2;
            LineArgs a = base_args(s, axis);
            a.in = sig;
            a.alpha = -frac;
            a.out[0] = vel[c];
            a.coef[0] = b;
            int epi = EPI_AXPY;
            if (base) { a.aux = base[c]; epi = EPI_BASE; }
            // the layer's memory variable advances with the state (an evaluation at
            // another time into a temporary leaves it unchanged)
            set_pml(s, a, axis, c, frac, base == nullptr);
            if (with_forces) {
                const int fid = c == 0 ? LOSS_F_V1 : LOSS_F_V3;
                attach_sources(s, a, 0, &fid, 1, true);
            }
            r = run_line(s, c == 0 ? KC_VEL_X : KC_VEL_Z, axis, SOLVE_D1, epi, a);
            if (r) return r;
        }
        return LOSS_OK;
    }
    // elastic: component i gets d_x sigma_{i1} + d_y sigma_{i2} + d_z sigma_{i3}
    static const int sidx[3][3] = {{LOSS_F_S11, LOSS_F_S12, LOSS_F_S13},
                                   {LOSS_F_S12, LOSS_F_S22, LOSS_F_S23},
                                   {LOSS_F_S13, LOSS_F_S23, LOSS_F_S33}};
    if (!base && !div_store && plane_ok(s)) return velocity_stage_planes(s, frac, vel, with_forces);
    if (!base) {
        // T = d_x sigma_{i1} (stored), T += d_y sigma_{i2}, v_i += frac b (T + d_z sigma_{i3})
        for (int i = 0; i < 3; ++i) {
            float *T = s->tmp[i];
            // with the layer each pass stores the stretched derivative and advances its
            // memory variable; the sum is still linear in the three
            LineArgs x = base_args(s, 0);
            x.in = s->f[sidx[i][0]];
            x.out[0] = T;
            set_pml(s, x, 0, 3 * i + 0, frac, true);
            if ((r = run_line(s, KC_VEL_X, 0, SOLVE_D1, EPI_STORE, x))) return r;
            LineArgs y = base_args(s, 1);
            y.in = s->f[sidx[i][1]];
            y.alpha = 1.f;
            y.out[0] = T;
            set_pml(s, y, 1, 3 * i + 1, frac, true);
            if ((r = run_line(s, KC_VEL_Y, 1, SOLVE_D1, EPI_AXPY, y))) return r;
            LineArgs z = base_args(s, 2);
            z.in = s->f[sidx[i][2]];
            z.alpha = frac;
            z.out[0] = vel[i];
            z.coef[0] = b;
            z.aux = T;
            set_pml(s, z, 2, 3 * i + 2, frac, true);
            if (div_store) {   // the drive sum_j d_j sigma_ij of v_i, for the buoyancy gradient
                z.div = div_store + i * field_elems(s);
                z.div_shot_stride = div_shot_stride;
            }
            if (with_forces) {
                const int fid = LOSS_F_EV1 + i;
                attach_sources(s, z, 0, &fid, 1, true);
            }
            if ((r = run_line(s, KC_VEL_Z, 2, SOLVE_D1, EPI_AXPY_AUX, z))) return r;
        }
        return LOSS_OK;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            LineArgs a = base_args(s, j);
            a.in = s->f[sidx[i][j]];
            a.alpha = frac;
            a.out[0] = vel[i];
            a.coef[0] = b;
            int epi = EPI_AXPY;
            if (base && j == 0) { a.aux = base[i]; epi = EPI_BASE; }
            set_pml(s, a, j, 3 * i + j, frac, base == nullptr);
            if (with_forces && j == 2) {
                const int fid = LOSS_F_EV1 + i;
                attach_sources(s, a, 0, &fid, 1, true);
            }
            r = run_line(s, KC_VEL_X + j, j, SOLVE_D1, epi, a);
            if (r) return r;
        }
    return LOSS_OK;
}

// ---- acoustic passes -----------------------------------------------------------
// T = d v1/dx into tmp[0]
loss_status acoustic_stress_x(loss_sim *s)
{
    LineArgs a = base_args(s, 0);
    a.in = s->f[LOSS_F_V1];
    a.out[0] = s->tmp[0];
    set_pml(s, a, 0, 2, 1.f, true);
    return run_line(s, KC_STRESS_X, 0, SOLVE_D1, EPI_STORE, a);
}

// sigma -= dt K (T + d v3/dz) (+ pressure sources); optional store of T + d v3/dz
loss_status acoustic_stress_z(loss_sim *s, float *div_store, int64_t div_shot_stride)
{
    LineArgs c = base_args(s, 2);
    c.in = s->f[LOSS_F_V3];
    c.out[0] = s->f[LOSS_F_SIGMA];
    c.coef[0] = s->med[0];
    c.aux = s->tmp[0];
    c.alpha = -1.f;
    c.div = div_store;
    c.div_shot_stride = div_shot_stride;
    set_pml(s, c, 2, 3, 1.f, true);
    const int fid = LOSS_F_SIGMA;
    attach_sources(s, c, -1, &fid, 1, false);
    if (s->d_rcol && s->d.trace_len > 0) {
        c.rcol = s->d_rcol;
        c.rrow = s->d_rrow;
        c.rtoff = s->d_rtoff;
        c.traces = s->traces;
        c.trace_len = s->d.trace_len;
    }
    return run_line(s, KC_STRESS_Z, 2, SOLVE_D1, EPI_AXPY_AUX, c);
}

// full velocity pass of component c (0: v1 along x, 1: v3 along z), no forces
loss_status acoustic_velocity(loss_sim *s, int c)
{
    const int axis = c == 0 ? 0 : 2;
    LineArgs a = base_args(s, axis);
    a.in = s->f[LOSS_F_SIGMA];
    a.alpha = -1.f;
    a.out[0] = s->f[c == 0 ? LOSS_F_V1 : LOSS_F_V3];
    a.coef[0] = s->med.back();
    set_pml(s, a, axis, c, 1.f, true);
    return run_line(s, c == 0 ? KC_VEL_X : KC_VEL_Z, axis, SOLVE_D1, EPI_AXPY, a);
}

// velocity pass along x of this step fused with the stress pass along x of the next
// one (which it opens: it advances the step counter)
loss_status acoustic_velocity_stress_x(loss_sim *s)
{
    LineArgs a = base_args(s, 0);
    a.in = s->f[LOSS_F_SIGMA];
    a.alpha = -1.f;
    a.out[0] = s->f[LOSS_F_V1];
    a.coef[0] = s->med.back();
    a.step_inc = s->d_step;
    set_pml(s, a, 0, 0, 1.f, true);
    s->pending_inc = false;
    loss_status r = timed_begin(s);
    if (r) return r;
    hipError_t e = launch_line_xx(a, s->tmp[0], pml_var(s, 2), s->st);
    if (e != hipSuccess) return fail(LOSS_EHIP, std::string("fused x kernel launch: ") + hipGetErrorString(e));
    return timed_end(s, KC_VEL_STRESS_X);
}

// The fused x schedule applies: acoustic, no body forces (the fused kernel's velocity
// half must not read the step counter it advances), no velocity receivers, a whole x
// line fits one block.
bool fused_x_ok(loss_sim *s)
{
    if (s->d.physics != LOSS_ACOUSTIC || s->nrec_vel > 0 || (s->d.flags & LOSS_FLAG_NO_FUSE_X)) return false;
    for (const auto &shot : s->src)
        for (const SrcHost &h : shot)
            if (h.kind >= LOSS_SRC_FORCE_X) return false;
    return line_xx_threads(base_args(s, 0)) > 0;
}

// ---- stress sub-flow (B) over dt with the velocity frozen --------------------
loss_status stress_stage(loss_sim *s, float *div_store, int64_t div_shot_stride)
{
    loss_status r;
    if (s->d.physics == LOSS_ACOUSTIC) {
        // T = d v1/dx ; sigma -= dt K (T + d v3/dz)
        if ((r = acoustic_stress_x(s))) return r;
        return acoustic_stress_z(s, div_store, div_shot_stride);
    }
    if (!div_store && plane_ok(s)) return stress_stage_planes(s);
    float *const *F = s->f.data();
    const float *lam = s->med[0], *mu = s->med[1], *l2m = s->med[2];
    // normal components: T1 = d1 v1 and T2 = d2 v2 stored, then the z pass updates all
    // three from T1, T2 and d3 v3: sigma_ii += (lambda + 2 mu) d_i v_i + lambda (sum of
    // the other two) (media hold dt lambda, dt mu, dt (lambda + 2 mu))
    // (with the layer every d_j v_i is stretched, memory variable 9 + 3i + j, and the
    // stress-strain law applies to the stretched derivatives)
    // (div_store, if given: six strain fields e11, e22, e33, g12, g13, g23 of this
    // step for the adjoint, field_elems apart)
    const int64_t fe = field_elems(s);
    for (int i = 0; i < 2; ++i) {
        LineArgs a = base_args(s, i);
        a.in = F[LOSS_F_EV1 + i];
        a.out[0] = s->tmp[i];
        set_pml(s, a, i, 9 + 4 * i, 1.f, true);
        if ((r = run_line(s, KC_STRESS_X + i, i, SOLVE_D1, EPI_STORE, a))) return r;
        if (div_store)
            HIPCHK(hipMemcpyAsync(div_store + i * fe, s->tmp[i], sizeof(float) * fe, hipMemcpyDeviceToDevice,
                                  s->st));
    }
    if (div_store) {
        // e33 as the pass below will see it: with the layer, the stretched derivative from
        // the current memory variable, which this evaluation leaves unchanged
        LineArgs a = base_args(s, 2);
        a.in = F[LOSS_F_EV3];
        a.out[0] = div_store + 2 * fe;
        set_pml(s, a, 2, 9 + 8, 1.f, false);
        if ((r = run_line(s, KC_STRESS_Z, 2, SOLVE_D1, EPI_STORE, a))) return r;
    }
    {
        LineArgs a = base_args(s, 2);
        a.in = F[LOSS_F_EV3];
        a.alpha = 1.f;
        a.nout = 3;
        a.out[0] = F[LOSS_F_S11]; a.out[1] = F[LOSS_F_S22]; a.out[2] = F[LOSS_F_S33];
        a.coef[0] = l2m;
        a.coef[1] = lam;
        a.aux = s->tmp[0];
        a.aux2 = s->tmp[1];
        set_pml(s, a, 2, 9 + 8, 1.f, true);
        const int fid[3] = {LOSS_F_S11, LOSS_F_S22, LOSS_F_S33};
        attach_sources(s, a, -1, fid, 3, false);
        if ((r = run_line(s, KC_STRESS_Z, 2, SOLVE_D1, EPI_NORMAL3, a))) return r;
    }
    // shear components: T = d_i v_j stored, then sigma_ij += dt mu (d_j v_i + T)
    static const int sh[3][3] = {{LOSS_F_S12, 0, 1}, {LOSS_F_S13, 0, 2}, {LOSS_F_S23, 1, 2}};
    for (int k = 0; k < 3; ++k) {
        const int i = sh[k][1], j = sh[k][2];
        LineArgs t = base_args(s, i);
        t.in = F[LOSS_F_EV1 + j];
        t.out[0] = s->tmp[k];
        set_pml(s, t, i, 9 + 3 * j + i, 1.f, true);
        if ((r = run_line(s, KC_STRESS_X + i, i, SOLVE_D1, EPI_STORE, t))) return r;
    }
    for (int k = 0; k < 3; ++k) {
        const int sij = sh[k][0], i = sh[k][1], j = sh[k][2];
        LineArgs a = base_args(s, j);
        a.in = F[LOSS_F_EV1 + i];
        a.alpha = 1.f;
        a.out[0] = F[sij];
        a.coef[0] = mu;
        a.aux = s->tmp[k];
        set_pml(s, a, j, 9 + 3 * i + j, 1.f, true);
        if (div_store) {
            a.div = div_store + (3 + k) * fe;
            a.div_shot_stride = div_shot_stride;
        }
        if ((r = run_line(s, KC_STRESS_X + j, j, SOLVE_D1, EPI_AXPY_AUX, a))) return r;
    }
    return LOSS_OK;
}

loss_status upload_sources(loss_sim *s)
{
    if (!s->src_dirty) return LOSS_OK;
    std::vector<SrcDev> sd;
    std::vector<float> wpool, wavpool;
    const int nax = s->d.ndim;
    const int axes[3] = {0, nax == 3 ? 1 : 2, 2};
    for (int shot = 0; shot < s->S; ++shot)
        for (const SrcHost &h : s->src[shot]) {
            SrcDev d{};
            d.shot = shot;
            d.kind = h.kind;
            d.force = h.kind >= LOSS_SRC_FORCE_X;
            if (d.force) {
                int comp = h.kind - LOSS_SRC_FORCE_X;   // 0 x, 1 y, 2 z
                if (s->d.physics == LOSS_ACOUSTIC) d.field0 = comp == 0 ? LOSS_F_V1 : LOSS_F_V3;
                else d.field0 = LOSS_F_EV1 + comp;
                d.nfield = 1;
            } else if (s->d.physics == LOSS_ACOUSTIC) {
                d.field0 = LOSS_F_SIGMA; d.nfield = 1;
            } else {
                d.field0 = LOSS_F_S11; d.nfield = 3;
            }
            // footprint box and Gaussian weights (unit integral)
            int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
            double hd = 1.0;
            for (int q = 0; q < nax; ++q) {
                const int ax = axes[q];
                const double hh = s->d.h[ax];
                hd *= hh;
                int c = (int)std::floor(h.pos[ax] / hh + 0.5);
                c = std::max(0, std::min((int)s->d.n[ax], c));
                int rad = h.spread > 0 ? (int)std::ceil(4.0 * h.spread / hh) : 0;
                lo[ax] = std::max(0, c - rad);
                hi[ax] = std::min((int)s->d.n[ax], c + rad);
            }
            d.x0 = lo[0]; d.y0 = lo[1]; d.z0 = lo[2];
            d.bx = hi[0] - lo[0] + 1; d.by = hi[1] - lo[1] + 1; d.bz = hi[2] - lo[2] + 1;
            std::vector<double> w((size_t)d.bx * d.by * d.bz);
            double sum = 0.0;
            for (int iz = 0; iz < d.bz; ++iz)
                for (int iy = 0; iy < d.by; ++iy)
                    for (int ix = 0; ix < d.bx; ++ix) {
                        double q = 1.0;
                        if (h.spread > 0) {
                            const double dx = (lo[0] + ix) * s->d.h[0] - h.pos[0];
                            const double dy = nax == 3 ? (lo[1] + iy) * s->d.h[1] - h.pos[1] : 0.0;
                            const double dz = (lo[2] + iz) * s->d.h[2] - h.pos[2];
                            q = std::exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * h.spread * h.spread));
                        }
                        w[((size_t)iz * d.by + iy) * d.bx + ix] = q;
                        sum += q;
                    }
            d.w_off = (int64_t)wpool.size();
            for (double q : w) wpool.push_back((float)(q / (sum * hd)));
            d.wav_off = (int64_t)wavpool.size();
            d.nt = (int)h.wavelet.size();
            wavpool.insert(wavpool.end(), h.wavelet.begin(), h.wavelet.end());
            sd.push_back(d);
        }
    for (int k = 0; k < 6; ++k) s->force_box[k] = 0;
    bool first_force = true;
    for (const SrcDev &d : sd) {
        if (!d.force) continue;
        const int lo[3] = {d.x0, d.y0, d.z0}, hi[3] = {d.x0 + d.bx, d.y0 + d.by, d.z0 + d.bz};
        for (int a = 0; a < 3; ++a) {
            s->force_box[2 * a] = first_force ? lo[a] : std::min(s->force_box[2 * a], lo[a]);
            s->force_box[2 * a + 1] = first_force ? hi[a] : std::max(s->force_box[2 * a + 1], hi[a]);
        }
        first_force = false;
    }
    std::vector<int> begin(s->S + 1, 0);
    for (const SrcDev &d : sd) begin[d.shot + 1]++;
    for (int k = 0; k < s->S; ++k) begin[k + 1] += begin[k];
    if (s->d_src_begin) { s->release(s->d_src_begin); s->d_src_begin = nullptr; }
    if (s->d_src) { s->release(s->d_src); s->d_src = nullptr; }
    if (s->d_wpool) { s->release(s->d_wpool); s->d_wpool = nullptr; }
    if (s->d_wavpool) { s->release(s->d_wavpool); s->d_wavpool = nullptr; }
    s->nsrc = (int)sd.size();
    if (s->nsrc) {
        loss_status r;
        if ((r = s->alloc(&s->d_src, sd.size()))) return r;
        if ((r = s->alloc(&s->d_wpool, wpool.size()))) return r;
        if ((r = s->alloc(&s->d_wavpool, wavpool.size()))) return r;
        HIPCHK(hipMemcpy(s->d_src, sd.data(), sd.size() * sizeof(SrcDev), hipMemcpyHostToDevice));
        if ((r = s->alloc(&s->d_src_begin, begin.size()))) return r;
        HIPCHK(hipMemcpy(s->d_src_begin, begin.data(), begin.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(s->d_wpool, wpool.data(), wpool.size() * sizeof(float), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(s->d_wavpool, wavpool.data(), wavpool.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    s->src_dirty = false;
    return LOSS_OK;
}

bool is_velocity(const loss_sim *s, int field)
{
    if (s->d.physics == LOSS_ACOUSTIC) return field == LOSS_F_V1 || field == LOSS_F_V3;
    return field <= LOSS_F_EV3;
}

loss_status upload_receivers(loss_sim *s)
{
    if (!s->rec_dirty) return LOSS_OK;
    std::vector<RecDev> vel, str;
    s->rec_off.assign(s->S, 0);
    int64_t off = 0;
    for (int shot = 0; shot < s->S; ++shot) {
        const RecHost &rh = s->rec[shot];
        s->rec_off[shot] = off;
        const int64_t nr = (int64_t)rh.idx.size() / 3;
        for (int64_t r = 0; r < nr; ++r) {
            RecDev d{};
            d.shot = shot;
            d.comp = rh.comp;
            const int64_t ix = rh.idx[3 * r], iy = rh.idx[3 * r + 1], iz = rh.idx[3 * r + 2];
            d.node = iz * s->plane + iy * s->pitch + ix;
            d.trace_off = off + r * s->d.trace_len;
            (is_velocity(s, rh.comp) ? vel : str).push_back(d);
        }
        off += nr * s->d.trace_len;
    }
    if (s->d_rec_vel) { s->release(s->d_rec_vel); s->d_rec_vel = nullptr; }
    if (s->d_rec_str) { s->release(s->d_rec_str); s->d_rec_str = nullptr; }
    if (s->d_rcol) { s->release(s->d_rcol); s->d_rcol = nullptr; }
    if (s->d_rrow) { s->release(s->d_rrow); s->d_rrow = nullptr; }
    if (s->d_rtoff) { s->release(s->d_rtoff); s->d_rtoff = nullptr; }
    if (s->traces) { s->release(s->traces); s->traces = nullptr; }
    loss_status r;
    s->nrec_vel = (int)vel.size();
    s->nrec_str = (int)str.size();
    if (s->nrec_vel) {
        if ((r = s->alloc(&s->d_rec_vel, vel.size()))) return r;
        HIPCHK(hipMemcpy(s->d_rec_vel, vel.data(), vel.size() * sizeof(RecDev), hipMemcpyHostToDevice));
    }
    if (s->nrec_str) {
        if ((r = s->alloc(&s->d_rec_str, str.size()))) return r;
        HIPCHK(hipMemcpy(s->d_rec_str, str.data(), str.size() * sizeof(RecDev), hipMemcpyHostToDevice));
    }
    // targets of the residual injection: receivers grouped by (shot, field, node), each
    // group in receiver order
    auto targets = [&](const std::vector<RecDev> &list, RecTarget **dt, int64_t **dtoff, int *nt) -> loss_status {
        if (*dt) { s->release(*dt); *dt = nullptr; }
        if (*dtoff) { s->release(*dtoff); *dtoff = nullptr; }
        std::vector<int> order(list.size());
        for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            const RecDev &x = list[a], &y = list[b];
            if (x.shot != y.shot) return x.shot < y.shot;
            if (x.comp != y.comp) return x.comp < y.comp;
            return x.node < y.node;
        });
        std::vector<RecTarget> tg;
        std::vector<int64_t> toff;
        for (int k : order) {
            const RecDev &d = list[k];
            if (tg.empty() || tg.back().shot != d.shot || tg.back().comp != d.comp || tg.back().node != d.node)
                tg.push_back(RecTarget{d.shot, d.comp, d.node, (int)toff.size(), 0});
            tg.back().count++;
            toff.push_back(d.trace_off);
        }
        *nt = (int)tg.size();
        if (tg.empty()) return LOSS_OK;
        loss_status q;
        if ((q = s->alloc(dt, tg.size())) || (q = s->alloc(dtoff, toff.size()))) return q;
        HIPCHK(hipMemcpy(*dt, tg.data(), tg.size() * sizeof(RecTarget), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(*dtoff, toff.data(), toff.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        return LOSS_OK;
    };
    if ((r = targets(vel, &s->d_tgt_vel, &s->d_toff_vel, &s->ntgt_vel))) return r;
    if ((r = targets(str, &s->d_tgt_str, &s->d_toff_str, &s->ntgt_str))) return r;
    // acoustic: the pressure receivers go to the z stress kernel, keyed by the
    // flattened z column (shot, y, x) of that kernel
    if (s->d.physics == LOSS_ACOUSTIC && !str.empty()) {
        const int64_t ncol = (int64_t)s->S * s->ny * s->pitch;
        std::vector<std::vector<std::pair<int, int64_t>>> bycol(ncol);
        for (const RecDev &d : str) {
            const int64_t z = d.node / s->plane, rem = d.node - z * s->plane;
            bycol[(int64_t)d.shot * s->ny * s->pitch + rem].push_back({(int)z, d.trace_off});
        }
        std::vector<int4> rcol(ncol, make_int4(0, 0, 0, -1));
        std::vector<int> rrow;
        std::vector<int64_t> rtoff;
        for (int64_t c = 0; c < ncol; ++c) {
            auto &v = bycol[c];
            if (v.empty()) continue;
            std::sort(v.begin(), v.end());
            rcol[c] = make_int4((int)rrow.size(), (int)v.size(), v.front().first, v.back().first);
            for (const auto &p : v) { rrow.push_back(p.first); rtoff.push_back(p.second); }
        }
        if ((r = s->alloc(&s->d_rcol, rcol.size())) || (r = s->alloc(&s->d_rrow, rrow.size())) ||
            (r = s->alloc(&s->d_rtoff, rtoff.size())))
            return r;
        HIPCHK(hipMemcpy(s->d_rcol, rcol.data(), rcol.size() * sizeof(int4), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(s->d_rrow, rrow.data(), rrow.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(s->d_rtoff, rtoff.data(), rtoff.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    }
    s->trace_total = off;
    if ((r = s->alloc(&s->traces, std::max<int64_t>(off, 1)))) return r;
    HIPCHK(hipMemsetAsync(s->traces, 0, sizeof(double) * std::max<int64_t>(off, 1), s->st));
    s->rec_dirty = false;
    return LOSS_OK;
}

void drop_graph(loss_sim *s)
{
    for (auto &g : s->gexec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    s->graphs_built = false;
}

// Convert (v at integer time) -> fused state (u half a step ahead), in place.
loss_status fuse(loss_sim *s)
{
    if (s->fused) return LOSS_OK;
    const float hdt = 0.5f;
    std::vector<float *> vel;
    if (s->d.physics == LOSS_ACOUSTIC) vel = {s->f[LOSS_F_V1], s->f[LOSS_F_V3]};
    else vel = {s->f[LOSS_F_EV1], s->f[LOSS_F_EV2], s->f[LOSS_F_EV3]};
    loss_status r = velocity_stage(s, hdt, vel.data(), nullptr);
    if (r) return r;
    r = inject(s, s->d_fields, 0, 0.5f, 1);
    if (r) return r;
    s->fused = true;
    return LOSS_OK;
}

// Velocity at the integer time from the fused state: v = u - (A half step), into tmp.
// Returns, per velocity component, the pointer that holds it.
loss_status unfused_velocity(loss_sim *s, std::vector<float *> &vout)
{
    std::vector<float *> vel;
    if (s->d.physics == LOSS_ACOUSTIC) vel = {s->f[LOSS_F_V1], s->f[LOSS_F_V3]};
    else vel = {s->f[LOSS_F_EV1], s->f[LOSS_F_EV2], s->f[LOSS_F_EV3]};
    if (!s->fused) { vout = vel; return LOSS_OK; }
    const int nv = (int)vel.size();
    std::vector<float *> dst(s->tmp, s->tmp + nv);
    std::vector<const float *> base(vel.begin(), vel.end());
    loss_status r = velocity_stage(s, -0.5f, dst.data(), base.data());
    if (r) return r;
    if (s->nsrc) {
        // forces: subtract the half-step force term, on a pointer table aimed at tmp
        std::vector<float *> tab(s->f.begin(), s->f.end());
        for (int c = 0; c < nv; ++c) {
            int fid = s->d.physics == LOSS_ACOUSTIC ? (c == 0 ? LOSS_F_V1 : LOSS_F_V3) : LOSS_F_EV1 + c;
            tab[fid] = dst[c];
        }
        HIPCHK(hipMemcpyAsync(s->d_tmpfields, tab.data(), sizeof(float *) * s->nf, hipMemcpyHostToDevice, s->st));
        r = inject(s, s->d_tmpfields, 0, -0.5f, 1);
        if (r) return r;
    }
    vout = dst;
    return LOSS_OK;
}

// Undo the fusion in place (before a user overwrites a field).
loss_status unfuse_in_place(loss_sim *s)
{
    if (!s->fused) return LOSS_OK;
    if (s->pml_mem) {
        // the layer's memory variables go back with the velocity: the exact velocity
        // sub-flow over -dt/2, in place
        std::vector<float *> vel;
        if (s->d.physics == LOSS_ACOUSTIC) vel = {s->f[LOSS_F_V1], s->f[LOSS_F_V3]};
        else vel = {s->f[LOSS_F_EV1], s->f[LOSS_F_EV2], s->f[LOSS_F_EV3]};
        loss_status r = velocity_stage(s, -0.5f, vel.data(), nullptr);
        if (r) return r;
        if ((r = inject(s, s->d_fields, 0, -0.5f, 1))) return r;
        s->fused = false;
        drop_graph(s);
        return LOSS_OK;
    }
    std::vector<float *> v;
    loss_status r = unfused_velocity(s, v);
    if (r) return r;
    const int nv = (int)v.size();
    for (int c = 0; c < nv; ++c) {
        int fid = s->d.physics == LOSS_ACOUSTIC ? (c == 0 ? LOSS_F_V1 : LOSS_F_V3) : LOSS_F_EV1 + c;
        HIPCHK(hipMemcpyAsync(s->f[fid], v[c], sizeof(float) * field_elems(s), hipMemcpyDeviceToDevice, s->st));
    }
    s->fused = false;
    drop_graph(s);
    return LOSS_OK;
}

// One fused step.  The first line kernel advances the step counter, so inside the
// step *d_step = n + 1: stress sources use sample n (offset -1, added in the stress
// epilogue), forces sample n + 1 (offset 0, velocity epilogue), traces slot n.
// Acoustic pressure receivers are recorded by the z stress kernel itself.
loss_status one_step(loss_sim *s, float *div_store, int64_t div_shot_stride)
{
    loss_status r;
    s->pending_inc = true;
    if ((r = stress_stage(s, div_store, div_shot_stride))) return r;
    // stress receivers not recorded by the stress kernel, and the first half of the
    // velocity receivers
    const int nstr = s->d_rcol ? 0 : s->nrec_str;
    if ((r = record(s, s->d_rec_str, nstr, 1.0f, 0, s->d_rec_vel, s->nrec_vel, 0.5f, 0))) return r;
    std::vector<float *> vel;
    if (s->d.physics == LOSS_ACOUSTIC) vel = {s->f[LOSS_F_V1], s->f[LOSS_F_V3]};
    else vel = {s->f[LOSS_F_EV1], s->f[LOSS_F_EV2], s->f[LOSS_F_EV3]};
    float *vdiv = (div_store && s->d.physics == LOSS_ELASTIC && s->strain_slots == 9)
                      ? div_store + 6 * field_elems(s) : nullptr;
    if ((r = velocity_stage(s, 1.0f, vel.data(), nullptr, true, vdiv, div_shot_stride))) return r;
    if ((r = record(s, s->d_rec_vel, s->nrec_vel, 0.5f, 1))) return r;
    return LOSS_OK;
}

// K acoustic steps with the x passes of consecutive steps fused (fused_x_ok):
//   stress_x(1); for n = 1..K: stress_z(n) (records the pressure receivers), vel_z(n),
//   then vel_x(n) + stress_x(n+1) fused (n < K) or vel_x(K).
// Each step's first kernel advances the step counter (stress_x or the fused kernel).
loss_status steps_fused_x(loss_sim *s, int64_t K, float *div_store, int64_t div_shot_stride)
{
    loss_status r;
    s->pending_inc = true;
    if ((r = acoustic_stress_x(s))) return r;
    for (int64_t n = 0; n < K; ++n) {
        float *ds = div_store ? div_store + n * s->S * div_shot_stride : nullptr;
        if ((r = acoustic_stress_z(s, ds, div_shot_stride))) return r;
        if (!s->d_rcol && (r = record(s, s->d_rec_str, s->nrec_str, 1.0f, 0))) return r;
        if ((r = acoustic_velocity(s, 1))) return r;
        r = (n + 1 < K) ? acoustic_velocity_stress_x(s) : acoustic_velocity(s, 0);
        if (r) return r;
    }
    return LOSS_OK;
}

// K steps on the stream, eagerly (no graph)
loss_status steps_eager(loss_sim *s, int64_t K, float *div_store = nullptr, int64_t div_shot_stride = 0)
{
    loss_status r;
    if (K > 0 && fused_x_ok(s)) return steps_fused_x(s, K, div_store, div_shot_stride);
    const int64_t nslot = s->d.physics == LOSS_ACOUSTIC ? 1 : s->strain_slots;
    for (int64_t done = 0; done < K; ++done) {
        float *ds = div_store ? div_store + done * nslot * s->S * div_shot_stride : nullptr;
        if ((r = one_step(s, ds, div_shot_stride))) return r;
    }
    return LOSS_OK;
}

loss_status ensure_ready(loss_sim *s)
{
    if (!s->media_set) return fail(LOSS_ESTATE, "loss_set_media must be called first");
    loss_status r;
    if ((r = upload_sources(s))) return r;
    if ((r = upload_receivers(s))) return r;
    return LOSS_OK;
}

// Queue the sentinel: every shot of field 0 (sigma, or v1 when elastic) checked for
// non-finite values; a NaN anywhere reaches every field within a step, since every
// derivative couples the nodes of a patch line.
loss_status queue_sentinel(loss_sim *s)
{
    if (launch_nonfinite(s->f[0], field_elems(s), s->d_bad, s->st) != hipSuccess)
        return fail(LOSS_EHIP, "non-finite check launch");
    HIPCHK(hipMemcpyAsync(s->h_bad, s->d_bad, sizeof(int), hipMemcpyDeviceToHost, s->st));
    return LOSS_OK;
}

// LOSS_EUNSTABLE once a queued check has seen a non-finite value
loss_status check_sentinel(const loss_sim *s)
{
    if (*(volatile int *)s->h_bad)
        return fail(LOSS_EUNSTABLE, "a wavefield holds NaN or infinity (the time step or the media may be "
                                    "unstable); loss_reset clears the state");
    return LOSS_OK;
}

// One graph per power of two up to 2^(kGraphLevels-1) steps, captured together the
// first time steps run on the current configuration: any step count is then replayed
// from at most a few graph launches and never captures inside a caller's timed loop.
loss_status build_graphs(loss_sim *s)
{
    drop_graph(s);
    for (int k = 0; k < loss_sim::kGraphLevels; ++k) {
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal));
        loss_status r = steps_eager(s, int64_t(1) << k);
        hipError_t e = hipStreamEndCapture(s->st, &g);
        if (r) { if (g) (void)hipGraphDestroy(g); drop_graph(s); return r; }
        if (e != hipSuccess) { drop_graph(s); return fail(LOSS_EHIP, std::string("graph capture: ") + hipGetErrorString(e)); }
        e = hipGraphInstantiate(&s->gexec[k], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            s->gexec[k] = nullptr;
            drop_graph(s);
            return fail(LOSS_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
    }
    s->graphs_built = true;
    return LOSS_OK;
}

loss_status run_steps(loss_sim *s, int64_t nsteps, float *div_store, int64_t div_shot_stride)
{
    loss_status r;
    if ((r = ensure_ready(s))) return r;
    if ((r = fuse(s))) return r;
    const bool use_graph = !(s->d.flags & LOSS_FLAG_NO_GRAPH) && !s->timing && div_store == nullptr;
    if (use_graph && nsteps > 0) {
        if (!s->graphs_built && (r = build_graphs(s))) return r;
        const int top = loss_sim::kGraphLevels - 1;
        int64_t left = nsteps;
        while (left >= (int64_t(1) << top)) {
            HIPCHK(hipGraphLaunch(s->gexec[top], s->st));
            left -= int64_t(1) << top;
            if (left > 0 && (r = queue_sentinel(s))) return r;
        }
        for (int k = top - 1; k >= 0; --k)
            if (left & (int64_t(1) << k)) HIPCHK(hipGraphLaunch(s->gexec[k], s->st));
    } else if ((r = steps_eager(s, nsteps, div_store, div_shot_stride))) {
        return r;
    }
    if (nsteps > 0 && (r = queue_sentinel(s))) return r;
    s->step += nsteps;
    return LOSS_OK;
}

loss_status copy_field_in(loss_sim *s, float *dst_padded, const float *src_dense, int mem, int64_t batch)
{
    const int64_t dense = (int64_t)s->nx * s->ny * s->nz;
    const float *src = src_dense;
    float *staging = nullptr;
    if (mem == LOSS_MEM_HOST) {
        loss_status r = s->alloc(&staging, dense * batch);
        if (r) return r;
        HIPCHK(hipMemcpyAsync(staging, src_dense, sizeof(float) * dense * batch, hipMemcpyHostToDevice, s->st));
        src = staging;
    }
    hipError_t e = launch_pad_copy(src, dst_padded, s->nx, (int)(batch * s->ny * s->nz), s->pitch, 1, s->st);
    if (staging) { (void)hipStreamSynchronize(s->st); s->release(staging); }
    if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
    return LOSS_OK;
}

loss_status copy_field_out(loss_sim *s, float *dst_dense, const float *src_padded, int mem, int64_t batch)
{
    const int64_t dense = (int64_t)s->nx * s->ny * s->nz;
    float *dst = dst_dense;
    float *staging = nullptr;
    if (mem == LOSS_MEM_HOST) {
        loss_status r = s->alloc(&staging, dense * batch);
        if (r) return r;
        dst = staging;
    }
    hipError_t e = launch_pad_copy(src_padded, dst, s->nx, (int)(batch * s->ny * s->nz), s->pitch, 0, s->st);
    if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
    if (staging) {
        HIPCHK(hipMemcpyAsync(dst_dense, staging, sizeof(float) * dense * batch, hipMemcpyDeviceToHost, s->st));
        HIPCHK(hipStreamSynchronize(s->st));
        s->release(staging);
    }
    return LOSS_OK;
}

loss_status upload_axis(loss_sim *s, int axis)
{
    const AxisHost &h = s->axh[axis];
    const int n = h.N + 1, np = n + kTabPad;
    // the line kernels derive the PMBC slots of a patch from its index
    for (int l = 0; l < h.p; ++l) {
        const int st = l * h.M, e = std::min(st + h.M, h.N);
        const int ss = h.end_mode == LOSS_END_NATURAL ? l - 1 : l;
        const int se = e == h.N ? (h.end_mode == LOSS_END_NATURAL ? -1 : h.p)
                                : (h.end_mode == LOSS_END_NATURAL ? l : l + 1);
        if (h.slot[st] != ss || h.slot[e] != se) return fail(LOSS_EINVAL, "internal: junction slot order");
    }
    std::vector<float4> lu(n), rc(n), luT(np, make_float4(0.f, 1.f, 0.f, 0.f)), lu2(n);
    std::vector<float2> lu2c(n), lum(np, make_float2(0.f, 1.f)), lum2(np, make_float2(0.f, 1.f));
    for (int i = 0; i < n; ++i) {
        lu[i] = make_float4((float)h.m[i], (float)h.invd[i], (float)h.sup[i], (float)h.kind[i]);
        rc[i] = make_float4((float)h.cm[i], (float)h.c0[i], (float)h.cp[i], (float)h.slot[i]);
        luT[i] = make_float4((float)h.mT[i], (float)h.invdT[i], (float)h.supT[i], (float)h.subT[i]);
        lu2[i] = make_float4((float)h.m2[i], (float)h.invd2[i], (float)h.sup2[i], 0.f);
        lu2c[i] = make_float2((float)h.m2c[i], (float)h.invd2c[i]);
        lum[i] = make_float2((float)h.m[i], (float)h.invd[i]);
        lum2[i] = make_float2((float)h.m2[i], (float)h.invd2[i]);
    }
    // at least one slot of taps: the kernels read slot 0 even on a line without junctions
    std::vector<float> tc(std::max<size_t>(h.tap_c.size(), 2 * h.halo + 1), 0.f), gc(h.g_c.begin(), h.g_c.end());
    // column j of the stencil part of G (junction rows of G are zero)
    std::vector<float4> adjw(n);
    for (int j = 0; j < n; ++j)
        adjw[j] = make_float4(j > 0 ? (float)h.cp[j - 1] : 0.f, (float)h.c0[j], j < h.N ? (float)h.cm[j + 1] : 0.f, 0.f);
    // columns of the plain interior form, without transposed PMBC taps (the gather
    // reads no table for them)
    const float s3f = (float)(3.0 / h.h);
    const float4 plain4 = make_float4(s3f, 0.f, -s3f, 0.f);
    std::vector<unsigned> plain((n + 31) / 32, 0u);
    for (int j = 0; j < n; ++j) {
        bool ok = adjw[j].x == plain4.x && adjw[j].y == plain4.y && adjw[j].z == plain4.z;
        for (int t = 0; t < h.gmax; ++t) ok = ok && h.g_node[(size_t)j * h.gmax + t] < 0;
        if (ok) plain[j >> 5] |= 1u << (j & 31);
    }
    std::vector<SpecialCol> spec;
    for (int j = 0; j < n; ++j) {
        if ((plain[j >> 5] >> (j & 31)) & 1u) continue;
        SpecialCol sc{};
        sc.aw = adjw[j];
        sc.row = j;
        spec.push_back(sc);
    }
    unsigned *dplain;
    SpecialCol *dspec;
    float4 *dadjw;
    std::copy(h.tap_c.begin(), h.tap_c.end(), tc.begin());
    float4 *dlu, *drc, *dluT, *dlu2;
    float2 *dlu2c, *dlum, *dlum2;
    int *dti, *dgn;
    float *dtc, *dgc;
    loss_status r;
    if ((r = s->alloc(&dlu, n)) || (r = s->alloc(&drc, n)) || (r = s->alloc(&dluT, np)) ||
        (r = s->alloc(&dlu2, n)) || (r = s->alloc(&dlu2c, n)) || (r = s->alloc(&dlum, np)) ||
        (r = s->alloc(&dlum2, np)) ||
        (r = s->alloc(&dti, std::max<size_t>(1, h.tap_idx.size()))) ||
        (r = s->alloc(&dtc, tc.size())) ||
        (r = s->alloc(&dgn, h.g_node.size())) || (r = s->alloc(&dgc, gc.size())) || (r = s->alloc(&dadjw, n)) ||
        (r = s->alloc(&dplain, plain.size())) || (r = s->alloc(&dspec, std::max<size_t>(1, spec.size()))))
        return r;
    if (!spec.empty())
        HIPCHK(hipMemcpy(dspec, spec.data(), spec.size() * sizeof(SpecialCol), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dplain, plain.data(), plain.size() * sizeof(unsigned), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dlu, lu.data(), n * sizeof(float4), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(drc, rc.data(), n * sizeof(float4), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dluT, luT.data(), np * sizeof(float4), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dlu2, lu2.data(), n * sizeof(float4), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dlu2c, lu2c.data(), n * sizeof(float2), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dlum, lum.data(), np * sizeof(float2), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dlum2, lum2.data(), np * sizeof(float2), hipMemcpyHostToDevice));
    if (!h.tap_idx.empty())
        HIPCHK(hipMemcpy(dti, h.tap_idx.data(), h.tap_idx.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dtc, tc.data(), tc.size() * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dgn, h.g_node.data(), h.g_node.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dadjw, adjw.data(), n * sizeof(float4), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dgc, gc.data(), gc.size() * sizeof(float), hipMemcpyHostToDevice));
    AxisDev &d = s->axd[axis];
    d.N = h.N; d.M = h.M; d.p = h.p; d.ntap = 2 * h.halo + 1; d.h = (float)h.h;
    d.s3 = (float)(3.0 / h.h);
    d.halo = h.halo;
    d.periodic = h.end_mode == LOSS_END_PERIODIC;
    d.ends = h.end_mode;
    d.reach = h.reach;
    d.lum = dlum; d.lum2 = dlum2;
    d.lu = dlu; d.rc = drc; d.luT = dluT; d.lu2 = dlu2; d.lu2c = dlu2c;
    d.tap_idx = dti; d.tap_c = dtc; d.g_node = dgn; d.g_c = dgc; d.gmax = h.gmax; d.adjw = dadjw;
    d.plain = dplain; d.adjw_plain = plain4;
    d.spec = dspec; d.nspec = (int)spec.size();
    return LOSS_OK;
}


// Elastic adjoint of the fused schedule that loss_forward_ckpt ran.  Forward step n:
//   B: sigma += (dt lambda) tr(e) I + 2 (dt mu) e, strains e of u^n; stress receivers
//      record sigma, velocity receivers half of u^n (the half-step-ahead state);
//   A: u_i += (dt b) sum_j D_j sigma_ij (+ forces); velocity receivers add half of the new u.
// Reverse step n (bars: adjoints of the fields after step n; the initial half step and
// the sources carry no parameter):
//   ubar += residual / 2 (velocity receivers); sigma_ij bar += D_j^T((dt b) u_i bar) for
//   every (i, j); sigma bar += residual (stress receivers); ubar += residual / 2;
//   dJ/dlambda, dJ/dmu from the stored strains of u^n and the stress bars; then
//   u_k bar += D_k^T(dt(lambda + 2 mu) sbar_kk + dt lambda (other normal bars)) and, per
//   shear pair i < j, u_i bar += D_j^T((dt mu) sbar_ij), u_j bar += D_i^T((dt mu) sbar_ij).
loss_status elastic_adjoint(loss_sim *s, const double *residual, int32_t param, double *grad, int32_t mem)
{
    if (param != LOSS_GRAD_LAME && param != LOSS_GRAD_VPVS && param != LOSS_GRAD_LAME_RHO &&
        param != LOSS_GRAD_VPVS_RHO)
        return fail(LOSS_EINVAL, "elastic gradients are LOSS_GRAD_LAME, LOSS_GRAD_VPVS or their _RHO forms");
    const bool want_b = param == LOSS_GRAD_LAME_RHO || param == LOSS_GRAD_VPVS_RHO;
    loss_status r;
    const int64_t fe = field_elems(s), ss = s->shot_stride;
    const int S = s->S;
    const int slots = want_b ? 9 : 6;
    if (s->divstore && s->divstore_slots < slots) { s->release(s->divstore); s->divstore = nullptr; }
    for (int k = 0; k < 11; ++k)
        if (!s->adj_el[k] && (r = s->alloc(&s->adj_el[k], fe))) return r;
    if (!s->d_adjtab) {
        if ((r = s->alloc(&s->d_adjtab, 9))) return r;
        HIPCHK(hipMemcpy(s->d_adjtab, s->adj_el, sizeof(float *) * 9, hipMemcpyHostToDevice));
    }
    if (!s->divstore) {
        if ((r = s->alloc(&s->divstore, (size_t)(slots * s->ck_every * fe)))) return r;
        s->divstore_slots = slots;
    }
    s->strain_slots = slots;
    if (!s->grad_pad && (r = s->alloc(&s->grad_pad, 3 * ss))) return r;
    if (!s->grad_dense && (r = s->alloc(&s->grad_dense, 3 * s->nodes))) return r;
    if (!s->res_dev && (r = s->alloc(&s->res_dev, std::max<int64_t>(1, s->trace_total)))) return r;
    if (s->trace_total > 0)
        HIPCHK(hipMemcpyAsync(s->res_dev, residual, sizeof(double) * s->trace_total,
                              mem == LOSS_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s->st));
    for (int k = 0; k < 9; ++k)
        if (launch_fill(s->adj_el[k], fe, 0.f, s->st) != hipSuccess) return fail(LOSS_EHIP, "fill");
    // with the layer: the bars of its 18 memory variables (0..8 psi_ij of the velocity
    // passes d_j sigma_ij, 9..17 phi_ij of the stress passes d_j v_i, numbered 3i + j as
    // in the forward), zero after the last step, and the operand of each pass
    const bool layer = s->pml_mem != nullptr;
    if (layer) {
        for (int k = 0; k < 19; ++k)
            if (!s->adj_pml_el[k] && (r = s->alloc(&s->adj_pml_el[k], fe))) return r;
        for (int k = 0; k < 18; ++k)
            if (launch_fill(s->adj_pml_el[k], fe, 0.f, s->st) != hipSuccess) return fail(LOSS_EHIP, "fill");
    }
    HIPCHK(hipMemsetAsync(s->grad_pad, 0, sizeof(double) * 3 * ss, s->st));
    double *gb = s->grad_pad + 2 * ss;
    float *const *A = s->adj_el;
    float *Y = s->adj_el[9], *Wop = s->adj_el[10];
    const float *lam = s->med[0], *mu = s->med[1], *l2m = s->med[2], *b = s->med[3];
    static const int sidx[3][3] = {{LOSS_F_S11, LOSS_F_S12, LOSS_F_S13},
                                   {LOSS_F_S12, LOSS_F_S22, LOSS_F_S23},
                                   {LOSS_F_S13, LOSS_F_S23, LOSS_F_S33}};
    static const int sh[3][3] = {{LOSS_F_S12, 0, 1}, {LOSS_F_S13, 0, 2}, {LOSS_F_S23, 1, 2}};
    const float *sbar[6] = {A[LOSS_F_S11], A[LOSS_F_S22], A[LOSS_F_S33], A[LOSS_F_S12], A[LOSS_F_S13],
                            A[LOSS_F_S23]};
    auto inject_res = [&](bool vel, int64_t n, float w) -> loss_status {
        const int nt = vel ? s->ntgt_vel : s->ntgt_str;
        if (nt == 0) return LOSS_OK;
        loss_status q = timed_begin(s);
        if (q) return q;
        const hipError_t e = launch_res_gather(vel ? s->d_tgt_vel : s->d_tgt_str, nt, vel ? s->d_toff_vel : s->d_toff_str,
                                               s->d_adjtab, nullptr, ss, s->res_dev, n, w, s->st);
        if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
        return timed_end(s, KC_RECEIVER);
    };
    // one transposed pass: target += D_axis^T (coef fbar), through the layer's flow of the
    // pass's memory variable mv when there is one (its bar updated in place)
    auto pass_t = [&](int axis, const float *fbar, const float *coef, int mv, float *target) -> loss_status {
        if (!layer) return adj_deriv(s, axis, fbar, coef, target, 1.f, EPI_AXPY, Y, S);
        loss_status q = timed_begin(s);
        if (q) return q;
        float *Wl = s->adj_pml_el[18];
        const hipError_t e = launch_pml_adj_operand(Wl, fbar, coef, 1.f, s->adj_pml_el[mv], s->pml_tab[axis], axis,
                                                    s->pml_w, (int)s->d.n[axis], s->nx, s->ny, s->pitch, ss, S, s->st);
        if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
        if ((q = timed_end(s, KC_GRAD))) return q;
        return adj_deriv(s, axis, Wl, nullptr, target, 1.f, EPI_AXPY, Y, S);
    };
    for (int64_t c = s->ck_nseg - 1; c >= 0; --c) {
        const int64_t n0 = c * s->ck_every, nc = std::min(s->ck_every, s->ck_steps - n0);
        // restore the fused state at step n0 (with the layer's memory variables) and
        // recompute the segment, keeping the strains
        for (int k = 0; k < s->nf; ++k)
            HIPCHK(hipMemcpyAsync(s->f[k], s->ckpt + (c * s->ck_fields + k) * fe, sizeof(float) * fe,
                                  hipMemcpyDeviceToDevice, s->st));
        if (layer)
            HIPCHK(hipMemcpyAsync(s->pml_mem, s->ckpt + (c * s->ck_fields + s->nf) * fe,
                                  sizeof(float) * s->npml * fe, hipMemcpyDeviceToDevice, s->st));
        HIPCHK(launch_set_step(s->d_step, n0, s->st));
        s->fused = true;
        if ((r = steps_eager(s, nc, s->divstore, ss))) return r;
        for (int64_t k = nc - 1; k >= 0; --k) {
            const int64_t n = n0 + k;
            if ((r = inject_res(true, n, 0.5f))) return r;
            if (want_b) {
                // the velocity step of step n drove u with (dt b)(sum_j D_j sigma_ij + f(t_{n+1}) w)
                const float *ub[3] = {A[LOSS_F_EV1], A[LOSS_F_EV2], A[LOSS_F_EV3]};
                const float *dv[3];
                for (int q = 0; q < 3; ++q) dv[q] = s->divstore + (k * slots + 6 + q) * fe;
                if ((r = timed_begin(s))) return r;
                hipError_t e = launch_el_grad_b(gb, ub, dv, s->d.dt, s->nx, s->pitch, ss, S, s->st);
                if (e == hipSuccess)
                    e = launch_el_grad_force(gb, s->d_src, s->nsrc, s->d_adjtab, s->d_wpool, s->d_wavpool, ss,
                                             s->pitch, s->plane, n + 1, s->d.dt, s->force_box, s->st);
                if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
                if ((r = timed_end(s, KC_GRAD))) return r;
            }
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    if ((r = pass_t(j, A[LOSS_F_EV1 + i], b, 3 * i + j, A[sidx[i][j]]))) return r;
            if ((r = inject_res(false, n, 1.f))) return r;
            if ((r = inject_res(true, n, 0.5f))) return r;
            const float *strain[6];
            for (int q = 0; q < 6; ++q) strain[q] = s->divstore + (k * slots + q) * fe;
            if ((r = timed_begin(s))) return r;
            hipError_t e = launch_el_grad_accum(s->grad_pad, s->grad_pad + ss, strain, sbar, s->d.dt, s->nx,
                                                s->pitch, ss, S, s->st);
            if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
            if ((r = timed_end(s, KC_GRAD))) return r;
            for (int kk = 0; kk < 3; ++kk) {
                e = launch_el_normal_operand(Wop, A[LOSS_F_S11], A[LOSS_F_S22], A[LOSS_F_S33], l2m, lam, kk, s->nx,
                                             s->pitch, ss, S, s->st);
                if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
                if ((r = pass_t(kk, Wop, nullptr, 9 + 4 * kk, A[LOSS_F_EV1 + kk]))) return r;
            }
            for (int q = 0; q < 3; ++q) {
                const int sij = sh[q][0], i = sh[q][1], j = sh[q][2];
                if ((r = pass_t(j, A[sij], mu, 9 + 3 * i + j, A[LOSS_F_EV1 + i]))) return r;
                if ((r = pass_t(i, A[sij], mu, 9 + 3 * j + i, A[LOSS_F_EV1 + j]))) return r;
            }
        }
    }
    hipError_t e = hipSuccess;
    if (want_b)   // the opening half step drove u with (dt/2) b f(t_0) w (the state starts at rest)
        e = launch_el_grad_force(gb, s->d_src, s->nsrc, s->d_adjtab, s->d_wpool, s->d_wavpool, ss, s->pitch,
                                 s->plane, 0, 0.5 * s->d.dt, s->force_box, s->st);
    if (e == hipSuccess) {
        const int mode = param == LOSS_GRAD_LAME ? 0 : param == LOSS_GRAD_VPVS ? 1 : param == LOSS_GRAD_LAME_RHO ? 2 : 3;
        e = launch_el_grad_unpad(s->grad_pad, s->grad_pad + ss, gb, s->grad_dense, s->nx, s->pitch, s->d_vp, s->d_vs,
                                 s->d_rho, mode, s->nodes, s->st);
    }
    if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
    HIPCHK(hipMemcpyAsync(grad, s->grad_dense, sizeof(double) * (want_b ? 3 : 2) * s->nodes,
                          mem == LOSS_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    s->step = s->ck_every < s->ck_steps ? s->ck_every : s->ck_steps;
    return LOSS_OK;
}

// ---- device scratch of loss_deriv_static ---------------------------------------
// Three slots (padded input, padded output, the transposed solve's Y) of
// LOSS_STATIC_SCRATCH_FLOATS / 3 floats each.  Each GPU the library runs on holds its own
// copy of the array until the process ends; host code reaches it only through the
// device address hipGetSymbolAddress returns for the current device.
constexpr int64_t kStaticSlot = LOSS_STATIC_SCRATCH_FLOATS / 3;
static __device__ __align__(256) float scratch[LOSS_STATIC_SCRATCH_FLOATS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of the scratch array (looked up once per device).
loss_status static_scratch(float **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LOSS_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LOSS_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (float *)p;
    }
    *out = g_scratch_ptr[dev];
    return LOSS_OK;
}

}  // namespace

extern "C" {

const char *loss_last_error(void) { return g_err.c_str(); }

const char *loss_status_str(loss_status s)
{
    switch (s) {
    case LOSS_OK: return "ok";
    case LOSS_EINVAL: return "invalid argument";
    case LOSS_ENOMEM: return "out of memory";
    case LOSS_EHIP: return "HIP runtime error";
    case LOSS_ESTATE: return "call out of order";
    case LOSS_EUNSUPPORTED: return "unsupported";
    case LOSS_EUNSTABLE: return "unstable";
    default: return "unknown status";
    }
}

loss_status loss_create(const loss_desc *desc, void *hip_stream, loss_sim **out)
{
    if (!desc || !out) return fail(LOSS_EINVAL, "null argument");
    *out = nullptr;
    const loss_desc &d = *desc;
    if (d.physics == LOSS_ACOUSTIC && d.ndim != 2) return fail(LOSS_EINVAL, "acoustic physics is 2-D (x, z)");
    if (d.physics == LOSS_ELASTIC && d.ndim != 3) return fail(LOSS_EINVAL, "elastic physics is 3-D");
    if (d.physics != LOSS_ACOUSTIC && d.physics != LOSS_ELASTIC) return fail(LOSS_EINVAL, "unknown physics");
    if (d.nshots < 1) return fail(LOSS_EINVAL, "nshots must be >= 1");
    if (!(d.dt > 0)) return fail(LOSS_EINVAL, "dt must be positive");
    if (d.trace_len < 0) return fail(LOSS_EINVAL, "trace_len must be >= 0");
    if (d.ndim == 2 && d.n[1] != 0) return fail(LOSS_EINVAL, "2-D grids have n[1] == 0");
    loss_sim *s = new loss_sim();
    s->d = d;
    s->nf = d.physics == LOSS_ACOUSTIC ? 3 : 9;
    s->S = d.nshots;
    s->nx = (int)d.n[0] + 1;
    s->ny = d.ndim == 3 ? (int)d.n[1] + 1 : 1;
    s->nz = (int)d.n[2] + 1;
    s->pitch = ((int64_t)s->nx + 3) / 4 * 4;
    s->plane = s->pitch * s->ny;
    s->shot_stride = s->plane * s->nz;
    s->nodes = (int64_t)s->nx * s->ny * s->nz;
    // the line kernels index within one shot's field in 32-bit arithmetic
    if (s->shot_stride >= (int64_t(1) << 31)) {
        loss_destroy(s);
        return fail(LOSS_EUNSUPPORTED, "a field of one shot holds 2^31 or more elements (padded)");
    }
    auto bail = [&](loss_status st) { loss_destroy(s); return st; };
    for (int a = 0; a < 3; ++a) {
        if (a == 1 && d.ndim == 2) continue;
        std::string err = build_axis(s->axh[a], (int)d.n[a], d.h[a], d.patch[a], d.halo, d.end_mode);
        if (!err.empty()) { loss_destroy(s); return fail(LOSS_EINVAL, "axis " + std::to_string(a) + ": " + err); }
        const int M = d.patch[a];
        if ((a == 0 && M > 1024) || (a != 0 && M > 1024))
            { loss_destroy(s); return fail(LOSS_EUNSUPPORTED, "patch length above 1024"); }
    }
    (void)hipGetDevice(&s->device);
    {
        // set-up of loss_deriv_static: the device address of the static scratch array
        // (the runtime materialises the array on this first lookup, not in that call)
        float *scr = nullptr;
        loss_status rs = static_scratch(&scr);
        if (rs) { loss_destroy(s); return rs; }
    }
    if (hip_stream) {
        s->st = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(LOSS_EHIP, "hipStreamCreate failed"));
        s->own_stream = true;
    }
    loss_status r;
    const int64_t fe = field_elems(s);
    s->f.assign(s->nf, nullptr);
    for (int i = 0; i < s->nf; ++i)
        if ((r = s->alloc(&s->f[i], fe))) return bail(r);
    for (int i = 0; i < 3; ++i)
        if ((r = s->alloc(&s->tmp[i], fe))) return bail(r);
    const int nmed = d.physics == LOSS_ACOUSTIC ? 2 : 4;
    s->med.assign(nmed, nullptr);
    for (int i = 0; i < nmed; ++i)
        if ((r = s->alloc(&s->med[i], s->shot_stride))) return bail(r);
    if ((r = s->alloc(&s->d_fields, s->nf)) || (r = s->alloc(&s->d_tmpfields, s->nf)) ||
        (r = s->alloc(&s->d_step, 1)) || (r = s->alloc(&s->d_bad, 1)))
        return bail(r);
    if (hipHostMalloc((void **)&s->h_bad, sizeof(int), 0) != hipSuccess) {
        s->h_bad = nullptr;
        return bail(fail(LOSS_ENOMEM, "hipHostMalloc of the sentinel flag"));
    }
    *s->h_bad = 0;
    if (hipMemcpy(s->d_bad, s->h_bad, sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(LOSS_EHIP, "sentinel flag"));
    for (int a = 0; a < 3; ++a) {
        if (a == 1 && d.ndim == 2) continue;
        if ((r = upload_axis(s, a))) return bail(r);
    }
    if (hipMemcpy(s->d_fields, s->f.data(), sizeof(float *) * s->nf, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(LOSS_EHIP, "pointer table upload"));
    if (hipEventCreate(&s->ev0) != hipSuccess || hipEventCreate(&s->ev1) != hipSuccess)
        return bail(fail(LOSS_EHIP, "hipEventCreate"));
    s->src.assign(s->S, {});
    s->rec.assign(s->S, RecHost());
    // zero state (fill kernels, no memset nodes)
    for (int i = 0; i < s->nf; ++i)
        if (launch_fill(s->f[i], fe, 0.f, s->st) != hipSuccess) return bail(fail(LOSS_EHIP, "fill"));
    for (int i = 0; i < 3; ++i)
        if (launch_fill(s->tmp[i], fe, 0.f, s->st) != hipSuccess) return bail(fail(LOSS_EHIP, "fill"));
    for (int i = 0; i < nmed; ++i)
        if (launch_fill(s->med[i], s->shot_stride, 0.f, s->st) != hipSuccess) return bail(fail(LOSS_EHIP, "fill"));
    int64_t zero = 0;
    if (hipMemcpy(s->d_step, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(LOSS_EHIP, "step counter"));
    if (hipStreamSynchronize(s->st) != hipSuccess) return bail(fail(LOSS_EHIP, "sync"));
    *out = s;
    return LOSS_OK;
}

loss_status loss_destroy(loss_sim *s)
{
    if (!s) return LOSS_OK;
    if (s->st) (void)hipStreamSynchronize(s->st);
    drop_graph(s);
    for (void *p : s->allocs) (void)hipFree(p);
    s->allocs.clear();
    if (s->ev0) (void)hipEventDestroy(s->ev0);
    if (s->ev1) (void)hipEventDestroy(s->ev1);
    if (s->h_bad) (void)hipHostFree(s->h_bad);
    if (s->own_stream && s->st) (void)hipStreamDestroy(s->st);
    delete s;
    return LOSS_OK;
}

loss_status loss_set_media(loss_sim *s, const float *vp, const float *vs, const float *rho, int32_t mem)
{
    if (!s || !vp || !rho) return fail(LOSS_EINVAL, "null argument");
    if (s->d.physics == LOSS_ELASTIC && !vs) return fail(LOSS_EINVAL, "elastic media need vs");
    const int64_t n = s->nodes;
    loss_status r;
    float *dv[3] = {nullptr, nullptr, nullptr};
    const float *srcs[3] = {vp, vs, rho};
    for (int i = 0; i < 3; ++i) {
        if (!srcs[i]) continue;
        if ((r = s->alloc(&dv[i], n))) return r;
        HIPCHK(hipMemcpyAsync(dv[i], srcs[i], sizeof(float) * n,
                              mem == LOSS_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s->st));
    }
    hipError_t e = launch_media(dv[0], dv[1], dv[2], s->med.data(), s->d.physics, s->nx, s->ny * s->nz,
                                s->pitch, s->d.dt, s->st);
    if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
    // keep dense vp and rho for the gradient map
    if (s->d_vp) s->release(s->d_vp);
    if (s->d_rho) s->release(s->d_rho);
    if (s->d_vs) s->release(s->d_vs);
    s->d_vp = dv[0];
    s->d_vs = dv[1];
    s->d_rho = dv[2];
    // stability bound of the Strang scheme with the spline symbol (max k* h = sqrt 3)
    std::vector<float> hv(n);
    HIPCHK(hipMemcpyAsync(hv.data(), s->d_vp, sizeof(float) * n, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    double cmax = 0;
    for (float v : hv) cmax = std::max(cmax, (double)v);
    s->cmax = cmax;
    double hmin = s->d.h[0];
    hmin = std::min(hmin, s->d.h[2]);
    if (s->d.ndim == 3) hmin = std::min(hmin, s->d.h[1]);
    s->media_set = true;
    drop_graph(s);
    s->ck_steps = 0;   // checkpoints belong to the previous media
    const double bound = 2.0 * hmin / (std::sqrt(3.0) * std::sqrt((double)s->d.ndim) * cmax);
    if (s->d.dt > bound)
        return fail(LOSS_EUNSTABLE, "dt " + std::to_string(s->d.dt) + " exceeds the stability bound " +
                                         std::to_string(bound));
    return LOSS_OK;
}

loss_status loss_add_source(loss_sim *s, int32_t shot, const double pos[3], int32_t kind, const float *wavelet,
                            int64_t nt, double spread_m)
{
    if (!s || !pos || (!wavelet && nt > 0)) return fail(LOSS_EINVAL, "null argument");
    if (shot < 0 || shot >= s->S) return fail(LOSS_EINVAL, "shot out of range");
    if (kind < LOSS_SRC_PRESSURE || kind > LOSS_SRC_FORCE_Z) return fail(LOSS_EINVAL, "unknown source kind");
    if (s->d.physics == LOSS_ACOUSTIC && kind == LOSS_SRC_FORCE_Y) return fail(LOSS_EINVAL, "2-D grid has no y force");
    if (spread_m < 0 || nt < 0 || nt > (1ll << 30)) return fail(LOSS_EINVAL, "bad spread or nt");
    if ((int)s->src[shot].size() >= 16) return fail(LOSS_EINVAL, "at most 16 sources per shot");
    for (int a = 0; a < 3; ++a) {
        if (a == 1 && s->d.ndim == 2) continue;
        if (!(pos[a] >= 0.0 && pos[a] <= s->d.n[a] * s->d.h[a])) return fail(LOSS_EINVAL, "source outside the grid");
    }
    SrcHost h;
    h.kind = kind;
    for (int a = 0; a < 3; ++a) h.pos[a] = pos[a];
    h.spread = spread_m;
    h.wavelet.assign(wavelet, wavelet + nt);
    s->src[shot].push_back(h);
    s->src_dirty = true;
    drop_graph(s);
    return LOSS_OK;
}

loss_status loss_add_receivers(loss_sim *s, int32_t shot, int64_t nrec, const int32_t *node_idx, int32_t component)
{
    if (!s || (nrec > 0 && !node_idx)) return fail(LOSS_EINVAL, "null argument");
    if (shot < 0 || shot >= s->S) return fail(LOSS_EINVAL, "shot out of range");
    if (component < 0 || component >= s->nf) return fail(LOSS_EINVAL, "bad receiver component");
    if (s->d.physics == LOSS_ACOUSTIC && component != LOSS_F_SIGMA)
        return fail(LOSS_EUNSUPPORTED, "acoustic receivers record sigma");
    const int lim[3] = {s->nx, s->ny, s->nz};
    for (int64_t r = 0; r < nrec; ++r)
        for (int a = 0; a < 3; ++a)
            if (node_idx[3 * r + a] < 0 || node_idx[3 * r + a] >= lim[a])
                return fail(LOSS_EINVAL, "receiver node outside the grid");
    RecHost h;
    h.idx.assign(node_idx, node_idx + 3 * nrec);
    h.comp = component;
    s->rec[shot] = h;
    s->rec_dirty = true;
    drop_graph(s);
    return LOSS_OK;
}

loss_status loss_set_pml(loss_sim *s, int32_t width, double reflection, double kmax, double f0)
{
    if (!s) return fail(LOSS_EINVAL, "null argument");
    if (width < 0 || width > s->d.n[0] / 2 || width > s->d.n[2] / 2 || (s->d.ndim == 3 && width > s->d.n[1] / 2))
        return fail(LOSS_EINVAL, "layer width must be in 0 .. n/2 on every axis");
    if (width > 0 && (!(reflection > 0.0 && reflection < 1.0) || !(kmax >= 1.0) || !(f0 > 0.0)))
        return fail(LOSS_EINVAL, "need 0 < reflection < 1, kmax >= 1, f0 > 0");
    if (width > 0 && !s->media_set) return fail(LOSS_ESTATE, "loss_set_media must be called first");
    loss_status r;
    if ((r = unfuse_in_place(s))) return r;
    drop_graph(s);
    // checkpoints were taken under the previous layer: an adjoint must not reuse them
    s->ck_steps = 0;
    for (int a = 0; a < 3; ++a) {
        if (s->pml_tab[a]) { s->release(s->pml_tab[a]); s->pml_tab[a] = nullptr; }
        s->axd[a].pml_w = 0;
    }
    if (s->pml_mem) { s->release(s->pml_mem); s->pml_mem = nullptr; }
    s->npml = 0;
    s->pml_w = width;
    if (width == 0) return LOSS_OK;
    const int64_t fe = field_elems(s);
    const int npml = s->d.physics == LOSS_ACOUSTIC ? 4 : 18;
    if ((r = s->alloc(&s->pml_mem, (size_t)(npml * fe)))) return r;
    s->npml = npml;
    if (launch_fill(s->pml_mem, npml * fe, 0.f, s->st) != hipSuccess) return fail(LOSS_EHIP, "fill");
    for (int a = 0; a < 3; ++a) {
        if (a == 1 && s->d.ndim == 2) continue;
        const int N = (int)s->d.n[a];
        const double h = s->d.h[a];
        const double d0 = -3.0 * s->cmax * std::log(reflection) / (2.0 * width * h);
        const double amax = 3.14159265358979323846 * f0;
        // per step fraction f and node: the exact sub-flow over tau = f dt with the
        // derivative D frozen, x = beta tau, beta = d/k + alpha,
        //   psi(tau) = e^{-x} psi0 - (d/k^2) tau phi1(x) D,
        //   effective derivative = (1/k - (d/k^2) tau phi2(x)) D + phi1(x) psi0,
        // phi1 = (1 - e^{-x})/x, phi2 = (x - 1 + e^{-x})/x^2 (series for small x), stored
        // as {e^{-x}, phi1, (d/k^2) tau phi1, 1/k - (d/k^2) tau phi2} in FP64 -> FP32
        std::vector<float4> tab(3 * (size_t)(N + 1));
        for (int fi = 0; fi < 3; ++fi) {
            const double tau = kPmlFrac[fi] * s->d.dt;
            for (int j = 0; j <= N; ++j) {
                int dist = 0;
                if (j < width) dist = width - j;
                if (j > N - width) dist = std::max(dist, j - (N - width));
                const double del = (double)dist / width;
                const double d = d0 * del * del, k = 1.0 + (kmax - 1.0) * del, al = amax * (1.0 - del);
                const double x = (d / k + al) * tau, dk2 = d / (k * k);
                double phi1, phi2;
                if (std::fabs(x) < 1e-2) {
                    phi1 = 1.0 - x / 2.0 + x * x / 6.0 - x * x * x / 24.0 + x * x * x * x / 120.0;
                    phi2 = 0.5 - x / 6.0 + x * x / 24.0 - x * x * x / 120.0 + x * x * x * x / 720.0;
                } else {
                    phi1 = -std::expm1(-x) / x;
                    phi2 = (x + std::expm1(-x)) / (x * x);
                }
                tab[(size_t)fi * (N + 1) + j] = make_float4((float)std::exp(-x), (float)phi1,
                                                            (float)(dk2 * tau * phi1),
                                                            (float)(1.0 / k - dk2 * tau * phi2));
            }
        }
        if ((r = s->alloc(&s->pml_tab[a], 3 * (size_t)(N + 1)))) return r;
        HIPCHK(hipMemcpy(s->pml_tab[a], tab.data(), sizeof(float4) * tab.size(), hipMemcpyHostToDevice));
        s->axd[a].pml_w = width;
    }
    HIPCHK(hipStreamSynchronize(s->st));
    return LOSS_OK;
}

loss_status loss_reset(loss_sim *s)
{
    if (!s) return fail(LOSS_EINVAL, "null argument");
    const int64_t fe = field_elems(s);
    for (int i = 0; i < s->nf; ++i)
        if (launch_fill(s->f[i], fe, 0.f, s->st) != hipSuccess) return fail(LOSS_EHIP, "fill");
    if (s->pml_mem && launch_fill(s->pml_mem, s->npml * fe, 0.f, s->st) != hipSuccess) return fail(LOSS_EHIP, "fill");
    if (s->traces && s->trace_total > 0)
        HIPCHK(hipMemsetAsync(s->traces, 0, sizeof(double) * s->trace_total, s->st));
    HIPCHK(launch_set_step(s->d_step, 0, s->st));
    HIPCHK(hipMemsetAsync(s->d_bad, 0, sizeof(int), s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    *s->h_bad = 0;
    s->step = 0;
    s->fused = false;
    return LOSS_OK;
}

loss_status loss_step(loss_sim *s, int64_t nsteps)
{
    if (!s) return fail(LOSS_EINVAL, "null argument");
    if (nsteps < 0) return fail(LOSS_EINVAL, "nsteps must be >= 0");
    loss_status r = check_sentinel(s);
    if (r) return r;
    return run_steps(s, nsteps, nullptr, 0);
}

loss_status loss_get_field(loss_sim *s, int32_t shot, int32_t field, float *dst, int32_t mem)
{
    if (!s || !dst) return fail(LOSS_EINVAL, "null argument");
    if (shot < 0 || shot >= s->S || field < 0 || field >= s->nf) return fail(LOSS_EINVAL, "bad shot or field");
    const float *src = s->f[field];
    if (is_velocity(s, field) && s->fused) {
        std::vector<float *> v;
        loss_status r = unfused_velocity(s, v);
        if (r) return r;
        int c = s->d.physics == LOSS_ACOUSTIC ? (field == LOSS_F_V1 ? 0 : 1) : field - LOSS_F_EV1;
        src = v[c];
    }
    return copy_field_out(s, dst, src + (int64_t)shot * s->shot_stride, mem, 1);
}

loss_status loss_set_field(loss_sim *s, int32_t shot, int32_t field, const float *src, int32_t mem)
{
    if (!s || !src) return fail(LOSS_EINVAL, "null argument");
    if (shot < 0 || shot >= s->S || field < 0 || field >= s->nf) return fail(LOSS_EINVAL, "bad shot or field");
    loss_status r = unfuse_in_place(s);
    if (r) return r;
    return copy_field_in(s, s->f[field] + (int64_t)shot * s->shot_stride, src, mem, 1);
}

loss_status loss_get_traces(loss_sim *s, int32_t shot, double *dst, int32_t mem)
{
    if (!s || !dst) return fail(LOSS_EINVAL, "null argument");
    if (shot < 0 || shot >= s->S) return fail(LOSS_EINVAL, "bad shot");
    loss_status r = upload_receivers(s);
    if (r) return r;
    const int64_t nr = (int64_t)s->rec[shot].idx.size() / 3;
    const int64_t cnt = nr * s->d.trace_len;
    if (cnt == 0) return LOSS_OK;
    HIPCHK(hipMemcpyAsync(dst, s->traces + s->rec_off[shot], sizeof(double) * cnt,
                          mem == LOSS_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s->st));
    if (mem == LOSS_MEM_HOST) HIPCHK(hipStreamSynchronize(s->st));
    return LOSS_OK;
}

loss_status loss_deriv(loss_sim *s, int32_t axis, int32_t order, const float *in, float *out, int64_t batch,
                       int32_t mem)
{
    if (!s || !in || !out) return fail(LOSS_EINVAL, "null argument");
    if (axis < 0 || axis > 2 || (axis == 1 && s->d.ndim == 2)) return fail(LOSS_EINVAL, "bad axis");
    if (order != 1 && order != 2 && order != -1) return fail(LOSS_EINVAL, "order must be 1, 2 or -1");
    if (batch < 1) return fail(LOSS_EINVAL, "batch must be >= 1");
    // tmp[1] and tmp[2] hold up to S fields each
    const int64_t dense = s->nodes;
    loss_status r = unfuse_in_place(s);
    if (r) return r;
    for (int64_t b0 = 0; b0 < batch; b0 += s->S) {
        const int64_t nb = std::min<int64_t>(s->S, batch - b0);
        if ((r = copy_field_in(s, s->tmp[1], in + b0 * dense, mem, nb))) return r;
        if (order == -1) {
            if ((r = adj_deriv(s, axis, s->tmp[1], nullptr, s->tmp[2], 1.f, EPI_STORE, s->tmp[0], (int)nb)))
                return r;
        } else {
            LineArgs a = base_args(s, axis);
            a.S = (int)nb;
            a.in = s->tmp[1];
            a.out[0] = s->tmp[2];
            if ((r = run_line(s, KC_VEL_X + axis, axis, order == 1 ? SOLVE_D1 : SOLVE_D2, EPI_STORE, a)))
                return r;
        }
        if ((r = copy_field_out(s, out + b0 * dense, s->tmp[2], mem, nb))) return r;
    }
    return LOSS_OK;
}

loss_status loss_deriv_static(loss_sim *s, int32_t axis, int32_t order, const float *in, float *out,
                              int64_t batch)
{
    if (!s || !in || !out) return fail(LOSS_EINVAL, "null argument");
    if (axis < 0 || axis > 2 || (axis == 1 && s->d.ndim == 2)) return fail(LOSS_EINVAL, "bad axis");
    if (order != 1 && order != 2 && order != -1) return fail(LOSS_EINVAL, "order must be 1, 2 or -1");
    if (batch < 1) return fail(LOSS_EINVAL, "batch must be >= 1");
    if (s->shot_stride > kStaticSlot)
        return fail(LOSS_EINVAL, "a field of this grid takes " + std::to_string(s->shot_stride) +
                                     " padded floats, above the static scratch slot of " + std::to_string(kStaticSlot));
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != s->device) return fail(LOSS_ESTATE, "the current device is not the simulation's");
    float *base = nullptr;
    loss_status r = static_scratch(&base);
    if (r) return r;
    float *pin = base, *pout = base + kStaticSlot, *Y = base + 2 * kStaticSlot;
    const int64_t dense = s->nodes;
    const int64_t chunk = kStaticSlot / s->shot_stride;   // fields per pass through the scratch
    for (int64_t b0 = 0; b0 < batch; b0 += chunk) {
        const int nb = (int)std::min<int64_t>(chunk, batch - b0);
        hipError_t e = launch_pad_copy(in + b0 * dense, pin, s->nx, (int)(nb * s->ny * s->nz), s->pitch, 1, s->st);
        if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
        if (order == -1) {
            if ((r = adj_deriv(s, axis, pin, nullptr, pout, 1.f, EPI_STORE, Y, nb))) return r;
        } else {
            LineArgs a = base_args(s, axis);
            a.S = nb;
            a.in = pin;
            a.out[0] = pout;
            if ((r = run_line(s, KC_VEL_X + axis, axis, order == 1 ? SOLVE_D1 : SOLVE_D2, EPI_STORE, a))) return r;
        }
        e = launch_pad_copy(pout, out + b0 * dense, s->nx, (int)(nb * s->ny * s->nz), s->pitch, 0, s->st);
        if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
    }
    return LOSS_OK;
}

loss_status loss_energy(loss_sim *s, double *energy)
{
    if (!s || !energy) return fail(LOSS_EINVAL, "null argument");
    if (!s->d_rho) return fail(LOSS_ESTATE, "loss_set_media must run first");
    std::vector<float *> v;
    loss_status r = unfused_velocity(s, v);   // the velocity at the state's integer time
    if (r) return r;
    EnergyArgs a{};
    const bool el = s->d.physics == LOSS_ELASTIC;
    a.nv = el ? 3 : 2;
    for (int c = 0; c < a.nv; ++c) a.v[c] = v[c];
    if (el) {
        a.ns = 6;
        for (int c = 0; c < 6; ++c) a.s[c] = s->f[LOSS_F_S11 + c];
    } else {
        a.ns = 1;
        a.s[0] = s->f[LOSS_F_SIGMA];
    }
    a.vp = s->d_vp;
    a.vs = s->d_vs;
    a.rho = s->d_rho;
    a.nx = s->nx;
    a.pitch = s->pitch;
    a.shot_stride = s->shot_stride;
    a.nodes = s->nodes;
    const int nblocks = 1024;
    if (!s->energy_buf && (r = s->alloc(&s->energy_buf, (size_t)(s->S * nblocks + s->S)))) return r;
    double cell = s->d.h[0] * s->d.h[2];
    if (el) cell *= s->d.h[1];
    const hipError_t e = launch_energy(a, (int)s->S, s->energy_buf, nblocks, cell, s->energy_buf + s->S * nblocks,
                                       s->st);
    if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
    HIPCHK(hipMemcpyAsync(energy, s->energy_buf + s->S * nblocks, sizeof(double) * s->S, hipMemcpyDeviceToHost,
                          s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return LOSS_OK;
}

loss_status loss_sync(loss_sim *s)
{
    if (!s) return fail(LOSS_EINVAL, "null argument");
    HIPCHK(hipStreamSynchronize(s->st));
    return check_sentinel(s);
}

loss_status loss_set_timing(loss_sim *s, int32_t on)
{
    if (!s) return fail(LOSS_EINVAL, "null argument");
    s->timing = on != 0;
    for (int i = 0; i < KC_COUNT; ++i) { s->kms[i] = 0; s->kcount[i] = 0; }
    return LOSS_OK;
}

loss_status loss_kernel_timing(loss_sim *s, int32_t id, double *ms, int64_t *launches, const char **name)
{
    if (!s) return fail(LOSS_EINVAL, "null argument");
    if (id < 0 || id >= KC_COUNT) return fail(LOSS_EINVAL, "no such kernel class");
    if (ms) *ms = s->kms[id];
    if (launches) *launches = s->kcount[id];
    if (name) *name = kKClassName[id];
    return LOSS_OK;
}

int64_t loss_current_step(const loss_sim *s) { return s ? s->step : -1; }

loss_status loss_autotune(loss_sim *s, int32_t trial_steps)
{
    if (!s) return fail(LOSS_EINVAL, "null argument");
    if (trial_steps < 1) return fail(LOSS_EINVAL, "trial_steps must be >= 1");
    loss_status r;
    if ((r = ensure_ready(s))) return r;
    // save the state
    const int64_t fe = field_elems(s);
    float *bk = nullptr;
    double *tbk = nullptr;
    const int npml = s->pml_mem ? s->npml : 0;
    if ((r = s->alloc(&bk, (size_t)((s->nf + npml) * fe)))) return r;
    if ((r = s->alloc(&tbk, (size_t)std::max<int64_t>(1, s->trace_total)))) return r;
    for (int f = 0; f < s->nf; ++f)
        HIPCHK(hipMemcpyAsync(bk + f * fe, s->f[f], sizeof(float) * fe, hipMemcpyDeviceToDevice, s->st));
    if (npml)
        HIPCHK(hipMemcpyAsync(bk + s->nf * fe, s->pml_mem, sizeof(float) * npml * fe, hipMemcpyDeviceToDevice, s->st));
    if (s->trace_total)
        HIPCHK(hipMemcpyAsync(tbk, s->traces, sizeof(double) * s->trace_total, hipMemcpyDeviceToDevice, s->st));
    const int64_t step0 = s->step;
    const bool fused0 = s->fused;
    const bool timing0 = s->timing;
    s->timing = false;
    if ((r = fuse(s))) return r;
    // time trial_steps steps of the current configuration
    auto trial = [&](float &ms) -> loss_status {
        loss_status q;
        if ((q = steps_eager(s, 2))) return q;   // warm this shape up
        HIPCHK(hipEventRecord(s->ev0, s->st));
        if ((q = steps_eager(s, trial_steps))) return q;
        HIPCHK(hipEventRecord(s->ev1, s->st));
        HIPCHK(hipEventSynchronize(s->ev1));
        HIPCHK(hipEventElapsedTime(&ms, s->ev0, s->ev1));
        return LOSS_OK;
    };
    // launch shapes of the line kernels along `axis`, the fastest kept; returns its time
    auto tune_axis = [&](int axis, float &best) -> loss_status {
        // candidates: x -> (nodes per lane, lines per wave); y, z -> (columns per wave,
        // nodes per lane)
        std::vector<std::pair<int, int>> cands;
        if (axis == 0) cands = {{4, 0}, {4, 1}, {8, 0}, {16, 0}, {4, 4}, {4, 8}};
        else cands = {{64, 8}, {64, 16}, {32, 16}, {16, 16}, {32, 8}, {16, 8}};
        best = 1e30f;
        std::pair<int, int> bestc = cands[0];
        for (const auto &cd : cands) {
            if (axis == 0) { s->cx = cd.first; s->xl = cd.second; }
            else { s->cw[axis] = cd.first; s->cs[axis] = cd.second; }
            float ms = 0.f;
            loss_status q = trial(ms);
            if (q) return q;
            if (ms < best) { best = ms; bestc = cd; }
        }
        if (axis == 0) { s->cx = bestc.first; s->xl = bestc.second; }
        else { s->cw[axis] = bestc.first; s->cs[axis] = bestc.second; }
        return LOSS_OK;
    };
    float t_line = 0.f;
    // the line-pass schedule (every axis), then for elastic grids that admit it the
    // plane schedule (its line kernels run along z only); the faster schedule is kept
    const int sched0 = s->elastic_schedule;
    s->elastic_schedule = 1;
    // elastic: the y axis is timed with its store passes held at 64 columns, then the
    // store passes' own shape is chosen
    if (s->d.physics == LOSS_ELASTIC) {
        s->cws[1] = 64;
        s->css[1] = 8;
    }
    for (int axis = 0; axis < 3; ++axis) {
        if (axis == 1 && s->d.ndim == 2) continue;
        if ((r = tune_axis(axis, t_line))) return r;
    }
    // elastic: the y store passes (two of the eighteen per step) may take their own shape
    if (s->d.physics == LOSS_ELASTIC) {
        const std::pair<int, int> sc[] = {{0, 0}, {64, 8}, {32, 8}};
        float best = 1e30f;
        std::pair<int, int> bestc = sc[0];
        for (const auto &cd : sc) {
            s->cws[1] = cd.first;
            s->css[1] = cd.second;
            float ms = 0.f;
            if ((r = trial(ms))) return r;
            if (ms < best) { best = ms; bestc = cd; }
        }
        s->cws[1] = bestc.first;
        s->css[1] = bestc.second;
        t_line = std::min(t_line, best);
    }
    s->elastic_schedule = sched0;
    if (s->d.physics == LOSS_ELASTIC) {
        s->elastic_schedule = 0;
        if (plane_ok(s)) {
            const int cw2 = s->cw[2], cs2 = s->cs[2];
            float t_plane = 0.f;
            if ((r = tune_axis(2, t_plane))) return r;
            if (t_plane > t_line) {
                s->elastic_schedule = 1;
                s->cw[2] = cw2;
                s->cs[2] = cs2;
            }
        } else {
            s->elastic_schedule = sched0;
        }
    }
    // restore
    for (int f = 0; f < s->nf; ++f)
        HIPCHK(hipMemcpyAsync(s->f[f], bk + f * fe, sizeof(float) * fe, hipMemcpyDeviceToDevice, s->st));
    if (npml)
        HIPCHK(hipMemcpyAsync(s->pml_mem, bk + s->nf * fe, sizeof(float) * npml * fe, hipMemcpyDeviceToDevice, s->st));
    if (s->trace_total)
        HIPCHK(hipMemcpyAsync(s->traces, tbk, sizeof(double) * s->trace_total, hipMemcpyDeviceToDevice, s->st));
    HIPCHK(launch_set_step(s->d_step, step0, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    s->release(bk);
    s->release(tbk);
    s->step = step0;
    s->fused = fused0;
    s->timing = timing0;
    drop_graph(s);
    return LOSS_OK;
}

loss_status loss_set_shape(loss_sim *s, int32_t axis, int32_t shape)
{
    if (s && (axis == 4 || axis == 5)) {   // the y / z store passes
        const int cw = shape / 100, cs = shape % 100;
        if (shape != 0 && !((cw == 8 || cw == 16 || cw == 32 || cw == 64) && (cs == 8 || cs == 16)))
            return fail(LOSS_EINVAL, "bad store shape");
        if (axis == 4 && s->d.ndim == 2) return fail(LOSS_EINVAL, "bad axis");
        s->cws[axis - 3] = cw;
        s->css[axis - 3] = cs;
        drop_graph(s);
        return LOSS_OK;
    }
    if (s && axis == 3) {
        if (shape != 0 && shape != 1) return fail(LOSS_EINVAL, "schedule must be 0 (plane) or 1 (line passes)");
        s->elastic_schedule = shape;
        drop_graph(s);
        return LOSS_OK;
    }
    if (!s || axis < 0 || axis > 2 || (axis == 1 && s->d.ndim == 2)) return fail(LOSS_EINVAL, "bad axis");
    if (axis == 0) {
        const int cx = shape % 100, xl = shape / 100;
        if (shape != 0 && !((cx == 4 || cx == 8 || cx == 16) && (xl == 0 || xl == 1 || xl == 2 || xl == 4 || xl == 8 || xl == 16)))
            return fail(LOSS_EINVAL, "bad x shape");
        s->cx = cx;
        s->xl = xl;
    } else {
        const int cw = shape / 100, cs = shape % 100;
        if (shape != 0 && !((cw == 8 || cw == 16 || cw == 32 || cw == 64) && (cs == 8 || cs == 16)))
            return fail(LOSS_EINVAL, "bad y/z shape");
        s->cw[axis] = cw;
        s->cs[axis] = cs;
    }
    drop_graph(s);
    return LOSS_OK;
}

loss_status loss_autotune_choice(loss_sim *s, int32_t axis, int32_t *cw)
{
    if (!s || !cw || axis < 0 || axis > 5) return fail(LOSS_EINVAL, "bad argument");
    if (axis == 3) {
        *cw = plane_ok(s) ? 0 : 1;
        return LOSS_OK;
    }
    if (axis > 3) {
        *cw = s->cws[axis - 3] * 100 + s->css[axis - 3];
        return LOSS_OK;
    }
    *cw = axis == 0 ? s->xl * 100 + s->cx : s->cw[axis] * 100 + s->cs[axis];
    return LOSS_OK;
}

loss_status loss_forward_ckpt(loss_sim *s, int64_t nsteps, int64_t ckpt_every)
{
    if (!s) return fail(LOSS_EINVAL, "null argument");
    if (nsteps < 1 || ckpt_every < 1) return fail(LOSS_EINVAL, "nsteps and ckpt_every must be >= 1");
    for (int a = 0; a < 3; ++a)
        if (!(a == 1 && s->d.ndim == 2) && s->d.patch[a] < 2)
            return fail(LOSS_EUNSUPPORTED, "the adjoint needs patches of at least 2 intervals");
    if (s->d.trace_len < nsteps) return fail(LOSS_EINVAL, "trace_len must cover nsteps");
    loss_status r;
    if ((r = ensure_ready(s))) return r;
    if ((r = loss_reset(s))) return r;
    if ((r = fuse(s))) return r;
    const int64_t nseg = (nsteps + ckpt_every - 1) / ckpt_every;
    const int64_t fe = field_elems(s);
    const int ckf = s->nf + (s->pml_mem ? s->npml : 0);
    if (s->ckpt && (s->ck_nseg != nseg || s->ck_fields != ckf)) { s->release(s->ckpt); s->ckpt = nullptr; }
    if (!s->ckpt && (r = s->alloc(&s->ckpt, (size_t)(nseg * ckf * fe)))) return r;
    s->ck_fields = ckf;
    if (s->divstore && s->ck_every != ckpt_every) { s->release(s->divstore); s->divstore = nullptr; }
    s->ck_nseg = nseg;
    s->ck_every = ckpt_every;
    s->ck_steps = 0;
    for (int64_t c = 0; c < nseg; ++c) {
        for (int k = 0; k < s->nf; ++k)
            HIPCHK(hipMemcpyAsync(s->ckpt + (c * ckf + k) * fe, s->f[k], sizeof(float) * fe,
                                  hipMemcpyDeviceToDevice, s->st));
        if (ckf > s->nf)   // the layer's memory variables go with the state
            HIPCHK(hipMemcpyAsync(s->ckpt + (c * ckf + s->nf) * fe, s->pml_mem, sizeof(float) * (ckf - s->nf) * fe,
                                  hipMemcpyDeviceToDevice, s->st));
        const int64_t nc = std::min(ckpt_every, nsteps - c * ckpt_every);
        if ((r = run_steps(s, nc, nullptr, 0))) return r;
    }
    s->ck_steps = nsteps;
    return LOSS_OK;
}

loss_status loss_adjoint(loss_sim *s, const double *residual, int32_t param, double *grad, int32_t mem)
{
    if (!s || !residual || !grad) return fail(LOSS_EINVAL, "null argument");
    if (s->ck_steps < 1)
        return fail(LOSS_ESTATE, "loss_forward_ckpt must run first (and again after loss_set_media or loss_set_pml)");
    if ((s->pml_mem != nullptr) != (s->ck_fields > s->nf))
        return fail(LOSS_ESTATE, "the checkpoints were taken with a different absorbing layer");
    if (s->d.physics == LOSS_ELASTIC) return elastic_adjoint(s, residual, param, grad, mem);
    if (param != LOSS_GRAD_K && param != LOSS_GRAD_VP) return fail(LOSS_EINVAL, "unknown gradient parameter");
    loss_status r;
    const int64_t fe = field_elems(s), S = s->S, ss = s->shot_stride;
    const float dt = (float)s->d.dt;
    for (int k = 0; k < 4; ++k)
        if (!s->adj[k] && (r = s->alloc(&s->adj[k], fe))) return r;
    if (!s->divstore && (r = s->alloc(&s->divstore, (size_t)(s->ck_every * fe)))) return r;
    if (!s->grad_pad && (r = s->alloc(&s->grad_pad, ss))) return r;
    if (!s->grad_dense && (r = s->alloc(&s->grad_dense, s->nodes))) return r;
    if (!s->res_dev && (r = s->alloc(&s->res_dev, std::max<int64_t>(1, s->trace_total)))) return r;
    if (s->trace_total > 0)
        HIPCHK(hipMemcpyAsync(s->res_dev, residual, sizeof(double) * s->trace_total,
                              mem == LOSS_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s->st));
    for (int k = 0; k < 3; ++k)
        if (launch_fill(s->adj[k], fe, 0.f, s->st) != hipSuccess) return fail(LOSS_EHIP, "fill");
    HIPCHK(hipMemsetAsync(s->grad_pad, 0, sizeof(double) * ss, s->st));
    float *lam = s->adj[0], *mu1 = s->adj[1], *mu3 = s->adj[2], *Y = s->adj[3];
    const float *K = s->med[0], *b = s->med[1];
    const bool layer = s->pml_mem != nullptr;
    if (layer) {
        for (int k = 0; k < 5; ++k)
            if (!s->adj_pml[k] && (r = s->alloc(&s->adj_pml[k], fe))) return r;
        for (int k = 0; k < 4; ++k)
            if (launch_fill(s->adj_pml[k], fe, 0.f, s->st) != hipSuccess) return fail(LOSS_EHIP, "fill");
    }
    bool lam_x_done = false;   // the coming step's lambda x pass already applied
    for (int64_t c = s->ck_nseg - 1; c >= 0; --c) {
        const int64_t n0 = c * s->ck_every, nc = std::min(s->ck_every, s->ck_steps - n0);
        // restore the fused state at step n0 and recompute the segment, keeping div u
        for (int k = 0; k < 3; ++k)
            HIPCHK(hipMemcpyAsync(s->f[k], s->ckpt + (c * s->ck_fields + k) * fe, sizeof(float) * fe,
                                  hipMemcpyDeviceToDevice, s->st));
        if (layer)
            HIPCHK(hipMemcpyAsync(s->pml_mem, s->ckpt + (c * s->ck_fields + 3) * fe, sizeof(float) * 4 * fe,
                                  hipMemcpyDeviceToDevice, s->st));
        HIPCHK(launch_set_step(s->d_step, n0, s->st));
        s->fused = true;
        if ((r = steps_eager(s, nc, s->divstore, ss))) return r;
        if (layer) {
            // every pass transposed through its layer operand (memory-variable bars 0 psi_x,
            // 1 psi_z of the velocity passes, 2 phi_x, 3 phi_z of the stress passes), then
            // the transposed derivative; the same order as the plain loop below
            float *W = s->adj_pml[4];
            auto pass_t = [&](int axis, const float *fbar, const float *coef, int mv, float *target) -> loss_status {
                if ((r = timed_begin(s))) return r;
                const hipError_t e = launch_pml_adj_operand(W, fbar, coef, -1.f, s->adj_pml[mv], s->pml_tab[axis], axis,
                                                            s->pml_w, (int)s->d.n[axis], s->nx, s->ny, s->pitch, ss,
                                                            (int)S, s->st);
                if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
                if ((r = timed_end(s, KC_GRAD))) return r;
                return adj_deriv(s, axis, W, nullptr, target, 1.f, EPI_AXPY, Y, (int)S);
            };
            for (int64_t k = nc - 1; k >= 0; --k) {
                const int64_t n = n0 + k;
                if ((r = pass_t(0, mu1, b, 0, lam))) return r;
                if ((r = pass_t(2, mu3, b, 1, lam))) return r;
                if ((r = timed_begin(s))) return r;
                hipError_t e = launch_res_gather(s->d_tgt_str, s->ntgt_str, s->d_toff_str, nullptr, lam, ss, s->res_dev,
                                                 n, 1.f, s->st);
                if (e == hipSuccess) e = launch_grad_accum(s->grad_pad, lam, s->divstore + k * fe, -dt, (int)S, ss, ss, s->st);
                if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
                if ((r = timed_end(s, KC_GRAD))) return r;
                if ((r = pass_t(2, lam, K, 3, mu3))) return r;
                if ((r = pass_t(0, lam, K, 2, mu1))) return r;
            }
            continue;
        }
        // reverse sweep over the segment.  Per step: lambda^{n+1} += -dt Dx^T(b mu1) (done
        // by the previous step's paired x pass, except at the first reverse step), the
        // residual, -dt Dz^T(b mu3); dJ/dK += -dt lambda^{n+1} div u^n; then
        // mu^n = mu^{n+1} - dt D^T(K lambda^{n+1}), whose x pass is paired with the next
        // step's lambda x pass (media hold dt b, dt K)
        for (int64_t k = nc - 1; k >= 0; --k) {
            const int64_t n = n0 + k;
            if (!lam_x_done && (r = adj_deriv(s, 0, mu1, b, lam, -1.f, EPI_AXPY, Y, (int)S))) return r;
            if ((r = timed_begin(s))) return r;
            hipError_t e = launch_res_gather(s->d_tgt_str, s->ntgt_str, s->d_toff_str, nullptr, lam, ss, s->res_dev, n,
                                             1.f, s->st);
            if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
            if ((r = timed_end(s, KC_RECEIVER))) return r;
            if ((r = adj_deriv(s, 2, mu3, b, lam, -1.f, EPI_AXPY, Y, (int)S))) return r;
            if ((r = timed_begin(s))) return r;
            e = launch_grad_accum(s->grad_pad, lam, s->divstore + k * fe, -dt, (int)S, ss, ss, s->st);
            if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
            if ((r = timed_end(s, KC_GRAD))) return r;
            if ((r = adj_deriv(s, 2, lam, K, mu3, -1.f, EPI_AXPY, Y, (int)S))) return r;
            if (n == 0) {
                if ((r = adj_deriv(s, 0, lam, K, mu1, -1.f, EPI_AXPY, Y, (int)S))) return r;
                lam_x_done = false;
            } else {
                if ((r = adj_x_pair(s, lam, K, mu1, b, Y, (int)S))) return r;
                lam_x_done = true;
            }
        }
    }
    hipError_t e = launch_grad_unpad(s->grad_pad, s->grad_dense, s->nx, s->ny * s->nz, s->pitch, s->d_vp,
                                     s->d_rho, param, s->st);
    if (e != hipSuccess) return fail(LOSS_EHIP, hipGetErrorString(e));
    HIPCHK(hipMemcpyAsync(grad, s->grad_dense, sizeof(double) * s->nodes,
                          mem == LOSS_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    // the wavefields now hold a recomputed intermediate state
    s->step = s->ck_every < s->ck_steps ? s->ck_every : s->ck_steps;
    return LOSS_OK;
}

}  // extern "C"
