// Internal declarations of the HIP library behind include/loss.h.
//
// Derivative of a line along one axis (paper Sec. 3.1-3.2), as computed on the GPU.
// The spline slopes w_i = (v~_{i+1} - v~_{i-1}) / (2h) of a patch with Hermite ends
// satisfy, at every patch-interior node, the three-term relation obtained by
// differencing two neighbouring collocation rows:
//     w_{i-1} + 4 w_i + w_{i+1} = (3/h) (u_{i+1} - u_{i-1}),
// with w = phi (the PMBC slope) at the junction rows, and at a natural end
//     2 w_0 + w_1 = (3/h)(u_1 - u_0),   w_{N-1} + 2 w_N = (3/h)(u_N - u_{N-1}).
// Every line is therefore one tridiagonal system T w = G u whose junction rows are
// identity rows; T decouples into the patches.  The GPU solves it with the LU
// factors of T (one table per axis, built in FP64 on the host) by chunked affine
// scans: each lane eliminates a chunk of C nodes in registers and the chunk carries
// are composed across lanes (wave shuffles) or waves (LDS).  The adjoint applies
// T^{-T} (another table) and G^T (stencil plus the transposed PMBC gather).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace loss {

constexpr int kMaxHalo = 64;
constexpr int kTabPad = 64;         // identity rows after row N of the per-row factor tables
// The carry a chunk leaves out of its elimination when it composes only the maps of
// the chunks within `reach` rows is at most kReachTol times the carry itself.
constexpr double kReachTol = 0x1p-44;

// Row kinds of the derivative system of one axis.
enum RowKind : int { ROW_INTERIOR = 0, ROW_JUNCTION = 1, ROW_NATURAL_L = 2, ROW_NATURAL_R = 3 };

// Host FP64 tables of one axis.
struct AxisHost {
    int N = 0, M = 0, p = 0, halo = 0, end_mode = 0;
    double h = 0.0;
    std::vector<int> kind;              // [N+1]
    std::vector<double> sub, diag, sup; // rows of T
    std::vector<double> cm, c0, cp;     // stencil rows of G (zero on junction rows)
    std::vector<int> slot;              // [N+1] junction slot or -1
    std::vector<int> tap_idx;           // [nslot][2*halo+1] node index, -1 = none
    std::vector<double> tap_c;          // [nslot][2*halo+1]
    std::vector<int> junction_node;     // [nslot]
    // LU of T (forward) and of T^T (adjoint), no pivoting
    std::vector<double> m, invd;        // T:   y_i = rhs_i - m_i y_{i-1}; w_i = (y_i - sup_i w_{i+1}) invd_i
    std::vector<double> mT, invdT, supT, subT;
    // transposed PMBC: for node j, up to gmax (junction node, coefficient) pairs, gmax
    // the most junction rows whose taps reach one node (about 2 halo / M + 1)
    int gmax = 1;
    std::vector<int> g_node;            // [N+1][gmax], -1 = none
    std::vector<double> g_c;
    // second-derivative system (per patch, Hermite/natural end rows)
    std::vector<double> m2, invd2, sup2;    // factors for rows as the first/interior row of a patch
    std::vector<double> m2c, invd2c;        // factors of node i as the closing row of the patch ending at i
    int reach = 0;                      // rows of carry composition (see kReachTol)
};

// Build the tables; returns an empty string on success, else the reason.
std::string build_axis(AxisHost &ax, int N, double h, int M, int halo, int end_mode);

// A node whose column of G^T is not the plain interior form: its stencil column and
// the transposed PMBC rows reaching it (gather of the adjoint x pass).
struct SpecialCol {
    float4 aw;             // {c+ of row j-1, c0 of row j, c- of row j+1, 0}
    int row, pad0, pad1, pad2;   // node j; its junction rows are row j of g_node / g_c
};

// Device copy of one axis (float32).
struct AxisDev {
    int N, M, p, ntap, halo, periodic;
    int ends;              // end mode (LOSS_END_*): junction slots of patch l are l-1, l (natural) or l, l+1
    int reach;             // rows of carry composition across chunks (see kReachTol)
    float h;
    float s3;              // 3/h, the stencil weight of interior rows of G
    const float2 *lum;     // {m, invd} of T (compact copy for interior rows; kTabPad rows past N)
    const float2 *lum2;    // {m2, invd2} of the moment system (compact, padded like lum)
    const float4 *lu;      // {m, invd, sup, kind}
    const float4 *rc;      // {cm, c0, cp, slot}
    const float4 *luT;     // {mT, invdT, supT, subT} (padded like lum)
    const float4 *lu2;     // {m2, invd2, sup2, 0}
    const float2 *lu2c;    // {m2c, invd2c}
    const int *tap_idx;    // [nslot][ntap]
    const float *tap_c;
    const int *g_node;     // [N+1][gmax]
    const float *g_c;
    int gmax;              // entries per node of g_node / g_c
    const float4 *adjw;    // [N+1] {c+ of row j-1, c0 of row j, c- of row j+1, 0}: column j of G's stencil
    const unsigned *plain; // bit j: column j is {s3, 0, -s3, 0} and no junction row's taps reach node j
    float4 adjw_plain;     // that column
    const SpecialCol *spec;  // the other nodes, by row
    int nspec;
    int pml_w;             // absorbing layer width in nodes (nodes j < pml_w or j > N - pml_w)
};

// Epilogue of a line kernel.
enum EpiKind : int {
    EPI_STORE = 0,        // out0 = D
    EPI_AXPY = 1,         // out_j += alpha * coef_j * D       (j < nout, coef_j may be null)
    EPI_AXPY_AUX = 2,     // out0 += alpha * coef0 * (D + aux); optional div store: div = D + aux
    EPI_BASE = 3,         // out0 = aux + alpha * coef0 * D
    EPI_NORMAL3 = 4,      // elastic normal stresses, this pass the last of d1 v1 = aux, d2 v2 = aux2,
                          // d3 v3 = D: out_i += alpha (coef0 d_i v_i + coef1 (sum of the other two))
};

// Which system the line kernel solves.
enum SolveKind : int {
    SOLVE_D1 = 0,         // first derivative, rhs = G u
    SOLVE_D2 = 1,         // second derivative, per-patch moment system
    SOLVE_T1 = 2,         // adjoint phase 1: y = T^{-T} z on patch interiors
};

struct SrcDev;

struct LineArgs {
    const float *in;
    const float *in_coef;  // optional per-node factor applied to `in` as it is read
    float *out[3];
    const float *coef[3];
    const float *aux;
    const float *aux2;     // second auxiliary field (EPI_NORMAL3)
    float *div;            // optional store of D + aux (EPI_AXPY_AUX)
    int64_t div_shot_stride;
    float alpha;
    int nout;
    // geometry (elements, padded layout [S][nz][ny][pitch])
    int S, nx, ny, nz;     // node counts
    int64_t pitch, plane, shot_stride;
    AxisDev ax;
    // step counter: if set, one thread adds 1 at kernel start (first kernel of a step)
    int64_t *step_inc;
    // sources added in the epilogue to out[j] when out_field[j] is one of their fields:
    // out += src_scale * wavelet[*d_step + src_time_offset] * weight (* b for forces)
    const SrcDev *src;
    const int *src_begin;  // [S+1] index of the first source of each shot
    const float *wpool, *wavpool, *bcoef;
    const int64_t *d_step;
    int src_time_offset;
    float src_scale;
    int out_field[3];
    int cw;                // strided kernels: columns per wave (16, 32, 64; 0 = automatic)
    int cx;                // x kernel: nodes per lane (4, 8, 16; 0 = automatic)
    int xl;                // x kernel: lines per wave over whole 16-lane units (2-16; 1: one unit per lane
                           // group; 0 = automatic)
    int cs;                // y/z kernels: nodes per lane (8 or 16; 0 = automatic)
    // receivers of out[0] recorded by the strided kernel as its update lands (trace
    // sample *d_step - 1): per flattened column {first, count, min row, max row} into
    // rrow / rtoff (row along the axis, trace offset), sorted by column
    const int4 *rcol;
    const int *rrow;
    const int64_t *rtoff;
    double *traces;
    int64_t trace_len;
    // absorbing layer: memory variable of this pass (layout of the fields), the per-node
    // exact sub-flow over this pass's time span, [N+1] {e^{-x}, phi1(x),
    // (d/k^2) tau phi1(x), 1/k - (d/k^2) tau phi2(x)} with x = (d/k + alpha) tau, and
    // whether the advanced variable is stored (a pass that only evaluates the field at
    // another time leaves it unchanged)
    float *pml_mem;
    const float4 *pml_tab;
    int pml_store;
};

// Elastic plane pass (plane_xy.hip): one workgroup per (shot, z plane, patch tile of
// the x-y plane).  The tile's nodes sit in LDS; its x lines and y lines are solved from
// there (PMBC taps outside the tile from global memory), and the epilogue combines the
// x and y derivatives of every input with the z derivatives T stored by the z passes.
//   stress (mode 0): in = v1, v2, v3; out = s11, s22, s33, s12, s13, s23;
//     sigma_ii += (l2m) d_i v_i + (lam)(sum of the other two), sigma_ij += (mu)(d_i v_j + d_j v_i)
//     with d3 v_i = T_i; explosive sources on the normal stresses.
//   velocity (mode 1): in = s11, s12, s22, s13, s23; out = v1, v2, v3;
//     v_i += alpha (b) (d1 sigma_i1 + d2 sigma_i2 + T_i) with T_i = d3 sigma_i3; body forces.
// Media hold dt lambda, dt mu, dt (lambda + 2 mu), dt b.  Patch lengths along x and y
// must be at most kPlaneMaxM and the halo at most kPlaneMaxHalo (the tile and its taps
// sit in LDS).
constexpr int kPlaneMaxM = 64;
constexpr int kPlaneMaxHalo = 12;

struct PlaneArgs {
    const float *in[5];
    const float *T[3];
    float *out[6];
    const float *lam, *mu, *l2m, *b;
    float alpha;
    int S, nx, ny, nz;
    int64_t pitch, plane, shot_stride;
    AxisDev ax, ay;
    LineArgs src;          // source fields of the epilogue (src, src_begin, pools, d_step, out_field, ...)
};

hipError_t launch_plane_xy(int mode, const PlaneArgs &a, hipStream_t st);

// Launch helpers (kernels.hip).  axis: 0 = x (contiguous), 1 = y, 2 = z.
hipError_t launch_line(int axis, int solve, int epi, const LineArgs &a, hipStream_t st);
// Adjoint phase 2: Y at the junction rows from the junction rows of T^T, then
// out (+)= alpha * (G^T Y) (EPI as for the line kernels).
hipError_t launch_adj_junctions(int axis, const LineArgs &a, float *Y, hipStream_t st);
hipError_t launch_adj_gather(int axis, int epi, const LineArgs &a, const float *Y, hipStream_t st);
// Fused adjoint x pass (solve, junction rows, gather); hipErrorNotSupported when the
// line does not fit one block or the epilogue is not STORE / AXPY.
hipError_t launch_adj_x(int epi, const LineArgs &a, hipStream_t st);
// Two adjoint x passes in one kernel: a.out[0] += a.alpha Dx^T(a.in_coef a.in), then
// out2 += alpha2 Dx^T(coef2 a.out[0]) with the updated a.out[0]; out2 may be a.in.
hipError_t launch_adj_xx(const LineArgs &a, const float *coef2, float *out2, float alpha2, hipStream_t st);
// Fused x passes of the acoustic step (velocity along x, then T = d v1/dx of the
// updated v1 into Tout): threads per block, 0 when a line does not fit one block.
int line_xx_threads(const LineArgs &a);
hipError_t launch_line_xx(const LineArgs &a, float *Tout, float *pml_mem_t, hipStream_t st);

struct SrcDev {
    int shot, kind, field0, nfield;   // fields field0 .. field0+nfield-1 (consecutive ids)
    int x0, y0, z0, bx, by, bz;       // footprint box (nodes)
    int64_t w_off, wav_off;           // offsets into the weight / wavelet pools
    int nt;
    int force;                        // 1: scale by b (body force), 0: stress rate
};
struct RecDev {
    int shot, comp;
    int64_t node;                     // padded node offset within a shot field
    int64_t trace_off;                // offset of sample 0 in the trace pool
};
// One node that receives trace residuals in the adjoint: the receivers at that node of
// that shot and field are entries first .. first + count - 1 of a trace-offset list, in
// receiver order (so the injection needs no atomics and sums in a fixed order).
struct RecTarget {
    int shot, comp;
    int64_t node;
    int first, count;
};

// adjoint through the absorbing layer (adjoint_layer.hip)
hipError_t launch_pml_adj_operand(float *w, const float *f, const float *coef, float alpha, float *m,
                                  const float4 *tab, int axis, int pml_w, int N, int nx, int ny, int64_t pitch,
                                  int64_t per_shot, int S, hipStream_t st);

// elastic adjoint (adjoint_elastic.hip)
hipError_t launch_el_normal_operand(float *w, const float *s11, const float *s22, const float *s33,
                                    const float *l2m, const float *lam, int k, int nx, int64_t pitch,
                                    int64_t per_shot, int S, hipStream_t st);
hipError_t launch_el_grad_accum(double *gl, double *gm, const float *const *strain, const float *const *sbar,
                                double dt, int nx, int64_t pitch, int64_t per_shot, int S, hipStream_t st);
hipError_t launch_el_grad_unpad(const double *gl, const double *gm, const double *gb, double *g, int nx,
                                int64_t pitch, const float *vp, const float *vs, const float *rho, int mode,
                                int64_t nodes, hipStream_t st);
hipError_t launch_el_grad_b(double *gb, const float *const *ubar, const float *const *div, double dt, int nx,
                            int64_t pitch, int64_t per_shot, int S, hipStream_t st);

hipError_t launch_inject(const SrcDev *src, int nsrc, float *const *fields, const float *b,
                         const float *wpool, const float *wavpool, int64_t shot_stride, int64_t pitch,
                         int64_t plane, const int64_t *d_step, int time_offset, float scale,
                         int want_force, hipStream_t st);
// dJ/db += scale f(t_n) w(x) ubar(x) of every force source; one thread per node of the box
// [x0, x1) x [y0, y1) x [z0, z1) covering all force footprints, sources summed in order
hipError_t launch_el_grad_force(double *gb, const SrcDev *src, int nsrc, float *const *adj, const float *wpool,
                                const float *wavpool, int64_t shot_stride, int64_t pitch, int64_t plane, int64_t n,
                                double scale, const int *box, hipStream_t st);
// field[target] += w * (sum of the target's residual samples n), one thread per target:
// fields = device table of field pointers by field id, or `single` for every target
hipError_t launch_res_gather(const RecTarget *tg, int nt, const int64_t *toff, float *const *fields, float *single,
                             int64_t shot_stride, const double *res, int64_t n, float w, hipStream_t st);
hipError_t launch_record(const RecDev *rec, int nrec, const float *const *fields, int64_t shot_stride,
                         double *traces, const int64_t *d_step, int64_t trace_len, float weight,
                         int accumulate, hipStream_t st);
// two receiver lists in one launch; sample index = *d_step + offset
hipError_t launch_record2(const RecDev *rec0, int nrec0, float w0, int acc0, const RecDev *rec1, int nrec1,
                          float w1, int acc1, const float *const *fields, int64_t shot_stride,
                          double *traces, const int64_t *d_step, int offset, int64_t trace_len,
                          hipStream_t st);
hipError_t launch_advance(int64_t *d_step, hipStream_t st);
hipError_t launch_set_step(int64_t *d_step, int64_t v, hipStream_t st);
// rows = number of x rows (batch * nz * ny); dense <-> padded (row pitch `pitch`)
hipError_t launch_pad_copy(const float *src, float *dst, int nx, int rows, int64_t pitch, int to_padded,
                           hipStream_t st);
hipError_t launch_media(const float *vp, const float *vs, const float *rho, float *const *media,
                        int physics, int nx, int rows, int64_t pitch, double dt, hipStream_t st);
hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t st);
hipError_t launch_axpby(float *y, const float *x, float a, float b, int64_t n, hipStream_t st);
hipError_t launch_grad_accum(double *g, const float *lam, const float *div, float scale, int S,
                             int64_t shot_stride, int64_t n, hipStream_t st);
hipError_t launch_grad_unpad(const double *gp, double *g, int nx, int rows, int64_t pitch, const float *vp,
                             const float *rho, int param, hipStream_t st);
hipError_t launch_nonfinite(const float *p, int64_t n, int *flag, hipStream_t st);
// Wavefield energy of each shot (energy.hip): velocity and stress fields (padded layout,
// shot_stride apart), the dense media vp, vs (elastic only), rho.
struct EnergyArgs {
    const float *v[3];
    const float *s[6];
    int nv, ns;               // acoustic 2, 1 (sigma); elastic 3, 6 (s11 s22 s33 s12 s13 s23)
    const float *vp, *vs, *rho;
    int nx;
    int64_t pitch, shot_stride, nodes;
};
hipError_t launch_energy(const EnergyArgs &a, int S, double *partial, int nblocks, double cell, double *out,
                         hipStream_t st);


}  // namespace loss
