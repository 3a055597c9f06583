// Elastic plane pass (gfx950): the x and y derivatives of a patch tile of one x-y plane
// from LDS, combined with the z derivatives of the same stage in one epilogue.
//
// The velocity-stress system (paper Sec. 2) needs, per Strang sub-flow (Sec. 3.3), the
// derivative of several fields along all three axes.  Passes along one axis at a time
// must park partial sums in full-size temporaries; here the z derivatives of a stage
// are stored first (three strided line passes), and then one workgroup per (shot, z
// plane, patch tile of the plane) loads each input's tile of (M+1) x (M+1) nodes into
// LDS once, solves the tile's x lines and y lines from LDS with the same patch solve as
// the line kernels (x_unit: the PMBC slope from the taps around each junction, Sec. 3.2,
// taps outside the tile read from global memory), and folds the results into the
// outputs.  Each output is read and written once per stage; the inputs are read once
// by the z passes and once here.
//
// Work of one workgroup, per input field f (the next field's tile loads are in flight
// while f is solved):
//   tile(f) -> LDS; x lines of the owned rows -> X tile; y lines of the owned columns ->
//   Y tile; the epilogue over the owned nodes (flattened, consecutive threads on
//   consecutive x) reads X and Y and keeps at most two partial sums per node in
//   registers until the output they feed is complete.
// The owned nodes of patch l along an axis are [s, e) and also N for the last patch.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "line_device.h"
#include "loss_internal.h"
#include "plane_index.h"

namespace loss {

namespace {

constexpr int kPlaneTile = kPlaneMaxM + 1;              // owned nodes per tile side, at most
constexpr int kPlaneWin = kPlaneTile + 2 * kPlaneMaxHalo;   // window side: the tile and its PMBC taps
constexpr int kLoadSlots = (kPlaneWin * kPlaneWin + kPlaneThreads - 1) / kPlaneThreads;
constexpr int kOwnSlots = (kPlaneTile * kPlaneTile + kPlaneThreads - 1) / kPlaneThreads;

template <int MODE>
struct Stage {
    // stress: three inputs, both axes each; velocity: s11 (x), s12 (x, y), s22 (y),
    // s13 (x), s23 (y)
    static constexpr int NF = MODE == 0 ? 3 : 5;
    static constexpr bool xs(int f) { return MODE == 0 || f == 0 || f == 1 || f == 3; }
    static constexpr bool ys(int f) { return MODE == 0 || f == 1 || f == 2 || f == 4; }
};

// Geometry of one workgroup's tile.  The window [wx0, wx1] x [wy0, wy1] holds the tile's
// nodes and the PMBC taps of its junctions (halo nodes beyond each junction; clipped to
// the grid, or on a periodic axis continued across the ends with the wrapped nodes), so
// the line solves read LDS only, at non-negative indices.
struct Tile {
    int shot, zz, lx, ly;
    Span sx, sy;
    int wx0, wx1, wy0, wy1, ww, wh;
    int64_t pbase, fbase;   // node (0, 0) of the plane: media, fields of the shot
    int pitch;
};

// Window loads of one input (kLoadSlots per thread), flat over wh x ww.
__device__ __forceinline__ void load_window(const float *__restrict__ f, const Tile &t, const AxisDev &ax,
                                            const AxisDev &ay, float (&pf)[kLoadSlots])
{
    const float *__restrict__ g = f + t.fbase;
    const int n = t.ww * t.wh;
    const float rw = 1.f / (float)t.ww;
#pragma unroll
    for (int j = 0; j < kLoadSlots; ++j) {
        int r, c;
        split_flat(min((int)threadIdx.x + j * kPlaneThreads, n - 1), t.ww, rw, r, c);
        pf[j] = g[window_node(r, t.wy0, ay.N) * t.pitch + window_node(c, t.wx0, ax.N)];
    }
}

__device__ __forceinline__ void store_window(float *tF, const Tile &t, const float (&pf)[kLoadSlots])
{
    const int n = t.ww * t.wh;
#pragma unroll
    for (int j = 0; j < kLoadSlots; ++j) {
        const int q = threadIdx.x + j * kPlaneThreads;
        if (q < n) tF[q] = pf[j];
    }
}

// Serial solve of patch l of one line of the window (one thread per line): the same
// factors and end rows as the lane-parallel solve of the line kernels (x_unit), applied
// as one forward elimination and one back substitution.  u(i) reads node i of the line
// from the window; y(i) is the LDS slot of node i's result, which holds the eliminated
// value after the forward sweep and the derivative after the back substitution.  Owned
// nodes: [s, e), and e when it is the grid's last node.
template <typename U, typename Y>
__device__ __forceinline__ void line_serial(const AxisDev &ax, int l, const Span &sp, U u, Y y)
{
    constexpr int B = 8;   // rows per batch: their LDS reads are issued before the recurrence
    const int s = sp.s, e = sp.e;
    // PMBC slopes of the patch's junction rows (eq. PMBC; zero at a natural end): all
    // taps read at once
    const int nt = ax.ntap;
    const int ss = slot_first(ax, l), se = slot_last(ax, l, e);
    float phs = 0.f, phe = 0.f;
#pragma unroll
    for (int t = 0; t < 2 * kPlaneMaxHalo + 1; ++t) {
        if (t < nt) {
            if (ss >= 0) phs = fmaf(ax.tap_c[ss * nt + t], u(tap_node(ax, s, t)), phs);
            if (se >= 0) phe = fmaf(ax.tap_c[se * nt + t], u(tap_node(ax, e, t)), phe);
        }
    }
    const EndRows er = end_rows<SOLVE_D1>(ax, s, e);
    // forward elimination: row s takes the slope phs as its carry
    float fm0, fi0, fs0;
    float um = u(s), u0 = u(s + 1);
    float yv = first_row<SOLVE_D1>(ax, er, um, u0, fm0, fi0, fs0);
    yv = fmaf(-fm0, phs, yv);
    y(s) = yv;
    int i = s + 1;
    for (; i + B <= e; i += B) {
        float up[B];
        float2 f[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            up[j] = u(i + j + 1);
            f[j] = ax.lum[i + j];
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            yv = fmaf(-f[j].x, yv, ax.s3 * (up[j] - um));
            y(i + j) = yv;
            um = u0;
            u0 = up[j];
        }
    }
    for (; i < e; ++i) {
        const float up = u(i + 1);
        yv = fmaf(-ax.lum[i].x, yv, ax.s3 * (up - um));
        y(i) = yv;
        um = u0;
        u0 = up;
    }
    // closing row e, then the back substitution (interior rows have sup = 1)
    float wv = last_row<SOLVE_D1>(ax, er, yv, um, u0, phe);
    if (e == ax.N) y(e) = wv;
    i = e - 1;
    for (; i - B >= s; i -= B) {
        float yy[B], iv[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            yy[j] = y(i - j);
            iv[j] = ax.lum[i - j].y;
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            wv = (yy[j] - wv) * iv[j];
            y(i - j) = wv;
        }
    }
    for (; i > s; --i) {
        wv = (y(i) - wv) * ax.lum[i].y;
        y(i) = wv;
    }
    y(s) = fmaf(-fs0, wv, y(s)) * fi0;
}

// x lines of the owned rows (waves 0, 1) and y lines of the owned columns (waves 2, 3)
// of the window in tF -> tX, tY
template <bool XS, bool YS>
__device__ __forceinline__ void solve_tile(const AxisDev &ax, const AxisDev &ay, const Tile &t, const float *tF,
                                           float *tX, float *tY)
{
    const int tid = threadIdx.x;
    if (XS && tid < 128 && tid < t.sy.n) {
        const int r = tid;
        const float *rl = tF + (t.sy.s + r - t.wy0) * t.ww;
        float *xo = tX + r * kPlaneTile - t.sx.s;
        const int wx0 = t.wx0, ww = t.ww, N = ax.N;
        line_serial(ax, t.lx, t.sx, [&](int i) { return rl[window_pos(i, wx0, ww, N)]; },
                    [&](int i) -> float & { return xo[i]; });
    } else if (YS && tid >= 128 && tid < 256 && tid - 128 < t.sx.n) {
        const int c = tid - 128;
        const float *cl = tF + (t.sx.s + c - t.wx0);
        float *yo = tY + c - t.sy.s * kPlaneTile;
        const int wy0 = t.wy0, wh = t.wh, ww = t.ww, N = ay.N;
        line_serial(ay, t.ly, t.sy, [&](int i) { return cl[window_pos(i, wy0, wh, N) * ww]; },
                    [&](int i) -> float & { return yo[i * kPlaneTile]; });
    }
}

// One input field FI of the stage: window to LDS (the next field's loads issued), the
// solves, the epilogue.
template <int MODE, int FI>
__device__ __forceinline__ void plane_field(const PlaneArgs &a, const Tile &t, float *sm, float (&pf)[kLoadSlots],
                                            float (&A)[kOwnSlots], float (&B)[kOwnSlots])
{
    using St = Stage<MODE>;
    float *tX = sm, *tY = sm + kPlaneTile * kPlaneTile, *tF = sm + 2 * kPlaneTile * kPlaneTile;
    __syncthreads();   // the previous solves have read the window, the previous epilogue X and Y
    store_window(tF, t, pf);
    if constexpr (FI + 1 < St::NF) load_window(a.in[FI + 1], t, a.ax, a.ay, pf);
    __syncthreads();
    solve_tile<St::xs(FI), St::ys(FI)>(a.ax, a.ay, t, tF, tX, tY);
    __syncthreads();
    const int nown = t.sy.n * t.sx.n;
    const float rsn = 1.f / (float)t.sx.n;
#pragma unroll
    for (int j = 0; j < kOwnSlots; ++j) {
        const int q = threadIdx.x + j * kPlaneThreads;
        if (q >= nown) continue;
        int r, c;
        split_flat(q, t.sx.n, rsn, r, c);
        float dx = 0.f, dy = 0.f;
        if constexpr (St::xs(FI)) dx = tX[r * kPlaneTile + c];
        if constexpr (St::ys(FI)) dy = tY[r * kPlaneTile + c];
        const int gx = t.sx.s + c, gy = t.sy.s + r;
        const int off = gy * t.pitch + gx;    // node within the plane
        if constexpr (MODE == 0) {
            if constexpr (FI == 0) {          // v1: keep d1 v1, d2 v1
                A[j] = dx;
                B[j] = dy;
            } else if constexpr (FI == 1) {   // v2: sigma12, and the normal stresses (d3 v3 is T2)
                float *o12 = a.out[3] + t.fbase;
                const float mu = a.mu[t.pbase + off];
                const float tt[3] = {A[j], dy, a.T[2][t.fbase + off]};
                const float l2m = a.l2m[t.pbase + off], lam = a.lam[t.pbase + off];
                o12[off] = fmaf(mu, B[j] + dx, o12[off]);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    float *oi = a.out[i] + t.fbase;
                    const float other = i == 0 ? tt[1] + tt[2] : (i == 1 ? tt[0] + tt[2] : tt[0] + tt[1]);
                    float v = fmaf(l2m, tt[i], lam * other) + oi[off];
                    if (a.src.src) v += source_terms(a.src, i, t.shot, gx, gy, t.zz, t.pbase + off);
                    oi[off] = v;
                }
            } else {                          // v3: sigma13, sigma23
                const float mu = a.mu[t.pbase + off];
                float *o13 = a.out[4] + t.fbase, *o23 = a.out[5] + t.fbase;
                o13[off] = fmaf(mu, a.T[0][t.fbase + off] + dx, o13[off]);
                o23[off] = fmaf(mu, a.T[1][t.fbase + off] + dy, o23[off]);
            }
        } else {
            // v_i += alpha (dt b) ((d1 sigma_i1 + d2 sigma_i2) + d3 sigma_i3)
            auto vel = [&](int i, float sum) {
                float *oi = a.out[i] + t.fbase;
                float v = fmaf(a.alpha * a.b[t.pbase + off], sum + a.T[i][t.fbase + off], oi[off]);
                if (a.src.src) v += source_terms(a.src, i, t.shot, gx, gy, t.zz, t.pbase + off);
                oi[off] = v;
            };
            if constexpr (FI == 0) {          // s11: d1
                A[j] = dx;
            } else if constexpr (FI == 1) {   // s12: v1 complete; keep d1 s12
                vel(0, A[j] + dy);
                A[j] = dx;
            } else if constexpr (FI == 2) {   // s22: v2 complete
                vel(1, A[j] + dy);
            } else if constexpr (FI == 3) {   // s13: d1
                A[j] = dx;
            } else {                          // s23: v3 complete
                vel(2, A[j] + dy);
            }
        }
    }
}

// Four waves per SIMD: two workgroups per CU.
template <int MODE>
__global__ void __launch_bounds__(kPlaneThreads, 4) k_plane_xy(PlaneArgs a, int nreal)
{
    extern __shared__ float sm[];
    // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous range of (shot, plane) rows of tiles, tiles fastest, so that the PMBC
    // taps one tile reads from its neighbours are in the same L2.
    const int lin = (int)((blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3));
    if (lin >= nreal) return;   // padding block (uniform across the block)
    const AxisDev &ax = a.ax, &ay = a.ay;
    const int ntiles = ax.p * ay.p;
    Tile t;
    const int tile = lin % ntiles;
    const int pz = lin / ntiles;   // shot * nz + z
    t.shot = pz / a.nz;
    t.zz = pz - t.shot * a.nz;
    t.lx = tile % ax.p;
    t.ly = tile / ax.p;
    t.sx = span_of(ax.N, ax.M, t.lx);
    t.sy = span_of(ay.N, ay.M, t.ly);
    window_of(t.sx, ax.N, ax.halo, ax.periodic, t.wx0, t.wx1);
    window_of(t.sy, ay.N, ay.halo, ay.periodic, t.wy0, t.wy1);
    t.ww = t.wx1 - t.wx0 + 1;
    t.wh = t.wy1 - t.wy0 + 1;
    t.pitch = (int)a.pitch;
    t.pbase = (int64_t)t.zz * a.plane;
    t.fbase = (int64_t)t.shot * a.shot_stride + t.pbase;
    float pf[kLoadSlots], A[kOwnSlots], B[kOwnSlots];
#pragma unroll
    for (int j = 0; j < kOwnSlots; ++j) A[j] = B[j] = 0.f;
    load_window(a.in[0], t, ax, ay, pf);
    plane_field<MODE, 0>(a, t, sm, pf, A, B);
    plane_field<MODE, 1>(a, t, sm, pf, A, B);
    plane_field<MODE, 2>(a, t, sm, pf, A, B);
    if constexpr (MODE == 1) {
        plane_field<MODE, 3>(a, t, sm, pf, A, B);
        plane_field<MODE, 4>(a, t, sm, pf, A, B);
    }
}

}  // namespace

hipError_t launch_plane_xy(int mode, const PlaneArgs &a, hipStream_t st)
{
    const AxisDev &ax = a.ax, &ay = a.ay;
    if (ax.M > kPlaneMaxM || ay.M > kPlaneMaxM || ax.halo > kPlaneMaxHalo || ay.halo > kPlaneMaxHalo)
        return hipErrorInvalidValue;
    const int ntiles = ax.p * ay.p;
    const int64_t nreal = (int64_t)ntiles * a.nz * a.S;
    if (nreal >= (1ll << 31) - 8) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((nreal + 7) / 8 * 8);
    const int wx = ax.periodic ? ax.M + 1 + 2 * ax.halo : std::min(ax.N + 1, ax.M + 1 + 2 * ax.halo);
    const int wy = ay.periodic ? ay.M + 1 + 2 * ay.halo : std::min(ay.N + 1, ay.M + 1 + 2 * ay.halo);
    const size_t shm = (2 * (size_t)kPlaneTile * kPlaneTile + (size_t)wx * wy) * sizeof(float);
    if (mode == 0)
        hipLaunchKernelGGL(k_plane_xy<0>, blocks, kPlaneThreads, shm, st, a, (int)nreal);
    else
        hipLaunchKernelGGL(k_plane_xy<1>, blocks, kPlaneThreads, shm, st, a, (int)nreal);
    return hipGetLastError();
}

}  // namespace loss
