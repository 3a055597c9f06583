// HIP kernels (gfx950) of the local spline simulator.
//
// Line kernels: one work unit = one patch of one grid line (paper Sec. 3.2: the
// patches are coupled only through the junction slopes phi).  A unit's nodes
// [s, e) are split into chunks of C consecutive nodes, one chunk per lane; the
// closing row e (the next junction, or the natural end N) is handled by the lane
// that holds e-1.  The tridiagonal solve (LU factors from the axis table) runs as
// two first-order linear recurrences (forward elimination, back substitution);
// each lane runs them over its chunk in registers from a zero carry, records the
// affine map carry_out = A * carry_in + B, and the carries are composed across the
// unit (wave shuffles for the contiguous x axis, LDS across waves for y and z),
// then every lane adds A_local * carry_in.  The derivative is fused with the
// field update (epilogue).
//
// Two properties of the factors keep the kernels short:
//  * the junction value of a patch (the PMBC slope, or its Hermite moment row)
//    enters the first row of the patch linearly, so it is the carry into the
//    patch: the slope's halo sum is formed while the chunks eliminate;
//  * the elimination factors of the [1 4 1] rows are at most about 0.29, so the
//    carry into a chunk depends on chunks more than `reach` rows back only through
//    a product below 2^-44 (the axis table computes reach from the factors): the
//    kernels compose the maps of the chunks within reach only.
// Every global load of a lane (its nodes, factor rows, PMBC taps and the epilogue
// operands) is issued before the solve, so a wave waits on memory once.
//
//   x axis: lanes own C = 4, 8 or 16 consecutive x nodes; G lanes per unit (power of 2).
//   y, z axes: lanes own one x column each (coalesced), lane groups of a block own
//             consecutive chunks of the unit along the axis.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "line_device.h"
#include "loss_internal.h"

namespace loss {

namespace {

template <int C, int SOLVE, int EPI>
__global__ void __launch_bounds__(256) k_line_x(LineArgs a, int G, int nunits)
{
    const AxisDev &ax = a.ax;
    const int lane = threadIdx.x & 63;
    const int lg = __builtin_ctz((unsigned)G);   // G is a power of two
    const int k = lane & (G - 1);
    const int upw = 64 >> lg;                     // units per wave
    const int N = ax.N, M = ax.M, p = ax.p;
    const int lps = a.nz * a.ny;                  // lines per shot
    // the wave's first unit, its line and shot (wave-uniform: scalar divisions)
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int u0 = (blockIdx.x * (blockDim.x >> 6) + wid) * upw;
    if (a.step_inc && blockIdx.x == 0 && threadIdx.x == 0) *a.step_inc += 1;
    if (u0 >= nunits) return;                     // the whole wave is past the last unit
    const int line0 = u0 / p;
    const int shot0 = line0 / lps;
    const int rl0 = line0 - shot0 * lps;
    // this lane's unit (lanes past the last unit repeat it): patch l of line line0 + dl
    const bool uact = (lane >> lg) < nunits - u0;
    int l = u0 - line0 * p + min(lane >> lg, nunits - 1 - u0), dl = 0;
    while (l >= p) { l -= p; ++dl; }
    int rl = rl0 + dl, shot = shot0;              // line within its shot
    while (rl >= lps) { rl -= lps; ++shot; }
    const int pitch = (int)a.pitch;
    const int64_t base = (int64_t)line0 * a.pitch + dl * pitch;   // scalar part + 32-bit lane part
    const int64_t mbase = rl * pitch;
    const int s = l * M;
    const int e = min(s + M, N);
    const int q = s + k * C;
    const float *__restrict__ in = a.in + base;

    // epilogue operands of the aligned whole-chunk case, source flag
    const bool vec = ((q & 3) == 0) && q + C <= e;
    Pre4 pre[C / 4];
    int rowz = 0, rowy = 0;                       // coordinates, only for source terms
    bool srcs = false;
    auto issue = [&]() {
        if (vec) {
#pragma unroll
            for (int g4 = 0; g4 < C / 4; ++g4) pre[g4] = pre_load4<EPI>(a, base + q + 4 * g4, mbase + q + 4 * g4);
        }
        if (a.src) {
            // (y, z) of the line from those of the wave's first line (scalar division)
            const int rz0 = rl0 / a.ny;
            rowz = rz0;
            rowy = rl0 - rz0 * a.ny + dl;
            if (shot != shot0) { rowz = 0; rowy = rl; }
            while (rowy >= a.ny) { rowy -= a.ny; ++rowz; }
            srcs = segment_has_source(a, shot, 0, 0, rowy, rowz, q, min(q + C, N));
        }
    };
    float w[C];
    const bool has_icf = a.in_coef != nullptr;    // uniform
    const float *__restrict__ icf = a.in_coef + mbase;
    auto val = [&](int i) { return has_icf ? in[i] * icf[i] : in[i]; };
    auto val4 = [&](int i) {
        float4 v = ld4(in + i);
        if (has_icf) {
            const float4 c = ld4(icf + i);
            v = make_float4(v.x * c.x, v.y * c.y, v.z * c.z, v.w * c.w);
        }
        return v;
    };
    // whole patches of 16 lanes (one DPP row each) take the unmasked solve; the choice is
    // per unit, the same in every kernel that solves x units, so that a unit's bits do not
    // depend on the kernel (a wave of whole units runs that path alone)
    float we;
    if (G == 16 && M == 16 * C && (l + 1) * M <= N)
        we = x_unit<C, SOLVE, true>(ax, k, G, l, true, val, val4, issue, w);
    else
        we = x_unit<C, SOLVE, false>(ax, k, G, l, true, val, val4, issue, w);

    if (uact) {
        const int kc = (e - 1 - s) / C;
        if (a.pml_mem) {
            pml_run<C>(ax, a.pml_tab, a.pml_mem, a.pml_store, q, e, base + q, 1, w);
            if (e == N && k == kc && in_pml(ax, N)) we = pml_adjust(a.pml_tab, a.pml_mem, a.pml_store, N, base + N, we);
        }
        if (vec) {
#pragma unroll
            for (int g4 = 0; g4 < C / 4; ++g4)
                epilogue4<EPI>(a, base + q + 4 * g4, mbase + q + 4 * g4, shot,
                               make_float4(w[4 * g4], w[4 * g4 + 1], w[4 * g4 + 2], w[4 * g4 + 3]), pre[g4],
                               q + 4 * g4, rowy, rowz, srcs);
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int i = q + c;
                if (i < e) epilogue<EPI>(a, base + i, mbase + i, shot, w[c], i, rowy, rowz, srcs);
            }
        }
        if (e == N && k == kc) epilogue<EPI>(a, base + N, mbase + N, shot, we, N, rowy, rowz, srcs);
    }
}

// x pass over whole units of 16 lanes (M = 16 C, N a multiple of M, p a multiple of the
// four units of a wave): a wave solves the same four patches on `lpw` consecutive lines
// (of any shots), so the patch's row factors, end rows, tap coefficients and tap nodes
// are read once per wave, and the line, its shot and its media row are wave-uniform.
// The next line's loads are issued before the current line is solved.  The same
// arithmetic as k_line_x (whose units take the same unmasked solve), so the bits agree.
template <int C, int SOLVE, int EPI>
__global__ void __launch_bounds__(256) k_line_xl(LineArgs a, int lpw, int nwaves)
{
    const AxisDev &ax = a.ax;
    const int lane = threadIdx.x & 63;
    const int k = lane & 15;
    const int N = ax.N, p = ax.p;
    const int lps = a.nz * a.ny;
    const int64_t nlines = (int64_t)a.S * lps;
    const int w = (int)(blockIdx.x * (blockDim.x >> 6)) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (a.step_inc && blockIdx.x == 0 && threadIdx.x == 0) *a.step_inc += 1;
    if (w >= nwaves) return;
    const int bpl = p >> 2;                      // four-unit blocks per line
    const int g = w / bpl;                       // line group (wave-uniform)
    const int l = (w - g * bpl) * 4 + (lane >> 4);
    const int64_t L0 = (int64_t)g * lpw;
    const int nl = (int)min((int64_t)lpw, nlines - L0);
    const XFix<C, SOLVE> f = x_fix<C, SOLVE, true>(ax, k, 16, l);
    const int q = f.q, e = f.e;
    const int pitch = (int)a.pitch;
    int shot = (int)(L0 / lps);
    int rl = (int)(L0 - (int64_t)shot * lps);
    const bool has_icf = a.in_coef != nullptr;

    // the loads of line L (row rl of its shot): node values and epilogue operands
    struct LineLoads {
        XVals<C> v;
        Pre4 pre[C / 4];
    };
    auto load = [&](int64_t L, int r) {
        const float *__restrict__ in = a.in + L * pitch;
        const float *__restrict__ icf = a.in_coef + (int64_t)r * pitch;
        auto val = [&](int i) { return has_icf ? in[i] * icf[i] : in[i]; };
        auto val4 = [&](int i) {
            float4 x = ld4(in + i);
            if (has_icf) {
                const float4 c = ld4(icf + i);
                x = make_float4(x.x * c.x, x.y * c.y, x.z * c.z, x.w * c.w);
            }
            return x;
        };
        LineLoads ll;
        x_vals_chunk<C, true>(ax, q, k, 16, true, val, val4, ll.v);
        x_vals_taps<C, SOLVE, true>(ax, f, k, 16, val, ll.v);
#pragma unroll
        for (int g4 = 0; g4 < C / 4; ++g4)
            ll.pre[g4] = pre_load4<EPI>(a, L * pitch + q + 4 * g4, (int64_t)r * pitch + q + 4 * g4);
        return ll;
    };
    LineLoads cur = load(L0, rl);
    for (int i = 0; i < nl; ++i) {
        const int64_t L = L0 + i;
        const int64_t base = L * pitch;
        const int64_t mbase = (int64_t)rl * pitch;
        int rn = rl + 1, sn = shot;                  // the next line's row and shot
        if (rn == lps) { rn = 0; ++sn; }
        LineLoads nxt;
        if (i + 1 < nl) nxt = load(L + 1, rn);
        const float *__restrict__ in = a.in + base;
        const float *__restrict__ icf = a.in_coef + mbase;
        auto val = [&](int j) { return has_icf ? in[j] * icf[j] : in[j]; };
        float wv[C];
        float we = x_solve<C, SOLVE, true>(ax, f, cur.v, k, 16, val, wv);
        int rowz = 0, rowy = 0;
        bool srcs = false;
        if (a.src) {
            rowz = rl / a.ny;
            rowy = rl - rowz * a.ny;
            srcs = segment_has_source(a, shot, 0, 0, rowy, rowz, q, min(q + C, N));
        }
        if (a.pml_mem) {
            pml_run<C>(ax, a.pml_tab, a.pml_mem, a.pml_store, q, e, base + q, 1, wv);
            if (e == N && k == 15 && in_pml(ax, N)) we = pml_adjust(a.pml_tab, a.pml_mem, a.pml_store, N, base + N, we);
        }
#pragma unroll
        for (int g4 = 0; g4 < C / 4; ++g4)
            epilogue4<EPI>(a, base + q + 4 * g4, mbase + q + 4 * g4, shot,
                           make_float4(wv[4 * g4], wv[4 * g4 + 1], wv[4 * g4 + 2], wv[4 * g4 + 3]), cur.pre[g4],
                           q + 4 * g4, rowy, rowz, srcs);
        if (e == N && k == 15) epilogue<EPI>(a, base + N, mbase + N, shot, we, N, rowy, rowz, srcs);
        if (i + 1 < nl) cur = nxt;
        rl = rn;
        shot = sn;
    }
}

// Velocity pass along x of one step fused with the stress pass along x of the next
// (acoustic, no body forces): v1 += alpha * coef0 * d(in)/dx, then Tout = d v1/dx of
// the updated v1.  One block holds every patch of one line (p*G lanes), so the
// updated line stays in LDS between the two solves and the stress pass reads its
// PMBC halos there.  Dynamic LDS: N + 1 floats.
template <int C>
__global__ void __launch_bounds__(512) k_line_xx(LineArgs a, float *__restrict__ Tout, float *__restrict__ pml_t,
                                                 int G)
{
    extern __shared__ float4 lds4[];
    float *line_s = reinterpret_cast<float *>(lds4);
    const AxisDev &ax = a.ax;
    const int N = ax.N, M = ax.M, p = ax.p;
    const int k = threadIdx.x & (G - 1);
    const int lraw = threadIdx.x / G;
    const bool uact = lraw < p;
    const int l = min(lraw, p - 1);
    const int line = blockIdx.x;
    const int lps = a.nz * a.ny;
    const int shot = line / lps;
    const int64_t base = (int64_t)line * a.pitch;
    const int64_t mbase = (int64_t)(line - shot * lps) * a.pitch;
    // the stress pass opens the next step (the velocity pass reads no step counter)
    if (a.step_inc && blockIdx.x == 0 && threadIdx.x == 0) *a.step_inc += 1;
    const int s = l * M;
    const int e = min(s + M, N);
    const int q = s + k * C;
    const int kc = (e - 1 - s) / C;
    const float *__restrict__ in = a.in + base;
    float *__restrict__ v1 = a.out[0] + base;
    const float *__restrict__ cf = a.coef[0] ? a.coef[0] + mbase : nullptr;

    // ---- velocity pass -------------------------------------------------------
    const bool vec = ((q & 3) == 0) && q + C <= e;
    Pre4 pre[C / 4];
    auto issue = [&]() {
        if (vec) {
#pragma unroll
            for (int g4 = 0; g4 < C / 4; ++g4) pre[g4] = pre_load4<EPI_AXPY>(a, base + q + 4 * g4, mbase + q + 4 * g4);
        }
    };
    float w[C];
    const bool full16 = G == 16 && M == 16 * C && (l + 1) * M <= N;   // as in k_line_x
    auto gval = [&](int i) { return in[i]; };
    auto gval4 = [&](int i) { return ld4(in + i); };
    float we = full16 ? x_unit<C, SOLVE_D1, true>(ax, k, G, l, true, gval, gval4, issue, w)
                      : x_unit<C, SOLVE_D1, false>(ax, k, G, l, true, gval, gval4, issue, w);
    if (uact) {
        if (a.pml_mem) {
            pml_run<C>(ax, a.pml_tab, a.pml_mem, 1, q, e, base + q, 1, w);
            if (e == N && k == kc && in_pml(ax, N)) we = pml_adjust(a.pml_tab, a.pml_mem, 1, N, base + N, we);
        }
        if (vec) {
#pragma unroll
            for (int g4 = 0; g4 < C / 4; ++g4) {
                const float4 v = fma4(a.alpha, pre[g4].c, make_float4(w[4 * g4], w[4 * g4 + 1], w[4 * g4 + 2],
                                                                      w[4 * g4 + 3]), pre[g4].o);
                st4(v1 + q + 4 * g4, v);
                lds4[(q >> 2) + g4] = v;
            }
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int i = q + c;
                if (i < e) {
                    const float v = fmaf(a.alpha * (cf ? cf[i] : 1.f), w[c], v1[i]);
                    v1[i] = v;
                    line_s[i] = v;
                }
            }
        }
        if (e == N && k == kc) {
            const float v = fmaf(a.alpha * (cf ? cf[N] : 1.f), we, v1[N]);
            v1[N] = v;
            line_s[N] = v;
        }
    }
    __syncthreads();

    // ---- stress pass: T = d v1 / dx from the line in LDS ------------------------
    auto lval = [&](int i) { return line_s[i]; };
    auto lval4 = [&](int i) { return lds4[i >> 2]; };
    auto none = [] {};
    we = full16 ? x_unit<C, SOLVE_D1, true>(ax, k, G, l, true, lval, lval4, none, w)
                : x_unit<C, SOLVE_D1, false>(ax, k, G, l, true, lval, lval4, none, w);
    if (uact) {
        float *__restrict__ T = Tout + base;
        if (pml_t) {
            pml_run<C>(ax, a.pml_tab, pml_t, 1, q, e, base + q, 1, w);
            if (e == N && k == kc && in_pml(ax, N)) we = pml_adjust(a.pml_tab, pml_t, 1, N, base + N, we);
        }
        if (vec) {
#pragma unroll
            for (int g4 = 0; g4 < C / 4; ++g4)
                st4(T + q + 4 * g4, make_float4(w[4 * g4], w[4 * g4 + 1], w[4 * g4 + 2], w[4 * g4 + 3]));
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (q + c < e) T[q + c] = w[c];
        }
        if (e == N && k == kc) T[N] = we;
    }
}

// ---------------------------------------------------------------------------
// y / z axes (strided).
// ---------------------------------------------------------------------------
constexpr int kMaxWaves = 16;
constexpr int kTapChunks = 16;     // chunks of a unit that share the PMBC taps
constexpr int kTapsPerChunk = 2;   // taps per chunk loaded ahead of the solve

// Columns are the flattened (shot, other coordinate, x) positions of the lines: one
// lane per column, CW consecutive columns per wave (64, 32, 16 or 8), the 64/CW lane
// groups of a wave and the waves of the block holding consecutive chunks of C nodes
// along the axis.  Chunk maps and PMBC partial sums meet in LDS: two barriers.
// WIDE (CW = 64, one chunk per wave): the chunk index and so the factor rows are
// wave-uniform (scalar loads, no vector registers for the factors), and the column
// decomposition is done once per wave.  Register bounds (measured on 513^3): the
// 64-column store and axpy with aux fit 8 waves per SIMD (63-64 VGPRs, four workgroups
// per CU; the axpy spills one register) and the normal stresses 7 (70 VGPRs); tighter
// bounds on the other epilogues spill more and run slower.
// Dynamic LDS: 6 * blockDim.x + 64 floats.
template <int C, int SOLVE, int EPI, bool WIDE>
__global__ void __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu((EPI == EPI_STORE || EPI == EPI_AXPY_AUX) && WIDE && C == 8
                                       ? 8
                                       : (EPI == EPI_NORMAL3 && WIDE && C == 8 ? 7 : 1))))
k_line_s(LineArgs a, int axis, int CW_, int gx_real)
{
    extern __shared__ float lds[];
    const int nthr = blockDim.x;
    float *sA = lds, *sB = lds + nthr, *sPs = lds + 2 * nthr, *sPe = lds + 3 * nthr;
    float *sQ = lds + 4 * nthr, *sW = lds + 5 * nthr, *sWe = lds + 6 * nthr;
    const AxisDev &ax = a.ax;
    // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, so give each XCD
    // a contiguous range of column groups (neighbouring groups share cache lines and
    // PMBC halo rows in that XCD's L2).  gridDim.x is padded to a multiple of 8.
    int bx, by;
    {
        const int total = gridDim.x * gridDim.y;
        const int lin = blockIdx.y * gridDim.x + blockIdx.x;
        const int logical = (lin & 7) * (total >> 3) + (lin >> 3);
        by = logical / (int)gridDim.x;
        bx = logical - by * (int)gridDim.x;
    }
    if (bx >= gx_real) return;   // padding block (uniform across the block)
    const int CW = WIDE ? 64 : CW_;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int SUB = WIDE ? 1 : 64 / CW;
    const int NCH = (nthr >> 6) * SUB;
    const int ci = lane & (CW - 1);
    const int chunk = WIDE ? __builtin_amdgcn_readfirstlane(wv) : wv * SUB + lane / CW;
    const int me = chunk * CW + ci;
    const int n_other = (axis == 1) ? a.nz : a.ny;
    const int pitch = (int)a.pitch;
    const int per_shot = n_other * pitch;
    const int fcol = bx * CW + ci;
    int shot0, o, col;
    if constexpr (WIDE) {
        // first column of the wave, then step this lane's column across row ends
        const int f0 = bx * 64;
        shot0 = f0 / per_shot;
        const int r0 = f0 - shot0 * per_shot;
        o = r0 / pitch;
        col = r0 - o * pitch + lane;
        while (col >= pitch) {
            col -= pitch;
            if (++o == n_other) { o = 0; ++shot0; }
        }
    } else {
        shot0 = fcol / per_shot;
        const int rem = fcol - shot0 * per_shot;
        o = rem / pitch;
        col = rem - o * pitch;
    }
    const bool cact = col < a.nx && shot0 < a.S;
    const int shot = min(shot0, a.S - 1);
    const int l = by;
    const int stride = (axis == 1) ? pitch : (int)a.plane;
    const int mbase = ((axis == 1) ? o * (int)a.plane : o * pitch) + min(col, a.nx - 1);
    const int64_t sbase = (int64_t)shot * a.shot_stride;   // start of the shot's field
    if (a.step_inc && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *a.step_inc += 1;
    // WIDE: the array pointers move to the lane's column once, so that the node indices
    // below are row offsets, wave-uniform (scalar), and every access costs one address
    // add; otherwise the indices carry the column (fo: fields, mo: media)
    const LineArgs la = WIDE ? lane_args(a, sbase + mbase, mbase, shot) : a;
    const int64_t fo = WIDE ? 0 : sbase + mbase;
    const int64_t mo = WIDE ? 0 : mbase;
    const float *__restrict__ in = la.in;
    const float *__restrict__ icf = la.in_coef;
    const int N = ax.N, M = ax.M;
    const int s = l * M;
    const int e = min(s + M, N);
    const int q = s + chunk * C;

    // ---- loads -------------------------------------------------------------
    float u[C + 2];
#pragma unroll
    for (int c = 0; c < C + 2; ++c) {
        const int r = clampi(q - 1 + c, 0, N) * stride;
        u[c] = a.in_coef ? in[fo + r] * icf[mo + r] : in[fo + r];
    }
    const int4 rinfo = (a.rcol && cact) ? a.rcol[fcol] : make_int4(0, 0, 0, -1);
    float fm[C], fi[C], fs[C];
    row_factors<C, SOLVE>(ax, q, fm, fi, fs);
    const EndRows er = end_rows<SOLVE>(ax, s, e);
    // PMBC partial sums of rows s and e: the first T chunks share the taps, chunk j
    // taking taps j, j+T, ... (kTapsPerChunk of them without a wait in between)
    const int T = min(NCH, kTapChunks);
    const int nt = ax.ntap;
    const int ss = slot_first(ax, l), se = slot_last(ax, l, e);
    float tcs[kTapsPerChunk] = {}, tvs[kTapsPerChunk] = {}, tce[kTapsPerChunk] = {}, tve[kTapsPerChunk] = {};
    if (SOLVE != SOLVE_T1 && chunk < T) {
#pragma unroll
        for (int h = 0; h < kTapsPerChunk; ++h) {
            const int t = min(chunk + h * T, nt - 1);
            tcs[h] = ax.tap_c[max(ss, 0) * nt + t];
            tce[h] = ax.tap_c[max(se, 0) * nt + t];
            tvs[h] = in[fo + tap_node(ax, s, t) * stride];
            tve[h] = in[fo + tap_node(ax, e, t) * stride];
        }
    }
    // epilogue operands (small chunks only: they cost 3 registers per node); the 64-column
    // axpy with aux loads them after the solve, which lets it run four workgroups per CU
    // (64 VGPRs) instead of two (101), the faster on 513^3
    constexpr bool kPre = C <= 8 && EPI != EPI_NORMAL3 && !(WIDE && EPI == EPI_AXPY_AUX);
    Pre pre[kPre ? C : 1];
    if constexpr (kPre) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int r = min(q + c, N) * stride;
            pre[c] = pre_load<EPI>(la, fo + r, mo + r);
        }
    }
    float ps = 0.f, pe = 0.f;
    if constexpr (SOLVE != SOLVE_T1) {
        if (chunk < T) {
#pragma unroll
            for (int h = 0; h < kTapsPerChunk; ++h) {
                const bool ok = chunk + h * T < nt;
                if (ss >= 0 && ok) ps = fmaf(tcs[h], tvs[h], ps);
                if (se >= 0 && ok) pe = fmaf(tce[h], tve[h], pe);
            }
            for (int t = chunk + kTapsPerChunk * T; t < nt; t += T) {   // wide halos
                if (ss >= 0) ps = fmaf(ax.tap_c[ss * nt + t], in[fo + tap_node(ax, s, t) * stride], ps);
                if (se >= 0) pe = fmaf(ax.tap_c[se * nt + t], in[fo + tap_node(ax, e, t) * stride], pe);
            }
        }
    }

    // ---- forward elimination: chunk maps (values recomputed from the carry) ------
    float yv = 0.f, pv = 1.f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float r = interior_rhs<SOLVE>(ax, u[c], u[c + 1], u[c + 2]);
        if constexpr (SOLVE != SOLVE_T1) {
            if (c == 0 && chunk == 0) r = first_row<SOLVE>(ax, er, u[1], u[2], fm[0], fi[0], fs[0]);
        }
        yv = fmaf(-fm[c], yv, r);
        pv = -fm[c] * pv;
    }
    sA[me] = pv;
    sB[me] = yv;
    sPs[me] = ps;
    sPe[me] = pe;
    __syncthreads();
    // carry: the maps of the chunks within reach, from the junction slope when the
    // window starts at the unit's first chunk
    const int Dc = (ax.reach + C - 1) / C;
    const int j0 = max(0, chunk - Dc);
    float yin = 0.f;
    if (SOLVE != SOLVE_T1 && j0 == 0) {
        for (int j = 0; j < T; ++j) yin += sPs[j * CW + ci];
    }
    for (int j = j0; j < chunk; ++j) yin = fmaf(sA[j * CW + ci], yin, sB[j * CW + ci]);
    float y[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float r = interior_rhs<SOLVE>(ax, opaque(u[c]), opaque(u[c + 1]), opaque(u[c + 2]));
        if constexpr (SOLVE != SOLVE_T1) {
            if (c == 0 && chunk == 0)
                r = first_row<SOLVE>(ax, er, opaque(u[1]), opaque(u[2]), fm[0], fi[0], fs[0]);
        }
        yin = fmaf(-fm[c], yin, r);
        y[c] = yin;
    }

    const int kc = (e - 1 - s) / C, cc = (e - 1 - s) - kc * C;
    if (chunk == kc) {
        float ylast = 0.f, ulast = 0.f, ue = 0.f;
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (c == cc) { ylast = y[c]; ulast = u[c + 1]; ue = u[c + 2]; }
        float phe = 0.f;
        if (SOLVE != SOLVE_T1)
            for (int j = 0; j < T; ++j) phe += sPe[j * CW + ci];
        sWe[ci] = last_row<SOLVE>(ax, er, ylast, ulast, ue, phe);
    }

    // ---- back substitution: chunk maps, composition, values (into y) -------------
    float wvv = 0.f, qv = 1.f;
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        if (q + c < e) {
            wvv = fmaf(-fs[c], wvv, y[c]) * fi[c];
            qv = -fs[c] * fi[c] * qv;
        }
    }
    sQ[me] = qv;
    sW[me] = wvv;
    __syncthreads();
    const float we = sWe[ci];
    float wr = we;   // chunks past kc hold identity maps
    for (int j = min(NCH - 1, chunk + Dc); j > chunk; --j) wr = fmaf(sQ[j * CW + ci], wr, sW[j * CW + ci]);
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        if (q + c < e) wr = fmaf(-fs[c], wr, y[c]) * fi[c];
        y[c] = wr;
    }

    if (cact) {
        if (a.pml_mem)
            pml_run<C>(ax, a.pml_tab, la.pml_mem, a.pml_store, q, e, fo + (int64_t)q * stride, stride, y);
        const int cy = axis == 1 ? 0 : o, cz = axis == 1 ? o : 0;
        const bool srcs = a.src && segment_has_source(a, shot, axis, col, cy, cz, q, min(q + C, N));
        // receivers of this column among the rows this lane updates: trace sample n
        int64_t n = -1;
        if (rinfo.y > 0 && rinfo.w >= q && rinfo.z < q + C) {
            n = *a.d_step - 1;
            if (n >= a.trace_len) n = -1;
        }
        // waves with no source and no receiver among their rows (nearly all of them) take
        // the epilogue without the per-node source and receiver tests
        auto rows_out = [&](auto plain_c) {
            constexpr bool P = decltype(plain_c)::value;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int i = q + c;
                if (i < e) {
                    const int r = i * stride;
                    const float D = y[c];
                    float v;
                    if constexpr (kPre)
                        v = epilogue_pre<EPI>(la, fo + r, mo + r, shot, D, pre[c], col, axis == 1 ? i : cy,
                                              axis == 1 ? cz : i, P ? false : srcs);
                    else
                        v = epilogue<EPI>(la, fo + r, mo + r, shot, D, col, axis == 1 ? i : cy,
                                          axis == 1 ? cz : i, P ? false : srcs);
                    if (!P && n >= 0 && i >= rinfo.z && i <= rinfo.w) record_row(a, rinfo, i, v, n);
                }
            }
        };
        if (!__any(srcs || n >= 0)) rows_out(std::true_type{});
        else rows_out(std::false_type{});
        if (e == N && chunk == kc) {
            const int r = N * stride;
            float D = we;
            if (a.pml_mem && in_pml(ax, N)) D = pml_adjust(a.pml_tab, la.pml_mem, a.pml_store, N, fo + r, D);
            const float v = epilogue<EPI>(la, fo + r, mo + r, shot, D, col, axis == 1 ? N : cy,
                                          axis == 1 ? cz : N, srcs);
            if (rinfo.y > 0 && rinfo.w == N) {
                const int64_t nn = *a.d_step - 1;
                if (nn >= 0 && nn < a.trace_len) record_row(a, rinfo, N, v, nn);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint phase 2.  The patch-interior solve of T^T y = z leaves y undefined at the
// junction rows; the junction row of T^T gives it:  y_J = z_J - subT_J y_{J-1} -
// supT_J y_{J+1}  (neighbours are patch-interior rows).  Then (G^T y)_j = the stencil
// column j of G (junction rows of G are zero) plus the transposed PMBC rows.
// ---------------------------------------------------------------------------

// One thread per (line, junction).  Junction slot k sits at node (k+1)M (natural
// ends: slots 0..p-2) or min(kM, N) (junction ends: slots 0..p).
__global__ void __launch_bounds__(256) k_adj_junctions(LineArgs a, float *__restrict__ Y, int axis, int nj,
                                                       int64_t total)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const AxisDev &ax = a.ax;
    int slot, x, yy, z, shot;
    if (axis == 0) {
        slot = (int)(idx % nj);
        int64_t row = idx / nj;
        const int rps = a.nz * a.ny;
        shot = (int)(row / rps);
        const int r2 = (int)(row - (int64_t)shot * rps);
        z = r2 / a.ny;
        yy = r2 - z * a.ny;
        x = 0;
    } else {
        x = (int)(idx % a.nx);
        int64_t t = idx / a.nx;
        const int n_other = axis == 1 ? a.nz : a.ny;
        const int so = (int)(t % ((int64_t)a.S * n_other));
        slot = (int)(t / ((int64_t)a.S * n_other));
        shot = so / n_other;
        const int o = so - shot * n_other;
        if (axis == 1) { z = o; yy = 0; } else { yy = o; z = 0; }
    }
    const int J = ax.ends == 0 ? (slot + 1) * ax.M : min(slot * ax.M, ax.N);
    const int64_t stride = axis == 0 ? 1 : (axis == 1 ? a.pitch : a.plane);
    const int64_t midx0 = (int64_t)z * a.plane + (int64_t)yy * a.pitch + x;   // node 0 of the line
    const int64_t lb = (int64_t)shot * a.shot_stride + midx0;
    const float4 t = ax.luT[J];
    float v = a.in[lb + J * stride];
    if (a.in_coef) v *= a.in_coef[midx0 + J * stride];
    if (J > 0) v = fmaf(-t.w, Y[lb + (J - 1) * stride], v);
    if (J < ax.N) v = fmaf(-t.z, Y[lb + (J + 1) * stride], v);
    Y[lb + J * stride] = v;
}

// One thread per node; blocks tile the rows of x (the grid is rows x blocks per row,
// so the row decomposition is per block).  Along x the node index varies across the
// lanes; along y or z it is uniform per block (table reads are scalar).
template <int EPI>
__global__ void __launch_bounds__(256) k_adj_gather(LineArgs a, const float *__restrict__ Y, int axis, int bpr)
{
    const int row = blockIdx.x / bpr;                 // (shot, z, y) row of the padded layout
    const int x = (blockIdx.x - row * bpr) * blockDim.x + threadIdx.x;
    if (x >= a.nx) return;
    const AxisDev &ax = a.ax;
    const int rps = a.nz * a.ny;
    const int shot = row / rps;
    const int r2 = row - shot * rps;
    const int z = r2 / a.ny;
    const int yy = r2 - z * a.ny;
    const int64_t midx = (int64_t)z * a.plane + (int64_t)yy * a.pitch + x;
    const int64_t oidx = (int64_t)shot * a.shot_stride + midx;
    const int j = axis == 0 ? x : (axis == 1 ? yy : z);
    const int64_t stride = axis == 0 ? 1 : (axis == 1 ? a.pitch : a.plane);
    const float *__restrict__ yl = Y + (oidx - j * stride);   // node 0 of the line
    const float4 w = ax.adjw[j];
    float out = w.y * yl[j * stride];
    out = fmaf(w.x, yl[max(j - 1, 0) * stride], out);
    out = fmaf(w.z, yl[min(j + 1, ax.N) * stride], out);
    const int *gn = ax.g_node + (int64_t)j * ax.gmax;
    const float *gc = ax.g_c + (int64_t)j * ax.gmax;
    for (int t = 0; t < ax.gmax; ++t) {
        const int J = gn[t];
        if (J >= 0) out = fmaf(gc[t], yl[J * stride], out);
    }
    epilogue<EPI>(a, oidx, midx, shot, out, x, yy, z);
}

// Gather along y or z: a thread owns kGatherRows consecutive rows of one column; the
// rows of a block are the same for all its lanes (blockIdx.y), so the stencil and tap
// tables are read once per block, and each y row is loaded once per segment.
constexpr int kGatherRows = 8;

template <int EPI>
__global__ void __launch_bounds__(256) k_adj_gather_s(LineArgs a, const float *__restrict__ Y, int axis, int cols)
{
    const AxisDev &ax = a.ax;
    const int N = ax.N;
    const int r0 = blockIdx.y * kGatherRows;
    const int gc0 = blockIdx.x * 256 + threadIdx.x;   // (shot, column) with x fastest
    const int shot = gc0 / cols;
    const int c = gc0 - shot * cols;
    const int pitch = (int)a.pitch;
    const int x = c % pitch;
    if (shot >= a.S || x >= a.nx) return;
    // node 0 of the column: axis 2 -> (y, x) = c; axis 1 -> (z, x)
    const int zc = axis == 1 ? c / pitch : 0;
    const int yc = axis == 2 ? c / pitch : 0;
    const int64_t stride = axis == 1 ? a.pitch : a.plane;
    const int64_t m0 = (int64_t)zc * a.plane + (int64_t)yc * a.pitch + x;
    const int64_t o0 = (int64_t)shot * a.shot_stride + m0;
    const float *__restrict__ yl = Y + o0;
    float yv[kGatherRows + 2];
#pragma unroll
    for (int i = 0; i < kGatherRows + 2; ++i) yv[i] = yl[clampi(r0 - 1 + i, 0, N) * stride];
    Pre pre[kGatherRows];
#pragma unroll
    for (int i = 0; i < kGatherRows; ++i) {
        const int64_t off = (int64_t)min(r0 + i, N) * stride;
        pre[i] = pre_load<EPI>(a, o0 + off, m0 + off);
    }
#pragma unroll
    for (int i = 0; i < kGatherRows; ++i) {
        const int r = r0 + i;
        if (r > N) break;
        const float4 w = ax.adjw[r];
        float out = w.y * yv[i + 1];
        out = fmaf(w.x, yv[r > 0 ? i : i + 1], out);
        out = fmaf(w.z, yv[r < N ? i + 2 : i + 1], out);
        const int *gn = ax.g_node + (int64_t)r * ax.gmax;
        const float *gcf = ax.g_c + (int64_t)r * ax.gmax;
        for (int t = 0; t < ax.gmax; ++t) {
            const int J = gn[t];
            if (J >= 0) out = fmaf(gcf[t], yl[J * stride], out);
        }
        const int64_t off = (int64_t)r * stride;
        epilogue_pre<EPI>(a, o0 + off, m0 + off, shot, out, pre[i], x, axis == 1 ? r : yc, axis == 2 ? r : zc, false);
    }
}

// The three adjoint phases of an x pass in one block per line (p*G lanes): the
// patch-interior solve of T^T y = z, the junction rows of T^T, then G^T y, with y kept
// in LDS between them.  Same arithmetic, in the same order, as the solve / junction /
// gather kernels above.
// One adjoint pass along x of the line held by the workgroup (every thread calls it;
// barriers inside): the patch-interior solve of T^T y = z with z_i = val(i), y to the
// LDS line ys, the junction rows, then for every node i the value (G^T y)_i handed to
// emit(i, D, r), where r is the thread's read-ahead slot of node i (node i = thread +
// r * blockDim for r < C + 1, read ahead by issue() together with the plain-column
// bits pw), or -1.  Plain columns ({s3, 0, -s3}, no PMBC row) need no table; the
// others (rows near junctions and ends) come from the packed table, one entry per
// thread.  Same arithmetic, in the same order, as the solve / junction / gather kernels.
template <int C, typename Val, typename Val4, typename Issue, typename Emit>
__device__ __forceinline__ void adj_x_pass(const AxisDev &ax, int G, float *ys, const unsigned *pw, Val val, Val4 val4,
                                           Issue issue, Emit emit)
{
    const int N = ax.N, M = ax.M, p = ax.p;
    const int k = threadIdx.x & (G - 1);
    const int lraw = threadIdx.x / G;
    const bool uact = lraw < p;
    const int l = min(lraw, p - 1);
    const int s = l * M;
    const int e = min(s + M, N);
    const int kc = (e - 1 - s) / C;
    // junction rows owned here: row s (lane 0; not at a natural end), row N (closing
    // lane of the last patch, junction ends only)
    const bool js = uact && k == 0 && (ax.ends != 0 || s > 0);
    const bool jn = uact && ax.ends != 0 && e == N && k == kc;
    const int J = jn ? N : s;
    float zJ = 0.f;
    float w[C];
    float we = x_unit<C, SOLVE_T1>(ax, k, G, l, true, val, val4, [&]() { issue(); zJ = val(J); }, w);
    const int q = s + k * C;
    if (uact) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (q + c < e) ys[q + c] = w[c];
        if (e == N && k == kc) ys[N] = we;
    }
    __syncthreads();
    // junction rows: y_J = z_J - sub_J y_{J-1} - sup_J y_{J+1} (neighbours are interior rows)
    if (js || jn) {
        const float4 t = ax.luT[J];
        float v = zJ;
        if (J > 0) v = fmaf(-t.w, ys[J - 1], v);
        if (J < N) v = fmaf(-t.z, ys[J + 1], v);
        ys[J] = v;
    }
    if (js && jn) {   // a one-lane last patch holding both of its junction rows
        const float4 t = ax.luT[s];
        float v = val(s);
        if (s > 0) v = fmaf(-t.w, ys[s - 1], v);
        v = fmaf(-t.z, ys[s + 1], v);
        ys[s] = v;
    }
    __syncthreads();
    // the stencil part of column i of G^T; the special columns add their junction rows
    auto col = [&](int i, float4 aw) {
        float o = aw.y * ys[i];
        o = fmaf(aw.x, ys[max(i - 1, 0)], o);
        o = fmaf(aw.z, ys[min(i + 1, N)], o);
        return o;
    };
    const int nthr = blockDim.x;
#pragma unroll
    for (int r = 0; r < C + 1; ++r) {
        const int i = (int)threadIdx.x + r * nthr;
        if (i <= N && ((pw[r] >> (i & 31)) & 1u)) emit(i, col(i, ax.adjw_plain), r);
    }
    for (int i = (int)threadIdx.x + (C + 1) * nthr; i <= N; i += nthr)
        if ((ax.plain[i >> 5] >> (i & 31)) & 1u) emit(i, col(i, ax.adjw_plain), -1);
    for (int t = threadIdx.x; t < ax.nspec; t += nthr) {
        const SpecialCol sc = ax.spec[t];
        float o = col(sc.row, sc.aw);
        const int *gn = ax.g_node + (int64_t)sc.row * ax.gmax;
        const float *gc = ax.g_c + (int64_t)sc.row * ax.gmax;
        for (int q = 0; q < ax.gmax; ++q) {
            const int J = gn[q];
            if (J >= 0) o = fmaf(gc[q], ys[J], o);
        }
        emit(sc.row, o, -1);
    }
}

// The three adjoint phases of an x pass in one block per line (p*G lanes), y in LDS.
template <int C, int EPI>
__global__ void __launch_bounds__(512) k_adj_x(LineArgs a, int G)
{
    extern __shared__ float4 lds4[];
    float *ys = reinterpret_cast<float *>(lds4);
    const AxisDev &ax = a.ax;
    const int N = ax.N;
    const int line = blockIdx.x;
    const int lps = a.nz * a.ny;
    const int shot = line / lps;
    const int64_t base = (int64_t)line * a.pitch;
    const int64_t mbase = (int64_t)(line - shot * lps) * a.pitch;
    const float *__restrict__ in = a.in + base;
    const float *__restrict__ icf = a.in_coef ? a.in_coef + mbase : nullptr;
    constexpr int PF = C + 1;
    const int nthr = blockDim.x;
    Pre pre[PF];
    unsigned pw[PF];
    auto val = [&](int i) { return icf ? in[i] * icf[i] : in[i]; };
    auto val4 = [&](int i) {
        float4 v = ld4(in + i);
        if (icf) {
            const float4 c = ld4(icf + i);
            v = make_float4(v.x * c.x, v.y * c.y, v.z * c.z, v.w * c.w);
        }
        return v;
    };
    auto issue = [&]() {
#pragma unroll
        for (int r = 0; r < PF; ++r) {
            const int i = min((int)threadIdx.x + r * nthr, N);
            pre[r] = pre_load<EPI>(a, base + i, mbase + i);
            pw[r] = ax.plain[i >> 5];
        }
    };
    auto emit = [&](int i, float D, int r) {
        Pre pr;
        if (r >= 0) {
#pragma unroll
            for (int t = 0; t < PF; ++t)
                if (t == r) pr = pre[t];
        } else {
            pr = pre_load<EPI>(a, base + i, mbase + i);
        }
        epilogue_pre<EPI>(a, base + i, mbase + i, shot, D, pr, i, 0, 0, false);
    };
    adj_x_pass<C>(ax, G, ys, pw, val, val4, issue, emit);
}

// Two adjoint x passes of consecutive reverse steps in one block per line:
// out += alpha Dx^T(coef in) (the mu1 update from lambda), the updated line kept in
// LDS, then out2 += alpha2 Dx^T(coef2 out) (the next step's lambda update, which reads
// only the new mu1); out2 is the array `in`, whose values phase 1 has finished reading.
template <int C>
__global__ void __launch_bounds__(512) k_adj_xx(LineArgs a, const float *__restrict__ coef2, float *__restrict__ out2,
                                                float alpha2, int G)
{
    extern __shared__ float4 lds4[];
    const AxisDev &ax = a.ax;
    const int N = ax.N;
    const int nl4 = (N + 4) / 4;
    float *ys = reinterpret_cast<float *>(lds4);
    float4 *ms4 = lds4 + nl4;
    float *ms = reinterpret_cast<float *>(ms4);
    const int line = blockIdx.x;
    const int lps = a.nz * a.ny;
    const int shot = line / lps;
    const int64_t base = (int64_t)line * a.pitch;
    const int64_t mbase = (int64_t)(line - shot * lps) * a.pitch;
    const float *__restrict__ in = a.in + base;
    const float *__restrict__ icf = a.in_coef + mbase;
    const float *__restrict__ c2 = coef2 + mbase;
    float *__restrict__ o1 = a.out[0] + base;
    float *__restrict__ o2 = out2 + base;
    constexpr int PF = C + 1;
    const int nthr = blockDim.x;
    float p1[PF], p2[PF];   // out and out2 at the thread's first nodes, read ahead
    unsigned pw[PF];
    auto issue1 = [&]() {
#pragma unroll
        for (int r = 0; r < PF; ++r) {
            const int i = min((int)threadIdx.x + r * nthr, N);
            p1[r] = o1[i];
            p2[r] = o2[i];
            pw[r] = ax.plain[i >> 5];
        }
    };
    auto pick = [&](const float (&arr)[PF], int r) {
        float v = 0.f;
#pragma unroll
        for (int t = 0; t < PF; ++t)
            if (t == r) v = arr[t];
        return v;
    };
    // phase 1: out = out + alpha D^T(coef in), also into LDS
    adj_x_pass<C>(
        ax, G, ys, pw, [&](int i) { return in[i] * icf[i]; },
        [&](int i) {
            const float4 v = ld4(in + i), c = ld4(icf + i);
            return make_float4(v.x * c.x, v.y * c.y, v.z * c.z, v.w * c.w);
        },
        issue1,
        [&](int i, float D, int r) {
            const float v = fmaf(a.alpha * 1.f, D, r >= 0 ? pick(p1, r) : o1[i]);
            o1[i] = v;
            ms[i] = v;
        });
    __syncthreads();
    // phase 2: out2 = out2 + alpha2 D^T(coef2 out_new), out_new from LDS
    adj_x_pass<C>(
        ax, G, ys, pw, [&](int i) { return ms[i] * c2[i]; },
        [&](int i) {
            const float4 v = ms4[i >> 2], c = ld4(c2 + i);
            return make_float4(v.x * c.x, v.y * c.y, v.z * c.z, v.w * c.w);
        },
        [] {},
        [&](int i, float D, int r) { o2[i] = fmaf(alpha2 * 1.f, D, r >= 0 ? pick(p2, r) : o2[i]); });
}

// ---------------------------------------------------------------------------
// sources, receivers, bookkeeping
// ---------------------------------------------------------------------------
__global__ void k_inject(const SrcDev *__restrict__ src, float *const *fields, const float *__restrict__ b,
                         const float *__restrict__ wpool, const float *__restrict__ wavpool,
                         int64_t shot_stride, int64_t pitch, int64_t plane, const int64_t *d_step,
                         int time_offset, float scale, int want_force)
{
    const SrcDev sd = src[blockIdx.x];
    if (sd.force != want_force) return;
    const int64_t n = *d_step + time_offset;
    if (n < 0 || n >= sd.nt) return;
    const float amp = scale * wavpool[sd.wav_off + n];
    const int tot = sd.bx * sd.by * sd.bz;
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        const int ix = t % sd.bx, iy = (t / sd.bx) % sd.by, iz = t / (sd.bx * sd.by);
        const int64_t midx = (int64_t)(sd.z0 + iz) * plane + (int64_t)(sd.y0 + iy) * pitch + (sd.x0 + ix);
        float v = amp * wpool[sd.w_off + t];
        if (sd.force) v *= b[midx];
        for (int f = 0; f < sd.nfield; ++f) {
            float *F = fields[sd.field0 + f];
            F[(int64_t)sd.shot * shot_stride + midx] += v;
        }
    }
}

__global__ void k_record(const RecDev *__restrict__ rec, int nrec, const float *const *fields,
                         int64_t shot_stride, double *traces, const int64_t *d_step, int64_t trace_len,
                         float weight, int accumulate)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrec) return;
    const int64_t n = *d_step;
    if (n >= trace_len) return;
    const RecDev rd = rec[r];
    const double v = (double)weight * (double)fields[rd.comp][(int64_t)rd.shot * shot_stride + rd.node];
    double *t = traces + rd.trace_off + n;
    *t = accumulate ? *t + v : v;
}

__global__ void k_advance(int64_t *d_step) { *d_step += 1; }

__global__ void k_record2(const RecDev *__restrict__ rec0, int nrec0, float w0, int acc0,
                          const RecDev *__restrict__ rec1, int nrec1, float w1, int acc1,
                          const float *const *fields, int64_t shot_stride, double *traces,
                          const int64_t *d_step, int offset, int64_t trace_len)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    const RecDev *rec = rec0;
    float w = w0;
    int acc = acc0;
    if (r >= nrec0) {
        r -= nrec0;
        if (r >= nrec1) return;
        rec = rec1; w = w1; acc = acc1;
    }
    const int64_t n = *d_step + offset;
    if (n < 0 || n >= trace_len) return;
    const RecDev rd = rec[r];
    const double v = (double)w * (double)fields[rd.comp][(int64_t)rd.shot * shot_stride + rd.node];
    double *t = traces + rd.trace_off + n;
    *t = acc ? *t + v : v;
}

__global__ void k_set_step(int64_t *d_step, int64_t v) { *d_step = v; }

// Residual injection of the adjoint: each target node sums its receivers' samples in
// receiver order (FP64) and adds the sum once; targets are distinct, so no atomics.
__global__ void k_res_gather(const RecTarget *__restrict__ tg, int nt, const int64_t *__restrict__ toff,
                             float *const *fields, float *single, int64_t shot_stride,
                             const double *__restrict__ res, int64_t n, float w)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const RecTarget g = tg[t];
    double acc = 0.0;
    for (int k = g.first; k < g.first + g.count; ++k) acc += res[toff[k] + n];
    float *f = single ? single : fields[g.comp];
    const int64_t i = (int64_t)g.shot * shot_stride + g.node;
    f[i] += w * (float)acc;
}

__global__ void k_pad_copy(const float *__restrict__ src, float *__restrict__ dst, int nx, int ny, int nz,
                           int64_t pitch, int to_padded, int64_t total)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int x = (int)(idx % nx);
    const int64_t row = idx / nx;  // (batch, z, y) rows
    const int64_t p = row * pitch + x;
    if (to_padded) dst[p] = src[idx];
    else dst[idx] = src[p];
}

// Media times the time step, formed in double and rounded once:
// acoustic dt K, dt b; elastic dt lambda, dt mu, dt (lambda + 2 mu), dt b.
__global__ void k_media(const float *__restrict__ vp, const float *__restrict__ vs,
                        const float *__restrict__ rho, float *m0, float *m1, float *m2, float *m3,
                        int physics, int nx, int64_t pitch, int64_t total, double dt)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int x = (int)(idx % nx);
    const int64_t p = (idx / nx) * pitch + x;
    const double r = rho[idx], c = vp[idx];
    if (physics == 0) {
        m0[p] = (float)(dt * r * c * c);   // dt K
        m1[p] = (float)(dt / r);           // dt b
    } else {
        const double cs = vs[idx];
        const double mu = r * cs * cs, lam = r * c * c - 2.0 * mu;
        m0[p] = (float)(dt * lam);
        m1[p] = (float)(dt * mu);
        m2[p] = (float)(dt * (lam + 2.0 * mu));
        m3[p] = (float)(dt / r);
    }
}

__global__ void k_fill(float *p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_axpby(float *y, const float *x, float a, float b, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = fmaf(a, x[i], b * y[i]);
}

// g[node] += scale * sum_shots lam[shot][node] * div[shot][node], fixed shot order.
__global__ void k_grad_accum(double *g, const float *__restrict__ lam, const float *__restrict__ div,
                             float scale, int S, int64_t shot_stride, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int s = 0; s < S; ++s)
        acc += (double)lam[(int64_t)s * shot_stride + i] * (double)div[(int64_t)s * shot_stride + i];
    g[i] += (double)scale * acc;
}

__global__ void k_grad_unpad(const double *gp, double *g, int nx, int64_t pitch, const float *vp,
                             const float *rho, int param, int64_t total)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int x = (int)(idx % nx);
    const int64_t p = (idx / nx) * pitch + x;
    double v = gp[p];
    if (param == 1) v *= 2.0 * (double)rho[idx] * (double)vp[idx];   // dK/dc = 2 rho c
    g[idx] = v;
}

// Sets *flag to 1 if any of p[0..n) is a NaN or an infinity (exponent bits all set);
// grid-stride over 16-byte loads, one store per wave that saw one.
__device__ __forceinline__ bool nonfinite_bits(float v) { return (__float_as_uint(v) & 0x7f800000u) == 0x7f800000u; }

__global__ void __launch_bounds__(256) k_nonfinite(const float *__restrict__ p, int64_t n, int *flag)
{
    const int64_t n4 = n >> 2;
    const float4 *__restrict__ p4 = reinterpret_cast<const float4 *>(p);
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
        const float4 v = p4[i];
        bad = bad || nonfinite_bits(v.x) || nonfinite_bits(v.y) || nonfinite_bits(v.z) || nonfinite_bits(v.w);
    }
    if (blockIdx.x == 0 && (int64_t)threadIdx.x < (n & 3)) bad = bad || nonfinite_bits(p[n4 * 4 + threadIdx.x]);
    if (__any(bad) && (threadIdx.x & 63) == 0) *flag = 1;
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// nodes per lane of the x kernels: the caller's choice if it fits 64 lanes per patch,
// else the smallest that does (0 = none fits)
int x_chunk(const LineArgs &a)
{
    int cx = a.cx;
    if (cx != 4 && cx != 8 && cx != 16) cx = 4;
    while (cx < 16 && cx * 64 < a.ax.M) cx *= 2;
    return cx * 64 < a.ax.M ? 0 : cx;
}

template <int C, int SOLVE>
hipError_t dispatch_x(int epi, const LineArgs &a, hipStream_t st)
{
    const int M = a.ax.M;
    int G = 1;
    while (G * C < M) G <<= 1;
    if (G > 64) return hipErrorInvalidValue;
    const int64_t lines = (int64_t)a.S * a.nz * a.ny;
    const int64_t nunits = lines * a.ax.p;
    if (nunits >= (1ll << 31)) return hipErrorInvalidValue;
    const int threads = 256;
    // whole units of 16 lanes, four per wave on every line: the multi-line kernel, with
    // the caller's lines per wave, else (automatic) the most of 16, 8, 4, 2 that still
    // gives 8192 waves (32 per CU)
    const int bpl = a.ax.p / 4;
    if (a.xl != 1 && G == 16 && M == 16 * C && a.ax.N % M == 0 && a.ax.p % 4 == 0) {
        int xl = a.xl;
        if (xl == 0) {
            xl = 16;
            while (xl > 1 && (lines + xl - 1) / xl * bpl < 8192) xl >>= 1;
        }
        if (xl > 1) {
            const int64_t nwaves = (lines + xl - 1) / xl * bpl;
            if (nwaves >= (1ll << 31)) return hipErrorInvalidValue;
            const unsigned bl = nblk(nwaves, threads / 64);
            const int nw = (int)nwaves;
            switch (epi) {
            case EPI_STORE: hipLaunchKernelGGL((k_line_xl<C, SOLVE, EPI_STORE>), bl, threads, 0, st, a, xl, nw); break;
            case EPI_AXPY: hipLaunchKernelGGL((k_line_xl<C, SOLVE, EPI_AXPY>), bl, threads, 0, st, a, xl, nw); break;
            case EPI_AXPY_AUX:
                hipLaunchKernelGGL((k_line_xl<C, SOLVE, EPI_AXPY_AUX>), bl, threads, 0, st, a, xl, nw);
                break;
            case EPI_BASE: hipLaunchKernelGGL((k_line_xl<C, SOLVE, EPI_BASE>), bl, threads, 0, st, a, xl, nw); break;
            default: return hipErrorInvalidValue;
            }
            return hipGetLastError();
        }
    }
    const int64_t units_per_block = (threads / 64) * (64 / G);
    const unsigned blocks = nblk(nunits, (int)units_per_block);
    const int nu = (int)nunits;
    switch (epi) {
    case EPI_STORE: hipLaunchKernelGGL((k_line_x<C, SOLVE, EPI_STORE>), blocks, threads, 0, st, a, G, nu); break;
    case EPI_AXPY: hipLaunchKernelGGL((k_line_x<C, SOLVE, EPI_AXPY>), blocks, threads, 0, st, a, G, nu); break;
    case EPI_AXPY_AUX: hipLaunchKernelGGL((k_line_x<C, SOLVE, EPI_AXPY_AUX>), blocks, threads, 0, st, a, G, nu); break;
    case EPI_BASE: hipLaunchKernelGGL((k_line_x<C, SOLVE, EPI_BASE>), blocks, threads, 0, st, a, G, nu); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int C, int SOLVE>
hipError_t dispatch_s(int axis, int epi, const LineArgs &a, hipStream_t st)
{
    const int M = a.ax.M;
    const int nch = (M + C - 1) / C;
    const int n_other = axis == 1 ? a.nz : a.ny;
    const int64_t F = (int64_t)a.S * n_other * a.pitch;
    // columns per wave: the caller's choice, else the widest that still gives
    // >= 2048 workgroups (or 16)
    int CW = a.cw;
    if (CW != 8 && CW != 16 && CW != 32 && CW != 64) {
        CW = 64;
        while (CW > 16 && ((F + CW - 1) / CW) * a.ax.p < 2048) CW >>= 1;
    }
    const int sub = 64 / CW;
    const int W = (nch + sub - 1) / sub;
    if (W > kMaxWaves) return hipErrorInvalidValue;
    const int gx = (int)((F + CW - 1) / CW);
    const int gxp = (gx + 7) / 8 * 8;
    dim3 grid((unsigned)gxp, a.ax.p, 1);
    const int threads = 64 * W;
    const size_t shm = (6 * (size_t)threads + 64) * sizeof(float);
    {
        if (CW == 64) {
            switch (epi) {
            case EPI_STORE: hipLaunchKernelGGL((k_line_s<C, SOLVE, EPI_STORE, true>), grid, threads, shm, st, a, axis, CW, gx); break;
            case EPI_AXPY: hipLaunchKernelGGL((k_line_s<C, SOLVE, EPI_AXPY, true>), grid, threads, shm, st, a, axis, CW, gx); break;
            case EPI_AXPY_AUX: hipLaunchKernelGGL((k_line_s<C, SOLVE, EPI_AXPY_AUX, true>), grid, threads, shm, st, a, axis, CW, gx); break;
            case EPI_BASE: hipLaunchKernelGGL((k_line_s<C, SOLVE, EPI_BASE, true>), grid, threads, shm, st, a, axis, CW, gx); break;
            case EPI_NORMAL3:
                if constexpr (SOLVE != SOLVE_D1) return hipErrorInvalidValue;
                else hipLaunchKernelGGL((k_line_s<C, SOLVE, EPI_NORMAL3, true>), grid, threads, shm, st, a, axis, CW, gx);
                break;
            default: return hipErrorInvalidValue;
            }
            return hipGetLastError();
        }
    }
    switch (epi) {
    case EPI_STORE: hipLaunchKernelGGL((k_line_s<C, SOLVE, EPI_STORE, false>), grid, threads, shm, st, a, axis, CW, gx); break;
    case EPI_AXPY: hipLaunchKernelGGL((k_line_s<C, SOLVE, EPI_AXPY, false>), grid, threads, shm, st, a, axis, CW, gx); break;
    case EPI_AXPY_AUX: hipLaunchKernelGGL((k_line_s<C, SOLVE, EPI_AXPY_AUX, false>), grid, threads, shm, st, a, axis, CW, gx); break;
    case EPI_BASE: hipLaunchKernelGGL((k_line_s<C, SOLVE, EPI_BASE, false>), grid, threads, shm, st, a, axis, CW, gx); break;
    case EPI_NORMAL3:
        if constexpr (SOLVE != SOLVE_D1) return hipErrorInvalidValue;
        else hipLaunchKernelGGL((k_line_s<C, SOLVE, EPI_NORMAL3, false>), grid, threads, shm, st, a, axis, CW, gx);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int SOLVE>
hipError_t dispatch_solve(int axis, int epi, const LineArgs &a, hipStream_t st)
{
    const int M = a.ax.M;
    if (axis == 0) {
        const int cx = x_chunk(a);
        if (!cx) return hipErrorInvalidValue;
        if (cx == 4) return dispatch_x<4, SOLVE>(epi, a, st);
        if (cx == 8) return dispatch_x<8, SOLVE>(epi, a, st);
        return dispatch_x<16, SOLVE>(epi, a, st);
    }
    // nodes per lane along y / z: the caller's choice if the patch fits the block
    const int cs = a.cs;
    if (cs == 8 && (M + 7) / 8 <= kMaxWaves * (64 / (a.cw ? a.cw : 64)))
        return dispatch_s<8, SOLVE>(axis, epi, a, st);
    if (M <= 16 * kMaxWaves) return dispatch_s<16, SOLVE>(axis, epi, a, st);
    if (M <= 64 * kMaxWaves) return dispatch_s<64, SOLVE>(axis, epi, a, st);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_line(int axis, int solve, int epi, const LineArgs &a, hipStream_t st)
{
    switch (solve) {
    case SOLVE_D1: return dispatch_solve<SOLVE_D1>(axis, epi, a, st);
    case SOLVE_D2: return dispatch_solve<SOLVE_D2>(axis, epi, a, st);
    case SOLVE_T1: return dispatch_solve<SOLVE_T1>(axis, epi, a, st);
    default: return hipErrorInvalidValue;
    }
}

int line_xx_threads(const LineArgs &a)
{
    const int cx = x_chunk(a);
    if (!cx) return 0;
    int G = 1;
    while (G * cx < a.ax.M) G <<= 1;
    const int threads = (a.ax.p * G + 63) / 64 * 64;
    const size_t shm = (size_t)(a.ax.N + 4) / 4 * 16;
    if (threads > 512 || shm > 65536) return 0;
    return threads;
}

hipError_t launch_line_xx(const LineArgs &a, float *Tout, float *pml_mem_t, hipStream_t st)
{
    const int threads = line_xx_threads(a);
    if (!threads) return hipErrorInvalidValue;
    const int cx = x_chunk(a);
    int G = 1;
    while (G * cx < a.ax.M) G <<= 1;
    const size_t shm = (size_t)(a.ax.N + 4) / 4 * 16;
    const int64_t lines = (int64_t)a.S * a.nz * a.ny;
    if (lines >= (1ll << 31)) return hipErrorInvalidValue;
    switch (cx) {
    case 4: hipLaunchKernelGGL(k_line_xx<4>, (unsigned)lines, threads, shm, st, a, Tout, pml_mem_t, G); break;
    case 8: hipLaunchKernelGGL(k_line_xx<8>, (unsigned)lines, threads, shm, st, a, Tout, pml_mem_t, G); break;
    default: hipLaunchKernelGGL(k_line_xx<16>, (unsigned)lines, threads, shm, st, a, Tout, pml_mem_t, G); break;
    }
    return hipGetLastError();
}

hipError_t launch_adj_x(int epi, const LineArgs &a, hipStream_t st)
{
    const int threads = line_xx_threads(a);
    if (!threads || (epi != EPI_STORE && epi != EPI_AXPY)) return hipErrorNotSupported;
    const int cx = x_chunk(a);
    int G = 1;
    while (G * cx < a.ax.M) G <<= 1;
    const size_t shm = (size_t)(a.ax.N + 4) / 4 * 16;
    const int64_t lines = (int64_t)a.S * a.nz * a.ny;
    if (lines >= (1ll << 31)) return hipErrorInvalidValue;
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, (unsigned)lines, threads, shm, st, a, G); };
    const bool store = epi == EPI_STORE;
    switch (cx) {
    case 4: store ? go(k_adj_x<4, EPI_STORE>) : go(k_adj_x<4, EPI_AXPY>); break;
    case 8: store ? go(k_adj_x<8, EPI_STORE>) : go(k_adj_x<8, EPI_AXPY>); break;
    default: store ? go(k_adj_x<16, EPI_STORE>) : go(k_adj_x<16, EPI_AXPY>); break;
    }
    return hipGetLastError();
}

hipError_t launch_adj_xx(const LineArgs &a, const float *coef2, float *out2, float alpha2, hipStream_t st)
{
    const int threads = line_xx_threads(a);
    if (!threads || !a.in_coef || !coef2) return hipErrorNotSupported;
    const int cx = x_chunk(a);
    int G = 1;
    while (G * cx < a.ax.M) G <<= 1;
    const size_t shm = 2 * ((size_t)(a.ax.N + 4) / 4 * 16);
    const int64_t lines = (int64_t)a.S * a.nz * a.ny;
    if (lines >= (1ll << 31)) return hipErrorInvalidValue;
    switch (cx) {
    case 4: hipLaunchKernelGGL(k_adj_xx<4>, (unsigned)lines, threads, shm, st, a, coef2, out2, alpha2, G); break;
    case 8: hipLaunchKernelGGL(k_adj_xx<8>, (unsigned)lines, threads, shm, st, a, coef2, out2, alpha2, G); break;
    default: hipLaunchKernelGGL(k_adj_xx<16>, (unsigned)lines, threads, shm, st, a, coef2, out2, alpha2, G); break;
    }
    return hipGetLastError();
}

hipError_t launch_adj_junctions(int axis, const LineArgs &a, float *Y, hipStream_t st)
{
    const int nj = a.ax.ends == 0 ? a.ax.p - 1 : a.ax.p + 1;
    if (nj <= 0) return hipSuccess;
    const int64_t lines = axis == 0 ? (int64_t)a.S * a.nz * a.ny
                                    : (int64_t)a.S * (axis == 1 ? a.nz : a.ny) * a.nx;
    const int64_t total = lines * nj;
    hipLaunchKernelGGL(k_adj_junctions, nblk(total, 256), 256, 0, st, a, Y, axis, nj, total);
    return hipGetLastError();
}

hipError_t launch_adj_gather(int axis, int epi, const LineArgs &a, const float *Y, hipStream_t st)
{
    if (axis != 0) {
        const int cols = (int)(axis == 1 ? a.nz * a.pitch : a.ny * a.pitch);
        const int64_t tot = (int64_t)a.S * cols;
        if (tot >= (1ll << 31) || a.shot_stride * a.S >= (1ll << 40)) return hipErrorInvalidValue;
        const dim3 grid((unsigned)((tot + 255) / 256), (unsigned)((a.ax.N + kGatherRows) / kGatherRows));
        switch (epi) {
        case EPI_STORE: hipLaunchKernelGGL(k_adj_gather_s<EPI_STORE>, grid, 256, 0, st, a, Y, axis, cols); break;
        case EPI_AXPY: hipLaunchKernelGGL(k_adj_gather_s<EPI_AXPY>, grid, 256, 0, st, a, Y, axis, cols); break;
        case EPI_AXPY_AUX: hipLaunchKernelGGL(k_adj_gather_s<EPI_AXPY_AUX>, grid, 256, 0, st, a, Y, axis, cols); break;
        case EPI_BASE: hipLaunchKernelGGL(k_adj_gather_s<EPI_BASE>, grid, 256, 0, st, a, Y, axis, cols); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const int bpr = (a.nx + 255) / 256;
    const int64_t rows = (int64_t)a.S * a.nz * a.ny;
    if (rows * bpr >= (1ll << 31) || a.shot_stride * a.S >= (1ll << 40)) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)(rows * bpr);
    switch (epi) {
    case EPI_STORE: hipLaunchKernelGGL(k_adj_gather<EPI_STORE>, blocks, 256, 0, st, a, Y, axis, bpr); break;
    case EPI_AXPY: hipLaunchKernelGGL(k_adj_gather<EPI_AXPY>, blocks, 256, 0, st, a, Y, axis, bpr); break;
    case EPI_AXPY_AUX: hipLaunchKernelGGL(k_adj_gather<EPI_AXPY_AUX>, blocks, 256, 0, st, a, Y, axis, bpr); break;
    case EPI_BASE: hipLaunchKernelGGL(k_adj_gather<EPI_BASE>, blocks, 256, 0, st, a, Y, axis, bpr); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_inject(const SrcDev *src, int nsrc, float *const *fields, const float *b,
                         const float *wpool, const float *wavpool, int64_t shot_stride, int64_t pitch,
                         int64_t plane, const int64_t *d_step, int time_offset, float scale,
                         int want_force, hipStream_t st)
{
    if (nsrc <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_inject, nsrc, 256, 0, st, src, fields, b, wpool, wavpool, shot_stride, pitch,
                       plane, d_step, time_offset, scale, want_force);
    return hipGetLastError();
}

hipError_t launch_record(const RecDev *rec, int nrec, const float *const *fields, int64_t shot_stride,
                         double *traces, const int64_t *d_step, int64_t trace_len, float weight,
                         int accumulate, hipStream_t st)
{
    if (nrec <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_record, nblk(nrec, 256), 256, 0, st, rec, nrec, fields, shot_stride, traces,
                       d_step, trace_len, weight, accumulate);
    return hipGetLastError();
}

hipError_t launch_res_gather(const RecTarget *tg, int nt, const int64_t *toff, float *const *fields, float *single,
                             int64_t shot_stride, const double *res, int64_t n, float w, hipStream_t st)
{
    if (nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_res_gather, nblk(nt, 256), 256, 0, st, tg, nt, toff, fields, single, shot_stride, res, n, w);
    return hipGetLastError();
}

hipError_t launch_set_step(int64_t *d_step, int64_t v, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_step, 1, 1, 0, st, d_step, v);
    return hipGetLastError();
}

hipError_t launch_record2(const RecDev *rec0, int nrec0, float w0, int acc0, const RecDev *rec1, int nrec1,
                          float w1, int acc1, const float *const *fields, int64_t shot_stride,
                          double *traces, const int64_t *d_step, int offset, int64_t trace_len,
                          hipStream_t st)
{
    const int tot = nrec0 + nrec1;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_record2, nblk(tot, 256), 256, 0, st, rec0, nrec0, w0, acc0, rec1, nrec1, w1, acc1,
                       fields, shot_stride, traces, d_step, offset, trace_len);
    return hipGetLastError();
}

hipError_t launch_advance(int64_t *d_step, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance, 1, 1, 0, st, d_step);
    return hipGetLastError();
}

hipError_t launch_pad_copy(const float *src, float *dst, int nx, int rows, int64_t pitch, int to_padded,
                           hipStream_t st)
{
    const int64_t total = (int64_t)rows * nx;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pad_copy, nblk(total, 256), 256, 0, st, src, dst, nx, 0, 0, pitch, to_padded,
                       total);
    return hipGetLastError();
}

hipError_t launch_media(const float *vp, const float *vs, const float *rho, float *const *media,
                        int physics, int nx, int rows, int64_t pitch, double dt, hipStream_t st)
{
    const int64_t total = (int64_t)rows * nx;
    hipLaunchKernelGGL(k_media, nblk(total, 256), 256, 0, st, vp, vs, rho, media[0], media[1],
                       physics ? media[2] : nullptr, physics ? media[3] : nullptr, physics, nx, pitch,
                       total, dt);
    return hipGetLastError();
}

hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, nblk(n, 256), 256, 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_axpby(float *y, const float *x, float a, float b, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpby, nblk(n, 256), 256, 0, st, y, x, a, b, n);
    return hipGetLastError();
}

hipError_t launch_grad_accum(double *g, const float *lam, const float *div, float scale, int S,
                             int64_t shot_stride, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_grad_accum, nblk(n, 256), 256, 0, st, g, lam, div, scale, S, shot_stride, n);
    return hipGetLastError();
}

hipError_t launch_grad_unpad(const double *gp, double *g, int nx, int rows, int64_t pitch, const float *vp,
                             const float *rho, int param, hipStream_t st)
{
    const int64_t total = (int64_t)rows * nx;
    hipLaunchKernelGGL(k_grad_unpad, nblk(total, 256), 256, 0, st, gp, g, nx, pitch, vp, rho, param, total);
    return hipGetLastError();
}

hipError_t launch_nonfinite(const float *p, int64_t n, int *flag, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (((uintptr_t)p & 15) != 0) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)std::min<int64_t>(std::max<int64_t>(1, nblk(n / 4, 256)), 4096);
    hipLaunchKernelGGL(k_nonfinite, blocks, 256, 0, st, p, n, flag);
    return hipGetLastError();
}

}  // namespace loss
