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

#include "loss_internal.h"

namespace loss {

namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Node of tap t of the PMBC row of junction J (eq. PMBC: taps J-halo .. J+halo),
// wrapped on a periodic axis; taps outside a non-periodic line carry a zero
// coefficient, so the clamped node stands in for them.
__device__ __forceinline__ int tap_node(const AxisDev &ax, int J, int t)
{
    int k = J - ax.halo + t;
    if (ax.periodic) k = k < 0 ? k + ax.N : (k >= ax.N ? k - ax.N : k);
    else k = clampi(k, 0, ax.N);
    return k;
}

// PMBC slots of the junction rows s and e of patch l (-1 at a natural end): the
// slots number the junction rows in node order.
__device__ __forceinline__ int slot_first(const AxisDev &ax, int l) { return ax.ends == 0 ? l - 1 : l; }
__device__ __forceinline__ int slot_last(const AxisDev &ax, int l, int e)
{
    return e == ax.N ? (ax.ends == 0 ? -1 : ax.p) : (ax.ends == 0 ? l : l + 1);
}

// value of the input at element `idx` (media element `midx`), times the optional factor
__device__ __forceinline__ float load_in(const LineArgs &a, int64_t idx, int64_t midx)
{
    const float v = a.in[idx];
    return a.in_coef ? v * a.in_coef[midx] : v;
}

// Source terms for output j at node (x, y, z) of `shot` (sources sorted by shot).
__device__ __forceinline__ float source_terms(const LineArgs &a, int j, int shot, int x, int y, int z,
                                              int64_t midx)
{
    const int fid = a.out_field[j];
    float add = 0.f;
    const int k1 = a.src_begin[shot + 1];
    for (int k = a.src_begin[shot]; k < k1; ++k) {
        const SrcDev &sd = a.src[k];
        if (fid < sd.field0 || fid >= sd.field0 + sd.nfield) continue;
        const unsigned ix = (unsigned)(x - sd.x0), iy = (unsigned)(y - sd.y0), iz = (unsigned)(z - sd.z0);
        if (ix >= (unsigned)sd.bx || iy >= (unsigned)sd.by || iz >= (unsigned)sd.bz) continue;
        const int64_t n = *a.d_step + a.src_time_offset;
        if (n < 0 || n >= sd.nt) continue;
        float v = a.src_scale * a.wavpool[sd.wav_off + n] *
                  a.wpool[sd.w_off + ((int64_t)iz * sd.by + iy) * sd.bx + ix];
        if (sd.force) v *= a.bcoef[midx];
        add += v;
    }
    return add;
}

// Does the segment [lo, hi] along `axis` through (x, y, z) of `shot` meet a source box?
__device__ __forceinline__ bool segment_has_source(const LineArgs &a, int shot, int axis, int x, int y, int z,
                                                int lo, int hi)
{
    const int k1 = a.src_begin[shot + 1];
    for (int k = a.src_begin[shot]; k < k1; ++k) {
        const SrcDev &sd = a.src[k];
        const int c0[3] = {sd.x0, sd.y0, sd.z0}, nb[3] = {sd.bx, sd.by, sd.bz}, p[3] = {x, y, z};
        bool hit = true;
        for (int d = 0; d < 3; ++d) {
            if (d == axis) hit = hit && hi >= c0[d] && lo < c0[d] + nb[d];
            else hit = hit && p[d] >= c0[d] && p[d] < c0[d] + nb[d];
        }
        if (hit) return true;
    }
    return false;
}

// Epilogue of one node; returns the value written to out[0].
template <int EPI>
__device__ __forceinline__ float epilogue(const LineArgs &a, int64_t oidx, int64_t midx, int shot, float D,
                                          int x, int y, int z, bool srcs = true)
{
    if constexpr (EPI == EPI_STORE) {
        a.out[0][oidx] = D;
        return D;
    } else if constexpr (EPI == EPI_AXPY) {
        float v0 = 0.f;
        for (int j = 0; j < a.nout; ++j) {
            const float c = a.coef[j] ? a.coef[j][midx] : 1.f;
            float v = fmaf(a.alpha * c, D, a.out[j][oidx]);
            if (srcs && a.src) v += source_terms(a, j, shot, x, y, z, midx);
            a.out[j][oidx] = v;
            if (j == 0) v0 = v;
        }
        return v0;
    } else if constexpr (EPI == EPI_AXPY_AUX) {
        const float dv = D + a.aux[oidx];
        const float c = a.coef[0] ? a.coef[0][midx] : 1.f;
        float v = fmaf(a.alpha * c, dv, a.out[0][oidx]);
        if (srcs && a.src) v += source_terms(a, 0, shot, x, y, z, midx);
        a.out[0][oidx] = v;
        if (a.div) a.div[(int64_t)shot * a.div_shot_stride + midx] = dv;
        return v;
    } else if constexpr (EPI == EPI_NORMAL3) {
        const float t[3] = {a.aux[oidx], a.aux2[oidx], D};
        const float l2m = a.coef[0][midx], lam = a.coef[1][midx];
        float v0 = 0.f;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float other = j == 0 ? t[1] + t[2] : (j == 1 ? t[0] + t[2] : t[0] + t[1]);
            float v = fmaf(a.alpha, fmaf(l2m, t[j], lam * other), a.out[j][oidx]);
            if (srcs && a.src) v += source_terms(a, j, shot, x, y, z, midx);
            a.out[j][oidx] = v;
            if (j == 0) v0 = v;
        }
        return v0;
    } else {  // EPI_BASE
        const float c = a.coef[0] ? a.coef[0][midx] : 1.f;
        const float v = fmaf(a.alpha * c, D, a.aux[oidx]);
        a.out[0][oidx] = v;
        return v;
    }
}

// Epilogue operands of one node read ahead of the solve: out0, coef0, aux.
struct Pre {
    float o, c, x;
};

template <int EPI>
__device__ __forceinline__ Pre pre_load(const LineArgs &a, int64_t oidx, int64_t midx)
{
    Pre r{0.f, 1.f, 0.f};
    if constexpr (EPI == EPI_AXPY || EPI == EPI_AXPY_AUX) r.o = a.out[0][oidx];
    if constexpr (EPI != EPI_STORE) r.c = a.coef[0] ? a.coef[0][midx] : 1.f;
    if constexpr (EPI == EPI_AXPY_AUX || EPI == EPI_BASE) r.x = a.aux[oidx];
    return r;
}

// Epilogue with out0 / coef0 / aux taken from `pr` (outputs j >= 1 are read here);
// returns the value written to out[0].
template <int EPI>
__device__ __forceinline__ float epilogue_pre(const LineArgs &a, int64_t oidx, int64_t midx, int shot, float D,
                                              const Pre &pr, int x, int y, int z, bool srcs)
{
    if (srcs) return epilogue<EPI>(a, oidx, midx, shot, D, x, y, z);
    float v = D;
    if constexpr (EPI == EPI_AXPY) {
        v = fmaf(a.alpha * pr.c, D, pr.o);
        for (int j = 1; j < a.nout; ++j) {
            const float c = a.coef[j] ? a.coef[j][midx] : 1.f;
            a.out[j][oidx] = fmaf(a.alpha * c, D, a.out[j][oidx]);
        }
    } else if constexpr (EPI == EPI_AXPY_AUX) {
        const float dv = D + pr.x;
        v = fmaf(a.alpha * pr.c, dv, pr.o);
        if (a.div) a.div[(int64_t)shot * a.div_shot_stride + midx] = dv;
    } else if constexpr (EPI == EPI_BASE) {
        v = fmaf(a.alpha * pr.c, D, pr.x);
    }
    a.out[0][oidx] = v;
    return v;
}

// Trace samples of the receivers at row `r` of a strided column ({first, count} in ri).
__device__ __forceinline__ void record_row(const LineArgs &a, const int4 &ri, int r, float v, int64_t n)
{
    for (int k = ri.x; k < ri.x + ri.y; ++k)
        if (a.rrow[k] == r) a.traces[a.rtoff[k] + n] = (double)v;
}

__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ void st4(float *p, float4 v) { *reinterpret_cast<float4 *>(p) = v; }

// Epilogue operands of four consecutive x nodes (16-byte aligned).
struct Pre4 {
    float4 o, c, x;
};

template <int EPI>
__device__ __forceinline__ Pre4 pre_load4(const LineArgs &a, int64_t oidx, int64_t midx)
{
    const float4 one = make_float4(1.f, 1.f, 1.f, 1.f), zero = make_float4(0.f, 0.f, 0.f, 0.f);
    Pre4 r{zero, one, zero};
    if constexpr (EPI == EPI_AXPY || EPI == EPI_AXPY_AUX) r.o = ld4(a.out[0] + oidx);
    if constexpr (EPI != EPI_STORE) r.c = a.coef[0] ? ld4(a.coef[0] + midx) : one;
    if constexpr (EPI == EPI_AXPY_AUX || EPI == EPI_BASE) r.x = ld4(a.aux + oidx);
    return r;
}

__device__ __forceinline__ float4 fma4(float a, float4 c, float4 d, float4 o)
{
    return make_float4(fmaf(a * c.x, d.x, o.x), fmaf(a * c.y, d.y, o.y), fmaf(a * c.z, d.z, o.z),
                       fmaf(a * c.w, d.w, o.w));
}

// Epilogue of four consecutive x nodes (16-byte aligned, all inside the unit).
template <int EPI>
__device__ __forceinline__ void epilogue4(const LineArgs &a, int64_t oidx, int64_t midx, int shot, float4 D,
                                          const Pre4 &pr, int x, int y, int z, bool srcs)
{
    if (srcs) {
        epilogue<EPI>(a, oidx, midx, shot, D.x, x, y, z);
        epilogue<EPI>(a, oidx + 1, midx + 1, shot, D.y, x + 1, y, z);
        epilogue<EPI>(a, oidx + 2, midx + 2, shot, D.z, x + 2, y, z);
        epilogue<EPI>(a, oidx + 3, midx + 3, shot, D.w, x + 3, y, z);
        return;
    }
    if constexpr (EPI == EPI_STORE) {
        st4(a.out[0] + oidx, D);
    } else if constexpr (EPI == EPI_AXPY) {
        st4(a.out[0] + oidx, fma4(a.alpha, pr.c, D, pr.o));
        const float4 one = make_float4(1.f, 1.f, 1.f, 1.f);
        for (int j = 1; j < a.nout; ++j) {
            const float4 c = a.coef[j] ? ld4(a.coef[j] + midx) : one;
            st4(a.out[j] + oidx, fma4(a.alpha, c, D, ld4(a.out[j] + oidx)));
        }
    } else if constexpr (EPI == EPI_AXPY_AUX) {
        const float4 dv = make_float4(D.x + pr.x.x, D.y + pr.x.y, D.z + pr.x.z, D.w + pr.x.w);
        st4(a.out[0] + oidx, fma4(a.alpha, pr.c, dv, pr.o));
        if (a.div) st4(a.div + (int64_t)shot * a.div_shot_stride + midx, dv);
    } else {
        st4(a.out[0] + oidx, fma4(a.alpha, pr.c, D, pr.x));
    }
}

// Factors of the special rows of a patch, read once per unit.
struct EndRows {
    float4 lus, rcs, lu2s;     // row s: LU of T, stencil of G, LU of the moment system
    float4 lue, rce, luTe;     // row e: LU of T, stencil of G, LU of T^T
    float2 lu2e;               // row e as the closing row of the moment system
};

template <int SOLVE>
__device__ __forceinline__ EndRows end_rows(const AxisDev &ax, int s, int e)
{
    EndRows r;
    if constexpr (SOLVE != SOLVE_T1) {
        r.lus = ax.lu[s];
        r.lue = ax.lu[e];
    }
    if constexpr (SOLVE == SOLVE_D1) {
        r.rcs = ax.rc[s];
        r.rce = ax.rc[e];
    }
    if constexpr (SOLVE == SOLVE_D2) {
        r.lu2s = ax.lu2[s];
        r.lu2e = ax.lu2c[e];
    }
    if constexpr (SOLVE == SOLVE_T1) r.luTe = ax.luT[e];
    return r;
}

// Row s as the first row of the forward elimination, y_s = r - fm * carry, where the
// carry into the patch is the junction slope phi_s (zero at a natural end):
//   D1 junction: w_s = phi_s                            -> r = 0, fm = -1;
//   D2 junction: Hermite moment row, rhs (6/h)((u_{s+1}-u_s)/h - phi_s)
//                                                       -> r = 6(u_{s+1}-u_s)/h^2, fm = 6/h;
//   natural end: the end row of the system, independent of the carry (fm = 0).
template <int SOLVE>
__device__ __forceinline__ float first_row(const AxisDev &ax, const EndRows &er, float u0, float up, float &fm,
                                           float &fi, float &fs)
{
    const bool junc = er.lus.w == (float)ROW_JUNCTION;
    if constexpr (SOLVE == SOLVE_D1) {
        fi = er.lus.y;
        fs = er.lus.z;
        fm = junc ? -1.f : er.lus.x;
        return junc ? 0.f : fmaf(er.rcs.y, u0, er.rcs.z * up);
    } else {
        const float ih = 1.f / ax.h;
        fi = er.lu2s.y;
        fs = er.lu2s.z;
        fm = junc ? 6.f * ih : er.lu2s.x;
        return junc ? 6.f * ih * ih * (up - u0) : 0.f;
    }
}

// Closing row e of a unit: given the eliminated value at e-1, the solution at e.
template <int SOLVE>
__device__ __forceinline__ float last_row(const AxisDev &ax, const EndRows &er, float ylast, float ulast,
                                          float ue, float phe)
{
    if constexpr (SOLVE == SOLVE_D1) {
        const float r = (er.lue.w == (float)ROW_JUNCTION) ? phe : fmaf(er.rce.x, ulast, er.rce.y * ue);
        return (r - er.lue.x * ylast) * er.lue.y;
    } else if constexpr (SOLVE == SOLVE_T1) {
        return (ue - er.luTe.x * ylast) * er.luTe.y;
    } else {
        float r = 0.f;
        if (er.lue.w != (float)ROW_NATURAL_R) {
            const float ih = 1.f / ax.h;
            r = 6.f * ih * fmaf(-(ue - ulast), ih, phe);
        }
        return (r - er.lu2e.x * ylast) * er.lu2e.y;
    }
}

// Factors {m, 1/d, sup} of rows q..q+C-1 (rows past N read the tables' identity padding).
template <int C, int SOLVE>
__device__ __forceinline__ void row_factors(const AxisDev &ax, int q, float (&fm)[C], float (&fi)[C],
                                            float (&fs)[C])
{
    const int qt = min(q, ax.N);
    if constexpr (SOLVE == SOLVE_T1) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float4 f = ax.luT[qt + c];
            fm[c] = f.x; fi[c] = f.y; fs[c] = f.z;
        }
    } else {
        const float2 *tab = (SOLVE == SOLVE_D1) ? ax.lum : ax.lum2;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float2 f = tab[qt + c];
            fm[c] = f.x; fi[c] = f.y; fs[c] = 1.f;   // sup = 1 on patch-interior rows
        }
    }
}

// Hides a value from common-subexpression elimination, so that an expression of it
// is recomputed instead of being kept in a register (emits no instruction).
__device__ __forceinline__ float opaque(float v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// Right-hand side of a patch-interior row from the node values u_{i-1}, u_i, u_{i+1}.
template <int SOLVE>
__device__ __forceinline__ float interior_rhs(const AxisDev &ax, float um, float u0, float up)
{
    if constexpr (SOLVE == SOLVE_D1) return ax.s3 * (up - um);
    else if constexpr (SOLVE == SOLVE_T1) return u0;
    else {
        const float ih = 1.f / ax.h;
        return 6.f * ih * ih * (um - 2.f * u0 + up);
    }
}

// Absorbing layer (ADE-PML, Sec. 3.3, exponential splitting).  With the derivative D
// of this pass frozen over tau, the memory variable psi of node j evolves exactly as
//   psi(tau) = e^{-x} psi0 - (d/k^2) tau phi1(x) D          (x = beta tau)
// and the field moves by -tau * coef * (D/k + phi1(x) psi0 - (d/k^2) tau phi2(x) D),
// phi1(x) = (1 - e^{-x})/x, phi2(x) = (x - 1 + e^{-x})/x^2.  Every factor depends only on
// the node and the pass's time span, so the host tabulates them (FP64, per step
// fraction); a node costs two loads and four FMAs.  The pass uses the effective
// derivative in place of D, so the epilogue keeps its plain form; psi(tau) is stored if
// asked.
__device__ __forceinline__ bool in_pml(const AxisDev &ax, int j)
{
    return j < ax.pml_w || j > ax.N - ax.pml_w;
}

// the sub-flow of one node from its table entry t = {e^{-x}, phi1, (d/k^2) tau phi1,
// 1/k - (d/k^2) tau phi2} and memory value psi0; psi(tau) into *psi1, the effective
// derivative returned
__device__ __forceinline__ float pml_flow(float4 t, float D, float psi0, float *psi1)
{
    *psi1 = fmaf(t.x, psi0, -t.z * D);
    return fmaf(t.w, D, t.y * psi0);
}

__device__ __forceinline__ float pml_adjust(const float4 *__restrict__ tab, float *__restrict__ mem, int store,
                                            int j, int64_t idx, float D)
{
    float psi1;
    const float r = pml_flow(tab[j], D, mem[idx], &psi1);
    if (store) mem[idx] = psi1;
    return r;
}

// The layer on the C nodes q .. q+C-1 of one lane (those below e), node q at memory index
// idx0 and the next ones `stride` apart: every table entry and memory value is loaded
// before any flow is evaluated, so the loads of a lane overlap.  Lanes whose nodes miss
// both bands return at once.
template <int C>
__device__ __forceinline__ void pml_run(const AxisDev &ax, const float4 *__restrict__ tab, float *__restrict__ mem,
                                        int store, int q, int e, int64_t idx0, int64_t stride, float *w)
{
    if (q >= ax.pml_w && q + C - 1 <= ax.N - ax.pml_w) return;
    float4 t[C];
    float m[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = min(q + c, e - 1);   // a node of the line (e > 0) whatever c
        t[c] = tab[j];
        m[c] = mem[idx0 + (int64_t)(j - q) * stride];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (q + c < e && in_pml(ax, q + c)) {
            float psi1;
            w[c] = pml_flow(t[c], w[c], m[c], &psi1);
            if (store) mem[idx0 + (int64_t)c * stride] = psi1;
        }
    }
}

// ---------------------------------------------------------------------------
// x axis (contiguous): G lanes per unit, C nodes per lane, 64/G units per wave.
// ---------------------------------------------------------------------------

// Solve of one unit (patch l) of an x line by its G lanes (lane k owns nodes
// q = s + kC .. q + C - 1).  `val(i)` reads node i of the line and `val4(i)` nodes
// i..i+3 (i 16-byte aligned, i + 3 <= N; used when `vec_in`).  `issue()` runs once
// the unit's loads are issued (the caller's epilogue prefetch goes there).  On return
// w[c] holds the derivative at node q + c for q + c < e; the function returns the
// derivative at the closing row e (the same value in every lane of the unit).
template <int C, int SOLVE, typename Val, typename Val4, typename Issue>
__device__ __forceinline__ float x_unit(const AxisDev &ax, int k, int G, int l, bool vec_in, Val val, Val4 val4,
                                        Issue issue, float (&w)[C])
{
    const int N = ax.N, M = ax.M;
    const int s = l * M;
    const int e = min(s + M, N);
    const int q = s + k * C;

    // ---- loads -------------------------------------------------------------
    // chunk values u[1..C] = nodes q..q+C-1; u[0], u[C+1] = the neighbouring lanes'
    // edge nodes
    float u[C + 2];
    if (vec_in && ((q & 3) == 0) && q + C - 1 <= N) {
#pragma unroll
        for (int g4 = 0; g4 < C / 4; ++g4) {
            const float4 v = val4(q + 4 * g4);
            u[1 + 4 * g4] = v.x; u[2 + 4 * g4] = v.y; u[3 + 4 * g4] = v.z; u[4 + 4 * g4] = v.w;
        }
    } else {
#pragma unroll
        for (int c = 1; c <= C; ++c) u[c] = val(min(q - 1 + c, N));
    }
    const float uright = val(min(q + C, N));   // kept by the unit's last lane
    float fm[C], fi[C], fs[C];
    row_factors<C, SOLVE>(ax, q, fm, fi, fs);
    const EndRows er = end_rows<SOLVE>(ax, s, e);
    // PMBC taps of rows s and e, shared by the G lanes of the unit: taps k and k+G
    // of this lane (loads without a wait in between; the products are selected later)
    const int nt = ax.ntap;
    const int ss = slot_first(ax, l), se = slot_last(ax, l, e);
    float tcs[2] = {0.f, 0.f}, tvs[2] = {0.f, 0.f}, tce[2] = {0.f, 0.f}, tve[2] = {0.f, 0.f};
    if constexpr (SOLVE != SOLVE_T1) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 0 || G < nt) {
                const int t = min(k + h * G, nt - 1);
                tcs[h] = ax.tap_c[max(ss, 0) * nt + t];
                tce[h] = ax.tap_c[max(se, 0) * nt + t];
                tvs[h] = val(tap_node(ax, s, t));
                tve[h] = val(tap_node(ax, e, t));
            }
        }
    }
    issue();
    float phs = 0.f, phe = 0.f;
    if constexpr (SOLVE != SOLVE_T1) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const bool ok = k + h * G < nt;
            if (ss >= 0 && ok) phs = fmaf(tcs[h], tvs[h], phs);
            if (se >= 0 && ok) phe = fmaf(tce[h], tve[h], phe);
        }
        for (int t = k + 2 * G; t < nt; t += G) {   // halos wider than two taps per lane
            if (ss >= 0) phs = fmaf(ax.tap_c[ss * nt + t], val(tap_node(ax, s, t)), phs);
            if (se >= 0) phe = fmaf(ax.tap_c[se * nt + t], val(tap_node(ax, e, t)), phe);
        }
    }

    // ---- solve -------------------------------------------------------------
    {
        const float left = __shfl_up(u[C], 1, G);
        const float right = __shfl_down(u[1], 1, G);
        u[0] = (k == 0) ? u[1] : left;   // row s never uses node s-1
        u[C + 1] = (k == G - 1) ? uright : right;
    }
    if constexpr (SOLVE != SOLVE_T1) {
        for (int d = G >> 1; d > 0; d >>= 1) {
            phs += __shfl_xor(phs, d, G);
            phe += __shfl_xor(phe, d, G);
        }
    }

    // forward elimination over the chunk from a zero carry
    float y[C], P[C];   // eliminated rhs, carry factor
    float yv = 0.f, pv = 1.f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float r = interior_rhs<SOLVE>(ax, u[c], u[c + 1], u[c + 2]);
        if constexpr (SOLVE != SOLVE_T1) {
            if (c == 0 && k == 0) r = first_row<SOLVE>(ax, er, u[1], u[2], fm[0], fi[0], fs[0]);
        }
        yv = fmaf(-fm[c], yv, r);
        pv = -fm[c] * pv;
        y[c] = yv;
        P[c] = pv;
    }
    // compose the forward carries of the lanes within reach (inclusive scan of
    // affine maps); the first lane's carry is the junction slope
    const int reach = ax.reach;
    float A = pv, B = yv;
    if (k == 0) { B = fmaf(A, phs, B); A = 0.f; }
    for (int d = 1; d < G && d * C < reach; d <<= 1) {
        const float Ap = __shfl_up(A, d, G), Bp = __shfl_up(B, d, G);
        if (k >= d) { B = fmaf(A, Bp, B); A = A * Ap; }
    }
    float yin = __shfl_up(B, 1, G);
    if (k == 0) yin = phs;
#pragma unroll
    for (int c = 0; c < C; ++c) y[c] = fmaf(P[c], yin, y[c]);

    // closing row
    const int kc = (e - 1 - s) / C, cc = (e - 1 - s) - kc * C;
    float we = 0.f;
    if (k == kc) {
        float ylast = 0.f, ulast = 0.f, ue = 0.f;
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (c == cc) { ylast = y[c]; ulast = u[c + 1]; ue = u[c + 2]; }
        we = last_row<SOLVE>(ax, er, ylast, ulast, ue, phe);
    }
    we = __shfl(we, kc, G);

    // back substitution
    float Q[C];
    float wv = 0.f, qv = 1.f;
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        if (q + c < e) {
            wv = fmaf(-fs[c], wv, y[c]) * fi[c];
            qv = -fs[c] * fi[c] * qv;
        }
        w[c] = wv;
        Q[c] = qv;
    }
    float Qm = qv, Wm = wv;
    for (int d = 1; d < G && d * C < reach; d <<= 1) {
        const float Qn = __shfl_down(Qm, d, G), Wn = __shfl_down(Wm, d, G);
        if (k + d < G) { Wm = fmaf(Qm, Wn, Wm); Qm = Qm * Qn; }
    }
    float Qx = __shfl_down(Qm, 1, G), Wx = __shfl_down(Wm, 1, G);
    if (k == G - 1) { Qx = 1.f; Wx = 0.f; }
    // lanes past the closing row hold identity maps, so the closing value enters
    // exactly where the window reaches it (elsewhere its factor is below the tolerance)
    const float wr = fmaf(Qx, we, Wx);
#pragma unroll
    for (int c = 0; c < C; ++c) w[c] = fmaf(Q[c], wr, w[c]);
    return we;
}

template <int C, int SOLVE, int EPI>
__global__ void __launch_bounds__(256) k_line_x(LineArgs a, int G, int nunits)
{
    const AxisDev &ax = a.ax;
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int k = lane & (G - 1);
    const int grp = lane / G;
    const int upw = 64 / G;
    int unit = (blockIdx.x * (blockDim.x >> 6) + wid) * upw + grp;
    const bool uact = unit < nunits;
    if (!uact) unit = nunits - 1;
    const int N = ax.N, M = ax.M, p = ax.p;
    const int line = unit / p;
    const int l = unit - line * p;
    const int lps = a.nz * a.ny;                 // lines per shot
    const int shot = line / lps;
    const int64_t base = (int64_t)line * a.pitch;
    const int64_t mbase = (int64_t)(line - shot * lps) * a.pitch;
    if (a.step_inc && blockIdx.x == 0 && threadIdx.x == 0) *a.step_inc += 1;
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
            const int r = line - shot * lps;
            rowz = r / a.ny;
            rowy = r - rowz * a.ny;
            srcs = segment_has_source(a, shot, 0, 0, rowy, rowz, q, min(q + C, N));
        }
    };
    float w[C];
    const float *__restrict__ icf = a.in_coef ? a.in_coef + mbase : nullptr;
    float we = x_unit<C, SOLVE>(
        ax, k, G, l, true, [&](int i) { return icf ? in[i] * icf[i] : in[i]; },
        [&](int i) {
            float4 v = ld4(in + i);
            if (icf) {
                const float4 c = ld4(icf + i);
                v = make_float4(v.x * c.x, v.y * c.y, v.z * c.z, v.w * c.w);
            }
            return v;
        },
        issue, w);

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
    float we = x_unit<C, SOLVE_D1>(
        ax, k, G, l, true, [&](int i) { return in[i]; }, [&](int i) { return ld4(in + i); }, issue, w);
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
    we = x_unit<C, SOLVE_D1>(
        ax, k, G, l, true, [&](int i) { return line_s[i]; }, [&](int i) { return lds4[i >> 2]; }, [] {}, w);
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
// decomposition is done once per wave.
// Dynamic LDS: 6 * blockDim.x + 64 floats.
template <int C, int SOLVE, int EPI, bool WIDE>
__global__ void __launch_bounds__(1024) k_line_s(LineArgs a, int axis, int CW_, int gx_real)
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
    const float *__restrict__ in = a.in + sbase;
    if (a.step_inc && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *a.step_inc += 1;
    const int N = ax.N, M = ax.M;
    const int s = l * M;
    const int e = min(s + M, N);
    const int q = s + chunk * C;

    // ---- loads -------------------------------------------------------------
    float u[C + 2];
#pragma unroll
    for (int c = 0; c < C + 2; ++c) {
        const int off = mbase + clampi(q - 1 + c, 0, N) * stride;
        u[c] = a.in_coef ? in[off] * a.in_coef[off] : in[off];
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
            tvs[h] = in[mbase + tap_node(ax, s, t) * stride];
            tve[h] = in[mbase + tap_node(ax, e, t) * stride];
        }
    }
    // epilogue operands (small chunks only: they cost 3 registers per node)
    constexpr bool kPre = C <= 8 && EPI != EPI_NORMAL3;
    Pre pre[kPre ? C : 1];
    if constexpr (kPre) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int off = mbase + min(q + c, N) * stride;
            pre[c] = pre_load<EPI>(a, sbase + off, off);
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
                if (ss >= 0) ps = fmaf(ax.tap_c[ss * nt + t], in[mbase + tap_node(ax, s, t) * stride], ps);
                if (se >= 0) pe = fmaf(ax.tap_c[se * nt + t], in[mbase + tap_node(ax, e, t) * stride], pe);
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
            pml_run<C>(ax, a.pml_tab, a.pml_mem, a.pml_store, q, e, sbase + mbase + (int64_t)q * stride, stride, y);
        const int cy = axis == 1 ? 0 : o, cz = axis == 1 ? o : 0;
        const bool srcs = a.src && segment_has_source(a, shot, axis, col, cy, cz, q, min(q + C, N));
        // receivers of this column among the rows this lane updates: trace sample n
        int64_t n = -1;
        if (rinfo.y > 0 && rinfo.w >= q && rinfo.z < q + C) {
            n = *a.d_step - 1;
            if (n >= a.trace_len) n = -1;
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int i = q + c;
            if (i < e) {
                const int off = mbase + i * stride;
                const float D = y[c];
                float v;
                if constexpr (kPre)
                    v = epilogue_pre<EPI>(a, sbase + off, off, shot, D, pre[c], col, axis == 1 ? i : cy,
                                          axis == 1 ? cz : i, srcs);
                else
                    v = epilogue<EPI>(a, sbase + off, off, shot, D, col, axis == 1 ? i : cy, axis == 1 ? cz : i,
                                      srcs);
                if (n >= 0 && i >= rinfo.z && i <= rinfo.w) record_row(a, rinfo, i, v, n);
            }
        }
        if (e == N && chunk == kc) {
            const int off = mbase + N * stride;
            float D = we;
            if (a.pml_mem && in_pml(ax, N)) D = pml_adjust(a.pml_tab, a.pml_mem, a.pml_store, N, sbase + off, D);
            const float v = epilogue<EPI>(a, sbase + off, off, shot, D, col, axis == 1 ? N : cy,
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
    const int *gn = ax.g_node + (int64_t)j * kMaxGatherTaps;
    const float *gc = ax.g_c + (int64_t)j * kMaxGatherTaps;
#pragma unroll
    for (int t = 0; t < kMaxGatherTaps; ++t) {
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
        const int *gn = ax.g_node + (int64_t)r * kMaxGatherTaps;
        const float *gcf = ax.g_c + (int64_t)r * kMaxGatherTaps;
#pragma unroll
        for (int t = 0; t < kMaxGatherTaps; ++t) {
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
    auto col = [&](int i, float4 aw, int4 gn, float4 gc) {
        float o = aw.y * ys[i];
        o = fmaf(aw.x, ys[max(i - 1, 0)], o);
        o = fmaf(aw.z, ys[min(i + 1, N)], o);
        if (gn.x >= 0) o = fmaf(gc.x, ys[gn.x], o);
        if (gn.y >= 0) o = fmaf(gc.y, ys[gn.y], o);
        if (gn.z >= 0) o = fmaf(gc.z, ys[gn.z], o);
        if (gn.w >= 0) o = fmaf(gc.w, ys[gn.w], o);
        return o;
    };
    const int4 none = make_int4(-1, -1, -1, -1);
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const int nthr = blockDim.x;
#pragma unroll
    for (int r = 0; r < C + 1; ++r) {
        const int i = (int)threadIdx.x + r * nthr;
        if (i <= N && ((pw[r] >> (i & 31)) & 1u)) emit(i, col(i, ax.adjw_plain, none, zero4), r);
    }
    for (int i = (int)threadIdx.x + (C + 1) * nthr; i <= N; i += nthr)
        if ((ax.plain[i >> 5] >> (i & 31)) & 1u) emit(i, col(i, ax.adjw_plain, none, zero4), -1);
    for (int t = threadIdx.x; t < ax.nspec; t += nthr) {
        const SpecialCol sc = ax.spec[t];
        emit(sc.row, col(sc.row, sc.aw, sc.gn, sc.gc), -1);
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

__global__ void k_residual_inject(const RecDev *__restrict__ rec, int nrec, float *lam, int64_t shot_stride,
                                  const double *__restrict__ res, int64_t n)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrec) return;
    const RecDev rd = rec[r];
    atomicAdd(lam + (int64_t)rd.shot * shot_stride + rd.node, (float)res[rd.trace_off + n]);
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

__global__ void k_nonfinite(const float *p, int64_t n, int *flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(p[i])) *flag = 1;
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
    if constexpr (C != 8) {
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

hipError_t launch_residual_inject(const RecDev *rec, int nrec, float *lam, int64_t shot_stride,
                                  const double *res, int64_t n, hipStream_t st)
{
    if (nrec <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_residual_inject, nblk(nrec, 256), 256, 0, st, rec, nrec, lam, shot_stride, res, n);
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
    hipLaunchKernelGGL(k_nonfinite, nblk(n, 256), 256, 0, st, p, n, flag);
    return hipGetLastError();
}

}  // namespace loss
