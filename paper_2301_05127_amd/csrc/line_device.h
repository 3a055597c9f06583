// Device building blocks of the line kernels (shared by every HIP source of the
// library): junction taps of the PMBC (paper Sec. 3.2, eq. PMBC), sources in the
// epilogues, the row factors of the per-axis derivative systems, the absorbing-layer
// sub-flow (Sec. 3.3), and the solve of one patch of one line by a group of G lanes
// (x_unit), which takes the line's node values through an accessor so that callers can
// serve them from global memory or from LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

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
#pragma unroll
        for (int j = 0; j < 3; ++j) {   // static indices: the pointers may live in registers
            if (j >= a.nout) break;
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
#pragma unroll
        for (int j = 1; j < 3; ++j) {
            if (j >= a.nout) break;
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

// The arguments with every array pointer moved to one lane's column: field arrays by
// `fe` elements (shot and column), media arrays by `me`, the divergence store to the
// shot's slice; null pointers stay null.  Node indices handed to the epilogue helpers
// with these arguments are then row offsets alone, the same for every lane of a wave
// whose lanes share their rows.
__device__ __forceinline__ LineArgs lane_args(const LineArgs &a, int64_t fe, int64_t me, int shot)
{
    LineArgs r = a;
    auto mv = [](auto *p, int64_t o) { return p ? p + o : p; };
    r.in = a.in + fe;
    r.in_coef = mv(a.in_coef, me);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        r.out[j] = mv(a.out[j], fe);
        r.coef[j] = mv(a.coef[j], me);
    }
    r.aux = mv(a.aux, fe);
    r.aux2 = mv(a.aux2, fe);
    r.div = mv(a.div, (int64_t)shot * a.div_shot_stride + me);
    r.div_shot_stride = 0;
    r.bcoef = mv(a.bcoef, me);
    r.pml_mem = mv(a.pml_mem, fe);
    return r;
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

// Lane exchanges inside the G lanes of a unit (G a power of two, units aligned to
// multiples of G).  When G <= 16 a unit lies inside one 16-lane DPP row and a shift by
// d is one row_shr / row_shl move (lane i of the row receives lane i - d, resp. i + d;
// sources outside the row give 0); wider units take the LDS permute.  Values that a
// shift brings in from outside the unit are for the caller to discard.
template <int D>
__device__ __forceinline__ float row_shift_up(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + D, 0xF, 0xF, true));
}
template <int D>
__device__ __forceinline__ float row_shift_down(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x100 + D, 0xF, 0xF, true));
}
// Row shifts whose lanes with a source outside the 16-lane row receive `fill` (DPP with
// the destination disabled for those lanes, its initial value kept).
template <int D>
__device__ __forceinline__ float row_shift_up_fill(float v, float fill)
{
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v), 0x110 + D, 0xF, 0xF, false));
}
template <int D>
__device__ __forceinline__ float row_shift_down_fill(float v, float fill)
{
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v), 0x100 + D, 0xF, 0xF, false));
}
struct UnitLanes {
    int G;
    template <int D>
    __device__ __forceinline__ float up(float v) const
    {
        if constexpr (D < 16) {
            if (G <= 16) return row_shift_up<D>(v);
        }
        return __shfl_up(v, D, G);
    }
    template <int D>
    __device__ __forceinline__ float down(float v) const
    {
        if constexpr (D < 16) {
            if (G <= 16) return row_shift_down<D>(v);
        }
        return __shfl_down(v, D, G);
    }
};

// Solve of one unit (patch l) of an x line by its G lanes (lane k owns nodes
// q = s + kC .. q + C - 1).  `val(i)` reads node i of the line and `val4(i)` nodes
// i..i+3 (i 16-byte aligned, i + 3 <= N; used when `vec_in`).  `issue()` runs once
// the unit's loads are issued (the caller's epilogue prefetch goes there).  On return
// w[c] holds the derivative at node q + c for q + c < e; the function returns the
// derivative at the closing row e (the same value in every lane of the unit).
// FULL16: the caller guarantees G = 16 and a whole unit (e - s = M = 16 C, so the
// closing row follows the last lane's last node); the lane exchanges are then row shifts
// that bring in the identity map from outside the unit, with no masks, and the closing
// lane is known.
template <int C, int SOLVE, bool FULL16 = false, typename Val, typename Val4, typename Issue>
__device__ __forceinline__ float x_unit(const AxisDev &ax, int k, int G, int l, bool vec_in, Val val, Val4 val4,
                                        Issue issue, float (&w)[C])
{
    if constexpr (FULL16) G = 16;
    const int N = ax.N, M = ax.M;
    const int s = l * M;
    const int e = FULL16 ? s + 16 * C : min(s + M, N);
    const int q = s + k * C;
    const UnitLanes lanes{G};
    using I = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I4 = std::integral_constant<int, 4>;
    using I8 = std::integral_constant<int, 8>;
    using I16 = std::integral_constant<int, 16>;
    using I32 = std::integral_constant<int, 32>;

    // ---- loads -------------------------------------------------------------
    // chunk values u[1..C] = nodes q..q+C-1; u[0], u[C+1] = the neighbouring lanes'
    // edge nodes
    float u[C + 2];
    if (FULL16 || (vec_in && ((q & 3) == 0) && q + C - 1 <= N)) {
#pragma unroll
        for (int g4 = 0; g4 < C / 4; ++g4) {
            const float4 v = val4(q + 4 * g4);
            u[1 + 4 * g4] = v.x; u[2 + 4 * g4] = v.y; u[3 + 4 * g4] = v.z; u[4 + 4 * g4] = v.w;
        }
    } else {
#pragma unroll
        for (int c = 1; c <= C; ++c) u[c] = val(min(q - 1 + c, N));
    }
    float uright = 0.f;   // the node past the unit's last chunk, read by its last lane
    if (k == G - 1) uright = val(min(q + C, N));
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
        const float left = lanes.up<1>(u[C]);
        const float right = lanes.down<1>(u[1]);
        u[0] = (k == 0) ? u[1] : left;   // row s never uses node s-1
        u[C + 1] = (k == G - 1) ? uright : right;
    }
    if constexpr (SOLVE != SOLVE_T1) {
        if constexpr (FULL16) {
            // the start junction's sum to lane 0 (suffix sums), the end junction's to the
            // closing lane 15 (prefix sums); sources outside the row bring in 0
            auto step = [&](auto dc) {
                constexpr int D = decltype(dc)::value;
                phs += row_shift_down_fill<D>(phs, 0.f);
                phe += row_shift_up_fill<D>(phe, 0.f);
            };
            step(I{}); step(I2{}); step(I4{}); step(I8{});
        } else {
            // the same sums and order: suffix sums to lane 0 for the start junction,
            // prefix sums to the last lane for the end junction
            auto step = [&](auto dc) {
                constexpr int D = decltype(dc)::value;
                if (D < G) {
                    const float a = lanes.down<D>(phs), b = lanes.up<D>(phe);
                    if (k + D < G) phs += a;
                    if (k >= D) phe += b;
                }
            };
            step(I{}); step(I2{}); step(I4{}); step(I8{}); step(I16{}); step(I32{});
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
    auto scan_up = [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        if constexpr (FULL16) {
            // lanes with no lane D back take the identity map (A 1, B 0)
            if (D < 16 && D * C < reach) {
                const float Ap = row_shift_up_fill<D < 16 ? D : 1>(A, 1.f);
                const float Bp = row_shift_up_fill<D < 16 ? D : 1>(B, 0.f);
                B = fmaf(A, Bp, B);
                A = A * Ap;
            }
        } else {
            if (D < G && D * C < reach) {
                const float Ap = lanes.up<D>(A), Bp = lanes.up<D>(B);
                if (k >= D) { B = fmaf(A, Bp, B); A = A * Ap; }
            }
        }
    };
    scan_up(I{}); scan_up(I2{}); scan_up(I4{}); scan_up(I8{}); scan_up(I16{}); scan_up(I32{});
    float yin = lanes.up<1>(B);
    if (k == 0) yin = phs;
#pragma unroll
    for (int c = 0; c < C; ++c) y[c] = fmaf(P[c], yin, y[c]);

    // closing row (its junction sum is the unit's end-junction sum)
    float we = 0.f;
    if constexpr (FULL16) {
        if (k == 15) we = last_row<SOLVE>(ax, er, y[C - 1], u[C], u[C + 1], phe);
        we = __shfl(we, 15, 16);
    } else {
        const int kc = (e - 1 - s) / C, cc = (e - 1 - s) - kc * C;
        if constexpr (SOLVE != SOLVE_T1) phe = __shfl(phe, G - 1, G);
        if (k == kc) {
            float ylast = 0.f, ulast = 0.f, ue = 0.f;
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (c == cc) { ylast = y[c]; ulast = u[c + 1]; ue = u[c + 2]; }
            we = last_row<SOLVE>(ax, er, ylast, ulast, ue, phe);
        }
        we = __shfl(we, kc, G);
    }

    // back substitution
    float Q[C];
    float wv = 0.f, qv = 1.f;
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        if (FULL16 || q + c < e) {
            wv = fmaf(-fs[c], wv, y[c]) * fi[c];
            qv = -fs[c] * fi[c] * qv;
        }
        w[c] = wv;
        Q[c] = qv;
    }
    float Qm = qv, Wm = wv;
    auto scan_down = [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        if constexpr (FULL16) {
            if (D < 16 && D * C < reach) {
                const float Qn = row_shift_down_fill<D < 16 ? D : 1>(Qm, 1.f);
                const float Wn = row_shift_down_fill<D < 16 ? D : 1>(Wm, 0.f);
                Wm = fmaf(Qm, Wn, Wm);
                Qm = Qm * Qn;
            }
        } else {
            if (D < G && D * C < reach) {
                const float Qn = lanes.down<D>(Qm), Wn = lanes.down<D>(Wm);
                if (k + D < G) { Wm = fmaf(Qm, Wn, Wm); Qm = Qm * Qn; }
            }
        }
    };
    scan_down(I{}); scan_down(I2{}); scan_down(I4{}); scan_down(I8{}); scan_down(I16{}); scan_down(I32{});
    float Qx, Wx;
    if constexpr (FULL16) {
        Qx = row_shift_down_fill<1>(Qm, 1.f);   // the last lane takes the identity map
        Wx = row_shift_down_fill<1>(Wm, 0.f);
    } else {
        Qx = lanes.down<1>(Qm);
        Wx = lanes.down<1>(Wm);
        if (k == G - 1) { Qx = 1.f; Wx = 0.f; }
    }
    // lanes past the closing row hold identity maps, so the closing value enters
    // exactly where the window reaches it (elsewhere its factor is below the tolerance)
    const float wr = fmaf(Qx, we, Wx);
#pragma unroll
    for (int c = 0; c < C; ++c) w[c] = fmaf(Q[c], wr, w[c]);
    return we;
}

// The solve of x_unit in three parts, for kernels that solve the same patches on many
// lines: XFix holds what depends only on the patch and the lane (row factors, end rows,
// PMBC tap coefficients and tap nodes), XVals the node values of one line (the lane's
// chunk and the node past the unit, x_vals_chunk; the tap values, x_vals_taps), and
// x_solve is x_unit's elimination from there on, operation for operation (the fields of
// the two forms are compared bit for bit), with `val` serving taps past the first two of
// a lane.  x_unit keeps its single-function form: written as these three parts it
// compiled the fused x kernel with 32-lane units (8 nodes per lane, patches of 256) a
// fifth slower.
template <int C, int SOLVE>
struct XFix {
    int s, e, q, ss, se;
    float fm[C], fi[C], fs[C];
    EndRows er;
    float tcs[2], tce[2];   // coefficients of taps k and k + G of rows s and e
    int ns[2], ne[2];       // their nodes
};

template <int C>
struct XVals {
    float u[C + 2];         // u[1..C] = nodes q..q+C-1 (u[0], u[C+1] filled by the solve)
    float uright;           // the node past the unit's last chunk (its last lane)
    float tvs[2], tve[2];   // values at the tap nodes
};

template <int C, int SOLVE, bool FULL16 = false>
__device__ __forceinline__ XFix<C, SOLVE> x_fix(const AxisDev &ax, int k, int G, int l)
{
    if constexpr (FULL16) G = 16;
    XFix<C, SOLVE> f;
    const int N = ax.N, M = ax.M;
    f.s = l * M;
    f.e = FULL16 ? f.s + 16 * C : min(f.s + M, N);
    f.q = f.s + k * C;
    row_factors<C, SOLVE>(ax, f.q, f.fm, f.fi, f.fs);
    f.er = end_rows<SOLVE>(ax, f.s, f.e);
    // PMBC taps of rows s and e, shared by the G lanes of the unit: taps k and k+G
    // of this lane (the products are selected in the solve)
    const int nt = ax.ntap;
    f.ss = slot_first(ax, l);
    f.se = slot_last(ax, l, f.e);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        f.tcs[h] = f.tce[h] = 0.f;
        f.ns[h] = f.ne[h] = 0;
    }
    if constexpr (SOLVE != SOLVE_T1) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 0 || G < nt) {
                const int t = min(k + h * G, nt - 1);
                f.tcs[h] = ax.tap_c[max(f.ss, 0) * nt + t];
                f.tce[h] = ax.tap_c[max(f.se, 0) * nt + t];
                f.ns[h] = tap_node(ax, f.s, t);
                f.ne[h] = tap_node(ax, f.e, t);
            }
        }
    }
    return f;
}

// the lane's chunk u[1..C] and, on the unit's last lane, the node past the unit
template <int C, bool FULL16 = false, typename Val, typename Val4>
__device__ __forceinline__ void x_vals_chunk(const AxisDev &ax, int q, int k, int G, bool vec_in, Val val, Val4 val4,
                                             XVals<C> &v)
{
    if constexpr (FULL16) G = 16;
    const int N = ax.N;
    if (FULL16 || (vec_in && ((q & 3) == 0) && q + C - 1 <= N)) {
#pragma unroll
        for (int g4 = 0; g4 < C / 4; ++g4) {
            const float4 x = val4(q + 4 * g4);
            v.u[1 + 4 * g4] = x.x; v.u[2 + 4 * g4] = x.y; v.u[3 + 4 * g4] = x.z; v.u[4 + 4 * g4] = x.w;
        }
    } else {
#pragma unroll
        for (int c = 1; c <= C; ++c) v.u[c] = val(min(q - 1 + c, N));
    }
    v.u[0] = v.u[C + 1] = 0.f;
    v.uright = 0.f;
    if (k == G - 1) v.uright = val(min(q + C, N));
}

// the values at the lane's tap nodes
template <int C, int SOLVE, bool FULL16 = false, typename Val>
__device__ __forceinline__ void x_vals_taps(const AxisDev &ax, const XFix<C, SOLVE> &f, int k, int G, Val val,
                                            XVals<C> &v)
{
    if constexpr (FULL16) G = 16;
#pragma unroll
    for (int h = 0; h < 2; ++h) v.tvs[h] = v.tve[h] = 0.f;
    if constexpr (SOLVE != SOLVE_T1) {
        const int nt = ax.ntap;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 0 || G < nt) {
                v.tvs[h] = val(f.ns[h]);
                v.tve[h] = val(f.ne[h]);
            }
        }
    }
}

// `val` serves the taps past the first two of each lane (halos wider than 2G - 1 nodes)
template <int C, int SOLVE, bool FULL16 = false, typename Val>
__device__ __forceinline__ float x_solve(const AxisDev &ax, const XFix<C, SOLVE> &f, XVals<C> &v, int k, int G,
                                         Val val, float (&w)[C])
{
    if constexpr (FULL16) G = 16;
    const int s = f.s, e = f.e, q = f.q;
    float(&u)[C + 2] = v.u;
    const UnitLanes lanes{G};
    using I = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I4 = std::integral_constant<int, 4>;
    using I8 = std::integral_constant<int, 8>;
    using I16 = std::integral_constant<int, 16>;
    using I32 = std::integral_constant<int, 32>;
    float fm[C], fi[C], fs[C];
#pragma unroll
    for (int c = 0; c < C; ++c) { fm[c] = f.fm[c]; fi[c] = f.fi[c]; fs[c] = f.fs[c]; }
    const EndRows &er = f.er;
    const int ss = f.ss, se = f.se;

    float phs = 0.f, phe = 0.f;
    if constexpr (SOLVE != SOLVE_T1) {
        const int nt = ax.ntap;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const bool ok = k + h * G < nt;
            if (ss >= 0 && ok) phs = fmaf(f.tcs[h], v.tvs[h], phs);
            if (se >= 0 && ok) phe = fmaf(f.tce[h], v.tve[h], phe);
        }
        for (int t = k + 2 * G; t < nt; t += G) {   // halos wider than two taps per lane
            if (ss >= 0) phs = fmaf(ax.tap_c[ss * nt + t], val(tap_node(ax, s, t)), phs);
            if (se >= 0) phe = fmaf(ax.tap_c[se * nt + t], val(tap_node(ax, e, t)), phe);
        }
    }

    // ---- solve -------------------------------------------------------------
    {
        const float left = lanes.up<1>(u[C]);
        const float right = lanes.down<1>(u[1]);
        u[0] = (k == 0) ? u[1] : left;   // row s never uses node s-1
        u[C + 1] = (k == G - 1) ? v.uright : right;
    }
    if constexpr (SOLVE != SOLVE_T1) {
        if constexpr (FULL16) {
            // the start junction's sum to lane 0 (suffix sums), the end junction's to the
            // closing lane 15 (prefix sums); sources outside the row bring in 0
            auto step = [&](auto dc) {
                constexpr int D = decltype(dc)::value;
                phs += row_shift_down_fill<D>(phs, 0.f);
                phe += row_shift_up_fill<D>(phe, 0.f);
            };
            step(I{}); step(I2{}); step(I4{}); step(I8{});
        } else {
            // the same sums and order: suffix sums to lane 0 for the start junction,
            // prefix sums to the last lane for the end junction
            auto step = [&](auto dc) {
                constexpr int D = decltype(dc)::value;
                if (D < G) {
                    const float a = lanes.down<D>(phs), b = lanes.up<D>(phe);
                    if (k + D < G) phs += a;
                    if (k >= D) phe += b;
                }
            };
            step(I{}); step(I2{}); step(I4{}); step(I8{}); step(I16{}); step(I32{});
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
    auto scan_up = [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        if constexpr (FULL16) {
            // lanes with no lane D back take the identity map (A 1, B 0)
            if (D < 16 && D * C < reach) {
                const float Ap = row_shift_up_fill<D < 16 ? D : 1>(A, 1.f);
                const float Bp = row_shift_up_fill<D < 16 ? D : 1>(B, 0.f);
                B = fmaf(A, Bp, B);
                A = A * Ap;
            }
        } else {
            if (D < G && D * C < reach) {
                const float Ap = lanes.up<D>(A), Bp = lanes.up<D>(B);
                if (k >= D) { B = fmaf(A, Bp, B); A = A * Ap; }
            }
        }
    };
    scan_up(I{}); scan_up(I2{}); scan_up(I4{}); scan_up(I8{}); scan_up(I16{}); scan_up(I32{});
    float yin = lanes.up<1>(B);
    if (k == 0) yin = phs;
#pragma unroll
    for (int c = 0; c < C; ++c) y[c] = fmaf(P[c], yin, y[c]);

    // closing row (its junction sum is the unit's end-junction sum)
    float we = 0.f;
    if constexpr (FULL16) {
        if (k == 15) we = last_row<SOLVE>(ax, er, y[C - 1], u[C], u[C + 1], phe);
        we = __shfl(we, 15, 16);
    } else {
        const int kc = (e - 1 - s) / C, cc = (e - 1 - s) - kc * C;
        if constexpr (SOLVE != SOLVE_T1) phe = __shfl(phe, G - 1, G);
        if (k == kc) {
            float ylast = 0.f, ulast = 0.f, ue = 0.f;
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (c == cc) { ylast = y[c]; ulast = u[c + 1]; ue = u[c + 2]; }
            we = last_row<SOLVE>(ax, er, ylast, ulast, ue, phe);
        }
        we = __shfl(we, kc, G);
    }

    // back substitution
    float Q[C];
    float wv = 0.f, qv = 1.f;
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        if (FULL16 || q + c < e) {
            wv = fmaf(-fs[c], wv, y[c]) * fi[c];
            qv = -fs[c] * fi[c] * qv;
        }
        w[c] = wv;
        Q[c] = qv;
    }
    float Qm = qv, Wm = wv;
    auto scan_down = [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        if constexpr (FULL16) {
            if (D < 16 && D * C < reach) {
                const float Qn = row_shift_down_fill<D < 16 ? D : 1>(Qm, 1.f);
                const float Wn = row_shift_down_fill<D < 16 ? D : 1>(Wm, 0.f);
                Wm = fmaf(Qm, Wn, Wm);
                Qm = Qm * Qn;
            }
        } else {
            if (D < G && D * C < reach) {
                const float Qn = lanes.down<D>(Qm), Wn = lanes.down<D>(Wm);
                if (k + D < G) { Wm = fmaf(Qm, Wn, Wm); Qm = Qm * Qn; }
            }
        }
    };
    scan_down(I{}); scan_down(I2{}); scan_down(I4{}); scan_down(I8{}); scan_down(I16{}); scan_down(I32{});
    float Qx, Wx;
    if constexpr (FULL16) {
        Qx = row_shift_down_fill<1>(Qm, 1.f);   // the last lane takes the identity map
        Wx = row_shift_down_fill<1>(Wm, 0.f);
    } else {
        Qx = lanes.down<1>(Qm);
        Wx = lanes.down<1>(Wm);
        if (k == G - 1) { Qx = 1.f; Wx = 0.f; }
    }
    // lanes past the closing row hold identity maps, so the closing value enters
    // exactly where the window reaches it (elsewhere its factor is below the tolerance)
    const float wr = fmaf(Qx, we, Wx);
#pragma unroll
    for (int c = 0; c < C; ++c) w[c] = fmaf(Q[c], wr, w[c]);
    return we;
}

}  // namespace
}  // namespace loss
