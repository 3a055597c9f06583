// Pointwise kernels of the elastic discrete adjoint (the transposed derivatives reuse
// the line kernels of kernels.hip).  The forward stress sub-flow B (Sec. 3.3, Strang
// splitting of the velocity-stress system of Sec. 2) is
//   sigma_kk += (dt lambda) tr(e) + 2 (dt mu) e_kk,  sigma_ij += (dt mu) g_ij  (i < j),
// e_kk = D_k v_k, g_ij = D_j v_i + D_i v_j; the media hold dt lambda, dt mu,
// dt (lambda + 2 mu) and dt / rho.  Fields are padded rows of `pitch` floats, shots
// `shot_stride` apart; only the nx valid columns of a row are touched.
#include <hip/hip_runtime.h>

#include "loss_internal.h"

namespace loss {

namespace {

__device__ __forceinline__ bool valid_node(int64_t i, int nx, int64_t pitch, int64_t per_shot, int S,
                                           int64_t *shot_off, int64_t *p)
{
    const int64_t rows = per_shot / pitch;
    const int64_t row = i / nx;                 // over all shots
    const int x = (int)(i - row * nx);
    const int64_t shot = row / rows;
    if (shot >= S) return false;
    *p = (row - shot * rows) * pitch + x;
    *shot_off = shot * per_shot;
    return true;
}

// w = (dt(lambda + 2 mu)) sbar_kk + (dt lambda) (sum of the other two normal bars): the
// operand of D_k^T in the transpose of B for velocity k.
__global__ void k_el_normal_operand(float *__restrict__ w, const float *__restrict__ s11,
                                    const float *__restrict__ s22, const float *__restrict__ s33,
                                    const float *__restrict__ l2m, const float *__restrict__ lam, int k, int nx,
                                    int64_t pitch, int64_t per_shot, int S, int64_t total)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    int64_t so, p;
    if (!valid_node(i, nx, pitch, per_shot, S, &so, &p)) return;
    const float a = s11[so + p], b = s22[so + p], c = s33[so + p];
    const float own = k == 0 ? a : (k == 1 ? b : c);
    const float others = k == 0 ? b + c : (k == 1 ? a + c : a + b);
    w[so + p] = fmaf(l2m[p], own, lam[p] * others);
}

// dJ/dlambda += dt tr(e) (sbar_11 + sbar_22 + sbar_33),
// dJ/dmu     += dt (2 sum_k e_kk sbar_kk + sum_{i<j} g_ij sbar_ij), summed over shots in
// FP64.  e: six strain fields (e11, e22, e33, g12, g13, g23) of the state B was applied
// to; sb: the six stress bars (11, 22, 33, 12, 13, 23).  g: two padded accumulators.
struct Six {
    const float *p[6];
};

__global__ void k_el_grad_accum(double *__restrict__ gl, double *__restrict__ gm, Six e, Six sb, double dt,
                                int nx, int64_t pitch, int64_t per_shot, int S, int64_t total_one_shot)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total_one_shot) return;
    int64_t so, p;
    if (!valid_node(i, nx, pitch, per_shot, 1, &so, &p)) return;
    double al = 0.0, am = 0.0;
    for (int s = 0; s < S; ++s) {
        const int64_t q = (int64_t)s * per_shot + p;
        const double e11 = e.p[0][q], e22 = e.p[1][q], e33 = e.p[2][q];
        const double b11 = sb.p[0][q], b22 = sb.p[1][q], b33 = sb.p[2][q];
        al += (e11 + e22 + e33) * (b11 + b22 + b33);
        am += 2.0 * (e11 * b11 + e22 * b22 + e33 * b33) + (double)e.p[3][q] * sb.p[3][q] +
              (double)e.p[4][q] * sb.p[4][q] + (double)e.p[5][q] * sb.p[5][q];
    }
    gl[p] += dt * al;
    gm[p] += dt * am;
}

// dJ/db += dt sum_i ubar_i (sum_j D_j sigma_ij) per velocity step (b = 1/rho drives the
// velocity sub-flow only), summed over shots in FP64; div: the three drives of the step,
// ubar: the velocity bars after it.
struct Three {
    const float *p[3];
};

__global__ void k_el_grad_b(double *__restrict__ gb, Three ub, Three dv, double dt, int nx, int64_t pitch,
                            int64_t per_shot, int S, int64_t total_one_shot)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total_one_shot) return;
    int64_t so, p;
    if (!valid_node(i, nx, pitch, per_shot, 1, &so, &p)) return;
    double acc = 0.0;
    for (int s = 0; s < S; ++s) {
        const int64_t q = (int64_t)s * per_shot + p;
#pragma unroll
        for (int c = 0; c < 3; ++c) acc += (double)ub.p[c][q] * (double)dv.p[c][q];
    }
    gb[p] += dt * acc;
}

// the body-force part of the same term: dJ/db += scale f(t_n) w(x) ubar_comp(x) of every
// force source; one thread per node of the box covering all force footprints, which sums
// the sources in their order (shots may share nodes) and adds once: no atomics
__global__ void k_el_grad_force(double *gb, const SrcDev *__restrict__ src, int nsrc, float *const *adj,
                                const float *__restrict__ wpool, const float *__restrict__ wavpool,
                                int64_t shot_stride, int64_t pitch, int64_t plane, int64_t n, double scale, int x0,
                                int y0, int z0, int bx, int by, int64_t total)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int x = x0 + (int)(t % bx), y = y0 + (int)((t / bx) % by), z = z0 + (int)(t / ((int64_t)bx * by));
    const int64_t midx = (int64_t)z * plane + (int64_t)y * pitch + x;
    double acc = 0.0;
    bool any = false;
    for (int k = 0; k < nsrc; ++k) {
        const SrcDev &sd = src[k];
        if (!sd.force || n < 0 || n >= sd.nt) continue;
        const unsigned ix = (unsigned)(x - sd.x0), iy = (unsigned)(y - sd.y0), iz = (unsigned)(z - sd.z0);
        if (ix >= (unsigned)sd.bx || iy >= (unsigned)sd.by || iz >= (unsigned)sd.bz) continue;
        const double amp = scale * (double)wavpool[sd.wav_off + n];
        const float *ub = adj[sd.field0] + (int64_t)sd.shot * shot_stride;
        acc += amp * (double)wpool[sd.w_off + ((int64_t)iz * sd.by + iy) * sd.bx + ix] * (double)ub[midx];
        any = true;
    }
    if (any) gb[midx] += acc;
}

// padded accumulators -> dense gradients.  mode 0: (dJ/dlambda, dJ/dmu); 1: (dJ/dvp,
// dJ/dvs) with rho fixed, from lambda = rho (vp^2 - 2 vs^2), mu = rho vs^2; 2: mode 0 and
// dJ/drho with lambda, mu fixed (= -b^2 dJ/db); 3: mode 1 and dJ/drho with vp, vs fixed
// (= dJ/dlambda (vp^2 - 2 vs^2) + dJ/dmu vs^2 - b^2 dJ/db).
__global__ void k_el_grad_unpad(const double *__restrict__ gl, const double *__restrict__ gm,
                                const double *__restrict__ gb, double *g, int nx, int64_t pitch,
                                const float *__restrict__ vp, const float *__restrict__ vs,
                                const float *__restrict__ rho, int mode, int64_t nodes)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nodes) return;
    const int x = (int)(idx % nx);
    const int64_t p = (idx / nx) * pitch + x;
    const double a = gl[p], b = gm[p];
    const double r = rho[idx], cp = vp[idx], cs = vs[idx];
    const bool vel = mode == 1 || mode == 3;
    g[idx] = vel ? a * 2.0 * r * cp : a;
    g[nodes + idx] = vel ? a * (-4.0 * r * cs) + b * 2.0 * r * cs : b;
    if (mode >= 2) {
        const double drho_lm = -gb[p] / (r * r);
        g[2 * nodes + idx] = mode == 2 ? drho_lm : a * (cp * cp - 2.0 * cs * cs) + b * cs * cs + drho_lm;
    }
}

}  // namespace

hipError_t launch_el_normal_operand(float *w, const float *s11, const float *s22, const float *s33,
                                    const float *l2m, const float *lam, int k, int nx, int64_t pitch,
                                    int64_t per_shot, int S, hipStream_t st)
{
    const int64_t total = (int64_t)S * (per_shot / pitch) * nx;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_el_normal_operand, blocks, 256, 0, st, w, s11, s22, s33, l2m, lam, k, nx, pitch,
                       per_shot, S, total);
    return hipGetLastError();
}

hipError_t launch_el_grad_accum(double *gl, double *gm, const float *const *strain, const float *const *sbar,
                                double dt, int nx, int64_t pitch, int64_t per_shot, int S, hipStream_t st)
{
    Six e, sb;
    for (int k = 0; k < 6; ++k) { e.p[k] = strain[k]; sb.p[k] = sbar[k]; }
    const int64_t total = (per_shot / pitch) * nx;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_el_grad_accum, blocks, 256, 0, st, gl, gm, e, sb, dt, nx, pitch, per_shot, S, total);
    return hipGetLastError();
}

hipError_t launch_el_grad_b(double *gb, const float *const *ubar, const float *const *div, double dt, int nx,
                            int64_t pitch, int64_t per_shot, int S, hipStream_t st)
{
    Three u, d;
    for (int k = 0; k < 3; ++k) { u.p[k] = ubar[k]; d.p[k] = div[k]; }
    const int64_t total = (per_shot / pitch) * nx;
    hipLaunchKernelGGL(k_el_grad_b, (unsigned)((total + 255) / 256), 256, 0, st, gb, u, d, dt, nx, pitch, per_shot, S,
                       total);
    return hipGetLastError();
}

hipError_t launch_el_grad_force(double *gb, const SrcDev *src, int nsrc, float *const *adj, const float *wpool,
                                const float *wavpool, int64_t shot_stride, int64_t pitch, int64_t plane, int64_t n,
                                double scale, const int *box, hipStream_t st)
{
    if (nsrc <= 0 || box[1] <= box[0]) return hipSuccess;
    const int bx = box[1] - box[0], by = box[3] - box[2], bz = box[5] - box[4];
    const int64_t total = (int64_t)bx * by * bz;
    hipLaunchKernelGGL(k_el_grad_force, (unsigned)((total + 255) / 256), 256, 0, st, gb, src, nsrc, adj, wpool,
                       wavpool, shot_stride, pitch, plane, n, scale, box[0], box[2], box[4], bx, by, total);
    return hipGetLastError();
}

hipError_t launch_el_grad_unpad(const double *gl, const double *gm, const double *gb, double *g, int nx,
                                int64_t pitch, const float *vp, const float *vs, const float *rho, int mode,
                                int64_t nodes, hipStream_t st)
{
    hipLaunchKernelGGL(k_el_grad_unpad, (unsigned)((nodes + 255) / 256), 256, 0, st, gl, gm, gb, g, nx, pitch, vp,
                       vs, rho, mode, nodes);
    return hipGetLastError();
}

}  // namespace loss
