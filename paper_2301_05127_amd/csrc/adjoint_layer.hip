// Pointwise kernel of the adjoint through the absorbing layer (ADE-PML, Sec. 3.3).  A
// pass with the layer updates out += alpha coef (B D + phi1 psi0) and psi' = E psi0 - A D
// at a band node (table entry {E, phi1, A, B} of the node along the pass's axis), and
// out += alpha coef D elsewhere.  Its transpose, given out-bar f (unchanged) and the
// memory variable's bar m (of psi'): D-bar = B alpha coef f - A m, and m becomes the bar
// of psi0, phi1 alpha coef f + E m.  The transposed derivative then takes D-bar.  A null
// coef stands for 1 (an operand the caller has already combined).
#include <hip/hip_runtime.h>

#include "loss_internal.h"

namespace loss {

namespace {

__global__ void k_pml_adj_operand(float *__restrict__ w, const float *__restrict__ f, const float *__restrict__ coef,
                                  float alpha, float *__restrict__ m, const float4 *__restrict__ tab, int axis,
                                  int pml_w, int N, int nx, int ny, int64_t pitch, int64_t per_shot, int S,
                                  int64_t total)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t rows = per_shot / pitch;       // ny * nz rows per shot
    const int64_t row = i / nx;
    const int x = (int)(i - row * nx);
    const int64_t shot = row / rows;
    if (shot >= S) return;
    const int64_t r = row - shot * rows;
    const int64_t p = r * pitch + x;             // node within the shot (media index)
    const int64_t q = shot * per_shot + p;
    const int j = axis == 0 ? x : (axis == 1 ? (int)(r % ny) : (int)(r / ny));
    const float c = alpha * (coef ? coef[p] : 1.f) * f[q];
    if (j < pml_w || j > N - pml_w) {
        const float4 t = tab[j];
        const float mb = m[q];
        w[q] = fmaf(t.w, c, -t.z * mb);
        m[q] = fmaf(t.y, c, t.x * mb);
    } else {
        w[q] = c;
    }
}

}  // namespace

hipError_t launch_pml_adj_operand(float *w, const float *f, const float *coef, float alpha, float *m,
                                  const float4 *tab, int axis, int pml_w, int N, int nx, int ny, int64_t pitch,
                                  int64_t per_shot, int S, hipStream_t st)
{
    const int64_t total = (int64_t)S * (per_shot / pitch) * nx;
    hipLaunchKernelGGL(k_pml_adj_operand, (unsigned)((total + 255) / 256), 256, 0, st, w, f, coef, alpha, m, tab, axis,
                       pml_w, N, nx, ny, pitch, per_shot, S, total);
    return hipGetLastError();
}

}  // namespace loss
