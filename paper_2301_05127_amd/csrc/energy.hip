// FP64 energy of the wavefield of each shot (a monitor of the velocity-stress system of
// paper Sec. 2: kinetic energy 1/2 rho |v|^2 plus the strain energy 1/2 sigma : C^-1 : sigma,
// summed over the nodes with the cell volume).  Isotropic compliance written through the
// deviator s = sigma - (tr sigma / 3) I:  sigma : C^-1 : sigma = s:s / (2 mu) + (tr sigma)^2 /
// (9 K), K = lambda + 2 mu / 3, so a node with mu = 0 (no shear stress) needs no division by
// mu.  Acoustic: 1/2 (rho (v1^2 + v3^2) + sigma^2 / K).  Every sum is FP64 and in a fixed
// order (per-block trees, then one block per shot over the block partials), so a repeated
// call gives the same bits.
#include <hip/hip_runtime.h>

#include "loss_internal.h"

namespace loss {

namespace {

constexpr int kEnergyThreads = 256;

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = kEnergyThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    return sh[0];
}

// grid (nblocks, S): block b of shot s sums nodes [b * per_block, (b + 1) * per_block)
__global__ void __launch_bounds__(kEnergyThreads) k_energy_partial(EnergyArgs a, int64_t per_block, double *partial)
{
    __shared__ double sh[kEnergyThreads];
    const int shot = blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.x * per_block;
    const int64_t i1 = min(i0 + per_block, a.nodes);
    const int64_t sbase = (int64_t)shot * a.shot_stride;
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kEnergyThreads) {
        const int64_t row = i / a.nx;                       // (z, y) row of the dense media
        const int x = (int)(i - row * a.nx);
        const int64_t p = sbase + row * a.pitch + x;        // padded field element
        const double rho = a.rho[i], vp = a.vp[i];
        double kin = 0.0;
        for (int c = 0; c < a.nv; ++c) {
            const double v = a.v[c][p];
            kin += v * v;
        }
        double e = 0.5 * rho * kin;
        if (a.ns == 1) {
            const double s = a.s[0][p];
            e += 0.5 * s * s / (rho * vp * vp);
        } else {
            const double vs = a.vs[i];
            const double mu = rho * vs * vs, K = rho * (vp * vp - 4.0 / 3.0 * vs * vs);
            const double s11 = a.s[0][p], s22 = a.s[1][p], s33 = a.s[2][p];
            const double s12 = a.s[3][p], s13 = a.s[4][p], s23 = a.s[5][p];
            const double tr = s11 + s22 + s33, m = tr / 3.0;
            const double dev = (s11 - m) * (s11 - m) + (s22 - m) * (s22 - m) + (s33 - m) * (s33 - m) +
                               2.0 * (s12 * s12 + s13 * s13 + s23 * s23);
            e += tr * tr / (18.0 * K);
            if (mu > 0.0) e += dev / (4.0 * mu);
        }
        acc += e;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)shot * gridDim.x + blockIdx.x] = t;
}

// one block per shot: the block partials in a fixed order, times the cell volume
__global__ void __launch_bounds__(kEnergyThreads) k_energy_final(const double *partial, int nblocks, double cell,
                                                                 double *out)
{
    __shared__ double sh[kEnergyThreads];
    const double *p = partial + (int64_t)blockIdx.x * nblocks;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kEnergyThreads) acc += p[b];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = t * cell;
}

}  // namespace

hipError_t launch_energy(const EnergyArgs &a, int S, double *partial, int nblocks, double cell, double *out,
                         hipStream_t st)
{
    if (nblocks < 1 || S < 1) return hipErrorInvalidValue;
    const int64_t per_block = (a.nodes + nblocks - 1) / nblocks;
    hipLaunchKernelGGL(k_energy_partial, dim3((unsigned)nblocks, (unsigned)S), kEnergyThreads, 0, st, a, per_block,
                       partial);
    hipLaunchKernelGGL(k_energy_final, dim3((unsigned)S), kEnergyThreads, 0, st, partial, nblocks, cell, out);
    return hipGetLastError();
}

}  // namespace loss
