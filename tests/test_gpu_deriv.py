"""GPU parity of the hot-path derivative (PMBC slopes, patch solve, D1/D2) against
the FP64 oracle, through the C ABI (loss_deriv).  Paper Sec. 3.1-3.2."""
import numpy as np
import pytest

from gpu_util import announce, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

# (ndim, n, M, halo, end_mode): several tiles, ragged tails, every end mode
CASES = [
    (2, (128, 0, 128), (64, 64, 64), 8, 0),
    (2, (100, 0, 77), (32, 16, 16), 6, 0),       # remainders 4 and 13
    (2, (96, 0, 96), (24, 24, 24), 8, 1),        # paper end stencil
    (2, (96, 0, 64), (32, 16, 16), 7, 2),        # periodic
    (2, (2048, 0, 130), (256, 256, 64), 12, 0),  # config-2 patch length along x
    (2, (130, 0, 600), (64, 64, 256), 12, 0),    # 256-long patches along z, 16 waves
    (3, (40, 36, 33), (16, 12, 8), 5, 0),
    (3, (64, 64, 64), (64, 32, 16), 10, 2),
    (2, (50, 0, 40), (50, 50, 40), 4, 0),        # one patch per axis (global spline)
    (2, (37, 0, 21), (3, 3, 3), 2, 0),           # very short patches
    (2, (96, 0, 80), (4, 4, 4), 12, 0),          # halo 3 patches wide
    (3, (48, 40, 44), (8, 8, 8), 20, 0),         # the halo 20 of the decay pin, 2.5 patches wide
    (2, (96, 0, 96), (8, 8, 8), 20, 2),          # periodic, halo wider than the patches
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("order", [1, 2])
def test_deriv_matches_oracle(orc, case, order):
    require_gpu()
    from paper_2301_05127_amd import inputs, loss
    ndim, n, M, halo, mode = case
    g = inputs.grid(ndim, n, (10.0, 7.0, 5.0), M, halo, mode)
    announce("deriv %s order %d" % (case, order))
    phys = loss.ACOUSTIC if ndim == 2 else loss.ELASTIC
    sim = loss.Simulation(g, phys, 1e-4, nshots=2)
    shape = sim.shape
    u = inputs.random_field((2,) + shape, seed=sum(n) + order)
    axes = [0, 2] if ndim == 2 else [0, 1, 2]
    for axis in axes:
        got = sim.deriv(axis, order, u.astype(np.float32))
        for b in range(2):
            ref = orc.field_deriv(g, axis, order, u[b].astype(np.float32).astype(np.float64))
            err = rel_l2(got[b], ref)
            mx = np.abs(got[b] - ref).max() / np.abs(ref).max()
            # FP32 solve of a diagonally dominant system, condition <= 3
            tol = 2e-6 if order == 1 else 5e-6
            assert err < tol and mx < 10 * tol, (axis, b, err, mx)
    sim.close()


@pytest.mark.parametrize("case", [c for c in CASES if c[0] == 3])
def test_transposed_deriv_3d_matches_dense(orc, case):
    """D^T along x, y and z of a 3-D batch (the adjoint's solve, junction rows and
    gather on every axis) against the dense FP64 line operator of the oracle."""
    require_gpu()
    from paper_2301_05127_amd import inputs, loss
    ndim, n, M, halo, mode = case
    hs = (10.0, 7.0, 5.0)
    g = inputs.grid(ndim, n, hs, M, halo, mode)
    announce("transposed deriv 3-D %s" % (case,))
    sim = loss.Simulation(g, loss.ELASTIC, 1e-4, nshots=2)
    w = inputs.random_field((2,) + sim.shape, seed=5).astype(np.float32)
    for axis in range(3):
        got = sim.deriv(axis, -1, w)
        D = orc.line_deriv_matrix(n[axis], hs[axis], M[axis], halo, mode)
        for b in range(2):
            w64 = w[b].astype(np.float64)
            ref = np.moveaxis(np.tensordot(np.moveaxis(w64, 2 - axis, -1), D, axes=([-1], [0])), -1, 2 - axis)
            assert rel_l2(got[b], ref) < 2e-6, (axis, b)
    sim.close()
