"""Pins of the oracle's elastic adjoint with the absorbing layer (Sec. 3.3 on every axis):
the vanishing-layer limit against the plain elastic adjoint (itself pinned by finite
differences), and directional derivatives of J along smooth perturbations of lambda, mu
and b against central finite differences of the oracle's layer forward run (which
evaluates each sub-flow by its closed form, not through the linear forms the adjoint
transposes), for velocity and stress receivers, with stress and force sources."""
import numpy as np
import pytest

from paper_2301_05127_amd import inputs


def _setup():
    N, M, n, h, dt, nsteps = 12, 6, 4, 10.0, 1e-3, 30
    g = inputs.grid(3, (N, N, N), (h, h, h), (M, M, M), n)
    shape = (N + 1,) * 3
    vp = inputs.gaussian_random_field(shape, h, 40.0, 31, 2800.0, 3300.0)
    vs = vp / np.sqrt(3.0) * (1.0 + 0.05 * inputs.gaussian_random_field(shape, h, 40.0, 32, -1.0, 1.0))
    rho = inputs.gaussian_random_field(shape, h, 40.0, 33, 2000.0, 2400.0)
    srcs = [{"kind": 1, "pos": (50.0, 60.0, 70.0), "spread": 15.0,
             "wavelet": inputs.ricker(60.0, 0.02, dt, nsteps + 1, 0.5)},
            {"kind": 3, "pos": (75.0, 50.0, 45.0), "spread": 15.0,
             "wavelet": inputs.ricker(60.0, 0.02, dt, nsteps + 1, 0.0)}]
    rec = np.array([[ix, 9, 10] for ix in range(1, N, 3)] + [[3, iy, 2] for iy in range(2, N, 4)],
                   dtype=np.int32)
    return g, dt, nsteps, vp, vs, rho, srcs, rec


# a 4-node layer the waves reach within the run
PML = dict(width=4, R=1e-4, kmax=1.0, f0=60.0)


@pytest.mark.parametrize("rec_comp", [2, 6])     # v3, sigma12
def test_vanishing_layer_is_the_plain_adjoint(orc, rec_comp):
    g, dt, nsteps, vp, vs, rho, srcs, rec = _setup()
    pml = dict(PML, R=1.0 - 1e-12, cmax=float(vp.max()))
    d = orc.run(g, 1, dt, nsteps, vp, rho, vs=vs, sources=srcs, receivers=rec, rec_comp=rec_comp)[1]
    gp = orc.elastic_adjoint_pml(g, pml, dt, nsteps, vp, vs, rho, srcs, rec, rec_comp, d, with_b=True)
    gn = orc.elastic_adjoint(g, dt, nsteps, vp, vs, rho, srcs, rec, rec_comp, d, with_b=True)
    for a, b in zip(gp, gn):
        assert np.abs(b).max() > 0
        assert orc.rel_l2(a, b) < 1e-9, orc.rel_l2(a, b)


@pytest.mark.parametrize("rec_comp,params", [(2, ("lambda", "b")), (6, ("mu",))])
def test_layer_adjoint_matches_fd(orc, rec_comp, params):
    g, dt, nsteps, vp, vs, rho, srcs, rec = _setup()
    shape = vp.shape
    pml = dict(PML, cmax=float(vp.max()))
    mu = rho * vs ** 2
    lam = rho * vp ** 2 - 2 * mu
    b = 1.0 / rho

    def traces(lm, mm, bb):
        r = 1.0 / bb
        return orc.run_pml_elastic(g, pml, dt, nsteps, np.sqrt((lm + 2 * mm) / r), np.sqrt(mm / r), r,
                                   sources=srcs, receivers=rec, rec_comp=rec_comp)[1]

    obs = orc.run_pml_elastic(g, pml, dt, nsteps, vp * 1.01, vs * 0.99, rho, sources=srcs, receivers=rec,
                              rec_comp=rec_comp)[1]
    J = lambda lm, mm, bb: 0.5 * np.sum((traces(lm, mm, bb) - obs) ** 2)
    d0 = traces(lam, mu, b)
    gl, gm, gb = orc.elastic_adjoint_pml(g, pml, dt, nsteps, vp, vs, rho, srcs, rec, rec_comp, d0 - obs,
                                         with_b=True)
    assert np.abs(gl).max() > 0 and np.abs(gm).max() > 0 and np.abs(gb).max() > 0
    # the layer carries part of the gradient: the plain adjoint of the same residual differs
    gn = orc.elastic_adjoint(g, dt, nsteps, vp, vs, rho, srcs, rec, rec_comp, d0 - obs)
    assert orc.rel_l2(gn[0], gl) > 1e-3
    for which, grad, seed, scale in (("lambda", gl, 4, 1e8), ("mu", gm, 5, 1e8), ("b", gb, 6, 1e-5)):
        if which not in params:
            continue
        dp = inputs.gaussian_random_field(shape, 10.0, 50.0, seed, -1.0, 1.0) * scale
        eps = 1e-3
        if which == "lambda":
            fd = (J(lam + eps * dp, mu, b) - J(lam - eps * dp, mu, b)) / (2 * eps)
        elif which == "mu":
            fd = (J(lam, mu + eps * dp, b) - J(lam, mu - eps * dp, b)) / (2 * eps)
        else:
            fd = (J(lam, mu, b + eps * dp) - J(lam, mu, b - eps * dp)) / (2 * eps)
        an = float(np.sum(grad * dp))
        assert abs(fd - an) <= 1e-7 * abs(an), (which, fd, an)
