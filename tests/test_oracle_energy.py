"""Pins of the oracle's wavefield energy (velocity-stress system, Sec. 2) against closed
forms of isotropic elasticity on uniform states: kinetic 1/2 rho v^2; hydrostatic stress
-p I: p^2 / (2 K), K = lambda + 2 mu / 3; pure shear sigma12 = tau: tau^2 / (2 mu); uniaxial
sigma11 = s: s^2 / (2 E), E = mu (3 lambda + 2 mu) / (lambda + mu); acoustic sigma^2 / (2 K).
Each pin fails for a plausible slip in the Voigt solve (a shear factor of 2, lambda and mu
swapped, a missing 1/2)."""
import numpy as np
import pytest

from paper_2301_05127_amd import inputs

pytestmark = pytest.mark.parametrize("n", [(6, 5, 4)])


def _setup(n):
    g = inputs.grid(3, n, (10.0, 12.0, 9.0), (3, 3, 3), 2)
    shape = inputs.field_shape(g)
    nodes = np.prod(shape)
    vol = 10.0 * 12.0 * 9.0
    rho, vp, vs = 2100.0, 3200.0, 1700.0
    mu = rho * vs ** 2
    lam = rho * vp ** 2 - 2 * mu
    full = lambda v: np.full(shape, v)
    return g, shape, nodes * vol, full(vp), full(rho), full(vs), lam, mu, rho


def test_kinetic(orc, n):
    g, shape, V, vp, rho, vs, lam, mu, r = _setup(n)
    f = np.zeros((9,) + shape)
    f[0], f[1], f[2] = 0.3, -0.4, 1.2
    e = orc.energy(g, 1, f, vp, rho, vs)
    assert abs(e - 0.5 * r * (0.09 + 0.16 + 1.44) * V) <= 1e-12 * e


def test_hydrostatic(orc, n):
    g, shape, V, vp, rho, vs, lam, mu, r = _setup(n)
    f = np.zeros((9,) + shape)
    p = 3.0e6
    f[3] = f[4] = f[5] = -p
    K = lam + 2 * mu / 3
    e = orc.energy(g, 1, f, vp, rho, vs)
    assert abs(e - p ** 2 / (2 * K) * V) <= 1e-12 * e


@pytest.mark.parametrize("comp", [6, 7, 8])
def test_pure_shear(orc, n, comp):
    g, shape, V, vp, rho, vs, lam, mu, r = _setup(n)
    f = np.zeros((9,) + shape)
    tau = 2.5e6
    f[comp] = tau
    e = orc.energy(g, 1, f, vp, rho, vs)
    assert abs(e - tau ** 2 / (2 * mu) * V) <= 1e-12 * e


@pytest.mark.parametrize("comp", [3, 4, 5])
def test_uniaxial(orc, n, comp):
    g, shape, V, vp, rho, vs, lam, mu, r = _setup(n)
    f = np.zeros((9,) + shape)
    s = 4.0e6
    f[comp] = s
    E = mu * (3 * lam + 2 * mu) / (lam + mu)
    e = orc.energy(g, 1, f, vp, rho, vs)
    assert abs(e - s ** 2 / (2 * E) * V) <= 1e-12 * e


def test_acoustic(orc, n):
    g = inputs.grid(2, (7, 0, 5), (10.0, 10.0, 8.0), (3, 3, 3), 2)
    shape = inputs.field_shape(g)
    V = np.prod(shape) * 10.0 * 8.0
    f = np.zeros((3,) + shape)
    f[0], f[1], f[2] = 2.0e6, 0.5, -0.25
    rho, c = 1800.0, 2500.0
    e = orc.energy(g, 0, f, np.full(shape, c), np.full(shape, rho))
    ref = (0.5 * rho * (0.25 + 0.0625) + 0.5 * 4.0e12 / (rho * c * c)) * V
    assert abs(e - ref) <= 1e-12 * ref
