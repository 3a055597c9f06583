"""Pins of the oracle's sources (reading of Sec. 4.3: source term A(x) f(t)).

The paper gives the source as a spatial amplitude A(x) times a wavelet and is silent on
A's shape and on the time level a sample enters the split step.  The readings pinned
here: A is a Gaussian exp(-d^2 / (2 s^2)) over the nodes within 4 s of the source,
normalised to unit integral (sum w h^d = 1); a point source is 1/h^d at the nearest
node; a stress-rate sample n enters step n (stress sub-flow), a force sample k enters
the velocity half steps at t_k.  Each pin is independent of the formula it checks:
the integral and the moments are what the Gaussian's definition fixes, and the
conservation pins follow from the fact that on a periodic grid the spline derivative
of any field sums to zero over the grid (its symbol vanishes at zero wavenumber), so
the sources alone change the grid totals.

The second half of the module plants each plausible mistake in a copy of the oracle's
C source, builds it on the CPU, and checks that a pin fails on it.
"""
import os
import re

import numpy as np
import pytest

from paper_2301_05127_amd import inputs

H = 10.0


def _grid2(n=80, M=40, halo=8, end_mode=0):
    return inputs.grid(2, (n, 0, n), (H, H, H), (M, M, M), halo, end_mode=end_mode)


def _grid3(n=40, M=20, halo=8, end_mode=0):
    return inputs.grid(3, (n, n, n), (H, H, H), (M, M, M), halo, end_mode=end_mode)


# ---- pins (each takes the oracle module, so the mutants below can run them) -------

def pin_unit_integral(orc):
    """sum w h^d = 1 in 2-D and 3-D, for several spreads and off-node positions."""
    worst = 0.0
    for g, pos, hd in ((_grid2(), (403.0, 0.0, 398.0), H ** 2), (_grid3(), (197.0, 205.0, 201.0), H ** 3)):
        for spread in (15.0, 20.0, 30.0):
            w = orc.source_weights(g, pos, spread)
            worst = max(worst, abs(w.sum() * hd - 1.0))
    return worst


def pin_second_moment(orc, spread_h=2.0):
    """Per-axis second moment of A about a node-centred source equals spread^2.

    A Gaussian sampled on a grid with spread >= 2h has the continuous moments up to
    exp(-2 pi^2 (s/h)^2) (Poisson summation); cutting it at 4 spreads changes the
    second moment by about 2 a phi(a) = 1.1e-3 at a = 4 plus endpoint corrections of
    the same order, so the relative deviation is bounded by 2.5e-3.  A width read as
    exp(-d^2/s^2) gives -0.5."""
    g = _grid2()
    s = spread_h * H
    w = orc.source_weights(g, (400.0, 0.0, 400.0), s)
    x = np.arange(81) * H - 400.0
    mx = float((w.sum(axis=0) * x * x).sum() * H * H)
    mz = float((w.sum(axis=1) * x * x).sum() * H * H)
    m1 = float((w.sum(axis=0) * x).sum() * H * H)
    return max(abs(mx / s ** 2 - 1.0), abs(mz / s ** 2 - 1.0)), abs(m1)


def pin_point_source(orc):
    """spread 0: weight 1/h^d at the nearest node and nothing elsewhere."""
    g = _grid3()
    w = orc.source_weights(g, (203.0, 207.0, 196.0), 0.0)
    nz = np.argwhere(w != 0)
    return nz.tolist(), float(w.max() * H ** 3)


def _periodic_acoustic(orc, nsteps, kind, pos=(320.0, 0.0, 300.0)):
    g = _grid2(n=64, M=32, halo=20, end_mode=2)
    dt = 1e-3
    shape = orc.field_shape(g)
    vp = np.full(shape, 2000.0)
    rho = np.full(shape, 1000.0)
    # sampled as the stepper consumes it: stress samples at t_n + dt/2, forces at t_k
    wav = inputs.ricker(15.0, 1.2 / 15.0, dt, nsteps + 2, shift=0.5 if kind == 0 else 0.0)
    f, _ = orc.run(g, 0, dt, nsteps, vp, rho, sources=[dict(kind=kind, pos=pos, spread=20.0, wavelet=wav)])
    return f, wav, dt, rho[0, 0]


def pin_periodic_stress_total(orc, nsteps=40):
    """Periodic acoustic grid, pressure-rate source: the grid total of sigma (node N is
    node 0, counted once) after n steps is dt * sum_{k<n} s_k, to the PMBC truncation
    level of halo 20 ((2 - sqrt 3)^20 ~ 4e-12).  Fixes the normalisation and the sample
    index of stress sources."""
    f, wav, dt, _ = _periodic_acoustic(orc, nsteps, 0)
    tot = float(f[0][:-1, :-1].sum() * H * H)
    want = dt * float(wav[:nsteps].sum())
    return abs(tot - want) / abs(want)


def pin_periodic_force_total(orc, nsteps=40):
    """Periodic acoustic grid, force along x: rho * the grid total of v1 after n steps is
    dt * sum_{k<n} (f_k + f_{k+1}) / 2 (the two velocity half steps of a Strang step
    take the force at t_k and t_{k+1}).  Fixes the force time levels."""
    f, wav, dt, rho = _periodic_acoustic(orc, nsteps, 2)
    tot = float(rho * f[1][:-1, :-1].sum() * H * H)
    want = dt * float(0.5 * (wav[:nsteps] + wav[1:nsteps + 1]).sum())
    return abs(tot - want) / abs(want)


def pin_periodic_explosive_elastic(orc, nsteps=16):
    """Periodic 3-D elastic grid, explosive source: each normal stress totals
    dt * sum_{k<n} s_k over the grid; the shear stresses total zero."""
    g = _grid3(n=48, M=24, halo=20, end_mode=2)
    dt = 1e-3
    shape = orc.field_shape(g)
    vp = np.full(shape, 3000.0)
    vs = np.full(shape, 1730.0)
    rho = np.full(shape, 2200.0)
    wav = inputs.ricker(25.0, 1.2 / 25.0, dt, nsteps + 2, shift=0.5)
    f, _ = orc.run(g, 1, dt, nsteps, vp, rho, vs=vs,
                   sources=[dict(kind=1, pos=(240.0, 230.0, 250.0), spread=20.0, wavelet=wav)])
    want = dt * float(wav[:nsteps].sum())
    tot = [float(f[k][:-1, :-1, :-1].sum() * H ** 3) for k in range(3, 9)]
    return max(abs(t - want) / abs(want) for t in tot[:3]), max(abs(t) for t in tot[3:]) / abs(want)


# ---- the pins on the oracle ---------------------------------------------------------

def test_source_unit_integral(orc):
    assert pin_unit_integral(orc) < 1e-14


def test_source_second_moment(orc):
    for sh in (2.0, 3.0):
        dev, m1 = pin_second_moment(orc, sh)
        assert dev < 2.5e-3, (sh, dev)
        assert m1 < 1e-12


def test_point_source(orc):
    nodes, wmax = pin_point_source(orc)
    assert nodes == [[20, 21, 20]]   # (z, y, x) of the nearest node to (203, 207, 196) m
    assert abs(wmax - 1.0) < 1e-14


def test_periodic_stress_source_total(orc):
    assert pin_periodic_stress_total(orc) < 1e-9


def test_periodic_force_total(orc):
    assert pin_periodic_force_total(orc) < 1e-9


def test_periodic_explosive_elastic_total(orc):
    normal, shear = pin_periodic_explosive_elastic(orc)
    assert normal < 1e-9 and shear < 1e-9, (normal, shear)


# ---- planted mistakes: each must make a pin fail ----------------------------------

_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "loss_oracle.c")

MUTANTS = {
    # the 1/h^d of the normalisation dropped
    "drop_hd": (r"\] /= sum \* hd;", "] /= sum;"),
    # the Gaussian width read as exp(-d^2/s^2)
    "width": (r"\(2\.0 \* spread \* spread\)", "(spread * spread)"),
    # the stress-rate sample of step n taken one step late
    "stress_index": (r"double s = sample\(&src\[k\], sn\);", "double s = sample(&src[k], sn + 1);"),
    # both velocity half steps take the force at t_n
    "force_level": (r"long fk = half == 0 \? sn : sn \+ 1;", "long fk = sn;"),
}


@pytest.fixture(scope="module")
def mutant_libs(tmp_path_factory, orc):
    text = open(_SRC).read()
    out = {}
    for name, (pat, rep) in MUTANTS.items():
        new, n = re.subn(pat, rep, text)
        assert n >= 1, "mutation %s found no site" % name
        d = tmp_path_factory.mktemp(name)
        out[name] = orc.build_variant(new, str(d / "liblossoracle_mut.so"))
    return out


def test_mutant_drop_hd_fails_unit_integral(orc, mutant_libs):
    with orc.use_library(mutant_libs["drop_hd"]):
        assert pin_unit_integral(orc) > 1e-3
        assert pin_periodic_stress_total(orc) > 1e-3


def test_mutant_width_fails_second_moment(orc, mutant_libs):
    with orc.use_library(mutant_libs["width"]):
        dev, _ = pin_second_moment(orc, 2.0)
        assert dev > 0.1


def test_mutant_stress_index_fails_conservation(orc, mutant_libs):
    with orc.use_library(mutant_libs["stress_index"]):
        assert pin_periodic_stress_total(orc) > 1e-3
        normal, _ = pin_periodic_explosive_elastic(orc)
        assert normal > 1e-3


def test_mutant_force_level_fails_force_total(orc, mutant_libs):
    with orc.use_library(mutant_libs["force_level"]):
        assert pin_periodic_force_total(orc) > 1e-3
