"""The multi-line x kernel (a wave solves the same four 16-lane patches on several
consecutive lines; the patch's row factors, end rows and PMBC tap coefficients are read
once per wave) against the x kernel that gives each lane group one unit.  Both take the
same unmasked solve of whole patches (Sec. 3.1-3.2), so fields and traces agree bit for
bit; the cases cover sources, receivers, the absorbing layer (Sec. 3.3), two shots whose
lines share a wave, a last wave with fewer lines, both derivative orders and the FP64
oracle."""
import numpy as np
import pytest

from gpu_util import announce, rel_l2, require_gpu
from test_gpu_acoustic import _f32

pytestmark = pytest.mark.gpu

# lines per shot 33 * 17 = 561 (two shots: 1122 lines; 1122 = 4 * 280 + 2 = 8 * 140 + 2)
GRID3 = dict(n=(256, 32, 16), M=(64, 16, 16), halo=8)


def _elastic(nsteps):
    from paper_2301_05127_amd import inputs
    g = inputs.grid(3, GRID3["n"], (10.0, 10.0, 10.0), GRID3["M"], GRID3["halo"])
    shape = inputs.field_shape(g)
    vp = 3000.0 * (1.0 + 0.05 * inputs.gaussian_random_field(shape, 10.0, 60.0, 17, -1.0, 1.0))
    vs = vp / np.sqrt(3.0)
    rho = 310.0 * vp ** 0.25
    dt = 0.8e-3
    # receivers of v1 off the sources' x columns (on a source's column v1 vanishes by symmetry)
    rec = np.array([[ix, 16, 8] for ix in range(4, 253, 12)], np.int32)
    wav = lambda: inputs.ricker(25.0, 0.04, dt, nsteps + 1, 0.5)
    shots = [{"sources": [{"kind": 1, "pos": (1280.0, 160.0, 80.0), "spread": 20.0, "wavelet": wav()}],
              "receivers": rec, "rec_comp": 0},
             {"sources": [{"kind": 1, "pos": (600.0, 150.0, 90.0), "spread": 20.0, "wavelet": wav()}],
              "receivers": rec, "rec_comp": 0}]
    return _f32(dict(grid=g, physics=1, dt=dt, nsteps=nsteps, vp=vp, vs=vs, rho=rho, shots=shots))


def _run_elastic(w, xshape, pml):
    from paper_2301_05127_amd import loss
    sim = loss.Simulation(w["grid"], 1, w["dt"], nshots=2, trace_len=w["nsteps"])
    sim.setup_workload(w)
    if pml:
        sim.set_pml(6, 1e-6, 1.0, 25.0)
    sim.set_shape([xshape, None, None])
    sim.step(w["nsteps"])
    out = [[sim.get_field(f, shot=s) for f in range(9)] for s in range(2)]
    tr = [sim.get_traces(s) for s in range(2)]
    sim.close()
    return out, tr


@pytest.mark.parametrize("pml", [False, True])
def test_multiline_x_elastic_bitwise(pml):
    require_gpu()
    w = _elastic(30)
    announce("multi-line x kernel, elastic 257x33x17, 2 shots, 30 steps, layer=%s" % pml)
    ref_f, ref_t = _run_elastic(w, 104, pml)
    for xs in (4, 204, 404, 804, 1604):
        f, t = _run_elastic(w, xs, pml)
        for s in range(2):
            for c in range(9):
                assert np.array_equal(f[s][c], ref_f[s][c]), (xs, s, c)
            assert np.array_equal(t[s], ref_t[s]), (xs, s)


def test_multiline_x_elastic_matches_oracle(orc):
    require_gpu()
    w = _elastic(30)
    announce("multi-line x kernel, elastic 257x33x17 against the oracle")
    f, t = _run_elastic(w, 404, False)
    for s in range(2):
        sh = w["shots"][s]
        rf, rt = orc.run(w["grid"], 1, w["dt"], w["nsteps"], w["vp"], w["rho"], vs=w["vs"],
                         sources=sh["sources"], receivers=sh["receivers"], rec_comp=sh["rec_comp"])
        errs = [rel_l2(f[s][c], rf[c]) for c in range(9)]
        et = rel_l2(t[s], rt)
        print("shot %d rel-L2 %s traces %.2e (trace norm %.2e)" % (s, " ".join("%.1e" % e for e in errs), et,
                                                                   np.linalg.norm(rt)))
        assert max(errs) < 1e-5 and et < 1e-5, (s, errs, et)


def test_multiline_x_acoustic_and_deriv_bitwise():
    """Unfused acoustic steps (the x passes in the multi-line kernel) and loss_deriv along
    x of both orders, against the one-unit kernel."""
    require_gpu()
    from paper_2301_05127_amd import inputs, loss
    g = inputs.grid(2, (256, 0, 96), (10.0, 10.0, 10.0), (64, 64, 32), 8)
    shape = inputs.field_shape(g)
    vp = 2000.0 * (1.0 + 0.05 * inputs.gaussian_random_field(shape, 10.0, 60.0, 3, -1.0, 1.0))
    rho = np.full(shape, 1000.0)
    dt = 1e-3
    rec = np.array([[ix, 0, 40] for ix in range(8, 249, 8)], np.int32)
    shots = [{"sources": [{"kind": 0, "pos": (1000.0 + 300.0 * s, 0.0, 500.0), "spread": 15.0,
                           "wavelet": inputs.ricker(20.0, 0.05, dt, 81, 0.5)}], "receivers": rec, "rec_comp": 0}
             for s in range(3)]
    w = _f32(dict(grid=g, physics=0, dt=dt, nsteps=80, vp=vp, vs=None, rho=rho, shots=shots))
    rng = np.random.default_rng(11)
    data = rng.standard_normal((5,) + shape).astype(np.float32)
    announce("multi-line x kernel, acoustic 257x97, 3 shots unfused, and loss_deriv")
    res = []
    for xs in (104, 4, 404, 1604):
        sim = loss.Simulation(g, 0, dt, nshots=3, trace_len=80, flags=loss.FLAG_NO_FUSE_X)
        sim.setup_workload(w)
        sim.set_shape([xs, None, None])
        sim.step(80)
        fields = [sim.get_field(f, shot=s) for s in range(3) for f in range(3)]
        traces = [sim.get_traces(s) for s in range(3)]
        ders = [sim.deriv(0, order, data) for order in (1, 2)]
        res.append((fields, traces, ders))
        sim.close()
    for r in res[1:]:
        for a, b in zip(r[0] + r[1] + r[2], res[0][0] + res[0][1] + res[0][2]):
            assert np.array_equal(a, b)


def test_shape_encoding_round_trip():
    """x shapes 100 * lines per wave + nodes per lane (lines 0 automatic, 1, 2, 4, 8, 16),
    y/z shapes 100 * columns per wave + nodes per lane: accepted values are reported back
    by loss_autotune_choice, the others refused with LOSS_EINVAL."""
    require_gpu()
    import ctypes
    from paper_2301_05127_amd import loss
    w = _elastic(4)
    announce("launch shape encoding")
    sim = loss.Simulation(w["grid"], 1, w["dt"], nshots=1)
    sim.set_media(w["vp"], w["rho"], w["vs"])

    def choice(axis):
        v = ctypes.c_int32()
        assert loss.lib().loss_autotune_choice(sim._h, axis, ctypes.byref(v)) == 0
        return v.value

    for xs in (4, 8, 16, 104, 204, 404, 804, 1604, 408, 1616):
        sim.set_shape([xs, None, None])
        assert choice(0) == xs, xs
    for ys in (6408, 3216, 1608, 808):
        sim.set_shape([None, ys, ys])
        assert choice(1) == ys and choice(2) == ys, ys
    einval = -1   # LOSS_EINVAL
    for bad in (2, 5, 304, 1704, 3204, 10004):
        assert loss.lib().loss_set_shape(sim._h, 0, bad) == einval, bad
    for bad in (6404, 6432, 4808, 16408):
        assert loss.lib().loss_set_shape(sim._h, 1, bad) == einval, bad
    for st in (6408, 3208, 1616, 0):
        sim.set_shape([None, None, None, None, st, st])
        assert choice(4) == st and choice(5) == st, st
    for bad in (6404, 4808, 16408):
        assert loss.lib().loss_set_shape(sim._h, 4, bad) == einval, bad
    sim.set_shape([None, None, None, None, 6408, 3208])
    sim.step(2)   # every accepted shape launches; the last ones set are in use
    sim.close()


def test_store_pass_shapes_match_oracle(orc):
    """The y and z store passes in their own launch shape (64 columns while the other
    passes of the axis take 32, and the reverse) against the FP64 oracle."""
    require_gpu()
    from paper_2301_05127_amd import loss
    w = _elastic(30)
    announce("store-pass shapes, elastic 257x33x17 against the oracle")
    refs = []
    for s in range(2):
        sh = w["shots"][s]
        refs.append(orc.run(w["grid"], 1, w["dt"], w["nsteps"], w["vp"], w["rho"], vs=w["vs"],
                            sources=sh["sources"], receivers=sh["receivers"], rec_comp=sh["rec_comp"]))
    for shape in ([404, 3208, 3208, 1, 6408, 6408], [404, 6408, 6408, 1, 3208, 3208]):
        sim = loss.Simulation(w["grid"], 1, w["dt"], nshots=2, trace_len=w["nsteps"])
        sim.setup_workload(w)
        sim.set_shape(shape)
        sim.step(w["nsteps"])
        for s in range(2):
            rf, rt = refs[s]
            errs = [rel_l2(sim.get_field(c, shot=s), rf[c]) for c in range(9)]
            et = rel_l2(sim.get_traces(s), rt)
            assert max(errs) < 1e-5 and et < 1e-5, (shape, s, errs, et)
        sim.close()
