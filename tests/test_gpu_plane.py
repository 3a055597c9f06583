"""GPU parity of the elastic plane schedule (per sub-flow: z derivatives stored, then one
pass solving the x and y lines of each patch tile of a plane from LDS) against the FP64
oracle and against the line-pass schedule, through the C ABI.
Paper Sec. 2 (velocity-stress system), Sec. 3.2 (patches, PMBC), Sec. 3.3 (Strang)."""
import math

import numpy as np
import pytest

from gpu_util import announce, rel_l2, require_gpu
from test_gpu_acoustic import _f32, _oracle

pytestmark = pytest.mark.gpu


def _elastic(n, M, halo, end_mode=0, nsteps=50, layered=True, h=10.0):
    from paper_2301_05127_amd import inputs
    g = inputs.grid(3, n, (h, h, h), M, halo, end_mode=end_mode)
    shape = (n[2] + 1, n[1] + 1, n[0] + 1)
    dt = 0.8e-3
    if layered:
        nz = n[2] + 1
        layer = np.minimum((np.arange(nz) * 4) // nz, 3)
        vlay = np.array([1800.0, 2867.0, 3933.0, 5000.0])[layer]
        pert = inputs.gaussian_random_field(shape, h, 60.0, 5127, -1.0, 1.0)
        vp = vlay[:, None, None] * (1.0 + 0.05 * pert)
        vs = vp / math.sqrt(3.0)
        rho = 310.0 * vp ** 0.25
    else:
        vp = np.full(shape, 3000.0)
        vs = np.full(shape, 1730.0)
        rho = np.full(shape, 2200.0)
    c = tuple(0.5 * n[a] * h + 3.0 for a in range(3))   # off-node centre
    # receivers on a vertical line a few nodes off the source, wavelet peak at 20 ms: the
    # traces carry the direct P and S arrivals within the run
    rec = np.array([[n[0] // 2 + 2, n[1] // 2 - 3, k] for k in range(2, n[2] - 1, 3)], np.int32)
    wav = lambda kind: inputs.ricker(30.0, 0.02, dt, nsteps + 1, 0.5 if kind < 2 else 0.0)
    shots = [{"sources": [{"kind": 1, "pos": c, "spread": 20.0, "wavelet": wav(1)},
                          {"kind": 2, "pos": (c[0] - 60.0, c[1] + 40.0, c[2]), "spread": 15.0, "wavelet": wav(2)}],
              "receivers": rec, "rec_comp": 2},
             {"sources": [{"kind": 4, "pos": c, "spread": 20.0, "wavelet": wav(4)},
                          {"kind": 3, "pos": (c[0] + 50.0, c[1], c[2] - 30.0), "spread": 0.0, "wavelet": wav(3)}],
              "receivers": rec, "rec_comp": 7}]
    return dict(name="elastic-plane", grid=g, physics=1, dt=dt, nsteps=nsteps, vp=vp, vs=vs, rho=rho,
                shots=shots)


def _run(w, schedule, flags=0):
    from paper_2301_05127_amd import loss
    sim = loss.Simulation(w["grid"], 1, w["dt"], nshots=2, trace_len=w["nsteps"], flags=flags)
    sim.setup_workload(w)
    sim.set_shape([None, None, None, schedule])
    sim.step(w["nsteps"])
    out = [[sim.get_field(f, shot=s) for f in range(9)] for s in range(2)]
    tr = [sim.get_traces(s) for s in range(2)]
    sim.close()
    return out, tr


GEOMS = [
    # (intervals, patch lengths, halo, end mode, steps)
    ((64, 64, 64), (32, 32, 32), 10, 0, 50),
    ((50, 50, 50), (16, 16, 16), 6, 0, 50),          # remainder patch of 2 intervals
    ((48, 40, 56), (16, 32, 24), 8, 0, 50),          # a different patch length per axis
    ((48, 48, 48), (24, 24, 24), 10, 2, 50),         # periodic
    ((48, 48, 48), (24, 24, 24), 8, 1, 50),          # the paper's end stencil
    # short patches: 30 steps, before the P wave reaches the natural ends (at 50 steps
    # both schedules are 1-3e-5 from the FP64 oracle there, FP32 noise growing at the
    # natural-end rows as in the acoustic runs; 5e-7 on periodic grids)
    ((40, 40, 40), (8, 8, 8), 6, 0, 30),
    ((130, 70, 40), (64, 64, 20), 12, 0, 50),        # full 64-interval tiles with a remainder
]


@pytest.mark.parametrize("geom", GEOMS, ids=[str(g[0]) + "M" + str(g[1][0]) + "e" + str(g[3]) for g in GEOMS])
def test_plane_schedule_matches_oracle_and_line_passes(orc, geom):
    require_gpu()
    n, M, halo, end, nsteps = geom
    w = _f32(_elastic(n, M, halo, end, nsteps=nsteps))
    announce("plane schedule n=%s M=%s halo=%d end=%d" % (n, M, halo, end))
    plane, tp = _run(w, 0)
    line, tl = _run(w, 1)
    eo = np.zeros((2, 10))
    el = np.zeros((2, 10))
    for s in range(2):
        rf, rt = _oracle(orc, w, s)
        for f in range(9):
            eo[s, f] = rel_l2(plane[s][f], rf[f])
            el[s, f] = max(rel_l2(line[s][f], rf[f]), 0.0)
        eo[s, 9] = rel_l2(tp[s], rt)
        el[s, 9] = rel_l2(tl[s], rt)
    np.set_printoptions(precision=2)
    print("rel-L2 vs the FP64 oracle per field (9 fields, traces), plane then line passes:\n", eo, "\n", el)
    # the paper's end stencil (end mode 1) makes the operator strongly non-normal: its
    # transient growth amplifies FP32 differences (1.4e-5 here); the other closures stay
    # below 7e-6
    tol = 2e-5 if end == 1 else 1e-5
    assert eo.max() < tol, eo
    assert el.max() < tol, el


def test_plane_graph_and_eager_bitwise_equal():
    require_gpu()
    from paper_2301_05127_amd import loss
    w = _f32(_elastic((64, 64, 64), (32, 32, 32), 10, nsteps=37))
    announce("plane schedule graph vs eager")
    a, ta = _run(w, 0)
    b, tb = _run(w, 0, flags=loss.FLAG_NO_GRAPH)
    for s in range(2):
        for f in range(9):
            assert np.array_equal(a[s][f], b[s][f]), (s, f)
        assert np.array_equal(ta[s], tb[s])


def test_autotune_reports_elastic_schedule():
    require_gpu()
    from paper_2301_05127_amd import loss
    w = _f32(_elastic((64, 64, 64), (32, 32, 32), 10, nsteps=10))
    announce("autotune elastic schedule")
    sim = loss.Simulation(w["grid"], 1, w["dt"], nshots=2, trace_len=10)
    sim.setup_workload(w)
    choice = sim.autotune(2)
    assert len(choice) == 6 and choice[3] in (0, 1), choice
    assert choice[4] in (0, 6408, 3208) and choice[5] == 0, choice
    sim.step(10)
    sim.sync()
    assert sim.current_step == 10
    sim.close()
