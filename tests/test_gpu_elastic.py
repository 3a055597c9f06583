"""GPU parity of the 3-D elastic velocity-stress stepper (9 fields, 18 directional
derivative passes per step) against the FP64 oracle, through the C ABI.
Paper Sec. 2 (velocity-stress system), Sec. 3.3 (Strang splitting), Sec. 4.3-4.4."""
import math

import numpy as np
import pytest

from gpu_util import announce, interior_rel_l2, rel_l2, require_gpu
from test_gpu_acoustic import _f32, _gpu, _oracle

pytestmark = pytest.mark.gpu


def _small_elastic(N=64, M=32, halo=10, nsteps=40, layered=False):
    from paper_2301_05127_amd import inputs
    g = inputs.grid(3, (N, N, N), (10.0, 10.0, 10.0), (M, M, M), halo)
    shape = (N + 1,) * 3
    dt = 1e-3
    if layered:
        nz = N + 1
        layer = np.minimum((np.arange(nz) * 4) // nz, 3)
        vlay = np.array([1800.0, 2867.0, 3933.0, 5000.0])[layer]
        pert = inputs.gaussian_random_field(shape, 10.0, 60.0, 5127, -1.0, 1.0)
        vp = vlay[:, None, None] * (1.0 + 0.05 * pert)
        vs = vp / math.sqrt(3.0)
        rho = 310.0 * vp ** 0.25
        dt = 0.8e-3
    else:
        vp = np.full(shape, 3000.0)
        vs = np.full(shape, 1730.0)
        rho = np.full(shape, 2200.0)
    c = (N * 5.0, N * 5.0, N * 5.0)
    rec = np.array([[N // 2, N // 2, k] for k in range(8, N - 7, 4)], np.int32)
    wav = lambda kind: inputs.ricker(25.0, 0.04, dt, nsteps + 1, 0.5 if kind < 2 else 0.0)
    shots = [{"sources": [{"kind": 1, "pos": c, "spread": 20.0, "wavelet": wav(1)}], "receivers": rec,
              "rec_comp": 2},
             {"sources": [{"kind": 4, "pos": c, "spread": 20.0, "wavelet": wav(4)}], "receivers": rec,
              "rec_comp": 2}]
    return dict(name="elastic-small", grid=g, physics=1, dt=dt, nsteps=nsteps, vp=vp, vs=vs, rho=rho,
                shots=shots)


@pytest.mark.parametrize("layered", [False, True])
def test_elastic_two_shots(orc, layered):
    """Explosive and vertical-force shots in one batch; all 9 fields and v3 traces."""
    require_gpu()
    w = _f32(_small_elastic(layered=layered))
    announce("elastic 65^3 2 shots 40 steps layered=%s" % layered)
    sim = _gpu(w)
    for s in range(2):
        rf, rt = _oracle(orc, w, s)
        errs = [rel_l2(sim.get_field(f, shot=s), rf[f]) for f in range(9)]
        et = rel_l2(sim.get_traces(s), rt)
        print("shot %d rel-L2 per field %s traces %.2e" % (s, " ".join("%.2e" % e for e in errs), et))
        for f, e in enumerate(errs):
            assert e < 1e-5, (s, f, e)
        assert et < 1e-5, s
    sim.close()


def test_elastic_longer_interior(orc):
    """120 steps: interior parity (natural-end corners excluded, see the acoustic test)."""
    require_gpu()
    w = _f32(_small_elastic(nsteps=120))
    announce("elastic 120 steps interior")
    sim = _gpu(w, nshots=1)
    rf, rt = _oracle(orc, w, 0)
    errs = [interior_rel_l2(sim.get_field(f), rf[f], 12) for f in range(9)]
    print("interior rel-L2 per field", " ".join("%.2e" % e for e in errs))
    for f, e in enumerate(errs):
        assert e < 1e-5, (f, e)
    sim.close()


def test_elastic_periodic_plane_wave(orc):
    """Periodic travelling P and S waves along x over 400 steps: FP32 vs FP64 within 1e-5.

    Travelling waves keep the velocity and the stress at constant amplitude; a
    standing wave sampled near a temporal zero of one field would magnify the
    FP32 phase drift relative to that field's momentary size."""
    require_gpu()
    from paper_2301_05127_amd import inputs, loss
    N, M, halo = 32, 16, 10
    g = inputs.grid(3, (N, N, N), (10.0, 10.0, 10.0), (M, M, M), halo, end_mode=2)
    shape = (N + 1,) * 3
    j = np.arange(N + 1)
    ph = 2 * math.pi * 2 / N * np.broadcast_to(j[None, None, :], shape)
    fin = np.zeros((9,) + shape)
    rho0, vp0, vs0 = 2200.0, 3000.0, 1730.0
    lam0 = rho0 * (vp0 ** 2 - 2 * vs0 ** 2)
    fin[0] = np.cos(ph)                               # P wave travelling along +x
    fin[3] = -rho0 * vp0 * fin[0]
    fin[4] = fin[5] = lam0 / (rho0 * vp0 ** 2) * fin[3]
    fin[1] = 0.3 * np.sin(ph)                         # S wave polarised along y
    fin[6] = -rho0 * vs0 * fin[1]
    vp = np.full(shape, vp0); vs = np.full(shape, vs0); rho = np.full(shape, rho0)
    announce("elastic periodic 400 steps")
    sim = loss.Simulation(g, 1, 1e-3, nshots=1)
    sim.set_media(vp, rho, vs)
    for f in range(9):
        sim.set_field(f, fin[f].astype(np.float32))
    sim.step(400)
    rf, _ = orc.run(g, 1, 1e-3, 400, vp, rho, vs=vs, fields_in=fin.astype(np.float32).astype(np.float64))
    for f in (0, 1, 3, 4, 5, 6):
        assert rel_l2(sim.get_field(f), rf[f]) < 1e-5, f
    sim.close()


def _pulse_fields(shape, h_nodes):
    """Smooth initial state so that a few steps move every node and every field at first
    order: an explosive stress pulse and off-centre pulses of v1, v2, v3 (Gaussians of
    width h_nodes), as float32."""
    c = [0.45 * (n - 1) for n in shape]
    g = lambda n, c0: np.exp(-(np.arange(n) - c0) ** 2 / (2 * h_nodes ** 2))

    def blob(dz, dy, dx):
        return (g(shape[0], c[0] + dz)[:, None, None] * g(shape[1], c[1] + dy)[None, :, None]
                * g(shape[2], c[2] + dx)[None, None, :]).astype(np.float32)

    fin = np.zeros((9,) + shape, np.float32)
    fin[3] = 1e6 * blob(0, 0, 0)
    fin[4] = fin[5] = fin[3]
    fin[0] = blob(-7, 0, 10)
    fin[1] = 0.8 * blob(5, 9, -8)
    fin[2] = 0.6 * blob(8, -11, 6)
    return fin


@pytest.mark.parametrize("name,nsteps,shape", [
    ("cfg3", 4, (4, 3208, 3208)),
    pytest.param("cfg4", 2, (4, 3208, 3208), marks=pytest.mark.timeout(400)),   # inputs + oracle ~1 min
])
def test_full_size_few_steps(orc, name, nsteps, shape):
    """257^3 (4^3 patches of 64, halo 10, two shots) and 513^3 (8^3 patches of 64, halo 12,
    layered medium): a few steps at full size in the launch shape the benchmark picks,
    every field against the FP64 oracle."""
    require_gpu()
    from paper_2301_05127_amd import inputs, loss
    w = _f32(inputs.config(name, nsteps=nsteps))
    S = len(w["shots"])
    announce("%s full size %d steps, %d shot(s), shape %s" % (name, nsteps, S, shape))
    sim = loss.Simulation(w["grid"], 1, w["dt"], nshots=S, trace_len=nsteps)
    sim.setup_workload(w)
    sim.set_shape(shape)
    fshape = sim.shape
    fin = _pulse_fields(fshape, 12.0)
    for s in range(S):
        for f in range(9):
            sim.set_field(f, fin[f], shot=s)
    sim.step(nsteps)
    for s in range(S):
        sh = w["shots"][s]
        rf, rt = orc.run(w["grid"], 1, w["dt"], nsteps, w["vp"], w["rho"], vs=w["vs"], sources=sh["sources"],
                         receivers=sh["receivers"], rec_comp=sh.get("rec_comp", 0),
                         fields_in=fin.astype(np.float64))
        for f in range(9):
            e = rel_l2(sim.get_field(f, shot=s), rf[f])
            assert e < 1e-5, (s, f, e)
        assert rel_l2(sim.get_traces(s), rt) < 1e-5, s
        del rf
    sim.close()
