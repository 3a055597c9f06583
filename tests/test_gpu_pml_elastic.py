"""GPU parity of the elastic absorbing layer (the ADE-PML of Sec. 3.3 applied to every
derivative of the 3-D elastic system, 18 memory variables) against the FP64 oracle's
layer, through the C ABI; graph replay against eager launches, and the memory variables
through field read-back and restart."""
import numpy as np
import pytest

from gpu_util import announce, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

PML = dict(width=10, R=1e-6, kmax=1.0, f0=25.0)


def _workload(nsteps):
    """48 x 40 x 44 intervals (patches 20 / 16 / 16 with remainders), halo 8, h = 10 m,
    smooth P velocity 2400-3200 m/s (vs = vp / sqrt 3), two shots: an explosive source
    and a vertical force off centre, a line of receivers (sigma11, v3)."""
    from paper_2301_05127_amd import inputs
    g = inputs.grid(3, (48, 40, 44), (10.0, 10.0, 10.0), (20, 16, 16), 8)
    shape = (45, 41, 49)
    vp = inputs.gaussian_random_field(shape, 10.0, 60.0, 11, 2400.0, 3200.0)
    vp = np.asarray(vp, np.float32).astype(np.float64)
    vs = np.asarray(vp / np.sqrt(3.0), np.float32).astype(np.float64)
    rho = np.full(shape, 2200.0)
    dt = 1e-3

    def src(kind, pos):
        s = inputs._src(kind, pos, 20.0, 25.0, 0.04, dt, nsteps + 1)
        s["wavelet"] = np.asarray(s["wavelet"], np.float32).astype(np.float64)
        return s

    # receivers in the physical region (a velocity receiver inside the layer records the
    # mean of the half steps, which the layer's exact sub-flow does not reproduce)
    rec = np.array([[ix, 20, 30] for ix in range(12, 37, 4)], dtype=np.int32)
    shots = [{"sources": [src(1, (250.0, 190.0, 210.0))], "receivers": rec, "rec_comp": 3},
             {"sources": [src(4, (220.0, 210.0, 240.0))], "receivers": rec, "rec_comp": 2}]
    return dict(grid=g, physics=1, dt=dt, nsteps=nsteps, vp=vp, vs=vs, rho=rho, shots=shots)


def _gpu(w, flags=0):
    from paper_2301_05127_amd import loss
    sim = loss.Simulation(w["grid"], 1, w["dt"], nshots=len(w["shots"]), trace_len=w["nsteps"], flags=flags)
    sim.setup_workload(w)
    sim.set_pml(PML["width"], PML["R"], PML["kmax"], PML["f0"])
    return sim


def test_elastic_pml_matches_oracle(orc):
    """240 steps in four legs: both wave types cross the layer.  Errors are measured
    against the largest norm each field reached (late fields are small once the layer
    has absorbed them)."""
    require_gpu()
    w = _workload(240)
    announce("elastic pml parity 240 steps, 2 shots")
    sim = _gpu(w)
    pml = dict(PML, cmax=float(w["vp"].max()))
    of = [None, None]
    peak = np.zeros((2, 9))
    errs = []
    for n0 in range(0, 240, 60):
        sim.step(60)
        row = []
        for s, sh in enumerate(w["shots"]):
            of[s], _ = orc.run_pml_elastic(w["grid"], pml, w["dt"], 60, w["vp"], w["vs"], w["rho"],
                                           sources=sh["sources"], fields_in=of[s], step0=n0)
            for f in range(9):
                peak[s, f] = max(peak[s, f], np.linalg.norm(of[s][f]))
            row.append([np.linalg.norm(sim.get_field(f, shot=s) - of[s][f]) for f in range(9)])
        errs.append(row)
    errs = np.array(errs) / peak[None]
    print("field errors / peak norm, worst leg per shot and field:", errs.max(axis=0))
    assert errs.max() < 1e-5, errs.max(axis=0)
    # the layer absorbed the waves: little is left inside
    for s in range(2):
        assert max(np.linalg.norm(of[s][f]) / peak[s, f] for f in range(9)) < 0.1
    for s, sh in enumerate(w["shots"]):
        _, rt = orc.run_pml_elastic(w["grid"], pml, w["dt"], 240, w["vp"], w["vs"], w["rho"],
                                    sources=sh["sources"], receivers=sh["receivers"], rec_comp=sh["rec_comp"])
        e = rel_l2(sim.get_traces(s), rt)
        print("shot %d traces rel-L2 %.2e" % (s, e))
        assert e < 1e-5, (s, e)
    sim.close()


def test_elastic_pml_graph_and_eager_bitwise():
    """Graph replay and eager launches of the elastic schedule with the layer: same bits."""
    require_gpu()
    from paper_2301_05127_amd import loss
    w = _workload(90)
    announce("elastic pml graph vs eager")
    out = []
    for flags in (0, loss.FLAG_NO_GRAPH):
        sim = _gpu(w, flags=flags)
        sim.step(90)
        out.append(([sim.get_field(f, shot=1) for f in range(9)], sim.get_traces(1)))
        sim.close()
    for f in range(9):
        assert np.array_equal(out[0][0][f], out[1][0][f]), f
    assert np.array_equal(out[0][1], out[1][1])


def test_elastic_pml_restart_through_fields():
    """Reading the nine fields (velocity at the integer time) and writing them back
    moves the layer's velocity memory variables back and forth with them: a run split
    at step 70 matches an uninterrupted one to rounding."""
    require_gpu()
    w = _workload(160)
    announce("elastic pml restart")
    a = _gpu(w)
    a.step(160)
    b = _gpu(w)
    b.step(70)
    for s in range(2):
        for f in range(9):
            b.set_field(f, b.get_field(f, shot=s), shot=s)
    b.step(90)
    for s in range(2):
        for f in range(9):
            assert rel_l2(b.get_field(f, shot=s), a.get_field(f, shot=s)) < 1e-5, (s, f)
    a.close(); b.close()


@pytest.mark.timeout(300)
def test_elastic_pml_full_size_few_steps(orc):
    """257^3 (4^3 patches of 64, halo 10, two shots) with a 20-node layer on every side:
    a smooth state centred inside the layer near a corner, 3 steps in the launch shape
    the benchmark picks, every field of both shots against the oracle's layer."""
    require_gpu()
    from paper_2301_05127_amd import inputs, loss
    nsteps = 3
    w = inputs.config("cfg3", nsteps=nsteps)
    for k in ("vp", "vs", "rho"):
        w[k] = np.asarray(w[k], np.float32).astype(np.float64)
    for sh in w["shots"]:
        for src in sh["sources"]:
            src["wavelet"] = np.asarray(src["wavelet"], np.float32).astype(np.float64)
    S = len(w["shots"])
    announce("elastic pml full size %d steps, %d shots" % (nsteps, S))
    sim = loss.Simulation(w["grid"], 1, w["dt"], nshots=S, trace_len=nsteps)
    sim.setup_workload(w)
    sim.set_pml(20, 1e-6, 1.0, 25.0)
    sim.set_shape((4, 3208, 3208))
    shape = sim.shape
    gz, gy, gx = (np.exp(-(np.arange(n) - c) ** 2 / (2 * 8.0 ** 2)) for n, c in zip(shape, (12, 240, 15)))
    blob = (gz[:, None, None] * gy[None, :, None] * gx[None, None, :]).astype(np.float32)
    fin = np.zeros((27,) + shape)
    for f, amp in ((0, 1.0), (1, -0.7), (2, 0.5), (3, 1e6), (4, 1e6), (5, 1e6), (6, 3e5)):
        fin[f] = amp * blob
    for s in range(S):
        for f in range(9):
            sim.set_field(f, fin[f].astype(np.float32), shot=s)
    sim.step(nsteps)
    pml = dict(width=20, R=1e-6, kmax=1.0, f0=25.0, cmax=float(w["vp"].max()))
    for s in range(S):
        sh = w["shots"][s]
        rf, _ = orc.run_pml_elastic(w["grid"], pml, w["dt"], nsteps, w["vp"], w["vs"], w["rho"],
                                    sources=sh["sources"], fields_in=fin)
        for f in range(9):
            e = rel_l2(sim.get_field(f, shot=s), rf[f])
            assert e < 1e-5, (s, f, e)
        del rf
    sim.close()


@pytest.mark.timeout(300)
def test_elastic_pml_1000_steps(orc):
    """1000 steps with the layer, both shots: the waves cross it, then what is left decays
    by four to five orders of magnitude.  Every field within 1e-5 of the FP64 oracle's
    layer relative to the largest norm it reached (checkpoints every 50 steps while the
    fields peak, every 250 after)."""
    require_gpu()
    w = _workload(1000)
    S = len(w["shots"])
    announce("elastic pml 1000 steps, 2 shots")
    sim = _gpu(w)
    pml = dict(PML, cmax=float(w["vp"].max()))
    of, peak, n0 = [None] * S, np.zeros((S, 9)), 0
    err = []
    for k in [50] * 5 + [250] * 3:
        sim.step(k)
        row = np.zeros((S, 9))
        for s, sh in enumerate(w["shots"]):
            of[s], _ = orc.run_pml_elastic(w["grid"], pml, w["dt"], k, w["vp"], w["vs"], w["rho"],
                                           sources=sh["sources"], fields_in=of[s], step0=n0)
            for f in range(9):
                peak[s, f] = max(peak[s, f], np.linalg.norm(of[s][f]))
                row[s, f] = np.linalg.norm(sim.get_field(f, shot=s) - of[s][f])
        err.append(row)
        n0 += k
    err = np.array(err) / peak[None]
    print("error / peak norm at steps 50..250, 500, 750, 1000 (worst field per shot):\n",
          err.max(axis=2).T)
    assert err.max() < 1e-5, err.max(axis=(0, 2))
    sim.close()


@pytest.mark.parametrize("ckpt_every", [25, 60])
def test_elastic_layer_gradient_matches_oracle(orc, ckpt_every):
    """Gradients through the layer: two shots (explosive with v3 receivers, y force with
    sigma12 receivers, all outside the 4-node layer the waves cross), 60 steps; dJ/dlambda,
    dJ/dmu and dJ/drho (lambda, mu fixed) against the FP64 oracle's layer adjoint, which
    is pinned by central differences of the oracle's layer forward."""
    require_gpu()
    from paper_2301_05127_amd import loss
    from test_gpu_adjoint_elastic import _small_elastic_fwi
    w = _small_elastic_fwi()
    w["shots"][0]["receivers"] = np.array([[ix, 10, 12] for ix in range(5, 22, 3)], dtype=np.int32)
    w["shots"][1]["receivers"] = np.array([[8, iy, 9] for iy in range(5, 16, 2)], dtype=np.int32)
    pml = dict(width=4, R=1e-4, kmax=1.0, f0=50.0, cmax=float(w["vp"].max()))
    S, nsteps = len(w["shots"]), w["nsteps"]
    announce("elastic layer gradient, 2 shots, 60 steps, checkpoints every %d" % ckpt_every)
    obs, ref = [], np.zeros((3,) + w["vp"].shape)
    for sh in w["shots"]:
        o = orc.run_pml_elastic(w["grid"], pml, w["dt"], nsteps, w["vp"] * 1.05, w["vs"] * 0.95, w["rho"],
                                sources=sh["sources"], receivers=sh["receivers"], rec_comp=sh["rec_comp"])[1]
        d = orc.run_pml_elastic(w["grid"], pml, w["dt"], nsteps, w["vp"], w["vs"], w["rho"],
                                sources=sh["sources"], receivers=sh["receivers"], rec_comp=sh["rec_comp"])[1]
        obs.append(o)
        ref += np.array(orc.elastic_adjoint_pml(w["grid"], pml, w["dt"], nsteps, w["vp"], w["vs"], w["rho"],
                                                sh["sources"], sh["receivers"], sh["rec_comp"], d - o, with_b=True))
    ref[2] = -ref[2] / w["rho"] ** 2          # dJ/drho with lambda, mu fixed = -dJ/db / rho^2
    sim = loss.Simulation(w["grid"], 1, w["dt"], nshots=S, trace_len=nsteps)
    sim.setup_workload(w)
    sim.set_pml(pml["width"], pml["R"], pml["kmax"], pml["f0"])
    sim.forward_ckpt(nsteps, ckpt_every)
    tr = [sim.get_traces(s) for s in range(S)]
    g = sim.adjoint(np.concatenate([(tr[s] - obs[s]).ravel() for s in range(S)]), loss.GRAD_LAME_RHO)
    sim.close()
    err = [rel_l2(g[k], ref[k]) for k in range(3)]
    print("layer gradient rel-L2 vs oracle: lambda %.2e mu %.2e rho %.2e" % tuple(err))
    assert all(np.abs(ref[k]).max() > 0 for k in range(3))
    assert max(err) < 1e-4, err


def test_layer_error_paths():
    """The layer's argument checks; checkpoints of a run with the layer."""
    require_gpu()
    from paper_2301_05127_amd import loss
    w = _workload(10)
    sim = _gpu(w)
    sim.forward_ckpt(10, 5)                    # the adjoint runs through the layer
    for bad in ((21, 1e-6, 1.0, 25.0),         # wider than half the 40-interval y axis
                (10, 1.5, 1.0, 25.0),          # reflection outside (0, 1)
                (10, 1e-6, 0.5, 25.0),         # kmax < 1
                (10, 1e-6, 1.0, 0.0)):         # f0 <= 0
        with pytest.raises(loss.LossError):
            sim.set_pml(*bad)
    sim.set_pml(0)                             # width 0 removes the layer
    sim.forward_ckpt(10, 5)
    sim.close()
