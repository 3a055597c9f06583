"""GPU adjoint: the transposed derivative operator and the checkpointed FWI gradient
of the acoustic Strang scheme, against the FP64 oracle (dense transposes) and
finite differences.  Paper Sec. 2 eq. acoustic_wave, Sec. 3.2-3.3."""
import numpy as np
import pytest

from gpu_util import announce, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

CASES = [
    ((128, 0, 96), (32, 32, 24), 8, 0),
    ((100, 0, 77), (32, 16, 16), 6, 0),
    ((96, 0, 96), (24, 24, 24), 8, 1),
    ((96, 0, 64), (32, 16, 16), 7, 2),
    ((2048, 0, 64), (256, 256, 64), 12, 0),
    ((96, 0, 80), (4, 4, 8), 12, 0),               # halo wider than the patches: up to 7
    ((96, 0, 96), (8, 8, 8), 20, 2),               # junction rows reach one node
]


@pytest.mark.parametrize("case", CASES)
def test_transpose_matches_dense(orc, case):
    require_gpu()
    from paper_2301_05127_amd import inputs, loss
    n, M, halo, mode = case
    g = inputs.grid(2, n, (10.0, 10.0, 10.0), M, halo, mode)
    announce("transpose %s" % (case,))
    sim = loss.Simulation(g, loss.ACOUSTIC, 1e-4, nshots=1)
    w = inputs.random_field(sim.shape, seed=7).astype(np.float32)
    u = inputs.random_field(sim.shape, seed=8).astype(np.float32)
    for axis, N, m in ((0, n[0], M[0]), (2, n[2], M[2])):
        got = sim.deriv(axis, -1, w[None])[0]
        D = orc.line_deriv_matrix(N, 10.0, m, halo, mode)
        w64 = w.astype(np.float64)
        ref = (w64 @ D) if axis == 0 else (D.T @ w64)
        assert rel_l2(got, ref) < 2e-6, axis
        # dot-product identity <D u, w> = <u, D^T w> with the GPU operators
        du = sim.deriv(axis, 1, u[None])[0].astype(np.float64)
        lhs = float(np.sum(du * w64))
        rhs = float(np.sum(u.astype(np.float64) * got))
        assert abs(lhs - rhs) <= 1e-5 * np.sqrt(np.sum(du ** 2) * np.sum(w64 ** 2))
    sim.close()


def _small_fwi(nshots=2, nsteps=140):
    from paper_2301_05127_amd import inputs
    N, M, halo, h, dt = 96, 32, 8, 10.0, 1e-3
    g = inputs.grid(2, (N, 0, N), (h, h, h), (M, M, M), halo)
    shape = (N + 1, N + 1)
    vp = inputs.gaussian_random_field(shape, h, 120.0, 1, 1800.0, 2600.0)
    vp = vp.astype(np.float32).astype(np.float64)
    rho = np.full(shape, 1000.0)
    rec = np.array([[ix, 0, 12] for ix in range(12, N - 11, 2)], np.int32)
    shots = []
    for s in range(nshots):
        wav = inputs.ricker(30.0, 0.04, dt, nsteps + 1, 0.5).astype(np.float32).astype(np.float64)
        shots.append({"sources": [{"kind": 0, "pos": (300.0 + 300.0 * s, 0.0, 150.0), "spread": 20.0,
                                   "wavelet": wav}], "receivers": rec, "rec_comp": 0})
    return dict(name="fwi-small", grid=g, physics=0, dt=dt, nsteps=nsteps, vp=vp, vs=None, rho=rho,
                shots=shots)


def test_gradient_matches_oracle_and_fd(orc):
    """Batched shots, checkpoints every 40 steps: dJ/dc vs the FP64 oracle adjoint and vs
    FP64 finite differences of J along a smooth direction."""
    require_gpu()
    from paper_2301_05127_amd import inputs, loss
    w = _small_fwi()
    S, nsteps = len(w["shots"]), w["nsteps"]
    announce("fwi gradient S=%d nsteps=%d" % (S, nsteps))
    obs = [orc.run(w["grid"], 0, w["dt"], nsteps, w["vp"] * 1.03, w["rho"], sources=sh["sources"],
                   receivers=sh["receivers"])[1] for sh in w["shots"]]
    sim = loss.Simulation(w["grid"], 0, w["dt"], nshots=S, trace_len=nsteps)
    sim.setup_workload(w)
    sim.forward_ckpt(nsteps, 40)
    tr = [sim.get_traces(s) for s in range(S)]
    res = np.concatenate([(tr[s] - obs[s]).ravel() for s in range(S)])
    g_gpu = sim.adjoint(res, loss.GRAD_VP)
    # FP64 oracle gradient, shot by shot
    g_ref = np.zeros_like(g_gpu)
    for s, sh in enumerate(w["shots"]):
        d0 = orc.run(w["grid"], 0, w["dt"], nsteps, w["vp"], w["rho"], sources=sh["sources"],
                     receivers=sh["receivers"])[1]
        gK = orc.acoustic_adjoint(w["grid"], w["dt"], nsteps, w["vp"], w["rho"], sh["sources"],
                                  sh["receivers"], d0 - obs[s])
        g_ref += gK * 2 * w["rho"] * w["vp"]
    e = rel_l2(g_gpu, g_ref)
    assert e < 1e-4, e
    # directional derivative vs FP64 central differences of the oracle's J
    dc = inputs.gaussian_random_field(g_gpu.shape, 10.0, 150.0, 3, -1.0, 1.0) * 15.0

    def J(v):
        tot = 0.0
        for s, sh in enumerate(w["shots"]):
            d = orc.run(w["grid"], 0, w["dt"], nsteps, v, w["rho"], sources=sh["sources"],
                        receivers=sh["receivers"])[1]
            tot += 0.5 * np.sum((d - obs[s]) ** 2)
        return tot

    eps = 1e-3
    fd = (J(w["vp"] + eps * dc) - J(w["vp"] - eps * dc)) / (2 * eps)
    an = float(np.sum(g_gpu * dc))
    assert abs(fd - an) <= 1e-4 * abs(fd), (fd, an)
    sim.close()


def test_forward_ckpt_traces_match_plain_run():
    """The checkpointed forward records the same traces as plain stepping."""
    require_gpu()
    from paper_2301_05127_amd import loss
    w = _small_fwi(nshots=2, nsteps=90)
    announce("ckpt traces")
    a = loss.Simulation(w["grid"], 0, w["dt"], nshots=2, trace_len=90)
    a.setup_workload(w)
    a.forward_ckpt(90, 25)
    b = loss.Simulation(w["grid"], 0, w["dt"], nshots=2, trace_len=90, flags=loss.FLAG_NO_GRAPH)
    b.setup_workload(w)
    b.step(90)
    for s in range(2):
        assert np.array_equal(a.get_traces(s), b.get_traces(s))
    a.close(); b.close()


@pytest.mark.parametrize("param", [0, 1])
def test_autograd_function_matches_adjoint(orc, param):
    """torch.autograd over the seismograms: J = 1/2 |traces - obs|^2 built in torch, its
    backward (the discrete adjoint fed the trace gradient from torch) equals the direct
    adjoint call with the same residual, and the traces equal the numpy readout."""
    require_gpu()
    import torch
    from paper_2301_05127_amd import autograd, loss
    w = _small_fwi(nshots=2, nsteps=90)
    S, nsteps = 2, 90
    announce("autograd seismograms param=%d" % param)
    obs = np.stack([orc.run(w["grid"], 0, w["dt"], nsteps, w["vp"] * 1.02, w["rho"], sources=sh["sources"],
                            receivers=sh["receivers"])[1] for sh in w["shots"]])
    rho = torch.tensor(w["rho"], dtype=torch.float32, device="cuda")
    vp = torch.tensor(w["vp"], dtype=torch.float64, device="cuda")
    m = (vp if param == loss.GRAD_VP else rho.double() * vp * vp).clone().requires_grad_(True)
    sim = loss.Simulation(w["grid"], 0, w["dt"], nshots=S, trace_len=nsteps)
    sim.setup_workload(w)
    tr = autograd.seismograms(sim, m, rho, nsteps, ckpt_every=30, param=param)
    J = 0.5 * ((tr - torch.tensor(obs, device="cuda")) ** 2).sum()
    J.backward()
    g_auto = m.grad.cpu().numpy()
    tr_np = tr.detach().cpu().numpy()
    # the direct path on a second handle with the same model and residual
    b = loss.Simulation(w["grid"], 0, w["dt"], nshots=S, trace_len=nsteps)
    b.setup_workload(w)
    b.set_media(vp.float().cpu().numpy() if param == loss.GRAD_VP else
                torch.sqrt(m.detach().float() / rho).cpu().numpy(), w["rho"])
    b.forward_ckpt(nsteps, 30)
    tb = np.stack([b.get_traces(s) for s in range(S)])
    assert np.array_equal(tr_np, tb)
    g_dir = b.adjoint(tb - obs, param)
    assert np.abs(J.item() - 0.5 * np.sum((tb - obs) ** 2)) <= 1e-12 * J.item()
    assert rel_l2(g_auto, g_dir) < 1e-12
    sim.close(); b.close()


@pytest.mark.parametrize("case", CASES)
def test_fused_x_adjoint_bitwise_equal(case):
    """The one-block x adjoint (solve, junction rows, gather with y in LDS) gives the bits
    of the three separate kernels, for the transposed derivative and its AXPY form."""
    require_gpu()
    from paper_2301_05127_amd import inputs, loss
    n, M, halo, mode = case
    g = inputs.grid(2, n, (10.0, 10.0, 10.0), M, halo, mode)
    announce("fused x adjoint %s" % (case,))
    out = []
    for flags in (0, loss.FLAG_NO_FUSE_X):
        sim = loss.Simulation(g, loss.ACOUSTIC, 1e-4, nshots=1, flags=flags)
        w = inputs.random_field(sim.shape, seed=11).astype(np.float32)
        out.append(sim.deriv(0, -1, np.stack([w, 2 * w])))
        sim.close()
    assert np.array_equal(out[0], out[1])


def test_fused_x_adjoint_gradient_bitwise_equal():
    """Whole FWI gradient with the fused x adjoint and with the separate kernels."""
    require_gpu()
    from paper_2301_05127_amd import loss
    w = _small_fwi(nshots=2, nsteps=70)
    announce("fused x adjoint gradient")
    grads = []
    for flags in (0, loss.FLAG_NO_FUSE_X):
        sim = loss.Simulation(w["grid"], 0, w["dt"], nshots=2, trace_len=70, flags=flags)
        sim.setup_workload(w)
        sim.forward_ckpt(70, 25)
        res = np.concatenate([sim.get_traces(s).ravel() for s in range(2)])
        grads.append(sim.adjoint(res, loss.GRAD_K))
        sim.close()
    assert np.array_equal(grads[0], grads[1])


@pytest.mark.timeout(400)   # the FP64 oracle adjoint takes ~30 s per shot at this size
def test_gradient_full_size_few_steps(orc):
    """1025^2 nodes, patches of 128, halo 12, 1024 receivers per shot (the batched-adjoint
    workload's grid), 2 shots, 12 steps with checkpoints every 5, in the launch shape of
    the benchmark: dJ/dK against the FP64 oracle adjoint for J = 1/2 sum d^2."""
    require_gpu()
    from paper_2301_05127_amd import inputs, loss
    nsteps = 12
    w = inputs.config("cfg5", nshots=2, nsteps=nsteps)
    for s, sh in enumerate(w["shots"]):   # sources already active in the first steps
        sh["sources"][0]["wavelet"] = inputs.ricker(15.0, 0.004 + 0.002 * s, w["dt"], nsteps + 1, 0.5)
    w = _f32_adj(w)
    announce("gradient full size 2 shots %d steps" % nsteps)
    resid, g_ref = [], np.zeros((1025, 1025))
    for sh in w["shots"]:
        d = orc.run(w["grid"], 0, w["dt"], nsteps, w["vp"], w["rho"], sources=sh["sources"],
                    receivers=sh["receivers"])[1]
        resid.append(d)
        g_ref += orc.acoustic_adjoint(w["grid"], w["dt"], nsteps, w["vp"], w["rho"], sh["sources"],
                                      sh["receivers"], d)
    sim = loss.Simulation(w["grid"], 0, w["dt"], nshots=2, trace_len=nsteps)
    sim.setup_workload(w)
    sim.set_shape([8, None, 1608])
    sim.forward_ckpt(nsteps, 5)
    g = sim.adjoint(np.concatenate([r.ravel() for r in resid]), loss.GRAD_K)
    e = rel_l2(g, g_ref)
    assert np.abs(g_ref).max() > 0 and e < 1e-4, e
    sim.close()


def _f32_adj(w):
    w = dict(w)
    w["vp"] = np.asarray(w["vp"], np.float32).astype(np.float64)
    w["rho"] = np.asarray(w["rho"], np.float32).astype(np.float64)
    w["shots"] = [dict(sh, sources=[dict(s, wavelet=np.asarray(s["wavelet"], np.float32).astype(np.float64))
                                    for s in sh["sources"]]) for sh in w["shots"]]
    return w


def test_gradient_bitwise_repeatable_with_repeated_receivers(orc):
    """Receivers listed twice at one node: two gradient runs agree bit for bit and the
    gradient matches the FP64 oracle adjoint (each node adds its receivers' residuals in
    receiver order, without atomics)."""
    require_gpu()
    from paper_2301_05127_amd import loss
    w = _small_fwi(nshots=2, nsteps=80)
    rec = w["shots"][0]["receivers"]
    rec2 = np.concatenate([rec, rec[::3]])
    for sh in w["shots"]:
        sh["receivers"] = rec2
    announce("acoustic gradient bitwise repeat, repeated receivers")
    grads = []
    for _ in range(2):
        sim = loss.Simulation(w["grid"], 0, w["dt"], nshots=2, trace_len=80)
        sim.setup_workload(w)
        sim.forward_ckpt(80, 30)
        tr = [sim.get_traces(s) for s in range(2)]
        res = np.concatenate([(0.5 * tr[s]).ravel() for s in range(2)])
        grads.append(sim.adjoint(res, loss.GRAD_K))
        sim.close()
    assert np.array_equal(grads[0], grads[1])
    gK = np.zeros_like(grads[0])
    for s, sh in enumerate(w["shots"]):
        d = orc.run(w["grid"], 0, w["dt"], 80, w["vp"], w["rho"], sources=sh["sources"], receivers=sh["receivers"])[1]
        gK += orc.acoustic_adjoint(w["grid"], w["dt"], 80, w["vp"], w["rho"], sh["sources"], sh["receivers"], 0.5 * d)
    e = rel_l2(grads[0], gK)
    print("rel-L2 vs oracle %.2e" % e)
    assert e < 1e-4, e
