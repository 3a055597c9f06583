"""GPU elastic adjoint (gradients of a trace misfit with respect to the Lame parameters
or to vp, vs) against the FP64 oracle's discrete adjoint and FP64 finite differences of
the oracle's misfit, through the C ABI: batched shots with velocity and stress
receivers, checkpoints with a ragged last segment."""
import numpy as np
import pytest

from gpu_util import announce, rel_l2, require_gpu

pytestmark = pytest.mark.gpu


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _small_elastic_fwi(nsteps=60):
    """26 x 20 x 22 intervals (patches 12 / 8 / 10 with remainders), halo 5, h = 10 m,
    smooth vp 2800-3300 m/s, vs near vp / sqrt 3, rho 2000-2400; shot 0 an explosive
    source with v3 receivers, shot 1 a y force with sigma12 receivers."""
    from paper_2301_05127_amd import inputs
    g = inputs.grid(3, (26, 20, 22), (10.0, 10.0, 10.0), (12, 8, 10), 5)
    shape = (23, 21, 27)
    vp = _f32(inputs.gaussian_random_field(shape, 10.0, 40.0, 31, 2800.0, 3300.0))
    vs = _f32(vp / np.sqrt(3.0) * (1.0 + 0.05 * inputs.gaussian_random_field(shape, 10.0, 40.0, 32, -1.0, 1.0)))
    rho = _f32(inputs.gaussian_random_field(shape, 10.0, 40.0, 33, 2000.0, 2400.0))
    dt = 1e-3

    def src(kind, pos, shift):
        return {"kind": kind, "pos": pos, "spread": 15.0,
                "wavelet": _f32(inputs.ricker(50.0, 0.025, dt, nsteps + 1, shift))}

    rec0 = np.array([[ix, 10, 18] for ix in range(2, 25, 3)], dtype=np.int32)
    # equal receiver counts per shot (the autograd view returns one [S][nrec][nt] tensor)
    rec1 = np.array([[5, iy, 4] for iy in range(1, 20, 3)] + [[20, 15, 14]], dtype=np.int32)
    shots = [{"sources": [src(1, (120.0, 90.0, 100.0), 0.5)], "receivers": rec0, "rec_comp": 2},
             {"sources": [src(3, (150.0, 110.0, 80.0), 0.0)], "receivers": rec1, "rec_comp": 6}]
    return dict(grid=g, physics=1, dt=dt, nsteps=nsteps, vp=vp, vs=vs, rho=rho, shots=shots)


def _obs(orc, w):
    # observed data from a medium 5 % off: the residual is then large against the FP32
    # rounding of the traces it is formed from
    return [orc.run(w["grid"], 1, w["dt"], w["nsteps"], w["vp"] * 1.05, w["rho"], vs=w["vs"] * 0.95,
                    sources=sh["sources"], receivers=sh["receivers"], rec_comp=sh["rec_comp"])[1]
            for sh in w["shots"]]


def _oracle_grad(orc, w, obs, vp=None, vs=None, with_b=False):
    vp = w["vp"] if vp is None else vp
    vs = w["vs"] if vs is None else vs
    gl = np.zeros_like(vp)
    gm = np.zeros_like(vp)
    gb = np.zeros_like(vp)
    for s, sh in enumerate(w["shots"]):
        d0 = orc.run(w["grid"], 1, w["dt"], w["nsteps"], vp, w["rho"], vs=vs, sources=sh["sources"],
                     receivers=sh["receivers"], rec_comp=sh["rec_comp"])[1]
        out = orc.elastic_adjoint(w["grid"], w["dt"], w["nsteps"], vp, vs, w["rho"], sh["sources"],
                                  sh["receivers"], sh["rec_comp"], d0 - obs[s], with_b=with_b)
        gl += out[0]
        gm += out[1]
        if with_b:
            gb += out[2]
    return (gl, gm, gb) if with_b else (gl, gm)


def _gpu_grad(w, obs, param, ckpt_every):
    from paper_2301_05127_amd import loss
    S, nsteps = len(w["shots"]), w["nsteps"]
    sim = loss.Simulation(w["grid"], 1, w["dt"], nshots=S, trace_len=nsteps)
    sim.setup_workload(w)
    sim.forward_ckpt(nsteps, ckpt_every)
    tr = [sim.get_traces(s) for s in range(S)]
    res = np.concatenate([(tr[s] - obs[s]).ravel() for s in range(S)])
    g = sim.adjoint(res, param)
    sim.close()
    return g, tr


@pytest.mark.parametrize("ckpt_every", [25, 60])
def test_lame_gradient_matches_oracle_and_fd(orc, ckpt_every):
    """Two shots, 60 steps (three checkpoint segments, the last one short, or one): dJ/dlambda
    and dJ/dmu against the FP64 oracle adjoint, and their directional derivatives along the
    oracle's gradients against FP64 central differences of the oracle's misfit."""
    require_gpu()
    from paper_2301_05127_amd import loss
    w = _small_elastic_fwi()
    announce("elastic gradient (lambda, mu), 2 shots, 60 steps, checkpoints every %d" % ckpt_every)
    obs = _obs(orc, w)
    g, tr = _gpu_grad(w, obs, loss.GRAD_LAME, ckpt_every)
    assert g.shape == (2,) + w["vp"].shape
    gl, gm = _oracle_grad(orc, w, obs)
    el, em = rel_l2(g[0], gl), rel_l2(g[1], gm)
    print("rel-L2 vs oracle: lambda %.2e mu %.2e" % (el, em))
    assert el < 1e-4 and em < 1e-4, (el, em)
    # the forward traces themselves
    for s, sh in enumerate(w["shots"]):
        d0 = orc.run(w["grid"], 1, w["dt"], w["nsteps"], w["vp"], w["rho"], vs=w["vs"], sources=sh["sources"],
                     receivers=sh["receivers"], rec_comp=sh["rec_comp"])[1]
        assert rel_l2(tr[s], d0) < 1e-5, s
    if ckpt_every != 25:
        return
    rho = w["rho"]
    mu = rho * w["vs"] ** 2
    lam = rho * w["vp"] ** 2 - 2 * mu

    def J(lm, mm):
        tot = 0.0
        for s, sh in enumerate(w["shots"]):
            d = orc.run(w["grid"], 1, w["dt"], w["nsteps"], np.sqrt((lm + 2 * mm) / rho), rho,
                        vs=np.sqrt(mm / rho), sources=sh["sources"], receivers=sh["receivers"],
                        rec_comp=sh["rec_comp"])[1]
            tot += 0.5 * np.sum((d - obs[s]) ** 2)
        return tot

    # directions: the oracle's own gradients (a random direction lets the dot product
    # cancel to a small fraction of its terms, below what FP32 gradients resolve)
    for k, gref in ((0, gl), (1, gm)):
        dp = gref / np.abs(gref).max() * 1e6          # at most 0.02 % of lambda or mu
        eps = 1.0
        if k == 0:
            fd = (J(lam + eps * dp, mu) - J(lam - eps * dp, mu)) / (2 * eps)
        else:
            fd = (J(lam, mu + eps * dp) - J(lam, mu - eps * dp)) / (2 * eps)
        an = float(np.sum(g[k] * dp))
        assert abs(fd - an) <= 1e-4 * abs(fd), (k, fd, an)


def test_velocity_gradient_is_the_chain_rule(orc):
    """GRAD_VPVS: (dJ/dvp, dJ/dvs) with rho fixed equals the chain rule applied to the
    oracle's Lame gradients: dJ/dvp = 2 rho vp dJ/dlambda,
    dJ/dvs = 2 rho vs (dJ/dmu - 2 dJ/dlambda)."""
    require_gpu()
    from paper_2301_05127_amd import loss
    w = _small_elastic_fwi()
    announce("elastic gradient (vp, vs)")
    obs = _obs(orc, w)
    g, _ = _gpu_grad(w, obs, loss.GRAD_VPVS, 25)
    gl, gm = _oracle_grad(orc, w, obs)
    rho, vp, vs = w["rho"], w["vp"], w["vs"]
    gvp = 2 * rho * vp * gl
    gvs = 2 * rho * vs * (gm - 2 * gl)
    e0, e1 = rel_l2(g[0], gvp), rel_l2(g[1], gvs)
    print("rel-L2 vs oracle chain rule: vp %.2e vs %.2e" % (e0, e1))
    assert e0 < 1e-4 and e1 < 1e-4, (e0, e1)


def test_elastic_adjoint_refuses_acoustic_parameters():
    require_gpu()
    from paper_2301_05127_amd import loss
    w = _small_elastic_fwi(nsteps=10)
    sim = loss.Simulation(w["grid"], 1, w["dt"], nshots=2, trace_len=10)
    sim.setup_workload(w)
    sim.forward_ckpt(10, 5)
    res = np.zeros(sum(len(sh["receivers"]) for sh in w["shots"]) * 10)
    with pytest.raises(loss.LossError):
        sim.adjoint(res, loss.GRAD_K)
    sim.close()


@pytest.mark.parametrize("param,with_rho", [(2, False), (3, False), (2, True), (3, True)])
def test_elastic_autograd_matches_adjoint(orc, param, with_rho):
    """torch.autograd over the elastic seismograms: J = 1/2 |traces - obs|^2 built in
    torch, its backward (the discrete adjoint fed the trace gradient from torch) equals
    the direct adjoint call with the same residual, for (lambda, mu) and for (vp, vs)."""
    require_gpu()
    import torch
    from paper_2301_05127_amd import autograd, loss
    w = _small_elastic_fwi(nsteps=40)
    announce("elastic autograd param=%d" % param)
    obs = np.stack(_obs(orc, w))
    S = len(w["shots"])
    dev = "cuda"
    rho = torch.tensor(w["rho"], dtype=torch.float32, device=dev)
    rho_in = rho.double().clone().requires_grad_(True) if with_rho else rho
    vp = torch.tensor(w["vp"], dtype=torch.float64, device=dev)
    vs = torch.tensor(w["vs"], dtype=torch.float64, device=dev)
    if param == loss.GRAD_VPVS:
        a, b = vp.clone(), vs.clone()
    else:
        mu = rho.double() * vs * vs
        a, b = rho.double() * vp * vp - 2 * mu, mu
    a.requires_grad_(True)
    b.requires_grad_(True)
    sim = loss.Simulation(w["grid"], 1, w["dt"], nshots=S, trace_len=40)
    sim.setup_workload(w)
    tr = autograd.elastic_seismograms(sim, a, b, rho_in, 40, ckpt_every=15, param=param)
    J = 0.5 * ((tr - torch.tensor(obs, device=dev)) ** 2).sum()
    J.backward()
    ga, gb = a.grad.cpu().numpy(), b.grad.cpu().numpy()
    # the direct path on a second handle with the same (float32) media and residual
    d = loss.Simulation(w["grid"], 1, w["dt"], nshots=S, trace_len=40)
    d.setup_workload(w)
    if param == loss.GRAD_LAME:
        vpf = torch.sqrt((a.detach().float() + 2.0 * b.detach().float()) / rho).cpu().numpy()
        vsf = torch.sqrt(b.detach().float() / rho).cpu().numpy()
    else:
        vpf, vsf = vp.float().cpu().numpy(), vs.float().cpu().numpy()
    d.set_media(vpf, w["rho"], vsf)
    d.forward_ckpt(40, 15)
    tb = np.stack([d.get_traces(s) for s in range(S)])
    assert np.array_equal(tr.detach().cpu().numpy(), tb)
    g = d.adjoint(tb - obs, param + 2 if with_rho else param)
    assert rel_l2(ga, g[0]) < 1e-12 and rel_l2(gb, g[1]) < 1e-12
    if with_rho:
        assert rel_l2(rho_in.grad.cpu().numpy(), g[2]) < 1e-12
    sim.close(); d.close()


def test_density_gradient_matches_oracle_and_fd(orc):
    """GRAD_LAME_RHO: dJ/drho with lambda and mu fixed (= -dJ/db / rho^2, b = 1/rho drives
    the velocity sub-flow and the body force) against the FP64 oracle, and its directional
    derivative along the oracle's gradient against FP64 central differences; GRAD_VPVS_RHO
    against the chain rule (dJ/drho with vp, vs fixed)."""
    require_gpu()
    from paper_2301_05127_amd import loss
    w = _small_elastic_fwi()
    announce("elastic gradient (lambda, mu, rho)")
    obs = _obs(orc, w)
    g, _ = _gpu_grad(w, obs, loss.GRAD_LAME_RHO, 25)
    assert g.shape == (3,) + w["vp"].shape
    gl, gm, gb = _oracle_grad(orc, w, obs, with_b=True)
    rho, vp, vs = w["rho"], w["vp"], w["vs"]
    grho = -gb / rho ** 2
    e = [rel_l2(g[0], gl), rel_l2(g[1], gm), rel_l2(g[2], grho)]
    print("rel-L2 vs oracle: lambda %.2e mu %.2e rho %.2e" % tuple(e))
    assert max(e) < 1e-4, e
    mu = rho * vs ** 2
    lam = rho * vp ** 2 - 2 * mu

    def J(r):
        tot = 0.0
        for s, sh in enumerate(w["shots"]):
            d = orc.run(w["grid"], 1, w["dt"], w["nsteps"], np.sqrt((lam + 2 * mu) / r), r, vs=np.sqrt(mu / r),
                        sources=sh["sources"], receivers=sh["receivers"], rec_comp=sh["rec_comp"])[1]
            tot += 0.5 * np.sum((d - obs[s]) ** 2)
        return tot

    dr = grho / np.abs(grho).max() * 0.2                 # at most 0.01 % of rho
    fd = (J(rho + dr) - J(rho - dr)) / 2.0
    an = float(np.sum(g[2] * dr))
    assert abs(fd - an) <= 1e-4 * abs(fd), (fd, an)
    gv, _ = _gpu_grad(w, obs, loss.GRAD_VPVS_RHO, 25)
    ref = [2 * rho * vp * gl, 2 * rho * vs * (gm - 2 * gl), gl * (vp ** 2 - 2 * vs ** 2) + gm * vs ** 2 + grho]
    ev = [rel_l2(gv[k], ref[k]) for k in range(3)]
    print("rel-L2 vs oracle chain rule: vp %.2e vs %.2e rho %.2e" % tuple(ev))
    assert max(ev) < 1e-4, ev


@pytest.mark.timeout(400)
def test_gradient_full_size_few_steps(orc):
    """257^3 nodes, patches of 64, halo 10 (the two-shot elastic workload's grid), the
    vertical-force shot with its line of v3 receivers through the source, 4 steps with
    checkpoints every 2, in the benchmark's launch shape: dJ/dlambda, dJ/dmu and dJ/drho
    against the FP64 oracle adjoint (dense line operators; about a minute of host time)
    for J = 1/2 sum d^2."""
    require_gpu()
    from paper_2301_05127_amd import inputs, loss
    nsteps = 4
    w = inputs.config("cfg3", nsteps=nsteps)
    w["shots"] = w["shots"][1:]
    sh = w["shots"][0]
    sh["sources"][0]["wavelet"] = _f32(inputs.ricker(15.0, 0.004, w["dt"], nsteps + 1, 0.0))   # active at once
    for k in ("vp", "vs", "rho"):
        w[k] = _f32(w[k])
    announce("elastic gradient full size, 1 shot, %d steps" % nsteps)
    d = orc.run(w["grid"], 1, w["dt"], nsteps, w["vp"], w["rho"], vs=w["vs"], sources=sh["sources"],
                receivers=sh["receivers"], rec_comp=sh["rec_comp"])[1]
    gl, gm, gb = orc.elastic_adjoint(w["grid"], w["dt"], nsteps, w["vp"], w["vs"], w["rho"], sh["sources"],
                                     sh["receivers"], sh["rec_comp"], d, with_b=True)
    sim = loss.Simulation(w["grid"], 1, w["dt"], nshots=1, trace_len=nsteps)
    sim.setup_workload(w)
    sim.set_shape([4, 3208, 3208])
    sim.forward_ckpt(nsteps, 2)
    g = sim.adjoint(d.ravel(), loss.GRAD_LAME_RHO)
    e = [rel_l2(g[0], gl), rel_l2(g[1], gm), rel_l2(g[2], -gb / w["rho"] ** 2)]
    print("rel-L2 vs oracle: lambda %.2e mu %.2e rho %.2e" % tuple(e))
    assert np.abs(gl).max() > 0 and max(e) < 1e-4, e
    sim.close()


@pytest.mark.parametrize("end_mode", [1, 2])
def test_gradient_other_end_modes(orc, end_mode):
    """The paper's one-sided end stencil and periodic lines (24^3 intervals, patches of
    12, halo 5, 30 steps, one explosive shot, checkpoints every 10): Lame gradients
    against the FP64 oracle adjoint."""
    require_gpu()
    from paper_2301_05127_amd import inputs, loss
    g = inputs.grid(3, (24, 24, 24), (10.0, 10.0, 10.0), (12, 12, 12), 5, end_mode=end_mode)
    shape = (25, 25, 25)
    vp = _f32(inputs.gaussian_random_field(shape, 10.0, 40.0, 41, 2800.0, 3300.0))
    vs = _f32(vp / np.sqrt(3.0))
    rho = np.full(shape, 2200.0)
    nsteps = 30
    src = {"kind": 1, "pos": (110.0, 120.0, 130.0), "spread": 15.0,
           "wavelet": _f32(inputs.ricker(50.0, 0.02, 1e-3, nsteps + 1, 0.5))}
    rec = np.array([[ix, 12, 6] for ix in range(0, 25, 3)], dtype=np.int32)
    w = dict(grid=g, physics=1, dt=1e-3, nsteps=nsteps, vp=vp, vs=vs, rho=rho,
             shots=[{"sources": [src], "receivers": rec, "rec_comp": 5}])
    announce("elastic gradient, end mode %d" % end_mode)
    obs = [orc.run(g, 1, 1e-3, nsteps, vp * 1.05, rho, vs=vs * 0.95, sources=[src], receivers=rec, rec_comp=5)[1]]
    gpu, _ = _gpu_grad(w, obs, loss.GRAD_LAME, 10)
    gl, gm = _oracle_grad(orc, w, obs)
    e = [rel_l2(gpu[0], gl), rel_l2(gpu[1], gm)]
    print("end mode %d rel-L2 vs oracle: lambda %.2e mu %.2e" % ((end_mode,) + tuple(e)))
    assert np.abs(gl).max() > 0 and max(e) < 1e-4, e


def test_gradient_bitwise_repeatable_with_shared_nodes(orc):
    """Two shots whose force footprints overlap, a second force in the same shot on the
    same nodes, and receivers listed twice: the density and Lame gradients of two runs
    agree bit for bit (the residual injection and the force term add each node's
    contributions in a fixed order, without atomics), and match the FP64 oracle."""
    require_gpu()
    from paper_2301_05127_amd import loss
    w = _small_elastic_fwi(nsteps=40)
    dt = w["dt"]
    from paper_2301_05127_amd import inputs

    def force(kind, pos):
        return {"kind": kind, "pos": pos, "spread": 15.0, "wavelet": _f32(inputs.ricker(50.0, 0.02, dt, 41, 0.0))}

    rec = np.array([[13, 10, 5], [13, 10, 5], [8, 10, 16], [20, 10, 16], [8, 10, 16]], dtype=np.int32)
    w["shots"] = [{"sources": [force(2, (130.0, 100.0, 110.0)), force(4, (130.0, 100.0, 110.0))],
                   "receivers": rec, "rec_comp": 0},
                  {"sources": [force(4, (140.0, 100.0, 100.0))], "receivers": rec, "rec_comp": 8}]
    announce("elastic gradient bitwise repeat, shared force footprints and repeated receivers")
    obs = _obs(orc, w)
    g1, _ = _gpu_grad(w, obs, loss.GRAD_LAME_RHO, 15)
    g2, _ = _gpu_grad(w, obs, loss.GRAD_LAME_RHO, 15)
    assert np.array_equal(g1, g2)
    gl, gm, gb = _oracle_grad(orc, w, obs, with_b=True)
    e = [rel_l2(g1[0], gl), rel_l2(g1[1], gm), rel_l2(g1[2], -gb / w["rho"] ** 2)]
    print("rel-L2 vs oracle: lambda %.2e mu %.2e rho %.2e" % tuple(e))
    assert np.abs(gb).max() > 0 and max(e) < 1e-4, e
