#!/usr/bin/env python3
"""Benchmark of the LOSS hot path on one MI355X.

Workload (default cfg4, the largest single-GPU configuration): 3-D elastic
velocity-stress, 512^3 intervals (513^3 nodes), h = 10 m, dt = 0.8 ms, 8^3 patches of
64 intervals, PMBC halo 12, four flat layers Vp 1800..5000 m/s with a +-5 % Gaussian
perturbation (seed 5127), Vs = Vp/sqrt(3), Gardner density, explosive 15 Hz Ricker,
receivers along a vertical line; synthetic inputs.  Other workloads (--workload): cfg1
(129^2 acoustic), cfg2 (2049^2 acoustic, smooth random velocity), cfg3 (257^3 elastic,
two shots in one batch), cfg5 (1025^2 acoustic, 64 shots).  --grad also times the
checkpointed forward and the adjoint of the workload itself.

Extra keys of the default run (--no-extras drops them): "gradient", the
gradient/forward time ratio of the batched acoustic adjoint (1025^2, 64 shots, 200
steps, checkpoints every 100), and "acoustic_2049", the 2049^2 acoustic rate.

One step = one Strang step of the whole hot path: PMBC junction slopes, patch
tridiagonal solves and derivative epilogues along every axis for the stress and the
velocity sub-flows, source injection, receiver recording.  Inputs are resident in
device memory before the timed region; the timed region replays the step graphs
(captured during the warm-up for every power-of-two step count up to 32).

Prints one JSON line.  value = Mcell-updates/s (nodes x shots x steps / time).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic (compulsory) bytes per node per launch of each kernel class, FP32:
# every field a kernel must read or write, counted once (halo re-reads excluded)
ALGO_BYTES = {
    0: {  # acoustic
        "stress_line_x": 8,      # read v1, write T = dv1/dx
        "stress_line_z": 20,     # read v3, T, sigma, K; write sigma
        "velocity_line_x": 16,   # read sigma, v1, b; write v1
        "velocity_line_z": 16,   # read sigma, v3, b; write v3
        "velocity_stress_x": 20,  # read sigma, v1, b; write v1 and T = d(v1 new)/dx
    },
    1: {  # elastic stress passes: x stores d1 v1, d1 v2, d1 v3 (read v, write T: 8 B each);
          # y stores d2 v2, d2 v3 (8 B each) and adds mu (d2 v1 + T) to sigma12 (read v1,
          # T, sigma12, mu; write sigma12: 20 B); z updates the three normal stresses (read
          # v3, T1, T2, 3 sigma, lambda, lambda+2mu; write 3 sigma: 44 B) and sigma13,
          # sigma23 (20 B each); velocity, per component: x stores T = d1 sigma_i1 (8 B),
          # y adds d2 sigma_i2 to T (read sigma, T; write T: 12 B), z updates v_i (read
          # sigma_i3, T, v_i, b; write v_i: 20 B)
        "stress_line_x": 24 / 3, "stress_line_y": 36 / 3, "stress_line_z": 84 / 3,
        "velocity_line_x": 8, "velocity_line_y": 12, "velocity_line_z": 20,
    },
}
STEP_BYTES = {0: 44, 1: 120}   # compulsory bytes per cell-step (whole step)
DEFAULT_STEPS = {"cfg1": 300, "cfg2": 2000, "cfg3": 1000, "cfg4": 1500, "cfg5": 3000}
CPU_SAMPLE_STEPS = {"cfg1": 3000, "cfg2": 240, "cfg3": 12, "cfg4": 2, "cfg5": 700}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's length)")
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--workload", default="cfg4", choices=sorted(DEFAULT_STEPS))
    p.add_argument("--shots", type=int, default=None, help="shots per batch (default: the workload's)")
    p.add_argument("--timing-steps", type=int, default=200)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-steps", type=int, default=None)
    p.add_argument("--grad", action="store_true",
                   help="also time the checkpointed forward and the adjoint (gradient/forward ratio)")
    p.add_argument("--no-autotune", action="store_true")
    p.add_argument("--shape", default=None,
                   help="launch shape per axis 'x,y,z' (loss_set_shape encoding); skips autotuning")
    p.add_argument("--pml", type=int, default=0,
                   help="absorbing layer of this many nodes on every side (R 1e-6, kmax 1, f0 of the source)")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the gradient/forward ratio and the 2049^2 acoustic rate of the default run")
    p.add_argument("--grad-steps", type=int, default=200, help="steps of the extra gradient/forward timing")
    p.add_argument("--copy-probe", action="store_true",
                   help="accepted for compatibility: the 1 GiB copy probe always runs")
    return p.parse_args()


def workload_desc(w, shots):
    g = w["grid"]
    n = g["n"]
    dims = "x".join(str(v) for v in ((n[0], n[2]) if g["ndim"] == 2 else n))
    return ("%s: %s %d-D, %s intervals, h=%g m, dt=%g s, patches of %s, halo %d, %d shot(s)"
            % (w["name"], "acoustic" if w["physics"] == 0 else "elastic", g["ndim"], dims, g["h"][0],
               w["dt"], "x".join(str(m) for m in (g["M"][0], g["M"][2])), g["halo"], shots))


def source_f0(name):
    """Dominant frequency of the workload's Ricker sources (sets the layer's alpha)."""
    return 20.0 if name == "cfg2" else 15.0


def cpu_baseline(w, nsteps, pml=0):
    import oracle
    oracle.build()
    sh = w["shots"][0]
    t0 = time.perf_counter()
    if pml:
        lay = dict(width=pml, R=1e-6, kmax=1.0, f0=source_f0(w["name"]), cmax=float(np.max(w["vp"])))
        if w["physics"] == 0:
            oracle.run_pml(w["grid"], lay, w["dt"], nsteps, w["vp"], w["rho"], sources=sh["sources"],
                           receivers=sh["receivers"])
        else:
            oracle.run_pml_elastic(w["grid"], lay, w["dt"], nsteps, w["vp"], w["vs"], w["rho"],
                                   sources=sh["sources"], receivers=sh["receivers"],
                                   rec_comp=sh.get("rec_comp", 0))
    else:
        oracle.run(w["grid"], w["physics"], w["dt"], nsteps, w["vp"], w["rho"], vs=w.get("vs"),
                   sources=sh["sources"], receivers=sh["receivers"], rec_comp=sh.get("rec_comp", 0))
    el = time.perf_counter() - t0
    n = w["grid"]["n"]
    nodes = (n[0] + 1) * (n[2] + 1) * (1 if w["grid"]["ndim"] == 2 else n[1] + 1)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": nodes * nsteps / el / 1e6, "unit": "Mcell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d steps of the same workload, one shot, FP64 C oracle (canonical unfused "
                      "Strang, OpenMP over lines%s), %.1f s wall" % (nsteps, ", same layer" if pml else "", el)}


def measured_traffic(workload_key, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 summary of this
    workload (profiles/line_kernels_<key>.md, FETCH_SIZE and WRITE_SIZE passes scaled by
    a 1 GiB copy), or None when the summary was taken on other kernel sources."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "line_kernels_%s.md" % workload_key)
    src = os.path.join(ROOT, "paper_2301_05127_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for line in open(path):
        if line.startswith("bench-traffic "):
            _, h, js = line.split(" ", 2)
            if h == sha:
                return json.loads(js).get(kernel)
    return None


PROFILE_KEYS = {"cfg1": "acoustic_129x129", "cfg2": "acoustic_2049x2049", "cfg3": "elastic_257cube_2shots",
                "cfg4": "elastic_513cube", "cfg5": "acoustic_1025x1025_64shots"}


def gradient_ratio(sim, w, S, nsteps, t_fwd):
    """Time forward-with-checkpoints + adjoint over the same steps as the plain forward
    (t_fwd); the residual is the recorded traces themselves (J = sum d^2 / 2)."""
    import torch
    every = int(w.get("ckpt_every", 100 if w["physics"] == 0 else 20))
    if w["physics"] == 1:
        # checkpoints (9 fields each) and the recompute's strain store (6 fields per step)
        # trade against each other; take the interval that needs least device memory
        nf, slots = 9, 6
        field_bytes = 4 * S * sim.nodes * 1.02
        need = lambda e: ((nsteps + e - 1) // e * nf + slots * e) * field_bytes
        every = min(range(1, nsteps + 1), key=need)
        free = torch.cuda.mem_get_info()[0]
        if need(every) > 0.8 * free:
            return {"steps": nsteps, "skipped": "checkpoints and strain store need %.0f GB, %.0f GB free"
                    % (need(every) / 1e9, free / 1e9)}
    sim.reset()
    sim.sync()
    t0 = time.perf_counter()
    sim.forward_ckpt(nsteps, every)
    sim.sync()
    torch.cuda.synchronize()
    t_ck = time.perf_counter() - t0
    res = np.stack([sim.get_traces(s) for s in range(S)])
    t0 = time.perf_counter()
    g = sim.adjoint(res)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    return {"steps": nsteps, "ckpt_every": every, "forward_s": round(t_fwd, 4),
            "forward_ckpt_s": round(t_ck, 4), "adjoint_s": round(t_adj, 4),
            "ratio": round((t_ck + t_adj) / t_fwd, 3), "finite": bool(np.isfinite(g).all()),
            "note": "adjoint time includes the host residual upload and gradient download"}


def timed_rate(name, steps, warmup):
    """Mcell-updates/s of one more workload (graphs replayed, autotuned launch shape)."""
    import torch
    from paper_2301_05127_amd import inputs, loss
    w = inputs.config(name, nsteps=steps + warmup)
    S = len(w["shots"])
    sim = loss.Simulation(w["grid"], w["physics"], w["dt"], nshots=S, trace_len=steps + warmup)
    sim.setup_workload(w)
    cw = sim.autotune(3)
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.close()
    return {"workload": workload_desc(w, S), "value": round(sim.nodes * S * steps / el / 1e6, 2),
            "unit": "Mcell-updates/s", "steps": steps, "ms_per_step": round(1e3 * el / steps, 5),
            "columns_per_wave": cw,
            "hbm_effective_frac": round(sim.nodes * S * steps / el * STEP_BYTES[w["physics"]] / 1e9
                                        / HBM_PEAK_GBS, 4)}


def extra_gradient(steps, warmup=10):
    """Gradient/forward time ratio of the batched acoustic adjoint (1025^2 nodes, 64 shots,
    checkpoints every 100 steps): plain forward, then checkpointed forward + adjoint."""
    import torch
    from paper_2301_05127_amd import inputs, loss
    w = inputs.config("cfg5", nsteps=steps)
    S = len(w["shots"])
    sim = loss.Simulation(w["grid"], w["physics"], w["dt"], nshots=S, trace_len=steps)
    sim.setup_workload(w)
    sim.autotune(3)
    sim.step(warmup)
    sim.reset()
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    out = gradient_ratio(sim, w, S, steps, t_fwd)
    out["workload"] = workload_desc(w, S)
    sim.close()
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: the library runs on one GPU; --gpus %d is not supported (shots, then "
              "blocks of patches, would be the units to shard across GPUs)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.grad and a.pml and a.workload in ("cfg3", "cfg4"):
        print("bench.py: the elastic adjoint is built without the absorbing layer; drop --pml or --grad",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2301_05127_amd import inputs, loss
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)
    torch.cuda.init()
    if a.steps is None:
        a.steps = DEFAULT_STEPS[a.workload]
    total = a.warmup + a.steps
    w = inputs.config(a.workload, nsteps=total)
    S = a.shots if a.shots is not None else len(w["shots"])
    shots = (w["shots"] * S)[:S]
    g = w["grid"]
    sim = loss.Simulation(g, w["physics"], w["dt"], nshots=S, trace_len=total)
    sim.setup_workload(w, shots=shots)
    if a.pml:
        sim.set_pml(a.pml, 1e-6, 1.0, source_f0(a.workload))
    nodes = sim.nodes
    if a.shape:
        cw = [int(v) for v in a.shape.split(",")]
        sim.set_shape(cw)
    else:
        cw = sim.autotune(3) if not a.no_autotune else [0, 0, 0]
    # warmup (also builds the step graph)
    sim.step(a.warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(a.steps)
    sim.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    value = nodes * S * a.steps / el / 1e6
    finite = bool(np.isfinite(sim.get_field(0)).all())

    # per-kernel durations (HIP events around every launch on the simulation stream)
    ts = min(a.timing_steps, a.steps)
    kt = []
    if ts > 0:
        sim.set_timing(True)
        sim.step(ts)
        sim.sync()
        kt = [(n, ms, c) for (n, ms, c) in sim.kernel_timing() if c > 0]
        sim.set_timing(False)
    kernels = {n: {"avg_us": 1e3 * ms / c, "launches": c, "total_ms": ms} for (n, ms, c) in kt}
    dom = max(kt, key=lambda t: t[1]) if kt else None
    algo = ALGO_BYTES.get(w["physics"], {})
    roof = None
    if dom and dom[0] in algo:
        bytes_per_launch = algo[dom[0]] * nodes * S
        avg_s = dom[1] / dom[2] / 1e3
        ach = bytes_per_launch / avg_s / 1e9
        tr = measured_traffic(PROFILE_KEYS[a.workload], dom[0]) if S == len(w["shots"]) and not a.pml else None
        roof = {"bound": "hbm", "kernel": dom[0], "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": tr,
                "bytes_per_node": round(algo[dom[0]], 3), "algorithmic_bytes": round(bytes_per_launch)}
    for n, d in kernels.items():
        if n in algo:
            d["algo_GBs"] = round(algo[n] * nodes * S / (d["avg_us"] * 1e-6) / 1e9, 1)
    step_bytes = STEP_BYTES[w["physics"]]
    eff = value * 1e6 * step_bytes / 1e9

    grad = None
    if a.grad:
        grad = gradient_ratio(sim, w, S, a.steps, el)

    # device-to-device copy of 1 GiB: the bandwidth a plain streaming kernel reaches here
    x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        y.copy_(x)
    e1.record()
    e1.synchronize()
    copy_gbs = 5 * 2 * x.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y

    res = {
        "metric": "Mcell-updates/s",
        "value": round(value, 2),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(1e3 * el / a.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload_desc(w, S) + (", absorbing layer of %d nodes" % a.pml if a.pml else ""),
                   "nodes": nodes, "shots": S,
                   "columns_per_wave": cw,
                   "hbm_effective_GBs": round(eff, 1),
                   "hbm_effective_frac": round(eff / HBM_PEAK_GBS, 4),
                   "compulsory_bytes_per_cell_step": step_bytes, "finite": finite,
                   "copy_1GiB_GBs": round(copy_gbs, 1)},
        "roofline": roof,
        "kernels": kernels,
    }
    if grad:
        res["gradient"] = grad
    sim.close()
    del sim
    if not a.no_extras and a.workload == "cfg4" and not a.pml:
        if "gradient" not in res:
            res["gradient"] = extra_gradient(a.grad_steps)
        res["acoustic_2049"] = timed_rate("cfg2", 200, 20)
    if not a.no_cpu_baseline:
        cs = a.cpu_sample_steps or CPU_SAMPLE_STEPS[a.workload]
        res["cpu_baseline"] = cpu_baseline(inputs.config(a.workload, nsteps=cs), cs, a.pml)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
