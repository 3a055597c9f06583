"""Parity report at full workload sizes: the HIP path against the FP64 oracle.

Not collected by pytest (the oracle needs minutes at these sizes).  Usage, on a machine
with the GPU and the built libraries:

    python tests/report_parity.py cfg1 cfg2 [cfg5 ...] [--steps N] [--shots K] [--out FILE]

For every workload it runs the GPU simulation and the oracle over the same seeded
inputs (the oracle in chunks of steps, printing progress), and prints one JSON line per
workload with rel-L2 errors of every field (whole grid and the interior 16 nodes from
every end) and of the traces.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def f32_inputs(w):
    """Round media and wavelets the way the GPU receives them."""
    w = dict(w)
    for k in ("vp", "vs", "rho"):
        if w.get(k) is not None:
            w[k] = np.asarray(w[k], np.float32).astype(np.float64)
    w["shots"] = [dict(sh, sources=[dict(s, wavelet=np.asarray(s["wavelet"], np.float32).astype(np.float64))
                                    for s in sh["sources"]]) for sh in w["shots"]]
    return w


def rel(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    d = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / d) if d > 0 else float(np.linalg.norm(x - ref))


def interior(a, band):
    sl = tuple(slice(band, -band) for _ in range(a.ndim))
    return a[sl]


def oracle_step(orc, w, shot, k, fields, step0, pml):
    sh = w["shots"][shot]
    if pml and w["physics"] == 1:
        return orc.run_pml_elastic(w["grid"], pml, w["dt"], k, w["vp"], w["vs"], w["rho"], sources=sh["sources"],
                                   receivers=sh["receivers"], rec_comp=sh.get("rec_comp", 0), fields_in=fields,
                                   step0=step0)
    if pml:
        return orc.run_pml(w["grid"], pml, w["dt"], k, w["vp"], w["rho"], sources=sh["sources"],
                           receivers=sh["receivers"], fields_in=fields, step0=step0)
    return orc.run(w["grid"], w["physics"], w["dt"], k, w["vp"], w["rho"], vs=w.get("vs"),
                   sources=sh["sources"], receivers=sh["receivers"], rec_comp=sh.get("rec_comp", 0),
                   fields_in=fields, step0=step0)


def oracle_chunked(orc, w, shot, nsteps, chunk, pml=None):
    fields, traces, done = None, [], 0
    t0 = time.time()
    while done < nsteps:
        k = min(chunk, nsteps - done)
        fields, tr = oracle_step(orc, w, shot, k, fields, done, pml)
        traces.append(tr)
        done += k
        print("  oracle shot %d: %d / %d steps, %.0f s" % (shot, done, nsteps, time.time() - t0), flush=True)
    return fields, np.concatenate(traces, axis=1)


def main():
    p = argparse.ArgumentParser()
    p.add_argument("workloads", nargs="+")
    p.add_argument("--steps", type=int, default=None)
    p.add_argument("--shots", type=int, default=None, help="shots compared (default: all)")
    p.add_argument("--chunk", type=int, default=50)
    p.add_argument("--out", default=None)
    p.add_argument("--grad", action="store_true",
                   help="acoustic: also compare the batched adjoint gradient dJ/dK with the oracle's, for the "
                        "residual = the oracle's traces")
    p.add_argument("--pml", type=int, default=0,
                   help="absorbing layer of this many nodes on every side (R = 1e-6, kmax = 1, f0 of the source)")
    p.add_argument("--save-diff", default=None,
                   help="write the GPU - oracle difference of field 0, shot 0, at the end (.npy)")
    p.add_argument("--checkpoints", default="",
                   help="comma-separated step counts at which the fields are also compared (shot 0)")
    p.add_argument("--coef-f32", action="store_true",
                   help="acoustic: give the oracle media whose update coefficients are the GPU's float32 "
                        "dt K and dt b (rho' = dt / fl32(dt b), vp' = sqrt(fl32(dt K) / (dt rho'))), so that "
                        "what remains is arithmetic rounding")
    a = p.parse_args()
    import oracle
    from paper_2301_05127_amd import inputs, loss
    oracle.build()
    results = []
    for name in a.workloads:
        w = f32_inputs(inputs.config(name, **({"nshots": a.shots} if name == "cfg5" and a.shots else {})))
        nsteps = a.steps or w["nsteps"]
        S = len(w["shots"]) if a.shots is None else min(a.shots, len(w["shots"]))
        w_gpu = w
        if a.coef_f32 and w["physics"] == 0:
            dt = w["dt"]
            dtb = np.asarray(dt / w["rho"], np.float32).astype(np.float64)
            dtK = np.asarray(((dt * w["rho"]) * w["vp"]) * w["vp"], np.float32).astype(np.float64)   # as k_media
            rho_o = dt / dtb
            w = dict(w, rho=rho_o, vp=np.sqrt(dtK / (dt * rho_o)))
        print("[%s] GPU, %d shot(s), %d steps" % (name, S, nsteps), flush=True)
        sim = loss.Simulation(w["grid"], w["physics"], w["dt"], nshots=S, trace_len=nsteps)
        sim.setup_workload(w_gpu, shots=w_gpu["shots"][:S])
        pml = None
        if a.pml:
            f0 = 15.0 if name != "cfg2" else 20.0
            pml = dict(width=a.pml, R=1e-6, kmax=1.0, f0=f0, cmax=float(np.max(w_gpu["vp"])))
            sim.set_pml(a.pml, 1e-6, 1.0, f0)
        nf = 3 if w["physics"] == 0 else 9
        res = {"workload": name, "steps": nsteps, "shots": S, "pml": a.pml, "coef_f32": bool(a.coef_f32),
               "fields": {}, "interior16": {}, "traces": {}, "checkpoints": {}}
        cps = sorted(int(c) for c in a.checkpoints.split(",") if c and int(c) < nsteps)
        shot0 = None
        if cps:
            # shot 0 at intermediate step counts, the oracle advanced alongside (and on
            # to the end: it is the final reference of shot 0)
            rf, done, trs = None, 0, []
            for cp in cps + [nsteps]:
                if cp != nsteps:
                    sim.step(cp - done)
                while done < cp:
                    k = min(a.chunk, cp - done)
                    rf, tr = oracle_step(oracle, w, 0, k, rf, done, pml)
                    trs.append(tr)
                    done += k
                    print("  oracle shot 0: %d / %d steps" % (done, nsteps), flush=True)
                if cp == nsteps:
                    break
                e = [rel(sim.get_field(f, shot=0), rf[f]) for f in range(nf)]
                ei = [rel(interior(sim.get_field(f, shot=0), 16), interior(rf[f], 16)) for f in range(nf)]
                res["checkpoints"][cp] = {"fields": e, "interior16": ei}
                print("  step %d: fields %s interior %s" % (cp, ["%.2e" % v for v in e], ["%.2e" % v for v in ei]),
                      flush=True)
            sim.step(nsteps - cps[-1])
            shot0 = (rf, np.concatenate(trs, axis=1))
        else:
            sim.step(nsteps)
        sim.sync()
        for s in range(S):
            rf, rt = shot0 if (s == 0 and shot0 is not None) else oracle_chunked(oracle, w, s, nsteps, a.chunk, pml)
            if s == 0 and a.save_diff:
                np.save(a.save_diff, (sim.get_field(0, shot=0) - rf[0]).astype(np.float32))
            for f in range(nf):
                g = sim.get_field(f, shot=s)
                res["fields"]["shot%d_f%d" % (s, f)] = rel(g, rf[f])
                res["interior16"]["shot%d_f%d" % (s, f)] = rel(interior(g, 16), interior(rf[f], 16))
            res["traces"]["shot%d" % s] = rel(sim.get_traces(s), rt)
        sim.close()
        if a.grad and w["physics"] == 0:
            # the oracle's traces of every shot as the residual (J = sum d^2 / 2)
            resid = np.zeros((S, len(w["shots"][0]["receivers"]), nsteps))
            gref = np.zeros(oracle.field_shape(w["grid"]))
            t0 = time.time()
            for sidx in range(S):
                sh = w["shots"][sidx]
                _, rt = oracle.run(w["grid"], 0, w["dt"], nsteps, w["vp"], w["rho"], sources=sh["sources"],
                                   receivers=sh["receivers"])
                resid[sidx] = rt
                gref += oracle.acoustic_adjoint(w["grid"], w["dt"], nsteps, w["vp"], w["rho"], sh["sources"],
                                                sh["receivers"], rt)
                print("  oracle adjoint shot %d: %.0f s" % (sidx, time.time() - t0), flush=True)
            g2 = loss.Simulation(w["grid"], 0, w["dt"], nshots=S, trace_len=nsteps)
            g2.setup_workload(w, shots=w["shots"][:S])
            g2.forward_ckpt(nsteps, int(w.get("ckpt_every", 100)))
            ggpu = g2.adjoint(resid, param=loss.GRAD_K)
            g2.close()
            res["gradient_K"] = rel(ggpu, gref)
            print("  gradient dJ/dK rel-L2 %.3e" % res["gradient_K"], flush=True)
        res["max_field"] = max(res["fields"].values())
        res["max_interior16"] = max(res["interior16"].values())
        res["max_traces"] = max(res["traces"].values())
        print(json.dumps(res), flush=True)
        results.append(res)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(results, fh, indent=1)


if __name__ == "__main__":
    main()
