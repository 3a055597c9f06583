"""Write the FP64 oracle goldens of the full-size workloads.

Calls only ``oracle`` (and the seeded input generators of ``paper_2301_05127_amd.inputs``,
which hold none of the method's arithmetic).  Usage:

    python tests/golden/make_goldens.py cfg3 cfg4 cfg3_pml cfg2_pml

* ``cfg3`` (257^3 nodes, explosive and vertical-force shots): every receiver trace over
  1000 steps and, at steps 400 (before the first arrival at the grid ends) and 1000, all
  nine fields on the lattice of every 16th node of each axis.
* ``cfg4`` (513^3 layered medium, explosive shot): every receiver trace over 100 steps
  and all nine fields at step 100 on the lattice of every 32nd node.
* ``cfg3_pml``: the 257^3 workload with the absorbing layer (Sec. 3.3) on every side,
  20 nodes wide, R = 1e-6, k_max = 1, alpha from the 15 Hz source frequency: 1000 steps,
  lattice of every 16th node at steps 400 and 1000.  With natural ends alone, FP32-sized
  perturbations grow exponentially at the grid corners of a 3-D elastic run (the FP64
  oracle fed such noise diverges like the GPU), so long runs take the layer, as the
  paper pairs natural ends with it.
* ``cfg2_pml``: the 2049^2 acoustic workload with a 50-node layer (R = 1e-6, k_max = 1,
  alpha from the 20 Hz source): 2000 steps, the three fields on the lattice of every 32nd
  node at steps 500, 1000 and 2000 (no traces: the receiver row lies inside the layer).

The oracle runs on the inputs the GPU receives: media and wavelets rounded to float32.
Output: ``tests/golden/<cfg>_oracle.npz`` (float64 arrays ``traces_s<shot>`` [rec][t],
``fields_s<shot>_n<step>`` [field][z][y][x] on the lattice, ``stride``, ``steps``,
``shots_done``; the file is rewritten after each shot).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2301_05127_amd import inputs  # noqa: E402

PLAN = {"cfg3": dict(steps=1000, snapshots=(400, 1000), stride=16),
        "cfg4": dict(steps=100, snapshots=(100,), stride=32),
        "cfg3_pml": dict(base="cfg3", steps=1000, snapshots=(400, 1000), stride=16,
                         pml=dict(width=20, R=1e-6, kmax=1.0, f0=15.0)),
        "cfg2_pml": dict(base="cfg2", steps=2000, snapshots=(500, 1000, 2000), stride=32,
                         pml=dict(width=50, R=1e-6, kmax=1.0, f0=20.0), traces=False)}


def f32_inputs(w):
    w = dict(w)
    for k in ("vp", "vs", "rho"):
        if w.get(k) is not None:
            w[k] = np.asarray(w[k], np.float32).astype(np.float64)
    w["shots"] = [dict(sh, sources=[dict(s, wavelet=np.asarray(s["wavelet"], np.float32).astype(np.float64))
                                    for s in sh["sources"]]) for sh in w["shots"]]
    return w


def make(name):
    plan = PLAN[name]
    w = f32_inputs(inputs.config(plan.get("base", name), nsteps=plan["steps"]))
    st = plan["stride"]
    pml = plan.get("pml")
    if pml is not None:
        pml = dict(pml, cmax=float(np.max(w["vp"])))
    out = {"stride": np.int64(st), "steps": np.int64(plan["steps"]),
           "snapshots": np.array(plan["snapshots"], np.int64)}
    if pml is not None:
        out["pml"] = np.array([pml["width"], pml["R"], pml["kmax"], pml["f0"]], np.float64)
    path = os.path.join(HERE, "%s_oracle.npz" % name)
    for shot, sh in enumerate(w["shots"]):
        fields, done, traces = None, 0, []
        for snap in plan["snapshots"]:
            t0 = time.time()
            rec = sh["receivers"] if plan.get("traces", True) else None
            if w["physics"] == 0 and pml is None:
                fields, tr = oracle.run(w["grid"], 0, w["dt"], snap - done, w["vp"], w["rho"],
                                        sources=sh["sources"], receivers=rec, fields_in=fields, step0=done)
            elif w["physics"] == 0:
                fields, tr = oracle.run_pml(w["grid"], pml, w["dt"], snap - done, w["vp"], w["rho"],
                                            sources=sh["sources"], receivers=rec, fields_in=fields, step0=done)
            elif pml is None:
                fields, tr = oracle.run(w["grid"], 1, w["dt"], snap - done, w["vp"], w["rho"], vs=w["vs"],
                                        sources=sh["sources"], receivers=sh["receivers"],
                                        rec_comp=sh.get("rec_comp", 0), fields_in=fields, step0=done)
            else:
                fields, tr = oracle.run_pml_elastic(w["grid"], pml, w["dt"], snap - done, w["vp"], w["vs"],
                                                    w["rho"], sources=sh["sources"], receivers=sh["receivers"],
                                                    rec_comp=sh.get("rec_comp", 0), fields_in=fields, step0=done)
            traces.append(tr)
            done = snap
            nf = 9 if w["physics"] == 1 else 3
            sub = (slice(0, nf),) + (slice(None, None, st),) * (fields.ndim - 1)
            out["fields_s%d_n%d" % (shot, snap)] = np.ascontiguousarray(fields[sub])
            print("%s shot %d: step %d (%.0f s)" % (name, shot, snap, time.time() - t0), flush=True)
        if plan.get("traces", True):
            out["traces_s%d" % shot] = np.concatenate(traces, axis=1)
        out["shots_done"] = np.int64(shot + 1)
        np.savez_compressed(path + ".tmp.npz", **out)
        os.replace(path + ".tmp.npz", path)
        print("wrote", path, os.path.getsize(path), "bytes", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["cfg3", "cfg4", "cfg3_pml", "cfg2_pml"]:
        make(name)
