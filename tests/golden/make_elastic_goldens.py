"""Write the FP64 oracle goldens of the full-size elastic workloads.

Calls only ``oracle`` (and the seeded input generators of ``paper_2301_05127_amd.inputs``,
which hold none of the method's arithmetic).  Usage:

    python tests/golden/make_elastic_goldens.py cfg3 cfg4

* ``cfg3`` (257^3 nodes, explosive and vertical-force shots): every receiver trace over
  1000 steps and, at steps 400 (before the first arrival at the grid ends) and 1000, all
  nine fields on the lattice of every 16th node of each axis.
* ``cfg4`` (513^3 layered medium, explosive shot): every receiver trace over 100 steps
  and all nine fields at step 100 on the lattice of every 32nd node.

The oracle runs on the inputs the GPU receives: media and wavelets rounded to float32.
Output: ``tests/golden/<cfg>_oracle.npz`` (float64 arrays ``traces_s<shot>`` [rec][t],
``fields_s<shot>_n<step>`` [field][z][y][x] on the lattice, ``stride``, ``steps``).
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
        "cfg4": dict(steps=100, snapshots=(100,), stride=32)}


def f32_inputs(w):
    w = dict(w)
    for k in ("vp", "vs", "rho"):
        w[k] = np.asarray(w[k], np.float32).astype(np.float64)
    w["shots"] = [dict(sh, sources=[dict(s, wavelet=np.asarray(s["wavelet"], np.float32).astype(np.float64))
                                    for s in sh["sources"]]) for sh in w["shots"]]
    return w


def make(name):
    plan = PLAN[name]
    w = f32_inputs(inputs.config(name, nsteps=plan["steps"]))
    st = plan["stride"]
    out = {"stride": np.int64(st), "steps": np.int64(plan["steps"]),
           "snapshots": np.array(plan["snapshots"], np.int64)}
    for shot, sh in enumerate(w["shots"]):
        fields, done, traces = None, 0, []
        for snap in plan["snapshots"]:
            t0 = time.time()
            fields, tr = oracle.run(w["grid"], 1, w["dt"], snap - done, w["vp"], w["rho"], vs=w["vs"],
                                    sources=sh["sources"], receivers=sh["receivers"],
                                    rec_comp=sh.get("rec_comp", 0), fields_in=fields, step0=done)
            traces.append(tr)
            done = snap
            out["fields_s%d_n%d" % (shot, snap)] = np.ascontiguousarray(fields[:, ::st, ::st, ::st])
            print("%s shot %d: step %d (%.0f s)" % (name, shot, snap, time.time() - t0), flush=True)
        out["traces_s%d" % shot] = np.concatenate(traces, axis=1)
    path = os.path.join(HERE, "%s_oracle.npz" % name)
    np.savez_compressed(path, **out)
    print("wrote", path, os.path.getsize(path), "bytes", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["cfg3", "cfg4"]:
        make(name)
