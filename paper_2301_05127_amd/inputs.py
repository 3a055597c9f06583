"""Seeded synthetic inputs shared by the tests, the benchmark and the CPU baseline.

This module holds none of the simulator's arithmetic: it only draws media, source
wavelets and acquisition geometry.  Both the HIP library and the FP64 oracle take
these arrays as inputs.

Workloads (the paper measures on synthetic models only, Sec. 4; none of its data is
available, and these recipes stand in for its experiments):

* ``cfg1`` 2-D acoustic, 128x128 intervals, h = 10 m, dt = 1 ms, c = 2000 m/s,
  2x2 patches of 64 intervals, halo 8, 15 Hz Ricker at the centre node, 300 steps;
  receivers on the row z = 320 m below the source.
* ``cfg2`` 2-D acoustic, 2048x2048 intervals, 8x8 patches of 256, halo 12,
  c = smooth Gaussian random field in [1500, 4500] m/s (seed 2301, correlation
  length 200 m), 20 Hz Ricker at the centre, 2000 steps.
* ``cfg3`` 3-D elastic, 256^3 intervals, 4^3 patches of 64, halo 10, homogeneous
  Vp 3000, Vs 1730, rho 2200; two shots: explosive and vertical force at the centre,
  15 Hz Ricker, 1000 steps.
* ``cfg4`` 3-D elastic, 512^3 intervals, 8^3 patches of 64, halo 12, four flat
  layers Vp 1800..5000 with a +-5 % Gaussian perturbation (seed 5127), Vs = Vp/sqrt(3),
  Gardner density, explosive source, 1500 steps.
* ``cfg5`` batched acoustic adjoint, 1024x1024 intervals, 8x8 patches of 128,
  halo 12, 64 shots along the top, 1024 receivers, c in [1500, 4000] (seed 1),
  3000 steps, checkpoints every 100 steps.
"""
from __future__ import annotations

import math

import numpy as np

RHO_ACOUSTIC = 1000.0


def ricker(f0: float, t0: float, dt: float, nt: int, shift: float = 0.0) -> np.ndarray:
    """Ricker wavelet (1 - 2 (pi f (t - t0))^2) exp(-(pi f (t - t0))^2) at t = (k + shift) dt."""
    t = (np.arange(nt, dtype=np.float64) + shift) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def gaussian_random_field(shape, h: float, corr_len: float, seed: int, lo: float, hi: float):
    """White noise on the node grid, Gaussian-filtered (std corr_len/h cells) in Fourier
    space, then mapped affinely onto [lo, hi]."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    sig = corr_len / h
    spec = np.fft.fftn(w)
    for ax, n in enumerate(shape):
        k = np.fft.fftfreq(n) * 2.0 * math.pi
        filt = np.exp(-0.5 * (k * sig) ** 2)
        sh = [1] * len(shape)
        sh[ax] = n
        spec = spec * filt.reshape(sh)
    f = np.real(np.fft.ifftn(spec))
    f = (f - f.min()) / max(f.max() - f.min(), 1e-300)
    return lo + (hi - lo) * f


def smooth(field, h: float, std_m: float):
    """Gaussian smoothing (std in metres) by FFT filtering; used for a starting model."""
    sig = std_m / h
    spec = np.fft.fftn(field - field.mean())
    for ax, n in enumerate(field.shape):
        k = np.fft.fftfreq(n) * 2.0 * math.pi
        filt = np.exp(-0.5 * (k * sig) ** 2)
        sh = [1] * field.ndim
        sh[ax] = n
        spec = spec * filt.reshape(sh)
    return np.real(np.fft.ifftn(spec)) + field.mean()


def grid(ndim, n, h, M, halo, end_mode=0):
    """Grid description dict shared by the oracle and the library bindings."""
    nn = list(n) + [0] * (3 - len(n))
    hh = list(h) + [h[-1]] * (3 - len(h))
    MM = list(M) + [M[-1]] * (3 - len(M))
    if ndim == 2:
        nn[1] = 0
    return {"ndim": ndim, "n": tuple(int(v) for v in nn), "h": tuple(float(v) for v in hh),
            "M": tuple(int(v) for v in MM), "halo": int(halo), "end_mode": int(end_mode)}


def field_shape(g):
    n = g["n"]
    if g["ndim"] == 2:
        return (n[2] + 1, n[0] + 1)
    return (n[2] + 1, n[1] + 1, n[0] + 1)


def config(name: str, **over):
    """Return a workload dict: grid, physics, dt, nsteps, media, shots (sources and
    receivers per shot).  Keyword overrides replace top-level entries (e.g. nsteps)."""
    if name == "cfg1":
        g = grid(2, (128, 0, 128), (10.0, 10.0, 10.0), (64, 64, 64), 8)
        shape = field_shape(g)
        dt, nsteps, f0 = 1e-3, 300, 15.0
        vp = np.full(shape, 2000.0)
        rho = np.full(shape, RHO_ACOUSTIC)
        rec = np.array([[ix, 0, 96] for ix in range(16, 113, 4)], dtype=np.int32)
        shots = [{"sources": [_src(0, (640.0, 0.0, 640.0), 20.0, f0, 1.2 / f0, dt, nsteps + 1)],
                  "receivers": rec, "rec_comp": 0}]
        w = dict(name=name, grid=g, physics=0, dt=dt, nsteps=nsteps, vp=vp, vs=None, rho=rho,
                 shots=shots)
    elif name == "cfg2":
        g = grid(2, (2048, 0, 2048), (10.0, 10.0, 10.0), (256, 256, 256), 12)
        shape = field_shape(g)
        dt, nsteps, f0 = 1e-3, 2000, 20.0
        vp = gaussian_random_field(shape, 10.0, 200.0, 2301, 1500.0, 4500.0)
        rho = np.full(shape, RHO_ACOUSTIC)
        shots = [{"sources": [_src(0, (10240.0, 0.0, 10240.0), 20.0, f0, 1.2 / f0, dt, nsteps + 1)],
                  "receivers": _rec_row(g, 2, step=1), "rec_comp": 0}]
        w = dict(name=name, grid=g, physics=0, dt=dt, nsteps=nsteps, vp=vp, vs=None, rho=rho,
                 shots=shots)
    elif name == "cfg3":
        g = grid(3, (256, 256, 256), (10.0, 10.0, 10.0), (64, 64, 64), 10)
        shape = field_shape(g)
        dt, nsteps, f0 = 1e-3, 1000, 15.0
        vp = np.full(shape, 3000.0)
        vs = np.full(shape, 1730.0)
        rho = np.full(shape, 2200.0)
        c = (1280.0, 1280.0, 1280.0)
        rec = np.array([[128, 128, k] for k in range(0, 257, 4)], dtype=np.int32)
        shots = [{"sources": [_src(1, c, 20.0, f0, 1.2 / f0, dt, nsteps + 1)], "receivers": rec,
                  "rec_comp": 2},
                 {"sources": [_src(4, c, 20.0, f0, 1.2 / f0, dt, nsteps + 1)], "receivers": rec,
                  "rec_comp": 2}]
        w = dict(name=name, grid=g, physics=1, dt=dt, nsteps=nsteps, vp=vp, vs=vs, rho=rho,
                 shots=shots)
    elif name == "cfg4":
        g = grid(3, (512, 512, 512), (10.0, 10.0, 10.0), (64, 64, 64), 12)
        shape = field_shape(g)
        dt, nsteps, f0 = 0.8e-3, 1500, 15.0
        nz = shape[0]
        layer = np.minimum((np.arange(nz) * 4) // nz, 3)
        vlay = np.array([1800.0, 2867.0, 3933.0, 5000.0])[layer]
        pert = gaussian_random_field(shape, 10.0, 100.0, 5127, -1.0, 1.0)
        pert = pert - pert.mean()
        pert = pert / np.abs(pert).max()
        vp = vlay[:, None, None] * (1.0 + 0.05 * pert)
        vs = vp / math.sqrt(3.0)
        rho = 310.0 * vp ** 0.25
        rec = np.array([[256, 256, k] for k in range(0, 513, 8)], dtype=np.int32)
        shots = [{"sources": [_src(1, (2560.0, 2560.0, 1280.0), 20.0, f0, 1.2 / f0, dt, nsteps + 1)],
                  "receivers": rec, "rec_comp": 2}]
        w = dict(name=name, grid=g, physics=1, dt=dt, nsteps=nsteps, vp=vp, vs=vs, rho=rho,
                 shots=shots)
    elif name == "cfg5":
        nshots = over.pop("nshots", 64)
        g = grid(2, (1024, 0, 1024), (10.0, 10.0, 10.0), (128, 128, 128), 12)
        shape = field_shape(g)
        dt, nsteps, f0 = 1e-3, 3000, 15.0
        vp = gaussian_random_field(shape, 10.0, 200.0, 1, 1500.0, 4000.0)
        rho = np.full(shape, RHO_ACOUSTIC)
        rec = np.array([[ix, 0, 2] for ix in range(0, 1024)], dtype=np.int32)
        shots = [{"sources": [_src(0, ((8 + 16 * s) * 10.0, 0.0, 20.0), 20.0, f0, 1.2 / f0, dt,
                                   nsteps + 1)], "receivers": rec, "rec_comp": 0}
                 for s in range(nshots)]
        w = dict(name=name, grid=g, physics=0, dt=dt, nsteps=nsteps, vp=vp, vs=None, rho=rho,
                 shots=shots, ckpt_every=100)
    else:
        raise KeyError(name)
    w.update(over)
    return w


def _src(kind, pos, spread, f0, t0, dt, nt):
    """A source dict.  Stress sources (kind 0, 1) are sampled at mid-step times
    t_n + dt/2, forces (kinds 2..4) at integer times t_k."""
    shift = 0.5 if kind in (0, 1) else 0.0
    return {"kind": kind, "pos": tuple(float(p) for p in pos), "spread": float(spread),
            "wavelet": ricker(f0, t0, dt, nt, shift)}


def _rec_row(g, iz, step=1):
    nx = g["n"][0] + 1
    return np.array([[ix, 0, iz] for ix in range(0, nx, step)], dtype=np.int32)


def random_field(shape, seed, dtype=np.float64):
    """Unit-variance white noise (derivative parity inputs)."""
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)
