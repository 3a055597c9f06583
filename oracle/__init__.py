"""FP64 CPU oracle of the local spline simulator (arXiv 2301.05127).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py``; never by the product package.  It shares no code
with the HIP library.  The arithmetic lives in ``loss_oracle.c`` (plain C, double
precision); this module only marshals numpy arrays through ctypes.

Grids are plain dicts: ``{"ndim": 2|3, "n": (nx, ny, nz) intervals, "h": (hx, hy, hz),
"M": (Mx, My, Mz) patch intervals, "halo": n_nb, "end_mode": 0|1|2}``; for a 2-D grid
``n[1] == 0``.  Fields are numpy arrays of shape ``(nz+1, ny+1, nx+1)`` (3-D) or
``(nz+1, nx+1)`` (2-D), x fastest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "loss_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblossoracle.so")

END_NATURAL, END_PAPER_STENCIL, END_PERIODIC = 0, 1, 2
ACOUSTIC, ELASTIC = 0, 1
SRC_PRESSURE, SRC_EXPLOSIVE, SRC_FORCE_X, SRC_FORCE_Y, SRC_FORCE_Z = 0, 1, 2, 3, 4
A_SIGMA, A_V1, A_V3 = 0, 1, 2
E_V1, E_V2, E_V3, E_S11, E_S22, E_S33, E_S12, E_S13, E_S23 = range(9)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into an in-tree shared library."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "loss_oracle.h"))
    ):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
               _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double * 3),
                ("M", ctypes.c_int * 3), ("halo", ctypes.c_int), ("end_mode", ctypes.c_int)]


class _Pml(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int), ("R", ctypes.c_double), ("kmax", ctypes.c_double),
                ("f0", ctypes.c_double), ("cmax", ctypes.c_double)]


class _Source(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("pos", ctypes.c_double * 3), ("spread", ctypes.c_double),
                ("wavelet", ctypes.POINTER(ctypes.c_double)), ("nt", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load(build())
    return _lib


def build_variant(src_text: str, out_path: str) -> str:
    """Compile another text of ``loss_oracle.c`` (the pin tests plant a mistake in a copy
    to show that a pin catches it) into ``out_path``."""
    d = os.path.dirname(out_path)
    src = os.path.join(d, "loss_oracle_variant.c")
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-I", _HERE, src,
                           "-o", out_path, "-lm"])
    return out_path


class use_library:
    """Context manager: route every oracle call through the library at ``path``."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.prev = _lib
        _lib = _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.prev


def _load(path):
    """Open an oracle library and declare the signatures of its entry points."""
    L = ctypes.CDLL(path)
    D = ctypes.POINTER(ctypes.c_double)
    I = ctypes.POINTER(ctypes.c_int)
    G = ctypes.POINTER(_Grid)
    S = ctypes.POINTER(_Source)
    c_int, c_double = ctypes.c_int, ctypes.c_double
    sig = {
        "or_global_spline": (None, [c_int, c_double, D, D]),
        "or_global_inverse_column": (None, [c_int, c_double, c_int, D]),
        "or_patch_lu": (None, [c_int, D, D]),
        "or_pmbc_row": (c_int, [c_int, c_double, c_int, c_int, c_int, c_int, D, I]),
        "or_line_deriv": (None, [c_int, c_double, c_int, c_int, c_int, D, D, D]),
        "or_line_deriv_matrix": (None, [c_int, c_double, c_int, c_int, c_int, D]),
        "or_field_deriv": (None, [G, c_int, c_int, D, D]),
        "or_source_weights": (None, [G, D, c_double, D]),
        "or_run_from": (c_int, [G, c_int, c_double, c_int, c_int, D, D, D, c_int, S, c_int, I,
                                c_int, D, D, D]),
        "or_acoustic_adjoint": (c_int, [G, c_double, c_int, D, D, c_int, S, c_int, I, D, D]),
        "or_num_fields": (c_int, [c_int]),
        "or_pml_flow": (None, [c_double, c_double, c_double, c_double, c_double, c_double, D, D]),
        "or_run_pml": (c_int, [G, ctypes.POINTER(_Pml), c_double, c_int, c_int, D, D, c_int, S, c_int,
                               I, D, D, D]),
        "or_acoustic_adjoint_pml": (c_int, [G, ctypes.POINTER(_Pml), c_double, c_int, D, D, c_int, S, c_int, I,
                                            D, D]),
        "or_elastic_adjoint": (c_int, [G, c_double, c_int, D, D, D, c_int, S, c_int, I, c_int, D, D, D, D]),
        "or_run_pml_elastic": (c_int, [G, ctypes.POINTER(_Pml), c_double, c_int, c_int, D, D, D, c_int, S,
                                       c_int, I, c_int, D, D, D]),
        "or_elastic_adjoint_pml": (c_int, [G, ctypes.POINTER(_Pml), c_double, c_int, D, D, D, c_int, S, c_int, I,
                                           c_int, D, D, D, D]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _grid(g) -> _Grid:
    s = _Grid()
    s.ndim = int(g["ndim"])
    for a in range(3):
        s.n[a] = int(g["n"][a])
        s.h[a] = float(g["h"][a])
        s.M[a] = int(g["M"][a])
    s.halo = int(g["halo"])
    s.end_mode = int(g.get("end_mode", END_NATURAL))
    return s


def field_shape(g):
    n = g["n"]
    if g["ndim"] == 2:
        return (n[2] + 1, n[0] + 1)
    return (n[2] + 1, n[1] + 1, n[0] + 1)


# ---- 1-D ------------------------------------------------------------------

def global_spline(N, h, v):
    v = _f64(v)
    out = np.zeros(N + 3)
    lib().or_global_spline(N, h, _dp(v), _dp(out))
    return out


def global_inverse_column(N, h, k):
    out = np.zeros(N + 3)
    lib().or_global_inverse_column(N, h, k, _dp(out))
    return out


def patch_lu(M):
    d = np.zeros(M + 3)
    l = np.zeros(M + 2)
    lib().or_patch_lu(M, _dp(d), _dp(l))
    return d, l


def pmbc_row(N, h, M, halo, end_mode, J):
    c = np.zeros(2 * halo + 1)
    idx = np.zeros(2 * halo + 1, dtype=np.int32)
    has = lib().or_pmbc_row(N, h, M, halo, end_mode, J, _dp(c), _ip(idx))
    return bool(has), c, idx


def line_deriv(N, h, M, halo, end_mode, u):
    u = _f64(u)
    d1 = np.zeros(N + 1)
    d2 = np.zeros(N + 1)
    lib().or_line_deriv(N, h, M, halo, end_mode, _dp(u), _dp(d1), _dp(d2))
    return d1, d2


def line_deriv_matrix(N, h, M, halo, end_mode):
    D = np.zeros((N + 1, N + 1))
    lib().or_line_deriv_matrix(N, h, M, halo, end_mode, _dp(D))
    return D


# ---- fields ---------------------------------------------------------------

def field_deriv(g, axis, order, field):
    f = _f64(field)
    out = np.zeros_like(f)
    gs = _grid(g)
    lib().or_field_deriv(ctypes.byref(gs), axis, order, _dp(f), _dp(out))
    return out


def source_weights(g, pos, spread):
    out = np.zeros(field_shape(g))
    gs = _grid(g)
    p = _f64(list(pos) + [0.0] * (3 - len(pos)))
    lib().or_source_weights(ctypes.byref(gs), _dp(p), float(spread), _dp(out))
    return out


def _sources(sources):
    """sources: list of dicts {kind, pos (3), spread, wavelet (1-D array)}."""
    keep = []
    arr = (_Source * max(1, len(sources)))()
    for i, s in enumerate(sources):
        w = _f64(s["wavelet"])
        keep.append(w)
        arr[i].kind = int(s["kind"])
        for a in range(3):
            arr[i].pos[a] = float(s["pos"][a])
        arr[i].spread = float(s.get("spread", 0.0))
        arr[i].wavelet = _dp(w)
        arr[i].nt = int(w.size)
    return arr, keep


def run(g, physics, dt, nsteps, vp, rho, vs=None, sources=(), receivers=None, rec_comp=0,
        fields_in=None, step0=0):
    """Run one shot; returns (fields (nfields, *shape), traces (nrec, nsteps))."""
    shape = field_shape(g)
    nf = 3 if physics == ACOUSTIC else 9
    vp = _f64(vp)
    rho = _f64(rho)
    vs = _f64(vs) if vs is not None else None
    src, keep = _sources(list(sources))
    rec = np.zeros((0, 3), dtype=np.int32) if receivers is None else np.ascontiguousarray(receivers, dtype=np.int32)
    nrec = rec.shape[0]
    fields = np.zeros((nf,) + shape)
    traces = np.zeros((nrec, nsteps))
    fin = _f64(fields_in) if fields_in is not None else None
    if fin is not None and fin.shape != fields.shape:
        raise ValueError("fields_in must have shape %s" % (fields.shape,))
    gs = _grid(g)
    rc = lib().or_run_from(ctypes.byref(gs), physics, float(dt), int(step0), int(nsteps), _dp(vp),
                           _dp(vs), _dp(rho), len(keep), src, nrec, _ip(rec), int(rec_comp),
                           _dp(fin), _dp(fields), _dp(traces))
    if rc != 0:
        raise ValueError("oracle or_run_from rejected its arguments (rc=%d)" % rc)
    return fields, traces


def pml_flow(d, k, alpha, tau, D, psi):
    """Exact flow of one ADE-PML memory variable and its field over tau with the
    derivative D frozen (Sec. 3.3); returns (psi(tau), (v(tau) - v(0)) / b)."""
    po, dv = ctypes.c_double(), ctypes.c_double()
    lib().or_pml_flow(float(d), float(k), float(alpha), float(tau), float(D), float(psi),
                      ctypes.byref(po), ctypes.byref(dv))
    return po.value, dv.value


def run_pml(g, pml, dt, nsteps, vp, rho, sources=(), receivers=None, fields_in=None, step0=0):
    """Acoustic 2-D run with the ADE-PML layer (Sec. 3.3).  pml: dict(width, R, kmax, f0,
    cmax).  Returns (fields (7, *shape): sigma, v1, v3, psi_x, psi_z, phi_x, phi_z,
    traces (nrec, nsteps) of sigma)."""
    shape = field_shape(g)
    vp = _f64(vp)
    rho = _f64(rho)
    src, keep = _sources(list(sources))
    rec = np.zeros((0, 3), dtype=np.int32) if receivers is None else np.ascontiguousarray(receivers, dtype=np.int32)
    fields = np.zeros((7,) + shape)
    traces = np.zeros((rec.shape[0], nsteps))
    fin = _f64(fields_in) if fields_in is not None else None
    if fin is not None and fin.shape != fields.shape:
        raise ValueError("fields_in must have shape %s (sigma, v1, v3 and four memory variables)" % (fields.shape,))
    p = _Pml(int(pml["width"]), float(pml["R"]), float(pml["kmax"]), float(pml["f0"]), float(pml["cmax"]))
    gs = _grid(g)
    rc = lib().or_run_pml(ctypes.byref(gs), ctypes.byref(p), float(dt), int(step0), int(nsteps), _dp(vp), _dp(rho),
                          len(keep), src, rec.shape[0], _ip(rec), _dp(fin), _dp(fields), _dp(traces))
    if rc != 0:
        raise ValueError("oracle or_run_pml rejected its arguments (rc=%d)" % rc)
    return fields, traces


def run_pml_elastic(g, pml, dt, nsteps, vp, vs, rho, sources=(), receivers=None, rec_comp=0, fields_in=None,
                    step0=0):
    """Elastic 3-D run with the ADE-PML layer on all three axes (Sec. 3.3, applied to
    every derivative of the elastic system).  pml: dict(width, R, kmax, f0, cmax).
    Returns (fields (27, *shape): the 9 elastic fields, psi[3i + j] of d_j sigma_ij,
    phi[3i + j] of d_j v_i; traces (nrec, nsteps) of field rec_comp)."""
    shape = field_shape(g)
    vp, vs, rho = _f64(vp), _f64(vs), _f64(rho)
    src, keep = _sources(list(sources))
    rec = np.zeros((0, 3), dtype=np.int32) if receivers is None else np.ascontiguousarray(receivers, dtype=np.int32)
    fields = np.zeros((27,) + shape)
    traces = np.zeros((rec.shape[0], nsteps))
    fin = _f64(fields_in) if fields_in is not None else None
    if fin is not None and fin.shape != fields.shape:
        raise ValueError("fields_in must have shape %s (9 fields and 18 memory variables)" % (fields.shape,))
    p = _Pml(int(pml["width"]), float(pml["R"]), float(pml["kmax"]), float(pml["f0"]), float(pml["cmax"]))
    gs = _grid(g)
    rc = lib().or_run_pml_elastic(ctypes.byref(gs), ctypes.byref(p), float(dt), int(step0), int(nsteps), _dp(vp),
                                  _dp(vs), _dp(rho), len(keep), src, rec.shape[0], _ip(rec), int(rec_comp),
                                  _dp(fin), _dp(fields), _dp(traces))
    if rc != 0:
        raise ValueError("oracle or_run_pml_elastic rejected its arguments (rc=%d)" % rc)
    return fields, traces


def acoustic_adjoint(g, dt, nsteps, vp, rho, sources, receivers, residual):
    """Gradient dJ/dK (K = rho c^2) at every node for J = 1/2 sum residual^2."""
    shape = field_shape(g)
    vp = _f64(vp)
    rho = _f64(rho)
    src, keep = _sources(list(sources))
    rec = np.ascontiguousarray(receivers, dtype=np.int32)
    res = _f64(residual)
    grad = np.zeros(shape)
    gs = _grid(g)
    rc = lib().or_acoustic_adjoint(ctypes.byref(gs), float(dt), int(nsteps), _dp(vp), _dp(rho),
                                   len(keep), src, rec.shape[0], _ip(rec), _dp(res), _dp(grad))
    if rc != 0:
        raise ValueError("oracle or_acoustic_adjoint rejected its arguments (rc=%d)" % rc)
    return grad


def acoustic_adjoint_pml(g, pml, dt, nsteps, vp, rho, sources, receivers, residual):
    """Gradient dJ/dK at every node of a run with the ADE-PML layer (pml: dict(width, R,
    kmax, f0, cmax)) for J = 1/2 sum residual^2 of the sigma traces."""
    shape = field_shape(g)
    vp, rho = _f64(vp), _f64(rho)
    src, keep = _sources(list(sources))
    rec = np.ascontiguousarray(receivers, dtype=np.int32)
    res = _f64(residual)
    grad = np.zeros(shape)
    p = _Pml(int(pml["width"]), float(pml["R"]), float(pml["kmax"]), float(pml["f0"]), float(pml["cmax"]))
    gs = _grid(g)
    rc = lib().or_acoustic_adjoint_pml(ctypes.byref(gs), ctypes.byref(p), float(dt), int(nsteps), _dp(vp), _dp(rho),
                                       len(keep), src, rec.shape[0], _ip(rec), _dp(res), _dp(grad))
    if rc != 0:
        raise ValueError("oracle or_acoustic_adjoint_pml rejected its arguments (rc=%d)" % rc)
    return grad


def elastic_adjoint(g, dt, nsteps, vp, vs, rho, sources, receivers, rec_comp, residual, with_b=False):
    """Gradients (dJ/dlambda, dJ/dmu) at every node for J = 1/2 sum residual^2 of the
    traces of field rec_comp; with_b: also dJ/db (b = 1/rho, lambda and mu fixed)."""
    shape = field_shape(g)
    vp, vs, rho = _f64(vp), _f64(vs), _f64(rho)
    src, keep = _sources(list(sources))
    rec = np.ascontiguousarray(receivers, dtype=np.int32)
    res = _f64(residual)
    gl, gm = np.zeros(shape), np.zeros(shape)
    gb = np.zeros(shape) if with_b else None
    gs = _grid(g)
    rc = lib().or_elastic_adjoint(ctypes.byref(gs), float(dt), int(nsteps), _dp(vp), _dp(vs), _dp(rho),
                                  len(keep), src, rec.shape[0], _ip(rec), int(rec_comp), _dp(res), _dp(gl),
                                  _dp(gm), _dp(gb))
    if rc != 0:
        raise ValueError("oracle or_elastic_adjoint rejected its arguments (rc=%d)" % rc)
    return (gl, gm, gb) if with_b else (gl, gm)


def elastic_adjoint_pml(g, pml, dt, nsteps, vp, vs, rho, sources, receivers, rec_comp, residual, with_b=False):
    """Gradients (dJ/dlambda, dJ/dmu[, dJ/db]) of a run with the ADE-PML layer on every
    axis (pml: dict(width, R, kmax, f0, cmax)) for J = 1/2 sum residual^2 of the traces of
    field rec_comp (the transpose of run_pml_elastic's sequence, Sec. 3.3)."""
    shape = field_shape(g)
    vp, vs, rho = _f64(vp), _f64(vs), _f64(rho)
    src, keep = _sources(list(sources))
    rec = np.ascontiguousarray(receivers, dtype=np.int32)
    res = _f64(residual)
    gl, gm = np.zeros(shape), np.zeros(shape)
    gb = np.zeros(shape) if with_b else None
    p = _Pml(int(pml["width"]), float(pml["R"]), float(pml["kmax"]), float(pml["f0"]), float(pml["cmax"]))
    gs = _grid(g)
    rc = lib().or_elastic_adjoint_pml(ctypes.byref(gs), ctypes.byref(p), float(dt), int(nsteps), _dp(vp), _dp(vs),
                                      _dp(rho), len(keep), src, rec.shape[0], _ip(rec), int(rec_comp), _dp(res),
                                      _dp(gl), _dp(gm), _dp(gb))
    if rc != 0:
        raise ValueError("oracle or_elastic_adjoint_pml rejected its arguments (rc=%d)" % rc)
    return (gl, gm, gb) if with_b else (gl, gm)


def energy(g, physics, fields, vp, rho, vs=None):
    """Wavefield energy (the velocity-stress system of Sec. 2): the sum over the nodes of
    1/2 rho |v|^2 + 1/2 sigma . epsilon, epsilon = C^-1 sigma, times the cell volume.
    fields: acoustic (sigma, v1, v3), elastic (v1, v2, v3, s11, s22, s33, s12, s13, s23),
    each of the grid's shape.  The strain is found by solving the isotropic stiffness
    system in Voigt form (normal rows lambda + 2 mu on the diagonal, lambda off it; shear
    rows mu acting on the engineering strain 2 eps_ij) at every node; acoustic: sigma / K.
    Plain FP64 numpy."""
    f = _f64(fields)
    rho = _f64(rho)
    vp = _f64(vp)
    gg = _grid(g)
    cell = gg.h[0] * gg.h[2] * (gg.h[1] if gg.ndim == 3 else 1.0)
    if physics == 0:
        K = rho * vp ** 2
        e = 0.5 * rho * (f[1] ** 2 + f[2] ** 2) + 0.5 * f[0] ** 2 / K
        return float(np.sum(e) * cell)
    vs = _f64(vs)
    mu = rho * vs ** 2
    lam = rho * vp ** 2 - 2.0 * mu
    n = rho.size
    C = np.zeros((n, 6, 6))
    for i in range(3):
        for j in range(3):
            C[:, i, j] = lam.ravel() + (2.0 * mu.ravel() if i == j else 0.0)
        C[:, 3 + i, 3 + i] = mu.ravel()
    sig = np.stack([f[3 + k].ravel() for k in range(6)], axis=1)        # s11 s22 s33 s12 s13 s23
    strain = np.linalg.solve(C, sig[:, :, None])[:, :, 0]               # eps11..33, 2 eps12..
    e = 0.5 * rho.ravel() * (f[0].ravel() ** 2 + f[1].ravel() ** 2 + f[2].ravel() ** 2) \
        + 0.5 * np.sum(sig * strain, axis=1)
    return float(np.sum(e) * cell)


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / den) if den > 0 else float(np.linalg.norm(x - ref))
