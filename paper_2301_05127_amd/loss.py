"""ctypes binding of libloss.so (include/loss.h): argument marshalling only.

Every step of the simulator runs in the HIP library; this module converts numpy
arrays / torch tensors into pointers and status codes into exceptions.  It raises
``LossLibraryMissing`` when the built library is absent (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LOSS_LIBRARY names another build of the same library (A/B timing of kernel variants)
LIB_PATH = os.environ.get("LOSS_LIBRARY", os.path.join(_HERE, "libloss.so"))

ACOUSTIC, ELASTIC = 0, 1
END_NATURAL, END_PAPER_STENCIL, END_PERIODIC = 0, 1, 2
MEM_HOST, MEM_DEVICE = 0, 1
F_SIGMA, F_V1, F_V3 = 0, 1, 2
F_EV1, F_EV2, F_EV3, F_S11, F_S22, F_S33, F_S12, F_S13, F_S23 = range(9)
SRC_PRESSURE, SRC_EXPLOSIVE, SRC_FORCE_X, SRC_FORCE_Y, SRC_FORCE_Z = range(5)
FLAG_NO_GRAPH = 1
FLAG_NO_FUSE_X = 2
FLAG_LINE_PASSES = 4
GRAD_K, GRAD_VP, GRAD_LAME, GRAD_VPVS, GRAD_LAME_RHO, GRAD_VPVS_RHO = 0, 1, 2, 3, 4, 5

EXPORTS = [
    "loss_create", "loss_destroy", "loss_set_media", "loss_add_source", "loss_add_receivers",
    "loss_reset", "loss_step", "loss_get_field", "loss_set_field", "loss_get_traces", "loss_deriv",
    "loss_forward_ckpt", "loss_adjoint", "loss_sync", "loss_energy", "loss_set_timing", "loss_kernel_timing",
    "loss_current_step", "loss_status_str", "loss_last_error", "loss_autotune",
    "loss_autotune_choice", "loss_set_shape", "loss_set_pml", "loss_deriv_static",
]


class LossLibraryMissing(RuntimeError):
    pass


class LossError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (_status_str(status), status, msg))
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [("physics", ctypes.c_int32), ("ndim", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
                ("h", ctypes.c_double * 3), ("dt", ctypes.c_double), ("patch", ctypes.c_int32 * 3),
                ("halo", ctypes.c_int32), ("end_mode", ctypes.c_int32), ("nshots", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("trace_len", ctypes.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LossLibraryMissing("libloss.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sigs = {
        "loss_create": (I32, [ctypes.POINTER(Desc), P, ctypes.POINTER(P)]),
        "loss_destroy": (I32, [P]),
        "loss_set_media": (I32, [P, P, P, P, I32]),
        "loss_add_source": (I32, [P, I32, ctypes.POINTER(D), I32, P, I64, D]),
        "loss_add_receivers": (I32, [P, I32, I64, P, I32]),
        "loss_reset": (I32, [P]),
        "loss_step": (I32, [P, I64]),
        "loss_get_field": (I32, [P, I32, I32, P, I32]),
        "loss_set_field": (I32, [P, I32, I32, P, I32]),
        "loss_get_traces": (I32, [P, I32, P, I32]),
        "loss_deriv": (I32, [P, I32, I32, P, P, I64, I32]),
        "loss_deriv_static": (I32, [P, I32, I32, P, P, I64]),
        "loss_forward_ckpt": (I32, [P, I64, I64]),
        "loss_adjoint": (I32, [P, P, I32, P, I32]),
        "loss_sync": (I32, [P]),
        "loss_energy": (I32, [P, P]),
        "loss_set_timing": (I32, [P, I32]),
        "loss_kernel_timing": (I32, [P, I32, ctypes.POINTER(D), ctypes.POINTER(I64),
                                     ctypes.POINTER(ctypes.c_char_p)]),
        "loss_current_step": (I64, [P]),
        "loss_autotune": (I32, [P, I32]),
        "loss_autotune_choice": (I32, [P, I32, ctypes.POINTER(I32)]),
        "loss_set_shape": (I32, [P, I32, I32]),
        "loss_set_pml": (I32, [P, I32, D, D, D]),
        "loss_status_str": (ctypes.c_char_p, [I32]),
        "loss_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _status_str(s):
    try:
        return lib().loss_status_str(s).decode()
    except Exception:
        return "status"


def _check(status):
    if status != 0:
        raise LossError(status, lib().loss_last_error().decode())


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype):
    """(pointer, mem, keepalive) for a numpy array or a torch tensor."""
    if _is_torch(x):
        import torch
        want = {np.float32: torch.float32, np.float64: torch.float64, np.int32: torch.int32}[dtype]
        if x.dtype != want or not x.is_contiguous():
            raise TypeError("tensor must be contiguous %s" % want)
        mem = MEM_DEVICE if x.is_cuda else MEM_HOST
        return ctypes.c_void_p(x.data_ptr()), mem, x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data_as(ctypes.c_void_p), MEM_HOST, a


class Simulation:
    """One simulation handle (a batch of shots on one grid and one medium)."""

    def __init__(self, grid, physics, dt, nshots=1, trace_len=0, flags=0):
        d = Desc()
        d.physics = physics
        d.ndim = grid["ndim"]
        for a in range(3):
            d.n[a] = grid["n"][a]
            d.h[a] = grid["h"][a]
            d.patch[a] = grid["M"][a]
        d.dt = dt
        d.halo = grid["halo"]
        d.end_mode = grid.get("end_mode", 0)
        d.nshots = nshots
        d.flags = flags
        d.trace_len = trace_len
        self.grid = grid
        self.physics = physics
        self.nshots = nshots
        self.trace_len = trace_len
        self.nfields = 3 if physics == ACOUSTIC else 9
        self._nrec = [0] * nshots
        n = grid["n"]
        self.shape = (n[2] + 1, n[0] + 1) if grid["ndim"] == 2 else (n[2] + 1, n[1] + 1, n[0] + 1)
        self.nodes = int(np.prod(self.shape))
        h = ctypes.c_void_p()
        _check(lib().loss_create(ctypes.byref(d), None, ctypes.byref(h)))
        self._h = h

    # ---- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().loss_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- setup ----------------------------------------------------------------
    def set_media(self, vp, rho, vs=None):
        pv, mem, k1 = _ptr(vp, np.float32)
        pr, _, k2 = _ptr(rho, np.float32)
        ps, _, k3 = (None, None, None) if vs is None else _ptr(vs, np.float32)
        _check(lib().loss_set_media(self._h, pv, ps, pr, mem))

    def add_source(self, shot, kind, pos, wavelet, spread=0.0):
        w = np.ascontiguousarray(wavelet, dtype=np.float32)
        p = (ctypes.c_double * 3)(*[float(v) for v in (list(pos) + [0.0] * (3 - len(pos)))])
        _check(lib().loss_add_source(self._h, shot, p, kind, w.ctypes.data_as(ctypes.c_void_p), w.size,
                                     float(spread)))

    def add_receivers(self, shot, idx, component=0):
        a = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 3)
        _check(lib().loss_add_receivers(self._h, shot, a.shape[0], a.ctypes.data_as(ctypes.c_void_p),
                                        component))
        self._nrec[shot] = a.shape[0]

    def setup_workload(self, w, shots=None):
        """Media, sources and receivers of an inputs.config workload."""
        self.set_media(w["vp"], w["rho"], w.get("vs"))
        for s, sh in enumerate(w["shots"] if shots is None else shots):
            for src in sh["sources"]:
                self.add_source(s, src["kind"], src["pos"], src["wavelet"], src.get("spread", 0.0))
            if sh.get("receivers") is not None and self.trace_len > 0:
                self.add_receivers(s, sh["receivers"], sh.get("rec_comp", 0))

    # ---- running --------------------------------------------------------------
    def reset(self):
        _check(lib().loss_reset(self._h))

    def set_pml(self, width, reflection=1e-6, kmax=1.0, f0=15.0):
        """Absorbing layer of `width` nodes on both ends of every axis (acoustic or
        elastic; see loss_set_pml).  Call after the media are set; width 0 removes it."""
        _check(lib().loss_set_pml(self._h, int(width), float(reflection), float(kmax), float(f0)))

    def step(self, n=1):
        _check(lib().loss_step(self._h, int(n)))

    def sync(self):
        _check(lib().loss_sync(self._h))

    def energy(self):
        """Wavefield energy of every shot at the state's time (FP64, reduced on the device)."""
        out = np.zeros(self.nshots, dtype=np.float64)
        _check(lib().loss_energy(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    @property
    def current_step(self):
        return int(lib().loss_current_step(self._h))

    def get_field(self, field, shot=0, out=None):
        if out is None:
            out = np.empty(self.shape, dtype=np.float32)
        p, mem, keep = _ptr(out, np.float32)
        _check(lib().loss_get_field(self._h, shot, field, p, mem))
        if mem == MEM_DEVICE:
            self.sync()
        return out

    def set_field(self, field, data, shot=0):
        p, mem, keep = _ptr(data, np.float32)
        _check(lib().loss_set_field(self._h, shot, field, p, mem))
        self.sync()

    def get_traces(self, shot=0):
        out = np.zeros((self._nrec[shot], self.trace_len), dtype=np.float64)
        if out.size:
            _check(lib().loss_get_traces(self._h, shot, out.ctypes.data_as(ctypes.c_void_p), MEM_HOST))
        return out

    def deriv(self, axis, order, data):
        """Patched spline derivative of a batch of fields (batch, *shape) along axis."""
        if _is_torch(data):
            import torch
            out = torch.empty_like(data)
            pi, mem, k1 = _ptr(data, np.float32)
            po, _, k2 = _ptr(out, np.float32)
            batch = data.numel() // self.nodes
            _check(lib().loss_deriv(self._h, axis, order, pi, po, batch, mem))
            self.sync()
            return out
        a = np.ascontiguousarray(data, dtype=np.float32)
        out = np.empty_like(a)
        batch = a.size // self.nodes
        _check(lib().loss_deriv(self._h, axis, order, a.ctypes.data_as(ctypes.c_void_p),
                                out.ctypes.data_as(ctypes.c_void_p), batch, MEM_HOST))
        return out

    def deriv_static(self, axis, order, data, out=None):
        """loss_deriv on a CUDA tensor (batch, *shape) through the library-static device
        scratch (allocates nothing in the library); returns `out` (a new tensor unless
        given) after synchronising the simulation stream."""
        import torch
        if out is None:
            out = torch.empty_like(data)
        pi, mem, k1 = _ptr(data, np.float32)
        po, mem2, k2 = _ptr(out, np.float32)
        if mem != MEM_DEVICE or mem2 != MEM_DEVICE:
            raise TypeError("deriv_static takes CUDA tensors")
        torch.cuda.current_stream(data.device).synchronize()
        _check(lib().loss_deriv_static(self._h, axis, order, pi, po, data.numel() // self.nodes))
        self.sync()
        return out

    # ---- gradient ----------------------------------------------------------------
    def forward_ckpt(self, nsteps, ckpt_every):
        _check(lib().loss_forward_ckpt(self._h, int(nsteps), int(ckpt_every)))

    def adjoint(self, residual, param=None):
        """Gradient of sum(residual * traces) over the run of the last forward_ckpt:
        acoustic with respect to K or c (GRAD_K, GRAD_VP, default GRAD_VP; shape of a
        field), elastic with respect to (lambda, mu) or (vp, vs) (GRAD_LAME, GRAD_VPVS,
        default GRAD_VPVS; shape (2, *field)), or those and rho (GRAD_LAME_RHO,
        GRAD_VPVS_RHO; shape (3, *field)).  residual [S][nrec][nt] FP64: a host array
        (the gradient comes back as a numpy array) or a contiguous CUDA tensor (the
        gradient is a CUDA tensor)."""
        elastic = self.physics == ELASTIC
        if param is None:
            param = GRAD_VPVS if elastic else GRAD_VP
        gshape = (((3,) if param in (GRAD_LAME_RHO, GRAD_VPVS_RHO) else (2,)) if elastic else ()) + tuple(self.shape)
        if _is_torch(residual) and residual.is_cuda:
            import torch
            if residual.dtype != torch.float64 or not residual.is_contiguous():
                raise TypeError("residual must be a contiguous float64 tensor")
            g = torch.empty(gshape, dtype=torch.float64, device=residual.device)
            # the library runs on its own stream: the residual must be complete first
            torch.cuda.current_stream(residual.device).synchronize()
            _check(lib().loss_adjoint(self._h, ctypes.c_void_p(residual.data_ptr()), param,
                                      ctypes.c_void_p(g.data_ptr()), MEM_DEVICE))
            return g
        r = np.ascontiguousarray(residual, dtype=np.float64)
        g = np.zeros(gshape, dtype=np.float64)
        _check(lib().loss_adjoint(self._h, r.ctypes.data_as(ctypes.c_void_p), param,
                                  g.ctypes.data_as(ctypes.c_void_p), MEM_HOST))
        return g

    def traces_tensor(self, device):
        """Traces of every shot as one CUDA tensor [S][nrec][trace_len] (FP64); shots must
        have equal receiver counts."""
        import torch
        if len(set(self._nrec)) != 1:
            raise ValueError("shots have different receiver counts")
        out = torch.empty((len(self._nrec), self._nrec[0], self.trace_len), dtype=torch.float64, device=device)
        torch.cuda.current_stream(out.device).synchronize()
        for s in range(len(self._nrec)):
            if out[s].numel():
                _check(lib().loss_get_traces(self._h, s, ctypes.c_void_p(out[s].data_ptr()), MEM_DEVICE))
        self.sync()
        return out

    # ---- launch-shape autotuning ----------------------------------------------------
    def autotune(self, trial_steps=5):
        """Pick the fastest launch shape of the line kernels (and, elastic, the faster of
        the plane and line-pass schedules); returns the choice per axis (loss_set_shape
        encoding), then, when elastic, the schedule (0 plane, 1 line passes) and the
        shapes of the y and z store passes (0: the axis's)."""
        _check(lib().loss_autotune(self._h, int(trial_steps)))
        out = []
        for axis in range(6 if self.physics == ELASTIC else 3):
            v = ctypes.c_int32()
            _check(lib().loss_autotune_choice(self._h, axis, ctypes.byref(v)))
            out.append(v.value)
        return out

    def set_shape(self, shapes):
        """Set the launch shape per axis (see loss_set_shape; a fourth entry is the elastic
        schedule, 0 plane passes, 1 line passes, a fifth and sixth the shapes of the y and
        z store passes); None entries are skipped."""
        for axis, v in enumerate(shapes):
            if v is None or (axis == 1 and self.grid["ndim"] == 2):
                continue
            _check(lib().loss_set_shape(self._h, axis, int(v)))

    # ---- timing ----------------------------------------------------------------
    def set_timing(self, on):
        _check(lib().loss_set_timing(self._h, 1 if on else 0))

    def kernel_timing(self):
        out = []
        i = 0
        while True:
            ms = ctypes.c_double()
            cnt = ctypes.c_int64()
            name = ctypes.c_char_p()
            st = lib().loss_kernel_timing(self._h, i, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(name))
            if st != 0:
                break
            out.append((name.value.decode(), ms.value, cnt.value))
            i += 1
        return out
