"""CPU checks of the C ABI boundary: the library exists, loads, and exports every
function include/loss.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "loss.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(loss_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("loss_create", "loss_destroy", "loss_set_media", "loss_add_source",
                     "loss_add_receivers", "loss_step", "loss_get_field", "loss_get_traces",
                     "loss_deriv", "loss_forward_ckpt", "loss_adjoint"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2301_05127_amd import loss
    assert os.path.exists(loss.LIB_PATH), "libloss.so must be built in-tree"
    L = ctypes.CDLL(loss.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert sorted(loss.EXPORTS) == declared_functions()


def test_status_strings_without_gpu():
    from paper_2301_05127_amd import loss
    L = loss.lib()
    assert L.loss_status_str(0) == b"ok"
    assert L.loss_status_str(-6) == b"unstable"


def test_desc_layout_matches_header():
    # offsets of loss_desc as laid out by a C compiler (int32, int32, int64[3], double[3],
    # double, int32[3], int32 x4, int64)
    from paper_2301_05127_amd.loss import Desc
    assert Desc.n.offset == 8 and Desc.h.offset == 32 and Desc.dt.offset == 56
    assert Desc.patch.offset == 64 and Desc.flags.offset == 88 and Desc.trace_len.offset == 96
    assert ctypes.sizeof(Desc) == 104


def _desc(**kw):
    from paper_2301_05127_amd.loss import Desc
    d = Desc()
    d.physics, d.ndim = 0, 2
    for a, (n, h, m) in enumerate([(64, 10.0, 32), (0, 10.0, 32), (64, 10.0, 32)]):
        d.n[a], d.h[a], d.patch[a] = n, h, m
    d.dt, d.halo, d.end_mode, d.nshots, d.flags, d.trace_len = 1e-3, 8, 0, 1, 0, 0
    for k, v in kw.items():
        if k in ("n", "h", "patch"):
            for a, x in enumerate(v):
                getattr(d, k)[a] = x
        else:
            setattr(d, k, v)
    return d


import pytest  # noqa: E402


@pytest.mark.parametrize("kw,needle", [
    (dict(ndim=3), "acoustic physics is 2-D"),
    (dict(physics=1), "elastic physics is 3-D"),
    (dict(physics=7), "unknown physics"),
    (dict(nshots=0), "nshots"),
    (dict(dt=0.0), "dt must be positive"),
    (dict(trace_len=-1), "trace_len"),
    (dict(n=(64, 5, 64)), "n[1] == 0"),
    (dict(halo=0), "halo must be in 1..64"),
    (dict(halo=65), "halo must be in 1..64"),
    (dict(n=(1, 0, 64)), "at least 2 intervals"),
    (dict(patch=(0, 32, 32)), "patch length"),
    (dict(end_mode=2, halo=40), "periodic axis needs"),
    (dict(end_mode=5), "unknown end mode"),
    (dict(h=(0.0, 10.0, 10.0)), "spacing"),
])
def test_create_rejects_bad_descriptions(kw, needle):
    """Invalid descriptions are rejected with LOSS_EINVAL before any device call."""
    import ctypes as C
    from paper_2301_05127_amd import loss
    L = loss.lib()
    d = _desc(**kw)
    h = C.c_void_p()
    st = L.loss_create(C.byref(d), None, C.byref(h))
    assert st == -1, (st, L.loss_last_error())
    assert needle in L.loss_last_error().decode(), L.loss_last_error()
    assert not h.value


def test_create_refuses_fields_past_32bit_indexing():
    """A per-shot field of 2^31 or more (padded) elements is refused with
    LOSS_EUNSUPPORTED before any device call (the line kernels index within a shot's
    field in 32-bit arithmetic)."""
    import ctypes as C
    from paper_2301_05127_amd import loss
    L = loss.lib()
    h = C.c_void_p()
    # 1292 x 1291 x 1291 padded nodes = 2.15e9 elements
    d = _desc(physics=1, ndim=3, n=(1290, 1290, 1290), patch=(64, 64, 64))
    assert L.loss_create(C.byref(d), None, C.byref(h)) == -5, L.loss_last_error()
    assert b"2^31" in L.loss_last_error()
    assert not h.value


def test_null_arguments():
    import ctypes as C
    from paper_2301_05127_amd import loss
    L = loss.lib()
    assert L.loss_create(None, None, None) == -1
    assert L.loss_destroy(None) == 0
    assert L.loss_step(None, 1) == -1
    assert L.loss_current_step(None) == -1


def test_autograd_wrapper_rejects_host_model():
    """The autograd view runs only on device tensors; a host model is refused before any
    library call."""
    import torch
    from paper_2301_05127_amd import autograd
    m = torch.ones((5, 5), dtype=torch.float64, requires_grad=True)
    with pytest.raises(ValueError, match="CUDA"):
        autograd.seismograms(None, m, torch.ones((5, 5)), 3)


def test_elastic_autograd_wrapper_rejects_host_model_and_bad_param():
    import torch
    from paper_2301_05127_amd import autograd, loss
    a = torch.ones((3, 3, 3), dtype=torch.float64, requires_grad=True)
    with pytest.raises(ValueError, match="CUDA"):
        autograd.elastic_seismograms(None, a, a, torch.ones((3, 3, 3)), 3)
    with pytest.raises(ValueError, match="GRAD_VPVS"):
        autograd.elastic_seismograms(None, a, a, torch.ones((3, 3, 3)), 3, param=loss.GRAD_VP)


@pytest.mark.parametrize("kw", [dict(patch=(4, 4, 4), halo=9), dict(patch=(4, 4, 4), halo=12),
                                dict(patch=(8, 8, 8), halo=20), dict(patch=(3, 3, 3), halo=30)])
def test_create_accepts_halos_wider_than_the_patches(kw):
    """A PMBC halo wider than the patches (Sec. 3.2 lets n_nb exceed M) passes the
    description checks and the table build: whatever loss_create then returns here, where
    no GPU is visible, it is not LOSS_EINVAL."""
    import ctypes as C
    from paper_2301_05127_amd import loss
    L = loss.lib()
    d = _desc(**kw)
    h = C.c_void_p()
    st = L.loss_create(C.byref(d), None, C.byref(h))
    if st == 0:
        L.loss_destroy(h)
    assert st != -1, L.loss_last_error()
