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
