"""The C-ABI library: it loads, exports every entry point the header declares,
and its argument checks and failure paths behave without a GPU.  No compute
call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hull2d.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hull2d_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_1508_05931_amd as hx
    if not os.path.exists(hx.LIB_PATH):
        pytest.fail("libhull2d.so is not built (run __graft_entry__.build())")
    return hx.load_library()


def test_header_declares_the_interface():
    names = _declared()
    for want in ["hull2d_create", "hull2d_compute", "hull2d_batch", "hull2d_destroy",
                 "hull2d_status_string"]:
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_the_exports():
    import paper_1508_05931_amd as hx
    assert sorted(hx.EXPORTED) == _declared()


def test_status_strings(lib):
    for s in range(9):
        assert lib.hull2d_status_string(s)
    assert lib.hull2d_status_string(2) == b"non-finite coordinate"


def test_argument_checks_without_device(lib):
    # null out-pointer
    assert lib.hull2d_create(None, 0, None, None) == 1
    # invalid context / arguments are rejected before any device work
    n_out = ctypes.c_int64(0)
    assert lib.hull2d_compute(None, None, 0, None, 0, ctypes.byref(n_out), None) == 1
    h = ctypes.c_void_p()
    st = lib.hull2d_create(ctypes.byref(h), 0, None, None)
    import torch
    if torch.cuda.is_available():
        assert st == 0
        lib.hull2d_destroy(h)
    else:
        assert st in (1, 6)   # no device: an error code, never a crash


def test_product_path_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_1508_05931_amd as hx
    monkeypatch.setattr(hx, "_lib", None)
    monkeypatch.setattr(hx, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        hx.load_library()


def test_shipped_batch_schedule_is_valid():
    """The autotuner's stored schedule names options the library accepts,
    and the binding's option struct has the header's size."""
    import paper_1508_05931_amd as hx
    if not os.path.exists(hx.TUNING):
        pytest.skip("no tuned schedule in the tree")
    t = hx.tuned_batch_schedule()
    assert t["batch_blocks_per_cu"] in (1, 2) and t["batch_order"] in (0, 1, 2)
    # uint32 struct_size and twelve int32 fields, as hull2d_options
    assert ctypes.sizeof(hx._Options) == 4 + 12 * 4
