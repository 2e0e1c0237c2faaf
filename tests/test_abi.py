"""The C-ABI library: it loads, exports every entry point the header declares,
and its argument checks and failure paths behave without a GPU.  No compute
call is made here."""
import ctypes
import os
import re
import subprocess

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
    tile = t.get("batch_tile", 0)
    assert tile == 0 or (1024 <= tile <= 65536 and tile & (tile - 1) == 0)
    assert t.get("batch_filter_bits", 0) == 0 or 4 <= t["batch_filter_bits"] <= 14
    assert t.get("batch_sort_bits", 0) == 0 or 4 <= t["batch_sort_bits"] <= 12
    assert -1 <= t.get("batch_side_sets", 0) <= 4096
    assert t.get("batch_items", 0) in (0, 2, 4, 8)


def test_option_struct_matches_header(tmp_path):
    """The binding's option struct has the size and field offsets the C
    compiler gives hull2d_options."""
    import paper_1508_05931_amd as hx
    names = [f[0] for f in hx._Options._fields_]
    src = tmp_path / "opt.c"
    body = "".join(f'    printf("%s %zu\\n", "{n}", offsetof(hull2d_options, {n}));\n' for n in names)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "hull2d.h"\nint main(void) {\n'
                   '    printf("size %zu\\n", sizeof(hull2d_options));\n' + body + '    return 0;\n}\n')
    exe = tmp_path / "opt"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    assert int(got["size"]) == ctypes.sizeof(hx._Options)
    for n in names:
        assert int(got[n]) == getattr(hx._Options, n).offset, n


def test_autotune_grid_is_valid():
    """Every schedule the autotuner times is one the library accepts (the
    ranges hull2d_batch checks), and each differs from the others."""
    from paper_1508_05931_amd import autotune as at
    seen = set()
    for kw in at.PERSISTENT:
        assert kw["batch_engine"] == 1
        assert kw["batch_blocks_per_cu"] in (1, 2) and kw["batch_order"] in (0, 1, 2)
        seen.add(tuple(sorted(kw.items())))
    for kw in at.TILED:
        assert kw["batch_engine"] == 0
        t = kw["batch_tile"]
        assert 1024 <= t <= 65536 and t & (t - 1) == 0
        assert 4 <= kw["batch_filter_bits"] <= 14 and 4 <= kw["batch_sort_bits"] <= 12
        assert kw["batch_side_sets"] == -1 or 1 <= kw["batch_side_sets"] <= 4096
        seen.add(tuple(sorted(kw.items())))
    assert len(seen) == len(at.PERSISTENT) + len(at.TILED)
    assert set(at.ITEMS) <= {2, 4, 8}
