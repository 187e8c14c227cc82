"""Host-only checks of the C ABI: the built library loads and exports every
function include/spgemm.h declares; host-side entry points behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "spgemm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(spg(?:emm)?_[A-Za-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ("spgemm_symbolic", "spgemm_numeric", "spg_create", "spg_destroy", "spg_get_stats",
                 "spg_status_string", "spg_last_error", "spg_check_errors"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_1801_03065_amd as spg

    L = spg.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_entry_points():
    import paper_1801_03065_amd as spg

    L = spg.lib()
    assert "gfx950" in spg.version()
    assert L.spg_status_string(0) == b"ok"
    assert b"structure differs" in L.spg_status_string(6)
    o = spg.options()
    assert o.compression == -1 and abs(o.cf_threshold - 0.85) < 1e-15 and o.accumulator == 0
    # NULL handle is rejected before any device work
    assert L.spgemm_symbolic(None, None, None, None, 0, None) == spg.SPG_ERR_INVALID_ARG
    assert L.spgemm_numeric(None, None, None, None) == spg.SPG_ERR_INVALID_ARG
    assert L.spg_destroy(None) == spg.SPG_ERR_INVALID_ARG
    st = spg.spg_stats()
    assert L.spg_get_stats(None, ctypes.byref(st)) == spg.SPG_ERR_INVALID_ARG


def test_options_reject_unknown_field():
    import paper_1801_03065_amd as spg

    with pytest.raises(KeyError):
        spg.options(no_such_option=1)


def test_paper_constants_fixture():
    """Constants the paper states, used by the host logic (tests/golden/paper_constants.json)."""
    import json

    c = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_constants.json")))
    import paper_1801_03065_amd as spg

    o = spg.options()
    assert abs(o.cf_threshold - c["compression_flop_ratio_threshold"]["value"]) < 1e-15
    ex = c["linear_probing_example"]
    assert ex["key"] & (ex["table_size"] - 1) == ex["slot"]


def test_create_without_device_fails_cleanly():
    """With no GPU visible, spg_create reports a HIP error and leaves no handle."""
    import torch

    import paper_1801_03065_amd as spg

    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    L = spg.lib()
    h = ctypes.c_void_p(123)
    rc = L.spg_create(ctypes.byref(h), None, None)
    assert rc == spg.SPG_ERR_HIP
    assert not h.value


def test_create_rejects_bad_options():
    """Options are validated before any device call."""
    import paper_1801_03065_amd as spg

    L = spg.lib()
    for bad in (dict(compression=2), dict(cf_threshold=0.0), dict(cf_threshold=1.5), dict(accumulator=9),
                dict(fp32_mode=3), dict(l1_hash_slots=100), dict(l1_hash_slots=4)):
        o = spg.options(**bad)
        h = ctypes.c_void_p(0)
        assert L.spg_create(ctypes.byref(h), None, ctypes.byref(o)) == spg.SPG_ERR_INVALID_ARG, bad
        assert not h.value


def test_batch_and_panel_entry_points_reject_null_handle():
    import paper_1801_03065_amd as spg

    L = spg.lib()
    assert L.spgemm_batch_symbolic(None, 1, None, None, None, 0, None) == spg.SPG_ERR_INVALID_ARG
    assert L.spgemm_batch_numeric(None, 1, None, None, None) == spg.SPG_ERR_INVALID_ARG
    assert L.spgemm_numeric_rows(None, None, None, 0, 0, None, None) == spg.SPG_ERR_INVALID_ARG
    assert L.spgemm_backward(None, None, None, None, None, None) == spg.SPG_ERR_INVALID_ARG
    assert L.spg_check_errors(None) == spg.SPG_ERR_INVALID_ARG
