"""The C-ABI library (CPU checks, no GPU needed): it loads, exports every
entry point include/axf.h declares, and rejects bad arguments before any
device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "axf.h")).read()
    return sorted(set(re.findall(r"\b(axf_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_api():
    names = _declared()
    for n in ("axf_plan_create", "axf_evaluate", "axf_evaluate_direct", "axf_adjoint",
              "axf_evaluate_grad", "axf_batch_create", "axf_batch_launch", "axf_plan_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2301_01179_amd import axf
    lib = axf.load_library()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def _params(**kw):
    from paper_2301_01179_amd import axf
    base = dict(n_modes=3, order=4, depth=2, max_leaf=32, nrhs=1, flags=0)
    base.update(kw)
    return axf.Params(**base)


@pytest.mark.parametrize("kw,status", [
    (dict(n_modes=0), 4), (dict(n_modes=65), 4), (dict(order=-1), 4), (dict(order=25), 4),
    (dict(depth=1), 4), (dict(depth=12), 4), (dict(depth=0, max_leaf=0), 1),
    (dict(nrhs=0), 4), (dict(nrhs=9), 4)])
def test_bad_params_rejected_before_device_work(kw, status):
    from paper_2301_01179_amd import axf
    lib = axf.load_library()
    p = _params(**kw)
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(8)
    st = lib.axf_plan_create(ctypes.byref(p), 10, dummy, dummy, 10, dummy, dummy, None, ctypes.byref(h), None)
    assert st == status
    assert h.value is None
    assert lib.axf_last_error().decode()


def test_null_and_size_errors():
    from paper_2301_01179_amd import axf
    lib = axf.load_library()
    p = _params()
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(8)
    assert lib.axf_plan_create(None, 10, dummy, dummy, 10, dummy, dummy, None, ctypes.byref(h), None) == 1
    assert lib.axf_plan_create(ctypes.byref(p), 0, dummy, dummy, 10, dummy, dummy, None, ctypes.byref(h), None) == 1
    assert lib.axf_plan_create(ctypes.byref(p), 10, None, dummy, 10, dummy, dummy, None, ctypes.byref(h), None) == 1
    assert lib.axf_plan_create(ctypes.byref(p), 10, dummy, dummy, 10, dummy, dummy, None, None, None) == 1
    assert lib.axf_evaluate(None, dummy, dummy, None) == 1
    assert lib.axf_adjoint(None, None, dummy, dummy, None, None, None) == 1
    assert lib.axf_plan_set_workspace(None, dummy, ctypes.c_size_t(1 << 20)) == 1
    lib.axf_plan_destroy(None)
    assert lib.axf_status_string(2) == b"AXF_ERR_INVALID_GEOMETRY"
    assert lib.axf_status_string(6) == b"AXF_ERR_WORKSPACE"


def test_mode_buckets_and_tile_widths_cover_limits():
    """Host-side launch shapes of the tiled S2L (mirror of the rule in the
    library): up to the maximum order the output slots of one (box, channel)
    -- per row, the even and the odd columns in blocks of lb -- fit in at
    most four waves with blocks of at most two columns, and every output
    (k, l) has exactly one slot."""
    import math

    def slot_cols(M, b):
        cols = []
        for k in range(M + 1):
            ncol = M + 1 - k
            for par in (0, 1):
                own = list(range(par, ncol, 2))
                cols += [(k, own[i:i + b]) for i in range(0, len(own), b)]
        return cols

    for M in range(0, 25):
        lb = next(b for b in range(1, 4) if len(slot_cols(M, b)) <= 256)
        cols = slot_cols(M, lb)
        assert lb <= 2 and math.ceil(len(cols) / 64) <= 4
        owned = sorted((k, l) for k, ls in cols for l in ls)
        assert owned == [(k, l) for k in range(M + 1) for l in range(M + 1 - k)]
