"""The C ABI library loads, exports every entry point declared in
include/cbic.h, and rejects invalid arguments without touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cbic.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cbic_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2602_19699_amd import cbic
    return cbic.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_2602_19699_amd import cbic
    assert set(declared()) == set(cbic._SIGS)


def test_opts_default_and_host_side_validation(lib):
    from paper_2602_19699_amd import cbic, inputs as I
    o = cbic.Options().c()
    assert o.struct_size == C.sizeof(cbic._Opts) and o.max_iter == 50 and o.ls_max_trials == 16
    # a system without a context is validated on the host only
    s = cbic.System(None, I.SYS_POINT_MASS, I.point_mass_params(0))
    assert (s.n, s.m) == (4, 2)
    ws = s.workspace_size(16384, 100)
    assert ws > 16384 * 100 * 8 * 16
    for bad in ([1.0, 2.0], np.r_[I.point_mass_params(0)[:-1], np.nan]):
        with pytest.raises(cbic.CbicError) as e:
            cbic.System(None, I.SYS_POINT_MASS, bad)
        assert e.value.code == cbic.E_INVALID
    with pytest.raises(cbic.CbicError):
        cbic.System(None, 9, I.point_mass_params(0))
    q = cbic.System(None, I.SYS_LQ, I.lq_random(5, 2))
    with pytest.raises(cbic.CbicError) as e:  # no kernel for this LQ size
        q.workspace_size(4, 10)
    assert e.value.code == cbic.E_UNSUPPORTED
    with pytest.raises(cbic.CbicError) as e:
        s.workspace_size(0, 100)
    assert e.value.code == cbic.E_INVALID
    with pytest.raises(cbic.CbicError) as e:
        s.workspace_size(4, 100, cbic.Options(ls_beta=1.5))
    assert e.value.code == cbic.E_INVALID
    for bad_occ in (-1, 3):  # instances per compute unit of the workgroup schedule: 0, 1 or 2
        with pytest.raises(cbic.CbicError) as e:
            s.workspace_size(4, 100, cbic.Options(wg_per_cu=bad_occ))
        assert e.value.code == cbic.E_INVALID and b"wg_per_cu" in lib.cbic_last_error()
    s.workspace_size(4, 100, cbic.Options(wg_per_cu=2))
    bad = cbic.Options().c()
    bad.struct_size = 8
    v = C.c_size_t()
    assert lib.cbic_workspace_size(s.h, 4, 10, C.byref(bad), C.byref(v)) == cbic.E_INVALID
    assert b"struct_size" in lib.cbic_last_error()
    # a solve without a context is rejected before any launch
    assert lib.cbic_solve_batch(None, s.h, 4, 10, None, None, None, None, None, None) == cbic.E_INVALID
