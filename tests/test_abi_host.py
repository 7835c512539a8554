"""Host-side checks of the C ABI: the library loads, exports what gsbs.h
declares, and its host-only logic (schedule planner, argument validation)
agrees with the oracle.  No device work is issued."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def g():
    from paper_2509_03313_amd import gsbs
    return gsbs


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "gsbs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsbs_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported(g):
    import ctypes
    lib = ctypes.CDLL(g.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 25
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(g.EXPORTED) == syms


def test_default_params(g):
    p = g.gsbs_default_params()
    assert p.c_cut == 5.0 and p.rounds == 4 and p.contact_only == 0
    assert p.dt0_ns == 1e-3 and p.ratio == 10.0 ** (6.0 / 1999.0)
    assert p.grid_config == -1 and p.autotune == 1


def test_invalid_arguments_fail_cleanly(g):
    with pytest.raises(g.GsbsError) as e:
        g.gsbs_create([(-1.0, 0)], 1)
    assert e.value.code == -1
    with pytest.raises(g.GsbsError):
        g.gsbs_plan_schedule(0.0, 1.0, [0.0], [], -1.0, 1.01, 1.0)
    with pytest.raises(g.GsbsError):
        g.gsbs_plan_schedule(2.0, 1.0, [0.0], [], 1e-3, 1.01, 1.0)


@pytest.mark.parametrize("case", ["single", "pulses", "capped", "offset_start"])
def test_schedule_matches_oracle_bit_exact(g, orc, case):
    ratio = 10.0 ** (6.0 / 1999.0)
    if case == "single":
        args = (0.0, 1000.0, [0.0], [0.0] + list(1e-3 * 10.0 ** (6.0 * np.arange(0, 2000, 20) / 1999.0)),
                1e-3, ratio, 1e9)
    elif case == "pulses":
        inj = [0.0, 100.0, 200.0, 1e6, 1e6 + 100.0]
        ev = sorted(set(inj + list(np.geomspace(1e-3, 2e6, 300))))
        args = (0.0, 2e6, inj, ev, 1e-3, ratio, 3.5e4)
    elif case == "capped":
        args = (0.0, 5e5, [0.0], [], 1e-3, ratio, 100.0)
    else:
        args = (37.5, 9e4, [0.0, 50.0], [60.0, 61.0, 8e4], 1e-3, ratio, 2e3)
    a = g.gsbs_plan_schedule(*args)
    b = orc.schedule(*args)
    assert len(a) == len(b) and np.array_equal(a, b)
    assert np.all(np.diff(np.concatenate([[args[0]], a])) > 0)
    assert a[-1] == args[1]
