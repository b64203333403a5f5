"""CPU checks of the C ABI: the library loads, exports every function that
include/dotsocp.h declares, and rejects invalid problems before touching a
device."""
import os
import re

import numpy as np
import pytest

from paper_2505_05424_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dotsocp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dot_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_binding_names():
    assert set(_declared()) == set(B.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = B.load()
    for name in _declared():
        assert hasattr(lib, name), name


def _bad(**kw):
    base = dict(D=1, n=(4, 8), rho0=np.ones(9) / 9, rho1=np.ones(9) / 9)
    base.update(kw)
    D = base.pop("D")
    n = base.pop("n")
    r0 = base.pop("rho0")
    r1 = base.pop("rho1")
    with pytest.raises(B.DotError) as e:
        B.dot_plan_create(D, n, r0, r1, **base)
    return str(e.value)


def test_invalid_problems_are_rejected():
    assert "equal" in _bad(rho1=np.r_[np.ones(8) / 9, 2.0 / 9])      # mass mismatch
    assert "non-negative" in _bad(rho0=np.r_[-1.0, np.ones(8) / 4])   # negative mass
    assert "finite" in _bad(rho0=np.r_[np.nan, np.ones(8) / 8])        # NaN
    assert "D must be" in _bad(D=4, n=(2, 2, 2, 2))
    assert "segment" in _bad(n=(0, 8))
    assert "tau" in _bad(tau=2.5)
    assert "positive total" in _bad(rho0=np.zeros(9), rho1=np.zeros(9))


@pytest.mark.parametrize("D,n,masked", [(1, (4, 10), False), (2, (6, 8, 12), True), (3, (4, 6, 4, 8), False)])
def test_coarsen_data_matches_the_oracle(D, n, masked):
    """Host arithmetic of the library (no device): the restriction of the
    data to the coarser grid equals the oracle's."""
    import dotgen
    from oracle import multilevel as ML
    inst = dotgen.tiny_instance(D, n, seed=11, floor=0.0, masked=masked)
    nc, r0, r1, mk = B.dot_coarsen_data(D, n, inst.rho0, inst.rho1, inst.mask)
    nc2, q0, q1, mk2 = ML.coarse_data(n, inst.rho0, inst.rho1, inst.mask)
    assert nc == nc2
    np.testing.assert_allclose(r0, q0, rtol=1e-14, atol=1e-17)
    np.testing.assert_allclose(r1, q1, rtol=1e-14, atol=1e-17)
    if masked:
        np.testing.assert_array_equal(mk, mk2)


def test_binding_structs_match_the_header_layout(tmp_path):
    """sizeof and every field offset of the ctypes structures equal those the
    C compiler gives the header's structures (plain gcc, no GPU)."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"dot_problem": B.dot_problem, "dot_result": B.dot_result, "dot_plan_info": B.dot_plan_info,
               "dot_schedule": B.dot_schedule}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dotsocp.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            parts = line.split()
            got[tuple(parts[:-1])] = int(parts[-1])
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
