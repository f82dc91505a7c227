"""CPU checks of the C ABI: the library loads, exports every entry point
declared in include/qoc.h, runs its host-side (p, n) rule like the oracle's
reading, and rejects invalid problems before touching any device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import workloads
from paper_1612_04929_amd import qoc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "qoc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qoc_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = qoc.load()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(qoc.EXPORTS) == set(names)


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors agree with a C compiler's layout of include/qoc.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "lay.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "qoc.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(qoc_problem_desc),'
        ' offsetof(qoc_problem_desc, taylor_tol), offsetof(qoc_problem_desc, device),'
        ' sizeof(qoc_info), offsetof(qoc_info, device_bytes), offsetof(qoc_info, flags));'
        ' return 0;}\n')
    exe = tmp_path / "lay"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert got == [C.sizeof(qoc.Desc), qoc.Desc.taylor_tol.offset, qoc.Desc.device.offset,
                   C.sizeof(qoc.Info), qoc.Info.device_bytes.offset, qoc.Info.flags.offset]


@pytest.mark.parametrize("theta", [0.0, 1e-6, 0.034, 0.37, 0.78, 1.22, 4.66, 6.5, 30.0])
@pytest.mark.parametrize("tol", [1e-10, 1e-15])
def test_host_taylor_rule_agrees_with_oracle_reading(theta, tol):
    assert qoc.taylor_select(theta, tol) == oracle.taylor_select(theta, tol)
    assert qoc.select_pair(theta, tol, qoc.QOC_FORM_HORNER) == oracle.taylor_select(theta, tol)
    assert qoc.select_pair(theta, tol, qoc.QOC_FORM_BATCHED) == oracle.taylor_select_ps(theta, tol)
    assert qoc.select_pair(theta, tol, qoc.QOC_FORM_ACTION) == oracle.action_select(theta, tol)


def test_taylor_select_rejects_bad_arguments():
    with pytest.raises(qoc.QocError) as e:
        qoc.taylor_select(-1.0, 1e-10)
    assert e.value.status == -1
    with pytest.raises(qoc.QocError):
        qoc.taylor_select(1.0, 0.0)
    with pytest.raises(qoc.QocError) as e:
        qoc.select_pair(1.0, 1e-10, 3)
    assert e.value.status == -1


def _expect(status, prob, **kw):
    with pytest.raises(qoc.QocError) as e:
        qoc.Problem(prob, **kw)
    assert e.value.status == status, str(e.value)


def test_validation_errors_are_reported_before_device_use():
    base = workloads.config1()
    bad = workloads.config1(); bad.S = 3
    bad.psi0 = np.eye(3, 2, dtype=complex); bad.psiT = np.eye(3, 2, dtype=complex)
    _expect(-2, bad)                                   # S > d
    bad = workloads.config1(); bad.H0 = np.array([[0, 1], [0, 0]], complex)
    _expect(-3, bad)                                   # not Hermitian
    bad = workloads.config1(); bad.Hk = bad.Hk.copy(); bad.Hk[1, 0, 1] = np.nan
    _expect(-4, bad)                                   # NaN
    bad = workloads.config1(); bad.dt = -0.1
    _expect(-1, bad)                                   # dt <= 0
    bad = workloads.config1(); bad.w = np.array([0.0, -1.0])
    _expect(-1, bad)                                   # negative weight
    _expect(-1, base, taylor_pn=(1, 0))                # p < 2
    _expect(-1, base, precision=7)


def test_create_without_gpu_reports_device_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    _expect(-6, workloads.config1())


def test_status_strings():
    lib = qoc.load()
    for s in range(-7, 1):
        assert lib.qoc_status_string(s)
    assert lib.qoc_version().decode().startswith("libqoc")


def test_set_taylor_validates_arguments():
    lib = qoc.load()
    assert lib.qoc_set_taylor(None, 8, 2) == -1


def test_set_sweep_validates_arguments():
    lib = qoc.load()
    assert lib.qoc_set_sweep(None, 0, 1) == -1
