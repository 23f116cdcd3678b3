"""The C-ABI library loads and exports every entry point include/apd.h
declares (no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "apd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(apd_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_paper_calls():
    names = _declared()
    for n in ("apd_assign", "apd_dual_objective_grad", "apd_fit_weights", "apd_lloyd_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2403_03571_amd as apd
    L = apd.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(apd.EXPORTS) == _declared()


def test_choose_resolution_matches_the_rule():
    """eq. (2.10) on the host side of the library (no kernel)."""
    import paper_2403_03571_amd as apd
    assert apd.apd_choose_resolution(2, 0.01, 1e-4) == 2001
    assert apd.apd_choose_resolution(3, 0.01, 1e-4) == 201
    assert apd.apd_choose_resolution(2, 0.01, 1.0 / 25) == 101
    with pytest.raises(apd.ApdError):
        apd.apd_choose_resolution(4, 0.01, 1e-4)


def test_library_has_no_oracle_dependency():
    """The product library links neither the oracle nor any CPU fallback."""
    import paper_2403_03571_amd as apd
    data = open(apd.LIB_PATH, "rb").read()
    assert b"orc_" not in data
    assert b"liboracle" not in data
    src = open(os.path.join(ROOT, "paper_2403_03571_amd", "__init__.py")).read()
    assert "import oracle" not in src and "from oracle" not in src


def test_null_context_is_rejected():
    import paper_2403_03571_amd as apd
    L = apd.lib()
    p = apd.apd_problem()
    assert L.apd_assign(None, ctypes.byref(p), None, None, None, 0) == 1
    assert L.apd_last_error(None) == b"no context"


def test_bench_refuses_more_than_one_gpu():
    """The library runs on one GPU: bench.py --gpus 2 exits with status 2
    and says so (before touching a device)."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes mirrors of the C structs have the sizes and
    field offsets a C compiler gives the header's structs."""
    import subprocess
    import paper_2403_03571_amd as apd
    checks = {"apd_problem": ["dim", "power", "n", "grid", "lo", "hi", "x", "A", "v", "mass"],
              "apd_fit_opts": ["eps", "max_iter", "warm", "prec", "refine", "gamma0", "coarse_eps"],
              "apd_fit_report": ["converged", "max_rel_err", "seconds", "grid", "refinements",
                                 "coarse_evals"],
              "apd_tune_result": ["variant", "pixels_per_lane", "pass_ms"],
              "apd_tune_batched_result": ["kernel", "pixels_per_lane", "fit_ms"],
              "apd_pass_stats": ["pixels", "rechecked", "pass_ms", "tiles_credited", "kernel",
                                 "pixels_per_lane"]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{ROOT}/include/apd.h"', "int main(void) {"]
    for t, fields in checks.items():
        lines.append(f'printf("{t} %zu\\n", sizeof({t}));')
        for f in fields:
            lines.append(f'printf("{t}.{f} %zu\\n", offsetof({t}, {f}));')
    lines.append('printf("APD_BF16_RECHECK %d\\n", (int)APD_BF16_RECHECK);')
    lines.append('printf("APD_KERNEL_FP32_HYBRID %d\\n", (int)APD_KERNEL_FP32_HYBRID);')
    lines.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", str(c), "-o", str(exe)], check=True, capture_output=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    assert int(got["APD_BF16_RECHECK"]) == apd.APD_BF16 == 2
    assert int(got["APD_KERNEL_FP32_HYBRID"]) == apd.KERNELS["fp32-hybrid"]
    for t, fields in checks.items():
        cls = getattr(apd, t)
        assert int(got[t]) == ctypes.sizeof(cls), t
        for f in fields:
            assert int(got[f"{t}.{f}"]) == getattr(cls, f).offset, (t, f)
