"""Host-side checks of the C ABI: symbols, struct layouts, argument validation.

No call here reaches the GPU: every call is rejected by host validation first.
"""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from paper_2603_00538_amd import ft

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ft.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ft.LIB_PATH):
        pytest.skip("libft.so not built")
    return ft.load()


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:ft_status|int64_t|int32_t|const char\*)\s+(ft_\w+)\(", text, re.M)))


def test_header_declares_the_binding_names():
    assert _declared_functions() == sorted(ft.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name
    nm = shutil.which("nm")
    if nm:
        out = subprocess.run([nm, "-D", "--defined-only", ft.LIB_PATH], capture_output=True, text=True).stdout
        exported = set(re.findall(r" T (ft_\w+)$", out, re.M))
        assert set(_declared_functions()) <= exported


def test_struct_layouts_match_header(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("gcc or HIP headers unavailable")
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ft.h"\n'
                   "#define P(T, f) printf(#T \".\" #f \" %zu\\n\", offsetof(T, f))\n"
                   "int main(void){\n"
                   'printf("ft_sample_cfg %zu\\n", sizeof(ft_sample_cfg));\n'
                   'printf("ft_solve_cfg %zu\\n", sizeof(ft_solve_cfg));\n'
                   'printf("ft_report %zu\\n", sizeof(ft_report));\n'
                   'printf("ft_target_info %zu\\n", sizeof(ft_target_info));\n'
                   'printf("ft_allocation %zu\\n", sizeof(ft_allocation));\n'
                   "P(ft_allocation, weight_sum); P(ft_allocation, predicted_stderr);\n"
                   "P(ft_sample_cfg, alpha); P(ft_sample_cfg, seed); P(ft_sample_cfg, stream_id); "
                   "P(ft_sample_cfg, precision);\n"
                   "P(ft_report, iters); P(ft_report, status); P(ft_report, n_nonfinite); "
                   "P(ft_report, sum_b_stderr);\n"
                   "P(ft_target_info, n_nodes); P(ft_target_info, n_inverted); P(ft_target_info, order);\n"
                   "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                    str(src), "-o", str(exe)], check=True, capture_output=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split("\n")
               if line)
    assert int(got["ft_sample_cfg"]) == ctypes.sizeof(ft.SampleCfg)
    assert int(got["ft_solve_cfg"]) == ctypes.sizeof(ft.SolveCfg)
    assert int(got["ft_report"]) == ctypes.sizeof(ft.Report)
    assert int(got["ft_target_info"]) == ctypes.sizeof(ft.TargetInfo)
    assert int(got["ft_allocation"]) == ctypes.sizeof(ft.Allocation)
    for cls, cname in [(ft.SampleCfg, "ft_sample_cfg"), (ft.Report, "ft_report"), (ft.TargetInfo, "ft_target_info"),
                       (ft.Allocation, "ft_allocation")]:
        for fname, _ in cls._fields_:
            key = f"{cname}.{fname}"
            if key in got:
                assert int(got[key]) == getattr(cls, fname).offset, key


def test_host_validation_rejects_bad_arguments(lib):
    P = ctypes.c_void_p
    h = P()
    fake = P(0x1000)    # never dereferenced: validation fails first
    assert lib.ft_target_create(7, 10, fake, 4, fake, None, ctypes.byref(h)) == ft.FT_E_ARG
    assert "dim" in lib.ft_last_error().decode()
    assert lib.ft_target_create(1, 10, fake, 4, fake, None, ctypes.byref(h)) == ft.FT_E_ARG
    assert lib.ft_target_create(2, 10, None, 4, fake, None, ctypes.byref(h)) == ft.FT_E_ARG
    assert lib.ft_target_create(2, 2, fake, 4, fake, None, ctypes.byref(h)) == ft.FT_E_ARG
    assert lib.ft_target_create(2, 10, fake, 0, fake, None, ctypes.byref(h)) == ft.FT_E_ARG
    assert lib.ft_target_create(2, 10, fake, 4, fake, None, None) == ft.FT_E_ARG
    assert lib.ft_target_create_p2(4, 10, fake, 4, fake, None, ctypes.byref(h)) == ft.FT_E_ARG
    assert lib.ft_target_create_p2(2, 5, fake, 1, fake, None, ctypes.byref(h)) == ft.FT_E_ARG   # < 6 nodes
    assert lib.ft_query_count(None, 4) == -1
    cfg = ft.SampleCfg(0, 1, 1.0, 0, 0, ft.FT_F64)
    assert lib.ft_sample_points(None, ctypes.byref(cfg), fake, None) == ft.FT_E_ARG
    assert lib.ft_consume_queries(None, ctypes.byref(cfg), fake, None) == ft.FT_E_ARG
    rep = ft.Report()
    scfg = ft.SolveCfg(1e-14, 100)
    assert lib.ft_project(None, ctypes.byref(scfg), fake, None, ctypes.byref(rep), None) == ft.FT_E_ARG
    assert lib.ft_source_create_p1(4, 10, fake, 4, fake, 1, fake, None, None, ctypes.byref(h)) == ft.FT_E_ARG
    assert lib.ft_source_create_p1(2, 10, fake, 4, fake, 0, fake, None, None, ctypes.byref(h)) == ft.FT_E_ARG
    assert lib.ft_source_eval(None, 10, fake, 10, 0, fake, 10, None, None) == ft.FT_E_ARG
    assert lib.ft_source_eval_queries(None, 4, 10, fake, 10, 0, fake, 10, None, None) == ft.FT_E_ARG
    assert lib.ft_batch_create(0, None, None, None, 0, None, ctypes.byref(h)) == ft.FT_E_ARG
    assert lib.ft_batch_create(1, None, None, None, 0, None, None) == ft.FT_E_ARG
    assert lib.ft_batch_run(None, None, None, None, None, None, None) == ft.FT_E_ARG
    assert lib.ft_batch_destroy(None) == ft.FT_OK
    assert lib.ft_source_get_info(None, None) == ft.FT_E_ARG
    assert lib.ft_target_destroy(None) == ft.FT_OK
    assert lib.ft_source_destroy(None) == ft.FT_OK
    al = ft.Allocation()
    assert lib.ft_allocate_samples(None, 0, 100, 2, 64, fake, ctypes.byref(al), None) == ft.FT_E_ARG
    assert lib.ft_sample_points_adaptive(None, ctypes.byref(cfg), fake, 100, fake, None) == ft.FT_E_ARG
    assert lib.ft_consume_queries_adaptive(None, ctypes.byref(cfg), fake, 100, fake, None) == ft.FT_E_ARG


def test_samples_for_tolerance_matches_oracle(lib):
    """Host-only entry point: the samples per element that bring the standard
    error of sum b to a relative target (it falls as N^-1/2), as the oracle's
    samples_for_tolerance computes it; the edge cases the header states."""
    from oracle import cvmc

    rng = np.random.default_rng(11)
    for _ in range(200):
        sb = float(rng.choice([-1.0, 1.0]) * 10 ** rng.uniform(-3, 3))
        se = abs(sb) * 10 ** rng.uniform(-7, -1)
        N = int(rng.integers(1, 512))
        tol = 10 ** rng.uniform(-6, -1)
        rep = ft.Report(sum_b=sb, sum_b_stderr=se)
        assert ft.ft_samples_for_tolerance(rep, N, tol) == cvmc.samples_for_tolerance(se, sb, N, tol)
    # halving the error takes four times the samples
    assert ft.ft_samples_for_tolerance({**ft.Report().as_dict(), "sum_b": 2.0, "sum_b_stderr": 1e-4}, 64,
                                       0.25e-4 * (1 + 1e-12)) == 256
    assert ft.ft_samples_for_tolerance(ft.Report(sum_b=1.0, sum_b_stderr=0.0), 64, 1e-6) == 1   # exact b
    assert ft.ft_samples_for_tolerance(ft.Report(sum_b=0.0, sum_b_stderr=1e-3), 64, 1e-6) == 1
    assert ft.ft_samples_for_tolerance(ft.Report(sum_b=1.0, sum_b_stderr=-1.0), 64, 1e-6) == -1  # no estimate
    assert ft.ft_samples_for_tolerance(ft.Report(sum_b=1.0, sum_b_stderr=1e-3), 0, 1e-6) == -1
    assert ft.ft_samples_for_tolerance(ft.Report(sum_b=1.0, sum_b_stderr=1e-3), 64, 0.0) == -1
    assert ft.ft_samples_for_tolerance(ft.Report(sum_b=1.0, sum_b_stderr=1.0), 64, 1e-9) == 1 << 20
    assert lib.ft_samples_for_tolerance(None, 64, 1e-3) == -1


def test_binding_refuses_to_run_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(ft, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        ft.load(str(tmp_path / "nope.so"))


def test_budget_for_tolerance_matches_oracle(lib):
    """Host-only: the total samples whose Neyman prediction W / sqrt(B) reaches
    rel_tol |sum b|, as the oracle computes it, and the stated edge cases."""
    from oracle import adaptive

    rng = np.random.default_rng(12)
    for _ in range(200):
        sb = float(rng.choice([-1.0, 1.0]) * 10 ** rng.uniform(-3, 3))
        W = abs(sb) * 10 ** rng.uniform(-5, 1)
        tol = 10 ** rng.uniform(-6, -1)
        B = ft.ft_budget_for_tolerance(W, sb, tol)
        assert B == adaptive.budget_for_tolerance(W, sb, tol)
        if 1 < B < 2 ** 40:
            assert W / np.sqrt(B) <= tol * abs(sb) * (1 + 1e-12) and W / np.sqrt(B - 1) > tol * abs(sb) * (1 - 1e-12)
    assert ft.ft_budget_for_tolerance(0.0, 1.0, 1e-3) == 1
    assert ft.ft_budget_for_tolerance(1.0, 0.0, 1e-3) == 1
    assert ft.ft_budget_for_tolerance(1.0, 1.0, 0.0) == -1
    assert ft.ft_budget_for_tolerance(-1.0, 1.0, 1e-3) == -1
    assert ft.ft_budget_for_tolerance(float("nan"), 1.0, 1e-3) == -1
    assert ft.ft_budget_for_tolerance(1.0, 1.0, 1e-30) == 2 ** 40
