"""The C-ABI library loads on a host without a GPU and exports every entry
point that include/hss.h declares.  No compute call is made here."""
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(hss_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hss_plan", "hss_partition", "hss_sort", "hss_plan_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = pytest.importorskip("paper_1803_01237_amd")
    import ctypes
    dll = ctypes.CDLL(lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(dll, n)]
    assert not missing, missing
    assert sorted(lib.EXPORTS) == declared_functions()


def test_status_strings_without_gpu():
    import paper_1803_01237_amd as lib
    assert lib._lib.hss_status_string(0) == b"ok"
    assert lib._lib.hss_status_string(-5) == b"not converged"
    assert lib._lib.hss_last_error() == b""


def test_plan_rejects_invalid_arguments_before_touching_the_device():
    import paper_1803_01237_amd as lib
    for n, p, eps in [(0, 1, 0.1), (10, 0, 0.1), (10, 11, 0.1), (10, 2, 0.0), (10, 2, 1.0),
                      (10, 2, float("nan"))]:
        with pytest.raises(lib.HssError) as ei:
            lib.Plan(n, p, eps)
        assert ei.value.status == -1


def test_no_oracle_in_product_path():
    """The product package never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_1803_01237_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "liboracle" not in text, fn
                assert "hss_oracle" not in text, fn


def test_bucket_and_staged_plans_reject_invalid_arguments_before_touching_the_device():
    import paper_1803_01237_amd as lib
    for n, p, q in [(100, 8, 0), (100, 8, 9), (0, 1, 1), (10, 11, 2)]:
        with pytest.raises(lib.HssError) as ei:
            lib.Plan(n, p, 0.05, buckets=q)
        assert ei.value.status == -1
    for n, p, r, e1, e2 in [(1000, 16, 3, 0.05, 0.05), (1000, 16, 0, 0.05, 0.05),
                            (1000, 16, 4, 0.0, 0.05), (1000, 16, 4, 0.05, 1.0),
                            (10, 16, 4, 0.05, 0.05), (1000, 16, 32, 0.05, 0.05)]:
        with pytest.raises(lib.HssError) as ei:
            lib.StagedPlan(n, p, r, e1, e2)
        assert ei.value.status == -1


def test_static_partition_limits_checked_on_the_host():
    """The fixed-workspace entry point refuses shapes beyond its limits before
    any device call, and the largest accepted shapes fit its array."""
    import ctypes
    import paper_1803_01237_amd as lib
    L = lib._lib
    a = 1 << 40   # aligned, far-apart addresses, never dereferenced
    for n, p in [((1 << 20) + 1, 16), (1 << 20, 257)]:
        st = L.hss_partition_static(n, p, 0.05, lib.HSS_U64, 1, a, None, a + (1 << 30), None,
                                    a + (1 << 31), None)
        assert st == -2
        assert b"at most" in L.hss_last_error()
    for kb in (4, 8):
        for pay in (False, True):
            for eps in (1e-6, 0.02, 0.999):
                st, need, cap = lib.static_workspace_bytes(1 << 20, 256, eps, kb, pay)
                assert st == 0 and 0 < need <= cap
    assert lib.static_workspace_bytes(10, 20, 0.05)[0] == -1


def test_workspace_limit_fails_before_touching_the_device():
    """A plan or batch whose workspace exceeds tuning.workspace_limit_mib fails
    with HSS_ERR_OUT_OF_MEMORY on the host: on a host without a GPU any
    device call would have failed with HSS_ERR_DEVICE first."""
    import paper_1803_01237_amd as lib
    for n, p, kb, pay in [(1 << 28, 1024, 8, False), (1 << 24, 4096, 8, True), (1 << 20, 16, 4, False)]:
        with pytest.raises(lib.HssError) as ei:
            lib.Plan(n, p, 0.05, key_bytes=kb, payload=pay, workspace_limit_mib=1)
        assert ei.value.status == -3
        assert "above the limit" in str(ei.value)
    with pytest.raises(lib.HssError) as ei:
        lib.BatchPlan([(1 << 20, 64, 0.05, 8), (1 << 16, 16, 0.05, 4)], workspace_limit_mib=1)
    assert ei.value.status == -3


def test_pick_sampler_options_checked_on_the_host():
    import paper_1803_01237_amd as lib
    with pytest.raises(lib.HssError) as ei:
        lib.Plan(1000, 10, 0.05, pick_sampler=True)   # needs probes_per_round
    assert ei.value.status == -1


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message and a
    non-zero status before touching the device."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
