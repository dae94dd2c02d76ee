"""The C ABI boundary without a GPU: the library loads, exports every function the header
declares (and nothing else of its own), the binding's list matches the header, and the
host-only entry points behave as documented.  No compute call is made."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpa_mi355x.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"RPA_API\s+[\w\s\*]+?\b(\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2407_19930_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2407_19930_amd import build
        build.build()
    return binding.load()


def test_header_declares_the_four_calls():
    names = header_functions()
    for f in ("build_chi0_tau", "chi0_tau_to_omega", "chi0_R_to_q", "rpa_correlation_energy"):
        assert f in names
    assert len(names) >= 24


def test_library_exports_every_declared_function(lib):
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_list_matches_header():
    from paper_2407_19930_amd.binding import EXPORTED
    assert sorted(EXPORTED) == header_functions()


def test_no_other_library_functions_exported(lib):
    from paper_2407_19930_amd import binding
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("nm not available")
    ours = set()
    for line in out.stdout.splitlines():
        parts = line.split()
        if len(parts) == 3 and parts[1] == "T":
            ours.add(parts[2])
    declared = set(header_functions())
    # kernels and helpers stay hidden (-fvisibility=hidden); only the ABI is visible
    extra = sorted(n for n in ours if (n.startswith("rpa_") or "chi0" in n or "launch" in n or "kernel" in n)
                   and n not in declared)
    assert not extra, extra
    assert declared <= ours


def test_host_only_entry_points(lib):
    # workspace size of the energy stage: positive, monotone in n, zero for bad sizes
    a = lib.rpa_ec_workspace_size(64, 2, 4)
    b = lib.rpa_ec_workspace_size(128, 2, 4)
    assert 0 < a < b
    assert lib.rpa_ec_workspace_size(0, 2, 4) == 0
    assert lib.rpa_ec_workspace_size(64, -1, 4) == 0
    # the complex matrices dominate: at least L for every q and one T and one B
    n, nq = 256, 3
    assert lib.rpa_ec_workspace_size(n, nq, 8) >= (nq + 2) * n * n * 16
    # null handles are rejected without touching a device
    assert lib.rpa_last_error(None) == b"null context"
    assert lib.rpa_plan_destroy(None) == 1
    assert lib.rpa_batch_run(None) == 1
    assert lib.rpa_batch_destroy(None) == 1
    assert lib.rpa_profile(None, 1) == 1
    out = ctypes.c_void_p()
    assert lib.rpa_create(None, 0, None) == 1
    assert lib.build_chi0_tau(None, 2.0, None, None, None, None, 0, None) == 1
    assert lib.rpa_batch_create(None, 1, 1, None, ctypes.byref(out)) == 1
    assert lib.rpa_plan_get_tuning(None, None) == 1
    assert lib.rpa_plan_set_tuning(None, None) == 1
    assert lib.rpa_plan_autotune(None, 2.0, None, None, None, None, 0, None, None) == 1
    # Green's-function workspace: X for the larger band set plus W, both complex per k
    nk, nb = 8, 26
    assert lib.rpa_green_workspace_size(nk, nb, 13) >= 2 * nk * nb * nb * 16 * 3 // 4
    assert lib.rpa_green_workspace_size(nk, nb, 0) >= 2 * nk * nb * nb * 16
    assert lib.rpa_green_workspace_size(nk, nb, nb + 1) == 0
    assert lib.rpa_green_workspace_size(0, nb, 1) == 0
    assert lib.build_green_tau(None, 1, 1, 0, 0.0, 1, None, None, None, None, None, None, 0, None, None) == 1
