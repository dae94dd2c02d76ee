"""The host code that builds a plan's tables (neighbour CSR, BvK fold, N offsets, work lists,
template classes, launch orders, workspace layout) under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU: api.hip compiled with RPA_HOST_TABLE_TEST (tables in host
memory, no kernel launched) and host-side sanitizers, linked with the library's other objects and
a driver (tests/host/plan_tables_driver.cpp) that runs rpa_plan_create on ragged and limit shapes
and on inputs the plan must reject, and checks the returned status.  The table summaries are then
checked against counts derived here from the inputs."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from tests._util import cfg, micro

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_19930_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
OTHERS = ["chi0_kernels", "chi0_bf16", "transform_kernels", "ec_kernels", "green_kernels", "screen_kernels", "session"]
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")


def case_text(name, expect, nao, naux, mesh, I, K, R, off, ntau=3, prec=0):
    lines = ["case %s %d %d %d %d %d %d %d" % (name, expect, len(nao), ntau, prec, *mesh),
             " ".join(str(int(x)) for x in nao), " ".join(str(int(x)) for x in naux), str(len(I))]
    for b in range(len(I)):
        lines.append("%d %d %d %d %d %d" % (I[b], K[b], R[b][0], R[b][1], R[b][2], off[b]))
    return "\n".join(lines) + "\n"


def from_inputs(name, inp, prec=0):
    b = inp.blocks
    return case_text(name, 0, inp.nao, inp.naux, inp.cell.mesh, b.I, b.K, b.R, b.off, inp.ntau, prec)


def expected(inp_like):
    nao, naux, mesh, K, natoms = inp_like
    nR = int(np.prod(mesh))
    npairs = natoms * (natoms + 1) // 2
    items = npairs * nR
    slices = int(sum(nao[k] for k in K))
    halves = sum((1 + (naux[V] > 64)) * nR for U in range(natoms) for V in range(U, natoms))
    return items, slices, halves


@pytest.fixture(scope="module")
def sanitized_driver():
    from paper_2407_19930_amd import build
    objdir = os.path.join(CSRC, "..", "_build")
    if not all(os.path.exists(os.path.join(objdir, o + ".o")) for o in OTHERS):
        build.build()
    tmp = tempfile.mkdtemp(prefix="rpa_asan_")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-DRPA_HOST_TABLE_TEST",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    api_o = os.path.join(tmp, "api_san.o")
    drv_o = os.path.join(tmp, "driver.o")
    exe = os.path.join(tmp, "plan_tables_san")
    steps = [
        [HIPCC] + flags + SAN_HOST + ["-c", os.path.join(CSRC, "api.hip"), "-o", api_o],
        [HIPCC, "-O1", "-g", "-std=c++17"] + SAN_HOST + ["-c", os.path.join(ROOT, "tests", "host",
                                                                             "plan_tables_driver.cpp"), "-o", drv_o],
        [HIPCC, "--offload-arch=gfx950"] + SAN_HOST + [drv_o, api_o] +
        [os.path.join(objdir, o + ".o") for o in OTHERS] + ["-o", exe],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
    yield exe
    shutil.rmtree(tmp, ignore_errors=True)


def run(exe, text, tmpdir):
    path = os.path.join(tmpdir, "cases.txt")
    with open(path, "w") as fh:
        fh.write(text)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, path], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return r.stdout


def test_plan_tables_under_sanitizers(sanitized_driver, tmp_path):
    tiny = cfg(0, with_coulomb=False)
    ragged = micro(seed=2, natoms=3, nao=(2, 5, 3), naux=(3, 6, 2), mesh=(3, 1, 2))
    limit = micro(seed=8, natoms=2, nao=(32, 1), naux=(128, 1), mesh=(1, 1, 1), rcut=3.5, edge=4.0)
    cases = [from_inputs("tiny_fp64", tiny, 0), from_inputs("tiny_bf16", tiny, 2), from_inputs("ragged_fp32", ragged, 1),
             from_inputs("ragged_bf16", ragged, 2), from_inputs("limit_bf16", limit, 2)]
    want = {"tiny_fp64": (tiny.nao, tiny.naux, tiny.cell.mesh, tiny.blocks.K, tiny.natoms),
            "ragged_fp32": (ragged.nao, ragged.naux, ragged.cell.mesh, ragged.blocks.K, ragged.natoms),
            "limit_bf16": (limit.nao, limit.naux, limit.cell.mesh, limit.blocks.K, limit.natoms)}
    # 1024 LRI blocks on one atom (the per-atom limit), images folding many times over a 4x1x1 mesh,
    # plus an atom without any block of its own
    n = 1024
    I = [0] * n
    K = [0] * (n // 2) + [1] * (n // 2)
    R = [(r - 512, 0, 0) for r in range(n)]
    off = list(np.cumsum([0] + [3 * 4 * (4 if k == 0 else 2) for k in K[:-1]]))
    cases.append(case_text("nbr1024", 0, [4, 2, 3], [3, 70, 5], (4, 1, 1), I, K, R, off, 2, 2))
    want["nbr1024"] = ([4, 2, 3], [3, 70, 5], (4, 1, 1), K, 3)
    # rejected: 1025 blocks on one atom, 33 NAOs, an atom index out of range, a negative offset,
    # a mesh of 1024
    cases.append(case_text("nbr1025", 7, [2], [2], (1, 1, 1), [0] * 1025, [0] * 1025, [(r, 0, 0) for r in range(1025)],
                           list(range(0, 4 * 1025, 4))))
    cases.append(case_text("nao33", 7, [33], [4], (1, 1, 1), [0], [0], [(0, 0, 0)], [0]))
    cases.append(case_text("badK", 2, [2, 2], [2, 2], (1, 1, 1), [0, 1], [0, 2], [(0, 0, 0), (0, 0, 0)], [0, 8]))
    cases.append(case_text("negoff", 2, [2], [2], (1, 1, 1), [0], [0], [(0, 0, 0)], [-4]))
    cases.append(case_text("mesh1024", 7, [2], [2], (1024, 1, 1), [0], [0], [(0, 0, 0)], [0]))
    out = run(sanitized_driver, "".join(cases), str(tmp_path))
    assert "cases %d" % len(cases) in out
    got = {}
    for line in out.splitlines():
        f = line.split()
        if f and f[0] == "summary":
            got[f[1]] = [int(x) for x in f[2:]]
    for name, spec in want.items():
        items, slices, halves = expected(spec)
        s = got[name]
        assert s[0] > 0 and s[1] == items and s[6] == slices and s[7] == halves, (name, s, items, slices, halves)
