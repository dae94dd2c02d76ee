"""GPU parity of the Green's-function-screened chi0 build (rpa_plan_set_screening) against the
screened FP64 oracle over the pair set U <= V (oracle/screening.py), through the C ABI.

The keep decisions are FP64 products of exact maxima on both sides, so the GPU keeps exactly the
neighbour entries and Z parts the oracle keeps (checked as integer counts), and chi follows at the
bars of the unscreened build: FP64 <= 1e-11, FP32 and split BF16 <= 1e-5 relative Frobenius, with
a per-block bar for the mixed paths.
"""
import numpy as np
import pytest

from oracle import screening as scr
from tests._gpu import device_inputs, make_plan
from tests._util import cfg, micro, rel

pytestmark = pytest.mark.gpu

SPECS = [dict(), dict(seed=2, natoms=3, nao=(2, 5, 3), naux=(3, 6, 2), mesh=(3, 1, 2)),
         dict(seed=11, natoms=3, nao=(3, 4, 2), naux=(4, 5, 3), mesh=(4, 2, 1), rcut=4.5, edge=3.5),
         dict(seed=5, natoms=3, nao=(20, 13, 26), naux=(70, 100, 120), mesh=(2, 1, 1), rcut=4.2, edge=3.0,
              ntau=2)]
BAR = {"fp64": 1e-11, "fp32": 1e-5, "bf16x3": 1e-5}
BLOCK_BAR = {"fp64": 1e-11, "fp32": 3e-5, "bf16x3": 3e-5}


def run_screened(inp, precision, theta, ctx=None):
    import torch
    from paper_2407_19930_amd import Context, build_chi0_tau
    ctx = ctx or Context(0)
    plan = make_plan(ctx, inp, precision)
    plan.set_screening(theta)
    d = device_inputs(inp)
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    chi = torch.full((inp.ntau, inp.nR, inp.nauxtot, inp.nauxtot), float("nan"), dtype=torch.float64,
                     device="cuda")
    build_chi0_tau(plan, inp.spin_factor, d["Gocc"], d["Gun"], d["C"], ws, chi)
    stats = plan.screening_stats()
    return chi.cpu().numpy(), stats, plan, ctx


def check_blocks(inp, got, ref, precision, what):
    scale = np.abs(ref).max()
    for U in range(inp.natoms):
        mu = slice(inp.aux_off[U], inp.aux_off[U] + inp.naux[U])
        for V in range(inp.natoms):
            nu = slice(inp.aux_off[V], inp.aux_off[V] + inp.naux[V])
            g, r = got[:, :, mu, nu], ref[:, :, mu, nu]
            nr = np.linalg.norm(r)
            if nr > 1e-3 * scale:
                assert rel(g, r) <= BLOCK_BAR[precision], (what, U, V, rel(g, r))
            else:
                assert np.abs(g - r).max() <= BLOCK_BAR[precision] * scale, (what, U, V)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("theta", [0.05, 0.2])
@pytest.mark.parametrize("idx", range(len(SPECS)))
def test_screened_micro(idx, theta, precision):
    inp = micro(**SPECS[idx])
    ref, ost = scr.chi0_alg1_screened_pairs(inp, theta)
    got, st, _, _ = run_screened(inp, precision, theta)
    assert np.all(np.isfinite(got))
    # identical decisions
    assert st["entries_kept"] == ost["slices_kept"] and st["entries_total"] == ost["slices_total"]
    assert st["z_kept"] == ost["z_kept"] and st["z_total"] == ost["z_total"]
    assert st["entries_kept"] < st["entries_total"] or st["z_kept"] < st["z_total"] or theta == 0.05
    assert rel(got, ref) <= BAR[precision], rel(got, ref)
    check_blocks(inp, got, ref, precision, (idx, theta))


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_screened_tiny_workload(precision):
    """The tiny workload at the case study's threshold 1e-3 and at a coarse one."""
    inp = cfg(0)
    for theta in (1e-3, 3e-2):
        ref, ost = scr.chi0_alg1_screened_pairs(inp, theta)
        got, st, _, _ = run_screened(inp, precision, theta)
        assert st["entries_kept"] == ost["slices_kept"] and st["z_kept"] == ost["z_kept"]
        assert rel(got, ref) <= BAR[precision], (theta, rel(got, ref))


def test_theta_zero_is_unscreened_bitwise():
    """Screening switched on with theta = 0 keeps every term: chi is bitwise the unscreened chi
    (same kernels, same order), and the statistics count everything."""
    from tests._gpu import gpu_chi_tau
    inp = micro(**SPECS[1])
    for precision in ("fp64", "bf16x3"):
        base, _, ctx = gpu_chi_tau(inp, precision)
        got, st, _, _ = run_screened(inp, precision, 0.0 + 1e-300, ctx)
        assert np.array_equal(got, base.cpu().numpy())
        assert st["entries_kept"] == st["entries_total"] and st["z_kept"] == st["z_total"]


def test_theta_above_one_gives_zero():
    inp = micro(**SPECS[2])
    got, st, _, _ = run_screened(inp, "fp32", 1.5)
    assert not np.any(got)
    assert st["entries_kept"] == 0 and st["slices_kept"] == 0 and st["z_kept"] == 0


def test_screening_errors():
    from paper_2407_19930_amd import Context, RpaError
    inp = micro()
    ctx = Context(0)
    plan = make_plan(ctx, inp, "fp64")
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(RpaError) as e:
            plan.set_screening(bad)
        assert e.value.code == 1
    plan.set_screening(0.1)
    with pytest.raises(RpaError) as e:       # no screened build yet
        plan.screening_stats()
    assert e.value.code == 1


def test_screened_fullsize_sampled_blocks():
    """The 8-atom workload (4x4x4 mesh, 16 tau) at the case study's threshold 1e-3, split BF16 in
    the launch configuration of the benchmark: sampled blocks (U < V, U = V, U > V; R = 0 and
    R != 0; first and last tau, where the screening drops the most and nothing) against the
    screened oracle, and the kept counts of those tau points."""
    import torch
    from oracle.chi0 import bvk_sub
    inp = cfg(1, with_coulomb=False)
    theta = 1e-3
    got, st, plan, _ = run_screened(inp, "bf16x3", theta)
    assert st["slices_kept"] < st["slices_total"]
    alg = scr.ScreenedAlg1(inp, theta)
    mesh = inp.cell.mesh
    for t in (0, inp.ntau - 1):
        for (U, V, R) in ((0, 3, 0), (2, 2, 21), (5, 1, 7), (7, 7, 0)):
            if U <= V:
                ref = alg.block(t, U, V, R)
            else:
                ref = alg.block(t, V, U, int(bvk_sub(0, R, mesh))).T
            g = got[t, R, inp.aux_off[U]:inp.aux_off[U] + inp.naux[U], inp.aux_off[V]:inp.aux_off[V] + inp.naux[V]]
            assert rel(g, ref) <= BLOCK_BAR["bf16x3"], (t, U, V, R, rel(g, ref))
    del got
    torch.cuda.empty_cache()
