"""Launch variants of the chi0 kernels and the autotuner (rpa_plan_autotune / _get_tuning /
_set_tuning).  Every variant must compute the same chi: the XCD-grouped tile and item orders
bitwise (each tile and item writes its own outputs), the N-stage K step within the path's
tolerance against the oracle.  chi is filled with NaN before every build, so a tile or item
that a permuted order dropped would show."""
import sys

import numpy as np
import pytest

from oracle import chi0 as ochi
from tests._gpu import device_inputs, make_plan, rel
from tests._util import cfg, micro

pytestmark = pytest.mark.gpu

CHI_TOL = {"fp64": 1e-11, "fp32": 1e-5, "bf16x3": 1e-5}
CASES = {"tiny": lambda: cfg(0),
         "ragged": lambda: micro(seed=2, natoms=3, nao=(2, 5, 3), naux=(3, 6, 2), mesh=(3, 1, 2)),
         # 128 ABF on one atom: both halves of the 4-wave single launch carry columns
         "wide": lambda: micro(seed=8, natoms=2, nao=(32, 1), naux=(128, 1), mesh=(2, 1, 1), rcut=3.5, edge=4.0)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cases():
    out = {}
    for name, make in CASES.items():
        inp = make()
        out[name] = (inp, ochi.chi0_alg1(inp))
    return out


def _build(ctx, plan, inp, d, ws):
    import torch
    from paper_2407_19930_amd import build_chi0_tau
    chi = torch.full((inp.ntau, inp.nR, inp.nauxtot, inp.nauxtot), float("nan"), dtype=torch.float64, device="cuda")
    build_chi0_tau(plan, inp.spin_factor, d["Gocc"], d["Gun"], d["C"], ws, chi)
    torch.cuda.synchronize()
    return chi.cpu().numpy()


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_every_variant_computes_the_same_chi(cases, case, precision):
    import torch
    from paper_2407_19930_amd import Context
    inp, ref = cases[case]
    say("case variants", case, precision)
    ctx = Context(0)
    plan = make_plan(ctx, inp, precision)
    d = device_inputs(inp)
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    t0 = plan.tuning
    assert (t0.nstage_order, t0.fused_order, t0.from_cache) == (0, 0, 0)
    ksteps = [0] if t0.nstage_kstep == 0 else [16, 32]
    assert t0.nstage_kstep in (0, 16)
    base = {}
    bms = (128, 256) if precision == "bf16x3" else (128,)
    for k in ksteps:
        for bm in bms:
            for no in (0, 1):
                for fo in (0, 1):
                    plan.set_tuning(no, k, fo, 0, bm)
                    chi = _build(ctx, plan, inp, d, ws)
                    e = rel(chi, ref)
                    say("  kstep %d bm %d nstage_order %d fused_order %d: rel err %.3g" % (k, bm, no, fo, e))
                    assert np.all(np.isfinite(chi))
                    assert e <= CHI_TOL[precision]
                    if k not in base:
                        base[k] = chi
                    else:
                        assert np.array_equal(chi, base[k])     # orders, tile rows: bitwise the same chi
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_autotune_choice_cache_and_result(cases, precision):
    import torch
    from paper_2407_19930_amd import Context
    inp, ref = cases["tiny"]
    say("case autotune", precision)
    ctx = Context(0)
    d = device_inputs(inp)
    plan = make_plan(ctx, inp, precision)
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    scratch = torch.empty(inp.nR * inp.nauxtot ** 2, dtype=torch.float64, device="cuda")
    t = plan.autotune(inp.spin_factor, d["Gocc"], d["Gun"], d["C"], ws, scratch)
    say("  tuned", t.as_dict())
    assert t.from_cache == 0 and t.nstage_ms > 0 and t.fused_ms > 0
    assert t.nstage_order in (0, 1) and t.fused_order in (0, 1)
    assert t.nstage_kstep in ((0,) if precision == "bf16x3" else (16, 32))
    got = plan.tuning
    assert (got.nstage_order, got.nstage_kstep, got.fused_order) == (t.nstage_order, t.nstage_kstep, t.fused_order)
    # the scratch holds chi of the first tau
    assert rel(scratch.view(inp.nR, inp.nauxtot, inp.nauxtot).cpu().numpy(), ref[0]) <= CHI_TOL[precision]
    chi = _build(ctx, plan, inp, d, ws)
    assert rel(chi, ref) <= CHI_TOL[precision]
    # a second plan of the same shape class takes the cached choice without timing
    plan2 = make_plan(ctx, inp, precision)
    t2 = plan2.autotune(inp.spin_factor, d["Gocc"], d["Gun"], d["C"], ws, scratch)
    say("  second plan", t2.as_dict())
    assert t2.from_cache == 1 and t2.nstage_ms == 0 and t2.fused_ms == 0
    assert (t2.nstage_order, t2.nstage_kstep, t2.fused_order) == (t.nstage_order, t.nstage_kstep, t.fused_order)
    assert np.array_equal(_build(ctx, plan2, inp, d, ws), chi)
    # another precision is another class
    plan3 = make_plan(ctx, inp, "fp64")
    t3 = plan3.autotune(inp.spin_factor, d["Gocc"], d["Gun"], d["C"], torch.empty(max(plan3.workspace_bytes, 1),
                        dtype=torch.uint8, device="cuda"), scratch)
    assert t3.from_cache == 0
    for p in (plan, plan2, plan3):
        p.close()


def test_set_tuning_rejects_out_of_range(cases):
    from paper_2407_19930_amd import Context, RpaError
    from paper_2407_19930_amd.binding import RPA_ERR_ARG
    inp, _ = cases["tiny"]
    say("case tuning errors")
    ctx = Context(0)
    plan = make_plan(ctx, inp, "fp32")
    plan.set_tuning(1, 32, 1)
    for bad in ((2, 16, 0), (0, 24, 0), (0, 16, -1), (0, 0, 0), (0, 16, 0, 0, 256)):
        with pytest.raises(RpaError) as e:
            plan.set_tuning(*bad)
        assert e.value.code == RPA_ERR_ARG
    with pytest.raises(RpaError) as e:
        plan.set_tuning(0, 16, 0, 1)         # the single fused launch is a split-BF16 variant
    assert e.value.code == RPA_ERR_ARG
    t = plan.tuning
    assert (t.nstage_order, t.nstage_kstep, t.fused_order) == (1, 32, 1)
    pb = make_plan(ctx, inp, "bf16x3")
    with pytest.raises(RpaError):
        pb.set_tuning(0, 16, 0)             # the split-BF16 N stage has no K-step choice
    pb.set_tuning(1, 0, 1)
    pb.set_tuning(0, 0, 0, 1)
    pb.set_tuning(0, 0, 0, 3)
    with pytest.raises(RpaError) as e:
        pb.set_tuning(0, 0, 0, 4)           # no such fused launch shape
    assert e.value.code == RPA_ERR_ARG
    for bad in (0, inp.ntau + 1):
        with pytest.raises(RpaError) as e:
            pb.set_tau_batch(bad)
        assert e.value.code == RPA_ERR_ARG
    plan.close()
    pb.close()


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_tau_batch_and_single_launch(cases, case, precision):
    """tau points per launch (rpa_plan_set_tau_batch) and the single fused launch over every
    template class: every combination gives bitwise the chi of the default launches (each tau,
    tile and item is computed by the same instructions, only the launches differ), with screening
    off and on (the same kept-term counts)."""
    import torch
    from paper_2407_19930_amd import Context
    inp, ref = cases[case]
    say("case tau batch", case, precision)
    ctx = Context(0)
    d = device_inputs(inp)
    for theta in (0.0, 0.05):
        plan = make_plan(ctx, inp, precision)
        if theta:
            plan.set_screening(theta)
        ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
        base = _build(ctx, plan, inp, d, ws)
        assert np.all(np.isfinite(base))
        if not theta:
            assert rel(base, ref) <= CHI_TOL[precision]
        stats = plan.screening_stats() if theta else None
        k0 = plan.tuning.nstage_kstep
        for slots in sorted({1, 2, inp.ntau}):
            grow = plan.set_tau_batch(slots)
            ws = torch.empty(max(grow, 1), dtype=torch.uint8, device="cuda")
            for single in ((0, 1, 2, 3) if precision == "bf16x3" else (0,)):
                plan.set_tuning(0, k0, 0, single)
                chi = _build(ctx, plan, inp, d, ws)
                say("  theta %g slots %d single %d: equal %s" % (theta, slots, single, np.array_equal(chi, base)))
                assert np.array_equal(chi, base)
                if theta:
                    assert plan.screening_stats() == stats
        plan.close()
