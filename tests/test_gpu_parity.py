"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded inputs.

Tolerances (stated by the target of the path): FP64 path relative Frobenius error of chi <= 1e-11;
mixed paths (FP32, split-BF16 3-term) <= 1e-5 and |dE_c| <= 1e-6 Ha/atom."""
import sys

import numpy as np
import pytest

from oracle import chi0 as ochi
from oracle.energy import correlation_energy, ec_terms_lu
from oracle.pipeline import ec_from_chi_tau
from oracle.transforms import cos_transform, fourier_R_to_q
from tests._util import micro, cfg
from tests._gpu import device_inputs, gpu_chi_tau, gpu_pipeline, rel

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11
FP32_TOL = 1e-5
CHI_TOL = {"fp64": FP64_TOL, "fp32": FP32_TOL, "bf16x3": FP32_TOL}
# per block (U, V) over all tau and R: an operand carried in 16 (split BF16) or 24 (FP32) bits
# leaves single blocks scattered around the whole-tensor error
BLOCK_TOL = {"fp64": FP64_TOL, "fp32": 3e-5, "bf16x3": 3e-5}
EC_TOL = {"fp64": 1e-10, "fp32": 1e-6, "bf16x3": 1e-6}      # Ha/atom
PRECISIONS = ["fp64", "fp32", "bf16x3"]

MICRO = [
    dict(),                                                                        # 2 atoms, mesh 3x2x1
    dict(seed=2, natoms=3, nao=(2, 5, 3), naux=(3, 6, 2), mesh=(3, 1, 2)),         # ragged, tiny tiles
    dict(seed=5, natoms=1, nao=(4,), naux=(5,), mesh=(4, 1, 1), rcut=5.0),         # images fold twice
    dict(seed=7, natoms=2, nao=(17, 9), naux=(33, 18), mesh=(2, 1, 1), rcut=4.0, edge=4.0),  # >16 NAO, >2 mu tiles
    dict(seed=8, natoms=2, nao=(32, 1), naux=(128, 1), mesh=(1, 1, 1), rcut=3.5, edge=4.0),  # kernel limits
]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def oracle_cache():
    return {}


def _oracle_chi(inp, key, cache):
    if key not in cache:
        cache[key] = ochi.chi0_alg1(inp)
    return cache[key]


def _check_blocks(inp, got, ref, precision):
    """Every atom-pair block chi_UV (all tau and R) within the per-block bar, relative to the
    block where it is not negligible (above 1e-3 of the largest block), else to the largest
    entry; returns the worst relative block error."""
    scale = np.abs(ref).max()
    norms = {}
    for U in range(inp.natoms):
        for V in range(inp.natoms):
            mu = slice(inp.aux_off[U], inp.aux_off[U] + inp.naux[U])
            nu = slice(inp.aux_off[V], inp.aux_off[V] + inp.naux[V])
            norms[U, V] = (np.linalg.norm(ref[:, :, mu, nu]), mu, nu)
    big = max(n for n, _, _ in norms.values())
    worst = 0.0
    for (U, V), (n, mu, nu) in norms.items():
        g, r = got[:, :, mu, nu], ref[:, :, mu, nu]
        if n > 1e-3 * big:
            e = rel(g, r)
            worst = max(worst, e)
            assert e <= BLOCK_TOL[precision], (U, V, e)
        else:
            assert np.abs(g - r).max() <= BLOCK_TOL[precision] * scale, (U, V)
    return worst


@pytest.mark.parametrize("idx", range(len(MICRO)))
@pytest.mark.parametrize("precision", PRECISIONS)
def test_chi_tau_micro(idx, precision, oracle_cache):
    spec = MICRO[idx]
    inp = micro(**spec)
    say("case chi_tau micro", idx, precision, spec)
    ref = _oracle_chi(inp, ("micro", idx), oracle_cache)
    chi, _, _ = gpu_chi_tau(inp, precision)
    got = chi.cpu().numpy()
    err = rel(got, ref)
    assert np.all(np.isfinite(got))
    assert err <= CHI_TOL[precision]
    worst = _check_blocks(inp, got, ref, precision)
    say("  rel err", err, "worst block", worst)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_chi_tau_tiny_workload(precision, oracle_cache):
    inp = cfg(0)
    say("case chi_tau tiny workload", precision)
    ref = _oracle_chi(inp, "cfg0", oracle_cache)
    chi, plan, _ = gpu_chi_tau(inp, precision)
    got = chi.cpu().numpy()
    err = rel(got, ref)
    per_tau = max(rel(got[t], ref[t]) for t in range(inp.ntau))
    worst = _check_blocks(inp, got, ref, precision)
    say("  rel err", err, "max per-tau", per_tau, "worst block", worst, "flops", plan.flops())
    assert err <= CHI_TOL[precision]
    # the stricter per-tau maximum of the chi error (one reading of its metric) within the same bar
    assert per_tau <= CHI_TOL[precision]


@pytest.mark.parametrize("case", ["cfg0", "micro1"])
@pytest.mark.parametrize("precision", PRECISIONS)
def test_chi_tau_block_order(case, precision, oracle_cache):
    """The plan groups each atom's LRI blocks by neighbour atom itself (the fused kernels walk
    the periodic images of one neighbour atom together): the same blocks passed in a random
    order (permuted block list over the same C buffer) give chi within the same bar."""
    import dataclasses
    inp, key = (cfg(0), "cfg0") if case == "cfg0" else (micro(**MICRO[1]), ("micro", 1))
    b = inp.blocks
    perm = np.random.default_rng(1234).permutation(len(b.I))
    shuffled = dataclasses.replace(inp, blocks=dataclasses.replace(
        b, I=b.I[perm], K=b.K[perm], R=b.R[perm], d=b.d[perm], off=b.off[perm]))
    say("case chi_tau block order", case, precision, "blocks", len(perm))
    ref = _oracle_chi(inp, key, oracle_cache)
    chi, _, _ = gpu_chi_tau(shuffled, precision)
    got = chi.cpu().numpy()
    err = rel(got, ref)
    say("  rel err", err)
    assert np.all(np.isfinite(got))
    assert err <= CHI_TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_tau_rescale_is_exact(precision):
    """G scaled by 2^-80: without the per-tau power-of-two scale the FP32 products (~1e-54) would
    underflow to zero; with it every device intermediate is unchanged, so chi must come out
    scaled by exactly 2^-160 (bitwise equal after undoing it)."""
    inp = micro(**MICRO[3])
    say("case tau rescale", precision)
    d = device_inputs(inp)
    a, _, ctx = gpu_chi_tau(inp, precision, dev_in=d)
    s = 2.0 ** -80
    b, _, _ = gpu_chi_tau(inp, precision, ctx=ctx, dev_in=dict(Gocc=d["Gocc"] * s, Gun=d["Gun"] * s, C=d["C"]))
    scaled = b * 2.0 ** 160
    say("  max abs chi", float(a.abs().max()), "max abs difference", float((scaled - a).abs().max()))
    assert float(a.abs().max()) > 0
    assert bool((scaled == a).all())


def test_transforms_match_oracle_on_same_input():
    """cosine and R->q transforms of the GPU applied to the oracle's chi(R, tau)."""
    import torch
    from paper_2407_19930_amd import Context, chi0_R_to_q, chi0_tau_to_omega
    inp = micro(**MICRO[1])
    say("case transforms")
    ref_tau = ochi.chi0_alg1(inp)
    ctx = Context(0)
    x = torch.from_numpy(ref_tau).cuda()
    nw = len(inp.omega)
    y = torch.empty((nw,) + ref_tau.shape[1:], dtype=torch.float64, device="cuda")
    chi0_tau_to_omega(ctx, inp.gamma_cos, x, y)
    q = torch.empty((nw, len(inp.kfrac)) + ref_tau.shape[2:], dtype=torch.complex128, device="cuda")
    chi0_R_to_q(ctx, inp.cell.mesh, inp.kfrac, y, q)
    torch.cuda.synchronize()
    ref_w = cos_transform(ref_tau, inp.gamma_cos)
    ref_q = fourier_R_to_q(ref_w, inp.Rvec, inp.kfrac)
    assert rel(y.cpu().numpy(), ref_w) < 1e-14
    assert rel(q.cpu().numpy(), ref_q) < 1e-14


def test_correlation_energy_matches_lu_on_same_input():
    """GPU Cholesky log-det route against the oracle's LU route, on the oracle's chi(q, i omega)."""
    import torch
    from paper_2407_19930_amd import Context, rpa_correlation_energy, rpa_ec_workspace_size
    inp = cfg(0)
    say("case E_c same input")
    ec_ref, perq_ref, chi_q = ec_from_chi_tau(inp, _oracle_chi(inp, "cfg0", {}))
    ctx = Context(0)
    n, nq, nw = inp.nauxtot, len(inp.kfrac), len(inp.omega)
    ws = torch.empty(rpa_ec_workspace_size(n, nq, nw), dtype=torch.uint8, device="cuda")
    ec, perq = rpa_correlation_energy(ctx, inp.womega, torch.from_numpy(chi_q).cuda(),
                                      torch.from_numpy(inp.vq).cuda(), ws)
    say("  E_c gpu", ec, "oracle", ec_ref)
    assert ec < 0
    assert abs(ec - ec_ref) <= 1e-11 * abs(ec_ref)
    assert np.max(np.abs(perq - perq_ref)) <= 1e-11 * abs(ec_ref)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_pipeline_tiny_workload(precision, oracle_cache):
    inp = cfg(0)
    say("case pipeline tiny", precision)
    ec_ref, _, _ = ec_from_chi_tau(inp, _oracle_chi(inp, "cfg0", oracle_cache))
    out = gpu_pipeline(inp, precision)
    d = abs(out["ec"] - ec_ref) / inp.natoms
    say("  E_c/atom gpu", out["ec"] / inp.natoms, "oracle", ec_ref / inp.natoms, "dE/atom", d)
    assert d <= EC_TOL[precision]


def test_errors_are_reported():
    import torch
    from paper_2407_19930_amd import Context, Plan, RpaError, build_chi0_tau, rpa_correlation_energy, \
        rpa_ec_workspace_size
    from paper_2407_19930_amd.binding import (RPA_ERR_ARG, RPA_ERR_NONFINITE, RPA_ERR_NOT_HPD, RPA_ERR_SHAPE,
                                              RPA_ERR_UNSUPPORTED, RPA_ERR_WORKSPACE)
    inp = micro()
    ctx = Context(0)
    say("case error paths")
    with pytest.raises(RpaError) as e:
        Plan(ctx, [33], [4], (1, 1, 1), [0], [0], [[0, 0, 0]], [0], 2)
    assert e.value.code == RPA_ERR_UNSUPPORTED
    plan = Plan(ctx, inp.nao, inp.naux, inp.cell.mesh, inp.blocks.I, inp.blocks.K, inp.blocks.R, inp.blocks.off,
                inp.ntau)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    z = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(RpaError) as e:
        build_chi0_tau(plan, 2.0, z, z, z, small, z)
    assert e.value.code == RPA_ERR_WORKSPACE
    # a sign-flipped (positive) chi makes 1 - L^H chi L indefinite
    n, nq, nw = 8, 1, 2
    chi_q = torch.zeros((nw, nq, n, n), dtype=torch.complex128, device="cuda")
    chi_q[:, 0] = 3.0 * torch.eye(n, dtype=torch.complex128, device="cuda")
    vq = torch.eye(n, dtype=torch.complex128, device="cuda").reshape(1, n, n).contiguous()
    ws = torch.empty(rpa_ec_workspace_size(n, nq, nw), dtype=torch.uint8, device="cuda")
    with pytest.raises(RpaError) as e:
        rpa_correlation_energy(ctx, np.ones(nw), chi_q, vq, ws)
    assert e.value.code == RPA_ERR_NOT_HPD
    # a NaN in chi: non-finite, not merely indefinite
    chi_q.zero_()
    chi_q[1, 0, 2, 5] = float("nan")
    with pytest.raises(RpaError) as e:
        rpa_correlation_energy(ctx, np.ones(nw), chi_q, vq, ws)
    assert e.value.code == RPA_ERR_NONFINITE
    # and in v(q)
    chi_q.zero_()
    vq[0, 3, 3] = float("inf")
    with pytest.raises(RpaError) as e:
        rpa_correlation_energy(ctx, np.ones(nw), chi_q, vq, ws)
    assert e.value.code == RPA_ERR_NONFINITE
    # inconsistent shapes: a block whose atom index is outside the cell, a mesh of zero
    with pytest.raises(RpaError) as e:
        Plan(ctx, inp.nao, inp.naux, inp.cell.mesh, inp.blocks.I, np.where(inp.blocks.K == 0, len(inp.nao), inp.blocks.K),
             inp.blocks.R, inp.blocks.off, inp.ntau)
    assert e.value.code == RPA_ERR_SHAPE
    with pytest.raises(RpaError) as e:
        Plan(ctx, inp.nao, inp.naux, (1, 0, 1), inp.blocks.I, inp.blocks.K, inp.blocks.R, inp.blocks.off, inp.ntau)
    assert e.value.code == RPA_ERR_ARG


def test_green_symmetry_check():
    """rpa_check_green_symmetry accepts the generator's G (real and symmetric, G(-R) = G(R)^T) and
    rejects one entry of G^occ(R) moved off its partner."""
    import torch
    from paper_2407_19930_amd import Context, RpaError, rpa_check_green_symmetry
    from paper_2407_19930_amd.binding import RPA_ERR_ARG
    inp = micro(**MICRO[1])
    ctx = Context(0)
    Go = torch.from_numpy(inp.Gocc).cuda()
    Gu = torch.from_numpy(inp.Gun).cuda()
    dev = rpa_check_green_symmetry(ctx, inp.cell.mesh, Go, Gu, 1e-12)
    say("case G symmetry: rel dev %.3g" % dev)
    assert dev <= 1e-13
    Go[inp.ntau - 1, 1, 0, 1] += 1e-6 * float(Go.abs().max())
    with pytest.raises(RpaError) as e:
        rpa_check_green_symmetry(ctx, inp.cell.mesh, Go, Gu, 1e-12)
    assert e.value.code == RPA_ERR_ARG
    assert rpa_check_green_symmetry(ctx, inp.cell.mesh, Go, Gu, 1e-3) > 1e-8


def test_context_dropped_before_plan_and_batch():
    """A context, two plans, a batch and a session of it left in one reference cycle and collected
    by the garbage collector, which finalises them in an order of its own (the context may go
    first): every finaliser either destroys its object while the context lives or, once the
    context is closed, does nothing; the process carries on and builds chi as before."""
    import gc
    import torch
    from paper_2407_19930_amd import Context, Session
    from paper_2407_19930_amd.batching import make_batch
    from tests._gpu import batch_cell, make_plan
    inp = micro(**MICRO[1])
    ref, _, _ = gpu_chi_tau(inp, "fp64")
    ref = ref.cpu().numpy()

    def garbage():
        ctx = Context(0)
        plans = [make_plan(ctx, inp, p) for p in ("fp64", "bf16x3")]
        batch, bplans, _ = make_batch(ctx, [batch_cell(inp)], 1, "fp32")
        sess = Session(ctx)
        batch.run()
        torch.cuda.synchronize()
        ctx.cycle = [ctx, plans, batch, bplans, sess]

    for _ in range(3):
        garbage()
        gc.collect()
    a, _, _ = gpu_chi_tau(inp, "fp64")
    assert np.array_equal(a.cpu().numpy(), ref)
