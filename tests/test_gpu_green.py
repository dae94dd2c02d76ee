"""GPU parity of the Green's-function build (build_chi0_tau's inputs, Eq. (green_mat)) against the
FP64 oracle (oracle.green) on the same seeded eigenpairs: FP64 throughout, so the bar is the
FP64 one, max |G_gpu - G_oracle| <= 1e-12 max |G|.  Cases: the tiny workload, ragged sizes
(10 NAOs, odd mesh), no occupied and no unoccupied bands, Gamma only, and the 8-atom workload
at full size (4 of its 16 tau points).  The GPU-built G then feeds the FP64 chi0 build, which
must meet its own bar against the oracle chi."""
import sys

import numpy as np
import pytest

from oracle import chi0 as ochi
from oracle.green import green_tau
from tests._gpu import rel
from tests._util import cfg, micro

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_green(ctx, inp, tau, nocc=None):
    import torch
    from paper_2407_19930_amd import build_green_tau, rpa_green_workspace_size
    nocc = inp.nocc if nocc is None else nocc
    nk, nb = inp.eps.shape
    eps = torch.from_numpy(np.ascontiguousarray(inp.eps)).cuda()
    wfc = torch.from_numpy(np.ascontiguousarray(inp.wfc)).cuda()
    ws = torch.empty(rpa_green_workspace_size(nk, nb, nocc), dtype=torch.uint8, device="cuda")
    shape = (len(tau), inp.nR, nb, nb)
    Go = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
    Gu = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
    build_green_tau(ctx, eps, wfc, nocc, inp.mu, tau, inp.cell.mesh, inp.kfrac, ws, Go, Gu)
    torch.cuda.synchronize()
    return Go, Gu


def _check(inp, tau, Go, Gu, nocc=None):
    nocc = inp.nocc if nocc is None else nocc
    ro, ru, im = green_tau(inp.eps, inp.wfc, nocc, inp.mu, tau, inp.kfrac, inp.Rvec)
    scale = max(np.abs(ro).max(), np.abs(ru).max())
    eo = np.abs(Go.cpu().numpy() - ro).max() / scale
    eu = np.abs(Gu.cpu().numpy() - ru).max() / scale
    say("  occ err %.3g, un err %.3g (oracle imag %.3g)" % (eo, eu, im / scale))
    assert eo <= 1e-12 and eu <= 1e-12
    return ro, ru


CASES = {"tiny": lambda: cfg(0, with_coulomb=False),
         "ragged": lambda: micro(seed=2, natoms=3, nao=(2, 5, 3), naux=(3, 6, 2), mesh=(3, 1, 2)),
         "gamma": lambda: micro(seed=5, natoms=2, nao=(7, 4), naux=(3, 3), mesh=(1, 1, 1), rcut=3.5, edge=4.0)}


@pytest.mark.parametrize("case", list(CASES))
def test_green_matches_oracle(case):
    from paper_2407_19930_amd import Context
    inp = CASES[case]()
    say("case green", case, "nb", inp.nb, "mesh", tuple(inp.cell.mesh), "ntau", inp.ntau)
    ctx = Context(0)
    Go, Gu = gpu_green(ctx, inp, inp.tau)
    _check(inp, inp.tau, Go, Gu)


@pytest.mark.parametrize("nocc", ["none", "all"])
def test_green_empty_channel(nocc):
    from paper_2407_19930_amd import Context
    inp = CASES["ragged"]()
    n = 0 if nocc == "none" else inp.nb
    say("case green nocc", n)
    ctx = Context(0)
    Go, Gu = gpu_green(ctx, inp, inp.tau[:2], nocc=n)
    _check(inp, inp.tau[:2], Go, Gu, nocc=n)
    assert float((Go if n == 0 else Gu).abs().max()) == 0.0


def test_green_feeds_the_fp64_chi0_build():
    import torch
    from paper_2407_19930_amd import Context, build_chi0_tau
    from tests._gpu import make_plan
    inp = CASES["tiny"]()
    say("case green -> chi0 fp64")
    ctx = Context(0)
    Go, Gu = gpu_green(ctx, inp, inp.tau)
    plan = make_plan(ctx, inp, "fp64")
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    chi = torch.empty((inp.ntau, inp.nR, inp.nauxtot, inp.nauxtot), dtype=torch.float64, device="cuda")
    C = torch.from_numpy(inp.blocks.C).cuda()
    build_chi0_tau(plan, inp.spin_factor, Go, Gu, C, ws, chi)
    torch.cuda.synchronize()
    e = rel(chi.cpu().numpy(), ochi.chi0_alg1(inp))
    say("  chi rel err %.3g" % e)
    assert e <= 1e-11
    plan.close()


def test_green_full_size_diamond():
    from paper_2407_19930_amd import Context
    inp = cfg(1, with_coulomb=False)
    tau = inp.tau[[0, 5, 10, 15]]
    say("case green full size: nb", inp.nb, "nk", len(inp.kfrac), "tau", len(tau))
    ctx = Context(0)
    Go, Gu = gpu_green(ctx, inp, tau)
    _check(inp, tau, Go, Gu)


def test_green_errors():
    import torch
    from paper_2407_19930_amd import Context, RpaError, build_green_tau
    from paper_2407_19930_amd.binding import RPA_ERR_ARG, RPA_ERR_UNSUPPORTED, RPA_ERR_WORKSPACE
    inp = CASES["ragged"]()
    say("case green errors")
    ctx = Context(0)
    nk, nb = inp.eps.shape
    eps = torch.from_numpy(inp.eps).cuda()
    wfc = torch.from_numpy(inp.wfc).cuda()
    G = torch.empty((1, inp.nR, nb, nb), dtype=torch.float64, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(RpaError) as e:
        build_green_tau(ctx, eps, wfc, inp.nocc, inp.mu, inp.tau[:1], inp.cell.mesh, inp.kfrac, small, G, G)
    assert e.value.code == RPA_ERR_WORKSPACE
    big = torch.empty(1 << 24, dtype=torch.uint8, device="cuda")
    with pytest.raises(RpaError) as e:
        build_green_tau(ctx, eps, wfc, nb + 1, inp.mu, inp.tau[:1], inp.cell.mesh, inp.kfrac, big, G, G)
    assert e.value.code == RPA_ERR_ARG
    # 4096 phases at most: a 65-point mesh with this cell's k list exceeds it
    k = np.repeat(inp.kfrac, 11, axis=0)[:nk * 11]
    eps11 = eps.repeat(11, 1)
    wfc11 = wfc.repeat(11, 1, 1)
    G65 = torch.empty((1, 65 * 1 * 1, nb, nb), dtype=torch.float64, device="cuda")
    with pytest.raises(RpaError) as e:
        build_green_tau(ctx, eps11, wfc11, inp.nocc, inp.mu, inp.tau[:1], (65, 1, 1), k, big, G65, G65)
    assert e.value.code == RPA_ERR_UNSUPPORTED
