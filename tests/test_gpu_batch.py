"""Batches of independent cells in one captured HIP graph (rpa_batch_*), on cells of the
serving workload (2-16 atoms, k-meshes 1x1x1, 2x2x2 and 3x3x3, 8-16 tau).

Every cell's E_c from the graph equals the one-cell API bitwise (same kernels in the same
order within a cell; lanes only change which cells overlap), replays of the graph with the
program's own eager work and synchronisations between them agree with the first one, and on
the cells small enough for the oracle both mixed paths meet the bar of 1e-6 Ha/atom."""
import sys

import numpy as np
import pytest

from oracle import chi0 as ochi
from oracle.pipeline import ec_from_chi_tau
from rpa_synth import make_inputs
from rpa_synth.configs import serving_cells
from tests._gpu import batch_cell, device_inputs, gpu_pipeline

pytestmark = pytest.mark.gpu

SMALL = [4, 7, 10, 14]      # 2, 2, 3, 4 atoms, Gamma only: the oracle takes seconds
LARGER = [2, 6, 27]         # 8 atoms on a 2x2x2 k-mesh; 3 atoms on a 3x3x3 k-mesh


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cells():
    allc = serving_cells()
    return {i: make_inputs(allc[i]) for i in SMALL + LARGER}


@pytest.fixture(scope="module")
def oracle_ec(cells):
    out = {}
    for i in SMALL:
        inp = cells[i]
        out[i] = ec_from_chi_tau(inp, ochi.chi0_alg1(inp))[0]
    return out


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_batch_graph_matches_single_cell_and_oracle(cells, oracle_ec, precision):
    import torch
    from paper_2407_19930_amd import Context
    from paper_2407_19930_amd.batching import make_batch
    ids = SMALL + LARGER
    say("case batch graph", precision, "serving cells", ids)
    ctx = Context(0)
    dev = {i: device_inputs(cells[i]) for i in ids}
    batch, plans, lanes = make_batch(ctx, [batch_cell(cells[i], dev[i]) for i in ids], nlanes=2,
                                     precision=precision)
    say("  lanes", lanes)
    batch.run()
    ec, ecq = batch.result()
    for k, i in enumerate(ids):
        inp = cells[i]
        single = gpu_pipeline(inp, precision, ctx=ctx)["ec"]
        say("  cell %d (%d atoms, mesh %s, %d tau): E_c batch %.15g single %.15g"
            % (i, inp.natoms, tuple(inp.cell.mesh), inp.ntau, ec[k], single))
        assert ec[k] == single
        if i in SMALL:
            d = abs(ec[k] - oracle_ec[i]) / inp.natoms
            say("    oracle %.15g, dE/atom %.3g" % (oracle_ec[i], d))
            assert d <= 1e-6
    assert np.all(ec < 0)
    for rep in range(3):
        x = torch.randn(1 << 20, device="cuda")
        float((x * 2.0).sum())                 # eager work and a synchronisation between replays
        batch.run()
        ec2, ecq2 = batch.result()
        say("  replay %d identical: %s" % (rep, bool(np.array_equal(ec2, ec) and np.array_equal(ecq2, ecq))))
        assert np.array_equal(ec2, ec) and np.array_equal(ecq2, ecq)
    batch.close()


def test_batch_rejects_bad_cells(cells):
    import torch
    from paper_2407_19930_amd import Batch, Context, RpaError
    from paper_2407_19930_amd.binding import RPA_ERR_ARG, RPA_ERR_WORKSPACE
    from tests._gpu import make_plan
    inp = cells[SMALL[0]]
    say("case batch errors")
    ctx = Context(0)
    c = batch_cell(inp)
    plan = make_plan(ctx, inp, "fp32")
    n, nR = inp.nauxtot, inp.nR
    nw, nq = len(inp.omega), len(inp.kfrac)
    x = torch.empty(max(inp.ntau, 2 * nw) * nR * n * n, dtype=torch.float64, device="cuda")
    io = dict(plan=plan, lane=0, spin_factor=c["spin_factor"], gamma_cos=c["gamma_cos"], womega=c["womega"],
              q_frac=c["q_frac"], G_occ=c["G_occ"], G_un=c["G_un"], C=c["C"], v_q=c["v_q"],
              build_workspace=torch.empty(16, dtype=torch.uint8, device="cuda"),
              chi0_tau=x[:inp.ntau * nR * n * n],
              chi0_omega=torch.empty(nw * nR * n * n, dtype=torch.float64, device="cuda"),
              chi0_q=x[:2 * nw * nR * n * n].view(torch.complex128),
              ec_workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    with pytest.raises(RpaError) as e:
        Batch(ctx, [io], 1)
    assert e.value.code == RPA_ERR_WORKSPACE and "cell 0" in str(e.value)
    with pytest.raises(RpaError) as e:
        Batch(ctx, [dict(io, lane=1)], 1)
    assert e.value.code == RPA_ERR_ARG
