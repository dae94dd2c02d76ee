"""Seeded input generator: determinism and the identities its outputs must satisfy."""
import numpy as np
import pytest

from rpa_synth import make_inputs
from rpa_synth.configs import micro_cell, config
from rpa_synth.inputs import green_functions, GAP
from tests._util import micro, cfg


def test_seeded_inputs_are_reproducible():
    a = make_inputs(micro_cell(3, mesh=(2, 1, 1)))
    b = make_inputs(micro_cell(3, mesh=(2, 1, 1)))
    assert np.array_equal(a.blocks.C, b.blocks.C)
    assert np.array_equal(a.Gocc, b.Gocc) and np.array_equal(a.Gun, b.Gun)
    assert np.array_equal(a.vq, b.vq)
    c = make_inputs(micro_cell(4, mesh=(2, 1, 1)))
    assert not np.array_equal(a.blocks.C[:10], c.blocks.C[:10])


@pytest.mark.parametrize("spec", [dict(), dict(natoms=3, nao=(2, 5, 3), naux=(3, 6, 2), mesh=(3, 1, 2))])
def test_green_completeness_trace_and_symmetry(spec):
    inp = micro(**spec)
    # completeness at tau = 0: G^occ(R,0) + G^un(R,0) = delta_{R,0} I  (Eq. (green_mat), f + (1-f) = 1)
    go, gu = green_functions(inp.eps, inp.wfc, inp.nocc, inp.mu, np.array([0.0]), inp.kfrac, inp.Rvec)
    tot = go[0] + gu[0]
    ref = np.zeros_like(tot)
    ref[0] = np.eye(inp.nb)
    assert np.max(np.abs(tot - ref)) < 1e-12
    # trace of the occupied projector in the home cell = number of occupied bands per k
    assert abs(np.trace(go[0, 0]) - inp.nocc) < 1e-12
    # real Hermitian: G(-R) = G(R)^T
    mesh = np.array(inp.cell.mesh)
    for r, n in enumerate(inp.Rvec):
        m = np.mod(-n, mesh)
        rm = (m[0] * mesh[1] + m[1]) * mesh[2] + m[2]
        for G in (inp.Gocc, inp.Gun):
            assert np.max(np.abs(G[:, rm] - np.swapaxes(G[:, r], 1, 2))) < 1e-13


def test_gap_and_chemical_potential():
    inp = micro(mesh=(2, 2, 1))
    vbm = inp.eps[:, :inp.nocc].max()
    cbm = inp.eps[:, inp.nocc:].min()
    assert abs((cbm - vbm) - GAP) < 1e-12
    assert vbm < inp.mu < cbm


@pytest.mark.parametrize("spec", [dict(natoms=3, nao=(2, 3, 4), naux=(2, 3, 4), mesh=(2, 2, 2)),
                                  # cutoff equal to the cell edge: images sit exactly on the cutoff
                                  dict(seed=7, natoms=2, nao=(17, 9), naux=(33, 18), mesh=(2, 1, 1), rcut=4.0,
                                       edge=4.0)])
def test_neighbour_list_is_symmetric_and_inside_cutoff(spec):
    inp = micro(**spec)
    b = inp.blocks
    keys = {(int(i), int(k), tuple(r)) for i, k, r in zip(b.I, b.K, b.R.tolist())}
    for i, k, r in list(keys):
        assert (k, i, tuple(-x for x in r)) in keys
    assert np.all(b.d < inp.cell.rcut)
    # every atom sees itself in the home cell
    for a in range(inp.natoms):
        assert (a, a, (0, 0, 0)) in keys


def test_config_shapes_match_workloads():
    c0 = cfg(0, with_coulomb=False)
    assert (c0.nb, c0.nauxtot, c0.nR, c0.ntau) == (26, 80, 8, 8)
    assert all(np.sum(c0.blocks.I == a) == 36 for a in range(2))
    c2 = config(2)
    assert c2.natoms == 32 and sorted(set(c2.species)) == ["A", "B"]
    assert int(c2.nao.sum()) == 24 * 13 + 8 * 26 and int(c2.naux.sum()) == 24 * 60 + 8 * 120
    c3 = config(3)
    assert int(c3.nao.sum()) == 1924 and int(c3.naux.sum()) == 7440


def test_grids_fit_quality():
    inp = cfg(0, with_coulomb=False)
    gi = inp.grid_info
    assert gi["tau_fit_err"] < 1e-2 and gi["omega_fit_err"] < 1e-2
    assert np.all(np.isfinite(inp.gamma_cos)) and np.all(inp.tau > 0) and np.all(inp.womega > 0)
    assert np.all(np.diff(inp.tau) > 0) and np.all(np.diff(inp.omega) > 0)


def test_coulomb_is_hermitian_positive_definite():
    inp = micro()
    for v in inp.vq:
        assert np.allclose(v, v.conj().T, atol=1e-14)
        lam = np.linalg.eigvalsh(v)
        assert lam.min() > 0 and abs(lam.max() - inp.cell.v_scale) < 1e-12
