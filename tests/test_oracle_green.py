"""Pins of the Green's-function oracle (oracle.green, Eq. (green_mat)) against facts that do not
come from its own formula: completeness and the trace (from the band energies alone), the
transpose symmetry of a time-reversal-symmetric H, the semigroup property in imaginary time
(a convolution over the BvK mesh), and the first-order expansion in tau for a Hamiltonian
built from known real-space hoppings (fixes the sign of the Bloch phase and which factor is
conjugated: the wrong choice returns h(-R) = h(R)^T instead of h(R))."""
import numpy as np
import pytest

from oracle.green import green_tau
from rpa_synth import lattice as lat
from tests._util import cfg


@pytest.fixture(scope="module")
def tiny():
    return cfg(0, with_coulomb=False)


def _minus(Rvec, mesh):
    return lat.fold_index(-np.asarray(Rvec), mesh)


def test_completeness_and_trace(tiny):
    inp = tiny
    Go, Gu, im = green_tau(inp.eps, inp.wfc, inp.nocc, inp.mu, [0.0], inp.kfrac, inp.Rvec)
    delta = np.zeros_like(Go[0])
    delta[0] = np.eye(inp.nb)                      # R = 0 is the first BvK vector
    assert np.abs(Go[0] + Gu[0] - delta).max() <= 1e-12
    assert im <= 1e-12
    Go, Gu, im = green_tau(inp.eps, inp.wfc, inp.nocc, inp.mu, inp.tau, inp.kfrac, inp.Rvec)
    assert im <= 1e-12 * np.abs(Go).max()
    nk = len(inp.kfrac)
    for t, tt in enumerate(inp.tau):
        e = inp.eps
        tr_occ = np.exp(-(inp.mu - e[:, :inp.nocc]) * tt).sum() / nk
        tr_un = np.exp(-(e[:, inp.nocc:] - inp.mu) * tt).sum() / nk
        assert abs(np.trace(Go[t, 0]) - tr_occ) <= 1e-12 * tr_occ
        assert abs(np.trace(Gu[t, 0]) - tr_un) <= 1e-12 * tr_un


def test_transpose_symmetry(tiny):
    inp = tiny
    Go, Gu, _ = green_tau(inp.eps, inp.wfc, inp.nocc, inp.mu, inp.tau[:3], inp.kfrac, inp.Rvec)
    mR = _minus(inp.Rvec, inp.cell.mesh)
    for G in (Go, Gu):
        assert np.abs(G[:, mR] - np.swapaxes(G, 2, 3)).max() <= 1e-13 * np.abs(G).max()


def test_semigroup_in_imaginary_time(tiny):
    """sum_{R'} G^s(R', t1) G^s(R - R', t2) = G^s(R, t1 + t2) for both channels."""
    inp = tiny
    t1, t2 = inp.tau[1], inp.tau[4]
    G1o, G1u, _ = green_tau(inp.eps, inp.wfc, inp.nocc, inp.mu, [t1], inp.kfrac, inp.Rvec)
    G2o, G2u, _ = green_tau(inp.eps, inp.wfc, inp.nocc, inp.mu, [t2], inp.kfrac, inp.Rvec)
    G3o, G3u, _ = green_tau(inp.eps, inp.wfc, inp.nocc, inp.mu, [t1 + t2], inp.kfrac, inp.Rvec)
    Rv, mesh = inp.Rvec, inp.cell.mesh
    for A, B, C in ((G1o, G2o, G3o), (G1u, G2u, G3u)):
        for r in range(len(Rv)):
            acc = np.zeros((inp.nb, inp.nb))
            for rp in range(len(Rv)):
                acc += A[0, rp] @ B[0, lat.fold_index(Rv[r] - Rv[rp], mesh)]
            assert np.abs(acc - C[0, r]).max() <= 1e-12 * max(np.abs(C).max(), 1e-300)


def test_first_order_in_tau_recovers_the_hoppings():
    """H(k) = sum_R e^{i k.R} h(R) from known hoppings on a 4-cell ring; then
    [G^un(R, d) + G^occ(R, -d) - delta_{R0} I] / d = -(h(R) - mu delta_{R0} I) + O(d)."""
    rng = np.random.default_rng(11)
    nb, mesh = 3, (4, 1, 1)
    h0 = rng.standard_normal((nb, nb))
    h0 = (h0 + h0.T) / 2
    h1 = rng.standard_normal((nb, nb))             # not symmetric: h(-R) = h(R)^T differs
    hop = {(0, 0, 0): h0, (1, 0, 0): h1, (-1, 0, 0): h1.T}
    kfrac = lat.kmesh(mesh)
    Rvec = lat.bvk_vectors(mesh)
    H = np.zeros((len(kfrac), nb, nb), dtype=np.complex128)
    for R, h in hop.items():
        H += np.exp(2j * np.pi * (kfrac @ np.asarray(R)))[:, None, None] * h[None]
    eps, wfc = np.linalg.eigh(H)
    mu, nocc, d = 0.3, 1, 1e-6
    Go, _, _ = green_tau(eps, wfc, nocc, mu, [-d], kfrac, Rvec)
    _, Gu, _ = green_tau(eps, wfc, nocc, mu, [d], kfrac, Rvec)
    expect = np.zeros((len(Rvec), nb, nb))
    for R, h in hop.items():
        expect[lat.fold_index(np.asarray(R), mesh)] += h
    expect[0] -= mu * np.eye(nb)
    got = -(Go[0] + Gu[0] - np.eye(nb)[None] * (np.arange(len(Rvec)) == 0)[:, None, None]) / d
    assert np.abs(got - expect).max() <= 1e-4
    # the mistaken conventions give the transposed hoppings, far from these
    assert np.abs(got[1] - h1.T).max() > 0.1
