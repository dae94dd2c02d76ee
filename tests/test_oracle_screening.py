"""Pins of the Green's-function-screened oracle (oracle/screening.py) on the CPU.

* theta = 0 drops nothing: bitwise Algorithm 1; theta > 1 drops every term: chi = 0 exactly
  (no product of two Green's-function bounds exceeds g^2).
* The block and neighbourhood bounds equal a brute-force evaluation written here with plain loops.
* Exact decomposition: chi_full - chi_screened equals the sum, over exactly the terms the rule
  drops (decided here independently), of those terms evaluated with the literal four-term
  formula of Sec. 2 (terms 1 and 2 for each dropped neighbour K(R1), terms 3 and 4 over all
  K(R1), L(dL) for a dropped Z part).  A slice dropped by mistake, a wrong lattice-vector index in
  the bounds, or a dropped term of the wrong kind fails it.
* The rigorous elementwise bound of the dropped terms holds.
* The rule is monotone: a larger threshold keeps no more terms.
"""
import numpy as np
import pytest

from oracle import chi0 as ochi
from oracle import screening as scr
from oracle.chi0 import bvk_sub, cblock, fold
from tests._util import micro

SPECS = [dict(), dict(seed=2, natoms=3, nao=(2, 5, 3), naux=(3, 6, 2), mesh=(3, 1, 2)),
         dict(seed=11, natoms=3, nao=(3, 4, 2), naux=(4, 5, 3), mesh=(4, 2, 1), rcut=4.5, edge=3.5)]


def brute_norms(inp, t):
    """gb and gn by explicit loops over matrix elements and LRI blocks."""
    na, nR, mesh = inp.natoms, inp.nR, inp.cell.mesh
    gb = np.zeros((na, na, nR))
    for R in range(nR):
        for p in range(inp.nb):
            U = int(np.searchsorted(inp.ao_off, p, side="right") - 1)
            for q in range(inp.nb):
                V = int(np.searchsorted(inp.ao_off, q, side="right") - 1)
                gb[U, V, R] = max(gb[U, V, R], abs(inp.Gocc[t, R, p, q]), abs(inp.Gun[t, R, p, q]))
    fR = fold(inp.blocks.R, mesh)
    gn = np.zeros((na, na, nR))
    for b in range(len(inp.blocks.I)):
        V, L = inp.blocks.I[b], inp.blocks.K[b]
        for K in range(na):
            for dR in range(nR):
                gn[V, K, dR] = max(gn[V, K, dR], gb[L, K, int(bvk_sub(dR, fR[b], mesh))])
    return gb, gn


def four_terms(inp, t, U, V, R, bu, which):
    """Literal four-term formula restricted to one neighbour block bu = K(R1) of U (terms 1+2,
    which='M') or summed over every K(R1) of U (terms 3+4, which='Z'), for chi_UV(R, tau_t)."""
    mesh = inp.cell.mesh
    fR = fold(inp.blocks.R, mesh)
    Go, Gu = inp.Gocc[t], inp.Gun[t]
    iU = slice(inp.ao_off[U], inp.ao_off[U] + inp.nao[U])
    iV = slice(inp.ao_off[V], inp.ao_off[V] + inp.nao[V])
    out = np.zeros((inp.naux[U], inp.naux[V]))
    ublocks = [bu] if which == "M" else list(np.nonzero(inp.blocks.I == U)[0])
    for b1 in ublocks:
        K, R1 = inp.blocks.K[b1], fR[b1]
        iK = slice(inp.ao_off[K], inp.ao_off[K] + inp.nao[K])
        Cu = cblock(inp, b1)
        for bv in np.nonzero(inp.blocks.I == V)[0]:
            L = inp.blocks.K[bv]
            iL = slice(inp.ao_off[L], inp.ao_off[L] + inp.nao[L])
            Cv = cblock(inp, bv)
            R2 = int(ochi._add(R, fR[bv], mesh))
            r12 = int(bvk_sub(R1, R2, mesh))
            r1r = int(bvk_sub(R1, R, mesh))
            if which == "M":
                W = np.einsum("ij,lk->ijkl", Gu[R, iU, iV], Go[r12, iL, iK]) + \
                    np.einsum("ij,lk->ijkl", Go[R, iU, iV], Gu[r12, iL, iK])
            else:
                W = np.einsum("jk,il->ijkl", Go[r1r, iV, iK], Gu[R2, iU, iL]) + \
                    np.einsum("jk,il->ijkl", Gu[r1r, iV, iK], Go[R2, iU, iL])
            out += -inp.spin_factor * np.einsum("mik,njl,ijkl->mn", Cu, Cv, W, optimize=True)
    return out


@pytest.mark.parametrize("idx", range(len(SPECS)))
def test_theta_zero_and_above_one(idx):
    inp = micro(**SPECS[idx])
    full = ochi.chi0_alg1(inp)
    s0, st0 = scr.chi0_alg1_screened(inp, 0.0)
    assert np.array_equal(s0, full)
    assert st0["slices_kept"] == st0["slices_total"] and st0["z_kept"] == st0["z_total"]
    s2, st2 = scr.chi0_alg1_screened(inp, 1.0000001)
    assert not np.any(s2)
    assert st2["slices_kept"] == 0 and st2["z_kept"] == 0


@pytest.mark.parametrize("idx", range(len(SPECS)))
def test_norms_match_brute_force(idx):
    inp = micro(**SPECS[idx])
    alg = scr.ScreenedAlg1(inp, 0.1)
    for t in (0, inp.ntau - 1):
        gb, gn, g = alg.norms(t)
        bgb, bgn = brute_norms(inp, t)
        assert np.array_equal(gb, bgb)
        assert np.array_equal(gn, bgn)
        assert g == bgb.max()


@pytest.mark.parametrize("theta", [0.05, 0.2])
@pytest.mark.parametrize("idx", [0, 1])
def test_exact_decomposition_into_dropped_terms(idx, theta):
    inp = micro(**SPECS[idx])
    mesh = inp.cell.mesh
    fR = fold(inp.blocks.R, mesh)
    t = 0
    full = ochi.chi0_alg1(inp, taus=[t])[0]
    got, _ = scr.chi0_alg1_screened(inp, theta, taus=[t])
    got = got[0]
    gb, gn = brute_norms(inp, t)
    cut = theta * gb.max() ** 2
    dropped = np.zeros_like(full)
    ndrop = 0
    for U in range(inp.natoms):
        mu = slice(inp.aux_off[U], inp.aux_off[U] + inp.naux[U])
        for V in range(inp.natoms):
            nu = slice(inp.aux_off[V], inp.aux_off[V] + inp.naux[V])
            for R in range(inp.nR):
                for bu in np.nonzero(inp.blocks.I == U)[0]:
                    K = inp.blocks.K[bu]
                    if gb[U, V, R] * gn[V, K, int(bvk_sub(fR[bu], R, mesh))] < cut:
                        dropped[R, mu, nu] += four_terms(inp, t, U, V, R, bu, "M")
                        ndrop += 1
                if gn[U, V, R] * gn[V, U, int(bvk_sub(0, R, mesh))] < cut:
                    dropped[R, mu, nu] += four_terms(inp, t, U, V, R, None, "Z")
                    ndrop += 1
    assert ndrop > 0                                   # the case is not vacuous
    scale = np.abs(full).max()
    np.testing.assert_allclose(full - got, dropped, rtol=0, atol=1e-12 * scale)


@pytest.mark.parametrize("theta", [1e-2, 0.05, 0.2, 0.5])
@pytest.mark.parametrize("idx", range(len(SPECS)))
def test_dropped_terms_within_bound(idx, theta):
    inp = micro(**SPECS[idx])
    full = ochi.chi0_alg1(inp)
    got, _ = scr.chi0_alg1_screened(inp, theta)
    scale = np.abs(full).max()
    for t in range(inp.ntau):
        B = scr.screening_bound(inp, theta, t)
        assert np.all(np.abs(got[t] - full[t]) <= B + 1e-13 * scale)


@pytest.mark.parametrize("idx", range(len(SPECS)))
def test_monotone_in_theta(idx):
    inp = micro(**SPECS[idx])
    kept = []
    for theta in (0.0, 1e-2, 0.05, 0.2, 0.5, 2.0):
        _, st = scr.chi0_alg1_screened(inp, theta)
        kept.append((st["slices_kept"], st["z_kept"]))
    for a, b in zip(kept, kept[1:]):
        assert b[0] <= a[0] and b[1] <= a[1]
    assert kept[-1] == (0, 0) and kept[0][0] > 0


def test_planted_wrong_shift_fails_decomposition(monkeypatch):
    """A screening decision taken with R1 + R instead of R1 - R (a plausible index slip) drops
    other terms than the rule names; the exact decomposition catches it."""
    inp = micro(**SPECS[1])
    orig = scr.ScreenedAlg1.masks

    def wrong(self, t, U, V, R):
        return orig(self, t, U, V, (-R) % inp.nR)
    monkeypatch.setattr(scr.ScreenedAlg1, "masks", wrong)
    with pytest.raises(AssertionError):
        test_exact_decomposition_into_dropped_terms(1, 0.2)


@pytest.mark.parametrize("idx", range(len(SPECS)))
def test_pair_set_without_screening_is_algorithm1(idx):
    """theta = 0 over the pair set U <= V with the Hermitian fill reproduces every block of the
    full build (independently computed U > V blocks), up to rounding."""
    inp = micro(**SPECS[idx])
    full = ochi.chi0_alg1(inp)
    got, st = scr.chi0_alg1_screened_pairs(inp, 0.0)
    assert np.abs(got - full).max() <= 1e-13 * np.abs(full).max()
    npairs = inp.natoms * (inp.natoms + 1) // 2
    assert st["z_total"] == npairs * inp.nR * inp.ntau == st["z_kept"]


@pytest.mark.parametrize("theta", [0.05, 0.2])
@pytest.mark.parametrize("idx", range(len(SPECS)))
def test_pair_set_blocks_and_bound(idx, theta):
    """The U <= V blocks of the pair-set build are the screened blocks themselves, the U > V blocks
    their transposes at -R, and the whole tensor is within the rigorous bound of the dropped terms
    (for U > V the transposed bound of the partner)."""
    inp = micro(**SPECS[idx])
    mesh = inp.cell.mesh
    full = ochi.chi0_alg1(inp)
    got, _ = scr.chi0_alg1_screened_pairs(inp, theta)
    alg = scr.ScreenedAlg1(inp, theta)
    scale = np.abs(full).max()
    for t in range(inp.ntau):
        B = scr.screening_bound(inp, theta, t)
        for U in range(inp.natoms):
            mu = slice(inp.aux_off[U], inp.aux_off[U] + inp.naux[U])
            for V in range(inp.natoms):
                nu = slice(inp.aux_off[V], inp.aux_off[V] + inp.naux[V])
                for R in range(inp.nR):
                    if U <= V:
                        assert np.array_equal(got[t, R, mu, nu], alg.block(t, U, V, R))
                        bound = B[R, mu, nu]
                    else:
                        r = int(bvk_sub(0, R, mesh))
                        assert np.array_equal(got[t, R, mu, nu], got[t, r, nu, mu].T)
                        bound = B[r, nu, mu].T
                    assert np.all(np.abs(got[t, R, mu, nu] - full[t, R, mu, nu]) <= bound + 1e-13 * scale)
