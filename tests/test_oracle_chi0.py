"""Pins of the oracle's chi(R, tau): independent routes must agree, and the result must be
Hermitian and negative semidefinite after R -> q.  Mutation tests plant plausible mistakes
in copies of the oracle (on the CPU) and check that a pin catches each one."""
import numpy as np
import pytest

from oracle import aw, chi0
from oracle.transforms import cos_transform, fourier_R_to_q
from tests._util import micro, cfg, rel

MICRO_SPECS = [
    dict(),                                                             # 2 atoms, 3x2x1 mesh
    dict(seed=2, natoms=3, nao=(2, 5, 3), naux=(3, 6, 2), mesh=(3, 1, 2)),
    dict(seed=5, natoms=1, nao=(4,), naux=(5,), mesh=(4, 1, 1), rcut=5.0),   # images fold twice
]


@pytest.mark.parametrize("spec", MICRO_SPECS)
def test_alg1_equals_plain_definition_and_bruteforce(spec):
    inp = micro(**spec)
    sc = chi0.chi0_supercell(inp)
    a1 = chi0.chi0_alg1(inp)
    assert rel(a1, sc) < 1e-13
    bf = np.array([chi0.chi0_bruteforce(inp, t) for t in range(inp.ntau)])
    assert rel(bf, sc) < 1e-13


@pytest.mark.parametrize("spec", MICRO_SPECS)
def test_sum_over_states_equals_space_time(spec):
    inp = micro(**spec)
    a1 = chi0.chi0_alg1(inp)
    awt = aw.chi0_aw_tau(inp, inp.tau)
    assert np.max(np.abs(awt.imag)) < 1e-12 * np.max(np.abs(awt))
    assert rel(awt.real, a1) < 1e-12


def _q_matrices(inp, chi_R):
    return fourier_R_to_q(chi_R, inp.Rvec, inp.kfrac)


@pytest.mark.parametrize("spec", MICRO_SPECS)
def test_hermitian_and_negative_semidefinite(spec):
    inp = micro(**spec)
    a1 = chi0.chi0_alg1(inp)          # every ordered (U, V) block computed on its own
    mesh = np.array(inp.cell.mesh)
    for r, n in enumerate(inp.Rvec):
        m = np.mod(-n, mesh)
        rm = (m[0] * mesh[1] + m[1]) * mesh[2] + m[2]
        assert np.max(np.abs(a1[:, rm] - np.swapaxes(a1[:, r], 1, 2))) < 1e-13 * np.max(np.abs(a1))
    chi_q = _q_matrices(inp, a1)
    scale = np.max(np.abs(chi_q))        # rounding is relative to the largest (small-tau) entries
    for t in range(inp.ntau):
        for q in range(len(inp.kfrac)):
            A = chi_q[t, q]
            assert np.max(np.abs(A - A.conj().T)) < 1e-13 * scale
            lam = np.linalg.eigvalsh(0.5 * (A + A.conj().T))
            assert lam.max() <= 1e-13 * scale
    chi_w = _q_matrices(inp, cos_transform(a1, inp.gamma_cos))
    # the fitted transform is not exactly positive, so NSD of chi(i omega) is checked on the exact
    # sum-over-states form
    aww = aw.chi0_aw_omega(inp, inp.omega)
    for k in range(len(inp.omega)):
        for q in range(len(inp.kfrac)):
            A = _q_matrices(inp, aww[k:k + 1])[0, q]
            assert np.linalg.eigvalsh(0.5 * (A + A.conj().T)).max() <= 1e-12 * np.abs(A).max()
    assert np.all(np.isfinite(chi_w))


@pytest.mark.parametrize("spec", MICRO_SPECS[:2])
def test_cosine_transform_within_its_error_bound(spec):
    """|| chi_ST(q, i w_k) - chi_AW(q, i w_k) ||_2 <= eta_k || chi(q, tau=0) ||_2 with
    eta_k = max_x |sum_j Gamma_kj e^{-x tau_j} - 2x/(x^2+w_k^2)| over the transition energies."""
    inp = micro(**spec)
    amp = aw.pair_amplitudes(inp)
    D = amp[1]
    emin, emax = D.min(), D.max()
    x = np.exp(np.linspace(np.log(emin), np.log(emax), 20000))
    E = np.exp(-np.outer(x, inp.tau))
    eta = np.max(np.abs(inp.gamma_cos @ E.T - 2 * x[None] / (x[None] ** 2 + inp.omega[:, None] ** 2)), axis=1)
    st = _q_matrices(inp, cos_transform(chi0.chi0_alg1(inp), inp.gamma_cos))
    ex = _q_matrices(inp, aw.chi0_aw_omega(inp, inp.omega, amp).real)
    c0 = _q_matrices(inp, aw.chi0_aw_tau(inp, [0.0], amp).real)[0]
    for k in range(len(inp.omega)):
        for q in range(len(inp.kfrac)):
            lhs = np.linalg.norm(st[k, q] - ex[k, q], 2)
            assert lhs <= eta[k] * np.linalg.norm(c0[q], 2) * (1 + 1e-9) + 1e-14


def test_tiny_cell_all_routes():
    """The tiny workload (2 atoms, 13 NAO / 40 ABF, 2x2x2 mesh): Alg. 1 against the plain
    definition on two tau points and against the sum-over-states form on all eight."""
    inp = cfg(0)
    a1 = chi0.chi0_alg1(inp)
    sc = chi0.chi0_supercell(inp, taus=[0, inp.ntau - 1])
    assert rel(a1[[0, inp.ntau - 1]], sc) < 1e-12
    awt = aw.chi0_aw_tau(inp, inp.tau)
    assert rel(awt.real, a1) < 1e-12


# ----------------------------------------------------------------------------
# mutation tests: a planted mistake in a copy of the oracle must fail a pin
# ----------------------------------------------------------------------------

class _DropTerm(chi0.Alg1):
    """Alg. 1 with the last Z term dropped."""
    @staticmethod
    def combine(M1, M2, Z1, Z2):
        return M1 + M2 + Z1


class _SwapChannels(chi0.Alg1):
    """Alg. 1 with occ and un exchanged in the M terms."""
    def N_all(self, t, V):
        out = super().N_all(t, V)
        return out[::-1]


def test_mutations_are_caught():
    inp = micro(**MICRO_SPECS[1])
    sc = chi0.chi0_supercell(inp)
    assert rel(_DropTerm(inp).full(), sc) > 1e-3
    assert rel(_SwapChannels(inp).full(), sc) > 1e-3
    # wrong sign of the BvK difference in the supercell Green's function
    orig = chi0.bvk_sub
    try:
        chi0.bvk_sub = lambda a, b, mesh: orig(b, a, mesh)
        bad = chi0.chi0_supercell(inp)
    finally:
        chi0.bvk_sub = orig
    assert rel(bad, chi0.chi0_alg1(inp)) > 1e-3
    # a transposed coefficient block (mu on the wrong atom of the pair) in the plain definition
    orig_t = chi0.supercell_lri_tensor

    def one_sum_only(inp_):
        T = np.zeros_like(orig_t(inp_))
        nR, nb, na = inp_.nR, inp_.nb, inp_.nauxtot
        for b in range(len(inp_.blocks.I)):
            U, K = inp_.blocks.I[b], inp_.blocks.K[b]
            C = chi0.cblock(inp_, b)
            r1 = chi0.fold(inp_.blocks.R[b], inp_.cell.mesh)
            for Ra in range(nR):
                Rk = int(chi0._add(Ra, r1, inp_.cell.mesh))
                rows = Ra * nb + inp_.ao_off[U] + np.arange(C.shape[1])
                cols = Rk * nb + inp_.ao_off[K] + np.arange(C.shape[2])
                al = Ra * na + inp_.aux_off[U] + np.arange(C.shape[0])
                T[np.ix_(al, rows, cols)] += C
        return T
    try:
        chi0.supercell_lri_tensor = one_sum_only
        bad = chi0.chi0_supercell(inp)
    finally:
        chi0.supercell_lri_tensor = orig_t
    assert rel(bad, sc) > 1e-3


@pytest.mark.parametrize("spec", MICRO_SPECS)
def test_bloch_form_equals_supercell_sum_over_states(spec):
    """The Bloch-resolved product chi(q, i omega) x (used for the spectral radius of chi v, which
    sets the Coulomb scale of the workloads) against the dense supercell sum over states taken
    to q, at every q of the mesh."""
    inp = micro(**spec)
    w = float(np.min(inp.omega))
    dense = fourier_R_to_q(aw.chi0_aw_omega(inp, [w]), inp.Rvec, inp.kfrac)[0]
    rng = np.random.default_rng(3)
    A = aw.bloch_c_all(inp)
    for iq in range(len(inp.kfrac)):
        x = rng.standard_normal(inp.nauxtot) + 1j * rng.standard_normal(inp.nauxtot)
        assert rel(aw.BlochChi(inp, iq, w, A)(x), dense[iq] @ x) < 1e-12


def test_bloch_form_catches_a_wrong_phase():
    inp = micro(**MICRO_SPECS[0])             # 3x2x1 mesh: the phases matter
    w = float(np.min(inp.omega))
    dense = fourier_R_to_q(aw.chi0_aw_omega(inp, [w]), inp.Rvec, inp.kfrac)[0]
    A = aw.bloch_c_all(inp)
    A = [a.conj() for a in A]                                  # e^{-2 pi i k.R1}: the wrong phase
    x = np.random.default_rng(4).standard_normal(inp.nauxtot).astype(np.complex128)
    assert max(rel(aw.BlochChi(inp, iq, w, A)(x), dense[iq] @ x) for iq in range(len(inp.kfrac))) > 1e-3


def test_spectral_radius_matches_dense_eigenvalues():
    """Lanczos on L^H chi L against the eigenvalues of the dense chi(q, i omega_1) v(q) of the
    tiny workload, whose Coulomb scale puts the maximum at 0.9."""
    inp = cfg(0)
    w = float(np.min(inp.omega))
    dense = fourier_R_to_q(aw.chi0_aw_omega(inp, [w]), inp.Rvec, inp.kfrac)[0]
    rho_dense = max(np.max(np.abs(np.linalg.eigvals(dense[q] @ inp.vq[q]))) for q in range(len(inp.kfrac)))
    rho, _ = aw.spectral_radius_chi_v(inp)
    assert abs(rho - rho_dense) <= 1e-9 * rho_dense
    assert abs(rho - 0.9) < 1e-3
