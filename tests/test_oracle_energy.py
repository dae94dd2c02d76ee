"""Pins of the oracle's transforms and correlation energy."""
import numpy as np
import pytest

from oracle import aw, chi0
from oracle.energy import correlation_energy, ec_terms_eig, ec_terms_lu
from oracle.pipeline import ec_from_chi_tau
from oracle.transforms import cos_transform, fourier_R_to_q
from rpa_synth import make_inputs
from rpa_synth.configs import micro_cell
from tests._util import micro, rel


def _gauss_legendre_semi_infinite(n, w0):
    """Nodes/weights on (0, inf) from Gauss-Legendre on t in (-1, 1), omega = w0 (1+t)/(1-t)."""
    t, w = np.polynomial.legendre.leggauss(n)
    om = w0 * (1 + t) / (1 - t)
    return om, w * 2 * w0 / (1 - t) ** 2


def test_two_level_closed_form():
    """One atom, two NAOs, one ABF, Gamma only, no periodic images inside the cutoff.
    chi(i w) = -A 2D/(D^2+w^2) with A = s Lambda^2, so with b = 2 A v D
    E_c = (1/2pi) int_0^inf [ln(1 + b/(D^2+w^2)) - b/(D^2+w^2)] dw = (sqrt(D^2+b) - D)/2 - b/(4D)
    (from int_0^inf ln((w^2+a^2)/(w^2+c^2)) dw = pi (a - c))."""
    inp = make_inputs(micro_cell(11, natoms=1, nao=(2,), naux=(1,), mesh=(1, 1, 1), rcut=2.0, edge=3.0, ntau=4))
    assert len(inp.blocks.I) == 1
    Lam, D = aw.pair_amplitudes(inp)
    D = float(D[0, 0])
    assert abs(D - 0.1) < 1e-12                      # the scissored gap
    A = inp.spin_factor * abs(Lam[0, 0, 0]) ** 2
    v = float(inp.vq[0, 0, 0].real)
    om, w = _gauss_legendre_semi_infinite(400, D)
    chi_w = aw.chi0_aw_omega(inp, om, (Lam, aw.pair_amplitudes(inp)[1]))   # [nw, R, 1, 1]
    chi_q = fourier_R_to_q(chi_w.real, inp.Rvec, inp.kfrac)
    ec, _ = correlation_energy(ec_terms_lu(chi_q, inp.vq), w)
    b = 2 * A * v * D
    exact = 0.5 * (np.sqrt(D * D + b) - D) - b / (4 * D)
    assert exact < 0
    assert abs(ec - exact) < 1e-10 * max(1.0, abs(exact))
    # the same system through the space-time chi(tau) and the fitted cosine transform is within
    # the transform's own error (a few percent at 4 points)
    sc = chi0.chi0_alg1(inp)
    ec_st, _, _ = ec_from_chi_tau(inp, sc)
    assert abs(ec_st - exact) < 0.1 * abs(exact)


def _random_nsd_chi_and_v(rng, n, nq, nw, rho):
    chi = np.empty((nw, nq, n, n), dtype=np.complex128)
    vq = np.empty((nq, n, n), dtype=np.complex128)
    for q in range(nq):
        L = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        vq[q] = L @ L.conj().T / n + 0.1 * np.eye(n)
        for k in range(nw):
            M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
            chi[k, q] = -(M @ M.conj().T)
    # scale so that the largest spectral radius of chi v equals rho
    r = max(np.max(np.abs(np.linalg.eigvals(chi[k, q] @ vq[q]))) for k in range(nw) for q in range(nq))
    return chi * (rho / r), vq


def test_small_coupling_series_and_sign():
    """ln det(1 - X) + Tr X = -sum_{n>=2} Tr(X^n)/n for spectral radius < 1, each term <= 0."""
    rng = np.random.default_rng(7)
    chi, vq = _random_nsd_chi_and_v(rng, 12, 2, 3, 0.5)
    f = ec_terms_lu(chi, vq)
    for k in range(3):
        for q in range(2):
            X = chi[k, q] @ vq[q]
            s, P = 0.0, np.eye(12, dtype=complex)
            for n in range(1, 120):
                P = P @ X
                if n >= 2:
                    s -= np.trace(P).real / n
            assert abs(f[k, q] - s) < 1e-12 * max(1.0, abs(s))
    assert np.all(f <= 0)
    # E_c(lambda v)/lambda^2 -> -(1/(4 pi Nq)) sum_qk w_k Tr[(chi v)^2]
    w = np.array([0.3, 0.5, 0.7])
    lead = -sum(w[k] * np.trace(chi[k, q] @ vq[q] @ chi[k, q] @ vq[q]).real
                for k in range(3) for q in range(2)) / (4 * np.pi * 2)
    prev = None
    for lam in (1e-2, 1e-3, 1e-4):
        e, _ = correlation_energy(ec_terms_lu(chi, vq * lam), w)
        dev = abs(e / lam ** 2 - lead)
        assert dev < 5 * lam * abs(lead)
        if prev is not None:
            assert dev < prev                       # converges linearly in lambda
        prev = dev


def test_lu_and_eigenvalue_routes_agree():
    rng = np.random.default_rng(3)
    chi, vq = _random_nsd_chi_and_v(rng, 20, 2, 2, 0.9)
    assert np.max(np.abs(ec_terms_lu(chi, vq) - ec_terms_eig(chi, vq))) < 1e-12


def test_fourier_identities():
    inp = micro(mesh=(3, 2, 1))
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, inp.nR, 4, 4))
    xq = fourier_R_to_q(x, inp.Rvec, inp.kfrac)
    gamma = int(np.nonzero(np.all(inp.kfrac == 0, axis=1))[0][0])
    assert np.max(np.abs(xq[:, gamma] - x.sum(axis=1))) < 1e-14 * np.abs(x).sum()
    # inverse DFT round trip: x(R) = (1/Nq) sum_q e^{-iqR} x(q)
    ph = np.exp(-2j * np.pi * (inp.Rvec @ inp.kfrac.T)) / len(inp.kfrac)
    back = np.einsum("rq,tqmn->trmn", ph, xq)
    assert np.max(np.abs(back - x)) < 1e-14 * np.abs(x).max() * inp.nR


def test_cos_transform_is_linear_in_tau_axis():
    rng = np.random.default_rng(1)
    G = rng.standard_normal((3, 5))
    x = rng.standard_normal((5, 2, 3, 3))
    y = cos_transform(x, G)
    assert np.allclose(y[1, 1], sum(G[1, j] * x[j, 1] for j in range(5)), atol=1e-14)


def test_pipeline_energy_negative_on_micro():
    inp = micro(seed=2, natoms=3, nao=(2, 5, 3), naux=(3, 6, 2), mesh=(3, 1, 2))
    ec, per_q, chi_q = ec_from_chi_tau(inp, chi0.chi0_alg1(inp))
    assert ec < 0 and np.all(per_q <= 1e-15)
