"""RPA correlation energy from chi(q, i omega) and v(q), FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

E_c = 1/(2 pi) 1/Nq sum_q sum_k w_k { ln det[1 - Pi(q, i omega_k)] + Tr Pi(q, i omega_k) },
Pi = chi v  (Sec. 2, the E_c^RPA equations, with Tr ln = ln det).  The
determinant is taken from an LU factorisation, as the paper does.
"""
from __future__ import annotations

import numpy as np


def ec_terms_lu(chi_q_omega, vq):
    """f[k, q] = ln det(1 - chi v) + Tr(chi v) from LU (numpy slogdet), real part.

    chi_q_omega: [nomega, nq, n, n] complex, vq: [nq, n, n] complex."""
    nw, nq, n, _ = chi_q_omega.shape
    f = np.empty((nw, nq))
    for k in range(nw):
        for q in range(nq):
            P = chi_q_omega[k, q] @ vq[q]
            sign, logabs = np.linalg.slogdet(np.eye(n) - P)
            tr = np.trace(P)
            if abs(sign.imag) > 1e-8 or sign.real <= 0:
                raise ValueError("det(1 - chi v) not positive at (k=%d, q=%d): %r" % (k, q, sign))
            if abs(tr.imag) > 1e-8 * max(1.0, abs(tr.real)):
                raise ValueError("Tr(chi v) not real")
            f[k, q] = logabs + tr.real
    return f


def ec_terms_eig(chi_q_omega, vq):
    """Same terms from the eigenvalues of I - L^H chi L, v = L L^H (Cholesky): an
    independent route to the determinant (Sylvester: det(1 - chi L L^H) = det(1 - L^H chi L))."""
    nw, nq, n, _ = chi_q_omega.shape
    f = np.empty((nw, nq))
    for q in range(nq):
        L = np.linalg.cholesky(vq[q])
        for k in range(nw):
            B = L.conj().T @ chi_q_omega[k, q] @ L
            B = 0.5 * (B + B.conj().T)
            lam = np.linalg.eigvalsh(B)
            f[k, q] = np.sum(np.log1p(-lam) + lam)
    return f


def correlation_energy(f_terms, womega, nq=None):
    """E_c = 1/(2 pi) (1/Nq) sum_q sum_k w_k f[k, q]  per unit cell (Hartree)."""
    nq = f_terms.shape[1] if nq is None else nq
    per_q = (np.asarray(womega)[:, None] * f_terms).sum(axis=0) / (2.0 * np.pi * nq)
    return float(per_q.sum()), per_q
