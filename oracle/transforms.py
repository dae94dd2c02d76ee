"""tau -> i omega cosine transform and R -> q Fourier transform, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np


def cos_transform(chi_tau, gamma_cos):
    """chi(R, i omega_k) = sum_j Gamma_kj chi(R, tau_j), Gamma_kj = gamma_kj cos(omega_k tau_j)
    (Sec. 2, the cosine-transform equation; the paper's -i and chi0 = i chi cancel)."""
    nt = chi_tau.shape[0]
    return (gamma_cos @ chi_tau.reshape(nt, -1)).reshape((gamma_cos.shape[0],) + chi_tau.shape[1:])


def fourier_R_to_q(chi_R, Rvec, qfrac):
    """chi(q) = sum_R exp(i q.R) chi(R) (Sec. 2, the R -> q transform), over the leading R axis
    of chi_R[..., R, mu, nu]; q.R = 2 pi q_frac . n_R."""
    ph = np.exp(2j * np.pi * (np.asarray(qfrac) @ np.asarray(Rvec).T))   # (nq, nR)
    return np.einsum("qr,...rmn->...qmn", ph, chi_R)
