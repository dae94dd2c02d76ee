"""Sum-over-states (Adler-Wiser) response function, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Derived from the definition chi(r, r', tau) = -s G^un(r, r', tau) G^occ(r', r, tau)
(Sec. 2, the space-time chi0 and Eq. (green_func)/(green_mat)) by expanding both
Green's functions over Bloch states and each product of two NAOs with
Eq. (eq:LRI):

  chi_{alpha beta}(tau)     = -s sum_{n occ, m un} exp(-(e_m - e_n) tau) L^alpha_nm conj(L^beta_nm)
  chi_{alpha beta}(i omega) = -s sum_{n occ, m un} 2 D/(D^2 + omega^2)  L^alpha_nm conj(L^beta_nm)

with D = e_m - e_n, the pair amplitudes L^alpha_nm = u_n^H T^alpha u_m, u_n the
supercell Bloch vectors u[(R, i)] = c_in(k) exp(2 pi i k.R)/sqrt(Nk), and T the
supercell LRI tensor.  The iomega form is the exact Fourier transform of the tau
form, 2 int_0^inf cos(omega tau) exp(-D tau) dtau = 2D/(D^2+omega^2), so it also
pins the tau -> iomega cosine transform.  Cost grows as N^4: small inputs only.
"""
from __future__ import annotations

import numpy as np

from .chi0 import supercell_lri_tensor


def bloch_vectors(inp):
    """Supercell columns u_n for all k, split into occupied and unoccupied sets."""
    nk, nb = inp.eps.shape
    ph = np.exp(2j * np.pi * (inp.Rvec @ inp.kfrac.T)) / np.sqrt(nk)   # (nR, nk)
    occ, un, eo, eu = [], [], [], []
    for k in range(nk):
        u = (ph[:, k][:, None, None] * inp.wfc[k][None]).reshape(inp.nR * nb, nb)
        occ.append(u[:, :inp.nocc])
        un.append(u[:, inp.nocc:])
        eo.append(inp.eps[k, :inp.nocc])
        eu.append(inp.eps[k, inp.nocc:])
    return np.hstack(occ), np.hstack(un), np.concatenate(eo), np.concatenate(eu)


def pair_amplitudes(inp):
    T = supercell_lri_tensor(inp)
    Uo, Uu, eo, eu = bloch_vectors(inp)
    Lam = np.einsum("pn,apq,qm->anm", Uo.conj(), T, Uu, optimize=True)
    D = eu[None, :] - eo[:, None]
    return Lam, D


def _assemble(inp, Lam, weight):
    """-s sum_nm weight_nm L^a_nm conj(L^b_nm), rows alpha in cell 0."""
    na, nR = inp.nauxtot, inp.nR
    A = Lam.reshape(Lam.shape[0], -1)
    chi = -inp.spin_factor * ((A[:na] * weight.reshape(-1)[None, :]) @ A.conj().T)
    return chi.reshape(na, nR, na).transpose(1, 0, 2)


def chi0_aw_tau(inp, taus, amplitudes=None):
    """[len(taus), nR, naux, naux] complex; imaginary part vanishes to rounding."""
    Lam, D = amplitudes or pair_amplitudes(inp)
    return np.array([_assemble(inp, Lam, np.exp(-D * t)) for t in taus])


def chi0_aw_omega(inp, omegas, amplitudes=None):
    Lam, D = amplitudes or pair_amplitudes(inp)
    return np.array([_assemble(inp, Lam, 2.0 * D / (D ** 2 + w ** 2)) for w in omegas])
