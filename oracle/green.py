"""Real-space imaginary-time Green's functions from Bloch eigenpairs, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 2, Eq. (green_mat), with the factors of i taken out (for tau > 0 the paper's
G(R, i tau) equals i G^un(R, tau) and G(R, -i tau) equals -i G^occ(R, tau)):

    G^occ_{ij}(R, tau) = (1/N_k) sum_k e^{-i k.R} sum_{n occupied}   c_{in}(k) c*_{jn}(k) e^{-(mu - eps_nk) tau}
    G^un_{ij}(R, tau)  = (1/N_k) sum_k e^{-i k.R} sum_{n unoccupied} c_{in}(k) c*_{jn}(k) e^{-(eps_nk - mu) tau}

with k.R = 2 pi k_frac . n_R for the integer BvK triples n_R and the Bloch sum convention
H(k) = sum_R e^{i k.R} h(R).  The band sum of one k is a matrix product; k and tau are plain
loops.  Both results are real when H(k)* = H(-k) (time reversal); the imaginary parts are
returned so that callers can check that.

Pins (tests/test_oracle_green.py): completeness G^occ(R, 0) + G^un(R, 0) = delta_{R0} I; the
trace of G^occ(0, tau) from the band energies alone; G(-R) = G(R)^T; the semigroup
G^un(tau1) * G^un(tau2) = G^un(tau1 + tau2) (convolution over the BvK mesh); and, for a
Hamiltonian built from known hoppings h(R), G^un(R, d) + G^occ(R, -d) = delta_{R0} I - d (h(R) -
mu delta_{R0} I) + O(d^2), which fixes the sign of the phase and the conjugated factor.
"""
from __future__ import annotations

import numpy as np


def green_tau(eps, wfc, nocc, mu, tau, kfrac, Rvec):
    """eps (nk, nb) band energies, wfc (nk, nb, nb) with c_{in}(k) = wfc[k, i, n], nocc occupied
    bands at every k, chemical potential mu, imaginary times tau (ntau,), fractional k (nk, 3),
    BvK integer triples Rvec (nR, 3).  Returns (G_occ, G_un, max_imag): real arrays
    (ntau, nR, nb, nb) and the largest |imaginary part| of either."""
    eps = np.asarray(eps, dtype=np.float64)
    wfc = np.asarray(wfc, dtype=np.complex128)
    nk, nb = eps.shape
    tau = np.atleast_1d(np.asarray(tau, dtype=np.float64))
    Rvec = np.asarray(Rvec)
    phase = np.exp(-2j * np.pi * (Rvec @ np.asarray(kfrac).T))          # (nR, nk): e^{-i k.R}
    occ = np.arange(nb) < nocc
    Gocc = np.zeros((len(tau), len(Rvec), nb, nb), dtype=np.complex128)
    Gun = np.zeros_like(Gocc)
    for t, tt in enumerate(tau):
        for k in range(nk):
            c = wfc[k]
            # weights of the occupied and unoccupied bands at this (k, tau); each exponential is
            # evaluated on its own channel's bands only (the other channel's would overflow)
            w_occ = np.zeros(nb)
            w_un = np.zeros(nb)
            w_occ[occ] = np.exp(-(mu - eps[k][occ]) * tt)
            w_un[~occ] = np.exp(-(eps[k][~occ] - mu) * tt)
            P_occ = (c * w_occ[None, :]) @ c.conj().T                     # sum_n c_in w_n c*_jn
            P_un = (c * w_un[None, :]) @ c.conj().T
            for r in range(len(Rvec)):
                Gocc[t, r] += phase[r, k] * P_occ
                Gun[t, r] += phase[r, k] * P_un
    Gocc /= nk
    Gun /= nk
    max_imag = max(float(np.abs(Gocc.imag).max()), float(np.abs(Gun.imag).max()))
    return Gocc.real.copy(), Gun.real.copy(), max_imag
