"""chi(R, tau) -> chi(R, i omega) -> chi(q, i omega) -> E_c for an input bundle, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np

from .chi0 import Alg1
from .energy import correlation_energy, ec_terms_lu
from .transforms import cos_transform, fourier_R_to_q


def ec_from_chi_tau(inp, chi_tau):
    """E_c (Ha per cell), per-q contributions and chi(q, i omega) from chi[t, R, mu, nu]."""
    chi_w = cos_transform(chi_tau, inp.gamma_cos)
    chi_q = fourier_R_to_q(chi_w, inp.Rvec, inp.kfrac)
    f = ec_terms_lu(chi_q, inp.vq)
    ec, per_q = correlation_energy(f, inp.womega)
    return ec, per_q, chi_q


def run(inp):
    """Whole path: Algorithm 1 for every block, transforms, LU log-det and quadrature."""
    chi_tau = Alg1(inp).full()
    ec, per_q, _ = ec_from_chi_tau(inp, chi_tau)
    return dict(chi_tau=chi_tau, ec=ec, ec_per_atom=ec / inp.natoms, ec_q=per_q)
