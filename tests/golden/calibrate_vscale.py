"""Calibrate the scale of the synthetic Coulomb matrices with the oracle (calls only oracle/).

v(q) = s (L L^H + 1e-3 I) / lambda_max(L L^H + 1e-3 I); s is chosen so that the largest spectral
radius of chi(q, i omega_k) v(q) over q and k is about 0.9, as the workload definition asks
(|| chi0 v || < 1).

* tiny cell: the full oracle chi(q, i omega) gives rho exactly; s = 0.9 / rho(s = 1).
* larger cells: the full oracle chi costs hours, so rho is estimated from the diagonal
  block chi_00(R=0, i omega_1) = sum_j Gamma_1j chi_00(R=0, tau_j) of atom 0, relative to the
  same block of the tiny cell:  rho_est = rho_tiny * ||chi_00||_2 / ||chi_00^tiny||_2.
  The spectral radius that results is measured and reported by the benchmark.

Usage: python tests/golden/calibrate_vscale.py [config ...]   (prints the V_SCALE entries)
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import chi0 as ochi                                   # noqa: E402
from oracle.transforms import cos_transform, fourier_R_to_q       # noqa: E402
from rpa_synth import config, make_inputs                          # noqa: E402
from rpa_synth import configs as registry                         # noqa: E402


def unit_scale_cell(i):
    c = config(i)
    c.v_scale = 1.0
    return c


def rho_full(inp):
    chi_w = fourier_R_to_q(cos_transform(ochi.chi0_alg1(inp), inp.gamma_cos), inp.Rvec, inp.kfrac)
    return max(np.max(np.abs(np.linalg.eigvals(chi_w[k, q] @ inp.vq[q])))
               for k in range(chi_w.shape[0]) for q in range(chi_w.shape[1]))


def diag_block_norm(inp):
    alg = ochi.Alg1(inp)
    blk = sum(inp.gamma_cos[0, t] * alg.block(t, 0, 0, 0) for t in range(inp.ntau))
    return np.linalg.norm(blk, 2)


def main(argv):
    which = [int(a) for a in argv] or [0, 1, 2]
    tiny = make_inputs(unit_scale_cell(0))
    rho0 = rho_full(tiny)
    n0 = diag_block_norm(tiny)
    print("tiny: rho(s=1) = %.6g, ||chi_00(0, w1)|| = %.6g -> V_SCALE[0] = %.6g" % (rho0, n0, 0.9 / rho0))
    for i in which:
        if i == 0:
            continue
        inp = make_inputs(unit_scale_cell(i), with_coulomb=False)
        n = diag_block_norm(inp)
        rho = rho0 * n / n0
        print("config %d: ||chi_00(0, w1)|| = %.6g, rho_est(s=1) = %.6g -> V_SCALE[%d] = %.6g"
              % (i, n, rho, i, 0.9 / rho))
    return 0


if __name__ == "__main__":
    registry.V_SCALE.update({k: 1.0 for k in registry.V_SCALE})
    sys.exit(main(sys.argv[1:]))
