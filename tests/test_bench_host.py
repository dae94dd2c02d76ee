"""Host logic of the benchmark (no GPU): the energy-stage flop model for each kind of q point and
the launch-variant matching of the committed counter summaries."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_energy_flop_model_by_kind_of_q_point():
    """Complex q: 20/3 n^3 per (q, omega) + 4/3 n^3 per q (T = chi L with triangular L 4 n^3,
    B = L^H T on the lower triangle 4/3 n^3, Cholesky of I - B 4/3 n^3, Cholesky of v 4/3 n^3);
    real chi with complex v: T at two real products per complex one (2 n^3); both real: every
    step real (n^3 + n^3/3 + n^3/3, and n^3/3 for v)."""
    n, nw = 10, 3
    n3 = float(n) ** 3
    q = [[0.0, 0.0, 0.0], [0.25, 0.0, 0.0], [0.5, 0.5, 0.0]]    # time-reversal invariant: 0 and 2
    kt = {"ec_stage": (2.0, 1)}
    r = bench.ec_stage_rate(n, q, [True, False, False], nw, kt, 1)
    complex_q = nw * 20.0 / 3.0 * n3 + 4.0 / 3.0 * n3
    real_q = nw * 5.0 / 3.0 * n3 + 1.0 / 3.0 * n3
    real_chi_q = nw * 14.0 / 3.0 * n3 + 4.0 / 3.0 * n3
    assert np.isclose(r["model_tflop"] * 1e12, 3 * complex_q)
    assert np.isclose(r["executed_tflop"] * 1e12, real_q + complex_q + real_chi_q)
    assert (r["real_chi_q"], r["real_q"], r["nq"]) == (2, 1, 3)
    assert np.isclose(r["executed_tflops"], r["executed_tflop"] / 2e-3)


def test_launch_variant_matching():
    # the N stage depends on its order, K step and tile rows; the fused kernel on its item order
    # and launch shape
    assert bench.same_variant("nstage", "1,0,0,1,128", "1,0,1,3,128")
    assert not bench.same_variant("nstage", "1,0,0,1,128", "0,0,0,1,128")
    assert not bench.same_variant("nstage", "1,0,0,1,128", "1,0,0,1,256")
    assert bench.same_variant("fused", "1,0,0,1,128", "0,0,0,1,256")
    assert not bench.same_variant("fused", "1,0,0,1,128", "1,0,0,3,128")
    assert bench.same_variant("nstage", "0,16,0", "0,16,0,0,128")

