"""Calibrate the scale of the synthetic Coulomb matrices with the oracle (calls only oracle/).

v(q) = s (L L^H + 1e-3 I) / lambda_max(L L^H + 1e-3 I); s is chosen so that the largest spectral
radius of chi(q, i omega_k) v(q) over q and k is 0.9, as the workload definition asks
(|| chi0 v || < 1).  The radius is linear in s, so one evaluation at s = 1 fixes s = 0.9 / rho(1).

rho(1) is exact: oracle.aw.spectral_radius_chi_v applies chi(q, i omega) in its Bloch
sum-over-states form (pinned against the dense supercell sum over states in
tests/test_oracle_chi0.py) at the smallest grid frequency, where chi(i omega) is largest, and
runs Lanczos on the Hermitian L^H chi(q) L for every q of the mesh.  For the serving workload
the one scale is set by the cell with the largest radius.

Usage: python tests/golden/calibrate_vscale.py [config ...] [--workers N]
(prints the V_SCALE entries; config 33 = the 75-atom sheet on the 2x2x1 mesh, config 4 = the 64
serving cells)
"""
import concurrent.futures as cf
import multiprocessing as mp
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle.aw import spectral_radius_chi_v                        # noqa: E402
from rpa_synth import config, make_inputs                          # noqa: E402
from rpa_synth import configs as registry                          # noqa: E402


def rho_unit_scale(cell):
    """rho(chi v) of one cell with s = 1 and the q index where it is largest."""
    from threadpoolctl import threadpool_limits
    cell.v_scale = 1.0
    t0 = time.time()
    single = bool(os.environ.get("CALIB_SINGLE_THREAD"))
    with threadpool_limits(1 if single else None):
        inp = make_inputs(cell, with_green=False)
        rho, iq = spectral_radius_chi_v(inp, workers=1 if single else int(os.environ.get("CALIB_WORKERS", "8")))
    return cell.name, inp.natoms, tuple(cell.mesh), rho, iq, time.time() - t0


def main(argv):
    workers = 4
    if "--workers" in argv:
        i = argv.index("--workers")
        workers = int(argv[i + 1])
        argv = argv[:i] + argv[i + 2:]
    which = [int(a) for a in argv] or [0, 1, 2, 3, 33, 4]
    for i in which:
        if i == 4:
            cells = registry.serving_cells()
            os.environ["CALIB_SINGLE_THREAD"] = "1"
            worst = (0.0, None)
            with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
                for name, nat, mesh, rho, iq, dt in ex.map(rho_unit_scale, cells):
                    print("  %s (%d atoms, mesh %s): rho(s=1) = %.6g at q %d (%.0f s)" % (name, nat, mesh, rho, iq, dt),
                          flush=True)
                    worst = max(worst, (rho, name))
            print("config 4: largest rho(s=1) = %.6g (%s) -> V_SCALE[4] = %.6g" % (worst[0], worst[1], 0.9 / worst[0]),
                  flush=True)
        else:
            name, nat, mesh, rho, iq, dt = rho_unit_scale(config(i))
            print("config %d (%s): rho(s=1) = %.6g at q %d (%.0f s) -> V_SCALE[%d] = %.6g"
                  % (i, name, rho, iq, dt, i, 0.9 / rho), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
