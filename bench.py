#!/usr/bin/env python3
"""Benchmark of the chi0(R, tau) -> E_c path on one MI355X.

A step is one pass of the whole path on device-resident inputs:
  build_chi0_tau -> chi0_tau_to_omega -> chi0_R_to_q -> rpa_correlation_energy.
Default workload: the largest single-GPU cell, a 72-atom hexagonal sheet (a = 2.46 A, 26 NAO / 100 ABF
per atom) with a bent triatomic 3 A above it (26/120 and 2 x 13/60), 15 A of vacuum, Gamma point,
24 tau/omega points, 12 A cutoff, on the split-BF16 (3-term) path; seeded synthetic inputs.  The
2x2x1 k-mesh of the same cell (`--workload sheet2x2x1`) quadruples every stage (9.9 s per step),
does not fit 20 + 5 steps into a ten-minute run, and leaves no room in the 288 GB for the FP64
comparison, so it is a separate command (`--no-fp64-check`).

Prints one JSON line.  `value` is the algorithmic flop count of the chi0 build (Algorithm 1
with its N intermediate evaluated once per (V, K, R1-R)) divided by the wall time of the whole
step, in TFLOP/s.  The same inputs run through the FP64 path (one untimed and one timed step,
outside the timed region) for the chi0 and E_c errors of the mixed path and for its build rate
and E_c time; the `gate` field says whether the mixed result meets the accuracy bars
(|dE_c| <= 1e-6 Ha/atom, relative chi0 Frobenius error <= 1e-5 against FP64).  The cpu_baseline leg times the FP64 oracle on
a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}
# split BF16 (3 products per FP32-equivalent product) on the 2.5 PFLOP/s dense bf16 MFMAs
PEAK_BF16X3_FP32EQ = 2500.0 / 3.0
# sources of the chi0 kernels; the HBM traffic recorded under profiles/ is used only while
# their hash matches the one the counters were taken with
KERNEL_SOURCES = ("paper_2407_19930_amd/csrc/chi0_kernels.hip", "paper_2407_19930_amd/csrc/chi0_bf16.hip",
                  "paper_2407_19930_amd/csrc/chi0_kernels.h", "paper_2407_19930_amd/csrc/item_table.h",
                  "paper_2407_19930_amd/csrc/common.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


WORKLOADS = {"tiny": 0, "diamond8": 1, "twospecies32": 2, "sheet": 3, "sheet2x2x1": 33, "serving": 4}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16x3", "fp64"])
    ap.add_argument("--workload", default="sheet",
                    help="workload: sheet (75-atom sheet + triatomic at Gamma, the default), sheet2x2x1 (the same "
                         "cell on a 2x2x1 k-mesh), diamond8 (8-atom diamond-like cell, 4x4x4), twospecies32 "
                         "(32-atom two-species cell, 3x3x1), serving (64 cells in one graph), tiny; or the "
                         "index 0-4 (33 = sheet2x2x1)")
    ap.add_argument("--lanes", type=int, default=8, help="concurrent lanes of the serving batch")
    ap.add_argument("--gen-workers", type=int, default=16, help="processes generating the serving cells")
    ap.add_argument("--ncells", type=int, default=64, help="serving cells used (the first n of 64)")
    ap.add_argument("--serving-oracle-cells", type=int, default=8,
                    help="serving cells of at most 4 atoms at Gamma checked against the FP64 oracle")
    ap.add_argument("--no-fp64-check", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", default="auto",
                    help="launch variants of the chi0 kernels: 'auto' (rpa_plan_autotune before the warm-up) or "
                         "NSTAGE_ORDER,NSTAGE_KSTEP,FUSED_ORDER[,FUSED_SINGLE[,NSTAGE_BM]] set explicitly (e.g. "
                         "0,16,0, the plan defaults)")
    ap.add_argument("--tau-batch", type=int, default=0,
                    help="tau points per N-stage / fused launch of the timed path (0: as many as keep the "
                         "per-tau workspace within --tau-batch-gib)")
    ap.add_argument("--tau-batch-gib", type=float, default=96.0)
    ap.add_argument("--screening", type=float, default=1e-3,
                    help="threshold of the extra screened build timed after the steps (0: none)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 1 GiB device copy first (reference dispatch for the byte counters)")
    a = ap.parse_args()
    a.workload = WORKLOADS[a.workload] if a.workload in WORKLOADS else int(a.workload)
    if a.workload not in WORKLOADS.values():
        ap.error("unknown workload %r" % a.workload)
    return a


def host_info():
    """Host CPU description for the cpu_baseline record: model name, logical CPUs the OS
    reports, CPUs this process may run on, and the BLAS threads numpy uses."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 0) for t in threadpool_info()] + [1])
    except Exception:
        threads = affinity
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "cpus_usable": affinity, "blas_threads": threads}


def recorded_counters(kernel, precision, workload):
    """MFMA-busy fraction of a kernel from the committed counter summary (a line
    `mfma_busy <kernel> <precision> <workload> <fraction> <hash>`), or None when absent or taken
    with other kernel sources."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s_%s.md" % (kernel, workload, precision))
    if not os.path.exists(path):
        return None
    cur = kernel_source_hash()
    with open(path) as fh:
        for line in fh:
            f = line.strip().strip("`").split()
            if len(f) == 6 and f[0] == "mfma_busy" and f[1:4] == [kernel, precision, workload]:
                return float(f[4]) if f[5] == cur else None
    return None


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def tuning_tag(tuning):
    """NSTAGE_ORDER,NSTAGE_KSTEP,FUSED_ORDER,FUSED_SINGLE,NSTAGE_BM of a tuning dict (the form
    --tuning takes)."""
    return "%d,%d,%d,%d,%d" % (tuning["nstage_order"], tuning["nstage_kstep"], tuning["fused_order"],
                               tuning.get("fused_single", 0), tuning.get("nstage_bm", 128))


def same_variant(kernel, tag_a, tag_b):
    """Whether two tuning tags launch `kernel` alike: the N stage depends on its order, K step and
    tile rows, the fused kernel on its item order and single-launch mode."""
    d = ["0", "16", "0", "0", "128"]
    a, b = tag_a.split(","), tag_b.split(",")
    a += d[len(a):]
    b += d[len(b):]
    return (a[:2] + a[4:]) == (b[:2] + b[4:]) if kernel == "nstage" else a[2:4] == b[2:4]


def recorded_traffic(kernel, precision, workload, tuning):
    """HBM bytes per tau point from the committed counter summary (the bench multiplies them by
    the tau points of one launch), or None when there is none for this kernel/precision/workload
    and launch variant, or the kernel sources changed since it was taken.  The summary holds lines
    `traffic <kernel> <precision> <workload> <bytes per tau> <hash> <tuning>`."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s_%s.md" % (kernel, workload, precision))
    if not os.path.exists(path):
        return None
    cur = kernel_source_hash()
    with open(path) as fh:
        for line in fh:
            f = line.strip().strip("`").split()
            if len(f) == 7 and f[0] == "traffic" and f[1:4] == [kernel, precision, workload] and \
                    same_variant(kernel, f[6], tuning_tag(tuning)):
                return float(f[4]) if f[5] == cur else None
    return None


def green_build(ctx, inp):
    """Time build_green_tau for every tau of the workload (FP64).  Flops: per (tau, channel, k)
    the complex product of nb x nbands by nbands x nb (8 nb^2 nbands), then the real part of the
    k -> R sum (4 flops per k, R and matrix element)."""
    import torch
    from paper_2407_19930_amd import build_green_tau, rpa_green_workspace_size
    nk, nb = inp.eps.shape
    eps = torch.from_numpy(np.ascontiguousarray(inp.eps)).cuda()
    wfc = torch.from_numpy(np.ascontiguousarray(inp.wfc)).cuda()
    ws = torch.empty(rpa_green_workspace_size(nk, nb, inp.nocc), dtype=torch.uint8, device="cuda")
    Go = torch.empty((inp.ntau, inp.nR, nb, nb), dtype=torch.float64, device="cuda")
    Gu = torch.empty_like(Go)
    build_green_tau(ctx, eps, wfc, inp.nocc, inp.mu, inp.tau, inp.cell.mesh, inp.kfrac, ws, Go, Gu)
    torch.cuda.synchronize()
    ctx.profile(True)
    build_green_tau(ctx, eps, wfc, inp.nocc, inp.mu, inp.tau, inp.cell.mesh, inp.kfrac, ws, Go, Gu)
    ms, _ = ctx.profile_read("green")
    ctx.profile(False)
    err = max(float((Go - torch.from_numpy(inp.Gocc).cuda()).abs().max()),
              float((Gu - torch.from_numpy(inp.Gun).cuda()).abs().max()))
    flops = inp.ntau * nk * (8.0 * nb * nb * nb + 2 * 4.0 * inp.nR * nb * nb)
    out_bytes = 2.0 * inp.ntau * inp.nR * nb * nb * 8
    return {"ms": ms, "tflops": flops / (ms * 1e-3) / 1e12, "G_written_GBps": out_bytes / (ms * 1e-3) / 1e9,
            "max_abs_diff_vs_input_G": err}


def cpu_baseline(inp, budget_s):
    """Time the FP64 oracle (Algorithm 1) on a bounded sample: tau_0, atom V = 0, its N
    intermediate for every (K, dR), then blocks (U, V=0, R) until the time budget is spent."""
    from oracle import chi0 as ochi
    host = host_info()
    alg = ochi.Alg1(inp)
    nao, naux, nR, nb = inp.nao, inp.naux, inp.nR, inp.nb
    S = [sum(nao[inp.blocks.K[b]] for b in alg.nbrs[a]) for a in range(inp.natoms)]
    V = 0
    t0 = time.perf_counter()
    alg.N_all(0, V)
    flops = 2.0 * nR * 2.0 * naux[V] * nao[V] * nb * S[V]
    nblk = 0
    for U in range(inp.natoms):
        for R in range(nR):
            if time.perf_counter() - t0 > budget_s:
                break
            alg.block(0, U, V, R)
            nU, aU, nV, aV = nao[U], naux[U], nao[V], naux[V]
            flops += 2.0 * 2.0 * nU * aV * nV * S[V] + 8.0 * nU * nV * aV * S[U] + 2.0 * aU * aV * nU * S[U]
            nblk += 1
    dt = time.perf_counter() - t0
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(host["blas_threads"]), "kind": "oracle",
            "sample": "tau_0, N intermediate of atom 0 for all (K, dR), then %d blocks (U, V=0, R) of "
                      "Algorithm 1; %.1f s, %.3g algorithmic flops" % (nblk, dt, flops),
            "host": host}


def _gen_cell(cell):
    from threadpoolctl import threadpool_limits
    from rpa_synth import make_inputs
    with threadpool_limits(1):
        return make_inputs(cell)


def serving_main(args):
    """Workload 4: 64 independent cells (2-16 atoms, k-meshes 1/8/27, 8-16 tau), the whole path
    of every cell in one captured graph; one step = one graph launch plus the result read."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import torch
    from paper_2407_19930_amd import Context
    from paper_2407_19930_amd.batching import make_batch
    from rpa_synth.configs import serving_cells
    cells = serving_cells()[:args.ncells]
    dev = "cuda"
    t0 = time.perf_counter()
    io, natoms, names, small = [], [], [], []
    with cf.ProcessPoolExecutor(max_workers=max(1, args.gen_workers), mp_context=mp.get_context("fork")) as ex:
        for k, inp in enumerate(ex.map(_gen_cell, cells)):
            if inp.natoms <= 4 and inp.nR == 1:
                small.append((k, inp))          # small enough for the FP64 oracle
            b = inp.blocks
            io.append(dict(nao=inp.nao, naux=inp.naux, mesh=inp.cell.mesh, blk_I=b.I, blk_K=b.K, blk_R=b.R,
                           blk_off=b.off, ntau=inp.ntau, spin_factor=inp.spin_factor, gamma_cos=inp.gamma_cos,
                           womega=inp.womega, q_frac=inp.kfrac, G_occ=torch.from_numpy(inp.Gocc).to(dev),
                           G_un=torch.from_numpy(inp.Gun).to(dev), C=torch.from_numpy(b.C).to(dev),
                           v_q=torch.from_numpy(inp.vq).to(dev)))
            natoms.append(inp.natoms)
            names.append(inp.cell.name)
            del inp
            log("cell %d/%d ready (%.0f s)" % (k + 1, len(cells), time.perf_counter() - t0))
    small = small[:args.serving_oracle_cells]
    gen_s = time.perf_counter() - t0
    natoms = np.array(natoms)
    ctx = Context(0)
    extra = {}
    ec64 = None
    if not args.no_fp64_check and args.precision != "fp64":
        t0 = time.perf_counter()
        b64, _, _ = make_batch(ctx, io, args.lanes, "fp64")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        b64.run()
        ec64, _ = b64.result()
        extra["fp64_ms_per_step"] = (time.perf_counter() - t1) * 1e3
        log("fp64 reference batch: capture %.1f s, run %.2f s" % (t1 - t0, extra["fp64_ms_per_step"] / 1e3))
        b64.close()
        del b64
        torch.cuda.empty_cache()
    t0 = time.perf_counter()
    batch, plans, lanes = make_batch(ctx, io, args.lanes, args.precision, tune=args.tuning == "auto")
    torch.cuda.synchronize()
    capture_s = time.perf_counter() - t0
    log("batch of %d cells in %d lanes captured in %.1f s" % (len(io), args.lanes, capture_s))
    alg = sum(p.flops()[0] for p in plans)
    for i in range(args.warmup):
        batch.run()
        batch.result()
        log("warmup step %d done" % i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        batch.run()
        ec, _ = batch.result()
        log("timed step %d done" % i)
    dt = (time.perf_counter() - t0) / args.steps
    if ec64 is not None:
        d = np.abs(ec - ec64) / natoms
        extra["max_dEc_per_atom_vs_fp64"] = float(d.max())
        extra["worst_cell"] = names[int(d.argmax())]
        extra["speedup_vs_fp64"] = extra["fp64_ms_per_step"] / (dt * 1e3)
    # the fused kernel of every cell once more, outside the graph and timed with HIP events
    # (the graph overlaps cells, so its kernels have no per-cell durations): the roofline of the
    # batch's dominant kernel over all cells
    from paper_2407_19930_amd import build_chi0_tau
    fused_ms, fused_alg = 0.0, 0.0
    for c, p in zip(io, plans):
        ws = torch.empty(max(p.workspace_bytes, 1), dtype=torch.uint8, device=dev)
        chi = torch.empty(p.ntau * p.nR * p.nauxtot ** 2, dtype=torch.float64, device=dev)
        ctx.profile(True)
        build_chi0_tau(p, c["spin_factor"], c["G_occ"], c["G_un"], c["C"], ws, chi)
        fused_ms += ctx.profile_read("fused")[0]
        ctx.profile(False)
        fused_alg += p.stage_flops(1)[0]
        del ws, chi
    peak = PEAK_BF16X3_FP32EQ if args.precision == "bf16x3" else PEAK_TFLOPS[args.precision]
    ach = fused_alg / (fused_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                "traffic": None, "kernel": "fused", "launches_per_step": None,
                "avg_launch_ms": fused_ms / len(io), "note": "sum over the cells' fused-kernel time, each cell "
                "built once outside the graph"}
    # per-cell E_c against the FP64 oracle on the cells small enough for it, and the oracle's
    # time on them as the CPU baseline (same algorithmic flop count per cell)
    cpu = None
    if small and not args.no_cpu_baseline:
        from oracle import chi0 as ochi
        from oracle.pipeline import ec_from_chi_tau
        host = host_info()
        t1 = time.perf_counter()
        dmax, worst, oflops = 0.0, None, 0.0
        for k, inp in small:
            ec_ref, _, _ = ec_from_chi_tau(inp, ochi.chi0_alg1(inp))
            dd = abs(ec[k] - ec_ref) / inp.natoms
            if dd >= dmax:
                dmax, worst = dd, names[k]
            oflops += plans[k].flops()[0]
        tcpu = time.perf_counter() - t1
        extra["oracle_cells"] = len(small)
        extra["max_dEc_per_atom_vs_oracle"] = dmax
        extra["worst_cell_vs_oracle"] = worst
        cpu = {"value": oflops / tcpu / 1e12, "unit": "TFLOP/s", "cores": int(host["blas_threads"]),
               "kind": "oracle", "cells_per_s": len(small) / tcpu,
               "sample": "%d serving cells of at most 4 atoms at Gamma, whole path (Algorithm 1, transforms, "
                         "LU log-det); %.1f s" % (len(small), tcpu), "host": host}
        log("oracle on %d small cells: max dE_c/atom %.3g, %.1f s" % (len(small), dmax, tcpu))
    rec = {
        "metric": "chi0(R,tau) build TFLOP/s + E_c time, mixed vs FP64 at |dE_c| <= 1e-6 Ha/atom",
        "value": alg / dt / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "serving: %d cells of 2-16 atoms (%d atoms), k-meshes 1/8/27, 8-16 tau, rcut 8 A, "
                               "one graph launch, %d lanes" % (len(io), int(natoms.sum()), args.lanes),
                   "ncells": len(io), "natoms_total": int(natoms.sum()), "lanes": args.lanes},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cells_per_s": len(io) / dt,
        "alg_tflop_per_step": alg / 1e12,
        "capture_s": capture_s,
        "input_generation_s": gen_s,
        "Ec_per_atom_range": [float((ec / natoms).min()), float((ec / natoms).max())],
    }
    rec.update(extra)
    print(json.dumps(rec))


def ec_stage_rate(n, q_frac, v_real, nomega, kt, steps):
    """FP64 rate of the energy stage (GEMMs and Cholesky factorisations, against the 78.6 TFLOP/s
    FP64 MFMA peak), with the usual flop counts (a complex multiply-add is 8 real flops).  Per
    (q, omega), complex: T = chi L with L lower triangular (n^3 / 2 complex multiply-adds, 4 n^3
    flops), B = L^H T on the lower triangle (n^3 / 6, 4 n^3 / 3 flops), the Cholesky of I - B
    (n^3 / 6, 4 n^3 / 3 flops): 20 n^3 / 3; per q the Cholesky of v(q), 4 n^3 / 3.  `model` counts
    every q as complex.  `executed` counts what the path runs: where chi(q) is real (time-reversal
    invariant q: every fractional component 0 or 1/2) T takes two real products per complex one
    (2 n^3), and where v(q) is real as well every step is real (n^3 + n^3 / 3 + n^3 / 3 per
    (q, omega), n^3 / 3 for the Cholesky of v)."""
    q = np.asarray(q_frac).reshape(-1, 3)
    nq = len(q)
    trim = np.all(np.isclose(np.mod(2.0 * q, 1.0), 0.0) | np.isclose(np.mod(2.0 * q, 1.0), 1.0), axis=1)
    both = trim & np.asarray(v_real, dtype=bool)
    n3 = float(n) ** 3
    model = nq * (nomega * 20.0 / 3.0 + 4.0 / 3.0) * n3
    executed = 0.0
    for t, r in zip(trim, both):
        if r:
            executed += (nomega * 5.0 / 3.0 + 1.0 / 3.0) * n3
        elif t:
            executed += (nomega * 14.0 / 3.0 + 4.0 / 3.0) * n3
        else:
            executed += (nomega * 20.0 / 3.0 + 4.0 / 3.0) * n3
    ms = kt["ec_stage"][0] / steps
    return {"ms": ms, "model_tflop": model / 1e12, "executed_tflop": executed / 1e12, "real_chi_q": int(trim.sum()),
            "real_q": int(both.sum()), "nq": nq,
            "model_tflops": model / (ms * 1e-3) / 1e12, "executed_tflops": executed / (ms * 1e-3) / 1e12,
            "executed_frac_fp64_peak": executed / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"]}


def gate(chi_err, dEc):
    """Accuracy bars of the mixed path against the FP64 path on the same inputs."""
    return {"chi_rel_err_vs_fp64": chi_err, "dEc_per_atom_vs_fp64": dEc, "chi_bar": 1e-5, "dEc_bar": 1e-6,
            "pass": bool(chi_err <= 1e-5 and dEc <= 1e-6)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the path is measured on one MI355X "
              "(multi-GPU sharding is a design note only); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == 4:
        return serving_main(args)
    import torch
    from paper_2407_19930_amd import (Context, Plan, build_chi0_tau, chi0_R_to_q, chi0_tau_to_omega,
                                      rpa_correlation_energy, rpa_ec_workspace_size)
    from rpa_synth import config, make_inputs

    cell = config(args.workload)
    t0 = time.perf_counter()
    inp = make_inputs(cell)
    log("inputs generated in %.1f s: %s natoms=%d nb=%d naux=%d nR=%d ntau=%d nblk=%d"
        % (time.perf_counter() - t0, cell.name, inp.natoms, inp.nb, inp.nauxtot, inp.nR, inp.ntau,
           len(inp.blocks.I)))
    dev = "cuda"
    Gocc = torch.from_numpy(inp.Gocc).to(dev)
    Gun = torch.from_numpy(inp.Gun).to(dev)
    C = torch.from_numpy(inp.blocks.C).to(dev)
    vq = torch.from_numpy(inp.vq).to(dev)
    N, nR, nt, nw, nq = inp.nauxtot, inp.nR, inp.ntau, len(inp.omega), len(inp.kfrac)
    # chi(tau) and chi(q, i omega) share one buffer: chi(tau) is dead once chi(i omega) exists
    big = torch.empty(max(nt * nR, 2 * nw * nq) * N * N, dtype=torch.float64, device=dev)
    chi_tau = big[:nt * nR * N * N].view(nt, nR, N, N)
    chi_w = torch.empty((nw, nR, N, N), dtype=torch.float64, device=dev)
    ws_ec = torch.empty(rpa_ec_workspace_size(N, nq, nw), dtype=torch.uint8, device=dev)
    ctx = Context(0)
    b = inp.blocks
    if args.calibrate_copy:
        # 2^28 floats: 1 GiB read and 1 GiB written by one copy kernel
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy done (1 GiB read, 1 GiB written)")

    def make_plan(prec):
        p = Plan(ctx, inp.nao, inp.naux, cell.mesh, b.I, b.K, b.R, b.off, nt, prec)
        return p, torch.empty(max(p.workspace_bytes, 1), dtype=torch.uint8, device=dev)

    def chi_q_view():
        return big[:2 * nw * nq * N * N].view(torch.complex128).view(nw, nq, N, N)

    def step(plan, ws, keep_chi=None):
        build_chi0_tau(plan, inp.spin_factor, Gocc, Gun, C, ws, chi_tau)
        if keep_chi is not None:
            keep_chi.copy_(chi_tau)
        chi0_tau_to_omega(ctx, inp.gamma_cos, chi_tau, chi_w)
        cq = chi_q_view()
        chi0_R_to_q(ctx, cell.mesh, inp.kfrac, chi_w, cq)
        return rpa_correlation_energy(ctx, inp.womega, cq, vq, ws_ec)

    build_kernels = ("pack_c", "pad_g", "screen", "nstage", "split_n", "fused")
    ec_kernels = ("cos_transform", "r2q", "ec_stage")

    def read_profile(steps):
        kt = {k: ctx.profile_read(k) for k in build_kernels + ec_kernels}
        return (kt, sum(kt[k][0] for k in build_kernels) / steps, sum(kt[k][0] for k in ec_kernels) / steps)

    extra = {}
    fp64 = None
    chi64 = None
    if not args.no_fp64_check and args.precision != "fp64":
        p64, ws64 = make_plan("fp64")
        chi64 = torch.empty_like(chi_tau)
        step(p64, ws64, chi64)                      # untimed
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        ec64, _ = step(p64, ws64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        _, b64, e64 = read_profile(1)
        ctx.profile(False)
        a64, _ = p64.flops()
        log("fp64 reference step %.2f s (build %.0f ms, E_c stage %.0f ms), E_c/atom %.12g"
            % (t64, b64, e64, ec64 / inp.natoms))
        del ws64, p64
        torch.cuda.empty_cache()
        fp64 = {"ms_per_step": t64 * 1e3, "build_ms": b64, "build_tflops": a64 / (b64 * 1e-3) / 1e12,
                "ec_time_ms": e64, "Ec_per_atom": ec64 / inp.natoms}
    plan, ws = make_plan(args.precision)
    # tau points per launch: as many as keep the per-tau part of the workspace within the budget
    ws1 = plan.workspace_bytes
    tb = args.tau_batch
    if tb <= 0:
        tb = nt
        while tb > 1:
            need = plan.set_tau_batch(tb)
            if need - ws1 <= args.tau_batch_gib * 2 ** 30:
                break
            tb = max(1, tb // 2)
    need = plan.set_tau_batch(min(tb, nt))
    del ws
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    log("tau points per launch: %d (workspace %.1f GB)" % (min(tb, nt), need / 1e9))
    alg_flops, exec_flops = plan.flops()
    if args.tuning == "auto":
        # times the variants on tau_0 (outside the timed steps); chi_tau[0] is the scratch
        t = plan.autotune(inp.spin_factor, Gocc, Gun, C, ws, chi_tau[0])
        log("autotune: %s" % t.as_dict())
    else:
        plan.set_tuning(*[int(x) for x in args.tuning.split(",")])
    tuning = plan.tuning.as_dict()
    for i in range(args.warmup):
        step(plan, ws)
        log("warmup step %d done" % i)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        ec, ecq = step(plan, ws)
        log("timed step %d done" % i)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    kt, build_ms, ec_ms = read_profile(args.steps)
    ctx.profile(False)
    if chi64 is not None:
        # one more build for the chi(tau) error (the timed steps overwrite chi(tau) with chi(q))
        build_chi0_tau(plan, inp.spin_factor, Gocc, Gun, C, ws, chi_tau)
        torch.cuda.synchronize()
        chi_err = float(torch.linalg.vector_norm(chi_tau - chi64) / torch.linalg.vector_norm(chi64))
    if args.screening > 0:
        # the Green's-function-screened build of the same plan (threshold of the paper's case
        # study by default), outside the timed steps: one untimed and one timed build, the kept
        # share of the fused kernel's K(R1) slices, and its chi and E_c against the FP64 path
        plan.set_screening(args.screening)
        build_chi0_tau(plan, inp.spin_factor, Gocc, Gun, C, ws, chi_tau)
        torch.cuda.synchronize()
        ctx.profile(True)
        build_chi0_tau(plan, inp.spin_factor, Gocc, Gun, C, ws, chi_tau)
        sb_ms = sum(ctx.profile_read(k)[0] for k in build_kernels)
        sf_ms = ctx.profile_read("fused")[0]
        ctx.profile(False)
        st = plan.screening_stats()
        rec_s = {"theta": args.screening, "build_ms": sb_ms, "fused_ms": sf_ms,
                 "build_speedup_vs_unscreened": build_ms / sb_ms,
                 "slices_kept_frac": st["slices_kept"] / max(st["slices_total"], 1),
                 "z_kept_frac": st["z_kept"] / max(st["z_total"], 1)}
        if chi64 is not None:
            rec_s["chi_rel_err_vs_fp64"] = float(torch.linalg.vector_norm(chi_tau - chi64) /
                                                 torch.linalg.vector_norm(chi64))
            chi0_tau_to_omega(ctx, inp.gamma_cos, chi_tau, chi_w)
            chi0_R_to_q(ctx, cell.mesh, inp.kfrac, chi_w, chi_q_view())
            ec_s, _ = rpa_correlation_energy(ctx, inp.womega, chi_q_view(), vq, ws_ec)
            rec_s["dEc_per_atom_vs_fp64"] = abs(ec_s - fp64["Ec_per_atom"] * inp.natoms) / inp.natoms
        plan.set_screening(0.0)
        extra["screened"] = rec_s
        log("screened build: %s" % rec_s)
    if chi64 is not None:
        del chi64
    # the step's device buffers are not needed any more (the 2x2x1 sheet fills most of the HBM)
    del ws, ws_ec, chi_w, chi_tau, big
    torch.cuda.empty_cache()

    # the Green's functions of the step's input, built on the GPU from the eigenpairs (outside the
    # timed steps, which take G as given): one untimed and one timed call
    if inp.wfc is not None:
        extra["green_build"] = green_build(ctx, inp)
        log("green build: %s" % extra["green_build"])

    # dominant kernel and its roofline
    dom = max(("nstage", "fused"), key=lambda k: kt[k][0])
    stage = 0 if dom == "nstage" else 1
    st_alg, st_exec = plan.stage_flops(stage)
    avg_ms = kt[dom][0] / max(kt[dom][1], 1)
    launches_per_step = kt[dom][1] / args.steps
    achieved = st_alg / launches_per_step / (avg_ms * 1e-3) / 1e12
    executed = st_exec / launches_per_step / (avg_ms * 1e-3) / 1e12
    # split-BF16 kernels are priced against the FP32-equivalent split-BF16 peak; a BF16X3 plan too
    # large for the split-BF16 N stage runs the FP32 one (it then has a K-step choice)
    if args.precision == "bf16x3":
        split_n = tuning["nstage_kstep"] == 0
        peak = PEAK_BF16X3_FP32EQ if (dom == "fused" or split_n) else PEAK_TFLOPS["fp32"]
    else:
        peak = PEAK_TFLOPS[args.precision]
    tr = recorded_traffic(dom, args.precision, cell.name, tuning)
    roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": tr * nt / launches_per_step if tr is not None else None, "kernel": dom,
                "launches_per_step": launches_per_step, "avg_launch_ms": avg_ms,
                "executed_achieved": executed, "executed_frac": executed / peak,
                "mfma_busy": recorded_counters(dom, args.precision, cell.name)}
    other = "fused" if dom == "nstage" else "nstage"
    o_alg, o_exec = plan.stage_flops(1 - stage)
    o_ms = kt[other][0] / args.steps
    extra["other_kernel"] = {"kernel": other, "ms_per_step": o_ms,
                             "achieved": o_alg / (o_ms * 1e-3) / 1e12 if o_ms > 0 else None,
                             "frac": o_alg / (o_ms * 1e-3) / 1e12 / peak if o_ms > 0 else None}

    if fp64 is not None:
        dEc = abs(ec - fp64["Ec_per_atom"] * inp.natoms) / inp.natoms
        extra["gate"] = gate(chi_err, dEc)
        extra["fp64"] = fp64
        extra["speedup_vs_fp64"] = fp64["ms_per_step"] / (dt * 1e3)
        extra["build_speedup_vs_fp64"] = fp64["build_ms"] / build_ms
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(inp, args.cpu_seconds)
        log("cpu baseline: %s" % cpu)

    rec = {
        "metric": "chi0(R,tau) build TFLOP/s + E_c time, mixed vs FP64 at |dE_c| <= 1e-6 Ha/atom",
        "value": alg_flops / dt / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "%s: %d atoms, %d NAO / %d ABF per cell, %dx%dx%d k-mesh, %d tau, rcut %.0f A"
                   % (cell.name, inp.natoms, inp.nb, N, *cell.mesh, nt, cell.rcut),
                   "natoms": inp.natoms, "nao_total": inp.nb, "naux_total": N, "mesh": list(cell.mesh),
                   "ntau": nt, "rcut": cell.rcut, "lri_blocks": int(len(b.I))},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "tuning": tuning,
        "alg_tflop_per_step": alg_flops / 1e12,
        "exec_tflop_per_step": exec_flops / 1e12,
        "build_ms": build_ms,
        "build_tflops": alg_flops / (build_ms * 1e-3) / 1e12,
        "ec_time_ms": ec_ms,
        "ec_stage": ec_stage_rate(N, inp.kfrac, [bool(np.all(v.imag == 0)) for v in inp.vq], len(inp.omega), kt,
                                  args.steps),
        "kernel_ms": {k: v[0] / args.steps for k, v in kt.items()},
        "Ec_per_atom": ec / inp.natoms,
    }
    rec.update(extra)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
