"""Assembly of a batch of independent cells for rpa_batch_create: one plan per cell, lanes
balanced by estimated work, per-lane scratch (chi arrays and workspaces) sized for the lane's
largest cell and shared by its cells.  Device memory comes from torch; every step runs in the
library."""
from __future__ import annotations

import numpy as np

from .binding import Batch, Plan, rpa_ec_workspace_size


# energy-stage workspace per lane: enough for a few hundred (q, omega) matrices of the serving
# cells at once, while many lanes share one GPU
EC_LANE_BYTES = 8 << 30


def _work(plan: Plan, nq: int, nomega: int) -> float:
    n = plan.nauxtot
    return plan.flops()[0] + 17.0 * nq * nomega * float(n) ** 3


# per-tau part of a cell's build workspace held at once (padded G and the N intermediate of
# several tau points, rpa_plan_set_tau_batch): every lane holds one such workspace
TAU_BATCH_LANE_BYTES = 6 << 30


def make_batch(ctx, cells, nlanes: int, precision: str = "fp32", tune: bool = False,
               tau_batch_bytes: int = TAU_BATCH_LANE_BYTES):
    """cells: list of dicts holding, per cell,
      host: nao, naux, mesh, blk_I, blk_K, blk_R, blk_off, ntau, spin_factor,
            gamma_cos [nomega, ntau], womega [nomega], q_frac [nq, 3]
      device (torch): G_occ, G_un, C (float64), v_q (complex128 [nq, n, n]).
    Each plan takes as many tau points per launch as keep the per-tau part of its workspace within
    tau_batch_bytes (all of them for most serving cells), and with tune=True its launch variants
    from rpa_plan_autotune on the cell's own inputs (cached by shape class in the context, so
    cells of one shape are timed once).  Returns (Batch, plans, lane of each cell)."""
    import torch
    dev = "cuda"
    plans, shapes = [], []
    for c in cells:
        p = Plan(ctx, c["nao"], c["naux"], c["mesh"], c["blk_I"], c["blk_K"], c["blk_R"], c["blk_off"], c["ntau"],
                 precision)
        nomega, nq = np.asarray(c["gamma_cos"]).shape[0], np.asarray(c["q_frac"]).reshape(-1, 3).shape[0]
        ws1 = p.workspace_bytes
        tb = p.ntau
        while tb > 1 and p.set_tau_batch(tb) - ws1 > tau_batch_bytes:
            tb = max(1, tb // 2)
        p.set_tau_batch(tb)
        if tune:
            ws = torch.empty(max(p.workspace_bytes, 1), dtype=torch.uint8, device=dev)
            scratch = torch.empty(p.nR * p.nauxtot ** 2, dtype=torch.float64, device=dev)
            p.autotune(c["spin_factor"], c["G_occ"], c["G_un"], c["C"], ws, scratch)
            del ws, scratch
        plans.append(p)
        shapes.append((p.nauxtot, p.nR, p.ntau, nomega, nq))
    # largest first onto the least loaded lane
    order = sorted(range(len(cells)), key=lambda i: -_work(plans[i], shapes[i][4], shapes[i][3]))
    load = [0.0] * nlanes
    lane = [0] * len(cells)
    for i in order:
        l = int(np.argmin(load))
        lane[i] = l
        load[l] += _work(plans[i], shapes[i][4], shapes[i][3])
    # per-lane scratch: X holds chi0_tau, later chi0_q (complex); Y holds chi0_omega
    need = [dict(x=0, y=0, bw=1, ew=1) for _ in range(nlanes)]
    for i, (n, nR, ntau, nomega, nq) in enumerate(shapes):
        d = need[lane[i]]
        d["x"] = max(d["x"], max(ntau, 2 * nomega) * nR * n * n)
        d["y"] = max(d["y"], nomega * nR * n * n)
        d["bw"] = max(d["bw"], plans[i].workspace_bytes)
        # the energy stage takes the largest (q, omega) batch that fits; lanes keep it modest
        d["ew"] = max(d["ew"], min(rpa_ec_workspace_size(n, nq, nomega), EC_LANE_BYTES))
    bufs = [dict(x=torch.empty(max(d["x"], 1), dtype=torch.float64, device=dev),
                 y=torch.empty(max(d["y"], 1), dtype=torch.float64, device=dev),
                 bw=torch.empty(d["bw"], dtype=torch.uint8, device=dev),
                 ew=torch.empty(d["ew"], dtype=torch.uint8, device=dev)) for d in need]
    io = []
    for i, c in enumerate(cells):
        n, nR, ntau, nomega, nq = shapes[i]
        b = bufs[lane[i]]
        io.append(dict(plan=plans[i], lane=lane[i], spin_factor=c["spin_factor"], gamma_cos=c["gamma_cos"],
                       womega=c["womega"], q_frac=np.asarray(c["q_frac"]).reshape(-1, 3), G_occ=c["G_occ"],
                       G_un=c["G_un"], C=c["C"], v_q=c["v_q"], build_workspace=b["bw"],
                       chi0_tau=b["x"][:ntau * nR * n * n],
                       chi0_omega=b["y"][:nomega * nR * n * n],
                       chi0_q=b["x"][:2 * nomega * nR * n * n].view(torch.complex128),
                       ec_workspace=b["ew"]))
    batch = Batch(ctx, io, nlanes)
    batch._keep.append(bufs)
    batch._keep.append(plans)
    return batch, plans, lane
