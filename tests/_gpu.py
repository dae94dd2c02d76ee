"""Run the HIP path (through the C ABI binding) on a seeded input bundle."""
from __future__ import annotations

import numpy as np


def device_inputs(inp):
    import torch
    dev = "cuda"
    return dict(Gocc=torch.from_numpy(inp.Gocc).to(dev), Gun=torch.from_numpy(inp.Gun).to(dev),
                C=torch.from_numpy(inp.blocks.C).to(dev))


def make_plan(ctx, inp, precision):
    from paper_2407_19930_amd import Plan
    b = inp.blocks
    return Plan(ctx, inp.nao, inp.naux, inp.cell.mesh, b.I, b.K, b.R, b.off, inp.ntau, precision)


def gpu_chi_tau(inp, precision="fp64", ctx=None, dev_in=None):
    import torch
    from paper_2407_19930_amd import Context, build_chi0_tau
    ctx = ctx or Context(0)
    plan = make_plan(ctx, inp, precision)
    d = dev_in or device_inputs(inp)
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    chi = torch.empty((inp.ntau, inp.nR, inp.nauxtot, inp.nauxtot), dtype=torch.float64, device="cuda")
    build_chi0_tau(plan, inp.spin_factor, d["Gocc"], d["Gun"], d["C"], ws, chi)
    torch.cuda.synchronize()
    return chi, plan, ctx


def gpu_pipeline(inp, precision="fp64", ctx=None):
    """chi(R,tau) -> chi(R,iw) -> chi(q,iw) -> E_c on the GPU; returns host arrays and E_c."""
    import torch
    from paper_2407_19930_amd import (Context, chi0_R_to_q, chi0_tau_to_omega, rpa_correlation_energy,
                                      rpa_ec_workspace_size)
    ctx = ctx or Context(0)
    chi, plan, _ = gpu_chi_tau(inp, precision, ctx)
    nw = len(inp.omega)
    nq = len(inp.kfrac)
    N = inp.nauxtot
    chi_w = torch.empty((nw, inp.nR, N, N), dtype=torch.float64, device="cuda")
    chi0_tau_to_omega(ctx, inp.gamma_cos, chi, chi_w)
    chi_q = torch.empty((nw, nq, N, N), dtype=torch.complex128, device="cuda")
    chi0_R_to_q(ctx, inp.cell.mesh, inp.kfrac, chi_w, chi_q)
    vq = torch.from_numpy(inp.vq).to("cuda")
    ws = torch.empty(rpa_ec_workspace_size(N, nq, nw), dtype=torch.uint8, device="cuda")
    ec, ecq = rpa_correlation_energy(ctx, inp.womega, chi_q, vq, ws)
    torch.cuda.synchronize()
    return dict(chi_tau=chi.cpu().numpy(), chi_w=chi_w.cpu().numpy(), chi_q=chi_q.cpu().numpy(), ec=ec, ecq=ecq,
                plan=plan)


def batch_cell(inp, dev_in=None):
    """Per-cell dict for paper_2407_19930_amd.batching.make_batch from a seeded input bundle."""
    import torch
    d = dev_in or device_inputs(inp)
    b = inp.blocks
    return dict(nao=inp.nao, naux=inp.naux, mesh=inp.cell.mesh, blk_I=b.I, blk_K=b.K, blk_R=b.R, blk_off=b.off,
                ntau=inp.ntau, spin_factor=inp.spin_factor, gamma_cos=inp.gamma_cos, womega=inp.womega,
                q_frac=inp.kfrac, G_occ=d["Gocc"], G_un=d["Gun"], C=d["C"],
                v_q=torch.from_numpy(inp.vq).to("cuda"))


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))
