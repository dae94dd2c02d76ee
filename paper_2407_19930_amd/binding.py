"""Thin ctypes binding of librpa_mi355x.so (include/rpa_mi355x.h).

Argument marshalling only: every step of the path runs in the HIP library.
torch tensors provide device memory and the HIP stream; host arrays are numpy.
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librpa_mi355x.so")

RPA_OK, RPA_ERR_ARG, RPA_ERR_SHAPE, RPA_ERR_WORKSPACE, RPA_ERR_NOT_HPD, RPA_ERR_NONFINITE, RPA_ERR_HIP, \
    RPA_ERR_UNSUPPORTED = range(8)
RPA_FP64, RPA_FP32, RPA_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": RPA_FP64, "fp32": RPA_FP32, "bf16x3": RPA_BF16X3}

EXPORTED = ["rpa_create", "rpa_set_stream", "rpa_destroy", "rpa_last_error", "rpa_plan_create",
            "rpa_plan_destroy", "rpa_plan_flops", "rpa_plan_stage_flops", "rpa_profile", "rpa_profile_read",
            "build_chi0_tau", "chi0_tau_to_omega", "chi0_R_to_q", "rpa_ec_workspace_size",
            "rpa_correlation_energy", "rpa_batch_create", "rpa_batch_run", "rpa_batch_result",
            "rpa_batch_destroy", "rpa_plan_autotune", "rpa_plan_get_tuning", "rpa_plan_set_tuning",
            "rpa_green_workspace_size", "build_green_tau", "rpa_noalloc_scratch_bytes",
            "rpa_correlation_energy_noalloc", "rpa_plan_set_screening", "rpa_plan_screening_stats",
            "rpa_plan_set_tau_batch", "rpa_plan_workspace_bytes", "rpa_session_create", "rpa_session_destroy",
            "rpa_session_last_error", "rpa_session_set_precision", "rpa_set_dimension", "rpa_set_wg_ekb_efermi",
            "rpa_set_ao_basis_wfc", "rpa_set_latvec_and_G", "rpa_set_kgrids_kvec_tot",
            "rpa_set_ibz2bz_index_and_weight", "rpa_set_ao_basis_aux", "rpa_set_aux_bare_coulomb_k_atom_pair",
            "rpa_set_aux_bare_coulomb_k_2D_block", "rpa_set_time_freq_grids", "rpa_get_rpa_correlation_energy",
            "rpa_check_green_symmetry"]


class RpaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("rpa error %d: %s" % (code, msg))
        self.code = code


class _Cell(ctypes.Structure):
    _fields_ = [("natoms", ctypes.c_int), ("nao", ctypes.POINTER(ctypes.c_int)),
                ("naux", ctypes.POINTER(ctypes.c_int)), ("mesh", ctypes.c_int * 3)]


class _Blocks(ctypes.Structure):
    _fields_ = [("nblk", ctypes.c_int), ("I", ctypes.POINTER(ctypes.c_int)), ("K", ctypes.POINTER(ctypes.c_int)),
                ("R", ctypes.POINTER(ctypes.c_int)), ("off", ctypes.POINTER(ctypes.c_longlong))]


class _BatchCell(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("lane", ctypes.c_int), ("nomega", ctypes.c_int), ("nq", ctypes.c_int),
                ("spin_factor", ctypes.c_double), ("gamma_cos", ctypes.c_void_p), ("womega", ctypes.c_void_p),
                ("q_frac", ctypes.c_void_p), ("G_occ", ctypes.c_void_p), ("G_un", ctypes.c_void_p),
                ("C", ctypes.c_void_p), ("v_q", ctypes.c_void_p), ("build_workspace", ctypes.c_void_p),
                ("build_workspace_bytes", ctypes.c_size_t), ("chi0_tau", ctypes.c_void_p),
                ("chi0_omega", ctypes.c_void_p), ("chi0_q", ctypes.c_void_p), ("ec_workspace", ctypes.c_void_p),
                ("ec_workspace_bytes", ctypes.c_size_t)]


class Tuning(ctypes.Structure):
    """rpa_tuning: launch variants of a plan's N-stage and fused kernels."""
    _fields_ = [("nstage_order", ctypes.c_int), ("nstage_kstep", ctypes.c_int), ("fused_order", ctypes.c_int),
                ("from_cache", ctypes.c_int), ("nstage_ms", ctypes.c_double), ("fused_ms", ctypes.c_double),
                ("fused_single", ctypes.c_int), ("nstage_bm", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the library (once).  Raises ImportError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("librpa_mi355x.so not built (run __graft_entry__.build() or "
                          "python paper_2407_19930_amd/build.py)")
    lib = ctypes.CDLL(path)
    vp, i, sz, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_double
    lib.rpa_create.argtypes = [ctypes.POINTER(vp), i, vp]
    lib.rpa_set_stream.argtypes = [vp, vp]
    lib.rpa_destroy.argtypes = [vp]
    lib.rpa_destroy.restype = None
    lib.rpa_last_error.argtypes = [vp]
    lib.rpa_last_error.restype = ctypes.c_char_p
    lib.rpa_plan_create.argtypes = [vp, ctypes.POINTER(_Cell), ctypes.POINTER(_Blocks), i, i,
                                    ctypes.POINTER(sz), ctypes.POINTER(vp)]
    lib.rpa_plan_destroy.argtypes = [vp]
    lib.rpa_plan_flops.argtypes = [vp, ctypes.POINTER(dp), ctypes.POINTER(dp)]
    lib.rpa_plan_stage_flops.argtypes = [vp, i, ctypes.POINTER(dp), ctypes.POINTER(dp)]
    lib.rpa_profile.argtypes = [vp, i]
    lib.rpa_profile_read.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(dp), ctypes.POINTER(i)]
    lib.build_chi0_tau.argtypes = [vp, dp, vp, vp, vp, vp, sz, vp]
    lib.chi0_tau_to_omega.argtypes = [vp, i, i, sz, vp, vp, vp]
    lib.chi0_R_to_q.argtypes = [vp, ctypes.POINTER(ctypes.c_int), i, sz, i, vp, vp, vp]
    lib.rpa_ec_workspace_size.argtypes = [i, i, i]
    lib.rpa_ec_workspace_size.restype = sz
    lib.rpa_green_workspace_size.argtypes = [i, i, i]
    lib.rpa_green_workspace_size.restype = sz
    lib.build_green_tau.argtypes = [vp, i, i, i, dp, i, vp, ctypes.POINTER(ctypes.c_int), vp, vp, vp, vp, sz, vp, vp]
    lib.rpa_correlation_energy.argtypes = [vp, i, i, i, vp, vp, vp, vp, sz, ctypes.POINTER(dp), vp]
    lib.rpa_noalloc_scratch_bytes.argtypes = []
    lib.rpa_noalloc_scratch_bytes.restype = sz
    lib.rpa_correlation_energy_noalloc.argtypes = [vp, i, i, i, vp, vp, vp, ctypes.POINTER(dp), vp]
    lib.rpa_batch_create.argtypes = [vp, i, i, ctypes.POINTER(_BatchCell), ctypes.POINTER(vp)]
    lib.rpa_batch_run.argtypes = [vp]
    lib.rpa_batch_result.argtypes = [vp, vp, vp]
    lib.rpa_batch_destroy.argtypes = [vp]
    lib.rpa_plan_autotune.argtypes = [vp, dp, vp, vp, vp, vp, sz, vp, ctypes.POINTER(Tuning)]
    lib.rpa_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    lib.rpa_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    lib.rpa_plan_set_screening.argtypes = [vp, dp]
    lib.rpa_plan_set_tau_batch.argtypes = [vp, i, ctypes.POINTER(sz)]
    lib.rpa_plan_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    lib.rpa_plan_screening_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong)]
    lib.rpa_check_green_symmetry.argtypes = [vp, i, ctypes.POINTER(ctypes.c_int), i, vp, vp, dp, ctypes.POINTER(dp)]
    lib.rpa_session_create.argtypes = [vp, ctypes.POINTER(vp)]
    lib.rpa_session_destroy.argtypes = [vp]
    lib.rpa_session_last_error.argtypes = [vp]
    lib.rpa_session_last_error.restype = ctypes.c_char_p
    lib.rpa_session_set_precision.argtypes = [vp, i]
    lib.rpa_set_dimension.argtypes = [vp, i, i, i, i, i]
    lib.rpa_set_wg_ekb_efermi.argtypes = [vp, i, i, i, vp, vp, dp]
    lib.rpa_set_ao_basis_wfc.argtypes = [vp, i, i, vp, vp]
    lib.rpa_set_latvec_and_G.argtypes = [vp, vp, vp]
    lib.rpa_set_kgrids_kvec_tot.argtypes = [vp, i, i, i, vp]
    lib.rpa_set_ibz2bz_index_and_weight.argtypes = [vp, i, vp, vp]
    lib.rpa_set_ao_basis_aux.argtypes = [vp, i, i, i, i, i, vp, vp, i]
    lib.rpa_set_aux_bare_coulomb_k_atom_pair.argtypes = [vp, i, i, i, i, i, vp, vp]
    lib.rpa_set_aux_bare_coulomb_k_2D_block.argtypes = [vp, i, i, i, i, i, i, vp, vp]
    lib.rpa_set_time_freq_grids.argtypes = [vp, i, vp, vp, vp]
    lib.rpa_get_rpa_correlation_energy.argtypes = [vp, ctypes.POINTER(dp), vp]
    for name in EXPORTED:
        if name not in ("rpa_destroy", "rpa_last_error", "rpa_ec_workspace_size", "rpa_green_workspace_size",
                        "rpa_noalloc_scratch_bytes", "rpa_session_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _dev(t, dtype=None):
    """Device pointer of a contiguous torch tensor (checked)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, t.dtype))
    return ctypes.c_void_p(t.data_ptr())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


class Context:
    """rpa_create / rpa_destroy.  Binds torch's current stream of `device` unless one is given."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.rpa_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if rc != RPA_OK:
            raise RpaError(rc, "rpa_create failed")
        self.h = h
        self._plans = weakref.WeakSet()
        self._batches = weakref.WeakSet()

    def check(self, rc):
        if rc != RPA_OK:
            raise RpaError(rc, self.lib.rpa_last_error(self.h).decode())

    def profile(self, enable: bool):
        """rpa_profile: HIP-event timing of every library kernel launch (resets totals)."""
        self.check(self.lib.rpa_profile(self.h, 1 if enable else 0))

    def profile_read(self, kernel: str):
        """rpa_profile_read: (total milliseconds, launches) of one kernel."""
        ms, n = ctypes.c_double(), ctypes.c_int()
        self.check(self.lib.rpa_profile_read(self.h, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "h", None):
            for b in list(getattr(self, "_batches", ())):
                b.close()               # batches hold graphs that read the plans' tables
            for p in list(getattr(self, "_plans", ())):
                p.close()               # plans hold a pointer to the context
            self.lib.rpa_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """rpa_plan_create for one cell.  Arguments mirror rpa_cell and rpa_lri_blocks."""

    def __init__(self, ctx: Context, nao, naux, mesh, blk_I, blk_K, blk_R, blk_off, ntau: int,
                 precision: str = "fp64"):
        self.ctx = ctx
        self._keep = []
        nao_a, nao_p = _host(nao, np.int32)
        naux_a, naux_p = _host(naux, np.int32)
        cell = _Cell(len(nao_a), ctypes.cast(nao_p, ctypes.POINTER(ctypes.c_int)),
                     ctypes.cast(naux_p, ctypes.POINTER(ctypes.c_int)), (ctypes.c_int * 3)(*[int(x) for x in mesh]))
        I_a, I_p = _host(blk_I, np.int32)
        K_a, K_p = _host(blk_K, np.int32)
        R_a, R_p = _host(np.asarray(blk_R).reshape(-1), np.int32)
        o_a, o_p = _host(blk_off, np.int64)
        blocks = _Blocks(len(I_a), ctypes.cast(I_p, ctypes.POINTER(ctypes.c_int)),
                         ctypes.cast(K_p, ctypes.POINTER(ctypes.c_int)), ctypes.cast(R_p, ctypes.POINTER(ctypes.c_int)),
                         ctypes.cast(o_p, ctypes.POINTER(ctypes.c_longlong)))
        ws = ctypes.c_size_t()
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.rpa_plan_create(ctx.h, ctypes.byref(cell), ctypes.byref(blocks), int(ntau),
                                          PRECISIONS[precision], ctypes.byref(ws), ctypes.byref(h)))
        self.h = h
        ctx._plans.add(self)
        self.workspace_bytes = ws.value
        self.ntau = int(ntau)
        self.precision = precision
        self.nauxtot = int(np.sum(naux_a))
        self.nR = int(np.prod(mesh))

    def flops(self):
        """rpa_plan_flops: (algorithmic, executed) flops of the whole chi0 build."""
        a, e = ctypes.c_double(), ctypes.c_double()
        self.ctx.check(self.ctx.lib.rpa_plan_flops(self.h, ctypes.byref(a), ctypes.byref(e)))
        return a.value, e.value

    def stage_flops(self, stage: int):
        """rpa_plan_stage_flops: stage 0 = N-stage kernel, 1 = fused kernel."""
        a, e = ctypes.c_double(), ctypes.c_double()
        self.ctx.check(self.ctx.lib.rpa_plan_stage_flops(self.h, int(stage), ctypes.byref(a), ctypes.byref(e)))
        return a.value, e.value

    def autotune(self, spin_factor: float, G_occ, G_un, C, workspace, chi0_scratch) -> Tuning:
        """rpa_plan_autotune on the first tau of the inputs; chi0_scratch: float64 device tensor of
        nR * naux_tot^2 elements.  Returns the chosen variants."""
        import torch
        f64 = torch.float64
        if chi0_scratch.numel() < self.nR * self.nauxtot ** 2:
            raise ValueError("chi0_scratch holds fewer than nR * naux_tot^2 elements")
        t = Tuning()
        self.ctx.check(self.ctx.lib.rpa_plan_autotune(self.h, float(spin_factor), _dev(G_occ, f64), _dev(G_un, f64),
                                                      _dev(C, f64), _dev(workspace),
                                                      workspace.numel() * workspace.element_size(),
                                                      _dev(chi0_scratch, f64), ctypes.byref(t)))
        return t

    @property
    def tuning(self) -> Tuning:
        t = Tuning()
        self.ctx.check(self.ctx.lib.rpa_plan_get_tuning(self.h, ctypes.byref(t)))
        return t

    def set_tuning(self, nstage_order: int, nstage_kstep: int, fused_order: int, fused_single: int = 0,
                   nstage_bm: int = 128):
        t = Tuning(int(nstage_order), int(nstage_kstep), int(fused_order), 0, 0.0, 0.0, int(fused_single),
                   int(nstage_bm))
        self.ctx.check(self.ctx.lib.rpa_plan_set_tuning(self.h, ctypes.byref(t)))

    def set_tau_batch(self, ntau_per_launch: int) -> int:
        """rpa_plan_set_tau_batch: tau points per launch; returns (and keeps) the new workspace size."""
        ws = ctypes.c_size_t()
        self.ctx.check(self.ctx.lib.rpa_plan_set_tau_batch(self.h, int(ntau_per_launch), ctypes.byref(ws)))
        self.workspace_bytes = ws.value
        return ws.value

    def set_screening(self, theta: float):
        """rpa_plan_set_screening: Green's-function screening threshold (0 = off)."""
        self.ctx.check(self.ctx.lib.rpa_plan_set_screening(self.h, float(theta)))

    def screening_stats(self) -> dict:
        """rpa_plan_screening_stats of the last screened build."""
        out = (ctypes.c_longlong * 6)()
        self.ctx.check(self.ctx.lib.rpa_plan_screening_stats(self.h, out))
        keys = ("entries_kept", "entries_total", "slices_kept", "slices_total", "z_kept", "z_total")
        return {k: int(v) for k, v in zip(keys, out)}

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            self.ctx.lib.rpa_plan_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_chi0_tau(plan: Plan, spin_factor: float, G_occ, G_un, C, workspace, chi0_tau):
    import torch
    f64 = torch.float64
    ctx = plan.ctx
    ctx.check(ctx.lib.build_chi0_tau(plan.h, float(spin_factor), _dev(G_occ, f64), _dev(G_un, f64),
                                     _dev(C, f64), _dev(workspace), workspace.numel() * workspace.element_size(),
                                     _dev(chi0_tau, f64)))


def chi0_tau_to_omega(ctx: Context, gamma_cos, chi0_tau, chi0_omega):
    import torch
    g, gp = _host(gamma_cos, np.float64)
    nomega, ntau = g.shape
    n = chi0_tau.numel() // ntau
    if chi0_tau.numel() != n * ntau or chi0_omega.numel() != n * nomega:
        raise ValueError("shape mismatch")
    ctx.check(ctx.lib.chi0_tau_to_omega(ctx.h, ntau, nomega, n, gp, _dev(chi0_tau, torch.float64),
                                        _dev(chi0_omega, torch.float64)))


def chi0_R_to_q(ctx: Context, mesh, q_frac, chi0_R, chi0_q):
    """chi0_R: [nbatch, nR, ...] float64; chi0_q: [nbatch, nq, ..., 2] float64 (re, im) or complex128."""
    import torch
    q, qp = _host(q_frac, np.float64)
    nq = q.shape[0]
    nR = int(np.prod(mesh))
    nbatch = chi0_R.shape[0]
    m = chi0_R.numel() // (nbatch * nR)
    if chi0_R.numel() != nbatch * nR * m:
        raise ValueError("shape mismatch")
    out = chi0_q
    if out.dtype == torch.complex128:
        out = torch.view_as_real(out)
    if out.numel() != nbatch * nq * m * 2:
        raise ValueError("output shape mismatch")
    mesh_a = (ctypes.c_int * 3)(*[int(x) for x in mesh])
    ctx.check(ctx.lib.chi0_R_to_q(ctx.h, mesh_a, nbatch, m, nq, qp, _dev(chi0_R, torch.float64), _dev(out)))


def rpa_check_green_symmetry(ctx: Context, mesh, G_occ, G_un, tol: float = 1e-12) -> float:
    """rpa_check_green_symmetry on device tensors [ntau, nR, nb, nb]; returns the relative deviation
    (raises RpaError with RPA_ERR_ARG when it exceeds tol)."""
    import torch
    f64 = torch.float64
    ntau, nR, nb = int(G_occ.shape[0]), int(G_occ.shape[1]), int(G_occ.shape[2])
    if tuple(G_un.shape) != tuple(G_occ.shape) or nR != int(np.prod(mesh)) or int(G_occ.shape[3]) != nb:
        raise ValueError("G_occ / G_un must both be [ntau, nR, nb, nb] on the mesh")
    m = (ctypes.c_int * 3)(*[int(x) for x in mesh])
    dev = ctypes.c_double()
    ctx.check(ctx.lib.rpa_check_green_symmetry(ctx.h, ntau, m, nb, _dev(G_occ, f64), _dev(G_un, f64), float(tol),
                                               ctypes.byref(dev)))
    return dev.value


def rpa_green_workspace_size(nk: int, nb: int, nocc: int) -> int:
    return int(load().rpa_green_workspace_size(int(nk), int(nb), int(nocc)))


def build_green_tau(ctx: Context, eps, wfc, nocc: int, mu: float, tau, mesh, kfrac, workspace, G_occ, G_un):
    """G^occ, G^un [ntau, nR, nb, nb] (float64 device) from band energies eps [nk, nb] (float64 device)
    and eigenvectors wfc [nk, nb, nb] (complex128 device, c_{in}(k) at [k, i, n])."""
    import torch
    nk, nb = eps.shape
    if tuple(wfc.shape) != (nk, nb, nb) or wfc.dtype != torch.complex128:
        raise ValueError("wfc must be complex128 [nk, nb, nb]")
    t, tp = _host(tau, np.float64)
    k, kp = _host(np.asarray(kfrac).reshape(-1, 3), np.float64)
    if k.shape[0] != nk:
        raise ValueError("kfrac must have one row per k")
    nR = int(np.prod(mesh))
    for G in (G_occ, G_un):
        if G.numel() != len(t) * nR * nb * nb:
            raise ValueError("G arrays must hold ntau * nR * nb * nb elements")
    m = (ctypes.c_int * 3)(*[int(x) for x in mesh])
    ctx.check(ctx.lib.build_green_tau(ctx.h, nk, nb, int(nocc), float(mu), len(t), tp, m, kp,
                                      _dev(eps, torch.float64), _dev(wfc, torch.complex128), _dev(workspace),
                                      workspace.numel() * workspace.element_size(), _dev(G_occ, torch.float64),
                                      _dev(G_un, torch.float64)))


def rpa_ec_workspace_size(n: int, nq: int, nomega: int) -> int:
    return int(load().rpa_ec_workspace_size(int(n), int(nq), int(nomega)))


def rpa_correlation_energy(ctx: Context, womega, chi0_q, v_q, workspace):
    """Returns (E_c per cell, per-q contributions).  chi0_q [nomega, nq, n, n] and v_q [nq, n, n]
    complex128 (or float64 with a trailing (re, im) axis)."""
    import torch
    w, wp = _host(womega, np.float64)
    cq = torch.view_as_real(chi0_q) if chi0_q.dtype == torch.complex128 else chi0_q
    vq = torch.view_as_real(v_q) if v_q.dtype == torch.complex128 else v_q
    nomega, nq, n = chi0_q.shape[0], chi0_q.shape[1], chi0_q.shape[2]
    ec = ctypes.c_double()
    ecq = np.zeros(nq)
    ctx.check(ctx.lib.rpa_correlation_energy(ctx.h, n, nq, nomega, wp, _dev(cq, torch.float64),
                                             _dev(vq, torch.float64), _dev(workspace),
                                             workspace.numel() * workspace.element_size(), ctypes.byref(ec),
                                             ecq.ctypes.data_as(ctypes.c_void_p)))
    return ec.value, ecq


def rpa_noalloc_scratch_bytes() -> int:
    return int(load().rpa_noalloc_scratch_bytes())


def rpa_correlation_energy_noalloc(ctx: Context, womega, chi0_q, v_q):
    """As rpa_correlation_energy, with the library's own device scratch instead of a workspace
    (no device allocation in the call).  Returns (E_c per cell, per-q contributions)."""
    import torch
    w, wp = _host(womega, np.float64)
    cq = torch.view_as_real(chi0_q) if chi0_q.dtype == torch.complex128 else chi0_q
    vq = torch.view_as_real(v_q) if v_q.dtype == torch.complex128 else v_q
    nomega, nq, n = chi0_q.shape[0], chi0_q.shape[1], chi0_q.shape[2]
    ec = ctypes.c_double()
    ecq = np.zeros(nq)
    ctx.check(ctx.lib.rpa_correlation_energy_noalloc(ctx.h, n, nq, nomega, wp, _dev(cq, torch.float64),
                                                     _dev(vq, torch.float64), ctypes.byref(ec),
                                                     ecq.ctypes.data_as(ctypes.c_void_p)))
    return ec.value, ecq


class Batch:
    """rpa_batch_create / run / result / destroy: many cells in one captured HIP graph.

    `cells` is a list of dicts with the fields of rpa_batch_cell: plan, lane, spin_factor,
    gamma_cos [nomega, ntau], womega [nomega], q_frac [nq, 3] (host arrays); G_occ, G_un, C,
    v_q (complex128 [nq, n, n]), build_workspace, chi0_tau, chi0_omega, chi0_q (complex128),
    ec_workspace (device tensors).  The tensors are kept alive with the batch, since the graph
    holds their addresses."""

    def __init__(self, ctx: Context, cells, nlanes: int):
        import torch
        f64 = torch.float64
        self.ctx = ctx
        self._keep = [cells]
        arr = (_BatchCell * len(cells))()
        self.nq = []
        for k, c in enumerate(cells):
            g, gp = _host(c["gamma_cos"], np.float64)
            w, wp = _host(c["womega"], np.float64)
            q, qp = _host(c["q_frac"], np.float64)
            self._keep += [g, w, q]
            cq = torch.view_as_real(c["chi0_q"]) if c["chi0_q"].dtype == torch.complex128 else c["chi0_q"]
            vq = torch.view_as_real(c["v_q"]) if c["v_q"].dtype == torch.complex128 else c["v_q"]
            bw, ew = c["build_workspace"], c["ec_workspace"]
            arr[k] = _BatchCell(c["plan"].h, int(c["lane"]), int(w.shape[0]), int(q.shape[0]), float(c["spin_factor"]),
                                gp, wp, qp, _dev(c["G_occ"], f64), _dev(c["G_un"], f64), _dev(c["C"], f64),
                                _dev(vq, f64), _dev(bw), bw.numel() * bw.element_size(), _dev(c["chi0_tau"], f64),
                                _dev(c["chi0_omega"], f64), _dev(cq, f64), _dev(ew), ew.numel() * ew.element_size())
            self.nq.append(int(q.shape[0]))
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.rpa_batch_create(ctx.h, len(cells), int(nlanes), arr, ctypes.byref(h)))
        self.h = h
        self.ncells = len(cells)
        ctx._batches.add(self)

    def run(self):
        """One graph launch of every cell on the context's stream (asynchronous)."""
        self.ctx.check(self.ctx.lib.rpa_batch_run(self.h))

    def result(self):
        """(E_c per cell, per-q terms of every cell concatenated); waits for the stream."""
        ec = np.zeros(self.ncells)
        ecq = np.zeros(sum(self.nq))
        self.ctx.check(self.ctx.lib.rpa_batch_result(self.h, ec.ctypes.data_as(ctypes.c_void_p),
                                                     ecq.ctypes.data_as(ctypes.c_void_p)))
        return ec, ecq

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            self.ctx.lib.rpa_batch_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Session:
    """Input session shaped like the paper's library interface (rpa_session_* and rpa_set_* of the
    C ABI).  Host numpy arrays in, E_c and the per-irreducible-q contributions out; the method
    names are the C names without the rpa_ prefix."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.rpa_session_create(ctx.h, ctypes.byref(h)))
        self.h = h
        self.nq = None
        ctx._plans.add(self)

    def _check(self, rc):
        if rc != 0:
            raise RpaError(rc, self.ctx.lib.rpa_session_last_error(self.h).decode())

    def set_precision(self, precision: str):
        self._check(self.ctx.lib.rpa_session_set_precision(self.h, PRECISIONS[precision]))

    def set_dimension(self, nspins, nkpts, nstates, nbasis, natoms):
        self._check(self.ctx.lib.rpa_set_dimension(self.h, int(nspins), int(nkpts), int(nstates), int(nbasis),
                                                   int(natoms)))
        self.nq = int(nkpts)

    def set_wg_ekb_efermi(self, nspins, nkpts, nstates, wg, ekb, efermi):
        w, wp = _host(wg, np.float64)
        e, ep = _host(ekb, np.float64)
        self._check(self.ctx.lib.rpa_set_wg_ekb_efermi(self.h, int(nspins), int(nkpts), int(nstates), wp, ep,
                                                       float(efermi)))

    def set_ao_basis_wfc(self, ispin, ik, wfc_real, wfc_imag):
        r, rp = _host(wfc_real, np.float64)
        m, mp = _host(wfc_imag, np.float64)
        self._check(self.ctx.lib.rpa_set_ao_basis_wfc(self.h, int(ispin), int(ik), rp, mp))

    def set_latvec_and_G(self, lat_mat, G_mat):
        a, ap = _host(lat_mat, np.float64)
        g, gp = _host(G_mat, np.float64)
        self._check(self.ctx.lib.rpa_set_latvec_and_G(self.h, ap, gp))

    def set_kgrids_kvec_tot(self, nk1, nk2, nk3, kvecs):
        k, kp = _host(kvecs, np.float64)
        self._check(self.ctx.lib.rpa_set_kgrids_kvec_tot(self.h, int(nk1), int(nk2), int(nk3), kp))

    def set_ibz2bz_index_and_weight(self, ibz2bz_index, wk_irk):
        i, ip = _host(ibz2bz_index, np.int32)
        w, wp = _host(wk_irk, np.float64)
        self._check(self.ctx.lib.rpa_set_ibz2bz_index_and_weight(self.h, len(i), ip, wp))
        self.nq = len(i)

    def set_ao_basis_aux(self, I, J, nbasis_i, nbasis_j, naux_mu, R, Cs, insert_index_only=0):
        r, rp = _host(R, np.int32)
        c, cp = _host(Cs, np.float64) if Cs is not None else (None, None)
        self._check(self.ctx.lib.rpa_set_ao_basis_aux(self.h, int(I), int(J), int(nbasis_i), int(nbasis_j),
                                                      int(naux_mu), rp, cp, int(insert_index_only)))

    def set_aux_bare_coulomb_k_atom_pair(self, ik, I, J, naux_mu, naux_nu, Vq_real, Vq_imag):
        r, rp = _host(Vq_real, np.float64)
        m, mp = _host(Vq_imag, np.float64)
        self._check(self.ctx.lib.rpa_set_aux_bare_coulomb_k_atom_pair(self.h, int(ik), int(I), int(J), int(naux_mu),
                                                                      int(naux_nu), rp, mp))

    def set_aux_bare_coulomb_k_2D_block(self, ik, max_naux, mu_begin, mu_end, nu_begin, nu_end, Vq_real, Vq_imag):
        r, rp = _host(Vq_real, np.float64)
        m, mp = _host(Vq_imag, np.float64)
        self._check(self.ctx.lib.rpa_set_aux_bare_coulomb_k_2D_block(self.h, int(ik), int(max_naux), int(mu_begin),
                                                                     int(mu_end), int(nu_begin), int(nu_end), rp, mp))

    def set_time_freq_grids(self, tau, omega_weights, gamma_cos):
        t, tp = _host(tau, np.float64)
        w, wp = _host(omega_weights, np.float64)
        g, gp = _host(gamma_cos, np.float64)
        self._check(self.ctx.lib.rpa_set_time_freq_grids(self.h, len(t), tp, wp, gp))

    def get_rpa_correlation_energy(self):
        """(E_c per cell, contributions of the irreducible q points)."""
        ec = ctypes.c_double()
        contrib = np.zeros(self.nq or 0)
        self._check(self.ctx.lib.rpa_get_rpa_correlation_energy(self.h, ctypes.byref(ec),
                                                                contrib.ctypes.data_as(ctypes.c_void_p)))
        return ec.value, contrib

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            self.ctx.lib.rpa_session_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
