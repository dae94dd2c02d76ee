"""FP64 CPU oracle of the Green's-function-screened chi0 build.

TEST INFRASTRUCTURE ONLY: imported by tests/ and the cpu_baseline leg of bench.py, never by the
GPU library or its binding.

The paper lets the spatial decay of the Green's function limit the range of the lattice vector R
on top of the neighbour-set locality of the LRI coefficients, which makes the response-function
build asymptotically linear in system size (Sec. 2, the closing paragraph of the discussion of
Algorithm 1), and its case study screens with a threshold of 1e-3 on the Green's functions
(Sec. 6).  It gives no rule of its own beyond that.  The rule used here (a reading, documented
with the others) bounds every term of Algorithm 1 by the largest entries of its two
Green's-function factors:

* block bound   gb(U, V, R) = max over channels s and i in U, j in V of |G^s_ij(R, tau)|;
* neighbourhood bound of the N intermediate
                gn(V, K, dR) = max over L(dL) in N[V] of gb(L, K, dR - dL),
  which bounds every Green's function that enters N(V, K, dR);
* g(tau) = the largest gb of the time point.

For the block chi_UV(R, tau) the M terms of a neighbour K(R1) of U (the products of G_UV(R) with
N(V, K, R1 - R)) are dropped when gb(U, V, R) gn(V, K, R1 - R) < theta g^2, and the Z terms of the
block (the products of G_VK(R1 - R) with X_UL(R + dL), over all K(R1) and L(dL)) are dropped when
gn(U, V, R) gn(V, U, -R) < theta g^2.  With theta = 0 nothing is dropped.

Each dropped term is bounded elementwise:
  M terms of K(R1): |d chi_mu nu| <= 2 s gb gn a_mu(U; K, R1) b_nu(V),
  Z terms:          |d chi_mu nu| <= 2 s gn(U, V, R) gn(V, U, -R) b_mu(U) b_nu(V),
with a_mu(U; K, R1) = sum_ik |C^mu_ik(R1)| over the block of K(R1) and
b_nu(V) = sum_j sum_{L(dL) in N[V]} sum_l |C^nu_jl(dL)|.  screening_bound() returns that sum.
"""
from __future__ import annotations

import numpy as np

from .chi0 import Alg1, bvk_sub, cblock


def block_norms(inp, t):
    """gb[U, V, R] = max_s max_{i in U, j in V} |G^s_ij(R, tau_t)|."""
    na, nR = inp.natoms, inp.nR
    out = np.zeros((na, na, nR))
    A = np.maximum(np.abs(inp.Gocc[t]), np.abs(inp.Gun[t]))
    for U in range(na):
        iU = slice(inp.ao_off[U], inp.ao_off[U] + inp.nao[U])
        for V in range(na):
            iV = slice(inp.ao_off[V], inp.ao_off[V] + inp.nao[V])
            out[U, V] = A[:, iU, iV].max(axis=(1, 2))
    return out


def neighbour_norms(inp, gb, nbrs, fR):
    """gn[V, K, dR] = max over L(dL) in N[V] of gb[L, K, dR - dL]."""
    na, nR, mesh = inp.natoms, inp.nR, inp.cell.mesh
    out = np.zeros((na, na, nR))
    for V in range(na):
        for b in nbrs[V]:
            L = inp.blocks.K[b]
            for dR in range(nR):
                r = int(bvk_sub(dR, fR[b], mesh))
                out[V, :, dR] = np.maximum(out[V, :, dR], gb[L, :, r])
    return out


class ScreenedAlg1(Alg1):
    """Algorithm 1 in the paper's order (X, N, M, Z, O, chi += C O) with the screened terms
    dropped.  Counts the kept and dropped neighbour slices and Z parts in `stats`."""

    def __init__(self, inp, theta):
        super().__init__(inp)
        self.theta = float(theta)
        self._norms = {}
        self.stats = {"slices_kept": 0, "slices_total": 0, "z_kept": 0, "z_total": 0}

    def norms(self, t):
        if t not in self._norms:
            gb = block_norms(self.inp, t)
            gn = neighbour_norms(self.inp, gb, self.nbrs, self.fR)
            self._norms = {t: (gb, gn, float(gb.max()))}
        return self._norms[t]

    def masks(self, t, U, V, R):
        """(keep flag of the M terms per neighbour of U, keep flag of the Z terms)."""
        gb, gn, g = self.norms(t)
        cut = self.theta * g * g
        mesh = self.mesh
        keep_m = np.array([gb[U, V, R] * gn[V, self.inp.blocks.K[b], int(bvk_sub(self.fR[b], R, mesh))] >= cut
                           for b in self.nbrs[U]], dtype=bool)
        keep_z = bool(gn[U, V, R] * gn[V, U, int(bvk_sub(0, R, mesh))] >= cut)
        return keep_m, keep_z

    def block(self, t, U, V, R, chunk=24):
        inp = self.inp
        keep_m, keep_z = self.masks(t, U, V, R)
        self.stats["slices_total"] += len(keep_m)
        self.stats["slices_kept"] += int(keep_m.sum())
        self.stats["z_total"] += 1
        self.stats["z_kept"] += int(keep_z)
        iU = slice(inp.ao_off[U], inp.ao_off[U] + inp.nao[U])
        iV = slice(inp.ao_off[V], inp.ao_off[V] + inp.nao[V])
        Go, Gu = inp.Gocc[t], inp.Gun[t]
        X = self.X(t, U, V, R)
        Nall = self.N_all(t, V)
        GuR, GoR = Gu[R, iU, iV], Go[R, iU, iV]
        chi = np.zeros((inp.naux[U], inp.naux[V]))
        nb = self.nbrs[U]
        zf = 1.0 if keep_z else 0.0
        for c0 in range(0, len(nb), chunk):
            Cs, Ns, Gvk_o, Gvk_u, mk = [], [], [], [], []
            for q, b in enumerate(nb[c0:c0 + chunk]):
                K = inp.blocks.K[b]
                iK = slice(inp.ao_off[K], inp.ao_off[K] + inp.nao[K])
                d = int(bvk_sub(self.fR[b], R, self.mesh))
                Cs.append(cblock(inp, b))
                Ns.append(Nall[:, d][..., iK])
                Gvk_o.append(Go[d, iV, iK])
                Gvk_u.append(Gu[d, iV, iK])
                mk.append(np.full(inp.nao[K], 1.0 if keep_m[c0 + q] else 0.0))
            Cb = np.concatenate(Cs, axis=2)
            N = np.concatenate(Ns, axis=3)
            Gvo = np.concatenate(Gvk_o, axis=1)
            Gvu = np.concatenate(Gvk_u, axis=1)
            m = np.concatenate(mk)                                     # per (K R1 k) column
            M1 = np.einsum("ij,vjk->ivk", GuR, N[0], optimize=True) * m
            M2 = np.einsum("ij,vjk->ivk", GoR, N[1], optimize=True) * m
            Z1 = np.einsum("jk,ivj->ivk", Gvo, X[1], optimize=True) * zf
            Z2 = np.einsum("jk,ivj->ivk", Gvu, X[0], optimize=True) * zf
            O = self.combine(M1, M2, Z1, Z2)
            chi += np.einsum("mik,ivk->mv", Cb, O, optimize=True)
        return -inp.spin_factor * chi


def chi0_alg1_screened(inp, theta, taus=None):
    """Screened chi[t, R, mu, nu] and the slice/Z statistics."""
    alg = ScreenedAlg1(inp, theta)
    return alg.full(taus), alg.stats


def chi0_alg1_screened_pairs(inp, theta, taus=None):
    """Screened chi over the atom-pair set the method computes (pairs U <= V, Sec. 3.2): every
    block chi_UV(R) with U <= V from its own keep decisions, and the blocks with U > V from the
    Hermitian relation chi_VU(-R) = chi_UV(R)^T.  Without screening this is Algorithm 1 again (the
    relation holds exactly for the full build); with screening the blocks U > V inherit the
    decisions of their partner.  Returns chi[t, R, mu, nu] and the slice/Z statistics of the
    U <= V blocks."""
    alg = ScreenedAlg1(inp, theta)
    taus = list(range(inp.ntau)) if taus is None else list(taus)
    out = np.zeros((len(taus), inp.nR, inp.nauxtot, inp.nauxtot))
    for it, t in enumerate(taus):
        for U in range(inp.natoms):
            mu = slice(inp.aux_off[U], inp.aux_off[U] + inp.naux[U])
            for V in range(U, inp.natoms):
                nu = slice(inp.aux_off[V], inp.aux_off[V] + inp.naux[V])
                for R in range(inp.nR):
                    blk = alg.block(t, U, V, R)
                    out[it, R, mu, nu] = blk
                    if V != U:
                        out[it, int(bvk_sub(0, R, inp.cell.mesh)), nu, mu] = blk.T
    return out, alg.stats


def screening_bound(inp, theta, t):
    """Elementwise bound B[R, mu, nu] on |chi_screened - chi_full| at tau_t from the terms the
    rule drops (see the module docstring)."""
    alg = ScreenedAlg1(inp, theta)
    gb, gn, g = alg.norms(t)
    cut = theta * g * g
    na, nR, s = inp.natoms, inp.nR, inp.spin_factor
    # b_nu(V): sum over j and the whole neighbourhood of V of |C^nu_jl|
    bvec = []
    for V in range(na):
        acc = np.zeros(inp.naux[V])
        for b in alg.nbrs[V]:
            acc += np.abs(cblock(inp, b)).sum(axis=(1, 2))
        bvec.append(acc)
    B = np.zeros((nR, inp.nauxtot, inp.nauxtot))
    for U in range(na):
        mu = slice(inp.aux_off[U], inp.aux_off[U] + inp.naux[U])
        for V in range(na):
            nu = slice(inp.aux_off[V], inp.aux_off[V] + inp.naux[V])
            for R in range(nR):
                am = np.zeros(inp.naux[U])
                for b in alg.nbrs[U]:
                    K = inp.blocks.K[b]
                    p = gb[U, V, R] * gn[V, K, int(bvk_sub(alg.fR[b], R, alg.mesh))]
                    if p < cut:
                        am += p * np.abs(cblock(inp, b)).sum(axis=(1, 2))
                blk = 2 * s * np.outer(am, bvec[V])
                pz = gn[U, V, R] * gn[V, U, int(bvk_sub(0, R, alg.mesh))]
                if pz < cut:
                    blk += 2 * s * pz * np.outer(bvec[U], bvec[V])
                B[R, mu, nu] = blk
    return B
