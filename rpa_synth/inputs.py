"""Seeded synthetic inputs of the chi0 / RPA correlation-energy path.

For a Cell this builds, in FP64 on the host:

* hopping blocks h_IK(R) = N(0,1) exp(-d / 2 A) for every neighbour pair inside
  the cutoff (on-site blocks symmetric), with h_KI(-R) = h_IK(R)^T so that
  H(k) = sum_R exp(2 pi i k.R) h(R) is Hermitian and H(-k) = conj(H(k));
* Kohn-Sham-like eigenpairs of H(k) on the Gamma-centred mesh, half of the bands
  occupied at every k, the unoccupied bands rigidly shifted so that the gap is
  exactly 0.1 Ha, chemical potential mid-gap;
* the real-space imaginary-time Green's functions on the BvK supercell, the
  occupied and unoccupied branches of the paper's Eq. (green_mat) written with
  the factors of i taken out (see gocc / gun below);
* LRI triple coefficients: one block C[I,K,R1] of shape [naux_I][nao_I][nao_K]
  per ordered neighbour pair, N(0,1) exp(-d / 3 A) entries, the ABF index on the
  first atom (the paper's Eq. (eq:LRI) stores C^{mu(0)}_{i(0),k(R1)} with mu on I);
* time/frequency grids and cosine weights (rpa_synth.grids);
* a synthetic Hermitian positive-definite Coulomb matrix per q.

The Green's-function lattice sum is input preparation for the chi0 path (the
path itself starts from G and C); it is checked by the oracle's sum-over-states
chi0 and by completeness and trace identities in the tests.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import lattice as lat
from .configs import Cell, rng_for, Q_HAMILTONIAN, Q_LRI, Q_COULOMB
from .grids import make_grids

SPIN_FACTOR = 2.0     # closed shell: each spatial orbital holds two electrons
GAP = 0.1             # Hartree


@dataclasses.dataclass
class LRIBlocks:
    I: np.ndarray        # (nblk,) first atom (carries the ABF index)
    K: np.ndarray        # (nblk,) second atom
    R: np.ndarray        # (nblk,3) unfolded integer lattice vector of K
    d: np.ndarray        # (nblk,) distance in Angstrom
    off: np.ndarray      # (nblk,) element offset into C
    C: np.ndarray        # flat FP64 coefficients, block b is C[off[b]:...] as [naux_I][nao_I][nao_K]
    margin: float        # min |d - rcut| seen during enumeration

    def block(self, b, naux, nao):
        i, k = self.I[b], self.K[b]
        n = naux[i] * nao[i] * nao[k]
        return self.C[self.off[b]:self.off[b] + n].reshape(naux[i], nao[i], nao[k])


@dataclasses.dataclass
class Inputs:
    cell: Cell
    nao: np.ndarray
    naux: np.ndarray
    ao_off: np.ndarray
    aux_off: np.ndarray
    nb: int                     # total NAOs per cell
    nauxtot: int                # total ABFs per cell
    Rvec: np.ndarray            # (nR,3) BvK integer triples
    kfrac: np.ndarray           # (nk,3) fractional k (== q mesh)
    blocks: LRIBlocks
    eps: np.ndarray | None      # (nk,nb) band energies after the scissor
    wfc: np.ndarray | None      # (nk,nb,nb) eigenvectors c_{i n}(k) in columns
    nocc: int
    mu: float
    tau: np.ndarray
    omega: np.ndarray
    womega: np.ndarray
    gamma_cos: np.ndarray       # (nomega, ntau)
    grid_info: dict
    Gocc: np.ndarray            # (ntau, nR, nb, nb)
    Gun: np.ndarray             # (ntau, nR, nb, nb)
    vq: np.ndarray | None       # (nq, nauxtot, nauxtot) complex128
    spin_factor: float = SPIN_FACTOR

    @property
    def natoms(self):
        return len(self.nao)

    @property
    def nR(self):
        return len(self.Rvec)

    @property
    def ntau(self):
        return len(self.tau)


def hopping_blocks(cell: Cell, I, K, R, d):
    """Real hopping blocks for the ordered neighbour pairs (same ordering as the input lists)."""
    rng = rng_for(cell.seed_key, Q_HAMILTONIAN)
    nao = cell.nao
    index = {(int(i), int(k), tuple(int(x) for x in r)): b for b, (i, k, r) in enumerate(zip(I, K, R))}
    blocks = [None] * len(I)
    for b in range(len(I)):
        i, k, r = int(I[b]), int(K[b]), tuple(int(x) for x in R[b])
        if blocks[b] is not None:
            continue
        if i == k and r == (0, 0, 0):
            a = rng.standard_normal((nao[i], nao[i]))
            a = np.triu(a) + np.triu(a, 1).T
            blocks[b] = a
            continue
        h = rng.standard_normal((nao[i], nao[k])) * np.exp(-d[b] / 2.0)
        blocks[b] = h
        partner = index[(k, i, tuple(-x for x in r))]
        blocks[partner] = h.T.copy()
    return blocks


def bloch_hamiltonian(cell: Cell, I, K, R, hblocks, kfrac):
    nao = cell.nao
    off = lat.offsets(nao)
    nb = int(nao.sum())
    H = np.zeros((len(kfrac), nb, nb), dtype=np.complex128)
    ph = np.exp(2j * np.pi * (R @ kfrac.T))        # (nblk, nk)
    for b in range(len(I)):
        i, k = I[b], K[b]
        H[:, off[i]:off[i] + nao[i], off[k]:off[k] + nao[k]] += ph[b][:, None, None] * hblocks[b][None]
    return H


def green_functions(eps, wfc, nocc, mu, tau, kfrac, Rvec):
    """G^occ_{ij}(R,tau) = (1/Nk) sum_k sum_{n occ} c_in c*_jn e^{-2 pi i k.R} e^{-(mu - eps) tau}
    G^un_{ij}(R,tau)  = (1/Nk) sum_k sum_{n un}  c_in c*_jn e^{-2 pi i k.R} e^{-(eps - mu) tau}

    These are the paper's Eq. (green_mat) with G(R, i tau) = i G^un(R, tau) and
    G(R, -i tau) = -i G^occ(R, tau) for tau > 0."""
    nk, nb = eps.shape
    ph = np.exp(-2j * np.pi * (Rvec @ kfrac.T)) / nk     # (nR, nk)
    out = []
    for occ in (True, False):
        sl = slice(0, nocc) if occ else slice(nocc, nb)
        c = wfc[:, :, sl]
        e = eps[:, sl]
        arg = (mu - e) if occ else (e - mu)
        G = np.empty((len(tau), len(Rvec), nb, nb))
        for t, tt in enumerate(tau):
            cw = c * np.exp(-arg * tt)[:, None, :]
            P = np.matmul(cw, np.conj(np.swapaxes(c, 1, 2)))   # (nk, nb, nb)
            g = (ph @ P.reshape(nk, -1)).reshape(len(Rvec), nb, nb)
            imag = np.max(np.abs(g.imag))
            scale = max(np.max(np.abs(g.real)), 1e-300)
            if imag > 1e-10 * scale:
                raise RuntimeError("Green's function not real: %g" % (imag / scale))
            G[t] = g.real
        out.append(G)
    return out[0], out[1]


def lri_blocks(cell: Cell, I, K, R, d, margin):
    rng = rng_for(cell.seed_key, Q_LRI)
    nao, naux = cell.nao, cell.naux
    sizes = naux[I] * nao[I] * nao[K]
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    C = np.empty(int(sizes.sum()))
    for b in range(len(I)):
        C[off[b]:off[b] + sizes[b]] = rng.standard_normal(int(sizes[b])) * np.exp(-d[b] / 3.0)
    return LRIBlocks(I, K, R, d, off, C, margin)


def time_reversal_invariant(q_frac):
    """Whether q = -q modulo the reciprocal lattice (every fractional coordinate 0 or 1/2)."""
    return bool(np.all(np.abs(2.0 * np.asarray(q_frac) - np.round(2.0 * np.asarray(q_frac))) < 1e-12))


def coulomb(cell: Cell, nauxtot, kfrac, note=None):
    """v(q) = s (L L^H + 1e-3 I) / lambda_max(L L^H + 1e-3 I), L complex Gaussian with
    Re, Im ~ N(0, 1/2); s = cell.v_scale.  At a time-reversal invariant q (q = -q modulo the
    reciprocal lattice: every fractional coordinate 0 or 1/2) v(q) = v(-q) = v(q)^* is real,
    as the Coulomb matrix of a real basis is there: L is then real, with entries N(0, 1) (the
    same draws as at any other q, so that the other q points keep their matrices).  note, if
    given, is called after each q."""
    rng = rng_for(cell.seed_key, Q_COULOMB)
    nq = len(kfrac)
    vq = np.empty((nq, nauxtot, nauxtot), dtype=np.complex128)
    for q in range(nq):
        Lr = rng.standard_normal((nauxtot, nauxtot))
        Li = rng.standard_normal((nauxtot, nauxtot))
        if time_reversal_invariant(kfrac[q]):
            v = (Lr @ Lr.T + 1e-3 * np.eye(nauxtot)).astype(np.complex128)
        else:
            L = (Lr + 1j * Li) * np.sqrt(0.5)
            v = L @ L.conj().T + 1e-3 * np.eye(nauxtot)
        v = 0.5 * (v + v.conj().T)
        vq[q] = v * (cell.v_scale / _lambda_max(v))
        if note:
            note("coulomb q %d of %d" % (q + 1, nq))
    return vq


def _lambda_max(v):
    """Largest eigenvalue of a Hermitian positive definite matrix: dense for small sizes,
    Lanczos from a fixed start vector (deterministic) for large ones."""
    n = v.shape[0]
    if n <= 2048:
        return float(np.linalg.eigvalsh(v)[-1])
    from scipy.sparse.linalg import eigsh
    return float(eigsh(v, k=1, which="LA", v0=np.ones(n, dtype=v.dtype), tol=1e-13,
                       return_eigenvectors=False)[0])


def make_inputs(cell: Cell, with_coulomb=True, keep_wfc=True, with_green=True, progress=None) -> Inputs:
    """All seeded inputs of one cell.  progress, if given, is called with the name of each
    stage as it finishes (large cells take minutes)."""
    note = progress or (lambda stage: None)
    I, K, R, d, margin = lat.neighbour_pairs(cell.lattice, cell.frac, cell.rcut)
    nao, naux = cell.nao, cell.naux
    nb, nauxtot = int(nao.sum()), int(naux.sum())
    kfrac = lat.kmesh(cell.mesh)
    Rvec = lat.bvk_vectors(cell.mesh)

    hb = hopping_blocks(cell, I, K, R, d)
    H = bloch_hamiltonian(cell, I, K, R, hb, kfrac)
    eps, wfc = np.linalg.eigh(H)
    note("bands")
    nocc = nb // 2
    vbm = eps[:, nocc - 1].max()
    cbm = eps[:, nocc].min()
    eps = eps.copy()
    eps[:, nocc:] += (vbm + GAP) - cbm
    mu = vbm + GAP / 2
    emin = GAP
    emax = float(eps.max() - eps.min())
    g = make_grids(cell.ntau, emin, emax)
    note("grids")
    Gocc, Gun = green_functions(eps, wfc, nocc, mu, g["tau"], kfrac, Rvec) if with_green else (None, None)
    note("green functions")
    blocks = lri_blocks(cell, I, K, R, d, margin)
    note("LRI blocks")
    vq = coulomb(cell, nauxtot, kfrac, note) if with_coulomb else None
    return Inputs(cell=cell, nao=nao, naux=naux, ao_off=lat.offsets(nao), aux_off=lat.offsets(naux),
                  nb=nb, nauxtot=nauxtot, Rvec=Rvec, kfrac=kfrac, blocks=blocks,
                  eps=eps if keep_wfc else None, wfc=wfc if keep_wfc else None, nocc=nocc, mu=mu,
                  tau=g["tau"], omega=g["omega"], womega=g["womega"], gamma_cos=g["gamma_cos"],
                  grid_info={k: g[k] for k in ("tau_fit_err", "omega_fit_err", "eta", "emin", "emax")},
                  Gocc=Gocc, Gun=Gun, vq=vq)
