"""Sum-over-states (Adler-Wiser) response function, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Derived from the definition chi(r, r', tau) = -s G^un(r, r', tau) G^occ(r', r, tau)
(Sec. 2, the space-time chi0 and Eq. (green_func)/(green_mat)) by expanding both
Green's functions over Bloch states and each product of two NAOs with
Eq. (eq:LRI):

  chi_{alpha beta}(tau)     = -s sum_{n occ, m un} exp(-(e_m - e_n) tau) L^alpha_nm conj(L^beta_nm)
  chi_{alpha beta}(i omega) = -s sum_{n occ, m un} 2 D/(D^2 + omega^2)  L^alpha_nm conj(L^beta_nm)

with D = e_m - e_n, the pair amplitudes L^alpha_nm = u_n^H T^alpha u_m, u_n the
supercell Bloch vectors u[(R, i)] = c_in(k) exp(2 pi i k.R)/sqrt(Nk), and T the
supercell LRI tensor.  The iomega form is the exact Fourier transform of the tau
form, 2 int_0^inf cos(omega tau) exp(-D tau) dtau = 2D/(D^2+omega^2), so it also
pins the tau -> iomega cosine transform.  Cost grows as N^4: small inputs only.
"""
from __future__ import annotations

import numpy as np

from .chi0 import supercell_lri_tensor


def bloch_vectors(inp):
    """Supercell columns u_n for all k, split into occupied and unoccupied sets."""
    nk, nb = inp.eps.shape
    ph = np.exp(2j * np.pi * (inp.Rvec @ inp.kfrac.T)) / np.sqrt(nk)   # (nR, nk)
    occ, un, eo, eu = [], [], [], []
    for k in range(nk):
        u = (ph[:, k][:, None, None] * inp.wfc[k][None]).reshape(inp.nR * nb, nb)
        occ.append(u[:, :inp.nocc])
        un.append(u[:, inp.nocc:])
        eo.append(inp.eps[k, :inp.nocc])
        eu.append(inp.eps[k, inp.nocc:])
    return np.hstack(occ), np.hstack(un), np.concatenate(eo), np.concatenate(eu)


def pair_amplitudes(inp):
    T = supercell_lri_tensor(inp)
    Uo, Uu, eo, eu = bloch_vectors(inp)
    Lam = np.einsum("pn,apq,qm->anm", Uo.conj(), T, Uu, optimize=True)
    D = eu[None, :] - eo[:, None]
    return Lam, D


def _assemble(inp, Lam, weight):
    """-s sum_nm weight_nm L^a_nm conj(L^b_nm), rows alpha in cell 0."""
    na, nR = inp.nauxtot, inp.nR
    A = Lam.reshape(Lam.shape[0], -1)
    chi = -inp.spin_factor * ((A[:na] * weight.reshape(-1)[None, :]) @ A.conj().T)
    return chi.reshape(na, nR, na).transpose(1, 0, 2)


def chi0_aw_tau(inp, taus, amplitudes=None):
    """[len(taus), nR, naux, naux] complex; imaginary part vanishes to rounding."""
    Lam, D = amplitudes or pair_amplitudes(inp)
    return np.array([_assemble(inp, Lam, np.exp(-D * t)) for t in taus])


def chi0_aw_omega(inp, omegas, amplitudes=None):
    Lam, D = amplitudes or pair_amplitudes(inp)
    return np.array([_assemble(inp, Lam, 2.0 * D / (D ** 2 + w ** 2)) for w in omegas])


# ----------------------------------------------------------------------------
# Bloch-resolved form at one q: spectral radius of chi(q, i omega) v(q)
# ----------------------------------------------------------------------------
#
# The supercell pair amplitudes above, L^{(Ra, mu)}_nm = u_n^H T^{(Ra, mu)} u_m, depend on the
# cell Ra of the ABF only through exp(2 pi i (k_m - k_n).Ra) / Nk.  Summing chi over R with the
# phases of the R -> q transform keeps the pairs with k_m = k_n + q:
#
#   chi_{mu nu}(q, i omega) = -(s/Nk) sum_k sum_{n occ at k, m un at k+q}
#                                 2 D/(D^2 + omega^2) Lam^mu_nm conj(Lam^nu_nm),
#   Lam^mu_nm = sum_{blocks (U, K, R1), mu on U} sum_{i in U, l in K} C^mu_{il}(R1)
#               [ conj(c_in(k)) c_lm(k+q) e^{2 pi i (k+q).R1} + conj(c_ln(k)) e^{-2 pi i k.R1} c_im(k+q) ],
#
# (the two terms are the two sums of Eq. (eq:LRI)).  chi(q) x is applied without forming Lam:
# y = Lam^H x = c_occ(k)^T S conj(c_un(k+q)) with S built from sum_nu x_nu C^nu, and
# chi x = sum_nm Lam^mu_nm w_nm y_nm through Q = conj(c_occ(k)) (w y) c_un(k+q)^T.

def _kindex(frac, mesh):
    n = np.mod(np.rint(np.asarray(frac) * np.asarray(mesh)).astype(np.int64), np.asarray(mesh))
    return int((n[0] * mesh[1] + n[1]) * mesh[2] + n[2])


def _bloch_c(inp, kf):
    """A_U(k)[mu, i, l'] = sum over blocks (U, K, R1) of C^mu_{il}(R1) e^{2 pi i k.R1}, l' = (K, l)."""
    A = [np.zeros((inp.naux[U], inp.nao[U], inp.nb), dtype=np.complex128) for U in range(inp.natoms)]
    R = np.asarray(inp.blocks.R, dtype=np.float64)
    ph = np.exp(2j * np.pi * (R @ np.asarray(kf)))
    for b in range(len(inp.blocks.I)):
        U, K = int(inp.blocks.I[b]), int(inp.blocks.K[b])
        k0 = inp.ao_off[K]
        A[U][:, :, k0:k0 + inp.nao[K]] += ph[b] * inp.blocks.block(b, inp.naux, inp.nao)
    return A


def bloch_c_all(inp):
    """Per atom U, A_U(k) of every k of the mesh stacked and flattened: [nk, a_U, n_U nb]."""
    nk = len(inp.kfrac)
    out = [np.zeros((nk, inp.naux[U], inp.nao[U] * inp.nb), dtype=np.complex128) for U in range(inp.natoms)]
    for k in range(nk):
        A = _bloch_c(inp, inp.kfrac[k])
        for U in range(inp.natoms):
            out[U][k] = A[U].reshape(inp.naux[U], -1)
    return out


class BlochChi:
    """x -> chi(q, i omega) x for one q index and one frequency (host FP64, Bloch form), all k
    at once.  Ak: bloch_c_all(inp) (shared between q points)."""

    def __init__(self, inp, iq, omega, Ak=None):
        mesh = inp.cell.mesh
        self.inp, self.omega = inp, float(omega)
        nk = len(inp.kfrac)
        self.kq = np.array([_kindex(inp.kfrac[k] + inp.kfrac[iq], mesh) for k in range(nk)])
        self.kqinv = np.argsort(self.kq)                      # k + q -> k
        self.Ak = Ak if Ak is not None else bloch_c_all(inp)
        no = inp.nocc
        self.co = np.stack([inp.wfc[k][:, :no] for k in range(nk)])            # [nk, nb, nocc]
        self.cu = np.stack([inp.wfc[self.kq[k]][:, no:] for k in range(nk)])   # [nk, nb, nun] at k + q
        D = np.stack([inp.eps[self.kq[k]][no:][None, :] - inp.eps[k][:no][:, None] for k in range(nk)])
        self.w = 2.0 * D / (D ** 2 + self.omega ** 2)
        self.n = inp.nauxtot

    def __call__(self, x):
        inp = self.inp
        nk, nb = self.co.shape[0], inp.nb
        S = np.zeros((nk, nb, nb), dtype=np.complex128)
        for U in range(inp.natoms):
            xs = x[inp.aux_off[U]:inp.aux_off[U] + inp.naux[U]]
            rows = slice(inp.ao_off[U], inp.ao_off[U] + inp.nao[U])
            t1 = (xs.conj() @ self.Ak[U]).conj().reshape(nk, inp.nao[U], nb)   # sum_mu x_mu conj(A_U(k'))
            S[:, rows, :] += t1[self.kq]                                   # ... at k' = k + q
            S[:, :, rows] += np.swapaxes((xs @ self.Ak[U]).reshape(nk, inp.nao[U], nb), 1, 2)
        y = np.swapaxes(self.co, 1, 2) @ S @ self.cu.conj()                # [nk, nocc, nun]
        Q = self.co.conj() @ (y * self.w) @ np.swapaxes(self.cu, 1, 2)     # [nk, nb, nb]
        z = np.zeros(self.n, dtype=np.complex128)
        for U in range(inp.natoms):
            rows = slice(inp.ao_off[U], inp.ao_off[U] + inp.nao[U])
            q1 = Q[:, rows, :].reshape(nk, -1, 1)[self.kqinv]              # indexed by k' = k + q
            q2 = np.swapaxes(Q[:, :, rows], 1, 2).reshape(nk, -1, 1)
            z[inp.aux_off[U]:inp.aux_off[U] + inp.naux[U]] += (
                (self.Ak[U] @ q1).sum(axis=0)[:, 0] + (self.Ak[U] @ q2.conj()).sum(axis=0)[:, 0].conj())
        return -(inp.spin_factor / nk) * z


def _rho_one_q(inp, vq, iq, omega, A, tol):
    from scipy.sparse.linalg import LinearOperator, eigsh
    op = BlochChi(inp, iq, omega, A)
    L = np.linalg.cholesky(vq[iq])
    n = inp.nauxtot
    M = LinearOperator((n, n), matvec=lambda x: -(L.conj().T @ op(L @ x)), dtype=np.complex128)
    return float(eigsh(M, k=1, which="LA", tol=tol, ncv=min(n - 1, 16), v0=np.ones(n, dtype=np.complex128),
                       return_eigenvectors=False)[0])


def spectral_radius_chi_v(inp, vq=None, qs=None, omega=None, tol=1e-5, workers=1):
    """max over q of rho(chi(q, i omega) v(q)) = the largest |eigenvalue| of the Hermitian
    negative semidefinite L^H chi(q) L, v(q) = L L^H (Lanczos, relative tolerance tol); omega
    defaults to the smallest grid frequency, where chi(i omega) is largest (every term
    2D/(D^2+omega^2) decreases).  q points are spread over `workers` forked processes.
    Returns (rho, q index of the maximum)."""
    vq = inp.vq if vq is None else vq
    omega = float(np.min(inp.omega)) if omega is None else float(omega)
    nk = len(inp.kfrac)
    A = bloch_c_all(inp)
    qs = list(range(nk)) if qs is None else list(qs)
    if workers > 1 and len(qs) > 1:
        import concurrent.futures as cf
        import multiprocessing as mp
        global _FORK_STATE
        _FORK_STATE = (inp, vq, omega, A, tol)
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
            rhos = list(ex.map(_rho_forked, qs))
    else:
        rhos = [_rho_one_q(inp, vq, iq, omega, A, tol) for iq in qs]
    i = int(np.argmax(rhos))
    return rhos[i], qs[i]


_FORK_STATE = None


def _rho_forked(iq):
    from threadpoolctl import threadpool_limits
    inp, vq, omega, A, tol = _FORK_STATE
    with threadpool_limits(1):
        return _rho_one_q(inp, vq, iq, omega, A, tol)
