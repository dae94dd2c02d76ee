"""FP64 CPU oracle for the real-space imaginary-time response function.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the GPU library or its binding.

Conventions (the paper's Sec. 2, Eq. (green_mat) and the chi0 formulas, with
the factors of i taken out):  for tau > 0 the paper's G(R, i tau) equals
i G^un(R, tau) and G(R, -i tau) equals -i G^occ(R, tau), both real; its
chi0(R, i tau) equals i chi(R, tau) with chi real and
    chi(r, r', tau) = -s G^un(r, r', tau) G^occ(r', r, tau),   s = 2 (spin).

Three independent evaluations of chi_{mu nu}(R, tau):

* chi0_supercell: the plain definition.  In the BvK supercell every product of
  two NAOs is expanded with the LRI formula Eq. (eq:LRI) (both sums, so on-site
  blocks count twice), which gives a symmetric tensor T^alpha_{pq}; then
  chi_{alpha beta} = -s Tr[T^alpha G^un T^beta G^occ].
* chi0_alg1: Algorithm 1 of the paper (intermediates X, N, M, Z, O, then
  chi += C O), with N evaluated once per (V, K, R1-R) since it depends on
  nothing else.
* chi0_aw_tau / chi0_aw_omega (module oracle.aw): sum over occupied/unoccupied
  Bloch states.

parity pins: supercell == Alg. 1 == sum-over-states (tests/test_oracle_chi0.py).
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------------------
# neighbour bookkeeping read from the LRI block list
# ----------------------------------------------------------------------------

def fold(R, mesh):
    R = np.asarray(R, dtype=np.int64)
    m = np.asarray(mesh, dtype=np.int64)
    f = np.mod(R, m)
    return (f[..., 0] * m[1] + f[..., 1]) * m[2] + f[..., 2]


def bvk_sub(a, b, mesh):
    """Flattened BvK index of (R_a - R_b) for flattened indices a, b."""
    m = np.asarray(mesh, dtype=np.int64)
    def unflat(x):
        x = np.asarray(x, dtype=np.int64)
        return np.stack([x // (m[1] * m[2]), (x // m[2]) % m[1], x % m[2]], axis=-1)
    return fold(unflat(a) - unflat(b), mesh)


def neighbours(inp, U):
    """Block indices b of the LRI list with first atom U: the set N[U] of K(R1)."""
    return np.nonzero(inp.blocks.I == U)[0]


def cblock(inp, b):
    return inp.blocks.block(b, inp.naux, inp.nao)


# ----------------------------------------------------------------------------
# plain definition in the BvK supercell
# ----------------------------------------------------------------------------

def supercell_lri_tensor(inp):
    """T[alpha, p, q] over the BvK supercell: alpha = (R_a, mu), p = (R_p, i).

    The product phi_p phi_q is expanded with both sums of Eq. (eq:LRI); images that
    fold onto the same supercell function add up."""
    nR, nb, na = inp.nR, inp.nb, inp.nauxtot
    M = nR * nb
    T = np.zeros((nR * na, M, M))
    mesh = inp.cell.mesh
    for b in range(len(inp.blocks.I)):
        U, K = inp.blocks.I[b], inp.blocks.K[b]
        C = cblock(inp, b)                           # [mu][i][k]
        r1 = fold(inp.blocks.R[b], mesh)
        a0, i0, k0 = inp.aux_off[U], inp.ao_off[U], inp.ao_off[K]
        nmu, ni, nk = C.shape
        for Ra in range(nR):
            Rk = int(_add(Ra, r1, mesh))                 # cell of K: Ra + R1
            rows = Ra * nb + i0 + np.arange(ni)
            cols = Rk * nb + k0 + np.arange(nk)
            al = Ra * na + a0 + np.arange(nmu)
            # first sum: mu on the atom of i (the product phi_i(U, Ra) phi_k(K, Ra+R1))
            T[np.ix_(al, rows, cols)] += C
            # second sum of the same expansion seen from the other order of the pair
            T[np.ix_(al, cols, rows)] += C.transpose(0, 2, 1)
    return T


def _add(a, r, mesh):
    m = np.asarray(mesh, dtype=np.int64)
    A = np.array([a // (m[1] * m[2]), (a // m[2]) % m[1], a % m[2]])
    Rv = np.array([r // (m[1] * m[2]), (r // m[2]) % m[1], r % m[2]])
    return fold(A + Rv, mesh)


def supercell_green(G, inp):
    """Supercell matrix script-G[(Ra,i),(Rb,j)] = G_ij(Rb - Ra) for one tau."""
    nR, nb = inp.nR, inp.nb
    S = np.empty((nR * nb, nR * nb))
    for Ra in range(nR):
        for Rb in range(nR):
            S[Ra * nb:(Ra + 1) * nb, Rb * nb:(Rb + 1) * nb] = G[int(bvk_sub(Rb, Ra, inp.cell.mesh))]
    return S


def chi0_supercell(inp, taus=None):
    """chi[t, R, mu, nu] = -s Tr[T^(0,mu) G^un T^(R,nu) G^occ]  (plain definition)."""
    taus = range(inp.ntau) if taus is None else taus
    T = supercell_lri_tensor(inp)
    nR, na = inp.nR, inp.nauxtot
    out = []
    for t in taus:
        Gu = supercell_green(inp.Gun[t], inp)
        Go = supercell_green(inp.Gocc[t], inp)
        Xa = np.matmul(T[:na], Gu)                  # T^alpha G^un, alpha in cell 0
        Yb = np.matmul(T, Go)                       # T^beta G^occ, all beta
        # Tr[A B] = sum_pr A_pr B_rp
        chi = -inp.spin_factor * (Xa.reshape(na, -1) @ np.swapaxes(Yb, 1, 2).reshape(nR * na, -1).T)
        out.append(chi.reshape(na, nR, na).transpose(1, 0, 2))
    return np.array(out)


# ----------------------------------------------------------------------------
# Algorithm 1
# ----------------------------------------------------------------------------

class Alg1:
    """Algorithm 1 on the real-valued Green's functions.

    For one (tau, R) and atom pair <U(0), V(R)>:
      X^{s,nu}_{ij}   = sum_{L(R2) in N[V(R)]} sum_l C^nu_{jl}(R2-R) G^s_{il}(R2)
      N^{s,nu}_{jk}   = sum_{L(R2) in N[V(R)]} sum_l C^nu_{jl}(R2-R) G^s_{lk}(R1-R2)
      M, Z and O      : O^nu_ik = sum_j [ G^un_ij(R) N^occ_jk + G^occ_ij(R) N^un_jk
                                          + G^occ_jk(R1-R) X^un_ij + G^un_jk(R1-R) X^occ_ij ]
      chi_{mu nu}    += -s sum_{ik} C^mu_{ik}(R1) O^nu_{ik}       for K(R1) in N[U]
    The loop over K(R1) is carried out on the neighbours concatenated along k.
    N depends only on (V, K, R1 - R); it is evaluated once per V for all K and
    all BvK differences (this changes no arithmetic, only how often it is done).
    """

    def __init__(self, inp):
        self.inp = inp
        self.mesh = inp.cell.mesh
        self.nbrs = [neighbours(inp, U) for U in range(inp.natoms)]
        self.fR = fold(inp.blocks.R, self.mesh)
        self._Ncache = {}

    # concatenated coefficients of atom U: Cbar[mu, i, (K R1 k)]
    def cbar(self, U):
        return np.concatenate([cblock(self.inp, b) for b in self.nbrs[U]], axis=2)

    def _ghat_rows(self, G, V, shift):
        """Rows (L(R2) l) of G_{l, :}(shift - R2) stacked over L(R2) in N[V]: [(L R2 l), all k]."""
        inp = self.inp
        parts = []
        for b in self.nbrs[V]:
            L = inp.blocks.K[b]
            r = int(bvk_sub(shift, self.fR[b], self.mesh))
            parts.append(G[r, inp.ao_off[L]:inp.ao_off[L] + inp.nao[L], :])
        return np.concatenate(parts, axis=0)

    def N_all(self, t, V):
        """N^{s,nu}_{j,k}(V, dR) for all dR in the BvK set and all k of the cell:
        array [s, dR, nu, j, k_all]."""
        key = (t, V)
        if key in self._Ncache:
            return self._Ncache[key]
        inp = self.inp
        Cb = self.cbar(V)                                       # [nu, j, (L R2 l)]
        av, nv, sv = Cb.shape
        out = np.empty((2, inp.nR, av, nv, inp.nb))
        for s, G in enumerate((inp.Gocc[t], inp.Gun[t])):
            for dR in range(inp.nR):
                Gh = self._ghat_rows(G, V, dR)                  # [(L R2 l), k_all]
                out[s, dR] = (Cb.reshape(av * nv, sv) @ Gh).reshape(av, nv, inp.nb)
        self._Ncache = {key: out}                               # keep one (t, V)
        return out

    def X(self, t, U, V, R):
        """X^{s,nu}_{ij}(U, V, R) = sum_{L(R2)} C^nu_{jl}(R2-R) G^s_{il}(R2): [s, i, nu, j]."""
        inp = self.inp
        Cb = self.cbar(V)                                       # [nu, j, (L dL l)], dL = R2 - R
        out = []
        for G in (inp.Gocc[t], inp.Gun[t]):
            cols = []
            for b in self.nbrs[V]:
                L = inp.blocks.K[b]
                r2 = int(_add(R, self.fR[b], self.mesh))        # R2 = R + dL
                cols.append(G[r2, inp.ao_off[U]:inp.ao_off[U] + inp.nao[U],
                              inp.ao_off[L]:inp.ao_off[L] + inp.nao[L]])
            Gc = np.concatenate(cols, axis=1)                    # [i, (L dL l)]
            out.append(np.einsum("il,vjl->ivj", Gc, Cb, optimize=True))
        return np.array(out)

    def block(self, t, U, V, R, chunk=24):
        """chi_{UV}(R, tau_t): [naux_U, naux_V].  The loop over K(R1) in N[U] runs in
        chunks of neighbours concatenated along k."""
        inp = self.inp
        iU = slice(inp.ao_off[U], inp.ao_off[U] + inp.nao[U])
        iV = slice(inp.ao_off[V], inp.ao_off[V] + inp.nao[V])
        Go, Gu = inp.Gocc[t], inp.Gun[t]
        X = self.X(t, U, V, R)                                   # [s, i, nu, j]
        Nall = self.N_all(t, V)                                  # [s, dR, nu, j, k_all]
        GuR, GoR = Gu[R, iU, iV], Go[R, iU, iV]
        chi = np.zeros((inp.naux[U], inp.naux[V]))
        nb = self.nbrs[U]
        for c0 in range(0, len(nb), chunk):
            Cs, Ns, Gvk_o, Gvk_u = [], [], [], []
            for b in nb[c0:c0 + chunk]:
                K = inp.blocks.K[b]
                iK = slice(inp.ao_off[K], inp.ao_off[K] + inp.nao[K])
                d = int(bvk_sub(self.fR[b], R, self.mesh))       # R1 - R
                Cs.append(cblock(inp, b))                        # C^mu_{ik}(R1)
                Ns.append(Nall[:, d][..., iK])                   # N^{s,nu}_{jk}(V, K, R1 - R)
                Gvk_o.append(Go[d, iV, iK])                      # G^occ_{jk}(R1 - R)
                Gvk_u.append(Gu[d, iV, iK])
            Cb = np.concatenate(Cs, axis=2)                      # [mu, i, (K R1 k)]
            N = np.concatenate(Ns, axis=3)                       # [s, nu, j, (K R1 k)]
            Gvo = np.concatenate(Gvk_o, axis=1)                  # [j, (K R1 k)]
            Gvu = np.concatenate(Gvk_u, axis=1)
            M1 = np.einsum("ij,vjk->ivk", GuR, N[0], optimize=True)    # G^un(R) N^occ
            M2 = np.einsum("ij,vjk->ivk", GoR, N[1], optimize=True)    # G^occ(R) N^un
            Z1 = np.einsum("jk,ivj->ivk", Gvo, X[1], optimize=True)    # G^occ(R1-R) X^un
            Z2 = np.einsum("jk,ivj->ivk", Gvu, X[0], optimize=True)    # G^un(R1-R) X^occ
            O = self.combine(M1, M2, Z1, Z2)                           # [i, nu, (K R1 k)]
            chi += np.einsum("mik,ivk->mv", Cb, O, optimize=True)
        return -inp.spin_factor * chi

    @staticmethod
    def combine(M1, M2, Z1, Z2):
        """O = M(i tau) + M*(-i tau) + Z(i tau) + Z*(-i tau) in the real convention."""
        return M1 + M2 + Z1 + Z2

    def full(self, taus=None):
        """chi[t, R, mu, nu] over all blocks (every ordered U, V and every R)."""
        inp = self.inp
        taus = range(inp.ntau) if taus is None else taus
        out = np.zeros((len(list(taus)), inp.nR, inp.nauxtot, inp.nauxtot))
        for it, t in enumerate(taus):
            for V in range(inp.natoms):
                self.N_all(t, V)
                for U in range(inp.natoms):
                    for R in range(inp.nR):
                        mu = slice(inp.aux_off[U], inp.aux_off[U] + inp.naux[U])
                        nu = slice(inp.aux_off[V], inp.aux_off[V] + inp.naux[V])
                        out[it, R, mu, nu] = self.block(t, U, V, R)
        return out


def chi0_alg1(inp, taus=None):
    return Alg1(inp).full(taus)


def chi0_alg1_block(inp, t, U, V, R, alg=None):
    alg = alg or Alg1(inp)
    return alg.block(t, U, V, R)


def chi0_bruteforce(inp, t):
    """Literal four-term matrix formula (Sec. 2, the chi0_{mu,nu}(R, i tau) equation) for one tau,
    with explicit sums over K(R1), L(R2) pairs; micro inputs only."""
    nR, na = inp.nR, inp.nauxtot
    mesh = inp.cell.mesh
    Go, Gu = inp.Gocc[t], inp.Gun[t]
    fR = fold(inp.blocks.R, mesh)
    out = np.zeros((nR, na, na))
    for R in range(nR):
        for bu in range(len(inp.blocks.I)):
            U, K = inp.blocks.I[bu], inp.blocks.K[bu]
            R1 = fR[bu]
            Cu = cblock(inp, bu)                                 # [mu, i, k]
            iU = slice(inp.ao_off[U], inp.ao_off[U] + inp.nao[U])
            iK = slice(inp.ao_off[K], inp.ao_off[K] + inp.nao[K])
            for bv in range(len(inp.blocks.I)):
                V, L = inp.blocks.I[bv], inp.blocks.K[bv]
                Cv = cblock(inp, bv)                             # [nu, j, l]
                iV = slice(inp.ao_off[V], inp.ao_off[V] + inp.nao[V])
                iL = slice(inp.ao_off[L], inp.ao_off[L] + inp.nao[L])
                R2 = int(_add(R, fR[bv], mesh))                  # cell of L
                r12 = int(bvk_sub(R1, R2, mesh))
                r1r = int(bvk_sub(R1, R, mesh))
                # four pairings of Green's functions
                t1 = np.einsum("ij,lk->ijkl", Gu[R, iU, iV], Go[r12, iL, iK])
                t2 = np.einsum("ij,lk->ijkl", Go[R, iU, iV], Gu[r12, iL, iK])
                t3 = np.einsum("jk,il->ijkl", Go[r1r, iV, iK], Gu[R2, iU, iL])
                t4 = np.einsum("jk,il->ijkl", Gu[r1r, iV, iK], Go[R2, iU, iL])
                W = t1 + t2 + t3 + t4
                mu = slice(inp.aux_off[U], inp.aux_off[U] + inp.naux[U])
                nu = slice(inp.aux_off[V], inp.aux_off[V] + inp.naux[V])
                out[R, mu, nu] += -inp.spin_factor * np.einsum("mik,njl,ijkl->mn", Cu, Cv, W, optimize=True)
    return out
