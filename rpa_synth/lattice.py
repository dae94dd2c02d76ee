"""Neighbour enumeration and BvK bookkeeping for the synthetic cells.

The neighbour set of atom I is every periodic image K(R1) with
|tau_K + R1 - tau_I| < rcut (strict, FP64), the atom itself included.  These
sets are the (I, K, R1) keys of the LRI triple-coefficient blocks and of the
hopping blocks (the neighbourhood N[U] of Algorithm 1's caption).
"""
from __future__ import annotations

import itertools

import numpy as np


def plane_spacings(lattice: np.ndarray) -> np.ndarray:
    """Distance between adjacent lattice planes along each reciprocal direction."""
    b = np.linalg.inv(lattice).T      # rows b_i with a_i . b_j = delta_ij
    return 1.0 / np.linalg.norm(b, axis=1)


def neighbour_pairs(lattice, frac, rcut):
    """All ordered (I, K, R1) with d(I, K+R1) < rcut, sorted lexicographically.

    Returns (I, K, R (n,3) int, d (n,) float, margin) where margin is the smallest
    |d - rcut| over all candidate pairs inside the search box (ties are reported,
    never resolved silently)."""
    cart = frac @ lattice
    nat = len(frac)
    sp = plane_spacings(lattice)
    nmax = [int(np.ceil(rcut / s)) + 1 for s in sp]
    rng = [range(-m, m + 1) for m in nmax]
    Rs = np.array(list(itertools.product(*rng)), dtype=np.int64)
    shifts = Rs @ lattice
    out_I, out_K, out_R, out_d = [], [], [], []
    margin = np.inf
    for I in range(nat):
        for K in range(nat):
            # (tau_K - tau_I) + R: negating the pair negates every rounding exactly, so
            # d(I, K, R) == d(K, I, -R) bit for bit and the list stays symmetric at ties
            d = np.linalg.norm((cart[K] - cart[I]) + shifts, axis=1)
            margin = min(margin, float(np.min(np.abs(d - rcut))))
            sel = np.nonzero(d < rcut)[0]
            for s in sel:
                out_I.append(I)
                out_K.append(K)
                out_R.append(Rs[s])
                out_d.append(d[s])
    I = np.array(out_I, dtype=np.int64)
    K = np.array(out_K, dtype=np.int64)
    R = np.array(out_R, dtype=np.int64).reshape(-1, 3)
    d = np.array(out_d)
    order = np.lexsort((R[:, 2], R[:, 1], R[:, 0], K, I))
    return I[order], K[order], R[order], d[order], margin


def bvk_vectors(mesh) -> np.ndarray:
    """Integer triples n in [0,N1)x[0,N2)x[0,N3), flattened index n1*N2*N3 + n2*N3 + n3."""
    return np.array(list(itertools.product(*[range(m) for m in mesh])), dtype=np.int64)


def fold_index(R, mesh) -> np.ndarray:
    """Flattened BvK index of (unfolded) integer lattice vectors R (..., 3)."""
    R = np.asarray(R, dtype=np.int64)
    m = np.asarray(mesh, dtype=np.int64)
    f = np.mod(R, m)
    return (f[..., 0] * m[1] + f[..., 1]) * m[2] + f[..., 2]


def kmesh(mesh) -> np.ndarray:
    """Gamma-centred k-points in fractional reciprocal coordinates, same ordering as bvk_vectors."""
    n = bvk_vectors(mesh)
    return n / np.asarray(mesh, dtype=np.float64)


def offsets(sizes) -> np.ndarray:
    """Exclusive prefix sum: start of each atom's block along a concatenated axis."""
    sizes = np.asarray(sizes, dtype=np.int64)
    return np.concatenate([[0], np.cumsum(sizes)[:-1]])
