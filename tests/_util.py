"""Cached seeded inputs for the tests (no method arithmetic here)."""
from __future__ import annotations

import functools

import numpy as np

from rpa_synth import config, make_inputs
from rpa_synth.configs import micro_cell


@functools.lru_cache(maxsize=None)
def micro(seed=1, natoms=2, nao=(3, 4), naux=(4, 5), mesh=(3, 2, 1), rcut=4.2, edge=3.0, ntau=3):
    return make_inputs(micro_cell(seed, natoms, nao, naux, mesh, rcut, edge, ntau))


@functools.lru_cache(maxsize=None)
def cfg(i, with_coulomb=True):
    return make_inputs(config(i), with_coulomb=with_coulomb)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))
