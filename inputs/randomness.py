"""Random numbers consumed by the method, drawn here and passed to both sides.

* ``bra_init_gaussians`` -- complex Gaussian tensors from which each side
  builds its generic right-canonical starting guess of the compression step
  (the paper leaves the initial guess unstated; a fixed generic guess per
  (n, chi, seed), identical for every chunk, is the reading used here).
* ``shot_uniforms`` -- the uniforms u in [0, 1) that decide sampled outcomes in
  single-path runs (outcome 0 when u < p_0), one per measurement of a shot.
* ``branch_chi_draw`` -- the per-branch bond cap drawn when a multi-path child
  is created (uneven-chi multi-path workload).

Only numpy's seeded generators are used; no simulation arithmetic lives here.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np


def bond_dims(n: int, chi: int) -> List[int]:
    """Padded bond dimensions chi_b = min(chi, 2^b, 2^(n-b)), b = 0..n; the
    shapes of the Gaussian tensors below."""
    return [min(chi, 2 ** b, 2 ** (n - b)) for b in range(n + 1)]


def bra_init_gaussians(n: int, chi: int, seed: int) -> List[np.ndarray]:
    """Site tensors G_j of shape (chi_j, 2, chi_{j+1}) with independent
    standard complex Gaussian entries (real and imaginary parts N(0, 1/2))."""
    rng = np.random.default_rng([int(seed), int(n), int(chi), 0xB7A])
    d = bond_dims(n, chi)
    out = []
    for j in range(n):
        shp = (d[j], 2, d[j + 1])
        g = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) / np.sqrt(2.0)
        out.append(np.ascontiguousarray(g, dtype=np.complex128))
    return out


def gaussians_for_shapes(shapes: Sequence[Sequence[int]], seed: int, tag: int) -> List[np.ndarray]:
    """Independent standard complex Gaussian tensors (real and imaginary parts
    N(0, 1/2)) of the given shapes, drawn in order from
    default_rng([seed, tag, 0x77E])."""
    rng = np.random.default_rng([int(seed), int(tag), 0x77E])
    out = []
    for shp in shapes:
        shp = tuple(int(x) for x in shp)
        g = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) / np.sqrt(2.0)
        out.append(np.ascontiguousarray(g, dtype=np.complex128))
    return out


def shot_uniforms(seed: int, shot: int, count: int) -> np.ndarray:
    """``count`` uniforms in [0, 1) (53-bit doubles) for one single-path shot."""
    rng = np.random.default_rng([int(seed), int(shot), 0x5A7])
    return rng.random(count)


def branch_chi_draw(seed: int, path: Sequence[int], choices: Sequence[int]) -> int:
    """Bond cap of the multi-path child reached by measurement outcomes
    ``path`` (a tuple of 0/1), drawn uniformly from ``choices``."""
    key = [int(seed), len(path)] + [int(b) for b in path] + [0xC41]
    rng = np.random.default_rng(key)
    return int(choices[int(rng.integers(len(choices)))])
