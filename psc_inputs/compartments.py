"""Compartment maps (one compartment id, 0..255, per voxel in the ABI's
linear order v = i + ni (j + nj k)) and a workload that uses them.

The maps are drawn in index space (i, j, k); they carry no lattice geometry.
A workload with compartments adds two keys to the plain workload dict:
  compartments: the map, a uint8 array of ni nj nk entries
  place_in: [(species id, count, compartment)] placements restricted to a
            compartment, made after `place`, in this order
"""
from __future__ import annotations

import numpy as np

from .workloads import D05, D1, RV


def ijk(dims):
    ni, nj, nk = (int(x) for x in dims)
    k, j, i = np.meshgrid(np.arange(nk), np.arange(nj), np.arange(ni), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def shell_map(dims, radius_frac: float = 0.35, thickness: float = 1.5) -> np.ndarray:
    """An ellipsoid in index space centred in the box with semi-axes
    radius_frac * dims: 2 inside, 1 on a shell about `thickness` voxels
    thick (a membrane), 0 outside."""
    i, j, k = ijk(dims)
    c = [(d - 1) / 2.0 for d in dims]
    R = [radius_frac * d for d in dims]
    e = np.sqrt(((i - c[0]) / R[0]) ** 2 + ((j - c[1]) / R[1]) ** 2 + ((k - c[2]) / R[2]) ** 2)
    inner = 1.0 - thickness / min(R)
    out = np.zeros(len(i), np.uint8)
    out[e < 1.0] = 1
    out[e < inner] = 2
    return out


def sub_box_map(dims, sub) -> np.ndarray:
    """0 on the sub-box [0, sub_i) x [0, sub_j) x [0, sub_k) at the origin,
    1 elsewhere."""
    i, j, k = ijk(dims)
    inside = (i < sub[0]) & (j < sub[1]) & (k < sub[2])
    return np.where(inside, 0, 1).astype(np.uint8)


def layered_map(dims, n: int = 4) -> np.ndarray:
    """n slabs along k, compartment = slab index (every slab's faces border
    another compartment, also across the periodic wrap when n > 1)"""
    i, j, k = ijk(dims)
    return (k * n // int(dims[2])).astype(np.uint8)


def membrane(dims=(24, 24, 24), seed: int = 5, events: int = 60, lattice: str = "hcp",
             boundary=None, radius_frac: float = 0.35) -> dict:
    """A cell-like box: cytosol outside (0), a membrane shell (1), a nucleus
    inside (2).  Species live in each: A, B and C in the cytosol and the
    nucleus, M on the membrane (slower), with collision reactions of one,
    two and four products and first-order reactions of zero to three
    products; every product stays in its reactant's compartment."""
    comp = shell_map(dims, radius_frac)
    n = [int(np.count_nonzero(comp == c)) for c in range(3)]
    w = dict(name="membrane", dims=tuple(dims), rv=RV, seed=seed,
             species=[("A", D1), ("B", D05), ("C", D1), ("M", 0.2 * D1), ("O", 0.0)],
             reactions=[((1, 2), (3,), 1e-18),            # A + B -> C
                        ((3,), (1, 2), 2000.0),           # C -> A + B
                        ((1, 4), (4, 1, 2, 2), 4e-20),    # A + M -> M + A + 2 B
                        ((2,), (), 300.0),                # B -> 0
                        ((4,), (4, 4), 60.0),             # M -> M + M
                        ((4, 4), (4,), 2e-20),            # M + M -> M
                        ((1,), (1, 3, 2), 200.0)],        # A -> A + C + B
             place=[],
             place_in=[(5, n[0] // 20, 0), (1, n[0] // 16, 0), (2, n[0] // 16, 0),
                       (4, max(1, n[1] // 8), 1),
                       (1, max(1, n[2] // 12), 2), (2, max(1, n[2] // 12), 2)],
             compartments=comp, events=events, track_displacement=True)
    if lattice == "fcc":
        w["lattice"] = "fcc"
    if boundary:
        w["boundary"] = boundary
    return w
