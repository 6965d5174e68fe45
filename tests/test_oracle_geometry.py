"""Geometry pins of the oracle (HCP lattice in twisted Cartesian coordinates,
paper 2.1 and Fig. 3).

The stencil is checked against Euclidean geometry, not against itself: the 12
neighbours of every voxel must be exactly the voxels at distance 2r (minimum
image), the hop vectors must equal the real displacements, the packing must be
the HCP density and stacking, and the coordination shells must be those of
the hcp net.
"""
import math
from collections import deque

import numpy as np
import pytest

import oracle

RV = 1.0


def positions(dims):
    nv = dims[0] * dims[1] * dims[2]
    return np.array([oracle.position(dims, v, RV) for v in range(nv)])


def box(dims):
    # periodic box edge lengths for the centres x = r(2i+s), y = r/sqrt3 (3j+p),
    # z = 2 sqrt(2/3) r k
    return np.array([2 * RV * dims[0], math.sqrt(3) * RV * dims[1],
                     2 * math.sqrt(2 / 3) * RV * dims[2]])


def min_image(d, L):
    return d - L * np.round(d / L)


@pytest.mark.parametrize("dims", [(4, 4, 4), (8, 8, 8), (4, 8, 12), (12, 8, 4)])
def test_neighbours_are_exactly_the_touching_voxels(dims):
    P = positions(dims)
    L = box(dims)
    nv = len(P)
    for v in range(nv):
        d = min_image(P - P[v], L)
        dist = np.sqrt((d ** 2).sum(axis=1))
        touching = set(np.nonzero(np.abs(dist - 2 * RV) < 1e-9)[0].tolist())
        # nothing closer than touching (exclusive voxels of radius r)
        assert np.all(dist[np.arange(nv) != v] > 2 * RV - 1e-9)
        nb = [oracle.neighbour(dims, v, n) for n in range(12)]
        assert len(set(nb)) == 12
        assert set(nb) == touching


@pytest.mark.parametrize("dims", [(4, 4, 4), (8, 12, 4)])
def test_hop_vectors_are_real_displacements(dims):
    P = positions(dims)
    L = box(dims)
    units = np.array([RV, RV / math.sqrt(3), 2 * math.sqrt(2 / 3) * RV])
    for v in range(len(P)):
        tot = np.zeros(3)
        for n in range(12):
            t = oracle.neighbour(dims, v, n)
            X, Y, Z = oracle.hop_vector(dims, v, n)
            real = min_image(P[t] - P[v], L)
            assert np.allclose(real, np.array([X, Y, Z]) * units, atol=1e-9)
            # exact integer form of |hop|^2 = 4 r^2
            assert 3 * X * X + Y * Y + 8 * Z * Z == 12
            tot += np.array([X, Y, Z])
        assert np.all(tot == 0)  # the 12 hops of one voxel sum to zero


def test_symmetric_adjacency():
    dims = (8, 8, 8)
    for v in range(8 ** 3):
        for n in range(12):
            t = oracle.neighbour(dims, v, n)
            assert v in [oracle.neighbour(dims, t, m) for m in range(12)]


def test_hcp_stacking_and_density():
    dims = (4, 4, 4)
    P = positions(dims)
    L = box(dims)
    # layers k and k+2 coincide in projection, k and k+1 do not (ABAB = HCP)
    def layer(k):
        sel = [v for v in range(64) if v // 16 == k]
        return {(round(P[v][0], 9) % L[0], round(P[v][1], 9) % L[1]) for v in sel}
    assert layer(0) == layer(2) and layer(1) == layer(3)
    assert layer(0).isdisjoint(layer(1))
    # packing fraction of touching spheres of radius r: pi / (3 sqrt 2)
    vol = L.prod() / 64
    frac = (4 / 3) * math.pi * RV ** 3 / vol
    assert abs(frac - 0.74048) < 5e-5


def test_coordination_shells_of_the_hcp_net():
    # number of voxels at graph distance 1, 2, 3: 12, 44, 96 for hcp
    dims = (16, 16, 16)
    dist = {0: 0}
    q = deque([0])
    while q:
        v = q.popleft()
        if dist[v] == 3:
            continue
        for n in range(12):
            t = oracle.neighbour(dims, v, n)
            if t not in dist:
                dist[t] = dist[v] + 1
                q.append(t)
    shells = [sum(1 for d in dist.values() if d == s) for s in (1, 2, 3)]
    assert shells == [12, 44, 96]


@pytest.mark.parametrize("dims", [(4, 4, 4), (8, 8, 8), (12, 8, 16), (16, 12, 8), (4, 8, 4)])
def test_colour_classes_are_three_hops_apart(dims):
    nv = dims[0] * dims[1] * dims[2]
    col = [oracle.colour(dims, v) for v in range(nv)]
    counts = np.bincount(col, minlength=16)
    assert len(counts) == 16 and np.all(counts == nv // 16)
    for v in range(nv):
        near = set()
        for n in range(12):
            t = oracle.neighbour(dims, v, n)
            near.add(t)
            for m in range(12):
                near.add(oracle.neighbour(dims, t, m))
        near.discard(v)
        assert all(col[u] != col[v] for u in near)
