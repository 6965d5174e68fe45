"""Face-centred cubic lattice in the twisted Cartesian coordinates (2.1 notes
that the same coordinates carry FCC, whose neighbours are closer to spherical
symmetry; the appendix on FCC gives figures only).  Layers are the close-packed
rows of the HCP case, stacked ABC instead of ABAB.

Pins that do not re-derive the oracle's stencil:
- geometry: the 12 neighbours of every voxel are exactly the voxels at
  minimum-image distance 2r, nothing is closer, in a closed box the in-box
  neighbours are the voxels at plain distance 2r;
- hop vectors are the real displacements, |hop| = 2r, and the 12 hops sum to
  zero with an isotropic second moment;
- stacking: layer k and k + 3 coincide in projection, k, k + 1, k + 2 are
  pairwise disjoint (ABC), packing fraction pi / (3 sqrt 2);
- the coordination sequence of the fcc net, 12, 42, 92 (it differs from the
  hcp net's 12, 44, 96, so an HCP stencil fails it), and the fcc lattice's
  numbers of closed n-step walks, n <= 8, from every layer phase;
- the 16 stage colours split the voxels evenly and every class is an
  independent set at graph distance <= 2 (what lets a stage run in any order);
- the walk: lone walkers have MSD 6 D t; runs in reversed intra-stage order
  are identical, with and without walls."""
import math
from collections import deque

import numpy as np
import pytest

import oracle
from psc_inputs import workload

RV = 1.0
F = oracle.FCC


def positions(dims):
    nv = dims[0] * dims[1] * dims[2]
    return np.array([oracle.position_l(dims, v, RV, F) for v in range(nv)])


def box(dims):
    return np.array([2 * RV * dims[0], math.sqrt(3) * RV * dims[1],
                     2 * math.sqrt(2 / 3) * RV * dims[2]])


def min_image(d, L):
    return d - L * np.round(d / L)


@pytest.mark.parametrize("dims", [(4, 4, 12), (8, 8, 12), (4, 8, 24), (12, 4, 12)])
def test_neighbours_are_exactly_the_touching_voxels(dims):
    P = positions(dims)
    L = box(dims)
    nv = len(P)
    for v in range(nv):
        d = min_image(P - P[v], L)
        dist = np.sqrt((d ** 2).sum(axis=1))
        touching = set(np.nonzero(np.abs(dist - 2 * RV) < 1e-9)[0].tolist())
        assert np.all(dist[np.arange(nv) != v] > 2 * RV - 1e-9)
        nb = [oracle.neighbour_l(dims, v, n, F) for n in range(12)]
        assert len(set(nb)) == 12
        assert set(nb) == touching


@pytest.mark.parametrize("dims", [(4, 4, 12), (8, 4, 12)])
def test_in_box_neighbours_of_a_closed_box(dims):
    P = positions(dims)
    for v in range(len(P)):
        d = np.sqrt(((P - P[v]) ** 2).sum(axis=1))
        want = set(np.nonzero(np.abs(d - 2 * RV) < 1e-9)[0].tolist())
        got = [oracle.neighbour_l(dims, v, n, F, oracle.REFLECT) for n in range(12)]
        inside = [t for t in got if t != oracle.OUTSIDE]
        assert len(set(inside)) == len(inside)
        assert set(inside) == want
        for n, t in enumerate(got):
            if t != oracle.OUTSIDE:
                assert t == oracle.neighbour_l(dims, v, n, F)


def test_hop_vectors_are_real_displacements():
    dims = (8, 4, 12)
    P = positions(dims)
    L = box(dims)
    units = np.array([RV, RV / math.sqrt(3), 2 * math.sqrt(2 / 3) * RV])
    for v in range(len(P)):
        tot = np.zeros(3)
        M = np.zeros((3, 3))
        for n in range(12):
            t = oracle.neighbour_l(dims, v, n, F)
            h = np.array(oracle.hop_vector_l(dims, v, n, F))
            real = min_image(P[t] - P[v], L)
            assert np.allclose(real, h * units, atol=1e-9)
            assert 3 * h[0] ** 2 + h[1] ** 2 + 8 * h[2] ** 2 == 12
            tot += h
            M += np.outer(real, real)
        assert np.all(tot == 0)
        # 12 hops of length 2r: second moment (12 * 4 r^2 / 3) I
        assert np.allclose(M, 16 * RV * RV * np.eye(3), atol=1e-9)


def test_abc_stacking_and_density():
    dims = (4, 4, 12)
    P = positions(dims)
    L = box(dims)

    def layer(k):
        sel = [v for v in range(len(P)) if v // 16 == k]
        return {(round(P[v][0] % L[0], 9), round(P[v][1] % L[1], 9)) for v in sel}
    for k in range(9):
        assert layer(k) == layer(k + 3)
        assert layer(k).isdisjoint(layer(k + 1))
        assert layer(k).isdisjoint(layer(k + 2))
    vol = L.prod() / len(P)
    frac = (4 / 3) * math.pi * RV ** 3 / vol
    assert abs(frac - math.pi / (3 * math.sqrt(2))) < 1e-12


def shells(dims, lattice, depth=3):
    dist = {0: 0}
    q = deque([0])
    while q:
        v = q.popleft()
        if dist[v] == depth:
            continue
        for n in range(12):
            t = oracle.neighbour_l(dims, v, n, lattice)
            if t not in dist:
                dist[t] = dist[v] + 1
                q.append(t)
    return [sum(1 for d in dist.values() if d == s) for s in range(1, depth + 1)]


def test_coordination_sequence_of_the_fcc_net():
    assert shells((16, 16, 24), F) == [12, 42, 92]
    assert shells((16, 16, 24), oracle.HCP) == [12, 44, 96]


# closed n-step walks on the fcc lattice, n = 0..8 (a classical lattice
# count, Domb 1960; OEIS A002899)
FCC_CLOSED_WALKS = [1, 0, 12, 48, 540, 4320, 42240, 403200, 4038300]


def test_closed_walk_counts_of_the_fcc_lattice():
    """Counted exactly from the oracle's stencil with integer powers of the
    adjacency matrix, on a box too large for a walk of 8 steps to wrap, from
    voxels in each of the three layer phases (FCC is a Bravais lattice: every
    site sees the same counts)."""
    import scipy.sparse as sp
    dims = (24, 24, 24)
    nb = oracle.neighbour_table_l(dims, F)
    nv = nb.shape[0]
    A = sp.csr_matrix((np.ones(nv * 12, np.int64), (nb.ravel(), np.repeat(np.arange(nv), 12))),
                      shape=(nv, nv))
    for start in (0, 24 * 24 * 1 + 5 * 24 + 7, 24 * 24 * 2 + 11 * 24 + 3):
        p = np.zeros(nv, np.int64)
        p[start] = 1
        counts = []
        for _ in FCC_CLOSED_WALKS:
            counts.append(int(p[start]))
            p = A @ p
        assert counts == FCC_CLOSED_WALKS, (start, counts)


@pytest.mark.parametrize("dims", [(8, 8, 12), (16, 8, 24), (8, 16, 12), (24, 8, 36)])
def test_colour_classes_are_three_hops_apart(dims):
    nv = dims[0] * dims[1] * dims[2]
    assert oracle.n_colours(F) == 16
    col = [oracle.colour_l(dims, v, F) for v in range(nv)]
    counts = np.bincount(col, minlength=16)
    assert len(counts) == 16 and np.all(counts == nv // 16)
    for v in range(nv):
        near = set()
        for n in range(12):
            t = oracle.neighbour_l(dims, v, n, F)
            near.add(t)
            for m in range(12):
                near.add(oracle.neighbour_l(dims, t, m, F))
        near.discard(v)
        assert all(col[u] != col[v] for u in near)


def test_lattice_kind_checks_the_stacking_and_colour_periods():
    # k: ABC stacking (3) and bricks (4); i and j: the colouring's period 8
    for dims in ((8, 8, 8), (12, 8, 12), (8, 12, 12), (8, 4, 12)):
        with pytest.raises(ValueError):
            oracle.Oracle(dims, 4.4e-9, 1, lattice=F)
    with pytest.raises(ValueError):
        oracle.Oracle((8, 8, 12), 4.4e-9, 1, lattice=7)
    oracle.Oracle((8, 8, 12), 4.4e-9, 1, lattice=F).close()
    # both lattices take the same 16-stage order of an event
    assert oracle.stage_order_n(3, 9, oracle.n_colours(F)) == oracle.stage_order(3, 9)


def test_msd_lone_walkers_is_6Dt():
    rv, D = 4.4e-9, 1e-12
    ratios = []
    for seed in (1, 2):
        o = oracle.Oracle((64, 64, 48), rv, seed, lattice=F)
        o.add_species(D)
        o.place_uniform(1, 300)
        traj = []
        for _ in range(1500):
            o.run(1, oracle.MODE_C)
            s = o.state(with_occ=False)
            traj.append(np.stack([s["dx"], s["dy"], s["dz"]]).astype(np.float64))
        traj = np.array(traj)
        tau = 2.0 * rv * rv / (3.0 * D)
        lags = np.arange(1, 11)
        msd = []
        for lag in lags:
            d = traj[lag:] - traj[:-lag]
            msd.append((rv ** 2 * (d[:, 0] ** 2 + d[:, 1] ** 2 / 3.0
                                   + 8.0 * d[:, 2] ** 2 / 3.0)).mean())
        t = lags * tau
        ratios.append(float((np.array(msd) * t).sum() / (t * t).sum()) / (6.0 * D))
    assert abs(np.mean(ratios) - 1.0) < 0.02, ratios


def build(w, boundary=oracle.PERIODIC):
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"], boundary=boundary, lattice=F)
    for _, D in w["species"]:
        o.add_species(D)
    for r, p, k in w["reactions"]:
        o.add_reaction(r, p, k)
    for s, c in w["place"]:
        o.place_uniform(s, c)
    return o


@pytest.mark.parametrize("name,boundary", [("small_reactive", oracle.PERIODIC),
                                           ("small_reactive", oracle.REFLECT),
                                           ("multiproduct", oracle.PERIODIC)])
def test_reversed_intra_stage_order_gives_identical_run(name, boundary):
    w = workload(name, dims=(16, 16, 12))
    a, b = build(w, boundary), build(w, boundary)
    a.run(40, oracle.MODE_C)
    b.run(40, oracle.MODE_C_REV)
    sa, sb = a.state(), b.state()
    for key in ("occ", "id", "vox", "species", "dx", "dy", "dz"):
        assert np.array_equal(sa[key], sb[key]), key
    assert sa["fired"].tolist() == sb["fired"].tolist()
    assert sa["hops"] == sb["hops"] and sa["collisions"] == sb["collisions"]
    assert sa["hops"] > 1000 and sum(sa["fired"]) > 0
    # the lattice changes the run
    h = oracle.Oracle(w["dims"], w["rv"], w["seed"], boundary=boundary)
    for _, D in w["species"]:
        h.add_species(D)
    for r, p, k in w["reactions"]:
        h.add_reaction(r, p, k)
    for s, c in w["place"]:
        h.place_uniform(s, c)
    h.run(40, oracle.MODE_C)
    assert not np.array_equal(sa["occ"], h.state()["occ"])


def test_tracked_displacement_is_the_real_displacement_in_a_closed_box():
    dims = (8, 8, 12)
    rv = 4.4e-9
    w = dict(workload("cfg1"), dims=dims, place=[(1, 30)], seed=5)
    o = build(w, oracle.REFLECT)
    s0 = o.state()
    p0 = {i: oracle.position_l(dims, int(v), rv, F) for i, v in zip(s0["id"], s0["vox"])}
    o.run(300, oracle.MODE_C)
    s = o.state()
    assert s["hops"] > 1000
    for i, v, dx, dy, dz in zip(s["id"], s["vox"], s["dx"], s["dy"], s["dz"]):
        real = np.subtract(oracle.position_l(dims, int(v), rv, F), p0[i])
        tracked = np.array([dx * rv, dy * rv / math.sqrt(3.0),
                            dz * 2.0 * math.sqrt(2.0 / 3.0) * rv])
        assert np.allclose(real, tracked, atol=1e-6 * rv), (i, real, tracked)
