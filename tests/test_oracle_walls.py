"""Boxes closed by walls (the oracle's reflecting boundary).  A move into
another compartment fails like a move into an occupied voxel (section 2.3);
the space beyond each face of a closed box is read as such a compartment.

Pins that do not re-derive the oracle's code:
- geometry: the in-box neighbours of every voxel are exactly the voxels of
  the box at plain (not minimum-image) Euclidean distance 2r;
- no hop crosses a wall: in a closed box a molecule's tracked displacement
  equals the difference of its real positions, exactly, for every molecule;
- the symmetric exclusion process in a closed box has the uniform stationary
  distribution, so long-run occupancy is flat over the voxels;
- coloured stages still commute with walls (reversed order is identical);
- products are never placed beyond a wall: an 11-product reaction in a
  corner, where fewer than 11 neighbours exist, always fails."""
import math

import numpy as np
import pytest

import oracle
from psc_inputs import workload

RV = 4.4e-9
H = 2.0 * math.sqrt(2.0 / 3.0) * RV


def build(w, boundary, state=None):
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"], boundary=boundary)
    for _, D in w["species"]:
        o.add_species(D)
    for r, p, k in w["reactions"]:
        o.add_reaction(r, p, k)
    for s, c in w["place"]:
        o.place_uniform(s, c)
    return o


@pytest.mark.parametrize("dims", [(4, 4, 4), (8, 4, 12), (8, 8, 8)])
def test_in_box_neighbours_are_the_voxels_at_distance_2r(dims):
    nv = int(np.prod(dims))
    pos = np.array([oracle.position(dims, v, RV) for v in range(nv)])
    for v in range(nv):
        d = np.sqrt(((pos - pos[v]) ** 2).sum(axis=1))
        want = set(np.nonzero(np.abs(d - 2 * RV) < 1e-6 * RV)[0].tolist())
        assert not np.any((d > 1e-6 * RV) & (d < 2 * RV * (1 - 1e-6)))
        got = [oracle.neighbour_b(dims, v, n, oracle.REFLECT) for n in range(12)]
        inside = [t for t in got if t != oracle.OUTSIDE]
        assert len(set(inside)) == len(inside)
        assert set(inside) == want, (v, sorted(want), sorted(inside))
        # rows that exist inside agree with the periodic stencil
        for n, t in enumerate(got):
            if t != oracle.OUTSIDE:
                assert t == oracle.neighbour(dims, v, n)


def test_tracked_displacement_is_the_real_displacement_in_a_closed_box():
    dims = (8, 8, 8)
    w = dict(workload("cfg1"), dims=dims, place=[(1, 24)], seed=5)
    o = build(w, oracle.REFLECT)
    s0 = o.state()
    p0 = {i: oracle.position(dims, int(v), RV) for i, v in zip(s0["id"], s0["vox"])}
    o.run(300, oracle.MODE_C)
    s = o.state()
    assert s["hops"] > 1000
    for i, v, dx, dy, dz in zip(s["id"], s["vox"], s["dx"], s["dy"], s["dz"]):
        p = oracle.position(dims, int(v), RV)
        real = np.subtract(p, p0[i])
        tracked = np.array([dx * RV, dy * RV / math.sqrt(3.0), dz * H])
        assert np.allclose(real, tracked, atol=1e-6 * RV), (i, real, tracked)
    # the same run on a periodic box wraps: some molecule crosses a face
    o = build(w, oracle.PERIODIC)
    o.run(300, oracle.MODE_C)
    s = o.state()
    crossed = 0
    for i, v, dx, dy, dz in zip(s["id"], s["vox"], s["dx"], s["dy"], s["dz"]):
        real = np.subtract(oracle.position(dims, int(v), RV), p0[i])
        tracked = np.array([dx * RV, dy * RV / math.sqrt(3.0), dz * H])
        crossed += not np.allclose(real, tracked, atol=1e-6 * RV)
    assert crossed > 0


def test_closed_box_walk_is_symmetric_and_occupancy_uniform():
    dims = (4, 4, 4)
    nv = 64
    # exact: one molecule at each voxel, each forced direction, one walk
    P = np.zeros((nv, nv))
    for v in range(nv):
        for n in range(12):
            o = oracle.Oracle(dims, RV, 1, boundary=oracle.REFLECT)
            a = o.add_species(1e-12)
            occ = np.zeros(nv, np.uint16)
            occ[v] = a
            o.load(occ, np.array([0], np.uint32), np.array([v], np.uint32), None, 0, 1)
            o.walk_forced([0], [n], [0])
            s = o.state(with_occ=False)
            P[v, s["vox"][0]] += 1.0 / 12.0
            assert s["attempts"] == 1 and s["collisions"] == 0
            t = oracle.neighbour_b(dims, v, n, oracle.REFLECT)
            assert s["vox"][0] == (v if t == oracle.OUTSIDE else t)
    assert np.allclose(P, P.T) and np.allclose(P.sum(axis=1), 1.0)
    assert np.allclose(np.full(nv, 1.0 / nv) @ P, 1.0 / nv)
    # statistical: the exclusion process in the closed box visits corners,
    # edges, faces and the interior equally often (class averages)
    w = dict(workload("cfg1"), dims=dims, place=[(1, 16)], seed=9)
    o = build(w, oracle.REFLECT)
    o.run(50, oracle.MODE_C)
    hist = np.zeros(nv)
    n = 40000
    for _ in range(n):
        o.run(1, oracle.MODE_C)
        hist[o.state(with_occ=False)["vox"]] += 1
    expect = 16 * n / nv
    deg = np.array([sum(oracle.neighbour_b(dims, v, k, oracle.REFLECT) != oracle.OUTSIDE
                        for k in range(12)) for v in range(nv)])
    assert len(set(deg.tolist())) >= 3
    for d in sorted(set(deg.tolist())):
        m = hist[deg == d].mean()
        assert abs(m - expect) < 0.04 * expect, (d, int((deg == d).sum()), m, expect)


@pytest.mark.parametrize("seed", [3, 4])
def test_stages_commute_with_walls(seed):
    w = workload("small_reactive", seed=seed)
    a = build(w, oracle.REFLECT)
    b = build(w, oracle.REFLECT)
    a.run(40, oracle.MODE_C)
    b.run(40, oracle.MODE_C_REV)
    sa, sb = a.state(), b.state()
    for key in ("occ", "id", "vox", "species", "dx", "dy", "dz"):
        assert np.array_equal(sa[key], sb[key]), key
    assert sa["fired"].tolist() == sb["fired"].tolist()
    assert sa["hops"] == sb["hops"] and sa["collisions"] == sb["collisions"]
    # the walls change the run
    c = build(w, oracle.PERIODIC)
    c.run(40, oracle.MODE_C)
    assert not np.array_equal(sa["occ"], c.state()["occ"])


def test_no_product_beyond_a_wall():
    dims = (8, 8, 8)
    nv = 512
    inside = sum(oracle.neighbour_b(dims, 0, n, oracle.REFLECT) != oracle.OUTSIDE
                 for n in range(12))
    assert inside < 11
    far = 4 + 8 * (4 + 8 * 4)   # voxel (4, 4, 4), away from voxel 0's neighbourhood
    for boundary, fails in ((oracle.REFLECT, 1), (oracle.PERIODIC, 0)):
        o = oracle.Oracle(dims, RV, 1, boundary=boundary)
        a = o.add_species(0.0)       # immobile reactant and products stay put
        b = o.add_species(0.0)
        c = o.add_species(1e-12)     # a walker far away drives the events
        o.add_reaction((a,), (a,) + (b,) * 10, 1e9)   # fires at once
        occ = np.zeros(nv, np.uint16)
        occ[0] = a
        occ[far] = c
        o.load(occ, np.array([0, 1], np.uint32), np.array([0, far], np.uint32), None, 0, 2)
        o.run(1, oracle.MODE_C)
        s = o.state()
        assert s["place_fail"] == fails
        assert int((s["species"] == b).sum()) == (0 if fails else 10)
        if not fails:
            # every product sits on a distinct neighbour of voxel 0 (periodic)
            nb = {oracle.neighbour(dims, 0, n) for n in range(12)}
            born = s["vox"][s["species"] == b].tolist()
            assert len(set(born)) == 10 and set(born) <= nb
