"""Collision reactions with more than two products (section 2.4: two
reactants may decay into several molecules, at most eleven).  The first
product takes the partner's voxel and id, the second the mover's voxel and
id, the others go to distinct vacant neighbours of the mover's voxel; with
too few vacant neighbours the reaction fails with no change.  Newborn ids are
given at the end of the walk in ascending (mover id, product index) order.

Pins (none re-derives the oracle's choice rule):
- placement: extra products land on distinct vacant neighbours of the
  mover's voxel, never elsewhere, and over many draws every vacant neighbour
  is chosen about equally often;
- failure: too few vacant neighbours leaves the state unchanged and counts
  one placement failure;
- ids: newborns are numbered by mover id, not by processing order, so a
  walk in reversed order gives the same ids;
- bookkeeping: with p = 1 every collision of the pair fires unless the
  placement fails, exactly."""
import numpy as np
import pytest

import oracle

RV = 4.4e-9
DIMS = (8, 8, 8)
NV = 512


def setup(boundary=oracle.PERIODIC, n_prod=4):
    o = oracle.Oracle(DIMS, RV, 1, boundary=boundary)
    a = o.add_species(1e-12)
    b = o.add_species(1e-12)
    c = o.add_species(1e-12)
    x = o.add_species(0.0)          # obstacle
    prods = (c,) * n_prod
    o.add_reaction((a, b), prods, 1e-15)   # p clamps to 1
    return o, a, b, c, x


def load(o, placed):
    occ = np.zeros(NV, np.uint16)
    ids, vox = [], []
    for i, (v, sp) in enumerate(placed):
        occ[v] = sp
        ids.append(i)
        vox.append(v)
    o.load(occ, np.array(ids, np.uint32), np.array(vox, np.uint32), None, 0, len(placed))


def test_extra_products_on_distinct_vacant_neighbours_uniformly():
    v0, d = 200, 3
    hits = {}
    for seed in range(300):
        o = oracle.Oracle(DIMS, RV, seed)
        a, b, c = o.add_species(1e-12), o.add_species(1e-12), o.add_species(1e-12)
        x = o.add_species(0.0)
        o.add_reaction((a, b), (c, c, c, c), 1e-15)
        t = oracle.neighbour(DIMS, v0, d)
        # block three neighbours of the mover with obstacles
        nb = [oracle.neighbour(DIMS, v0, n) for n in range(12)]
        blocked = [u for u in nb if u != t][:3]
        load(o, [(v0, a), (t, b)] + [(u, x) for u in blocked])
        o.walk_forced([0], [d, 0] + [0] * 3, [1, 0] + [0] * 3)
        s = o.state()
        assert s["fired"][0] == 1 and s["place_fail"] == 0
        by_id = dict(zip(s["id"].tolist(), zip(s["vox"].tolist(), s["species"].tolist())))
        assert by_id[1] == (t, c) and by_id[0] == (v0, c)   # partner id on t, mover id on v0
        born = [by_id[i] for i in (5, 6)]                     # next ids after 0..4
        assert all(sp == c for _, sp in born)
        vs = [v for v, _ in born]
        vacant = set(nb) - {t} - set(blocked)
        assert len(set(vs)) == 2 and set(vs) <= vacant
        for v in vs:
            hits[v] = hits.get(v, 0) + 1
    assert set(hits) == vacant
    counts = np.array([hits[v] for v in sorted(vacant)])
    expect = 600 / len(vacant)
    assert np.all(np.abs(counts - expect) < 0.4 * expect), counts


def test_too_few_vacant_neighbours_fails_with_no_change():
    o, a, b, c, x = setup(n_prod=3)
    v0, d = 200, 5
    t = oracle.neighbour(DIMS, v0, d)
    others = [oracle.neighbour(DIMS, v0, n) for n in range(12) if n != d]
    load(o, [(v0, a), (t, b)] + [(u, x) for u in others])
    before = o.state()
    o.walk_forced([0], [d] + [0] * 12, [1] + [0] * 12)
    s = o.state()
    assert s["place_fail"] == 1 and s["fired"][0] == 0 and s["collisions"] == 1
    for key in ("occ", "id", "vox", "species"):
        assert np.array_equal(s[key], before[key]), key
    # one vacant neighbour is enough for three products
    o, a, b, c, x = setup(n_prod=3)
    load(o, [(v0, a), (t, b)] + [(u, x) for u in others[1:]])
    o.walk_forced([0], [d] + [0] * 11, [1] + [0] * 11)
    s = o.state()
    assert s["place_fail"] == 0 and s["fired"][0] == 1
    assert s["occ"][others[0]] == c and s["id"][-1] == 2 + 10


def test_newborn_ids_follow_mover_ids_not_processing_order():
    o, a, b, c, x = setup(n_prod=3)
    # two reacting pairs far apart; molecule 2 (a mover) is processed first
    v1, v2 = 100, 400
    t1, t2 = oracle.neighbour(DIMS, v1, 0), oracle.neighbour(DIMS, v2, 0)
    load(o, [(v1, a), (t1, b), (v2, a), (t2, b)])
    o.walk_forced([2, 0], [0, 0, 0, 0], [1, 0, 1, 0])
    s = o.state()
    born = {int(i): int(v) for i, v in zip(s["id"], s["vox"]) if i >= 4}
    nb1 = {oracle.neighbour(DIMS, v1, n) for n in range(12)}
    nb2 = {oracle.neighbour(DIMS, v2, n) for n in range(12)}
    assert born[4] in nb1 and born[5] in nb2   # id 4 from mover 0, id 5 from mover 2


@pytest.mark.parametrize("boundary", [oracle.PERIODIC, oracle.REFLECT])
def test_runs_commute_and_balance(boundary):
    dims = (16, 12, 8)
    o = {}
    for mode in (oracle.MODE_C, oracle.MODE_C_REV):
        q = oracle.Oracle(dims, RV, 7, boundary=boundary)
        a, b, c = q.add_species(1e-12), q.add_species(0.5e-12), q.add_species(2e-12)
        q.add_reaction((a, b), (b, a, c, c), 1e-15)     # p = 1
        q.add_reaction((c,), (), 3000.0)
        q.place_uniform(a, 150)
        q.place_uniform(b, 150)
        q.run(30, mode)
        o[mode] = q.state()
    sc, sr = o[oracle.MODE_C], o[oracle.MODE_C_REV]
    for key in ("occ", "id", "vox", "species", "dx", "dy", "dz"):
        assert np.array_equal(sc[key], sr[key]), key
    assert sc["fired"].tolist() == sr["fired"].tolist()
    assert sc["fired"][0] > 20
    # A and B are conserved by the pair reaction; every C ever born is alive
    # or was removed by the first-order decay
    n_a = int((sc["species"] == 1).sum())
    n_b = int((sc["species"] == 2).sum())
    n_c = int((sc["species"] == 3).sum())
    assert n_a == 150 and n_b == 150
    assert n_c == 2 * int(sc["fired"][0]) - int(sc["fired"][1])


def test_every_collision_of_the_pair_fires_or_fails_to_place():
    dims = (16, 16, 16)
    q = oracle.Oracle(dims, RV, 3)
    a, b, c = q.add_species(1e-12), q.add_species(1e-12), q.add_species(0.0)
    q.add_reaction((a, b), (a, b) + (c,) * 9, 1e-15)   # p = 1, nine extra products
    q.place_uniform(a, 300)
    q.place_uniform(b, 300)
    q.run(40, oracle.MODE_C)
    s = q.state()
    n_c = int((s["species"] == c).sum())
    assert s["fired"][0] > 0 and s["place_fail"] > 0
    assert n_c == 9 * int(s["fired"][0])
    # A-A, B-B and A/B-C collisions do not react; A-B ones fire or fail
    assert s["fired"][0] + s["place_fail"] <= s["collisions"]
