"""Exhaustive checks of the oracle's walk on a 4x4x4 periodic lattice.

For a handful of molecules every combination of neighbour choices (12^n) --
and, with reactions, every fire/no-fire outcome -- is enumerated:
  * inside a colour stage the processing order does not change the result
    (same-colour closed neighbourhoods are disjoint), so the coloured schedule
    is a valid sequential order of the paper's one-by-one walk (2.3);
  * a molecule hops for exactly as many of its 12 choices as it has vacant
    neighbours (2.3: it moves only if the chosen voxel is vacant);
  * the Philox-driven event equals the forced walk driven by the same draws.
"""
import itertools

import numpy as np
import pytest

import oracle

DIMS = (4, 4, 4)
NV = 64
RV = 4.4e-9


def make(state, reactions=()):
    o = oracle.Oracle(DIMS, RV, seed=77)
    o.add_species(1e-12)   # A
    o.add_species(1e-12)   # B
    o.add_species(1e-12)   # C
    for r, p, k in reactions:
        o.add_reaction(r, p, k)
    o.load(state["occ"], state["id"], state["vox"])
    return o


def state_of(vox, species, ids=None):
    vox = np.asarray(vox, np.uint32)
    species = np.asarray(species, np.uint16)
    ids = np.arange(len(vox), dtype=np.uint32) if ids is None else np.asarray(ids, np.uint32)
    occ = np.zeros(NV, np.uint16)
    occ[vox] = species
    return {"occ": occ, "id": ids, "vox": vox}


def snapshot(o):
    s = o.state()
    return (s["occ"].tobytes(), s["id"].tobytes(), s["vox"].tobytes(),
            s["species"].tobytes(), s["hops"], s["collisions"], tuple(s["fired"]))


def stage_grouped(vox, ids, order16, within):
    """molecule ids grouped by colour stage; `within` orders each group"""
    out = []
    for c in order16:
        grp = [i for v, i in zip(vox, ids) if oracle.colour(DIMS, int(v)) == c]
        out.extend(within(sorted(grp)))
    return out


def pick_cluster(rng, n):
    """n voxels: one seed voxel, one voxel of the same colour (3 hops away at
    most on 4^3), the rest neighbours of the seed"""
    v0 = int(rng.integers(NV))
    same = [u for u in range(NV) if u != v0 and oracle.colour(DIMS, u) == oracle.colour(DIMS, v0)]
    vox = [v0, int(rng.choice(same))]
    nb = [oracle.neighbour(DIMS, v0, m) for m in range(12)]
    rng.shuffle(nb)
    for u in nb:
        if len(vox) == n:
            break
        if u not in vox:
            vox.append(int(u))
    return vox[:n]


@pytest.mark.parametrize("n,seed", [(2, 1), (3, 2), (3, 3), (4, 4)])
def test_intra_stage_order_is_irrelevant_pure_diffusion(n, seed):
    rng = np.random.default_rng(seed)
    vox = pick_cluster(rng, n)
    st = state_of(vox, [1] * n)
    order16 = list(rng.permutation(16))
    fwd = stage_grouped(vox, st["id"], order16, lambda g: g)
    rev = stage_grouped(vox, st["id"], order16, lambda g: g[::-1])
    fire = np.zeros(n, np.uint8)
    for dirs in itertools.product(range(12), repeat=n):
        d = np.array(dirs, np.uint8)
        a = make(st)
        a.walk_forced(fwd, d, fire)
        b = make(st)
        b.walk_forced(rev, d, fire)
        assert snapshot(a) == snapshot(b)


@pytest.mark.parametrize("n,seed", [(3, 5), (3, 6)])
def test_intra_stage_order_is_irrelevant_with_reactions(n, seed):
    rng = np.random.default_rng(seed)
    vox = pick_cluster(rng, n)
    species = [1, 2, 1][:n]
    st = state_of(vox, species)
    rx = [((1, 2), (3,), 1e-18), ((1, 1), (2, 3), 1e-18)]
    order16 = list(rng.permutation(16))
    fwd = stage_grouped(vox, st["id"], order16, lambda g: g)
    rev = stage_grouped(vox, st["id"], order16, lambda g: g[::-1])
    for dirs in itertools.product(range(12), repeat=n):
        for fire in itertools.product((0, 1), repeat=n):
            d = np.array(dirs, np.uint8)
            f = np.array(fire, np.uint8)
            a = make(st, rx)
            a.walk_forced(fwd, d, f)
            b = make(st, rx)
            b.walk_forced(rev, d, f)
            assert snapshot(a) == snapshot(b)


def test_hop_count_equals_vacant_neighbours():
    rng = np.random.default_rng(9)
    for _ in range(20):
        vox = [int(x) for x in rng.choice(NV, size=6, replace=False)]
        st = state_of(vox, [1] * 6)
        mover = 0
        vacant = sum(1 for m in range(12) if st["occ"][oracle.neighbour(DIMS, vox[mover], m)] == 0)
        hops = 0
        for d in range(12):
            o = make(st)
            dirs = np.zeros(6, np.uint8)
            dirs[mover] = d
            o.walk_forced([mover], dirs, np.zeros(6, np.uint8))
            s = o.state()
            hops += s["hops"]
            assert s["attempts"] == 1
        assert hops == vacant


def test_collision_products_keep_identities():
    # A (id 0) moves onto B (id 1): A + B -> C + A puts C on B's voxel with
    # B's id and A on the mover's voxel with the mover's id; A + B -> C with
    # one product removes the mover
    a_v = 0
    d = 0
    b_v = oracle.neighbour(DIMS, a_v, d)
    st = state_of([a_v, b_v], [1, 2])
    o = make(st, [((1, 2), (3, 1), 1e-18)])
    o.walk_forced([0, 1], np.array([d, 0], np.uint8), np.array([1, 0], np.uint8))
    s = o.state()
    assert list(s["id"]) == [0, 1]
    assert list(s["vox"]) == [a_v, b_v]
    assert list(s["species"]) == [1, 3]
    assert s["attempts"] == 1  # the partner reacted, so it does not walk
    o = make(st, [((1, 2), (3,), 1e-18)])
    o.walk_forced([0, 1], np.array([d, 0], np.uint8), np.array([1, 0], np.uint8))
    s = o.state()
    assert list(s["id"]) == [1] and list(s["vox"]) == [b_v] and list(s["species"]) == [3]
    assert s["occ"][a_v] == 0


def test_philox_event_equals_forced_walk():
    rng = np.random.default_rng(11)
    seed, e = 77, 0
    key = (seed & 0xFFFFFFFF, seed >> 32)
    D = 1e-12
    k = 3e-20
    T = oracle.second_order_threshold(k, D, D, RV)
    assert 0 < T < 2**32
    for trial in range(10):
        n = int(rng.integers(4, 14))
        vox = rng.choice(NV, size=n, replace=False)
        species = rng.integers(1, 3, size=n)
        ids = np.sort(rng.choice(200, size=n, replace=False)).astype(np.uint32)
        st = state_of(vox, species, ids)
        rx = [((1, 2), (3,), k)]
        a = make(st, rx)
        a.run(1, oracle.MODE_C)
        # the same event driven by hand from the draws: direction from word 0,
        # collision test from word 1, molecules by stage then ascending id
        dirs = np.zeros(200, np.uint8)
        fire = np.zeros(200, np.uint8)
        for i in ids:
            r = oracle.philox4x32((e, int(i), 0, 0), key)
            dirs[i] = (int(r[0]) * 12) >> 32
            fire[i] = 1 if int(r[1]) < T else 0
        order = stage_grouped(vox, ids, oracle.stage_order(seed, e), lambda g: g)
        b = make(st, rx)
        b.walk_forced(order, dirs, fire)
        assert snapshot(a) == snapshot(b)


@pytest.mark.parametrize("mode", [oracle.MODE_C, oracle.MODE_S])
def test_first_order_products_go_to_distinct_vacant_neighbours(mode):
    # A -> A + B + B with an enormous rate: the first product stays, the two
    # others land on distinct vacant neighbours of the parent (2.4.1)
    for seed in range(12):
        o = oracle.Oracle(DIMS, RV, seed)
        A = o.add_species(1e-12)
        B = o.add_species(0.0)
        o.add_reaction((A,), (A, B, B), 1e9)
        rng = np.random.default_rng(seed)
        v0 = int(rng.integers(NV))
        blocked = [oracle.neighbour(DIMS, v0, m) for m in rng.choice(12, size=8, replace=False)]
        occ = np.zeros(NV, np.uint16)
        occ[v0] = A
        occ[blocked] = B
        vox = np.array(sorted([v0] + blocked), np.uint32)
        ids = np.arange(len(vox), dtype=np.uint32)
        o.load(occ, ids, vox)
        parent_id = int(ids[list(vox).index(v0)])
        o.run(1, mode)
        s = o.state()
        born = s["id"] >= len(vox)
        # the per-molecule law fires at most once per event; Gillespie's
        # method may fire again while the parent still has room (4 free
        # neighbours: two firings)
        assert born.sum() == (2 if mode == oracle.MODE_C else 4)
        nbrs = {oracle.neighbour(DIMS, v0, m) for m in range(12)}
        free = nbrs - set(blocked)
        kids = set(s["vox"][born].tolist())
        assert len(kids) == born.sum() and kids <= free
        assert all(s["species"][born] == B)
        # the parent keeps its id (it may have walked one hop afterwards)
        assert parent_id in s["id"].tolist()
