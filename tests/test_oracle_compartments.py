"""Compartments (section 2: a cell is groups of voxels; 2.3: a move into a
voxel of another compartment fails as a move into an occupied one).

Pins that do not re-derive the oracle's code:
- a compartment that is a sub-box at the origin of a periodic lattice twice
  its size, every other voxel in a second, empty compartment, behaves
  exactly as the same box closed by walls (whose in-box neighbours are
  pinned to the voxels at Euclidean distance 2r): the same state loaded into
  both runs bit for bit alike, with every rule (first-order and collision
  products, placement failures), on both lattices;
- molecules never leave their compartment: over a run of every rule on a
  cell-like map (cytosol, a membrane shell, a nucleus) the compartment of
  each molecule's voxel never changes, and every newborn sits in a
  compartment that held a molecule of a species able to produce it;
- a hop towards another compartment counts as an attempt, moves nothing and
  is no collision, even onto a registered partner (forced walks);
- placement restricted to a compartment puts every molecule there, uniformly
  (chi-square over the compartment's voxels, pooled by region);
- coloured stages still commute (reversed order inside stages is identical)."""
import numpy as np
import pytest

import oracle
from psc_inputs import layered_map, membrane, shell_map, sub_box_map, workload


def build(w, comp=None, boundary=None, lattice=None, place=True):
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"],
                      boundary=boundary if boundary is not None else (
                          oracle.REFLECT if w.get("boundary") == "walls" else oracle.PERIODIC),
                      lattice=lattice if lattice is not None else (
                          oracle.FCC if w.get("lattice") == "fcc" else oracle.HCP))
    for _, D in w["species"]:
        o.add_species(D)
    for r, p, k in w["reactions"]:
        o.add_reaction(r, p, k)
    c = comp if comp is not None else w.get("compartments")
    if c is not None:
        o.set_compartments(c)
    if place:
        for s, n in w["place"]:
            o.place_uniform(s, n)
        for s, n, cc in w.get("place_in", []):
            o.place_uniform_in(s, n, cc)
    return o


def same(a, b, keys=("id", "species", "dx", "dy", "dz")):
    for k in keys:
        assert np.array_equal(a[k], b[k]), k
    for k in ("attempts", "hops", "collisions", "place_fail", "next_id", "event"):
        assert a[k] == b[k], (k, a[k], b[k])
    assert np.array_equal(a["fired"], b["fired"])


@pytest.mark.parametrize("lattice,small", [(oracle.HCP, (8, 8, 8)), (oracle.HCP, (12, 8, 16)),
                                           (oracle.FCC, (8, 8, 12)), (oracle.FCC, (16, 8, 12))])
@pytest.mark.parametrize("seed", [3, 4])
def test_sub_box_compartment_equals_the_box_closed_by_walls(lattice, small, seed):
    big = tuple(2 * x for x in small)
    net = workload("small_reactive", dims=small, seed=seed, events=50)
    mp = workload("multiproduct", dims=small, seed=seed)
    # every rule: the small network plus a four-product collision
    net = dict(net, reactions=net["reactions"] + [((3, 5), (5, 3, 2, 2), 3e-20)])
    walled = build(net, boundary=oracle.REFLECT, lattice=lattice)
    s0 = walled.state()
    # the same molecules at the same (i, j, k) inside the big periodic box
    ni, nj, nk = small
    i, j, k = s0["vox"] % ni, (s0["vox"] // ni) % nj, s0["vox"] // (ni * nj)
    vbig = i + big[0] * (j + big[1] * k)
    occ = np.zeros(int(np.prod(big)), np.uint16)
    occ[vbig] = s0["species"]
    boxed = build(dict(net, dims=big), comp=sub_box_map(big, small), boundary=oracle.PERIODIC,
                  lattice=lattice, place=False)
    boxed.load(occ, s0["id"], vbig, next_id=s0["next_id"])
    for _ in range(5):
        walled.run(10)
        boxed.run(10)
        a, b = walled.state(), boxed.state()
        same(a, b)
        ai, aj, ak = a["vox"] % ni, (a["vox"] // ni) % nj, a["vox"] // (ni * nj)
        assert np.array_equal(b["vox"], ai + big[0] * (aj + big[1] * ak))
    assert a["fired"].sum() > 0 and a["place_fail"] >= 0
    del mp


@pytest.mark.parametrize("lattice,dims", [(oracle.HCP, (24, 24, 24)), (oracle.FCC, (24, 24, 24))])
def test_molecules_never_leave_their_compartment(lattice, dims):
    w = membrane(dims=dims, seed=7, lattice="fcc" if lattice == oracle.FCC else "hcp")
    comp = w["compartments"]
    o = build(w)
    s = o.state()
    home = dict(zip(s["id"].tolist(), comp[s["vox"]].tolist()))
    # which species occur in which compartment at the start (products of a
    # reaction share the compartment of its reactants)
    fired_total = 0
    for _ in range(8):
        o.run(10)
        s = o.state()
        c = comp[s["vox"]]
        for mid, cc in zip(s["id"].tolist(), c.tolist()):
            if mid in home:
                assert home[mid] == cc, mid
            else:
                home[mid] = cc
        fired_total = int(s["fired"].sum())
    # the membrane species M never appears off the membrane, the cytosol and
    # nucleus species never on it
    assert np.all(c[s["species"] == 4] == 1)
    assert np.all(c[np.isin(s["species"], [1, 2, 3])] != 1)
    assert fired_total > 100
    # every compartment still holds molecules
    assert set(np.unique(c).tolist()) == {0, 1, 2}


def test_hop_into_another_compartment_is_blocked_and_no_collision():
    dims = (8, 8, 8)
    w = dict(workload("small_reactive", dims=dims, seed=1), place=[])
    nb = oracle.neighbour_table(dims)
    v, n = 100, 3
    t = int(nb[v, n])
    comp = np.zeros(512, np.uint8)
    comp[t] = 1
    # an A at v, a registered partner B (A + B -> C) in the other compartment at t
    occ = np.zeros(512, np.uint16)
    occ[v], occ[t] = 2, 3
    for fire in (0, 1):
        o = build(w, comp=comp, place=False)
        o.load(occ, np.array([0, 1], np.uint32), np.array([v, t], np.uint32), next_id=2)
        dirs = np.zeros(2, np.uint8)
        dirs[0] = n
        o.walk_forced([0], dirs, np.array([fire, 0], np.uint8))
        s = o.state()
        assert (s["attempts"], s["hops"], s["collisions"]) == (1, 0, 0)
        assert list(s["vox"]) == [v, t] and list(s["species"]) == [2, 3]
        assert s["fired"].sum() == 0
    # the same pair in one compartment: a collision that fires
    o = build(w, comp=np.zeros(512, np.uint8), place=False)
    o.load(occ, np.array([0, 1], np.uint32), np.array([v, t], np.uint32), next_id=2)
    o.walk_forced([0], dirs, np.array([1, 0], np.uint8))
    s = o.state()
    assert (s["attempts"], s["collisions"]) == (1, 1) and s["fired"][0] == 1


def test_placement_in_a_compartment_is_uniform_there():
    dims = (32, 32, 32)
    comp = shell_map(dims, radius_frac=0.3, thickness=2.0)
    w = dict(workload("cfg1"), dims=dims, place=[], seed=11)
    o = build(w, comp=comp, place=False)
    inner = np.nonzero(comp == 2)[0]
    count = len(inner) // 3
    o.place_uniform_in(1, count, 2)
    s = o.state()
    assert len(s["id"]) == count and np.all(comp[s["vox"]] == 2)
    # pooled by octant of the box: each octant holds its share of the
    # compartment's voxels
    def octant(v):
        i, j, k = v % 32, (v // 32) % 32, v // 1024
        return (i >= 16) + 2 * (j >= 16) + 4 * (k >= 16)
    share = np.bincount(octant(inner), minlength=8) / len(inner)
    got = np.bincount(octant(s["vox"]), minlength=8)
    exp = share * count
    chi2 = float(((got - exp) ** 2 / exp).sum())
    assert chi2 < 24.3  # 7 dof, p = 1e-3
    # too many for the compartment: refused
    with pytest.raises(ValueError):
        o.place_uniform_in(1, len(inner), 2)


@pytest.mark.parametrize("comp_kind", ["shell", "layers"])
def test_stages_commute_with_compartments(comp_kind):
    dims = (16, 16, 16)
    w = membrane(dims=dims, seed=9, radius_frac=0.4)
    if comp_kind == "layers":
        w = dict(w, compartments=layered_map(dims, 4),
                 place_in=[(1, 120, 0), (2, 120, 1), (4, 60, 2), (1, 100, 3), (2, 100, 3)])
    a, b = build(w), build(w)
    a.run(40, oracle.MODE_C)
    b.run(40, oracle.MODE_C_REV)
    sa, sb = a.state(), b.state()
    same(sa, sb)
    assert np.array_equal(sa["vox"], sb["vox"]) and np.array_equal(sa["occ"], sb["occ"])
