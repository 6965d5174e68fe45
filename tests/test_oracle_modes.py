"""Whole-run checks of the oracle: stage commutativity over many events with
every reaction rule, checkpoint/resume equivalence, and conservation
invariants (occupancy <-> molecule table, one hop per event at most, species
balance against the fired-reaction counters)."""
import numpy as np
import pytest

import oracle
from psc_inputs import workload


def build(w, state=None):
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"])
    for _, D in w["species"]:
        o.add_species(D)
    for r, p, k in w["reactions"]:
        o.add_reaction(r, p, k)
    if state is None:
        for s, c in w["place"]:
            o.place_uniform(s, c)
    else:
        o.load(state["occ"], state["id"], state["vox"],
               (state["dx"], state["dy"], state["dz"]), state["event"], state["next_id"])
    return o


def same_state(a, b):
    for key in ("occ", "id", "vox", "species", "dx", "dy", "dz"):
        assert np.array_equal(a[key], b[key]), key
    for key in ("attempts", "hops", "collisions", "place_fail", "event", "next_id"):
        assert a[key] == b[key], key
    assert a["time"] == b["time"]
    assert np.array_equal(a["fired"], b["fired"])


def check_consistent(w, s):
    nv = int(np.prod(w["dims"]))
    occ = s["occ"]
    assert len(np.unique(s["vox"])) == len(s["vox"])
    assert np.all(occ[s["vox"]] == s["species"])
    assert int((occ != 0).sum()) == len(s["id"])
    assert np.all(np.diff(s["id"].astype(np.int64)) > 0)
    assert len(occ) == nv


@pytest.mark.parametrize("seed", [7, 8])
def test_reversed_intra_stage_order_gives_identical_run(seed):
    w = workload("small_reactive", seed=seed, events=60)
    a = build(w)
    a.run(w["events"], oracle.MODE_C)
    b = build(w)
    b.run(w["events"], oracle.MODE_C_REV)
    sa, sb = a.state(), b.state()
    same_state(sa, sb)
    # the run actually exercised the rules
    assert sa["hops"] > 0 and sa["collisions"] > 0
    assert np.all(sa["fired"] > 0), sa["fired"]


@pytest.mark.parametrize("mode", [oracle.MODE_C, oracle.MODE_S])
def test_checkpoint_resume_is_exact(mode):
    w = workload("small_reactive", events=50)
    full = build(w)
    full.run(50, mode)
    part = build(w)
    part.run(20, mode)
    st = part.state()
    st_counters = {k: st[k] for k in ("attempts", "hops", "collisions", "place_fail")}
    res = build(w, state=st)
    res.run(30, mode)
    sf, sr = full.state(), res.state()
    for key in ("occ", "id", "vox", "species", "dx", "dy", "dz"):
        assert np.array_equal(sf[key], sr[key]), key
    assert sf["event"] == sr["event"] and sf["next_id"] == sr["next_id"]
    assert sf["time"] == sr["time"]
    assert sf["attempts"] == st_counters["attempts"] + sr["attempts"]


@pytest.mark.parametrize("mode", [oracle.MODE_C, oracle.MODE_S])
def test_invariants_every_event(mode):
    w = workload("small_reactive", events=1)
    o = build(w)
    prev = o.state()
    nrx = len(w["reactions"])
    counts0 = {s: int((prev["species"] == s).sum()) for s in range(1, len(w["species"]) + 1)}
    for e in range(60):
        o.run(1, mode)
        s = o.state()
        check_consistent(w, s)
        # molecules that survive with the same id move at most one hop
        common, ia, ib = np.intersect1d(prev["id"], s["id"], return_indices=True)
        dX = s["dx"][ib] - prev["dx"][ia]
        dY = s["dy"][ib] - prev["dy"][ia]
        dZ = s["dz"][ib] - prev["dz"][ia]
        q = 3 * dX.astype(np.int64) ** 2 + dY.astype(np.int64) ** 2 + 8 * dZ.astype(np.int64) ** 2
        assert set(np.unique(q).tolist()) <= {0, 12}
        prev = s
    # species balance: final - initial = sum over reactions of fired x net change
    fired = prev["fired"]
    for sp in range(1, len(w["species"]) + 1):
        net = 0
        for r, (reac, prod, _) in enumerate(w["reactions"]):
            net += int(fired[r]) * (list(prod).count(sp) - list(reac).count(sp))
        assert int((prev["species"] == sp).sum()) - counts0[sp] == net, sp
    assert nrx == len(fired)


def test_placement_counts_and_exclusivity():
    w = workload("small_reactive")
    o = build(w)
    s = o.state()
    check_consistent(w, s)
    for sp, c in w["place"]:
        assert int((s["species"] == sp).sum()) == c
    assert list(s["id"]) == list(range(len(s["id"])))


def test_placement_is_uniform():
    # voxel hit counts over many placements: chi-square against uniform
    dims = (8, 8, 8)
    hits = np.zeros(512)
    for seed in range(40):
        o = oracle.Oracle(dims, 4.4e-9, seed)
        o.add_species(1e-12)
        o.place_uniform(1, 64)
        hits[o.state()["vox"]] += 1
    exp = hits.sum() / 512
    chi2 = float(((hits - exp) ** 2 / exp).sum())
    # 511 dof: mean 511, sd ~32 (sampling without replacement lowers it)
    assert chi2 < 511 + 5 * 32
