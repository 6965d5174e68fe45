"""Randomised models against the oracle: for each seed, a random reaction
network (2-6 species, some immobile; second-order pairs with 1-11 products;
first-order reactions with 0-3 products), a random lattice kind, boundary,
box and occupancy, with or without displacement tracking.  The GPU run must
equal the oracle's coloured-stage run bit for bit after 20 events.  The
models are drawn by `random_model`, which holds no arithmetic of the method
(it only picks parameters)."""
import numpy as np
import pytest

import oracle
from paper_1605_03726_amd import psc

RV = 4.4e-9


def random_model(seed: int) -> dict:
    rng = np.random.default_rng(1000 + seed)
    fcc = bool(rng.integers(2))
    if fcc:
        dims = [(8, 8, 12), (16, 8, 12), (16, 16, 12), (8, 16, 24)][rng.integers(4)]
    else:
        dims = [(8, 8, 8), (12, 8, 4), (16, 12, 8), (4, 16, 12)][rng.integers(4)]
    nv = dims[0] * dims[1] * dims[2]
    n_sp = int(rng.integers(2, 7))
    D = [float(rng.choice([0.0, 0.5e-12, 1e-12, 2e-12])) for _ in range(n_sp)]
    D[0] = 1e-12                                  # at least one walker
    species = [("S%d" % s, D[s]) for s in range(n_sp)]
    ids = list(range(1, n_sp + 1))
    reactions, pairs = [], set()
    for _ in range(int(rng.integers(1, 5))):
        a, b = sorted(int(x) for x in rng.choice(ids, 2))
        if (a, b) in pairs or (D[a - 1] == 0.0 and D[b - 1] == 0.0):
            continue
        pairs.add((a, b))
        n_p = int(rng.choice([1, 1, 2, 2, 3, 4, 11]))
        prods = tuple(int(x) for x in rng.choice(ids, n_p))
        k = float(10.0 ** rng.uniform(-20, -16))
        reactions.append(((a, b), prods, k))
    for _ in range(int(rng.integers(0, 4))):
        a = int(rng.choice(ids))
        n_p = int(rng.integers(0, 4))
        prods = tuple(int(x) for x in rng.choice(ids, n_p))
        reactions.append(((a,), prods, float(10.0 ** rng.uniform(1, 3.7))))
    place = [(s, int(nv * rng.uniform(0.01, 0.12))) for s in ids[: int(rng.integers(1, n_sp + 1))]]
    w = dict(name="random_%d" % seed, dims=dims, rv=RV, seed=int(rng.integers(1, 1 << 30)),
             species=species, reactions=reactions, place=place, events=20,
             track_displacement=bool(rng.integers(2)))
    if fcc:
        w["lattice"] = "fcc"
    if rng.integers(2):
        w["boundary"] = "walls"
    return w


def oracle_state(w):
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"],
                      boundary=oracle.REFLECT if w.get("boundary") == "walls" else oracle.PERIODIC,
                      lattice=oracle.FCC if w.get("lattice") == "fcc" else oracle.HCP)
    for _, D in w["species"]:
        o.add_species(D)
    for r, p, k in w["reactions"]:
        o.add_reaction(r, p, k)
    for s, c in w["place"]:
        o.place_uniform(s, c)
    o.run(w["events"], oracle.MODE_C)
    return o.state()


@pytest.mark.gpu
@pytest.mark.parametrize("seed", range(64))
def test_random_model_equals_the_oracle(seed):
    w = random_model(seed)
    nv = int(np.prod(w["dims"]))
    lat = psc.lattice_from_workload(w, max_molecules=nv)
    lat.step(w["events"])
    g = lat.read_state()
    s = oracle_state(w)
    disp = w["track_displacement"]
    for key in ("occ", "id", "vox", "species") + (("dx", "dy", "dz") if disp else ()):
        assert np.array_equal(g[key], s[key]), (key, w)
    for key in ("attempts", "hops", "collisions", "place_fail", "event", "next_id"):
        assert g[key] == s[key], (key, g[key], s[key], w)
    assert g["time"] == s["time"]
    assert np.array_equal(g["fired"], s["fired"]), (g["fired"], s["fired"], w)


def test_random_models_are_valid_and_varied():
    # the oracle accepts every drawn model, and the draws cover both lattices,
    # both boundaries, many-product collisions and first-order reactions
    kinds = set()
    for seed in range(96):
        w = random_model(seed)
        s = oracle_state(w)
        assert s["attempts"] > 0
        kinds.add(("fcc" if w.get("lattice") else "hcp", w.get("boundary", "periodic")))
        kinds.add(("many", max((len(p) for r, p, k in w["reactions"] if len(r) == 2), default=0) > 2))
        kinds.add(("first", any(len(r) == 1 for r, p, k in w["reactions"])))
    assert {("fcc", "walls"), ("fcc", "periodic"), ("hcp", "walls"), ("hcp", "periodic"),
            ("many", True), ("first", True)} <= kinds


@pytest.mark.gpu
def test_random_models_in_one_ensemble():
    """32 further random models (both lattices, both boundaries, every kind of
    reaction) advanced together as one batched ensemble: each member equals
    the oracle."""
    ws = [random_model(seed) for seed in range(64, 96)]
    lats = [psc.lattice_from_workload(w, max_molecules=int(np.prod(w["dims"]))) for w in ws]
    ens = psc.Ensemble(lats)
    ens.step(20)
    ens.sync()
    for w, lat in zip(ws, lats):
        g = lat.read_state()
        s = oracle_state(w)
        disp = w["track_displacement"]
        for key in ("occ", "id", "vox", "species") + (("dx", "dy", "dz") if disp else ()):
            assert np.array_equal(g[key], s[key]), (key, w)
        for key in ("attempts", "hops", "collisions", "place_fail", "event", "next_id"):
            assert g[key] == s[key], (key, g[key], s[key], w)
        assert np.array_equal(g["fired"], s["fired"]), (g["fired"], s["fired"], w)


@pytest.mark.gpu
@pytest.mark.parametrize("seed", range(16))
def test_random_model_checkpoint_and_resume(seed):
    """10 events, the state read and loaded into a fresh lattice, 10 more:
    the same as the oracle's 20 events (the resumed lattice's counters start
    at the load, so the state, event, next id and time are compared)."""
    w = random_model(seed)
    nv = int(np.prod(w["dims"]))
    first = psc.lattice_from_workload(w, max_molecules=nv)
    first.step(10)
    mid = first.read_state()
    first.close()
    second = psc.lattice_from_workload(w, max_molecules=nv, place=False)
    second.load_state(mid)
    second.step(10)
    g = second.read_state()
    s = oracle_state(w)
    disp = w["track_displacement"]
    for key in ("occ", "id", "vox", "species") + (("dx", "dy", "dz") if disp else ()):
        assert np.array_equal(g[key], s[key]), (key, w)
    assert g["event"] == s["event"] and g["next_id"] == s["next_id"] and g["time"] == s["time"]
