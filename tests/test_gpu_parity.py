"""GPU path (through the C ABI) against the CPU oracle's coloured-stage mode:
bit-exact occupancy, molecule table (id, voxel, species, displacement),
counters, fired reactions, event index, time and next id.

Sizes span several workgroups and ragged bin tails; the full-size workloads
run a prefix of their events (the oracle is single-threaded)."""
import numpy as np
import pytest

import oracle
from paper_1605_03726_amd import psc
from psc_inputs import random_state, workload

pytestmark = pytest.mark.gpu


def build_oracle(w, state=None):
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"],
                      boundary=oracle.REFLECT if w.get("boundary") == "walls" else oracle.PERIODIC,
                      lattice=oracle.FCC if w.get("lattice") == "fcc" else oracle.HCP)
    for _, D in w["species"]:
        o.add_species(D)
    for r, p, k in w["reactions"]:
        o.add_reaction(r, p, k)
    if state is None:
        for s, c in w["place"]:
            o.place_uniform(s, c)
    else:
        o.load(state["occ"], state["id"], state["vox"],
               (state["dx"], state["dy"], state["dz"]), state.get("event", 0), state["next_id"])
    return o


def build_gpu(w, state=None, max_molecules=None):
    lat = psc.lattice_from_workload(w, max_molecules=max_molecules, place=state is None)
    if state is not None:
        lat.load_state(state)
    return lat


def assert_same(g, o, disp=True):
    for key in ("occ", "id", "vox", "species") + (("dx", "dy", "dz") if disp else ()):
        if g[key] is None and o[key] is None:
            continue
        if not np.array_equal(g[key], o[key]):
            a, b = g[key], o[key]
            n = min(len(a), len(b))
            bad = np.nonzero(a[:n] != b[:n])[0]
            raise AssertionError(f"{key}: lengths {len(a)} vs {len(b)}, first mismatches "
                                 f"{bad[:5]} gpu {a[bad[:5]]} oracle {b[bad[:5]]}")
    for key in ("attempts", "hops", "collisions", "place_fail", "event", "next_id"):
        assert g[key] == o[key], (key, g[key], o[key])
    assert g["time"] == o["time"]
    assert np.array_equal(g["fired"], o["fired"]), (g["fired"], o["fired"])


def run_pair(w, events, state=None, chunks=1, max_molecules=None):
    lat = build_gpu(w, state, max_molecules)
    o = build_oracle(w, state)
    per = events // chunks
    for c in range(chunks):
        n = per if c < chunks - 1 else events - per * (chunks - 1)
        lat.step(n)
    g = lat.read_state()
    o.run(events, oracle.MODE_C)
    s = o.state()
    assert_same(g, s, disp=w.get("track_displacement", False))
    return g, s


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_small_reactive_all_rules(seed):
    w = workload("small_reactive", seed=seed)
    g, s = run_pair(w, 40)
    assert s["hops"] > 0 and s["collisions"] > 0 and np.all(s["fired"] > 0), s["fired"]


@pytest.mark.parametrize("dims", [(4, 4, 4), (4, 8, 12), (12, 8, 16), (20, 4, 8)])
def test_small_reactive_shapes(dims):
    w = workload("small_reactive", dims=dims, seed=11)
    run_pair(w, 30)


def fused_case(case):
    if case == "reactive":
        return workload("small_reactive", seed=7), 60
    if case == "reactive_ragged":
        return workload("small_reactive", dims=(20, 4, 8), seed=12), 60
    if case == "reactive_walls":
        return dict(workload("small_reactive", seed=8), boundary="walls"), 60
    if case == "reactive_fcc":
        return dict(workload("small_reactive", seed=9, dims=(16, 16, 12)), lattice="fcc"), 60
    return workload("cfg1"), 150


@pytest.mark.parametrize("case", ["reactive", "reactive_ragged", "reactive_walls", "reactive_fcc",
                                  "diffusion"])
def test_event_end_fused_with_next_opening(case):
    """A step of many events, once the last event reported few reacted
    partners, runs each event's end in one kernel with the next event's
    opening; a step of one event always ends in its own launch.  Both leave
    the oracle's state."""
    w, events = fused_case(case)
    single = build_gpu(w)
    for _ in range(events):
        single.step(1)
    a = single.read_state()
    fused = build_gpu(w)
    fused.step(1)
    fused.sync()  # the event's counts are on the host before the next step starts
    fused.step(events - 1)
    b = fused.read_state()
    o = build_oracle(w)
    o.run(events, oracle.MODE_C)
    s = o.state()
    disp = w.get("track_displacement", False)
    assert_same(a, s, disp=disp)
    assert_same(b, s, disp=disp)
    assert s["hops"] > 0
    if case != "diffusion":
        assert np.all(s["fired"] > 0), s["fired"]


def test_diffusion_64cubed_full_run():
    w = workload("cfg1")
    g, s = run_pair(w, w["events"], chunks=4)
    assert s["attempts"] == 2621 * 1000


def test_crowded_reaction_scaled():
    w = workload("cfg2", dims=(64, 64, 64), events=300)
    g, s = run_pair(w, 300, chunks=3)
    assert s["fired"][0] > 0


def test_crowded_reaction_full_size_prefix():
    w = workload("cfg2", events=12)
    run_pair(w, 12)


def test_mapk_network_scaled():
    w = workload("cfg3", dims=(128, 128, 64), events=60)
    # faster first-order rates would rarely fire in 60 events at 0.1..10 /s,
    # so the network is run as given and the check is exactness
    run_pair(w, 60)


def test_random_loaded_state_with_id_gaps():
    w = workload("small_reactive", dims=(16, 16, 8), seed=21)
    st = random_state(w["dims"], [(1, 150), (2, 60), (3, 60), (4, 20), (5, 30)], seed=5,
                      event=17)
    run_pair(w, 35, state=st)


def test_checkpoint_resume_is_exact():
    w = workload("small_reactive", seed=31)
    lat = build_gpu(w)
    lat.step(20)
    mid = lat.read_state()
    res = build_gpu(w, state=mid)
    res.step(25)
    g = res.read_state()
    o = build_oracle(w)
    o.run(45, oracle.MODE_C)
    s = o.state()
    for key in ("occ", "id", "vox", "species", "dx", "dy", "dz"):
        assert np.array_equal(g[key], s[key]), key
    assert g["event"] == s["event"] and g["next_id"] == s["next_id"] and g["time"] == s["time"]


def test_deterministic_and_step_split_invariant():
    w = workload("cfg2", dims=(32, 32, 32), events=50)
    a = build_gpu(w)
    a.step(50)
    b = build_gpu(w)
    for _ in range(50):
        b.step(1)
    ga, gb = a.read_state(), b.read_state()
    for key in ("occ", "id", "vox", "species", "attempts", "hops", "collisions"):
        assert np.array_equal(np.asarray(ga[key]), np.asarray(gb[key])), key


def test_empty_lattice():
    w = dict(workload("cfg1"), place=[], events=5)
    g, s = run_pair(w, 5)
    assert len(g["id"]) == 0 and g["attempts"] == 0


def test_full_lattice_has_no_hops():
    dims = (4, 4, 8)
    w = dict(workload("cfg1"), dims=dims, place=[(1, 128)], events=6)
    g, s = run_pair(w, 6)
    assert g["hops"] == 0 and g["collisions"] == g["attempts"] == 128 * 6


def test_partial_probability_and_immobile_reactant():
    # p < 1 exercises the threshold comparison; an immobile reactant with a
    # first-order reaction stays in the bins and is converted in place
    n = 16 * 16 * 16
    w = dict(name="threshold", dims=(16, 16, 16), rv=4.4e-9, seed=13,
             species=[("A", 1e-12), ("E", 0.0), ("C", 2e-12), ("X", 0.0)],
             reactions=[((1, 2), (3,), 3e-20), ((3, 1), (1, 1), 4e-20),
                        ((2,), (4,), 800.0), ((4,), (2, 1), 900.0)],
             place=[(1, n // 8), (2, n // 10), (3, n // 20)], events=40,
             track_displacement=True)
    g, s = run_pair(w, 40)
    assert np.all(s["fired"] > 0), s["fired"]


def test_many_products_and_placement_failures():
    # crowded: first-order reactions with up to 11 products often fail
    n = 8 * 8 * 8
    w = dict(name="many_products", dims=(8, 8, 8), rv=4.4e-9, seed=17,
             species=[("A", 1e-12), ("B", 1e-12), ("O", 0.0)],
             reactions=[((1,), (2,) * 11, 3000.0), ((2,), (1, 1, 1), 2000.0),
                        ((2,), (), 500.0)],
             place=[(3, n // 3), (1, n // 8)], events=30, track_displacement=True)
    g, s = run_pair(w, 30, max_molecules=n)
    assert s["place_fail"] > 0 and s["fired"][0] > 0


@pytest.mark.timeout(1200)
def test_mapk_full_size_prefix(capsys):
    # the 2^32-voxel workload at full size (8 GiB occupancy, 12.9 M molecules)
    # in the benchmark's launch shape, against the oracle after 6 events (the
    # partner marks and flags carried across event parities) and after 60
    # (about 7.7 x 10^8 attempts; a few CPU minutes)
    w = workload("cfg3")
    lat = build_gpu(w, max_molecules=int(0.003 * 2 ** 32 * 1.25))
    o = build_oracle(w)
    done = 0
    for events in (6, 60):
        lat.step(events - done)
        g = lat.read_state()
        while done < events:   # a few seconds per oracle event: report progress
            o.run(6, oracle.MODE_C)
            done += 6
            with capsys.disabled():  # shown even when output is captured
                print("oracle at event %d" % done, flush=True)
        s = o.state()
        assert_same(g, s, disp=False)
        del g, s
    lat.close()
    o.close()


def test_mapk_full_run_invariants():
    """The MAPK workload as the benchmark runs it (2^32 voxels, the default
    launch shape, 10 + 2000 events), checked by what holds at any size: the
    occupancy and the molecule table agree voxel for voxel, the device's
    per-species counts equal the table's, and the three moieties that every
    reaction of the network conserves (MAPK, MAPKK, phosphatase, free or in a
    complex) keep their initial totals."""
    w = workload("cfg3")
    nv = 2 ** 32
    placed = sum(c for _, c in w["place"])
    lat = build_gpu(w, max_molecules=min(nv, int(placed * 1.25) + 4096))
    lat.step(10)
    lat.step(2000)
    st = lat.stats()
    g = lat.read_state()
    lat.close()
    occ, vox, sp = g["occ"], g["vox"], g["species"]
    assert g["event"] == 2010 and g["attempts"] > 2 * 10 ** 10
    # complexes form and break up (some of the rarer pairs never meet in 2000
    # events)
    assert g["fired"][0] > 10 ** 6 and np.count_nonzero(g["fired"]) >= 10, g["fired"]
    assert len(np.unique(vox)) == len(vox)
    assert np.array_equal(occ[vox], sp)
    assert np.count_nonzero(occ) == len(vox)
    counts = np.bincount(sp, minlength=11)
    assert np.array_equal(counts[1:11], st["species_count"][1:11].astype(np.int64))
    names = [n for n, _ in w["species"]]
    moieties = {"K": 0, "KK": 0, "P": 0}
    for i, name in enumerate(names, start=1):
        for part in name.split("."):
            moieties[part.rstrip("p") or part] += int(counts[i])
    start = dict(w["place"])
    assert moieties == {"K": start[1], "KK": start[4], "P": start[5]}, moieties


@pytest.mark.parametrize("name,kw,events", [("small_reactive", {"seed": 4}, 40),
                                            ("cfg2", {"dims": (32, 32, 32)}, 60)])
def test_device_statistics(name, kw, events):
    # per-species counts kept on the device through every reaction, and the
    # displacement sum behind the mean squared displacement
    w = workload(name, **kw)
    lat = build_gpu(w)
    lat.step(events)
    st = lat.stats()
    g = lat.read_state()
    o = build_oracle(w)
    o.run(events, oracle.MODE_C)
    s = o.state()
    for sp in range(1, len(w["species"]) + 1):
        assert st["species_count"][sp] == int((s["species"] == sp).sum()) == o.species_count(sp)
    if w.get("track_displacement"):
        X, Y, Z = (s[k].astype(np.int64) for k in ("dx", "dy", "dz"))
        assert st["disp_sum"] == int((3 * X * X + Y * Y + 8 * Z * Z).sum())
    assert np.array_equal(g["species"], s["species"])


def test_paper_mapk_model_prefix():
    # the paper's own MAPK model (9 species, 12 reactions, 480^3, r_v 10 nm)
    w = workload("mapk_paper", events=40)
    g, s = run_pair(w, 40, chunks=2)
    assert s["collisions"] > 0


@pytest.mark.parametrize("name,kw,events", [("small_reactive", {"seed": 12}, 40),
                                            ("cfg2", {"dims": (64, 64, 64)}, 80),
                                            ("cfg3", {"dims": (128, 128, 64)}, 40)])
def test_linear_layout_gives_the_same_result(name, kw, events):
    # the occupancy layout (4x4x4 bricks by default, or linear) changes
    # addresses only
    w = workload(name, **kw)
    lat = psc.lattice_from_workload(w, linear_layout=True)
    lat.step(events)
    g = lat.read_state()
    o = build_oracle(w)
    o.run(events, oracle.MODE_C)
    assert_same(g, o.state(), disp=w.get("track_displacement", False))


@pytest.mark.parametrize("items", [1, 4, 16])
def test_launch_shapes_on_a_reactive_lattice(items):
    """Items per thread select different kernel instances (16 items per
    thread exceed the register file and spill); every shape must equal the
    oracle over many reactive events."""
    w = workload("cfg2", dims=(128, 128, 128))
    lat = build_gpu(w, max_molecules=1 << 20)
    lat.set_launch(items, 64)
    o = build_oracle(w)
    lat.step(60)
    o.run(60, oracle.MODE_C)
    s = o.state()
    assert_same(lat.read_state(), s, disp=False)
    assert s["fired"][0] > 1000


# ---- boxes closed by walls (PSC_BOUNDARY_WALLS) --------------------------------

@pytest.mark.parametrize("seed", [7, 8, 9])
def test_walls_small_reactive_all_rules(seed):
    """Every rule next to walls: a 16 x 12 x 8 box has most voxels on or near a
    face, so hops, collisions and first-order product placement all meet them."""
    w = dict(workload("small_reactive", seed=seed), boundary="walls")
    g, s = run_pair(w, 40)
    assert s["hops"] > 0 and s["collisions"] > 0 and np.all(s["fired"] > 0), s["fired"]
    # the walls change the run
    gp = build_gpu(dict(w, boundary=None))
    gp.step(40)
    assert not np.array_equal(gp.read_state()["occ"], g["occ"])


@pytest.mark.parametrize("dims", [(4, 4, 4), (20, 4, 8)])
def test_walls_shapes(dims):
    w = dict(workload("small_reactive", dims=dims, seed=11), boundary="walls")
    run_pair(w, 30)


def test_walls_displacement_and_crowding():
    w = dict(workload("cfg1", events=200), dims=(32, 32, 32), place=[(1, 3000)],
             boundary="walls")
    g, s = run_pair(w, 200)
    assert s["hops"] > 100000
    w = dict(workload("cfg2", dims=(64, 64, 64)), boundary="walls")
    run_pair(w, 120)


@pytest.mark.parametrize("items", [1, 4])
def test_walls_launch_shapes(items):
    w = dict(workload("cfg2", dims=(64, 64, 64)), boundary="walls")
    lat = build_gpu(w)
    lat.set_launch(items, 16)
    o = build_oracle(w)
    lat.step(60)
    o.run(60, oracle.MODE_C)
    assert_same(lat.read_state(), o.state(), disp=False)


# ---- collisions with more than two products --------------------------------------

@pytest.mark.parametrize("seed,boundary", [(3, None), (4, "walls"), (5, None)])
def test_multiproduct_collisions(seed, boundary):
    w = workload("multiproduct", seed=seed, boundary=boundary, n_a=16 * 12 * 8 // 5)
    g, s = run_pair(w, 40)
    assert s["fired"][0] > 0 and s["fired"][1] > 0 and s["place_fail"] > 0, (s["fired"], s["place_fail"])


def test_first_order_decisions_over_workgroups():
    """Events with many first-order candidates (here ~10 k: a fast decay on
    ~80 k walkers) take their decisions in a launch of many workgroups
    instead of inside the one-workgroup first-order pass; the result is the
    oracle's either way, over event splits and launch shapes."""
    w = workload("multiproduct", dims=(96, 96, 64), seed=9, n_a=40000)
    g, s = run_pair(w, 30, chunks=3)
    assert s["fired"][2] > 20000, s["fired"]       # C -> 0 fired a lot
    lat = build_gpu(w)
    lat.set_launch(1, 33)
    lat.step(30)
    assert_same(lat.read_state(), s)


@pytest.mark.parametrize("events", [1, 6])
def test_more_newborns_per_event_than_the_lds_numbering_holds(events):
    """Newborn ids come from the rank of each birth key among the event's keys,
    counted in LDS up to 2048 newborns; beyond that the keys are sorted in
    global memory.  Here both kinds of births pass 2048 in every event:
    A -> A + C (a fast decay: ~2.7 k first-order newborns) and
    A + B -> A + B + C with p = 1 at 15 % occupancy of B (~3.6 k collision
    newborns)."""
    w = dict(name="births", dims=(64, 64, 64), rv=4.4e-9, seed=5,
             species=[("A", 1e-12), ("B", 1e-12), ("C", 0.0)],
             reactions=[((1,), (1, 3), 20000.0), ((1, 2), (1, 2, 3), 1e-15)],
             place=[(1, 12000), (2, 40000)], events=events, track_displacement=True)
    lat = build_gpu(w, max_molecules=64 ** 3)
    o = build_oracle(w)
    lat.step(events)
    o.run(events, oracle.MODE_C)
    s = o.state()
    assert_same(lat.read_state(), s)
    assert s["fired"][0] > 2048 * events and s["fired"][1] > 2048 * events, s["fired"]


def test_many_newborns_numbered_in_one_workgroup_in_an_ensemble():
    """The batched kernels number every member's newborns in the member's
    one workgroup (a sort in global memory beyond the LDS ranking): the
    births workload above as a one-member ensemble equals the oracle too."""
    w = dict(name="births", dims=(64, 64, 64), rv=4.4e-9, seed=6,
             species=[("A", 1e-12), ("B", 1e-12), ("C", 0.0)],
             reactions=[((1,), (1, 3), 20000.0), ((1, 2), (1, 2, 3), 1e-15)],
             place=[(1, 12000), (2, 40000)], events=4, track_displacement=True)
    lat = build_gpu(w, max_molecules=64 ** 3)
    ens = psc.Ensemble([lat])
    ens.step(4)
    o = build_oracle(w)
    o.run(4, oracle.MODE_C)
    s = o.state()
    assert_same(ens.read(0), s)
    assert s["fired"][0] > 2048 * 4 and s["fired"][1] > 2048 * 4, s["fired"]
    ens.close()


@pytest.mark.timeout(600)
def test_tens_of_thousands_of_newborns_per_event():
    """~20 k first-order and ~14 k collision newborns per event, numbered by
    launches over the whole GPU."""
    w = dict(name="births", dims=(128, 128, 128), rv=4.4e-9, seed=8,
             species=[("A", 1e-12), ("B", 1e-12), ("C", 0.0)],
             reactions=[((1,), (1, 3), 20000.0), ((1, 2), (1, 2, 3), 1e-15)],
             place=[(1, 90000), (2, 150000)], events=3, track_displacement=False)
    lat = build_gpu(w, max_molecules=128 ** 3)
    o = build_oracle(w)
    lat.step(3)
    o.run(3, oracle.MODE_C)
    s = o.state()
    assert_same(lat.read_state(), s, disp=False)
    assert s["fired"][0] > 15000 * 3 and s["fired"][1] > 10000 * 3, s["fired"]


@pytest.mark.parametrize("kind", ["hcp", "fcc_walls"])
def test_first_order_firings_per_event_crossing_one_workgroup(kind):
    """The first-order pass applies an event's firings one per thread when
    they fit in its workgroup (1024) and loops over them otherwise.  A dense
    decaying population (23-24 % occupancy; A -> 0 and A -> C + C) fires
    ~1,900 times in the first event and ~300 in the last, so the run crosses
    from one form to the other, with many firings deferred for touching
    neighbourhoods and products placed among them; also on the FCC lattice
    in a box closed by walls (neighbourhoods cut by the walls)."""
    dims = (64, 64, 64) if kind == "hcp" else (64, 64, 60)
    w = dict(name="fire_sweep", dims=dims, rv=4.4e-9, seed=9,
             species=[("A", 1e-12), ("C", 0.0)],
             reactions=[((1,), (), 1300.0), ((1,), (2, 2), 1300.0)],
             place=[(1, 60000)], events=60, track_displacement=True)
    if kind == "fcc_walls":
        w = fcc(w, boundary="walls")
    lat = build_gpu(w, max_molecules=dims[0] * dims[1] * dims[2])
    o = build_oracle(w)
    per, prev = [], 0
    for chunk in (1, 4, 15, 20, 20):
        for _ in range(chunk):
            o.run(1, oracle.MODE_C)
            f = int(sum(o.state(with_occ=False)["fired"]))
            per.append(f - prev)
            prev = f
        lat.step(chunk)
        assert_same(lat.read_state(), o.state())
    assert max(per) > 1024 and min(per) < 512, per


def test_multiproduct_collisions_many_events_and_shapes():
    w = workload("multiproduct", dims=(48, 48, 32), seed=6, n_a=6000)
    nv = 48 * 48 * 32
    lat = build_gpu(w, max_molecules=nv)
    o = build_oracle(w)
    for n in (1, 30, 90):
        lat.step(n)
        o.run(n, oracle.MODE_C)
        assert_same(lat.read_state(), o.state())
    staged = build_gpu(w, max_molecules=nv)
    staged.set_launch(1, 7)
    staged.step(121)
    assert_same(staged.read_state(), o.state())


# ---- the face-centred cubic lattice (PSC_LATTICE_FCC) ------------------------------

def fcc(w, **kw):
    return dict(w, lattice="fcc", **kw)


@pytest.mark.parametrize("seed", [7, 8])
def test_fcc_small_reactive_all_rules(seed):
    """Every rule on the FCC lattice; 16 x 16 x 12 spans several chunks per
    stage and ragged bin tails."""
    w = fcc(workload("small_reactive", seed=seed, dims=(16, 16, 12)))
    g, s = run_pair(w, 40)
    assert s["hops"] > 0 and s["collisions"] > 0 and np.all(s["fired"] > 0), s["fired"]
    # the lattice changes the run
    gh = build_gpu(dict(w, lattice=None))
    gh.step(40)
    assert not np.array_equal(gh.read_state()["occ"], g["occ"])


@pytest.mark.parametrize("dims,boundary", [((8, 8, 12), None), ((24, 8, 24), None),
                                           ((8, 8, 12), "walls"), ((24, 8, 24), "walls")])
def test_fcc_shapes(dims, boundary):
    w = fcc(workload("small_reactive", dims=dims, seed=11), boundary=boundary)
    run_pair(w, 30)


def test_fcc_displacement_and_crowding():
    w = fcc(dict(workload("cfg1", events=200), dims=(32, 32, 36), place=[(1, 3000)]))
    g, s = run_pair(w, 200)
    assert s["hops"] > 100000
    run_pair(fcc(workload("cfg2", dims=(64, 64, 48))), 120)
    run_pair(fcc(workload("cfg2", dims=(64, 64, 48)), boundary="walls"), 60)


@pytest.mark.parametrize("items", [1, 4, 16])
def test_fcc_launch_shapes(items):
    w = fcc(workload("cfg2", dims=(96, 96, 96)))
    lat = build_gpu(w, max_molecules=1 << 19)
    lat.set_launch(items, 64)
    o = build_oracle(w)
    lat.step(60)
    o.run(60, oracle.MODE_C)
    s = o.state()
    assert_same(lat.read_state(), s, disp=False)
    assert s["fired"][0] > 500


@pytest.mark.parametrize("boundary", [None, "walls"])
def test_fcc_multiproduct_and_mapk(boundary):
    w = fcc(workload("multiproduct", seed=3, dims=(16, 16, 12), n_a=16 * 16 * 12 // 5),
            boundary=boundary)
    g, s = run_pair(w, 40)
    assert s["fired"][0] > 0 and s["fired"][1] > 0
    run_pair(fcc(workload("cfg3", dims=(64, 64, 48)), boundary=boundary), 40, chunks=2)


def test_fcc_linear_layout_statistics_and_checkpoint():
    w = fcc(workload("small_reactive", seed=21, dims=(16, 8, 24)))
    lat = psc.lattice_from_workload(w, linear_layout=True)
    lat.step(25)
    mid = lat.read_state()
    lat.step(15)
    st = lat.stats()
    g = lat.read_state()
    o = build_oracle(w)
    o.run(40, oracle.MODE_C)
    s = o.state()
    assert_same(g, s)
    for sp in range(1, len(w["species"]) + 1):
        assert st["species_count"][sp] == int((s["species"] == sp).sum())
    X, Y, Z = (s[k].astype(np.int64) for k in ("dx", "dy", "dz"))
    assert st["disp_sum"] == int((3 * X * X + Y * Y + 8 * Z * Z).sum())
    # resume from the event-25 state on a fresh lattice (its counters start at
    # the load, so the state, event, next id and time are compared)
    r = build_gpu(w, state=mid)
    r.step(15)
    gr = r.read_state()
    for key in ("occ", "id", "vox", "species", "dx", "dy", "dz"):
        assert np.array_equal(gr[key], s[key]), key
    assert gr["event"] == s["event"] and gr["next_id"] == s["next_id"] and gr["time"] == s["time"]


@pytest.mark.timeout(900)
def test_fcc_full_size_prefix():
    # the MAPK workload on an FCC lattice of 2048 x 2048 x 1020 voxels (just
    # under 2^32; nk a multiple of 12), six events
    events = 6
    w = fcc(workload("cfg3", dims=(2048, 2048, 1020)))
    lat = build_gpu(w, max_molecules=int(0.003 * 2 ** 32 * 1.25))
    lat.step(events)
    g = lat.read_state()
    lat.close()
    o = build_oracle(w)
    o.run(events, oracle.MODE_C)
    s = o.state()
    o.close()
    assert_same(g, s, disp=False)


@pytest.mark.parametrize("fcc", [False, True])
def test_msd_is_6Dt_at_scale(fcc):
    """The paper's diffusion check (3.1, eq. 7) on the GPU at a size the
    oracle does not reach: 10 k walkers at 0.5 % occupancy on 128^3 voxels,
    400 events; the mean squared displacement from the device's own
    displacement sum, r^2 sum(3X^2 + Y^2 + 8Z^2) / (3n), grows as
    6 D t = 4 r^2 N (N events), within 3 %, and linearly in time."""
    dims = (128, 128, 120) if fcc else (128, 128, 128)
    nv = dims[0] * dims[1] * dims[2]
    w = dict(name="msd", dims=dims, rv=4.4e-9, seed=17, species=[("A", 1e-12)], reactions=[],
             place=[(1, nv // 200)], events=400, track_displacement=True)
    if fcc:
        w["lattice"] = "fcc"
    lat = build_gpu(w)
    ratios = []
    for n in (200, 400):
        lat.step(n - (200 if n == 400 else 0))
        st = lat.stats()
        msd_r2 = st["disp_sum"] / (3.0 * st["n_walkers"])
        ratios.append(msd_r2 / (4.0 * n))
    assert all(abs(r - 1.0) < 0.03 for r in ratios), ratios
    assert abs(ratios[0] - ratios[1]) < 0.02, ratios


@pytest.mark.parametrize("k", [0.135, 1.35, 13.5])
def test_first_order_decay_closed_form_at_scale(k):
    """The paper's first-order check (3.2.1) with its 64,000 molecules and
    rate constants: immobile A -> B + C, the event interval set by one fast
    walker (2000 events up to t = 2/k); the device's count of A follows
    A0 exp(-k t) within 2 % at t = 1/k and 2/k (binomial spread ~0.5 %)."""
    rv, n0, events = 5e-9, 64000, 2000
    tau = 2.0 / k / events
    dz = 2.0 * rv * rv / (3.0 * tau)
    w = dict(name="decay", dims=(128, 128, 128), rv=rv, seed=23,
             species=[("Z", dz), ("A", 0.0), ("B", 0.0), ("C", 0.0)],
             reactions=[((2,), (3, 4), k)], place=[(1, 1), (2, n0)], events=events)
    lat = build_gpu(w, max_molecules=3 * n0 + 1024)
    for half in (1, 2):
        lat.step(events // 2)
        a = int(lat.stats()["species_count"][2])
        expect = n0 * np.exp(-float(half))
        assert abs(a / expect - 1.0) < 0.02, (k, half, a, expect)
    assert lat.read_state(with_occ=False)["place_fail"] == 0


def test_second_order_reaction_limited_rate_at_scale():
    """The paper's second-order check (3.2.2) in the reaction-limited regime
    (k_f = 0.027 1/(nM s), D = 10 um^2/s, r = 5 nm: p = 0.053) with 20,000
    molecules each of A and B on 128^3 voxels: 1/N_A(t) - 1/N_0 grows as
    k_eff t / V, and k_eff / k = 1 / (1 + p (G(0) - 1)) = 0.982 for the
    lattice walk (Collins-Kimball on the lattice, G(0) = 1.345), within 3 %."""
    kf = 0.027 * 1e9 * 1e-3 / 6.02214076e23
    rv, D, n0, dims = 5e-9, 10e-12, 20000, (128, 128, 128)
    p = kf / (6 * np.sqrt(2) * 2 * D * rv)
    w = dict(name="second_order", dims=dims, rv=rv, seed=29,
             species=[("A", D), ("B", D), ("C", D)], reactions=[((1, 2), (3,), kf)],
             place=[(1, n0), (2, n0)], events=2000)
    lat = build_gpu(w)
    tau = 2.0 * rv * rv / (3.0 * D)
    ts, inv = [], []
    for c in range(20):
        lat.step(100)
        ts.append((c + 1) * 100 * tau)
        inv.append(1.0 / float(lat.stats()["species_count"][1]) - 1.0 / n0)
    ts, inv = np.array(ts), np.array(inv)
    V = np.prod(dims) * 4.0 * np.sqrt(2.0) * rv ** 3
    ratio = float((inv * ts).sum() / (ts * ts).sum()) * V / kf
    expect = 1.0 / (1.0 + p * (1.345 - 1.0))
    assert abs(ratio / expect - 1.0) < 0.03, (ratio, expect)


def reversible_workload(dims, n0, kf, kb, seed, events):
    """B + C <-> A (3.2.2): D = 10 um^2/s, r = 5 nm, A alone at the start"""
    return dict(name="reversible", dims=dims, rv=5e-9, seed=seed,
                species=[("A", 10e-12), ("B", 10e-12), ("C", 10e-12)],
                reactions=[((2, 3), (1,), kf), ((1,), (2, 3), kb)],
                place=[(1, n0)], events=events)


def test_reversible_reaction_equals_the_oracle():
    """B + C <-> A on 48^3 voxels from 4,000 A over 150 events, rates set
    (k_b tau = 1/600) so that about 950 A dissociate and, as B and C build
    up, a few dozen pairs associate."""
    rv, D, dims, n0 = 5e-9, 10e-12, (48, 48, 48), 4000
    V = dims[0] * dims[1] * dims[2] * 4.0 * np.sqrt(2.0) * rv ** 3
    kb = 3.0 * D / (2.0 * rv * rv) / 600.0
    w = reversible_workload(dims, n0, kb * V / (n0 / 2), kb, 43, 150)
    g, s = run_pair(w, 150, chunks=3, max_molecules=2 * n0 + 1024)
    assert s["fired"][0] > 20 and s["fired"][1] > 500, s["fired"]


@pytest.mark.timeout(600)
def test_reversible_reaction_equilibrium_at_scale():
    """The reversible check of 3.2.2 at the paper's parameters (k_f = 0.027
    1/(nM s), k_b = 1.35 1/s, D = 10 um^2/s, r = 5 nm, 64,000 A to start:
    the text's 0, 0, 64,000 for A, B, C cannot react, its figure's caption
    has A dissociating) on an eighth of its 1000 x 960 x 1100 lattice
    (500 x 480 x 552) with both rate constants times 4 (p = 0.21), so that
    the relaxation takes about 12,000 events instead of a few hundred
    thousand.  The equilibrium is where the mean fluxes balance,
    k_f <N_B N_C> / V = k_b <N_A>, which this volume puts at about 51,800 A
    and 12,200 B and C.  After 60,000 events (5 relaxation times) the means
    over 40,000 more meet it within 3 % (spread about 1 %)."""
    rv, D, dims, n0 = 5e-9, 10e-12, (500, 480, 552), 64000
    kf = 4 * 0.027 * 1e9 * 1e-3 / 6.02214076e23
    kb = 4 * 1.35
    V = dims[0] * dims[1] * dims[2] * 4.0 * np.sqrt(2.0) * rv ** 3
    p = kf / (6.0 * np.sqrt(2.0) * 2.0 * D * rv)
    assert 0.2 < p < 0.22
    w = reversible_workload(dims, n0, kf, kb, 47, 100000)
    lat = build_gpu(w, max_molecules=2 * n0 + 4096)
    lat.step(60000)
    na, nbc = [], []
    for _ in range(40):
        lat.step(1000)
        c = lat.stats()["species_count"].astype(np.float64)
        assert c[2] == c[3] and c[1] + c[2] == n0
        na.append(c[1])
        nbc.append(c[2] * c[3])
    ratio = kf * np.mean(nbc) / (V * kb * np.mean(na))
    x = kf / (V * kb)
    b_eq = (-1.0 + np.sqrt(1.0 + 4.0 * x * n0)) / (2.0 * x)
    print("reversible: mean A %.0f (mass action %.0f), flux ratio %.4f"
          % (np.mean(na), n0 - b_eq, ratio), flush=True)
    assert abs(ratio - 1.0) < 0.03, ratio
    lat.close()


def test_launch_shapes_follow_recent_counts_as_firings_grow():
    """Launch shapes for an event come partly from the counts of the last
    event of the previous step (first-order firings and newborns).  An
    autocatalytic A -> A + A on 64^3 (k tau = 0.5: about 40 % of the A fire
    per event) starts with 300 A among 20,000 inert walkers B: the
    candidates expected from the walkers call for the first-order launches
    over the GPU, but the first steps see few firings and drop them; the
    A then grow within one step to thousands of firings and newborns per
    event (past one workgroup's threads and its LDS ranking), handled by the
    one-workgroup path, before the last step takes the launches again.
    Stepped in chunks of 1, 1, 2, 8 and 2 events, against the oracle."""
    rv, D = 4.4e-9, 1e-12
    tau = 2.0 * rv * rv / (3.0 * D)
    w = dict(name="growth", dims=(64, 64, 64), rv=rv, seed=53,
             species=[("A", D), ("B", D)],
             reactions=[((1,), (1, 1), 0.5 / tau)],
             place=[(1, 300), (2, 20000)], events=14, track_displacement=True)
    lat = build_gpu(w, max_molecules=64 ** 3)
    o = build_oracle(w)
    done = 0
    for n in (1, 1, 2, 8, 2):
        lat.step(n)
        done += n
    o.run(done, oracle.MODE_C)
    s = o.state()
    assert_same(lat.read_state(), s)
    n_a = int(np.count_nonzero(s["species"] == 1))
    assert n_a > 10000 and s["fired"][0] > 10000, (n_a, s["fired"])
