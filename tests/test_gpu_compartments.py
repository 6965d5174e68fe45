"""Interior compartments on the GPU (through the C ABI) against the CPU
oracle, bit for bit: a cell-like map (cytosol, a membrane shell, a nucleus)
with every rule on both lattices, both boundaries, both layouts and several
launch shapes; slabs whose faces wrap around the periodic box; a sub-box
compartment against the same box closed by walls, on the GPU alone; members
with and without compartments in one batched ensemble."""
import numpy as np
import pytest

import oracle
from paper_1605_03726_amd import psc
from psc_inputs import layered_map, membrane, sub_box_map, workload

pytestmark = pytest.mark.gpu


def build_oracle(w):
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"],
                      boundary=oracle.REFLECT if w.get("boundary") == "walls" else oracle.PERIODIC,
                      lattice=oracle.FCC if w.get("lattice") == "fcc" else oracle.HCP)
    for _, D in w["species"]:
        o.add_species(D)
    for r, p, k in w["reactions"]:
        o.add_reaction(r, p, k)
    if w.get("compartments") is not None:
        o.set_compartments(w["compartments"])
    for s, c in w["place"]:
        o.place_uniform(s, c)
    for s, c, cc in w.get("place_in", []):
        o.place_uniform_in(s, c, cc)
    return o


def assert_same(g, o, disp=True):
    for key in ("occ", "id", "vox", "species") + (("dx", "dy", "dz") if disp else ()):
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


def run_pair(w, events, chunks=2, linear=False, items=0):
    lat = psc.lattice_from_workload(w, linear_layout=linear)
    if items:
        lat.set_launch(items_per_thread=items)
    o = build_oracle(w)
    per = events // chunks
    for c in range(chunks):
        lat.step(per if c < chunks - 1 else events - per * (chunks - 1))
    g = lat.read_state()
    o.run(events, oracle.MODE_C)
    s = o.state()
    assert_same(g, s, disp=w.get("track_displacement", False))
    lat.close()
    return g, s


@pytest.mark.parametrize("lattice,dims", [("hcp", (24, 24, 24)), ("hcp", (32, 20, 28)),
                                          ("fcc", (24, 24, 24)), ("fcc", (16, 32, 36))])
@pytest.mark.parametrize("boundary", [None, "walls"])
def test_membrane_cell_all_rules(lattice, dims, boundary):
    w = membrane(dims=dims, seed=13, lattice=lattice, boundary=boundary, events=60)
    g, s = run_pair(w, 60)
    comp = w["compartments"]
    assert s["fired"].sum() > 50 and s["place_fail"] >= 0
    # molecules of each kind where they belong
    assert np.all(comp[g["vox"][g["species"] == 4]] == 1)


@pytest.mark.parametrize("linear,items", [(True, 0), (False, 1), (False, 16)])
def test_membrane_layouts_and_launch_shapes(linear, items):
    w = membrane(dims=(28, 24, 20), seed=17, events=50)
    run_pair(w, 50, chunks=3, linear=linear, items=items)


@pytest.mark.parametrize("lattice", ["hcp", "fcc"])
def test_slabs_across_the_periodic_wrap(lattice):
    dims = (16, 16, 24)
    w = membrane(dims=dims, seed=19, lattice=lattice, events=40)
    w = dict(w, compartments=layered_map(dims, 4),
             place_in=[(1, 150, 0), (2, 150, 1), (4, 80, 2), (1, 120, 3), (2, 100, 3),
                       (5, 60, 1)])
    run_pair(w, 40)


@pytest.mark.parametrize("lattice,small", [("hcp", (16, 12, 8)), ("fcc", (16, 8, 12))])
def test_sub_box_compartment_equals_walls_on_the_gpu(lattice, small):
    big = tuple(2 * x for x in small)
    net = workload("small_reactive", dims=small, seed=23, events=60)
    net = dict(net, reactions=net["reactions"] + [((3, 5), (5, 3, 2, 2), 3e-20)])
    if lattice == "fcc":
        net["lattice"] = "fcc"
    walled = psc.lattice_from_workload(dict(net, boundary="walls"))
    s0 = walled.read_state()
    ni, nj, _ = small
    i, j, k = s0["vox"] % ni, (s0["vox"] // ni) % nj, s0["vox"] // (ni * nj)
    vbig = i + big[0] * (j + big[1] * k)
    occ = np.zeros(int(np.prod(big)), np.uint16)
    occ[vbig] = s0["species"]
    boxed = psc.lattice_from_workload(dict(net, dims=big, compartments=sub_box_map(big, small)),
                                      place=False)
    boxed.load_state(dict(occ=occ, id=s0["id"], vox=vbig, species=s0["species"],
                          dx=s0["dx"], dy=s0["dy"], dz=s0["dz"], next_id=s0["next_id"]))
    walled.step(60)
    boxed.step(60)
    a, b = walled.read_state(), boxed.read_state()
    for key in ("id", "species", "dx", "dy", "dz"):
        assert np.array_equal(a[key], b[key]), key
    for key in ("attempts", "hops", "collisions", "place_fail", "next_id"):
        assert a[key] == b[key], key
    assert np.array_equal(a["fired"], b["fired"])
    ai, aj, ak = a["vox"] % ni, (a["vox"] // ni) % nj, a["vox"] // (ni * nj)
    assert np.array_equal(b["vox"], ai + big[0] * (aj + big[1] * ak))
    walled.close()
    boxed.close()


def test_ensemble_members_with_and_without_compartments():
    ws = [membrane(dims=(20, 20, 20), seed=29 + a, events=30) for a in range(3)]
    ws += [dict(workload("small_reactive", dims=(16, 12, 8), seed=31), events=30)]
    ws += [membrane(dims=(24, 24, 24), seed=41, lattice="fcc", boundary="walls", events=30)]
    lats = [psc.lattice_from_workload(w) for w in ws]
    ens = psc.Ensemble(lats)
    ens.step(30)
    ens.sync()
    for w, lat in zip(ws, lats):
        o = build_oracle(w)
        o.run(30, oracle.MODE_C)
        assert_same(lat.read_state(), o.state(), disp=w.get("track_displacement", False))
    ens.close()
