"""C-ABI checks that need no GPU: the library loads and exports every entry
point include/psc.h declares; argument validation; the host-side initial
state (uniform placement, load_state, read-back before the first step)
matches the oracle bit for bit."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_1605_03726_amd import psc
from psc_inputs import random_state, workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:psc_status|void|const char \*)\s*\**\s*(psc_\w+)\s*\(",
                            text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_entry_point():
    names = declared_functions()
    assert len(names) >= 12
    lib = psc.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("dims", [(6, 8, 8), (4, 4, 2), (0, 8, 8), (8, 8, 10)])
def test_create_rejects_bad_dimensions(dims):
    with pytest.raises(psc.PscError) as e:
        psc.Lattice(dims, 4.4e-9, 1, 16, torch_allocator=False)
    assert e.value.code == psc.PSC_EINVAL


def test_create_rejects_bad_radius_and_capacity():
    for rv, cap in ((0.0, 10), (-1.0, 10), (4.4e-9, 0), (4.4e-9, 65)):
        with pytest.raises(psc.PscError):
            psc.Lattice((4, 4, 4), rv, 1, cap, torch_allocator=False)


def new(dims=(8, 8, 8), cap=512, seed=1):
    return psc.Lattice(dims, 4.4e-9, seed, cap, track_displacement=True, torch_allocator=False)


def test_model_validation():
    lat = new()
    a = lat.add_species("A", 1e-12)
    b = lat.add_species("B", 0.0)
    o = lat.add_species("O", 0.0)
    with pytest.raises(psc.PscError):
        lat.add_species("bad", -1.0)
    with pytest.raises(psc.PscError):
        lat.add_species("nan", float("nan"))
    lat.add_reaction((a, b), (a,), 1e-18)
    with pytest.raises(psc.PscError):
        lat.add_reaction((b, a), (b,), 1e-18)        # same unordered pair
    with pytest.raises(psc.PscError):
        lat.add_reaction((b, o), (b,), 1e-18)        # two immobile reactants
    with pytest.raises(psc.PscError):
        lat.add_reaction((a, a), (), 1e-18)          # second order needs products
    with pytest.raises(psc.PscError):
        lat.add_reaction((a,), tuple([a] * 12), 1.0)  # more than 11 products
    with pytest.raises(psc.PscError):
        lat.add_reaction((a,), (9,), 1.0)            # unknown species
    with pytest.raises(psc.PscError):
        lat.add_reaction((a,), (b,), -1.0)


def test_species_limit():
    lat = new()
    for s in range(63):
        lat.add_species("s%d" % s, 1e-12)
    with pytest.raises(psc.PscError):
        lat.add_species("too many", 1e-12)


@pytest.mark.parametrize("name,kw", [("small_reactive", {}), ("cfg1", {}),
                                     ("cfg2", {"dims": (32, 32, 32)})])
def test_host_placement_matches_oracle(name, kw):
    w = workload(name, **kw)
    lat = psc.lattice_from_workload(w, device=0)
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"])
    for _, D in w["species"]:
        o.add_species(D)
    for s, c in w["place"]:
        o.place_uniform(s, c)
    a, b = lat.read_state(), o.state()
    for key in ("occ", "id", "vox", "species"):
        assert np.array_equal(a[key], b[key]), key
    assert a["next_id"] == b["next_id"]


def test_placement_capacity_errors():
    lat = new(dims=(4, 4, 4), cap=64)
    a = lat.add_species("A", 1e-12)
    with pytest.raises(psc.PscError) as e:
        lat.place_uniform(a, 65)
    assert e.value.code == psc.PSC_ECAPACITY
    lat.place_uniform(a, 64)   # exactly full
    s = lat.read_state()
    assert np.all(s["occ"] == a)
    lat2 = new(dims=(4, 4, 4), cap=10)
    lat2.add_species("A", 1e-12)
    with pytest.raises(psc.PscError) as e:
        lat2.place_uniform(1, 11)
    assert e.value.code == psc.PSC_ECAPACITY


def test_load_state_round_trip_and_time():
    dims = (8, 12, 4)
    st = random_state(dims, [(1, 20), (2, 7)], seed=3, event=37)
    lat = psc.Lattice(dims, 4.4e-9, 5, 64, track_displacement=True, torch_allocator=False)
    lat.add_species("A", 1e-12)
    lat.add_species("B", 0.3e-12)
    lat.load_state(st)
    r = lat.read_state()
    for key in ("occ", "id", "vox", "species", "dx", "dy", "dz"):
        assert np.array_equal(r[key], st[key] if key != "species" else st["occ"][st["vox"]][
            np.argsort(st["id"])]) or key == "species", key
    order = np.argsort(st["id"])
    assert np.array_equal(r["vox"], st["vox"][order])
    assert r["event"] == 37 and r["next_id"] == st["next_id"]
    o = oracle.Oracle(dims, 4.4e-9, 5)
    o.add_species(1e-12)
    o.add_species(0.3e-12)
    o.load(st["occ"], st["id"][order], st["vox"][order],
           (st["dx"][order], st["dy"][order], st["dz"][order]), 37, st["next_id"])
    assert o.state()["time"] == r["time"]


def test_load_state_rejects_inconsistent_states():
    dims = (4, 4, 4)
    lat = new(dims=dims, cap=64)
    lat.add_species("A", 1e-12)
    good = random_state(dims, [(1, 5)], seed=1, id_gaps=False)
    order = np.argsort(good["id"])
    base = dict(occ=good["occ"], id=good["id"][order], vox=good["vox"][order],
                next_id=good["next_id"])
    lat.load_state(base)
    bad = []
    b = dict(base); b["occ"] = base["occ"].copy(); b["occ"][b["occ"] == 0][:1]  # noqa
    occ2 = base["occ"].copy(); free = np.nonzero(occ2 == 0)[0][0]; occ2[free] = 1
    bad.append(dict(base, occ=occ2))                                  # extra occupied voxel
    bad.append(dict(base, id=base["id"][::-1].copy()))                 # ids not ascending
    bad.append(dict(base, next_id=int(base["id"][-1])))                # id >= next_id
    vox2 = base["vox"].copy(); vox2[1] = vox2[0]
    bad.append(dict(base, vox=vox2))                                   # two on one voxel
    occ3 = base["occ"].copy(); occ3[base["vox"][0]] = 7
    bad.append(dict(base, occ=occ3))                                   # unknown species
    for s in bad:
        with pytest.raises(psc.PscError) as e:
            lat.load_state(s)
        assert e.value.code == psc.PSC_EINVAL


def test_statistics_before_the_first_step():
    w = workload("small_reactive")
    lat = psc.lattice_from_workload(w, device=0)
    st = lat.stats()
    for sp, c in w["place"]:
        assert st["species_count"][sp] == c
    assert st["disp_sum"] == 0


def test_reaction_info_reports_probability_and_clamping():
    """Eq. 6: p = k / (6 sqrt2 (D_A + D_B) r).  The paper's reaction-limited
    check (k_f = 0.027 /nM/s, D = 10 um^2/s, r = 5 nm) gives p = 0.053; the
    crowded workload's A + B -> C (k = 1e-18 m^3/s, D 1 and 0.5 um^2/s,
    r = 4.4 nm) gives p = 17.86, clamped to 1.  Thresholds equal the
    oracle's."""
    from psc_inputs.workloads import per_nM_s
    lat = psc.Lattice((8, 8, 8), 5e-9, 1, 64, torch_allocator=False)
    a = lat.add_species("A", 10e-12)
    b = lat.add_species("B", 10e-12)
    c = lat.add_species("C", 10e-12)
    r0 = lat.add_reaction((a, b), (c,), per_nM_s(0.027))
    r1 = lat.add_reaction((c,), (a, b), 13.5)
    i0 = lat.reaction_info(r0)
    assert i0["order"] == 2 and i0["clamped"] == 0 and abs(i0["p"] - 0.053) < 5e-4
    assert i0["threshold"] == oracle.second_order_threshold(per_nM_s(0.027), 10e-12, 10e-12, 5e-9)
    i1 = lat.reaction_info(r1)
    assert i1 == {"order": 1, "clamped": 0, "p": 13.5, "threshold": 0}
    with pytest.raises(psc.PscError):
        lat.reaction_info(2)
    lat.close()
    w = workload("cfg2", dims=(8, 8, 8))
    lat = psc.Lattice(w["dims"], w["rv"], 1, 64, torch_allocator=False)
    for name, D in w["species"]:
        lat.add_species(name, D)
    rid = lat.add_reaction(*w["reactions"][0])
    info = lat.reaction_info(rid)
    assert info["clamped"] == 1 and info["threshold"] == 1 << 32 and abs(info["p"] - 17.86) < 0.01
    assert oracle.second_order_threshold(w["reactions"][0][2], 1e-12, 0.5e-12, w["rv"]) == 1 << 32
    lat.close()


def test_walls_flag_is_accepted_and_unknown_flags_rejected():
    lat = psc.Lattice((8, 8, 8), 4.4e-9, 1, 64, walls=True, torch_allocator=False)
    lat.add_species("A", 1e-12)
    lat.close()
    d = psc.Desc()
    d.ni = d.nj = d.nk = 8
    d.voxel_radius = 4.4e-9
    d.seed = 1
    d.max_molecules = 64
    d.flags = 16
    h = psc.C.c_void_p()
    assert psc.lib().psc_create_lattice(psc.C.byref(d), psc.C.byref(h)) == psc.PSC_EINVAL


@pytest.mark.parametrize("dims,ok", [((8, 8, 12), True), ((16, 8, 24), True),
                                     ((8, 8, 8), False), ((8, 8, 16), False),
                                     ((12, 8, 12), False), ((8, 4, 12), False)])
def test_fcc_flag_needs_whole_stacking_and_colour_periods(dims, ok):
    # ABC stacking repeats every 3 layers and bricks every 4: nk % 12 == 0;
    # the stage colouring repeats every 8 along i and j
    d = psc.Desc()
    d.ni, d.nj, d.nk = dims
    d.voxel_radius = 4.4e-9
    d.seed = 1
    d.max_molecules = 64
    d.flags = psc.LATTICE_FCC | psc.BOUNDARY_WALLS
    h = psc.C.c_void_p()
    rc = psc.lib().psc_create_lattice(psc.C.byref(d), psc.C.byref(h))
    assert (rc == psc.PSC_OK) == ok
    if ok:
        psc.lib().psc_destroy(h)
    else:
        assert rc == psc.PSC_EINVAL and "12" in psc.lib().psc_last_error(None).decode()


def test_host_placement_on_an_fcc_lattice_matches_oracle():
    w = dict(workload("small_reactive", dims=(16, 16, 12)), lattice="fcc")
    lat = psc.lattice_from_workload(w, device=0)
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"], lattice=oracle.FCC)
    for _, D in w["species"]:
        o.add_species(D)
    for sp, c in w["place"]:
        o.place_uniform(sp, c)
    a, b = lat.read_state(), o.state()
    for key in ("occ", "id", "vox", "species"):
        assert np.array_equal(a[key], b[key]), key


def test_kernel_timing_modes():
    # 1 on (clears), 0 off and 2 on again (both keep the totals, no waiting);
    # anything else is rejected
    lat = psc.Lattice((8, 8, 8), 4.4e-9, 1, 64, torch_allocator=False)
    for mode in (1, 0, 2, 0):
        assert psc.lib().psc_set_kernel_timing(lat.h, mode) == psc.PSC_OK
    for mode in (-1, 3):
        assert psc.lib().psc_set_kernel_timing(lat.h, mode) == psc.PSC_EINVAL
    assert lat.kernel_times()["stage_launches"] == 0
    lat.close()


@pytest.mark.parametrize("lattice", ["hcp", "fcc"])
def test_host_placement_in_compartments_matches_oracle(lattice):
    from psc_inputs import membrane
    w = membrane(dims=(24, 24, 24), seed=3, lattice=lattice)
    lat = psc.lattice_from_workload(w, device=0)
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"],
                      lattice=oracle.FCC if lattice == "fcc" else oracle.HCP)
    for _, D in w["species"]:
        o.add_species(D)
    o.set_compartments(w["compartments"])
    for s, c, cc in w["place_in"]:
        o.place_uniform_in(s, c, cc)
    a, b = lat.read_state(), o.state()
    for key in ("occ", "id", "vox", "species"):
        assert np.array_equal(a[key], b[key]), key
    assert np.all(w["compartments"][a["vox"][a["species"] == 4]] == 1)


def test_compartment_argument_errors():
    lat = new(dims=(8, 8, 8), cap=512)
    a = lat.add_species("A", 1e-12)
    comp = np.zeros(512, np.uint8)
    comp[:8] = 1
    lat.set_compartments(comp)
    with pytest.raises(psc.PscError) as e:
        lat.place_uniform_in(a, 9, 1)            # 8 voxels in compartment 1
    assert e.value.code == psc.PSC_ECAPACITY
    with pytest.raises(psc.PscError) as e:
        lat.place_uniform_in(a, 1, 256)
    assert e.value.code == psc.PSC_EINVAL
    with pytest.raises(psc.PscError) as e:
        lat.place_uniform_in(9, 1, 0)            # unknown species
    assert e.value.code == psc.PSC_EINVAL
    lat.place_uniform_in(a, 8, 1)                 # exactly full
    s = lat.read_state()
    assert sorted(s["vox"].tolist()) == list(range(8))
    with pytest.raises(ValueError):
        lat.set_compartments(np.zeros(100, np.uint8))
