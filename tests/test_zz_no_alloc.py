"""psc_read_state_noalloc (the read-back for callers that cannot allocate
device memory) against psc_read_state, through the C ABI on the GPU: the
same state, field by field, on two calls in a row on different lattices, the
second smaller (the static buffer keeps the first call's contents), in both
device layouts and over several buffer-sized ranges; a lattice whose layer
of bricks exceeds the buffer is refused without reading anything."""
import numpy as np
import pytest

from paper_1605_03726_amd import psc
from psc_inputs import workload

pytestmark = pytest.mark.gpu

FIELDS = ("occ", "id", "vox", "species", "dx", "dy", "dz", "fired")
SCALARS = ("attempts", "hops", "collisions", "place_fail", "event", "time", "next_id")


def run(dims, seed, linear, events=15):
    w = workload("small_reactive", dims=dims, seed=seed, events=events)
    lat = psc.lattice_from_workload(w, linear_layout=linear)
    lat.step(events)
    return lat


def same(a, b):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k
    for k in SCALARS:
        assert a[k] == b[k], k


@pytest.mark.parametrize("linear", [False, True])
def test_noalloc_read_equals_read_state_on_two_calls(linear):
    big = run((64, 48, 40), 5, linear)
    small = run((16, 12, 8), 6, linear)
    for lat in (big, small):          # the second call reads a smaller lattice
        a = lat.read_state()
        b = lat.read_state(noalloc=True)
        same(a, b)
        assert b["occ"].shape == (lat.nv,) and np.count_nonzero(b["occ"]) == len(b["id"])
    big.close()
    small.close()


def test_noalloc_read_spans_several_buffer_loads():
    # 2048 x 2048 voxels per k-layer: one layer of bricks fills the 32 MiB
    # buffer exactly, so 8 k-layers take two loads of it
    w = workload("small_reactive", seed=9, events=3)
    w = dict(w, dims=(2048, 2048, 8), place=[(s, 20000) for s, _ in w["place"]])
    lat = psc.lattice_from_workload(w, max_molecules=200000)
    lat.step(3)
    same(lat.read_state(), lat.read_state(noalloc=True))
    lat.close()


def test_noalloc_read_refuses_a_layer_beyond_the_buffer():
    w = workload("small_reactive", seed=4, events=1)
    w = dict(w, dims=(4096, 2048, 4), place=[(s, 1000) for s, _ in w["place"]])
    lat = psc.lattice_from_workload(w, max_molecules=20000)
    lat.step(1)
    with pytest.raises(psc.PscError) as e:
        lat.read_state(noalloc=True)
    assert e.value.code == psc.PSC_EINVAL and "static staging buffer" in str(e.value)
    lat.read_state()  # the allocating read-back still works
    lat.close()
