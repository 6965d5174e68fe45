"""The GPU path's geometry against the oracle, on the CPU: the stencils (HCP
and FCC), wall handling, stage colours, hop vectors and the 4x4x4 brick
layout of `psc_core.h`, compiled for the host from the library's own header,
must give what the oracle gives for every voxel and direction (2.1; the FCC
stencil as the oracle derives it from ABC-stacked positions).  The oracle's
geometry is pinned to Euclidean geometry by the oracle tests; this closes
the loop without a GPU.  The kernels' Philox4x32-10, compiled the same way,
must reproduce the generator's published known-answer vectors."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1605_03726_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    out = str(tmp_path_factory.mktemp("geo") / "libgeo.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-shared",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I", CSRC, "-o", out, os.path.join(HERE, "device_geometry_probe.cpp")],
                   check=True, stderr=subprocess.DEVNULL)
    L = C.CDLL(out)
    u32p = C.POINTER(C.c_uint32)
    L.probe_neighbours.argtypes = [C.c_uint32] * 3 + [C.c_int] * 3 + [u32p]
    L.probe_colours.argtypes = [C.c_uint32] * 3 + [C.c_int, u32p]
    L.probe_hop.argtypes = [C.c_uint32, C.c_int32, C.c_int, C.POINTER(C.c_int32)]
    L.probe_philox.argtypes = [u32p, u32p, u32p]
    L.probe_n_colours.argtypes = [C.c_int]
    L.probe_n_colours.restype = C.c_int
    return L


CASES = [((4, 4, 4), oracle.HCP), ((8, 12, 16), oracle.HCP), ((20, 8, 8), oracle.HCP),
         ((8, 8, 12), oracle.FCC), ((8, 16, 24), oracle.FCC), ((24, 8, 12), oracle.FCC)]


@pytest.mark.parametrize("dims,lattice", CASES)
@pytest.mark.parametrize("boundary", [oracle.PERIODIC, oracle.REFLECT])
@pytest.mark.parametrize("brick", [1, 0])
def test_neighbours_equal_the_oracle(probe, dims, lattice, boundary, brick):
    nv = dims[0] * dims[1] * dims[2]
    got = np.zeros(12 * nv, np.uint32)
    probe.probe_neighbours(*dims, lattice, 1 if boundary == oracle.REFLECT else 0, brick,
                           got.ctypes.data_as(C.POINTER(C.c_uint32)))
    want = np.array([[oracle.neighbour_l(dims, v, n, lattice, boundary) for n in range(12)]
                     for v in range(nv)], np.uint32).ravel()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dims,lattice", CASES)
def test_colours_and_hop_vectors_equal_the_oracle(probe, dims, lattice):
    nv = dims[0] * dims[1] * dims[2]
    assert probe.probe_n_colours(lattice) == oracle.n_colours(lattice)
    got = np.zeros(nv, np.uint32)
    probe.probe_colours(*dims, lattice, got.ctypes.data_as(C.POINTER(C.c_uint32)))
    want = np.array([oracle.colour_l(dims, v, lattice) for v in range(nv)], np.uint32)
    assert np.array_equal(got, want)
    out = (C.c_int32 * 3)()
    for v in range(0, nv, 7):
        k = v // (dims[0] * dims[1])
        for n in range(12):
            probe.probe_hop(n, k, lattice, out)
            assert tuple(out) == oracle.hop_vector_l(dims, v, n, lattice), (v, n)


def test_device_philox_known_answers(probe):
    from test_oracle_philox import philox4x32_kat
    u32p = C.POINTER(C.c_uint32)
    for ctr, key, want in philox4x32_kat():
        c = np.array(ctr, np.uint32)
        k = np.array(key, np.uint32)
        out = np.zeros(4, np.uint32)
        probe.probe_philox(c.ctypes.data_as(u32p), k.ctypes.data_as(u32p), out.ctypes.data_as(u32p))
        assert tuple(int(x) for x in out) == want, (ctr, key)
