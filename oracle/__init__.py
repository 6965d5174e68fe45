"""Python view of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  It wraps ``libpsc_oracle.so`` (plain C, see ``psc_oracle.h``)
with ctypes and adds nothing to the arithmetic.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libpsc_oracle.so")
SRC = os.path.join(HERE, "psc_oracle.c")

MODE_C, MODE_S, MODE_C_REV = 0, 1, 2
PERIODIC, REFLECT = 0, 1
HCP, FCC = 0, 1
OUTSIDE = 0xFFFFFFFF
CNT_ATTEMPTS, CNT_HOPS, CNT_COLLISIONS, CNT_PLACE_FAIL, CNT_N = range(5)


def build() -> str:
    """Compile the oracle with gcc (-ffp-contract=off keeps FP64 rounding plain)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-ffp-contract=off", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    L = C.CDLL(LIB)
    u32p = C.POINTER(C.c_uint32)
    u64p = C.POINTER(C.c_uint64)
    L.orc_philox4x32.argtypes = [u32p, u32p, u32p]
    L.orc_philox4x64.argtypes = [u64p, u64p, u64p]
    L.orc_neighbour.argtypes = [C.c_uint32] * 4 + [C.c_int]
    L.orc_neighbour.restype = C.c_uint32
    L.orc_neighbour_b.argtypes = [C.c_uint32] * 4 + [C.c_int, C.c_int]
    L.orc_neighbour_b.restype = C.c_uint32
    L.orc_set_boundary.argtypes = [C.c_void_p, C.c_int]
    L.orc_set_boundary.restype = C.c_int
    L.orc_set_lattice.argtypes = [C.c_void_p, C.c_int]
    L.orc_set_lattice.restype = C.c_int
    L.orc_neighbour_l.argtypes = [C.c_uint32] * 4 + [C.c_int, C.c_int, C.c_int]
    L.orc_neighbour_l.restype = C.c_uint32
    L.orc_hop_vector_l.argtypes = [C.c_uint32] * 4 + [C.c_int, C.c_int, C.POINTER(C.c_int32)]
    L.orc_position_l.argtypes = [C.c_uint32] * 4 + [C.c_double, C.c_int,
                                                    C.POINTER(C.c_double)]
    L.orc_colour_l.argtypes = [C.c_uint32] * 4 + [C.c_int]
    L.orc_colour_l.restype = C.c_int
    L.orc_n_colours.argtypes = [C.c_int]
    L.orc_n_colours.restype = C.c_int
    L.orc_stage_order_n.argtypes = [C.c_uint64, C.c_uint64, C.c_int, C.POINTER(C.c_uint8)]
    L.orc_neighbour_table.argtypes = [C.c_uint32] * 3 + [u32p]
    L.orc_neighbour_table_l.argtypes = [C.c_uint32] * 3 + [C.c_int, C.c_int, u32p]
    L.orc_hop_vector.argtypes = [C.c_uint32] * 4 + [C.c_int, C.POINTER(C.c_int32)]
    L.orc_position.argtypes = [C.c_uint32] * 4 + [C.c_double, C.POINTER(C.c_double)]
    L.orc_colour.argtypes = [C.c_uint32] * 4
    L.orc_colour.restype = C.c_int
    L.orc_stage_order.argtypes = [C.c_uint64, C.c_uint64, C.POINTER(C.c_uint8)]
    L.orc_second_order_threshold.argtypes = [C.c_double] * 4
    L.orc_second_order_threshold.restype = C.c_uint64
    L.orc_prob_to_u32.argtypes = [C.c_double]
    L.orc_prob_to_u32.restype = C.c_uint32
    L.orc_tau.argtypes = [C.c_double, C.c_double]
    L.orc_tau.restype = C.c_double
    L.orc_create.argtypes = [C.c_uint32] * 3 + [C.c_double, C.c_uint64]
    L.orc_create.restype = C.c_void_p
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_add_species.argtypes = [C.c_void_p, C.c_double]
    L.orc_add_species.restype = C.c_int
    L.orc_add_reaction.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_uint16), C.c_int,
                                   C.POINTER(C.c_uint16), C.c_double]
    L.orc_add_reaction.restype = C.c_int
    L.orc_place_uniform.argtypes = [C.c_void_p, C.c_uint16, C.c_uint64]
    L.orc_place_uniform.restype = C.c_int
    L.orc_set_compartments.argtypes = [C.c_void_p, C.POINTER(C.c_uint8)]
    L.orc_set_compartments.restype = C.c_int
    L.orc_place_uniform_in.argtypes = [C.c_void_p, C.c_uint16, C.c_uint64, C.c_int]
    L.orc_place_uniform_in.restype = C.c_int
    i32p = C.POINTER(C.c_int32)
    L.orc_load.argtypes = [C.c_void_p, C.POINTER(C.c_uint16), C.c_uint64, u32p, u32p,
                           i32p, i32p, i32p, C.c_uint64, C.c_uint32]
    L.orc_load.restype = C.c_int
    L.orc_run.argtypes = [C.c_void_p, C.c_uint64, C.c_int]
    L.orc_run.restype = C.c_int
    L.orc_walk_forced.argtypes = [C.c_void_p, C.c_uint64, u32p, C.POINTER(C.c_uint8),
                                  C.POINTER(C.c_uint8)]
    L.orc_walk_forced.restype = C.c_int
    L.orc_n_molecules.argtypes = [C.c_void_p]
    L.orc_n_molecules.restype = C.c_uint64
    L.orc_n_voxels.argtypes = [C.c_void_p]
    L.orc_n_voxels.restype = C.c_uint64
    L.orc_read.argtypes = [C.c_void_p, C.POINTER(C.c_uint16), u32p, u32p,
                           C.POINTER(C.c_uint16), i32p, i32p, i32p]
    L.orc_counters.argtypes = [C.c_void_p, u64p]
    L.orc_reactions_fired.argtypes = [C.c_void_p, u64p]
    L.orc_species_count.argtypes = [C.c_void_p, C.c_uint16]
    L.orc_species_count.restype = C.c_uint64
    L.orc_event.argtypes = [C.c_void_p]
    L.orc_event.restype = C.c_uint64
    L.orc_time.argtypes = [C.c_void_p]
    L.orc_time.restype = C.c_double
    L.orc_next_id.argtypes = [C.c_void_p]
    L.orc_next_id.restype = C.c_uint32
    _lib = L
    return L


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


# ---------------------------------------------------------------- primitives
def philox4x32(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def philox4x64(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64(_p(c, C.c_uint64), _p(k, C.c_uint64), _p(out, C.c_uint64))
    return out


def neighbour(dims, v: int, n: int) -> int:
    return lib().orc_neighbour(dims[0], dims[1], dims[2], v, n)


def neighbour_b(dims, v: int, n: int, boundary: int) -> int:
    """neighbour n of v; OUTSIDE beyond a wall of a closed box"""
    return lib().orc_neighbour_b(dims[0], dims[1], dims[2], v, n, boundary)


def neighbour_table(dims) -> np.ndarray:
    nv = int(dims[0]) * int(dims[1]) * int(dims[2])
    out = np.zeros(nv * 12, np.uint32)
    lib().orc_neighbour_table(dims[0], dims[1], dims[2], _p(out, C.c_uint32))
    return out.reshape(nv, 12)


def neighbour_table_l(dims, lattice: int, boundary: int = PERIODIC) -> np.ndarray:
    nv = int(dims[0]) * int(dims[1]) * int(dims[2])
    out = np.zeros(nv * 12, np.uint32)
    lib().orc_neighbour_table_l(dims[0], dims[1], dims[2], lattice, boundary,
                                _p(out, C.c_uint32))
    return out.reshape(nv, 12)


def hop_vector(dims, v: int, n: int):
    out = (C.c_int32 * 3)()
    lib().orc_hop_vector(dims[0], dims[1], dims[2], v, n, out)
    return tuple(out)


def position(dims, v: int, rv: float):
    out = (C.c_double * 3)()
    lib().orc_position(dims[0], dims[1], dims[2], v, rv, out)
    return tuple(out)


def colour(dims, v: int) -> int:
    return lib().orc_colour(dims[0], dims[1], dims[2], v)


def stage_order(seed: int, event: int) -> list:
    out = (C.c_uint8 * 16)()
    lib().orc_stage_order(seed, event, out)
    return list(out)


# either lattice (HCP or FCC)
def neighbour_l(dims, v: int, n: int, lattice: int, boundary: int = PERIODIC) -> int:
    return lib().orc_neighbour_l(dims[0], dims[1], dims[2], v, n, lattice, boundary)


def hop_vector_l(dims, v: int, n: int, lattice: int):
    out = (C.c_int32 * 3)()
    lib().orc_hop_vector_l(dims[0], dims[1], dims[2], v, n, lattice, out)
    return tuple(out)


def position_l(dims, v: int, rv: float, lattice: int):
    out = (C.c_double * 3)()
    lib().orc_position_l(dims[0], dims[1], dims[2], v, rv, lattice, out)
    return tuple(out)


def colour_l(dims, v: int, lattice: int) -> int:
    return lib().orc_colour_l(dims[0], dims[1], dims[2], v, lattice)


def n_colours(lattice: int) -> int:
    return lib().orc_n_colours(lattice)


def stage_order_n(seed: int, event: int, n: int) -> list:
    out = (C.c_uint8 * 24)()
    lib().orc_stage_order_n(seed, event, n, out)
    return list(out)[:n]


def second_order_threshold(k, DA, DB, rv) -> int:
    return lib().orc_second_order_threshold(k, DA, DB, rv)


def prob_to_u32(p: float) -> int:
    return lib().orc_prob_to_u32(p)


def tau(rv: float, D: float) -> float:
    return lib().orc_tau(rv, D)


# ---------------------------------------------------------------- simulation
class Oracle:
    """One lattice simulated by the CPU oracle."""

    def __init__(self, dims, rv: float, seed: int, boundary: int = 0, lattice: int = 0):
        self.L = lib()
        self.dims = tuple(int(x) for x in dims)
        h = self.L.orc_create(self.dims[0], self.dims[1], self.dims[2], rv, seed)
        if not h:
            raise ValueError(f"oracle: bad lattice {dims}")
        self.h = h
        self.n_rx = 0
        if self.L.orc_set_boundary(self.h, boundary) != 0:
            raise ValueError(f"oracle: bad boundary {boundary}")
        if self.L.orc_set_lattice(self.h, lattice) != 0:
            raise ValueError(f"oracle: bad lattice kind {lattice} for {dims}")

    def close(self):
        if self.h:
            self.L.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_species(self, D: float) -> int:
        r = self.L.orc_add_species(self.h, D)
        if r < 0:
            raise ValueError("oracle: add_species")
        return r

    def add_reaction(self, reactants, products, k: float) -> int:
        ra = np.array(reactants, np.uint16)
        pa = np.array(list(products) + [0], np.uint16)
        r = self.L.orc_add_reaction(self.h, len(reactants), _p(ra, C.c_uint16),
                                    len(products), _p(pa, C.c_uint16), k)
        if r < 0:
            raise ValueError("oracle: add_reaction")
        self.n_rx += 1
        return r

    def place_uniform(self, species: int, count: int):
        if self.L.orc_place_uniform(self.h, species, count):
            raise ValueError("oracle: place_uniform")

    def set_compartments(self, comp):
        """comp[v]: the compartment (0..255) of every voxel v, linear order"""
        comp = np.ascontiguousarray(comp, np.uint8)
        if comp.shape != (int(np.prod(self.dims)),):
            raise ValueError("oracle: one compartment per voxel")
        if self.L.orc_set_compartments(self.h, _p(comp, C.c_uint8)):
            raise ValueError("oracle: set_compartments")

    def place_uniform_in(self, species: int, count: int, compartment: int):
        if self.L.orc_place_uniform_in(self.h, species, count, compartment):
            raise ValueError("oracle: place_uniform_in")

    def load(self, occ, ids, vox, disp=None, event=0, next_id=None):
        occ = np.ascontiguousarray(occ, np.uint16)
        ids = np.ascontiguousarray(ids, np.uint32)
        vox = np.ascontiguousarray(vox, np.uint32)
        if next_id is None:
            next_id = int(ids.max()) + 1 if len(ids) else 0
        if disp is None:
            dx = dy = dz = None
        else:
            dx, dy, dz = (np.ascontiguousarray(d, np.int32) for d in disp)
        rc = self.L.orc_load(self.h, _p(occ, C.c_uint16), len(ids), _p(ids, C.c_uint32),
                             _p(vox, C.c_uint32),
                             None if dx is None else _p(dx, C.c_int32),
                             None if dy is None else _p(dy, C.c_int32),
                             None if dz is None else _p(dz, C.c_int32),
                             event, next_id)
        if rc:
            raise ValueError("oracle: load rejected the state")

    def run(self, n_events: int, mode: int = MODE_C):
        if self.L.orc_run(self.h, n_events, mode):
            raise RuntimeError("oracle: run failed")

    def walk_forced(self, order_ids, dirs, fire):
        o = np.ascontiguousarray(order_ids, np.uint32)
        d = np.ascontiguousarray(dirs, np.uint8)
        f = np.ascontiguousarray(fire, np.uint8)
        if self.L.orc_walk_forced(self.h, len(o), _p(o, C.c_uint32), _p(d, C.c_uint8),
                                  _p(f, C.c_uint8)):
            raise RuntimeError("oracle: walk_forced failed")

    @property
    def n_molecules(self) -> int:
        return self.L.orc_n_molecules(self.h)

    @property
    def n_voxels(self) -> int:
        return self.L.orc_n_voxels(self.h)

    def state(self, with_occ: bool = True) -> dict:
        n = self.n_molecules
        occ = np.zeros(self.n_voxels, np.uint16) if with_occ else None
        ids = np.zeros(n, np.uint32)
        vox = np.zeros(n, np.uint32)
        sp = np.zeros(n, np.uint16)
        dx = np.zeros(n, np.int32)
        dy = np.zeros(n, np.int32)
        dz = np.zeros(n, np.int32)
        self.L.orc_read(self.h, None if occ is None else _p(occ, C.c_uint16),
                        _p(ids, C.c_uint32), _p(vox, C.c_uint32), _p(sp, C.c_uint16),
                        _p(dx, C.c_int32), _p(dy, C.c_int32), _p(dz, C.c_int32))
        cnt = np.zeros(CNT_N, np.uint64)
        self.L.orc_counters(self.h, _p(cnt, C.c_uint64))
        fired = np.zeros(max(self.n_rx, 1), np.uint64)
        self.L.orc_reactions_fired(self.h, _p(fired, C.c_uint64))
        return {
            "occ": occ, "id": ids, "vox": vox, "species": sp,
            "dx": dx, "dy": dy, "dz": dz,
            "attempts": int(cnt[CNT_ATTEMPTS]), "hops": int(cnt[CNT_HOPS]),
            "collisions": int(cnt[CNT_COLLISIONS]),
            "place_fail": int(cnt[CNT_PLACE_FAIL]),
            "fired": fired[: self.n_rx].copy(),
            "event": int(self.L.orc_event(self.h)),
            "time": float(self.L.orc_time(self.h)),
            "next_id": int(self.L.orc_next_id(self.h)),
        }

    def species_count(self, species: int) -> int:
        return self.L.orc_species_count(self.h, species)
