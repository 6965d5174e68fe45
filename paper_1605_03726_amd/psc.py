"""ctypes binding of libpsc (include/psc.h): argument marshalling only.

Every step of the walk runs in the HIP kernels of libpsc.so.  PyTorch provides
device memory (through the caching allocator hooks) and streams.  If the
library is not built, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpsc.so")

PSC_OK, PSC_EINVAL, PSC_ESTATE, PSC_ENOMEM, PSC_ECAPACITY, PSC_EDEVICE = 0, -1, -2, -3, -4, -5
TRACK_DISPLACEMENT = 1
LAYOUT_LINEAR = 2
BOUNDARY_WALLS = 4
LATTICE_FCC = 8

_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Desc(C.Structure):
    _fields_ = [("ni", C.c_uint32), ("nj", C.c_uint32), ("nk", C.c_uint32),
                ("voxel_radius", C.c_double), ("seed", C.c_uint64),
                ("max_molecules", C.c_uint64), ("flags", C.c_uint32), ("device", C.c_int32),
                ("alloc", _ALLOC), ("free", _FREE), ("alloc_user", C.c_void_p)]


class Counters(C.Structure):
    _fields_ = [("attempts", C.c_uint64), ("hops", C.c_uint64), ("collisions", C.c_uint64),
                ("placement_failures", C.c_uint64)]


class ReactionInfo(C.Structure):
    _fields_ = [("order", C.c_uint32), ("clamped", C.c_uint32), ("p", C.c_double),
                ("threshold", C.c_uint64)]


class KernelTimes(C.Structure):
    _fields_ = [("begin_ms", C.c_double), ("stage_ms", C.c_double), ("end_ms", C.c_double),
                ("begin_launches", C.c_uint64), ("stage_launches", C.c_uint64),
                ("end_launches", C.c_uint64)]


class Launch(C.Structure):
    _fields_ = [("items_per_thread", C.c_uint32), ("stage_blocks", C.c_uint32)]


class StateView(C.Structure):
    _fields_ = [("occupancy", C.POINTER(C.c_uint16)), ("n_molecules", C.c_uint64),
                ("id", C.POINTER(C.c_uint32)), ("voxel", C.POINTER(C.c_uint32)),
                ("species", C.POINTER(C.c_uint16)), ("dx", C.POINTER(C.c_int32)),
                ("dy", C.POINTER(C.c_int32)), ("dz", C.POINTER(C.c_int32)),
                ("event", C.c_uint64), ("next_id", C.c_uint32), ("time", C.c_double),
                ("counters", Counters), ("reactions_fired", C.POINTER(C.c_uint64))]


class PscError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"psc error {code}: {msg}")
        self.code = code


_lib = None


def _hip_runtimes() -> set:
    """paths of every HIP runtime mapped into this process"""
    out = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    out.add(line.split()[-1])
    except OSError:
        pass
    return out


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run paper_1605_03726_amd/build.py "
                          "(or __graft_entry__.build())")
    # torch ships its own HIP runtime.  It is loaded first so that libpsc's
    # dependency (same soname) binds to it: one runtime per process, which is
    # what lets libpsc use torch's device memory and streams.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    rts = _hip_runtimes()
    if len(rts) > 1:
        raise ImportError("two HIP runtimes are loaded (%s); import torch before any other "
                          "HIP library" % ", ".join(sorted(rts)))
    vp = C.c_void_p
    L.psc_create_lattice.argtypes = [C.POINTER(Desc), C.POINTER(vp)]
    L.psc_create_lattice.restype = C.c_int32
    L.psc_destroy.argtypes = [vp]
    L.psc_destroy.restype = None
    L.psc_last_error.argtypes = [vp]
    L.psc_last_error.restype = C.c_char_p
    L.psc_add_species.argtypes = [vp, C.c_char_p, C.c_double, C.POINTER(C.c_uint16)]
    L.psc_add_species.restype = C.c_int32
    L.psc_add_reaction.argtypes = [vp, C.POINTER(C.c_uint16), C.c_uint32, C.POINTER(C.c_uint16),
                                   C.c_uint32, C.c_double, C.POINTER(C.c_uint32)]
    L.psc_add_reaction.restype = C.c_int32
    L.psc_get_reaction_info.argtypes = [vp, C.c_uint32, C.POINTER(ReactionInfo)]
    L.psc_get_reaction_info.restype = C.c_int32
    L.psc_place_uniform.argtypes = [vp, C.c_uint16, C.c_uint64]
    L.psc_place_uniform.restype = C.c_int32
    L.psc_set_compartments.argtypes = [vp, C.POINTER(C.c_uint8)]
    L.psc_set_compartments.restype = C.c_int32
    L.psc_place_uniform_in.argtypes = [vp, C.c_uint16, C.c_uint64, C.c_uint32]
    L.psc_place_uniform_in.restype = C.c_int32
    L.psc_load_state.argtypes = [vp, C.POINTER(StateView)]
    L.psc_load_state.restype = C.c_int32
    L.psc_step.argtypes = [vp, C.c_uint64, vp]
    L.psc_step.restype = C.c_int32
    L.psc_sync.argtypes = [vp]
    L.psc_sync.restype = C.c_int32
    L.psc_read_state.argtypes = [vp, C.POINTER(StateView), vp]
    L.psc_read_state.restype = C.c_int32
    L.psc_read_state_noalloc.argtypes = [vp, C.POINTER(StateView), vp]
    L.psc_read_state_noalloc.restype = C.c_int32
    L.psc_query_sizes.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                  C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
    L.psc_query_sizes.restype = C.c_int32
    L.psc_device_bytes.argtypes = [vp, C.POINTER(C.c_uint64)]
    L.psc_device_bytes.restype = C.c_int32
    L.psc_read_counters.argtypes = [vp, C.POINTER(Counters), C.POINTER(C.c_uint64)]
    L.psc_read_counters.restype = C.c_int32
    L.psc_set_launch.argtypes = [vp, C.POINTER(Launch)]
    L.psc_set_launch.restype = C.c_int32
    L.psc_get_launch.argtypes = [vp, C.POINTER(Launch)]
    L.psc_get_launch.restype = C.c_int32
    L.psc_read_stats.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                 C.POINTER(C.c_uint64)]
    L.psc_read_stats.restype = C.c_int32
    L.psc_set_graph_replay.argtypes = [vp, C.c_int]
    L.psc_set_graph_replay.restype = C.c_int32
    L.psc_set_kernel_timing.argtypes = [vp, C.c_int]
    L.psc_set_kernel_timing.restype = C.c_int32
    L.psc_get_kernel_times.argtypes = [vp, C.POINTER(KernelTimes)]
    L.psc_get_kernel_times.restype = C.c_int32
    L.psc_ensemble_create.argtypes = [C.POINTER(vp), C.c_uint32, C.POINTER(vp)]
    L.psc_ensemble_create.restype = C.c_int32
    L.psc_ensemble_step.argtypes = [vp, C.c_uint64, vp]
    L.psc_ensemble_step.restype = C.c_int32
    L.psc_ensemble_sync.argtypes = [vp]
    L.psc_ensemble_sync.restype = C.c_int32
    L.psc_ensemble_set_launch.argtypes = [vp, C.POINTER(Launch)]
    L.psc_ensemble_set_launch.restype = C.c_int32
    L.psc_ensemble_get_launch.argtypes = [vp, C.POINTER(Launch)]
    L.psc_ensemble_get_launch.restype = C.c_int32
    L.psc_ensemble_autotune.argtypes = [vp, C.c_uint32]
    L.psc_ensemble_autotune.restype = C.c_int32
    L.psc_ensemble_tuned.argtypes = [vp, C.POINTER(Launch), C.POINTER(C.c_double)]
    L.psc_ensemble_tuned.restype = C.c_int32
    L.psc_ensemble_read.argtypes = [vp, C.c_uint32, C.POINTER(StateView), vp]
    L.psc_ensemble_read.restype = C.c_int32
    L.psc_required_sizes.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                     C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
    L.psc_required_sizes.restype = C.c_int32
    L.psc_ensemble_destroy.argtypes = [vp]
    L.psc_ensemble_destroy.restype = None
    L.psc_ensemble_last_error.argtypes = [vp]
    L.psc_ensemble_last_error.restype = C.c_char_p
    _lib = L
    return L


def _ptr(a, ct):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


def _torch_hooks(device: int):
    """allocator hooks backed by torch's caching allocator"""
    import torch

    def alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=device)
        except Exception:
            return None

    def free(ptr, user):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except (AttributeError, TypeError):
            pass  # interpreter shutdown: torch's allocator is already gone

    return _ALLOC(alloc), _FREE(free)


def current_stream():
    """torch's current HIP stream (None, the default stream, without a GPU)"""
    import torch
    if not torch.cuda.is_available():
        return None
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Lattice:
    """One lattice on the GPU (see include/psc.h): HCP, or FCC with fcc=True."""

    def __init__(self, dims, voxel_radius: float, seed: int, max_molecules: int,
                 track_displacement: bool = False, device: int = 0,
                 torch_allocator: bool = True, linear_layout: bool = False,
                 walls: bool = False, fcc: bool = False):
        self.L = lib()
        self.dims = tuple(int(x) for x in dims)
        self.nv = self.dims[0] * self.dims[1] * self.dims[2]
        d = Desc()
        d.ni, d.nj, d.nk = self.dims
        d.voxel_radius = voxel_radius
        d.seed = seed
        d.max_molecules = max_molecules
        d.flags = (TRACK_DISPLACEMENT if track_displacement else 0) | (
            LAYOUT_LINEAR if linear_layout else 0) | (BOUNDARY_WALLS if walls else 0) | (
            LATTICE_FCC if fcc else 0)
        d.device = device
        self._hooks = None
        if torch_allocator:
            self._hooks = _torch_hooks(device)
            d.alloc, d.free = self._hooks
        h = C.c_void_p()
        rc = self.L.psc_create_lattice(C.byref(d), C.byref(h))
        if rc != PSC_OK:
            raise PscError(rc, self.L.psc_last_error(None).decode())
        self.h = h
        self.n_rx = 0
        self.n_species = 0

    def _check(self, rc):
        if rc != PSC_OK:
            raise PscError(rc, self.L.psc_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.L.psc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_species(self, name: str, D: float) -> int:
        out = C.c_uint16()
        self._check(self.L.psc_add_species(self.h, name.encode(), D, C.byref(out)))
        self.n_species += 1
        return out.value

    def add_reaction(self, reactants, products, k: float) -> int:
        r = np.array(reactants, np.uint16)
        p = np.array(list(products) + [0], np.uint16)
        out = C.c_uint32()
        self._check(self.L.psc_add_reaction(self.h, _ptr(r, C.c_uint16), len(reactants),
                                            _ptr(p, C.c_uint16), len(products), k, C.byref(out)))
        self.n_rx += 1
        return out.value

    def reaction_info(self, reaction_id: int) -> dict:
        ri = ReactionInfo()
        self._check(self.L.psc_get_reaction_info(self.h, reaction_id, C.byref(ri)))
        return {f: getattr(ri, f) for f, _ in ReactionInfo._fields_}

    def place_uniform(self, species: int, count: int):
        self._check(self.L.psc_place_uniform(self.h, species, count))

    def set_compartments(self, comp):
        """comp[v]: the compartment (0..255) of every voxel v, linear order"""
        c = np.ascontiguousarray(comp, np.uint8)
        if c.shape != (self.nv,):
            raise ValueError("one compartment per voxel")
        self._check(self.L.psc_set_compartments(self.h, _ptr(c, C.c_uint8)))

    def place_uniform_in(self, species: int, count: int, compartment: int):
        self._check(self.L.psc_place_uniform_in(self.h, species, count, compartment))

    def load_state(self, st: dict):
        occ = np.ascontiguousarray(st["occ"], np.uint16)
        ids = np.ascontiguousarray(st["id"], np.uint32)
        vox = np.ascontiguousarray(st["vox"], np.uint32)
        sp = st.get("species")
        sp = None if sp is None else np.ascontiguousarray(sp, np.uint16)
        d = [None if st.get(k) is None else np.ascontiguousarray(st[k], np.int32)
             for k in ("dx", "dy", "dz")]
        v = StateView()
        v.occupancy = _ptr(occ, C.c_uint16)
        v.n_molecules = len(ids)
        v.id = _ptr(ids, C.c_uint32)
        v.voxel = _ptr(vox, C.c_uint32)
        v.species = _ptr(sp, C.c_uint16)
        v.dx, v.dy, v.dz = (_ptr(a, C.c_int32) for a in d)
        v.event = int(st.get("event", 0))
        v.next_id = int(st["next_id"])
        self._check(self.L.psc_load_state(self.h, C.byref(v)))

    def step(self, n_events: int, stream=None):
        s = current_stream() if stream is None else stream
        self._check(self.L.psc_step(self.h, n_events, s))

    def sync(self):
        self._check(self.L.psc_sync(self.h))

    def n_molecules(self) -> int:
        n = C.c_uint64()
        self._check(self.L.psc_query_sizes(self.h, None, C.byref(n), None, None))
        return n.value

    def counters(self) -> dict:
        c = Counters()
        e = C.c_uint64()
        self._check(self.L.psc_read_counters(self.h, C.byref(c), C.byref(e)))
        out = {f: getattr(c, f) for f, _ in Counters._fields_}
        out["event"] = e.value
        return out

    def set_launch(self, items_per_thread: int = 0, stage_blocks: int = 0):
        l = Launch(items_per_thread, stage_blocks)
        self._check(self.L.psc_set_launch(self.h, C.byref(l)))

    def get_launch(self) -> dict:
        l = Launch()
        self._check(self.L.psc_get_launch(self.h, C.byref(l)))
        return {"items_per_thread": l.items_per_thread, "stage_blocks": l.stage_blocks}

    def stats(self) -> dict:
        counts = np.zeros(self.n_species + 1, np.uint64)
        dsum = C.c_uint64()
        nw = C.c_uint64()
        self._check(self.L.psc_read_stats(self.h, _ptr(counts, C.c_uint64), C.byref(dsum),
                                          C.byref(nw)))
        return {"species_count": counts, "disp_sum": dsum.value, "n_walkers": nw.value}

    def set_graph_replay(self, on: bool):
        self._check(self.L.psc_set_graph_replay(self.h, 1 if on else 0))

    def set_kernel_timing(self, on: bool, keep: bool = False):
        """on: record per-launch times (clearing the totals unless keep);
        off keeps the totals.  Switching with keep never waits for the
        device."""
        self._check(self.L.psc_set_kernel_timing(self.h, (2 if keep else 1) if on else 0))

    def kernel_times(self) -> dict:
        t = KernelTimes()
        self._check(self.L.psc_get_kernel_times(self.h, C.byref(t)))
        return {f: getattr(t, f) for f, _ in KernelTimes._fields_}

    def device_bytes(self) -> int:
        b = C.c_uint64()
        self._check(self.L.psc_device_bytes(self.h, C.byref(b)))
        return b.value

    def read_state(self, with_occ: bool = True, stream=None, noalloc: bool = False) -> dict:
        """the state (psc_read_state); noalloc: through psc_read_state_noalloc,
        which allocates no device memory"""
        fn = self.L.psc_read_state_noalloc if noalloc else self.L.psc_read_state
        s = None if stream is None else stream
        return _read_view(self.nv if with_occ else 0, self.n_molecules(), self.n_rx,
                          lambda v: self._check(fn(self.h, C.byref(v), s)))


def _read_view(n_voxels: int, cap: int, n_rx: int, call) -> dict:
    """host arrays for a state of up to `cap` molecules (occupancy too unless
    n_voxels is 0), filled by call(view); the state as a dict"""
    occ = np.zeros(n_voxels, np.uint16) if n_voxels else None
    arrays = {k: np.zeros(cap, t) for k, t in (("id", np.uint32), ("vox", np.uint32),
                                                ("species", np.uint16), ("dx", np.int32),
                                                ("dy", np.int32), ("dz", np.int32))}
    fired = np.zeros(max(n_rx, 1), np.uint64)
    v = StateView()
    v.occupancy = _ptr(occ, C.c_uint16)
    v.n_molecules = cap
    v.id = _ptr(arrays["id"], C.c_uint32)
    v.voxel = _ptr(arrays["vox"], C.c_uint32)
    v.species = _ptr(arrays["species"], C.c_uint16)
    v.dx = _ptr(arrays["dx"], C.c_int32)
    v.dy = _ptr(arrays["dy"], C.c_int32)
    v.dz = _ptr(arrays["dz"], C.c_int32)
    v.reactions_fired = _ptr(fired, C.c_uint64)
    call(v)
    n = v.n_molecules
    out = {k: a[:n].copy() for k, a in arrays.items()}
    out.update(occ=occ, attempts=v.counters.attempts, hops=v.counters.hops,
               collisions=v.counters.collisions,
               place_fail=v.counters.placement_failures,
               fired=fired[:n_rx].copy(), event=v.event, time=v.time,
               next_id=v.next_id)
    return out


def lattice_from_workload(w: dict, max_molecules: int | None = None, device: int = 0,
                          place: bool = True, linear_layout: bool = False) -> Lattice:
    """Builds a Lattice from a workload description (species, reactions,
    uniform placements)."""
    nv = int(np.prod(w["dims"]))
    if max_molecules is None:
        placed = sum(c for _, c in w["place"]) + sum(c for _, c, _ in w.get("place_in", []))
        max_molecules = min(nv, max(1024, int(placed * 1.5) + 1024))
    lat = Lattice(w["dims"], w["rv"], w["seed"], max_molecules,
                  track_displacement=w.get("track_displacement", False), device=device,
                  linear_layout=linear_layout, walls=w.get("boundary") == "walls",
                  fcc=w.get("lattice") == "fcc")
    for name, D in w["species"]:
        lat.add_species(name, D)
    for r, p, k in w["reactions"]:
        lat.add_reaction(r, p, k)
    if w.get("compartments") is not None:
        lat.set_compartments(w["compartments"])
    if place:
        for s, c in w["place"]:
            lat.place_uniform(s, c)
        for s, c, cc in w.get("place_in", []):
            lat.place_uniform_in(s, c, cc)
    return lat


class Ensemble:
    """Independent lattices advanced together in batched launches (see
    psc_ensemble_* in include/psc.h)."""

    def __init__(self, members):
        self.L = lib()
        self.members = list(members)
        arr = (C.c_void_p * len(self.members))(*[m.h for m in self.members])
        h = C.c_void_p()
        rc = self.L.psc_ensemble_create(arr, len(self.members), C.byref(h))
        if rc != PSC_OK:
            raise PscError(rc, self.L.psc_ensemble_last_error(None).decode())
        self.h = h

    def _check(self, rc):
        if rc != PSC_OK:
            raise PscError(rc, self.L.psc_ensemble_last_error(self.h).decode())

    def step(self, n_events: int, stream=None):
        s = current_stream() if stream is None else stream
        self._check(self.L.psc_ensemble_step(self.h, n_events, s))

    def sync(self):
        self._check(self.L.psc_ensemble_sync(self.h))

    def set_launch(self, items_per_thread: int = 0, stage_blocks: int = 0):
        l = Launch(items_per_thread, stage_blocks)
        self._check(self.L.psc_ensemble_set_launch(self.h, C.byref(l)))

    def get_launch(self) -> dict:
        l = Launch()
        self._check(self.L.psc_ensemble_get_launch(self.h, C.byref(l)))
        return {"items_per_thread": l.items_per_thread, "stage_blocks": l.stage_blocks}

    def read(self, i: int, stream=None) -> dict:
        """member i's state (psc_ensemble_read)"""
        s = None if stream is None else stream
        if not 0 <= i < len(self.members):
            # the library refuses it (sizes come from the member)
            self._check(self.L.psc_ensemble_read(self.h, i, C.byref(StateView()), s))
        m = self.members[i]
        return _read_view(m.nv, m.n_molecules(), m.n_rx,
                          lambda v: self._check(self.L.psc_ensemble_read(self.h, i, C.byref(v), s)))

    def autotune(self, trial_events: int):
        self._check(self.L.psc_ensemble_autotune(self.h, trial_events))

    def tuned(self) -> dict:
        l = Launch()
        ms = C.c_double()
        self._check(self.L.psc_ensemble_tuned(self.h, C.byref(l), C.byref(ms)))
        return {"items_per_thread": l.items_per_thread, "stage_blocks": l.stage_blocks,
                "ms_per_event": ms.value}

    def close(self):
        if getattr(self, "h", None):
            self.L.psc_ensemble_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ServerOptions(C.Structure):
    _fields_ = [("device", C.c_int32), ("budget_bytes", C.c_uint64),
                ("quantum_events", C.c_uint32), ("max_active", C.c_uint32),
                ("builders", C.c_uint32)]


class ReactionDesc(C.Structure):
    _fields_ = [("n_r", C.c_uint32), ("n_p", C.c_uint32), ("reactants", C.c_uint16 * 2),
                ("products", C.c_uint16 * 11), ("k", C.c_double)]


class PlaceDesc(C.Structure):
    _fields_ = [("species", C.c_uint16), ("count", C.c_uint64)]


class JobDesc(C.Structure):
    _fields_ = [("ni", C.c_uint32), ("nj", C.c_uint32), ("nk", C.c_uint32),
                ("voxel_radius", C.c_double), ("seed", C.c_uint64),
                ("max_molecules", C.c_uint64), ("flags", C.c_uint32),
                ("n_species", C.c_uint32), ("D", C.POINTER(C.c_double)),
                ("n_reactions", C.c_uint32), ("reactions", C.POINTER(ReactionDesc)),
                ("n_place", C.c_uint32), ("place", C.POINTER(PlaceDesc)),
                ("n_events", C.c_uint64), ("keep_state", C.c_uint32)]


class JobStatus(C.Structure):
    _fields_ = [("state", C.c_int32), ("error", C.c_int32), ("submit_s", C.c_double),
                ("admit_s", C.c_double), ("done_s", C.c_double), ("events_done", C.c_uint64),
                ("counters", Counters)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("admitted", C.c_uint64), ("done", C.c_uint64),
                ("failed", C.c_uint64), ("active", C.c_uint64), ("queued", C.c_uint64),
                ("device_bytes_in_use", C.c_uint64), ("attempts", C.c_uint64),
                ("quanta", C.c_uint64), ("busy_s", C.c_double), ("peak_active", C.c_uint64),
                ("cancelled", C.c_uint64)]


JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED, JOB_CANCELLED = 0, 1, 2, 3, 4


def _server_lib():
    L = lib()
    if getattr(L, "_server_bound", False):
        return L
    vp = C.c_void_p
    L.psc_server_start.argtypes = [C.c_uint64, C.c_int32, C.POINTER(vp)]
    L.psc_server_start.restype = C.c_int32
    L.psc_server_create.argtypes = [C.POINTER(ServerOptions), C.POINTER(vp)]
    L.psc_server_create.restype = C.c_int32
    L.psc_server_submit.argtypes = [vp, C.POINTER(JobDesc), C.POINTER(C.c_uint64)]
    L.psc_server_submit.restype = C.c_int32
    L.psc_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(JobStatus)]
    L.psc_server_poll.restype = C.c_int32
    L.psc_server_wait.argtypes = [vp, C.c_uint64, C.POINTER(JobStatus)]
    L.psc_server_wait.restype = C.c_int32
    L.psc_server_read_state.argtypes = [vp, C.c_uint64, C.POINTER(StateView)]
    L.psc_server_read_state.restype = C.c_int32
    L.psc_server_cancel.argtypes = [vp, C.c_uint64]
    L.psc_server_cancel.restype = C.c_int32
    L.psc_server_release.argtypes = [vp, C.c_uint64]
    L.psc_server_release.restype = C.c_int32
    L.psc_server_stats_get.argtypes = [vp, C.POINTER(ServerStats)]
    L.psc_server_stats_get.restype = C.c_int32
    L.psc_server_last_error.argtypes = [vp]
    L.psc_server_last_error.restype = C.c_char_p
    L.psc_server_job_bytes.argtypes = [C.POINTER(JobDesc), C.POINTER(C.c_uint64)]
    L.psc_server_job_bytes.restype = C.c_int32
    L.psc_server_destroy.argtypes = [vp]
    L.psc_server_destroy.restype = None
    L._server_bound = True
    return L


def _status(st: JobStatus) -> dict:
    return {"state": st.state, "error": st.error, "submit_s": st.submit_s,
            "admit_s": st.admit_s, "done_s": st.done_s, "events_done": st.events_done,
            "attempts": st.counters.attempts, "hops": st.counters.hops,
            "collisions": st.counters.collisions,
            "place_fail": st.counters.placement_failures}


class Server:
    """Continuous-batching serving loop (psc_server_* in include/psc.h);
    defaults=True starts it with psc_server_start's default options."""

    def __init__(self, budget_bytes: int, quantum_events: int = 64, max_active: int = 4096,
                 device: int = 0, builders: int = 0, defaults: bool = False):
        self.L = _server_lib()
        h = C.c_void_p()
        if defaults:
            rc = self.L.psc_server_start(budget_bytes, device, C.byref(h))
        else:
            o = ServerOptions(device, budget_bytes, quantum_events, max_active, builders)
            rc = self.L.psc_server_create(C.byref(o), C.byref(h))
        if rc != PSC_OK:
            raise PscError(rc, "server create failed")
        self.h = h
        self._meta = {}

    def _check(self, rc):
        if rc != PSC_OK:
            raise PscError(rc, self.L.psc_server_last_error(self.h).decode())

    def submit(self, w: dict, keep_state: bool = False, max_molecules: int | None = None) -> int:
        d, keep = job_desc(w, keep_state, max_molecules)
        jid = C.c_uint64()
        self._check(self.L.psc_server_submit(self.h, C.byref(d), C.byref(jid)))
        nv = int(w["dims"][0]) * int(w["dims"][1]) * int(w["dims"][2])
        self._meta[jid.value] = (nv, len(w["reactions"]))
        return jid.value

    @staticmethod
    def job_bytes(w: dict, max_molecules: int | None = None) -> int:
        d, keep = job_desc(w, False, max_molecules)
        b = C.c_uint64()
        rc = _server_lib().psc_server_job_bytes(C.byref(d), C.byref(b))
        if rc != PSC_OK:
            raise PscError(rc, "job_bytes")
        return b.value

    def poll(self, job_id: int) -> dict:
        st = JobStatus()
        self._check(self.L.psc_server_poll(self.h, job_id, C.byref(st)))
        return _status(st)

    def wait(self, job_id: int) -> dict:
        st = JobStatus()
        self._check(self.L.psc_server_wait(self.h, job_id, C.byref(st)))
        return _status(st)

    def read_state(self, job_id: int, max_molecules: int) -> dict:
        nv, n_rx = self._meta[job_id]
        occ = np.zeros(nv, np.uint16)
        arrays = {k: np.zeros(max_molecules, t) for k, t in (
            ("id", np.uint32), ("vox", np.uint32), ("species", np.uint16), ("dx", np.int32),
            ("dy", np.int32), ("dz", np.int32))}
        fired = np.zeros(max(n_rx, 1), np.uint64)
        v = StateView()
        v.occupancy = _ptr(occ, C.c_uint16)
        v.n_molecules = max_molecules
        v.id = _ptr(arrays["id"], C.c_uint32)
        v.voxel = _ptr(arrays["vox"], C.c_uint32)
        v.species = _ptr(arrays["species"], C.c_uint16)
        v.dx, v.dy, v.dz = (_ptr(arrays[k], C.c_int32) for k in ("dx", "dy", "dz"))
        v.reactions_fired = _ptr(fired, C.c_uint64)
        self._check(self.L.psc_server_read_state(self.h, job_id, C.byref(v)))
        n = v.n_molecules
        out = {k: a[:n].copy() for k, a in arrays.items()}
        out.update(occ=occ, attempts=v.counters.attempts, hops=v.counters.hops,
                   collisions=v.counters.collisions, place_fail=v.counters.placement_failures,
                   fired=fired[:n_rx].copy(), event=v.event, time=v.time, next_id=v.next_id)
        return out

    def cancel(self, job_id: int):
        self._check(self.L.psc_server_cancel(self.h, job_id))

    def release(self, job_id: int):
        self._check(self.L.psc_server_release(self.h, job_id))

    def stats(self) -> dict:
        s = ServerStats()
        self._check(self.L.psc_server_stats_get(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.L.psc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def job_desc(w: dict, keep_state: bool = False, max_molecules: int | None = None):
    """psc_job_desc for a workload dict; the second value keeps the arrays
    the descriptor points to alive"""
    nv = int(w["dims"][0]) * int(w["dims"][1]) * int(w["dims"][2])
    placed = sum(c for _, c in w["place"])
    if max_molecules is None:
        max_molecules = min(nv, max(1024, int(placed * 1.5) + 1024))
    D = (C.c_double * max(len(w["species"]), 1))(*[d for _, d in w["species"]])
    rxs = (ReactionDesc * max(len(w["reactions"]), 1))()
    for i, (r, p, k) in enumerate(w["reactions"]):
        rxs[i].n_r, rxs[i].n_p, rxs[i].k = len(r), len(p), k
        for a, x in enumerate(r):
            rxs[i].reactants[a] = x
        for a, x in enumerate(p):
            rxs[i].products[a] = x
    pl = (PlaceDesc * max(len(w["place"]), 1))(*[PlaceDesc(s, c) for s, c in w["place"]])
    d = JobDesc()
    d.ni, d.nj, d.nk = (int(x) for x in w["dims"])
    d.voxel_radius = w["rv"]
    d.seed = w["seed"]
    d.max_molecules = max_molecules
    d.flags = (TRACK_DISPLACEMENT if w.get("track_displacement") else 0) | (
        BOUNDARY_WALLS if w.get("boundary") == "walls" else 0) | (
        LATTICE_FCC if w.get("lattice") == "fcc" else 0)
    d.n_species, d.D = len(w["species"]), D
    d.n_reactions, d.reactions = len(w["reactions"]), rxs
    d.n_place, d.place = len(w["place"]), pl
    d.n_events = w["events"]
    d.keep_state = 1 if keep_state else 0
    return d, (D, rxs, pl)
