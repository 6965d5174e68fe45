"""Host logic of bench.py, on the CPU: the one-GPU guard, the reader of the
committed walk-stage traffic summary (used only while the kernel source
matches the one the counters were taken on), the workload picker and the
oracle baseline leg's fields."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 2
    assert p.stdout == ""
    assert "one GPU" in p.stderr and "--gpus 2" in p.stderr


def summary(sha, per_dispatch="159800000", per_attempt="229.6"):
    return "\n".join(["# HBM traffic of the walk-stage kernel (k_stage), workload w",
                      "# fetch command: rocprofv3 --pmc FETCH_SIZE ...",
                      "source_sha: %s" % sha,
                      "traffic_bytes_per_dispatch: %s" % per_dispatch,
                      "traffic_bytes_per_attempt: %s" % per_attempt]) + "\n"


def test_traffic_summary_is_read_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    assert bench.read_traffic("w") is None                       # no summary
    f = tmp_path / "walk_stage_traffic_w.txt"
    f.write_text(summary(bench.kernel_source_sha()))
    assert bench.read_traffic("w") == {"per_dispatch": 159800000.0, "per_attempt": 229.6}
    f.write_text(summary("0" * 16))                              # another source
    assert bench.read_traffic("w") is None
    f.write_text(summary(bench.kernel_source_sha(), per_attempt="n/a"))
    assert bench.read_traffic("w") is None


def test_kernel_source_sha_covers_every_kernel_source(tmp_path, monkeypatch):
    """The hash covers the walk-stage kernel's translation units and every
    local header they include, directly or not."""
    sha = bench.kernel_source_sha()
    assert len(sha) == 16 and int(sha, 16) >= 0
    csrc = tmp_path / "paper_1605_03726_amd" / "csrc"
    csrc.mkdir(parents=True)
    src = os.path.join(ROOT, "paper_1605_03726_amd", "csrc")
    closure, todo = set(), ["psc_stage_hcp.hip", "psc_stage_fcc.hip"]
    while todo:
        f = todo.pop()
        if f in closure or not os.path.exists(os.path.join(src, f)):
            continue
        closure.add(f)
        for line in open(os.path.join(src, f)):
            if line.startswith('#include "'):
                todo.append(line.split('"')[1])
    assert set(bench.KERNEL_SOURCES) == closure
    for f in bench.KERNEL_SOURCES:
        (csrc / f).write_bytes(open(os.path.join(src, f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_sha() == sha
    for f in bench.KERNEL_SOURCES:
        original = (csrc / f).read_bytes()
        (csrc / f).write_bytes(original + b"\n")
        assert bench.kernel_source_sha() != sha, f
        (csrc / f).write_bytes(original)
    assert bench.kernel_source_sha() == sha


def test_workload_picker():
    w = bench.pick_workload("cfg3")
    assert tuple(w["dims"]) == (2048, 2048, 1024)
    m = bench.pick_workload("multiproduct")
    assert m["name"] == "multiproduct_256x256x256" and tuple(m["dims"]) == (256, 256, 256)
    assert m["track_displacement"] is False
    with pytest.raises(SystemExit):
        bench.pick_workload("nonesuch")


def test_cpu_baseline_fields():
    w = dict(bench.pick_workload("cfg1"))
    r = bench.cpu_baseline(w, 2)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["unit"] == "attempts/s"
    assert r["value"] > 0
    assert "first 2 events of %s" % w["name"] in r["sample"]
    # the same events in the paper's order: the same number of attempts
    # (no reactions in this workload), timed on its own
    seq = r["sequential_order"]
    assert seq["value"] > 0 and seq["cores"] == 1 and seq["attempts"] > 0
    assert r["host_cpus"] >= 1 and 1 <= r["host_cpus_usable"] <= r["host_cpus"]


@pytest.mark.parametrize("lattice,dims", [("hcp", (16, 16, 16)), ("fcc", (16, 16, 24))])
def test_cross_brick_fraction_is_the_stencils(lattice, dims):
    """The share of hops whose target lies in another 4x4x4 brick, counted
    over every voxel and direction of the oracle's neighbour table on a
    periodic box that holds whole bricks and whole stencil periods."""
    import numpy as np

    import oracle
    nb = oracle.neighbour_table_l(dims, oracle.FCC if lattice == "fcc" else oracle.HCP)
    nv = nb.shape[0]

    def brick(u):
        return (u % dims[0]) // 4, (u // dims[0]) % dims[1] // 4, u // (dims[0] * dims[1]) // 4
    src = np.repeat(np.arange(nv), 12)
    same = np.all(np.array(brick(src)) == np.array(brick(nb.ravel())), axis=0)
    assert (1.0 - same.mean()) == bench.CROSS_BRICK_FRACTION[lattice]
