"""Host-side logic of bench.py (no GPU): the one-GPU guard, the lookup of
counted HBM traffic by kernel and source hash, and the roofline arithmetic."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}),
                                      ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ)
    e.update(env)
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv],
                       capture_output=True, text=True, env=e, timeout=120)
    assert p.returncode == 2
    assert p.stdout == ""
    assert "one GPU" in p.stderr


def test_traffic_lookup_by_kernel_and_source_hash(tmp_path, monkeypatch):
    src = bench.sweep_source_hash()
    f = tmp_path / "pmc.txt"
    f.write_text("# counters\n"
                 f"traffic fofr fp32 512 1 {src} 1.5e9 5.0e8\n"
                 f"traffic symmetron fp32 512 2 {src} 2.5e9 5.0e8\n"
                 "traffic fofr fp64 512 1 0000000000000000 9e9 9e9\n"
                 "traffic fofr fp32 512 1 junk\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("fofr", "fp32", 512, 1) == pytest.approx(2.0e9)
    assert bench.measured_traffic("symmetron", "fp32", 512, 2) == pytest.approx(3.0e9)
    # recorded for other sources (the kernel changed since): not reported
    assert bench.measured_traffic("fofr", "fp64", 512, 1) is None
    # another temporal block or grid is another kernel
    assert bench.measured_traffic("symmetron", "fp32", 512, 1) is None
    assert bench.measured_traffic("fofr", "fp32", 256, 1) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("fofr", "fp32", 512, 1) is None


def test_source_hash_tracks_the_sweep_sources(tmp_path, monkeypatch):
    h0 = bench.sweep_source_hash()
    assert len(h0) == 16 and int(h0, 16) >= 0
    for rel in bench.SWEEP_SOURCES:
        d = tmp_path / os.path.dirname(rel)
        d.mkdir(parents=True, exist_ok=True)
        with open(os.path.join(ROOT, rel), "rb") as fh:
            (tmp_path / rel).write_bytes(fh.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.sweep_source_hash() == h0
    p = tmp_path / bench.SWEEP_SOURCES[1]
    p.write_bytes(p.read_bytes() + b"\n")
    assert bench.sweep_source_hash() != h0


def test_committed_traffic_lines_are_well_formed():
    lines = [ln.split() for ln in open(bench.TRAFFIC_FILE) if ln.startswith("traffic ")]
    assert lines
    for f in lines:
        assert len(f) == 8
        assert f[1] in bench.MODEL_TYPES and f[2] in bench.TYPES
        assert int(f[3]) > 0 and int(f[4]) in (1, 2) and len(f[5]) == 16
        assert float(f[6]) > 0 and float(f[7]) > 0
    # the dominant kernel of the benchmark (FP32 f(R), one sweep per pass)
    assert any(f[1:5] == ["fofr", "fp32", "512", "1"] for f in lines)


def test_roofline_head_is_the_kernel_with_most_time(monkeypatch):
    monkeypatch.setattr(bench, "measured_traffic", lambda *a: None)
    n = 512
    b32 = 3 * 4 * n ** 3
    kern = {
        ("symmetron", "fp32"): dict(ms=10 * 0.6, launches=10, bytes=10 * b32, tb=2),
        ("fofr", "fp32"): dict(ms=52 * 0.4, launches=52, bytes=52 * b32, tb=1),
    }
    head, ks = bench.roofline(kern, n)
    assert [k["model"] for k in ks] == ["fofr", "symmetron"]
    assert head["model"] == "fofr" and head["bound"] == "hbm" and head["unit"] == "GB/s"
    assert head["avg_launch_ms"] == pytest.approx(0.4)
    assert head["achieved"] == pytest.approx(b32 / 0.4e-3 / 1e9)
    assert head["frac"] == pytest.approx(head["achieved"] / 8000.0)
    assert head["peak"] == 8000.0 and head["traffic"] is None
    assert ", 1, " in head["kernel"] and ", 2, " in ks[1]["kernel"]


def test_solve_bytes_counts_every_kernel_once():
    """The whole-solve byte model of the benchmark's roofline, by hand on a
    16^3 FP64 solve of one V-cycle (levels 16, 8, 4; per-colour kernels): the
    density hierarchy (8 B per cell over 8/7 of the cells), cold start and
    r_ref (32 B), per level 4 smoothing passes of 3 (4 with Sigma) values, the
    descent, the coarse source, the correction, the 4^3 level and the judge."""
    import types

    import bench
    n3 = 16 ** 3
    st = types.SimpleNamespace(cycles=1, cycles_fp32=0, restriction=0)
    want = n3 * (8 * 8 / 7 + 32)
    want += n3 * (4 * 3 * 8 + (2 * 8 + 3) + 4 + (16 + 2))          # level 16
    want += 512 * (4 * 4 * 8 + (3 * 8 + 3) + 4 + (16 + 2))          # level 8
    want += 64 * 4 * 8                                               # level 4
    want += n3 * 16                                                  # judge
    assert abs(bench.solve_bytes(16, st, 0, (2, 2), False) - want) <= 1e-9 * want
    # full weighting adds the fine defect's write and read on levels 16 and 8
    st.restriction = 1
    fw = want + 2 * 8 * (n3 + 512)
    assert abs(bench.solve_bytes(16, st, 0, (2, 2), False) - fw) <= 1e-9 * fw
    # in single precision only below 64^3: a 128^3 FP32 cycle's levels 128 and
    # 64 restrict by full weighting in one pass, levels 32, 16 and 8 in two
    st32 = types.SimpleNamespace(cycles=1, cycles_fp32=1, restriction=0, judged_cycles=1)
    mean = bench.solve_bytes(128, st32, 0, (2, 2), True)
    st32.restriction = 1
    got = bench.solve_bytes(128, st32, 0, (2, 2), True)
    assert abs(got - mean - 2 * 4 * (32 ** 3 + 16 ** 3 + 8 ** 3)) <= 1e-9 * got
    # tiled descents (sides >= 64) write Sigma_c themselves: only eta_c is
    # read for it, instead of the coarse source's 4 values per coarse cell
    c64 = 64 ** 3
    lvl = c64 * 8 * (4 * 4 + (3 + 3 / 8) + 1 / 8 + 2 / 8 + 2)
    assert abs(bench.level_bytes(64, 8, 4, True, False, False) - lvl) <= 1e-9 * lvl
    assert abs(bench.level_bytes(64, 8, 4, True, True, False)
               - (lvl + c64 * 8 * (2 + 3 / 8))) <= 1e-9 * lvl    # FP64 full weighting: two passes
    assert abs(bench.level_bytes(64, 4, 4, True, True, False) - lvl / 2) <= 1e-9 * lvl
    # restriction 2: full weighting in the first two cycles, the mean after
    st2 = types.SimpleNamespace(cycles=4, cycles_fp32=0, restriction=2)
    st0 = types.SimpleNamespace(cycles=2, cycles_fp32=0, restriction=0)
    st1 = types.SimpleNamespace(cycles=2, cycles_fp32=0, restriction=1)
    base = bench.solve_bytes(16, types.SimpleNamespace(cycles=0, cycles_fp32=0, restriction=0),
                             0, (2, 2), False)
    mixed = bench.solve_bytes(16, st2, 0, (2, 2), False)
    parts = (bench.solve_bytes(16, st0, 0, (2, 2), False) - base
             + bench.solve_bytes(16, st1, 0, (2, 2), False) - base + base)
    assert abs(mixed - parts) <= 1e-9 * mixed
    # a light judge (FP32 iterate and FP32 density) instead of the FP64 judge
    # of an FP32 iterate (FP32 iterate and FP64 density): 4 B per cell less
    stl = types.SimpleNamespace(cycles=3, cycles_fp32=2, restriction=0, judged_cycles=3,
                                judged_fp32=1)
    st64j = types.SimpleNamespace(cycles=3, cycles_fp32=2, restriction=0, judged_cycles=3)
    d = bench.solve_bytes(128, st64j, 0, (2, 2), True) - bench.solve_bytes(128, stl, 0, (2, 2), True)
    assert abs(d - 4 * 128 ** 3) <= 1e-9 * 128 ** 3
    # the fused sweep levels (>= 256^3, temporal block >= 1) apply the
    # correction inside the first post-smoothing pass: no pass of its own
    st512 = types.SimpleNamespace(cycles=1, cycles_fp32=1, restriction=0, judged_cycles=1)
    plain = bench.solve_bytes(512, st512, 0, (2, 2), True)
    fused = bench.solve_bytes(512, st512, 1, (2, 2), True)
    assert abs(plain - fused - 2 * 4 * (512 ** 3 + 256 ** 3)) <= 1e-9 * plain
    # not with two sweeps per pass: there the correction keeps its own pass
    # (and the two post-smoothing sweeps take one pass instead of two)
    tb2 = bench.solve_bytes(512, st512, 2, (2, 2), True)
    assert abs(fused - tb2 - 2 * 12 * (512 ** 3 + 256 ** 3) - 2 * 4 * (256 ** 3)
               + 2 * 4 * (512 ** 3 + 256 ** 3)) <= 1e-9 * plain
