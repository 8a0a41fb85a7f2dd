"""bench.py's command-line contract on the CPU: more than one GPU is refused with a message,
and the per-kernel byte model matches the closed forms stated for each kernel."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_byte_model_closed_forms():
    N, s, M = 1000, 8, 8
    # extrapolation: k stored slots + the FP64 guess; ring store: FP64 in, one slot out
    assert bench.kernel_bytes("extrap", "form", N, s, 8, M, False) == [N * (8 * s + 8)]
    assert bench.kernel_bytes("extrap", "update", N, s, 8, M, False) == [N * (8 + s)]
    # projection form at d columns: dots d s + 8, combine d s + 8
    assert sum(bench.kernel_bytes("proj", "form", N, s, 5, M, False)) == 2 * N * (5 * s + 8)
    # classic Gram-Schmidt update at d: 5 d s + 2 s + 40; restart 8 + 2 s
    assert sum(bench.kernel_bytes("proj", "update", N, s, 5, M, False)) == N * (5 * 5 * s + 2 * s + 40)
    assert sum(bench.kernel_bytes("proj", "update", N, s, 0, M, True)) == N * (8 + 2 * s)
    # l2 form reads B only in the second pass: 4 d s + 2 s + 40
    assert sum(bench.kernel_bytes("proj_l2", "update", N, s, 5, M, False)) == N * (4 * 5 * s + 2 * s + 40)
    # rolling drop at d = M: 7 M s + 40
    assert sum(bench.kernel_bytes("projqr", "update", N, s, M, M, False)) == N * (7 * M * s + 40)
    # variable coefficient: the fused apply also reads the face arrays
    assert bench.kernel_bytes("proj", "update", N, s, 5, M, False, faces=123)[0] == N * (16 + 5 * s) + 123
    # FP16: the Gram-Schmidt pass also forms x - X c1 (for the pair's exponent), a restart
    # writes A x before the pair is stored, and a ring store may store its slot twice
    assert sum(bench.kernel_bytes("proj_l2", "update", N, 2, 5, M, False, dtype="f16")) == N * (5 * 5 * 2 + 4 + 48)
    assert sum(bench.kernel_bytes("proj", "update", N, 2, 0, M, True, dtype="f16")) == N * (32 + 4)
    assert bench.kernel_bytes("extrap", "update", N, 2, 8, M, False, dtype="f16") == [N * 10, 0]
    assert bench.kernel_bytes("extrap", "update", N, 2, 8, M, False, dtype="f16", fixed=True) == [N * 10, N * 10]
    assert bench.kernel_names("extrap", "update", "f16") == ["ring_store", "ring_fix"]


def test_mode_flags_parse(monkeypatch):
    """The measurement modes and their options are accepted (they run only on a GPU)."""
    for argv, check in (
        (["--isolated", "--shard-nz", "32"], lambda a: a.isolated and a.shard_nz == 32),
        (["--adjoint", "--adjoint-n", "64", "--adjoint-steps", "10"],
         lambda a: a.adjoint and a.adjoint_n == 64 and a.adjoint_steps == 10),
        (["--concurrent", "--n", "64"], lambda a: a.concurrent and a.n == 64),
        (["--no-small-sequence", "--no-cpu-baseline"], lambda a: not a.small and not a.cpu),
        (["--fields", "ins", "--rhs", "gaussian", "--stop-rule", "initresid"],
         lambda a: a.fields == "ins" and a.rhs == "gaussian" and a.stop_rule == "initresid"),
        ([], lambda a: a.eps_rel == 0.0 and a.small and a.cpu and a.steps == 20 and a.warmup == 10),
    ):
        monkeypatch.setattr(sys, "argv", ["bench.py"] + argv)
        assert check(bench.parse()), argv


def test_read_write_split_and_mixed_roof():
    """Every kernel's bytes split into read and written parts that sum to the byte model, and
    the mixed roof is the harmonic combination of the read and write roofs."""
    N, M = 1000, 8
    for method in ("extrap", "last", "spextrap", "proj", "projqr", "proj_l2", "projqr_l2"):
        for dtype, s in (("f64", 8), ("f32", 4), ("f16", 2), ("bf16", 2)):
            for call in ("form", "update"):
                for d in range(0, M + 1):
                    for restart in (False, True):
                        rw = bench.kernel_rw(method, call, N, s, d, M, restart, 0, dtype, True)
                        assert [r + w for r, w in rw] == bench.kernel_bytes(method, call, N, s, d, M, restart, 0,
                                                                           dtype, True)
    # extrapolation form reads k s and writes 8; ring store reads 8 and writes s
    assert bench.kernel_rw("extrap", "form", N, 8, 8, M, False) == [(N * 64, N * 8)]
    assert bench.kernel_rw("extrap", "update", N, 8, 8, M, False) == [(N * 8, N * 8)]
    assert bench.mixed_roof(1.0, 0.0, 6000.0, 5000.0) == 6000.0
    assert bench.mixed_roof(0.0, 1.0, 6000.0, 5000.0) == 5000.0
    assert abs(bench.mixed_roof(1.0, 1.0, 6000.0, 4000.0) - 4800.0) < 1e-9


def test_traffic_summary_from_counter_csvs(tmp_path, monkeypatch):
    """--traffic-summary: counters scaled by the copy kernel's reading, totals over the launches
    that moved data (a launch that returns at once is left out), beside the profiled run's own
    algorithmic bytes; the summary names its sources' hash so that the bench can tell it is
    current."""
    import csv
    import json
    import types

    def write(folder, rows):
        folder.mkdir()
        with open(folder / "x_counter_collection.csv", "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for r in rows:
                w.writerow(r)

    kib = 1024.0
    row = lambda k, c, v: {"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v}  # noqa: E731
    # copy kernel of 1 GiB -> 1 GiB: FETCH_SIZE reads half, WRITE_SIZE all
    write(tmp_path / "fc", [row("lg::copy_kernel(a)", "FETCH_SIZE", (1 << 30) / 2 / kib)])
    write(tmp_path / "wc", [row("lg::copy_kernel(a)", "WRITE_SIZE", (1 << 30) / kib)])
    # proj_dots: two launches of 800 KiB read (counter reads half), one that returned at once
    write(tmp_path / "f", [row("void lg::proj_dots_kernel<0, 0>(a)", "FETCH_SIZE", 400.0)] * 2 +
          [row("void lg::proj_dots_kernel<0, 0>(a)", "FETCH_SIZE", 0.5),
           row("void lg::pcg_b_kernel<false>(a)", "FETCH_SIZE", 8.0)])
    write(tmp_path / "w", [row("void lg::proj_dots_kernel<0, 0>(a)", "WRITE_SIZE", 1.0)] * 2 +
          [row("void lg::pcg_b_kernel<false>(a)", "WRITE_SIZE", 8.0)])
    run = {"config": {"n": 16, "workload": "test"}, "kernels": {"proj_dots": {"bytes_per_launch": 800 * kib,
                                                                               "launches": 2}}}
    (tmp_path / "f" / "bench.json").write_text(json.dumps(run) + "\n")
    profiles = tmp_path / "root" / "profiles"
    profiles.mkdir(parents=True)
    for f in bench.TRAFFIC_SOURCES:
        (tmp_path / "root" / f).parent.mkdir(parents=True, exist_ok=True)
        (tmp_path / "root" / f).write_text(f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path / "root"))
    args = types.SimpleNamespace(traffic_summary=[str(tmp_path / d) for d in ("f", "w", "fc", "wc")])
    bench.traffic_summary(args)
    rec = {}
    for line in open(profiles / "hbm_traffic.txt"):
        if line.strip() and not line.startswith("#"):
            k, v = line.split("=", 1)
            rec[k.strip()] = v.strip()
    assert float(rec["fetch_scale"]) == 2.0 and float(rec["write_scale"]) == 1.0
    assert float(rec["proj_dots.read_bytes_per_launch"]) == 800 * kib
    assert float(rec["proj_dots.write_bytes_per_launch"]) == kib
    assert rec["proj_dots.ratio"] == f"{801 / 800:.4f}"
    assert float(rec["pcg_b.algorithmic_bytes_per_launch"]) == 24 * 16 ** 3
    assert bench.hbm_traffic("proj_dots") == (801 * kib, 800 * kib)
