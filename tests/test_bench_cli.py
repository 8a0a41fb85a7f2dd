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
