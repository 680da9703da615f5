"""bench.py's arithmetic and contract paths that need no GPU: level sizes and
seed counts, the algorithmic byte model (every candidate gather of the
schedule counted once), the per-kernel roofline table, the kernel-code hash
that gates the traffic figure, and the one-GPU message for --gpus > 1."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_level_dims_and_seed_counts():
    assert bench.level_dims(1242, 375, 4) == [(1242, 375), (621, 187), (310, 93), (155, 46)]
    # coarsest 155 x 46, seeds on a stride-3 grid from the origin: 52 x 16
    assert bench.seed_counts(1242, 375, 4) == (52 * 16, 155 * 46)
    assert bench.seed_counts(1242, 375, 1) == (414 * 125, 1242 * 375)
    assert bench.seed_counts(7, 5, 1, stride=3) == (3 * 2, 35)


def test_byte_model_counts_every_gather_of_the_schedule():
    """Row phase: LR + RL sweeps (one gather each) and one random-search
    pass of J = 5 trials at R = 16; column phase: TB and BT sweeps and two
    passes; each phase also reads the own descriptor (16 B) and the state
    (8 B) once and writes the state (8 B) once."""
    J = (16).bit_length()
    assert J == 5
    assert bench.ROW_BYTES_PER_PX == (2 + J) * 16 + 16 + 8 + 8
    assert bench.COL_BYTES_PER_PX == (2 + 2 * J) * 16 + 16 + 8 + 8
    assert bench.CEN_COL_BYTES_PER_PX == (2 + 2 * J) * 8 + 2 * 8 + 8 + 8
    # the roofline's per-launch figure: 2 iterations x 4 levels x 2 phases
    # per step, both directions, 64 pairs; col launches average over 8
    px = sum(w * h for w, h in bench.level_dims(bench.W0, bench.H0, bench.LEVELS))
    per_launch = bench.COL_BYTES_PER_PX * px * 2 * 64 * 2 / 8
    assert per_launch == pytest.approx(4.428655616e9)


def test_kernel_rooflines_from_a_profile():
    steps, batch = 4, 64
    prof = {"col_phase": (8 * steps, 4.0 * steps), "row_phase": (8 * steps, 3.0 * steps), "fb": (steps, 0.4 * steps)}
    out = bench.kernel_rooflines(prof, batch, steps)
    assert set(out) == {"col_phase", "row_phase", "fb"}
    col = out["col_phase"]
    assert col["us_per_step"] == pytest.approx(4000.0)
    assert col["bytes_per_step"] == 2 * bench.COL_BYTES_PER_PX * sum(
        w * h for w, h in bench.level_dims(bench.W0, bench.H0, bench.LEVELS)) * 2 * batch
    assert col["frac"] == pytest.approx(col["achieved"] / bench.HBM_PEAK_GBS)
    assert col["achieved"] == pytest.approx(col["bytes_per_step"] / 4e-3 / 1e9)


def test_kernel_hash_ignores_comments_and_follows_code(tmp_path):
    """The traffic figure is reported only for the kernel code it was
    measured on: comment and blank-line edits keep the hash, code edits
    change it."""
    a = tmp_path / "a.hip"
    a.write_text("int f(int x)\n{\n    return x + 1;   // one more\n}\n")
    b = tmp_path / "b.hip"
    b.write_text("// a header comment\nint f(int x)\n{\n\n    return x + 1;   // a different note\n}\n")
    c = tmp_path / "c.hip"
    c.write_text("int f(int x)\n{\n    return x + 2;   // one more\n}\n")
    assert bench.kernel_sha(str(a)) == bench.kernel_sha(str(b))
    assert bench.kernel_sha(str(a)) != bench.kernel_sha(str(c))
    assert len(bench.kernel_sha()) == 16


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
