"""The benchmark's command-line contract and its flop models (CPU only)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_henon_heiles_flop_model():
    # per step: 3 drifts (12) + 4 state kicks (16) + 3 forces (18) + 3 scaled
    # Hessians (15) + 6 vectors x (3 kicks x 8 + 3 drifts x 4) + LD (6) = 283;
    # checkpoint / 10: 2 renormalisations (26), SALI (22), 4-vector MGS
    # (4 x 13 + 6 x 15 = 142), energy (14) -> 19.8
    assert bench.flops_per_step(2, 2, 4, True, True, True, 10) == pytest.approx(302.8)
    # the gate's and the batched form's two-vector kernels
    assert bench.flops_per_step(2, 2, 0, True, False, True, 10) == pytest.approx(143.6)
    assert bench.flops_per_step(2, 2, 0, False, True, True, 10) == pytest.approx(139.0)


def test_dop853_flop_model():
    # per stage: FMA per non-zero a_ij and component (50 in all) + the add to
    # the start value; state: 12 forces (6) and h-scalings (4); vectors: 12
    # scaled Hessians (5), 2x2 mat-vecs (8) and h-scalings (2); final sums
    # over the 8 weighted stages; LD at those stages; checkpoints / 10
    # as for Yoshida-4
    sums = 2 * 4 * 50 + 4 * 11
    final = 2 * 4 * 8 + 4
    state = sums + 12 * 6 + 12 * 4 + final
    vec = sums + 12 * (5 + 8 + 2) + final
    assert bench.flops_per_step_dop853(2, 2, 4, True, True, True, 10) == pytest.approx(
        state + 6 * vec + 8 * 5 + 2 + 19.8)
    assert bench.DOP853_ROW_NNZ == (0, 1, 2, 2, 3, 3, 4, 5, 6, 7, 8, 9)


def test_adaptive_attempt_flop_model():
    # the fixed step with LD and 2 vectors (state 632 + 2 x 692 + LD 42) plus,
    # for each of the 12 components, the fifth-order difference (8 FMA), the
    # third-order difference (3 FMA), the scale (FMA) and two squared ratios
    # (FMA), plus 8 for the controller
    assert bench.flops_per_attempt_dop853(2, 2, 0, True) == pytest.approx(
        632 + 2 * 692 + 42 + 12 * (16 + 6 + 2 + 4) + 8)


def test_dop853_tableau_pattern_matches_the_oracle():
    from oracle import oracle as O
    c, a, b = O.dop853_tableau()
    assert tuple(int(v) for v in (a != 0).sum(axis=1)) == bench.DOP853_ROW_NNZ
    assert int((b != 0).sum()) == bench.DOP853_B_NNZ


def test_mlp_training_flop_model():
    # products of one row: forward 2 (6*256 + 256*256 + 256*2), the same
    # for the weight gradients, activation gradients 2 (2*256 + 256*256)
    assert bench.mlp_train_flops_per_row() == 135168 + 135168 + 132096
    assert bench.mlp_train_flops_per_row(True) == 147456 + 147456 + 139264


def test_fput_and_quartic_flop_models():
    assert bench.flops_per_step_fput(16, 16, 32, False, True, True, 10) == pytest.approx(26202.0)
    assert bench.flops_per_step_fput(8, 8, 16, False, True, True, 10) == pytest.approx(5999.6)
    assert bench.flops_per_step_fput(16, 2, 0, False, True, True, 10) == pytest.approx(1797.2)
    assert bench.flops_per_step_quartic(3, 2, False, True, True, 10) == pytest.approx(333.8)
    # the vector work grows like M N and the Gram-Schmidt like n_l^2 N
    a = bench.flops_per_step_fput(16, 0, 8, False, False, False, 10)
    b = bench.flops_per_step_fput(16, 0, 16, False, False, False, 10)
    assert b - a > 8 * 24 * 16


def test_traffic_record_needs_matching_kernel_code(tmp_path, monkeypatch):
    f = tmp_path / "t.md"
    f.write_text("kernel-code-sha256: `deadbeef`\ntraffic-bytes-per-launch: `123`\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.recorded_traffic() is None
    monkeypatch.setattr(bench, "kernel_code_hash", lambda: "deadbeef")
    assert bench.recorded_traffic() == 123.0


def test_kernel_code_hash_finds_the_benchmarked_kernel():
    # the built library holds the kernel's gfx950 code and descriptor; a
    # symbol that is not there gives None
    h = bench.kernel_code_hash()
    assert h is not None and len(h) == 64
    assert bench.kernel_code_hash(symbol="_Z_no_such_kernel") is None
