"""Argument handling of bench.py (CPU only): any K >= 1 timed and W >= 0 warm-up Trotter
steps are accepted, and the C(t) pair plus the odd extra step time exactly K steps."""
import pytest

import bench


@pytest.mark.parametrize("K,W", [(20, 5), (1, 0), (7, 3), (2, 0), (60, 6)])
def test_accepts_driver_arguments(K, W):
    args = bench.parse_args(["--steps", str(K), "--warmup", str(W)])
    assert (args.steps, args.warmup, args.gpus) == (K, W, 1)
    for k in (K, W):
        pairs, extra = bench.step_split(k)
        assert 2 * pairs + extra == k and extra in (0, 1)


def test_defaults_are_single_gpu():
    args = bench.parse_args([])
    assert args.gpus == 1 and args.steps >= 1 and args.warmup >= 0


@pytest.mark.parametrize("argv", [["--steps", "0"], ["--warmup", "-1"], ["--dtypes", "c32"]])
def test_rejects_bad_arguments(argv):
    with pytest.raises(SystemExit):
        bench.parse_args(argv)


def test_more_than_one_gpu_exits_with_message(capsys):
    with pytest.raises(SystemExit) as e:
        bench.main(["--gpus", "8"])
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err


def test_algorithmic_bytes_floor():
    # N = 27 complex128: 20 layers x (read + write) x 2 GiB = 85.9 GB per Trotter step
    assert bench.algorithmic_bytes_per_step(27, 16) == 20 * 2 * (1 << 27) * 16
    assert abs(bench.algorithmic_bytes_per_step(27, 16) / 1e9 - 85.9) < 0.05
