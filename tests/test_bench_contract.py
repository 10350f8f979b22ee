"""bench.py on the CPU: its refusals (more than one GPU, no GPU visible) and the
byte / flop models and committed traffic figure its roofline line is built on."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _run(*args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=300)


def test_more_than_one_gpu_is_refused():
    for args, extra in ((("--gpus", "2"), None), ((), {"WORLD_SIZE": "4"})):
        r = _run(*args, env_extra=extra)
        assert r.returncode == 2
        assert "one GPU" in r.stderr
        assert r.stdout.strip() == ""  # no JSON line


def test_no_gpu_fails_without_a_number():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    r = _run("--no-extras", "--no-cpu-baseline", "--steps", "1", "--warmup", "0")
    assert r.returncode != 0
    assert "no GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_models(bench):
    # read x and write y once, K once per element: 8 + 8 + 8/64 B at Q3 in FP64
    assert bench.alg_bytes_per_dof(4, 8, 8, 8) == 16.125
    assert bench.alg_bytes_per_dof(4, 4, 4, 4) == 8.0625
    assert bench.alg_bytes_per_dof(5, 2, 4, 4) == 6 + 4 / 125
    # affine 14 n + 48, trilinear 24 n + 288 + 810 / n (about 581 at n = 8)
    assert bench.flops_per_dof(4) == 104
    assert bench.flops_per_dof(8, trilinear=True) == 24 * 8 + 288 + 810 / 8
    assert abs(bench.flops_per_dof(8, trilinear=True) - 581) < 1


def test_committed_traffic_figure(bench):
    """The traffic figure is either withheld (kernel sources changed since the
    counters were taken) or the committed one, between the algorithmic bytes and
    twice them for the 32,768,000-DOF headline launch (64^3 Q4)."""
    assert bench.HEADLINE == "mixed_q4_64"
    t = bench.measured_traffic()
    if t is None:
        pytest.skip("kernel sources changed since the HBM counters were taken")
    alg = (16 + 8 / 125) * 32768000
    assert alg <= t <= 2 * alg
