"""The benchmark's host-side pieces on the CPU: the one-GPU contract, the
counted cost model, and the rule that HBM traffic is reported only for the
sources the committed counter summary was taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_cost_model_counts():
    # T10 5-point rule: 12 + 21 + 20 + 20 + 19 non-zero parent-gradient entries
    assert sum(bench.NZ[bench.T10]) == 92
    fwd = bench.flops_per_element("fwd", bench.T10, bench.NH, True)
    vjp = bench.flops_per_element("vjp", bench.T10, bench.NH, True)
    assert (fwd, vjp) == (4293, 7647)
    # the adjoint counts the parameter rows only when they are wanted
    assert bench.flops_per_element("vjp", bench.T10, bench.NH, True, gtheta=True) > vjp
    # damping adds work in every operation
    for op in ("fwd", "vjp", "jvp"):
        assert bench.flops_per_element(op, bench.T10, bench.NH, True) > bench.flops_per_element(op, bench.T10, bench.NH, False)
    # compulsory bytes: X, x, v, f at 24 B per node plus int32 connectivity
    assert bench.bytes_per_call("fwd", 100, 10, 10, True) == 4 * 24 * 100 + 4 * 10 * 10


def test_traffic_only_for_matching_sources(monkeypatch):
    key = "tlfea::k_vjp<0,2,true,false>"
    have = bench.traffic_from_profile(key)
    monkeypatch.setattr(bench, "source_hash", lambda: "0" * 64)
    assert bench.traffic_from_profile(key) is None
    if have is not None:
        assert have > bench.bytes_per_call("vjp", 1414035, 1020000, 10, True)
