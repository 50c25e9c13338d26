"""Host side of bench.py, no GPU needed: the one-GPU guard, the byte model of
the SSP-RK stages and the traffic-record lookup."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
bench = pytest.importorskip("bench")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""                              # no JSON line


def test_stage_byte_model():
    # Shu-Osher forms: stage 1 reads w and writes a register (16 B per FP64
    # DOF), every later stage also reads the base register (24 B)
    assert bench.stage_bytes_per_dof(1) == [16.0]
    b3, b5 = bench.stage_bytes_per_dof(3), bench.stage_bytes_per_dof(5)
    assert sum(b3) / 3 == pytest.approx(64.0 / 3.0)
    assert sum(b5) / 5 == pytest.approx(22.4)


def test_traffic_record_unknown_kernel():
    assert bench.traffic_record("no_such_kernel", "driven_turbulence_3d") is None
