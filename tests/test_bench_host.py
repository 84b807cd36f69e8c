"""Host-side logic of bench.py (no GPU): the step plan over the config-3 workload and the refusal
of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_config3_steps_cover_every_point_once():
    combos, make, desc = bench.workload("config3")
    assert len(combos) == 24 and len(set(combos)) == 24          # 3 gaps x 8 k_par
    for kps, nsteps in ((8, 3), (4, 6), (3, 9)):
        groups = bench.step_groups(combos, kps)
        assert len(groups) == nsteps
        seen = [(key, ik) for key, iks in groups for ik in iks]
        assert sorted(seen) == sorted(combos)                   # each (gap, k_par) exactly once
        assert all(len(iks) <= kps for _, iks in groups)
        assert all(len(set(iks)) == len(iks) for _, iks in groups)   # distinct k_par of one gap


def test_default_step_is_eight_kpar_of_one_gap():
    old = sys.argv   # parse() reads sys.argv
    try:
        sys.argv = ["bench.py"]
        a = bench.parse()
    finally:
        sys.argv = old
    assert a.kpar_per_step == 8 and a.gpus == 1 and a.time_budget == 150.0
    groups = bench.step_groups(bench.workload("config3")[0], a.kpar_per_step)
    assert [len(iks) for _, iks in groups] == [8, 8, 8]


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""
