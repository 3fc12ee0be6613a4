"""Work list of the persistent batched launch (csrc/persist_schedule.h),
checked on the host: every (grid, round, workgroup) listed once, thresholds
equal to the waves of the grid's earlier rounds, earlier rounds of a grid
queued first, and a simulated queue with 1 to 64 persistent workgroups that
finish in random order always drains (no deadlock for any number of resident
workgroups)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2001_01473_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not found")
    exe = str(tmp_path_factory.mktemp("persist") / "persist_schedule_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "persist_schedule_check.cpp"),
                    "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("grids,workers", [(1, 1), (3, 2), (16, 7), (64, 64), (64, 1)])
def test_persistent_work_list(checker, seed, grids, workers):
    out = subprocess.run([checker, str(seed), str(grids), str(workers)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout
