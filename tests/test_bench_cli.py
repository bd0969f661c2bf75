"""bench.py command line on a host without a GPU: more than one GPU is refused with a
message before anything is built or timed."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("mode", [[], ["--edt"], ["--ogm"], ["--serving"], ["--variants"],
                                  ["--paper-shaped"]])
def test_more_than_one_gpu_is_refused(mode):
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"] + mode,
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU only" in res.stderr
    assert res.stdout == ""
