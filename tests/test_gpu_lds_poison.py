"""The LDS-poison checking build against libpond.so.

libpond_ldspoison.so is the same source built with every LDS window filled
with NaN before it is staged.  A kernel that read a window value it had not
staged (a placement or bounds mistake) would return NaN, or a different
value, there.  The cases of tests/lds_cases.py run in a child process with
the poisoned library and here with libpond.so: the forward outputs must be
equal bit for bit, the adjoint's within the rounding of its atomic sums.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1806_05089_amd import build as hip_build
from tests import lds_cases

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_poisoned_lds_changes_nothing(gpu, tmp_path):
    assert os.path.exists(hip_build.POISON_LIB), "build the checking library first"
    path = str(tmp_path / "poison.npz")
    env = dict(os.environ, POND_LIBRARY=hip_build.POISON_LIB)
    print("running the cases with the LDS-poison library", flush=True)
    subprocess.run([sys.executable, "-m", "tests.lds_cases", path], cwd=ROOT, env=env,
                   check=True, timeout=300)
    poisoned = dict(np.load(path))
    ref = lds_cases.run()
    assert set(poisoned) == set(ref)
    for k, v in ref.items():
        p = poisoned[k]
        assert np.array_equal(np.isnan(v), np.isnan(p)), k
        assert not np.any(np.isnan(v)), k
        if k.startswith("adjoint"):
            scale = np.max(np.abs(v))
            err = np.max(np.abs(p - v)) / scale
            print(f"{k}: max difference {err:.2e} of the largest entry", flush=True)
            assert err < 1e-12, k
        else:
            assert np.array_equal(v, p), (k, np.max(np.abs(v - p)))
    print(f"{len(ref)} outputs equal", flush=True)
