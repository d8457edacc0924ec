"""The binding and torch share one HIP runtime whatever is imported first (GPU)."""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, %r)
import numpy as np
from paper_2009_09500_amd import binding, workloads
binding.vox_tuning_cache_set((256, 256, 256), 256, binding.make_tuning((8, 6, 5)))  # the library before torch
import torch
c = workloads.small_uniform(n=256)
s = torch.from_numpy(c["segs"]).to("cuda:0")
g = binding.segments_to_grid(s, c["dims"])
torch.cuda.synchronize()
from oracle import oracle
assert np.array_equal(g.cpu().numpy().view(np.uint32), oracle.grid(c["segs"], c["dims"]))
print("ok")
"""


def test_library_loaded_before_torch():
    r = subprocess.run([sys.executable, "-c", SCRIPT % ROOT], cwd=ROOT, capture_output=True, text=True,
                       timeout=90)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-2000:]
