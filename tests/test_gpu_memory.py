"""The QS_MAX_BYTES cap on library-allocated amplitude buffers, on the GPU
(in a child process, since the cap is read once per process)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np, torch
import paper_2609_19147_amd as qs, workloads as W
n = 20                                    # 8 MiB per complex64 buffer
st = qs.State(n, "c64", lazy_scratch=True)   # torch memory: not counted
assert qs.memory_info() == (0, 12 << 20), qs.memory_info()
plan = qs.Plan(n, W.random_perm_block(n, 40, 3))
qs.apply(st, plan)                        # the gather's scratch half: 8 MiB from the library
torch.cuda.synchronize()
assert qs.memory_info()[0] == 8 << 20, qs.memory_info()
insts = W.qaoa_instances(1, 1, depth=1, n_choices=(20,))
p = qs.Plan(20, W.qaoa_stream(insts[0], h_layer=False))
try:
    qs.Batch([p], init="plus")            # another 8 MiB: over the 12 MiB cap
    raise SystemExit("batch allocated over the cap")
except qs.QsError as e:
    assert "QS_MAX_BYTES" in str(e), str(e)
assert qs.memory_info()[0] == 8 << 20
del st
import gc; gc.collect()
assert qs.memory_info()[0] == 0, qs.memory_info()
B = qs.Batch([p], init="plus")            # fits now
B.run()
torch.cuda.synchronize()
print("ok", qs.memory_info()[0])
"""


def test_max_bytes_cap_counts_library_buffers():
    env = dict(os.environ, QS_MAX_BYTES=str(12 << 20))
    out = subprocess.run([sys.executable, "-c", CHILD], env=env, cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, (out.stdout[-2000:], out.stderr[-3000:])
    assert out.stdout.strip().splitlines()[-1] == f"ok {8 << 20}"
