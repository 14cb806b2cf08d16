"""The library and PyTorch share one HIP runtime whatever is used first.

A fresh process calls the host-buffer entry point before touching PyTorch,
then allocates a torch tensor on the device and runs a device-buffer
alignment on it; both results must equal the oracle's.
"""
import subprocess
import sys
from pathlib import Path

import pytest

pytestmark = pytest.mark.gpu

ROOT = Path(__file__).resolve().parents[1]

SCRIPT = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np
import paper_2311_17530_amd as msa
from msa_inputs import workload
from oracle import oracle_align
j = workload("dna_k3_40")
s0, r0, _ = oracle_align(j.seqs, j.sub, j.gap)
s1, r1 = msa.align(j.seqs, j.sub, j.gap)            # library first
assert s1 == s0 and np.array_equal(r1, r0)
import torch
assert torch.cuda.is_available()
dev = msa.DeviceAligner(j.lens, j.sub, j.gap)     # then torch memory
dev.set_sequences(j.seqs)
dev.run()
s2, r2 = dev.result()
assert s2 == s0 and np.array_equal(r2, r0)
print("runtime order ok", flush=True)
"""


def test_library_before_torch_in_fresh_process():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(root=str(ROOT))],
                       capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "runtime order ok" in r.stdout
