"""Register budget of the persistent fill kernels, and no scratch memory in
any kernel (CPU only: device-only compiles of the kernel sources with the
compiler's resource-usage remarks).

The persistent fill kernels keep every workgroup that fits on a compute unit
busy, so their throughput scales with occupancy.  A change that moves the job
descriptor fields from scalar to vector registers (for instance reading them
through a pointer the compiler cannot prove unwritten) costs a third or more
of the batched throughput without changing any result; this test fails on it.
So does any use of scratch memory (register spills, or a private copy of the
descriptor, which taking a by-value kernel argument's address produces).
"""
import re
import subprocess

import pytest

from paper_2311_17530_amd import build as B

# kernel (demangled prefix) -> fewest waves per SIMD it must keep
# (the compiler's figure, limited by registers and by the LDS a workgroup
# declares)
FLOORS = {
    "msa::fill_kernel<3, 256>": 6,
    "msa::fill_kernel<4, 256>": 5,
    "msa::fill_kernel<5, 256>": 5,
    "msa::fill_kernel<6, 256>": 4,
    "msa::batch_fill_kernel<2, 4, 256>": 5,
    "msa::batch_fill_kernel<5, 5, 256>": 5,
    "msa::batch_fill_kernel<6, 6, 256>": 4,
}


def _demangle(names):
    r = subprocess.run(["c++filt"], input="\n".join(names), capture_output=True, text=True,
                       check=True)
    return r.stdout.splitlines()


def _remarks(name):
    src = B.CSRC / name
    cmd = [B.HIPCC, *B.COMMON, "--cuda-device-only", "-Rpass-analysis=kernel-resource-usage",
           "-c", str(src), "-o", "/dev/null"]
    return subprocess.run(cmd, capture_output=True, text=True)


@pytest.fixture(scope="module")
def usage():
    from concurrent.futures import ThreadPoolExecutor
    names = sorted(p.name for p in B.CSRC.glob("*.hip"))
    with ThreadPoolExecutor(max_workers=len(names)) as ex:
        runs = list(ex.map(_remarks, names))
    for r in runs:
        assert r.returncode == 0, r.stderr[-2000:]
    return _parse("\n".join(r.stderr for r in runs))


def _parse(stderr):
    names, vgprs, occ, scratch = [], [], [], []
    for line in stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            names.append(m.group(1))
            continue
        m = re.search(r"remark:\s+ScratchSize \[bytes/lane\]: (\d+)", line)
        if m:
            scratch.append(int(m.group(1)))
            continue
        m = re.search(r"remark:\s+VGPRs: (\d+)", line)
        if m:
            vgprs.append(int(m.group(1)))
            continue
        m = re.search(r"remark:\s+Occupancy \[waves/SIMD\]: (\d+)", line)
        if m:
            occ.append(int(m.group(1)))
    assert len(names) == len(vgprs) == len(occ) == len(scratch) and names
    return {d: (v, o, sc) for d, v, o, sc in zip(_demangle(names), vgprs, occ, scratch)}


@pytest.mark.parametrize("kernel", sorted(FLOORS))
def test_fill_kernel_occupancy(usage, kernel):
    hits = [(d, vo) for d, vo in usage.items() if d.startswith("void " + kernel + "(")]
    assert len(hits) == 1, (kernel, [d for d in usage if "fill_kernel" in d])
    d, (v, o, sc) = hits[0]
    assert o >= FLOORS[kernel], f"{d}: {v} VGPRs, {o} waves/SIMD < {FLOORS[kernel]}"
    assert sc == 0, f"{d}: {sc} bytes of scratch per lane"


def test_no_kernel_uses_scratch(usage):
    used = {d: sc for d, (v, o, sc) in usage.items() if sc}
    assert not used, used
