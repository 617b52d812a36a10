"""No kernel of the library uses per-thread scratch (private) memory.

A local array indexed with a value the compiler cannot resolve, or registers
spilled beyond the register file, are placed in scratch memory, which every
access then reaches through the memory hierarchy: a D3Q27 two-component step
whose velocity-layer loop stayed rolled ran 30 times slower that way.  This
test compiles every kernel source of the library for gfx950 with the
library's own flags (device code only, to assembly, in a temporary
directory) and reads the private segment size the compiler records for each
kernel; all must be zero.  It needs hipcc (cross-compilation, no GPU) and
skips without it.
"""
import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2301_01622_amd import build as B

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")

_SIZE = re.compile(r"^\s*\.set\s+(\S+)\.private_seg_size,\s*(\d+)", re.M)


def _kernel_sources():
    return sorted(os.path.join(B.CSRC, f) for f in os.listdir(B.CSRC) if f.endswith(".hip"))


def _private_sizes(src, out_dir):
    asm = os.path.join(out_dir, os.path.basename(src) + ".s")
    flags = [f for f in B.COMMON if f != "-fPIC"]
    r = subprocess.run(["hipcc", *flags, "--cuda-device-only", "-S", src, "-o", asm], capture_output=True, text=True)
    assert r.returncode == 0, f"hipcc failed for {src}:\n{r.stderr[-2000:]}"
    with open(asm) as fh:
        return [(name, int(size)) for name, size in _SIZE.findall(fh.read())]


def test_no_kernel_uses_scratch_memory():
    with tempfile.TemporaryDirectory() as tmp:
        with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
            results = list(ex.map(lambda s: (s, _private_sizes(s, tmp)), _kernel_sources()))
    kernels = [(os.path.basename(s), name, size) for s, sizes in results for name, size in sizes]
    assert kernels, "no kernel found in the compiled sources"
    offenders = [(f, name, size) for f, name, size in kernels if size != 0]
    assert not offenders, f"kernels using scratch memory (bytes per thread): {offenders[:5]}"
