"""The library and torch share one HIP runtime whatever the import order.

A fresh interpreter imports the binding before torch (the order in which
pytest collects the host tests) and lists the shared objects mapped into the
process: exactly one HIP runtime and one ROCr must be there.  Two copies mean
the library's runtime never sees the device torch initialised."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2407_00769_amd", "libtnc.so")

PROBE = r"""
import sys
sys.path.insert(0, {root!r})
import paper_2407_00769_amd._tnc as T   # the binding first
import torch                               # then torch
libs = set()
for line in open('/proc/self/maps'):
    parts = line.split()
    if len(parts) >= 6:
        libs.add(parts[5])
hip = sorted(p for p in libs if 'libamdhip64' in p)
hsa = sorted(p for p in libs if 'libhsa-runtime64' in p)
print('HIP', len(hip), *hip)
print('HSA', len(hsa), *hsa)
"""


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtnc.so not built")
@pytest.mark.parametrize("first", ["binding", "torch"])
def test_one_hip_runtime_in_the_process(first):
    code = PROBE.format(root=ROOT)
    if first == "torch":
        code = code.replace("import paper_2407_00769_amd._tnc as T   # the binding first\nimport torch",
                            "import torch\nimport paper_2407_00769_amd._tnc as T")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    lines = {ln.split()[0]: ln.split()[1:] for ln in r.stdout.splitlines() if ln.split()}
    assert lines["HIP"][0] == "1", r.stdout
    assert lines["HSA"][0] == "1", r.stdout
