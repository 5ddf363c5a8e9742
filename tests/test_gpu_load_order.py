"""The library shares torch's HIP runtime whatever the import order.

torch ships its own HIP runtime; a library loaded before torch would bind
to another copy, and its calls on torch's streams and memory would fail.
load_library() therefore brings torch in first.  Checked in a fresh
interpreter (the test process has imported torch long before): load the
library, only then import torch, and solve a small Poisson problem.
"""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = """
import sys
sys.path.insert(0, {root!r})
import paper_1608_00802_amd as pm
pm.load_library()
import math, torch
n = 16
ctx = pm.PMContext(pm.make_params(n, n ** 3, float(n), four_pi_G_rhobar=1.0), device="cuda:0")
x = torch.arange(n, dtype=torch.float64, device="cuda:0")
d = torch.sin(2 * math.pi * x / n).view(n, 1, 1).expand(n, n, n).contiguous().float().view(-1)
phi = torch.empty_like(d)
ctx.poisson(d, phi)
torch.cuda.synchronize()
ok = bool(torch.isfinite(phi).all()) and float(phi.abs().max()) > 0.0
print("phi ok" if ok else "phi bad", flush=True)
sys.exit(0 if ok else 1)
"""


def test_library_loaded_before_torch(gpu):
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT)], capture_output=True,
                       text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and "phi ok" in r.stdout
