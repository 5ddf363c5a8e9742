"""pm_poisson_static (the Poisson solve without a context or workspace, for
callers that cannot allocate) against pm_poisson through a context, on two
calls in a row, the second on a smaller mesh; sizes above the scratch
array's maximum are rejected."""

import ctypes

import numpy as np
import pytest

from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu


def _call(pm, n, S, d, phi, stream):
    lib = pm.load_library()
    return lib.pm_poisson_static(n, ctypes.c_double(S), ctypes.c_void_p(d.data_ptr()),
                                 ctypes.c_void_p(phi.data_ptr()),
                                 ctypes.c_void_p(stream.cuda_stream))


def test_poisson_static_matches_context_path(gpu):
    import torch
    import paper_1608_00802_amd as pm
    stream = torch.cuda.current_stream(gpu)
    for call, (n, S) in enumerate([(128, 0.9), (64, 1.7)]):
        rng = np.random.default_rng(700 + n)
        d = torch.from_numpy(rng.standard_normal(n ** 3).astype(np.float32)).to(gpu)
        phi_s = torch.full((n ** 3,), float("nan"), dtype=torch.float32, device=gpu)
        assert _call(pm, n, S, d, phi_s, stream) == pm._lib.PM_OK
        ctx = pm.PMContext(pm.make_params(n, n ** 3, float(n), four_pi_G_rhobar=S), device=gpu)
        phi_c = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
        ctx.poisson(d, phi_c)
        torch.cuda.synchronize()
        a, b = phi_s.cpu().numpy(), phi_c.cpu().numpy()
        assert np.all(np.isfinite(a))
        err = rel_l2(a, b)
        print(f"call {call}: N = {n}, static vs context rel-L2 {err:.2e}", flush=True)
        assert err < 1e-6
        ctx.close()
    big = torch.zeros(256 ** 3, dtype=torch.float32, device=gpu)
    assert _call(pm, 256, 1.0, big, big, stream) == pm._lib.PM_ENOMEM
    assert _call(pm, 48, 1.0, big, big, stream) == pm._lib.PM_EUNSUPPORTED
