"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, sizes workspaces and rejects bad arguments before touching
a device.  No GPU needed: no call here reaches a HIP runtime function."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdmpm.h")

pm = pytest.importorskip("paper_1608_00802_amd")
from paper_1608_00802_amd import _lib  # noqa: E402


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libfdmpm.so is not built (run __graft_entry__.build())")
    return _lib.load_library()


def test_header_declarations_exported(lib):
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:pm_status|const char\*)\s+(pm_\w+)\s*\(", text, re.M))
    assert declared == set(_lib.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name


def test_flag_values_match_header():
    text = open(HEADER).read()
    assert re.search(r"#define PM_CONTINUE 1\b", text)
    assert re.search(r"#define PM_SORT_AUTO \(1 << 24\)", text)
    assert _lib.PM_CONTINUE == 1 and _lib.PM_SORT_AUTO == 1 << 24
    # PM_SORT_EVERY(k) occupies bits 8..23, clear of both single-bit flags
    assert _lib.PM_SORT_EVERY(0xffff) == 0xffff << 8
    assert _lib.PM_SORT_EVERY(0xffff) & (_lib.PM_CONTINUE | _lib.PM_SORT_AUTO) == 0


def test_struct_layout_matches_header():
    # pm_params: int32, int32, int64, double, int32, int32, 7 doubles -> 88 bytes
    assert ctypes.sizeof(_lib.PMParams) == 88
    assert _lib.PMParams.n_part.offset == 8
    assert _lib.PMParams.box.offset == 16
    assert _lib.PMParams.four_pi_G_rhobar.offset == 32
    assert _lib.PMParams.rho_fp64_below.offset == 80
    assert ctypes.sizeof(_lib.PMEnergies) == 32
    assert ctypes.sizeof(_lib.PMKineticParts) == 24


def _params(**kw):
    base = dict(n_mesh=64, n_part=64 ** 3, box=10.0)
    base.update(kw)
    return _lib.make_params(**base)


def test_workspace_bytes(lib):
    for n in (16, 32, 64, 128, 256, 512):
        b = _lib.pm_workspace_bytes(_params(n_mesh=n, n_part=n ** 3))
        cells = n ** 3
        npart = n ** 3
        # int64 mass + delta + phi + Q + half spectrum, the particle sort
        # (key, rank, position/velocity/id copies: 36 B per particle), tables
        need = 8 * cells + 12 * cells + 8 * (n // 2 + 1) * n * n + 36 * npart
        assert b >= need
        # plus energy partials (stencil blocks, and one |p|^2 partial per
        # gather block: at most 65536 unsorted or one per tile chunk) and the
        # sort's sliced tile counters and prefix sums
        kpart = 8 * max(65536, cells // 1024 + npart // 8192 + 1)
        assert b < need + 8 * 2 * cells // 256 + kpart + cells // 8 + 65536
        assert b % 256 == 0


@pytest.mark.parametrize("bad,status", [
    (dict(n_mesh=48), _lib.PM_EUNSUPPORTED),
    (dict(n_mesh=8), _lib.PM_EUNSUPPORTED),
    (dict(n_mesh=1024), _lib.PM_EUNSUPPORTED),
    (dict(n_mesh=0), _lib.PM_EUNSUPPORTED),
    (dict(n_mesh=-64), _lib.PM_EUNSUPPORTED),
    (dict(n_mesh=2 ** 30 + 1), _lib.PM_EUNSUPPORTED),
    (dict(n_mesh=2 ** 31 - 1), _lib.PM_EUNSUPPORTED),
    (dict(n_part=0), _lib.PM_EINVAL),
    (dict(box=0.0), _lib.PM_EINVAL),
    (dict(box=float("nan")), _lib.PM_EINVAL),
    (dict(precision=7), _lib.PM_EINVAL),
    (dict(hbar_over_m=-1.0), _lib.PM_EINVAL),
    (dict(rho_floor=0.0), _lib.PM_EINVAL),
    (dict(comoving=True, h0=0.0), _lib.PM_EINVAL),
    (dict(comoving=True, omega_m=-0.1), _lib.PM_EINVAL),
    (dict(n_part=8 * 64 ** 3 + 1), _lib.PM_EINVAL),
    (dict(n_part=8 * 64 ** 3), None),
    (dict(n_part=2 ** 24, precision=_lib.PM_FP32), None),
])
def test_param_validation(lib, bad, status):
    p = _params(**bad)
    n = ctypes.c_size_t(0)
    got = lib.pm_workspace_bytes(ctypes.byref(p), ctypes.byref(n))
    assert got == (status if status is not None else _lib.PM_OK)


def test_init_rejects_before_device_access(lib):
    p = _params()
    need = _lib.pm_workspace_bytes(p)
    ctx = ctypes.c_void_p(None)
    # null workspace, misaligned workspace, too small workspace: all host-side
    assert lib.pm_init(ctypes.byref(p), None, need, None, ctypes.byref(ctx)) == _lib.PM_EINVAL
    assert lib.pm_init(ctypes.byref(p), ctypes.c_void_p(0x1000 + 8), need, None,
                       ctypes.byref(ctx)) == _lib.PM_EINVAL
    assert lib.pm_init(ctypes.byref(p), ctypes.c_void_p(0x100000), need - 256, None,
                       ctypes.byref(ctx)) == _lib.PM_ENOMEM
    assert ctx.value is None


def test_poisson_static_rejects_before_device_access(lib):
    # argument errors come back before the call touches a device (none here)
    fake = ctypes.c_void_p(0x100000)
    for n in (0, 8, 48, 100, 2 ** 31 - 1):
        assert lib.pm_poisson_static(n, 1.0, fake, fake, None) == _lib.PM_EUNSUPPORTED, n
    for n in (256, 512, 2 ** 30):
        assert lib.pm_poisson_static(n, 1.0, fake, fake, None) == _lib.PM_ENOMEM, n
    assert lib.pm_poisson_static(64, 1.0, None, fake, None) == _lib.PM_EINVAL
    assert lib.pm_poisson_static(64, 1.0, fake, None, None) == _lib.PM_EINVAL
    assert lib.pm_poisson_static(64, float("nan"), fake, fake, None) == _lib.PM_EINVAL


def test_null_context_calls(lib):
    d = ctypes.c_double(0.0)
    assert lib.pm_deposit(None, None, None) == _lib.PM_EINVAL
    assert lib.pm_poisson(None, None, None) == _lib.PM_EINVAL
    assert lib.pm_qpot(None, None, None) == _lib.PM_EINVAL
    assert lib.pm_force(None, None, None, None, None, 1.0) == _lib.PM_EINVAL
    assert lib.pm_step(None, None, None, ctypes.byref(d), 1, 0) == _lib.PM_EINVAL
    assert lib.pm_energy(None, None, None, 1.0, None) == _lib.PM_EINVAL
    kp = _lib.PMKineticParts()
    assert lib.pm_kinetic_split(None, None, None, 1.0, ctypes.byref(kp)) == _lib.PM_EINVAL
    rms, cells = ctypes.c_double(), ctypes.c_int64()
    assert lib.pm_density_rms_diff(None, None, None, ctypes.byref(rms),
                                   ctypes.byref(cells)) == _lib.PM_EINVAL
    arr = (ctypes.c_double * 4)()
    assert lib.pm_power_spectrum(None, None, 4, arr, arr, arr) == _lib.PM_EINVAL
    assert lib.pm_spline_density(None, None, 3.5, None) == _lib.PM_EINVAL
    assert lib.pm_spline_qforce(None, None, None, 3.5, None) == _lib.PM_EINVAL
    assert lib.pm_spline_step(None, None, None, ctypes.byref(d), 1, 3.5) == _lib.PM_EINVAL
    assert lib.pm_spline_energy(None, None, None, 3.5, 1.0, None) == _lib.PM_EINVAL
    assert lib.pm_destroy(None) == _lib.PM_EINVAL


def test_strerror(lib):
    for s in (0, -1, -2, -3, -4, -5):
        assert len(lib.pm_strerror(s)) > 1
    assert lib.pm_strerror(99) == b"unknown status"
