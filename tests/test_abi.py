"""C-ABI contract checks that need no GPU: the library loads, exports every
function the header declares, and rejects bad descriptors before any device
call (on a machine without a GPU a valid descriptor yields LETKF_EDEVICE)."""
import ctypes
import math

import pytest

from paper_2308_03310_amd import letkf as L


@pytest.fixture(scope="module")
def lib():
    try:
        return L.load_library()
    except OSError as e:
        pytest.fail(f"library not built: {e}")


def test_exports_every_declared_function(lib):
    names = L.header_functions()
    assert {"letkf_plan", "letkf_analyze", "letkf_cycle", "letkf_status", "letkf_plan_destroy",
            "letkf_strerror", "letkf_eigh_batched", "letkf_plan_workspace_bytes", "letkf_tune",
            "letkf_set_tuning"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_strerror_covers_codes(lib):
    seen = set()
    for c in range(7):
        s = L.letkf_strerror(c)
        assert s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 7
    assert L.letkf_strerror(99) == "unknown status"


GOOD = dict(nx=32, ny=32, k=16, n_obs_max=128, loc_len=4.0, infl=1.1)


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-3), dict(nx=40000), dict(k=1), dict(k=65), dict(n_obs_max=-1),
    dict(loc_len=0.0), dict(loc_len=math.nan), dict(loc_len=math.inf), dict(infl=0.0),
    dict(infl=-1.0), dict(infl=math.inf),
])
def test_plan_rejects_bad_descriptors(lib, bad):
    kw = dict(GOOD)
    kw.update(bad)
    p = L.make_problem(**kw)
    rc, h = L.letkf_plan([p], raise_on_error=False)
    assert rc == L.LETKF_EINVAL and h is None


def test_plan_rejects_bad_enums_and_counts(lib):
    for loc, prec in [(3, 0), (-1, 0), (0, 7)]:
        p = L.make_problem(**GOOD, loc=loc, precision=prec)
        assert L.letkf_plan([p], raise_on_error=False)[0] == L.LETKF_EINVAL
    assert L.letkf_plan([], raise_on_error=False)[0] == L.LETKF_EINVAL
    h = ctypes.c_void_p()
    assert lib.letkf_plan(None, 1, None, ctypes.byref(h)) == L.LETKF_EINVAL
    p = L.make_problem(**GOOD)
    assert lib.letkf_plan(ctypes.byref(p), 1, None, None) == L.LETKF_EINVAL


def test_budget_checked_before_device(lib):
    p = L.make_problem(**GOOD)
    rc, h = L.letkf_plan([p], hbm_budget_bytes=1024, raise_on_error=False)
    assert rc == L.LETKF_ENOMEM and h is None


def test_null_handles(lib):
    assert lib.letkf_plan_destroy(None) == L.LETKF_OK
    assert lib.letkf_status(None, 1) == L.LETKF_EINVAL
    assert lib.letkf_analyze(None, None, 0, None) == L.LETKF_EINVAL
    assert lib.letkf_plan_workspace_bytes(None) == 0
    assert lib.letkf_eigh_batched(None, 4, 70, None, None, None, None) == L.LETKF_EINVAL
    assert lib.letkf_eigh_batched(None, 0, 8, None, None, None, None) == L.LETKF_OK
    assert lib.letkf_eigh_batched(None, 3, 8, None, None, None, None) == L.LETKF_EINVAL


def test_valid_descriptor_without_gpu_is_edevice(lib):
    from conftest import gpu_available
    if gpu_available():
        pytest.skip("GPU present")
    p = L.make_problem(**GOOD)
    rc, h = L.letkf_plan([p], raise_on_error=False)
    assert rc == L.LETKF_EDEVICE and h is None


def test_tuning_calls_reject_bad_arguments(lib):
    t = L.letkf_tuning(8, 0, 0.0)
    assert lib.letkf_set_tuning(None, ctypes.byref(t)) == L.LETKF_EINVAL
    assert lib.letkf_tune(None, None, 0, None, ctypes.byref(t)) == L.LETKF_EINVAL
