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
    for c in range(8):
        s = L.letkf_strerror(c)
        assert s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 8
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


def test_plan_rejects_bad_options(lib):
    """Unknown flags, a nonzero reserved field and GRAPH_CAPTURE together
    with PHASE_TIMING are refused on the host, before any device call."""
    p = L.make_problem(**GOOD)
    for flags in (64, 1 << 20, -1, L.LETKF_FLAG_GRAPH_CAPTURE | L.LETKF_FLAG_PHASE_TIMING):
        rc, h = L.letkf_plan([p], flags=flags, raise_on_error=False)
        assert rc == L.LETKF_EINVAL and h is None, flags
    opt = L.letkf_options(0, 0, 1, None)
    h = ctypes.c_void_p()
    assert lib.letkf_plan(ctypes.byref(p), 1, ctypes.byref(opt), ctypes.byref(h)) == L.LETKF_EINVAL


def test_struct_layouts_match_header(lib, tmp_path):
    """Every struct of the header as the binding lays it out: size and field
    offsets equal to what the host C compiler gives them (gcc on a probe that
    includes the header)."""
    import os
    import subprocess
    structs = [L.letkf_problem, L.letkf_options, L.letkf_io, L.letkf_cycle_io, L.letkf_tuning]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "letkf.h"', 'int main(void) {']
    for st in structs:
        n = st.__name__
        lines.append(f'  printf("{n} %zu\\n", sizeof({n}));')
        for f, _ in st._fields_:
            lines.append(f'  printf("{n}.{f} %zu\\n", offsetof({n}, {f}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    inc = os.path.join(os.path.dirname(L.HEADER))
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.split("\n") if l)
    for st in structs:
        n = st.__name__
        assert int(out[n]) == ctypes.sizeof(st), n
        for f, _ in st._fields_:
            assert int(out[f"{n}.{f}"]) == getattr(st, f).offset, (n, f)


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
    assert lib.letkf_analyze_noalloc(None, None, None, None) == L.LETKF_EINVAL
    assert lib.letkf_invsqrt_batched(None, 4, 65, None, None, None, None) == L.LETKF_EINVAL
    assert lib.letkf_invsqrt_batched(None, 0, 8, None, None, None, None) == L.LETKF_OK
    assert lib.letkf_invsqrt_batched(None, 3, 8, None, None, None, None) == L.LETKF_EINVAL


def test_noalloc_host_checks(lib):
    # bad problem, too many observations, missing arrays: refused before the device
    x = ctypes.c_double(0.0)
    st = ctypes.c_int32(0)
    bad = L.make_problem(32, 32, 1, 10, 4.0, 1.1)
    io = L.letkf_io(0, 0, ctypes.addressof(x), ctypes.addressof(x), 0, 0, 0, 0, 0)
    assert lib.letkf_analyze_noalloc(ctypes.byref(bad), ctypes.byref(io), ctypes.addressof(st),
                                     None) == L.LETKF_EINVAL
    p = L.make_problem(**GOOD)
    many = L.letkf_io(0, p.n_obs_max + 1, ctypes.addressof(x), ctypes.addressof(x), 0, 0, 0, 0, 0)
    assert lib.letkf_analyze_noalloc(ctypes.byref(p), ctypes.byref(many), ctypes.addressof(st),
                                     None) == L.LETKF_EINVAL
    noarr = L.letkf_io(0, 1, ctypes.addressof(x), ctypes.addressof(x), 0, 0, 0, 0, 0)
    assert lib.letkf_analyze_noalloc(ctypes.byref(p), ctypes.byref(noarr), ctypes.addressof(st),
                                     None) == L.LETKF_EINVAL
    assert lib.letkf_analyze_noalloc(ctypes.byref(p), ctypes.byref(io), None,
                                     None) == L.LETKF_EINVAL


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


def test_build_scratch_limits():
    """The build rejects a kernel that spills more than its unit allows: none
    at all in the fused units, up to MAX_SCRATCH bytes per lane elsewhere."""
    from paper_2308_03310_amd import build as B

    def remarks(n):
        return ("k.h:1:1: remark: Function Name: _ZN5letkf1kEv [-Rpass-analysis=kernel-resource-usage]\n"
                f"k.h:1:1: remark:     ScratchSize [bytes/lane]: {n} [-Rpass-analysis=kernel-resource-usage]\n")

    B._check_scratch("k_fused64.hip", remarks(0))
    B._check_scratch("k_xf32.hip", remarks(B.MAX_SCRATCH))
    with pytest.raises(RuntimeError, match="spills 8 bytes"):
        B._check_scratch("k_fused64.hip", remarks(8))
    with pytest.raises(RuntimeError, match="limit 256"):
        B._check_scratch("k_xf32.hip", remarks(B.MAX_SCRATCH + 4))
