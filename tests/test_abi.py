"""CPU checks of the C-ABI library: it loads, exports every entry point the
header declares, and validates arguments before touching the device."""
import ctypes
import re

import pytest

from paper_1702_08521_amd import slmpp, workloads


def _declared_symbols():
    text = open(slmpp.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(slmpp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = slmpp.lib()
    declared = _declared_symbols()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(L, name), name
    # and the binding wraps exactly the declared entry points
    assert sorted(slmpp.SIGNATURES) == declared


def test_abi_version():
    m = re.search(r"#define SLMPP_ABI_VERSION (\d+)", open(slmpp.HEADER).read())
    assert m and int(m.group(1)) == slmpp.ABI_VERSION
    assert slmpp.lib().slmpp_abi_version() == slmpp.ABI_VERSION


def _desc(**kw):
    s = workloads.landau_1d1v(nx=16, nv=32)
    d = slmpp.make_desc(s)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_workspace_bytes_positive_for_valid_desc():
    assert slmpp.workspace_bytes(_desc()) > 0
    s3 = workloads.landau_3d3v(n=8)
    assert slmpp.workspace_bytes(slmpp.make_desc(s3, slmpp.F32)) > 0


@pytest.mark.parametrize("field,value,code", [
    ("D", 0, slmpp.ERR_INVALID),
    ("D", 4, slmpp.ERR_INVALID),
    ("order", 6, slmpp.ERR_INVALID),
    ("limiter", 3, slmpp.ERR_INVALID),
    ("poisson_order", 3, slmpp.ERR_INVALID),
    ("storage", 2, slmpp.ERR_INVALID),
    ("x_bc", 5, slmpp.ERR_INVALID),
    ("flags", 16, slmpp.ERR_INVALID),
    ("alpha", float("nan"), slmpp.ERR_NONFINITE),
    ("alpha", -1.0, slmpp.ERR_NONFINITE),
])
def test_validate_rejects_bad_fields(field, value, code):
    d = _desc(**{field: value})
    st, msg = slmpp.validate(d)
    assert st == code and msg
    assert slmpp.workspace_bytes(d) == 0


def test_validate_rejects_bad_axes():
    d = _desc()
    d.nx[0] = 0
    assert slmpp.validate(d)[0] == slmpp.ERR_SHAPE
    d = _desc()
    d.nv[0] = 5000
    assert slmpp.validate(d)[0] == slmpp.ERR_SHAPE
    d = _desc()
    d.x_hi[0] = d.x_lo[0]
    assert slmpp.validate(d)[0] == slmpp.ERR_SHAPE
    d = _desc()
    d.v_lo[0] = float("inf")
    assert slmpp.validate(d)[0] == slmpp.ERR_NONFINITE


def test_create_rejects_null_buffers_without_device():
    L = slmpp.lib()
    d = _desc()
    h = ctypes.c_void_p()
    st = L.slmpp_create(ctypes.byref(d), None, None, 0, None, ctypes.byref(h))
    assert st == slmpp.ERR_INVALID and not h.value
    assert b"NULL" in L.slmpp_last_error(None)
    st = L.slmpp_create(ctypes.byref(d), ctypes.c_void_p(256), ctypes.c_void_p(512), 16, None,
                        ctypes.byref(h))
    assert st == slmpp.ERR_WORKSPACE and not h.value


def test_null_context_is_rejected():
    L = slmpp.lib()
    assert L.slmpp_advect_x(None, 0, 0.1) == slmpp.ERR_INVALID
    assert L.slmpp_step(None, 0.1, 1) == slmpp.ERR_INVALID
    assert L.slmpp_kick(None, 0.1) == slmpp.ERR_INVALID
    assert L.slmpp_batch_set_fast_min_cells(None, 0) == slmpp.ERR_INVALID
    assert L.slmpp_batch_step_bytes(None) == 0.0
    assert L.slmpp_destroy(None) == slmpp.ERR_INVALID


def test_copy_rejects_misaligned():
    L = slmpp.lib()
    assert L.slmpp_copy_device(ctypes.c_void_p(16), ctypes.c_void_p(32), 17, None) == slmpp.ERR_INVALID
    assert L.slmpp_copy_device(None, ctypes.c_void_p(32), 16, None) == slmpp.ERR_INVALID


# ---- batched ensembles: host-side validation (no device work) ----------
def _ensemble():
    return [slmpp.make_desc(workloads.landau_1d1v(nx=16, nv=32), slmpp.F32),
            slmpp.make_desc(workloads.twostream_1d1v(nx=32, nv=48, order=7), slmpp.F32),
            slmpp.make_desc(workloads.landau_3d3v(n=4, nv=6, order=5, D=2), slmpp.F32)]


def test_batch_workspace_bytes_valid_and_invalid():
    descs = _ensemble()
    total = slmpp.batch_workspace_bytes(descs)
    assert total > 0
    # grows with the ensemble
    assert slmpp.batch_workspace_bytes(descs + descs) > total
    # mixed storage types cannot form a batch
    mixed = _ensemble()
    mixed[1].storage = slmpp.F64
    assert slmpp.batch_workspace_bytes(mixed) == 0
    # batched runs use the SL-MPP limiter
    lim = _ensemble()
    lim[0].limiter = slmpp.LIM_MP
    assert slmpp.batch_workspace_bytes(lim) == 0
    # at most 2048 spatial cells per run
    big = _ensemble()
    big[0].nx[0] = 4096
    assert slmpp.batch_workspace_bytes(big) == 0
    # an invalid description anywhere
    bad = _ensemble()
    bad[2].order = 6
    assert slmpp.batch_workspace_bytes(bad) == 0
    assert slmpp.lib().slmpp_batch_workspace_bytes(None, 3) == 0


def test_batch_create_rejects_before_device_work():
    L = slmpp.lib()
    descs = _ensemble()
    arr = slmpp._desc_array(descs)
    n = len(descs)
    dts = (ctypes.c_double * n)(0.1, 0.1, float("nan"))
    fp = (ctypes.c_void_p * n)(256, 512, 768)
    out = ctypes.c_void_p()
    need = slmpp.batch_workspace_bytes(descs)
    # NULL out
    assert L.slmpp_batch_create(arr, dts, n, fp, ctypes.c_void_p(4096), need, None, None) == slmpp.ERR_INVALID
    # non-finite dt
    st = L.slmpp_batch_create(arr, dts, n, fp, ctypes.c_void_p(4096), need, None, ctypes.byref(out))
    assert st == slmpp.ERR_NONFINITE and not out.value
    assert b"dt" in L.slmpp_batch_last_error(None)
    dts[2] = 0.1
    # misaligned workspace
    st = L.slmpp_batch_create(arr, dts, n, fp, ctypes.c_void_p(4100), need, None, ctypes.byref(out))
    assert st == slmpp.ERR_INVALID
    # too small a workspace
    st = L.slmpp_batch_create(arr, dts, n, fp, ctypes.c_void_p(4096), need - 1, None, ctypes.byref(out))
    assert st == slmpp.ERR_WORKSPACE
    # misaligned f
    fp[1] = 520
    st = L.slmpp_batch_create(arr, dts, n, fp, ctypes.c_void_p(4096), need, None, ctypes.byref(out))
    assert st == slmpp.ERR_INVALID
    # invalid description: the message names the run
    bad = _ensemble()
    bad[1].D = 4
    st = L.slmpp_batch_create(slmpp._desc_array(bad), dts, n, fp, ctypes.c_void_p(4096), need, None,
                              ctypes.byref(out))
    assert st == slmpp.ERR_INVALID and b"run 1" in L.slmpp_batch_last_error(None)


def test_batch_null_handle_calls():
    L = slmpp.lib()
    assert L.slmpp_batch_destroy(None) == slmpp.ERR_INVALID
    assert L.slmpp_batch_step(None, 1) == slmpp.ERR_INVALID
    assert L.slmpp_batch_step_eager(None, 1) == slmpp.ERR_INVALID
    assert L.slmpp_batch_get_f(None, 0, None, 0) == slmpp.ERR_INVALID
    assert L.slmpp_batch_autotune(None, None) == slmpp.ERR_INVALID
    assert L.slmpp_batch_init_separable(None, 0, None, None, None, None) == slmpp.ERR_INVALID
    assert L.slmpp_batch_tile_width(None, 0, 0) == 0


def test_rk_flag_accepted_and_workspace_grows():
    d = _desc()
    base = slmpp.workspace_bytes(d)
    d.flags = slmpp.FLAG_RK3
    st, _ = slmpp.validate(d)
    assert st == slmpp.OK
    ncell = 16 * 32
    assert slmpp.workspace_bytes(d) >= base + 8 * ncell
    # batched ensembles use the SL-MPP scheme only
    e = _ensemble()
    e[0].flags = slmpp.FLAG_RK3
    assert slmpp.batch_workspace_bytes(e) == 0


def test_isolated_flag_needs_three_dimensions():
    d = _desc()
    d.flags = slmpp.FLAG_ISOLATED
    st, msg = slmpp.validate(d)
    assert st == slmpp.ERR_INVALID and "D = 3" in msg
    d3 = slmpp.make_desc(workloads.collapse_3d3v(nx=8, nv=4))
    assert d3.flags == slmpp.FLAG_ISOLATED
    assert slmpp.validate(d3)[0] == slmpp.OK
    plain = slmpp.make_desc(dict(workloads.collapse_3d3v(nx=8, nv=4), field_bc="periodic"))
    assert slmpp.workspace_bytes(d3) >= slmpp.workspace_bytes(plain) + 40 * 8 * 512


def test_advect_v_noalloc_rejects_before_touching_the_device():
    """Argument errors of the allocation-free velocity sweep come back before
    any device call (fake, never dereferenced device pointers)."""
    L = slmpp.lib()
    d = _desc()
    fake = ctypes.c_void_p(4096)
    st = L.slmpp_advect_v_noalloc(ctypes.byref(d), fake, 1, 0.1, fake, None)
    assert st == slmpp.ERR_INVALID  # dim outside 0..D-1
    st = L.slmpp_advect_v_noalloc(ctypes.byref(d), fake, 0, float("nan"), fake, None)
    assert st == slmpp.ERR_NONFINITE
    st = L.slmpp_advect_v_noalloc(ctypes.byref(d), None, 0, 0.1, fake, None)
    assert st == slmpp.ERR_INVALID
    # a table beyond the 16 MiB scratch: 64^3 spatial cells in FP64 (80 B each)
    big = slmpp.make_desc(workloads.landau_3d3v(n=64, nv=4), slmpp.F64)
    st = L.slmpp_advect_v_noalloc(ctypes.byref(big), fake, 0, 0.1, fake, None)
    assert st == slmpp.ERR_SHAPE
    assert b"scratch" in L.slmpp_last_error(None)


def test_alloc_device_rejects_before_touching_the_device():
    """slmpp_alloc_device checks its arguments before any device call."""
    L = slmpp.lib()
    p = ctypes.c_void_p(1234)
    assert L.slmpp_alloc_device(0, 1, ctypes.byref(p)) == slmpp.ERR_INVALID
    assert p.value is None  # *out cleared on failure
    assert L.slmpp_alloc_device(1 << 20, 1, None) == slmpp.ERR_INVALID
    assert b"alloc_device" in L.slmpp_last_error(None)
    assert L.slmpp_free_device(None) == slmpp.OK
