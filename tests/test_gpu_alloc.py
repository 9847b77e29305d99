"""Caller buffers from slmpp_alloc_device: physically contiguous (or plain)
device memory holding f.  The sweeps read and write f through the same
addresses whatever backs them, so whole Strang steps over such a buffer must
equal the same steps over a torch allocation bit for bit, and both must match
the FP64 oracle (L1 relative 1e-12 in FP64 storage, 1e-5 in FP32, as for the
other whole-step tests)."""
import numpy as np
import pytest

import oracle as O
from paper_1702_08521_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_08521_amd import slmpp

    slmpp.lib()
    return slmpp


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("contiguous", [1, 0])
def test_steps_on_alloc_device_buffer(S, storage, contiguous):
    import torch

    spec = W.landau_3d3v(n=12, nv=16, order=7, D=3, amp=0.2)
    nsteps = 3
    say(f"case alloc_device contiguous={contiguous} storage={storage} 12^3 x 16^3, {nsteps} steps")
    sx, gv = W.separable_factors(spec)
    desc = S.make_desc(spec, storage)
    shape = tuple(spec["nx"][:3]) + tuple(spec["nv"][:3])
    tdt = torch.float64 if storage == 0 else torch.float32
    nbytes = int(np.prod(shape)) * (8 if storage == 0 else 4)
    buf = S.DeviceBuffer(nbytes, contiguous=bool(contiguous))
    try:
        f = buf.tensor(shape, tdt)
        assert f.data_ptr() == buf.ptr and f.is_contiguous()
        a = S.Context(desc, f=f)
        a.init_f_separable(sx, gv)
        a.step(spec["dt"], nsteps)
        got = a.get_f()
        a.close()
        del f
    finally:
        torch.cuda.synchronize()
        buf.free()
    b = S.Context(desc)
    b.init_f_separable(sx, gv)
    b.step(spec["dt"], nsteps)
    ref = b.get_f()
    b.close()
    assert np.array_equal(got, ref)
    run = O.Run(spec)
    run.step(spec["dt"], nsteps)
    want = run.f
    l1 = float(np.abs(got - want).sum() / np.abs(want).sum())
    say(f"  L1 rel vs oracle {l1:.3e}")
    assert l1 <= (1e-12 if storage == 0 else 1e-5)


def test_alloc_device_view_bounds(S):
    import torch

    buf = S.DeviceBuffer(1024, contiguous=False)
    try:
        with pytest.raises(S.SlmppError):
            buf.tensor((257,), torch.float32)
        t = buf.tensor((256,), torch.float32)
        t.fill_(1.0)
        assert float(t.sum()) == 256.0
        del t
    finally:
        torch.cuda.synchronize()
        buf.free()


def test_alloc_device_view_keeps_buffer_alive(S):
    """A tensor view holds its buffer: dropping the last other reference
    frees nothing until the view is gone."""
    import gc
    import weakref

    import torch

    buf = S.DeviceBuffer(4096, contiguous=True)
    t = buf.tensor((1024,), torch.float32)
    w = weakref.ref(buf)
    del buf
    gc.collect()
    assert w() is not None
    t.fill_(2.0)
    assert float(t.sum()) == 2048.0
    torch.cuda.synchronize()
    del t
    gc.collect()
    assert w() is None


def test_alloc_device_refusal_leaves_the_device_usable(S):
    """An allocation the driver cannot satisfy comes back as an error and
    leaves nothing behind: later work on the device is unaffected."""
    import torch

    with pytest.raises(S.SlmppError) as ei:
        S.DeviceBuffer(1 << 50, contiguous=True)  # 1 PiB
    assert ei.value.status == S.ERR_DEVICE
    spec = W.landau_1d1v(nx=32, nv=64, amp=0.2)
    ctx = S.Context(S.make_desc(spec, 0))
    ctx.init_f_separable(*W.separable_factors(spec))
    ctx.step(spec["dt"], 3)
    got = ctx.get_f()
    ctx.close()
    run = O.Run(spec)
    run.step(spec["dt"], 3)
    assert float(np.abs(got - run.f).sum() / np.abs(run.f).sum()) <= 1e-12
    torch.cuda.synchronize()
