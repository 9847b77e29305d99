"""Test-1 of Sec. 3.1 through the GPU sweeps: the design order on a
sinusoid and positivity on a quartic sine.

A 1D1V grid with one velocity row at speed 1 on x in [0, 1) (periodic):
every x-sweep advects the profile by nu = 0.2 cells; after t = 1 the exact
solution is the initial profile.  Checked against the values the paper
states (tests/golden/paper_values.json):
* Test-1b, 1 + sin(2 pi x), SL-MP5 / SL-MP7: L1 error slopes of five and
  seven over N (FP64);
* Test-1c, sin^4(4 pi x), N = 64: without the PP limiter the solution goes
  negative, with it it does not (FP64; FP32 to rounding), and with it the order
  approaches five at N = 128, 256.
The GPU errors also equal the oracle's.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1702_08521_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
NU = 0.2


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


def _gpu_advect(S, profile, order, lim, N, storage=0, t=1.0):
    """(L1 error / L1 norm, min, max over the run) of the GPU run."""
    spec = W.advection_1d1v(N, 1, 0.5, 1.5, profile, order=order, limiter=lim)
    x = W.centers(0.0, 1.0, N)
    f0 = W.test1_profile(profile, x)
    ctx = S.Context(S.make_desc(spec, storage))
    ctx.init_f_host(f0.reshape(N, 1))
    ref = ctx.get_f().ravel()  # the stored initial profile
    dt = NU / N  # speed 1, dx = 1/N
    lo, hi = ref.min(), ref.max()
    nsteps = int(round(t / dt))
    for k in range(nsteps):
        ctx.advect_x(0, dt)
        if k % 16 == 15 or k == nsteps - 1:
            g = ctx.get_f().ravel()
            lo, hi = min(lo, g.min()), max(hi, g.max())
    g = ctx.get_f().ravel()
    ctx.close()
    return np.abs(g - ref).sum() / np.abs(ref).sum(), lo, hi, g


def _oracle_advect(profile, order, lim, N, t=1.0):
    g = W.test1_profile(profile, W.centers(0.0, 1.0, N))
    for _ in range(int(round(t / (NU / N)))):
        g = O.sweep_pencil(g, NU, order=order, limiter=lim)
    return g


def _slope(errs, Ns):
    return -np.polyfit(np.log(Ns), np.log(errs), 1)[0]


@pytest.mark.parametrize("order", [5, 7])
def test_design_order_on_sinusoid(S, order):
    Ns = [16, 32, 64] if order == 7 else [32, 64, 128]
    res = [_gpu_advect(S, "sin", order, W.LIM_MP, N) for N in Ns]
    errs = [r[0] for r in res]
    slope = _slope(errs, Ns)
    say(f"Test-1b SL-MP{order}: errors {['%.3e' % e for e in errs]}, slope {slope:.2f}")
    assert slope == pytest.approx(GOLD["order_sine_no_pp"]["value"][str(order)], abs=0.15)
    want = _oracle_advect("sin", order, W.LIM_MP, Ns[0])
    assert np.max(np.abs(res[0][3] - want)) <= 1e-12


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("order", [5, 7])
def test_positivity_on_quartic_sine(S, order, storage):
    mp = _gpu_advect(S, "sin4", order, W.LIM_MP, 64, storage)
    mpp = _gpu_advect(S, "sin4", order, W.LIM_MPP, 64, storage)
    say(f"Test-1c order {order} storage {storage}: min MP {mp[1]:.3e}, min MPP {mpp[1]:.3e}")
    assert mp[1] < -1e-3
    # FP32 storage: the limited fluxes keep every half-update non-negative,
    # the final rounding to FP32 may leave values of rounding size below zero
    assert mpp[1] >= (0.0 if storage == 0 else -64 * 2.0 ** -24)
    if storage == 0:
        want = _oracle_advect("sin4", order, W.LIM_MPP, 64)
        assert np.max(np.abs(mpp[3] - want)) <= 1e-12


@pytest.mark.parametrize("order", [5, 7])
def test_order_on_quartic_sine_with_pp(S, order):
    Ns = [128, 256]
    res = [_gpu_advect(S, "sin4", order, W.LIM_MPP, N) for N in Ns]
    slope = _slope([r[0] for r in res], Ns)
    say(f"Test-1c SL-MPP{order}: slope {slope:.2f}")
    assert min(r[1] for r in res) >= 0.0
    assert slope > GOLD["order_quartic_sine"]["value"] - 0.5
