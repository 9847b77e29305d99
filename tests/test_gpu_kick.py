"""GPU parity of the two-axis kick pass: the sweeps along v_{D-1} and v_D of
every velocity kick done in one pass over f (square velocity planes of 24,
32, 48 or 64 cells, outflow velocity boundaries, SL-MPP).

Each case runs whole Strang steps twice on the GPU, with the pass and with
SLMPP_FLAG_SEPARATE_KICKS; the two results must be identical bit for bit
(the pass performs the same operations on every pencil), and the first must
match the FP64 oracle (L1 relative 1e-12 in FP64 storage, 1e-5 in FP32, as
for the other whole-step tests).  The timing classes show which path ran.
A field 100 times stronger than the electrostatic one moves velocity
pencils by up to tens of cells (shifts beyond the on-chip ghost cells and
beyond the grid)."""
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


def l1rel(a, b):
    return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))


def _spec(D, nx, nv, order, kappa=-1.0, merge=False):
    s = W.landau_run(D, nx[0], nv[-1], 0.5, 0.3, order)
    s["nx"] = list(nx) + [1] * (3 - D)
    s["nv"] = list(nv) + [1] * (3 - D)
    s["kappa"] = kappa
    s["merge_kicks"] = merge
    return s


CASES = [
    (2, [8, 8], [32, 32], 5),
    (2, [6, 5], [24, 24], 7),
    (2, [4, 4], [48, 48], 7),
    (2, [4, 3], [64, 64], 5),
    (2, [4, 3], [64, 64], 7),
    (3, [4, 3, 4], [8, 24, 24], 5),
    (3, [3, 3, 2], [6, 32, 32], 7),
    (3, [2, 2, 2], [5, 48, 48], 5),
]


def _run(S, spec, storage, nsteps, separate):
    s = dict(spec, separate_kicks=separate)
    ctx = S.Context(S.make_desc(s, storage))
    sx, gv = W.separable_factors(s)
    ctx.init_f_separable(sx, gv)
    ctx.timing_enable(True)
    ctx.step(s["dt"], nsteps)
    tim = ctx.timing_read()
    f = ctx.get_f()
    d = ctx.diag()
    ctx.close()
    return f, tim, d


def _oracle(spec, storage, nsteps):
    f0 = None
    if storage == 1:
        sx, gv = W.separable_factors(spec)
        f0 = O.init_separable(O.make_grid(spec), sx, gv).astype(np.float32).astype(np.float64)
    run = O.Run(spec, f0)
    run.step(spec["dt"], nsteps)
    return run.f


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_kick_pass_equals_separate_sweeps_and_oracle(S, ci, storage):
    D, nx, nv, order = CASES[ci]
    spec = _spec(D, nx, nv, order)
    n = 3
    say(f"case kick pass D={D} nx={nx} nv={nv} order={order} storage={storage}")
    fa, ta, da = _run(S, spec, storage, n, False)
    fb, tb, _ = _run(S, spec, storage, n, True)
    assert ta["kick_plane"]["launches"] == 2 * n and tb["kick_plane"]["launches"] == 0
    assert np.array_equal(fa, fb), np.abs(fa - fb).max()
    err = l1rel(fa, _oracle(spec, storage, n))
    say(f"  L1 rel vs oracle {err:.3e}")
    assert err <= (1e-12 if storage == 0 else 1e-5)
    assert da["nonfinite"] == 0


@pytest.mark.parametrize("storage", [0, 1])
def test_kick_pass_with_merged_kicks(S, storage):
    spec = _spec(3, [3, 2, 3], [6, 32, 32], 7, merge=True)
    n = 4
    say(f"case kick pass + merged kicks storage={storage}")
    fa, ta, _ = _run(S, spec, storage, n, False)
    fb, _, _ = _run(S, spec, storage, n, True)
    assert ta["kick_plane"]["launches"] == n + 1
    assert np.array_equal(fa, fb)
    assert l1rel(fa, _oracle(spec, storage, n)) <= (1e-12 if storage == 0 else 1e-5)


@pytest.mark.parametrize("storage", [0, 1])
def test_kick_pass_large_shifts(S, storage):
    """kappa = -100: velocity shifts far beyond the ghost cells, mass leaving
    through the outflow velocity boundaries."""
    spec = _spec(2, [8, 6], [32, 32], 7, kappa=-100.0)
    n = 3
    say(f"case kick pass large shifts storage={storage}")
    fa, _, da = _run(S, spec, storage, n, False)
    fb, _, _ = _run(S, spec, storage, n, True)
    assert np.array_equal(fa, fb)
    ref = _oracle(spec, storage, n)
    err = l1rel(fa, ref)
    say(f"  L1 rel vs oracle {err:.3e}; mass {da['mass']:.6g}")
    assert err <= (1e-12 if storage == 0 else 1e-5)


@pytest.mark.parametrize("storage", [0, 1])
def test_kick_entry_point_matches_oracle(S, storage):
    """slmpp_kick: every velocity axis by dt with the context's field, on a
    3D3V grid whose (v2, v3) planes take the two-axis pass."""
    spec = _spec(3, [3, 2, 3], [6, 24, 24], 5)
    grid = O.make_grid(spec)
    sx, gv = W.separable_factors(spec)
    f0 = O.init_separable(grid, sx, gv)
    if storage == 1:
        f0 = f0.astype(np.float32).astype(np.float64)
    ctx = S.Context(S.make_desc(spec, storage))
    ctx.init_f_host(f0)
    ctx.field()
    _, acc = ctx.get_field()
    ctx.timing_enable(True)
    ctx.kick(0.7 * spec["dt"])
    assert ctx.timing_read()["kick_plane"]["launches"] == 1
    got = ctx.get_f()
    ctx.close()
    ref = f0.copy()
    nxs = int(np.prod(spec["nx"][:3]))
    for l in range(3):
        O.advect_v(grid, ref, l, 0.7 * spec["dt"], acc[l * nxs:(l + 1) * nxs])
        if storage == 1:
            ref = ref.astype(np.float32).astype(np.float64)
    err = l1rel(got, ref)
    say(f"case slmpp_kick storage={storage}: L1 rel {err:.3e}")
    assert err <= (1e-13 if storage == 0 else 1e-6)
