"""GPU parity of batched ensembles (slmpp_batch_*) against the FP64 oracle.

An ensemble of uneven runs -- 1D1V, 2D2V and 3D3V, SL-MPP5 and SL-MPP7,
electrostatic and gravitational, sub-cell and multi-cell CFL, ragged sizes
-- is advanced together; every run must match the oracle advancing that run
alone (FP64 storage: L1 relative <= 1e-12; FP32 storage: <= 1e-5, the same
bars as single runs).  The captured step graph must give bit-identical
results to the same launches enqueued eagerly, on every replay, with other
work on the stream between replays.
"""
import os

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


def ensemble():
    ragged = W.landau_3d3v(n=5, nv=7, order=5, D=3)
    ragged["nx"] = [5, 4, 6]
    ragged["nv"] = [7, 6, 8]
    return [
        W.landau_1d1v(nx=32, nv=64),                               # MPP5, CFL 0.5
        W.twostream_1d1v(nx=64, nv=96, order=7, cfl=3.0),          # integer shifts
        W.landau_nl_1d1v(nx=48, nv=80, order=5, cfl=1.5),
        W.landau_3d3v(n=8, nv=12, order=7, D=2),                   # 2D2V
        W.jeans_3d3v(n=6, nv=10, order=5, D=2),                    # gravity
        ragged,                                                    # ragged 3D3V
        W.landau_1d1v(nx=20, nv=36, order=7, amp=0.3),
    ]


def _batch(S, specs, storage):
    descs = [S.make_desc(s, storage) for s in specs]
    b = S.Batch(descs, [s["dt"] for s in specs])
    for r, s in enumerate(specs):
        sx, gv = W.separable_factors(s)
        b.init_separable(r, sx, gv)
    return b


def _oracle_runs(specs, storage, nsteps):
    out = []
    for s in specs:
        f0 = None
        if storage == 1:
            sx, gv = W.separable_factors(s)
            f0 = O.init_separable(O.make_grid(s), sx, gv).astype(np.float32).astype(np.float64)
        run = O.Run(s, f0)
        run.step(s["dt"], nsteps)
        out.append(run.f)
    return out


@pytest.mark.parametrize("storage", [0, 1])
def test_batch_every_run_matches_oracle(S, storage):
    specs = ensemble()
    nsteps = 20
    say(f"case batch ensemble of {len(specs)} runs storage={storage} graph {nsteps} steps")
    b = _batch(S, specs, storage)
    b.step(nsteps)
    refs = _oracle_runs(specs, storage, nsteps)
    tol = 1e-12 if storage == 0 else 1e-5
    for r, (s, ref) in enumerate(zip(specs, refs)):
        got = b.get_f(r)
        err = l1rel(got, ref)
        say(f"  run {r} {s['name']} D={s['D']} order={s['order']}: L1 rel {err:.3e}")
        assert np.isfinite(got).all()
        assert err <= tol, (r, s["name"], err)
    b.close()


def test_batch_graph_replays_equal_eager(S):
    import torch

    specs = ensemble()
    say("case batch graph vs eager, FP32, 4 replays")
    g = _batch(S, specs, 1)
    e = _batch(S, specs, 1)
    junk = torch.zeros(1 << 20, device="cuda")
    for rep in range(4):
        g.step(1)
        e.step_eager(1)
        # other eager work and synchronisations between the replays
        junk.add_(1.0)
        torch.cuda.synchronize()
        for r in range(len(specs)):
            a, c = g.get_f(r), e.get_f(r)
            assert np.array_equal(a, c), (rep, r, np.abs(a - c).max())
    # several replays in one call
    g.step(3)
    e.step_eager(3)
    for r in range(len(specs)):
        assert np.array_equal(g.get_f(r), e.get_f(r)), r
    g.close()
    e.close()


def test_batch_autotune_and_cache(S, tmp_path):
    specs = ensemble()
    cache = str(tmp_path / "widths.txt")
    say("case batch autotune")
    b = _batch(S, specs, 1)
    b.autotune(cache)
    widths = {}
    for r, s in enumerate(specs):
        for axis in range(2 * s["D"]):
            w = b.tile_width(r, axis)
            assert w in (8, 16, 32, 64, 128), (r, axis, w)
            widths[(r, axis)] = w
    lines = open(cache).read().split("\n")
    lines = [l for l in lines if l.strip()]
    assert lines and all(len(l.split()) == 5 for l in lines)
    # a second ensemble takes its widths from the cache, adding nothing
    b2 = _batch(S, specs, 1)
    b2.autotune(cache)
    assert open(cache).read().count("\n") == len(lines)
    for (r, axis), w in widths.items():
        assert b2.tile_width(r, axis) == w
    # stepping with the tuned widths still matches the oracle
    b2.step(5)
    refs = _oracle_runs(specs, 1, 5)
    for r, ref in enumerate(refs):
        assert l1rel(b2.get_f(r), ref) <= 1e-5, r
    b.close()
    b2.close()


def test_batch_forced_widths_agree(S, tmp_path):
    """Every tile width gives the same result: a cache forcing W = 8 for
    every shape against the default widths, bit for bit."""
    specs = ensemble()
    say("case batch forced width 8")
    a = _batch(S, specs, 0)
    keys = set()
    for s in specs:
        D = s["D"]
        dims = list(s["nx"][:D]) + list(s["nv"][:D])
        for axis in range(2 * D):
            inner = int(np.prod(dims[axis + 1:])) if axis + 1 < 2 * D else 1
            keys.add(f"f64 {s['order']} {dims[axis]} {inner} 8")
    cache = str(tmp_path / "w8.txt")
    with open(cache, "w") as fh:
        fh.write("\n".join(sorted(keys)) + "\n")
    b = _batch(S, specs, 0)
    b.autotune(cache)
    for r, s in enumerate(specs):
        for axis in range(2 * s["D"]):
            assert b.tile_width(r, axis) == 8
    a.step(3)
    b.step(3)
    for r in range(len(specs)):
        assert np.array_equal(a.get_f(r), b.get_f(r)), r
    a.close()
    b.close()


def same_geometry_ensemble():
    """Runs sharing geometries with different k, amplitude and dt, so that
    the persistent kernels take several runs per launch (sweeps and the
    two-axis kick pass); plus a ragged run that stays in the tile launch."""
    ragged = W.landau_3d3v(n=5, nv=7, order=5, D=3)
    ragged["nx"] = [5, 4, 6]
    ragged["nv"] = [7, 6, 8]
    runs = [W.landau_run(1, 64, 128, k, a, 7) for k, a in ((0.3, 0.01), (0.45, 0.2), (0.6, 0.5))]
    runs += [W.landau_run(2, 16, 32, k, a, 5) for k, a in ((0.35, 0.05), (0.5, 0.3))]
    runs.append(W.landau_run(1, 48, 96, 0.4, 0.1, 5))
    runs.append(ragged)
    runs.append(W.landau_run(3, 4, 24, 0.45, 0.1, 7))  # 24^2 velocity planes, v1 separate
    return runs


@pytest.mark.parametrize("storage", [0, 1])
def test_batch_fast_groups_match_oracle_and_tile_launch(S, storage):
    specs = same_geometry_ensemble()
    nsteps = 10
    say(f"case batch fast groups storage={storage} {len(specs)} runs {nsteps} steps")
    a = _batch(S, specs, storage)
    a.set_fast_min_cells(1)  # every sweep the persistent kernel takes
    b = _batch(S, specs, storage)
    b.set_fast_min_cells(-1)  # none
    changed = sum(a.tile_width(r, ax) != b.tile_width(r, ax)
                  for r, s in enumerate(specs) for ax in range(2 * s["D"]))
    # the last two velocity axes of the 2D2V and 3D3V runs: the two-axis pass
    for r, s in enumerate(specs):
        if s["D"] >= 2 and s["nv"][s["D"] - 2] == s["nv"][s["D"] - 1] in (24, 32, 48, 64):
            D = s["D"]
            assert a.tile_width(r, 2 * D - 2) == a.tile_width(r, 2 * D - 1) == s["nv"][D - 1], r
    a.step(nsteps)
    b.step(nsteps)
    refs = _oracle_runs(specs, storage, nsteps)
    tol = 1e-12 if storage == 0 else 1e-5
    # the sweeps agree bit for bit; the velocity moment of grouped x_1
    # sweeps is summed from tile row sums (another rounding order)
    same = 1e-14 if storage == 0 else 1e-6
    for r, (s, ref) in enumerate(zip(specs, refs)):
        ga, gb = a.get_f(r), b.get_f(r)
        err = l1rel(ga, ref)
        say(f"  run {r} {s['name']} D={s['D']} order={s['order']}: L1 rel {err:.3e}, "
            f"grouped vs tiles {l1rel(ga, gb):.1e}")
        assert l1rel(ga, gb) <= same, (r, np.abs(ga - gb).max())
        assert err <= tol, (r, s["name"], err)
    assert changed > 0
    # the eager form of the grouped launches against its graph, bit for bit
    c = _batch(S, specs, storage)
    c.set_fast_min_cells(1)
    c.step_eager(nsteps)
    for r in range(len(specs)):
        assert np.array_equal(a.get_f(r), c.get_f(r)), r
    # back to the default grouping
    a.set_fast_min_cells(4 << 20)
    a.step(1)
    b.step(1)
    for r in range(len(specs)):
        assert l1rel(a.get_f(r), b.get_f(r)) <= same, r
    a.close()
    b.close()
    c.close()


@pytest.mark.parametrize("storage", [0, 1])
def test_batch_merged_kicks_match_oracle(S, storage):
    """SLMPP_FLAG_MERGE_KICKS on every run: a call of n steps is an opening
    half-kick, n - 1 bodies ending in a full kick and a last body ending in
    a half-kick, as the oracle does for one run.  Graph replay with the
    grouped launches against eager launches with the tile launch only (to
    the rounding order of the fused moment); two calls in a row."""
    specs = [dict(s, merge_kicks=True) for s in same_geometry_ensemble()]
    say(f"case batch merged kicks storage={storage}")
    a = _batch(S, specs, storage)
    a.set_fast_min_cells(1)
    b = _batch(S, specs, storage)
    b.set_fast_min_cells(-1)
    a.step(5)
    b.step_eager(5)
    a.step(3)
    b.step_eager(3)
    tol = 1e-12 if storage == 0 else 1e-5
    for r, s in enumerate(specs):
        f0 = None
        if storage == 1:
            sx, gv = W.separable_factors(s)
            f0 = O.init_separable(O.make_grid(s), sx, gv).astype(np.float32).astype(np.float64)
        run = O.Run(s, f0)
        run.step(s["dt"], 5)
        run.step(s["dt"], 3)
        ga, gb = a.get_f(r), b.get_f(r)
        err = l1rel(ga, run.f)
        say(f"  run {r} {s['name']} D={s['D']}: L1 rel {err:.3e}")
        assert l1rel(ga, gb) <= (1e-14 if storage == 0 else 1e-6), r
        assert err <= tol, (r, err)
    a.close()
    b.close()


def test_batch_error_paths(S):
    specs = ensemble()[:2]
    b = _batch(S, specs, 0)
    with pytest.raises(S.SlmppError) as e:
        b.get_f(5)
    assert e.value.status == S.ERR_INVALID
    with pytest.raises(S.SlmppError) as e:
        b.step(0)
    assert e.value.status == S.ERR_INVALID
    assert b.tile_width(0, 2) == 0  # a 1D1V run has axes 0 and 1
    b.close()


@pytest.mark.parametrize("storage", [0, 1])
def test_batch_ensemble_shaped_2d2v_members(S, storage):
    """2D2V runs shaped like the 256-run ensemble's members (64^2 velocity
    planes, 32-cell x_1 pencils) but 32 x 4 in space, SL-MPP5 and SL-MPP7,
    two runs per order, plus one 1D1V run.  With every eligible sweep
    grouped, the x_1 sweeps take the persistent kernel's 128-pencil tiles of
    16 cells with the fused moment and the kicks the two-axis pass over the
    64^2 planes, at both orders; with none grouped, the tile launch (its
    x_1 tiles leave the moment's row sums too).  Both against the oracle
    for three steps."""
    specs = []
    for order in (5, 7):
        for k, a in ((0.35, 0.05), (0.55, 0.3)):
            s = W.landau_run(2, 32, 64, k, a, order)
            s["nx"] = [32, 4, 1]
            specs.append(s)
    specs.append(W.landau_1d1v(nx=32, nv=64, order=7))
    nsteps = 3
    refs = _oracle_runs(specs, storage, nsteps)
    tol = 1e-12 if storage == 0 else 1e-5
    for min_cells in (1, -1):
        say(f"case batch ensemble-shaped 2d2v storage={storage} min_cells={min_cells}")
        b = _batch(S, specs, storage)
        b.set_fast_min_cells(min_cells)
        if min_cells == 1:
            for r in range(4):
                assert b.tile_width(r, 0) == 128, (r, b.tile_width(r, 0))
                assert b.tile_width(r, 2) == b.tile_width(r, 3) == 64, r
        b.step(nsteps)
        for r, (s, ref) in enumerate(zip(specs, refs)):
            got = b.get_f(r)
            err = l1rel(got, ref)
            say(f"  run {r} D={s['D']} order={s['order']}: L1 rel {err:.3e}")
            assert err <= tol, (min_cells, r, err)
        b.close()
