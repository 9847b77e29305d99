"""Parity at the benchmark sizes, in the launch configuration bench.py uses.

The grids are too large for the oracle as a whole (48^3 x 48^3 = 1.2e10
cells), so each sweep is checked on sampled pencils: the pencil is read
before the GPU sweep, the oracle advances it alone (same speed, same dt,
FP64 arithmetic on the stored FP32 values), and the GPU result must agree to
64 FP32 ulps of the pencil's largest value.  Whole steps are checked through
properties that hold at any size: finiteness, positivity, mass balance and
(for an x1-only perturbation) independence of x2 and x3.  The 32^3 x 32^3
Jeans grid (8.6 GB in FP64) is also stepped whole on the oracle and compared
over every cell.
"""
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


def _pencil_index(shape, axis, rng):
    idx = [int(rng.integers(0, n)) for n in shape]
    idx[axis] = slice(None)
    return tuple(idx)


def _sampled_sweeps(S, spec, npencils=48, seed=7, fp64=False):
    import torch

    D = spec["D"]
    ctx = S.Context(S.make_desc(spec, S.F64 if fp64 else S.F32))
    s, gv = W.separable_factors(spec)
    ctx.init_f_separable(s, gv)
    ctx.field()
    ctx.sync()
    f = ctx.f
    shape = tuple(f.shape)
    grid = O.make_grid(spec)
    rng = np.random.default_rng(seed)
    dt = spec["dt"]
    worst = 0.0
    for axis in range(2 * D):
        _, acc = ctx.get_field()
        nxs = int(np.prod(shape[:D]))
        picks = [_pencil_index(shape, axis, rng) for _ in range(npencils)]
        before = [f[p].double().cpu().numpy() for p in picks]
        l = axis if axis < D else axis - D
        if axis < D:
            h = (spec["x_hi"][l] - spec["x_lo"][l]) / spec["nx"][l]
            ctx.advect_x(l, dt)
            bc = spec["x_bc"]
        else:
            h = (spec["v_hi"][l] - spec["v_lo"][l]) / spec["nv"][l]
            comp = torch.tensor(acc[l * nxs:(l + 1) * nxs], dtype=torch.float64, device=f.device)
            ctx.advect_v(l, 0.5 * dt, comp)
            bc = spec["v_bc"]
        ctx.sync()
        say(f"case {spec['name']} axis={axis}")
        for p, g0 in zip(picks, before):
            if axis < D:
                jv = p[D + l]
                c = O.cell_center(spec["v_lo"][l], spec["v_hi"][l], spec["nv"][l], jv)
                xi = O.xi(c, dt, h)
            else:
                ix = int(np.ravel_multi_index(p[:D], shape[:D]))
                xi = O.xi(acc[l * nxs + ix], 0.5 * dt, h)
            want = O.sweep_pencil(g0, xi, order=spec["order"], limiter=spec["limiter"],
                                  alpha=spec["alpha"], bc=bc)
            got = f[p].double().cpu().numpy()
            err = np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)
            worst = max(worst, err)
            assert err <= (1e-13 if fp64 else 64 * 2.0 ** -24), (axis, p, err)
    return ctx, worst, grid


@pytest.mark.parametrize("which", ["landau_3d3v_48", "jeans_3d3v_32", "landau_3d3v_48_f64"])
def test_fullsize_sampled_pencils_and_step(S, which):
    """Every axis swept once at the benchmark size (FP32, and FP64 storage
    for the 48^3 x 48^3 grid: 98 GB of f), sampled pencils against the
    oracle, then two whole steps checked by their invariants."""
    spec = W.jeans_3d3v(n=32, order=5) if which == "jeans_3d3v_32" else W.landau_3d3v(n=48, order=7)
    fp64 = which.endswith("_f64")
    ctx, worst, _ = _sampled_sweeps(S, spec, fp64=fp64)
    say(f"  worst sampled-pencil error {worst:.3e} (FP32 ulps of max: {worst / 2.0 ** -24:.1f})")
    d0 = ctx.diag()
    ctx.step(spec["dt"], 2)
    d1 = ctx.diag()
    say(f"  mass {d0['mass']:.12e} -> {d1['mass']:.12e}, f_min {d1['f_min']:.3e}")
    assert d1["nonfinite"] == 0
    assert d1["f_min"] >= -1e-6 * d1["f_max"]
    # periodic space, outflow velocity with ~e^-12 .. e^-18 at the edge:
    # the mass changes by far less than FP32 rounding of the values
    assert abs(d1["mass"] - d0["mass"]) <= (1e-9 if fp64 else 1e-6) * abs(d0["mass"])
    ctx.close()


def test_fullsize_jeans_independent_of_x2_x3(S):
    """The Jeans perturbation depends on x1 only; after steps at 32^3 x 32^3
    every (x2, x3) column must hold the same values (x2/x3 sweeps act on
    uniform pencils, where the MP constraint returns the data exactly)."""
    import torch

    spec = W.jeans_3d3v(n=32, order=5)
    ctx = S.Context(S.make_desc(spec, S.F32))
    s, gv = W.separable_factors(spec)
    ctx.init_f_separable(s, gv)
    ctx.step(spec["dt"], 3)
    ctx.sync()
    f = ctx.f
    ref = f[:, 0, 0].double()
    rng = np.random.default_rng(3)
    for _ in range(16):
        i2, i3 = (int(x) for x in rng.integers(0, 32, size=2))
        col = f[:, i2, i3].double()
        rel = (torch.abs(col - ref).max() / torch.abs(ref).max()).item()
        assert rel <= 1e-6, (i2, i3, rel)
    ctx.close()


@pytest.mark.parametrize("which", ["landau_3d3v_48", "jeans_3d3v_32", "landau_3d3v_48_f64"])
def test_fullsize_kick_velocity_blocks(S, which):
    """A velocity kick at the benchmark size (v1 sweep, then the two-axis
    pass over the (v2, v3) planes), checked on the whole velocity block of
    sampled spatial cells: the kick acts on each block alone with that
    cell's acceleration.  In FP32 the oracle rounds to FP32 after each sweep,
    as the GPU stores between sweeps (in HBM after v1, in LDS after v2)."""
    spec = W.jeans_3d3v(n=32, order=5) if which == "jeans_3d3v_32" else W.landau_3d3v(n=48, order=7)
    fp64 = which.endswith("_f64")
    D = spec["D"]
    ctx = S.Context(S.make_desc(spec, S.F64 if fp64 else S.F32))
    s, gv = W.separable_factors(spec)
    ctx.init_f_separable(s, gv)
    ctx.field()
    _, acc = ctx.get_field()
    f = ctx.f
    shape = tuple(f.shape)
    nxs = int(np.prod(shape[:D]))
    rng = np.random.default_rng(11)
    cells = [tuple(int(rng.integers(0, n)) for n in shape[:D]) for _ in range(6)]
    before = [f[c].double().cpu().numpy() for c in cells]
    dt = 0.5 * spec["dt"]
    ctx.timing_enable(True)
    ctx.kick(dt)
    tim = ctx.timing_read()
    assert tim["kick_plane"]["launches"] == 1
    say(f"case {which} kick on {len(cells)} velocity blocks")
    worst = 0.0
    for c, blk in zip(cells, before):
        ix = int(np.ravel_multi_index(c, shape[:D]))
        ref = blk.copy()
        for l in range(D):
            h = (spec["v_hi"][l] - spec["v_lo"][l]) / spec["nv"][l]
            xi = O.xi(acc[l * nxs + ix], dt, h)
            O.sweep_lines(ref, l, xi, order=spec["order"], limiter=spec["limiter"],
                          alpha=spec["alpha"], bc=spec["v_bc"])
            if not fp64:
                ref = ref.astype(np.float32).astype(np.float64)
        got = f[c].double().cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
        assert err <= (1e-13 if fp64 else 64 * 2.0 ** -24), (c, err)
    say(f"  worst block error {worst:.3e} (FP32 ulps of max: {worst / 2.0 ** -24:.1f})")
    ctx.close()


def test_fullsize_jeans_32_steps_vs_oracle(S):
    """The Jeans workload at its full size, 32^3 x 32^3 (1.07e9 cells: 8.6 GB
    of FP64 on the host), two Strang steps on the GPU against two on the
    oracle, compared over the whole of f: L1 and max relative <= 1e-12 with
    FP64 storage, <= 1e-5 with FP32 storage (FP64 moment and field in both)."""
    spec = W.jeans_3d3v(n=32, order=5)
    nsteps = 2
    say(f"case jeans_3d3v_32 oracle {nsteps} steps")
    run = O.Run(spec)
    run.step(spec["dt"], nsteps)
    want = run.f
    del run
    norm1 = np.abs(want).sum()
    normx = np.abs(want).max()
    s, gv = W.separable_factors(spec)
    for fp64 in (True, False):
        say(f"case jeans_3d3v_32 gpu fp64={fp64} {nsteps} steps")
        ctx = S.Context(S.make_desc(spec, S.F64 if fp64 else S.F32))
        ctx.init_f_separable(s, gv)
        ctx.step(spec["dt"], nsteps)
        got = ctx.get_f()
        ctx.close()
        got -= want
        np.abs(got, out=got)
        l1 = got.sum() / norm1
        mx = got.max() / normx
        del got
        say(f"  L1 rel {l1:.3e}, max rel {mx:.3e}")
        assert l1 <= (1e-12 if fp64 else 1e-5)
        assert mx <= (1e-12 if fp64 else 1e-5)
