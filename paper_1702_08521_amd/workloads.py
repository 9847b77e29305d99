"""Seeded, synthetic workloads shaped like the paper's test problems.

This module only *generates inputs*: grid descriptions, initial-condition
factor tables and seeded random data.  It holds none of the scheme's
arithmetic, so both the HIP path and the CPU oracle may take their inputs
from it.

Every initial condition used here is separable,
    f(x, v) = s(x) * g_1(v_1) * ... * g_D(v_D),
so a workload is fully described by the spatial factor s (prod(nx) values)
and one velocity factor per axis (nv_l values).  Values are point samples
at cell centres (the paper compares cell values with point values of the
analytic solution, e.g. the L1 error of Test-1 in Sec. 3.1).

Workloads (named by what they are):
  landau_1d1v     linear Landau damping, Test-3 of Sec. 3.3: k = 0.5,
                  A = 0.01, x in [0, 4 pi), v in [-6, 6], 64 x 128, SL-MPP5.
  landau_nl_1d1v  nonlinear Landau damping (A = 0.5), 256 x 512, SL-MPP7,
                  v in [-8, 8], time step at x-CFL 3.
  twostream_1d1v  two-stream instability, f0 = (1 + 0.05 cos 0.5x)
                  v^2 exp(-v^2/2)/sqrt(2 pi), same grid as above.
  jeans_3d3v      self-gravitating Maxwellian with a 1% density wave,
                  32^3 x 32^3, box L = 1, G = sigma = 1, v in [-5, 5]^3,
                  mean density from k/k_J (0.5 or 1.1), SL-MPP5.
  landau_3d3v     electrostatic Landau damping in three dimensions,
                  48^3 x 48^3, x in [0, 4 pi)^3, v in [-6, 6]^3, SL-MPP7.
  collapse_3d3v   spherical collapse of a uniform-density sphere (Test-4),
                  64^3 x 32^3, isolated field boundaries, outflow in x, v.
  ensemble        256 independent Landau-type runs of uneven sizes (224
                  1D1V up to 256 x 512, 32 2D2V at 32^2 x 64^2), mixed
                  SL-MPP5/7, seeded k and amplitude.
"""
from __future__ import annotations

import math

import numpy as np

BC_PERIODIC = 0
BC_OUTFLOW = 1
LIM_NONE = 0
LIM_MP = 1
LIM_MPP = 2

SQRT_2PI = math.sqrt(2.0 * math.pi)


def spec(D, nx, nv, x_lo, x_hi, v_lo, v_hi, *, order=5, limiter=LIM_MPP, alpha=4.0,
         kappa=-1.0, poisson_order=6, x_bc=BC_PERIODIC, v_bc=BC_OUTFLOW, **extra):
    def v3(x, fill):
        x = list(x) if isinstance(x, (list, tuple)) else [x] * D
        return x + [fill] * (3 - len(x))

    s = dict(D=D, nx=v3(nx, 1), nv=v3(nv, 1), x_lo=v3(x_lo, 0.0), x_hi=v3(x_hi, 1.0),
             v_lo=v3(v_lo, 0.0), v_hi=v3(v_hi, 1.0), order=order, limiter=limiter,
             alpha=alpha, kappa=kappa, poisson_order=poisson_order, x_bc=x_bc, v_bc=v_bc)
    s.update(extra)
    return s


def centers(lo, hi, n):
    """Cell centres lo + (j + 1/2) (hi - lo)/n, j = 0..n-1."""
    d = (hi - lo) / n
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * d


def spacing(lo, hi, n):
    return (hi - lo) / n


def maxwellian(v, sigma=1.0):
    return np.exp(-v * v / (2.0 * sigma * sigma)) / (SQRT_2PI * sigma)


# ----------------------------------------------------------------------------
# workload specs
# ----------------------------------------------------------------------------
def landau_1d1v(nx=64, nv=128, amp=0.01, k=0.5, order=5, cfl=0.5):
    L = 2.0 * math.pi / k
    s = spec(1, nx, nv, 0.0, L, -6.0, 6.0, order=order, kappa=-1.0, ic="landau",
             amp=amp, k=k, name="landau_1d1v")
    s["dt"] = cfl * spacing(0.0, L, nx) / 6.0
    return s


def landau_nl_1d1v(nx=256, nv=512, order=7, cfl=3.0):
    L = 4.0 * math.pi
    s = spec(1, nx, nv, 0.0, L, -8.0, 8.0, order=order, kappa=-1.0, ic="landau",
             amp=0.5, k=0.5, name="landau_nl_1d1v")
    s["dt"] = cfl * spacing(0.0, L, nx) / 8.0
    return s


def twostream_1d1v(nx=256, nv=512, order=7, cfl=3.0, amp=0.05):
    L = 4.0 * math.pi
    s = spec(1, nx, nv, 0.0, L, -8.0, 8.0, order=order, kappa=-1.0, ic="twostream",
             amp=amp, k=0.5, name="twostream_1d1v")
    s["dt"] = cfl * spacing(0.0, L, nx) / 8.0
    return s


def jeans_3d3v(n=32, k_over_kj=0.5, order=5, cfl=0.2, D=3, nv=None):
    """Gravity, G = sigma = 1, L = 1, k = 2 pi;  k_J^2 = 4 pi G rho_bar."""
    nv = n if nv is None else nv
    k = 2.0 * math.pi
    kj = k / k_over_kj
    rho_bar = kj * kj / (4.0 * math.pi)
    s = spec(D, n, nv, 0.0, 1.0, -5.0, 5.0, order=order, kappa=4.0 * math.pi,
             ic="jeans", amp=0.01, k=k, rho_bar=rho_bar, name="jeans_%dd%dv" % (D, D))
    s["dt"] = cfl * spacing(0.0, 1.0, n) / 5.0
    return s


def landau_3d3v(n=48, order=7, cfl=0.2, D=3, nv=None, amp=0.01):
    nv = n if nv is None else nv
    L = 4.0 * math.pi
    s = spec(D, n, nv, 0.0, L, -6.0, 6.0, order=order, kappa=-1.0, ic="landau_sum",
             amp=amp, k=0.5, name="landau_%dd%dv" % (D, D))
    s["dt"] = cfl * spacing(0.0, L, n) / 6.0
    return s


def landau_run(D, nx, nv, k, amp, order, cfl=0.5):
    """Landau-type run (1 + A sum_l cos k x_l) Maxwellian on [0, 2 pi/k)^D
    x [-6, 6]^D with dt at x-CFL `cfl` for the fastest velocity."""
    L = 2.0 * math.pi / k
    s = spec(D, nx, nv, 0.0, L, -6.0, 6.0, order=order, kappa=-1.0, ic="landau_sum",
             amp=amp, k=k, name="landau_%dd%dv" % (D, D))
    s["dt"] = cfl * spacing(0.0, L, nx) / 6.0
    return s


ENSEMBLE_SEED = 170208521


def ensemble(n_runs=256, n_2d=32, seed=ENSEMBLE_SEED, nx_1d=(32, 48, 64, 96, 128, 192, 256),
             nv_1d=(64, 96, 128, 192, 256, 384, 512), shape_2d=(32, 64)):
    """Seeded ensemble of independent Landau-type runs of uneven sizes:
    n_runs - n_2d 1D1V runs with N_x, N_v drawn from the lists, n_2d 2D2V
    runs at shape_2d[0]^2 x shape_2d[1]^2; k ~ U[0.3, 0.6], amplitude
    ~ logU[1e-3, 0.5], order 5 or 7 with equal odds, dt at x-CFL 0.5."""
    rng = np.random.default_rng(seed)
    runs = []
    for r in range(n_runs):
        two = r >= n_runs - n_2d
        k = float(rng.uniform(0.3, 0.6))
        amp = float(math.exp(rng.uniform(math.log(1e-3), math.log(0.5))))
        order = 5 if rng.random() < 0.5 else 7
        if two:
            nx, nv, D = shape_2d[0], shape_2d[1], 2
        else:
            nx = int(rng.choice(nx_1d))
            nv = int(rng.choice(nv_1d))
            D = 1
        runs.append(landau_run(D, nx, nv, k, amp, order))
    return runs


def collapse_3d3v(nx=64, nv=32, order=5, cfl=0.5):
    """Test-4 of Sec. 3.4: a uniform-density sphere of mass M = 1 and radius
    2R (R = 1, G = 1, so T = V = 1) with the Maxwellian of sigma^2 = GM/(20R)
    at every point inside; x, v in [-3, 3]^3, outflow in both, isolated
    field boundaries."""
    L, V = 3.0, 3.0
    s = spec(3, nx, nv, -L, L, -V, V, order=order, kappa=4.0 * math.pi, x_bc=BC_OUTFLOW,
             v_bc=BC_OUTFLOW, ic="collapse", rho0=3.0 / (32.0 * math.pi), sigma2=0.05,
             radius=2.0, field_bc="isolated", name="collapse_3d3v")
    s["dt"] = cfl * spacing(-L, L, nx) / V
    return s


def advection_1d1v(nx, nv, v_lo, v_hi, profile, order=5, limiter=LIM_MPP):
    """Free streaming (no field): every v-row is advected along x with
    speed v; used with a spatial profile of Test-1."""
    return spec(1, nx, nv, 0.0, 1.0, v_lo, v_hi, order=order, limiter=limiter,
                kappa=0.0, ic="profile", profile=profile, name="advection_1d1v")


# ----------------------------------------------------------------------------
# initial conditions
# ----------------------------------------------------------------------------
def test1_profile(name, x):
    """Initial profiles of Test-1 (Sec. 3.1)."""
    if name == "rect":
        return np.where((x >= 0.25) & (x <= 0.75), 1.0, 0.0)
    if name == "sin":
        return 1.0 + np.sin(2.0 * np.pi * x)
    if name == "sin4":
        return np.sin(4.0 * np.pi * x) ** 4
    raise ValueError(name)


def separable_factors(s):
    """(s_x, [g_1, .., g_D]) for the workload spec s."""
    D = s["D"]
    xs = [centers(s["x_lo"][l], s["x_hi"][l], s["nx"][l]) for l in range(D)]
    vs = [centers(s["v_lo"][l], s["v_hi"][l], s["nv"][l]) for l in range(D)]
    grids = np.meshgrid(*xs, indexing="ij")
    ic = s["ic"]
    if ic == "landau":
        sx = 1.0 + s["amp"] * np.cos(s["k"] * grids[0])
        gv = [maxwellian(v) for v in vs]
    elif ic == "landau_sum":
        sx = 1.0 + s["amp"] * sum(np.cos(s["k"] * g) for g in grids)
        gv = [maxwellian(v) for v in vs]
    elif ic == "twostream":
        sx = 1.0 + s["amp"] * np.cos(s["k"] * grids[0])
        gv = [vs[0] * vs[0] * np.exp(-vs[0] * vs[0] / 2.0) / SQRT_2PI] + \
             [maxwellian(v) for v in vs[1:]]
    elif ic == "jeans":
        sx = s["rho_bar"] * (1.0 + s["amp"] * np.cos(s["k"] * grids[0]))
        gv = [maxwellian(v) for v in vs]
    elif ic == "collapse":
        r2 = sum(gg * gg for gg in grids)
        sx = np.where(r2 < s["radius"] ** 2, s["rho0"], 0.0)
        sig = math.sqrt(s["sigma2"])
        gv = [maxwellian(v, sig) for v in vs]
    elif ic == "profile":
        sx = test1_profile(s["profile"], grids[0])
        gv = [np.ones_like(v) for v in vs]
    else:
        raise ValueError(ic)
    return np.ascontiguousarray(sx, dtype=np.float64).ravel(), \
        [np.ascontiguousarray(g, dtype=np.float64) for g in gv]


# ----------------------------------------------------------------------------
# seeded random data
# ----------------------------------------------------------------------------
def random_field(shape, seed, zeros=0.2, spikes=0.01, spike_scale=100.0):
    """U[0,1) with a fraction of exact zeros and of large spikes."""
    rng = np.random.default_rng(seed)
    f = rng.random(shape)
    f[rng.random(shape) < zeros] = 0.0
    sp = rng.random(shape) < spikes
    f[sp] *= spike_scale
    return f


def random_accel(n_space, D, seed, scale):
    rng = np.random.default_rng(seed)
    return (rng.random(D * n_space) * 2.0 - 1.0) * scale
