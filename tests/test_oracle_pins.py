"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each check is a closed form,
an exact invariant, a special case with a known answer, a number printed in
the paper (tests/golden/paper_values.json, each with its citation) or a root
of a dispersion relation computed here with scipy.  They run on the CPU.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1702_08521_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# ---------------------------------------------------------------------------
# CSL flux polynomial (Sec. 2.1.2)
# ---------------------------------------------------------------------------
def _poly_cell_averages(coef, j, h=1.0):
    """Exact cell averages of the polynomial sum coef[k] x^k over
    [ (j-1/2) h, (j+1/2) h ]."""
    P = np.polynomial.Polynomial(coef).integ()
    lo = (j - 0.5) * h
    hi = (j + 0.5) * h
    return (P(hi) - P(lo)) / h


def _foot_average(coef, x_face, zeta, h=1.0):
    """(1/(zeta h)) * integral of the polynomial over [x_face - zeta h, x_face]:
    the exact flux of the CSL identity for a speed c > 0."""
    P = np.polynomial.Polynomial(coef).integ()
    return (P(x_face) - P(x_face - zeta * h)) / (zeta * h)


@pytest.mark.parametrize("order,degree", [(5, 0), (5, 2), (5, 4), (7, 4), (7, 6)])
@pytest.mark.parametrize("zeta", [0.05, 0.2, 0.37, 0.5, 0.8, 1.0])
def test_csl_flux_exact_for_polynomials(oracle, order, degree, zeta):
    """The CSL flux is the exact foot average whenever the data are cell
    averages of a polynomial of degree <= order-1."""
    rng = np.random.default_rng(1000 * order + degree)
    for _ in range(5):
        coef = rng.normal(size=degree + 1)
        half = order // 2 + 1  # stencil f_{i-3..i+1} (5) or f_{i-4..i+2} (7)
        js = np.arange(-half, order - half)  # cell indices relative to i
        avg = _poly_cell_averages(coef, js)
        got = oracle.csl_flux(avg, order, zeta)
        want = _foot_average(coef, -0.5, zeta)  # interface i-1/2 at x = -1/2
        assert got == pytest.approx(want, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("order", [5, 7])
def test_csl_flux_not_exact_beyond_design_degree(oracle, order):
    """Sanity of the pin above: one degree more is no longer reproduced."""
    coef = np.zeros(order + 1)
    coef[order] = 1.0
    half = order // 2 + 1
    js = np.arange(-half, order - half)
    got = oracle.csl_flux(_poly_cell_averages(coef, js), order, 0.3)
    want = _foot_average(coef, -0.5, 0.3)
    assert abs(got - want) > 1e-6


@pytest.mark.parametrize("order", [5, 7])
def test_csl_flux_limits(oracle, order):
    """zeta = 1: the whole upwind cell crosses the face, Phi = f_{i-1};
    zeta -> 0: Phi is the MP5/MP7 interface value printed in Sec. 2.1.1."""
    rng = np.random.default_rng(7)
    key = "mp5_interface_weights" if order == 5 else "mp7_interface_weights"
    w = np.array(GOLD[key]["value"], dtype=float) / GOLD[key]["denominator"]
    for _ in range(20):
        s = rng.random(order)
        upwind = s[order // 2]  # f_{i-1}
        assert oracle.csl_flux(s, order, 1.0) == pytest.approx(upwind, rel=1e-14, abs=1e-15)
        assert oracle.csl_flux(s, order, 0.0) == pytest.approx(float(w @ s), rel=1e-14, abs=1e-15)


# ---------------------------------------------------------------------------
# MP constraint (App. A) and PP limiter (Sec. 2.1.1)
# ---------------------------------------------------------------------------
def test_minmod_median_definitions(oracle):
    assert oracle.minmod2(2.0, 3.0) == 2.0
    assert oracle.minmod2(-2.0, -3.0) == -2.0
    assert oracle.minmod2(2.0, -3.0) == 0.0
    assert oracle.minmod4(1.0, 2.0, 0.5, 3.0) == 0.5
    assert oracle.minmod4(-1.0, -2.0, -0.5, -3.0) == -0.5
    assert oracle.minmod4(1.0, 2.0, -0.5, 3.0) == 0.0
    for a, b, c in [(1, 2, 3), (3, 1, 2), (2, 3, 1), (5, 5, 1), (-1, 4, 0)]:
        assert oracle.median3(a, b, c) == sorted([a, b, c])[1]


def test_mp_constant_data_passes_bitwise(oracle):
    for c in [0.0, 1.0, 3.7e-5, 123.456]:
        for fint in [c, c * 1.1 + 0.3, -2.0]:
            assert oracle.mp(fint, c, c, c, c, c) == c


def test_mp_leaves_smooth_monotone_data_alone(oracle):
    """Linear data: the exact interface value lies between f_i and f_{i+1}
    and must pass unchanged (App. A step 3)."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        a, b = rng.normal(), rng.normal()
        f = a + b * np.arange(-2, 3)  # f_{i-2..i+2}
        exact = a + b * 0.5           # value at the face i+1/2
        assert oracle.mp(exact, *f) == pytest.approx(exact, rel=1e-14, abs=1e-14)


def test_mp_caps_an_overshoot_at_a_step(oracle):
    """A step 0,0,0,1,1: any interface value above 1 (overshoot) is brought
    back into [0, 1]."""
    for fint in [1.3, 2.0, -0.4]:
        v = oracle.mp(fint, 0.0, 0.0, 0.0, 1.0, 1.0)
        assert 0.0 <= v <= 1.0


def test_mp_hand_worked_examples(oracle):
    """Two cases worked by hand through the seven steps of App. A.

    (a) steep rise 0, 0, 1, 10, 20 with f^int = 100: no early accept
        (f* = 1 + minmod(9, 4) = 5), curvature bounds vanish (mixed signs),
        f^UL = 1 + alpha, f^min = 1, f^max = min(10, f^UL) -> result f^UL.
    (b) smooth maximum 0, 0.8, 1, 0.8, 0 with f^int = 1.2: d = (-0.6, -0.4,
        -0.6), d^M4 = -0.4 on both sides, f^MD = 0.9 + 0.2 = 1.1,
        f^max = min(1.1, 1.8) -> result f^MD = 1.1."""
    for alpha in (4.0, 3.0, 2.5):
        assert oracle.mp(100.0, 0.0, 0.0, 1.0, 10.0, 20.0, alpha) == pytest.approx(1.0 + alpha)
    assert oracle.mp(1.2, 0.0, 0.8, 1.0, 0.8, 0.0) == pytest.approx(1.1, rel=1e-14)
    # below the lower bound on the same maximum: f^min = max(0.8, f^LC) = 0.8
    assert oracle.mp(0.3, 0.0, 0.8, 1.0, 0.8, 0.0) == pytest.approx(0.8, rel=1e-14)


def test_pp_theta_closed_form(oracle):
    """f_i = 1, Phibar = 3: U+ = 1 - 2 nu 3 < 0 -> theta = (1-2nu)/((1-2nu) - U+)
    so the limited flux is f_i / (2 nu) (outflow capped at half the cell)."""
    assert oracle.pp(3.0, 1.0, 1.0, 0.2) == pytest.approx(1.0 / 0.4, rel=1e-15)
    assert oracle.pp(3.0, 1.0, 1.0, 0.5) == pytest.approx(1.0, rel=1e-15)
    # no limiting when both half-updates stay non-negative
    assert oracle.pp(0.9, 1.0, 1.0, 0.2) == 0.9
    # negative flux into the downwind cell: U- = f_R + 2 nu Phi < 0
    got = oracle.pp(-5.0, 1.0, 1.0, 0.25)
    u_up = 1.0 + 2 * 0.25 * 1.0
    u = 1.0 + 2 * 0.25 * -5.0
    th = u_up / (u_up - u)
    assert got == pytest.approx(th * -5.0 + (1 - th) * 1.0, rel=1e-15)


def test_pp_is_continuous_below_half_courant_and_jumps_above(oracle):
    """With nu <= 1/2 the limited flux is continuous in Phibar: where U+
    changes sign theta = U^UP / (U^UP - U+) -> 1 (U^UP = (1 - 2 nu) f_i
    >= 0).  Above 1/2 U^UP < 0, theta drops from 1 to 0 at the sign change
    and the flux jumps from f_i / (2 nu) to f_i (the PP property itself
    needs nu < 1/2, Sec. 2.1.1)."""
    eps = 1e-9
    for nu in (0.2, 0.4, 0.5):
        t = 1.0 / (2 * nu)  # U+ = 0 at Phibar = f_i / (2 nu), f_i = 1
        below, above = oracle.pp(t - eps, 1.0, 1.0, nu), oracle.pp(t + eps, 1.0, 1.0, nu)
        assert abs(above - below) <= 1e-8, nu
    nu = 0.9
    t = 1.0 / (2 * nu)
    assert oracle.pp(t - eps, 1.0, 1.0, nu) == pytest.approx(t, abs=1e-8)
    assert oracle.pp(t + eps, 1.0, 1.0, nu) == 1.0


def test_pp_keeps_random_pencils_non_negative(oracle):
    """Positivity (Sec. 2.1.1): f >= 0 and |zeta| <= 1/2 give f^{n+1} >= 0,
    for any integer shift, on data with zeros and large spikes.  In floating
    point a cell that is exactly zero may end a few ulps of max(f) below
    zero (the difference of two nearly equal limited fluxes)."""
    rng = np.random.default_rng(11)
    for order in (5, 7):
        for bc in (W.BC_PERIODIC, W.BC_OUTFLOW):
            f = W.random_field((400, 64), seed=order * 10 + bc)
            for xi in rng.uniform(-3.0, 3.0, size=12):
                g = f.copy()
                oracle.sweep_lines(g, 1, float(xi), order=order, limiter=W.LIM_MPP, bc=bc)
                assert g.min() >= -1e-15 * f.max(), (order, bc, xi)


def test_mp_alone_goes_negative_on_quartic_sine(oracle):
    """Test-1c (Sec. 3.1.3): without the PP limiter negative values appear;
    with it they do not."""
    N = 64
    x = W.centers(0.0, 1.0, N)
    f0 = W.test1_profile("sin4", x)
    mins = {}
    for lim in (W.LIM_MP, W.LIM_MPP):
        g = f0.copy()
        for _ in range(int(round(1.0 / (0.2 / N)))):
            g = oracle.sweep_pencil(g, 0.2, order=5, limiter=lim)
        mins[lim] = g.min()
    assert mins[W.LIM_MP] < -1e-3
    assert mins[W.LIM_MPP] >= 0.0


# ---------------------------------------------------------------------------
# transport identities
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lim", [W.LIM_NONE, W.LIM_MP, W.LIM_MPP])
@pytest.mark.parametrize("order", [5, 7])
def test_integer_shift_is_exact(oracle, lim, order):
    rng = np.random.default_rng(5)
    g = W.random_field(37, seed=9)
    for k in [-5, -3, -1, 0, 1, 2, 3, 40]:
        out = oracle.sweep_pencil(g, float(k), order=order, limiter=lim, bc=W.BC_PERIODIC)
        assert np.array_equal(out, np.roll(g, k))
        out = oracle.sweep_pencil(g, float(k), order=order, limiter=lim, bc=W.BC_OUTFLOW)
        want = np.zeros_like(g)
        if k >= 0:
            want[k:] = g[: g.size - k] if k < g.size else []
        else:
            want[:k] = g[-k:]
        assert np.array_equal(out, want)
    del rng


def test_dyadic_free_streaming_is_bitwise(oracle):
    """dx = 1/64, speed 1, dt = 3/64: xi = 3 exactly, so three x-sweeps move
    the profile by nine cells without any rounding."""
    s = W.advection_1d1v(64, 1, 0.5, 1.5, "sin4")
    g = oracle.make_grid(s)
    f = oracle.init_separable(g, *W.separable_factors(s))
    f0 = f.copy()
    for _ in range(3):
        oracle.advect_x(g, f, 0, 3.0 / 64.0)
    assert np.array_equal(f, np.roll(f0, 9, axis=0))


def test_translation_and_reflection_equivariance(oracle):
    rng = np.random.default_rng(21)
    g = W.random_field(50, seed=4)
    for xi in rng.uniform(-2.4, 2.4, size=10):
        if abs(abs(xi - math.floor(xi)) - 0.5) < 1e-6:
            continue
        for order in (5, 7):
            a = oracle.sweep_pencil(np.roll(g, 7), xi, order=order)
            b = np.roll(oracle.sweep_pencil(g, xi, order=order), 7)
            assert np.array_equal(a, b)
            for bc in (W.BC_PERIODIC, W.BC_OUTFLOW):
                a = oracle.sweep_pencil(g[::-1], -xi, order=order, bc=bc)
                b = oracle.sweep_pencil(g, xi, order=order, bc=bc)[::-1]
                assert np.array_equal(a, b)


def test_periodic_sweep_conserves_mass(oracle):
    rng = np.random.default_rng(8)
    f = W.random_field((300, 48), seed=2)
    m0 = f.sum()
    for xi in rng.uniform(-3.0, 3.0, size=10):
        for order in (5, 7):
            oracle.sweep_lines(f, 1, float(xi), order=order)
    assert abs(f.sum() - m0) <= 1e-13 * m0


# ---------------------------------------------------------------------------
# the half-integer tie of the departure split (reading R1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order", [5, 7])
def test_half_integer_tie_is_the_limit_from_above(oracle, order):
    """N = floor(xi + 1/2) jumps at xi = k + 1/2: below the tie the pencil
    is shifted by k and moved by zeta -> +1/2 with the flux of each face
    taken from its left (upwind) cell, above it shifted by k + 1 and moved
    back by zeta -> -1/2 with the mirrored construction.  Without limiters
    both sides give the same cell values (each new cell is the average over
    half of two old cells, and at zeta = 1/2 the odd-width primitive
    stencils are centred on those cells either way), so the unlimited sweep
    is continuous there.  The MP constraint and the PP limiter act on the
    upwind cell of each face, which differs between the two sides: that is
    the scheme's one discontinuity in xi.  Ties go up (zeta = -1/2), so the
    sweep at an exact tie equals the limit from above (within O(eps) of the
    sweep at xi + eps, every limiter being continuous in zeta) and, with a
    limiter, differs by O(1) from the sweep at xi - eps on random data."""
    g = W.random_field(40, seed=31)
    scale = np.abs(g).max()
    eps = 2.0 ** -36
    for lim in (W.LIM_NONE, W.LIM_MP, W.LIM_MPP):
        for bc in (W.BC_PERIODIC, W.BC_OUTFLOW):
            for k in (-4, -2, -1, 0, 1, 3):
                xi = k + 0.5
                kw = dict(order=order, limiter=lim, bc=bc)
                tie = oracle.sweep_pencil(g, xi, **kw)
                above = oracle.sweep_pencil(g, xi + eps, **kw)
                below = oracle.sweep_pencil(g, xi - eps, **kw)
                assert np.abs(tie - above).max() <= 1e-9 * scale, (lim, bc, k)
                if lim == W.LIM_NONE:
                    assert np.abs(tie - below).max() <= 1e-9 * scale, (lim, bc, k)
                else:
                    assert np.abs(tie - below).max() >= 1e-3 * scale, (lim, bc, k)


@pytest.mark.parametrize("order,degree", [(5, 4), (7, 6)])
def test_half_integer_tie_transports_polynomials_exactly(oracle, order, degree):
    """At xi = k + 1/2 (shift k + 1, mirrored flux with zeta = 1/2) the
    unlimited sweep moves cell averages of a polynomial of degree <=
    order - 1 exactly: each interior cell gets the average of the
    polynomial over the cell moved back by k + 1/2 cells (CSL identity of
    Sec. 2.1.2)."""
    n = 48
    rng = np.random.default_rng(77 + order)
    coef = rng.normal(size=degree + 1) / float(n) ** np.arange(degree + 1)
    j = np.arange(n)
    g = _poly_cell_averages(coef, j)
    for k in (-3, -1, 0, 2):
        xi = k + 0.5
        out = oracle.sweep_pencil(g, xi, order=order, limiter=W.LIM_NONE, bc=W.BC_OUTFLOW)
        want = _poly_cell_averages(coef, j - xi)
        # cells whose stencil after the shift stays inside the pencil
        m = 6 + abs(k)
        inside = slice(m, n - m)
        assert np.abs(out[inside] - want[inside]).max() <= 1e-12 * np.abs(want).max(), k


# ---------------------------------------------------------------------------
# accuracy of Test-1 (Sec. 3.1)
# ---------------------------------------------------------------------------
def _advect_error(oracle, profile, order, lim, N, t=1.0, nu=0.2):
    x = W.centers(0.0, 1.0, N)
    f = W.test1_profile(profile, x)
    g = f.copy()
    lo, hi = 1.0, 0.0
    for _ in range(int(round(t / (nu / N)))):
        g = oracle.sweep_pencil(g, nu, order=order, limiter=lim)
        lo, hi = min(lo, g.min()), max(hi, g.max())
    return np.abs(g - f).sum() / np.abs(f).sum(), lo, hi


def _slope(errs, Ns):
    return -np.polyfit(np.log(Ns), np.log(errs), 1)[0]


@pytest.mark.parametrize("order", [5, 7])
def test_design_order_on_sinusoid_without_pp(oracle, order):
    """Test-1b, SL-MP5 / SL-MP7: fifth / seventh order."""
    Ns = [16, 32, 64] if order == 7 else [32, 64, 128]
    errs = [_advect_error(oracle, "sin", order, W.LIM_MP, N)[0] for N in Ns]
    want = GOLD["order_sine_no_pp"]["value"][str(order)]
    assert _slope(errs, Ns) == pytest.approx(want, abs=0.15)


@pytest.mark.parametrize("order", [5, 7])
def test_order_and_positivity_on_quartic_sine(oracle, order):
    """Test-1c with SL-MPP: f stays >= 0 and the order approaches five."""
    Ns = [128, 256]
    res = [_advect_error(oracle, "sin4", order, W.LIM_MPP, N) for N in Ns]
    assert min(r[1] for r in res) >= 0.0
    slope = _slope([r[0] for r in res], Ns)
    assert slope > GOLD["order_quartic_sine"]["value"] - 0.5


def test_rectangle_first_order_no_overshoot(oracle):
    """Test-1a: bounded by [0, 1] throughout, error ~ first order."""
    Ns = [32, 64, 128]
    res = [_advect_error(oracle, "rect", 7, W.LIM_MPP, N) for N in Ns]
    assert all(r[1] >= 0.0 and r[2] <= 1.0 for r in res)
    assert 0.6 < _slope([r[0] for r in res], Ns) < 1.2


def test_pp_as_printed_is_active_at_quadratic_minimum(oracle):
    """Reading of the PP limiter (2 nu split, Sec. 2.1.1).  At the quadratic
    minimum of 1 + sin(2 pi x) even the exact outflow exceeds half the
    upwind cell, so the printed limiter engages and the observed order drops
    below the design order; the limited run is never less accurate than
    first order and stays positive."""
    Ns = [32, 64, 128]
    mp = [_advect_error(oracle, "sin", 5, W.LIM_MP, N)[0] for N in Ns]
    mpp = [_advect_error(oracle, "sin", 5, W.LIM_MPP, N) for N in Ns]
    assert all(b[0] > a for a, b in zip(mp, mpp))
    assert 2.0 < _slope([r[0] for r in mpp], Ns) < 3.5
    assert min(r[1] for r in mpp) >= 0.0


@pytest.mark.parametrize("order", [5, 7])
def test_two_dimensional_split_order(oracle, order):
    """Test-1d: the split 2D sinusoid keeps the 1D order; velocities (1, 0.5)."""
    Ns = [16, 32] if order == 7 else [32, 64]
    errs = []
    for N in Ns:
        x = W.centers(0.0, 1.0, N)
        X, Y = np.meshgrid(x, x, indexing="ij")
        f0 = 1.0 + 0.5 * np.sin(2 * np.pi * X) + 0.5 * np.sin(2 * np.pi * Y)
        f = f0.copy()
        nu = 0.2
        for _ in range(int(round(1.0 / (nu / N)))):
            oracle.sweep_lines(f, 1, 0.5 * nu, order=order, limiter=W.LIM_MP)
            oracle.sweep_lines(f, 0, nu, order=order, limiter=W.LIM_MP)
        # after t = 1: x moved by 1 (identity), y by 0.5 (half a period)
        ref = 1.0 + 0.5 * np.sin(2 * np.pi * X) + 0.5 * np.sin(2 * np.pi * (Y - 0.5))
        errs.append(np.abs(f - ref).sum() / np.abs(ref).sum())
    assert _slope(errs, Ns) == pytest.approx(GOLD["order_2d_sine"]["value"][str(order)], abs=0.35)


# ---------------------------------------------------------------------------
# Poisson solver (Sec. 2.2, App. C)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [2, 4, 6])
def test_laplacian_symbol_matches_stencil(oracle, p):
    """The symbol equals the discrete Laplacian stencils of App. C applied to
    exp(i k x) (with Delta = 1)."""
    stencils = {
        2: ([1, -2, 1], 1.0),
        4: ([-1, 16, -30, 16, -1], 12.0),
        6: ([2, -27, 270, -490, 270, -27, 2], 180.0),
    }
    w, den = stencils[p]
    half = len(w) // 2
    for th in np.linspace(0.01, np.pi, 17):
        sym = sum(c * np.exp(1j * th * (k - half)) for k, c in enumerate(w)) / den
        assert abs(sym.imag) < 1e-12
        assert oracle.laplacian_symbol(th, p) == pytest.approx(sym.real, rel=1e-12, abs=1e-13)


def test_poisson_orders_app_c(oracle):
    """App. C test: rho = rho_bar (1 + A sin kx) with 16 waves; potential and
    force converge with orders 2, 4, 6."""
    L, A, G = 1.0, GOLD["poisson_test"]["A"], 1.0
    k = 2 * np.pi * GOLD["poisson_test"]["waves"] / L
    for p in GOLD["poisson_orders"]["value"]:
        ep, ef = [], []
        Ns = [128, 256, 512]
        for N in Ns:
            s = W.spec(1, N, 4, 0.0, L, -1.0, 1.0, kappa=4 * np.pi * G, poisson_order=p)
            g = oracle.make_grid(s)
            x = W.centers(0.0, L, N)
            phi, acc = oracle.poisson_solve(g, 1.0 + A * np.sin(k * x))
            ep.append(np.mean(np.abs(phi + 4 * np.pi * G * A / k ** 2 * np.sin(k * x))))
            ef.append(np.mean(np.abs(acc - 4 * np.pi * G * A / k * np.cos(k * x))))
        assert _slope(ep, Ns) == pytest.approx(p, abs=0.15)
        assert _slope(ef, Ns) == pytest.approx(p, abs=0.2)


def test_poisson_3d_plane_wave_and_zero_mode(oracle):
    """A plane wave along x2 in a 3D box: only that axis' force is nonzero,
    and a uniform density gives no force (k = 0 removed)."""
    n = 8
    s = W.spec(3, n, 2, 0.0, 2 * np.pi, -1.0, 1.0, kappa=4 * np.pi, poisson_order=6)
    g = oracle.make_grid(s)
    x = W.centers(0.0, 2 * np.pi, n)
    X1, X2, X3 = np.meshgrid(x, x, x, indexing="ij")
    rho = 3.0 + np.cos(X2)
    phi, acc = oracle.poisson_solve(g, rho.ravel())
    acc = acc.reshape(3, n, n, n)
    assert np.abs(acc[0]).max() < 1e-12 and np.abs(acc[2]).max() < 1e-12
    # sixth-order solution of lap(phi) = 4 pi cos(x2): phi ~ -4 pi cos(x2)
    assert np.abs(phi.reshape(n, n, n) + 4 * np.pi * np.cos(X2)).max() < 5e-3
    phi0, acc0 = oracle.poisson_solve(g, np.full(n ** 3, 2.5))
    assert np.abs(acc0).max() < 1e-12


# ---------------------------------------------------------------------------
# Vlasov-Poisson runs (Sec. 3.2, 3.3)
# ---------------------------------------------------------------------------
def _Z(z):
    from scipy.special import wofz
    return 1j * np.sqrt(np.pi) * wofz(z)


def _root(F, guess):
    from scipy.optimize import fsolve

    def g(p):
        r = F(p[0] + 1j * p[1])
        return [r.real, r.imag]

    s = fsolve(g, guess, xtol=1e-13)
    return s[0] + 1j * s[1]


def _mode_history(oracle, spec, T, mode=1):
    run = oracle.Run(spec)
    dt, nx = spec["dt"], spec["nx"][0]
    n = int(round(T / dt))
    ts, amp = [], []
    for k in range(n + 1):
        ts.append(k * dt)
        amp.append(abs(np.fft.fft(run.accel[:nx])[mode]))
        if k < n:
            run.step(dt)
    return np.array(ts), np.array(amp), run


def test_linear_landau_damping_rate(oracle):
    """Test-3: gamma = 0.153 (printed); the root of 1 + k^-2 (1 + z Z(z)) = 0
    at k = 0.5 is 1.41566 - 0.15336i.  Peaks of |E_1| over 5 < t < 40."""
    k = 0.5
    w = _root(lambda w: 1 + (1 + (w / (k * np.sqrt(2))) * _Z(w / (k * np.sqrt(2)))) / k ** 2,
              [1.4, -0.15])
    assert -w.imag == pytest.approx(GOLD["landau_gamma"]["value"], abs=0.001)
    s = W.landau_1d1v(nx=64, nv=128)
    ts, a, _ = _mode_history(oracle, s, 40.0)
    pk = [i for i in range(1, len(a) - 1) if a[i] > a[i - 1] and a[i] >= a[i + 1]]
    tp, ap = ts[pk], np.log(a[pk])
    sel = (tp > 5) & (tp < 40)
    gamma = -np.polyfit(tp[sel], ap[sel], 1)[0]
    assert gamma == pytest.approx(-w.imag, rel=0.03)
    omega = np.pi / np.diff(tp[sel]).mean()
    assert omega == pytest.approx(w.real, rel=0.03)


def test_recurrence_time_formula():
    """t_R = 2 pi / (k dv) = 67 for N_v = 64 on [-6, 6] (Sec. 3.3)."""
    g = GOLD["landau_recurrence"]
    dv = (g["v_range"][1] - g["v_range"][0]) / g["nv"]
    assert 2 * np.pi / (g["k"] * dv) == pytest.approx(g["value"], abs=0.5)


def test_two_stream_growth_rate(oracle):
    """f0 ~ v^2 exp(-v^2/2): growth from the root of the dispersion relation
    (purely growing, 0.2593 at k = 0.5)."""
    k = 0.5

    def eps(w):
        # eps = 1 - k^-2 int f0'(v) / (v - u) dv,  u = w/k,  f0 = v^2 M(v)
        # f0' = 2 v M - v^3 M;  J_n = int v^n M / (v - u) dv
        #     = u^n J_0 + sum_j u^(n-1-j) m_j,  J_0 = Z(u/sqrt2)/sqrt2,
        # m_j the moments of M (1, 0, 1, 0).
        u = w / k
        J0 = _Z(u / np.sqrt(2)) / np.sqrt(2)
        m = [1.0, 0.0, 1.0, 0.0]

        def J(n):
            return u ** n * J0 + sum(u ** (n - 1 - j) * m[j] for j in range(n))

        return 1 - (2 * J(1) - J(3)) / k ** 2

    w = _root(eps, [0.0, 0.26])
    assert abs(w.real) < 1e-8 and w.imag == pytest.approx(0.2593, abs=1e-3)
    s = W.twostream_1d1v(nx=64, nv=128, order=5, cfl=0.5, amp=1e-4)
    ts, a, _ = _mode_history(oracle, s, 22.0)
    sel = (ts > 6) & (ts < 22)
    rate = np.polyfit(ts[sel], np.log(a[sel]), 1)[0]
    assert rate == pytest.approx(w.imag, rel=0.05)


@pytest.mark.parametrize("ratio", [0.5, 1.1])
def test_jeans_rate(oracle, ratio):
    """Test-2 physics in 1D: growth (k/k_J = 0.5) or damping (1.1) of the
    density wave, from 1 - (k_J/k)^2 (1 + z Z(z)) = 0."""
    k = 2 * np.pi
    w = _root(lambda w: 1 - (1 + (w / (k * np.sqrt(2))) * _Z(w / (k * np.sqrt(2)))) / ratio ** 2,
              [0.0, 1.37 * k] if ratio < 1 else [0.0, -0.15 * k])
    s = W.jeans_3d3v(n=64, k_over_kj=ratio, D=1, nv=128)
    s["v_lo"][0], s["v_hi"][0] = -6.0, 6.0
    s["dt"] = 0.5 * (1.0 / 64) / 6.0
    if ratio < 1:
        assert w.imag / k == pytest.approx(1.3744, abs=1e-3)
        ts, a, _ = _mode_history(oracle, s, 0.45)
        sel = (ts > 0.1) & (ts < 0.4)
        rate = np.polyfit(ts[sel], np.log(a[sel]), 1)[0]
        assert rate == pytest.approx(w.imag, rel=0.02)
    else:
        assert abs(w.real) < 1e-8 and w.imag / k == pytest.approx(-0.14825, abs=1e-4)
        ts, a, _ = _mode_history(oracle, s, 1.6)
        sel = (ts > 0.4) & (ts < 1.6)
        rate = np.polyfit(ts[sel], np.log(a[sel]), 1)[0]
        assert rate == pytest.approx(w.imag, rel=0.1)


def test_mass_conserved_with_periodic_velocity(oracle):
    """All sweeps conserve sum(f) on periodic axes (flux form, Eq. (SL))."""
    s = W.landau_1d1v(nx=32, nv=64, amp=0.3)
    s["v_bc"] = W.BC_PERIODIC
    run = oracle.Run(s)
    m0 = oracle.mass(run.grid, run.f)
    run.step(s["dt"] * 3.0, 100)  # x-CFL 1.5 exercises the shift path
    assert abs(oracle.mass(run.grid, run.f) - m0) <= 1e-14 * 100 * abs(m0)


def test_mass_is_the_phase_space_integral(oracle):
    """oracle_mass = dx^D dv^D sum f, pinned by its absolute value.  f is a
    product over axes of (1 + 0.3 cos(2 pi x_l / L_l)) and a unit Gaussian
    centred inside [v_lo, v_hi] at least ten thermal speeds from either end,
    sampled at cell centres with dv = 1/2.  Its phase-space integral is
    prod_l L_l: the midpoint sum of the cosine over a whole period vanishes
    (discrete orthogonality) and that of the Gaussian equals one to far below
    rounding (the Poisson-summation error exp(-2 pi^2 / dv^2) ~ 1e-34, the
    tails beyond ten speeds ~ 1e-23).  Unequal axes in 1D, 2D and 3D catch a
    wrong or swapped volume factor."""
    cases = [
        (1, [32], [48], [4 * math.pi], [(-12.0, 12.0)], [0.0]),
        (2, [12, 10], [44, 48], [2 * math.pi, 3.0], [(-10.0, 12.0), (-13.0, 11.0)], [1.0, -1.0]),
        (3, [6, 5, 4], [40, 42, 44], [1.0, 2.5, 4.0], [(-10.0, 10.0), (-11.0, 10.0), (-10.0, 12.0)],
         [0.0, -0.5, 1.0]),
    ]
    for D, nx, nv, L, vr, u in cases:
        s = W.spec(D, nx, nv, [0.0] * D, L, [a for a, _ in vr], [b for _, b in vr])
        g = oracle.make_grid(s)
        f = np.ones(())
        for l in range(D):
            x = W.centers(0.0, L[l], nx[l])
            f = np.multiply.outer(f, 1.0 + 0.3 * np.cos(2 * math.pi * x / L[l]))
        for l in range(D):
            v = W.centers(vr[l][0], vr[l][1], nv[l])
            f = np.multiply.outer(f, np.exp(-0.5 * (v - u[l]) ** 2) / math.sqrt(2 * math.pi))
        f = np.ascontiguousarray(f)
        assert f.shape == g.shape
        want = float(np.prod(L))
        assert oracle.mass(g, f) == pytest.approx(want, rel=1e-13), D


def test_separability_2d2v_equals_1d1v(oracle):
    """An x1-only perturbation of a 2D2V Maxwellian evolves as the 1D1V run
    times the untouched v2 factor (to round-off).  The 1D run starts from
    f * Z2 with Z2 = dv sum g(v2), so that both runs see the same density."""
    s1 = W.landau_1d1v(nx=16, nv=32, amp=0.2)
    s2 = W.landau_3d3v(n=16, nv=32, D=2, order=5, amp=0.2)
    s2["nx"][1] = 8
    s2["ic"] = "landau"
    g2 = W.maxwellian(W.centers(-6.0, 6.0, 32))
    z2 = (12.0 / 32) * g2.sum()
    f1 = oracle.init_separable(oracle.make_grid(s1), *W.separable_factors(s1)) * z2
    r1, r2 = oracle.Run(s1, f1), oracle.Run(s2)
    r1.step(s1["dt"], 20)
    r2.step(s1["dt"], 20)
    want = (r1.f / z2)[:, None, :, None] * g2[None, None, None, :]
    assert np.abs(r2.f - want).max() <= 1e-12 * np.abs(want).max()


# ---------------------------------------------------------------------------
# RK-MP(P)5/7: method of lines with the three-stage TVD-RK (Sec. 2.1.1)
# ---------------------------------------------------------------------------
def _cell_avg_monomial(k, a, b):
    return (b ** (k + 1) - a ** (k + 1)) / ((k + 1) * (b - a))


@pytest.mark.parametrize("order", [5, 7])
def test_rk_interpolation_exact_for_polynomials(oracle, order):
    """f^int_{i-1/2} from cell averages reproduces the point value at the
    interface for polynomials of degree <= order - 1, and not beyond."""
    lo = -3 if order == 5 else -4
    cells = [(lo + j, lo + j + 1) for j in range(order)]  # interface at x = 0
    for k in range(order + 1):
        s = [_cell_avg_monomial(k, a, b) for a, b in cells]
        got = oracle.rk_interp(s, order)
        want = 1.0 if k == 0 else 0.0
        if k < order:
            assert got == pytest.approx(want, abs=1e-12), k
        else:
            assert abs(got - want) > 1e-4, k


@pytest.mark.parametrize("order", [5, 7])
def test_rk_interpolation_is_the_csl_flux_at_zero_courant(oracle, order):
    """The RK interface value (Sec. 2.1.1) and the CSL flux polynomial
    (Sec. 2.1.2) at zeta = 0 are the same interpolation."""
    rng = np.random.default_rng(11)
    for _ in range(50):
        s = rng.normal(size=order)
        assert oracle.rk_interp(s, order) == pytest.approx(oracle.csl_flux(s, order, 0.0),
                                                           rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("order", [5, 7])
def test_rk_step_is_third_order_taylor_on_a_fourier_mode(oracle, order):
    """Without limiters the scheme is linear: a Fourier mode is multiplied by
    1 + a + a^2/2 + a^3/6 with a = -nu * lambda(theta), the TVD-RK property
    for linear operators, where lambda is the symbol of L built from the
    oracle's own interpolation."""
    n, mode, nu = 32, 3, 0.3
    th = 2 * np.pi * mode / n
    off = np.arange(order) - (3 if order == 5 else 4)
    # symbol of f^int_{i-1/2} relative to cell i: sum_k c_k e^{i th off_k}
    s_re = oracle.rk_interp(np.cos(th * off), order)
    s_im = oracle.rk_interp(np.sin(th * off), order)
    interp = s_re + 1j * s_im
    lam = (np.exp(1j * th) - 1.0) * interp  # fint_{i+1/2} - fint_{i-1/2}
    a = -nu * lam
    G = 1 + a + a * a / 2 + a ** 3 / 6
    j = np.arange(n)
    for phase in (0.0, 0.7):
        g = np.cos(th * j + phase)
        got = oracle.rk_pencil(g, nu, order, oracle.LIM_NONE)
        want = np.real(G * np.exp(1j * (th * j + phase)))
        assert np.abs(got - want).max() <= 1e-13


def test_rk_mp5_is_fifth_order_at_small_courant(oracle):
    """Test-1b without PP: RK-MP5 converges at fifth order (nu = 0.05, where
    the third-order time error of TVD-RK stays below the spatial error)."""
    xg, wg = np.polynomial.legendre.leggauss(8)
    errs = []
    for N in (16, 32, 64, 128):
        h = 1.0 / N
        c = (np.arange(N) + 0.5) * h
        g0 = sum(w * (1 + np.sin(2 * np.pi * (c + 0.5 * h * x))) for x, w in zip(xg, wg)) / 2
        g = g0.copy()
        for _ in range(int(round(N / 0.05))):
            g = oracle.rk_pencil(g, 0.05, 5, oracle.LIM_MP)
        errs.append(np.abs(g - g0).sum() / np.abs(g0).sum())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (orders > 4.7).all(), orders


def test_rk_quartic_sine_positivity(oracle):
    """Test-1c at N = 64 to t = 8: RK-MP5 goes negative near the minima,
    RK-MPP5 does not (Sec. 3.1.3)."""
    N, nu = 64, 0.4
    x = (np.arange(N) + 0.5) / N
    g0 = np.sin(4 * np.pi * x) ** 4
    a, b = g0.copy(), g0.copy()
    for _ in range(int(round(8 * N / nu))):
        a = oracle.rk_pencil(a, nu, 5, oracle.LIM_MP)
        b = oracle.rk_pencil(b, nu, 5, oracle.LIM_MPP)
    assert a.min() < -1e-2
    assert b.min() >= 0.0


def test_rk_mpp_positivity_random_pencils(oracle):
    """RK-MPP keeps f >= 0 for nu < 1/2 (Sec. 2.1.1), on random pencils with
    zeros and spikes, both orders, both boundary conditions, both signs."""
    rng = np.random.default_rng(5)
    for t in range(400):
        g = W.random_field(40, 100 + t)
        nu = rng.uniform(-0.49, 0.49)
        order = 5 if t % 2 else 7
        bc = oracle.BC_PERIODIC if t % 3 else oracle.BC_OUTFLOW
        out = oracle.rk_pencil(g, nu, order, oracle.LIM_MPP, bc=bc)
        assert out.min() >= -1e-14 * g.max(), (t, out.min())


def test_rk_conservation_symmetry_and_limits(oracle):
    rng = np.random.default_rng(8)
    g = W.random_field(48, 9)
    for order in (5, 7):
        for lim in (oracle.LIM_NONE, oracle.LIM_MP, oracle.LIM_MPP):
            out = oracle.rk_pencil(g, 0.37, order, lim)
            assert out.sum() == pytest.approx(g.sum(), rel=1e-14)
            # reflection: a negative speed is the mirrored positive one
            m = oracle.rk_pencil(g[::-1].copy(), -0.37, order, lim)[::-1]
            assert np.array_equal(m, out)
    c = np.full(20, 0.625)
    assert np.array_equal(oracle.rk_pencil(c, 0.3, 7, oracle.LIM_MPP), c)
    with pytest.raises(ValueError):
        oracle.rk_pencil(g, 1.5)


# ---------------------------------------------------------------------------
# velocity-space diagnostics (Sec. 2.3 moments, Sec. 3.3 F(v))
# ---------------------------------------------------------------------------
def test_velocity_moments_of_shifted_maxwellians(oracle):
    """A shifted, scaled Maxwellian per spatial cell has density n0, mean
    u0 and dispersion s0^2; on a wide velocity grid the midpoint sums match
    these to near rounding (the integrand is smooth and decays)."""
    spec = W.spec(2, [3, 2], [120, 96], [0.0, 0.0], [1.0, 1.0], [-12.0, -10.0], [12.0, 10.0])
    g = oracle.make_grid(spec)
    rng = np.random.default_rng(2)
    n0 = rng.uniform(0.5, 2.0, size=6)
    u0 = rng.uniform(-1.0, 1.0, size=(2, 6))
    s0 = rng.uniform(0.7, 1.3, size=(2, 6))
    v1 = W.centers(-12.0, 12.0, 120)
    v2 = W.centers(-10.0, 10.0, 96)
    f = np.empty(g.shape)
    for ix in range(6):
        i, j = divmod(ix, 2)
        a = np.exp(-(v1 - u0[0, ix]) ** 2 / (2 * s0[0, ix] ** 2)) / (np.sqrt(2 * np.pi) * s0[0, ix])
        b = np.exp(-(v2 - u0[1, ix]) ** 2 / (2 * s0[1, ix] ** 2)) / (np.sqrt(2 * np.pi) * s0[1, ix])
        f[i, j] = n0[ix] * np.outer(a, b)
    rho, mean, disp = oracle.velocity_moments(g, f)
    assert rho == pytest.approx(n0, rel=1e-12)
    assert mean.reshape(2, 6) == pytest.approx(u0, abs=1e-11)
    assert disp.reshape(2, 6) == pytest.approx(s0 ** 2, rel=1e-11)


def test_velocity_distribution_and_energy_identity(oracle):
    """F(v) of a separable f = s(x) g(v) is (dx^D sum s) g(v); and the
    kinetic energy from the moments, sum_x dx^D rho (|u|^2 + sum sigma^2)/2,
    equals 1/2 sum f |v|^2 dx^D dv^D taken directly."""
    spec = W.landau_3d3v(n=4, nv=6, order=5, D=2, amp=0.3)
    g = oracle.make_grid(spec)
    s, gv = W.separable_factors(spec)
    f = oracle.init_separable(g, s, gv)
    F = oracle.velocity_distribution(g, f)
    dx = np.prod([(spec["x_hi"][l] - spec["x_lo"][l]) / spec["nx"][l] for l in range(2)])
    dv = np.prod([(spec["v_hi"][l] - spec["v_lo"][l]) / spec["nv"][l] for l in range(2)])
    assert F == pytest.approx(dx * s.sum() * np.outer(gv[0], gv[1]).ravel(), rel=1e-13)
    rng = np.random.default_rng(4)
    fr = W.random_field(g.shape, 12)
    rho, mean, disp = oracle.velocity_moments(g, fr)
    nxs = g.n_space
    k_mom = 0.5 * dx * sum(rho[ix] * sum(mean[l * nxs + ix] ** 2 + disp[l * nxs + ix]
                                         for l in range(2)) for ix in range(nxs))
    v1 = W.centers(spec["v_lo"][0], spec["v_hi"][0], spec["nv"][0])
    v2 = W.centers(spec["v_lo"][1], spec["v_hi"][1], spec["nv"][1])
    vv = v1[:, None] ** 2 + v2[None, :] ** 2
    k_dir = 0.5 * dx * dv * float((fr * vv[None, None]).sum())
    assert k_mom == pytest.approx(k_dir, rel=1e-12)


# ---------------------------------------------------------------------------
# merged velocity half-steps across consecutive steps
# ---------------------------------------------------------------------------
def test_merged_kicks_single_step_and_free_streaming(oracle):
    """One step merges nothing (bitwise equal); with no field the velocity
    sweeps are the identity and merging changes nothing either."""
    s = W.landau_1d1v(nx=32, nv=64, amp=0.2)
    a = oracle.Run(s)
    a.step(s["dt"], 1)
    m = dict(s, merge_kicks=True)
    b = oracle.Run(m)
    b.step(s["dt"], 1)
    assert np.array_equal(a.f, b.f)
    free = W.advection_1d1v(32, 16, -2.0, 2.0, "sin4")
    free["dt"] = 0.01
    c = oracle.Run(free)
    c.step(free["dt"], 7)
    d = oracle.Run(dict(free, merge_kicks=True))
    d.step(free["dt"], 7)
    assert np.array_equal(c.f, d.f)


def test_merged_kicks_keep_the_landau_rate(oracle):
    """Test-3 with merged half-steps: the damping rate and frequency still
    match the dispersion-relation root (the splitting stays second order)."""
    s = dict(W.landau_1d1v(nx=64, nv=128), merge_kicks=True)
    run = oracle.Run(s)
    dt, nx, chunk = s["dt"], 64, 5
    n = int(round(40.0 / dt)) // chunk
    # advanced in calls of 5 merged steps; |E_1| is read after each call
    ts, amp = [0.0], [abs(np.fft.fft(run.accel[:nx])[1])]
    for k in range(n):
        run.step(dt, chunk)
        ts.append((k + 1) * chunk * dt)
        amp.append(abs(np.fft.fft(run.accel[:nx])[1]))
    ts, amp = np.array(ts), np.array(amp)
    pk = [i for i in range(1, len(amp) - 1) if amp[i] > amp[i - 1] and amp[i] >= amp[i + 1]]
    tp, ap = ts[pk], np.log(amp[pk])
    sel = (tp > 5) & (tp < 40)
    gamma = -np.polyfit(tp[sel], ap[sel], 1)[0]
    assert gamma == pytest.approx(0.15336, rel=0.03)


# ---------------------------------------------------------------------------
# isolated boundaries: doubling-up method (Sec. 2.2)
# ---------------------------------------------------------------------------
def test_box_inverse_r_matches_quadrature(oracle):
    from scipy import integrate

    for a, b, c in ((0.5, 0.5, 0.5), (0.3, 0.7, 0.5), (0.1, 0.2, 0.9)):
        q, _ = integrate.tplquad(lambda z, y, x: 1.0 / np.sqrt(x * x + y * y + z * z),
                                 0, a, 0, b, 0, c, epsabs=1e-12, epsrel=1e-12)
        assert oracle.box_inverse_r(a, b, c) == pytest.approx(8 * q, rel=1e-10)


def _iso_grid(oracle, n=(8, 6, 10), order=6):
    spec = W.spec(3, list(n), [2, 2, 2], [-1.0, -0.6, -1.5], [1.0, 0.9, 1.0], [-1, -1, -1],
                  [1, 1, 1], kappa=4 * np.pi, poisson_order=order, field_bc="isolated")
    return spec, oracle.make_grid(spec)


def test_isolated_point_mass_is_newtonian(oracle):
    """A unit mass in one cell (G = 1): the doubled-grid convolution is the
    direct sum, so phi = -1/r exactly at every other cell (no periodic
    images), and the cell-mean Green function at the mass itself."""
    spec, g = _iso_grid(oracle)
    n = np.array(spec["nx"][:3])
    h = (np.array(spec["x_hi"][:3]) - np.array(spec["x_lo"][:3])) / n
    src = (1, 4, 8)  # near the edges: images would show
    rho = np.zeros(int(n.prod()))
    rho[np.ravel_multi_index(src, n)] = 1.0 / h.prod()
    phi, acc = oracle.poisson_isolated(g, rho)
    idx = np.indices(n).reshape(3, -1).T
    d = (idx - np.array(src)) * h
    r = np.sqrt((d * d).sum(1))
    self_ = r == 0
    assert np.abs(phi[~self_] + 1.0 / r[~self_]).max() <= 1e-13 * (1.0 / r[~self_]).max()
    want_self = -oracle.box_inverse_r(*(0.5 * h)) / h.prod()
    assert phi[self_][0] == pytest.approx(want_self, rel=1e-13)
    # the force points to the mass and falls off as 1/r^2 (sixth-order FDA,
    # away from the mass so that no stencil reaches its cell)
    spec, g = _iso_grid(oracle, n=(16, 16, 16))
    n = np.array(spec["nx"][:3])
    h = (np.array(spec["x_hi"][:3]) - np.array(spec["x_lo"][:3])) / n
    src = (7, 8, 6)
    rho = np.zeros(int(n.prod()))
    rho[np.ravel_multi_index(src, n)] = 1.0 / h.prod()
    _, acc = oracle.poisson_isolated(g, rho)
    idx = np.indices(n).reshape(3, -1).T
    d = (idx - np.array(src)) * h
    r = np.sqrt((d * d).sum(1))
    a = acc.reshape(3, -1).T
    far = r >= 6 * h.max()
    want = -d[far] / r[far, None] ** 3
    err = np.abs(a[far] - want).max(axis=1) / (1.0 / r[far] ** 2)
    assert err.max() < 1e-2


def test_isolated_solve_is_linear_and_sign_follows_kappa(oracle):
    spec, g = _iso_grid(oracle, n=(6, 6, 6), order=4)
    rng = np.random.default_rng(3)
    r1, r2 = rng.random(216), rng.random(216)
    p1, a1 = oracle.poisson_isolated(g, r1)
    p2, a2 = oracle.poisson_isolated(g, r2)
    p12, a12 = oracle.poisson_isolated(g, 2.0 * r1 + r2)
    assert np.abs(p12 - (2 * p1 + p2)).max() <= 1e-12 * np.abs(p12).max()
    assert np.abs(a12 - (2 * a1 + a2)).max() <= 1e-12 * np.abs(a12).max()
    assert (p1 < 0).all()  # gravity: every cell sees a potential well
    spec["kappa"] = -1.0
    ge = oracle.make_grid(spec)
    pe, _ = oracle.poisson_isolated(ge, r1)
    assert np.abs(pe + p1 / (4 * np.pi)).max() <= 1e-13 * np.abs(pe).max()
