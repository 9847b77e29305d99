"""FP64 CPU oracle for the SL-MPP5/7 Vlasov sweeps -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding in ``paper_1702_08521_amd``) never imports, loads or calls it.

The arithmetic lives in ``slmpp_oracle.c`` (plain C, double precision, built
with ``-ffp-contract=off`` and no fast-math); this module only marshals numpy
arrays through ctypes.  See the header of ``slmpp_oracle.c`` for the readings
of points the paper leaves open.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slmpp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_PERIODIC = 0
BC_OUTFLOW = 1
LIM_NONE = 0
LIM_MP = 1
LIM_MPP = 2
TIME_SL = 0
TIME_RK3 = 1


_LIB_NATIVE = os.path.join(_HERE, "liboracle_native.so")
_use_native = False


def build(native: bool = False) -> str:
    """Compile the oracle with gcc.  ``native``: -O3 -march=native into a
    library of its own (the arithmetic is unchanged: contraction stays off,
    no fast-math), used only to time the oracle."""
    out = _LIB_NATIVE if native else _LIB
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    cmd = ["gcc", *opt, "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-Wall", _SRC, "-o", out + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def use_native():
    """Switch this process to the -O3 -march=native build (built on first
    use).  Call before the first oracle call."""
    global _use_native, _lib
    if _lib is not None and not _use_native:
        raise RuntimeError("the oracle library is already loaded")
    _use_native = True


class Grid(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("limiter", ctypes.c_int32),
        ("poisson_order", ctypes.c_int32),
        ("nx", ctypes.c_int64 * 3),
        ("nv", ctypes.c_int64 * 3),
        ("x_lo", ctypes.c_double * 3),
        ("x_hi", ctypes.c_double * 3),
        ("v_lo", ctypes.c_double * 3),
        ("v_hi", ctypes.c_double * 3),
        ("alpha", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("x_bc", ctypes.c_int32),
        ("v_bc", ctypes.c_int32),
        ("time_scheme", ctypes.c_int32),
        ("merge_kicks", ctypes.c_int32),
        ("isolated", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]

    @property
    def shape(self):
        return tuple(self.nx[: self.D]) + tuple(self.nv[: self.D])

    @property
    def n_space(self):
        return int(np.prod(self.nx[: self.D]))


def make_grid(spec) -> Grid:
    """Build an oracle Grid from a workload spec (a mapping with keys D, nx,
    nv, x_lo, x_hi, v_lo, v_hi, order, limiter, alpha, kappa, poisson_order,
    x_bc, v_bc)."""
    g = Grid()
    D = int(spec["D"])
    g.D = D
    g.order = int(spec.get("order", 5))
    g.limiter = int(spec.get("limiter", LIM_MPP))
    g.poisson_order = int(spec.get("poisson_order", 6))
    for l in range(3):
        g.nx[l] = int(spec["nx"][l]) if l < D else 1
        g.nv[l] = int(spec["nv"][l]) if l < D else 1
        g.x_lo[l] = float(spec["x_lo"][l]) if l < D else 0.0
        g.x_hi[l] = float(spec["x_hi"][l]) if l < D else 1.0
        g.v_lo[l] = float(spec["v_lo"][l]) if l < D else 0.0
        g.v_hi[l] = float(spec["v_hi"][l]) if l < D else 1.0
    g.alpha = float(spec.get("alpha", 4.0))
    g.kappa = float(spec.get("kappa", -1.0))
    g.x_bc = int(spec.get("x_bc", BC_PERIODIC))
    g.v_bc = int(spec.get("v_bc", BC_OUTFLOW))
    g.time_scheme = TIME_RK3 if spec.get("time", "sl") == "rk3" else TIME_SL
    g.merge_kicks = 1 if spec.get("merge_kicks", False) else 0
    g.isolated = 1 if spec.get("field_bc", "periodic") == "isolated" else 0
    return g


_lib = None
_D = ctypes.c_double
_I = ctypes.c_int
_I64 = ctypes.c_int64
_P = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        path = _LIB_NATIVE if _use_native else _LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build(native=_use_native)
        L = ctypes.CDLL(path)
        sig = {
            "oracle_minmod2": (_D, [_D, _D]),
            "oracle_minmod4": (_D, [_D, _D, _D, _D]),
            "oracle_median3": (_D, [_D, _D, _D]),
            "oracle_mp": (_D, [_D, _D, _D, _D, _D, _D, _D]),
            "oracle_pp": (_D, [_D, _D, _D, _D]),
            "oracle_csl_flux": (_D, [_P, _I, _D]),
            "oracle_laplacian_symbol": (_D, [_D, _I]),
            "oracle_cell_center": (_D, [_D, _D, _I64, _I64]),
            "oracle_xi": (_D, [_D, _D, _D]),
            "oracle_sweep_pencil": (None, [_P, _I64, _I64, _D, _I, _I, _D, _I]),
            "oracle_sweep_lines": (None, [_P, _I64, _I64, _I64, _D, _I, _I, _D, _I]),
            "oracle_rk_pencil": (_I, [_P, _I64, _I64, _D, _I, _I, _D, _I]),
            "oracle_rk_interp": (_D, [_P, _I]),
            "oracle_advect_x": (_I, [ctypes.POINTER(Grid), _P, _I, _D]),
            "oracle_advect_v": (_I, [ctypes.POINTER(Grid), _P, _I, _D, _P]),
            "oracle_density_moment": (None, [ctypes.POINTER(Grid), _P, _P]),
            "oracle_velocity_moments": (None, [ctypes.POINTER(Grid), _P, _P, _P, _P]),
            "oracle_velocity_distribution": (None, [ctypes.POINTER(Grid), _P, _P]),
            "oracle_poisson_solve": (None, [ctypes.POINTER(Grid), _P, _P, _P]),
            "oracle_field": (None, [ctypes.POINTER(Grid), _P, _P]),
            "oracle_poisson_isolated": (None, [ctypes.POINTER(Grid), _P, _P, _P]),
            "oracle_box_inverse_r": (_D, [_D, _D, _D]),
            "oracle_step": (None, [ctypes.POINTER(Grid), _P, _D, _P]),
            "oracle_steps": (None, [ctypes.POINTER(Grid), _P, _D, _I64, _P]),
            "oracle_init_separable": (None, [ctypes.POINTER(Grid), _P, _P, _P, _P, _P]),
            "oracle_mass": (_D, [ctypes.POINTER(Grid), _P]),
            "oracle_abi_version": (_I, []),
            "oracle_set_threads": (None, [_I]),
            "oracle_max_threads": (_I, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_P)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---- scalar pieces --------------------------------------------------------
def minmod2(a, b):
    return lib().oracle_minmod2(a, b)


def minmod4(a, b, c, d):
    return lib().oracle_minmod4(a, b, c, d)


def median3(a, b, c):
    return lib().oracle_median3(a, b, c)


def mp(fint, fm2, fm1, f0, fp1, fp2, alpha=4.0):
    return lib().oracle_mp(fint, fm2, fm1, f0, fp1, fp2, alpha)


def pp(phibar, fl, fr, nu):
    return lib().oracle_pp(phibar, fl, fr, nu)


def csl_flux(stencil, order, zeta):
    s = _f64(stencil)
    assert s.size == order
    return lib().oracle_csl_flux(_ptr(s), order, zeta)


def laplacian_symbol(theta, order):
    return lib().oracle_laplacian_symbol(theta, order)


def cell_center(lo, hi, n, j):
    return lib().oracle_cell_center(lo, hi, n, j)


def xi(c, dt, h):
    return lib().oracle_xi(c, dt, h)


# ---- sweeps ---------------------------------------------------------------
def sweep_pencil(g, xi_, order=5, limiter=LIM_MPP, alpha=4.0, bc=BC_PERIODIC):
    """Return the pencil g after one SL step with departure offset xi_ cells."""
    a = _f64(g).copy()
    lib().oracle_sweep_pencil(_ptr(a), a.size, 1, xi_, order, limiter, alpha, bc)
    return a


def rk_interp(stencil, order):
    """f^int_{i-1/2} of the RK-MP schemes from f_{i-3..i+1} (order 5) or
    f_{i-4..i+2} (order 7)."""
    s = _f64(stencil)
    assert s.size == order
    return lib().oracle_rk_interp(_ptr(s), order)


def rk_pencil(g, nu, order=5, limiter=LIM_MPP, alpha=4.0, bc=BC_PERIODIC):
    """Return the pencil g after one RK-MP(P) step (TVD-RK3, Sec. 2.1.1)
    with CFL number nu = c dt / h (|nu| <= 1)."""
    a = _f64(g).copy()
    if lib().oracle_rk_pencil(_ptr(a), a.size, 1, nu, order, limiter, alpha, bc) != 0:
        raise ValueError("RK time integration needs |nu| <= 1")
    return a


def sweep_lines(f, axis, xi_, order=5, limiter=LIM_MPP, alpha=4.0, bc=BC_PERIODIC):
    """All pencils of the C-contiguous float64 array f along `axis`, in place."""
    assert f.dtype == np.float64 and f.flags.c_contiguous
    outer = int(np.prod(f.shape[:axis]))
    n = f.shape[axis]
    inner = int(np.prod(f.shape[axis + 1:]))
    lib().oracle_sweep_lines(_ptr(f), outer, n, inner, xi_, order, limiter, alpha, bc)
    return f


def advect_x(grid, f, dim, dt):
    if lib().oracle_advect_x(ctypes.byref(grid), _ptr(f), dim, dt) != 0:
        raise ValueError("RK time integration needs |c dt / h| <= 1")
    return f


def advect_v(grid, f, dim, dt, accel_component):
    a = _f64(accel_component)
    if lib().oracle_advect_v(ctypes.byref(grid), _ptr(f), dim, dt, _ptr(a)) != 0:
        raise ValueError("RK time integration needs |c dt / h| <= 1")
    return f


def density_moment(grid, f):
    rho = np.empty(grid.n_space, dtype=np.float64)
    lib().oracle_density_moment(ctypes.byref(grid), _ptr(f), _ptr(rho))
    return rho


def velocity_moments(grid, f):
    """(rho, mean, disp): density, mean velocity and velocity dispersion of
    every spatial cell (mean, disp: D * prod(nx), component-major)."""
    n = grid.n_space
    rho = np.empty(n)
    mean = np.empty(grid.D * n)
    disp = np.empty(grid.D * n)
    lib().oracle_velocity_moments(ctypes.byref(grid), _ptr(f), _ptr(rho), _ptr(mean), _ptr(disp))
    return rho, mean, disp


def velocity_distribution(grid, f):
    """F(v) = dx^D sum_x f, prod(nv) values."""
    nvs = int(np.prod(grid.nv[: grid.D]))
    F = np.empty(nvs)
    lib().oracle_velocity_distribution(ctypes.byref(grid), _ptr(f), _ptr(F))
    return F


def poisson_solve(grid, rho):
    r = _f64(rho)
    phi = np.empty(grid.n_space, dtype=np.float64)
    acc = np.empty(grid.D * grid.n_space, dtype=np.float64)
    lib().oracle_poisson_solve(ctypes.byref(grid), _ptr(r), _ptr(phi), _ptr(acc))
    return phi, acc


def poisson_isolated(grid, rho):
    """(phi, accel) of the isolated-boundary solve (D = 3)."""
    r = _f64(rho)
    phi = np.empty(grid.n_space, dtype=np.float64)
    acc = np.empty(grid.D * grid.n_space, dtype=np.float64)
    lib().oracle_poisson_isolated(ctypes.byref(grid), _ptr(r), _ptr(phi), _ptr(acc))
    return phi, acc


def box_inverse_r(a, b, c):
    """Integral of 1/r over the box [-a, a] x [-b, b] x [-c, c]."""
    return lib().oracle_box_inverse_r(a, b, c)


def field(grid, f):
    acc = np.empty(grid.D * grid.n_space, dtype=np.float64)
    lib().oracle_field(ctypes.byref(grid), _ptr(f), _ptr(acc))
    return acc


def step(grid, f, dt, accel):
    lib().oracle_step(ctypes.byref(grid), _ptr(f), dt, _ptr(accel))
    return f


def init_separable(grid, s, gv):
    f = np.empty(grid.shape, dtype=np.float64)
    s = _f64(s)
    gs = [_f64(x) for x in gv] + [np.zeros(1)] * (3 - len(gv))
    lib().oracle_init_separable(ctypes.byref(grid), _ptr(f), _ptr(s), _ptr(gs[0]),
                                _ptr(gs[1]), _ptr(gs[2]))
    return f


def set_threads(n):
    """Threads of the oracle's loops over pencils (timing only)."""
    lib().oracle_set_threads(int(n))


def max_threads():
    return int(lib().oracle_max_threads())


def mass(grid, f):
    return lib().oracle_mass(ctypes.byref(grid), _ptr(f))


class Run:
    """A Vlasov-Poisson run on the oracle: f, the field, and Strang steps."""

    def __init__(self, spec, f0=None):
        self.grid = make_grid(spec)
        if f0 is None:
            from paper_1702_08521_amd import workloads
            s, gv = workloads.separable_factors(spec)
            f0 = init_separable(self.grid, s, gv)
        self.f = _f64(f0).reshape(self.grid.shape).copy()
        self.accel = field(self.grid, self.f)

    def step(self, dt, nsteps=1):
        lib().oracle_steps(ctypes.byref(self.grid), _ptr(self.f), dt, nsteps, _ptr(self.accel))
        return self.f
