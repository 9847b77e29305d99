"""Thin ctypes binding of libslmpp.so (include/slmpp.h).

Argument marshalling only: every step of the sweeps, moment, Poisson solve
and diagnostics runs in the HIP library.  PyTorch provides device memory
and the stream.  Importing this module loads the library and raises if it
is missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libslmpp.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "slmpp.h")

OK, ERR_INVALID, ERR_SHAPE, ERR_NONFINITE, ERR_WORKSPACE, ERR_DEVICE, ERR_STATE = range(7)
F64, F32 = 0, 1
BC_PERIODIC, BC_OUTFLOW = 0, 1
LIM_NONE, LIM_MP, LIM_MPP = 0, 1, 2
FLAG_RK3 = 1
FLAG_MERGE_KICKS = 2
FLAG_ISOLATED = 4
FLAG_SEPARATE_KICKS = 8
TIMING_CLASSES = 8
TIMING_NAMES = ("sweep_strided_wide", "sweep_contiguous", "moment", "poisson",
                "sweep_strided_other", "pencil_table", "sweep_x1_moment", "kick_plane")


class SlmppError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"slmpp status {status}: {message}")
        self.status = status


class GridDesc(ctypes.Structure):
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
        ("storage", ctypes.c_int32),
        ("flags", ctypes.c_int32),
    ]


class DiagOut(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double),
        ("f_min", ctypes.c_double),
        ("f_max", ctypes.c_double),
        ("field_energy", ctypes.c_double),
        ("mode_amp", ctypes.c_double),
        ("nonfinite", ctypes.c_int64),
    ]


class Timing(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_int64 * TIMING_CLASSES),
        ("total_ms", ctypes.c_double * TIMING_CLASSES),
        ("bytes", ctypes.c_double * TIMING_CLASSES),
        ("cells", ctypes.c_double * TIMING_CLASSES),
    ]


_VP = ctypes.c_void_p
_D = ctypes.c_double
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_S = ctypes.c_int  # slmpp_status

# name -> (restype, argtypes); the C-ABI entry points of include/slmpp.h
SIGNATURES = {
    "slmpp_abi_version": (_I32, []),
    "slmpp_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(GridDesc)]),
    "slmpp_validate": (_S, [ctypes.POINTER(GridDesc), ctypes.c_char_p, ctypes.c_size_t]),
    "slmpp_create": (_S, [ctypes.POINTER(GridDesc), _VP, _VP, ctypes.c_size_t, _VP,
                          ctypes.POINTER(_VP)]),
    "slmpp_destroy": (_S, [_VP]),
    "slmpp_last_error": (ctypes.c_char_p, [_VP]),
    "slmpp_init_f_host": (_S, [_VP, _VP, _I64]),
    "slmpp_init_f_separable": (_S, [_VP, _VP, _VP, _VP, _VP]),
    "slmpp_advect_x": (_S, [_VP, _I32, _D]),
    "slmpp_advect_v": (_S, [_VP, _I32, _D, _VP]),
    "slmpp_advect_v_noalloc": (_S, [_VP, _VP, _I32, _D, _VP, _VP]),
    "slmpp_kick": (_S, [_VP, ctypes.c_double]),
    "slmpp_density_moment": (_S, [_VP, _VP]),
    "slmpp_poisson_solve": (_S, [_VP, _VP, _VP, _VP]),
    "slmpp_velocity_moments": (_S, [_VP, _VP, _VP, _VP]),
    "slmpp_velocity_distribution": (_S, [_VP, _VP]),
    "slmpp_field": (_S, [_VP]),
    "slmpp_field_ptrs": (_S, [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP)]),
    "slmpp_get_field": (_S, [_VP, _VP, _VP]),
    "slmpp_step": (_S, [_VP, _D, _I32]),
    "slmpp_get_f": (_S, [_VP, _VP, _I64]),
    "slmpp_diag": (_S, [_VP, ctypes.POINTER(DiagOut)]),
    "slmpp_sync": (_S, [_VP]),
    "slmpp_timing_enable": (_S, [_VP, _I32]),
    "slmpp_timing_read": (_S, [_VP, ctypes.POINTER(Timing)]),
    "slmpp_copy_device": (_S, [_VP, _VP, ctypes.c_size_t, _VP]),
    "slmpp_alloc_device": (_S, [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(_VP)]),
    "slmpp_free_device": (_S, [_VP]),
    "slmpp_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(GridDesc), _I32]),
    "slmpp_batch_create": (_S, [ctypes.POINTER(GridDesc), ctypes.POINTER(_D), _I32,
                                ctypes.POINTER(_VP), _VP, ctypes.c_size_t, _VP,
                                ctypes.POINTER(_VP)]),
    "slmpp_batch_destroy": (_S, [_VP]),
    "slmpp_batch_last_error": (ctypes.c_char_p, [_VP]),
    "slmpp_batch_init_separable": (_S, [_VP, _I32, _VP, _VP, _VP, _VP]),
    "slmpp_batch_step": (_S, [_VP, _I32]),
    "slmpp_batch_step_eager": (_S, [_VP, _I32]),
    "slmpp_batch_get_f": (_S, [_VP, _I32, _VP, _I64]),
    "slmpp_batch_autotune": (_S, [_VP, ctypes.c_char_p]),
    "slmpp_batch_tile_width": (_I32, [_VP, _I32, _I32]),
    "slmpp_batch_set_fast_min_cells": (_S, [_VP, ctypes.c_int64]),
    "slmpp_batch_step_bytes": (ctypes.c_double, [_VP]),
}

_lib = None


# SLMPP_ABI_VERSION of include/slmpp.h that these signatures follow
ABI_VERSION = 3


def lib():
    """Load libslmpp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        v = L.slmpp_abi_version()
        if v != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI version {v}, this binding expects "
                               f"{ABI_VERSION}: rebuild the library")
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status != OK:
        msg = lib().slmpp_last_error(ctx)
        raise SlmppError(status, msg.decode() if msg else "")


def make_desc(spec, storage=F64) -> GridDesc:
    """GridDesc from a workload spec (see workloads.spec)."""
    d = GridDesc()
    D = int(spec["D"])
    d.D = D
    d.order = int(spec.get("order", 5))
    d.limiter = int(spec.get("limiter", LIM_MPP))
    d.poisson_order = int(spec.get("poisson_order", 6))
    for l in range(3):
        d.nx[l] = int(spec["nx"][l]) if l < D else 1
        d.nv[l] = int(spec["nv"][l]) if l < D else 1
        d.x_lo[l] = float(spec["x_lo"][l]) if l < D else 0.0
        d.x_hi[l] = float(spec["x_hi"][l]) if l < D else 1.0
        d.v_lo[l] = float(spec["v_lo"][l]) if l < D else 0.0
        d.v_hi[l] = float(spec["v_hi"][l]) if l < D else 1.0
    d.alpha = float(spec.get("alpha", 4.0))
    d.kappa = float(spec.get("kappa", -1.0))
    d.x_bc = int(spec.get("x_bc", BC_PERIODIC))
    d.v_bc = int(spec.get("v_bc", BC_OUTFLOW))
    d.storage = int(storage)
    d.flags = (FLAG_RK3 if spec.get("time", "sl") == "rk3" else 0) | \
        (FLAG_MERGE_KICKS if spec.get("merge_kicks", False) else 0) | \
        (FLAG_ISOLATED if spec.get("field_bc", "periodic") == "isolated" else 0) | \
        (FLAG_SEPARATE_KICKS if spec.get("separate_kicks", False) else 0)
    return d


def workspace_bytes(desc: GridDesc) -> int:
    return int(lib().slmpp_workspace_bytes(ctypes.byref(desc)))


def validate(desc: GridDesc):
    buf = ctypes.create_string_buffer(256)
    st = lib().slmpp_validate(ctypes.byref(desc), buf, 256)
    return st, buf.value.decode()


def _host_f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_VP)


class Context:
    """A library context over device memory held by torch tensors.

    f: a CUDA tensor with the grid's cells in the storage dtype (allocated
    here if not given).  The workspace is a uint8 CUDA tensor.  All work is
    enqueued on `stream` (a torch.cuda.Stream; the current stream if None).
    """

    def __init__(self, desc: GridDesc, f=None, stream=None, device=None):
        import torch

        self.desc = desc
        self.torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        D = desc.D
        self.shape = tuple(desc.nx[:D]) + tuple(desc.nv[:D])
        self.ncell = int(np.prod(self.shape))
        self.nxs = int(np.prod(desc.nx[:D]))
        tdt = torch.float64 if desc.storage == F64 else torch.float32
        if f is None:
            f = torch.empty(self.shape, dtype=tdt, device=self.device)
        if f.dtype != tdt or not f.is_contiguous() or f.numel() != self.ncell:
            raise SlmppError(ERR_SHAPE, "f must be a contiguous %s tensor of %d cells" % (tdt, self.ncell))
        self.f = f
        nbytes = workspace_bytes(desc)
        if nbytes == 0:
            st, msg = validate(desc)
            raise SlmppError(st, msg)
        self.work = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.work.data_ptr()
        self._work_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _VP()
        st = lib().slmpp_create(ctypes.byref(desc), _VP(f.data_ptr()), _VP(self._work_ptr),
                                nbytes, _VP(self.stream.cuda_stream), ctypes.byref(h))
        _check(st, None)
        self.h = h

    # ---- lifetime ----
    def close(self):
        if getattr(self, "h", None):
            lib().slmpp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _c(self, st):
        _check(st, self.h)

    # ---- the C-ABI, same names ----
    def init_f_host(self, f_host):
        a, p = _host_f64(np.asarray(f_host).ravel())
        self._c(lib().slmpp_init_f_host(self.h, p, a.size))

    def init_f_separable(self, s, gv):
        s, ps = _host_f64(s)
        gs = [_host_f64(g) for g in gv]
        ptrs = [g[1] for g in gs] + [None] * (3 - len(gs))
        self._c(lib().slmpp_init_f_separable(self.h, ps, *ptrs))

    def advect_x(self, dim, dt):
        self._c(lib().slmpp_advect_x(self.h, int(dim), float(dt)))

    def advect_v(self, dim, dt, accel):
        """accel: CUDA float64 tensor of prod(nx) values (this component)."""
        self._c(lib().slmpp_advect_v(self.h, int(dim), float(dt), _VP(accel.data_ptr())))

    def kick(self, dt):
        """All velocity axes by dt with the context's acceleration."""
        self._c(lib().slmpp_kick(self.h, float(dt)))

    def density_moment(self, rho):
        self._c(lib().slmpp_density_moment(self.h, _VP(rho.data_ptr())))

    def velocity_moments(self, rho, mean, disp):
        """CUDA float64 tensors of prod(nx), D*prod(nx), D*prod(nx) values."""
        self._c(lib().slmpp_velocity_moments(self.h, _VP(rho.data_ptr()), _VP(mean.data_ptr()),
                                             _VP(disp.data_ptr())))

    def velocity_distribution(self, F):
        """CUDA float64 tensor of prod(nv) values."""
        self._c(lib().slmpp_velocity_distribution(self.h, _VP(F.data_ptr())))

    def poisson_solve(self, rho, accel, phi=None):
        self._c(lib().slmpp_poisson_solve(self.h, _VP(rho.data_ptr()),
                                          _VP(phi.data_ptr()) if phi is not None else None,
                                          _VP(accel.data_ptr())))

    def field(self):
        self._c(lib().slmpp_field(self.h))

    def field_ptrs(self):
        r, p, a = _VP(), _VP(), _VP()
        self._c(lib().slmpp_field_ptrs(self.h, ctypes.byref(r), ctypes.byref(p), ctypes.byref(a)))
        return r.value, p.value, a.value

    def step(self, dt, nsteps=1):
        self._c(lib().slmpp_step(self.h, float(dt), int(nsteps)))

    def get_f(self):
        out = np.empty(self.shape, dtype=np.float64)
        self._c(lib().slmpp_get_f(self.h, out.ctypes.data_as(_VP), out.size))
        return out

    def diag(self):
        d = DiagOut()
        self._c(lib().slmpp_diag(self.h, ctypes.byref(d)))
        return {k: getattr(d, k) for k, _ in DiagOut._fields_}

    def sync(self):
        self._c(lib().slmpp_sync(self.h))

    def timing_enable(self, on=True):
        self._c(lib().slmpp_timing_enable(self.h, 1 if on else 0))

    def timing_read(self):
        t = Timing()
        self._c(lib().slmpp_timing_read(self.h, ctypes.byref(t)))
        return {name: dict(launches=t.launches[i], total_ms=t.total_ms[i], bytes=t.bytes[i],
                           cells=t.cells[i]) for i, name in enumerate(TIMING_NAMES)}

    def get_field(self):
        """(rho, accel) of the context as numpy arrays (accel: D*prod(nx))."""
        rho = np.empty(self.nxs, dtype=np.float64)
        acc = np.empty(self.desc.D * self.nxs, dtype=np.float64)
        self._c(lib().slmpp_get_field(self.h, rho.ctypes.data_as(_VP), acc.ctypes.data_as(_VP)))
        return rho, acc


def advect_v_noalloc(desc: GridDesc, f, dim, dt, accel, stream=None):
    """slmpp_advect_v_noalloc: one velocity sweep of the grid `desc` held in
    the CUDA tensor f (no context, no workspace); accel: CUDA float64 tensor
    of prod(nx) values.  Enqueued on `stream` (a torch.cuda.Stream; the
    current stream if None)."""
    import torch

    s = stream if stream is not None else torch.cuda.current_stream(f.device)
    _check(lib().slmpp_advect_v_noalloc(ctypes.byref(desc), _VP(f.data_ptr()), int(dim), float(dt),
                                        _VP(accel.data_ptr()), _VP(s.cuda_stream)))


class DeviceBuffer:
    """Device memory from slmpp_alloc_device (contiguous: physically
    contiguous placement, raising SlmppError when the driver cannot provide
    it); tensor() views it as a torch tensor, which keeps the buffer alive.
    free() releases the memory at once (the caller makes sure that no view
    is used afterwards and no work on it is pending); otherwise it goes when
    the buffer and all its views are gone."""

    def __init__(self, nbytes, contiguous=True):
        p = _VP()
        st = lib().slmpp_alloc_device(int(nbytes), 1 if contiguous else 0, ctypes.byref(p))
        if st != OK:
            raise SlmppError(st, (lib().slmpp_last_error(None) or b"").decode())
        self.ptr = p.value
        self.nbytes = int(nbytes)

    def tensor(self, shape, dtype, device=None):
        import torch

        n = int(np.prod(shape)) * torch.empty((), dtype=dtype).element_size()
        if n > self.nbytes:
            raise SlmppError(ERR_SHAPE, "view of %d bytes exceeds the buffer's %d" % (n, self.nbytes))
        typestr = {torch.float32: "<f4", torch.float64: "<f8"}[dtype]

        class _View:
            pass

        v = _View()
        v.__cuda_array_interface__ = {"shape": tuple(int(x) for x in shape), "typestr": typestr,
                                      "data": (self.ptr, False), "version": 2}
        v.owner = self  # torch holds the interface object as long as the tensor's storage
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        return torch.as_tensor(v, device=dev)

    def free(self):
        if self.ptr:
            lib().slmpp_free_device(_VP(self.ptr))
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def copy_device(dst_ptr, src_ptr, nbytes, stream=None):
    st = lib().slmpp_copy_device(_VP(dst_ptr), _VP(src_ptr), int(nbytes),
                                 _VP(stream.cuda_stream) if stream is not None else None)
    _check(st, None)


def _desc_array(descs):
    arr = (GridDesc * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = d
    return arr


def batch_workspace_bytes(descs) -> int:
    return int(lib().slmpp_batch_workspace_bytes(_desc_array(descs), len(descs)))


class Batch:
    """An ensemble of independent runs advanced together (slmpp_batch_*).

    descs: GridDesc per run (one storage type); dts: time step per run.
    f: per-run CUDA tensors (allocated here if not given).  The workspace
    is one uint8 CUDA tensor; all work goes to `stream`.
    """

    def __init__(self, descs, dts, fs=None, stream=None, device=None):
        import torch

        self.torch = torch
        self.descs = list(descs)
        n = len(self.descs)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.shapes = []
        for d in self.descs:
            D = d.D
            self.shapes.append(tuple(d.nx[:D]) + tuple(d.nv[:D]))
        tdt = torch.float64 if self.descs[0].storage == F64 else torch.float32
        if fs is None:
            fs = [torch.empty(sh, dtype=tdt, device=self.device) for sh in self.shapes]
        self.f = list(fs)
        arr = _desc_array(self.descs)
        nbytes = int(lib().slmpp_batch_workspace_bytes(arr, n))
        if nbytes == 0:
            for d in self.descs:
                st, msg = validate(d)
                if st != OK:
                    raise SlmppError(st, msg)
            raise SlmppError(ERR_INVALID, "the runs cannot form a batch")
        self.work = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        wp = (self.work.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        dts_c = (_D * n)(*[float(x) for x in dts])
        fp = (_VP * n)(*[t.data_ptr() for t in self.f])
        h = _VP()
        st = lib().slmpp_batch_create(arr, dts_c, n, fp, _VP(wp), nbytes,
                                      _VP(self.stream.cuda_stream), ctypes.byref(h))
        if st != OK:
            raise SlmppError(st, (lib().slmpp_batch_last_error(None) or b"").decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().slmpp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, st):
        if st != OK:
            raise SlmppError(st, (lib().slmpp_batch_last_error(self.h) or b"").decode())

    def init_separable(self, run, s, gv):
        s, ps = _host_f64(s)
        gs = [_host_f64(g) for g in gv]
        ptrs = [g[1] for g in gs] + [None] * (3 - len(gs))
        self._c(lib().slmpp_batch_init_separable(self.h, int(run), ps, *ptrs))

    def step(self, nsteps=1):
        self._c(lib().slmpp_batch_step(self.h, int(nsteps)))

    def step_eager(self, nsteps=1):
        self._c(lib().slmpp_batch_step_eager(self.h, int(nsteps)))

    def get_f(self, run):
        shape = self.shapes[run] if 0 <= run < len(self.shapes) else (0,)
        out = np.empty(shape, dtype=np.float64)
        self._c(lib().slmpp_batch_get_f(self.h, int(run), out.ctypes.data_as(_VP), out.size))
        return out

    def autotune(self, cache_path=None):
        self._c(lib().slmpp_batch_autotune(self.h, cache_path.encode() if cache_path else None))

    def tile_width(self, run, axis):
        return int(lib().slmpp_batch_tile_width(self.h, int(run), int(axis)))

    def set_fast_min_cells(self, min_cells):
        self._c(lib().slmpp_batch_set_fast_min_cells(self.h, int(min_cells)))

    def step_bytes(self):
        return float(lib().slmpp_batch_step_bytes(self.h))
