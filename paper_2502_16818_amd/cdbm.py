"""Thin Python binding of libcdbm.so (include/cdbm.h) over torch device tensors.

Only argument marshalling happens here: every step of the method runs in the
HIP kernels behind the C ABI.  torch provides device memory and the current
stream.  If the library has not been built, or no GPU is present, the calls
raise instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcdbm.so")

OK, EINVAL, ESINGULAR, ENONPHYS, EHIP, ENOMEM = 0, -1, -2, -3, -4, -5
PERIODIC, ZERO_GRADIENT = 0, 1
FP64, MIXED, MIXED_COMP = 0, 1, 2
STEP_AUTO, STEP_FUSED, STEP_SPLIT, STEP_FUSED2 = 0, 1, 2, 3

EXPORTS = (
    "cdbm_last_error", "cdbm_create", "cdbm_destroy", "cdbm_get_params", "cdbm_init",
    "cdbm_step", "cdbm_moments", "cdbm_tne", "cdbm_tne_raw", "cdbm_conserved_totals",
    "cdbm_step_adjoint",
    "cdbm_step_keep_stage", "cdbm_step_adjoint_stage", "cdbm_tau_collect",
    "cdbm_init_adjoint", "cdbm_moments_adjoint", "cdbm_batch_create", "cdbm_batch_destroy",
    "cdbm_batch_init", "cdbm_batch_step", "cdbm_conserved_totals_static",
    "cdbm_batch_get_launch", "cdbm_batch_set_launch", "cdbm_batch_autotune",
)


BATCH_CONTIGUOUS, BATCH_ROW_PIECES = 0, 1


class BatchLaunch(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_int32), ("fill_rows", ctypes.c_int32),
                ("piece_rows", ctypes.c_int32), ("tail_rows", ctypes.c_int32)]

    def as_dict(self):
        return {"layout": self.layout, "fill_rows": self.fill_rows, "piece_rows": self.piece_rows,
                "tail_rows": self.tail_rows}


class CdbmError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed with code {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dt", ctypes.c_double),
        ("tau", ctypes.c_double), ("gamma", ctypes.c_double),
        ("v", ctypes.c_double * 4), ("eta", ctypes.c_double * 4),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("step_form", ctypes.c_int32), ("dof_given", ctypes.c_int32),
        ("extra_dof", ctypes.c_double),
    ]


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32


def load() -> ctypes.CDLL:
    """Load libcdbm.so and declare the signatures of include/cdbm.h."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2502_16818_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(Params)
    sig = {
        "cdbm_last_error": ([], ctypes.c_char_p),
        "cdbm_create": ([P, ctypes.POINTER(_vp)], _i32),
        "cdbm_destroy": ([_vp], _i32),
        "cdbm_get_params": ([_vp, P], _i32),
        "cdbm_init": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
        "cdbm_step": ([_vp, _vp, _vp, _i32, _vp], _i32),
        "cdbm_moments": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
        "cdbm_tne": ([_vp, _vp, _vp, _vp], _i32),
        "cdbm_tne_raw": ([_vp, _vp, _vp, _vp], _i32),
        "cdbm_conserved_totals": ([_vp, _vp, _vp, _vp], _i32),
        "cdbm_conserved_totals_static": ([P, _vp, _vp, _vp], _i32),
        "cdbm_step_adjoint": ([_vp, _vp, _vp, _vp, _vp, _vp], _i32),
        "cdbm_step_keep_stage": ([_vp, _vp, _vp, _vp, _vp], _i32),
        "cdbm_step_adjoint_stage": ([_vp] * 7, _i32),
        "cdbm_tau_collect": ([_vp, _vp, _vp], _i32),
        "cdbm_init_adjoint": ([_vp] * 11, _i32),
        "cdbm_moments_adjoint": ([_vp] * 8, _i32),
        "cdbm_batch_create": ([P, _i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_vp)], _i32),
        "cdbm_batch_destroy": ([_vp], _i32),
        "cdbm_batch_init": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
        "cdbm_batch_step": ([_vp, _vp, _vp, _i32, _vp], _i32),
        "cdbm_batch_get_launch": ([_vp, ctypes.POINTER(BatchLaunch)], _i32),
        "cdbm_batch_set_launch": ([_vp, ctypes.POINTER(BatchLaunch)], _i32),
        "cdbm_batch_autotune": ([_vp, _vp, _vp, ctypes.c_char_p, ctypes.POINTER(BatchLaunch), _vp],
                                _i32),
    }
    for name, (args, res) in sig.items():
        if not hasattr(lib, name):
            continue
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != OK:
        raise CdbmError(rc, where, load().cdbm_last_error().decode())


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor], dtype: Optional[torch.dtype] = None,
         numel: Optional[int] = None) -> Optional[int]:
    """Device address of t after checking what the C ABI cannot: a contiguous
    tensor on the current GPU, of the element type and (at least) the number
    of elements the call reads or writes."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("CDBM buffers must be device tensors")
    if t.device.index != torch.cuda.current_device():
        raise ValueError("CDBM buffers must be on the current GPU")
    if not t.is_contiguous():
        raise ValueError("CDBM buffers must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"CDBM buffer has dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"CDBM buffer has {t.numel()} elements, the call needs {numel}")
    return t.data_ptr()


def make_params(nx, ny, dx, dy, dt, tau, gamma, v, eta, bc_x=PERIODIC, bc_y=PERIODIC,
                precision=FP64, step_form=0, extra_dof=None) -> Params:
    """cdbm_params; with extra_dof given, the gas is set by I and gamma is ignored."""
    p = Params()
    if extra_dof is not None:
        p.dof_given, p.extra_dof = 1, float(extra_dof)
    p.nx, p.ny = int(nx), int(ny)
    p.dx, p.dy, p.dt, p.tau = float(dx), float(dy), float(dt), float(tau)
    p.gamma = 0.0 if gamma is None else float(gamma)
    for k in range(4):
        p.v[k] = float(v[k])
        p.eta[k] = float(eta[k])
    p.bc_x, p.bc_y, p.precision = int(bc_x), int(bc_y), int(precision)
    p.step_form = int(step_form)
    return p


class Solver:
    """One grid of the method behind a cdbm_handle."""

    def __init__(self, params: Params):
        lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("the CDBM library needs a GPU")
        h = _vp()
        _check(lib.cdbm_create(ctypes.byref(params), ctypes.byref(h)), "cdbm_create")
        self._h = h
        self.params = params
        self.nx, self.ny = params.nx, params.ny
        self.dtype = torch.float32 if params.precision in (MIXED, MIXED_COMP) else torch.float64
        # a compensated state carries four residual planes after the 16 of f
        self.planes = 20 if params.precision == MIXED_COMP else 16

    @classmethod
    def from_run(cls, run, precision=FP64, step_form=0) -> "Solver":
        return cls(make_params(run.nx, run.ny, run.dx, run.dy, run.dt, run.tau, run.gamma, run.v,
                               run.eta, run.bc_x, run.bc_y, precision, step_form))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().cdbm_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers -----------------------------------------------------------
    def empty_f(self) -> torch.Tensor:
        return torch.empty((self.planes, self.ny, self.nx), dtype=self.dtype, device="cuda")

    def empty_field(self, *lead) -> torch.Tensor:
        return torch.empty(tuple(lead) + (self.ny, self.nx), dtype=torch.float64, device="cuda")

    def _f(self, t: torch.Tensor) -> int:
        return _ptr(t, self.dtype, self.planes * self.nx * self.ny)

    def _lam(self, t: torch.Tensor) -> int:
        return _ptr(t, torch.float64, 16 * self.nx * self.ny)

    def _field(self, a) -> torch.Tensor:
        t = torch.as_tensor(a, dtype=torch.float64)
        return t.to("cuda").contiguous().reshape(self.ny, self.nx)

    # -- forward -----------------------------------------------------------
    def init(self, rho, ux, uy, T, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        fs = [self._field(a) for a in (rho, ux, uy, T)]
        out = self.empty_f() if out is None else out
        _check(load().cdbm_init(self._h, *[_ptr(a) for a in fs], self._f(out), _stream()),
               "cdbm_init")
        return out

    def step(self, f_in: torch.Tensor, f_out: Optional[torch.Tensor] = None,
             nsteps: int = 1) -> torch.Tensor:
        f_out = self.empty_f() if f_out is None else f_out
        _check(load().cdbm_step(self._h, self._f(f_in), self._f(f_out), int(nsteps), _stream()),
               "cdbm_step")
        return f_out

    def step_keep_stage(self, f_in: torch.Tensor, f1_out: Optional[torch.Tensor] = None,
                        f_out: Optional[torch.Tensor] = None):
        """One step that also returns its first Runge-Kutta stage f_in + dt L(f_in):
        (f1_out, f_out)."""
        f1_out = self.empty_f() if f1_out is None else f1_out
        f_out = self.empty_f() if f_out is None else f_out
        _check(load().cdbm_step_keep_stage(self._h, self._f(f_in), self._f(f1_out),
                                           self._f(f_out), _stream()), "cdbm_step_keep_stage")
        return f1_out, f_out

    def moments(self, f: torch.Tensor) -> Tuple[torch.Tensor, ...]:
        outs = [self.empty_field() for _ in range(4)]
        _check(load().cdbm_moments(self._h, self._f(f), *[_ptr(o) for o in outs], _stream()),
               "cdbm_moments")
        return tuple(outs)

    def tne(self, f: torch.Tensor) -> torch.Tensor:
        out = self.empty_field(12)
        _check(load().cdbm_tne(self._h, self._f(f), _ptr(out), _stream()), "cdbm_tne")
        return out

    def tne_raw(self, f: torch.Tensor) -> torch.Tensor:
        """The same measures at the raw velocities (raw-moment construction)."""
        out = self.empty_field(12)
        _check(load().cdbm_tne_raw(self._h, self._f(f), _ptr(out), _stream()), "cdbm_tne_raw")
        return out

    def totals(self, f: torch.Tensor) -> torch.Tensor:
        out = torch.empty(4, dtype=torch.float64, device="cuda")
        _check(load().cdbm_conserved_totals(self._h, self._f(f), _ptr(out), _stream()),
               "cdbm_conserved_totals")
        return out

    # -- reverse mode (adjoint vectors are float64 in both forms) -------------
    def empty_lam(self) -> torch.Tensor:
        return torch.empty((16, self.ny, self.nx), dtype=torch.float64, device="cuda")

    def step_adjoint(self, f_n: torch.Tensor, lam_np1: torch.Tensor,
                     lam_n: Optional[torch.Tensor] = None,
                     dtau: Optional[torch.Tensor] = None,
                     f1: Optional[torch.Tensor] = None,
                     defer_tau: bool = False):
        """Transpose of one step; f1, if given, is the step's first stage (as
        step_keep_stage returns it) and saves its recomputation.  With
        defer_tau the step's dL/dtau term goes to the handle's accumulator
        (see tau_collect) and the returned dtau is None."""
        lam_n = self.empty_lam() if lam_n is None else lam_n
        if defer_tau:
            if dtau is not None:
                raise ValueError("defer_tau takes no dtau")
            dptr = None
        else:
            dtau = torch.zeros(1, dtype=torch.float64, device="cuda") if dtau is None else dtau
            dptr = _ptr(dtau, torch.float64, 1)
        if f1 is None:
            _check(load().cdbm_step_adjoint(self._h, self._f(f_n), self._lam(lam_np1),
                                            self._lam(lam_n), dptr, _stream()),
                   "cdbm_step_adjoint")
        else:
            _check(load().cdbm_step_adjoint_stage(self._h, self._f(f_n), self._f(f1),
                                                  self._lam(lam_np1), self._lam(lam_n), dptr,
                                                  _stream()), "cdbm_step_adjoint_stage")
        return lam_n, dtau

    def tau_collect(self, dtau: Optional[torch.Tensor] = None) -> torch.Tensor:
        """dtau += the dL/dtau terms of the step adjoints run with defer_tau
        since the last collect; clears them."""
        dtau = torch.zeros(1, dtype=torch.float64, device="cuda") if dtau is None else dtau
        _check(load().cdbm_tau_collect(self._h, _ptr(dtau, torch.float64, 1), _stream()),
               "cdbm_tau_collect")
        return dtau

    def init_adjoint(self, rho, ux, uy, T, lam_f0: torch.Tensor):
        fs = [self._field(a) for a in (rho, ux, uy, T)]
        outs = [self.empty_field() for _ in range(4)]
        _check(load().cdbm_init_adjoint(self._h, *[_ptr(a) for a in fs], self._lam(lam_f0),
                                        *[_ptr(o) for o in outs], _stream()), "cdbm_init_adjoint")
        return tuple(outs)

    def moments_adjoint(self, f: torch.Tensor, g_rho, g_ux, g_uy, g_T,
                        out: Optional[torch.Tensor] = None) -> torch.Tensor:
        gs = [self._field(g) for g in (g_rho, g_ux, g_uy, g_T)]
        out = self.empty_lam() if out is None else out
        _check(load().cdbm_moments_adjoint(self._h, self._f(f), *[_ptr(g) for g in gs],
                                           self._lam(out), _stream()), "cdbm_moments_adjoint")
        return out


class Batch:
    """Independent grids advanced together (cdbm_batch_*)."""

    def __init__(self, params: Sequence[Params]):
        lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("the CDBM library needs a GPU")
        n = len(params)
        arr = (Params * n)(*params)
        sizes = [16 * p.nx * p.ny for p in params]
        offs = [0]
        for s in sizes[:-1]:
            offs.append(offs[-1] + s)
        self.offsets = offs
        self.sizes = sizes
        self.total = sum(sizes)
        self.params = list(params)
        self.dtype = torch.float32 if params[0].precision == MIXED else torch.float64
        c_offs = (ctypes.c_int64 * n)(*offs)
        b = _vp()
        _check(lib.cdbm_batch_create(arr, n, c_offs, ctypes.byref(b)), "cdbm_batch_create")
        self._b = b

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            load().cdbm_batch_destroy(self._b)
            self._b = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty_f(self) -> torch.Tensor:
        return torch.empty(self.total, dtype=self.dtype, device="cuda")

    def view(self, f: torch.Tensor, k: int) -> torch.Tensor:
        p = self.params[k]
        return f[self.offsets[k]:self.offsets[k] + self.sizes[k]].view(16, p.ny, p.nx)

    def init(self, fields: Sequence[Tuple], out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if len(fields) != len(self.params):
            raise ValueError(f"{len(fields)} field sets for {len(self.params)} grids")
        for fl, p in zip(fields, self.params):
            for a in fl:
                if torch.as_tensor(a).numel() != p.nx * p.ny:
                    raise ValueError(f"a field of a {p.nx} x {p.ny} grid has {torch.as_tensor(a).numel()} values")
        cat = [torch.cat([torch.as_tensor(fl[q], dtype=torch.float64).reshape(-1) for fl in fields])
               .to("cuda").contiguous() for q in range(4)]
        out = self.empty_f() if out is None else out
        _check(load().cdbm_batch_init(self._b, *[_ptr(c) for c in cat],
                                      _ptr(out, self.dtype, self.total), _stream()),
               "cdbm_batch_init")
        return out

    def get_launch(self) -> dict:
        out = BatchLaunch()
        _check(load().cdbm_batch_get_launch(self._b, ctypes.byref(out)), "cdbm_batch_get_launch")
        return out.as_dict()

    def set_launch(self, layout: int = BATCH_CONTIGUOUS, fill_rows: int = 14,
                   piece_rows: int = 0, tail_rows: int = 0) -> None:
        l = BatchLaunch(int(layout), int(fill_rows), int(piece_rows), int(tail_rows))
        _check(load().cdbm_batch_set_launch(self._b, ctypes.byref(l)), "cdbm_batch_set_launch")

    def autotune(self, f_in: torch.Tensor, f_out: torch.Tensor,
                 cache_path: Optional[str] = None) -> dict:
        """Pick the launch layout by timing (or from the JSON cache file);
        f_out is overwritten.  Returns the layout applied."""
        out = BatchLaunch()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(load().cdbm_batch_autotune(self._b, _ptr(f_in, self.dtype, self.total),
                                          _ptr(f_out, self.dtype, self.total), path,
                                          ctypes.byref(out), _stream()), "cdbm_batch_autotune")
        return out.as_dict()

    def step(self, f_in: torch.Tensor, f_out: Optional[torch.Tensor] = None,
             nsteps: int = 1) -> torch.Tensor:
        f_out = self.empty_f() if f_out is None else f_out
        _check(load().cdbm_batch_step(self._b, _ptr(f_in, self.dtype, self.total),
                                      _ptr(f_out, self.dtype, self.total), int(nsteps), _stream()),
               "cdbm_batch_step")
        return f_out
