"""ctypes binding of libbpm.so (include/bpm.h): argument marshalling only.

Every step of the march runs in the library's gfx950 kernels; PyTorch only
provides device memory and streams.  If the library is not built the import
fails loudly -- there is no fallback.
"""

from __future__ import annotations

import ctypes
import math
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbpm.so")

BPM_OK, BPM_EINVAL, BPM_ENOMEM, BPM_EHIP, BPM_EUNSUPPORTED = 0, -1, -2, -3, -4
PRECISION = {"fp64": 0, "fp32": 1, "fp32s": 2}
SCHEDULE = {"auto": -1, "stockham": 0, "fourstep": 1, "split": 2}
NOALLOC_MAX_BYTES = 128 << 20        # BPM_NOALLOC_MAX_BYTES of include/bpm.h
_CODES = {BPM_EINVAL: "EINVAL", BPM_ENOMEM: "ENOMEM", BPM_EHIP: "EHIP",
          BPM_EUNSUPPORTED: "EUNSUPPORTED"}


class BpmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bpm error {_CODES.get(code, code)}: {msg}")
        self.code = code


class bpm_complex(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class bpm_job(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("E0_in", ctypes.c_void_p),
                ("u_field", ctypes.c_void_p), ("E0_out", ctypes.c_void_p),
                ("Eh_out", ctypes.c_void_p), ("workspace", ctypes.c_void_p)]


_lib = None
_lock = threading.Lock()

# (name, restype, argtypes) of every exported function
_SIGNATURES = [
    ("bpm_plan_create", ctypes.c_void_p,
     [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
      bpm_complex, bpm_complex, bpm_complex, ctypes.c_double, ctypes.c_double,
      ctypes.c_int]),
    ("bpm_plan_create_3d", ctypes.c_void_p,
     [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
      ctypes.c_int, bpm_complex, bpm_complex, bpm_complex, ctypes.c_double,
      ctypes.c_double, ctypes.c_int]),
    ("bpm_plan_set_precision", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("bpm_plan_set_crystal", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]),
    ("bpm_plan_set_detuning", ctypes.c_int,
     [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    ("bpm_plan_set_options", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    ("bpm_plan_set_schedule", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("bpm_plan_set_time_grid", ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    ("bpm_plan_set_mask", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("bpm_time_to_frequency", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("bpm_frequency_to_time", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("bpm_plan_get_schedule", ctypes.c_int, [ctypes.c_void_p]),
    ("bpm_plan_get_constants", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    ("bpm_workspace_bytes", ctypes.c_size_t, [ctypes.c_void_p]),
    ("bpm_propagate", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_void_p, ctypes.c_void_p]),
    ("bpm_propagate_noalloc", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_void_p, ctypes.c_void_p]),
    ("bpm_propagate_ws", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("bpm_deformation_table", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("bpm_march", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_void_p, ctypes.c_void_p]),
    ("bpm_batch_create", ctypes.c_void_p, [ctypes.POINTER(bpm_job), ctypes.c_int]),
    ("bpm_batch_launch", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("bpm_batch_info", ctypes.c_int,
     [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
      ctypes.POINTER(ctypes.c_int)]),
    ("bpm_batch_destroy", None, [ctypes.c_void_p]),
    ("bpm_propagate_batch", ctypes.c_int,
     [ctypes.POINTER(bpm_job), ctypes.c_int, ctypes.c_void_p]),
    ("bpm_march_segment", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("bpm_plan_destroy", None, [ctypes.c_void_p]),
    ("bpm_last_error", ctypes.c_char_p, []),
]


def lib():
    """The loaded library (raises if libbpm.so has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(
                    f"{LIB_PATH} is missing: build it with "
                    "paper_2201_08500_amd.build.build() (no fallback path exists)")
            handle = ctypes.CDLL(LIB_PATH)
            for name, res, args in _SIGNATURES:
                fn = getattr(handle, name)
                fn.restype = res
                fn.argtypes = args
            _lib = handle
    return _lib


def last_error() -> str:
    return lib().bpm_last_error().decode()


def _check(rc):
    if rc != BPM_OK:
        raise BpmError(rc, last_error())


def _cx(z) -> bpm_complex:
    z = complex(z)
    return bpm_complex(z.real, z.imag)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """Owns a bpm_plan (see include/bpm.h for the meaning of every argument)."""

    Ny = 1   # rows along y (Plan3D)

    def __init__(self, Nx, dx, dz, Nz, chi0, chih, chihbar, theta_B, lam,
                 Nomega, precision="fp64", x_front=None, thickness=None,
                 delta=None, split_order=1, zassenhaus=True, schedule=None,
                 time_step=None, mask=None, _handle=None):
        L = lib()
        self._h = None
        if _handle is None:
            h = L.bpm_plan_create(int(Nx), float(dx), float(dz), int(Nz),
                                  _cx(chi0), _cx(chih), _cx(chihbar),
                                  float(theta_B), float(lam), int(Nomega))
        else:
            h = _handle
        if not h:
            raise BpmError(BPM_EINVAL, last_error())
        self._h = ctypes.c_void_p(h)
        self.Nx, self.Nz, self.Nomega = int(Nx), int(Nz), int(Nomega)
        self.precision = precision
        _check(L.bpm_plan_set_precision(self._h, PRECISION[precision]))
        if x_front is not None or thickness is not None:
            _check(L.bpm_plan_set_crystal(
                self._h, float(0.0 if x_front is None else x_front),
                float(math.inf if thickness is None else thickness)))
        if delta is not None:
            delta = [float(d) for d in delta]
            if len(delta) != self.Nomega:
                raise ValueError(f"delta has {len(delta)} values for {self.Nomega} slices")
            arr = (ctypes.c_double * self.Nomega)(*delta)
            _check(L.bpm_plan_set_detuning(self._h, arr))
        self.time_step = None
        if time_step is not None:
            if delta is not None:
                raise ValueError("time_step sets the detuning grid; do not pass delta too")
            _check(L.bpm_plan_set_time_grid(self._h, float(time_step)))
            self.time_step = float(time_step)
        if mask is not None:
            import numpy as np
            m = np.ascontiguousarray(np.asarray(mask) != 0, dtype=np.uint8)
            if m.shape != self.u_shape:
                raise ValueError(f"mask must have shape {self.u_shape}")
            _check(L.bpm_plan_set_mask(self._h, m.ctypes.data_as(ctypes.c_void_p)))
        if split_order != 1 or not zassenhaus:
            _check(L.bpm_plan_set_options(self._h, int(split_order),
                                          int(bool(zassenhaus))))
        if schedule is None and _handle is None:
            from .autotune import cached_choice
            schedule = cached_choice(precision, Nx)
        if schedule is not None:
            _check(L.bpm_plan_set_schedule(self._h, SCHEDULE[schedule]
                                           if isinstance(schedule, str) else int(schedule)))

    @property
    def schedule(self) -> int:
        return int(lib().bpm_plan_get_schedule(self._h))

    @classmethod
    def from_workload(cls, w, precision="fp64", **kw):
        return cls(w.Nx, w.dx, w.dz, w.Nz, w.chi0, w.chih, w.chihbar,
                   w.theta_B, w.lam, w.Nomega, precision=precision,
                   x_front=w.x_front, thickness=w.thickness, delta=w.delta, **kw)

    @property
    def handle(self):
        return self._h

    @property
    def field_dtype(self):
        import torch
        return torch.complex128 if self.precision == "fp64" else torch.complex64

    def constants(self, w: int):
        out = (ctypes.c_double * 8)()
        _check(lib().bpm_plan_get_constants(self._h, int(w), out))
        return list(out)

    def workspace_bytes(self) -> int:
        return int(lib().bpm_workspace_bytes(self._h))

    @property
    def field_shape(self):
        return (self.Nomega, self.Nx)

    @property
    def u_shape(self):
        return (self.Nz, self.Nx)

    def _check_field(self, t, name):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()
                and t.dtype == self.field_dtype
                and tuple(t.shape) == self.field_shape):
            raise ValueError(f"{name} must be a contiguous CUDA {self.field_dtype} "
                             f"tensor of shape {self.field_shape}")

    def _check_u(self, u):
        import torch
        if not (isinstance(u, torch.Tensor) and u.is_cuda and u.is_contiguous()
                and u.dtype == torch.float64 and tuple(u.shape) == self.u_shape):
            raise ValueError(f"u must be a contiguous CUDA float64 tensor of shape "
                             f"{self.u_shape}")

    def propagate(self, E0_in, u=None, E0_out=None, Eh_out=None,
                  workspace=None, stream=None):
        """bpm_propagate (or bpm_propagate_ws when a workspace is given);
        returns (E0_out, Eh_out).  Asynchronous on the stream."""
        import torch
        self._check_field(E0_in, "E0_in")
        if u is not None:
            self._check_u(u)
        if E0_out is None:
            E0_out = torch.empty_like(E0_in)
        if Eh_out is None:
            Eh_out = torch.empty_like(E0_in)
        self._check_field(E0_out, "E0_out")
        self._check_field(Eh_out, "Eh_out")
        s = _stream_handle(stream)
        if workspace is None:
            rc = lib().bpm_propagate(self._h, _ptr(E0_in), _ptr(u), _ptr(E0_out),
                                     _ptr(Eh_out), s)
        else:
            if workspace.numel() * workspace.element_size() < self.workspace_bytes():
                raise ValueError("workspace too small")
            rc = lib().bpm_propagate_ws(self._h, _ptr(E0_in), _ptr(u),
                                        _ptr(E0_out), _ptr(Eh_out),
                                        _ptr(workspace), s)
        _check(rc)
        return E0_out, Eh_out

    def propagate_noalloc(self, E0_in, u, E0_out, Eh_out, stream=None):
        """bpm_propagate_noalloc: bpm_propagate with its workspace in the
        library's static device array (no device allocation by the call;
        the outputs are caller-provided)."""
        import torch
        self._check_field(E0_in, "E0_in")
        self._check_field(E0_out, "E0_out")
        self._check_field(Eh_out, "Eh_out")
        if u is not None:
            self._check_u(u)
        _check(lib().bpm_propagate_noalloc(self._h, _ptr(E0_in), _ptr(u), _ptr(E0_out),
                                           _ptr(Eh_out), _stream_handle(stream)))
        return E0_out, Eh_out

    def deformation_table(self, u, workspace, stream=None):
        """bpm_deformation_table: exp(i h u) for every cell into workspace."""
        self._check_u(u)
        if workspace.numel() * workspace.element_size() < self.workspace_bytes():
            raise ValueError("workspace too small")
        _check(lib().bpm_deformation_table(self._h, _ptr(u), _ptr(workspace),
                                           _stream_handle(stream)))
        return workspace

    def march(self, E0_in, table, E0_out, Eh_out, stream=None):
        """bpm_march: the Nz-step march reading a deformation table (or None)."""
        self._check_field(E0_in, "E0_in")
        self._check_field(E0_out, "E0_out")
        self._check_field(Eh_out, "Eh_out")
        _check(lib().bpm_march(self._h, _ptr(E0_in), _ptr(table), _ptr(E0_out),
                               _ptr(Eh_out), _stream_handle(stream)))
        return E0_out, Eh_out

    def march_segment(self, E0_in, Eh_in, table, n0, nsteps, E0_out, Eh_out,
                      stream=None):
        """bpm_march_segment: steps n0 .. n0+nsteps-1 from (E0_in, Eh_in)."""
        self._check_field(E0_in, "E0_in")
        if Eh_in is not None:
            self._check_field(Eh_in, "Eh_in")
        self._check_field(E0_out, "E0_out")
        self._check_field(Eh_out, "Eh_out")
        _check(lib().bpm_march_segment(self._h, _ptr(E0_in), _ptr(Eh_in),
                                       _ptr(table), int(n0), int(nsteps),
                                       _ptr(E0_out), _ptr(Eh_out),
                                       _stream_handle(stream)))
        return E0_out, Eh_out

    def to_frequency(self, field_t, out=None, stream=None):
        """bpm_time_to_frequency of a [Nomega][Nx] pulse field (time first)."""
        import torch
        self._check_field(field_t, "field_t")
        out = torch.empty_like(field_t) if out is None else out
        self._check_field(out, "out")
        _check(lib().bpm_time_to_frequency(self._h, _ptr(field_t), _ptr(out),
                                           _stream_handle(stream)))
        return out

    def to_time(self, field_w, out=None, stream=None):
        """bpm_frequency_to_time of a [Nomega][Nx] field (frequency first)."""
        import torch
        self._check_field(field_w, "field_w")
        out = torch.empty_like(field_w) if out is None else out
        self._check_field(out, "out")
        _check(lib().bpm_frequency_to_time(self._h, _ptr(field_w), _ptr(out),
                                           _stream_handle(stream)))
        return out

    def propagate_pulse(self, field_t, u=None, stream=None):
        """Incident pulse in time -> (transmitted, reflected) pulses in time:
        bpm_time_to_frequency, bpm_propagate, bpm_frequency_to_time (both
        outputs transformed in place)."""
        E0 = self.to_frequency(field_t, stream=stream)
        a, b = self.propagate(E0, u, stream=stream)
        self.to_time(a, out=a, stream=stream)
        self.to_time(b, out=b, stream=stream)
        return a, b

    def close(self):
        if self._h is not None and _lib is not None:
            _lib.bpm_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan3D(Plan):
    """A plan on a 3D grid (bpm_plan_create_3d): Ny rows of dy along y, any Nx
    along x; fields (Nomega, Ny, Nx), displacement (Nz, Ny, Nx).  Supports
    propagate (with or without a caller workspace), deformation_table, march,
    march_segment, the pulse transforms and the precision, crystal (slab or
    a general mask of shape (Nz, Ny, Nx)), detuning, splitting and time-grid
    settings of Plan."""

    def __init__(self, Nx, Ny, dx, dy, dz, Nz, chi0, chih, chihbar, theta_B, lam,
                 Nomega, precision="fp64", x_front=None, thickness=None,
                 delta=None, split_order=1, zassenhaus=True, time_step=None, mask=None):
        h = lib().bpm_plan_create_3d(int(Nx), int(Ny), float(dx), float(dy), float(dz),
                                     int(Nz), _cx(chi0), _cx(chih), _cx(chihbar),
                                     float(theta_B), float(lam), int(Nomega))
        if not h:
            raise BpmError(BPM_EINVAL, last_error())
        self.Ny = int(Ny)
        super().__init__(Nx, dx, dz, Nz, chi0, chih, chihbar, theta_B, lam, Nomega,
                         precision=precision, x_front=x_front, thickness=thickness,
                         delta=delta, split_order=split_order, zassenhaus=zassenhaus,
                         time_step=time_step, mask=mask, _handle=h)

    @classmethod
    def from_workload(cls, w, precision="fp64", **kw):
        return cls(w.Nx, w.Ny, w.dx, w.dy, w.dz, w.Nz, w.chi0, w.chih, w.chihbar,
                   w.theta_B, w.lam, w.Nomega, precision=precision,
                   x_front=w.x_front, thickness=w.thickness, delta=w.delta, **kw)

    @property
    def field_shape(self):
        return (self.Nomega, self.Ny, self.Nx)

    @property
    def u_shape(self):
        return (self.Nz, self.Ny, self.Nx)


class Job:
    """One batch entry: a Plan and its device buffers (outputs allocated if
    not given; a workspace is allocated for a deformed job if not given)."""

    def __init__(self, plan, E0_in, u=None, E0_out=None, Eh_out=None,
                 workspace=None):
        import torch
        plan._check_field(E0_in, "E0_in")
        self.plan, self.E0_in, self.u = plan, E0_in, u
        self.E0_out = torch.empty_like(E0_in) if E0_out is None else E0_out
        self.Eh_out = torch.empty_like(E0_in) if Eh_out is None else Eh_out
        plan._check_field(self.E0_out, "E0_out")
        plan._check_field(self.Eh_out, "Eh_out")
        if u is not None:
            plan._check_u(u)
            if workspace is None:
                workspace = torch.empty(plan.workspace_bytes(), dtype=torch.uint8,
                                        device=E0_in.device)
        self.workspace = workspace

    def as_struct(self) -> bpm_job:
        return bpm_job(self.plan.handle, self.E0_in.data_ptr(),
                       None if self.u is None else self.u.data_ptr(),
                       self.E0_out.data_ptr(), self.Eh_out.data_ptr(),
                       None if self.workspace is None else self.workspace.data_ptr())


def _job_array(jobs):
    arr = (bpm_job * len(jobs))(*[j.as_struct() for j in jobs])
    return arr


class Batch:
    """bpm_batch: prepared once, launched (or graph-captured) many times."""

    def __init__(self, jobs):
        self.jobs = list(jobs)           # keeps plans and buffers alive
        h = lib().bpm_batch_create(_job_array(self.jobs), len(self.jobs))
        if not h:
            raise BpmError(BPM_EINVAL, last_error())
        self._h = ctypes.c_void_p(h)

    def launch(self, stream=None):
        _check(lib().bpm_batch_launch(self._h, _stream_handle(stream)))

    def info(self):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().bpm_batch_info(self._h, ctypes.byref(a), ctypes.byref(b),
                                    ctypes.byref(c)))
        return dict(launches=a.value, slices=b.value, workgroups=c.value)

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.bpm_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def propagate_batch(jobs, stream=None):
    """bpm_propagate_batch over Job objects (asynchronous on the stream)."""
    jobs = list(jobs)
    _check(lib().bpm_propagate_batch(_job_array(jobs), len(jobs),
                                     _stream_handle(stream)))
    return jobs
