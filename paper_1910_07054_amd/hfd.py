"""Python binding of the HIP library ``libhfd.so`` (C ABI in include/hfd.h).

Argument marshalling only: every step of the field computation runs in the
library's kernels.  PyTorch supplies device memory (``tensor.data_ptr()``) and
the current HIP stream.  If the library has not been built the first call
raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfd.so")

HFD_OK, HFD_EINVAL, HFD_ENOMEM, HFD_EHIP, HFD_EBATCH, HFD_EHANDLE, HFD_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
HFD_FP32, HFD_FP64, HFD_MIX_SPLIT_BF16, HFD_SPLIT_PASSES, HFD_STORE_DTENSOR = 0, 1, 2, 4, 8
HFD_MIX_BATCHED_FP32 = 16
HFD_EQUIDISTANT = 32

STATUS_NAMES = {0: "HFD_OK", -1: "HFD_EINVAL", -2: "HFD_ENOMEM", -3: "HFD_EHIP", -4: "HFD_EBATCH",
                -5: "HFD_EHANDLE", -6: "HFD_ENOTSUP"}

# every function declared in include/hfd.h and include/hfd_mm.h
EXPORTS = (
    "hfd_setup_tensor", "hfd_set_thickness", "hfd_demag_field", "hfd_demag_vjp", "hfd_time_stages",
    "hfd_autotune", "hfd_get_info", "hfd_export_fourier_tensor", "hfd_export_real_tensor",
    "hfd_forward_spectrum", "hfd_destroy", "hfd_last_error", "hfd_set_path",
    "hfd_demag_field_noalloc", "hfd_set_fused",
    "hfd_mm_create", "hfd_mm_set_bias", "hfd_mm_energy_grad", "hfd_mm_destroy",
)


class HFDError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Info(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("n_geom", ctypes.c_int), ("batch_max", ctypes.c_int), ("Lx", ctypes.c_int),
                ("Ly", ctypes.c_int), ("fused", ctypes.c_int), ("fp64", ctypes.c_int),
                ("mix_bf16", ctypes.c_int), ("tensor_bytes", ctypes.c_longlong),
                ("work_bytes", ctypes.c_longlong), ("equidistant", ctypes.c_int),
                ("Lz", ctypes.c_int), ("tensor_slots", ctypes.c_int)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libhfd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build the HIP library first "
                           "(python -m paper_1910_07054_amd.build)")
    # torch first, so that the library binds to the HIP runtime torch has loaded
    # (loading the library first can bring in a second runtime, and then the
    # library's HIP calls fail on tensors torch allocated)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    i, d, p, ll = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_longlong
    sig = {
        "hfd_setup_tensor": [ctypes.POINTER(p), i, i, d, d, i, p, p, i, i, ctypes.c_uint, p],
        "hfd_set_thickness": [p, p, p, p],
        "hfd_demag_field": [p, p, p, i, p],
        "hfd_demag_field_noalloc": [p, p, p, i, p],
        "hfd_demag_vjp": [p, p, p, p, p, i, p],
        "hfd_time_stages": [p, p, p, i, i, p, p, p, p, i],
        "hfd_autotune": [p, i, p, p, i],
        "hfd_set_path": [p, i, i, i],
        "hfd_set_fused": [p, i, i, i],
        "hfd_mm_create": [ctypes.POINTER(p), p, p, d, d, d, p],
        "hfd_mm_set_bias": [p, p, p],
        "hfd_mm_energy_grad": [p, p, p, p, p, p, p, p],
        "hfd_mm_destroy": [p],
        "hfd_get_info": [p, ctypes.POINTER(Info)],
        "hfd_export_fourier_tensor": [p, i, p, ll],
        "hfd_export_real_tensor": [p, i, i, i, p, p],
        "hfd_forward_spectrum": [p, p, p, ll, i, p],
        "hfd_destroy": [p],
        "hfd_last_error": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "hfd_last_error" else ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != HFD_OK:
        msg = load().hfd_last_error()
        raise HFDError(status, msg.decode() if msg else "")


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dptr(t) -> int:
    return int(t.data_ptr())


def check_field_tensor(t, name: str, nz: int, ny: int, nx: int, fp64: bool, batch_max: int,
                       n_geom: int = 1, device=None, batch=None) -> int:
    """Check a field-shaped tensor before its pointer goes to the library:
    a torch tensor on the GPU (on ``device`` if given), float64 for FP64 plans
    and float32 otherwise, contiguous, of shape [B, 3, nz, ny, nx] with
    1 <= B <= batch_max and B a multiple of n_geom (and B == batch if given).
    Returns B; raises ValueError (TypeError for a non-tensor)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU (got device {t.device})")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the plan on {device}")
    want = torch.float64 if fp64 else torch.float32
    if t.dtype != want:
        raise ValueError(f"{name} must be {want} for this plan (got {t.dtype})")
    if t.dim() != 5 or tuple(t.shape[1:]) != (3, nz, ny, nx):
        raise ValueError(f"{name} must have shape [B, 3, {nz}, {ny}, {nx}] (got {tuple(t.shape)})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    B = int(t.shape[0])
    if B < 1 or B > batch_max:
        raise ValueError(f"{name}: batch {B} outside [1, {batch_max}]")
    if B % n_geom:
        raise ValueError(f"{name}: batch {B} is not a multiple of n_geom = {n_geom}")
    if batch is not None and B != batch:
        raise ValueError(f"{name}: batch {B} differs from {batch}")
    return B


class Plan:
    """A geometry (nx, ny, dx, dy and one or more layer stacks) with its Fourier
    tensor on the GPU.  ``thickness`` and ``z_bottom`` are [nz] or [n_geom][nz]
    host arrays (z_bottom None stacks the layers without gaps)."""

    def __init__(self, nx: int, ny: int, dx: float, dy: float, thickness, z_bottom=None,
                 batch_max: int = 1, flags: int = HFD_FP32, stream=None):
        lib = load()
        t = np.ascontiguousarray(np.atleast_2d(np.asarray(thickness, dtype=np.float64)))
        z = None if z_bottom is None else np.ascontiguousarray(
            np.atleast_2d(np.asarray(z_bottom, dtype=np.float64)))
        if z is not None and z.shape != t.shape:
            raise ValueError("z_bottom must have the shape of thickness")
        self.n_geom, self.nz = t.shape
        self.nx, self.ny, self.dx, self.dy = int(nx), int(ny), float(dx), float(dy)
        self.flags = int(flags)
        self.batch_max = int(batch_max)
        self.thickness = t.copy()
        self.z_bottom = None if z is None else z.copy()
        import torch
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        _check(lib.hfd_setup_tensor(ctypes.byref(h), self.nx, self.ny, self.dx, self.dy, self.nz,
                                    t.ctypes.data, None if z is None else z.ctypes.data,
                                    self.n_geom, self.batch_max, self.flags,
                                    _stream_handle(stream)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    @property
    def fp64(self) -> bool:
        return bool(self.flags & HFD_FP64)

    def info(self) -> Info:
        inf = Info()
        _check(load().hfd_get_info(self.handle, ctypes.byref(inf)))
        return inf

    def set_thickness(self, thickness, z_bottom=None, stream=None):
        t = np.ascontiguousarray(np.atleast_2d(np.asarray(thickness, dtype=np.float64)))
        z = None if z_bottom is None else np.ascontiguousarray(
            np.atleast_2d(np.asarray(z_bottom, dtype=np.float64)))
        _check(load().hfd_set_thickness(self.handle, t.ctypes.data,
                                        None if z is None else z.ctypes.data,
                                        _stream_handle(stream)))
        self.thickness = t.copy()
        self.z_bottom = None if z is None else z.copy()

    def check(self, t, name: str, batch=None) -> int:
        """Validate a [B, 3, nz, ny, nx] tensor for this plan (see check_field_tensor)."""
        return check_field_tensor(t, name, self.nz, self.ny, self.nx, self.fp64, self.batch_max,
                                  self.n_geom, self.device, batch)

    # -- field ---------------------------------------------------------------
    def field(self, m, out=None, stream=None):
        """h = -N * m for m of shape [B, 3, nz, ny, nx] (torch, on the GPU)."""
        import torch
        B = self.check(m, "m")
        if out is None:
            out = torch.empty_like(m, memory_format=torch.contiguous_format)
        self.check(out, "out", B)
        _check(load().hfd_demag_field(self.handle, _dptr(m), _dptr(out), int(B),
                                      _stream_handle(stream)))
        return out

    def field_noalloc(self, m, out, stream=None):
        """h = -N * m into `out` through hfd_demag_field_noalloc (the x-pass
        spectra in the library's per-GPU device scratch; nothing allocated)."""
        B = self.check(m, "m")
        self.check(out, "out", B)
        _check(load().hfd_demag_field_noalloc(self.handle, _dptr(m), _dptr(out), int(B),
                                              _stream_handle(stream)))
        return out

    def vjp(self, m, grad_h, want_m: bool = True, want_t: bool = True, stream=None):
        """(grad_m, grad_thickness[B, nz] float64) of <grad_h, h(m, t)>."""
        import torch
        B = self.check(grad_h, "grad_h")
        if want_t:
            if m is None:
                raise ValueError("m is needed for the thickness gradient")
            self.check(m, "m", B)
        gm = torch.empty_like(grad_h, memory_format=torch.contiguous_format) if want_m else None
        gt = torch.empty((B, self.nz), dtype=torch.float64, device=grad_h.device) if want_t else None
        _check(load().hfd_demag_vjp(self.handle, _dptr(m) if m is not None else None, _dptr(grad_h),
                                    _dptr(gm) if gm is not None else None,
                                    _dptr(gt) if gt is not None else None, int(B),
                                    _stream_handle(stream)))
        return gm, gt

    def forward_spectrum(self, m, stream=None):
        import torch
        inf = self.info()
        B = self.check(m, "m")
        dt = torch.complex128 if self.fp64 else torch.complex64
        out = torch.empty((B, 3, self.nz, inf.Lx // 2, inf.Ly), dtype=dt, device=m.device)
        _check(load().hfd_forward_spectrum(self.handle, _dptr(m), _dptr(out),
                                           out.numel() * out.element_size(), int(B),
                                           _stream_handle(stream)))
        return out

    def time_stages(self, m, h, reps: int = 20, stream=None):
        B = self.check(m, "m")
        self.check(h, "h", B)
        ms = (ctypes.c_double * 8)()
        n = ctypes.c_int()
        names = ctypes.create_string_buffer(256)
        _check(load().hfd_time_stages(self.handle, _dptr(m), _dptr(h), int(m.shape[0]), int(reps),
                                      _stream_handle(stream), ms, ctypes.byref(n), names, 256))
        labels = names.value.decode().split(";")
        return {labels[k]: ms[k] for k in range(n.value)}

    def autotune(self, batch: int = 1, stream=None) -> str:
        rep = ctypes.create_string_buffer(1024)
        _check(load().hfd_autotune(self.handle, int(batch), _stream_handle(stream), rep, 1024))
        return rep.value.decode()

    def set_path(self, batch: int, path: int, x_tile: int = 0):
        """Pin the field path and x-pass tile for `batch` states (path < 0: unpin)."""
        _check(load().hfd_set_path(self.handle, int(batch), int(path), int(x_tile)))

    def set_fused(self, batch: int, chunk: int = 0, generic: bool = False):
        """Pin the fused path's states per run (0: whole batch) and kernel
        variant (generic: run-time layer count) for `batch` states."""
        _check(load().hfd_set_fused(self.handle, int(batch), int(chunk), int(bool(generic))))

    # -- inspection ----------------------------------------------------------
    def export_fourier_tensor(self, geom: int = 0) -> np.ndarray:
        """[Lx/2+1][P][5][Ly/2+1]; equidistant plans: [Lx/2+1][Lz/2+1][6][Ly/2+1]."""
        inf = self.info()
        P = self.nz * (self.nz + 1) // 2
        QX, QY = inf.Lx // 2 + 1, inf.Ly // 2 + 1
        shape = (QX, inf.Lz // 2 + 1, 6, QY) if inf.equidistant else (QX, P, 5, QY)
        out = np.empty(shape, dtype=np.float64 if self.fp64 else np.float32)
        _check(load().hfd_export_fourier_tensor(self.handle, int(geom), out.ctypes.data, out.nbytes))
        return out

    def export_real_tensor(self, i: int, j: int, geom: int = 0, stream=None) -> np.ndarray:
        out = np.empty((6, 2 * self.ny - 1, 2 * self.nx - 1), dtype=np.float64)
        _check(load().hfd_export_real_tensor(self.handle, int(geom), int(i), int(j), out.ctypes.data,
                                             _stream_handle(stream)))
        return out

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            _check(load().hfd_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _autograd():
    import torch

    class DemagField(torch.autograd.Function):
        """h = -N(t) * m with gradients for m and for the layer thicknesses.

        forward(m, thickness, plan): ``thickness`` must equal the plan's
        thicknesses ([n_geom, nz] float64 tensor); the backward pass returns
        d/dm through the transposed field kernel and d/dthickness through the
        thickness derivative of the Newell tensor (layers above a thickened
        layer move up, gaps fixed)."""

        @staticmethod
        def forward(ctx, m, thickness, plan):
            tt = thickness.detach().cpu().numpy().reshape(plan.n_geom, plan.nz)
            if not np.array_equal(tt, plan.thickness):
                raise ValueError("thickness differs from the plan geometry; call plan.set_thickness")
            m = m.contiguous()
            ctx.plan = plan
            ctx.t_device, ctx.t_dtype, ctx.t_shape = thickness.device, thickness.dtype, thickness.shape
            ctx.save_for_backward(m)
            return plan.field(m)

        @staticmethod
        def backward(ctx, grad_h):
            (m,) = ctx.saved_tensors
            plan = ctx.plan
            need_m, need_t = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            gm, gt = plan.vjp(m, grad_h.contiguous(), want_m=need_m, want_t=need_t)
            gthick = None
            if need_t:
                # states b * bpg .. (b + 1) * bpg - 1 use stack b: their gradients add up
                B = gt.shape[0]
                gthick = gt.reshape(plan.n_geom, B // plan.n_geom, plan.nz).sum(1)
                gthick = gthick.to(device=ctx.t_device, dtype=ctx.t_dtype).reshape(ctx.t_shape)
            return gm, gthick, None

    return DemagField


def demag_field(m, thickness, plan: Plan):
    """Differentiable h = -N(thickness) * m (see DemagField)."""
    return _autograd().apply(m, thickness, plan)
