"""MI355X-native complex-to-complex 3D FFT: CROFT's method on one GPU.

A thin ctypes binding of ``libcroft.so`` (the C ABI declared in
``include/croft.h``).  The functions keep the C names and only marshal
arguments: every step of the transform runs in the library's HIP kernels.
Torch tensors are accepted wherever the C call takes a device pointer (their
``data_ptr()`` is passed) and ``stream=None`` means torch's current stream on
the tensor's device.  Status codes other than CROFT_SUCCESS raise
``ValueError`` (argument, size and dtype errors) or ``RuntimeError``.

The library must be built (``__graft_entry__.build()``); importing the
binding without it fails with RuntimeError at the first call.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcroft.so")

CROFT_C64, CROFT_C128, CROFT_C16F, CROFT_C16B = 0, 1, 2, 3
CROFT_FORWARD, CROFT_BACKWARD = -1, 1
CROFT_SUCCESS = 0
CROFT_ERR_INVALID_VALUE = 1
CROFT_ERR_UNSUPPORTED_SIZE = 2
CROFT_ERR_UNSUPPORTED_DTYPE = 3
CROFT_ERR_OUT_OF_MEMORY = 4
CROFT_ERR_HIP = 5
CROFT_ERR_INTERNAL = 6
CROFT_ESTIMATE, CROFT_MEASURE, CROFT_FORCE_GENERIC, CROFT_NO_WISDOM, CROFT_PERSISTENT = 0, 1, 2, 4, 8
CROFT_UNFUSED = 16
CROFT_GRAPH = 32
CROFT_MAX_PASSES = 8
CROFT_MAX_STAGES = 12

# every symbol include/croft.h declares
EXPORTED = (
    "croft_plan_create", "croft_plan_create_ex", "croft_execute", "croft_execute_scaled",
    "croft_plan_destroy", "croft_last_error", "croft_last_status", "croft_plan_create_batched",
    "croft_plan_batched_offsets", "croft_execute_batched", "croft_plan_info",
    "croft_plan_describe", "croft_plan_profile", "croft_plan_profile_read",
    "croft_plan_create_real", "croft_plan_describe_real", "croft_plan_create_convolution",
    "croft_execute_convolution", "croft_plan_describe_convolution", "croft_execute_scaled_noalloc",
)
CROFT_NOALLOC_SCRATCH_BYTES = 4 << 20


class CroftError(RuntimeError):
    pass


class PassInfo(ctypes.Structure):
    _fields_ = [("axis", ctypes.c_int), ("n", ctypes.c_int), ("kind", ctypes.c_int),
                ("generic", ctypes.c_int), ("nstages", ctypes.c_int),
                ("radices", ctypes.c_int * CROFT_MAX_STAGES),
                ("threads_per_line", ctypes.c_int), ("lines_per_block", ctypes.c_int),
                ("block_threads", ctypes.c_int), ("blocks", ctypes.c_longlong),
                ("lds_bytes", ctypes.c_size_t), ("bluestein", ctypes.c_int)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("dtype", ctypes.c_int), ("dir", ctypes.c_int), ("batched_count", ctypes.c_int),
                ("slabs", ctypes.c_int), ("npasses", ctypes.c_int),
                ("pass_", PassInfo * CROFT_MAX_PASSES),
                ("elements", ctypes.c_size_t), ("element_bytes", ctypes.c_size_t),
                ("work_bytes", ctypes.c_size_t), ("algorithmic_bytes", ctypes.c_double),
                ("flops", ctypes.c_double), ("real", ctypes.c_int), ("convolution", ctypes.c_int),
                ("graph_replay", ctypes.c_int)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "pass_"}
        d["passes"] = []
        for i in range(self.npasses):
            p = self.pass_[i]
            pd = {k: getattr(p, k) for k, _ in PassInfo._fields_ if k != "radices"}
            pd["radices"] = [p.radices[s] for s in range(p.nstages)]
            d["passes"].append(pd)
        return d


_lib = None


def load():
    """The loaded libcroft.so (raises RuntimeError if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: the HIP library must be built "
                           "(__graft_entry__.build()); there is no fallback")
    lib = ctypes.CDLL(LIB_PATH)
    i, p, vp = ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p
    lib.croft_plan_create.argtypes = [i, i, i, i, i]
    lib.croft_plan_create.restype = p
    lib.croft_plan_create_ex.argtypes = [i, i, i, i, i, i, i]
    lib.croft_plan_create_ex.restype = p
    lib.croft_execute.argtypes = [p, vp, vp, vp]
    lib.croft_execute.restype = i
    lib.croft_execute_scaled.argtypes = [p, vp, vp, vp, vp, vp]
    lib.croft_execute_scaled.restype = i
    lib.croft_execute_scaled_noalloc.argtypes = [p, vp, vp, vp, vp, vp]
    lib.croft_execute_scaled_noalloc.restype = i
    lib.croft_plan_destroy.argtypes = [p]
    lib.croft_plan_destroy.restype = i
    lib.croft_last_error.argtypes = []
    lib.croft_last_error.restype = ctypes.c_char_p
    lib.croft_last_status.argtypes = []
    lib.croft_last_status.restype = i
    lib.croft_plan_create_batched.argtypes = [i, ctypes.POINTER(ctypes.c_int), i, i, i]
    lib.croft_plan_create_batched.restype = p
    lib.croft_plan_batched_offsets.argtypes = [p, ctypes.POINTER(ctypes.c_size_t)]
    lib.croft_plan_batched_offsets.restype = i
    lib.croft_execute_batched.argtypes = [p, vp, vp, vp]
    lib.croft_execute_batched.restype = i
    lib.croft_plan_info.argtypes = [p, ctypes.POINTER(PlanInfo)]
    lib.croft_plan_info.restype = i
    lib.croft_plan_describe.argtypes = [i, i, i, i, i, ctypes.c_char_p, ctypes.c_size_t]
    lib.croft_plan_describe.restype = i
    lib.croft_plan_create_real.argtypes = [i, i, i, i, i, i]
    lib.croft_plan_create_real.restype = p
    lib.croft_plan_describe_real.argtypes = [i, i, i, i, i, ctypes.c_char_p, ctypes.c_size_t]
    lib.croft_plan_describe_real.restype = i
    lib.croft_plan_create_convolution.argtypes = [i, i, i, i, i]
    lib.croft_plan_create_convolution.restype = p
    lib.croft_execute_convolution.argtypes = [p, vp, vp, vp, vp, vp]
    lib.croft_execute_convolution.restype = i
    lib.croft_plan_describe_convolution.argtypes = [i, i, i, i, ctypes.c_char_p, ctypes.c_size_t]
    lib.croft_plan_describe_convolution.restype = i
    lib.croft_plan_profile.argtypes = [p, i]
    lib.croft_plan_profile.restype = i
    lib.croft_plan_profile_read.argtypes = [p, ctypes.POINTER(ctypes.c_double), i,
                                            ctypes.POINTER(ctypes.c_int)]
    lib.croft_plan_profile_read.restype = i
    _lib = lib
    return lib


def croft_last_error() -> str:
    return load().croft_last_error().decode()


def _check(status: int) -> None:
    if status == CROFT_SUCCESS:
        return
    msg = croft_last_error()
    if status in (CROFT_ERR_INVALID_VALUE, CROFT_ERR_UNSUPPORTED_SIZE, CROFT_ERR_UNSUPPORTED_DTYPE):
        raise ValueError(f"croft status {status}: {msg}")
    raise CroftError(f"croft status {status}: {msg}")


def croft_last_status() -> int:
    return load().croft_last_status()


def _created(handle):
    if not handle:
        status = croft_last_status()
        _check(status if status != CROFT_SUCCESS else CROFT_ERR_INTERNAL)
    return handle


def _ptr(x):
    """Device pointer of a torch tensor, or an int address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream, *tensors):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    dev = next((t.device for t in tensors if hasattr(t, "device")), None)
    return torch.cuda.current_stream(dev).cuda_stream


def croft_plan_create(nx, ny, nz, dtype=CROFT_C64, dir=CROFT_FORWARD):
    return _created(load().croft_plan_create(nx, ny, nz, dtype, dir))


def croft_plan_create_ex(nx, ny, nz, dtype=CROFT_C64, dir=CROFT_FORWARD, flags=0, slabs=1):
    return _created(load().croft_plan_create_ex(nx, ny, nz, dtype, dir, flags, slabs))


def croft_execute(plan, inp, out, stream=None) -> None:
    _check(load().croft_execute(plan, _ptr(inp), _ptr(out), _stream(stream, inp, out)))


def croft_execute_scaled(plan, inp, in_exp, out, out_exp, stream=None) -> None:
    _check(load().croft_execute_scaled(plan, _ptr(inp), _ptr(in_exp), _ptr(out), _ptr(out_exp),
                                       _stream(stream, inp, out)))


def croft_execute_scaled_noalloc(plan, inp, in_exp, out, out_exp, stream=None) -> None:
    _check(load().croft_execute_scaled_noalloc(plan, _ptr(inp), _ptr(in_exp), _ptr(out), _ptr(out_exp),
                                               _stream(stream, inp, out)))


def croft_plan_destroy(plan) -> None:
    _check(load().croft_plan_destroy(plan))


def croft_plan_create_batched(dims, dtype=CROFT_C64, dir=CROFT_FORWARD, flags=0):
    flat = [int(v) for row in dims for v in row]
    arr = (ctypes.c_int * len(flat))(*flat)
    return _created(load().croft_plan_create_batched(len(flat) // 3, arr, dtype, dir, flags))


def croft_plan_batched_offsets(plan, count: int) -> list:
    arr = (ctypes.c_size_t * (count + 1))()
    _check(load().croft_plan_batched_offsets(plan, arr))
    return list(arr)


def croft_execute_batched(plan, inp, out, stream=None) -> None:
    _check(load().croft_execute_batched(plan, _ptr(inp), _ptr(out), _stream(stream, inp, out)))


def croft_plan_info(plan) -> dict:
    info = PlanInfo()
    _check(load().croft_plan_info(plan, ctypes.byref(info)))
    return info.as_dict()


def croft_plan_describe(nx, ny, nz, dtype=CROFT_C64, dir=CROFT_FORWARD) -> str:
    buf = ctypes.create_string_buffer(8192)
    _check(load().croft_plan_describe(nx, ny, nz, dtype, dir, buf, len(buf)))
    return buf.value.decode()


def croft_plan_create_real(nx, ny, nz, dtype=CROFT_C64, dir=CROFT_FORWARD, flags=0):
    return _created(load().croft_plan_create_real(nx, ny, nz, dtype, dir, flags))


def croft_plan_describe_real(nx, ny, nz, dtype=CROFT_C64, dir=CROFT_FORWARD) -> str:
    buf = ctypes.create_string_buffer(8192)
    _check(load().croft_plan_describe_real(nx, ny, nz, dtype, dir, buf, len(buf)))
    return buf.value.decode()


def croft_plan_create_convolution(nx, ny, nz, dtype=CROFT_C64, flags=0):
    return _created(load().croft_plan_create_convolution(nx, ny, nz, dtype, flags))


def croft_execute_convolution(plan, inp, mul, out, energy=None, stream=None) -> None:
    """energy: None, or a one-element float64 device tensor (or address)."""
    _check(load().croft_execute_convolution(plan, _ptr(inp), _ptr(mul), _ptr(out), _ptr(energy),
                                            _stream(stream, inp, out)))


def croft_plan_describe_convolution(nx, ny, nz, dtype=CROFT_C64) -> str:
    buf = ctypes.create_string_buffer(8192)
    _check(load().croft_plan_describe_convolution(nx, ny, nz, dtype, buf, len(buf)))
    return buf.value.decode()


def croft_plan_profile(plan, enable: bool) -> None:
    _check(load().croft_plan_profile(plan, 1 if enable else 0))


def croft_plan_profile_read(plan, max_passes: int = CROFT_MAX_PASSES):
    """(per-pass total ms list, execute count)."""
    arr = (ctypes.c_double * max_passes)()
    n = ctypes.c_int(0)
    _check(load().croft_plan_profile_read(plan, arr, max_passes, ctypes.byref(n)))
    return list(arr), n.value


class Plan:
    """Owning wrapper of a single-grid plan: ``Plan(nx, ny, nz, dtype, dir)``.

    ``plan(inp, out)`` runs croft_execute (C64/C128) and
    ``plan.scaled(inp, in_exp, out, out_exp)`` runs croft_execute_scaled.
    Tensors must be contiguous device tensors of shape (nz, ny, nx) (complex64 /
    complex128) or (nz, ny, nx, 2) (float16 / bfloat16); the wrapper checks
    shapes and dtypes, then passes pointers through.
    """

    _TORCH = {CROFT_C64: "complex64", CROFT_C128: "complex128", CROFT_C16F: "float16",
              CROFT_C16B: "bfloat16"}

    def __init__(self, nx, ny, nz, dtype=CROFT_C64, dir=CROFT_FORWARD, flags=0, slabs=1):
        self.shape = (nz, ny, nx)
        self.dtype = dtype
        self.handle = croft_plan_create_ex(nx, ny, nz, dtype, dir, flags, slabs)

    def _check_tensor(self, t, name):
        want = self.shape if self.dtype in (CROFT_C64, CROFT_C128) else self.shape + (2,)
        if tuple(t.shape) != want:
            raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {want}")
        if str(t.dtype).replace("torch.", "") != self._TORCH[self.dtype]:
            raise ValueError(f"{name}: dtype {t.dtype}, expected {self._TORCH[self.dtype]}")
        if not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"{name}: must be a contiguous device tensor")

    def __call__(self, inp, out, stream=None):
        self._check_tensor(inp, "in")
        self._check_tensor(out, "out")
        croft_execute(self.handle, inp, out, stream)
        return out

    def scaled(self, inp, in_exp, out, out_exp, stream=None):
        self._check_tensor(inp, "in")
        self._check_tensor(out, "out")
        nz, ny, nx = self.shape
        if in_exp is not None and in_exp.numel() != ny * nz:
            raise ValueError("in_exp must hold ny*nz exponents")
        if out_exp.numel() != nx * ny:
            raise ValueError("out_exp must hold nx*ny exponents")
        croft_execute_scaled(self.handle, inp, in_exp, out, out_exp, stream)
        return out, out_exp

    def info(self) -> dict:
        return croft_plan_info(self.handle)

    def destroy(self):
        if self.handle:
            croft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _check_tensor(t, name, shape, dtype_name):
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if str(t.dtype).replace("torch.", "") != dtype_name:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype_name}")
    if not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError(f"{name}: must be a contiguous device tensor")


class RealPlan:
    """Owning wrapper of croft_plan_create_real: ``RealPlan(nx, ny, nz, dtype, dir)``.

    Forward: ``plan(x, y)`` with x real (nz, ny, nx) and y complex
    (nz, ny, nx//2 + 1); backward the other way round.  float32/complex64 for
    CROFT_C64, float64/complex128 for CROFT_C128.
    """

    _REAL = {CROFT_C64: "float32", CROFT_C128: "float64"}
    _CPLX = {CROFT_C64: "complex64", CROFT_C128: "complex128"}

    def __init__(self, nx, ny, nz, dtype=CROFT_C64, dir=CROFT_FORWARD, flags=0):
        self.real_shape = (nz, ny, nx)
        self.spec_shape = (nz, ny, nx // 2 + 1)
        self.dtype, self.dir = dtype, dir
        self.handle = croft_plan_create_real(nx, ny, nz, dtype, dir, flags)

    def __call__(self, inp, out, stream=None):
        r = (self.real_shape, self._REAL[self.dtype])
        c = (self.spec_shape, self._CPLX[self.dtype])
        (si, di), (so, do) = (r, c) if self.dir == CROFT_FORWARD else (c, r)
        _check_tensor(inp, "in", si, di)
        _check_tensor(out, "out", so, do)
        croft_execute(self.handle, inp, out, stream)
        return out

    def info(self) -> dict:
        return croft_plan_info(self.handle)

    def destroy(self):
        if self.handle:
            croft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class ConvolutionPlan:
    """Owning wrapper of croft_plan_create_convolution:
    ``ConvolutionPlan(nx, ny, nz, dtype)``; ``plan(x, g, out, energy=None)``
    with x and out real (nz, ny, nx), g real (nz, ny, nx//2 + 1) and energy a
    one-element float64 device tensor or None."""

    _REAL = {CROFT_C64: "float32", CROFT_C128: "float64"}

    def __init__(self, nx, ny, nz, dtype=CROFT_C64, flags=0):
        self.real_shape = (nz, ny, nx)
        self.spec_shape = (nz, ny, nx // 2 + 1)
        self.dtype = dtype
        self.handle = croft_plan_create_convolution(nx, ny, nz, dtype, flags)

    def __call__(self, inp, mul, out, energy=None, stream=None):
        _check_tensor(inp, "in", self.real_shape, self._REAL[self.dtype])
        _check_tensor(mul, "mul", self.spec_shape, self._REAL[self.dtype])
        _check_tensor(out, "out", self.real_shape, self._REAL[self.dtype])
        if energy is not None:
            _check_tensor(energy, "energy", (1,), "float64")
        croft_execute_convolution(self.handle, inp, mul, out, energy, stream)
        return out

    def info(self) -> dict:
        return croft_plan_info(self.handle)

    def destroy(self):
        if self.handle:
            croft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
