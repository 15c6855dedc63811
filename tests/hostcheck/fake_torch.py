"""The few torch calls the GPU tests make, over the host-only HIP stand-in.

Installed as ``torch`` in the sanitizer runs of the GPU tests: "cuda"
tensors are allocations of the stand-in's device memory (inaccessible to
host code except through its copies), CPU tensors are numpy arrays.  It
covers what the tests and the binding use (creation, slicing, copies to and
from the host, views), nothing more.
"""
from __future__ import annotations

import builtins
import ctypes
import math
import types

import numpy as np

_L = None
H2D, D2H, D2D = 1, 2, 3

int32 = np.dtype(np.int32)
int64 = np.dtype(np.int64)
uint8 = np.dtype(np.uint8)
float32 = np.dtype(np.float32)
float64 = np.dtype(np.float64)
bfloat16 = np.dtype(np.uint16)
int = int32          # noqa: A001  (torch's names)
long = int64
float = float32      # noqa: A001
double = float64
bool = np.dtype(np.bool_)   # noqa: A001


def bind(lib):
    global _L
    _L = lib
    lib.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    lib.hipFree.argtypes = [ctypes.c_void_p]
    lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    lib.hipMemset.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]
    lib.hostcheck_device_bytes.restype = ctypes.c_size_t


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with {rc}")


class _Block:
    """One device allocation, freed when the last tensor on it goes."""

    def __init__(self, nbytes):
        p = ctypes.c_void_p()
        _check(_L.hipMalloc(ctypes.byref(p), max(nbytes, 1)), "hipMalloc")
        self.ptr = p.value

    def __del__(self):
        if _L is not None and self.ptr:
            _L.hipFree(ctypes.c_void_p(self.ptr))
            self.ptr = None


class HostTensor(np.ndarray):
    is_cuda = False

    def numpy(self):
        return np.asarray(self)

    def cpu(self):
        return self

    def cuda(self):
        return DevTensor._from_host(np.ascontiguousarray(np.asarray(self)))

    def numel(self):
        return self.size

    def is_contiguous(self):
        return self.flags.c_contiguous

    def data_ptr(self):
        return self.ctypes.data

    def allclose(self, other, rtol=1e-5, atol=1e-8):
        return np.allclose(np.asarray(self), np.asarray(other), rtol=rtol, atol=atol)

    def float(self):
        return np.asarray(self, np.float32).view(HostTensor)

    def double(self):
        return np.asarray(self, np.float64).view(HostTensor)

    def long(self):
        return np.asarray(self, np.int64).view(HostTensor)


def _host(a):
    return np.asarray(a).view(HostTensor)


def _shape(size):
    if len(size) == 1 and isinstance(size[0], (tuple, list)):
        size = tuple(size[0])
    return tuple(builtins.int(s) for s in size)


def _is_dev(device):
    return device is not None and str(device).startswith("cuda")


class DevTensor:
    is_cuda = True

    def __init__(self, shape, dtype, block=None, offset=0):
        self.shape = tuple(builtins.int(s) for s in shape)
        self.dtype = np.dtype(dtype)
        self._block = block if block is not None else _Block(self.nbytes)
        self._off = offset

    # -- geometry
    @property
    def nbytes(self):
        return math.prod(self.shape) * self.dtype.itemsize

    def numel(self):
        return math.prod(self.shape)

    def dim(self):
        return len(self.shape)

    def size(self, i=None):
        return self.shape if i is None else self.shape[i]

    def element_size(self):
        return self.dtype.itemsize

    def __len__(self):
        return self.shape[0]

    def is_contiguous(self):
        return True

    def data_ptr(self):
        return self._block.ptr + self._off

    # -- copies
    @staticmethod
    def _from_host(a):
        t = DevTensor(a.shape, a.dtype)
        if a.nbytes:
            _check(_L.hipMemcpy(ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(a.ctypes.data), a.nbytes, H2D),
                   "hipMemcpy H2D")
        return t

    def cpu(self):
        out = np.empty(self.shape, self.dtype)
        if out.nbytes:
            _check(_L.hipMemcpy(ctypes.c_void_p(out.ctypes.data), ctypes.c_void_p(self.data_ptr()), out.nbytes,
                                D2H), "hipMemcpy D2H")
        return out.view(HostTensor)

    def cuda(self):
        return self

    def numpy(self):
        raise TypeError("can't convert a cuda tensor to numpy; call .cpu() first")

    def tolist(self):
        return self.cpu().tolist()

    def item(self):
        return self.cpu().item()

    def sum(self, *a, **k):
        return self.cpu().sum(*a, **k)

    def clone(self):
        return DevTensor._from_host(np.ascontiguousarray(self.cpu()))

    def copy_(self, src):
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(src.cpu() if isinstance(src, DevTensor) else src,
                                                            self.dtype), self.shape))
        if a.nbytes:
            _check(_L.hipMemcpy(ctypes.c_void_p(self.data_ptr()), ctypes.c_void_p(a.ctypes.data), a.nbytes, H2D),
                   "hipMemcpy H2D")
        return self

    def fill_(self, v):
        return self.copy_(np.full(self.shape, v, self.dtype))

    def zero_(self):
        if self.nbytes:
            _check(_L.hipMemset(ctypes.c_void_p(self.data_ptr()), 0, self.nbytes), "hipMemset")
        return self

    def float(self):
        return DevTensor._from_host(np.ascontiguousarray(self.cpu(), np.float32))

    def long(self):
        return DevTensor._from_host(np.ascontiguousarray(self.cpu(), np.int64))

    # -- views
    def _row_bytes(self):
        return math.prod(self.shape[1:]) * self.dtype.itemsize

    def __getitem__(self, key):
        if isinstance(key, slice):
            start, stop, step = key.indices(self.shape[0])
            if step != 1:
                raise NotImplementedError("strided device slices")
            n = max(0, stop - start)
            return DevTensor((n,) + self.shape[1:], self.dtype, self._block, self._off + start * self._row_bytes())
        if isinstance(key, (builtins.int, np.integer)):
            k = builtins.int(key)
            if k < 0:
                k += self.shape[0]
            if not 0 <= k < self.shape[0]:
                raise IndexError(key)
            return DevTensor(self.shape[1:], self.dtype, self._block, self._off + k * self._row_bytes())
        raise NotImplementedError(f"device index {key!r}")

    def __setitem__(self, key, value):
        self[key].copy_(value)

    def view(self, *args):
        if len(args) == 1 and not isinstance(args[0], (tuple, list, builtins.int)):
            dt = np.dtype(args[0])
            last = self.shape[-1] * self.dtype.itemsize // dt.itemsize
            return DevTensor(self.shape[:-1] + (last,), dt, self._block, self._off)
        return self.reshape(*args)

    def reshape(self, *shape):
        if len(shape) == 1 and isinstance(shape[0], (tuple, list)):
            shape = tuple(shape[0])
        shape = list(builtins.int(s) for s in shape)
        if -1 in shape:
            i = shape.index(-1)
            rest = math.prod(s for j, s in enumerate(shape) if j != i)
            shape[i] = self.numel() // rest
        return DevTensor(tuple(shape), self.dtype, self._block, self._off)

    def __repr__(self):
        return f"DevTensor(shape={self.shape}, dtype={self.dtype}, ptr={self.data_ptr():#x})"


Tensor = DevTensor


def _make(shape, dtype, device, fill):
    shape = _shape(shape)
    dtype = np.dtype(dtype if dtype is not None else np.float32)
    if not _is_dev(device):
        return _host(np.full(shape, fill, dtype) if fill is not None else np.zeros(shape, dtype))
    t = DevTensor(shape, dtype)
    if fill is None or fill == 0:
        t.zero_()
    else:
        t.fill_(fill)
    return t


def zeros(*size, dtype=None, device=None):
    return _make(size, dtype, device, 0)


def ones(*size, dtype=None, device=None):
    return _make(size, dtype, device, 1)


def empty(*size, dtype=None, device=None):
    # "empty" device memory is left as the stand-in hands it out (zeros)
    shape = _shape(size)
    dtype = np.dtype(dtype if dtype is not None else np.float32)
    return DevTensor(shape, dtype) if _is_dev(device) else _host(np.empty(shape, dtype))


def full(size, value, dtype=None, device=None):
    return _make((size,) if not isinstance(size, (tuple, list)) else tuple(size), dtype, device, value)


def zeros_like(t, dtype=None, device=None):
    dev = device if device is not None else ("cuda" if isinstance(t, DevTensor) else None)
    return zeros(*t.shape, dtype=dtype or t.dtype, device=dev)


def from_numpy(a):
    return np.asarray(a).view(HostTensor)


def equal(a, b):
    a = a.cpu() if isinstance(a, DevTensor) else a
    b = b.cpu() if isinstance(b, DevTensor) else b
    return np.array_equal(np.asarray(a), np.asarray(b))


def manual_seed(_):
    return None


class _Stream:
    cuda_stream = 0


def _synchronize():
    _check(_L.hipDeviceSynchronize(), "hipDeviceSynchronize")


cuda = types.SimpleNamespace(
    is_available=lambda: True,
    device_count=lambda: 1,
    set_device=lambda i: None,
    current_device=lambda: 0,
    synchronize=_synchronize,
    current_stream=lambda *a: _Stream(),
    empty_cache=lambda: None,
)
