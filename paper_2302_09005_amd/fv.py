"""Python binding of the C ABI in include/fv.h (argument marshalling only).

Every function here forwards to libfv.so (HIP kernels for gfx950) with device
pointers taken from torch tensors and the current torch stream; no step of the
update runs in Python or on the CPU.  If the library is missing, every call
raises: there is no fallback.

Tensors: solution buffers are contiguous float64 CUDA (HIP) tensors of any
shape (they are flat arrays of patch blocks); descriptors are a device tensor
holding ``workloads.PATCH_DTYPE`` records (see :func:`upload_patches`);
neighbour tables are int64 device tensors of shape [n, 2*dim].
"""
import ctypes
import os

import numpy as np

from .workloads import PATCH_DTYPE

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libfv.so")

FV_OK = 0
FV_EINVAL = -1
FV_EUNSUPPORTED = -2
FV_EHIP = -3
FV_OFFSETS_IN = 0
FV_OFFSETS_OUT = 1

_lib = None


class FVError(RuntimeError):
    """A libfv call returned a non-zero status."""

    def __init__(self, code, msg):
        super().__init__(f"libfv error {code}: {msg}")
        self.code = code


def library():
    """Load libfv.so (built by ``python -m paper_2302_09005_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FVError(FV_EHIP, f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2302_09005_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.fv_last_error.argtypes = []
    lib.fv_last_error.restype = ctypes.c_char_p
    lib.fv_abi_version.argtypes = []
    lib.fv_abi_version.restype = i32
    lib.fv_supported.argtypes = [i32, i32]
    lib.fv_supported.restype = i32
    lib.fv_check_patches.argtypes = [vp, i64, i32, i32, i32, i64, i64]
    lib.fv_check_patches.restype = i32
    lib.fv_batch_update.argtypes = [vp, i64, vp, i64, vp, i64, i32, i32, i32, i32, i32, f64,
                                    vp, vp, vp]
    lib.fv_batch_update.restype = i32
    lib.fv_max_eigenvalue.argtypes = [vp, i64, vp, i64, i32, i32, i32, i32, i32, f64, vp, vp, vp]
    lib.fv_max_eigenvalue.restype = i32
    lib.fv_cfl_timestep.argtypes = [vp, i64, vp, i32, f64, vp, vp, vp]
    lib.fv_cfl_timestep.restype = i32
    lib.fv_fill_halo.argtypes = [vp, i64, vp, vp, i64, i32, i32, i32, i32, i32, vp]
    lib.fv_fill_halo.restype = i32
    _lib = lib
    return lib


def _check(rc):
    if rc != FV_OK:
        raise FVError(rc, library().fv_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 device tensor")
    return t


def _n_patches(patches):
    nbytes = patches.numel() * patches.element_size()
    if nbytes % PATCH_DTYPE.itemsize:
        raise ValueError("descriptor tensor size is not a multiple of 64 bytes")
    return nbytes // PATCH_DTYPE.itemsize


def abi_version():
    return library().fv_abi_version()


def supported(dim, p):
    return bool(library().fv_supported(dim, p))


def check_patches(desc, dim, p, q_out_halo, q_in_len, q_out_len):
    """Validate a host descriptor array (numpy, PATCH_DTYPE) with fv_check_patches."""
    desc = np.ascontiguousarray(desc, dtype=PATCH_DTYPE)
    _check(library().fv_check_patches(desc.ctypes.data_as(ctypes.c_void_p), desc.shape[0],
                                      dim, p, int(bool(q_out_halo)), int(q_in_len),
                                      int(q_out_len)))


def upload_patches(desc, device="cuda", *, dim=None, p=None, q_out_halo=None, q_in_len=None,
                   q_out_len=None):
    """Copy a host descriptor array to the device (as a uint8 tensor).

    When dim/p/lengths are given the array is validated first with
    fv_check_patches.
    """
    import torch
    desc = np.ascontiguousarray(desc, dtype=PATCH_DTYPE)
    if dim is not None:
        check_patches(desc, dim, p, q_out_halo, q_in_len, q_out_len)
    raw = torch.from_numpy(desc.view(np.uint8).reshape(-1).copy())
    return raw.to(device)


def batch_update(patches, q_in, q_out, *, dim, p, gamma=1.4, q_out_halo=True, dt=None,
                 max_eig=None, stream=None):
    """fv_batch_update: one explicit Euler step of every patch (see include/fv.h)."""
    _dev_f64(q_in, "q_in")
    _dev_f64(q_out, "q_out")
    if max_eig is not None:
        _dev_f64(max_eig, "max_eig")
    if dt is not None:
        _dev_f64(dt, "dt")
    n = _n_patches(patches)
    if max_eig is not None and max_eig.numel() < n:
        raise ValueError("max_eig needs one entry per patch")
    _check(library().fv_batch_update(_ptr(patches), n, _ptr(q_in), q_in.numel(), _ptr(q_out),
                                     q_out.numel(), int(bool(q_out_halo)), dim, p, 1, dim + 2,
                                     float(gamma), _ptr(dt), _ptr(max_eig), _stream(stream)))


def max_eigenvalue(patches, q, per_patch, global_out=None, *, dim, p, gamma=1.4, q_halo=True,
                   which=FV_OFFSETS_IN, stream=None):
    """fv_max_eigenvalue: per-patch (and optionally global) largest eigenvalue of q."""
    _dev_f64(q, "q")
    _dev_f64(per_patch, "per_patch")
    if global_out is not None:
        _dev_f64(global_out, "global_out")
    n = _n_patches(patches)
    if per_patch.numel() < n:
        raise ValueError("per_patch needs one entry per patch")
    _check(library().fv_max_eigenvalue(_ptr(patches), n, _ptr(q), q.numel(), int(bool(q_halo)),
                                       which, dim, p, dim + 2, float(gamma), _ptr(per_patch),
                                       _ptr(global_out), _stream(stream)))


def cfl_timestep(patches, per_patch, *, dim, cfl=0.4, lambda_out=None, dt_out=None,
                 stream=None):
    """fv_cfl_timestep: Lambda and dt = cfl * min dx / (dim * Lambda) on the device."""
    _dev_f64(per_patch, "per_patch")
    n = _n_patches(patches)
    for t, name in ((lambda_out, "lambda_out"), (dt_out, "dt_out")):
        if t is not None:
            _dev_f64(t, name)
    _check(library().fv_cfl_timestep(_ptr(patches), n, _ptr(per_patch), dim, float(cfl),
                                     _ptr(lambda_out), _ptr(dt_out), _stream(stream)))


def fill_halo(patches, neighbours, q, *, dim, p, which=FV_OFFSETS_IN, stream=None):
    """fv_fill_halo: face-halo exchange in place (neighbour -1 = transmissive)."""
    import torch
    _dev_f64(q, "q")
    n = _n_patches(patches)
    if not (neighbours.is_cuda and neighbours.dtype == torch.int64 and neighbours.is_contiguous()
            and neighbours.numel() == 2 * dim * n):
        raise TypeError("neighbours must be a contiguous int64 device tensor [n, 2*dim]")
    _check(library().fv_fill_halo(_ptr(patches), n, _ptr(neighbours), _ptr(q), q.numel(), which,
                                  dim, p, 1, dim + 2, _stream(stream)))


class Stepper:
    """Device-resident multi-step driver over one patch batch (halo'd ping-pong).

    Each step: dt from the current per-patch maxima (fv_cfl_timestep), update
    into the other buffer (fv_batch_update, which also yields the next per-patch
    maxima), face-halo fill (fv_fill_halo), swap.  Nothing leaves the device.
    """

    def __init__(self, desc, neighbours, q0, *, dim, p, gamma=1.4, cfl=0.4, device="cuda"):
        import torch
        desc = np.ascontiguousarray(desc, dtype=PATCH_DTYPE)
        if not np.array_equal(desc["q_in"], desc["q_out"]):
            raise ValueError("the ping-pong stepper needs q_in == q_out offsets")
        q0 = np.ascontiguousarray(q0, dtype=np.float64)
        self.dim, self.p, self.gamma, self.cfl = dim, p, gamma, cfl
        self.n = desc.shape[0]
        self.patches = upload_patches(desc, device, dim=dim, p=p, q_out_halo=True,
                                      q_in_len=q0.size, q_out_len=q0.size)
        self.neighbours = torch.from_numpy(np.ascontiguousarray(neighbours, np.int64)).to(device)
        self.a = torch.from_numpy(q0).to(device)
        self.b = self.a.clone()
        self.per_patch = torch.empty(self.n, dtype=torch.float64, device=device)
        self.lam = torch.empty(1, dtype=torch.float64, device=device)
        self.dt = torch.empty(1, dtype=torch.float64, device=device)
        max_eigenvalue(self.patches, self.a, self.per_patch, dim=dim, p=p, gamma=gamma)

    def step(self, stream=None):
        cfl_timestep(self.patches, self.per_patch, dim=self.dim, cfl=self.cfl,
                     lambda_out=self.lam, dt_out=self.dt, stream=stream)
        batch_update(self.patches, self.a, self.b, dim=self.dim, p=self.p, gamma=self.gamma,
                     q_out_halo=True, dt=self.dt, max_eig=self.per_patch, stream=stream)
        fill_halo(self.patches, self.neighbours, self.b, dim=self.dim, p=self.p, stream=stream)
        self.a, self.b = self.b, self.a

    def state(self):
        return self.a
