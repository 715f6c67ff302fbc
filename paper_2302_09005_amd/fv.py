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
FV_SCHED_PER_SIZE = 0
FV_SCHED_PERSISTENT = 1
FV_SCHED_PATCHWISE = 2
SCHEDULES = {"per_size": FV_SCHED_PER_SIZE, "persistent": FV_SCHED_PERSISTENT,
             "patchwise": FV_SCHED_PATCHWISE}


class WorkUnit(ctypes.Structure):
    """fv_work_unit (include/fv.h)."""
    _fields_ = [("p", ctypes.c_int32), ("count", ctypes.c_int32), ("first", ctypes.c_int64)]


class MixedPlan(ctypes.Structure):
    """fv_mixed_plan (include/fv.h)."""
    _fields_ = [("order", ctypes.c_void_p), ("units", ctypes.c_void_p),
                ("n_units", ctypes.c_int64), ("class_p", ctypes.c_int32 * 3),
                ("class_first", ctypes.c_int64 * 3), ("class_count", ctypes.c_int64 * 3)]

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
    # torch's wheel ships its own HIP runtime under the same soname
    # (libamdhip64.so.7).  Loaded after torch, libfv binds to that copy, so the
    # process has one HIP runtime and torch's device memory and streams are
    # valid in libfv's calls.  Loaded before torch, the dynamic linker would
    # map the system copy as well, and the two runtimes do not share devices.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.fv_last_error.argtypes = []
    lib.fv_last_error.restype = ctypes.c_char_p
    lib.fv_abi_version.argtypes = []
    lib.fv_abi_version.restype = i32
    lib.fv_supported.argtypes = [i32, i32]
    lib.fv_supported.restype = i32
    lib.fv_set_launch_events.argtypes = [vp, vp]
    lib.fv_set_launch_events.restype = i32
    lib.fv_check_patches.argtypes = [vp, i64, i32, i32, i32, i32, i64, i64]
    lib.fv_check_patches.restype = i32
    lib.fv_batch_update.argtypes = [vp, i64, vp, i64, vp, i64, i32, i32, i32, i32, i32, f64,
                                    vp, vp, vp]
    lib.fv_batch_update.restype = i32
    lib.fv_batch_update_gather.argtypes = [vp, i64, vp, vp, i64, vp, i64, i32, i32, i32, i32,
                                           f64, vp, vp, vp]
    lib.fv_batch_update_gather.restype = i32
    lib.fv_step_gather.argtypes = [vp, i64, vp, vp, i64, vp, i64, i32, i32, i32, f64, f64, vp, vp,
                                   vp, vp, vp, i64, vp]
    lib.fv_step_gather.restype = i32
    lib.fv_step_halo.argtypes = [vp, i64, vp, vp, i64, vp, i64, i32, i32, i32, i32, f64, f64, vp,
                                 vp, vp, vp, vp, i64, vp]
    lib.fv_step_halo.restype = i32
    lib.fv_step_gather_pipelined.argtypes = [vp, i64, vp, vp, i64, vp, i64, i32, i32, i32, f64,
                                             f64, i32, vp, vp, vp, vp, vp, i64, vp]
    lib.fv_step_gather_pipelined.restype = i32
    lib.fv_step_gather_pipelined_f32.argtypes = lib.fv_step_gather_pipelined.argtypes
    lib.fv_step_gather_pipelined_f32.restype = i32
    lib.fv_step_pipelined_workspace_words.argtypes = [i64, i32, i32]
    lib.fv_step_pipelined_workspace_words.restype = i64
    lib.fv_step_gather_noalloc.argtypes = lib.fv_step_gather.argtypes[:-3] + [vp]
    lib.fv_step_gather_noalloc.restype = i32
    lib.fv_step_workspace_words.argtypes = [i64, i32, i32]
    lib.fv_step_workspace_words.restype = i64
    lib.fv_max_eigenvalue.argtypes = [vp, i64, vp, i64, i32, i32, i32, i32, i32, f64, vp, vp, vp]
    lib.fv_max_eigenvalue.restype = i32
    for base in ("fv_batch_update", "fv_batch_update_gather", "fv_step_gather",
                 "fv_max_eigenvalue"):
        f32 = getattr(lib, base + "_f32")
        f32.argtypes = getattr(lib, base).argtypes
        f32.restype = i32
    for name in ("fv_conserved_totals", "fv_conserved_totals_f32"):
        getattr(lib, name).argtypes = [vp, i64, vp, i64, i32, i32, i32, i32, i32, vp, vp, vp]
        getattr(lib, name).restype = i32
    lib.fv_plan_mixed.argtypes = [vp, i64, i32, vp, vp, ctypes.POINTER(MixedPlan)]
    lib.fv_plan_mixed.restype = i32
    for name in ("fv_step_local", "fv_step_local_f32"):
        getattr(lib, name).argtypes = [vp, i64, vp, ctypes.POINTER(MixedPlan), vp, i64, vp, i64,
                                       i32, i32, f64, f64, vp, i32, i32, vp]
        getattr(lib, name).restype = i32
    lib.fv_local_timestep.argtypes = [vp, i64, vp, i32, f64, vp]
    lib.fv_local_timestep.restype = i32
    lib.fv_learned_flux_accumulate.argtypes = [vp, i32, i32, i32, i32, i32, f64, f64, vp, vp,
                                               vp]
    lib.fv_learned_coarse_grain.argtypes = [vp, i32, i32, i32, i32, vp, vp]
    lib.fv_learned_face_samples.argtypes = [vp, i32, i32, i32, i32, f64, vp, vp, vp, vp, vp, vp]
    lib.fv_mlp_fit_normalization.argtypes = [vp, i64, i32, i32, vp, i64, vp, vp, vp]
    lib.fv_mlp_workspace_words.argtypes = [i32]
    lib.fv_mlp_train_step.argtypes = [vp, vp, i32, ctypes.c_float, vp, vp, i64, vp, i32, vp, i64,
                                      vp, vp]
    lib.fv_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
    lib.fv_batch_update_learned_2d.argtypes = [vp, i64, vp, vp, i64, vp, i64, f64, vp, vp, f64,
                                               vp, vp]
    for name in ("fv_learned_flux_accumulate", "fv_learned_coarse_grain",
                 "fv_learned_face_samples", "fv_mlp_fit_normalization", "fv_mlp_workspace_words",
                 "fv_mlp_train_step", "fv_mlp_forward", "fv_batch_update_learned_2d"):
        getattr(lib, name).restype = i32
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


def _dev_state(t, name):
    """A solution buffer: float64 or float32; returns the entry-point suffix."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()
            and t.dtype in (torch.float64, torch.float32)):
        raise TypeError(f"{name} must be a contiguous float64 or float32 device tensor")
    return "" if t.dtype == torch.float64 else "_f32"


def _same_state(a, b):
    sa, sb = _dev_state(a, "q_in"), _dev_state(b, "q_out")
    if sa != sb:
        raise TypeError("q_in and q_out must have the same dtype")
    return sa


def _n_patches(patches):
    nbytes = patches.numel() * patches.element_size()
    if nbytes % PATCH_DTYPE.itemsize:
        raise ValueError("descriptor tensor size is not a multiple of 64 bytes")
    return nbytes // PATCH_DTYPE.itemsize


def set_launch_events(start=None, stop=None):
    """fv_set_launch_events: raw hipEvent_t handles (ints) recorded by the
    dispatch of the following update launches; None, None to stop."""
    _check(library().fv_set_launch_events(start, stop))


def abi_version():
    return library().fv_abi_version()


def supported(dim, p):
    return bool(library().fv_supported(dim, p))


def check_patches(desc, dim, p, q_out_halo, q_in_len, q_out_len, q_in_halo=True):
    """Validate a host descriptor array (numpy, PATCH_DTYPE) with fv_check_patches."""
    desc = np.ascontiguousarray(desc, dtype=PATCH_DTYPE)
    _check(library().fv_check_patches(desc.ctypes.data_as(ctypes.c_void_p), desc.shape[0],
                                      dim, p, int(bool(q_in_halo)), int(bool(q_out_halo)),
                                      int(q_in_len), int(q_out_len)))


def upload_patches(desc, device="cuda", *, dim=None, p=None, q_out_halo=None, q_in_len=None,
                   q_out_len=None, q_in_halo=True):
    """Copy a host descriptor array to the device (as a uint8 tensor).

    When dim/p/lengths are given the array is validated first with
    fv_check_patches.
    """
    import torch
    desc = np.ascontiguousarray(desc, dtype=PATCH_DTYPE)
    if dim is not None:
        check_patches(desc, dim, p, q_out_halo, q_in_len, q_out_len, q_in_halo)
    raw = torch.from_numpy(desc.view(np.uint8).reshape(-1).copy())
    return raw.to(device)


def batch_update(patches, q_in, q_out, *, dim, p, gamma=1.4, q_out_halo=True, dt=None,
                 max_eig=None, stream=None):
    """fv_batch_update[_f32]: one explicit Euler step of every patch (see include/fv.h)."""
    sfx = _same_state(q_in, q_out)
    if max_eig is not None:
        _dev_f64(max_eig, "max_eig")
    if dt is not None:
        _dev_f64(dt, "dt")
    n = _n_patches(patches)
    if max_eig is not None and max_eig.numel() < n:
        raise ValueError("max_eig needs one entry per patch")
    fn = getattr(library(), "fv_batch_update" + sfx)
    _check(fn(_ptr(patches), n, _ptr(q_in), q_in.numel(), _ptr(q_out), q_out.numel(),
              int(bool(q_out_halo)), dim, p, 1, dim + 2, float(gamma), _ptr(dt), _ptr(max_eig),
              _stream(stream)))


def _dev_nbr(neighbours, n, dim):
    import torch
    if not (isinstance(neighbours, torch.Tensor) and neighbours.is_cuda
            and neighbours.dtype == torch.int64 and neighbours.is_contiguous()
            and neighbours.numel() == 2 * dim * n):
        raise TypeError("neighbours must be a contiguous int64 device tensor [n, 2*dim]")
    return neighbours


def batch_update_gather(patches, neighbours, q_in, q_out, *, dim, p, gamma=1.4,
                        q_out_halo=False, dt=None, max_eig=None, stream=None):
    """fv_batch_update_gather[_f32]: update with the face-halo exchange fused into the gather."""
    sfx = _same_state(q_in, q_out)
    if max_eig is not None:
        _dev_f64(max_eig, "max_eig")
    if dt is not None:
        _dev_f64(dt, "dt")
    n = _n_patches(patches)
    _dev_nbr(neighbours, n, dim)
    if max_eig is not None and max_eig.numel() < n:
        raise ValueError("max_eig needs one entry per patch")
    fn = getattr(library(), "fv_batch_update_gather" + sfx)
    _check(fn(_ptr(patches), n, _ptr(neighbours), _ptr(q_in), q_in.numel(), _ptr(q_out),
              q_out.numel(), int(bool(q_out_halo)), dim, p, dim + 2, float(gamma), _ptr(dt),
              _ptr(max_eig), _stream(stream)))


def step_workspace_words(n, dim, p):
    """Words of the zero-initialised int64 workspace fv_step_gather needs."""
    return int(library().fv_step_workspace_words(n, dim, p))


def step_gather(patches, neighbours, q_in, q_out, dt, dt_next, workspace, *, dim, p, gamma=1.4,
                cfl=0.4, max_eig=None, lambda_out=None, stream=None):
    """fv_step_gather[_f32]: update (halo exchange fused) + next CFL time step, one launch."""
    import torch
    sfx = _same_state(q_in, q_out)
    _dev_f64(dt, "dt")
    _dev_f64(dt_next, "dt_next")
    for t, name in ((max_eig, "max_eig"), (lambda_out, "lambda_out")):
        if t is not None:
            _dev_f64(t, name)
    n = _n_patches(patches)
    need = step_workspace_words(n, dim, p)
    if not (workspace.is_cuda and workspace.dtype in (torch.int64, torch.uint64)
            and workspace.numel() >= need and workspace.is_contiguous()):
        raise TypeError(f"workspace must be a contiguous 64-bit integer device tensor of "
                        f">= {need} words")
    _dev_nbr(neighbours, n, dim)
    if max_eig is not None and max_eig.numel() < n:
        raise ValueError("max_eig needs one entry per patch")
    fn = getattr(library(), "fv_step_gather" + sfx)
    _check(fn(_ptr(patches), n, _ptr(neighbours), _ptr(q_in), q_in.numel(), _ptr(q_out),
              q_out.numel(), dim, p, dim + 2, float(gamma), float(cfl), _ptr(dt), _ptr(max_eig),
              _ptr(dt_next), _ptr(lambda_out), _ptr(workspace), workspace.numel(),
              _stream(stream)))


def pipelined_workspace_words(n, dim, p):
    """Words of the zero-initialised int64 workspace fv_step_gather_pipelined needs."""
    return int(library().fv_step_pipelined_workspace_words(n, dim, p))


def _pipelined_args(patches, neighbours, q_in, q_out, workspace, dim, p, gamma, cfl, phase,
                    dt_in, dt_used, max_eig, lambda_out):
    """Checks the arguments of fv_step_gather_pipelined[_f32]; returns the
    entry point and its argument tuple (without the stream)."""
    import torch
    sfx = _same_state(q_in, q_out)
    for t, name in ((dt_in, "dt_in"), (dt_used, "dt_used"), (max_eig, "max_eig"),
                    (lambda_out, "lambda_out")):
        if t is not None:
            _dev_f64(t, name)
    if phase not in (0, 1, 2):
        raise ValueError("phase must be 0, 1 or 2")
    n = _n_patches(patches)
    need = pipelined_workspace_words(n, dim, p)
    if not (workspace.is_cuda and workspace.dtype in (torch.int64, torch.uint64)
            and workspace.numel() >= need and workspace.is_contiguous()):
        raise TypeError(f"workspace must be a contiguous 64-bit integer device tensor of "
                        f">= {need} words")
    _dev_nbr(neighbours, n, dim)
    if max_eig is not None and max_eig.numel() < n:
        raise ValueError("max_eig needs one entry per patch")
    fn = getattr(library(), "fv_step_gather_pipelined" + sfx)
    return fn, (_ptr(patches), n, _ptr(neighbours), _ptr(q_in), q_in.numel(), _ptr(q_out),
                q_out.numel(), dim, p, dim + 2, float(gamma), float(cfl), int(phase),
                _ptr(dt_in), _ptr(dt_used), _ptr(max_eig), _ptr(lambda_out), _ptr(workspace),
                workspace.numel())


def step_gather_pipelined(patches, neighbours, q_in, q_out, workspace, *, dim, p, phase,
                          dt_in=None, dt_used=None, gamma=1.4, cfl=0.4, max_eig=None,
                          lambda_out=None, stream=None):
    """fv_step_gather_pipelined[_f32]: the fused step with the CFL reduction
    done by the next call (phase 0, 1, 2, 0, ... over a run; dt_in on the
    first call only)."""
    fn, args = _pipelined_args(patches, neighbours, q_in, q_out, workspace, dim, p, gamma, cfl,
                               phase, dt_in, dt_used, max_eig, lambda_out)
    _check(fn(*args, _stream(stream)))


def step_halo(patches, neighbours, q_in, q_out, dt, dt_next, workspace, *, dim, p, gamma=1.4,
              cfl=0.4, max_eig=None, lambda_out=None, stream=None):
    """fv_step_halo: the paper's halo'd layout, update + face-halo exchange of
    the new state (pushed into the output halos) + next CFL step, one launch
    (float64 state; the neighbour table must be mutual)."""
    import torch
    if _same_state(q_in, q_out) != "":
        raise TypeError("fv_step_halo takes float64 state")
    _dev_f64(dt, "dt")
    _dev_f64(dt_next, "dt_next")
    for t, name in ((max_eig, "max_eig"), (lambda_out, "lambda_out")):
        if t is not None:
            _dev_f64(t, name)
    n = _n_patches(patches)
    need = step_workspace_words(n, dim, p)
    if not (workspace.is_cuda and workspace.dtype in (torch.int64, torch.uint64)
            and workspace.numel() >= need and workspace.is_contiguous()):
        raise TypeError(f"workspace must be a contiguous 64-bit integer device tensor of "
                        f">= {need} words")
    _dev_nbr(neighbours, n, dim)
    if max_eig is not None and max_eig.numel() < n:
        raise ValueError("max_eig needs one entry per patch")
    _check(library().fv_step_halo(
        _ptr(patches), n, _ptr(neighbours), _ptr(q_in), q_in.numel(), _ptr(q_out), q_out.numel(),
        dim, p, 1, dim + 2, float(gamma), float(cfl), _ptr(dt), _ptr(max_eig), _ptr(dt_next),
        _ptr(lambda_out), _ptr(workspace), workspace.numel(), _stream(stream)))


def step_gather_noalloc(patches, neighbours, q_in, q_out, dt, dt_next, *, dim, p, gamma=1.4,
                        cfl=0.4, max_eig=None, lambda_out=None, stream=None):
    """fv_step_gather_noalloc: fv_step_gather with the library's own scratch
    array as workspace (FP64 state; nothing is allocated on any call)."""
    if _same_state(q_in, q_out) != "":
        raise TypeError("fv_step_gather_noalloc takes float64 state")
    _dev_f64(dt, "dt")
    _dev_f64(dt_next, "dt_next")
    for t, name in ((max_eig, "max_eig"), (lambda_out, "lambda_out")):
        if t is not None:
            _dev_f64(t, name)
    n = _n_patches(patches)
    _dev_nbr(neighbours, n, dim)
    if max_eig is not None and max_eig.numel() < n:
        raise ValueError("max_eig needs one entry per patch")
    _check(library().fv_step_gather_noalloc(
        _ptr(patches), n, _ptr(neighbours), _ptr(q_in), q_in.numel(), _ptr(q_out), q_out.numel(),
        dim, p, dim + 2, float(gamma), float(cfl), _ptr(dt), _ptr(max_eig), _ptr(dt_next),
        _ptr(lambda_out), _stream(stream)))


def max_eigenvalue(patches, q, per_patch, global_out=None, *, dim, p, gamma=1.4, q_halo=True,
                   which=FV_OFFSETS_IN, stream=None):
    """fv_max_eigenvalue[_f32]: per-patch (and optionally global) largest eigenvalue of q."""
    sfx = _dev_state(q, "q")
    _dev_f64(per_patch, "per_patch")
    if global_out is not None:
        _dev_f64(global_out, "global_out")
    n = _n_patches(patches)
    if per_patch.numel() < n:
        raise ValueError("per_patch needs one entry per patch")
    fn = getattr(library(), "fv_max_eigenvalue" + sfx)
    _check(fn(_ptr(patches), n, _ptr(q), q.numel(), int(bool(q_halo)), which, dim, p, dim + 2,
              float(gamma), _ptr(per_patch), _ptr(global_out), _stream(stream)))


def conserved_totals(patches, q, per_patch, totals=None, *, dim, p, q_halo=True,
                     which=FV_OFFSETS_IN, stream=None):
    """fv_conserved_totals[_f32]: FP64 totals of the conserved unknowns (per patch, and summed)."""
    sfx = _dev_state(q, "q")
    _dev_f64(per_patch, "per_patch")
    if totals is not None:
        _dev_f64(totals, "totals")
    n = _n_patches(patches)
    if per_patch.numel() < n * (dim + 2):
        raise ValueError("per_patch needs (dim+2) entries per patch")
    _check(getattr(library(), "fv_conserved_totals" + sfx)(
        _ptr(patches), n, _ptr(q), q.numel(), int(bool(q_halo)), which, dim, p, dim + 2,
        _ptr(per_patch), _ptr(totals), _stream(stream)))


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
    _dev_f64(q, "q")
    n = _n_patches(patches)
    _dev_nbr(neighbours, n, dim)
    _check(library().fv_fill_halo(_ptr(patches), n, _ptr(neighbours), _ptr(q), q.numel(), which,
                                  dim, p, 1, dim + 2, _stream(stream)))


# ---------------------------------------------------------------------------
# Learned face-flux correction (2-D)
# ---------------------------------------------------------------------------
MLP_BLOB_WORDS = 5548
MLP_TRAINED_WORDS = 5508  # W1 .. b3
BLOB_OFFSETS = {"x_mean": 0, "x_scale": 16, "w1": 32, "b1": 1056, "w2": 1120, "b2": 5216,
                "w3": 5280, "b3": 5536, "y_scale": 5540, "y_mean": 5544}


def _dev_f32(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 device tensor")
    return t


def learned_flux_accumulate(q_fine, acc_x, acc_y, *, npx, npy, p=16, r=4, bc=0, weight=0.25,
                            gamma=1.4, stream=None):
    """fv_learned_flux_accumulate (see include/fv.h)."""
    _dev_f64(q_fine, "q_fine")
    _dev_f64(acc_x, "acc_x")
    _dev_f64(acc_y, "acc_y")
    ncx, ncy = npx * p // r, npy * p // r
    if acc_x.numel() != 4 * ncy * (ncx + 1) or acc_y.numel() != 4 * (ncy + 1) * ncx:
        raise ValueError("accumulator sizes do not match the coarse grid")
    if q_fine.numel() < npx * npy * 4 * p * p:
        raise ValueError("q_fine is smaller than the patch grid")
    _check(library().fv_learned_flux_accumulate(_ptr(q_fine), npx, npy, p, r, bc, float(gamma),
                                                float(weight), _ptr(acc_x), _ptr(acc_y),
                                                _stream(stream)))


def learned_coarse_grain(q_fine, q_coarse, *, npx, npy, p=16, r=4, stream=None):
    _dev_f64(q_fine, "q_fine")
    _dev_f64(q_coarse, "q_coarse")
    if q_fine.numel() < npx * npy * 4 * p * p or \
            q_coarse.numel() < (npx // r) * (npy // r) * 4 * p * p:
        raise ValueError("buffers smaller than the patch grids")
    _check(library().fv_learned_coarse_grain(_ptr(q_fine), npx, npy, p, r, _ptr(q_coarse),
                                             _stream(stream)))


def learned_face_samples(q_coarse, acc_x, acc_y, features, targets, indicator, *, npx, npy,
                         p=16, bc=0, gamma=1.4, stream=None):
    _dev_f64(q_coarse, "q_coarse")
    _dev_f64(acc_x, "acc_x")
    _dev_f64(acc_y, "acc_y")
    if acc_x.numel() != 4 * npy * p * (npx * p + 1) or acc_y.numel() != 4 * (npy * p + 1) * npx * p:
        raise ValueError("accumulator sizes do not match the grid")
    for t, name in ((features, "features"), (targets, "targets"), (indicator, "indicator")):
        _dev_f32(t, name)
    nx, ny = npx * p, npy * p
    nfaces = ny * (nx + 1) + (ny + 1) * nx
    if features.numel() < 16 * nfaces or targets.numel() < 4 * nfaces or \
            indicator.numel() < nfaces or q_coarse.numel() < npx * npy * 4 * p * p:
        raise ValueError("sample buffers too small")
    _check(library().fv_learned_face_samples(_ptr(q_coarse), npx, npy, p, bc, float(gamma),
                                             _ptr(acc_x), _ptr(acc_y), _ptr(features),
                                             _ptr(targets), _ptr(indicator), _stream(stream)))


def mlp_fit_normalization(x, cols, mean_out, scale_out, *, mode, rows=None, stream=None):
    _dev_f32(x, "x")
    x_rows = x.numel() // cols
    n = 0 if rows is None else rows.numel()
    _check(library().fv_mlp_fit_normalization(_ptr(x), x_rows, cols, mode, _ptr(rows), n,
                                              _ptr(mean_out), _ptr(scale_out), _stream(stream)))


def mlp_workspace_words(batch):
    return int(library().fv_mlp_workspace_words(batch))


def mlp_train_step(blob, adam, step, lr, features, targets, batch_idx, workspace, grad_out=None,
                   stream=None):
    _dev_f32(blob, "blob")
    _dev_f32(adam, "adam")
    _dev_f32(workspace, "workspace")
    if blob.numel() != MLP_BLOB_WORDS or adam.numel() < 2 * MLP_TRAINED_WORDS:
        raise ValueError("blob or adam state has the wrong size")
    if grad_out is not None and (_dev_f32(grad_out, "grad_out").numel() < MLP_TRAINED_WORDS):
        raise ValueError(f"grad_out needs {MLP_TRAINED_WORDS} words")
    _dev_f32(features, "features")
    _dev_f32(targets, "targets")
    n_rows = features.numel() // 16
    if targets.numel() < 4 * n_rows:
        raise ValueError("targets need 4 values per feature row")
    _check(library().fv_mlp_train_step(_ptr(blob), _ptr(adam), int(step), float(lr),
                                       _ptr(features), _ptr(targets), n_rows, _ptr(batch_idx),
                                       batch_idx.numel(), _ptr(workspace), workspace.numel(),
                                       _ptr(grad_out), _stream(stream)))


def mlp_forward(blob, features, out, stream=None):
    _dev_f32(blob, "blob")
    _dev_f32(features, "features")
    _dev_f32(out, "out")
    n = features.numel() // 16
    if out.numel() < 4 * n:
        raise ValueError("out needs 4 values per row")
    _check(library().fv_mlp_forward(_ptr(blob), _ptr(features), n, _ptr(out), _stream(stream)))


def batch_update_learned_2d(patches, neighbours, q_in, q_out, blob, *, gamma=1.4, dt=None,
                            threshold=0.2, max_eig=None, stream=None):
    """fv_batch_update_learned_2d: 16^2 patches, compact blocks, corrected fluxes."""
    _dev_f64(q_in, "q_in")
    _dev_f64(q_out, "q_out")
    _dev_f32(blob, "blob")
    if dt is not None:
        _dev_f64(dt, "dt")
    if max_eig is not None:
        _dev_f64(max_eig, "max_eig")
    n = _n_patches(patches)
    _dev_nbr(neighbours, n, 2)
    if blob.numel() != MLP_BLOB_WORDS:
        raise ValueError("blob has the wrong size")
    _check(library().fv_batch_update_learned_2d(_ptr(patches), n, _ptr(neighbours), _ptr(q_in),
                                                q_in.numel(), _ptr(q_out), q_out.numel(),
                                                float(gamma), _ptr(dt), _ptr(blob),
                                                float(threshold), _ptr(max_eig),
                                                _stream(stream)))


class Plan:
    """A work plan for an uneven batch (fv_plan_mixed), with its order and
    work units uploaded to the device.  ``order`` (host) lists the patch
    indices sorted by size, 16^3 first; ``units`` (host) is the work list."""

    def __init__(self, desc, device="cuda", dim=3):
        import torch
        desc = np.ascontiguousarray(desc, dtype=PATCH_DTYPE)
        n = desc.shape[0]
        self.order = np.zeros(max(n, 1), dtype=np.int64)
        self.units = (WorkUnit * max(n, 1))()
        self.c = MixedPlan()
        _check(library().fv_plan_mixed(desc.ctypes.data_as(ctypes.c_void_p), n, dim,
                                       self.order.ctypes.data_as(ctypes.c_void_p),
                                       ctypes.cast(self.units, ctypes.c_void_p),
                                       ctypes.byref(self.c)))
        self.order = self.order[:n]
        nu = self.c.n_units
        raw = np.frombuffer(bytes(self.units), dtype=np.uint8)[:nu * ctypes.sizeof(WorkUnit)]
        self.units_host = raw.view(np.dtype([("p", "<i4"), ("count", "<i4"), ("first", "<i8")]))
        self.order_dev = torch.from_numpy(self.order.copy()).to(device)
        self.units_dev = torch.from_numpy(raw.copy()).to(device)
        self.c.order = self.order_dev.data_ptr() if n else None
        self.c.units = self.units_dev.data_ptr() if nu else None
        self.n = n

    @property
    def n_units(self):
        return int(self.c.n_units)

    def classes(self):
        """[(p, first, count)] of the size classes present, in plan order."""
        return [(int(self.c.class_p[k]), int(self.c.class_first[k]), int(self.c.class_count[k]))
                for k in range(3) if self.c.class_count[k] > 0]


def step_local(patches, neighbours, plan, q_in, q_out, *, dim=3, gamma=1.4, cfl=0.4,
               max_eig=None, schedule="persistent", workgroups=0, stream=None):
    """fv_step_local[_f32]: one step of an uneven batch with local time steps
    (each patch advances by its own descriptor dt; t and dt are updated)."""
    sfx = _same_state(q_in, q_out)
    if max_eig is not None:
        _dev_f64(max_eig, "max_eig")
    n = _n_patches(patches)
    _dev_nbr(neighbours, n, dim)
    if max_eig is not None and max_eig.numel() < n:
        raise ValueError("max_eig needs one entry per patch")
    if schedule not in SCHEDULES:
        raise ValueError(f"schedule must be one of {sorted(SCHEDULES)}")
    fn = getattr(library(), "fv_step_local" + sfx)
    _check(fn(_ptr(patches), n, _ptr(neighbours), ctypes.byref(plan.c), _ptr(q_in), q_in.numel(),
              _ptr(q_out), q_out.numel(), dim, dim + 2, float(gamma), float(cfl), _ptr(max_eig),
              SCHEDULES[schedule], int(workgroups), _stream(stream)))


def local_timestep(patches, per_patch, *, dim, cfl=0.4, stream=None):
    """fv_local_timestep: patches[b].dt = cfl * min dx_b / (dim * per_patch[b])."""
    _dev_f64(per_patch, "per_patch")
    n = _n_patches(patches)
    if per_patch.numel() < n:
        raise ValueError("per_patch needs one entry per patch")
    _check(library().fv_local_timestep(_ptr(patches), n, _ptr(per_patch), dim, float(cfl),
                                       _stream(stream)))


class LocalStepper:
    """Device-resident driver for an uneven 3-D batch with local time steps.

    The descriptors are stored on the device in plan order (16^3, then 8^3,
    then 4^3 patches), with the neighbour table renumbered to match, so each
    size class is one contiguous range; the state buffers keep the caller's
    layout.  The first local steps come from the initial state (per class
    fv_max_eigenvalue, then fv_local_timestep); each step is fv_step_local
    under the chosen schedule, and swaps the state buffers.
    """

    def __init__(self, desc, neighbours, q0, *, gamma=1.4, cfl=0.4, schedule="persistent",
                 workgroups=0, device="cuda", dtype=None):
        import torch
        desc = np.ascontiguousarray(desc, dtype=PATCH_DTYPE)
        n = desc.shape[0]
        q0 = np.ascontiguousarray(q0, dtype=np.float64 if dtype is None else dtype)
        self.gamma, self.cfl = gamma, cfl
        self.schedule, self.workgroups = schedule, workgroups
        base = Plan(desc, device)
        self.perm = base.order                         # device position -> patch
        self.inv = np.empty(n, dtype=np.int64)
        self.inv[self.perm] = np.arange(n)
        sdesc = desc[self.perm]
        nbr = np.ascontiguousarray(neighbours, np.int64).reshape(n, 6)[self.perm]
        nbr = np.where(nbr >= 0, self.inv[np.maximum(nbr, 0)], nbr)
        self.plan = Plan(sdesc, device)                # order is the identity now
        self.n = n
        for p, first, count in self.plan.classes():
            check_patches(sdesc[first:first + count], 3, p, False, q0.size, q0.size,
                          q_in_halo=False)
        self.patches = upload_patches(sdesc, device)
        self.neighbours = torch.from_numpy(np.ascontiguousarray(nbr)).to(device)
        self.a = torch.from_numpy(q0).to(device)
        self.b = self.a.clone()
        self.per_patch = torch.empty(max(n, 1), dtype=torch.float64, device=device)
        rec = PATCH_DTYPE.itemsize
        for p, first, count in self.plan.classes():
            max_eigenvalue(self.patches[first * rec:(first + count) * rec], self.a,
                           self.per_patch[first:first + count], dim=3, p=p, gamma=gamma,
                           q_halo=False)
        if n:
            local_timestep(self.patches, self.per_patch, dim=3, cfl=cfl)

    def step(self, stream=None):
        step_local(self.patches, self.neighbours, self.plan, self.a, self.b, gamma=self.gamma,
                   cfl=self.cfl, max_eig=self.per_patch, schedule=self.schedule,
                   workgroups=self.workgroups, stream=stream)
        self.a, self.b = self.b, self.a

    def state(self):
        return self.a

    def descriptors(self):
        """Host copy of the descriptors in the caller's patch order."""
        raw = self.patches.cpu().numpy()
        return raw.view(PATCH_DTYPE)[self.inv].copy()

    def max_eig(self):
        """Host copy of the per-patch maxima of the latest state, caller's order."""
        return self.per_patch[:self.n].cpu().numpy()[self.inv]


class Stepper:
    """Device-resident multi-step driver over one patch batch (ping-pong buffers).

    mode "fused" (default): compact blocks [s][p^d]; each step is ONE launch of
    fv_step_gather (update with the halo exchange fused into the gather, plus
    the next step's CFL time step).  mode "gather": the same arithmetic as two
    launches, fv_cfl_timestep + fv_batch_update_gather.  mode "halo": blocks
    with halo [s][(p+2)^d]; fv_cfl_timestep + fv_batch_update + fv_fill_halo
    (the paper's interface, halo kept consistent by a separate pass).  mode
    "halo_step": the same blocks and results as "halo" in ONE launch per step
    (fv_step_halo: the exchange pushed into the output halos, the next CFL
    step from the fused reduction; float64 state).  mode "pipelined": the
    results of "fused" in ONE launch of fv_step_gather_pipelined per step,
    each launch taking its time step from the maxima the previous one folded
    (the first from the constructor's CFL step).  The time
    step always comes from the per-patch maxima of the previous step's state;
    nothing leaves the device.  q0 must be laid out for the mode
    (workloads.PatchGrid.pack for "halo", pack_compact otherwise).
    """

    def __init__(self, desc, neighbours, q0, *, dim, p, gamma=1.4, cfl=0.4, mode="fused",
                 device="cuda", dtype=None):
        import torch
        if mode not in ("fused", "gather", "halo", "halo_step", "pipelined"):
            raise ValueError("mode must be 'fused', 'gather', 'halo', 'halo_step' or "
                             "'pipelined'")
        if mode == "halo_step" and dtype not in (None, np.float64):
            raise ValueError("mode 'halo_step' takes float64 state")
        desc = np.ascontiguousarray(desc, dtype=PATCH_DTYPE)
        if not np.array_equal(desc["q_in"], desc["q_out"]):
            raise ValueError("the ping-pong stepper needs q_in == q_out offsets")
        q0 = np.ascontiguousarray(q0, dtype=np.float64 if dtype is None else dtype)
        self.mode = mode
        self.halo = mode in ("halo", "halo_step")
        # one launch per step that also computes the next step's dt
        self.one_launch = mode in ("fused", "halo_step", "pipelined")
        self.dim, self.p, self.gamma, self.cfl = dim, p, gamma, cfl
        self.n = desc.shape[0]
        self.patches = upload_patches(desc, device, dim=dim, p=p, q_out_halo=self.halo,
                                      q_in_len=q0.size, q_out_len=q0.size, q_in_halo=self.halo)
        self.neighbours = torch.from_numpy(np.ascontiguousarray(neighbours, np.int64)).to(device)
        self.a = torch.from_numpy(q0).to(device)
        self.b = self.a.clone()
        self.per_patch = torch.empty(self.n, dtype=torch.float64, device=device)
        self.lam = torch.empty(1, dtype=torch.float64, device=device)
        self.dt = torch.empty(1, dtype=torch.float64, device=device)
        self.dt_next = torch.empty(1, dtype=torch.float64, device=device)
        words = (pipelined_workspace_words if mode == "pipelined" else step_workspace_words)(
            self.n, dim, p)
        self.workspace = torch.zeros(max(3, words), dtype=torch.int64, device=device)
        self._fused_args = None  # per buffer order: checked argument tuples of fv_step_gather
        self._parity = 0
        self._k = 0  # steps taken (pipelined: the phase is _k % 3, dt given on step 0)
        self._pipe_args = {}  # (state buffers, phase, first step) -> (entry point, arguments)
        self.dt_used = torch.zeros(1, dtype=torch.float64, device=device)
        max_eigenvalue(self.patches, self.a, self.per_patch, dim=dim, p=p, gamma=gamma,
                       q_halo=self.halo)
        if self.one_launch:
            # the first step's dt; later ones come out of the fused launch
            cfl_timestep(self.patches, self.per_patch, dim=dim, cfl=cfl, lambda_out=self.lam,
                         dt_out=self.dt)

    def cfl_step(self, stream=None):
        if self.one_launch:
            return  # computed by the previous fused launch (or the constructor)
        cfl_timestep(self.patches, self.per_patch, dim=self.dim, cfl=self.cfl,
                     lambda_out=self.lam, dt_out=self.dt, stream=stream)

    def update(self, stream=None):
        if self.mode == "pipelined":
            key = (self.a.data_ptr(), self.b.data_ptr(), self._k % 3, self._k == 0)
            call = self._pipe_args.get(key)
            if call is None:
                # checked once per (buffer order, phase), then kept: eager
                # stepping costs one call
                call = _pipelined_args(self.patches, self.neighbours, self.a, self.b,
                                       self.workspace, self.dim, self.p, self.gamma, self.cfl,
                                       self._k % 3, self.dt if self._k == 0 else None,
                                       self.dt_used, self.per_patch, self.lam)
                self._pipe_args[key] = call
            _check(call[0](*call[1], _stream(stream)))
            return
        if self.mode == "halo_step":
            step_halo(self.patches, self.neighbours, self.a, self.b, self.dt, self.dt_next,
                      self.workspace, dim=self.dim, p=self.p, gamma=self.gamma, cfl=self.cfl,
                      max_eig=self.per_patch, lambda_out=self.lam, stream=stream)
        elif self.mode == "halo":
            batch_update(self.patches, self.a, self.b, dim=self.dim, p=self.p, gamma=self.gamma,
                         q_out_halo=True, dt=self.dt, max_eig=self.per_patch, stream=stream)
        elif self.mode == "gather":
            batch_update_gather(self.patches, self.neighbours, self.a, self.b, dim=self.dim,
                                p=self.p, gamma=self.gamma, q_out_halo=False, dt=self.dt,
                                max_eig=self.per_patch, stream=stream)
        else:
            bufs = (self.a.data_ptr(), self.b.data_ptr(), self.dt.data_ptr())
            if self._fused_args is None or bufs != self._fused_bufs[self._parity]:
                # checks every argument once, through the checked binding, then
                # keeps the two argument tuples of the ping-pong (the same
                # buffers every step) so that eager stepping costs one call
                step_gather(self.patches, self.neighbours, self.a, self.b, self.dt, self.dt_next,
                            self.workspace, dim=self.dim, p=self.p, gamma=self.gamma,
                            cfl=self.cfl, max_eig=self.per_patch, lambda_out=self.lam,
                            stream=stream)
                fn = getattr(library(), "fv_step_gather" + _same_state(self.a, self.b))

                def args(qa, qb, d0, d1):
                    return (_ptr(self.patches), self.n, _ptr(self.neighbours), _ptr(qa),
                            qa.numel(), _ptr(qb), qb.numel(), self.dim, self.p, self.dim + 2,
                            float(self.gamma), float(self.cfl), _ptr(d0), _ptr(self.per_patch),
                            _ptr(d1), _ptr(self.lam), _ptr(self.workspace),
                            self.workspace.numel())

                self._fn = fn
                self._parity = 0
                self._fused_args = (args(self.a, self.b, self.dt, self.dt_next),
                                    args(self.b, self.a, self.dt_next, self.dt))
                self._fused_bufs = (bufs, (bufs[1], bufs[0], self.dt_next.data_ptr()))
                return
            _check(self._fn(*self._fused_args[self._parity], _stream(stream)))

    def exchange(self, stream=None):
        if self.mode == "halo":
            fill_halo(self.patches, self.neighbours, self.b, dim=self.dim, p=self.p,
                      stream=stream)

    def swap(self):
        """Swap the state buffers (and, fused, the dt buffers): the new state
        becomes the input of the next step."""
        self._swap_roles()
        self._k += 1

    def _swap_roles(self):
        self.a, self.b = self.b, self.a
        if self.one_launch and self.mode != "pipelined":
            self.dt, self.dt_next = self.dt_next, self.dt
            self._parity ^= 1

    def graph_period(self):
        """Steps after which the launch arguments repeat (a graph of k steps
        can be replayed back to back only when k is a multiple of it)."""
        return 6 if self.mode == "pipelined" else 2

    def position(self):
        """Steps the host side has issued (update + swap pairs)."""
        return self._k

    def seek(self, k):
        """Set the host side to step k without launching anything (after
        graph replays moved the data there).  In mode 'pipelined' step 0 is
        the one that takes the constructor's time step on a clean workspace,
        so once a step has been issued k must be >= 1."""
        if self.mode == "pipelined" and k < 1 and self._k > 0:
            raise ValueError("a pipelined run cannot go back to its first step")
        if (k - self._k) % 2:
            self._swap_roles()
        self._k = k

    def step(self, stream=None):
        self.cfl_step(stream)
        self.update(stream)
        self.exchange(stream)
        self.swap()

    def last_dt(self):
        """Device tensor holding the time step used by the most recent step."""
        if self.mode == "pipelined":
            return self.dt_used
        return self.dt_next if self.one_launch else self.dt

    def state(self):
        return self.a
