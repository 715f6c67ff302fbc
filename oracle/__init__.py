"""CPU oracle for the batched Finite Volume patch update (TEST INFRASTRUCTURE).

Plain, slow, FP64 reference written from the paper ("GPU Offloading in ExaHyPE
Through C++ Standard Algorithms", arXiv 2302.09005): Section 2 eqs. (1)-(5) and
Algorithm 1.  The arithmetic lives in ``fv_oracle.c`` (built by
``oracle/build.py`` into ``liboracle.so``); this module only marshals numpy
arrays.  ``riemann.py`` holds the exact Riemann solution used to pin the
oracle's shock-tube behaviour.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library and never imports it.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FV_ORACLE_LIB names another build of fv_oracle.c (the sanitizer test loads
# an AddressSanitizer / UBSan build this way)
_LIB_PATH = os.environ.get("FV_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_flux.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp]
    lib.oracle_flux.restype = None
    lib.oracle_eigenvalue.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double]
    lib.oracle_eigenvalue.restype = ctypes.c_double
    lib.oracle_max_eigenvalue_state.argtypes = [_dp, ctypes.c_int, ctypes.c_double]
    lib.oracle_max_eigenvalue_state.restype = ctypes.c_double
    lib.oracle_rusanov.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp]
    lib.oracle_rusanov.restype = None
    lib.oracle_fv_step.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   _i64p, _i64p, ctypes.c_int, _dp, _dp, _dp, _dp, _dp,
                                   ctypes.c_int]
    lib.oracle_fv_step.restype = ctypes.c_int
    lib.oracle_fv_step_alg1.argtypes = lib.oracle_fv_step.argtypes
    lib.oracle_fv_step_alg1.restype = ctypes.c_int
    lib.oracle_max_eigenvalue.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, _i64p, ctypes.c_int, _dp, _dp, _dp]
    lib.oracle_max_eigenvalue.restype = ctypes.c_int
    lib.oracle_cfl_dt.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, _dp, ctypes.c_double, _dp]
    lib.oracle_cfl_dt.restype = ctypes.c_double
    lib.oracle_local_dt.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, _dp, ctypes.c_double, _dp]
    lib.oracle_local_dt.restype = None
    lib.oracle_fill_halo.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, _i64p, _i64p, _dp]
    lib.oracle_fill_halo.restype = ctypes.c_int
    lib.oracle_totals.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, _i64p,
                                  ctypes.c_int, _dp, _dp]
    lib.oracle_totals.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_i64p)


def flux(q, d, direction, gamma=1.4):
    """Physical flux f^direction(q) of the Euler equations (Section 2, eq. (2))."""
    q, qp = _f64(q)
    out = np.empty(d + 2)
    _load().oracle_flux(qp, d, direction, gamma, out.ctypes.data_as(_dp))
    return out


def eigenvalue(q, d, direction, gamma=1.4):
    """|u_direction| + c (Section 2, eq. (5))."""
    q, qp = _f64(q)
    return _load().oracle_eigenvalue(qp, d, direction, gamma)


def max_eigenvalue_state(q, d, gamma=1.4):
    q, qp = _f64(q)
    return _load().oracle_max_eigenvalue_state(qp, d, gamma)


def rusanov(left, right, d, direction, gamma=1.4):
    """Rusanov face flux (Section 2, eq. (4))."""
    left, lp = _f64(left)
    right, rp = _f64(right)
    out = np.empty(d + 2)
    _load().oracle_rusanov(lp, rp, d, direction, gamma, out.ctypes.data_as(_dp))
    return out


def fv_step(q_in_off, q_out_off, dx, dt, q_in, d, p, gamma=1.4, *, q_out=None,
            out_halo=False, out_len=None, nthreads=0, order="faces"):
    """One explicit Euler step of every patch (Section 2 eqs. (3)-(5), Algorithm 1).

    q_in_off / q_out_off: int64[n] element offsets of each patch block.
    dx: float64[n, 3]; dt: float64[n].
    order: "faces" (one Rusanov flux difference per face) or "alg1" (the step
    order of Algorithm 1: copy, dissipative parts, central parts; equal up to
    rounding).
    Returns (q_out, max_eig[n]).  When q_out is given it is updated in place
    (only the interior volumes of each output block are written).
    """
    if order not in ("faces", "alg1"):
        raise ValueError("order must be 'faces' or 'alg1'")
    lib = _load()
    q_in_off, ip = _i64(q_in_off)
    q_out_off, op = _i64(q_out_off)
    n = q_in_off.shape[0]
    dx = np.ascontiguousarray(np.broadcast_to(np.asarray(dx, np.float64), (n, 3)))
    dx, dxp = _f64(dx)
    dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, np.float64), (n,)))
    dt, dtp = _f64(dt)
    q_in, qip = _f64(q_in)
    if q_out is None:
        blk = (d + 2) * (p + 2 if out_halo else p) ** d
        size = out_len if out_len is not None else (int(q_out_off.max()) + blk if n else 0)
        q_out = np.zeros(size)
    if q_out.dtype != np.float64 or not q_out.flags.c_contiguous:
        raise ValueError("q_out must be a contiguous float64 array")
    me = np.empty(n)
    fn = lib.oracle_fv_step if order == "faces" else lib.oracle_fv_step_alg1
    rc = fn(n, d, p, gamma, ip, op, int(bool(out_halo)), dxp, dtp, qip,
            q_out.ctypes.data_as(_dp), me.ctypes.data_as(_dp), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_fv_step rejected its arguments")
    return q_out, me


def max_eigenvalue(off, q, d, p, halo, gamma=1.4):
    """Per-patch and global largest eigenvalue over interior volumes."""
    lib = _load()
    off, op = _i64(off)
    n = off.shape[0]
    q, qp = _f64(q)
    per = np.empty(n)
    g = ctypes.c_double(0.0)
    rc = lib.oracle_max_eigenvalue(n, d, p, gamma, op, int(bool(halo)), qp,
                                   per.ctypes.data_as(_dp), ctypes.byref(g))
    if rc != 0:
        raise ValueError("oracle_max_eigenvalue rejected its arguments")
    return per, g.value


def cfl_dt(dx, max_eig, d, cfl=0.4):
    """(dt, Lambda) from the CFL condition dt = cfl * min dx / (d * Lambda)."""
    max_eig, mp = _f64(max_eig)
    n = max_eig.shape[0]
    dx = np.ascontiguousarray(np.broadcast_to(np.asarray(dx, np.float64), (n, 3)))
    dx, dxp = _f64(dx)
    lam = ctypes.c_double(0.0)
    dt = _load().oracle_cfl_dt(n, d, dxp, mp, cfl, ctypes.byref(lam))
    return dt, lam.value


def local_dt(dx, max_eig, d, cfl=0.4):
    """Per-patch CFL steps dt[b] = cfl * min dx[b] / (d * max_eig[b]) (Section 4)."""
    max_eig, mp = _f64(max_eig)
    n = max_eig.shape[0]
    dx = np.ascontiguousarray(np.broadcast_to(np.asarray(dx, np.float64), (n, 3)))
    dx, dxp = _f64(dx)
    dt = np.empty(n)
    _load().oracle_local_dt(n, d, dxp, mp, cfl, dt.ctypes.data_as(_dp))
    return dt


def fill_halo(off, neighbours, q, d, p):
    """Face-halo fill in place (periodic via the neighbour table; -1 = transmissive)."""
    off, op = _i64(off)
    neighbours, np_ = _i64(neighbours)
    n = off.shape[0]
    if neighbours.size != 2 * d * n:
        raise ValueError("neighbours must have 2*d entries per patch")
    if q.dtype != np.float64 or not q.flags.c_contiguous:
        raise ValueError("q must be a contiguous float64 array")
    rc = _load().oracle_fill_halo(n, d, p, op, np_, q.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError("oracle_fill_halo rejected its arguments")
    return q


def totals(off, q, d, p, halo):
    off, op = _i64(off)
    q, qp = _f64(q)
    out = np.empty(d + 2)
    rc = _load().oracle_totals(off.shape[0], d, p, op, int(bool(halo)), qp,
                               out.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError("oracle_totals rejected its arguments")
    return out


def num_threads():
    return _load().oracle_num_threads()


def run_steps(q_in_off, dx, q, neighbours, d, p, steps, gamma=1.4, cfl=0.4,
              nthreads=0, t_end=None):
    """Multi-step driver: halo'd ping-pong, global CFL step each step.

    Each step: Lambda from the current state (first step) or from the previous
    step's per-patch maxima, dt = cfl*min dx/(d*Lambda) (clipped to reach
    t_end exactly when given), update, face-halo fill.  The halo of q must be
    filled on entry.  Returns (q, t, list of dt).
    """
    off = np.ascontiguousarray(q_in_off, dtype=np.int64)
    a = np.array(q, dtype=np.float64, copy=True)
    b = a.copy()
    per, _ = max_eigenvalue(off, a, d, p, True, gamma)
    t = 0.0
    dts = []
    for _ in range(steps):
        dt, _lam = cfl_dt(dx, per, d, cfl)
        if t_end is not None:
            if t >= t_end:
                break
            dt = min(dt, t_end - t)
        b, per = fv_step(off, off, dx, np.full(off.shape[0], dt), a, d, p, gamma,
                         q_out=b, out_halo=True, nthreads=nthreads)
        fill_halo(off, neighbours, b, d, p)
        a, b = b, a
        t += dt
        dts.append(dt)
    return a, t, dts


def run_local_steps(off, sizes, dx, neighbours, q, steps, dt=None, t=None, gamma=1.4, cfl=0.4,
                    nthreads=0):
    """Local time stepping over a 3-D batch of mixed patch sizes (Section 4).

    off, sizes: int64[n] offsets of compact blocks [5][p_b^3] in q and their
    p_b; dx: float64[n, 3]; neighbours: int64[n, 6] (a neighbour must have the
    same p; -1 = transmissive).  Each step, for every patch b: fill its face
    halo, advance it by its own dt[b] (fv_step), t[b] += dt[b], then take
    dt[b] = local_dt from the new state's maximum.  When dt is None the first
    steps come from the initial state.  Patches of different size never
    interact, so each size class runs as one halo'd batch.
    Returns (q, dt, t, max_eig) after ``steps`` steps.
    """
    off = np.ascontiguousarray(off, dtype=np.int64)
    sizes = np.ascontiguousarray(sizes, dtype=np.int64)
    n = off.shape[0]
    dx = np.ascontiguousarray(np.broadcast_to(np.asarray(dx, np.float64), (n, 3)))
    nbr = np.ascontiguousarray(neighbours, dtype=np.int64).reshape(n, 6)
    q = np.array(q, dtype=np.float64, copy=True)
    t = np.zeros(n) if t is None else np.array(t, dtype=np.float64, copy=True)
    me = np.full(n, np.nan)
    classes = []
    for p in sorted(set(int(v) for v in sizes)):
        idx = np.nonzero(sizes == p)[0]
        pos = np.full(n, -1, dtype=np.int64)
        pos[idx] = np.arange(idx.shape[0])
        sub = nbr[idx]
        if ((sub >= 0) & (sizes[np.maximum(sub, 0)] != p)).any():
            raise ValueError("a neighbour has a different patch size")
        local_nbr = np.where(sub >= 0, pos[np.maximum(sub, 0)], -1)
        w = p + 2
        hoff = np.arange(idx.shape[0], dtype=np.int64) * 5 * w ** 3
        classes.append((p, idx, local_nbr, hoff))
    if dt is None:
        dt = np.empty(n)
        for p, idx, _, _ in classes:
            blocks = np.concatenate([q[off[b]:off[b] + 5 * p ** 3] for b in idx])
            coff = np.arange(idx.shape[0], dtype=np.int64) * 5 * p ** 3
            per, _ = max_eigenvalue(coff, blocks, 3, p, False, gamma)
            dt[idx] = local_dt(dx[idx], per, 3, cfl)
    else:
        dt = np.array(dt, dtype=np.float64, copy=True)
    for _ in range(steps):
        for p, idx, local_nbr, hoff in classes:
            w = p + 2
            m = idx.shape[0]
            a = np.full((m, 5, w, w, w), np.nan)
            for j, b in enumerate(idx):
                a[j, :, 1:-1, 1:-1, 1:-1] = q[off[b]:off[b] + 5 * p ** 3].reshape(5, p, p, p)
            a = a.reshape(-1)
            fill_halo(hoff, local_nbr, a, 3, p)
            coff = np.arange(m, dtype=np.int64) * 5 * p ** 3
            out, per = fv_step(hoff, coff, dx[idx], dt[idx], a, 3, p, gamma, out_halo=False,
                               out_len=m * 5 * p ** 3, nthreads=nthreads)
            for j, b in enumerate(idx):
                q[off[b]:off[b] + 5 * p ** 3] = out[coff[j]:coff[j] + 5 * p ** 3]
            t[idx] += dt[idx]
            me[idx] = per
            dt[idx] = local_dt(dx[idx], per, 3, cfl)
    return q, dt, t, me
