"""Oracle for the learned face-flux correction on 2-D Euler grids (TEST
INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU leg
use it; it shares no code with the GPU library).

The method (an extension of the paper's Rusanov update, Section 2 eqs.
(2)-(5); the correction itself is not in the paper) is written out here on
whole periodic or transmissive grids in plain numpy:

* Face frame.  A face with normal along axis k sits between volumes L (index
  i-1 along k) and R (index i).  Its state vectors are read in the face
  frame (rho, j_n, j_t, E): the normal momentum first, the tangential one
  second.
* Features: the four volumes i-2, i-1, i, i+1 along the normal, each
  (rho, j_n, j_t, E), 16 values in that order.  Normalised per feature,
  x_hat = (x - x_mean) * x_scale.
* MLP 16 -> 64 -> 64 -> 4: h1 = tanh(W1 b(x_hat) + b1), h2 = tanh(W2 b(h1) +
  b2), o = W3 b(h2) + b3, where b() rounds to bfloat16 (the matrix products
  take bfloat16 operands, weights rounded the same way) and sums, biases and
  tanh are float32.
* Correction in the face frame: dF = o * y_scale + y_mean, rotated back to
  the grid axes, set to 0 where the density-jump indicator
  |rho_R - rho_L| / min(rho_L, rho_R) exceeds the threshold (0.2): there the
  plain Rusanov flux is used.
* Face flux F = F_rusanov + dF (float64), and the explicit update
  q - (dt/dx)(F_x(i+1/2) - F_x(i-1/2)) - (dt/dy)(F_y(j+1/2) - F_y(j-1/2)),
  x first, as the plain oracle does.

Parameter blob (float32, one flat array), the layout the GPU library reads:
x_mean[16], x_scale[16], W1[64][16], b1[64], W2[64][64], b2[64], W3[4][64],
b3[4], y_scale[4], y_mean[4].
"""
import numpy as np

GAMMA = 1.4
THRESHOLD = 0.2
NF, NH, NO = 16, 64, 4

# (name, shape) in blob order
BLOB_LAYOUT = [("x_mean", (NF,)), ("x_scale", (NF,)), ("w1", (NH, NF)), ("b1", (NH,)),
               ("w2", (NH, NH)), ("b2", (NH,)), ("w3", (NO, NH)), ("b3", (NO,)),
               ("y_scale", (NO,)), ("y_mean", (NO,))]
BLOB_SIZE = sum(int(np.prod(s)) for _, s in BLOB_LAYOUT)


def unpack_blob(blob):
    """Dict of float32 arrays (views) from a parameter blob."""
    blob = np.asarray(blob, dtype=np.float32).reshape(-1)
    if blob.size != BLOB_SIZE:
        raise ValueError(f"parameter blob must hold {BLOB_SIZE} floats")
    out, o = {}, 0
    for name, shape in BLOB_LAYOUT:
        n = int(np.prod(shape))
        out[name] = blob[o:o + n].reshape(shape)
        o += n
    return out


def pack_blob(params):
    return np.concatenate([np.asarray(params[name], dtype=np.float32).reshape(-1)
                           for name, _ in BLOB_LAYOUT])


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as
    float32.  bfloat16 keeps the upper 16 bits of the binary32 pattern; the
    lower 16 are rounded away.  NaN stays NaN."""
    x = np.asarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).copy()
    nan = np.isnan(x)
    out[nan] = x[nan]
    return out


def _nanmax(a, b):
    out = np.where(a > b, a, b)
    out = np.where(np.isnan(b), b, out)
    return np.where(np.isnan(a), a, out)


def euler_flux_2d(q, k, gamma=GAMMA):
    """f^k(q) for 2-D states q[4, ...] (Section 2 eq. (2)), operations in
    the order of the C oracle."""
    rho, E = q[0], q[3]
    jj = 0.0 + q[1] * q[1]
    jj = jj + q[2] * q[2]
    p = (gamma - 1.0) * (E - 0.5 * jj / rho)
    jd = q[1 + k]
    f = np.empty_like(q)
    f[0] = jd
    for m in range(2):
        f[1 + m] = jd * q[1 + m] / rho
        if m == k:
            f[1 + m] = f[1 + m] + p
    f[3] = (E + p) * jd / rho
    return f, p


def rusanov_2d(L, R, k, gamma=GAMMA):
    """Rusanov flux (eq. (4)) with a = max of |u_k| + c on both sides (eq. (5))."""
    fL, pL = euler_flux_2d(L, k, gamma)
    fR, pR = euler_flux_2d(R, k, gamma)
    lamL = np.abs(L[1 + k] / L[0]) + np.sqrt(gamma * pL / L[0])
    lamR = np.abs(R[1 + k] / R[0]) + np.sqrt(gamma * pR / R[0])
    a = _nanmax(lamL, lamR)
    return 0.5 * ((fL + fR) - a * (R - L))


def to_face_frame(q, k):
    """(rho, j_n, j_t, E) for a face with normal along axis k."""
    return q[[0, 1 + k, 2 - k, 3]]


def mlp_forward(x_hat, params):
    """MLP on normalised features x_hat[n, 16] -> o[n, 4] (float32, bfloat16
    operands of every product)."""
    w1, w2, w3 = (bf16_round(params[w]) for w in ("w1", "w2", "w3"))
    x = bf16_round(x_hat)
    h1 = np.tanh((x @ w1.T).astype(np.float32) + params["b1"]).astype(np.float32)
    h2 = np.tanh((bf16_round(h1) @ w2.T).astype(np.float32) + params["b2"]).astype(np.float32)
    return ((bf16_round(h2) @ w3.T).astype(np.float32) + params["b3"]).astype(np.float32)


def _pad(q, bc, h=2):
    mode = "wrap" if bc == "periodic" else "edge"
    return np.pad(q, ((0, 0), (h, h), (h, h)), mode=mode)


def face_data(q, k, bc):
    """For every face with normal along k of the grid q[4, Ny, Nx]: left and
    right states, the 4-volume stencil in the face frame [16, ...] and the
    indicator.  x faces: shape (Ny, Nx+1); y faces: (Ny+1, Nx)."""
    qp = _pad(q, bc)
    ny, nx = q.shape[1:]
    if k == 0:
        sl = [qp[:, 2:2 + ny, o:o + nx + 1] for o in range(0, 4)]
    else:
        sl = [qp[:, o:o + ny + 1, 2:2 + nx] for o in range(0, 4)]
    L, R = sl[1], sl[2]
    feats = np.concatenate([to_face_frame(v, k) for v in sl], axis=0)
    ind = np.abs(R[0] - L[0]) / np.minimum(L[0], R[0])
    return L, R, feats, ind


def face_correction(feats, ind, k, params, threshold=THRESHOLD):
    """dF[4, ...] in grid axes for faces with features feats[16, ...]."""
    shape = feats.shape[1:]
    x = feats.reshape(NF, -1).T.astype(np.float32)
    x_hat = ((x - params["x_mean"]) * params["x_scale"]).astype(np.float32)
    o = mlp_forward(x_hat, params)
    d = (o * params["y_scale"] + params["y_mean"]).astype(np.float32)
    d = d.T.reshape((NO,) + shape).astype(np.float64)
    d = d[[0, 1 + k, 2 - k, 3]]  # face frame -> grid axes (the swap is its own inverse)
    return np.where(ind > threshold, 0.0, d)


def learned_step_2d(q, dx, dy, dt, params=None, bc="periodic", gamma=GAMMA,
                    threshold=THRESHOLD):
    """One explicit step of the 2-D grid q[4, Ny, Nx] with corrected fluxes
    (params None: the plain Rusanov update).  Returns (q_new, F_x, F_y)."""
    q = np.asarray(q, dtype=np.float64)
    fluxes = []
    for k in (0, 1):
        L, R, feats, ind = face_data(q, k, bc)
        F = rusanov_2d(L, R, k, gamma)
        if params is not None:
            F = F + face_correction(feats, ind, k, params, threshold)
        fluxes.append(F)
    Fx, Fy = fluxes
    qn = q - (dt / dx) * (Fx[:, :, 1:] - Fx[:, :, :-1])
    qn = qn - (dt / dy) * (Fy[:, 1:, :] - Fy[:, :-1, :])
    return qn, Fx, Fy


def max_eigenvalue_2d(q, gamma=GAMMA):
    """Largest |u_k| + c over the grid."""
    rho = q[0]
    p = (gamma - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / rho)
    c = np.sqrt(gamma * p / rho)
    return float(np.max(np.maximum(np.abs(q[1] / rho), np.abs(q[2] / rho)) + c))


# ---------------------------------------------------------------------------
# Training data: coarse-graining of 4x finer runs
# ---------------------------------------------------------------------------

def coarse_grain(qf, r=4):
    """Conservative r x r averages of a fine grid qf[4, r*Ny, r*Nx]."""
    s, nyf, nxf = qf.shape
    return qf.reshape(s, nyf // r, r, nxf // r, r).mean(axis=(2, 4))


def coarse_face_flux(qf, k, bc, r=4, gamma=GAMMA):
    """Average over the r fine faces that make up each coarse face (normal
    along k) of the fine Rusanov fluxes.  Shape as the coarse faces."""
    L, R, _, _ = face_data(qf, k, bc)
    F = rusanov_2d(L, R, k, gamma)
    if k == 0:
        F = F[:, :, ::r]                       # fine faces on coarse x faces
        s, nyf, nxc1 = F.shape
        return F.reshape(s, nyf // r, r, nxc1).mean(axis=2)
    F = F[:, ::r, :]
    s, nyc1, nxf = F.shape
    return F.reshape(s, nyc1, nxf // r, r).mean(axis=3)


def face_samples(qc, Fx_star, Fy_star, bc, gamma=GAMMA):
    """(features[n,16], targets[n,4], indicator[n]) for every coarse face, x
    faces first (row-major), then y faces.  Target: the face-frame difference
    between the reference flux F_star and the coarse Rusanov flux."""
    feats, targ, inds = [], [], []
    for k, Fs in ((0, Fx_star), (1, Fy_star)):
        L, R, f, ind = face_data(qc, k, bc)
        d = to_face_frame(Fs - rusanov_2d(L, R, k, gamma), k)
        feats.append(f.reshape(NF, -1).T)
        targ.append(d.reshape(NO, -1).T)
        inds.append(ind.reshape(-1))
    return np.concatenate(feats), np.concatenate(targ), np.concatenate(inds)


# ---------------------------------------------------------------------------
# Training: mean-squared error of the float32 network (no bfloat16 rounding)
# ---------------------------------------------------------------------------

def mlp_loss_grads(x_hat, y_hat, params):
    """Loss L = mean over samples and outputs of (o - y_hat)^2 for the
    network without rounding, and dL/d(w1, b1, w2, b2, w3, b3), by the chain
    rule in float64."""
    x = np.asarray(x_hat, np.float64)
    y = np.asarray(y_hat, np.float64)
    w1, b1, w2, b2, w3, b3 = (np.asarray(params[k], np.float64)
                              for k in ("w1", "b1", "w2", "b2", "w3", "b3"))
    n = x.shape[0]
    h1 = np.tanh(x @ w1.T + b1)
    h2 = np.tanh(h1 @ w2.T + b2)
    o = h2 @ w3.T + b3
    loss = np.mean((o - y) ** 2)
    do = 2.0 * (o - y) / (n * NO)
    g = {"w3": do.T @ h2, "b3": do.sum(0)}
    d2 = (do @ w3) * (1.0 - h2 * h2)
    g["w2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ w2) * (1.0 - h1 * h1)
    g["w1"] = d1.T @ x
    g["b1"] = d1.sum(0)
    return loss, g


def adam_update(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015) on the weight and bias arrays, in
    place; m, v: dicts of first and second moment arrays; step counts from 1."""
    for k in ("w1", "b1", "w2", "b2", "w3", "b3"):
        g = np.asarray(grads[k], np.float64)
        m[k] = beta1 * m[k] + (1.0 - beta1) * g
        v[k] = beta2 * v[k] + (1.0 - beta2) * g * g
        mh = m[k] / (1.0 - beta1 ** step)
        vh = v[k] / (1.0 - beta2 ** step)
        params[k] = (params[k] - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
