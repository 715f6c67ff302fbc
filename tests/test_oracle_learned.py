"""Pins of the learned-correction oracle (oracle/learned.py) against things
other than itself: the C oracle's plain update, torch's bfloat16 rounding
and Linear/Tanh layers with autograd, closed forms (uniform states, constant
corrections, exact averages), the telescoping identity between fine and
coarse updates, and finite differences of the loss."""
import math

import numpy as np
import pytest

import oracle
from oracle import learned as L
from paper_2302_09005_amd import workloads as W

EPS = 2.0 ** -52


def _random_grid(n, seed, rho=(0.5, 1.5)):
    rng = np.random.default_rng(seed)
    shape = (n, n)
    return W.to_conserved(rng.uniform(*rho, shape), [rng.uniform(-0.5, 0.5, shape) for _ in range(2)],
                          rng.uniform(0.5, 2.0, shape))


def _random_params(seed, scale=0.3, y_scale=1e-3):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in L.BLOB_LAYOUT:
        p[name] = rng.normal(0.0, scale, shape).astype(np.float32)
    p["x_mean"] = rng.uniform(-0.5, 1.5, L.NF).astype(np.float32)
    p["x_scale"] = rng.uniform(0.5, 2.0, L.NF).astype(np.float32)
    p["y_scale"] = np.full(L.NO, y_scale, np.float32)
    p["y_mean"] = np.zeros(L.NO, np.float32)
    return p


def test_bf16_rounding_values_and_torch():
    import torch
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -(1 + 2 ** -8),
                  np.inf, -np.inf, 3.4e38, 1e-40, 0.0, -0.0], np.float32)
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -1.0, np.inf, -np.inf, np.inf],
                    np.float32)
    got = L.bf16_round(x)
    np.testing.assert_array_equal(got[:8], want)
    assert np.isnan(L.bf16_round(np.array([np.nan], np.float32)))[0]
    rng = np.random.default_rng(0)
    y = (rng.standard_normal(100000) * 10.0 ** rng.uniform(-30, 30, 100000)).astype(np.float32)
    ref = torch.from_numpy(y).to(torch.bfloat16).float().numpy()
    np.testing.assert_array_equal(L.bf16_round(y), ref)
    np.testing.assert_array_equal(L.bf16_round(x), torch.from_numpy(x).to(torch.bfloat16).float().numpy())


@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_plain_update_equals_c_oracle(bc):
    """Without parameters the numpy update is the plain method: bit for bit the
    C oracle's update of the same grid cut into 16^2 patches."""
    q = _random_grid(64, 1)
    counts = (4, 4)
    grid = W.PatchGrid(2, 16, counts, 1.0 / 64, bc=(bc, bc))
    dt = 2e-3
    ref_flat, _ = oracle.fv_step(grid.offsets(), grid.offsets(), np.full((grid.n, 3), grid.dx),
                                 np.full(grid.n, dt), grid.pack(q), 2, 16, out_halo=True,
                                 out_len=grid.buffer_len(True))
    got, _, _ = L.learned_step_2d(q, grid.dx, grid.dx, dt, None, bc)
    np.testing.assert_array_equal(got, grid.unpack(ref_flat))


def test_zero_network_is_the_plain_update():
    q = _random_grid(32, 2)
    p = _random_params(3)
    for name in ("w1", "w2", "w3", "b1", "b2", "b3", "y_mean"):
        p[name][...] = 0.0
    a, Fa, Ga = L.learned_step_2d(q, 1 / 32, 1 / 32, 1e-3, p)
    b, Fb, Gb = L.learned_step_2d(q, 1 / 32, 1 / 32, 1e-3, None)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(Fa, Fb)


def test_constant_correction_closed_form():
    """A network that outputs the constant c: every unflagged face gets dF = c
    in the face frame (tangential and normal momenta swap on y faces), the
    flagged ones none."""
    q = W.to_conserved(np.where(np.arange(32)[None, :] < 16, 1.0, 0.5) * np.ones((32, 32)),
                       [0.1, -0.2], 1.0)  # a density jump of 1 (indicator 1.0) at x = 16 and 0
    p = _random_params(4)
    for name in ("w1", "w2", "w3", "b1", "b2"):
        p[name][...] = 0.0
    c = np.array([0.25, -0.5, 0.75, 1.0], np.float32)
    p["b3"][...] = c
    p["y_scale"][...] = 1.0
    p["y_mean"][...] = 0.0
    _, Fx, Fy = L.learned_step_2d(q, 1 / 32, 1 / 32, 1e-3, p)
    _, Px, Py = L.learned_step_2d(q, 1 / 32, 1 / 32, 1e-3, None)
    dx, dy = Fx - Px, Fy - Py
    flagged = np.zeros(Fx.shape[1:], bool)
    flagged[:, 0] = flagged[:, 16] = flagged[:, 32] = True  # periodic: x = 0 and 32 see the jump
    cx = c.astype(np.float64)[:, None, None]
    cy = c.astype(np.float64)[[0, 2, 1, 3], None, None]
    tol = 4 * EPS * (np.abs(Px) + 1)
    assert (np.abs(np.where(flagged, dx, dx - cx)) <= tol).all()
    assert (np.abs(dy - cy) <= 4 * EPS * (np.abs(Py) + 1)).all()


def test_transposed_grid_gives_transposed_result():
    q = _random_grid(24, 5)
    p = _random_params(6)
    a, _, _ = L.learned_step_2d(q, 1 / 24, 1 / 24, 2e-3, p)
    qt = q[[0, 2, 1, 3]].transpose(0, 2, 1).copy()
    b, _, _ = L.learned_step_2d(qt, 1 / 24, 1 / 24, 2e-3, p)
    bt = b[[0, 2, 1, 3]].transpose(0, 2, 1)
    assert np.abs(a - bt).max() <= 1e-14 * np.abs(a).max()


def test_correction_changes_the_update_where_unflagged():
    q = _random_grid(16, 7)
    p = _random_params(8)
    a, _, _ = L.learned_step_2d(q, 1 / 16, 1 / 16, 1e-3, p)
    b, _, _ = L.learned_step_2d(q, 1 / 16, 1 / 16, 1e-3, None)
    assert np.abs(a - b).max() > 1e-7


def test_coarse_grain_closed_forms():
    y, x = np.meshgrid(np.arange(64.0), np.arange(64.0), indexing="ij")
    qf = np.stack([1.0 + 0 * x, x, y, x + 2 * y])
    qc = L.coarse_grain(qf)
    yc, xc = np.meshgrid(np.arange(16.0), np.arange(16.0), indexing="ij")
    np.testing.assert_allclose(qc[1], 4 * xc + 1.5, rtol=0, atol=1e-12)
    np.testing.assert_allclose(qc[2], 4 * yc + 1.5, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(qc[0], 1.0)
    qr = _random_grid(64, 9)
    np.testing.assert_allclose(L.coarse_grain(qr).sum(axis=(1, 2)) * 16, qr.sum(axis=(1, 2)),
                               rtol=1e-13)


def test_uniform_state_fluxes_and_zero_targets():
    q = W.to_conserved(np.full((32, 32), 0.7), [0.3, -0.1], 1.2)
    f0, _ = L.euler_flux_2d(q, 0)
    for k in (0, 1):
        F = L.coarse_face_flux(q, k, "periodic")
        fk, _ = L.euler_flux_2d(q[:, :1, :1], k)
        assert np.abs(F - fk).max() <= 4 * EPS * np.abs(fk).max()
    qc = L.coarse_grain(q)
    feats, targ, ind = L.face_samples(qc, L.coarse_face_flux(q, 0, "periodic"),
                                      L.coarse_face_flux(q, 1, "periodic"), "periodic")
    assert np.abs(targ).max() <= 4 * EPS * np.abs(f0).max()
    assert (ind == 0).all()
    np.testing.assert_array_equal(feats[:, 0:4], feats[:, 4:8])


@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_telescoping_fine_fluxes_reproduce_the_coarse_grained_update(bc):
    """Four fine steps of dt on the 4x finer grid, coarse-grained, equal the
    coarse state advanced by 4 dt with the time- and face-averaged fine
    fluxes through the coarse faces (conservation, to rounding)."""
    qf = _random_grid(64, 10)
    dxf, dt = 1 / 64, 5e-4
    Fx = Fy = 0.0
    q = qf
    for _ in range(4):
        Fx = Fx + L.coarse_face_flux(q, 0, bc) / 4
        Fy = Fy + L.coarse_face_flux(q, 1, bc) / 4
        q, _, _ = L.learned_step_2d(q, dxf, dxf, dt, None, bc)
    qc0, qc1 = L.coarse_grain(qf), L.coarse_grain(q)
    dtc, dxc = 4 * dt, 4 * dxf
    pred = qc0 - (dtc / dxc) * (Fx[:, :, 1:] - Fx[:, :, :-1]) - (dtc / dxc) * (Fy[:, 1:] - Fy[:, :-1])
    assert np.abs(pred - qc1).max() <= 1e-13 * np.abs(qc1).max()
    # and a wrong weight breaks it
    bad = qc0 - (dtc / dxc) * 0.5 * (Fx[:, :, 1:] - Fx[:, :, :-1]) - (dtc / dxc) * (Fy[:, 1:] - Fy[:, :-1])
    assert np.abs(bad - qc1).max() > 1e-6


def test_loss_gradients_against_finite_differences():
    rng = np.random.default_rng(11)
    x = rng.standard_normal((40, 16))
    y = rng.standard_normal((40, 4)) * 0.5
    p = {k: v.astype(np.float64) for k, v in _random_params(12, scale=0.4).items()}
    loss, g = L.mlp_loss_grads(x, y, p)
    for name, idx in (("w1", (3, 5)), ("b1", (7,)), ("w2", (10, 20)), ("b2", (1,)),
                      ("w3", (2, 33)), ("b3", (3,))):
        h = 1e-6
        pp = {k: v.copy() for k, v in p.items()}
        pp[name][idx] += h
        lp, _ = L.mlp_loss_grads(x, y, pp)
        pp[name][idx] -= 2 * h
        lm, _ = L.mlp_loss_grads(x, y, pp)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[name][idx]) <= 1e-7 * max(1.0, abs(fd)), (name, fd, g[name][idx])


def test_adam_matches_the_published_first_step():
    """Adam's first step moves every parameter by lr * sign(grad) (bias
    correction makes m_hat / sqrt(v_hat) = g / |g|), up to eps."""
    p = {k: np.ones((2, 2), np.float32) for k in ("w1", "b1", "w2", "b2", "w3", "b3")}
    g = {k: np.array([[0.5, -2.0], [1e-3, -7.0]]) for k in p}
    m = {k: np.zeros((2, 2)) for k in p}
    v = {k: np.zeros((2, 2)) for k in p}
    L.adam_update(p, g, m, v, 1, 0.01)
    for k in p:
        np.testing.assert_allclose(p[k], 1.0 - 0.01 * np.sign(g[k]), rtol=0, atol=1e-5)


def test_blob_layout_round_trip():
    p = _random_params(13)
    blob = L.pack_blob(p)
    assert blob.size == L.BLOB_SIZE == 5548
    q = L.unpack_blob(blob)
    for k in p:
        np.testing.assert_array_equal(q[k], p[k])


def _torch_mlp(params, dtype):
    import torch
    net = torch.nn.Sequential(torch.nn.Linear(16, 64), torch.nn.Tanh(), torch.nn.Linear(64, 64),
                              torch.nn.Tanh(), torch.nn.Linear(64, 4)).to(dtype)
    with torch.no_grad():
        for layer, (w, b) in zip((net[0], net[2], net[4]), (("w1", "b1"), ("w2", "b2"), ("w3", "b3"))):
            layer.weight.copy_(torch.from_numpy(np.asarray(params[w], np.float64)))
            layer.bias.copy_(torch.from_numpy(np.asarray(params[b], np.float64)))
    return net


def test_network_definition_against_torch_layers():
    """The oracle's network is torch's Linear-Tanh-Linear-Tanh-Linear with
    weights stored [out][in]: the float64 loss and its gradients match torch
    autograd, and the bfloat16-operand forward stays within bfloat16 rounding
    of the float64 one (a transposed square W2 would not)."""
    import torch
    rng = np.random.default_rng(21)
    p = {k: v.astype(np.float64) for k, v in _random_params(22, scale=0.4).items()}
    x = rng.standard_normal((50, 16))
    y = rng.standard_normal((50, 4))
    loss, g = L.mlp_loss_grads(x, y, p)
    net = _torch_mlp(p, torch.float64)
    out = net(torch.from_numpy(x))
    tl = torch.mean((out - torch.from_numpy(y)) ** 2)
    tl.backward()
    assert abs(tl.item() - loss) <= 1e-14 * loss
    for layer, (w, b) in zip((net[0], net[2], net[4]), (("w1", "b1"), ("w2", "b2"), ("w3", "b3"))):
        np.testing.assert_allclose(g[w], layer.weight.grad.numpy(), rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(g[b], layer.bias.grad.numpy(), rtol=1e-11, atol=1e-14)
    p32 = {k: v.astype(np.float32) for k, v in p.items()}
    o_bf = L.mlp_forward(x.astype(np.float32), p32)
    with torch.no_grad():
        o64 = net(torch.from_numpy(x)).numpy()
    assert np.abs(o_bf - o64).max() <= 0.05 * np.abs(o64).max()
    pt = dict(p32)
    pt["w2"] = p32["w2"].T.copy()
    assert np.abs(L.mlp_forward(x.astype(np.float32), pt) - o64).max() > 0.1 * np.abs(o64).max()


# ---------------------------------------------------------------------------
# face frame and stencil order, pinned by hand values
# ---------------------------------------------------------------------------
def _labelled_grid(ny=4, nx=5):
    """q[m, y, x] = 1000 m + 10 y + x + 1: every value names its volume."""
    m, y, x = np.meshgrid(np.arange(4), np.arange(ny), np.arange(nx), indexing="ij")
    return (1000.0 * m + 10.0 * y + x + 1.0)


def test_face_features_match_hand_values():
    """The 16 features of chosen x and y faces (interior, periodic and
    transmissive boundaries) equal the hand-written stencil of
    tests/golden/learned_face_stencil.txt: volumes i-2 .. i+1 along the
    normal, each as (rho, j_n, j_t, E).  A reversed stencil, a swapped j_n /
    j_t or a wrong halo rule fails here."""
    from conftest import read_golden
    q = _labelled_grid()
    rows = read_golden("learned_face_stencil.txt")
    assert len(rows) == 7
    for name, vals in rows:
        bc = ("periodic", "transmissive")[int(vals[0])]
        k, row, col = int(vals[1]), int(vals[2]), int(vals[3])
        want = np.array(vals[4:])
        assert want.size == 16, name
        Lq, Rq, feats, ind = L.face_data(q, k, bc)
        assert feats.shape == ((16, 4, 6) if k == 0 else (16, 5, 5)), name
        np.testing.assert_array_equal(feats[:, row, col], want, err_msg=name)
        # L and R are the two middle volumes (grid axes), and the indicator
        # compares their densities
        assert Lq[0, row, col] == want[4] and Rq[0, row, col] == want[8], name
        assert ind[row, col] == abs(want[8] - want[4]) / min(want[4], want[8]), name


def test_face_frame_of_each_axis():
    """to_face_frame reads (rho, j_n, j_t, E): j_x first on x faces, j_y first
    on y faces."""
    q = np.array([1.0, 2.0, 3.0, 4.0])
    np.testing.assert_array_equal(L.to_face_frame(q, 0), [1.0, 2.0, 3.0, 4.0])
    np.testing.assert_array_equal(L.to_face_frame(q, 1), [1.0, 3.0, 2.0, 4.0])


def test_targets_are_face_frame_differences():
    """A reference flux that exceeds the coarse Rusanov flux by D (grid axes:
    rho, j_x, j_y, E) gives the target D on x faces and (D_rho, D_jy, D_jx,
    D_E) on y faces, x faces first in row-major order."""
    qc = _random_grid(6, 41)
    D = np.array([0.5, -1.25, 2.0, 4.0])
    stars = []
    for k in (0, 1):
        Lq, Rq, _, _ = L.face_data(qc, k, "periodic")
        stars.append(L.rusanov_2d(Lq, Rq, k) + D[:, None, None])
    feats, targ, ind = L.face_samples(qc, stars[0], stars[1], "periodic")
    nx_faces = 6 * 7
    assert feats.shape == (2 * nx_faces, 16) and targ.shape == (2 * nx_faces, 4)
    np.testing.assert_allclose(targ[:nx_faces], np.broadcast_to(D, (nx_faces, 4)), atol=1e-12)
    np.testing.assert_allclose(targ[nx_faces:], np.broadcast_to(D[[0, 2, 1, 3]], (nx_faces, 4)),
                               atol=1e-12)
    # row-major face order: x face (row 2, column 3) and y face (row 4, column 1)
    _, _, fx, _ = L.face_data(qc, 0, "periodic")
    _, _, fy, _ = L.face_data(qc, 1, "periodic")
    np.testing.assert_array_equal(feats[2 * 7 + 3], fx[:, 2, 3])
    np.testing.assert_array_equal(feats[nx_faces + 4 * 6 + 1], fy[:, 4, 1])


def test_axis_swap_gives_identical_features():
    """Transposing the grid and swapping j_x with j_y turns x faces into y
    faces with the same 16 features and indicator (the face frame makes the
    features axis-free)."""
    q = _random_grid(7, 42)
    qt = q[[0, 2, 1, 3]].transpose(0, 2, 1).copy()
    for bc in ("periodic", "transmissive"):
        _, _, fx, ix = L.face_data(q, 0, bc)
        _, _, fy, iy = L.face_data(qt, 1, bc)
        np.testing.assert_array_equal(fy, fx.transpose(0, 2, 1))
        np.testing.assert_array_equal(iy, ix.T)
