"""Pins of the oracle's local time stepping over uneven 3-D batches
(Section 4: every patch advances with a time step from its own maximum
eigenvalue; Section 2: factor-3 refinement levels)."""
import math

import numpy as np
import pytest

import oracle
from paper_2302_09005_amd import workloads as W

GAMMA = 1.4


def _self_periodic(sizes, levels, blocks):
    """An UnevenBatch whose patch b holds blocks[b] ([5, p, p, p])."""
    batch = W.UnevenBatch(np.array(sizes), np.array(levels))
    q = np.concatenate([np.asarray(b, dtype=np.float64).reshape(-1) for b in blocks])
    return batch, q


def _run(batch, q, steps, dt=None):
    dx = np.repeat(batch.dx[:, None], 3, axis=1)
    return oracle.run_local_steps(batch.offsets(), batch.sizes, dx, batch.neighbours(), q, steps,
                                  dt=dt)


def _smooth_block(p, seed):
    b, q = W.uneven_batch(1, seed, sizes=(p,), ratio=(1,), levels=(3,))
    return q.reshape(5, p, p, p)


def test_local_dt_is_the_cfl_rule_per_patch():
    rng = np.random.default_rng(0)
    dx = rng.uniform(1e-3, 1e-1, size=(7, 3))
    lam = rng.uniform(0.5, 3.0, size=7)
    dt = oracle.local_dt(dx, lam, 3, 0.4)
    for b in range(7):
        ref, lam_b = oracle.cfl_dt(dx[b:b + 1], lam[b:b + 1], 3, 0.4)
        assert dt[b] == ref and lam_b == lam[b]
    # NaN maximum gives a NaN step
    assert np.isnan(oracle.local_dt(dx[:1], np.array([np.nan]), 3))[0]


def test_uniform_state_closed_form_and_free_stream():
    """A uniform patch stays uniform bit for bit; its step is
    cfl * dx / (3 (|u|_max + c)) with c = sqrt(gamma p / rho), and t adds up."""
    rho, u, pres = 0.8, (0.3, -0.2, 0.1), 1.3
    blocks, sizes = [], (4, 8, 16)
    for p in sizes:
        prim = W.to_conserved(np.full((p, p, p), rho), [np.full((p, p, p), v) for v in u],
                              np.full((p, p, p), pres))
        blocks.append(prim)
    batch, q = _self_periodic(sizes, (2, 3, 4), blocks)
    q1, dt, t, me = _run(batch, q, 3)
    assert np.array_equal(q1, q)
    c = math.sqrt(GAMMA * pres / rho)
    lam = 0.3 + c
    np.testing.assert_allclose(me, lam, rtol=4 * 2.0 ** -53)
    np.testing.assert_allclose(dt, 0.4 * batch.dx / (3 * lam), rtol=8 * 2.0 ** -53)
    np.testing.assert_allclose(t, 3 * dt, rtol=8 * 2.0 ** -53)


def test_tiled_patches_give_tiled_results_exactly():
    """A p^3 field tiled 2x2x2 into a (2p)^3 patch of the same dx is the same
    periodic problem: after every step the big patch is the tiling of the
    small one, bit for bit, with the same t and dt."""
    small4 = _smooth_block(4, 11)
    small8 = _smooth_block(8, 12)
    tile = lambda a: np.tile(a, (1, 2, 2, 2))
    sizes = (4, 8, 8, 16)
    batch = W.UnevenBatch(np.array(sizes), np.array([3, 3, 3, 3]))
    dx = np.array([0.01, 0.01, 0.005, 0.005])   # each pair shares its dx
    q = np.concatenate([small4.ravel(), tile(small4).ravel(), small8.ravel(),
                        tile(small8).ravel()])
    dxa = np.repeat(dx[:, None], 3, axis=1)
    q1, dt, t, me = oracle.run_local_steps(batch.offsets(), batch.sizes, dxa,
                                           batch.neighbours(), q, 4)
    blk = [batch.block(q1, b) for b in range(4)]
    assert np.array_equal(blk[1], tile(blk[0]))
    assert np.array_equal(blk[3], tile(blk[2]))
    assert dt[0] == dt[1] and dt[2] == dt[3] and t[0] == t[1] and t[2] == t[3]
    assert me[0] == me[1] and me[2] == me[3]
    assert not np.array_equal(blk[0], small4)   # something happened


def test_agrees_with_the_global_step_when_all_patches_are_alike():
    """Identical self-periodic patches all take the global CFL step, so the
    local run equals the global driver on one self-periodic patch."""
    blk = _smooth_block(8, 5)
    batch, q = _self_periodic((8, 8, 8), (3, 3, 3), [blk, blk, blk])
    q1, dt, t, _ = _run(batch, q, 5)
    grid = W.PatchGrid(3, 8, (1, 1, 1), float(batch.dx[0]))
    glob = blk
    ref, t_ref, dts = oracle.run_steps(grid.offsets(), float(batch.dx[0]), grid.pack(glob),
                                       grid.neighbours(), 3, 8, 5)
    for b in range(3):
        np.testing.assert_array_equal(batch.block(q1, b), grid.unpack(ref))
    np.testing.assert_allclose(t, t_ref, rtol=1e-15)
    assert dt[0] == dt[1] == dt[2]


def test_levels_scale_dt_by_three():
    """The update depends on dt/dx only: the same field one level finer takes
    a step three times smaller and gives the same state (to rounding)."""
    blk = _smooth_block(8, 9)
    batch, q = _self_periodic((8, 8), (2, 3), [blk, blk])
    q1, dt, t, _ = _run(batch, q, 2)
    np.testing.assert_allclose(dt[0] / dt[1], 3.0, rtol=1e-14)
    a, b = batch.block(q1, 0), batch.block(q1, 1)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def test_self_periodic_patches_conserve_their_totals():
    batch, q = W.uneven_batch(60, 4)
    q1, _, _, _ = _run(batch, q, 5)
    for b in range(batch.n):
        before, after = batch.block(q, b), batch.block(q1, b)
        for k in range(5):
            scale = math.fsum(np.abs(before[k]).ravel())
            assert abs(math.fsum(after[k].ravel()) - math.fsum(before[k].ravel())) \
                <= 1e-13 * scale


def test_patches_are_independent():
    """A patch's result does not depend on the other patches of the batch."""
    batch, q = W.uneven_batch(40, 6)
    q1, dt, t, me = _run(batch, q, 3)
    for b in (0, 7, 23):
        p = int(batch.sizes[b])
        one = W.UnevenBatch(batch.sizes[b:b + 1], batch.levels[b:b + 1])
        r, dt1, t1, me1 = _run(one, batch.block(q, b).ravel().copy(), 3)
        np.testing.assert_array_equal(r.reshape(5, p, p, p), batch.block(q1, b))
        assert dt1[0] == dt[b] and t1[0] == t[b] and me1[0] == me[b]


def test_uneven_batch_recipe():
    batch, q = W.uneven_batch(7000, 0)
    frac = np.array([(batch.sizes == p).mean() for p in (4, 8, 16)])
    np.testing.assert_allclose(frac, np.array([4, 2, 1]) / 7, atol=0.02)
    assert set(np.unique(batch.levels)) == {2, 3, 4}
    np.testing.assert_allclose(batch.dx, 3.0 ** -batch.levels.astype(float) / batch.sizes)
    assert np.isfinite(q).all() and q.size == batch.buffer_len()
    rho = np.concatenate([batch.block(q, b)[0].ravel() for b in range(50)])
    assert rho.min() >= 0.5 and rho.max() <= 1.5
    with pytest.raises(ValueError):
        W.UnevenBatch(np.array([4, 8]), np.array([2]))
