"""GPU parity for uneven 3-D batches with local time stepping: the HIP path
(fv_step_local through the C ABI, every schedule) against the CPU oracle's
run_local_steps.

Bar (FP64): normwise relative error per unknown <= 1e-12 (as for the
regular batches), per-patch maxima, local dt and t within 1e-14 after one
step and 1e-13 after several; every schedule gives the same bits; FP32 state
within 1e-5 relative L2 and L-infinity of the FP64 oracle.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2302_09005_amd import autotune, fv
from paper_2302_09005_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL32 = 1e-5


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    fv.library()


def by_unknown(batch, flat):
    """[5, cells] array: every patch's values of unknown k, patch order."""
    flat = np.asarray(flat, dtype=np.float64)
    return np.concatenate([batch.block(flat, b).reshape(5, -1) for b in range(batch.n)], axis=1)


def normwise(got, ref):
    scale = np.abs(ref).max()
    return max(np.abs(got[k] - ref[k]).max() / (np.abs(ref[k]).max() or scale)
               for k in range(ref.shape[0]))


def rel_l2_linf(got, ref):
    l2 = max(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k]) for k in range(5))
    li = max(np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max() for k in range(5))
    return l2, li


def oracle_run(batch, q, steps):
    dx = np.repeat(batch.dx[:, None], 3, axis=1)
    return oracle.run_local_steps(batch.offsets(), batch.sizes, dx, batch.neighbours(), q, steps)


def gpu_run(batch, q, steps, schedule="persistent", workgroups=0, dtype=None):
    import torch
    st = fv.LocalStepper(batch.descriptors(), batch.neighbours(), q, schedule=schedule,
                         workgroups=workgroups, dtype=dtype)
    for _ in range(steps):
        st.step()
    torch.cuda.synchronize()
    desc = st.descriptors()
    return st.state().cpu().numpy(), desc["dt"].copy(), desc["t"].copy(), st.max_eig(), st


SCHEDULES = [("per_size", 0), ("persistent", 0), ("persistent", 5), ("patchwise", 0)]


@pytest.mark.parametrize("schedule,wg", SCHEDULES)
@pytest.mark.parametrize("steps", [1, 5])
def test_uneven_parity(schedule, wg, steps):
    batch, q = W.uneven_batch(150, 3)
    _say(f"[uneven parity] 150 patches seed 3, {schedule} wg={wg}, {steps} steps")
    ref, dt_ref, t_ref, me_ref = oracle_run(batch, q, steps)
    got, dt, t, me, _ = gpu_run(batch, q, steps, schedule, wg)
    err = normwise(by_unknown(batch, got), by_unknown(batch, ref))
    _say(f"    normwise error {err:.2e}")
    assert err <= TOL
    rt = 1e-14 if steps == 1 else 1e-13
    np.testing.assert_allclose(me, me_ref, rtol=rt, atol=0)
    np.testing.assert_allclose(dt, dt_ref, rtol=rt, atol=0)
    np.testing.assert_allclose(t, t_ref, rtol=rt, atol=0)


def test_schedules_give_identical_bits():
    batch, q = W.uneven_batch(200, 8)
    runs = [gpu_run(batch, q, 3, s, wg) for s, wg in SCHEDULES + [("persistent", 1)]]
    for r in runs[1:]:
        for a, b in zip(runs[0][:4], r[:4]):
            assert np.array_equal(a, b)


def test_unsorted_batch_through_the_abi():
    """fv_step_local on descriptors in the caller's (unsorted) order: the
    plan's order array carries the indirection."""
    import torch
    batch, q = W.uneven_batch(90, 12)
    dx = np.repeat(batch.dx[:, None], 3, axis=1)
    _, dt0, _, _ = oracle.run_local_steps(batch.offsets(), batch.sizes, dx, batch.neighbours(),
                                          q, 0)
    ref, dt_ref, t_ref, me_ref = oracle.run_local_steps(batch.offsets(), batch.sizes, dx,
                                                        batch.neighbours(), q, 1, dt=dt0)
    desc = batch.descriptors()
    desc["dt"] = dt0
    desc["t"] = 0.25
    plan = fv.Plan(desc)
    assert not np.array_equal(plan.order, np.arange(batch.n))
    for sched in ("persistent", "per_size"):
        pd = fv.upload_patches(desc)
        nb = torch.from_numpy(batch.neighbours()).cuda()
        qi = torch.from_numpy(q).cuda()
        qo = torch.full_like(qi, float("nan"))
        me = torch.empty(batch.n, dtype=torch.float64, device="cuda")
        fv.step_local(pd, nb, plan, qi, qo, max_eig=me, schedule=sched)
        torch.cuda.synchronize()
        out = pd.cpu().numpy().view(W.PATCH_DTYPE)
        assert normwise(by_unknown(batch, qo.cpu().numpy()), by_unknown(batch, ref)) <= TOL
        np.testing.assert_allclose(me.cpu().numpy(), me_ref, rtol=1e-14)
        np.testing.assert_allclose(out["dt"], dt_ref, rtol=1e-14)
        assert np.array_equal(out["t"], 0.25 + dt0)
        assert np.array_equal(out["q_in"], desc["q_in"]) and np.array_equal(out["dx"], desc["dx"])


def test_tiled_patches_exact_on_gpu():
    """A p^3 field tiled 2x2x2 into a (2p)^3 patch of the same dx evolves as
    the tiling of the small patch's result, bit for bit."""
    small = {}
    for p, seed in ((4, 21), (8, 22)):
        _, qs = W.uneven_batch(1, seed, sizes=(p,), ratio=(1,), levels=(3,))
        small[p] = qs.reshape(5, p, p, p)
    tile = lambda a: np.tile(a, (1, 2, 2, 2))
    batch = W.UnevenBatch(np.array([4, 8, 8, 16]), np.array([3, 3, 3, 3]))
    desc_dx = np.array([0.01, 0.01, 0.005, 0.005])
    q = np.concatenate([small[4].ravel(), tile(small[4]).ravel(), small[8].ravel(),
                        tile(small[8]).ravel()])
    desc = batch.descriptors()
    desc["dx"] = desc_dx[:, None]
    import torch
    st = fv.LocalStepper(desc, batch.neighbours(), q)
    for _ in range(4):
        st.step()
    torch.cuda.synchronize()
    got = st.state().cpu().numpy()
    blk = [batch.block(got, b) for b in range(4)]
    assert np.array_equal(blk[1], tile(blk[0])) and np.array_equal(blk[3], tile(blk[2]))
    d = st.descriptors()
    assert d["dt"][0] == d["dt"][1] and d["dt"][2] == d["dt"][3]


@pytest.mark.parametrize("sizes", [(16, 16, 16), (4,) * 17 + (8,) * 5, (4, 8, 16), (8,)])
def test_ragged_and_single_class_batches(sizes):
    rng = np.random.default_rng(len(sizes))
    n = len(sizes)
    batch = W.UnevenBatch(np.array(sizes), rng.choice([2, 3, 4], size=n))
    blocks = []
    for b, p in enumerate(sizes):
        _, qs = W.uneven_batch(1, 100 + b, sizes=(p,), ratio=(1,), levels=(3,))
        blocks.append(qs)
    q = np.concatenate(blocks)
    ref, dt_ref, t_ref, me_ref = oracle_run(batch, q, 2)
    for sched, wg in (("persistent", 0), ("per_size", 0), ("persistent", 1)):
        got, dt, t, me, _ = gpu_run(batch, q, 2, sched, wg)
        assert normwise(by_unknown(batch, got), by_unknown(batch, ref)) <= TOL
        np.testing.assert_allclose(dt, dt_ref, rtol=1e-13)
        np.testing.assert_allclose(t, t_ref, rtol=1e-13)


def test_uniform_patches_stay_uniform_bitwise():
    sizes = (4, 8, 16, 4, 8)
    batch = W.UnevenBatch(np.array(sizes), np.array([2, 3, 4, 4, 2]))
    state = (0.9, (0.2, -0.3, 0.4), 1.7)
    q = np.concatenate([W.to_conserved(np.full((p,) * 3, state[0]),
                                       [np.full((p,) * 3, v) for v in state[1]],
                                       np.full((p,) * 3, state[2])).ravel() for p in sizes])
    got, dt, t, me, _ = gpu_run(batch, q, 3)
    assert np.array_equal(got, q)
    _, dt_ref, t_ref, me_ref = oracle_run(batch, q, 3)
    np.testing.assert_allclose(me, me_ref, rtol=1e-15)
    np.testing.assert_allclose(dt, dt_ref, rtol=1e-15)


def test_graph_replay_matches_eager():
    """Ten steps captured in one graph and replayed three times, with other
    eager work and synchronisations between replays, match ten eager steps
    after every replay, bit for bit (state, dt, t)."""
    import torch
    batch, q = W.uneven_batch(120, 31)
    g_st = fv.LocalStepper(batch.descriptors(), batch.neighbours(), q)
    e_st = fv.LocalStepper(batch.descriptors(), batch.neighbours(), q)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for _ in range(10):
                g_st.step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    x = torch.randn(1 << 16, device="cuda", dtype=torch.float64)
    for rep in range(3):
        graph.replay()
        for _ in range(10):
            e_st.step()
        y = (x * x).sum().item()   # unrelated eager work and a sync
        torch.cuda.synchronize()
        _say(f"[graph replay {rep}] {y:.3f}")
        assert torch.equal(g_st.state(), e_st.state())
        assert torch.equal(g_st.patches, e_st.patches)
        assert torch.equal(g_st.per_patch, e_st.per_patch)


@pytest.mark.parametrize("steps", [1, 10, 100])
def test_fp32_uneven_errors(steps):
    batch, q = W.uneven_batch(150, 41)
    ref, _, _, _ = oracle_run(batch, q, steps)
    got, _, _, me, _ = gpu_run(batch, q, steps, dtype=np.float32)
    l2, li = rel_l2_linf(by_unknown(batch, got), by_unknown(batch, ref))
    _say(f"[fp32 uneven vs fp64 oracle] {steps} steps: rel L2 {l2:.2e} rel Linf {li:.2e}")
    assert l2 <= TOL32 and li <= TOL32


def test_full_size_batch_sampled_patches():
    """The 20 000-patch batch in the launch the benchmark times, one step;
    64 sampled patches checked against the oracle one by one (the patches
    are independent)."""
    batch, q = W.uneven_batch(20000, 0)
    _say(f"[uneven full size] 20000 patches, {batch.cells} volumes")
    got, dt, t, me, _ = gpu_run(batch, q, 1, "persistent", 0)
    rng = np.random.default_rng(0)
    pick = np.sort(rng.choice(batch.n, size=64, replace=False))
    sub = W.UnevenBatch(batch.sizes[pick], batch.levels[pick])
    qs = np.concatenate([batch.block(q, b).ravel() for b in pick])
    ref, dt_ref, t_ref, me_ref = oracle_run(sub, qs, 1)
    gs = np.concatenate([batch.block(got, b).ravel() for b in pick])
    assert normwise(by_unknown(sub, gs), by_unknown(sub, ref)) <= TOL
    np.testing.assert_allclose(dt[pick], dt_ref, rtol=1e-14)
    np.testing.assert_allclose(me[pick], me_ref, rtol=1e-14)
    assert np.isfinite(got).all()


def test_fp32_full_size_batch_sampled_patches_at_1_10_100_steps():
    """The 20 000-patch uneven batch with FP32 state (the benchmarked FP32
    uneven run), 100 local steps; 64 sampled patches against the FP64 oracle
    after 1, 10 and 100 steps (self-periodic patches with local time steps
    evolve independently, so a sample is its own small batch)."""
    import torch
    batch, q = W.uneven_batch(20000, 0)
    st = fv.LocalStepper(batch.descriptors(), batch.neighbours(), q, dtype=np.float32)
    rng = np.random.default_rng(1)
    pick = np.sort(rng.choice(batch.n, size=64, replace=False))
    sub = W.UnevenBatch(batch.sizes[pick], batch.levels[pick])
    ref = np.concatenate([batch.block(q, b).ravel() for b in pick])
    dx = np.repeat(sub.dx[:, None], 3, axis=1)
    dt = t = None
    done = 0
    for k in (1, 10, 100):
        for _ in range(k - done):
            st.step()
        torch.cuda.synchronize()
        got = st.state().cpu().numpy().astype(np.float64)
        ref, dt, t, _ = oracle.run_local_steps(sub.offsets(), sub.sizes, dx, sub.neighbours(),
                                               ref, k - done, dt=dt, t=t)
        done = k
        gs = np.concatenate([batch.block(got, b).ravel() for b in pick])
        l2, li = rel_l2_linf(by_unknown(sub, gs), by_unknown(sub, ref))
        _say(f"[fp32 uneven 20000, 64 sampled vs fp64 oracle] {k} steps: rel L2 {l2:.2e} "
             f"rel Linf {li:.2e}")
        assert l2 <= TOL32 and li <= TOL32
        desc = st.descriptors()
        np.testing.assert_allclose(desc["t"][pick], t, rtol=1e-5)


def test_autotuner_restores_the_run_and_picks_a_candidate():
    import torch
    batch, q = W.uneven_batch(400, 51)
    st = fv.LocalStepper(batch.descriptors(), batch.neighbours(), q)
    ref = fv.LocalStepper(batch.descriptors(), batch.neighbours(), q)
    best, table = autotune.tune(st, steps=2, warmup=1, patchwise=True)
    _say("[autotune 400 patches] " + ", ".join(f"{s}/{w}: {u:.1f} us" for s, w, u in table))
    assert best in [(s, w) for s, w, _ in table]
    for _ in range(2):
        st.step()
        ref.step()
    torch.cuda.synchronize()
    assert torch.equal(st.state(), ref.state()) and torch.equal(st.patches, ref.patches)
