"""fv_step_gather_pipelined: the fused step with its CFL reduction moved to the
next launch (each launch takes its time step from the maxima the previous one
folded).  Through the C ABI a pipelined run must equal a run of
fv_step_gather bit for bit: the state after every step, the time step each
step takes, the per-patch maxima and the Lambda each time step came from;
for every kernel shape (one patch per wave, several patches per wave, several
waves per patch), in FP64 and FP32, eagerly and replayed from HIP graphs
whose step count is not a multiple of the three-launch slot cycle."""
import sys

import numpy as np
import pytest

from paper_2302_09005_amd import fv
from paper_2302_09005_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    fv.library()
    yield


def _random_state(grid, seed):
    rng = np.random.default_rng(seed)
    shape = grid.shape
    return W.to_conserved(rng.uniform(0.5, 1.5, shape),
                          [rng.uniform(-0.5, 0.5, shape) for _ in range(grid.d)],
                          rng.uniform(0.5, 2.0, shape))


def _grid(dim, p, counts, seed):
    grid = W.PatchGrid(dim, p, counts, 1.0 / (p * counts[0]))
    return grid, _random_state(grid, seed)


def _pair(grid, q, dtype):
    desc = grid.descriptors(out_halo=False, in_halo=False)
    mk = lambda mode: fv.Stepper(desc, grid.neighbours(), grid.pack_compact(q), dim=grid.d,
                                 p=grid.p, mode=mode, dtype=dtype)
    return mk("fused"), mk("pipelined")


# (dim, p, patches per axis): one patch per wave (3-D 8^3, 2-D 16^2 in row
# chunks), several patches per wave (3-D 4^3, 2-D 4^2), several waves per
# patch (3-D 16^3); ragged counts so that the last workgroup group is partial
CASES = [(3, 8, (5, 4, 3)), (2, 16, (9, 7)), (3, 4, (6, 5, 4)), (2, 4, (13, 11)),
         (3, 16, (3, 2, 2)), (2, 17, (5, 3))]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("dim,p,counts", CASES)
def test_pipelined_run_equals_fused_run_bitwise(dim, p, counts, dtype):
    import torch
    grid, q = _grid(dim, p, counts, seed=11 + p)
    ref, st = _pair(grid, q, dtype)
    _say(f"[pipelined vs fused] dim={dim} p={p} n={grid.n} {np.dtype(dtype).name}")
    lam_prev = None
    for k in range(12):
        ref.step()
        st.step()
        torch.cuda.synchronize()
        assert torch.equal(st.state(), ref.state()), f"state differs after step {k}"
        assert torch.equal(st.last_dt(), ref.last_dt()), f"dt differs at step {k}"
        assert torch.equal(st.per_patch, ref.per_patch), f"maxima differ at step {k}"
        if lam_prev is not None:
            # the Lambda a pipelined step's dt came from: the previous new state's
            assert torch.equal(st.lam, lam_prev), f"Lambda differs at step {k}"
        lam_prev = ref.lam.clone()
    assert bool(torch.isfinite(st.state()).all())


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_headline_workload_100_steps_bitwise(dtype):
    """The benchmarked workload (4096 x 8^3, FP64 and FP32 state) over 100
    steps: the same state and time-step sequence as fv_step_gather."""
    import torch
    grid, q = W.grid_3d_random_smooth(16, 8, seed=0)
    ref, st = _pair(grid, q, dtype)
    dts_ref, dts = [], []
    for _ in range(100):
        ref.step()
        st.step()
        dts_ref.append(ref.last_dt().clone())
        dts.append(st.last_dt().clone())
    torch.cuda.synchronize()
    assert torch.equal(st.state(), ref.state())
    assert torch.equal(torch.cat(dts), torch.cat(dts_ref))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("steps", [7, 6])
def test_graph_replays_equal_eager_bitwise(steps, dtype):
    """Captured as HIP graphs the way the benchmark does (one graph per start
    position of the six-step argument cycle when the step count is not a
    multiple of it), replayed several times with other eager work and
    synchronisations between the replays: every replay leaves the eager run's
    state, time step and maxima bit for bit."""
    import torch
    import bench
    grid, q = W.grid_3d_random_smooth(6, 8, seed=5)
    desc = grid.descriptors(out_halo=False, in_halo=False)
    mk = lambda: fv.Stepper(desc, grid.neighbours(), grid.pack_compact(q), dim=3, p=8,
                            mode="pipelined", dtype=dtype)
    g_st, e_st = mk(), mk()
    with pytest.raises(ValueError):
        bench.StepGraphs(g_st, steps)  # the first step reads the given dt: not capturable
    for st in (g_st, e_st):
        for _ in range(2):
            st.step()
    graphs = bench.StepGraphs(g_st, steps)
    assert len(graphs.graphs) == 6 // np.gcd(steps, 6)
    x = torch.randn(1 << 16, device="cuda", dtype=torch.float64)
    for rep in range(4):
        graphs.replay()
        for _ in range(steps):
            e_st.step()
        y = float((x * x).sum().item())
        torch.cuda.synchronize()
        _say(f"[pipelined graph replay {rep}, {steps} steps, {np.dtype(dtype).name}] {y:.3f}")
        assert torch.equal(g_st.b if (rep + 1) * steps % 2 else g_st.a, e_st.state())
        assert torch.equal(g_st.dt_used, e_st.dt_used)
        assert torch.equal(g_st.per_patch, e_st.per_patch)
    graphs.finish()
    assert g_st.position() == e_st.position()
    # the host side is back in step with the data: eager steps continue the run
    for _ in range(4):
        g_st.step()
        e_st.step()
    torch.cuda.synchronize()
    assert torch.equal(g_st.state(), e_st.state())
    assert torch.equal(g_st.last_dt(), e_st.last_dt())


def test_nan_state_gives_nan_time_step_next():
    """A NaN in the state reaches the next launch's Lambda and time step, as
    in the fused step."""
    import torch
    grid, q = _grid(3, 8, (4, 4, 4), seed=3)
    _, st = _pair(grid, q, None)
    st.step()
    torch.cuda.synchronize()
    assert np.isfinite(st.last_dt().item())
    st.a[17] = float("nan")
    st.step()   # takes the finite dt folded before the NaN was planted
    st.step()   # its maxima include the NaN patch
    torch.cuda.synchronize()
    assert np.isnan(st.last_dt().item()) and np.isnan(st.lam.item())


def test_workspace_reuse_and_fresh_run():
    """A second run on the same workspace that continues the phase sequence
    gives the same results as a run on a fresh workspace."""
    import torch
    grid, q = _grid(3, 8, (4, 3, 3), seed=9)
    desc = grid.descriptors(out_halo=False, in_halo=False)
    n, dim, p = grid.n, 3, 8
    pat = fv.upload_patches(desc, "cuda", dim=dim, p=p, q_out_halo=False,
                            q_in_len=q.size, q_out_len=q.size, q_in_halo=False)
    nbr = torch.from_numpy(grid.neighbours()).cuda()
    ws = torch.zeros(fv.pipelined_workspace_words(n, dim, p), dtype=torch.int64, device="cuda")
    me = torch.empty(n, dtype=torch.float64, device="cuda")
    dt0 = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
    used = torch.empty(1, dtype=torch.float64, device="cuda")

    def run(first_phase, workspace, steps=5):
        a = torch.from_numpy(grid.pack_compact(q)).cuda()
        b = torch.empty_like(a)
        out = []
        for k in range(steps):
            fv.step_gather_pipelined(pat, nbr, a, b, workspace, dim=dim, p=p,
                                     phase=(first_phase + k) % 3, dt_in=dt0 if k == 0 else None,
                                     dt_used=used, max_eig=me)
            out.append(used.clone())
            a, b = b, a
        torch.cuda.synchronize()
        return a, torch.cat(out)

    a1, d1 = run(0, ws)           # phases 0..4 % 3; leaves sets dirty
    a2, d2 = run(5 % 3, ws)       # continues the phase sequence on the same words
    fresh = torch.zeros_like(ws)
    a3, d3 = run(1, fresh)
    assert torch.equal(a1, a2) and torch.equal(a1, a3)
    assert torch.equal(d1, d2) and torch.equal(d1, d3)
    assert d1[0].item() == 1e-3
