"""fv_step_halo: the paper's halo'd layout, one launch per step (update, the
face-halo exchange of the new state pushed into the output halos, next CFL
step).  Through the C ABI it must equal fv_batch_update (halo'd output), then
fv_fill_halo on the output, then fv_cfl_timestep, bit for bit: interior, face
halos, untouched edge and corner halos, per-patch maxima and the time step.
Over many steps it must equal the three-launch stepper and the oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_2302_09005_amd import fv
from paper_2302_09005_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    fv.library()
    yield


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _normwise(got, want, s):
    """max over unknowns of max |got - want| / max |want| (the largest
    unknown's scale for an unknown that is identically zero)."""
    got, want = np.asarray(got).reshape(s, -1), np.asarray(want).reshape(s, -1)
    scale = np.abs(want).max()
    den = np.abs(want).max(axis=1)
    den = np.where(den > 0, den, scale)
    return (np.abs(got - want).max(axis=1) / den).max()


def _random_state(grid, seed):
    rng = np.random.default_rng(seed)
    shape = grid.shape
    return W.to_conserved(rng.uniform(0.5, 1.5, shape),
                          [rng.uniform(-0.5, 0.5, shape) for _ in range(grid.d)],
                          rng.uniform(0.5, 2.0, shape))


def _both(grid, q, dt0):
    """(fused step, reference three launches): q_out buffers, maxima, dt_next."""
    import torch
    d, p, n = grid.d, grid.p, grid.n
    flat = grid.pack(q, corners=-7.0)
    desc = grid.descriptors(dt=dt0)
    pd = fv.upload_patches(desc)
    nbr = _dev(grid.neighbours())
    qin = _dev(flat)
    dt = torch.tensor([dt0], dtype=torch.float64, device="cuda")
    out = []
    for fused in (True, False):
        qout = torch.full_like(qin, -123.0)
        me = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
        dt_next = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        lam = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        if fused:
            ws = torch.zeros(fv.step_workspace_words(n, d, p), dtype=torch.int64, device="cuda")
            fv.step_halo(pd, nbr, qin, qout, dt, dt_next, ws, dim=d, p=p, max_eig=me,
                         lambda_out=lam)
        else:
            fv.batch_update(pd, qin, qout, dim=d, p=p, q_out_halo=True, dt=dt, max_eig=me)
            fv.fill_halo(pd, nbr, qout, dim=d, p=p, which=fv.FV_OFFSETS_OUT)
            fv.cfl_timestep(pd, me, dim=d, lambda_out=lam, dt_out=dt_next)
        torch.cuda.synchronize()
        if fused:
            assert (ws.cpu().numpy() == 0).all()
        out.append((qout.cpu().numpy(), me.cpu().numpy(), dt_next.item(), lam.item()))
    return out


@pytest.mark.parametrize("d,p,counts", [(2, 4, (5, 3)), (2, 8, (3, 3)), (2, 16, (3, 2)),
                                        (2, 17, (3, 2)), (2, 32, (2, 2)), (3, 4, (3, 2, 2)),
                                        (3, 8, (3, 2, 2)), (3, 16, (2, 2, 1))])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_step_halo_equals_update_fill_cfl_bitwise(d, p, counts, bc):
    _say(f"[step_halo d={d} p={p} counts={counts} bc={bc}]")
    bcs = (W.PERIODIC,) * d if bc == "periodic" else (W.TRANSMISSIVE,) + (W.PERIODIC,) * (d - 1)
    grid = W.PatchGrid(d, p, counts, 1.0 / (counts[0] * p), bcs)
    q = _random_state(grid, 10 * d + p)
    per, _ = oracle.max_eigenvalue(grid.offsets(), grid.pack(q), d, p, True)
    dt0, _ = oracle.cfl_dt(np.full((grid.n, 3), grid.dx), per, d)
    (a, me_a, dt_a, lam_a), (b, me_b, dt_b, lam_b) = _both(grid, q, dt0)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(me_a, me_b)
    assert dt_a == dt_b and lam_a == lam_b
    # the interior against the oracle; the face halos against a global repack
    desc = grid.descriptors(dt=dt0)
    ref, me_ref = oracle.fv_step(desc["q_in"], desc["q_out"], desc["dx"], desc["dt"],
                                 grid.pack(q), d, p, out_halo=True)
    new = grid.unpack(ref)
    got = grid.unpack(a)
    err = _normwise(got, new, d + 2)
    assert err <= TOL, err
    np.testing.assert_allclose(me_a, me_ref, rtol=1e-14, atol=0)
    # face halos: what packing the new global state gives; edges and corners
    # of every output block were never written
    want = grid.pack(got, corners=-123.0)
    np.testing.assert_array_equal(a, want)


def test_steps_match_three_launch_stepper_and_oracle():
    """100 steps of 4096 x 8^3: the one-launch stepper equals the paper's
    three-launch stepper bit for bit (state with halos, dt sequence), and
    the oracle's 100 steps to 1e-12."""
    import torch
    _say("[step_halo 4096x8^3, 100 steps vs three launches and oracle]")
    grid, q = W.grid_3d_random_smooth(16, 8, seed=0)
    flat = grid.pack(q)
    desc = grid.descriptors()
    runs = []
    for mode in ("halo_step", "halo"):
        st = fv.Stepper(desc, grid.neighbours(), flat, dim=3, p=8, mode=mode)
        dts = []
        for _ in range(100):
            st.step()
            dts.append(st.last_dt().item())
        torch.cuda.synchronize()
        runs.append((st.state().cpu().numpy(), dts))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    assert runs[0][1] == runs[1][1]
    ref, _, dts_ref = oracle.run_steps(grid.offsets(), np.full((grid.n, 3), grid.dx), flat,
                                       grid.neighbours(), 3, 8, 100, nthreads=0)
    np.testing.assert_allclose(runs[0][1], dts_ref, rtol=1e-12)
    err = _normwise(grid.unpack(runs[0][0]), grid.unpack(ref), 5)
    _say(f"    err after 100 steps = {err:.3e}")
    assert err <= TOL


def test_sod_one_launch_steps_match_oracle():
    """Sod shock tube (transmissive in x), 20 one-launch steps against the
    oracle's 20 steps."""
    import torch
    _say("[step_halo sod 512 patches, 20 steps]")
    grid, q = W.grid_sod()
    flat = grid.pack(q)
    st = fv.Stepper(grid.descriptors(), grid.neighbours(), flat, dim=3, p=8, mode="halo_step")
    for _ in range(20):
        st.step()
    torch.cuda.synchronize()
    ref, _, _ = oracle.run_steps(grid.offsets(), np.full((grid.n, 3), grid.dx), flat,
                                 grid.neighbours(), 3, 8, 20, nthreads=0)
    err = _normwise(grid.unpack(st.state().cpu().numpy()), grid.unpack(ref), 5)
    _say(f"    err after 20 steps = {err:.3e}")
    assert err <= TOL, err


def test_non_mutual_neighbour_entry_gives_nan():
    """A patch with a neighbour entry that is not mutual is not updated,
    pushes nothing and gets NaN as its maximum; so does the patch that names
    it across the opposite face without being named back; the time step is
    NaN."""
    import torch
    _say("[step_halo non-mutual table]")
    grid = W.PatchGrid(3, 8, (3, 2, 2), 1.0 / 24)
    q = _random_state(grid, 3)
    nb = grid.neighbours().copy()
    nb[4, 1] = 7  # patch 4's +x neighbour is not 7's -x neighbour
    assert nb[7, 0] != 4
    flat = grid.pack(q)
    pd = fv.upload_patches(grid.descriptors(dt=1e-3))
    qin = _dev(flat)
    qout = torch.full_like(qin, -123.0)
    me = torch.full((grid.n,), -1.0, dtype=torch.float64, device="cuda")
    dt = torch.tensor([1e-3], dtype=torch.float64, device="cuda")
    dt_next = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = torch.zeros(fv.step_workspace_words(grid.n, 3, 8), dtype=torch.int64, device="cuda")
    fv.step_halo(pd, _dev(nb), qin, qout, dt, dt_next, ws, dim=3, p=8, max_eig=me)
    torch.cuda.synchronize()
    m = me.cpu().numpy()
    # 4 names 7 across +x, 7 names 6 across -x; 5 names 4 across -x, 4 names 7
    assert np.isnan(m[[4, 5]]).all() and np.isfinite(np.delete(m, [4, 5])).all()
    assert np.isnan(dt_next.item())
    blocks = qout.cpu().numpy().reshape(grid.n, 5, 10, 10, 10)
    assert (blocks[[4, 5], :, 1:-1, 1:-1, 1:-1] == -123.0).all()
    assert (blocks[[0, 1, 2, 3, 6, 7, 8, 9, 10, 11], :, 1:-1, 1:-1, 1:-1] != -123.0).all()
    assert (ws.cpu().numpy() == 0).all()
