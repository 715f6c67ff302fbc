"""fv_step_gather_noalloc (the library's static scratch array as workspace)
against fv_step_gather (a caller workspace), through the C ABI: the same
kernel, so the same bits, on two calls in a row, the second with a smaller
batch; the state is also checked against the oracle (normwise 1e-12)."""
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


def _normwise(got, ref, s):
    got = np.asarray(got).reshape(s, -1)
    ref = np.asarray(ref).reshape(s, -1)
    return max(np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max() for k in range(s))


def _one_step(grid, q, noalloc):
    import torch
    flat = grid.pack_compact(q)
    desc = grid.descriptors(out_halo=False, in_halo=False)
    per, _ = oracle.max_eigenvalue(grid.offsets(), grid.pack(q), grid.d, grid.p, True)
    dt0, _ = oracle.cfl_dt(np.full((grid.n, 3), grid.dx), per, grid.d)
    pd = fv.upload_patches(desc)
    nbr = torch.from_numpy(grid.neighbours()).to("cuda")
    qin = torch.from_numpy(flat).to("cuda")
    qout = torch.full_like(qin, -123.0)
    dt = torch.tensor([dt0], dtype=torch.float64, device="cuda")
    dt_next = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    lam = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    me = torch.full((grid.n,), -1.0, dtype=torch.float64, device="cuda")
    if noalloc:
        fv.step_gather_noalloc(pd, nbr, qin, qout, dt, dt_next, dim=grid.d, p=grid.p,
                               max_eig=me, lambda_out=lam)
    else:
        ws = torch.zeros(fv.step_workspace_words(grid.n, grid.d, grid.p), dtype=torch.int64,
                         device="cuda")
        fv.step_gather(pd, nbr, qin, qout, dt, dt_next, ws, dim=grid.d, p=grid.p, max_eig=me,
                       lambda_out=lam)
    torch.cuda.synchronize()
    if not noalloc:
        assert (ws.cpu().numpy() == 0).all()
    return (qout.cpu().numpy(), me.cpu().numpy(), dt_next.item(), lam.item(), dt0)


@pytest.mark.parametrize("sizes", [((16, 8, 3), (4, 8, 3)), ((8, 16, 2), (3, 16, 2))])
def test_noalloc_step_matches_workspace_step(sizes):
    import torch
    assert torch.cuda.is_available()
    for call, (npa, p, d) in enumerate(sizes):
        _say(f"[noalloc call {call}: {npa}^{d} patches of {p}^{d}]")
        if d == 3:
            grid, q = W.grid_3d_random_smooth(npa, p, seed=40 + call)
        else:
            grid, q = W.grid_2d_smooth(npa, p, seed=40 + call)
        got = _one_step(grid, q, noalloc=True)
        ref = _one_step(grid, q, noalloc=False)
        np.testing.assert_array_equal(got[0], ref[0])
        np.testing.assert_array_equal(got[1], ref[1])
        assert got[2] == ref[2] and got[3] == ref[3]
        # repeated: the scratch array was left zero by the previous call
        again = _one_step(grid, q, noalloc=True)
        np.testing.assert_array_equal(again[0], got[0])
        assert again[2] == got[2] and again[3] == got[3]
        desc = grid.descriptors(dt=got[4], out_halo=False)
        want, me_want = oracle.fv_step(desc["q_in"], desc["q_out"], desc["dx"], desc["dt"],
                                       grid.pack(q), d, p, out_halo=False,
                                       out_len=grid.buffer_len(False))
        err = _normwise(got[0], want, d + 2)
        _say(f"    err vs oracle {err:.3e}")
        assert err <= TOL
        assert np.abs(got[1] - me_want).max() <= 1e-14 * me_want.max()
        dt_want, _ = oracle.cfl_dt(np.full((grid.n, 3), grid.dx), me_want, d)
        assert got[2] == pytest.approx(dt_want, rel=1e-14)
        assert got[3] == pytest.approx(me_want.max(), rel=1e-14)
