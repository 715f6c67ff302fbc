"""Checkpoint and resume: the per-patch state the method carries from one step
to the next is the solution Q plus, per patch, its time stamp t and time-step
size dt (the paper's per-patch metadata, Appendix A; local time stepping,
Section 4).  Saving it to the host after k steps and starting a new driver from
the saved copy must continue the run bit for bit."""
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


def _run(st, steps):
    import torch
    dts = []
    for _ in range(steps):
        st.step()
        dts.append(st.last_dt().item())
    torch.cuda.synchronize()
    return dts


@pytest.mark.parametrize("mode", ["fused", "pipelined", "halo"])
def test_global_step_resumes_bitwise(mode):
    """100 steps of 512 patches of 8^3 in one run == 50 steps, a host
    checkpoint of Q (and the time step it implies), then 50 more steps from a
    new stepper built from the checkpoint."""
    _say(f"[checkpoint/resume, global CFL, mode={mode}]")
    grid, q = W.grid_3d_random_smooth(8, 8, seed=31)
    halo = mode == "halo"
    flat = grid.pack(q) if halo else grid.pack_compact(q)
    desc = grid.descriptors(out_halo=halo, in_halo=halo)
    nbr = grid.neighbours()
    full = fv.Stepper(desc, nbr, flat, dim=3, p=8, mode=mode)
    dts_full = _run(full, 100)
    first = fv.Stepper(desc, nbr, flat, dim=3, p=8, mode=mode)
    dts_a = _run(first, 50)
    ckpt_q = first.state().cpu().numpy().copy()
    resumed = fv.Stepper(desc, nbr, ckpt_q, dim=3, p=8, mode=mode)
    if mode == "fused":
        # the time step of step 51: held on the device by the first run (from
        # its fused launch), recomputed from the checkpoint by the new one
        assert resumed.dt.item() == first.dt.item()
    dts_b = _run(resumed, 50)
    assert dts_a + dts_b == dts_full
    np.testing.assert_array_equal(resumed.state().cpu().numpy(), full.state().cpu().numpy())


@pytest.mark.parametrize("schedule", ["per_size", "persistent"])
def test_local_time_stepping_resumes_bitwise(schedule):
    """Uneven batch with local time steps: 20 steps == 10 steps, a checkpoint
    of Q and every patch's (t, dt), 10 more steps from a new driver."""
    _say(f"[checkpoint/resume, local time stepping, schedule={schedule}]")
    batch, q = W.uneven_batch(300, seed=5)
    nbr = batch.neighbours()
    full = fv.LocalStepper(batch.descriptors(), nbr, q, schedule=schedule)
    for _ in range(20):
        full.step()
    first = fv.LocalStepper(batch.descriptors(), nbr, q, schedule=schedule)
    for _ in range(10):
        first.step()
    ckpt_desc = first.descriptors()
    ckpt_q = first.state().cpu().numpy().copy()
    assert (ckpt_desc["t"] > 0).all()
    resumed = fv.LocalStepper(ckpt_desc, nbr, ckpt_q, schedule=schedule)
    # the resumed driver derives each patch's dt from the saved state: the
    # same bits the first run stored in its descriptors
    d0 = resumed.descriptors()
    np.testing.assert_array_equal(d0["dt"], ckpt_desc["dt"])
    np.testing.assert_array_equal(d0["t"], ckpt_desc["t"])
    for _ in range(10):
        resumed.step()
    import torch
    torch.cuda.synchronize()
    np.testing.assert_array_equal(resumed.state().cpu().numpy(), full.state().cpu().numpy())
    df, dr = full.descriptors(), resumed.descriptors()
    np.testing.assert_array_equal(dr["t"], df["t"])
    np.testing.assert_array_equal(dr["dt"], df["dt"])
