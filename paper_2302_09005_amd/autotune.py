"""Schedule autotuner for uneven batches (host side; launches only libfv).

The paper compares two loop orders for a batch of patches (Section 3): one
kernel per patch ("patch-wise") and one loop over all patches and volumes
("batched").  For a batch of mixed patch sizes there are more choices:
one batched launch per size class, or one persistent launch over a
size-sorted work list whose grid is a free parameter.  ``tune`` times every
candidate on the caller's own stepper (on copies of its state and
descriptors, restored afterwards, so tuning leaves the run unchanged) and
keeps the fastest.
"""
import statistics


def candidates(n_units, compute_units, patchwise=False):
    """(schedule, workgroups) pairs to try: per size class, persistent with
    one workgroup per unit, and persistent grids of 2, 4 and 8 workgroups
    per compute unit (two resident per unit at two waves per SIMD)."""
    out = [("per_size", 0), ("persistent", 0)]
    for k in (2, 4, 8):
        g = k * compute_units
        if g < n_units:
            out.append(("persistent", g))
    if patchwise:
        out.append(("patchwise", 0))
    return out


def _time_steps(stepper, steps, warmup):
    import torch
    for _ in range(warmup):
        stepper.step()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    for i in range(steps):
        ev[2 * i].record()
        stepper.step()
        ev[2 * i + 1].record()
    torch.cuda.synchronize()
    return [ev[2 * i].elapsed_time(ev[2 * i + 1]) * 1e3 for i in range(steps)]  # us


def tune(stepper, steps=5, warmup=2, patchwise=False, cands=None):
    """Time each candidate and set the fastest on ``stepper``.

    Returns (best (schedule, workgroups), [(schedule, workgroups, median us)]).
    """
    import torch
    cus = torch.cuda.get_device_properties(stepper.a.device).multi_processor_count
    cands = cands or candidates(stepper.plan.n_units, cus, patchwise)
    a0, b0 = stepper.a.clone(), stepper.b.clone()
    d0, m0 = stepper.patches.clone(), stepper.per_patch.clone()
    keep = (stepper.a, stepper.b, stepper.schedule, stepper.workgroups)
    table = []
    for sched, wg in cands:
        stepper.schedule, stepper.workgroups = sched, wg
        n = 1 if sched == "patchwise" else steps
        us = _time_steps(stepper, n, 0 if sched == "patchwise" else warmup)
        table.append((sched, wg, statistics.median(us)))
        # restore the run
        stepper.a, stepper.b = keep[0], keep[1]
        stepper.a.copy_(a0)
        stepper.b.copy_(b0)
        stepper.patches.copy_(d0)
        stepper.per_patch.copy_(m0)
    torch.cuda.synchronize()
    best = min(table, key=lambda r: r[2])
    stepper.schedule, stepper.workgroups = best[0], best[1]
    return (best[0], best[1]), table
