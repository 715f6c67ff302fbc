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


def _warm(stepper, seconds):
    """Run steps for about ``seconds`` of wall time: after an idle period the
    GPU runs FP64-heavy kernels slower for the first tens of milliseconds, and
    a candidate timed then would lose to the ones timed after it."""
    import time
    import torch
    t_end = time.perf_counter() + seconds
    while True:
        for _ in range(4):
            stepper.step()
        torch.cuda.synchronize()
        if time.perf_counter() >= t_end:
            return


def _capture(stepper, steps):
    """A HIP graph of ``steps`` steps (an even count: the state buffers return
    to where they were).  Capturing launches nothing."""
    import torch
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for _ in range(steps):
                stepper.step()
    torch.cuda.current_stream().wait_stream(side)
    return graph


def _time_graph(graph, steps, reps):
    import torch
    graph.replay()  # first replay: uploads the graph
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for r in range(reps):
        graph.replay()
        ev[r + 1].record()
    torch.cuda.synchronize()
    return [ev[r].elapsed_time(ev[r + 1]) * 1e3 / steps for r in range(reps)]  # us per step


def tune(stepper, steps=4, warmup=2, patchwise=False, cands=None, rounds=3, warm_s=0.3,
         graph=True):
    """Time each candidate and set the fastest on ``stepper``.

    The clock is brought up first (``warm_s`` seconds of steps), then the
    candidates are timed round-robin, ``rounds`` times each, so that a drift
    of the clock during tuning hits every candidate alike.  With ``graph``
    (the default) a candidate is timed as replays of a HIP graph of
    ``steps`` steps (rounded up to even), the way a multi-step run is
    launched: eager launches pay a cache write-back and invalidation between
    kernels that a graph's launches do not, and rank the schedules
    differently.  Otherwise ``steps`` eager steps after ``warmup`` untimed
    ones.  Patch-wise (thousands of launches a step) is timed once, one
    eager step.  The run is restored after every timing.

    Returns (best (schedule, workgroups), [(schedule, workgroups, median us)]).
    """
    import torch
    cus = torch.cuda.get_device_properties(stepper.a.device).multi_processor_count
    cands = cands or candidates(stepper.plan.n_units, cus, patchwise)
    a0, b0 = stepper.a.clone(), stepper.b.clone()
    d0, m0 = stepper.patches.clone(), stepper.per_patch.clone()
    keep = (stepper.a, stepper.b, stepper.schedule, stepper.workgroups)

    def restore():
        stepper.a, stepper.b = keep[0], keep[1]
        stepper.a.copy_(a0)
        stepper.b.copy_(b0)
        stepper.patches.copy_(d0)
        stepper.per_patch.copy_(m0)

    n_cap = steps + steps % 2
    graphs = {}
    if graph:
        for sched, wg in cands:
            if sched != "patchwise":
                stepper.schedule, stepper.workgroups = sched, wg
                graphs[(sched, wg)] = _capture(stepper, n_cap)
                stepper.a, stepper.b = keep[0], keep[1]
    if warm_s > 0:
        stepper.schedule, stepper.workgroups = keep[2], keep[3]
        _warm(stepper, warm_s)
        restore()
    samples = {c: [] for c in cands}
    for r in range(max(1, rounds)):
        for sched, wg in cands:
            if sched == "patchwise":
                if r == 0:
                    stepper.schedule, stepper.workgroups = sched, wg
                    samples[(sched, wg)] += _time_steps(stepper, 1, 0)
                    restore()
                continue
            if graph:
                samples[(sched, wg)] += _time_graph(graphs[(sched, wg)], n_cap, 1)
            else:
                stepper.schedule, stepper.workgroups = sched, wg
                samples[(sched, wg)] += _time_steps(stepper, steps, warmup)
            restore()
    torch.cuda.synchronize()
    table = [(s_, w_, statistics.median(samples[(s_, w_)])) for s_, w_ in cands]
    best = min(table, key=lambda r: r[2])
    stepper.schedule, stepper.workgroups = best[0], best[1]
    return (best[0], best[1]), table
