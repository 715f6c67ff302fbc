#!/usr/bin/env python3
"""Benchmark: batched FP64 Finite Volume update of 3-D Euler 8^3 patches on one MI355X.

Workload (the paper-shaped headline case): 4096 patches of 8^3 volumes (a
periodic 128^3 domain, dx = 1/128), s = 5 unknowns, halo 1, seeded random
smooth fields (rho in [0.5,1.5], p in [0.5,2], u in [-0.5,0.5]).  One "step"
is the whole hot path on the device: CFL time step from the per-patch maxima
(fv_cfl_timestep), the Rusanov update of every patch (fv_batch_update, which
also yields the next per-patch maxima) and the face-halo exchange
(fv_fill_halo).  Inputs are resident in HBM before the timed region starts.

Prints ONE JSON line: cell-updates/s over the timed steps, the roofline of the
dominant kernel (fv_batch_update; algorithmic bytes / its average duration
measured with HIP events on the stream it runs on) and the CPU oracle timed on
a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 100] [--warmup 5] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s and % HBM peak, 3D Euler 8^3 patches, vs FP64 plain form"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fv_update_3d_p8_4096_traffic.txt")
KERNEL_SOURCES = ["paper_2302_09005_amd/csrc/fv_update.hip",
                  "paper_2302_09005_amd/csrc/fv_euler.hpp",
                  "paper_2302_09005_amd/csrc/fv_internal.hpp"]


def algorithmic_bytes_per_cell(d, p, s, elem):
    """Bytes the update must move per interior cell: read the interior and the
    2d face-halo layers of the halo'd input, write the interior."""
    reads = (p ** d + 2 * d * p ** (d - 1)) * s * elem
    writes = p ** d * s * elem
    return (reads + writes) / p ** d


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per update launch from the committed rocprofv3 counter
    summary, or None when absent or taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            line = line.strip()
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(grid, flat, budget_s, max_steps):
    """The CPU oracle (unchanged) on a bounded sample of the same workload."""
    import oracle
    off = grid.offsets()
    dx = np.full((grid.n, 3), grid.dx)
    nb = grid.neighbours()
    threads = oracle.num_threads()
    # one untimed step to fault pages in, then whole steps until the budget
    oracle.run_steps(off, dx, flat, nb, grid.d, grid.p, 1)
    a = flat.copy()
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps and time.perf_counter() - t0 < budget_s:
        a, _, _ = oracle.run_steps(off, dx, a, nb, grid.d, grid.p, 1)
        steps += 1
    el = time.perf_counter() - t0
    return {"value": grid.cells * steps / el, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} full steps (CFL + update + halo fill) of the 4096x8^3 workload, "
                      f"seed 0, plain C oracle, OpenMP over patches with {threads} threads, "
                      f"{el:.1f} s"}


def copy_calibration(mib=1024, reps=5):
    """Plain device copy of a known size, for scaling rocprofv3 byte counters."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "copy_calibration_bytes_written": n * 8,
                      "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of CPU-oracle work for the baseline sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(patches would be sharded across GPUs with a face-halo exchange; "
              "see DESIGN.md). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration()
        return

    from paper_2302_09005_amd import fv
    from paper_2302_09005_amd import workloads as W

    grid, q = W.grid_3d_random_smooth(16, 8, seed=args.seed)
    flat = grid.pack(q)
    d, p, s = grid.d, grid.p, grid.s
    st = fv.Stepper(grid.descriptors(), grid.neighbours(), flat, dim=d, p=p)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        st.step()
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    marks = [(ev(), ev(), ev(), ev()) for _ in range(args.steps)]
    t_start, t_end = ev(), ev()
    torch.cuda.synchronize()
    t_start.record(stream)
    for (e0, e1, e2, e3) in marks:
        e0.record(stream)
        fv.cfl_timestep(st.patches, st.per_patch, dim=d, cfl=st.cfl, lambda_out=st.lam,
                        dt_out=st.dt)
        e1.record(stream)
        fv.batch_update(st.patches, st.a, st.b, dim=d, p=p, gamma=st.gamma, q_out_halo=True,
                        dt=st.dt, max_eig=st.per_patch)
        e2.record(stream)
        fv.fill_halo(st.patches, st.neighbours, st.b, dim=d, p=p)
        e3.record(stream)
        st.a, st.b = st.b, st.a
    t_end.record(stream)
    torch.cuda.synchronize()

    total_ms = t_start.elapsed_time(t_end)
    cfl_ms = np.array([a.elapsed_time(b) for a, b, _, _ in marks])
    upd_ms = np.array([b.elapsed_time(c) for _, b, c, _ in marks])
    halo_ms = np.array([c.elapsed_time(e) for _, _, c, e in marks])
    state = st.state()
    finite = bool(torch.isfinite(state[~torch.isnan(state)]).all().item())
    lam_final = st.lam.item()

    cells = grid.cells
    value = cells * args.steps / (total_ms * 1e-3)
    bpc = algorithmic_bytes_per_cell(d, p, s, 8)
    upd_s = upd_ms.mean() * 1e-3
    achieved = bpc * cells / upd_s / 1e9
    traffic = read_traffic()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded random smooth 3-D Euler fields)",
        "config": {"workload": "3d-euler-fp64-4096x8^3-periodic", "patches": grid.n, "p": p,
                   "d": d, "s": s, "halo": 1, "dx": grid.dx, "cfl": st.cfl, "seed": args.seed,
                   "step": "cfl_timestep + batch_update + fill_halo"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "fv_update_kernel<double,3,8>",
                     "algorithmic_bytes_per_cell": bpc,
                     "kernel_avg_us": upd_ms.mean() * 1e3},
        "detail": {"update_cell_updates_per_s": cells / upd_s,
                   "update_us_median": float(np.median(upd_ms) * 1e3),
                   "halo_us_mean": float(halo_ms.mean() * 1e3),
                   "cfl_us_mean": float(cfl_ms.mean() * 1e3),
                   "final_lambda": lam_final, "state_finite": finite},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(grid, flat, args.cpu_budget, 100)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
