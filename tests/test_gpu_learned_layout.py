"""A sharper check of the matrix-core network's lane and fragment layouts
than the absolute bars of test_gpu_learned.py.

A bfloat16 rounding that lands on the other side of a boundary (the float32
sums run in a different order on the matrix cores) moves one face's outputs
by about 2^-8 of a weight, so a few faces may differ; a wrong lane layout,
fragment order or unit order would give wrong outputs on most faces.  So:
per face, the largest output difference to the oracle, and the share of
faces above 1e-4 must stay small, on inputs spread over the whole feature
range and on random weights of both signs."""
import sys

import numpy as np
import pytest

from oracle import learned as OL
from paper_2302_09005_amd import fv

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("seed", [7, 8])
def test_network_agrees_on_almost_every_face(seed):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    rng = np.random.default_rng(seed)
    p = {name: rng.normal(0.0, 0.3, shape).astype(np.float32) for name, shape in OL.BLOB_LAYOUT}
    p["x_mean"] = rng.uniform(-0.5, 1.0, 16).astype(np.float32)
    p["x_scale"] = rng.uniform(0.5, 2.0, 16).astype(np.float32)
    p["y_scale"] = np.full(4, 1.0, np.float32)
    p["y_mean"] = np.zeros(4, np.float32)
    n = 4096
    x = rng.uniform(-1.0, 2.0, (n, 16)).astype(np.float32)
    blob = torch.from_numpy(OL.pack_blob(p)).cuda()
    out = torch.empty(n * 4, dtype=torch.float32, device="cuda")
    fv.mlp_forward(blob, torch.from_numpy(x).cuda(), out)
    got = out.cpu().numpy().reshape(n, 4)
    ref = OL.mlp_forward(((x - p["x_mean"]) * p["x_scale"]).astype(np.float32), p)
    per_face = np.abs(got - ref).max(axis=1)
    share = float((per_face > 1e-4).mean())
    _say(f"[mlp layout seed={seed}] |o| ~ {np.abs(ref).mean():.2e}; faces above 1e-4: "
         f"{100 * share:.2f} %; per-face error quantiles 50/90/99 %: "
         f"{np.quantile(per_face, 0.5):.1e} {np.quantile(per_face, 0.9):.1e} "
         f"{np.quantile(per_face, 0.99):.1e}")
    assert share <= 0.05
    assert np.quantile(per_face, 0.9) <= 1e-4
