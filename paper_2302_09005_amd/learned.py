"""Learned face-flux correction for 2-D Euler: training data, training and
evaluation, driven from Python with every arithmetic step in libfv.

The correction targets a coarse grid of 16 x 16 patches of 16^2 volumes.
Training data come from plain runs of seeded 2-D Riemann problems on the grid
four times finer (64 x 64 patches): at the start of each coarse step the fine
state is coarse-grained, the fine Rusanov fluxes through every coarse face
are averaged over its four fine faces and the four fine steps of the coarse
step, and each coarse face yields a sample (its 4-volume stencil, the
averaged fine flux minus the coarse Rusanov flux, the density-jump
indicator).  Faces above the indicator threshold are left out: the update
uses the plain flux there.  The network is then trained by minibatch Adam.

See include/fv.h for the exact definitions of the features, the network and
the correction.
"""
import numpy as np

from . import fv
from . import workloads as W

THRESHOLD = 0.2
R = 4          # refinement factor of the reference runs
P = 16         # patch size
COARSE = 16    # coarse patches per axis (256 patches of 16^2)
CFL = 0.4


def _nb_bc(grid):
    return 0 if grid.bc[0] == W.PERIODIC else 1


class PatchRun:
    """A 2-D run on a regular patch grid with compact blocks (device state)."""

    def __init__(self, grid, q, device="cuda"):
        import torch
        self.grid = grid
        desc = grid.descriptors(out_halo=False, in_halo=False)
        self.patches = fv.upload_patches(desc, device)
        self.neighbours = torch.from_numpy(grid.neighbours()).to(device)
        self.a = torch.from_numpy(grid.pack_compact(q)).to(device)
        self.b = torch.empty_like(self.a)
        self.per = torch.empty(grid.n, dtype=torch.float64, device=device)
        self.dt = torch.empty(1, dtype=torch.float64, device=device)

    def cfl_dt(self, cfl):
        """dt = cfl * dx / (2 Lambda) of the current state, on the device."""
        import torch
        fv.max_eigenvalue(self.patches, self.a, self.per, dim=2, p=P, q_halo=False)
        out = torch.empty_like(self.dt)
        fv.cfl_timestep(self.patches, self.per, dim=2, cfl=cfl, dt_out=out)
        return out

    def step_plain(self, dt):
        fv.batch_update_gather(self.patches, self.neighbours, self.a, self.b, dim=2, p=P, dt=dt)
        self.a, self.b = self.b, self.a

    def step_learned(self, dt, blob, threshold=THRESHOLD):
        fv.batch_update_learned_2d(self.patches, self.neighbours, self.a, self.b, blob, dt=dt,
                                   threshold=threshold)
        self.a, self.b = self.b, self.a

    def global_state(self):
        return self.grid.unpack(self.a.cpu().numpy(), halo=False)


def fine_run(seed, coarse_steps, device="cuda", collect=True, threshold=THRESHOLD):
    """A reference run of the seeded Riemann problem on the fine grid.

    Returns (samples, truth, dts): samples = (features, targets) device
    tensors of the faces with indicator <= threshold over all coarse steps
    (None unless collect), truth = list of coarse-grained fine states (device,
    coarse patch layout) at the start of each coarse step and after the last,
    dts = list of device scalars, the coarse step of each coarse step.
    """
    import torch
    grid, q = W.grid_riemann_2d(COARSE * R, P, seed)
    run = PatchRun(grid, q, device)
    bc = _nb_bc(grid)
    npx = npy = COARSE * R
    ncx = ncy = COARSE * P
    acc_x = torch.zeros(4 * ncy * (ncx + 1), dtype=torch.float64, device=device)
    acc_y = torch.zeros(4 * (ncy + 1) * ncx, dtype=torch.float64, device=device)
    nfaces = ncy * (ncx + 1) + (ncy + 1) * ncx
    feats = torch.empty(nfaces * 16, dtype=torch.float32, device=device)
    targ = torch.empty(nfaces * 4, dtype=torch.float32, device=device)
    ind = torch.empty(nfaces, dtype=torch.float32, device=device)
    truth, dts, f_all, t_all = [], [], [], []
    cblock = COARSE * COARSE * 4 * P * P
    for _ in range(coarse_steps):
        qc = torch.empty(cblock, dtype=torch.float64, device=device)
        fv.learned_coarse_grain(run.a, qc, npx=npx, npy=npy, p=P, r=R)
        truth.append(qc)
        dt_f = run.cfl_dt(CFL)
        dt_c = run.cfl_dt(CFL * R)
        dts.append(dt_c)
        acc_x.zero_()
        acc_y.zero_()
        for _s in range(R):
            fv.learned_flux_accumulate(run.a, acc_x, acc_y, npx=npx, npy=npy, p=P, r=R, bc=bc,
                                       weight=1.0 / R)
            run.step_plain(dt_f)
        if collect:
            fv.learned_face_samples(qc, acc_x, acc_y, feats, targ, ind, npx=COARSE, npy=COARSE,
                                    p=P, bc=bc)
            keep = torch.nonzero(ind <= threshold).reshape(-1)
            f_all.append(feats.view(nfaces, 16)[keep].clone())
            t_all.append(targ.view(nfaces, 4)[keep].clone())
    qc = torch.empty(cblock, dtype=torch.float64, device=device)
    fv.learned_coarse_grain(run.a, qc, npx=npx, npy=npy, p=P, r=R)
    truth.append(qc)
    samples = (torch.cat(f_all), torch.cat(t_all)) if collect else None
    return samples, truth, dts


def train(features, targets, *, epochs=20, batch=1024, lr=1e-3, seed=0, init_scale=None,
          device="cuda", log_every=0):
    """Minibatch Adam on (features, targets) (device tensors [n,16], [n,4]).
    Returns (blob, per-epoch mean loss).  Weights start from a seeded
    Glorot-uniform draw (host RNG, a documented input), biases at 0; the
    normalisation slots are fitted on the data first."""
    import torch
    n = features.shape[0]
    rng = np.random.default_rng(seed)
    blob = np.zeros(fv.MLP_BLOB_WORDS, np.float32)
    o = fv.BLOB_OFFSETS
    for name, fan_in, fan_out in (("w1", 16, 64), ("w2", 64, 64), ("w3", 64, 4)):
        lim = np.sqrt(6.0 / (fan_in + fan_out)) if init_scale is None else init_scale
        blob[o[name]:o[name] + fan_in * fan_out] = rng.uniform(-lim, lim, fan_in * fan_out)
    blob_d = torch.from_numpy(blob).to(device)
    feats = features.contiguous().view(-1)
    targ = targets.contiguous().view(-1)
    fv.mlp_fit_normalization(feats, 16, blob_d[o["x_mean"]:o["x_mean"] + 16],
                             blob_d[o["x_scale"]:o["x_scale"] + 16], mode=0)
    fv.mlp_fit_normalization(targ, 4, blob_d[o["y_mean"]:o["y_mean"] + 4],
                             blob_d[o["y_scale"]:o["y_scale"] + 4], mode=1)
    adam = torch.zeros(2 * fv.MLP_TRAINED_WORDS, dtype=torch.float32, device=device)
    ws = torch.empty(fv.mlp_workspace_words(batch), dtype=torch.float32, device=device)
    losses = []
    step = 0
    nws = fv.mlp_workspace_words(batch)
    loss_rows = ws[nws - batch:nws]  # per-sample squared errors of the last step
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n).astype(np.int64)).to(device)
        tot, cnt = torch.zeros((), dtype=torch.float64, device=device), 0
        for i in range(0, n - batch + 1, batch):
            step += 1
            fv.mlp_train_step(blob_d, adam, step, lr, feats, targ, perm[i:i + batch], ws)
            tot += loss_rows.double().sum()
            cnt += batch
        losses.append(float(tot.item()) / max(cnt, 1))
        if log_every and (ep + 1) % log_every == 0:
            print(f"  epoch {ep + 1}: loss {losses[-1]:.4e}", flush=True)
    return blob_d, losses


def evaluate(blob, seed, coarse_steps, device="cuda", threshold=THRESHOLD):
    """Coarse plain and learned runs of a held-out Riemann problem against the
    coarse-grained fine run, with the fine run's coarse steps.  Returns L1
    errors per unknown (mean over volumes) after every coarse step."""
    _, truth, dts = fine_run(seed, coarse_steps, device, collect=False)
    grid, _ = W.grid_riemann_2d(COARSE, P, seed)
    q0 = grid.unpack(truth[0].cpu().numpy(), halo=False)
    plain = PatchRun(grid, q0, device)
    learn = PatchRun(grid, q0, device)
    out = {"plain": [], "learned": []}
    for k in range(coarse_steps):
        plain.step_plain(dts[k])
        learn.step_learned(dts[k], blob, threshold)
        ref = grid.unpack(truth[k + 1].cpu().numpy(), halo=False)
        for name, run in (("plain", plain), ("learned", learn)):
            err = np.abs(run.global_state() - ref).mean(axis=(1, 2))
            out[name].append(err.tolist())
    return out
