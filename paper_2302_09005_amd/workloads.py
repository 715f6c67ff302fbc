"""Seeded synthetic inputs: patch grids, descriptors, neighbour tables, fields.

This module builds inputs only.  It holds none of the update's arithmetic (no
flux, eigenvalue or time-step code); both the GPU library and the CPU oracle
consume what it produces.  The one physical relation used here is the ideal-gas
equation of state, to turn prescribed primitive fields (rho, u, p) into the
conserved unknowns (rho, rho*u, E) that the update takes as input.

Layout conventions (shared with the C ABI in include/fv.h):
  * a patch block is unknown-major, x fastest: [s][z][y][x];
  * a block with halo covers (p+2)^d volumes, one without covers p^d;
  * patches are numbered lexicographically over the patch grid (px fastest);
  * global grids are arrays [s][Z][Y][X] (2-D: [s][Y][X]).
"""
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np

GAMMA = 1.4

#: One patch descriptor; the record layout of ``fv_patch`` in include/fv.h.
PATCH_DTYPE = np.dtype([
    ("q_in", "<i8"),
    ("q_out", "<i8"),
    ("p", "<i4"),
    ("flags", "<i4"),
    ("dx", "<f8", (3,)),
    ("dt", "<f8"),
    ("t", "<f8"),
], align=True)
assert PATCH_DTYPE.itemsize == 64

#: Boundary kinds along one axis of the patch grid.
PERIODIC = "periodic"
TRANSMISSIVE = "transmissive"


@dataclass
class PatchGrid:
    """A uniform Cartesian arrangement of d-dimensional patches of p^d volumes.

    counts: patches per axis (x, y[, z]); domain is [0, L_x] x ... with
    L = counts * p * dx.  bc: boundary kind per axis.
    """
    d: int
    p: int
    counts: Tuple[int, ...]
    dx: float
    bc: Tuple[str, ...] = field(default=None)

    def __post_init__(self):
        if self.d not in (2, 3):
            raise ValueError("d must be 2 or 3")
        self.counts = tuple(int(c) for c in self.counts)
        if len(self.counts) != self.d:
            raise ValueError("counts needs one entry per axis")
        if self.bc is None:
            self.bc = (PERIODIC,) * self.d
        self.bc = tuple(self.bc)

    # sizes -----------------------------------------------------------------
    @property
    def s(self) -> int:
        return self.d + 2

    @property
    def n(self) -> int:
        return int(np.prod(self.counts))

    @property
    def block_halo(self) -> int:
        return self.s * (self.p + 2) ** self.d

    @property
    def block_compact(self) -> int:
        return self.s * self.p ** self.d

    @property
    def cells(self) -> int:
        return self.n * self.p ** self.d

    @property
    def shape(self) -> Tuple[int, ...]:
        """Global grid shape, slowest axis first (z, y, x)."""
        return tuple(c * self.p for c in reversed(self.counts))

    def patch_coords(self) -> np.ndarray:
        """[n, d] integer patch coordinates (x, y[, z]), x fastest."""
        grids = np.meshgrid(*[np.arange(c) for c in reversed(self.counts)], indexing="ij")
        return np.stack([g.ravel() for g in reversed(grids)], axis=1)

    def cell_centres(self):
        """Tuple of 1-D centre coordinates per axis (x, y[, z])."""
        return tuple((np.arange(c * self.p) + 0.5) * self.dx for c in self.counts)

    # layout ------------------------------------------------------------------
    def offsets(self, halo: bool = True, order: Optional[Sequence[int]] = None,
                gap: int = 0) -> np.ndarray:
        """Element offset of every patch's block.

        order: storage slot of each patch (a permutation); gap: extra unused
        elements between consecutive blocks (ragged placement).
        """
        blk = self.block_halo if halo else self.block_compact
        slot = np.arange(self.n) if order is None else np.asarray(order, dtype=np.int64)
        return (slot * (blk + gap)).astype(np.int64)

    def buffer_len(self, halo: bool = True, gap: int = 0) -> int:
        blk = self.block_halo if halo else self.block_compact
        return self.n * (blk + gap)

    def descriptors(self, dt: float = 0.0, out_halo: bool = True, in_order=None,
                    out_order=None, gap: int = 0, in_halo: bool = True) -> np.ndarray:
        desc = np.zeros(self.n, dtype=PATCH_DTYPE)
        desc["q_in"] = self.offsets(in_halo, in_order, gap)
        desc["q_out"] = self.offsets(out_halo, out_order, gap)
        desc["p"] = self.p
        desc["dx"][:, : self.d] = self.dx
        desc["dx"][:, self.d:] = 1.0
        desc["dt"] = dt
        return desc

    def neighbours(self) -> np.ndarray:
        """[n, 2d] face neighbours (order -x, +x, -y, +y[, -z, +z]).

        Periodic axes wrap; transmissive axes use -1 at the domain boundary.
        """
        pc = self.patch_coords()
        strides = np.cumprod((1,) + self.counts[:-1])
        out = np.empty((self.n, 2 * self.d), dtype=np.int64)
        for a in range(self.d):
            for side, step in ((0, -1), (1, 1)):
                c = pc[:, a] + step
                inside = (c >= 0) & (c < self.counts[a])
                cw = np.mod(c, self.counts[a])
                nb = (pc * strides).sum(1) + (cw - pc[:, a]) * strides[a]
                if self.bc[a] == PERIODIC:
                    out[:, 2 * a + side] = nb
                else:
                    out[:, 2 * a + side] = np.where(inside, nb, -1)
        return out

    # packing -----------------------------------------------------------------
    def _axis_index(self, a: int) -> np.ndarray:
        """[counts[a], p+2] global indices of a patch's halo'd extent on axis a."""
        ntot = self.counts[a] * self.p
        idx = (np.arange(self.counts[a])[:, None] * self.p +
               np.arange(-1, self.p + 1)[None, :])
        if self.bc[a] == PERIODIC:
            return np.mod(idx, ntot)
        return np.clip(idx, 0, ntot - 1)

    def pack(self, glob: np.ndarray, corners=np.nan, order=None, gap: int = 0,
             fill=np.nan) -> np.ndarray:
        """Global grid [s][...] -> flat buffer of halo'd patch blocks.

        Face-halo volumes take the neighbouring global values (periodic wrap or
        zero-gradient copy at a transmissive boundary); edge and corner halo
        volumes are set to `corners` (NaN by default: the update must never
        read them).  `order`/`gap` place blocks as in :meth:`offsets`; unused
        elements are set to `fill`.
        """
        glob = np.asarray(glob, dtype=np.float64)
        s, p, d = self.s, self.p, self.d
        w = p + 2
        if d == 2:
            iy, ix = self._axis_index(1), self._axis_index(0)
            blocks = glob[:, iy[:, :, None, None], ix[None, None, :, :]]  # s,ny,w,nx,w
            blocks = blocks.transpose(1, 3, 0, 2, 4)  # ny,nx,s,w,w
        else:
            iz, iy, ix = self._axis_index(2), self._axis_index(1), self._axis_index(0)
            blocks = glob[:, iz[:, :, None, None, None, None],
                          iy[None, None, :, :, None, None],
                          ix[None, None, None, None, :, :]]  # s,nz,w,ny,w,nx,w
            blocks = blocks.transpose(1, 3, 5, 0, 2, 4, 6)  # nz,ny,nx,s,w,w,w
        blocks = np.ascontiguousarray(blocks).reshape(self.n, s, *([w] * d))
        halo_count = np.zeros([w] * d, dtype=np.int32)
        for a in range(d):
            sl = [slice(None)] * d
            for e in (0, w - 1):
                sl[a] = e
                halo_count[tuple(sl)] += 1
        blocks[:, :, halo_count >= 2] = corners
        blocks = blocks.reshape(self.n, -1)
        if order is None and gap == 0:
            return blocks.reshape(-1).copy()
        out = np.full(self.buffer_len(True, gap), fill, dtype=np.float64)
        off = self.offsets(True, order, gap)
        for b in range(self.n):
            out[off[b]: off[b] + self.block_halo] = blocks[b]
        return out

    def pack_compact(self, glob: np.ndarray, order=None, gap: int = 0,
                     fill=np.nan) -> np.ndarray:
        """Global grid [s][...] -> flat buffer of compact blocks [s][p^d] (no halo)."""
        w = self.p + 2
        blocks = self.pack(glob).reshape(self.n, self.s, *([w] * self.d))
        inner = (slice(None), slice(None)) + (slice(1, -1),) * self.d
        blocks = np.ascontiguousarray(blocks[inner]).reshape(self.n, -1)
        if order is None and gap == 0:
            return blocks.reshape(-1).copy()
        out = np.full(self.buffer_len(False, gap), fill, dtype=np.float64)
        off = self.offsets(False, order, gap)
        for b in range(self.n):
            out[off[b]: off[b] + self.block_compact] = blocks[b]
        return out

    def unpack(self, flat: np.ndarray, halo: bool = True, order=None,
               gap: int = 0) -> np.ndarray:
        """Flat buffer of patch blocks -> global grid [s][...] (interior only)."""
        s, p, d = self.s, self.p, self.d
        w = p + 2 if halo else p
        o = 1 if halo else 0
        off = self.offsets(halo, order, gap)
        blk = s * w ** d
        idx = off[:, None] + np.arange(blk)[None, :]
        blocks = np.asarray(flat)[idx].reshape(self.n, s, *([w] * d))
        inner = (slice(None), slice(None)) + (slice(o, o + p),) * d
        blocks = blocks[inner]
        if d == 2:
            ny, nx = self.counts[1], self.counts[0]
            g = blocks.reshape(ny, nx, s, p, p).transpose(2, 0, 3, 1, 4)
        else:
            nz, ny, nx = self.counts[2], self.counts[1], self.counts[0]
            g = blocks.reshape(nz, ny, nx, s, p, p, p).transpose(3, 0, 4, 1, 5, 2, 6)
        return np.ascontiguousarray(g).reshape(s, *self.shape)


# ----------------------------------------------------------------------------
# primitive -> conserved (input construction only)
# ----------------------------------------------------------------------------
def to_conserved(rho, vel, p, gamma: float = GAMMA) -> np.ndarray:
    """Stack (rho, rho*u_1..rho*u_d, E) from primitive fields, E = p/(g-1) + rho|u|^2/2."""
    rho = np.asarray(rho, dtype=np.float64)
    vel = [np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape) for v in vel]
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    ke = 0.5 * rho * sum(v * v for v in vel)
    return np.stack([rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + ke])


# ----------------------------------------------------------------------------
# the paper-shaped workloads (seeded)
# ----------------------------------------------------------------------------
def grid_2d_smooth(patches_per_axis: int = 8, p: int = 16, seed: int = 0,
                   noise: float = 1e-3) -> Tuple[PatchGrid, np.ndarray]:
    """2-D Euler smooth field with seeded noise on a periodic unit square.

    rho = 1 + 0.1 sin(2 pi x) sin(2 pi y) + noise * xi, xi ~ U[-1, 1) drawn by
    numpy.random.default_rng(seed) over the global grid (row-major, y slowest);
    u = v = 0, p = 1.  Default: 8 x 8 patches of 16^2, dx = 1/128.
    """
    n = patches_per_axis * p
    grid = PatchGrid(2, p, (patches_per_axis, patches_per_axis), 1.0 / n)
    x, y = grid.cell_centres()
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=(n, n))
    rho = 1.0 + 0.1 * np.sin(2 * np.pi * x)[None, :] * np.sin(2 * np.pi * y)[:, None] + noise * xi
    return grid, to_conserved(rho, [0.0, 0.0], 1.0)


def random_smooth_field(rng, coords, modes: int = 4, kmax: int = 2) -> np.ndarray:
    """g = (1/modes) sum_m sin(2 pi k_m . x + phi_m), values in [-1, 1].

    For each mode: an integer wave vector k_m with entries in [-kmax, kmax]
    (redrawn while zero), then a phase phi_m ~ U[0, 2 pi).  coords: tuple of
    1-D centre arrays (x, y[, z]); the result has shape (Z, Y, X).
    """
    d = len(coords)
    mesh = np.meshgrid(*reversed(coords), indexing="ij")  # z, y, x order
    mesh = list(reversed(mesh))  # x, y, z
    g = np.zeros(mesh[0].shape)
    for _ in range(modes):
        k = np.zeros(d, dtype=np.int64)
        while not k.any():
            k = rng.integers(-kmax, kmax + 1, size=d)
        phi = rng.uniform(0.0, 2 * np.pi)
        arg = sum(2 * np.pi * k[a] * mesh[a] for a in range(d)) + phi
        g += np.sin(arg)
    return g / modes


def grid_3d_random_smooth(patches_per_axis: int = 16, p: int = 8, seed: int = 0
                          ) -> Tuple[PatchGrid, np.ndarray]:
    """3-D Euler seeded random smooth field on a periodic unit cube.

    For rho, p, u, v, w in that order: g = random_smooth_field(rng, ...) with
    rng = numpy.random.default_rng(seed); rho = 1 + 0.5 g, p = 1.25 + 0.75 g,
    u_j = 0.5 g.  Ranges: rho in [0.5, 1.5], p in [0.5, 2], u_j in
    [-0.5, 0.5].  Default: 16^3 patches of 8^3, dx = 1/128.
    """
    n = patches_per_axis * p
    grid = PatchGrid(3, p, (patches_per_axis,) * 3, 1.0 / n)
    coords = grid.cell_centres()
    rng = np.random.default_rng(seed)
    g_rho = random_smooth_field(rng, coords)
    g_p = random_smooth_field(rng, coords)
    g_u = [random_smooth_field(rng, coords) for _ in range(3)]
    rho = 1.0 + 0.5 * g_rho
    pres = 1.25 + 0.75 * g_p
    return grid, to_conserved(rho, [0.5 * g for g in g_u], pres)


SOD_LEFT = (1.0, 0.0, 1.0)     # rho, u, p
SOD_RIGHT = (0.125, 0.0, 0.1)


def grid_sod(d: int = 3, px: int = 128, pt: int = 2, p: int = 8, x0: float = 0.5,
             left=SOD_LEFT, right=SOD_RIGHT) -> Tuple[PatchGrid, np.ndarray]:
    """Shock tube along x on [0, 1]: px patches along x, pt along y (and z).

    Transmissive in x, periodic in the other axes.  Default (3-D): 128 x 2 x 2
    patches of 8^3 = 512 patches, dx = 1/1024.  The interface x0 = 0.5 falls on
    a face for any even number of cells along x.
    """
    counts = (px,) + (pt,) * (d - 1)
    grid = PatchGrid(d, p, counts, 1.0 / (px * p),
                     (TRANSMISSIVE,) + (PERIODIC,) * (d - 1))
    x = grid.cell_centres()[0]
    shape = grid.shape
    lft = (x < x0)
    rho = np.broadcast_to(np.where(lft, left[0], right[0]), shape)
    u = np.broadcast_to(np.where(lft, left[1], right[1]), shape)
    pr = np.broadcast_to(np.where(lft, left[2], right[2]), shape)
    vel = [u] + [0.0] * (d - 1)
    return grid, to_conserved(rho, vel, pr)


def grid_entropy_wave(d: int, counts, p: int, u0, p0: float = 1.0,
                      amp: float = 0.2, t: float = 0.0, direction=None
                      ) -> Tuple[PatchGrid, np.ndarray]:
    """Exact Euler solution: rho = 1 + amp sin(2 pi n.(x - u0 t)), u = u0, p = p0.

    n = direction (integer vector, default e_x) keeps the field periodic on
    the unit box; dx = 1 / (counts[0] * p) with equal cell widths on all axes.
    """
    counts = tuple(counts)
    grid = PatchGrid(d, p, counts, 1.0 / (counts[0] * p))
    nvec = np.zeros(d) if direction is None else np.asarray(direction, dtype=np.float64)
    if direction is None:
        nvec[0] = 1.0
    u0 = np.asarray(u0, dtype=np.float64)
    coords = grid.cell_centres()
    mesh = list(reversed(np.meshgrid(*reversed(coords), indexing="ij")))
    arg = sum(nvec[a] * (mesh[a] - u0[a] * t) for a in range(d))
    rho = 1.0 + amp * np.sin(2 * np.pi * arg)
    return grid, to_conserved(rho, list(u0), p0)


def grid_uniform(d: int, counts, p: int, state, dx: float = None) -> Tuple[PatchGrid, np.ndarray]:
    """Free stream: the conserved state `state` (length d+2) everywhere."""
    counts = tuple(counts)
    grid = PatchGrid(d, p, counts, dx if dx is not None else 1.0 / (counts[0] * p))
    q = np.empty((d + 2,) + grid.shape)
    for k in range(d + 2):
        q[k] = state[k]
    return grid, q


# ---------------------------------------------------------------------------
# Uneven batches: independent 3-D patches of mixed size and resolution level
# ---------------------------------------------------------------------------
UNEVEN_SIZES = (4, 8, 16)
UNEVEN_RATIO = (4, 2, 1)
UNEVEN_LEVELS = (2, 3, 4)


@dataclass
class UnevenBatch:
    """A batch of 3-D patches of mixed size p_b and level l_b.

    Patch b covers a cube of side 3^-l_b (factor-3 refinement, Section 2) with
    p_b^3 volumes, so dx_b = 3^-l_b / p_b on every axis.  Every patch is
    periodic onto itself (each face's neighbour is the patch itself), so the
    patches are independent, as the patches of one batch handed to the
    update are.  Blocks are compact [s][p^3], stored back to back in patch
    order (``offsets``).
    """
    sizes: np.ndarray       # int[n]
    levels: np.ndarray      # int[n]

    def __post_init__(self):
        self.sizes = np.asarray(self.sizes, dtype=np.int64)
        self.levels = np.asarray(self.levels, dtype=np.int64)
        if self.sizes.shape != self.levels.shape:
            raise ValueError("sizes and levels differ in length")

    @property
    def n(self) -> int:
        return int(self.sizes.shape[0])

    @property
    def d(self) -> int:
        return 3

    @property
    def s(self) -> int:
        return 5

    @property
    def dx(self) -> np.ndarray:
        """float[n]: volume width of each patch."""
        return 3.0 ** (-self.levels.astype(np.float64)) / self.sizes

    def block_len(self) -> np.ndarray:
        return self.s * self.sizes ** 3

    def offsets(self) -> np.ndarray:
        bl = self.block_len()
        return np.concatenate([[0], np.cumsum(bl)[:-1]]).astype(np.int64) if self.n else \
            np.zeros(0, np.int64)

    def buffer_len(self) -> int:
        return int(self.block_len().sum())

    @property
    def cells(self) -> int:
        return int((self.sizes ** 3).sum())

    def descriptors(self, dt=0.0) -> np.ndarray:
        desc = np.zeros(self.n, dtype=PATCH_DTYPE)
        off = self.offsets()
        desc["q_in"] = off
        desc["q_out"] = off
        desc["p"] = self.sizes
        desc["dx"] = self.dx[:, None]
        desc["dt"] = dt
        return desc

    def neighbours(self) -> np.ndarray:
        """int64[n, 6]: every face's neighbour is the patch itself."""
        return np.repeat(np.arange(self.n, dtype=np.int64), 6).reshape(self.n, 6)

    def block(self, flat: np.ndarray, b: int) -> np.ndarray:
        """View of patch b's block in a flat buffer, shape [s, p, p, p]."""
        p = int(self.sizes[b])
        o = int(self.offsets()[b])
        return flat[o:o + self.s * p ** 3].reshape(self.s, p, p, p)


def uneven_batch(n: int = 20000, seed: int = 0, sizes=UNEVEN_SIZES, ratio=UNEVEN_RATIO,
                 levels=UNEVEN_LEVELS, modes: int = 2) -> Tuple[UnevenBatch, np.ndarray]:
    """Seeded uneven batch and its initial state (flat compact buffer).

    With rng = numpy.random.default_rng(seed): sizes drawn per patch from
    ``sizes`` with probabilities proportional to ``ratio`` (4^3 : 8^3 : 16^3
    = 4 : 2 : 1 by default), then levels drawn uniformly from ``levels``, in
    patch order.  Fields, per size class in ascending p and patch order: for
    rho, p, u, v, w in that order, g = mean over ``modes`` modes of
    sin(2 pi k . x + phi) in patch-local coordinates x = (i + 1/2) / p_b, with
    k drawn from {-1, 0, 1}^3 minus zero (periodic on the patch) and phi from
    U[0, 2 pi); then rho = 1 + 0.5 g, p = 1.25 + 0.75 g, u_j = 0.5 g, as for
    the 4096 x 8^3 grid.
    """
    rng = np.random.default_rng(seed)
    prob = np.asarray(ratio, dtype=np.float64)
    prob = prob / prob.sum()
    sz = rng.choice(np.asarray(sizes, dtype=np.int64), size=n, p=prob)
    lv = rng.choice(np.asarray(levels, dtype=np.int64), size=n)
    batch = UnevenBatch(sz, lv)
    q = np.empty(batch.buffer_len())
    off = batch.offsets()
    for p in sorted(set(int(v) for v in sz)):
        idx = np.nonzero(sz == p)[0]
        m = idx.shape[0]
        x = (np.arange(p) + 0.5) / p
        zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
        fields = []
        for _ in range(5):
            g = np.zeros((m, p, p, p))
            for _ in range(modes):
                k = rng.integers(-1, 2, size=(m, 3))
                zero = ~k.any(axis=1)
                while zero.any():
                    k[zero] = rng.integers(-1, 2, size=(int(zero.sum()), 3))
                    zero = ~k.any(axis=1)
                phi = rng.uniform(0.0, 2 * np.pi, size=m)
                arg = (2 * np.pi * (k[:, 0, None, None, None] * xx + k[:, 1, None, None, None] * yy
                                    + k[:, 2, None, None, None] * zz) + phi[:, None, None, None])
                g += np.sin(arg)
            fields.append(g / modes)
        rho = 1.0 + 0.5 * fields[0]
        pres = 1.25 + 0.75 * fields[1]
        qc = to_conserved(rho, [0.5 * g for g in fields[2:]], pres)  # [s, m, p, p, p]
        qc = np.moveaxis(qc, 1, 0).reshape(m, -1)
        blk = 5 * p ** 3
        for j, b in enumerate(idx):
            q[off[b]:off[b] + blk] = qc[j]
    return batch, q


def grid_riemann_2d(patches_per_axis: int = 16, p: int = 16, seed: int = 0,
                    rho=(0.1, 1.0), pres=(0.1, 1.0), vel=(-1.0, 1.0)
                    ) -> Tuple[PatchGrid, np.ndarray]:
    """Seeded 2-D four-quadrant Riemann problem on the unit square.

    With rng = numpy.random.default_rng(seed): the split point (x0, y0) ~
    U[0.3, 0.7]^2, then for the quadrants (x < x0, y < y0), (x >= x0, y < y0),
    (x < x0, y >= y0), (x >= x0, y >= y0) in that order rho ~ U[rho], p ~
    U[pres], u ~ U[vel], v ~ U[vel].  Transmissive boundaries on both axes.
    """
    n = patches_per_axis * p
    grid = PatchGrid(2, p, (patches_per_axis, patches_per_axis), 1.0 / n,
                     bc=(TRANSMISSIVE, TRANSMISSIVE))
    x, y = grid.cell_centres()
    rng = np.random.default_rng(seed)
    x0, y0 = rng.uniform(0.3, 0.7, size=2)
    states = []
    for _ in range(4):
        states.append((rng.uniform(*rho), rng.uniform(*pres), rng.uniform(*vel),
                       rng.uniform(*vel)))
    X, Y = np.meshgrid(x, y, indexing="xy")
    quad = (X >= x0).astype(int) + 2 * (Y >= y0).astype(int)
    r = np.choose(quad, [s[0] for s in states])
    pr = np.choose(quad, [s[1] for s in states])
    u = np.choose(quad, [s[2] for s in states])
    v = np.choose(quad, [s[3] for s in states])
    return grid, to_conserved(r, [u, v], pr)
