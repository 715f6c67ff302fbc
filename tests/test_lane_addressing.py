"""CPU model of the per-lane addressing of the update kernels.

The plane-marching update (every instance of fv_update_kernel, the mixed-size
persistent kernel's 256-thread bodies) and the learned-correction update
compute their global and LDS addresses from the thread index, the patch
geometry and the neighbour table.  This file restates that index arithmetic
for every thread of a workgroup and checks, on the CPU, that

  * every global load of an active lane falls inside a block the lane may
    read (its own input block, or a face neighbour's block in the gather
    form), and every store inside its own output block, interior only;
  * every LDS index lies inside the lane's own part of the workgroup's LDS
    (its chunk's slot), and the slots of a workgroup do not overlap;
  * the halo cells read from LDS are exactly those the load phase wrote,
    and every face flux read was written;
  * the values each lane loads are the ones the scheme needs (the own
    column, the face-halo ring of each plane, the facing neighbour layer).

It is a model: it does not run the kernels, it re-derives their addresses
from the same layout rules, so a kernel edit that changes its indexing must
be mirrored here.
"""
import itertools
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ceil_div(a, b):
    return -(-a // b)


def zsplit(d, p):
    """Chunks along the marching axis of the single-size kernels."""
    return {(3, 8): 1, (2, 16): 4, (2, 17): 3, (2, 32): 2}.get((d, p), 1)


class Geo:
    """Patch geometry and thread layout of one update instance."""

    def __init__(self, d, p, ntw=64, zs=None):
        self.d, self.p, self.ntw = d, p, ntw
        self.zs = zsplit(d, p) if zs is None else zs
        self.s = d + 2
        self.w = p + 2
        self.vin = self.w ** d
        self.vout = p ** d
        self.sm = self.w ** (d - 1)
        self.smo = p ** (d - 1)
        self.lanes = p ** (d - 1)
        self.pc = ceil_div(p, self.zs)
        self.tpp = self.zs * self.lanes
        self.ppw = 1 if self.tpp >= ntw else ntw // self.tpp
        self.nt = ceil_div(self.ppw * self.tpp, 64) * 64
        self.ring = 4 * p if d == 3 else 2
        self.nextra = 2 * p if d == 3 else 1
        self.ncell = self.lanes + self.ring
        self.nv = self.s + 3
        self.nf = self.lanes + (p if d == 3 else 1)
        self.cellbuf = self.nv * self.ncell
        self.facebuf = (d - 1) * self.s * self.nf
        self.slot = max(self.cellbuf, self.facebuf)
        self.nred = max(self.nt // 64, self.ppw * self.zs)
        self.uneven = p % self.zs != 0
        # the kernels' static_asserts
        assert self.ring <= self.lanes
        assert self.zs == 1 or self.lanes == 64 or self.zs * self.lanes <= 64
        assert p % self.zs == 0 or self.zs * self.lanes <= 64
        assert (self.zs - 1) * self.pc < p
        assert self.nextra <= self.lanes
        assert self.ppw * self.tpp <= self.nt


SINGLE = [(2, 4), (2, 8), (2, 16), (2, 17), (2, 32), (3, 4), (3, 8), (3, 16)]
MIXED = [(3, 4), (3, 8), (3, 16)]


def lds_elements_single(g):
    return g.ppw * g.zs * g.slot


def mixed_geo(p):
    """Body geometry of one work unit of the persistent mixed-size kernel: a
    16^3 patch takes the whole 256-thread workgroup; 8^3 and 4^3 units are
    run wave by wave with the one-wave body (one 8^3 or four 4^3 patches per
    wave), each wave in its own LDS and reduction region."""
    return Geo(3, p, 256, 1) if p == 16 else Geo(3, p, 64, 1)


def mixed_waves(p):
    return 1 if p == 16 else 4


def wave_lds_mixed():
    """LDS elements each wave owns in the per-wave bodies: the larger of the
    8^3 and 4^3 needs, so that wave w's region is the same for both sizes."""
    return max(mixed_geo(p).ppw * mixed_geo(p).slot for p in (4, 8))


def wave_red_mixed():
    return max(mixed_geo(p).nred for p in (4, 8))


def lds_elements_mixed():
    return max(mixed_geo(16).slot, 4 * wave_lds_mixed())


def red_elements_mixed():
    return max(mixed_geo(16).nred, 4 * wave_red_mixed())


class Block:
    """A block of one patch: (patch id, kind) where kind is 'in' or 'out'."""


def thread_accesses(g, gather, out_halo, nb_present):
    """Every access of every thread of one workgroup whose slots all hold
    patches.  Patch slot k is patch k; its face neighbours are patches
    100 + 2d*k + f when nb_present[f] (gather form), else the face is
    transmissive.  Returns a list of records
      (tid, kind, block, index)   kind 'ld' / 'st' / 'lds_w' / 'lds_r' / 'red_w' / 'red_r'
    with block = (patch, 'in' | 'out') and index the element index inside
    that block, or block None and index the element index into the
    workgroup's LDS (or reduction) array."""
    d, p, s = g.d, g.p, g.s
    K = d - 1
    CS = g.vout if gather else g.vin
    PS = g.smo if gather else g.sm
    rec = []
    for tid in range(g.nt):
        slot = 0 if g.ppw == 1 else tid // g.tpp
        tp = tid if g.ppw == 1 else tid - slot * g.tpp
        chunk = 0 if g.zs == 1 else tp // g.lanes
        l = tp if g.zs == 1 else tp - chunk * g.lanes
        p0 = chunk * g.pc
        nrows = min(p - p0, g.pc) if g.uneven else g.pc
        in_patch = g.ppw * g.tpp == g.nt or tid < g.ppw * g.tpp
        in_range = in_patch and (g.ppw == 1 or slot < g.ppw)
        act = in_range  # every descriptor valid
        x = l % p
        y = l // p if d == 3 else 0
        has_ring = l < g.ring
        q4 = l // p if d == 3 else l
        rr = l - q4 * p if d == 3 else 0
        if not act:
            continue
        own = (slot, "in")
        # neighbour blocks of the gather form: face order -x, +x, -y, +y, -z, +z
        nbk = [(100 + 2 * d * slot + f, "in") if nb_present[f] else None for f in range(2 * d)]
        col_c = x + (y * p if d == 3 else 0)
        col_h = (x + 1) + ((y + 1) * g.w if d == 3 else 0)
        if d == 3:
            ring_h = [(rr + 1) * g.w, (p + 1) + (rr + 1) * g.w, rr + 1,
                      (rr + 1) + (p + 1) * g.w][q4] if q4 < 4 else (rr + 1) + (p + 1) * g.w
        else:
            ring_h = 0 if l == 0 else p + 1
        col_in = col_c if gather else col_h
        jin = p0 if gather else p0 + 1
        # (block, element index) of the first unknown of each source column
        gin = (own, col_in + jin * PS)
        last = (p - 1) * g.smo
        fl, fh = 2 * K, 2 * K + 1
        if gather and chunk == 0:
            glo = (nbk[fl], last + col_c) if nbk[fl] else (own, col_c)
        else:
            glo = (own, gin[1] - PS)
        if gather and chunk == g.zs - 1:
            ghi = (nbk[fh], col_c) if nbk[fh] else (own, last + col_c)
        else:
            ghi = (own, gin[1] + nrows * PS)
        if gather:
            if has_ring:
                hasnb = nbk[q4] is not None
                if d == 3:
                    idx = [(p - 1 if hasnb else 0) + p * rr, (0 if hasnb else p - 1) + p * rr,
                           rr + p * (p - 1 if hasnb else 0), rr + p * (0 if hasnb else p - 1)][q4]
                else:
                    idx = (p - 1 if hasnb else 0) if q4 == 0 else (0 if hasnb else p - 1)
                gring = (nbk[q4] if hasnb else own, idx + p0 * PS)
            else:
                gring = (own, col_c + p0 * PS)
        else:
            gring = (own, ring_h + PS + p0 * PS)

        def ld_own(j, m):
            if j == 0:
                return (glo[0], glo[1] + m * CS)
            if j == nrows + 1:
                return (ghi[0], ghi[1] + m * CS)
            return (own, gin[1] + m * CS + (j - 1) * PS)

        def ld_ring(j, m):
            return (gring[0], gring[1] + m * CS + (j - 1) * PS)

        for m in range(s):
            rec.append((tid, "ld", *ld_own(0, m)))
            rec.append((tid, "ld", *ld_own(1, m)))
            rec.append((tid, "ld", *ld_ring(1, m)))
        cell = (slot * g.zs + chunk) * g.slot
        col_out = col_h + g.sm if out_halo else col_c
        ostride = g.sm if out_halo else g.smo
        ocomp = g.vin if out_halo else g.vout
        fx_lo = l
        fx_hi = l + 1 if x < p - 1 else g.lanes + (y if d == 3 else 0)
        fy_lo = l
        fy_hi = l + p
        for pl in range(g.pc):
            live = not g.uneven or pl < nrows
            if not live:
                continue
            if pl + 1 < nrows:
                for m in range(s):
                    rec.append((tid, "ld", *ld_ring(pl + 2, m)))
            for m in range(s):
                rec.append((tid, "ld", *ld_own(pl + 2, m)))
            # A
            for m in range(g.nv):
                rec.append((tid, "lds_w", None, cell + m * g.ncell + l))
                if has_ring:
                    rec.append((tid, "lds_w", None, cell + m * g.ncell + g.lanes + l))
            # B
            if l < g.nextra:
                ydir = d == 3 and l >= p
                t = l - p if ydir else l
                if d == 3:
                    lc = (p - 1) * p + t if ydir else t * p + (p - 1)
                    rc = g.lanes + 3 * p + t if ydir else g.lanes + p + t
                else:
                    lc, rc = p - 1, g.lanes + 1
                for m in range(g.nv):
                    rec.append((tid, "lds_r", None, cell + m * g.ncell + lc))
                    rec.append((tid, "lds_r", None, cell + m * g.ncell + rc))
            nb = l - 1 if x > 0 else g.lanes + (y if d == 3 else 0)
            for m in range(g.nv):
                rec.append((tid, "lds_r", None, cell + m * g.ncell + nb))
            if d == 3:
                nb = l - p if y > 0 else g.lanes + 2 * p + x
                for m in range(g.nv):
                    rec.append((tid, "lds_r", None, cell + m * g.ncell + nb))
            # C
            for m in range(s):
                rec.append((tid, "lds_wf", None, cell + m * g.nf + fx_lo))
                if d == 3:
                    rec.append((tid, "lds_wf", None, cell + (s + m) * g.nf + fy_lo))
            if l < g.nextra:
                ydir = d == 3 and l >= p
                t = l - p if ydir else l
                base = s * g.nf + p * p + t if ydir else g.lanes + t
                for m in range(s):
                    rec.append((tid, "lds_wf", None, cell + base + m * g.nf))
            # D
            for m in range(s):
                rec.append((tid, "lds_rf", None, cell + m * g.nf + fx_hi))
                rec.append((tid, "lds_rf", None, cell + m * g.nf + fx_lo))
                if d == 3:
                    rec.append((tid, "lds_rf", None, cell + (s + m) * g.nf + fy_hi))
                    rec.append((tid, "lds_rf", None, cell + (s + m) * g.nf + fy_lo))
                rec.append((tid, "st", (slot, "out"),
                            col_out + (p0 * ostride) + m * ocomp + pl * ostride))
        # per-patch maximum
        pow2 = (g.lanes & (g.lanes - 1)) == 0
        if pow2:
            if g.lanes > 64:
                if (tid & 63) == 0:
                    rec.append((tid, "red_w", None, tid >> 6))
                if tid == 0:
                    for wv in range(1, g.lanes // 64):
                        rec.append((tid, "red_r", None, wv))
            elif g.zs > 1:
                if l == 0:
                    rec.append((tid, "red_w", None, slot * g.zs + chunk))
                if l == 0 and chunk == 0:
                    for c in range(1, g.zs):
                        rec.append((tid, "red_r", None, slot * g.zs + c))
        else:
            rec.append((tid, "lds_max_w", None, tid if tid < g.ppw * g.slot else 0))
            if l == 0 and chunk == 0:
                for i in range(1, g.tpp):
                    rec.append((tid, "lds_max_r", None, slot * g.tpp + i))
    return rec


def _instances():
    for (d, p), gather, out_halo in itertools.product(SINGLE, (False, True), (False, True)):
        yield Geo(d, p), lds_elements_single(Geo(d, p)), gather, out_halo, "single"
    for d, p in MIXED:
        # one wave's body (8^3, 4^3) or the workgroup's (16^3); its LDS region
        # of the mixed kernel's array is checked against the whole array
        yield mixed_geo(p), lds_elements_mixed(), True, False, "mixed"


def _nb_cases(g, gather):
    if not gather:
        return [(True,) * (2 * g.d)]
    return [(True,) * (2 * g.d), (False,) * (2 * g.d),
            tuple(f % 2 == 0 for f in range(2 * g.d)), tuple(f % 3 == 1 for f in range(2 * g.d))]


@pytest.mark.parametrize("g,lds_total,gather,out_halo,kind",
                         list(_instances()),
                         ids=lambda v: (f"d{v.d}p{v.p}nt{v.ntw}" if isinstance(v, Geo) else str(v)))
def test_update_lane_addresses_stay_in_their_blocks(g, lds_total, gather, out_halo, kind):
    d, p, s = g.d, g.p, g.s
    blk_in = s * (g.vout if gather else g.vin)
    blk_out = s * (g.vin if out_halo else g.vout)
    for nbp in _nb_cases(g, gather):
        rec = thread_accesses(g, gather, out_halo, nbp)
        stores = {}
        for tid, kindr, blk, idx in rec:
            slot = 0 if g.ppw == 1 else tid // g.tpp
            chunk = 0 if g.zs == 1 else (tid - slot * g.tpp) // g.lanes
            if kindr == "ld":
                assert blk is not None
                pid, role = blk
                assert role == "in"
                # own block, or a face neighbour of this thread's patch
                assert pid == slot or 100 + 2 * d * slot <= pid < 100 + 2 * d * (slot + 1), \
                    (tid, blk)
                assert 0 <= idx < blk_in, (tid, blk, idx)
            elif kindr == "st":
                pid, role = blk
                assert pid == slot and role == "out"
                assert 0 <= idx < blk_out, (tid, idx)
                stores.setdefault(pid, []).append(idx)
            elif kindr in ("lds_w", "lds_r"):
                lo = (slot * g.zs + chunk) * g.slot
                assert lo <= idx < lo + g.cellbuf, (tid, kindr, idx)
                assert idx < lds_total
            elif kindr in ("lds_wf", "lds_rf"):
                lo = (slot * g.zs + chunk) * g.slot
                assert lo <= idx < lo + g.facebuf, (tid, kindr, idx)
                assert idx < lds_total
            elif kindr in ("red_w", "red_r"):
                assert 0 <= idx < g.nred, (tid, kindr, idx)
            elif kindr in ("lds_max_w", "lds_max_r"):
                assert 0 <= idx < lds_total, (tid, kindr, idx)
            else:
                raise AssertionError(kindr)
        # every interior volume of every output block is stored exactly once
        # per unknown, and nothing else
        for pid in range(g.ppw):
            got = np.sort(np.array(stores[pid]))
            want = []
            for m in range(s):
                for z in range(p if d == 3 else 1):
                    for y in range(p):
                        for x in range(p):
                            if out_halo:
                                i = (x + 1) + g.w * (y + 1) + (g.w * g.w * (z + 1) if d == 3 else 0)
                                want.append(m * g.vin + i)
                            else:
                                want.append(m * g.vout + x + p * y + p * p * z)
            np.testing.assert_array_equal(got, np.sort(np.array(want)))


def _column_coords(g, idx, gather):
    """Coordinates (x, y[, z]) of an element index inside a block (unknown
    stripped), halo'd when not gather."""
    v = g.vout if gather else g.vin
    w = g.p if gather else g.w
    i = idx % v
    c = []
    for _ in range(g.d):
        c.append(i % w)
        i //= w
    return tuple(c)


@pytest.mark.parametrize("d,p", SINGLE)
@pytest.mark.parametrize("gather", [False, True])
def test_update_loads_read_the_stencil(d, p, gather):
    """The volumes a patch loads are its interior and exactly its 2d face-halo
    layers (halo form: the block's own halo; gather form: the facing layer of
    each neighbour, or the own boundary layer at a transmissive face), never
    an edge or corner."""
    g = Geo(d, p)
    for nbp in _nb_cases(g, gather):
        rec = thread_accesses(g, gather, False, nbp)
        seen = set()
        for tid, kindr, blk, idx in rec:
            if kindr != "ld":
                continue
            slot = 0 if g.ppw == 1 else tid // g.tpp
            if slot != 0:
                continue
            c = _column_coords(g, idx, gather)
            pid = blk[0]
            if pid == 0:
                if gather:
                    seen.add(("own",) + c)
                else:
                    seen.add(("halo",) + tuple(ci - 1 for ci in c))
            else:
                f = pid - 100
                seen.add(("nb", f) + c)
        # expected set, in patch-interior coordinates (-1 .. p on each axis)
        want = set()
        for c in itertools.product(range(p), repeat=d):
            want.add(("own",) + c if gather else ("halo",) + c)
        for f in range(2 * d):
            ax, side = divmod(f, 2)
            for t in itertools.product(range(p), repeat=d - 1):
                tl = list(t)
                c = tl[:ax] + [(-1 if side == 0 else p)] + tl[ax:]
                if not gather:
                    want.add(("halo",) + tuple(c))
                elif nbp[f]:
                    # the facing layer of the neighbour
                    c2 = list(c)
                    c2[ax] = p - 1 if side == 0 else 0
                    want.add(("nb", 2 * d * 0 + f) + tuple(c2))
                else:
                    c2 = list(c)
                    c2[ax] = 0 if side == 0 else p - 1
                    want.add(("own",) + tuple(c2))
        assert seen == want, (sorted(seen - want)[:5], sorted(want - seen)[:5])


def test_workgroup_lds_fits_and_slots_are_disjoint():
    """Each chunk's slot is within the static LDS array and the reduction
    array holds one entry per chunk or wave; the learned update's LDS layout
    fits the 160 KB of a CU (64 KB per workgroup as declared)."""
    for d, p in SINGLE:
        g = Geo(d, p)
        assert g.ppw * g.zs * g.slot == lds_elements_single(g)
        assert g.nred >= g.ppw * g.zs and g.nred >= g.nt // 64
        assert lds_elements_single(g) * 8 + g.nred * 8 <= 64 * 1024
    assert lds_elements_mixed() * 8 <= 64 * 1024
    # the mixed kernel's per-wave regions: wave w of a unit owns elements
    # [w * W, (w + 1) * W) and reduction entries [w * R, (w + 1) * R) for
    # both per-wave sizes; each size's needs fit its wave's region
    for p in (4, 8):
        g = mixed_geo(p)
        assert g.nt == 64 and g.ppw * g.tpp == 64
        assert g.ppw * g.slot <= wave_lds_mixed() and g.nred <= wave_red_mixed()
    assert 4 * wave_lds_mixed() <= lds_elements_mixed()
    assert 4 * wave_red_mixed() <= red_elements_mixed()
    # patches per work unit, as the host plan counts them (fv_plan_mixed)
    assert [mixed_waves(p) * mixed_geo(p).ppw for p in (16, 8, 4)] == [1, 4, 16]


def _regions(p, w):
    g = mixed_geo(p)
    lds = (w * wave_lds_mixed(), w * wave_lds_mixed() + g.ppw * g.slot)
    red = (w * wave_red_mixed(), w * wave_red_mixed() + g.nred)
    return lds, red


def test_mixed_waves_never_share_a_region():
    """A wave of the persistent kernel moves from its 8^3 units to 4^3 units
    without waiting for the other waves: the region wave w uses for either
    size overlaps no region of another wave for either size.  (With each
    size's own stride, 768 and 1024 doubles, they overlapped.)  The 16^3
    units, which use the whole array, end with a workgroup barrier."""
    overlap = lambda a, b: a[0] < b[1] and b[0] < a[1]
    for p, p2 in itertools.product((8, 4), repeat=2):
        for w, w2 in itertools.product(range(4), repeat=2):
            if w == w2:
                continue
            (l1, r1), (l2, r2) = _regions(p, w), _regions(p2, w2)
            assert not overlap(l1, l2) and not overlap(r1, r2), (p, w, p2, w2)
    g8, g4 = mixed_geo(8), mixed_geo(4)
    assert g8.ppw * g8.slot != g4.ppw * g4.slot  # why the common stride matters
    src = open(os.path.join(ROOT, "paper_2302_09005_amd", "csrc", "fv_update_kernels.hpp")).read()
    body = src[src.index("fv_mixed_kernel("):]
    body = body[:body.index("\n}\n")]
    assert body.count("lds + wave * kMixedWaveLds, red + wave * kMixedWaveRed") == 2
    first = body[body.index("for (; u < u8;"):body.index("for (; u < u4;")]
    assert "__syncthreads()" in first


# ---------------------------------------------------------------------------
# the learned-correction update (2-D, 16 x 16 patches, two-volume face halo)
# ---------------------------------------------------------------------------
LP, LH = 16, 2
LW = LP + 2 * LH
NXF = (LP + 1) * LP
NFACE = 2 * NXF


def learned_loaded_cells(nb_present):
    """LDS cells (y, x) of s.q the load phase writes, and the source (block,
    y, x) of each: 256 interior threads and 128 halo threads."""
    cells = {}
    for tid in range(LP * LP):
        x, y = tid & 15, tid >> 4
        cells[(y + LH, x + LH)] = ("own", y, x)
    for tid in range(128):
        side, t = tid >> 5, tid & 31
        layer, pos = t >> 4, t & 15
        has = nb_present[side]
        if side == 0:
            hx, hy, sx, sy = layer, pos + LH, (LP - 2 + layer if has else 0), pos
        elif side == 1:
            hx, hy, sx, sy = LP + LH + layer, pos + LH, (layer if has else LP - 1), pos
        elif side == 2:
            hx, hy, sx, sy = pos + LH, layer, pos, (LP - 2 + layer if has else 0)
        else:
            hx, hy, sx, sy = pos + LH, LP + LH + layer, pos, (layer if has else LP - 1)
        assert 0 <= sx < LP and 0 <= sy < LP
        assert (hy, hx) not in cells
        cells[(hy, hx)] = (("nb", side) if has else "own", sy, sx)
    return cells


@pytest.mark.parametrize("nb_present", [(True,) * 4, (False,) * 4, (True, False, False, True)])
@pytest.mark.parametrize("nth", [256, 512])
def test_learned_update_reads_only_loaded_cells_and_written_fluxes(nb_present, nth):
    cells = learned_loaded_cells(nb_present)
    # the transmissive halo repeats the boundary volume; a neighbour's halo is
    # its facing two layers
    for (hy, hx), (src, sy, sx) in cells.items():
        iy, ix = hy - LH, hx - LH
        if 0 <= iy < LP and 0 <= ix < LP:
            assert (sy, sx) == (iy, ix) and src == "own"
        elif src == "own":
            assert (sy, sx) == (min(max(iy, 0), LP - 1), min(max(ix, 0), LP - 1))
        else:
            assert (sy, sx) == (iy % LP, ix % LP)
    fx_w, fy_w = set(), set()
    waves = nth // 64
    for wave in range(waves):
        batch = wave
        while batch * 64 < NFACE:
            for l in range(64):
                f = batch * 64 + l
                real = f < NFACE
                ff = f if real else NFACE - 1
                xdir = ff < NXF
                gidx = ff if xdir else ff - NXF
                if xdir:
                    I, J = gidx % (LP + 1), gidx // (LP + 1)
                else:
                    I, J = gidx % LP, gidx // LP
                for o in range(4):
                    cx = I - 2 + o + LH if xdir else I + LH
                    cy = J + LH if xdir else J - 2 + o + LH
                    assert 0 <= cx < LW and 0 <= cy < LW
                    assert (cy, cx) in cells, (xdir, I, J, o)
                if real:
                    if xdir:
                        assert 0 <= I <= LP and 0 <= J < LP
                        fx_w.add((J, I))
                    else:
                        assert 0 <= I < LP and 0 <= J <= LP
                        fy_w.add((J, I))
            batch += waves
    # every face written once overall, and the update reads only those
    assert len(fx_w) == NXF and len(fy_w) == NXF
    for tid in range(LP * LP):
        x, y = tid & 15, tid >> 4
        assert {(y, x), (y, x + 1)} <= fx_w and {(y, x), (y + 1, x)} <= fy_w


def _push_stores(g, counts, bcs):
    """The PUSH form (halo'd input and output, the new state's boundary
    volumes also stored into the face halos that read them) on a small patch
    grid: every push store of every thread of every patch, as
    (destination element, source patch, unknown, source coords).  Output
    block b sits at element offset b * s * (p+2)^d.  The pushed shift per
    face restates the kernel: to the neighbour's block, moved by P along the
    face axis away from the face (low face) or towards it (high face), or at
    a transmissive face by one volume out of the own block."""
    d, p, s, w = g.d, g.p, g.s, g.w
    K = d - 1
    npat = int(np.prod(counts))
    blk = s * g.vin
    pc_ = np.array(np.unravel_index(np.arange(npat), counts[::-1]))[::-1].T  # (x, y[, z])
    strides = np.cumprod((1,) + tuple(counts[:-1]))

    def nb(b, f):
        a, side = f // 2, f % 2
        c = pc_[b].copy()
        c[a] += 1 if side else -1
        if c[a] < 0 or c[a] >= counts[a]:
            if bcs[a] == "transmissive":
                return -1
            c[a] %= counts[a]
        return int((c * strides).sum())

    out = []
    for b in range(npat):
        off_out = b * blk
        pshift = []
        for f in range(2 * d):
            a_str = 1 if f < 2 else (w if f < 4 else w * w)
            n_ = nb(b, f)
            hi = f & 1
            if n_ >= 0:
                assert nb(n_, f ^ 1) == b  # a grid's table is mutual
                pshift.append((n_ * blk - off_out) + (-p if hi else p) * a_str)
            else:
                pshift.append(a_str if hi else -a_str)
        for tid in range(g.tpp):
            chunk = 0 if g.zs == 1 else tid // g.lanes
            l = tid if g.zs == 1 else tid - chunk * g.lanes
            p0 = chunk * g.pc
            nrows = min(p - p0, g.pc) if g.uneven else g.pc
            x = l % p
            y = l // p if d == 3 else 0
            col_h = (x + 1) + ((y + 1) * w if d == 3 else 0)
            col_out = col_h + g.sm
            for pl in range(g.pc):
                if g.uneven and pl >= nrows:
                    continue
                zz = p0 + pl
                src = (x, y, zz) if d == 3 else (x, zz)
                faces = [f for f in range(2 * K)
                         if (x if f // 2 == 0 else y) == (p - 1 if f & 1 else 0)]
                if zz == 0:
                    faces.append(2 * K)
                if zz == p - 1:
                    faces.append(2 * K + 1)
                for f in faces:
                    for m in range(s):
                        dst = off_out + col_out + p0 * g.sm + m * g.vin + pl * g.sm + pshift[f]
                        out.append((dst, b, m, src))
    return out, nb, npat, blk


@pytest.mark.parametrize("d,p,counts", [(2, 4, (5, 3)), (2, 8, (3, 3)), (2, 16, (3, 2)),
                                        (2, 17, (3, 2)), (2, 32, (2, 2)), (3, 4, (3, 2, 2)),
                                        (3, 8, (3, 2, 2)), (3, 16, (2, 2, 1))])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_push_stores_fill_every_face_halo_once(d, p, counts, bc):
    """Every face-halo slot of every output block receives exactly one push,
    of the volume the pull-form halo fill would copy there (the facing
    boundary volume of the neighbour, or the own boundary volume at a
    transmissive face); no push lands on an interior, edge or corner slot."""
    g = Geo(d, p)
    bcs = ("periodic",) * d if bc == "periodic" else ("transmissive",) + ("periodic",) * (d - 1)
    stores, nb, npat, blk = _push_stores(g, counts, bcs)
    w, s = g.w, g.s
    seen = {}
    for dst, b, m, src in stores:
        assert 0 <= dst < npat * blk
        assert dst not in seen, dst
        seen[dst] = (b, m, src)
    want = {}
    for b in range(npat):
        for f in range(2 * d):
            a, hi = f // 2, f & 1
            n_ = nb(b, f)
            for m in range(s):
                for t in itertools.product(range(p), repeat=d - 1):
                    hc = list(t[:a]) + [0] + list(t[a:])
                    hc = [c + 1 for c in hc]
                    hc[a] = w - 1 if hi else 0
                    sc = [c - 1 for c in hc]
                    if n_ >= 0:
                        sc[a] = 0 if hi else p - 1
                        srcp = n_
                    else:
                        sc[a] = p - 1 if hi else 0
                        srcp = b
                    idx = sum(c * w ** k for k, c in enumerate(hc))
                    want[b * blk + m * g.vin + idx] = (srcp, m, tuple(sc))
    assert set(seen) == set(want)
    for k, v in want.items():
        assert seen[k] == v, (k, seen[k], v)


# ---------------------------------------------------------------------------
# CFL workspace words of the fused and the pipelined step (the kernels'
# index arithmetic restated): every word a launch touches lies inside the
# workspace the library asks for, and the pipelined step's three slot sets
# keep their roles apart.
# ---------------------------------------------------------------------------
CFL_GROUP, CFL_WORD = 64, 32
CFL_SLOT = 3 * CFL_WORD
PIPE_SLOTS = 16


def _fused_words(nwg):
    """Words of fv_step_gather's tree: group slots (count, lambda, h) and the top count."""
    ngrp = ceil_div(nwg, CFL_GROUP)
    words = {0}  # top arrival count
    for w in range(nwg):
        g = w // CFL_GROUP
        base = CFL_SLOT * (g + 1)
        words |= {base, base + CFL_WORD, base + 2 * CFL_WORD}
    return words, ngrp


def _pipelined_words(nwg, phase, dt_given):
    """(read, folded, cleared) words of one fv_step_gather_pipelined launch."""
    rd = set()
    if not dt_given:
        base = CFL_SLOT * PIPE_SLOTS * ((phase + 2) % 3)
        rd = {base + CFL_SLOT * s + k for s in range(PIPE_SLOTS) for k in (CFL_WORD, 2 * CFL_WORD)}
    fold = set()
    for w in range(nwg):
        base = CFL_SLOT * (PIPE_SLOTS * phase + w % PIPE_SLOTS)
        fold |= {base + CFL_WORD, base + 2 * CFL_WORD}
    base = CFL_SLOT * PIPE_SLOTS * ((phase + 1) % 3)
    clr = {base + CFL_SLOT * s + k for s in range(PIPE_SLOTS) for k in (CFL_WORD, 2 * CFL_WORD)}
    return rd, fold, clr


@pytest.mark.parametrize("d,p,n", [(3, 8, 4096), (3, 8, 4097), (3, 8, 1), (2, 16, 100),
                                   (3, 4, 1000), (2, 4, 77), (3, 16, 130), (3, 8, 32768)])
def test_cfl_workspace_words_stay_inside_the_workspace(d, p, n):
    from paper_2302_09005_amd import fv
    g = Geo(d, p)
    nwg = ceil_div(n, g.ppw)
    words, _ = _fused_words(nwg)
    assert max(words) < fv.step_workspace_words(n, d, p)
    need = fv.pipelined_workspace_words(n, d, p)
    for phase in range(3):
        for given in (False, True):
            rd, fold, clr = _pipelined_words(nwg, phase, given)
            assert max(rd | fold | clr) < need
            # a launch reads one set, folds into another and clears the third
            assert not (rd & fold) and not (rd & clr) and not (fold & clr)


def test_pipelined_slot_sets_cycle_through_write_read_clear():
    """Launch j folds into a set, launch j+1 reads it, launch j+2 clears it
    and launch j+3 folds into it again: each set is cleared after its last
    read and before its next fold."""
    nwg = 300
    for first in range(3):
        roles = []
        for j in range(9):
            roles.append(_pipelined_words(nwg, (first + j) % 3, j == 0))
        for j in range(1, 6):
            assert roles[j][0] == roles[j - 1][1]      # j reads what j-1 folded
            assert roles[j + 1][2] == roles[j - 1][1]  # j+1 clears it after that read
            assert roles[j + 2][1] == roles[j + 1][2]  # j+2 folds into the cleared set
