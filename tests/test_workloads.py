"""Host-side checks of the seeded input generators (CPU)."""
import numpy as np
import pytest

from paper_2302_09005_amd import workloads as W


def test_descriptor_record_is_64_bytes():
    assert W.PATCH_DTYPE.itemsize == 64
    assert W.PATCH_DTYPE.fields["dx"][1] == 24
    assert W.PATCH_DTYPE.fields["dt"][1] == 48


@pytest.mark.parametrize("d", [2, 3])
def test_pack_unpack_roundtrip_and_nan_corners(d):
    rng = np.random.default_rng(0)
    grid = W.PatchGrid(d, 4, (3, 2, 2)[:d], 0.1)
    q = rng.standard_normal((d + 2,) + grid.shape)
    flat = grid.pack(q)
    assert flat.size == grid.buffer_len()
    np.testing.assert_array_equal(grid.unpack(flat), q)
    w = grid.p + 2
    n_corner = w ** d - grid.p ** d - 2 * d * grid.p ** (d - 1)
    assert np.isnan(flat).sum() == grid.n * (d + 2) * n_corner
    order = rng.permutation(grid.n)
    flat2 = grid.pack(q, order=order, gap=5, fill=0.0)
    np.testing.assert_array_equal(grid.unpack(flat2, order=order, gap=5), q)


def test_neighbours_periodic_and_transmissive():
    grid = W.PatchGrid(3, 2, (3, 2, 2), 0.1, ("transmissive", "periodic", "periodic"))
    nb = grid.neighbours()
    pc = grid.patch_coords()
    for b in range(grid.n):
        x, y, z = pc[b]
        assert nb[b, 0] == (-1 if x == 0 else b - 1)
        assert nb[b, 1] == (-1 if x == 2 else b + 1)
        assert pc[nb[b, 2]].tolist() == [x, (y - 1) % 2, z]
        assert pc[nb[b, 5]].tolist() == [x, y, (z + 1) % 2]


def test_paper_shaped_fields_ranges_and_seeds():
    g, q = W.grid_3d_random_smooth(2, 4, seed=0)
    _, q2 = W.grid_3d_random_smooth(2, 4, seed=0)
    _, q3 = W.grid_3d_random_smooth(2, 4, seed=1)
    np.testing.assert_array_equal(q, q2)
    assert not np.array_equal(q, q3)
    rho = q[0]
    u = q[1:4] / rho
    p = 0.4 * (q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / rho)
    assert rho.min() >= 0.5 and rho.max() <= 1.5
    assert p.min() >= 0.5 - 1e-12 and p.max() <= 2.0 + 1e-12
    assert np.abs(u).max() <= 0.5 + 1e-12
    g2, q2d = W.grid_2d_smooth()
    assert g2.n == 64 and g2.p == 16 and g2.dx == 1 / 128
    assert abs(q2d[0] - 1).max() <= 0.1 + 1e-3
    gs, qs = W.grid_sod()
    assert gs.n == 512 and gs.dx == 1 / 1024 and gs.bc[0] == "transmissive"
