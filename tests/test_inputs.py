"""The seeded input generators: reproducible, and with the shapes and
statistics the workloads ask for."""
import numpy as np

from paper_2111_08666_amd import inputs as I


def test_disc_medium_is_seeded_and_hits_porosity():
    a = I.disc_medium(128, 64, 3.0, 8.0, 0.6, seed=1)
    b = I.disc_medium(128, 64, 3.0, 8.0, 0.6, seed=1)
    assert np.array_equal(a, b)
    assert a.shape == (64, 128) and a.dtype == np.uint8
    assert a[0].all() and a[-1].all()
    win = a[1:-1, 8:120]
    assert abs((1 - win.mean()) - 0.6) < 0.02
    assert not a[1:-1, :8].any() and not a[1:-1, -8:].any()  # clear reservoirs


def test_sphere_medium_porosity_and_walls():
    m = I.sphere_medium(48, 32, 32, 3.0, 6.0, 0.4, seed=5)
    assert m.shape == (32, 32, 48)
    assert m[:, 0].all() and m[:, -1].all() and m[0].all() and m[-1].all()
    win = m[1:-1, 1:-1, 8:40]
    assert abs((1 - win.mean()) - 0.4) < 0.02
    assert not m[1:-1, 1:-1, :8].any()


def test_reservoir_front_and_droplet():
    m = np.zeros((4, 10), np.uint8)
    m[0] = 1
    r = I.reservoir_front(m, 3, 1.0, 0.01)
    assert r[0, 1, 2] == 1.0 and r[1, 1, 2] == 0.01 and r[0, 1, 3] == 0.01
    assert (r[:, 0] == 0).all()
    d = I.tanh_droplet((41, 41), (20, 20), 10.0, rho_in=(1.0, 0.02), rho_out=(0.02, 1.0))
    assert abs(d[0, 20, 20] - 1.0) < 1e-3 and abs(d[0, 0, 0] - 0.02) < 1e-6
    assert abs(d[0, 20, 30] - 0.51) < 1e-12  # on the circle: the mean of in and out


def test_batch_instances_are_uneven_and_in_range():
    b = I.batch_instances(8, nx_range=(256, 512))
    sizes = {p.nx for p in b}
    assert len(sizes) > 1 and all(p.nx % 64 == 0 and p.ny == p.nx // 2 for p in b)
    for p in b:
        assert 30 <= p.theta <= 150 and 1e-4 <= p.dp <= 5e-3


def test_close_narrow_throats():
    """One-node passages along x or y are filled until none is left; wider
    passages stay open, and no fluid node is left between two solid ones."""
    m = np.zeros((9, 12), np.uint8)
    m[1, :] = 1
    m[3, :] = 1          # row 2: a one-node channel along x
    m[7, :] = 1          # rows 4-6: a three-node channel
    m[4:7, 8] = 1
    m[4:7, 10] = 1       # column 9 of rows 4-6: a one-node channel along y
    out = I.close_narrow_throats(m)
    assert np.all(out >= m)
    assert out[2].all() and out[4:7, 9].all()
    assert not out[4:7, :8].any() and not out[0].any() and not out[8].any()
    pad = np.pad(out.astype(bool), 1)
    fluid = ~out.astype(bool)
    assert not np.any(fluid & ((pad[1:-1, :-2] & pad[1:-1, 2:]) | (pad[:-2, 1:-1] & pad[2:, 1:-1])))
    assert np.array_equal(I.close_narrow_throats(out), out)
    p = I.large_drainage()
    closed = I.close_narrow_throats(p.mask)
    assert np.all(closed >= p.mask) and 0 < int(closed.sum() - p.mask.sum()) < 0.01 * p.n_fluid
