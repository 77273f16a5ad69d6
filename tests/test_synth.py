"""Statistics and layout of the seeded input generators."""
import numpy as np

import synth


def test_lognormal_field_statistics():
    N, ell = 256, 1.0 / 32.0
    a = synth.lognormal_coefficient(N, ell, 1).reshape(N, N)
    g = np.log(a)
    assert abs(g.mean()) < 0.15
    assert abs(g.var() - 1.0) < 0.2
    lag = int(round(ell * N))
    c = np.mean((g[:, :-lag] - g.mean()) * (g[:, lag:] - g.mean())) / g.var()
    assert abs(c - np.exp(-1.0)) < 0.1


def test_periodic_coefficient_range():
    a = synth.periodic_coefficient(128)
    assert a.min() > 0.1 - 1e-12 and a.max() < 2.1 + 1e-12


def test_boundary_data_layout_and_continuity():
    N = 32
    b = synth.global_boundary_nodes(N)
    assert len({tuple(x) for x in b}) == 4 * N
    f = synth.fourier_boundary(N, [0, 1, 2])
    assert f.shape == (3, 4 * N)
    # consecutive boundary nodes (including the wrap-around) differ by a bounded step
    step = np.abs(np.diff(np.concatenate([f, f[:, :1]], axis=1), axis=1)).max()
    assert step < 0.5
    assert np.array_equal(f[1], synth.fourier_boundary(N, [1])[0])


def test_overlap_draw_is_seeded_coin():
    d = synth.overlap_draw(16, (16, 32), 3)
    assert set(np.unique(d)) <= {16, 32} and 60 < (d == 16).sum() < 196
    assert np.array_equal(d, synth.overlap_draw(16, (16, 32), 3))
