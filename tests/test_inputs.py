"""Seeded input generators: deterministic and shaped as documented."""
import numpy as np

from paper_1511_05578_amd import inputs


def test_point_sources_seeded_and_uniform_on_sphere():
    L = 64
    t, p, a = inputs.point_sources(L, 4000, seed=3)
    assert t.min() >= 0 and t.max() < L and p.min() >= 0 and p.max() < 2 * L - 1
    assert np.all((a >= 1.0) & (a <= 10.0))
    t2, p2, a2 = inputs.point_sources(L, 4000, seed=3)
    assert np.array_equal(t, t2) and np.array_equal(p, p2) and np.array_equal(a, a2)
    # uniform on the sphere: about half the sources in the polar caps |cos theta| > 1/2
    ct = np.cos(np.pi * (2 * t + 1) / (2 * L - 1))
    assert 0.45 < np.mean(np.abs(ct) > 0.5) < 0.55


def test_add_point_sources():
    m = np.ones((8, 15))
    src = (np.array([0, 3, 3]), np.array([1, 2, 2]), np.array([2.0, 3.0, 4.0]))
    inputs.add_point_sources(m, src)
    assert m[0, 1] == 3.0 and m[3, 2] == 8.0
    assert np.isclose(m.sum(), 120 + 9.0)


def test_gaussian_flm_reality_and_variance():
    L = 64
    f = inputs.gaussian_real_flm(L, seed=0)
    for l in (3, 40):
        for m in range(1, l + 1):
            assert f[l * l + l - m] == (-1) ** m * np.conj(f[l * l + l + m])
    # empirical power per l close to (l+1)^-2 (2l+1 samples; loose)
    pw = np.array([np.mean(np.abs(f[l * l:(l + 1) * (l + 1)]) ** 2) * (l + 1) ** 2 for l in range(8, L)])
    assert 0.7 < pw.mean() < 1.3
