"""Seeded input generators: deterministic and shaped as documented."""
import numpy as np

from paper_1511_05578_amd import inputs


def test_point_sources_distinct_and_seeded():
    t, p, a = inputs.point_sources(64, 64, seed=3)
    assert len(set(zip(t.tolist(), p.tolist()))) == 64
    assert t.min() >= 0 and t.max() < 64 and p.min() >= 0 and p.max() < 127
    assert np.all((a >= 0.5) & (a <= 1.5))
    t2, p2, a2 = inputs.point_sources(64, 64, seed=3)
    assert np.array_equal(t, t2) and np.array_equal(p, p2) and np.array_equal(a, a2)


def test_add_point_sources():
    m = np.zeros((8, 15))
    src = inputs.point_sources(8, 5, seed=1)
    inputs.add_point_sources(m, src)
    assert np.count_nonzero(m) == 5
    assert np.isclose(m.sum(), src[2].sum())


def test_gaussian_flm_reality_and_variance():
    L = 64
    f = inputs.gaussian_real_flm(L, seed=0)
    for l in (3, 40):
        for m in range(1, l + 1):
            assert f[l * l + l - m] == (-1) ** m * np.conj(f[l * l + l + m])
    # empirical power per l close to (l+1)^-2 (2l+1 samples; loose)
    pw = np.array([np.mean(np.abs(f[l * l:(l + 1) * (l + 1)]) ** 2) * (l + 1) ** 2 for l in range(8, L)])
    assert 0.7 < pw.mean() < 1.3
