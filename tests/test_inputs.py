"""Seeded input generators: deterministic and shaped as documented."""
import numpy as np

from paper_1511_05578_amd import inputs


def test_point_sources_seeded_and_uniform_on_sphere():
    th, ph, a = inputs.point_sources(4000, seed=3)
    assert np.all((th >= 0) & (th <= np.pi)) and np.all((ph >= 0) & (ph < 2 * np.pi))
    assert np.all((a >= 1.0) & (a <= 10.0))
    th2, ph2, a2 = inputs.point_sources(4000, seed=3)
    assert np.array_equal(th, th2) and np.array_equal(ph, ph2) and np.array_equal(a, a2)
    # uniform on the sphere: about half the sources in the polar caps |cos theta| > 1/2
    assert 0.45 < np.mean(np.abs(np.cos(th)) > 0.5) < 0.55


def test_source_amplitudes():
    # a field with only f_00 = c is the constant c Y_00 = c / sqrt(4 pi): its rms
    L = 16
    f = np.zeros(L * L, dtype=np.complex128)
    f[0] = 3.0
    A = inputs.source_amplitudes(np.array([1.0, 2.0]), f, L)
    rms = 3.0 / np.sqrt(4 * np.pi)
    assert np.allclose(A, np.array([1.0, 2.0]) * rms * 4 * np.pi / L ** 2, rtol=1e-15)


def test_gaussian_flm_reality_and_variance():
    L = 64
    f = inputs.gaussian_real_flm(L, seed=0)
    for l in (3, 40):
        for m in range(1, l + 1):
            assert f[l * l + l - m] == (-1) ** m * np.conj(f[l * l + l + m])
    # empirical power per l close to (l+1)^-2 (2l+1 samples; loose)
    pw = np.array([np.mean(np.abs(f[l * l:(l + 1) * (l + 1)]) ** 2) * (l + 1) ** 2 for l in range(8, L)])
    assert 0.7 < pw.mean() < 1.3
