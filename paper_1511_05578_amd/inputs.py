"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

Holds none of the transform's arithmetic: it only draws random harmonic
coefficients in a fixed order so that every consumer sees the same numbers.

Harmonic arrays are flat complex128 of length L^2 with index l^2 + l + m.
"""
import numpy as np


def gaussian_real_flm(L, seed=0):
    """Coefficients of a real band-limited map with power ~ (l+1)^-2.

    For each l = 0..L-1 and m = 0..l, in that order: m = 0 draws one value
    f_l0 ~ N(0, (l+1)^-2); m > 0 draws Re then Im, each ~ N(0, (l+1)^-2 / 2).
    Negative m follow the reality condition f_{l,-m} = (-1)^m conj(f_lm).
    Draws come from ``numpy.random.default_rng(seed).standard_normal``.
    """
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(L * L)
    out = np.zeros(L * L, dtype=np.complex128)
    k = 0
    for l in range(L):
        sd = 1.0 / (l + 1)
        base = l * l + l
        out[base] = sd * z[k]
        k += 1
        if l == 0:
            continue
        re = z[k:k + 2 * l:2] * (sd / np.sqrt(2.0))
        im = z[k + 1:k + 2 * l:2] * (sd / np.sqrt(2.0))
        k += 2 * l
        ms = np.arange(1, l + 1)
        vals = re + 1j * im
        out[base + ms] = vals
        out[base - ms] = ((-1.0) ** ms) * np.conj(vals)
    return out


def uniform_complex_flm(L, seed=0):
    """Coefficients of a complex map: Re and Im of every f_lm ~ U[-1, 1]
    (the random test signals of the paper's accuracy experiment)."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1.0, 1.0, size=(L * L, 2))
    return v[:, 0] + 1j * v[:, 1]


def serving_trace(n_requests=1024, bandlimits=(64, 128, 256, 512), rate_hz=100.0,
                  seed_arrivals=1, seed_sizes=2):
    """Arrival times (s, Poisson process of the given rate) and band-limits
    (uniform over ``bandlimits``) of a request trace."""
    ra = np.random.default_rng(seed_arrivals)
    rs = np.random.default_rng(seed_sizes)
    gaps = ra.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    Ls = rs.choice(np.asarray(bandlimits), size=n_requests)
    return t, Ls


def point_sources(n=64, seed=1):
    """n point sources uniform on the sphere with relative amplitudes.

    Draws cos(theta) ~ U[-1, 1], phi ~ U[0, 2 pi) and a relative amplitude
    a ~ U[1, 10] per source from ``numpy.random.default_rng(seed)`` (all
    cos(theta), then all phi, then all a).  Returns (theta, phi, a)."""
    rng = np.random.default_rng(seed)
    ct = rng.uniform(-1.0, 1.0, size=n)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=n)
    amp = rng.uniform(1.0, 10.0, size=n)
    return np.arccos(ct), ph, amp


def source_amplitudes(a, field_flm, L):
    """Harmonic amplitudes A_k of band-limited point sources whose peaks are
    a_k times the rms of the field with coefficients ``field_flm``.

    A source A conj(Y_lm(omega_k)) (l < L) peaks at omega_k with height
    A L^2 / (4 pi) (the sum over l < L and |m| <= l of |Y_lm|^2), and the rms
    of a field over the sphere is sqrt(sum |f_lm|^2 / (4 pi)) (Parseval), so
    A_k = a_k rms 4 pi / L^2.  The coefficients themselves,
    sum_k A_k conj(Y_lm(omega_k)), are formed by each consumer."""
    rms = float(np.sqrt(np.sum(np.abs(field_flm) ** 2) / (4.0 * np.pi)))
    return np.asarray(a, dtype=np.float64) * rms * 4.0 * np.pi / (L * L)
