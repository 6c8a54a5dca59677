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


def point_sources(L, n=64, seed=1):
    """n point sources uniform on the sphere, snapped to MW samples of band-limit L.

    Draws cos(theta) ~ U[-1, 1], phi ~ U[0, 2 pi) and a relative amplitude
    a ~ U[1, 10] per source from ``numpy.random.default_rng(seed)`` (all
    cos(theta), then all phi, then all a).  Returns (t, p, a): the nearest MW
    sample indices (theta_t = pi(2t+1)/(2L-1), phi_p = 2 pi p/(2L-1)) and a."""
    rng = np.random.default_rng(seed)
    ct = rng.uniform(-1.0, 1.0, size=n)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=n)
    amp = rng.uniform(1.0, 10.0, size=n)
    theta = np.arccos(ct)
    t = np.clip(np.rint((theta * (2 * L - 1) / np.pi - 1.0) / 2.0), 0, L - 1).astype(np.int64)
    p = np.rint(ph * (2 * L - 1) / (2.0 * np.pi)).astype(np.int64) % (2 * L - 1)
    return t, p, amp


def add_point_sources(fmap, sources):
    """fmap (L x (2L-1) samples, modified in place) plus, at each source's
    sample, a spike of height a * rms(fmap) (rms of the samples before any
    source is added); returns fmap.  The result is not band-limited: consumers
    project it onto band-limit L with their own SHT pair."""
    t, p, amp = sources
    rms = float(np.sqrt(np.mean(fmap * fmap)))
    np.add.at(fmap, (t, p), amp * rms)
    return fmap
