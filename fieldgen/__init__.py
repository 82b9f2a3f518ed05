"""Seeded synthetic density fields shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the correlation method itself: it only draws
inputs.  The recipe stands in for the turbulent-ISM simulation cubes the paper
measures (Sec. 4, the CATS MHD run), which are not available here:

1. white noise w ~ N(0, 1) in float64 from numpy's PCG64 with the given seed;
2. g_hat = FFT(w) * sqrt(P(|k|)), k = 2*pi*fftfreq(N) per axis, P(0) = 0,
   P(k) = k**(-n_s);
3. g = Re IFFT(g_hat), shifted and scaled to zero mean and unit variance;
4. rho = exp(sigma * g) (lognormal);
5. delta = rho / mean(rho) - 1 (density contrast, Sec. 2.5);
6. the mean is subtracted again in float64 and the field is cast to the
   requested dtype.  The cast values are the canonical input: the oracle
   upcasts those same values to float64.
"""
from __future__ import annotations

import numpy as np

__all__ = ["lognormal_field", "gaussian_field", "c3_fields", "c4_batch", "c5_batch", "sparse_unit_field",
           "linear_edges"]


def linear_edges(rmax: float, nbins: int) -> np.ndarray:
    """Bin edges e_b = rmax * b / nbins, b = 0..nbins (linear bins over (0, rmax])."""
    return np.array([rmax * b / nbins for b in range(nbins + 1)], dtype=np.float64)


def _gaussian(shape, seed: int, spectral_index: float | None) -> np.ndarray:
    """Steps 1-3 of the recipe: the zero-mean, unit-variance Gaussian field (float64)."""
    shape = tuple(int(s) for s in shape)
    nd = len(shape)
    if spectral_index is None:
        spectral_index = 11.0 / 3.0 if nd == 3 else 8.0 / 3.0
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal(shape)
    ks = np.meshgrid(*[2.0 * np.pi * np.fft.fftfreq(n) for n in shape], indexing="ij")
    k2 = np.zeros(shape)
    for k in ks:
        k2 += k * k
    kmag = np.sqrt(k2)
    amp = np.zeros(shape)
    nz = kmag > 0
    amp[nz] = kmag[nz] ** (-0.5 * spectral_index)
    g = np.fft.ifftn(np.fft.fftn(w) * amp).real
    return (g - g.mean()) / g.std()


def gaussian_field(shape, seed: int, spectral_index: float | None = None, dtype=np.float32) -> np.ndarray:
    """Gaussian field with the power spectrum of lognormal_field (steps 1-3 only): the
    starting point of the synthesis demo."""
    return np.ascontiguousarray(_gaussian(shape, seed, spectral_index).astype(dtype))


def lognormal_field(shape, seed: int, sigma: float = 1.0, spectral_index: float | None = None,
                    dtype=np.float32) -> np.ndarray:
    """Lognormal density contrast on a periodic grid of the given shape.

    ``spectral_index`` n_s defaults to 11/3 in 3D and 8/3 in 2D (Kolmogorov-like
    slopes for a 3D cube and a 2D slice)."""
    g = _gaussian(shape, seed, spectral_index)
    rho = np.exp(sigma * g)
    delta = rho / rho.mean() - 1.0
    delta = delta - delta.mean()
    return np.ascontiguousarray(delta.astype(dtype))


def c3_fields(n: int = 256):
    """The two full-3PCF fields: sigma 0.5 (seed 0) and sigma 1.5 (seed 1)."""
    return [lognormal_field((n, n, n), seed=0, sigma=0.5),
            lognormal_field((n, n, n), seed=1, sigma=1.5)]


def c4_batch(n: int = 128, count: int = 16, base_seed: int = 0):
    """Batch of lognormal fields with sigma_i ~ U[0.5, 2] drawn from seed base_seed + 10**6."""
    aux = np.random.Generator(np.random.PCG64(base_seed + 10 ** 6))
    sigmas = aux.uniform(0.5, 2.0, size=count)
    return [lognormal_field((n, n, n), seed=base_seed + i, sigma=float(sigmas[i]))
            for i in range(count)], sigmas


def c5_shapes(count: int = 48, base_seed: int = 0, sizes=(64, 96, 128, 160, 192)):
    """Cubic grid edges drawn uniformly from ``sizes`` (seed base_seed + 10**6)."""
    aux = np.random.Generator(np.random.PCG64(base_seed + 10 ** 6))
    picks = aux.integers(0, len(sizes), size=count)
    return [int(sizes[p]) for p in picks]


def c5_batch(count: int = 48, base_seed: int = 0):
    """Uneven batch: field i is a sigma = 1 lognormal cube of edge c5_shapes()[i]."""
    edges = c5_shapes(count, base_seed)
    return [lognormal_field((n, n, n), seed=base_seed + i, sigma=1.0)
            for i, n in enumerate(edges)], edges


def sparse_unit_field(shape, count: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Empty grid with ``count`` randomly chosen cells set to weight one (the
    particle-on-grid inputs of the validation described in Sec. 2.5)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(np.prod(shape))
    idx = rng.choice(n, size=count, replace=False)
    f = np.zeros(n, dtype=dtype)
    f[idx] = 1.0
    return f.reshape(shape)
