"""Seeded synthetic permeability fields.

Two families stand in for the fields the paper runs on (a Gaussian field of
its own, SPE10 layers), which are not available here:

* ``lognormal_grf``: ln K = sigma * xi with xi a stationary, zero-mean,
  unit-variance Gaussian field with exponential covariance exp(-r / ell),
  sampled exactly on the cell centres by circulant embedding (Dietrich and
  Newsam, 1997) on a doubled periodic grid.
* ``channelized_field``: a binary matrix/channel field made of sinusoidal
  bands, the high-contrast channelized structure of the paper's section 5.3
  and 5.5 examples.

Cell (i, j), i along x, is stored at ``j * nx + i`` in the returned flat
arrays.
"""
from __future__ import annotations

import numpy as np


def lognormal_grf(nx: int, ny: int, lx: float, ly: float, variance: float,
                  corr_len: float, seed: int, return_info: bool = False):
    """Log-normal permeability K = exp(sqrt(variance) * xi).

    xi is sampled with covariance C(r) = exp(-r / corr_len), r the Euclidean
    distance between cell centres, through circulant embedding on a
    2nx x 2ny periodic grid.  Negative embedding eigenvalues (none are
    expected for corr_len well below the domain size) are clipped to zero and
    their count and total mass are reported when ``return_info`` is set.
    """
    hx, hy = lx / nx, ly / ny
    mx, my = 2 * nx, 2 * ny
    ix = np.arange(mx)
    iy = np.arange(my)
    dx = np.minimum(ix, mx - ix) * hx
    dy = np.minimum(iy, my - iy) * hy
    r = np.sqrt(dx[None, :] ** 2 + dy[:, None] ** 2)
    c = np.exp(-r / corr_len)
    lam = np.fft.fft2(c).real
    neg = lam < 0
    info = {"clipped": int(neg.sum()), "clipped_mass": float(-lam[neg].sum()),
            "total_mass": float(np.abs(lam).sum())}
    lam = np.where(neg, 0.0, lam)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = mx * my
    eps = rng.standard_normal((my, mx)) + 1j * rng.standard_normal((my, mx))
    y = np.fft.fft2(np.sqrt(lam / n) * eps)
    xi = y.real[:ny, :nx]
    perm = np.exp(np.sqrt(variance) * xi).reshape(-1).astype(np.float64)
    if return_info:
        return perm, info
    return perm


def channelized_field(nx: int, ny: int, lx: float, ly: float, k_matrix: float,
                      k_channel: float, seed: int, min_fraction: float = 0.30,
                      width_cells=(4, 8)):
    """Binary channelized field: sinusoidal channels in a uniform matrix.

    Each channel is the band |y - y_c(x)| <= w*hy/2 around
    y_c(x) = y0 + A sin(2 pi x / wavelength + phase), with y0 ~ U(0, ly),
    A ~ U(0.05, 0.15) ly, wavelength ~ U(0.3, 1) lx, phase ~ U(0, 2 pi) and
    width w ~ U{4..8} cells.  Channels are added until at least
    ``min_fraction`` of the cells are channel cells.
    """
    hx, hy = lx / nx, ly / ny
    xc = (np.arange(nx) + 0.5) * hx
    yc = (np.arange(ny) + 0.5) * hy
    X, Y = np.meshgrid(xc, yc)
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = np.zeros((ny, nx), dtype=bool)
    n_channels = 0
    while mask.mean() < min_fraction:
        y0 = rng.uniform(0.0, ly)
        amp = rng.uniform(0.05, 0.15) * ly
        wavelength = rng.uniform(0.3, 1.0) * lx
        phase = rng.uniform(0.0, 2.0 * np.pi)
        w = int(rng.integers(width_cells[0], width_cells[1] + 1))
        ycen = y0 + amp * np.sin(2.0 * np.pi * X / wavelength + phase)
        mask |= np.abs(Y - ycen) <= 0.5 * w * hy
        n_channels += 1
        if n_channels > 10000:  # pragma: no cover - defensive
            raise RuntimeError("channel generator did not reach the target fraction")
    perm = np.where(mask, k_channel, k_matrix).reshape(-1).astype(np.float64)
    return perm
