"""Seeded velocity models, returned as squared slowness gamma = 1/c^2.

The paper's control is the squared slowness (Section 2, below the Helmholtz
equation with PML; gamma = c^-2).  Grids are [nz][nx] row-major with node
(i, j) at x = i*h, z = j*h; the listed grid includes the PML strips.
"""

import numpy as np
from scipy.ndimage import gaussian_filter


def gaussian_smooth(field, sigma_cells):
    """Gaussian-smoothed copy of a 2-D field (edge values repeated)."""
    return gaussian_filter(np.asarray(field, dtype=np.float64), sigma=sigma_cells,
                           mode="nearest")


def layered_model(nx, nz, npml, seed=0, velocities=(1500., 2000., 2500., 3000., 3500., 4000.),
                  min_gap_cells=2):
    """Flat layers, top to bottom, with seed-drawn interface rows inside the core.

    Returns the velocity c [nz][nx] in m/s.  Interfaces are rows drawn uniformly
    in the core (npml <= j < nz - npml), sorted and at least ``min_gap_cells``
    apart; layer l occupies rows at or below interface l-1 and above interface l.
    """
    rng = np.random.default_rng(seed)
    nlay = len(velocities)
    lo, hi = npml + 1, nz - npml - 1
    while True:
        rows = np.sort(rng.integers(lo, hi, size=nlay - 1))
        if np.all(np.diff(rows) >= min_gap_cells) and rows[0] - npml >= min_gap_cells:
            break
    c = np.empty((nz, nx))
    j = np.arange(nz)
    layer = np.searchsorted(rows, j, side="right")
    c[:, :] = np.asarray(velocities)[layer][:, None]
    return c


class FaultedLensModel:
    """A layered model with dipping normal faults and a Gaussian high-velocity lens.

    Defined in physical coordinates on [0, Lx] x [0, Lz] (metres) so that the
    same seeded earth can be sampled on any grid.  Layer velocities rise from
    1500 m/s at the top to about 4500 m/s; each fault drops the layering on its
    hanging-wall side by a throw; the lens peak is exactly ``v_lens``.
    """

    def __init__(self, seed=1, lx=4000.0, lz=1400.0, nlayers=8, v_top=1500.0,
                 v_bottom=4500.0, jitter=150.0, nfaults=3, v_lens=5500.0,
                 v_clip=(1500.0, 5500.0)):
        rng = np.random.default_rng(seed)
        self.lx, self.lz = lx, lz
        # interfaces between nlayers layers, inside the depth range below the
        # top absorbing strip and above the bottom one
        while True:
            depths = np.sort(rng.uniform(0.18 * lz, 0.82 * lz, size=nlayers - 1))
            if np.all(np.diff(depths) >= 0.03 * lz):
                break
        self.depths = depths
        v = v_top + (v_bottom - v_top) * np.arange(nlayers) / (nlayers - 1)
        v[1:] += rng.uniform(-jitter, jitter, size=nlayers - 1)
        self.vlayers = v
        faults = []
        for _ in range(nfaults):
            xf = rng.uniform(0.2, 0.8) * lx
            dip = np.deg2rad(rng.uniform(55.0, 75.0))
            side = 1.0 if rng.uniform() < 0.5 else -1.0
            throw = rng.uniform(50.0, 150.0)
            faults.append((xf, dip, side, throw))
        self.faults = faults
        self.lens_x = rng.uniform(0.35, 0.65) * lx
        self.lens_z = rng.uniform(0.5, 0.7) * lz
        self.lens_sx, self.lens_sz = 300.0, 150.0
        self.v_lens = v_lens
        self.v_clip = v_clip

    def _layers(self, x, z):
        zeff = np.array(z, dtype=np.float64, copy=True)
        for xf, dip, side, throw in self.faults:
            # fault trace at depth z; the hanging wall is the side the plane dips toward
            xtrace = xf + side * z / np.tan(dip)
            hanging = (x - xtrace) * side > 0.0
            zeff = np.where(hanging, zeff - throw, zeff)
        layer = np.searchsorted(self.depths, zeff, side="right")
        return self.vlayers[layer]

    def velocity(self, x, z):
        x = np.asarray(x, dtype=np.float64)
        z = np.asarray(z, dtype=np.float64)
        v = self._layers(x, z)
        v0 = self._layers(np.array(self.lens_x), np.array(self.lens_z))
        bump = np.exp(-0.5 * ((x - self.lens_x) / self.lens_sx) ** 2
                      - 0.5 * ((z - self.lens_z) / self.lens_sz) ** 2)
        v = v + (self.v_lens - v0) * bump
        return np.clip(v, *self.v_clip)


def faulted_lens_model(nx, nz, h, seed=1):
    """Velocity [nz][nx] of the seeded faulted-lens earth sampled at x=i*h, z=j*h."""
    m = FaultedLensModel(seed=seed)
    x = np.arange(nx) * h
    z = np.arange(nz) * h
    xx, zz = np.meshgrid(x, z)
    return m.velocity(xx, zz)


def model_pair(c_true, npml, sigma_cells):
    """(gamma_true, gamma_0) with the PML strips of gamma_true taken from gamma_0.

    gamma_0 is the Gaussian-smoothed squared slowness.  The control lives on the
    core only, so the PML values are frozen at gamma_0 in both models; copying
    them into gamma_true makes the observed data reachable from gamma_0.
    """
    g_true = 1.0 / np.asarray(c_true, dtype=np.float64) ** 2
    g0 = gaussian_smooth(g_true, sigma_cells)
    nz, nx = g_true.shape
    core = np.zeros_like(g_true, dtype=bool)
    core[npml:nz - npml, npml:nx - npml] = True
    g_true = np.where(core, g_true, g0)
    return np.ascontiguousarray(g_true), np.ascontiguousarray(g0)
