"""Workload configurations and the acquisition geometry.

Five workloads are shaped like the paper's experiments (Section 6: one
Gauss-Newton step, then a sweep over frequencies) on seeded synthetic earth
models:

* ``c0``  101x51 nodes, h=20 m, 10-cell PML, 6 flat layers, 8 sources, 5 Hz, FP64.
* ``c1``  401x141, h=10 m, 20-cell PML, faulted lens model, 40 sources, 3/5/7 Hz.
* ``c2``  801x281, h=5 m, 40-cell PML, same earth, 80 sources, 5 Hz (mixed precision).
* ``c3``  gradient check on the c0 setup; timed on the c2 setup.
* ``c4``  2/4/6/8/10 Hz on five grids (201x71 ... 1001x351), 100 sources each.

Sources and receivers sit on the first core row (j = npml).  Receivers cover
every column of that row; sources are spread evenly over the core columns.
The regularisation weight eps of each (config, frequency) is a literal read
from ``eps_table.json``, which a script next to the oracle writes.
"""

import json
import os

import numpy as np

from .models import layered_model, faulted_lens_model, model_pair

_HERE = os.path.dirname(os.path.abspath(__file__))
EPS_TABLE_PATH = os.path.join(_HERE, "eps_table.json")

CONFIGS = {
    "c0": dict(grids=[(101, 51, 20.0, 10)], freqs=[5.0], K=8, model="layered", seed=0,
               sigma_cells=5.0, pml_r0=1e-3, pml_cref=4000.0, tol=1e-8),
    "c1": dict(grids=[(401, 141, 10.0, 20)], freqs=[3.0, 5.0, 7.0], K=40, model="faulted",
               seed=1, sigma_cells=15.0, pml_r0=1e-3, pml_cref=5500.0, tol=1e-6,
               newton_steps=5),
    "c2": dict(grids=[(801, 281, 5.0, 40)], freqs=[5.0], K=80, model="faulted", seed=1,
               sigma_cells=30.0, pml_r0=1e-3, pml_cref=5500.0, tol=1e-6),
    "c4": dict(grids=[(201, 71, 20.0, 20), (401, 141, 10.0, 20), (601, 211, 20.0 / 3.0, 20),
                      (801, 281, 5.0, 20), (1001, 351, 4.0, 20)],
               freqs=[2.0, 4.0, 6.0, 8.0, 10.0], K=100, model="faulted", seed=1,
               # same physical smoothing length (150 m) on every grid
               sigma_m=150.0, pml_r0=1e-3, pml_cref=5500.0, tol=1e-6),
}
CONFIGS["c3"] = dict(CONFIGS["c0"])


def get_config(name):
    return CONFIGS[name]


def geometry(nx, nz, npml, K):
    """Source and receiver node indices on the first core row.

    Source k sits at column npml + floor((k + 1/2) * ncore_x / K); receivers are
    all nx columns.  Returns (src_ix, src_iz, rec_ix, rec_iz) as int32 arrays.
    """
    ncx = nx - 2 * npml
    k = np.arange(K)
    src_ix = (npml + np.floor((k + 0.5) * ncx / K)).astype(np.int32)
    src_iz = np.full(K, npml, dtype=np.int32)
    rec_ix = np.arange(nx, dtype=np.int32)
    rec_iz = np.full(nx, npml, dtype=np.int32)
    return src_ix, src_iz, rec_ix, rec_iz


def load_eps(name, freq, grid_index=0):
    if not os.path.exists(EPS_TABLE_PATH):
        return None
    with open(EPS_TABLE_PATH) as fh:
        tab = json.load(fh)
    return tab.get(f"{name}/g{grid_index}/{freq:g}")


def make_problem_inputs(name, freq_index=0, grid_index=None, K=None):
    """All inputs of one (config, frequency) problem as plain numpy arrays.

    Keys: nx, nz, h, npml, freq, omega, gamma_true, gamma0, src_ix, src_iz,
    rec_ix, rec_iz, w, eps, pml_r0, pml_cref.  ``w`` is the [K][nrec] weight
    array (identity weights).  ``eps`` is None when the table has no entry.
    """
    cfg = CONFIGS[name]
    if grid_index is None:
        grid_index = freq_index if len(cfg["grids"]) > 1 else 0
    nx, nz, h, npml = cfg["grids"][grid_index]
    K = cfg["K"] if K is None else K
    if cfg["model"] == "layered":
        c = layered_model(nx, nz, npml, seed=cfg["seed"])
        sigma = cfg["sigma_cells"]
    else:
        c = faulted_lens_model(nx, nz, h, seed=cfg["seed"])
        sigma = cfg["sigma_cells"] if "sigma_cells" in cfg else cfg["sigma_m"] / h
    g_true, g0 = model_pair(c, npml, sigma)
    src_ix, src_iz, rec_ix, rec_iz = geometry(nx, nz, npml, K)
    freq = cfg["freqs"][freq_index]
    return dict(name=name, nx=nx, nz=nz, h=h, npml=npml, freq=freq, omega=2.0 * np.pi * freq,
                gamma_true=g_true, gamma0=g0, src_ix=src_ix, src_iz=src_iz,
                rec_ix=rec_ix, rec_iz=rec_iz, w=np.ones((K, nx)), K=K,
                eps=load_eps(name, freq, grid_index), pml_r0=cfg["pml_r0"],
                pml_cref=cfg["pml_cref"], tol=cfg["tol"])
