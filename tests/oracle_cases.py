"""Small seeded problems shared by the oracle pins and the GPU parity tests."""

import numpy as np

from synthetic import layered_model, model_pair, geometry


def tiny_inputs(nx=21, nz=15, npml=4, K=3, nrec=None, h=25.0, freq=6.0, seed=0,
                eps=None, sigma=2.0, weights="ones"):
    """A small layered problem: gamma_true / gamma0 and top-row acquisition.

    ``nrec`` limits the receivers to evenly spaced columns; ``weights`` is
    "ones" or "random" (seeded positive weights)."""
    c = layered_model(nx, nz, npml, seed=seed,
                      velocities=(1500., 2200., 2900., 3600.), min_gap_cells=1)
    g_true, g0 = model_pair(c, npml, sigma)
    src_ix, src_iz, rec_ix, rec_iz = geometry(nx, nz, npml, K)
    if nrec is not None:
        sel = np.linspace(0, nx - 1, nrec).round().astype(np.int32)
        rec_ix, rec_iz = rec_ix[sel], rec_iz[sel]
    rng = np.random.default_rng(seed + 17)
    if weights == "ones":
        w = np.ones((K, len(rec_ix)))
    else:
        w = rng.uniform(0.5, 2.0, size=(K, len(rec_ix)))
    return dict(nx=nx, nz=nz, h=h, npml=npml, freq=freq, omega=2 * np.pi * freq,
                gamma_true=g_true, gamma0=g0, src_ix=src_ix, src_iz=src_iz,
                rec_ix=rec_ix.astype(np.int32), rec_iz=rec_iz.astype(np.int32), w=w, K=K,
                eps=eps, pml_r0=1e-3, pml_cref=3600.0)
