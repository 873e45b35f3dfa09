"""Pins of the oracle's PML, Helmholtz matrix and banded LU (CPU only).

Each test ties the oracle to something other than itself: a textbook matrix,
a closed-form solution, a continuous-model identity or an independent library
factorisation.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.integrate import quad
from scipy.special import hankel1

from oracle.helmholtz import assemble_A, BandedLU
from oracle.pml import sigma_profile, stretch


def laplacian_1d(n, h):
    """Textbook second-difference matrix with Dirichlet ends: (2, -1, -1)/h^2."""
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]) / h ** 2


def test_no_pml_is_textbook_laplacian_minus_mass():
    """Without PML the operator is -Laplacian - omega^2 diag(s) (Section 2, the no-PML case)."""
    nx, nz, h, omega = 13, 9, 7.0, 2 * np.pi * 3.0
    rng = np.random.default_rng(3)
    gamma = rng.uniform(1 / 4000 ** 2, 1 / 1500 ** 2, size=(nz, nx))
    A = assemble_A(nx, nz, h, 0, omega, gamma)
    lap = sp.kron(sp.identity(nz), laplacian_1d(nx, h)) + sp.kron(laplacian_1d(nz, h), sp.identity(nx))
    ref = lap - omega ** 2 * sp.diags(gamma.ravel())
    assert abs(A - ref).max() <= 1e-12 * abs(ref).max()


def test_pml_profile_gives_design_reflection():
    """The quadratic profile's normal-incidence continuous reflection exp(-2/c int sigma) equals R0."""
    n, h, npml, r0, c = 101, 10.0, 20, 1e-3, 3000.0
    width = npml * h
    integral, _ = quad(lambda x: sigma_profile(np.array([x]), n, h, npml, r0, c)[0], 0.0, width)
    assert np.exp(-2.0 * integral / c) == pytest.approx(r0, rel=1e-10)
    s = sigma_profile(np.arange(n) * h, n, h, npml, r0, c)
    assert np.all(s[npml:n - npml] == 0.0)
    assert np.all(np.diff(s[:npml + 1]) < 0) and np.all(np.diff(s[n - npml - 1:]) > 0)


def test_stretch_factor_is_one_in_core_and_damping_outside():
    n, h, npml, om = 41, 5.0, 8, 2 * np.pi * 4
    xn, xh = stretch(n, h, npml, om, 1e-3, 2000.0)
    assert np.all(xn[npml:n - npml] == 1.0)
    assert np.all(xn.real == 1.0) and np.all(xn.imag >= 0.0)
    assert xh.shape == (n + 1,) and np.all(xh[npml + 1:n - npml] == 1.0)


def test_pml_operator_is_complex_symmetric():
    """The conservative PML stencil gives A^T = A, hence A^* = conj(A)."""
    nx, nz = 23, 17
    rng = np.random.default_rng(5)
    gamma = rng.uniform(1 / 4000 ** 2, 1 / 1500 ** 2, size=(nz, nx))
    A = assemble_A(nx, nz, 10.0, 5, 2 * np.pi * 5, gamma, 1e-3, 4000.0)
    assert abs(A - A.T).max() == 0.0
    assert abs(A - A.conj().T).max() > 0.0          # complex, non-Hermitian with PML


@pytest.mark.parametrize("nx,nz", [(19, 11), (11, 19), (16, 16)])
def test_banded_lu_matches_splu_and_dense(nx, nz):
    rng = np.random.default_rng(nx * 100 + nz)
    gamma = rng.uniform(1 / 4000 ** 2, 1 / 1500 ** 2, size=(nz, nx))
    A = assemble_A(nx, nz, 15.0, 3, 2 * np.pi * 6, gamma, 1e-3, 4000.0)
    lu = BandedLU(A, nx, nz)
    b = rng.standard_normal((3, nz, nx)) + 1j * rng.standard_normal((3, nz, nx))
    x = lu.solve(b)
    xa = lu.solve(b, adjoint=True)
    Ad = A.toarray()
    for k in range(3):
        ref = np.linalg.solve(Ad, b[k].ravel())
        ref_a = np.linalg.solve(Ad.conj().T, b[k].ravel())
        ref_s = spla.splu(A.tocsc()).solve(b[k].ravel())
        assert np.linalg.norm(x[k].ravel() - ref) <= 1e-12 * np.linalg.norm(ref)
        assert np.linalg.norm(x[k].ravel() - ref_s) <= 1e-12 * np.linalg.norm(ref)
        assert np.linalg.norm(xa[k].ravel() - ref_a) <= 1e-12 * np.linalg.norm(ref_a)
        assert np.linalg.norm(A @ x[k].ravel() - b[k].ravel()) <= 1e-13 * np.linalg.norm(b[k])


def _green_error(ppw, v=2000.0, freq=5.0):
    """Relative L2 error of the discrete point-source field vs (i/4) H0^(1)(k r)
    on the annulus 5h <= r <= one wavelength, PML one wavelength wide."""
    lam = v / freq
    h = lam / ppw
    npml = int(round(ppw))
    half_core = int(np.ceil((lam + 10 * h) / h))
    n = 2 * (half_core + npml) + 1
    c = n // 2
    omega = 2 * np.pi * freq
    gamma = np.full((n, n), 1.0 / v ** 2)
    A = assemble_A(n, n, h, npml, omega, gamma, 1e-6, v)
    f = np.zeros((n, n), np.complex128)
    f[c, c] = 1.0 / h ** 2                       # unit discrete delta
    u = BandedLU(A, n, n).solve(f)
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    r = h * np.hypot(ii - c, jj - c)
    ring = (r >= 5 * h) & (r <= lam)
    k = omega / v
    exact = 0.25j * hankel1(0, k * r[ring])      # outgoing for the e^{-i w t} convention
    return np.linalg.norm(u[ring] - exact) / np.linalg.norm(exact)


def test_point_source_matches_hankel_green_function():
    """Constant velocity, PML: the field is the free-space Green's function (i/4) H0(kr)."""
    assert _green_error(60) <= 0.01


def test_second_order_convergence_to_green_function():
    e = [_green_error(p) for p in (15, 30, 60)]
    orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all((orders > 1.8) & (orders < 2.2)), (e, orders)
