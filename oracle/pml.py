"""Grid and PML stretch factors (oracle; test infrastructure only).

Section 2 writes the Helmholtz equation with complex one-dimensional factors
X(x), Z(z) that equal 1 in the core and deviate from 1 only inside the damping
strips (the PML figure).  The paper does not print the profile; this oracle
takes the common quadratic one:

    sigma(d) = sigma_max * (d / Lpml)^2,  sigma_max = 3 c_ref / (2 Lpml) * ln(1 / R0),
    X(x)     = 1 + i sigma(d(x)) / omega,

where d(x) is the distance from x into the strip and Lpml = npml * h.  Node i
sits at x = i*h; the core is npml <= i <= n-1-npml.
"""

import numpy as np


def sigma_profile(x, n, h, npml, r0, cref):
    """Damping sigma(x) at positions x (metres) for an axis of n nodes."""
    x = np.asarray(x, dtype=np.float64)
    if npml == 0:
        return np.zeros_like(x)
    width = npml * h
    sigma_max = 3.0 * cref / (2.0 * width) * np.log(1.0 / r0)
    x_left = npml * h
    x_right = (n - 1 - npml) * h
    d = np.maximum(np.maximum(x_left - x, x - x_right), 0.0)
    return sigma_max * (d / width) ** 2


def stretch(n, h, npml, omega, r0, cref):
    """(at_nodes[n], at_half_nodes[n+1]) of the factor 1 + i sigma / omega.

    at_half_nodes[i] is the value at position (i - 1/2) * h, i = 0..n, so the
    two faces of node i are at_half_nodes[i] (minus side) and
    at_half_nodes[i + 1] (plus side).
    """
    xn = np.arange(n) * h
    xh = (np.arange(n + 1) - 0.5) * h
    fn = 1.0 + 1j * sigma_profile(xn, n, h, npml, r0, cref) / omega
    fh = 1.0 + 1j * sigma_profile(xh, n, h, npml, r0, cref) / omega
    return fn, fh


def core_mask(nx, nz, npml):
    """Boolean [nz][nx] mask of the core (control) nodes."""
    m = np.zeros((nz, nx), dtype=bool)
    m[npml:nz - npml, npml:nx - npml] = True
    return m
