"""Angular quadrature rules (section 2.1).

A rule is returned as (ox, oy, w): direction components in the X-Y plane and
normalised weights with sum(w) == 1.  In 1D slab geometry oy is all zero.
"""
import numpy as np


def gauss_legendre_normalised(n):
    """n-point Gauss-Legendre rule on [-1, 1] with weights scaled to sum to 1
    (the normalised rule used for the z-component in section 2.1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w / 2.0


def slab_gl(n):
    """1D S_n: ordinates mu_j = GL nodes, weights w_j / 2 (App. A uses a
    symmetric rule {(+-v_j, w_j)})."""
    x, w = gauss_legendre_normalised(n)
    return x.copy(), np.zeros_like(x), w


def chebyshev_legendre(n_theta, n_z, folded=False):
    """CL(N_theta, N_z) product rule of section 2.1.

    theta_j1 = 2 j1 pi / N_theta - pi / N_theta with weight 1/N_theta, times
    the normalised N_z-point GL rule in Omega_z; ordinate index
    j = (j2 - 1) N_theta + j1 (j1 fastest).

    folded=True keeps only the nodes with Omega_z > 0 and doubles their
    weights.  In X-Y geometry the transport operator depends on (Omega_x,
    Omega_y) only, and the GL nodes come in +-Omega_z pairs with equal
    weights, so the folded rule gives the same discrete operator T.
    """
    j1 = np.arange(1, n_theta + 1)
    theta = 2.0 * j1 * np.pi / n_theta - np.pi / n_theta
    wth = np.full(n_theta, 1.0 / n_theta)
    oz, wz = gauss_legendre_normalised(n_z)
    if folded:
        keep = oz > 0
        oz, wz = oz[keep], 2.0 * wz[keep]
    ox, oy, w = [], [], []
    for j2 in range(len(oz)):
        s = np.sqrt(1.0 - oz[j2] ** 2)
        for a in range(n_theta):
            ox.append(np.cos(theta[a]) * s)
            oy.append(np.sin(theta[a]) * s)
            w.append(wth[a] * wz[j2])
    return np.array(ox), np.array(oy), np.array(w)


def make_rule(spec):
    if spec[0] == "gl":
        return slab_gl(spec[1])
    if spec[0] == "cl":
        return chebyshev_legendre(spec[1], spec[2], spec[3] if len(spec) > 3 else False)
    raise ValueError(spec)
