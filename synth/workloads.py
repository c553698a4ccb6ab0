"""Seeded synthetic workloads shaped like the paper's test problems.

This module is shared by the CPU oracle, the tests and the benchmark.  It only
*describes* problems (grids, region maps, per-region cross sections, parameter
draws) and synthesises the source input; it holds none of the solver's
arithmetic (no transport operator, no sweep, no Krylov, no ROM).

A problem is a plain dict:

  dim            1 (slab) or 2 (X-Y)
  nx, ny         cells per direction (ny == 1 in 1D)
  box            (x0, x1, y0, y1)   (y0, y1 unused in 1D)
  quad           ('gl', n)                    1D Gauss-Legendre S_n
                 ('cl', n_theta, n_z, folded) Chebyshev-Legendre product rule
  region         int32 [ncell]  region id of each cell, cell = k*nx + i
  sigma_t        float64 [R]    total cross section per region
  sigma_s        float64 [R]    scattering cross section per region
  source         float64 [ncell*nloc] DG moments of the isotropic source
  inflow         float          isotropic constant inflow value g
  mu             float64 [d]    the parameter the problem was made from

DG moment convention (the library's layout): dof = cell*nloc + p + 2*q, with
the per-cell orthonormal tensor Legendre basis e_p(x) e_q(y),
e_0 = 1/sqrt(h), e_1 = sqrt(3) s / sqrt(h), s in [-1, 1] the local coordinate.
The source moments are the L2 projection of G computed with a 4x4 (4 in 1D)
Gauss-Legendre rule per cell; that rule is part of the workload definition.
"""
import numpy as np

__all__ = [
    "source_moments", "cfg1", "cfg2", "cfg3_mu", "cfg3_problem", "cfg3_train_test",
    "cfg4_batch", "tiny_2d", "tiny_1d", "CFG3_BOX_LO", "CFG3_BOX_HI", "cfg3_box_centre",
    "cfg3_sigma", "cfg3_sources", "cfg3_features", "cfg5_sets", "pincell_problem", "pincell_sets",
    "twomat_problem", "twomat_sets", "varscat_shape", "varscat_problem", "varscat_sets",
    "field_point_values", "FIELD_NQ", "with_field_values",
]

_GL4_X, _GL4_W = np.polynomial.legendre.leggauss(4)


def source_moments(func, dim, nx, ny, box):
    """DG moments of func(x, y) on the uniform grid (4-point rule per axis)."""
    x0, x1, y0, y1 = box
    hx = (x1 - x0) / nx
    if dim == 1:
        xc = x0 + (np.arange(nx) + 0.5) * hx
        X = xc[:, None] + 0.5 * hx * _GL4_X[None, :]
        F = func(X, np.zeros_like(X))
        w = 0.5 * hx * _GL4_W
        m0 = (F * w).sum(1) / np.sqrt(hx)
        m1 = (F * w * np.sqrt(3.0) * _GL4_X).sum(1) / np.sqrt(hx)
        return np.stack([m0, m1], 1).reshape(-1)
    hy = (y1 - y0) / ny
    xc = x0 + (np.arange(nx) + 0.5) * hx
    yc = y0 + (np.arange(ny) + 0.5) * hy
    # points [ky, ix, gy, gx]
    X = xc[None, :, None, None] + 0.5 * hx * _GL4_X[None, None, None, :]
    Y = yc[:, None, None, None] + 0.5 * hy * _GL4_X[None, None, :, None]
    X, Y = np.broadcast_arrays(X, Y)
    F = func(X, Y)
    wx = 0.5 * hx * _GL4_W
    wy = 0.5 * hy * _GL4_W
    W = wy[:, None] * wx[None, :]
    bx = [np.ones(4), np.sqrt(3.0) * _GL4_X]
    out = np.empty((ny, nx, 4))
    for q in range(2):
        for p in range(2):
            B = bx[q][:, None] * bx[p][None, :]
            out[:, :, p + 2 * q] = (F * (W * B)[None, None]).sum((2, 3)) / np.sqrt(hx * hy)
    return out.reshape(-1)


def _block_regions(nx, ny, nbx, nby):
    """Region id of each cell for an nbx x nby block layout (region = by*nbx + bx)."""
    i = np.arange(nx)
    k = np.arange(ny)
    bx = (i * nbx) // nx
    by = (k * nby) // ny
    return (by[:, None] * nbx + bx[None, :]).reshape(-1).astype(np.int32)


def cfg1(seed=1, nx=128, n_ord=16):
    """1D slab [0,1], P1 DG, S16 GL; sigma_s = mu1 on [0,.5), mu2 on [.5,1];
    sigma_a = 0.1, G = 1, zero inflow.  mu1, mu2 ~ U[1, 100]."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(1.0, 100.0, size=2)
    region = (np.arange(nx) * 2 // nx).astype(np.int32)
    sig_a = 0.1
    sigma_s = mu.copy()
    sigma_t = sigma_s + sig_a
    box = (0.0, 1.0, 0.0, 1.0)
    G = source_moments(lambda x, y: np.ones_like(x), 1, nx, 1, box)
    return dict(dim=1, nx=nx, ny=1, box=box, quad=("gl", n_ord), region=region,
                sigma_t=sigma_t, sigma_s=sigma_s, source=G, inflow=0.0, mu=mu)


def cfg2(seed=2, n=64, n_theta=16, n_z=16, width=0.1):
    """2D [0,1]^2, Q1 DG, CL(16,16) folded (128 ordinates); 4x4 blocks with
    sigma_s ~ 10^U[-1,2], sigma_a ~ U[0,1]; Gaussian source of width 0.1 at
    the centre; zero inflow."""
    rng = np.random.default_rng(seed)
    sig_s = 10.0 ** rng.uniform(-1.0, 2.0, size=16)
    sig_a = rng.uniform(0.0, 1.0, size=16)
    box = (0.0, 1.0, 0.0, 1.0)
    G = source_moments(lambda x, y: np.exp(-((x - 0.5) ** 2 + (y - 0.5) ** 2) / width ** 2),
                       2, n, n, box)
    return dict(dim=2, nx=n, ny=n, box=box, quad=("cl", n_theta, n_z, True),
                region=_block_regions(n, n, 4, 4), sigma_t=sig_s + sig_a, sigma_s=sig_s,
                source=G, inflow=0.0, mu=np.concatenate([sig_s, sig_a]))


# ---- parametric checkerboard family (configs 3, 4, 5) -------------------------------
# mu = (mu1, mu2, mu3, mu4): scattering levels of the two checkerboard colours
# (log10 mu1, log10 mu2 ~ U[0, 2]), absorption (U[0, 1]) and source width
# (U[0.05, 0.2]).  The box used for normalisation is in (log10 mu1, log10 mu2,
# mu3, mu4) coordinates.
CFG3_BOX_LO = np.array([0.0, 0.0, 0.0, 0.05])
CFG3_BOX_HI = np.array([2.0, 2.0, 1.0, 0.20])


def cfg3_mu(rng, n):
    u = rng.uniform(size=(n, 4))
    z = CFG3_BOX_LO + u * (CFG3_BOX_HI - CFG3_BOX_LO)
    return np.stack([10.0 ** z[:, 0], 10.0 ** z[:, 1], z[:, 2], z[:, 3]], 1)


def cfg3_box_centre():
    z = 0.5 * (CFG3_BOX_LO + CFG3_BOX_HI)
    return np.array([10.0 ** z[0], 10.0 ** z[1], z[2], z[3]])


def cfg3_problem(mu, n=96, n_theta=16, n_z=16):
    """Checkerboard of 4x4 blocks: colour A (bx+by even) scatters with mu1,
    colour B with mu2; sigma_a = mu3 everywhere; G = exp(-|x-c|^2/mu4^2)."""
    mu = np.asarray(mu, dtype=np.float64)
    blocks = _block_regions(n, n, 4, 4)
    bx = blocks % 4
    by = blocks // 4
    region = ((bx + by) % 2).astype(np.int32)
    sigma_s = np.array([mu[0], mu[1]])
    sigma_t = sigma_s + mu[2]
    box = (0.0, 1.0, 0.0, 1.0)
    w = mu[3]
    G = source_moments(lambda x, y: np.exp(-((x - 0.5) ** 2 + (y - 0.5) ** 2) / w ** 2),
                       2, n, n, box)
    return dict(dim=2, nx=n, ny=n, box=box, quad=("cl", n_theta, n_z, True),
                region=region, sigma_t=sigma_t, sigma_s=sigma_s, source=G, inflow=0.0,
                mu=mu)


def cfg3_train_test(n_train=64, n_test=256, seed_train=30, seed_test=31):
    """Training set = box centre followed by n_train-1 draws; test set = n_test draws."""
    tr = np.concatenate([cfg3_box_centre()[None], cfg3_mu(np.random.default_rng(seed_train),
                                                            n_train - 1)], 0)
    te = cfg3_mu(np.random.default_rng(seed_test), n_test)
    return tr, te


def cfg3_sigma(mus):
    """Per-region (sigma_t, sigma_s) [n, 2] of config-3 parameters (regions 0 = A, 1 = B)."""
    mus = np.atleast_2d(np.asarray(mus, dtype=np.float64))
    ss = mus[:, :2].copy()
    return ss + mus[:, 2:3], ss


def cfg3_sources(mus, n=96):
    """Source moments [len(mus), n*n*4] of config-3 parameters.  The Gaussian
    factorises in x and y, so each moment is a product of two 1D projections;
    equal to source_moments of the same Gaussian up to rounding."""
    mus = np.atleast_2d(np.asarray(mus, dtype=np.float64))
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    X = c[:, None] + 0.5 * h * _GL4_X[None, :]                    # [cell, gauss]
    w = 0.5 * h * _GL4_W
    basis = np.stack([np.ones(4), np.sqrt(3.0) * _GL4_X])         # [p, gauss]
    out = np.empty((len(mus), n, n, 4))
    for k, mu in enumerate(mus):
        f = np.exp(-((X - 0.5) ** 2) / mu[3] ** 2)                  # same factor in x and y
        m = (f[:, None, :] * (w * basis)[None]).sum(2) / np.sqrt(h)  # [cell, p]
        for q in range(2):
            for p in range(2):
                out[k, :, :, p + 2 * q] = m[:, q][:, None] * m[:, p][None, :]
    return out.reshape(len(mus), -1)


def cfg3_features(mus):
    """Parameter features in [0, 1]^4 for the learned correction:
    (log10 mu1, log10 mu2, mu3, mu4) mapped linearly from the parameter box."""
    mus = np.atleast_2d(np.asarray(mus, dtype=np.float64))
    z = np.stack([np.log10(mus[:, 0]), np.log10(mus[:, 1]), mus[:, 2], mus[:, 3]], 1)
    return (z - CFG3_BOX_LO) / (CFG3_BOX_HI - CFG3_BOX_LO)


def cfg5_sets(n_train=64, n_snap=10240, n_test=1024, seed_train=50, seed_snap=52, seed_test=51):
    """Config-3 parameter law for the learned-preconditioner workload: ROM
    training set (box centre + draws), snapshot-generation parameters, and
    fresh test parameters."""
    tr = np.concatenate([cfg3_box_centre()[None], cfg3_mu(np.random.default_rng(seed_train),
                                                            n_train - 1)], 0)
    sn = cfg3_mu(np.random.default_rng(seed_snap), n_snap)
    te = cfg3_mu(np.random.default_rng(seed_test), n_test)
    return tr, sn, te


def pincell_problem(mu, n=80, n_theta=30, n_z=6):
    """The pin-cell problem of section 5.2: [-1,1]^2, zero inflow, source
    exp(-100 (x^2 + y^2)); outer region (|x| > 0.5 or |y| > 0.5, region 0) a
    pure scatterer with sigma_s = 100; inner square (region 1) with
    (sigma_a, sigma_s) = (mu_a, mu_s).  CL(30, 6), z-folded (90 ordinates)."""
    mu = np.asarray(mu, dtype=np.float64)
    h = 2.0 / n
    c = -1.0 + (np.arange(n) + 0.5) * h
    inner = (np.abs(c)[None, :] <= 0.5) & (np.abs(c)[:, None] <= 0.5)   # [k, i]
    region = inner.reshape(-1).astype(np.int32)
    sigma_s = np.array([100.0, mu[1]])
    sigma_t = np.array([100.0, mu[0] + mu[1]])
    box = (-1.0, 1.0, -1.0, 1.0)
    G = source_moments(lambda x, y: np.exp(-100.0 * (x ** 2 + y ** 2)), 2, n, n, box)
    return dict(dim=2, nx=n, ny=n, box=box, quad=("cl", n_theta, n_z, True), region=region,
                sigma_t=sigma_t, sigma_s=sigma_s, source=G, inflow=0.0, mu=mu)


def pincell_sets(n_test=10, seed=60):
    """Training: the 5 x 5 uniform grid of (mu_a, mu_s) on [0.05, 0.5]^2, its
    centre (0.275, 0.275) first; test: n_test uniform draws."""
    g = np.linspace(0.05, 0.5, 5)
    grid = [(a, b) for a in g for b in g]
    centre = (0.275, 0.275)
    grid.remove(centre)
    tr = np.array([centre] + grid)
    te = np.random.default_rng(seed).uniform(0.05, 0.5, size=(n_test, 2))
    return tr, te


def twomat_problem(mu, n=64, n_theta=60, n_z=6):
    """The two-material problem with parametric inflow of section 5.4:
    [-1,1]^2, no source; inner square (|x|, |y| <= 0.5, region 1) a pure
    scatterer with sigma_s = mu_s; outer region (region 0) a pure absorber with
    sigma_a = 1; isotropic inflow mu_bc on the left side only.  CL(60, 6),
    z-folded (180 ordinates).  (The paper prints sigma_s twice; the second
    definition is read as sigma_a.)"""
    mu = np.asarray(mu, dtype=np.float64)
    h = 2.0 / n
    c = -1.0 + (np.arange(n) + 0.5) * h
    inner = (np.abs(c)[None, :] <= 0.5) & (np.abs(c)[:, None] <= 0.5)
    region = inner.reshape(-1).astype(np.int32)
    sigma_s = np.array([0.0, mu[0]])
    sigma_t = np.array([1.0, mu[0]])
    return dict(dim=2, nx=n, ny=n, box=(-1.0, 1.0, -1.0, 1.0), quad=("cl", n_theta, n_z, True),
                region=region, sigma_t=sigma_t, sigma_s=sigma_s, source=np.zeros(n * n * 4),
                inflow={"L": float(mu[1])}, mu=mu)


def twomat_sets(n_test=10, seed=70):
    """Training: mu_s = 1 + j/2 (j = 0..8) x mu_bc = 0.5 + k/10 (k = 0..10), with
    mu_1 = (3, 1) first; test: n_test uniform draws on [1,5] x [0.5,1.5]."""
    grid = [(1.0 + j / 2.0, 0.5 + k / 10.0) for j in range(9) for k in range(11)]
    first = grid.pop(4 * 11 + 5)
    assert abs(first[0] - 3.0) < 1e-12 and abs(first[1] - 1.0) < 1e-12
    tr = np.array([first] + grid)
    rng = np.random.default_rng(seed)
    te = np.stack([rng.uniform(1.0, 5.0, n_test), rng.uniform(0.5, 1.5, n_test)], 1)
    return tr, te


def cfg4_batch(seed=4, n_inst=512):
    """Uneven batch: grid in {32,64,96,128}^2, ordinates in {64, 128}; mu as config 3.
    64 ordinates = CL(16, 8) folded, 128 = CL(16, 16) folded."""
    rng = np.random.default_rng(seed)
    grids = rng.choice([32, 64, 96, 128], size=n_inst)
    nords = rng.choice([64, 128], size=n_inst)
    mus = cfg3_mu(rng, n_inst)
    return [(int(g), int(no), m) for g, no, m in zip(grids, nords, mus)]


def tiny_2d(seed=0, nx=3, ny=3, quad=("cl", 4, 2, False), n_regions=2, inflow=0.0,
            smooth_source=True):
    """Small random 2D problem for brute-force checks."""
    rng = np.random.default_rng(seed)
    region = rng.integers(0, n_regions, size=nx * ny).astype(np.int32)
    sig_s = rng.uniform(0.5, 3.0, size=n_regions)
    sig_a = rng.uniform(0.1, 1.0, size=n_regions)
    box = (0.0, 1.0, 0.0, 1.5)
    if smooth_source:
        G = source_moments(lambda x, y: 1.0 + np.sin(2 * x) * np.cos(3 * y), 2, nx, ny, box)
    else:
        G = rng.uniform(-1, 1, size=nx * ny * 4)
    return dict(dim=2, nx=nx, ny=ny, box=box, quad=quad, region=region,
                sigma_t=sig_s + sig_a, sigma_s=sig_s, source=G, inflow=inflow,
                mu=np.concatenate([sig_s, sig_a]))


def tiny_1d(seed=0, nx=4, n_ord=4, n_regions=2, inflow=0.0):
    rng = np.random.default_rng(seed)
    region = rng.integers(0, n_regions, size=nx).astype(np.int32)
    sig_s = rng.uniform(0.5, 3.0, size=n_regions)
    sig_a = rng.uniform(0.1, 1.0, size=n_regions)
    box = (0.0, 1.0, 0.0, 1.0)
    G = source_moments(lambda x, y: 1.0 + x * x, 1, nx, 1, box)
    return dict(dim=1, nx=nx, ny=1, box=box, quad=("gl", n_ord), region=region,
                sigma_t=sig_s + sig_a, sigma_s=sig_s, source=G, inflow=inflow,
                mu=np.concatenate([sig_s, sig_a]))


# ---------------------------------------------------------------- variable scattering (section 5.3)
FIELD_NQ = 6  # Gauss-Legendre points per axis at which a varying cross section is sampled per cell


def varscat_shape(x, y):
    """The spatial shape of the section-5.3 scattering cross section:
    r^4 (2 - r^2)^2 inside the unit disk, 1 outside (r^2 = x^2 + y^2)."""
    r2 = x * x + y * y
    return np.where(r2 <= 1.0, r2 * r2 * (2.0 - r2) ** 2, 1.0)


def _one(x, y):
    return np.ones_like(x)


def varscat_problem(mu_s, n=80, n_theta=30, n_z=6):
    """The variable-scattering problem of section 5.3: [-1,1]^2, zero inflow,
    sigma_a = 0, sigma_s(x) = mu_s s(x) + 0.1 with s = varscat_shape, source
    (10 / pi) exp(-100 (x^2 + y^2)); CL(30, 6) z-folded (90 ordinates).  The
    cross sections vary inside the cells: they are given as coefficients
    (sigma_t, sigma_s) of the shape functions (s, 1) in sigma_fields."""
    box = (-1.0, 1.0, -1.0, 1.0)
    G = source_moments(lambda x, y: 10.0 / np.pi * np.exp(-100.0 * (x ** 2 + y ** 2)), 2, n, n, box)
    coef = np.array([float(mu_s), 0.1])
    spec = dict(dim=2, nx=n, ny=n, box=box, quad=("cl", n_theta, n_z, True),
                region=np.zeros(n * n, dtype=np.int32), sigma_fields=[varscat_shape, _one],
                sigma_t=coef.copy(), sigma_s=coef.copy(), source=G, inflow=0.0,
                mu=np.array([float(mu_s)]))
    spec["field_values"] = _field_values_cached(n, box)
    return spec


_FV_CACHE = {}


def _field_values_cached(n, box):
    key = (n, box)
    if key not in _FV_CACHE:
        _FV_CACHE[key] = field_point_values(dict(nx=n, ny=n, box=box, sigma_fields=[varscat_shape, _one]))
    return _FV_CACHE[key]


def varscat_sets(n_test=10, seed=90):
    """51 uniformly spaced training values of mu_s on [49.9, 99.9] (the first
    sample mu_s = 74.9 is index 25) and n_test fresh uniform draws."""
    tr = np.linspace(49.9, 99.9, 51)
    te = np.random.default_rng(seed).uniform(49.9, 99.9, n_test)
    return tr, te


def field_point_values(spec, nq=FIELD_NQ):
    """Values of each shape function of spec["sigma_fields"] at the nq x nq
    Gauss-Legendre points of every cell: [n_fields][ncell][nq * nq], point
    index gy * nq + gx, cell = k * nx + i."""
    x0, x1, y0, y1 = spec["box"]
    nx, ny = spec["nx"], spec["ny"]
    hx, hy = (x1 - x0) / nx, (y1 - y0) / ny
    g, _ = np.polynomial.legendre.leggauss(nq)
    xc = x0 + (np.arange(nx) + 0.5) * hx
    yc = y0 + (np.arange(ny) + 0.5) * hy
    X = xc[None, :, None, None] + 0.5 * hx * g[None, None, None, :]
    Y = yc[:, None, None, None] + 0.5 * hy * g[None, None, :, None]
    X, Y = np.broadcast_arrays(X, Y)   # [k, i, gy, gx]
    return np.stack([np.asarray(f(X, Y), dtype=np.float64).reshape(nx * ny, nq * nq)
                     for f in spec["sigma_fields"]])


def with_field_values(spec, nq=FIELD_NQ):
    """spec with "field_values" (the library's input) sampled from its sigma_fields."""
    return dict(spec, field_values=field_point_values(spec, nq))
