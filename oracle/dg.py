"""Upwind discontinuous Galerkin operators on a uniform rectangular mesh,
assembled by numerical quadrature straight from their integral definitions
(sections 2.2-2.3: the weak form, the upwind flux and the matrix definitions
of D_j, Sigma_t, Sigma_s, G and g_j^(bc); App. A: D_C and D_J).

Basis: per cell the orthonormal tensor Legendre functions
eta_(p,q)(x, y) = e_p(x) e_q(y), e_0 = 1/sqrt(h), e_1 = sqrt(3) s / sqrt(h)
with s the local coordinate in [-1, 1].  Local index l = p + 2 q (l = p in 1D),
global index cell * nloc + l with cell = k * nx + i.

Every matrix M is stored so that (M psi)_k = sum_l M[k, l] psi_l with k the
test-function index, matching (D_j)_{kl} in section 2.3.
"""
import numpy as np
import scipy.sparse as sp

_QX, _QW = np.polynomial.legendre.leggauss(3)  # exact up to degree 5 per axis


class Mesh:
    def __init__(self, dim, nx, ny, box):
        self.dim = dim
        self.nx = nx
        self.ny = ny if dim == 2 else 1
        self.box = box
        self.hx = (box[1] - box[0]) / nx
        self.hy = (box[3] - box[2]) / self.ny if dim == 2 else 1.0
        self.nloc = 4 if dim == 2 else 2
        self.ncell = self.nx * self.ny
        self.ndof = self.ncell * self.nloc

    @staticmethod
    def of(problem):
        return Mesh(problem["dim"], problem["nx"], problem["ny"], problem["box"])


def _e(p, s, h):
    return (np.ones_like(s) if p == 0 else np.sqrt(3.0) * s) / np.sqrt(h)


def _de(p, s, h):  # d/dx of e_p, chain rule ds/dx = 2/h
    return (np.zeros_like(s) if p == 0 else np.sqrt(3.0) * 2.0 / h * np.ones_like(s)) / np.sqrt(h)


def _local_index(mesh):
    if mesh.dim == 1:
        return [(0, 0), (1, 0)]
    return [(0, 0), (1, 0), (0, 1), (1, 1)]


def _basis_at(mesh, sx, sy):
    """Values [nloc, npts] of the cell basis at local coordinates (sx, sy)."""
    vals = []
    for p, q in _local_index(mesh):
        v = _e(p, sx, mesh.hx)
        if mesh.dim == 2:
            v = v * _e(q, sy, mesh.hy)
        vals.append(v)
    return np.array(vals)


def _dbasis_at(mesh, sx, sy, axis):
    vals = []
    for p, q in _local_index(mesh):
        if axis == 0:
            v = _de(p, sx, mesh.hx)
            if mesh.dim == 2:
                v = v * _e(q, sy, mesh.hy)
        else:
            v = _e(p, sx, mesh.hx) * _de(q, sy, mesh.hy)
        vals.append(v)
    return np.array(vals)


def _volume_points(mesh):
    if mesh.dim == 1:
        return _QX, np.zeros_like(_QX), _QW * mesh.hx / 2
    SX, SY = np.meshgrid(_QX, _QX, indexing="xy")
    W = np.outer(_QW, _QW) * (mesh.hx / 2) * (mesh.hy / 2)
    return SX.ravel(), SY.ravel(), W.ravel()


# Faces of a cell: name -> (outward normal, local coordinates of face points,
# weights, neighbour offset (di, dk), coordinates of the same points seen from
# the neighbour cell)
def _faces(mesh):
    out = {}
    if mesh.dim == 1:
        one = np.array([1.0])
        out["L"] = ((-1.0, 0.0), (-one, 0 * one), one, (-1, 0), (one, 0 * one))
        out["R"] = ((1.0, 0.0), (one, 0 * one), one, (1, 0), (-one, 0 * one))
        return out
    wy = _QW * mesh.hy / 2
    wx = _QW * mesh.hx / 2
    on = np.ones_like(_QX)
    out["L"] = ((-1.0, 0.0), (-on, _QX), wy, (-1, 0), (on, _QX))
    out["R"] = ((1.0, 0.0), (on, _QX), wy, (1, 0), (-on, _QX))
    out["B"] = ((0.0, -1.0), (_QX, -on), wx, (0, -1), (_QX, on))
    out["T"] = ((0.0, 1.0), (_QX, on), wx, (0, 1), (_QX, -on))
    return out


def _cells(mesh):
    k, i = np.divmod(np.arange(mesh.ncell), mesh.nx)
    return i, k


def _scatter(mesh, blocks):
    """blocks: list of (rows_cell[nc], cols_cell[nc], B[nloc, nloc]) -> CSR."""
    nl = mesh.nloc
    R, C, V = [], [], []
    for rc, cc, B in blocks:
        rr = (rc[:, None, None] * nl + np.arange(nl)[None, :, None])
        cc2 = (cc[:, None, None] * nl + np.arange(nl)[None, None, :])
        rr, cc2 = np.broadcast_arrays(rr, cc2)
        R.append(rr.ravel())
        C.append(cc2.ravel())
        V.append(np.broadcast_to(B[None], rr.shape).ravel())
    return sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))),
                         shape=(mesh.ndof, mesh.ndof))


def mass_local(mesh):
    sx, sy, w = _volume_points(mesh)
    B = _basis_at(mesh, sx, sy)
    return (B * w) @ B.T


def sigma_matrix(mesh, sigma_cell):
    """(Sigma)_{kl} = sum_i int_{T_i} sigma eta_k eta_l with sigma constant per cell."""
    M = mass_local(mesh)
    i, k = _cells(mesh)
    c = np.arange(mesh.ncell)
    nl = mesh.nloc
    R = (c[:, None, None] * nl + np.arange(nl)[None, :, None])
    C = (c[:, None, None] * nl + np.arange(nl)[None, None, :])
    R, C = np.broadcast_arrays(R, C)
    V = sigma_cell[:, None, None] * M[None]
    return sp.csr_matrix((V.ravel(), (R.ravel(), C.ravel())), shape=(mesh.ndof, mesh.ndof))


def field_matrix(mesh, func, nq=6):
    """(Sigma)_{kl} = sum_i int_{T_i} f eta_k eta_l for a cross section f(x, y)
    that varies inside the cells (section 5.3), each cell integrated with the
    nq x nq Gauss-Legendre product rule (nq = 6 is exact for polynomials of
    degree 10 per axis: f of degree 8 times the degree-2 products of the
    basis)."""
    xq, wq = np.polynomial.legendre.leggauss(nq)
    if mesh.dim == 1:
        sx, sy, w = xq, np.zeros_like(xq), wq * mesh.hx / 2
    else:
        SX, SY = np.meshgrid(xq, xq, indexing="xy")
        sx, sy = SX.ravel(), SY.ravel()
        w = np.outer(wq, wq).ravel() * (mesh.hx / 2) * (mesh.hy / 2)
    B = _basis_at(mesh, sx, sy)
    i, k = _cells(mesh)
    x0, _, y0, _ = mesh.box
    X = x0 + (i[:, None] + 0.5 + 0.5 * sx[None]) * mesh.hx
    Y = (y0 + (k[:, None] + 0.5 + 0.5 * sy[None]) * mesh.hy) if mesh.dim == 2 else 0 * X
    F = func(X, Y)                                   # [ncell, npts]
    V = np.einsum("cq,kq,lq->ckl", F * w[None], B, B)  # [ncell, nloc, nloc]
    c = np.arange(mesh.ncell)
    nl = mesh.nloc
    R = (c[:, None, None] * nl + np.arange(nl)[None, :, None])
    C = (c[:, None, None] * nl + np.arange(nl)[None, None, :])
    R, C = np.broadcast_arrays(R, C)
    return sp.csr_matrix((V.ravel(), (R.ravel(), C.ravel())), shape=(mesh.ndof, mesh.ndof))


def advection(mesh, ox, oy):
    """(D_j)_{kl} = -sum_i int_{T_i} (Omega . grad eta_k) eta_l
                    + sum over cell faces not on the inflow boundary of
                      int_F H(Omega, eta_l, n) eta_k,
    with the upwind flux H = (Omega.n) eta_l^- if Omega.n > 0 (own trace) and
    (Omega.n) eta_l^+ (neighbour trace) otherwise (equation of the upwind flux).
    """
    sx, sy, w = _volume_points(mesh)
    B = _basis_at(mesh, sx, sy)
    dBx = _dbasis_at(mesh, sx, sy, 0)
    grad_dot = ox * dBx
    if mesh.dim == 2:
        grad_dot = grad_dot + oy * _dbasis_at(mesh, sx, sy, 1)
    vol = -(grad_dot * w) @ B.T  # [k, l]
    i, k = _cells(mesh)
    c = np.arange(mesh.ncell)
    blocks = [(c, c, vol)]
    for name, (n, (fx, fy), fw, (di, dk), (gx, gy)) in _faces(mesh).items():
        on = ox * n[0] + oy * n[1]
        if on == 0.0:
            continue
        Bown = _basis_at(mesh, fx, fy)  # test and own-trace values on the face
        if on > 0:
            blocks.append((c, c, on * (Bown * fw) @ Bown.T))
        else:
            ni, nk = i + di, k + dk
            inside = (ni >= 0) & (ni < mesh.nx) & (nk >= 0) & (nk < mesh.ny)
            Bnb = _basis_at(mesh, gx, gy)  # neighbour's basis at the same points
            blocks.append((c[inside], (nk * mesh.nx + ni)[inside], on * (Bown * fw) @ Bnb.T))
    return _scatter(mesh, blocks)


def inflow_vector(mesh, ox, oy, g):
    """(g_j^(bc))_k = -sum over inflow-boundary faces of int_F g eta_k Omega.n.
    g is a constant, a callable g(x, y), or a dict of per-side constants with
    keys "L", "R", "B", "T" (missing sides: zero inflow)."""
    out = np.zeros(mesh.ndof)
    i, k = _cells(mesh)
    x0, _, y0, _ = mesh.box
    for name, (n, (fx, fy), fw, (di, dk), _) in _faces(mesh).items():
        on = ox * n[0] + oy * n[1]
        if on >= 0.0:
            continue
        ni, nk = i + di, k + dk
        bnd = ~((ni >= 0) & (ni < mesh.nx) & (nk >= 0) & (nk < mesh.ny))
        Bown = _basis_at(mesh, fx, fy)
        for c in np.nonzero(bnd)[0]:
            xs = x0 + (i[c] + 0.5 + 0.5 * fx) * mesh.hx
            ys = (y0 + (k[c] + 0.5 + 0.5 * fy) * mesh.hy) if mesh.dim == 2 else 0 * xs
            if isinstance(g, dict):
                gv = np.full_like(xs, float(g.get(name, 0.0)))
            else:
                gv = g(xs, ys) if callable(g) else np.full_like(xs, float(g))
            out[c * mesh.nloc:(c + 1) * mesh.nloc] += -on * (Bown * fw) @ gv
    return out


def project(mesh, func):
    """L2 projection coefficients int_T f eta_k (orthonormal basis)."""
    sx, sy, w = _volume_points(mesh)
    B = _basis_at(mesh, sx, sy)
    i, k = _cells(mesh)
    x0, _, y0, _ = mesh.box
    X = x0 + (i[:, None] + 0.5 + 0.5 * sx[None]) * mesh.hx
    Y = (y0 + (k[:, None] + 0.5 + 0.5 * sy[None]) * mesh.hy) if mesh.dim == 2 else 0 * X
    F = func(X, Y)
    return ((F * w[None]) @ B.T).reshape(-1)


def central_and_jump(mesh, axis, include_boundary_faces=True):
    """App. A operators along one axis (tensor extension in 2D):
       (D_C)_{kl} = -sum_i int_{T_i} d_e eta_k eta_l - sum_faces int {eta_l}[eta_k],
       (D_J)_{kl} = -sum_faces int [eta_l][eta_k],
    [eta] = eta(+side) - eta(-side), {eta} = average; faces normal to `axis`.
    A boundary face has a zero exterior trace; with include_boundary_faces=False
    only the faces printed in App. A (x_{i+1/2}, i = 1..N_x, i.e. all but the
    first) are kept."""
    sx, sy, w = _volume_points(mesh)
    B = _basis_at(mesh, sx, sy)
    dB = _dbasis_at(mesh, sx, sy, axis)
    vol = -(dB * w) @ B.T
    i, k = _cells(mesh)
    c = np.arange(mesh.ncell)
    DC = [(c, c, vol)]
    DJ = []
    faces = _faces(mesh)
    # every face normal to `axis` is visited once, from its minus-side cell
    # (the cell whose outward normal along +axis crosses it); boundary faces on
    # the low side are visited from the plus-side cell.
    fname_hi, fname_lo = ("R", "L") if axis == 0 else ("T", "B")
    n, (fx, fy), fw, (di, dk), (gx, gy) = faces[fname_hi]
    Bm = _basis_at(mesh, fx, fy)      # minus side (this cell) at the face
    Bp = _basis_at(mesh, gx, gy)      # plus side (neighbour) at the same points
    ni, nk = i + di, k + dk
    inside = (ni >= 0) & (ni < mesh.nx) & (nk >= 0) & (nk < mesh.ny)
    cm = c
    cp = nk * mesh.nx + ni
    # jump [eta] = eta^+ - eta^-, average {eta} = (eta^+ + eta^-)/2
    # test k and trial l each live on one side; enumerate side pairs
    for sk, Bk in (("m", -Bm), ("p", Bp)):  # jump factor of the test function
        for sl, Bl, jl in (("m", Bm, -1.0), ("p", Bp, 1.0)):
            avg = -0.5 * (Bk * fw) @ Bl.T     # -{eta_l}[eta_k]
            jmp = -jl * (Bk * fw) @ Bl.T      # -[eta_l][eta_k]
            rows = cm if sk == "m" else cp
            cols = cm if sl == "m" else cp
            sel = inside if (sk == "p" or sl == "p") else np.ones_like(inside)
            # the (minus, minus) pair also covers high-side boundary faces,
            # where the exterior (plus) trace is zero
            DC.append((rows[sel], cols[sel], avg))
            DJ.append((rows[sel], cols[sel], jmp))
    if include_boundary_faces:
        # low-side boundary faces: the cell is the plus side, exterior minus trace 0
        n2, (fx2, fy2), fw2, (di2, dk2), _ = faces[fname_lo]
        Bp2 = _basis_at(mesh, fx2, fy2)
        ni2, nk2 = i + di2, k + dk2
        bsel = ~((ni2 >= 0) & (ni2 < mesh.nx) & (nk2 >= 0) & (nk2 < mesh.ny))
        avg = -0.5 * (Bp2 * fw2) @ Bp2.T
        jmp = -(Bp2 * fw2) @ Bp2.T
        DC.append((c[bsel], c[bsel], avg))
        DJ.append((c[bsel], c[bsel], jmp))
    return _scatter(mesh, DC), _scatter(mesh, DJ)
