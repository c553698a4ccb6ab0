// Fully consistent DSA (App. A) for slab and X-Y geometry.
//
// The correction equation's zeroth and first angular moments under the P1
// ansatz delta psi_j = dphi + 3 Omega_j . dJ give, with the central-flux and
// jump operators D_C^e, D_J^e of App. A (D_j = sum_e Omega_e (D_C^e -
// sgn(Omega_e)/2 D_J^e)) and the quadrature moments
//   m_e = sum w O_e, beta_e = sum w |O_e| / 2, a_ef = sum w O_e O_f,
//   b_ef = sum w |O_e| O_f, bm_de = sum w O_d |O_e|, t_def = sum w O_d O_e O_f,
//   c_def = sum w O_d |O_e| O_f,
// the system
//   [sum_e (m_e DC^e - beta_e DJ^e) + (st - ss)] dphi
//     + 3 sum_f [sum_e (a_ef DC^e - b_ef DJ^e / 2) + m_f st] dJ_f = ss v
//   [sum_e (a_de DC^e - bm_de DJ^e / 2) + m_d (st - ss)] dphi
//     + 3 sum_f [sum_e (t_def DC^e - c_def DJ^e / 2) + a_df st] dJ_f = m_d ss v.
// Unknowns per cell: [dphi(nloc), dJ_x(nloc) (, dJ_y(nloc))], stored unknown-major
// per instance (unknown u of cell c at u * ncell + c) so that neighbouring
// threads read neighbouring cells.
//
// D_C, D_J along one axis, orthonormal P1 basis on cells of width h (traces
// R = (1, sqrt3)/sqrt h at the right end, L = (1, -sqrt3)/sqrt h at the left):
//   D_C: own block  -int e_k' e_l + (R R^T - L L^T)/2,  right neighbour R L^T/2,
//        left neighbour -L R^T/2;
//   D_J: own block -(R R^T + L L^T),  right neighbour R L^T,  left neighbour L R^T.
// With both boundary faces included the own blocks are the same for every
// cell; boundary cells simply lack the neighbour couplings.  X-Y operators are
// tensor products with the identity along the other axis.
//
// The system is solved with geometric multigrid: V-cycles over grids coarsened
// by 2 x 2 cell agglomeration, the same moment system rediscretised on every
// level with cell-averaged cross sections, red-black block Gauss-Seidel
// smoothing with exact inverses of the per-cell diagonal blocks, and the
// natural injection of the coarse degree-1 space into the fine one as
// prolongation (its transpose restricts).  A DSA application is either a fixed
// number of V-cycles (a linear preconditioner, the production setting) or
// restarted GMRES preconditioned by one V-cycle, run to a tolerance.
#include <algorithm>
#include <cmath>

#include "krylov.h"

namespace rte {

constexpr int DMAX = 12;  // unknowns per cell in 2D (3 fields x 4 dofs)

// Per instance: 5 neighbour blocks (self, x-, x+, y-, y+) of size nu x nu,
// and the sigma_t / sigma_s coefficient blocks (nu = 4 in 1D, 12 in 2D).
struct DsaStencil {
  double blk[5][DMAX * DMAX];
  double St[DMAX * DMAX];
  double Ss[DMAX * DMAX];
  double m[2];  // m_x, m_y (right-hand side weights of the first-moment rows)
  int nu;
  // reflection-symmetric X-Y rules (m = b = bm = t = 0, a_xy = 0, c_xey = c_yex = 0):
  // the scalars of the structured form used by the fast kernels
  int sym;
  double ax, ay, bex, bey, cxx, cxy, cyx, cyy, hx, hy;
  // The smoother's cell blocks are always those of the FC system: bcxx..bcyy
  // are the FC jump coefficients of the first-moment rows (the structured
  // form) and blkd the FC self block (general form).  For PC, whose blocks
  // lack the jump terms in the first-moment rows, red-black block
  // Gauss-Seidel with its own blocks diverges (dJ couples to the neighbours'
  // dphi through central fluxes only); with the FC blocks a V(2,2) cycle is
  // a good GMRES preconditioner for it, though no dependable stationary
  // iteration, so PC solves always run the Krylov method (restart >= 1).
  double bcxx, bcxy, bcyx, bcyy;
  double blkd[DMAX * DMAX];
};

__device__ static void axis_ops(double h, double DCs[4], double DCp[4], double DCm[4], double DJs[4],
                                double DJp[4], double DJm[4]) {
  const double r3 = 1.7320508075688772935;
  const double R[2] = {1.0, r3}, L[2] = {1.0, -r3};
  const double vol[4] = {0.0, 0.0, -2.0 * r3, 0.0};  // -int e_k' e_l, [k][l]
  for (int k = 0; k < 2; ++k)
    for (int l = 0; l < 2; ++l) {
      const int kl = k * 2 + l;
      DCs[kl] = vol[kl] * (1.0 / h) + (R[k] * R[l] - L[k] * L[l]) / (2.0 * h);
      DCp[kl] = R[k] * L[l] / (2.0 * h);
      DCm[kl] = -L[k] * R[l] / (2.0 * h);
      DJs[kl] = -(R[k] * R[l] + L[k] * L[l]) / h;
      DJp[kl] = R[k] * L[l] / h;
      DJm[kl] = L[k] * R[l] / h;
    }
}

// One thread per instance builds its stencil (moments in a fixed order).
// pc: the partially consistent variant (App. A, last paragraph), whose
// first-moment rows keep only the central-flux part of the advection.
__global__ void k_dsa_setup(int n_inst, const InstDev* __restrict__ insts,
                            const double* __restrict__ ox, const double* __restrict__ oy,
                            const double* __restrict__ w, DsaStencil* __restrict__ out, int pc) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_inst) return;
  const InstDev I = insts[b];
  const int dim = I.dim;
  const int nl = I.nloc;
  const int ne = dim;          // number of axes
  const int nu = nl * (1 + dim);
  double m[2] = {0, 0}, be[2] = {0, 0}, a[2][2] = {{0}}, bb[2][2] = {{0}}, bm[2][2] = {{0}};
  double t[2][2][2] = {{{0}}}, c[2][2][2] = {{{0}}};
  for (int s = 0; s < I.n_ord; ++s) {
    const int js = I.ord_off + s;
    const double O[2] = {ox[js], dim == 2 ? oy[js] : 0.0};
    const double A[2] = {fabs(O[0]), fabs(O[1])};
    const double ww = w[js];
    for (int e = 0; e < 2; ++e) {
      m[e] += ww * O[e];
      be[e] += 0.5 * ww * A[e];
      for (int f = 0; f < 2; ++f) {
        a[e][f] += ww * O[e] * O[f];
        bb[e][f] += ww * A[e] * O[f];
        bm[e][f] += ww * O[e] * A[f];
        for (int g = 0; g < 2; ++g) {
          t[e][f][g] += ww * O[e] * O[f] * O[g];
          c[e][f][g] += ww * O[e] * A[f] * O[g];
        }
      }
    }
  }
  // per-axis local operators (2x2 in the axis' own mode index)
  double DCs[2][4], DCp[2][4], DCm[2][4], DJs[2][4], DJp[2][4], DJm[2][4];
  axis_ops(I.hx, DCs[0], DCp[0], DCm[0], DJs[0], DJp[0], DJm[0]);
  axis_ops(I.hy, DCs[1], DCp[1], DCm[1], DJs[1], DJp[1], DJm[1]);
  // embed an axis operator into the nl x nl cell block (tensor with identity)
  auto emb = [&](const double* op, int e, int k, int l) -> double {
    if (dim == 1) return op[k * 2 + l];
    const int pk = k & 1, qk = k >> 1, pl = l & 1, ql = l >> 1;
    if (e == 0) return (qk == ql) ? op[pk * 2 + pl] : 0.0;
    return (pk == pl) ? op[qk * 2 + ql] : 0.0;
  };
  DsaStencil S;
  S.nu = nu;
  S.m[0] = m[0];
  S.m[1] = m[1];
  {
    const double tz = 1e-13;
    bool sy = dim == 2 && fabs(m[0]) < tz && fabs(m[1]) < tz && fabs(a[0][1]) < tz && fabs(a[1][0]) < tz;
    for (int e = 0; e < 2; ++e)
      for (int f = 0; f < 2; ++f) {
        sy = sy && fabs(bb[e][f]) < tz && fabs(bm[e][f]) < tz && fabs(c[0][e][1]) < tz &&
             fabs(c[1][e][0]) < tz;
        for (int g = 0; g < 2; ++g) sy = sy && fabs(t[e][f][g]) < tz;
      }
    S.sym = sy ? 1 : 0;
    if (sy) S.m[0] = S.m[1] = 0.0;  // a reflection-symmetric rule's first moments vanish exactly
    S.ax = a[0][0];
    S.ay = a[1][1];
    S.bex = be[0];
    S.bey = be[1];
    // the jump terms of the first-moment rows (none in PC-DSA)
    S.cxx = pc ? 0.0 : c[0][0][0];
    S.cxy = pc ? 0.0 : c[0][1][0];
    S.cyx = pc ? 0.0 : c[1][0][1];
    S.cyy = pc ? 0.0 : c[1][1][1];
    S.hx = I.hx;
    S.hy = I.hy;
    S.bcxx = c[0][0][0];
    S.bcxy = c[0][1][0];
    S.bcyx = c[1][0][1];
    S.bcyy = c[1][1][1];
  }
  for (int z = 0; z < 5; ++z)
    for (int q = 0; q < DMAX * DMAX; ++q) S.blk[z][q] = 0.0;
  for (int q = 0; q < DMAX * DMAX; ++q) S.St[q] = S.Ss[q] = S.blkd[q] = 0.0;
  // field blocks: coefficient (alpha_C[e], alpha_J[e]) for field row F, column F'
  // F = 0: dphi, F = 1 + d: dJ_d
  for (int F = 0; F <= ne; ++F)
    for (int Fp = 0; Fp <= ne; ++Fp) {
      double aC[2] = {0, 0}, aJ[2] = {0, 0}, aJf[2] = {0, 0};  // aJf: FC jump weights
      for (int e = 0; e < ne; ++e) {
        if (F == 0 && Fp == 0) {
          aC[e] = m[e];
          aJ[e] = -be[e];
        } else if (F == 0) {
          const int f = Fp - 1;
          aC[e] = 3.0 * a[e][f];
          aJ[e] = -1.5 * bb[e][f];
        } else if (Fp == 0) {
          const int d = F - 1;
          aC[e] = a[d][e];
          aJf[e] = -0.5 * bm[d][e];
          aJ[e] = pc ? 0.0 : aJf[e];
        } else {
          const int d = F - 1, f = Fp - 1;
          aC[e] = 3.0 * t[d][e][f];
          aJf[e] = -1.5 * c[d][e][f];
          aJ[e] = pc ? 0.0 : aJf[e];
        }
        if (F == 0) aJf[e] = aJ[e];
      }
      for (int k = 0; k < nl; ++k)
        for (int l = 0; l < nl; ++l) {
          const int row = F * nl + k, col = Fp * nl + l, q = row * nu + col;
          double self = 0.0, selff = 0.0;
          for (int e = 0; e < ne; ++e) {
            self += aC[e] * emb(DCs[e], e, k, l) + aJ[e] * emb(DJs[e], e, k, l);
            selff += aC[e] * emb(DCs[e], e, k, l) + aJf[e] * emb(DJs[e], e, k, l);
          }
          S.blk[0][q] = self;
          S.blkd[q] = selff;
          S.blk[1][q] = aC[0] * emb(DCm[0], 0, k, l) + aJ[0] * emb(DJm[0], 0, k, l);
          S.blk[2][q] = aC[0] * emb(DCp[0], 0, k, l) + aJ[0] * emb(DJp[0], 0, k, l);
          if (dim == 2) {
            S.blk[3][q] = aC[1] * emb(DCm[1], 1, k, l) + aJ[1] * emb(DJm[1], 1, k, l);
            S.blk[4][q] = aC[1] * emb(DCp[1], 1, k, l) + aJ[1] * emb(DJp[1], 1, k, l);
          }
          if (k == l) {
            // sigma terms (mass matrix = identity in the orthonormal basis)
            double ct = 0.0, cs = 0.0;
            if (F == 0 && Fp == 0) { ct = 1.0; cs = -1.0; }
            else if (F == 0) { ct = 3.0 * m[Fp - 1]; }
            else if (Fp == 0) { ct = m[F - 1]; cs = -m[F - 1]; }
            else { ct = 3.0 * a[F - 1][Fp - 1]; }
            S.St[q] = ct;
            S.Ss[q] = cs;
          }
        }
    }
  out[b] = S;
}

// Inverse of the diagonal block of every (instance, region): Gauss-Jordan
// with partial pivoting, one thread each.
__global__ void k_dsa_blockinv(int n_inst, int max_regions, const InstDev* __restrict__ insts,
                               const DsaStencil* __restrict__ st_, const double* __restrict__ sigma_t,
                               const double* __restrict__ sigma_s, double* __restrict__ inv) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = id / max_regions, rg = id % max_regions;
  if (b >= n_inst) return;
  if (rg >= insts[b].n_regions) return;
  const DsaStencil& S = st_[b];
  const int nu = S.nu;
  const double ts = sigma_t[(int64_t)b * max_regions + rg], ss = sigma_s[(int64_t)b * max_regions + rg];
  double A[DMAX][2 * DMAX];
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j < nu; ++j) {
      A[i][j] = S.blkd[i * nu + j] + ts * S.St[i * nu + j] + ss * S.Ss[i * nu + j];
      A[i][nu + j] = (i == j) ? 1.0 : 0.0;
    }
  for (int col = 0; col < nu; ++col) {
    int piv = col;
    double best = fabs(A[col][col]);
    for (int r = col + 1; r < nu; ++r)
      if (fabs(A[r][col]) > best) {
        best = fabs(A[r][col]);
        piv = r;
      }
    if (piv != col)
      for (int j = 0; j < 2 * nu; ++j) {
        const double tmp = A[col][j];
        A[col][j] = A[piv][j];
        A[piv][j] = tmp;
      }
    const double d = A[col][col];
    const double f = d != 0.0 ? 1.0 / d : 0.0;
    for (int j = 0; j < 2 * nu; ++j) A[col][j] *= f;
    for (int r = 0; r < nu; ++r) {
      if (r == col) continue;
      const double x = A[r][col];
      if (x == 0.0) continue;
      for (int j = 0; j < 2 * nu; ++j) A[r][j] -= x * A[col][j];
    }
  }
  double* o = inv + ((int64_t)b * max_regions + rg) * nu * nu;  // same stride the stencil reads
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j < nu; ++j) o[i * nu + j] = A[i][nu + j];
}

// rhs = [ss v, m_x ss v (, m_y ss v)] per cell
template <typename real>
__global__ void k_dsa_rhs(const InstDev* __restrict__ insts, const DsaStencil* __restrict__ st_,
                          const int32_t* __restrict__ region, const double* __restrict__ sigma_s,
                          int max_regions, const int64_t* __restrict__ off,
                          const double* __restrict__ v, real* __restrict__ rhs,
                          const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const InstDev I = insts[b];
  const DsaStencil& S = st_[b];
  const int nl = I.nloc;
  const int ncell = I.nx * I.ny;
  for (int cell = blockIdx.x * blockDim.x + threadIdx.x; cell < ncell; cell += gridDim.x * blockDim.x) {
    const double ss = sigma_s[(int64_t)b * max_regions + region[I.region_off + cell]];
    for (int l = 0; l < nl; ++l) {
      const double sv = ss * v[I.dof_off + (int64_t)cell * nl + l];
      rhs[off[b] + (int64_t)l * ncell + cell] = (real)sv;
      for (int d = 0; d < I.dim; ++d)
        rhs[off[b] + (int64_t)((1 + d) * nl + l) * ncell + cell] = (real)(S.m[d] * sv);
    }
  }
}

// z = v + dphi (the first nloc unknowns of every cell)
template <typename real>
__global__ void k_dsa_out(const InstDev* __restrict__ insts, const DsaStencil* __restrict__ st_,
                          const int64_t* __restrict__ off, const real* __restrict__ u,
                          const double* __restrict__ v, double* __restrict__ z,
                          const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const InstDev I = insts[b];
  const int nl = I.nloc;
  const int64_t ncell = (int64_t)I.nx * I.ny, nd = ncell * nl;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < nd;
       d += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = d / nl, l = d % nl;
    z[I.dof_off + d] = v[I.dof_off + d] + (double)u[off[b] + l * ncell + cell];
  }
}

// y += x over each active instance's block of the level-0 DSA vector
template <typename real>
__global__ void k_dsa_axpy(const int64_t* __restrict__ off, const int64_t* __restrict__ len,
                           const real* __restrict__ x, real* __restrict__ y, const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int64_t lo = off[b], n = len[b];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[lo + e] += x[lo + e];
}

// Cross sections varying inside the cells (section 5.3): rhs = [Sigma_s v,
// m_d Sigma_s v] with the cells' full scattering blocks.
__global__ void k_dsa_rhs_field(const InstDev* __restrict__ insts, const DsaStencil* __restrict__ st_,
                                const double* __restrict__ fblk, int nf, int64_t fcell,
                                const double* __restrict__ sigma_s, int max_regions, const int64_t* __restrict__ off,
                                const double* __restrict__ v, double* __restrict__ rhs,
                                const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const InstDev I = insts[b];
  const DsaStencil& S = st_[b];
  const int ncell = I.nx * I.ny;
  const double* th = sigma_s + (int64_t)b * max_regions;
  for (int cell = blockIdx.x * blockDim.x + threadIdx.x; cell < ncell; cell += gridDim.x * blockDim.x) {
    double B[16];
    field_block(fblk, nf, fcell, cell, th, B);
    const double* vc = v + I.dof_off + 4 * (int64_t)cell;
    for (int l = 0; l < 4; ++l) {
      const double sv = B[4 * l] * vc[0] + B[4 * l + 1] * vc[1] + B[4 * l + 2] * vc[2] + B[4 * l + 3] * vc[3];
      rhs[off[b] + (int64_t)l * ncell + cell] = sv;
      for (int d = 0; d < 2; ++d) rhs[off[b] + (int64_t)((1 + d) * 4 + l) * ncell + cell] = S.m[d] * sv;
    }
  }
}

// y += sign (K - K_avg) x on level 0 of a field-mode DSA: the sigma terms of
// the moment system with every cell's full mass blocks in place of the cell
// averages (the (0, 0) entries) that the multigrid hierarchy uses.  The
// coefficient of field F' in the rows of field F is the stencil's sigma
// pattern (St, Ss: identity over the moments for piecewise-constant cross
// sections).
__global__ void k_dsa_field_corr(const InstDev* __restrict__ insts, const DsaStencil* __restrict__ st_,
                                 const double* __restrict__ fblk, int nf, int64_t fcell,
                                 const double* __restrict__ sigma_t, const double* __restrict__ sigma_s,
                                 int max_regions, const int64_t* __restrict__ off, const double* __restrict__ x,
                                 double* __restrict__ y, double sign, const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const InstDev I = insts[b];
  const DsaStencil& S = st_[b];
  const int ncell = I.nx * I.ny;
  const int nu = 12;
  const double* tt = sigma_t + (int64_t)b * max_regions;
  const double* ts = sigma_s + (int64_t)b * max_regions;
  for (int cell = blockIdx.x * blockDim.x + threadIdx.x; cell < ncell; cell += gridDim.x * blockDim.x) {
    double Bt[16], Bs[16];
    field_block(fblk, nf, fcell, cell, tt, Bt);
    field_block(fblk, nf, fcell, cell, ts, Bs);
    const double at = Bt[0], as = Bs[0];
    for (int k = 0; k < 4; ++k) {
      Bt[5 * k] -= at;
      Bs[5 * k] -= as;
    }
    const double* xb = x + off[b];
    double* yb = y + off[b];
    for (int F = 0; F < 3; ++F)
      for (int Fp = 0; Fp < 3; ++Fp) {
        const double ct = S.St[(F * 4) * nu + Fp * 4], cs = S.Ss[(F * 4) * nu + Fp * 4];
        if (ct == 0.0 && cs == 0.0) continue;
        double xv[4];
        for (int l = 0; l < 4; ++l) xv[l] = xb[(int64_t)(Fp * 4 + l) * ncell + cell];
        for (int k = 0; k < 4; ++k) {
          double acc = 0.0;
          for (int l = 0; l < 4; ++l) acc += (ct * Bt[4 * k + l] + cs * Bs[4 * k + l]) * xv[l];
          yb[(int64_t)(F * 4 + k) * ncell + cell] += sign * acc;
        }
      }
  }
}

// ------------------------------------------------------------------ multigrid
struct LvlInst {
  int32_t nx, ny, dim, nloc;
  double hx, hy;
  int64_t cell_off;   // first cell of this instance in the level's cell arrays
};

// Level-0 per-cell cross sections from the region tables.
__global__ void k_mg_sigma0(const InstDev* __restrict__ insts, const LvlInst* __restrict__ li,
                            const int32_t* __restrict__ region, const double* __restrict__ sigma_t,
                            const double* __restrict__ sigma_s, int max_regions,
                            double* __restrict__ st, double* __restrict__ ss) {
  const int b = blockIdx.y;
  const InstDev I = insts[b];
  const LvlInst L = li[b];
  const int nc = L.nx * L.ny;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    const int rg = region[I.region_off + c];
    st[L.cell_off + c] = sigma_t[(int64_t)b * max_regions + rg];
    ss[L.cell_off + c] = sigma_s[(int64_t)b * max_regions + rg];
  }
}

// Level-0 per-cell cross sections of a field-mode batch: the cell averages,
// the (0, 0) entries of the full blocks.
__global__ void k_mg_sigma0_field(const InstDev* __restrict__ insts, const LvlInst* __restrict__ li,
                                  const double* __restrict__ fblk, int nf, int64_t fcell,
                                  const double* __restrict__ sigma_t, const double* __restrict__ sigma_s,
                                  int max_regions, double* __restrict__ st, double* __restrict__ ss) {
  const int b = blockIdx.y;
  const LvlInst L = li[b];
  const int nc = L.nx * L.ny;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    double t = 0.0, u = 0.0;
    for (int f = 0; f < nf; ++f) {
      const double m00 = fblk[((int64_t)f * fcell + c) * 16];
      t += sigma_t[(int64_t)b * max_regions + f] * m00;
      u += sigma_s[(int64_t)b * max_regions + f] * m00;
    }
    st[L.cell_off + c] = t;
    ss[L.cell_off + c] = u;
  }
}

// Coarse cross sections: average over the 2 x 2 (slab: 2) children.
__global__ void k_mg_sigma_coarsen(const LvlInst* __restrict__ lf, const LvlInst* __restrict__ lc,
                                   const double* __restrict__ stf, const double* __restrict__ ssf,
                                   double* __restrict__ stc, double* __restrict__ ssc) {
  const int b = blockIdx.y;
  const LvlInst F = lf[b], Cc = lc[b];
  const int nc = Cc.nx * Cc.ny;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    const int I = c % Cc.nx, K = c / Cc.nx;
    double t = 0.0, u = 0.0;
    int cnt = 0;
    for (int dk = 0; dk < (F.dim == 2 ? 2 : 1); ++dk)
      for (int di = 0; di < 2; ++di) {
        const int f = (F.dim == 2 ? (2 * K + dk) * F.nx : 0) + 2 * I + di;
        t += stf[F.cell_off + f];
        u += ssf[F.cell_off + f];
        ++cnt;
      }
    stc[Cc.cell_off + c] = t / cnt;
    ssc[Cc.cell_off + c] = u / cnt;
  }
}

template <int NU>
__device__ void invert_block(const double* M, double* out) {
  double A[NU][2 * NU];
  for (int i = 0; i < NU; ++i)
    for (int j = 0; j < NU; ++j) {
      A[i][j] = M[i * NU + j];
      A[i][NU + j] = (i == j) ? 1.0 : 0.0;
    }
  for (int col = 0; col < NU; ++col) {
    int piv = col;
    double best = fabs(A[col][col]);
    for (int r = col + 1; r < NU; ++r)
      if (fabs(A[r][col]) > best) {
        best = fabs(A[r][col]);
        piv = r;
      }
    if (piv != col)
      for (int j = 0; j < 2 * NU; ++j) {
        const double tmp = A[col][j];
        A[col][j] = A[piv][j];
        A[piv][j] = tmp;
      }
    const double d = A[col][col];
    const double f = d != 0.0 ? 1.0 / d : 0.0;
    for (int j = 0; j < 2 * NU; ++j) A[col][j] *= f;
    for (int r = 0; r < NU; ++r) {
      if (r == col) continue;
      const double x = A[r][col];
      if (x == 0.0) continue;
      for (int j = 0; j < 2 * NU; ++j) A[r][j] -= x * A[col][j];
    }
  }
  for (int i = 0; i < NU; ++i)
    for (int j = 0; j < NU; ++j) out[i * NU + j] = A[i][NU + j];
}

// Per-cell inverse of the diagonal block (coarse levels).
template <int NU>
__global__ void k_mg_inv_cells(const LvlInst* __restrict__ li, const DsaStencil* __restrict__ st_,
                               const double* __restrict__ st, const double* __restrict__ ss,
                               double* __restrict__ inv, const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const LvlInst L = li[b];
  const DsaStencil& S = st_[b];
  const int nc = L.nx * L.ny;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    const double t = st[L.cell_off + c], u = ss[L.cell_off + c];
    double M[NU * NU];
    for (int q = 0; q < NU * NU; ++q) M[q] = S.blkd[q] + t * S.St[q] + u * S.Ss[q];
    invert_block<NU>(M, inv + (L.cell_off + c) * NU * NU);
  }
}

__device__ __forceinline__ int lvl_inv_index(int per_cell, int64_t cell_global, int b, int max_regions,
                                             int rg) {
  return per_cell ? (int)cell_global : b * max_regions + rg;
}

// mode 0: y = K x; mode 1: y = b - K x (residual);
// mode 2 (color c): x_c += inv_c (b - K x)_c for cells with (i + k) % 2 == c.
template <int NU>
__global__ void __launch_bounds__(256) k_mg_stencil(int mode, int color, const LvlInst* __restrict__ li,
                             const DsaStencil* __restrict__ st_, const double* __restrict__ st,
                             const double* __restrict__ ss, const double* __restrict__ inv,
                             int per_cell_inv, const int32_t* __restrict__ region0,
                             const InstDev* __restrict__ insts, int max_regions,
                             const double* __restrict__ bvec, double* __restrict__ x,
                             double* __restrict__ y, const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const LvlInst L = li[b];
  __shared__ double blk[7 * NU * NU];
  const DsaStencil& S = st_[b];
  for (int q = threadIdx.x; q < NU * NU; q += blockDim.x) {
#pragma unroll
    for (int z = 0; z < 5; ++z) blk[z * NU * NU + q] = S.blk[z][q];
    blk[5 * NU * NU + q] = S.St[q];
    blk[6 * NU * NU + q] = S.Ss[q];
  }
  __syncthreads();
  const int nc = L.nx * L.ny;
  const int64_t vo = L.cell_off * NU;
  for (int cell = blockIdx.x * blockDim.x + threadIdx.x; cell < nc; cell += gridDim.x * blockDim.x) {
    const int i = cell % L.nx, k = cell / L.nx;
    if (mode == 2 && ((i + k) & 1) != color) continue;
    const double t = st[L.cell_off + cell], u = ss[L.cell_off + cell];
    double acc[NU], xc[NU];
#pragma unroll
    for (int r = 0; r < NU; ++r) xc[r] = x[vo + (int64_t)r * nc + cell];
#pragma unroll
    for (int r = 0; r < NU; ++r) {
      double a = 0.0;
#pragma unroll
      for (int c = 0; c < NU; ++c)
        a += (blk[r * NU + c] + t * blk[5 * NU * NU + r * NU + c] + u * blk[6 * NU * NU + r * NU + c]) * xc[c];
      acc[r] = a;
    }
    const int nb[4] = {i > 0 ? cell - 1 : -1, i < L.nx - 1 ? cell + 1 : -1,
                       k > 0 ? cell - L.nx : -1, k < L.ny - 1 ? cell + L.nx : -1};
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      if (nb[z] < 0) continue;
      double xn[NU];
#pragma unroll
      for (int c = 0; c < NU; ++c) xn[c] = x[vo + (int64_t)c * nc + nb[z]];
      const double* B = blk + (z + 1) * NU * NU;
#pragma unroll
      for (int r = 0; r < NU; ++r) {
        double a = 0.0;
#pragma unroll
        for (int c = 0; c < NU; ++c) a += B[r * NU + c] * xn[c];
        acc[r] += a;
      }
    }
    if (mode == 0) {
#pragma unroll
      for (int r = 0; r < NU; ++r) y[vo + (int64_t)r * nc + cell] = acc[r];
    } else if (mode == 1) {
#pragma unroll
      for (int r = 0; r < NU; ++r)
        y[vo + (int64_t)r * nc + cell] = bvec[vo + (int64_t)r * nc + cell] - acc[r];
    } else {
      const int rg = per_cell_inv ? 0 : region0[insts[b].region_off + cell];
      const double* M = inv + (int64_t)lvl_inv_index(per_cell_inv, L.cell_off + cell, b, max_regions, rg) * NU * NU;
      double res[NU];
#pragma unroll
      for (int r = 0; r < NU; ++r) res[r] = bvec[vo + (int64_t)r * nc + cell] - acc[r];
#pragma unroll
      for (int r = 0; r < NU; ++r) {
        double a = 0.0;
#pragma unroll
        for (int c = 0; c < NU; ++c) a += M[r * NU + c] * res[c];
        x[vo + (int64_t)r * nc + cell] = xc[r] + a;
      }
    }
  }
}

// Structured apply for reflection-symmetric rules.  Along one axis, with
// R = (1, sqrt3), L = (1, -sqrt3) the end traces (times sqrt h):
//   D_C: own sqrt3/h [[0, 1], [-1, 0]], upper neighbour R L^T/(2h), lower -L R^T/(2h)
//   D_J: own -diag(2, 6)/h,          upper neighbour R L^T/h,    lower  L R^T/h,
// so with P = R (L.x_up)/h and Q = L (R.x_lo)/h:
//   D_C x = S_C x + (P - Q)/2,  D_J x = S_J x + P + Q.
// Absent neighbours are passed as zeros (no coupling across the boundary).
template <typename real>
__device__ __forceinline__ void axis_cj(const real Xc[4], const real Xhi[4], const real Xlo[4], int axis,
                                        real ih, real C[4], real J[4]) {
  const real r3 = (real)1.7320508075688772935;
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int i0 = axis == 0 ? 2 * g : g;
    const int i1 = axis == 0 ? 2 * g + 1 : g + 2;
    const real dl = (Xhi[i0] - r3 * Xhi[i1]) * ih;
    const real dr = (Xlo[i0] + r3 * Xlo[i1]) * ih;
    C[i0] = r3 * ih * Xc[i1] + (real)0.5 * (dl - dr);
    C[i1] = -r3 * ih * Xc[i0] + (real)0.5 * r3 * (dl + dr);
    J[i0] = (real)-2 * ih * Xc[i0] + dl + dr;
    J[i1] = (real)-6 * ih * Xc[i1] + r3 * (dl - dr);
  }
}

// The scalars of the structured form (one set per instance and level).
template <typename real>
struct SymCoef {
  real ax, ay, bex, bey, cxx, cxy, cyx, cyy, ihx, ihy;
  real kxx, kxy, kyx, kyy;  // the block solves' jump coefficients (FC)
};

template <typename real>
__device__ __forceinline__ SymCoef<real> sym_coef(const DsaStencil& G) {
  SymCoef<real> c;
  c.ax = (real)G.ax; c.ay = (real)G.ay; c.bex = (real)G.bex; c.bey = (real)G.bey;
  c.cxx = (real)G.cxx; c.cxy = (real)G.cxy; c.cyx = (real)G.cyx; c.cyy = (real)G.cyy;
  c.ihx = (real)(1.0 / G.hx); c.ihy = (real)(1.0 / G.hy);
  c.kxx = (real)G.bcxx; c.kxy = (real)G.bcxy; c.kyx = (real)G.bcyx; c.kyy = (real)G.bcyy;
  return c;
}

// A cell of an instance's level grid and which neighbours it has.
struct CellPos {
  int cell, nx;
  int64_t nc;
  bool hl, hr, hb, ht;
};

__device__ __forceinline__ CellPos cell_pos(int i, int k, int nx, int ny) {
  CellPos p;
  p.cell = k * nx + i;
  p.nx = nx;
  p.nc = (int64_t)nx * ny;
  p.hl = i > 0;
  p.hr = i < nx - 1;
  p.hb = k > 0;
  p.ht = k < ny - 1;
  return p;
}

// Field f (4 unknowns) of a cell and of its four neighbours (zeros where
// absent; the cell's own values are zeros too unless OWN).  An absent
// neighbour reads the cell itself and the value is then replaced by zero:
// with no branch around a load, the loads issue back to back and are waited
// for once instead of one at a time.
template <typename real, bool OWN = true>
__device__ __forceinline__ void load_field(const real* __restrict__ x, const CellPos& P, int f, real c[4],
                                           real l[4], real r[4], real b[4], real t[4]) {
  const int ol = P.hl ? -1 : 0, orr = P.hr ? 1 : 0, ob = P.hb ? -P.nx : 0, ot = P.ht ? P.nx : 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const real* q = x + (int64_t)(4 * f + m) * P.nc + P.cell;
    const real vl = q[ol], vr = q[orr], vb = q[ob], vt = q[ot];
    c[m] = OWN ? q[0] : (real)0;
    l[m] = P.hl ? vl : (real)0;
    r[m] = P.hr ? vr : (real)0;
    b[m] = P.hb ? vb : (real)0;
    t[m] = P.ht ? vt : (real)0;
  }
}

// y = K x for one cell (12 unknowns: phi, J_x, J_y), reflection-symmetric rule,
// one field at a time to keep few values live.  !OWN: the cell's own values
// are taken as zero (the neighbour coupling only).
template <typename real, bool OWN = true>
__device__ __forceinline__ void sym_cell_apply(const SymCoef<real>& S, real st, real ss,
                                               const real* __restrict__ x, const CellPos& P, real y[12]) {
  real c[4], l[4], r[4], b[4], t[4], Cx[4], Jx[4], Cy[4], Jy[4];
  // phi: its own row, and the J rows' D_C phi terms
  load_field<real, OWN>(x, P, 0, c, l, r, b, t);
  axis_cj(c, r, l, 0, S.ihx, Cx, Jx);
  axis_cj(c, t, b, 1, S.ihy, Cy, Jy);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    y[m] = (st - ss) * c[m] - S.bex * Jx[m] - S.bey * Jy[m];
    y[4 + m] = S.ax * Cx[m];
    y[8 + m] = S.ay * Cy[m];
  }
  // J_x: D_C^x J_x into the phi row; sigma_t, D_J^x, D_J^y into its own row
  load_field<real, OWN>(x, P, 1, c, l, r, b, t);
  axis_cj(c, r, l, 0, S.ihx, Cx, Jx);
  axis_cj(c, t, b, 1, S.ihy, Cy, Jy);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    y[m] += (real)3 * S.ax * Cx[m];
    y[4 + m] += (real)3 * S.ax * st * c[m] - (real)1.5 * (S.cxx * Jx[m] + S.cxy * Jy[m]);
  }
  // J_y likewise
  load_field<real, OWN>(x, P, 2, c, l, r, b, t);
  axis_cj(c, r, l, 0, S.ihx, Cx, Jx);
  axis_cj(c, t, b, 1, S.ihy, Cy, Jy);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    y[m] += (real)3 * S.ay * Cy[m];
    y[8 + m] += (real)3 * S.ay * st * c[m] - (real)1.5 * (S.cyx * Jx[m] + S.cyy * Jy[m]);
  }
}

// Reciprocal for the block solves: the hardware approximation (1 ulp) in
// FP32, where the hierarchy only preconditions; a correctly rounded division
// in FP64.
__device__ __forceinline__ float blk_inv(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double blk_inv(double v) { return 1.0 / v; }

// Exact solve with the cell's diagonal block for a reflection-symmetric rule
// (the FC block: jump coefficients kxx..kyy).
// The own-cell parts are: phi row diagonal Dphi, J rows diagonal dJx, dJy, and
// the skew couplings a_xx S_x, a_yy S_y (S = sqrt3/h [[0,1],[-1,0]] along its
// axis).  Eliminating J_x, J_y leaves a diagonal Schur complement because
// S dJ^{-1} S is diagonal:
//   (Dphi + 3 a_xx^2 s_x^2 / dJx[1-p, q] + 3 a_yy^2 s_y^2 / dJy[p, 1-q]) phi
//       = r_phi - 3 a_xx S_x dJx^{-1} r_Jx - 3 a_yy S_y dJy^{-1} r_Jy.
template <typename real>
__device__ __forceinline__ void sym_block_solve(const SymCoef<real>& S, real st, real ss, const real r[12],
                                                real out[12]) {
  const real r3 = (real)1.7320508075688772935;
  const real sx = r3 * S.ihx, sy = r3 * S.ihy;
  real dphi[4], ijx[4], ijy[4], tx[4], ty[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const int p = l & 1, q = l >> 1;
    const real gx = (real)(p ? 6 : 2) * S.ihx, gy = (real)(q ? 6 : 2) * S.ihy;
    dphi[l] = (st - ss) + S.bex * gx + S.bey * gy;
    ijx[l] = blk_inv((real)3 * S.ax * st + (real)1.5 * (S.kxx * gx + S.kxy * gy));  // 1 / dJx
    ijy[l] = blk_inv((real)3 * S.ay * st + (real)1.5 * (S.kyx * gx + S.kyy * gy));
    tx[l] = r[4 + l] * ijx[l];  // dJx^{-1} r_Jx
    ty[l] = r[8 + l] * ijy[l];
  }
  // S_x acts on p: (S u)[0,q] = s u[1,q], (S u)[1,q] = -s u[0,q]; S_y likewise on q
  const real ax3 = (real)3 * S.ax * sx, ay3 = (real)3 * S.ay * sy;
  real rhs[4];
  rhs[0] = r[0] - ax3 * tx[1] - ay3 * ty[2];
  rhs[1] = r[1] + ax3 * tx[0] - ay3 * ty[3];
  rhs[2] = r[2] - ax3 * tx[3] + ay3 * ty[0];
  rhs[3] = r[3] + ax3 * tx[2] + ay3 * ty[1];
  const real kx = (real)3 * S.ax * S.ax * sx * sx, ky = (real)3 * S.ay * S.ay * sy * sy;
  out[0] = rhs[0] * blk_inv(dphi[0] + kx * ijx[1] + ky * ijy[2]);  // (1-p, q) and (p, 1-q) partners
  out[1] = rhs[1] * blk_inv(dphi[1] + kx * ijx[0] + ky * ijy[3]);
  out[2] = rhs[2] * blk_inv(dphi[2] + kx * ijx[3] + ky * ijy[0]);
  out[3] = rhs[3] * blk_inv(dphi[3] + kx * ijx[2] + ky * ijy[1]);
  // J = dJ^{-1} (r_J - a S phi)
  const real axs = S.ax * sx, ays = S.ay * sy;
  out[4] = (r[4] - axs * out[1]) * ijx[0];
  out[5] = (r[5] + axs * out[0]) * ijx[1];
  out[6] = (r[6] - axs * out[3]) * ijx[2];
  out[7] = (r[7] + axs * out[2]) * ijx[3];
  out[8] = (r[8] - ays * out[2]) * ijy[0];
  out[9] = (r[9] - ays * out[3]) * ijy[1];
  out[10] = (r[10] + ays * out[0]) * ijy[2];
  out[11] = (r[11] + ays * out[1]) * ijy[3];
}

// Red-black index: work item t of colour `color` -> (i, k), for even nx
// (nx / 2 cells of each colour per row).
__device__ __forceinline__ void rb_cell(int t, int nx, int color, int& i, int& k) {
  const int h = nx >> 1;
  k = t / h;
  i = 2 * (t - k * h) + ((k + color) & 1);
}

// mode 0: y = K x; mode 1: y = b - K x;
// mode 2 (colour c): x_c += D_c^{-1} (b - K x)_c on cells with (i + k) % 2 == c;
// mode 3: the first colour-0 half sweep from x = 0: x = D^{-1} b on colour 0,
//         reading no x; colour 1 is left unwritten for mode 4;
// mode 4: the colour-1 half sweep that follows mode 3: x = D^{-1} (b - K x) on
//         colour 1 with its own x taken as zero (only colour 0 is read).
// vsrc (modes 3 and 4 on level 0 only, nullable): b is formed from the DG
// vector v as [ss v, m_x ss v, m_y ss v] instead of read, and mode 3 stores
// its colour-0 part in bout for the restriction that follows (the scalar-flux
// field only: with a reflection-symmetric rule m_x = m_y = 0, so the
// current fields of b vanish).
template <typename real>
__global__ void __launch_bounds__(256) k_mg_stencil_sym(int mode, int color, const LvlInst* __restrict__ li,
                                 const DsaStencil* __restrict__ st_, const double* __restrict__ st,
                                 const double* __restrict__ ss, const real* __restrict__ bvec,
                                 real* __restrict__ x, real* __restrict__ y,
                                 const int32_t* __restrict__ active,
                                 const double* __restrict__ vsrc = nullptr,
                                 const InstDev* __restrict__ insts = nullptr, real* __restrict__ bout = nullptr) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const LvlInst L = li[b];
  const SymCoef<real> S = sym_coef<real>(st_[b]);
  const double* __restrict__ vb = vsrc ? vsrc + insts[b].dof_off : nullptr;
  const double mxr = st_[b].m[0], myr = st_[b].m[1];
  const int nx = L.nx, ny = L.ny, nc = nx * ny;
  const int64_t vo = L.cell_off * 12;
  const real* __restrict__ bb = bvec ? bvec + vo : nullptr;
  real* __restrict__ xb = x + vo;
  const bool half = mode >= 2;  // one colour per launch
  const bool compact = half && (nx & 1) == 0;
  const int nwork = compact ? nc / 2 : nc;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nwork; t += gridDim.x * blockDim.x) {
    int i, k;
    if (compact) {
      rb_cell(t, nx, color, i, k);
    } else {
      i = t % nx;
      k = t / nx;
      if (half && ((i + k) & 1) != color) continue;
    }
    const CellPos P = cell_pos(i, k, nx, ny);
    const real tt = (real)st[L.cell_off + P.cell], uu = (real)ss[L.cell_off + P.cell];
    real r[12];
    if (vb && mode >= 3) {
      const double sd = ss[L.cell_off + P.cell];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const double sv = sd * vb[4 * P.cell + m];
        r[m] = (real)sv;
        r[4 + m] = (real)(mxr * sv);
        r[8 + m] = (real)(myr * sv);
      }
      if (mode == 3 && bout) {
        real* __restrict__ bo = bout + vo;
#pragma unroll
        for (int q = 0; q < 4; ++q) bo[(int64_t)q * nc + P.cell] = r[q];
      }
    } else if (mode >= 3) {
#pragma unroll
      for (int q = 0; q < 12; ++q) r[q] = bb[(int64_t)q * nc + P.cell];
    }
    if (mode == 3) {
      real d[12];
      sym_block_solve(S, tt, uu, r, d);
#pragma unroll
      for (int q = 0; q < 12; ++q) xb[(int64_t)q * nc + P.cell] = d[q];
      continue;
    }
    real yy[12];
    if (mode == 4) {
      sym_cell_apply<real, false>(S, tt, uu, xb, P, yy);
      real d[12];
#pragma unroll
      for (int q = 0; q < 12; ++q) r[q] -= yy[q];
      sym_block_solve(S, tt, uu, r, d);
#pragma unroll
      for (int q = 0; q < 12; ++q) xb[(int64_t)q * nc + P.cell] = d[q];
      continue;
    }
    sym_cell_apply(S, tt, uu, xb, P, yy);
    if (mode == 0) {
#pragma unroll
      for (int q = 0; q < 12; ++q) y[vo + (int64_t)q * nc + P.cell] = yy[q];
    } else if (mode == 1) {
#pragma unroll
      for (int q = 0; q < 12; ++q) y[vo + (int64_t)q * nc + P.cell] = bb[(int64_t)q * nc + P.cell] - yy[q];
    } else {
      real r[12], d[12];
#pragma unroll
      for (int q = 0; q < 12; ++q) r[q] = bb[(int64_t)q * nc + P.cell] - yy[q];
      sym_block_solve(S, tt, uu, r, d);
#pragma unroll
      for (int q = 0; q < 12; ++q) xb[(int64_t)q * nc + P.cell] += d[q];
    }
  }
}

// Coarsest level: `sweeps` red-black Gauss-Seidel sweeps from x = 0 in one
// launch, one work group per instance.
template <typename real>
__global__ void __launch_bounds__(256) k_mg_coarse_sym(int sweeps, const LvlInst* __restrict__ li,
                                const DsaStencil* __restrict__ st_, const double* __restrict__ st,
                                const double* __restrict__ ss, const real* __restrict__ bvec,
                                real* __restrict__ x, const int32_t* __restrict__ active) {
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  const LvlInst L = li[b];
  const SymCoef<real> S = sym_coef<real>(st_[b]);
  const int nx = L.nx, ny = L.ny, nc = nx * ny;
  const int64_t vo = L.cell_off * 12;
  const real* __restrict__ bb = bvec + vo;
  real* __restrict__ xb = x + vo;
  for (int e = threadIdx.x; e < nc * 12; e += blockDim.x) xb[e] = (real)0;
  __syncthreads();
  for (int sw = 0; sw < sweeps; ++sw)
    for (int color = 0; color < 2; ++color) {
      for (int cell = threadIdx.x; cell < nc; cell += blockDim.x) {
        const int i = cell % nx, k = cell / nx;
        if (((i + k) & 1) != color) continue;
        const CellPos P = cell_pos(i, k, nx, ny);
        const real tt = (real)st[L.cell_off + cell], uu = (real)ss[L.cell_off + cell];
        real yy[12], r[12], d[12];
        sym_cell_apply(S, tt, uu, xb, P, yy);
#pragma unroll
        for (int q = 0; q < 12; ++q) r[q] = bb[(int64_t)q * nc + cell] - yy[q];
        sym_block_solve(S, tt, uu, r, d);
#pragma unroll
        for (int q = 0; q < 12; ++q) xb[(int64_t)q * nc + cell] += d[q];
      }
      __syncthreads();
    }
}

// Degree-1 Legendre injection of a coarse cell's modes into child `side`
// (0 = low half, 1 = high half), [child mode][coarse mode].
__device__ __forceinline__ double inj1d(int side, int p, int P) {
  const double s2 = 1.4142135623730950488, r3 = 1.7320508075688772935;
  if (p == 0) return P == 0 ? 1.0 / s2 : (side ? r3 / (2.0 * s2) : -r3 / (2.0 * s2));
  return P == 0 ? 0.0 : 1.0 / (2.0 * s2);
}

// mode 0: restrict  bc[C] = sum_children P_f^T rf[f]
// mode 1: prolong   xf[f] += P_f xc[C]
template <int NU, typename real>
__global__ void k_mg_transfer(int mode, const LvlInst* __restrict__ lf, const LvlInst* __restrict__ lc,
                              const real* __restrict__ fine_in, real* __restrict__ fine_out,
                              const real* __restrict__ coarse_in, real* __restrict__ coarse_out,
                              const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const LvlInst F = lf[b], Cc = lc[b];
  const int nl = F.nloc;
  const int nf = NU / nl;  // fields
  const int nc = Cc.nx * Cc.ny;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    const int I = c % Cc.nx, K = c / Cc.nx;
    real acc[NU];
    if (mode == 0)
      for (int r = 0; r < NU; ++r) acc[r] = (real)0;
    else
      for (int r = 0; r < NU; ++r) acc[r] = coarse_in[Cc.cell_off * NU + (int64_t)r * nc + c];
    for (int dk = 0; dk < (F.dim == 2 ? 2 : 1); ++dk)
      for (int di = 0; di < 2; ++di) {
        const int f = (F.dim == 2 ? (2 * K + dk) * F.nx : 0) + 2 * I + di;
        const int64_t fo = F.cell_off * NU + f, nfc = (int64_t)F.nx * F.ny;
        for (int fld = 0; fld < nf; ++fld)
          for (int l = 0; l < nl; ++l) {      // child mode (p + 2q)
            const int p = l & 1, q = l >> 1;
            if (mode == 0) {
              const real rv = fine_in[fo + (fld * nl + l) * nfc];
              for (int L2 = 0; L2 < nl; ++L2) {  // coarse mode
                const int P = L2 & 1, Q = L2 >> 1;
                const real w = (real)(inj1d(di, p, P) * (F.dim == 2 ? inj1d(dk, q, Q) : 1.0));
                acc[fld * nl + L2] += w * rv;
              }
            } else {
              real v = (real)0;
              for (int L2 = 0; L2 < nl; ++L2) {
                const int P = L2 & 1, Q = L2 >> 1;
                const real w = (real)(inj1d(di, p, P) * (F.dim == 2 ? inj1d(dk, q, Q) : 1.0));
                v += w * acc[fld * nl + L2];
              }
              fine_out[fo + (fld * nl + l) * nfc] += v;
            }
          }
      }
    if (mode == 0)
      for (int r = 0; r < NU; ++r) coarse_out[Cc.cell_off * NU + (int64_t)r * nc + c] = acc[r];
  }
}

// z = v + (x + P x_c) on the scalar-flux unknowns (field 0) of level 0, X-Y:
// for a single V-cycle without post-smoothing on level 0 the prolongation of
// the coarse correction and the output pass are one (the current unknowns of
// level 0 are never needed).
__global__ void k_dsa_out_prolong(const InstDev* __restrict__ insts, const LvlInst* __restrict__ lf,
                                  const LvlInst* __restrict__ lc, const float* __restrict__ xf,
                                  const float* __restrict__ xc, const double* __restrict__ v,
                                  double* __restrict__ z, const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const InstDev I = insts[b];
  const LvlInst F = lf[b], Cc = lc[b];
  const int nfc = F.nx * F.ny, ncc = Cc.nx * Cc.ny;
  const float* __restrict__ xb = xf + F.cell_off * 12;
  const float* __restrict__ cb = xc + Cc.cell_off * 12;
  // one cell (its 4 DoFs, contiguous in v and z) per thread
  for (int cell = blockIdx.x * blockDim.x + threadIdx.x; cell < nfc; cell += gridDim.x * blockDim.x) {
    const int i = cell % F.nx, k = cell / F.nx;
    const int parent = (k >> 1) * Cc.nx + (i >> 1);
    float xc[4];
#pragma unroll
    for (int L2 = 0; L2 < 4; ++L2) xc[L2] = cb[L2 * ncc + parent];
    const double2* vp = reinterpret_cast<const double2*>(v + I.dof_off + 4 * (int64_t)cell);
    double2* zp = reinterpret_cast<double2*>(z + I.dof_off + 4 * (int64_t)cell);
    double out[4];
    const double2 v01 = vp[0], v23 = vp[1];
    const double vv[4] = {v01.x, v01.y, v23.x, v23.y};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      float corr = 0.f;
#pragma unroll
      for (int L2 = 0; L2 < 4; ++L2)
        corr += (float)(inj1d(i & 1, m & 1, L2 & 1) * inj1d(k & 1, m >> 1, L2 >> 1)) * xc[L2];
      out[m] = vv[m] + (double)(xb[m * nfc + cell] + corr);
    }
    double2 o01, o23;
    o01.x = out[0];
    o01.y = out[1];
    o23.x = out[2];
    o23.y = out[3];
    zp[0] = o01;
    zp[1] = o23;
  }
}

// The finest level's part of the FP32 V-cycle of one DSA application
// (reflection-symmetric rules, one from-zero sweep), in one pass over tiles
// of FF_T x FF_T cells: b = [sigma_s v, 0, 0] (the rule's first moments are
// zero), the colour-0 half sweep x = D^{-1} b on the tile and a two-cell halo,
// the colour-1 half sweep x = D^{-1} (b - K x) on the tile and a one-cell halo,
// then the residual of the tile's colour-0 cells (colour 1 has none after its
// half sweep) restricted into the coarse b, and the scalar-flux field of x
// for the output pass.  The same values as the separate half sweeps and the
// residual-restriction pass, with x and b kept in LDS instead of HBM.
constexpr int FF_T = 24;
constexpr int FF_W = FF_T + 4;  // even: each local row holds FF_W / 2 cells of each colour
constexpr int FF_N = FF_W * FF_W;

__global__ void __launch_bounds__(512) k_mg_fine_fused(const LvlInst* __restrict__ lf, const LvlInst* __restrict__ lc,
                                                       const DsaStencil* __restrict__ st_f,
                                                       const double* __restrict__ st, const double* __restrict__ ss,
                                                       const InstDev* __restrict__ insts, const double* __restrict__ v,
                                                       float* __restrict__ xphi, float* __restrict__ coarse_b,
                                                       const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const LvlInst F = lf[b], Cc = lc[b];
  const int nx = F.nx, ny = F.ny, nfc = nx * ny;
  const int tiles_x = (nx + FF_T - 1) / FF_T, tiles_y = (ny + FF_T - 1) / FF_T;
  if ((int)blockIdx.x >= tiles_x * tiles_y) return;
  const int ox = ((int)blockIdx.x % tiles_x) * FF_T, oy = ((int)blockIdx.x / tiles_x) * FF_T;
  const int tw = min(FF_T, nx - ox), th = min(FF_T, ny - oy);  // even: the grid coarsens
  const SymCoef<float> S = sym_coef<float>(st_f[b]);
  __shared__ float lx[12 * FF_N];  // x on the tile and its halo, [field mode][local cell]
  __shared__ float lb[4 * FF_N];   // scalar-flux field of b
  __shared__ float lsg[2 * FF_N];  // sigma_t, sigma_s
  const double* __restrict__ vb = v + insts[b].dof_off;
  // local cell e <-> grid cell (ox - 2 + e % FF_W, oy - 2 + e / FF_W)
  auto lpos = [&](int i, int k) {
    CellPos p;
    p.cell = (i - ox + 2) + FF_W * (k - oy + 2);
    p.nx = FF_W;
    p.nc = FF_N;
    p.hl = i > 0;
    p.hr = i < nx - 1;
    p.hb = k > 0;
    p.ht = k < ny - 1;
    return p;
  };
  for (int e = threadIdx.x; e < FF_N; e += blockDim.x) {
    const int i = ox - 2 + e % FF_W, k = oy - 2 + e / FF_W;
    if (i < 0 || i >= nx || k < 0 || k >= ny) continue;
    const int cell = k * nx + i;
    const double sd = ss[F.cell_off + cell];
    lsg[e] = (float)st[F.cell_off + cell];
    lsg[FF_N + e] = (float)sd;
#pragma unroll
    for (int m = 0; m < 4; ++m) lb[m * FF_N + e] = (float)(sd * vb[4 * cell + m]);
  }
  __syncthreads();
  // the half sweeps take one colour's local cells only (tile origins are even,
  // so a local cell's colour is that of its local coordinates)
  for (int t = threadIdx.x; t < FF_N / 2; t += blockDim.x) {  // colour 0, halo 2
    const int lk = t / (FF_W / 2), li = 2 * (t % (FF_W / 2)) + (lk & 1);
    const int e = lk * FF_W + li;
    const int i = ox - 2 + li, k = oy - 2 + lk;
    if (i < 0 || i >= nx || k < 0 || k >= ny) continue;
    float r[12], d[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) r[q] = q < 4 ? lb[q * FF_N + e] : 0.f;
    sym_block_solve(S, lsg[e], lsg[FF_N + e], r, d);
#pragma unroll
    for (int q = 0; q < 12; ++q) lx[q * FF_N + e] = d[q];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < FF_N / 2; t += blockDim.x) {  // colour 1, halo 1
    const int lk = t / (FF_W / 2), li = 2 * (t % (FF_W / 2)) + ((lk + 1) & 1);
    const int e = lk * FF_W + li;
    const int i = ox - 2 + li, k = oy - 2 + lk;
    if (li < 1 || li > FF_W - 2 || lk < 1 || lk > FF_W - 2) continue;
    if (i < 0 || i >= nx || k < 0 || k >= ny) continue;
    const CellPos P = lpos(i, k);
    float yy[12], r[12], d[12];
    sym_cell_apply<float, false>(S, lsg[e], lsg[FF_N + e], lx, P, yy);
#pragma unroll
    for (int q = 0; q < 12; ++q) r[q] = (q < 4 ? lb[q * FF_N + e] : 0.f) - yy[q];
    sym_block_solve(S, lsg[e], lsg[FF_N + e], r, d);
#pragma unroll
    for (int q = 0; q < 12; ++q) lx[q * FF_N + e] = d[q];
  }
  __syncthreads();
  const int ncc = Cc.nx * Cc.ny;
  const int cw = tw / 2, ch_ = th / 2;
  for (int c = threadIdx.x; c < cw * ch_; c += blockDim.x) {  // the tile's coarse cells
    const int I = ox / 2 + c % cw, K = oy / 2 + c / cw;
    float acc[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = 0.f;
#pragma unroll 1
    for (int ch = 0; ch < 4; ch += 3) {  // the colour-0 children (0, 0) and (1, 1)
      const int di = ch & 1, dk = ch >> 1;
      const CellPos P = lpos(2 * I + di, 2 * K + dk);
      const int e = P.cell;
      float yy[12];
      sym_cell_apply(S, lsg[e], lsg[FF_N + e], lx, P, yy);
#pragma unroll
      for (int fld = 0; fld < 3; ++fld)
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          const float bq = fld == 0 ? lb[l * FF_N + e] : 0.f;
          const float rv = bq - yy[4 * fld + l];
          const int p = l & 1, q = l >> 1;
#pragma unroll
          for (int L2 = 0; L2 < 4; ++L2)
            acc[4 * fld + L2] += (float)(inj1d(di, p, L2 & 1) * inj1d(dk, q, L2 >> 1)) * rv;
        }
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) coarse_b[Cc.cell_off * 12 + (int64_t)q * ncc + K * Cc.nx + I] = acc[q];
  }
  float* __restrict__ xo = xphi + F.cell_off * 12;
  for (int e = threadIdx.x; e < tw * th; e += blockDim.x) {  // scalar-flux field of x on the tile
    const int i = ox + e % tw, k = oy + e / tw;
    const int l = (i - ox + 2) + FF_W * (k - oy + 2);
#pragma unroll
    for (int m = 0; m < 4; ++m) xo[(int64_t)m * nfc + k * nx + i] = lx[m * FF_N + l];
  }
}

// Residual and restriction in one pass (reflection-symmetric rules): each
// coarse cell forms b - K x on its 2 x 2 children and accumulates P_f^T of it.
// After a red-black half sweep of colour 1 the residual of every colour-1 cell
// is zero (its neighbours all have colour 0 and did not change since), so with
// zero_c1 only the two colour-0 children, (0, 0) and (1, 1), are formed.
// bphi: only the scalar-flux field of b is stored (its current fields are
// zero; the fine right-hand side formed from v with a reflection-symmetric
// rule).
template <typename real>
__global__ void __launch_bounds__(256) k_mg_resrestrict_sym(const LvlInst* __restrict__ lf, const LvlInst* __restrict__ lc,
                                     const DsaStencil* __restrict__ st_f, const double* __restrict__ st,
                                     const double* __restrict__ ss, const real* __restrict__ bvec,
                                     const real* __restrict__ x, real* __restrict__ coarse_b, int zero_c1,
                                     const int32_t* __restrict__ active, int bphi = 0) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const LvlInst F = lf[b], Cc = lc[b];
  const SymCoef<real> S = sym_coef<real>(st_f[b]);
  const int nfx = F.nx, nfy = F.ny, nfc = nfx * nfy, ncc = Cc.nx * Cc.ny;
  const int64_t vf = F.cell_off * 12;
  const real* __restrict__ xb = x + vf;
  const real* __restrict__ bb = bvec + vf;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncc; c += gridDim.x * blockDim.x) {
    const int I = c % Cc.nx, K = c / Cc.nx;
    real acc[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = (real)0;
#pragma unroll 1
    for (int ch = 0; ch < 4; ch += zero_c1 ? 3 : 1) {  // children one at a time keeps few values live
        const int di = ch & 1, dk = ch >> 1;
        const int i = 2 * I + di, k = 2 * K + dk;
        const CellPos P = cell_pos(i, k, nfx, nfy);
        real yy[12];
        sym_cell_apply(S, (real)st[F.cell_off + P.cell], (real)ss[F.cell_off + P.cell], xb, P, yy);
#pragma unroll
        for (int fld = 0; fld < 3; ++fld)
#pragma unroll
          for (int l = 0; l < 4; ++l) {
            const real bq = (bphi && fld > 0) ? (real)0 : bb[(int64_t)(4 * fld + l) * nfc + P.cell];
            const real rv = bq - yy[4 * fld + l];
            const int p = l & 1, q = l >> 1;
#pragma unroll
            for (int L2 = 0; L2 < 4; ++L2)
              acc[4 * fld + L2] += (real)(inj1d(di, p, L2 & 1) * inj1d(dk, q, L2 >> 1)) * rv;
          }
      }
#pragma unroll
    for (int q = 0; q < 12; ++q) coarse_b[Cc.cell_off * 12 + (int64_t)q * ncc + c] = acc[q];
  }
}

// ---------------------------------------------------------------- small levels
// The coarse end of the hierarchy (every level from `first` down) fits in LDS:
// one work group per instance runs that part of the V-cycle with each level's
// x and b in shared memory, replacing a chain of small launches.
constexpr int MG_TAIL_MAX = 10;
// threads of the tail's work group: a level of up to 32 x 32 cells updates one
// colour in one pass; FP64 keeps 256 for its larger register footprint
constexpr int MG_TAIL_THREADS_F32 = 512, MG_TAIL_THREADS_F64 = 256;

struct MgTailLevel {
  const LvlInst* li;
  const DsaStencil* st;
  const double* sigt;
  const double* sigs;
};

// One red-black half sweep of `color` on an LDS level: mode 0 updates x; mode
// 1 (colour 0, x = 0 beforehand) sets x = D^{-1} b and leaves colour 1
// unwritten; mode 2 (colour 1 after mode 1) sets x = D^{-1} (b - K x) with its
// own x taken as zero.
template <typename real, typename sreal>
__device__ __forceinline__ void tail_half_sweep(const SymCoef<real>& S, const LvlInst& L, const sreal* st, const sreal* ss,
                                const real* bv, real* x, int color, int mode) {
  const int nx = L.nx, ny = L.ny, nc = nx * ny;
  // even rows: the threads take only this colour's cells (nc / 2 of them)
  const bool compact = (nx & 1) == 0;
  const int nwork = compact ? nc / 2 : nc;
  const int stride = blockDim.x;
  // two cells per thread and pass, both read before either is written (cells
  // of one colour do not read each other), so that their loads overlap
  for (int t0 = threadIdx.x; t0 < nwork; t0 += 2 * stride) {
    bool on[2];
    int cellv[2];
    real d[2][12];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int t = t0 + j * stride;
      int i = 0, k = 0;
      on[j] = t < nwork;
      if (on[j]) {
        if (compact) {
          rb_cell(t, nx, color, i, k);
        } else {
          i = t % nx;
          k = t / nx;
          on[j] = ((i + k) & 1) == color;
        }
      }
      cellv[j] = k * nx + i;
      if (!on[j]) continue;
      const int cell = cellv[j];
      const CellPos P = cell_pos(i, k, nx, ny);
      const real tt = (real)st[cell], uu = (real)ss[cell];
      real r[12];
      if (mode == 1) {
#pragma unroll
        for (int q = 0; q < 12; ++q) r[q] = bv[q * nc + cell];
      } else {
        real yy[12];
        if (mode == 2)
          sym_cell_apply<real, false>(S, tt, uu, x, P, yy);
        else
          sym_cell_apply(S, tt, uu, x, P, yy);
#pragma unroll
        for (int q = 0; q < 12; ++q) r[q] = bv[q * nc + cell] - yy[q];
      }
      sym_block_solve(S, tt, uu, r, d[j]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (!on[j]) continue;
      const int cell = cellv[j];
#pragma unroll
      for (int q = 0; q < 12; ++q) x[q * nc + cell] = mode == 0 ? x[q * nc + cell] + d[j][q] : d[j][q];
    }
  }
  __syncthreads();
}

// A value from another lane of the same quad (aligned group of 4 lanes):
// quad_perm [1,0,3,2] (lane xor 1) or [2,3,0,1] (lane xor 2).  The lanes of a
// quad are active together wherever these are used.
template <int X>
__device__ __forceinline__ float quad_xor(float v) {
  constexpr int ctrl = X == 1 ? 0xB1 : 0x4E;
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xF, 0xF, true));
}
template <int X>
__device__ __forceinline__ double quad_xor(double v) {
  constexpr int ctrl = X == 1 ? 0xB1 : 0x4E;
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), ctrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), ctrl, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// One moment m of axis_cj's outputs: the lane's pair along the axis is
// (i0, i1) with m one of them (hi: i1 = m); xc, xh, xl: the pair's own, upper
// and lower neighbour values (x0 the i0 entry, x1 the i1 entry).  The same
// expressions as axis_cj.
template <typename real>
__device__ __forceinline__ void axis_cj_m(real xc0, real xc1, real xh0, real xh1, real xl0, real xl1, bool hi,
                                          real ih, real& C, real& J) {
  const real r3 = (real)1.7320508075688772935;
  const real dl = (xh0 - r3 * xh1) * ih;
  const real dr = (xl0 + r3 * xl1) * ih;
  if (!hi) {
    C = r3 * ih * xc1 + (real)0.5 * (dl - dr);
    J = (real)-2 * ih * xc0 + dl + dr;
  } else {
    C = -r3 * ih * xc0 + (real)0.5 * r3 * (dl + dr);
    J = (real)-6 * ih * xc1 + r3 * (dl - dr);
  }
}

// A red-black half sweep on a small LDS level (at most blockDim / 4 cells of
// the colour): four lanes per cell, lane m computing moment m of the three
// fields of the cell's apply and block solve (the partners of its moment
// along x and y, m ^ 1 and m ^ 2, exchanged within the quad), so a lane's
// chain of dependent operations is about a third of a whole cell's.  Modes
// and results as tail_half_sweep.
template <typename real>
__device__ __forceinline__ void tail_half_sweep_quad(const SymCoef<real>& S, const LvlInst& L, const real* st,
                                                     const real* ss, const real* bv, real* x, int color,
                                                     int mode) {
  const int nx = L.nx, ny = L.ny, nc = nx * ny;
  const bool compact = (nx & 1) == 0;
  const int nwork = compact ? nc / 2 : nc;
  const int m = threadIdx.x & 3, p = m & 1, q = m >> 1;
  const int mx = m ^ 1, my = m ^ 2;
  // the lane's pairs: along x (i0x, i1x) = (m & ~1, m | 1); along y
  // (i0y, i1y) = (m & 1, (m & 1) + 2)
  const int i0x = m & 2, i1x = (m & 2) | 1, i0y = p, i1y = p + 2;
  for (int t = threadIdx.x >> 2; t < nwork; t += blockDim.x >> 2) {
    int i = 0, k = 0;
    bool on = true;
    if (compact) {
      rb_cell(t, nx, color, i, k);
    } else {
      i = t % nx;
      k = t / nx;
      on = ((i + k) & 1) == color;
    }
    if (!on) continue;
    const int cell = k * nx + i;
    const CellPos P = cell_pos(i, k, nx, ny);
    const real tt = st[cell], uu = ss[cell];
    real r0, r1, r2;  // moment m of the residual's phi, J_x, J_y rows
    if (mode == 1) {
      r0 = bv[m * nc + cell];
      r1 = bv[(4 + m) * nc + cell];
      r2 = bv[(8 + m) * nc + cell];
    } else {
      const bool own = mode == 0;
      const int ol = P.hl ? -1 : 0, orr = P.hr ? 1 : 0, ob = P.hb ? -nx : 0, ot = P.ht ? nx : 0;
      real y0 = (real)0, y1 = (real)0, y2 = (real)0;
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        const real* xf = x + 4 * f * nc + cell;
        // own values (zero when !own) and the neighbours of the lane's pairs
        const real c_m = own ? xf[m * nc] : (real)0;
        const real cx0 = own ? xf[i0x * nc] : (real)0, cx1 = own ? xf[i1x * nc] : (real)0;
        const real cy0 = own ? xf[i0y * nc] : (real)0, cy1 = own ? xf[i1y * nc] : (real)0;
        const real rv0 = xf[i0x * nc + orr], rv1 = xf[i1x * nc + orr];
        const real lv0 = xf[i0x * nc + ol], lv1 = xf[i1x * nc + ol];
        const real tv0 = xf[i0y * nc + ot], tv1 = xf[i1y * nc + ot];
        const real bv0 = xf[i0y * nc + ob], bv1 = xf[i1y * nc + ob];
        real Cx, Jx, Cy, Jy;
        axis_cj_m(cx0, cx1, P.hr ? rv0 : (real)0, P.hr ? rv1 : (real)0, P.hl ? lv0 : (real)0,
                  P.hl ? lv1 : (real)0, p == 1, S.ihx, Cx, Jx);
        axis_cj_m(cy0, cy1, P.ht ? tv0 : (real)0, P.ht ? tv1 : (real)0, P.hb ? bv0 : (real)0,
                  P.hb ? bv1 : (real)0, q == 1, S.ihy, Cy, Jy);
        if (f == 0) {
          y0 = (tt - uu) * c_m - S.bex * Jx - S.bey * Jy;
          y1 = S.ax * Cx;
          y2 = S.ay * Cy;
        } else if (f == 1) {
          y0 += (real)3 * S.ax * Cx;
          y1 += (real)3 * S.ax * tt * c_m - (real)1.5 * (S.cxx * Jx + S.cxy * Jy);
        } else {
          y0 += (real)3 * S.ay * Cy;
          y2 += (real)3 * S.ay * tt * c_m - (real)1.5 * (S.cyx * Jx + S.cyy * Jy);
        }
      }
      r0 = bv[m * nc + cell] - y0;
      r1 = bv[(4 + m) * nc + cell] - y1;
      r2 = bv[(8 + m) * nc + cell] - y2;
    }
    // the block solve of sym_block_solve, moment m
    const real r3 = (real)1.7320508075688772935;
    const real sx = r3 * S.ihx, sy = r3 * S.ihy;
    const real gx = (real)(p ? 6 : 2) * S.ihx, gy = (real)(q ? 6 : 2) * S.ihy;
    const real dphi = (tt - uu) + S.bex * gx + S.bey * gy;
    const real ijx = blk_inv((real)3 * S.ax * tt + (real)1.5 * (S.kxx * gx + S.kxy * gy));
    const real ijy = blk_inv((real)3 * S.ay * tt + (real)1.5 * (S.kyx * gx + S.kyy * gy));
    const real tx = r1 * ijx, ty = r2 * ijy;
    const real tx_p = quad_xor<1>(tx), ijx_p = quad_xor<1>(ijx);
    const real ty_p = quad_xor<2>(ty), ijy_p = quad_xor<2>(ijy);
    const real ax3 = (real)3 * S.ax * sx, ay3 = (real)3 * S.ay * sy;
    real rhs = r0 + (p ? ax3 : -ax3) * tx_p;
    rhs = rhs + (q ? ay3 : -ay3) * ty_p;
    const real kx = (real)3 * S.ax * S.ax * sx * sx, ky = (real)3 * S.ay * S.ay * sy * sy;
    const real o0 = rhs * blk_inv(dphi + kx * ijx_p + ky * ijy_p);
    const real o0x = quad_xor<1>(o0), o0y = quad_xor<2>(o0);
    const real axs = S.ax * sx, ays = S.ay * sy;
    const real o1 = (r1 + (p ? axs : -axs) * o0x) * ijx;
    const real o2 = (r2 + (q ? ays : -ays) * o0y) * ijy;
    real* xm = x + m * nc + cell;
    if (mode == 0) {
      xm[0] += o0;
      xm[4 * nc] += o1;
      xm[8 * nc] += o2;
    } else {
      xm[0] = o0;
      xm[4 * nc] = o1;
      xm[8 * nc] = o2;
    }
  }
  __syncthreads();
}

// One red-black sweep of a tail level (colour 0, then colour 1); the first
// of a smoothing from x = 0 knows x = 0 beforehand in both half sweeps.
template <typename real, typename sreal>
__device__ __forceinline__ void tail_sweep(const SymCoef<real>& S, const LvlInst& L, const sreal* st,
                                           const sreal* ss, const real* bv, real* x, bool from_zero) {
  tail_half_sweep(S, L, st, ss, bv, x, 0, from_zero ? 1 : 0);
  tail_half_sweep(S, L, st, ss, bv, x, 1, from_zero ? 2 : 0);
}

// A half sweep of an LDS level: four lanes per cell where the colour has at
// most a quarter of the work group's threads in cells.
template <typename real>
__device__ __forceinline__ void tail_half_sweep_lds(const SymCoef<real>& S, const LvlInst& L, const real* st,
                                                    const real* ss, const real* bv, real* x, int color, int mode) {
  const int nc = L.nx * L.ny;
  const int nwork = (L.nx & 1) == 0 ? nc / 2 : nc;
  if (4 * nwork <= (int)blockDim.x)
    tail_half_sweep_quad(S, L, st, ss, bv, x, color, mode);
  else
    tail_half_sweep(S, L, st, ss, bv, x, color, mode);
}

template <typename real>
__device__ __forceinline__ void tail_sweep_lds(const SymCoef<real>& S, const LvlInst& L, const real* st,
                                               const real* ss, const real* bv, real* x, bool from_zero) {
  tail_half_sweep_lds(S, L, st, ss, bv, x, 0, from_zero ? 1 : 0);
  tail_half_sweep_lds(S, L, st, ss, bv, x, 1, from_zero ? 2 : 0);
}

// Residual of a tail level after a sweep that ended with colour 1 (so only
// the colour-0 children (0, 0) and (1, 1) have one), restricted into the next
// level's b.
template <typename real, typename sreal>
__device__ __forceinline__ void tail_restrict(const SymCoef<real>& S, const LvlInst& L, const LvlInst& C, const sreal* sgt,
                              const sreal* sgs, const real* x, const real* bv, real* bc) {
  const int nc = L.nx * L.ny, ncc = C.nx * C.ny;
  for (int c = threadIdx.x; c < ncc; c += blockDim.x) {
    const int I = c % C.nx, K = c / C.nx;
    real acc[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = (real)0;
#pragma unroll 1
    for (int ch = 0; ch < 4; ch += 3) {
      const int di = ch & 1, dk = ch >> 1;
      const CellPos P = cell_pos(2 * I + di, 2 * K + dk, L.nx, L.ny);
      real yy[12];
      sym_cell_apply(S, (real)sgt[P.cell], (real)sgs[P.cell], x, P, yy);
#pragma unroll
      for (int fld = 0; fld < 3; ++fld)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const real rv = bv[(4 * fld + m) * nc + P.cell] - yy[4 * fld + m];
#pragma unroll
          for (int L2 = 0; L2 < 4; ++L2)
            acc[4 * fld + L2] += (real)(inj1d(di, m & 1, L2 & 1) * inj1d(dk, m >> 1, L2 >> 1)) * rv;
        }
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) bc[q * ncc + c] = acc[q];
  }
  __syncthreads();
}

// x_dst = x_src + P xc on a tail level (x_src may be x_dst): the four
// children's values are read first, so their loads overlap.
template <typename real>
__device__ __forceinline__ void tail_prolong(const LvlInst& L, const LvlInst& C, const real* xc, const real* x_src, real* x_dst) {
  const int nc = L.nx * L.ny, ncc = C.nx * C.ny;
  for (int c = threadIdx.x; c < ncc; c += blockDim.x) {
    const int I = c % C.nx, K = c / C.nx;
    real xcv[12], xf[4][12];
#pragma unroll
    for (int q = 0; q < 12; ++q) xcv[q] = xc[q * ncc + c];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      const int f = (2 * K + (ch >> 1)) * L.nx + 2 * I + (ch & 1);
#pragma unroll
      for (int q = 0; q < 12; ++q) xf[ch][q] = x_src[q * nc + f];
    }
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      const int di = ch & 1, dk = ch >> 1;
      const int f = (2 * K + dk) * L.nx + 2 * I + di;
#pragma unroll
      for (int fld = 0; fld < 3; ++fld)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          real v = (real)0;
#pragma unroll
          for (int L2 = 0; L2 < 4; ++L2)
            v += (real)(inj1d(di, m & 1, L2 & 1) * inj1d(dk, m >> 1, L2 >> 1)) * xcv[4 * fld + L2];
          x_dst[(4 * fld + m) * nc + f] = xf[ch][4 * fld + m] + v;
        }
    }
  }
  __syncthreads();
}

// g0 = 0: every level's x, b and cross sections live in LDS ([x|b|sigma]
// per level); b_first is copied in and x_first receives the first level's x.
// g0 = 1: the first level is too large to sit in LDS next to the others.  Its
// b and cross sections are read from global memory (b_first, the level's
// FP64 arrays) and its x lives in LDS only while the coarser levels do not:
// LDS = [sigma of levels 1..][x of level 1][R], where R holds the first
// level's x during its smoothing and the coarser levels' b (and x from level
// 2 on) in between.  The first level's residual goes to level 1 through
// b1_scratch (global) and its x through x_first; it is smoothed nu0 times
// before and after the coarse correction.
// zout (nullable; the FP32 V-cycle whose tail starts at level 1): instead of
// storing the first level's x, the launch writes the DSA output z = v +
// (x_fine + P x) on the finest level's scalar-flux unknowns (x_fine: the
// finest level's scalar-flux field in xfine, v and z in the DG layout of
// insts), the pass the separate output kernel would make.
template <typename real, int NT>
__global__ void __launch_bounds__(NT) k_mg_tail_sym(const MgTailLevel* __restrict__ tl, int nlev, int nu_smooth,
                                                     int coarse_sweeps, const real* __restrict__ b_first,
                                                     real* __restrict__ x_first,
                                                     const int32_t* __restrict__ active, int g0, int nu0,
                                                     real* __restrict__ b1_scratch,
                                                     const InstDev* __restrict__ insts = nullptr,
                                                     const LvlInst* __restrict__ lf0 = nullptr,
                                                     const float* __restrict__ xfine = nullptr,
                                                     const double* __restrict__ vout = nullptr,
                                                     double* __restrict__ zout = nullptr) {
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  // every level's descriptor and stencil scalars, loaded once by one thread
  // per level (the phases below would otherwise each start with a chain of
  // dependent global loads)
  __shared__ LvlInst lvl[MG_TAIL_MAX];
  __shared__ SymCoef<real> scf[MG_TAIL_MAX];
  if ((int)threadIdx.x < nlev) {
    lvl[threadIdx.x] = tl[threadIdx.x].li[b];
    scf[threadIdx.x] = sym_coef<real>(tl[threadIdx.x].st[b]);
  }
  __syncthreads();
  extern __shared__ unsigned char smem_raw[];
  real* lds = reinterpret_cast<real*>(smem_raw);
  // per level: offsets of x, b and the cross sections in LDS (-1: not in LDS)
  __shared__ int xo[MG_TAIL_MAX], bo[MG_TAIL_MAX], so[MG_TAIL_MAX], r_off;
  if (threadIdx.x == 0) {
    if (!g0) {
      int o = 0;
      for (int l = 0; l < nlev; ++l) {
        const LvlInst Li = lvl[l];
        const int nc = Li.nx * Li.ny;
        xo[l] = o;
        bo[l] = o + 12 * nc;
        so[l] = o + 24 * nc;
        o += 26 * nc;
      }
      r_off = 0;
    } else {
      int o = 0;
      for (int l = 1; l < nlev; ++l) {
        const LvlInst Li = lvl[l];
        so[l] = o;
        o += 2 * Li.nx * Li.ny;
      }
      const LvlInst L1 = lvl[1];
      xo[1] = o;
      o += 12 * L1.nx * L1.ny;
      r_off = o;  // R: the first level's x, later the coarser levels' b and x
      for (int l = 1; l < nlev; ++l) {
        const LvlInst Li = lvl[l];
        const int nc = Li.nx * Li.ny;
        bo[l] = o;
        o += 12 * nc;
        if (l >= 2) {
          xo[l] = o;
          o += 12 * nc;
        }
      }
      xo[0] = r_off;
      bo[0] = -1;
      so[0] = -1;
    }
  }
  __syncthreads();
  for (int l = g0 ? 1 : 0; l < nlev; ++l) {  // cross sections of the LDS levels, once
    const LvlInst Li = lvl[l];
    const int nc = Li.nx * Li.ny;
    real* sg = lds + so[l];
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      sg[c] = (real)tl[l].sigt[Li.cell_off + c];
      sg[nc + c] = (real)tl[l].sigs[Li.cell_off + c];
    }
  }
  const LvlInst L0 = lvl[0];
  const int nc0 = L0.nx * L0.ny;
  if (!g0) {  // b of the first level
    const real* src = b_first + L0.cell_off * 12;
    for (int e = threadIdx.x; e < 12 * nc0; e += blockDim.x) lds[bo[0] + e] = src[e];
  }
  __syncthreads();
  // down: pre-smooth from zero, then residual -> next level's b
  for (int l = 0; l + 1 < nlev; ++l) {
    const LvlInst L = lvl[l], C = lvl[l + 1];
    const SymCoef<real> S = scf[l];
    const int nc = L.nx * L.ny, ncc = C.nx * C.ny;
    real* x = lds + xo[l];
    if (g0 && l == 0) {
      const real* bv = b_first + L.cell_off * 12;
      const double* sgt = tl[0].sigt + L.cell_off;
      const double* sgs = tl[0].sigs + L.cell_off;
      for (int k = 0; k < nu0; ++k) tail_sweep(S, L, sgt, sgs, bv, x, k == 0);
      // level 1's b cannot sit in LDS next to this level's x: through global
      real* bs = b1_scratch + C.cell_off * 12;
      tail_restrict(S, L, C, sgt, sgs, x, bv, bs);
      real* xg = x_first + L.cell_off * 12;
      for (int e = threadIdx.x; e < 12 * nc; e += blockDim.x) xg[e] = x[e];
      __syncthreads();
      real* bc = lds + bo[1];
      for (int e = threadIdx.x; e < 12 * ncc; e += blockDim.x) bc[e] = bs[e];
      __syncthreads();
    } else {
      real* bv = lds + bo[l];
      const real* sgt = lds + so[l];
      const real* sgs = sgt + nc;
      for (int k = 0; k < nu_smooth; ++k) tail_sweep_lds(S, L, sgt, sgs, bv, x, k == 0);
      tail_restrict(S, L, C, sgt, sgs, x, bv, lds + bo[l + 1]);
    }
  }
  {  // coarsest: red-black sweeps from zero
    const int l = nlev - 1;
    const LvlInst L = lvl[l];
    const SymCoef<real> S = scf[l];
    const int nc = L.nx * L.ny;
    const real* sgt = lds + so[l];
    for (int k = 0; k < coarse_sweeps; ++k) tail_sweep_lds(S, L, sgt, sgt + nc, lds + bo[l], lds + xo[l], k == 0);
  }
  // up: prolong the correction, post-smooth in reverse colour order
  for (int l = nlev - 2; l >= 0; --l) {
    const LvlInst L = lvl[l], C = lvl[l + 1];
    const SymCoef<real> S = scf[l];
    const int nc = L.nx * L.ny;
    real* x = lds + xo[l];
    const real* xc = lds + xo[l + 1];
    if (g0 && l == 0) {
      // x comes back from global memory plus the correction, into R (the
      // coarser levels are done with it)
      real* xg = x_first + L.cell_off * 12;
      tail_prolong(L, C, xc, xg, x);
      const real* bv = b_first + L.cell_off * 12;
      const double* sgt = tl[0].sigt + L.cell_off;
      const double* sgs = tl[0].sigs + L.cell_off;
      for (int k = 0; k < nu0; ++k) {
        tail_half_sweep(S, L, sgt, sgs, bv, x, 1, 0);
        tail_half_sweep(S, L, sgt, sgs, bv, x, 0, 0);
      }
      if (!zout)
        for (int e = threadIdx.x; e < 12 * nc; e += blockDim.x) xg[e] = x[e];
    } else {
      tail_prolong(L, C, xc, x, x);
      const real* sgt = lds + so[l];
      const real* bv = lds + bo[l];
      for (int k = 0; k < nu_smooth; ++k) {
        tail_half_sweep_lds(S, L, sgt, sgt + nc, bv, x, 1, 0);
        tail_half_sweep_lds(S, L, sgt, sgt + nc, bv, x, 0, 0);
      }
    }
  }
  if (zout) {
    // z = v + (x_fine + P x) on the finest level's scalar-flux unknowns (the
    // arithmetic of k_dsa_out_prolong, with the first level's x from LDS)
    const InstDev I = insts[b];
    const LvlInst F = lf0[b];
    const int nfc = F.nx * F.ny;
    const float* __restrict__ xb = xfine + F.cell_off * 12;
    const real* xl = lds + xo[0];
    for (int cell = threadIdx.x; cell < nfc; cell += blockDim.x) {
      const int i = cell % F.nx, k = cell / F.nx;
      const int parent = (k >> 1) * L0.nx + (i >> 1);
      float xc[4];
#pragma unroll
      for (int L2 = 0; L2 < 4; ++L2) xc[L2] = (float)xl[L2 * nc0 + parent];
      const double2* vp = reinterpret_cast<const double2*>(vout + I.dof_off + 4 * (int64_t)cell);
      double2* zp = reinterpret_cast<double2*>(zout + I.dof_off + 4 * (int64_t)cell);
      const double2 v01 = vp[0], v23 = vp[1];
      const double vv[4] = {v01.x, v01.y, v23.x, v23.y};
      double o[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        float corr = 0.f;
#pragma unroll
        for (int L2 = 0; L2 < 4; ++L2)
          corr += (float)(inj1d(i & 1, m & 1, L2 & 1) * inj1d(k & 1, m >> 1, L2 >> 1)) * xc[L2];
        o[m] = vv[m] + (double)(xb[m * nfc + cell] + corr);
      }
      zp[0] = make_double2(o[0], o[1]);
      zp[1] = make_double2(o[2], o[3]);
    }
  } else if (!g0) {  // x of the first level
    real* dst = x_first + L0.cell_off * 12;
    for (int e = threadIdx.x; e < 12 * nc0; e += blockDim.x) dst[e] = lds[xo[0] + e];
  }
}

// ------------------------------------------------------------------ host side
struct MgLevel {
  std::vector<LvlInst> li;
  LvlInst* d_li = nullptr;
  int64_t ncell = 0;
  int max_nx = 0, max_ny = 0;
  DsaStencil* d_st = nullptr;
  double *st = nullptr, *ss = nullptr, *inv = nullptr, *x = nullptr, *b = nullptr, *r = nullptr;
};

struct DsaSolver {
  rte_batch* b = nullptr;
  int nu = 12;
  int restart = 0;
  std::vector<MgLevel> lv;
  double* inv0 = nullptr;   // level 0 inverses per (instance, region)
  double *X = nullptr, *T = nullptr, *rhs = nullptr, *tol = nullptr, *rn = nullptr;
  int32_t* d_live = nullptr;
  Krylov K;                 // only with restart >= 1
  Space sp;                 // DSA space of level 0
  bool sym = false;         // every instance has a reflection-symmetric rule
  // Stationary V-cycles (restart == 0) with structured kernels keep the whole
  // hierarchy in FP32: a fixed preconditioner needs no more, and the level
  // sweeps are bound by memory traffic.  Exact solves (restart >= 1) and the
  // general-rule kernels stay in FP64.
  bool f32 = false;
  size_t esz() const { return f32 ? sizeof(float) : sizeof(double); }
  // the LDS-resident tail of the hierarchy (structured kernels only)
  int tail_first = -1;
  size_t tail_lds = 0;
  int tail_g0 = 0;  // the tail's first level keeps x and b in HBM (FP32 only)
  MgTailLevel* d_tail = nullptr;
  // smoothing sweeps before and after the coarse correction: nu_smooth on the
  // LDS-resident levels; on the levels streamed through HBM of the FP32
  // stationary V-cycle nu_hbm before and after, except none after on the
  // finest level (a sweep there costs more time than the extra FGMRES
  // iterations it saves); nu_smooth everywhere in the FP64 hierarchy
  int nu_smooth = 2, nu_hbm = 1, nu_hbm_finest_post = 0, coarse_sweeps = 4;
  // set by apply for one FP32 V-cycle: level 0 stops after the coarse
  // correction, which k_dsa_out_prolong then adds while writing the output
  bool defer_fine_prolong = false;
  // set by apply when the tail (starting at level 1) writes the output z itself
  const double* tail_out_v = nullptr;
  double* tail_out_z = nullptr;
  const float* tail_out_xf = nullptr;
  // set by apply for that V-cycle too: level 0's first two half sweeps form
  // the right-hand side from v (the first stores its colour-0 part)
  const double* rhs_from_v = nullptr;
  int pc = 0;  // partially consistent variant
  int init(rte_batch* batch, int restart_, int pc_);
  void release();
  int prepare(const double* sigma_t, const double* sigma_s, const int32_t* active, hipStream_t s);
  int stencil(int l, int mode, int color, const double* bv, double* x, double* y, const int32_t* act,
              hipStream_t s);
  int smooth(int l, int sweeps, bool reverse, bool from_zero, const double* bv, double* x,
             const int32_t* act, hipStream_t s);
  int vcycle(int l, const double* bv, double* x, const int32_t* act, hipStream_t s);
  int precond(const double* in, double* out, const int32_t* act, hipStream_t s);
  int field_corr(const double* sigma_t, const double* sigma_s, const double* x, double* y, double sign,
                 const int32_t* act, hipStream_t s);
  int apply(const double* sigma_t, const double* sigma_s, const double* v, double* z, double inner_tol,
            int inner_max, const int32_t* active, int32_t* iters_host, bool prep, hipStream_t s);
  dim3 grid(int l) const {
    const int c = lv[l].max_nx * lv[l].max_ny;
    return dim3((unsigned)std::max(1, std::min(1024, (c + 255) / 256)), b->n_inst);
  }
};

int DsaSolver::init(rte_batch* batch, int restart_, int pc_) {
  pc = pc_;
  b = batch;
  restart = restart_;
  nu = b->dim == 2 ? 12 : 4;
  const int n = b->n_inst;
  // levels: coarsen while every instance can be halved
  int nlev = 1;
  {
    bool ok = true;
    int f = 1;
    while (ok) {
      for (const auto& I : b->inst) {
        const int nx = I.nx / f, ny = I.ny / f;
        const bool can = (nx % 2 == 0) && nx >= 4 && (I.dim == 1 || (ny % 2 == 0 && ny >= 4));
        ok = ok && can;
      }
      if (ok) {
        ++nlev;
        f *= 2;
      }
      if (nlev >= 12) break;
    }
  }
  lv.resize(nlev);
  for (int l = 0; l < nlev; ++l) {
    MgLevel& L = lv[l];
    L.li.resize(n);
    int64_t off = 0;
    for (int k = 0; k < n; ++k) {
      const auto& I = b->inst[k];
      const int f = 1 << l;
      LvlInst q{};
      q.nx = I.nx / f;
      q.ny = I.dim == 2 ? I.ny / f : 1;
      q.dim = I.dim;
      q.nloc = I.nloc;
      q.hx = I.hx * f;
      q.hy = I.dim == 2 ? I.hy * f : 1.0;
      q.cell_off = off;
      off += (int64_t)q.nx * q.ny;
      L.max_nx = std::max(L.max_nx, q.nx);
      L.max_ny = std::max(L.max_ny, q.ny);
      L.li[k] = q;
    }
    L.ncell = off;
    if (hipMalloc(&L.d_li, sizeof(LvlInst) * n) != hipSuccess ||
        hipMalloc(&L.d_st, sizeof(DsaStencil) * n) != hipSuccess ||
        hipMalloc(&L.st, sizeof(double) * off) != hipSuccess ||
        hipMalloc(&L.ss, sizeof(double) * off) != hipSuccess ||
        hipMalloc(&L.x, sizeof(double) * off * nu) != hipSuccess ||
        hipMalloc(&L.b, sizeof(double) * off * nu) != hipSuccess ||
        hipMalloc(&L.r, sizeof(double) * off * nu) != hipSuccess ||
        (l > 0 && hipMalloc(&L.inv, sizeof(double) * off * nu * nu) != hipSuccess))
      return RTE_ENOMEM;
    RTE_HIP(hipMemcpy(L.d_li, L.li.data(), sizeof(LvlInst) * n, hipMemcpyHostToDevice));
    // per-level stencil: the same construction with this level's cell sizes
    std::vector<InstDev> tmp = b->inst;
    for (int k = 0; k < n; ++k) {
      tmp[k].hx = L.li[k].hx;
      tmp[k].hy = L.li[k].hy;
    }
    InstDev* d_tmp = nullptr;
    if (hipMalloc(&d_tmp, sizeof(InstDev) * n) != hipSuccess) return RTE_ENOMEM;
    RTE_HIP(hipMemcpy(d_tmp, tmp.data(), sizeof(InstDev) * n, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_dsa_setup, dim3((n + 63) / 64), dim3(64), 0, 0, n, d_tmp, b->d_ox, b->d_oy,
                       b->d_w, L.d_st, pc);
    RTE_HIP(hipGetLastError());
    RTE_HIP(hipDeviceSynchronize());
    (void)hipFree(d_tmp);
  }
  {
    std::vector<DsaStencil> hs(n);
    RTE_HIP(hipMemcpy(hs.data(), lv[0].d_st, sizeof(DsaStencil) * n, hipMemcpyDeviceToHost));
    sym = nu == 12;
    for (int k = 0; k < n; ++k) sym = sym && hs[k].sym;
    f32 = sym && restart == 0;
  }
  if (sym) {
    // first level l >= 1 from which every level's x, b and cross sections fit
    // in the work group's LDS
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    int dev = 0, lds_max = 64 * 1024;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    const size_t budget = (size_t)std::max(16 * 1024, std::min(lds_max, 160 * 1024) - 4 * 1024);
    auto pick = [&](size_t cap) {
      tail_first = -1;
      tail_lds = 0;
      tail_g0 = 0;
      size_t need = 0;
      for (int l = nlev - 1; l >= 1; --l) {
        need += (size_t)26 * lv[l].max_nx * lv[l].max_ny * es;
        if (need > cap || nlev - l > MG_TAIL_MAX) break;
        tail_first = l;
        tail_lds = need;
      }
      // FP32: one more level (from level 1 on) whose b and cross sections
      // stay in HBM and whose x shares LDS with the coarser levels' b and x
      // (the launch's g0 layout)
      const int l0 = tail_first - 1;
      if (f32 && tail_first >= 2 && nlev - l0 <= MG_TAIL_MAX) {
        auto cells = [&](int l) { return (size_t)lv[l].max_nx * lv[l].max_ny; };
        size_t sg = 0, rest = 0;
        for (int l = l0 + 1; l < nlev; ++l) {
          sg += 2 * cells(l);
          rest += 12 * cells(l) * (l >= l0 + 2 ? 2 : 1);
        }
        const size_t g0_need = (sg + 12 * cells(l0 + 1) + std::max(12 * cells(l0), rest)) * es;
        if (g0_need <= cap) {
          tail_first = l0;
          tail_lds = g0_need;
          tail_g0 = 1;
        }
      }
    };
    pick(budget);
    if (tail_lds > 60 * 1024) {  // beyond the default dynamic LDS limit: opt in, else stay within it
      const hipError_t e1 = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mg_tail_sym<float, MG_TAIL_THREADS_F32>),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)tail_lds);
      const hipError_t e2 = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mg_tail_sym<double, MG_TAIL_THREADS_F64>),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)tail_lds);
      if (e1 != hipSuccess || e2 != hipSuccess) {
        (void)hipGetLastError();
        pick(60 * 1024);
      }
    }
    if (tail_first > 0) {
      std::vector<MgTailLevel> h;
      for (int l = tail_first; l < nlev; ++l) h.push_back({lv[l].d_li, lv[l].d_st, lv[l].st, lv[l].ss});
      if (hipMalloc(&d_tail, sizeof(MgTailLevel) * h.size()) != hipSuccess) return RTE_ENOMEM;
      RTE_HIP(hipMemcpy(d_tail, h.data(), sizeof(MgTailLevel) * h.size(), hipMemcpyHostToDevice));
    }
  }
  std::vector<int64_t> lens(n);
  for (int k = 0; k < n; ++k) lens[k] = (int64_t)lv[0].li[k].nx * lv[0].li[k].ny * nu;
  RTE_TRY(sp.init(lens));
  if (restart > 0) RTE_TRY(K.init(lens, restart, false));
  const int64_t tot = sp.total;
  if (hipMalloc(&inv0, sizeof(double) * n * b->max_regions * DMAX * DMAX) != hipSuccess ||
      hipMalloc(&X, sizeof(double) * tot) != hipSuccess ||
      hipMalloc(&T, sizeof(double) * tot) != hipSuccess ||
      hipMalloc(&rhs, sizeof(double) * tot) != hipSuccess ||
      hipMalloc(&tol, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&rn, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&d_live, sizeof(int32_t) * n) != hipSuccess)
    return RTE_ENOMEM;
  return RTE_OK;
}

void DsaSolver::release() {
  if (restart > 0) K.release();
  sp.release();
  for (auto& L : lv)
    for (void* p : {(void*)L.d_li, (void*)L.d_st, (void*)L.st, (void*)L.ss, (void*)L.inv, (void*)L.x,
                    (void*)L.b, (void*)L.r})
      (void)hipFree(p);
  lv.clear();
  for (void* p : {(void*)inv0, (void*)X, (void*)T, (void*)rhs, (void*)tol, (void*)rn, (void*)d_live,
                  (void*)d_tail})
    (void)hipFree(p);
  d_tail = nullptr;
  tail_first = -1;
  tail_g0 = 0;
  inv0 = X = T = rhs = tol = rn = nullptr;
  d_live = nullptr;
}

int DsaSolver::prepare(const double* sigma_t, const double* sigma_s, const int32_t* active,
                       hipStream_t s) {
  const int n = b->n_inst;
  const int mr = b->max_regions;
  if (b->n_fields > 0)
    hipLaunchKernelGGL(k_mg_sigma0_field, grid(0), dim3(256), 0, s, b->d_inst, lv[0].d_li, b->d_fblk, b->n_fields,
                       b->field_ncell, sigma_t, sigma_s, mr, lv[0].st, lv[0].ss);
  else
    hipLaunchKernelGGL(k_mg_sigma0, grid(0), dim3(256), 0, s, b->d_inst, lv[0].d_li, b->d_region, sigma_t,
                       sigma_s, mr, lv[0].st, lv[0].ss);
  if (!sym)
    hipLaunchKernelGGL(k_dsa_blockinv, dim3((n * mr + 63) / 64), dim3(64), 0, s, n, mr, b->d_inst,
                       lv[0].d_st, sigma_t, sigma_s, inv0);
  for (size_t l = 1; l < lv.size(); ++l) {
    hipLaunchKernelGGL(k_mg_sigma_coarsen, grid(l), dim3(256), 0, s, lv[l - 1].d_li, lv[l].d_li,
                       lv[l - 1].st, lv[l - 1].ss, lv[l].st, lv[l].ss);
    if (sym) continue;  // block solves are explicit for symmetric rules
    if (nu == 12)
      hipLaunchKernelGGL(k_mg_inv_cells<12>, grid(l), dim3(64), 0, s, lv[l].d_li, lv[l].d_st, lv[l].st,
                         lv[l].ss, lv[l].inv, active);
    else
      hipLaunchKernelGGL(k_mg_inv_cells<4>, grid(l), dim3(64), 0, s, lv[l].d_li, lv[l].d_st, lv[l].st,
                         lv[l].ss, lv[l].inv, active);
  }
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int DsaSolver::stencil(int l, int mode, int color, const double* bv, double* x, double* y,
                       const int32_t* act, hipStream_t s) {
  MgLevel& L = lv[l];
  const double* inv = l == 0 ? inv0 : L.inv;
  const int per_cell = l == 0 ? 0 : 1;
  dim3 gs = grid(l);
  if (mode >= 2) gs.x = (gs.x + 1) / 2;  // one colour: half the cells (grid-stride loop either way)
  const bool from_v = rhs_from_v && l == 0 && mode >= 3;
  if (sym && f32)
    hipLaunchKernelGGL(k_mg_stencil_sym<float>, gs, dim3(256), 0, s, mode, color, L.d_li, L.d_st, L.st,
                       L.ss, reinterpret_cast<const float*>(bv), reinterpret_cast<float*>(x),
                       reinterpret_cast<float*>(y), act, from_v ? rhs_from_v : nullptr, b->d_inst,
                       from_v ? reinterpret_cast<float*>(const_cast<double*>(bv)) : nullptr);
  else if (sym)
    hipLaunchKernelGGL(k_mg_stencil_sym<double>, gs, dim3(256), 0, s, mode, color, L.d_li, L.d_st, L.st,
                       L.ss, bv, x, y, act);
  else if (nu == 12)
    hipLaunchKernelGGL(k_mg_stencil<12>, grid(l), dim3(256), 0, s, mode, color, L.d_li, L.d_st, L.st,
                       L.ss, inv, per_cell, b->d_region, b->d_inst, b->max_regions, bv, x, y, act);
  else
    hipLaunchKernelGGL(k_mg_stencil<4>, grid(l), dim3(256), 0, s, mode, color, L.d_li, L.d_st, L.st,
                       L.ss, inv, per_cell, b->d_region, b->d_inst, b->max_regions, bv, x, y, act);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

// `sweeps` red-black sweeps on x (colour 0 first, or colour 1 first if reverse);
// from_zero: x holds no values yet and the first half sweep starts from zero.
int DsaSolver::smooth(int l, int sweeps, bool reverse, bool from_zero, const double* bv, double* x,
                      const int32_t* act, hipStream_t s) {
  for (int k = 0; k < sweeps; ++k) {
    if (k == 0 && from_zero && sym && !reverse) {  // both half sweeps know x = 0 beforehand
      RTE_TRY(stencil(l, 3, 0, bv, x, nullptr, act, s));
      RTE_TRY(stencil(l, 4, 1, bv, x, nullptr, act, s));
      continue;
    }
    if (k == 0 && from_zero) RTE_HIP(hipMemsetAsync(x, 0, esz() * lv[l].ncell * nu, s));
    RTE_TRY(stencil(l, 2, reverse ? 1 : 0, bv, x, nullptr, act, s));
    RTE_TRY(stencil(l, 2, reverse ? 0 : 1, bv, x, nullptr, act, s));
  }
  return RTE_OK;
}

// x = V-cycle approximation of K_l^{-1} bv (bv and x must not alias)
int DsaSolver::vcycle(int l, const double* bv, double* x, const int32_t* act, hipStream_t s) {
  MgLevel& L = lv[l];
  if (l == tail_first) {
    const int nt = (int)lv.size() - l;
    if (f32)
      hipLaunchKernelGGL((k_mg_tail_sym<float, MG_TAIL_THREADS_F32>), dim3(b->n_inst), dim3(MG_TAIL_THREADS_F32), tail_lds, s, d_tail, nt, nu_smooth,
                         coarse_sweeps, reinterpret_cast<const float*>(bv), reinterpret_cast<float*>(x), act,
                         tail_g0, nu_hbm, tail_g0 ? reinterpret_cast<float*>(lv[l + 1].b) : (float*)nullptr,
                         b->d_inst, lv[0].d_li, tail_out_xf, tail_out_v, tail_out_z);
    else
      hipLaunchKernelGGL((k_mg_tail_sym<double, MG_TAIL_THREADS_F64>), dim3(b->n_inst), dim3(MG_TAIL_THREADS_F64), tail_lds, s, d_tail, nt, nu_smooth,
                         coarse_sweeps, bv, x, act, 0, nu_smooth, (double*)nullptr);
    RTE_HIP(hipGetLastError());
    return RTE_OK;
  }
  if (l == (int)lv.size() - 1) {
    if (sym && l > 0) {  // whole coarsest smoothing in one launch
      if (f32)
        hipLaunchKernelGGL(k_mg_coarse_sym<float>, dim3(b->n_inst), dim3(256), 0, s, coarse_sweeps, L.d_li,
                           L.d_st, L.st, L.ss, reinterpret_cast<const float*>(bv), reinterpret_cast<float*>(x),
                           act);
      else
        hipLaunchKernelGGL(k_mg_coarse_sym<double>, dim3(b->n_inst), dim3(256), 0, s, coarse_sweeps, L.d_li,
                           L.d_st, L.st, L.ss, bv, x, act);
      RTE_HIP(hipGetLastError());
      return RTE_OK;
    }
    return smooth(l, coarse_sweeps, false, true, bv, x, act, s);
  }
  if (l == 0 && sym && f32 && rhs_from_v && defer_fine_prolong && nu_hbm == 1) {
    // the finest level's part (right-hand side from v, one from-zero sweep,
    // residual and restriction) in one pass over tiles
    MgLevel& C = lv[1];
    int tiles = 0;
    for (const auto& q : L.li) tiles = std::max(tiles, ((q.nx + FF_T - 1) / FF_T) * ((q.ny + FF_T - 1) / FF_T));
    hipLaunchKernelGGL(k_mg_fine_fused, dim3(tiles, b->n_inst), dim3(512), 0, s, L.d_li, C.d_li, L.d_st, L.st,
                       L.ss, b->d_inst, rhs_from_v, reinterpret_cast<float*>(x), reinterpret_cast<float*>(C.b),
                       act);
    RTE_HIP(hipGetLastError());
    return vcycle(1, C.b, C.x, act, s);
  }
  // smoothing sweeps before and after the coarse correction on this level
  const int pre = f32 ? nu_hbm : nu_smooth;
  const int post = f32 ? (l == 0 ? nu_hbm_finest_post : nu_hbm) : nu_smooth;
  RTE_TRY(smooth(l, pre, false, true, bv, x, act, s));
  MgLevel& C = lv[l + 1];
  const dim3 g = grid(l + 1);
  if (sym && f32) {
    // the pre-smoothing ended with a colour-1 half sweep
    hipLaunchKernelGGL(k_mg_resrestrict_sym<float>, g, dim3(256), 0, s, L.d_li, C.d_li, L.d_st, L.st, L.ss,
                       reinterpret_cast<const float*>(bv), reinterpret_cast<const float*>(x),
                       reinterpret_cast<float*>(C.b), 1, act, (rhs_from_v && l == 0) ? 1 : 0);
  } else if (sym) {
    hipLaunchKernelGGL(k_mg_resrestrict_sym<double>, g, dim3(256), 0, s, L.d_li, C.d_li, L.d_st, L.st, L.ss,
                       bv, x, C.b, 1, act);
  } else {
    RTE_TRY(stencil(l, 1, 0, bv, x, L.r, act, s));
    if (nu == 12)
      hipLaunchKernelGGL((k_mg_transfer<12, double>), g, dim3(256), 0, s, 0, L.d_li, C.d_li, L.r,
                         (double*)nullptr, (const double*)nullptr, C.b, act);
    else
      hipLaunchKernelGGL((k_mg_transfer<4, double>), g, dim3(256), 0, s, 0, L.d_li, C.d_li, L.r,
                         (double*)nullptr, (const double*)nullptr, C.b, act);
  }
  RTE_HIP(hipGetLastError());
  RTE_TRY(vcycle(l + 1, C.b, C.x, act, s));
  if (l == 0 && defer_fine_prolong) return RTE_OK;
  if (f32)
    hipLaunchKernelGGL((k_mg_transfer<12, float>), g, dim3(256), 0, s, 1, L.d_li, C.d_li, (const float*)nullptr,
                       reinterpret_cast<float*>(x), reinterpret_cast<const float*>(C.x), (float*)nullptr, act);
  else if (nu == 12)
    hipLaunchKernelGGL((k_mg_transfer<12, double>), g, dim3(256), 0, s, 1, L.d_li, C.d_li,
                       (const double*)nullptr, x, C.x, (double*)nullptr, act);
  else
    hipLaunchKernelGGL((k_mg_transfer<4, double>), g, dim3(256), 0, s, 1, L.d_li, C.d_li,
                       (const double*)nullptr, x, C.x, (double*)nullptr, act);
  RTE_HIP(hipGetLastError());
  return smooth(l, post, true, false, bv, x, act, s);
}

// out = V-cycle(in) on level 0 (in and out may alias)
int DsaSolver::precond(const double* in, double* out, const int32_t* act, hipStream_t s) {
  if (in == out) {
    RTE_HIP(hipMemcpyAsync(lv[0].b, in, esz() * sp.total, hipMemcpyDeviceToDevice, s));
    in = lv[0].b;
  }
  return vcycle(0, in, out, act, s);
}

__global__ void k_scale_tol(int n, const double* __restrict__ rn, double rtol, double* __restrict__ tol) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n) tol[b] = rtol * rn[b];
}

int DsaSolver::field_corr(const double* sigma_t, const double* sigma_s, const double* x, double* y, double sign,
                          const int32_t* act, hipStream_t s) {
  hipLaunchKernelGGL(k_dsa_field_corr, grid(0), dim3(256), 0, s, b->d_inst, lv[0].d_st, b->d_fblk, b->n_fields,
                     b->field_ncell, sigma_t, sigma_s, b->max_regions, sp.d_off, x, y, sign, act);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int DsaSolver::apply(const double* sigma_t, const double* sigma_s, const double* v, double* z,
                     double inner_tol, int inner_max, const int32_t* active, int32_t* iters_host,
                     bool prep, hipStream_t s) {
  const int n = b->n_inst;
  const int mr = b->max_regions;
  // every instance's data, so that later calls with other masks find it ready
  if (prep) RTE_TRY(prepare(sigma_t, sigma_s, nullptr, s));
  // one V-cycle whose finest level sees b only in its single from-zero sweep
  // (formed from v there; only the scalar-flux field is kept for the
  // restriction) and whose fine correction goes straight into z
  const bool fused_out = restart == 0 && inner_max == 1 && f32 && sym && lv.size() >= 2 &&
                         nu_hbm_finest_post == 0 && tail_first != 0 && nu_hbm == 1;
  // the V-cycle's tail starts at level 1: it writes z itself
  const bool tail_out = fused_out && tail_first == 1;
  if (fused_out) {
    // the V-cycle forms the right-hand side itself
  } else if (b->n_fields > 0)
    hipLaunchKernelGGL(k_dsa_rhs_field, grid(0), dim3(256), 0, s, b->d_inst, lv[0].d_st, b->d_fblk, b->n_fields,
                       b->field_ncell, sigma_s, mr, sp.d_off, v, rhs, active);
  else if (f32)
    hipLaunchKernelGGL(k_dsa_rhs<float>, grid(0), dim3(256), 0, s, b->d_inst, lv[0].d_st, b->d_region, sigma_s,
                       mr, sp.d_off, v, reinterpret_cast<float*>(rhs), active);
  else
    hipLaunchKernelGGL(k_dsa_rhs<double>, grid(0), dim3(256), 0, s, b->d_inst, lv[0].d_st, b->d_region,
                       sigma_s, mr, sp.d_off, v, rhs, active);
  RTE_HIP(hipGetLastError());
  std::vector<int32_t> iters(n, 0);
  if (restart == 0) {
    // stationary: X <- X + V(rhs - K X), inner_max cycles
    for (int k = 0; k < inner_max; ++k) {
      if (k == 0) {
        defer_fine_prolong = fused_out;
        rhs_from_v = fused_out ? v : nullptr;
        if (tail_out) {
          tail_out_v = v;
          tail_out_z = z;
          tail_out_xf = reinterpret_cast<const float*>(X);
        }
        const int st = precond(rhs, X, active, s);
        defer_fine_prolong = false;
        rhs_from_v = nullptr;
        tail_out_v = nullptr;
        tail_out_z = nullptr;
        tail_out_xf = nullptr;
        RTE_TRY(st);
      } else {
        RTE_TRY(stencil(0, 1, 0, rhs, X, lv[0].b, active, s));
        RTE_TRY(vcycle(0, lv[0].b, lv[0].x, active, s));
        if (f32)
          hipLaunchKernelGGL(k_dsa_axpy<float>, grid(0), dim3(256), 0, s, sp.d_off, sp.d_len,
                             reinterpret_cast<const float*>(lv[0].x), reinterpret_cast<float*>(X), active);
        else
          hipLaunchKernelGGL(k_dsa_axpy<double>, grid(0), dim3(256), 0, s, sp.d_off, sp.d_len, lv[0].x, X,
                             active);
        RTE_HIP(hipGetLastError());
      }
    }
    for (int q = 0; q < n; ++q) iters[q] = inner_max;
  } else {
    std::vector<int32_t> act(n, 1);
    if (active) RTE_HIP(hipMemcpyAsync(act.data(), active, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    RTE_HIP(hipStreamSynchronize(s));
    RTE_HIP(hipMemcpyAsync(d_live, act.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    RTE_HIP(hipMemsetAsync(X, 0, sizeof(double) * sp.total, s));
    RTE_TRY(knorm(sp, rhs, K.partA, rn, 1, d_live, s));
    hipLaunchKernelGGL(k_scale_tol, dim3((n + 63) / 64), dim3(64), 0, s, n, rn, inner_tol, tol);
    int done_iters = 0;
    std::vector<int32_t> jd(n), live_h = act;
    while (true) {
      if (done_iters == 0) {
        RTE_TRY(kcopy(sp, rhs, T, d_live, s));
      } else {
        RTE_TRY(stencil(0, 1, 0, rhs, X, T, d_live, s));
        if (b->n_fields > 0) RTE_TRY(field_corr(sigma_t, sigma_s, X, T, -1.0, d_live, s));
      }
      RTE_HIP(hipMemcpyAsync(K.active, d_live, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
      RTE_TRY(kstart(K, T, tol, s));
      int j = 0;
      for (; j < restart && done_iters + j < inner_max; ++j) {
        RTE_TRY(precond(K.v(j), T, K.active, s));
        RTE_TRY(stencil(0, 0, 0, nullptr, T, K.v(j + 1), K.active, s));
        if (b->n_fields > 0) RTE_TRY(field_corr(sigma_t, sigma_s, T, K.v(j + 1), 1.0, K.active, s));
        RTE_TRY(arnoldi_mgs(K, j, s));
        if ((j + 1) % 4 == 0) {
          std::vector<int32_t> a(n);
          RTE_HIP(hipMemcpyAsync(a.data(), K.active, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
          RTE_HIP(hipStreamSynchronize(s));
          bool any = false;
          for (int q = 0; q < n; ++q) any = any || a[q];
          if (!any) {
            ++j;
            break;
          }
        }
      }
      RTE_HIP(hipMemsetAsync(T, 0, sizeof(double) * sp.total, s));
      RTE_TRY(kylov_solve_update(K, K.V, T, s));
      RTE_TRY(precond(T, T, d_live, s));
      RTE_TRY(kaxpby(sp, 1.0, T, 1.0, X, d_live, s));
      std::vector<double> sc(8 * n), tl(n);
      RTE_HIP(hipMemcpyAsync(jd.data(), K.jdone, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
      RTE_HIP(hipMemcpyAsync(sc.data(), K.scal, sizeof(double) * 8 * n, hipMemcpyDeviceToHost, s));
      RTE_HIP(hipMemcpyAsync(tl.data(), tol, sizeof(double) * n, hipMemcpyDeviceToHost, s));
      RTE_HIP(hipStreamSynchronize(s));
      done_iters += j;
      bool any = false;
      for (int q = 0; q < n; ++q) {
        if (!live_h[q]) continue;
        iters[q] += jd[q];
        if (sc[8 * q + 2] <= tl[q]) live_h[q] = 0;
        any = any || live_h[q];
      }
      if (!any || done_iters >= inner_max || j == 0) break;
      RTE_HIP(hipMemcpyAsync(d_live, live_h.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    }
  }
  if (tail_out) {
    // z written by the tail
  } else if (fused_out)
    hipLaunchKernelGGL(k_dsa_out_prolong, grid(0), dim3(256), 0, s, b->d_inst, lv[0].d_li, lv[1].d_li,
                       reinterpret_cast<const float*>(X), reinterpret_cast<const float*>(lv[1].x), v, z, active);
  else if (f32)
    hipLaunchKernelGGL(k_dsa_out<float>, grid(0), dim3(256), 0, s, b->d_inst, lv[0].d_st, sp.d_off,
                       reinterpret_cast<const float*>(X), v, z, active);
  else
    hipLaunchKernelGGL(k_dsa_out<double>, grid(0), dim3(256), 0, s, b->d_inst, lv[0].d_st, sp.d_off, X, v, z,
                       active);
  RTE_HIP(hipGetLastError());
  if (iters_host) {
    RTE_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < n; ++q) iters_host[q] = iters[q];
  }
  return RTE_OK;
}

// registry: one DSA solver per (batch, restart, variant) kept alive with the batch
struct DsaCache {
  rte_batch* b;
  int restart, pc;
  DsaSolver* s;
};
static std::vector<DsaCache> g_dsa;

DsaSolver* dsa_for(rte_batch* b, int restart, int pc) {
  for (auto& c : g_dsa)
    if (c.b == b && c.restart == restart && c.pc == pc) return c.s;
  auto* s = new DsaSolver();
  if (s->init(b, restart, pc) != RTE_OK) {
    s->release();
    delete s;
    return nullptr;
  }
  g_dsa.push_back({b, restart, pc, s});
  return s;
}

void dsa_forget(rte_batch* b) {
  for (size_t i = 0; i < g_dsa.size();) {
    if (g_dsa[i].b == b) {
      g_dsa[i].s->release();
      delete g_dsa[i].s;
      g_dsa.erase(g_dsa.begin() + i);
    } else {
      ++i;
    }
  }
}

int dsa_apply(rte_batch* b, const double* sigma_t, const double* sigma_s, const double* v, double* z,
              double inner_tol, int inner_max, int restart, const int32_t* active, int32_t* iters,
              hipStream_t s, bool prepare, int variant) {
  // cross sections varying inside the cells: only the exact solve (whose
  // GMRES sees the full blocks) on the structured path of symmetric rules
  if (b->n_fields > 0 && (restart < 1 || b->dim != 2)) return RTE_EINVAL;
  DsaSolver* d = dsa_for(b, restart, variant == RTE_DSA_PC ? 1 : 0);
  if (!d) return RTE_ENOMEM;
  if (b->n_fields > 0 && !d->sym) return RTE_EINVAL;
  return d->apply(sigma_t, sigma_s, v, z, inner_tol, inner_max, active, iters, prepare, s);
}

}  // namespace rte

extern "C" int rte_dsa_apply(const rte_batch* cb, const double* sigma_t, const double* sigma_s,
                             const double* v, double* z, double inner_tol, int inner_max, int restart,
                             int variant, int32_t* stats_iters, void* stream) {
  auto* b = const_cast<rte_batch*>(cb);
  if (!b || !sigma_t || !sigma_s || !v || !z || inner_max < 1 || restart < 0 || restart > 500 ||
      !(inner_tol >= 0.0) || (variant != RTE_DSA_FC && variant != RTE_DSA_PC) ||
      (variant == RTE_DSA_PC && restart == 0))
    return RTE_EINVAL;
  return rte::dsa_apply(b, sigma_t, sigma_s, v, z, inner_tol, inner_max, restart, nullptr,
                        stats_iters, reinterpret_cast<hipStream_t>(stream), true, variant);
}
