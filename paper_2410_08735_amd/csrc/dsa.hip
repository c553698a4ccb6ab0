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
// Unknowns per cell (cell-major): [dphi(nloc), dJ_x(nloc) (, dJ_y(nloc))].
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
// The system is solved by restarted GMRES preconditioned on the right with
// the exact inverse of each cell's diagonal block (block Jacobi); the
// diagonal block depends only on the cell's region, so its inverse is formed
// once per (instance, region).
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
__global__ void k_dsa_setup(int n_inst, const InstDev* __restrict__ insts,
                            const double* __restrict__ ox, const double* __restrict__ oy,
                            const double* __restrict__ w, DsaStencil* __restrict__ out) {
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
  for (int z = 0; z < 5; ++z)
    for (int q = 0; q < DMAX * DMAX; ++q) S.blk[z][q] = 0.0;
  for (int q = 0; q < DMAX * DMAX; ++q) S.St[q] = S.Ss[q] = 0.0;
  // field blocks: coefficient (alpha_C[e], alpha_J[e]) for field row F, column F'
  // F = 0: dphi, F = 1 + d: dJ_d
  for (int F = 0; F <= ne; ++F)
    for (int Fp = 0; Fp <= ne; ++Fp) {
      double aC[2] = {0, 0}, aJ[2] = {0, 0};
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
          aJ[e] = -0.5 * bm[d][e];
        } else {
          const int d = F - 1, f = Fp - 1;
          aC[e] = 3.0 * t[d][e][f];
          aJ[e] = -1.5 * c[d][e][f];
        }
      }
      for (int k = 0; k < nl; ++k)
        for (int l = 0; l < nl; ++l) {
          const int row = F * nl + k, col = Fp * nl + l, q = row * nu + col;
          double self = 0.0;
          for (int e = 0; e < ne; ++e)
            self += aC[e] * emb(DCs[e], e, k, l) + aJ[e] * emb(DJs[e], e, k, l);
          S.blk[0][q] = self;
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
      A[i][j] = S.blk[0][i * nu + j] + ts * S.St[i * nu + j] + ss * S.Ss[i * nu + j];
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
  double* o = inv + ((int64_t)b * max_regions + rg) * DMAX * DMAX;
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j < nu; ++j) o[i * nu + j] = A[i][nu + j];
}

// y = K x (matrix-free), one thread per cell.
template <int NU>
__global__ void k_dsa_apply(const InstDev* __restrict__ insts, const DsaStencil* __restrict__ st_,
                            const int32_t* __restrict__ region, const double* __restrict__ sigma_t,
                            const double* __restrict__ sigma_s, int max_regions,
                            const int64_t* __restrict__ off, const double* __restrict__ x,
                            double* __restrict__ y, const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const InstDev I = insts[b];
  __shared__ double blk[7 * NU * NU];
  const DsaStencil& S = st_[b];
  constexpr int nu = NU;
  for (int q = threadIdx.x; q < nu * nu; q += blockDim.x) {
    for (int z = 0; z < 5; ++z) blk[z * nu * nu + q] = S.blk[z][q];
    blk[5 * nu * nu + q] = S.St[q];
    blk[6 * nu * nu + q] = S.Ss[q];
  }
  __syncthreads();
  const int ncell = I.nx * I.ny;
  const double* xb = x + off[b];
  double* yb = y + off[b];
  for (int cell = blockIdx.x * blockDim.x + threadIdx.x; cell < ncell; cell += gridDim.x * blockDim.x) {
    const int i = cell % I.nx, k = cell / I.nx;
    const int rg = region[I.region_off + cell];
    const double ts = sigma_t[(int64_t)b * max_regions + rg];
    const double ss = sigma_s[(int64_t)b * max_regions + rg];
    double acc[NU];
    double xc[NU];
#pragma unroll
    for (int r = 0; r < nu; ++r) xc[r] = xb[(int64_t)cell * nu + r];
#pragma unroll
    for (int r = 0; r < nu; ++r) {
      double t = 0.0;
#pragma unroll
      for (int c = 0; c < nu; ++c)
        t += (blk[r * nu + c] + ts * blk[5 * nu * nu + r * nu + c] + ss * blk[6 * nu * nu + r * nu + c]) * xc[c];
      acc[r] = t;
    }
    const int nb[4] = {i > 0 ? cell - 1 : -1, i < I.nx - 1 ? cell + 1 : -1,
                       k > 0 ? cell - I.nx : -1, k < I.ny - 1 ? cell + I.nx : -1};
    for (int z = 0; z < 4; ++z) {
      if (nb[z] < 0) continue;
      const double* xn = xb + (int64_t)nb[z] * nu;
#pragma unroll
      for (int c = 0; c < nu; ++c) xc[c] = xn[c];
      const double* B = blk + (z + 1) * nu * nu;
#pragma unroll
      for (int r = 0; r < nu; ++r) {
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < nu; ++c) t += B[r * nu + c] * xc[c];
        acc[r] += t;
      }
    }
#pragma unroll
    for (int r = 0; r < nu; ++r) yb[(int64_t)cell * nu + r] = acc[r];
  }
}

// y = blockdiag(inv[region]) x
template <int NU>
__global__ void k_dsa_jacobi(const InstDev* __restrict__ insts, const DsaStencil* __restrict__ st_,
                             const int32_t* __restrict__ region, const double* __restrict__ inv,
                             int max_regions, const int64_t* __restrict__ off,
                             const double* __restrict__ x, double* __restrict__ y,
                             const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const InstDev I = insts[b];
  constexpr int nu = NU;
  const int ncell = I.nx * I.ny;
  for (int cell = blockIdx.x * blockDim.x + threadIdx.x; cell < ncell; cell += gridDim.x * blockDim.x) {
    const int rg = region[I.region_off + cell];
    const double* M = inv + ((int64_t)b * max_regions + rg) * DMAX * DMAX;
    double xc[NU];
#pragma unroll
    for (int c = 0; c < nu; ++c) xc[c] = x[off[b] + (int64_t)cell * nu + c];
#pragma unroll
    for (int r = 0; r < nu; ++r) {
      double t = 0.0;
#pragma unroll
      for (int c = 0; c < nu; ++c) t += M[r * nu + c] * xc[c];
      y[off[b] + (int64_t)cell * nu + r] = t;
    }
  }
}

// rhs = [ss v, m_x ss v (, m_y ss v)] per cell
__global__ void k_dsa_rhs(const InstDev* __restrict__ insts, const DsaStencil* __restrict__ st_,
                          const int32_t* __restrict__ region, const double* __restrict__ sigma_s,
                          int max_regions, const int64_t* __restrict__ off,
                          const double* __restrict__ v, double* __restrict__ rhs,
                          const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const InstDev I = insts[b];
  const DsaStencil& S = st_[b];
  const int nl = I.nloc, nu = S.nu;
  const int ncell = I.nx * I.ny;
  for (int cell = blockIdx.x * blockDim.x + threadIdx.x; cell < ncell; cell += gridDim.x * blockDim.x) {
    const double ss = sigma_s[(int64_t)b * max_regions + region[I.region_off + cell]];
    for (int l = 0; l < nl; ++l) {
      const double sv = ss * v[I.dof_off + (int64_t)cell * nl + l];
      rhs[off[b] + (int64_t)cell * nu + l] = sv;
      for (int d = 0; d < I.dim; ++d) rhs[off[b] + (int64_t)cell * nu + (1 + d) * nl + l] = S.m[d] * sv;
    }
  }
}

// z = v + dphi (the first nloc unknowns of every cell)
__global__ void k_dsa_out(const InstDev* __restrict__ insts, const DsaStencil* __restrict__ st_,
                          const int64_t* __restrict__ off, const double* __restrict__ u,
                          const double* __restrict__ v, double* __restrict__ z,
                          const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const InstDev I = insts[b];
  const int nl = I.nloc, nu = st_[b].nu;
  const int64_t nd = (int64_t)I.nx * I.ny * nl;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < nd;
       d += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = d / nl, l = d % nl;
    z[I.dof_off + d] = v[I.dof_off + d] + u[off[b] + cell * nu + l];
  }
}

// ------------------------------------------------------------------ host side
struct DsaSolver {
  rte_batch* b = nullptr;
  int32_t* d_live = nullptr;
  DsaStencil* d_st = nullptr;
  double* d_inv = nullptr;
  Krylov K;
  double* X = nullptr;     // solution (DSA space)
  double* T = nullptr;     // temporary (DSA space)
  double* rhs = nullptr;
  double* tol = nullptr;   // [n] absolute tolerances
  double* rn = nullptr;    // [n] rhs norms
  int restart = 0;
  int init(rte_batch* batch, int restart_);
  void release();
  int apply(const double* sigma_t, const double* sigma_s, const double* v, double* z, double inner_tol,
            int inner_max, const int32_t* active, int32_t* iters_host, hipStream_t s);
  int launch_apply(dim3 cg, hipStream_t s, const double* x, double* y, const double* st,
                   const double* ss, const int32_t* act) {
    if (b->dim == 2)
      hipLaunchKernelGGL(k_dsa_apply<12>, cg, dim3(256), 0, s, b->d_inst, d_st, b->d_region, st, ss,
                         b->max_regions, K.sp.d_off, x, y, act);
    else
      hipLaunchKernelGGL(k_dsa_apply<4>, cg, dim3(256), 0, s, b->d_inst, d_st, b->d_region, st, ss,
                         b->max_regions, K.sp.d_off, x, y, act);
    RTE_HIP(hipGetLastError());
    return RTE_OK;
  }
  int launch_jacobi(dim3 cg, hipStream_t s, const double* x, double* y, const int32_t* act) {
    if (b->dim == 2)
      hipLaunchKernelGGL(k_dsa_jacobi<12>, cg, dim3(256), 0, s, b->d_inst, d_st, b->d_region, d_inv,
                         b->max_regions, K.sp.d_off, x, y, act);
    else
      hipLaunchKernelGGL(k_dsa_jacobi<4>, cg, dim3(256), 0, s, b->d_inst, d_st, b->d_region, d_inv,
                         b->max_regions, K.sp.d_off, x, y, act);
    RTE_HIP(hipGetLastError());
    return RTE_OK;
  }
};

int DsaSolver::init(rte_batch* batch, int restart_) {
  b = batch;
  restart = restart_;
  std::vector<int64_t> lens(b->n_inst);
  for (int k = 0; k < b->n_inst; ++k) {
    const auto& I = b->inst[k];
    lens[k] = (int64_t)I.nx * I.ny * I.nloc * (1 + I.dim);
  }
  RTE_TRY(K.init(lens, restart, false));
  const int64_t tot = K.sp.total;
  if (hipMalloc(&d_st, sizeof(DsaStencil) * b->n_inst) != hipSuccess ||
      hipMalloc(&d_inv, sizeof(double) * b->n_inst * b->max_regions * DMAX * DMAX) != hipSuccess ||
      hipMalloc(&X, sizeof(double) * tot) != hipSuccess ||
      hipMalloc(&T, sizeof(double) * tot) != hipSuccess ||
      hipMalloc(&rhs, sizeof(double) * tot) != hipSuccess ||
      hipMalloc(&tol, sizeof(double) * b->n_inst) != hipSuccess ||
      hipMalloc(&rn, sizeof(double) * b->n_inst) != hipSuccess ||
      hipMalloc(&d_live, sizeof(int32_t) * b->n_inst) != hipSuccess)
    return RTE_ENOMEM;
  hipLaunchKernelGGL(k_dsa_setup, dim3((b->n_inst + 63) / 64), dim3(64), 0, 0, b->n_inst, b->d_inst,
                     b->d_ox, b->d_oy, b->d_w, d_st);
  RTE_HIP(hipGetLastError());
  RTE_HIP(hipDeviceSynchronize());
  return RTE_OK;
}

void DsaSolver::release() {
  K.release();
  for (void* p : {(void*)d_st, (void*)d_inv, (void*)X, (void*)T, (void*)rhs, (void*)tol, (void*)rn,
                  (void*)d_live})
    (void)hipFree(p);
  d_live = nullptr;
  d_st = nullptr;
  d_inv = X = T = rhs = tol = rn = nullptr;
}

__global__ void k_scale_tol(int n, const double* __restrict__ rn, double rtol, double* __restrict__ tol) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n) tol[b] = rtol * rn[b];
}

int DsaSolver::apply(const double* sigma_t, const double* sigma_s, const double* v, double* z,
                     double inner_tol, int inner_max, const int32_t* active, int32_t* iters_host,
                     hipStream_t s) {
  const int n = b->n_inst;
  const Space& sp = K.sp;
  const int mr = b->max_regions;
  const dim3 cg((unsigned)std::max(1, std::min(1024, (b->max_nx * b->max_ny + 255) / 256)), n);
  hipLaunchKernelGGL(k_dsa_blockinv, dim3((n * mr + 63) / 64), dim3(64), 0, s, n, mr, b->d_inst, d_st,
                     sigma_t, sigma_s, d_inv);
  hipLaunchKernelGGL(k_dsa_rhs, cg, dim3(256), 0, s, b->d_inst, d_st, b->d_region, sigma_s, mr,
                     sp.d_off, v, rhs, active);
  RTE_HIP(hipGetLastError());
  std::vector<int32_t> act(n, 1);
  if (active) RTE_HIP(hipMemcpyAsync(act.data(), active, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  RTE_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> iters(n, 0);
  // d_live: instances still iterating (converged instances drop out)
  RTE_HIP(hipMemcpyAsync(d_live, act.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
  RTE_HIP(hipMemsetAsync(X, 0, sizeof(double) * sp.total, s));
  RTE_TRY(knorm(sp, rhs, K.partA, rn, 1, d_live, s));
  hipLaunchKernelGGL(k_scale_tol, dim3((n + 63) / 64), dim3(64), 0, s, n, rn, inner_tol, tol);
  int done_iters = 0;
  std::vector<int32_t> jd(n), live_h = act;
  int status = RTE_OK;
  while (true) {
    // residual r = rhs - K X  (first cycle: X = 0 -> r = rhs)
    if (done_iters == 0) {
      RTE_TRY(kcopy(sp, rhs, T, d_live, s));
    } else {
      RTE_TRY(launch_apply(cg, s, X, T, sigma_t, sigma_s, d_live));
      RTE_TRY(kaxpby(sp, 1.0, rhs, -1.0, T, d_live, s));
    }
    RTE_HIP(hipMemcpyAsync(K.active, d_live, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    RTE_TRY(kstart(K, T, tol, s));
    int j = 0;
    for (; j < restart && done_iters + j < inner_max; ++j) {
      RTE_TRY(launch_jacobi(cg, s, K.v(j), T, K.active));
      RTE_TRY(launch_apply(cg, s, T, K.v(j + 1), sigma_t, sigma_s, K.active));
      RTE_TRY(arnoldi_mgs(K, j, s));
      if ((j + 1) % 8 == 0) {
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
    // X += M^{-1} (V y)
    RTE_HIP(hipMemsetAsync(T, 0, sizeof(double) * sp.total, s));
    RTE_TRY(kylov_solve_update(K, K.V, T, s));
    RTE_TRY(launch_jacobi(cg, s, T, K.v(0), d_live));
    RTE_TRY(kaxpby(sp, 1.0, K.v(0), 1.0, X, d_live, s));
    RTE_HIP(hipMemcpyAsync(jd.data(), K.jdone, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    // estimate of each instance: scal[b*8+2]
    std::vector<double> sc(8 * n), tl(n);
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
  const dim3 vg((unsigned)std::max<int64_t>(1, std::min<int64_t>((sp.max_len + 255) / 256, 1024)), n);
  (void)vg;
  RTE_HIP(hipMemcpyAsync(d_live, act.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_dsa_out, cg, dim3(256), 0, s, b->d_inst, d_st, sp.d_off, X, v, z, d_live);
  RTE_HIP(hipGetLastError());
  RTE_HIP(hipStreamSynchronize(s));
  if (iters_host)
    for (int q = 0; q < n; ++q) iters_host[q] = iters[q];
  return status;
}

// registry: one DSA solver per (batch, restart) kept alive with the batch
struct DsaCache {
  rte_batch* b;
  int restart;
  DsaSolver* s;
};
static std::vector<DsaCache> g_dsa;

DsaSolver* dsa_for(rte_batch* b, int restart) {
  for (auto& c : g_dsa)
    if (c.b == b && c.restart == restart) return c.s;
  auto* s = new DsaSolver();
  if (s->init(b, restart) != RTE_OK) {
    s->release();
    delete s;
    return nullptr;
  }
  g_dsa.push_back({b, restart, s});
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
              hipStream_t s) {
  DsaSolver* d = dsa_for(b, restart);
  if (!d) return RTE_ENOMEM;
  return d->apply(sigma_t, sigma_s, v, z, inner_tol, inner_max, active, iters, s);
}

}  // namespace rte

extern "C" int rte_dsa_apply(const rte_batch* cb, const double* sigma_t, const double* sigma_s,
                             const double* v, double* z, double inner_tol, int inner_max, int restart,
                             int32_t* stats_iters, void* stream) {
  auto* b = const_cast<rte_batch*>(cb);
  if (!b || !sigma_t || !sigma_s || !v || !z || inner_max < 1 || restart < 1 || restart > 500 ||
      !(inner_tol >= 0.0))
    return RTE_EINVAL;
  return rte::dsa_apply(b, sigma_t, sigma_s, v, z, inner_tol, inner_max, restart, nullptr,
                        stats_iters, reinterpret_cast<hipStream_t>(stream));
}
