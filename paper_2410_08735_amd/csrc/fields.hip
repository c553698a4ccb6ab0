// Cross sections that vary inside the cells (the variable-scattering problem
// of section 5.3): sigma(x) = sum_f theta_f s_f(x) with shape functions s_f
// sampled at the Gauss-Legendre points of every cell.  Every mass-weighted
// block int_T s_f e_a e_b (orthonormal tensor Legendre basis) is formed once
// here; the kernels of the sweep, the DSA and the ROM combine the blocks with
// each instance's coefficients.
#include <algorithm>
#include <cmath>
#include <vector>

#include "rte_internal.h"

namespace rte {

// B_f(cell)[a][b] = sum_q w_q s_f(x_q) e_a(x_q) e_b(x_q) over the nq x nq
// Gauss-Legendre points (point gy * nq + gx); with the orthonormal basis the
// volume factor h_x h_y / 4 and the normalisation 1 / (h_x h_y) leave w / 4.
// e_0 = 1, e_1 = sqrt3 s (times 1/sqrt h per axis, absorbed above).
__global__ void k_field_blocks(int nf, int64_t ncell, int nq, const double* __restrict__ gx,
                               const double* __restrict__ gw, const double* __restrict__ vals,
                               double* __restrict__ blk) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)nf * ncell) return;
  const double r3 = 1.7320508075688772935;
  const double* v = vals + id * nq * nq;
  double acc[16];
  for (int e = 0; e < 16; ++e) acc[e] = 0.0;
  for (int qy = 0; qy < nq; ++qy)
    for (int qx = 0; qx < nq; ++qx) {
      const double w = 0.25 * gw[qx] * gw[qy] * v[qy * nq + qx];
      const double ex[2] = {1.0, r3 * gx[qx]}, ey[2] = {1.0, r3 * gx[qy]};
      double e[4];
      for (int q = 0; q < 2; ++q)
        for (int p = 0; p < 2; ++p) e[p + 2 * q] = ex[p] * ey[q];
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 4; ++c) acc[4 * a + c] += w * e[a] * e[c];
    }
  double* o = blk + id * 16;
  for (int e = 0; e < 16; ++e) o[e] = acc[e];
}

// y = Sigma x per cell (4 moments) of every masked instance
__global__ void k_field_apply(const InstDev* __restrict__ insts, const double* __restrict__ fblk, int nf,
                              int64_t fcell, const double* __restrict__ theta, int max_regions,
                              const double* __restrict__ x, double* __restrict__ y, int add,
                              const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const InstDev I = insts[b];
  const int64_t nc = (int64_t)I.nx * I.ny;
  const double* th = theta + (int64_t)b * max_regions;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
    double B[16];
    field_block(fblk, nf, fcell, c, th, B);
    const double* xc = x + I.dof_off + 4 * c;
    double* yc = y + I.dof_off + 4 * c;
    const double x0 = xc[0], x1 = xc[1], x2 = xc[2], x3 = xc[3];
    for (int a = 0; a < 4; ++a) {
      const double v = B[4 * a] * x0 + B[4 * a + 1] * x1 + B[4 * a + 2] * x2 + B[4 * a + 3] * x3;
      yc[a] = add ? yc[a] + v : v;
    }
  }
}

int field_apply(const rte_batch* b, const double* theta, const double* x, double* y, bool add,
                const int32_t* active, hipStream_t s) {
  if (b->n_fields <= 0) return RTE_EINVAL;
  const dim3 grid((unsigned)std::min<int64_t>((b->field_ncell + 255) / 256, 1024), b->n_inst);
  hipLaunchKernelGGL(k_field_apply, grid, dim3(256), 0, s, b->d_inst, b->d_fblk, b->n_fields, b->field_ncell,
                     theta, b->max_regions, x, y, add ? 1 : 0, active);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on the Legendre recurrence)
static void gl_rule(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;  // ascending
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

}  // namespace rte

extern "C" int rte_batch_set_fields(rte_batch* b, int n_fields, int nq, const double* values) {
  if (!b || n_fields < 1 || n_fields > 16 || nq < 1 || nq > 16 || !values || b->dim != 2 || !b->uniform ||
      n_fields > b->max_regions)
    return RTE_EINVAL;
  for (const auto& I : b->inst)
    if (I.n_regions < n_fields) return RTE_EINVAL;
  const int64_t ncell = (int64_t)b->inst[0].nx * b->inst[0].ny;
  std::vector<double> gx, gw;
  rte::gl_rule(nq, gx, gw);
  double *d_vals = nullptr, *d_gx = nullptr, *blk = nullptr;
  const size_t nv = (size_t)n_fields * ncell * nq * nq;
  if (hipMalloc(&d_vals, sizeof(double) * nv) != hipSuccess ||
      hipMalloc(&d_gx, sizeof(double) * 2 * nq) != hipSuccess ||
      hipMalloc(&blk, sizeof(double) * n_fields * ncell * 16) != hipSuccess) {
    (void)hipFree(d_vals);
    (void)hipFree(d_gx);
    (void)hipFree(blk);
    return RTE_ENOMEM;
  }
  std::vector<double> gxw(gx);
  gxw.insert(gxw.end(), gw.begin(), gw.end());
  int st = RTE_OK;
  if (hipMemcpy(d_vals, values, sizeof(double) * nv, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_gx, gxw.data(), sizeof(double) * 2 * nq, hipMemcpyHostToDevice) != hipSuccess)
    st = RTE_EHIP;
  if (st == RTE_OK) {
    const int64_t n = (int64_t)n_fields * ncell;
    hipLaunchKernelGGL(rte::k_field_blocks, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, 0, n_fields, ncell, nq,
                       d_gx, d_gx + nq, d_vals, blk);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) st = RTE_EHIP;
  }
  (void)hipFree(d_vals);
  (void)hipFree(d_gx);
  if (st != RTE_OK) {
    (void)hipFree(blk);
    return st;
  }
  (void)hipFree(b->d_fblk);
  b->d_fblk = blk;
  b->n_fields = n_fields;
  b->field_ncell = ncell;
  // plans were tuned for the region kernels; cached operator graphs launch them
  b->plan[0].tuned = b->plan[1].tuned = false;
  b->plan[0].variant = b->plan[1].variant = 0;
  ++b->gen;
  return RTE_OK;
}
