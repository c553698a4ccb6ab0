// ROMSAD preconditioner (section 4.3) and greedy ROM construction (section
// 4.4, App. B) on the GPU.
//
// The basis U_r lives in psi-space, [r][n_ord][ndof] with ordinates in their
// original order.  For region-wise constant cross sections the reduced
// operator is affine (eq. of the affine assumption):
//   U^T A(mu) U = A_D + sum_R sigma_t,R G_R - sum_R sigma_s,R S_R,
//   A_D = sum_j U_j^T D_j U_j, G_R = sum_j U_j^T M_R U_j, S_R = W_1^T M_R W_w,
// with M_R the mass matrix restricted to region R (the identity on the dofs
// of region-R cells in the orthonormal basis).  All three are region-masked
// inner products, formed column by column as the basis grows.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "fgmres.h"

namespace rte {

constexpr int ROM_RMAX = 64;     // maximum basis size
constexpr int ROM_REGMAX = 16;   // maximum number of regions of a ROM

// What the online kernels read of the ROM that serves one instance.
struct RomDev {
  const double *W1, *Ww, *AD, *G, *S;
  int32_t r, ld, nreg, pad;
  int64_t nd;
};

// ------------------------------------------------------------------ kernels
__device__ __forceinline__ double bsum256(double v, double* sh) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
  return t;
}

// psi-space advection y_j = D_j u_j (upwind DG operator of section 2.3,
// inflow faces excluded), one thread per (ordinate, cell).
__global__ void k_advect(int dim, int nx, int ny, double hx, double hy, int n_ord,
                         const double* __restrict__ ox, const double* __restrict__ oy,
                         const double* __restrict__ u, double* __restrict__ y) {
  const int j = blockIdx.y;
  const int ncell = nx * ny;
  const int nl = dim == 2 ? 4 : 2;
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= ncell || j >= n_ord) return;
  const double r3 = 1.7320508075688772935;
  const double o1 = ox[j], o2 = dim == 2 ? oy[j] : 0.0;
  const double sx = o1 < 0.0 ? -1.0 : 1.0, sy = o2 < 0.0 ? -1.0 : 1.0;
  const double a = fabs(o1) / hx, b = fabs(o2) / hy;
  const int64_t nd = (int64_t)ncell * nl;
  const double* uj = u + (int64_t)j * nd;
  double* yj = y + (int64_t)j * nd;
  const int i = cell % nx, k = cell / nx;
  if (dim == 1) {
    const double u0 = uj[2 * cell], u1 = sx * uj[2 * cell + 1];
    double y0 = a * (u0 + r3 * u1), y1 = a * (-r3 * u0 + 3.0 * u1);
    const int in = i - (int)sx;
    if (in >= 0 && in < nx) {
      const double T = uj[2 * in] + r3 * sx * uj[2 * in + 1];
      y0 -= a * T;
      y1 += a * r3 * T;
    }
    yj[2 * cell] = y0;
    yj[2 * cell + 1] = sx * y1;
    return;
  }
  const double* uc = uj + 4 * (int64_t)cell;
  const double m[4] = {uc[0], sx * uc[1], sy * uc[2], sx * sy * uc[3]};
  double yy[4];
  // a (K (x) I) m + b (I (x) K) m
  yy[0] = a * (m[0] + r3 * m[1]) + b * (m[0] + r3 * m[2]);
  yy[1] = a * (-r3 * m[0] + 3.0 * m[1]) + b * (m[1] + r3 * m[3]);
  yy[2] = a * (m[2] + r3 * m[3]) + b * (-r3 * m[0] + 3.0 * m[2]);
  yy[3] = a * (-r3 * m[2] + 3.0 * m[3]) + b * (-r3 * m[1] + 3.0 * m[3]);
  const int ixn = i - (int)sx;
  if (a != 0.0 && ixn >= 0 && ixn < nx) {
    const double* un = uj + 4 * (int64_t)(k * nx + ixn);
    const double T0 = un[0] + r3 * sx * un[1];
    const double T1 = sy * un[2] + r3 * sx * sy * un[3];
    yy[0] -= a * T0;
    yy[1] += a * r3 * T0;
    yy[2] -= a * T1;
    yy[3] += a * r3 * T1;
  }
  const int kyn = k - (int)sy;
  if (b != 0.0 && kyn >= 0 && kyn < ny) {
    const double* un = uj + 4 * (int64_t)(kyn * nx + i);
    const double T0 = un[0] + r3 * sy * un[2];
    const double T1 = sx * un[1] + r3 * sx * sy * un[3];
    yy[0] -= b * T0;
    yy[2] += b * r3 * T0;
    yy[1] -= b * T1;
    yy[3] += b * r3 * T1;
  }
  double* yc = yj + 4 * (int64_t)cell;
  yc[0] = yy[0];
  yc[1] = sx * yy[1];
  yc[2] = sy * yy[2];
  yc[3] = sx * sy * yy[3];
}

// W1 = sum_j u_j, Ww = sum_j w_j u_j for one psi-space column
__global__ void k_angle_sums(int n_ord, int64_t nd, const double* __restrict__ w,
                             const double* __restrict__ u, double* __restrict__ w1,
                             double* __restrict__ ww) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nd) return;
  double s1 = 0.0, sw = 0.0;
  for (int j = 0; j < n_ord; ++j) {
    const double v = u[(int64_t)j * nd + e];
    s1 += v;
    sw += w[j] * v;
  }
  w1[e] = s1;
  ww[e] = sw;
}

// Region-masked inner products of x with vectors Y_i (stride ystride):
// part[(i * nch + c) * nreg + R] over elements of chunk c.
constexpr int MD_CHUNK = 2048;
__global__ void k_mdot(int64_t len, int64_t nd, int nl, const int32_t* __restrict__ region,
                       int nreg, const double* __restrict__ x, const double* __restrict__ Y,
                       int64_t ystride, double* __restrict__ part, int nch) {
  __shared__ double sh[4];
  const int i = blockIdx.y, c = blockIdx.x;
  const double* yi = Y + (int64_t)i * ystride;
  double acc[ROM_REGMAX];
  for (int R = 0; R < nreg; ++R) acc[R] = 0.0;
  const int64_t start = (int64_t)c * MD_CHUNK;
  const int64_t end = min(len, start + (int64_t)MD_CHUNK);
  for (int64_t e = start + threadIdx.x; e < end; e += blockDim.x) {
    const int cell = (int)((e % nd) / nl);
    const int R = region[cell];
    acc[R] += x[e] * yi[e];
  }
  for (int R = 0; R < nreg; ++R) {
    const double t = bsum256(acc[R], sh);
    if (threadIdx.x == 0) part[((int64_t)i * nch + c) * nreg + R] = t;
  }
}

__global__ void k_mdot_sum(int ny_, int nch, int nreg, const double* __restrict__ part,
                           double* __restrict__ out) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ny_ * nreg) return;
  const int i = id / nreg, R = id % nreg;
  double t = 0.0;
  for (int c = 0; c < nch; ++c) t += part[((int64_t)i * nch + c) * nreg + R];
  out[id] = t;
}

// place the new row/column r of A_D, G_R, S_R from the multi-dot results
// d_adc[i] = <U_i, DU_r>, d_adr[i] = <U_r, DU_i>, d_g[i][R] = <U_i, U_r>_R,
// d_sc[i][R] = <W1_i, Ww_r>_R, d_sr[i][R] = <W1_r, Ww_i>_R   (i = 0..r)
__global__ void k_place(int r, int rcap, int nreg, const double* __restrict__ d_adc,
                        const double* __restrict__ d_adr, const double* __restrict__ d_g,
                        const double* __restrict__ d_sc, const double* __restrict__ d_sr,
                        double* __restrict__ AD, double* __restrict__ G, double* __restrict__ S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > r) return;
  double ac = 0.0, ar = 0.0;
  for (int R = 0; R < nreg; ++R) {
    ac += d_adc[i * nreg + R];
    ar += d_adr[i * nreg + R];
  }
  AD[(int64_t)i * rcap + r] = ac;
  AD[(int64_t)r * rcap + i] = ar;
  for (int R = 0; R < nreg; ++R) {
    const int64_t base = (int64_t)R * rcap * rcap;
    G[base + (int64_t)i * rcap + r] = d_g[i * nreg + R];
    G[base + (int64_t)r * rcap + i] = d_g[i * nreg + R];
    S[base + (int64_t)i * rcap + r] = d_sc[i * nreg + R];
    S[base + (int64_t)r * rcap + i] = d_sr[i * nreg + R];
  }
}

// g[b][k] partials: sum over a chunk of W[k][e] * (sigma_s(cell) v[b][e]), with
// W = W_1 (which = 0) or W_w (which = 1) of the instance's ROM.
constexpr int PJ_CHUNK = 2048;
__global__ void k_rom_project(const InstDev* __restrict__ insts, const int32_t* __restrict__ region,
                              const double* __restrict__ sigma_s, int max_regions,
                              const RomDev* __restrict__ tab, int which,
                              const double* __restrict__ v, double* __restrict__ part, int nch,
                              const int32_t* __restrict__ active) {
  __shared__ double sh[4];
  const int b = blockIdx.y, c = blockIdx.x;
  if (active && !active[b]) return;
  const InstDev I = insts[b];
  const RomDev R = tab[b];
  const double* __restrict__ W = which ? R.Ww : R.W1;
  const int64_t nd = R.nd;
  const int r = R.r;
  const int64_t start = (int64_t)c * PJ_CHUNK;
  if (start >= nd) {  // chunk beyond this instance: zero partials
    for (int k = threadIdx.x; k < r; k += blockDim.x) part[((int64_t)b * nch + c) * ROM_RMAX + k] = 0.0;
    return;
  }
  double sv[PJ_CHUNK / 256];
#pragma unroll
  for (int q = 0; q < PJ_CHUNK / 256; ++q) {
    const int64_t e = start + threadIdx.x + 256 * q;
    double x = 0.0;
    if (e < nd) {
      x = v[I.dof_off + e];
      if (sigma_s) x *= sigma_s[(int64_t)b * max_regions + region[I.region_off + (int)(e / I.nloc)]];
    }
    sv[q] = x;
  }
  for (int k = 0; k < r; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < PJ_CHUNK / 256; ++q) {
      const int64_t e = start + threadIdx.x + 256 * q;
      if (e < nd) acc += W[(int64_t)k * nd + e] * sv[q];
    }
    const double t = bsum256(acc, sh);
    if (threadIdx.x == 0) part[((int64_t)b * nch + c) * ROM_RMAX + k] = t;
  }
}

// The same projection for a batch served by one ROM, on the matrix cores:
// g[b][k] = sum_e W[k][e] (sigma_s v_b)[e] is the product of the batch's
// vectors (instances x DoFs) with the basis (DoFs x rank).  A wave takes 16
// instances and every rank column over PM_DOF DoFs, in steps of 32 DoFs with
// v_mfma_f64_16x16x4: lane l supplies instance l % 16 (A) and basis row
// 16 c + l % 16 (B) at DoFs 8 (l / 16) + i of the step for i = 0..7, so each
// lane reads runs of 8 consecutive DoFs; the accumulator of column block c
// holds, in lane l and item j, instance l / 16 + 4 j and rank column
// 16 c + l % 16.  Partial sums per (instance, DoF chunk) as above.
constexpr int PM_DOF = 256;
// DoFs per work group of the LDS-staged projection and lift: short chunks give
// a launch many work groups (16 KiB of LDS each at rank 32) to hide the load
// latency, at the cost of more partial sums for the projection
constexpr int PJL_DOF = 64, LFL_DOF = 64;
typedef double rom_d4 __attribute__((ext_vector_type(4)));
template <int NL>  // moments per cell (4 in X-Y, 2 in slab geometry)
__global__ void __launch_bounds__(256) k_rom_project_mfma(const InstDev* __restrict__ insts,
                                                          const int32_t* __restrict__ region,
                                                          const double* __restrict__ sigma_s, int max_regions,
                                                          const double* __restrict__ W, int r, int nd,
                                                          int n, const double* __restrict__ v,
                                                          double* __restrict__ part, int nch,
                                                          const int32_t* __restrict__ active) {
  const int lane = threadIdx.x & 63;
  const int chunk = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= nch) return;  // the whole wave
  const int row = lane & 15, kq = lane >> 4;
  const int b = blockIdx.y * 16 + row;
  const bool on = b < n && (!active || active[b]);
  const double* vb = v;
  const int32_t* rb = region;
  const double* sb = nullptr;
  if (on) {
    const InstDev I = insts[b];
    vb = v + I.dof_off;
    rb = region + I.region_off;
    if (sigma_s) sb = sigma_s + (int64_t)b * max_regions;
  }
  const int ncb = (r + 15) >> 4;
  rom_d4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = rom_d4{0.0, 0.0, 0.0, 0.0};
  const int e0 = chunk * PM_DOF;
  for (int st = 0; st < PM_DOF / 32; ++st) {
    const int eb = e0 + st * 32 + kq * 8;  // multiple of 8, so of NL
    if (eb - kq * 8 >= nd) break;  // past the end for the whole wave
    double a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = eb + i;
      a[i] = (on && e < nd) ? vb[e] : 0.0;
    }
    if (sb) {
#pragma unroll
      for (int q = 0; q < 8 / NL; ++q) {  // the run covers 8 / NL whole cells
        const int cell = eb / NL + q;
        const double sg = (on && cell * NL < nd) ? sb[rb[cell]] : 0.0;
#pragma unroll
        for (int i = 0; i < NL; ++i) a[q * NL + i] *= sg;
      }
    }
    double w[4][8];  // every basis value of the step first: the loads overlap
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int k = 16 * c + row;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = eb + i;
        w[c][i] = (c < ncb && k < r && e < nd) ? W[(int64_t)k * nd + e] : 0.0;
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < ncb)
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], w[c][i], acc[c], 0, 0, 0);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c >= ncb) break;
    const int k = 16 * c + row;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int bi = blockIdx.y * 16 + kq + 4 * j;
      if (bi < n && k < r) part[((int64_t)bi * nch + chunk) * ROM_RMAX + k] = acc[c][j];
    }
  }
}

// Stages the chunk [e0, e0 + ne) of r basis vectors in LDS in the order the
// projection's matrix-core steps read them: the value for column block c,
// step st, item i, lane (kq, row) (basis row 16 c + row, DoF
// e0 + 32 st + 8 kq + i) at (((c NS + st) 8 + i) 4 + kq) 16 + row, so that
// one read of item i by the 64 lanes of a wave covers 64 consecutive doubles
// (no bank conflicts); zeros past ne and for rows at or past r.  Eight
// global reads in flight per thread.
template <int CH>
__device__ __forceinline__ void stage_basis_mfma_b(const double* __restrict__ W, int r, int nd, int e0, int ne,
                                                   double* Wl) {
  constexpr int NS = CH / 32;
  const int ncb = (r + 15) >> 4;
  const int total = ncb * NS * 8 * 64;  // slots
  // thread by slot: the LDS writes of a wave are 64 consecutive doubles; the
  // reads gather 16 basis rows (from the cache after the first touch)
  for (int base = 0; base < total; base += 8 * (int)blockDim.x) {
    double w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int sl = base + u * (int)blockDim.x + (int)threadIdx.x;
      const int row = sl & 15, kq = (sl >> 4) & 3, i = (sl >> 6) & 7, cst = sl >> 9;
      const int st = cst % NS, c = cst / NS;
      const int k = 16 * c + row, el = 32 * st + 8 * kq + i;
      const bool in = sl < total && k < r && el < ne;
      const double x = W[(int64_t)(in ? k : 0) * nd + e0 + (in ? el : 0)];
      w[u] = in ? x : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int sl = base + u * (int)blockDim.x + (int)threadIdx.x;
      if (sl < total) Wl[sl] = w[u];
    }
  }
}

// The same projection with each basis chunk shared by the four waves of a
// work group: a work group takes 64 instances (16 per wave, as above) and one
// chunk of PJL_DOF DoFs, stages the chunk of every basis vector (r x PJL_DOF
// values) in LDS once and lets the four waves read it there, so the basis is
// read once per 64 instances instead of once per 16.  The runs of v are read
// as 16-byte pairs at clamped addresses (a pair past the end, or of an
// inactive instance, reads the instance's first pair and becomes zero), each
// cell's region with its run and sigma_s from the instance's table.
template <int NL>
__global__ void __launch_bounds__(256) k_rom_project_lds(const InstDev* __restrict__ insts,
                                                         const int32_t* __restrict__ region,
                                                         const double* __restrict__ sigma_s, int max_regions,
                                                         const double* __restrict__ W, int r, int nd, int n,
                                                         const double* __restrict__ v, double* __restrict__ part,
                                                         int nch, const int32_t* __restrict__ active) {
  extern __shared__ double Wl[];  // the basis chunk in the order of the steps (stage_basis_mfma_b)
  const int chunk = blockIdx.x;
  const int e0 = chunk * PJL_DOF;
  const int ne = min(PJL_DOF, nd - e0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4;
  const int b = blockIdx.y * 64 + wave * 16 + row;
  const bool on = b < n && (!active || active[b]);
  const double* vb = v;
  const int32_t* rb = region;
  const double* sb = sigma_s;
  if (on) {
    const InstDev I = insts[b];
    vb = v + I.dof_off;
    rb = region + I.region_off;
    if (sigma_s) sb = sigma_s + (int64_t)b * max_regions;
  }
  const int ncb = (r + 15) >> 4;
  // every run of v the wave needs first (clamped addresses), then the
  // regions of their cells, then sigma_s: three rounds of loads, each all in
  // flight together, and the basis chunk while the last is
  constexpr int NS = PJL_DOF / 32, NC = 8 / NL;  // steps; cells per run
  double a[NS][8];
#pragma unroll
  for (int st = 0; st < NS; ++st) {  // steps past the chunk's end add zeros
    const int el = st * 32 + kq * 8;  // multiple of 8, so of NL
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = e0 + el + 2 * i;
      const bool in = on && e < nd;
      const double2 x = *reinterpret_cast<const double2*>(vb + (in ? e : 0));
      a[st][2 * i] = in ? x.x : 0.0;
      a[st][2 * i + 1] = in ? x.y : 0.0;
    }
  }
  if (sigma_s) {
    int rg[NS][NC];
#pragma unroll
    for (int st = 0; st < NS; ++st)
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const int cell = (e0 + st * 32 + kq * 8) / NL + q;
        rg[st][q] = rb[(on && cell * NL < nd) ? cell : 0];
      }
#pragma unroll
    for (int st = 0; st < NS; ++st)
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const int cell = (e0 + st * 32 + kq * 8) / NL + q;
        const double sg = (on && cell * NL < nd) ? sb[rg[st][q]] : 0.0;
#pragma unroll
        for (int i = 0; i < NL; ++i) a[st][q * NL + i] *= sg;
      }
  }
  stage_basis_mfma_b<PJL_DOF>(W, r, nd, e0, ne, Wl);
  __syncthreads();
  rom_d4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = rom_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int st = 0; st < NS; ++st) {
    const int el = st * 32 + kq * 8;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < ncb) {
        const double* wr = Wl + ((c * NS + st) * 8 * 4 + kq) * 16 + row;
#pragma unroll
        for (int i = 0; i < 8; ++i)
          acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st][i], wr[i * 64], acc[c], 0, 0, 0);
      }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c >= ncb) break;
    const int k = 16 * c + row;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int bi = blockIdx.y * 64 + wave * 16 + kq + 4 * j;
      if (bi < n && k < r) part[((int64_t)bi * nch + chunk) * ROM_RMAX + k] = acc[c][j];
    }
  }
}

// g[b][k] = the sum over chunks of part, four waves per instance: wave q sums
// the q-th quarter of the chunks in order (lane k: basis column k), and wave
// 0 adds the four quarter sums in order.
__global__ void __launch_bounds__(256) k_rom_gsum4(int n, int nch, const RomDev* __restrict__ tab,
                                                   const double* __restrict__ part, double* __restrict__ g,
                                                   const int32_t* __restrict__ active) {
  __shared__ double qs[3][64];
  const int b = blockIdx.x, k = threadIdx.x & 63, q = threadIdx.x >> 6;
  if (active && !active[b]) return;  // the whole work group
  const int r = tab[b].r;
  const int c0 = (int)((int64_t)nch * q / 4), c1 = (int)((int64_t)nch * (q + 1) / 4);
  double t = 0.0;
  if (k < r) {
    const double* pb = part + (int64_t)b * nch * ROM_RMAX + k;
#pragma unroll 8
    for (int c = c0; c < c1; ++c) t += pb[(int64_t)c * ROM_RMAX];
  }
  if (q > 0) qs[q - 1][k] = t;
  __syncthreads();
  if (q == 0 && k < r) g[(int64_t)b * ROM_RMAX + k] = ((t + qs[0][k]) + qs[1][k]) + qs[2][k];
}

__global__ void k_rom_gsum(int n, int nch, const RomDev* __restrict__ tab, const double* __restrict__ part,
                           double* __restrict__ g, const int32_t* __restrict__ active) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * ROM_RMAX) return;
  const int b = id / ROM_RMAX, k = id % ROM_RMAX;
  if ((active && !active[b]) || k >= tab[b].r) return;
  double t = 0.0;
  for (int c = 0; c < nch; ++c) t += part[((int64_t)b * nch + c) * ROM_RMAX + k];
  g[(int64_t)b * ROM_RMAX + k] = t;
}

// c = (A_D + sum_R st_R G_R - ss_R S_R)^{-1} g, LU with partial pivoting on
// the matrix augmented by g, one work group of 256 threads per instance: the
// pivot search in one wave, row swaps and the elimination over all threads.
// lu_out / piv_out (nullable, [n][ROM_RMAX][ROM_RMAX] and [n][ROM_RMAX]) keep
// the factors: L (unit, below the diagonal) and U in the final row order, and
// the row permutation (row i of the factors is row piv[i] of A_r; piv[0] =
// -1: singular).
__global__ void __launch_bounds__(256) k_rom_solve(int n, const RomDev* __restrict__ tab,
                                                   const double* __restrict__ sigma_t,
                                                   const double* __restrict__ sigma_s, int max_regions,
                                                   const double* __restrict__ g, double* __restrict__ c,
                                                   int gstride, int32_t* __restrict__ singular,
                                                   const int32_t* __restrict__ active,
                                                   double* __restrict__ lu_out = nullptr,
                                                   int32_t* __restrict__ piv_out = nullptr) {
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  const RomDev Rd = tab[b];
  const int r = Rd.r, ld = Rd.ld, nreg = Rd.nreg;
  const double* __restrict__ AD = Rd.AD;
  const double* __restrict__ G = Rd.G;
  const double* __restrict__ S = Rd.S;
  __shared__ double A[ROM_RMAX][ROM_RMAX + 1];  // column r holds the right-hand side
  __shared__ double st_s[ROM_REGMAX], ss_s[ROM_REGMAX];
  __shared__ double amax_s, cb[ROM_RMAX];
  __shared__ int piv_s, perm_s[ROM_RMAX];
  const int t = threadIdx.x;
  for (int R = t; R < nreg; R += blockDim.x) {
    st_s[R] = sigma_t[(int64_t)b * max_regions + R];
    ss_s[R] = sigma_s[(int64_t)b * max_regions + R];
  }
  __syncthreads();
  for (int idx = t; idx < r * r; idx += blockDim.x) {
    const int i = idx / r, k = idx - i * r;
    double v = AD[(int64_t)i * ld + k];
    for (int R = 0; R < nreg; ++R) {
      const int64_t q = (int64_t)R * ld * ld + (int64_t)i * ld + k;
      v += st_s[R] * G[q] - ss_s[R] * S[q];
    }
    A[i][k] = v;
  }
  for (int i = t; i < r; i += blockDim.x) A[i][r] = g[(int64_t)b * gstride + i];
  __syncthreads();
  if (t < 64) {  // max |A| for the singularity threshold
    double m = 0.0;
    for (int idx = t; idx < r * r; idx += 64) m = fmax(m, fabs(A[idx / r][idx % r]));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (t == 0) amax_s = m;
  }
  __syncthreads();
  bool sing = false;
  for (int col = 0; col < r; ++col) {
    if (t < 64) {  // first row of the largest |A[i][col]|, i >= col
      const int i = col + t;
      double best = i < r ? fabs(A[i][col]) : -1.0;
      int bi = i;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (t == 0) piv_s = bi;
    }
    __syncthreads();
    const int p = piv_s;
    if (t == 0) {  // the row permutation so far
      if (col == 0)
        for (int i = 0; i < r; ++i) perm_s[i] = i;
      const int q = perm_s[col];
      perm_s[col] = perm_s[p];
      perm_s[p] = q;
    }
    if (p != col)
      for (int k = t; k <= r; k += blockDim.x) {
        const double tmp = A[col][k];
        A[col][k] = A[p][k];
        A[p][k] = tmp;
      }
    __syncthreads();
    const double d = A[col][col];
    if (!(fabs(d) > 1e-14 * amax_s)) {
      sing = true;
      break;
    }
    for (int i = col + 1 + t; i < r; i += blockDim.x) A[i][col] /= d;  // the multipliers
    __syncthreads();
    const int w = r - col;  // columns col + 1 .. r (the last is the right-hand side)
    for (int idx = t; idx < (r - col - 1) * w; idx += blockDim.x) {
      const int i = col + 1 + idx / w, k = col + 1 + idx % w;
      A[i][k] -= A[i][col] * A[col][k];
    }
    __syncthreads();
  }
  if (lu_out) {
    if (sing) {
      if (t == 0) piv_out[(int64_t)b * ROM_RMAX] = -1;
    } else {
      double* f = lu_out + (int64_t)b * ROM_RMAX * ROM_RMAX;
      for (int idx = t; idx < r * r; idx += blockDim.x) f[(idx / r) * ROM_RMAX + idx % r] = A[idx / r][idx % r];
      for (int i = t; i < r; i += blockDim.x) piv_out[(int64_t)b * ROM_RMAX + i] = perm_s[i];
    }
  }
  if (t == 0) {
    double* out = c + (int64_t)b * gstride;
    if (sing) {
      for (int i = 0; i < r; ++i) out[i] = 0.0;
      if (singular) singular[b] = 1;
    } else {
      for (int i = r - 1; i >= 0; --i) {
        double v = A[i][r];
        for (int k = i + 1; k < r; ++k) v -= A[i][k] * cb[k];
        cb[i] = v / A[i][i];
        out[i] = cb[i];
      }
    }
  }
}

// c = A_r^{-1} g from the factors k_rom_solve kept, one wave per instance,
// lane i holding row i of the factors in registers and entry i of the
// solution: x = P g, then forward substitution with the unit L and back
// substitution with U, column by column (each column's entry broadcast across
// the wave).  An instance whose factorisation was singular gets c = 0.
__global__ void __launch_bounds__(64) k_rom_lusolve(int n, const RomDev* __restrict__ tab,
                                                    const double* __restrict__ lu, const int32_t* __restrict__ piv,
                                                    const double* __restrict__ g, double* __restrict__ c,
                                                    int gstride, const int32_t* __restrict__ active) {
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  const int r = tab[b].r, t = threadIdx.x;
  const int32_t* pv = piv + (int64_t)b * ROM_RMAX;
  double* out = c + (int64_t)b * gstride;
  if (pv[0] < 0) {
    if (t < r) out[t] = 0.0;
    return;
  }
  const int ti = t < r ? t : 0;  // lanes past the rank read row 0 and take no part
  const double* f = lu + (int64_t)b * ROM_RMAX * ROM_RMAX + (int64_t)ti * ROM_RMAX;
  double row[ROM_RMAX];
#pragma unroll
  for (int k = 0; k < ROM_RMAX; ++k) row[k] = k < r ? f[k] : 0.0;
  double xi = g[(int64_t)b * gstride + pv[ti]];
#pragma unroll
  for (int col = 0; col + 1 < ROM_RMAX; ++col) {
    if (col + 1 < r) {
      const double xc = __shfl(xi, col, 64);
      if (t > col) xi -= row[col] * xc;
    }
  }
#pragma unroll
  for (int k = ROM_RMAX - 1; k >= 0; --k) {
    if (k >= r) continue;
    if (t == k) xi = xi / row[k];
    const double xk = __shfl(xi, k, 64);
    if (t < k) xi -= row[k] * xk;
  }
  if (t < r) out[t] = xi;
}

// z = v + sum_k c[b][k] Ww[k]
__global__ void k_rom_lift(const InstDev* __restrict__ insts, const RomDev* __restrict__ tab,
                           const double* __restrict__ v, const double* __restrict__ c, double* __restrict__ z,
                           const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const RomDev R = tab[b];
  const double* __restrict__ Ww = R.Ww;
  const int r = R.r;
  const int64_t nd = R.nd;
  __shared__ double cs[ROM_RMAX];
  for (int k = threadIdx.x; k < r; k += blockDim.x) cs[k] = c[(int64_t)b * ROM_RMAX + k];
  __syncthreads();
  const InstDev I = insts[b];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nd;
       e += (int64_t)gridDim.x * blockDim.x) {
    double acc = v ? v[I.dof_off + e] : 0.0;
    for (int k = 0; k < r; ++k) acc += cs[k] * Ww[(int64_t)k * nd + e];
    z[I.dof_off + e] = acc;
  }
}

// The same lift for a batch served by one ROM, on the matrix cores:
// Z (instances x DoFs) = C (instances x rank) W (rank x DoFs) + V.  A wave
// takes 16 instances over PL_DOF DoFs in tiles of 16 DoFs, ceil(r / 4)
// v_mfma_f64_16x16x4 per tile: lane l supplies C[l % 16][4 s + l / 16] (held in
// registers) and W[4 s + l / 16][tile + l % 16]; lane l, item j of the result
// is instance l / 16 + 4 j at DoF tile + l % 16.
constexpr int PL_DOF = 256;
__global__ void __launch_bounds__(256) k_rom_lift_mfma(const InstDev* __restrict__ insts,
                                                       const double* __restrict__ W, int r, int nd, int n,
                                                       const double* __restrict__ v,
                                                       const double* __restrict__ c, double* __restrict__ z,
                                                       const int32_t* __restrict__ active) {
  const int lane = threadIdx.x & 63;
  const int e0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * PL_DOF;
  if (e0 >= nd) return;  // the whole wave
  const int row = lane & 15, kq = lane >> 4;
  const int ba = blockIdx.y * 16 + row;
  double ca[ROM_RMAX / 4];
#pragma unroll
  for (int st = 0; st < ROM_RMAX / 4; ++st) {
    const int k = 4 * st + kq;
    ca[st] = (ba < n && k < r) ? c[(int64_t)ba * ROM_RMAX + k] : 0.0;
  }
  int64_t off[4];
  bool on[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int bo = blockIdx.y * 16 + kq + 4 * j;
    on[j] = bo < n && (!active || active[bo]);
    off[j] = on[j] ? insts[bo].dof_off : 0;
  }
  const int ns = (r + 3) >> 2;
#pragma unroll 2
  for (int t = 0; t < PL_DOF / 16; ++t) {
    if (e0 + t * 16 >= nd) break;  // the whole wave
    const int e = e0 + t * 16 + row;
    double wv[ROM_RMAX / 4];  // every basis value of the tile first: the loads overlap
#pragma unroll
    for (int st = 0; st < ROM_RMAX / 4; ++st) {
      const int k = 4 * st + kq;
      wv[st] = (st < ns && k < r && e < nd) ? W[(int64_t)k * nd + e] : 0.0;
    }
    rom_d4 acc = rom_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < ROM_RMAX / 4; ++st)
      if (st < ns) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[st], wv[st], acc, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (on[j] && e < nd) z[off[j] + e] = (v ? v[off[j] + e] : 0.0) + acc[j];
  }
}

// Stages the chunk [e0, e0 + ne) of r basis vectors in LDS in the order the
// lift's matrix-core steps read them: for DoF step t, basis step st and lane
// (kq, row) (basis row 4 st + kq, DoF e0 + 16 t + row) at
// ((t ns + st) 4 + kq) 16 + row with ns = ceil(r / 4), so that one read by
// the 64 lanes of a wave covers 64 consecutive doubles; zeros past ne and
// for rows at or past r.
template <int CH>
__device__ __forceinline__ void stage_basis_mfma_lift(const double* __restrict__ W, int r, int nd, int e0, int ne,
                                                      double* Wl) {
  const int ns = (r + 3) >> 2;
  const int total = (CH / 16) * ns * 64;
  for (int base = 0; base < total; base += 8 * (int)blockDim.x) {
    double w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int sl = base + u * (int)blockDim.x + (int)threadIdx.x;
      const int row = sl & 15, kq = (sl >> 4) & 3, tst = sl >> 6;
      const int st = tst % ns, t = tst / ns;
      const int k = 4 * st + kq, el = 16 * t + row;
      const bool in = sl < total && k < r && el < ne;
      const double x = W[(int64_t)(in ? k : 0) * nd + e0 + (in ? el : 0)];
      w[u] = in ? x : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int sl = base + u * (int)blockDim.x + (int)threadIdx.x;
      if (sl < total) Wl[sl] = w[u];
    }
  }
}

// The lift with each basis chunk shared by the four waves of a work group:
// 64 instances (16 per wave, as k_rom_lift_mfma) and one chunk of LFL_DOF
// DoFs per work group, the chunk of every basis vector staged in LDS once.
// v is read at clamped addresses (no branch around a load); only the stores
// of z are conditional.
__global__ void __launch_bounds__(256) k_rom_lift_lds(const InstDev* __restrict__ insts,
                                                      const double* __restrict__ W, int r, int nd, int n,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ c, double* __restrict__ z,
                                                      const int32_t* __restrict__ active) {
  extern __shared__ double Wl[];  // the basis chunk in the order of the steps (stage_basis_mfma_lift)
  const int e0 = blockIdx.x * LFL_DOF;
  const int ne = min(LFL_DOF, nd - e0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4;
  const int g0 = blockIdx.y * 64 + wave * 16;
  const int ba = g0 + row;
  double ca[ROM_RMAX / 4];
#pragma unroll
  for (int st = 0; st < ROM_RMAX / 4; ++st) {
    const int k = 4 * st + kq;
    ca[st] = (ba < n && k < r) ? c[(int64_t)ba * ROM_RMAX + k] : 0.0;
  }
  int64_t off[4];
  bool on[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int bo = g0 + kq + 4 * j;
    on[j] = bo < n && (!active || active[bo]);
    off[j] = on[j] ? insts[bo].dof_off : 0;
  }
  const int ns = (r + 3) >> 2;
  // every value of v the wave needs first (clamped addresses), so that the
  // loads are all in flight together
  double vv[LFL_DOF / 16][4];
  const double* vs = v ? v : z;  // without v: any valid address, the values are dropped
#pragma unroll
  for (int t = 0; t < LFL_DOF / 16; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = e0 + t * 16 + row;
      const int64_t o = (on[j] && e < nd) ? off[j] + e : 0;
      vv[t][j] = vs[o];
    }
  if (!v)
#pragma unroll
    for (int t = 0; t < LFL_DOF / 16; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) vv[t][j] = 0.0;
  // the basis chunk while those loads are in flight
  stage_basis_mfma_lift<LFL_DOF>(W, r, nd, e0, ne, Wl);
  __syncthreads();
#pragma unroll
  for (int t = 0; t < LFL_DOF / 16; ++t) {  // past the chunk's end no store
    const int el = t * 16 + row;
    const int e = e0 + el;
    rom_d4 acc = rom_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < ROM_RMAX / 4; ++st)
      if (st < ns)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[st], Wl[((t * ns + st) * 4 + kq) * 16 + row], acc, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (on[j] && e < nd) z[off[j] + e] = vv[t][j] + acc[j];
  }
}

// Greedy residual indicator: for every listed parameter (training instance)
// and ordinate j, partial sums of
//   || sum_k c_k (D_j U_k,j + st U_k,j) - ss (W_w c) - eta0 ||^2
// over chunks of one ordinate's dofs.
constexpr int GR_MB = 8;
__global__ void k_greedy_res(int r, int rcap, int n_ord, int64_t nd, int nl,
                             const int32_t* __restrict__ region, const double* __restrict__ U,
                             const double* __restrict__ DU, const double* __restrict__ Ww,
                             int nmu, const int32_t* __restrict__ mu_idx,
                             const double* __restrict__ c, const double* __restrict__ sigma_t,
                             const double* __restrict__ sigma_s, int max_regions,
                             const double* __restrict__ eta0, double* __restrict__ part, int nch) {
  __shared__ double sh[4];
  const int j = blockIdx.y, ch = blockIdx.x;
  const int64_t e = (int64_t)ch * 256 + threadIdx.x;
  const bool on = e < nd;
  const int rg = on ? region[(int)(e / nl)] : 0;
  const int64_t psi_e = (int64_t)j * nd + e;
  for (int mb = 0; mb < nmu; mb += GR_MB) {
    double res[GR_MB];
    double st[GR_MB], ss[GR_MB];
#pragma unroll
    for (int q = 0; q < GR_MB; ++q) {
      res[q] = 0.0;
      const int mi = mb + q < nmu ? mu_idx[mb + q] : 0;
      st[q] = sigma_t[(int64_t)mi * max_regions + rg];
      ss[q] = sigma_s[(int64_t)mi * max_regions + rg];
    }
    if (on) {
      for (int k = 0; k < r; ++k) {
        const double uu = U[(int64_t)k * n_ord * nd + psi_e];
        const double du = DU[(int64_t)k * n_ord * nd + psi_e];
        const double wv = Ww[(int64_t)k * nd + e];
#pragma unroll
        for (int q = 0; q < GR_MB; ++q) {
          const double ck = mb + q < nmu ? c[(int64_t)(mb + q) * rcap + k] : 0.0;
          res[q] += ck * (du + st[q] * uu - ss[q] * wv);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < GR_MB; ++q) {
      double sq = 0.0;
      if (on && mb + q < nmu) {
        const double d = res[q] - eta0[(int64_t)mu_idx[mb + q] * nd + e];
        sq = d * d;
      }
      const double t = bsum256(sq, sh);
      if (threadIdx.x == 0 && mb + q < nmu) part[((int64_t)(mb + q) * n_ord + j) * nch + ch] = t;
    }
  }
}

__global__ void k_greedy_max(int nmu, int n_ord, int nch, const double* __restrict__ part,
                             double* __restrict__ out) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nmu) return;
  double best = 0.0;
  for (int j = 0; j < n_ord; ++j) {
    double t = 0.0;
    for (int c = 0; c < nch; ++c) t += part[((int64_t)m * n_ord + j) * nch + c];
    best = fmax(best, sqrt(t));
  }
  out[m] = best;
}

// y_v = B_f x_v per cell for nvec vectors of nd = 4 ncell dofs (B_f the
// mass block of shape function f alone)
__global__ void k_field_apply_vecs(const double* __restrict__ fblk, int f, int64_t ncell, int nvec,
                                   const double* __restrict__ x, double* __restrict__ y) {
  const int v = blockIdx.y;
  const int64_t nd = 4 * ncell;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * blockDim.x) {
    const double* B = fblk + ((int64_t)f * ncell + c) * 16;
    const double* xc = x + (int64_t)v * nd + 4 * c;
    double* yc = y + (int64_t)v * nd + 4 * c;
    const double x0 = xc[0], x1 = xc[1], x2 = xc[2], x3 = xc[3];
    for (int a = 0; a < 4; ++a) yc[a] = B[4 * a] * x0 + B[4 * a + 1] * x1 + B[4 * a + 2] * x2 + B[4 * a + 3] * x3;
  }
}

// out[i * nf + f] = col[i], i < n
__global__ void k_put_col(int n, int nf, int f, const double* __restrict__ col, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i * nf + f] = col[i];
}

// The greedy residual indicator with cross sections varying inside the
// cells: per listed parameter, ordinate j and cell, the 4 moments of
//   sum_k c_k (D_j U_k,j) + Sigma_t(mu) (U c)_j - Sigma_s(mu) (W_w c) - eta0,
// the full blocks applied to the accumulated vectors; partial sums of the
// squares per chunk of 256 cells.
constexpr int GRF_MB = 4;
__global__ void k_greedy_res_field(int r, int rcap, int n_ord, int64_t ncell, const double* __restrict__ U,
                                   const double* __restrict__ DU, const double* __restrict__ Ww, int nmu,
                                   const int32_t* __restrict__ mu_idx, const double* __restrict__ c,
                                   const double* __restrict__ fblk, int nf, const double* __restrict__ sigma_t,
                                   const double* __restrict__ sigma_s, int max_regions,
                                   const double* __restrict__ eta0, double* __restrict__ part, int nch) {
  __shared__ double sh[4];
  const int j = blockIdx.y, ch = blockIdx.x;
  const int64_t cell = (int64_t)ch * 256 + threadIdx.x;
  const bool on = cell < ncell;
  const int64_t nd = 4 * ncell;
  const int64_t pe = (int64_t)j * nd + 4 * cell;
  for (int mb = 0; mb < nmu; mb += GRF_MB) {
    double adu[GRF_MB][4], au[GRF_MB][4], aw[GRF_MB][4];
#pragma unroll
    for (int q = 0; q < GRF_MB; ++q)
#pragma unroll
      for (int a = 0; a < 4; ++a) adu[q][a] = au[q][a] = aw[q][a] = 0.0;
    if (on) {
      for (int k = 0; k < r; ++k) {
        const double* uk = U + (int64_t)k * n_ord * nd + pe;
        const double* dk = DU + (int64_t)k * n_ord * nd + pe;
        const double* wk = Ww + (int64_t)k * nd + 4 * cell;
#pragma unroll
        for (int q = 0; q < GRF_MB; ++q) {
          const double ck = mb + q < nmu ? c[(int64_t)(mb + q) * rcap + k] : 0.0;
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            adu[q][a] = fma(ck, dk[a], adu[q][a]);
            au[q][a] = fma(ck, uk[a], au[q][a]);
            aw[q][a] = fma(ck, wk[a], aw[q][a]);
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < GRF_MB; ++q) {
      double sq = 0.0;
      if (on && mb + q < nmu) {
        const int mi = mu_idx[mb + q];
        double Bt[16], Bs[16];
        field_block(fblk, nf, ncell, cell, sigma_t + (int64_t)mi * max_regions, Bt);
        field_block(fblk, nf, ncell, cell, sigma_s + (int64_t)mi * max_regions, Bs);
        const double* e0 = eta0 + (int64_t)mi * nd + 4 * cell;
        for (int a = 0; a < 4; ++a) {
          double v = adu[q][a] - e0[a];
          for (int bb = 0; bb < 4; ++bb) v += Bt[4 * a + bb] * au[q][bb] - Bs[4 * a + bb] * aw[q][bb];
          sq += v * v;
        }
      }
      const double t = bsum256(sq, sh);
      if (threadIdx.x == 0 && mb + q < nmu) part[((int64_t)(mb + q) * n_ord + j) * nch + ch] = t;
    }
  }
}

__global__ void k_scale_sigma(const InstDev* __restrict__ insts, const int32_t* __restrict__ region,
                              const double* __restrict__ sigma, int max_regions,
                              const double* __restrict__ x, double* __restrict__ y) {
  const int b = blockIdx.y;
  const InstDev I = insts[b];
  const int64_t nd = (int64_t)I.nx * I.ny * I.nloc;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nd;
       e += (int64_t)gridDim.x * blockDim.x)
    y[I.dof_off + e] = sigma[(int64_t)b * max_regions + region[I.region_off + (int)(e / I.nloc)]] *
                       x[I.dof_off + e];
}

__global__ void k_axpy_dev(int64_t n, const double* __restrict__ alpha, double sign,
                           const double* __restrict__ x, double* __restrict__ y) {
  const double a = sign * alpha[0];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] += a * x[e];
}

// ------------------------------------------------------------------ host
struct RomScratch {
  const rte_batch* b = nullptr;
  int n = 0;
  double *g = nullptr, *c = nullptr, *part = nullptr;
  double* sv = nullptr;  // Sigma_s v of a field-mode batch [total_dof]
  int32_t* sing = nullptr;
  int64_t part_elems = 0;
  // factors of A_r(mu) kept by the per-solve singularity check ([n][ROM_RMAX]^2,
  // [n][ROM_RMAX]), allocated on first use
  double* lu = nullptr;
  int32_t* piv = nullptr;
  // per-instance ROM table of the last ROM used on this batch
  RomDev* d_tab = nullptr;
  std::vector<RomDev> h_tab;
  const rte_rom* tab_rom = nullptr;
  int64_t tab_key = -1;
};
static std::vector<RomScratch> g_rs;

static RomScratch* scratch_for(const rte_batch* b, int64_t part_elems) {
  for (auto& s : g_rs)
    if (s.b == b) {
      if (s.part_elems < part_elems) {
        (void)hipFree(s.part);
        if (hipMalloc(&s.part, sizeof(double) * part_elems) != hipSuccess) return nullptr;
        s.part_elems = part_elems;
      }
      return &s;
    }
  RomScratch s;
  s.b = b;
  s.n = b->n_inst;
  if (hipMalloc(&s.g, sizeof(double) * s.n * ROM_RMAX) != hipSuccess ||
      hipMalloc(&s.c, sizeof(double) * s.n * ROM_RMAX) != hipSuccess ||
      hipMalloc(&s.sing, sizeof(int32_t) * s.n) != hipSuccess ||
      hipMalloc(&s.part, sizeof(double) * part_elems) != hipSuccess)
    return nullptr;
  s.part_elems = part_elems;
  g_rs.push_back(s);
  return &g_rs.back();
}

static RomDev rom_dev(const rte_rom* m) {
  RomDev d;
  d.W1 = m->W1;
  d.Ww = m->Ww;
  d.AD = m->AD;
  d.G = m->G;
  d.S = m->S;
  d.r = m->r;
  d.ld = m->rcap;
  d.nreg = m->n_regions;
  d.pad = 0;
  d.nd = m->ndof;
  return d;
}

// The per-instance table of the ROM (or ROM set) serving batch b, rebuilt
// when the ROM or the rank of any member changed since the last call.
static const RomDev* rom_table(const rte_rom* rom, RomScratch* sc, const rte_batch* b, hipStream_t s) {
  int64_t key = 0;
  if (rom->is_set())
    for (const rte_rom* m : rom->members) key = key * 131 + m->r + 1;
  else
    key = rom->r + 1;
  if (sc->tab_rom == rom && sc->tab_key == key && sc->d_tab) return sc->d_tab;
  if (!sc->d_tab && hipMalloc(&sc->d_tab, sizeof(RomDev) * b->n_inst) != hipSuccess) return nullptr;
  sc->h_tab.resize(b->n_inst);
  for (int k = 0; k < b->n_inst; ++k)
    sc->h_tab[k] = rom_dev(rom->is_set() ? rom->members[rom->member_of[k]] : rom);
  if (hipMemcpyAsync(sc->d_tab, sc->h_tab.data(), sizeof(RomDev) * b->n_inst, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return nullptr;
  sc->tab_rom = rom;
  sc->tab_key = key;
  return sc->d_tab;
}

static int rom_max_rank(const rte_rom* rom) {
  if (!rom->is_set()) return rom->r;
  int r = 0;
  for (const rte_rom* m : rom->members) r = std::max(r, m->r);
  return r;
}

static int64_t rom_max_ndof(const rte_rom* rom) {
  if (!rom->is_set()) return rom->ndof;
  int64_t nd = 0;
  for (const rte_rom* m : rom->members) nd = std::max(nd, m->ndof);
  return nd;
}

void rom_scratch_forget(const rte_batch* b) {
  for (size_t i = 0; i < g_rs.size();) {
    if (g_rs[i].b == b) {
      (void)hipFree(g_rs[i].g);
      (void)hipFree(g_rs[i].c);
      (void)hipFree(g_rs[i].part);
      (void)hipFree(g_rs[i].sing);
      (void)hipFree(g_rs[i].lu);
      (void)hipFree(g_rs[i].piv);
      (void)hipFree(g_rs[i].sv);
      (void)hipFree(g_rs[i].d_tab);
      g_rs.erase(g_rs.begin() + i);
    } else {
      ++i;
    }
  }
}

int rom_alloc(rte_rom* rom, const rte_batch* b, int rcap) {
  const InstDev& I = b->inst[0];
  rom->rcap = rcap;
  rom->r = 0;
  rom->dim = I.dim;
  rom->nx = I.nx;
  rom->ny = I.ny;
  rom->nloc = I.nloc;
  rom->n_ord = I.n_ord;
  rom->n_regions = I.n_regions;
  rom->ndof = (int64_t)I.nx * I.ny * I.nloc;
  rom->npsi = rom->ndof * I.n_ord;
  // ordinates and weights back in original order
  rom->ox.assign(I.n_ord, 0.0);
  rom->w.assign(I.n_ord, 0.0);
  std::vector<double> oy(I.n_ord, 0.0);
  for (int s = 0; s < I.n_ord; ++s) {
    const int j = b->perm[I.ord_off + s];
    rom->ox[j] = b->ox[I.ord_off + s];
    oy[j] = b->oy[I.ord_off + s];
    rom->w[j] = b->w[I.ord_off + s];
  }
  rom->region.assign(I.nx * I.ny, 0);
  rom->fields = b->n_fields > 0;
  if (rom->fields) {
    rom->n_regions = b->n_fields;  // the affine pieces belong to the shape functions; no region map
  } else {
    RTE_HIP(hipMemcpy(rom->region.data(), b->d_region + I.region_off, sizeof(int32_t) * I.nx * I.ny,
                      hipMemcpyDeviceToHost));
  }
  const int R = rom->n_regions;
  if (hipMalloc(&rom->U, sizeof(double) * rcap * rom->npsi) != hipSuccess ||
      hipMalloc(&rom->DU, sizeof(double) * rcap * rom->npsi) != hipSuccess ||
      hipMalloc(&rom->W1, sizeof(double) * rcap * rom->ndof) != hipSuccess ||
      hipMalloc(&rom->Ww, sizeof(double) * rcap * rom->ndof) != hipSuccess ||
      hipMalloc(&rom->AD, sizeof(double) * rcap * rcap) != hipSuccess ||
      hipMalloc(&rom->G, sizeof(double) * R * rcap * rcap) != hipSuccess ||
      hipMalloc(&rom->S, sizeof(double) * R * rcap * rcap) != hipSuccess ||
      hipMalloc(&rom->d_region, sizeof(int32_t) * I.nx * I.ny) != hipSuccess ||
      hipMalloc(&rom->d_w, sizeof(double) * 3 * I.n_ord) != hipSuccess)
    return RTE_ENOMEM;
  RTE_HIP(hipMemset(rom->AD, 0, sizeof(double) * rcap * rcap));
  RTE_HIP(hipMemset(rom->G, 0, sizeof(double) * R * rcap * rcap));
  RTE_HIP(hipMemset(rom->S, 0, sizeof(double) * R * rcap * rcap));
  RTE_HIP(hipMemcpy(rom->d_region, rom->region.data(), sizeof(int32_t) * I.nx * I.ny,
                    hipMemcpyHostToDevice));
  // d_w holds [w | ox | oy] in original ordinate order
  RTE_HIP(hipMemcpy(rom->d_w, rom->w.data(), sizeof(double) * I.n_ord, hipMemcpyHostToDevice));
  RTE_HIP(hipMemcpy(rom->d_w + I.n_ord, rom->ox.data(), sizeof(double) * I.n_ord, hipMemcpyHostToDevice));
  RTE_HIP(hipMemcpy(rom->d_w + 2 * I.n_ord, oy.data(), sizeof(double) * I.n_ord, hipMemcpyHostToDevice));
  rom->oyv = oy;
  rom->hx = I.hx;
  rom->hy = I.hy;
  return RTE_OK;
}

void rom_free(rte_rom* rom) {
  for (void* p : {(void*)rom->U, (void*)rom->DU, (void*)rom->W1, (void*)rom->Ww, (void*)rom->AD,
                  (void*)rom->G, (void*)rom->S, (void*)rom->d_region, (void*)rom->d_w})
    (void)hipFree(p);
  rom->U = rom->DU = rom->W1 = rom->Ww = rom->AD = rom->G = rom->S = rom->d_w = nullptr;
  rom->d_region = nullptr;
}

static int mdot_n(const rte_rom* rom, int nreg, int64_t len, int64_t nd, const double* x, const double* Y,
                  int64_t ystride, int ny_, double* part, double* out, hipStream_t s) {
  const int nch = (int)((len + MD_CHUNK - 1) / MD_CHUNK);
  hipLaunchKernelGGL(k_mdot, dim3(nch, ny_), dim3(256), 0, s, len, nd, rom->nloc, rom->d_region, nreg, x, Y,
                     ystride, part, nch);
  hipLaunchKernelGGL(k_mdot_sum, dim3((ny_ * nreg + 63) / 64), dim3(64), 0, s, ny_, nch, nreg, part, out);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

static int mdot(const rte_rom* rom, int64_t len, int64_t nd, const double* x, const double* Y,
                int64_t ystride, int ny_, double* part, double* out, hipStream_t s) {
  return mdot_n(rom, rom->n_regions, len, nd, x, Y, ystride, ny_, part, out, s);
}

// The new row/column r of A_D, G_f, S_f of a field-mode ROM: plain inner
// products (the region map is all zeros: one region) of the shape-weighted
// vectors M_f u_r, M_f W_w,r and M_f W_1,r with the basis.
static int field_columns(rte_rom* rom, const rte_batch* b, const double* u, const double* du, int r, double* part,
                         double* adc, double* adr, double* gg, double* sc, double* sr, hipStream_t s) {
  const int nf = rom->n_regions, ny_ = r + 1;
  const int64_t nd = rom->ndof, np = rom->npsi, ncell = nd / 4;
  double *mu = nullptr, *tmp = nullptr;
  if (hipMalloc(&mu, sizeof(double) * np) != hipSuccess || hipMalloc(&tmp, sizeof(double) * ny_) != hipSuccess) {
    (void)hipFree(mu);
    return RTE_ENOMEM;
  }
  int st = RTE_OK;
  const dim3 gpsi((unsigned)std::min<int64_t>((ncell + 255) / 256, 1024), rom->n_ord), gdof(gpsi.x, 1);
  auto put = [&](double* out, int f) {
    hipLaunchKernelGGL(k_put_col, dim3((ny_ + 63) / 64), dim3(64), 0, s, ny_, nf, f, tmp, out);
    return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EHIP;
  };
  if (hipMemsetAsync(adc, 0, sizeof(double) * ny_ * nf, s) != hipSuccess ||
      hipMemsetAsync(adr, 0, sizeof(double) * ny_ * nf, s) != hipSuccess)
    st = RTE_EHIP;
  if (st == RTE_OK) st = mdot_n(rom, 1, np, nd, du, rom->U, np, ny_, part, tmp, s);   // <U_i, DU_r>
  if (st == RTE_OK) st = put(adc, 0);
  if (st == RTE_OK) st = mdot_n(rom, 1, np, nd, u, rom->DU, np, ny_, part, tmp, s);   // <U_r, DU_i>
  if (st == RTE_OK) st = put(adr, 0);
  for (int f = 0; f < nf && st == RTE_OK; ++f) {
    hipLaunchKernelGGL(k_field_apply_vecs, gpsi, dim3(256), 0, s, b->d_fblk, f, ncell, rom->n_ord, u, mu);
    st = mdot_n(rom, 1, np, nd, mu, rom->U, np, ny_, part, tmp, s);                    // <U_i, M_f U_r>
    if (st == RTE_OK) st = put(gg, f);
    if (st == RTE_OK) {
      hipLaunchKernelGGL(k_field_apply_vecs, gdof, dim3(256), 0, s, b->d_fblk, f, ncell, 1,
                         rom->Ww + (int64_t)r * nd, mu);
      st = mdot_n(rom, 1, nd, nd, mu, rom->W1, nd, ny_, part, tmp, s);                 // <W1_i, M_f Ww_r>
    }
    if (st == RTE_OK) st = put(sc, f);
    if (st == RTE_OK) {
      hipLaunchKernelGGL(k_field_apply_vecs, gdof, dim3(256), 0, s, b->d_fblk, f, ncell, 1,
                         rom->W1 + (int64_t)r * nd, mu);
      st = mdot_n(rom, 1, nd, nd, mu, rom->Ww, nd, ny_, part, tmp, s);                 // <M_f W1_r, Ww_i>
    }
    if (st == RTE_OK) st = put(sr, f);
  }
  if (hipStreamSynchronize(s) != hipSuccess && st == RTE_OK) st = RTE_EHIP;
  (void)hipFree(mu);
  (void)hipFree(tmp);
  return st;
}

int rom_add_column(rte_rom* rom, const rte_batch* b, hipStream_t s) {
  (void)b;
  const int r = rom->r;
  if (r >= rom->rcap) return RTE_EINVAL;
  const int64_t nd = rom->ndof, np = rom->npsi;
  double* u = rom->U + (int64_t)r * np;
  double* du = rom->DU + (int64_t)r * np;
  const int ncell = rom->nx * rom->ny;
  hipLaunchKernelGGL(k_advect, dim3((ncell + 255) / 256, rom->n_ord), dim3(256), 0, s, rom->dim,
                     rom->nx, rom->ny, rom->hx, rom->hy, rom->n_ord, rom->d_w + rom->n_ord,
                     rom->d_w + 2 * rom->n_ord, u, du);
  hipLaunchKernelGGL(k_angle_sums, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, s, rom->n_ord, nd,
                     rom->d_w, u, rom->W1 + (int64_t)r * nd, rom->Ww + (int64_t)r * nd);
  RTE_HIP(hipGetLastError());
  const int R = rom->n_regions;
  const int ny_ = r + 1;
  const int64_t nchp = (np + MD_CHUNK - 1) / MD_CHUNK;
  double *part = nullptr, *res = nullptr;
  if (hipMalloc(&part, sizeof(double) * nchp * ny_ * R) != hipSuccess ||
      hipMalloc(&res, sizeof(double) * 5 * ny_ * R) != hipSuccess)
    return RTE_ENOMEM;
  double* adc = res;
  double* adr = res + ny_ * R;
  double* gg = res + 2 * ny_ * R;
  double* sc = res + 3 * ny_ * R;
  double* sr = res + 4 * ny_ * R;
  int st = RTE_OK;
  if (rom->fields) {
    if (!b || b->n_fields != R) st = RTE_EINVAL;
    if (st == RTE_OK) st = field_columns(rom, b, u, du, r, part, adc, adr, gg, sc, sr, s);
    if (st == RTE_OK) {
      hipLaunchKernelGGL(k_place, dim3((ny_ + 63) / 64), dim3(64), 0, s, r, rom->rcap, R, adc, adr, gg, sc, sr,
                         rom->AD, rom->G, rom->S);
      if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) st = RTE_EHIP;
    }
    (void)hipFree(part);
    (void)hipFree(res);
    if (st == RTE_OK) rom->r = r + 1;
    return st;
  }
  if (st == RTE_OK) st = mdot(rom, np, nd, du, rom->U, np, ny_, part, adc, s);   // <U_i, DU_r>
  if (st == RTE_OK) st = mdot(rom, np, nd, u, rom->DU, np, ny_, part, adr, s);   // <U_r, DU_i>
  if (st == RTE_OK) st = mdot(rom, np, nd, u, rom->U, np, ny_, part, gg, s);     // <U_i, U_r>_R
  if (st == RTE_OK) st = mdot(rom, nd, nd, rom->Ww + (int64_t)r * nd, rom->W1, nd, ny_, part, sc, s);
  if (st == RTE_OK) st = mdot(rom, nd, nd, rom->W1 + (int64_t)r * nd, rom->Ww, nd, ny_, part, sr, s);
  if (st == RTE_OK) {
    hipLaunchKernelGGL(k_place, dim3((ny_ + 63) / 64), dim3(64), 0, s, r, rom->rcap, R, adc, adr, gg,
                       sc, sr, rom->AD, rom->G, rom->S);
    if (hipGetLastError() != hipSuccess) st = RTE_EHIP;
  }
  if (hipStreamSynchronize(s) != hipSuccess) st = RTE_EHIP;
  (void)hipFree(part);
  (void)hipFree(res);
  if (st == RTE_OK) rom->r = r + 1;
  return st;
}

static bool rom_matches_inst(const rte_rom* rom, const rte_batch* b, int k) {
  const InstDev& I = b->inst[k];
  if (I.dim != rom->dim || I.nx != rom->nx || I.ny != rom->ny || I.n_ord != rom->n_ord ||
      I.n_regions > rom->n_regions)
    return false;
  for (int s = 0; s < I.n_ord; ++s) {
    const int j = b->perm[I.ord_off + s];
    if (b->ox[I.ord_off + s] != rom->ox[j] || b->w[I.ord_off + s] != rom->w[j]) return false;
  }
  return true;
}

bool rom_matches(const rte_rom* rom, const rte_batch* b) {
  if (rom->is_set() ? b->n_fields > 0 : rom->fields != (b->n_fields > 0)) return false;
  if (rom->fields && b->n_fields != rom->n_regions) return false;
  if (rom->is_set()) {
    if ((int)rom->member_of.size() != b->n_inst) return false;
    for (int k = 0; k < b->n_inst; ++k)
      if (!rom_matches_inst(rom->members[rom->member_of[k]], b, k)) return false;
    return true;
  }
  for (int k = 0; k < b->n_inst; ++k) {
    const InstDev& I = b->inst[k];
    if (I.dim != rom->dim || I.nx != rom->nx || I.ny != rom->ny || I.n_ord != rom->n_ord ||
        I.n_regions > rom->n_regions)
      return false;
    for (int s = 0; s < I.n_ord; ++s) {
      const int j = b->perm[I.ord_off + s];
      if (b->ox[I.ord_off + s] != rom->ox[j] || b->w[I.ord_off + s] != rom->w[j]) return false;
    }
  }
  return true;
}

// partial sums per instance of either projection kernel
static int64_t rom_part_elems(const rte_batch* b, int64_t nd) {
  return (int64_t)b->n_inst * ((nd + PJL_DOF - 1) / PJL_DOF) * ROM_RMAX;  // the shorter chunk
}

int rom_project(const rte_rom* rom, rte_batch* b, const double* sigma_s, const double* v, double* g,
                const int32_t* active, hipStream_t s, const double* W) {
  const int64_t nd = rom_max_ndof(rom);
  const int nch = (int)((nd + PJ_CHUNK - 1) / PJ_CHUNK);
  RomScratch* sc = scratch_for(b, rom_part_elems(b, nd));
  if (!sc) return RTE_ENOMEM;
  const RomDev* tab = rom_table(rom, sc, b, s);
  if (!tab) return RTE_EHIP;
  const int which = (W && !rom->is_set() && W == rom->Ww) ? 1 : 0;
  if (W && !which) return RTE_EINVAL;  // only W_1 or W_w of the ROM itself
  if (sigma_s && b->n_fields > 0) {  // Sigma_s v with the cells' full blocks, then the plain projection
    if (!sc->sv && hipMalloc(&sc->sv, sizeof(double) * b->total_dof) != hipSuccess) return RTE_ENOMEM;
    RTE_TRY(field_apply(b, sigma_s, v, sc->sv, false, active, s));
    v = sc->sv;
    sigma_s = nullptr;
  }
  // the LDS-staged kernel may take up to ROM_RMAX x PJL_DOF doubles
  static int lds_ok = -1;
  if (lds_ok < 0) {
    const int bytes = (int)(sizeof(double) * ROM_RMAX * PJL_DOF);
    lds_ok = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rom_project_lds<4>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess &&
                     hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rom_project_lds<2>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess
                 ? 1
                 : 0;
    if (!lds_ok) (void)hipGetLastError();
  }
  if (lds_ok && !rom->is_set() && nd < (1 << 30) && (nd & 1) == 0) {
    // the basis chunk staged in LDS, shared by 64 instances
    const int nchm = (int)((nd + PJL_DOF - 1) / PJL_DOF);
    const dim3 grid(nchm, (b->n_inst + 63) / 64);
    const size_t lds = sizeof(double) * 16 * ((rom->r + 15) / 16) * PJL_DOF;
    const double* Wp = which ? rom->Ww : rom->W1;
    if (b->inst[0].nloc == 4)
      hipLaunchKernelGGL(k_rom_project_lds<4>, grid, dim3(256), lds, s, b->d_inst, b->d_region, sigma_s,
                         b->max_regions, Wp, rom->r, (int)nd, b->n_inst, v, sc->part, nchm, active);
    else
      hipLaunchKernelGGL(k_rom_project_lds<2>, grid, dim3(256), lds, s, b->d_inst, b->d_region, sigma_s,
                         b->max_regions, Wp, rom->r, (int)nd, b->n_inst, v, sc->part, nchm, active);
    hipLaunchKernelGGL(k_rom_gsum4, dim3(b->n_inst), dim3(256), 0, s, b->n_inst, nchm, tab, sc->part, g,
                       active);
    RTE_HIP(hipGetLastError());
    return RTE_OK;
  }
  if (!rom->is_set() && nd < (1 << 30)) {
    const int nchm = (int)((nd + PM_DOF - 1) / PM_DOF);
    const dim3 grid((nchm + 3) / 4, (b->n_inst + 15) / 16);
    const double* Wp = which ? rom->Ww : rom->W1;
    if (b->inst[0].nloc == 4)
      hipLaunchKernelGGL(k_rom_project_mfma<4>, grid, dim3(256), 0, s, b->d_inst, b->d_region, sigma_s,
                         b->max_regions, Wp, rom->r, (int)nd, b->n_inst, v, sc->part, nchm, active);
    else
      hipLaunchKernelGGL(k_rom_project_mfma<2>, grid, dim3(256), 0, s, b->d_inst, b->d_region, sigma_s,
                         b->max_regions, Wp, rom->r, (int)nd, b->n_inst, v, sc->part, nchm, active);
    hipLaunchKernelGGL(k_rom_gsum, dim3((b->n_inst * ROM_RMAX + 63) / 64), dim3(64), 0, s, b->n_inst, nchm,
                       tab, sc->part, g, active);
    RTE_HIP(hipGetLastError());
    return RTE_OK;
  }
  hipLaunchKernelGGL(k_rom_project, dim3(nch, b->n_inst), dim3(256), 0, s, b->d_inst, b->d_region,
                     sigma_s, b->max_regions, tab, which, v, sc->part, nch, active);
  hipLaunchKernelGGL(k_rom_gsum, dim3((b->n_inst * ROM_RMAX + 63) / 64), dim3(64), 0, s, b->n_inst, nch, tab,
                     sc->part, g, active);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int rom_lift(const rte_rom* rom, rte_batch* b, const double* v, const double* c, double* z,
             const int32_t* active, hipStream_t s) {
  const int64_t nd = rom_max_ndof(rom);
  RomScratch* sc = scratch_for(b, 1);
  if (!sc) return RTE_ENOMEM;
  const RomDev* tab = rom_table(rom, sc, b, s);
  if (!tab) return RTE_EHIP;
  static int lds_ok = -1;  // up to ROM_RMAX x LFL_DOF doubles of LDS
  if (lds_ok < 0) {
    lds_ok = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rom_lift_lds),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(sizeof(double) * ROM_RMAX * LFL_DOF)) == hipSuccess
                 ? 1
                 : 0;
    if (!lds_ok) (void)hipGetLastError();
  }
  if (lds_ok && !rom->is_set() && nd < (1 << 30) && (nd & 1) == 0) {
    // the basis chunk staged in LDS, shared by 64 instances
    const int nw = (int)((nd + LFL_DOF - 1) / LFL_DOF);
    hipLaunchKernelGGL(k_rom_lift_lds, dim3(nw, (b->n_inst + 63) / 64), dim3(256),
                       sizeof(double) * 4 * ((rom->r + 3) / 4) * LFL_DOF,
                       s, b->d_inst, rom->Ww, rom->r, (int)nd, b->n_inst, v, c, z, active);
    RTE_HIP(hipGetLastError());
    return RTE_OK;
  }
  if (!rom->is_set() && nd < (1 << 30)) {
    const int nw = (int)((nd + PL_DOF - 1) / PL_DOF);
    hipLaunchKernelGGL(k_rom_lift_mfma, dim3((nw + 3) / 4, (b->n_inst + 15) / 16), dim3(256), 0, s, b->d_inst,
                       rom->Ww, rom->r, (int)nd, b->n_inst, v, c, z, active);
    RTE_HIP(hipGetLastError());
    return RTE_OK;
  }
  dim3 grid((unsigned)std::min<int64_t>((nd + 255) / 256, 256), b->n_inst);
  hipLaunchKernelGGL(k_rom_lift, grid, dim3(256), 0, s, b->d_inst, tab, v, c, z, active);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int romsad_apply_internal(const rte_rom* rom, rte_batch* b, const double* sigma_t,
                          const double* sigma_s, const double* v, double* z, const int32_t* active,
                          hipStream_t s, double* gout, double* cout, int32_t* singular, bool use_factors) {
  if (rom_max_rank(rom) == 0) {
    RTE_HIP(hipMemcpyAsync(z, v, sizeof(double) * b->total_dof, hipMemcpyDeviceToDevice, s));
    return RTE_OK;
  }
  const int64_t nd = rom_max_ndof(rom);
  RomScratch* sc = scratch_for(b, rom_part_elems(b, nd));
  if (!sc) return RTE_ENOMEM;
  const RomDev* tab = rom_table(rom, sc, b, s);
  if (!tab) return RTE_EHIP;
  double* g = gout ? gout : sc->g;
  double* c = cout ? cout : sc->c;
  int32_t* sing = singular ? singular : sc->sing;
  RTE_TRY(rom_project(rom, b, sigma_s, v, g, active, s));
  if (use_factors) {
    if (!sc->lu) return RTE_EINVAL;  // no singularity check kept factors
    hipLaunchKernelGGL(k_rom_lusolve, dim3(b->n_inst), dim3(64), 0, s, b->n_inst, tab, sc->lu, sc->piv, g, c,
                       ROM_RMAX, active);
  } else {
    RTE_HIP(hipMemsetAsync(sing, 0, sizeof(int32_t) * b->n_inst, s));
    hipLaunchKernelGGL(k_rom_solve, dim3(b->n_inst), dim3(256), 0, s, b->n_inst, tab, sigma_t, sigma_s,
                       b->max_regions, g, c, ROM_RMAX, sing, active);
  }
  RTE_HIP(hipGetLastError());
  return rom_lift(rom, b, v, c, z, active, s);
}

int rom_solve_coeffs(const rte_rom* rom, rte_batch* b, const double* sigma_t, const double* sigma_s,
                     const double* g, double* c, const int32_t* active, hipStream_t s) {
  if (rom_max_rank(rom) == 0) return RTE_OK;
  RomScratch* sc = scratch_for(b, rom_part_elems(b, rom_max_ndof(rom)));
  if (!sc) return RTE_ENOMEM;
  const RomDev* tab = rom_table(rom, sc, b, s);
  if (!tab) return RTE_EHIP;
  hipLaunchKernelGGL(k_rom_solve, dim3(b->n_inst), dim3(256), 0, s, b->n_inst, tab, sigma_t, sigma_s,
                     b->max_regions, g, c, ROM_RMAX, (int32_t*)nullptr, active);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

// sing[b] = 1 where A_r(mu_b) has a pivot below 1e-14 max |A_r| (the test of
// k_rom_solve), for every instance; the operator depends on mu only, so one
// factorisation (with a zero right-hand side) per solve decides it.
int rom_singular_check(const rte_rom* rom, rte_batch* b, const double* sigma_t, const double* sigma_s,
                       int32_t* sing, hipStream_t s) {
  RTE_HIP(hipMemsetAsync(sing, 0, sizeof(int32_t) * b->n_inst, s));
  if (rom_max_rank(rom) == 0) return RTE_OK;
  RomScratch* sc = scratch_for(b, rom_part_elems(b, rom_max_ndof(rom)));
  if (!sc) return RTE_ENOMEM;
  const RomDev* tab = rom_table(rom, sc, b, s);
  if (!tab) return RTE_EHIP;
  if (!sc->lu && (hipMalloc(&sc->lu, sizeof(double) * sc->n * ROM_RMAX * ROM_RMAX) != hipSuccess ||
                  hipMalloc(&sc->piv, sizeof(int32_t) * sc->n * ROM_RMAX) != hipSuccess)) {
    (void)hipFree(sc->lu);
    sc->lu = nullptr;
    return RTE_ENOMEM;
  }
  RTE_HIP(hipMemsetAsync(sc->g, 0, sizeof(double) * b->n_inst * ROM_RMAX, s));
  hipLaunchKernelGGL(k_rom_solve, dim3(b->n_inst), dim3(256), 0, s, b->n_inst, tab, sigma_t, sigma_s,
                     b->max_regions, sc->g, sc->c, ROM_RMAX, sing, nullptr, sc->lu, sc->piv);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

}  // namespace rte

// ------------------------------------------------------------------ C ABI
using namespace rte;

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" int rte_rom_from_basis(const rte_batch* cb, const double* U, int r, rte_rom** out,
                                  void* stream) {
  auto* b = const_cast<rte_batch*>(cb);
  if (!b || !U || r < 1 || r > ROM_RMAX || !out) return RTE_EINVAL;
  if (b->inst[0].n_regions > ROM_REGMAX) return RTE_EINVAL;
  hipStream_t s = as_stream(stream);
  auto* rom = new rte_rom();
  int st = rom_alloc(rom, b, r);
  if (st == RTE_OK)
    st = hipMemcpyAsync(rom->U, U, sizeof(double) * r * rom->npsi, hipMemcpyDeviceToDevice, s) ==
                 hipSuccess ? RTE_OK : RTE_EHIP;
  for (int k = 0; k < r && st == RTE_OK; ++k) st = rom_add_column(rom, b, s);
  if (st != RTE_OK) {
    rom_free(rom);
    delete rom;
    return st;
  }
  *out = rom;
  return RTE_OK;
}

extern "C" int romsad_apply(const rte_rom* rom, const rte_batch* cb, const double* sigma_t,
                            const double* sigma_s, const double* v, double* z, void* stream) {
  auto* b = const_cast<rte_batch*>(cb);
  if (!rom || !b || !sigma_t || !sigma_s || !v || !z) return RTE_EINVAL;
  if (!rom_matches(rom, b)) return RTE_EINVAL;
  hipStream_t s = as_stream(stream);
  int32_t* sing = nullptr;
  if (hipMalloc(&sing, sizeof(int32_t) * b->n_inst) != hipSuccess) return RTE_ENOMEM;
  int st = romsad_apply_internal(rom, b, sigma_t, sigma_s, v, z, nullptr, s, nullptr, nullptr, sing);
  std::vector<int32_t> h(b->n_inst, 0);
  if (st == RTE_OK &&
      hipMemcpyAsync(h.data(), sing, sizeof(int32_t) * b->n_inst, hipMemcpyDeviceToHost, s) != hipSuccess)
    st = RTE_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess && st == RTE_OK) st = RTE_EHIP;
  (void)hipFree(sing);
  if (st != RTE_OK) return st;
  for (int q = 0; q < b->n_inst; ++q)
    if (h[q]) return RTE_ESINGULAR;
  return RTE_OK;
}

extern "C" int rte_rom_rank(const rte_rom* rom) { return rom ? rom_max_rank(rom) : -1; }

extern "C" int rte_rom_set_create(const rte_batch* b, const rte_rom* const* roms, int n_roms,
                                  const int32_t* rom_of_instance, rte_rom** out) {
  if (!b || !roms || n_roms < 1 || !rom_of_instance || !out) return RTE_EINVAL;
  auto* set = new rte_rom();
  for (int i = 0; i < n_roms; ++i) {
    if (!roms[i] || roms[i]->is_set()) {
      delete set;
      return RTE_EINVAL;
    }
    set->members.push_back(roms[i]);
  }
  set->member_of.assign(rom_of_instance, rom_of_instance + b->n_inst);
  for (int k = 0; k < b->n_inst; ++k)
    if (set->member_of[k] < 0 || set->member_of[k] >= n_roms) {
      delete set;
      return RTE_EINVAL;
    }
  if (!rom_matches(set, b)) {
    delete set;
    return RTE_EINVAL;
  }
  set->r = rom_max_rank(set);
  *out = set;
  return RTE_OK;
}

static int copy_mat(double* dst, const double* src, int r, int ld) {
  std::vector<double> tmp((size_t)ld * ld);
  RTE_HIP(hipMemcpy(tmp.data(), src, sizeof(double) * ld * ld, hipMemcpyDeviceToHost));
  for (int i = 0; i < r; ++i)
    for (int k = 0; k < r; ++k) dst[i * r + k] = tmp[(size_t)i * ld + k];
  return RTE_OK;
}

extern "C" int rte_rom_export(const rte_rom* rom, double* U, double* W1, double* Ww, double* AD,
                              double* G, double* S) {
  if (!rom || rom->is_set()) return RTE_EINVAL;
  RTE_HIP(hipDeviceSynchronize());
  const int r = rom->r;
  if (U) RTE_HIP(hipMemcpy(U, rom->U, sizeof(double) * r * rom->npsi, hipMemcpyDeviceToHost));
  if (W1) RTE_HIP(hipMemcpy(W1, rom->W1, sizeof(double) * r * rom->ndof, hipMemcpyDeviceToHost));
  if (Ww) RTE_HIP(hipMemcpy(Ww, rom->Ww, sizeof(double) * r * rom->ndof, hipMemcpyDeviceToHost));
  if (AD) RTE_TRY(copy_mat(AD, rom->AD, r, rom->rcap));
  for (int R = 0; R < rom->n_regions; ++R) {
    const size_t o = (size_t)R * rom->rcap * rom->rcap;
    if (G) RTE_TRY(copy_mat(G + (size_t)R * r * r, rom->G + o, r, rom->rcap));
    if (S) RTE_TRY(copy_mat(S + (size_t)R * r * r, rom->S + o, r, rom->rcap));
  }
  return RTE_OK;
}

extern "C" void rte_rom_destroy(rte_rom* rom) {
  if (!rom) return;
  for (auto& sc : g_rs) sc.tab_rom = nullptr;  // cached per-instance tables may point into it
  if (!rom->is_set()) rom_free(rom);
  delete rom;
}

// File format (little-endian): magic "RTEROM1\0", ints dim nx ny nloc n_ord
// n_regions r rcap, doubles hx hy, ordinates ox[n_ord] oy[n_ord] w[n_ord],
// region[nx*ny] (int32), then U, DU [r][npsi], W1, Ww [r][ndof], AD [rcap^2],
// G, S [n_regions][rcap^2].
extern "C" int rte_rom_save(const rte_rom* rom, const char* path) {
  if (!rom || !path || rom->is_set()) return RTE_EINVAL;
  FILE* f = std::fopen(path, "wb");
  if (!f) return RTE_EIO;
  RTE_HIP(hipDeviceSynchronize());
  // "RTEROM1": piecewise-constant cross sections; "RTEROMF": shape functions
  const char magic[8] = {'R', 'T', 'E', 'R', 'O', 'M', rom->fields ? 'F' : '1', 0};
  int32_t hdr[8] = {rom->dim, rom->nx, rom->ny, rom->nloc, rom->n_ord, rom->n_regions, rom->r, rom->rcap};
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(hdr), 1, f) == 1;
  double hh[2] = {rom->hx, rom->hy};
  ok = ok && std::fwrite(hh, sizeof(hh), 1, f) == 1;
  ok = ok && std::fwrite(rom->ox.data(), sizeof(double), rom->n_ord, f) == (size_t)rom->n_ord;
  ok = ok && std::fwrite(rom->oyv.data(), sizeof(double), rom->n_ord, f) == (size_t)rom->n_ord;
  ok = ok && std::fwrite(rom->w.data(), sizeof(double), rom->n_ord, f) == (size_t)rom->n_ord;
  ok = ok && std::fwrite(rom->region.data(), sizeof(int32_t), rom->region.size(), f) == rom->region.size();
  auto dump = [&](const double* d, size_t n) {
    std::vector<double> h(n);
    if (n && hipMemcpy(h.data(), d, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess) return false;
    return std::fwrite(h.data(), sizeof(double), n, f) == n;
  };
  const size_t r = rom->r, rc = rom->rcap, R = rom->n_regions;
  ok = ok && dump(rom->U, r * rom->npsi) && dump(rom->DU, r * rom->npsi) && dump(rom->W1, r * rom->ndof) &&
       dump(rom->Ww, r * rom->ndof) && dump(rom->AD, rc * rc) && dump(rom->G, R * rc * rc) &&
       dump(rom->S, R * rc * rc);
  ok = (std::fclose(f) == 0) && ok;
  return ok ? RTE_OK : RTE_EIO;
}

extern "C" int rte_rom_load(const char* path, rte_rom** out) {
  if (!path || !out) return RTE_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) return RTE_EIO;
  char magic[8];
  int32_t hdr[8];
  double hh[2];
  auto* rom = new rte_rom();
  auto fail = [&](int code) {
    std::fclose(f);
    rom_free(rom);
    delete rom;
    return code;
  };
  if (std::fread(magic, 1, 8, f) != 8 ||
      (std::memcmp(magic, "RTEROM1", 8) != 0 && std::memcmp(magic, "RTEROMF", 8) != 0) ||
      std::fread(hdr, sizeof(hdr), 1, f) != 1 || std::fread(hh, sizeof(hh), 1, f) != 1)
    return fail(RTE_EIO);
  rom->dim = hdr[0]; rom->nx = hdr[1]; rom->ny = hdr[2]; rom->nloc = hdr[3]; rom->n_ord = hdr[4];
  rom->n_regions = hdr[5]; rom->r = hdr[6]; rom->rcap = hdr[7];
  rom->fields = magic[6] == 'F';
  if (rom->dim < 1 || rom->dim > 2 || rom->nx < 1 || rom->ny < 1 || rom->n_ord < 1 || rom->rcap < rom->r ||
      rom->r < 0 || rom->rcap > ROM_RMAX || rom->n_regions < 1 || rom->n_regions > ROM_REGMAX ||
      (int64_t)rom->nx * rom->ny > (1 << 26))
    return fail(RTE_EIO);
  rom->hx = hh[0];
  rom->hy = hh[1];
  rom->ndof = (int64_t)rom->nx * rom->ny * rom->nloc;
  rom->npsi = rom->ndof * rom->n_ord;
  rom->ox.resize(rom->n_ord);
  rom->oyv.resize(rom->n_ord);
  rom->w.resize(rom->n_ord);
  rom->region.resize((size_t)rom->nx * rom->ny);
  if (std::fread(rom->ox.data(), sizeof(double), rom->n_ord, f) != (size_t)rom->n_ord ||
      std::fread(rom->oyv.data(), sizeof(double), rom->n_ord, f) != (size_t)rom->n_ord ||
      std::fread(rom->w.data(), sizeof(double), rom->n_ord, f) != (size_t)rom->n_ord ||
      std::fread(rom->region.data(), sizeof(int32_t), rom->region.size(), f) != rom->region.size())
    return fail(RTE_EIO);
  for (int32_t rg : rom->region)
    if (rg < 0 || rg >= rom->n_regions) return fail(RTE_EIO);
  const size_t rc = rom->rcap, R = rom->n_regions;
  if (hipMalloc(&rom->U, sizeof(double) * std::max<size_t>(rc, 1) * rom->npsi) != hipSuccess ||
      hipMalloc(&rom->DU, sizeof(double) * std::max<size_t>(rc, 1) * rom->npsi) != hipSuccess ||
      hipMalloc(&rom->W1, sizeof(double) * std::max<size_t>(rc, 1) * rom->ndof) != hipSuccess ||
      hipMalloc(&rom->Ww, sizeof(double) * std::max<size_t>(rc, 1) * rom->ndof) != hipSuccess ||
      hipMalloc(&rom->AD, sizeof(double) * std::max<size_t>(rc * rc, 1)) != hipSuccess ||
      hipMalloc(&rom->G, sizeof(double) * std::max<size_t>(R * rc * rc, 1)) != hipSuccess ||
      hipMalloc(&rom->S, sizeof(double) * std::max<size_t>(R * rc * rc, 1)) != hipSuccess ||
      hipMalloc(&rom->d_region, sizeof(int32_t) * rom->region.size()) != hipSuccess ||
      hipMalloc(&rom->d_w, sizeof(double) * 3 * rom->n_ord) != hipSuccess)
    return fail(RTE_ENOMEM);
  auto load = [&](double* d, size_t n) {
    std::vector<double> h(n);
    if (std::fread(h.data(), sizeof(double), n, f) != n) return false;
    return n == 0 || hipMemcpy(d, h.data(), sizeof(double) * n, hipMemcpyHostToDevice) == hipSuccess;
  };
  const size_t r = rom->r;
  if (!(load(rom->U, r * rom->npsi) && load(rom->DU, r * rom->npsi) && load(rom->W1, r * rom->ndof) &&
        load(rom->Ww, r * rom->ndof) && load(rom->AD, rc * rc) && load(rom->G, R * rc * rc) &&
        load(rom->S, R * rc * rc)))
    return fail(RTE_EIO);
  if (hipMemcpy(rom->d_region, rom->region.data(), sizeof(int32_t) * rom->region.size(),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(rom->d_w, rom->w.data(), sizeof(double) * rom->n_ord, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(rom->d_w + rom->n_ord, rom->ox.data(), sizeof(double) * rom->n_ord, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(rom->d_w + 2 * rom->n_ord, rom->oyv.data(), sizeof(double) * rom->n_ord,
                hipMemcpyHostToDevice) != hipSuccess)
    return fail(RTE_EHIP);
  std::fclose(f);
  *out = rom;
  return RTE_OK;
}

// ------------------------------------------------------------------ greedy
static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

extern "C" int romsad_build_greedy(const rte_batch* cb, const double* sigma_t, const double* sigma_s,
                                   const double* G, const double* inflow, int window, int mu1_index,
                                   double eps_rom, int n_giter, double eps_qr, double hf_rtol,
                                   double hf_dsa_tol, rte_rom** out, rte_greedy_report* rep,
                                   void* stream) {
  auto* b = const_cast<rte_batch*>(cb);
  if (!b || !sigma_t || !sigma_s || !G || !out || window < 1 || n_giter < 1 || mu1_index < 0 ||
      mu1_index >= b->n_inst || !(eps_qr >= 0.0) || !(hf_rtol > 0.0) || n_giter > 256 ||
      !(hf_dsa_tol >= 0.0) ||
      (int64_t)n_giter * window > ROM_RMAX || !b->uniform || b->inst[0].n_regions > ROM_REGMAX)
    return RTE_EINVAL;
  if (b->n_fields > 0 && !(hf_dsa_tol > 0.0)) return RTE_EINVAL;  // field mode: exact-solve DSA only
  hipStream_t s = as_stream(stream);
  RTE_TRY(validate_cross_sections(b, sigma_t, sigma_s, s));
  const int n = b->n_inst;
  double t_step[5] = {0, 0, 0, 0, 0};
  auto* rom = new rte_rom();
  auto cleanup = [&](int code) {
    rom_free(rom);
    delete rom;
    return code;
  };
  int st = rom_alloc(rom, b, n_giter * window);
  if (st != RTE_OK) return cleanup(st);
  const int64_t nd = rom->ndof, np = rom->npsi;
  const int R = rom->n_regions;
  // workspace
  double *btil = nullptr, *eta0 = nullptr, *phi = nullptr, *psi = nullptr, *xi = nullptr,
         *u = nullptr, *dsc = nullptr, *gq = nullptr, *cq = nullptr, *part = nullptr, *rmu = nullptr;
  int32_t *mask = nullptr, *midx = nullptr;
  const int ncell = rom->nx * rom->ny;
  const int nch_res = (int)((nd + 255) / 256);
  if (hipMalloc(&btil, sizeof(double) * b->total_dof) != hipSuccess ||
      hipMalloc(&eta0, sizeof(double) * b->total_dof) != hipSuccess ||
      hipMalloc(&phi, sizeof(double) * b->total_dof) != hipSuccess ||
      hipMalloc(&psi, sizeof(double) * b->total_psi) != hipSuccess ||
      hipMalloc(&xi, sizeof(double) * window * b->total_dof) != hipSuccess ||
      hipMalloc(&u, sizeof(double) * np) != hipSuccess ||
      hipMalloc(&dsc, sizeof(double) * 8) != hipSuccess ||
      hipMalloc(&gq, sizeof(double) * n * ROM_GSTRIDE) != hipSuccess ||
      hipMalloc(&cq, sizeof(double) * n * ROM_GSTRIDE) != hipSuccess ||
      hipMalloc(&part, sizeof(double) * (size_t)n * rom->n_ord * nch_res) != hipSuccess ||
      hipMalloc(&rmu, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&mask, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&midx, sizeof(int32_t) * n) != hipSuccess)
    st = RTE_ENOMEM;
  auto release = [&]() {
    for (void* p : {(void*)btil, (void*)eta0, (void*)phi, (void*)psi, (void*)xi, (void*)u, (void*)dsc,
                    (void*)gq, (void*)cq, (void*)part, (void*)rmu, (void*)mask, (void*)midx})
      (void)hipFree(p);
  };
  Space sp1;  // one psi-space vector
  if (st == RTE_OK) st = sp1.init({np});
  Fgmres* fg = st == RTE_OK ? fgmres_for(b, 40) : nullptr;
  if (st == RTE_OK && !fg) st = RTE_ENOMEM;
  std::vector<int32_t> sampled{mu1_index};
  std::vector<double> maxres;
  int truncated = 0;
  double t0 = now_s();
  // step 1: b~ and eta0 = Sigma_s b~ for every training parameter
  if (st == RTE_OK) st = autotune_sweep(b, 0, sigma_t, s);
  if (st == RTE_OK) st = sweep_launch(b, 0, sigma_t, nullptr, nullptr, G, inflow, nullptr, s);
  if (st == RTE_OK) st = reduce_partials(b, 0, 1.0, nullptr, 0.0, btil, s);
  if (st == RTE_OK) {
    if (b->n_fields > 0) {
      st = field_apply(b, sigma_s, btil, eta0, false, nullptr, s);
    } else {
      dim3 grid((unsigned)std::min<int64_t>((nd + 255) / 256, 1024), n);
      hipLaunchKernelGGL(k_scale_sigma, grid, dim3(256), 0, s, b->d_inst, b->d_region, sigma_s,
                         b->max_regions, btil, eta0);
    }
    if (st == RTE_OK && hipStreamSynchronize(s) != hipSuccess) st = RTE_EHIP;
  }
  t_step[0] += now_s() - t0;
  std::vector<rte_solve_stats> stats(n);
  std::vector<int32_t> onehot(n, 0);
  for (int k = 1; st == RTE_OK; ++k) {
    const int cur = sampled.back();
    // step 2(a): FP64 FGMRES-DSA solve with zero initial guess, xi recurrence
    t0 = now_s();
    std::fill(onehot.begin(), onehot.end(), 0);
    onehot[cur] = 1;
    if (hipMemcpy(mask, onehot.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice) != hipSuccess) {
      st = RTE_EHIP;
      break;
    }
    rte_solve_opts o{};
    o.precond = RTE_PC_DSA;
    o.m = 40;
    o.max_cycles = 20;
    o.sweep_dtype = RTE_F64;
    o.rtol = hf_rtol;
    o.window = 0;
    if (hf_dsa_tol > 0.0) {   // V-cycle-preconditioned GMRES to hf_dsa_tol
      o.dsa_inner_max = 4000;
      o.dsa_restart = 60;
      o.dsa_inner_tol = hf_dsa_tol;
    } else {                  // one multigrid V-cycle per DSA application
      o.dsa_inner_max = 1;
      o.dsa_restart = 0;
      o.dsa_inner_tol = 0.0;
    }
    SolveCtx c{};
    c.opts = &o;
    c.sigma_t = sigma_t;
    c.sigma_s = sigma_s;
    c.G = G;
    c.inflow = inflow;
    c.init_active = mask;
    c.keep = window;
    st = fg->solve(c, phi, stats.data(), s);
    if (st < 0) break;
    st = RTE_OK;
    const int jd = fg->rec_jdone[cur];
    const int nxi = std::min(window, jd + 1);
    std::vector<double> Hh((size_t)(window + 1) * window), beta(n);
    if (hipMemcpy(Hh.data(), fg->recH + (size_t)cur * (window + 1) * window,
                  sizeof(double) * (window + 1) * window, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(beta.data(), fg->recBeta, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess) {
      st = RTE_EHIP;
      break;
    }
    const int64_t off = b->inst[cur].dof_off;
    // xi_0 = phi / beta ; xi_l = (z_{l-1} - sum_{i<l} H[i][l-1] xi_i) / H[l][l-1]
    Space spd;
    if ((st = spd.init({nd})) != RTE_OK) break;
    st = kaxpby(spd, 1.0 / beta[cur], phi + off, 0.0, xi + off, nullptr, s);
    int made = 1;
    for (int l = 1; l < nxi && st == RTE_OK; ++l) {
      const double hll = Hh[(size_t)l * window + (l - 1)];
      if (!(hll != 0.0)) break;
      double* xl = xi + (int64_t)l * b->total_dof + off;
      st = kaxpby(spd, 1.0, fg->recZ + (int64_t)(l - 1) * b->total_dof + off, 0.0, xl, nullptr, s);
      for (int i = 0; i < l && st == RTE_OK; ++i)
        st = kaxpby(spd, -Hh[(size_t)i * window + (l - 1)], xi + (int64_t)i * b->total_dof + off, 1.0, xl,
                    nullptr, s);
      if (st == RTE_OK) st = kaxpby(spd, 0.0, xl, 1.0 / hll, xl, nullptr, s);
      ++made;
    }
    spd.release();
    if (hipStreamSynchronize(s) != hipSuccess) st = RTE_EHIP;
    t_step[1] += now_s() - t0;
    // steps 2(b) + 2(c): psi-storing sweeps, MGS with truncation, reduced operators
    for (int l = 0; l < made && st == RTE_OK; ++l) {
      t0 = now_s();
      st = sweep_launch(b, 0, sigma_t, sigma_s, xi + (int64_t)l * b->total_dof, nullptr, nullptr, psi, s, mask);
      if (st == RTE_OK && hipStreamSynchronize(s) != hipSuccess) st = RTE_EHIP;
      t_step[2] += now_s() - t0;
      t0 = now_s();
      if (st == RTE_OK)
        st = hipMemcpyAsync(u, psi + b->inst[cur].psi_off, sizeof(double) * np, hipMemcpyDeviceToDevice, s) ==
                     hipSuccess ? RTE_OK : RTE_EHIP;
      for (int i = 0; i < rom->r && st == RTE_OK; ++i) {
        const double* Ui = rom->U + (int64_t)i * np;
        st = kdot(sp1, Ui, u, part, dsc, 1, nullptr, s);
        if (st == RTE_OK) {
          hipLaunchKernelGGL(k_axpy_dev, dim3(1024), dim3(256), 0, s, np, dsc, -1.0, Ui, u);
          if (hipGetLastError() != hipSuccess) st = RTE_EHIP;
        }
      }
      double nrm = 0.0;
      if (st == RTE_OK) st = knorm(sp1, u, part, dsc, 1, nullptr, s);
      if (st == RTE_OK && (hipMemcpyAsync(&nrm, dsc, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                           hipStreamSynchronize(s) != hipSuccess))
        st = RTE_EHIP;
      if (st == RTE_OK) {
        if (nrm > eps_qr && rom->r < rom->rcap) {
          st = kaxpby(sp1, 1.0 / nrm, u, 0.0, rom->U + (int64_t)rom->r * np, nullptr, s);
          if (st == RTE_OK) st = rom_add_column(rom, b, s);
        } else {
          ++truncated;
        }
      }
      t_step[3] += now_s() - t0;
    }
    if (st != RTE_OK || k == n_giter) break;
    // step 3: ROM solves and residual indicator for every unsampled parameter
    t0 = now_s();
    std::vector<int32_t> unsampled;
    std::vector<int32_t> um(n, 1);
    for (int q : sampled) um[q] = 0;
    for (int q = 0; q < n; ++q)
      if (um[q]) unsampled.push_back(q);
    if (unsampled.empty()) {
      t_step[4] += now_s() - t0;
      break;
    }
    if (hipMemcpy(mask, um.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(midx, unsampled.data(), sizeof(int32_t) * unsampled.size(), hipMemcpyHostToDevice) != hipSuccess) {
      st = RTE_EHIP;
      break;
    }
    st = rom_project(rom, b, nullptr, eta0, gq, mask, s);
    if (st != RTE_OK) break;
    {
      RomScratch* rsc = scratch_for(b, 1);
      const RomDev* tab = rsc ? rom_table(rom, rsc, b, s) : nullptr;
      if (!tab) {
        st = RTE_EHIP;
        break;
      }
      hipLaunchKernelGGL(k_rom_solve, dim3(n), dim3(256), 0, s, n, tab, sigma_t, sigma_s, b->max_regions, gq, cq,
                         ROM_GSTRIDE, (int32_t*)nullptr, mask);
    }
    // compact c to the unsampled order for the residual kernel
    std::vector<double> ch((size_t)n * ROM_GSTRIDE), cc((size_t)unsampled.size() * ROM_GSTRIDE, 0.0);
    if (hipMemcpyAsync(ch.data(), cq, sizeof(double) * n * ROM_GSTRIDE, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = RTE_EHIP;
      break;
    }
    for (size_t q = 0; q < unsampled.size(); ++q)
      for (int kk = 0; kk < rom->r; ++kk) cc[q * ROM_GSTRIDE + kk] = ch[(size_t)unsampled[q] * ROM_GSTRIDE + kk];
    if (hipMemcpy(gq, cc.data(), sizeof(double) * cc.size(), hipMemcpyHostToDevice) != hipSuccess) {
      st = RTE_EHIP;
      break;
    }
    const int nmu = (int)unsampled.size();
    int nch_used = nch_res;
    if (b->n_fields > 0) {
      const int64_t ncell_f = nd / 4;
      nch_used = (int)((ncell_f + 255) / 256);
      hipLaunchKernelGGL(k_greedy_res_field, dim3(nch_used, rom->n_ord), dim3(256), 0, s, rom->r, ROM_GSTRIDE,
                         rom->n_ord, ncell_f, rom->U, rom->DU, rom->Ww, nmu, midx, gq, b->d_fblk, b->n_fields,
                         sigma_t, sigma_s, b->max_regions, eta0, part, nch_used);
    } else {
      hipLaunchKernelGGL(k_greedy_res, dim3(nch_res, rom->n_ord), dim3(256), 0, s, rom->r, ROM_GSTRIDE,
                         rom->n_ord, nd, rom->nloc, rom->d_region, rom->U, rom->DU, rom->Ww, nmu, midx,
                         gq, sigma_t, sigma_s, b->max_regions, eta0, part, nch_res);
    }
    hipLaunchKernelGGL(k_greedy_max, dim3((nmu + 63) / 64), dim3(64), 0, s, nmu, rom->n_ord, nch_used,
                       part, rmu);
    std::vector<double> rh(nmu);
    if (hipMemcpyAsync(rh.data(), rmu, sizeof(double) * nmu, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = RTE_EHIP;
      break;
    }
    int best = -1;
    double bv = -1.0;
    for (int q = 0; q < nmu; ++q)
      if (rh[q] > bv) {  // strict: ties keep the lowest training index
        bv = rh[q];
        best = unsampled[q];
      }
    maxres.push_back(bv);
    t_step[4] += now_s() - t0;
    if (bv < eps_rom) break;
    sampled.push_back(best);
  }
  (void)ncell;
  sp1.release();
  release();
  if (st != RTE_OK) return cleanup(st);
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->n_sampled = (int)sampled.size();
    for (size_t q = 0; q < sampled.size() && q < 256; ++q) rep->sampled[q] = sampled[q];
    for (size_t q = 0; q < maxres.size() && q < 256; ++q) rep->max_residual[q] = maxres[q];
    rep->rank = rom->r;
    rep->truncated = truncated;
    for (int q = 0; q < 5; ++q) rep->seconds_step[q] = t_step[q];
  }
  *out = rom;
  return RTE_OK;
}
