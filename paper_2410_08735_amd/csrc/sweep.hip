// Transport sweep (section 3.1) and the quadrature reduction phi = sum_j w_j psi_j.
//
// X-Y geometry, Q1 upwind DG.  One work group handles one instance, one
// quadrant of directions and a block of G ordinates of that quadrant.  Cells
// are visited by anti-diagonals of the quadrant's upwind order (the KBA
// wavefront): every cell on diagonal s depends only on cells of diagonal
// s - 1, so the whole diagonal times G ordinates is processed in parallel and
// one barrier separates diagonals.  Outgoing face traces go to LDS: the
// x-trace of a cell indexed by its row, the y-trace by its column; no two
// cells of one diagonal share a row or a column, so a single LDS buffer of each
// kind needs no double buffering.
//
// Every cell is solved in the quadrant's mirrored coordinates (s -> -s along
// each reversed axis, which flips the sign of the odd Legendre modes), where
// the local system is always
//   (sigma I + a K (x) I + b I (x) K) psi = q + inflow terms,
//   K = [[1, sqrt3], [-sqrt3, 3]],  a = |Omega_x| / h_x,  b = |Omega_y| / h_y,
// with K the upwind-flux matrix of the orthonormal degree-1 Legendre basis
// for a positive direction.  The 4x4 solve is done in closed form: the
// matrices aI + bK form a commutative algebra (K^2 = 4K - 6I), so the block
// elimination along y needs one reciprocal per cell.
//
// The G lanes holding one cell's ordinates are adjacent; their weighted sum
// (the quadrature reduction) is formed with cross-lane shuffles and written
// once per cell as one partial scalar flux of the ordinate block.  A second,
// deterministic pass sums the partials in a fixed order (reduce_partials).
#include <algorithm>
#include <cmath>

#include "rte_internal.h"

namespace rte {

template <typename real>
struct Vec4 {
  real v[4];
};

// Cross-lane moves inside a 16-lane DPP row: quad_perm [1,0,3,2] (xor 1),
// quad_perm [2,3,0,1] (xor 2), row_half_mirror (i <-> 7 - i within 8 lanes) and
// row_mirror (i <-> 15 - i).  Every lane reads a valid source lane, so
// bound_ctrl (set: it lets the compiler fold a move into the add that uses it)
// changes no value.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffll), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// The work item of this work group.  per_xcd > 0: the hardware deals work
// groups to the 8 XCDs round robin, and this mapping gives each XCD a
// contiguous run of per_xcd items (an instance's ordinate blocks share one
// L2).  per_xcd = 0: work group b takes item b (items already in the order
// they should start, dealt round robin over the XCDs by the hardware).
__device__ __forceinline__ int work_item(int per_xcd) {
  return per_xcd > 0 ? (int)(blockIdx.x % 8u) * per_xcd + (int)(blockIdx.x / 8u) : (int)blockIdx.x;
}

// Sum over each aligned group of G adjacent lanes; every lane of the group
// receives the group's sum.  Steps inside a row use DPP; across rows (G = 32)
// a cross-lane shuffle.
template <int G, typename real>
__device__ __forceinline__ real group_sum(real c) {
  if (G >= 2) c += dpp_move<0xB1>(c);
  if (G >= 4) c += dpp_move<0x4E>(c);
  if (G >= 8) c += dpp_move<0x141>(c);
  if (G >= 16) c += dpp_move<0x140>(c);
  if (G >= 32) c += __shfl_xor(c, 16, 32);
  return c;
}

// a * b + c as one fused multiply-add (written out so that a product shared by
// two sums is not formed once and added twice).
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1/x: the hardware reciprocal (1 ulp) in FP32, a correctly rounded division in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Closed-form solve of (sig I + a K(x)I + b I(x)K) x = r, dof order p + 2q.
// Algebra elements (al, be) stand for al I + be K acting on the p-pair.
template <typename real>
__device__ __forceinline__ void local_solve(real sig, real a, real b, const real r[4], real x[4]) {
  const real r3 = (real)1.7320508075688772935;
  const real a0 = sig + b;
  const real a1 = sig + (real)3 * b;
  const real adj0a = a0 + (real)4 * a, adj0b = -a;
  const real det0 = a0 * a0 + (real)4 * a0 * a + (real)6 * a * a;
  const real b2 = (real)3 * b * b;
  const real sa = det0 * a1 + b2 * adj0a;
  const real sb = (det0 - b2) * a;
  const real detS = sa * sa + (real)4 * sa * sb + (real)6 * sb * sb;
  const real adjSa = sa + (real)4 * sb, adjSb = -sb;
  const real inv = recip(det0 * detS);
  // u = adj0 r0, r0 = (r[0], r[1])
  real k0 = r[0] + r3 * r[1], k1 = -r3 * r[0] + (real)3 * r[1];
  const real u0 = adj0a * r[0] + adj0b * k0, u1 = adj0a * r[1] + adj0b * k1;
  const real br3 = b * r3;
  const real t0 = det0 * r[2] + br3 * u0, t1 = det0 * r[3] + br3 * u1;
  k0 = t0 + r3 * t1;
  k1 = -r3 * t0 + (real)3 * t1;
  const real f1 = det0 * inv;
  x[2] = (adjSa * t0 + adjSb * k0) * f1;
  x[3] = (adjSa * t1 + adjSb * k1) * f1;
  const real e0 = r[0] - br3 * x[2], e1 = r[1] - br3 * x[3];
  k0 = e0 + r3 * e1;
  k1 = -r3 * e0 + (real)3 * e1;
  const real f0 = detS * inv;
  x[0] = (adj0a * e0 + adj0b * k0) * f0;
  x[1] = (adj0a * e1 + adj0b * k1) * f0;
}

// The same solve with its (sigma, a, b)-dependent part precomputed.  Every
// 2 x 2 block above is al I - be K, and K^2 = 4 K - 6 I, so such blocks commute
// and each is kept as (al - be, al - 3 be, sqrt3 be):
//   (al I - be K) v = ((al - be) v0 - sqrt3 be v1, (al - 3 be) v1 + sqrt3 be v0).
// With M = adj0 / det0 and N = det0 adjS / detS the solve is
//   v = M r_lo,  s = r_hi + sqrt3 b v,  x_hi = N s,  x_lo = M (r_lo - sqrt3 b x_hi),
// c[0..2] = M, c[3..5] = N, and c[6..8] = sqrt3 b M, with which the last step
// is x_lo = v - (sqrt3 b M) x_hi, the subtraction fused into its multiply-adds
// (14 operations instead of 16); c[9] = 0 pads the table.  Coefficients in
// FP64 whatever the sweep's precision.
__device__ __forceinline__ void solve_coef(double sig, double a, double b, double c[10]) {
  const double r3 = 1.7320508075688772935;
  const double a0 = sig + b, a1 = sig + 3.0 * b;
  const double adj0a = a0 + 4.0 * a;
  const double det0 = a0 * a0 + 4.0 * a0 * a + 6.0 * a * a;
  const double b2 = 3.0 * b * b;
  const double sa = det0 * a1 + b2 * adj0a;
  const double sb = (det0 - b2) * a;
  const double detS = sa * sa + 4.0 * sa * sb + 6.0 * sb * sb;
  const double adjSa = sa + 4.0 * sb;
  const double ma = adj0a / det0, mb = a / det0;
  const double na = det0 * adjSa / detS, nb = det0 * sb / detS;
  c[0] = ma - mb;
  c[1] = ma - 3.0 * mb;
  c[2] = r3 * mb;
  c[3] = na - nb;
  c[4] = na - 3.0 * nb;
  c[5] = r3 * nb;
  c[6] = r3 * b * c[0];
  c[7] = r3 * b * c[1];
  c[8] = r3 * b * c[2];
  c[9] = 0.0;
}

template <typename real>
__device__ __forceinline__ void solve_apply(const real c[6], real br3, const real r[4], real x[4]) {
  const real v0 = c[0] * r[0] - c[2] * r[1], v1 = c[1] * r[1] + c[2] * r[0];
  const real s0 = r[2] + br3 * v0, s1 = r[3] + br3 * v1;
  x[2] = c[3] * s0 - c[5] * s1;
  x[3] = c[4] * s1 + c[5] * s0;
  const real e0 = r[0] - br3 * x[2], e1 = r[1] - br3 * x[3];
  x[0] = c[0] * e0 - c[2] * e1;
  x[1] = c[1] * e1 + c[2] * e0;
}

// The same with the last step as x_lo = v - Q x_hi, Q = sqrt3 b M in c[6..8].
template <typename real>
__device__ __forceinline__ void solve_apply_q(const real c[9], real br3, const real r[4], real x[4]) {
  const real v0 = fmadd(-c[2], r[1], c[0] * r[0]), v1 = fmadd(c[2], r[0], c[1] * r[1]);
  const real s0 = fmadd(br3, v0, r[2]), s1 = fmadd(br3, v1, r[3]);
  x[2] = fmadd(-c[5], s1, c[3] * s0);
  x[3] = fmadd(c[5], s0, c[4] * s1);
  x[0] = fmadd(-c[6], x[2], fmadd(c[8], x[3], v0));
  x[1] = fmadd(-c[7], x[3], fmadd(-c[8], x[2], v1));
}

// Planes of two reals per (region, lane ordinate) in the row-slot kernel's
// coefficient table: M and N (three planes), and in FP32 also Q (two more).
template <typename real>
__host__ __device__ constexpr int coef_planes() {
  return sizeof(real) == 4 ? 5 : 3;
}

// Two reals, the unit of the coefficient table in LDS.
template <typename real>
struct Pair2;
template <>
struct Pair2<float> {
  using T = float2;
};
template <>
struct Pair2<double> {
  using T = double2;
};

// The ordinates one lane carries (OPL of them: lane g of a cell group holds
// ordinates g*OPL .. g*OPL+OPL-1 of the work item) and what the sweep needs
// of each: advection coefficients, quadrature weight, angular-flux output.
template <typename real, int OPL>
struct LaneOrds {
  real a[OPL], b[OPL], wt[OPL];
  double* psi[OPL];
};

template <typename real, int G, int OPL>
__device__ __forceinline__ LaneOrds<real, OPL> lane_ords(const SweepItem& it, const InstDev& I, int g,
                                                         const double* __restrict__ ox,
                                                         const double* __restrict__ oy,
                                                         const double* __restrict__ w,
                                                         const int32_t* __restrict__ perm, double* psi_out) {
  LaneOrds<real, OPL> L;
#pragma unroll
  for (int o = 0; o < OPL; ++o) {
    const bool on = g * OPL + o < it.count;
    const int js = I.ord_off + it.first + (on ? g * OPL + o : 0);
    L.a[o] = (real)(fabs(ox[js]) / I.hx);
    L.b[o] = (real)(fabs(oy[js]) / I.hy);
    L.wt[o] = on ? (real)w[js] : (real)0;
    L.psi[o] = (psi_out && on) ? psi_out + I.psi_off + (int64_t)perm[js] * I.nx * I.ny * 4 : nullptr;
  }
  return L;
}

// One cell (mirrored column i, row r; physical index cell) for the lane's
// ordinates: inflow traces from LDS (or the boundary value), the closed-form
// local solve, outflow traces back to LDS, and the lane's weighted sum c.
template <typename real, int G, int OPL>
__device__ __forceinline__ void cell_update(const LaneOrds<real, OPL>& L, int g, int i, int r, int64_t cell,
                                            real sig, real q0, real q1, real q2, real q3, real gx, real gy,
                                            real mx, real my, real* xtr, real* ytr, real c[4]) {
  const real r3 = (real)1.7320508075688772935;
  c[0] = c[1] = c[2] = c[3] = (real)0;
#pragma unroll
  for (int o = 0; o < OPL; ++o) {
    // trace slots [row or column][o][g][2]: the G lanes of a cell touch one
    // contiguous run of LDS per ordinate (no bank conflicts within a cell)
    const int xo = ((r * OPL + o) * G + g) * 2, yo = ((i * OPL + o) * G + g) * 2;
    const real a = L.a[o], b = L.b[o];
    real tx0, tx1, ty0, ty1;
    if (i == 0) { tx0 = gx; tx1 = 0; } else { tx0 = xtr[xo]; tx1 = xtr[xo + 1]; }
    if (r == 0) { ty0 = gy; ty1 = 0; } else { ty0 = ytr[yo]; ty1 = ytr[yo + 1]; }
    real rhs[4];
    rhs[0] = q0 + a * tx0 + b * ty0;
    rhs[1] = mx * q1 - r3 * a * tx0 + b * ty1;
    rhs[2] = my * q2 + a * tx1 - r3 * b * ty0;
    rhs[3] = mx * my * q3 - r3 * (a * tx1 + b * ty1);
    real x[4];
    local_solve<real>(sig, a, b, rhs, x);
    xtr[xo] = fmadd(r3, x[1], x[0]);
    xtr[xo + 1] = fmadd(r3, x[3], x[2]);
    ytr[yo] = fmadd(r3, x[2], x[0]);
    ytr[yo + 1] = fmadd(r3, x[3], x[1]);
#pragma unroll
    for (int d = 0; d < 4; ++d) c[d] += L.wt[o] * x[d];
    if (L.psi[o]) {
      double* out = L.psi[o] + 4 * cell;
      out[0] = (double)x[0];
      out[1] = (double)(mx * x[1]);
      out[2] = (double)(my * x[2]);
      out[3] = (double)(mx * my * x[3]);
    }
  }
}

// Reals per column of the row-slot kernel's y-trace buffer: the 2 G OPL
// traces of the column, padded in FP32 so that consecutive columns (the ones
// the slots of a wave touch together, one column apart) start 2 G banks apart
// and the slots of a wave read disjoint banks.  FP64 keeps the unpadded
// layout (its buffer would not fit the LDS budget at 96 columns).
template <typename real, int G, int OPL>
__host__ __device__ constexpr int ytr_stride() {
  return sizeof(real) == 4 ? 2 * G * OPL + ((2 * G - 2 * G * OPL) % 64 + 64) % 64 : 2 * G * OPL;
}

// The same for the row-slot kernel, where a slot owns whole rows: the x trace
// passes to the slot's next cell of the row in registers (xt, holding the
// inflow trace before the first column), the y trace to the next row through
// LDS (ytr, preloaded with the inflow trace), and the local solve reads its
// precomputed coefficients (ctab: this cell's region's block of Pair2 entries
// [plane][OPL][G], so every address is a compile-time offset from the
// lane's base).  q0..q3 arrive scaled and already in mirrored orientation.
// One ordinate o of one cell from its inflow traces (tx along x, ty along y):
// the right-hand side, the local solve with the coefficients at e (planes
// OPL * G apart), and the solution x in mirrored orientation.
template <typename real, int G, int OPL>
__device__ __forceinline__ void ordinate_solve(const LaneOrds<real, OPL>& L, int o, real q0, real q1, real q2,
                                               real q3, real tx0, real tx1, real ty0, real ty1,
                                               const typename Pair2<real>::T* e, real x[4]) {
  const real r3 = (real)1.7320508075688772935;
  const real a = L.a[o], b = L.b[o];
  const real ra = r3 * a, rb = r3 * b;
  real rhs[4];
  rhs[0] = fmadd(b, ty0, fmadd(a, tx0, q0));
  rhs[1] = fmadd(b, ty1, fmadd(-ra, tx0, q1));
  rhs[2] = fmadd(-rb, ty0, fmadd(a, tx1, q2));
  rhs[3] = fmadd(-rb, ty1, fmadd(-ra, tx1, q3));
  if constexpr (coef_planes<real>() == 5) {
    const typename Pair2<real>::T p0 = e[0], p1 = e[OPL * G], p2 = e[2 * OPL * G], p3 = e[3 * OPL * G],
                                  p4 = e[4 * OPL * G];
    const real cf[9] = {p0.x, p0.y, p1.x, p1.y, p2.x, p2.y, p3.x, p3.y, p4.x};
    solve_apply_q<real>(cf, rb, rhs, x);
  } else {
    const typename Pair2<real>::T p0 = e[0], p1 = e[OPL * G], p2 = e[2 * OPL * G];
    const real cf[6] = {p0.x, p0.y, p1.x, p1.y, p2.x, p2.y};
    solve_apply<real>(cf, rb, rhs, x);
  }
}

// The angular flux of one ordinate in physical orientation, in FP64.
template <typename real>
__device__ __forceinline__ void store_psi(double* out, const real x[4], real mx, real my) {
  out[0] = (double)x[0];
  out[1] = (double)(mx * x[1]);
  out[2] = (double)(my * x[2]);
  out[3] = (double)(mx * my * x[3]);
}

template <typename real, int G, int OPL, bool PSI>
__device__ __forceinline__ void cell_update_rows(const LaneOrds<real, OPL>& L, int g, int i, int64_t cell,
                                                 real q0, real q1, real q2, real q3, real mx, real my,
                                                 real xt[OPL][2], real* ytr, real c[4],
                                                 const typename Pair2<real>::T* ctab) {
  const real r3 = (real)1.7320508075688772935;
  c[0] = c[1] = c[2] = c[3] = (real)0;
#pragma unroll
  for (int o = 0; o < OPL; ++o) {
    const int yo = i * ytr_stride<real, G, OPL>() + (o * G + g) * 2;  // [column (padded)][o][g][2]
    real x[4];
    ordinate_solve<real, G, OPL>(L, o, q0, q1, q2, q3, xt[o][0], xt[o][1], ytr[yo], ytr[yo + 1], ctab + o * G, x);
    xt[o][0] = fmadd(r3, x[1], x[0]);
    xt[o][1] = fmadd(r3, x[3], x[2]);
    ytr[yo] = fmadd(r3, x[2], x[0]);
    ytr[yo + 1] = fmadd(r3, x[3], x[1]);
#pragma unroll
    for (int d = 0; d < 4; ++d) c[d] = fmadd(L.wt[o], x[d], c[d]);
    if (PSI && L.psi[o]) store_psi<real>(L.psi[o] + 4 * cell, x, mx, my);
  }
}

// The same for the wave-per-item kernel: the y traces in registers (yi in,
// yo out; the kernel moves them between rows), one lane per cell.
template <typename real, int OPL, bool PSI>
__device__ __forceinline__ void cell_update_wave(const LaneOrds<real, OPL>& L, int64_t cell, real q0, real q1,
                                                 real q2, real q3, real mx, real my, real xt[OPL][2],
                                                 const real yi[OPL][2], real yo[OPL][2], real c[4],
                                                 const typename Pair2<real>::T* ctab) {
  const real r3 = (real)1.7320508075688772935;
  c[0] = c[1] = c[2] = c[3] = (real)0;
#pragma unroll
  for (int o = 0; o < OPL; ++o) {
    real x[4];
    ordinate_solve<real, 1, OPL>(L, o, q0, q1, q2, q3, xt[o][0], xt[o][1], yi[o][0], yi[o][1], ctab + o, x);
    xt[o][0] = fmadd(r3, x[1], x[0]);
    xt[o][1] = fmadd(r3, x[3], x[2]);
    yo[o][0] = fmadd(r3, x[2], x[0]);
    yo[o][1] = fmadd(r3, x[3], x[1]);
#pragma unroll
    for (int d = 0; d < 4; ++d) c[d] = fmadd(L.wt[o], x[d], c[d]);
    if (PSI && L.psi[o]) store_psi<real>(L.psi[o] + 4 * cell, x, mx, my);
  }
}

// The group's quadrature sum, written once per cell in physical orientation.
template <typename real, int G>
__device__ __forceinline__ void store_partial(real c[4], int g, real mx, real my, real* P, int64_t cell) {
  if constexpr (G == 4 || G == 8) {
    // a reduce-scatter: each exchange halves the moments a lane carries (4
    // exchanges for G = 8 instead of 12), and the lanes that end with a
    // moment's sum store it.  First exchange: the partner differs in the
    // group's top lane bit; a lane keeps moments {0, 1} (bit clear) or {2, 3}.
    const bool hi = (g & (G / 2)) != 0;
    real ka = hi ? c[2] : c[0], kb = hi ? c[3] : c[1];
    const real sa = hi ? c[0] : c[2], sb = hi ? c[1] : c[3];
    if constexpr (G == 8) {  // half-row mirror: lane g with 7 - g
      ka += dpp_move<0x141>(sa);
      kb += dpp_move<0x141>(sb);
    } else {  // lane g with g ^ 2
      ka += dpp_move<0x4E>(sa);
      kb += dpp_move<0x4E>(sb);
    }
    // second exchange: the partner differs in the next bit; a lane keeps
    // moment 2 hi + mid
    const bool mid = (g & (G / 4)) != 0;
    real k = mid ? kb : ka;
    const real sk = mid ? ka : kb;
    if constexpr (G == 8) {
      k += dpp_move<0x4E>(sk);
      k += dpp_move<0xB1>(k);  // the two lanes of a pair hold the same moment
    } else {
      k += dpp_move<0xB1>(sk);
    }
    const int m = (hi ? 2 : 0) + (mid ? 1 : 0);
    if (G == 4 || (g & 1) == 0) {
      const real f = ((m & 1) ? mx : (real)1) * ((m & 2) ? my : (real)1);
      P[4 * cell + m] = f * k;
    }
  } else {
#pragma unroll
    for (int d = 0; d < 4; ++d) c[d] = group_sum<G, real>(c[d]);
    if (g == 0) {
      real* o = P + 4 * cell;
      o[0] = c[0];
      o[1] = mx * c[1];
      o[2] = my * c[2];
      o[3] = mx * my * c[3];
    }
  }
}

template <typename real, int G, int OPL>
__global__ void __launch_bounds__(512) sweep2d_kernel(
    const InstDev* __restrict__ insts, const SweepItem* __restrict__ items,
    const double* __restrict__ ox, const double* __restrict__ oy, const double* __restrict__ w,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ region,
    const double* __restrict__ sigma_t, const double* __restrict__ sigma_s, int max_regions,
    const double* __restrict__ qx, const double* __restrict__ qadd,
    const double* __restrict__ inflow, real* __restrict__ part, double* __restrict__ psi_out,
    const int32_t* __restrict__ active, int n_items, int per_xcd) {
  // Work groups are dealt to the 8 XCDs round robin; give each XCD a contiguous
  // run of items, so an instance's ordinate blocks share one L2.
  const int item = work_item(per_xcd);
  if (item >= n_items) return;
  const SweepItem it = items[item];
  if (active && !active[it.inst]) return;
  const InstDev I = insts[it.inst];
  const int tid = threadIdx.x;
  const int g = tid % G;
  const int slot = tid / G;
  const int S = blockDim.x / G;
  const int nx = I.nx, ny = I.ny;
  const LaneOrds<real, OPL> L = lane_ords<real, G, OPL>(it, I, g, ox, oy, w, perm, psi_out);
  const bool fx = it.quadrant & 1, fy = it.quadrant & 2;
  const real mx = fx ? (real)-1 : (real)1, my = fy ? (real)-1 : (real)1;
  // inflow [n_inst][4] = left, right, bottom, top; in mirrored coordinates the
  // x-inflow face is the left one unless Omega_x < 0, the y-inflow face the
  // bottom one unless Omega_y < 0
  const double gsc = sqrt(I.hx * I.hy);
  const real gx = inflow ? (real)(inflow[4 * it.inst + (fx ? 1 : 0)] * gsc) : (real)0;
  const real gy = inflow ? (real)(inflow[4 * it.inst + (fy ? 3 : 2)] * gsc) : (real)0;
  extern __shared__ unsigned char smem_raw[];
  real* xtr = reinterpret_cast<real*>(smem_raw);  // [ny][OPL][G][2]
  real* ytr = xtr + (size_t)ny * G * OPL * 2;     // [nx][OPL][G][2]
  const double* st = sigma_t + (size_t)it.inst * max_regions;
  const double* ss = sigma_s ? sigma_s + (size_t)it.inst * max_regions : nullptr;
  const int32_t* reg = region + I.region_off;
  const double* qxi = qx ? qx + I.dof_off : nullptr;
  const double* qai = qadd ? qadd + I.dof_off : nullptr;
  real* P = part + it.part_off;

  for (int s = 0; s < nx + ny - 1; ++s) {
    const int r_lo = max(0, s - nx + 1), r_hi = min(ny - 1, s);
    for (int r = r_lo + slot; r <= r_hi; r += S) {
      const int i = s - r;
      const int ip = fx ? nx - 1 - i : i;
      const int kp = fy ? ny - 1 - r : r;
      const int cell = kp * nx + ip;
      double q[4] = {0.0, 0.0, 0.0, 0.0};
      const int rg = reg[cell];
      if (qxi) {
        const double sg = ss[rg];
        const double4 v = *reinterpret_cast<const double4*>(qxi + 4 * (int64_t)cell);
        q[0] = sg * v.x; q[1] = sg * v.y; q[2] = sg * v.z; q[3] = sg * v.w;
      }
      if (qai) {
        const double4 v = *reinterpret_cast<const double4*>(qai + 4 * (int64_t)cell);
        q[0] += v.x; q[1] += v.y; q[2] += v.z; q[3] += v.w;
      }
      real c[4];
      cell_update<real, G, OPL>(L, g, i, r, cell, (real)st[rg], (real)q[0], (real)q[1], (real)q[2], (real)q[3],
                                gx, gy, mx, my, xtr, ytr, c);
      store_partial<real, G>(c, g, mx, my, P, cell);
    }
    __syncthreads();
  }
}

// Cross sections that vary inside the cells (section 5.3): the local matrix
// of a cell-ordinate is the cell's full sigma_t mass block (mirrored with the
// quadrant: entry (a, b) times s_a s_b, s = (1, mx, my, mx my)) plus the
// upwind advection a K (x) I + b I (x) K, and is solved by Gaussian
// elimination without pivoting (its symmetric part is positive definite:
// that of the mass block and of K, diag(1, 3), are).
template <typename real>
__device__ __forceinline__ void solve4_nopivot(real A[16], real x[4]) {
  real inv[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    inv[k] = (real)1 / A[5 * k];
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      const real f = A[4 * i + k] * inv[k];
#pragma unroll
      for (int j = k + 1; j < 4; ++j) A[4 * i + j] = fmadd(-f, A[4 * k + j], A[4 * i + j]);
      x[i] = fmadd(-f, x[k], x[i]);
    }
  }
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    real t = x[i];
#pragma unroll
    for (int j = i + 1; j < 4; ++j) t = fmadd(-A[4 * i + j], x[j], t);
    x[i] = t * inv[i];
  }
}

// One cell of the field kernel for the lane's ordinates: Sm is the mirrored
// sigma_t block, q0..q3 the mirrored source moments; traces and the weighted
// sum as in cell_update.
template <typename real, int G, int OPL>
__device__ __forceinline__ void cell_update_field(const LaneOrds<real, OPL>& L, int g, int i, int r, int64_t cell,
                                                  const real Sm[16], real q0, real q1, real q2, real q3, real gx,
                                                  real gy, real mx, real my, real* xtr, real* ytr, real c[4]) {
  const real r3 = (real)1.7320508075688772935;
  c[0] = c[1] = c[2] = c[3] = (real)0;
#pragma unroll
  for (int o = 0; o < OPL; ++o) {
    const int xo = ((r * OPL + o) * G + g) * 2, yo = ((i * OPL + o) * G + g) * 2;
    const real a = L.a[o], b = L.b[o];
    real tx0, tx1, ty0, ty1;
    if (i == 0) { tx0 = gx; tx1 = 0; } else { tx0 = xtr[xo]; tx1 = xtr[xo + 1]; }
    if (r == 0) { ty0 = gy; ty1 = 0; } else { ty0 = ytr[yo]; ty1 = ytr[yo + 1]; }
    real x[4];
    x[0] = q0 + a * tx0 + b * ty0;
    x[1] = q1 - r3 * a * tx0 + b * ty1;
    x[2] = q2 + a * tx1 - r3 * b * ty0;
    x[3] = q3 - r3 * (a * tx1 + b * ty1);
    real A[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) A[e] = Sm[e];
    // a K on the x-mode pair of each y-mode, b K on the y-mode pair of each x-mode
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      A[(2 * q) * 4 + 2 * q] += a;
      A[(2 * q) * 4 + 2 * q + 1] += r3 * a;
      A[(2 * q + 1) * 4 + 2 * q] -= r3 * a;
      A[(2 * q + 1) * 4 + 2 * q + 1] += (real)3 * a;
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      A[p * 4 + p] += b;
      A[p * 4 + p + 2] += r3 * b;
      A[(p + 2) * 4 + p] -= r3 * b;
      A[(p + 2) * 4 + p + 2] += (real)3 * b;
    }
    solve4_nopivot<real>(A, x);
    xtr[xo] = fmadd(r3, x[1], x[0]);
    xtr[xo + 1] = fmadd(r3, x[3], x[2]);
    ytr[yo] = fmadd(r3, x[2], x[0]);
    ytr[yo + 1] = fmadd(r3, x[3], x[1]);
#pragma unroll
    for (int d = 0; d < 4; ++d) c[d] = fmadd(L.wt[o], x[d], c[d]);
    if (L.psi[o]) {
      double* out = L.psi[o] + 4 * cell;
      out[0] = (double)x[0];
      out[1] = (double)(mx * x[1]);
      out[2] = (double)(my * x[2]);
      out[3] = (double)(mx * my * x[3]);
    }
  }
}

// The diagonal-slot sweep with cross sections that vary inside the cells:
// per cell the lanes form the sigma_t block and (for the operator) the
// source sigma_s z from the shape blocks and the instance's coefficients.
template <typename real, int G, int OPL>
__global__ void __launch_bounds__(512) sweep2d_field_kernel(
    const InstDev* __restrict__ insts, const SweepItem* __restrict__ items,
    const double* __restrict__ ox, const double* __restrict__ oy, const double* __restrict__ w,
    const int32_t* __restrict__ perm, const double* __restrict__ fblk, int nf, int64_t fcell,
    const double* __restrict__ sigma_t, const double* __restrict__ sigma_s, int max_regions,
    const double* __restrict__ qx, const double* __restrict__ qadd,
    const double* __restrict__ inflow, real* __restrict__ part, double* __restrict__ psi_out,
    const int32_t* __restrict__ active, int n_items, int per_xcd) {
  const int item = work_item(per_xcd);
  if (item >= n_items) return;
  const SweepItem it = items[item];
  if (active && !active[it.inst]) return;
  const InstDev I = insts[it.inst];
  const int tid = threadIdx.x;
  const int g = tid % G;
  const int slot = tid / G;
  const int S = blockDim.x / G;
  const int nx = I.nx, ny = I.ny;
  const LaneOrds<real, OPL> L = lane_ords<real, G, OPL>(it, I, g, ox, oy, w, perm, psi_out);
  const bool fx = it.quadrant & 1, fy = it.quadrant & 2;
  const real mx = fx ? (real)-1 : (real)1, my = fy ? (real)-1 : (real)1;
  const double gsc = sqrt(I.hx * I.hy);
  const real gx = inflow ? (real)(inflow[4 * it.inst + (fx ? 1 : 0)] * gsc) : (real)0;
  const real gy = inflow ? (real)(inflow[4 * it.inst + (fy ? 3 : 2)] * gsc) : (real)0;
  extern __shared__ unsigned char smem_raw[];
  real* xtr = reinterpret_cast<real*>(smem_raw);  // [ny][OPL][G][2]
  real* ytr = xtr + (size_t)ny * G * OPL * 2;     // [nx][OPL][G][2]
  const double* tht = sigma_t + (size_t)it.inst * max_regions;
  const double* ths = sigma_s ? sigma_s + (size_t)it.inst * max_regions : nullptr;
  const double* qxi = qx ? qx + I.dof_off : nullptr;
  const double* qai = qadd ? qadd + I.dof_off : nullptr;
  real* P = part + it.part_off;
  const double sgn[4] = {1.0, fx ? -1.0 : 1.0, fy ? -1.0 : 1.0, (fx != fy) ? -1.0 : 1.0};

  for (int s = 0; s < nx + ny - 1; ++s) {
    const int r_lo = max(0, s - nx + 1), r_hi = min(ny - 1, s);
    for (int r = r_lo + slot; r <= r_hi; r += S) {
      const int i = s - r;
      const int ip = fx ? nx - 1 - i : i;
      const int kp = fy ? ny - 1 - r : r;
      const int cell = kp * nx + ip;
      double B[16], q[4] = {0.0, 0.0, 0.0, 0.0};
      if (qxi) {
        field_block(fblk, nf, fcell, cell, ths, B);
        const double4 v = *reinterpret_cast<const double4*>(qxi + 4 * (int64_t)cell);
#pragma unroll
        for (int a = 0; a < 4; ++a) q[a] = B[4 * a] * v.x + B[4 * a + 1] * v.y + B[4 * a + 2] * v.z + B[4 * a + 3] * v.w;
      }
      if (qai) {
        const double4 v = *reinterpret_cast<const double4*>(qai + 4 * (int64_t)cell);
        q[0] += v.x; q[1] += v.y; q[2] += v.z; q[3] += v.w;
      }
      field_block(fblk, nf, fcell, cell, tht, B);
      real Sm[16];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b2 = 0; b2 < 4; ++b2) Sm[4 * a + b2] = (real)(sgn[a] * sgn[b2] * B[4 * a + b2]);
      real c[4];
      cell_update_field<real, G, OPL>(L, g, i, r, cell, Sm, (real)q[0], (real)(sgn[1] * q[1]), (real)(sgn[2] * q[2]),
                                      (real)(sgn[3] * q[3]), gx, gy, mx, my, xtr, ytr, c);
      store_partial<real, G>(c, g, mx, my, P, cell);
    }
    __syncthreads();
  }
}

// LDS-only work-group barrier: this wave's LDS operations complete, then
// s_barrier.  Global loads stay in flight across it (they feed the next
// diagonal); the empty asm statements stop the compiler from moving memory
// accesses across the barrier.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt left open
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

constexpr int SWEEP_SIGMA_TAB = 256;  // regions whose cross sections are staged in LDS
constexpr int SWEEP_COEF_ENTRIES = 512;  // (region, lane ordinate) solve-coefficient entries in LDS
// Largest work group of the row-slot kernel: 1024 threads with one row per
// slot (512 for FP64 with 8 ordinates per lane, whose registers would not fit
// the 128 per lane that 1024 threads leave), else 512.
__host__ __device__ constexpr int rows_max_threads(int rows_per_slot, size_t elem, int opl) {
  return rows_per_slot <= 1 && (elem == 4 || opl <= 4) ? 1024 : 512;
}

// Stages a work item's per-region tables in LDS: the source scalings (s,
// mx s, my s, mx my s), s = sigma_s (SCALED) or 1, at tab[4 * region], and
// per (region, lane ordinate) the local-solve coefficients as coef_planes
// planes of Pair2 at ctab[region][plane][OPL][G] (formed in FP64 from sigma_t
// and the ordinate's a and b).
template <typename real, int G, int OPL, bool SCALED>
__device__ __forceinline__ void stage_region_tables(const SweepItem& it, const InstDev& I,
                                                    const double* __restrict__ ox, const double* __restrict__ oy,
                                                    const double* __restrict__ sigma_t,
                                                    const double* __restrict__ sigma_s, int max_regions, real mx,
                                                    real my, real* tab, typename Pair2<real>::T* ctab) {
  using P2 = typename Pair2<real>::T;
  constexpr int NPL = coef_planes<real>();
  const int nreg = I.n_regions, per_reg = NPL * OPL * G;
  const double* st = sigma_t + (size_t)it.inst * max_regions;
  const double* ss = SCALED ? sigma_s + (size_t)it.inst * max_regions : nullptr;
  for (int e = threadIdx.x; e < nreg; e += blockDim.x) {
    const real sv = SCALED ? (real)ss[e] : (real)1;
    tab[4 * e] = sv;
    tab[4 * e + 1] = mx * sv;
    tab[4 * e + 2] = my * sv;
    tab[4 * e + 3] = mx * my * sv;
  }
  for (int e = threadIdx.x; e < nreg * OPL * G; e += blockDim.x) {
    const int rg = e / (G * OPL), j = e % (G * OPL);  // lane j / OPL, its ordinate j % OPL
    const bool on = j < it.count;
    const int js = I.ord_off + it.first + (on ? j : 0);
    double cf[10];
    solve_coef(st[rg], fabs(ox[js]) / I.hx, fabs(oy[js]) / I.hy, cf);
    P2* d = ctab + rg * per_reg + (j % OPL) * G + j / OPL;
#pragma unroll
    for (int p = 0; p < NPL; ++p) {
      P2 v;
      v.x = (real)cf[2 * p];
      v.y = (real)cf[2 * p + 1];
      d[p * OPL * G] = v;
    }
  }
}

// The same sweep with a fixed row -> slot assignment (row r is handled by slot
// r mod S), so a slot walks along its rows one cell per diagonal and loads the
// source of its next cell while the current diagonal is processed: the global
// load latency leaves the diagonal-to-diagonal dependence chain.  Every slot
// issues the loads of all its rows on every diagonal (addresses clamped to the
// grid), so the prefetched registers are plain loop-carried values; the x
// traces along a row stay in the slot's registers.  MAXR
// bounds the rows per slot (ceil(ny / S) <= MAXR).  Per region the work group
// stages sigma_s and, for each of its ordinates, the local-solve coefficients
// (formed once from sigma_t, a and b, instead of once per cell) in LDS
// (n_regions <= SWEEP_SIGMA_TAB, n_regions * G * OPL <= SWEEP_COEF_ENTRIES).
// SCALED: the source is sigma_s * q, else q as is (qsrc must be given).
template <typename real, int G, int OPL, int MAXR, bool SCALED, bool PSI>
__global__ void __launch_bounds__(rows_max_threads(MAXR, sizeof(real), OPL)) sweep2d_rows_kernel(
    const InstDev* __restrict__ insts, const SweepItem* __restrict__ items,
    const double* __restrict__ ox, const double* __restrict__ oy, const double* __restrict__ w,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ region,
    const double* __restrict__ sigma_t, const double* __restrict__ sigma_s, int max_regions,
    const double* __restrict__ qsrc, const double* __restrict__ inflow,
    real* __restrict__ part, double* __restrict__ psi_out, const int32_t* __restrict__ active, int n_items,
    int per_xcd) {
  const int item = work_item(per_xcd);
  if (item >= n_items) return;
  const SweepItem it = items[item];
  if (active && !active[it.inst]) return;
  const InstDev I = insts[it.inst];
  const int tid = threadIdx.x;
  const int g = tid % G;
  const int slot = tid / G;
  const int S = blockDim.x / G;
  const int nx = I.nx, ny = I.ny;
  const LaneOrds<real, OPL> L = lane_ords<real, G, OPL>(it, I, g, ox, oy, w, perm, psi_out);
  const bool fx = it.quadrant & 1, fy = it.quadrant & 2;
  const real mx = fx ? (real)-1 : (real)1, my = fy ? (real)-1 : (real)1;
  const double gsc = sqrt(I.hx * I.hy);
  const real gx = inflow ? (real)(inflow[4 * it.inst + (fx ? 1 : 0)] * gsc) : (real)0;
  const real gy = inflow ? (real)(inflow[4 * it.inst + (fy ? 3 : 2)] * gsc) : (real)0;
  extern __shared__ unsigned char smem_raw[];
  constexpr int YS = ytr_stride<real, G, OPL>();
  real* ytr = reinterpret_cast<real*>(smem_raw);  // [nx][YS]: [OPL][G][2] and padding
  // per region the source scaling with the quadrant's mirror signs folded in:
  // (s, mx s, my s, mx my s), s = sigma_s (SCALED) or 1
  const int nreg = I.n_regions;
  real* tab = ytr + (size_t)nx * YS;               // [n_regions][4]
  using P2 = typename Pair2<real>::T;
  P2* ctab = reinterpret_cast<P2*>(tab + 4 * nreg);  // [n_regions][coef_planes][OPL][G]
  const int per_reg = coef_planes<real>() * OPL * G;
  {
    stage_region_tables<real, G, OPL, SCALED>(it, I, ox, oy, sigma_t, sigma_s, max_regions, mx, my, tab, ctab);
    // inflow traces (g, 0) where each column enters the grid
    for (int e = tid; e < nx * G * OPL; e += blockDim.x) {
      real* t = ytr + (e / (G * OPL)) * YS + 2 * (e % (G * OPL));
      t[0] = gy;
      t[1] = (real)0;
    }
  }
  __syncthreads();
  const int32_t* reg = region + I.region_off;
  const double* qi = qsrc + I.dof_off;
  real* P = part + it.part_off;
  // a row's cells in sweep order are consecutive physical cells, dx apart
  const int dx = fx ? -1 : 1;

  double4 qn[MAXR];
  int rn[MAXR];
  uint32_t cn[MAXR];      // physical index of each row's next cell
  real xt[MAXR][OPL][2];  // x traces of the slot's rows, the inflow trace first
#pragma unroll
  for (int kk = 0; kk < MAXR; ++kk)
#pragma unroll
    for (int o = 0; o < OPL; ++o) {
      xt[kk][o][0] = gx;
      xt[kk][o][1] = (real)0;
    }
#pragma unroll
  for (int kk = 0; kk < MAXR; ++kk) {  // each row's first cell (rows past the grid: the last row's)
    const int r = min(slot + kk * S, ny - 1);
    cn[kk] = (uint32_t)((fy ? ny - 1 - r : r) * nx + (fx ? nx - 1 : 0));
    rn[kk] = reg[cn[kk]];
    qn[kk] = *reinterpret_cast<const double4*>(qi + 4u * cn[kk]);
  }

  for (int s = 0; s < nx + ny - 1; ++s) {
#pragma unroll
    for (int kk = 0; kk < MAXR; ++kk) {
      const int r = slot + kk * S;
      const int i = s - r;
      if (r < ny && i >= 0 && i < nx) {
        const double4 v = qn[kk];
        const int rg = rn[kk];
        const uint32_t cell = cn[kk];
        const real* sc = tab + 4 * rg;
        real c[4];
        cell_update_rows<real, G, OPL, PSI>(L, g, i, cell, sc[0] * (real)v.x, sc[1] * (real)v.y, sc[2] * (real)v.z,
                                       sc[3] * (real)v.w, mx, my, xt[kk], ytr, c, ctab + rg * per_reg + g);
        store_partial<real, G>(c, g, mx, my, P, cell);
        // source of the row's next cell (issued after the last use of the
        // current one, so it can land in the same registers); none after the
        // row's last cell, so whole waves skip it
        if (i + 1 < nx) {
          cn[kk] = cell + dx;
          rn[kk] = reg[cell + dx];
          qn[kk] = *reinterpret_cast<const double4*>(qi + 4u * (cell + dx));
        }
      }
    }
    lds_barrier();
  }
}

// A wave-wide shift by one lane (lane l receives lane l - 1's value; lane 0
// receives `first`): DPP wave_shr:1, whose lane 0 has no source and keeps the
// old value when bound_ctrl is off.
__device__ __forceinline__ float wave_shift_up(float v, float first) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(first), __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ double wave_shift_up(double v, double first) {
  const long long a = __double_as_longlong(v), f = __double_as_longlong(first);
  const int lo = __builtin_amdgcn_update_dpp((int)(f & 0xffffffffll), (int)(a & 0xffffffffll), 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(f >> 32), (int)(a >> 32), 0x138, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Lane 63's value, in every lane.
__device__ __forceinline__ float lane63(float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63)); }
__device__ __forceinline__ double lane63(double v) {
  const long long a = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(a & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(a >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

constexpr int SWEEP_WAVE_MAXR = 4;  // rows per lane of the wave-per-item kernel (ny <= 256)

// Wave-per-item sweep for batches too small to fill the chip with work
// groups of many slots (one instance: the single-instance sweep).  A work
// item is one wave of 64 lanes; lane l owns rows l, l + 64, ... (up to MAXR),
// one cell per diagonal and OPL ordinates per lane (G = 1).  The x trace of a
// row stays in its lane's registers; the y trace that row r leaves on a
// diagonal is the inflow of row r + 1 on the next one, handed over by a
// wave-wide lane shift (lane 63 passes to lane 0 of the next row group), so
// the wavefront needs no barrier and no LDS round trip.  LDS holds only the
// per-region tables.  Each lane writes its own cell's weighted sum over the
// item's OPL ordinates.
template <typename real, int OPL, int MAXR, bool SCALED, bool PSI>
__global__ void __launch_bounds__(64) sweep2d_wave_kernel(
    const InstDev* __restrict__ insts, const SweepItem* __restrict__ items,
    const double* __restrict__ ox, const double* __restrict__ oy, const double* __restrict__ w,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ region,
    const double* __restrict__ sigma_t, const double* __restrict__ sigma_s, int max_regions,
    const double* __restrict__ qsrc, const double* __restrict__ inflow,
    real* __restrict__ part, double* __restrict__ psi_out, const int32_t* __restrict__ active, int n_items,
    int per_xcd) {
  const int item = work_item(per_xcd);
  if (item >= n_items) return;
  const SweepItem it = items[item];
  if (active && !active[it.inst]) return;
  const InstDev I = insts[it.inst];
  const int lane = threadIdx.x;
  const int nx = I.nx, ny = I.ny;
  const LaneOrds<real, OPL> L = lane_ords<real, 1, OPL>(it, I, 0, ox, oy, w, perm, psi_out);
  const bool fx = it.quadrant & 1, fy = it.quadrant & 2;
  const real mx = fx ? (real)-1 : (real)1, my = fy ? (real)-1 : (real)1;
  const double gsc = sqrt(I.hx * I.hy);
  const real gx = inflow ? (real)(inflow[4 * it.inst + (fx ? 1 : 0)] * gsc) : (real)0;
  const real gy = inflow ? (real)(inflow[4 * it.inst + (fy ? 3 : 2)] * gsc) : (real)0;
  extern __shared__ unsigned char smem_raw[];
  real* tab = reinterpret_cast<real*>(smem_raw);  // [n_regions][4]
  using P2 = typename Pair2<real>::T;
  P2* ctab = reinterpret_cast<P2*>(tab + 4 * I.n_regions);  // [n_regions][coef_planes][OPL]
  const int per_reg = coef_planes<real>() * OPL;
  stage_region_tables<real, 1, OPL, SCALED>(it, I, ox, oy, sigma_t, sigma_s, max_regions, mx, my, tab, ctab);
  __syncthreads();
  const int32_t* reg = region + I.region_off;
  const double* qi = qsrc + I.dof_off;
  real* P = part + it.part_off;
  const int dx = fx ? -1 : 1;

  // Sources and regions two cells ahead: a wave runs alone on its SIMD, so
  // one diagonal is too short to hide a load.  Buffer A serves the steps of
  // even parity, B the odd ones, so no register moves wait on a load: a row
  // whose first step is even holds cells 0, 2, ... in A and 1, 3, ... in B
  // (the other way round for an odd first step), and after using a cell the
  // row loads the cell two ahead into the same buffer.
  double4 qa[MAXR], qb[MAXR];
  int ra[MAXR], rb[MAXR];
  uint32_t cn[MAXR];      // physical index of each row's next cell
  real xt[MAXR][OPL][2];  // x traces of the lane's rows, the inflow trace first
  real yo[MAXR][OPL][2];  // y traces the lane's rows left on the previous diagonal
#pragma unroll
  for (int kk = 0; kk < MAXR; ++kk) {
#pragma unroll
    for (int o = 0; o < OPL; ++o) {
      xt[kk][o][0] = gx;
      xt[kk][o][1] = (real)0;
      yo[kk][o][0] = yo[kk][o][1] = (real)0;
    }
    const int r = min(lane + 64 * kk, ny - 1);
    cn[kk] = (uint32_t)((fy ? ny - 1 - r : r) * nx + (fx ? nx - 1 : 0));
    const uint32_t c1 = nx > 1 ? cn[kk] + dx : cn[kk];
    const double4 q0 = *reinterpret_cast<const double4*>(qi + 4u * cn[kk]);
    const double4 q1 = *reinterpret_cast<const double4*>(qi + 4u * c1);
    const int r0 = reg[cn[kk]], r1 = reg[c1];
    const bool even = ((lane + 64 * kk) & 1) == 0;
    qa[kk] = even ? q0 : q1;
    qb[kk] = even ? q1 : q0;
    ra[kk] = even ? r0 : r1;
    rb[kk] = even ? r1 : r0;
  }

  // one diagonal, the buffers of its parity
  auto diagonal = [&](int s, double4 (&qn)[MAXR], int (&rn)[MAXR]) {
    // inflow y traces of this diagonal: the row below's outflow of the last one
    real yi[MAXR][OPL][2];
#pragma unroll
    for (int kk = 0; kk < MAXR; ++kk)
#pragma unroll
      for (int o = 0; o < OPL; ++o)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const real first = kk == 0 ? (t == 0 ? gy : (real)0) : lane63(yo[kk - 1][o][t]);
          yi[kk][o][t] = wave_shift_up(yo[kk][o][t], first);
        }
#pragma unroll
    for (int kk = 0; kk < MAXR; ++kk) {
      const int r = lane + 64 * kk;
      const int i = s - r;
      if (r < ny && i >= 0 && i < nx) {
        const double4 v = qn[kk];
        const int rg = rn[kk];
        const uint32_t cell = cn[kk];
        const real* sc = tab + 4 * rg;
        real c[4];
        cell_update_wave<real, OPL, PSI>(L, cell, sc[0] * (real)v.x, sc[1] * (real)v.y, sc[2] * (real)v.z,
                                         sc[3] * (real)v.w, mx, my, xt[kk], yi[kk], yo[kk], c,
                                         ctab + rg * per_reg);
        real* o = P + 4u * cell;
        o[0] = c[0];
        o[1] = mx * c[1];
        o[2] = my * c[2];
        o[3] = mx * my * c[3];
        cn[kk] = cell + dx;
        if (i + 2 < nx) {
          rn[kk] = reg[cell + 2 * dx];
          qn[kk] = *reinterpret_cast<const double4*>(qi + 4u * (cell + 2 * dx));
        }
      }
    }
  };
  const int nd = nx + ny - 1;
  for (int s = 0; s < nd; s += 2) {
    diagonal(s, qa, ra);
    if (s + 1 < nd) diagonal(s + 1, qb, rb);
  }
}

// Slab geometry, P1: one thread per (instance, ordinate), cells in upwind order.
template <typename real>
__global__ void sweep1d_kernel(const InstDev* __restrict__ insts, const InstPart* __restrict__ parts,
                               const double* __restrict__ ox, const double* __restrict__ w,
                               const int32_t* __restrict__ perm, const int32_t* __restrict__ region,
                               const double* __restrict__ sigma_t,
                               const double* __restrict__ sigma_s, int max_regions,
                               const double* __restrict__ qx, const double* __restrict__ qadd,
                               const double* __restrict__ inflow, real* __restrict__ part,
                               double* __restrict__ psi_out, const int32_t* __restrict__ active) {
  const int inst = blockIdx.x;
  if (active && !active[inst]) return;
  const InstDev I = insts[inst];
  const int js_loc = threadIdx.x;
  if (js_loc >= I.n_ord) return;
  const int js = I.ord_off + js_loc;
  const real r3 = (real)1.7320508075688772935;
  const double mu = ox[js];
  const bool flip = mu < 0.0;
  const real m1 = flip ? (real)-1 : (real)1;
  const real a = (real)(fabs(mu) / I.hx);
  const real wt = (real)w[js];
  const int nx = I.nx;
  const double* st = sigma_t + (size_t)inst * max_regions;
  const double* ss = sigma_s ? sigma_s + (size_t)inst * max_regions : nullptr;
  const int32_t* reg = region + I.region_off;
  real* P = part + parts[inst].off + (int64_t)js_loc * nx * 2;
  double* psi_j = psi_out ? psi_out + I.psi_off + (int64_t)perm[js] * nx * 2 : nullptr;
  real T = inflow ? (real)(inflow[4 * inst + (flip ? 1 : 0)] * sqrt(I.hx)) : (real)0;  // left / right
  for (int i = 0; i < nx; ++i) {
    const int cell = flip ? nx - 1 - i : i;
    const int rg = reg[cell];
    double q0 = 0.0, q1 = 0.0;
    if (qx) {
      q0 = ss[rg] * qx[I.dof_off + 2 * cell];
      q1 = ss[rg] * qx[I.dof_off + 2 * cell + 1];
    }
    if (qadd) {
      q0 += qadd[I.dof_off + 2 * cell];
      q1 += qadd[I.dof_off + 2 * cell + 1];
    }
    const real sig = (real)st[rg];
    const real r0 = (real)q0 + a * T;
    const real r1 = m1 * (real)q1 - r3 * a * T;
    // (sig I + a K) x = r: adj = (sig + 4a) I - a K, det = sig^2 + 4 sig a + 6 a^2
    const real det = sig * sig + (real)4 * sig * a + (real)6 * a * a;
    const real inv = (real)1 / det;
    const real k0 = r0 + r3 * r1, k1 = -r3 * r0 + (real)3 * r1;
    const real x0 = ((sig + (real)4 * a) * r0 - a * k0) * inv;
    const real x1 = ((sig + (real)4 * a) * r1 - a * k1) * inv;
    T = x0 + r3 * x1;
    P[2 * cell] = wt * x0;
    P[2 * cell + 1] = wt * m1 * x1;
    if (psi_j) {
      psi_j[2 * cell] = (double)x0;
      psi_j[2 * cell + 1] = (double)(m1 * x1);
    }
  }
}

// sum_k p[k * nd] in order k = 0, 1, ... (the loads four at a time, so that
// several are in flight; the additions keep their order)
template <typename real>
__device__ __forceinline__ double sum_partials(const real* __restrict__ p, int n, int64_t nd) {
  double t = 0.0;
  int k = 0;
  for (; k + 4 <= n; k += 4) {
    const real a0 = p[(int64_t)k * nd], a1 = p[(int64_t)(k + 1) * nd];
    const real a2 = p[(int64_t)(k + 2) * nd], a3 = p[(int64_t)(k + 3) * nd];
    t += (double)a0;
    t += (double)a1;
    t += (double)a2;
    t += (double)a3;
  }
  for (; k < n; ++k) t += (double)p[(int64_t)k * nd];
  return t;
}

template <typename real>
__global__ void reduce_partials_kernel(const InstDev* __restrict__ insts,
                                       const InstPart* __restrict__ parts,
                                       const real* __restrict__ part, double alpha,
                                       const double* __restrict__ x, double beta,
                                       const double* __restrict__ y, double gamma,
                                       double* __restrict__ out, const int32_t* __restrict__ active) {
  const int inst = blockIdx.y;
  if (active && !active[inst]) return;
  const InstDev I = insts[inst];
  const int64_t nd = (int64_t)I.nx * I.ny * I.nloc;
  const InstPart pp = parts[inst];
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, step = (int64_t)gridDim.x * blockDim.x;
  if (((pp.off | I.dof_off | nd) & 1) == 0) {
    // pairs of DoFs per access; each DoF's partials summed in the same order
    using P2 = typename Pair2<real>::T;
    const int64_t st2 = nd / 2;
    for (int64_t q2 = t0; 2 * q2 < nd; q2 += step) {
      const int64_t d = 2 * q2;
      const P2* q = reinterpret_cast<const P2*>(part + pp.off + d);
      double a0s = 0.0, a1s = 0.0;
      int k = 0;
      for (; k + 4 <= pp.n; k += 4) {
        const P2 u0 = q[(int64_t)k * st2], u1 = q[(int64_t)(k + 1) * st2];
        const P2 u2 = q[(int64_t)(k + 2) * st2], u3 = q[(int64_t)(k + 3) * st2];
        a0s += (double)u0.x; a1s += (double)u0.y;
        a0s += (double)u1.x; a1s += (double)u1.y;
        a0s += (double)u2.x; a1s += (double)u2.y;
        a0s += (double)u3.x; a1s += (double)u3.y;
      }
      for (; k < pp.n; ++k) {
        const P2 u = q[(int64_t)k * st2];
        a0s += (double)u.x;
        a1s += (double)u.y;
      }
      double2 v;
      v.x = alpha * a0s;
      v.y = alpha * a1s;
      if (x) {
        const double2 xv = *reinterpret_cast<const double2*>(x + I.dof_off + d);
        v.x += beta * xv.x;
        v.y += beta * xv.y;
      }
      if (y) {
        const double2 yv = *reinterpret_cast<const double2*>(y + I.dof_off + d);
        v.x += gamma * yv.x;
        v.y += gamma * yv.y;
      }
      *reinterpret_cast<double2*>(out + I.dof_off + d) = v;
    }
  } else {
    for (int64_t d = t0; d < nd; d += step) {
      const double acc = sum_partials(part + pp.off + d, pp.n, nd);
      double v = alpha * acc;
      if (x) v += beta * x[I.dof_off + d];
      if (y) v += gamma * y[I.dof_off + d];
      out[I.dof_off + d] = v;
    }
  }
}

// reduce_partials_kernel fused with the partial dot products <out, dotv>
// (<out, out> when dotv is null): one work group per chunk of `chunk` DoFs,
// threads strided over it, then a wave-shuffle and cross-wave sum (256
// threads).
template <typename real>
__global__ void __launch_bounds__(256) reduce_partials_dot_kernel(
    const InstDev* __restrict__ insts, const InstPart* __restrict__ parts, const real* __restrict__ part,
    double alpha, const double* __restrict__ x, double beta, double* __restrict__ out,
    const double* __restrict__ dotv, double* __restrict__ dpart, int maxc, int chunk,
    const int32_t* __restrict__ active) {
  __shared__ double sh[4];
  const int inst = blockIdx.y, c = blockIdx.x;
  if (active && !active[inst]) return;
  const InstDev I = insts[inst];
  const int64_t nd = (int64_t)I.nx * I.ny * I.nloc, start = (int64_t)c * chunk;
  if (start >= nd) return;
  const int64_t end = min(nd, start + (int64_t)chunk);
  const InstPart pp = parts[inst];
  double acc = 0.0;
  if (((pp.off | I.dof_off | start | end) & 1) == 0) {
    // pairs of DoFs per access (whole cells keep every offset even); each
    // DoF's partials are summed in the same order as below
    using P2 = typename Pair2<real>::T;
    for (int64_t d = start + 2 * threadIdx.x; d < end; d += 2 * blockDim.x) {
      const P2* q = reinterpret_cast<const P2*>(part + pp.off + d);
      const int64_t st2 = nd / 2;
      double t0 = 0.0, t1 = 0.0;
      int k = 0;
      for (; k + 4 <= pp.n; k += 4) {
        const P2 a0 = q[(int64_t)k * st2], a1 = q[(int64_t)(k + 1) * st2];
        const P2 a2 = q[(int64_t)(k + 2) * st2], a3 = q[(int64_t)(k + 3) * st2];
        t0 += (double)a0.x; t1 += (double)a0.y;
        t0 += (double)a1.x; t1 += (double)a1.y;
        t0 += (double)a2.x; t1 += (double)a2.y;
        t0 += (double)a3.x; t1 += (double)a3.y;
      }
      for (; k < pp.n; ++k) {
        const P2 a = q[(int64_t)k * st2];
        t0 += (double)a.x;
        t1 += (double)a.y;
      }
      double2 v;
      v.x = alpha * t0;
      v.y = alpha * t1;
      if (x) {
        const double2 xv = *reinterpret_cast<const double2*>(x + I.dof_off + d);
        v.x += beta * xv.x;
        v.y += beta * xv.y;
      }
      *reinterpret_cast<double2*>(out + I.dof_off + d) = v;
      const double2 dv = dotv ? *reinterpret_cast<const double2*>(dotv + I.dof_off + d) : v;
      acc += v.x * dv.x + v.y * dv.y;
    }
  } else {
    for (int64_t d = start + threadIdx.x; d < end; d += blockDim.x) {
      const double t = sum_partials(part + pp.off + d, pp.n, nd);
      double v = alpha * t;
      if (x) v += beta * x[I.dof_off + d];
      out[I.dof_off + d] = v;
      acc += v * (dotv ? dotv[I.dof_off + d] : v);
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tsum = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) tsum += sh[k];
    dpart[(int64_t)inst * maxc + c] = tsum;
  }
}

__global__ void scalar_flux_kernel(const InstDev* __restrict__ insts, const double* __restrict__ w,
                                   const int32_t* __restrict__ perm,
                                   const double* __restrict__ psi, double* __restrict__ phi) {
  const int inst = blockIdx.y;
  const InstDev I = insts[inst];
  const int64_t nd = (int64_t)I.nx * I.ny * I.nloc;
  extern __shared__ double wl[];  // weights in original ordinate order
  for (int s = threadIdx.x; s < I.n_ord; s += blockDim.x) wl[perm[I.ord_off + s]] = w[I.ord_off + s];
  __syncthreads();
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < nd;
       d += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    const double* p = psi + I.psi_off + d;
    for (int j = 0; j < I.n_ord; ++j) acc += wl[j] * p[(int64_t)j * nd];
    phi[I.dof_off + d] = acc;
  }
}

int ensure_partials(rte_batch* b, int64_t elems) {
  if (elems <= b->part_capacity) return RTE_OK;
  (void)hipFree(b->d_part);
  b->d_part = nullptr;
  b->part_capacity = 0;
  ++b->gen;
  if (hipMalloc(&b->d_part, sizeof(double) * elems) != hipSuccess) return RTE_ENOMEM;
  b->part_capacity = elems;
  return RTE_OK;
}

int make_plan(rte_batch* b, int prec, int G, int threads, int opl) {
  Plan& p = b->plan[prec];
  p.G = G;
  p.opl = opl;
  p.threads = threads;
  const int per_item = G * opl;  // ordinates per work item
  p.items.clear();
  p.parts.clear();
  int64_t off = 0;
  for (int k = 0; k < b->n_inst; ++k) {
    const InstDev& I = b->inst[k];
    const int64_t nd = (int64_t)I.nx * I.ny * I.nloc;
    InstPart ip{};
    ip.off = off;
    if (I.dim == 1) {
      ip.n = I.n_ord;
    } else {
      int n = 0;
      for (int qd = 0; qd < 4; ++qd) {
        for (int f = 0; f < I.quad_count[qd]; f += per_item) {
          SweepItem it{};
          it.inst = k;
          it.quadrant = qd;
          it.first = I.quad_first[qd] + f;
          it.count = std::min(per_item, I.quad_count[qd] - f);
          it.part_off = off + (int64_t)n * nd;
          p.items.push_back(it);
          ++n;
        }
      }
      ip.n = n;
    }
    off += (int64_t)ip.n * nd;
    p.parts.push_back(ip);
  }
  p.part_elems = off;
  p.n_items = (int)p.items.size();
  if (p.order == 1)  // the largest items first (their partial-flux offsets stay as they are)
    std::stable_sort(p.items.begin(), p.items.end(), [&](const SweepItem& x, const SweepItem& y) {
      const InstDev& X = b->inst[x.inst];
      const InstDev& Y = b->inst[y.inst];
      return (int64_t)X.nx * X.ny * x.count > (int64_t)Y.nx * Y.ny * y.count;
    });
  ++b->gen;
  (void)hipFree(p.d_items);
  (void)hipFree(p.d_parts);
  p.d_items = nullptr;
  p.d_parts = nullptr;
  if (p.n_items > 0) {
    if (hipMalloc(&p.d_items, sizeof(SweepItem) * p.n_items) != hipSuccess) return RTE_ENOMEM;
    RTE_HIP(hipMemcpy(p.d_items, p.items.data(), sizeof(SweepItem) * p.n_items,
                      hipMemcpyHostToDevice));
  }
  if (hipMalloc(&p.d_parts, sizeof(InstPart) * b->n_inst) != hipSuccess) return RTE_ENOMEM;
  RTE_HIP(hipMemcpy(p.d_parts, p.parts.data(), sizeof(InstPart) * b->n_inst,
                    hipMemcpyHostToDevice));
  return ensure_partials(b, off);
}

// Whether the row-slot kernel can take this batch with G lanes per cell, OPL
// ordinates per lane and T threads (rows per slot, and the per-region tables).
static bool rows_variant_fits(const rte_batch* b, int G, int opl, int T, size_t es) {
  const int slots = T / G;
  if (slots <= 0) return false;
  const int nr = (b->max_ny + slots - 1) / slots;
  return b->n_fields == 0 && nr <= 8 && T <= rows_max_threads(nr, es, opl) && b->max_regions <= SWEEP_SIGMA_TAB &&
         b->max_regions * G * opl <= SWEEP_COEF_ENTRIES;
}

// Whether the wave-per-item kernel (variant 2: G = 1, 64 threads) can take
// this batch with OPL ordinates per lane.
static bool wave_variant_fits(const rte_batch* b, int opl) {
  return b->n_fields == 0 && (opl == 1 || opl == 2 || opl == 4) && b->max_ny <= 64 * SWEEP_WAVE_MAXR &&
         b->max_regions <= SWEEP_SIGMA_TAB && b->max_regions * opl <= SWEEP_COEF_ENTRIES;
}

static size_t wave_lds(const rte_batch* b, int opl, size_t es) {
  const size_t planes = es == 4 ? coef_planes<float>() : coef_planes<double>();
  return (4 * (size_t)b->max_regions + 2 * planes * b->max_regions * opl) * es;
}

template <typename real, int OPL>
static int launch_wave(rte_batch* b, const Plan& p, const double* sigma_t, const double* sigma_s, const double* qx,
                       const double* qadd, const double* inflow, double* psi_out, hipStream_t s,
                       const int32_t* active, void* part) {
  if ((qx != nullptr) == (qadd != nullptr)) return RTE_EINVAL;  // one source form
  const int per_xcd = p.order == 0 ? (p.n_items + 7) / 8 : 0;
  const unsigned nwg = per_xcd > 0 ? 8u * per_xcd : (unsigned)p.n_items;
  const int nr = (b->max_ny + 63) / 64;
  const size_t lds = wave_lds(b, OPL, sizeof(real));
  const double* src = qx ? qx : qadd;
#define RTE_WAVE_LAUNCH1(R, SC, PS)                                                                           \
  hipLaunchKernelGGL((sweep2d_wave_kernel<real, OPL, R, SC, PS>), dim3(nwg), dim3(64), lds, s, b->d_inst, \
                     p.d_items, b->d_ox, b->d_oy, b->d_w, b->d_perm, b->d_region, sigma_t, sigma_s,             \
                     b->max_regions, src, inflow, reinterpret_cast<real*>(part), psi_out, active, p.n_items,   \
                     per_xcd)
#define RTE_WAVE_LAUNCH(R, SC)                      \
  do {                                              \
    if (psi_out) RTE_WAVE_LAUNCH1(R, SC, true);     \
    else RTE_WAVE_LAUNCH1(R, SC, false);            \
  } while (0)
  if (qx) {
    if (nr <= 1) RTE_WAVE_LAUNCH(1, true);
    else if (nr <= 2) RTE_WAVE_LAUNCH(2, true);
    else RTE_WAVE_LAUNCH(4, true);
  } else {
    if (nr <= 1) RTE_WAVE_LAUNCH(1, false);
    else if (nr <= 2) RTE_WAVE_LAUNCH(2, false);
    else RTE_WAVE_LAUNCH(4, false);
  }
#undef RTE_WAVE_LAUNCH
#undef RTE_WAVE_LAUNCH1
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

// LDS bytes of a 2D sweep work group (traces of G * OPL ordinates: x and y, or
// y only for the row-slot kernel, which also stages the sigma_s table and the
// solve coefficients).
static size_t sweep_lds(const rte_batch* b, int G, int opl, int variant, size_t es) {
  size_t n = (size_t)(b->max_nx + b->max_ny) * G * opl * 2;
  if (variant == 1) {
    const int ys = es == 4 ? 2 * G * opl + ((2 * G - 2 * G * opl) % 64 + 64) % 64 : 2 * G * opl;
    const size_t planes = es == 4 ? coef_planes<float>() : coef_planes<double>();
    n = (size_t)b->max_nx * ys + 4 * (size_t)b->max_regions + 2 * planes * b->max_regions * G * opl;
  }
  return n * es;
}

template <typename real, int G, int OPL>
static int launch2d(rte_batch* b, const Plan& p, const double* sigma_t, const double* sigma_s,
                    const double* qx, const double* qadd, const double* inflow, double* psi_out,
                    hipStream_t s, const int32_t* active, void* part) {
  const int per_xcd = p.order == 0 ? (p.n_items + 7) / 8 : 0;
  const unsigned nwg = per_xcd > 0 ? 8u * per_xcd : (unsigned)p.n_items;
  const int tdiag = std::min(p.threads, 512);  // the diagonal-slot kernels take at most 512 threads
  if (b->n_fields > 0) {  // cross sections varying inside the cells: the diagonal-slot field kernel
    const size_t lds = sweep_lds(b, G, OPL, 0, sizeof(real));
    if (lds > 64 * 1024) return RTE_EINVAL;
    hipLaunchKernelGGL((sweep2d_field_kernel<real, G, OPL>), dim3(nwg), dim3(tdiag), lds, s, b->d_inst,
                       p.d_items, b->d_ox, b->d_oy, b->d_w, b->d_perm, b->d_fblk, b->n_fields, b->field_ncell,
                       sigma_t, sigma_s, b->max_regions, qx, qadd, inflow, reinterpret_cast<real*>(part), psi_out,
                       active, p.n_items, per_xcd);
    RTE_HIP(hipGetLastError());
    return RTE_OK;
  }
  if (p.variant == 1 && (qx != nullptr) != (qadd != nullptr) && rows_variant_fits(b, G, OPL, p.threads, sizeof(real))) {
    const int slots = p.threads / G;
    const int nr = (b->max_ny + slots - 1) / slots;
    const size_t lds = sweep_lds(b, G, OPL, 1, sizeof(real));
    if (lds > 64 * 1024) return RTE_EINVAL;
    const double* src = qx ? qx : qadd;
#define RTE_ROWS_LAUNCH1(R, SC, PS)                                                                          \
  hipLaunchKernelGGL((sweep2d_rows_kernel<real, G, OPL, R, SC, PS>), dim3(nwg), dim3(p.threads), lds, s, \
                     b->d_inst, p.d_items, b->d_ox, b->d_oy, b->d_w, b->d_perm, b->d_region, sigma_t,        \
                     sigma_s, b->max_regions, src, inflow, reinterpret_cast<real*>(part), psi_out,           \
                     active, p.n_items, per_xcd)
#define RTE_ROWS_LAUNCH(R, SC)              \
  do {                                      \
    if (psi_out) RTE_ROWS_LAUNCH1(R, SC, true); \
    else RTE_ROWS_LAUNCH1(R, SC, false);    \
  } while (0)
    if (qx) {
      if (nr <= 1) RTE_ROWS_LAUNCH(1, true);
      else if (nr <= 2) RTE_ROWS_LAUNCH(2, true);
      else if (nr <= 4) RTE_ROWS_LAUNCH(4, true);
      else RTE_ROWS_LAUNCH(8, true);
    } else {
      if (nr <= 1) RTE_ROWS_LAUNCH(1, false);
      else if (nr <= 2) RTE_ROWS_LAUNCH(2, false);
      else if (nr <= 4) RTE_ROWS_LAUNCH(4, false);
      else RTE_ROWS_LAUNCH(8, false);
    }
#undef RTE_ROWS_LAUNCH
#undef RTE_ROWS_LAUNCH1
    RTE_HIP(hipGetLastError());
    return RTE_OK;
  }
  const size_t lds = sweep_lds(b, G, OPL, 0, sizeof(real));
  if (lds > 64 * 1024) return RTE_EINVAL;  // per-work-group LDS limit used by this library
  hipLaunchKernelGGL((sweep2d_kernel<real, G, OPL>), dim3(nwg), dim3(tdiag), lds, s,
                     b->d_inst, p.d_items, b->d_ox, b->d_oy, b->d_w, b->d_perm, b->d_region,
                     sigma_t, sigma_s, b->max_regions, qx, qadd, inflow,
                     reinterpret_cast<real*>(part), psi_out, active, p.n_items, per_xcd);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

// The (G, OPL) pairs that have kernels: G lanes per cell, OPL ordinates per lane.
static bool plan_shape_ok(int G, int opl) {
  const bool g_ok = G == 1 || G == 2 || G == 4 || G == 8 || G == 16 || G == 32;
  return g_ok && (opl == 1 || (opl == 2 && G >= 4 && G <= 16) || (opl == 4 && G >= 4 && G <= 8) ||
                  (opl == 8 && G == 4));
}

template <typename real>
static int launch2d_g(rte_batch* b, const Plan& p, const double* st, const double* ss,
                      const double* qx, const double* qa, const double* inf, double* psi,
                      hipStream_t s, const int32_t* act, void* part) {
  if (p.variant == 2) {
    if (p.G != 1 || p.threads != 64 || !wave_variant_fits(b, p.opl)) return RTE_EINVAL;
    if (p.opl == 1) return launch_wave<real, 1>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
    if (p.opl == 2) return launch_wave<real, 2>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
    return launch_wave<real, 4>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
  }
  if (p.opl == 8) {
    if (p.G == 4) return launch2d<real, 4, 8>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
    return RTE_EINVAL;
  }
  if (p.opl == 4) {
    switch (p.G) {
      case 4: return launch2d<real, 4, 4>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
      case 8: return launch2d<real, 8, 4>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
      default: return RTE_EINVAL;
    }
  }
  if (p.opl == 2) {
    switch (p.G) {
      case 4: return launch2d<real, 4, 2>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
      case 8: return launch2d<real, 8, 2>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
      case 16: return launch2d<real, 16, 2>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
      default: return RTE_EINVAL;
    }
  }
  switch (p.G) {
    case 1: return launch2d<real, 1, 1>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
    case 2: return launch2d<real, 2, 1>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
    case 4: return launch2d<real, 4, 1>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
    case 8: return launch2d<real, 8, 1>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
    case 16: return launch2d<real, 16, 1>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
    case 32: return launch2d<real, 32, 1>(b, p, st, ss, qx, qa, inf, psi, s, act, part);
    default: return RTE_EINVAL;
  }
}

static int sweep_launch_impl(rte_batch* b, int prec, const double* sigma_t, const double* sigma_s,
                             const double* qx, const double* qadd, const double* inflow,
                             double* psi_out, hipStream_t s, const int32_t* active, void* part);

int sweep_launch(rte_batch* b, int prec, const double* sigma_t, const double* sigma_s,
                 const double* qx, const double* qadd, const double* inflow, double* psi_out,
                 hipStream_t s, const int32_t* active, double prof_units, void* part_buf) {
  void* part = part_buf ? part_buf : b->d_part;
  if (!prof_enabled() || prof_units < -1.5)
    return sweep_launch_impl(b, prec, sigma_t, sigma_s, qx, qadd, inflow, psi_out, s, active, part);
  const int slot = prec == 0 ? PROF_SWEEP_F64 : PROF_SWEEP_F32;
  prof_begin(slot, s);
  const int st = sweep_launch_impl(b, prec, sigma_t, sigma_s, qx, qadd, inflow, psi_out, s, active, part);
  prof_end(slot, s, prof_units >= 0.0 ? prof_units : batch_cell_ordinates(b, nullptr));
  return st;
}

double batch_cell_ordinates(const rte_batch* b, const int32_t* mask) {
  double u = 0.0;
  for (int k = 0; k < b->n_inst; ++k)
    if (!mask || mask[k]) u += (double)b->inst[k].nx * b->inst[k].ny * b->inst[k].n_ord;
  return u;
}

static int sweep_launch_impl(rte_batch* b, int prec, const double* sigma_t, const double* sigma_s,
                             const double* qx, const double* qadd, const double* inflow,
                             double* psi_out, hipStream_t s, const int32_t* active, void* part) {
  const Plan& p = b->plan[prec];
  if (b->dim == 1) {
    if (b->max_ord > 1024) return RTE_EINVAL;
    int threads = ((b->max_ord + 63) / 64) * 64;
    if (prec == 0)
      hipLaunchKernelGGL(sweep1d_kernel<double>, dim3(b->n_inst), dim3(threads), 0, s, b->d_inst,
                         p.d_parts, b->d_ox, b->d_w, b->d_perm, b->d_region, sigma_t, sigma_s,
                         b->max_regions, qx, qadd, inflow, reinterpret_cast<double*>(part),
                         psi_out, active);
    else
      hipLaunchKernelGGL(sweep1d_kernel<float>, dim3(b->n_inst), dim3(threads), 0, s, b->d_inst,
                         p.d_parts, b->d_ox, b->d_w, b->d_perm, b->d_region, sigma_t, sigma_s,
                         b->max_regions, qx, qadd, inflow, reinterpret_cast<float*>(part),
                         psi_out, active);
    RTE_HIP(hipGetLastError());
    return RTE_OK;
  }
  if (prec == 0)
    return launch2d_g<double>(b, p, sigma_t, sigma_s, qx, qadd, inflow, psi_out, s, active, part);
  return launch2d_g<float>(b, p, sigma_t, sigma_s, qx, qadd, inflow, psi_out, s, active, part);
}

int reduce_partials(rte_batch* b, int prec, double alpha, const double* x, double beta, double* out,
                    hipStream_t s, const int32_t* active, const double* y, double gamma, const void* part_buf) {
  const Plan& p = b->plan[prec];
  const void* part = part_buf ? part_buf : b->d_part;
  int64_t maxnd = 0;
  for (const auto& I : b->inst) maxnd = std::max<int64_t>(maxnd, (int64_t)I.nx * I.ny * I.nloc);
  dim3 grid((unsigned)std::min<int64_t>((maxnd + 255) / 256, 1024), b->n_inst);
  if (prec == 0)
    hipLaunchKernelGGL(reduce_partials_kernel<double>, grid, dim3(256), 0, s, b->d_inst, p.d_parts,
                       reinterpret_cast<const double*>(part), alpha, x, beta, y, gamma, out,
                       active);
  else
    hipLaunchKernelGGL(reduce_partials_kernel<float>, grid, dim3(256), 0, s, b->d_inst, p.d_parts,
                       reinterpret_cast<const float*>(part), alpha, x, beta, y, gamma, out,
                       active);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int reduce_partials_dot(rte_batch* b, int prec, double alpha, const double* x, double beta, double* out,
                        const double* dotv, double* part, int maxc, int chunk, hipStream_t s,
                        const int32_t* active) {
  const Plan& p = b->plan[prec];
  const dim3 grid((unsigned)maxc, b->n_inst);
  if (prec == 0)
    hipLaunchKernelGGL(reduce_partials_dot_kernel<double>, grid, dim3(256), 0, s, b->d_inst, p.d_parts,
                       reinterpret_cast<const double*>(b->d_part), alpha, x, beta, out, dotv, part, maxc, chunk,
                       active);
  else
    hipLaunchKernelGGL(reduce_partials_dot_kernel<float>, grid, dim3(256), 0, s, b->d_inst, p.d_parts,
                       reinterpret_cast<const float*>(b->d_part), alpha, x, beta, out, dotv, part, maxc, chunk,
                       active);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int scalar_flux(rte_batch* b, const double* psi, double* phi, hipStream_t s) {
  int64_t maxnd = 0;
  for (const auto& I : b->inst) maxnd = std::max<int64_t>(maxnd, (int64_t)I.nx * I.ny * I.nloc);
  dim3 grid((unsigned)std::min<int64_t>((maxnd + 255) / 256, 1024), b->n_inst);
  hipLaunchKernelGGL(scalar_flux_kernel, grid, dim3(256), sizeof(double) * b->max_ord, s,
                     b->d_inst, b->d_w, b->d_perm, psi, phi);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int set_sweep_order(rte_batch* b, int prec, int order) {
  if (!b || prec < 0 || prec > 1 || order < 0 || order > 1) return RTE_EINVAL;
  Plan& p = b->plan[prec];
  p.order = order;
  const int variant = p.variant;
  const bool tuned = p.tuned;
  RTE_TRY(make_plan(b, prec, p.G, p.threads, p.opl));
  p.variant = variant;
  p.tuned = tuned;
  return RTE_OK;
}

int set_sweep_plan(rte_batch* b, int prec, int variant, int G, int opl, int threads) {
  if (!b || prec < 0 || prec > 1 || variant < 0 || variant > 2) return RTE_EINVAL;
  b->plan[prec].order = 0;
  if (variant == 2) {  // wave per item: one lane per cell, 64 threads
    if (b->dim != 2 || G != 1 || threads != 64 || !wave_variant_fits(b, opl) ||
        wave_lds(b, opl, prec == 0 ? 8 : 4) > 64 * 1024)
      return RTE_EINVAL;
    RTE_TRY(make_plan(b, prec, G, threads, opl));
    b->plan[prec].variant = variant;
    b->plan[prec].tuned = true;
    return RTE_OK;
  }
  if (threads < 64 || threads > 1024 || threads % 64 || !plan_shape_ok(G, opl) || threads % G ||
      (threads > 512 && (variant != 1 || b->dim != 2)))
    return RTE_EINVAL;
  if (b->dim == 2) {
    if (sweep_lds(b, G, opl, variant, prec == 0 ? 8 : 4) > 64 * 1024) return RTE_EINVAL;
    if (variant == 1 && !rows_variant_fits(b, G, opl, threads, prec == 0 ? 8 : 4)) return RTE_EINVAL;
  }
  RTE_TRY(make_plan(b, prec, G, threads, opl));
  b->plan[prec].variant = variant;
  b->plan[prec].tuned = true;
  return RTE_OK;
}

// Pick the plan (kernel variant, G lanes per cell, OPL ordinates per lane,
// work-group size) for this batch by timing sweeps of each candidate that
// fits; the fastest plan is kept.
int autotune_sweep(rte_batch* b, int prec, const double* sigma_t, hipStream_t s, const double* sigma_s) {
  Plan& cur = b->plan[prec];
  if (cur.tuned || b->dim == 1) return RTE_OK;
  const int cand_G[] = {4, 8, 16, 32};
  const int cand_T[] = {128, 256, 512, 768, 1024};  // above 512: row-slot kernel, one row per slot
  hipEvent_t e0, e1;
  RTE_HIP(hipEventCreate(&e0));
  RTE_HIP(hipEventCreate(&e1));
  // a constant nonzero source (every byte 0x3F: each entry is 4.8e-4) keeps the
  // arithmetic as in a solve; large batches are timed on an evenly strided
  // sample of 256 instances (enough to fill the chip)
  double* q = nullptr;
  int32_t* mask = nullptr;
  if (hipMalloc(&q, sizeof(double) * b->total_dof) != hipSuccess) return RTE_ENOMEM;
  RTE_HIP(hipMemsetAsync(q, 0x3F, sizeof(double) * b->total_dof, s));
  const int n = b->n_inst, ns = std::min(n, 256);
  if (ns < n) {
    std::vector<int32_t> h(n, 0);
    for (int k = 0; k < ns; ++k) h[(int64_t)k * n / ns] = 1;
    if (hipMalloc(&mask, sizeof(int32_t) * n) != hipSuccess) {
      (void)hipFree(q);
      return RTE_ENOMEM;
    }
    RTE_HIP(hipMemcpy(mask, h.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
  }
  struct Cand {
    int V, O, G, T;
    float ms;
    int order = 0;
  };
  std::vector<Cand> cands;
  // the operator's form (sigma_s-scaled source) when sigma_s is given
  const double* qx = sigma_s ? q : nullptr;
  const double* qa = sigma_s ? nullptr : q;
  auto time_plan = [&](const Cand& c, int trials, float& ms) -> int {
    b->plan[prec].order = c.order;
    RTE_TRY(make_plan(b, prec, c.G, c.T, c.O));
    b->plan[prec].variant = c.V;
    RTE_TRY(sweep_launch(b, prec, sigma_t, sigma_s, qx, qa, nullptr, nullptr, s, mask, -2.0));
    for (int trial = 0; trial < trials; ++trial) {  // best of `trials` timings of 4 sweeps
      RTE_HIP(hipEventRecord(e0, s));
      for (int rep = 0; rep < 4; ++rep)
        RTE_TRY(sweep_launch(b, prec, sigma_t, sigma_s, qx, qa, nullptr, nullptr, s, mask, -2.0));
      RTE_HIP(hipEventRecord(e1, s));
      RTE_HIP(hipEventSynchronize(e1));
      float t = 0.f;
      RTE_HIP(hipEventElapsedTime(&t, e0, e1));
      ms = std::min(ms, t);
    }
    return RTE_OK;
  };
  // wave per item (variant 2): for small batches, whose few work items
  // leave the chip idle with the larger work groups (its partial fluxes,
  // one vector per OPL ordinates, would cost large batches too much)
  if (b->n_inst <= 16)
    for (int O = 1; O <= 4; O *= 2) {
      if (!wave_variant_fits(b, O) || wave_lds(b, O, prec == 0 ? 8 : 4) > 64 * 1024) continue;
      Cand c{2, O, 1, 64, 1e30f};
      RTE_TRY(time_plan(c, 3, c.ms));
      cands.push_back(c);
    }
  for (int V = 0; V < 2; ++V) {
    for (int O = 1; O <= 8; O *= 2) {
      for (int G : cand_G) {
        if (!plan_shape_ok(G, O) || G * O > 32) continue;
        for (int T : cand_T) {
          if (T % G || T / G < 1 || (V == 0 && T > 512)) continue;
          if (V == 1 && !rows_variant_fits(b, G, O, T, prec == 0 ? 8 : 4)) continue;
          if (sweep_lds(b, G, O, V, prec == 0 ? 8 : 4) > 64 * 1024) continue;
          Cand c{V, O, G, T, 1e30f};
          RTE_TRY(time_plan(c, 3, c.ms));
          cands.push_back(c);
        }
      }
    }
  }
  // the three fastest again, in turn, so that drift between the first timings
  // cannot decide between near-equal plans
  std::sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& c) { return a.ms < c.ms; });
  size_t top = std::min<size_t>(3, cands.size());
  cands.resize(top);
  // in a batch of unequal instances, each of them also with its largest work
  // items started first
  bool uneven = false;
  for (const auto& I : b->inst)
    uneven = uneven || (int64_t)I.nx * I.ny * I.n_ord != (int64_t)b->inst[0].nx * b->inst[0].ny * b->inst[0].n_ord;
  if (uneven)
    for (size_t k = 0; k < top; ++k) {
      Cand c = cands[k];
      c.order = 1;
      cands.push_back(c);
    }
  top = cands.size();
  for (size_t k = 0; k < top; ++k) cands[k].ms = 1e30f;
  for (int round = 0; round < 4; ++round)
    for (size_t k = 0; k < top; ++k) RTE_TRY(time_plan(cands[k], 1, cands[k].ms));
  size_t bk = 0;
  for (size_t k = 1; k < top; ++k)
    if (cands[k].ms < cands[bk].ms) bk = k;
  (void)hipFree(q);
  (void)hipFree(mask);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (top == 0) {  // nothing admissible to time: the current shape, diagonal-slot kernel
    cur.order = 0;
    RTE_TRY(make_plan(b, prec, cur.G, cur.threads, cur.opl));
    cur.variant = 0;
    cur.tuned = true;
    return RTE_OK;
  }
  const Cand& c = cands[bk];
  b->plan[prec].order = c.order;
  RTE_TRY(make_plan(b, prec, c.G, c.T, c.O));
  b->plan[prec].variant = c.V;
  b->plan[prec].tuned = true;
  return RTE_OK;
}

}  // namespace rte
