// Batched FP64 Krylov kernels: reductions are deterministic (per-work-group
// partial sums, then a fixed-order sum per instance; or one work group per
// instance, summing in a fixed order), every kernel skips instances whose mask
// entry is 0.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "krylov.h"

namespace rte {

int Space::init(const std::vector<int64_t>& lens) {
  n = (int)lens.size();
  len = lens;
  off.resize(n);
  total = 0;
  max_len = 0;
  for (int b = 0; b < n; ++b) {
    off[b] = total;
    total += lens[b];
    max_len = std::max(max_len, lens[b]);
  }
  if (hipMalloc(&d_off, sizeof(int64_t) * n) != hipSuccess ||
      hipMalloc(&d_len, sizeof(int64_t) * n) != hipSuccess)
    return RTE_ENOMEM;
  RTE_HIP(hipMemcpy(d_off, off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice));
  RTE_HIP(hipMemcpy(d_len, len.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice));
  return RTE_OK;
}

void Space::release() {
  (void)hipFree(d_off);
  (void)hipFree(d_len);
  d_off = d_len = nullptr;
}

int Krylov::init(const std::vector<int64_t>& lens, int m_, bool flex) {
  RTE_TRY(sp.init(lens));
  m = m_;
  flexible = flex;
  const int n = sp.n;
  const int mc = sp.max_chunks();
  auto al = [](void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 8)) == hipSuccess; };
  bool ok = al((void**)&V, sizeof(double) * (m + 1) * sp.total) &&
            (!flex || al((void**)&Z, sizeof(double) * m * sp.total)) &&
            al((void**)&H, sizeof(double) * n * (m + 1) * m) &&
            al((void**)&R, sizeof(double) * n * (m + 1) * m) &&
            al((void**)&cs, sizeof(double) * n * m) && al((void**)&sn, sizeof(double) * n * m) &&
            al((void**)&g, sizeof(double) * n * (m + 1)) && al((void**)&y, sizeof(double) * n * m) &&
            al((void**)&partA, sizeof(double) * n * mc) &&
            al((void**)&partB, sizeof(double) * n * mc) &&
            al((void**)&scal, sizeof(double) * n * 8) && al((void**)&active, sizeof(int32_t) * n) &&
            al((void**)&jdone, sizeof(int32_t) * n) && al((void**)&fail, sizeof(int32_t) * n);
  if (!ok) return RTE_ENOMEM;
  RTE_HIP(hipMemset(fail, 0, sizeof(int32_t) * n));
  RTE_HIP(hipMemset(H, 0, sizeof(double) * n * (m + 1) * m));
  RTE_HIP(hipMemset(scal, 0, sizeof(double) * n * 8));
  return RTE_OK;
}

void Krylov::release() {
  for (void* p : {(void*)V, (void*)Z, (void*)H, (void*)R, (void*)cs, (void*)sn, (void*)g, (void*)y,
                  (void*)partA, (void*)partB, (void*)scal, (void*)active, (void*)jdone, (void*)fail})
    (void)hipFree(p);
  V = Z = H = R = cs = sn = g = y = partA = partB = scal = nullptr;
  active = jdone = fail = nullptr;
  sp.release();
}

__device__ __forceinline__ double block_sum256(double v, double* sh) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
  __syncthreads();
  return t;  // valid in thread 0
}

__global__ void k_dot_part(const int64_t* __restrict__ off, const int64_t* __restrict__ len,
                           const double* __restrict__ x, const double* __restrict__ y,
                           double* __restrict__ part, int maxc, const int32_t* __restrict__ active) {
  __shared__ double sh[KTHREADS / 64];
  const int b = blockIdx.y, c = blockIdx.x;
  if (active && !active[b]) return;
  const int64_t n = len[b], base = off[b], start = (int64_t)c * KCHUNK;
  if (start >= n) return;
  const int64_t end = min(n, start + (int64_t)KCHUNK);
  double acc = 0.0;
  if (((base | start | end) & 1) == 0) {  // pairs of DoFs per 16-byte load
    for (int64_t e = start + 2 * threadIdx.x; e < end; e += 2 * blockDim.x) {
      const double2 xv = *reinterpret_cast<const double2*>(x + base + e);
      const double2 yv = y ? *reinterpret_cast<const double2*>(y + base + e) : xv;
      acc += xv.x * yv.x + xv.y * yv.y;
    }
  } else {
    for (int64_t e = start + threadIdx.x; e < end; e += blockDim.x) {
      const double xv = x[base + e];
      acc += xv * (y ? y[base + e] : xv);
    }
  }
  acc = block_sum256(acc, sh);
  if (threadIdx.x == 0) part[(int64_t)b * maxc + c] = acc;
}

__global__ void k_finish(int n, const int64_t* __restrict__ len, const double* __restrict__ part,
                         int maxc, double* __restrict__ out, int stride, int take_sqrt,
                         const int32_t* __restrict__ active) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n || (active && !active[b])) return;
  const int nc = (int)((len[b] + KCHUNK - 1) / KCHUNK);
  double t = 0.0;
  for (int c = 0; c < nc; ++c) t += part[(int64_t)b * maxc + c];
  out[(int64_t)b * stride] = take_sqrt ? sqrt(t) : t;
}

__global__ void k_scale(const int64_t* __restrict__ off, const int64_t* __restrict__ len,
                        const double* __restrict__ x, const double* __restrict__ sc, int stride,
                        double* __restrict__ y, const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int64_t n = len[b], base = off[b];
  const double d = sc[(int64_t)b * stride];
  const double f = d != 0.0 ? 1.0 / d : 0.0;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, step = (int64_t)gridDim.x * blockDim.x;
  if (((base | n) & 1) == 0) {  // pairs of DoFs per 16-byte access
    for (int64_t p = t0; 2 * p < n; p += step) {
      double2 v = *reinterpret_cast<const double2*>(x + base + 2 * p);
      v.x *= f;
      v.y *= f;
      *reinterpret_cast<double2*>(y + base + 2 * p) = v;
    }
  } else {
    for (int64_t e = t0; e < n; e += step) y[base + e] = x[base + e] * f;
  }
}

__global__ void k_axpby(const int64_t* __restrict__ off, const int64_t* __restrict__ len, double a,
                        const double* __restrict__ x, double bc, double* __restrict__ y,
                        const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int64_t n = len[b], base = off[b];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    y[base + e] = a * x[base + e] + (bc == 0.0 ? 0.0 : bc * y[base + e]);
}

// One MGS projection: h = <w, v_i> (from the partial sums of the previous
// pass), w -= h v_i, then partial sums of <w, v_{i+1}> (or <w, w> at the end).
__global__ void k_mgs_step(const int64_t* __restrict__ off, const int64_t* __restrict__ len,
                           double* __restrict__ w, const double* __restrict__ vi,
                           const double* __restrict__ vnext, const double* __restrict__ part_in,
                           double* __restrict__ part_out, int maxc, double* __restrict__ H, int m,
                           int i, int j, const int32_t* __restrict__ active) {
  __shared__ double sh[KTHREADS / 64];
  __shared__ double hs;
  const int b = blockIdx.y, c = blockIdx.x;
  if (active && !active[b]) return;
  const int64_t n = len[b], base = off[b], start = (int64_t)c * KCHUNK;
  if (start >= n) return;
  const int nc = (int)((n + KCHUNK - 1) / KCHUNK);
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < nc; ++k) t += part_in[(int64_t)b * maxc + k];
    hs = t;
    if (c == 0) H[(int64_t)b * (m + 1) * m + (int64_t)i * m + j] = t;
  }
  __syncthreads();
  const double h = hs;
  const int64_t end = min(n, start + (int64_t)KCHUNK);
  double acc = 0.0;
  if (((base | start | end) & 1) == 0) {
    // pairs of DoFs per load (16 B): offsets and lengths are even (whole cells)
    for (int64_t e = start + 2 * threadIdx.x; e < end; e += 2 * blockDim.x) {
      const double2 wp = *reinterpret_cast<const double2*>(w + base + e);
      const double2 vp = *reinterpret_cast<const double2*>(vi + base + e);
      double2 o;
      o.x = wp.x - h * vp.x;
      o.y = wp.y - h * vp.y;
      *reinterpret_cast<double2*>(w + base + e) = o;
      if (vnext) {
        const double2 np = *reinterpret_cast<const double2*>(vnext + base + e);
        acc += o.x * np.x + o.y * np.y;
      } else {
        acc += o.x * o.x + o.y * o.y;
      }
    }
  } else {
    for (int64_t e = start + threadIdx.x; e < end; e += blockDim.x) {
      const double wv = w[base + e] - h * vi[base + e];
      w[base + e] = wv;
      acc += wv * (vnext ? vnext[base + e] : wv);
    }
  }
  acc = block_sum256(acc, sh);
  if (threadIdx.x == 0) part_out[(int64_t)b * maxc + c] = acc;
}

// H[j+1][j] = ||w|| from the final partials; scal[4] = ||w||.
__global__ void k_arnoldi_tail(int n, const int64_t* __restrict__ len, const double* __restrict__ part,
                               int maxc, double* __restrict__ H, int m, int j,
                               double* __restrict__ scal, const int32_t* __restrict__ active) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n || !active[b]) return;
  const int nc = (int)((len[b] + KCHUNK - 1) / KCHUNK);
  double t = 0.0;
  for (int c = 0; c < nc; ++c) t += part[(int64_t)b * maxc + c];
  const double nw = sqrt(t);
  H[(int64_t)b * (m + 1) * m + (int64_t)(j + 1) * m + j] = nw;
  scal[b * 8 + 4] = nw;
}

// Givens update of column j; est = |g_{j+1}|; stop the instance when
// est <= tol_abs or on a breakdown H_{j+1,j} <= bt ||H(:, j)|| (Alg. 1 ends
// there).  A breakdown whose rotated diagonal entry rho is not above
// bt ||H(:, j)|| leaves the least squares singular (unhappy breakdown): column
// j is dropped and fail = KFAIL_BREAKDOWN.  A non-finite rho or estimate
// drops the column as well (fail = KFAIL_NONFINITE), so the update keeps the
// last finite iterate.  hc: column j of H (entry i at hc[i * hs]); c_old,
// s_old: the rotations of columns 0 .. j-1 (read before c and s are written).
__device__ __forceinline__ void givens_column(int b, const double* hc, int hs, double* __restrict__ Rb,
                                              const double* c_old, const double* s_old,
                                              double* __restrict__ c, double* __restrict__ s,
                                              double* __restrict__ gb, int m, int j,
                                              double* __restrict__ scal, int32_t* __restrict__ active,
                                              int32_t* __restrict__ jdone, int32_t* __restrict__ fail,
                                              double bt) {
  double colsq = 0.0;
  for (int i = 0; i <= j + 1; ++i) {
    Rb[i * m + j] = hc[i * hs];
    colsq += hc[i * hs] * hc[i * hs];
  }
  for (int k = 0; k < j; ++k) {
    const double a = Rb[k * m + j], bb = Rb[(k + 1) * m + j];
    Rb[k * m + j] = c_old[k] * a + s_old[k] * bb;
    Rb[(k + 1) * m + j] = -s_old[k] * a + c_old[k] * bb;
  }
  const double a = Rb[j * m + j], bb = Rb[(j + 1) * m + j];
  const double rho = hypot(a, bb);
  double cj = 1.0, sj = 0.0;
  if (rho > 0.0) {
    cj = a / rho;
    sj = bb / rho;
  }
  c[j] = cj;
  s[j] = sj;
  Rb[j * m + j] = rho;
  Rb[(j + 1) * m + j] = 0.0;
  const double gj = gb[j];
  gb[j] = cj * gj;
  gb[j + 1] = -sj * gj;
  const double est = fabs(gb[j + 1]);
  const double cn = sqrt(colsq);
  const bool finite = isfinite(rho) && isfinite(est) && isfinite(cn);
  const bool breakdown = hc[(j + 1) * hs] <= bt * cn;
  const bool unhappy = finite && breakdown && !(rho > bt * cn);
  scal[b * 8 + 5] = scal[b * 8 + 2];  // previous estimate
  if (!finite || unhappy) {
    // the least squares keeps columns 0 .. j-1, whose residual is |g_j| before this rotation
    jdone[b] = j;
    scal[b * 8 + 2] = fabs(gj);
    gb[j] = gj;
    fail[b] = finite ? KFAIL_BREAKDOWN : KFAIL_NONFINITE;
    active[b] = 0;
    return;
  }
  scal[b * 8 + 2] = est;
  jdone[b] = j + 1;
  if (est <= scal[b * 8 + 1] || breakdown) active[b] = 0;
}

__global__ void k_givens(int n, const double* __restrict__ H, double* __restrict__ R,
                         double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
                         int m, int j, double* __restrict__ scal, int32_t* __restrict__ active,
                         int32_t* __restrict__ jdone, int32_t* __restrict__ fail, double bt) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n || !active[b]) return;
  double* c = cs + (int64_t)b * m;
  double* s = sn + (int64_t)b * m;
  givens_column(b, H + (int64_t)b * (m + 1) * m + j, m, R + (int64_t)b * (m + 1) * m, c, s, c, s,
                g + (int64_t)b * (m + 1), m, j, scal, active, jdone, fail, bt);
}

// Sum over the work group, the same value in every thread (fixed order: a
// butterfly within each wave, then the waves in turn).  sh holds one slot per
// wave; alternate two such arrays between consecutive calls, so that no
// second barrier is needed before the next call writes its slots.
template <int NT>
__device__ __forceinline__ double group_sum_all(double v, double* sh) {
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) v += __shfl_xor(v, k, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) t += sh[k];
  return t;
}

// w = z - sum_p part_p on a thread's pairs (pair k at byte offset
// t 16 + k NT 16 of the FP64 arrays), the partials summed in order in FP64
// (one pass over the pairs per partial, accumulating in w) and combined as
// the partial-flux reduction combines them; returns the thread's share of
// <w, v_0>.  Pairs past the end (nbytes) read the first pair and become zeros.
template <int NT, int NP, int GROUP, typename preal>
__device__ __forceinline__ double form_w(double2 (&w)[NP], const preal* __restrict__ pb, int np, int64_t n,
                                         const double* __restrict__ zb, const double* __restrict__ v0, int t,
                                         uint32_t nbytes) {
  using P2 = typename std::conditional<sizeof(preal) == 4, float2, double2>::type;
#pragma unroll
  for (int k = 0; k < NP; ++k) w[k] = make_double2(0.0, 0.0);
  for (int q = 0; q < np; ++q) {
    uint32_t tb = (uint32_t)t * 16u;
    asm volatile("" : "+v"(tb));
    const preal* pq = pb + (int64_t)q * n;
#pragma unroll
    for (int k0 = 0; k0 < NP; k0 += GROUP) {
#pragma unroll
      for (int k = k0; k < k0 + GROUP && k < NP; ++k) {
        const uint32_t ob = tb + (uint32_t)(k * NT * 16);
        const P2 a = *reinterpret_cast<const P2*>(pq + ((ob < nbytes ? ob : 0u) >> 3));
        w[k].x += (double)a.x;
        w[k].y += (double)a.y;
      }
#pragma unroll
      for (int k = k0; k < k0 + GROUP && k < NP; ++k) asm volatile("" : "+v"(w[k].x), "+v"(w[k].y)::"memory");
    }
  }
  uint32_t tb = (uint32_t)t * 16u;
  asm volatile("" : "+v"(tb));
  double acc = 0.0;
#pragma unroll
  for (int k0 = 0; k0 < NP; k0 += GROUP) {
#pragma unroll
    for (int k = k0; k < k0 + GROUP && k < NP; ++k) {
      const uint32_t ob = tb + (uint32_t)(k * NT * 16);
      const bool in = ob < nbytes;
      const uint32_t e = (in ? ob : 0u) >> 3;
      const double2 z = *reinterpret_cast<const double2*>(zb + e);
      const double2 v = *reinterpret_cast<const double2*>(v0 + e);
      double wx = -1.0 * w[k].x, wy = -1.0 * w[k].y;
      wx += 1.0 * z.x;
      wy += 1.0 * z.y;
      w[k] = in ? make_double2(wx, wy) : make_double2(0.0, 0.0);
      acc += w[k].x * v.x + w[k].y * v.y;
    }
    asm volatile("" : "+v"(acc)::"memory");
  }
  return acc;
}

// Arnoldi step j of every active instance, one work group per instance: w
// (= V[j+1], PT values per thread, pairs of DoFs 2 (t + k NT)) stays in
// registers through the MGS projections, each one pass that subtracts
// h_i v_i and forms the next projection's dot, <w, v_{i+1}> (the squared norm
// after the last); then w is normalised and stored once, and thread 0 applies
// the Givens rotations of column j (the column and the earlier rotations
// staged in LDS).  The MGS of the chunked kernels in one launch, with w read
// and written once instead of once per projection.  part0 (nullable): chunk
// partials of <w, v_0> that the operator's reduction left, else the first
// dot is a pass of its own.  Needs len <= NT * PT and even offsets/lengths.
constexpr int ARN_MAX_M = 500;
template <int NT, int PT, int FORM>
__global__ void __launch_bounds__(NT) k_arnoldi_reg(
    const int64_t* __restrict__ off, const int64_t* __restrict__ len, double* __restrict__ V, int64_t total,
    const double* __restrict__ part0, int maxc, double* __restrict__ H, double* __restrict__ R,
    double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g, int m, int j,
    double* __restrict__ scal, int32_t* __restrict__ active, int32_t* __restrict__ jdone,
    int32_t* __restrict__ fail, double bt, const InstPart* __restrict__ parts, const void* __restrict__ part,
    const double* __restrict__ zsrc) {
  constexpr int NP = PT / 2;
  // pairs per group of loads: fewer where w takes most registers
  constexpr int ARN_GROUP = PT > 32 ? 2 : 4;
  __shared__ double sh[2][NT / 64];
  __shared__ double hcol[ARN_MAX_M + 1], c_old[ARN_MAX_M], s_old[ARN_MAX_M];
  const int b = blockIdx.x;
  if (!active[b]) return;
  const int t = threadIdx.x;
  const int64_t n = len[b], base = off[b];
  for (int k = t; k < j; k += NT) {
    c_old[k] = cs[(int64_t)b * m + k];
    s_old[k] = sn[(int64_t)b * m + k];
  }
  // byte offsets (32-bit) of a thread's pairs from an instance's start: pair
  // k at tb + k NT 16.  tb passes through an empty asm statement in every
  // pass, so the compiler forms each pair's address where it is used rather
  // than holding one per pair across the passes (their registers would
  // spill).  A pair past the instance's end reads the instance's first pair
  // and takes zeros instead, so every address stays in bounds.
  const uint32_t nbytes = (uint32_t)(n * 8);
  auto pair = [nbytes](const double* p, uint32_t ob) {
    const bool in = ob < nbytes;
    const double2 v = *reinterpret_cast<const double2*>(reinterpret_cast<const char*>(p) + (in ? ob : 0u));
    return in ? v : make_double2(0.0, 0.0);
  };
  double* wp = V + (int64_t)(j + 1) * total + base;
  double2 w[NP];
  int par = 0;
  double h;
  if constexpr (FORM != 0) {
    // w = z - (the sum of the operator's partial fluxes: FP32 with FORM 1,
    // FP64 with FORM 2), formed as the partial-flux reduction forms it (same
    // order, same rounding), and its dot with v_0 on the way
    using preal = typename std::conditional<FORM == 1, float, double>::type;
    const InstPart pp = parts[b];
    const double acc = form_w<NT, NP, ARN_GROUP, preal>(w, reinterpret_cast<const preal*>(part) + pp.off, pp.n,
                                                        n, zsrc + base, V + base, t, nbytes);
    h = group_sum_all<NT>(acc, sh[par]);
    par ^= 1;
  } else {
    {
      uint32_t tb = (uint32_t)t * 16u;
      asm volatile("" : "+v"(tb));
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        const uint32_t ob = tb + (uint32_t)(k * NT * 16);
        w[k] = pair(wp, ob);
      }
    }
    if (part0) {
      if (t == 0) {
        const int nc = (int)((n + KCHUNK - 1) / KCHUNK);
        double s0 = 0.0;
        for (int c = 0; c < nc; ++c) s0 += part0[(int64_t)b * maxc + c];
        sh[1][0] = s0;
      }
      __syncthreads();
      h = sh[1][0];
    } else {
      const double* v0 = V + base;
      uint32_t tb = (uint32_t)t * 16u;
      asm volatile("" : "+v"(tb));
      double acc = 0.0;
#pragma unroll
      for (int k0 = 0; k0 < NP; k0 += ARN_GROUP) {
#pragma unroll
        for (int k = k0; k < k0 + ARN_GROUP && k < NP; ++k) {
          const double2 v = pair(v0, tb + (uint32_t)(k * NT * 16));
          acc += w[k].x * v.x + w[k].y * v.y;
        }
        asm volatile("" : "+v"(acc)::"memory");
      }
      h = group_sum_all<NT>(acc, sh[par]);
      par ^= 1;
    }
  }
  for (int i = 0; i <= j; ++i) {
    if (t == 0) hcol[i] = h;
    const double* vi = V + (int64_t)i * total + base;
    // the next dot: <w, v_{i+1}>, or <w, w> after the last projection (then
    // u repeats v_i's loads, from the cache, and is not used)
    const bool last = i == j;
    const double* un = last ? vi : V + (int64_t)(i + 1) * total + base;
    uint32_t tb = (uint32_t)t * 16u;
    asm volatile("" : "+v"(tb));
    double acc = 0.0;
    // groups of ARN_GROUP pairs: the empty asm statement after each group
    // takes the group's dot (so its arithmetic is done there) and orders
    // memory, which keeps the compiler from hoisting every load of the pass
    // ahead of the arithmetic
#pragma unroll
    for (int k0 = 0; k0 < NP; k0 += ARN_GROUP) {
#pragma unroll
      for (int k = k0; k < k0 + ARN_GROUP && k < NP; ++k) {
        const uint32_t ob = tb + (uint32_t)(k * NT * 16);
        const double2 v = pair(vi, ob), u = pair(un, ob);
        w[k].x -= h * v.x;
        w[k].y -= h * v.y;
        acc += w[k].x * (last ? w[k].x : u.x) + w[k].y * (last ? w[k].y : u.y);
      }
      asm volatile("" : "+v"(acc)::"memory");
    }
    h = group_sum_all<NT>(acc, sh[par]);
    par ^= 1;
  }
  const double nw = sqrt(h);
  const double f = nw != 0.0 ? 1.0 / nw : 0.0;
  {
    uint32_t tb = (uint32_t)t * 16u;
    asm volatile("" : "+v"(tb));
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const uint32_t ob = tb + (uint32_t)(k * NT * 16);
      if (ob < nbytes)
        *reinterpret_cast<double2*>(reinterpret_cast<char*>(wp) + ob) = make_double2(w[k].x * f, w[k].y * f);
    }
  }
  if (t == 0) {
    hcol[j + 1] = nw;
    double* Hb = H + (int64_t)b * (m + 1) * m;
    for (int i = 0; i <= j + 1; ++i) Hb[i * m + j] = hcol[i];
    scal[b * 8 + 4] = nw;
    givens_column(b, hcol, 1, R + (int64_t)b * (m + 1) * m, c_old, s_old, cs + (int64_t)b * m,
                  sn + (int64_t)b * m, g + (int64_t)b * (m + 1), m, j, scal, active, jdone, fail, bt);
  }
}

__global__ void k_backsolve(int n, const double* __restrict__ R, const double* __restrict__ g, int m,
                            const int32_t* __restrict__ jdone, double* __restrict__ y,
                            const int32_t* __restrict__ incycle) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n || (incycle && !incycle[b])) return;
  const int jd = jdone[b];
  const double* Rb = R + (int64_t)b * (m + 1) * m;
  const double* gb = g + (int64_t)b * (m + 1);
  double* yb = y + (int64_t)b * m;
  for (int i = jd - 1; i >= 0; --i) {
    double t = gb[i];
    for (int k = i + 1; k < jd; ++k) t -= Rb[i * m + k] * yb[k];
    const double d = Rb[i * m + i];
    yb[i] = d != 0.0 ? t / d : 0.0;
  }
}

__global__ void k_update(const int64_t* __restrict__ off, const int64_t* __restrict__ len,
                         int64_t total, const double* __restrict__ basis, const double* __restrict__ y,
                         int m, const int32_t* __restrict__ jdone, double* __restrict__ X,
                         const int32_t* __restrict__ incycle) {
  const int b = blockIdx.y;
  if (incycle && !incycle[b]) return;
  const int jd = jdone[b];
  if (jd == 0) return;
  const int64_t n = len[b], base = off[b];
  const double* yb = y + (int64_t)b * m;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, step = (int64_t)gridDim.x * blockDim.x;
  if (((base | n | total) & 1) == 0) {  // pairs of DoFs per 16-byte access
    for (int64_t p = t0; 2 * p < n; p += step) {
      const int64_t e = base + 2 * p;
      double2 acc = *reinterpret_cast<const double2*>(X + e);
      for (int i = 0; i < jd; ++i) {
        const double2 v = *reinterpret_cast<const double2*>(basis + (int64_t)i * total + e);
        acc.x += yb[i] * v.x;
        acc.y += yb[i] * v.y;
      }
      *reinterpret_cast<double2*>(X + e) = acc;
    }
  } else {
    for (int64_t e = t0; e < n; e += step) {
      double acc = X[base + e];
      for (int i = 0; i < jd; ++i) acc += yb[i] * basis[(int64_t)i * total + base + e];
      X[base + e] = acc;
    }
  }
}

__global__ void k_start(int n, double* __restrict__ scal, double* __restrict__ g, int m,
                        const double* __restrict__ tol_abs, double cycle_rel,
                        int32_t* __restrict__ active, int32_t* __restrict__ jdone) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  jdone[b] = 0;
  if (!active[b]) return;
  const double beta = scal[b * 8 + 0];
  scal[b * 8 + 1] = fmax(tol_abs[b], cycle_rel * beta);
  scal[b * 8 + 2] = beta;
  double* gb = g + (int64_t)b * (m + 1);
  gb[0] = beta;
  for (int i = 1; i <= m; ++i) gb[i] = 0.0;
  if (beta <= tol_abs[b]) active[b] = 0;  // already converged: no cycle
}

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static dim3 vgrid(const Space& sp) {
  return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((sp.max_len + 255) / 256, 512)), sp.n);
}

int fill_i32(int32_t* p, int n, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int knorm(const Space& sp, const double* x, double* part, double* out, int stride,
          const int32_t* active, hipStream_t s) {
  const int mc = sp.max_chunks();
  hipLaunchKernelGGL(k_dot_part, dim3(mc, sp.n), dim3(KTHREADS), 0, s, sp.d_off, sp.d_len, x,
                     (const double*)nullptr, part, mc, active);
  hipLaunchKernelGGL(k_finish, dim3((sp.n + 63) / 64), dim3(64), 0, s, sp.n, sp.d_len, part, mc, out,
                     stride, 1, active);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int knorm_finish(const Space& sp, const double* part, double* out, int stride, const int32_t* active,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3((sp.n + 63) / 64), dim3(64), 0, s, sp.n, sp.d_len, part, sp.max_chunks(),
                     out, stride, 1, active);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int kdot(const Space& sp, const double* x, const double* y, double* part, double* out, int stride,
         const int32_t* active, hipStream_t s) {
  const int mc = sp.max_chunks();
  hipLaunchKernelGGL(k_dot_part, dim3(mc, sp.n), dim3(KTHREADS), 0, s, sp.d_off, sp.d_len, x, y,
                     part, mc, active);
  hipLaunchKernelGGL(k_finish, dim3((sp.n + 63) / 64), dim3(64), 0, s, sp.n, sp.d_len, part, mc, out,
                     stride, 0, active);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int kscale(const Space& sp, const double* x, const double* sc, int stride, double* y,
           const int32_t* active, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, vgrid(sp), dim3(256), 0, s, sp.d_off, sp.d_len, x, sc, stride, y,
                     active);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int kaxpby(const Space& sp, double a, const double* x, double bc, double* y, const int32_t* active,
           hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, vgrid(sp), dim3(256), 0, s, sp.d_off, sp.d_len, a, x, bc, y, active);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int kcopy(const Space& sp, const double* x, double* y, const int32_t* active, hipStream_t s) {
  return kaxpby(sp, 1.0, x, 0.0, y, active, s);
}

int kstart(Krylov& K, const double* r, const double* tol_abs, hipStream_t s, double cycle_rel) {
  const Space& sp = K.sp;
  RTE_TRY(knorm(sp, r, K.partA, K.scal + 0, 8, K.active, s));
  hipLaunchKernelGGL(k_start, dim3((sp.n + 63) / 64), dim3(64), 0, s, sp.n, K.scal, K.g, K.m, tol_abs,
                     cycle_rel, K.active, K.jdone);
  RTE_HIP(hipGetLastError());
  return kscale(sp, r, K.scal + 0, 8, K.v(0), K.active, s);
}

// The register-resident step: NT threads of PT values each cover every
// instance, all offsets and lengths even (whole pairs of DoFs).
template <int NT, int PT>
static void launch_arnoldi_reg(Krylov& K, int j, hipStream_t s, bool first_dot_ready, const PartialSrc* src) {
  const Space& sp = K.sp;
  const double* p0 = first_dot_ready ? (const double*)K.partA : nullptr;
  const InstPart* parts = src ? src->parts : nullptr;
  const void* part = src ? src->part : nullptr;
  const double* z = src ? src->z : nullptr;
  if (!src)
    hipLaunchKernelGGL((k_arnoldi_reg<NT, PT, 0>), dim3(sp.n), dim3(NT), 0, s, sp.d_off, sp.d_len, K.V, sp.total, p0,
                       sp.max_chunks(), K.H, K.R, K.cs, K.sn, K.g, K.m, j, K.scal, K.active, K.jdone, K.fail, K.bt,
                       parts, part, z);
  else if (src->f32)
    hipLaunchKernelGGL((k_arnoldi_reg<NT, PT, 1>), dim3(sp.n), dim3(NT), 0, s, sp.d_off, sp.d_len, K.V, sp.total, p0,
                       sp.max_chunks(), K.H, K.R, K.cs, K.sn, K.g, K.m, j, K.scal, K.active, K.jdone, K.fail, K.bt,
                       parts, part, z);
  else
    hipLaunchKernelGGL((k_arnoldi_reg<NT, PT, 2>), dim3(sp.n), dim3(NT), 0, s, sp.d_off, sp.d_len, K.V, sp.total, p0,
                       sp.max_chunks(), K.H, K.R, K.cs, K.sn, K.g, K.m, j, K.scal, K.active, K.jdone, K.fail, K.bt,
                       parts, part, z);
}

// Up to 1024 x 48 values (w in 96 of the 128 registers a thread has with
// 1024 threads); longer vectors take the chunked kernels.
constexpr int64_t ARN_MAX_LEN = 1024 * 48;

bool arnoldi_in_registers(const Krylov& K) {
  const Space& sp = K.sp;
  bool even = (sp.total & 1) == 0;
  for (int q = 0; q < sp.n && even; ++q) even = ((sp.off[q] | sp.len[q]) & 1) == 0;
  return even && K.m <= ARN_MAX_M && sp.max_len <= ARN_MAX_LEN;
}

int arnoldi_mgs(Krylov& K, int j, hipStream_t s, bool first_dot_ready, const PartialSrc* src) {
  const Space& sp = K.sp;
  const int mc = sp.max_chunks();
  double* w = K.v(j + 1);
  const bool reg = arnoldi_in_registers(K);
  if (src && !reg) return RTE_EINVAL;  // w from partials: the register-resident step only
  if (reg) {
    const int64_t L = sp.max_len;
    if (L <= 1024 * 8) launch_arnoldi_reg<1024, 8>(K, j, s, first_dot_ready, src);
    else if (L <= 1024 * 16) launch_arnoldi_reg<1024, 16>(K, j, s, first_dot_ready, src);
    else if (L <= 1024 * 24) launch_arnoldi_reg<1024, 24>(K, j, s, first_dot_ready, src);
    else if (L <= 1024 * 32) launch_arnoldi_reg<1024, 32>(K, j, s, first_dot_ready, src);
    else if (L <= 1024 * 36) launch_arnoldi_reg<1024, 36>(K, j, s, first_dot_ready, src);
    else if (L <= 1024 * 40) launch_arnoldi_reg<1024, 40>(K, j, s, first_dot_ready, src);
    else launch_arnoldi_reg<1024, 48>(K, j, s, first_dot_ready, src);
    RTE_HIP(hipGetLastError());
    return RTE_OK;
  }
  if (!first_dot_ready)
    hipLaunchKernelGGL(k_dot_part, dim3(mc, sp.n), dim3(KTHREADS), 0, s, sp.d_off, sp.d_len, w, K.v(0),
                       K.partA, mc, K.active);
  double* pin = K.partA;
  double* pout = K.partB;
  for (int i = 0; i <= j; ++i) {
    const double* vn = (i < j) ? K.v(i + 1) : nullptr;
    hipLaunchKernelGGL(k_mgs_step, dim3(mc, sp.n), dim3(KTHREADS), 0, s, sp.d_off, sp.d_len, w,
                       K.v(i), vn, pin, pout, mc, K.H, K.m, i, j, K.active);
    std::swap(pin, pout);
  }
  hipLaunchKernelGGL(k_arnoldi_tail, dim3((sp.n + 63) / 64), dim3(64), 0, s, sp.n, sp.d_len, pin, mc,
                     K.H, K.m, j, K.scal, K.active);
  RTE_TRY(kscale(sp, w, K.scal + 4, 8, w, K.active, s));
  hipLaunchKernelGGL(k_givens, dim3((sp.n + 63) / 64), dim3(64), 0, s, sp.n, K.H, K.R, K.cs, K.sn,
                     K.g, K.m, j, K.scal, K.active, K.jdone, K.fail, K.bt);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

int kylov_solve_update(Krylov& K, const double* basis, double* X, hipStream_t s) {
  const Space& sp = K.sp;
  hipLaunchKernelGGL(k_backsolve, dim3((sp.n + 63) / 64), dim3(64), 0, s, sp.n, K.R, K.g, K.m,
                     K.jdone, K.y, (const int32_t*)nullptr);
  hipLaunchKernelGGL(k_update, vgrid(sp), dim3(256), 0, s, sp.d_off, sp.d_len, sp.total, basis, K.y,
                     K.m, K.jdone, X, (const int32_t*)nullptr);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

}  // namespace rte
