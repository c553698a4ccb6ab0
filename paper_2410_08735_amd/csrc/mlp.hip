// Learned flexible preconditioner: a GELU MLP that maps (normalised mu,
// normalised reduced residual coefficients g = W_1^T Sigma_s v) to reduced
// correction coefficients c, used as z = v + W_w c ||g|| in the first window
// iterations of FGMRES (which admits any nonlinear preconditioner, section 4.2).
//
// Matrix products run on the matrix cores: v_mfma_f32_16x16x16_bf16 with
// operands rounded to bfloat16 (round to nearest even) and FP32 accumulation;
// master weights, activations and Adam state are FP32.  An FP32 vector path
// (same kernels, no rounding) serves exact checks.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fgmres.h"

struct rte_mlp {
  int n_in = 0, width = 0, depth = 0, n_out = 0;
  std::vector<int> dims;            // n_in, width x depth, n_out
  std::vector<int64_t> woff, boff;  // offsets of W_l, b_l in the flat parameter vector
  int64_t nparams = 0;
  float* P = nullptr;               // parameters (FP32 master copy)
  float* M = nullptr;               // Adam first moment
  float* V = nullptr;               // Adam second moment
  float* G = nullptr;               // gradient
  float* yscale = nullptr;          // [n_out] output standardisation: y = net * scale + shift
  float* yshift = nullptr;
  int64_t adam_t = 0;
  // activation workspace for up to cap rows
  int cap = 0;
  std::vector<float*> H, Z;         // H[l]: layer-l input rows; Z[l]: pre-activations
  float *dA = nullptr, *dB = nullptr, *lossbuf = nullptr;
  float* ws = nullptr;              // split-K partial sums of the weight-gradient products
  int64_t ws_elems = 0;
};

namespace rte {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even on the upper 16 bits
__device__ __forceinline__ short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// C(m, n) = sum_k A(m, k) B(k, n) [+ bias(n)], strided operands, then an
// optional epilogue: act 1 stores Z = C and C = gelu(C).  FP32 on the vector
// units, one thread per entry (the exact path of the parity checks).
__global__ void k_gemm_f32(int Mr, int Nc, int Kd, const float* __restrict__ A, int64_t sam, int64_t sak,
                           const float* __restrict__ Bm, int64_t sbk, int64_t sbn, float* __restrict__ C,
                           int64_t scm, int64_t scn, const float* __restrict__ bias, int act,
                           float* __restrict__ Zout, int accumulate) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)Mr * Nc) return;
  const int m = (int)(id / Nc), n = (int)(id % Nc);
  float v = 0.f;
  for (int k = 0; k < Kd; ++k) v += A[m * sam + k * sak] * Bm[k * sbk + n * sbn];
  if (accumulate) v += C[m * scm + n * scn];
  if (bias) v += bias[n];
  if (act == 1) {
    Zout[m * scm + n * scn] = v;
    v = gelu_f(v);
  }
  C[m * scm + n * scn] = v;
}

// The BF16 product on the matrix cores, LDS-tiled: a work group of 256
// threads (4 waves) computes a 64 x 64 block of C.  Per K-chunk of 32 the
// group loads the 64 x 32 block of A and the 32 x 64 block of B from global
// memory once (consecutive threads along whichever operand index has unit
// stride), rounds them to bfloat16 (nearest even) into LDS, and each wave
// multiplies its 32 x 32 quarter as 2 x 2 v_mfma_f32_16x16x16_bf16 tiles per
// 16-deep step, reading its fragments as 8-byte LDS words.  Epilogue as in
// k_gemm_f32.  Operand layout of one MFMA (lane = r + 16 g): A(m0 + r, k0 + 4 g + q),
// B(k0 + 4 g + q, n0 + r) for q = 0..3; the result C(m0 + 4 g + q, n0 + r).
constexpr int GT_BM = 64, GT_BN = 64, GT_BK = 32, GT_LD = GT_BK + 4;  // LDS row pitch (shorts)

__global__ void __launch_bounds__(256) k_gemm_tiled(int Mr, int Nc, int Kd, const float* __restrict__ A, int64_t sam,
                                                    int64_t sak, const float* __restrict__ Bm, int64_t sbk,
                                                    int64_t sbn, float* __restrict__ C, int64_t scm, int64_t scn,
                                                    const float* __restrict__ bias, int act,
                                                    float* __restrict__ Zout, int accumulate) {
  __shared__ short As[GT_BM * GT_LD];  // [m][k]
  __shared__ short Bs[GT_BN * GT_LD];  // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int mb = blockIdx.y * GT_BM, nb = blockIdx.x * GT_BN;
  const int r = lane & 15, g = lane >> 4;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool a_rowmajor = sak == 1, b_rowmajor = sbn == 1;
  for (int k0 = 0; k0 < Kd; k0 += GT_BK) {
#pragma unroll
    for (int i = 0; i < (GT_BM * GT_BK) / 256; ++i) {
      const int e = tid + 256 * i;
      const int m = a_rowmajor ? e / GT_BK : e % GT_BM, k = a_rowmajor ? e % GT_BK : e / GT_BM;
      const int gm = mb + m, gk = k0 + k;
      const float v = (gm < Mr && gk < Kd) ? A[gm * sam + gk * sak] : 0.f;
      As[m * GT_LD + k] = f2bf(v);
    }
#pragma unroll
    for (int i = 0; i < (GT_BN * GT_BK) / 256; ++i) {
      const int e = tid + 256 * i;
      const int n = b_rowmajor ? e % GT_BN : e / GT_BK, k = b_rowmajor ? e / GT_BN : e % GT_BK;
      const int gn = nb + n, gk = k0 + k;
      const float v = (gn < Nc && gk < Kd) ? Bm[gk * sbk + gn * sbn] : 0.f;
      Bs[n * GT_LD + k] = f2bf(v);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GT_BK; kk += 16) {
      bf16x4 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const bf16x4*>(&As[(wm + 16 * i + r) * GT_LD + kk + 4 * g]);
        b[i] = *reinterpret_cast<const bf16x4*>(&Bs[(wn + 16 * i + r) * GT_LD + kk + 4 * g]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = mb + wm + 16 * i + 4 * g + q, n = nb + wn + 16 * j + r;
        if (m >= Mr || n >= Nc) continue;
        float v = acc[i][j][q];
        if (accumulate) v += C[m * scm + n * scn];
        if (bias) v += bias[n];
        if (act == 1) {
          Zout[m * scm + n * scn] = v;
          v = gelu_f(v);
        }
        C[m * scm + n * scn] = v;
      }
}

// The same product for operands whose unit-stride index is a multiple of 4
// long with 16-byte aligned rows (every product of the network): a work group
// of 256 threads (2 x 2 waves) computes a BM x BN block of C, each wave a
// (BM / 2) x (BN / 2) part as (BM / 32) x (BN / 32) MFMA tiles.  Operands come
// in as 16-byte loads along their unit-stride index, one K-chunk of 32 ahead:
// the loads of chunk t + 1 are in flight while the matrix cores work on chunk
// t from LDS, and are then rounded to bfloat16 into the other of two LDS
// buffers (one barrier per chunk).  With part set, the work group takes the
// K range [z kchunk, (z + 1) kchunk) of blockIdx.z and writes its raw sums to
// part[z] (the epilogue is then k_splitk_reduce's).  Rounding and the order of
// the 16-deep MFMA steps along K are those of k_gemm_tiled.
template <int BM, int BN>
__global__ void __launch_bounds__(256) k_gemm_pipe(int Mr, int Nc, int Kd, const float* __restrict__ A, int64_t sam,
                                                   int64_t sak, const float* __restrict__ Bm, int64_t sbk,
                                                   int64_t sbn, float* __restrict__ C, int64_t scm, int64_t scn,
                                                   const float* __restrict__ bias, int act,
                                                   float* __restrict__ Zout, int accumulate, int kchunk,
                                                   float* __restrict__ part) {
  constexpr int BK = 32, LD = BK + 4;              // LDS row pitch in shorts (72 B: 8-byte aligned rows)
  constexpr int TM = BM / 32, TN = BN / 32;        // MFMA tiles per wave along m and n
  constexpr int NA = BM * BK / 4 / 256, NB = BN * BK / 4 / 256;  // float4 loads per thread
  __shared__ short As[2][BM * LD];                 // [m][k]
  __shared__ short Bs[2][BN * LD];                 // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int mb = blockIdx.y * BM, nb = blockIdx.x * BN;
  const int r = lane & 15, g = lane >> 4;
  const int wm = (w >> 1) * (BM / 2), wn = (w & 1) * (BN / 2);
  const int kbeg = blockIdx.z * kchunk, kend = min(Kd, kbeg + kchunk);
  const bool a_k = sak == 1, b_k = sbk == 1;       // unit stride along k (else along m / n)
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float4 ra[NA], rb[NB];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + 256 * i;
      const int m = a_k ? e / (BK / 4) : (e % (BM / 4)) * 4, k = a_k ? (e % (BK / 4)) * 4 : e / (BM / 4);
      const int gm = mb + m, gk = k0 + k;
      ra[i] = (gm < Mr && gk < kend) ? *reinterpret_cast<const float4*>(A + gm * sam + gk * sak)
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + 256 * i;
      const int n = b_k ? e / (BK / 4) : (e % (BN / 4)) * 4, k = b_k ? (e % (BK / 4)) * 4 : e / (BN / 4);
      const int gn = nb + n, gk = k0 + k;
      rb[i] = (gn < Nc && gk < kend) ? *reinterpret_cast<const float4*>(Bm + gk * sbk + gn * sbn)
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + 256 * i;
      const bf16x4 v = {f2bf(ra[i].x), f2bf(ra[i].y), f2bf(ra[i].z), f2bf(ra[i].w)};
      if (a_k) {
        *reinterpret_cast<bf16x4*>(&As[buf][(e / (BK / 4)) * LD + (e % (BK / 4)) * 4]) = v;
      } else {
        const int m = (e % (BM / 4)) * 4, k = e / (BM / 4);
#pragma unroll
        for (int q = 0; q < 4; ++q) As[buf][(m + q) * LD + k] = v[q];
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + 256 * i;
      const bf16x4 v = {f2bf(rb[i].x), f2bf(rb[i].y), f2bf(rb[i].z), f2bf(rb[i].w)};
      if (b_k) {
        *reinterpret_cast<bf16x4*>(&Bs[buf][(e / (BK / 4)) * LD + (e % (BK / 4)) * 4]) = v;
      } else {
        const int n = (e % (BN / 4)) * 4, k = e / (BN / 4);
#pragma unroll
        for (int q = 0; q < 4; ++q) Bs[buf][(n + q) * LD + k] = v[q];
      }
    }
  };
  int buf = 0;
  if (kbeg < kend) {
    load(kbeg);
    stage(0);
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) load(k0 + BK);  // in flight during the products below
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      bf16x4 a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = *reinterpret_cast<const bf16x4*>(&As[buf][(wm + 16 * i + r) * LD + kk + 4 * g]);
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = *reinterpret_cast<const bf16x4*>(&Bs[buf][(wn + 16 * j + r) * LD + kk + 4 * g]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) stage(buf ^ 1);  // the other buffer: its last readers passed the previous barrier
    __syncthreads();
    buf ^= 1;
  }
  float* P = part ? part + (int64_t)blockIdx.z * Mr * Nc : nullptr;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = mb + wm + 16 * i + 4 * g + q, n = nb + wn + 16 * j + r;
        if (m >= Mr || n >= Nc) continue;
        float v = acc[i][j][q];
        if (P) {
          P[(int64_t)m * Nc + n] = v;
          continue;
        }
        if (accumulate) v += C[m * scm + n * scn];
        if (bias) v += bias[n];
        if (act == 1) {
          Zout[m * scm + n * scn] = v;
          v = gelu_f(v);
        }
        C[m * scm + n * scn] = v;
      }
}

// The split-K sums in the order z = 0, 1, ... and the epilogue of the product.
__global__ void k_splitk_reduce(int Mr, int Nc, int nz, const float* __restrict__ part, float* __restrict__ C,
                                int64_t scm, int64_t scn, const float* __restrict__ bias, int act,
                                float* __restrict__ Zout, int accumulate) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t mn = (int64_t)Mr * Nc;
  if (id >= mn) return;
  const int m = (int)(id / Nc), n = (int)(id % Nc);
  float v = part[id];
  for (int z = 1; z < nz; ++z) v += part[z * mn + id];
  if (accumulate) v += C[m * scm + n * scn];
  if (bias) v += bias[n];
  if (act == 1) {
    Zout[m * scm + n * scn] = v;
    v = gelu_f(v);
  }
  C[m * scm + n * scn] = v;
}

// dY = 2 (Y_net * scale + shift - T) * scale / (rows * cols) in network units, loss partials
__global__ void k_mse_grad(int rows, int cols, const float* __restrict__ Y, const float* __restrict__ T,
                           const float* __restrict__ scale, const float* __restrict__ shift,
                           float* __restrict__ dY, float* __restrict__ loss) {
  __shared__ float sh[256];
  const int64_t n = (int64_t)rows * cols;
  float acc = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % cols);
    const float d = Y[i] * scale[c] + shift[c] - T[i];
    dY[i] = 2.f * d * scale[c] / (float)n;
    acc += d * d;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[blockIdx.x] = sh[0];
}

// acc[0] += scale * sum(parts[0..255]): the epoch's mean loss stays on the device
__global__ void k_loss_acc(const float* __restrict__ parts, float* __restrict__ acc, float scale) {
  __shared__ float sh[256];
  sh[threadIdx.x] = parts[threadIdx.x];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[0] += scale * sh[0];
}

__global__ void k_gelu_back(int64_t n, const float* __restrict__ Z, float* __restrict__ d) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] *= gelu_grad_f(Z[i]);
}

// db[o] = sum_rows d[row][o]: a work group of 64 x 8 threads takes 64
// columns; thread (c, y) sums rows y, y + 8, ... (four accumulators, so that
// loads overlap), and the 8 partial sums are added in a fixed order.
constexpr int COLSUM_ROWS = 8;
__global__ void __launch_bounds__(64 * COLSUM_ROWS) k_colsum(int rows, int cols, const float* __restrict__ d,
                                                              float* __restrict__ out) {
  __shared__ float part[COLSUM_ROWS][64];
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
  const int c = blockIdx.x * 64 + tx;
  float s[4] = {0.f, 0.f, 0.f, 0.f};
  if (c < cols) {
    int r = ty;
    for (; r + 3 * COLSUM_ROWS < rows; r += 4 * COLSUM_ROWS)
#pragma unroll
      for (int k = 0; k < 4; ++k) s[k] += d[(int64_t)(r + k * COLSUM_ROWS) * cols + c];
    for (; r < rows; r += COLSUM_ROWS) s[0] += d[(int64_t)r * cols + c];
  }
  part[ty][tx] = (s[0] + s[1]) + (s[2] + s[3]);
  __syncthreads();
  if (ty == 0 && c < cols) {
    float t = part[0][tx];
#pragma unroll
    for (int k = 1; k < COLSUM_ROWS; ++k) t += part[k][tx];
    out[c] = t;
  }
}

// Adam (Kingma & Ba) on the flat parameter vector
__global__ void k_adam(int64_t n, float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M,
                       float* __restrict__ V, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float g = G[i];
    const float m = b1 * M[i] + (1.f - b1) * g;
    const float v = b2 * V[i] + (1.f - b2) * g * g;
    M[i] = m;
    V[i] = v;
    P[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
  }
}

__global__ void k_gather_rows(int rows, int cols, const int32_t* __restrict__ idx, const float* __restrict__ src,
                              float* __restrict__ dst) {
  const int64_t n = (int64_t)rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / cols), c = (int)(i % cols);
    dst[i] = src[(int64_t)idx[r] * cols + c];
  }
}

// y = y * scale + shift (network units -> target units)
__global__ void k_unscale(int rows, int cols, float* __restrict__ Y, const float* __restrict__ scale,
                          const float* __restrict__ shift) {
  const int64_t n = (int64_t)rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % cols);
    Y[i] = Y[i] * scale[c] + shift[c];
  }
}

// column mean and standard deviation of T [rows][cols] (two passes, FP64 accumulation)
__global__ void k_col_stats(int rows, int cols, const float* __restrict__ T, float* __restrict__ shift,
                            float* __restrict__ scale) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int r = 0; r < rows; ++r) s += T[(int64_t)r * cols + c];
  const double mean = s / rows;
  double q = 0.0;
  for (int r = 0; r < rows; ++r) {
    const double d = T[(int64_t)r * cols + c] - mean;
    q += d * d;
  }
  const double sd = sqrt(q / rows);
  shift[c] = (float)mean;
  scale[c] = (float)(sd > 1e-12 ? sd : 1.0);
}

// Whether an operand suits k_gemm_pipe's 16-byte loads: a unit stride along
// one of its indices, that index's length and the other stride multiples of
// 4, and a 16-byte aligned base.
static bool vec4_operand(const float* p, int64_t s_row, int64_t s_col, int rows, int cols) {
  if (reinterpret_cast<uintptr_t>(p) % 16) return false;
  if (s_col == 1) return cols % 4 == 0 && s_row % 4 == 0;
  if (s_row == 1) return rows % 4 == 0 && s_col % 4 == 0;
  return false;
}

// ws (ws_elems floats): room for split-K partial sums; without it no split.
static int gemm(bool bf16, int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B,
                int64_t sbk, int64_t sbn, float* C, int64_t scm, int64_t scn, const float* bias, int act,
                float* Z, int accumulate, hipStream_t s, float* ws = nullptr, int64_t ws_elems = 0) {
  if (M <= 0 || N <= 0) return RTE_OK;
  if (bf16) {
    if (!vec4_operand(A, sam, sak, M, K) || !vec4_operand(B, sbk, sbn, K, N)) {
      hipLaunchKernelGGL(k_gemm_tiled, dim3((N + GT_BN - 1) / GT_BN, (M + GT_BM - 1) / GT_BM), dim3(256), 0, s, M, N,
                         K, A, sam, sak, B, sbk, sbn, C, scm, scn, bias, act, Z, accumulate);
      RTE_HIP(hipGetLastError());
      return RTE_OK;
    }
    const int64_t t128 = (int64_t)((M + 127) / 128) * ((N + 127) / 128);
    const int64_t t64 = (int64_t)((M + 63) / 64) * ((N + 63) / 64);
    // a long K with few output tiles (the weight gradients: K = rows) is
    // split into chunks of whole 32-deep steps, summed in a fixed order
    int nz = 1, kchunk = K;
    if (ws && t64 < 128 && K >= 2048) {
      nz = (int)std::min<int64_t>({16, K / 512, (256 + t64 - 1) / t64, ws_elems / ((int64_t)M * N)});
      nz = std::max(nz, 1);
      kchunk = ((K + nz - 1) / nz + 31) / 32 * 32;
      nz = (K + kchunk - 1) / kchunk;
    }
    float* part = nz > 1 ? ws : nullptr;
    if (t128 >= 256)
      hipLaunchKernelGGL((k_gemm_pipe<128, 128>), dim3((N + 127) / 128, (M + 127) / 128, nz), dim3(256), 0, s, M, N,
                         K, A, sam, sak, B, sbk, sbn, C, scm, scn, bias, act, Z, accumulate, kchunk, part);
    else
      hipLaunchKernelGGL((k_gemm_pipe<64, 64>), dim3((N + 63) / 64, (M + 63) / 64, nz), dim3(256), 0, s, M, N, K, A,
                         sam, sak, B, sbk, sbn, C, scm, scn, bias, act, Z, accumulate, kchunk, part);
    if (part) {
      const int64_t mn = (int64_t)M * N;
      hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, M, N, nz, part, C,
                         scm, scn, bias, act, Z, accumulate);
    }
  } else {
    const int64_t n = (int64_t)M * N;
    hipLaunchKernelGGL(k_gemm_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, M, N, K, A, sam,
                       sak, B, sbk, sbn, C, scm, scn, bias, act, Z, accumulate);
  }
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

static int mlp_reserve(rte_mlp* m, int rows) {
  if (rows <= m->cap) return RTE_OK;
  for (float* p : m->H) (void)hipFree(p);
  for (float* p : m->Z) (void)hipFree(p);
  (void)hipFree(m->dA);
  (void)hipFree(m->dB);
  (void)hipFree(m->lossbuf);
  m->H.assign(m->dims.size(), nullptr);
  m->Z.assign(m->dims.size(), nullptr);
  int wmax = 0;
  for (int d : m->dims) wmax = std::max(wmax, d);
  for (size_t l = 0; l < m->dims.size(); ++l) {
    if (hipMalloc(&m->H[l], sizeof(float) * (size_t)rows * m->dims[l]) != hipSuccess ||
        hipMalloc(&m->Z[l], sizeof(float) * (size_t)rows * m->dims[l]) != hipSuccess)
      return RTE_ENOMEM;
  }
  if (hipMalloc(&m->dA, sizeof(float) * (size_t)rows * wmax) != hipSuccess ||
      hipMalloc(&m->dB, sizeof(float) * (size_t)rows * wmax) != hipSuccess ||
      hipMalloc(&m->lossbuf, sizeof(float) * 1024) != hipSuccess)
    return RTE_ENOMEM;
  if (!m->ws) {
    m->ws_elems = (int64_t)16 * wmax * wmax;
    if (hipMalloc(&m->ws, sizeof(float) * (size_t)m->ws_elems) != hipSuccess) {
      m->ws_elems = 0;
      return RTE_ENOMEM;
    }
  }
  m->cap = rows;
  return RTE_OK;
}

// forward of `rows` rows already in H[0]; output (network units) in H[L]
static int mlp_forward_ws(rte_mlp* m, int rows, bool bf16, hipStream_t s) {
  const int L = (int)m->dims.size() - 1;
  for (int l = 0; l < L; ++l) {
    const int in = m->dims[l], out = m->dims[l + 1];
    RTE_TRY(gemm(bf16, rows, out, in, m->H[l], in, 1, m->P + m->woff[l], 1, in, m->H[l + 1], out, 1,
                 m->P + m->boff[l], l < L - 1 ? 1 : 0, m->Z[l + 1], 0, s));
  }
  return RTE_OK;
}

// gradient of the MSE loss for targets T (target units); result in m->G
static int mlp_backward_ws(rte_mlp* m, int rows, const float* T, bool bf16, hipStream_t s) {
  const int L = (int)m->dims.size() - 1;
  const int out = m->dims[L];
  hipLaunchKernelGGL(k_mse_grad, dim3(256), dim3(256), 0, s, rows, out, m->H[L], T, m->yscale, m->yshift,
                     m->dA, m->lossbuf);
  float* d = m->dA;     // gradient w.r.t. the current layer's output (pre-activation after gelu_back)
  float* dn = m->dB;
  for (int l = L - 1; l >= 0; --l) {
    const int in = m->dims[l], o = m->dims[l + 1];
    if (l < L - 1) {
      const int64_t n = (int64_t)rows * o;
      hipLaunchKernelGGL(k_gelu_back, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s, n,
                         m->Z[l + 1], d);
    }
    // dW[o][i] = sum_r d[r][o] H[r][i];  db[o] = sum_r d[r][o]
    RTE_TRY(gemm(bf16, o, in, rows, d, 1, o, m->H[l], in, 1, m->G + m->woff[l], in, 1, nullptr, 0, nullptr, 0, s,
                 m->ws, m->ws_elems));
    hipLaunchKernelGGL(k_colsum, dim3((o + 63) / 64), dim3(64 * COLSUM_ROWS), 0, s, rows, o, d, m->G + m->boff[l]);
    if (l > 0)  // d_in[r][i] = sum_o d[r][o] W[o][i]
      RTE_TRY(gemm(bf16, rows, in, o, d, o, 1, m->P + m->woff[l], in, 1, dn, in, 1, nullptr, 0, nullptr, 0, s));
    std::swap(d, dn);
  }
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

// ------------------------------------------------------------------ preconditioner
__global__ void k_mlp_features(int n, int r, int mu_dim, const double* __restrict__ mu,
                               const double* __restrict__ g, int gstride, float* __restrict__ X,
                               double* __restrict__ gnorm, const int32_t* __restrict__ active) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n || (active && !active[b])) return;
  double s = 0.0;
  for (int k = 0; k < r; ++k) s += g[(int64_t)b * gstride + k] * g[(int64_t)b * gstride + k];
  const double nrm = sqrt(s);
  gnorm[b] = nrm;
  const int cols = mu_dim + r;
  for (int k = 0; k < mu_dim; ++k) X[(int64_t)b * cols + k] = (float)mu[(int64_t)b * mu_dim + k];
  for (int k = 0; k < r; ++k)
    X[(int64_t)b * cols + mu_dim + k] = nrm > 0.0 ? (float)(g[(int64_t)b * gstride + k] / nrm) : 0.f;
}

__global__ void k_mlp_coeffs(int n, int r, const float* __restrict__ Y, const double* __restrict__ gnorm,
                             double* __restrict__ c, int cstride, const int32_t* __restrict__ active) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n * r) return;
  const int b = id / r, k = id % r;
  if (active && !active[b]) return;
  c[(int64_t)b * cstride + k] = (double)Y[(int64_t)b * r + k] * gnorm[b];
}

__global__ void k_masks(int n, const int32_t* __restrict__ active, const int32_t* __restrict__ off,
                        int32_t* __restrict__ use_mlp, int32_t* __restrict__ use_rom) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const int a = active ? active[b] : 1;
  use_mlp[b] = a && !off[b];
  use_rom[b] = a && off[b];
}

struct MlpScratch {
  const rte_batch* b = nullptr;
  double *g = nullptr, *c = nullptr, *gn = nullptr;
  int32_t *um = nullptr, *ur = nullptr;
  // comparison of the learned correction with the ROM: the ROM solve's coefficients, the
  // Gram matrix of W_w (of gram_rom), and per-instance sums and counts of
  // ||W_w (c_MLP - c_ROM)|| / ||W_w c_ROM|| over the network's steps
  double *crom = nullptr, *gram = nullptr, *jsum = nullptr;
  int32_t* jcnt = nullptr;
  const rte_rom* gram_rom = nullptr;
  int gram_r = 0;
};
static std::vector<MlpScratch> g_ms;

static MlpScratch* mlp_scratch(const rte_batch* b) {
  for (auto& s : g_ms)
    if (s.b == b) return &s;
  MlpScratch s;
  s.b = b;
  const int n = b->n_inst;
  if (hipMalloc(&s.g, sizeof(double) * n * ROM_GSTRIDE) != hipSuccess ||
      hipMalloc(&s.c, sizeof(double) * n * ROM_GSTRIDE) != hipSuccess ||
      hipMalloc(&s.gn, sizeof(double) * n) != hipSuccess || hipMalloc(&s.um, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&s.ur, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&s.crom, sizeof(double) * n * ROM_GSTRIDE) != hipSuccess ||
      hipMalloc(&s.gram, sizeof(double) * ROM_GSTRIDE * ROM_GSTRIDE) != hipSuccess ||
      hipMalloc(&s.jsum, sizeof(double) * n) != hipSuccess || hipMalloc(&s.jcnt, sizeof(int32_t) * n) != hipSuccess ||
      hipMemset(s.jsum, 0, sizeof(double) * n) != hipSuccess || hipMemset(s.jcnt, 0, sizeof(int32_t) * n) != hipSuccess)
    return nullptr;
  g_ms.push_back(s);
  return &g_ms.back();
}

void mlp_scratch_forget(const rte_batch* b) {
  for (size_t i = 0; i < g_ms.size();) {
    if (g_ms[i].b == b) {
      for (void* p : {(void*)g_ms[i].g, (void*)g_ms[i].c, (void*)g_ms[i].gn, (void*)g_ms[i].um, (void*)g_ms[i].ur,
                      (void*)g_ms[i].crom, (void*)g_ms[i].gram, (void*)g_ms[i].jsum, (void*)g_ms[i].jcnt})
        (void)hipFree(p);
      g_ms.erase(g_ms.begin() + i);
    } else {
      ++i;
    }
  }
}

__global__ void k_gram(int r, int64_t nd, const double* __restrict__ W, double* __restrict__ G);

// jsum[b] += ||W_w d|| / ||W_w c_ROM||, d = c_MLP - c_ROM, with the Gram matrix
// of W_w (so the norms are those of the lifted scalar-flux corrections)
__global__ void k_mlp_rom_diff(int n, int r, const double* __restrict__ gram, const double* __restrict__ cm,
                            const double* __restrict__ cr, int stride, double* __restrict__ jsum,
                            int32_t* __restrict__ jcnt, const int32_t* __restrict__ on) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n || !on[b]) return;
  const double* x = cm + (int64_t)b * stride;
  const double* y = cr + (int64_t)b * stride;
  double dd = 0.0, rr = 0.0;
  for (int i = 0; i < r; ++i) {
    double gd = 0.0, gr = 0.0;
    for (int k = 0; k < r; ++k) {
      gd += gram[i * r + k] * (x[k] - y[k]);
      gr += gram[i * r + k] * y[k];
    }
    dd += (x[i] - y[i]) * gd;
    rr += y[i] * gr;
  }
  if (rr > 0.0) {
    jsum[b] += sqrt(fmax(dd, 0.0) / rr);
    jcnt[b] += 1;
  }
}

int mlp_rom_diff_reset(const rte_batch* b, hipStream_t s) {
  for (auto& m : g_ms)
    if (m.b == b) {
      RTE_HIP(hipMemsetAsync(m.jsum, 0, sizeof(double) * b->n_inst, s));
      RTE_HIP(hipMemsetAsync(m.jcnt, 0, sizeof(int32_t) * b->n_inst, s));
    }
  return RTE_OK;
}

// mean relative difference per instance (0 where the network made no step); syncs s
int mlp_rom_diff_read(const rte_batch* b, std::vector<double>& out, hipStream_t s) {
  out.assign(b->n_inst, 0.0);
  for (auto& m : g_ms)
    if (m.b == b) {
      std::vector<double> sm(b->n_inst);
      std::vector<int32_t> ct(b->n_inst);
      RTE_HIP(hipMemcpyAsync(sm.data(), m.jsum, sizeof(double) * b->n_inst, hipMemcpyDeviceToHost, s));
      RTE_HIP(hipMemcpyAsync(ct.data(), m.jcnt, sizeof(int32_t) * b->n_inst, hipMemcpyDeviceToHost, s));
      RTE_HIP(hipStreamSynchronize(s));
      for (int q = 0; q < b->n_inst; ++q) out[q] = ct[q] ? sm[q] / ct[q] : 0.0;
    }
  return RTE_OK;
}

// z = v + W_w (MLP(mu, g/|g|) |g|) for instances with off[b] == 0, ROMSAD for off[b] == 1.
int mlp_precond(const rte_mlp* cm, const rte_rom* rom, rte_batch* b, const double* sigma_t,
                const double* sigma_s, const double* mu, int mu_dim, const double* v, double* z,
                const int32_t* active, hipStream_t s, int32_t* off) {
  auto* m = const_cast<rte_mlp*>(cm);
  const int n = b->n_inst;
  const int r = rom->r;
  if (m->n_out != r || m->n_in != mu_dim + r) return RTE_EINVAL;
  MlpScratch* sc = mlp_scratch(b);
  if (!sc) return RTE_ENOMEM;
  RTE_TRY(mlp_reserve(m, n));
  hipLaunchKernelGGL(k_masks, dim3((n + 63) / 64), dim3(64), 0, s, n, active, off, sc->um, sc->ur);
  {
    const int st = romsad_apply_internal(rom, b, sigma_t, sigma_s, v, z, sc->ur, s);
    if (st < 0 && st != RTE_ESINGULAR) return st;
  }
  RTE_TRY(rom_project(rom, b, sigma_s, v, sc->g, sc->um, s));
  hipLaunchKernelGGL(k_mlp_features, dim3((n + 63) / 64), dim3(64), 0, s, n, r, mu_dim, mu, sc->g, ROM_GSTRIDE,
                     m->H[0], sc->gn, sc->um);
  RTE_TRY(mlp_forward_ws(m, n, true, s));
  const int L = (int)m->dims.size() - 1;
  hipLaunchKernelGGL(k_unscale, dim3(64), dim3(256), 0, s, n, r, m->H[L], m->yscale, m->yshift);
  hipLaunchKernelGGL(k_mlp_coeffs, dim3((n * r + 255) / 256), dim3(256), 0, s, n, r, m->H[L], sc->gn, sc->c,
                     ROM_GSTRIDE, sc->um);
  RTE_HIP(hipGetLastError());
  // the comparison: the ROM solve's coefficients for the same reduced right-hand side
  if (sc->gram_rom != rom || sc->gram_r != r) {
    hipLaunchKernelGGL(k_gram, dim3(r * r), dim3(256), 0, s, r, rom->ndof, rom->Ww, sc->gram);
    RTE_HIP(hipGetLastError());
    sc->gram_rom = rom;
    sc->gram_r = r;
  }
  RTE_TRY(rom_solve_coeffs(rom, b, sigma_t, sigma_s, sc->g, sc->crom, sc->um, s));
  hipLaunchKernelGGL(k_mlp_rom_diff, dim3((n + 63) / 64), dim3(64), 0, s, n, r, sc->gram, sc->c, sc->crom, ROM_GSTRIDE,
                     sc->jsum, sc->jcnt, sc->um);
  RTE_HIP(hipGetLastError());
  return rom_lift(rom, b, v, sc->c, z, sc->um, s);
}

}  // namespace rte

// ------------------------------------------------------------------ C ABI
using namespace rte;

extern "C" int rte_mlp_create(int n_in, int width, int depth, int n_out, rte_mlp** out) {
  if (n_in < 1 || width < 1 || depth < 1 || n_out < 1 || !out || n_in > 4096 || width > 4096 ||
      depth > 16 || n_out > 4096)
    return RTE_EINVAL;
  auto* m = new rte_mlp();
  m->n_in = n_in;
  m->width = width;
  m->depth = depth;
  m->n_out = n_out;
  m->dims.push_back(n_in);
  for (int d = 0; d < depth; ++d) m->dims.push_back(width);
  m->dims.push_back(n_out);
  int64_t off = 0;
  for (size_t l = 0; l + 1 < m->dims.size(); ++l) {
    m->woff.push_back(off);
    off += (int64_t)m->dims[l] * m->dims[l + 1];
    m->boff.push_back(off);
    off += m->dims[l + 1];
  }
  m->nparams = off;
  if (hipMalloc(&m->P, sizeof(float) * off) != hipSuccess || hipMalloc(&m->M, sizeof(float) * off) != hipSuccess ||
      hipMalloc(&m->V, sizeof(float) * off) != hipSuccess || hipMalloc(&m->G, sizeof(float) * off) != hipSuccess ||
      hipMalloc(&m->yscale, sizeof(float) * n_out) != hipSuccess ||
      hipMalloc(&m->yshift, sizeof(float) * n_out) != hipSuccess) {
    delete m;
    return RTE_ENOMEM;
  }
  RTE_HIP(hipMemset(m->P, 0, sizeof(float) * off));
  RTE_HIP(hipMemset(m->M, 0, sizeof(float) * off));
  RTE_HIP(hipMemset(m->V, 0, sizeof(float) * off));
  std::vector<float> one(n_out, 1.f), zero(n_out, 0.f);
  RTE_HIP(hipMemcpy(m->yscale, one.data(), sizeof(float) * n_out, hipMemcpyHostToDevice));
  RTE_HIP(hipMemcpy(m->yshift, zero.data(), sizeof(float) * n_out, hipMemcpyHostToDevice));
  *out = m;
  return RTE_OK;
}

extern "C" void rte_mlp_destroy(rte_mlp* m) {
  if (!m) return;
  for (void* p : {(void*)m->P, (void*)m->M, (void*)m->V, (void*)m->G, (void*)m->yscale, (void*)m->yshift,
                  (void*)m->dA, (void*)m->dB, (void*)m->lossbuf, (void*)m->ws})
    (void)hipFree(p);
  for (float* p : m->H) (void)hipFree(p);
  for (float* p : m->Z) (void)hipFree(p);
  delete m;
}

extern "C" int64_t rte_mlp_num_params(const rte_mlp* m) { return m ? m->nparams : -1; }

extern "C" int rte_mlp_set_params(rte_mlp* m, const float* host_params, const float* host_scale,
                                  const float* host_shift) {
  if (!m || !host_params) return RTE_EINVAL;
  RTE_HIP(hipMemcpy(m->P, host_params, sizeof(float) * m->nparams, hipMemcpyHostToDevice));
  if (host_scale) RTE_HIP(hipMemcpy(m->yscale, host_scale, sizeof(float) * m->n_out, hipMemcpyHostToDevice));
  if (host_shift) RTE_HIP(hipMemcpy(m->yshift, host_shift, sizeof(float) * m->n_out, hipMemcpyHostToDevice));
  RTE_HIP(hipMemset(m->M, 0, sizeof(float) * m->nparams));
  RTE_HIP(hipMemset(m->V, 0, sizeof(float) * m->nparams));
  m->adam_t = 0;
  return RTE_OK;
}

extern "C" int rte_mlp_get_params(const rte_mlp* m, float* host_params, float* host_scale, float* host_shift) {
  if (!m || !host_params) return RTE_EINVAL;
  RTE_HIP(hipDeviceSynchronize());
  RTE_HIP(hipMemcpy(host_params, m->P, sizeof(float) * m->nparams, hipMemcpyDeviceToHost));
  if (host_scale) RTE_HIP(hipMemcpy(host_scale, m->yscale, sizeof(float) * m->n_out, hipMemcpyDeviceToHost));
  if (host_shift) RTE_HIP(hipMemcpy(host_shift, m->yshift, sizeof(float) * m->n_out, hipMemcpyDeviceToHost));
  return RTE_OK;
}

extern "C" int rte_mlp_forward(rte_mlp* m, const float* X, float* Y, int rows, int dtype, void* stream) {
  if (!m || !X || !Y || rows < 1 || (dtype != RTE_F32 && dtype != RTE_BF16)) return RTE_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  RTE_TRY(mlp_reserve(m, rows));
  RTE_HIP(hipMemcpyAsync(m->H[0], X, sizeof(float) * (size_t)rows * m->n_in, hipMemcpyDeviceToDevice, s));
  RTE_TRY(mlp_forward_ws(m, rows, dtype == RTE_BF16, s));
  const int L = (int)m->dims.size() - 1;
  hipLaunchKernelGGL(k_unscale, dim3(256), dim3(256), 0, s, rows, m->n_out, m->H[L], m->yscale, m->yshift);
  RTE_HIP(hipMemcpyAsync(Y, m->H[L], sizeof(float) * (size_t)rows * m->n_out, hipMemcpyDeviceToDevice, s));
  return RTE_OK;
}

extern "C" int rte_mlp_grad(rte_mlp* m, const float* X, const float* T, int rows, int dtype, float* loss,
                            float* grad, void* stream) {
  if (!m || !X || !T || rows < 1 || (dtype != RTE_F32 && dtype != RTE_BF16)) return RTE_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  RTE_TRY(mlp_reserve(m, rows));
  RTE_HIP(hipMemcpyAsync(m->H[0], X, sizeof(float) * (size_t)rows * m->n_in, hipMemcpyDeviceToDevice, s));
  RTE_TRY(mlp_forward_ws(m, rows, dtype == RTE_BF16, s));
  RTE_TRY(mlp_backward_ws(m, rows, T, dtype == RTE_BF16, s));
  if (grad) RTE_HIP(hipMemcpyAsync(grad, m->G, sizeof(float) * m->nparams, hipMemcpyDeviceToDevice, s));
  if (loss) {
    std::vector<float> lb(256);
    RTE_HIP(hipMemcpyAsync(lb.data(), m->lossbuf, sizeof(float) * 256, hipMemcpyDeviceToHost, s));
    RTE_HIP(hipStreamSynchronize(s));
    double t = 0.0;
    for (float v : lb) t += v;
    *loss = (float)(t / ((double)rows * m->n_out));
  }
  return RTE_OK;
}

extern "C" int rte_mlp_adam_step(rte_mlp* m, const float* grad, float lr, void* stream) {
  if (!m || !grad || !(lr > 0.f)) return RTE_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  m->adam_t++;
  const float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(1024), dim3(256), 0, s, m->nparams, m->P, grad, m->M, m->V, lr, b1, b2, eps, c1,
                     c2);
  RTE_HIP(hipGetLastError());
  return RTE_OK;
}

// SplitMix64 (Steele, Lea and Flood), used for the epoch shuffles
static uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Glorot-uniform weights U(-a, a), a = sqrt(6 / (fan_in + fan_out)), zero biases,
// unit output scale, zero shift and a fresh Adam state.
extern "C" int rte_mlp_init(rte_mlp* m, uint64_t seed) {
  if (!m) return RTE_EINVAL;
  std::vector<float> p(m->nparams, 0.f);
  uint64_t st = seed;
  for (size_t l = 0; l + 1 < m->dims.size(); ++l) {
    const int fi = m->dims[l], fo = m->dims[l + 1];
    const double a = std::sqrt(6.0 / (fi + fo));
    for (int64_t e = 0; e < (int64_t)fi * fo; ++e) {
      const double u = (double)(splitmix64(st) >> 11) * 0x1.0p-53;  // [0, 1)
      p[m->woff[l] + e] = (float)((2.0 * u - 1.0) * a);
    }
  }
  std::vector<float> one(m->n_out, 1.f), zero(m->n_out, 0.f);
  RTE_HIP(hipMemcpy(m->P, p.data(), sizeof(float) * m->nparams, hipMemcpyHostToDevice));
  RTE_HIP(hipMemset(m->M, 0, sizeof(float) * m->nparams));
  RTE_HIP(hipMemset(m->V, 0, sizeof(float) * m->nparams));
  RTE_HIP(hipMemcpy(m->yscale, one.data(), sizeof(float) * m->n_out, hipMemcpyHostToDevice));
  RTE_HIP(hipMemcpy(m->yshift, zero.data(), sizeof(float) * m->n_out, hipMemcpyHostToDevice));
  m->adam_t = 0;
  return RTE_OK;
}

extern "C" int rte_mlp_train(rte_mlp* m, const float* X, const float* T, int n, int epochs, int batch, float lr,
                             uint64_t seed, int standardize, float* loss_hist, void* stream) {
  if (!m || !X || !T || n < 1 || epochs < 1 || batch < 1 || !(lr > 0.f)) return RTE_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  batch = std::min(batch, n);
  RTE_TRY(mlp_reserve(m, batch));
  if (standardize)
    hipLaunchKernelGGL(k_col_stats, dim3((m->n_out + 63) / 64), dim3(64), 0, s, n, m->n_out, T, m->yshift,
                       m->yscale);
  float* Tb = nullptr;
  float* hist = nullptr;
  int32_t* idx = nullptr;
  if (hipMalloc(&Tb, sizeof(float) * (size_t)batch * m->n_out) != hipSuccess ||
      hipMalloc(&idx, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&hist, sizeof(float) * epochs) != hipSuccess) {
    (void)hipFree(Tb);
    (void)hipFree(idx);
    return RTE_ENOMEM;
  }
  std::vector<int32_t> perm(n);
  uint64_t st = seed;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const int nb = n / batch;
  int status = hipMemsetAsync(hist, 0, sizeof(float) * epochs, s) == hipSuccess ? RTE_OK : RTE_EHIP;
  for (int ep = 0; ep < epochs && status == RTE_OK; ++ep) {
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int i = n - 1; i > 0; --i) {  // Fisher-Yates
      const int j = (int)(splitmix64(st) % (uint64_t)(i + 1));
      std::swap(perm[i], perm[j]);
    }
    // the permutation is pageable host memory: the copy completes before it returns
    if (hipMemcpyAsync(idx, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      status = RTE_EHIP;
      break;
    }
    for (int b0 = 0; b0 + batch <= n; b0 += batch) {
      hipLaunchKernelGGL(k_gather_rows, dim3(256), dim3(256), 0, s, batch, m->n_in, idx + b0, X, m->H[0]);
      hipLaunchKernelGGL(k_gather_rows, dim3(256), dim3(256), 0, s, batch, m->n_out, idx + b0, T, Tb);
      if ((status = mlp_forward_ws(m, batch, true, s)) != RTE_OK) break;
      if ((status = mlp_backward_ws(m, batch, Tb, true, s)) != RTE_OK) break;
      m->adam_t++;
      const float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
      hipLaunchKernelGGL(k_adam, dim3(1024), dim3(256), 0, s, m->nparams, m->P, m->G, m->M, m->V, lr, b1, b2, eps,
                         c1, c2);
      hipLaunchKernelGGL(k_loss_acc, dim3(1), dim3(256), 0, s, m->lossbuf, hist + ep,
                         1.f / ((float)batch * m->n_out * nb));
    }
  }
  if (status == RTE_OK && hipGetLastError() != hipSuccess) status = RTE_EHIP;
  if (status == RTE_OK && loss_hist &&
      hipMemcpyAsync(loss_hist, hist, sizeof(float) * epochs, hipMemcpyDeviceToHost, s) != hipSuccess)
    status = RTE_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess && status == RTE_OK) status = RTE_EHIP;
  (void)hipFree(hist);
  (void)hipFree(Tb);
  (void)hipFree(idx);
  return status;
}

// ------------------------------------------------------------------ training data
namespace rte {

// xi_0 = phi / beta; xi_l = (z_{l-1} - sum_{i<l} H[i][l-1] xi_i) / H[l][l-1]
__global__ void k_xi(int l, int w, const InstDev* __restrict__ insts, int64_t total,
                     const double* __restrict__ phi, const double* __restrict__ recZ,
                     const double* __restrict__ recH, const double* __restrict__ beta,
                     const int32_t* __restrict__ jdone, double* __restrict__ xi) {
  const int b = blockIdx.y;
  const InstDev I = insts[b];
  const int64_t nd = (int64_t)I.nx * I.ny * I.nloc;
  const double* Hb = recH + (int64_t)b * (w + 1) * w;
  const bool ok = l == 0 ? beta[b] != 0.0 : (l <= jdone[b] && Hb[l * w + (l - 1)] != 0.0);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nd; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = I.dof_off + e;
    double v = 0.0;
    if (ok) {
      if (l == 0) {
        v = phi[o] / beta[b];
      } else {
        v = recZ[(int64_t)(l - 1) * total + o];
        for (int i = 0; i < l; ++i) v -= Hb[i * w + (l - 1)] * xi[(int64_t)i * total + o];
        v /= Hb[l * w + (l - 1)];
      }
    }
    xi[(int64_t)l * total + o] = v;
  }
}

// d = xi - v
__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ d) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = a[i] - b[i];
}

// Gram matrix of the columns of W [r][nd]
__global__ void k_gram(int r, int64_t nd, const double* __restrict__ W, double* __restrict__ G) {
  __shared__ double sh[256];
  const int i = blockIdx.x / r, k = blockIdx.x % r;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < nd; e += blockDim.x) acc += W[(int64_t)i * nd + e] * W[(int64_t)k * nd + e];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) G[i * r + k] = sh[0];
}

// c = G^{-1} h per instance (G shared, r <= 64), LU with partial pivoting in one thread
__global__ void k_shared_solve(int n, int r, const double* __restrict__ G, const double* __restrict__ h,
                               int stride, double* __restrict__ c) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  double A[64 * 65];
  for (int i = 0; i < r; ++i) {
    for (int k = 0; k < r; ++k) A[i * 65 + k] = G[i * r + k];
    A[i * 65 + r] = h[(int64_t)b * stride + i];
  }
  for (int col = 0; col < r; ++col) {
    int p = col;
    for (int i = col + 1; i < r; ++i)
      if (fabs(A[i * 65 + col]) > fabs(A[p * 65 + col])) p = i;
    if (p != col)
      for (int k = 0; k <= r; ++k) {
        const double t = A[col * 65 + k];
        A[col * 65 + k] = A[p * 65 + k];
        A[p * 65 + k] = t;
      }
    const double d = A[col * 65 + col];
    if (d == 0.0) continue;
    for (int i = col + 1; i < r; ++i) {
      const double f = A[i * 65 + col] / d;
      for (int k = col; k <= r; ++k) A[i * 65 + k] -= f * A[col * 65 + k];
    }
  }
  for (int i = r - 1; i >= 0; --i) {
    double v = A[i * 65 + r];
    for (int k = i + 1; k < r; ++k) v -= A[i * 65 + k] * c[(int64_t)b * stride + k];
    c[(int64_t)b * stride + i] = A[i * 65 + i] != 0.0 ? v / A[i * 65 + i] : 0.0;
  }
}

__global__ void k_snap_rows(int n, int r, int l, int w, int mu_dim, const double* __restrict__ mu,
                            const double* __restrict__ g, const double* __restrict__ c, int stride,
                            const int32_t* __restrict__ jdone, float* __restrict__ X, float* __restrict__ T,
                            int32_t* __restrict__ valid) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  double s = 0.0;
  for (int k = 0; k < r; ++k) s += g[(int64_t)b * stride + k] * g[(int64_t)b * stride + k];
  const double nrm = sqrt(s);
  const int row = b * w + l;
  const int cols = mu_dim + r;
  const bool ok = nrm > 0.0 && l <= jdone[b];
  valid[row] = ok ? 1 : 0;
  for (int k = 0; k < mu_dim; ++k) X[(int64_t)row * cols + k] = (float)mu[(int64_t)b * mu_dim + k];
  for (int k = 0; k < r; ++k) {
    X[(int64_t)row * cols + mu_dim + k] = ok ? (float)(g[(int64_t)b * stride + k] / nrm) : 0.f;
    T[(int64_t)row * r + k] = ok ? (float)(c[(int64_t)b * stride + k] / nrm) : 0.f;
  }
}

}  // namespace rte

extern "C" int rte_mlp_snapshots(const rte_batch* cb, const double* sigma_t, const double* sigma_s,
                                 const double* G, const double* inflow, const rte_rom* rom,
                                 const rte_solve_opts* opts, const double* mu, int mu_dim, float* X, float* T,
                                 int32_t* valid, void* stream) {
  auto* b = const_cast<rte_batch*>(cb);
  if (!b || !sigma_t || !sigma_s || !G || !rom || !opts || !mu || mu_dim < 0 || !X || !T || !valid ||
      rom->is_set() || rom->r < 1 || opts->window < 1 || opts->m < opts->window || !rom_matches(rom, b) ||
      opts->precond == RTE_PC_MLP || b->n_fields > 0)
    return RTE_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  RTE_TRY(validate_cross_sections(b, sigma_t, sigma_s, s));
  const int n = b->n_inst, w = opts->window, r = rom->r;
  Fgmres* f = fgmres_for(b, opts->m);
  if (!f) return RTE_ENOMEM;
  std::vector<rte_solve_stats> stats(n);
  double *phi = nullptr, *xi = nullptr, *d = nullptr, *gq = nullptr, *hq = nullptr, *cq = nullptr, *gram = nullptr;
  int32_t* jd = nullptr;
  const int64_t tot = b->total_dof;
  int st = RTE_OK;
  if (hipMalloc(&phi, sizeof(double) * tot) != hipSuccess || hipMalloc(&xi, sizeof(double) * w * tot) != hipSuccess ||
      hipMalloc(&d, sizeof(double) * tot) != hipSuccess ||
      hipMalloc(&gq, sizeof(double) * n * ROM_GSTRIDE) != hipSuccess ||
      hipMalloc(&hq, sizeof(double) * n * ROM_GSTRIDE) != hipSuccess ||
      hipMalloc(&cq, sizeof(double) * n * ROM_GSTRIDE) != hipSuccess ||
      hipMalloc(&gram, sizeof(double) * r * r) != hipSuccess || hipMalloc(&jd, sizeof(int32_t) * n) != hipSuccess)
    st = RTE_ENOMEM;
  if (st == RTE_OK) {
    SolveCtx c{};
    c.opts = opts;
    c.sigma_t = sigma_t;
    c.sigma_s = sigma_s;
    c.G = G;
    c.inflow = inflow;
    c.rom = rom;
    c.keep = w;
    st = f->solve(c, phi, stats.data(), s);
    if (st > 0) st = RTE_OK;  // unconverged instances still give usable early snapshots
  }
  if (st == RTE_OK && hipMemcpyAsync(jd, f->rec_jdone.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s) != hipSuccess)
    st = RTE_EHIP;
  if (st == RTE_OK) {
    hipLaunchKernelGGL(k_gram, dim3(r * r), dim3(256), 0, s, r, rom->ndof, rom->Ww, gram);
    int64_t maxnd = 0;
    for (const auto& I : b->inst) maxnd = std::max<int64_t>(maxnd, (int64_t)I.nx * I.ny * I.nloc);
    const dim3 grid((unsigned)std::min<int64_t>((maxnd + 255) / 256, 1024), n);
    for (int l = 0; l < w && st == RTE_OK; ++l) {
      hipLaunchKernelGGL(k_xi, grid, dim3(256), 0, s, l, w, b->d_inst, tot, phi, f->recZ, f->recH, f->recBeta, jd, xi);
      const double* vl = f->recV + (int64_t)l * tot;
      hipLaunchKernelGGL(k_sub, dim3(2048), dim3(256), 0, s, tot, xi + (int64_t)l * tot, vl, d);
      st = rom_project(rom, b, sigma_s, vl, gq, nullptr, s);
      if (st == RTE_OK) st = rom_project(rom, b, nullptr, d, hq, nullptr, s, rom->Ww);
      if (st == RTE_OK) {
        hipLaunchKernelGGL(k_shared_solve, dim3((n + 63) / 64), dim3(64), 0, s, n, r, gram, hq, ROM_GSTRIDE, cq);
        hipLaunchKernelGGL(k_snap_rows, dim3((n + 63) / 64), dim3(64), 0, s, n, r, l, w, mu_dim, mu, gq, cq,
                           ROM_GSTRIDE, jd, X, T, valid);
        if (hipGetLastError() != hipSuccess) st = RTE_EHIP;
      }
    }
  }
  if (hipStreamSynchronize(s) != hipSuccess && st == RTE_OK) st = RTE_EHIP;
  for (void* p : {(void*)phi, (void*)xi, (void*)d, (void*)gq, (void*)hq, (void*)cq, (void*)gram, (void*)jd})
    (void)hipFree(p);
  return st;
}
