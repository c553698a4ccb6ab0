// Batched FP64 Krylov building blocks (Arnoldi with modified Gram-Schmidt,
// Givens least squares, solution update) over a family of per-instance
// vectors packed one after another.
#pragma once
#include "rte_internal.h"

namespace rte {

constexpr int KCHUNK = 4096;   // elements per work group in reductions
constexpr int KTHREADS = 256;
// Krylov::fail codes: an unhappy breakdown (singular least squares at a
// breakdown: the column is dropped), a non-finite estimate (column dropped).
constexpr int KFAIL_BREAKDOWN = 1;
constexpr int KFAIL_NONFINITE = 2;

// A family of per-instance vectors: instance b occupies [off[b], off[b]+len[b]).
struct Space {
  int n = 0;
  std::vector<int64_t> off, len;
  int64_t total = 0, max_len = 0;
  int64_t* d_off = nullptr;
  int64_t* d_len = nullptr;
  int max_chunks() const { return (int)((max_len + KCHUNK - 1) / KCHUNK); }
  int init(const std::vector<int64_t>& lens);
  void release();
};

// Workspace of one batched (F)GMRES cycle of dimension m.
struct Krylov {
  Space sp;
  int m = 0;
  bool flexible = true;
  double* V = nullptr;      // (m + 1) vectors of sp.total
  double* Z = nullptr;      // m vectors (flexible only)
  double* H = nullptr;      // [n][(m + 1) * m] Arnoldi coefficients, H[i * m + j]
  double* R = nullptr;      // [n][(m + 1) * m] rotated copy (upper triangular)
  double* cs = nullptr;     // [n][m]
  double* sn = nullptr;     // [n][m]
  double* g = nullptr;      // [n][m + 1]
  double* y = nullptr;      // [n][m]
  double* partA = nullptr;  // [n][max_chunks]
  double* partB = nullptr;
  double* scal = nullptr;   // [n][8]: 0 beta, 1 tol_abs, 2 est, 3 wnorm_pre, 4 tmp
  int32_t* active = nullptr;  // [n] 1 = iterate in this cycle
  int32_t* jdone = nullptr;   // [n] columns built in this cycle
  int32_t* fail = nullptr;    // [n] 0, KFAIL_BREAKDOWN or KFAIL_NONFINITE (sticky)
  double bt = 1e-14;          // breakdown: H_{j+1,j} <= bt ||H(:, j)||
  int init(const std::vector<int64_t>& lens, int m, bool flexible);
  void release();
  double* v(int j) const { return V + (int64_t)j * sp.total; }
  double* z(int j) const { return Z + (int64_t)j * sp.total; }
};

// out[b] = ||x_b||_2 (device, indexed scal-style with stride), masked
int knorm(const Space& sp, const double* x, double* part, double* out, int out_stride,
          const int32_t* active, hipStream_t s);
// out[b] = sqrt of the sum of part[b][0 .. chunks of len[b]) (chunk partials
// of a squared norm in the layout of knorm)
int knorm_finish(const Space& sp, const double* part, double* out, int out_stride, const int32_t* active,
                 hipStream_t s);
// out[b] = <x_b, y_b>
int kdot(const Space& sp, const double* x, const double* y, double* part, double* out,
         int out_stride, const int32_t* active, hipStream_t s);
// y = x / s[b*stride] (zero if the divisor is zero)
int kscale(const Space& sp, const double* x, const double* sc, int stride, double* y,
           const int32_t* active, hipStream_t s);
// y = a*x + b*y (scalars)
int kaxpby(const Space& sp, double a, const double* x, double bcoef, double* y,
           const int32_t* active, hipStream_t s);
int kcopy(const Space& sp, const double* x, double* y, const int32_t* active, hipStream_t s);
// The operator's partial fluxes (one sweep's per-work-item partial sums, in
// the plan's layout), from which the register-resident Arnoldi step forms
// w = z - (their sum) itself instead of reading a reduced w.
struct PartialSrc {
  const InstPart* parts;  // device, per instance
  const void* part;       // the partial buffer
  int f32;                // partials in FP32 (else FP64)
  const double* z;        // the vector the operator was applied to
};
// Whether arnoldi_mgs takes the register-resident step (one launch, w held in
// registers): instances of up to 48 Ki DoFs, even offsets and lengths.
bool arnoldi_in_registers(const Krylov& K);
// Arnoldi step j: w (= V[j+1] slot) orthogonalised against V[0..j] by MGS,
// H[:, j] filled, w normalised, Givens rotation applied, est and active updated.
// Register-resident where arnoldi_in_registers, else one launch per
// projection.  first_dot_ready: partA already holds the chunk partials of
// <w, v_0> (the operator's reduction produced them).  src (register-resident
// step only, else RTE_EINVAL): w is formed from the operator's partials and
// V[j+1] need not hold it.
int arnoldi_mgs(Krylov& K, int j, hipStream_t s, bool first_dot_ready = false, const PartialSrc* src = nullptr);
// y = R^{-1} g per instance (jdone columns); X += sum_i y_i * basis_i
int kylov_solve_update(Krylov& K, const double* basis, double* X, hipStream_t s);
// start a cycle: V[0] = r / ||r||, g = (beta, 0, ...); the cycle stops at
// max(tol_abs, cycle_rel * beta)
int kstart(Krylov& K, const double* r, const double* tol_abs, hipStream_t s, double cycle_rel = 0.0);
int fill_i32(int32_t* p, int n, int32_t v, hipStream_t s);

}  // namespace rte
