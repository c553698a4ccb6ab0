// ROMSAD reduced-order model (section 4.3) shared by the FGMRES driver and
// the greedy builder.
#pragma once
#include "krylov.h"

struct rte_rom {
  int r = 0, rcap = 0;
  int dim = 2, nx = 0, ny = 0, nloc = 4, n_ord = 0, n_regions = 1;
  int64_t ndof = 0, npsi = 0;
  std::vector<double> ox, w;          // ordinates (original order) for validation
  std::vector<int32_t> region;        // cell -> region
  double* U = nullptr;    // [rcap][n_ord][ndof]
  double* DU = nullptr;   // [rcap][n_ord][ndof]  D_j U_j
  double* W1 = nullptr;   // [rcap][ndof]
  double* Ww = nullptr;   // [rcap][ndof]
  double* AD = nullptr;   // [rcap][rcap]
  double* G = nullptr;    // [n_regions][rcap][rcap]
  double* S = nullptr;    // [n_regions][rcap][rcap]
  int32_t* d_region = nullptr;
  double* d_w = nullptr;  // [w | omega_x | omega_y], original ordinate order
  std::vector<double> oyv;
  double hx = 1.0, hy = 1.0;
  // A ROM set (rte_rom_set_create): per-instance members of a batch with
  // instances of several grids / quadratures; the members are not owned.
  // built on a batch whose cross sections vary inside the cells: the affine
  // pieces G_R, S_R belong to the shape functions (M_R = the shape-weighted
  // mass matrix) instead of regions
  bool fields = false;
  std::vector<const rte_rom*> members;
  std::vector<int32_t> member_of;   // [n_inst of the batch it was made for]
  bool is_set() const { return !members.empty(); }
};

// A view of a single MLP network (defined in mlp.hip)
struct rte_mlp;

namespace rte {

int rom_alloc(rte_rom* rom, const rte_batch* b, int rcap);
void rom_free(rte_rom* rom);
// add column U[r] (already orthonormal, stored at U + r*npsi): compute DU,
// W1, Ww and extend A_D, G_R, S_R.
int rom_add_column(rte_rom* rom, const rte_batch* b, hipStream_t s);
// z = v + W_w A_r(mu)^{-1} W_1^T Sigma_s v for the masked instances.
// gout (nullable, [n][rcap]) receives W_1^T Sigma_s v; cout (nullable) the solve.
// use_factors: solve with the factors that the last rom_singular_check on
// this batch kept (the caller guarantees the same ROM and cross sections;
// singular is then not written).
int romsad_apply_internal(const rte_rom* rom, rte_batch* b, const double* sigma_t,
                          const double* sigma_s, const double* v, double* z, const int32_t* active,
                          hipStream_t s, double* gout = nullptr, double* cout = nullptr,
                          int32_t* singular = nullptr, bool use_factors = false);
bool rom_matches(const rte_rom* rom, const rte_batch* b);
// sing[b] (device [n_inst]) = 1 where the reduced operator A_r(mu_b) is singular;
// the factors of every A_r(mu_b) are kept for romsad_apply_internal(use_factors)
int rom_singular_check(const rte_rom* rom, rte_batch* b, const double* sigma_t, const double* sigma_s,
                       int32_t* sing, hipStream_t s);
// z = v + W_w c for given coefficients c [n][rcap] (no solve)
int rom_lift(const rte_rom* rom, rte_batch* b, const double* v, const double* c, double* z,
             const int32_t* active, hipStream_t s);
// g = W^T Sigma_s v  ([n][ROM_GSTRIDE]); W = W_1 when null, Sigma_s = I when null
int rom_project(const rte_rom* rom, rte_batch* b, const double* sigma_s, const double* v,
                double* g, const int32_t* active, hipStream_t s, const double* W = nullptr);
void rom_scratch_forget(const rte_batch* b);
constexpr int ROM_GSTRIDE = 64;  // stride of per-instance reduced vectors g, c

// c = A_r(mu)^{-1} g per masked instance (g, c [n][ROM_GSTRIDE]), no lift
int rom_solve_coeffs(const rte_rom* rom, rte_batch* b, const double* sigma_t, const double* sigma_s,
                     const double* g, double* c, const int32_t* active, hipStream_t s);
int mlp_rom_diff_reset(const rte_batch* b, hipStream_t s);
int mlp_rom_diff_read(const rte_batch* b, std::vector<double>& out, hipStream_t s);
int mlp_precond(const rte_mlp* mlp, const rte_rom* rom, rte_batch* b, const double* sigma_t,
                const double* sigma_s, const double* mu, int mu_dim, const double* v, double* z,
                const int32_t* active, hipStream_t s, int32_t* fallback_flags);

}  // namespace rte
