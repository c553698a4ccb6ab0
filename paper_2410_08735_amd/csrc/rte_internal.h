// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/rte_romsad.h"

#define RTE_HIP(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      std::fprintf(stderr, "rte: HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, \
                   __LINE__);                                                               \
      return RTE_EHIP;                                                                      \
    }                                                                                       \
  } while (0)

#define RTE_TRY(call)          \
  do {                         \
    int s_ = (call);           \
    if (s_ < 0) return s_;     \
  } while (0)

namespace rte {

// Device-side description of one instance (read by every kernel).
struct InstDev {
  int32_t dim, nx, ny, nloc;
  double hx, hy;
  int32_t n_ord;
  int32_t ord_off;    // offset into the batch's ordinate arrays
  int64_t dof_off;    // offset into packed dof vectors
  int64_t psi_off;    // offset into packed angular-flux vectors
  int32_t region_off; // offset into the packed cell -> region map
  int32_t n_regions;
  int32_t quad_first[4]; // first sorted ordinate of each quadrant (2D) / sign (1D)
  int32_t quad_count[4];
};

// Where one instance's partial flux vectors live in the partial buffer.
struct InstPart {
  int64_t off;   // element offset
  int32_t n;     // number of partial vectors (each ndof long)
  int32_t pad;
};

// One sweep work item: an instance, a quadrant and a block of <= G ordinates
// of that quadrant (indices into the instance's quadrant-sorted ordinate list).
struct SweepItem {
  int32_t inst;
  int32_t quadrant;  // bit 0: Omega_x < 0, bit 1: Omega_y < 0
  int32_t first;     // position in the instance's sorted ordinate list
  int32_t count;
  int64_t part_off;  // element offset of this item's partial flux vector
  int64_t pad;
};

struct Plan {
  int G = 8;       // ordinates per work group (2D); 1D uses one thread per ordinate
  int threads = 256;
  int variant = 0;  // 2D kernel: 0 = diagonal-slot order, 1 = row-slot order with source prefetch
  int opl = 1;      // ordinates per lane (2D): a work item holds G * opl ordinates
  int order = 0;    // work items: 0 = in instance order, each XCD a contiguous run (an
                    // instance's blocks share one L2); 1 = by decreasing cell-ordinates,
                    // dealt round robin over the XCDs (the largest start first)
  std::vector<SweepItem> items;
  std::vector<InstPart> parts;
  SweepItem* d_items = nullptr;
  InstPart* d_parts = nullptr;
  int n_items = 0;
  int64_t part_elems = 0;
  bool tuned = false;
};

}  // namespace rte

struct rte_batch {
  int n_inst = 0;
  int max_regions = 1;
  int max_nx = 0, max_ny = 0, max_ord = 0;
  int64_t total_dof = 0, total_psi = 0;
  std::vector<rte::InstDev> inst;      // host copy
  rte::InstDev* d_inst = nullptr;
  // ordinates packed per instance, sorted by quadrant (sorted order is what
  // kernels see; perm maps sorted position -> original ordinate index)
  std::vector<double> ox, oy, w;
  std::vector<int32_t> perm;
  double *d_ox = nullptr, *d_oy = nullptr, *d_w = nullptr;
  int32_t* d_perm = nullptr;
  int32_t* d_region = nullptr;
  int64_t total_cells = 0;
  // plans for the 2D sweep, per precision (0 = f64, 1 = f32), and the 1D plan
  rte::Plan plan[2];
  // scratch owned by the batch
  void* d_part = nullptr;   // sweep partial fluxes (sized for f64)
  int64_t part_capacity = 0;
  bool uniform = true;      // every instance has the same grid and ordinates
  int dim = 2;
  // bumped whenever a plan's device tables or the partial buffer are
  // (re)allocated: captured graphs that embed their addresses are stale then
  uint64_t gen = 1;
  // cross sections that vary inside the cells (rte_batch_set_fields): the
  // 4x4 mass blocks of n_fields shape functions on every cell of the common
  // grid, [n_fields][ncell][16]; the per-instance cross-section arrays then
  // hold the shapes' coefficients
  int n_fields = 0;
  int64_t field_ncell = 0;
  double* d_fblk = nullptr;
};

namespace rte {

int ensure_partials(rte_batch* b, int64_t elems);

// The mass block of a cell for coefficients theta[0..nf): sum_f theta_f B_f(cell)
// (row-major 4x4, orthonormal basis, dof p + 2 q).
__device__ __forceinline__ void field_block(const double* __restrict__ fblk, int nf, int64_t ncell, int64_t cell,
                                            const double* __restrict__ theta, double out[16]) {
#pragma unroll
  for (int e = 0; e < 16; ++e) out[e] = 0.0;
  for (int f = 0; f < nf; ++f) {
    const double t = theta[f];
    const double* B = fblk + ((int64_t)f * ncell + cell) * 16;
#pragma unroll
    for (int e = 0; e < 16; ++e) out[e] = fma(t, B[e], out[e]);
  }
}
// y = Sigma(theta_b) x on every (masked) instance of a field-mode batch; with
// add, y += Sigma x.  theta: [n_inst][max_regions].
int field_apply(const rte_batch* b, const double* theta, const double* x, double* y, bool add,
                const int32_t* active, hipStream_t s);
// RTE_EINVAL unless every region of every instance has a finite sigma_t > 0
// and a finite sigma_s >= 0 (reads both device arrays on the host; syncs s).
int validate_cross_sections(const rte_batch* b, const double* sigma_t, const double* sigma_s, hipStream_t s);
int make_plan(rte_batch* b, int prec, int G, int threads, int opl = 1);
int set_sweep_plan(rte_batch* b, int prec, int variant, int G, int opl, int threads);
int set_sweep_order(rte_batch* b, int prec, int order);
// prof_units: cell-ordinates processed by this launch (for the event profiler);
// -1 = every instance of the batch; below -1.5 = no profiler events (used
// while a stream is being captured into a graph).  part_buf: where the
// partial scalar fluxes go (plan.part_elems entries of the sweep's precision);
// null = the batch's own buffer.
int sweep_launch(rte_batch* b, int prec, const double* sigma_t, const double* sigma_s,
                 const double* qx, const double* qadd, const double* inflow, double* psi_out,
                 hipStream_t s, const int32_t* active = nullptr, double prof_units = -1.0,
                 void* part_buf = nullptr);

// Event profiler: per-slot HIP event pairs around kernel launches.
enum { PROF_SWEEP_F64 = 0, PROF_SWEEP_F32 = 1, PROF_DSA_OP = 2, PROF_MGS = 3, PROF_ROM = 4,
       PROF_SLOTS = 5 };
bool prof_enabled();
void prof_begin(int slot, hipStream_t s);
void prof_end(int slot, hipStream_t s, double units);
// The index of a slot's most recent record (-1 if none), and a later change of
// a record's units (units < 0: the record is left out of the totals).
int prof_last(int slot);
void prof_set_units(int slot, int idx, double units);
double batch_cell_ordinates(const rte_batch* b, const int32_t* host_mask);
// out = alpha * sum_partials + beta * x + gamma * y   (x, y nullable)
// The same (y unused) with the partial sums of <out, dotv> (<out, out> when
// dotv is null) per instance and chunk of `chunk` DoFs written to
// part[inst * maxc + chunk index], in the order of the Krylov dot-product
// kernel.
int reduce_partials_dot(rte_batch* b, int prec, double alpha, const double* x, double beta, double* out,
                        const double* dotv, double* part, int maxc, int chunk, hipStream_t s,
                        const int32_t* active);
int reduce_partials(rte_batch* b, int prec, double alpha, const double* x, double beta, double* out,
                    hipStream_t s, const int32_t* active = nullptr, const double* y = nullptr,
                    double gamma = 0.0, const void* part_buf = nullptr);
// sigma_s (nullable): time the plans on the operator's sigma_s-scaled source
int autotune_sweep(rte_batch* b, int prec, const double* sigma_t, hipStream_t s,
                   const double* sigma_s = nullptr);
int scalar_flux(rte_batch* b, const double* psi, double* phi, hipStream_t s);
// restart == 0: inner_max V-cycles; restart >= 1: V-cycle-preconditioned
// GMRES(restart) to inner_tol.  prepare = rebuild the sigma-dependent
// multigrid data (cross sections per level, block inverses).
int dsa_apply(rte_batch* b, const double* sigma_t, const double* sigma_s, const double* v, double* z,
              double inner_tol, int inner_max, int restart, const int32_t* active, int32_t* iters,
              hipStream_t s, bool prepare = true, int variant = RTE_DSA_FC);
void dsa_forget(rte_batch* b);
void fgmres_forget(rte_batch* b);
void rom_scratch_forget(const rte_batch* b);
void mlp_scratch_forget(const rte_batch* b);
void si_forget(rte_batch* b);

}  // namespace rte
