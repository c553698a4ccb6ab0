// Batch handles, quadrature rules and status strings.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "rte_internal.h"

extern "C" const char* rte_status_string(int s) {
  switch (s) {
    case RTE_OK: return "ok";
    case RTE_EINVAL: return "invalid argument";
    case RTE_EHIP: return "HIP runtime error";
    case RTE_ENOMEM: return "out of device memory";
    case RTE_EBREAKDOWN: return "Krylov breakdown";
    case RTE_ESINGULAR: return "singular reduced operator";
    case RTE_EIO: return "file I/O error";
    case RTE_ENONFINITE: return "non-finite value";
    case RTE_WNOTCONV: return "not converged";
    default: return "unknown status";
  }
}

// Gauss-Legendre nodes by Newton iteration on P_n from the Chebyshev guess
// cos(pi (i - 1/4) / (n + 1/2)), weights 2 / ((1 - x^2) P_n'(x)^2).
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? z : p1;
      double pm = (n == 1) ? 1.0 : p0;
      dp = n * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // one more evaluation of the derivative at the converged node
        p0 = 1.0;
        p1 = z;
        for (int k = 2; k <= n; ++k) {
          double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        pn = (n == 1) ? z : p1;
        pm = (n == 1) ? 1.0 : p0;
        dp = n * (z * pn - pm) / (z * z - 1.0);
        break;
      }
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  if (n % 2) x[n / 2] = 0.0;
}

extern "C" int rte_quadrature_gl(int n, double* ox, double* oy, double* w) {
  if (n < 1 || !ox || !w) return RTE_EINVAL;
  std::vector<double> x, wt;
  gauss_legendre(n, x, wt);
  for (int i = 0; i < n; ++i) {
    ox[i] = x[i];
    if (oy) oy[i] = 0.0;
    w[i] = wt[i] / 2.0;
  }
  return RTE_OK;
}

extern "C" int rte_quadrature_cl(int n_theta, int n_z, int folded, double* ox, double* oy, double* w) {
  if (n_theta < 1 || n_z < 1 || !ox || !oy || !w) return RTE_EINVAL;
  if (folded && (n_z % 2)) return RTE_EINVAL;
  std::vector<double> z, wz;
  gauss_legendre(n_z, z, wz);
  int o = 0;
  for (int j2 = 0; j2 < n_z; ++j2) {
    if (folded && z[j2] <= 0.0) continue;
    double wzj = (folded ? 2.0 : 1.0) * wz[j2] / 2.0;
    double s = std::sqrt(1.0 - z[j2] * z[j2]);
    for (int j1 = 1; j1 <= n_theta; ++j1) {
      double th = 2.0 * j1 * M_PI / n_theta - M_PI / n_theta;
      ox[o] = std::cos(th) * s;
      oy[o] = std::sin(th) * s;
      w[o] = wzj / n_theta;
      ++o;
    }
  }
  return RTE_OK;
}

static int quadrant_of(double ox, double oy) {
  // sgn(0) = +1: a zero component gives no coupling in that direction, so
  // either sweep order along it is a valid upwind order.
  return (ox < 0.0 ? 1 : 0) | (oy < 0.0 ? 2 : 0);
}

extern "C" int rte_batch_create(const rte_instance_desc* desc, int n_inst, rte_batch** out) {
  if (!desc || n_inst < 1 || !out) return RTE_EINVAL;
  auto* b = new rte_batch();
  b->n_inst = n_inst;
  int64_t dof = 0, psi = 0, cells = 0;
  int ord = 0;
  std::vector<int32_t> region;
  for (int k = 0; k < n_inst; ++k) {
    const auto& d = desc[k];
    bool ok = (d.dim == 1 || d.dim == 2) && d.nx >= 1 && d.ny >= 1 && d.n_ord >= 1 &&
              d.omega_x && d.weight && d.region && d.n_regions >= 1 && d.x1 > d.x0 &&
              (d.dim == 1 || (d.omega_y && d.y1 > d.y0)) && (d.dim == 2 || d.ny == 1) &&
              d.nx <= 4096 && d.ny <= 4096 && d.n_ord <= 4096;
    if (!ok) {
      delete b;
      return RTE_EINVAL;
    }
    rte::InstDev I{};
    I.dim = d.dim;
    I.nx = d.nx;
    I.ny = d.ny;
    I.nloc = d.dim == 2 ? 4 : 2;
    I.hx = (d.x1 - d.x0) / d.nx;
    I.hy = d.dim == 2 ? (d.y1 - d.y0) / d.ny : 1.0;
    I.n_ord = d.n_ord;
    I.ord_off = ord;
    I.dof_off = dof;
    I.psi_off = psi;
    I.region_off = (int32_t)cells;
    I.n_regions = d.n_regions;
    int64_t nd = (int64_t)d.nx * d.ny * I.nloc;
    // sort ordinates by quadrant (stable), remembering the original index
    std::vector<int> idx(d.n_ord);
    std::iota(idx.begin(), idx.end(), 0);
    auto quad = [&](int j) {
      return d.dim == 2 ? quadrant_of(d.omega_x[j], d.omega_y[j]) : (d.omega_x[j] < 0.0 ? 1 : 0);
    };
    std::stable_sort(idx.begin(), idx.end(), [&](int p, int q) { return quad(p) < quad(q); });
    for (int qd = 0; qd < 4; ++qd) {
      I.quad_first[qd] = 0;
      I.quad_count[qd] = 0;
    }
    double wsum = 0.0;
    for (int s = 0; s < d.n_ord; ++s) {
      int j = idx[s];
      int qd = quad(j);
      if (I.quad_count[qd] == 0) I.quad_first[qd] = s;
      I.quad_count[qd]++;
      b->ox.push_back(d.omega_x[j]);
      b->oy.push_back(d.dim == 2 ? d.omega_y[j] : 0.0);
      b->w.push_back(d.weight[j]);
      b->perm.push_back(j);
      wsum += d.weight[j];
    }
    for (int c = 0; c < d.nx * d.ny; ++c) {
      if (d.region[c] < 0 || d.region[c] >= d.n_regions) {
        delete b;
        return RTE_EINVAL;
      }
      region.push_back(d.region[c]);
    }
    b->inst.push_back(I);
    b->max_regions = std::max(b->max_regions, d.n_regions);
    b->max_nx = std::max(b->max_nx, d.nx);
    b->max_ny = std::max(b->max_ny, d.ny);
    b->max_ord = std::max(b->max_ord, d.n_ord);
    if (k > 0) {
      const auto& d0 = desc[0];
      bool same = d.dim == d0.dim && d.nx == d0.nx && d.ny == d0.ny && d.n_ord == d0.n_ord &&
                  d.x0 == d0.x0 && d.x1 == d0.x1 && d.y0 == d0.y0 && d.y1 == d0.y1 &&
                  d.n_regions == d0.n_regions;
      for (int j = 0; same && j < d.n_ord; ++j)
        same = d.omega_x[j] == d0.omega_x[j] && d.weight[j] == d0.weight[j] &&
               (d.dim == 1 || d.omega_y[j] == d0.omega_y[j]);
      for (int c = 0; same && c < d.nx * d.ny; ++c) same = d.region[c] == d0.region[c];
      b->uniform = b->uniform && same;
    }
    dof += nd;
    psi += nd * d.n_ord;
    cells += (int64_t)d.nx * d.ny;
    ord += d.n_ord;
    (void)wsum;
  }
  for (int k = 1; k < n_inst; ++k)
    if (desc[k].dim != desc[0].dim) {
      delete b;
      return RTE_EINVAL;  // a batch holds one geometry kind
    }
  b->dim = desc[0].dim;
  b->total_dof = dof;
  b->total_psi = psi;
  b->total_cells = cells;
  auto fail = [&](int code) {
    rte_batch_destroy(b);
    return code;
  };
  if (hipMalloc(&b->d_inst, sizeof(rte::InstDev) * n_inst) != hipSuccess ||
      hipMalloc(&b->d_ox, sizeof(double) * ord) != hipSuccess ||
      hipMalloc(&b->d_oy, sizeof(double) * ord) != hipSuccess ||
      hipMalloc(&b->d_w, sizeof(double) * ord) != hipSuccess ||
      hipMalloc(&b->d_perm, sizeof(int32_t) * ord) != hipSuccess ||
      hipMalloc(&b->d_region, sizeof(int32_t) * cells) != hipSuccess)
    return fail(RTE_ENOMEM);
  if (hipMemcpy(b->d_inst, b->inst.data(), sizeof(rte::InstDev) * n_inst,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_ox, b->ox.data(), sizeof(double) * ord, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_oy, b->oy.data(), sizeof(double) * ord, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_w, b->w.data(), sizeof(double) * ord, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_perm, b->perm.data(), sizeof(int32_t) * ord, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(b->d_region, region.data(), sizeof(int32_t) * cells, hipMemcpyHostToDevice) !=
          hipSuccess)
    return fail(RTE_EHIP);
  // default sweep plans (the autotuner may replace them on first use)
  for (int prec = 0; prec < 2; ++prec) {
    int st = rte::make_plan(b, prec, 8, 256);
    if (st < 0) return fail(st);
  }
  *out = b;
  return RTE_OK;
}

extern "C" void rte_batch_destroy(rte_batch* b) {
  if (!b) return;
  rte::dsa_forget(b);
  rte::fgmres_forget(b);
  rte::rom_scratch_forget(b);
  rte::mlp_scratch_forget(b);
  rte::si_forget(b);
  (void)hipFree(b->d_inst);
  (void)hipFree(b->d_ox);
  (void)hipFree(b->d_oy);
  (void)hipFree(b->d_w);
  (void)hipFree(b->d_perm);
  (void)hipFree(b->d_region);
  (void)hipFree(b->d_part);
  (void)hipFree(b->d_fblk);
  for (auto& p : b->plan) {
    (void)hipFree(p.d_items);
    (void)hipFree(p.d_parts);
  }
  delete b;
}

extern "C" int rte_batch_size(const rte_batch* b) { return b ? b->n_inst : 0; }
extern "C" int64_t rte_batch_ndof(const rte_batch* b, int k) {
  if (!b || k < 0 || k >= b->n_inst) return -1;
  const auto& I = b->inst[k];
  return (int64_t)I.nx * I.ny * I.nloc;
}
extern "C" int64_t rte_batch_offset(const rte_batch* b, int k) {
  if (!b || k < 0 || k >= b->n_inst) return -1;
  return b->inst[k].dof_off;
}
extern "C" int64_t rte_batch_total_dof(const rte_batch* b) { return b ? b->total_dof : -1; }
extern "C" int64_t rte_batch_psi_offset(const rte_batch* b, int k) {
  if (!b || k < 0 || k >= b->n_inst) return -1;
  return b->inst[k].psi_off;
}
extern "C" int64_t rte_batch_total_psi(const rte_batch* b) { return b ? b->total_psi : -1; }
extern "C" int rte_batch_max_regions(const rte_batch* b) { return b ? b->max_regions : -1; }

namespace rte {

int validate_cross_sections(const rte_batch* b, const double* sigma_t, const double* sigma_s, hipStream_t s) {
  const size_t n = (size_t)b->n_inst * b->max_regions;
  std::vector<double> st(n), ss(n);
  RTE_HIP(hipMemcpyAsync(st.data(), sigma_t, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  if (sigma_s) RTE_HIP(hipMemcpyAsync(ss.data(), sigma_s, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  RTE_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < b->n_inst; ++k)
    for (int R = 0; R < b->inst[k].n_regions; ++R) {
      const size_t e = (size_t)k * b->max_regions + R;
      if (!(std::isfinite(st[e]) && st[e] > 0.0)) return RTE_EINVAL;
      if (sigma_s && !(std::isfinite(ss[e]) && ss[e] >= 0.0)) return RTE_EINVAL;
    }
  return RTE_OK;
}

}  // namespace rte
