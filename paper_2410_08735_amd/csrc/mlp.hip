// Learned flexible preconditioner (placeholder until the network lands).
#include "rom.h"

struct rte_mlp {
  int dummy;
};

namespace rte {
int mlp_precond(const rte_mlp*, const rte_rom*, rte_batch*, const double*, const double*,
                const double*, int, const double*, double*, const int32_t*, hipStream_t, int32_t*) {
  return RTE_EINVAL;
}
}  // namespace rte
