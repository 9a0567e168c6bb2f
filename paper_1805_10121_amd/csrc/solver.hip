// Placeholder for the outer loop; replaced by the device-resident solver.
#include "internal.h"

using namespace chase;

extern "C" {

size_t chase_workspace_bytes(const chase_config* cfg) {
  if (!cfg || cfg->n <= 0) return 0;
  const size_t nb = static_cast<size_t>(cfg->nev + cfg->nex);
  return 4 * static_cast<size_t>(cfg->n) * nb * 16;
}

int chase_solve(chase_ctx* ctx, const chase_config*, const void*, int64_t, void*, int64_t, double*,
                double*, chase_stats*) {
  return set_error(ctx, CHASE_EINVAL, "chase_solve: not built");
}

int chase_seq_create(chase_ctx* ctx, const chase_config*, chase_seq**) {
  return set_error(ctx, CHASE_EINVAL, "chase_seq_create: not built");
}
int chase_seq_solve(chase_seq*, const void*, int64_t, double*, double*, chase_stats*) {
  return CHASE_EINVAL;
}
int chase_seq_vectors(chase_seq*, void**, int64_t*) { return CHASE_EINVAL; }
void chase_seq_destroy(chase_seq*) {}

}  // extern "C"
