// Acyclic-network estimator (Eq. (2), Algorithms 2-5): placeholder until the
// recursive-sketch kernels land.
#include "plan.h"

namespace tn {

struct M2Plan {};

int m2_build(tn_plan *, const tn_network *, const std::vector<NetCheck> &) {
  return set_error(TN_ERR_UNSUPPORTED, "acyclic method not built yet");
}
int m2_estimate(tn_plan *, hipStream_t, double *) {
  return set_error(TN_ERR_UNSUPPORTED, "acyclic method not built yet");
}
int m2_get_sketches(tn_plan *, int64_t, int64_t, hipStream_t, double *) {
  return set_error(TN_ERR_UNSUPPORTED, "acyclic method not built yet");
}
void m2_release(tn_plan *p) { p->m2 = nullptr; }

}  // namespace tn
