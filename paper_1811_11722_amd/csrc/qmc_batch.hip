// Batched estimates and the autotuner (filled in below).
#include "qmc_runtime.hpp"

namespace qmc {
struct qmc_plan_extra {};
void plan_release_extra(qmc_plan_s *p) {
    delete p->extra;
    p->extra = nullptr;
}
}  // namespace qmc

using namespace qmc;

extern "C" {
qmc_status qmc_integrate_batch(uint32_t, const qmc_plan_t *, qmc_family, const void *const *,
                               const qmc_batch_opts *, qmc_result *) {
    return fail(QMC_EUNSUPPORTED, "batch not built yet");
}
qmc_status qmc_autotune(qmc_plan_t, qmc_family, const void *, qmc_launch *) {
    return fail(QMC_EUNSUPPORTED, "autotune not built yet");
}
}
