// Batched form: many independent problems in one persistent launch per phase.
#include "lc_internal.hpp"

using namespace lc;

extern "C" {

lc_status lc_batch_create(int32_t n_problems, const lc_problem_t* problems, lc_batch_t* out) {
    (void)n_problems;
    (void)problems;
    if (out) *out = nullptr;
    set_error("batched form not available in this build");
    return LC_ERR_UNSUPPORTED;
}

lc_status lc_batch_step(lc_batch_t batch, int32_t n_steps, double c, void* stream) {
    (void)batch;
    (void)n_steps;
    (void)c;
    (void)stream;
    set_error("batched form not available in this build");
    return LC_ERR_UNSUPPORTED;
}

lc_status lc_batch_free(lc_batch_t batch) {
    (void)batch;
    return LC_OK;
}

}  // extern "C"
