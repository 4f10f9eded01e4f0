// Batched solves and the launch-parameter autotuner.
#include <cstring>

#include "common.hpp"

namespace jsw {

int solve_batch(int32_t n, Graph *const *graphs, const jsweep_problem *problems, int32_t mode, double tol,
                int32_t max_iter, const jsweep_params *params, jsweep_solve_stats *stats, hipStream_t s) {
    fail(JSWEEP_E_INVALID_ARG, "batched solve not available yet");
}

int autotune(int32_t n, Graph *const *graphs, int32_t mode, jsweep_params *out) {
    fail(JSWEEP_E_INVALID_ARG, "autotune not available yet");
}

}  // namespace jsw
