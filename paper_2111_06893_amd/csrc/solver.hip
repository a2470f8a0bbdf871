// Krylov solve of A u = b (Sec. 2.3).
#include <hip/hip_runtime.h>

#include <string>

#include "context.h"

namespace dgtn {

struct SolverState {};

dgtn_status prepare_levels(dgtn_ctx* c, const dgtn_solve_opts* opts) {
    (void)c;
    (void)opts;
    return DGTN_OK;
}

void plan_solver(dgtn_ctx* c, const dgtn_solve_opts* opts, Layout& lay) {
    (void)c;
    (void)opts;
    (void)lay;
}

dgtn_status bind_solver(dgtn_ctx* c, hipStream_t s) {
    (void)c;
    (void)s;
    return DGTN_OK;
}

}  // namespace dgtn

dgtn_ctx::~dgtn_ctx() { delete solver; }

extern "C" dgtn_status dgtn_solve(dgtn_ctx* c, const dgtn_solve_opts* opts, const double* b, double* u,
                                  dgtn_solve_stats* stats, hipStream_t s) {
    (void)c;
    (void)opts;
    (void)b;
    (void)u;
    (void)stats;
    (void)s;
    dgtn::set_error("solver not built yet");
    return DGTN_EINVAL;
}
