// Low-order solver entry points shared with the multilevel step (not part of
// the C ABI).
#pragma once

#include "../../include/lc.h"

namespace lc {

// lc_loqd_solve; with defer, a one-workgroup solve queues the copies of its
// convergence report on the stream without waiting for them, and the caller
// checks it with loqd_check_deferred after its next synchronisation of that
// stream (a later solve on the handle waits and checks first).  iters and
// resid are filled only without defer.
lc_status loqd_solve(lc_loqd_t h, double c, double c_dt, const double* kappa, const double* planck,
                     const double* E_prev, const double* F_prev, const double* f_cell, const double* f_face,
                     const double* bnd, double* E_cell, double* E_face, double* F_face, double rtol,
                     int32_t max_iter, int32_t* iters, double* resid, void* stream, bool defer);

// Checks a deferred report: LC_ERR_UNSUPPORTED if a group missed rtol;
// iters (may be NULL) receives the most iterations of any group.
lc_status loqd_check_deferred(lc_loqd_t h, int32_t* iters);

}  // namespace lc
