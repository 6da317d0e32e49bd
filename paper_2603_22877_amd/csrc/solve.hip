// Batched annealed solver (filled in below the per-call path).
#include <hip/hip_runtime.h>

#include "fsmt_internal.hpp"

extern "C" fsmt_status fsmt_solve_batched(const fsmt_xbdd *const *insts, int32_t n_inst, const fsmt_solve_opts *opts,
                                          const fsmt_solve_state *states, void *stream) {
    (void)insts; (void)n_inst; (void)opts; (void)states; (void)stream;
    return fsmt::set_error(FSMT_EUNSUPPORTED, "batched solver not built yet");
}
