// mrhs.hip -- one sketch, many right-hand sides (placeholder until the
// matrix-core solver lands).
#include "csk_mrhs.h"

namespace csk {

size_t mrhs_ws_bytes(int64_t d, int64_t n, int64_t nrhs)
{
    (void)d; (void)n; (void)nrhs;
    return 256;
}

csk_status mrhs_run(const void*, csk_dtype, int64_t, const double*, int64_t, int64_t, int64_t, const double*,
                    int64_t, int64_t, const double*, const double*, double*, int64_t, const double*, int64_t,
                    const csk_solve_opts*, csk_solve_result*, void*, size_t, hipStream_t)
{
    set_error("multi-right-hand-side solver not built");
    return CSK_ERR_UNSUPPORTED;
}

}  // namespace csk
