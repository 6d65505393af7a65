// Compressed operator: H2 in space x MACA across frequencies (placeholder
// until the compressed path is built; the modes are rejected at solve time).
#include "internal.h"

namespace cqm {
size_t h2_workspace_bytes(const Problem&) { return 0; }
void h2_prepare(Problem&, hipStream_t) { throw Error(CQM_EINVAL, "compressed modes are not available in this build"); }
void h2_release(Problem&) {}
template <typename R>
void h2_apply(Problem&, int, int, const cplx<R>*, int64_t, cplx<R>*, int64_t, const int*, hipStream_t) {
  throw Error(CQM_EINVAL, "compressed modes are not available in this build");
}
template void h2_apply<float>(Problem&, int, int, const cf32*, int64_t, cf32*, int64_t, const int*, hipStream_t);
template void h2_apply<double>(Problem&, int, int, const cf64*, int64_t, cf64*, int64_t, const int*, hipStream_t);
void h2_stats(const Problem&, cqm_diag*) {}
}  // namespace cqm
