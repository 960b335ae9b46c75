// mfma.hip -- thermometer int8 matrix-core path for integer-level data.
#include "ps_internal.h"

namespace ps {

size_t mfma_workspace_bytes(int64_t n_f, int64_t n_v, int levels) {
    (void)n_f; (void)n_v; (void)levels;
    return 0;
}

hipError_t launch_mfma2(const MfmaLaunch& a, hipStream_t st) {
    (void)a; (void)st;
    return hipErrorNotSupported;
}

}  // namespace ps
