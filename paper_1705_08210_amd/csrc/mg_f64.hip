// mg_f64.hip -- instantiation of the VALU min-product kernels for PS_F64
// (FP64 data, the paper's double-precision build): 2-way and 3-way.  The
// batched calls do not take FP64.
#include <type_traits>

#include "mgemm_kernels.h"

namespace ps {

namespace {
// Compiled tile configurations, in the order of kValuCfgs.
template <class Go>
hipError_t dispatch(int cfg, Go go) {
    using std::integral_constant;
    switch (cfg) {
    case 0: return go(integral_constant<int, 8>(), integral_constant<int, 32>());
    case 1: return go(integral_constant<int, 4>(), integral_constant<int, 32>());
    case 2: return go(integral_constant<int, 8>(), integral_constant<int, 16>());
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_mg2_f64(const Mg2Launch& a, hipStream_t st) {
    return dispatch(a.cfg, [&](auto tm, auto bkw) {
        return go_mg2<PS_F64, decltype(tm)::value, decltype(bkw)::value>(a, st);
    });
}

hipError_t launch_mg3_f64(const Mg3Launch& a, hipStream_t st) {
    hipError_t e = go_mg3_all<PS_F64>(a, [](int cfg, auto go) { return dispatch(cfg, go); }, st);
    return e == hipSuccess ? go_c3_finish<PS_F64>(a, st) : e;
}

}  // namespace ps
