// mg_f16.hip -- instantiation of the VALU min-product kernels for PS_F16.
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

hipError_t launch_mg2_f16(const Mg2Launch& a, hipStream_t st) {
    return dispatch(a.cfg, [&](auto tm, auto bkw) {
        return go_mg2<PS_F16, decltype(tm)::value, decltype(bkw)::value>(a, st);
    });
}

hipError_t launch_mg3_f16(const Mg3Launch& a, hipStream_t st) {
    hipError_t e = go_mg3_all<PS_F16>(a, [](int cfg, auto go) { return dispatch(cfg, go); }, st);
    return e == hipSuccess ? go_c3_finish<PS_F16>(a, st) : e;
}

hipError_t launch_mgb_f16(const MgBatchLaunch& a, hipStream_t st) {
    return dispatch(a.cfg, [&](auto tm, auto bkw) {
        return go_mgb<PS_F16, decltype(tm)::value, decltype(bkw)::value>(a, st);
    });
}

}  // namespace ps
