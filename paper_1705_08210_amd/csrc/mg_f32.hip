// mg_f32.hip -- instantiation of the VALU min-product kernels for PS_F32.
#include <type_traits>

#include "mgemm_kernels.h"

namespace ps {

namespace {
template <bool kAllowBlocked, class Go>
hipError_t dispatch(int cfg, int acc, Go go) {
    using std::integral_constant;
    constexpr bool kFloat = kAllowBlocked && PS_F32 != PS_U8;
    const bool bl = kFloat && acc == PS_ACC_BLOCKED;
    switch (cfg) {
    case 0:
        if constexpr (kFloat) if (bl) return go(integral_constant<int, 8>(), integral_constant<int, 32>(), std::true_type());
        return go(integral_constant<int, 8>(), integral_constant<int, 32>(), std::false_type());
    case 1:
        if constexpr (kFloat) if (bl) return go(integral_constant<int, 4>(), integral_constant<int, 32>(), std::true_type());
        return go(integral_constant<int, 4>(), integral_constant<int, 32>(), std::false_type());
    case 2:
        if constexpr (kFloat) if (bl) return go(integral_constant<int, 8>(), integral_constant<int, 16>(), std::true_type());
        return go(integral_constant<int, 8>(), integral_constant<int, 16>(), std::false_type());
    default:
        return hipErrorInvalidValue;
    }
}
}  // namespace

// 2-way and 3-way tiles accumulate plainly; PS_ACC_BLOCKED is carried out by
// the field-chunk split (Mg2Launch::nchunks) around them.
hipError_t launch_mg2_f32(const Mg2Launch& a, hipStream_t st) {
    return dispatch<false>(a.cfg, PS_ACC_PLAIN, [&](auto tm, auto bkw, auto bl) {
        return go_mg2<PS_F32, decltype(tm)::value, decltype(bkw)::value, decltype(bl)::value>(a, st);
    });
}

hipError_t launch_mg3_f32(const Mg3Launch& a, hipStream_t st) {
    hipError_t e = dispatch<false>(a.cfg, PS_ACC_PLAIN, [&](auto tm, auto bkw, auto bl) {
        return go_mg3<PS_F32, decltype(tm)::value, decltype(bkw)::value, decltype(bl)::value>(a, st);
    });
    return e == hipSuccess ? go_c3_finish<PS_F32>(a, st) : e;
}

hipError_t launch_mgb_f32(const MgBatchLaunch& a, hipStream_t st) {
    return dispatch<true>(a.cfg, a.acc, [&](auto tm, auto bkw, auto bl) {
        return go_mgb<PS_F32, decltype(tm)::value, decltype(bkw)::value, decltype(bl)::value>(a, st);
    });
}

}  // namespace ps
