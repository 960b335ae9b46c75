// mg_b1.hip -- the BITS path: binary data (values 0 and 1, the Sorensen case
// of Section 2.3) where min(a, b) = a AND b.  A packing pass turns each
// uint8 row into bits, 32 fields to a word; the VALU min-product kernels then
// run on the packed words with op = popcount(a AND b) (2-way) and
// X_j = V AND v_j (3-way slices).  All sums are exact integers.
#include <type_traits>

#include "mgemm_kernels.h"

namespace ps {

// ---------------------------------------------------------------------------
// Packing.  One thread per output word: 32 bytes in, 4 bytes out (HBM-bound).
// For each byte b, ((b & 0x7f) + 0x7f) | b has bit 7 set iff b != 0, four
// bytes at a time; the four flag bits at 7, 15, 23, 31 are gathered into a
// nibble by one multiply (no two partial products share a bit position, so
// nothing carries into bits 28..31).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t nonzero_nibble(uint32_t x) {
    const uint32_t f = ((((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x) >> 7) & 0x01010101u;
    return (f * 0x10204080u) >> 28;   // bit k of the result = flag of byte k
}

__global__ __launch_bounds__(256) void ps_pack_bits_kernel(const uint8_t* V, int64_t n_f,
                                                           int64_t n_v, int64_t ld, int64_t W,
                                                           uint32_t* P) {
    const int64_t total = n_v * W;
    const bool vec = ((uintptr_t)V % 16 == 0) && (ld % 16 == 0);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = t / W, w = t % W;
        const int64_t q0 = w * kBitsPerWord;
        const uint8_t* src = V + row * ld + q0;
        union { uint4 v[2]; uint32_t u[8]; uint8_t b[32]; } in;
        if (vec && q0 + 32 <= n_f) {
            in.v[0] = *(const uint4*)src;
            in.v[1] = *(const uint4*)(src + 16);
        } else {
            in.v[0] = in.v[1] = make_uint4(0, 0, 0, 0);
            for (int e = 0; e < 32; ++e)
                if (q0 + e < n_f) in.b[e] = src[e];
        }
        uint32_t bits = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) bits |= nonzero_nibble(in.u[k]) << (4 * k);
        P[t] = bits;
    }
}

hipError_t launch_pack_bits(const uint8_t* V, int64_t n_f, int64_t n_v, int64_t ld,
                            uint32_t* P, hipStream_t st) {
    const int64_t W = bits_row_words(n_f);
    const int64_t total = n_v * W;
    if (total == 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(ps_pack_bits_kernel, dim3((unsigned)blocks), dim3(256), 0, st, V, n_f,
                       n_v, ld, W, P);
    return hipGetLastError();
}

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

// a.V is the packed matrix, a.n_f its words per row in use, a.ld its row
// length in words.
hipError_t launch_mg2_b1(const Mg2Launch& a, hipStream_t st) {
    return dispatch(a.cfg, [&](auto tm, auto bkw) {
        return go_mg2<PS_B1, decltype(tm)::value, decltype(bkw)::value>(a, st);
    });
}

hipError_t launch_mg3_b1(const Mg3Launch& a, hipStream_t st) {
    hipError_t e = go_mg3_all<PS_B1>(a, [](int cfg, auto go) { return dispatch(cfg, go); }, st);
    return e == hipSuccess ? go_c3_finish<PS_B1>(a, st) : e;
}

hipError_t launch_c3_finish_int(const Mg3Launch& a, hipStream_t st) {
    return go_c3_finish<PS_B1>(a, st);
}

}  // namespace ps
