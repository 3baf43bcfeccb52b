// Population storage codecs.  Every storage keeps the shifted value
// g = f - w_a rho0, so the rest state is exactly zero and the small
// deviations that carry the flow keep their significant bits.
//   F64:  double g, FP64 arithmetic.
//   F32:  float g, FP32 arithmetic.
//   BF16: bfloat16 round-to-nearest-even of g, FP32 arithmetic.
//   F16:  binary16 round-to-nearest-even of g * 2^s, FP32 arithmetic.
// Decoding is exact in every case.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmbp {

struct CodecF64 {
    using T = double;      // stored element
    using R = double;      // arithmetic type
    static constexpr int id = 0;
    __device__ static inline R dec(T v, R) { return v; }
    __device__ static inline T enc(R g, R) { return g; }
};

struct CodecF32 {
    using T = float;
    using R = float;
    static constexpr int id = 1;
    __device__ static inline R dec(T v, R) { return v; }
    __device__ static inline T enc(R g, R) { return g; }
};

struct CodecBF16 {
    using T = uint16_t;    // raw bfloat16 bits
    using R = float;
    static constexpr int id = 2;
    __device__ static inline R dec(T v, R) { return __uint_as_float(uint32_t(v) << 16); }
    __device__ static inline T enc(R g, R) { return __builtin_bit_cast(uint16_t, (__bf16)g); }
};

struct CodecF16 {
    using T = uint16_t;    // raw binary16 bits
    using R = float;
    static constexpr int id = 3;
    // scale argument: 2^s for enc, 2^-s for dec (powers of two: exact)
    __device__ static inline R dec(T v, R inv_scale) {
        return float(__builtin_bit_cast(_Float16, v)) * inv_scale;
    }
    __device__ static inline T enc(R g, R scale) {
        return __builtin_bit_cast(uint16_t, (_Float16)(g * scale));
    }
};

}  // namespace lbmbp
