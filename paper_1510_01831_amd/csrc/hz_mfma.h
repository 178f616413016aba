// Matrix-core (MFMA) helpers for gfx950, 16x16x4 shapes in FP64 and FP32.
//
// Operand layouts (checked on the device): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; the 16x16 result sits in 4 accumulator slots per
// lane, slot v holding D[row(l, v)][l % 16] with row = l/16 + 4v for FP64 and
// row = 4(l/16) + v for FP32.  A complex tile product uses four real MFMAs:
// Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br.
#pragma once
#include "hz_common.h"

namespace hz {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Mf;
template <> struct Mf<double> {
    using acc = v4d;
    __device__ static inline acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <> struct Mf<float> {
    using acc = v4f;
    __device__ static inline acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int l, int v) { return 4 * (l >> 4) + v; }
};

template <typename T>
__device__ inline typename Mf<T>::acc mf_zero() {
    typename Mf<T>::acc z = {0, 0, 0, 0};
    return z;
}

// complex tile product: (cr, ci) += (ar + i ai)(br + i bi)
template <typename T>
__device__ inline void cmma(T ar, T ai, T br, T bi, typename Mf<T>::acc& cr,
                            typename Mf<T>::acc& ci) {
    cr = Mf<T>::mma(ar, br, cr);
    cr = Mf<T>::mma(-ai, bi, cr);
    ci = Mf<T>::mma(ar, bi, ci);
    ci = Mf<T>::mma(ai, br, ci);
}

}  // namespace hz
