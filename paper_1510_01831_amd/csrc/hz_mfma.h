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

// Complex accumulator of one 16x16 output tile.  G3 selects Gauss's
// three-multiplication form: P1 += Ar Br, P2 += Ai Bi, P3 += (Ar + Ai)(Br + Bi),
// then Re = P1 - P2 and Im = P3 - P1 - P2 -- three real MFMAs per complex tile
// step instead of four (normwise error of the same order as the four-product
// form), at the cost of a third accumulator.  Kernels choose per tile shape:
// where the extra accumulator costs a wave of occupancy the four-product form
// is faster.  HZ_GAUSS3=0 turns the three-product form off everywhere.
#ifndef HZ_GAUSS3
#define HZ_GAUSS3 1
#endif
template <typename T, bool G3>
struct CAcc;

template <typename T>
struct CAcc<T, true> {
    using acc = typename Mf<T>::acc;
    acc p1, p2, p3;
    __device__ inline void zero() { p1 = mf_zero<T>(); p2 = mf_zero<T>(); p3 = mf_zero<T>(); }
    __device__ inline void add(T ar, T ai, T br, T bi) {
        p1 = Mf<T>::mma(ar, br, p1);
        p2 = Mf<T>::mma(ai, bi, p2);
        p3 = Mf<T>::mma(ar + ai, br + bi, p3);
    }
    __device__ inline T re(int v) const { return p1[v] - p2[v]; }
    __device__ inline T im(int v) const { return p3[v] - p1[v] - p2[v]; }
};

template <typename T>
struct CAcc<T, false> {
    using acc = typename Mf<T>::acc;
    acc r, i;
    __device__ inline void zero() { r = mf_zero<T>(); i = mf_zero<T>(); }
    __device__ inline void add(T ar, T ai, T br, T bi) { cmma<T>(ar, ai, br, bi, r, i); }
    __device__ inline T re(int v) const { return r[v]; }
    __device__ inline T im(int v) const { return i[v]; }
};

}  // namespace hz
