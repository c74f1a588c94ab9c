// Complex matrix-core tiles for gfx950.
//
// A complex 16x16 output tile is accumulated by one wavefront with four real
// products per 4-deep slice of the contraction:
//   Cr += Ar Br - Ai Bi,  Ci += Ar Bi + Ai Br
// using v_mfma_f64_16x16x4f64 (binary64) or v_mfma_f32_16x16x4f32 (binary32).
// Operand/result lane layout of both instructions (64 lanes, L = lane):
//   A[i][k]: i = L % 16, k = L / 16          (one value per lane)
//   B[k][j]: j = L % 16, k = L / 16          (one value per lane)
//   C[i][j]: j = L % 16 and, for the r-th of the 4 values of a lane,
//            i = 4 * (L / 16) + r   (binary32)
//            i = L / 16 + 4 * r     (binary64; measured on gfx950)
#pragma once
#include <hip/hip_runtime.h>

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct MF;

template <>
struct MF<double> {
    typedef v4d acc;
    static __device__ __forceinline__ acc mac(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
};

template <>
struct MF<float> {
    typedef v4f acc;
    static __device__ __forceinline__ acc mac(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
};

template <typename T>
struct CAcc {
    typename MF<T>::acc re, im;
    __device__ __forceinline__ void clear() {
        re = MF<T>::zero();
        im = MF<T>::zero();
    }
};

// c += A(i0.., 0..K) * B(0..K, j0..) for a 16x16 tile.  fa(i, k, re, im) and
// fb(k, j, re, im) return operand elements in type T.
template <typename T, int K, typename FA, typename FB>
__device__ __forceinline__ void cgemm_tile(CAcc<T>& c, const FA& fa, const FB& fb, int i0, int j0) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
    for (int k0 = 0; k0 < K; k0 += 4) {
        T ar, ai, br, bi;
        fa(i0 + li, k0 + lk, ar, ai);
        fb(k0 + lk, j0 + li, br, bi);
        c.re = MF<T>::mac(ar, br, c.re);
        c.re = MF<T>::mac(-ai, bi, c.re);
        c.im = MF<T>::mac(ar, bi, c.im);
        c.im = MF<T>::mac(ai, br, c.im);
    }
}

// Row/column of the r-th accumulator value held by this lane.
template <typename T>
__device__ __forceinline__ int tile_row(int r) {
    return sizeof(T) == 8 ? ((threadIdx.x & 63) >> 4) + 4 * r : 4 * ((threadIdx.x & 63) >> 4) + r;
}
__device__ __forceinline__ int tile_col() { return threadIdx.x & 15; }
