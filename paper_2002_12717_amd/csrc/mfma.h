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
    typename MF<T>::acc vr, vi;
    __device__ __forceinline__ void clear() {
        vr = MF<T>::zero();
        vi = MF<T>::zero();
    }
    __device__ __forceinline__ T re(int r) const { return vr[r]; }
    __device__ __forceinline__ T im(int r) const { return vi[r]; }
    __device__ __forceinline__ void conj() { vi = -vi; }
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
        c.vr = MF<T>::mac(ar, br, c.vr);
        c.vr = MF<T>::mac(-ai, bi, c.vr);
        c.vi = MF<T>::mac(ar, bi, c.vi);
        c.vi = MF<T>::mac(ai, br, c.vi);
    }
}

// The same tile product with four independent accumulation chains
// (Ar Br, Ai Bi, Ar Bi, Ai Br): the four matrix-core instructions of a k-step
// do not depend on each other, so none waits for the previous result.  It
// pays where a wave owns a single output tile; with several tiles per wave the
// two-chain form keeps enough independent work at fewer registers.
template <typename T>
struct CAcc4 {
    typename MF<T>::acc rr, ii, ri, ir;
    __device__ __forceinline__ void clear() {
        rr = MF<T>::zero();
        ii = MF<T>::zero();
        ri = MF<T>::zero();
        ir = MF<T>::zero();
    }
    // c += a b for one complex operand pair of a k-step
    __device__ __forceinline__ void mac(T ar, T ai, T br, T bi) {
        rr = MF<T>::mac(ar, br, rr);
        ii = MF<T>::mac(ai, bi, ii);
        ri = MF<T>::mac(ar, bi, ri);
        ir = MF<T>::mac(ai, br, ir);
    }
    __device__ __forceinline__ T re(int r) const { return rr[r] - ii[r]; }
    __device__ __forceinline__ T im(int r) const { return ri[r] + ir[r]; }
    __device__ __forceinline__ void conj() {
        ri = -ri;
        ir = -ir;
    }
};

template <typename T, int K, typename FA, typename FB>
__device__ __forceinline__ void cgemm_tile(CAcc4<T>& c, const FA& fa, const FB& fb, int i0, int j0) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += 4) {
        T ar, ai, br, bi;
        fa(i0 + li, k0 + lk, ar, ai);
        fb(k0 + lk, j0 + li, br, bi);
        c.rr = MF<T>::mac(ar, br, c.rr);
        c.ii = MF<T>::mac(ai, bi, c.ii);
        c.ri = MF<T>::mac(ar, bi, c.ri);
        c.ir = MF<T>::mac(ai, br, c.ir);
    }
}

// Row/column of the r-th accumulator value held by this lane.
template <typename T>
__device__ __forceinline__ int tile_row(int r) {
    return sizeof(T) == 8 ? ((threadIdx.x & 63) >> 4) + 4 * r : 4 * ((threadIdx.x & 63) >> 4) + r;
}
__device__ __forceinline__ int tile_col() { return threadIdx.x & 15; }
