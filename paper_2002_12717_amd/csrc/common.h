// Device helpers shared by the kernels of the G1-G2 library (complex binary64
// arithmetic on double2, Runge-Kutta register update modes).
#pragma once
#include <hip/hip_runtime.h>

typedef double2 cd;

__host__ __device__ __forceinline__ cd cmk(double r, double i) { return make_double2(r, i); }
__host__ __device__ __forceinline__ cd cadd(cd a, cd b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ cd csub(cd a, cd b) { return cmk(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ cd cmul(cd a, cd b) {
    return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ cd cconj(cd a) { return cmk(a.x, -a.y); }
__host__ __device__ __forceinline__ cd cscale(cd a, double s) { return cmk(a.x * s, a.y * s); }
// i * a and -i * a
__host__ __device__ __forceinline__ cd cmul_i(cd a) { return cmk(-a.y, a.x); }
__host__ __device__ __forceinline__ cd cmul_mi(cd a) { return cmk(a.y, -a.x); }
// acc + a * b
__host__ __device__ __forceinline__ cd cfma(cd acc, cd a, cd b) {
    return cmk(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
// acc + a * conj(b)
__host__ __device__ __forceinline__ cd cfma_conjb(cd acc, cd a, cd b) {
    return cmk(fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.y, b.x, fma(-a.x, b.y, acc.y)));
}

// Divergence guard of the Runge-Kutta steps.  div[0] counts the steps begun:
// the host sets it to the number of completed steps before it launches steps,
// and one thread of the first stage of every step advances it, so the last
// stage of a step reads that step's number.  div[1 + c] keeps the first step at
// whose end cluster c (0 for the general basis) failed the guard (~0: never),
// and *flag says whether any cluster did.
struct DivGuard {
    int* flag;
    unsigned long long* div;
};
__device__ __forceinline__ void guard_begin_step(const DivGuard& g) { g.div[0] += 1ull; }
__device__ __forceinline__ void guard_fire(const DivGuard& g, int cluster, unsigned long long step) {
    atomicOr(g.flag, 1);
    atomicMin(g.div + 1 + cluster, step);
}
// The guard itself: a non-finite element, or an occupation n_ii = Im G^<_ii
// far outside [0, 1].
__device__ __forceinline__ bool guard_bad(cd v, bool diagonal) {
    return !(isfinite(v.x) && isfinite(v.y)) || (diagonal && (v.y < -0.5 || v.y > 1.5));
}

// Complex loads and stores from binary64 or binary32 storage; arithmetic is
// always binary64.
__device__ __forceinline__ cd ld_c(const cd* __restrict__ p, long long i) { return p[i]; }
__device__ __forceinline__ cd ld_c(const float2* __restrict__ p, long long i) {
    const float2 v = p[i];
    return cmk((double)v.x, (double)v.y);
}
__device__ __forceinline__ void st_c(cd* __restrict__ p, long long i, cd v) { p[i] = v; }
__device__ __forceinline__ void st_c(float2* __restrict__ p, long long i, cd v) {
    p[i] = make_float2((float)v.x, (float)v.y);
}

// Classical RK4 as a sequence of fused register updates.  With registers y
// (state at t_n), acc (running sum) and a stage input/output pair:
//   RK_RHS   : out = f
//   RK_FIRST : acc = y + cb f ; out = y + cc f          (stage input is y)
//   RK_MID   : acc = acc + cb f ; out = y + cc f
//   RK_LAST  : y = acc + cb f                          (out aliases y)
// with cb = dt/6, dt/3, dt/3, dt/6 and cc = dt/2, dt/2, dt for stages 1..4.
enum { RK_RHS = 0, RK_FIRST = 1, RK_MID = 2, RK_LAST = 3 };

// Streaming (non-temporal) loads and stores: data touched once per kernel,
// kept from displacing operands that are reused from the caches.
__device__ __forceinline__ cd ld_nt(const cd* p) {
    return cmk(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}
__device__ __forceinline__ void st_nt(cd* p, cd v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}
__device__ __forceinline__ void st_nt(float2* p, cd v) {
    __builtin_nontemporal_store((float)v.x, &p->x);
    __builtin_nontemporal_store((float)v.y, &p->y);
}

// The stage output `out` may be binary32 storage (mixed precision); y and acc
// are always binary64.  NT streams y, acc and out past the caches.
template <int MODE, typename TO, bool NT = false>
__device__ __forceinline__ void rk_update(int e, cd f, cd yin_if_first, const cd* __restrict__ y,
                                          cd* __restrict__ acc, TO* __restrict__ out,
                                          double cb, double cc) {
    auto ld = [&](const cd* p) { return NT ? ld_nt(p) : *p; };
    auto st = [&](auto* p, cd v) {
        if (NT) st_nt(p, v);
        else st_c(p, 0, v);
    };
    if (MODE == RK_RHS) {
        st(out + e, f);
    } else if (MODE == RK_FIRST) {
        cd yv = yin_if_first;
        st(acc + e, cmk(fma(cb, f.x, yv.x), fma(cb, f.y, yv.y)));
        st(out + e, cmk(fma(cc, f.x, yv.x), fma(cc, f.y, yv.y)));
    } else if (MODE == RK_MID) {
        cd av = ld(acc + e);
        cd yv = ld(y + e);
        st(acc + e, cmk(fma(cb, f.x, av.x), fma(cb, f.y, av.y)));
        st(out + e, cmk(fma(cc, f.x, yv.x), fma(cc, f.y, yv.y)));
    } else {
        cd av = ld(acc + e);
        st(out + e, cmk(fma(cb, f.x, av.x), fma(cb, f.y, av.y)));
    }
}
