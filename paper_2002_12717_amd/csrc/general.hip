// General-basis G1-G2 kernels (Secs. III.C and IV.C) on the gfx950 matrix cores.
//
// Internally every index runs over nbp = roundup(nb, 16) values; G2 and the
// interaction are nbp^2 x nbp^2 "pair matrices" [(ij),(kl)] built from
// contiguous nbp x nbp row blocks X_ab = X[a][b][:][:].
//
// Right-hand side of the G2 equation of the second-Born selfenergy
// (eq:result_eom_soa), i dG2/dt = [h2, G2] + Psi^-, evaluated as
//     [h2, G2] + Psi^- = D - D^dagger,   D = T^dagger - R,
//     R = G2 h2                    (row action: R_ab = h^T C_ab + C_ab h)
//     T = (G>xG>) W^- (G<xG<)      (Psi^- = T^dagger - T, eq:psi-pm-def)
// which uses the Hermiticity of G2, h2, W^- and the anti-Hermiticity of G^><
// (eq:Gsymm_b, eq:wsymm_b).  T is a two-sided sandwich; it is computed as
//     V_pq = G<^T W^-_pq G<   on row blocks of W^- (kernel gen_vt), stored
//                             transposed: Vt[k][l][p][q] = V_pq[k][l],
//     T^dagger row block ab = conj(G> Vt_ab G>^T)       (kernel gen_main).
// gen_main also accumulates the collision integral eq:eom_gone-I,
//     I = -i sum_{lp} Wc_lp C_lp^T,   Wc_lp[i][k] = w_iklp,
// from the same row blocks.  gen_combine forms -i (D - D^dagger) with an
// LDS-tiled pair transpose and applies the Runge-Kutta register update.
//
// GW (eq:g2-eq-gw-pi) adds Pi - [Pi_lkji]^*, Pi_ijkl = sum_pq h^eps_qjpl G2_ipkq
// (eq:gwpi), evaluated as one (nbp^2)^3 complex GEMM
//     Pi[(i,k)][(j,l)] = sum_(p,q) B[(i,k)][(p,q)] H[(p,q)][(j,l)],
//     B[(i,k)][(p,q)] = G2_ipkq,   H[(p,q)][(j,l)] = h^eps_qjpl,
// with h^eps (eq:gwhcorr) built per (p,q) block as H_pq = i [G<, M_pq],
// M_pq[s][r] = w_sqrp (G^> = G^< - i 1 removes the G<...G< terms).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "ctx.h"
#include "mfma.h"

namespace {

template <int NB>
struct Shape {
    static constexpr int NT = NB / 16;
    static constexpr int TILES = NT * NT;
    static constexpr int WAVES = (TILES % 4 == 0) ? 4 : ((TILES % 3 == 0) ? 3 : 1);
    static constexpr int TPW = TILES / WAVES;
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int LD = NB + 1;
};

template <typename T>
__device__ __forceinline__ void ldc(const cd* p, T& r, T& i) {
    cd v = *p;
    r = (T)v.x;
    i = (T)v.y;
}
template <typename T>
__device__ __forceinline__ void ldc(const float2* p, T& r, T& i) {
    float2 v = *p;
    r = (T)v.x;
    i = (T)v.y;
}
__device__ __forceinline__ void stc(cd* p, double r, double i) { *p = make_double2(r, i); }
__device__ __forceinline__ void stc(float2* p, double r, double i) { *p = make_float2((float)r, (float)i); }

// Work-groups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Logical block b of a grid of g work-groups (g a multiple of 8) is
// mapped so that each XCD owns a contiguous range of logical blocks, which
// keeps neighbouring blocks (adjacent output lines) in one L2.
__device__ __forceinline__ int xcd_block(int b, int g) { return (b & 7) * (g >> 3) + (b >> 3); }

template <typename T, typename S, int NB>
__device__ __forceinline__ void stage_block(const S* __restrict__ src, T* re, T* im) {
    constexpr int LD = Shape<NB>::LD;
    for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
        int r = idx / NB, c = idx % NB;
        T a, b;
        ldc(src + idx, a, b);
        re[r * LD + c] = a;
        im[r * LD + c] = b;
    }
}

// --------------------------------------------------------------------------- K1
// h^HF_ij = h0_ij - i sum_kl w^-_ikjl G^<_lk (eq:h_HF) and G^> = G^< - i 1.
// One work-group per element (ij): coalesced reads of the row (ij) of w^-,
// cross-lane sums and one barrier.  The rows run as extra work-groups of the
// gen_vt launch (K2), which does not depend on them: the memory-bound mean
// field overlaps the matrix-core sandwich.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct HfArgs {
    const cd* whf;   // [i][j][l][k] = w^-_ikjl
    const cd* h0;
    const cd* gl;
    cd* hhf;
    cd* gg;          // G^>
    int nbp, nb;
    double ws;       // switching factor phi(t) of the interaction (1 without a ramp)
};

// Row (ij) of h^HF by one work-group of THREADS threads, of which at most four
// waves sum the row: the order of the sum, and so h^HF to the last bit, does not
// depend on the block size of the launch the rows run in.
template <int THREADS>
__device__ __forceinline__ void hf_row(const HfArgs& a, int ij) {
    constexpr int EFF = THREADS < 256 ? THREADS : 256;
    constexpr int NW = EFF / 64;
    __shared__ double part[2][NW];
    const int nbp = a.nbp, n2 = nbp * nbp;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // row (ij) of whf is stored in the order (l,k) of G^<_lk, so both operands
    // are read contiguously
    const cd* row = a.whf + (size_t)ij * n2;
    double ar[2] = {0.0, 0.0}, ai[2] = {0.0, 0.0};
    for (int m0 = threadIdx.x; threadIdx.x < EFF && m0 < n2; m0 += 4 * EFF) {
        cd w[4], g[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int m = m0 + EFF * u;
            w[u] = m < n2 ? row[m] : make_double2(0.0, 0.0);
            g[u] = m < n2 ? a.gl[m] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ar[u & 1] = fma(w[u].x, g[u].x, fma(-w[u].y, g[u].y, ar[u & 1]));
            ai[u & 1] = fma(w[u].x, g[u].y, fma(w[u].y, g[u].x, ai[u & 1]));
        }
    }
    const double wr = wave_sum(ar[0] + ar[1]), wi = wave_sum(ai[0] + ai[1]);
    if (lane == 0 && wave < NW) {
        part[0][wave] = wr;
        part[1][wave] = wi;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        sr += part[0][w];
        si += part[1][w];
    }
    const cd h = a.h0[ij];
    // h0 - i (sr + i si) = h0 + si - i sr
    a.hhf[ij] = make_double2(h.x + a.ws * si, h.y - a.ws * sr);
    const int i = ij / nbp, j = ij % nbp;
    const cd g = a.gl[ij];
    a.gg[ij] = (i == j && i < a.nb) ? make_double2(g.x, g.y - 1.0) : g;
}

// --------------------------------------------------------------------------- K2
// Right sandwich on row blocks of W: Vt[k][l][p][q] = (G<^T W_pq G<)[k][l].
// Work-groups nvt.. of the launch compute the rows of h^HF (K1).
// Nb = 64 takes eight waves of two tiles; the other sizes take Shape's waves.
template <int NB>
__host__ __device__ constexpr int vt_threads() { return NB == 64 ? 512 : Shape<NB>::THREADS; }

template <typename T, typename S, int NB>
__global__ __launch_bounds__(vt_threads<NB>()) void gen_vt_kernel(const S* __restrict__ wrows,
                                                                 const cd* __restrict__ gl,
                                                                 S* __restrict__ vt, int nvt,
                                                                 HfArgs hf) {
    typedef Shape<NB> SH;
    constexpr int LD = SH::LD;
    if ((int)blockIdx.x >= nvt) {
        hf_row<vt_threads<NB>()>(hf, blockIdx.x - nvt);
        return;
    }
    __shared__ T w_re[NB * LD], w_im[NB * LD], q_re[NB * LD], q_im[NB * LD];
    const int wave = threadIdx.x >> 6;
    const int b0 = xcd_block(blockIdx.x, nvt);
    if constexpr (NB == 64) {
        // Wave w computes the first product's tiles (o, 2h), (o, 2h + 1) and the
        // second product's tiles (2h, o), (2h + 1, o), with o = w / 2, h = w % 2.
        // The G^< operand of both is then the same per lane,
        //   first  A[i][k] = G^<_(k, 16 o + i),  second B[k][j] = G^<_(k, 16 o + j),
        // and is held in registers for the whole launch; W and Q come from LDS,
        // and the next W block is loaded into registers during the products.
        // Each tile's k-steps run in the order of cgemm_tile, so the results
        // equal those of the general path bit for bit.
        constexpr int TH = vt_threads<NB>(), PER = NB * NB / TH;
        const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
        const int o = wave >> 1, h = wave & 1;
        T g_re[NB / 4], g_im[NB / 4];
#pragma unroll
        for (int s4 = 0; s4 < NB / 4; ++s4) ldc(gl + (4 * s4 + lk) * NB + o * 16 + li, g_re[s4], g_im[s4]);
        T pw_re[PER], pw_im[PER];
        auto fetch = [&](int blk) {
#pragma unroll
            for (int q = 0; q < PER; ++q)
                ldc(wrows + (size_t)blk * NB * NB + threadIdx.x + q * TH, pw_re[q], pw_im[q]);
        };
        auto put = [&]() {
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int idx = threadIdx.x + q * TH, r = idx / NB, cc = idx % NB;
                w_re[r * LD + cc] = pw_re[q];
                w_im[r * LD + cc] = pw_im[q];
            }
        };
        if (b0 < NB * NB) {
            fetch(b0);
            put();
        }
        __syncthreads();
        for (int blk = b0; blk < NB * NB; blk += nvt) {
            const int nxt = blk + nvt;
            if (nxt < NB * NB) fetch(nxt);
            CAcc<T> acc[2];
            acc[0].clear();
            acc[1].clear();
#pragma unroll
            for (int s4 = 0; s4 < NB / 4; ++s4) {
                const int k = 4 * s4 + lk;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int j = (2 * h + t) * 16 + li;
                    const T br = w_re[k * LD + j], bi = w_im[k * LD + j];
                    acc[t].vr = MF<T>::mac(g_re[s4], br, acc[t].vr);
                    acc[t].vr = MF<T>::mac(-g_im[s4], bi, acc[t].vr);
                    acc[t].vi = MF<T>::mac(g_re[s4], bi, acc[t].vi);
                    acc[t].vi = MF<T>::mac(g_im[s4], br, acc[t].vi);
                }
            }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int r4 = 0; r4 < 4; ++r4) {
                    const int row = o * 16 + tile_row<T>(r4), col = (2 * h + t) * 16 + tile_col();
                    q_re[row * LD + col] = acc[t].re(r4);
                    q_im[row * LD + col] = acc[t].im(r4);
                }
            __syncthreads();
            acc[0].clear();
            acc[1].clear();
#pragma unroll
            for (int s4 = 0; s4 < NB / 4; ++s4) {
                const int k = 4 * s4 + lk;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int i = (2 * h + t) * 16 + li;
                    const T ar = q_re[i * LD + k], ai = q_im[i * LD + k];
                    acc[t].vr = MF<T>::mac(ar, g_re[s4], acc[t].vr);
                    acc[t].vr = MF<T>::mac(-ai, g_im[s4], acc[t].vr);
                    acc[t].vi = MF<T>::mac(ar, g_im[s4], acc[t].vi);
                    acc[t].vi = MF<T>::mac(ai, g_re[s4], acc[t].vi);
                }
            }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int r4 = 0; r4 < 4; ++r4) {
                    const int row = (2 * h + t) * 16 + tile_row<T>(r4), col = o * 16 + tile_col();
                    stc(vt + (size_t)(row * NB + col) * NB * NB + blk, hf.ws * acc[t].re(r4),
                        hf.ws * acc[t].im(r4));
                }
            if (nxt < NB * NB) put();   // every read of W ended at the barrier above
            __syncthreads();
        }
        return;
    }
    if constexpr (SH::TPW == 1) {
        constexpr int PER = NB * NB / SH::THREADS;
        const int ti = wave / SH::NT, tj = wave % SH::NT;
        const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
        T ga_re[NB / 4], ga_im[NB / 4], gb_re[NB / 4], gb_im[NB / 4];
#pragma unroll
        for (int s4 = 0; s4 < NB / 4; ++s4) {
            ldc(gl + (4 * s4 + lk) * NB + ti * 16 + li, ga_re[s4], ga_im[s4]);
            ldc(gl + (4 * s4 + lk) * NB + tj * 16 + li, gb_re[s4], gb_im[s4]);
        }
        T pw_re[PER], pw_im[PER];
        auto fetch = [&](int blk) {
#pragma unroll
            for (int q = 0; q < PER; ++q)
                ldc(wrows + (size_t)blk * NB * NB + threadIdx.x + q * SH::THREADS, pw_re[q], pw_im[q]);
        };
        if (b0 < NB * NB) fetch(b0);
        for (int blk = b0; blk < NB * NB; blk += nvt) {
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int idx = threadIdx.x + q * SH::THREADS, r = idx / NB, cc = idx % NB;
                w_re[r * LD + cc] = pw_re[q];
                w_im[r * LD + cc] = pw_im[q];
            }
            __syncthreads();
            const int nxt = blk + nvt;
            if (nxt < NB * NB) fetch(nxt);
            CAcc4<T> acc;
            acc.clear();
#pragma unroll
            for (int s4 = 0; s4 < NB / 4; ++s4) {
                const int k = 4 * s4 + lk, j = tj * 16 + li;
                acc.mac(ga_re[s4], ga_im[s4], w_re[k * LD + j], w_im[k * LD + j]);
            }
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                int row = ti * 16 + tile_row<T>(r4), col = tj * 16 + tile_col();
                q_re[row * LD + col] = acc.re(r4);
                q_im[row * LD + col] = acc.im(r4);
            }
            __syncthreads();
            acc.clear();
#pragma unroll
            for (int s4 = 0; s4 < NB / 4; ++s4) {
                const int k = 4 * s4 + lk, i = ti * 16 + li;
                acc.mac(q_re[i * LD + k], q_im[i * LD + k], gb_re[s4], gb_im[s4]);
            }
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                int row = ti * 16 + tile_row<T>(r4), col = tj * 16 + tile_col();
                stc(vt + (size_t)(row * NB + col) * NB * NB + blk, hf.ws * acc.re(r4), hf.ws * acc.im(r4));
            }
            __syncthreads();
        }
        return;
    }
    for (int blk = b0; blk < NB * NB; blk += nvt) {
        stage_block<T, S, NB>(wrows + (size_t)blk * NB * NB, w_re, w_im);
        __syncthreads();
        for (int t = 0; t < SH::TPW; ++t) {
            const int tile = wave * SH::TPW + t, ti = tile / SH::NT, tj = tile % SH::NT;
            CAcc<T> acc;
            acc.clear();
            cgemm_tile<T, NB>(
                acc, [&](int i, int k, T& r, T& m) { ldc(gl + k * NB + i, r, m); },
                [&](int k, int j, T& r, T& m) {
                    r = w_re[k * LD + j];
                    m = w_im[k * LD + j];
                },
                ti * 16, tj * 16);
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                int row = ti * 16 + tile_row<T>(r4), col = tj * 16 + tile_col();
                q_re[row * LD + col] = acc.re(r4);
                q_im[row * LD + col] = acc.im(r4);
            }
        }
        __syncthreads();
        for (int t = 0; t < SH::TPW; ++t) {
            const int tile = wave * SH::TPW + t, ti = tile / SH::NT, tj = tile % SH::NT;
            CAcc<T> acc;
            acc.clear();
            cgemm_tile<T, NB>(
                acc,
                [&](int i, int k, T& r, T& m) {
                    r = q_re[i * LD + k];
                    m = q_im[i * LD + k];
                },
                [&](int k, int j, T& r, T& m) { ldc(gl + k * NB + j, r, m); }, ti * 16, tj * 16);
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                int row = ti * 16 + tile_row<T>(r4), col = tj * 16 + tile_col();
                stc(vt + (size_t)(row * NB + col) * NB * NB + blk, hf.ws * acc.re(r4), hf.ws * acc.im(r4));
            }
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------- K3
// Per row block ab:  D_ab = conj(G> Vt_ab G>^T) - (h^T C_ab + C_ab h),
// and the collision partial  sum_ab Wc_ab C_ab^T  (binary64 across blocks).
// For nb <= 32 the small operators G^> and h^HF are staged in LDS once per
// work-group; for larger blocks they are read through the caches.
template <typename T, int NB, bool STAGE>
struct SmallOps {
    static constexpr int LD = Shape<NB>::LD;
    T g_re[STAGE ? NB * LD : 1], g_im[STAGE ? NB * LD : 1];
    T h_re[STAGE ? NB * LD : 1], h_im[STAGE ? NB * LD : 1];
};

// Nb = 64 runs eight waves of two tiles instead of four waves of four.  In
// gen_main (one work-group per compute unit) that is two waves per SIMD: 0.82
// instead of 1.11 ms per launch in binary64; holding a wave's rows of G> in
// registers as well gained nothing in binary64 and lost in binary32.  In
// gen_heps (two work-groups per compute unit) it is 0.30 instead of 0.36 ms;
// gen_hlad (one work-group per compute unit) takes the same shape.
template <int NB>
struct MainShape : Shape<NB> {
    static constexpr int WAVES = NB == 64 ? 8 : Shape<NB>::WAVES;
    static constexpr int TPW = Shape<NB>::TILES / WAVES;
    static constexpr int THREADS = 64 * WAVES;
};

template <typename T, typename S, int NB>
__global__ __launch_bounds__(MainShape<NB>::THREADS) void gen_main_kernel(
    const cd* __restrict__ g2, const S* __restrict__ vt, const S* __restrict__ wcoll,
    const cd* __restrict__ gg, const cd* __restrict__ hhf, S* __restrict__ dout,
    cd* __restrict__ ipart, double ws) {
    typedef MainShape<NB> SH;
    constexpr int LD = SH::LD;
    using Acc = typename std::conditional<SH::TPW == 1, CAcc4<T>, CAcc<T>>::type;
    constexpr bool STAGE = NB <= 32;
    __shared__ T b0_re[NB * LD], b0_im[NB * LD], b1_re[NB * LD], b1_im[NB * LD];
    __shared__ SmallOps<T, NB, STAGE> ops;
    if constexpr (STAGE) {
        stage_block<T, cd, NB>(gg, ops.g_re, ops.g_im);
        stage_block<T, cd, NB>(hhf, ops.h_re, ops.h_im);
    }
    auto G = [&](int i, int k, T& r, T& m) {   // G^>[i][k]
        if constexpr (STAGE) {
            r = ops.g_re[i * LD + k];
            m = ops.g_im[i * LD + k];
        } else {
            ldc(gg + i * NB + k, r, m);
        }
    };
    auto H = [&](int i, int k, T& r, T& m) {   // h^HF[i][k]
        if constexpr (STAGE) {
            r = ops.h_re[i * LD + k];
            m = ops.h_im[i * LD + k];
        } else {
            ldc(hhf + i * NB + k, r, m);
        }
    };
    const int wave = threadIdx.x >> 6;
    double isum[SH::TPW][2][4];
    for (int t = 0; t < SH::TPW; ++t)
        for (int r4 = 0; r4 < 4; ++r4) isum[t][0][r4] = isum[t][1][r4] = 0.0;

    const int bfirst = xcd_block(blockIdx.x, gridDim.x);
    // Nb <= 32: the next operand blocks are prefetched into registers, so their
    // global loads overlap the matrix-core work of the current phase
    constexpr bool PRE = SH::TPW == 1;
    constexpr int PER = PRE ? NB * NB / SH::THREADS : 1;
    T pv_re[PER], pv_im[PER], pc_re[PER], pc_im[PER];
    auto fetch = [&](auto src, T* re, T* im) {
#pragma unroll
        for (int q = 0; q < PER; ++q) ldc(src + threadIdx.x + q * SH::THREADS, re[q], im[q]);
    };
    auto put = [&](const T* re, const T* im, T* dre, T* dim) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = threadIdx.x + q * SH::THREADS, r = idx / NB, cc = idx % NB;
            dre[r * LD + cc] = re[q];
            dim[r * LD + cc] = im[q];
        }
    };
    if constexpr (PRE)
        if (bfirst < NB * NB) fetch(vt + (size_t)bfirst * NB * NB, pv_re, pv_im);
    for (int blk = bfirst; blk < NB * NB; blk += gridDim.x) {
        if constexpr (PRE) {
            put(pv_re, pv_im, b0_re, b0_im);
            fetch(g2 + (size_t)blk * NB * NB, pc_re, pc_im);
        } else {
            stage_block<T, S, NB>(vt + (size_t)blk * NB * NB, b0_re, b0_im);
        }
        __syncthreads();
        // P = G> Vt_ab
        for (int t = 0; t < SH::TPW; ++t) {
            const int tile = wave * SH::TPW + t, ti = tile / SH::NT, tj = tile % SH::NT;
            Acc acc;
            acc.clear();
            cgemm_tile<T, NB>(
                acc, G,
                [&](int k, int j, T& r, T& m) {
                    r = b0_re[k * LD + j];
                    m = b0_im[k * LD + j];
                },
                ti * 16, tj * 16);
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                int row = ti * 16 + tile_row<T>(r4), col = tj * 16 + tile_col();
                b1_re[row * LD + col] = acc.re(r4);
                b1_im[row * LD + col] = acc.im(r4);
            }
        }
        __syncthreads();
        if constexpr (PRE) {   // C = G2 row block; the next Vt block starts loading
            put(pc_re, pc_im, b0_re, b0_im);
            const int nxt = blk + gridDim.x;
            if (nxt < NB * NB) fetch(vt + (size_t)nxt * NB * NB, pv_re, pv_im);
        } else {
            stage_block<T, cd, NB>(g2 + (size_t)blk * NB * NB, b0_re, b0_im);  // C = G2 row block
        }
        __syncthreads();
        for (int t = 0; t < SH::TPW; ++t) {
            const int tile = wave * SH::TPW + t, ti = tile / SH::NT, tj = tile % SH::NT;
            Acc acc;
            acc.clear();
            // P G>^T
            cgemm_tile<T, NB>(
                acc,
                [&](int i, int k, T& r, T& m) {
                    r = b1_re[i * LD + k];
                    m = b1_im[i * LD + k];
                },
                [&](int k, int j, T& r, T& m) { G(j, k, r, m); }, ti * 16, tj * 16);
            acc.conj();
            // - h^T C
            cgemm_tile<T, NB>(
                acc,
                [&](int i, int k, T& r, T& m) {
                    H(k, i, r, m);
                    r = -r;
                    m = -m;
                },
                [&](int k, int j, T& r, T& m) {
                    r = b0_re[k * LD + j];
                    m = b0_im[k * LD + j];
                },
                ti * 16, tj * 16);
            // - C h
            cgemm_tile<T, NB>(
                acc,
                [&](int i, int k, T& r, T& m) {
                    r = -b0_re[i * LD + k];
                    m = -b0_im[i * LD + k];
                },
                H, ti * 16, tj * 16);
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                int row = ti * 16 + tile_row<T>(r4), col = tj * 16 + tile_col();
                stc(dout + (size_t)blk * NB * NB + row * NB + col, acc.re(r4), acc.im(r4));
            }
            // collision partial: Wc_ab C_ab^T
            Acc ic;
            ic.clear();
            const S* wc = wcoll + (size_t)blk * NB * NB;
            cgemm_tile<T, NB>(
                ic, [&](int i, int k, T& r, T& m) { ldc(wc + i * NB + k, r, m); },
                [&](int k, int j, T& r, T& m) {
                    r = b0_re[j * LD + k];
                    m = b0_im[j * LD + k];
                },
                ti * 16, tj * 16);
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                isum[t][0][r4] += (double)ic.re(r4);
                isum[t][1][r4] += (double)ic.im(r4);
            }
        }
        __syncthreads();
    }
    // collision partials element-major, ipart[(i,j)][part], with the logical
    // (XCD-contiguous) block number as the part: one element's parts are one
    // contiguous read for the reduction, and a cache line of them is written
    // from a single XCD
    for (int t = 0; t < SH::TPW; ++t) {
        const int tile = wave * SH::TPW + t, ti = tile / SH::NT, tj = tile % SH::NT;
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
            int row = ti * 16 + tile_row<T>(r4), col = tj * 16 + tile_col();
            ipart[(size_t)(row * NB + col) * gridDim.x + bfirst] =
                make_double2(ws * isum[t][0][r4], ws * isum[t][1][r4]);
        }
    }
}

// --------------------------------------------------------------------------- K5
// G1 equation eq:eom_gone-2, evaluated by one wavefront per element pair:
// I_ij and I_ji from the collision partials, [h^HF, G^<], the Runge-Kutta
// update of G1 and, at the last stage, the divergence check.  Runs as the
// leading work-groups of the combine launch, beside its G2 work.
struct G1Args {
    const cd* ipart;   // [nbp^2][nparts] partial sums of sum_lp Wc_lp C_lp^T
    int nparts;
    const cd* hhf;
    const cd* gl;      // G^< of the stage
    const cd* y;
    cd* acc;
    cd* out;
    cd* icoll;         // I, written by right-hand-side evaluations
    int nb;
    DivGuard guard;
};

template <int MODE>
__device__ __forceinline__ void g1_update(const G1Args& g, int e, cd comm, cd Iij, cd Iji, int nbp,
                                          double cb, double cc) {
    const cd f = cmul_mi(cadd(comm, cadd(Iij, cconj(Iji))));
    if (MODE == RK_RHS) g.icoll[e] = Iij;
    rk_update<MODE>(e, f, g.gl[e], g.y, g.acc, g.out, cb, cc);
    const int i = e / nbp, j = e % nbp;
    if (MODE == RK_FIRST && e == 0) guard_begin_step(g.guard);   // one thread per launch
    if (MODE == RK_LAST && i < g.nb && guard_bad(g.out[e], i == j)) guard_fire(g.guard, 0, g.guard.div[0]);
}

// The elements (i,j) and (j,i), i <= j: both need I_ij and I_ji, so each
// partial row is read once.
template <int MODE>
__device__ __forceinline__ void g1_pair(const G1Args& g, int i, int j, int lane, int nbp, double cb,
                                        double cc) {
    const int e = i * nbp + j, et = j * nbp + i;
    const cd* pe = g.ipart + (size_t)e * g.nparts;
    const cd* pt = g.ipart + (size_t)et * g.nparts;
    double sr = 0, si = 0, tr = 0, ti = 0;
#pragma unroll 4
    for (int p = lane; p < g.nparts; p += 64) {
        const cd a = pe[p], b = pt[p];
        sr += a.x;
        si += a.y;
        tr += b.x;
        ti += b.y;
    }
    // [h^HF, G^<] at (i,j) and (j,i)
    double cr = 0, ci = 0, dr = 0, di = 0;
    for (int p = lane; p < nbp; p += 64) {
        const cd a = cmul(g.hhf[i * nbp + p], g.gl[p * nbp + j]);
        const cd b = cmul(g.gl[i * nbp + p], g.hhf[p * nbp + j]);
        const cd a2 = cmul(g.hhf[j * nbp + p], g.gl[p * nbp + i]);
        const cd b2 = cmul(g.gl[j * nbp + p], g.hhf[p * nbp + i]);
        cr += a.x - b.x;
        ci += a.y - b.y;
        dr += a2.x - b2.x;
        di += a2.y - b2.y;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    tr = wave_sum(tr);
    ti = wave_sum(ti);
    cr = wave_sum(cr);
    ci = wave_sum(ci);
    dr = wave_sum(dr);
    di = wave_sum(di);
    if (lane != 0) return;
    const cd Iij = make_double2(si, -sr);  // -i (sr + i si)
    const cd Iji = make_double2(ti, -tr);
    g1_update<MODE>(g, e, make_double2(cr, ci), Iij, Iji, nbp, cb, cc);
    if (et != e) g1_update<MODE>(g, et, make_double2(dr, di), Iji, Iij, nbp, cb, cc);
}

// --------------------------------------------------------------------------- K4
// dG2 = -i (D - D^dagger) [+ -i (Pi - conj(Pi_lkji)) for GW], fused RK4 update;
// the G1 equation (K5) on the same launch, in work-groups of its own, so that
// the latency of its partial-sum reads overlaps the G2 streaming.
template <int MODE, typename S, bool GW>
__global__ __launch_bounds__(256) void gen_combine_kernel(const S* __restrict__ D, int n,
                                                         const cd* __restrict__ in,
                                                         const cd* __restrict__ y,
                                                         cd* __restrict__ acc, cd* __restrict__ out,
                                                         const cd* __restrict__ pim, int nbp,
                                                         double cb, double cc, G1Args g1, int ng1) {
    __shared__ double t1r[32][33], t1i[32][33], t2r[32][33], t2i[32][33];
    auto tri = [](int t, int& hi, int& lo) {   // t = hi (hi + 1) / 2 + lo, lo <= hi
        int h = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while ((h + 1) * (h + 2) / 2 <= t) ++h;
        while (h * (h + 1) / 2 > t) --h;
        hi = h;
        lo = t - h * (h + 1) / 2;
    };
    // the first ng1 work-groups: the G1 element pairs (i <= j), one per
    // wavefront; they run beside the G2 tile work instead of after it
    if ((int)blockIdx.x < ng1) {
        const int pair = blockIdx.x * 4 + (threadIdx.x >> 6);
        if (pair < nbp * (nbp + 1) / 2) {
            int j, i;
            tri(pair, j, i);
            g1_pair<MODE>(g1, i, j, threadIdx.x & 63, nbp, cb, cc);
        }
        return;
    }
    // work-group -> tile pair (by, bx), bx <= by, in triangular order; both
    // tiles of the pair are updated from one read of D_(by,bx) and D_(bx,by)
    const int tb = blockIdx.x - ng1;
    int by = (int)((sqrtf(8.0f * (float)tb + 1.0f) - 1.0f) * 0.5f);
    while ((by + 1) * (by + 2) / 2 <= tb) ++by;
    while (by * (by + 1) / 2 > tb) --by;
    const int bx = tb - by * (by + 1) / 2;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        double a, b;
        ldc(D + (size_t)(by * 32 + r) * n + bx * 32 + tx, a, b);
        t1r[r][tx] = a;
        t1i[r][tx] = b;
        ldc(D + (size_t)(bx * 32 + r) * n + by * 32 + tx, a, b);
        t2r[r][tx] = a;
        t2i[r][tx] = b;
    }
    __syncthreads();
    auto update = [&](int row, int col, double zr, double zi) {
        const size_t e = (size_t)row * n + col;
        if (GW) {   // Pi_ijkl and the partner Pi_lkji, both stored at e (see gen_gemm)
            cd p1 = pim[e];
            cd p2 = pim[(size_t)n * n + e];
            zr += p1.x - p2.x;
            zi += p1.y + p2.y;
        }
        cd f = make_double2(zi, -zr);  // -i z
        cd yin = make_double2(0.0, 0.0);
        if (MODE == RK_FIRST) yin = in[e];
        rk_update<MODE>((int)e, f, yin, y, acc, out, cb, cc);
    };
    for (int r = ty; r < 32; r += 8) {
        // D_rc - conj(D_cr) on tile (by, bx) and, off the diagonal, on (bx, by)
        update(by * 32 + r, bx * 32 + tx, t1r[r][tx] - t2r[tx][r], t1i[r][tx] + t2i[tx][r]);
        if (bx != by) update(bx * 32 + r, by * 32 + tx, t2r[r][tx] - t1r[tx][r], t2i[r][tx] + t1i[tx][r]);
    }
}

// --------------------------------------------------------------------------- GW kernels
// H[(p,q)][(j,l)] = h^eps_qjpl = i (G< M_pq - M_pq G<)[j][l], M_pq[s][r] = w_sqrp.
template <typename T, typename S, int NB>
__global__ __launch_bounds__(MainShape<NB>::THREADS) void gen_heps_kernel(const S* __restrict__ wgw,
                                                                     const cd* __restrict__ gl,
                                                                     S* __restrict__ heps, double ws) {
    typedef MainShape<NB> SH;
    constexpr int LD = SH::LD;
    __shared__ T m_re[NB * LD], m_im[NB * LD];
    const int wave = threadIdx.x >> 6;
    for (int blk = blockIdx.x; blk < NB * NB; blk += gridDim.x) {
        stage_block<T, S, NB>(wgw + (size_t)blk * NB * NB, m_re, m_im);
        __syncthreads();
        for (int t = 0; t < SH::TPW; ++t) {
            const int tile = wave * SH::TPW + t, ti = tile / SH::NT, tj = tile % SH::NT;
            CAcc<T> acc;
            acc.clear();
            cgemm_tile<T, NB>(
                acc, [&](int i, int k, T& r, T& m) { ldc(gl + i * NB + k, r, m); },
                [&](int k, int j, T& r, T& m) {
                    r = m_re[k * LD + j];
                    m = m_im[k * LD + j];
                },
                ti * 16, tj * 16);
            cgemm_tile<T, NB>(
                acc,
                [&](int i, int k, T& r, T& m) {
                    r = -m_re[i * LD + k];
                    m = -m_im[i * LD + k];
                },
                [&](int k, int j, T& r, T& m) { ldc(gl + k * NB + j, r, m); }, ti * 16, tj * 16);
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                int row = ti * 16 + tile_row<T>(r4), col = tj * 16 + tile_col();
                // i * acc
                stc(heps + (size_t)blk * NB * NB + row * NB + col, -ws * (double)acc.im(r4),
                    ws * (double)acc.re(r4));
            }
        }
        __syncthreads();
    }
}

// B[(i,k)][(p,q)] = G2_ipkq
// Quasi-Hamiltonians of the two T-matrix ladders, one column-pair block of
// the interaction at a time (G^> = G^< - i):
//   KIND 0, eq:HTPPcorr:  h^pp_ijkl = -sum_pq (G>_ip G>_jq - G<_ip G<_jq) w_pqkl
//                         = [-(G> M G>^T) + (G< M G<^T)]_ij,  M_pq = w_pqkl, block (k,l)
//   KIND 1, eq:HTPHcorr:  h^ph_ijkl = -sum_pq (G>_ip G<_ql - G<_ip G>_ql) w_pjkq
//                         = [-(G> M G<) + (G< M G>)]_il,      M_pq = w_pjkq, block (j,k)
// wl holds the blocks M contiguously (w_pp / w_ph layouts).  The NB x NB
// result (r, c) of block blk is stored at out[(r NB + c) NB^2 + blk], which is
// h^pp as the pair matrix [(ij)][(kl)]; h^ph, the left GEMM operand of
// Lambda^ph_ijkl = sum_pq h^ph_ipql G2_qjkp (eq:lambdaph), is stored with its
// column pair swapped, [(il)][(kj)]: the product runs over K = (q, p), so that
// its right operand G2_qjkp is contiguous along the inner index p.
template <typename T, typename S, int NB, int KIND>
__global__ __launch_bounds__(MainShape<NB>::THREADS) void gen_hlad_kernel(const S* __restrict__ wl,
                                                                     const cd* __restrict__ gl,
                                                                     const cd* __restrict__ gg,
                                                                     S* __restrict__ out, double ws) {
    typedef MainShape<NB> SH;
    constexpr int LD = SH::LD;
    __shared__ T m_re[NB * LD], m_im[NB * LD], q_re[NB * LD], q_im[NB * LD];
    const int wave = threadIdx.x >> 6;
    const int b0 = xcd_block(blockIdx.x, gridDim.x);
    auto Ggt = [&](int i, int k, T& r, T& m) { ldc(gg + i * NB + k, r, m); };   // G>[i][k]
    auto Glt = [&](int i, int k, T& r, T& m) { ldc(gl + i * NB + k, r, m); };   // G<[i][k]
    auto Mop = [&](int k, int j, T& r, T& m) {
        r = m_re[k * LD + j];
        m = m_im[k * LD + j];
    };
    auto Qop = [&](int i, int k, T& r, T& m) {
        r = q_re[i * LD + k];
        m = q_im[i * LD + k];
    };
    for (int blk = b0; blk < NB * NB; blk += gridDim.x) {
        stage_block<T, S, NB>(wl + (size_t)blk * NB * NB, m_re, m_im);
        __syncthreads();
        CAcc<T> acc[SH::TPW];
#pragma unroll
        for (int t = 0; t < SH::TPW; ++t) acc[t].clear();
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            // q = -G> M (half 0) or +G< M (half 1)
#pragma unroll
            for (int t = 0; t < SH::TPW; ++t) {
                const int tile = wave * SH::TPW + t, ti = tile / SH::NT, tj = tile % SH::NT;
                CAcc<T> p;
                p.clear();
                if (half == 0) cgemm_tile<T, NB>(p, Ggt, Mop, ti * 16, tj * 16);
                else cgemm_tile<T, NB>(p, Glt, Mop, ti * 16, tj * 16);
                const T sg = half == 0 ? (T)-1 : (T)1;
#pragma unroll
                for (int r4 = 0; r4 < 4; ++r4) {
                    int row = ti * 16 + tile_row<T>(r4), col = tj * 16 + tile_col();
                    q_re[row * LD + col] = sg * p.re(r4);
                    q_im[row * LD + col] = sg * p.im(r4);
                }
            }
            __syncthreads();
            // acc += q R:  pp R = G>^T (half 0), G<^T (half 1);  ph R = G< (half 0), G> (half 1)
#pragma unroll
            for (int t = 0; t < SH::TPW; ++t) {
                const int tile = wave * SH::TPW + t, ti = tile / SH::NT, tj = tile % SH::NT;
                if (KIND == 0) {
                    if (half == 0) cgemm_tile<T, NB>(acc[t], Qop, [&](int k, int j, T& r, T& m) { Ggt(j, k, r, m); }, ti * 16, tj * 16);
                    else cgemm_tile<T, NB>(acc[t], Qop, [&](int k, int j, T& r, T& m) { Glt(j, k, r, m); }, ti * 16, tj * 16);
                } else {
                    if (half == 0) cgemm_tile<T, NB>(acc[t], Qop, Glt, ti * 16, tj * 16);
                    else cgemm_tile<T, NB>(acc[t], Qop, Ggt, ti * 16, tj * 16);
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int t = 0; t < SH::TPW; ++t) {
            const int tile = wave * SH::TPW + t, ti = tile / SH::NT, tj = tile % SH::NT;
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                int row = ti * 16 + tile_row<T>(r4), col = tj * 16 + tile_col();
                stc(out + (size_t)(row * NB + col) * NB * NB + (KIND == 1 ? (blk % NB) * NB + blk / NB : blk),
                    ws * acc[t].re(r4), ws * acc[t].im(r4));
            }
        }
    }
}

// Permuted copy of G2 as a GEMM operand (the left one of the GW product, the
// right one of the ladder products):
//   MODE 0 (GW):   b[(i,k)][(p,q)] = G2_ipkq
//   MODE 1 (TPP):  b[(p,q)][(k,l)] = G2_pqkl
//   MODE 2 (TPH):  b[(q,p)][(j,k)] = G2_qjkp   (the TPH product runs over K = (q, p))
// The binary64 products read G2 in place, so these copies are made for the
// binary32 operands only.
template <typename S, int MODE>
__global__ __launch_bounds__(256) void gen_bmat_kernel(const cd* __restrict__ g2, S* __restrict__ b,
                                                      int nbp) {
    const size_t n4 = (size_t)nbp * nbp * nbp * nbp;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n4;
         e += (size_t)gridDim.x * blockDim.x) {
        size_t x3 = e % nbp, t = e / nbp;
        size_t x2 = t % nbp;
        t /= nbp;
        size_t x1 = t % nbp, x0 = t / nbp;
        size_t src;
        if (MODE == 0) src = ((x0 * nbp + x2) * nbp + x1) * nbp + x3;        // (i,k,p,q) <- G2_ipkq
        else if (MODE == 1) src = e;
        else src = ((x0 * nbp + x2) * nbp + x3) * nbp + x1;                  // (q,p,j,k) <- G2_qjkp
        cd v = g2[src];
        stc(b + e, v.x, v.y);
    }
}

// Pi[(i,k)][(j,l)] = sum_K B[(i,k)][K] H[K][(j,l)], stored as pim[i][j][k][l].
// 64x64 output tile per work-group, four waves of 32x32, K staged in slices of 16.
// With T = float the products are accumulated in binary32 over 64-deep chunks
// and the chunk sums are added in binary64 (chunked compensated summation).
// OUT selects the epilogue:
//   0 (GW):  pim[i][j][k][l] = C[(i,k)][(j,l)], and the same value at
//            pim[n^2 + ((l nbp + k) nbp + j) nbp + i]          (binary64 buffer)
//   1 (TPP): D[(i,j)][(k,l)] += C[(i,j)][(k,l)]               (D in storage S)
//   2 (TPH): D[(i,j)][(k,l)] += C[(i,l)][(j,k)]
// AG2 reads the GW operand B[(i,k)][(p,q)] = G2_ipkq in place from the binary64
// G2 instead of a permuted copy: within a K slice p = k0 / nbp is uniform and q
// runs over 16 consecutive values, so the loads keep their 256-byte rows.
// BG2T reads the TPH operand B[(q,p)][(j,k)] = G2_qjkp in place, at
// q nbp^3 + (j nbp + k) nbp + p: a K slice is one q and 16 consecutive p, so a
// column's 16 values are one 256-byte row; they are stored to LDS transposed.
template <typename T, typename S, int OUT, bool AG2 = false, bool BG2T = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void gen_gemm_kernel(const S* __restrict__ A, const S* __restrict__ B,
                                                      void* __restrict__ dst, int n, int nbp) {
    constexpr int KS = 16;                    // depth of one staged K slice
    constexpr int PER = 64 * KS / 256;          // elements of A (and of B) per thread and slice
    // three real products per complex multiply-add instead of four,
    //   Re = Ar Br - Ai Bi,  Im = (Ar + Ai)(Br + Bi) - Ar Br - Ai Bi;
    // the operand sums are formed from the values read for the first two
    // products (one add per operand and MFMA step) rather than staged in LDS.
    // The slices are kept as interleaved complex values, so an operand pair is
    // one 16-byte (binary64) or 8-byte LDS access.  Measured per Nb = 64
    // launch in binary64: split re/im arrays with staged sums (51 KB) 6.85 ms,
    // without the sums (34 KB) 6.42 ms, interleaved (34 KB) 6.27 ms; a 32-deep
    // slice or a second LDS buffer was slower
    typedef typename std::conditional<sizeof(T) == 8, double2, float2>::type CT;
    __shared__ CT a_c[64][KS + 1];
    __shared__ CT b_c[KS][65];
    const int bm = blockIdx.y * 64, bn = blockIdx.x * 64;
    const int wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    double accd[2][2][2][4];
    typename MF<T>::acc p1[2][2], p2[2][2], p3[2][2];   // Ar Br, Ai Bi, (Ar + Ai)(Br + Bi)
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            p1[a][b] = p2[a][b] = p3[a][b] = MF<T>::zero();
            for (int r4 = 0; r4 < 4; ++r4) accd[a][b][0][r4] = accd[a][b][1][r4] = 0.0;
        }
    // the next K slice is loaded into registers while the current one runs
    T pa_re[PER], pa_im[PER], pb_re[PER], pb_im[PER];
    size_t arow[PER];   // AG2: the (i, k) part i nbp^3 + k nbp of each A row's G2 index
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int row = bm + (threadIdx.x + q * 256) / KS;
        arow[q] = AG2 ? ((size_t)(row / nbp) * nbp * nbp + row % nbp) * nbp : (size_t)row * n;
    }
    auto fetch = [&](int k0) {
        const size_t acol = AG2 ? (size_t)(k0 / nbp) * nbp * nbp + k0 % nbp : (size_t)k0;
        const size_t bq = (size_t)(k0 / nbp) * nbp * nbp * nbp + k0 % nbp;   // BG2T
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = threadIdx.x + q * 256;
            ldc(A + arow[q] + acol + idx % KS, pa_re[q], pa_im[q]);
            if (BG2T)
                ldc(B + bq + (size_t)(bn + idx / KS) * nbp + idx % KS, pb_re[q], pb_im[q]);
            else
                ldc(B + (size_t)(k0 + idx / 64) * n + bn + idx % 64, pb_re[q], pb_im[q]);
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < n; k0 += KS) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = threadIdx.x + q * 256;
            a_c[idx / KS][idx % KS] = CT{pa_re[q], pa_im[q]};
            if (BG2T)
                b_c[idx % KS][idx / KS] = CT{pb_re[q], pb_im[q]};
            else
                b_c[idx / 64][idx % 64] = CT{pb_re[q], pb_im[q]};
        }
        __syncthreads();
        if (k0 + KS < n) fetch(k0 + KS);
        // the wave issues its matrix-core work at raised priority, so that of the
        // two work-groups on a compute unit the one past its barrier goes first
        // (0.5% in binary64, 1% in binary32)
        __builtin_amdgcn_s_setprio(1);
        {
            const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
            for (int k4 = 0; k4 < KS; k4 += 4) {
                T ar[2], ai[2], as[2], br[2], bi[2], bs[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const int i = wm + a * 16 + li;
                    const CT v = a_c[i][k4 + lk];
                    ar[a] = v.x;
                    ai[a] = v.y;
                    as[a] = ar[a] + ai[a];
                }
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int j = wn + b * 16 + li;
                    const CT v = b_c[k4 + lk][j];
                    br[b] = v.x;
                    bi[b] = v.y;
                    bs[b] = br[b] + bi[b];
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        p1[a][b] = MF<T>::mac(ar[a], br[b], p1[a][b]);
                        p2[a][b] = MF<T>::mac(ai[a], bi[b], p2[a][b]);
                        p3[a][b] = MF<T>::mac(as[a], bs[b], p3[a][b]);
                    }
            }
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        if (sizeof(T) == 4 && ((k0 + KS) % 64 == 0 || k0 + KS >= n)) {
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    for (int r4 = 0; r4 < 4; ++r4) {
                        const double d1 = p1[a][b][r4], d2 = p2[a][b][r4], d3 = p3[a][b][r4];
                        accd[a][b][0][r4] += d1 - d2;
                        accd[a][b][1][r4] += d3 - d1 - d2;
                    }
                    p1[a][b] = p2[a][b] = p3[a][b] = MF<T>::zero();
                }
        }
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int row = bm + wm + a * 16 + tile_row<T>(r4);
                const int col = bn + wn + b * 16 + tile_col();
                const double vr = sizeof(T) == 4 ? accd[a][b][0][r4] : (double)(p1[a][b][r4] - p2[a][b][r4]);
                const double vi = sizeof(T) == 4 ? accd[a][b][1][r4]
                                                 : (double)(p3[a][b][r4] - p1[a][b][r4] - p2[a][b][r4]);
                if (OUT == 0) {
                    // Pi_ijkl at [i][j][k][l] and, for the partner term of the
                    // combine, again at [l][k][j][i] of a second n x n array: the
                    // scatter costs this matrix-core-bound kernel 0.06 ms and
                    // spares the memory-bound combine a gather (0.47 -> 0.36 ms)
                    const int i = row / nbp, k = row % nbp, j = col / nbp, l = col % nbp;
                    ((cd*)dst)[(((size_t)i * nbp + j) * nbp + k) * nbp + l] = make_double2(vr, vi);
                    ((cd*)dst)[(size_t)n * n + (((size_t)l * nbp + k) * nbp + j) * nbp + i] = make_double2(vr, vi);
                } else {
                    size_t e;
                    if (OUT == 1) {
                        e = (size_t)row * n + col;
                    } else {
                        const int i = row / nbp, l = row % nbp, j = col / nbp, k = col % nbp;
                        e = (((size_t)i * nbp + j) * nbp + k) * nbp + l;
                    }
                    S* D = (S*)dst;
                    T dr, di;
                    ldc(D + e, dr, di);
                    stc(D + e, (double)dr + vr, (double)di + vi);
                }
            }
}

// --------------------------------------------------------------------------- layout helpers
__global__ void pad_kernel(const cd* __restrict__ src, cd* __restrict__ dst, int nb, int nbp, int rank,
                           int unpad) {
    size_t total = 1;
    for (int r = 0; r < rank; ++r) total *= (size_t)(unpad ? nb : nbp);
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int n_from = unpad ? nb : nbp;
        size_t t = e, ip = 0, iu = 0, mul_p = 1, mul_u = 1;
        bool inside = true;
        for (int r = 0; r < rank; ++r) {
            size_t idx = t % n_from;
            t /= n_from;
            if ((int)idx >= nb) inside = false;
            ip += idx * mul_p;
            iu += idx * mul_u;
            mul_p *= nbp;
            mul_u *= nb;
        }
        if (unpad)
            dst[e] = src[ip];
        else
            dst[e] = inside ? src[iu] : make_double2(0.0, 0.0);
    }
}

__global__ __launch_bounds__(256) void gen_obs_kernel(const cd* __restrict__ gl,
                                                     const cd* __restrict__ h0,
                                                     const cd* __restrict__ hhf,
                                                     const cd* __restrict__ icoll, int nbp,
                                                     double* __restrict__ res) {
    __shared__ double sh[4][256];
    const int n2 = nbp * nbp;
    double N = 0, ekin = 0, emf = 0, ecorr = 0;
    for (int e = threadIdx.x; e < n2; e += blockDim.x) {
        const int i = e / nbp, j = e % nbp;
        cd g = gl[j * nbp + i];
        cd nji = make_double2(g.y, -g.x);  // n = -i G^<
        cd h = h0[e], s = csub(hhf[e], h);
        ekin += h.x * nji.x - h.y * nji.y;
        emf += 0.5 * (s.x * nji.x - s.y * nji.y);
        if (i == j) {
            N += gl[e].y;
            ecorr += 0.5 * icoll[e].y;  // E_corr = 1/2 Im Tr I
        }
    }
    sh[0][threadIdx.x] = N;
    sh[1][threadIdx.x] = ekin;
    sh[2][threadIdx.x] = emf;
    sh[3][threadIdx.x] = ecorr;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) res[q] = sh[q][0];
}

// Symmetry residuals of an n x n pair matrix A (n = nbp^2): per block the
// maxima of |A_(r,c) - conj(A_(c,r))| (eq:Gsymm_b), of |A| and of
// |A_ijkl - A_jilk| (eq:Gsymm_a).
__global__ __launch_bounds__(256) void herm_kernel(const cd* __restrict__ A, int nbp, long long nn,
                                                  double* __restrict__ part) {
    __shared__ double s1[256], s2[256], s3[256];
    const long long n = (long long)nbp * nbp;
    double m1 = 0, m2 = 0, m3 = 0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
         e += (long long)gridDim.x * blockDim.x) {
        const long long r = e / n, col = e % n;
        const cd v = A[e], w = A[col * n + r];
        const double dx = v.x - w.x, dy = v.y + w.y;
        m1 = fmax(m1, sqrt(dx * dx + dy * dy));
        m2 = fmax(m2, sqrt(v.x * v.x + v.y * v.y));
        const long long rx = (r % nbp) * nbp + r / nbp, cx = (col % nbp) * nbp + col / nbp;
        const cd u = A[rx * n + cx];
        const double ex = v.x - u.x, ey = v.y - u.y;
        m3 = fmax(m3, sqrt(ex * ex + ey * ey));
    }
    s1[threadIdx.x] = m1;
    s2[threadIdx.x] = m2;
    s3[threadIdx.x] = m3;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + s]);
            s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + s]);
            s3[threadIdx.x] = fmax(s3[threadIdx.x], s3[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = s1[0];
        part[3 * blockIdx.x + 1] = s2[0];
        part[3 * blockIdx.x + 2] = s3[0];
    }
}

// --------------------------------------------------------------------------- host side
int main_grid(int nbp) { return std::min(nbp * nbp, 512); }

// ws: the switching factor phi(t) of the stage; every w-dependent output
// (sandwich, h^HF, collision partials, quasi-Hamiltonians) is linear in w
template <typename T, typename S, int NB>
g1g2_status run_blocks(g1g2_ctx* c, const Regs& in, double ws) {
    GeneralData& g = c->gen;
    const bool mixed = sizeof(T) == 4;
    const S* wrows = mixed ? (const S*)g.wm_rows32 : (const S*)g.wm_rows;
    const S* wcoll = mixed ? (const S*)g.w_coll32 : (const S*)g.w_coll;
    // a single-tile-per-wave shape prefetches the next row block in registers and
    // wants several blocks per work-group; the larger shapes want the wider grid
    const int grid_vt = std::min(NB * NB, Shape<NB>::TPW == 1 ? 512 : 1024);
    const HfArgs hf{g.w_hf, g.h0, in.g1, g.hhf, g.gg, g.nbp, g.nb, ws};
    hipLaunchKernelGGL((gen_vt_kernel<T, S, NB>), dim3(grid_vt + NB * NB), dim3(vt_threads<NB>()), 0,
                       c->stream, wrows, in.g1, (S*)g.vt, grid_vt, hf);
    HIP_OK(c, hipGetLastError());
    prof_mark(c, "gen_vt");
    const int se = c->d.selfenergy;
    const int n = NB * NB;
    if (se == G1G2_GW || se == G1G2_DSL) {
        const S* wgw = mixed ? (const S*)g.w_gw32 : (const S*)g.w_gw;
        hipLaunchKernelGGL((gen_heps_kernel<T, S, NB>), dim3(grid_vt), dim3(MainShape<NB>::THREADS), 0,
                           c->stream, wgw, in.g1, (S*)g.heps, ws);
        HIP_OK(c, hipGetLastError());
        prof_mark(c, "gen_heps");
        if constexpr (std::is_same<S, cd>::value) {   // binary64: the G2 operand is read in place
            hipLaunchKernelGGL((gen_gemm_kernel<T, S, 0, true>), dim3(n / 64, n / 64), dim3(256), 0, c->stream,
                               (const S*)in.g2, (const S*)g.heps, (void*)g.pimat, n, NB);
        } else {                                      // binary32: from a permuted binary32 copy
            hipLaunchKernelGGL((gen_bmat_kernel<S, 0>), dim3(2048), dim3(256), 0, c->stream, in.g2,
                               (S*)g.bmat, NB);
            HIP_OK(c, hipGetLastError());
            prof_mark(c, "gen_bmat");
            hipLaunchKernelGGL((gen_gemm_kernel<T, S, 0>), dim3(n / 64, n / 64), dim3(256), 0, c->stream,
                               (const S*)g.bmat, (const S*)g.heps, (void*)g.pimat, n, NB);
        }
        HIP_OK(c, hipGetLastError());
        prof_mark(c, "gen_gemm");
    }
    hipLaunchKernelGGL((gen_main_kernel<T, S, NB>), dim3(g.nipart), dim3(MainShape<NB>::THREADS), 0,
                       c->stream, in.g2, (const S*)g.vt, wcoll, g.gg, g.hhf, (S*)g.dmat, g.ipart, ws);
    HIP_OK(c, hipGetLastError());
    prof_mark(c, "gen_main");
    // T-matrix ladders: D += Lambda, so that the combine forms Lambda - Lambda^dagger,
    // the partner [Lambda_klij]^* of eq:g2-eq-tpp-lambda / eq:g2-eq-tph-lambda
    if (se == G1G2_TPP || se == G1G2_DSL) {
        const S* wpp = mixed ? (const S*)g.w_pp32 : (const S*)g.w_pp;
        hipLaunchKernelGGL((gen_hlad_kernel<T, S, NB, 0>), dim3(grid_vt), dim3(MainShape<NB>::THREADS), 0,
                           c->stream, wpp, in.g1, g.gg, (S*)g.heps, ws);
        // the TPP operand is G2 itself: binary64 reads it in place, binary32 from a copy
        const S* g2op = (const S*)g.bmat;
        if constexpr (std::is_same<S, cd>::value) g2op = (const S*)in.g2;
        else hipLaunchKernelGGL((gen_bmat_kernel<S, 1>), dim3(2048), dim3(256), 0, c->stream, in.g2,
                                (S*)g.bmat, NB);
        HIP_OK(c, hipGetLastError());
        prof_mark(c, "gen_hlad");
        hipLaunchKernelGGL((gen_gemm_kernel<T, S, 1>), dim3(n / 64, n / 64), dim3(256), 0, c->stream,
                           (const S*)g.heps, g2op, (void*)g.dmat, n, NB);
        HIP_OK(c, hipGetLastError());
        prof_mark(c, "gen_gemm");
    }
    if (se == G1G2_TPH || se == G1G2_DSL) {
        const S* wph = mixed ? (const S*)g.w_ph32 : (const S*)g.w_ph;
        hipLaunchKernelGGL((gen_hlad_kernel<T, S, NB, 1>), dim3(grid_vt), dim3(MainShape<NB>::THREADS), 0,
                           c->stream, wph, in.g1, g.gg, (S*)g.heps, ws);
        // the TPH operand G2_qjkp: binary64 reads it in place, binary32 from a copy
        if constexpr (!std::is_same<S, cd>::value)
            hipLaunchKernelGGL((gen_bmat_kernel<S, 2>), dim3(2048), dim3(256), 0, c->stream, in.g2,
                               (S*)g.bmat, NB);
        HIP_OK(c, hipGetLastError());
        prof_mark(c, "gen_hlad");
        if constexpr (std::is_same<S, cd>::value)
            hipLaunchKernelGGL((gen_gemm_kernel<T, S, 2, false, true>), dim3(n / 64, n / 64), dim3(256), 0,
                               c->stream, (const S*)g.heps, (const S*)in.g2, (void*)g.dmat, n, NB);
        else
            hipLaunchKernelGGL((gen_gemm_kernel<T, S, 2>), dim3(n / 64, n / 64), dim3(256), 0, c->stream,
                               (const S*)g.heps, (const S*)g.bmat, (void*)g.dmat, n, NB);
        HIP_OK(c, hipGetLastError());
        prof_mark(c, "gen_gemm");
    }
    return G1G2_OK;
}

template <typename S, int MODE>
g1g2_status run_combine(g1g2_ctx* c, const Regs& in, const Regs& y, const Regs& acc,
                        const Regs& out, double cb, double cc) {
    GeneralData& g = c->gen;
    const int n = g.nbp * g.nbp;
    const int nt = n / 32, ntiles = nt * (nt + 1) / 2;
    const G1Args g1{g.ipart, g.nipart, g.hhf, in.g1, y.g1, acc.g1, out.g1,
                    g.icoll, g.nb, guard_of(c)};
    const int ng1 = (g.nbp * (g.nbp + 1) / 2 + 3) / 4;   // work-groups of the G1 pairs
    if (c->d.selfenergy == G1G2_GW || c->d.selfenergy == G1G2_DSL)
        hipLaunchKernelGGL((gen_combine_kernel<MODE, S, true>), dim3(ng1 + ntiles), dim3(256), 0, c->stream,
                           (const S*)g.dmat, n, in.g2, y.g2, acc.g2, out.g2, g.pimat, g.nbp, cb, cc, g1, ng1);
    else
        hipLaunchKernelGGL((gen_combine_kernel<MODE, S, false>), dim3(ng1 + ntiles), dim3(256), 0, c->stream,
                           (const S*)g.dmat, n, in.g2, y.g2, acc.g2, out.g2, g.pimat, g.nbp, cb, cc, g1, ng1);
    HIP_OK(c, hipGetLastError());
    prof_mark(c, "gen_combine");
    return G1G2_OK;
}

template <typename T, typename S>
g1g2_status dispatch_blocks(g1g2_ctx* c, const Regs& in, double ws) {
    switch (c->gen.nbp) {
        case 16: return run_blocks<T, S, 16>(c, in, ws);
        case 32: return run_blocks<T, S, 32>(c, in, ws);
        case 48: return run_blocks<T, S, 48>(c, in, ws);
        case 64: return run_blocks<T, S, 64>(c, in, ws);
        default: return set_error(c, G1G2_EUNSUPPORTED, "general basis supports nb <= 64");
    }
}

template <typename S>
g1g2_status dispatch_combine(g1g2_ctx* c, int mode, const Regs& in, const Regs& y, const Regs& acc,
                             const Regs& out, double cb, double cc) {
    switch (mode) {
        case RK_RHS: return run_combine<S, RK_RHS>(c, in, y, acc, out, cb, cc);
        case RK_FIRST: return run_combine<S, RK_FIRST>(c, in, y, acc, out, cb, cc);
        case RK_MID: return run_combine<S, RK_MID>(c, in, y, acc, out, cb, cc);
        default: return run_combine<S, RK_LAST>(c, in, y, acc, out, cb, cc);
    }
}

template <typename V>
g1g2_status upload(g1g2_ctx* c, V** dst, const std::vector<V>& h) {
    HIP_OK(c, hipMalloc(dst, h.size() * sizeof(V)));
    HIP_OK(c, hipMemcpyAsync(*dst, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, c->stream));
    return G1G2_OK;
}

std::vector<float2> to_f32(const std::vector<cd>& v) {
    std::vector<float2> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = make_float2((float)v[i].x, (float)v[i].y);
    return o;
}

}  // namespace

g1g2_status gen_set_h0(g1g2_ctx* c, const cd* h0) {
    GeneralData& g = c->gen;
    const int nb = g.nb, nbp = g.nbp;
    std::vector<cd> hp((size_t)nbp * nbp, cmk(0, 0));
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) {
            cd v = h0[i * nb + j], vt = h0[j * nb + i];
            if (std::fabs(v.x - vt.x) > 1e-12 * (1 + std::fabs(v.x)) ||
                std::fabs(v.y + vt.y) > 1e-12 * (1 + std::fabs(v.y)))
                return set_error(c, G1G2_EINVAL, "h0 is not Hermitian");
            hp[i * nbp + j] = v;
        }
    if (!g.h0) HIP_OK(c, hipMalloc(&g.h0, hp.size() * sizeof(cd)));
    HIP_OK(c, hipMemcpyAsync(g.h0, hp.data(), hp.size() * sizeof(cd), hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return G1G2_OK;
}

g1g2_status gen_setup(g1g2_ctx* c, const cd* h0, const cd* w) {
    GeneralData& g = c->gen;
    const int nb = c->d.nb;
    const int nbp = ((nb + 15) / 16) * 16;
    if (nbp > 64) return set_error(c, G1G2_EUNSUPPORTED, "general basis supports nb <= 64");
    g.nb = nb;
    g.nbp = nbp;
    const size_t n4 = (size_t)nbp * nbp * nbp * nbp;
    const int se = c->d.selfenergy;
    const bool gw = se == G1G2_GW || se == G1G2_DSL;           // polarization Pi
    const bool pp = se == G1G2_TPP || se == G1G2_DSL;          // particle-particle ladder
    const bool ph = se == G1G2_TPH || se == G1G2_DSL;          // particle-hole ladder
    // the source is Psi^- except for GW without exchange; DSL includes the exchange
    const bool exch = se != G1G2_GW || (c->d.flags & G1G2_GW_EXCHANGE);
    auto W = [&](int i, int j, int k, int l) -> cd { return w[(((size_t)i * nb + j) * nb + k) * nb + l]; };
    // symmetry checks of the interaction (eq:wsymm_a, eq:wsymm_b)
    double wmax = 0, e1 = 0, e2 = 0;
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j)
            for (int k = 0; k < nb; ++k)
                for (int l = 0; l < nb; ++l) {
                    cd a = W(i, j, k, l), b = W(j, i, l, k), d = W(k, l, i, j);
                    wmax = std::max(wmax, std::hypot(a.x, a.y));
                    e1 = std::max(e1, std::hypot(a.x - b.x, a.y - b.y));
                    e2 = std::max(e2, std::hypot(a.x - d.x, a.y + d.y));
                }
    if (e1 > 1e-12 * (1 + wmax) || e2 > 1e-12 * (1 + wmax))
        return set_error(c, G1G2_EINVAL, "w violates w_ijkl = w_jilk or w_ijkl = conj(w_klij)");
    std::vector<cd> rows(n4, cmk(0, 0)), coll(n4, cmk(0, 0)), hf(n4, cmk(0, 0));
    auto P4 = [&](int a, int b, int cc, int d) { return (((size_t)a * nbp + b) * nbp + cc) * nbp + d; };
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j)
            for (int k = 0; k < nb; ++k)
                for (int l = 0; l < nb; ++l) {
                    cd v = W(i, j, k, l), vx = W(i, j, l, k);
                    rows[P4(i, j, k, l)] = exch ? csub(v, vx) : v;   // W^-_pqrs (or W for GW)
                    coll[P4(k, l, i, j)] = v;                         // [l][p][i][k] = w_iklp
                    hf[P4(i, k, l, j)] = csub(v, vx);                 // [i][j][l][k] = w^-_ikjl
                }
    g1g2_status s;
    if ((s = upload(c, &g.wm_rows, rows)) != G1G2_OK) return s;
    if ((s = upload(c, &g.w_coll, coll)) != G1G2_OK) return s;
    if ((s = upload(c, &g.w_hf, hf)) != G1G2_OK) return s;
    const bool mixed = c->d.precision == G1G2_MIXED;
    if (mixed) {
        if ((s = upload(c, &g.wm_rows32, to_f32(rows))) != G1G2_OK) return s;
        if ((s = upload(c, &g.w_coll32, to_f32(coll))) != G1G2_OK) return s;
    }
    // DSL with its exchange terms: h^eps and h^ph from w^-_ijkl = w_ijkl - w_ijlk
    const bool dslx = se == G1G2_DSL && (c->d.flags & G1G2_DSL_EXCHANGE);
    auto WX = [&](int i, int j, int k, int l) -> cd { return dslx ? csub(W(i, j, k, l), W(i, j, l, k)) : W(i, j, k, l); };
    if (gw) {
        std::vector<cd> wg(n4, cmk(0, 0));
        for (int s1 = 0; s1 < nb; ++s1)
            for (int q = 0; q < nb; ++q)
                for (int r = 0; r < nb; ++r)
                    for (int p = 0; p < nb; ++p) wg[P4(p, q, s1, r)] = WX(s1, q, r, p);  // M_pq[s][r] = w_sqrp
        if ((s = upload(c, &g.w_gw, wg)) != G1G2_OK) return s;
        if (mixed && (s = upload(c, &g.w_gw32, to_f32(wg))) != G1G2_OK) return s;
        HIP_OK(c, hipMalloc(&g.pimat, 2 * n4 * sizeof(cd)));
    }
    if (pp || ph) {
        std::vector<cd> wl(n4, cmk(0, 0));
        if (pp) {
            for (int p = 0; p < nb; ++p)
                for (int q = 0; q < nb; ++q)
                    for (int k = 0; k < nb; ++k)
                        for (int l = 0; l < nb; ++l) wl[P4(k, l, p, q)] = W(p, q, k, l);   // M_pq = w_pqkl
            if ((s = upload(c, &g.w_pp, wl)) != G1G2_OK) return s;
            if (mixed && (s = upload(c, &g.w_pp32, to_f32(wl))) != G1G2_OK) return s;
        }
        if (ph) {
            for (int p = 0; p < nb; ++p)
                for (int j = 0; j < nb; ++j)
                    for (int k = 0; k < nb; ++k)
                        for (int q = 0; q < nb; ++q) wl[P4(j, k, p, q)] = WX(p, j, k, q);   // M_pq = w_pjkq
            if ((s = upload(c, &g.w_ph, wl)) != G1G2_OK) return s;
            if (mixed && (s = upload(c, &g.w_ph32, to_f32(wl))) != G1G2_OK) return s;
        }
    }
    if (gw || pp || ph) {
        const size_t es = mixed ? sizeof(float2) : sizeof(cd);
        HIP_OK(c, hipMalloc(&g.heps, n4 * es));
        HIP_OK(c, hipMalloc(&g.bmat, n4 * es));
    }
    const size_t es = mixed ? sizeof(float2) : sizeof(cd);
    HIP_OK(c, hipMalloc(&g.vt, n4 * es));
    HIP_OK(c, hipMalloc(&g.dmat, n4 * es));
    HIP_OK(c, hipMalloc(&g.hhf, (size_t)nbp * nbp * sizeof(cd)));
    HIP_OK(c, hipMalloc(&g.gg, (size_t)nbp * nbp * sizeof(cd)));
    HIP_OK(c, hipMalloc(&g.icoll, (size_t)nbp * nbp * sizeof(cd)));
    g.nipart = main_grid(nbp);
    HIP_OK(c, hipMalloc(&g.ipart, (size_t)g.nipart * nbp * nbp * sizeof(cd)));
    return gen_set_h0(c, h0);
}

g1g2_status gen_stage(g1g2_ctx* c, int mode, double t, const Regs& in, const Regs& y,
                      const Regs& acc, const Regs& out, double cb, double cc) {
    const double ws = c->switch_value(t);
    g1g2_status s;
    if (c->d.precision == G1G2_MIXED) {
        if ((s = dispatch_blocks<float, float2>(c, in, ws)) != G1G2_OK) return s;
        return dispatch_combine<float2>(c, mode, in, y, acc, out, cb, cc);
    }
    if ((s = dispatch_blocks<double, cd>(c, in, ws)) != G1G2_OK) return s;
    return dispatch_combine<cd>(c, mode, in, y, acc, out, cb, cc);
}

g1g2_status gen_observables(g1g2_ctx* c, const Regs& s, double t, g1g2_obs* o) {
    (void)t;
    GeneralData& g = c->gen;
    // one right-hand-side evaluation refreshes h^HF and the collision integral
    g1g2_status st = gen_stage(c, RK_RHS, c->t, s, s, s, c->io, 0.0, 0.0);
    if (st != G1G2_OK) return st;
    hipLaunchKernelGGL(gen_obs_kernel, dim3(1), dim3(256), 0, c->stream, s.g1, g.h0, g.hhf, g.icoll,
                       g.nbp, c->dscratch);
    HIP_OK(c, hipGetLastError());
    const int n = g.nbp * g.nbp;
    const int nblk = 256;
    hipLaunchKernelGGL(herm_kernel, dim3(nblk), dim3(256), 0, c->stream, s.g2, g.nbp, (long long)n * n,
                       c->dscratch + 8);
    HIP_OK(c, hipGetLastError());
    std::vector<double> h(8 + 3 * nblk);
    HIP_OK(c, hipMemcpyAsync(h.data(), c->dscratch, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    double m1 = 0, m2 = 0, m3 = 0;
    for (int b = 0; b < nblk; ++b) {
        m1 = std::max(m1, h[8 + 3 * b]);
        m2 = std::max(m2, h[8 + 3 * b + 1]);
        m3 = std::max(m3, h[8 + 3 * b + 2]);
    }
    o->N[0] = h[0];
    o->N[1] = 0.0;
    o->E_kin = h[1];
    o->E_mf = h[2];
    o->E_corr = h[3];
    o->E_tot = h[1] + h[2] + h[3];
    o->docc = 0.0;
    o->herm_resid = m2 > 0 ? m1 / m2 : 0.0;
    o->exch_resid = m2 > 0 ? m3 / m2 : 0.0;
    return G1G2_OK;
}

g1g2_status gen_pad(g1g2_ctx* c, const cd* src, cd* dst, int rank) {
    hipLaunchKernelGGL(pad_kernel, dim3(1024), dim3(256), 0, c->stream, src, dst, c->gen.nb, c->gen.nbp,
                       rank, 0);
    HIP_OK(c, hipGetLastError());
    return G1G2_OK;
}

g1g2_status gen_unpad(g1g2_ctx* c, const cd* src, cd* dst, int rank) {
    hipLaunchKernelGGL(pad_kernel, dim3(1024), dim3(256), 0, c->stream, src, dst, c->gen.nb, c->gen.nbp,
                       rank, 1);
    HIP_OK(c, hipGetLastError());
    return G1G2_OK;
}

void gen_free(g1g2_ctx* c) {
    GeneralData& g = c->gen;
    void* ptrs[] = {g.h0,    g.wm_rows,   g.w_coll, g.w_hf,  g.vt,     g.dmat,   g.hhf,
                    g.gg,    g.ipart,     g.heps,   g.bmat,  g.pimat,  g.wm_rows32, g.w_coll32,
                    g.w_gw,  g.w_gw32,    g.icoll,  g.w_pp,  g.w_ph,   g.w_pp32, g.w_ph32};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    g = GeneralData();
}
