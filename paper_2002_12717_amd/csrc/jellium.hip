// Jellium (uniform electron gas) G1-G2 kernels in a plane-wave basis (Sec.
// III.E, Sec. IV.D).
//
// Momenta live on a periodic grid (dims Lx, Ly, Lz; index n = x + Lx (y + Ly
// z); components add modulo the grid), so momentum conservation is exact in
// the finite basis.  G1 is diagonal: G^{<,s}_p, [2][nb].  G2 is kept in the
// momentum-transfer form of eq:g2-def-jellium, one [nb]^3 block per spin pair
// (up-up, up-down, down-down; down-up follows from eq:Gsymm_a):
//   G2[c][P][Pb][Q] = G2^{a b a b}_{(P-Q, a), (Pb+Q, b), (P, a), (Pb, b)}.
// Every element of the right-hand side (eq:jellium-g2, eq:jellium-gwpi) is a
// pointwise function of the element, of G1 at four momenta and, for GW, of the
// polarization sums S^a_{P,Q} = sum_{s,K} G2^{a s}_{P,K,Q}; the collision
// integral is I^a_P = -i sum_Q v_Q S^a_{P,Q} (eq:jellium-g1).  A stage is
// therefore one streaming pass over G2 (no inner sum, no neighbour reads: the
// O(nb^3) cost of Tab. I) plus a small prologue on nb^2 numbers:
//   jel_prep  : S of the stage input from the partial sums the previous pass
//               left, I, the G1 update, h^HF of the stage input;
//   jel_stage : the G2 right-hand side with its fused Runge-Kutta update, and
//               the partial sums of S of the values it writes (the next stage
//               input), so that no separate pass over G2 computes them.
// The middle sums (over Pb) are exact per work-group; the down-spin sums that
// the up-down block feeds (a sum over its first momentum) are accumulated with
// binary64 atomics.
//
// The T-matrix closures (eq:jellium-lambdapp, eq:jellium-lambdaph) need the
// ladder sums of the stage input before the stage pass:
//   jel_lad (TPP): L[c][P][Pb][Q]  = sum_K G2[c][P][Pb][K] v_{K-Q}
//   jel_lad (TPH): M[c][P][S][Pb]  = sum_K G2[c][P][K][S-K] v_{Pb-K}
// (TPH sums along the anti-diagonals Pb + Q = S of a (Pb, Q) plane).  Both are
// cyclic correlations or convolutions over the periodic grid, so per row they
// are a discrete Fourier transform, a product with the transform of v and
// the inverse transform, each transform taken one grid dimension at a time:
// Lx + Ly + Lz multiply-adds per output instead of the nb of the direct sum
// (O(nb^3 (Lx + Ly + Lz)) per stage against the O(nb^4) of Tab. I; the same
// sums up to rounding).  The stage pass adds Lambda = -f L at the element and
// the partner's -conj(Lambda_{P-Q, Pb+Q, -Q}), both read from that buffer.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "ctx.h"

namespace {

constexpr int JEL_PB = 4;        // momenta P per work-group (one per inner iteration)
constexpr int JEL_MAX_NB = 1024; // momenta of the grid (the stage kernel stages h and G1 in LDS)
constexpr int JEL_QB = 64;       // momenta Q per work-group (one per lane)
constexpr int JEL_THREADS = 256; // prologue and observables
constexpr int JEL_WAVES = 8;     // stage pass: wave w takes Pb = w, w + JEL_WAVES, ...
enum { LAD_NONE = 0, LAD_PP = 1, LAD_PH = 2 };

struct JGrid {
    int lx, ly, lz, nb;
};

__device__ __forceinline__ int jwrap(int a, int L) { return a < 0 ? a + L : (a >= L ? a - L : a); }

struct JMom {   // components of one momentum
    int x, y, z;
};

__device__ __forceinline__ JMom jdec(const JGrid& g, int n) {
    JMom m;
    m.x = n % g.lx;
    const int r = n / g.lx;
    m.y = r % g.ly;
    m.z = r / g.ly;
    return m;
}
__device__ __forceinline__ int jenc(const JGrid& g, int x, int y, int z) { return x + g.lx * (y + g.ly * z); }
__device__ __forceinline__ int jadd(const JGrid& g, const JMom& a, const JMom& b) {
    return jenc(g, jwrap(a.x + b.x, g.lx), jwrap(a.y + b.y, g.ly), jwrap(a.z + b.z, g.lz));
}
__device__ __forceinline__ JMom jsubm(const JGrid& g, const JMom& a, const JMom& b) {
    JMom m;
    m.x = jwrap(a.x - b.x, g.lx);
    m.y = jwrap(a.y - b.y, g.ly);
    m.z = jwrap(a.z - b.z, g.lz);
    return m;
}
__device__ __forceinline__ int jidx(const JGrid& g, const JMom& a) { return jenc(g, a.x, a.y, a.z); }

// spins (a, b) of block c: up-up, up-down, down-down
__host__ __device__ __forceinline__ int spin_a(int c) { return c == 2 ? 1 : 0; }
__host__ __device__ __forceinline__ int spin_b(int c) { return c == 0 ? 0 : 1; }

struct PrepArgs {
    JGrid g;
    const double* eps;        // [2][nb]
    const double* v;          // [nb]
    const cd* in1;            // stage-input G1 [2][nb]
    const cd* y1;
    cd* acc1;
    cd* out1;
    double cb, cc;
    const cd* sc;             // [3][nb][nb] middle sums of the stage input
    const cd* sb;             // [nb][nb] down-spin sums from the up-down block
    cd* sb_next;              // zeroed here: the stage pass accumulates into it
    cd* stot;                 // [2][nb][nb] S^a_{P,Q} of the stage input (out)
    cd* skew;                 // [2][nb][nb] skew[a][Pb][Q] = S^a_{Pb+Q,Q} (out; GW partner, coalesced)
    cd* hhf;                  // [2][nb] h^HF of the stage input (out)
    DivGuard guard;
};

// One work-group per (spin a, momentum P); threads over Q (and over the summed
// momentum of h^HF).
template <int MODE>
__global__ __launch_bounds__(JEL_THREADS) void jel_prep_kernel(PrepArgs s) {
    __shared__ double red[4][JEL_THREADS];
    const JGrid g = s.g;
    const int nb = g.nb;
    const int a = blockIdx.x / nb, P = blockIdx.x - a * nb;
    const int tid = threadIdx.x;
    const JMom mP = jdec(g, P);
    double ir = 0.0, ii = 0.0, hr = 0.0, hi = 0.0;
    for (int q = tid; q < nb; q += JEL_THREADS) {
        const size_t pq = (size_t)P * nb + q;
        cd S = a == 0 ? cadd(s.sc[pq], s.sc[(size_t)nb * nb + pq]) : cadd(s.sc[2 * (size_t)nb * nb + pq], s.sb[pq]);
        s.stot[(size_t)a * nb * nb + pq] = S;
        s.skew[((size_t)a * nb + jidx(g, jsubm(g, mP, jdec(g, q)))) * nb + q] = S;
        const double vq = s.v[q];
        ir += vq * S.x;
        ii += vq * S.y;
        // h^HF_P = eps_P + i sum_pb v[P - pb] G^<_pb
        const cd gl = s.in1[a * nb + q];
        const double vpq = s.v[jidx(g, jsubm(g, mP, jdec(g, q)))];
        hr -= vpq * gl.y;
        hi += vpq * gl.x;
        if (a == 0 && s.sb_next) s.sb_next[pq] = cmk(0.0, 0.0);
    }
    red[0][tid] = ir;
    red[1][tid] = ii;
    red[2][tid] = hr;
    red[3][tid] = hi;
    __syncthreads();
    for (int st = JEL_THREADS / 2; st > 0; st >>= 1) {
        if (tid < st)
            for (int k = 0; k < 4; ++k) red[k][tid] += red[k][tid + st];
        __syncthreads();
    }
    if (tid != 0) return;
    const int e = a * nb + P;
    s.hhf[e] = cmk(s.eps[e] + red[2][0], red[3][0]);
    // I = -i sum_Q v_Q S_{P,Q};  dG^</dt = -i (I + conj(I)) = -2 i Re(I)
    const cd I = cmul_mi(cmk(red[0][0], red[1][0]));
    const cd f = cmk(0.0, -2.0 * I.x);
    if (MODE == RK_FIRST && e == 0) guard_begin_step(s.guard);
    rk_update<MODE>(e, f, s.in1[e], s.y1, s.acc1, s.out1, s.cb, s.cc);
    if (MODE == RK_LAST && guard_bad(s.out1[e], true)) guard_fire(s.guard, 0, s.guard.div[0]);
}

struct StageArgsJ {
    JGrid g;
    const double* v;          // [nb]
    const cd* g1;             // stage-input G1 [2][nb]
    const cd* hhf;            // [2][nb]
    const cd* stot;           // [2][nb][nb] (GW)
    const cd* skew;           // [2][nb][nb] S^a_{Pb+Q,Q} at [a][Pb][Q] (GW)
    const void* in2;          // stage input G2 [3][nb]^3 (binary64 or binary32 storage)
    const cd* y2;
    cd* acc2;
    void* out2;
    double cb, cc;
    int exch;                 // source with the exchange term (Psi^-)
    const cd* lad;            // [3][nb]^3 ladder sums of the stage input (TPP: L, TPH: M)
    cd* sc_next;              // [3][nb][nb] middle sums of the values written (exact)
    cd* sb_next;              // [nb][nb] their down-spin sums from the up-down block (atomics)
};

template <typename TO>
__device__ __forceinline__ cd stored_value(cd v) {
    if constexpr (std::is_same<TO, float2>::value) return cmk((double)(float)v.x, (double)(float)v.y);
    else return v;
}

__device__ __forceinline__ void atomic_add_c(cd* p, cd v) {
    atomicAdd(&p->x, v.x);
    atomicAdd(&p->y, v.y);
}

// Work-group (block c, JEL_PB momenta P, JEL_QB momenta Q); lane = Q, wave w
// takes Pb = w, w + JEL_WAVES, ... and, for each, the JEL_PB momenta P.  The
// P-dependent factors stay in registers (about 250 VGPRs, two waves per SIMD):
// measured, reading them from LDS per element instead (four waves per SIMD)
// was slower for GW (0.61 against 0.47 ms per launch on 6x6x6).  Loads of a
// fixed (P, Pb) are JEL_QB consecutive elements.  REDUCE: only the partial sums
// of the input (no right-hand side); MODE == RK_RHS: the right-hand side into
// out2, no sums.
template <int MODE, bool GW, typename TI, typename TO, bool REDUCE, int LAD>
__global__ __launch_bounds__(64 * JEL_WAVES) void jel_stage_kernel(StageArgsJ s) {
    // h^HF and G1 of both spins and v, staged in LDS (dynamic: 2 nb + 2 nb complex, nb real)
    extern __shared__ cd sh_dyn[];
    cd* sh_h = sh_dyn;
    cd* sh_g = sh_dyn + 2 * s.g.nb;
    double* sh_v = reinterpret_cast<double*>(sh_dyn + 4 * s.g.nb);
    __shared__ cd sh_red[JEL_WAVES][JEL_PB][JEL_QB];
    const JGrid g = s.g;
    const int nb = g.nb;
    const int npb = (nb + JEL_PB - 1) / JEL_PB, nqb = (nb + JEL_QB - 1) / JEL_QB;
    int b = blockIdx.x;
    const int c = b / (npb * nqb);
    b -= c * npb * nqb;
    const int pblk = b / nqb, qblk = b - pblk * nqb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (!REDUCE) {
        for (int q = tid; q < 2 * nb; q += 64 * JEL_WAVES) {
            sh_h[q] = s.hhf[q];
            sh_g[q] = s.g1[q];
        }
        for (int q = tid; q < nb; q += 64 * JEL_WAVES) sh_v[q] = s.v[q];
        __syncthreads();
    }
    const int sa = spin_a(c), sb = spin_b(c);
    const int Q = qblk * JEL_QB + lane;
    const bool qok = Q < nb;
    const int Qc = qok ? Q : 0;
    const JMom mQ = jdec(g, Qc);
    const int negQ = jidx(g, jsubm(g, JMom{0, 0, 0}, mQ));
    const cd* hA = sh_h + sa * nb;
    const cd* hB = sh_h + sb * nb;
    const cd* gA = sh_g + sa * nb;
    const cd* gB = sh_g + sb * nb;
    // per owned P: index of P - Q, its components, and the P-dependent factors
    int Pv[JEL_PB], Pm[JEL_PB];
    JMom mPm[JEL_PB];
    cd ePm[JEL_PB], gPm[JEL_PB], gP[JEL_PB], SaP[JEL_PB];
    cd sa_acc[JEL_PB];
#pragma unroll
    for (int j = 0; j < JEL_PB; ++j) {
        const int P = pblk * JEL_PB + j;
        Pv[j] = P < nb ? P : -1;
        const int Pc = P < nb ? P : 0;
        mPm[j] = jsubm(g, jdec(g, Pc), mQ);
        Pm[j] = jidx(g, mPm[j]);
        sa_acc[j] = cmk(0.0, 0.0);
        if (!REDUCE) {
            ePm[j] = csub(hA[Pm[j]], hA[Pc]);          // h^a_{P-Q} - h^a_P
            gPm[j] = gA[Pm[j]];
            gP[j] = gA[Pc];
            SaP[j] = GW && qok ? s.stot[((size_t)sa * nb + Pc) * nb + Qc] : cmk(0.0, 0.0);
        }
    }
    const double vQ = REDUCE ? 0.0 : sh_v[Qc];
    const size_t n3 = (size_t)nb * nb * nb;
    const TI* in = static_cast<const TI*>(s.in2) + c * n3;
    const cd* y = s.y2 + c * n3;
    cd* acc = s.acc2 + c * n3;
    TO* out = static_cast<TO*>(s.out2) + c * n3;
    for (int Pb = wave; Pb < nb; Pb += JEL_WAVES) {
        const JMom mPb = jdec(g, __builtin_amdgcn_readfirstlane(Pb));
        const int Pbp = jidx(g, JMom{jwrap(mPb.x + mQ.x, g.lx), jwrap(mPb.y + mQ.y, g.ly), jwrap(mPb.z + mQ.z, g.lz)});
        cd hb = cmk(0.0, 0.0), gl2 = cmk(0.0, 0.0), gl4 = cmk(0.0, 0.0), SbP = cmk(0.0, 0.0);
        if (!REDUCE) {
            hb = csub(hB[Pbp], hB[Pb]);                   // h^b_{Pb+Q} - h^b_Pb
            gl2 = gB[Pbp];
            gl4 = gB[Pb];
            if (GW && qok) SbP = s.skew[((size_t)sb * nb + Pb) * nb + Qc];
        }
        cd sb_sum = cmk(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < JEL_PB; ++j) {
            if (!qok || Pv[j] < 0) continue;
            const size_t e = ((size_t)Pv[j] * nb + Pb) * nb + Q;
            const cd av = ld_c(in, (long long)e);
            cd o;
            if (REDUCE) {
                o = av;
            } else {
                // commutator: G2 (h^a_{P-Q} + h^b_{Pb+Q} - h^a_P - h^b_Pb)
                cd r = cmul(av, cadd(ePm[j], hb));
                // source (eq:jellium-g2): -w Phi, w = v_Q - delta_ab v_{P-Q-Pb}
                const cd gl1 = gPm[j], gl3 = gP[j];
                const cd gg1 = cmk(gl1.x, gl1.y - 1.0), gg2 = cmk(gl2.x, gl2.y - 1.0);
                const cd gg3 = cmk(gl3.x, gl3.y - 1.0), gg4 = cmk(gl4.x, gl4.y - 1.0);
                const cd phi = csub(cmul(cmul(gg1, gg2), cmul(gl3, gl4)), cmul(cmul(gl1, gl2), cmul(gg3, gg4)));
                double w = vQ;
                if (s.exch && sa == sb) w -= sh_v[jidx(g, jsubm(g, mPm[j], mPb))];
                r = csub(r, cscale(phi, w));
                if (GW) {   // Pi - conj(Pi^{ba}_{Pb+Q, P-Q, Q}) (eq:jellium-gwpi)
                    const cd fb = csub(cmul(gg2, gl4), cmul(gl2, gg4));
                    const cd fa = csub(cmul(gg3, gl1), cmul(gl3, gg1));
                    const cd pi = cscale(cmul(fb, SaP[j]), vQ);
                    const cd pt = cscale(cmul(fa, SbP), vQ);
                    r = cadd(r, csub(pi, cconj(pt)));
                }
                if (LAD != LAD_NONE) {
                    // Lambda - conj(Lambda_{P-Q, Pb+Q, -Q}), Lambda = -f L with
                    //   pp (eq:jellium-lambdapp): f = G>_{P-Q} G>_{Pb+Q} - G<_{P-Q} G<_{Pb+Q}
                    //   ph (eq:jellium-lambdaph): f = G>_{P-Q} G<_{Pb} - G<_{P-Q} G>_{Pb}
                    // and f at the partner element from the same four G1 values
                    const cd* __restrict__ L = s.lad + c * n3;
                    cd lo, lp, fo, fp;
                    // both ladders are stored in the layout of G2: the own sum at
                    // e, the partner's at (P - Q, Pb + Q, -Q)
                    lo = L[e];
                    lp = L[((size_t)Pm[j] * nb + Pbp) * nb + negQ];
                    if (LAD == LAD_PP) {
                        fo = csub(cmul(gg1, gg2), cmul(gl1, gl2));
                        fp = csub(cmul(gg3, gg4), cmul(gl3, gl4));
                    } else {
                        fo = csub(cmul(gg1, gl4), cmul(gl1, gg4));
                        fp = csub(cmul(gg3, gl2), cmul(gl3, gg2));
                    }
                    r = csub(r, csub(cmul(fo, lo), cconj(cmul(fp, lp))));
                }
                const cd f = cmul_mi(r);
                if (MODE == RK_RHS) {
                    o = f;
                    st_c(out, (long long)e, f);
                } else if (MODE == RK_FIRST) {
                    acc[e] = cmk(fma(s.cb, f.x, av.x), fma(s.cb, f.y, av.y));
                    o = cmk(fma(s.cc, f.x, av.x), fma(s.cc, f.y, av.y));
                    st_c(out, (long long)e, o);
                } else if (MODE == RK_MID) {
                    const cd ac = acc[e], yv = y[e];
                    acc[e] = cmk(fma(s.cb, f.x, ac.x), fma(s.cb, f.y, ac.y));
                    o = cmk(fma(s.cc, f.x, yv.x), fma(s.cc, f.y, yv.y));
                    st_c(out, (long long)e, o);
                } else {
                    const cd ac = acc[e];
                    o = cmk(fma(s.cb, f.x, ac.x), fma(s.cb, f.y, ac.y));
                    st_c(out, (long long)e, o);
                }
                o = stored_value<TO>(o);                    // as stored (rounded when binary32)
            }
            if (MODE != RK_RHS) {
                sa_acc[j] = cadd(sa_acc[j], o);
                sb_sum = cadd(sb_sum, o);
            }
        }
        if (MODE != RK_RHS && c == 1 && qok) atomic_add_c(s.sb_next + (size_t)Pb * nb + negQ, sb_sum);
    }
    if (MODE == RK_RHS) return;
#pragma unroll
    for (int j = 0; j < JEL_PB; ++j) sh_red[wave][j][lane] = sa_acc[j];
    __syncthreads();
    if (wave == 0 && qok) {
#pragma unroll
        for (int j = 0; j < JEL_PB; ++j) {
            if (Pv[j] < 0) continue;
            cd t = sh_red[0][j][lane];
            for (int w = 1; w < JEL_WAVES; ++w) t = cadd(t, sh_red[w][j][lane]);
            s.sc_next[((size_t)c * nb + Pv[j]) * nb + Q] = t;
        }
    }
}

struct LadArgs {
    int nb;                   // momenta
    int len[3], stride[3];    // grid lengths and index strides (1, Lx, Lx Ly)
    int toff[3];              // offsets of each dimension's twiddles
    const void* in2;          // stage input G2 [3][nb]^3
    const cd* vhat;           // [nb] the transform of v over nb: sum_m v_m e^{-2 pi i k.m/L} / nb
    const cd* tw;             // e^{-2 pi i q / L_d}, q < L_d, for d = 0, 1, 2
    const int* subt;          // [nb][nb] index of S - K (TPH)
    cd* out;                  // [3][nb]^3
};

// rows per work-group of the ladder transform: four where their two copies fit
// the 64 KB of LDS a launch gets by default (nb <= 512), else two; four rows
// took the 6x6x6 TPH transform from 0.62 to 0.56 ms (TPP 0.565 -> 0.554)
constexpr int LAD_ROWS_MAX = 4;
int lad_rows(const g1g2_ctx* c) {
    if (c->d.flags & G1G2_JEL_LAD_ROWS2) return 2;
    return 2 * LAD_ROWS_MAX * c->jel.nb * (int)sizeof(cd) <= 65536 ? LAD_ROWS_MAX : 2;
}

// The ladder sums of ROWS rows per work-group, rows (c, P, X):
//   TPP: g[K] = G2[c][P][X][K]      (X = Pb), out = F-[vhat F+[g]]
//   TPH: h[K] = G2[c][P][K][X - K]  (X = S),  out = F+[vhat F-[h]]
// Both are stored in the layout of G2, L[c][P][Pb][Q] (TPH: output Pb of row
// (c, P, S) at Q = S - Pb).
// with F+/- the transforms with e^{+/-2 pi i k.m/L} over the grid, each the
// product of one-dimensional transforms along x, y and z.  Thread n owns
// momentum n of every row: in a pass along d it sums the L_d elements of its
// line of each row (read from LDS) times its twiddles, so its line offset and
// twiddle index are computed once per pass.  The rows and a ping-pong copy
// live in LDS.
template <int KIND, typename TI, int ROWS>
__global__ __launch_bounds__(JEL_MAX_NB) void jel_lad_kernel(LadArgs s) {
    extern __shared__ cd lad_sh[];   // [2][ROWS][nb]
    const int nb = s.nb, n = threadIdx.x;
    cd* const buf0 = lad_sh;
    cd* const buf1 = lad_sh + ROWS * nb;
    const bool nok = n < nb;
    const long long nn = (long long)nb * nb, rows = 3 * nn;
    const long long r0 = (long long)blockIdx.x * ROWS;
    const TI* __restrict__ in = static_cast<const TI*>(s.in2);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const long long row = r0 + r;
        cd x = cmk(0.0, 0.0);
        if (nok && row < rows) {
            const int c = (int)(row / nn);
            const int rem = (int)(row - c * nn), P = rem / nb, X = rem - P * nb;
            const size_t idx = (size_t)c * nn * nb +
                               (KIND == LAD_PP ? ((size_t)P * nb + X) * nb + n
                                               : ((size_t)P * nb + n) * nb + s.subt[X * nb + n]);
            x = ld_c(in, (long long)idx);
        }
        if (nok) buf0[r * nb + n] = x;
    }
    __syncthreads();
    bool cur = false;   // false: data in buf0
    auto passes = [&](bool plus) {
        for (int d = 0; d < 3; ++d) {
            const int L = s.len[d], sd = s.stride[d];
            if (L == 1) continue;
            const cd* __restrict__ src = cur ? buf1 : buf0;
            cd* __restrict__ dst = cur ? buf0 : buf1;
            if (nok) {
                const cd* __restrict__ t = s.tw + s.toff[d];
                const int kd = (n / sd) % L, base = n - kd * sd;
                cd acc[ROWS];
#pragma unroll
                for (int r = 0; r < ROWS; ++r) acc[r] = cmk(0.0, 0.0);
                int q = 0;
                for (int m = 0; m < L; ++m) {
                    const cd w = t[q];
                    const double wi = plus ? -w.y : w.y;
#pragma unroll
                    for (int r = 0; r < ROWS; ++r) {
                        const cd x = src[r * nb + base + m * sd];
                        acc[r].x = fma(x.x, w.x, fma(-x.y, wi, acc[r].x));
                        acc[r].y = fma(x.x, wi, fma(x.y, w.x, acc[r].y));
                    }
                    q += kd;
                    if (q >= L) q -= L;
                }
#pragma unroll
                for (int r = 0; r < ROWS; ++r) dst[r * nb + n] = acc[r];
            }
            __syncthreads();
            cur = !cur;
        }
    };
    passes(KIND == LAD_PP);
    if (nok) {
        cd* b = cur ? buf1 : buf0;
        const cd vh = s.vhat[n];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) b[r * nb + n] = cmul(b[r * nb + n], vh);
    }
    __syncthreads();
    passes(KIND != LAD_PP);
    const cd* res = cur ? buf1 : buf0;
    if (KIND == LAD_PP) {
        if (nok)
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
                if (r0 + r < rows) s.out[(r0 + r) * nb + n] = res[r * nb + n];   // L[c][P][Pb][Q], Q = n
    } else {
        // output m of row (c, P, S) is M[P][m][S - m]: stored at [c][P][m][S - m],
        // the layout of the stage's own element, so the stage reads it coalesced.
        // Consecutive lanes take the ROWS outputs of one m (adjacent S - m), so a
        // store instruction writes pieces of 16 ROWS bytes rather than 16 bytes
        for (int e = threadIdx.x; e < ROWS * nb; e += blockDim.x) {
            const int m = e / ROWS, r = e - m * ROWS;
            const long long row = r0 + r;
            if (row >= rows) continue;
            const int c = (int)(row / nn);
            const int rem = (int)(row - c * nn), P = rem / nb, X = rem - P * nb;
            s.out[((size_t)(c * nb + P) * nb + m) * nb + s.subt[X * nb + m]] = res[r * nb + m];
        }
    }
}

int lad_blocks(const g1g2_ctx* c) {
    const long long rows = 3LL * c->jel.nb * c->jel.nb;
    const int r = lad_rows(c);
    return (int)((rows + r - 1) / r);
}

int lad_threads(const g1g2_ctx* c) { return (c->jel.nb + 63) / 64 * 64; }

// Observables from G1 and S of the state (one work-group): N^s, E_kin = sum eps n,
// the Fock energy -1/2 sum_s sum v[p - pb] n^s_p n^s_pb and E_corr = -1/2 Re sum v_Q S.
__global__ __launch_bounds__(JEL_THREADS) void jel_obs_kernel(JGrid g, const double* __restrict__ eps,
                                                           const double* __restrict__ v,
                                                           const cd* __restrict__ g1,
                                                           const cd* __restrict__ sc,
                                                           const cd* __restrict__ sb,
                                                           double* __restrict__ res) {
    __shared__ double red[5][JEL_THREADS];
    const int nb = g.nb, tid = threadIdx.x;
    double nu = 0, nd = 0, ek = 0, ef = 0, ec = 0;
    for (int e = tid; e < 2 * nb; e += JEL_THREADS) {
        const int s = e / nb, p = e - s * nb;
        const double n = g1[e].y;
        if (s == 0) nu += n;
        else nd += n;
        ek += eps[e] * n;
        const JMom mp = jdec(g, p);
        for (int q = 0; q < nb; ++q) ef -= 0.5 * v[jidx(g, jsubm(g, mp, jdec(g, q)))] * n * g1[s * nb + q].y;
    }
    const size_t nn = (size_t)nb * nb;
    for (size_t e = tid; e < nn; e += JEL_THREADS) {
        const double vq = v[e % nb];
        const cd su = cadd(sc[e], sc[nn + e]), sd = cadd(sc[2 * nn + e], sb[e]);
        ec -= 0.5 * vq * (su.x + sd.x);
    }
    red[0][tid] = nu;
    red[1][tid] = nd;
    red[2][tid] = ek;
    red[3][tid] = ef;
    red[4][tid] = ec;
    __syncthreads();
    for (int st = JEL_THREADS / 2; st > 0; st >>= 1) {
        if (tid < st)
            for (int k = 0; k < 5; ++k) red[k][tid] += red[k][tid + st];
        __syncthreads();
    }
    if (tid == 0)
        for (int k = 0; k < 5; ++k) res[k] = red[k][0];
}

__global__ void jel_zero_kernel(cd* p, size_t n) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        p[e] = cmk(0.0, 0.0);
}

JGrid grid_of(const g1g2_ctx* c) {
    const JelliumData& J = c->jel;
    return JGrid{J.dims[0], J.dims[1], J.dims[2], J.nb};
}

int stage_blocks(const g1g2_ctx* c) {
    const int nb = c->jel.nb;
    return 3 * ((nb + JEL_PB - 1) / JEL_PB) * ((nb + JEL_QB - 1) / JEL_QB);
}

size_t stage_lds(const g1g2_ctx* c) { return (size_t)c->jel.nb * (4 * sizeof(cd) + sizeof(double)); }

// Partial sums of S of a G2 register (binary64) into buffer set `buf`.
g1g2_status jel_reduce(g1g2_ctx* c, const cd* g2, int buf) {
    JelliumData& J = c->jel;
    const size_t nn = (size_t)J.nb * J.nb;
    hipLaunchKernelGGL(jel_zero_kernel, dim3(256), dim3(256), 0, c->stream, J.sb[buf], nn);
    StageArgsJ s{};
    s.g = grid_of(c);
    s.in2 = g2;
    s.sc_next = J.sc[buf];
    s.sb_next = J.sb[buf];
    hipLaunchKernelGGL((jel_stage_kernel<RK_FIRST, false, cd, cd, true, LAD_NONE>), dim3(stage_blocks(c)),
                       dim3(64 * JEL_WAVES), stage_lds(c), c->stream, s);
    HIP_OK(c, hipGetLastError());
    prof_mark(c, "jel_reduce");
    return G1G2_OK;
}

template <int MODE, bool GW, bool MIXED, int LAD>
void launch_stage(g1g2_ctx* c, const StageArgsJ& s) {
    using TI = typename std::conditional<MIXED && (MODE == RK_MID || MODE == RK_LAST), float2, cd>::type;
    using TO = typename std::conditional<MIXED && (MODE == RK_FIRST || MODE == RK_MID), float2, cd>::type;
    if constexpr (LAD != LAD_NONE) {   // the ladder sums of the stage input first
        const JelliumData& J = c->jel;
        LadArgs la{};
        la.nb = J.nb;
        for (int d = 0; d < 3; ++d) la.len[d] = J.dims[d];
        la.stride[0] = 1;
        la.stride[1] = J.dims[0];
        la.stride[2] = J.dims[0] * J.dims[1];
        la.toff[0] = 0;
        la.toff[1] = J.dims[0];
        la.toff[2] = J.dims[0] + J.dims[1];
        la.in2 = s.in2;
        la.vhat = J.vhat;
        la.tw = J.tw;
        la.subt = J.subt;
        la.out = J.lad;
        const int lr = lad_rows(c);
        if (lr == LAD_ROWS_MAX)
            hipLaunchKernelGGL((jel_lad_kernel<LAD, TI, LAD_ROWS_MAX>), dim3(lad_blocks(c)), dim3(lad_threads(c)),
                               2 * lr * J.nb * sizeof(cd), c->stream, la);
        else
            hipLaunchKernelGGL((jel_lad_kernel<LAD, TI, 2>), dim3(lad_blocks(c)), dim3(lad_threads(c)),
                               2 * lr * J.nb * sizeof(cd), c->stream, la);
        prof_mark(c, "jel_lad");
    }
    hipLaunchKernelGGL((jel_stage_kernel<MODE, GW, TI, TO, false, LAD>), dim3(stage_blocks(c)),
                       dim3(64 * JEL_WAVES), stage_lds(c), c->stream, s);
}

template <int MODE>
g1g2_status jel_stage_t(g1g2_ctx* c, const Regs& in, const Regs& y, const Regs& acc, const Regs& out, double cb,
                        double cc, int rbuf, int wbuf) {
    JelliumData& J = c->jel;
    PrepArgs p{};
    p.g = grid_of(c);
    p.eps = J.eps;
    p.v = J.v;
    p.in1 = in.g1;
    p.y1 = y.g1;
    p.acc1 = acc.g1;
    p.out1 = out.g1;
    p.cb = cb;
    p.cc = cc;
    p.sc = J.sc[rbuf];
    p.sb = J.sb[rbuf];
    p.sb_next = MODE == RK_RHS ? nullptr : J.sb[wbuf];   // a plain right-hand side accumulates nothing
    p.stot = J.stot;
    p.skew = J.skew;
    p.hhf = J.hhf;
    p.guard = guard_of(c);
    hipLaunchKernelGGL(jel_prep_kernel<MODE>, dim3(2 * J.nb), dim3(JEL_THREADS), 0, c->stream, p);
    HIP_OK(c, hipGetLastError());
    prof_mark(c, "jel_prep");
    StageArgsJ s{};
    s.g = p.g;
    s.v = J.v;
    s.g1 = in.g1;
    s.hhf = J.hhf;
    s.stot = J.stot;
    s.skew = J.skew;
    s.in2 = in.g2;
    s.y2 = y.g2;
    s.acc2 = acc.g2;
    s.out2 = out.g2;
    s.cb = cb;
    s.cc = cc;
    s.exch = c->d.selfenergy != G1G2_GW || (c->d.flags & G1G2_GW_EXCHANGE) ? 1 : 0;
    s.sc_next = J.sc[wbuf];
    s.sb_next = J.sb[wbuf];
    s.lad = J.lad;
    const int se = c->d.selfenergy;
    const bool mixed = MODE != RK_RHS && c->d.precision == G1G2_MIXED;
    if (se == G1G2_GW) {
        if (mixed) launch_stage<MODE, true, true, LAD_NONE>(c, s);
        else launch_stage<MODE, true, false, LAD_NONE>(c, s);
    } else if (se == G1G2_TPP) {
        if (mixed) launch_stage<MODE, false, true, LAD_PP>(c, s);
        else launch_stage<MODE, false, false, LAD_PP>(c, s);
    } else if (se == G1G2_TPH) {
        if (mixed) launch_stage<MODE, false, true, LAD_PH>(c, s);
        else launch_stage<MODE, false, false, LAD_PH>(c, s);
    } else {
        if (mixed) launch_stage<MODE, false, true, LAD_NONE>(c, s);
        else launch_stage<MODE, false, false, LAD_NONE>(c, s);
    }
    HIP_OK(c, hipGetLastError());
    prof_mark(c, "jel_stage");
    return G1G2_OK;
}

}  // namespace

int jel_max_nb() { return JEL_MAX_NB; }

g1g2_status jel_setup(g1g2_ctx* c, const int* dims, const double* eps, const double* v) {
    JelliumData& J = c->jel;
    J.dims[0] = dims[0];
    J.dims[1] = dims[1];
    J.dims[2] = dims[2];
    J.nb = dims[0] * dims[1] * dims[2];
    const size_t nb = J.nb, nn = nb * nb;
    const int se = c->d.selfenergy;
    if (se == G1G2_TPP || se == G1G2_TPH) {
        // the ladder sums' operands: the transform of v over the grid divided
        // by nb, the twiddles of each dimension, the index table of S - K
        // (TPH) and the [3][nb]^3 buffer of the sums
        const double tpi = 6.283185307179586476925286766559;
        auto comp = [&](int n, int d) {
            return d == 0 ? n % dims[0] : (d == 1 ? (n / dims[0]) % dims[1] : n / (dims[0] * dims[1]));
        };
        std::vector<cd> vh(nb), tw(dims[0] + dims[1] + dims[2]);
        for (size_t k = 0; k < nb; ++k) {
            double re = 0.0, im = 0.0;
            for (size_t m = 0; m < nb; ++m) {
                double ph = 0.0;
                for (int d = 0; d < 3; ++d) ph += (double)((comp((int)k, d) * comp((int)m, d)) % dims[d]) / dims[d];
                re += v[m] * std::cos(tpi * ph);
                im -= v[m] * std::sin(tpi * ph);
            }
            vh[k] = cmk(re / nb, im / nb);
        }
        for (int d = 0, o = 0; d < 3; o += dims[d], ++d)
            for (int q = 0; q < dims[d]; ++q)
                tw[o + q] = cmk(std::cos(tpi * q / dims[d]), -std::sin(tpi * q / dims[d]));
        std::vector<int> st(nn);
        for (int a = 0; a < J.nb; ++a)
            for (int b = 0; b < J.nb; ++b) {
                int x = (comp(a, 0) - comp(b, 0) + dims[0]) % dims[0];
                int y = (comp(a, 1) - comp(b, 1) + dims[1]) % dims[1];
                int z = (comp(a, 2) - comp(b, 2) + dims[2]) % dims[2];
                st[(size_t)a * nb + b] = x + dims[0] * (y + dims[1] * z);
            }
        HIP_OK(c, hipMalloc(&J.vhat, vh.size() * sizeof(cd)));
        HIP_OK(c, hipMalloc(&J.tw, tw.size() * sizeof(cd)));
        HIP_OK(c, hipMalloc(&J.subt, st.size() * sizeof(int)));
        HIP_OK(c, hipMalloc(&J.lad, 3 * nn * nb * sizeof(cd)));
        HIP_OK(c, hipMemcpyAsync(J.vhat, vh.data(), vh.size() * sizeof(cd), hipMemcpyHostToDevice, c->stream));
        HIP_OK(c, hipMemcpyAsync(J.tw, tw.data(), tw.size() * sizeof(cd), hipMemcpyHostToDevice, c->stream));
        HIP_OK(c, hipMemcpyAsync(J.subt, st.data(), st.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
        HIP_OK(c, hipStreamSynchronize(c->stream));
    }
    HIP_OK(c, hipMalloc(&J.eps, 2 * nb * sizeof(double)));
    HIP_OK(c, hipMalloc(&J.v, nb * sizeof(double)));
    HIP_OK(c, hipMalloc(&J.hhf, 2 * nb * sizeof(cd)));
    HIP_OK(c, hipMalloc(&J.stot, 2 * nn * sizeof(cd)));
    HIP_OK(c, hipMalloc(&J.skew, 2 * nn * sizeof(cd)));
    for (int b = 0; b < 3; ++b) {
        HIP_OK(c, hipMalloc(&J.sc[b], 3 * nn * sizeof(cd)));
        HIP_OK(c, hipMalloc(&J.sb[b], nn * sizeof(cd)));
    }
    HIP_OK(c, hipMemcpyAsync(J.eps, eps, 2 * nb * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipMemcpyAsync(J.v, v, nb * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return G1G2_OK;
}

void jel_free(g1g2_ctx* c) {
    JelliumData& J = c->jel;
    for (void* p : {(void*)J.eps, (void*)J.v, (void*)J.hhf, (void*)J.stot, (void*)J.skew, (void*)J.lad,
                    (void*)J.vhat, (void*)J.tw, (void*)J.subt})
        if (p) (void)hipFree(p);
    for (int b = 0; b < 3; ++b) {
        if (J.sc[b]) (void)hipFree(J.sc[b]);
        if (J.sb[b]) (void)hipFree(J.sb[b]);
    }
    J = JelliumData{};
}

g1g2_status jel_state_changed(g1g2_ctx* c) {
    c->jel.parity = 0;
    return jel_reduce(c, c->y.g2, 0);
}

g1g2_status jel_stage(g1g2_ctx* c, int mode, const Regs& in, const Regs& y, const Regs& acc, const Regs& out,
                      double cb, double cc) {
    JelliumData& J = c->jel;
    if (mode == RK_RHS) {   // a plain right-hand side of a caller state: its sums in buffer set 2
        g1g2_status s = jel_reduce(c, in.g2, 2);
        if (s != G1G2_OK) return s;
        return jel_stage_t<RK_RHS>(c, in, y, acc, out, cb, cc, 2, 2);
    }
    // the propagated registers alternate between buffer sets 0 and 1: a step
    // starts with the sums of y in set 0 and its last stage leaves those of the
    // new y there again (four stages per step)
    const int rbuf = J.parity, wbuf = J.parity ^ 1;
    J.parity ^= 1;
    switch (mode) {
        case RK_FIRST: return jel_stage_t<RK_FIRST>(c, in, y, acc, out, cb, cc, rbuf, wbuf);
        case RK_MID: return jel_stage_t<RK_MID>(c, in, y, acc, out, cb, cc, rbuf, wbuf);
        default: return jel_stage_t<RK_LAST>(c, in, y, acc, out, cb, cc, rbuf, wbuf);
    }
}

g1g2_status jel_observables(g1g2_ctx* c, const Regs& s, g1g2_obs* o) {
    JelliumData& J = c->jel;
    g1g2_status st = jel_reduce(c, s.g2, 2);
    if (st != G1G2_OK) return st;
    hipLaunchKernelGGL(jel_obs_kernel, dim3(1), dim3(JEL_THREADS), 0, c->stream, grid_of(c), J.eps, J.v, s.g1,
                       J.sc[2], J.sb[2], c->dscratch);
    HIP_OK(c, hipGetLastError());
    double h[5];
    HIP_OK(c, hipMemcpyAsync(h, c->dscratch, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    o->N[0] = h[0];
    o->N[1] = h[1];
    o->E_kin = h[2];
    o->E_mf = h[3];
    o->E_corr = h[4];
    o->E_tot = h[2] + h[3] + h[4];
    return G1G2_OK;
}
