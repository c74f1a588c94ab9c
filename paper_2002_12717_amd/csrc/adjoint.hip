// Discrete adjoint of the RK4 propagation of the driven Hubbard SOA system.
//
// Loss  L = sum_i a_i d_i(T) + sum_i b_i (n^up_ii(T) + n^dn_ii(T)),
// n_ii = Im G^<_ii (n = -i G^<), d_i = n^up_ii n^dn_ii - Re A_iiii.
// Parameters: drive coefficients c_m (through s(t) = sum_m c_m phi_m(t), which
// adds s(t) x_i to the diagonal of h0 for both spins) and U.
//
// Complex cotangents follow zbar = dL/dRe z + i dL/dIm z: for w = M z
// (complex linear) zbar += M^H wbar; for w = a b, abar += conj(b) wbar.
//
// One RK4 step y -> y + dt/6 (k1 + 2 k2 + 2 k3 + k4), k_s = f(Y_s, t_s), is
// reversed as
//   g4 = dt/6 l, m4 = J(Y4)^T g4, g3 = dt/3 l + dt m4, m3 = J(Y3)^T g3,
//   g2 = dt/3 l + dt/2 m3, m2 = J(Y2)^T g2, g1 = dt/6 l + dt/2 m2,
//   m1 = J(Y1)^T g1,  l <- l + m1 + m2 + m3 + m4,
// with y_n checkpointed every K steps; each segment is recomputed forward
// once, keeping y_n and the stage states Y2, Y3, Y4 of every step in device
// memory (four states per step of a segment).  The vector-Jacobian product of
// the right-hand side of eq:g2-hubbard / eq:eom_g1_hubbard is split into
//   adj_slice_red : in one pass over the cotangent, the G2 cotangent
//               (stencil of the commutator applied to the cotangent, plus the
//               collision-integral entries) and five of the six reductions of
//               the source Psi (eq:soa-cubic-scheme) differentiated with
//               respect to X and Y (per-slice partials),
//   adj_lane_red : the sixth reduction, reading contiguous rows,
//   adj_e, adj_g1e, adj_gsum : the G1 cotangents, the diagonal of h^HF,
//               dL/ds and dL/dU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.h"
#include "hub_common.h"

using hub::Cl;
using hub::hf_diag;
using hub::make_cl;

namespace {

struct AdjArgs {
    Cl a;                       // stage state (X, Y) and model data
    const void* A;              // stage state G2: binary64, or binary32 (a32) for the
    int a32;                    // mixed-precision stage copies Y2, Y3, Y4
    const cd* gin1;             // cotangent of dG1 (scaled by gscale)
    const cd* gin2;             // cotangent of dG2
    double gscale;
    const cd* lam1;             // lambda (running cotangent of y_n)
    const cd* lam2;
    cd* lacc1;                  // lambda accumulator
    cd* lacc2;
    cd* gnext1;                 // next stage cotangent = alpha lambda + beta mu
    cd* gnext2;
    double alpha, beta;
    int init, has_next;
    cd* red;                    // reduction buffers (see adj_red)
    cd* part;                   // partial sums of the kind-3 lane reduction [nparts][ns][ns][2]
    int pairs_per_part, nparts;
    cd* spart;                  // per-slice partials of kinds 0, 2, 4, 5 [8][ns^3]
    cd* ebar;                   // [2][ns] cotangents of the h^HF diagonals
    double* gpart;              // [2 + blocks of adj_g1e]: partial dL/ds, dL/dU
    double* grads;              // [2]: dL/ds, dL/dU of this stage
};

// reduction buffer layout (each ns^2 complex): RX[6], RY[6], M02, M13, UPART
enum { R_X = 0, R_Y = 6, R_M02 = 12, R_M13 = 13, R_UP = 14, R_N = 15 };

__device__ __forceinline__ cd cmul3(cd a, cd b, cd c) { return cmul(cmul(a, b), c); }

// Element e of the stage state G2 (binary64 arithmetic whatever its storage).
__device__ __forceinline__ cd ld_a(const AdjArgs& s, long long e) {
    return s.a32 ? ld_c(static_cast<const float2*>(s.A), e) : ld_c(static_cast<const cd*>(s.A), e);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ cd wsum(cd v) { return cmk(wsum(v.x), wsum(v.y)); }

// Reductions of the source term (eq:soa-cubic-scheme) differentiated with
// respect to X and Y, B = i gs g the scaled cotangent.  Each kind sums over the
// pair complementary to its free pair:
//   kind 0 free (i,k): X cotangent and M02 = sum conj(A) B
//   kind 1 free (i,j): X and Y cotangents and the U partial Re(conj(Psi/U) B)
//   kind 2 free (j,k), kind 3 free (k,l), kind 4 free (i,l): X and Y cotangents
//   kind 5 free (j,l): Y cotangent and M13 = sum conj(A) B
// Kinds 0, 1, 2, 4 and 5 come from one pass over the cotangent: one work-group
// per (i, j) slice, wave w over the rows k = w, w + 4, ... with lane = l.  Kind
// 1 is summed over the slice; kinds 0 and 2 over l within a row, leaving
// partials per (i, j, k) that adj_slice_fin_kernel sums over j or i; kinds 4
// and 5 over k, leaving partials per (i, j, l).  Kind 3 is adj_lane_red_kernel.
//
// The same pass computes the G2 cotangent mu = i gs [conj(E) g + hop stencil
// applied to g] + collision entries (the commutator stencil is its own
// adjoint up to the conjugate of the diagonal) and updates the running sum and
// the next stage's cotangent: the l-neighbours of the stencil are other lanes
// (cross-lane permute), the other neighbours whole rows; neighbour tables are
// staged in LDS padded to four entries (a missing neighbour is the site itself
// with hopping 0).
__global__ __launch_bounds__(256) void adj_slice_red_kernel(AdjArgs s) {
    constexpr int ZR = 4;
    __shared__ cd sh4[4][4][64];   // per wave and lane: kinds 4 (X, Y) and 5 (Y, M13)
    __shared__ double sh1[4][5];   // per wave: kind 1 (X re, im, Y re, im, U)
    __shared__ cd eu[64], ed[64];
    __shared__ int snb[2 * 64 * ZR];
    __shared__ cd shp[2 * 64 * ZR];
    const Cl& a = s.a;
    const int ns = a.ns, ns2 = ns * ns, ns3 = ns2 * ns, z = a.zmax;
    const int i = blockIdx.x / ns, j = blockIdx.x % ns;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool lane_ok = lane < ns;
    const int l = lane_ok ? lane : 0;
    const cd* X = a.X;
    const cd* Y = a.Y;
    const double U = a.U, gs = s.gscale;
    for (int q = tid; q < ns; q += blockDim.x) {
        eu[q] = hf_diag(a, 0, q);
        ed[q] = hf_diag(a, 1, q);
    }
    for (int q = tid; q < 2 * ns * ZR; q += blockDim.x) {
        const int row = q / ZR, qq = q - row * ZR, site = row % ns;
        const int p = qq < z ? a.nbr[row * z + qq] : -1;
        snb[q] = p >= 0 ? p : site;
        shp[q] = p >= 0 ? a.hop[row * z + qq] : cmk(0.0, 0.0);
    }
    __syncthreads();
    const int* nbu = snb;
    const int* nbd = snb + ns * ZR;
    const cd* hu = shp;
    const cd* hd = shp + ns * ZR;
    const cd* __restrict__ G = s.gin2;
    int src[ZR];
#pragma unroll
    for (int q = 0; q < ZR; ++q) src[q] = lane_ok ? nbd[l * ZR + q] : lane;
    const cd ei = eu[i], ej = ed[j], el = ed[l];
    const cd xij = X[i * ns + j], yji = Y[j * ns + i];
    const cd xil = X[i * ns + l], yjl = Y[j * ns + l], yil = Y[i * ns + l];
    cd x1 = cmk(0, 0), y1 = cmk(0, 0);
    double up = 0.0;
    cd a4x = cmk(0, 0), a4y = cmk(0, 0), a5y = cmk(0, 0), a5m = cmk(0, 0);
    cd* P = s.spart;
    for (int k = wave; k < ns; k += 4) {
        cd r0x = cmk(0, 0), r0m = cmk(0, 0), r2x = cmk(0, 0), r2y = cmk(0, 0);
        const int e = ((i * ns + j) * ns + k) * ns + l;
        const cd g = lane_ok ? G[e] : cmk(0.0, 0.0);
        cd vl[ZR];
#pragma unroll
        for (int q = 0; q < ZR; ++q) {
            vl[q].x = __shfl(g.x, src[q], 64);
            vl[q].y = __shfl(g.y, src[q], 64);
        }
        if (lane_ok) {
            // G2 cotangent of this element
            const cd ek = eu[k];
            const cd E = cmk(ei.x + ej.x - ek.x - el.x, ei.y + ej.y - ek.y - el.y);
            cd hsum = cmul(cconj(E), g);
#pragma unroll
            for (int q = 0; q < ZR; ++q) {
                hsum = cfma(hsum, hu[i * ZR + q], G[e + (nbu[i * ZR + q] - i) * ns3]);
                hsum = cfma(hsum, hd[j * ZR + q], G[e + (nbd[j * ZR + q] - j) * ns2]);
                hsum = csub(hsum, cmul(G[e + (nbu[k * ZR + q] - k) * ns], cconj(hu[k * ZR + q])));
                hsum = csub(hsum, cmul(vl[q], cconj(hd[l * ZR + q])));
            }
            cd mu = cscale(cmul_i(hsum), gs);
            if (j == i && l == i) {
                cd bxa = cscale(cmul_i(s.gin1[i * ns + k]), gs), bxb = cscale(cmul_i(s.gin1[k * ns + i]), gs);
                mu = cadd(mu, cscale(cmul_i(cadd(bxa, cconj(bxb))), a.U));
            }
            if (j == i && k == i) {
                const cd* gy = s.gin1 + ns2;
                cd bya = cscale(cmul_i(gy[i * ns + l]), gs), byb = cscale(cmul_i(gy[l * ns + i]), gs);
                mu = cadd(mu, cscale(cmul_i(cadd(bya, cconj(byb))), a.U));
            }
            const cd base = s.init ? s.lam2[e] : s.lacc2[e];
            s.lacc2[e] = cadd(base, mu);
            if (s.has_next) {
                const cd lv = s.lam2[e];
                s.gnext2[e] = cmk(s.alpha * lv.x + s.beta * mu.x, s.alpha * lv.y + s.beta * mu.y);
            }
            // source-term reductions
            const cd B = cscale(cmul_i(g), gs);
            const cd cav = cconj(ld_a(s, e));
            const cd xik = X[i * ns + k], xjk = X[j * ns + k], yjk = Y[j * ns + k];
            // X_lk = -conj(X_kl) (G^< is anti-Hermitian, as the forward stage reads it): a row
            // read instead of a column gather
            const cd xkl = X[k * ns + l], ykl = Y[k * ns + l];
            const cd xlk = cmk(-xkl.x, xkl.y);
            const double dd = (double)(i == j) - (double)(k == l);
            // kind 0
            cd w0 = cscale(cconj(yjl), U * dd);
            w0 = cadd(w0, cscale(cmul_i(cconj(cmul(yji, yil))), -U));
            w0 = cadd(w0, cscale(cmul_i(cconj(cmul(ykl, yjk))), U));
            r0x = cmul(w0, B);
            r0m = cmul(cav, B);
            // kind 1
            x1 = cfma(x1, cscale(cmul_i(cconj(cmul(xjk, yjl))), -U), B);
            y1 = cfma(y1, cscale(cmul_i(cconj(cmul(yil, xik))), -U), B);
            const cd t1 = cmul(csub(cmul(xij, xjk), cmul(xlk, xil)), yjl);
            const cd t2 = cmul(csub(cmul(yji, yil), cmul(ykl, yjk)), xik);
            const cd psi1 = cadd(cscale(cmul(xik, yjl), dd), cmul_i(cadd(t1, t2)));   // Psi / U
            up += psi1.x * B.x + psi1.y * B.y;
            // kind 2
            r2x = cmul(cscale(cmul_i(cconj(cmul(xij, yjl))), -U), B);
            r2y = cmul(cscale(cmul_i(cconj(cmul(ykl, xik))), U), B);
            // kind 4
            a4x = cfma(a4x, cscale(cmul_i(cconj(cmul(xlk, yjl))), U), B);
            a4y = cfma(a4y, cscale(cmul_i(cconj(cmul(yji, xik))), -U), B);
            // kind 5
            cd w5 = cscale(cconj(xik), U * dd);
            w5 = cadd(w5, cscale(cmul_i(cconj(cmul(xij, xjk))), -U));
            w5 = cadd(w5, cscale(cmul_i(cconj(cmul(xlk, xil))), U));
            a5y = cfma(a5y, w5, B);
            a5m = cfma(a5m, cav, B);
        }
        r0x = wsum(r0x);
        r0m = wsum(r0m);
        r2x = wsum(r2x);
        r2y = wsum(r2y);
        if (lane == 0) {
            const size_t o = ((size_t)i * ns + j) * ns + k;
            P[0 * (size_t)ns3 + o] = r0x;
            P[1 * (size_t)ns3 + o] = r0m;
            P[2 * (size_t)ns3 + o] = r2x;
            P[3 * (size_t)ns3 + o] = r2y;
        }
    }
    sh4[wave][0][lane] = a4x;
    sh4[wave][1][lane] = a4y;
    sh4[wave][2][lane] = a5y;
    sh4[wave][3][lane] = a5m;
    x1 = wsum(x1);
    y1 = wsum(y1);
    up = wsum(up);
    if (lane == 0) {
        sh1[wave][0] = x1.x;
        sh1[wave][1] = x1.y;
        sh1[wave][2] = y1.x;
        sh1[wave][3] = y1.y;
        sh1[wave][4] = up;
    }
    __syncthreads();
    if (wave != 0) return;
    if (lane_ok) {
        const size_t o = ((size_t)i * ns + j) * ns + l;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            P[(4 + q) * (size_t)ns3 + o] = cadd(cadd(sh4[0][q][lane], sh4[1][q][lane]),
                                                cadd(sh4[2][q][lane], sh4[3][q][lane]));
    }
    if (lane == 0) {
        double v[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) v[q] = (sh1[0][q] + sh1[1][q]) + (sh1[2][q] + sh1[3][q]);
        cd* R = s.red;
        R[(R_X + 1) * ns2 + i * ns + j] = cmk(v[0], v[1]);
        R[(R_Y + 1) * ns2 + j * ns + i] = cmk(v[2], v[3]);
        R[R_UP * ns2 + i * ns + j] = cmk(v[4], 0.0);
    }
}

// Kinds 0, 2, 4, 5 from the per-slice partials: one thread per output pair;
// kinds 0 and 4 sum over j, kinds 2 and 5 over i (fixed order).  Threads
// 8 ns^2 .. 9 ns^2 - 1 add up the per-part sums of kind 3 (adj_lane_red).
__global__ __launch_bounds__(256) void adj_slice_fin_kernel(AdjArgs s) {
    const int ns = s.a.ns, ns2 = ns * ns, ns3 = ns2 * ns;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 9 * ns2) return;
    if (t >= 8 * ns2) {   // kind 3: the X cotangent at (l, k), the Y cotangent at (k, l)
        const int kl = t - 8 * ns2, k = kl / ns, l = kl % ns;
        cd v0 = cmk(0, 0), v1 = cmk(0, 0);
        for (int p = 0; p < s.nparts; ++p) {
            const cd* P = s.part + ((size_t)p * ns2 + kl) * 2;
            v0 = cadd(v0, P[0]);
            v1 = cadd(v1, P[1]);
        }
        s.red[(R_X + 3) * ns2 + l * ns + k] = v0;
        s.red[(R_Y + 3) * ns2 + k * ns + l] = v1;
        return;
    }
    const int q = t / ns2, o = t - q * ns2, p0 = o / ns, p1 = o - p0 * ns;
    const bool over_j = q == 0 || q == 1 || q == 4 || q == 5;
    const cd* P = s.spart + (size_t)q * ns3;
    cd v = cmk(0, 0);
    for (int r = 0; r < ns; ++r)
        v = cadd(v, over_j ? P[((size_t)p0 * ns + r) * ns + p1] : P[((size_t)r * ns + p0) * ns + p1]);
    static constexpr int slot[8] = {R_X + 0, R_M02, R_X + 2, R_Y + 2, R_X + 4, R_Y + 4, R_Y + 5, R_M13};
    s.red[slot[q] * ns2 + o] = v;
}

// Kind 3 of the source-term reductions (free (k,l)), with lane = l so that
// every load is a contiguous row.  Work-group (k, part): part a range of the
// summed pairs (i, j) split over the four waves; per-part sums go to s.part and
// adj_slice_fin_kernel adds them up.
__global__ __launch_bounds__(256) void adj_lane_red_kernel(AdjArgs s) {
    __shared__ cd sh[4][2][64];
    const Cl& a = s.a;
    const int ns = a.ns, ns2 = ns * ns;
    const int k = blockIdx.x % ns, part = blockIdx.x / ns;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool lane_ok = lane < ns;
    const int l = lane_ok ? lane : 0;
    const cd* X = a.X;
    const cd* Y = a.Y;
    const double U = a.U, gs = s.gscale;
    cd v0 = cmk(0, 0), v1 = cmk(0, 0);
    const int p0 = part * s.pairs_per_part, p1 = min(ns2, p0 + s.pairs_per_part);
    if (lane_ok) {
        for (int pr = p0 + wave; pr < p1; pr += 4) {
            const int i = pr / ns, j = pr % ns;
            const int e = ((i * ns + j) * ns + k) * ns + l;
            const cd B = cscale(cmul_i(s.gin2[e]), gs);
            v0 = cfma(v0, cscale(cmul_i(cconj(cmul(X[i * ns + l], Y[j * ns + l]))), U), B);
            v1 = cfma(v1, cscale(cmul_i(cconj(cmul(Y[j * ns + k], X[i * ns + k]))), U), B);
        }
    }
    sh[wave][0][lane] = v0;
    sh[wave][1][lane] = v1;
    __syncthreads();
    if (wave == 0 && lane_ok) {
        cd t0 = cadd(cadd(sh[0][0][lane], sh[1][0][lane]), cadd(sh[2][0][lane], sh[3][0][lane]));
        cd t1 = cadd(cadd(sh[0][1][lane], sh[1][1][lane]), cadd(sh[2][1][lane], sh[3][1][lane]));
        cd* P = s.part + ((size_t)part * ns2 + k * ns + l) * 2;
        P[0] = t0;
        P[1] = t1;
    }
}

// Cotangents of the h^HF diagonals (ebar), the drive and U parts that depend
// on them, and the sum of the U partials of the source (one work-group; four
// threads per site).
__global__ __launch_bounds__(256) void adj_e_kernel(AdjArgs s) {
    __shared__ double sh[2][256];
    const Cl& a = s.a;
    const int ns = a.ns, ns2 = ns * ns, t = threadIdx.x;
    const cd* R = s.red;
    const double gs = s.gscale;
    const cd* X = a.X;
    const cd* Y = a.Y;
    const cd* gx = s.gin1;
    const cd* gy = s.gin1 + ns2;
    double sbar = 0.0, ubar = 0.0;
    const int i = t >> 2, sub = t & 3;
    cd eu = cmk(0, 0), ed = cmk(0, 0);
    if (i < ns) {
        for (int p = sub; p < ns; p += 4) {
            // (BX X^H - X^H BX)_ii with BX = i gs gX
            cd bx_ip = cscale(cmul_i(gx[i * ns + p]), gs), bx_pi = cscale(cmul_i(gx[p * ns + i]), gs);
            eu = cadd(eu, csub(cmul(bx_ip, cconj(X[i * ns + p])), cmul(cconj(X[p * ns + i]), bx_pi)));
            cd by_ip = cscale(cmul_i(gy[i * ns + p]), gs), by_pi = cscale(cmul_i(gy[p * ns + i]), gs);
            ed = cadd(ed, csub(cmul(by_ip, cconj(Y[i * ns + p])), cmul(cconj(Y[p * ns + i]), by_pi)));
            eu = cadd(eu, csub(R[R_M02 * ns2 + i * ns + p], R[R_M02 * ns2 + p * ns + i]));
            ed = cadd(ed, csub(R[R_M13 * ns2 + i * ns + p], R[R_M13 * ns2 + p * ns + i]));
        }
    }
    // sum the four partial sums of a site (lanes 4i .. 4i+3)
    for (int o = 1; o < 4; o <<= 1) {
        eu.x += __shfl_xor(eu.x, o, 64);
        eu.y += __shfl_xor(eu.y, o, 64);
        ed.x += __shfl_xor(ed.x, o, 64);
        ed.y += __shfl_xor(ed.y, o, 64);
    }
    if (i < ns && sub == 0) {
        s.ebar[i] = eu;
        s.ebar[ns + i] = ed;
        sbar = a.xdrv[i] * (eu.x + ed.x);
        // e^up_i = ... - i U Y_ii, e^dn_i = ... - i U X_ii: Ubar += Re(conj(-i Y_ii) ebar)
        cd myi = cmul_mi(Y[i * ns + i]), mxi = cmul_mi(X[i * ns + i]);
        ubar = myi.x * eu.x + myi.y * eu.y + mxi.x * ed.x + mxi.y * ed.y;
    }
    for (int q = t; q < ns2; q += blockDim.x) ubar += R[R_UP * ns2 + q].x;
    sh[0][t] = sbar;
    sh[1][t] = ubar;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (t < st) {
            sh[0][t] += sh[0][t + st];
            sh[1][t] += sh[1][t + st];
        }
        __syncthreads();
    }
    if (t == 0) {
        s.gpart[0] = sh[0][0];
        s.gpart[1] = sh[1][0];
    }
}

// G1 cotangents, one thread per element of [X | Y]; partial dL/dU of the
// collision integral per work-group into s.gpart[2 + block].
__global__ __launch_bounds__(256) void adj_g1e_kernel(AdjArgs s) {
    __shared__ double sh[256];
    const Cl& a = s.a;
    const int ns = a.ns, ns2 = ns * ns, z = a.zmax;
    const cd* R = s.red;
    const double gs = s.gscale;
    const cd* gx = s.gin1;
    const cd* gy = s.gin1 + ns2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double ubar = 0.0;
    if (e < 2 * ns2) {
        const int sig = e / ns2, r = e % ns2, i = r / ns, j = r % ns;
        const cd* gg = sig ? gy : gx;
        const cd* eb = s.ebar + (sig ? 0 : ns);   // X_ii enters e^dn, Y_ii enters e^up
        const int* nb = a.nbr + sig * ns * z;
        const cd* hp = a.hop + sig * ns * z;
        // [h^H, B]_ij, B = i gs g
        cd ei = hf_diag(a, sig, i), ej = hf_diag(a, sig, j);
        cd bij = gg[r];
        cd c = csub(cmul(cconj(ei), bij), cmul(bij, cconj(ej)));
        for (int q = 0; q < z; ++q) {
            int p = nb[i * z + q];
            if (p >= 0) c = cfma(c, hp[i * z + q], gg[p * ns + j]);
        }
        for (int q = 0; q < z; ++q) {
            int p = nb[j * z + q];
            if (p >= 0) c = csub(c, cmul(gg[i * ns + p], cconj(hp[j * z + q])));
        }
        cd mu = cscale(cmul_i(c), gs);
        // source-term reductions: X receives kinds 0-4, Y kinds 1-5
        for (int kd = sig ? 1 : 0; kd < (sig ? 6 : 5); ++kd) mu = cadd(mu, R[((sig ? R_Y : R_X) + kd) * ns2 + r]);
        if (i == j) mu = cadd(mu, cscale(cmul_i(eb[i]), a.U));
        // collision-integral part of dL/dU: I_ij = -i U A..., Ibar_ij = B_ij + conj(B_ji)
        cd bb = cadd(cscale(cmul_i(gg[r]), gs), cconj(cscale(cmul_i(gg[j * ns + i]), gs)));
        cd av = sig == 0 ? ld_a(s, ((i * ns + i) * ns + j) * ns + i) : ld_a(s, ((i * ns + i) * ns + i) * ns + j);
        cd dI = cmul_mi(av);   // dI/dU
        ubar = dI.x * bb.x + dI.y * bb.y;
        cd base = s.init ? s.lam1[e] : s.lacc1[e];
        s.lacc1[e] = cadd(base, mu);
        if (s.has_next) {
            cd lv = s.lam1[e];
            s.gnext1[e] = cmk(s.alpha * lv.x + s.beta * mu.x, s.alpha * lv.y + s.beta * mu.y);
        }
    }
    sh[threadIdx.x] = ubar;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) s.gpart[2 + blockIdx.x] = sh[0];
}

// dL/ds and dL/dU of the stage from the partials (fixed summation order).
__global__ void adj_gsum_kernel(AdjArgs s, int nblocks) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double u = s.gpart[1];
    for (int b = 0; b < nblocks; ++b) u += s.gpart[2 + b];
    s.grads[0] = s.gpart[0];
    s.grads[1] = u;
}

// Terminal cotangent of the loss and its value.
__global__ void adj_terminal_kernel(Cl a, const cd* __restrict__ A, const double* __restrict__ wa,
                                    const double* __restrict__ wb, cd* __restrict__ l1,
                                    cd* __restrict__ l2, double* __restrict__ loss) {
    const int ns = a.ns;
    double L = 0.0;
    for (int i = 0; i < ns; ++i) {
        const int ii = i * ns + i;
        const int e = ((i * ns + i) * ns + i) * ns + i;
        double nu = a.X[ii].y, nd = a.Y[ii].y;
        L += wa[i] * (nu * nd - A[e].x) + wb[i] * (nu + nd);
        l1[ii] = cmk(0.0, wa[i] * nd + wb[i]);            // dL/dIm X_ii
        l1[ns * ns + ii] = cmk(0.0, wa[i] * nu + wb[i]);  // dL/dIm Y_ii
        l2[e] = cmk(-wa[i], 0.0);                         // dL/dRe A_iiii
    }
    *loss = L;
}

}  // namespace

// ---------------------------------------------------------------------------- host
namespace {

struct AdjState {
    int64_t nsteps = 0;
    bool mixed = false;        // binary32 G2 stage copies (Y2, Y3, Y4), as the mixed forward stages
    int interval = 0;
    double dt = 0.0, t0 = 0.0;
    int nck = 0;
    std::vector<Regs> ckpt;
    // one segment of the forward pass, recomputed from its checkpoint: the
    // state y_n and the stage states Y2, Y3, Y4 of every step
    std::vector<Regs> seg, seg2, seg3, seg4;
    Regs LAM, LACC, CA, CB;
    cd* red = nullptr;
    cd* part = nullptr;        // kind-3 lane-reduction partials
    cd* spart = nullptr;       // per-slice partials of kinds 0, 2, 4, 5
    int nparts = 0, pairs_per_part = 0;
    cd* ebar = nullptr;
    double* gpart = nullptr;
    double* grads = nullptr;   // [4 nsteps][2]
    double* dev_ab = nullptr;  // weights a, b and the loss
};

constexpr int ADJ_PAIRS_PER_PART = 64;

AdjState* adj_of(g1g2_ctx* c) { return reinterpret_cast<AdjState*>(c->adj); }

// half32: the G2 part holds binary32 values only (a mixed-precision stage copy)
g1g2_status alloc_reg(g1g2_ctx* c, Regs& r, bool half32 = false) {
    HIP_OK(c, hipMalloc(&r.g1, c->n1 * sizeof(cd)));
    HIP_OK(c, hipMalloc(&r.g2, c->n2 * (half32 ? sizeof(float2) : sizeof(cd))));
    return G1G2_OK;
}

void free_reg(Regs& r) {
    if (r.g1) (void)hipFree(r.g1);
    if (r.g2) (void)hipFree(r.g2);
    r = Regs();
}

g1g2_status copy_reg(g1g2_ctx* c, const Regs& dst, const Regs& src) {
    HIP_OK(c, hipMemcpyAsync(dst.g1, src.g1, c->n1 * sizeof(cd), hipMemcpyDeviceToDevice, c->stream));
    HIP_OK(c, hipMemcpyAsync(dst.g2, src.g2, c->n2 * sizeof(cd), hipMemcpyDeviceToDevice, c->stream));
    prof_mark(c, "state_copy");
    return G1G2_OK;
}

// S32: the G2 of S holds binary32 values (a mixed-precision stage copy).
AdjArgs make_adj(g1g2_ctx* c, double t, const Regs& S, bool S32, const Regs& gin, double gscale,
                 const Regs& lam, const Regs& lacc, const Regs& gnext, double alpha, double beta, int init,
                 int has_next, double* grads) {
    HubbardData& H = c->hub;
    AdjState* st = adj_of(c);
    const ClusterDesc& d = H.hdesc[0];
    AdjArgs s;
    Cl a;
    a.ns = d.ns;
    a.zmax = d.zmax;
    a.U = d.U;
    a.s_drive = H.drive_value(t);
    a.nbr = H.nbr;
    a.hop = H.hop;
    a.d0 = H.d0;
    a.xdrv = H.xdrv;
    a.X = S.g1;
    a.Y = S.g1 + d.ns * d.ns;
    s.a = a;
    s.A = S.g2;
    s.a32 = S32 ? 1 : 0;
    s.gin1 = gin.g1;
    s.gin2 = gin.g2;
    s.gscale = gscale;
    s.lam1 = lam.g1;
    s.lam2 = lam.g2;
    s.lacc1 = lacc.g1;
    s.lacc2 = lacc.g2;
    s.gnext1 = gnext.g1;
    s.gnext2 = gnext.g2;
    s.alpha = alpha;
    s.beta = beta;
    s.init = init;
    s.has_next = has_next;
    s.red = st->red;
    s.part = st->part;
    s.spart = st->spart;
    s.pairs_per_part = st->pairs_per_part;
    s.nparts = st->nparts;
    s.ebar = st->ebar;
    s.gpart = st->gpart;
    s.grads = grads;
    return s;
}

g1g2_status vjp(g1g2_ctx* c, const AdjArgs& s) {
    const int ns = s.a.ns, ns2 = ns * ns;
    hipLaunchKernelGGL(adj_slice_red_kernel, dim3(ns2), dim3(256), 0, c->stream, s);
    prof_mark(c, "adj_slice_red");
    hipLaunchKernelGGL(adj_lane_red_kernel, dim3(ns * s.nparts), dim3(256), 0, c->stream, s);
    prof_mark(c, "adj_lane_red");
    hipLaunchKernelGGL(adj_slice_fin_kernel, dim3((9 * ns2 + 255) / 256), dim3(256), 0, c->stream, s);
    prof_mark(c, "adj_slice_fin");
    HIP_OK(c, hipGetLastError());
    const int g1blocks = (2 * ns2 + 255) / 256;
    hipLaunchKernelGGL(adj_e_kernel, dim3(1), dim3(256), 0, c->stream, s);
    prof_mark(c, "adj_e");
    hipLaunchKernelGGL(adj_g1e_kernel, dim3(g1blocks), dim3(256), 0, c->stream, s);
    prof_mark(c, "adj_g1e");
    hipLaunchKernelGGL(adj_gsum_kernel, dim3(1), dim3(64), 0, c->stream, s, g1blocks);
    prof_mark(c, "adj_gsum");
    HIP_OK(c, hipGetLastError());
    return G1G2_OK;
}

g1g2_status stage_fwd(g1g2_ctx* c, int mode, double t, const Regs& in, const Regs& y, const Regs& acc,
                      const Regs& out, double cb, double cc) {
    return hub_stage(c, mode, t, in, y, acc, out, cb, cc);
}

}  // namespace

void adj_free(g1g2_ctx* c) {
    AdjState* st = adj_of(c);
    if (!st) return;
    for (auto* v : {&st->ckpt, &st->seg, &st->seg2, &st->seg3, &st->seg4})
        for (auto& r : *v) free_reg(r);
    for (Regs* r : {&st->LAM, &st->LACC, &st->CA, &st->CB}) free_reg(*r);
    if (st->red) (void)hipFree(st->red);
    if (st->part) (void)hipFree(st->part);
    if (st->spart) (void)hipFree(st->spart);
    if (st->ebar) (void)hipFree(st->ebar);
    if (st->gpart) (void)hipFree(st->gpart);
    if (st->grads) (void)hipFree(st->grads);
    if (st->dev_ab) (void)hipFree(st->dev_ab);
    delete st;
    c->adj = nullptr;
}

extern "C" {

g1g2_status g1g2_forward_checkpointed(g1g2_ctx* c, double dt, int64_t nsteps, int32_t interval) {
    if (!c || nsteps < 1 || !(dt > 0.0)) return G1G2_EINVAL;
    if (c->d.basis != G1G2_HUBBARD || c->d.selfenergy != G1G2_SOA || c->hub.ncl != 1)
        return set_error(c, G1G2_EUNSUPPORTED, "the adjoint covers the single-cluster Hubbard SOA system");
    if (c->hub.hdesc[0].ns > 64) return set_error(c, G1G2_EUNSUPPORTED, "adjoint supports ns <= 64");
    if (c->has_switch())
        return set_error(c, G1G2_EUNSUPPORTED, "the adjoint takes a constant U (switching is set)");
    adj_free(c);
    AdjState* st = new AdjState();
    c->adj = st;
    st->nsteps = nsteps;
    st->mixed = c->d.precision == G1G2_MIXED;
    // default: the interval that minimizes checkpoints + four states per segment step
    st->interval = interval > 0 ? interval
                                : std::max<int>(1, (int)std::ceil(std::sqrt((double)nsteps / 4.0)));
    st->dt = dt;
    st->t0 = c->t;
    st->nck = (int)((nsteps + st->interval - 1) / st->interval);
    g1g2_status s;
    st->ckpt.resize(st->nck + 1);       // last slot keeps the final state
    for (auto& r : st->ckpt)
        if ((s = alloc_reg(c, r)) != G1G2_OK) return s;
    for (auto* v : {&st->seg, &st->seg2, &st->seg3, &st->seg4}) {
        v->resize(st->interval);
        for (auto& r : *v)
            if ((s = alloc_reg(c, r, st->mixed && v != &st->seg)) != G1G2_OK) return s;
    }
    for (Regs* r : {&st->LAM, &st->LACC, &st->CA, &st->CB})
        if ((s = alloc_reg(c, *r)) != G1G2_OK) return s;
    const int ns = c->hub.hdesc[0].ns;
    HIP_OK(c, hipMalloc(&st->red, (size_t)R_N * ns * ns * sizeof(cd)));
    HIP_OK(c, hipMemsetAsync(st->red, 0, (size_t)R_N * ns * ns * sizeof(cd), c->stream));
    st->pairs_per_part = ADJ_PAIRS_PER_PART;
    st->nparts = (ns * ns + ADJ_PAIRS_PER_PART - 1) / ADJ_PAIRS_PER_PART;
    HIP_OK(c, hipMalloc(&st->part, (size_t)st->nparts * ns * ns * 2 * sizeof(cd)));
    HIP_OK(c, hipMalloc(&st->spart, (size_t)8 * ns * ns * ns * sizeof(cd)));
    HIP_OK(c, hipMalloc(&st->ebar, (size_t)2 * ns * sizeof(cd)));
    HIP_OK(c, hipMalloc(&st->gpart, (size_t)(2 + (2 * ns * ns + 255) / 256) * sizeof(double)));
    HIP_OK(c, hipMalloc(&st->grads, (size_t)4 * nsteps * 2 * sizeof(double)));
    HIP_OK(c, hipMalloc(&st->dev_ab, (size_t)(2 * ns + 8) * sizeof(double)));
    for (int q = 0; q < st->nck; ++q) {
        if ((s = copy_reg(c, st->ckpt[q], c->y)) != G1G2_OK) return s;
        const int64_t n = std::min<int64_t>(st->interval, nsteps - (int64_t)q * st->interval);
        if ((s = g1g2_step_rk4(c, dt, n)) != G1G2_OK) return s;
    }
    return copy_reg(c, st->ckpt[st->nck], c->y);
}

g1g2_status g1g2_adjoint(g1g2_ctx* c, const double* wa, const double* wb, double* grad_c,
                         double* grad_U, double* loss) {
    if (!c || !wa || !wb) return G1G2_EINVAL;
    AdjState* st = adj_of(c);
    if (!st) return set_error(c, G1G2_ESTATE, "call g1g2_forward_checkpointed first");
    HubbardData& H = c->hub;
    const int ns = H.hdesc[0].ns;
    const double dt = st->dt;
    g1g2_status s;
    // terminal cotangent
    HIP_OK(c, hipMemcpyAsync(st->dev_ab, wa, ns * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipMemcpyAsync(st->dev_ab + ns, wb, ns * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipMemsetAsync(st->LAM.g1, 0, c->n1 * sizeof(cd), c->stream));
    HIP_OK(c, hipMemsetAsync(st->LAM.g2, 0, c->n2 * sizeof(cd), c->stream));
    prof_mark(c, "adj_init");
    {
        const Regs& fin = st->ckpt[st->nck];
        AdjArgs tmp = make_adj(c, st->t0 + st->nsteps * dt, fin, false, fin, 1.0, fin, fin, fin, 0, 0, 0, 0, nullptr);
        hipLaunchKernelGGL(adj_terminal_kernel, dim3(1), dim3(1), 0, c->stream, tmp.a, fin.g2, st->dev_ab,
                           st->dev_ab + ns, st->LAM.g1, st->LAM.g2, st->dev_ab + 2 * ns);
        HIP_OK(c, hipGetLastError());
        prof_mark(c, "adj_terminal");
    }
    Regs lam = st->LAM, lacc = st->LACC;
    for (int q = st->nck - 1; q >= 0; --q) {
        const int64_t n0 = (int64_t)q * st->interval;
        const int64_t n1 = std::min<int64_t>(n0 + st->interval, st->nsteps);
        // recompute the segment forward, keeping y_n and the stage states of every step
        if ((s = copy_reg(c, c->y, st->ckpt[q])) != G1G2_OK) return s;
        for (int64_t n = n0; n < n1; ++n) {
            const int m = (int)(n - n0);
            if ((s = copy_reg(c, st->seg[m], c->y)) != G1G2_OK) return s;
            const double t = st->t0 + (double)n * dt;
            if ((s = stage_fwd(c, RK_FIRST, t, c->y, c->y, c->acc, st->seg2[m], dt / 6.0, dt / 2.0)) != G1G2_OK) return s;
            if ((s = stage_fwd(c, RK_MID, t + 0.5 * dt, st->seg2[m], c->y, c->acc, st->seg3[m], dt / 3.0, dt / 2.0)) != G1G2_OK) return s;
            if ((s = stage_fwd(c, RK_MID, t + 0.5 * dt, st->seg3[m], c->y, c->acc, st->seg4[m], dt / 3.0, dt)) != G1G2_OK) return s;
            if (n + 1 < n1)
                if ((s = stage_fwd(c, RK_LAST, t + dt, st->seg4[m], c->y, c->acc, c->y, dt / 6.0, 0.0)) != G1G2_OK) return s;
        }
        // reverse over the segment: Y2 = y + dt/2 k1, Y3 = y + dt/2 k2, Y4 = y + dt k3
        for (int64_t n = n1 - 1; n >= n0; --n) {
            const int m = (int)(n - n0);
            const Regs& y = st->seg[m];
            const double t = st->t0 + (double)n * dt;
            double* g = st->grads + (size_t)8 * n;
            const bool m32 = st->mixed;   // the stage copies Y2, Y3, Y4 are binary32 in mixed precision
            if ((s = vjp(c, make_adj(c, t + dt, st->seg4[m], m32, lam, dt / 6.0, lam, lacc, st->CA, dt / 3.0, dt, 1, 1, g + 6))) != G1G2_OK) return s;
            if ((s = vjp(c, make_adj(c, t + 0.5 * dt, st->seg3[m], m32, st->CA, 1.0, lam, lacc, st->CB, dt / 3.0, dt / 2.0, 0, 1, g + 4))) != G1G2_OK) return s;
            if ((s = vjp(c, make_adj(c, t + 0.5 * dt, st->seg2[m], m32, st->CB, 1.0, lam, lacc, st->CA, dt / 6.0, dt / 2.0, 0, 1, g + 2))) != G1G2_OK) return s;
            if ((s = vjp(c, make_adj(c, t, y, false, st->CA, 1.0, lam, lacc, st->CB, 0.0, 0.0, 0, 0, g + 0))) != G1G2_OK) return s;
            std::swap(lam, lacc);
        }
    }
    // restore the final state
    if ((s = copy_reg(c, c->y, st->ckpt[st->nck])) != G1G2_OK) return s;
    std::vector<double> gr((size_t)8 * st->nsteps);
    double L = 0.0;
    HIP_OK(c, hipMemcpyAsync(gr.data(), st->grads, gr.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipMemcpyAsync(&L, st->dev_ab + 2 * ns, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    const double cs[4] = {0.0, 0.5, 0.5, 1.0};
    const int M = (int)H.drive_c.size();
    double gU = 0.0;
    if (grad_c)
        for (int m = 0; m < M; ++m) grad_c[m] = 0.0;
    for (int64_t n = 0; n < st->nsteps; ++n)
        for (int q = 0; q < 4; ++q) {
            const double sb = gr[8 * n + 2 * q], ub = gr[8 * n + 2 * q + 1];
            gU += ub;
            const double ts = st->t0 + ((double)n + cs[q]) * dt;
            if (grad_c)
                for (int m = 0; m < M; ++m) {
                    const double d = ts - H.drive_tc[m];
                    grad_c[m] += sb * std::exp(-d * d / (2.0 * H.drive_tau * H.drive_tau));
                }
        }
    if (grad_U) *grad_U = gU;
    if (loss) *loss = L;
    return G1G2_OK;
}

}  // extern "C"
