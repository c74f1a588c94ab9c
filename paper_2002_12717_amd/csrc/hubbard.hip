// Hubbard-basis G1-G2 kernels (Sec. III.D, Sec. V.A, Sec. VII).
//
// State per cluster: G1 = [X | Y] with X = G^{<,up}, Y = G^{<,down} (ns x ns
// each) and G2 = A = G2^{up down up down} ([ns]^4; GW and DSL add the
// equal-spin channels B and C).  Every G2 element is produced from a fixed number of
// neighbours, so a stage is a bandwidth-bound stream: the O(ns^5) sums of the
// direct formulation are replaced by the paper's reformulations that carry no
// inner sum (eq:soa-cubic-scheme for the source, the sparse-h commutator of
// Sec. VII.A, the reformulated ladders of Sec. VII.C, the polarization of
// Sec. VII.B).  Three stage kernels compute the same right-hand side: the
// slice kernel (whole (i,j) slices staged in LDS), the row kernel (one wave
// per G2 row) and the per-element kernel (any lattice; not GW or DSL).
//
// A context holds a ragged batch of clusters.  One launch per Runge-Kutta
// stage processes a flat work list: every item is either a range of one
// cluster's G2 (slices, rows or elements, by kernel) or the G1 update of one
// cluster.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "ctx.h"
#include "hub_common.h"

namespace {

using hub::Cl;
using hub::hf_diag;
using hub::make_cl;

// Selfenergies of the stage kernels.  DSL (Sec. VI) is GW on the three
// channels with both ladders added on channel A.
enum { SE_SOA = 0, SE_TPP = 1, SE_TPH = 2, SE_GW = 3, SE_DSL = 4 };

__host__ __device__ constexpr bool has_pol(int se) { return se == SE_GW || se == SE_DSL; }
__host__ __device__ constexpr bool has_pp(int se) { return se == SE_TPP || se == SE_DSL; }
__host__ __device__ constexpr bool has_ph(int se) { return se == SE_TPH || se == SE_DSL; }

// G2 channels stored per cluster and diagonal tensors gathered per stage
// (GW's six layouts first, then the particle-hole ladder's two).
__host__ __device__ constexpr int n_channels(int se) { return has_pol(se) ? 3 : 1; }
__host__ __device__ constexpr int n_diag(int se) { return (has_pol(se) ? 6 : 0) + (has_ph(se) ? 2 : 0); }

// Right-hand side of one element e = ((i ns + j) ns + k) ns + l of the
// cluster's block A = G2^{up down up down}:
//   dA/dt = -i ( [h2_{ud}, A] + Psi + [L - (L_klij)^*] ),
// L the particle-particle (TPP) or particle-hole (TPH) ladder, none for SOA.
// PRE: the diagonals of h^{HF} are read from a.hdg (computed once per stage);
// RH: every hopping is real and read from a.hopr (a real-by-complex product)
template <int SE, typename TA, bool PRE = false, bool RH = false>
__device__ __forceinline__ cd hub_g2_rhs(const Cl& a, const TA* __restrict__ A, int i, int j, int k,
                                         int l, int e, cd aval) {
    const int ns = a.ns, ns2 = ns * ns, ns3 = ns2 * ns, z = a.zmax;
    const int* nbu = a.nbr;
    const int* nbd = a.nbr + ns * z;
    const cd* hu = a.hop;
    const cd* hd = a.hop + ns * z;
    // two-particle commutator (Sec. VII.A with the on-site terms of h0 + drive)
    cd ei, ej, ek, el;
    if constexpr (PRE) {
        ei = a.hdg[i];
        ej = a.hdg[ns + j];
        ek = a.hdg[k];
        el = a.hdg[ns + l];
    } else {
        ei = hf_diag(a, 0, i);
        ej = hf_diag(a, 1, j);
        ek = hf_diag(a, 0, k);
        el = hf_diag(a, 1, l);
    }
    cd c = cmul(cmk(ei.x + ej.x - ek.x - el.x, ei.y + ej.y - ek.y - el.y), aval);
    const double* hru = a.hopr;
    const double* hrd = a.hopr + ns * z;
    // acc + h v for a real hopping h
    auto rfma = [](cd acc, double h, cd v) { return cmk(fma(h, v.x, acc.x), fma(h, v.y, acc.y)); };
    for (int q = 0; q < z; ++q) {
        int p = nbu[i * z + q];
        if (p >= 0) {
            const cd v = ld_c(A, e + (p - i) * ns3);
            c = RH ? rfma(c, hru[i * z + q], v) : cfma(c, hu[i * z + q], v);
        }
    }
    for (int q = 0; q < z; ++q) {
        int p = nbd[j * z + q];
        if (p >= 0) {
            const cd v = ld_c(A, e + (p - j) * ns2);
            c = RH ? rfma(c, hrd[j * z + q], v) : cfma(c, hd[j * z + q], v);
        }
    }
    cd r = cmk(0.0, 0.0);
    for (int q = 0; q < z; ++q) {  // sum_p A_ijpl h_pk, h_pk = conj(h_kp)
        int p = nbu[k * z + q];
        if (p >= 0) {
            const cd v = ld_c(A, e + (p - k) * ns);
            r = RH ? rfma(r, hru[k * z + q], v) : cfma_conjb(r, v, hu[k * z + q]);
        }
    }
    for (int q = 0; q < z; ++q) {  // sum_p A_ijkp h_pl
        int p = nbd[l * z + q];
        if (p >= 0) {
            const cd v = ld_c(A, e + (p - l));
            r = RH ? rfma(r, hrd[l * z + q], v) : cfma_conjb(r, v, hd[l * z + q]);
        }
    }
    c = csub(c, r);
    // source Psi = U Phi / (i)^2 with Phi from eq:soa-cubic-scheme
    const cd* X = a.X;
    const cd* Y = a.Y;
    cd xik = X[i * ns + k], xij = X[i * ns + j], xjk = X[j * ns + k], xlk = X[l * ns + k],
       xil = X[i * ns + l];
    cd yjl = Y[j * ns + l], yji = Y[j * ns + i], yil = Y[i * ns + l], ykl = Y[k * ns + l],
       yjk = Y[j * ns + k];
    double dd = (double)(i == j) - (double)(k == l);
    cd t1 = cmul(csub(cmul(xij, xjk), cmul(xlk, xil)), yjl);
    cd t2 = cmul(csub(cmul(yji, yil), cmul(ykl, yjk)), xik);
    cd psi = cadd(cscale(cmul(xik, yjl), a.U * dd), cscale(cmul_i(cadd(t1, t2)), a.U));
    c = cadd(c, psi);
    if (SE == SE_TPH) {
        // L_ijkl = i U (Y_il A_ijki - X_il A_ljkl)   (Sec. VII.C)
        cd a1 = ld_c(A, ((i * ns + j) * ns + k) * ns + i), a2 = ld_c(A, ((l * ns + j) * ns + k) * ns + l);
        cd l1 = cmul_i(csub(cmul(yil, a1), cmul(xil, a2)));
        cd b1 = ld_c(A, ((k * ns + l) * ns + i) * ns + k), b2 = ld_c(A, ((j * ns + l) * ns + i) * ns + j);
        cd ykj = Y[k * ns + j], xkj = X[k * ns + j];
        cd l2 = cmul_i(csub(cmul(ykj, b1), cmul(xkj, b2)));
        c = cadd(c, cscale(csub(l1, cconj(l2)), a.U));
    }
    if (SE == SE_TPP) {
        // L_ijkl = delta_ij U A_iikl + i U (Y_ji A_iikl + X_ij A_jjkl)   (Sec. VII.C)
        const int kl = k * ns + l, ij = i * ns + j;
        cd dii = ld_c(A, (i * ns + i) * ns2 + kl), djj = ld_c(A, (j * ns + j) * ns2 + kl);
        cd l1 = cmul_i(cadd(cmul(yji, dii), cmul(xij, djj)));
        if (i == j) l1 = cadd(l1, dii);
        cd dkk = ld_c(A, (k * ns + k) * ns2 + ij), dll = ld_c(A, (l * ns + l) * ns2 + ij);
        cd ylk = Y[l * ns + k], xkl = X[k * ns + l];
        cd l2 = cmul_i(cadd(cmul(ylk, dkk), cmul(xkl, dll)));
        if (k == l) l2 = cadd(l2, dkk);
        c = cadd(c, cscale(csub(l1, cconj(l2)), a.U));
    }
    return cmul_mi(c);
}

// G1 equations (eq:eom_g1_hubbard): dG^{<,s}/dt = -i([h^{HF,s}, G^{<,s}] + I^s + I^s^dagger)
// with I^up_ij = -i U A_iiji and I^down_ij = -i U A_iiij.
template <typename TA>
__device__ __forceinline__ cd hub_g1_rhs(const Cl& a, const TA* __restrict__ A, int sig, int i, int j) {
    const int ns = a.ns, z = a.zmax;
    const cd* G = sig ? a.Y : a.X;
    const int* nb = a.nbr + sig * ns * z;
    const cd* hp = a.hop + sig * ns * z;
    cd gij = G[i * ns + j];
    cd ei = hf_diag(a, sig, i), ej = hf_diag(a, sig, j);
    cd c = csub(cmul(ei, gij), cmul(gij, ej));
    for (int q = 0; q < z; ++q) {
        int p = nb[i * z + q];
        if (p >= 0) c = cfma(c, hp[i * z + q], G[p * ns + j]);
    }
    for (int q = 0; q < z; ++q) {
        int p = nb[j * z + q];
        if (p >= 0) c = csub(c, cmul(G[i * ns + p], cconj(hp[j * z + q])));
    }
    cd Iij, Iji;
    if (sig == 0) {
        Iij = ld_c(A, ((i * ns + i) * ns + j) * ns + i);
        Iji = ld_c(A, ((j * ns + j) * ns + i) * ns + j);
    } else {
        Iij = ld_c(A, ((i * ns + i) * ns + i) * ns + j);
        Iji = ld_c(A, ((j * ns + j) * ns + j) * ns + i);
    }
    // I = -i U A...,  I + I^dagger with (I^dagger)_ij = conj(I_ji)
    cd coll = cadd(cscale(cmul_mi(Iij), a.U), cconj(cscale(cmul_mi(Iji), a.U)));
    return cmul_mi(cadd(c, coll));
}

struct StageArgs {
    const ClusterDesc* __restrict__ desc;
    const WorkItem* __restrict__ work;
    const int* __restrict__ nbr;
    const cd* __restrict__ hop;
    const double* __restrict__ d0;
    const double* __restrict__ xdrv;
    double s_drive;
    double u_scale;   // switching factor phi(t) of the stage
    const cd* in1;
    const cd* in2;
    const cd* y1;
    const cd* y2;
    cd* acc1;
    cd* acc2;
    cd* out1;
    cd* out2;
    double cb, cc;
    DivGuard guard;
    const cd* diag;   // per cluster: GW's six [ns]^3 layouts, then TPH's R and S (hub_diag_kernel)
};

// Storage of the G2 stage registers.  Mixed precision keeps the stage copies
// (the inputs of stages 2-4 and the outputs of stages 1-3) in binary32; y and
// acc, and every G1 register, stay binary64.
template <int MODE, bool MIXED>
struct StageTypes {
    using In = typename std::conditional<MIXED && (MODE == RK_MID || MODE == RK_LAST), float2, cd>::type;
    using Out = typename std::conditional<MIXED && (MODE == RK_FIRST || MODE == RK_MID), float2, cd>::type;
};

template <int MODE, int SE, bool MIXED>
__global__ __launch_bounds__(256) void hub_stage_kernel(StageArgs s) {
    using TI = typename StageTypes<MODE, MIXED>::In;
    using TO = typename StageTypes<MODE, MIXED>::Out;
    const WorkItem w = s.work[blockIdx.x];
    const ClusterDesc d = s.desc[w.cluster];
    const Cl a = make_cl(d, s.nbr, s.hop, s.d0, s.xdrv, s.in1, s.s_drive, s.u_scale);
    const int ns = d.ns;
    const TI* A = reinterpret_cast<const TI*>(s.in2) + d.g2off;
    if (w.start >= 0) {
        const cd* y = s.y2 + d.g2off;
        cd* acc = s.acc2 + d.g2off;
        TO* out = reinterpret_cast<TO*>(s.out2) + d.g2off;
        for (int e = w.start + threadIdx.x; e < w.end; e += blockDim.x) {
            int l = e % ns, tq = e / ns;
            int k = tq % ns;
            tq /= ns;
            int j = tq % ns, i = tq / ns;
            cd av = ld_c(A, e);
            cd f = hub_g2_rhs<SE, TI>(a, A, i, j, k, l, e, av);
            rk_update<MODE>(e, f, av, y, acc, out, s.cb, s.cc);
        }
    } else {
        const cd* g1 = s.in1 + d.g1off;
        const cd* y = s.y1 + d.g1off;
        cd* acc = s.acc1 + d.g1off;
        cd* out = s.out1 + d.g1off;
        const int ns2 = ns * ns;
        if (MODE == RK_FIRST && w.cluster == 0 && threadIdx.x == 0) guard_begin_step(s.guard);
        const unsigned long long step = MODE == RK_LAST ? s.guard.div[0] : 0ull;
        for (int e = threadIdx.x; e < 2 * ns2; e += blockDim.x) {
            int sig = e / ns2, r = e % ns2, i = r / ns, j = r % ns;
            cd f = hub_g1_rhs(a, A, sig, i, j);
            rk_update<MODE>(e, f, g1[e], y, acc, out, s.cb, s.cc);
            if (MODE == RK_LAST && guard_bad(out[e], i == j)) guard_fire(s.guard, w.cluster, step);
        }
    }
}

// "Diagonal" elements of the stage input that the ladder and polarization
// terms need, gathered once per stage into contiguous layouts so that the
// stage kernel reads them as rows (a work item is a range [start, end) of the
// ns^3 index triples of one cluster):
//   TPH (channel A = G2^{up dn up dn}):
//     R[a][b][c] = A_cabc,  S[b][c][a] = A_cabc
//   GW (channels A, B = G2^{up up up up}, C = G2^{dn dn dn dn}):
//     UA[a][c][b] = A_abcb, TA[b][c][a] = A_abcb, VA[b][d][a] = A_abad,
//     WA[a][d][b] = A_abad, UB[a][c][b] = B_abcb, TC[b][c][a] = C_abcb
//   DSL: the six GW layouts, then R and S
template <typename TI, int SE>
__global__ __launch_bounds__(256) void hub_diag_kernel(const ClusterDesc* __restrict__ desc,
                                                      const WorkItem* __restrict__ dwork,
                                                      const cd* __restrict__ in2, cd* __restrict__ diag) {
    const WorkItem w = dwork[blockIdx.x];
    const ClusterDesc d = desc[w.cluster];
    const int ns = d.ns, ns2 = ns * ns, ns3 = ns2 * ns;
    const long long n4 = (long long)ns2 * ns2;
    const TI* A = reinterpret_cast<const TI*>(in2) + d.g2off;
    cd* D = diag + (long long)n_diag(SE) * d.doff;
    cd* DRS = D + (has_pol(SE) ? 6 * ns3 : 0);
    for (int t = w.start + threadIdx.x; t < w.end; t += blockDim.x) {
        const int x = t / ns2, y = (t / ns) % ns, z = t % ns;
        if (has_ph(SE)) {   // (x, y, z) = (a, b, c)
            const cd v = ld_c(A, ((z * ns + x) * ns + y) * ns + z);
            DRS[t] = v;
            DRS[ns3 + (y * ns + z) * ns + x] = v;
        }
        if (has_pol(SE)) {
            // (x, y, z) = (a, b, c): P_abcb of A, B, C
            const long long e1 = ((x * ns + y) * ns + z) * ns + y;
            const cd va = ld_c(A, e1), vb = ld_c(A, n4 + e1), vc = ld_c(A, 2 * n4 + e1);
            D[(x * ns + z) * ns + y] = va;                   // UA
            D[ns3 + (y * ns + z) * ns + x] = va;             // TA
            D[4 * ns3 + (x * ns + z) * ns + y] = vb;         // UB
            D[5 * ns3 + (y * ns + z) * ns + x] = vc;         // TC
            // (x, y, z) = (a, b, d): A_abad
            const cd vd = ld_c(A, ((x * ns + y) * ns + x) * ns + z);
            D[2 * ns3 + (y * ns + z) * ns + x] = vd;         // VA
            D[3 * ns3 + (x * ns + z) * ns + y] = vd;         // WA
        }
    }
}

// Row version of the stage (every cluster has ns <= 64 and at most Z_MAX_ROW
// neighbours per site).  A wave evaluates rpw = min(64 / ns, ns) rows
// A[i][j][k][:] of one (i, j) slice at a time, lane = r ns + l.  The
// l-neighbours of the commutator are other lanes of the same row (cross-lane
// permute); k-, i- and j-neighbours are whole rows read from global memory.
// Values that depend only on (i, j) or on l are loaded once per slice.  The
// source term reads X_lk as -conj(X_kl) and the ladder Y_lk as -conj(Y_kl)
// (G^< is anti-Hermitian), so that every operand row is contiguous.
//
// A work item is a range [start, end) of wave units u = slice * nkb + kb,
// nkb = ceil(ns / rpw); wave w of the work-group takes units start + w,
// start + w + 4, ...
constexpr int NS_MAX_ROW = 64;
constexpr int Z_MAX_ROW = 4;

// A wave-uniform value moved to scalar registers.
__device__ __forceinline__ double wave_uniform(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b & 0xffffffffLL));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ cd wave_uniform(cd v) { return cmk(wave_uniform(v.x), wave_uniform(v.y)); }
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Element i of an array below 4 GiB, addressed as base + 32-bit byte offset:
// with a wave-uniform base the load takes the scalar-base + vector-offset form
// and needs no 64-bit address arithmetic per lane.
template <typename T>
__device__ __forceinline__ cd ldo(const T* __restrict__ p, unsigned i) {
    return ld_c(reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + i * (unsigned)sizeof(T)), 0);
}

// REALH: every hopping of the launch is real (h_pq = h_qp), so each neighbour
// term is a real-by-complex product.
template <int MODE, int SE, bool MIXED, bool REALH>
__global__ __launch_bounds__(256) void hub_row_kernel(StageArgs s) {
    constexpr bool TPP = has_pp(SE), TPH = has_ph(SE), GW = has_pol(SE);
    using TI = typename StageTypes<MODE, MIXED>::In;
    using TO = typename StageTypes<MODE, MIXED>::Out;
    constexpr int ZR = Z_MAX_ROW;
    __shared__ cd eu[NS_MAX_ROW], ed[NS_MAX_ROW];
    // neighbour tables padded to ZR entries per site: a missing neighbour points
    // at the site itself with hopping 0, so every neighbour sum is branch-free
    __shared__ int snb[2 * NS_MAX_ROW * ZR];
    __shared__ int sok[2 * NS_MAX_ROW * ZR];   // (p - site) ns: element offset of a k-neighbour row
    __shared__ cd shp[2 * NS_MAX_ROW * ZR];
    const WorkItem w = s.work[blockIdx.x];
    const ClusterDesc d = s.desc[w.cluster];
    const Cl a = make_cl(d, s.nbr, s.hop, s.d0, s.xdrv, s.in1, s.s_drive, s.u_scale);
    const int ns = d.ns, z = d.zmax, ns2 = ns * ns, ns3 = ns2 * ns;
    const TI* __restrict__ A = reinterpret_cast<const TI*>(s.in2) + d.g2off;
    const int tid = threadIdx.x;
    if (w.start < 0) {  // G1 update of the cluster
        const cd* g1 = s.in1 + d.g1off;
        const cd* y = s.y1 + d.g1off;
        cd* acc = s.acc1 + d.g1off;
        cd* out = s.out1 + d.g1off;
        if (MODE == RK_FIRST && w.cluster == 0 && tid == 0) guard_begin_step(s.guard);
        const unsigned long long step = MODE == RK_LAST ? s.guard.div[0] : 0ull;
        for (int e = tid; e < 2 * ns2; e += blockDim.x) {
            int sig = e / ns2, r = e % ns2, i = r / ns, j = r % ns;
            cd f = hub_g1_rhs(a, A, sig, i, j);
            rk_update<MODE>(e, f, g1[e], y, acc, out, s.cb, s.cc);
            if (MODE == RK_LAST && guard_bad(out[e], i == j)) guard_fire(s.guard, w.cluster, step);
        }
        return;
    }
    for (int q = tid; q < ns; q += blockDim.x) {
        eu[q] = hf_diag(a, 0, q);
        ed[q] = hf_diag(a, 1, q);
    }
    for (int q = tid; q < 2 * ns * ZR; q += blockDim.x) {
        const int row = q / ZR, qq = q - row * ZR, site = row % ns;
        const int p = qq < z ? a.nbr[row * z + qq] : -1;
        snb[q] = p >= 0 ? p : site;
        sok[q] = p >= 0 ? (p - site) * ns : 0;
        shp[q] = p >= 0 ? a.hop[row * z + qq] : cmk(0.0, 0.0);
    }
    __syncthreads();
    // neighbour tables and h^HF diagonals per index slot (i, j, k, l): spin
    // up on i, k and down on j, l for A; the equal-spin GW channels B and C
    // use spin up or spin down on all four
    const int* nbu = snb;
    const int* nbd = snb + ns * ZR;
    const cd* hu = shp;
    const cd* hd = shp + ns * ZR;
    const int *nbI = nbu, *nbJ = nbd, *nbL = nbd;
    const int* okK = sok;   // k-neighbour offsets for the spin of the k index
    const cd *hI = hu, *hJ = hd, *hK = hu, *hL = hd;
    const cd *eI = eu, *eJ = ed, *eK = eu, *eL = ed;
    const cd* __restrict__ X = a.X;
    const cd* __restrict__ Y = a.Y;
    const long long n4 = (long long)ns2 * ns2;
    const int rpw = min(64 / ns, ns);
    const int nkb = (ns + rpw - 1) / rpw;
    const int lane = tid & 63;
    const int sub = lane / ns, l = lane - sub * ns;
    const bool lane_ok = sub < rpw;
    // l-neighbours: source lanes of the permute (the lane itself where there is none)
    int src[ZR];
#pragma unroll
    for (int q = 0; q < ZR; ++q) src[q] = lane_ok ? sub * ns + nbL[l * ZR + q] : lane;
    cd el = lane_ok ? eL[l] : cmk(0.0, 0.0);
    // per slice: element offsets of the i- and j-neighbour rows (wave-uniform)
    int oI[ZR], oJ[ZR];
    // first unit of this wave; units run over channel, slice, k-block
    int u = w.start + __builtin_amdgcn_readfirstlane(tid >> 6);
    int slice = u / nkb, kb = u - slice * nkb;   // slice counts (channel, i, j)
    int cur = -1, ch = 0;
    int i = 0, j = 0;
    const TI* __restrict__ Ach = A;
    const cd* y = s.y2 + d.g2off;
    cd* acc = s.acc2 + d.g2off;
    TO* out = reinterpret_cast<TO*>(s.out2) + d.g2off;
    // GW: diagonal tensors and the G1 blocks of the two polarization terms
    const cd* __restrict__ DG = GW ? s.diag + (long long)n_diag(SE) * d.doff : nullptr;
    const cd *D1 = nullptr, *D2 = nullptr, *S1 = Y, *S2 = X;
    cd ei = cmk(0, 0), ej = cmk(0, 0), xij = cmk(0, 0), yji = cmk(0, 0);
    cd xil = cmk(0, 0), yjl = cmk(0, 0), yil = cmk(0, 0), dll = cmk(0, 0), sijl = cmk(0, 0);
    double dij = 0.0;
    // R[a][b][c] and S[b][c][a], after GW's six layouts for DSL
    const cd* __restrict__ DR = TPH ? s.diag + (long long)n_diag(SE) * d.doff + (GW ? 6 * ns3 : 0) : nullptr;
    const cd* __restrict__ DS = TPH ? DR + ns3 : nullptr;
    for (; u < w.end; u += 4) {
        if (slice != cur) {   // wave-uniform
            cur = slice;
            if (GW) {
                const int nch = slice / ns2;
                if (nch != ch || D1 == nullptr) {
                    ch = nch;
                    const int* nbs = ch == 2 ? nbd : nbu;
                    const cd* hs = ch == 2 ? hd : hu;
                    const cd* es = ch == 2 ? ed : eu;
                    nbI = ch == 0 ? nbu : nbs;
                    nbJ = ch == 0 ? nbd : nbs;
                    okK = (ch == 2) ? sok + ns * ZR : sok;
                    nbL = nbJ;
                    hI = ch == 0 ? hu : hs;
                    hJ = ch == 0 ? hd : hs;
                    hK = hI;
                    hL = hJ;
                    eI = ch == 0 ? eu : es;
                    eJ = ch == 0 ? ed : es;
                    eK = eI;
                    eL = eJ;
#pragma unroll
                    for (int q = 0; q < ZR; ++q) src[q] = lane_ok ? sub * ns + nbL[l * ZR + q] : lane;
                    el = lane_ok ? eL[l] : cmk(0.0, 0.0);
                    Ach = A + ch * n4;
                    y = s.y2 + d.g2off + ch * n4;
                    acc = s.acc2 + d.g2off + ch * n4;
                    out = reinterpret_cast<TO*>(s.out2) + d.g2off + ch * n4;
                    // Pi_1 = -i U S1_jl (D1[i][k][j] - D1[i][k][l]),
                    // Pi_2 = -i U S2_ki (D2[k][j][l] - D2[i][j][l]), term Pi_1 - conj(Pi_2)
                    const long long n3 = (long long)ns2 * ns;
                    D1 = DG + (ch == 0 ? 4 : (ch == 1 ? 0 : 2)) * n3;   // UB, UA, VA
                    D2 = DG + (ch == 0 ? 5 : (ch == 1 ? 1 : 3)) * n3;   // TC, TA, WA
                    S1 = ch == 1 ? X : Y;
                    S2 = ch == 2 ? Y : X;
                }
            }
            const int sl = GW ? slice - ch * ns2 : slice;
            i = sl / ns;
            j = sl - i * ns;
            ei = wave_uniform(eI[i]);
            ej = wave_uniform(eJ[j]);
#pragma unroll
            for (int q = 0; q < ZR; ++q) {
                oI[q] = __builtin_amdgcn_readfirstlane((nbI[i * ZR + q] - i) * ns3);
                oJ[q] = __builtin_amdgcn_readfirstlane((nbJ[j * ZR + q] - j) * ns2);
            }
            xij = wave_uniform(X[i * ns + j]);
            yji = wave_uniform(Y[j * ns + i]);
            dij = (double)(i == j);
            if (lane_ok) {
                xil = ldo(X, i * ns + l);
                yjl = ldo(Y, j * ns + l);
                yil = ldo(Y, i * ns + l);
                if (TPP && ch == 0) dll = ldo(A, (l * ns + l) * ns2 + sl);
                if (TPH && ch == 0) sijl = ldo(DS, (i * ns + j) * ns + l);
            }
        }
        const int k = kb * rpw + sub;
        const bool act = lane_ok && k < ns;
        const int kk = act ? k : 0;
        const int slc = GW ? slice - ch * ns2 : slice;   // (i, j) of this channel
        const int e = slc * ns2 + kk * ns + l;
        const cd av = act ? ldo(Ach, e) : cmk(0.0, 0.0);
        cd vl[ZR];
#pragma unroll
        for (int q = 0; q < ZR; ++q) {
            vl[q].x = __shfl(av.x, src[q], 64);
            vl[q].y = __shfl(av.y, src[q], 64);
        }
        if (act) {
            // sum_p A_ijpl h_pk + sum_p A_ijkp h_pl, with h_pk = conj(h_kp)
            cd r = cmk(0.0, 0.0);
            const int* okk = okK + kk * ZR;
            const cd* hkk = hK + kk * ZR;
#pragma unroll
            for (int q = 0; q < ZR; ++q) {
                const cd vk = ldo(Ach, e + okk[q]);
                if (REALH) {
                    const double hq = hL[l * ZR + q].x;
                    r.x = fma(vl[q].x, hq, fma(vk.x, hkk[q].x, r.x));
                    r.y = fma(vl[q].y, hq, fma(vk.y, hkk[q].x, r.y));
                } else {
                    r = cfma_conjb(r, vl[q], hL[l * ZR + q]);
                    r = cfma_conjb(r, vk, hkk[q]);
                }
            }
            const cd ek = eK[kk];
            cd c = cmul(cmk(ei.x + ej.x - ek.x - el.x, ei.y + ej.y - ek.y - el.y), av);
            c = csub(c, r);
            const cd* hii = hI + i * ZR;
            const cd* hjj = hJ + j * ZR;
#pragma unroll
            for (int q = 0; q < ZR; ++q) {
                const cd vi = ldo(Ach, e + oI[q]), vj = ldo(Ach, e + oJ[q]);
                if (REALH) {
                    c.x = fma(hii[q].x, vi.x, fma(hjj[q].x, vj.x, c.x));
                    c.y = fma(hii[q].x, vi.y, fma(hjj[q].x, vj.y, c.y));
                } else {
                    c = cfma(c, hii[q], vi);
                    c = cfma(c, hjj[q], vj);
                }
            }
            if (GW) {   // polarization terms of the channel (Sec. VII.B, reading of the partner spins)
                const cd s1 = ldo(S1, j * ns + l), s2 = ldo(S2, kk * ns + i);
                const cd p1 = cmul_mi(cmul(s1, csub(ldo(D1, (i * ns + kk) * ns + j), ldo(D1, (i * ns + kk) * ns + l))));
                const cd p2 = cmul_mi(cmul(s2, csub(ldo(D2, (kk * ns + j) * ns + l), ldo(D2, (i * ns + j) * ns + l))));
                c = cadd(c, cscale(csub(p1, cconj(p2)), a.U));
            }
            const cd xkl = ldo(X, kk * ns + l), ykl = ldo(Y, kk * ns + l);
            if (!GW || ch == 0) {   // source (eq:soa-cubic-scheme), channel A only
            const cd xik = ldo(X, i * ns + kk), xjk = ldo(X, j * ns + kk), yjk = ldo(Y, j * ns + kk);
            const cd xlk = cmk(-xkl.x, xkl.y);
            const double dd = dij - (double)(kk == l);
            cd t1 = cmul(csub(cmul(xij, xjk), cmul(xlk, xil)), yjl);
            cd t2 = cmul(csub(cmul(yji, yil), cmul(ykl, yjk)), xik);
            c = cadd(c, cadd(cscale(cmul(xik, yjl), a.U * dd), cscale(cmul_i(cadd(t1, t2)), a.U)));
            }
            if (TPP && ch == 0) {   // ladder (Sec. VII.C) and its partner, channel A only
                const int kl = kk * ns + l;
                cd dii = ldo(A, (i * ns + i) * ns2 + kl), djj = ldo(A, (j * ns + j) * ns2 + kl);
                cd l1 = cmul_i(cadd(cmul(yji, dii), cmul(xij, djj)));
                if (i == j) l1 = cadd(l1, dii);
                cd dkk = ldo(A, (kk * ns + kk) * ns2 + slc);
                cd ylk = cmk(-ykl.x, ykl.y);
                cd l2 = cmul_i(cadd(cmul(ylk, dkk), cmul(xkl, dll)));
                if (kk == l) l2 = cadd(l2, dkk);
                c = cadd(c, cscale(csub(l1, cconj(l2)), a.U));
            }
            if (TPH && ch == 0) {   // particle-hole ladder (Sec. VII.C) and its partner, channel A only
                //   L_ijkl = i U (Y_il A_ijki - X_il A_ljkl)
                //   L_klij = i U (Y_kj A_klik - X_kj A_jlij)
                const cd rjki = ldo(DR, (j * ns + kk) * ns + i), rjkl = ldo(DR, (j * ns + kk) * ns + l);
                const cd sikl = ldo(DS, (i * ns + kk) * ns + l);
                const cd ykj = ldo(Y, kk * ns + j), xkj = ldo(X, kk * ns + j);
                cd l1 = cmul_i(csub(cmul(yil, rjki), cmul(xil, rjkl)));
                cd l2 = cmul_i(csub(cmul(ykj, sikl), cmul(xkj, sijl)));
                c = cadd(c, cscale(csub(l1, cconj(l2)), a.U));
            }
            rk_update<MODE, TO, true>(e, cmul_mi(c), av, y, acc, out, s.cb, s.cc);
        }
        kb += 4;
        while (kb >= nkb) {
            kb -= nkb;
            ++slice;
        }
    }
}

// Slice version of the stage (every selfenergy; every cluster with ns <= 64 and
// at most Z_MAX_ROW neighbours per site).  A work-group of SLICE_THREADS threads
// (SLICE_THREADS_BIG for one cluster in items of SLICE_ELEMS elements: twice the
// waves per compute unit for the same LDS, while the ragged batch, whose items
// are shorter, stays faster with SLICE_THREADS; row64_threads for the ns = 64
// row form below) stages up to floor(SLICE_ELEMS / ns^2) consecutive (i, j)
// slices A[i][j][:][:] of one channel of the stage input in LDS with coalesced
// loads and then gives one element to each thread (m = tid, tid + blockDim,
// ... over the staged elements), so the lanes are filled whatever ns is.  The
// k- and
// l-neighbours of the commutator lie in the same slice and are read from LDS;
// the i- and j-neighbours, the ladder's diagonal slices and the Runge-Kutta
// registers come from global memory.  A work item is a range [start, end) of
// slices (channel ns^2 + i ns + j) of one channel of one cluster, at most
// floor(SLICE_ELEMS / ns^2) long.
constexpr int SLICE_THREADS = 512;
constexpr int SLICE_THREADS_BIG = 1024;
// ns = 64 row form: two work-groups per compute unit (64 KB of staged slice
// each) of 12 waves (80 registers per thread), or of 16 waves for TPH (64
// registers).  Measured per stage on the 8x8 cluster, 12 against 16 waves:
// SOA 0.332 / 0.366 ms (16 waves spill in the middle stage), TPP 0.358 /
// 0.367, GW 1.090 / 1.093, mixed SOA, TPP and GW 3-11% faster; TPH 0.378 /
// 0.373 and mixed TPH 3% slower.
__host__ __device__ constexpr int row64_waves(int se, bool) { return se == SE_TPH ? 8 : 6; }
__host__ __device__ constexpr int row64_threads(int se, bool mixed) { return 128 * row64_waves(se, mixed); }
constexpr int SLICE_ELEMS = 4096;
// TPP: the diagonal entries A_ppij of the staged slices (p < ns), kept in LDS;
// a TPP item holds at most SLICE_DIAG / ns slices
constexpr int SLICE_DIAG = 128;
// below this many G2 elements in all, the row kernel is the default: whole
// slices would give too few work-groups
constexpr long long SLICE_MIN_ELEMS = 1LL << 20;
// except for one small cluster with a single-channel closure (at most
// SMALL_SLICE_MAX elements): the slice kernel in items of at most SLICE_SMALL
// elements, which spreads a stage over enough work-groups (measured on the
// 8-site chain: SOA 62k, TPP 55k and TPH 36k steps/s, against 28k, 22k and 18k
// for the row kernel and 34k, 27k and 28k for the persistent work-group)
constexpr long long SMALL_SLICE_MAX = 4096;
constexpr int SLICE_SMALL = 256;

// n / d for n < 2^16 and 1 <= d <= 4096, with mg = slice_magic(d)
__host__ __device__ constexpr unsigned slice_magic(unsigned d) { return d == 1 ? 0u : 0xffffffffu / d + 1u; }
__device__ __forceinline__ int slice_div(int n, unsigned mg) {
    return mg == 0u ? n : (int)__umulhi((unsigned)n, mg);
}

template <int MODE, int SE, bool MIXED, bool REALH, bool ROW64>
__global__ __launch_bounds__(SLICE_THREADS_BIG) __attribute__((amdgpu_waves_per_eu(ROW64 ? row64_waves(SE, MIXED) : 1))) void hub_slice_kernel(StageArgs s) {
    constexpr bool TPP = has_pp(SE), TPH = has_ph(SE), GW = has_pol(SE);
    using TI = typename StageTypes<MODE, MIXED>::In;
    using TO = typename StageTypes<MODE, MIXED>::Out;
    constexpr int ZR = Z_MAX_ROW;
    // the staged slices: as many elements as the longest item of the launch
    // (at most SLICE_ELEMS), so that shorter items leave LDS for more work-groups
    extern __shared__ cd P[];
    __shared__ cd eu[NS_MAX_ROW], ed[NS_MAX_ROW];
    // per site and neighbour slot (padded to ZR; a missing neighbour has offset
    // 0 and hopping 0): element offsets of the neighbour along l (p - l),
    // k ((p - k) ns), i ((p - i) ns^3) and j ((p - j) ns^2), each for the spin
    // that index carries in the work item's channel
    // (ROW64 keeps the i and j ones in scalar registers and the hoppings, all
    // real there, as binary64 reals: the LDS of two 1,024-thread work-groups
    // per compute unit)
    __shared__ int ofl[NS_MAX_ROW * ZR], ofk[NS_MAX_ROW * ZR];
    __shared__ int ofi[ROW64 ? 1 : NS_MAX_ROW * ZR], ofj[ROW64 ? 1 : NS_MAX_ROW * ZR];
    __shared__ cd shp[ROW64 ? 1 : 2 * NS_MAX_ROW * ZR];   // hoppings [spin][site][slot]
    __shared__ double shr[ROW64 ? 2 * NS_MAX_ROW * ZR : 1];
    __shared__ cd DK[TPP ? (ROW64 ? 64 : SLICE_DIAG) : 1];   // TPP: DK[slice][p] = A_pp,ij
    // ROW64: the entries of G1 and of the diagonal tensors that the item's
    // slice (i, j) indexes by i, j or k only, one per index q < 64: X_iq, Y_iq,
    // X_jq, Y_jq, then X_qj, Y_qj, R_jqi (TPH, from RT), S2_qi, D1_iqj (GW,
    // from RG)
    constexpr int RT = 4, RG = 4 + (TPH ? 3 : 0);
    __shared__ cd rowv[ROW64 ? (RG + (GW ? 2 : 0)) * 64 : 1];
    const WorkItem w = s.work[blockIdx.x];
    const ClusterDesc d = s.desc[w.cluster];
    const Cl a = make_cl(d, s.nbr, s.hop, s.d0, s.xdrv, s.in1, s.s_drive, s.u_scale);
    const int ns = d.ns, z = d.zmax, ns2 = ns * ns, ns3 = ns2 * ns;
    const TI* __restrict__ A = reinterpret_cast<const TI*>(s.in2) + d.g2off;
    const int tid = threadIdx.x, nthr = blockDim.x;
    if (w.start < 0) {   // G1 update of the cluster (the collision integral reads channel A)
        const cd* g1 = s.in1 + d.g1off;
        const cd* y = s.y1 + d.g1off;
        cd* acc = s.acc1 + d.g1off;
        cd* out = s.out1 + d.g1off;
        if (MODE == RK_FIRST && w.cluster == 0 && tid == 0) guard_begin_step(s.guard);
        const unsigned long long step = MODE == RK_LAST ? s.guard.div[0] : 0ull;
        for (int e = tid; e < 2 * ns2; e += nthr) {
            int sig = e / ns2, r = e % ns2, i = r / ns, j = r % ns;
            cd f = hub_g1_rhs(a, A, sig, i, j);
            rk_update<MODE>(e, f, g1[e], y, acc, out, s.cb, s.cc);
            if (MODE == RK_LAST && guard_bad(out[e], i == j)) guard_fire(s.guard, w.cluster, step);
        }
        return;
    }
    for (int q = tid; q < ns; q += nthr) {
        eu[q] = hf_diag(a, 0, q);
        ed[q] = hf_diag(a, 1, q);
    }
    // channel of the work item (items do not cross channels) and the spin of
    // the indices (i, j, k, l): A = (up, dn, up, dn); GW's B and C are all up
    // and all down
    const int ch = GW ? w.start / ns2 : 0;
    const int sI = ch == 2 ? 1 : 0, sJ = ch == 1 ? 0 : 1;
    for (int q = tid; q < 2 * ns * ZR; q += nthr) {
        const int row = q / ZR, qq = q - row * ZR, spin = row / ns, site = row - spin * ns;
        const int p = qq < z ? a.nbr[row * z + qq] : -1;
        const int dp = p >= 0 ? p - site : 0;
        if constexpr (ROW64)
            shr[q] = p >= 0 ? a.hop[row * z + qq].x : 0.0;
        else
            shp[q] = p >= 0 ? a.hop[row * z + qq] : cmk(0.0, 0.0);
        if (spin == sI) {
            ofk[site * ZR + qq] = dp * ns;
            if (!ROW64) ofi[site * ZR + qq] = dp * ns3;
        }
        if (spin == sJ) {
            ofl[site * ZR + qq] = dp;
            if (!ROW64) ofj[site * ZR + qq] = dp * ns2;
        }
    }
    // stage the slices [start, end) of the channel
    const long long n4 = (long long)ns2 * ns2;
    const TI* __restrict__ Ach = A + ch * n4;
    const int E = (w.end - w.start) * ns2;
    const int slice0 = w.start - ch * ns2;   // first (i, j) of the item
    const unsigned e0 = (unsigned)slice0 * (unsigned)ns2;
    for (int m = tid; m < E; m += nthr) P[m] = ldo(Ach, e0 + (unsigned)m);
    if (TPP && ch == 0)   // the host keeps (end - start) ns <= SLICE_DIAG for these items
        for (int q = tid; q < min((w.end - w.start) * ns, SLICE_DIAG); q += nthr) {
            const int sl = q / ns, p = q - sl * ns;
            DK[q] = ldo(A, (p * ns + p) * ns2 + slice0 + sl);
        }
    if constexpr (ROW64) {
        const int i = slice0 >> 6, j = slice0 & 63;
        const cd* __restrict__ Xs = a.X;
        const cd* __restrict__ Ys = a.Y;
        for (int q = tid; q < 64; q += nthr) {
            rowv[q] = ldo(Xs, i * 64 + q);
            rowv[64 + q] = ldo(Ys, i * 64 + q);
            rowv[2 * 64 + q] = ldo(Xs, j * 64 + q);
            rowv[3 * 64 + q] = ldo(Ys, j * 64 + q);
            if (TPH && (!GW || ch == 0)) {
                const cd* R = s.diag + (long long)n_diag(SE) * d.doff + (GW ? 6 * ns3 : 0);
                rowv[RT * 64 + q] = ldo(Xs, q * 64 + j);
                rowv[(RT + 1) * 64 + q] = ldo(Ys, q * 64 + j);
                rowv[(RT + 2) * 64 + q] = ldo(R, (j * 64 + q) * 64 + i);
            }
            if (GW) {
                const cd* G = s.diag + (long long)n_diag(SE) * d.doff;
                rowv[RG * 64 + q] = ldo(ch == 2 ? Ys : Xs, q * 64 + i);
                rowv[(RG + 1) * 64 + q] = ldo(G + (ch == 0 ? 4 : (ch == 1 ? 0 : 2)) * (long long)ns3, (i * 64 + q) * 64 + j);
            }
        }
    }
    __syncthreads();
    const unsigned mg2 = slice_magic((unsigned)ns2), mg1 = slice_magic((unsigned)ns);
    const cd* hI = shp + sI * ns * ZR;   // hoppings of the spin of i and k
    const cd* hJ = shp + sJ * ns * ZR;   // of j and l
    const double* hIr = shr + sI * ns * ZR;   // the same, ROW64
    const double* hJr = shr + sJ * ns * ZR;
    const cd* eI = sI ? ed : eu;
    const cd* eJ = sJ ? ed : eu;
    const cd* __restrict__ X = a.X;
    const cd* __restrict__ Y = a.Y;
    const cd* y = s.y2 + d.g2off + ch * n4;
    cd* acc = s.acc2 + d.g2off + ch * n4;
    TO* out = reinterpret_cast<TO*>(s.out2) + d.g2off + ch * n4;
    // R[a][b][c] and S[b][c][a], after GW's six layouts for DSL
    const cd* __restrict__ DR = TPH ? s.diag + (long long)n_diag(SE) * d.doff + (GW ? 6 * ns3 : 0) : nullptr;
    const cd* __restrict__ DS = TPH ? DR + ns3 : nullptr;
    // GW: diagonal tensors of the channel's two polarization terms
    //   Pi_1 = -i U S1_jl (D1[i][k][j] - D1[i][k][l]),
    //   Pi_2 = -i U S2_ki (D2[k][j][l] - D2[i][j][l]), term Pi_1 - conj(Pi_2)
    const cd* __restrict__ DG = GW ? s.diag + (long long)n_diag(SE) * d.doff : nullptr;
    const long long n3 = ns3;
    const cd* __restrict__ D1 = GW ? DG + (ch == 0 ? 4 : (ch == 1 ? 0 : 2)) * n3 : nullptr;   // UB, UA, VA
    const cd* __restrict__ D2 = GW ? DG + (ch == 0 ? 5 : (ch == 1 ? 1 : 3)) * n3 : nullptr;   // TC, TA, WA
    const cd* __restrict__ S1 = ch == 1 ? X : Y;
    const cd* __restrict__ S2 = ch == 2 ? Y : X;
    const bool src = !GW || ch == 0;   // the source and the ladders live on channel A only
    // ROW64 (every cluster has ns = 64): an item is one (i, j) slice and a wave
    // one row (i, j, k) with lane = l.  The G1 and diagonal-tensor entries
    // indexed by i, j and k only (and rows i and j of G1) come from the rows
    // staged in LDS, the neighbour tables of i and j sit in scalar registers,
    // and only the entries that depend on k and l take vector loads.
    // Otherwise every entry is a vector load where it is used.
    static_assert(!ROW64 || REALH, "the ns = 64 form is built for real hoppings");
    int oi[ZR], oj[ZR];
    double hi_[ZR], hj_[ZR];
    if constexpr (ROW64) {
        const int i = slice0 >> 6, j = slice0 & 63;
#pragma unroll
        for (int q = 0; q < ZR; ++q) {
            const int pi = q < z ? a.nbr[(sI * ns + i) * z + q] : -1;
            const int pj = q < z ? a.nbr[(sJ * ns + j) * z + q] : -1;
            oi[q] = wave_uniform(pi >= 0 ? (pi - i) * ns3 : 0);
            oj[q] = wave_uniform(pj >= 0 ? (pj - j) * ns2 : 0);
            hi_[q] = wave_uniform(hIr[i * ZR + q]);
            hj_[q] = wave_uniform(hJr[j * ZR + q]);
        }
    }
    // values indexed by i, j or k only: in ROW64 mode wave-uniform, kept in
    // scalar registers
    auto uni = [](auto v) {
        if constexpr (ROW64) return wave_uniform(v);
        else return v;
    };
    auto element = [&](const int m, const int sl, const int k, const int l, const int i, const int j) {
        const unsigned e = e0 + (unsigned)m;
        const cd av = P[m];
        // sum_p A_ijpl h_pk + sum_p A_ijkp h_pl, with h_pk = conj(h_kp)
        cd rr = cmk(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < ZR; ++q) {
            const cd vl = P[m + ofl[l * ZR + q]], vk = P[m + uni(ofk[k * ZR + q])];
            const cd hl = ROW64 ? cmk(hJr[l * ZR + q], 0.0) : hJ[l * ZR + q];
            const cd hk = ROW64 ? cmk(uni(hIr[k * ZR + q]), 0.0) : hI[k * ZR + q];
            if (REALH) {
                rr.x = fma(vl.x, hl.x, fma(vk.x, hk.x, rr.x));
                rr.y = fma(vl.y, hl.x, fma(vk.y, hk.x, rr.y));
            } else {
                rr = cfma_conjb(rr, vl, hl);
                rr = cfma_conjb(rr, vk, hk);
            }
        }
        const cd ei = uni(eI[i]), ej = uni(eJ[j]), ek = uni(eI[k]), el = eJ[l];
        cd c = cmul(cmk(ei.x + ej.x - ek.x - el.x, ei.y + ej.y - ek.y - el.y), av);
        c = csub(c, rr);
#pragma unroll
        for (int q = 0; q < ZR; ++q) {
            const cd hi = ROW64 ? cmk(hi_[q], 0.0) : hI[i * ZR + q], hj = ROW64 ? cmk(hj_[q], 0.0) : hJ[j * ZR + q];
            const cd vi = ldo(Ach, e + (ROW64 ? oi[q] : ofi[i * ZR + q]));
            const cd vj = ldo(Ach, e + (ROW64 ? oj[q] : ofj[j * ZR + q]));
            if (REALH) {
                c.x = fma(hi.x, vi.x, fma(hj.x, vj.x, c.x));
                c.y = fma(hi.x, vi.y, fma(hj.x, vj.y, c.y));
            } else {
                c = cfma(c, hi, vi);
                c = cfma(c, hj, vj);
            }
        }
        if (GW) {   // polarization terms of the channel (Sec. VII.B, reading of the partner spins)
            const cd s1 = ldo(S1, j * ns + l);
            const cd s2 = ROW64 ? uni(rowv[RG * 64 + k]) : ldo(S2, k * ns + i);
            const cd d1j = ROW64 ? uni(rowv[(RG + 1) * 64 + k]) : ldo(D1, (i * ns + k) * ns + j);
            const cd p1 = cmul_mi(cmul(s1, csub(d1j, ldo(D1, (i * ns + k) * ns + l))));
            const cd p2 = cmul_mi(cmul(s2, csub(ldo(D2, (k * ns + j) * ns + l), ldo(D2, (i * ns + j) * ns + l))));
            c = cadd(c, cscale(csub(p1, cconj(p2)), a.U));
        }
        if (src) {
            const cd xil = ROW64 ? rowv[l] : ldo(X, i * ns + l), yil = ROW64 ? rowv[64 + l] : ldo(Y, i * ns + l);
            const cd xkl = ldo(X, k * ns + l), ykl = ldo(Y, k * ns + l);
            const cd xij = ROW64 ? uni(rowv[j]) : ldo(X, i * ns + j);
            const cd yji = ROW64 ? uni(rowv[3 * 64 + i]) : ldo(Y, j * ns + i);
            {   // source (eq:soa-cubic-scheme), channel A only; X_lk = -conj(X_kl)
                const cd yjl = ROW64 ? rowv[3 * 64 + l] : ldo(Y, j * ns + l);
                const cd xik = ROW64 ? uni(rowv[k]) : ldo(X, i * ns + k);
                const cd xjk = ROW64 ? uni(rowv[2 * 64 + k]) : ldo(X, j * ns + k);
                const cd yjk = ROW64 ? uni(rowv[3 * 64 + k]) : ldo(Y, j * ns + k);
                const cd xlk = cmk(-xkl.x, xkl.y);
                const double dd = (double)(i == j) - (double)(k == l);
                const cd t1 = cmul(csub(cmul(xij, xjk), cmul(xlk, xil)), yjl);
                const cd t2 = cmul(csub(cmul(yji, yil), cmul(ykl, yjk)), xik);
                c = cadd(c, cadd(cscale(cmul(xik, yjl), a.U * dd), cscale(cmul_i(cadd(t1, t2)), a.U)));
            }
            if (TPP) {   // ladder (Sec. VII.C) and its partner, channel A only
                const int kl = k * ns + l;
                const cd dii = ldo(A, (i * ns + i) * ns2 + kl), djj = ldo(A, (j * ns + j) * ns2 + kl);
                cd l1 = cmul_i(cadd(cmul(yji, dii), cmul(xij, djj)));
                if (i == j) l1 = cadd(l1, dii);
                const cd dkk = DK[sl * ns + k], dll = DK[sl * ns + l];
                const cd ylk = cmk(-ykl.x, ykl.y);
                cd l2 = cmul_i(cadd(cmul(ylk, dkk), cmul(xkl, dll)));
                if (k == l) l2 = cadd(l2, dkk);
                c = cadd(c, cscale(csub(l1, cconj(l2)), a.U));
            }
            if (TPH) {   // particle-hole ladder (Sec. VII.C) and its partner, channel A only
                //   L_ijkl = i U (Y_il A_ijki - X_il A_ljkl)
                //   L_klij = i U (Y_kj A_klik - X_kj A_jlij)
                const cd rjki = ROW64 ? uni(rowv[(RT + 2) * 64 + k]) : ldo(DR, (j * ns + k) * ns + i);
                const cd rjkl = ldo(DR, (j * ns + k) * ns + l);
                const cd sikl = ldo(DS, (i * ns + k) * ns + l), sijl = ldo(DS, (i * ns + j) * ns + l);
                const cd ykj = ROW64 ? uni(rowv[(RT + 1) * 64 + k]) : ldo(Y, k * ns + j);
                const cd xkj = ROW64 ? uni(rowv[RT * 64 + k]) : ldo(X, k * ns + j);
                const cd l1 = cmul_i(csub(cmul(yil, rjki), cmul(xil, rjkl)));
                const cd l2 = cmul_i(csub(cmul(ykj, sikl), cmul(xkj, sijl)));
                c = cadd(c, cscale(csub(l1, cconj(l2)), a.U));
            }
        }
        rk_update<MODE, TO, true>((int)e, cmul_mi(c), av, y, acc, out, s.cb, s.cc);
    };
    if constexpr (ROW64) {
        const int wid = __builtin_amdgcn_readfirstlane(tid >> 6), nw = nthr >> 6;
        const int i = slice0 >> 6, j = slice0 & 63;
#pragma unroll 1
        for (int k = wid; k < 64; k += nw) {
            // l is the lane; kept opaque so that its LDS reads stay in the loop
            // instead of holding registers across it
            int l = tid & 63;
            asm volatile("" : "+v"(l));
            element(k * 64 + l, 0, k, l, i, j);
        }
    } else {
        for (int m = tid; m < E; m += nthr) {
            const int sl = slice_div(m, mg2), r2 = m - sl * ns2;
            const int k = slice_div(r2, mg1), l = r2 - k * ns;
            const int slice = slice0 + sl;
            const int i = slice_div(slice, mg1), j = slice - i * ns;
            element(m, sl, k, l, i, j);
        }
    }
}

// Whole Runge-Kutta steps of one small cluster in one work-group (the
// latency-bound case: up to a few thousand G2 elements, where four launches per
// step cost more than their work; measured on chains, one work-group beats the
// graph-replayed row-kernel stages 2.3x at ns = 2 and 2.4x at ns = 7; the
// kernel holds up to 4,096 elements, and is dispatched up to ns = 7).  The stage input of G2 and G1 is double-buffered in LDS; y and the
// running sum acc stay in the registers of the thread that owns the element
// (PERSIST_PER G2 elements, their indices packed one byte each, and at most
// one G1 element per thread); the 2 ns diagonals of h^HF are computed once per
// stage; with real hoppings (RH) the neighbour terms read binary64 reals; a
// step is four stages separated by work-group barriers.  Each
// element's right-hand side is the per-element one (hub_g2_rhs, hub_g1_rhs),
// and the updates are those of rk_update, so the arithmetic is that of the
// launched stages.  Single-channel closures (SOA, TPP, TPH), no drive, no
// switching ramp.  MIXED keeps the G2 stage copies in binary32 as the launched
// mixed stages do: sA[0] then holds the binary64 y (the input of stage 1) and
// sA[1] two binary32 buffers F0, F1; stage 1 writes F0, stage 2 reads F0 and
// writes F1, stage 3 reads F1 and writes F0, stage 4 reads F0 and writes the
// new y to sA[0].
constexpr int PERSIST_THREADS = 1024;
constexpr int PERSIST_G2 = 4096;   // ns^4 <= 4096: ns <= 8
constexpr int PERSIST_G1 = 128;    // 2 ns^2
constexpr int PERSIST_PER = PERSIST_G2 / PERSIST_THREADS;
constexpr int PERSIST_NBR = 128;   // 2 ns zmax: neighbour table and hoppings, staged in LDS
// the dispatcher takes the persistent work-group up to ns = 7 (2,401 elements);
// at ns = 8 the slice kernel in small items is faster (SMALL_SLICE_MAX)
constexpr int PERSIST_MAX_G2 = 2401;

struct PersistArgs {
    const ClusterDesc* desc;
    const int* nbr;
    const cd* hop;
    const double* d0;
    const double* xdrv;
    cd* y1;        // G1 state [2][ns][ns]: read at the start, written at the end
    cd* y2;        // G2 state [ns]^4
    double dt;
    int nsteps;
    DivGuard guard;   // steps are numbered from guard.div[0] as the launch finds it
};

template <int SE, bool MIXED, bool RH>
__global__ __launch_bounds__(PERSIST_THREADS) void hub_persistent_kernel(PersistArgs p) {
    __shared__ cd sA[2][PERSIST_G2];
    float2* const sF = reinterpret_cast<float2*>(sA[1]);
    __shared__ cd sG[2][PERSIST_G1];
    // the cluster's neighbour table, hoppings, h0 diagonal and drive profile
    // (a few hundred bytes, read by every element every stage) in LDS
    __shared__ int snbr[PERSIST_NBR];
    __shared__ cd shop[PERSIST_NBR];
    __shared__ double shr[PERSIST_NBR];   // real parts of the hoppings (RH: all are real)
    __shared__ double sd0[PERSIST_G1], sxd[PERSIST_G1];
    __shared__ cd shd[16];   // diagonals of h^{HF} at the stage (2 ns <= 16)
    const ClusterDesc d = p.desc[0];
    const int ns = d.ns, ns2 = ns * ns, n2 = ns2 * ns2, n1 = 2 * ns2;
    const int tid = threadIdx.x;
    for (int q = tid; q < 2 * ns * d.zmax; q += PERSIST_THREADS) {
        snbr[q] = p.nbr[d.nbroff + q];
        shop[q] = p.hop[d.nbroff + q];
        shr[q] = p.hop[d.nbroff + q].x;
    }
    if (tid < 2 * ns) sd0[tid] = p.d0[d.d0off + tid];
    if (tid < ns) sxd[tid] = p.xdrv[d.xoff + tid];
    cd y2[PERSIST_PER], acc2[PERSIST_PER];
    cd y1 = cmk(0.0, 0.0), acc1 = cmk(0.0, 0.0);
    // the indices (i, j, k, l) of each owned element, one byte each (ns <= 8)
    unsigned pk[PERSIST_PER];
#pragma unroll
    for (int q = 0; q < PERSIST_PER; ++q) {
        const int e = tid + q * PERSIST_THREADS;
        const int l = e % ns, k = (e / ns) % ns, j = (e / ns2) % ns, i = e / (ns2 * ns);
        pk[q] = (unsigned)i | ((unsigned)j << 8) | ((unsigned)k << 16) | ((unsigned)l << 24);
        y2[q] = e < n2 ? p.y2[e] : cmk(0.0, 0.0);
        acc2[q] = cmk(0.0, 0.0);
        if (e < n2) sA[0][e] = y2[q];
    }
    if (tid < n1) {
        y1 = p.y1[tid];
        sG[0][tid] = y1;
    }
    __syncthreads();
    const double h = p.dt;
    const unsigned long long step0 = p.guard.div[0];
    int cur = 0;
    for (int step = 0; step < p.nsteps; ++step) {
#pragma unroll 1
        for (int st = 0; st < 4; ++st) {
            // stage weights of the classical RK4 step: acc gets cb f, the next stage
            // input is y + cc f (the last stage writes y = acc + cb f)
            const double cb = (st == 0 || st == 3) ? h / 6.0 : h / 3.0;
            const double cc = st < 2 ? 0.5 * h : h;
            Cl a = make_cl(d, p.nbr, p.hop, p.d0, p.xdrv, sG[cur], 0.0, 1.0);
            a.nbr = snbr;
            a.hop = shop;
            a.hopr = shr;
            a.d0 = sd0;
            a.xdrv = sxd;
            if (tid < 2 * ns) shd[tid] = hf_diag(a, tid / ns, tid % ns);
            __syncthreads();
            a.hdg = shd;
            const cd* A = MIXED ? sA[0] : sA[cur];
            cd* outA = MIXED ? sA[0] : sA[cur ^ 1];
            const float2* inF = sF + (st == 2 ? PERSIST_G2 : 0);
            float2* outF = sF + (st == 1 ? PERSIST_G2 : 0);
            // an opaque copy of the thread index: the element indices are
            // recomputed every stage instead of being hoisted out of the step
            // loop, where holding them for all elements would spill registers
            int tq = tid;
            asm volatile("" : "+v"(tq));
            cd* outG = sG[cur ^ 1];
            // one element at a time (the barrier keeps the scheduler from
            // overlapping the right-hand sides, whose registers would spill);
            // the output goes to the other buffer, which no thread reads now
#pragma unroll
            for (int q = 0; q < PERSIST_PER; ++q) {
                const int e = tq + q * PERSIST_THREADS;
                if (e < n2) {
                    unsigned u = pk[q];
                    asm volatile("" : "+v"(u));   // keep derived offsets out of the step loop
                    const int i = u & 255, j = (u >> 8) & 255, k = (u >> 16) & 255, l = u >> 24;
                    cd f;
                    if (MIXED && st > 0) f = hub_g2_rhs<SE, float2, true, RH>(a, inF, i, j, k, l, e, ld_c(inF, e));
                    else f = hub_g2_rhs<SE, cd, true, RH>(a, A, i, j, k, l, e, A[e]);
                    cd o;
                    if (st == 0) {
                        acc2[q] = cmk(fma(cb, f.x, y2[q].x), fma(cb, f.y, y2[q].y));
                        o = cmk(fma(cc, f.x, y2[q].x), fma(cc, f.y, y2[q].y));
                    } else if (st < 3) {
                        acc2[q] = cmk(fma(cb, f.x, acc2[q].x), fma(cb, f.y, acc2[q].y));
                        o = cmk(fma(cc, f.x, y2[q].x), fma(cc, f.y, y2[q].y));
                    } else {
                        y2[q] = cmk(fma(cb, f.x, acc2[q].x), fma(cb, f.y, acc2[q].y));
                        o = y2[q];
                    }
                    if (MIXED && st < 3) st_c(outF, e, o);
                    else outA[e] = o;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            cd f1 = cmk(0.0, 0.0);
            if (tq < n1) {
                const int sig = tq / ns2, r = tq - sig * ns2;
                f1 = (MIXED && st > 0) ? hub_g1_rhs(a, inF, sig, r / ns, r % ns)
                                       : hub_g1_rhs(a, A, sig, r / ns, r % ns);
            }
            if (tid < n1) {
                cd o;
                if (st == 0) {
                    acc1 = cmk(fma(cb, f1.x, y1.x), fma(cb, f1.y, y1.y));
                    o = cmk(fma(cc, f1.x, y1.x), fma(cc, f1.y, y1.y));
                } else if (st < 3) {
                    acc1 = cmk(fma(cb, f1.x, acc1.x), fma(cb, f1.y, acc1.y));
                    o = cmk(fma(cc, f1.x, y1.x), fma(cc, f1.y, y1.y));
                } else {
                    y1 = cmk(fma(cb, f1.x, acc1.x), fma(cb, f1.y, acc1.y));
                    o = y1;
                    const int r = tid % ns2, i = r / ns, j = r % ns;
                    if (guard_bad(o, i == j)) guard_fire(p.guard, 0, step0 + step + 1);
                }
                outG[tid] = o;
            }
            __syncthreads();
            cur ^= 1;
        }
    }
#pragma unroll
    for (int q = 0; q < PERSIST_PER; ++q) {
        const int e = tid + q * PERSIST_THREADS;
        if (e < n2) p.y2[e] = y2[q];
    }
    if (tid < n1) p.y1[tid] = y1;
    __syncthreads();   // every thread has read guard.div[0]
    if (tid == 0) p.guard.div[0] = step0 + (unsigned long long)p.nsteps;
}

StageArgs make_stage(g1g2_ctx* c, double t, const Regs& in, const Regs& y, const Regs& acc,
                     const Regs& out, double cb, double cc) {
    HubbardData& H = c->hub;
    StageArgs s;
    s.desc = H.desc;
    s.work = H.work;
    s.nbr = H.nbr;
    s.hop = H.hop;
    s.d0 = H.d0;
    s.xdrv = H.xdrv;
    s.s_drive = H.drive_value(t);
    s.u_scale = c->switch_value(t);
    s.in1 = in.g1;
    s.in2 = in.g2;
    s.y1 = y.g1;
    s.y2 = y.g2;
    s.acc1 = acc.g1;
    s.acc2 = acc.g2;
    s.out1 = out.g1;
    s.out2 = out.g2;
    s.cb = cb;
    s.cc = cc;
    s.guard = guard_of(c);
    s.diag = H.diag;
    return s;
}

template <int MODE, int SE, bool MIXED>
void launch_stage_t(g1g2_ctx* c, const StageArgs& s) {
    if (n_diag(SE) > 0) {
        using TI = typename StageTypes<MODE, MIXED>::In;
        hipLaunchKernelGGL((hub_diag_kernel<TI, SE>), dim3(c->hub.ndwork), dim3(256), 0, c->stream,
                           c->hub.desc, c->hub.dwork, s.in2, const_cast<cd*>(s.diag));
    }
    if (c->hub.slices) {
        const size_t lds = (size_t)c->hub.slice_elems * sizeof(cd);
        const int nthr = c->hub.row64 ? row64_threads(SE, MIXED)
                         : c->hub.ncl == 1 && c->hub.slice_elems == SLICE_ELEMS ? SLICE_THREADS_BIG : SLICE_THREADS;
        if (SE != SE_DSL && c->hub.realhop && c->hub.row64)
            hipLaunchKernelGGL((hub_slice_kernel<MODE, SE, MIXED, true, SE != SE_DSL>), dim3(c->hub.nwork),
                               dim3(nthr), lds, c->stream, s);
        else if (c->hub.realhop)
            hipLaunchKernelGGL((hub_slice_kernel<MODE, SE, MIXED, true, false>), dim3(c->hub.nwork), dim3(nthr),
                               lds, c->stream, s);
        else
            hipLaunchKernelGGL((hub_slice_kernel<MODE, SE, MIXED, false, false>), dim3(c->hub.nwork), dim3(nthr),
                               lds, c->stream, s);
        return;
    }
    if constexpr (!has_pol(SE)) {   // GW and DSL run on the row and slice kernels only (checked at setup)
        if (!c->hub.rows) {
            hipLaunchKernelGGL((hub_stage_kernel<MODE, SE, MIXED>), dim3(c->hub.nwork), dim3(256), 0, c->stream,
                               s);
            return;
        }
    }
    if (c->hub.realhop)
        hipLaunchKernelGGL((hub_row_kernel<MODE, SE, MIXED, true>), dim3(c->hub.nwork), dim3(256), 0, c->stream,
                           s);
    else
        hipLaunchKernelGGL((hub_row_kernel<MODE, SE, MIXED, false>), dim3(c->hub.nwork), dim3(256), 0,
                           c->stream, s);
}

template <int MODE, int SE>
void launch_stage_p(g1g2_ctx* c, const StageArgs& s, bool mixed) {
    if (mixed) launch_stage_t<MODE, SE, true>(c, s);
    else launch_stage_t<MODE, SE, false>(c, s);
}

template <int MODE>
g1g2_status launch_stage(g1g2_ctx* c, const StageArgs& s) {
    // a plain right-hand side (g1g2_rhs) always works on binary64 caller buffers
    const bool mixed = MODE != RK_RHS && c->d.precision == G1G2_MIXED;
    switch (c->d.selfenergy) {
        case G1G2_TPP: launch_stage_p<MODE, SE_TPP>(c, s, mixed); break;
        case G1G2_TPH: launch_stage_p<MODE, SE_TPH>(c, s, mixed); break;
        case G1G2_GW: launch_stage_p<MODE, SE_GW>(c, s, mixed); break;
        case G1G2_DSL: launch_stage_p<MODE, SE_DSL>(c, s, mixed); break;
        default: launch_stage_p<MODE, SE_SOA>(c, s, mixed); break;
    }
    HIP_OK(c, hipGetLastError());
    prof_mark(c, "hub_stage");
    return G1G2_OK;
}

// Observables: one work-group per cluster; partial sums in binary64.
__global__ __launch_bounds__(256) void hub_obs_kernel(const ClusterDesc* __restrict__ desc,
                                                     const int* __restrict__ nbr,
                                                     const cd* __restrict__ hop,
                                                     const double* __restrict__ d0,
                                                     const double* __restrict__ xdrv, double s_drive,
                                                     double u_scale, const cd* __restrict__ g1,
                                                     const cd* __restrict__ g2,
                                                     double* __restrict__ res) {
    constexpr int NV = 7;
    __shared__ double sh[NV][256];
    const ClusterDesc d = desc[blockIdx.x];
    const Cl a = make_cl(d, nbr, hop, d0, xdrv, g1, s_drive, u_scale);
    const cd* A = g2 + d.g2off;
    const int ns = a.ns, z = a.zmax, tid = threadIdx.x;
    double nu = 0, nd = 0, ekin = 0, emf = 0, ecorr = 0, docc = 0, imb = 0;
    for (int i = tid; i < ns; i += blockDim.x) {
        double niu = a.X[i * ns + i].y, nid = a.Y[i * ns + i].y;
        nu += niu;
        nd += nid;
        // sites with negative drive profile count as left, positive as right
        const double xi = a.xdrv[i];
        imb += (xi < 0.0 ? 1.0 : (xi > 0.0 ? -1.0 : 0.0)) * (niu + nid);
        for (int sig = 0; sig < 2; ++sig) {
            const cd* G = sig ? a.Y : a.X;
            double dii = a.d0[sig * ns + i] + a.s_drive * a.xdrv[i];
            ekin += dii * G[i * ns + i].y;
            for (int q = 0; q < z; ++q) {  // h_ip n_pi, n = -i G
                int p = a.nbr[(sig * ns + i) * z + q];
                if (p >= 0) {
                    cd h = a.hop[(sig * ns + i) * z + q];
                    cd g = G[p * ns + i];
                    cd n = cmk(g.y, -g.x);
                    ekin += h.x * n.x - h.y * n.y;
                }
            }
        }
        double aiiii = A[((i * ns + i) * ns + i) * ns + i].x;
        emf += a.U * niu * nid;
        ecorr += -a.U * aiiii;
        docc += niu * nid - aiiii;
    }
    double v[NV] = {nu, nd, ekin, emf, ecorr, docc, imb};
    for (int q = 0; q < NV; ++q) sh[q][tid] = v[q];
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (tid < st)
            for (int q = 0; q < NV; ++q) sh[q][tid] += sh[q][tid + st];
        __syncthreads();
    }
    if (tid == 0)
        for (int q = 0; q < NV; ++q) res[blockIdx.x * 8 + q] = sh[q][0];
}

// max |A_(r,c) - conj(A_(c,r))| and max |A| per block, A an n x n pair matrix
__global__ __launch_bounds__(256) void herm_resid_kernel(const cd* __restrict__ A, int n, long long nn,
                                                        double* __restrict__ part) {
    __shared__ double s1[256], s2[256];
    double m1 = 0, m2 = 0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
         e += (long long)gridDim.x * blockDim.x) {
        long long r = e / n, col = e % n;
        cd v = A[e], w = A[col * n + r];
        double dx = v.x - w.x, dy = v.y + w.y;
        m1 = fmax(m1, sqrt(dx * dx + dy * dy));
        m2 = fmax(m2, sqrt(v.x * v.x + v.y * v.y));
    }
    s1[threadIdx.x] = m1;
    s2[threadIdx.x] = m2;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + s]);
            s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1[0];
        part[2 * blockIdx.x + 1] = s2[0];
    }
}

__global__ void hub_site_kernel(const ClusterDesc* __restrict__ desc, const int* __restrict__ nbr,
                                const cd* __restrict__ hop, const double* __restrict__ d0,
                                const double* __restrict__ xdrv, const cd* __restrict__ g1,
                                const cd* __restrict__ g2, double* __restrict__ out) {
    const ClusterDesc d = desc[0];
    const Cl a = make_cl(d, nbr, hop, d0, xdrv, g1, 0.0, 1.0);   // U is not used
    const cd* A = g2 + d.g2off;
    const int ns = a.ns;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x) {
        double niu = a.X[i * ns + i].y, nid = a.Y[i * ns + i].y;
        out[i] = niu;
        out[ns + i] = nid;
        out[2 * ns + i] = niu * nid - A[((i * ns + i) * ns + i) * ns + i].x;
    }
}

template <typename V>
g1g2_status upload(g1g2_ctx* c, V** dst, const std::vector<V>& h) {
    if (*dst) (void)hipFree(*dst);
    *dst = nullptr;
    HIP_OK(c, hipMalloc(dst, std::max<size_t>(h.size(), 1) * sizeof(V)));
    if (!h.empty())
        HIP_OK(c, hipMemcpyAsync(*dst, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, c->stream));
    return G1G2_OK;
}

}  // namespace

double HubbardData::drive_value(double t) const {
    double s = 0.0;
    for (size_t m = 0; m < drive_c.size(); ++m) {
        double d = t - drive_tc[m];
        s += drive_c[m] * std::exp(-d * d / (2.0 * drive_tau * drive_tau));
    }
    return s;
}

void hub_free(g1g2_ctx* c) {
    HubbardData& H = c->hub;
    void* ptrs[] = {H.desc, H.work, H.dwork, H.diag, H.nbr, H.hop, H.d0, H.xdrv};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    std::vector<double> dc = H.drive_c, dtc = H.drive_tc, dx = H.drive_x;
    double tau = H.drive_tau;
    H = HubbardData();
    H.drive_c = dc;
    H.drive_tc = dtc;
    H.drive_x = dx;
    H.drive_tau = tau;
}

// Work-groups are dispatched round-robin over the 8 XCDs of the device
// (work-group b runs on XCD b mod 8), each XCD with its own L2.  For a batch,
// the G2 work items (in cluster order) are split into 8 contiguous groups of
// equal cost, one per XCD, and interleaved so that work-group b takes the next
// item of group b mod 8.  A cluster's rows, and the neighbour rows its
// commutator stencil re-reads, are then all processed behind one L2 (on the
// 512-cluster batch this halves the fabric reads of a stage).  Each group
// starts with the G1 updates of its clusters, which then overlap the G2 items
// instead of trailing them; shorter groups are padded with empty items.
std::vector<WorkItem> xcd_order(const std::vector<WorkItem>& g2, const std::vector<long long>& cost,
                                const std::vector<WorkItem>& g1) {
    constexpr int NX = 8;
    long long total = 0;
    for (long long v : cost) total += v;
    std::vector<std::vector<WorkItem>> grp(NX), g2grp(NX);
    std::vector<int> first_group(g1.size(), -1);
    long long prefix = 0;
    for (size_t q = 0; q < g2.size(); ++q) {
        const long long mid2 = 2 * prefix + cost[q];   // twice the item's midpoint
        const int x = total > 0 ? (int)std::min<long long>(NX - 1, mid2 * NX / (2 * total)) : 0;
        prefix += cost[q];
        g2grp[x].push_back(g2[q]);
        if (first_group[g2[q].cluster] < 0) first_group[g2[q].cluster] = x;
    }
    for (size_t cl = 0; cl < g1.size(); ++cl) grp[std::max(first_group[cl], 0)].push_back(g1[cl]);
    size_t m = 0;
    for (int x = 0; x < NX; ++x) {
        grp[x].insert(grp[x].end(), g2grp[x].begin(), g2grp[x].end());
        m = std::max(m, grp[x].size());
    }
    std::vector<WorkItem> out(m * NX);
    for (size_t b = 0; b < out.size(); ++b) {
        const std::vector<WorkItem>& gx = grp[b % NX];
        const size_t r = b / NX;
        out[b] = r < gx.size() ? gx[r] : WorkItem{gx.empty() ? 0 : gx[0].cluster, 0, 0};
    }
    return out;
}

g1g2_status hub_setup(g1g2_ctx* c, int ncl, const int* nsv, const double* Uv, const cd* const* h0s,
                      const int* chunk_in) {
    HubbardData& H = c->hub;
    const int sel = c->d.selfenergy;
    const int se = sel == G1G2_GW ? SE_GW
                 : sel == G1G2_DSL ? SE_DSL
                 : sel == G1G2_TPH ? SE_TPH
                 : sel == G1G2_TPP ? SE_TPP : SE_SOA;
    const int nch = n_channels(se);
    std::vector<ClusterDesc> desc(ncl);
    std::vector<int> nbr_all;
    std::vector<cd> hop_all;
    std::vector<double> d0_all;
    std::vector<WorkItem> work, g1work, dwork;
    std::vector<long long> wcost;   // elements of each G2 work item
    bool realhop = true;            // every hopping of every cluster is real
    std::vector<int> chunks(ncl);
    bool rowk = true;
    for (int cl = 0; cl < ncl; ++cl) {
        if (nsv[cl] > NS_MAX_ROW) rowk = false;
        if (chunk_in && chunk_in[cl] < 0) rowk = false;   // per-element kernel requested
        // the row kernel keeps at most Z_MAX_ROW l-neighbours per lane
        const cd* h0 = h0s[cl];
        const int ns = nsv[cl];
        for (int sgm = 0; sgm < 2 && rowk; ++sgm)
            for (int i = 0; i < ns && rowk; ++i) {
                int z = 0;
                for (int j = 0; j < ns; ++j) {
                    cd v = h0[(size_t)sgm * ns * ns + i * ns + j];
                    if (i != j && (v.x != 0.0 || v.y != 0.0)) ++z;
                }
                if (z > Z_MAX_ROW) rowk = false;
            }
    }
    // the slice kernel takes every selfenergy wherever the row kernel could run,
    // by default for systems of at least SLICE_MIN_ELEMS G2 elements
    const int fl = c->d.flags;
    if ((fl & G1G2_HUB_ROW_KERNEL) && (fl & G1G2_HUB_SLICE_KERNEL))
        return set_error(c, G1G2_EINVAL, "G1G2_HUB_ROW_KERNEL and G1G2_HUB_SLICE_KERNEL exclude each other");
    long long total = 0;
    for (int cl = 0; cl < ncl; ++cl) total += (long long)nsv[cl] * nsv[cl] * nsv[cl] * nsv[cl];
    const bool small1 = ncl == 1 && nch == 1 && total <= SMALL_SLICE_MAX;
    const bool slicek = rowk && !(fl & G1G2_HUB_ROW_KERNEL) &&
                        ((fl & G1G2_HUB_SLICE_KERNEL) || total * nch >= SLICE_MIN_ELEMS || small1);
    long long g2off = 0;
    long long g1off = 0, xoff = 0, doff = 0;
    int slice_elems = 0;
    for (int cl = 0; cl < ncl; ++cl) {
        const int ns = nsv[cl];
        const cd* h0 = h0s[cl];
        std::vector<std::vector<std::pair<int, cd>>> rows(2 * ns);
        std::vector<double> d0(2 * ns);
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < ns; ++i)
                for (int j = 0; j < ns; ++j) {
                    cd v = h0[(size_t)s * ns * ns + i * ns + j];
                    cd vt = h0[(size_t)s * ns * ns + j * ns + i];
                    if (std::fabs(v.x - vt.x) > 1e-12 * (1 + std::fabs(v.x)) ||
                        std::fabs(v.y + vt.y) > 1e-12 * (1 + std::fabs(v.y)))
                        return set_error(c, G1G2_EINVAL,
                                         "h0 is not Hermitian (cluster " + std::to_string(cl) + ")");
                    if (i == j)
                        d0[s * ns + i] = v.x;
                    else if (v.x != 0.0 || v.y != 0.0) {
                        rows[s * ns + i].push_back({j, v});
                        if (v.y != 0.0) realhop = false;
                    }
                }
        int zmax = 1;
        for (auto& r : rows) zmax = std::max<int>(zmax, (int)r.size());
        ClusterDesc& d = desc[cl];
        d.ns = ns;
        d.zmax = zmax;
        d.g1off = (int)g1off;
        d.nbroff = (int)nbr_all.size();
        d.d0off = (int)d0_all.size();
        d.xoff = (int)xoff;
        d.g2off = g2off;
        d.doff = doff;
        d.U = Uv[cl];
        for (int r = 0; r < 2 * ns; ++r)
            for (int q = 0; q < zmax; ++q) {
                bool has = q < (int)rows[r].size();
                nbr_all.push_back(has ? rows[r][q].first : -1);
                hop_all.push_back(has ? rows[r][q].second : cmk(0, 0));
            }
        d0_all.insert(d0_all.end(), d0.begin(), d0.end());
        const long long n4 = (long long)ns * ns * ns * ns;
        if (slicek) {
            // slice items: at most floor(SLICE_ELEMS / ns^2) whole (i, j) slices of
            // one channel each, or fewer when chunk (elements per item) asks for
            // it; slice index = channel ns^2 + i ns + j
            int per = SLICE_ELEMS / (ns * ns);
            if (chunk_in && chunk_in[cl] > 0) per = std::max(1, std::min(per, chunk_in[cl] / (ns * ns)));
            // the particle-particle ladder keeps the diagonal entries of its slices in LDS
            if (has_pp(se)) per = std::max(1, std::min(per, SLICE_DIAG / ns));
            if (small1) per = std::max(1, std::min(per, SLICE_SMALL / (ns * ns)));
            const int nsl = ns * ns;
            chunks[cl] = per * ns * ns;
            slice_elems = std::max(slice_elems, per * ns * ns);
            for (int chn = 0; chn < nch; ++chn)
                for (int s0 = 0; s0 < nsl; s0 += per) {
                    const int s1 = std::min(nsl, s0 + per);
                    work.push_back({cl, chn * nsl + s0, chn * nsl + s1});
                    wcost.push_back((long long)(s1 - s0) * ns * ns);
                }
        } else if (rowk) {
            // wave units of rpw rows (rpw ns elements) over (channel, i, j, k-block);
            // chunk = elements per work-group
            const int rpw = std::min(64 / ns, ns);
            const int nkb = (ns + rpw - 1) / rpw;
            const long long nunits = (long long)nch * ns * ns * nkb;
            int want = (chunk_in && chunk_in[cl] > 0) ? chunk_in[cl] : 1024;
            int upw = std::max(4, (int)std::lround((double)want / (rpw * ns)));
            upw = (upw + 3) / 4 * 4;
            chunks[cl] = upw * rpw * ns;
            for (long long u0 = 0; u0 < nunits; u0 += upw) {
                const long long u1 = std::min<long long>(nunits, u0 + upw);
                work.push_back({cl, (int)u0, (int)u1});
                wcost.push_back((u1 - u0) * rpw * ns);
            }
        } else {
            int ch = (chunk_in && chunk_in[cl] != 0) ? std::abs(chunk_in[cl]) : 1024;
            chunks[cl] = ch;
            for (long long st = 0; st < n4; st += ch) {
                const long long e1 = std::min<long long>(n4, st + ch);
                work.push_back({cl, (int)st, (int)e1});
                wcost.push_back(e1 - st);
            }
        }
        g1work.push_back({cl, -1, -1});
        const int n3 = ns * ns * ns;
        // diagonal gather items of 1024 index triples: its loads are strided, so it
        // wants many work-groups in flight (256 for an 8x8 cluster)
        for (int t0 = 0; t0 < n3; t0 += 1024) dwork.push_back({cl, t0, std::min(n3, t0 + 1024)});
        doff += n3;
        g2off += nch * n4;
        g1off += 2LL * ns * ns;
        xoff += ns;
    }
    if (ncl > 1) {
        work = xcd_order(work, wcost, g1work);
    } else {   // one cluster: its G1 update first, then the rows in order
        work.insert(work.begin(), g1work.begin(), g1work.end());
    }
    if (has_pol(se) && !rowk)
        return set_error(c, G1G2_EUNSUPPORTED,
                         "Hubbard GW and DSL need ns <= 64, at most 4 neighbours per site and chunk > 0");
    hub_free(c);
    H.ncl = ncl;
    H.rows = rowk;
    H.slices = slicek;
    H.realhop = realhop;
    // every cluster has ns = 64: one (i, j) slice per item, a wave per row.
    // Measured per stage on the 8x8 cluster against the general slice form:
    // SOA 0.333 / 0.354 ms, TPP 0.367 / 0.399, TPH 0.373 / 0.412, GW 1.09 /
    // 1.15, and 9-15% faster for every closure in mixed precision.  DSL needs
    // too much LDS for two work-groups per compute unit and keeps the general
    // form.
    H.row64 = slicek && std::all_of(nsv, nsv + ncl, [](int n) { return n == 64; }) && se != SE_DSL;
    H.ndwork = (int)dwork.size();
    H.slice_elems = slice_elems;
    H.diag_elems = n_diag(se) > 0 ? n_diag(se) * doff : 0;
    H.hdesc = desc;
    H.chunk = chunks;
    H.nwork = (int)work.size();
    H.h_d0 = d0_all;
    g1g2_status s;
    if ((s = upload(c, &H.desc, desc)) != G1G2_OK) return s;
    if ((s = upload(c, &H.work, work)) != G1G2_OK) return s;
    if (n_diag(se) > 0) {
        if ((s = upload(c, &H.dwork, dwork)) != G1G2_OK) return s;
        HIP_OK(c, hipMalloc(&H.diag, std::max<long long>(n_diag(se) * doff, 1) * sizeof(cd)));
    }
    if ((s = upload(c, &H.nbr, nbr_all)) != G1G2_OK) return s;
    if ((s = upload(c, &H.hop, hop_all)) != G1G2_OK) return s;
    if ((s = upload(c, &H.d0, d0_all)) != G1G2_OK) return s;
    HIP_OK(c, hipMalloc(&H.xdrv, std::max<long long>(xoff, 1) * sizeof(double)));
    HIP_OK(c, hipMemsetAsync(H.xdrv, 0, std::max<long long>(xoff, 1) * sizeof(double), c->stream));
    if (ncl == 1 && (long long)H.drive_x.size() == xoff)
        HIP_OK(c, hipMemcpyAsync(H.xdrv, H.drive_x.data(), xoff * sizeof(double), hipMemcpyHostToDevice,
                                 c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return G1G2_OK;
}

bool hub_persistent_ok(const g1g2_ctx* c) {
    const HubbardData& H = c->hub;
    if (H.ncl != 1 || H.has_drive() || c->has_switch() || c->prof) return false;
    if (c->d.flags & (G1G2_HUB_ROW_KERNEL | G1G2_HUB_SLICE_KERNEL)) return false;
    const int sel = c->d.selfenergy;
    if (sel != G1G2_SOA && sel != G1G2_TPP && sel != G1G2_TPH) return false;
    const long long ns = H.hdesc[0].ns, z = H.hdesc[0].zmax;
    return ns * ns * ns * ns <= PERSIST_MAX_G2 && 2 * ns * ns <= PERSIST_G1 && 2 * ns * z <= PERSIST_NBR;
}

template <bool MIXED, bool RH>
void launch_persistent(g1g2_ctx* c, const PersistArgs& p) {
    switch (c->d.selfenergy) {
        case G1G2_TPP:
            hipLaunchKernelGGL((hub_persistent_kernel<SE_TPP, MIXED, RH>), dim3(1), dim3(PERSIST_THREADS), 0,
                               c->stream, p);
            break;
        case G1G2_TPH:
            hipLaunchKernelGGL((hub_persistent_kernel<SE_TPH, MIXED, RH>), dim3(1), dim3(PERSIST_THREADS), 0,
                               c->stream, p);
            break;
        default:
            hipLaunchKernelGGL((hub_persistent_kernel<SE_SOA, MIXED, RH>), dim3(1), dim3(PERSIST_THREADS), 0,
                               c->stream, p);
            break;
    }
}

g1g2_status hub_step_persistent(g1g2_ctx* c, double dt, int64_t nsteps) {
    HubbardData& H = c->hub;
    // bounded launches: at most 1024 steps (a few ms) per launch
    for (int64_t n = 0; n < nsteps;) {
        const int chunk = (int)std::min<int64_t>(nsteps - n, 1024);
        PersistArgs p{H.desc, H.nbr, H.hop, H.d0, H.xdrv, c->y.g1, c->y.g2, dt, chunk, guard_of(c)};
        const bool mixed = c->d.precision == G1G2_MIXED;
        if (H.realhop) {
            if (mixed) launch_persistent<true, true>(c, p);
            else launch_persistent<false, true>(c, p);
        } else {
            if (mixed) launch_persistent<true, false>(c, p);
            else launch_persistent<false, false>(c, p);
        }
        HIP_OK(c, hipGetLastError());
        n += chunk;
    }
    return G1G2_OK;
}

g1g2_status hub_stage(g1g2_ctx* c, int mode, double t, const Regs& in, const Regs& y,
                      const Regs& acc, const Regs& out, double cb, double cc) {
    return hub_stage_diag(c, mode, t, in, y, acc, out, cb, cc, c->hub.diag);
}

g1g2_status hub_stage_diag(g1g2_ctx* c, int mode, double t, const Regs& in, const Regs& y,
                           const Regs& acc, const Regs& out, double cb, double cc, cd* diag) {
    StageArgs s = make_stage(c, t, in, y, acc, out, cb, cc);
    s.diag = diag;
    switch (mode) {
        case RK_RHS: return launch_stage<RK_RHS>(c, s);
        case RK_FIRST: return launch_stage<RK_FIRST>(c, s);
        case RK_MID: return launch_stage<RK_MID>(c, s);
        default: return launch_stage<RK_LAST>(c, s);
    }
}

g1g2_status hub_batch_observables(g1g2_ctx* c, const Regs& s, double t, g1g2_obs* o) {
    HubbardData& H = c->hub;
    const int n = H.ncl;
    double* res = nullptr;
    HIP_OK(c, hipMalloc((void**)&res, (size_t)n * 8 * sizeof(double)));
    hipLaunchKernelGGL(hub_obs_kernel, dim3(n), dim3(256), 0, c->stream, H.desc, H.nbr, H.hop, H.d0,
                       H.xdrv, H.drive_value(t), c->switch_value(t), s.g1, s.g2, res);
    hipError_t e1 = hipGetLastError();
    std::vector<double> h((size_t)n * 8);
    hipError_t e2 = hipMemcpyAsync(h.data(), res, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                                   c->stream);
    hipError_t e3 = hipStreamSynchronize(c->stream);
    (void)hipFree(res);
    HIP_OK(c, e1);
    HIP_OK(c, e2);
    HIP_OK(c, e3);
    for (int cl = 0; cl < n; ++cl) {
        const double* r = &h[(size_t)cl * 8];
        g1g2_obs& ob = o[cl];
        ob.N[0] = r[0];
        ob.N[1] = r[1];
        ob.E_kin = r[2];
        ob.E_mf = r[3];
        ob.E_corr = r[4];
        ob.E_tot = r[2] + r[3] + r[4];
        ob.docc = r[5] / H.hdesc[cl].ns;
        ob.imbalance = (r[0] + r[1]) > 0.0 ? r[6] / (r[0] + r[1]) : 0.0;
        ob.herm_resid = 0.0;
        ob.exch_resid = 0.0;
    }
    return G1G2_OK;
}

g1g2_status hub_observables(g1g2_ctx* c, const Regs& s, double t, g1g2_obs* o) {
    g1g2_status st = hub_batch_observables(c, s, t, o);
    if (st != G1G2_OK) return st;
    const int ns = c->hub.hdesc[0].ns;
    long long n4 = (long long)ns * ns * ns * ns;
    const int nblk = 256;
    hipLaunchKernelGGL(herm_resid_kernel, dim3(nblk), dim3(256), 0, c->stream, s.g2, ns * ns, n4,
                       c->dscratch + 8);
    HIP_OK(c, hipGetLastError());
    std::vector<double> h(2 * nblk);
    HIP_OK(c, hipMemcpyAsync(h.data(), c->dscratch + 8, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    double m1 = 0, m2 = 0;
    for (int b = 0; b < nblk; ++b) {
        m1 = std::max(m1, h[2 * b]);
        m2 = std::max(m2, h[2 * b + 1]);
    }
    o->herm_resid = m2 > 0 ? m1 / m2 : 0.0;
    return G1G2_OK;
}

g1g2_status hub_site_observables(g1g2_ctx* c, const Regs& s, double* nu, double* nd, double* docc) {
    HubbardData& H = c->hub;
    const int ns = H.hdesc[0].ns;
    hipLaunchKernelGGL(hub_site_kernel, dim3((ns + 255) / 256), dim3(256), 0, c->stream, H.desc, H.nbr,
                       H.hop, H.d0, H.xdrv, s.g1, s.g2, c->dscratch);
    HIP_OK(c, hipGetLastError());
    std::vector<double> h(3 * ns);
    HIP_OK(c, hipMemcpyAsync(h.data(), c->dscratch, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (nu) std::memcpy(nu, h.data(), ns * sizeof(double));
    if (nd) std::memcpy(nd, h.data() + ns, ns * sizeof(double));
    if (docc) std::memcpy(docc, h.data() + 2 * ns, ns * sizeof(double));
    return G1G2_OK;
}

// --------------------------------------------------------------------------- allocation-free RHS
// The right-hand side of one Hubbard cluster without any allocation: the
// diagonal gathers of TPH, GW and DSL (n_diag ns^3 complex elements) go to a
// static device array of NOALLOC_SCRATCH_BYTES instead of the context's
// buffer.  Each GPU holds its own copy of the array until the process ends;
// every call on a GPU shares it.  Host code never passes the array's name to a
// kernel: its device address is looked up per device at context set-up
// (hub_noalloc_setup) and that address is what the kernels receive.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(32) << 20;   // DSL at ns = 64: 8 * 64^3 * 16 B
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
void* noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

size_t hub_diag_bytes(const g1g2_ctx* c) { return (size_t)c->hub.diag_elems * sizeof(cd); }

g1g2_status hub_noalloc_setup(g1g2_ctx* c) {
    int dev = -1;
    HIP_OK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return set_error(c, G1G2_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (noalloc_ptr[dev]) return G1G2_OK;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return set_error(c, G1G2_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    noalloc_ptr[dev] = p;
    return G1G2_OK;
}

extern "C" g1g2_status g1g2_rhs_noalloc(g1g2_ctx* c, double t, const void* G1, const void* G2, void* dG1,
                                        void* dG2) {
    if (!c || !G1 || !G2 || !dG1 || !dG2) return G1G2_EINVAL;
    if (c->d.basis != G1G2_HUBBARD)
        return set_error(c, G1G2_EUNSUPPORTED, "g1g2_rhs_noalloc: Hubbard basis only");
    if (c->hub.ncl != 1) return set_error(c, G1G2_ESTATE, "g1g2_rhs_noalloc: single-cluster call on a batch");
    const size_t need = hub_diag_bytes(c);
    if (need > NOALLOC_SCRATCH_BYTES)
        return set_error(c, G1G2_EINVAL,
                         "g1g2_rhs_noalloc: the diagonal gathers need " + std::to_string(need) +
                             " bytes of scratch, more than its " + std::to_string(NOALLOC_SCRATCH_BYTES));
    void* ptr = nullptr;
    if (c->device >= 0 && c->device < NOALLOC_MAX_DEVICES) {
        std::lock_guard<std::mutex> lock(noalloc_mu);
        ptr = noalloc_ptr[c->device];
    }
    if (!ptr) return set_error(c, G1G2_ESTATE, "g1g2_rhs_noalloc: no scratch address for the context's device");
    Regs in{(cd*)G1, (cd*)G2};
    Regs out{(cd*)dG1, (cd*)dG2};
    return hub_stage_diag(c, RK_RHS, t, in, in, in, out, 0.0, 0.0, (cd*)ptr);
}
