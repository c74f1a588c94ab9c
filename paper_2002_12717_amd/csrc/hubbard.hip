// Hubbard-basis G1-G2 kernels (Sec. III.D, Sec. V.A, Sec. VII).
//
// State per register: G1 = [X | Y] with X = G^{<,up}, Y = G^{<,down} (ns x ns
// each) and G2 = A = G2^{up down up down} ([ns]^4).  Every G2 element is
// produced by one thread from a fixed number of neighbours, so the kernel is a
// bandwidth-bound stream: the O(ns^5) sums of the direct formulation are
// replaced by the paper's reformulations that carry no inner sum
// (eq:soa-cubic-scheme for the source, the tridiagonal-h commutator of
// Sec. VII.A, the reformulated ladder of Sec. VII.C).
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.h"

namespace {

struct HubArgs {
    int ns, zmax;
    double U, s_drive;
    const int* __restrict__ nbr;    // [2][ns][zmax]
    const cd* __restrict__ hop;     // [2][ns][zmax]
    const double* __restrict__ d0;  // [2][ns]
    const double* __restrict__ xdrv;
    const cd* __restrict__ X;       // stage-input G^{<,up}
    const cd* __restrict__ Y;       // stage-input G^{<,down}
};

// Diagonal of h^{HF,sigma} (Sec. III.D): h0_ii + v_i(t) - i U G^{<,-sigma}_ii.
__device__ __forceinline__ cd hf_diag(const HubArgs& a, int sig, int i) {
    const cd* other = sig ? a.X : a.Y;
    cd g = other[i * a.ns + i];
    double re = a.d0[sig * a.ns + i] + a.s_drive * a.xdrv[i];
    // -i U (g.x + i g.y) = U g.y - i U g.x
    return cmk(re + a.U * g.y, -a.U * g.x);
}

// Right-hand side of one element of A = G2^{up down up down}:
//   dA/dt = -i ( [h2_{ud}, A] + Psi + [L^pp - (L^pp_klij)^*] )
template <bool TPP>
__device__ __forceinline__ cd hub_g2_rhs(const HubArgs& a, const cd* __restrict__ A, int i, int j,
                                         int k, int l, int e, cd aval) {
    const int ns = a.ns, ns2 = ns * ns, ns3 = ns2 * ns, z = a.zmax;
    const int* nbu = a.nbr;
    const int* nbd = a.nbr + ns * z;
    const cd* hu = a.hop;
    const cd* hd = a.hop + ns * z;
    // two-particle commutator (Sec. VII.A with the on-site terms of h0 + drive)
    cd ei = hf_diag(a, 0, i), ej = hf_diag(a, 1, j), ek = hf_diag(a, 0, k), el = hf_diag(a, 1, l);
    cd c = cmul(cmk(ei.x + ej.x - ek.x - el.x, ei.y + ej.y - ek.y - el.y), aval);
    for (int q = 0; q < z; ++q) {
        int p = nbu[i * z + q];
        if (p >= 0) c = cfma(c, hu[i * z + q], A[e + (p - i) * ns3]);
    }
    for (int q = 0; q < z; ++q) {
        int p = nbd[j * z + q];
        if (p >= 0) c = cfma(c, hd[j * z + q], A[e + (p - j) * ns2]);
    }
    cd r = cmk(0.0, 0.0);
    for (int q = 0; q < z; ++q) {  // sum_p A_ijpl h_pk, h_pk = conj(h_kp)
        int p = nbu[k * z + q];
        if (p >= 0) r = cfma_conjb(r, A[e + (p - k) * ns], hu[k * z + q]);
    }
    for (int q = 0; q < z; ++q) {  // sum_p A_ijkp h_pl
        int p = nbd[l * z + q];
        if (p >= 0) r = cfma_conjb(r, A[e + (p - l)], hd[l * z + q]);
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
    if (TPP) {
        // L_ijkl = delta_ij U A_iikl + i U (Y_ji A_iikl + X_ij A_jjkl)   (Sec. VII.C)
        int kl = k * ns + l, ij = i * ns + j;
        cd dii = A[(i * ns + i) * ns2 + kl], djj = A[(j * ns + j) * ns2 + kl];
        cd l1 = cmul_i(cadd(cmul(yji, dii), cmul(xij, djj)));
        if (i == j) l1 = cadd(l1, dii);
        cd dkk = A[(k * ns + k) * ns2 + ij], dll = A[(l * ns + l) * ns2 + ij];
        cd ylk = Y[l * ns + k], xkl = X[k * ns + l];
        cd l2 = cmul_i(cadd(cmul(ylk, dkk), cmul(xkl, dll)));
        if (k == l) l2 = cadd(l2, dkk);
        c = cadd(c, cscale(csub(l1, cconj(l2)), a.U));
    }
    return cmul_mi(c);
}

template <int MODE, bool TPP>
__global__ __launch_bounds__(256) void hub_g2_kernel(HubArgs a, const cd* __restrict__ in,
                                                    const cd* __restrict__ y, cd* __restrict__ acc,
                                                    cd* __restrict__ out, double cb, double cc) {
    const int ns = a.ns;
    const int n4 = ns * ns * ns * ns;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n4; e += gridDim.x * blockDim.x) {
        int l = e % ns, tq = e / ns;
        int k = tq % ns;
        tq /= ns;
        int j = tq % ns, i = tq / ns;
        cd av = in[e];
        cd f = hub_g2_rhs<TPP>(a, in, i, j, k, l, e, av);
        rk_update<MODE>(e, f, av, y, acc, out, cb, cc);
    }
}

// G1 equations (eq:eom_g1_hubbard): dG^{<,s}/dt = -i([h^{HF,s}, G^{<,s}] + I^s + I^s^dagger)
// with I^up_ij = -i U A_iiji and I^down_ij = -i U A_iiij.
template <int MODE>
__global__ __launch_bounds__(256) void hub_g1_kernel(HubArgs a, const cd* __restrict__ A,
                                                    const cd* __restrict__ in,
                                                    const cd* __restrict__ y, cd* __restrict__ acc,
                                                    cd* __restrict__ out, double cb, double cc,
                                                    int* __restrict__ flag) {
    const int ns = a.ns, ns2 = ns * ns, z = a.zmax;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 2 * ns2; e += gridDim.x * blockDim.x) {
        int sig = e / ns2, r = e % ns2, i = r / ns, j = r % ns;
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
            Iij = A[((i * ns + i) * ns + j) * ns + i];
            Iji = A[((j * ns + j) * ns + i) * ns + j];
        } else {
            Iij = A[((i * ns + i) * ns + i) * ns + j];
            Iji = A[((j * ns + j) * ns + j) * ns + i];
        }
        // I = -i U A...,  I + I^dagger with (I^dagger)_ij = conj(I_ji)
        cd coll = cadd(cscale(cmul_mi(Iij), a.U), cconj(cscale(cmul_mi(Iji), a.U)));
        cd f = cmul_mi(cadd(c, coll));
        rk_update<MODE>(e, f, gij, y, acc, out, cb, cc);
        if (MODE == RK_LAST) {
            cd v = out[e];
            bool bad = !(isfinite(v.x) && isfinite(v.y));
            if (i == j && (v.y < -0.5 || v.y > 1.5)) bad = true;  // n_ii = -i G_ii = G_ii.y
            if (bad) atomicOr(flag, 1);
        }
    }
}

HubArgs make_args(g1g2_ctx* c, double t, const Regs& in) {
    HubArgs a;
    a.ns = c->hub.ns;
    a.zmax = c->hub.zmax;
    a.U = c->d.U;
    a.s_drive = c->hub.drive_value(t);
    a.nbr = c->hub.nbr;
    a.hop = c->hub.hop;
    a.d0 = c->hub.d0;
    a.xdrv = c->hub.xdrv;
    a.X = in.g1;
    a.Y = in.g1 + (size_t)a.ns * a.ns;
    return a;
}

template <int MODE>
g1g2_status launch_stage(g1g2_ctx* c, const HubArgs& a, const Regs& in, const Regs& y,
                         const Regs& acc, const Regs& out, double cb, double cc) {
    const int ns = a.ns;
    const int n4 = ns * ns * ns * ns;
    int blocks = (n4 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    bool tpp = c->d.selfenergy == G1G2_TPP;
    if (tpp)
        hipLaunchKernelGGL((hub_g2_kernel<MODE, true>), dim3(blocks), dim3(256), 0, c->stream, a,
                           in.g2, y.g2, acc.g2, out.g2, cb, cc);
    else
        hipLaunchKernelGGL((hub_g2_kernel<MODE, false>), dim3(blocks), dim3(256), 0, c->stream, a,
                           in.g2, y.g2, acc.g2, out.g2, cb, cc);
    HIP_OK(c, hipGetLastError());
    prof_mark(c, "hub_g2");
    int b1 = (2 * ns * ns + 255) / 256;
    hipLaunchKernelGGL((hub_g1_kernel<MODE>), dim3(b1), dim3(256), 0, c->stream, a, in.g2, in.g1,
                       y.g1, acc.g1, out.g1, cb, cc, c->dflag);
    HIP_OK(c, hipGetLastError());
    prof_mark(c, "hub_g1");
    return G1G2_OK;
}

// Observables: one work-group; partial sums in binary64.
__global__ __launch_bounds__(256) void hub_obs_kernel(HubArgs a, const cd* __restrict__ A,
                                                     double* __restrict__ res) {
    __shared__ double sh[8][256];
    const int ns = a.ns, z = a.zmax, tid = threadIdx.x;
    double nu = 0, nd = 0, ekin = 0, emf = 0, ecorr = 0, docc = 0;
    for (int i = tid; i < ns; i += blockDim.x) {
        double niu = a.X[i * ns + i].y, nid = a.Y[i * ns + i].y;
        nu += niu;
        nd += nid;
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
    double v[6] = {nu, nd, ekin, emf, ecorr, docc};
    for (int q = 0; q < 6; ++q) sh[q][tid] = v[q];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s)
            for (int q = 0; q < 6; ++q) sh[q][tid] += sh[q][tid + s];
        __syncthreads();
    }
    if (tid == 0)
        for (int q = 0; q < 6; ++q) res[q] = sh[q][0];
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

__global__ void hub_site_kernel(HubArgs a, const cd* __restrict__ A, double* __restrict__ out) {
    const int ns = a.ns;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x) {
        double niu = a.X[i * ns + i].y, nid = a.Y[i * ns + i].y;
        out[i] = niu;
        out[ns + i] = nid;
        out[2 * ns + i] = niu * nid - A[((i * ns + i) * ns + i) * ns + i].x;
    }
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

g1g2_status hub_setup(g1g2_ctx* c, const cd* h0) {
    const int ns = c->d.nb;
    // Hermiticity check and sparsity pattern
    int zmax = 0;
    std::vector<std::vector<std::pair<int, cd>>> rows(2 * ns);
    std::vector<double> d0(2 * ns);
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < ns; ++i)
            for (int j = 0; j < ns; ++j) {
                cd v = h0[(size_t)s * ns * ns + i * ns + j];
                cd vt = h0[(size_t)s * ns * ns + j * ns + i];
                if (std::fabs(v.x - vt.x) > 1e-12 * (1 + std::fabs(v.x)) ||
                    std::fabs(v.y + vt.y) > 1e-12 * (1 + std::fabs(v.y)))
                    return set_error(c, G1G2_EINVAL, "h0 is not Hermitian");
                if (i == j) {
                    d0[s * ns + i] = v.x;
                } else if (v.x != 0.0 || v.y != 0.0) {
                    rows[s * ns + i].push_back({j, v});
                }
            }
    for (auto& r : rows) zmax = std::max<int>(zmax, (int)r.size());
    if (zmax < 1) zmax = 1;
    std::vector<int> nbr((size_t)2 * ns * zmax, -1);
    std::vector<cd> hop((size_t)2 * ns * zmax, cmk(0, 0));
    for (int r = 0; r < 2 * ns; ++r)
        for (size_t q = 0; q < rows[r].size(); ++q) {
            nbr[(size_t)r * zmax + q] = rows[r][q].first;
            hop[(size_t)r * zmax + q] = rows[r][q].second;
        }
    auto& H = c->hub;
    if (H.nbr) {
        (void)hipFree(H.nbr);
        (void)hipFree(H.hop);
        H.nbr = nullptr;
        H.hop = nullptr;
    }
    H.ns = ns;
    H.zmax = zmax;
    HIP_OK(c, hipMalloc(&H.nbr, nbr.size() * sizeof(int)));
    HIP_OK(c, hipMalloc(&H.hop, hop.size() * sizeof(cd)));
    if (!H.d0) HIP_OK(c, hipMalloc(&H.d0, 2 * ns * sizeof(double)));
    if (!H.xdrv) {
        HIP_OK(c, hipMalloc(&H.xdrv, ns * sizeof(double)));
        HIP_OK(c, hipMemsetAsync(H.xdrv, 0, ns * sizeof(double), c->stream));
    }
    HIP_OK(c, hipMemcpyAsync(H.nbr, nbr.data(), nbr.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipMemcpyAsync(H.hop, hop.data(), hop.size() * sizeof(cd), hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipMemcpyAsync(H.d0, d0.data(), d0.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    H.h_d0 = d0;
    return G1G2_OK;
}

g1g2_status hub_stage(g1g2_ctx* c, int mode, double t, const Regs& in, const Regs& y,
                      const Regs& acc, const Regs& out, double cb, double cc) {
    HubArgs a = make_args(c, t, in);
    switch (mode) {
        case RK_RHS: return launch_stage<RK_RHS>(c, a, in, y, acc, out, cb, cc);
        case RK_FIRST: return launch_stage<RK_FIRST>(c, a, in, y, acc, out, cb, cc);
        case RK_MID: return launch_stage<RK_MID>(c, a, in, y, acc, out, cb, cc);
        default: return launch_stage<RK_LAST>(c, a, in, y, acc, out, cb, cc);
    }
}

g1g2_status hub_observables(g1g2_ctx* c, const Regs& s, double t, g1g2_obs* o) {
    HubArgs a = make_args(c, t, s);
    hipLaunchKernelGGL(hub_obs_kernel, dim3(1), dim3(256), 0, c->stream, a, s.g2, c->dscratch);
    HIP_OK(c, hipGetLastError());
    const int ns = a.ns;
    long long n4 = (long long)ns * ns * ns * ns;
    int nblk = 256;
    hipLaunchKernelGGL(herm_resid_kernel, dim3(nblk), dim3(256), 0, c->stream, s.g2, ns * ns, n4,
                       c->dscratch + 8);
    HIP_OK(c, hipGetLastError());
    std::vector<double> h(8 + 2 * nblk);
    HIP_OK(c, hipMemcpyAsync(h.data(), c->dscratch, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    double m1 = 0, m2 = 0;
    for (int b = 0; b < nblk; ++b) {
        m1 = std::max(m1, h[8 + 2 * b]);
        m2 = std::max(m2, h[8 + 2 * b + 1]);
    }
    o->N[0] = h[0];
    o->N[1] = h[1];
    o->E_kin = h[2];
    o->E_mf = h[3];
    o->E_corr = h[4];
    o->E_tot = h[2] + h[3] + h[4];
    o->docc = h[5] / ns;
    o->herm_resid = m2 > 0 ? m1 / m2 : 0.0;
    return G1G2_OK;
}

g1g2_status hub_site_observables(g1g2_ctx* c, const Regs& s, double* nu, double* nd, double* docc) {
    HubArgs a = make_args(c, c->t, s);
    const int ns = a.ns;
    hipLaunchKernelGGL(hub_site_kernel, dim3((ns + 255) / 256), dim3(256), 0, c->stream, a, s.g2,
                       c->dscratch);
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
