// Per-cluster view of the Hubbard data used by the forward and adjoint kernels.
#pragma once
#include "ctx.h"

namespace hub {

struct Cl {
    int ns, zmax;
    double U, s_drive;   // U of the cluster at the stage time (switching applied)
    const int* __restrict__ nbr;    // [2][ns][zmax]
    const cd* __restrict__ hop;     // [2][ns][zmax]
    const double* __restrict__ d0;  // [2][ns]
    const double* __restrict__ xdrv;
    const cd* __restrict__ X;       // stage-input G^{<,up}
    const cd* __restrict__ Y;       // stage-input G^{<,down}
    const cd* __restrict__ hdg;     // [2][ns] diagonals of h^{HF} when precomputed, else unused
    const double* __restrict__ hopr; // [2][ns][zmax] real parts of hop when all hoppings are real, else unused
};

__device__ __forceinline__ Cl make_cl(const ClusterDesc& d, const int* nbr, const cd* hop,
                                      const double* d0, const double* xdrv, const cd* g1,
                                      double s_drive, double u_scale) {
    Cl a;
    a.ns = d.ns;
    a.zmax = d.zmax;
    a.U = d.U * u_scale;
    a.s_drive = s_drive;
    a.nbr = nbr + d.nbroff;
    a.hop = hop + d.nbroff;
    a.d0 = d0 + d.d0off;
    a.xdrv = xdrv + d.xoff;
    a.X = g1 + d.g1off;
    a.Y = a.X + d.ns * d.ns;
    a.hdg = nullptr;
    a.hopr = nullptr;
    return a;
}

// Diagonal of h^{HF,sigma} (Sec. III.D): h0_ii + v_i(t) - i U G^{<,-sigma}_ii.
__device__ __forceinline__ cd hf_diag(const Cl& a, int sig, int i) {
    const cd* other = sig ? a.X : a.Y;
    cd g = other[i * a.ns + i];
    double re = a.d0[sig * a.ns + i] + a.s_drive * a.xdrv[i];
    // -i U (g.x + i g.y) = U g.y - i U g.x
    return cmk(re + a.U * g.y, -a.U * g.x);
}

}  // namespace hub
