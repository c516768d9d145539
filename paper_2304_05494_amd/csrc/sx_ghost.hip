// sx_ghost.hip -- on-device ghost-cell fill of a ghosted state.
//
// The paper keeps ng ghost layers around every block (ghosted w array,
// Section 3.2) and fills them by exchange or boundary conditions; it states
// no boundary formulas. Readings used here: periodic copies; isothermal
// no-slip wall by reflection about the wall face (velocity odd, pressure
// even, T_g = 2 T_wall - T_m, density from the equation of state);
// zeroth-order extrapolation; frozen (caller-owned Dirichlet) faces are left
// alone. Directions are filled x, then y over the full ghosted x range, then
// z over the full ghosted x and y ranges, so edges and corners are consistent.
#include "sx_internal.h"

namespace sx {

// One thread per ghost node of direction D (both sides, all layers).
template <int D>
__global__ void __launch_bounds__(256) k_ghost(KGrid g, KGas gas, double* __restrict__ W)
{
    const int ng = g.ng;
    // extents of the face-parallel index ranges (a: fastest, b: slowest)
    int na, nb, alo, blo;
    if (D == 0) { na = g.ny; nb = g.nz; alo = 0; blo = 0; }
    else if (D == 1) { na = g.nx + 2 * ng; nb = g.nz; alo = -ng; blo = 0; }
    else { na = g.nx + 2 * ng; nb = g.ny + 2 * ng; alo = -ng; blo = -ng; }
    const long long per_side = (long long)na * nb * ng;
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * per_side) return;
    int side = (int)(t / per_side);
    long long rem = t - side * per_side;
    int l, a, b;
    if (D == 0) {   // layer fastest: neighbouring threads touch neighbouring columns
        l = (int)(rem % ng);
        long long q = rem / ng;
        a = (int)(q % na) + alo;
        b = (int)(q / na) + blo;
    } else {        // row index fastest (coalesced along x)
        a = (int)(rem % na) + alo;
        long long q = rem / na;
        l = (int)(q % ng);
        b = (int)(q / ng) + blo;
    }
    const int n = D == 0 ? g.nx : (D == 1 ? g.ny : g.nz);
    const int bc = g.bc[2 * D + side];
    if (bc == SX_BC_FROZEN) return;
    int gd, md;
    if (side == 0) {
        gd = -1 - l;
        md = bc == SX_BC_PERIODIC ? n - 1 - l : (bc == SX_BC_WALL ? l : 0);
    } else {
        gd = n + l;
        md = bc == SX_BC_PERIODIC ? l : (bc == SX_BC_WALL ? n - 1 - l : n - 1);
    }
    long long gi, mi;
    if (D == 0) {
        gi = g.base + b * g.sz + a * g.sy + gd;
        mi = g.base + b * g.sz + a * g.sy + md;
    } else if (D == 1) {
        gi = g.base + b * g.sz + (long long)gd * g.sy + a;
        mi = g.base + b * g.sz + (long long)md * g.sy + a;
    } else {
        gi = g.base + (long long)gd * g.sz + (long long)b * g.sy + a;
        mi = g.base + (long long)md * g.sz + (long long)b * g.sy + a;
    }
    if (bc != SX_BC_WALL) {
#pragma unroll
        for (int v = 0; v < NV; ++v) W[v * g.sv + gi] = W[v * g.sv + mi];
        return;
    }
    const double rho = W[mi];
    const double ri = 1.0 / rho;
    const double u = W[g.sv + mi] * ri, v = W[2 * g.sv + mi] * ri, w = W[3 * g.sv + mi] * ri;
    double p, Tm;
    if (gas.thermo) {   // thermally perfect: T from the internal energy
        Tm = tp_T_of_e(gas, W[4 * g.sv + mi] * ri - 0.5 * (u * u + v * v + w * w));
        p = rho * Tm * gas.igM2;
    } else {
        p = gas.gm1 * (W[4 * g.sv + mi] - 0.5 * rho * (u * u + v * v + w * w));
        Tm = gas.gM2 * p * ri;
    }
    const double Tg = 2.0 * gas.t_wall - Tm;
    const double rg = gas.gM2 * p / Tg;
    W[gi] = rg;
    W[g.sv + gi] = -rg * u;
    W[2 * g.sv + gi] = -rg * v;
    W[3 * g.sv + gi] = -rg * w;
    const double eg = gas.thermo ? rg * gas.igM2 * tp_eR(gas, Tg) : p / gas.gm1;
    W[4 * g.sv + gi] = eg + 0.5 * rg * (u * u + v * v + w * w);
}

hipError_t launch_ghost_fill(const KGrid& g, const KGas& gas, double* W, hipStream_t st)
{
    const int ng = g.ng;
    long long n0 = 2LL * g.ny * g.nz * ng;
    long long n1 = 2LL * (g.nx + 2 * ng) * g.nz * ng;
    long long n2 = 2LL * (g.nx + 2 * ng) * (g.ny + 2 * ng) * ng;
    const int B = 256;
    hipLaunchKernelGGL(k_ghost<0>, dim3((unsigned)((n0 + B - 1) / B)), dim3(B), 0, st, g, gas, W);
    hipLaunchKernelGGL(k_ghost<1>, dim3((unsigned)((n1 + B - 1) / B)), dim3(B), 0, st, g, gas, W);
    hipLaunchKernelGGL(k_ghost<2>, dim3((unsigned)((n2 + B - 1) / B)), dim3(B), 0, st, g, gas, W);
    return hipGetLastError();
}

}  // namespace sx
