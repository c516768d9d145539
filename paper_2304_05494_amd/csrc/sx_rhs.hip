// sx_rhs.hip -- fused right-hand side (+ low-storage RK3 update) for the
// central split-form path: convective x/y/z derivatives, Laplacian-form
// viscous and heat-flux terms (Section 2 of the paper), one kernel per
// substep.
//
// Mapping (gfx950, wave64): a workgroup owns a TX x TY column tile (lanes
// along contiguous x, so every row load is coalesced) and marches along z
// over a chunk of planes. Each iteration stages two planes of primitives
// (rho, u, v, w, T) with an S-wide halo in LDS:
//   * the arrival plane k+S feeds per-column register queues: primitives
//     for the z stencils, and the in-plane derivatives (D_x w, D_y w,
//     D_x u + D_y v) whose z-derivatives are the mixed viscous terms;
//   * the output plane k feeds the in-plane (x, y) stencils.
// The y-derivatives of u and v are also computed over the x-halo columns
// into a small LDS row so D_x(D_y .) costs one short stencil. The RHS of a
// node never leaves registers: in update mode the kernel applies the RK3
// substep and writes the new state and the RK register directly, so HBM
// traffic per substep is one read of W, one write of W' and the RK register.
#include "sx_internal.h"

namespace sx {

struct Prim {
    double r, u, v, w, T;
};

__device__ __forceinline__ Prim load_prim(const double* __restrict__ W, long long n, long long sv,
                                          const KGas& gas)
{
    Prim q;
    const double rho = W[n];
    const double ri = 1.0 / rho;
    q.r = rho;
    q.u = W[n + sv] * ri;
    q.v = W[n + 2 * sv] * ri;
    q.w = W[n + 3 * sv] * ri;
    const double p = gas.gm1 * (W[n + 4 * sv] - 0.5 * rho * (q.u * q.u + q.v * q.v + q.w * q.w));
    q.T = gas.gM2 * p * ri;
    return q;
}

// Convective derivative along one direction from 2S+1 nodes (centre S),
// pair-difference form of the split flux:
//   F_{i+1/2} - F_{i-1/2} = sum_l 2 a_l [P_l(i) - P_l(i-l)],
//   P_l(n) = 1/8 (rho_n + rho_{n+l})(ud_n + ud_{n+l})(phi_n + phi_{n+l}),
// phi in {1, u, v, w, H}, pressure 1/2 (p_n + p_{n+l}) in the D-momentum.
// Subtracts scale * (flux difference) from acc.
template <int S, int D>
__device__ __forceinline__ void conv_dir(const double (&r)[2 * S + 1], const double (&u)[2 * S + 1],
                                         const double (&v)[2 * S + 1], const double (&w)[2 * S + 1],
                                         const double (&T)[2 * S + 1], const KGas& gas, double scale,
                                         double (&acc)[NV])
{
    double p[2 * S + 1], H[2 * S + 1];
#pragma unroll
    for (int t = 0; t < 2 * S + 1; ++t) {
        p[t] = r[t] * T[t] * gas.igM2;
        H[t] = gas.cp * T[t] + 0.5 * (u[t] * u[t] + v[t] * v[t] + w[t] * w[t]);
    }
    const double(&ud)[2 * S + 1] = D == 0 ? u : (D == 1 ? v : w);
    double f0 = 0.0, f1 = 0.0, f2 = 0.0, f3 = 0.0, f4 = 0.0, fp = 0.0;
#pragma unroll
    for (int l = 1; l <= S; ++l) {
        const double cl = 0.25 * Coef<S>::a[l];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int A = side == 0 ? S : S - l;
            const int B = A + l;
            const double c = side == 0 ? cl : -cl;
            const double mf = c * (r[A] + r[B]) * (ud[A] + ud[B]);
            f0 += 2.0 * mf;
            f1 += mf * (u[A] + u[B]);
            f2 += mf * (v[A] + v[B]);
            f3 += mf * (w[A] + w[B]);
            f4 += mf * (H[A] + H[B]);
            fp += 4.0 * c * (p[A] + p[B]);
        }
    }
    if (D == 0) f1 += fp;
    if (D == 1) f2 += fp;
    if (D == 2) f3 += fp;
    acc[0] -= scale * f0;
    acc[1] -= scale * f1;
    acc[2] -= scale * f2;
    acc[3] -= scale * f3;
    acc[4] -= scale * f4;
}

template <int S>
__device__ __forceinline__ double d1(const double (&f)[2 * S + 1])
{
    double s = 0.0;
#pragma unroll
    for (int l = 1; l <= S; ++l) s += Coef<S>::a[l] * (f[S + l] - f[S - l]);
    return s;
}

template <int S>
__device__ __forceinline__ double d2(const double (&f)[2 * S + 1])
{
    double s = 0.0;
#pragma unroll
    for (int l = 1; l <= S; ++l) s += Coef<S>::b[l] * ((f[S + l] - 2.0 * f[S]) + f[S - l]);
    return s;
}

template <int S, int TX, int TY, bool UPD>
__global__ void __attribute__((amdgpu_flat_work_group_size(TX * TY, TX * TY)))
k_rhs_central(const double* __restrict__ W, double* __restrict__ out, double* __restrict__ Rp,
              KGrid g, KGas gas, StepCoef sc, unsigned mask, int kc)
{
    constexpr int NT = TX * TY;
    constexpr int HX = TX + 2 * S, HY = TY + 2 * S, HP = HX * HY;
    constexpr int Q = 2 * S + 1;
    __shared__ double sa[5][HP];      // arrival plane k+S
    __shared__ double so[5][HP];      // output plane k
    __shared__ double gyl[2][TY][HX]; // D_y u, D_y v of plane k over x-halo columns

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
    const int k0 = blockIdx.z * kc;
    const int k1 = min(k0 + kc, g.nz);
    const int i = i0 + tx, j = j0 + ty;
    const bool active = i < g.nx && j < g.ny;
    const int c = (ty + S) * HX + (tx + S);
    const double ey = active ? g.eta_y[j] : 0.0;
    const double eyy = active ? g.eta_yy[j] : 0.0;
    const double dxi = g.dxi, dzi = g.dzi;

    double zq[5][Q];  // primitives of this column, planes k-S .. k+S
    double mq[3][Q];  // D_x w, D_y w, D_x u + D_y v of this column
#pragma unroll
    for (int t = 0; t < Q; ++t) {
#pragma unroll
        for (int q = 0; q < 5; ++q) zq[q][t] = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) mq[q][t] = 0.0;
    }

    auto load_plane = [&](double (*buf)[HP], int k) {
        for (int p = tid; p < HP; p += NT) {
            const int hx = p % HX, hy = p / HX;
            const int gi = i0 - S + hx, gj = j0 - S + hy;
            Prim q{1.0, 0.0, 0.0, 0.0, 1.0};
            if (gi >= -g.ng && gi < g.nx + g.ng && gj >= -g.ng && gj < g.ny + g.ng)
                q = load_prim(W, g.base + (long long)k * g.sz + (long long)gj * g.sy + gi, g.sv, gas);
            buf[0][p] = q.r;
            buf[1][p] = q.u;
            buf[2][p] = q.v;
            buf[3][p] = q.w;
            buf[4][p] = q.T;
        }
    };

    // arrival: fill the last queue slot from sa (plane already staged)
    auto arrive = [&]() {
        if (!active) return;
#pragma unroll
        for (int q = 0; q < 5; ++q) zq[q][Q - 1] = sa[q][c];
        double xw[Q], yw[Q], xu[Q], yv[Q];
#pragma unroll
        for (int t = 0; t < Q; ++t) {
            xw[t] = sa[3][c + t - S];
            xu[t] = sa[1][c + t - S];
            yw[t] = sa[3][c + (t - S) * HX];
            yv[t] = sa[2][c + (t - S) * HX];
        }
        mq[0][Q - 1] = dxi * d1<S>(xw);
        mq[1][Q - 1] = ey * d1<S>(yw);
        mq[2][Q - 1] = dxi * d1<S>(xu) + ey * d1<S>(yv);
    };

    auto shift = [&]() {
#pragma unroll
        for (int t = 0; t < Q - 1; ++t) {
#pragma unroll
            for (int q = 0; q < 5; ++q) zq[q][t] = zq[q][t + 1];
#pragma unroll
            for (int q = 0; q < 3; ++q) mq[q][t] = mq[q][t + 1];
        }
    };

    // prologue: planes k0-S .. k0+S-1 into queue slots 0 .. 2S-1
    for (int t = 0; t < 2 * S; ++t) {
        load_plane(sa, k0 - S + t);
        __syncthreads();
        arrive();
        shift();
        __syncthreads();
    }

    for (int k = k0; k < k1; ++k) {
        load_plane(sa, k + S);
        load_plane(so, k);
        __syncthreads();
        arrive();
        // y-derivatives of u, v at plane k over the x-extended columns
        for (int p = tid; p < TY * HX; p += NT) {
            const int hx = p % HX, rr = p / HX;
            const int jj = j0 + rr;
            if (jj < g.ny) {
                const double e = g.eta_y[jj];
                double su = 0.0, sv = 0.0;
#pragma unroll
                for (int l = 1; l <= S; ++l) {
                    const int up = (rr + S + l) * HX + hx, dn = (rr + S - l) * HX + hx;
                    su += Coef<S>::a[l] * (so[1][up] - so[1][dn]);
                    sv += Coef<S>::a[l] * (so[2][up] - so[2][dn]);
                }
                gyl[0][rr][hx] = e * su;
                gyl[1][rr][hx] = e * sv;
            }
        }
        __syncthreads();

        if (active) {
            double acc[NV] = {0.0, 0.0, 0.0, 0.0, 0.0};
            double xr[Q], xu[Q], xv[Q], xw[Q], xT[Q];
            double yr[Q], yu[Q], yv[Q], yw[Q], yT[Q];
#pragma unroll
            for (int t = 0; t < Q; ++t) {
                const int cx = c + t - S, cy = c + (t - S) * HX;
                xr[t] = so[0][cx]; xu[t] = so[1][cx]; xv[t] = so[2][cx]; xw[t] = so[3][cx]; xT[t] = so[4][cx];
                yr[t] = so[0][cy]; yu[t] = so[1][cy]; yv[t] = so[2][cy]; yw[t] = so[3][cy]; yT[t] = so[4][cy];
            }
            if (mask & SX_CONV_X) conv_dir<S, 0>(xr, xu, xv, xw, xT, gas, dxi, acc);
            if (mask & SX_CONV_Y) conv_dir<S, 1>(yr, yu, yv, yw, yT, gas, ey, acc);
            if (mask & SX_CONV_Z) conv_dir<S, 2>(zq[0], zq[1], zq[2], zq[3], zq[4], gas, dzi, acc);

            if (mask & SX_VISC) {
                const double uc = zq[1][S], vc = zq[2][S], wc = zq[3][S], Tc = zq[4][S];
                // gradient tensor gab = d_b u_a and temperature gradient
                const double g00 = dxi * d1<S>(xu), g01 = ey * d1<S>(yu), g02 = dzi * d1<S>(zq[1]);
                const double g10 = dxi * d1<S>(xv), g11 = ey * d1<S>(yv), g12 = dzi * d1<S>(zq[2]);
                const double g20 = dxi * d1<S>(xw), g21 = ey * d1<S>(yw), g22 = dzi * d1<S>(zq[3]);
                const double Tx = dxi * d1<S>(xT), Ty = ey * d1<S>(yT), Tz = dzi * d1<S>(zq[4]);
                const double dxi2 = dxi * dxi, dzi2 = dzi * dzi, ey2 = ey * ey;
                const double uxx = dxi2 * d2<S>(xu), uyy = ey2 * d2<S>(yu) + eyy * d1<S>(yu), uzz = dzi2 * d2<S>(zq[1]);
                const double vxx = dxi2 * d2<S>(xv), vyy = ey2 * d2<S>(yv) + eyy * d1<S>(yv), vzz = dzi2 * d2<S>(zq[2]);
                const double wxx = dxi2 * d2<S>(xw), wyy = ey2 * d2<S>(yw) + eyy * d1<S>(yw), wzz = dzi2 * d2<S>(zq[3]);
                const double Txx = dxi2 * d2<S>(xT), Tyy = ey2 * d2<S>(yT) + eyy * d1<S>(yT), Tzz = dzi2 * d2<S>(zq[4]);
                // mixed derivatives
                double gyu[Q], gyv[Q];
#pragma unroll
                for (int t = 0; t < Q; ++t) {
                    gyu[t] = gyl[0][ty][tx + t];
                    gyv[t] = gyl[1][ty][tx + t];
                }
                const double dxy_u = dxi * d1<S>(gyu);   // d_x d_y u
                const double dxy_v = dxi * d1<S>(gyv);   // d_x d_y v
                const double dxz_w = dzi * d1<S>(mq[0]); // d_z d_x w
                const double dyz_w = dzi * d1<S>(mq[1]); // d_z d_y w
                const double dz_div = dzi * d1<S>(mq[2]); // d_z (d_x u + d_y v)
                const double th = g00 + g11 + g22;
                const double dth0 = uxx + dxy_v + dxz_w;
                const double dth1 = vyy + dxy_u + dyz_w;
                const double dth2 = wzz + dz_div;
                const double mu = pow(Tc, gas.s) * gas.ire;
                const double kc_ = mu * gas.cp * gas.ipr;
                const double smt = gas.s / Tc;
                const double dmu0 = smt * mu * Tx, dmu1 = smt * mu * Ty, dmu2 = smt * mu * Tz;
                const double t3 = 2.0 / 3.0;
                const double V0 = mu * ((uxx + uyy + uzz) + dth0 * (1.0 / 3.0)) + dmu0 * (g00 + g00) +
                                  dmu1 * (g01 + g10) + dmu2 * (g02 + g20) - t3 * dmu0 * th;
                const double V1 = mu * ((vxx + vyy + vzz) + dth1 * (1.0 / 3.0)) + dmu0 * (g10 + g01) +
                                  dmu1 * (g11 + g11) + dmu2 * (g12 + g21) - t3 * dmu1 * th;
                const double V2 = mu * ((wxx + wyy + wzz) + dth2 * (1.0 / 3.0)) + dmu0 * (g20 + g02) +
                                  dmu1 * (g21 + g12) + dmu2 * (g22 + g22) - t3 * dmu2 * th;
                // tau_ab d_b u_a
                const double s01 = g01 + g10, s02 = g02 + g20, s12 = g12 + g21;
                const double diss = mu * ((2.0 * g00 - t3 * th) * g00 + (2.0 * g11 - t3 * th) * g11 +
                                          (2.0 * g22 - t3 * th) * g22 + s01 * s01 + s02 * s02 + s12 * s12);
                const double dk = smt * kc_;
                const double VE = uc * V0 + vc * V1 + wc * V2 + diss + kc_ * (Txx + Tyy + Tzz) +
                                  dk * (Tx * Tx + Ty * Ty + Tz * Tz);
                acc[1] += V0;
                acc[2] += V1;
                acc[3] += V2;
                acc[4] += VE;
            }

            const long long m = ((long long)k * g.ny + j) * g.nx + i;
            if (UPD) {
                const long long n = g.base + (long long)k * g.sz + (long long)j * g.sy + i;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double nv = W[v * g.sv + n] + sc.cg * acc[v];
                    if (sc.read_prev) nv += sc.cz * Rp[v * g.nint + m];
                    out[v * g.sv + n] = nv;
                    if (sc.write_prev) Rp[v * g.nint + m] = acc[v];
                }
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v) out[v * g.nint + m] = acc[v];
            }
        }
        shift();
        __syncthreads();
    }
}

template <int S>
static hipError_t launch_rhs_S(const KGrid& g, const KGas& gas, const double* W, double* out,
                               double* Rprev, const StepCoef* step, unsigned mask, hipStream_t st)
{
    constexpr int TX = 64, TY = 4;
    const int kc = g.nz;  // one march over the whole z extent per tile
    dim3 grid((g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, (g.nz + kc - 1) / kc);
    if (step) {
        hipLaunchKernelGGL((k_rhs_central<S, TX, TY, true>), grid, dim3(TX * TY), 0, st, W, out, Rprev,
                           g, gas, *step, (unsigned)SX_ALL, kc);
    } else {
        StepCoef none{0.0, 0.0, 0, 0};
        hipLaunchKernelGGL((k_rhs_central<S, TX, TY, false>), grid, dim3(TX * TY), 0, st, W, out,
                           Rprev, g, gas, none, mask, kc);
    }
    return hipGetLastError();
}

hipError_t launch_rhs(const KGrid& g, const KGas& gas, const KScheme& sc, const double* W,
                      double* out, double* Rprev, const StepCoef* step, unsigned mask,
                      hipStream_t st)
{
    switch (sc.L) {
    case 1: return launch_rhs_S<1>(g, gas, W, out, Rprev, step, mask, st);
    case 2: return launch_rhs_S<2>(g, gas, W, out, Rprev, step, mask, st);
    case 3: return launch_rhs_S<3>(g, gas, W, out, Rprev, step, mask, st);
    case 4: return launch_rhs_S<4>(g, gas, W, out, Rprev, step, mask, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sx
