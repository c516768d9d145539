// sx_rhs.hip -- fused right-hand side (+ low-storage RK3 update) for the
// central split-form path: convective x/y/z derivatives and the
// Laplacian-form viscous and heat-flux terms (Section 2 of the paper), one
// kernel per substep.
//
// Mapping (gfx950, wave64): a workgroup owns a TX x TY column tile (lanes
// along contiguous x, so every row load is coalesced) and marches along z.
// Per plane step, LDS holds
//   * the arrival plane k+S (u, v, w with an S-wide halo), whose in-plane
//     derivatives D_x w, D_y w, D_x u + D_y v enter per-column register
//     queues: their z-derivatives are the mixed viscous terms;
//   * the output plane k (records rho, u, v, w, T, p, H with halo) for the
//     x and y stencils, and D_y u, D_y v over the x-halo columns for the
//     mixed x-y terms;
//   * a ring of the last 2S+1 planes of every column's own primitives,
//     which serves the z stencils.
// Global loads of iteration k+1 are issued before the compute of iteration
// k; the stores of iteration k are issued after the staging of k+1. The
// RHS of a node never leaves registers: in update mode the kernel applies
// the RK3 substep and writes the new state and the RK register, so the HBM
// traffic of a substep is one read of W and Rprev, one write of W' and
// Rprev.
//
// FP64 splits the work of a column between two waves: one holds the
// convective terms, the mixed x-y viscous terms and the update, the other
// the mixed-derivative queues and the remaining viscous terms, and passes
// its part of the RHS through LDS. Each wave then needs under 256
// registers, so every SIMD runs two waves whose instruction streams hide
// each other's LDS and memory latencies (one wave of the unsplit FP64 march
// needs ~390 registers and leaves the SIMD idle on every wait). FP32 halves
// the registers and keeps the unsplit march at two waves per SIMD.
//
// Single-block FP64 launches run the plane-ring march (march_ring): each
// plane is fetched from HBM once, with its halo, by both waves together,
// and kept in LDS as primitive records while it serves as arrival plane,
// z-neighbour and output plane, its interior columns then moving to a ring
// of past planes. The batched kernel, whose tiles do not all fit that
// working set, runs march_split, which stages the arrival plane, the output
// plane and the column ring separately; both derive the same values in the
// same order, so a block gives the same bits either way.
//
// Precision forms: R = double (FP64 path) or R = float (FP32-flux form:
// primitives are computed in FP64 and converted once per node, pressure
// and enthalpy shifted by constant reference values first; all stencil and
// flux arithmetic and the RHS accumulation run in FP32; the state, the RK
// register and the update stay FP64). The shifts are exact corrections:
// a constant pressure drops out of every difference, and a constant
// enthalpy shift H' = H - H_ref changes the energy flux by H_ref times the
// mass flux, added back in FP64 at the end.
#include <stdlib.h>
#include <string.h>

#include <type_traits>

#include "sx_internal.h"

namespace sx {

// 1/x: hardware reciprocal refined by two Newton steps (about 1 ulp).
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// fused multiply-add in the arithmetic type (FP32 stays FP32)
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int S, typename R>
__device__ __forceinline__ R d1(const R (&f)[2 * S + 1])
{
    R s = R(0);
#pragma unroll
    for (int l = 1; l <= S; ++l) s += R(Coef<S>::a[l]) * (f[S + l] - f[S - l]);
    return s;
}

// First derivative of order 2V centred on entry H of a window of 2H+1
// values (V <= H).
template <int V, int H, typename R>
__device__ __forceinline__ R d1c(const R (&f)[2 * H + 1])
{
    R s = R(0);
#pragma unroll
    for (int l = 1; l <= V; ++l) s += R(Coef<V>::a[l]) * (f[H + l] - f[H - l]);
    return s;
}

// Half-width of the stencils of a kernel: the larger of the convective and
// viscous half-orders.
template <int SC, int SV>
struct Halo {
    static constexpr int S = SC > SV ? SC : SV;
};

// A constant handed to the arithmetic as a scalar-register operand at its
// point of use (FP64 constants other than a few inline values need a
// register; held in vector registers across a loop they cost 2 registers
// each and a copy per use).
__device__ __forceinline__ double kconst(double c)
{
    asm volatile("" : "+s"(c));
    return c;
}

// Viscosity law T^s: FP64 through exp(s log T); FP32 through the hardware
// base-2 logarithm and exponential.
template <typename R>
__device__ __forceinline__ R visc_pow(R T, const KGas& gas);
// FP64 T^s = exp(s ln T) for T > 0 from two short series (relative error a
// few ulp): ln m = 2 atanh z, z = (m-1)/(m+1), m in [1/sqrt2, sqrt2) (odd
// series in z, |z| < 0.172, 12 terms), and exp r for |r| <= ln2/2 (Taylor,
// 14 terms), with the exponents split off by frexp / ldexp and ln 2 carried
// in two parts.
__device__ __forceinline__ double visc_pow_f64(double T, double s)
{
    int e;
    double m = frexp(T, &e);                       // T = m 2^e, m in [0.5, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double z = (m - 1.0) * rcp(m + 1.0);
    const double z2 = z * z;
    // atanh(z)/z = sum z^(2k) / (2k+1)
    double q = kconst(1.0 / 23.0);
    q = __builtin_fma(q, z2, kconst(1.0 / 21.0));
    q = __builtin_fma(q, z2, kconst(1.0 / 19.0));
    q = __builtin_fma(q, z2, kconst(1.0 / 17.0));
    q = __builtin_fma(q, z2, kconst(1.0 / 15.0));
    q = __builtin_fma(q, z2, kconst(1.0 / 13.0));
    q = __builtin_fma(q, z2, kconst(1.0 / 11.0));
    q = __builtin_fma(q, z2, kconst(1.0 / 9.0));
    q = __builtin_fma(q, z2, kconst(1.0 / 7.0));
    q = __builtin_fma(q, z2, kconst(1.0 / 5.0));
    q = __builtin_fma(q, z2, kconst(1.0 / 3.0));
    const double lnm = 2.0 * __builtin_fma(z * z2, q, z);
    constexpr double LN2_HI = 6.93147180369123816490e-01, LN2_LO = 1.90821492927058770002e-10;
    // y = s ln T = s (e ln2 + ln m), ln2 in two parts
    const double de = double(e);
    const double y = s * __builtin_fma(de, LN2_HI, __builtin_fma(de, LN2_LO, lnm));
    // exp(y) = 2^n exp(r), r = y - n ln2
    const double n = rint(y * 1.44269504088896340736);
    const double r = __builtin_fma(-n, LN2_LO, __builtin_fma(-n, LN2_HI, y));
    double p = kconst(1.0 / 87178291200.0);                // 1/14!
    p = __builtin_fma(p, r, kconst(1.0 / 6227020800.0));
    p = __builtin_fma(p, r, kconst(1.0 / 479001600.0));
    p = __builtin_fma(p, r, kconst(1.0 / 39916800.0));
    p = __builtin_fma(p, r, kconst(1.0 / 3628800.0));
    p = __builtin_fma(p, r, kconst(1.0 / 362880.0));
    p = __builtin_fma(p, r, kconst(1.0 / 40320.0));
    p = __builtin_fma(p, r, kconst(1.0 / 5040.0));
    p = __builtin_fma(p, r, kconst(1.0 / 720.0));
    p = __builtin_fma(p, r, kconst(1.0 / 120.0));
    p = __builtin_fma(p, r, kconst(1.0 / 24.0));
    p = __builtin_fma(p, r, kconst(1.0 / 6.0));
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return ldexp(p, int(n));
}
template <>
__device__ __forceinline__ double visc_pow<double>(double T, const KGas& gas) { return visc_pow_f64(T, gas.s); }
template <>
__device__ __forceinline__ float visc_pow<float>(float T, const KGas& gas)
{
    return __builtin_amdgcn_exp2f(gas.sf * __builtin_amdgcn_logf(T));
}

template <typename R>
__device__ __forceinline__ R rcpr(R x);
template <>
__device__ __forceinline__ double rcpr<double>(double x) { return rcp(x); }
template <>
__device__ __forceinline__ float rcpr<float>(float x) { return 1.0f / x; }

// Node values along one stencil direction.
template <typename R>
struct Node {
    R r, u, v, w, T, p, H;
};

// LDS record layouts. FP64: plane and ring records of 6 doubles read as
// three 128-bit loads, ordered (u, v | w, T | rho, H) so the viscous terms,
// which need u, v, w, T only, read the first two; the pressure is derived on
// read, p = rho T / (gamma M^2), the same way on every FP64 path, so that
// single-block and batched launches agree bitwise. (The 48-byte stride is
// bank conflict free for 128-bit accesses.) FP32: 7-float records (rho, u,
// v, w, T, p', H') read as 32-bit loads (stride 7 is coprime with the 64
// banks).
template <typename R>
struct Layout;
template <>
struct Layout<double> {
    static constexpr int PREC = 6;   // plane record
    static constexpr int ZREC = 6;   // ring record
    static constexpr int OU = 0, OV = 1;   // offsets of u and v in a plane record
};
template <>
struct Layout<float> {
    static constexpr int PREC = 7;
    static constexpr int ZREC = 7;
    static constexpr int OU = 1, OV = 2;
};

// 16-byte vector of two doubles with its natural alignment, so that LDS
// accesses at a run-time record index stay single 128-bit operations (split
// into two 64-bit halves, records 48 bytes apart would fall on the same
// banks two lanes at a time).
typedef double dbl2 __attribute__((ext_vector_type(2)));

template <typename R>
__device__ __forceinline__ void plane_write(R* so, int q, double rho, double u, double v,
                                            double w, double T, double p, double H)
{
    if constexpr (std::is_same<R, double>::value) {
        dbl2* rec = reinterpret_cast<dbl2*>(so + 6 * q);
        rec[0] = dbl2{u, v};
        rec[1] = dbl2{w, T};
        rec[2] = dbl2{rho, H};
        (void)p;
    } else {
        R* rec = so + 7 * q;
        rec[0] = R(rho); rec[1] = R(u); rec[2] = R(v); rec[3] = R(w);
        rec[4] = R(T); rec[5] = R(p); rec[6] = R(H);
    }
}

template <typename R>
__device__ __forceinline__ Node<R> plane_read(const R* so, int q, R igM2)
{
    if constexpr (std::is_same<R, double>::value) {
        const dbl2* rec = reinterpret_cast<const dbl2*>(so + 6 * q);
        const dbl2 a = rec[0], b = rec[1], e = rec[2];
        return Node<double>{e.x, a.x, a.y, b.x, b.y, e.x * b.y * igM2, e.y};
    } else {
        const R* rec = so + 7 * q;
        return Node<R>{rec[0], rec[1], rec[2], rec[3], rec[4], rec[5], rec[6]};
    }
}

// u and v of plane record q (FP64: one 128-bit load)
template <typename R>
__device__ __forceinline__ void plane_uv(const R* so, int q, R& u, R& v)
{
    if constexpr (std::is_same<R, double>::value) {
        const dbl2 a = reinterpret_cast<const dbl2*>(so + 6 * q)[0];
        u = a.x;
        v = a.y;
    } else {
        u = so[7 * q + 1];
        v = so[7 * q + 2];
    }
}

template <typename R>
__device__ __forceinline__ void ring_write(R* z, double rho, double u, double v, double w,
                                           double T, double p, double H)
{
    if constexpr (std::is_same<R, double>::value) {
        dbl2* rec = reinterpret_cast<dbl2*>(z);
        rec[0] = dbl2{u, v};
        rec[1] = dbl2{w, T};
        rec[2] = dbl2{rho, H};
        (void)p;
    } else {
        z[0] = R(rho); z[1] = R(u); z[2] = R(v); z[3] = R(w); z[4] = R(T); z[5] = R(p); z[6] = R(H);
    }
}

template <typename R>
__device__ __forceinline__ Node<R> ring_read(const R* z, R igM2)
{
    if constexpr (std::is_same<R, double>::value) {
        const dbl2* rec = reinterpret_cast<const dbl2*>(z);
        const dbl2 a = rec[0], b = rec[1], e = rec[2];
        return Node<double>{e.x, a.x, a.y, b.x, b.y, e.x * b.y * igM2, e.y};
    } else {
        return Node<R>{z[0], z[1], z[2], z[3], z[4], z[5], z[6]};
    }
}

// One direction of the output node over the stencil pairs l = 1..S (FP64
// reads every node first; FP32 streams the pairs so only the centre and the
// two nodes at distance l are live). Adds the convective derivative in the
// pair-difference form of the split flux,
//   F_{i+1/2} - F_{i-1/2} = sum_l 2 a_l [P_l(i) - P_l(i-l)],
//   P_l(n) = 1/8 (rho_n + rho_{n+l})(ud_n + ud_{n+l})(phi_n + phi_{n+l}),
// phi in {1, u, v, w, H}, pressure 1/2 (p_n + p_{n+l}) in the D-momentum
// (FP64: differences of rho T, scaled once by 1/(gamma M^2)), to acc and
// returns first derivatives gd = (u, v, w, T)_n and the pure second
// derivatives dd = (u, v, w, T)_nn, the latter in FP64 as
// sum_l b_l (f_{n+l} + f_{n-l}) - 2 (sum_l b_l) f_n (sc: metric 1/h or
// eta_y; sc2 = sc^2; scy = eta_yy along y, 0 otherwise; kgas: the gas,
// needed by the convective FP64 and KEEP-n forms).
// KEEP-n two-point flux (FP64). The entropy-conserving, kinetic-energy
// preserving pair flux of nodes A, B along direction D:
//   F_rho = rho_ln (ud_A + ud_B)/2,  F_mom = F_rho (u_A + u_B)/2 + (p_A + p_B)/2 e_D,
//   F_E   = F_rho (1/((gamma-1) b_ln) + u_A.u_B/2) + (p_A ud_B + p_B ud_A)/2,
// b = rho/p, x_ln the logarithmic mean. With b = gamma M^2 / T,
// 1/((gamma-1) b_ln) = T_A T_B / ((gamma-1) gamma M^2) * 1/T_ln, and
// 1/x_ln = 2/(x_A+x_B) sum_{m=0..n} xi^(2m)/(2m+1), xi = (x_B-x_A)/(x_B+x_A),
// cut after n terms (n < 0: the exact mean; its series up to m = 16 where
// |xi| < 0.1, the logarithms elsewhere).
__device__ __forceinline__ double keep_inv_log_mean(double a, double b, int n)
{
    constexpr double inv_odd[17] = {1.0,        1.0 / 3.0,  1.0 / 5.0,  1.0 / 7.0,  1.0 / 9.0,  1.0 / 11.0,
                                    1.0 / 13.0, 1.0 / 15.0, 1.0 / 17.0, 1.0 / 19.0, 1.0 / 21.0, 1.0 / 23.0,
                                    1.0 / 25.0, 1.0 / 27.0, 1.0 / 29.0, 1.0 / 31.0, 1.0 / 33.0};
    const double rs = rcp(a + b);
    const double xi = (b - a) * rs;
    if (n < 0) {
        if (fabs(xi) >= 0.1) return (log(b) - log(a)) / (b - a);
        n = 16;
    }
    const double x2 = xi * xi;
    double S = inv_odd[n];
    for (int m = n - 1; m >= 0; --m) S = __builtin_fma(S, x2, inv_odd[m]);
    return 2.0 * rs * S;
}

template <int D>
__device__ __forceinline__ void keep_pair(const Node<double>& A, const Node<double>& B, const KGas& gas,
                                          double (&F)[NV])
{
    const double udA = D == 0 ? A.u : (D == 1 ? A.v : A.w);
    const double udB = D == 0 ? B.u : (D == 1 ? B.v : B.w);
    const double frho = 0.5 * (udA + udB) * rcp(keep_inv_log_mean(A.r, B.r, gas.keep_n));
    const double uu = A.u * B.u + A.v * B.v + A.w * B.w;
    const double K = gas.cvg * (A.T * B.T) * keep_inv_log_mean(A.T, B.T, gas.keep_n) + 0.5 * uu;
    F[0] = frho;
    F[1] = frho * (0.5 * (A.u + B.u));
    F[2] = frho * (0.5 * (A.v + B.v));
    F[3] = frho * (0.5 * (A.w + B.w));
    F[1 + D] += 0.5 * (A.p + B.p);
    F[4] = frho * K + 0.5 * (A.p * udB + B.p * udA);
}

template <int SC, int SV, int D, bool CONV, bool VISC, bool KEEP = false, bool D1 = false, typename R,
          typename Get>
__device__ __forceinline__ void stencil_dir(Get get, R sc, R sc2, R scy, R (&acc)[NV], R (&gd)[4],
                                            R (&dd)[4], const KGas* kgas)
{
    // D1 (convective only): gd[0..2] return the differences u, v, w of the
    // two nodes at distance 1, for the second-order sensor
    // convective pairs up to SC, viscous differences up to SV
    constexpr int SL = CONV && VISC ? Halo<SC, SV>::S : (CONV ? SC : SV);
    const Node<R> C = get(0);
    R f0 = 0, f1 = 0, f2 = 0, f3 = 0, f4 = 0, fp = 0;
    R s1[4] = {0, 0, 0, 0}, s2[4] = {0, 0, 0, 0};
    // FP64: every stencil node is read before the arithmetic starts, so the
    // LDS reads of a direction are in flight together (the FP32 form streams
    // the pairs, for its register budget)
    constexpr bool PRE = std::is_same<R, double>::value;
    Node<R> Ms[SL], Ps[SL];
    if constexpr (PRE) {
#pragma unroll
        for (int l = 1; l <= SL; ++l) {
            Ms[l - 1] = get(-l);
            Ps[l - 1] = get(l);
        }
    }
#pragma unroll
    for (int l = 1; l <= SL; ++l) {
        const Node<R> M = PRE ? Ms[l - 1] : get(-l), P = PRE ? Ps[l - 1] : get(l);
        if constexpr (D1 && !VISC) {
            if (l == 1) {
                gd[0] = P.u - M.u;
                gd[1] = P.v - M.v;
                gd[2] = P.w - M.w;
            }
        }
        if constexpr (KEEP) {
            if (CONV && l <= SC) {
                // F(C, P) - F(M, C) with the KEEP-n pair flux
                double Fp[NV], Fm[NV];
                keep_pair<D>(C, P, *kgas, Fp);
                keep_pair<D>(M, C, *kgas, Fm);
                const double c2 = 2.0 * Coef<SC>::a[l];
                f0 += c2 * (Fp[0] - Fm[0]);
                f1 += c2 * (Fp[1] - Fm[1]);
                f2 += c2 * (Fp[2] - Fm[2]);
                f3 += c2 * (Fp[3] - Fm[3]);
                f4 += c2 * (Fp[4] - Fm[4]);
            }
        } else if (CONV && l <= SC) {
            const R cl = R(0.25 * Coef<SC>::a[l]);
            const R udC = D == 0 ? C.u : (D == 1 ? C.v : C.w);
            const R udP = D == 0 ? P.u : (D == 1 ? P.v : P.w);
            const R udM = D == 0 ? M.u : (D == 1 ? M.v : M.w);
            const R mp = cl * (C.r + P.r) * (udC + udP);    // pair (C, P), +
            const R mm = cl * (M.r + C.r) * (udM + udC);    // pair (M, C), -
            // mp (C.phi + P.phi) - mm (M.phi + C.phi): the C.phi parts of all
            // pairs sum to C.phi (f0 / 2), added after the loop
            f0 += mp - mm;
            f1 = fmar(mp, P.u, fmar(-mm, M.u, f1));
            f2 = fmar(mp, P.v, fmar(-mm, M.v, f2));
            f3 = fmar(mp, P.w, fmar(-mm, M.w, f3));
            f4 = fmar(mp, P.H, fmar(-mm, M.H, f4));
            if constexpr (std::is_same<R, double>::value) {
                // p = rho T / (gamma M^2): the pair differences of rho T, scaled once below
                fp = fmar(R(4) * cl, fmar(P.r, P.T, -(M.r * M.T)), fp);
            } else {
                fp += (R(4) * cl) * (P.p - M.p);
            }
        }
        if (VISC && l <= SV) {
            const R al = R(Coef<SV>::a[l]), bl = R(Coef<SV>::b[l]);
            s1[0] += al * (P.u - M.u);
            s1[1] += al * (P.v - M.v);
            s1[2] += al * (P.w - M.w);
            s1[3] += al * (P.T - M.T);
            if constexpr (std::is_same<R, double>::value) {
                s2[0] += bl * (P.u + M.u);
                s2[1] += bl * (P.v + M.v);
                s2[2] += bl * (P.w + M.w);
                s2[3] += bl * (P.T + M.T);
            } else {   // FP32 keeps the per-pair second differences (smaller rounding)
                s2[0] += bl * ((P.u - R(2) * C.u) + M.u);
                s2[1] += bl * ((P.v - R(2) * C.v) + M.v);
                s2[2] += bl * ((P.w - R(2) * C.w) + M.w);
                s2[3] += bl * ((P.T - R(2) * C.T) + M.T);
            }
        }
    }
    if (CONV) {
        if constexpr (!KEEP) {
            f1 = fmar(C.u, f0, f1);
            f2 = fmar(C.v, f0, f2);
            f3 = fmar(C.w, f0, f3);
            f4 = fmar(C.H, f0, f4);
            f0 *= R(2);
            if constexpr (std::is_same<R, double>::value) fp *= R(kgas->igM2);
            if (D == 0) f1 += fp;
            if (D == 1) f2 += fp;
            if (D == 2) f3 += fp;
        }
        acc[0] -= sc * f0;
        acc[1] -= sc * f1;
        acc[2] -= sc * f2;
        acc[3] -= sc * f3;
        acc[4] -= sc * f4;
    }
    if (VISC) {
        if constexpr (std::is_same<R, double>::value) {
            constexpr double B2 = 2.0 * Coef<SV>::bsum;
            s2[0] = fmar(R(-B2), C.u, s2[0]);
            s2[1] = fmar(R(-B2), C.v, s2[1]);
            s2[2] = fmar(R(-B2), C.w, s2[2]);
            s2[3] = fmar(R(-B2), C.T, s2[3]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            gd[q] = sc * s1[q];
            // the metric term eta_yy D_eta f exists along y only
            dd[q] = D == 1 ? sc2 * s2[q] + scy * s1[q] : sc2 * s2[q];
        }
    }
}

// Linear viscous pieces of one direction d, consumed at once:
// mu (u_i)_dd (+ mu/3 (u_d)_dd into momentum d), k T_dd, and their work
// u_i (...) into the energy.
template <int D, typename R>
__device__ __forceinline__ void visc_linear(const R (&dd)[4], R mu, R kc, R uc, R vc, R wc,
                                            R (&acc)[NV])
{
    const R o3 = R(1.0 / 3.0);
    R a0 = mu * dd[0], a1 = mu * dd[1], a2 = mu * dd[2];
    if (D == 0) a0 += (mu * o3) * dd[0];
    if (D == 1) a1 += (mu * o3) * dd[1];
    if (D == 2) a2 += (mu * o3) * dd[2];
    acc[1] += a0;
    acc[2] += a1;
    acc[3] += a2;
    acc[4] += uc * a0 + vc * a1 + wc * a2 + kc * dd[3];
}

// Conserved values of up to NPT halo points of one plane, fetched into
// registers one iteration ahead of their use.
template <int NPT>
struct PlaneFetch {
    double q[NPT][5];
};

// LDS working set of one workgroup (see the file header).
template <int S, int TX, int TY, typename R>
struct Smem {
    static constexpr int NT = TX * TY;
    static constexpr int HX = TX + 2 * S, HY = TY + 2 * S, HP = HX * HY;
    static constexpr int Q = 2 * S + 1;
    R sa[3][HP];                                                    // arrival plane: u, v, w
    __attribute__((aligned(16))) R so[Layout<R>::PREC * HP];        // output plane records
    R gyl[2][TY][HX];                                               // D_y u, D_y v of plane k
    __attribute__((aligned(16))) R zring[Q * NT * Layout<R>::ZREC]; // column records
    double fred[NT];                                                // bulk-forcing partial sums
};

// March one column tile (i0, j0) of one block over planes [k0, k1).
// PIMG: every direction is periodic and the new state is also written into
// its periodic ghost images, so the next substep needs no ghost fill.
// Load / store at a byte offset from a base pointer.
template <typename T>
__device__ __forceinline__ T ldo(const T* base, unsigned bo)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + bo);
}
template <typename T>
__device__ __forceinline__ void sto(T* base, unsigned bo, T v)
{
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + bo) = v;
}

// Bulk forcing: the workgroup's sum of V R_rhou over its output nodes,
// written to its slot of g.fpart (fixed tree order). Every thread of the
// workgroup calls this; the first n threads contribute v.
template <int NTH>
__device__ __forceinline__ void force_partial(double* red, int n, double v, const KGrid& g)
{
    __syncthreads();
    if ((int)threadIdx.x < n) red[threadIdx.x] = v;
    __syncthreads();
    for (int s = n / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        g.fpart[blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z)] = red[0];
    (void)NTH;
}

template <int SC, int SV, int TX, int TY, typename R, bool UPD, bool PIMG, int VAR = 0>
__device__ __forceinline__ void march(Smem<Halo<SC, SV>::S, TX, TY, R>& sm, const double* __restrict__ W,
                                      double* __restrict__ out, double* __restrict__ Rp,
                                      const KGrid& g, const KGas& gas, const StepCoef& sc,
                                      unsigned mask_in, int i0, int j0, int k0, int k1)
{
    const unsigned mask = UPD ? (unsigned)SX_ALL : mask_in;   // an update always takes every term
    constexpr int S = Halo<SC, SV>::S;
    constexpr bool THERMO = VAR == 2;   // thermally perfect gas (the KEEP-n flux runs split only)
    static_assert(VAR != 1, "KEEP-n runs in the split march");
    using L = Layout<R>;
    constexpr int NT = TX * TY;
    constexpr int HX = TX + 2 * S, HY = TY + 2 * S, HP = HX * HY;
    constexpr int NPT = (HP + NT - 1) / NT;
    constexpr int Q = 2 * S + 1;
    auto& sa = sm.sa;
    R* const so = sm.so;
    auto& gyl = sm.gyl;
    R* const zring = sm.zring;
    (void)HY;

    constexpr bool f32 = std::is_same<R, float>::value;
    const double pref = f32 ? gas.pref : 0.0, href = f32 ? gas.href : 0.0;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool active = i < g.nx && j < g.ny;
    const int c = (ty + S) * HX + (tx + S);
    const R ey = active ? R(g.eta_y[j]) : R(0);
    const R eyy = active ? R(g.eta_yy[j]) : R(0);
    const R dxi = R(g.dxi), dzi = R(g.dzi);
    const R igM2 = R(gas.igM2);
    static_assert(64 % TX == 0, "every row of the tile lies in one wave");
    const R eyr = j < g.ny ? R(g.eta_y[j]) : R(0);            // eta_y of this row
    // bulk forcing: cell volume of this column's nodes, running sum of V R_rhou
    const double fvol = active && g.fpart ? g.dx * g.y_eta[j] * g.dz : 0.0;
    double fsum = 0.0;

    R m0[Q], m1[Q], m2[Q];   // D_x w, D_y w, D_x u + D_y v of this column
#pragma unroll
    for (int t = 0; t < Q; ++t) m0[t] = m1[t] = m2[t] = R(0);

    // Global accesses: per-variable base pointer plus a 32-bit byte offset
    // (in-plane part per thread, plane part uniform); see march_split.
    // inactive threads (ragged tiles) load the nearest interior column; only
    // active threads store
    const int ic = min(i, g.nx - 1), jc = min(j, g.ny - 1);
    const unsigned colbo = (unsigned)((g.base + (long long)jc * g.sy + ic) * 8);
    const unsigned jibo = (unsigned)(((long long)jc * g.nx + ic) * 8);
    auto kbo = [&](int k) { return (unsigned)((long long)k * g.sz * 8); };
    auto kbr = [&](int k) { return (unsigned)((long long)k * g.ny * g.nx * 8); };
    // Halo points outside the ghosted block (ragged tiles, the unused tail
    // of the last round) load the nearest ghosted node instead: valid data,
    // no branch; no active output reads them.
    unsigned hbo[NPT];
#pragma unroll
    for (int a = 0; a < NPT; ++a) {
        const int q = tid + a * NT;
        const int hx = q % HX, hy = q / HX;
        const int gi = min(max(i0 - S + hx, -g.ng), g.nx + g.ng - 1);
        const int gj = min(max(j0 - S + hy, -g.ng), g.ny + g.ng - 1);
        hbo[a] = (unsigned)((g.base + (long long)gj * g.sy + gi) * 8);
    }
    auto fetch = [&](PlaneFetch<NPT>& f, int k, int nvar) {
        const unsigned kb = kbo(k);
#pragma unroll
        for (int a = 0; a < NPT; ++a) {
            if (a + 1 < NPT || tid + a * NT < HP) {   // the last round covers the tail of the plane
                const unsigned bo = hbo[a] + kb;
#pragma unroll
                for (int v = 0; v < 5; ++v)
                    if (v < nvar) f.q[a][v] = ldo(W + v * g.sv, bo);
            }
        }
    };
    auto fetch_col = [&](double (&cq)[5], int k) {
        const unsigned bn = colbo + kbo(k);
#pragma unroll
        for (int v = 0; v < 5; ++v) cq[v] = ldo(W + v * g.sv, bn);
    };
    double wc[5] = {}, rp[5] = {};   // centre state and RK register of the next output node
    auto fetch_centre = [&](int k) {
        const unsigned bn = colbo + kbo(k), bm = jibo + kbr(k);
        if (UPD) {
#pragma unroll
            for (int v = 0; v < 5; ++v) wc[v] = ldo(W + v * g.sv, bn);
            if (sc.read_prev) {
#pragma unroll
                for (int v = 0; v < 5; ++v) rp[v] = ldo(Rp + v * g.nint, bm);
            }
        }
    };
    auto stage_arrival = [&](const PlaneFetch<NPT>& f) {
#pragma unroll
        for (int a = 0; a < NPT; ++a) {
            const int q = tid + a * NT;
            if (q < HP) {
                const double ri = rcp(f.q[a][0]);
                sa[0][q] = R(f.q[a][1] * ri);
                sa[1][q] = R(f.q[a][2] * ri);
                sa[2][q] = R(f.q[a][3] * ri);
            }
        }
    };
    // FP64 primitives of conserved values (pressure / enthalpy shifted by
    // the reference values in the FP32 form)
    auto prims = [&](const double* w5, double& rho, double& u, double& v, double& w, double& T,
                     double& p, double& H) {
        rho = w5[0];
        const double ri = rcp(rho);
        u = w5[1] * ri;
        v = w5[2] * ri;
        w = w5[3] * ri;
        double pr;
        if constexpr (THERMO) {   // thermally perfect: T from the internal energy
            T = tp_T_of_e(gas, w5[4] * ri - 0.5 * (u * u + v * v + w * w));
            pr = rho * T * gas.igM2;
        } else {
            pr = gas.gm1 * (w5[4] - 0.5 * rho * (u * u + v * v + w * w));
            T = gas.gM2 * pr * ri;
        }
        H = (w5[4] + pr) * ri - href;
        p = pr - pref;
    };
    auto stage_output = [&](const PlaneFetch<NPT>& f) {
#pragma unroll
        for (int a = 0; a < NPT; ++a) {
            const int q = tid + a * NT;
            if (q < HP) {
                double rho, u, v, w, T, p, H;
                prims(f.q[a], rho, u, v, w, T, p, H);
                plane_write<R>(so, q, rho, u, v, w, T, p, H);
            }
        }
    };
    auto stage_column = [&](int slot, const double (&cq)[5]) {
        double rho, u, v, w, T, p, H;
        prims(cq, rho, u, v, w, T, p, H);
        ring_write<R>(zring + L::ZREC * (slot * NT + tid), rho, u, v, w, T, p, H);
    };
    auto znode = [&](int slot) { return ring_read<R>(zring + L::ZREC * (slot * NT + tid), igM2); };
    // newest mixed-queue slot from the staged arrival plane
    auto arrive = [&]() {
        if (!active) return;
        constexpr int QV = 2 * SV + 1;
        R xw[QV], yw[QV], xu[QV], yv[QV];
#pragma unroll
        for (int t = 0; t < QV; ++t) {
            xu[t] = sa[0][c + t - SV];
            xw[t] = sa[2][c + t - SV];
            yv[t] = sa[1][c + (t - SV) * HX];
            yw[t] = sa[2][c + (t - SV) * HX];
        }
        m0[Q - 1] = dxi * d1<SV>(xw);
        m1[Q - 1] = ey * d1<SV>(yw);
        m2[Q - 1] = dxi * d1<SV>(xu) + ey * d1<SV>(yv);
    };
    auto shift = [&]() {
#pragma unroll
        for (int t = 0; t < Q - 1; ++t) {
            m0[t] = m0[t + 1];
            m1[t] = m1[t + 1];
            m2[t] = m2[t + 1];
        }
    };

    PlaneFetch<NPT> fa, fo;
    double cq[5];

    // prologue: planes k0-S .. k0+S-1 -> ring slots 0 .. 2S-1, mixed queue
    for (int t = 0; t < 2 * S; ++t) {
        fetch(fa, k0 - S + t, 4);
        fetch_col(cq, k0 - S + t);
        stage_arrival(fa);
        stage_column(t, cq);
        __syncthreads();
        arrive();
        shift();
        __syncthreads();
    }

    fetch(fa, k0 + S, 4);
    fetch(fo, k0, 5);
    fetch_col(cq, k0 + S);
    fetch_centre(k0);

    // results of the previous output plane, stored one iteration late
    double pend[NV] = {0, 0, 0, 0, 0};
    double pend_w[NV] = {0, 0, 0, 0, 0};
    int pend_k = -1;   // plane of the pending stores, -1: none
    auto flush = [&]() {
        if (pend_k < 0) return;
        if (UPD) {
            const unsigned bn = colbo + kbo(pend_k);
#pragma unroll
            for (int v = 0; v < NV; ++v) sto(out + v * g.sv, bn, pend_w[v]);
            if constexpr (PIMG) {
                // periodic images of node (i, j, pend_k) inside the ghost layers
                const int kk = pend_k;
                const int ox = i < g.ng ? g.nx : (i >= g.nx - g.ng ? -g.nx : 0);
                const int oy = j < g.ng ? g.ny : (j >= g.ny - g.ng ? -g.ny : 0);
                const int oz = kk < g.ng ? g.nz : (kk >= g.nz - g.ng ? -g.nz : 0);
                for (int c3 = 1; c3 < 8; ++c3) {
                    const int dx = (c3 & 1) ? ox : 0, dy = (c3 & 2) ? oy : 0, dz = (c3 & 4) ? oz : 0;
                    if (((c3 & 1) && !ox) || ((c3 & 2) && !oy) || ((c3 & 4) && !oz)) continue;
                    const unsigned be = bn + (unsigned)((dx + (long long)dy * g.sy + (long long)dz * g.sz) * 8);
#pragma unroll
                    for (int v = 0; v < NV; ++v) sto(out + v * g.sv, be, pend_w[v]);
                }
            }
            if (sc.write_prev) {
                const unsigned bm = jibo + kbr(pend_k);
#pragma unroll
                for (int v = 0; v < NV; ++v) sto(Rp + v * g.nint, bm, pend[v]);
            }
        } else {
            const unsigned bm = jibo + kbr(pend_k);
#pragma unroll
            for (int v = 0; v < NV; ++v) sto(out + v * g.nint, bm, pend[v]);
        }
        pend_k = -1;
    };

    int slot_k = S;   // ring slot of the output plane k (plane k0-S sits in slot 0)
    for (int k = k0; k < k1; ++k) {
        const int slot_new = slot_k + S >= Q ? slot_k + S - Q : slot_k + S;   // plane k+S
        stage_arrival(fa);
        stage_output(fo);
        stage_column(slot_new, cq);
        double wcur[5], rcur[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            wcur[v] = wc[v];
            rcur[v] = rp[v];
        }
        flush();                       // stores of plane k-1
        __syncthreads();
        arrive();
        if (k + 1 < k1) {              // loads of iteration k+1
            fetch(fa, k + 1 + S, 4);
            fetch(fo, k + 1, 5);
            fetch_col(cq, k + 1 + S);
            fetch_centre(k + 1);
        }
        sched_fence();
        // y-derivatives of u, v at plane k over the x-extended columns of
        // this thread's row. Only threads of the same row read them and a row
        // lies in one wave, whose LDS accesses execute in order, so a
        // wavefront-scope fence stands in for a workgroup barrier.
        auto gy_at = [&](int hx) {
            R su = 0, sv = 0;
#pragma unroll
            for (int l = 1; l <= SV; ++l) {
                R uu, vu, ud, vd;
                plane_uv<R>(so, (ty + S + l) * HX + hx, uu, vu);
                plane_uv<R>(so, (ty + S - l) * HX + hx, ud, vd);
                su += R(Coef<SV>::a[l]) * (uu - ud);
                sv += R(Coef<SV>::a[l]) * (vu - vd);
            }
            gyl[0][ty][hx] = eyr * su;
            gyl[1][ty][hx] = eyr * sv;
        };
        if (j < g.ny) {
            gy_at(tx + S);
            if (tx < 2 * S) gy_at(tx < S ? tx : TX + tx);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        if (active) {
            R acc[NV] = {0, 0, 0, 0, 0};
            const bool visc = mask & SX_VISC;
            const Node<R> Cz = znode(slot_k);
            const R uc = Cz.u, vc = Cz.v, wc_ = Cz.w, Tc = Cz.T;
            R mu = 0, kcd = 0, smt = 0, skt = 0;
            if (visc) {
                mu = visc_pow<R>(Tc, gas) * R(gas.ire);
                smt = R(gas.s) * rcpr<R>(Tc);
                if constexpr (THERMO) {   // k = mu c_p(T) / Pr, grad k = k (s/T + c_p'/c_p) grad T
                    const double cpr = tp_cpR(gas, double(Tc));
                    kcd = mu * R(gas.igM2 * cpr * gas.ipr);
                    skt = smt + R(tp_dcpR(gas, double(Tc)) / cpr);
                } else {
                    kcd = mu * R(gas.cp * gas.ipr);
                    skt = smt;
                }
            }
            R gx[4] = {0, 0, 0, 0}, gy[4] = {0, 0, 0, 0}, gz[4] = {0, 0, 0, 0}, dd[4];
            auto getx = [&](int t) { return plane_read<R>(so, c + t, igM2); };
            auto gety = [&](int t) { return plane_read<R>(so, c + t * HX, igM2); };
            auto getz = [&](int t) {
                int sl = slot_k + t;
                sl = sl < 0 ? sl + Q : (sl >= Q ? sl - Q : sl);
                return znode(sl);
            };
            if (mask & SX_CONV_X) {
                if (visc) stencil_dir<SC, SV, 0, true, true>(getx, dxi, dxi * dxi, R(0), acc, gx, dd, &gas);
                else stencil_dir<SC, SV, 0, true, false>(getx, dxi, dxi * dxi, R(0), acc, gx, dd, &gas);
            } else if (visc) {
                stencil_dir<SC, SV, 0, false, true>(getx, dxi, dxi * dxi, R(0), acc, gx, dd, nullptr);
            }
            if (visc) visc_linear<0>(dd, mu, kcd, uc, vc, wc_, acc);
            if (mask & SX_CONV_Y) {
                if (visc) stencil_dir<SC, SV, 1, true, true>(gety, ey, ey * ey, eyy, acc, gy, dd, &gas);
                else stencil_dir<SC, SV, 1, true, false>(gety, ey, ey * ey, eyy, acc, gy, dd, &gas);
            } else if (visc) {
                stencil_dir<SC, SV, 1, false, true>(gety, ey, ey * ey, eyy, acc, gy, dd, nullptr);
            }
            if (visc) visc_linear<1>(dd, mu, kcd, uc, vc, wc_, acc);
            if (mask & SX_CONV_Z) {
                if (visc) stencil_dir<SC, SV, 2, true, true>(getz, dzi, dzi * dzi, R(0), acc, gz, dd, &gas);
                else stencil_dir<SC, SV, 2, true, false>(getz, dzi, dzi * dzi, R(0), acc, gz, dd, &gas);
            } else if (visc) {
                stencil_dir<SC, SV, 2, false, true>(getz, dzi, dzi * dzi, R(0), acc, gz, dd, nullptr);
            }
            // enthalpy shift correction of the convective energy flux (FP64)
            const double accE_shift = href * double(acc[0]);
            if (visc) {
                visc_linear<2>(dd, mu, kcd, uc, vc, wc_, acc);
                // mixed parts of mu/3 d_i(div u): d_x d_y, d_x d_z, d_y d_z
                R gyu[Q], gyv[Q];
#pragma unroll
                for (int t = 0; t < Q; ++t) {
                    gyu[t] = gyl[0][ty][tx + t];
                    gyv[t] = gyl[1][ty][tx + t];
                }
                const R m3 = mu * R(1.0 / 3.0);
                const R mx = m3 * (dxi * d1c<SV, S>(gyv) + dzi * d1c<SV, S>(m0));   // d_x d_y v + d_z d_x w
                const R my = m3 * (dxi * d1c<SV, S>(gyu) + dzi * d1c<SV, S>(m1));   // d_x d_y u + d_z d_y w
                const R mz = m3 * (dzi * d1c<SV, S>(m2));                      // d_z (d_x u + d_y v)
                acc[1] += mx;
                acc[2] += my;
                acc[3] += mz;
                acc[4] += uc * mx + vc * my + wc_ * mz;
                // nonlinear parts: grad mu (= s mu/T grad T) terms and dissipation
                const R g00 = gx[0], g10 = gx[1], g20 = gx[2], Tx = gx[3];
                const R g01 = gy[0], g11 = gy[1], g21 = gy[2], Ty = gy[3];
                const R g02 = gz[0], g12 = gz[1], g22 = gz[2], Tz = gz[3];
                const R th = g00 + g11 + g22;
                const R sm = smt * mu;
                const R dmu0 = sm * Tx, dmu1 = sm * Ty, dmu2 = sm * Tz;
                const R t3 = R(2.0 / 3.0);
                const R s01 = g01 + g10, s02 = g02 + g20, s12 = g12 + g21;
                const R N0 = dmu0 * (R(2) * g00 - t3 * th) + dmu1 * s01 + dmu2 * s02;
                const R N1 = dmu0 * s01 + dmu1 * (R(2) * g11 - t3 * th) + dmu2 * s12;
                const R N2 = dmu0 * s02 + dmu1 * s12 + dmu2 * (R(2) * g22 - t3 * th);
                const R diss = mu * ((R(2) * g00 - t3 * th) * g00 + (R(2) * g11 - t3 * th) * g11 +
                                     (R(2) * g22 - t3 * th) * g22 + s01 * s01 + s02 * s02 + s12 * s12);
                acc[1] += N0;
                acc[2] += N1;
                acc[3] += N2;
                acc[4] += uc * N0 + vc * N1 + wc_ * N2 + diss + (skt * kcd) * (Tx * Tx + Ty * Ty + Tz * Tz);
            }
            pend_k = k;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double r = double(acc[v]);
                if (f32 && v == 4) r += accE_shift;
                if (v == 1) fsum = __builtin_fma(fvol, r, fsum);
                pend[v] = r;
                if (UPD) {
                    double nv = __builtin_fma(sc.cg, r, wcur[v]);
                    if (sc.read_prev) nv = __builtin_fma(sc.cz, rcur[v], nv);
                    pend_w[v] = nv;
                }
            }
        }
        shift();
        slot_k = slot_k + 1 == Q ? 0 : slot_k + 1;
        __syncthreads();
    }
    flush();
    if (g.fpart) force_partial<NT>(sm.fred, NT, fsum, g);
}

// LDS working set of the role-split march: the non-split set plus the
// viscous part of the RHS handed from the viscous to the convective role.
template <int S, int TX, int TY, typename R>
struct SmemSplit {
    static constexpr int NR = TX * TY;
    static constexpr int HX = TX + 2 * S, HY = TY + 2 * S, HP = HX * HY;
    static constexpr int Q = 2 * S + 1;
    R sa[3][HP];                                                    // arrival plane: u, v, w
    __attribute__((aligned(16))) R so[Layout<R>::PREC * HP];        // output plane records
    R gyl[2][TY][HX];                                               // D_y u, D_y v of plane k
    __attribute__((aligned(16))) R zring[Q * NR * Layout<R>::ZREC]; // column records
    R xch[NV][NR];                                                  // viscous RHS of plane k
    R vmu[NR];                                                      // viscosity of plane k (role 1 -> 0)
    double fred[NR];                                                // bulk-forcing partial sums
};

// Role-split march: the workgroup holds two threads per tile column. Role 0
// (the first TX*TY threads) stages the output plane and the column ring,
// evaluates the convective terms and the mixed x-y viscous terms and
// applies the update; role 1 stages the arrival plane, keeps the
// mixed-derivative queues, evaluates the viscosity before the plane barrier
// (the ring record of plane k was staged S planes earlier) and the other
// viscous terms after it, and passes them to role 0 through LDS. Each wave has one role, so the
// two halves run as separate instruction streams that the SIMDs interleave,
// and each holds half the per-column state. The work is divided so that
// both roles reach the barriers at about the same time.
//
// Two barriers per plane: (1) after staging, (2) after the viscous hand-over.
// No third one is needed before the next staging: every LDS buffer staged
// for plane k+1 (output plane, arrival plane, the ring slot of plane k-S)
// was last read before barrier 2 of plane k, the hand-over arrays are read
// by role 0 before it reaches barrier 1 of plane k+1 and written again by
// role 1 only after it, and the D_y rows are private to one wave.
template <int SC, int SV, int TX, int TY, typename R, bool UPD, bool PIMG, int VAR = 0>
__device__ __forceinline__ void march_split(SmemSplit<Halo<SC, SV>::S, TX, TY, R>& sm, const double* __restrict__ W,
                                            double* __restrict__ out, double* __restrict__ Rp,
                                            const KGrid& g, const KGas& gas, const StepCoef& sc,
                                            unsigned mask_in, int i0, int j0, int k0, int k1)
{
    const unsigned mask = UPD ? (unsigned)SX_ALL : mask_in;
    constexpr int S = Halo<SC, SV>::S;
    // variants: 1 KEEP-n central flux, 2 thermally perfect gas
    constexpr bool KEEP = VAR == 1, THERMO = VAR == 2;
    using L = Layout<R>;
    constexpr int NR = TX * TY;
    constexpr int HX = TX + 2 * S, HP = HX * (TY + 2 * S);
    constexpr int NPT = (HP + NR - 1) / NR;
    constexpr int Q = 2 * S + 1;
    static_assert(NR % 64 == 0, "each role fills whole waves");
    static_assert(64 % TX == 0, "every row of the tile lies in one wave");
    auto& sa = sm.sa;
    R* const so = sm.so;
    auto& gyl = sm.gyl;
    R* const zring = sm.zring;
    auto& xch = sm.xch;
    auto& vmu = sm.vmu;

    constexpr bool f32 = std::is_same<R, float>::value;
    const double pref = f32 ? gas.pref : 0.0, href = f32 ? gas.href : 0.0;
    const int role = threadIdx.x / NR;
    const int tid = threadIdx.x - role * NR;
    const int tx = tid % TX, ty = tid / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool active = i < g.nx && j < g.ny;
    const int c = (ty + S) * HX + (tx + S);
    const R ey = active ? R(g.eta_y[j]) : R(0);
    const R eyy = active ? R(g.eta_yy[j]) : R(0);
    const R dxi = R(g.dxi), dzi = R(g.dzi);
    const R igM2 = R(gas.igM2);
    const bool visc = mask & SX_VISC;

    // Global accesses take a per-variable base pointer (uniform, scalar
    // registers) plus a 32-bit byte offset: the in-plane part is fixed per
    // thread, the plane part k*sz is uniform, so each load or store costs
    // one vector add. The host keeps every array of one variable below
    // 4 GiB.
    // inactive threads (ragged tiles) load the nearest interior column; only
    // active threads store
    const int ic = min(i, g.nx - 1), jc = min(j, g.ny - 1);
    const unsigned colbo = (unsigned)((g.base + (long long)jc * g.sy + ic) * 8);
    const unsigned jibo = (unsigned)(((long long)jc * g.nx + ic) * 8);
    auto kbo = [&](int k) { return (unsigned)((long long)k * g.sz * 8); };
    auto kbr = [&](int k) { return (unsigned)((long long)k * g.ny * g.nx * 8); };
    // Halo points outside the ghosted block (ragged tiles, the unused tail
    // of the last round) load the nearest ghosted node instead: valid data,
    // no branch; no active output reads them.
    unsigned hbo[NPT];
#pragma unroll
    for (int a = 0; a < NPT; ++a) {
        const int q = tid + a * NR;
        const int hx = q % HX, hy = q / HX;
        const int gi = min(max(i0 - S + hx, -g.ng), g.nx + g.ng - 1);
        const int gj = min(max(j0 - S + hy, -g.ng), g.ny + g.ng - 1);
        hbo[a] = (unsigned)((g.base + (long long)gj * g.sy + gi) * 8);
    }
    auto fetch = [&](PlaneFetch<NPT>& f, int k, int nvar) {
        const unsigned kb = kbo(k);
#pragma unroll
        for (int a = 0; a < NPT; ++a) {
            if (a + 1 < NPT || tid + a * NR < HP) {   // the last round covers the tail of the plane
                const unsigned bo = hbo[a] + kb;
#pragma unroll
                for (int v = 0; v < 5; ++v)
                    if (v < nvar) f.q[a][v] = ldo(W + v * g.sv, bo);
            }
        }
    };
    auto prims = [&](const double* w5, double& rho, double& u, double& v, double& w, double& T,
                     double& p, double& H) {
        rho = w5[0];
        const double ri = rcp(rho);
        u = w5[1] * ri;
        v = w5[2] * ri;
        w = w5[3] * ri;
        double pr;
        if constexpr (THERMO) {   // thermally perfect: T from the internal energy
            T = tp_T_of_e(gas, w5[4] * ri - 0.5 * (u * u + v * v + w * w));
            pr = rho * T * gas.igM2;
        } else {
            pr = gas.gm1 * (w5[4] - 0.5 * rho * (u * u + v * v + w * w));
            T = gas.gM2 * pr * ri;
        }
        H = (w5[4] + pr) * ri - href;
        p = pr - pref;
    };
    auto znode = [&](int slot) { return ring_read<R>(zring + L::ZREC * (slot * NR + tid), igM2); };
    auto getx = [&](int t) { return plane_read<R>(so, c + t, igM2); };
    auto gety = [&](int t) { return plane_read<R>(so, c + t * HX, igM2); };
    // bulk forcing: cell volume of this column's nodes, running sum of V R_rhou (role 0)
    const double fvol = active && g.fpart ? g.dx * g.y_eta[j] * g.dz : 0.0;
    double fsum = 0.0;
    // the column ring (z stencils of both roles) is staged by role 0
    auto fetch_col = [&](double (&cq)[5], int k) {
        const unsigned bn = colbo + kbo(k);
#pragma unroll
        for (int v = 0; v < 5; ++v) cq[v] = ldo(W + v * g.sv, bn);
    };
    auto stage_column = [&](int slot, const double (&cq)[5]) {
        double rho, u, v, w, T, p, H;
        prims(cq, rho, u, v, w, T, p, H);
        ring_write<R>(zring + L::ZREC * (slot * NR + tid), rho, u, v, w, T, p, H);
    };

    if (role == 0) {
        // ---- convective terms, column ring, update ----------------------
        double wc[5] = {}, rp[5] = {};
        auto fetch_centre = [&](int k) {
            const unsigned bn = colbo + kbo(k), bm = jibo + kbr(k);
            if (UPD) {
#pragma unroll
                for (int v = 0; v < 5; ++v) wc[v] = ldo(W + v * g.sv, bn);
                if (sc.read_prev) {
#pragma unroll
                    for (int v = 0; v < 5; ++v) rp[v] = ldo(Rp + v * g.nint, bm);
                }
            }
        };
        auto stage_output = [&](const PlaneFetch<NPT>& f) {
#pragma unroll
            for (int a = 0; a < NPT; ++a) {
                const int q = tid + a * NR;
                if (q < HP) {
                    double rho, u, v, w, T, p, H;
                    prims(f.q[a], rho, u, v, w, T, p, H);
                    plane_write<R>(so, q, rho, u, v, w, T, p, H);
                }
            }
        };
        PlaneFetch<NPT> fo;
        double cq[5];
        for (int t = 0; t < 2 * S; ++t) {
            fetch_col(cq, k0 - S + t);
            stage_column(t, cq);
            __syncthreads();
            __syncthreads();
        }
        fetch(fo, k0, 5);
        fetch_centre(k0);
        fetch_col(cq, k0 + S);

        double pend[NV] = {0, 0, 0, 0, 0};
        double pend_w[NV] = {0, 0, 0, 0, 0};
        int pend_k = -1;   // plane of the pending stores, -1: none
        auto flush = [&]() {
            if (pend_k < 0) return;
            if (UPD) {
                const unsigned bn = colbo + kbo(pend_k);
#pragma unroll
                for (int v = 0; v < NV; ++v) sto(out + v * g.sv, bn, pend_w[v]);
                if constexpr (PIMG) {
                    const int kk = pend_k;
                    const int ox = i < g.ng ? g.nx : (i >= g.nx - g.ng ? -g.nx : 0);
                    const int oy = j < g.ng ? g.ny : (j >= g.ny - g.ng ? -g.ny : 0);
                    const int oz = kk < g.ng ? g.nz : (kk >= g.nz - g.ng ? -g.nz : 0);
                    for (int c3 = 1; c3 < 8; ++c3) {
                        const int dx = (c3 & 1) ? ox : 0, dy = (c3 & 2) ? oy : 0, dz = (c3 & 4) ? oz : 0;
                        if (((c3 & 1) && !ox) || ((c3 & 2) && !oy) || ((c3 & 4) && !oz)) continue;
                        const unsigned be = bn + (unsigned)((dx + (long long)dy * g.sy + (long long)dz * g.sz) * 8);
#pragma unroll
                        for (int v = 0; v < NV; ++v) sto(out + v * g.sv, be, pend_w[v]);
                    }
                }
                if (sc.write_prev) {
                    const unsigned bm = jibo + kbr(pend_k);
#pragma unroll
                    for (int v = 0; v < NV; ++v) sto(Rp + v * g.nint, bm, pend[v]);
                }
            } else {
                const unsigned bm = jibo + kbr(pend_k);
#pragma unroll
                for (int v = 0; v < NV; ++v) sto(out + v * g.nint, bm, pend[v]);
            }
            pend_k = -1;
        };

        const R eyr = j < g.ny ? R(g.eta_y[j]) : R(0);
        int slot_k = S;
        for (int k = k0; k < k1; ++k) {
            const int slot_new = slot_k + S >= Q ? slot_k + S - Q : slot_k + S;
            stage_output(fo);
            stage_column(slot_new, cq);
            double wcur[5], rcur[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                wcur[v] = wc[v];
                rcur[v] = rp[v];
            }
            flush();
            __syncthreads();                                   // 1: planes staged
            if (k + 1 < k1) {
                fetch(fo, k + 1, 5);
                fetch_centre(k + 1);
                fetch_col(cq, k + 1 + S);
            }
            sched_fence();
            R acc[NV] = {0, 0, 0, 0, 0};
            // D_y u, D_y v over the x-extended columns of this thread's row;
            // only this wave reads them (wavefront-scope ordering)
            auto gy_at = [&](int hx) {
                R su = 0, sv = 0;
#pragma unroll
                for (int l = 1; l <= SV; ++l) {
                    R uu, vu, ud, vd;
                    plane_uv<R>(so, (ty + S + l) * HX + hx, uu, vu);
                    plane_uv<R>(so, (ty + S - l) * HX + hx, ud, vd);
                    su += R(Coef<SV>::a[l]) * (uu - ud);
                    sv += R(Coef<SV>::a[l]) * (vu - vd);
                }
                gyl[0][ty][hx] = eyr * su;
                gyl[1][ty][hx] = eyr * sv;
            };
            if (visc && j < g.ny) {
                gy_at(tx + S);
                if (tx < 2 * S) gy_at(tx < S ? tx : TX + tx);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (active && visc) {
                // mixed x-y parts of mu/3 d_i(div u): d_x d_y v into x-momentum,
                // d_x d_y u into y-momentum
                R gyu[Q], gyv[Q];
#pragma unroll
                for (int t = 0; t < Q; ++t) {
                    gyu[t] = gyl[0][ty][tx + t];
                    gyv[t] = gyl[1][ty][tx + t];
                }
                const Node<R> Cc = getx(0);
                const R m3 = vmu[tid] * R(1.0 / 3.0);
                const R mxy = m3 * (dxi * d1c<SV, S>(gyv));
                const R myx = m3 * (dxi * d1c<SV, S>(gyu));
                acc[1] += mxy;
                acc[2] += myx;
                acc[4] += Cc.u * mxy + Cc.v * myx;
            }
            if (active) {
                R gd[4], dd[4];
                auto getz = [&](int t) {
                    int sl = slot_k + t;
                    sl = sl < 0 ? sl + Q : (sl >= Q ? sl - Q : sl);
                    return znode(sl);
                };
                if (mask & SX_CONV_X) stencil_dir<SC, SV, 0, true, false, KEEP>(getx, dxi, dxi, R(0), acc, gd, dd, &gas);
                if (mask & SX_CONV_Y) stencil_dir<SC, SV, 1, true, false, KEEP>(gety, ey, ey, R(0), acc, gd, dd, &gas);
                if (mask & SX_CONV_Z) stencil_dir<SC, SV, 2, true, false, KEEP>(getz, dzi, dzi, R(0), acc, gd, dd, &gas);
            }
            __syncthreads();                                   // 2: viscous part ready
            if (active) {
                // enthalpy shift correction of the convective energy flux (FP64)
                const double accE_shift = href * double(acc[0]);
                pend_k = k;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double r = double(acc[v] + xch[v][tid]);
                    if (f32 && v == 4) r += accE_shift;
                    if (v == 1) fsum = __builtin_fma(fvol, r, fsum);
                    pend[v] = r;
                    if (UPD) {
                        double nv = __builtin_fma(sc.cg, r, wcur[v]);
                        if (sc.read_prev) nv = __builtin_fma(sc.cz, rcur[v], nv);
                        pend_w[v] = nv;
                    }
                }
            }
            slot_k = slot_k + 1 == Q ? 0 : slot_k + 1;
        }
        flush();
    } else {
        // ---- arrival plane, mixed-derivative queues, viscous terms -------
        R m0[Q], m1[Q], m2[Q];   // D_x w, D_y w, D_x u + D_y v of this column
#pragma unroll
        for (int t = 0; t < Q; ++t) m0[t] = m1[t] = m2[t] = R(0);
        auto stage_arrival = [&](const PlaneFetch<NPT>& f) {
#pragma unroll
            for (int a = 0; a < NPT; ++a) {
                const int q = tid + a * NR;
                if (q < HP) {
                    const double ri = rcp(f.q[a][0]);
                    sa[0][q] = R(f.q[a][1] * ri);
                    sa[1][q] = R(f.q[a][2] * ri);
                    sa[2][q] = R(f.q[a][3] * ri);
                }
            }
        };
        auto arrive = [&]() {
            if (!active) return;
            constexpr int QV = 2 * SV + 1;
            R xw[QV], yw[QV], xu[QV], yv[QV];
#pragma unroll
            for (int t = 0; t < QV; ++t) {
                xu[t] = sa[0][c + t - SV];
                xw[t] = sa[2][c + t - SV];
                yv[t] = sa[1][c + (t - SV) * HX];
                yw[t] = sa[2][c + (t - SV) * HX];
            }
            m0[Q - 1] = dxi * d1<SV>(xw);
            m1[Q - 1] = ey * d1<SV>(yw);
            m2[Q - 1] = dxi * d1<SV>(xu) + ey * d1<SV>(yv);
        };
        auto shift = [&]() {
#pragma unroll
            for (int t = 0; t < Q - 1; ++t) {
                m0[t] = m0[t + 1];
                m1[t] = m1[t + 1];
                m2[t] = m2[t + 1];
            }
        };
        PlaneFetch<NPT> fa;
        for (int t = 0; t < 2 * S; ++t) {
            fetch(fa, k0 - S + t, 4);
            stage_arrival(fa);
            __syncthreads();
            arrive();
            shift();
            __syncthreads();
        }
        fetch(fa, k0 + S, 4);

        int slot_k = S;
        for (int k = k0; k < k1; ++k) {
            stage_arrival(fa);
            // viscosity of plane k from this thread's own ring record
            R uc = 0, vc = 0, wc_ = 0, mu = 0, kcd = 0, smt = 0, skt = 0;
            if (active && visc) {
                const Node<R> Cz = znode(slot_k);
                uc = Cz.u;
                vc = Cz.v;
                wc_ = Cz.w;
                const R Tc = Cz.T;
                mu = visc_pow<R>(Tc, gas) * R(gas.ire);
                smt = R(gas.s) * rcpr<R>(Tc);
                if constexpr (THERMO) {   // k = mu c_p(T) / Pr, grad k = k (s/T + c_p'/c_p) grad T
                    const double cpr = tp_cpR(gas, double(Tc));
                    kcd = mu * R(gas.igM2 * cpr * gas.ipr);
                    skt = smt + R(tp_dcpR(gas, double(Tc)) / cpr);
                } else {
                    kcd = mu * R(gas.cp * gas.ipr);
                    skt = smt;
                }
                vmu[tid] = mu;
            }
            __syncthreads();                                   // 1: planes staged
            arrive();
            if (k + 1 < k1) fetch(fa, k + 1 + S, 4);
            sched_fence();
            R acc[NV] = {0, 0, 0, 0, 0};
            if (active && visc) {
                R gx[4], gy[4], gz[4], dd[4];
                auto getz = [&](int t) {
                    int sl = slot_k + t;
                    sl = sl < 0 ? sl + Q : (sl >= Q ? sl - Q : sl);
                    return znode(sl);
                };
                stencil_dir<SC, SV, 0, false, true>(getx, dxi, dxi * dxi, R(0), acc, gx, dd, nullptr);
                visc_linear<0>(dd, mu, kcd, uc, vc, wc_, acc);
                stencil_dir<SC, SV, 1, false, true>(gety, ey, ey * ey, eyy, acc, gy, dd, nullptr);
                visc_linear<1>(dd, mu, kcd, uc, vc, wc_, acc);
                stencil_dir<SC, SV, 2, false, true>(getz, dzi, dzi * dzi, R(0), acc, gz, dd, nullptr);
                visc_linear<2>(dd, mu, kcd, uc, vc, wc_, acc);
                // mixed z parts of mu/3 d_i(div u): d_z d_x w, d_z d_y w,
                // d_z (d_x u + d_y v) (the x-y parts are the convective role's)
                const R m3 = mu * R(1.0 / 3.0);
                const R mx = m3 * (dzi * d1c<SV, S>(m0));
                const R my = m3 * (dzi * d1c<SV, S>(m1));
                const R mz = m3 * (dzi * d1c<SV, S>(m2));
                acc[1] += mx;
                acc[2] += my;
                acc[3] += mz;
                acc[4] += uc * mx + vc * my + wc_ * mz;
                // nonlinear parts: grad mu (= s mu/T grad T) terms and dissipation
                const R g00 = gx[0], g10 = gx[1], g20 = gx[2], Tx = gx[3];
                const R g01 = gy[0], g11 = gy[1], g21 = gy[2], Ty = gy[3];
                const R g02 = gz[0], g12 = gz[1], g22 = gz[2], Tz = gz[3];
                const R th = g00 + g11 + g22;
                const R smu = smt * mu;
                const R dmu0 = smu * Tx, dmu1 = smu * Ty, dmu2 = smu * Tz;
                const R t3 = R(2.0 / 3.0);
                const R s01 = g01 + g10, s02 = g02 + g20, s12 = g12 + g21;
                const R N0 = dmu0 * (R(2) * g00 - t3 * th) + dmu1 * s01 + dmu2 * s02;
                const R N1 = dmu0 * s01 + dmu1 * (R(2) * g11 - t3 * th) + dmu2 * s12;
                const R N2 = dmu0 * s02 + dmu1 * s12 + dmu2 * (R(2) * g22 - t3 * th);
                const R diss = mu * ((R(2) * g00 - t3 * th) * g00 + (R(2) * g11 - t3 * th) * g11 +
                                     (R(2) * g22 - t3 * th) * g22 + s01 * s01 + s02 * s02 + s12 * s12);
                acc[1] += N0;
                acc[2] += N1;
                acc[3] += N2;
                acc[4] += uc * N0 + vc * N1 + wc_ * N2 + diss + (skt * kcd) * (Tx * Tx + Ty * Ty + Tz * Tz);
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) xch[v][tid] = acc[v];
            __syncthreads();                                   // 2: viscous part ready
            shift();
            slot_k = slot_k + 1 == Q ? 0 : slot_k + 1;
        }
    }
    if (g.fpart) force_partial<2 * NR>(sm.fred, NR, fsum, g);
}

// LDS working set of the plane-ring march (FP64): the halo planes k..k+S
// (records (u, v | w, T | rho, H), pressure p = rho T / (gamma M^2)), the
// interior columns of the past planes k-S..k-1 in the same records, and the
// split march's D_y rows, hand-over and reduction arrays.
template <int S, int TX, int TY>
struct SmemRing {
    static constexpr int NR = TX * TY;
    static constexpr int HX = TX + 2 * S, HY = TY + 2 * S, HP = HX * HY;
    __attribute__((aligned(16))) double halo[(S + 1) * HP * 6];   // planes k .. k+S
    __attribute__((aligned(16))) double past[S * NR * 6];         // planes k-S .. k-1, interior columns
    double gyl[2][TY][HX];                                          // D_y u, D_y v of plane k
    double xch[NV][NR];                                             // viscous RHS of plane k
    double vmu[NR];                                                 // viscosity of plane k (role 1 -> 0)
    double fred[NR];                                                // bulk-forcing partial sums
};

// Plane-ring march (FP64, two roles as in march_split). Every plane of the
// march is fetched from global memory once, with its x/y halo, by all the
// workgroup's threads, and staged as primitive records into one of S+1
// halo slots; it serves as the arrival plane k+S (mixed-derivative queues),
// then as a z-neighbour, then as the output plane k (x and y stencils), and
// when its slot is reused S+1 planes later its interior columns move to the
// past ring, which serves the z stencils of planes k-S..k-1. The thread
// staging a point of plane k+S first copies that point's record of plane
// k-1 (the slot's previous plane) to the past ring, so no extra barrier is
// needed. Besides the plane, role 0 fetches the centre state and the RK
// register of the next output node.
//
// Per plane: (A) stage plane k+S (all threads), role 0 stores plane k-1 and
// role 1 evaluates the viscosity of plane k from its column record; barrier
// 1; (B) role 0 issues its loads of plane k+S+1 (and the next centre) and
// evaluates the convective and mixed x-y terms (with VAR 3 also the sensor
// byte); role 1 forms the in-plane derivatives of plane k+S and the x
// viscous stencil, then issues its loads of plane k+S+1, then the remaining
// viscous terms; barrier 2 (viscous hand-over); role 0 completes the update.
// Every slot written in (A) of plane k+1 (halo slot of plane k, past slot of
// plane k-S) was last read before barrier 2 of plane k.
template <int SC, int SV, int TX, int TY, bool UPD, bool PIMG, int VAR = 0>
__device__ __forceinline__ void march_ring(SmemRing<Halo<SC, SV>::S, TX, TY>& sm, const double* __restrict__ W,
                                           double* __restrict__ out, double* __restrict__ Rp,
                                           const KGrid& g, const KGas& gas, const StepCoef& sc,
                                           unsigned mask_in, int i0, int j0, int k0, int k1)
{
    using R = double;
    const unsigned mask = UPD ? (unsigned)SX_ALL : mask_in;
    constexpr int S = Halo<SC, SV>::S;
    // variants: 1 KEEP-n central flux, 2 thermally perfect gas, 3 the default
    // scheme plus the Ducros sensor of the hybrid step
    constexpr bool KEEP = VAR == 1, THERMO = VAR == 2, SENS = VAR == 3;
    constexpr int NR = TX * TY;
    constexpr int HX = TX + 2 * S, HP = HX * (TY + 2 * S);
    constexpr int NPT = (HP + 2 * NR - 1) / (2 * NR);   // staged points per thread (both roles)
    constexpr int Q = 2 * S + 1;
    constexpr int NH = S + 1;                           // halo slots
    static_assert(NR % 64 == 0, "each role fills whole waves");
    static_assert(64 % TX == 0, "every row of the tile lies in one wave");
    double* const halo = sm.halo;
    double* const past = sm.past;
    auto& gyl = sm.gyl;
    auto& xch = sm.xch;
    auto& vmu = sm.vmu;

    const int role = threadIdx.x / NR;
    const int tid = threadIdx.x - role * NR;
    const int tx = tid % TX, ty = tid / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool active = i < g.nx && j < g.ny;
    const int c = (ty + S) * HX + (tx + S);   // this column in a halo plane
    const R ey = active ? R(g.eta_y[j]) : R(0);
    const R eyy = active ? R(g.eta_yy[j]) : R(0);
    const R dxi = R(g.dxi), dzi = R(g.dzi);
    const R igM2 = R(gas.igM2);
    const bool visc = mask & SX_VISC;

    // global addressing as in march_split (uniform base + 32-bit offsets)
    const int ic = min(i, g.nx - 1), jc = min(j, g.ny - 1);
    const unsigned colbo = (unsigned)((g.base + (long long)jc * g.sy + ic) * 8);
    const unsigned jibo = (unsigned)(((long long)jc * g.nx + ic) * 8);
    auto kbo = [&](int k) { return (unsigned)((long long)k * g.sz * 8); };
    auto kbr = [&](int k) { return (unsigned)((long long)k * g.ny * g.nx * 8); };
    // the points this thread stages: q = threadIdx.x + a * 2 NR; halo points
    // outside the ghosted block load the nearest ghosted node
    unsigned hbo[NPT];
    int hcol[NPT];   // past-ring column of an interior point, -1 otherwise
#pragma unroll
    for (int a = 0; a < NPT; ++a) {
        const int q = threadIdx.x + a * 2 * NR;
        const int hx = q % HX, hy = q / HX;
        const int gi = min(max(i0 - S + hx, -g.ng), g.nx + g.ng - 1);
        const int gj = min(max(j0 - S + hy, -g.ng), g.ny + g.ng - 1);
        hbo[a] = (unsigned)((g.base + (long long)gj * g.sy + gi) * 8);
        const bool in = q < HP && hx >= S && hx < S + TX && hy >= S && hy < S + TY;
        hcol[a] = in ? (hy - S) * TX + (hx - S) : -1;
    }
    auto fetch = [&](PlaneFetch<NPT>& f, int k) {
        const unsigned kb = kbo(k);
#pragma unroll
        for (int a = 0; a < NPT; ++a) {
            if (a + 1 < NPT || (int)threadIdx.x + a * 2 * NR < HP) {
                const unsigned bo = hbo[a] + kb;
#pragma unroll
                for (int v = 0; v < 5; ++v) f.q[a][v] = ldo(W + v * g.sv, bo);
            }
        }
    };
    auto prims = [&](const double* w5, double& rho, double& u, double& v, double& w, double& T, double& H) {
        rho = w5[0];
        const double ri = rcp(rho);
        u = w5[1] * ri;
        v = w5[2] * ri;
        w = w5[3] * ri;
        double pr;
        if constexpr (THERMO) {   // thermally perfect: T from the internal energy
            T = tp_T_of_e(gas, w5[4] * ri - 0.5 * (u * u + v * v + w * w));
            pr = rho * T * gas.igM2;
        } else {
            pr = gas.gm1 * (w5[4] - 0.5 * rho * (u * u + v * v + w * w));
            T = gas.gM2 * pr * ri;
        }
        H = (w5[4] + pr) * ri;
    };
    // stage plane p (fetched in f) into its halo slot; interior points first
    // move the slot's previous plane p-S-1 to the past ring
    auto stage = [&](const PlaneFetch<NPT>& f, int p) {
        const int hs = ((p % NH) + NH) % NH;
        const int ps = (((p - NH) % S) + S) % S;
#pragma unroll
        for (int a = 0; a < NPT; ++a) {
            const int q = threadIdx.x + a * 2 * NR;
            if (q < HP) {
                double* rec = halo + 6 * (hs * HP + q);
                if (hcol[a] >= 0) {
                    const dbl2* o = reinterpret_cast<const dbl2*>(rec);
                    const dbl2 o0 = o[0], o1 = o[1], o2 = o[2];
                    dbl2* d = reinterpret_cast<dbl2*>(past + 6 * (ps * NR + hcol[a]));
                    d[0] = o0;
                    d[1] = o1;
                    d[2] = o2;
                }
                double rho, u, v, w, T, H;
                prims(f.q[a], rho, u, v, w, T, H);
                ring_write<R>(rec, rho, u, v, w, T, 0.0, H);
            }
        }
    };
    // plane p = k + t of this column (t in -S..S) at output plane k
    auto znode_at = [&](int k, int t) {
        const int p = k + t;
        if (t < 0) return ring_read<R>(past + 6 * ((((p % S) + S) % S) * NR + tid), igM2);
        return ring_read<R>(halo + 6 * ((((p % NH) + NH) % NH) * HP + c), igM2);
    };
    // bulk forcing: cell volume of this column's nodes, running sum of V R_rhou (role 0)
    const double fvol = active && g.fpart ? g.dx * g.y_eta[j] * g.dz : 0.0;
    double fsum = 0.0;

    PlaneFetch<NPT> fb;
    // prologue: planes k0-S .. k0+S-1 staged; role 1 forms their in-plane
    // derivatives (queue entries of planes k0-S .. k0+S-1)
    R m0[Q], m1[Q], m2[Q];   // role 1: D_x w, D_y w, D_x u + D_y v of this column
#pragma unroll
    for (int t = 0; t < Q; ++t) m0[t] = m1[t] = m2[t] = R(0);
    auto arrive = [&](int p) {
        if (!active) return;
        const double* hp = halo + 6 * ((((p % NH) + NH) % NH) * HP);
        constexpr int QV = 2 * SV + 1;
        R xw[QV], yw[QV], xu[QV], yv[QV];
#pragma unroll
        for (int t = 0; t < QV; ++t) {
            // the two values needed from each record as one 64-bit pair
            // read ((u, w) along x, (v, w) along y). Half-used 128-bit reads
            // recycle their dead halves as the next read's destination,
            // which serialises the reads; the pair reads cost 2-way bank
            // conflicts at the 48-byte record stride but run faster than
            // whole 128-bit records held live until all are issued
            const double* rx = hp + 6 * (c + t - SV);
            const double* ry = hp + 6 * (c + (t - SV) * HX);
            xu[t] = rx[0];
            xw[t] = rx[2];
            yv[t] = ry[1];
            yw[t] = ry[2];
        }
        m0[Q - 1] = dxi * d1<SV>(xw);
        m1[Q - 1] = ey * d1<SV>(yw);
        m2[Q - 1] = dxi * d1<SV>(xu) + ey * d1<SV>(yv);
    };
    auto shift = [&]() {
#pragma unroll
        for (int t = 0; t < Q - 1; ++t) {
            m0[t] = m0[t + 1];
            m1[t] = m1[t + 1];
            m2[t] = m2[t + 1];
        }
    };
    for (int t = 0; t < 2 * S; ++t) {
        fetch(fb, k0 - S + t);
        stage(fb, k0 - S + t);
        __syncthreads();
        if (role == 1) {
            arrive(k0 - S + t);
            shift();
        }
        __syncthreads();
    }
    fetch(fb, k0 + S);

    auto getx = [&](int k, int t) { return ring_read<R>(halo + 6 * ((k % NH) * HP + c + t), igM2); };
    auto gety = [&](int k, int t) { return ring_read<R>(halo + 6 * ((k % NH) * HP + c + t * HX), igM2); };

    if (role == 0) {
        // ---- convective terms, mixed x-y terms, update ------------------
        double wc[5] = {}, rp[5] = {};
        auto fetch_centre = [&](int k) {
            const unsigned bn = colbo + kbo(k), bm = jibo + kbr(k);
            if (UPD) {
#pragma unroll
                for (int v = 0; v < 5; ++v) wc[v] = ldo(W + v * g.sv, bn);
                if (sc.read_prev) {
#pragma unroll
                    for (int v = 0; v < 5; ++v) rp[v] = ldo(Rp + v * g.nint, bm);
                }
            }
        };
        fetch_centre(k0);
        double pend[NV] = {0, 0, 0, 0, 0};
        double pend_w[NV] = {0, 0, 0, 0, 0};
        int pend_k = -1;   // plane of the pending stores, -1: none
        auto flush = [&]() {
            if (pend_k < 0) return;
            if (UPD) {
                const unsigned bn = colbo + kbo(pend_k);
#pragma unroll
                for (int v = 0; v < NV; ++v) sto(out + v * g.sv, bn, pend_w[v]);
                if constexpr (PIMG) {
                    const int kk = pend_k;
                    const int ox = i < g.ng ? g.nx : (i >= g.nx - g.ng ? -g.nx : 0);
                    const int oy = j < g.ng ? g.ny : (j >= g.ny - g.ng ? -g.ny : 0);
                    const int oz = kk < g.ng ? g.nz : (kk >= g.nz - g.ng ? -g.nz : 0);
                    for (int c3 = 1; c3 < 8; ++c3) {
                        const int dx = (c3 & 1) ? ox : 0, dy = (c3 & 2) ? oy : 0, dz = (c3 & 4) ? oz : 0;
                        if (((c3 & 1) && !ox) || ((c3 & 2) && !oy) || ((c3 & 4) && !oz)) continue;
                        const unsigned be = bn + (unsigned)((dx + (long long)dy * g.sy + (long long)dz * g.sz) * 8);
#pragma unroll
                        for (int v = 0; v < NV; ++v) sto(out + v * g.sv, be, pend_w[v]);
                    }
                }
                if (sc.write_prev) {
                    const unsigned bm = jibo + kbr(pend_k);
#pragma unroll
                    for (int v = 0; v < NV; ++v) sto(Rp + v * g.nint, bm, pend[v]);
                }
            } else {
                const unsigned bm = jibo + kbr(pend_k);
#pragma unroll
                for (int v = 0; v < NV; ++v) sto(out + v * g.nint, bm, pend[v]);
            }
            pend_k = -1;
        };

        const R eyr = j < g.ny ? R(g.eta_y[j]) : R(0);
        for (int k = k0; k < k1; ++k) {
            stage(fb, k + S);
            double wcur[5], rcur[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                wcur[v] = wc[v];
                rcur[v] = rp[v];
            }
            flush();
            __syncthreads();                                   // 1: plane k+S staged
            if (k + 1 < k1) {
                fetch(fb, k + 1 + S);
                fetch_centre(k + 1);
            }
            sched_fence();
            const int hk = k % NH;
            const double* so = halo + 6 * (hk * HP);
            R acc[NV] = {0, 0, 0, 0, 0};
            // D_y u, D_y v over the x-extended columns of this thread's row;
            // only this wave reads them (wavefront-scope ordering)
            auto gy_at = [&](int hx) {
                R su = 0, sv = 0;
#pragma unroll
                for (int l = 1; l <= SV; ++l) {
                    R uu, vu, ud, vd;
                    plane_uv<R>(so, (ty + S + l) * HX + hx, uu, vu);
                    plane_uv<R>(so, (ty + S - l) * HX + hx, ud, vd);
                    su += R(Coef<SV>::a[l]) * (uu - ud);
                    sv += R(Coef<SV>::a[l]) * (vu - vd);
                }
                gyl[0][ty][hx] = eyr * su;
                gyl[1][ty][hx] = eyr * sv;
            };
            if (visc && j < g.ny) {
                gy_at(tx + S);
                if (tx < 2 * S) gy_at(tx < S ? tx : TX + tx);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            auto gx_ = [&](int t) { return getx(k, t); };
            auto gy_ = [&](int t) { return gety(k, t); };
            if (active && visc) {
                // mixed x-y parts of mu/3 d_i(div u)
                R gyu[Q], gyv[Q];
#pragma unroll
                for (int t = 0; t < Q; ++t) {
                    gyu[t] = gyl[0][ty][tx + t];
                    gyv[t] = gyl[1][ty][tx + t];
                }
                const Node<R> Cc = gx_(0);
                const R m3 = vmu[tid] * R(1.0 / 3.0);
                const R mxy = m3 * (dxi * d1c<SV, S>(gyv));
                const R myx = m3 * (dxi * d1c<SV, S>(gyu));
                acc[1] += mxy;
                acc[2] += myx;
                acc[4] += Cc.u * mxy + Cc.v * myx;
            }
            if (!SENS && active) {
                R gd[4], dd[4];
                auto gz_ = [&](int t) { return znode_at(k, t); };
                if (mask & SX_CONV_X) stencil_dir<SC, SV, 0, true, false, KEEP>(gx_, dxi, dxi, R(0), acc, gd, dd, &gas);
                if (mask & SX_CONV_Y) stencil_dir<SC, SV, 1, true, false, KEEP>(gy_, ey, ey, R(0), acc, gd, dd, &gas);
                if (mask & SX_CONV_Z) stencil_dir<SC, SV, 2, true, false, KEEP>(gz_, dzi, dzi, R(0), acc, gd, dd, &gas);
            }
            if constexpr (SENS) {
                // the Ducros sensor of the input state at this node, from the
                // second-order differences of the velocities the convective
                // stencils load anyway, compared with the threshold: one byte
                // per node for the face flags
                if (active) {
                    R dx[4], dy[4], dz[4], dd[4];
                    stencil_dir<SC, SV, 0, true, false, false, true>(gx_, dxi, dxi, R(0), acc, dx, dd, &gas);
                    stencil_dir<SC, SV, 1, true, false, false, true>(gy_, ey, ey, R(0), acc, dy, dd, &gas);
                    auto gz_ = [&](int t) { return znode_at(k, t); };
                    stencil_dir<SC, SV, 2, true, false, false, true>(gz_, dzi, dzi, R(0), acc, dz, dd, &gas);
                    const double ix = 0.5 * g.dxi, iy = 0.5 * g.eta_y[j], iz = 0.5 * g.dzi;
                    const double ux = dx[0] * ix, vx = dx[1] * ix, wx = dx[2] * ix;
                    const double uy = dy[0] * iy, vy = dy[1] * iy, wy = dy[2] * iy;
                    const double uz = dz[0] * iz, vz = dz[1] * iz, wz = dz[2] * iz;
                    const double div = ux + vy + wz;
                    const double o1 = wy - vz, o2 = uz - wx, o3 = vx - uy;
                    const double eps = g.sens_eps;
                    const double t = -div / sqrt(div * div + (o1 * o1 + o2 * o2 + o3 * o3) + eps * eps);
                    g.sens[((long long)k * g.ny + j) * g.nx + i] = (t > 0.0 ? t : 0.0) > g.sens_thr;
                }
            }
            __syncthreads();                                   // 2: viscous part ready
            if (active) {
                pend_k = k;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const double r = acc[v] + xch[v][tid];
                    if (v == 1) fsum = __builtin_fma(fvol, r, fsum);
                    pend[v] = r;
                    if (UPD) {
                        double nv = __builtin_fma(sc.cg, r, wcur[v]);
                        if (sc.read_prev) nv = __builtin_fma(sc.cz, rcur[v], nv);
                        pend_w[v] = nv;
                    }
                }
            }
        }
        flush();
    } else {
        // ---- in-plane derivative queues, viscous terms -------------------
        for (int k = k0; k < k1; ++k) {
            stage(fb, k + S);
            // viscosity of plane k from this column's record
            R uc = 0, vc = 0, wc_ = 0, mu = 0, kcd = 0, smt = 0, skt = 0;
            if (active && visc) {
                const Node<R> Cz = znode_at(k, 0);
                uc = Cz.u;
                vc = Cz.v;
                wc_ = Cz.w;
                const R Tc = Cz.T;
                mu = visc_pow<R>(Tc, gas) * R(gas.ire);
                smt = R(gas.s) * rcpr<R>(Tc);
                if constexpr (THERMO) {   // k = mu c_p(T) / Pr, grad k = k (s/T + c_p'/c_p) grad T
                    const double cpr = tp_cpR(gas, double(Tc));
                    kcd = mu * R(gas.igM2 * cpr * gas.ipr);
                    skt = smt + R(tp_dcpR(gas, double(Tc)) / cpr);
                } else {
                    kcd = mu * R(gas.cp * gas.ipr);
                    skt = smt;
                }
                vmu[tid] = mu;
            }
            __syncthreads();                                   // 1: plane k+S staged
            arrive(k + S);
            R acc[NV] = {0, 0, 0, 0, 0};
            R gx[4], gy[4], gz[4], dd[4];
            auto gx_ = [&](int t) { return getx(k, t); };
            auto gy_ = [&](int t) { return gety(k, t); };
            auto gz_ = [&](int t) { return znode_at(k, t); };
            if (active && visc) {
                stencil_dir<SC, SV, 0, false, true>(gx_, dxi, dxi * dxi, R(0), acc, gx, dd, nullptr);
                visc_linear<0>(dd, mu, kcd, uc, vc, wc_, acc);
            }
            // the loads of plane k+S+1 go out here, after the x stencil,
            // rather than with the convective role's just after the barrier:
            // spreading the two roles' load bursts over the phase measured
            // 9 % faster per launch on MI355X
            sched_fence();
            if (k + 1 < k1) fetch(fb, k + 1 + S);
            sched_fence();
            if (active && visc) {
                stencil_dir<SC, SV, 1, false, true>(gy_, ey, ey * ey, eyy, acc, gy, dd, nullptr);
                visc_linear<1>(dd, mu, kcd, uc, vc, wc_, acc);
            }
            if (active && visc) {
                stencil_dir<SC, SV, 2, false, true>(gz_, dzi, dzi * dzi, R(0), acc, gz, dd, nullptr);
                visc_linear<2>(dd, mu, kcd, uc, vc, wc_, acc);
            }
            if (active && visc) {
                // mixed z parts of mu/3 d_i(div u): d_z d_x w, d_z d_y w,
                // d_z (d_x u + d_y v) (the x-y parts are the convective role's)
                const R m3 = mu * R(1.0 / 3.0);
                const R mx = m3 * (dzi * d1c<SV, S>(m0));
                const R my = m3 * (dzi * d1c<SV, S>(m1));
                const R mz = m3 * (dzi * d1c<SV, S>(m2));
                acc[1] += mx;
                acc[2] += my;
                acc[3] += mz;
                acc[4] += uc * mx + vc * my + wc_ * mz;
                // nonlinear parts: grad mu (= s mu/T grad T) terms and dissipation
                const R g00 = gx[0], g10 = gx[1], g20 = gx[2], Tx = gx[3];
                const R g01 = gy[0], g11 = gy[1], g21 = gy[2], Ty = gy[3];
                const R g02 = gz[0], g12 = gz[1], g22 = gz[2], Tz = gz[3];
                const R th = g00 + g11 + g22;
                const R smu = smt * mu;
                const R dmu0 = smu * Tx, dmu1 = smu * Ty, dmu2 = smu * Tz;
                const R t3 = R(2.0 / 3.0);
                const R s01 = g01 + g10, s02 = g02 + g20, s12 = g12 + g21;
                const R N0 = dmu0 * (R(2) * g00 - t3 * th) + dmu1 * s01 + dmu2 * s02;
                const R N1 = dmu0 * s01 + dmu1 * (R(2) * g11 - t3 * th) + dmu2 * s12;
                const R N2 = dmu0 * s02 + dmu1 * s12 + dmu2 * (R(2) * g22 - t3 * th);
                const R diss = mu * ((R(2) * g00 - t3 * th) * g00 + (R(2) * g11 - t3 * th) * g11 +
                                     (R(2) * g22 - t3 * th) * g22 + s01 * s01 + s02 * s02 + s12 * s12);
                acc[1] += N0;
                acc[2] += N1;
                acc[3] += N2;
                acc[4] += uc * N0 + vc * N1 + wc_ * N2 + diss + (skt * kcd) * (Tx * Tx + Ty * Ty + Tz * Tz);
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) xch[v][tid] = acc[v];
            __syncthreads();                                   // 2: viscous part ready
            shift();
        }
    }
    if (g.fpart) force_partial<2 * NR>(sm.fred, NR, fsum, g);
}

template <int S, int TX, int TY, typename R, bool SPLIT>
struct SmemOf {
    using type = Smem<S, TX, TY, R>;
};
template <int S, int TX, int TY, typename R>
struct SmemOf<S, TX, TY, R, true> {
    using type = SmemSplit<S, TX, TY, R>;
};
// FP64 kernels run the plane-ring march wherever its working set fits the
// 160 KB of LDS of a CU (every single-block tile; the 32-wide batch tiles)
template <int S, int TX, int TY, typename R, bool SPLIT>
struct RingOf {
    static constexpr bool value =
        SPLIT && std::is_same<R, double>::value && sizeof(SmemRing<S, TX, TY>) + 64 <= 160 * 1024;
    using type = typename std::conditional<value, SmemRing<S, TX, TY>, typename SmemOf<S, TX, TY, R, SPLIT>::type>::type;
};

template <int SC, int SV, int TX, int TY, int WPE, typename R, bool UPD, bool PIMG, bool SPLIT, int VAR = 0>
__global__ void __attribute__((amdgpu_flat_work_group_size(TX * TY * (SPLIT ? 2 : 1), TX * TY * (SPLIT ? 2 : 1)),
                               amdgpu_waves_per_eu(WPE)))
k_rhs_central(const double* __restrict__ W, double* __restrict__ out, double* __restrict__ Rp,
              KGrid g, KGas gas, StepCoef sc, unsigned mask, int kc)
{
    using RO = RingOf<Halo<SC, SV>::S, TX, TY, R, SPLIT>;
    __shared__ typename RO::type sm;
    // XCD-aware tile numbering: the hardware deals workgroup b to XCD b % 8,
    // each XCD with its own L2; XCD x takes the x-th eighth of the tiles in
    // x-fastest order, so the tiles marching side by side on one XCD are
    // neighbours and share their halo columns in its L2 (HBM reads of the
    // channel launch 4.84 -> 3.35 GB)
    int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
    const int ntl = gridDim.x * gridDim.y * gridDim.z;
    if (ntl % 8 == 0) {
        const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        const int l = (b % 8) * (ntl / 8) + b / 8;
        bx = l % gridDim.x;
        by = (l / gridDim.x) % gridDim.y;
        bz = l / (gridDim.x * gridDim.y);
    }
    const int k0 = bz * kc;
    if constexpr (RO::value)
        march_ring<SC, SV, TX, TY, UPD, PIMG, VAR>(sm, W, out, Rp, g, gas, sc, mask, bx * TX, by * TY, k0,
                                                   min(k0 + kc, g.nz));
    else if constexpr (SPLIT)
        march_split<SC, SV, TX, TY, R, UPD, PIMG, VAR>(sm, W, out, Rp, g, gas, sc, mask, bx * TX, by * TY, k0,
                                                       min(k0 + kc, g.nz));
    else
        march<SC, SV, TX, TY, R, UPD, PIMG, VAR>(sm, W, out, Rp, g, gas, sc, mask, bx * TX, by * TY, k0,
                                                 min(k0 + kc, g.nz));
}

// Persistent batched kernel: each workgroup pulls (box, column tile,
// z-chunk) work items from a device counter until the list is exhausted.
// The time step is read from device memory, so a captured launch stays
// valid when dt changes; cg = dt gamma_k and cz = dt zeta_k are formed as on
// the host path.
template <int S, int TX, int TY, int WPE, typename R, bool SPLIT>
__global__ void __attribute__((amdgpu_flat_work_group_size(TX * TY * (SPLIT ? 2 : 1), TX * TY * (SPLIT ? 2 : 1)),
                               amdgpu_waves_per_eu(WPE)))
k_rhs_batch(const double* __restrict__ Wsrc, double* __restrict__ Wdst, double* __restrict__ Rp,
            const BoxDesc* __restrict__ boxes, const TileDesc* __restrict__ tiles, int ntiles,
            int* __restrict__ counter, const double* __restrict__ dtp, double gk, double zk,
            int substep)
{
    using RO = RingOf<S, TX, TY, R, SPLIT>;
    __shared__ typename RO::type sm;
    __shared__ int cur;
    const double dt = *dtp;
    const StepCoef sc{dt * gk, dt * zk, substep > 0 ? 1 : 0, substep < 2 ? 1 : 0};
    for (;;) {
        if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
        __syncthreads();
        const int t = cur;
        __syncthreads();
        if (t >= ntiles) break;
        const TileDesc td = tiles[t];
        const BoxDesc& bd = boxes[td.box];
        if constexpr (RO::value)
            march_ring<S, S, TX, TY, true, true>(sm, Wsrc + bd.woff, Wdst + bd.woff, Rp + bd.roff, bd.g, bd.gas,
                                                 sc, (unsigned)SX_ALL, td.i0, td.j0, td.k0, td.k1);
        else if constexpr (SPLIT)
            march_split<S, S, TX, TY, R, true, true>(sm, Wsrc + bd.woff, Wdst + bd.woff, Rp + bd.roff, bd.g,
                                                  bd.gas, sc, (unsigned)SX_ALL, td.i0, td.j0, td.k0, td.k1);
        else
            march<S, S, TX, TY, R, true, true>(sm, Wsrc + bd.woff, Wdst + bd.woff, Rp + bd.roff, bd.g,
                                            bd.gas, sc, (unsigned)SX_ALL, td.i0, td.j0, td.k0, td.k1);
        __syncthreads();
    }
}

__global__ void k_reset_counter(int* c)
{
    if (threadIdx.x == 0) c[0] = 0;
}

__global__ void k_set_value(double* p, double v)
{
    if (threadIdx.x == 0) p[0] = v;
}

// Compute units of the current device (queried once).
static int device_cus()
{
    static int n = 0;
    if (!n) {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
            c = 256;
        n = c;
    }
    return n;
}

// Tile shapes (columns along x by rows along y): FP64 runs the two-role
// split, 32x8 columns (512 threads) up to sixth order -- the smaller halo
// ratio (38x14 staged nodes per 256 outputs instead of 70x10) outweighs the
// shorter rows. FP32 up to sixth order runs the unsplit march on 64x8 tiles,
// two waves per SIMD. At eighth order the nine-plane column ring and the
// wider halo leave LDS for 32x4 split tiles only (256 threads), in both
// precision forms: FP32 then fits two workgroups per CU (two waves per
// SIMD), FP64 one.
template <typename R, int S>
struct Tile {
    static constexpr bool F32 = std::is_same<R, float>::value;
    static constexpr bool SPLIT = !F32 || S > 3;
    static constexpr int TX = SPLIT ? 32 : 64;
    static constexpr int TY = S <= 3 ? 8 : 4;
    static constexpr int NTH = TX * TY * (SPLIT ? 2 : 1);
    // waves per SIMD: FP64 at S = 4 holds a whole CU's LDS with one
    // 256-thread workgroup, so its waves may use the full register file
    static constexpr int WPE = (!F32 && S > 3) ? 1 : 2;
};

// Bulk forcing (the paper's force_rhs_1 sum reduction): f = -sum V R_rhou /
// sum V from the fused launch's nwg partial sums (fixed order), stored
// after them.
__global__ void __launch_bounds__(256) k_force_final(KGrid g, int nwg)
{
    __shared__ double ra[256], rv[256];
    double a = 0.0, v = 0.0;
    for (int b = threadIdx.x; b < nwg; b += 256) a += g.fpart[b];
    for (int j = threadIdx.x; j < g.ny; j += 256) v += g.y_eta[j];
    ra[threadIdx.x] = a;
    rv[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            ra[threadIdx.x] += ra[threadIdx.x + s];
            rv[threadIdx.x] += rv[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) g.fpart[nwg] = -ra[0] / (rv[0] * (g.dx * g.nx) * (g.dz * g.nz));
}

// The force into a right-hand side (R, interior layout) or, after a fused
// update, into the new state and the RK register: rho u += c f, rho E += c f u
// with u of the state the right-hand side was evaluated on.
__global__ void __launch_bounds__(256) k_force_apply(KGrid g, const double* __restrict__ W,
                                                     double* __restrict__ out, double* __restrict__ Rp,
                                                     int nwg, double cg, int upd, int write_prev)
{
    const double f = g.fpart[nwg];
    const long long T = (long long)gridDim.x * 256;
    for (long long m = (long long)blockIdx.x * 256 + threadIdx.x; m < g.nint; m += T) {
        const int i = (int)(m % g.nx);
        const long long jk = m / g.nx;
        const int j = (int)(jk % g.ny);
        const int k = (int)(jk / g.ny);
        const long long n = g.base + (long long)k * g.sz + (long long)j * g.sy + i;
        const double u = W[g.sv + n] / W[n];
        if (upd) {
            out[g.sv + n] += cg * f;
            out[4 * g.sv + n] += cg * (f * u);
            if (write_prev) {
                Rp[g.nint + m] += f;
                Rp[4 * g.nint + m] += f * u;
            }
        } else {
            out[g.nint + m] += f;
            out[4 * g.nint + m] += f * u;
        }
    }
}

static hipError_t launch_force(const KGrid& g, int nwg, const double* W, double* out, double* Rp,
                               const StepCoef* step, hipStream_t st)
{
    hipLaunchKernelGGL(k_force_final, dim3(1), dim3(256), 0, st, g, nwg);
    const long long nb = min((g.nint + 255) / 256, (long long)4096);
    hipLaunchKernelGGL(k_force_apply, dim3((unsigned)nb), dim3(256), 0, st, g, W, out, Rp, nwg,
                       step ? step->cg : 0.0, step ? 1 : 0, step ? step->write_prev : 0);
    return hipGetLastError();
}

template <int SC, int SV, typename R>
static hipError_t launch_rhs_SR(const KGrid& g, const KGas& gas, const double* W, double* out,
                                double* Rprev, const StepCoef* step, unsigned mask, bool pimg,
                                hipStream_t st, int var)
{
    constexpr int S = Halo<SC, SV>::S;
    constexpr int TX = Tile<R, S>::TX, TY = Tile<R, S>::TY, WPE = Tile<R, S>::WPE;
    constexpr bool SP = Tile<R, S>::SPLIT;
    constexpr int NTH = Tile<R, S>::NTH;
    // z is cut into nch chunks, each marched by its own workgroup after a
    // 2S-plane prologue. The count minimises the modelled march length:
    // rounds of workgroups over the CUs (one resident workgroup per CU)
    // times the planes each one steps through. Blocks with at least one
    // tile per CU march whole columns; small blocks, latency-bound, get
    // short chunks (a 32^3 block: one plane per workgroup).
    const int ntiles = ((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY);
    const int cus = device_cus();
    int nch = 1;
    if (ntiles < cus) {
        long long best = -1;
        const int cmax = min(g.nz, 2 * cus);
        for (int c = 1; c <= cmax; ++c) {
            const int kcc = (g.nz + c - 1) / c;
            const long long rounds = ((long long)ntiles * ((g.nz + kcc - 1) / kcc) + cus - 1) / cus;
            const long long t = rounds * (kcc + 2 * S);
            if (best < 0 || t < best) {
                best = t;
                nch = c;
            }
        }
    }
    const int kc = (g.nz + nch - 1) / nch;
    dim3 grid((g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, (g.nz + kc - 1) / kc);
    const int nwg = (int)(grid.x * grid.y * grid.z);
    // bulk forcing on a full right-hand side, after the fused launch
    const bool force = g.fpart && (step || mask == (unsigned)SX_ALL);
    if (var == 1) {
        // KEEP-n flux: FP64, equal orders, no periodic images (checked at init)
        if constexpr (SC == SV && std::is_same<R, double>::value && SP) {
            if (pimg) return hipErrorInvalidValue;
            StepCoef none{0.0, 0.0, 0, 0};
            if (step)
                hipLaunchKernelGGL((k_rhs_central<SC, SV, TX, TY, WPE, R, true, false, SP, 1>), grid, dim3(NTH),
                                   0, st, W, out, Rprev, g, gas, *step, (unsigned)SX_ALL, kc);
            else
                hipLaunchKernelGGL((k_rhs_central<SC, SV, TX, TY, WPE, R, false, false, SP, 1>), grid,
                                   dim3(NTH), 0, st, W, out, Rprev, g, gas, none, mask, kc);
            hipError_t e = hipGetLastError();
            if (e == hipSuccess && force) e = launch_force(g, nwg, W, out, Rprev, step, st);
            return e;
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (var == 2) {
        // thermally perfect gas: equal orders, no periodic images (checked at init)
        if constexpr (SC == SV) {
            if (pimg) return hipErrorInvalidValue;
            StepCoef none{0.0, 0.0, 0, 0};
            if (step)
                hipLaunchKernelGGL((k_rhs_central<SC, SV, TX, TY, WPE, R, true, false, SP, 2>), grid, dim3(NTH),
                                   0, st, W, out, Rprev, g, gas, *step, (unsigned)SX_ALL, kc);
            else
                hipLaunchKernelGGL((k_rhs_central<SC, SV, TX, TY, WPE, R, false, false, SP, 2>), grid,
                                   dim3(NTH), 0, st, W, out, Rprev, g, gas, none, mask, kc);
            hipError_t e = hipGetLastError();
            if (e == hipSuccess && force) e = launch_force(g, nwg, W, out, Rprev, step, st);
            return e;
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (g.sens) {
        // hybrid step: the fused kernel also writes the sensor bytes (FP64
        // plane-ring march, update mode, no periodic images; the handle
        // selects it only then)
        if constexpr (RingOf<S, TX, TY, R, SP>::value) {
            if (!step || pimg || var != 0) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_rhs_central<SC, SV, TX, TY, WPE, R, true, false, SP, 3>), grid, dim3(NTH), 0, st,
                               W, out, Rprev, g, gas, *step, (unsigned)SX_ALL, kc);
            hipError_t e = hipGetLastError();
            if (e == hipSuccess && force) e = launch_force(g, nwg, W, out, Rprev, step, st);
            return e;
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (step && pimg) {
        // periodic images are written only by the equal-order kernels (the
        // handle never selects them for mixed orders)
        if constexpr (SC == SV)
            hipLaunchKernelGGL((k_rhs_central<SC, SV, TX, TY, WPE, R, true, true, SP>), grid, dim3(NTH), 0, st,
                               W, out, Rprev, g, gas, *step, (unsigned)SX_ALL, kc);
        else
            return hipErrorInvalidValue;
    } else if (step) {
        hipLaunchKernelGGL((k_rhs_central<SC, SV, TX, TY, WPE, R, true, false, SP>), grid, dim3(NTH), 0, st,
                           W, out, Rprev, g, gas, *step, (unsigned)SX_ALL, kc);
    } else {
        StepCoef none{0.0, 0.0, 0, 0};
        hipLaunchKernelGGL((k_rhs_central<SC, SV, TX, TY, WPE, R, false, false, SP>), grid, dim3(NTH), 0,
                           st, W, out, Rprev, g, gas, none, mask, kc);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && force) e = launch_force(g, nwg, W, out, Rprev, step, st);
    return e;
}

template <int SC, typename R>
static hipError_t launch_rhs_CR(int Lv, const KGrid& g, const KGas& gas, const double* W, double* out,
                                double* Rprev, const StepCoef* step, unsigned mask, bool pimg,
                                hipStream_t st, int var)
{
    switch (Lv) {
    case 1: return launch_rhs_SR<SC, 1, R>(g, gas, W, out, Rprev, step, mask, pimg, st, var);
    case 2: return launch_rhs_SR<SC, 2, R>(g, gas, W, out, Rprev, step, mask, pimg, st, var);
    case 3: return launch_rhs_SR<SC, 3, R>(g, gas, W, out, Rprev, step, mask, pimg, st, var);
    case 4: return launch_rhs_SR<SC, 4, R>(g, gas, W, out, Rprev, step, mask, pimg, st, var);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
static hipError_t launch_rhs_R(const KGrid& g, const KGas& gas, const KScheme& sc, const double* W,
                               double* out, double* Rprev, const StepCoef* step, unsigned mask,
                               bool pimg, hipStream_t st)
{
    const int var = sc.flux == SX_FLUX_KEEP ? 1 : (gas.thermo ? 2 : 0);
    switch (sc.L) {
    case 1: return launch_rhs_CR<1, R>(sc.Lv, g, gas, W, out, Rprev, step, mask, pimg, st, var);
    case 2: return launch_rhs_CR<2, R>(sc.Lv, g, gas, W, out, Rprev, step, mask, pimg, st, var);
    case 3: return launch_rhs_CR<3, R>(sc.Lv, g, gas, W, out, Rprev, step, mask, pimg, st, var);
    case 4: return launch_rhs_CR<4, R>(sc.Lv, g, gas, W, out, Rprev, step, mask, pimg, st, var);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rhs(const KGrid& g, const KGas& gas, const KScheme& sc, const double* W,
                      double* out, double* Rprev, const StepCoef* step, unsigned mask, bool pimg,
                      hipStream_t st)
{
    if (sc.precision == SX_FP32_FLUX)
        return launch_rhs_R<float>(g, gas, sc, W, out, Rprev, step, mask, pimg, st);
    return launch_rhs_R<double>(g, gas, sc, W, out, Rprev, step, mask, pimg, st);
}

// Batched tile shapes, at the single-block kernel's thread count: variant 0
// is 64 wide, variant 1 is 32 wide (every lane busy on blocks whose x
// extent is 32 or 96).
template <typename R, int S, int V>
struct BTile {
    static constexpr int NT = Tile<R, S>::TX * Tile<R, S>::TY;
    static constexpr int TX = V == 0 ? 64 : 32;
    static constexpr int TY = NT / TX;
    static constexpr int WPE = Tile<R, S>::WPE;
    static constexpr bool SPLIT = Tile<R, S>::SPLIT;
    static constexpr int NTH = Tile<R, S>::NTH;
};

template <int S, typename R, int V>
static hipError_t launch_batch_SRV(const BatchLaunch& b, hipStream_t st)
{
    constexpr int TX = BTile<R, S, V>::TX, TY = BTile<R, S, V>::TY, WPE = BTile<R, S, V>::WPE;
    constexpr bool SP = BTile<R, S, V>::SPLIT;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, b.counter);
    hipLaunchKernelGGL((k_rhs_batch<S, TX, TY, WPE, R, SP>), dim3(b.nwg), dim3(BTile<R, S, V>::NTH), 0, st, b.Wsrc,
                       b.Wdst, b.Rp, b.boxes, b.tiles, b.ntiles, b.counter, b.dt, b.gk, b.zk,
                       b.substep);
    return hipGetLastError();
}

template <int S, typename R, int V>
static int occupancy_SRV()
{
    constexpr int TX = BTile<R, S, V>::TX, TY = BTile<R, S, V>::TY, WPE = BTile<R, S, V>::WPE;
    constexpr bool SP = BTile<R, S, V>::SPLIT;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rhs_batch<S, TX, TY, WPE, R, SP>, BTile<R, S, V>::NTH, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

template <typename R, int V>
static hipError_t launch_batch_RV(int L, const BatchLaunch& b, hipStream_t st)
{
    switch (L) {
    case 1: return launch_batch_SRV<1, R, V>(b, st);
    case 2: return launch_batch_SRV<2, R, V>(b, st);
    case 3: return launch_batch_SRV<3, R, V>(b, st);
    case 4: return launch_batch_SRV<4, R, V>(b, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int V>
static int occupancy_RV(int L)
{
    switch (L) {
    case 1: return occupancy_SRV<1, R, V>();
    case 2: return occupancy_SRV<2, R, V>();
    case 3: return occupancy_SRV<3, R, V>();
    case 4: return occupancy_SRV<4, R, V>();
    default: return 0;
    }
}

hipError_t launch_batch(const KScheme& sc, int variant, const BatchLaunch& b, hipStream_t st)
{
    const bool f32 = sc.precision == SX_FP32_FLUX;
    if (variant == 0)
        return f32 ? launch_batch_RV<float, 0>(sc.L, b, st) : launch_batch_RV<double, 0>(sc.L, b, st);
    if (variant == 1)
        return f32 ? launch_batch_RV<float, 1>(sc.L, b, st) : launch_batch_RV<double, 1>(sc.L, b, st);
    return hipErrorInvalidValue;
}

hipError_t launch_set_value(double* p, double v, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_value, dim3(1), dim3(64), 0, st, p, v);
    return hipGetLastError();
}

int batch_occupancy(const KScheme& sc, int variant)
{
    const bool f32 = sc.precision == SX_FP32_FLUX;
    if (variant == 0) return f32 ? occupancy_RV<float, 0>(sc.L) : occupancy_RV<double, 0>(sc.L);
    if (variant == 1) return f32 ? occupancy_RV<float, 1>(sc.L) : occupancy_RV<double, 1>(sc.L);
    return 0;
}

template <typename R>
static void tile_shape_R(int L, int variant, int* tx, int* ty)
{
    const bool v1 = variant == 1;
    switch (L) {
    case 1: *tx = v1 ? BTile<R, 1, 1>::TX : BTile<R, 1, 0>::TX; *ty = v1 ? BTile<R, 1, 1>::TY : BTile<R, 1, 0>::TY; break;
    case 2: *tx = v1 ? BTile<R, 2, 1>::TX : BTile<R, 2, 0>::TX; *ty = v1 ? BTile<R, 2, 1>::TY : BTile<R, 2, 0>::TY; break;
    case 3: *tx = v1 ? BTile<R, 3, 1>::TX : BTile<R, 3, 0>::TX; *ty = v1 ? BTile<R, 3, 1>::TY : BTile<R, 3, 0>::TY; break;
    default: *tx = v1 ? BTile<R, 4, 1>::TX : BTile<R, 4, 0>::TX; *ty = v1 ? BTile<R, 4, 1>::TY : BTile<R, 4, 0>::TY; break;
    }
}

void batch_tile_shape(const KScheme& sc, int variant, int* tx, int* ty)
{
    if (sc.precision == SX_FP32_FLUX) tile_shape_R<float>(sc.L, variant, tx, ty);
    else tile_shape_R<double>(sc.L, variant, tx, ty);
}

}  // namespace sx
