// sx_weno.hip -- shock-capturing part of the hybrid scheme (Section 2 of the
// paper): modified Ducros sensor, face flags, and the WENO characteristic
// flux on flagged faces.
//
// The fused kernel (sx_rhs.hip) applies the central split-form flux on every
// face. This pass then visits only nodes next to a flagged face and adds,
// for each flagged face, the difference between the WENO characteristic
// flux and the central flux of that face:
//   dR_i = -scale (dF_{i+1/2} - dF_{i-1/2}),  dF = F_weno - F_central,
// to the RHS (rhs mode) or, after the fused RK update, to the new state
// (W' += dt gamma_k dR) and to the RK register (Rprev += dR). Each node
// gathers its own faces (a face shared by two listed nodes is evaluated by
// both), so results do not depend on list order and need no atomics on the
// state.
//
// Sensor: theta = max(0, -div u / sqrt(div u^2 + |curl u|^2 + eps^2)) with
// second-order central differences at interior nodes; a face i+1/2 uses WENO
// iff the largest theta over the WENO stencil nodes i-r+1 .. i+r exceeds the
// threshold; ghost nodes take theta of their periodic image, else of their
// mirror interior node. Flags are decided in FP64 in both precision forms.
//
// WENO flux at a face: Roe average of the two adjacent nodes, eigenvectors
// of the Euler flux Jacobian in (rho, rho u_n, rho u_t1, rho u_t2, rho E),
// local Lax-Friedrichs splitting per characteristic field with
// lambda_k = max over the stencil of |eigenvalue k|, Jiang-Shu WENO of order
// 2r-1 on g+ (left-biased) and g- (mirrored), projection back with the right
// eigenvectors.
#include "sx_internal.h"

namespace sx {

namespace {

constexpr int WB = 256;

__device__ __forceinline__ int map_ghost(int i, int n, int bc_lo, int bc_hi)
{
    if (i < 0) return bc_lo == SX_BC_PERIODIC ? i + n : -1 - i;
    if (i >= n) return bc_hi == SX_BC_PERIODIC ? i - n : 2 * n - 1 - i;
    return i;
}

// theta at interior nodes, stored [nz][ny][nx]
__global__ void __launch_bounds__(WB) k_theta(KGrid g, double eps, const double* __restrict__ W,
                                              double* __restrict__ theta)
{
    const long long m = (long long)blockIdx.x * WB + threadIdx.x;
    if (m >= g.nint) return;
    const int i = (int)(m % g.nx);
    const long long jk = m / g.nx;
    const int j = (int)(jk % g.ny);
    const int k = (int)(jk / g.ny);
    const long long n = g.base + (long long)k * g.sz + (long long)j * g.sy + i;
    auto vel = [&](long long q, double& u, double& v, double& w) {
        const double ri = 1.0 / W[q];
        u = W[q + g.sv] * ri;
        v = W[q + 2 * g.sv] * ri;
        w = W[q + 3 * g.sv] * ri;
    };
    double up, vp, wp, um, vm, wm;
    const double ix = 0.5 * g.dxi, iy = 0.5 * g.eta_y[j], iz = 0.5 * g.dzi;
    vel(n + 1, up, vp, wp);
    vel(n - 1, um, vm, wm);
    const double ux = (up - um) * ix, vx = (vp - vm) * ix, wx = (wp - wm) * ix;
    vel(n + g.sy, up, vp, wp);
    vel(n - g.sy, um, vm, wm);
    const double uy = (up - um) * iy, vy = (vp - vm) * iy, wy = (wp - wm) * iy;
    vel(n + g.sz, up, vp, wp);
    vel(n - g.sz, um, vm, wm);
    const double uz = (up - um) * iz, vz = (vp - vm) * iz, wz = (wp - wm) * iz;
    const double div = ux + vy + wz;
    const double o1 = wy - vz, o2 = uz - wx, o3 = vx - uy;
    const double t = -div / sqrt(div * div + (o1 * o1 + o2 * o2 + o3 * o3) + eps * eps);
    theta[m] = t > 0.0 ? t : 0.0;
}

// Face flags: f[d] holds n_d + 1 faces per line (entry f is the face
// between nodes f-1 and f). One thread per interior node writes its "+"
// faces, node 0 of a line also its "-" face; it appends itself to the list
// when any of its six faces is flagged. A flags override (three arrays
// uploaded by the caller) replaces the sensor.
__global__ void __launch_bounds__(WB) k_flags(KGrid g, int r, double thr,
                                              const double* __restrict__ theta,
                                              unsigned char* __restrict__ fx,
                                              unsigned char* __restrict__ fy,
                                              unsigned char* __restrict__ fz, int use_override,
                                              int* __restrict__ list, int* __restrict__ count)
{
    const long long m = (long long)blockIdx.x * WB + threadIdx.x;
    if (m >= g.nint) return;
    const int i = (int)(m % g.nx);
    const long long jk = m / g.nx;
    const int j = (int)(jk % g.ny);
    const int k = (int)(jk / g.ny);
    auto th = [&](int a, int b, int c) -> double {
        const int ia = map_ghost(a, g.nx, g.bc[0], g.bc[1]);
        const int jb = map_ghost(b, g.ny, g.bc[2], g.bc[3]);
        const int kc = map_ghost(c, g.nz, g.bc[4], g.bc[5]);
        return theta[((long long)kc * g.ny + jb) * g.nx + ia];
    };
    // flag of the face after node (a,b,c) along d
    auto face = [&](int d, int a, int b, int c) -> unsigned char {
        double mx = 0.0;
        for (int t = -r + 1; t <= r; ++t) {
            const double v = d == 0 ? th(a + t, b, c) : (d == 1 ? th(a, b + t, c) : th(a, b, c + t));
            mx = v > mx ? v : mx;
        }
        return mx > thr ? 1 : 0;
    };
    const long long ix = ((long long)k * g.ny + j) * (g.nx + 1) + i;       // face i-1/2 in fx
    const long long iy = ((long long)k * (g.ny + 1) + j) * g.nx + i;       // face j-1/2 in fy
    const long long iz = ((long long)k * g.ny + j) * g.nx + i;             // face k-1/2 in fz
    const long long sfy = g.nx, sfz = (long long)g.ny * g.nx;
    unsigned char any = 0;
    if (use_override) {
        any = fx[ix] | fx[ix + 1] | fy[iy] | fy[iy + sfy] | fz[iz] | fz[iz + sfz];
    } else {
        const unsigned char xp = face(0, i, j, k), yp = face(1, i, j, k), zp = face(2, i, j, k);
        const unsigned char xm = face(0, i - 1, j, k), ym = face(1, i, j - 1, k), zm = face(2, i, j, k - 1);
        fx[ix + 1] = xp;
        fy[iy + sfy] = yp;
        fz[iz + sfz] = zp;
        if (i == 0) fx[ix] = xm;
        if (j == 0) fy[iy] = ym;
        if (k == 0) fz[iz] = zm;
        any = xp | yp | zp | xm | ym | zm;
    }
    if (any) {
        const int slot = atomicAdd(count, 1);
        list[slot] = (int)m;
    }
}

__global__ void k_zero_int(int* p) { *p = 0; }

struct Prim {
    double r, u, v, w, p, H, W[5];
};

// Jiang-Shu WENO reconstruction at i+1/2 from v[0 .. 2r-2] = v_{i-r+1 .. i+r-1}
template <int RW>
__device__ __forceinline__ double weno_left(const double* v, double eps)
{
    if (RW == 1) return v[0];
    if (RW == 2) {
        const double vm = v[0], v0 = v[1], vp = v[2];
        const double q0 = 0.5 * (-vm + 3.0 * v0), q1 = 0.5 * (v0 + vp);
        const double b0 = (v0 - vm) * (v0 - vm), b1 = (vp - v0) * (vp - v0);
        const double a0 = (1.0 / 3.0) / ((eps + b0) * (eps + b0));
        const double a1 = (2.0 / 3.0) / ((eps + b1) * (eps + b1));
        return (a0 * q0 + a1 * q1) / (a0 + a1);
    }
    const double vmm = v[0], vm = v[1], v0 = v[2], vp = v[3], vpp = v[4];
    const double q0 = (2.0 * vmm - 7.0 * vm + 11.0 * v0) * (1.0 / 6.0);
    const double q1 = (-vm + 5.0 * v0 + 2.0 * vp) * (1.0 / 6.0);
    const double q2 = (2.0 * v0 + 5.0 * vp - vpp) * (1.0 / 6.0);
    double t, b0, b1, b2;
    t = vmm - 2.0 * vm + v0; b0 = (13.0 / 12.0) * t * t;
    t = vmm - 4.0 * vm + 3.0 * v0; b0 += 0.25 * t * t;
    t = vm - 2.0 * v0 + vp; b1 = (13.0 / 12.0) * t * t;
    t = vm - vp; b1 += 0.25 * t * t;
    t = v0 - 2.0 * vp + vpp; b2 = (13.0 / 12.0) * t * t;
    t = 3.0 * v0 - 4.0 * vp + vpp; b2 += 0.25 * t * t;
    const double a0 = 0.1 / ((eps + b0) * (eps + b0));
    const double a1 = 0.6 / ((eps + b1) * (eps + b1));
    const double a2 = 0.3 / ((eps + b2) * (eps + b2));
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

// WENO minus central flux of the face between stencil positions HALF-1 and
// HALF (nodes nd[0 .. 2*HALF-1], face in the middle) along direction d.
template <int L, int RW, int HALF>
__device__ void face_delta(const Prim (&nd)[2 * HALF], int d, const KGas& gas, double eps,
                           double (&dF)[NV])
{
    // central split-form face flux, pairs (A, B) = (c-m, c-m+l), c = HALF-1
    double Fc[NV] = {0, 0, 0, 0, 0}, P = 0.0;
#pragma unroll
    for (int l = 1; l <= L; ++l) {
        const double cl = 2.0 * Coef<L>::a[l];
#pragma unroll
        for (int mm = 0; mm < l; ++mm) {
            const Prim& A = nd[HALF - 1 - mm];
            const Prim& B = nd[HALF - 1 - mm + l];
            const double udA = d == 0 ? A.u : (d == 1 ? A.v : A.w);
            const double udB = d == 0 ? B.u : (d == 1 ? B.v : B.w);
            const double mf = 0.125 * (A.r + B.r) * (udA + udB);
            Fc[0] += cl * (mf * 2.0);
            Fc[1] += cl * (mf * (A.u + B.u));
            Fc[2] += cl * (mf * (A.v + B.v));
            Fc[3] += cl * (mf * (A.w + B.w));
            Fc[4] += cl * (mf * (A.H + B.H));
            P += cl * (0.5 * (A.p + B.p));
        }
    }
    Fc[1 + d] += P;

    // characteristic basis at the Roe average of the two face nodes
    const int perm[NV] = {0, 1 + d, 1 + (d + 1) % 3, 1 + (d + 2) % 3, 4};
    const Prim& a = nd[HALF - 1];
    const Prim& b = nd[HALF];
    const double sa = sqrt(a.r), sb = sqrt(b.r), si = 1.0 / (sa + sb);
    auto vel = [&](const Prim& q, int c) { return c == 0 ? q.u : (c == 1 ? q.v : q.w); };
    const double un = (sa * vel(a, d) + sb * vel(b, d)) * si;
    const double ut1 = (sa * vel(a, (d + 1) % 3) + sb * vel(b, (d + 1) % 3)) * si;
    const double ut2 = (sa * vel(a, (d + 2) % 3) + sb * vel(b, (d + 2) % 3)) * si;
    const double Hb = (sa * a.H + sb * b.H) * si;
    const double q2 = un * un + ut1 * ut1 + ut2 * ut2;
    const double cb = sqrt(gas.gm1 * (Hb - 0.5 * q2));
    const double b1 = gas.gm1 / (cb * cb);
    const double b2 = 0.5 * q2 * b1;
    const double ic = 1.0 / cb;
    const double Lm[5][5] = {
        {0.5 * (b2 + un * ic), 0.5 * (-b1 * un - ic), -0.5 * b1 * ut1, -0.5 * b1 * ut2, 0.5 * b1},
        {-ut1, 0.0, 1.0, 0.0, 0.0},
        {-ut2, 0.0, 0.0, 1.0, 0.0},
        {1.0 - b2, b1 * un, b1 * ut1, b1 * ut2, -b1},
        {0.5 * (b2 - un * ic), 0.5 * (-b1 * un + ic), -0.5 * b1 * ut1, -0.5 * b1 * ut2, 0.5 * b1}};

    constexpr int NS = 2 * RW;          // WENO stencil nodes
    constexpr int OFF = HALF - RW;      // first WENO node in nd[]
    double g[NS][NV], qc[NS][NV], lam[NV] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const Prim& n = nd[OFF + t];
        const double unt = vel(n, d);
        const double ct = sqrt(gas.gamma * n.p / n.r);
        const double ev[NV] = {fabs(unt - ct), fabs(unt), fabs(unt), fabs(unt), fabs(unt + ct)};
        double wp[NV], fp[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) wp[v] = n.W[perm[v]];
        fp[0] = wp[0] * unt;
        fp[1] = wp[1] * unt + n.p;
        fp[2] = wp[2] * unt;
        fp[3] = wp[3] * unt;
        fp[4] = (wp[4] + n.p) * unt;
#pragma unroll
        for (int kk = 0; kk < NV; ++kk) {
            double sg = 0.0, sq = 0.0;
#pragma unroll
            for (int mm = 0; mm < NV; ++mm) {
                sg += Lm[kk][mm] * fp[mm];
                sq += Lm[kk][mm] * wp[mm];
            }
            g[t][kk] = sg;
            qc[t][kk] = sq;
            lam[kk] = ev[kk] > lam[kk] ? ev[kk] : lam[kk];
        }
    }
    double Fh[NV];
#pragma unroll
    for (int kk = 0; kk < NV; ++kk) {
        double vl[2 * RW - 1], vr[2 * RW - 1];
#pragma unroll
        for (int t = 0; t < 2 * RW - 1; ++t) {
            vl[t] = 0.5 * (g[t][kk] + lam[kk] * qc[t][kk]);
            vr[t] = 0.5 * (g[NS - 1 - t][kk] - lam[kk] * qc[NS - 1 - t][kk]);
        }
        Fh[kk] = weno_left<RW>(vl, eps) + weno_left<RW>(vr, eps);
    }
    // right eigenvectors applied to the reconstructed characteristic flux
    const double Rm[5][5] = {
        {1.0, 0.0, 0.0, 1.0, 1.0},
        {un - cb, 0.0, 0.0, un, un + cb},
        {ut1, 1.0, 0.0, ut1, ut1},
        {ut2, 0.0, 1.0, ut2, ut2},
        {Hb - un * cb, ut1, ut2, 0.5 * q2, Hb + un * cb}};
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double s = 0.0;
#pragma unroll
        for (int kk = 0; kk < NV; ++kk) s += Rm[v][kk] * Fh[kk];
        dF[perm[v]] = s - Fc[perm[v]];
    }
}

__device__ __forceinline__ Prim load_node(const double* __restrict__ W, long long q, long long sv,
                                          const KGas& gas)
{
    Prim n;
#pragma unroll
    for (int v = 0; v < NV; ++v) n.W[v] = W[q + v * sv];
    n.r = n.W[0];
    const double ri = 1.0 / n.r;
    n.u = n.W[1] * ri;
    n.v = n.W[2] * ri;
    n.w = n.W[3] * ri;
    n.p = gas.gm1 * (n.W[4] - 0.5 * n.r * (n.u * n.u + n.v * n.v + n.w * n.w));
    n.H = (n.W[4] + n.p) * ri;
    return n;
}

// Correction of one listed node: for each direction with a flagged face,
// dR -= scale (dF_plus - dF_minus). mode 0: R += dR (rhs); mode 1: update
// (out = W', cg = dt gamma_k; Rp += dR when write_prev).
template <int L, int RW>
__global__ void __launch_bounds__(WB) k_weno(KGrid g, KGas gas, double eps, unsigned mask,
                                             const double* __restrict__ W,
                                             const unsigned char* __restrict__ fx,
                                             const unsigned char* __restrict__ fy,
                                             const unsigned char* __restrict__ fz,
                                             const int* __restrict__ list,
                                             const int* __restrict__ count, int mode, double cg,
                                             int write_prev, double* __restrict__ out,
                                             double* __restrict__ Rp)
{
    constexpr int HALF = L > RW ? L : RW;
    const int t = blockIdx.x * WB + threadIdx.x;
    if (t >= *count) return;
    const long long m = list[t];
    const int i = (int)(m % g.nx);
    const long long jk = m / g.nx;
    const int j = (int)(jk % g.ny);
    const int k = (int)(jk / g.ny);
    const long long n = g.base + (long long)k * g.sz + (long long)j * g.sy + i;
    const long long ix = ((long long)k * g.ny + j) * (g.nx + 1) + i;
    const long long iy = ((long long)k * (g.ny + 1) + j) * g.nx + i;
    const long long iz = ((long long)k * g.ny + j) * g.nx + i;
    const unsigned char fl[3][2] = {{fx[ix], fx[ix + 1]},
                                    {fy[iy], fy[iy + g.nx]},
                                    {fz[iz], fz[iz + (long long)g.ny * g.nx]}};
    double dR[NV] = {0, 0, 0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        if (!(mask & (1u << d))) continue;
        if (!fl[d][0] && !fl[d][1]) continue;
        const long long s = d == 0 ? 1 : (d == 1 ? g.sy : g.sz);
        const double scale = d == 0 ? g.dxi : (d == 1 ? g.eta_y[j] : g.dzi);
        // nodes i-HALF .. i+HALF: the two faces share 2*HALF-1 of them
        Prim nd[2 * HALF + 1];
#pragma unroll
        for (int q = 0; q < 2 * HALF + 1; ++q) nd[q] = load_node(W, n + (q - HALF) * s, g.sv, gas);
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            if (!fl[d][side]) continue;
            Prim sub[2 * HALF];
#pragma unroll
            for (int q = 0; q < 2 * HALF; ++q) sub[q] = nd[q + side];   // face i-1/2 (side 0) / i+1/2
            double dF[NV];
            face_delta<L, RW, HALF>(sub, d, gas, eps, dF);
            const double sg = side == 1 ? -scale : scale;
#pragma unroll
            for (int v = 0; v < NV; ++v) dR[v] += sg * dF[v];
        }
    }
    if (mode == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) out[v * g.nint + m] += dR[v];
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            out[v * g.sv + n] = __builtin_fma(cg, dR[v], out[v * g.sv + n]);
            if (write_prev) Rp[v * g.nint + m] += dR[v];
        }
    }
}

template <int L>
hipError_t launch_weno_L(int RW, const KGrid& g, const KGas& gas, double eps, unsigned mask,
                         const double* W, const unsigned char* fx, const unsigned char* fy,
                         const unsigned char* fz, const int* list, const int* count, int mode,
                         double cg, int write_prev, double* out, double* Rp, hipStream_t st)
{
    const dim3 grid((unsigned)((g.nint + WB - 1) / WB));
    switch (RW) {
    case 1: hipLaunchKernelGGL((k_weno<L, 1>), grid, dim3(WB), 0, st, g, gas, eps, mask, W, fx, fy, fz,
                               list, count, mode, cg, write_prev, out, Rp); break;
    case 2: hipLaunchKernelGGL((k_weno<L, 2>), grid, dim3(WB), 0, st, g, gas, eps, mask, W, fx, fy, fz,
                               list, count, mode, cg, write_prev, out, Rp); break;
    default: hipLaunchKernelGGL((k_weno<L, 3>), grid, dim3(WB), 0, st, g, gas, eps, mask, W, fx, fy,
                                fz, list, count, mode, cg, write_prev, out, Rp); break;
    }
    return hipGetLastError();
}

// Integer face counts per direction (exact, order independent).
__global__ void __launch_bounds__(WB) k_count(const unsigned char* __restrict__ f, long long n,
                                              unsigned long long* __restrict__ out)
{
    __shared__ unsigned long long red[WB];
    unsigned long long a = 0;
    for (long long e = (long long)blockIdx.x * WB + threadIdx.x; e < n; e += (long long)gridDim.x * WB)
        a += f[e];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int s = WB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

__global__ void k_zero_u64(unsigned long long* p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

}  // namespace

hipError_t launch_count_flags(const KGrid& g, const unsigned char* fx, const unsigned char* fy,
                              const unsigned char* fz, unsigned long long* counts, hipStream_t st)
{
    const long long nf[3] = {(long long)g.nz * g.ny * (g.nx + 1), (long long)g.nz * (g.ny + 1) * g.nx,
                             (long long)(g.nz + 1) * g.ny * g.nx};
    const unsigned char* f[3] = {fx, fy, fz};
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, counts, 3);
    for (int d = 0; d < 3; ++d)
        hipLaunchKernelGGL(k_count, dim3(1024), dim3(WB), 0, st, f[d], nf[d], counts + d);
    return hipGetLastError();
}

hipError_t launch_sensor_flags(const KGrid& g, const KScheme& sc, const double* W, double* theta,
                               unsigned char* fx, unsigned char* fy, unsigned char* fz,
                               int use_override, int* list, int* count, hipStream_t st)
{
    const dim3 grid((unsigned)((g.nint + WB - 1) / WB));
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, count);
    if (!use_override)
        hipLaunchKernelGGL(k_theta, grid, dim3(WB), 0, st, g, sc.sensor_eps, W, theta);
    hipLaunchKernelGGL(k_flags, grid, dim3(WB), 0, st, g, sc.r, sc.sensor_thr, theta, fx, fy, fz,
                       use_override, list, count);
    return hipGetLastError();
}

// The grid of the correction kernel covers every node; threads past the
// (device-side) list length return at once.
hipError_t launch_weno(const KGrid& g, const KGas& gas, const KScheme& sc, unsigned mask,
                       const double* W, const unsigned char* fx, const unsigned char* fy,
                       const unsigned char* fz, const int* list, const int* count, int mode,
                       double cg, int write_prev, double* out, double* Rp, hipStream_t st)
{
    switch (sc.L) {
    case 1: return launch_weno_L<1>(sc.r, g, gas, sc.weno_eps, mask, W, fx, fy, fz, list, count, mode, cg, write_prev, out, Rp, st);
    case 2: return launch_weno_L<2>(sc.r, g, gas, sc.weno_eps, mask, W, fx, fy, fz, list, count, mode, cg, write_prev, out, Rp, st);
    case 3: return launch_weno_L<3>(sc.r, g, gas, sc.weno_eps, mask, W, fx, fy, fz, list, count, mode, cg, write_prev, out, Rp, st);
    default: return launch_weno_L<4>(sc.r, g, gas, sc.weno_eps, mask, W, fx, fy, fz, list, count, mode, cg, write_prev, out, Rp, st);
    }
}

}  // namespace sx
