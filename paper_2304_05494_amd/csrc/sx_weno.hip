// sx_weno.hip -- shock-capturing part of the hybrid scheme (Section 2 of the
// paper): modified Ducros sensor, face flags, and the WENO characteristic
// flux on flagged faces.
//
// The fused kernel (sx_rhs.hip) applies the central split-form flux on every
// face. This pass then corrects the flagged faces only, in three steps:
//   1. k_flaglist (after k_theta): every node decides the flags of its six
//      faces, writes those it owns (the face after it along each direction,
//      plus the first face of each line), appends its owned flagged faces to
//      one list per direction and itself to a node list when any of its six
//      faces is flagged (one atomic per list per workgroup); injected flags
//      are listed by k_lists;
//   2. k_weno_face: one thread per flagged face evaluates
//      dF = F_weno - F_central once and stores it by face index, so the
//      wave's lanes all run the same characteristic-flux code (no per-node
//      branching over faces and directions);
//   3. k_weno_node: one thread per listed node gathers the dF of its flagged
//      faces (known from the node list's face masks) in a fixed order, dR = -scale (dF_{i+1/2} - dF_{i-1/2}) per
//      direction, and adds dR to the RHS (rhs mode) or, after the fused RK
//      update, to the new state (W' += dt gamma_k dR) and to the RK register
//      (Rprev += dR).
// The order of the lists does not change any result.
//
// Sensor: theta = max(0, -div u / sqrt(div u^2 + |curl u|^2 + eps^2)) with
// second-order central differences at interior nodes; a face i+1/2 uses WENO
// iff the largest theta over the WENO stencil nodes i-r+1 .. i+r exceeds the
// threshold, that is iff any of them exceeds it; ghost nodes take theta of
// their periodic image, else of their mirror interior node. theta and its
// comparison are FP64 in both precision forms.
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

// theta at interior nodes, compared with the threshold once: a face's
// flag only asks whether the largest theta of its window exceeds the
// threshold, i.e. whether any node's does, so one byte per node (stored
// [nz][ny][nx]) carries all the flags need. A workgroup owns a TXT x TYT
// column tile and marches a chunk of TZT planes; velocities of three planes
// (tile + one halo node, read from the ghosted state) sit in an LDS ring,
// so each node's velocity is formed once.
constexpr int TXT = 64, TYT = 8, TZT = 16;
__global__ void __launch_bounds__(TXT * TYT) k_theta(KGrid g, double eps, double thr,
                                                     const double* __restrict__ W,
                                                     unsigned char* __restrict__ sens)
{
    constexpr int HXT = TXT + 2, HYT = TYT + 2, HPT = HXT * HYT;
    __shared__ double vel[3][3][HPT];   // ring slot, component, node
    const int tx = threadIdx.x % TXT, ty = threadIdx.x / TXT;
    const int i0 = blockIdx.x * TXT, j0 = blockIdx.y * TYT;
    const int i = i0 + tx, j = j0 + ty;
    const int k0 = blockIdx.z * TZT, k1 = min(k0 + TZT, g.nz);
    const bool active = i < g.nx && j < g.ny;
    auto stage = [&](int slot, int k) {
        for (int q = threadIdx.x; q < HPT; q += TXT * TYT) {
            const int a = i0 - 1 + q % HXT, bb = j0 - 1 + q / HXT;
            double u = 0.0, v = 0.0, w = 0.0;
            if (a < g.nx + g.ng && bb < g.ny + g.ng) {
                const long long n = g.base + (long long)k * g.sz + (long long)bb * g.sy + a;
                const double ri = 1.0 / W[n];
                u = W[n + g.sv] * ri;
                v = W[n + 2 * g.sv] * ri;
                w = W[n + 3 * g.sv] * ri;
            }
            vel[slot][0][q] = u;
            vel[slot][1][q] = v;
            vel[slot][2][q] = w;
        }
    };
    stage(0, k0 - 1);
    stage(1, k0);
    const double ix = 0.5 * g.dxi, iz = 0.5 * g.dzi;
    const double iy = active ? 0.5 * g.eta_y[j] : 0.0;
    const int c = (ty + 1) * HXT + tx + 1;
    for (int k = k0; k < k1; ++k) {
        const int sm = (k - k0) % 3, s0 = (k - k0 + 1) % 3, sp = (k - k0 + 2) % 3;   // planes k-1, k, k+1
        stage(sp, k + 1);
        __syncthreads();
        if (active) {
            const double ux = (vel[s0][0][c + 1] - vel[s0][0][c - 1]) * ix;
            const double vx = (vel[s0][1][c + 1] - vel[s0][1][c - 1]) * ix;
            const double wx = (vel[s0][2][c + 1] - vel[s0][2][c - 1]) * ix;
            const double uy = (vel[s0][0][c + HXT] - vel[s0][0][c - HXT]) * iy;
            const double vy = (vel[s0][1][c + HXT] - vel[s0][1][c - HXT]) * iy;
            const double wy = (vel[s0][2][c + HXT] - vel[s0][2][c - HXT]) * iy;
            const double uz = (vel[sp][0][c] - vel[sm][0][c]) * iz;
            const double vz = (vel[sp][1][c] - vel[sm][1][c]) * iz;
            const double wz = (vel[sp][2][c] - vel[sm][2][c]) * iz;
            const double div = ux + vy + wz;
            const double o1 = wy - vz, o2 = uz - wx, o3 = vx - uy;
            const double t = -div / sqrt(div * div + (o1 * o1 + o2 * o2 + o3 * o3) + eps * eps);
            sens[((long long)k * g.ny + j) * g.nx + i] = (t > 0.0 ? t : 0.0) > thr;
        }
        __syncthreads();
    }
}

// Face flags: f[d] holds n_d + 1 faces per line (entry f is the face
// between nodes f-1 and f); a face is flagged iff the largest theta over
// the 2r nodes of its WENO stencil exceeds the threshold.

// Wave-aggregated append into a workgroup's LDS cursor: returns this lane's
// slot (relative to the workgroup's block of the list) or -1.
__device__ __forceinline__ int wave_slot(bool pred, int* cursor)
{
    const unsigned long long mask = __ballot(pred);
    if (!mask) return -1;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(cursor, __popcll(mask));
    base = __shfl(base, leader);
    return pred ? base + __popcll(mask & ((1ull << lane) - 1ull)) : -1;
}

// Lists from the face flags. Workgroup w owns nodes [w*WB*LPT, (w+1)*WB*LPT):
// a counting pass sizes its share of each list (flagged faces it owns per
// direction, and its nodes with any flagged face), one global atomic per
// list reserves the space, a second pass writes the entries.
constexpr int LPT = 16;   // nodes per thread
__global__ void __launch_bounds__(WB) k_lists(KGrid g, WenoBufs b)
{
    __shared__ int cur[4], base[4];
    if (threadIdx.x < 4) cur[threadIdx.x] = 0;
    __syncthreads();
    const long long m0 = (long long)blockIdx.x * WB * LPT;
    const long long sfy = g.nx, sfz = (long long)g.ny * g.nx;
    auto visit = [&](bool write) {
        for (int it = 0; it < LPT; ++it) {
            const long long m = m0 + (long long)it * WB + threadIdx.x;
            const bool in = m < g.nint;
            bool own[6] = {false, false, false, false, false, false}, node = false;
            unsigned nb = 0;
            long long e[6] = {0, 0, 0, 0, 0, 0};
            if (in) {
                const int i = (int)(m % g.nx);
                const long long jk = m / g.nx;
                const int j = (int)(jk % g.ny);
                const int k = (int)(jk / g.ny);
                const long long ix = ((long long)k * g.ny + j) * (g.nx + 1) + i;
                const long long iy = ((long long)k * (g.ny + 1) + j) * g.nx + i;
                const long long iz = ((long long)k * g.ny + j) * g.nx + i;
                const bool xm = b.f[0][ix], xp = b.f[0][ix + 1];
                const bool ym = b.f[1][iy], yp = b.f[1][iy + sfy];
                const bool zm = b.f[2][iz], zp = b.f[2][iz + sfz];
                own[0] = xp; e[0] = ix + 1;
                own[1] = i == 0 && xm; e[1] = ix;
                own[2] = yp; e[2] = iy + sfy;
                own[3] = j == 0 && ym; e[3] = iy;
                own[4] = zp; e[4] = iz + sfz;
                own[5] = k == 0 && zm; e[5] = iz;
                node = xm || xp || ym || yp || zm || zp;
                nb = xm | (xp << 1) | (ym << 2) | (yp << 3) | (zm << 4) | (zp << 5);
            }
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const int slot = wave_slot(own[q], &cur[q / 2]);
                if (write && slot >= 0) b.flist[q / 2][base[q / 2] + slot] = (int)e[q];
            }
            const int slot = wave_slot(node, &cur[3]);
            if (write && slot >= 0) {
                b.nlist[base[3] + slot] = (int)m;
                b.nmask[base[3] + slot] = (unsigned char)nb;
            }
        }
    };
    visit(false);
    __syncthreads();
    if (threadIdx.x < 4) {
        base[threadIdx.x] = cur[threadIdx.x] ? atomicAdd(&b.counts[threadIdx.x], cur[threadIdx.x]) : 0;
        cur[threadIdx.x] = 0;
    }
    __syncthreads();
    visit(true);
}

// Flags and lists in one pass (the sensor path; injected flags go through
// k_lists). A workgroup owns a GX x GY column tile and marches a chunk of
// GZ planes: the sensor bytes of the plane with an r-wide x/y halo sit in
// LDS (x and y windows), each thread keeps its column's last 2r+1 in
// registers (z windows). Every node decides all six of its faces
// (the "+" faces it owns and the "-" faces, whose windows it reads from the
// same LDS plane and register window), so it knows at once which faces it
// lists and whether it is a listed node. Those bits stay in LDS over the
// chunk while the workgroup counts its entries; one global atomic per list
// then reserves its share and a second sweep over the bits writes the
// entries. A face's flag is written by the node after it (and the first
// face of each line by the line's first node).
constexpr int GX = 64, GY = 8, GZ = 32;
template <int RW>
__global__ void __launch_bounds__(GX * GY) k_flaglist(KGrid g, const unsigned char* __restrict__ sens, WenoBufs b)
{
    constexpr int HXF = GX + 2 * RW, HYF = GY + 2 * RW, HPF = HXF * HYF;
    constexpr int NPF = (HPF + GX * GY - 1) / (GX * GY);
    __shared__ unsigned pl[HYF][HXF];
    __shared__ unsigned char bits[GZ][GX * GY];   // flags of the node's faces x-, x+, y-, y+, z-, z+
    __shared__ int cur[4], base[4];
    if (threadIdx.x < 4) cur[threadIdx.x] = 0;
    const int tx = threadIdx.x % GX, ty = threadIdx.x / GX;
    const int i0 = blockIdx.x * GX, j0 = blockIdx.y * GY;
    const int i = i0 + tx, j = j0 + ty;
    const bool active = i < g.nx && j < g.ny;
    const int k0 = blockIdx.z * GZ, k1 = min(k0 + GZ, g.nz);
    const long long psz = (long long)g.ny * g.nx;
    // in-plane offsets of this thread's halo points (x and y mapped once;
    // ghost positions take the sensor of their periodic image or mirror node)
    // and of its own column; the plane part is uniform
    int hoff[NPF];
#pragma unroll
    for (int a = 0; a < NPF; ++a) {
        const int q = threadIdx.x + a * GX * GY;
        const int x = min(i0 - RW + q % HXF, g.nx + RW - 1), y = min(j0 - RW + q / HXF, g.ny + RW - 1);
        hoff[a] = map_ghost(y, g.ny, g.bc[2], g.bc[3]) * g.nx + map_ghost(x, g.nx, g.bc[0], g.bc[1]);
    }
    const int coff = (active ? j : 0) * g.nx + (active ? i : 0);
    auto plane = [&](int k) { return sens + map_ghost(k, g.nz, g.bc[4], g.bc[5]) * psz; };
    unsigned win[2 * RW + 1];   // sensor of this column at planes k-r .. k+r
#pragma unroll
    for (int t = 1; t <= 2 * RW; ++t) win[t] = plane(k0 - RW - 1 + t)[coff];   // planes k0-r .. k0+r-1
    win[0] = 0;
    auto wave_count = [&](bool pred, int* c) {
        const unsigned long long m = __ballot(pred);
        if (m && __lane_id() == __ffsll((long long)m) - 1) atomicAdd(c, __popcll(m));
    };
    // sensor of the next plane (this thread's halo points, its column's new
    // window value) is loaded while the current plane is decided
    unsigned hv[NPF], wv;
    auto load_plane = [&](int k) {
        const unsigned char* tp = plane(k);
#pragma unroll
        for (int a = 0; a < NPF; ++a)
            if (a + 1 < NPF || threadIdx.x + a * GX * GY < HPF) hv[a] = tp[hoff[a]];
        wv = plane(k + RW)[coff];
    };
    // per-thread parts of the face indices (k-independent)
    const int fxo = j * (g.nx + 1) + i, fyo = j * g.nx + i;
    const long long fxk = (long long)g.ny * (g.nx + 1), fyk = (long long)(g.ny + 1) * g.nx;
    // faces a node lists: those after it, and the first face of each line
    auto owned = [&](unsigned bt, int k) {
        return (bt & 0x2a) | ((bt & 1) && i == 0 ? 1u : 0u) | ((bt & 4) && j == 0 ? 4u : 0u) |
               ((bt & 16) && k == 0 ? 16u : 0u);
    };
    load_plane(k0);
    for (int k = k0; k < k1; ++k) {
#pragma unroll
        for (int t = 0; t < 2 * RW; ++t) win[t] = win[t + 1];
        win[2 * RW] = wv;
        __syncthreads();
#pragma unroll
        for (int a = 0; a < NPF; ++a) {
            const int q = threadIdx.x + a * GX * GY;
            if (a + 1 < NPF || q < HPF) pl[q / HXF][q % HXF] = hv[a];
        }
        __syncthreads();
        if (k + 1 < k1) load_plane(k + 1);
        unsigned bt = 0;
        if (active) {
            const int cx = tx + RW, cy = ty + RW;
            // "+" face: nodes -r+1 .. r around the node; "-" face: -r .. r-1
            unsigned xc = 0, yc = 0, zc = 0;
#pragma unroll
            for (int t = -RW + 1; t <= RW - 1; ++t) {
                xc |= pl[cy][cx + t];
                yc |= pl[cy + t][cx];
            }
#pragma unroll
            for (int t = 1; t < 2 * RW; ++t) zc |= win[t];
            const bool fxm = xc | pl[cy][cx - RW], fym = yc | pl[cy - RW][cx], fzm = zc | win[0];
            const bool fxp = xc | pl[cy][cx + RW], fyp = yc | pl[cy + RW][cx], fzp = zc | win[2 * RW];
            unsigned char* const fx = b.f[0] + k * fxk;
            unsigned char* const fy = b.f[1] + k * fyk;
            unsigned char* const fz = b.f[2] + k * psz;
            fx[fxo + 1] = fxp;
            fy[fyo + g.nx] = fyp;
            fz[fyo + psz] = fzp;
            if (i == 0) fx[fxo] = fxm;
            if (j == 0) fy[fyo] = fym;
            if (k == 0) fz[fyo] = fzm;
            bt = fxm | (fxp << 1) | (fym << 2) | (fyp << 3) | (fzm << 4) | (fzp << 5);
        }
        bits[k - k0][threadIdx.x] = (unsigned char)bt;
        const unsigned ow = owned(bt, k);
        wave_count(ow & 1, &cur[0]);
        wave_count(ow & 2, &cur[0]);
        wave_count(ow & 4, &cur[1]);
        wave_count(ow & 8, &cur[1]);
        wave_count(ow & 16, &cur[2]);
        wave_count(ow & 32, &cur[2]);
        wave_count(bt != 0, &cur[3]);
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        base[threadIdx.x] = cur[threadIdx.x] ? atomicAdd(&b.counts[threadIdx.x], cur[threadIdx.x]) : 0;
        cur[threadIdx.x] = 0;
    }
    __syncthreads();
    for (int k = k0; k < k1; ++k) {
        const unsigned bt = bits[k - k0][threadIdx.x];
        if (!__ballot(bt != 0)) continue;
        // face and node indices fit in int (init keeps the interior below 2^29 points)
        const int ix = (int)(k * fxk) + fxo, iy = (int)(k * fyk) + fyo, iz = (int)(k * psz) + fyo;
        const int e[6] = {ix, ix + 1, iy, iy + g.nx, iz, iz + (int)psz};
        const unsigned ow = owned(bt, k);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int slot = wave_slot((ow >> q) & 1, &cur[q / 2]);
            if (slot >= 0) b.flist[q / 2][base[q / 2] + slot] = e[q];
        }
        const int slot = wave_slot(bt != 0, &cur[3]);
        if (slot >= 0) {
            b.nlist[base[3] + slot] = iz;
            b.nmask[base[3] + slot] = (unsigned char)bt;
        }
    }
}

template <int RW>
static void launch_flaglist(const KGrid& g, const WenoBufs& b, hipStream_t st)
{
    const dim3 grid((unsigned)((g.nx + GX - 1) / GX), (unsigned)((g.ny + GY - 1) / GY), (unsigned)((g.nz + GZ - 1) / GZ));
    hipLaunchKernelGGL(k_flaglist<RW>, grid, dim3(GX * GY), 0, st, g, b.sens, b);
}

__global__ void k_zero_counts(int* p)
{
    if (threadIdx.x < 4) p[threadIdx.x] = 0;
}

// Seventh-order WENO (Balsara-Shu) at i+1/2 from v[0 .. 6] = v_{i-3 .. i+3}.
// Candidate k interpolates the cell averages of cells i-3+k .. i+k by a
// cubic P in the cell index t (t = 0 at cell i); the reconstruction of cell
// i's polynomial at its right face is v_i + P'(0)/2 + P''(0)/12, and the
// Jiang-Shu indicator (the integral over the cell of the squared first to
// third derivatives, scaled by powers of the width) is
// P1^2 + 13/3 P2^2 + 781/20 P3^2 with P = sum_n P_n t^n -- a sum of squares,
// which keeps it accurate on smooth data where it is tiny. P_n come from the
// forward differences of the four values (Newton form about the first).
// Linear weights (1, 12, 18, 4)/35.
template <typename R>
__device__ __forceinline__ R weno7_left(const R* v, R eps)
{
    R q[4], a[4];
    const R dw[4] = {R(1.0 / 35.0), R(12.0 / 35.0), R(18.0 / 35.0), R(4.0 / 35.0)};
    // P1 = d1 + c1 d2 + c2 d3, P2 = d2/2 + c3 d3, P3 = d3/6, for first node a = k-3
    const R c1[4] = {R(2.5), R(1.5), R(0.5), R(-0.5)};
    const R c2[4] = {R(11.0 / 6.0), R(1.0 / 3.0), R(-1.0 / 6.0), R(1.0 / 3.0)};
    const R c3[4] = {R(1.0), R(0.5), R(0.0), R(-0.5)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const R y0 = v[k], y1 = v[k + 1], y2 = v[k + 2], y3 = v[k + 3];
        const R d1 = y1 - y0;
        const R d2 = (y2 - y1) - d1;
        const R d3 = ((y3 - y2) - (y2 - y1)) - d2;
        const R P1 = d1 + c1[k] * d2 + c2[k] * d3;
        const R P2 = R(0.5) * d2 + c3[k] * d3;
        const R P3 = d3 * R(1.0 / 6.0);
        q[k] = v[3] + R(0.5) * P1 + P2 * R(1.0 / 6.0);
        const R b = P1 * P1 + R(13.0 / 3.0) * P2 * P2 + R(781.0 / 20.0) * P3 * P3;
        a[k] = (eps + b) * (eps + b);   // s_k^2
    }
    if constexpr (std::is_same<R, double>::value) {
        // d_k / s_k^2 times the product of all s_j^2: one division
        const R s01 = a[0] * a[1], s23 = a[2] * a[3];
        const R w0 = dw[0] * (a[1] * s23), w1 = dw[1] * (a[0] * s23), w2 = dw[2] * (s01 * a[3]), w3 = dw[3] * (s01 * a[2]);
        return (w0 * q[0] + w1 * q[1] + w2 * q[2] + w3 * q[3]) / (w0 + w1 + w2 + w3);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = dw[k] / a[k];
    return (a[0] * q[0] + a[1] * q[1] + a[2] * q[2] + a[3] * q[3]) / (a[0] + a[1] + a[2] + a[3]);
}

// Jiang-Shu WENO reconstruction at i+1/2 from v[0 .. 2r-2] = v_{i-r+1 .. i+r-1}
template <int RW, typename R>
__device__ __forceinline__ R weno_left(const R* v, R eps)
{
    if (RW == 1) return v[0];
    if (RW == 4) return weno7_left<R>(v, eps);
    if (RW == 2) {
        const R vm = v[0], v0 = v[1], vp = v[2];
        const R q0 = R(0.5) * (-vm + R(3) * v0), q1 = R(0.5) * (v0 + vp);
        const R b0 = (v0 - vm) * (v0 - vm), b1 = (vp - v0) * (vp - v0);
        // weights d_k / s_k^2 times the other s_j^2: one division
        const R p0 = (eps + b0) * (eps + b0), p1 = (eps + b1) * (eps + b1);
        const R a0 = R(1.0 / 3.0) * p1, a1 = R(2.0 / 3.0) * p0;
        return (a0 * q0 + a1 * q1) / (a0 + a1);
    }
    const R vmm = v[0], vm = v[1], v0 = v[2], vp = v[3], vpp = v[4];
    const R q0 = (R(2) * vmm - R(7) * vm + R(11) * v0) * R(1.0 / 6.0);
    const R q1 = (-vm + R(5) * v0 + R(2) * vp) * R(1.0 / 6.0);
    const R q2 = (R(2) * v0 + R(5) * vp - vpp) * R(1.0 / 6.0);
    R t, b0, b1, b2;
    t = vmm - R(2) * vm + v0; b0 = R(13.0 / 12.0) * t * t;
    t = vmm - R(4) * vm + R(3) * v0; b0 += R(0.25) * t * t;
    t = vm - R(2) * v0 + vp; b1 = R(13.0 / 12.0) * t * t;
    t = vm - vp; b1 += R(0.25) * t * t;
    t = v0 - R(2) * vp + vpp; b2 = R(13.0 / 12.0) * t * t;
    t = R(3) * v0 - R(4) * vp + vpp; b2 += R(0.25) * t * t;
    // the nonlinear weights d_k / s_k^2 (s_k = eps + beta_k) times the
    // product of the other s_j^2, so a single division normalises them
    // (products of two squares: with eps = 1e-6 they stay within the range
    // of FP32 as of FP64)
    const R p0 = (eps + b0) * (eps + b0), p1 = (eps + b1) * (eps + b1), p2 = (eps + b2) * (eps + b2);
    const R a0 = R(0.1) * (p1 * p2), a1 = R(0.6) * (p0 * p2), a2 = R(0.3) * (p0 * p1);
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

// Values of one stencil node, in the face's frame: x[0..4] = (rho,
// rho u_n, rho u_t1, rho u_t2, rho E), primitive u, v, w, H, p.
template <typename R>
struct FNode {
    R x[NV];
    R r, u, v, w, H, p;
};

// WENO minus central flux of the face between stencil nodes HALF-1 and HALF
// (node q at W + n0 + q s) along direction d; FP64 primitives, arithmetic in R.
template <int L, int RW, int HALF, int d, typename R>
__device__ __forceinline__ void face_delta(const double* __restrict__ W, long long n0, long long s,
                                           long long sv, const KGas& gas, R eps, double (&dF)[NV])
{
    constexpr int perm[NV] = {0, 1 + d, 1 + (d + 1) % 3, 1 + (d + 2) % 3, 4};
    constexpr int NS = 2 * RW;          // WENO stencil nodes
    constexpr int OFF = HALF - RW;      // first WENO node in nd[]
    constexpr bool F64 = std::is_same<R, double>::value;
    FNode<R> nd[2 * HALF];
    // local Lax-Friedrichs speeds: largest |u_n - c|, |u_n|, |u_n + c| over
    // the WENO stencil (FP64: taken while the nodes load, c from 1/rho)
    R lm = R(0), l0 = R(0), lp = R(0);
#pragma unroll
    for (int q = 0; q < 2 * HALF; ++q) {
        double w5[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) w5[v] = W[n0 + q * s + v * sv];
        const double ri = 1.0 / w5[0];
        const double u = w5[1] * ri, v = w5[2] * ri, w = w5[3] * ri;
        const double p = gas.gm1 * (w5[4] - 0.5 * w5[0] * (u * u + v * v + w * w));
        FNode<R>& f = nd[q];
#pragma unroll
        for (int c = 0; c < NV; ++c) f.x[c] = R(w5[perm[c]]);
        f.r = R(w5[0]);
        f.u = R(u);
        f.v = R(v);
        f.w = R(w);
        f.p = R(p);
        f.H = R((w5[4] + p) * ri);
        if constexpr (F64) {
            if (q >= OFF && q < OFF + NS) {
                const double unt = w5[perm[1]] * ri, ct = sqrt(gas.gamma * p * ri);
                lm = fmax(lm, fabs(unt - ct));
                l0 = fmax(l0, fabs(unt));
                lp = fmax(lp, fabs(unt + ct));
            }
        }
    }
    auto vel = [&](const FNode<R>& q, int c) { return c == 0 ? q.u : (c == 1 ? q.v : q.w); };

    // central split-form face flux, pairs (A, B) = (c-m, c-m+l), c = HALF-1
    R Fc[NV] = {0, 0, 0, 0, 0}, P = R(0);
#pragma unroll
    for (int l = 1; l <= L; ++l) {
        const R cl = R(2.0 * Coef<L>::a[l]);
#pragma unroll
        for (int mm = 0; mm < l; ++mm) {
            const FNode<R>& A = nd[HALF - 1 - mm];
            const FNode<R>& B = nd[HALF - 1 - mm + l];
            const R mf = R(0.125) * (A.r + B.r) * (vel(A, d) + vel(B, d));
            Fc[0] += cl * (mf * R(2));
            Fc[1] += cl * (mf * (A.u + B.u));
            Fc[2] += cl * (mf * (A.v + B.v));
            Fc[3] += cl * (mf * (A.w + B.w));
            Fc[4] += cl * (mf * (A.H + B.H));
            P += cl * (R(0.5) * (A.p + B.p));
        }
    }
    Fc[1 + d] += P;

    // characteristic basis at the Roe average of the two face nodes
    const FNode<R>& a = nd[HALF - 1];
    const FNode<R>& bn = nd[HALF];
    const R sa = sqrt(a.r), sb = sqrt(bn.r), si = R(1) / (sa + sb);
    const R un = (sa * vel(a, d) + sb * vel(bn, d)) * si;
    const R ut1 = (sa * vel(a, (d + 1) % 3) + sb * vel(bn, (d + 1) % 3)) * si;
    const R ut2 = (sa * vel(a, (d + 2) % 3) + sb * vel(bn, (d + 2) % 3)) * si;
    const R Hb = (sa * a.H + sb * bn.H) * si;
    const R q2 = un * un + ut1 * ut1 + ut2 * ut2;
    const R cb = sqrt(R(gas.gm1) * (Hb - R(0.5) * q2));
    const R b1 = R(gas.gm1) / (cb * cb);
    const R b2 = R(0.5) * q2 * b1;
    const R ic = R(1) / cb;
    // rows of the left eigenvector matrix applied to a vector x
    auto lrow = [&](int kk, const R (&x)[NV]) -> R {
        const R tang = -R(0.5) * b1 * (ut1 * x[2] + ut2 * x[3]);
        switch (kk) {
        case 0: return R(0.5) * (b2 + un * ic) * x[0] + R(0.5) * (-b1 * un - ic) * x[1] + tang + R(0.5) * b1 * x[4];
        case 1: return -ut1 * x[0] + x[2];
        case 2: return -ut2 * x[0] + x[3];
        case 3: return (R(1) - b2) * x[0] + b1 * (un * x[1] + ut1 * x[2] + ut2 * x[3]) - b1 * x[4];
        default: return R(0.5) * (b2 - un * ic) * x[0] + R(0.5) * (-b1 * un + ic) * x[1] + tang + R(0.5) * b1 * x[4];
        }
    };

    if constexpr (!F64) {
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const FNode<R>& n = nd[OFF + t];
            const R unt = vel(n, d);
            const R ct = sqrt(R(gas.gamma) * n.p / n.r);
            lm = fmax(lm, fabs(unt - ct));
            l0 = fmax(l0, fabs(unt));
            lp = fmax(lp, fabs(unt + ct));
        }
    }
    R Fh[NV];
#pragma unroll
    for (int kk = 0; kk < NV; ++kk) {
        const R lam = kk == 0 ? lm : (kk == 4 ? lp : l0);
        R gq[NS][2];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const FNode<R>& n = nd[OFF + t];
            const R unt = vel(n, d);
            R fl[NV];
            fl[0] = n.x[1];
            fl[1] = n.x[1] * unt + n.p;
            fl[2] = n.x[2] * unt;
            fl[3] = n.x[3] * unt;
            fl[4] = (n.x[4] + n.p) * unt;
            gq[t][0] = lrow(kk, fl);
            gq[t][1] = lrow(kk, n.x);
        }
        R vl[2 * RW - 1], vr[2 * RW - 1];
#pragma unroll
        for (int t = 0; t < 2 * RW - 1; ++t) {
            vl[t] = R(0.5) * (gq[t][0] + lam * gq[t][1]);
            vr[t] = R(0.5) * (gq[NS - 1 - t][0] - lam * gq[NS - 1 - t][1]);
        }
        Fh[kk] = weno_left<RW, R>(vl, eps) + weno_left<RW, R>(vr, eps);
    }
    // right eigenvectors applied to the reconstructed characteristic flux
    const R G[NV] = {Fh[0] + Fh[3] + Fh[4],
                     (un - cb) * Fh[0] + un * Fh[3] + (un + cb) * Fh[4],
                     ut1 * (Fh[0] + Fh[3] + Fh[4]) + Fh[1],
                     ut2 * (Fh[0] + Fh[3] + Fh[4]) + Fh[2],
                     (Hb - un * cb) * Fh[0] + ut1 * Fh[1] + ut2 * Fh[2] + R(0.5) * q2 * Fh[3] +
                         (Hb + un * cb) * Fh[4]};
#pragma unroll
    for (int v = 0; v < NV; ++v) dF[perm[v]] = double(G[v]) - double(Fc[perm[v]]);
}

// One thread per flagged face of direction d (grid-stride over the list):
// dF of the face, stored at its face index.
template <int L, int RW, int d, typename R>
__global__ void __launch_bounds__(WB) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : 2)))
k_weno_face(KGrid g, KGas gas, double eps,
                                                  const double* __restrict__ W, WenoBufs b)
{
    constexpr int HALF = L > RW ? L : RW;
    const int nf = b.counts[d];
    const long long nface = d == 0 ? (long long)g.nz * g.ny * (g.nx + 1)
                                   : (d == 1 ? (long long)g.nz * (g.ny + 1) * g.nx
                                             : (long long)(g.nz + 1) * g.ny * g.nx);
    const int* __restrict__ fl = b.flist[d];
    double* __restrict__ out = b.dF[d];
    const long long s = d == 0 ? 1 : (d == 1 ? g.sy : g.sz);
    for (int t = blockIdx.x * WB + threadIdx.x; t < nf; t += gridDim.x * WB) {
        const long long e = fl[t];
        int i, j, k;   // the node after the face
        if (d == 0) {
            i = (int)(e % (g.nx + 1));
            const long long jk = e / (g.nx + 1);
            j = (int)(jk % g.ny);
            k = (int)(jk / g.ny);
        } else if (d == 1) {
            i = (int)(e % g.nx);
            const long long jk = e / g.nx;
            j = (int)(jk % (g.ny + 1));
            k = (int)(jk / (g.ny + 1));
        } else {
            i = (int)(e % g.nx);
            const long long jk = e / g.nx;
            j = (int)(jk % g.ny);
            k = (int)(jk / g.ny);
        }
        const long long n = g.base + (long long)k * g.sz + (long long)j * g.sy + i;
        double dF[NV];
        face_delta<L, RW, HALF, d, R>(W, n - HALF * s, s, g.sv, gas, R(eps), dF);
#pragma unroll
        for (int v = 0; v < NV; ++v) out[v * nface + e] = dF[v];
    }
}

// One thread per listed node (grid-stride): dR from the dF of its flagged
// faces, directions x, y, z and within each the "-" face then the "+" face.
// mode 0: R += dR (rhs); mode 1: update (out = W', cg = dt gamma_k;
// Rp += dR when write_prev).
__global__ void __launch_bounds__(WB) k_weno_node(KGrid g, unsigned mask, WenoBufs b, int mode,
                                                  double cg, int write_prev, double* __restrict__ out,
                                                  double* __restrict__ Rp)
{
    const int nn = b.counts[3];
    const long long nfx = (long long)g.nz * g.ny * (g.nx + 1);
    const long long nfy = (long long)g.nz * (g.ny + 1) * g.nx;
    const long long nfz = (long long)(g.nz + 1) * g.ny * g.nx;
    for (int t = blockIdx.x * WB + threadIdx.x; t < nn; t += gridDim.x * WB) {
        const long long m = b.nlist[t];
        const unsigned nb = b.nmask[t];
        const int i = (int)(m % g.nx);
        const long long jk = m / g.nx;
        const int j = (int)(jk % g.ny);
        const int k = (int)(jk / g.ny);
        const long long fidx[3][2] = {{((long long)k * g.ny + j) * (g.nx + 1) + i, 0},
                                      {((long long)k * (g.ny + 1) + j) * g.nx + i, 0},
                                      {((long long)k * g.ny + j) * g.nx + i, 0}};
        const long long step[3] = {1, g.nx, (long long)g.ny * g.nx};
        const long long nface[3] = {nfx, nfy, nfz};
        double dR[NV] = {0, 0, 0, 0, 0};
        for (int d = 0; d < 3; ++d) {
            if (!(mask & (1u << d))) continue;
            const double scale = d == 0 ? g.dxi : (d == 1 ? g.eta_y[j] : g.dzi);
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                if (!((nb >> (2 * d + side)) & 1)) continue;
                const long long e = fidx[d][0] + side * step[d];
                const double sg = side == 1 ? -scale : scale;
#pragma unroll
                for (int v = 0; v < NV; ++v) dR[v] += sg * b.dF[d][v * nface[d] + e];
            }
        }
        if (mode == 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v * g.nint + m] += dR[v];
        } else {
            const long long n = g.base + (long long)k * g.sz + (long long)j * g.sy + i;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                out[v * g.sv + n] = __builtin_fma(cg, dR[v], out[v * g.sv + n]);
                if (write_prev) Rp[v * g.nint + m] += dR[v];
            }
        }
    }
}

// Grid of the grid-stride face and node passes: four 256-thread workgroups
// per CU (measured on the shock/boundary-layer block: the node pass 14 %
// faster than with eight, the face passes unchanged, one or two per CU
// slower).
int persistent_blocks()
{
    static int nb = 0;
    if (!nb) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        nb = 4 * cus;
    }
    return nb;
}

template <int L, int RW, typename R>
hipError_t launch_faces(const KGrid& g, const KGas& gas, double eps, unsigned mask, const double* W,
                        const WenoBufs& b, hipStream_t st)
{
    const dim3 grid(persistent_blocks());
    if (mask & SX_CONV_X) hipLaunchKernelGGL((k_weno_face<L, RW, 0, R>), grid, dim3(WB), 0, st, g, gas, eps, W, b);
    if (mask & SX_CONV_Y) hipLaunchKernelGGL((k_weno_face<L, RW, 1, R>), grid, dim3(WB), 0, st, g, gas, eps, W, b);
    if (mask & SX_CONV_Z) hipLaunchKernelGGL((k_weno_face<L, RW, 2, R>), grid, dim3(WB), 0, st, g, gas, eps, W, b);
    return hipGetLastError();
}

template <int L, typename R>
hipError_t launch_faces_L(int RW, const KGrid& g, const KGas& gas, double eps, unsigned mask,
                          const double* W, const WenoBufs& b, hipStream_t st)
{
    switch (RW) {
    case 1: return launch_faces<L, 1, R>(g, gas, eps, mask, W, b, st);
    case 2: return launch_faces<L, 2, R>(g, gas, eps, mask, W, b, st);
    case 3: return launch_faces<L, 3, R>(g, gas, eps, mask, W, b, st);
    default: return launch_faces<L, 4, R>(g, gas, eps, mask, W, b, st);
    }
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

hipError_t launch_sensor_flags(const KGrid& g, const KScheme& sc, const double* W,
                               const WenoBufs& b, int use_override, int sens_done, hipStream_t st)
{
    const dim3 grid((unsigned)((g.nint + WB - 1) / WB));
    hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(64), 0, st, b.counts);
    if (!use_override) {
        const dim3 tgrid((unsigned)((g.nx + TXT - 1) / TXT), (unsigned)((g.ny + TYT - 1) / TYT),
                         (unsigned)((g.nz + TZT - 1) / TZT));
        if (!sens_done)
            hipLaunchKernelGGL(k_theta, tgrid, dim3(TXT * TYT), 0, st, g, sc.sensor_eps, sc.sensor_thr, W, b.sens);
        switch (sc.r) {
        case 1: launch_flaglist<1>(g, b, st); break;
        case 2: launch_flaglist<2>(g, b, st); break;
        case 3: launch_flaglist<3>(g, b, st); break;
        default: launch_flaglist<4>(g, b, st); break;
        }
        return hipGetLastError();
    }
    const long long per = (long long)WB * LPT;
    hipLaunchKernelGGL(k_lists, dim3((unsigned)((g.nint + per - 1) / per)), dim3(WB), 0, st, g, b);
    return hipGetLastError();
}

// Face pass over the flagged faces of the directions in `mask`, then the
// node pass over the listed nodes (persistent grids; list lengths stay on
// the device).
hipError_t launch_weno(const KGrid& g, const KGas& gas, const KScheme& sc, unsigned mask,
                       const double* W, const WenoBufs& b, int mode, double cg, int write_prev,
                       double* out, double* Rp, hipStream_t st)
{
    hipError_t e;
    const bool f32 = sc.precision == SX_FP32_FLUX;
    switch (sc.L) {
    case 1: e = f32 ? launch_faces_L<1, float>(sc.r, g, gas, sc.weno_eps, mask, W, b, st)
                    : launch_faces_L<1, double>(sc.r, g, gas, sc.weno_eps, mask, W, b, st); break;
    case 2: e = f32 ? launch_faces_L<2, float>(sc.r, g, gas, sc.weno_eps, mask, W, b, st)
                    : launch_faces_L<2, double>(sc.r, g, gas, sc.weno_eps, mask, W, b, st); break;
    case 3: e = f32 ? launch_faces_L<3, float>(sc.r, g, gas, sc.weno_eps, mask, W, b, st)
                    : launch_faces_L<3, double>(sc.r, g, gas, sc.weno_eps, mask, W, b, st); break;
    default: e = f32 ? launch_faces_L<4, float>(sc.r, g, gas, sc.weno_eps, mask, W, b, st)
                     : launch_faces_L<4, double>(sc.r, g, gas, sc.weno_eps, mask, W, b, st); break;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_weno_node, dim3(persistent_blocks()), dim3(WB), 0, st, g, mask, b, mode, cg,
                       write_prev, out, Rp);
    return hipGetLastError();
}

}  // namespace sx
