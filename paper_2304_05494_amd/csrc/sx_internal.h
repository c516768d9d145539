// sx_internal.h -- shared definitions of the HIP library (device + host).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sx.h"

namespace sx {

constexpr int NV = 5;

// Kernel-side description of one grid block. Passed by value.
struct KGrid {
    int nx, ny, nz, ng, ox;
    long long sy, sz, sv;       // strides of y, z and variable (doubles)
    long long base;             // offset of interior node (0,0,0)
    long long nint;             // nx*ny*nz
    int bc[6];
    double dxi, dzi;            // 1/dx, 1/dz
    double dx, dz;
    const double* eta_y;        // [ny] 1 / y_eta
    const double* eta_yy;       // [ny] -y_etaeta / y_eta^3
    const double* y_eta;        // [ny]
    double* fpart;              // bulk forcing: one partial sum per workgroup (nullptr: off)
    unsigned char* sens;        // hybrid step: sensor bytes written by the fused kernel (nullptr: off)
    double sens_eps, sens_thr;  // sensor epsilon and threshold
};

struct KGas {
    double gamma, gm1;          // gamma, gamma - 1
    double gM2;                 // gamma M^2   (T = gM2 p / rho)
    double igM2;                // 1/(gamma M^2)
    double cp;                  // 1/((gamma-1) M^2)
    double s;                   // viscosity exponent
    float sf;                   // s in FP32
    double ire;                 // 1/Re
    double ipr;                 // 1/Pr
    double t_wall;
    double pref;                // reference pressure 1/(gamma M^2) (FP32-flux shift)
    double href;                // reference enthalpy c_p (FP32-flux shift)
    double cvg;                 // 1/((gamma-1) gamma M^2): KEEP-n energy term
    int keep_n;                 // KEEP-n series terms beyond the first (< 0: exact)
    int thermo;                 // 1: thermally perfect gas
    double tcp[5];              // c_p / R_g = sum_k tcp[k] T^k  (NASA a_k t_ref^k)
    double tce[5];              // e / R_g   = sum_k tce[k] T^(k+1)
};

// Thermally perfect gas (gas constant R_g = igM2): c_p / R_g and its
// T-derivative, e / R_g, and T of a specific internal energy by Newton's
// method on e(T) (started from the T = 1 heat capacity, stopped at a
// relative step of 1e-15).
__device__ __forceinline__ double tp_cpR(const KGas& g, double T)
{
    return (((g.tcp[4] * T + g.tcp[3]) * T + g.tcp[2]) * T + g.tcp[1]) * T + g.tcp[0];
}
__device__ __forceinline__ double tp_dcpR(const KGas& g, double T)
{
    return ((4.0 * g.tcp[4] * T + 3.0 * g.tcp[3]) * T + 2.0 * g.tcp[2]) * T + g.tcp[1];
}
__device__ __forceinline__ double tp_eR(const KGas& g, double T)
{
    return ((((g.tce[4] * T + g.tce[3]) * T + g.tce[2]) * T + g.tce[1]) * T + g.tce[0]) * T;
}
__device__ __forceinline__ double tp_T_of_e(const KGas& g, double e)
{
    const double eR = e / g.igM2;
    double T = eR / (tp_cpR(g, 1.0) - 1.0);
    for (int it = 0; it < 100; ++it) {
        const double dT = (tp_eR(g, T) - eR) / (tp_cpR(g, T) - 1.0);
        T -= dT;
        if (fabs(dT) <= 1e-15 * fabs(T)) break;
    }
    return T;
}
// ratio of specific heats at T
__device__ __forceinline__ double tp_gamma(const KGas& g, double T)
{
    if (!g.thermo) return g.gamma;
    const double c = tp_cpR(g, T);
    return c / (c - 1.0);
}

struct KScheme {
    int L;                      // central half-order
    int Lv;                     // viscous half-order
    int r;                      // WENO half-width
    int sensor;
    double sensor_thr, sensor_eps, weno_eps;
    int precision;              // SX_FP64 or SX_FP32_FLUX
    int flux;                   // SX_FLUX_SPLIT or SX_FLUX_KEEP
};

// Central first-derivative weights a_l (D1 f = sum a_l (f_{+l} - f_{-l})) and
// narrow second-derivative weights b_l (D2 f = sum b_l (f_{+l} - 2 f + f_{-l}))
// of order 2S on a unit-spaced grid (Taylor-series stencils).
template <int S> struct Coef;
template <> struct Coef<1> {
    static constexpr double a[2] = {0.0, 0.5};
    static constexpr double b[2] = {0.0, 1.0};
    static constexpr double bsum = b[1];   // sum of the b_l
};
template <> struct Coef<2> {
    static constexpr double a[3] = {0.0, 2.0 / 3.0, -1.0 / 12.0};
    static constexpr double b[3] = {0.0, 4.0 / 3.0, -1.0 / 12.0};
    static constexpr double bsum = b[1] + b[2];   // sum of the b_l
};
template <> struct Coef<3> {
    static constexpr double a[4] = {0.0, 3.0 / 4.0, -3.0 / 20.0, 1.0 / 60.0};
    static constexpr double b[4] = {0.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0};
    static constexpr double bsum = b[1] + b[2] + b[3];   // sum of the b_l
};
template <> struct Coef<4> {
    static constexpr double a[5] = {0.0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};
    static constexpr double b[5] = {0.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
    static constexpr double bsum = b[1] + b[2] + b[3] + b[4];   // sum of the b_l
};

// RK3 (Wray) coefficients of one substep, premultiplied by dt.
struct StepCoef {
    double cg;      // dt * gamma_k
    double cz;      // dt * zeta_k
    int read_prev;  // zeta_k != 0
    int write_prev; // another substep follows
};

// One block of a batch: its grid, gas and offsets into the state arenas.
struct BoxDesc {
    KGrid g;
    KGas gas;
    long long woff;   // offset of the box's ghosted state in a state arena
    long long roff;   // offset of the box's RK register in the register arena
};

// One work item of the persistent batched kernel.
struct TileDesc {
    int box, i0, j0, k0, k1;
};

// ---- host-side launchers (one per translation unit) --------------------
hipError_t launch_ghost_fill(const KGrid& g, const KGas& gas, double* W, hipStream_t st);
hipError_t launch_rhs(const KGrid& g, const KGas& gas, const KScheme& sc, const double* W,
                      double* out, double* Rprev, const StepCoef* step, unsigned mask, bool pimg,
                      hipStream_t st);
// Arguments of one persistent batched launch (one RK3 substep).
struct BatchLaunch {
    const double* Wsrc;
    double* Wdst;
    double* Rp;
    const BoxDesc* boxes;
    const TileDesc* tiles;
    int ntiles;
    int* counter;        // work-queue head, reset by the launch itself
    const double* dt;    // device copy of the time step
    double gk, zk;       // RK3 coefficients gamma_k, zeta_k of the substep
    int substep;
    int nwg;             // workgroups of the persistent grid
};
hipError_t launch_batch(const KScheme& sc, int variant, const BatchLaunch& b, hipStream_t st);
// Slots of the bulk-forcing partial array of a block: one per workgroup of
// any fused launch (tiles of at least 32 x 4 columns, chunks of at least one
// plane), plus the force value.
inline long long force_slots(int nx, int ny, int nz)
{
    return (long long)((nx + 31) / 32) * ((ny + 3) / 4) * nz + 2;
}
hipError_t launch_set_value(double* p, double v, hipStream_t st);
int batch_occupancy(const KScheme& sc, int variant);   // resident workgroups per CU
void batch_tile_shape(const KScheme& sc, int variant, int* tx, int* ty);
hipError_t launch_diagnostics(const KGrid& g, const KGas& gas, const KScheme& sc,
                              const double* W, const double* R, double* scratch,
                              int nscratch_blocks, hipStream_t st);
hipError_t launch_diagnostics_rows(const KGrid& g, const KGas& gas, const double* W, const double* R,
                                   double* part, int nblk, double* res, hipStream_t st);
hipError_t launch_max_rate(const KGrid& g, const KGas& gas, const double* W, double* scratch,
                           int nscratch_blocks, hipStream_t st);
// Buffers of the hybrid (sensor + WENO) path.
struct WenoBufs {
    unsigned char* sens;        // theta > threshold at interior nodes [nz][ny][nx]
    unsigned char* f[3];        // face flags per direction (n_d + 1 faces per line)
    int* flist[3];              // flagged faces per direction (face indices)
    int* nlist;                 // nodes with a flagged face (interior indices)
    unsigned char* nmask;       // flags of each listed node's faces, in node-list order:
                                // bits x-, x+, y-, y+, z-, z+
    int* counts;                // list lengths: faces x, y, z, nodes
    double* dF[3];              // WENO minus central flux per face, [5][faces_d]
};
// sens_done: the sensor bytes were written by the fused kernel of this substep
hipError_t launch_sensor_flags(const KGrid& g, const KScheme& sc, const double* W,
                               const WenoBufs& b, int use_override, int sens_done, hipStream_t st);
hipError_t launch_weno(const KGrid& g, const KGas& gas, const KScheme& sc, unsigned mask,
                       const double* W, const WenoBufs& b, int mode, double cg, int write_prev,
                       double* out, double* Rp, hipStream_t st);
hipError_t launch_count_flags(const KGrid& g, const unsigned char* fx, const unsigned char* fy,
                              const unsigned char* fz, unsigned long long* counts, hipStream_t st);

constexpr int kReduceBlocks = 1024;   // partial-result slots of the reductions
constexpr int kDiagVals = 16;

}  // namespace sx
