// sx_reduce.hip -- deterministic FP64 reductions: diagnostics (the paper's
// compute_residual sum reduction, Table 2) and the CFL rate (compute_dt max
// reduction). Two passes with a fixed point-to-thread assignment and fixed
// tree order, so repeated calls give bitwise-identical results.
#include "sx_internal.h"

namespace sx {

namespace {

constexpr int RB = 256;  // threads per reduction block

enum {
    D_MASS = 0, D_MX, D_MY, D_MZ, D_E, D_KE, D_MACH, D_RMIN, D_PMIN, D_NONFIN, D_NONPHYS,
    D_RES, D_WX, D_WY, D_WZ, D_VOL
};

__device__ __forceinline__ double combine(int q, double a, double b)
{
    if (q == D_MACH) return fmax(a, b);
    if (q == D_RMIN || q == D_PMIN) return fmin(a, b);
    return a + b;
}

__device__ __forceinline__ double neutral(int q)
{
    if (q == D_MACH) return 0.0;
    if (q == D_RMIN || q == D_PMIN) return __builtin_huge_val();
    return 0.0;
}

__global__ void __launch_bounds__(RB) k_diag_partial(KGrid g, KGas gas, const double* __restrict__ W,
                                                     const double* __restrict__ R,
                                                     double* __restrict__ part)
{
    __shared__ double red[kDiagVals][RB];
    double acc[kDiagVals];
#pragma unroll
    for (int q = 0; q < kDiagVals; ++q) acc[q] = neutral(q);
    const long long T = (long long)gridDim.x * RB;
    for (long long m = (long long)blockIdx.x * RB + threadIdx.x; m < g.nint; m += T) {
        const int i = (int)(m % g.nx);
        const long long jk = m / g.nx;
        const int j = (int)(jk % g.ny);
        const int k = (int)(jk / g.ny);
        const long long n = g.base + (long long)k * g.sz + (long long)j * g.sy + i;
        const double vol = g.dx * g.y_eta[j] * g.dz;
        double w[NV];
        bool fin = true;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            w[v] = W[v * g.sv + n];
            fin = fin && isfinite(w[v]);
        }
        acc[D_VOL] += vol;
        if (R) {
            const double r = R[g.nint + m];
            acc[D_RES] += r * r;
        }
        acc[D_MASS] += vol * w[0];
        acc[D_MX] += vol * w[1];
        acc[D_MY] += vol * w[2];
        acc[D_MZ] += vol * w[3];
        acc[D_E] += vol * w[4];
        if (!fin) {
            acc[D_NONFIN] += 1.0;
            continue;
        }
        const double ri = 1.0 / w[0];
        const double u = w[1] * ri, v = w[2] * ri, ww = w[3] * ri;
        const double q2 = u * u + v * v + ww * ww;
        double p, gm = gas.gamma;
        if (gas.thermo) {
            const double T = tp_T_of_e(gas, w[4] * ri - 0.5 * q2);
            p = w[0] * T * gas.igM2;
            gm = tp_gamma(gas, T);
        } else {
            p = gas.gm1 * (w[4] - 0.5 * w[0] * q2);
        }
        acc[D_KE] += vol * (0.5 * w[0] * q2);
        if (!(w[0] > 0.0) || !(p > 0.0)) acc[D_NONPHYS] += 1.0;
        acc[D_RMIN] = fmin(acc[D_RMIN], w[0]);
        acc[D_PMIN] = fmin(acc[D_PMIN], p);
        if (w[0] > 0.0 && p > 0.0) acc[D_MACH] = fmax(acc[D_MACH], sqrt(q2 * w[0] / (gm * p)));
    }
#pragma unroll
    for (int q = 0; q < kDiagVals; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int q = 0; q < kDiagVals; ++q)
                red[q][threadIdx.x] = combine(q, red[q][threadIdx.x], red[q][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x < kDiagVals) part[(long long)blockIdx.x * kDiagVals + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(RB) k_final(const double* __restrict__ part, int nblk, int nvals,
                                              int mode, double* __restrict__ res)
{
    // mode 0: diagnostics combine rules per value; mode 1: max of value 0
    __shared__ double red[RB];
    for (int q = 0; q < nvals; ++q) {
        const int rule = mode == 1 ? D_MACH : q;
        double a = neutral(rule);
        for (int b = threadIdx.x; b < nblk; b += RB) a = combine(rule, a, part[(long long)b * nvals + q]);
        red[threadIdx.x] = a;
        __syncthreads();
        for (int s = RB / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] = combine(rule, red[threadIdx.x], red[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0) res[q] = red[0];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(RB) k_rate_partial(KGrid g, KGas gas, const double* __restrict__ W,
                                                     double* __restrict__ part)
{
    __shared__ double red[RB];
    double a = 0.0;
    const long long T = (long long)gridDim.x * RB;
    for (long long m = (long long)blockIdx.x * RB + threadIdx.x; m < g.nint; m += T) {
        const int i = (int)(m % g.nx);
        const long long jk = m / g.nx;
        const int j = (int)(jk % g.ny);
        const int k = (int)(jk / g.ny);
        const long long n = g.base + (long long)k * g.sz + (long long)j * g.sy + i;
        const double rho = W[n];
        const double ri = 1.0 / rho;
        const double u = W[g.sv + n] * ri, v = W[2 * g.sv + n] * ri, w = W[3 * g.sv + n] * ri;
        double p, T_, gm = gas.gamma;
        if (gas.thermo) {
            T_ = tp_T_of_e(gas, W[4 * g.sv + n] * ri - 0.5 * (u * u + v * v + w * w));
            p = rho * T_ * gas.igM2;
            gm = tp_gamma(gas, T_);
        } else {
            p = gas.gm1 * (W[4 * g.sv + n] - 0.5 * rho * (u * u + v * v + w * w));
            T_ = gas.gM2 * p * ri;
        }
        const double cs = sqrt(gm * p * ri);
        const double mu = pow(T_, gas.s) * gas.ire;
        const double hy = g.y_eta[j];
        const double conv = (fabs(u) + cs) * g.dxi + (fabs(v) + cs) / hy + (fabs(w) + cs) * g.dzi;
        const double visc = 2.0 * gm * mu * ri * gas.ipr *
                            (g.dxi * g.dxi + 1.0 / (hy * hy) + g.dzi * g.dzi);
        a = fmax(a, conv + visc);
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace

// scratch: nblk*kDiagVals partials followed by kDiagVals results.
hipError_t launch_diagnostics(const KGrid& g, const KGas& gas, const KScheme&, const double* W,
                              const double* R, double* scratch, int nblk, hipStream_t st)
{
    hipLaunchKernelGGL(k_diag_partial, dim3(nblk), dim3(RB), 0, st, g, gas, W, R, scratch);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(RB), 0, st, scratch, nblk, kDiagVals, 0,
                       scratch + (long long)nblk * kDiagVals);
    return hipGetLastError();
}

// Partials in part[0 .. nblk*kDiagVals), the kDiagVals results in res.
hipError_t launch_diagnostics_rows(const KGrid& g, const KGas& gas, const double* W, const double* R,
                                   double* part, int nblk, double* res, hipStream_t st)
{
    hipLaunchKernelGGL(k_diag_partial, dim3(nblk), dim3(RB), 0, st, g, gas, W, R, part);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(RB), 0, st, part, nblk, kDiagVals, 0, res);
    return hipGetLastError();
}

// scratch: nblk partials followed by one result (largest CFL rate).
hipError_t launch_max_rate(const KGrid& g, const KGas& gas, const double* W, double* scratch,
                           int nblk, hipStream_t st)
{
    hipLaunchKernelGGL(k_rate_partial, dim3(nblk), dim3(RB), 0, st, g, gas, W, scratch);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(RB), 0, st, scratch, nblk, 1, 1, scratch + nblk);
    return hipGetLastError();
}

}  // namespace sx

// ---- diagnostics without allocation ---------------------------------------
// Scratch of the no-allocation diagnostics: the partial rows of the
// reduction workgroups, one result row per block (up to kNoallocMaxBoxes
// blocks of a batch) and the three flagged-face counters. One copy per
// device, held until the process ends; every call on a device shares it.
#include <mutex>

#include "sx_handle.h"

namespace {
constexpr int kNoallocMaxBoxes = 256;
constexpr long long kNoallocPart = (long long)sx::kReduceBlocks * sx::kDiagVals;
constexpr long long kNoallocRows = kNoallocPart;                                   // result rows
constexpr long long kNoallocCount = kNoallocRows + (long long)kNoallocMaxBoxes * sx::kDiagVals;  // counters
constexpr long long kNoallocDoubles = kNoallocCount + 4;
}  // namespace

static __device__ __align__(256) double scratch[kNoallocDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current. The array's name in host code is only a
// host-side stand-in; kernels get this address.
hipError_t noalloc_scratch(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Single block: the result row, with the flagged-face fractions (sensor
// on) formed from the counters exactly as the synchronising call does.
__global__ void k_emit_single(const double* __restrict__ res, const unsigned long long* __restrict__ fc,
                              int sensor, double nfx, double nfy, double nfz, double* __restrict__ out)
{
    const int q = threadIdx.x;
    if (q >= sx::kDiagVals) return;
    double v = res[q];
    if (sensor) {
        if (q == 12) v = (double)fc[0] / nfx;
        if (q == 13) v = (double)fc[1] / nfy;
        if (q == 14) v = (double)fc[2] / nfz;
    }
    out[q] = v;
}

// Batch: the per-block rows combined in block order with the rules of the
// synchronising call (sums; largest Mach number; smallest density and
// pressure; no flagged faces).
__global__ void k_emit_batch(const double* __restrict__ rows, int nbox, double* __restrict__ out)
{
    if (threadIdx.x != 0) return;
    double v[sx::kDiagVals];
    for (int k = 0; k < sx::kDiagVals; ++k) v[k] = 0.0;
    v[6] = -__builtin_huge_val();
    v[7] = v[8] = __builtin_huge_val();
    for (int b = 0; b < nbox; ++b) {
        const double* a = rows + (long long)b * sx::kDiagVals;
        for (int k = 0; k < sx::kDiagVals; ++k)
            if (k <= 5 || k == 9 || k == 10 || k == 11 || k == 15) v[k] += a[k];
        v[6] = fmax(v[6], a[6]);
        v[7] = fmin(v[7], a[7]);
        v[8] = fmin(v[8], a[8]);
    }
    for (int k = 0; k < sx::kDiagVals; ++k) out[k] = v[k];
}

}  // namespace

extern "C" int sx_diagnostics_noalloc(sx_handle* h, const double* R, double* out)
{
    if (!h) return SX_EINVAL;
    if (!out) return sx_fail(h, SX_EINVAL, "sx_diagnostics_noalloc: null output");
    if (!h->bound) return sx_fail(h, SX_ESTATE, "sx_diagnostics_noalloc: no buffers bound");
    if (h->batch && (int)h->boxes.size() > kNoallocMaxBoxes)
        return sx_fail(h, SX_EINVAL, "sx_diagnostics_noalloc: more blocks than the no-allocation scratch "
                                     "holds result rows for (256)");
    double* s = nullptr;
    hipError_t e = noalloc_scratch(&s);
    if (e != hipSuccess) return sx_hip_fail(h, e, "sx_diagnostics_noalloc: scratch address");
    const int nb = sx::kReduceBlocks, nv = sx::kDiagVals;
    double* part = s;
    double* rows = s + kNoallocRows;
    unsigned long long* fc = reinterpret_cast<unsigned long long*>(s + kNoallocCount);
    if (h->batch) {
        for (size_t b = 0; b < h->boxes.size() && e == hipSuccess; ++b) {
            const SxBox& x = h->boxes[b];
            e = sx::launch_diagnostics_rows(x.kg, x.kgas, h->W[h->cur] + x.woff, R ? R + x.roff : nullptr,
                                            part, nb, rows + (long long)b * nv, h->st);
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_emit_batch, dim3(1), dim3(64), 0, h->st, rows, (int)h->boxes.size(), out);
            e = hipGetLastError();
        }
    } else {
        e = sx::launch_diagnostics_rows(h->kg, h->kgas, h->W[h->cur], R, part, nb, rows, h->st);
        if (e == hipSuccess && h->ks.sensor) {
            double* Wc = h->W[h->cur];
            e = sx::launch_ghost_fill(h->kg, h->kgas, Wc, h->st);
            if (e == hipSuccess)
                e = sx::launch_sensor_flags(h->kg, h->ks, Wc, h->wb, h->flag_override, 0, h->st);
            if (e == hipSuccess)
                e = sx::launch_count_flags(h->kg, h->wb.f[0], h->wb.f[1], h->wb.f[2], fc, h->st);
        }
        if (e == hipSuccess) {
            const sx_grid& g = h->grid;
            hipLaunchKernelGGL(k_emit_single, dim3(1), dim3(64), 0, h->st, rows, fc, h->ks.sensor,
                               (double)g.nz * g.ny * (g.nx + 1), (double)g.nz * (g.ny + 1) * g.nx,
                               (double)(g.nz + 1) * g.ny * g.nx, out);
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) return sx_hip_fail(h, e, "sx_diagnostics_noalloc");
    return SX_OK;
}
