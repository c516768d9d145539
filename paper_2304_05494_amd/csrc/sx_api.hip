// sx_api.hip -- C ABI of the library (declared in include/sx.h).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <utility>
#include <vector>

#include "sx_handle.h"

int sx_fail(sx_handle* h, int code, const char* msg)
{
    if (h) h->err = msg;
    return code;
}

int sx_hip_fail(sx_handle* h, hipError_t e, const char* where)
{
    if (h) {
        char buf[256];
        snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
        h->err = buf;
    }
    return SX_EHIP;
}

namespace {

// y node coordinate of index j (ghost indices continue the mapping).
double y_node(const sx_grid& g, int j)
{
    if (g.ymap == SX_Y_TANH2) {
        const double eta = -1.0 + (2.0 * j + 1.0) / g.ny;
        return 0.5 * g.ly * tanh(g.beta * eta) / tanh(g.beta);
    }
    if (g.ymap == SX_Y_TANH1) {
        const double eta = (j + 0.5) / g.ny;
        return g.ly * (1.0 - tanh(g.beta * (1.0 - eta)) / tanh(g.beta));
    }
    return g.y0 + j * (g.ly / g.ny);
}

bool valid_order(int o) { return o == 2 || o == 4 || o == 6 || o == 8; }


}  // namespace

// Event pair around launches on the bound stream (timing mode).
hipError_t sx_timed_begin(sx_handle* h, std::pair<hipEvent_t, hipEvent_t>* ev)
{
    if (!h->ev_free.empty()) {
        *ev = h->ev_free.back();
        h->ev_free.pop_back();
    } else {
        hipError_t e = hipEventCreate(&ev->first);
        if (e != hipSuccess) return e;
        e = hipEventCreate(&ev->second);
        if (e != hipSuccess) return e;
    }
    return hipEventRecord(ev->first, h->st);
}

hipError_t sx_timed_end(sx_handle* h, const std::pair<hipEvent_t, hipEvent_t>& ev)
{
    h->ev_used.push_back(ev);
    return hipEventRecord(ev.second, h->st);
}

// Host metrics: y_eta = D1(y), y_etaeta = D2(y) with the central stencil of
// half-order L applied to the node coordinates (unit eta spacing).
void sx_host_metrics(const sx_grid& g, int L, double* y_eta, double* y_ee)
{
    static const double A[5][5] = {{0}, {0, 0.5}, {0, 2.0 / 3.0, -1.0 / 12.0},
                                   {0, 0.75, -0.15, 1.0 / 60.0},
                                   {0, 0.8, -0.2, 4.0 / 105.0, -1.0 / 280.0}};
    static const double B[5][5] = {{0}, {0, 1.0}, {0, 4.0 / 3.0, -1.0 / 12.0},
                                   {0, 1.5, -0.15, 1.0 / 90.0},
                                   {0, 1.6, -0.2, 8.0 / 315.0, -1.0 / 560.0}};
    for (int j = 0; j < g.ny; ++j) {
        if (g.ymap == SX_Y_UNIFORM) {
            y_eta[j] = g.ly / g.ny;
            y_ee[j] = 0.0;
            continue;
        }
        const double yc = y_node(g, j);
        double d1 = 0.0, d2 = 0.0;
        for (int l = 1; l <= L; ++l) {
            const double yp = y_node(g, j + l), ym = y_node(g, j - l);
            d1 += A[L][l] * (yp - ym);
            d2 += B[L][l] * ((yp - 2.0 * yc) + ym);
        }
        y_eta[j] = d1;
        y_ee[j] = d2;
    }
}

// Validates one block description; returns SX_OK and the ghost width.
int sx_validate(const sx_grid& g, const sx_gas& gas, const sx_scheme& s, int* ng_out)
{
    if (!valid_order(s.central_order) || !valid_order(s.visc_order)) return SX_EINVAL;
    if (s.weno_order != 1 && s.weno_order != 3 && s.weno_order != 5 && s.weno_order != 7) return SX_EINVAL;
    if (s.sensor != 0 && s.sensor != 1) return SX_EINVAL;
    if (s.precision != SX_FP64 && s.precision != SX_FP32_FLUX) return SX_EINVAL;
    if (s.central_flux != SX_FLUX_SPLIT && s.central_flux != SX_FLUX_KEEP) return SX_EINVAL;
    if (s.central_flux == SX_FLUX_KEEP && s.keep_n > 16) return SX_EINVAL;
    if (s.bulk_forcing != 0 && s.bulk_forcing != 1) return SX_EINVAL;
    if (!(gas.gamma > 1.0) || !(gas.mach > 0.0) || !(gas.reynolds > 0.0) || !(gas.prandtl > 0.0))
        return SX_EINVAL;
    if (gas.thermo != 0 && gas.thermo != 1) return SX_EINVAL;
    if (gas.thermo && !(gas.t_ref > 0.0)) return SX_EINVAL;
    if (!(g.lx > 0.0) || !(g.ly > 0.0) || !(g.lz > 0.0)) return SX_EINVAL;

    if (g.ymap < SX_Y_UNIFORM || g.ymap > SX_Y_TANH1) return SX_EINVAL;
    if (g.ymap != SX_Y_UNIFORM && !(g.beta > 0.0)) return SX_EINVAL;
    const int L = s.central_order / 2, Lv = s.visc_order / 2, r = (s.weno_order + 1) / 2;
    int ng = L > Lv ? L : Lv;
    if (r > ng) ng = r;
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int d = 0; d < 3; ++d) {
        if (n[d] < ng || n[d] > (1 << 20)) return SX_EINVAL;
        for (int sd = 0; sd < 2; ++sd)
            if (g.bc[2 * d + sd] < SX_BC_PERIODIC || g.bc[2 * d + sd] > SX_BC_FROZEN) return SX_EINVAL;
        if ((g.bc[2 * d] == SX_BC_PERIODIC) != (g.bc[2 * d + 1] == SX_BC_PERIODIC)) return SX_EINVAL;
    }
    // the kernels address one variable of the ghosted state, and of the RK
    // register, with 32-bit byte offsets: each must stay below 4 GiB
    const long long px = ((16LL + g.nx + ng + 15) / 16) * 16;
    const long long var_bytes = 8 * px * (g.ny + 2LL * ng) * (g.nz + 2LL * ng);
    const long long int_bytes = 8LL * g.nx * g.ny * g.nz;
    if (var_bytes >= (1LL << 32) || int_bytes >= (1LL << 32)) return SX_EINVAL;
    // thermally perfect gas: central split-form path with one order for
    // convective and viscous terms (WENO eigenvectors and the KEEP-n entropy
    // flux assume a constant gamma)
    if (gas.thermo && (s.sensor || s.central_flux != SX_FLUX_SPLIT || s.visc_order != s.central_order))
        return SX_EUNSUPPORTED;
    // bulk forcing: central path (the force is formed from the fused kernel's sums)
    if (s.bulk_forcing && s.sensor) return SX_EUNSUPPORTED;
    // KEEP-n: FP64, sensor off, one order for convective and viscous terms
    if (s.central_flux == SX_FLUX_KEEP &&
        (s.precision != SX_FP64 || s.sensor || s.visc_order != s.central_order))
        return SX_EUNSUPPORTED;
    *ng_out = ng;
    return SX_OK;
}

void sx_fill_kernel_params(const sx_grid& g, const sx_gas& gas, const sx_scheme& s, int ng,
                           sx_layout* lay, sx::KGrid* kg, sx::KGas* kgas, sx::KScheme* ks)
{
    lay->ng = ng;
    lay->ox = 16;
    lay->px = ((lay->ox + g.nx + ng + 15) / 16) * 16;
    lay->py = g.ny + 2 * ng;
    lay->pz = g.nz + 2 * ng;
    lay->var_stride = lay->px * lay->py * lay->pz;
    lay->elems = 5 * lay->var_stride;
    lay->interior = (long long)g.nx * g.ny * g.nz;

    kg->nx = g.nx;
    kg->ny = g.ny;
    kg->nz = g.nz;
    kg->ng = ng;
    kg->ox = lay->ox;
    kg->sy = lay->px;
    kg->sz = lay->px * lay->py;
    kg->sv = lay->var_stride;
    kg->base = ng * kg->sz + ng * kg->sy + lay->ox;
    kg->nint = lay->interior;
    for (int f = 0; f < 6; ++f) kg->bc[f] = g.bc[f];
    kg->dx = g.lx / g.nx;
    kg->dz = g.lz / g.nz;
    kg->dxi = 1.0 / kg->dx;
    kg->dzi = 1.0 / kg->dz;
    kg->fpart = nullptr;
    kg->sens = nullptr;
    kg->sens_eps = kg->sens_thr = 0.0;

    kgas->gamma = gas.gamma;
    kgas->gm1 = gas.gamma - 1.0;
    kgas->gM2 = gas.gamma * gas.mach * gas.mach;
    kgas->igM2 = 1.0 / kgas->gM2;
    kgas->cp = 1.0 / (kgas->gm1 * gas.mach * gas.mach);
    kgas->s = gas.visc_exp;
    kgas->sf = (float)gas.visc_exp;
    kgas->ire = 1.0 / gas.reynolds;
    kgas->ipr = 1.0 / gas.prandtl;
    kgas->t_wall = gas.t_wall;
    kgas->pref = kgas->igM2;
    kgas->href = kgas->cp;
    kgas->cvg = 1.0 / (kgas->gm1 * kgas->gM2);
    kgas->keep_n = s.central_flux == SX_FLUX_KEEP ? s.keep_n : 0;
    kgas->thermo = gas.thermo;
    {
        double tk = 1.0;
        for (int k = 0; k < 5; ++k) {
            const double a = gas.thermo ? gas.nasa[k] : (k == 0 ? gas.gamma / (gas.gamma - 1.0) : 0.0);
            kgas->tcp[k] = a * tk;
            kgas->tce[k] = (k == 0 ? a - 1.0 : a * tk) / (k + 1);
            tk *= gas.thermo ? gas.t_ref : 1.0;
        }
    }

    ks->L = s.central_order / 2;
    ks->Lv = s.visc_order / 2;
    ks->r = (s.weno_order + 1) / 2;
    ks->sensor = s.sensor;
    ks->sensor_thr = s.sensor_thr;
    ks->sensor_eps = s.sensor_eps;
    ks->weno_eps = s.weno_eps;
    ks->precision = s.precision;
    ks->flux = s.central_flux;
}

// Metrics of one block on the host, uploaded; sets the KGrid pointers.
hipError_t sx_upload_metrics(const sx_grid& g, int L, double** d_metrics, sx::KGrid* kg)
{
    const int ny = g.ny;
    std::vector<double> hm(3 * ny), yee(ny);
    sx_host_metrics(g, L, hm.data() + 2 * ny, yee.data());
    for (int j = 0; j < ny; ++j) {
        const double ye = hm[2 * ny + j];
        hm[j] = 1.0 / ye;
        hm[ny + j] = -yee[j] / (ye * ye * ye);
    }
    hipError_t e = hipMalloc(d_metrics, sizeof(double) * 3 * ny);
    if (e == hipSuccess) e = hipMemcpy(*d_metrics, hm.data(), sizeof(double) * 3 * ny, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        kg->eta_y = *d_metrics;
        kg->eta_yy = *d_metrics + ny;
        kg->y_eta = *d_metrics + 2 * ny;
    }
    return e;
}

extern "C" {

int sx_init(const sx_grid* grid, const sx_gas* gas, const sx_scheme* scheme, sx_handle** out)
{
    if (!out) return SX_EINVAL;
    *out = nullptr;
    if (!grid || !gas || !scheme) return SX_EINVAL;
    const sx_grid& g = *grid;
    const sx_scheme& s = *scheme;
    int ng = 0;
    const int rc = sx_validate(g, *gas, s, &ng);
    if (rc != SX_OK) return rc;

    sx_handle* h = new sx_handle();
    h->grid = g;
    h->gas = *gas;
    h->scheme = s;
    sx_fill_kernel_params(g, *gas, s, ng, &h->lay, &h->kg, &h->kgas, &h->ks);
    if (h->lay.elems >= (1LL << 40)) {
        delete h;
        return SX_EINVAL;
    }
    bool all_periodic = true;
    for (int f = 0; f < 6; ++f) all_periodic = all_periodic && g.bc[f] == SX_BC_PERIODIC;
    h->pimg = all_periodic && !s.sensor && s.visc_order == s.central_order && !s.bulk_forcing &&
              !gas->thermo &&
              s.central_flux == SX_FLUX_SPLIT && g.nx >= 2 * ng && g.ny >= 2 * ng && g.nz >= 2 * ng;

    hipError_t e = sx_upload_metrics(g, h->ks.L, &h->d_metrics, &h->kg);
    if (e == hipSuccess)
        e = hipMalloc(&h->d_scratch, sizeof(double) * (sx::kReduceBlocks + 1) * sx::kDiagVals);
    if (e == hipSuccess && s.bulk_forcing) {
        e = hipMalloc(&h->d_force, sizeof(double) * sx::force_slots(g.nx, g.ny, g.nz));
        h->kg.fpart = h->d_force;
    }
    if (e == hipSuccess && s.sensor) {
        const long long ni = h->lay.interior;
        const long long nf[3] = {(long long)g.nz * g.ny * (g.nx + 1), (long long)g.nz * (g.ny + 1) * g.nx,
                                 (long long)(g.nz + 1) * g.ny * g.nx};
        sx::WenoBufs& b = h->wb;
        e = hipMalloc(&b.sens, (size_t)ni);
        for (int d = 0; d < 3 && e == hipSuccess; ++d) {
            e = hipMalloc(&b.f[d], (size_t)nf[d]);
            if (e == hipSuccess) e = hipMemset(b.f[d], 0, (size_t)nf[d]);
            if (e == hipSuccess) e = hipMalloc(&b.flist[d], sizeof(int) * nf[d]);
            if (e == hipSuccess) e = hipMalloc(&b.dF[d], sizeof(double) * sx::NV * nf[d]);
        }
        if (e == hipSuccess) e = hipMalloc(&b.nlist, sizeof(int) * ni);
        if (e == hipSuccess) e = hipMalloc(&b.nmask, (size_t)ni);
        if (e == hipSuccess) e = hipMalloc(&b.counts, sizeof(int) * 4);
        if (e == hipSuccess) e = hipMalloc(&h->d_fcount, sizeof(unsigned long long) * 3);
    }
    if (e != hipSuccess) {
        sx_finalize(h);
        return e == hipErrorOutOfMemory ? SX_ENOMEM : SX_EHIP;
    }
    *out = h;
    return SX_OK;
}

void sx_finalize(sx_handle* h)
{
    if (!h) return;
    const sx::WenoBufs& b = h->wb;
    for (void* p : {(void*)h->d_metrics, (void*)h->d_scratch, (void*)h->d_force, (void*)b.sens, (void*)b.f[0],
                    (void*)b.f[1], (void*)b.f[2], (void*)b.flist[0], (void*)b.flist[1],
                    (void*)b.flist[2], (void*)b.dF[0], (void*)b.dF[1], (void*)b.dF[2],
                    (void*)b.nlist, (void*)b.nmask, (void*)b.counts, (void*)h->d_fcount})
        if (p) (void)hipFree(p);
    for (auto* v : {&h->ev_used, &h->ev_free})
        for (auto& p : *v) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
    if (h->batch) sx_batch_free(h);
    delete h;
}

int sx_get_layout(const sx_handle* h, sx_layout* out)
{
    if (!h || !out) return SX_EINVAL;
    *out = h->lay;
    return SX_OK;
}

int sx_bind(sx_handle* h, double* W0, double* W1, double* Rprev, void* stream)
{
    if (!h) return SX_EINVAL;
    if (!W0 || !W1 || !Rprev || W0 == W1) return sx_fail(h, SX_EINVAL, "sx_bind: null or aliased buffer");
    if (((uintptr_t)W0 | (uintptr_t)W1 | (uintptr_t)Rprev) & 255)
        return sx_fail(h, SX_EINVAL, "sx_bind: buffers must be 256-byte aligned");
    h->W[0] = W0;
    h->W[1] = W1;
    h->Rprev = Rprev;
    h->st = (hipStream_t)stream;
    h->cur = 0;
    h->ghosts_valid[0] = h->ghosts_valid[1] = false;
    if (h->batch) {
        const int rc = sx_batch_bind(h);
        if (rc == SX_OK) {
            h->bound = true;
            h->err.clear();
        }
        return rc;
    }
    hipError_t e = hipMemcpyAsync(W1, W0, sizeof(double) * h->lay.elems, hipMemcpyDeviceToDevice, h->st);
    if (e == hipSuccess)
        e = hipMemsetAsync(Rprev, 0, sizeof(double) * 5 * h->lay.interior, h->st);
    if (e != hipSuccess) return sx_hip_fail(h, e, "sx_bind");
    h->bound = true;
    h->err.clear();
    return SX_OK;
}

int sx_current(const sx_handle* h, int* which)
{
    if (!h || !which) return SX_EINVAL;
    *which = h->cur;
    return SX_OK;
}

int sx_fill_ghosts(sx_handle* h, double* W)
{
    if (!h) return SX_EINVAL;
    if (!W) return sx_fail(h, SX_EINVAL, "sx_fill_ghosts: null state");
    if (h->batch) return sx_batch_fill_ghosts(h, W);
    hipError_t e = sx::launch_ghost_fill(h->kg, h->kgas, W, h->st);
    if (e != hipSuccess) return sx_hip_fail(h, e, "sx_fill_ghosts");
    for (int b = 0; b < 2; ++b)
        if (W == h->W[b]) h->ghosts_valid[b] = true;
    return SX_OK;
}

int sx_rhs(sx_handle* h, double* W, double* R, unsigned term_mask)
{
    if (!h) return SX_EINVAL;
    if (!W || !R || W == R) return sx_fail(h, SX_EINVAL, "sx_rhs: null or aliased buffer");
    if (term_mask & ~(unsigned)SX_ALL) return sx_fail(h, SX_EINVAL, "sx_rhs: unknown term bits");
    if (h->batch) return sx_batch_rhs(h, W, R, term_mask);
    hipError_t e = sx::launch_ghost_fill(h->kg, h->kgas, W, h->st);
    if (e == hipSuccess)
        e = sx::launch_rhs(h->kg, h->kgas, h->ks, W, R, nullptr, nullptr, term_mask, false, h->st);
    if (e == hipSuccess && h->ks.sensor && (term_mask & (SX_CONV_X | SX_CONV_Y | SX_CONV_Z))) {
        e = sx::launch_sensor_flags(h->kg, h->ks, W, h->wb, h->flag_override, 0, h->st);
        if (e == hipSuccess)
            e = sx::launch_weno(h->kg, h->kgas, h->ks, term_mask, W, h->wb, 0, 0.0, 0, R, nullptr, h->st);
    }
    if (e != hipSuccess) return sx_hip_fail(h, e, "sx_rhs");
    for (int b = 0; b < 2; ++b)
        if (W == h->W[b]) h->ghosts_valid[b] = true;
    return SX_OK;
}

int sx_rk3_step(sx_handle* h, double dt)
{
    static const double gk[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
    static const double zk[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};
    if (!h) return SX_EINVAL;
    if (!h->bound) return sx_fail(h, SX_ESTATE, "sx_rk3_step: no buffers bound");
    if (!(dt > 0.0) || !isfinite(dt)) return sx_fail(h, SX_EINVAL, "sx_rk3_step: dt must be positive");
    if (h->batch) return sx_batch_step(h, dt);
    // hybrid step on the FP64 default scheme: the fused kernel evaluates the
    // sensor of its input state on the way (it holds every plane's
    // velocities), so the separate sensor pass is skipped
    const bool fused_sensor = h->ks.sensor && !h->flag_override && !h->pimg && h->ks.precision == SX_FP64 &&
                              h->ks.flux != SX_FLUX_KEEP && !h->kgas.thermo;
    sx::KGrid kgs = h->kg;
    if (fused_sensor) {
        kgs.sens = h->wb.sens;
        kgs.sens_eps = h->ks.sensor_eps;
        kgs.sens_thr = h->ks.sensor_thr;
    }
    for (int s = 0; s < 3; ++s) {
        double* src = h->W[h->cur];
        double* dst = h->W[1 - h->cur];
        sx::StepCoef sc{dt * gk[s], dt * zk[s], s > 0 ? 1 : 0, s < 2 ? 1 : 0};
        hipError_t e = hipSuccess;
        if (!h->pimg || !h->ghosts_valid[h->cur]) e = sx::launch_ghost_fill(h->kg, h->kgas, src, h->st);
        std::pair<hipEvent_t, hipEvent_t> ev{};
        if (e == hipSuccess && h->timing) e = sx_timed_begin(h, &ev);
        if (e == hipSuccess)
            e = sx::launch_rhs(kgs, h->kgas, h->ks, src, dst, h->Rprev, &sc, SX_ALL, h->pimg, h->st);
        if (e == hipSuccess && h->timing) e = sx_timed_end(h, ev);
        if (e == hipSuccess && h->ks.sensor) {
            e = sx::launch_sensor_flags(h->kg, h->ks, src, h->wb, h->flag_override, fused_sensor, h->st);
            if (e == hipSuccess)
                e = sx::launch_weno(h->kg, h->kgas, h->ks, SX_ALL, src, h->wb, 1, sc.cg, sc.write_prev,
                                    dst, h->Rprev, h->st);
        }
        if (e != hipSuccess) return sx_hip_fail(h, e, "sx_rk3_step");
        h->ghosts_valid[h->cur] = true;
        h->ghosts_valid[1 - h->cur] = h->pimg;
        h->cur = 1 - h->cur;
    }
    return SX_OK;
}

int sx_compute_dt(sx_handle* h, double cfl, double* dt)
{
    if (!h || !dt) return SX_EINVAL;
    if (!h->bound) return sx_fail(h, SX_ESTATE, "sx_compute_dt: no buffers bound");
    if (!(cfl > 0.0)) return sx_fail(h, SX_EINVAL, "sx_compute_dt: cfl must be positive");
    if (h->batch) return sx_batch_dt(h, cfl, dt);
    const int nb = sx::kReduceBlocks;
    double rate = 0.0;
    hipError_t e = sx::launch_max_rate(h->kg, h->kgas, h->W[h->cur], h->d_scratch, nb, h->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&rate, h->d_scratch + nb, sizeof(double), hipMemcpyDeviceToHost, h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) return sx_hip_fail(h, e, "sx_compute_dt");
    if (!(rate > 0.0) || !isfinite(rate)) return sx_fail(h, SX_ENONFINITE, "sx_compute_dt: rate not finite");
    *dt = cfl / rate;
    return SX_OK;
}

int sx_diagnostics(sx_handle* h, const double* R, sx_diag* out)
{
    if (!h || !out) return SX_EINVAL;
    if (!h->bound) return sx_fail(h, SX_ESTATE, "sx_diagnostics: no buffers bound");
    double v[sx::kDiagVals];
    if (h->batch) {
        const int rc = sx_batch_diagnostics(h, R, v);
        if (rc != SX_OK) return rc;
    } else {
        const int nb = sx::kReduceBlocks;
        hipError_t e = sx::launch_diagnostics(h->kg, h->kgas, h->ks, h->W[h->cur], R, h->d_scratch, nb, h->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(v, h->d_scratch + (long long)nb * sx::kDiagVals, sizeof v,
                               hipMemcpyDeviceToHost, h->st);
        unsigned long long fc[3] = {0, 0, 0};
        if (e == hipSuccess && h->ks.sensor) {
            double* Wc = h->W[h->cur];
            e = sx::launch_ghost_fill(h->kg, h->kgas, Wc, h->st);
            if (e == hipSuccess)
                e = sx::launch_sensor_flags(h->kg, h->ks, Wc, h->wb, h->flag_override, 0, h->st);
            if (e == hipSuccess)
                e = sx::launch_count_flags(h->kg, h->wb.f[0], h->wb.f[1], h->wb.f[2], h->d_fcount, h->st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(fc, h->d_fcount, sizeof fc, hipMemcpyDeviceToHost, h->st);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(h->st);
        if (e != hipSuccess) return sx_hip_fail(h, e, "sx_diagnostics");
        if (h->ks.sensor) {
            const sx_grid& g = h->grid;
            v[12] = (double)fc[0] / ((double)g.nz * g.ny * (g.nx + 1));
            v[13] = (double)fc[1] / ((double)g.nz * (g.ny + 1) * g.nx);
            v[14] = (double)fc[2] / ((double)(g.nz + 1) * g.ny * g.nx);
        }
    }
    out->mass = v[0];
    out->momentum[0] = v[1];
    out->momentum[1] = v[2];
    out->momentum[2] = v[3];
    out->energy = v[4];
    out->kinetic = v[5];
    out->max_mach = v[6];
    out->min_rho = v[7];
    out->min_p = v[8];
    out->nonfinite = v[9];
    out->nonphysical = v[10];
    out->residual_rhou = R ? v[11] : 0.0;
    out->weno_fraction[0] = v[12];
    out->weno_fraction[1] = v[13];
    out->weno_fraction[2] = v[14];
    out->volume = v[15];
    if (v[9] > 0.0 || v[10] > 0.0)
        return sx_fail(h, SX_ENONFINITE, "sx_diagnostics: non-finite or non-physical state");
    return SX_OK;
}

int sx_set_flag_override(sx_handle* h, const unsigned char* fx, const unsigned char* fy,
                         const unsigned char* fz)
{
    if (!h) return SX_EINVAL;
    if (!h->ks.sensor || h->batch) return sx_fail(h, SX_ESTATE, "sx_set_flag_override: sensor is off");
    if (!fx && !fy && !fz) {
        h->flag_override = 0;
        return SX_OK;
    }
    if (!fx || !fy || !fz) return sx_fail(h, SX_EINVAL, "sx_set_flag_override: need all three arrays");
    const sx_grid& g = h->grid;
    hipError_t e = hipMemcpyAsync(h->wb.f[0], fx, (size_t)g.nz * g.ny * (g.nx + 1), hipMemcpyDefault, h->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->wb.f[1], fy, (size_t)g.nz * (g.ny + 1) * g.nx, hipMemcpyDefault, h->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->wb.f[2], fz, (size_t)(g.nz + 1) * g.ny * g.nx, hipMemcpyDefault, h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) return sx_hip_fail(h, e, "sx_set_flag_override");
    h->flag_override = 1;
    return SX_OK;
}

int sx_get_flags(sx_handle* h, unsigned char* fx, unsigned char* fy, unsigned char* fz)
{
    if (!h) return SX_EINVAL;
    if (!h->ks.sensor || h->batch) return sx_fail(h, SX_ESTATE, "sx_get_flags: sensor is off");
    if (!fx || !fy || !fz) return sx_fail(h, SX_EINVAL, "sx_get_flags: need all three arrays");
    const sx_grid& g = h->grid;
    hipError_t e = hipMemcpyAsync(fx, h->wb.f[0], (size_t)g.nz * g.ny * (g.nx + 1), hipMemcpyDefault, h->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(fy, h->wb.f[1], (size_t)g.nz * (g.ny + 1) * g.nx, hipMemcpyDefault, h->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(fz, h->wb.f[2], (size_t)(g.nz + 1) * g.ny * g.nx, hipMemcpyDefault, h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) return sx_hip_fail(h, e, "sx_get_flags");
    return SX_OK;
}

int sx_timing_enable(sx_handle* h, int enable)
{
    if (!h) return SX_EINVAL;
    h->timing = enable != 0;
    return SX_OK;
}

int sx_timing_read(sx_handle* h, long long* launches, double* total_ms)
{
    if (!h || !launches || !total_ms) return SX_EINVAL;
    double tot = 0.0;
    for (auto& p : h->ev_used) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(p.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.first, p.second);
        if (e != hipSuccess) return sx_hip_fail(h, e, "sx_timing_read");
        tot += ms;
    }
    *launches = (long long)h->ev_used.size() * h->launches_per_interval;
    *total_ms = tot;
    h->ev_free.insert(h->ev_free.end(), h->ev_used.begin(), h->ev_used.end());
    h->ev_used.clear();
    return SX_OK;
}

const char* sx_last_error(const sx_handle* h)
{
    return h ? h->err.c_str() : "null handle";
}

}  // extern "C"
