// sx_handle.h -- the handle behind the C ABI (internal).
#pragma once

#include <string>
#include <utility>
#include <vector>

#include "sx_internal.h"

// Host-side record of one block of a batch.
struct SxBox {
    sx_grid grid;
    sx_gas gas;
    sx_layout lay;
    sx::KGrid kg;
    sx::KGas kgas;
    long long woff = 0, roff = 0;   // offsets into the state / register arenas
    double* d_metrics = nullptr;
    int kc = 0;                     // z-chunk length of its work items
};

struct sx_handle {
    sx_grid grid;
    sx_gas gas;
    sx_scheme scheme;
    sx_layout lay;
    sx::KGrid kg;
    sx::KGas kgas;
    sx::KScheme ks;
    double* d_metrics = nullptr;  // eta_y, eta_yy, y_eta  (3*ny)
    double* d_scratch = nullptr;  // reduction partials + results
    double* d_force = nullptr;    // bulk forcing: per-workgroup partial sums + force
    // hybrid scheme (sensor on): sensor exceedance, face flags, face and node lists, dF
    sx::WenoBufs wb = {};
    unsigned long long* d_fcount = nullptr;
    int flag_override = 0;
    double* W[2] = {nullptr, nullptr};
    double* Rprev = nullptr;
    hipStream_t st = nullptr;
    int cur = 0;
    bool bound = false;
    bool timing = false;
    int launches_per_interval = 1;   // kernel launches inside one timed interval
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_free;
    std::string err;
    // single block, all faces periodic, no sensor: the fused kernel writes
    // periodic ghost images, so a bound buffer's ghosts stay valid
    bool pimg = false;
    bool ghosts_valid[2] = {false, false};
    // batched form
    bool batch = false;
    std::vector<SxBox> boxes;
    sx::BoxDesc* d_boxes = nullptr;
    sx::TileDesc* d_tiles = nullptr;
    int ntiles = 0, tiles_cap = 0;
    int* d_counter = nullptr;
    double* d_dt = nullptr;                           // device copy of dt
    double dt_set = 0.0;                              // value last written to d_dt
    int variant = 0;                                  // tile shape variant
    int zchunk = 0;                                   // target z-chunk of the work items
    int nwg = 0;                                      // workgroups of the persistent launch
    int cus = 0;
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;                 // capture stream of the step graph
    hipGraphExec_t graph[2] = {nullptr, nullptr};     // one per starting buffer
};

// shared helpers of the API translation units
int sx_fail(sx_handle* h, int code, const char* msg);
int sx_hip_fail(sx_handle* h, hipError_t e, const char* where);
void sx_host_metrics(const sx_grid& g, int L, double* y_eta, double* y_ee);
int sx_validate(const sx_grid& g, const sx_gas& gas, const sx_scheme& s, int* ng_out);
void sx_fill_kernel_params(const sx_grid& g, const sx_gas& gas, const sx_scheme& s, int ng,
                           sx_layout* lay, sx::KGrid* kg, sx::KGas* kgas, sx::KScheme* ks);
hipError_t sx_upload_metrics(const sx_grid& g, int L, double** d_metrics, sx::KGrid* kg);
hipError_t sx_timed_begin(sx_handle* h, std::pair<hipEvent_t, hipEvent_t>* ev);
hipError_t sx_timed_end(sx_handle* h, const std::pair<hipEvent_t, hipEvent_t>& ev);

// batched form (sx_batch.hip)
int sx_batch_bind(sx_handle* h);
int sx_batch_step(sx_handle* h, double dt);
int sx_batch_fill_ghosts(sx_handle* h, double* W);
int sx_batch_rhs(sx_handle* h, double* W, double* R, unsigned mask);
int sx_batch_dt(sx_handle* h, double cfl, double* dt);
int sx_batch_diagnostics(sx_handle* h, const double* R, double* v);
void sx_batch_free(sx_handle* h);
