// sx_batch.hip -- batched form: many independent periodic blocks advanced by
// one persistent launch per RK3 substep, three substeps captured in a HIP
// graph, and an autotuner for the work-item shape (C ABI in include/sx.h).
//
// State arena: block b's ghosted state (the single-block layout of its own
// size) starts at woff_b in each of the two state buffers; its RK register
// ([5][nz][ny][nx]) starts at roff_b in the register arena. Offsets are
// multiples of 64 doubles, so every block keeps the 128-byte row alignment.
//
// Work items are (block, column tile, z-chunk) triples sorted by decreasing
// cost, pulled from a device counter (longest-processing-time-first list
// scheduling, which bounds the imbalance of uneven blocks). All blocks are
// periodic: the kernel writes the periodic ghost images of every node it
// updates, so substeps need no ghost-fill launches and no block depends on
// another.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "sx_handle.h"

namespace {

constexpr long long kAlign = 64;   // doubles
const double kGk[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
const double kZk[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};

long long align_up(long long v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Destroys the step graphs (after the device has finished any replay).
void drop_graphs(sx_handle* h)
{
    if (h->graph[0] || h->graph[1]) (void)hipDeviceSynchronize();
    for (int b = 0; b < 2; ++b)
        if (h->graph[b]) {
            (void)hipGraphExecDestroy(h->graph[b]);
            h->graph[b] = nullptr;
        }
}

// Builds the work-item list for tile variant v and target chunk zc.
std::vector<sx::TileDesc> make_tiles(const sx_handle* h, int v, int zc)
{
    int tx = 0, ty = 0;
    sx::batch_tile_shape(h->ks, v, &tx, &ty);
    struct Item {
        sx::TileDesc t;
        long long cost;
    };
    std::vector<Item> items;
    const int S = h->ks.L;
    for (int b = 0; b < (int)h->boxes.size(); ++b) {
        const sx_grid& g = h->boxes[b].grid;
        const int nch = (g.nz + zc - 1) / zc;
        const int kc = (g.nz + nch - 1) / nch;
        for (int k0 = 0; k0 < g.nz; k0 += kc)
            for (int j0 = 0; j0 < g.ny; j0 += ty)
                for (int i0 = 0; i0 < g.nx; i0 += tx) {
                    const int k1 = std::min(k0 + kc, g.nz);
                    // plane steps including the 2S-plane prologue, times the tile area
                    const long long cost = (long long)(k1 - k0 + 2 * S) * tx * ty;
                    items.push_back({sx::TileDesc{b, i0, j0, k0, k1}, cost});
                }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const Item& a, const Item& b) { return a.cost > b.cost; });
    std::vector<sx::TileDesc> out;
    out.reserve(items.size());
    for (auto& it : items) out.push_back(it.t);
    return out;
}

int chunk_of(int nz, int zc)
{
    const int nch = (nz + zc - 1) / zc;
    return (nz + nch - 1) / nch;
}

// Uploads a work-item list (host-synchronous) and sizes the launch.
int apply_tiling(sx_handle* h, int v, int zc, int nwg)
{
    const int occ = sx::batch_occupancy(h->ks, v);
    if (occ <= 0) return sx_fail(h, SX_EHIP, "batch: occupancy query failed");
    std::vector<sx::TileDesc> t = make_tiles(h, v, zc);
    if (t.empty()) return sx_fail(h, SX_EINVAL, "batch: no work items");
    hipError_t e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) return sx_hip_fail(h, e, "batch: synchronize");
    if ((int)t.size() > h->tiles_cap) {
        if (h->d_tiles) e = hipFree(h->d_tiles);
        h->d_tiles = nullptr;
        h->tiles_cap = 0;
        if (e == hipSuccess) e = hipMalloc(&h->d_tiles, sizeof(sx::TileDesc) * t.size());
        if (e != hipSuccess) return sx_hip_fail(h, e, "batch: work-item table");
        h->tiles_cap = (int)t.size();
    }
    e = hipMemcpy(h->d_tiles, t.data(), sizeof(sx::TileDesc) * t.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return sx_hip_fail(h, e, "batch: work-item upload");
    h->ntiles = (int)t.size();
    h->variant = v;
    h->zchunk = zc;
    h->nwg = nwg > 0 ? nwg : occ * h->cus;
    for (auto& b : h->boxes) b.kc = chunk_of(b.grid.nz, zc);
    drop_graphs(h);
    return SX_OK;
}

int tile_x_of(const sx_handle* h, int v)
{
    int tx = 0, ty = 0;
    sx::batch_tile_shape(h->ks, v, &tx, &ty);
    return tx;
}

void fill_tiling(const sx_handle* h, sx_tiling* t, double ms)
{
    int tx = 0, ty = 0;
    sx::batch_tile_shape(h->ks, h->variant, &tx, &ty);
    t->tile_x = tx;
    t->tile_y = ty;
    t->zchunk = h->zchunk;
    t->workgroups = h->nwg;
    t->work_items = h->ntiles;
    t->ms_per_substep = ms;
}

hipError_t substep_launch(sx_handle* h, int src, int s, hipStream_t st)
{
    sx::BatchLaunch b;
    b.Wsrc = h->W[src];
    b.Wdst = h->W[1 - src];
    b.Rp = h->Rprev;
    b.boxes = h->d_boxes;
    b.tiles = h->d_tiles;
    b.ntiles = h->ntiles;
    b.counter = h->d_counter;
    b.dt = h->d_dt;
    b.gk = kGk[s];
    b.zk = kZk[s];
    b.substep = s;
    b.nwg = h->nwg;
    return sx::launch_batch(h->ks, h->variant, b, st);
}

// Captures the three substeps starting from buffer `start` into a graph.
int capture(sx_handle* h, int start)
{
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return sx_hip_fail(h, e, "batch: begin capture");
    hipError_t el = hipSuccess;
    for (int s = 0; s < 3 && el == hipSuccess; ++s) el = substep_launch(h, (start + s) & 1, s, h->cap_stream);
    e = hipStreamEndCapture(h->cap_stream, &g);
    if (el != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return sx_hip_fail(h, el, "batch: captured launch");
    }
    if (e != hipSuccess) return sx_hip_fail(h, e, "batch: end capture");
    e = hipGraphInstantiate(&h->graph[start], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        h->graph[start] = nullptr;
        return sx_hip_fail(h, e, "batch: graph instantiate");
    }
    return SX_OK;
}

int set_dt(sx_handle* h, double dt)
{
    if (dt == h->dt_set) return SX_OK;
    hipError_t e = sx::launch_set_value(h->d_dt, dt, h->st);
    if (e != hipSuccess) return sx_hip_fail(h, e, "batch: dt");
    h->dt_set = dt;
    return SX_OK;
}

// ---- autotune cache: one JSON object, one entry per line ----------------
std::string tune_key(const sx_handle* h)
{
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    std::vector<std::string> dims;
    for (auto& b : h->boxes) {
        char buf[64];
        snprintf(buf, sizeof buf, "%dx%dx%d", b.grid.nx, b.grid.ny, b.grid.nz);
        dims.push_back(buf);
    }
    std::sort(dims.begin(), dims.end());
    uint64_t hash = 1469598103934665603ull;   // FNV-1a 64
    for (auto& d : dims) {
        for (char c : d) hash = (hash ^ (unsigned char)c) * 1099511628211ull;
        hash = (hash ^ ';') * 1099511628211ull;
    }
    char key[256];
    snprintf(key, sizeof key, "%s/cu%d/%s/o%d/n%d/%016llx", arch.c_str(), h->cus,
             h->ks.precision == SX_FP32_FLUX ? "fp32flux" : "fp64", 2 * h->ks.L,
             (int)h->boxes.size(), (unsigned long long)hash);
    for (char* c = key; *c; ++c)
        if (*c == '"' || *c == '\\') *c = '_';
    return key;
}

struct TuneEntry {
    int tile_x, zchunk;
    double ms;
};

std::map<std::string, TuneEntry> read_cache(const char* path)
{
    std::map<std::string, TuneEntry> m;
    FILE* f = fopen(path, "r");
    if (!f) return m;
    char line[1024];
    while (fgets(line, sizeof line, f)) {
        const char* q0 = strchr(line, '"');
        if (!q0) continue;
        const char* q1 = strchr(q0 + 1, '"');
        if (!q1) continue;
        TuneEntry e{0, 0, 0.0};
        const char* body = strchr(q1, '{');
        if (!body) continue;
        if (sscanf(body, "{\"tile_x\": %d, \"zchunk\": %d, \"ms_per_substep\": %lf", &e.tile_x,
                   &e.zchunk, &e.ms) == 3)
            m[std::string(q0 + 1, q1)] = e;
    }
    fclose(f);
    return m;
}

bool write_cache(const char* path, const std::map<std::string, TuneEntry>& m)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fprintf(f, "{\n");
    size_t n = 0;
    for (auto& kv : m) {
        fprintf(f, "  \"%s\": {\"tile_x\": %d, \"zchunk\": %d, \"ms_per_substep\": %.6f}%s\n",
                kv.first.c_str(), kv.second.tile_x, kv.second.zchunk, kv.second.ms,
                ++n < m.size() ? "," : "");
    }
    fprintf(f, "}\n");
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path) == 0;
}

}  // namespace

// ---- per-box helpers used by the generic entry points -------------------

int sx_batch_fill_ghosts(sx_handle* h, double* W)
{
    for (auto& b : h->boxes) {
        hipError_t e = sx::launch_ghost_fill(b.kg, b.kgas, W + b.woff, h->st);
        if (e != hipSuccess) return sx_hip_fail(h, e, "sx_fill_ghosts (batch)");
    }
    for (int k = 0; k < 2; ++k)
        if (W == h->W[k]) h->ghosts_valid[k] = true;
    return SX_OK;
}

int sx_batch_bind(sx_handle* h)
{
    const int rc = sx_batch_fill_ghosts(h, h->W[0]);
    if (rc != SX_OK) return rc;
    hipError_t e = hipMemcpyAsync(h->W[1], h->W[0], sizeof(double) * h->lay.elems,
                                  hipMemcpyDeviceToDevice, h->st);
    if (e == hipSuccess) e = hipMemsetAsync(h->Rprev, 0, sizeof(double) * 5 * h->lay.interior, h->st);
    if (e != hipSuccess) return sx_hip_fail(h, e, "sx_bind (batch)");
    h->ghosts_valid[0] = h->ghosts_valid[1] = true;
    h->dt_set = 0.0;  // rewrite dt on the (possibly new) stream
    drop_graphs(h);   // the graphs hold buffer addresses
    return SX_OK;
}

int sx_batch_rhs(sx_handle* h, double* W, double* R, unsigned mask)
{
    for (auto& b : h->boxes) {
        hipError_t e = sx::launch_ghost_fill(b.kg, b.kgas, W + b.woff, h->st);
        if (e == hipSuccess)
            e = sx::launch_rhs(b.kg, b.kgas, h->ks, W + b.woff, R + b.roff, nullptr, nullptr, mask,
                               false, h->st);
        if (e != hipSuccess) return sx_hip_fail(h, e, "sx_rhs (batch)");
    }
    for (int k = 0; k < 2; ++k)
        if (W == h->W[k]) h->ghosts_valid[k] = true;
    return SX_OK;
}

int sx_batch_step(sx_handle* h, double dt)
{
    int rc = SX_OK;
    if (!h->ghosts_valid[h->cur]) rc = sx_batch_fill_ghosts(h, h->W[h->cur]);
    if (rc == SX_OK) rc = set_dt(h, dt);
    if (rc != SX_OK) return rc;
    if (h->use_graph && !h->graph[h->cur]) {
        rc = capture(h, h->cur);
        if (rc != SX_OK) return rc;
    }
    // one timed interval spans the three substep launches
    std::pair<hipEvent_t, hipEvent_t> ev{};
    hipError_t e = hipSuccess;
    if (h->timing) e = sx_timed_begin(h, &ev);
    if (e == hipSuccess) {
        if (h->use_graph) {
            e = hipGraphLaunch(h->graph[h->cur], h->st);
        } else {
            for (int s = 0; s < 3 && e == hipSuccess; ++s) e = substep_launch(h, (h->cur + s) & 1, s, h->st);
        }
    }
    if (e == hipSuccess && h->timing) e = sx_timed_end(h, ev);
    if (e != hipSuccess) return sx_hip_fail(h, e, "sx_rk3_step (batch)");
    h->cur = 1 - h->cur;
    h->ghosts_valid[0] = h->ghosts_valid[1] = true;
    return SX_OK;
}

int sx_batch_dt(sx_handle* h, double cfl, double* dt)
{
    const int nb = sx::kReduceBlocks;
    std::vector<double> rates(h->boxes.size(), 0.0);
    hipError_t e = hipSuccess;
    for (size_t b = 0; b < h->boxes.size() && e == hipSuccess; ++b) {
        const SxBox& x = h->boxes[b];
        e = sx::launch_max_rate(x.kg, x.kgas, h->W[h->cur] + x.woff, h->d_scratch, nb, h->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&rates[b], h->d_scratch + nb, sizeof(double), hipMemcpyDeviceToHost, h->st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) return sx_hip_fail(h, e, "sx_compute_dt (batch)");
    double rate = 0.0;
    for (double r : rates) {
        if (!(r > 0.0) || !isfinite(r)) return sx_fail(h, SX_ENONFINITE, "sx_compute_dt: rate not finite");
        rate = std::max(rate, r);
    }
    *dt = cfl / rate;
    return SX_OK;
}

// Sums, maxima and minima of the per-block diagnostics.
int sx_batch_diagnostics(sx_handle* h, const double* R, double* v)
{
    const int nb = sx::kReduceBlocks, nv = sx::kDiagVals;
    std::vector<double> all(h->boxes.size() * nv, 0.0);
    hipError_t e = hipSuccess;
    for (size_t b = 0; b < h->boxes.size() && e == hipSuccess; ++b) {
        const SxBox& x = h->boxes[b];
        e = sx::launch_diagnostics(x.kg, x.kgas, h->ks, h->W[h->cur] + x.woff, R ? R + x.roff : nullptr,
                                   h->d_scratch, nb, h->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&all[b * nv], h->d_scratch + (long long)nb * nv, sizeof(double) * nv,
                               hipMemcpyDeviceToHost, h->st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) return sx_hip_fail(h, e, "sx_diagnostics (batch)");
    for (int k = 0; k < nv; ++k) v[k] = 0.0;
    v[6] = -INFINITY;
    v[7] = v[8] = INFINITY;
    for (size_t b = 0; b < h->boxes.size(); ++b) {
        const double* a = &all[b * nv];
        for (int k : {0, 1, 2, 3, 4, 5, 9, 10, 11, 15}) v[k] += a[k];
        v[6] = std::max(v[6], a[6]);
        v[7] = std::min(v[7], a[7]);
        v[8] = std::min(v[8], a[8]);
    }
    return SX_OK;
}

void sx_batch_free(sx_handle* h)
{
    drop_graphs(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (void* p : {(void*)h->d_boxes, (void*)h->d_tiles, (void*)h->d_counter, (void*)h->d_dt})
        if (p) (void)hipFree(p);
    for (auto& b : h->boxes)
        if (b.d_metrics) (void)hipFree(b.d_metrics);
    h->boxes.clear();
}

extern "C" {

int sx_init_batch(int nbox, const sx_grid* grids, const sx_gas* gases, const sx_scheme* scheme,
                  sx_handle** out)
{
    if (!out) return SX_EINVAL;
    *out = nullptr;
    if (nbox <= 0 || nbox > (1 << 16) || !grids || !gases || !scheme) return SX_EINVAL;
    if (scheme->sensor) return SX_EUNSUPPORTED;   // the batched form is the central path
    int ng = 0;
    for (int b = 0; b < nbox; ++b) {
        int ngb = 0;
        const int rc = sx_validate(grids[b], gases[b], *scheme, &ngb);
        if (rc != SX_OK) return rc;
        for (int f = 0; f < 6; ++f)
            if (grids[b].bc[f] != SX_BC_PERIODIC) return SX_EUNSUPPORTED;
        if (grids[b].nx < 2 * ngb || grids[b].ny < 2 * ngb || grids[b].nz < 2 * ngb) return SX_EUNSUPPORTED;
        ng = ngb;
    }
    // the persistent kernels are built for equal convective and viscous orders
    // and the split-form flux
    if (scheme->visc_order != scheme->central_order || scheme->central_flux != SX_FLUX_SPLIT ||
        scheme->bulk_forcing)
        return SX_EUNSUPPORTED;
    for (int b = 0; b < nbox; ++b)
        if (gases[b].thermo) return SX_EUNSUPPORTED;
    sx_handle* h = new sx_handle();
    h->batch = true;
    h->scheme = *scheme;
    h->grid = grids[0];
    h->gas = gases[0];
    h->pimg = true;
    h->launches_per_interval = 3;
    sx_fill_kernel_params(grids[0], gases[0], *scheme, ng, &h->lay, &h->kg, &h->kgas, &h->ks);
    long long woff = 0, roff = 0;
    h->boxes.resize(nbox);
    hipError_t e = hipSuccess;
    std::vector<sx::BoxDesc> bd(nbox);
    for (int b = 0; b < nbox && e == hipSuccess; ++b) {
        SxBox& x = h->boxes[b];
        sx::KScheme ks;
        x.grid = grids[b];
        x.gas = gases[b];
        sx_fill_kernel_params(x.grid, x.gas, *scheme, ng, &x.lay, &x.kg, &x.kgas, &ks);
        x.woff = woff;
        x.roff = roff;
        woff = align_up(woff + x.lay.elems);
        roff = align_up(roff + 5 * x.lay.interior);
        e = sx_upload_metrics(x.grid, h->ks.L, &x.d_metrics, &x.kg);
        bd[b] = sx::BoxDesc{x.kg, x.kgas, x.woff, x.roff};
    }
    // arena sizes: elems = state arena (doubles), interior = register arena / 5
    h->lay.px = h->lay.py = h->lay.pz = 0;
    h->lay.var_stride = 0;
    h->lay.elems = woff;
    h->lay.interior = (roff + 4) / 5;
    int dev = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipMalloc(&h->d_scratch, sizeof(double) * (sx::kReduceBlocks + 1) * sx::kDiagVals);
    if (e == hipSuccess) e = hipMalloc(&h->d_boxes, sizeof(sx::BoxDesc) * nbox);
    if (e == hipSuccess) e = hipMemcpy(h->d_boxes, bd.data(), sizeof(sx::BoxDesc) * nbox, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&h->d_counter, 64 * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&h->d_dt, 64 * sizeof(double));
    if (e == hipSuccess) e = hipMemset(h->d_dt, 0, 64 * sizeof(double));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        sx_finalize(h);
        return e == hipErrorOutOfMemory ? SX_ENOMEM : SX_EHIP;
    }
    // default work items: single-block tile, whole z extent per item
    int maxnz = 0;
    for (auto& x : h->boxes) maxnz = std::max(maxnz, x.grid.nz);
    const int rc = apply_tiling(h, 0, maxnz, 0);
    if (rc != SX_OK) {
        sx_finalize(h);
        return rc;
    }
    *out = h;
    return SX_OK;
}

int sx_get_box(const sx_handle* h, int box, sx_layout* lay, long long* w_offset, long long* r_offset)
{
    if (!h || !lay || !w_offset || !r_offset) return SX_EINVAL;
    if (!h->batch || box < 0 || box >= (int)h->boxes.size()) return SX_EINVAL;
    *lay = h->boxes[box].lay;
    *w_offset = h->boxes[box].woff;
    *r_offset = h->boxes[box].roff;
    return SX_OK;
}

int sx_set_tiling(sx_handle* h, const sx_tiling* t)
{
    if (!h || !t) return SX_EINVAL;
    if (!h->batch) return sx_fail(h, SX_ESTATE, "sx_set_tiling: not a batch handle");
    int v = -1;
    for (int c = 0; c < 2; ++c)
        if (tile_x_of(h, c) == t->tile_x) v = c;
    if (v < 0) return sx_fail(h, SX_EINVAL, "sx_set_tiling: unsupported tile_x");
    if (t->zchunk < 1 || t->workgroups < 0) return sx_fail(h, SX_EINVAL, "sx_set_tiling: bad zchunk/workgroups");
    return apply_tiling(h, v, t->zchunk, t->workgroups);
}

int sx_get_tiling(const sx_handle* h, sx_tiling* t)
{
    if (!h || !t) return SX_EINVAL;
    if (!h->batch) return SX_ESTATE;
    fill_tiling(h, t, 0.0);
    return SX_OK;
}

int sx_set_graph(sx_handle* h, int enable)
{
    if (!h) return SX_EINVAL;
    if (!h->batch) return sx_fail(h, SX_ESTATE, "sx_set_graph: not a batch handle");
    h->use_graph = enable != 0;
    return SX_OK;
}

int sx_autotune(sx_handle* h, const char* cache_path, sx_tiling* chosen)
{
    if (!h) return SX_EINVAL;
    if (!h->batch) return sx_fail(h, SX_ESTATE, "sx_autotune: not a batch handle");
    if (!h->bound) return sx_fail(h, SX_ESTATE, "sx_autotune: no buffers bound");
    const std::string key = tune_key(h);
    std::map<std::string, TuneEntry> cache;
    if (cache_path) {
        cache = read_cache(cache_path);
        auto it = cache.find(key);
        if (it != cache.end()) {
            int v = -1;
            for (int c = 0; c < 2; ++c)
                if (tile_x_of(h, c) == it->second.tile_x) v = c;
            if (v >= 0 && it->second.zchunk >= 1) {
                const int rc = apply_tiling(h, v, it->second.zchunk, 0);
                if (rc != SX_OK) return rc;
                if (chosen) fill_tiling(h, chosen, it->second.ms);
                return SX_OK;
            }
        }
    }
    // Candidates are timed on substep 0 from the current buffer: it reads
    // only that buffer and writes the other buffer and the RK register, both
    // of which the next step overwrites before reading.
    int rc = SX_OK;
    if (!h->ghosts_valid[h->cur]) rc = sx_batch_fill_ghosts(h, h->W[h->cur]);
    if (rc == SX_OK) rc = set_dt(h, h->dt_set > 0.0 ? h->dt_set : 1e-6);
    if (rc != SX_OK) return rc;
    int maxnz = 0;
    for (auto& x : h->boxes) maxnz = std::max(maxnz, x.grid.nz);
    std::vector<int> chunks = {16, 24, 32, 48, 64};
    if (maxnz > 64) chunks.push_back(maxnz);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return sx_fail(h, SX_EHIP, "sx_autotune: event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return sx_fail(h, SX_EHIP, "sx_autotune: event");
    }
    double best = INFINITY;
    int bv = 0, bz = maxnz;
    const int reps = 5;
    for (int v = 0; v < 2 && rc == SX_OK; ++v)
        for (int zc : chunks) {
            if (zc > maxnz && zc != chunks.front()) continue;
            rc = apply_tiling(h, v, zc, 0);
            if (rc != SX_OK) break;
            hipError_t e = hipSuccess;
            for (int w = 0; w < 2 && e == hipSuccess; ++w) e = substep_launch(h, h->cur, 0, h->st);
            if (e == hipSuccess) e = hipEventRecord(e0, h->st);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = substep_launch(h, h->cur, 0, h->st);
            if (e == hipSuccess) e = hipEventRecord(e1, h->st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = sx_hip_fail(h, e, "sx_autotune: timing");
                break;
            }
            const double per = ms / reps;
            if (per < best) {
                best = per;
                bv = v;
                bz = zc;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->ghosts_valid[1 - h->cur] = false;
    if (rc != SX_OK) return rc;
    rc = apply_tiling(h, bv, bz, 0);
    if (rc != SX_OK) return rc;
    if (chosen) fill_tiling(h, chosen, best);
    if (cache_path) {
        cache[key] = TuneEntry{tile_x_of(h, bv), bz, best};
        if (!write_cache(cache_path, cache)) return sx_fail(h, SX_EINVAL, "sx_autotune: cannot write cache");
    }
    return SX_OK;
}

}  // extern "C"
