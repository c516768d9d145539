/*
 * sx.h -- C ABI of the MI355X (gfx950) right-hand-side / RK3 library for the
 * compressible Navier-Stokes hot path of STREAmS-2 (Sathyanarayana et al.,
 * "High-speed turbulent flows towards the exascale: STREAmS-2 porting and
 * performance").
 *
 * What is computed (Section 2 of the paper): on a Cartesian grid stretched
 * in y, the right-hand side R = dW/dt of W = (rho, rho u, rho v, rho w, rho E)
 * made of the convective derivatives in x, y, z (skew-symmetric split form
 * cast as face fluxes, hybridised with WENO characteristic fluxes where a
 * modified Ducros sensor flags a face), the Laplacian-form viscous and
 * heat-flux terms, and the third-order low-storage Runge-Kutta update. The
 * kernel names of the paper's Table 2 map onto this library as:
 * euler_{x,y,z}_{central,weno} + visflx + update_flux -> sx_rhs / sx_rk3_step,
 * compute_dt -> sx_compute_dt, compute_residual -> sx_diagnostics.
 *
 * Conventions
 *  - All device pointers are HIP device pointers owned by the caller unless
 *    stated otherwise; the library never frees them.
 *  - Every function returns an sx_status; none aborts or throws. On failure
 *    sx_last_error() describes the cause.
 *  - Calls are asynchronous on the stream given to sx_bind() unless stated.
 *    One handle per stream; a handle is not thread-safe.
 *  - Ghosted state layout (the C form of the Fortran w(x,y,z,v) array of the
 *    paper's Section 3.2): double W[5][pz][py][px], x fastest. Interior node
 *    (i,j,k), 0 <= i < nx etc., of variable v sits at
 *        v*var_stride + (k+ng)*px*py + (j+ng)*px + (i+ox)
 *    with ng ghost layers in every direction; columns [ox-ng, ox) and
 *    [ox+nx, ox+nx+ng) are x ghosts, the rest of a row is padding that is
 *    never read. ox is chosen so interior rows start 128-byte aligned.
 *  - Interior arrays (R, Rprev) are dense double R[5][nz][ny][nx] (the
 *    paper's fln array, no ghosts).
 */
#ifndef SX_H
#define SX_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SX_OK = 0,
    SX_EINVAL = 1,        /* bad argument: order, size, null pointer, layout */
    SX_EUNSUPPORTED = 2,  /* valid request this build does not implement */
    SX_EHIP = 3,          /* HIP runtime error (detail in sx_last_error) */
    SX_ENOMEM = 4,        /* device allocation failed */
    SX_ENONFINITE = 5,    /* diagnostics found non-finite or non-physical state */
    SX_ESTATE = 6         /* call order violated (e.g. step before bind) */
} sx_status;

/* Boundary condition of one face. */
enum {
    SX_BC_PERIODIC = 0,   /* both faces of a direction must be periodic */
    SX_BC_WALL = 1,       /* isothermal no-slip wall by reflection (T_wall) */
    SX_BC_EXTRAP = 2,     /* zeroth-order extrapolation (outflow) */
    SX_BC_FROZEN = 3      /* Dirichlet: ghost cells keep the caller's values */
};

/* y mapping of the uniform index coordinate eta. */
enum {
    SX_Y_UNIFORM = 0,     /* y_j = y0 + j ly/ny */
    SX_Y_TANH2 = 1,       /* two walls at the faces y = -ly/2, +ly/2 */
    SX_Y_TANH1 = 2        /* one wall at the face y = 0, top face y = ly */
};

/* term_mask bits of sx_rhs. */
enum { SX_CONV_X = 1, SX_CONV_Y = 2, SX_CONV_Z = 4, SX_VISC = 8, SX_ALL = 15 };

/* precision of the flux arithmetic (state and RK registers are FP64). */
enum { SX_FP64 = 0, SX_FP32_FLUX = 1 };

/* Central convective flux (Section 2): the skew-symmetric split form, or the
 * optional KEEP-n flux (kinetic-energy and entropy preserving: the
 * entropy-conserving two-point flux with logarithmic means of density and of
 * rho/p, each mean's series cut after keep_n terms). KEEP-n is built for the
 * FP64 path of single blocks with the sensor off and equal convective and
 * viscous orders; other combinations return SX_EUNSUPPORTED. */
enum { SX_FLUX_SPLIT = 0, SX_FLUX_KEEP = 1 };

typedef struct {
    int nx, ny, nz;           /* interior nodes */
    double lx, ly, lz;        /* domain lengths (x, z uniform: dx = lx/nx) */
    double y0;                /* first node of a uniform y grid */
    int ymap;                 /* SX_Y_* */
    double beta;              /* tanh stretching parameter */
    int bc[6];                /* x-lo, x-hi, y-lo, y-hi, z-lo, z-hi: SX_BC_* */
} sx_grid;

typedef struct {
    double gamma;             /* ratio of specific heats */
    double mach;              /* reference Mach number */
    double reynolds;          /* reference Reynolds number */
    double prandtl;
    double visc_exp;          /* mu = T^visc_exp / Re */
    double t_wall;            /* isothermal wall temperature */
    int thermo;               /* 0 calorically perfect; 1 thermally perfect
                                 (Section 2: specific heats from a NASA
                                 polynomial): c_p / R = sum_k nasa[k] theta^k,
                                 k = 0..4, theta = T t_ref in kelvin, R the gas
                                 constant 1/(gamma mach^2) of the reference state;
                                 e(T) = int_0^T c_v, T from e by Newton's method,
                                 heat conductivity mu c_p(T) / Pr. Single blocks,
                                 central split form, sensor off, equal orders;
                                 otherwise SX_EUNSUPPORTED */
    double nasa[5];           /* polynomial coefficients a1..a5 (per kelvin^k) */
    double t_ref;             /* kelvin at T = 1 */
} sx_gas;

typedef struct {
    int central_order;        /* 2, 4, 6, 8 */
    int weno_order;           /* 1, 3, 5, 7 */
    int visc_order;           /* 2, 4, 6, 8 (independent of central_order; the
                                 batched form needs them equal) */
    int sensor;               /* 0 off (pure central), 1 Ducros hybrid; the hybrid
                                 allocates at sx_init the sensor, face flags,
                                 face and node lists and the per-face WENO
                                 flux differences: about 150 bytes per node */
    double sensor_thr;        /* WENO where max sensor over the stencil > thr */
    double sensor_eps;        /* epsilon of the sensor denominator */
    double weno_eps;          /* epsilon of the WENO weights */
    int precision;            /* SX_FP64 or SX_FP32_FLUX */
    int central_flux;         /* SX_FLUX_SPLIT (default) or SX_FLUX_KEEP */
    int keep_n;               /* KEEP-n: terms of the logarithmic-mean series
                                 beyond the first (0..16); < 0 = exact means */
    int bulk_forcing;         /* 1: channel bulk forcing (the paper's force_rhs_1,
                                 Table 2): a uniform streamwise body force set at
                                 every full right-hand side so that the volume
                                 integral of d(rho u)/dt vanishes, its work f u
                                 added to the energy. Single blocks, sensor off;
                                 sx_rhs applies it only with term_mask SX_ALL. */
} sx_scheme;

typedef struct {
    int ng;                   /* ghost layers */
    int ox;                   /* x offset of interior column 0 in a row */
    long long px, py, pz;     /* padded extents: row, plane, volume pitch */
    long long var_stride;     /* doubles between variables (= px*py*pz) */
    long long elems;          /* doubles of one ghosted state (5*var_stride) */
    long long interior;       /* nx*ny*nz */
} sx_layout;

/* Diagnostics (Section 3.2 reductions; cell volume dx * y_eta * dz). */
typedef struct {
    double mass;              /* sum V rho */
    double momentum[3];       /* sum V rho u_i */
    double energy;            /* sum V rho E */
    double kinetic;           /* sum V rho |u|^2 / 2 */
    double max_mach;
    double min_rho;
    double min_p;
    double nonfinite;         /* interior nodes with a non-finite variable */
    double nonphysical;       /* nodes with rho <= 0 or p <= 0 */
    double residual_rhou;     /* sum over nodes of R_rhou^2 (if R given) */
    double weno_fraction[3];  /* fraction of WENO faces per direction */
    double volume;            /* sum V */
} sx_diag;

typedef struct sx_handle sx_handle;

/* Validates the description, computes the y metrics on the host (D1/D2 of
 * the node coordinates, central order) and uploads them. Allocates the
 * library-owned device buffers: metrics and reduction scratch, plus the
 * hybrid scheme's work arrays when the sensor is on (see sx_scheme). On
 * error *out is NULL. SX_EINVAL also when one variable of the ghosted
 * state, or of the interior RK register, would exceed 4 GiB (the kernels
 * address within a variable by 32-bit byte offsets). */
int sx_init(const sx_grid* grid, const sx_gas* gas, const sx_scheme* scheme,
            sx_handle** out);

/* Frees library-owned memory. Safe on NULL. */
void sx_finalize(sx_handle* h);

/* Ghosted layout the caller must allocate (host pointer out). */
int sx_get_layout(const sx_handle* h, sx_layout* out);

/* Binds caller-owned device buffers and a HIP stream (hipStream_t, may be
 * NULL for the default stream): W0 and W1 are two ghosted states of
 * layout.elems doubles (W0 holds the initial state; W1 is the ping-pong
 * partner and receives a copy of W0, ghosts included, so frozen Dirichlet
 * ghosts live in both), Rprev is an interior array of 5*interior doubles
 * (the low-storage RK register). 256-byte alignment is required. */
int sx_bind(sx_handle* h, double* W0, double* W1, double* Rprev, void* stream);

/* Index (0 or 1) of the bound buffer holding the current state. Each RK3
 * step (three substeps) flips it. */
int sx_current(const sx_handle* h, int* which);

/* Fills the ghost layers of a ghosted state in place (periodic copies,
 * wall reflection, extrapolation; frozen faces untouched). */
int sx_fill_ghosts(sx_handle* h, double* W);

/* R = dW/dt of state W restricted to the terms in term_mask (SX_CONV_X,
 * SX_CONV_Y, SX_CONV_Z, SX_VISC). Fills the ghosts of W first (side effect).
 * R is an interior array; W and R must not alias. */
int sx_rhs(sx_handle* h, double* W, double* R, unsigned term_mask);

/* One full RK3 step (three substeps) of the bound state with time step dt:
 * per substep W <- W + dt (gamma_k R(W) + zeta_k Rprev), Rprev <- R(W), with
 * the Wray coefficients gamma = (8/15, 5/12, 3/4), zeta = (0, -17/60, -5/12).
 * Asynchronous; no host synchronisation. */
int sx_rk3_step(sx_handle* h, double dt);

/* CFL time step from the current bound state (synchronises the stream):
 * dt = cfl / max over nodes of sum_d (|u_d|+c)/h_d
 *      + 2 gamma mu/(rho Pr) sum_d 1/h_d^2. */
int sx_compute_dt(sx_handle* h, double cfl, double* dt);

/* Diagnostics of the current bound state (R may be NULL; if given, an
 * interior array whose rho-u component gives residual_rhou). Synchronises
 * the stream. Returns SX_ENONFINITE when nonfinite or nonphysical > 0
 * (the struct is still filled). */
int sx_diagnostics(sx_handle* h, const double* R, sx_diag* out);

/* Face flags of the hybrid scheme supplied by the caller instead of the
 * sensor (parity checks with injected flags; Section 2 hybrid switch).
 * fx: uint8 [nz][ny][nx+1], fy: [nz][ny+1][nx], fz: [nz+1][ny][nx]; entry
 * f of a line is the face between nodes f-1 and f; nonzero = WENO. Host or
 * device pointers; the data is copied (synchronising). Passing three NULLs
 * returns to the sensor. SX_ESTATE if the sensor is off. */
int sx_set_flag_override(sx_handle* h, const unsigned char* fx, const unsigned char* fy,
                         const unsigned char* fz);

/* Face flags of the last hybrid evaluation on this handle (the sensor's, or
 * the injected ones): the switch of Section 2 that selects WENO fluxes on a
 * face. Written by sx_rhs, by every substep of sx_rk3_step (the last one
 * wins) and by sx_diagnostics; all zero before the first. Same layouts as
 * sx_set_flag_override (fx [nz][ny][nx+1], fy [nz][ny+1][nx],
 * fz [nz+1][ny][nx], 1 = WENO); host or device pointers owned by the
 * caller. Synchronises the stream. SX_ESTATE if the sensor is off. */
int sx_get_flags(sx_handle* h, unsigned char* fx, unsigned char* fy, unsigned char* fz);

/* For callers that cannot allocate device memory at call time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the diagnostics of sx_diagnostics, written asynchronously on the bound
 * stream into out, a caller-owned device array of 16 doubles in the field
 * order of sx_diag (mass, momentum[3], energy, kinetic, max_mach, min_rho,
 * min_p, nonfinite, nonphysical, residual_rhou, weno_fraction[3], volume).
 * Same kernels and summation order as sx_diagnostics, so the values are
 * bitwise equal; R as there. Nothing is allocated and nothing synchronises:
 * the reduction partials, per-block result rows and flagged-face counters
 * live in one fixed device array of the library (about 164 KB per GPU,
 * allocated by the HIP runtime with the code object and held until the
 * process ends). Every call on a GPU uses that GPU's array and overwrites
 * what the previous call left there, so calls whose launches overlap on one
 * GPU (different streams, or host threads) race. The status is not checked
 * here: out[9] and out[10] count non-finite and non-physical nodes.
 * SX_EINVAL for a batch handle of more than 256 blocks (the array holds 256
 * result rows) or a null out; SX_ESTATE before sx_bind. */
int sx_diagnostics_noalloc(sx_handle* h, const double* R, double* out);

/* Kernel timing for measurement. When enabled, sx_rk3_step brackets every
 * launch of the fused right-hand-side/update kernel with HIP events recorded
 * on the bound stream. sx_timing_read synchronises the recorded events,
 * returns how many launches were timed and their summed duration in
 * milliseconds, and clears the record. Disabled by default. */
int sx_timing_enable(sx_handle* h, int enable);
int sx_timing_read(sx_handle* h, long long* launches, double* total_ms);

/* ---- Batched form ---------------------------------------------------------
 * Many independent blocks of uneven size advanced together: one persistent
 * launch per RK3 substep works through a list of (block, column tile,
 * z-chunk) work items, and the three substeps of a step are captured in a
 * HIP graph that sx_rk3_step replays. The paper runs one block per GPU; the
 * autotuned work-item shape is the counterpart of its launch-bound and
 * thread-block tuning (Section 4.1, Table 3) and of the per-kernel launch
 * settings its translation tool reads from a configuration file (Section
 * 3.3). Every block follows the single-block equations.
 *
 * Every block must be periodic on all six faces (the kernel writes the
 * periodic ghost images, so no ghost-fill launches sit between substeps),
 * at least twice the ghost width in every direction, and share one scheme
 * (sensor off). A batch handle is used with the generic calls:
 *   sx_get_layout  elems = length of one state arena (doubles); interior =
 *                  length of the RK-register arena / 5 (rounded up);
 *   sx_bind        W0, W1 = state arenas, Rprev = register arena; block b's
 *                  state is the single-block layout of its own size at
 *                  w_offset (sx_get_box), its register [5][nz][ny][nx] at
 *                  r_offset. Ghosts of W0 are filled by the library;
 *   sx_rk3_step    replays the step graph (captured on first use per
 *                  starting buffer, and again after sx_bind/sx_set_tiling;
 *                  dt lives in device memory, so a new dt needs no capture);
 *   sx_rhs         R = register-layout arena, per-block launches;
 *   sx_compute_dt  min over blocks; sx_diagnostics: sums over blocks of the
 *                  sums and counts, max/min over blocks of the extrema.
 * With timing on, each recorded interval spans one whole step (three
 * substep launches) and sx_timing_read counts three launches per step.
 * Returns SX_EUNSUPPORTED for non-periodic blocks, a sensor, unequal
 * convective and viscous orders, or blocks
 * smaller than twice the ghost width; SX_EINVAL for other bad input. */
int sx_init_batch(int nbox, const sx_grid* grids, const sx_gas* gases, const sx_scheme* scheme,
                  sx_handle** out);

/* Layout and arena offsets (doubles) of block `box`. SX_EINVAL for a
 * single-block handle or an index out of range. */
int sx_get_box(const sx_handle* h, int box, sx_layout* lay, long long* w_offset,
               long long* r_offset);

/* Work-item shape of the persistent launch. */
typedef struct {
    int tile_x;               /* column-tile width: 64 or 32 (in: selects shape) */
    int tile_y;               /* column-tile height (out: follows from tile_x) */
    int zchunk;               /* at most this many planes per work item; each
                                 block's z extent is cut into equal chunks */
    int workgroups;           /* persistent workgroups (in: 0 = fill the device) */
    int work_items;           /* out: number of work items */
    double ms_per_substep;    /* out of sx_autotune: measured (or cached) time */
} sx_tiling;

/* Sets / reads the work-item shape (host-synchronous; drops the captured
 * graphs). SX_ESTATE on a single-block handle. */
int sx_set_tiling(sx_handle* h, const sx_tiling* t);
int sx_get_tiling(const sx_handle* h, sx_tiling* t);

/* Picks the work-item shape by timing substep launches over the candidate
 * tile widths and z-chunks, then applies it. With cache_path non-NULL the
 * choice is looked up in (and, after timing, written to) a JSON file keyed
 * by device, precision, order and the multiset of block sizes. Needs bound
 * buffers; the current state is left unchanged, the inactive state buffer
 * and the register arena are overwritten (the next step overwrites both
 * before reading them). Host-synchronous. */
int sx_autotune(sx_handle* h, const char* cache_path, sx_tiling* chosen);

/* Batch handles: 1 (default) replays the captured step graph, 0 launches
 * the three substeps directly. The results are identical. */
int sx_set_graph(sx_handle* h, int enable);

/* Message of the last failing call on this handle ("" if none). */
const char* sx_last_error(const sx_handle* h);

#ifdef __cplusplus
}
#endif
#endif
