/*
 * oracle.h -- plain FP64 CPU oracle for the STREAmS-2 right-hand side and
 * low-storage RK3 update (Sathyanarayana et al., "High-speed turbulent flows
 * towards the exascale: STREAmS-2 porting and performance", Section 2).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library may include,
 * link or call this. Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py use it. It shares no code, header, table or
 * layout with the HIP path.
 *
 * Array layout (the oracle's own): every field is double[nv][NZ][NY][NX]
 * with NX = nx + 2*ng etc., x fastest, ghost origin at index 0 (interior
 * node i lives at i + ng). Interior-only arrays (R) are [5][nz][ny][nx].
 */
#ifndef ORC_ORACLE_H
#define ORC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_PERIODIC = 0, ORC_BC_WALL = 1, ORC_BC_EXTRAP = 2, ORC_BC_FROZEN = 3 };
enum { ORC_Y_UNIFORM = 0, ORC_Y_TANH2 = 1, ORC_Y_TANH1 = 2 };
enum { ORC_CONV_X = 1, ORC_CONV_Y = 2, ORC_CONV_Z = 4, ORC_VISC = 8, ORC_ALL = 15 };
enum { ORC_NDIAG = 16 };

typedef struct {
    int nx, ny, nz;
    double lx, ly, lz;      /* domain lengths */
    double y0;              /* first y node of a uniform y grid */
    int ymap;               /* ORC_Y_* */
    double beta;            /* tanh stretching parameter */
    int bc[6];              /* x-lo, x-hi, y-lo, y-hi, z-lo, z-hi */
    double gamma, mach, reynolds, prandtl, visc_exp, t_wall;
    int central_order;      /* 2,4,6,8 */
    int weno_order;         /* 1,3,5,7 */
    int visc_order;         /* 2,4,6,8 */
    int sensor;             /* 0 off, 1 Ducros */
    double sensor_thr, sensor_eps, weno_eps;
    int central_flux;       /* 0 split form (Pirozzoli), 1 KEEP-n */
    int keep_n;             /* KEEP-n: terms of the log-mean series beyond
                               the first; < 0 = exact logarithmic means */
    int bulk_forcing;       /* 1: uniform streamwise body force holding the
                               bulk x-momentum fixed (full right-hand side) */
    int thermo;             /* 0 calorically perfect, 1 thermally perfect:
                               c_p / R = sum_k nasa[k] (T t_ref)^k, k = 0..4 */
    double nasa[5];         /* NASA polynomial coefficients a1..a5 (kelvin) */
    double t_ref;           /* reference temperature in kelvin (T = 1) */
} orc_params;

/* Thermally perfect gas at nondimensional temperature T: out = (c_p, c_v,
 * e, dc_p/dT) per unit mass, nondimensional (gas constant 1/(gamma M^2)). */
void   orc_thermo_eval(const orc_params* p, double T, double* out);
/* Temperature of specific internal energy e (Newton on e(T)). */
double orc_thermo_T(const orc_params* p, double e);

int    orc_validate(const orc_params* p);
int    orc_ng(const orc_params* p);
void   orc_y_nodes(const orc_params* p, int jlo, int jhi, double* y);
void   orc_metrics(const orc_params* p, double* y_eta, double* y_etaeta);
void   orc_fill_ghosts(const orc_params* p, double* W);
void   orc_primitives(const orc_params* p, const double* W, double* Q);
void   orc_theta(const orc_params* p, const double* W, double* theta);
void   orc_face_flags(const orc_params* p, const double* theta,
                      unsigned char* fx, unsigned char* fy, unsigned char* fz);
void   orc_rhs(const orc_params* p, double* W, double* R, unsigned mask,
               const unsigned char* fx, const unsigned char* fy,
               const unsigned char* fz);
void   orc_rhs_points(const orc_params* p, double* W, int npts, const int* ijk,
                      double* out, unsigned mask);
void   orc_rk3_step(const orc_params* p, double* W, double* Rprev, double dt);
double orc_compute_dt(const orc_params* p, double* W, double cfl);
void   orc_diagnostics(const orc_params* p, double* W, const double* R,
                       double* out);

int    orc_num_threads(void);
void   orc_set_num_threads(int n);   /* OpenMP threads of later calls */

/* 1-D building blocks exposed for the pin tests. */
void   orc_fd_coeffs(int order, double* a, double* b);
double orc_weno_left(int order, double eps, const double* v);
void   orc_weno_smoothness(int order, const double* v, double* beta);
void   orc_char_basis(double gamma, double un, double ut1, double ut2,
                      double H, double* Rm, double* Lm);
void   orc_face_flux_1d(double gamma, int central_order, int weno_order,
                        double weno_eps, int use_weno, const double* W1d,
                        double* F);

#ifdef __cplusplus
}
#endif
#endif
