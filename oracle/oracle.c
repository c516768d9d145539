/*
 * oracle.c -- plain, slow, FP64 CPU oracle of the STREAmS-2 hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h). Compiled with
 * -O2 -fno-fast-math -ffp-contract=off so every product and sum is rounded
 * exactly as written. Loops are plain; OpenMP only splits k-planes.
 *
 * What it computes follows Section 2 (Numerical Methods) of the paper:
 *  - compressible Navier-Stokes, ideal gas, Cartesian finite differences;
 *  - convective terms in the skew-symmetric split form written as face
 *    fluxes (Pirozzoli 2010, cited there), central order 2..8, or the
 *    optional KEEP-n flux (Tamaki, Kuya and Kawai, cited there);
 *  - WENO reconstruction of characteristic fluxes, projected back on the
 *    right eigenvectors, on faces a modified Ducros sensor flags
 *    (STREAmS-1, cited there);
 *  - viscous terms expanded in Laplacian form, central FD order 2..8;
 *  - optionally, the channel's bulk forcing (a uniform streamwise force
 *    holding the mass flow);
 *  - third-order low-storage Runge-Kutta in time.
 * The paper states these only in words; every concrete formula below is the
 * published method it names or, where the paper is silent, the reading
 * stated at the function.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NV 5

/* ------------------------------------------------------------------ */
/* Central finite-difference coefficients (Section 2: central schemes  */
/* "up to eighth order"). First derivative: D1 f = sum_l a_l (f_{+l} -  */
/* f_{-l}); narrow second derivative: D2 f = b_0 f + sum_l b_l (f_{+l}  */
/* + f_{-l}). Standard Taylor-series central stencils of order 2L.       */
/* ------------------------------------------------------------------ */
static void fd_coeffs(int L, double* a, double* b)
{
    int l;
    for (l = 0; l <= 4; ++l) { a[l] = 0.0; b[l] = 0.0; }
    switch (L) {
    case 1:
        a[1] = 1.0 / 2.0;
        b[0] = -2.0; b[1] = 1.0;
        break;
    case 2:
        a[1] = 2.0 / 3.0; a[2] = -1.0 / 12.0;
        b[0] = -5.0 / 2.0; b[1] = 4.0 / 3.0; b[2] = -1.0 / 12.0;
        break;
    case 3:
        a[1] = 3.0 / 4.0; a[2] = -3.0 / 20.0; a[3] = 1.0 / 60.0;
        b[0] = -49.0 / 18.0; b[1] = 3.0 / 2.0; b[2] = -3.0 / 20.0; b[3] = 1.0 / 90.0;
        break;
    case 4:
        a[1] = 4.0 / 5.0; a[2] = -1.0 / 5.0; a[3] = 4.0 / 105.0; a[4] = -1.0 / 280.0;
        b[0] = -205.0 / 72.0; b[1] = 8.0 / 5.0; b[2] = -1.0 / 5.0;
        b[3] = 8.0 / 315.0; b[4] = -1.0 / 560.0;
        break;
    default:
        break;
    }
}

void orc_fd_coeffs(int order, double* a, double* b) { fd_coeffs(order / 2, a, b); }

/* ------------------------------------------------------------------ */
/* Parameters and ghost width                                          */
/* ------------------------------------------------------------------ */
int orc_ng(const orc_params* p)
{
    int L = p->central_order / 2, Lv = p->visc_order / 2, r = (p->weno_order + 1) / 2;
    int ng = L;
    if (Lv > ng) ng = Lv;
    if (r > ng) ng = r;
    return ng;
}

int orc_validate(const orc_params* p)
{
    int d;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return 1;
    if (p->central_order < 2 || p->central_order > 8 || p->central_order % 2) return 2;
    if (p->visc_order < 2 || p->visc_order > 8 || p->visc_order % 2) return 3;
    if (p->weno_order != 1 && p->weno_order != 3 && p->weno_order != 5 && p->weno_order != 7) return 4;
    if (p->central_flux != 0 && p->central_flux != 1) return 7;
    /* the thermally perfect gas is read for the central path (the WENO     */
    /* eigenvectors and the KEEP-n entropy flux assume a constant gamma)     */
    if (p->thermo && (p->sensor || p->central_flux)) return 8;
    for (d = 0; d < 3; ++d) {
        int n = d == 0 ? p->nx : (d == 1 ? p->ny : p->nz);
        if ((p->bc[2 * d] == ORC_BC_PERIODIC) != (p->bc[2 * d + 1] == ORC_BC_PERIODIC)) return 5;
        if (n < orc_ng(p)) return 6;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Grid and metrics. x and z are uniform; y is mapped from a uniform    */
/* index coordinate eta (spacing 1). Ghost coordinates come from the    */
/* analytic continuation of the mapping. The metric y_eta and y_etaeta  */
/* are the D1 / D2 stencils of the central order applied to the node    */
/* coordinates (discrete metrics of the Grid object, Section 3.1).      */
/* ------------------------------------------------------------------ */
static double y_of_j(const orc_params* p, int j)
{
    double eta;
    switch (p->ymap) {
    case ORC_Y_TANH2:   /* two walls, faces at y = -ly/2 and y = +ly/2 */
        eta = -1.0 + (2.0 * j + 1.0) / (double)p->ny;
        return 0.5 * p->ly * tanh(p->beta * eta) / tanh(p->beta);
    case ORC_Y_TANH1:   /* one wall at y = 0 (face), top face at y = ly */
        eta = (j + 0.5) / (double)p->ny;
        return p->ly * (1.0 - tanh(p->beta * (1.0 - eta)) / tanh(p->beta));
    default:            /* uniform */
        return p->y0 + j * (p->ly / p->ny);
    }
}

void orc_y_nodes(const orc_params* p, int jlo, int jhi, double* y)
{
    int j;
    for (j = jlo; j < jhi; ++j) y[j - jlo] = y_of_j(p, j);
}

void orc_metrics(const orc_params* p, double* y_eta, double* y_etaeta)
{
    int j, l, L = p->central_order / 2;
    double a[5], b[5];
    fd_coeffs(L, a, b);
    for (j = 0; j < p->ny; ++j) {
        if (p->ymap == ORC_Y_UNIFORM) {
            y_eta[j] = p->ly / p->ny;
            y_etaeta[j] = 0.0;
            continue;
        }
        double d1 = 0.0, d2 = 0.0, yj = y_of_j(p, j);
        for (l = 1; l <= L; ++l) {
            d1 += a[l] * (y_of_j(p, j + l) - y_of_j(p, j - l));
            d2 += b[l] * ((y_of_j(p, j + l) - 2.0 * yj) + y_of_j(p, j - l));
        }
        y_eta[j] = d1;
        y_etaeta[j] = d2;
    }
}

/* ------------------------------------------------------------------ */
/* Working context                                                     */
/* ------------------------------------------------------------------ */
typedef struct {
    const orc_params* p;
    int ng, L, Lv, r;
    int NX, NY, NZ;
    long sxyz[3];          /* strides of x, y, z */
    long nvol;
    double dx, dz;
    double* y_eta;         /* ny */
    double* eta_y;         /* ny: 1 / y_eta */
    double* eta_yy;        /* ny: -y_etaeta / y_eta^3 */
    double a[5], b[5];     /* convective central coefficients (order L) */
    double av[5], bv[5];   /* viscous coefficients (order Lv) */
    double* Q;             /* 7 primitive fields over the ghosted box */
    double cp;             /* 1 / ((gamma-1) M^2) */
} ctx;

enum { Q_RHO = 0, Q_U, Q_V, Q_W, Q_P, Q_T, Q_H, NQ };

static long vidx(const ctx* c, int i, int j, int k)
{
    return ((long)(k + c->ng) * c->NY + (j + c->ng)) * c->NX + (i + c->ng);
}

static void ctx_init(ctx* c, const orc_params* p)
{
    int j;
    double* yee;
    c->p = p;
    c->ng = orc_ng(p);
    c->L = p->central_order / 2;
    c->Lv = p->visc_order / 2;
    c->r = (p->weno_order + 1) / 2;
    c->NX = p->nx + 2 * c->ng;
    c->NY = p->ny + 2 * c->ng;
    c->NZ = p->nz + 2 * c->ng;
    c->sxyz[0] = 1;
    c->sxyz[1] = c->NX;
    c->sxyz[2] = (long)c->NX * c->NY;
    c->nvol = (long)c->NX * c->NY * c->NZ;
    c->dx = p->lx / p->nx;
    c->dz = p->lz / p->nz;
    c->y_eta = (double*)malloc(sizeof(double) * p->ny);
    c->eta_y = (double*)malloc(sizeof(double) * p->ny);
    c->eta_yy = (double*)malloc(sizeof(double) * p->ny);
    yee = (double*)malloc(sizeof(double) * p->ny);
    orc_metrics(p, c->y_eta, yee);
    for (j = 0; j < p->ny; ++j) {
        c->eta_y[j] = 1.0 / c->y_eta[j];
        c->eta_yy[j] = -yee[j] / (c->y_eta[j] * c->y_eta[j] * c->y_eta[j]);
    }
    free(yee);
    fd_coeffs(c->L, c->a, c->b);
    fd_coeffs(c->Lv, c->av, c->bv);
    c->Q = NULL;
    c->cp = 1.0 / ((p->gamma - 1.0) * p->mach * p->mach);
}

static void ctx_free(ctx* c)
{
    free(c->y_eta);
    free(c->eta_y);
    free(c->eta_yy);
    free(c->Q);
}

/* ------------------------------------------------------------------ */
/* Equation of state (ideal gas, Section 2), nondimensional with        */
/* reference density, velocity, temperature and length:                */
/*   p = (gamma-1)(rhoE - rho|u|^2/2),  T = gamma M^2 p / rho,          */
/*   H = (rhoE + p) / rho,  c^2 = gamma p / rho = T / M^2,              */
/*   mu = T^s / Re,  k = mu / ((gamma-1) M^2 Pr).                       */
/* ------------------------------------------------------------------ */
/* ------------------------------------------------------------------ */
/* Thermally perfect gas (Section 2, last paragraph: specific heats      */
/* depending on temperature through NASA polynomials, McBride et al.).  */
/* Reading: one 7-coefficient NASA range, c_p / R_g = sum_k a_k theta^k, */
/* k = 0..4, theta = T t_ref the dimensional temperature; the gas stays */
/* thermally ideal, p = rho R_g T with R_g = 1/(gamma M^2) (gamma, M of  */
/* the reference state). Per unit mass, nondimensional:                  */
/*   c_p(T) = R_g P(T),  c_v = c_p - R_g,                                */
/*   e(T) = int_0^T c_v = R_g [(a_0 - 1) T + sum_{k>=1} a_k t_ref^k       */
/*          T^(k+1) / (k+1)],                                              */
/* and T from e by Newton's method on e(T) - e = 0. With a_0 = gamma /    */
/* (gamma - 1) and a_k = 0 otherwise this is the calorically perfect gas. */
/* The heat conductivity is k = mu c_p(T) / Pr.                           */
/* ------------------------------------------------------------------ */
static double rgas(const orc_params* p) { return 1.0 / (p->gamma * p->mach * p->mach); }

void orc_thermo_eval(const orc_params* p, double T, double* out)
{
    double R = rgas(p), th = T * p->t_ref, P = 0.0, dP = 0.0, E = 0.0, tk = 1.0;
    int k;
    for (k = 0; k <= 4; ++k) {
        P += p->nasa[k] * tk;                                  /* theta^k */
        if (k >= 1) dP += k * p->nasa[k] * tk / th * p->t_ref; /* dP/dT */
        tk *= th;
    }
    /* e = R [ (a0-1) T + sum_{k>=1} a_k t_ref^k T^(k+1)/(k+1) ] */
    tk = T;
    for (k = 0; k <= 4; ++k) {
        double a = k == 0 ? p->nasa[0] - 1.0 : p->nasa[k];
        E += a * tk / (k + 1);
        tk *= th;
    }
    out[0] = R * P;
    out[1] = R * (P - 1.0);
    out[2] = R * E;
    out[3] = R * dP;
}

double orc_thermo_T(const orc_params* p, double e)
{
    double f[4], T, dT;
    int it;
    orc_thermo_eval(p, 1.0, f);
    T = e / f[1];
    for (it = 0; it < 100; ++it) {
        orc_thermo_eval(p, T, f);
        dT = (f[2] - e) / f[1];
        T -= dT;
        if (fabs(dT) <= 1e-15 * fabs(T)) break;
    }
    return T;
}

static void cons_to_prim(const orc_params* p, const double w[NV], double q[NQ])
{
    double rho = w[0];
    double u = w[1] / rho, v = w[2] / rho, ww = w[3] / rho;
    double pr, T;
    if (p->thermo) {
        T = orc_thermo_T(p, w[4] / rho - 0.5 * (u * u + v * v + ww * ww));
        pr = rho * T * rgas(p);
    } else {
        pr = (p->gamma - 1.0) * (w[4] - 0.5 * rho * (u * u + v * v + ww * ww));
        T = p->gamma * p->mach * p->mach * pr / rho;
    }
    q[Q_RHO] = rho;
    q[Q_U] = u;
    q[Q_V] = v;
    q[Q_W] = ww;
    q[Q_P] = pr;
    q[Q_T] = T;
    q[Q_H] = (w[4] + pr) / rho;
}

static void prim_to_cons(const orc_params* p, double rho, double u, double v,
                         double w, double pr, double out[NV])
{
    out[0] = rho;
    out[1] = rho * u;
    out[2] = rho * v;
    out[3] = rho * w;
    if (p->thermo) {
        double f[4];
        orc_thermo_eval(p, pr / (rho * rgas(p)), f);
        out[4] = rho * f[2] + 0.5 * rho * (u * u + v * v + w * w);
    } else {
        out[4] = pr / (p->gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
    }
}

/* Ratio of specific heats at a node (gamma, or c_p/c_v of the thermally */
/* perfect gas).                                                         */
static double gamma_at(const orc_params* p, double T)
{
    double f[4];
    if (!p->thermo) return p->gamma;
    orc_thermo_eval(p, T, f);
    return f[0] / f[1];
}

void orc_primitives(const orc_params* p, const double* W, double* Q)
{
    ctx c;
    long n;
    ctx_init(&c, p);
#pragma omp parallel for
    for (n = 0; n < c.nvol; ++n) {
        double w[NV], q[NQ];
        int v;
        for (v = 0; v < NV; ++v) w[v] = W[v * c.nvol + n];
        cons_to_prim(p, w, q);
        for (v = 0; v < NQ; ++v) Q[v * c.nvol + n] = q[v];
    }
    ctx_free(&c);
}

/* ------------------------------------------------------------------ */
/* Ghost fill (the paper states no boundary formulas; the readings     */
/* used are listed below). Directions are filled in the order x, y, z; */
/* each covers the full ghosted extent of the directions filled before */
/* it, so edge and corner ghosts are consistent.                        */
/*  periodic : ghost i = -1-l <- nx-1-l,  i = nx+l <- l                 */
/*  wall     : isothermal no-slip by reflection about the wall face:    */
/*             u,v,w odd, p even, T_g = 2 T_w - T_m, rho from the EOS   */
/*  extrap   : zeroth-order extrapolation (copy of the last interior)   */
/*  frozen   : ghosts left untouched (caller-provided Dirichlet data)   */
/* ------------------------------------------------------------------ */
static void fill_dir(const ctx* c, double* W, int d)
{
    const orc_params* p = c->p;
    int n[3] = {p->nx, p->ny, p->nz};
    int lo[3], hi[3], a, b, l, side, v;
    int ng = c->ng;
    /* ranges of the two other directions */
    for (a = 0; a < 3; ++a) {
        if (a < d) { lo[a] = -ng; hi[a] = n[a] + ng; }
        else { lo[a] = 0; hi[a] = n[a]; }
    }
    int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
    for (side = 0; side < 2; ++side) {
        int bc = p->bc[2 * d + side];
        if (bc == ORC_BC_FROZEN) continue;
        for (a = lo[d2]; a < hi[d2]; ++a)
            for (b = lo[d1]; b < hi[d1]; ++b)
                for (l = 0; l < ng; ++l) {
                    int g[3], m[3];
                    g[d1] = b; g[d2] = a; m[d1] = b; m[d2] = a;
                    if (side == 0) {
                        g[d] = -1 - l;
                        if (bc == ORC_BC_PERIODIC) m[d] = n[d] - 1 - l;
                        else if (bc == ORC_BC_WALL) m[d] = l;
                        else m[d] = 0;
                    } else {
                        g[d] = n[d] + l;
                        if (bc == ORC_BC_PERIODIC) m[d] = l;
                        else if (bc == ORC_BC_WALL) m[d] = n[d] - 1 - l;
                        else m[d] = n[d] - 1;
                    }
                    long gi = vidx(c, g[0], g[1], g[2]);
                    long mi = vidx(c, m[0], m[1], m[2]);
                    if (bc != ORC_BC_WALL) {
                        for (v = 0; v < NV; ++v) W[v * c->nvol + gi] = W[v * c->nvol + mi];
                    } else {
                        double w[NV], q[NQ], o[NV];
                        for (v = 0; v < NV; ++v) w[v] = W[v * c->nvol + mi];
                        cons_to_prim(p, w, q);
                        double Tg = 2.0 * p->t_wall - q[Q_T];
                        double rg = p->gamma * p->mach * p->mach * q[Q_P] / Tg;
                        prim_to_cons(p, rg, -q[Q_U], -q[Q_V], -q[Q_W], q[Q_P], o);
                        for (v = 0; v < NV; ++v) W[v * c->nvol + gi] = o[v];
                    }
                }
    }
}

void orc_fill_ghosts(const orc_params* p, double* W)
{
    ctx c;
    ctx_init(&c, p);
    fill_dir(&c, W, 0);
    fill_dir(&c, W, 1);
    fill_dir(&c, W, 2);
    ctx_free(&c);
}

/* ------------------------------------------------------------------ */
/* Modified Ducros sensor (Section 2; STREAmS-1 reference):             */
/*   theta = max(0, -div u / sqrt(div u^2 + |curl u|^2 + eps^2))        */
/* with second-order central differences. Evaluated at interior nodes;  */
/* a ghost node takes the value of its periodic image, or of its mirror */
/* interior node on a non-periodic side.                                */
/* ------------------------------------------------------------------ */
static double theta_interior(const ctx* c, int i, int j, int k)
{
    const double* Q = c->Q;
    long n = vidx(c, i, j, k), sx = c->sxyz[0], sy = c->sxyz[1], sz = c->sxyz[2];
    const double* U = Q + Q_U * c->nvol;
    const double* V = Q + Q_V * c->nvol;
    const double* Wv = Q + Q_W * c->nvol;
    double ix = 0.5 / c->dx, iy = 0.5 * c->eta_y[j], iz = 0.5 / c->dz;
    double ux = (U[n + sx] - U[n - sx]) * ix, uy = (U[n + sy] - U[n - sy]) * iy, uz = (U[n + sz] - U[n - sz]) * iz;
    double vx = (V[n + sx] - V[n - sx]) * ix, vy = (V[n + sy] - V[n - sy]) * iy, vz = (V[n + sz] - V[n - sz]) * iz;
    double wx = (Wv[n + sx] - Wv[n - sx]) * ix, wy = (Wv[n + sy] - Wv[n - sy]) * iy, wz = (Wv[n + sz] - Wv[n - sz]) * iz;
    double div = ux + vy + wz;
    double o1 = wy - vz, o2 = uz - wx, o3 = vx - uy;
    double om2 = o1 * o1 + o2 * o2 + o3 * o3;
    double eps = c->p->sensor_eps;
    double t = -div / sqrt(div * div + om2 + eps * eps);
    return t > 0.0 ? t : 0.0;
}

static int map_ghost(int i, int n, int bc_lo, int bc_hi)
{
    if (i < 0) return bc_lo == ORC_BC_PERIODIC ? i + n : -1 - i;
    if (i >= n) return bc_hi == ORC_BC_PERIODIC ? i - n : 2 * n - 1 - i;
    return i;
}

static void theta_field(const ctx* c, double* theta)
{
    const orc_params* p = c->p;
    int k;
    double* tin = (double*)malloc(sizeof(double) * (long)p->nx * p->ny * p->nz);
#pragma omp parallel for
    for (k = 0; k < p->nz; ++k) {
        int i, j;
        for (j = 0; j < p->ny; ++j)
            for (i = 0; i < p->nx; ++i)
                tin[((long)k * p->ny + j) * p->nx + i] = theta_interior(c, i, j, k);
    }
#pragma omp parallel for
    for (k = -c->ng; k < p->nz + c->ng; ++k) {
        int i, j;
        for (j = -c->ng; j < p->ny + c->ng; ++j)
            for (i = -c->ng; i < p->nx + c->ng; ++i) {
                int mi = map_ghost(i, p->nx, p->bc[0], p->bc[1]);
                int mj = map_ghost(j, p->ny, p->bc[2], p->bc[3]);
                int mk = map_ghost(k, p->nz, p->bc[4], p->bc[5]);
                theta[vidx(c, i, j, k)] = tin[((long)mk * p->ny + mj) * p->nx + mi];
            }
    }
    free(tin);
}

void orc_theta(const orc_params* p, const double* W, double* theta)
{
    ctx c;
    ctx_init(&c, p);
    c.Q = (double*)malloc(sizeof(double) * NQ * c.nvol);
    orc_primitives(p, W, c.Q);
    theta_field(&c, theta);
    ctx_free(&c);
}

/* Face i+1/2 along d uses WENO iff the largest theta over the nodes of
 * its WENO stencil (i-r+1 .. i+r) exceeds the threshold. Face arrays hold
 * n_d + 1 faces per line: entry f is the face between nodes f-1 and f. */
static unsigned char flag_of_face(const ctx* c, const double* theta, int d, int i, int j, int k)
{
    int t;
    long n = vidx(c, i, j, k), s = c->sxyz[d];
    double m = 0.0;
    for (t = -c->r + 1; t <= c->r; ++t) {
        double th = theta[n + t * s];
        if (th > m) m = th;
    }
    return m > c->p->sensor_thr ? 1 : 0;
}

void orc_face_flags(const orc_params* p, const double* theta,
                    unsigned char* fx, unsigned char* fy, unsigned char* fz)
{
    ctx c;
    int i, j, k;
    ctx_init(&c, p);
    for (k = 0; k < p->nz; ++k)
        for (j = 0; j < p->ny; ++j)
            for (i = -1; i < p->nx; ++i)
                fx[((long)k * p->ny + j) * (p->nx + 1) + i + 1] =
                    p->sensor ? flag_of_face(&c, theta, 0, i, j, k) : 0;
    for (k = 0; k < p->nz; ++k)
        for (j = -1; j < p->ny; ++j)
            for (i = 0; i < p->nx; ++i)
                fy[((long)k * (p->ny + 1) + j + 1) * p->nx + i] =
                    p->sensor ? flag_of_face(&c, theta, 1, i, j, k) : 0;
    for (k = -1; k < p->nz; ++k)
        for (j = 0; j < p->ny; ++j)
            for (i = 0; i < p->nx; ++i)
                fz[((long)(k + 1) * p->ny + j) * p->nx + i] =
                    p->sensor ? flag_of_face(&c, theta, 2, i, j, k) : 0;
    ctx_free(&c);
}

/* ------------------------------------------------------------------ */
/* Central face flux in the skew-symmetric split form (Pirozzoli 2010)  */
/* of order 2L, face between node n and node n+s:                       */
/*   F^phi = sum_l 2 a_l sum_{m<l} 1/8 (rho_A+rho_B)(ud_A+ud_B)(phi_A+phi_B) */
/*   with A = n - m s, B = n + (l-m) s, phi in {1, u, v, w, H};         */
/*   pressure: P = sum_l 2 a_l sum_{m<l} 1/2 (p_A + p_B) in d-momentum. */
/* ------------------------------------------------------------------ */
static void central_flux_line(int L, const double* a, int d,
                              const double* rho, const double* u, const double* v,
                              const double* w, const double* pr, const double* H,
                              long n, long s, double F[NV])
{
    int l, m, q;
    const double* ud = d == 0 ? u : (d == 1 ? v : w);
    double P = 0.0;
    for (q = 0; q < NV; ++q) F[q] = 0.0;
    for (l = 1; l <= L; ++l) {
        double cl = 2.0 * a[l];
        for (m = 0; m < l; ++m) {
            long A = n - m * s, B = n + (l - m) * s;
            double mf = 0.125 * (rho[A] + rho[B]) * (ud[A] + ud[B]);
            F[0] += cl * (mf * 2.0);
            F[1] += cl * (mf * (u[A] + u[B]));
            F[2] += cl * (mf * (v[A] + v[B]));
            F[3] += cl * (mf * (w[A] + w[B]));
            F[4] += cl * (mf * (H[A] + H[B]));
            P += cl * (0.5 * (pr[A] + pr[B]));
        }
    }
    F[1 + d] += P;
}

/* ------------------------------------------------------------------ */
/* KEEP-n central flux (Section 2: the optional kinetic-energy and      */
/* entropy preserving scheme of Tamaki, Kuya and Kawai). Reading: the    */
/* two-point flux that conserves the entropy rho s / (gamma - 1), with   */
/* s = ln p - gamma ln rho, and is kinetic-energy preserving (momentum   */
/* flux = mass flux times the mean velocity plus the mean pressure):      */
/*   F_rho = rho_ln  (ud_A + ud_B)/2                                       */
/*   F_mom = F_rho   (u_A + u_B)/2 + (p_A + p_B)/2 e_d                     */
/*   F_E   = F_rho ( 1 / ((gamma-1) b_ln) + (u_A.u_B)/2 )                  */
/*           + (p_A ud_B + p_B ud_A)/2,            b = rho / p,            */
/* where x_ln = (x_B - x_A)/(ln x_B - ln x_A) is the logarithmic mean. The */
/* "n" of KEEP-n: 1/x_ln = 2/(x_A+x_B) * sum_m xi^(2m)/(2m+1), xi =        */
/* (x_B-x_A)/(x_B+x_A), cut after the terms m = 0..n (n < 0: the exact     */
/* mean). Used in the same high-order form as the split flux:              */
/*   F_{i+1/2} = sum_l 2 a_l sum_{m<l} F(node n - m s, node n + (l-m) s).   */
/* ------------------------------------------------------------------ */
static double inv_log_mean(double xa, double xb, int nterms)
{
    double sum = xa + xb, xi = (xb - xa) / sum, x2 = xi * xi, t = 1.0, S = 0.0;
    int m;
    if (nterms < 0) {
        if (fabs(xi) >= 0.1) return (log(xb) - log(xa)) / (xb - xa);
        nterms = 16;   /* xi^34/35 < 1e-35: exact to rounding */
    }
    for (m = 0; m <= nterms; ++m) {
        S += t / (2.0 * m + 1.0);
        t *= x2;
    }
    return 2.0 / sum * S;
}

static void keep_pair_flux(const orc_params* p, int d, const double* qa, const double* qb,
                           double F[NV])
{
    double uda = qa[Q_U + d], udb = qb[Q_U + d];
    double frho = 0.5 * (uda + udb) / inv_log_mean(qa[Q_RHO], qb[Q_RHO], p->keep_n);
    double ba = qa[Q_RHO] / qa[Q_P], bb = qb[Q_RHO] / qb[Q_P];
    double uu = qa[Q_U] * qb[Q_U] + qa[Q_V] * qb[Q_V] + qa[Q_W] * qb[Q_W];
    double K = inv_log_mean(ba, bb, p->keep_n) / (p->gamma - 1.0) + 0.5 * uu;
    F[0] = frho;
    F[1] = frho * 0.5 * (qa[Q_U] + qb[Q_U]);
    F[2] = frho * 0.5 * (qa[Q_V] + qb[Q_V]);
    F[3] = frho * 0.5 * (qa[Q_W] + qb[Q_W]);
    F[1 + d] += 0.5 * (qa[Q_P] + qb[Q_P]);
    F[4] = frho * K + 0.5 * (qa[Q_P] * udb + qb[Q_P] * uda);
}

/* KEEP-n face flux between node n and node n+s (primitive field Q with  */
/* variable stride nvol).                                                */
static void keep_flux_line(const orc_params* p, int L, const double* a, int d, const double* Q,
                           long nvol, long n, long s, double F[NV])
{
    int l, m, q, v;
    for (q = 0; q < NV; ++q) F[q] = 0.0;
    for (l = 1; l <= L; ++l) {
        double cl = 2.0 * a[l];
        for (m = 0; m < l; ++m) {
            long A = n - m * s, B = n + (l - m) * s;
            double qa[NQ], qb[NQ], f[NV];
            for (v = 0; v < NQ; ++v) {
                qa[v] = Q[v * nvol + A];
                qb[v] = Q[v * nvol + B];
            }
            keep_pair_flux(p, d, qa, qb, f);
            for (q = 0; q < NV; ++q) F[q] += cl * f[q];
        }
    }
}

/* ------------------------------------------------------------------ */
/* WENO characteristic flux (Section 2): characteristic fluxes are      */
/* reconstructed with WENO and projected back on the right eigenvectors */
/* of the Euler equations. Textbook pieces used:                        */
/*  - Roe average of the two nodes adjacent to the face;                */
/*  - eigenvectors of the Euler flux Jacobian (e.g. Toro, ch. 3) in the */
/*    basis (rho, rho u_n, rho u_t1, rho u_t2, rho E);                   */
/*  - local Lax-Friedrichs splitting per characteristic field, lambda_k */
/*    = max over the stencil nodes of |eigenvalue k|;                    */
/*  - Jiang-Shu WENO of order 2r-1 (r = 1, 2, 3), and for the paper's   */
/*    "up to seventh order" the Balsara-Shu scheme (r = 4).             */
/* ------------------------------------------------------------------ */
/* Smoothness indicators of the r candidate stencils (Jiang-Shu: the sum
 * over derivative orders l = 1..r-1 of the integral over the reconstruction
 * cell of h^(2l-1) (d^l p_k / dx^l)^2, p_k the stencil's reconstruction
 * polynomial). v holds v_{i-r+1} .. v_{i+r-1}. Order 7 is the Balsara-Shu
 * scheme; its indicators are written as sums of squares of the cubic's
 * derivatives (the same quadratic forms as the published ones with
 * denominator 240, without their cancellation on smooth data). */
static void weno_smoothness(int order, const double* v, double* beta)
{
    double t;
    if (order == 3) {
        double vm = v[0], v0 = v[1], vp = v[2];
        beta[0] = (v0 - vm) * (v0 - vm);
        beta[1] = (vp - v0) * (vp - v0);
    } else if (order == 5) {
        double vmm = v[0], vm = v[1], v0 = v[2], vp = v[3], vpp = v[4];
        t = vmm - 2.0 * vm + v0; beta[0] = 13.0 / 12.0 * t * t;
        t = vmm - 4.0 * vm + 3.0 * v0; beta[0] += 0.25 * t * t;
        t = vm - 2.0 * v0 + vp; beta[1] = 13.0 / 12.0 * t * t;
        t = vm - vp; beta[1] += 0.25 * t * t;
        t = v0 - 2.0 * vp + vpp; beta[2] = 13.0 / 12.0 * t * t;
        t = 3.0 * v0 - 4.0 * vp + vpp; beta[2] += 0.25 * t * t;
    } else if (order == 7) {
        /* beta_k = s1^2 + 13/3 s2^2 + 781/20 s3^2 with s1 = p' + p'''/24,
         * s2 = p''/2 and s3 = p'''/6 at the centre of the reconstruction
         * cell of stencil k's cubic p (unit spacing) */
        int k;
        static const double S1[4][4] = {{-2.0, 9.0, -18.0, 11.0}, {1.0, -6.0, 3.0, 2.0},
                                        {-2.0, -3.0, 6.0, -1.0}, {-11.0, 18.0, -9.0, 2.0}};
        static const double S2[4][4] = {{-1.0, 4.0, -5.0, 2.0}, {0.0, 1.0, -2.0, 1.0},
                                        {1.0, -2.0, 1.0, 0.0}, {2.0, -5.0, 4.0, -1.0}};
        for (k = 0; k < 4; ++k) {
            const double* w = v + k;
            double s1 = (S1[k][0] * w[0] + S1[k][1] * w[1] + S1[k][2] * w[2] + S1[k][3] * w[3]) / 6.0;
            double s2 = (S2[k][0] * w[0] + S2[k][1] * w[1] + S2[k][2] * w[2] + S2[k][3] * w[3]) / 2.0;
            double s3 = (-w[0] + 3.0 * w[1] - 3.0 * w[2] + w[3]) / 6.0;
            beta[k] = s1 * s1 + 13.0 / 3.0 * s2 * s2 + 781.0 / 20.0 * s3 * s3;
        }
    }
}

void orc_weno_smoothness(int order, const double* v, double* beta) { weno_smoothness(order, v, beta); }

double orc_weno_left(int order, double eps, const double* v)
{
    /* v holds the 2r-1 values v_{i-r+1} .. v_{i+r-1}; returns v at i+1/2 */
    double b[4];
    if (order == 1) return v[0];
    weno_smoothness(order, v, b);
    if (order == 3) {
        double vm = v[0], v0 = v[1], vp = v[2];
        double q0 = 0.5 * (-vm + 3.0 * v0);
        double q1 = 0.5 * (v0 + vp);
        double a0 = (1.0 / 3.0) / ((eps + b[0]) * (eps + b[0]));
        double a1 = (2.0 / 3.0) / ((eps + b[1]) * (eps + b[1]));
        return (a0 * q0 + a1 * q1) / (a0 + a1);
    }
    if (order == 5) {
        double vmm = v[0], vm = v[1], v0 = v[2], vp = v[3], vpp = v[4];
        double q0 = (2.0 * vmm - 7.0 * vm + 11.0 * v0) / 6.0;
        double q1 = (-vm + 5.0 * v0 + 2.0 * vp) / 6.0;
        double q2 = (2.0 * v0 + 5.0 * vp - vpp) / 6.0;
        double a0 = 0.1 / ((eps + b[0]) * (eps + b[0]));
        double a1 = 0.6 / ((eps + b[1]) * (eps + b[1]));
        double a2 = 0.3 / ((eps + b[2]) * (eps + b[2]));
        return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
    }
    {
        /* order 7: four cubic candidates, linear weights (1, 12, 18, 4)/35 */
        double q0 = (-3.0 * v[0] + 13.0 * v[1] - 23.0 * v[2] + 25.0 * v[3]) / 12.0;
        double q1 = (v[1] - 5.0 * v[2] + 13.0 * v[3] + 3.0 * v[4]) / 12.0;
        double q2 = (-v[2] + 7.0 * v[3] + 7.0 * v[4] - v[5]) / 12.0;
        double q3 = (3.0 * v[3] + 13.0 * v[4] - 5.0 * v[5] + v[6]) / 12.0;
        double a0 = (1.0 / 35.0) / ((eps + b[0]) * (eps + b[0]));
        double a1 = (12.0 / 35.0) / ((eps + b[1]) * (eps + b[1]));
        double a2 = (18.0 / 35.0) / ((eps + b[2]) * (eps + b[2]));
        double a3 = (4.0 / 35.0) / ((eps + b[3]) * (eps + b[3]));
        return (a0 * q0 + a1 * q1 + a2 * q2 + a3 * q3) / (a0 + a1 + a2 + a3);
    }
}

/* Right (columns) and left (rows) eigenvectors, row-major 5x5:
 * Rm[row*5+col], column k is eigenvector k for eigenvalue
 * (un-c, un, un, un, un+c); Lm = Rm^{-1} written out analytically. */
void orc_char_basis(double gamma, double un, double ut1, double ut2,
                    double H, double* Rm, double* Lm)
{
    double q2 = un * un + ut1 * ut1 + ut2 * ut2;
    double c = sqrt((gamma - 1.0) * (H - 0.5 * q2));
    double b1 = (gamma - 1.0) / (c * c);
    double b2 = 0.5 * q2 * b1;
    double R[5][5] = {
        {1.0, 0.0, 0.0, 1.0, 1.0},
        {un - c, 0.0, 0.0, un, un + c},
        {ut1, 1.0, 0.0, ut1, ut1},
        {ut2, 0.0, 1.0, ut2, ut2},
        {H - un * c, ut1, ut2, 0.5 * q2, H + un * c}};
    double Lx[5][5] = {
        {0.5 * (b2 + un / c), 0.5 * (-b1 * un - 1.0 / c), -0.5 * b1 * ut1, -0.5 * b1 * ut2, 0.5 * b1},
        {-ut1, 0.0, 1.0, 0.0, 0.0},
        {-ut2, 0.0, 0.0, 1.0, 0.0},
        {1.0 - b2, b1 * un, b1 * ut1, b1 * ut2, -b1},
        {0.5 * (b2 - un / c), 0.5 * (-b1 * un + 1.0 / c), -0.5 * b1 * ut1, -0.5 * b1 * ut2, 0.5 * b1}};
    int i, j;
    for (i = 0; i < 5; ++i)
        for (j = 0; j < 5; ++j) {
            Rm[i * 5 + j] = R[i][j];
            Lm[i * 5 + j] = Lx[i][j];
        }
}

/* Face flux between nodes n and n+s along d from WENO of characteristic
 * fluxes. Wn[t][v], qn[t][*] hold conserved states and primitives at the
 * 2r stencil nodes t = 0 .. 2r-1 (node n-r+1+t); conserved vectors are
 * permuted to (rho, rho u_d, rho u_d+1, rho u_d+2, rho E). */
static void weno_flux_nodes(double gamma, int order, double eps, int r, int d,
                            double Wn[8][NV], double qn[8][NQ], double F[NV])
{
    int perm[NV] = {0, 1 + d, 1 + (d + 1) % 3, 1 + (d + 2) % 3, 4};
    int iu[3] = {Q_U + d, Q_U + (d + 1) % 3, Q_U + (d + 2) % 3};
    int A = r - 1, B = r; /* positions of the two face-adjacent nodes */
    double sa = sqrt(qn[A][Q_RHO]), sb = sqrt(qn[B][Q_RHO]);
    double un = (sa * qn[A][iu[0]] + sb * qn[B][iu[0]]) / (sa + sb);
    double ut1 = (sa * qn[A][iu[1]] + sb * qn[B][iu[1]]) / (sa + sb);
    double ut2 = (sa * qn[A][iu[2]] + sb * qn[B][iu[2]]) / (sa + sb);
    double Hb = (sa * qn[A][Q_H] + sb * qn[B][Q_H]) / (sa + sb);
    double Rm[25], Lm[25];
    double g[8][NV], qc[8][NV], lam[NV];
    double gp[8][NV], gm[8][NV];
    double Fc[NV];
    int t, k, v, m;
    orc_char_basis(gamma, un, ut1, ut2, Hb, Rm, Lm);
    for (k = 0; k < NV; ++k) lam[k] = 0.0;
    for (t = 0; t < 2 * r; ++t) {
        double wp[NV], fp[NV];
        double unt = qn[t][iu[0]];
        double ct = sqrt(gamma * qn[t][Q_P] / qn[t][Q_RHO]);
        double ev[NV] = {fabs(unt - ct), fabs(unt), fabs(unt), fabs(unt), fabs(unt + ct)};
        for (v = 0; v < NV; ++v) wp[v] = Wn[t][perm[v]];
        /* physical flux along d, permuted basis */
        fp[0] = wp[0] * unt;
        fp[1] = wp[1] * unt + qn[t][Q_P];
        fp[2] = wp[2] * unt;
        fp[3] = wp[3] * unt;
        fp[4] = (wp[4] + qn[t][Q_P]) * unt;
        for (k = 0; k < NV; ++k) {
            double sg = 0.0, sq = 0.0;
            for (m = 0; m < NV; ++m) {
                sg += Lm[k * 5 + m] * fp[m];
                sq += Lm[k * 5 + m] * wp[m];
            }
            g[t][k] = sg;
            qc[t][k] = sq;
            if (ev[k] > lam[k]) lam[k] = ev[k];
        }
    }
    for (t = 0; t < 2 * r; ++t)
        for (k = 0; k < NV; ++k) {
            gp[t][k] = 0.5 * (g[t][k] + lam[k] * qc[t][k]);
            gm[t][k] = 0.5 * (g[t][k] - lam[k] * qc[t][k]);
        }
    for (k = 0; k < NV; ++k) {
        double vl[7], vr[7];
        /* g+ : nodes i-r+1 .. i+r-1 (positions 0 .. 2r-2) */
        for (t = 0; t < 2 * r - 1; ++t) vl[t] = gp[t][k];
        /* g- : mirrored, nodes i+r .. i-r+2 (positions 2r-1 .. 1) */
        for (t = 0; t < 2 * r - 1; ++t) vr[t] = gm[2 * r - 1 - t][k];
        Fc[k] = orc_weno_left(order, eps, vl) + orc_weno_left(order, eps, vr);
    }
    for (v = 0; v < NV; ++v) {
        double s = 0.0;
        for (k = 0; k < NV; ++k) s += Rm[v * 5 + k] * Fc[k];
        F[perm[v]] = s;
    }
}

void orc_face_flux_1d(double gamma, int central_order, int weno_order,
                      double weno_eps, int use_weno, const double* W1d, double* F)
{
    /* W1d: 8 conserved states (x direction), face between entries 3 and 4 */
    orc_params p;
    double q[8][NQ];
    int t, v;
    memset(&p, 0, sizeof(p));
    p.gamma = gamma;
    p.mach = 1.0;
    for (t = 0; t < 8; ++t) cons_to_prim(&p, W1d + t * NV, q[t]);
    if (!use_weno) {
        double rho[8], u[8], vv[8], w[8], pr[8], H[8], a[5], b[5];
        for (t = 0; t < 8; ++t) {
            rho[t] = q[t][Q_RHO]; u[t] = q[t][Q_U]; vv[t] = q[t][Q_V];
            w[t] = q[t][Q_W]; pr[t] = q[t][Q_P]; H[t] = q[t][Q_H];
        }
        fd_coeffs(central_order / 2, a, b);
        central_flux_line(central_order / 2, a, 0, rho, u, vv, w, pr, H, 3, 1, F);
    } else {
        int r = (weno_order + 1) / 2;
        double Wn[8][NV], qn[8][NQ];
        for (t = 0; t < 2 * r; ++t) {
            int src = 3 - r + 1 + t;
            for (v = 0; v < NV; ++v) Wn[t][v] = W1d[src * NV + v];
            for (v = 0; v < NQ; ++v) qn[t][v] = q[src][v];
        }
        weno_flux_nodes(gamma, weno_order, weno_eps, r, 0, Wn, qn, F);
    }
}

/* Face flux of the hybrid scheme for the face between n and n+s. */
static void face_flux(const ctx* c, const double* W, int d, long n, int use_weno, double F[NV])
{
    const double* Q = c->Q;
    long s = c->sxyz[d];
    if (!use_weno && c->p->central_flux == 1) {
        keep_flux_line(c->p, c->L, c->a, d, Q, c->nvol, n, s, F);
    } else if (!use_weno) {
        central_flux_line(c->L, c->a, d, Q + Q_RHO * c->nvol, Q + Q_U * c->nvol,
                          Q + Q_V * c->nvol, Q + Q_W * c->nvol, Q + Q_P * c->nvol,
                          Q + Q_H * c->nvol, n, s, F);
    } else {
        double Wn[8][NV], qn[8][NQ];
        int t, v;
        for (t = 0; t < 2 * c->r; ++t) {
            long m = n + (t - c->r + 1) * s;
            for (v = 0; v < NV; ++v) Wn[t][v] = W[v * c->nvol + m];
            for (v = 0; v < NQ; ++v) qn[t][v] = Q[v * c->nvol + m];
        }
        weno_flux_nodes(c->p->gamma, c->p->weno_order, c->p->weno_eps, c->r, d, Wn, qn, F);
    }
}

/* ------------------------------------------------------------------ */
/* Viscous terms in Laplacian form (Section 2), central FD of order 2Lv. */
/* With Theta = div u, mu and k already holding 1/Re:                    */
/*   V_i = mu (lap u_i + 1/3 d_i Theta) + d_j mu (d_j u_i + d_i u_j)     */
/*         - 2/3 d_i mu Theta                                            */
/*   V_E = u_i V_i + tau_ij d_j u_i + k lap T + d_j k d_j T              */
/*   tau_ij = mu (d_j u_i + d_i u_j - 2/3 delta_ij Theta)               */
/* d_i Theta = narrow D2_ii u_i + sum_{j!=i} D_i(D_j u_j);              */
/* grad mu = s mu/T grad T and grad k = s k/T grad T (chain rule of the  */
/* power law). y-derivatives: d/dy = eta_y D_eta,                        */
/* d2/dy2 = eta_y^2 D2_eta + eta_yy D_eta.                               */
/* ------------------------------------------------------------------ */
static double d1v(const ctx* c, const double* f, long n, int d, int j)
{
    int l;
    long s = c->sxyz[d];
    double acc = 0.0;
    for (l = 1; l <= c->Lv; ++l) acc += c->av[l] * (f[n + l * s] - f[n - l * s]);
    if (d == 0) return acc / c->dx;
    if (d == 1) return c->eta_y[j] * acc;
    return acc / c->dz;
}

static double d2v(const ctx* c, const double* f, long n, int d, int j)
{
    int l;
    long s = c->sxyz[d];
    /* b_0 = -2 sum_l b_l, so D2 f = sum_l b_l (f_{+l} - 2 f + f_{-l});
     * this form is exactly zero on a constant field. */
    double acc = 0.0;
    for (l = 1; l <= c->Lv; ++l) acc += c->bv[l] * ((f[n + l * s] - 2.0 * f[n]) + f[n - l * s]);
    if (d == 0) return acc / (c->dx * c->dx);
    if (d == 2) return acc / (c->dz * c->dz);
    {
        double a1 = 0.0;
        for (l = 1; l <= c->Lv; ++l) a1 += c->av[l] * (f[n + l * s] - f[n - l * s]);
        return c->eta_y[j] * c->eta_y[j] * acc + c->eta_yy[j] * a1;
    }
}

/* D_o (D_in f) at node n (interior row j): outer direction o, inner in. */
static double dmixed(const ctx* c, const double* f, long n, int o, int in, int j)
{
    int l;
    long s = c->sxyz[o];
    double acc = 0.0;
    for (l = 1; l <= c->Lv; ++l) {
        int jp = o == 1 ? j + l : j, jm = o == 1 ? j - l : j;
        acc += c->av[l] * (d1v(c, f, n + l * s, in, jp) - d1v(c, f, n - l * s, in, jm));
    }
    if (o == 0) return acc / c->dx;
    if (o == 1) return c->eta_y[j] * acc;
    return acc / c->dz;
}

static void viscous_point(const ctx* c, long n, int j, double Vout[NV])
{
    const orc_params* p = c->p;
    const double* u[3] = {c->Q + Q_U * c->nvol, c->Q + Q_V * c->nvol, c->Q + Q_W * c->nvol};
    const double* T = c->Q + Q_T * c->nvol;
    double g[3][3], gT[3], lap[3], lapT = 0.0, dth[3], theta = 0.0;
    int a, b;
    double Tc = T[n];
    double mu = pow(Tc, p->visc_exp) / p->reynolds;
    double kc = mu * c->cp / p->prandtl, kT = 0.0;   /* kT = (dk/dT) / k beyond s/T */
    if (p->thermo) {
        double f[4];
        orc_thermo_eval(p, Tc, f);
        kc = mu * f[0] / p->prandtl;
        kT = f[3] / f[0];
    }
    double dmu[3], dk[3];
    for (a = 0; a < 3; ++a) {          /* g[a][b] = d_b u_a */
        for (b = 0; b < 3; ++b) g[a][b] = d1v(c, u[a], n, b, j);
        gT[a] = d1v(c, T, n, a, j);
    }
    for (a = 0; a < 3; ++a) {
        lap[a] = 0.0;
        for (b = 0; b < 3; ++b) lap[a] += d2v(c, u[a], n, b, j);
        lapT += d2v(c, T, n, a, j);
        theta += g[a][a];
    }
    for (a = 0; a < 3; ++a) {
        dth[a] = d2v(c, u[a], n, a, j);
        for (b = 0; b < 3; ++b)
            if (b != a) dth[a] += dmixed(c, u[b], n, a, b, j);
        dmu[a] = p->visc_exp * mu / Tc * gT[a];
        dk[a] = (p->visc_exp * kc / Tc + kc * kT) * gT[a];
    }
    double VE = 0.0;
    for (a = 0; a < 3; ++a) {
        double Va = mu * (lap[a] + dth[a] / 3.0);
        for (b = 0; b < 3; ++b) Va += dmu[b] * (g[a][b] + g[b][a]);
        Va -= 2.0 / 3.0 * dmu[a] * theta;
        Vout[1 + a] = Va;
        VE += u[a][n] * Va;
    }
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b) {
            double tau = mu * (g[a][b] + g[b][a] - (a == b ? 2.0 / 3.0 * theta : 0.0));
            VE += tau * g[a][b];
        }
    VE += kc * lapT;
    for (a = 0; a < 3; ++a) VE += dk[a] * gT[a];
    Vout[0] = 0.0;
    Vout[4] = VE;
}

/* ------------------------------------------------------------------ */
/* Right-hand side R = dW/dt = -(C_x + C_y + C_z) + V at one interior    */
/* node. C_d = (F_{i+1/2} - F_{i-1/2}) / dx (x, z) or * eta_y (y).       */
/* ------------------------------------------------------------------ */
typedef struct {
    const unsigned char* f[3];
} flagset;

static int face_flag(const ctx* c, const flagset* fs, int d, int i, int j, int k)
{
    /* face d+1/2 after node (i,j,k) along d; indices may be -1 on d */
    const orc_params* p = c->p;
    if (!fs->f[d]) return 0;
    if (d == 0) return fs->f[0][((long)k * p->ny + j) * (p->nx + 1) + i + 1];
    if (d == 1) return fs->f[1][((long)k * (p->ny + 1) + j + 1) * p->nx + i];
    return fs->f[2][((long)(k + 1) * p->ny + j) * p->nx + i];
}

static void rhs_point(const ctx* c, const double* W, const flagset* fs, unsigned mask,
                      int i, int j, int k, double Rout[NV])
{
    long n = vidx(c, i, j, k);
    int d, v;
    for (v = 0; v < NV; ++v) Rout[v] = 0.0;
    for (d = 0; d < 3; ++d) {
        double Fp[NV], Fm[NV], sc;
        int im = d == 0 ? i - 1 : i, jm = d == 1 ? j - 1 : j, km = d == 2 ? k - 1 : k;
        if (!(mask & (1u << d))) continue;
        face_flux(c, W, d, n, face_flag(c, fs, d, i, j, k), Fp);
        face_flux(c, W, d, n - c->sxyz[d], face_flag(c, fs, d, im, jm, km), Fm);
        sc = d == 0 ? 1.0 / c->dx : (d == 1 ? c->eta_y[j] : 1.0 / c->dz);
        for (v = 0; v < NV; ++v) Rout[v] -= sc * (Fp[v] - Fm[v]);
    }
    if (mask & ORC_VISC) {
        double V[NV];
        viscous_point(c, n, j, V);
        for (v = 1; v < NV; ++v) Rout[v] += V[v];
    }
}

/* Prepare primitives and (if the sensor is on and no override) flags. */
static void prepare(ctx* c, double* W, flagset* fs, unsigned char** own,
                    const unsigned char* fx, const unsigned char* fy, const unsigned char* fz)
{
    const orc_params* p = c->p;
    orc_fill_ghosts(p, W);
    c->Q = (double*)malloc(sizeof(double) * NQ * c->nvol);
    orc_primitives(p, W, c->Q);
    own[0] = own[1] = own[2] = NULL;
    if (fx || fy || fz) {
        fs->f[0] = fx; fs->f[1] = fy; fs->f[2] = fz;
    } else if (p->sensor) {
        double* th = (double*)malloc(sizeof(double) * c->nvol);
        theta_field(c, th);
        own[0] = (unsigned char*)malloc((long)p->nz * p->ny * (p->nx + 1));
        own[1] = (unsigned char*)malloc((long)p->nz * (p->ny + 1) * p->nx);
        own[2] = (unsigned char*)malloc((long)(p->nz + 1) * p->ny * p->nx);
        orc_face_flags(p, th, own[0], own[1], own[2]);
        free(th);
        fs->f[0] = own[0]; fs->f[1] = own[1]; fs->f[2] = own[2];
    } else {
        fs->f[0] = fs->f[1] = fs->f[2] = NULL;
    }
}

static double pairwise(const double* x, long n);

/* ------------------------------------------------------------------ */
/* Bulk forcing of the channel (the paper's force_rhs_1, a sum          */
/* reduction, Table 2). Reading: a spatially uniform streamwise body    */
/* force f, set at every evaluation of the full right-hand side so that */
/* the volume integral of the x-momentum right-hand side vanishes (the  */
/* bulk momentum, hence the mass flow, stays fixed):                     */
/*   f = - sum V R_rhou / sum V,  R_rhou += f,  R_rhoE += f u,           */
/* with the force's work f u at every node and V = dx y_eta dz.           */
/* ------------------------------------------------------------------ */
static void bulk_force(const ctx* c, double* R)
{
    const orc_params* p = c->p;
    long nint = (long)p->nx * p->ny * p->nz, m;
    double* t = (double*)malloc(sizeof(double) * nint);
    double* vol = (double*)malloc(sizeof(double) * nint);
    double f;
    int i, j, k;
    for (k = 0; k < p->nz; ++k)
        for (j = 0; j < p->ny; ++j)
            for (i = 0; i < p->nx; ++i) {
                m = ((long)k * p->ny + j) * p->nx + i;
                vol[m] = c->dx * c->y_eta[j] * c->dz;
                t[m] = vol[m] * R[1 * nint + m];
            }
    f = -pairwise(t, nint) / pairwise(vol, nint);
    for (k = 0; k < p->nz; ++k)
        for (j = 0; j < p->ny; ++j)
            for (i = 0; i < p->nx; ++i) {
                m = ((long)k * p->ny + j) * p->nx + i;
                R[1 * nint + m] += f;
                R[4 * nint + m] += f * c->Q[Q_U * c->nvol + vidx(c, i, j, k)];
            }
    free(t);
    free(vol);
}

void orc_rhs(const orc_params* p, double* W, double* R, unsigned mask,
             const unsigned char* fx, const unsigned char* fy, const unsigned char* fz)
{
    ctx c;
    flagset fs;
    unsigned char* own[3];
    int k;
    long nint = (long)p->nx * p->ny * p->nz;
    ctx_init(&c, p);
    prepare(&c, W, &fs, own, fx, fy, fz);
#pragma omp parallel for schedule(dynamic)
    for (k = 0; k < p->nz; ++k) {
        int i, j, v;
        for (j = 0; j < p->ny; ++j)
            for (i = 0; i < p->nx; ++i) {
                double Rp[NV];
                rhs_point(&c, W, &fs, mask, i, j, k, Rp);
                for (v = 0; v < NV; ++v) R[v * nint + ((long)k * p->ny + j) * p->nx + i] = Rp[v];
            }
    }
    if (p->bulk_forcing && mask == ORC_ALL) bulk_force(&c, R);
    free(own[0]); free(own[1]); free(own[2]);
    ctx_free(&c);
}

void orc_rhs_points(const orc_params* p, double* W, int npts, const int* ijk,
                    double* out, unsigned mask)
{
    ctx c;
    flagset fs;
    unsigned char* own[3];
    int t;
    ctx_init(&c, p);
    prepare(&c, W, &fs, own, NULL, NULL, NULL);
#pragma omp parallel for
    for (t = 0; t < npts; ++t)
        rhs_point(&c, W, &fs, mask, ijk[3 * t], ijk[3 * t + 1], ijk[3 * t + 2], out + NV * t);
    free(own[0]); free(own[1]); free(own[2]);
    ctx_free(&c);
}

/* ------------------------------------------------------------------ */
/* Third-order low-storage Runge-Kutta (Section 2). Coefficients of the */
/* Wray / Spalart-Moser-Rogers scheme: per substep                      */
/*   W <- W + dt (gamma_k R(W) + zeta_k R_prev),  R_prev <- R(W)        */
/* gamma = (8/15, 5/12, 3/4), zeta = (0, -17/60, -5/12).                */
/* ------------------------------------------------------------------ */
void orc_rk3_step(const orc_params* p, double* W, double* Rprev, double dt)
{
    static const double gk[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
    static const double zk[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};
    long nint = (long)p->nx * p->ny * p->nz;
    double* R = (double*)malloc(sizeof(double) * NV * nint);
    ctx c;
    int s;
    ctx_init(&c, p);
    for (s = 0; s < 3; ++s) {
        int k;
        orc_rhs(p, W, R, ORC_ALL, NULL, NULL, NULL);
#pragma omp parallel for
        for (k = 0; k < p->nz; ++k) {
            int i, j, v;
            for (j = 0; j < p->ny; ++j)
                for (i = 0; i < p->nx; ++i) {
                    long m = ((long)k * p->ny + j) * p->nx + i;
                    long n = vidx(&c, i, j, k);
                    for (v = 0; v < NV; ++v) {
                        double r = R[v * nint + m];
                        double rp = Rprev[v * nint + m];
                        W[v * c.nvol + n] = W[v * c.nvol + n] + dt * (gk[s] * r + zk[s] * rp);
                        Rprev[v * nint + m] = r;
                    }
                }
        }
    }
    orc_fill_ghosts(p, W);
    ctx_free(&c);
    free(R);
}

/* ------------------------------------------------------------------ */
/* CFL time step: dt = cfl / max over interior nodes of                 */
/*  sum_d (|u_d| + c) / h_d + 2 gamma mu / (rho Pr) sum_d 1 / h_d^2      */
/* with h_y = y_eta (the paper's compute_dt max reduction, Table 2).    */
/* ------------------------------------------------------------------ */
double orc_compute_dt(const orc_params* p, double* W, double cfl)
{
    ctx c;
    int k;
    double gmax = 0.0;
    ctx_init(&c, p);
    orc_fill_ghosts(p, W);
    c.Q = (double*)malloc(sizeof(double) * NQ * c.nvol);
    orc_primitives(p, W, c.Q);
    for (k = 0; k < p->nz; ++k) {
        int i, j;
        for (j = 0; j < p->ny; ++j)
            for (i = 0; i < p->nx; ++i) {
                long n = vidx(&c, i, j, k);
                double rho = c.Q[Q_RHO * c.nvol + n];
                double gm = gamma_at(p, c.Q[Q_T * c.nvol + n]);
                double cs = sqrt(gm * c.Q[Q_P * c.nvol + n] / rho);
                double mu = pow(c.Q[Q_T * c.nvol + n], p->visc_exp) / p->reynolds;
                double hy = c.y_eta[j];
                double conv = (fabs(c.Q[Q_U * c.nvol + n]) + cs) / c.dx +
                              (fabs(c.Q[Q_V * c.nvol + n]) + cs) / hy +
                              (fabs(c.Q[Q_W * c.nvol + n]) + cs) / c.dz;
                double visc = 2.0 * gm * mu / (rho * p->prandtl) *
                              (1.0 / (c.dx * c.dx) + 1.0 / (hy * hy) + 1.0 / (c.dz * c.dz));
                if (conv + visc > gmax) gmax = conv + visc;
            }
    }
    ctx_free(&c);
    return cfl / gmax;
}

/* ------------------------------------------------------------------ */
/* Diagnostics: metric-weighted volume integrals (cell volume           */
/* dx * y_eta * dz), extrema and counts; sums are pairwise.             */
/* out[0] mass, [1..3] momentum, [4] total energy, [5] kinetic energy,  */
/* [6] max Mach, [7] min rho, [8] min p, [9] non-finite nodes,           */
/* [10] nodes with rho<=0 or p<=0, [11] sum (R_rhou)^2 over interior    */
/* nodes if R is given (the paper's residual), [12..14] fraction of     */
/* WENO faces per direction, [15] total volume.                          */
/* ------------------------------------------------------------------ */
static double pairwise(const double* x, long n)
{
    if (n <= 8) {
        double s = 0.0;
        long i;
        for (i = 0; i < n; ++i) s += x[i];
        return s;
    }
    return pairwise(x, n / 2) + pairwise(x + n / 2, n - n / 2);
}

void orc_diagnostics(const orc_params* p, double* W, const double* R, double* out)
{
    ctx c;
    long nint = (long)p->nx * p->ny * p->nz, m;
    double* t = (double*)malloc(sizeof(double) * nint);
    int q, k;
    double mach = 0.0, rmin = INFINITY, pmin = INFINITY, nonfin = 0.0, nonphys = 0.0;
    ctx_init(&c, p);
    orc_fill_ghosts(p, W);
    c.Q = (double*)malloc(sizeof(double) * NQ * c.nvol);
    orc_primitives(p, W, c.Q);
    for (q = 0; q < 6; ++q) {
        for (k = 0; k < p->nz; ++k) {
            int i, j;
            for (j = 0; j < p->ny; ++j)
                for (i = 0; i < p->nx; ++i) {
                    long n = vidx(&c, i, j, k);
                    double vol = c.dx * c.y_eta[j] * c.dz;
                    double val;
                    if (q < 5) val = W[q * c.nvol + n];
                    else {
                        double u = c.Q[Q_U * c.nvol + n], v = c.Q[Q_V * c.nvol + n], w = c.Q[Q_W * c.nvol + n];
                        val = 0.5 * c.Q[Q_RHO * c.nvol + n] * (u * u + v * v + w * w);
                    }
                    t[((long)k * p->ny + j) * p->nx + i] = vol * val;
                }
        }
        out[q] = pairwise(t, nint);
    }
    for (k = 0; k < p->nz; ++k) {
        int i, j, v;
        for (j = 0; j < p->ny; ++j)
            for (i = 0; i < p->nx; ++i) {
                long n = vidx(&c, i, j, k);
                int bad = 0;
                for (v = 0; v < NV; ++v)
                    if (!isfinite(W[v * c.nvol + n])) bad = 1;
                if (bad) { nonfin += 1.0; continue; }
                double rho = c.Q[Q_RHO * c.nvol + n], pr = c.Q[Q_P * c.nvol + n];
                if (!(rho > 0.0) || !(pr > 0.0)) { nonphys += 1.0; }
                if (rho < rmin) rmin = rho;
                if (pr < pmin) pmin = pr;
                if (rho > 0.0 && pr > 0.0) {
                    double u = c.Q[Q_U * c.nvol + n], vv = c.Q[Q_V * c.nvol + n], w = c.Q[Q_W * c.nvol + n];
                    double ma = sqrt((u * u + vv * vv + w * w) * rho /
                                     (gamma_at(p, c.Q[Q_T * c.nvol + n]) * pr));
                    if (ma > mach) mach = ma;
                }
            }
    }
    out[6] = mach;
    out[7] = rmin;
    out[8] = pmin;
    out[9] = nonfin;
    out[10] = nonphys;
    if (R) {
        for (m = 0; m < nint; ++m) t[m] = R[1 * nint + m] * R[1 * nint + m];
        out[11] = pairwise(t, nint);
    } else {
        out[11] = 0.0;
    }
    out[12] = out[13] = out[14] = 0.0;
    if (p->sensor) {
        double* th = (double*)malloc(sizeof(double) * c.nvol);
        long nf[3] = {(long)p->nz * p->ny * (p->nx + 1), (long)p->nz * (p->ny + 1) * p->nx,
                      (long)(p->nz + 1) * p->ny * p->nx};
        unsigned char* f[3];
        int d;
        theta_field(&c, th);
        for (d = 0; d < 3; ++d) f[d] = (unsigned char*)malloc(nf[d]);
        orc_face_flags(p, th, f[0], f[1], f[2]);
        for (d = 0; d < 3; ++d) {
            long cnt = 0, e;
            for (e = 0; e < nf[d]; ++e) cnt += f[d][e];
            out[12 + d] = (double)cnt / (double)nf[d];
            free(f[d]);
        }
        free(th);
    }
    for (k = 0; k < p->nz; ++k) {
        int i, j;
        for (j = 0; j < p->ny; ++j)
            for (i = 0; i < p->nx; ++i) t[((long)k * p->ny + j) * p->nx + i] = c.dx * c.y_eta[j] * c.dz;
    }
    out[15] = pairwise(t, nint);
    free(t);
    ctx_free(&c);
}

/* Threads the OpenMP loops of this oracle use (1 without OpenMP). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
