"""Pins of the oracle's hybrid (sensor + WENO) pieces and of the diagnostics
fields against facts fixed outside the oracle:

- the face-flag window of the hybrid switch: one hot sensor node flags
  exactly the faces whose WENO stencil contains it (Section 2 hybrid switch,
  the stencil-maximum reading);
- the assembled characteristic WENO flux against an independent
  construction on the one-dimensional Euler system (numerical eigenvectors of
  the Roe-averaged Jacobian, local Lax-Friedrichs speeds over the whole
  stencil), on states whose largest wave speed sits at an end node of the
  stencil;
- convergence of the all-WENO scheme to the exact solution of Sod's Riemann
  problem (Toro, Riemann Solvers and Numerical Methods for Fluid Dynamics,
  ch. 4), with the y/z-uniform box staying uniform bitwise;
- closed forms of the diagnostics (maximum Mach number, residual, WENO face
  fractions) and of the viscous limit of the time step.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2304_05494_amd import inputs
from tests.helpers import embed, oracle_for

TWO_PI = 2.0 * math.pi


def _case(n=(16, 14, 12), **kw):
    base = dict(name="pin", nx=n[0], ny=n[1], nz=n[2], lx=TWO_PI, ly=TWO_PI, lz=TWO_PI,
                mach=0.3, reynolds=100.0, sensor=1)
    base.update(kw)
    return inputs.Case(**base)


# ---------------------------------------------------------------------------
# face-flag window
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("weno_order", [1, 3, 5, 7])
def test_single_hot_sensor_node_flags_exactly_its_stencil_faces(weno_order):
    """Face f of a line (between nodes f-1 and f) is WENO iff a node of its
    stencil f-r .. f+r-1 exceeds the threshold: a single hot node m flags
    exactly the faces m-r+1 .. m+r of its line in each direction, and no
    face of any other line."""
    r = (weno_order + 1) // 2
    case = _case(weno_order=weno_order, central_order=2, visc_order=2)
    o = oracle_for(case)
    g = o.ng
    m = (7, 6, 5)                                  # hot node (i, j, k), away from the edges
    th = np.zeros(o.ghosted_shape)
    th[m[2] + g, m[1] + g, m[0] + g] = 0.9
    fx, fy, fz = o.face_flags_from_theta(th)
    ex = np.zeros_like(fx)
    ex[m[2], m[1], m[0] - r + 1:m[0] + r + 1] = 1
    ey = np.zeros_like(fy)
    ey[m[2], m[1] - r + 1:m[1] + r + 1, m[0]] = 1
    ez = np.zeros_like(fz)
    ez[m[2] - r + 1:m[2] + r + 1, m[1], m[0]] = 1
    assert np.array_equal(fx, ex)
    assert np.array_equal(fy, ey)
    assert np.array_equal(fz, ez)
    assert fx.sum() == fy.sum() == fz.sum() == 2 * r


def test_flag_threshold_is_strict_and_reads_ghost_nodes():
    """A node exactly at the threshold flags nothing; a hot ghost node (the
    periodic image supplied in the sensor field) flags the first faces of
    its line only."""
    case = _case(sensor_thr=0.5)
    o = oracle_for(case)
    g, r = o.ng, 3
    th = np.zeros(o.ghosted_shape)
    th[g + 2, g + 3, g + 4] = 0.5
    fx, fy, fz = o.face_flags_from_theta(th)
    assert fx.sum() == fy.sum() == fz.sum() == 0
    th[:] = 0.0
    th[g + 2, g + 3, g - 1] = 0.75                 # ghost node i = -1 of line (j=3, k=2)
    fx, fy, fz = o.face_flags_from_theta(th)
    ex = np.zeros_like(fx)
    ex[2, 3, 0:r] = 1                              # faces 0 .. r-1 hold node -1 in their stencils
    assert np.array_equal(fx, ex)
    assert fy.sum() == fz.sum() == 0


def test_sensor_ghost_nodes_are_images():
    """Sensor at ghost nodes: the periodic image on periodic sides, the
    mirror interior node on wall sides."""
    case = inputs.channel_case(12, 16, 8)
    case = inputs.Case(**{**case.__dict__, "sensor": 1, "name": "channel-sensor"})
    o = oracle_for(case)
    W = np.ascontiguousarray(inputs.fields(case))
    th = o.theta(W)
    g = o.ng
    nx, ny, nz = case.nx, case.ny, case.nz
    inner = th[g:g + nz, g:g + ny, g:g + nx]
    assert inner.max() > 0.0
    for l in range(g):
        # x periodic
        np.testing.assert_array_equal(th[g:g + nz, g:g + ny, g - 1 - l], inner[:, :, nx - 1 - l])
        np.testing.assert_array_equal(th[g:g + nz, g:g + ny, g + nx + l], inner[:, :, l])
        # y walls: mirror
        np.testing.assert_array_equal(th[g:g + nz, g - 1 - l, g:g + nx], inner[:, l, :])
        np.testing.assert_array_equal(th[g:g + nz, g + ny + l, g:g + nx], inner[:, ny - 1 - l, :])


# ---------------------------------------------------------------------------
# assembled characteristic WENO flux
# ---------------------------------------------------------------------------
def _flux_1d(Wv, gamma):
    rho, m, E = Wv
    u = m / rho
    p = (gamma - 1.0) * (E - 0.5 * m * u)
    return np.array([m, m * u + p, (E + p) * u])


def _prims_1d(Wv, gamma):
    rho, m, E = Wv
    u = m / rho
    p = (gamma - 1.0) * (E - 0.5 * m * u)
    return rho, u, p, (E + p) / rho


def _reference_char_weno_flux(W6, order, gamma, eps):
    """Face flux between the two middle nodes of the 2r nodes W6 (rows are
    (rho, rho u, rho E) of the one-dimensional Euler system), built
    independently of the oracle's analytic eigenvectors:
      1. Roe average of the two face nodes;
      2. Jacobian of the flux at the Roe state by complex-step
         differentiation, eigenvectors by numpy (sorted u-c, u, u+c);
      3. per characteristic field, local Lax-Friedrichs speed = largest
         |eigenvalue| over all 2r stencil nodes;
      4. WENO of the split characteristic fluxes, g+ over nodes 0..2r-2,
         g- mirrored over nodes 2r-1..1;
      5. back with the right eigenvectors."""
    r = W6.shape[0] // 2
    A, B = r - 1, r
    ra, ua, _, Ha = _prims_1d(W6[A], gamma)
    rb, ub, _, Hb = _prims_1d(W6[B], gamma)
    sa, sb = math.sqrt(ra), math.sqrt(rb)
    u = (sa * ua + sb * ub) / (sa + sb)
    H = (sa * Ha + sb * Hb) / (sa + sb)
    Wroe = np.array([1.0, u, (H + 0.5 * (gamma - 1.0) * u * u) / gamma])
    J = np.zeros((3, 3))
    for m in range(3):
        d = np.zeros(3, complex)
        d[m] = 1e-30j
        J[:, m] = np.imag(_flux_1d(Wroe + d, gamma)) / 1e-30
    ev, Rv = np.linalg.eig(J)
    order_idx = np.argsort(ev.real)
    Rv = np.real(Rv[:, order_idx])
    Lv = np.linalg.inv(Rv)
    lam = np.zeros(3)
    for t in range(2 * r):
        rho, ut, p, _ = _prims_1d(W6[t], gamma)
        c = math.sqrt(gamma * p / rho)
        lam = np.maximum(lam, np.abs([ut - c, ut, ut + c]))
    g = np.array([Lv @ _flux_1d(W6[t], gamma) for t in range(2 * r)])
    q = np.array([Lv @ W6[t] for t in range(2 * r)])
    gp = 0.5 * (g + lam[None, :] * q)
    gm = 0.5 * (g - lam[None, :] * q)
    Fh = np.zeros(3)
    for k in range(3):
        Fh[k] = (O.weno_left(order, eps, gp[0:2 * r - 1, k]) +
                 O.weno_left(order, eps, gm[2 * r - 1:0:-1, k]))
    return Rv @ Fh


@pytest.mark.parametrize("weno_order", [3, 5, 7])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_char_weno_flux_with_fastest_node_at_stencil_end(weno_order, seed):
    """The oracle's characteristic WENO face flux equals the independent
    construction on rough 1-D states whose fastest nodes (largest |u+c|
    and largest |u-c|) are the two end nodes of the 2r-node stencil, so the
    local Lax-Friedrichs speeds differ from those of the two face nodes."""
    gamma = 1.4
    eps = 1e-40                      # weights invariant under eigenvector scaling
    r = (weno_order + 1) // 2
    rng = np.random.default_rng(100 + seed)
    prim = []
    for t in range(8):
        prim.append((0.6 + 0.8 * rng.random(), 0.4 * rng.normal(), 0.5 + rng.random()))
    s0 = 3 - r + 1                   # first stencil entry of the 8-node input
    rho, _, p = prim[s0]
    prim[s0] = (rho, 2.5, p)         # fastest right-running wave at the left end
    rho, _, p = prim[s0 + 2 * r - 1]
    prim[s0 + 2 * r - 1] = (rho, -2.5, p)   # fastest left-running wave at the right end
    W8 = np.array([inputs.conserved(gamma, rh, u, 0.0, 0.0, pp) for rh, u, pp in prim])
    F = O.face_flux_1d(gamma, W8, weno_order=weno_order, weno_eps=eps, use_weno=True)
    W6 = W8[s0:s0 + 2 * r][:, [0, 1, 4]]
    ref = _reference_char_weno_flux(W6, weno_order, gamma, eps)
    np.testing.assert_allclose(F[[0, 1, 4]], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    assert F[2] == 0.0 and F[3] == 0.0
    # the check is not vacuous: speeds of the two face nodes alone give
    # another flux
    alt = W6.copy()
    for t in list(range(0, r - 1)) + list(range(r + 1, 2 * r)):
        alt[t] = W6[r - 1] if t < r else W6[r]
    lam_face = _reference_char_weno_flux(alt, weno_order, gamma, eps)
    assert np.abs(lam_face - ref).max() > 1e-3 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# Sod's problem with WENO on every face
# ---------------------------------------------------------------------------
def exact_riemann(left, right, gamma, xi):
    """Exact solution (rho, u, p) of the Riemann problem at similarity
    coordinates xi = (x - x0)/t (Toro ch. 4: pressure function, Newton
    iteration for the star pressure, sampling of the wave pattern)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    g1 = (gamma - 1.0) / (2.0 * gamma)

    def fk(p, rk, pk, ck):
        if p > pk:
            a, b = 2.0 / ((gamma + 1.0) * rk), (gamma - 1.0) / (gamma + 1.0) * pk
            f = (p - pk) * math.sqrt(a / (p + b))
            return f, math.sqrt(a / (b + p)) * (1.0 - 0.5 * (p - pk) / (b + p))
        f = 2.0 * ck / (gamma - 1.0) * ((p / pk) ** g1 - 1.0)
        return f, (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma)) / (rk * ck)

    p = 0.5 * (pl + pr)
    for _ in range(100):
        f1, d1 = fk(p, rl, pl, cl)
        f2, d2 = fk(p, rr, pr, cr)
        pn = max(1e-12, p - (f1 + f2 + ur - ul) / (d1 + d2))
        if abs(pn - p) < 1e-15 * p:
            p = pn
            break
        p = pn
    ps = p
    us = 0.5 * (ul + ur) + 0.5 * (fk(ps, rr, pr, cr)[0] - fk(ps, rl, pl, cl)[0])
    gr = (gamma - 1.0) / (gamma + 1.0)
    out = np.zeros((3, len(xi)))
    for n, s in enumerate(xi):
        if s <= us:                                # left of the contact
            if ps > pl:
                sl = ul - cl * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pl + g1)
                st = (rl, ul, pl) if s <= sl else (rl * (ps / pl + gr) / (gr * ps / pl + 1.0), us, ps)
            else:
                csl = cl * (ps / pl) ** g1
                if s <= ul - cl:
                    st = (rl, ul, pl)
                elif s > us - csl:
                    st = (rl * (ps / pl) ** (1.0 / gamma), us, ps)
                else:
                    u = 2.0 / (gamma + 1.0) * (cl + 0.5 * (gamma - 1.0) * ul + s)
                    c = 2.0 / (gamma + 1.0) * (cl + 0.5 * (gamma - 1.0) * (ul - s))
                    st = (rl * (c / cl) ** (2.0 / (gamma - 1.0)), u, pl * (c / cl) ** (2.0 * gamma / (gamma - 1.0)))
        else:                                      # right of the contact
            if ps > pr:
                sr = ur + cr * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pr + g1)
                st = (rr, ur, pr) if s >= sr else (rr * (ps / pr + gr) / (gr * ps / pr + 1.0), us, ps)
            else:
                csr = cr * (ps / pr) ** g1
                if s >= ur + cr:
                    st = (rr, ur, pr)
                elif s < us + csr:
                    st = (rr * (ps / pr) ** (1.0 / gamma), us, ps)
                else:
                    u = 2.0 / (gamma + 1.0) * (-cr + 0.5 * (gamma - 1.0) * ur + s)
                    c = 2.0 / (gamma + 1.0) * (cr - 0.5 * (gamma - 1.0) * (ur - s))
                    st = (rr * (c / cr) ** (2.0 / (gamma - 1.0)), u, pr * (c / cr) ** (2.0 * gamma / (gamma - 1.0)))
        out[:, n] = st
    return out


def test_exact_riemann_solver_reproduces_sod_star_state():
    """Toro's Table 4.2 star values of test 1 (Sod): p* = 0.30313,
    u* = 0.92745 (checks the reference solver of the pin below)."""
    sol = exact_riemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, np.array([0.5]))
    assert sol[2, 0] == pytest.approx(0.30313, abs=1e-5)
    assert sol[1, 0] == pytest.approx(0.92745, abs=1e-5)


def _sod_run(nx, weno_order=5, t_end=0.2):
    gamma = 1.4
    nyz = 4
    dx = 1.0 / nx
    case = inputs.Case(name=f"sod{nx}", nx=nx, ny=nyz, nz=nyz, lx=1.0, ly=nyz * dx, lz=nyz * dx,
                       bc=(inputs.EXTRAP, inputs.EXTRAP, 0, 0, 0, 0), gamma=gamma, mach=1.0,
                       reynolds=1e300, weno_order=weno_order, sensor=1, sensor_thr=-1.0)
    o = oracle_for(case)
    xc = (np.arange(nx) + 0.5) * dx
    left = xc < 0.5
    shape = (nyz, nyz, nx)
    rho = np.broadcast_to(np.where(left, 1.0, 0.125), shape).copy()
    p = np.broadcast_to(np.where(left, 1.0, 0.1), shape).copy()
    z = np.zeros(shape)
    W = embed(inputs.conserved(gamma, rho, z, z, z, p), o.ng)
    nsteps = int(math.ceil(t_end / (0.4 * dx / 2.0)))
    dt = t_end / nsteps
    Rp = np.zeros((5, nyz, nyz, nx))
    for _ in range(nsteps):
        o.rk3_step(W, Rp, dt)
    Wi = o.interior(W)
    return xc, Wi


@pytest.mark.parametrize("weno_order", [5, 7])
def test_sod_with_weno_everywhere_converges_to_exact_solution(weno_order):
    """Sod's problem as a y/z-uniform box, WENO characteristic fluxes on
    every face: density and pressure converge in L1 to the exact solution
    at t = 0.2, and every (y, z) line stays identical bitwise."""
    errs = []
    for nx in (50, 100, 200):
        xc, Wi = _sod_run(nx, weno_order)
        ref = exact_riemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, (xc - 0.5) / 0.2)
        for k in range(Wi.shape[1]):
            for j in range(Wi.shape[2]):
                assert np.array_equal(Wi[:, k, j, :], Wi[:, 0, 0, :])
        assert np.all(Wi[2] == 0.0) and np.all(Wi[3] == 0.0)
        rho = Wi[0, 0, 0]
        u = Wi[1, 0, 0] / rho
        p = 0.4 * (Wi[4, 0, 0] - 0.5 * rho * u * u)
        errs.append((np.abs(rho - ref[0]).mean(), np.abs(p - ref[2]).mean(), np.abs(u - ref[1]).mean()))
    errs = np.array(errs)
    # first order at the discontinuities: each refinement cuts the L1 error
    # by at least a factor 1.5; the finest grid is within 1 % of the jumps
    assert np.all(errs[1] < errs[0] / 1.5) and np.all(errs[2] < errs[1] / 1.5), errs
    assert errs[2, 0] < 0.01 and errs[2, 1] < 0.01, errs


# ---------------------------------------------------------------------------
# diagnostics fields and the viscous time-step limit
# ---------------------------------------------------------------------------
def _resting(case, rho=1.0, p=2.0):
    shape = (case.nz + 2 * case.ng, case.ny + 2 * case.ng, case.nx + 2 * case.ng)
    z = np.zeros(shape)
    return np.ascontiguousarray(inputs.conserved(case.gamma, np.full(shape, rho), z, z, z, np.full(shape, p)))


def test_diagnostics_max_mach_and_residual_closed_forms():
    case = _case((8, 8, 8), sensor=0)
    o = oracle_for(case)
    g = o.ng
    W = _resting(case, rho=1.5, p=2.0)
    # one interior node moving at speed 0.9 along a diagonal
    u = np.array([0.3, -0.6, 0.6])
    W[1:4, g + 2, g + 5, g + 1] = 1.5 * u
    W[4, g + 2, g + 5, g + 1] += 0.5 * 1.5 * (u @ u)
    rng = np.random.default_rng(3)
    R = rng.normal(size=(5, 8, 8, 8))
    d = o.diagnostics(W, R)
    c = math.sqrt(1.4 * 2.0 / 1.5)
    assert d[6] == pytest.approx(0.9 / c, rel=1e-14)
    assert d[11] == pytest.approx(math.fsum((R[1] ** 2).ravel()), rel=1e-13)
    assert d[7] == 1.5 and d[8] == pytest.approx(2.0, rel=1e-14)


@pytest.mark.parametrize("thr,expect", [(-1.0, 1.0), (2.0, 0.0)])
def test_diagnostics_weno_fractions_at_the_limits(thr, expect):
    """With the threshold below the sensor's range every face is WENO, above
    it none is."""
    case = _case((10, 8, 6), sensor_thr=thr)
    o = oracle_for(case)
    W = np.ascontiguousarray(inputs.tgv_fields(inputs.Case(**{**case.__dict__, "name": "tgv"})))
    d = o.diagnostics(W)
    assert list(d[12:15]) == [expect] * 3


def test_compute_dt_viscous_limit_of_resting_gas():
    """Resting gas at low Reynolds number on a uniform cube: dt = cfl /
    (3 c / h + 2 gamma mu / (rho Pr) 3 / h^2) with mu = T^s / Re."""
    n = 8
    case = _case((n, n, n), sensor=0, reynolds=0.05, mach=0.5, visc_exp=0.7)
    o = oracle_for(case)
    W = _resting(case, rho=1.5, p=2.0)
    c = math.sqrt(1.4 * 2.0 / 1.5)
    T = 1.4 * 0.25 * 2.0 / 1.5
    mu = T ** 0.7 / 0.05
    h = TWO_PI / n
    rate = 3.0 * c / h + 2.0 * 1.4 * mu / (1.5 * 0.72) * 3.0 / (h * h)
    assert rate > 10 * 3.0 * c / h          # the viscous part dominates
    assert o.compute_dt(W, 0.5) == pytest.approx(0.5 / rate, rel=1e-14)


# ---------------------------------------------------------------------------
# WENO-7 (Balsara-Shu) and the smoothness indicators of every order
# ---------------------------------------------------------------------------
def _cell_average_poly(vals, offs):
    """Coefficients (ascending powers of x) of the polynomial of degree
    len(vals)-1 whose averages over the unit cells centred at `offs` are
    `vals` (the reconstruction polynomial of a WENO stencil)."""
    n = len(vals)
    A = np.array([[((o + 0.5) ** (m + 1) - (o - 0.5) ** (m + 1)) / (m + 1) for m in range(n)] for o in offs])
    return np.linalg.solve(A, np.asarray(vals, dtype=float))


def _smoothness_from_definition(c):
    """sum_{l>=1} integral over [-1/2, 1/2] of (d^l p / dx^l)^2 (unit h)."""
    P = np.polynomial.Polynomial(c)
    tot = 0.0
    for l in range(1, len(c)):
        d = P.deriv(l)
        q = (d * d).integ()
        tot += q(0.5) - q(-0.5)
    return tot


@pytest.mark.parametrize("order", [3, 5, 7])
def test_smoothness_indicators_match_their_definition(order):
    r = (order + 1) // 2
    rng = np.random.default_rng(order)
    for _ in range(20):
        v = rng.normal(size=2 * r - 1)
        beta = O.weno_smoothness(order, v)
        for k in range(r):
            offs = list(range(-r + 1 + k, k + 1))
            c = _cell_average_poly(v[k:k + r], offs)
            ref = _smoothness_from_definition(c)
            assert beta[k] == pytest.approx(ref, rel=1e-11, abs=1e-12 * np.abs(v).max() ** 2)


def test_weno7_linear_weights_limit_is_the_seventh_order_reconstruction():
    """With equal nonlinear weights WENO-7 returns the value at the face of
    the degree-6 polynomial with the seven given cell averages."""
    rng = np.random.default_rng(7)
    for _ in range(10):
        v = rng.normal(size=7)
        c = _cell_average_poly(v, list(range(-3, 4)))
        ref = np.polynomial.Polynomial(c)(0.5)
        assert O.weno_left(7, 1e30, v) == pytest.approx(ref, rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("eps,ns,expect", [
    (1e30, (32, 64, 128), 6.9),       # linear weights: exactly seventh order
    (1e-6, (32, 64, 128), 6.5),       # smoothness-weighted: the order holds
])
def test_weno7_reconstruction_order_on_smooth_data(eps, ns, expect):
    r = 4
    errs = []
    for n in ns:
        h = TWO_PI / n
        x = np.arange(n) * h
        f = np.sin(x) + 0.3 * np.cos(2 * x)
        fh = np.array([O.weno_left(7, eps, np.roll(f, -(i - r + 1))[:2 * r - 1]) for i in range(n)])
        d = (fh - np.roll(fh, 1)) / h
        errs.append(np.abs(d - (np.cos(x) - 0.6 * np.sin(2 * x))).max())
    assert math.log2(errs[1] / errs[2]) > expect, errs


def test_weno7_is_nonoscillatory_at_a_step():
    v = np.array([1.0, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    out = O.weno_left(7, 1e-6, v)
    assert -1e-9 <= out <= 1.0 + 1e-9
    assert out == pytest.approx(1.0, abs=1e-3)
