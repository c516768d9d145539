"""Pins of the oracle's thermally perfect gas (Section 2: specific heats
depending on temperature through NASA polynomials):
  * a constant polynomial c_p/R = gamma/(gamma-1) reproduces the calorically
    perfect gas (right-hand sides, walls, time step, diagnostics);
  * the caloric functions are consistent: c_p - c_v = R, de/dT = c_v and
    dc_p/dT agree with high-order differences, T(e(T)) = T;
  * the right-hand side conserves all five variables on a periodic block
    (inviscid), a wall's ghost node mirrors T about T_wall at equal pressure;
  * design order 2L against an independent spectral evaluation of the
    divergence-form equations with the same gas.
The polynomial here has the NASA form but made-up coefficients (c_p/R from
3.5 near 300 K rising to about 4.1 near 1200 K); it is not a real species."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2304_05494_amd import inputs
from tests.helpers import oracle_for, spectral_deriv

NASA = (3.30, 5.0e-4, 1.5e-7, -2.5e-10, 8.0e-14)
TREF = 300.0


def _periodic(n=24, thermo=1, nasa=NASA, order=6, **kw):
    two_pi = 2 * math.pi
    return inputs.Case(name="thermo", nx=n, ny=n - 4, nz=n - 8, lx=two_pi, ly=two_pi, lz=two_pi,
                       mach=0.5, reynolds=200.0, central_order=order, visc_order=order,
                       thermo=thermo, nasa=nasa, t_ref=TREF, **kw)


def _state(case, T, rho, u, v, w):
    """Conserved variables of a thermally perfect state (energy from the
    oracle's own caloric function, node by node)."""
    o = oracle_for(case)
    e = np.vectorize(lambda t: o.thermo_eval(t)[2])(T)
    E = rho * e + 0.5 * rho * (u * u + v * v + w * w)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, rho * w, E]))


def _smooth(case, amp=1.0):
    g = case.ng
    ax = [np.arange(-g, n + g) * 2 * math.pi / n for n in (case.nx, case.ny, case.nz)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    rho = 1 + 0.2 * amp * np.sin(X + 0.4) * np.cos(Y) + 0.1 * np.sin(Z + 1)
    T = 2.0 + 0.8 * amp * np.cos(X - Y + Z) + 0.3 * np.sin(2 * Z)
    u = 0.5 * np.sin(Y + Z) + 0.1
    v = 0.4 * np.cos(X + 2 * Z)
    w = 0.3 * np.sin(X + Y)
    return T, rho, u, v, w


def test_constant_polynomial_is_the_calorically_perfect_gas():
    gam = 1.4
    base = inputs.channel_case(40, 24, 10)
    cp_case = inputs.Case(**{**base.__dict__, "thermo": 0})
    tp_case = inputs.Case(**{**base.__dict__, "thermo": 1, "nasa": (gam / (gam - 1), 0, 0, 0, 0)})
    W = np.ascontiguousarray(inputs.fields(cp_case))
    a, b = oracle_for(cp_case), oracle_for(tp_case)
    Ra, Rb = a.rhs(W.copy()), b.rhs(W.copy())
    sc = np.abs(Ra).max(axis=(1, 2, 3))
    assert np.all(np.abs(Ra - Rb).max(axis=(1, 2, 3)) <= 1e-12 * sc)
    Wa, Wb = W.copy(), W.copy()
    a.fill_ghosts(Wa)
    b.fill_ghosts(Wb)
    assert np.abs(Wa - Wb).max() <= 1e-13 * np.abs(Wa).max()
    assert b.compute_dt(W.copy(), 0.5) == pytest.approx(a.compute_dt(W.copy(), 0.5), rel=1e-13)
    np.testing.assert_allclose(b.diagnostics(W.copy()), a.diagnostics(W.copy()), rtol=1e-13, atol=0)


def test_caloric_functions_consistent():
    o = oracle_for(_periodic())
    R = 1.0 / (1.4 * 0.5 ** 2)
    for T in (0.4, 1.0, 2.5, 4.0):
        cp, cv, e, dcp = o.thermo_eval(T)
        assert cp - cv == pytest.approx(R, rel=1e-14)
        h = 1e-3
        E = [o.thermo_eval(T + k * h)[2] for k in (-2, -1, 1, 2)]
        C = [o.thermo_eval(T + k * h)[0] for k in (-2, -1, 1, 2)]
        de = (E[0] - 8 * E[1] + 8 * E[2] - E[3]) / (12 * h)
        dc = (C[0] - 8 * C[1] + 8 * C[2] - C[3]) / (12 * h)
        assert de == pytest.approx(cv, rel=1e-10)
        assert dc == pytest.approx(dcp, rel=1e-8)
        assert o.thermo_T(e) == pytest.approx(T, rel=1e-14)
    # the polynomial makes c_p vary over the range used here
    assert o.thermo_eval(4.0)[0] > 1.1 * o.thermo_eval(1.0)[0]


def test_inviscid_conservation():
    case = _periodic()
    W = _state(case, *_smooth(case))
    R = oracle_for(case).rhs(W.copy(), mask=O.CONV_X | O.CONV_Y | O.CONV_Z)
    for v in range(5):
        assert abs(R[v].sum()) <= 1e-14 * np.abs(R[v]).sum()


def test_wall_ghost_mirrors_temperature_at_equal_pressure():
    base = inputs.channel_case(24, 16, 6)
    case = inputs.Case(**{**base.__dict__, "thermo": 1, "nasa": NASA, "t_ref": TREF, "t_wall": 1.3})
    o = oracle_for(case)
    W = np.ascontiguousarray(inputs.fields(case))
    o.fill_ghosts(W)
    Q = o.primitives(W)        # rho, u, v, w, p, T, H over the ghosted box
    g = case.ng
    for l in range(g):
        ghost, mirror = g - 1 - l, g + l             # y-lo wall between j = -1 and j = 0
        Tg, Tm = Q[5][:, ghost, g:-g], Q[5][:, mirror, g:-g]
        np.testing.assert_allclose(Tg, 2 * case.t_wall - Tm, rtol=1e-13)
        np.testing.assert_allclose(Q[4][:, ghost, g:-g], Q[4][:, mirror, g:-g], rtol=1e-13)
        np.testing.assert_allclose(Q[1][:, ghost, g:-g], -Q[1][:, mirror, g:-g], rtol=1e-13, atol=1e-15)


def _exact_rhs_thermo(case, o, T, rho, u, v, w):
    """Divergence-form Navier-Stokes with the same gas, spectral derivatives
    (independent of the oracle's discretisation)."""
    lx, ly, lz = case.lx, case.ly, case.lz
    D = [lambda f: spectral_deriv(f, 2, lx), lambda f: spectral_deriv(f, 1, ly),
         lambda f: spectral_deriv(f, 0, lz)]
    R = 1.0 / (case.gamma * case.mach ** 2)
    f = np.vectorize(lambda t: tuple(o.thermo_eval(t)), otypes=[float] * 4)(T)
    cp, e = f[0], f[2]
    p = rho * R * T
    vel = [u, v, w]
    E = rho * e + 0.5 * rho * (u * u + v * v + w * w)
    out = np.zeros((5,) + rho.shape)
    for d in range(3):
        out[0] -= D[d](rho * vel[d])
        for i in range(3):
            out[1 + i] -= D[d](rho * vel[d] * vel[i] + (p if i == d else 0.0))
        out[4] -= D[d](vel[d] * (E + p))
    mu = T ** case.visc_exp / case.reynolds
    k = mu * cp / case.prandtl
    g = [[D[j](vel[i]) for j in range(3)] for i in range(3)]
    div = g[0][0] + g[1][1] + g[2][2]
    tau = [[mu * (g[i][j] + g[j][i] - (2.0 / 3.0 * div if i == j else 0.0)) for j in range(3)]
           for i in range(3)]
    for i in range(3):
        out[1 + i] += sum(D[j](tau[i][j]) for j in range(3))
    for j in range(3):
        out[4] += D[j](sum(vel[i] * tau[i][j] for i in range(3)) + k * D[j](T))
    return out


@pytest.mark.parametrize("order", [4, 6])
def test_design_order(order):
    errs = []
    for n in (16, 32):
        two_pi = 2 * math.pi
        case = inputs.Case(name="thermo", nx=n, ny=n, nz=n, lx=two_pi, ly=two_pi, lz=two_pi, mach=0.5,
                           reynolds=50.0, central_order=order, visc_order=order, thermo=1, nasa=NASA,
                           t_ref=TREF)
        o = oracle_for(case)
        fields = _smooth(case, amp=0.5)
        W = _state(case, *fields)
        Rn = o.rhs(W.copy())
        gq = case.ng
        inner = tuple(slice(gq, -gq) for _ in range(3))
        ex = _exact_rhs_thermo(case, o, *[f[inner] for f in fields])
        errs.append(np.abs(Rn - ex).max())
    rate = math.log2(errs[0] / errs[1])
    assert rate > order - 0.7, (errs, rate)
