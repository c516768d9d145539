"""Pins of the oracle's KEEP-n central flux (the optional kinetic-energy and
entropy preserving scheme of Section 2) against what the mathematics fixes:
  * with exact logarithmic means the semi-discrete entropy production of the
    periodic inviscid right-hand side vanishes to rounding (the two-point
    flux satisfies Tadmor's entropy-conservation condition, and the central
    high-order flux form carries that to any order);
  * with the log-mean series cut after n terms the production is small and
    shrinks as n grows;
  * pressure equilibrium: uniform velocity and pressure with varying density
    keep velocity and pressure steady for every n;
  * kinetic-energy preservation: sum u.C_mom - |u|^2/2 C_rho equals the
    pressure work sum u . D p;
  * telescoping conservation of all five variables, a free stream gives an
    exactly zero right-hand side, and the design order 2L against the exact
    divergence-form derivative on smooth periodic data."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2304_05494_amd import inputs
from tests.helpers import exact_rhs, oracle_for

CONV = O.CONV_X | O.CONV_Y | O.CONV_Z
GAMMA = 1.4


def _case(n=24, keep_n=-1, order=6, nx=None, ny=None, nz=None, **kw):
    two_pi = 2 * math.pi
    return inputs.Case(name="keep", nx=nx or n, ny=ny or (n - 4), nz=nz or (n - 8), lx=two_pi,
                       ly=two_pi, lz=two_pi, mach=0.5, central_order=order, visc_order=order,
                       central_flux=1, keep_n=keep_n, **kw)


def _grid(case):
    g = case.ng
    ax = [np.arange(-g, n + g) * 2 * math.pi / n for n in (case.nx, case.ny, case.nz)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X, Y, Z


def _smooth(case, amp=0.3):
    X, Y, Z = _grid(case)
    rho = 1 + amp * np.sin(X + 0.4) * np.cos(Y) + 0.2 * np.sin(Z + 1)
    u = 0.5 * np.sin(Y + Z) + 0.1
    v = 0.4 * np.cos(X + 2 * Z)
    w = 0.3 * np.sin(X + Y)
    p = (1 / (GAMMA * case.mach ** 2)) * (1 + 0.2 * np.cos(X - Y + Z))
    return np.ascontiguousarray(inputs.conserved(GAMMA, rho, u, v, w, p))


def _prims(Wi):
    rho = Wi[0]
    u, v, w = Wi[1] / rho, Wi[2] / rho, Wi[3] / rho
    p = (GAMMA - 1) * (Wi[4] - 0.5 * rho * (u * u + v * v + w * w))
    return rho, u, v, w, p


def _entropy_production(case, W):
    o = oracle_for(case)
    R = o.rhs(W.copy(), mask=CONV)
    rho, u, v, w, p = _prims(o.interior(W))
    s = np.log(p) - GAMMA * np.log(rho)
    # entropy variables of U = -rho s / (gamma - 1)
    ev = [(GAMMA - s) / (GAMMA - 1) - rho * (u * u + v * v + w * w) / (2 * p),
          rho * u / p, rho * v / p, rho * w / p, -rho / p]
    terms = [e * r for e, r in zip(ev, R)]
    return float(sum(t.sum() for t in terms)), float(sum(np.abs(t).sum() for t in terms))


@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_exact_log_means_conserve_entropy(order):
    case = _case(keep_n=-1, order=order)
    prod, scale = _entropy_production(case, _smooth(case))
    assert abs(prod) <= 1e-13 * scale, prod / scale


def test_split_form_does_not_conserve_entropy():
    """The same check is not vacuous: the Pirozzoli split form produces
    entropy at truncation level on the same data."""
    case = inputs.Case(**{**_case(keep_n=-1).__dict__, "central_flux": 0})
    prod, scale = _entropy_production(case, _smooth(case, amp=0.6))
    assert abs(prod) > 1e-10 * scale


def test_truncated_series_converges_to_exact_log_means():
    """Cutting the log-mean series after n terms leaves an error of the order
    of the next term, xi^(2n+2)/(2n+3): the right-hand side approaches the
    exact-mean one geometrically in n, and so does the entropy production
    (signed sums of the pair errors, so not monotonically)."""
    ce = _case(keep_n=-1)
    W = _smooth(ce, amp=0.6)
    Rex = oracle_for(ce).rhs(W.copy(), mask=CONV)
    dev, prod = [], []
    for n in range(6):
        c = _case(keep_n=n)
        dev.append(np.abs(oracle_for(c).rhs(W.copy(), mask=CONV) - Rex).max() / np.abs(Rex).max())
        pr, sc = _entropy_production(c, W)
        prod.append(abs(pr) / sc)
    assert dev[0] > 1e-4
    for a, b in zip(dev, dev[1:]):
        assert b < a / 3, dev
    assert prod[0] > 1e-9 and prod[5] < prod[0] / 10, prod


@pytest.mark.parametrize("keep_n", [0, 2, -1])
def test_pressure_equilibrium_preserved(keep_n):
    case = _case(keep_n=keep_n)
    X, Y, Z = _grid(case)
    rho = 1 + 0.5 * np.sin(X) * np.cos(2 * Y) + 0.3 * np.cos(Z + 0.3)
    u0, v0, w0, p0 = 0.7, -0.4, 0.25, 1 / (GAMMA * case.mach ** 2)
    W = np.ascontiguousarray(inputs.conserved(GAMMA, rho, u0 + 0 * X, v0 + 0 * X, w0 + 0 * X, p0 + 0 * X))
    o = oracle_for(case)
    R = o.rhs(W.copy(), mask=CONV)
    Wi = o.interior(W)
    # d u_i/dt = (R_mom - u_i R_rho) / rho, d p/dt = (gamma-1)(R_E - u.R_mom + |u|^2/2 R_rho)
    du = [(R[1 + i] - c * R[0]) / Wi[0] for i, c in enumerate((u0, v0, w0))]
    q2 = u0 * u0 + v0 * v0 + w0 * w0
    dp = (GAMMA - 1) * (R[4] - u0 * R[1] - v0 * R[2] - w0 * R[3] + 0.5 * q2 * R[0])
    scale = np.abs(R[0]).max()
    assert scale > 1e-2          # density does change
    for d in du:
        assert np.abs(d).max() < 1e-12 * scale * 10
    assert np.abs(dp).max() < 1e-12 * scale * p0 * 10


def test_kinetic_energy_identity():
    case = _case(keep_n=1)
    W = _smooth(case, amp=0.6)
    o = oracle_for(case)
    R = o.rhs(W.copy(), mask=CONV)        # R = -C
    rho, u, v, w, p = _prims(o.interior(W))
    lhs = -(u * R[1] + v * R[2] + w * R[3]) + 0.5 * (u * u + v * v + w * w) * R[0]
    # pressure work sum u . D p with the same central first derivative
    a, _ = O.fd_coeffs(case.central_order)
    hx = 2 * math.pi / case.nx, 2 * math.pi / case.ny, 2 * math.pi / case.nz

    def D(f, axis, h):
        return sum(a[l] * (np.roll(f, -l, axis) - np.roll(f, l, axis)) for l in range(1, 4)) / h

    work = u * D(p, 2, hx[0]) + v * D(p, 1, hx[1]) + w * D(p, 0, hx[2])
    scale = np.abs(work).sum()
    assert abs(lhs.sum() - work.sum()) < 1e-13 * scale


def test_conservation_and_free_stream():
    case = _case(keep_n=2)
    W = _smooth(case, amp=0.6)
    o = oracle_for(case)
    R = o.rhs(W.copy(), mask=CONV)
    for v in range(5):
        assert abs(R[v].sum()) < 1e-14 * np.abs(R[v]).sum()
    g = case.ng
    shape = (case.nz + 2 * g, case.ny + 2 * g, case.nx + 2 * g)
    one = np.ones(shape)
    Wf = np.ascontiguousarray(inputs.conserved(GAMMA, 1.3 * one, 0.2 * one, -0.1 * one, 0.3 * one, 2.0 * one))
    assert np.all(o.rhs(Wf, mask=CONV) == 0.0)


@pytest.mark.parametrize("order", [4, 6])
def test_design_order(order):
    errs = []
    for n in (16, 32):
        case = _case(keep_n=-1, order=order, nx=n, ny=n, nz=n)
        W = _smooth(case, amp=0.3)
        o = oracle_for(case)
        R = o.rhs(W.copy(), mask=CONV)
        prim = _prims(o.interior(W))
        ex = exact_rhs(prim, (case.lx, case.ly, case.lz), GAMMA, case.mach, case.reynolds,
                       case.prandtl, case.visc_exp, conv=True, visc=False)
        errs.append(np.abs(R - ex).max())
    rate = math.log2(errs[0] / errs[1])
    assert rate > order - 0.6, (errs, rate)
