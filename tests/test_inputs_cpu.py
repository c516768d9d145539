"""CPU checks of the seeded synthetic inputs against the physics they are
built from: the oblique shock of the shock/boundary-layer block satisfies the
Rankine-Hugoniot jump conditions in the shock-normal frame and turns the flow
by the stated deflection; the decaying-turbulence field is solenoidal with
unit rms velocity; the Taylor-Green field is isothermal; the channel field
has unit bulk velocity and no-slip walls; the batch draw is deterministic and
stays inside the stated size / Mach ranges."""
import math

import numpy as np
import pytest

from paper_2304_05494_amd import inputs


def _prims(W, gamma):
    rho = W[0]
    u, v, w = W[1] / rho, W[2] / rho, W[3] / rho
    p = (gamma - 1.0) * (W[4] - 0.5 * rho * (u * u + v * v + w * w))
    return rho, u, v, w, p


def test_oblique_shock_satisfies_rankine_hugoniot():
    """Pre- and post-shock states of the generated block: mass, normal
    momentum and total enthalpy fluxes through the shock agree, the
    tangential velocity is continuous, the post-shock flow is turned by 8
    degrees; the weak-shock angle for M = 2 is 37.2 degrees."""
    case = inputs.shock_bl_case(64, 48, 4)
    g = case.gamma
    W = inputs.fields(case)
    ng = case.ng
    rho, u, v, w, p = (a[ng, :, :] for a in _prims(W, g))   # one z plane, ghosts included
    sh = inputs._oblique_shock(case.mach, 8.0, g)
    beta = sh["beta"]
    assert math.degrees(beta) == pytest.approx(37.21, abs=0.01)
    x, y, _ = inputs._coords(case)
    X, Y = np.meshgrid(x, y)
    shocked = Y > case.ly - X * math.tan(beta)
    free = Y > 5.0                                            # well outside the boundary layer
    above, below_free = shocked & free, (~shocked) & free
    assert above.any() and below_free.any()
    # uniform states on each side (the noise is confined to the layer)
    s1 = [a[below_free] for a in (rho, u, v, p)]
    s2 = [a[above] for a in (rho, u, v, p)]
    for a in s1 + s2:
        assert np.ptp(a) < 1e-12 * max(1.0, np.abs(a).max())
    r1, u1, v1, p1 = (a[0] for a in s1)
    r2, u2, v2, p2 = (a[0] for a in s2)
    assert math.degrees(math.atan2(-v2, u2)) == pytest.approx(8.0, abs=1e-9)
    # shock-normal frame: the shock runs down and to the right at angle beta
    n = np.array([math.sin(beta), math.cos(beta)])             # unit normal (upstream -> downstream)
    t = np.array([math.cos(beta), -math.sin(beta)])            # unit tangent
    un1, un2 = u1 * n[0] + v1 * n[1], u2 * n[0] + v2 * n[1]
    ut1, ut2 = u1 * t[0] + v1 * t[1], u2 * t[0] + v2 * t[1]
    h = lambda r, pp: g / (g - 1.0) * pp / r
    assert r1 * un1 == pytest.approx(r2 * un2, rel=1e-12)
    assert p1 + r1 * un1 ** 2 == pytest.approx(p2 + r2 * un2 ** 2, rel=1e-12)
    assert h(r1, p1) + 0.5 * un1 ** 2 == pytest.approx(h(r2, p2) + 0.5 * un2 ** 2, rel=1e-12)
    assert ut1 == pytest.approx(ut2, rel=1e-12)
    assert p2 / p1 == pytest.approx(1.540, abs=1e-3)


def test_decaying_turbulence_is_solenoidal_with_unit_rms():
    case = [c for c in inputs.batch_cases(48) if c.extra["kind"] == "hit" and c.nx == 32][0]
    W = inputs.fields(case)
    g = case.ng
    rho, u, v, w, p = (a[g:-g, g:-g, g:-g] for a in _prims(W, case.gamma))
    rms = math.sqrt(float(np.mean(u * u + v * v + w * w)) / 3.0)
    assert rms == pytest.approx(1.0, rel=1e-12)
    k = [np.fft.fftfreq(n, d=L / n / (2 * math.pi)) for n, L in ((case.nz, case.lz), (case.ny, case.ly), (case.nx, case.lx))]
    KZ, KY, KX = np.meshgrid(*k, indexing="ij")
    div = KX * np.fft.fftn(u) + KY * np.fft.fftn(v) + KZ * np.fft.fftn(w)
    # the derivative of a real field's Nyquist modes is not defined: leave
    # out every wavevector with a Nyquist component
    nyq = np.zeros(div.shape, dtype=bool)
    for ax, n in enumerate(div.shape):
        idx = [slice(None)] * 3
        idx[ax] = n // 2
        nyq[tuple(idx)] = True
    assert np.abs(div[~nyq]).max() < 1e-10 * np.abs(np.fft.fftn(u)).max()
    assert np.ptp(rho) == 0.0 and np.ptp(p) < 1e-12 * p.max()


def test_taylor_green_is_isothermal():
    case = inputs.tgv_case(16, mach=0.2)
    rho, u, v, w, p = _prims(inputs.fields(case), case.gamma)
    T = case.gamma * case.mach ** 2 * p / rho
    assert np.abs(T - 1.0).max() < 1e-13
    assert np.abs(w).max() == 0.0


def test_channel_bulk_velocity_and_walls():
    case = inputs.channel_case(64, 48, 16)
    rho, u, v, w, p = _prims(inputs.fields(case), case.gamma)
    g = case.ng
    j = np.arange(case.ny)
    y = inputs._y_nodes(case, j)
    ui = u[g:-g, g:-g, g:-g]
    laminar = 1.5 * (1.0 - y ** 2)
    # bulk velocity: midpoint rule in the mapping coordinate eta (nodes sit
    # at cell centres of eta in [-1, 1]), dy/deta from the tanh mapping
    eta = -1.0 + (2.0 * j + 1.0) / case.ny
    dy = 0.5 * case.ly * case.beta / np.cosh(case.beta * eta) ** 2 / math.tanh(case.beta)
    assert float(np.sum(laminar * dy) * (2.0 / case.ny)) / case.ly == pytest.approx(1.0, abs=1e-3)
    # the noise is 5 % of the bulk velocity, damped by (1 - y^2) toward the walls
    z = (ui - laminar[None, :, None]) / (0.05 * (1.0 - y ** 2))[None, :, None]
    assert abs(float(z.std()) - 1.0) < 0.02 and abs(float(z.mean())) < 0.02
    assert np.ptp(rho) == 0.0 and np.abs(v[g:-g, g:-g, g:-g]).max() < 0.05 * 6


def test_batch_draw_is_deterministic_and_in_range():
    a, b = inputs.batch_cases(48), inputs.batch_cases(48)
    assert [(c.nx, c.ny, c.nz, c.mach, c.extra["kind"]) for c in a] == \
           [(c.nx, c.ny, c.nz, c.mach, c.extra["kind"]) for c in b]
    sizes = set(inputs.BOX_SIZES)
    for c in a:
        assert (c.nx, c.ny, c.nz) in sizes
        assert 0.1 <= c.mach <= 0.5
        h = c.lx / c.nx
        assert c.ly / c.ny == pytest.approx(h) and c.lz / c.nz == pytest.approx(h)
    assert {c.extra["kind"] for c in a} == {"tgv", "hit"}
