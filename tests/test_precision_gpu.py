"""FP32-flux precision form against the FP64 oracle.

The form computes primitives in FP64, converts them once per node and runs
all stencil, flux and viscous arithmetic in FP32; the state, the RK
register and the update are FP64. Its error is bounded by FP32 rounding of
the stencil sums relative to the flux magnitudes, not by the discretisation,
so the tests bound it against both: well below the FP32-epsilon-scaled
flux scale, and far below the sixth-order truncation error of the same RHS
(the difference between the RHS on N and 2N points of the smooth TGV)."""
import math

import numpy as np
import pytest

from paper_2304_05494_amd import inputs, sx
from tests.helpers import oracle_for, rel_err_per_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EPS32 = 2.0 ** -24


def _run_rhs(case, precision):
    h = sx.Handle(case, precision=precision)
    Wn = np.ascontiguousarray(inputs.fields(case))
    W = h.to_layout(Wn)
    h.sx_bind(W)
    R = h.sx_rhs(W)
    torch.cuda.synchronize()
    return Wn, R.cpu().numpy()


def flux_scale(case, Wn):
    """Per conserved variable: the largest |convective flux| over nodes and
    directions, with the pressure measured from the reference value the FP32
    form subtracts (that shift is exact), over the smallest grid spacing.
    The energy scale keeps the full enthalpy: the form adds back H_ref times
    the FP32 mass flux, whose rounding therefore enters the energy RHS
    scaled by H_ref = c_p."""
    g = case.ng
    W = Wn[:, g:-g, g:-g, g:-g]
    rho = W[0]
    u = [W[1] / rho, W[2] / rho, W[3] / rho]
    q2 = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    p = (case.gamma - 1) * (W[4] - 0.5 * rho * q2)
    gm2 = case.gamma * case.mach ** 2
    cp = 1.0 / ((case.gamma - 1) * case.mach ** 2)
    H = (W[4] + p) / rho - cp
    dp = np.abs(p - 1.0 / gm2)
    un = np.max([np.abs(x) for x in u], axis=0)
    F = [np.abs(rho * un).max(),
         (rho * un * un + dp).max(), (rho * un * un + dp).max(), (rho * un * un + dp).max(),
         np.abs(rho * un * H).max() + cp * np.abs(rho * un).max()]
    if case.ymap == inputs.Y_UNIFORM:
        h = min(case.lx / case.nx, case.ly / case.ny, case.lz / case.nz)
    else:
        y = inputs._y_nodes(case, np.arange(-1, case.ny + 1))
        h = min(case.lx / case.nx, np.diff(y).min(), case.lz / case.nz)
    return np.array(F) / h


@pytest.mark.parametrize("case", [inputs.tgv_case(32), inputs.channel_case(70, 36, 20),
                                  inputs.tgv_case(24, central_order=2, visc_order=2),
                                  inputs.tgv_case(24, central_order=4, visc_order=4),
                                  inputs.tgv_case(24, central_order=8, visc_order=8),
                                  inputs.channel_case(70, 36, 20, central_order=8, visc_order=8)],
                         ids=lambda c: f"{c.name}-C{c.central_order}")
def test_fp32_flux_rhs_error_is_fp32_rounding(case):
    Wn, got = _run_rhs(case, sx.SX_FP32_FLUX)
    ref = oracle_for(case).rhs(Wn.copy())
    err = np.abs(got - ref).max(axis=(1, 2, 3))
    bound = 64 * EPS32 * flux_scale(case, Wn)
    print("FP32-flux RHS max error per field:", err, "bound 64 eps32 F/h:", bound)
    assert np.all(err < bound), (err, bound)
    assert err.max() > 0.0       # really computed in FP32


def test_fp32_flux_error_far_below_truncation_error():
    """TGV: per conserved variable, the FP32 error of the RHS is at least ten
    times smaller than the C6/V6 truncation error (RHS on 16^3 vs the same
    nodes of the 32^3 grid)."""
    c32 = inputs.tgv_case(32)
    c16 = inputs.tgv_case(16)
    Wn32, r32 = _run_rhs(c32, sx.SX_FP32_FLUX)
    ref32 = oracle_for(c32).rhs(Wn32.copy())
    ref16 = oracle_for(c16).rhs(np.ascontiguousarray(inputs.fields(c16)))
    trunc = np.abs(ref16 - ref32[:, ::2, ::2, ::2]).max(axis=(1, 2, 3))
    fp32 = np.abs(r32 - ref32).max(axis=(1, 2, 3))
    print("per field: truncation", trunc, "fp32", fp32, "ratio", fp32 / trunc)
    assert np.all(fp32 < 0.1 * trunc)


def test_fp32_flux_steps_error_bound():
    """Channel block (walls, stretching) advanced 20 RK3 steps in the
    FP32-flux form vs the FP64 oracle: per-field error bounded."""
    case = inputs.channel_case(70, 36, 20)
    o = oracle_for(case)
    Wn = np.ascontiguousarray(inputs.fields(case))
    dt = o.compute_dt(Wn.copy(), case.cfl)
    h = sx.Handle(case, precision=sx.SX_FP32_FLUX)
    h.sx_bind(h.to_layout(Wn))
    for _ in range(20):
        h.sx_rk3_step(dt)
    torch.cuda.synchronize()
    got = h.interior(h.state)
    Wo = Wn.copy()
    Rp = np.zeros((5, case.nz, case.ny, case.nx))
    for _ in range(20):
        o.rk3_step(Wo, Rp, dt)
    ref = o.interior(Wo)
    err = rel_err_per_field(got, ref)
    l2 = np.sqrt(((got - ref) ** 2).mean(axis=(1, 2, 3))) / np.sqrt((ref ** 2).mean(axis=(1, 2, 3)))
    print("FP32-flux after 20 steps: Linf", err, "L2", l2)
    assert np.all(err < 1e-5), err


def test_fp32_flux_hybrid_rhs_error():
    """Shock/boundary-layer block with the sensor and WENO-5 (FP32 face
    fluxes, FP64 flags): per conserved variable the RHS error against the
    FP64 oracle stays within 1024 FP32 epsilons of the flux scale (full
    pressure: the WENO flux carries it unshifted). The nonlinear weights
    amplify rounding where the smoothness indicators are near the WENO
    epsilon, hence the wider bound than for the central form."""
    case = inputs.shock_bl_case(200, 64, 12)
    Wn, got = _run_rhs(case, sx.SX_FP32_FLUX)
    ref = oracle_for(case).rhs(Wn.copy())
    err = np.abs(got - ref).max(axis=(1, 2, 3))
    F = flux_scale(case, Wn)
    F[1:4] += (1.0 / (case.gamma * case.mach ** 2)) / min(case.lx / case.nx, case.lz / case.nz)
    bound = 1024 * EPS32 * F
    print("FP32-flux hybrid RHS max error per field:", err, "relative to flux scale:", err / F)
    assert np.all(err < bound), (err, bound)
    assert err.max() > 0.0
