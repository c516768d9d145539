"""Seeded synthetic inputs shaped like the paper's per-GPU blocks.

This module serves both the HIP path and the oracle, so it holds none of the
solver's arithmetic: only grid descriptions (plain data) and initial fields.
Fields are returned over the whole ghosted index range in a neutral layout
``float64[5, nz+2g, ny+2g, nx+2g]`` (x fastest, node (i,j,k) at index
(k+g, j+g, i+g)) holding the conserved variables (rho, rho u, rho v, rho w,
rho E); ghost entries carry the analytic initial data, which a solver
overwrites except on caller-frozen (Dirichlet) faces.

The paper runs its benchmarks on a 420x250x320 block without stating the
flow (Section 4.1); it uses no public dataset. The cases below stand in for
that block: a Taylor-Green vortex, a channel-like block with isothermal walls,
a shock/boundary-layer block and a batch of uneven periodic boxes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

PERIODIC, WALL, EXTRAP, FROZEN = 0, 1, 2, 3
Y_UNIFORM, Y_TANH2, Y_TANH1 = 0, 1, 2


@dataclass(frozen=True)
class Case:
    """Grid, gas and scheme description (plain data)."""
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    y0: float = 0.0
    ymap: int = Y_UNIFORM
    beta: float = 0.0
    bc: tuple = (PERIODIC,) * 6
    gamma: float = 1.4
    mach: float = 0.1
    reynolds: float = 1600.0
    prandtl: float = 0.72
    visc_exp: float = 0.76
    t_wall: float = 1.0
    central_order: int = 6
    weno_order: int = 5
    visc_order: int = 6
    sensor: int = 0
    sensor_thr: float = 0.5
    sensor_eps: float = 1.0
    weno_eps: float = 1e-6
    central_flux: int = 0          # 0 split form (Pirozzoli), 1 KEEP-n
    keep_n: int = 0                # KEEP-n: log-mean series terms beyond the first
    bulk_forcing: int = 0          # 1: uniform streamwise force holding the bulk momentum
    thermo: int = 0                # 1: thermally perfect gas (NASA polynomial c_p(T))
    nasa: tuple = (3.5, 0.0, 0.0, 0.0, 0.0)   # c_p/R = sum_k nasa[k] (T t_ref)^k
    t_ref: float = 300.0           # kelvin at nondimensional T = 1
    cfl: float = 0.5
    steps: int = 10
    seed: int | None = None
    extra: dict = field(default_factory=dict, compare=False, hash=False)

    @property
    def ng(self) -> int:
        return max(self.central_order // 2, self.visc_order // 2, (self.weno_order + 1) // 2)

    @property
    def points(self) -> int:
        return self.nx * self.ny * self.nz

    def resized(self, nx: int, ny: int, nz: int) -> "Case":
        return replace(self, nx=nx, ny=ny, nz=nz, name=f"{self.name}@{nx}x{ny}x{nz}")


def _y_nodes(case: Case, j: np.ndarray) -> np.ndarray:
    """Node coordinates of the y mapping (input-side copy, used only to
    shape initial profiles)."""
    if case.ymap == Y_TANH2:
        eta = -1.0 + (2.0 * j + 1.0) / case.ny
        return 0.5 * case.ly * np.tanh(case.beta * eta) / math.tanh(case.beta)
    if case.ymap == Y_TANH1:
        eta = (j + 0.5) / case.ny
        return case.ly * (1.0 - np.tanh(case.beta * (1.0 - eta)) / math.tanh(case.beta))
    return case.y0 + j * (case.ly / case.ny)


def _coords(case: Case):
    g = case.ng
    i = np.arange(-g, case.nx + g, dtype=np.float64)
    j = np.arange(-g, case.ny + g, dtype=np.float64)
    k = np.arange(-g, case.nz + g, dtype=np.float64)
    x = i * (case.lx / case.nx)
    y = _y_nodes(case, j)
    z = k * (case.lz / case.nz)
    return x, y, z


def conserved(gamma: float, rho, u, v, w, p) -> np.ndarray:
    """Conserved vector from density, velocity and pressure (definition of
    total energy for a calorically perfect gas)."""
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E]).astype(np.float64)


# ---------------------------------------------------------------------------
# Config 1: compressible Taylor-Green vortex on [0, 2 pi)^3
# ---------------------------------------------------------------------------
def tgv_case(n: int = 32, mach: float = 0.1, **kw) -> Case:
    two_pi = 2.0 * math.pi
    return Case(name=f"tgv{n}", nx=n, ny=n, nz=n, lx=two_pi, ly=two_pi, lz=two_pi,
                mach=mach, reynolds=1600.0, steps=10, **kw)


def tgv_fields(case: Case) -> np.ndarray:
    """u = sin x cos y cos z, v = -cos x sin y cos z, w = 0,
    p = 1/(gamma M^2) + (cos 2x + cos 2y)(cos 2z + 2)/16, T = 1 (so
    rho = gamma M^2 p). Seed-free."""
    x, y, z = _coords(case)
    # one period per box length (the cubic 2 pi box gives the standard TGV)
    kx, ky, kz = (2.0 * math.pi / L for L in (case.lx, case.ly, case.lz))
    Z, Y, X = np.meshgrid(kz * z, ky * y, kx * x, indexing="ij")
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -(kx / ky) * np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(u)
    g = case.gamma
    p = 1.0 / (g * case.mach ** 2) + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    rho = g * case.mach ** 2 * p
    return conserved(g, rho, u, v, w, p)


# ---------------------------------------------------------------------------
# Config 2: channel-like block, periodic x/z, isothermal walls in y
# ---------------------------------------------------------------------------
def channel_case(nx: int = 512, ny: int = 256, nz: int = 256, **kw) -> Case:
    return Case(name=f"channel{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                lx=2.0 * math.pi, ly=2.0, lz=math.pi, ymap=Y_TANH2, beta=1.8,
                bc=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC),
                mach=1.5, reynolds=6000.0, t_wall=1.0, steps=20, seed=2, **kw)


def channel_fields(case: Case, noise: float = 0.05) -> np.ndarray:
    """Laminar profile u = 1.5 (1 - y^2) (bulk velocity 1), rho = T = 1,
    plus i.i.d. Gaussian velocity noise of standard deviation noise*U_b,
    damped by (1 - y^2) so the walls stay no-slip."""
    rng = np.random.Generator(np.random.PCG64(case.seed))
    x, y, z = _coords(case)
    shape = (z.size, y.size, x.size)
    yy = np.broadcast_to(y[None, :, None], shape)
    damp = np.clip(1.0 - yy * yy, 0.0, None)
    u = 1.5 * damp + noise * damp * rng.standard_normal(shape)
    v = noise * damp * rng.standard_normal(shape)
    w = noise * damp * rng.standard_normal(shape)
    g = case.gamma
    rho = np.ones(shape)
    p = np.full(shape, 1.0 / (g * case.mach ** 2))
    return conserved(g, rho, u, v, w, p)


# ---------------------------------------------------------------------------
# Config 3: shock / boundary-layer block
# ---------------------------------------------------------------------------
def shock_bl_case(nx: int = 1024, ny: int = 256, nz: int = 128, **kw) -> Case:
    M = 2.0
    pr = 0.72
    gam = 1.4
    t_rec = 1.0 + math.sqrt(pr) * (gam - 1.0) / 2.0 * M * M
    return Case(name=f"shockbl{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                lx=60.0, ly=10.0, lz=6.0, ymap=Y_TANH1, beta=1.8,
                bc=(FROZEN, EXTRAP, WALL, FROZEN, PERIODIC, PERIODIC),
                mach=M, reynolds=1.0e4, prandtl=pr, t_wall=t_rec, sensor=1,
                steps=20, seed=3, **kw)


def _blasius(eta_max: float = 12.0, n: int = 4001):
    """Incompressible Blasius f''' + f f''/2 = 0 by shooting (RK4)."""
    def integrate(fpp0):
        h = eta_max / (n - 1)
        y = np.array([0.0, 0.0, fpp0])
        out = np.zeros((n, 3))
        out[0] = y
        f = lambda s: np.array([s[1], s[2], -0.5 * s[0] * s[2]])
        for m in range(1, n):
            k1 = f(y); k2 = f(y + 0.5 * h * k1); k3 = f(y + 0.5 * h * k2); k4 = f(y + h * k3)
            y = y + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
            out[m] = y
        return out
    lo, hi = 0.2, 0.5
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if integrate(mid)[-1, 1] > 1.0:
            hi = mid
        else:
            lo = mid
    sol = integrate(0.5 * (lo + hi))
    eta = np.linspace(0.0, eta_max, n)
    return eta, sol[:, 1]


def _oblique_shock(M1: float, deflection_deg: float, gam: float):
    """Weak oblique shock for a given flow deflection (theta-beta-M)."""
    th = math.radians(deflection_deg)
    def tb(b):
        return math.atan(2.0 / math.tan(b) * (M1 ** 2 * math.sin(b) ** 2 - 1.0)
                         / (M1 ** 2 * (gam + math.cos(2 * b)) + 2.0)) - th
    lo, hi = math.asin(1.0 / M1) + 1e-9, math.radians(64.0)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if tb(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    b = 0.5 * (lo + hi)
    mn1 = M1 * math.sin(b)
    p21 = 1.0 + 2.0 * gam / (gam + 1.0) * (mn1 ** 2 - 1.0)
    r21 = (gam + 1.0) * mn1 ** 2 / ((gam - 1.0) * mn1 ** 2 + 2.0)
    T21 = p21 / r21
    mn2 = math.sqrt((1.0 + 0.5 * (gam - 1.0) * mn1 ** 2) / (gam * mn1 ** 2 - 0.5 * (gam - 1.0)))
    M2 = mn2 / math.sin(b - th)
    return dict(beta=b, p21=p21, r21=r21, T21=T21, M2=M2)


def _box_filter(a: np.ndarray, axes=(0, 1, 2)) -> np.ndarray:
    for ax in axes:
        a = (np.roll(a, 1, ax) + a + np.roll(a, -1, ax)) / 3.0
    return a


def shock_bl_fields(case: Case, noise: float = 0.03, deflection: float = 8.0,
                    filter_passes: int = 2) -> np.ndarray:
    """Mach-2 flat-plate boundary layer (Blasius profile mapped by
    Howarth-Dorodnitsyn with the Crocco-Busemann temperature, thickness 1 at
    the inflow) with an oblique shock of the given flow deflection entering at
    (x=0, y=ly); 3 % filtered velocity noise inside the layer."""
    g = case.gamma
    M = case.mach
    x, y, z = _coords(case)
    shape = (z.size, y.size, x.size)
    eta, fp = _blasius()
    Tw = case.t_wall
    # Crocco-Busemann: T = Tw + (1 - Tw) u + (Tr - 1 - (Tr-1)) ... with Tr = Tw
    Tu = Tw - (Tw - 1.0) * fp * fp
    ycomp = np.concatenate([[0.0], np.cumsum(0.5 * (Tu[1:] + Tu[:-1]) * np.diff(eta))])
    d99 = np.interp(0.99, fp, ycomp)
    ys = ycomp / d99
    yy = np.clip(y, 0.0, None)
    u_prof = np.interp(yy, ys, fp, right=1.0)
    T_prof = Tw - (Tw - 1.0) * u_prof * u_prof
    u = np.broadcast_to(u_prof[None, :, None], shape).copy()
    T = np.broadcast_to(T_prof[None, :, None], shape).copy()
    v = np.zeros(shape)
    w = np.zeros(shape)
    p = np.full(shape, 1.0 / (g * M * M))
    sh = _oblique_shock(M, deflection, g)
    X = np.broadcast_to(x[None, None, :], shape)
    Y = np.broadcast_to(y[None, :, None], shape)
    above = Y > case.ly - X * math.tan(sh["beta"])
    U2 = sh["M2"] * math.sqrt(sh["T21"]) / M  # |u2| / U_inf (c2 / c_inf = sqrt(T2/T1))
    th = math.radians(deflection)
    u = np.where(above, U2 * math.cos(th), u)
    v = np.where(above, -U2 * math.sin(th), v)
    T = np.where(above, sh["T21"], T)
    p = np.where(above, p * sh["p21"], p)
    rng = np.random.Generator(np.random.PCG64(case.seed))
    damp = np.broadcast_to((u_prof * (1.0 - u_prof) * 4.0)[None, :, None], shape)
    nz = [_box_filter(rng.standard_normal(shape)) for _ in range(3)]
    for _ in range(filter_passes - 1):
        nz = [_box_filter(a) for a in nz]
    scale = noise / max(1e-30, float(np.std(nz[0])))
    u = u + scale * damp * nz[0]
    v = v + scale * damp * nz[1]
    w = w + scale * damp * nz[2]
    rho = g * M * M * p / T
    return conserved(g, rho, u, v, w, p)


# ---------------------------------------------------------------------------
# Config 4: config 2 in the FP32-flux precision form (same fields)
# ---------------------------------------------------------------------------
def precision_case(nx: int = 512, ny: int = 256, nz: int = 256) -> Case:
    return replace(channel_case(nx, ny, nz), steps=100, name=f"channel-fp32flux{nx}x{ny}x{nz}")


# ---------------------------------------------------------------------------
# Config 5: batch of uneven periodic boxes
# ---------------------------------------------------------------------------
BOX_SIZES = ((32, 32, 32), (48, 48, 48), (64, 64, 64), (96, 96, 96), (128, 64, 64))


def batch_cases(nbox: int = 48, seed: int = 5):
    """Sizes drawn uniformly from BOX_SIZES, Mach in [0.1, 0.5], type TGV or
    decaying turbulence with probability 1/2. Domain 2 pi per unit of the
    largest dimension so the spacing is uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cases = []
    for b in range(nbox):
        nx, ny, nz = BOX_SIZES[int(rng.integers(len(BOX_SIZES)))]
        mach = float(rng.uniform(0.1, 0.5))
        kind = "tgv" if rng.random() < 0.5 else "hit"
        h = 2.0 * math.pi / max(nx, ny, nz)
        cases.append(Case(name=f"box{b}-{kind}{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                          lx=nx * h, ly=ny * h, lz=nz * h, mach=mach, reynolds=1600.0,
                          steps=20, seed=5000 + b, extra={"kind": kind}))
    return cases


def hit_fields(case: Case, k0: float = 4.0) -> np.ndarray:
    """Solenoidal random Fourier velocity with E(k) ~ k^4 exp(-2 k^2/k0^2),
    rms velocity 1 (reference velocity), rho = T = 1."""
    rng = np.random.Generator(np.random.PCG64(case.seed))
    nx, ny, nz = case.nx, case.ny, case.nz
    kx = np.fft.fftfreq(nx, d=case.lx / nx / (2 * math.pi))
    ky = np.fft.fftfreq(ny, d=case.ly / ny / (2 * math.pi))
    kz = np.fft.fftfreq(nz, d=case.lz / nz / (2 * math.pi))
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    kk = np.sqrt(k2)
    amp = np.where(kk > 0, np.sqrt(kk ** 4 * np.exp(-2.0 * k2 / k0 ** 2)) / np.maximum(kk, 1e-30), 0.0)
    comps = []
    for _ in range(3):
        comps.append(amp * (rng.standard_normal(k2.shape) + 1j * rng.standard_normal(k2.shape)))
    ax, ay, az = comps
    kd = (KX * ax + KY * ay + KZ * az) / np.where(k2 > 0, k2, 1.0)
    ax, ay, az = ax - KX * kd, ay - KY * kd, az - KZ * kd
    u, v, w = (np.real(np.fft.ifftn(a)) for a in (ax, ay, az))
    rms = math.sqrt(float(np.mean(u * u + v * v + w * w)) / 3.0)
    u, v, w = u / rms, v / rms, w / rms
    g = case.ng
    pad = lambda a: np.pad(a, g, mode="wrap")
    u, v, w = pad(u), pad(v), pad(w)
    gam = case.gamma
    rho = np.ones_like(u)
    p = np.full_like(u, 1.0 / (gam * case.mach ** 2))
    return conserved(gam, rho, u, v, w, p)


def fields(case: Case) -> np.ndarray:
    """Initial conserved fields for any case built by this module."""
    if case.name.startswith("tgv") or case.extra.get("kind") == "tgv":
        return tgv_fields(case)
    if case.extra.get("kind") == "hit":
        return hit_fields(case)
    if case.name.startswith("channel"):
        return channel_fields(case)
    if case.name.startswith("shockbl"):
        return shock_bl_fields(case)
    raise ValueError(f"no generator for case {case.name}")
