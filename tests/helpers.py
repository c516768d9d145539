"""Test-side helpers: map input cases to oracle parameters, independent exact
references (spectral derivatives of the divergence-form equations), and the
parity metric."""
from __future__ import annotations

import numpy as np

import oracle as O
from paper_2304_05494_amd import inputs


def oracle_params(case: inputs.Case, **over) -> O.Params:
    kw = {k: getattr(case, k) for k in O.Params.__dataclass_fields__}
    kw.update(over)
    return O.Params(**kw)


def oracle_for(case: inputs.Case, **over) -> O.Oracle:
    return O.Oracle(oracle_params(case, **over))


# ---------------------------------------------------------------------------
# Exact right-hand side on a uniform periodic grid, written independently of
# the oracle: conservative (divergence) form of the compressible Navier-Stokes
# equations, derivatives by FFT (exact for resolved trigonometric
# polynomials, spectrally accurate for smooth periodic data).
# ---------------------------------------------------------------------------
def spectral_deriv(f: np.ndarray, axis: int, length: float) -> np.ndarray:
    n = f.shape[axis]
    k = np.fft.fftfreq(n, d=length / n / (2 * np.pi))
    shape = [1] * f.ndim
    shape[axis] = n
    kk = (1j * k).reshape(shape)
    if n % 2 == 0:
        kk = kk.copy()
        idx = [slice(None)] * f.ndim
        idx[axis] = n // 2
        kk[tuple(idx)] = 0.0
    return np.real(np.fft.ifft(kk * np.fft.fft(f, axis=axis), axis=axis))


def exact_rhs(prim, lengths, gamma, mach, re, pr, s, conv=True, visc=True):
    """prim = (rho, u, v, w, p) interior arrays [nz, ny, nx];
    lengths = (lx, ly, lz). Returns dW/dt as [5, nz, ny, nx]."""
    rho, u, v, w, p = prim
    lx, ly, lz = lengths
    D = [lambda f: spectral_deriv(f, 2, lx), lambda f: spectral_deriv(f, 1, ly),
         lambda f: spectral_deriv(f, 0, lz)]
    vel = [u, v, w]
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    R = np.zeros((5,) + rho.shape)
    if conv:
        for d in range(3):
            ud = vel[d]
            R[0] -= D[d](rho * ud)
            for i in range(3):
                R[1 + i] -= D[d](rho * ud * vel[i] + (p if i == d else 0.0))
            R[4] -= D[d](ud * (E + p))
    if visc:
        T = gamma * mach ** 2 * p / rho
        mu = T ** s / re
        kc = mu / ((gamma - 1.0) * mach ** 2 * pr)
        g = [[D[j](vel[i]) for j in range(3)] for i in range(3)]
        div = g[0][0] + g[1][1] + g[2][2]
        tau = [[mu * (g[i][j] + g[j][i] - (2.0 / 3.0 * div if i == j else 0.0)) for j in range(3)]
               for i in range(3)]
        for i in range(3):
            R[1 + i] += sum(D[j](tau[i][j]) for j in range(3))
        for j in range(3):
            R[4] += D[j](sum(vel[i] * tau[i][j] for i in range(3)) + kc * D[j](T))
    return R


def embed(Wint: np.ndarray, ng: int) -> np.ndarray:
    """Interior conserved array -> oracle ghosted array (ghosts zero)."""
    nz, ny, nx = Wint.shape[1:]
    W = np.zeros((5, nz + 2 * ng, ny + 2 * ng, nx + 2 * ng))
    W[:, ng:ng + nz, ng:ng + ny, ng:ng + nx] = Wint
    return W


def rel_err_per_field(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """max|a-b| / max|b| per conserved variable; momentum components share
    the max momentum magnitude as denominator."""
    out = np.zeros(5)
    mom = np.sqrt((b[1:4] ** 2).sum(axis=0)).max()
    for v in range(5):
        den = mom if v in (1, 2, 3) else np.abs(b[v]).max()
        out[v] = np.abs(a[v] - b[v]).max() / max(den, 1e-300)
    return out
