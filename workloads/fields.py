"""Analytic source fields of the synthetic workloads.

Each field is written once against an array namespace ``xp`` (``numpy`` or
``torch``) so the same expression can be sampled on the CPU or on the device.
A field is used two ways: interpolated at the nodes of a source mesh (the P1
source of the benchmark), or called directly as a point-query black box.

Input generators only; none of the transfer method's arithmetic lives here.
"""
from __future__ import annotations

import numpy as np


def paper_f1(xp, x, y):
    """First smooth test function of the convergence study (cubic polynomial)."""
    return 5.0 * y ** 3 + x ** 2 + 2.0 * y + 3.0


def paper_f2(xp, x, y):
    """Second smooth test function of the convergence study (trigonometric)."""
    return xp.sin(x) * xp.cos(y) + 2.0


def paper_f3(xp, x, y):
    """Third smooth test function of the convergence study (exponential)."""
    return xp.exp(x ** 2) + 2.0 * y


def smooth_2d(xp, x, y):
    """sin(2 pi x) cos(2 pi y) + x^2 / 2 on the unit square; integral 1/6."""
    return xp.sin(2.0 * np.pi * x) * xp.cos(2.0 * np.pi * y) + 0.5 * x * x


def front_2d(xp, x, y):
    """tanh(20 (r - 0.3)) + 0.1 sin(8 pi x), r = |(x,y) - (0.5,0.5)|: a sharp circular front."""
    r = xp.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2)
    return xp.tanh(20.0 * (r - 0.3)) + 0.1 * xp.sin(8.0 * np.pi * x)


def affine(xp, *xs, c0=1.25, c=(0.75, -2.0, 0.5)):
    """An affine field: exactly representable in every P1 space."""
    out = c0 + 0.0 * xs[0]
    for ci, xi in zip(c, xs):
        out = out + ci * xi
    return out


def constant(xp, *xs, c0=2.5):
    return c0 + 0.0 * xs[0]


def gaussian_centers(seed: int = 13, count: int = 8) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(count, 3))


def gaussian_bumps_3d(xp, x, y, z, centers=None):
    """Sum over seeded centres c of exp(-|x - c|^2 / 0.02)."""
    if centers is None:
        centers = gaussian_centers()
    out = 0.0 * x
    for c in centers:
        out = out + xp.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / 0.02)
    return out


def fourier_modes(seed: int = 13, n_fields: int = 64, n_modes: int = 16, kmax: int = 8):
    """Integer wave vectors in {1..kmax}^3, N(0,1) amplitudes, U[0, 2 pi) phases."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, kmax + 1, size=(n_fields, n_modes, 3))
    a = rng.standard_normal(size=(n_fields, n_modes))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=(n_fields, n_modes))
    return k, a, phi


def fourier_fields_3d(xp, x, y, z, modes=None):
    """Stack of fields sum_q a_q cos(2 pi k_q . x + phi_q): shape (F, n)."""
    if modes is None:
        modes = fourier_modes()
    k, a, phi = modes
    outs = []
    for f in range(k.shape[0]):
        acc = 0.0 * x
        for q in range(k.shape[1]):
            arg = 2.0 * np.pi * (k[f, q, 0] * x + k[f, q, 1] * y + k[f, q, 2] * z) + phi[f, q]
            acc = acc + a[f, q] * xp.cos(arg)
        outs.append(acc)
    return xp.stack(outs, 0)


FIELDS = {
    "paper_f1": paper_f1,
    "paper_f2": paper_f2,
    "paper_f3": paper_f3,
    "smooth_2d": smooth_2d,
    "front_2d": front_2d,
    "affine": affine,
    "constant": constant,
    "gaussian_bumps_3d": gaussian_bumps_3d,
    "fourier_fields_3d": fourier_fields_3d,
}


def phase_space(xp, *xs):
    """A distribution-function-like field on [0,1]^d (d >= 2): spatial
    modulation along x_1 times a drifting Gaussian in the other coordinates,
    (1 + 0.3 cos(2 pi x_1)) exp(-sum_{i>1} (x_i - 0.5 - 0.05 sin(2 pi x_1))^2 / 0.08)."""
    x1 = xs[0]
    shift = 0.5 + 0.05 * xp.sin(2.0 * np.pi * x1)
    r2 = 0.0 * x1
    for xi in xs[1:]:
        r2 = r2 + (xi - shift) ** 2
    return (1.0 + 0.3 * xp.cos(2.0 * np.pi * x1)) * xp.exp(-r2 / 0.08)


FIELDS["phase_space"] = phase_space


def phase_space_integral(dim: int) -> float:
    """Integral of phase_space over [0,1]^dim: for fixed x_1 the other
    coordinates separate, each giving G(s) = sqrt(0.08 pi)/2 (erf((1-s)/sqrt(0.08))
    + erf(s/sqrt(0.08))) with s = 0.5 + 0.05 sin(2 pi x_1); the remaining
    one-dimensional integral by adaptive quadrature."""
    from scipy.integrate import quad
    from scipy.special import erf

    c = np.sqrt(0.08)

    def g(x1):
        sh = 0.5 + 0.05 * np.sin(2.0 * np.pi * x1)
        G = 0.5 * np.sqrt(np.pi) * c * (erf((1.0 - sh) / c) + erf(sh / c))
        return (1.0 + 0.3 * np.cos(2.0 * np.pi * x1)) * G ** (dim - 1)

    val, _ = quad(g, 0.0, 1.0, epsabs=0.0, epsrel=1e-13, limit=200)
    return float(val)


def evaluate(name: str, xp, coords):
    """Evaluate a named field at points ``coords`` of shape (n, dim); returns (F, n)."""
    fn = FIELDS[name]
    cols = [coords[:, i] for i in range(coords.shape[1])]
    v = fn(xp, *cols)
    if v.ndim == 1:
        v = v[None, :]
    return v
