"""Seeded synthetic workloads: initial fields and moment fields.

This module holds no arithmetic of the method itself (no quasiequilibrium,
no entropy, no collision): it only produces the macroscopic initial fields
(rho0, u0[, 2E0]), moment fields M and the parameter sets of the
configurations, so that the GPU library and the CPU oracle can be fed the
same inputs.  Noise comes from SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014) evaluated as a
counter-based generator on (seed, component, site).
"""
from __future__ import annotations

import math

import numpy as np

# boundary-condition codes (same values as the C-ABI and the oracle)
PERIODIC, ZEROGRAD, FREESLIP, INLET_EQ, OUTLET_EQ, OUTLET_EQ_PREV = 0, 1, 2, 3, 4, 5
QE_POLY, QE_ENTROPIC_MM, QE_ENTROPIC_M = 0, 1, 2

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to a uint64 counter array."""
    with np.errstate(over="ignore"):
        z = x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def noise(seed: int, component: int, n: int) -> np.ndarray:
    """Uniform noise in [-1, 1) for sites 0..n-1 of one (seed, component)."""
    site = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = (np.uint64(seed) * np.uint64(0x9E3779B97F4A7C15)) ^ (np.uint64(component) << np.uint64(48))
        z = splitmix64(site ^ key)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


# ---------------------------------------------------------------------------
# Configurations
# ---------------------------------------------------------------------------

def shock_tube(nx: int = 800, split: int = 400, rho_left: float = 1.0, rho_right: float = 0.5,
               nu: float = 1e-9, delta: float = 1e-3, k: int = 4, inclusive: bool = False):
    """1-D shock tube: rho = rho_left for x < split (x <= split if inclusive),
    rho_right otherwise, u = 0; zero-gradient ends; D1Q3, FP64."""
    x = np.arange(nx)
    left = (x <= split) if inclusive else (x < split)
    rho = np.where(left, rho_left, rho_right).astype(np.float64).reshape(1, nx)
    u = np.zeros((1, 1, nx))
    cfg = dict(Q=3, qe=QE_POLY, nx=nx, ny=1, nu=nu, delta=delta, k=k,
               bc=(ZEROGRAD, ZEROGRAD, PERIODIC, PERIODIC))
    return cfg, rho, u


def cylinder(nx: int = 1200, ny: int = 400, side: int = 40, centre=(300, 200), u_inf: float = 0.05,
             re: float = 1000.0, delta: float = 1e-3, k: int = 64, seed: int = 2,
             noise_amp: float = 1e-4, qe: int = QE_POLY):
    """Flow past a square cylinder: solid x in [cx - side/2, cx + side/2),
    same in y; inlet equilibrium at the west, zero-gradient east, free-slip
    south and north; u = (u_inf, 0) + noise_amp * xi on fluid, 0 in solid;
    nu = u_inf * side / Re."""
    x0, y0 = centre[0] - side // 2, centre[1] - side // 2
    n = nx * ny
    rho = np.ones((ny, nx))
    u = np.zeros((2, ny, nx))
    u[0] = u_inf + noise_amp * noise(seed, 1, n).reshape(ny, nx)
    u[1] = noise_amp * noise(seed, 2, n).reshape(ny, nx)
    u[:, y0:y0 + side, x0:x0 + side] = 0.0
    nu = u_inf * side / re
    cfg = dict(Q=9, qe=qe, nx=nx, ny=ny, nu=nu, delta=delta, k=k,
               bc=(INLET_EQ, ZEROGRAD, FREESLIP, FREESLIP), inlet_rho=1.0, inlet_u=(u_inf, 0.0),
               solid=(x0, y0, side, side))
    return cfg, rho, u


def cylinder_paper(re: float, L: int = 20, u_inf: float = 0.05, seed: int = 2, noise_amp: float = 1e-4,
                   qe: int = QE_ENTROPIC_MM, outlet: int = ZEROGRAD):
    """The square-cylinder channel of Sec. 4.2: 30L x 25L sites, side L, centre
    10.5L from the inlet on the centre line (solid x in [10.5L - L/2,
    10.5L + L/2), y in [12.5L - L/2, 12.5L + L/2)); (k, delta) = (L/2, 1e-3);
    inlet quasiequilibrium at (1, u_inf); outlet zero-gradient (default) or
    OUTLET_EQ, the paper's quasiequilibrium of the penultimate column;
    free-slip walls; nu = u_inf L / Re; u = (u_inf, 0) + noise_amp * xi on
    fluid, 0 in the solid.  Returns (cfg, rho, u, meta) with meta the
    monitoring point (4L, -2L) from the centre and the run length
    1250 L / u_inf."""
    nx, ny = 30 * L, 25 * L
    x0, y0 = (21 * L) // 2 - L // 2, ny // 2 - L // 2
    n = nx * ny
    rho = np.ones((ny, nx))
    u = np.zeros((2, ny, nx))
    u[0] = u_inf + noise_amp * noise(seed, 1, n).reshape(ny, nx)
    u[1] = noise_amp * noise(seed, 2, n).reshape(ny, nx)
    u[:, y0:y0 + L, x0:x0 + L] = 0.0
    cfg = dict(Q=9, qe=qe, nx=nx, ny=ny, nu=u_inf * L / re, delta=1e-3, k=L // 2,
               bc=(INLET_EQ, outlet, FREESLIP, FREESLIP), inlet_rho=1.0, inlet_u=(u_inf, 0.0),
               solid=(x0, y0, L, L))
    meta = dict(L=L, u_inf=u_inf, probe=(x0 + L // 2 + 4 * L, y0 + L // 2 - 2 * L),
                t_max=int(round(1250 * L / u_inf)), window=0.25)
    return cfg, rho, u, meta


def shear_layer(nx: int = 8192, ny: int = 4096, seed: int = 3, nu: float = 1e-6,
                delta: float = 1e-4, k: int = 4096, u0: float = 0.04, width: float = 80.0,
                v0: float = 0.002, rho_noise: float = 1e-5):
    """Doubly periodic double shear layer on x = i/nx, y = j/ny:
    u1 = u0 tanh(width (y - 1/4)) for y <= 1/2, u0 tanh(width (3/4 - y))
    otherwise; u2 = v0 sin(2 pi (x + 1/4)); rho = 1 + rho_noise * xi."""
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    X, Y = np.meshgrid(x, y)
    u = np.zeros((2, ny, nx))
    u[0] = np.where(Y <= 0.5, u0 * np.tanh(width * (Y - 0.25)), u0 * np.tanh(width * (0.75 - Y)))
    u[1] = v0 * np.sin(2.0 * math.pi * (X + 0.25))
    rho = 1.0 + rho_noise * noise(seed, 0, nx * ny).reshape(ny, nx)
    cfg = dict(Q=9, qe=QE_POLY, nx=nx, ny=ny, nu=nu, delta=delta, k=k,
               bc=(PERIODIC, PERIODIC, PERIODIC, PERIODIC))
    return cfg, rho, u


def _smooth(seed: int, comp: int, nx: int, ny: int, modes: int = 8) -> np.ndarray:
    """Sum of `modes` seeded plane waves on the unit torus, scaled to [-1, 1]."""
    r = noise(seed, 100 + comp, 4 * modes)
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    X, Y = np.meshgrid(x, y)
    s = np.zeros((ny, nx))
    for m in range(modes):
        kx = int(np.floor((r[4 * m] + 1.0) * 2.5))          # 0..4
        ky = int(np.floor((r[4 * m + 1] + 1.0) * 2.5)) - 2  # -2..2
        if kx == 0 and ky == 0:
            kx = 1
        a = 0.5 + 0.5 * abs(r[4 * m + 2])
        ph = math.pi * r[4 * m + 3]
        s += a * np.sin(2.0 * math.pi * (kx * X + ky * Y) + ph)
    s -= s.min()
    s /= max(s.max(), 1e-300)
    return 2.0 * s - 1.0


def iso_energy(u1: np.ndarray, u2: np.ndarray) -> np.ndarray:
    """Isothermal reference energy per mass used to place the synthetic
    moment field: -2/3 + (2/3) (sqrt(1 + 3 u1^2) + sqrt(1 + 3 u2^2))."""
    return -2.0 / 3.0 + (2.0 / 3.0) * (np.sqrt(1.0 + 3.0 * u1 ** 2) + np.sqrt(1.0 + 3.0 * u2 ** 2))


def moment_field(nx: int = 4096, ny: int = 2048, seed: int = 4, umax: float = 0.1,
                 energy_band: float = 0.05) -> np.ndarray:
    """Smooth synthetic moment field M[4][ny*nx] = (rho, rho u1, rho u2, 2E):
    rho in [0.5, 1.5], |u| <= umax, 2E/rho = iso(u) (1 + energy_band s)."""
    s0, s1, s2, s3 = (_smooth(seed, c, nx, ny) for c in range(4))
    rho = 1.0 + 0.5 * s0
    u1 = umax * s1 / math.sqrt(2.0)
    u2 = umax * s2 / math.sqrt(2.0)
    e = iso_energy(u1, u2) * (1.0 + energy_band * s3)
    M = np.stack([rho, rho * u1, rho * u2, rho * e]).reshape(4, -1)
    return np.ascontiguousarray(M)


def random_moments(n: int, seed: int, umax: float = 0.1, energy_band: float = 0.05) -> np.ndarray:
    """Unstructured moment samples with the same ranges as moment_field."""
    rho = 1.0 + 0.5 * noise(seed, 0, n)
    a = noise(seed, 1, n)
    b = noise(seed, 2, n)
    u1 = umax * a / math.sqrt(2.0)
    u2 = umax * b / math.sqrt(2.0)
    e = iso_energy(u1, u2) * (1.0 + energy_band * noise(seed, 3, n))
    return np.ascontiguousarray(np.stack([rho, rho * u1, rho * u2, rho * e]))


# named presets: the five configurations of the study and small parity cases
CONFIGS = {
    "shock_tube_800": lambda: shock_tube(),
    "shock_tube_801_paper": lambda: shock_tube(nx=801, split=400, inclusive=True, delta=1e-4),
    "cylinder_1200x400_re1000": lambda: cylinder(re=1000.0),
    "cylinder_1200x400_re5000": lambda: cylinder(re=5000.0),
    "cylinder_1200x400_re20000": lambda: cylinder(re=20000.0),
    "shear_8192x4096": lambda: shear_layer(),
    "cylinder_paper_600x500_re1000": lambda: cylinder_paper(1000.0)[:3],
    "cylinder_paper_600x500_re20000": lambda: cylinder_paper(20000.0)[:3],
    "cylinder_2400x800_re20000_fstarM": lambda: cylinder(nx=2400, ny=800, side=80, centre=(600, 400),
                                                         re=20000.0, k=256, qe=QE_ENTROPIC_M),
}


def mlp_norm(wide: bool = False):
    """Fixed input/output scalings of the warm-start network, sized for the
    moment distribution above (|u| <= 0.1, energy within 5% of isothermal),
    or with wide=True for |u| <= 0.3 and energy within 30%: features
    (u1, u2, 2E/rho, |u|^2) and targets (mu0 - ln rho, mu1, mu2, mu3) are
    mapped to O(1) by x = (value - shift) * scale."""
    if wide:
        return ([0.0, 0.0, 0.7, 0.03], [8.0, 8.0, 8.0, 50.0],
                [-0.87, 0.0, 0.0, -1.4], [5.0, 2.5, 2.5, 3.3])
    in_shift = [0.0, 0.0, 2.0 / 3.0, 0.005]
    in_scale = [20.0, 20.0, 20.0, 200.0]
    out_shift = [math.log(4.0 / 9.0), 0.0, 0.0, -math.log(4.0)]
    out_scale = [10.0, 5.0, 5.0, 10.0]
    return in_shift, in_scale, out_shift, out_scale
