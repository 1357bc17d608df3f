"""Seeded synthetic workloads: problem parameters and input arrays.

This module holds only problem descriptions and random input generation.  It
contains none of the method's arithmetic, so both the GPU library's tests and
the CPU oracle can consume the same arrays.

The paper's examples (Sec. 4) use geometries that exist only in its figures,
so these generators stand in for them with the paper's parameter ranges:

* density: N(0,1) noise on the design grid, separable periodic Gaussian blur
  (sigma = 3 cells, truncated at 4 sigma), standardised, then
  gamma = sigmoid(3 z); the margin is fluid (gamma = 0) by construction;
* motion: chi_a(t) = 0.5 + (amp * sin(2 pi t / nt + phase_a) + sigma_n * eps) / span,
  clipped to [0, 1]; psi likewise with a rotation amplitude, or a ramp of one
  full revolution for the rotating 3D case.

All arrays are float64 numpy arrays in the layouts documented by the C headers:
gamma [mz][my][mx] (inner design points only), chi [nt][3], psi [nt].
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np


@dataclasses.dataclass
class Problem:
    """Parameters of one LKS + Brinkman run (lattice units, dx = dt = 1)."""

    d: int = 2                                # 2 -> D2Q9, 3 -> D3Q15
    n: Tuple[int, int, int] = (64, 64, 1)     # analysis nodes per axis
    bc: Tuple[int, int, int] = (0, 1, 0)      # 0 periodic, 1 walls
    u_wall: Tuple = ((( 0.0,) * 3,) * 2,) * 3  # [axis][lo/hi][comp]
    dp_seam: Tuple[float, float, float] = (0.0, 0.0, 0.0)  # oracle test mode only
    nu: float = 0.1
    kappa_max: float = 300.0
    q: float = 0.1
    m: Tuple[int, int, int] = (32, 32, 1)     # inner design points
    margin: int = 4
    xg_min: Tuple[float, float, float] = (24.0, 24.0, 0.0)
    xg_max: Tuple[float, float, float] = (40.0, 40.0, 0.0)
    th_min: float = -0.4
    th_max: float = 0.4
    nt: int = 200
    r_t: int = 20
    r_w: int = 20
    tgt_lo: Tuple[int, int, int] = (0, 1, 0)
    tgt_hi: Tuple[int, int, int] = (1, 63, 1)
    ndir: Tuple[float, float, float] = (1.0, 0.0, 0.0)
    phi: float = 0.0
    precision: int = 1                        # GPU state: 0 = FP32, 1 = FP64
    ckpt_k: int = 0                           # checkpoint interval (0 = nt)
    body_tape: int = 0                        # body fields kept: 1 all steps, -1 a segment, 0 auto
    scheme: int = 0                           # reverse sweep: 0 exact adjoint, 1 the paper's ALKS
    objective: int = 0                        # 0: J1 (flow rate), 1: J2 (oar force, 2D)
    w_d: float = 0.0                          # J2 weight of the drag work F_D
    w_t: float = 0.0                          # J2 weight of the torque work T
    l_m: float = 1.0                          # J2 moment arm
    rot: int = 0                              # 0: one angle about z; 1: three angles (3D)
    tilt_min: Tuple[float, float] = (0.0, 0.0)  # rot = 1: ranges of the angles about x, y
    tilt_max: Tuple[float, float] = (0.0, 0.0)

    @property
    def N(self) -> int:
        return int(np.prod(self.n[: self.d]))

    @property
    def design_shape(self) -> Tuple[int, int, int]:
        """Design grid incl. margin as (Dz, Dy, Dx)."""
        D = [self.m[a] + 2 * self.margin if a < self.d else 1 for a in range(3)]
        return (D[2], D[1], D[0])

    @property
    def M(self) -> int:
        return int(np.prod(self.m[: self.d]))

    @property
    def Mtot(self) -> int:
        return int(np.prod(self.design_shape))

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def _blur_periodic(a: np.ndarray, sigma: float) -> np.ndarray:
    r = int(math.ceil(4 * sigma))
    k = np.exp(-0.5 * (np.arange(-r, r + 1) / sigma) ** 2)
    k /= k.sum()
    out = a
    for ax in range(a.ndim):
        if a.shape[ax] == 1:
            continue
        acc = np.zeros_like(out)
        for j, kv in zip(range(-r, r + 1), k):
            acc += kv * np.roll(out, j, axis=ax)
        out = acc
    return out


def density(p: Problem, seed: int, sigma: float = 3.0) -> np.ndarray:
    """Smooth random pseudo-density in (0, 1) on the inner design grid."""
    rng = np.random.default_rng(seed)
    shape = (p.m[2] if p.d == 3 else 1, p.m[1], p.m[0])
    z = _blur_periodic(rng.standard_normal(shape), sigma)
    z = (z - z.mean()) / max(z.std(), 1e-300)
    return (1.0 / (1.0 + np.exp(-3.0 * z))).astype(np.float64)


def motion(p: Problem, seed: int, amp: float = 4.0, sigma_n: float = 0.25,
           th_amp: float = 0.1, th_sigma: float = 0.01, th_ramp: bool = False,
           cycles: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """Seeded sinusoidal translation and rotation design variables."""
    rng = np.random.default_rng(seed + 7919)
    t = np.arange(1, p.nt + 1, dtype=np.float64)
    chi = np.full((p.nt, 3), 0.5)
    phases = rng.uniform(0, 2 * math.pi, size=3)
    for a in range(p.d):
        span = p.xg_max[a] - p.xg_min[a]
        if span <= 0:
            continue
        x = amp * np.sin(2 * math.pi * cycles * t / p.nt + phases[a]) \
            + sigma_n * rng.standard_normal(p.nt)
        chi[:, a] = np.clip(0.5 + x / span, 0.0, 1.0)
    tspan = p.th_max - p.th_min
    if th_ramp:
        th = tspan * t / p.nt + th_sigma * rng.standard_normal(p.nt)
        psi = np.clip(th / tspan, 0.0, 1.0)
    elif tspan > 0:
        th = th_amp * np.sin(2 * math.pi * cycles * t / p.nt + rng.uniform(0, 2 * math.pi)) \
            + th_sigma * rng.standard_normal(p.nt)
        psi = np.clip((th - p.th_min) / tspan, 0.0, 1.0)
    else:
        psi = np.full(p.nt, 0.5)
    return chi, psi


def _centred(n: int, half: float) -> Tuple[float, float]:
    c = 0.5 * (n - 1)
    return (c - half, c + half)


def make_2d(nside: int, mside: int, nt: int, r_t: int, nu: float, seed: int,
            kappa_max: float = 300.0, phi: float = 0.0, amp: float = 4.0,
            sigma_n: float = 0.25, th_amp: float = 0.1, precision: int = 1,
            ckpt_k: int = 0, ny: Optional[int] = None, th_sigma: float = 0.01):
    """D2Q9 channel: periodic x, walls in y, target = column x = 0."""
    ny = nside if ny is None else ny
    lo0, hi0 = _centred(nside, 8.0)
    lo1, hi1 = _centred(ny, 8.0)
    p = Problem(d=2, n=(nside, ny, 1), bc=(0, 1, 0), nu=nu, kappa_max=kappa_max,
                m=(mside, mside, 1), margin=4, xg_min=(lo0, lo1, 0.0),
                xg_max=(hi0, hi1, 0.0), th_min=-0.4, th_max=0.4, nt=nt, r_t=r_t, r_w=r_t,
                tgt_lo=(0, 1, 0), tgt_hi=(1, ny - 1, 1), ndir=(1.0, 0.0, 0.0), phi=phi,
                precision=precision, ckpt_k=ckpt_k)
    gamma = density(p, seed)
    chi, psi = motion(p, seed, amp=amp, sigma_n=sigma_n, th_amp=th_amp, th_sigma=th_sigma)
    return p, gamma, chi, psi


def make_3d(nside: int, mside: int, nt: int, r_t: int, nu: float, seed: int,
            kappa_max: float = 100.0, phi: float = 0.1, amp: float = 2.0,
            precision: int = 0, ckpt_k: int = 100, th_ramp: bool = True):
    """D3Q15 box: walls in x and y, periodic z; body rotates about z.

    Target box and flow direction follow the 3D pump layout: a box below
    the top of the domain with n = (0, 0, 1)."""
    lo0, hi0 = _centred(nside, 4.0)
    s = nside / 128.0
    tz0, tz1 = int(round(102 * s)), int(round(115 * s))
    tx0, tx1 = int(round(32 * s)), int(round(96 * s))
    p = Problem(d=3, n=(nside, nside, nside), bc=(1, 1, 0), nu=nu, kappa_max=kappa_max,
                m=(mside, mside, mside), margin=4, xg_min=(lo0, lo0, lo0),
                xg_max=(hi0, hi0, hi0),
                th_min=0.0 if th_ramp else -0.4,
                th_max=2 * math.pi if th_ramp else 0.4, nt=nt, r_t=r_t, r_w=r_t,
                tgt_lo=(tx0, tx0, tz0), tgt_hi=(tx1, tx1, max(tz1, tz0 + 1)),
                ndir=(0.0, 0.0, 1.0), phi=phi, precision=precision, ckpt_k=ckpt_k)
    gamma = density(p, seed)
    chi, psi = motion(p, seed, amp=amp, sigma_n=0.05, th_sigma=0.01, th_ramp=th_ramp)
    return p, gamma, chi, psi


def reynolds_nu(u_ref: float, length: float, re: float) -> float:
    """Viscosity giving Reynolds number re for speed u_ref and length."""
    return u_ref * length / re


# Named workloads (lattice, grid, design grid, steps).  Viscosities follow the
# Re ~ 100 target with U_ref = max |u^G| + max |omega| * r_max and L = design side.
def c1(seed: int = 0, precision: int = 1):
    """D2Q9 64x64, 32x32 design, 200 steps (small parity case)."""
    return make_2d(64, 32, 200, 20, nu=0.064, seed=seed, precision=precision)


def c2(seed: int = 1, precision: int = 0, nt: int = 20000):
    """D2Q9 512x512, 256x256 design, 20000 steps."""
    return make_2d(512, 256, nt, 2000, nu=0.018, seed=seed, precision=precision, ckpt_k=200)


def oar(nside: int = 512, mside: int = 256, nt: int = 4000, seed: int = 4, precision: int = 0,
        ckpt_k: int = 100):
    """The 2D oar setting of Sec. 4.2 on a D2Q9 channel (periodic x, walls
    in y): objective J2 with w_D = 0.01, w_T = 0.15 and l_m half the design
    grid's diagonal; the design grid translates vertically only and rotates;
    nu = 0.1, kappa_max = 300, q = 0.1, R_t = 1000 and R_w = 2000 steps
    (capped at nt).  The domain size is not given in the text: a square
    channel of side nside with an mside^2 design grid stands in for it."""
    p, gamma, chi, psi = make_2d(nside, mside, nt, min(1000, nt), nu=0.1, seed=seed,
                                 precision=precision, ckpt_k=min(ckpt_k, nt))
    x0 = p.xg_min[0] + 0.5 * (p.xg_max[0] - p.xg_min[0])
    p = p.replace(xg_min=(x0, p.xg_min[1], 0.0), xg_max=(x0, p.xg_max[1], 0.0),
                  r_w=min(2000, nt), objective=1, w_d=0.01, w_t=0.15,
                  l_m=0.5 * math.sqrt(2.0) * mside)
    return p, gamma, chi, psi


def c3(seed: int = 2, precision: int = 0, nt: int = 10000, ckpt_k: int = 100):
    """D2Q9 1024x1024, 512x512 design, 10000 steps."""
    return make_2d(1024, 512, nt, 1000, nu=0.02, seed=seed, precision=precision,
                   ckpt_k=ckpt_k)


def c4(seed: int = 3, precision: int = 0, nt: int = 5000, ckpt_k: int = 100):
    """D3Q15 128^3, 64^3 design, 5000 steps, rotation about z."""
    return make_3d(128, 64, nt, 500, nu=0.04, seed=seed, precision=precision, ckpt_k=ckpt_k)


def c5_instances(seed: int = 4, nt: int = 4000, precision: int = 0):
    """16 uneven D2Q9 instances (sides in 128..384), Re and filter radius round-robin."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(128, 385, size=16)
    res = [50, 100, 200, 400]
    radii = [1, 3, 5, 9]
    out = []
    for k, s in enumerate(sides):
        s = int(s)
        ms = s // 2
        u_ref = 2 * math.pi * 4.0 / nt + 2 * math.pi * 0.1 / nt * ms * 0.7071
        nu = max(reynolds_nu(u_ref, ms, res[k % 4]), 0.005)
        rt = radii[k % 4]
        sig = 0.01 if rt < 5 else 0.25
        # rotation noise sized so the body's rim moves by about sigma_n cells:
        # with little temporal filtering a 0.01 rad per-step jitter would move
        # the rim of a large body faster than the lattice allows
        out.append(make_2d(s, ms, nt, rt, nu=nu, seed=seed * 100 + k, precision=precision,
                           sigma_n=sig, th_sigma=sig / (0.7071 * ms), ckpt_k=200))
    return out
