"""Seeded synthetic workloads for the FFT BPM z-march.

Every workload is a symmetric-Bragg slab problem in the (x, z) plane of the
paper's Section 2.1: x transverse (the reciprocal vector h is along x), z the
marching axis, crystal occupying x_front <= x < x_front + thickness.

A workload holds
  * the plan parameters (Nx, dx, dz, Nz, chi0, chih, chihbar, theta_B, lambda,
    Nomega), the relative frequency offset delta_w of each slice, the slab;
  * E0_in[w, j]: the transmitted-beam envelope at z = 0, i.e. the incident
    field with the carrier exp(i h x / 2) removed (envelope definition,
    Eq. fov7), sampled at x_j = (j - Nx/2) dx;
  * u[n, j]: the displacement along h (metres) used by z-step n, or None.

The incident beam is the Gaussian of Section 3.1 (rocking-curve example) with
the source at its waist (z_x = 0, so the prefactor is 1).  A pulse is the
Gaussian of Eq. tdp transformed to frequency: one slice per frequency offset,
amplitude exp(-(omega_0 delta)^2 sigma_t^2 / 2) times a seeded random spectral
phase.  Displacements are the constant strain gradient of Section 3.2
(u = x^2 / (2R), i.e. B = 1/(2R)) and a Gaussian thermal bump standing in for
the finite-element field of Section 3.4, plus seeded white-noise strain.

Nothing here propagates a field: these are inputs only.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

C_LIGHT = 299792458.0

# Shared defaults: 1.24 Angstrom, 45 degree symmetric Bragg, synthetic
# susceptibilities (real parts of x-ray susceptibilities are negative; the
# small positive imaginary parts give absorption with exp(+i k z) propagation).
LAMBDA = 1.24e-10
THETA_B = math.pi / 4
CHI0 = complex(-1.5e-5, 1e-8)
CHIH = complex(3.8e-6, 0.9e-8)
DX = 0.5e-6
DZ = 0.5e-6
W0 = 50e-6
X0 = -100e-6


@dataclass
class Workload:
    name: str
    Nx: int
    dx: float
    dz: float
    Nz: int
    chi0: complex
    chih: complex
    chihbar: complex
    theta_B: float
    lam: float
    Nomega: int
    delta: np.ndarray                 # (Nomega,) relative frequency offsets
    E0_in: np.ndarray                 # (Nomega, Nx) complex128
    u: Optional[np.ndarray] = None    # (Nz, Nx) float64 or None
    x_front: float = 0.0
    thickness: float = math.inf
    meta: dict = field(default_factory=dict)

    @property
    def cell_updates(self) -> int:
        return self.Nx * self.Nz * self.Nomega

    def plan_args(self) -> dict:
        return dict(Nx=self.Nx, dx=self.dx, dz=self.dz, Nz=self.Nz,
                    chi0=self.chi0, chih=self.chih, chihbar=self.chihbar,
                    theta_B=self.theta_B, lam=self.lam, Nomega=self.Nomega)

    def subset(self, slices) -> "Workload":
        """Same problem restricted to the listed frequency slices."""
        idx = np.asarray(slices, dtype=np.int64)
        return Workload(self.name + f"[{len(idx)} slices]", self.Nx, self.dx,
                        self.dz, self.Nz, self.chi0, self.chih, self.chihbar,
                        self.theta_B, self.lam, len(idx), self.delta[idx].copy(),
                        self.E0_in[idx].copy(), self.u, self.x_front,
                        self.thickness, dict(self.meta))


def x_grid(Nx: int, dx: float) -> np.ndarray:
    """Sample positions x_j = (j - Nx/2) dx."""
    return (np.arange(Nx, dtype=np.float64) - Nx // 2) * dx


def darwin_relative_width(chih: complex, chihbar: complex, theta_B: float) -> float:
    """Full Darwin width of a symmetric Bragg reflection in relative photon
    energy, |sqrt(chih chihbar)| / sin^2(theta_B) (textbook dynamical theory)."""
    return abs(np.sqrt(complex(chih) * complex(chihbar))) / math.sin(theta_B) ** 2


def detuning_grid(Nomega: int, eps_D: float, span_widths: float = 10.0) -> np.ndarray:
    """Nomega cell-centred relative frequency offsets spanning
    +-span_widths/2 Darwin widths; a single slice sits at zero offset."""
    if Nomega == 1:
        return np.zeros(1)
    j = np.arange(Nomega, dtype=np.float64)
    return eps_D * (-span_widths / 2 + span_widths * (j + 0.5) / Nomega)


def incident_envelope(Nx, dx, lam, theta_B, delta, theta_i, amp,
                      x0=X0, w0=W0) -> np.ndarray:
    """Gaussian beam exp(-(x-x0)^2/W0^2) travelling at glancing angle theta_i,
    one row per frequency slice (wavenumber k0 (1 + delta_w)), with the
    carrier exp(i h x / 2), h = 2 k0 sin(theta_B), removed."""
    x = x_grid(Nx, dx)
    k0 = 2.0 * math.pi / lam
    h = 2.0 * k0 * math.sin(theta_B)
    g = np.exp(-((x - x0) / w0) ** 2)
    d = np.asarray(delta, dtype=np.float64)
    tilt = k0 * (1.0 + d) * math.sin(theta_i) - 0.5 * h
    amp = np.asarray(amp, dtype=np.complex128)
    return (amp[:, None] * g[None, :]) * np.exp(1j * (tilt[:, None] * x[None, :]))


def pulse_field(Nx, dx, N, dt, lam, theta_B, theta_i, sigma_t, x0=X0, w0=W0,
                t0=0.0) -> np.ndarray:
    """Incident pulse in the time domain, [N][Nx] on t_i = (i - N/2) dt:
    a Gaussian of rms duration sigma_t (Eq. tdp, read with the minus sign,
    normalised by 1/(sqrt(2 pi) sigma_t)) times the beam exp(-(x-x0)^2/W0^2),
    travelling at glancing angle theta_i, so that its front reaches x at
    t0 + (x - x0) sin(theta_i)/c, with the carrier exp(i h x/2),
    h = 2 k0 sin(theta_B), removed."""
    x = x_grid(Nx, dx)
    t = (np.arange(N) - N // 2) * float(dt)
    k0 = 2.0 * math.pi / lam
    h = 2.0 * k0 * math.sin(theta_B)
    tau = t[:, None] - t0 - (x[None, :] - x0) * math.sin(theta_i) / C_LIGHT
    g = np.exp(-0.5 * (tau / sigma_t) ** 2) / (math.sqrt(2.0 * math.pi) * sigma_t)
    beam = np.exp(-((x - x0) / w0) ** 2) * np.exp(1j * (k0 * math.sin(theta_i) - 0.5 * h) * x)
    return g * beam[None, :]


def pulse_amplitudes(delta, lam, sigma_t, rng, phase_amp=0.1) -> np.ndarray:
    """Spectral amplitudes of a Gaussian pulse of rms duration sigma_t with a
    seeded random spectral phase of amplitude phase_amp (radians)."""
    omega0 = 2.0 * math.pi * C_LIGHT / lam
    mag = np.exp(-0.5 * (omega0 * np.asarray(delta) * sigma_t) ** 2)
    ph = phase_amp * rng.uniform(-1.0, 1.0, size=len(delta))
    return mag * np.exp(1j * ph)


def bent_displacement(Nx, dx, Nz, R, x_front=0.0) -> np.ndarray:
    """Constant strain gradient u = (x - x_front)^2 / (2R), the same in every
    z row (Section 3.2 with B = 1/(2R))."""
    xs = x_grid(Nx, dx) - x_front
    row = xs * xs / (2.0 * R)
    return np.broadcast_to(row, (Nz, Nx)).copy()


def bump_factors(Nx, dx, Nz, dz, sigma, x_front=0.0):
    """Separable Gaussian bump exp(-(x^2 + (z - zc)^2)/(2 sigma^2)) with zc at
    mid-depth: returns (gz, gx); a bump of amplitude A is
    bump[n, j] = (A * gz[n]) * gx[j]."""
    xs = x_grid(Nx, dx) - x_front
    z = np.arange(Nz, dtype=np.float64) * dz
    zc = Nz * dz / 2.0
    gx = np.exp(-xs * xs / (2.0 * sigma * sigma))
    gz = np.exp(-(z - zc) ** 2 / (2.0 * sigma * sigma))
    return gz, gx


def _common(name, Nx, Nz, Nomega, delta, E0, u, **meta) -> Workload:
    return Workload(name, Nx, DX, DZ, Nz, CHI0, CHIH, CHIH, THETA_B, LAMBDA,
                    Nomega, np.asarray(delta, dtype=np.float64), E0, u,
                    0.0, math.inf, dict(meta))


def small(Nx=256, Nz=40, Nomega=3, seed=0, deformed=True, dx=DX, dz=DZ,
          x_front=0.0, thickness=math.inf, x0=None, w0=None) -> Workload:
    """Small seeded problem for parity tests: a pulse of Nomega slices on a
    bent crystal with a thermal bump and noise strain, sized so that the
    oracle runs in well under a second; the beam is centred on the crystal
    face unless x0 is given."""
    rng = np.random.default_rng(seed)
    eps = darwin_relative_width(CHIH, CHIH, THETA_B)
    delta = detuning_grid(Nomega, eps)
    amp = pulse_amplitudes(delta, LAMBDA, 10e-15, rng)
    L = Nx * dx
    xg = x_grid(Nx, dx)
    # default: the beam centred on the crystal face (clamped into the window),
    # so that the reflected field is a large part of the result after a few
    # tens of steps and each output field can be checked on its own
    x0 = min(max(x_front, xg[0]), xg[-1]) if x0 is None else x0
    w0 = 0.08 * L if w0 is None else w0
    E0 = incident_envelope(Nx, dx, LAMBDA, THETA_B, delta, THETA_B, amp, x0, w0)
    u = None
    if deformed:
        x_ref = min(max(x_front, xg[0]), xg[-1])   # bend measured from the slab face
        u = bent_displacement(Nx, dx, Nz, rng.uniform(1.0, 100.0), x_ref)
        amp = rng.uniform(0.2e-10, 1e-10)
        gz, gx = bump_factors(Nx, dx, Nz, dz, 0.2 * L, x_ref)
        u += (amp * gz)[:, None] * gx[None, :]
        strain = rng.normal(0.0, 1e-7, size=(Nz, Nx))
        cs = np.cumsum(strain, axis=1)
        j0 = int(np.searchsorted(xg, x_ref))
        u += dx * (cs - cs[:, min(j0, Nx - 1)][:, None])
    return Workload(f"small-{Nx}x{Nz}x{Nomega}-s{seed}", Nx, dx, dz, Nz, CHI0,
                    CHIH, CHIH, THETA_B, LAMBDA, Nomega, delta, E0, u,
                    x_front, thickness, {"seed": seed})


def c1_perfect_crystal() -> Workload:
    """Monochromatic perfect crystal, 1024 x 2000 steps, one slice, incidence
    at the refraction-shifted Darwin centre, no deformation."""
    Nx, Nz = 1024, 2000
    theta_i = THETA_B + 1.5e-5
    delta = np.zeros(1)
    E0 = incident_envelope(Nx, DX, LAMBDA, THETA_B, delta, theta_i, np.ones(1))
    return _common("perfect-crystal-1024x2000x1", Nx, Nz, 1, delta, E0, None,
                   theta_i=theta_i)


def c2_bent_crystal(seed: int = 2) -> Workload:
    """Bent crystal (R = 10 m), 2048 x 4000 steps, 256 slices of a 10 fs pulse
    spanning +-5 Darwin widths with a random spectral phase of 0.1 rad."""
    Nx, Nz, Nw = 2048, 4000, 256
    rng = np.random.default_rng(seed)
    eps = darwin_relative_width(CHIH, CHIH, THETA_B)
    delta = detuning_grid(Nw, eps)
    amp = pulse_amplitudes(delta, LAMBDA, 10e-15, rng)
    E0 = incident_envelope(Nx, DX, LAMBDA, THETA_B, delta, THETA_B, amp)
    u = bent_displacement(Nx, DX, Nz, 10.0)
    return _common("bent-crystal-2048x4000x256", Nx, Nz, Nw, delta, E0, u,
                   R=10.0, sigma_t=10e-15, seed=seed)


def c3_thermal_bump(seed: int = 3, Nomega: int = 1024) -> Workload:
    """Thermal bump (1e-10 m, sigma 100 um) plus white-noise strain of rms
    1e-7, 4096 x 8192 steps, 1024 pulse slices."""
    Nx, Nz = 4096, 8192
    rng = np.random.default_rng(seed)
    eps = darwin_relative_width(CHIH, CHIH, THETA_B)
    delta = detuning_grid(Nomega, eps)
    amp = pulse_amplitudes(delta, LAMBDA, 10e-15, rng)
    E0 = incident_envelope(Nx, DX, LAMBDA, THETA_B, delta, THETA_B, amp)
    gz, gx = bump_factors(Nx, DX, Nz, DZ, 100e-6)
    u = (1e-10 * gz)[:, None] * gx[None, :]
    strain = rng.normal(0.0, 1e-7, size=(Nz, Nx))
    cs = np.cumsum(strain, axis=1)
    j0 = Nx // 2
    u += DX * (cs - cs[:, j0][:, None])
    return _common("thermal-bump-4096x8192x1024", Nx, Nz, Nomega, delta, E0, u,
                   sigma_t=10e-15, seed=seed)


C4_NX = (256, 512, 1024, 2048, 4096)
C4_NOMEGA = (1, 16, 64, 256)


def c4_problem_specs(n: int = 512, seed: int = 4) -> list:
    """Sizes and parameters of the uneven batch: Nx in {256..4096}, Nz uniform
    in [500, 8000], Nomega in {1, 16, 64, 256}, bend radius R in [1, 100] m,
    bump amplitude in [0, 1e-10] m; one sub-seed per problem."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n):
        specs.append(dict(
            index=i,
            Nx=int(rng.choice(C4_NX)),
            Nz=int(rng.integers(500, 8001)),
            Nomega=int(rng.choice(C4_NOMEGA)),
            R=float(rng.uniform(1.0, 100.0)),
            bump=float(rng.uniform(0.0, 1e-10)),
            seed=int(rng.integers(0, 2**31 - 1)),
        ))
    return specs


def c4_problem(spec: dict, with_u: bool = True) -> Workload:
    """Materialise one batch problem: pulse as in the bent-crystal workload,
    u = x^2/(2R) + separable Gaussian bump (sigma 100 um).  The displacement
    is also returned in separable form in meta['u_factors'] = (row, gz, gx,
    amp) with u[n, j] = row[j] + (amp * gz[n]) * gx[j]."""
    Nx, Nz, Nw = spec["Nx"], spec["Nz"], spec["Nomega"]
    rng = np.random.default_rng(spec["seed"])
    eps = darwin_relative_width(CHIH, CHIH, THETA_B)
    delta = detuning_grid(Nw, eps)
    amp = pulse_amplitudes(delta, LAMBDA, 10e-15, rng)
    E0 = incident_envelope(Nx, DX, LAMBDA, THETA_B, delta, THETA_B, amp)
    xs = x_grid(Nx, DX)
    row = xs * xs / (2.0 * spec["R"])
    gz, gx = bump_factors(Nx, DX, Nz, DZ, 100e-6)
    u = None
    if with_u:
        u = row[None, :] + (spec["bump"] * gz)[:, None] * gx[None, :]
    meta = {k: v for k, v in spec.items() if k not in ("Nx", "Nz", "Nomega")}
    w = _common(f"batch-{spec['index']}-{Nx}x{Nz}x{Nw}", Nx, Nz, Nw, delta, E0,
                u, **meta)
    w.meta["u_factors"] = (row, gz, gx, spec["bump"])
    return w


def c5_request_trace(rate: float = 200.0, duration: float = 60.0, seed: int = 5):
    """Poisson arrival trace: list of (arrival_time_s, spec, precision) with
    sizes drawn as in the uneven batch and precision 'fp64' or 'fp32' with
    probability 1/2 each."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    i = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        spec = dict(
            index=i,
            Nx=int(rng.choice(C4_NX)),
            Nz=int(rng.integers(500, 8001)),
            Nomega=int(rng.choice(C4_NOMEGA)),
            R=float(rng.uniform(1.0, 100.0)),
            bump=float(rng.uniform(0.0, 1e-10)),
            seed=int(rng.integers(0, 2**31 - 1)),
        )
        prec = "fp64" if rng.uniform() < 0.5 else "fp32"
        out.append((t, spec, prec))
        i += 1
    return out


@dataclass
class Workload3D:
    """A problem on a 3D grid: rows y_i = (i - Ny/2) dy, columns
    x_j = (j - Nx/2) dx; E0_in (Nomega, Ny, Nx), u (Nz, Ny, Nx) or None."""
    name: str
    Nx: int
    Ny: int
    dx: float
    dy: float
    dz: float
    Nz: int
    chi0: complex
    chih: complex
    chihbar: complex
    theta_B: float
    lam: float
    Nomega: int
    delta: np.ndarray
    E0_in: np.ndarray
    u: Optional[np.ndarray] = None
    x_front: float = 0.0
    thickness: float = math.inf
    meta: dict = field(default_factory=dict)

    @property
    def cell_updates(self) -> int:
        return self.Nx * self.Ny * self.Nz * self.Nomega

    def subset(self, slices) -> "Workload3D":
        idx = np.asarray(slices, dtype=np.int64)
        return Workload3D(self.name + f"[{len(idx)} slices]", self.Nx, self.Ny, self.dx,
                          self.dy, self.dz, self.Nz, self.chi0, self.chih, self.chihbar,
                          self.theta_B, self.lam, len(idx), self.delta[idx].copy(),
                          self.E0_in[idx].copy(), self.u, self.x_front, self.thickness,
                          dict(self.meta))


def beam_3d(Nx, Ny, dx, dy, lam, theta_B, delta, theta_i, amp, x0, y0, w0x, w0y):
    """The Gaussian beam exp(-(x-x0)^2/w0x^2 - (y-y0)^2/w0y^2) at glancing
    angle theta_i in the (x, z) plane, carrier exp(i h x / 2) removed, one
    (Ny, Nx) plane per slice."""
    rows = incident_envelope(Nx, dx, lam, theta_B, delta, theta_i, amp, x0, w0x)
    y = x_grid(Ny, dy)
    gy = np.exp(-((y - y0) / w0y) ** 2)
    return rows[:, None, :] * gy[None, :, None]


def small3d(Nx=60, Ny=6, Nz=20, Nomega=2, seed=0, deformed=True, dx=DX, dy=None,
            dz=DZ, x_front=0.0, thickness=math.inf) -> Workload3D:
    """Small seeded 3D problem for parity tests: a pulse of Nomega slices, a
    beam centred on the crystal face in x and on the window in y, a bent
    crystal with a bump that varies along y and seeded noise strain."""
    rng = np.random.default_rng(seed)
    dy = 4 * dx if dy is None else dy
    eps = darwin_relative_width(CHIH, CHIH, THETA_B)
    delta = detuning_grid(Nomega, eps)
    amp = pulse_amplitudes(delta, LAMBDA, 10e-15, rng)
    Lx, Ly = Nx * dx, Ny * dy
    xg = x_grid(Nx, dx)
    x0 = min(max(x_front, xg[0]), xg[-1])
    E0 = beam_3d(Nx, Ny, dx, dy, LAMBDA, THETA_B, delta, THETA_B, amp, x0, 0.0,
                 0.08 * Lx + 2 * dx, 0.3 * Ly + dy)
    u = None
    if deformed:
        y = x_grid(Ny, dy)
        R = rng.uniform(1.0, 100.0)
        row = (xg - x0) ** 2 / (2.0 * R)
        z = np.arange(Nz) * dz
        bump = rng.uniform(0.2e-10, 1e-10) * np.exp(
            -((xg[None, None, :] - x0) ** 2 + y[None, :, None] ** 2
              + (z[:, None, None] - Nz * dz / 2) ** 2) / (2 * (0.2 * max(Lx, Ly)) ** 2))
        strain = rng.normal(0.0, 1e-7, size=(Nz, Ny, Nx))
        u = row[None, None, :] + bump + dx * np.cumsum(strain, axis=2)
    return Workload3D(f"small3d-{Nx}x{Ny}x{Nz}x{Nomega}-s{seed}", Nx, Ny, dx, dy, dz, Nz,
                      CHI0, CHIH, CHIH, THETA_B, LAMBDA, Nomega, delta, E0, u,
                      x_front, thickness, {"seed": seed})


def heat_bump_3d(Nomega: int = 16, seed: int = 6, Nz: int = 1842) -> Workload3D:
    """The grid of the paper's finite-element example (Section 3.4): 22 rows
    along y by 4267 samples along x, 1842 steps; dx = dz = 0.5 um, dy = 5 um.
    A pulse of Nomega slices over +-5 Darwin widths, a 30 um rms beam centred
    on the crystal face, and a Gaussian thermal bump (1e-10 m, sigma 100 um
    in x and z, 30 um in y) plus seeded noise strain standing in for the
    finite-element displacement."""
    Nx, Ny, dy = 4267, 22, 5e-6
    rng = np.random.default_rng(seed)
    eps = darwin_relative_width(CHIH, CHIH, THETA_B)
    delta = detuning_grid(Nomega, eps)
    amp = pulse_amplitudes(delta, LAMBDA, 10e-15, rng)
    w0 = 30e-6 * math.sqrt(2.0)                 # 30 um rms intensity width
    E0 = beam_3d(Nx, Ny, DX, dy, LAMBDA, THETA_B, delta, THETA_B, amp, 0.0, 0.0,
                 w0, w0)
    xg, y = x_grid(Nx, DX), x_grid(Ny, dy)
    z = np.arange(Nz) * DZ
    gz = np.exp(-(z - Nz * DZ / 2) ** 2 / (2 * (100e-6) ** 2))
    gxy = np.exp(-xg[None, :] ** 2 / (2 * (100e-6) ** 2)) * np.exp(-y[:, None] ** 2 / (2 * (30e-6) ** 2))
    u = (1e-10 * gz)[:, None, None] * gxy[None, :, :]
    strain = rng.normal(0.0, 1e-7, size=(Nz, Ny, Nx))
    cs = np.cumsum(strain, axis=2)
    u += DX * (cs - cs[:, :, Nx // 2][:, :, None])
    return Workload3D(f"heat-bump-3d-{Nx}x{Ny}x{Nz}x{Nomega}", Nx, Ny, DX, dy, DZ, Nz,
                      CHI0, CHIH, CHIH, THETA_B, LAMBDA, Nomega, delta, E0, u,
                      0.0, math.inf, {"seed": seed, "sigma_t": 10e-15})


def by_name(name: str) -> Workload:
    table = {
        "perfect-crystal-1024x2000x1": c1_perfect_crystal,
        "bent-crystal-2048x4000x256": c2_bent_crystal,
        "thermal-bump-4096x8192x1024": c3_thermal_bump,
    }
    return table[name]()
