"""Seeded synthetic problem instances for the phonon BTE time step.

This module only *generates inputs*: the Cartesian mesh and its walls, the
initial temperature field, the discrete direction set (unit vectors and
solid-angle weights) and the per-band material tables (frequency, band width,
group velocity, relaxation time, density of states, polarisation degeneracy).
It holds none of the solver's arithmetic: no equilibrium intensity, no flux,
no temperature inversion.  Both the HIP library and the CPU oracle consume the
arrays produced here, and nothing else is shared between them.

Paper context (Sec. 3.1 "Model"): the intensity I(x, t, s, omega) is
discretised into directions d and frequency bands b; 40 frequency bands give
55 band entries once the 15 bands that also carry the transverse branch are
counted, and 3D problems use 20 x 20 = 400 directions.  The paper takes its
silicon dispersion and relaxation data from outside references that are not
reproduced here, so the tables below are synthetic, Si-like stand-ins.

Layout conventions (shared with ``include/bte.h``):
  * cell index  P = x + nx * (y + ny * z)      (x fastest)
  * wall order  -x, +x, -y, +y, -z, +z
  * wall-face arrays run over the two other axes, lower axis fastest:
    +-x walls: y + ny*z;  +-y walls: x + nx*z;  +-z walls: x + nx*y
  * in 2D, nz = 1, hz = 1 (quantities per unit depth) and s_z is ignored.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

WALL_ISOTHERMAL = 0
WALL_SPECULAR = 1
WALL_SYMMETRY = 2
WALL_DIFFUSE = 3

SCHEME_IMPLICIT_JACOBI = 0
SCHEME_EXPLICIT_EULER = 1

PRECISION_FP64 = 0
PRECISION_FP32_MIXED = 1

TDEF_TAU_WEIGHTED = 0
TDEF_ENERGY = 1


@dataclasses.dataclass
class Instance:
    """One synthetic BTE problem: mesh, walls, directions, bands, run settings."""

    name: str
    dim: int
    n: List[int]                       # cells per axis (nz = 1 in 2D)
    h: List[float]                     # cell size per axis [m] (hz = 1 in 2D)
    wall: List[int]                    # 6 wall kinds, order -x,+x,-y,+y,-z,+z
    wall_T: List[Optional[np.ndarray]]  # per-face temperature [K] or None
    T_init: np.ndarray                 # [N_c] initial temperature [K]
    s: np.ndarray                      # [N_d, 3] unit direction vectors
    w: np.ndarray                      # [N_d] solid-angle weights [sr]
    omega: np.ndarray                  # [N_b] band angular frequency [rad/s]
    domega: np.ndarray                 # [N_b] band width [rad/s]
    pol: np.ndarray                    # [N_b] 0 = longitudinal, 1 = transverse
    vg: np.ndarray                     # [N_b] group speed [m/s]
    tau: np.ndarray                    # [N_b] relaxation time [s]
    dos: np.ndarray                    # [N_b] density of states per polarisation [s/m^3]
    deg: np.ndarray                    # [N_b] polarisation degeneracy
    dt: float = 1e-12
    tol: float = 1e-4
    max_inner: int = 200
    nsteps: int = 1
    scheme: int = SCHEME_IMPLICIT_JACOBI
    precision: int = PRECISION_FP64
    t_definition: int = TDEF_TAU_WEIGHTED
    seed: int = 0
    # temperature-dependent relaxation: tau_b(T) = tau_b (tau_T0 / T)^tau_exp_b
    # (None: constant tau)
    tau_exp: Optional[np.ndarray] = None
    tau_T0: float = 300.0

    @property
    def n_cells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def n_dirs(self) -> int:
        return int(self.s.shape[0])

    @property
    def n_bands(self) -> int:
        return int(self.omega.shape[0])

    @property
    def n_dof(self) -> int:
        return self.n_cells * self.n_dirs * self.n_bands

    def wall_face_count(self, side: int) -> int:
        nx, ny, nz = self.n
        axis = side // 2
        return (ny * nz, nx * nz, nx * ny)[axis]

    def copy(self, **changes) -> "Instance":
        inst = dataclasses.replace(self)
        inst.n = list(self.n)
        inst.h = list(self.h)
        inst.wall = list(self.wall)
        inst.wall_T = [None if a is None else a.copy() for a in self.wall_T]
        for k in ("T_init", "s", "w", "omega", "domega", "pol", "vg", "tau", "dos", "deg"):
            setattr(inst, k, getattr(self, k).copy())
        if self.tau_exp is not None:
            inst.tau_exp = self.tau_exp.copy()
        for k, v in changes.items():
            setattr(inst, k, v)
        return inst


# --------------------------------------------------------------------------
# Direction sets
# --------------------------------------------------------------------------
def product_quadrature(n_polar: int, n_azimuthal: int):
    """Polar x azimuthal product set (Sec. 3.1: 20 x 20 = 400 directions in 3D).

    theta_i = (i + 1/2) pi / n_polar, phi_j = (j + 1/2) 2 pi / n_azimuthal, so no
    direction is parallel to a mesh axis.  The weight of (i, j) is the exact
    solid angle of its cell on the unit sphere, dphi * (cos theta_i^- - cos
    theta_i^+), so the weights sum to 4 pi.  Ordering: d = i * n_azimuthal + j.
    With n_polar = 1 every direction lies in the xy-plane.
    """
    if n_polar < 1 or n_azimuthal < 1:
        raise ValueError("quadrature needs at least one polar and one azimuthal level")
    dphi = 2.0 * math.pi / n_azimuthal
    s = np.empty((n_polar * n_azimuthal, 3))
    w = np.empty(n_polar * n_azimuthal)
    for i in range(n_polar):
        th = (i + 0.5) * math.pi / n_polar
        th_lo = i * math.pi / n_polar
        th_hi = (i + 1) * math.pi / n_polar
        wi = dphi * (math.cos(th_lo) - math.cos(th_hi))
        for j in range(n_azimuthal):
            ph = (j + 0.5) * dphi
            d = i * n_azimuthal + j
            s[d] = (math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th))
            w[d] = wi
    if n_polar == 1:
        s[:, 2] = 0.0  # exactly in-plane
    return s, w


# --------------------------------------------------------------------------
# Band tables
# --------------------------------------------------------------------------
def linear_bands(n_bands: int, omega_max: float, rng: np.random.Generator,
                 v_range=(1e3, 9e3), tau_range=(1e-12, 1e-9)):
    """Linear (Debye-like) bands: omega_b = (b+1) omega_max / N_b, width omega_max / N_b.

    One polarisation per entry; density of states of a linear branch,
    D = omega^2 / (2 pi^2 v^3); group speed uniform in v_range and relaxation time
    log-uniform in tau_range, drawn from ``rng``.
    """
    b = np.arange(n_bands)
    omega = (b + 1) * omega_max / n_bands
    domega = np.full(n_bands, omega_max / n_bands)
    vg = rng.uniform(v_range[0], v_range[1], n_bands)
    tau = np.exp(rng.uniform(math.log(tau_range[0]), math.log(tau_range[1]), n_bands))
    dos = omega ** 2 / (2.0 * math.pi ** 2 * vg ** 3)
    deg = np.ones(n_bands)
    pol = np.zeros(n_bands, dtype=np.int32)
    return dict(omega=omega, domega=domega, vg=vg, tau=tau, dos=dos, deg=deg, pol=pol)


# Synthetic Si-like quadratic branches omega(k) = v k + c k^2 on k in [0, k_max].
# The constants are chosen so that the transverse branch tops out at 3/8 of the
# longitudinal maximum: with 40 equal frequency bands exactly 15 band centres lie
# under the transverse maximum, giving 40 + 15 = 55 band entries (Sec. 3.1).
K_MAX = 1.2e10
LA_V, LA_C = 9.0e3, -2.0e-7
TA_V, TA_C = 4.5375e3, -1.719e-7


def _branch_omega_max(v, c):
    return v * K_MAX + c * K_MAX ** 2


def quadratic_bands(n_freq: int, rng: np.random.Generator, tau_range=(1e-12, 1e-9)):
    """n_freq equal frequency bands over the longitudinal branch, plus a
    transverse entry for every band whose centre lies under the transverse maximum.

    Entries are ordered all longitudinal bands first, then the transverse ones.
    For each entry the wavevector k solves v k + c k^2 = omega_b (smaller root);
    group speed v_g = v + 2 c k; density of states per polarisation
    D = k^2 / (2 pi^2 v_g); degeneracy 1 (LA) or 2 (two TA branches).
    Relaxation times are log-uniform per entry, drawn from ``rng``.
    """
    wmax = _branch_omega_max(LA_V, LA_C)
    wmax_ta = _branch_omega_max(TA_V, TA_C)
    dw = wmax / n_freq
    centres = (np.arange(n_freq) + 0.5) * dw
    rows = []
    for wc in centres:
        rows.append((wc, 0))
    for wc in centres:
        if wc < wmax_ta:
            rows.append((wc, 1))
    omega = np.array([r[0] for r in rows])
    pol = np.array([r[1] for r in rows], dtype=np.int32)
    v = np.where(pol == 0, LA_V, TA_V)
    c = np.where(pol == 0, LA_C, TA_C)
    k = (-v + np.sqrt(v * v + 4.0 * c * omega)) / (2.0 * c)
    vg = v + 2.0 * c * k
    dos = k * k / (2.0 * math.pi ** 2 * vg)
    deg = np.where(pol == 0, 1.0, 2.0)
    domega = np.full(omega.shape, dw)
    tau = np.exp(rng.uniform(math.log(tau_range[0]), math.log(tau_range[1]), omega.shape[0]))
    return dict(omega=omega, domega=domega, vg=vg, tau=tau, dos=dos, deg=deg, pol=pol)


# --------------------------------------------------------------------------
# Generic builder
# --------------------------------------------------------------------------
def make_instance(name, dim, n, h, wall, wall_T, T_init, s, w, bands, **run):
    n = [int(v) for v in n] + [1] * (3 - len(n))
    h = [float(v) for v in h] + [1.0] * (3 - len(h))
    if dim == 2:
        n[2] = 1
        h[2] = 1.0
    inst = Instance(name=name, dim=dim, n=n, h=h, wall=list(wall),
                    wall_T=[None if a is None else np.ascontiguousarray(a, dtype=np.float64)
                            for a in wall_T],
                    T_init=np.ascontiguousarray(T_init, dtype=np.float64).reshape(-1),
                    s=np.ascontiguousarray(s, dtype=np.float64),
                    w=np.ascontiguousarray(w, dtype=np.float64),
                    omega=np.ascontiguousarray(bands["omega"], dtype=np.float64),
                    domega=np.ascontiguousarray(bands["domega"], dtype=np.float64),
                    pol=np.ascontiguousarray(bands["pol"], dtype=np.int32),
                    vg=np.ascontiguousarray(bands["vg"], dtype=np.float64),
                    tau=np.ascontiguousarray(bands["tau"], dtype=np.float64),
                    dos=np.ascontiguousarray(bands["dos"], dtype=np.float64),
                    deg=np.ascontiguousarray(bands["deg"], dtype=np.float64),
                    **run)
    return inst


def uniform_walls(inst_n, dim, kinds, temps):
    """Per-face temperature arrays for 6 walls; ``temps[i]`` is a scalar or None."""
    nx, ny, nz = inst_n
    counts = (ny * nz, ny * nz, nx * nz, nx * nz, nx * ny, nx * ny)
    out = []
    for side in range(6):
        if side >= 2 * dim or kinds[side] != WALL_ISOTHERMAL:
            out.append(None)
        else:
            out.append(np.full(counts[side], float(temps[side])))
    return out


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------
def config_c1(seed: int = 1) -> Instance:
    """2D 16x16 cells of 10 nm, 16 azimuthal x 1 polar directions, 4 linear bands
    (v_b ~ U[1e3, 9e3] m/s, tau_b log-uniform in [1e-12, 1e-9] s, omega_b evenly
    spaced up to 1e14 rad/s).  300 K with a seeded 4x4 hot spot at 310 K; all four
    walls isothermal at 300 K.  Implicit dt = 1 ps, tolerance 1e-4, 50 steps, FP64.
    """
    rng = np.random.default_rng(seed)
    nx = ny = 16
    bands = linear_bands(4, 1e14, rng)
    x0, y0 = (int(v) for v in rng.integers(1, 12, size=2))
    T = np.full((ny, nx), 300.0)
    T[y0:y0 + 4, x0:x0 + 4] = 310.0
    s, w = product_quadrature(1, 16)
    kinds = [WALL_ISOTHERMAL] * 4 + [WALL_ISOTHERMAL] * 2
    n = [nx, ny, 1]
    return make_instance("c1_2d16_d16_b4", 2, n, [1e-8, 1e-8], kinds,
                         uniform_walls(n, 2, kinds, [300.0] * 6), T.reshape(-1), s, w, bands,
                         dt=1e-12, tol=1e-4, max_inner=200, nsteps=50,
                         precision=PRECISION_FP64, seed=seed)


def strip_2d(nx: int, ny: int, n_polar: int, n_azimuthal: int, n_freq: int, seed: int,
             strip_cells: int = 8, name: Optional[str] = None, nsteps: int = 200) -> Instance:
    """2D strip-heater problem: top (+y) wall isothermal with a centred strip of
    ``strip_cells`` face cells at 350 K and 300 K elsewhere, bottom (-y) wall
    isothermal at 300 K, specular side walls; body initially at 300 K.  The
    layout mirrors the paper's demonstration scenario (Sec. 3.1): hot source on
    one isothermal wall, cold opposite wall, symmetric sides."""
    rng = np.random.default_rng(seed)
    bands = quadratic_bands(n_freq, rng)
    s, w = product_quadrature(n_polar, n_azimuthal)
    kinds = [WALL_SPECULAR, WALL_SPECULAR, WALL_ISOTHERMAL, WALL_ISOTHERMAL,
             WALL_ISOTHERMAL, WALL_ISOTHERMAL]
    n = [nx, ny, 1]
    wt = uniform_walls(n, 2, kinds, [300.0] * 6)
    top = np.full(nx, 300.0)
    lo = nx // 2 - strip_cells // 2
    top[max(lo, 0):min(lo + strip_cells, nx)] = 350.0
    wt[3] = top
    return make_instance(name or f"strip2d_{nx}x{ny}_d{n_polar}x{n_azimuthal}_f{n_freq}", 2, n,
                         [1e-8, 1e-8], kinds, wt, np.full(nx * ny, 300.0), s, w, bands,
                         dt=1e-12, tol=1e-4, max_inner=200, nsteps=nsteps,
                         precision=PRECISION_FP64, seed=seed)


def config_c2(seed: int = 2) -> Instance:
    """2D 128x128 cells, 20 polar x 20 azimuthal = 400 directions, 40 frequency
    bands -> 55 entries (quadratic LA/TA dispersion), 8-cell 350 K strip on the
    top wall, bottom 300 K, specular sides; 200 implicit steps of 1 ps, FP64."""
    return strip_2d(128, 128, 20, 20, 40, seed, name="c2_2d128_d400_b55", nsteps=200)


def gaussian_3d(nx: int, ny: int, nz: int, n_polar: int, n_azimuthal: int, n_freq: int,
                seed: int, sigma_cells: float = 6.0, peak: float = 50.0,
                name: Optional[str] = None, nsteps: int = 100,
                precision: int = PRECISION_FP32_MIXED) -> Instance:
    """3D body at 300 K with a seeded Gaussian hot spot (peak +``peak`` K,
    standard deviation ``sigma_cells`` cells, centre drawn in the middle half of
    each axis); all six walls isothermal at 300 K."""
    rng = np.random.default_rng(seed)
    bands = quadratic_bands(n_freq, rng)
    s, w = product_quadrature(n_polar, n_azimuthal)
    n = [nx, ny, nz]
    c = [rng.uniform(0.25 * m, 0.75 * m) for m in n]
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                          indexing="ij")
    r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
    T = 300.0 + peak * np.exp(-r2 / (2.0 * sigma_cells ** 2))
    kinds = [WALL_ISOTHERMAL] * 6
    return make_instance(name or f"gauss3d_{nx}x{ny}x{nz}_d{n_polar}x{n_azimuthal}_f{n_freq}",
                         3, n, [1e-8, 1e-8, 1e-8], kinds, uniform_walls(n, 3, kinds, [300.0] * 6),
                         T.reshape(-1), s, w, bands, dt=1e-12, tol=1e-4, max_inner=200,
                         nsteps=nsteps, precision=precision, seed=seed)


def config_c3(seed: int = 3) -> Instance:
    """3D 64^3 cells, 400 directions, 55 band entries, Gaussian hot spot (+50 K,
    sigma 6 cells), six isothermal 300 K walls; 100 steps, FP32 intensities with
    FP64 reductions and temperature inversion."""
    return gaussian_3d(64, 64, 64, 20, 20, 40, seed, name="c3_3d64_d400_b55", nsteps=100)


def config_c4(seed: int = 4) -> Instance:
    """3D 96^3 cells, 400 directions, 55 band entries, Gaussian hot-spot family;
    100 steps, FP32 intensities (learned warm start of T_{n+1})."""
    return gaussian_3d(96, 96, 96, 20, 20, 40, seed, name="c4_3d96_d400_b55", nsteps=100)


def hotspot_field(n, dim, rng, peak, sigma_cells):
    """300 K body with one Gaussian hot spot whose centre lies in the middle half of
    each axis; ``n`` is [nx, ny, nz] (nz = 1 in 2D)."""
    nx, ny, nz = n
    c = [rng.uniform(0.25 * m, 0.75 * m) for m in n[:dim]] + [0.5] * (3 - dim)
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                          indexing="ij")
    r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 if dim == 3 else \
        (x - c[0]) ** 2 + (y - c[1]) ** 2
    return (300.0 + peak * np.exp(-r2 / (2.0 * sigma_cells ** 2))).reshape(-1)


def batch_geometry(rng: np.random.Generator, index: int, cells_range=(4e3, 2.6e5),
                   dirs_range=(80, 400), entries_range=(8, 40), nsteps: int = 20) -> Instance:
    """One member of the batched workload: 2D or 3D (equal odds), cell count
    log-uniform in ``cells_range`` with a random aspect ratio, a product
    direction set with N_d in ``dirs_range`` (even azimuthal count, so every wall
    mirror maps the set onto itself), a number of band entries drawn directly
    from ``entries_range`` (the longitudinal entries of the quadratic
    dispersion over that many equal bands), one Gaussian hot spot (+10..50 K,
    sigma 2..8 cells) and a random wall mix (each wall isothermal at a
    temperature in [300, 320] K, specular or symmetry; at least one
    isothermal).  FP32 intensities, implicit steps of 1 ps to tolerance 1e-4."""
    dim = int(rng.integers(2, 4))
    cells = math.exp(rng.uniform(math.log(cells_range[0]), math.log(cells_range[1])))
    if dim == 2:
        ar = math.exp(rng.uniform(math.log(0.5), math.log(2.0)))
        nx = max(4, int(round(math.sqrt(cells * ar))))
        n = [nx, max(4, int(round(cells / nx))), 1]
    else:
        a = np.exp(rng.uniform(math.log(0.7), math.log(1.4), size=3))
        a /= np.prod(a) ** (1.0 / 3.0)
        side = cells ** (1.0 / 3.0)
        n = [max(4, int(round(side * v))) for v in a]
    n_polar = int(rng.integers(4, 21))
    lo = 2 * math.ceil(dirs_range[0] / n_polar / 2)
    hi = 2 * math.floor(dirs_range[1] / n_polar / 2)
    n_az = int(2 * rng.integers(lo // 2, hi // 2 + 1))
    n_entries = int(rng.integers(entries_range[0], entries_range[1] + 1))
    full = quadratic_bands(n_entries, rng)
    bands = {k: np.asarray(v)[:n_entries] for k, v in full.items()}  # longitudinal entries
    s, w = product_quadrature(n_polar, n_az)
    kinds = [int(rng.choice([WALL_ISOTHERMAL, WALL_SPECULAR, WALL_SYMMETRY], p=[0.5, 0.3, 0.2]))
             for _ in range(2 * dim)]
    if WALL_ISOTHERMAL not in kinds:
        kinds[int(rng.integers(0, 2 * dim))] = WALL_ISOTHERMAL
    kinds += [WALL_ISOTHERMAL] * (6 - 2 * dim)
    wall_temps = [float(rng.uniform(300.0, 320.0)) for _ in range(6)]
    peak = rng.uniform(10.0, 50.0)
    sigma = rng.uniform(2.0, 8.0)
    T = hotspot_field(n, dim, rng, peak, sigma)
    h = [1e-8] * dim
    return make_instance(f"c5_{index:02d}_{dim}d_" + "x".join(str(v) for v in n[:dim]) +
                         f"_d{n_polar * n_az}_b{n_entries}", dim, n, h, kinds,
                         uniform_walls(n, dim, kinds, wall_temps), T, s, w, bands,
                         dt=1e-12, tol=1e-4, max_inner=200, nsteps=nsteps,
                         precision=PRECISION_FP32_MIXED, seed=index)


def config_c5(seed: int = 5, count: int = 64, cells_range=(4e3, 2.6e5),
              nsteps: int = 20) -> List[Instance]:
    """Batched workload: ``count`` independent 2D/3D geometries drawn by
    ``batch_geometry`` from one seeded stream (cells log-uniform in
    ``cells_range``, 80-400 directions, 8-40 band entries, hot spots and wall
    mixes), FP32 intensities, 20 steps.

    The 64 geometries of the full draw hold 2.19e10 DOF; with FP32 storage and
    the learned warm start their workspaces take 277 GB of the device's
    309 GB (288 GiB)."""
    rng = np.random.default_rng(seed)
    return [batch_geometry(rng, i, cells_range=cells_range, nsteps=nsteps) for i in range(count)]


def paper_demo(n: int = 120, length: float = 525e-6, seed: int = 6, n_freq: int = 40,
               n_dirs: int = 20, dt: float = 1e-12, nsteps: int = 100,
               name: Optional[str] = None) -> Instance:
    """The paper's demonstration scenario (Sec. 3.1 and its schematic figure):
    a square of side ``length`` on an n x n mesh, initially at 300 K; the
    bottom (-y) wall isothermal at 300 K (the cold wall); the top (+y) wall
    isothermal with a centred Gaussian hot spot peaking at 350 K whose
    temperature falls to 1/e^2 of its rise 10 um from the centre,
    T(x) = 300 + 50 exp(-2 (x - x_c)^2 / (10 um)^2), evaluated at the face
    centres; symmetry walls left and right; ``n_dirs`` in-plane directions
    spread uniformly; 40 frequency bands -> 55 entries; forward Euler,
    ``nsteps`` steps of ``dt``.

    The paper's silicon tables are not available: the synthetic quadratic
    dispersion stands in for them, with relaxation times log-uniform in
    [2 ps, 1 ns], so that forward Euler with the appendix's dt = 1 ps keeps
    every update a convex combination (dt / tau_b + dt v_b sum |s_a| / h <= 1;
    the advective share is below 0.003 at 4.375 um cells)."""
    rng = np.random.default_rng(seed)
    bands = quadratic_bands(n_freq, rng, tau_range=(2e-12, 1e-9))
    s, w = product_quadrature(1, n_dirs)
    h = length / n
    kinds = [WALL_SYMMETRY, WALL_SYMMETRY, WALL_ISOTHERMAL, WALL_ISOTHERMAL,
             WALL_ISOTHERMAL, WALL_ISOTHERMAL]
    wt = uniform_walls([n, n, 1], 2, kinds, [300.0] * 6)
    xf = (np.arange(n) + 0.5) * h
    wt[3] = 300.0 + 50.0 * np.exp(-2.0 * (xf - 0.5 * length) ** 2 / (10e-6) ** 2)
    return make_instance(name or f"f1_paper_demo_{n}x{n}_d{n_dirs}_f{n_freq}", 2, [n, n, 1],
                         [h, h], kinds, wt, np.full(n * n, 300.0), s, w, bands, dt=dt, tol=1e-4,
                         max_inner=1, nsteps=nsteps, scheme=SCHEME_EXPLICIT_EULER,
                         precision=PRECISION_FP64, seed=seed)


def config_f1(seed: int = 6) -> Instance:
    """The paper's own workload: 525 um square, 120 x 120 cells, 20 directions
    x 55 band entries (1.58e7 DOF), Gaussian hot spot on one isothermal wall,
    cold opposite wall, symmetry sides; 100 forward-Euler steps of 1 ps, FP64."""
    return paper_demo(seed=seed, name="f1_paper_demo_120x120_d20_b55")


CONFIGS = {"c1": config_c1, "c2": config_c2, "c3": config_c3, "c4": config_c4,
           "f1": config_f1}


def dof_counts(n_freq: int = 40):
    """(longitudinal entries, transverse entries) of ``quadratic_bands``."""
    wmax = _branch_omega_max(LA_V, LA_C)
    wmax_ta = _branch_omega_max(TA_V, TA_C)
    centres = (np.arange(n_freq) + 0.5) * wmax / n_freq
    return n_freq, int(np.sum(centres < wmax_ta))
