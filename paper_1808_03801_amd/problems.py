"""Problem statements (inputs) for the USP-ESBGK particle solver.

This module only *describes* problems: gas constants, geometry, boundary
conditions, numerics and the initial macroscopic fields of every cell.  It
holds none of the solver's per-step arithmetic; the GPU library and the CPU
oracle each receive the plain numbers built here and compute everything else
with their own code.

Setup quantities that the paper's Section 4 uses to *choose* a workload
(standard-state number density, the mean free path of Eq. 36 and the mean
collision time of Eq. 37 at the initial state) are evaluated here once, so
that a time step "dt = 5 tau_c" or a channel height "H = lambda_0 / Kn"
becomes one double that both solvers receive bit-identically.

Gas constants follow the paper's argon setup (Section 4, Eq. 35): the paper
gives no numeric m, mu_ref, T_ref or Pr; the values used are argon's
(m = 6.63e-26 kg, mu_ref = 2.117e-5 Pa s at 273 K, Pr = 2/3).
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

K_B = 1.380649e-23
M_AR = 6.63e-26
MU_REF_AR = 2.117e-5
T_REF_AR = 273.0
P_ATM = 101325.0

# boundary kinds (same integer codes on both solvers' interfaces); BC_OPEN is
# a face to a reservoir: particles leaving through it are gone, and the
# reservoir's gas enters through it every step
BC_DIFFUSE, BC_SPECULAR, BC_PERIODIC, BC_OPEN = 0, 1, 2, 3
# P_ne modes: fixed value, GLL Knudsen number from instantaneous or
# time-averaged fields (Eq. 16-18)
PNE_FIXED, PNE_GLL_INST, PNE_GLL_AVG = 0, 1, 2
# weight of added particles: consistent with the represented PDF for every
# dt*nu_ES, or Eq. 26 as printed
WEIGHT_CONSISTENT, WEIGHT_LITERAL = 0, 1
# per-cell conservation after the relaxation step
CONSERVE_FULL, CONSERVE_NONE = 0, 1
# moments that build the added particles and the ES target: instantaneous
# (Eq. 1) or exponentially time-averaged (Eq. 34, steady flows)
JMOM_INST, JMOM_AVG = 0, 1

# the per-step scheme: USP-ESBGK (Table 2) or the SP-ESBGK baseline (Table 1)
SCHEME_USP, SCHEME_SP = 0, 1
# f_G(t) of step 6: alpha at a per-particle time sample (Eq. 29-32), or its
# expectation over the time distribution (one Gaussian per cell)
ES_SAMPLED, ES_MEAN = 0, 1
# velocity term of the GLL Knudsen number (Eq. 18): lambda |grad |u|| over
# max(|u|, sound speed) (the criterion's authors' convention) or over |u|
GLL_U_SOUND, GLL_U_LITERAL = 0, 1
# step 5 of USP-ESBGK: a Bernoulli trial per particle, or Eq. 9's count
SELECT_BERNOULLI, SELECT_COUNT = 0, 1
# step 6 sampler of f_G(t): its Cholesky factor, or Eq. 11's linear map
ES_CHOLESKY, ES_LINEAR = 0, 1

FACE_XLO, FACE_XHI, FACE_YLO, FACE_YHI = 0, 1, 2, 3


@dataclass
class Gas:
    m: float = M_AR
    kB: float = K_B
    mu_ref: float = MU_REF_AR
    T_ref: float = T_REF_AR
    omega: float = 0.81
    Pr: float = 2.0 / 3.0

    @property
    def R(self) -> float:
        return self.kB / self.m

    def mu(self, T: float) -> float:
        return self.mu_ref * (T / self.T_ref) ** self.omega

    def mean_free_path(self, rho: float, p: float, T: float) -> float:
        # Eq. 36
        return 16.0 / (5.0 * math.sqrt(2.0 * math.pi)) * self.mu(T) / math.sqrt(rho * p)

    def mean_speed(self, T: float) -> float:
        return math.sqrt(8.0 * self.kB * T / (math.pi * self.m))

    def collision_time(self, rho: float, p: float, T: float) -> float:
        # Eq. 37
        return self.mean_free_path(rho, p, T) / self.mean_speed(T)


@dataclass
class Face:
    """A domain face: kind, wall or reservoir temperature T and velocity u
    (diffuse walls: the wall's; open faces: the reservoir gas's, with no
    component normal to the face).  Open faces: reservoir number density n;
    on the part of the face whose tangential coordinate is >= split (2-D),
    density n_b and temperature T_b instead."""

    kind: int = BC_SPECULAR
    T: float = 273.0
    u: Sequence[float] = (0.0, 0.0, 0.0)
    n: float = 0.0
    split: float = math.inf
    n_b: float = 0.0
    T_b: float = 273.0


@dataclass
class Problem:
    """A complete, plain-number description of one solver instance.

    1-D problems resolve the y axis only (cells along y, the x extent is one
    unit-length slab); 2-D problems resolve x and y.  Velocities always carry
    three components.  Cells are numbered iy * nx + ix.
    """

    name: str
    gas: Gas
    dim: int
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    dx: float
    dy: float
    inv_dx: float
    inv_dy: float
    vcell: float
    faces: List[Face]
    accel: Sequence[float]
    dt: float
    Np: float
    init_n: np.ndarray  # [ncell] number density (1/m^3)
    init_u: np.ndarray  # [ncell, 3] m/s
    init_T: np.ndarray  # [ncell] K
    r_p: float = 10.0
    Kn_c: float = 0.1
    pne_mode: int = PNE_GLL_AVG
    pne_fixed: float = 1.0
    n_avg: int = 1000
    avg_start: int = 0
    precision: int = 32
    weight_mode: int = WEIGHT_CONSISTENT
    conserve_mode: int = CONSERVE_FULL
    seed: int = 0
    max_ppc: int = 2048
    jmom_mode: int = JMOM_INST
    spawn_projection: int = 0
    avg_init: int = 0
    # internal plate (2-D): a thin diffuse wall at rest at plate_T on the line
    # x = plate_x for plate_ylo <= y <= plate_yhi
    plate: int = 0
    plate_x: float = 0.0
    plate_ylo: float = 0.0
    plate_yhi: float = 0.0
    plate_T: float = 273.0
    scheme: int = SCHEME_USP
    es_mode: int = ES_SAMPLED
    gll_u: int = GLL_U_SOUND
    select_mode: int = SELECT_BERNOULLI
    es_sampler: int = ES_CHOLESKY
    meta: dict = field(default_factory=dict)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)

    def expected_particles(self) -> int:
        return int(np.sum(np.floor(self.init_n * self.vcell / self.Np + 0.5)))

    def cap_limit(self) -> int:
        """largest max_ppc the GPU library takes for this problem: 2048, or
        1344 with open faces or the plate (that kernel variant stops at the
        256 x (4 | 6) shape)"""
        xb = self.plate or any(f.kind == BC_OPEN for f in self.faces)
        return 1344 if xb else 2048

    def _capacity_for(self, ppc: int, factor: float = 3.0) -> "Problem":
        cap = int(min(self.cap_limit(), max(64, -(-int(factor * ppc) // 64) * 64)))
        return self.replace(max_ppc=cap)

    def with_capacity(self, factor: float = 3.0) -> "Problem":
        """max_ppc = factor x the fullest initial cell (multiple of 64, at
        most cap_limit())"""
        full = float(np.max(np.floor(self.init_n * self.vcell / self.Np + 0.5)))
        cap = int(min(self.cap_limit(), max(64, -(-int(factor * full) // 64) * 64)))
        return self.replace(max_ppc=cap)


def _faces_1d(lo: Face, hi: Face) -> List[Face]:
    # x faces are inert in 1-D
    return [Face(BC_PERIODIC), Face(BC_PERIODIC), lo, hi]


def _grid_1d(ny: int, H: float):
    dy = H / ny
    return dict(dim=1, nx=1, ny=ny, x0=0.0, x1=1.0, y0=0.0, y1=H, dx=1.0, dy=dy,
                inv_dx=1.0, inv_dy=ny / H, vcell=dy)


def standard_state(gas: Gas, T0: float = 273.0, p0: float = P_ATM):
    n0 = p0 / (gas.kB * T0)
    rho0 = gas.m * n0
    lam0 = gas.mean_free_path(rho0, p0, T0)
    tau0 = gas.collision_time(rho0, p0, T0)
    return n0, rho0, lam0, tau0


def couette_1d(Kn=0.1, U_w=100.0, T_w=273.0, ncell=100, ppc=100, dt_over_tau=1.0,
               omega=0.5, precision=64, seed=0, pne_mode=PNE_GLL_AVG, jmom_mode=JMOM_AVG,
               avg_init=1, name="couette") -> Problem:
    """Planar Couette flow between diffuse plates moving at -U_w (bottom) and
    +U_w (top) along x (Section 4.1); Kn = lambda_0 / H.  The added particles
    and the ES target take sigma and q from the Eq. 34 averages started at
    the initial state (with instantaneous moments, 100 particles per cell
    overflow a cell's capacity within a hundred steps)."""
    gas = Gas(omega=omega)
    n0, rho0, lam0, tau0 = standard_state(gas, T_w)
    H = lam0 / Kn
    g = _grid_1d(ncell, H)
    return _sized(Problem(name=name, gas=gas, **g,
                   faces=_faces_1d(Face(BC_DIFFUSE, T_w, (-U_w, 0.0, 0.0)),
                                   Face(BC_DIFFUSE, T_w, (U_w, 0.0, 0.0))),
                   accel=(0.0, 0.0, 0.0), dt=dt_over_tau * tau0, Np=n0 * g["vcell"] / ppc,
                   init_n=np.full(ncell, n0), init_u=np.zeros((ncell, 3)),
                   init_T=np.full(ncell, T_w), precision=precision, seed=seed,
                   pne_mode=pne_mode, jmom_mode=jmom_mode, avg_init=avg_init,
                   meta=dict(H=H, lam0=lam0, tau0=tau0, n0=n0, U_w=U_w, T_w=T_w, Kn=Kn)))


def thermal_couette_1d(Kn=1e-3, dT=10.0, T_w=273.0, ncell=1000, ppc=500, dt_over_tau=5.0,
                       omega=0.81, precision=32, seed=0, init_ns=True,
                       pne_mode=PNE_GLL_AVG, jmom_mode=JMOM_AVG, spawn_projection=0, avg_init=1,
                       name="thermal_couette") -> Problem:
    """Stationary diffuse plates at T_w + dT (bottom) and T_w - dT (top)
    (Section 4.1).  With init_ns the gas starts on the Fourier profile of a
    gas with mu ~ T^omega (T^(1+omega) linear in y) at uniform pressure."""
    gas = Gas(omega=omega)
    n0, rho0, lam0, tau0 = standard_state(gas, T_w)
    H = lam0 / Kn
    g = _grid_1d(ncell, H)
    yc = (np.arange(ncell) + 0.5) * g["dy"]
    Tb, Tt = T_w + dT, T_w - dT
    if init_ns:
        a = omega + 1.0
        T = (Tb ** a + (Tt ** a - Tb ** a) * yc / H) ** (1.0 / a)
    else:
        T = np.full(ncell, T_w)
    n = P_ATM / (gas.kB * T)
    return _sized(Problem(name=name, gas=gas, **g,
                   faces=_faces_1d(Face(BC_DIFFUSE, Tb), Face(BC_DIFFUSE, Tt)),
                   accel=(0.0, 0.0, 0.0), dt=dt_over_tau * tau0, Np=n0 * g["vcell"] / ppc,
                   init_n=n, init_u=np.zeros((ncell, 3)), init_T=T, precision=precision,
                   seed=seed, pne_mode=pne_mode, jmom_mode=jmom_mode,
                   spawn_projection=spawn_projection, avg_init=avg_init,
                   meta=dict(H=H, lam0=lam0, tau0=tau0, n0=n0, T_bottom=Tb, T_top=Tt, Kn=Kn)))


def sod_1d(Kn=1e-3, L=1.0, ncell=1000, mean_ppc=500, rho_ratio=8.0, p_ratio=10.0,
           T_l=273.0, dt_over_tau=5.0, omega=0.81, precision=32, seed=0,
           pne_mode=PNE_GLL_INST, jmom_mode=JMOM_AVG, spawn_projection=1, open_ends=False,
           name="sod") -> Problem:
    """Sod shock tube along the resolved axis (Section 4.3), closed by
    specular ends, or with open_ends by open faces to reservoirs holding the
    initial left and right states (the paper's open boundaries; the waves do
    not reach the ends before t_final).  rho_l is chosen so that
    lambda_l = Kn * L.  At a few
    hundred particles per cell and dt = 5 tau_c the instantaneous-moment
    scheme is unstable (the paper used 2.5e4-2e5 particles per cell), so the
    stress and heat flux of the added particles are time-averaged here too."""
    gas = Gas(omega=omega)
    T_r = T_l * rho_ratio / p_ratio
    lam_l = Kn * L
    c = 16.0 / (5.0 * math.sqrt(2.0 * math.pi))
    rho_l = c * gas.mu(T_l) / (lam_l * math.sqrt(gas.R * T_l))
    n_l = rho_l / gas.m
    n_r = n_l / rho_ratio
    p_l = n_l * gas.kB * T_l
    tau_l = gas.collision_time(rho_l, p_l, T_l)
    g = _grid_1d(ncell, L)
    yc = (np.arange(ncell) + 0.5) * g["dy"]
    left = yc < 0.5 * L
    n = np.where(left, n_l, n_r)
    T = np.where(left, T_l, T_r)
    ppc_l = 2.0 * mean_ppc * rho_ratio / (rho_ratio + 1.0)
    if open_ends:
        ends = (Face(BC_OPEN, T_l, n=n_l), Face(BC_OPEN, T_r, n=n_r))
    else:
        ends = (Face(BC_SPECULAR), Face(BC_SPECULAR))
    return _sized(Problem(name=name, gas=gas, **g,
                   faces=_faces_1d(*ends),
                   accel=(0.0, 0.0, 0.0), dt=dt_over_tau * tau_l, Np=n_l * g["vcell"] / ppc_l,
                   init_n=n, init_u=np.zeros((ncell, 3)), init_T=T, precision=precision,
                   seed=seed, pne_mode=pne_mode, jmom_mode=jmom_mode,
                   spawn_projection=spawn_projection,
                   meta=dict(L=L, lam_l=lam_l, tau_l=tau_l, rho_l=rho_l, p_l=p_l, T_r=T_r, Kn=Kn)))


# Table 4: (rho_l in kg/m^3, [(N_cell, dt / tau_c,l), ...]) of the two Sod cases;
# rho_r = rho_l / 8 and the two initial temperatures of Section 4.3
SOD_TABLE4 = {1: (1e-5, [(400, 0.2), (100, 0.8), (50, 1.5)]),
              2: (1e-4, [(1200, 0.2), (240, 1.0), (60, 4.0)])}
SOD_T_L, SOD_T_R = 273.008012, 273.00641
SOD_T_FINAL = 6.8e-4


def sod_table4(case, row, mean_ppc=500, omega=0.81, precision=32, seed=0, open_ends=False,
               **kw) -> Problem:
    """One row of the paper's Sod series (Section 4.3, Table 4): tube of 1 m,
    rho_l of the case, rho_r = rho_l / 8, the given T_l and T_r (pressure
    ratio 8.00005), N_cell cells and dt = (dt / tau_c,l) tau_c,l with tau_c,l
    of Eq. 37 at the left state.  Specular ends by default (no wave reaches
    an end before t_final); open_ends gives the paper's open boundaries, for
    which the GPU library holds at most 1365 particles per cell (at 500 per
    cell the dense side outgrows that: take mean_ppc of about 350 there).
    The paper's 2e5 / 2.5e4 particles per cell (left / right) are replaced by
    mean_ppc (left 2 * 8/9 mean_ppc, right 2/9 of it); meta t_final =
    6.8e-4 s and the number of steps that reaches it.  The added particles
    take the weights of Eq. 26 as printed: at these counts the consistent
    weights (1 / (nu_ES dt) larger on the dilute side, where nu_ES dt is
    about 0.07) let an occasional run grow a weight of thousands and
    overflow a cell, the printed ones do not."""
    rho_l, rows = SOD_TABLE4[case]
    ncell, dto = rows[row]
    gas = Gas(omega=omega)
    p_l = rho_l * gas.R * SOD_T_L
    kn = gas.mean_free_path(rho_l, p_l, SOD_T_L)  # lambda_l / L with L = 1 m
    pb = sod_1d(Kn=kn, ncell=ncell, mean_ppc=mean_ppc, rho_ratio=8.0,
                p_ratio=8.0 * SOD_T_L / SOD_T_R, T_l=SOD_T_L, dt_over_tau=dto, omega=omega,
                precision=precision, seed=seed, open_ends=open_ends,
                name="sod_t4_%d_%d" % (case, row), **kw)
    steps = int(round(SOD_T_FINAL / pb.dt))
    meta = dict(pb.meta, case=case, row=row, t_final=SOD_T_FINAL, steps=steps)
    return pb.replace(meta=meta, weight_mode=WEIGHT_LITERAL)


def poiseuille_1d(Kn=1e-3, dpdx=4.0e6, T_w=273.0, ncell=100, ppc=500, dt_over_tau=5.0,
                  omega=0.81, precision=32, seed=0, pne_mode=PNE_GLL_AVG,
                  jmom_mode=JMOM_AVG, spawn_projection=0, avg_init=1, name="poiseuille") -> Problem:
    """Plane Poiseuille flow (Section 4.2, Table 3) driven by a uniform body
    acceleration a_x = (dp/dx) / rho_0 along the plates."""
    gas = Gas(omega=omega)
    n0, rho0, lam0, tau0 = standard_state(gas, T_w)
    H = lam0 / Kn
    g = _grid_1d(ncell, H)
    return _sized(Problem(name=name, gas=gas, **g,
                   faces=_faces_1d(Face(BC_DIFFUSE, T_w), Face(BC_DIFFUSE, T_w)),
                   accel=(dpdx / rho0, 0.0, 0.0), dt=dt_over_tau * tau0,
                   Np=n0 * g["vcell"] / ppc, init_n=np.full(ncell, n0),
                   init_u=np.zeros((ncell, 3)), init_T=np.full(ncell, T_w),
                   precision=precision, seed=seed, pne_mode=pne_mode, jmom_mode=jmom_mode,
                   spawn_projection=spawn_projection, avg_init=avg_init,
                   meta=dict(H=H, lam0=lam0, tau0=tau0, rho0=rho0, n0=n0, dpdx=dpdx, T_w=T_w,
                             Kn=Kn)))


def cavity_2d(Kn=1e-3, n=128, ppc=200, U_lid=50.0, T_w=273.0, omega=0.81, precision=32,
              seed=0, pne_mode=PNE_GLL_AVG, jmom_mode=JMOM_AVG, spawn_projection=0, avg_init=1,
              name="cavity") -> Problem:
    """Lid-driven square cavity (Section 4.4): four diffuse walls at T_w, the
    top one moving at U_lid along x; dt = 0.3 dx / mean speed (the
    dt/tau_c = 0.3 dx/lambda entry of Tables 5-6)."""
    gas = Gas(omega=omega)
    n0, rho0, lam0, tau0 = standard_state(gas, T_w)
    L = lam0 / Kn
    d = L / n
    still = Face(BC_DIFFUSE, T_w)
    faces = [still, still, still, Face(BC_DIFFUSE, T_w, (U_lid, 0.0, 0.0))]
    nc = n * n
    return _sized(Problem(name=name, gas=gas, dim=2, nx=n, ny=n, x0=0.0, x1=L, y0=0.0, y1=L, dx=d,
                   dy=d, inv_dx=n / L, inv_dy=n / L, vcell=d * d, faces=faces,
                   accel=(0.0, 0.0, 0.0), dt=0.3 * d / gas.mean_speed(T_w),
                   Np=n0 * d * d / ppc, init_n=np.full(nc, n0), init_u=np.zeros((nc, 3)),
                   init_T=np.full(nc, T_w), precision=precision, seed=seed, pne_mode=pne_mode,
                   jmom_mode=jmom_mode, spawn_projection=spawn_projection, avg_init=avg_init,
                   meta=dict(L=L, lam0=lam0, tau0=tau0, n0=n0, U_lid=U_lid, Kn=Kn)))


def open_channel_1d(Kn=0.1, ncell=50, ppc=100, n_hi=1.0, T_lo=273.0, T_hi=273.0, omega=0.5,
                    precision=64, seed=0, empty=False, pne_mode=PNE_GLL_AVG,
                    jmom_mode=JMOM_AVG, avg_init=1, name="open_channel") -> Problem:
    """A 1-D channel between two reservoirs: at y = 0 the standard state at
    T_lo (n0 = p_atm / (k T_lo)), at y = H the density n_hi * n0 at T_hi;
    H = lambda_0 / Kn, dt = 0.3 dy / mean speed.  The gas starts at the low
    reservoir's state (or as vacuum with `empty`)."""
    gas = Gas(omega=omega)
    n0, rho0, lam0, tau0 = standard_state(gas, T_lo)
    H = lam0 / Kn
    g = _grid_1d(ncell, H)
    lo = Face(BC_OPEN, T_lo, n=n0)
    hi = Face(BC_OPEN, T_hi, n=n_hi * n0)
    init_n = np.full(ncell, 0.0 if empty else n0)
    return _sized(Problem(name=name, gas=gas, **g, faces=_faces_1d(lo, hi),
                   accel=(0.0, 0.0, 0.0), dt=0.3 * g["dy"] / gas.mean_speed(T_lo),
                   Np=n0 * g["vcell"] / ppc, init_n=init_n, init_u=np.zeros((ncell, 3)),
                   init_T=np.full(ncell, T_lo), precision=precision, seed=seed,
                   pne_mode=pne_mode, jmom_mode=jmom_mode, avg_init=avg_init,
                   meta=dict(H=H, lam0=lam0, tau0=tau0, n0=n0, Kn=Kn)))._capacity_for(ppc)


def slit_2d(Kn=0.01, a_cells=20, ppc=100, p_ratio=2.0, T1=273.0, n1=1.0e20, omega=0.5,
            precision=32, seed=0, pne_mode=PNE_GLL_AVG, jmom_mode=JMOM_AVG,
            spawn_projection=0, avg_init=1, n_avg=300, weight_mode=WEIGHT_LITERAL, cfl=0.3,
            extent=10, name="slit") -> Problem:
    """Flow through a slit of width a between two chambers (Section 4.5),
    half domain by the symmetry plane y = 0: x in [-E a, E a], y in [0, E a]
    with E = extent (10: the paper's domain height 20a), cell size
    a / a_cells (400 x 200 cells at a_cells = 20).  A thin diffuse
    plate at T1 on x = 0 for y >= a/2; specular symmetry plane at y = 0; open
    faces to the upstream reservoir (n1, T1) on the left and on the top of
    the left chamber, to the downstream reservoir (n1 / p_ratio, T1) on the
    right and on the top of the right chamber.  Kn = lambda_1 / a with the
    Eq. 36 mean free path of the upstream state; hard spheres by default (the
    paper's slit gas).  The chambers start at their reservoirs' states;
    ppc is the mean over the domain; dt = cfl dx / mean speed (cfl = 0.3: nu_ES dt =
    0.08 at Kn = 0.1 and 0.8 at Kn = 0.01).  Added-particle weights as Eq. 26
    prints them: with the consistent weights (1 / (nu_ES dt) larger) the
    conservation correction of those heavy particles heats the downstream
    jet (at Kn = 0.1 its chamber reached 700 K mean and lost half its mass
    in 3000 steps; at Kn = 0.01 cells on the axis overflowed).  The jet forms
    over the first thousand steps, so the Eq. 34 averages that feed the added
    particles use a window of 300 steps (100 is too noisy at 100 particles
    per cell)."""
    gas = Gas(omega=omega)
    n2 = n1 / p_ratio
    p1 = n1 * gas.kB * T1
    lam1 = gas.mean_free_path(gas.m * n1, p1, T1)
    a = lam1 / Kn
    d = a / a_cells
    nx, ny = 2 * extent * a_cells, extent * a_cells
    xs = -extent * a + (np.arange(nx) + 0.5) * d
    n = np.tile(np.where(xs < 0.0, n1, n2), ny)
    nc = nx * ny
    faces = [Face(BC_OPEN, T1, n=n1), Face(BC_OPEN, T1, n=n2), Face(BC_SPECULAR),
             Face(BC_OPEN, T1, n=n1, split=0.0, n_b=n2, T_b=T1)]
    return _sized(Problem(name=name, gas=gas, dim=2, nx=nx, ny=ny, x0=-extent * a,
                   x1=extent * a, y0=0.0, y1=extent * a, dx=d, dy=d, inv_dx=1.0 / d, inv_dy=1.0 / d,
                   vcell=d * d, faces=faces, accel=(0.0, 0.0, 0.0),
                   dt=cfl * d / gas.mean_speed(T1), Np=0.5 * (n1 + n2) * d * d / ppc,
                   init_n=n, init_u=np.zeros((nc, 3)), init_T=np.full(nc, T1),
                   precision=precision, seed=seed, pne_mode=pne_mode, jmom_mode=jmom_mode,
                   spawn_projection=spawn_projection, avg_init=avg_init, n_avg=n_avg,
                   weight_mode=weight_mode, plate=1, plate_x=0.0,
                   plate_ylo=0.5 * a, plate_yhi=extent * a, plate_T=T1,
                   meta=dict(a=a, lam1=lam1, n1=n1, n2=n2, p1=p1, T1=T1, Kn=Kn)))


def homogeneous_box(ncell=64, ppc=1000, nu_dt=1.0, T=273.0, precision=64, seed=0,
                    pne=1.0, omega=0.5, name="box") -> Problem:
    """Spatially homogeneous gas in a periodic 1-D box whose cells are
    independent replicas; dt is set so that nu * dt = nu_dt at (n0, T)."""
    gas = Gas(omega=omega)
    n0, rho0, lam0, tau0 = standard_state(gas, T)
    nu = P_ATM / gas.mu(T)
    H = 100.0 * lam0
    g = _grid_1d(ncell, H)
    per = Face(BC_PERIODIC)
    return _sized(Problem(name=name, gas=gas, **g, faces=_faces_1d(per, per),
                   accel=(0.0, 0.0, 0.0), dt=nu_dt / nu, Np=n0 * g["vcell"] / ppc,
                   init_n=np.full(ncell, n0), init_u=np.zeros((ncell, 3)),
                   init_T=np.full(ncell, T), precision=precision, seed=seed,
                   pne_mode=PNE_FIXED, pne_fixed=pne,
                   meta=dict(n0=n0, nu=nu, tau0=tau0, lam0=lam0, H=H)))


def sp_esbgk(pb: Problem) -> Problem:
    """The same problem under the SP-ESBGK baseline (Table 1): no added
    particles (P_ne fixed at 0), the Eq. 9 count of particles reassigned,
    velocities through the linear map of Eq. 10-11."""
    return pb.replace(scheme=SCHEME_SP, pne_mode=PNE_FIXED, pne_fixed=0.0,
                      name=pb.name + "_sp")


def _sized(pb: Problem) -> Problem:
    return pb.with_capacity()


def config(name: str, **kw) -> Problem:
    """The named workloads: C1 Couette (FP64), C2 thermal Couette and Sod,
    C3 cavity at three Kn, C5 slit at two Kn."""
    if name == "c1":
        return couette_1d(**kw)
    if name == "c2_tc":
        return thermal_couette_1d(**kw)
    if name == "c2_sod":
        return sod_1d(**kw)
    if name.startswith("c3"):
        kn = {"c3": 1e-3, "c3_kn1e-3": 1e-3, "c3_kn1e-2": 1e-2, "c3_kn1e-1": 0.1}[name]
        return cavity_2d(Kn=kn, **kw)
    if name.startswith("c5"):
        kn = {"c5": 0.01, "c5_kn1e-2": 0.01, "c5_kn1e-1": 0.1}[name]
        return slit_2d(Kn=kn, **kw)
    raise KeyError(name)
