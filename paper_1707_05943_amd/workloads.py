"""Seeded synthetic workloads for the delay-PDE march.

This module only names problem instances: grid sizes, physical parameters
and seeded random draws.  It holds none of the scheme's arithmetic, so both
the GPU path and the CPU oracle can take their inputs from it.

Conventions (paper, Table 1 and App. B):
  * Absolute units (hbar = c = 1).  Delta is the grid step in x and t.
  * D = n_x = 2a/Delta is an even integer; a is re-derived as D*Delta/2.
  * Columns j = 0..Nx sit at x_j = -a + j*Delta (j = 0 is x = -a); rows
    r = 0..Nt sit at t_r = r*Delta.
  * The incident two-photon state is a Gaussian packet phi with |phi|^2 of
    standard deviation `width`, centred at x0 = -a - 8*width, carrier k0,
    truncated to x <= -a, times a global phase exp(i*theta).  The emitter
    frequency is on resonance with the carrier (omega0 = k0), and k0*a is
    fixed per workload (App. B: omega0*a = k0*a = n*pi).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict, field

import numpy as np

# incident families (Table 1 init_cond 1-3, plus the Gaussian packet)
INC_PLANE = 1      # two-photon plane wave, Eqs. (5)-(6)
INC_EXP1 = 2       # stimulated emission: one exponential photon, emitter excited, Eqs. (7)-(9)
INC_EXP2 = 3       # two exponential photons, Eqs. (10)-(13) (identical, or different: identical_photons = 0)
INC_GAUSS2 = 4     # two identical Gaussian photons


@dataclass
class Instance:
    name: str
    Nx: int
    D: int
    Nt: int
    Delta: float
    omega0: float
    Gamma: float
    incident: int = INC_GAUSS2
    k: float = 0.0          # carrier wavenumber (absolute units)
    alpha: float = 0.0      # exponential packet width, units of Gamma
    x0: float = 0.0         # Gaussian centre
    width: float = 1.0      # Gaussian std of |phi|^2
    phase: float = 0.0      # global phase theta of the two-photon state
    seed: int = 0
    boundary: int = 0       # how the library computes E(t_r): 0 delay series, 1 delay equation
    identical_photons: int = 1   # 0: two different exponential photons (k1, alpha1), (k2, alpha2) (Table 1)
    k1: float = 0.0
    k2: float = 0.0
    alpha1: float = 0.0
    alpha2: float = 0.0
    read_mode: int = 0      # 1: the paper's own reads at x <= -a (diag_cols marched columns there)
    diag_cols: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def a(self) -> float:
        return 0.5 * self.D * self.Delta

    def as_dict(self) -> dict:
        return asdict(self)


def even_D(a: float, Delta: float) -> int:
    """Number of grid steps in the round trip 2a, rounded to an even integer >= 2."""
    return 2 * max(1, int(round(a / Delta)))


def gaussian_instance(name: str, *, Gamma: float, two_a: float, Delta: float,
                      k0a: float, width: float, Nx: int, Nt: int, seed: int) -> Instance:
    D = even_D(0.5 * two_a, Delta)
    a = 0.5 * D * Delta
    k0 = k0a / a
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = float(2.0 * math.pi * rng.random())
    return Instance(name=name, Nx=int(Nx), D=D, Nt=int(Nt), Delta=float(Delta),
                    omega0=k0, Gamma=float(Gamma), incident=INC_GAUSS2, k=k0,
                    x0=-a - 8.0 * width, width=float(width), phase=theta, seed=seed)


def small_gauss(seed: int = 1) -> Instance:
    """D=100, Nx=4000, Nt=4000: Gamma=1, 2a=1, Delta=0.01, k0*a=pi/2, width 1."""
    return gaussian_instance("gauss_D100_Nx4000_Nt4000", Gamma=1.0, two_a=1.0, Delta=0.01,
                             k0a=0.5 * math.pi, width=1.0, Nx=4000, Nt=4000, seed=seed)


def large_gauss(seed: int = 2) -> Instance:
    """D=10000, Nx=262144, Nt=131072: Gamma=1, 2a=10, Delta=1e-3, k0*a=pi/2, width 1."""
    return gaussian_instance("gauss_D10000_Nx262144_Nt131072", Gamma=1.0, two_a=10.0, Delta=1e-3,
                             k0a=0.5 * math.pi, width=1.0, Nx=262144, Nt=131072, seed=seed)


def large_stimulated() -> Instance:
    """Stimulated emission (Eqs. 7-9) on the grid of large_gauss (D=10000,
    Nx=262144, Nt=131072, Delta=1e-3, Gamma=1, k0*a=pi/2 on resonance): an
    exponential packet with alpha=0.5 meets the excited emitter.  The family
    the non-Markovian measures of App. D are defined for."""
    k0 = 0.5 * math.pi / 5.0
    return Instance(name="stim_D10000_Nx262144_Nt131072", Nx=262144, D=10000, Nt=131072, Delta=1e-3, omega0=k0,
                    Gamma=1.0, incident=INC_EXP1, k=k0, alpha=0.5)


def paper_sets() -> dict:
    """The parameter sets of the paper's figures, in the paper's absolute
    units, Ny = Nt + 1.  Validation figures: a two-photon plane wave (identical
    photons, Eqs. 5-6).
    * the error snapshots: nx = 200, Nx = 4000, Ny = 4e4, Delta = 1e-2,
      k = omega0 = pi/2, Gamma = pi/40;
    * |chi|^2 at k0 a = pi/4: nx = 50, Nx = 1e4, Ny = 2.5e4, Delta = 1e-2,
      omega0 = pi, Gamma = pi/20, with k = omega0 and k = omega0 - Gamma;
    * |chi|^2 at k0 a = pi/2: nx = 200, Nx = 1e4, Ny = 2e4, Delta = 1e-2,
      omega0 = pi/2, Gamma = pi/40, with k = omega0 and k = omega0 - Gamma;
    * the strongly non-Markovian cases k0 a = 10.5 pi and 20.5 pi: Nx = 64800,
      Ny = 6e4, Delta = pi/12000, k = omega0 = 100, Gamma = 1 (nx = 2a/Delta =
      2520 and 4920).
    The timing figure (elapsed time against threads): stimulated emission
    (Eqs. 7-9), Nx = 64800, Ny = 6e4, nx = 960, Delta = 2.618e-4,
    k = omega0 = 100, Gamma = 5, alpha = 0.5."""
    def plane(name, D, Nx, Ny, Delta, omega0, Gamma, k):
        return Instance(name=name, Nx=int(Nx), D=int(D), Nt=int(Ny) - 1, Delta=float(Delta),
                        omega0=float(omega0), Gamma=float(Gamma), incident=INC_PLANE, k=float(k))
    pi = math.pi
    out = {}
    for inst in (
        plane("paper_error_snapshots", 200, 4000, 40000, 1e-2, pi / 2, pi / 40, pi / 2),
        plane("paper_chi_k0a_pi4_res", 50, 10000, 25000, 1e-2, pi, pi / 20, pi),
        plane("paper_chi_k0a_pi4_det", 50, 10000, 25000, 1e-2, pi, pi / 20, pi - pi / 20),
        plane("paper_chi_k0a_pi2_res", 200, 10000, 20000, 1e-2, pi / 2, pi / 40, pi / 2),
        plane("paper_chi_k0a_pi2_det", 200, 10000, 20000, 1e-2, pi / 2, pi / 40, pi / 2 - pi / 40),
        plane("paper_chi_nonmarkov_10.5pi", 2520, 64800, 60000, pi / 12000, 100.0, 1.0, 100.0),
        plane("paper_chi_nonmarkov_20.5pi", 4920, 64800, 60000, pi / 12000, 100.0, 1.0, 100.0),
        Instance(name="paper_timing_stimulated", Nx=64800, D=960, Nt=59999, Delta=2.618e-4, omega0=100.0,
                 Gamma=5.0, incident=INC_EXP1, k=100.0, alpha=0.5),
    ):
        out[inst.name] = inst
    return out


def paper_reads(inst: Instance, diag_cols: int | None = None) -> Instance:
    """The instance marched with the paper's own reads at x <= -a.  The
    paper's grid spans x/Delta in [-Nx, Nx] about x = -a, and a point reads
    the delay term D + 1 columns to its left, so the points it can march at
    x <= -a are the Nx - D columns next to -a (the default); left of them it
    supplies the exact solution."""
    d = inst.as_dict()
    d.update(read_mode=1, diag_cols=int(inst.Nx - inst.D if diag_cols is None else diag_cols),
             name=f"{inst.name}_paper_reads")
    return Instance(**d)


def with_sizes(inst: Instance, *, Nx: int | None = None, Nt: int | None = None,
               name: str | None = None) -> Instance:
    """Same physics and grid step, other box sizes (a column window or a row prefix)."""
    d = inst.as_dict()
    if Nx is not None:
        d["Nx"] = int(Nx)
    if Nt is not None:
        d["Nt"] = int(Nt)
    d["name"] = name or f"{inst.name}_Nx{d['Nx']}_Nt{d['Nt']}"
    return Instance(**d)


def tiny_gauss(D: int = 10, Nx: int = 64, Nt: int = 120, seed: int = 3,
               Delta: float = 0.05, k0a: float = 0.5 * math.pi, width: float = 0.5,
               Gamma: float = 1.0) -> Instance:
    """Small grids for oracle cross-checks; x0 is moved close so the packet arrives early."""
    a = 0.5 * D * Delta
    k0 = k0a / a
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = float(2.0 * math.pi * rng.random())
    return Instance(name=f"tiny_D{D}_Nx{Nx}_Nt{Nt}", Nx=Nx, D=D, Nt=Nt, Delta=Delta,
                    omega0=k0, Gamma=Gamma, incident=INC_GAUSS2, k=k0,
                    x0=-a - 4.0 * width, width=width, phase=theta, seed=seed)


def sweep_draw(n: int, seed: int) -> list[Instance]:
    """Heterogeneous parameter sweep: Gamma*2a ~ U[0.1,10], k0*a ~ U[0,2pi),
    width ~ logU[0.2,5]/Gamma, Delta in {0.01, 0.005, 0.002}; Nx is the power of
    two that holds the strip, the packet and its decay (clamped to 1024..16384),
    Nt = 4*Nx."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    Gamma = 1.0
    for i in range(n):
        two_a = float(rng.uniform(0.1, 10.0)) / Gamma
        k0a = float(rng.uniform(0.0, 2.0 * math.pi))
        width = float(math.exp(rng.uniform(math.log(0.2), math.log(5.0)))) / Gamma
        Delta = float(rng.choice([0.01, 0.005, 0.002]))
        theta = float(2.0 * math.pi * rng.random())
        D = even_D(0.5 * two_a, Delta)
        a = 0.5 * D * Delta
        need = max(2 * D, int(math.ceil((16 * width + 2 * a + 10.0 / Gamma) / (4 * Delta))))
        Nx = 1 << max(0, (need - 1).bit_length())
        Nx = min(max(Nx, 1024), 16384)
        k0 = k0a / a
        out.append(Instance(name=f"sweep{seed}_{i}", Nx=Nx, D=D, Nt=4 * Nx, Delta=Delta,
                            omega0=k0, Gamma=Gamma, incident=INC_GAUSS2, k=k0,
                            x0=-a - 8.0 * width, width=width, phase=theta, seed=seed * 100003 + i,
                            boundary=1))
    return out


def sweep_draw_arrays(n: int, seed: int) -> dict:
    """The distribution of sweep_draw as arrays, for draws too large to hold
    as Instance objects (a million points): Gamma = 1; each column is drawn
    as a whole (so the points differ from sweep_draw's for the same seed).
    Keys: two_a, k0a, width, Delta, theta and the derived D, a, Nx, Nt, k0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    two_a = rng.uniform(0.1, 10.0, n)
    k0a = rng.uniform(0.0, 2.0 * math.pi, n)
    width = np.exp(rng.uniform(math.log(0.2), math.log(5.0), n))
    Delta = rng.choice(np.array([0.01, 0.005, 0.002]), n)
    theta = 2.0 * math.pi * rng.random(n)
    D = 2 * np.maximum(1, np.round(0.5 * two_a / Delta).astype(np.int64))
    a = 0.5 * D * Delta
    need = np.maximum(2 * D, np.ceil((16.0 * width + 2.0 * a + 10.0) / (4.0 * Delta)).astype(np.int64))
    Nx = np.clip(1 << np.ceil(np.log2(np.maximum(need, 1))).astype(np.int64), 1024, 16384)
    Nx = np.where(Nx < need, 2 * Nx, Nx).clip(1024, 16384)       # guard the float log2 at exact powers
    return {"two_a": two_a, "k0a": k0a, "width": width, "Delta": Delta, "theta": theta, "D": D, "a": a,
            "Nx": Nx, "Nt": 4 * Nx, "k0": k0a / a, "seed": seed}


def sweep_point(d: dict, i: int) -> Instance:
    """point i of a sweep_draw_arrays draw as an Instance"""
    a, w = float(d["a"][i]), float(d["width"][i])
    k0 = float(d["k0"][i])
    return Instance(name=f"sweepA{d['seed']}_{i}", Nx=int(d["Nx"][i]), D=int(d["D"][i]), Nt=int(d["Nt"][i]),
                    Delta=float(d["Delta"][i]), omega0=k0, Gamma=1.0, incident=INC_GAUSS2, k=k0,
                    x0=-a - 8.0 * w, width=w, phase=float(d["theta"][i]), seed=int(d["seed"]) * 1000003 + i,
                    boundary=1)
