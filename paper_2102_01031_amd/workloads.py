"""The synthetic workloads the library is tested and measured on (program units).

Pure data plus calls into ``inputs`` for the seeded initial conditions.
H_STAR = kappa * sqrt(V(phi0)/3) with kappa = f_*/m_p = 0.5, V(phi0) = 1/4 for
phi0 = 1, lambda = 1: the homogeneous Hubble rate used for the fixed radiation
background (alpha = 1, w = 1/3 gives a(eta) = 1 + H_STAR eta) and for the -H dphi
term of the initial momenta.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

from . import inputs

H_STAR = 0.14433756729740643
KAPPA2 = 0.25


@dataclass(frozen=True)
class FieldIC:
    phi0: float     # homogeneous value
    amp: float      # fluctuation amplitude constant
    mass2: float    # effective mass^2 in w_k
    seed: int


@dataclass(frozen=True)
class ScalarWorkload:
    name: str
    N: int
    dx: float
    dt: float
    steps: int
    integrator: str             # "lf" | "vv2" | "vv4"
    expansion: str              # "none" | "fixed" | "self"
    potential: str              # "phi4" | "phi4_chi2"
    fields: Tuple[FieldIC, ...]
    lam: float = 1.0
    q: float = 0.0
    alpha: float = 1.0
    kappa2: float = KAPPA2
    w_eos: float = 1.0 / 3.0
    H0: float = H_STAR
    a0: float = 1.0
    H_ic: float = H_STAR

    @property
    def nfields(self) -> int:
        return len(self.fields)

    def initial_fields(self, N: int | None = None):
        """(phi list, pi list) of float64 (N,N,N) arrays."""
        n = self.N if N is None else N
        return inputs.scalar_fields(n, self.dx,
                                    [(f.phi0, f.amp, f.mass2, f.seed) for f in self.fields],
                                    self.H_ic, self.a0, self.alpha)


PHI_IC = FieldIC(1.0, 1e-4, 3.0, 1000)

# single-field lambda phi^4, fixed radiation-dominated background, leapfrog
LPHI4_32 = ScalarWorkload("lphi4-32^3-LF-fixedRD", N=32, dx=0.5, dt=0.01, steps=1000,
                          integrator="lf", expansion="fixed", potential="phi4",
                          fields=(PHI_IC,))

_TWO = (FieldIC(1.0, 1e-4, 3.0, 1001), FieldIC(0.0, 1e-6, 100.0, 1002))

# two-field preheating, q = 100, 4th-order Yoshida velocity-Verlet, self-consistent expansion
PREHEAT_128 = ScalarWorkload("preheat-128^3-VV4-self", N=128, dx=0.3, dt=0.005, steps=20,
                             integrator="vv4", expansion="self", potential="phi4_chi2",
                             fields=_TWO, q=100.0)
PREHEAT_256 = ScalarWorkload("preheat-256^3-VV4-self", N=256, dx=0.3, dt=0.005, steps=5,
                             integrator="vv4", expansion="self", potential="phi4_chi2",
                             fields=_TWO, q=100.0)

# differentiable two-field run (no expansion), 2000 VV2 steps at 64^3
ADJ_64 = ScalarWorkload("adjoint-64^3-VV2", N=64, dx=0.3, dt=0.005, steps=2000,
                        integrator="vv2", expansion="none", potential="phi4_chi2",
                        fields=_TWO, q=100.0, H_ic=0.0)


@dataclass(frozen=True)
class U1Workload:
    name: str
    N: int
    dx: float
    dt: float
    steps: int
    lam: float = 1.0
    v: float = 1.0
    e: float = 0.5
    kappa_g: float = 1.0
    amplitude: float = 0.1
    seed: int = 1003

    def initial_fields(self, N: int | None = None):
        return inputs.random_phase_u1(self.N if N is None else N, self.amplitude, self.seed)


ABELIAN_HIGGS_128 = U1Workload("abelian-higgs-128^3-LF", N=128, dx=0.4, dt=0.02, steps=50)


@dataclass(frozen=True)
class SU2Workload:
    """SU(2) doublet with SU(2) links: the non-Abelian counterpart of the U(1) run
    (doublet of modulus ``amplitude`` with a white-noise direction per site around
    the symmetric point, links at the identity, no electric field)."""
    name: str
    N: int
    dx: float
    dt: float
    steps: int
    lam: float = 1.0
    v: float = 1.0
    g: float = 0.5
    amplitude: float = 0.1
    seed: int = 1004

    def initial_fields(self, N: int | None = None):
        return inputs.random_direction_su2(self.N if N is None else N, self.amplitude, self.seed)


SU2_HIGGS_128 = SU2Workload("su2-higgs-128^3-LF", N=128, dx=0.4, dt=0.02, steps=50)


@dataclass(frozen=True)
class BatchWorkload:
    name: str = "batch-256x{24,32,48,64}^3-LF-fixedRD-fp32"
    n_real: int = 256
    size_seed: int = 2024
    seed_base: int = 5000
    steps: int = 2000
    base: ScalarWorkload = field(default_factory=lambda: LPHI4_32)

    def sizes(self):
        return inputs.batch_sizes(self.n_real, self.size_seed)

    def initial_fields(self, r: int, N: int):
        f = self.base.fields[0]
        return inputs.scalar_fields(N, self.base.dx, [(f.phi0, f.amp, f.mass2, self.seed_base + r)],
                                    self.base.H_ic, self.base.a0, self.base.alpha)


BATCH = BatchWorkload()
