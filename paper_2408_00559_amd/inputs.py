"""Problem descriptions and seeded synthetic workloads.

This module holds data only: parameter sets, grid specifications and seeded parameter draws.  It
contains none of the method's arithmetic, imports neither the GPU library nor the CPU oracle, and is
the one place both sides take their inputs from.

Model (Section 2 of the paper): N-1 forward rates F_1..F_{N-1} and one common stochastic volatility
V = F_N; parameters beta (elasticity), sigma (volatility of V), alpha_i, phi_i (F_i-V correlation),
rho_ij (rate-rate correlation), tau_i (accrual periods).  Boundary data: Dirichlet payoff on the
lower faces, homogeneous Neumann on the upper faces (eq. bound1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

CAPLET = "caplet"
SWAPTION = "swaption"
NEUMANN = "neumann"
DIRICHLET = "dirichlet"


@dataclass
class Problem:
    """One pricing instance: the PDE data of eq. (mmNd) plus payoff, domain and evaluation point."""

    d: int                       # N: number of spatial axes (d-1 rates + V)
    beta: float
    sigma: float
    alpha: List[float]           # length d-1
    phi: List[float]             # length d-1
    tau: List[float]             # length d-1
    rho: List[List[float]]       # (d-1) x (d-1), unit diagonal
    xmax: List[float]            # length d: F_1^max .. F_{d-1}^max, V^max
    T: float                     # time to maturity (the PDE horizon)
    payoff: str                  # CAPLET (on F_1) or SWAPTION (Section 2 formula)
    K: float
    xeval: List[float]           # length d: (F_1(0), ..., V(0))
    discount: float = 1.0        # price = discount * u(T, xeval)
    boundary: str = "neumann"    # upper faces of the rate axes: NEUMANN (eq. bound1) or DIRICHLET
                                 # (the payoff, eq. bound1_0); V = V^max is Neumann in both

    def check(self) -> "Problem":
        n = self.d - 1
        assert len(self.alpha) == n and len(self.phi) == n and len(self.tau) == n
        assert len(self.rho) == n and all(len(r) == n for r in self.rho)
        assert len(self.xmax) == self.d and len(self.xeval) == self.d
        assert self.boundary in (NEUMANN, DIRICHLET)
        return self


@dataclass
class GridSpec:
    """Either one full grid with per-axis `levels` (M_i = 2^level_i), or the (modified) combination
    technique at level n with offset psi (psi = 0 is the standard technique)."""

    full: bool
    levels: Optional[List[int]] = None
    n: int = 0
    psi: int = 0


def full_grid(levels) -> GridSpec:
    return GridSpec(full=True, levels=list(levels))


def combination(n: int, psi: int) -> GridSpec:
    return GridSpec(full=False, n=n, psi=psi)


def corr_exp(n: int, lam: float, times=None) -> List[List[float]]:
    """rho_ij = exp(-lam |T_i - T_j|) (Section 2); with times=None the index distance is used."""
    t = list(range(n)) if times is None else list(times)
    return [[math.exp(-lam * abs(t[i] - t[j])) for j in range(n)] for i in range(n)]


# ----------------------------------------------------------------------------------------------
# The paper's hypothetical market data (Section 6, Table marketData): tenor 0, 0.5, ..., 5 years,
# tau = 0.5, strike K = 0.011, F^max = 0.04, V^max = 3.5, beta = 1, evaluation at V = 1.
PAPER_T = [0.0, 0.5, 1.0, 1.5, 2.0, 2.5]
PAPER_F0 = [0.0112, 0.0118, 0.0122, 0.0126, 0.0130, 0.0135]
PAPER_ALPHA = [0.0, 0.2366, 0.2145, 0.2221, 0.2068, 0.1932]
PAPER_K = 0.011
PAPER_TAU = 0.5


def paper_caplet(sigma: float = 0.0, phi: float = 0.0, fmax: float = 0.04, vmax: float = 3.5) -> Problem:
    """Caplet with expiry T_1 on F_1, paid at T_2 (Section 6.1): d = 2, beta = 1, discounted with
    P(0,T_2) = 1/((1+tau F_0(0))(1+tau F_1(0)))."""
    disc = 1.0 / ((1.0 + PAPER_TAU * PAPER_F0[0]) * (1.0 + PAPER_TAU * PAPER_F0[1]))
    return Problem(d=2, beta=1.0, sigma=sigma, alpha=[PAPER_ALPHA[1]], phi=[phi], tau=[PAPER_TAU],
                   rho=[[1.0]], xmax=[fmax, vmax], T=PAPER_T[1], payoff=CAPLET, K=PAPER_K,
                   xeval=[PAPER_F0[1], 1.0], discount=disc).check()


def paper_swaption(n_rates: int, sigma: float = 0.3, phi: float = 0.4, lam: float = 0.1,
                   fmax: float = 0.04, vmax: float = 3.5) -> Problem:
    """T_1 x (T_{1+n} - T_1) swaption on F_1..F_n (Section 6), beta = 1, rho_ij = exp(-lam|T_i-T_j|),
    discounted with P(0,T_1) = 1/(1+tau F_0(0))."""
    n = n_rates
    disc = 1.0 / (1.0 + PAPER_TAU * PAPER_F0[0])
    return Problem(d=n + 1, beta=1.0, sigma=sigma, alpha=PAPER_ALPHA[1:1 + n], phi=[phi] * n,
                   tau=[PAPER_TAU] * n, rho=corr_exp(n, lam, PAPER_T[1:1 + n]),
                   xmax=[fmax] * n + [vmax], T=PAPER_T[1], payoff=SWAPTION, K=PAPER_K,
                   xeval=PAPER_F0[1:1 + n] + [1.0], discount=disc).check()


# ----------------------------------------------------------------------------------------------
# Synthetic benchmark workloads.  Domain F_i in [0, 0.2], V in [0, 1.2], alpha_i = 1 (V carries the
# volatility level), tau_i = 0.5, flat initial curve F_i(0) = F0, evaluation point (F0, ..., F0, V0).

def _sabr_instance(d: int, beta: float, sigma: float, phi: float, F0: float, V0: float, K: float,
                   T: float, lam: float, payoff: str) -> Problem:
    n = d - 1
    return Problem(d=d, beta=beta, sigma=sigma, alpha=[1.0] * n, phi=[phi] * n, tau=[0.5] * n,
                   rho=corr_exp(n, lam), xmax=[0.2] * n + [1.2], T=T, payoff=payoff, K=K,
                   xeval=[F0] * n + [V0], discount=1.0).check()


def workload_fg2d() -> dict:
    """d = 2 full grid 65 x 65, FP64, 50 steps: beta 0.5, sigma 0.3, phi -0.3, F0 0.04, V0 0.25,
    caplet 0.5 (F - 0.04)^+ at T = 1."""
    p = _sabr_instance(2, 0.5, 0.3, -0.3, 0.04, 0.25, 0.04, 1.0, 0.1, CAPLET)
    return dict(name="fg2d_65x65", problems=[p], grid=full_grid([6, 6]), steps=50, richardson=False)


def workload_ct4(seed: int = 2, n: int = 7, psi: int = 3, steps: int = 100) -> dict:
    """d = 4 (3 rates + V), modified combination technique n = 7, psi = 3 (every axis >= 9 points),
    beta 0.5, sigma 0.3, phi -0.3, rho_ij = exp(-0.1|i-j|), F0 ~ U[0.02,0.05], V0 ~ U[0.15,0.35]
    (seeded), at-the-money swaption (K = F0), T = 1, 100 steps."""
    rng = np.random.default_rng(seed)
    F0 = float(rng.uniform(0.02, 0.05))
    V0 = float(rng.uniform(0.15, 0.35))
    p = _sabr_instance(4, 0.5, 0.3, -0.3, F0, V0, F0, 1.0, 0.1, SWAPTION)
    return dict(name=f"ct4_n{n}_psi{psi}", problems=[p], grid=combination(n, psi), steps=steps,
                richardson=False)


DOMAIN_FACTOR_D6 = 4.0   # d = 6: upper boundaries at 4x the evaluation point (Section 6 practice)


def relative_domain(p: Problem, factor: float = DOMAIN_FACTOR_D6) -> Problem:
    """Upper boundaries at `factor` times the evaluation point on every axis, as the paper places
    them between 3 and 4 times the point of interest (Section 6)."""
    p.xmax = [factor * x for x in p.xeval]
    return p


def workload_ct6(seed: int = 3, n: int = 8, psi: int = 1, steps: int = 200) -> dict:
    """d = 6 (5 rates + V), modified combination n = 8, psi = 1; parameters drawn as for the d = 4
    workload, domain 4x the evaluation point; Richardson-extrapolated AMFR-W2 (steps and 2*steps)
    for fourth order in time."""
    rng = np.random.default_rng(seed)
    F0 = float(rng.uniform(0.02, 0.05))
    V0 = float(rng.uniform(0.15, 0.35))
    p = relative_domain(_sabr_instance(6, 0.5, 0.3, -0.3, F0, V0, F0, 1.0, 0.1, SWAPTION))
    return dict(name=f"ct6_n{n}_psi{psi}", problems=[p], grid=combination(n, psi), steps=steps,
                richardson=True)


def draw_instances(count: int, seed: int, d: int = 4, T_range=None, lam_range=None) -> List[Problem]:
    """Seeded batch of SABR-LMM swaption instances: beta ~ U[0.3,0.7], sigma ~ U[0.1,0.5],
    phi ~ U[-0.6,0], F0 ~ U[0.02,0.05], V0 ~ U[0.15,0.35], K = F0 U[0.8,1.2]; T = 1 and lambda = 0.1
    unless ranges are given."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        beta = float(rng.uniform(0.3, 0.7))
        sigma = float(rng.uniform(0.1, 0.5))
        phi = float(rng.uniform(-0.6, 0.0))
        F0 = float(rng.uniform(0.02, 0.05))
        V0 = float(rng.uniform(0.15, 0.35))
        K = F0 * float(rng.uniform(0.8, 1.2))
        T = 1.0 if T_range is None else float(rng.uniform(*T_range))
        lam = 0.1 if lam_range is None else float(rng.uniform(*lam_range))
        out.append(_sabr_instance(d, beta, sigma, phi, F0, V0, K, T, lam, SWAPTION))
    return out


def workload_batch4(count: int = 512, seed: int = 4, n: int = 6, psi: int = 1, steps: int = 100) -> dict:
    """Batched serving: `count` seeded parameter sets, d = 4, modified combination n = 6, psi = 1."""
    return dict(name=f"batch4_{count}x_n{n}_psi{psi}", problems=draw_instances(count, seed),
                grid=combination(n, psi), steps=steps, richardson=False)


def surrogate_instances(count: int, seed: int, d: int = 6) -> List[Problem]:
    """Training / held-out instances of the surrogate: the batch distributions plus T ~ U[0.5,1.5]
    and lambda ~ U[0.05,0.3], domain 4x the evaluation point."""
    return [relative_domain(p) for p in draw_instances(count, seed, d=d, T_range=(0.5, 1.5),
                                                        lam_range=(0.05, 0.3))]


def workload_surrogate_labels(count: int, seed: int, n: int = 5, psi: int = 1, steps: int = 100) -> dict:
    """Label generation for the surrogate: d = 6 modified combination n = 5, psi = 1, 100 steps."""
    return dict(name=f"surrogate_d6_n{n}_psi{psi}_seed{seed}", problems=surrogate_instances(count, seed),
                grid=combination(n, psi), steps=steps, richardson=False)


def surrogate_features(p: Problem) -> List[float]:
    """The 8 surrogate inputs (beta, sigma, phi, F0, V0, K, T, lambda) of a drawn instance."""
    lam = -math.log(p.rho[0][1]) if p.d > 2 else 0.1
    return [p.beta, p.sigma, p.phi[0], p.xeval[0], p.xeval[-1], p.K, p.T, lam]
