"""Pins of the oracle's variants: the Dirichlet upper faces of eq. (bound1_0), the W-method with
W = P (the theta-method with a fixed number of Gauss-Seidel sweeps, Section 4.2), the generic
s-stage driver of eq. (row-s), and the stability reading nu = theta at d = 5 and 6.

As in test_oracle_pins.py, every check is against something other than the oracle itself: closed
forms, dense linear algebra on matrices assembled column by column from the operator, the exact
solution of the semi-discrete ODE, and eigenvalues of one-step matrices.
"""
import math

import numpy as np
import pytest
from scipy import linalg as sla

from paper_2408_00559_amd import inputs as I
from test_oracle_pins import _dense_operator, _generator_on_quadratic, _isolate_axis


def _dirichlet(p):
    p.boundary = I.DIRICHLET
    return p


def _coords(orc, p, levels):
    shp = orc.grid_shape(levels)
    h = [p.xmax[i] / (1 << levels[i]) for i in range(p.d)]
    out = []
    for J in range(orc.grid_size(levels)):
        idx = np.unravel_index(J, shp)[::-1]          # axis 1 fastest
        out.append((idx, np.array([idx[i] * h[i] for i in range(p.d)])))
    return out


def _outer(p, idx, M):
    """Outer nodes of eq. (bound1_0): any lower face, or the upper face of a rate axis."""
    if min(idx) == 0:
        return True
    return p.boundary == I.DIRICHLET and any(idx[i] == M[i] for i in range(p.d - 1))


# ----------------------------------------------------------------------------------------------
# Dirichlet upper faces, eq. (bound1_0)

@pytest.mark.parametrize("d,beta", [(2, 0.5), (3, 1.0), (4, 0.5)])
def test_dirichlet_operator_exact_on_quadratics(orc, d, beta):
    """With the payoff held on the upper rate faces there is no ghost value: central differences
    see the stored face values, so on a quadratic Sketch 1 equals the generator at EVERY unknown
    node off the V = V^max face, including those next to the rate faces; Outer rows (lower faces
    and the rate faces) are null."""
    rng = np.random.default_rng(20 + d)
    p = _dirichlet(I.draw_instances(1, seed=d, d=d)[0])
    p.beta = beta
    p.phi = list(rng.uniform(-0.6, 0.6, d - 1))
    levels = [3, 2, 2, 3][:d]
    M = [1 << l for l in levels]
    b = rng.normal(size=d)
    Q = rng.normal(size=(d, d))
    co = _coords(orc, p, levels)
    Y = np.array([b @ x + x @ Q @ x for _, x in co])
    F = orc.eval_F(p, levels, Y)
    adjacent = 0
    for J, (idx, x) in enumerate(co):
        if _outer(p, idx, M):
            assert F[J] == 0.0
            continue
        if idx[d - 1] == M[d - 1]:                   # V^max stays Neumann
            continue
        ref = _generator_on_quadratic(p, x, b, Q)
        assert abs(F[J] - ref) <= 1e-9 * (1 + abs(ref)), (idx, F[J], ref)
        adjacent += any(idx[i] == M[i] - 1 for i in range(d - 1))
    assert adjacent > 0


@pytest.mark.parametrize("d,levels", [(2, [3, 2]), (3, [2, 3, 2]), (4, [2, 2, 1, 2])])
def test_dirichlet_axis_solve_vs_dense(orc, d, levels):
    """Directional systems with Dirichlet rate faces (size M_i - 1 along a rate axis) against a dense
    solve of (I - nu dt A_i), A_i assembled column by column from the isolated operator."""
    p = _dirichlet(I.draw_instances(1, seed=8, d=d)[0])
    n = orc.grid_size(levels)
    M = [1 << l for l in levels]
    co = _coords(orc, p, levels)
    rng = np.random.default_rng(6)
    nudt = 0.41
    G = np.array([0.0 if _outer(p, idx, M) else rng.normal() for idx, _ in co])
    for ax in range(d):
        q = _isolate_axis(p, ax)
        A = np.zeros((n, n))
        for J in range(n):
            e = np.zeros(n)
            e[J] = 1.0
            A[:, J] = orc.eval_F(q, levels, e)
        ref = np.linalg.solve(np.eye(n) - nudt * A, G)
        K = orc.solve_axis(p, levels, ax, nudt, G)
        np.testing.assert_allclose(K, ref, rtol=1e-11, atol=1e-13)


def _bachelier_interval(F0, K, kappa, L, tau, t, terms=400):
    """u_t = kappa u_FF on [0, L], u(0) = g(0) = 0, u(L) = g(L), u(t=0) = g = tau (F - K)^+: the
    linear steady state plus the sine series of the transient (separation of variables)."""
    gL = tau * (L - K)
    u = gL * F0 / L
    for n in range(1, terms + 1):
        k = n * math.pi / L

        def prim(a, c, F):        # antiderivative of (a F + c) sin(k F)
            return -(a * F + c) * math.cos(k * F) / k + a * math.sin(k * F) / (k * k)

        # g - linear part: -gL F / L on [0, K], (tau - gL / L) F - tau K on [K, L]
        bn = 2.0 / L * (prim(-gL / L, 0.0, K) - prim(-gL / L, 0.0, 0.0)
                        + prim(tau - gL / L, -tau * K, L) - prim(tau - gL / L, -tau * K, K))
        u += bn * math.exp(-kappa * k * k * t) * math.sin(k * F0)
    return u


def test_dirichlet_bachelier_on_an_interval(orc):
    """sigma = 0, beta = 0 freezes V and makes each V-line the heat equation u_t = (alpha V)^2/2 u_FF.
    With the payoff held at F = 0 and F = F^max (eq. bound1_0) the exact solution on the interval is
    the linear steady state plus a decaying sine series; the boundary is close enough to the strike
    that the Neumann condition gives a visibly different price.  The oracle's error falls at second
    order in h and its h-extrapolation reaches the series."""
    V0, F0, K, T, alpha, L = 0.25, 0.04, 0.04, 0.5, 0.12, 0.08
    p = _dirichlet(I.Problem(d=2, beta=0.0, sigma=0.0, alpha=[alpha], phi=[0.0], tau=[0.5], rho=[[1.0]],
                             xmax=[L, 4 * V0], T=T, payoff="caplet", K=K, xeval=[F0, V0]))
    ref = _bachelier_interval(F0, K, 0.5 * (alpha * V0) ** 2, L, 0.5, T)
    prices = [orc.price(p, I.full_grid([lv, 2]), 64) for lv in (7, 8, 9)]
    errs = [abs(x - ref) for x in prices]
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, (errs, ref)
    extrap = (4 * prices[2] - prices[1]) / 3
    assert abs(extrap - ref) / ref < 2e-6, (prices, extrap, ref)
    p.boundary = I.NEUMANN
    neu = orc.price(p, I.full_grid([9, 2]), 64)
    assert abs(neu - ref) / ref > 100 * abs(extrap - ref) / ref, (neu, ref)


def test_dirichlet_far_boundary_reproduces_black(orc):
    """With the rate face far from the strike both boundary kinds give the paper's caplet at level 9
    (Table fg_sigma0: 6.058877 bps, error 7.58e-5 bps with 256 steps)."""
    p = I.paper_caplet()
    neu = orc.price(p, I.full_grid([9, 9]), 256) * 1e4
    dirp = orc.price(_dirichlet(I.paper_caplet()), I.full_grid([9, 9]), 256) * 1e4
    assert abs(dirp - 6.058877) < 1e-4 and abs(dirp - neu) < 1e-8, (dirp, neu)


def test_dirichlet_degenerate_grids_hold_the_payoff(orc):
    """A level-0 rate axis has only its two faces, both boundary data under eq. (bound1_0): the grid
    has no unknowns, so its solution stays the payoff for all t (the degenerate grids of Section 5)."""
    p = _dirichlet(I.draw_instances(1, seed=4, d=3)[0])
    levels = [0, 3, 2]
    Y0 = orc.initial_data(p, levels)
    Y = orc.solve_grid(p, levels, 7)
    assert np.array_equal(Y, Y0)
    p.boundary = I.NEUMANN
    assert not np.array_equal(orc.solve_grid(p, levels, 7), Y0)


# ----------------------------------------------------------------------------------------------
# W = P: theta-method + Gauss-Seidel as a W-method (Section 4.2)

def _lower_dense(orc, p, levels):
    """Inner-node block of A (columns F(e_J) of Sketch 1) and its lower triangle in theta_0 order."""
    A = _dense_operator(orc, p, levels)
    return A, np.tril(A)


@pytest.mark.parametrize("d,levels,bc", [(2, [3, 2], I.NEUMANN), (3, [2, 2, 1], I.NEUMANN),
                                          (3, [2, 1, 2], I.DIRICHLET), (4, [1, 2, 1, 2], I.NEUMANN)])
def test_lower_solve_vs_dense(orc, d, levels, bc):
    """(I - theta dt P) K = R by forward substitution against a dense triangular solve, P the lower
    triangle (with diagonal) of the matrix whose columns are Sketch 1 applied to unit vectors."""
    p = I.draw_instances(1, seed=13, d=d)[0]
    p.boundary = bc
    n = orc.grid_size(levels)
    M = [1 << l for l in levels]
    co = _coords(orc, p, levels)
    outer = np.array([_outer(p, idx, M) for idx, _ in co])
    A, Pm = _lower_dense(orc, p, levels)
    thdt = 0.173
    rng = np.random.default_rng(2)
    R = np.where(outer, 0.0, rng.normal(size=n))
    Mx = np.eye(n) - thdt * Pm
    ref = sla.solve_triangular(Mx, R, lower=True)
    K = orc.solve_lower(p, levels, thdt, R)
    np.testing.assert_allclose(K, ref, rtol=1e-11, atol=1e-13)
    assert np.all(K[outer] == 0.0)


def _order(orc, p, levels, scheme, steps_list):
    A = _dense_operator(orc, p, levels)
    Y0 = orc.initial_data(p, levels)
    exact = sla.expm(p.T * A) @ Y0
    errs = []
    for steps in steps_list:
        Y = orc.solve_grid(p, levels, steps, scheme=scheme)
        errs.append(np.max(np.abs(Y - exact)))
    return errs, [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


@pytest.mark.parametrize("stages", [2, 3])
def test_theta_gauss_seidel_second_order_at_half(orc, stages):
    """Section 4.2: with s >= 2 Gauss-Seidel sweeps the scheme has order (at least) 2 at
    theta = 1/2 (Crank-Nicolson); with s = 2 exactly 2 ..."""
    p = I.draw_instances(1, seed=11, d=2)[0]
    p.T = 0.5
    errs, rates = _order(orc, p, [3, 2], orc.scheme_theta_gs(0.5, stages), (256, 512, 1024, 2048))
    if stages == 2:
        assert 1.9 < rates[-1] < 2.1 and 1.85 < rates[-2] < 2.15, (errs, rates)
    else:
        assert rates[-1] > 1.9 and rates[-2] > 1.85, (errs, rates)


def test_theta_gauss_seidel_first_order_otherwise(orc):
    """... and order 1 for theta != 1/2 (seen once the sweeps' own error, which shrinks like dt^s,
    falls below that of the theta-method: s = 4 sweeps)."""
    p = I.draw_instances(1, seed=11, d=2)[0]
    p.T = 0.5
    errs, rates = _order(orc, p, [3, 2], orc.scheme_theta_gs(1.0, 4), (1024, 2048, 4096))
    assert all(0.95 < r < 1.05 for r in rates), (errs, rates)


def test_generic_stages_are_theta_method_iterations(orc):
    """eq. (row-s) with a_rj = theta, q_rj = -1, b_r = 1 is s fixed-point sweeps of the theta-method
    preconditioned by (I - theta dt W) for ANY W (the derivation of Section 4.2).  With the AMF W of
    eq. (Wmat1) the generic s-stage driver must therefore approach the dense theta-method step
    (I - theta dt A)^-1 (I + (1 - theta) dt A) Y as s grows, geometrically."""
    p = I.draw_instances(1, seed=21, d=3)[0]
    levels = [2, 2, 2]
    A = _dense_operator(orc, p, levels)
    n = A.shape[0]
    Y0 = orc.initial_data(p, levels)
    th, dt = 0.5, 0.02
    exact = np.linalg.solve(np.eye(n) - th * dt * A, (np.eye(n) + (1 - th) * dt * A) @ Y0)
    dist = []
    for s in range(1, 7):
        sc = orc.scheme_generic([[th] * r for r in range(s)], [[-1.0] * r for r in range(s)],
                                [1.0] * s, th, th)
        Y = Y0.copy()
        orc.advance(p, levels, Y, dt, 1, scheme=sc)
        dist.append(np.max(np.abs(Y - exact)))
    assert all(dist[i + 1] < 0.5 * dist[i] for i in range(5)), dist
    assert dist[-1] < 1e-6 * np.max(np.abs(exact - Y0)), dist


# ----------------------------------------------------------------------------------------------
# Stability of nu = theta at d = 5 and d = 6 (the bound of Section 4.1 grows with N)

def _step_radius(orc, p, levels, dt):
    n = orc.grid_size(levels)
    shp = orc.grid_shape(levels)
    inner = [J for J in range(n) if min(np.unravel_index(J, shp)) > 0]
    R = np.zeros((len(inner), len(inner)))
    for c, J in enumerate(inner):
        Y = np.zeros(n)
        Y[J] = 1.0
        orc.advance(p, levels, Y, dt, 1)
        R[:, c] = Y[inner]
    return float(np.max(np.abs(np.linalg.eigvals(R))))


@pytest.mark.parametrize("which,levels", [("ct6", [2, 1, 1, 1, 1, 2]), ("ct6", [3, 2, 1, 1, 1, 1]),
                                           ("ct6", [1, 1, 1, 1, 2, 3]), ("labels", [3, 1, 1, 1, 1, 1]),
                                           ("d5", [3, 2, 1, 1, 1])])
def test_step_is_stable_at_d5_d6(orc, which, levels):
    """nu = theta: one-step matrices of AMFR-W2 have spectral radius <= 1 over the d = 6 workload's
    dt (0.0025 fine, 0.005 coarse), the surrogate labels' dt range (0.005 to 0.015) and far beyond
    (dt = 1), for d = 6 and d = 5 parameter draws."""
    if which == "ct6":
        ps = I.workload_ct6()["problems"]
    elif which == "labels":
        ps = I.surrogate_instances(3, 5)
    else:
        ps = I.draw_instances(2, seed=3, d=5)
    for p in ps:
        for dt in (0.0025, 0.005, 0.015, 1.0):
            rad = _step_radius(orc, p, levels, dt)
            assert rad <= 1.0 + 1e-12, (levels, dt, rad)
