"""Pins of the oracle's branch model and branch solver (CPU only).

What pins what:
* flows and admittances: the textbook pi-model complex power
  S_ij = V_i conj(Y_ff V_i + Y_ft V_j) in numpy complex arithmetic (eq. acopf
  and the admittance definitions below it), plus the lossless closed form;
* gradient and Hessian of the branch objective (eq. branch): central
  finite differences with Richardson extrapolation of the oracle's own f;
* the branch objective value: an independent complex-phasor evaluation;
* TRON's minimizer: brute-force search on a fine grid around it, and the
  projected-gradient first-order condition;
* the augmented-Lagrangian loop (6-variable branches): KKT of the line-limited
  problem with a non-negative multiplier, and a brute-force search over the
  feasible voltage points.
"""
import numpy as np
import pytest

import oracle as O
from paper_2110_06879_amd.gridgen import gridgen

TWO_PI = 2 * np.pi


def pi_model(r, x, b, tap, shift):
    ys = 1.0 / (r + 1j * x)
    a = tap * np.exp(1j * shift)
    Yff = (ys + 1j * b / 2) / abs(a) ** 2
    Yft = -ys / np.conj(a)
    Ytf = -ys / a
    Ytt = ys + 1j * b / 2
    return Yff, Yft, Ytf, Ytt


def phasor_flows(Y, vi, vj, ti, tj):
    Yff, Yft, Ytf, Ytt = Y
    Vi = vi * np.exp(1j * ti)
    Vj = vj * np.exp(1j * tj)
    Sij = Vi * np.conj(Yff * Vi + Yft * Vj)
    Sji = Vj * np.conj(Ytf * Vi + Ytt * Vj)
    return Sij, Sji


def random_grid_with_taps(seed=11):
    g = gridgen(12, 3, 20, 1.0, seed)
    rng = np.random.default_rng(seed)
    g.tap = rng.uniform(0.9, 1.1, g.n_branch)
    g.shift = rng.uniform(-0.2, 0.2, g.n_branch)
    return g


def adm8(ad_row):
    return ad_row[:8]


def test_admittance_and_flows_match_complex_power():
    g = random_grid_with_taps()
    o = O.Oracle(g, cold=False)
    ad = o.admittance()
    rng = np.random.default_rng(0)
    for l in range(g.n_branch):
        Y = pi_model(g.r[l], g.x[l], g.b[l], g.tap[l], g.shift[l])
        data = O.pack_branch(adm8(ad[l]), np.full(6, -10.0), np.full(6, 10.0),
                             np.zeros(8), np.zeros(8), np.zeros(8), np.ones(8))
        for _ in range(5):
            vi, vj = rng.uniform(0.9, 1.1, 2)
            ti, tj = rng.uniform(-1, 1, 2)
            _, _, _, a = O.branch_eval(data, 4, [0, 0], 0.0, [vi, vj, ti, tj])
            Sij, Sji = phasor_flows(Y, vi, vj, ti, tj)
            np.testing.assert_allclose(a[:4], [Sij.real, Sij.imag, Sji.real, Sji.imag],
                                       rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(a[4:], [vi * vi, ti, vj * vj, tj], rtol=0, atol=0)


def test_lossless_line_closed_form():
    # r = 0, b = 0, tap 1: p_ij = -p_ji = vi vj sin(ti - tj)/x,
    # q_ij = (vi^2 - vi vj cos)/x, q_ji = (vj^2 - vi vj cos)/x
    g = gridgen(4, 1, 3, 1.0, 5)
    g.r[:] = 0.0
    g.b[:] = 0.0
    o = O.Oracle(g, cold=False)
    ad = o.admittance()
    rng = np.random.default_rng(1)
    for l in range(g.n_branch):
        x = g.x[l]
        data = O.pack_branch(adm8(ad[l]), np.full(6, -10.0), np.full(6, 10.0),
                             np.zeros(8), np.zeros(8), np.zeros(8), np.ones(8))
        vi, vj = rng.uniform(0.9, 1.1, 2)
        ti, tj = rng.uniform(-0.5, 0.5, 2)
        _, _, _, a = O.branch_eval(data, 4, [0, 0], 0.0, [vi, vj, ti, tj])
        d = ti - tj
        exp = [vi * vj * np.sin(d) / x, (vi ** 2 - vi * vj * np.cos(d)) / x,
               -vi * vj * np.sin(d) / x, (vj ** 2 - vi * vj * np.cos(d)) / x]
        np.testing.assert_allclose(a[:4], exp, rtol=1e-12, atol=1e-13)
        # reactive losses are non-negative: |Vi - Vj|^2 / x
        Vi, Vj = vi * np.exp(1j * ti), vj * np.exp(1j * tj)
        assert abs(a[1] + a[3] - abs(Vi - Vj) ** 2 / x) < 1e-12


def random_branch(rng, n, ad_row, scale_y=50.0):
    lo = np.array([0.94, 0.94, -TWO_PI, -TWO_PI, -4.0, -4.0])
    hi = np.array([1.06, 1.06, TWO_PI, TWO_PI, 0.0, 0.0])
    vb = np.concatenate([rng.normal(0, 0.5, 4), rng.uniform(0.9, 1.1, 1),
                         rng.normal(0, 0.1, 1), rng.uniform(0.9, 1.1, 1),
                         rng.normal(0, 0.1, 1)])
    z = rng.normal(0, 0.01, 8)
    y = rng.normal(0, scale_y, 8)
    rho = np.array([400.0] * 4 + [4000.0] * 4)
    return O.pack_branch(adm8(ad_row), lo, hi, vb, z, y, rho), lo, hi


def phasor_objective(Y, data, n, ltil, rtil, x):
    """Eq. (branch) evaluated with complex power, independent of the oracle."""
    vb, z, y, rho = data[20:28], data[28:36], data[36:44], data[44:52]
    vi, vj, ti, tj = x[:4]
    Sij, Sji = phasor_flows(Y, vi, vj, ti, tj)
    a = np.array([Sij.real, Sij.imag, Sji.real, Sji.imag, vi * vi, ti, vj * vj, tj])
    r = a - vb + z
    F = np.sum(y * r + 0.5 * rho * r * r)
    if n == 6:
        for e in range(2):
            c = a[2 * e] ** 2 + a[2 * e + 1] ** 2 + x[4 + e]
            F += ltil[e] * c + 0.5 * rtil * c * c
    return F


@pytest.mark.parametrize("n", [4, 6])
def test_branch_objective_value_and_derivatives(n):
    g = random_grid_with_taps(3)
    o = O.Oracle(g, cold=False)
    ad = o.admittance()
    rng = np.random.default_rng(2 + n)
    for l in range(6):
        data, lo, hi = random_branch(rng, n, ad[l])
        Y = pi_model(g.r[l], g.x[l], g.b[l], g.tap[l], g.shift[l])
        ltil = rng.normal(0, 5, 2)
        rtil = 37.0
        x0 = np.concatenate([rng.uniform(0.95, 1.05, 2), rng.uniform(-0.3, 0.3, 2),
                             rng.uniform(-3, -0.1, 2)])[:n]
        f, gr, H, _ = O.branch_eval(data, n, ltil, rtil, x0)
        assert abs(f - phasor_objective(Y, data, n, ltil, rtil, x0)) <= 1e-10 * (1 + abs(f))

        def fval(x):
            return O.branch_eval(data, n, ltil, rtil, x)[0]

        def grad(x):
            return O.branch_eval(data, n, ltil, rtil, x)[1]

        # Richardson-extrapolated central differences
        def rich(fun, x, i, h):
            e = np.zeros(n)
            e[i] = 1.0
            d1 = (fun(x + h * e) - fun(x - h * e)) / (2 * h)
            d2 = (fun(x + h / 2 * e) - fun(x - h / 2 * e)) / h
            return (4 * d2 - d1) / 3

        g_fd = np.array([rich(fval, x0, i, 1e-3) for i in range(n)])
        np.testing.assert_allclose(gr, g_fd, rtol=1e-7, atol=1e-6 * (1 + np.abs(gr).max()))
        H_fd = np.array([rich(grad, x0, i, 1e-4) for i in range(n)]).T
        np.testing.assert_allclose(H, H.T, rtol=0, atol=1e-9 * (1 + np.abs(H).max()))
        np.testing.assert_allclose(H, H_fd, rtol=1e-6, atol=1e-6 * (1 + np.abs(H).max()))


def proj_grad(x, g, lo, hi):
    return np.clip(x - g, lo, hi) - x


def test_branch_solve_4var_is_a_local_minimum_bruteforce():
    g = random_grid_with_taps(4)
    o = O.Oracle(g, cold=False)
    ad = o.admittance()
    rng = np.random.default_rng(7)
    for l in range(4):
        Y = pi_model(g.r[l], g.x[l], g.b[l], g.tap[l], g.shift[l])
        data, lo, hi = random_branch(rng, 4, ad[l])
        x0 = np.array([1.0, 1.0, 0.0, 0.0, 0.0, 0.0])
        x, lt, rt, u, st = O.branch_solve(data, 4, x0, [0, 0], 10.0)
        f, gr, H, a = O.branch_eval(data, 4, [0, 0], 0.0, x[:4])
        # first-order condition
        assert np.abs(proj_grad(x[:4], gr, lo[:4], hi[:4])).max() < 1e-6
        np.testing.assert_allclose(u, a, rtol=0, atol=0)
        # brute force: no point of a 21^4 grid in a small box beats f
        deltas = np.linspace(-2e-3, 2e-3, 21)
        V1, V2, T1, T2 = np.meshgrid(deltas, deltas, deltas, deltas, indexing="ij")
        X = np.stack([x[0] + V1, x[1] + V2, x[2] + T1, x[3] + T2], -1).reshape(-1, 4)
        X = np.clip(X, lo[:4], hi[:4])
        Fs = np.array([phasor_objective(Y, data, 4, [0, 0], 0, xx) for xx in X[::7]])
        assert Fs.min() >= f - 1e-9 * (1 + abs(f))


def test_branch_solve_6var_al_kkt_and_feasible_bruteforce():
    """A heavily loaded rated branch: the line limit binds."""
    g = random_grid_with_taps(6)
    g.tap[:] = 1.0
    g.shift[:] = 0.0
    o = O.Oracle(g, cold=False)
    ad = o.admittance()
    l = 0
    Y = pi_model(g.r[l], g.x[l], g.b[l], 1.0, 0.0)
    rate2 = 0.5 ** 2
    lo = np.array([0.94, 0.94, -TWO_PI, -TWO_PI, -rate2, -rate2])
    hi = np.array([1.06, 1.06, TWO_PI, TWO_PI, 0.0, 0.0])
    # bus side asks for a large flow (1.5 p.u.) over a 0.5 p.u. line
    Sij, Sji = phasor_flows(Y, 1.0, 1.0, 0.0, -0.15)
    vb = np.array([Sij.real, Sij.imag, Sji.real, Sji.imag, 1.0, 0.0, 1.0, -0.15])
    rho = np.array([400.0] * 4 + [4000.0] * 4)
    data = O.pack_branch(adm8(ad[l]), lo, hi, vb, np.zeros(8), np.zeros(8), rho)
    x0 = np.array([1.0, 1.0, 0.0, 0.0, -rate2, -rate2])
    params = O.OracleParams()
    x, lt, rt, u, st = O.branch_solve(data, 6, x0, [0, 0], 10.0, params)
    c = np.array([u[0] ** 2 + u[1] ** 2 + x[4], u[2] ** 2 + u[3] ** 2 + x[5]])
    assert np.abs(c).max() <= params.al_tol
    # constrained KKT: grad of the ADMM terms + mu * grad(p^2+q^2) = 0 on the
    # voltage variables, mu >= 0 where the limit binds. The stored ltil is
    # the first-order multiplier estimate ltil + rtil c of the last AL round
    # (the update is applied after every round, the last one included).
    mu = lt
    f0, g0, _, a = O.branch_eval(data, 4, [0, 0], 0.0, x[:4])
    assert mu.min() >= -1e-6
    binding = x[4:] <= -rate2 + 1e-12
    assert binding.any()
    _, g6, _, _ = O.branch_eval(data, 6, mu, 0.0, x)
    # with rtil = 0 the gradient of F is grad(ADMM terms) + mu grad(c)
    assert np.abs(proj_grad(x[:4], g6[:4], lo[:4], hi[:4])).max() < 1e-5 * (1 + np.abs(g0).max())
    # brute force over feasible voltage points near the solution
    d = np.linspace(-3e-3, 3e-3, 17)
    V1, V2, T1, T2 = np.meshgrid(d, d, d, d, indexing="ij")
    X = np.stack([x[0] + V1, x[1] + V2, x[2] + T1, x[3] + T2], -1).reshape(-1, 4)
    X = np.clip(X, lo[:4], hi[:4])
    best = np.inf
    for xx in X[::3]:
        S1, S2 = phasor_flows(Y, *xx)
        if abs(S1) ** 2 <= rate2 and abs(S2) ** 2 <= rate2:
            best = min(best, phasor_objective(Y, data, 4, [0, 0], 0, xx))
    assert best >= f0 - 1e-6 * (1 + abs(f0))


def test_counting_mode_is_bitwise_identical():
    g = random_grid_with_taps(8)
    o = O.Oracle(g, cold=False)
    ad = o.admittance()
    rng = np.random.default_rng(9)
    for l in range(5):
        data, lo, hi = random_branch(rng, 6, ad[l])
        x0 = np.array([1.0, 1.0, 0.0, 0.0, -1.0, -1.0])
        r1 = O.branch_solve(data, 6, x0, [0.3, 0.1], 10.0, count=False)
        r2 = O.branch_solve(data, 6, x0, [0.3, 0.1], 10.0, count=True)
        for a, b in zip(r1[:4], r2[:4]):
            assert np.array_equal(np.asarray(a), np.asarray(b))
        assert r2[4]["flops"] > 0 and r2[4]["trig"] > 0
        assert r1[4]["flops"] == 0


def test_series_sincos_accuracy():
    """The oracle's series sin/cos against the C library on [-4 pi, 4 pi]
    (branch angle differences lie in this range: each angle is in
    [-2 pi, 2 pi]), including quadrant boundaries and tiny arguments."""
    import math
    rng = np.random.default_rng(123)
    xs = list(rng.uniform(-4 * np.pi, 4 * np.pi, 20000))
    xs += [k * np.pi / 4 + d for k in range(-16, 17) for d in (-1e-9, 0.0, 1e-9)]
    xs += [0.0, 1e-300, -1e-12, 1e-8, 0.5, -0.5]
    worst = 0.0
    for x in xs:
        s, c = O.sincos(x)
        es, ec = math.sin(x), math.cos(x)
        worst = max(worst, abs(s - es), abs(c - ec))
        assert abs(s - es) <= 4e-16 * max(1.0, abs(x)) and abs(c - ec) <= 4e-16 * max(1.0, abs(x)), x
        assert abs(s * s + c * c - 1.0) < 1e-15
    assert worst < 2e-15


def test_branch_solve_independent_of_cauchy_start():
    """The Cauchy step length a branch solve starts its projected search from
    (carried from the branch's previous solve) changes the path of the
    trust-region method, not its answer: started from 1, from 1e-4 and from
    50, the 4-variable solve reaches the same first-order point; the step
    length it returns is positive and finite."""
    g = random_grid_with_taps(4)
    o = O.Oracle(g, cold=False)
    ad = o.admittance()
    rng = np.random.default_rng(17)
    for l in range(4):
        data, lo, hi = random_branch(rng, 4, ad[l])
        x0 = np.array([1.0, 1.0, 0.0, 0.0, 0.0, 0.0])
        sols = []
        for a0 in (1.0, 1e-4, 50.0):
            x, lt, rt, u, st = O.branch_solve(data, 4, x0, [0, 0], 10.0, alpha=a0)
            assert np.isfinite(st["alpha"]) and st["alpha"] > 0.0
            f, gr, H, a = O.branch_eval(data, 4, [0, 0], 0.0, x[:4])
            assert np.abs(proj_grad(x[:4], gr, lo[:4], hi[:4])).max() < 1e-6
            sols.append(x[:4])
        for x in sols[1:]:
            np.testing.assert_allclose(x, sols[0], rtol=0, atol=1e-6)
