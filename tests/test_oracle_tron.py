"""Pins of the oracle's trust-region Newton method (Lin & More 1999).

* strictly convex box-constrained QPs (n <= 6): the exact minimizer found by
  enumerating all 3^n active sets (each variable at its lower bound, at its
  upper bound, or free) and keeping the one that satisfies the KKT conditions;
* nonconvex quadratics in a box: first-order (projected gradient) and
  second-order (free Hessian positive semidefinite) conditions at the result,
  and a brute-force grid check of local minimality;
* Rosenbrock's function in a box containing (1, 1): the known minimizer;
  and in a box excluding it: the KKT conditions;
* every one of the above on both the fixed-sequence path and the textbook
  path of the oracle;
* its building blocks on their own: the square-root-free Cholesky factors
  L E L' against numpy's Cholesky (L sqrt(E)) and the matrix itself, the
  solve with them against numpy.linalg.solve, a non-positive pivot reported
  for indefinite and singular matrices, and the quadratic model against
  g's + s'Hs/2 evaluated by numpy.
"""
import itertools

import numpy as np
import pytest

import oracle as O


def exact_box_qp(Q, c, lo, hi):
    """min 1/2 x'Qx + c'x on [lo, hi] by active-set enumeration (Q > 0)."""
    n = len(c)
    best = None
    for pattern in itertools.product((0, 1, 2), repeat=n):
        x = np.zeros(n)
        free = [i for i in range(n) if pattern[i] == 2]
        fixed = [i for i in range(n) if pattern[i] != 2]
        for i in fixed:
            x[i] = lo[i] if pattern[i] == 0 else hi[i]
        if free:
            QF = Q[np.ix_(free, free)]
            rhs = -(c[free] + Q[np.ix_(free, fixed)] @ x[fixed])
            x[free] = np.linalg.solve(QF, rhs)
        if np.any(x < lo - 1e-12) or np.any(x > hi + 1e-12):
            continue
        g = Q @ x + c
        ok = True
        for i in fixed:
            if pattern[i] == 0 and g[i] < -1e-9:
                ok = False
            if pattern[i] == 1 and g[i] > 1e-9:
                ok = False
        if ok:
            f = 0.5 * x @ Q @ x + c @ x
            if best is None or f < best[0]:
                best = (f, x)
    return best[1]


def quad_cbs(Q, c):
    def f(x):
        return 0.5 * x @ Q @ x + c @ x

    def fgh(x):
        return f(x), Q @ x + c, Q

    return f, fgh


@pytest.mark.parametrize("textbook", [False, True])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_tron_matches_exact_box_qp(n, textbook):
    rng = np.random.default_rng(100 + n)
    p = O.OracleParams(tron_gtol=1e-12, tron_ftol=1e-16)
    for trial in range(6):
        A = rng.normal(size=(n, n))
        Q = A @ A.T + 0.1 * np.eye(n)
        if trial % 2:
            Q = Q * np.logspace(0, 3, n)[:, None] * np.logspace(0, 3, n)[None, :]
        c = rng.normal(scale=3.0, size=n)
        lo = -rng.uniform(0.1, 1.0, n)
        hi = rng.uniform(0.1, 1.0, n)
        x_star = exact_box_qp(Q, c, lo, hi)
        f, fgh = quad_cbs(Q, c)
        x0 = rng.uniform(lo, hi)
        x, status, st = O.tron_generic(f, fgh, x0, lo, hi, p, textbook=textbook)
        assert status == 0
        scale = 1 + np.abs(x_star).max()
        np.testing.assert_allclose(x, x_star, rtol=0, atol=1e-7 * scale)


@pytest.mark.parametrize("textbook", [False, True])
def test_tron_nonconvex_quadratic_local_min(textbook):
    rng = np.random.default_rng(7)
    n = 5
    p = O.OracleParams(tron_gtol=1e-11, tron_ftol=1e-16)
    for _ in range(10):
        A = rng.normal(size=(n, n))
        Q = 0.5 * (A + A.T)  # indefinite
        c = rng.normal(size=n)
        lo, hi = -np.ones(n), np.ones(n)
        f, fgh = quad_cbs(Q, c)
        x, status, st = O.tron_generic(f, fgh, np.zeros(n), lo, hi, p, textbook=textbook)
        assert status in (0, 2)
        g = Q @ x + c
        pg = np.clip(x - g, lo, hi) - x
        assert np.abs(pg).max() < 1e-8
        free = (x > lo + 1e-9) & (x < hi - 1e-9)
        if free.any():
            ev = np.linalg.eigvalsh(Q[np.ix_(free, free)])
            assert ev.min() > -1e-8
        # local minimality against random feasible perturbations
        for _ in range(200):
            d = rng.normal(scale=1e-3, size=n)
            xt = np.clip(x + d, lo, hi)
            assert f(xt) >= f(x) - 1e-12
        # negative curvature was followed somewhere: the result is not the
        # (saddle) stationary point of the unconstrained problem
        assert f(x) <= f(np.zeros(n)) + 1e-12


def rosen(x):
    return 100 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2


def rosen_fgh(x):
    g = np.array([-400 * x[0] * (x[1] - x[0] ** 2) - 2 * (1 - x[0]),
                  200 * (x[1] - x[0] ** 2)])
    H = np.array([[1200 * x[0] ** 2 - 400 * x[1] + 2, -400 * x[0]],
                  [-400 * x[0], 200.0]])
    return rosen(x), g, H


@pytest.mark.parametrize("textbook", [False, True])
def test_tron_rosenbrock_interior_minimum(textbook):
    p = O.OracleParams(tron_gtol=1e-10, tron_ftol=1e-18, tron_maxit=500)
    x, status, st = O.tron_generic(rosen, rosen_fgh, np.array([-1.2, 1.0]),
                                   np.array([-2.0, -2.0]), np.array([2.0, 2.0]), p,
                                   textbook=textbook)
    assert status == 0
    np.testing.assert_allclose(x, [1.0, 1.0], atol=1e-8)


@pytest.mark.parametrize("textbook", [False, True])
def test_tron_rosenbrock_bound_active(textbook):
    # box excludes (1,1): x0 <= 0.5. KKT: at x0 = 0.5 the minimizer over x1
    # is x1 = 0.25 and df/dx0 there must be <= 0.
    p = O.OracleParams(tron_gtol=1e-10, tron_ftol=1e-18, tron_maxit=500)
    lo, hi = np.array([-2.0, -2.0]), np.array([0.5, 2.0])
    x, status, st = O.tron_generic(rosen, rosen_fgh, np.array([-1.2, 1.0]), lo, hi, p,
                                   textbook=textbook)
    np.testing.assert_allclose(x, [0.5, 0.25], atol=1e-8)
    g = rosen_fgh(x)[1]
    assert g[0] <= 0.0


@pytest.mark.parametrize("textbook", [False, True])
def test_tron_starting_at_solution_takes_no_step(textbook):
    Q = np.diag([2.0, 3.0])
    c = np.array([-2.0, -3.0])
    f, fgh = quad_cbs(Q, c)
    x, status, st = O.tron_generic(f, fgh, np.array([1.0, 1.0]),
                                   np.array([-5.0, -5.0]), np.array([5.0, 5.0]),
                                   textbook=textbook)
    assert status == 0 and st["tron_iters"] == 0
    np.testing.assert_array_equal(x, [1.0, 1.0])


def spd(rng, n, cond=1e3):
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.exp(rng.uniform(0.0, np.log(cond), n))
    return (Q * ev) @ Q.T


def test_ldlt_factors_match_cholesky_and_solve():
    rng = np.random.default_rng(31)
    for n in range(1, 7):
        for _ in range(20):
            A = spd(rng, n)
            A = 0.5 * (A + A.T)
            out = O.ldlt(A)
            assert out is not None
            L, rd = out
            e = 1.0 / rd
            assert np.all(e > 0.0)
            np.testing.assert_array_equal(np.diag(L), np.ones(n))
            assert np.all(np.triu(L, 1) == 0.0)
            np.testing.assert_allclose(L @ np.diag(e) @ L.T, A, rtol=1e-12,
                                       atol=1e-12 * np.abs(A).max())
            C = np.linalg.cholesky(A)
            np.testing.assert_allclose(L * np.sqrt(e), C, rtol=1e-10, atol=1e-12 * np.abs(C).max())
            r = rng.normal(size=n)
            z = O.ldlt_solve(L, rd, r)
            np.testing.assert_allclose(z, np.linalg.solve(A, r), rtol=1e-9,
                                       atol=1e-12 * np.abs(z).max())


def test_ldlt_reports_non_positive_pivots():
    rng = np.random.default_rng(32)
    for n in range(2, 7):
        Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
        ev = rng.uniform(0.5, 2.0, n)
        ev[rng.integers(n)] = -0.3          # one negative eigenvalue
        A = (Q * ev) @ Q.T
        assert O.ldlt(0.5 * (A + A.T)) is None
        B = np.zeros((n, n))
        B[0, 0] = 1.0                       # singular: zero pivot at column 1
        assert O.ldlt(B) is None


def test_model_matches_quadratic_form():
    rng = np.random.default_rng(33)
    for n in range(1, 7):
        for _ in range(20):
            H = rng.normal(size=(n, n))
            H = H + H.T
            g = rng.normal(size=n)
            s = rng.normal(size=n)
            want = g @ s + 0.5 * s @ H @ s
            got = O.model(g, H, s)
            assert abs(got - want) <= 1e-13 * (abs(g) @ abs(s) + abs(s) @ abs(H) @ abs(s))
