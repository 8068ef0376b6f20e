"""The oracle's two paths pinned to each other and to exact derivatives (CPU).

The oracle evaluates the branch subproblem of eq. (branch) (Sec. II-C) and
the trust-region method of Sec. III-B in two ways:

* the fixed-sequence path, whose IEEE operation sequence the GPU reproduces:
  f/g/H by a grouped chain rule, fused multiply-adds, series sin/cos, the
  square-root-free L E L' factorization of H_FF + alpha diag(|H_ii|),
  squared-norm tests, the model from the lower triangle of H;
* the textbook path: eq. (branch) summed term by term with the gradient and
  Hessian of every coupling value written out, libm sin/cos, plain
  arithmetic, Lin & More's Cholesky factor of D H_FF D + alpha I with
  D = diag(|H_ii|^(-1/2)), norms with square roots, the full model.

Pins here:
* the textbook f, g, H against exact derivatives of an independent
  complex-phasor form of eq. (branch) (S = V conj(Y V)), taken by hyper-dual
  numbers (first and second derivatives without truncation error);
* the fixed-sequence f, g, H against the textbook ones to 1e-13;
* the textbook Cholesky factor and preconditioner against numpy;
* single branch solves, 50 whole ADMM iterations (30-bus, 2k-bus, and a
  2k-bus grid with tightened ratings where line limits bind) and a converged
  2k-bus solve: the two paths agree to rounding-level differences.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2110_06879_amd.gridgen import config_grid, gridgen

from test_oracle_branch import phasor_objective, pi_model, random_branch, random_grid_with_taps


class HD:
    """Hyper-dual number a + b e1 + c e2 + d e1 e2 with e1^2 = e2^2 = 0: f(x +
    e1 u + e2 w) carries f, the directional derivatives along u and w, and
    u' H w, with no truncation error."""
    __slots__ = ("a", "b", "c", "d")

    def __init__(self, a, b=0.0, c=0.0, d=0.0):
        self.a, self.b, self.c, self.d = float(a), float(b), float(c), float(d)

    @staticmethod
    def lift(v):
        return v if isinstance(v, HD) else HD(v)

    def __add__(self, o):
        o = HD.lift(o)
        return HD(self.a + o.a, self.b + o.b, self.c + o.c, self.d + o.d)

    __radd__ = __add__

    def __neg__(self):
        return HD(-self.a, -self.b, -self.c, -self.d)

    def __sub__(self, o):
        return self + (-HD.lift(o))

    def __rsub__(self, o):
        return HD.lift(o) - self

    def __mul__(self, o):
        o = HD.lift(o)
        return HD(self.a * o.a, self.a * o.b + self.b * o.a, self.a * o.c + self.c * o.a,
                  self.a * o.d + self.b * o.c + self.c * o.b + self.d * o.a)

    __rmul__ = __mul__


def hsin(x):
    s, c = math.sin(x.a), math.cos(x.a)
    return HD(s, c * x.b, c * x.c, c * x.d - s * x.b * x.c)


def hcos(x):
    s, c = math.sin(x.a), math.cos(x.a)
    return HD(c, -s * x.b, -s * x.c, -s * x.d - c * x.b * x.c)


class Cx:
    """Complex number over hyper-duals (phasor arithmetic)."""

    def __init__(self, re, im):
        self.re, self.im = HD.lift(re), HD.lift(im)

    def __add__(self, o):
        return Cx(self.re + o.re, self.im + o.im)

    def __mul__(self, o):
        return Cx(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    def conj(self):
        return Cx(self.re, -self.im)


def cconst(z):
    return Cx(HD(z.real), HD(z.imag))


def phasor_objective_hd(Y, data, n, ltil, rtil, x):
    """Eq. (branch) through complex power S = V conj(Y V) on hyper-duals."""
    vb, z, y, rho = data[20:28], data[28:36], data[36:44], data[44:52]
    Yff, Yft, Ytf, Ytt = (cconst(c) for c in Y)
    vi, vj, ti, tj = x[:4]
    Vi = Cx(vi * hcos(ti), vi * hsin(ti))
    Vj = Cx(vj * hcos(tj), vj * hsin(tj))
    Sij = Vi * (Yff * Vi + Yft * Vj).conj()
    Sji = Vj * (Ytf * Vi + Ytt * Vj).conj()
    a = [Sij.re, Sij.im, Sji.re, Sji.im, vi * vi, ti, vj * vj, tj]
    F = HD(0.0)
    for k in range(8):
        r = a[k] - vb[k] + z[k]
        F = F + y[k] * r + 0.5 * rho[k] * r * r
    if n == 6:
        for e in range(2):
            c = a[2 * e] * a[2 * e] + a[2 * e + 1] * a[2 * e + 1] + x[4 + e]
            F = F + ltil[e] * c + 0.5 * rtil * c * c
    return F


def exact_fgh(Y, data, n, ltil, rtil, x0):
    g = np.zeros(n)
    H = np.zeros((n, n))
    f = None
    for i in range(n):
        for j in range(i, n):
            xs = [HD(x0[k], 1.0 if k == i else 0.0, 1.0 if k == j else 0.0) for k in range(n)]
            F = phasor_objective_hd(Y, data, n, ltil, rtil, xs)
            f = F.a
            g[i] = F.b
            H[i, j] = H[j, i] = F.d
    return f, g, H


def relerr(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def branch_cases(n, seed, count=6):
    g = random_grid_with_taps(seed)
    o = O.Oracle(g, cold=False)
    ad = o.admittance()
    rng = np.random.default_rng(seed + 10 * n)
    for l in range(count):
        data, lo, hi = random_branch(rng, n, ad[l])
        Y = pi_model(g.r[l], g.x[l], g.b[l], g.tap[l], g.shift[l])
        ltil = rng.normal(0, 5, 2)
        rtil = float(rng.choice([10.0, 37.0, 1e4]))
        x0 = np.concatenate([rng.uniform(0.95, 1.05, 2), rng.uniform(-0.6, 0.6, 2),
                             rng.uniform(-3, -0.1, 2)])[:n]
        yield data, lo, hi, Y, ltil, rtil, x0


def test_hyperdual_arithmetic_on_known_derivatives():
    # f = sin(x) y^2 + x y: df/dx = cos(x) y^2 + y, d2f/dxdy = 2 y cos(x) + 1,
    # d2f/dx2 = -sin(x) y^2
    x0, y0 = 0.7, -1.3
    F = hsin(HD(x0, 1.0, 0.0)) * HD(y0, 0.0, 1.0) * HD(y0, 0.0, 1.0) + HD(x0, 1.0, 0.0) * HD(y0, 0.0, 1.0)
    assert abs(F.b - (math.cos(x0) * y0 ** 2 + y0)) < 1e-15
    assert abs(F.d - (2 * y0 * math.cos(x0) + 1)) < 1e-15
    G = hcos(HD(x0, 1.0, 1.0))
    assert abs(G.d - (-math.cos(x0))) < 1e-15
    G = hsin(HD(x0, 1.0, 1.0)) * y0 * y0
    assert abs(G.d - (-math.sin(x0) * y0 ** 2)) < 1e-15


@pytest.mark.parametrize("n", [4, 6])
def test_textbook_fgh_matches_exact_phasor_derivatives(n):
    for data, lo, hi, Y, ltil, rtil, x0 in branch_cases(n, 3):
        f, g, H, _ = O.branch_eval(data, n, ltil, rtil, x0, textbook=True)
        fe, ge, He = exact_fgh(Y, data, n, ltil, rtil, x0)
        assert abs(f - fe) <= 1e-12 * (1 + abs(fe))
        assert abs(f - phasor_objective(Y, data, n, ltil, rtil, x0)) <= 1e-12 * (1 + abs(fe))
        assert relerr(g, ge) < 1e-12
        assert relerr(H, He) < 1e-12
        assert relerr(H, H.T) < 1e-15


@pytest.mark.parametrize("n", [4, 6])
def test_fixed_sequence_fgh_matches_textbook(n):
    """The grouped chain rule (mu/nu merges, MR/MI sums), the fused
    multiply-adds and the series sin/cos give the textbook f, g, H."""
    for seed in (3, 5, 7):
        for data, lo, hi, Y, ltil, rtil, x0 in branch_cases(n, seed):
            f, g, H, a = O.branch_eval(data, n, ltil, rtil, x0)
            ft, gt, Ht, at = O.branch_eval(data, n, ltil, rtil, x0, textbook=True)
            assert abs(f - ft) <= 1e-13 * max(1.0, abs(ft))
            assert relerr(g, gt) < 1e-13
            assert relerr(H, Ht) < 1e-13
            assert relerr(a, at) < 1e-14


def test_textbook_cholesky_and_preconditioner():
    rng = np.random.default_rng(21)
    for n in range(1, 7):
        Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
        A = (Q * np.exp(rng.uniform(0, np.log(1e4), n))) @ Q.T
        L = O.chol_textbook(A)
        np.testing.assert_allclose(L, np.linalg.cholesky(A), rtol=1e-12, atol=1e-12)
        D = rng.uniform(0.3, 3.0, n)
        r = rng.normal(size=n)
        z = O.precond_textbook(L, D, r)
        # M = D^-1 L L' D^-1, so z = M^-1 r = D (L L')^-1 D r
        M = np.diag(1 / D) @ A @ np.diag(1 / D)
        np.testing.assert_allclose(z, np.linalg.solve(M, r), rtol=1e-10)
        if n > 1:
            B = A.copy()
            B[0, 0] = -1.0
            assert O.chol_textbook(B) is None


@pytest.mark.parametrize("n", [4, 6])
def test_branch_solves_agree_between_paths(n):
    for seed in (4, 6):
        for data, lo, hi, Y, ltil, rtil, x0 in branch_cases(n, seed, count=5):
            xs = np.concatenate([x0, np.zeros(6 - n)])
            r1 = O.branch_solve(data, n, xs, ltil, 10.0)
            r2 = O.branch_solve(data, n, xs, ltil, 10.0, textbook=True)
            # same rules, so the same event counts; x to rounding level
            for k in ("tron_iters", "al_iters", "cg_iters", "n_fgh"):
                assert r1[4][k] == r2[4][k], k
            assert relerr(r1[0], r2[0]) < 1e-10
            assert relerr(r1[3], r2[3]) < 1e-10


def tightened_2k():
    """The 2k-bus grid with every rating scaled by 0.15, so that line limits
    bind (about 90 branches after 50 iterations) and the AL loop of eq.
    (branch) runs several rounds."""
    g = config_grid("c2_2kbus")
    g.rate = g.rate * 0.15
    return g


PARITY_FLOOR = {"ltil": 1.0}


@pytest.mark.parametrize("case", ["c1_30bus", "c2_2kbus", "c2_tight"])
def test_fifty_iterations_agree_between_paths(case):
    """After 50 inner iterations of Algorithm 1 from the cold start, every
    state vector of the fixed-sequence path equals the textbook path's to
    1e-8 (norm-wise; measured: below 1e-10). ltil is compared above a floor
    of 1: on grids where no limit binds every ltil is the solvers' stopping
    noise (1e-16 to 1e-12), which the two paths resolve differently."""
    if case == "c1_30bus":
        g, p = config_grid("c1_30bus"), O.OracleParams(rho_pq=400.0, rho_va=400.0)
    elif case == "c2_2kbus":
        g, p = config_grid("c2_2kbus"), O.OracleParams()
    else:
        g, p = tightened_2k(), O.OracleParams()
    a = O.Oracle(g, p)
    b = O.Oracle(g, p)
    b.set_textbook(True)
    a.solve(50)
    b.solve(50)
    for k in ("u", "v", "z", "y", "lam", "bx", "ltil", "rtil", "calpha"):
        x, y = a.get(k), b.get(k)
        den = max(np.abs(y).max(), PARITY_FLOOR.get(k, 1e-30))
        assert np.abs(x - y).max() / den <= 1e-8, k
    if case == "c2_tight":
        lt, rt = a.get("ltil"), a.get("rtil")
        assert (np.abs(lt) > 1e-3).sum() >= 50
        assert (rt > p.al_rho0).sum() >= 100
        sa, sb = a.stats(), b.stats()
        assert sa["al_iters"] == sb["al_iters"] > 2600 * 50


@pytest.mark.slow
@pytest.mark.parametrize("name", ["c3_70kbus", "c3_70kbus_full"])
def test_70k_thirty_iterations_agree_between_paths(name):
    """The 70k-bus benchmark grid after 30 inner iterations from the cold
    start: every state vector of the fixed-sequence path equals the textbook
    path's to 1e-8 (norm-wise), both run over the host's threads. At the
    stated load distribution (`_full`) about 170 line limits bind and the two
    paths take the same AL rounds; a handful of TRON decisions at rounding
    level differ (8 of 6.8 million iterations), and the vectors still agree
    to 4e-9."""
    import os
    g, p = config_grid(name), O.OracleParams()
    a = O.Oracle(g, p)
    b = O.Oracle(g, p)
    b.set_textbook(True)
    for o in (a, b):
        o.set_threads(max(1, min(8, os.cpu_count() or 1)))
        o.solve(30)
    for k in ("u", "v", "z", "y", "lam", "bx", "ltil", "rtil", "calpha"):
        x, y = a.get(k), b.get(k)
        den = max(np.abs(y).max(), PARITY_FLOOR.get(k, 1e-30))
        assert np.abs(x - y).max() / den <= 1e-8, k
    assert a.stats()["al_iters"] == b.stats()["al_iters"]
    if name.endswith("_full"):
        assert (np.abs(a.get("ltil")) > 1e-3).sum() >= 100


@pytest.mark.slow
def test_converged_2k_solve_agrees_between_paths():
    """Cold solve of the 2k-bus grid to the 1e-4 tests: the same iteration
    count (within 2%) and the same objective (1e-6 relative) on both paths."""
    g, p = config_grid("c2_2kbus"), O.OracleParams()
    a = O.Oracle(g, p)
    b = O.Oracle(g, p)
    b.set_textbook(True)
    na, nb = a.solve(0), b.solve(0)
    assert a.scalars()["status"] == 0 and b.scalars()["status"] == 0
    assert abs(na - nb) <= 0.02 * na
    assert abs(a.objective() - b.objective()) <= 1e-6 * abs(b.objective())
