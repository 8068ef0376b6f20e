"""Pins of the oracle's closed-form ADMM steps and of the whole iteration.

* generator step (eq. qp-bound): a bounded scalar minimizer (scipy) of the
  generator's augmented Lagrangian;
* bus step (eq. qp-bus): the full KKT system [Q A'; A 0] solved by
  numpy.linalg.solve, and the power balance rows (eqs. pg, qg) holding after
  the step;
* z and y (two-level scheme, multiplier updates): stationarity of the z
  subproblem and the y recursion;
* outer step: projection of lambda and the beta rule;
* invariants of Algorithm 1: cold start has u = v and z = 0, bounds hold at
  every iterate;
* whole ADMM on a 3-bus grid: converges to the solution of the dense NLP
  (scipy SLSQP on polar power flow), also when warm-started after new loads;
* the Cauchy step length carried between a branch's trust-region solves:
  the same iterations and objective as restarting it at 1 (the method's own
  start) before every ADMM iteration, with about half the Cauchy trials.
"""
import dataclasses
import json
import os

import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

import oracle as O
from paper_2110_06879_amd.gridgen import Grid, config_grid, gridgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def randomize_state(o, rng, scale=1.0):
    m = o.m
    o.set("v", o.get("v") + rng.normal(0, 0.05 * scale, m))
    o.set("z", rng.normal(0, 0.02 * scale, m))
    o.set("y", rng.normal(0, 20 * scale, m))
    o.set("lam", rng.normal(0, 5 * scale, m))
    o.set("u", o.get("u") + rng.normal(0, 0.05 * scale, m))


def test_generator_step_matches_scalar_minimizer():
    g = config_grid("c1_30bus")
    for s in (1.0, 0.3):
        o = O.Oracle(g, O.OracleParams(obj_scale=s))
        randomize_state(o, np.random.default_rng(3), scale=10)
        v, z, y, rho = o.get("v"), o.get("z"), o.get("y"), o.get("rho")
        o.gen_step()
        u = o.get("u")
        B = g.base_mva
        for k in range(g.n_gen):
            kp, kq = 2 * k, 2 * k + 1

            def fp(p):
                P = B * p
                r = p - v[kp] + z[kp]
                return s * (g.c2[k] * P * P + g.c1[k] * P + g.c0[k]) + y[kp] * r + 0.5 * rho[kp] * r * r

            def fq(q):
                r = q - v[kq] + z[kq]
                return y[kq] * r + 0.5 * rho[kq] * r * r

            rp = minimize_scalar(fp, bounds=(g.pmin[k], g.pmax[k]), method="bounded",
                                 options=dict(xatol=1e-12))
            rq = minimize_scalar(fq, bounds=(g.qmin[k], g.qmax[k]), method="bounded",
                                 options=dict(xatol=1e-12))
            assert abs(u[kp] - rp.x) < 1e-7
            assert abs(u[kq] - rq.x) < 1e-7
            # exact at a bound when the bound is active
            assert g.pmin[k] <= u[kp] <= g.pmax[k]


def bus_kkt_reference(g, o, i):
    """Build eq. (qp-bus) for bus i from the raw arrays and solve the KKT."""
    ng = g.n_gen
    u, z, y, rho = o.get("u"), o.get("z"), o.get("y"), o.get("rho")
    vars_, aP, aQ = [], [], []
    for k in range(ng):
        if g.gen_bus[k] == i:
            vars_ += [2 * k, 2 * k + 1]
            aP += [1, 0]
            aQ += [0, 1]
    for l in range(g.n_branch):
        b0 = 2 * ng + 8 * l
        if g.br_from[l] == i:
            vars_ += [b0, b0 + 1]
            aP += [-1, 0]
            aQ += [0, -1]
        if g.br_to[l] == i:
            vars_ += [b0 + 2, b0 + 3]
            aP += [-1, 0]
            aQ += [0, -1]
    wk = [2 * ng + 8 * l + 4 for l in range(g.n_branch) if g.br_from[l] == i] + \
         [2 * ng + 8 * l + 6 for l in range(g.n_branch) if g.br_to[l] == i]
    K = len(vars_)
    n = K + 1
    Q = np.zeros((n, n))
    c = np.zeros(n)
    for t, k in enumerate(vars_):
        Q[t, t] = rho[k]
        c[t] = rho[k] * (u[k] + z[k]) + y[k]
    for k in wk:
        Q[K, K] += rho[k]
        c[K] += rho[k] * (u[k] + z[k]) + y[k]
    A = np.zeros((2, n))
    A[0, :K] = aP
    A[1, :K] = aQ
    A[0, K] = -g.gs[i]
    A[1, K] = g.bs[i]
    b = np.array([g.pd[i], g.qd[i]])
    KKT = np.block([[Q, A.T], [A, np.zeros((2, 2))]])
    sol = np.linalg.solve(KKT, np.concatenate([c, b]))
    return vars_, wk, sol[:n], A, b


def test_bus_step_matches_kkt_solve_and_balances():
    g = gridgen(40, 8, 55, 1.0, 21)
    rng = np.random.default_rng(5)
    g.gs = rng.uniform(0, 0.05, g.n_bus)
    g.bs = rng.uniform(-0.05, 0.05, g.n_bus)
    o = O.Oracle(g)
    randomize_state(o, rng)
    o.bus_step()
    v = o.get("v")
    for i in range(g.n_bus):
        vars_, wk, x, A, b = bus_kkt_reference(g, o, i)
        np.testing.assert_allclose(v[vars_], x[:-1], rtol=1e-10, atol=1e-11)
        for k in wk:
            assert abs(v[k] - x[-1]) < 1e-11
        # Ax = b with the step's own output
        xx = np.concatenate([v[vars_], [v[wk[0]]]])
        np.testing.assert_allclose(A @ xx, b, atol=1e-12)


def test_bus_angle_average_and_reference():
    g = config_grid("c1_30bus")
    o = O.Oracle(g)
    rng = np.random.default_rng(8)
    randomize_state(o, rng)
    o.bus_step()
    u, z, y, rho, v = (o.get(k) for k in ("u", "z", "y", "rho", "v"))
    ng = g.n_gen
    for i in range(g.n_bus):
        ks = [2 * ng + 8 * l + 5 for l in range(g.n_branch) if g.br_from[l] == i] + \
             [2 * ng + 8 * l + 7 for l in range(g.n_branch) if g.br_to[l] == i]
        # argmin of sum_k y_k (u_k - t + z_k) + rho_k/2 (u_k - t + z_k)^2
        res = minimize_scalar(lambda t: sum(y[k] * (u[k] - t + z[k]) + 0.5 * rho[k] * (u[k] - t + z[k]) ** 2 for k in ks))
        want = 0.0 if i == g.ref_bus else res.x
        for k in ks:
            assert abs(v[k] - want) < 1e-7


def test_z_and_y_steps_stationarity():
    g = config_grid("c1_30bus")
    o = O.Oracle(g)
    rng = np.random.default_rng(4)
    randomize_state(o, rng)
    beta = o.scalars()["beta"]
    y0 = o.get("y")
    o.z_step()
    u, v, z, lam, rho = (o.get(k) for k in ("u", "v", "z", "lam", "rho"))
    stat = lam + beta * z + y0 + rho * (u - v + z)
    assert np.abs(stat).max() < 1e-12 * (1 + np.abs(y0).max())
    o.y_step()
    np.testing.assert_allclose(o.get("y"), y0 + rho * (u - v + z), rtol=1e-15, atol=1e-13)


def test_outer_step_projection_and_beta_rule():
    g = config_grid("c1_30bus")
    p = O.OracleParams(lambda_max=3.0, beta0=10.0, beta_gamma=6.0, beta_omega=0.8)
    o = O.Oracle(g, p)
    rng = np.random.default_rng(1)
    z = rng.normal(0, 0.5, o.m)
    lam = rng.normal(0, 2.0, o.m)
    o.set("z", z)
    o.set("lam", lam)
    o.residuals()
    o.outer_step()
    np.testing.assert_allclose(o.get("lam"), np.clip(lam + 10.0 * z, -3, 3), rtol=0, atol=1e-15)
    s = o.scalars()
    assert s["beta"] == 10.0  # first outer step: no previous ||z||
    # ||z|| not reduced by omega: beta grows by gamma
    o.set("z", z * 0.9)
    o.residuals()
    o.outer_step()
    assert o.scalars()["beta"] == 60.0
    # ||z|| reduced enough: beta kept
    o.set("z", z * 0.1)
    o.residuals()
    o.outer_step()
    assert o.scalars()["beta"] == 60.0


def test_cold_start_and_bounds_invariants():
    g = config_grid("c1_30bus")
    o = O.Oracle(g)
    u, v, z = o.get("u"), o.get("v"), o.get("z")
    assert np.array_equal(u, v) and not z.any()
    ng = g.n_gen
    # bus-side angle copies start at zero, w copies equal v^2 of the midpoint
    a = u[2 * ng:].reshape(-1, 8)
    assert not a[:, 5].any() and not a[:, 7].any()
    np.testing.assert_allclose(a[:, 4], 1.0, atol=1e-15)
    rate2 = (0.99 * g.rate) ** 2
    for _ in range(30):
        o.iterate(fixed=True)
        u, bx = o.get("u"), o.get("bx").reshape(-1, 6)
        assert np.all(u[0:2 * ng:2] >= g.pmin) and np.all(u[0:2 * ng:2] <= g.pmax)
        assert np.all(u[1:2 * ng:2] >= g.qmin) and np.all(u[1:2 * ng:2] <= g.qmax)
        assert np.all(bx[:, 0] >= g.vmin[g.br_from]) and np.all(bx[:, 0] <= g.vmax[g.br_from])
        assert np.all(bx[:, 1] >= g.vmin[g.br_to]) and np.all(bx[:, 1] <= g.vmax[g.br_to])
        assert np.all(np.abs(bx[:, 2:4]) <= 2 * np.pi)
        assert np.all(bx[:, 4] >= -rate2) and np.all(bx[:, 4] <= 0)
        # bus balance holds exactly after every bus step
        v = o.get("v")
        for i in range(g.n_bus):
            P = sum(v[2 * k] for k in range(ng) if g.gen_bus[k] == i)
            P -= sum(v[2 * ng + 8 * l] for l in range(g.n_branch) if g.br_from[l] == i)
            P -= sum(v[2 * ng + 8 * l + 2] for l in range(g.n_branch) if g.br_to[l] == i)
            assert abs(P - g.pd[i]) < 1e-12


def load_three_bus():
    with open(os.path.join(GOLDEN, "three_bus.json")) as f:
        d = json.load(f)
    nb, ng, nl = len(d["pd"]), len(d["gen_bus"]), len(d["br_from"])
    A = lambda k, t=np.float64: np.asarray(d[k], dtype=t)  # noqa: E731
    return Grid(name="three_bus", base_mva=d["base_mva"], ref_bus=d["ref_bus"],
                pd=A("pd"), qd=A("qd"), gs=np.zeros(nb), bs=np.zeros(nb),
                vmin=A("vmin"), vmax=A("vmax"), gen_bus=A("gen_bus", np.int32),
                pmin=A("pmin"), pmax=A("pmax"), qmin=A("qmin"), qmax=A("qmax"),
                c2=A("c2"), c1=A("c1"), c0=A("c0"),
                br_from=A("br_from", np.int32), br_to=A("br_to", np.int32),
                r=A("r"), x=A("x"), b=A("b"), tap=np.ones(nl), shift=np.zeros(nl),
                rate=A("rate"))


def dense_acopf(g, rate_scale=0.99):
    """ACOPF (eq. acopf) in polar form, solved by scipy SLSQP."""
    nb, ng = g.n_bus, g.n_gen
    Y = np.zeros((nb, nb), dtype=complex)
    Ysh = []
    for l in range(g.n_branch):
        i, j = g.br_from[l], g.br_to[l]
        ys = 1 / (g.r[l] + 1j * g.x[l])
        yff, yft, ytf, ytt = ys + 0.5j * g.b[l], -ys, -ys, ys + 0.5j * g.b[l]
        Y[i, i] += yff; Y[i, j] += yft; Y[j, i] += ytf; Y[j, j] += ytt
        Ysh.append((i, j, yff, yft, ytf, ytt))
    B = g.base_mva

    def unpack(z):
        return z[:ng], z[ng:2 * ng], z[2 * ng:2 * ng + nb], z[2 * ng + nb:]

    def obj(z):
        p = unpack(z)[0] * B
        return float(np.sum(g.c2 * p * p + g.c1 * p + g.c0))

    def balance(z):
        p, q, vm, va = unpack(z)
        V = vm * np.exp(1j * va)
        S = V * np.conj(Y @ V)
        Sg = np.zeros(nb, dtype=complex)
        for k in range(ng):
            Sg[g.gen_bus[k]] += p[k] + 1j * q[k]
        mis = Sg - (g.pd + 1j * g.qd) - S
        return np.concatenate([mis.real, mis.imag, [va[g.ref_bus]]])

    def limits(z):
        _, _, vm, va = unpack(z)
        V = vm * np.exp(1j * va)
        out = []
        for l, (i, j, yff, yft, ytf, ytt) in enumerate(Ysh):
            r2 = (rate_scale * g.rate[l]) ** 2
            Sij = V[i] * np.conj(yff * V[i] + yft * V[j])
            Sji = V[j] * np.conj(ytf * V[i] + ytt * V[j])
            out += [r2 - abs(Sij) ** 2, r2 - abs(Sji) ** 2]
        return np.array(out)

    z0 = np.concatenate([(g.pmin + g.pmax) / 2, (g.qmin + g.qmax) / 2,
                         (g.vmin + g.vmax) / 2, np.zeros(nb)])
    bounds = list(zip(g.pmin, g.pmax)) + list(zip(g.qmin, g.qmax)) + \
        list(zip(g.vmin, g.vmax)) + [(-2 * np.pi, 2 * np.pi)] * nb
    res = minimize(obj, z0, method="SLSQP", bounds=bounds,
                   constraints=[{"type": "eq", "fun": balance},
                                {"type": "ineq", "fun": limits}],
                   options=dict(ftol=1e-14, maxiter=500))
    assert res.success, res.message
    return unpack(res.x)


@pytest.mark.slow
def test_three_bus_admm_converges_to_dense_acopf():
    g = load_three_bus()
    p_ref, q_ref, vm_ref, va_ref = dense_acopf(g)
    p = O.OracleParams(rho_pq=400.0, rho_va=4000.0, obj_scale=0.01,
                       eps_pri=1e-7, eps_dual=1e-7, eps_z=1e-7,
                       max_inner=20000, max_outer=40)
    o = O.Oracle(g, p)
    o.solve(0)
    s = o.scalars()
    assert s["status"] == 0, s
    u, v = o.get("u"), o.get("v")
    ng = g.n_gen
    np.testing.assert_allclose(u[0:2 * ng:2], p_ref, atol=1e-4)
    # bus voltage magnitudes from the bus-side w copies
    vm = np.zeros(g.n_bus)
    for l in range(g.n_branch):
        vm[g.br_from[l]] = np.sqrt(v[2 * ng + 8 * l + 4])
        vm[g.br_to[l]] = np.sqrt(v[2 * ng + 8 * l + 6])
    np.testing.assert_allclose(vm, vm_ref, atol=1e-4)
    f_admm = o.objective()
    f_ref = float(np.sum(g.c2 * (100 * p_ref) ** 2 + g.c1 * 100 * p_ref))
    assert abs(f_admm - f_ref) <= 1e-5 * f_ref


@pytest.mark.slow
def test_three_bus_warm_start_reaches_the_new_dense_optimum():
    """Warm start (Sec. IV-C): after new loads the oracle keeps its primal and
    dual state, restarts beta and the outer counter, and iterates to the
    solution of the ACOPF with the new loads (dense SLSQP), not the old one."""
    g = load_three_bus()
    p = O.OracleParams(rho_pq=400.0, rho_va=4000.0, obj_scale=0.01,
                       eps_pri=1e-7, eps_dual=1e-7, eps_z=1e-7,
                       max_inner=20000, max_outer=40)
    o = O.Oracle(g, p)
    o.solve(0)
    assert o.scalars()["status"] == 0
    p_old = o.get("u")[0:2 * g.n_gen:2].copy()
    x_old = o.get("bx").copy()
    pd2, qd2 = g.pd * 1.04, g.qd * 0.97
    g2 = dataclasses.replace(g, pd=pd2, qd=qd2)
    p_ref, _, vm_ref, _ = dense_acopf(g2)
    assert np.max(np.abs(p_ref - p_old)) > 1e-3   # the optimum moves
    o.update_loads(pd2, qd2)
    s = o.scalars()
    assert s["outer"] == 0 and s["inner_total"] == 0 and s["beta"] == p.beta0
    np.testing.assert_array_equal(o.get("bx"), x_old)   # state kept
    o.solve(0)
    s = o.scalars()
    assert s["status"] == 0, s
    ng = g.n_gen
    u, v = o.get("u"), o.get("v")
    np.testing.assert_allclose(u[0:2 * ng:2], p_ref, atol=1e-4)
    vm = np.zeros(g.n_bus)
    for l in range(g.n_branch):
        vm[g.br_from[l]] = np.sqrt(v[2 * ng + 8 * l + 4])
        vm[g.br_to[l]] = np.sqrt(v[2 * ng + 8 * l + 6])
    np.testing.assert_allclose(vm, vm_ref, atol=1e-4)


def ybus_quality(g, v, u):
    """||c(x)||_inf over eq. acopf from the textbook bus-injection form: complex
    voltages V = sqrt(w) e^{j theta}, branch currents through the pi model with
    a = tap e^{j shift} (series 1/(r + jx), charging jb/2 per end), S = V conj(I),
    bus shunts (g_s - j b_s) |V|^2. v and u are canonical coupling vectors."""
    ng, nl, nb = g.n_gen, g.n_branch, g.n_bus
    w = np.empty(nb)
    th = np.empty(nb)
    first = {}
    for l in range(nl):   # first incident end per bus: from-ends, then to-ends
        first.setdefault(("f", g.br_from[l]), l)
    for l in range(nl):
        first.setdefault(("t", g.br_to[l]), l)
    for i in range(nb):
        if ("f", i) in first:
            k = 2 * ng + 8 * first[("f", i)] + 4
        else:
            k = 2 * ng + 8 * first[("t", i)] + 6
        w[i], th[i] = v[k], v[k + 1]
    V = np.sqrt(w) * np.exp(1j * th)
    inj = np.zeros(nb, dtype=complex)
    line = 0.0
    for l in range(nl):
        i, j = g.br_from[l], g.br_to[l]
        ys = 1.0 / (g.r[l] + 1j * g.x[l])
        a = g.tap[l] * np.exp(1j * g.shift[l])
        yff = (ys + 0.5j * g.b[l]) / abs(a) ** 2
        yft = -ys / np.conj(a)
        ytf = -ys / a
        ytt = ys + 0.5j * g.b[l]
        Sf = V[i] * np.conj(yff * V[i] + yft * V[j])
        St = V[j] * np.conj(ytf * V[i] + ytt * V[j])
        inj[i] += Sf
        inj[j] += St
        if g.rate[l] > 0:
            line = max(line, abs(Sf) - g.rate[l], abs(St) - g.rate[l])
    inj += (g.gs - 1j * g.bs) * np.abs(V) ** 2
    sg = np.zeros(nb, dtype=complex)
    for k in range(ng):
        sg[g.gen_bus[k]] += u[2 * k] + 1j * u[2 * k + 1]
    mis = sg - (g.pd + 1j * g.qd) - inj
    vm = np.abs(V)
    volt = max(0.0, float(np.max(np.maximum(g.vmin - vm, vm - g.vmax))))
    ang = max(0.0, float(np.max(np.abs(th) - 2 * np.pi)))
    parts = [float(np.max(np.abs(mis.real))), float(np.max(np.abs(mis.imag))), max(line, 0.0),
             volt, ang]
    return [max(parts)] + parts


def test_quality_matches_bus_injection_form():
    """The oracle's solution-quality evaluator (Sec. IV-A: flows recomputed from
    the bus voltages) against S = V conj(I) with complex admittances, on a grid
    with taps, phase shifters, bus shunts and rated branches, at an ADMM
    iterate and at a perturbed state where every limit is violated."""
    g = gridgen(67, 9, 70, 0.5, 32, load_factor=0.2)
    rng = np.random.default_rng(7)
    g.gs = rng.uniform(0, 0.02, g.n_bus)
    g.bs = rng.uniform(-0.02, 0.02, g.n_bus)
    g.tap = rng.uniform(0.95, 1.05, g.n_branch)
    g.shift = rng.uniform(-0.1, 0.1, g.n_branch)
    o = O.Oracle(g, O.OracleParams(rho_pq=400.0, rho_va=4000.0))
    o.solve(40)
    names = O.QUALITY_NAMES
    for case in ("iterate", "perturbed"):
        if case == "perturbed":
            v = o.get("v")
            m0 = 2 * g.n_gen
            for l in range(g.n_branch):   # push voltages out of range, angles past 2 pi
                v[m0 + 8 * l + 4] *= 1.3
                v[m0 + 8 * l + 5] += 7.0
            o.set("v", v)
        q = o.quality()
        ref = ybus_quality(g, o.get("v"), o.get("u"))
        for name, r in zip(names, ref):
            assert abs(q[name] - r) <= 1e-11 * max(1.0, abs(r)), (case, name, q[name], r)
        if case == "perturbed":
            assert q["voltage_limit"] > 0.1 and q["angle_limit"] > 0.5 and q["line_limit"] > 0
        assert q["max_violation"] == max(q[n] for n in names[1:])


def test_carried_cauchy_step_matches_restart_at_one():
    """Each branch keeps its trust-region Cauchy step length between ADMM
    iterations. Against the same ADMM with the step length reset to 1 before
    every iteration (each TRON call then starts its Cauchy search at 1): the
    30-bus case converges in the same number of inner and outer iterations to
    the same objective, with far fewer Cauchy trials."""
    g = config_grid("c1_30bus")
    p = O.OracleParams(rho_pq=400.0, rho_va=400.0)
    a = O.Oracle(g, p)
    a.solve(0)
    b = O.Oracle(g, p)
    ones = np.ones(g.n_branch)
    for _ in range(p.max_outer * p.max_inner):
        b.set("calpha", ones)
        if b.iterate():
            break
    sa, sb = a.scalars(), b.scalars()
    assert sa["status"] == 0 and sb["status"] == 0
    assert abs(sa["inner_total"] - sb["inner_total"]) <= 0.02 * sb["inner_total"]
    assert sa["outer"] == sb["outer"]
    assert abs(a.objective() - b.objective()) <= 1e-6 * abs(b.objective())
    ca, cb = a.stats(), b.stats()
    assert ca["cauchy_trials"] / ca["tron_iters"] < 0.7 * cb["cauchy_trials"] / cb["tron_iters"]
    al = a.get("calpha")
    assert np.all(np.isfinite(al)) and np.all(al > 0.0)


def test_solution_recovery_matches_phasor_flows():
    """The oracle's solution of Sec. IV-A: generator outputs are the
    generator-side couplings, |V|^2 and theta are the bus copies w and theta
    of each bus's first branch end, and the branch flows equal the complex
    power S = V conj(I) of the pi model (numpy complex arithmetic) at those
    voltages, with taps and phase shifters."""
    from test_oracle_branch import phasor_flows, pi_model, random_grid_with_taps
    g = random_grid_with_taps(19)
    o = O.Oracle(g, O.OracleParams(rho_va=4000.0))
    o.solve(30)
    sol = o.solution()
    u, v = o.get("u"), o.get("v")
    np.testing.assert_array_equal(sol["pg"], u[0:2 * g.n_gen:2])
    np.testing.assert_array_equal(sol["qg"], u[1:2 * g.n_gen:2])
    base = 2 * g.n_gen
    for i in range(g.n_bus):
        frm = np.nonzero(g.br_from == i)[0]
        to = np.nonzero(g.br_to == i)[0]
        k = base + 8 * frm[0] + 4 if len(frm) else base + 8 * to[0] + 6
        assert sol["vm"][i] == np.sqrt(v[k]) and sol["va"][i] == v[k + 1]
    for l in range(g.n_branch):
        i, j = g.br_from[l], g.br_to[l]
        Y = pi_model(g.r[l], g.x[l], g.b[l], g.tap[l], g.shift[l])
        Sij, Sji = phasor_flows(Y, sol["vm"][i], sol["vm"][j], sol["va"][i], sol["va"][j])
        np.testing.assert_allclose([sol["pij"][l], sol["qij"][l], sol["pji"][l], sol["qji"][l]],
                                   [Sij.real, Sij.imag, Sji.real, Sji.imag], rtol=0, atol=1e-12)
