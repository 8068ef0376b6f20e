// Serial FP64 CPU oracle for the component-wise two-level ADMM for ACOPF
// (Kim & Kim, "Accelerated Computation and Tracking of AC Optimal Power Flow
// Solutions Using GPUs", PSCC 2022).
//
// TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the
// GPU path is checked against. Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark may load it. It shares no code, header or
// constant with the HIP library: it is written from the paper (and from Lin &
// More 1999 for the trust-region Newton method) on its own.
//
// Build: g++ -O2 -ffp-contract=off -fno-fast-math -mfma -fopenmp -fPIC
// -shared: no implicit contraction; OpenMP only for the optional parallel
// loops over independent elements (ora_set_threads; serial by default); the
// fused multiply-adds written out below (std::fma) are correctly rounded
// whether done by the FMA instruction or the library;
// IEEE division and square root; sin/cos of branch angles by the series
// below.
//
// Layout of the coupling vectors (canonical order, shared with the library's
// get_state only as a documented convention): generator g owns couplings
// 2g (p_g) and 2g+1 (q_g); branch l owns 2*n_gen + 8l + k for
// k = 0..7: p_ij, q_ij, p_ji, q_ji, w_i(ij), theta_i(ij), w_j(ij), theta_j(ij).
// Each coupling reads u_k - v_k + z_k = 0 with u the generator/branch side
// and v the bus side (Section II-B, II-C).
//
// Parity status per function (what the CPU tests pin it to) is listed in the
// test files; every function here is pinned there. (The random load changes
// of warm-start workloads are drawn by the shared input generators, not
// here.)

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Counting scalar: wraps a double and counts + - * / sqrt (1 each) and sin,
// cos (separately). Used to obtain the exact algorithmic flop count of a
// branch solve; the doubles it carries are bit-identical to plain double
// evaluation of the same expressions.
// ---------------------------------------------------------------------------
struct FlopTally {
  long long addsub = 0, mul = 0, div = 0, sqrt_ = 0, trig = 0;
  long long total() const { return addsub + mul + div + sqrt_; }
};
thread_local FlopTally g_tally;

struct CR {
  double v;
  CR() : v(0.0) {}
  CR(double d) : v(d) {}  // NOLINT: implicit on purpose
  CR& operator+=(CR o) { ++g_tally.addsub; v += o.v; return *this; }
  CR& operator-=(CR o) { ++g_tally.addsub; v -= o.v; return *this; }
  CR& operator*=(CR o) { ++g_tally.mul; v *= o.v; return *this; }
  CR& operator/=(CR o) { ++g_tally.div; v /= o.v; return *this; }
};
inline CR operator+(CR a, CR b) { ++g_tally.addsub; return CR(a.v + b.v); }
inline CR operator-(CR a, CR b) { ++g_tally.addsub; return CR(a.v - b.v); }
inline CR operator*(CR a, CR b) { ++g_tally.mul; return CR(a.v * b.v); }
inline CR operator/(CR a, CR b) { ++g_tally.div; return CR(a.v / b.v); }
inline CR operator-(CR a) { return CR(-a.v); }
inline bool operator<(CR a, CR b) { return a.v < b.v; }
inline bool operator>(CR a, CR b) { return a.v > b.v; }
inline bool operator<=(CR a, CR b) { return a.v <= b.v; }
inline bool operator>=(CR a, CR b) { return a.v >= b.v; }
inline bool operator==(CR a, CR b) { return a.v == b.v; }
inline bool operator!=(CR a, CR b) { return a.v != b.v; }
inline CR sqrt(CR a) { ++g_tally.sqrt_; return CR(std::sqrt(a.v)); }
// Fused multiply-add a*b + c with one rounding (IEEE 754 fusedMultiplyAdd),
// counted as one multiplication and one addition.
inline CR rfma(CR a, CR b, CR c) {
  ++g_tally.mul;
  ++g_tally.addsub;
  return CR(std::fma(a.v, b.v, c.v));
}
inline double rfma(double a, double b, double c) { return std::fma(a, b, c); }
inline double val(CR a) { return a.v; }
inline double val(double a) { return a; }

// sin and cos of the branch angle difference: Cody-Waite reduction by pi/2
// (pi/2 split into a 33-bit head and a tail, so k * head is exact) followed
// by the Taylor series of sin and cos on |r| <= pi/4, truncated after r^17
// and r^18 (remainders below 1e-19), evaluated by Horner's rule with fused
// multiply-adds. Written out
// here rather than taken from the C library so that the result is a fixed
// sequence of IEEE operations.
constexpr double kPio2Hi = 1.5707963267341256;       // 0x1.921fb544p+0
constexpr double kPio2Lo = 6.077100506506192e-11;    // pi/2 - kPio2Hi
constexpr double kTwoOverPi = 0.6366197723675814;
// (-1)^j / (2j+1)!, j = 1..8  and  (-1)^j / (2j)!, j = 1..9
constexpr double kSinC[8] = {-0.16666666666666666, 0.008333333333333333,
                             -0.0001984126984126984, 2.7557319223985893e-06,
                             -2.505210838544172e-08, 1.6059043836821613e-10,
                             -7.647163731819816e-13, 2.8114572543455206e-15};
constexpr double kCosC[9] = {-0.5, 0.041666666666666664, -0.001388888888888889,
                             2.48015873015873e-05, -2.755731922398589e-07,
                             2.08767569878681e-09, -1.1470745597729725e-11,
                             4.779477332387385e-14, -1.5619206968586225e-16};

inline void series_sincos(double x, double* s, double* c) {
  const double k = std::nearbyint(x * kTwoOverPi);
  const double r = std::fma(-k, kPio2Lo, std::fma(-k, kPio2Hi, x));
  const double r2 = r * r;
  double ps = kSinC[7];
  for (int j = 6; j >= 0; --j) ps = std::fma(r2, ps, kSinC[j]);
  double pc = kCosC[8];
  for (int j = 7; j >= 0; --j) pc = std::fma(r2, pc, kCosC[j]);
  const double sr = std::fma(r, r2 * ps, r);
  const double cr = std::fma(r2, pc, 1.0);
  const long long q = static_cast<long long>(k) & 3;
  if (q == 0) { *s = sr; *c = cr; }
  else if (q == 1) { *s = cr; *c = -sr; }
  else if (q == 2) { *s = -sr; *c = -cr; }
  else { *s = -cr; *c = sr; }
}

inline void rsincos(double x, double& s, double& c) { series_sincos(x, &s, &c); }
inline void rsincos(CR x, CR& s, CR& c) {
  g_tally.trig += 2;
  series_sincos(x.v, &s.v, &c.v);
}

template <class R> inline R rabs(R a) { return a < R(0.0) ? -a : a; }
template <class R> inline R rmin(R a, R b) { return b < a ? b : a; }
template <class R> inline R rmax(R a, R b) { return a < b ? b : a; }
template <class R> inline R rsqrt_(R a) { using std::sqrt; return sqrt(a); }

constexpr int NMAX = 8;
constexpr double TWO_PI = 6.283185307179586476925286766559;
constexpr double INF = std::numeric_limits<double>::infinity();

}  // namespace

extern "C" {

// Parameters of the method. Defaults live in the Python binding.
typedef struct {
  double rho_pq, rho_va;      // ADMM penalties (Table 1: power / voltage)
  double obj_scale;           // objective scaling inside the ADMM (Sec. IV-A)
  double rate_scale;          // line-limit tightening, 0.99 (Sec. IV-A)
  double beta0, beta_gamma, beta_omega, beta_max, lambda_max;  // outer level
  double eps_pri, eps_dual, eps_z;                             // termination
  int32_t max_outer, max_inner;
  double tron_gtol, tron_ftol;
  int32_t tron_maxit;
  double al_rho0, al_rho_growth, al_rho_max, al_tol, al_shrink;
  int32_t al_maxit;
} ora_params;

// Event counters of branch solves (summed over calls).
typedef struct {
  long long branch_solves, tron_calls, tron_iters, n_fgh, n_f, cauchy_trials,
      cg_iters, chol_attempts, ps_trials, al_iters, tron_converged,
      tron_maxit, tron_stall, flops, trig;
} ora_stats;

}  // extern "C"

namespace {

enum { TRON_CONVERGED = 0, TRON_MAXIT = 1, TRON_STALL = 2 };

// ---------------------------------------------------------------------------
// Trust-region Newton method for  min f(x)  s.t.  lo <= x <= hi  (n <= NMAX)
// after Lin & More (1999), as used for the branch subproblems (Sec. III-B):
// a generalized Cauchy step along the projected gradient, then subspace
// steps by preconditioned conjugate gradients with Steihaug's treatment of
// negative curvature and the trust-region boundary, each followed by a
// projected search; the trust-region ratio test decides acceptance.
// A dense Cholesky factorization of the scaled free Hessian (shifted when
// not positive definite), in its square-root-free form L E L', is the
// preconditioner: for n <= 6 the incomplete factorization of Lin & More is
// the complete one.
// ---------------------------------------------------------------------------
struct TronConst {
  double eta0 = 1e-4, eta1 = 0.25, eta2 = 0.75;
  double sigma1 = 0.25, sigma2 = 0.5, sigma3 = 4.0;
  double mu0 = 0.01, interpf = 0.1, extrapf = 10.0;
  int max_trials = 20;
  double cgtol = 0.1;
  double shift_min = 1e-3;
  int max_chol = 20;
};

template <class R>
inline R clampd(R t, double lo, double hi) {
  // projection onto [lo, hi] (lo <= hi), as fmin(fmax(t, lo), hi): the same
  // value as comparing with the bounds; a NaN t gives lo
  return R(std::fmin(std::fmax(val(t), lo), hi));
}

// q(s) = g's + 1/2 s'Hs
template <class R>
R model_q(int n, const R* g, const R* H, const R* s) {
  // q(s) = g's + s'Hs / 2 with H symmetric: s'Hs = sum_i s_i (H_ii s_i +
  // sum_{j<i} H_ij (2 s_j)), doubling being exact
  R t[NMAX];
  for (int j = 0; j < n; ++j) t[j] = R(2.0) * s[j];
  R gs = R(0.0), sHs = R(0.0);
  for (int i = 0; i < n; ++i) {
    gs = rfma(g[i], s[i], gs);
    R hi = H[i * n + i] * s[i];
    for (int j = 0; j < i; ++j) hi = rfma(H[i * n + j], t[j], hi);
    sHs = rfma(s[i], hi, sHs);
  }
  return rfma(R(0.5), sHs, gs);
}

template <class R>
R dotv(int n, const R* a, const R* b) {
  R t = R(0.0);
  for (int i = 0; i < n; ++i) t = rfma(a[i], b[i], t);
  return t;
}

// Step from a to the sphere ||a + tau p|| = delta, tau >= 0.
template <class R>
R to_boundary(int n, const R* a, const R* p, R delta) {
  R ap = dotv(n, a, p), pp = dotv(n, p, p), aa = dotv(n, a, a);
  R dd = delta * delta - aa;
  if (dd < R(0.0)) dd = R(0.0);
  R rad = ap * ap + pp * dd;
  R sq = rsqrt_(rad);
  R tau;
  if (ap >= R(0.0)) {
    R den = ap + sq;
    tau = den > R(0.0) ? dd / den : R(0.0);
  } else {
    tau = (sq - ap) / pp;
  }
  return tau;
}

// Generalized Cauchy point (Lin & More, Sec. 3).
template <class R>
void cauchy_step(int n, const R* x, const R* g, const R* H, const double* lo,
                 const double* hi, R delta, R& alpha, R* w, ora_stats* st,
                 const TronConst& C) {
  // largest breakpoint of the projected path x(alpha) = P(x - alpha g)
  R brpt = R(0.0);
  for (int i = 0; i < n; ++i) {
    R bp = R(0.0);
    if (g[i] > R(0.0)) {
      bp = lo[i] == -INF ? R(INF) : (x[i] - R(lo[i])) / g[i];
    } else if (g[i] < R(0.0)) {
      bp = hi[i] == INF ? R(INF) : (x[i] - R(hi[i])) / g[i];
    }
    brpt = rmax(brpt, bp);
  }
  R s[NMAX], wt[NMAX], st2[NMAX];
  auto trial = [&](R a, R* wout, R* sout) {
    for (int i = 0; i < n; ++i) {
      wout[i] = clampd(rfma(-a, g[i], x[i]), lo[i], hi[i]);
      sout[i] = wout[i] - x[i];
    }
  };
  auto accept = [&](const R* sv) {
    if (dotv(n, sv, sv) > delta * delta) return false;
    R q = model_q(n, g, H, sv);
    return q <= R(C.mu0) * dotv(n, g, sv);
  };
  trial(alpha, w, s);
  ++st->cauchy_trials;
  if (accept(s)) {
    // extrapolate while the conditions hold and the path still bends
    for (int t = 0; t < C.max_trials; ++t) {
      if (alpha > brpt) break;
      R a2 = alpha * R(C.extrapf);
      trial(a2, wt, st2);
      ++st->cauchy_trials;
      if (!accept(st2)) break;
      alpha = a2;
      for (int i = 0; i < n; ++i) w[i] = wt[i];
    }
  } else {
    for (int t = 0; t < C.max_trials; ++t) {
      alpha = alpha * R(C.interpf);
      trial(alpha, w, s);
      ++st->cauchy_trials;
      if (accept(s)) break;
    }
  }
}

// Square-root-free Cholesky A = L E L' (L unit lower, E diagonal; row-major,
// m x m), column by column: with v_k = L_jk e_k, the pivot is
// e_j = A_jj - sum_k L_jk v_k and the column below it is
// L_ij = (A_ij - sum_k L_ik v_k) / e_j, the division done as a multiplication
// by the reciprocal pivot, which is kept in rd for the solve. The same
// factorization as L~ L~' with L~ = L E^(1/2), without square roots.
// Returns false when a pivot is not positive.
template <class R>
bool ldlt(int m, const R* A, R* L, R* rd) {
  R e[NMAX];
  for (int i = 0; i < m * m; ++i) L[i] = R(0.0);
  for (int j = 0; j < m; ++j) {
    R v[NMAX];
    for (int k = 0; k < j; ++k) v[k] = L[j * m + k] * e[k];
    R d = A[j * m + j];
    for (int k = 0; k < j; ++k) d = rfma(-L[j * m + k], v[k], d);
    if (!(d > R(0.0))) return false;
    e[j] = d;
    L[j * m + j] = R(1.0);
    R rj = R(1.0) / d;
    rd[j] = rj;
    for (int i = j + 1; i < m; ++i) {
      R t = A[i * m + j];
      for (int k = 0; k < j; ++k) t = rfma(-L[i * m + k], v[k], t);
      L[i * m + j] = t * rj;
    }
  }
  return true;
}

// z = M^{-1} r with M = L E L'; rd holds the reciprocal pivots 1/e: forward
// solve with L, scaling by rd, backward solve with L'.
template <class R>
void precond(int m, const R* L, const R* rd, const R* r, R* z) {
  R t[NMAX];
  for (int i = 0; i < m; ++i) {
    R a = r[i];
    for (int k = 0; k < i; ++k) a = rfma(-L[i * m + k], t[k], a);
    t[i] = a;
  }
  for (int i = 0; i < m; ++i) t[i] = t[i] * rd[i];
  for (int i = m - 1; i >= 0; --i) {
    R a = t[i];
    for (int k = i + 1; k < m; ++k) a = rfma(-L[k * m + i], z[k], a);
    z[i] = a;
  }
}

// Subspace steps from the Cauchy point w (in/out). s = w - x on exit.
template <class R>
void subspace_step(int n, const R* x, const R* g, const R* H, const double* lo,
                   const double* hi, R delta, R* w, ora_stats* st,
                   const TronConst& C) {
  R s[NMAX];
  for (int i = 0; i < n; ++i) s[i] = w[i] - x[i];
  for (int pass = 0; pass < n; ++pass) {
    int F[NMAX], nf = 0;
    for (int i = 0; i < n; ++i)
      if (w[i] > R(lo[i]) && w[i] < R(hi[i])) F[nf++] = i;
    if (nf == 0) break;
    // gradient of the model at w
    R gq[NMAX];
    for (int i = 0; i < n; ++i) {
      R t = g[i];
      for (int j = 0; j < n; ++j) t = rfma(H[i * n + j], s[j], t);
      gq[i] = t;
    }
    R r[NMAX], B[NMAX * NMAX];
    for (int a = 0; a < nf; ++a) {
      r[a] = -gq[F[a]];
      for (int b = 0; b < nf; ++b) B[a * nf + b] = H[F[a] * n + F[b]];
    }
    R rr0 = dotv(nf, r, r);  // squared norm of the initial residual
    if (!(rr0 > R(0.0))) break;
    // preconditioner: Lin & More factor D B D + shift I with the scaling
    // D = diag(|B_aa|^(-1/2)) (1 where B_aa = 0), so that the preconditioner
    // is M = D^-1 (D B D + shift I) D^-1 = B + shift D^-2. It is formed here
    // as that matrix directly: the L E L' factorization of B + shift S with
    // S = diag(|B_aa|, or 1 where B_aa = 0). The scaled diagonal entries
    // D_a B_aa D_a are the signs of B_aa, whose minimum sets the shift.
    R Sd[NMAX], L[NMAX * NMAX], rd[NMAX];
    R mind = R(INF);
    for (int a = 0; a < nf; ++a) {
      R baa = B[a * nf + a];
      Sd[a] = baa == R(0.0) ? R(1.0) : rabs(baa);
      R sgn = baa > R(0.0) ? R(1.0) : (baa < R(0.0) ? R(-1.0) : R(0.0));
      mind = rmin(mind, sgn);
    }
    R shift = mind > R(0.0) ? R(0.0) : R(C.shift_min) - mind;
    bool ok = false;
    for (int att = 0; att < C.max_chol; ++att) {
      R A[NMAX * NMAX];
      for (int q = 0; q < nf * nf; ++q) A[q] = B[q];
      for (int a = 0; a < nf; ++a) A[a * nf + a] = rfma(shift, Sd[a], A[a * nf + a]);
      ++st->chol_attempts;
      if (ldlt(nf, A, L, rd)) { ok = true; break; }
      shift = rmax(R(2.0) * shift, R(C.shift_min));
    }
    if (!ok) {
      for (int q = 0; q < nf * nf; ++q) L[q] = R(0.0);
      for (int a = 0; a < nf; ++a) { L[a * nf + a] = R(1.0); rd[a] = R(1.0); }
    }
    // Steihaug PCG on min 1/2 d'Bd - r'd  s.t. ||s + d|| <= delta
    R d[NMAX], res[NMAX], zz[NMAX], p[NMAX], Bp[NMAX];
    for (int a = 0; a < nf; ++a) { d[a] = R(0.0); res[a] = r[a]; }
    precond(nf, L, rd, res, zz);
    for (int a = 0; a < nf; ++a) p[a] = zz[a];
    R rz = dotv(nf, res, zz);
    bool boundary = false;
    for (int k = 0; k < nf; ++k) {
      ++st->cg_iters;
      for (int a = 0; a < nf; ++a) {
        R t = R(0.0);
        for (int b = 0; b < nf; ++b) t = rfma(B[a * nf + b], p[b], t);
        Bp[a] = t;
      }
      R pBp = dotv(nf, p, Bp);
      // full-space vectors for the trust-region test
      R sd[NMAX], pf[NMAX];
      for (int i = 0; i < n; ++i) { sd[i] = s[i]; pf[i] = R(0.0); }
      for (int a = 0; a < nf; ++a) { sd[F[a]] = s[F[a]] + d[a]; pf[F[a]] = p[a]; }
      if (!(pBp > R(0.0))) {
        R tau = to_boundary(n, sd, pf, delta);
        for (int a = 0; a < nf; ++a) d[a] = rfma(tau, p[a], d[a]);
        boundary = true;
        break;
      }
      R alpha = rz / pBp;
      R tr[NMAX];
      for (int i = 0; i < n; ++i) tr[i] = rfma(alpha, pf[i], sd[i]);
      if (dotv(n, tr, tr) >= delta * delta) {
        R tau = to_boundary(n, sd, pf, delta);
        for (int a = 0; a < nf; ++a) d[a] = rfma(tau, p[a], d[a]);
        boundary = true;
        break;
      }
      for (int a = 0; a < nf; ++a) {
        d[a] = rfma(alpha, p[a], d[a]);
        res[a] = rfma(-alpha, Bp[a], res[a]);
      }
      if (dotv(nf, res, res) <= R(C.cgtol * C.cgtol) * rr0) break;
      precond(nf, L, rd, res, zz);
      R rzn = dotv(nf, res, zz);
      R bcg = rzn / rz;
      rz = rzn;
      for (int a = 0; a < nf; ++a) p[a] = rfma(bcg, p[a], zz[a]);
    }
    // projected search along d from w
    R qw = model_q(n, g, H, s);
    R beta = R(1.0);
    bool acc = false;
    R wt[NMAX], stv[NMAX];
    for (int t = 0; t < C.max_trials; ++t) {
      ++st->ps_trials;
      for (int i = 0; i < n; ++i) wt[i] = w[i];
      for (int a = 0; a < nf; ++a) {
        int i = F[a];
        wt[i] = clampd(rfma(beta, d[a], w[i]), lo[i], hi[i]);
      }
      for (int i = 0; i < n; ++i) stv[i] = wt[i] - x[i];
      R dw[NMAX];
      for (int i = 0; i < n; ++i) dw[i] = wt[i] - w[i];
      R qt = model_q(n, g, H, stv);
      if (qt <= rfma(R(C.mu0), dotv(n, gq, dw), qw)) { acc = true; break; }
      beta = beta * R(0.5);
    }
    if (!acc) break;
    bool hit = false;
    for (int a = 0; a < nf; ++a) {
      int i = F[a];
      if (wt[i] == R(lo[i]) || wt[i] == R(hi[i])) hit = true;
    }
    for (int i = 0; i < n; ++i) { w[i] = wt[i]; s[i] = stv[i]; }
    if (boundary || !hit) break;
  }
}

// Problem interface: f(x) and (f, g, H)(x) with H dense row-major n x n.
// alpha0 holds the Cauchy step length the projected search starts from; it
// receives the length the solve ends with.
template <class R, class P>
int tron(P& prob, int n, R* x, const double* lo, const double* hi,
         const ora_params& prm, ora_stats* st, const TronConst& C, double* alpha0) {
  ++st->tron_calls;
  for (int i = 0; i < n; ++i) x[i] = clampd(x[i], lo[i], hi[i]);
  R f, g[NMAX], H[NMAX * NMAX];
  prob.fgh(x, f, g, H);
  ++st->n_fgh;
  R pg2 = R(0.0);
  for (int i = 0; i < n; ++i) {
    R t = clampd(x[i] - g[i], lo[i], hi[i]) - x[i];
    pg2 = rfma(t, t, pg2);
  }
  R delta = rsqrt_(pg2);
  if (!(delta > R(0.0))) delta = R(1.0);
  R alphac = R(*alpha0);
  int status = TRON_MAXIT;
  for (int it = 0; it < prm.tron_maxit; ++it) {
    R pginf = R(0.0);
    for (int i = 0; i < n; ++i)
      pginf = rmax(pginf, rabs(clampd(x[i] - g[i], lo[i], hi[i]) - x[i]));
    if (pginf <= R(prm.tron_gtol)) { status = TRON_CONVERGED; break; }
    ++st->tron_iters;
    R w[NMAX], s[NMAX];
    cauchy_step(n, x, g, H, lo, hi, delta, alphac, w, st, C);
    subspace_step(n, x, g, H, lo, hi, delta, w, st, C);
    for (int i = 0; i < n; ++i) s[i] = w[i] - x[i];
    R prered = -model_q(n, g, H, s);
    R snorm = rsqrt_(dotv(n, s, s));
    if (!(prered > R(0.0))) { status = TRON_STALL; break; }
    // a full (interior) Newton-type step whose predicted decrease is at
    // the rounding level of f: accept it and stop
    if (snorm < delta &&
        prered <= R(prm.tron_ftol) * (R(1.0) + rabs(f))) {
      for (int i = 0; i < n; ++i) x[i] = w[i];
      status = TRON_CONVERGED;
      break;
    }
    R fw = prob.f(w);
    ++st->n_f;
    R actred = f - fw;
    R ratio = actred / prered;
    if (ratio <= R(C.eta0)) {
      delta = R(C.sigma2) * rmin(snorm, delta);
    } else if (ratio <= R(C.eta1)) {
      delta = rmax(R(C.sigma1) * delta, R(C.sigma2) * rmin(snorm, delta));
    } else if (ratio >= R(C.eta2)) {
      delta = rmin(R(C.sigma3) * delta, rmax(delta, R(C.sigma3) * snorm));
    }
    if (ratio > R(C.eta0)) {
      for (int i = 0; i < n; ++i) x[i] = w[i];
      prob.fgh(x, f, g, H);
      ++st->n_fgh;
    }
    // Delta <= 1e-15 max(1, ||x||), compared in squares
    R xx = dotv(n, x, x);
    if (delta * delta <= R(1e-30) * rmax(R(1.0), xx)) { status = TRON_STALL; break; }
  }
  *alpha0 = val(alphac);
  if (status == TRON_CONVERGED) ++st->tron_converged;
  else if (status == TRON_MAXIT) ++st->tron_maxit;
  else ++st->tron_stall;
  return status;
}

// ---------------------------------------------------------------------------
// Branch subproblem, eq. (branch): variables x = (v_i, v_j, theta_i(ij),
// theta_j(ij)[, s_ij, s_ji]); flows from eqs. (pij)-(qji) with
// w^R = v_i v_j cos(theta_i - theta_j), w^I = v_i v_j sin(theta_i - theta_j).
// ---------------------------------------------------------------------------
struct BranchData {
  double gii, bii, gij, bij, gji, bji, gjj, bjj;
  double lo[6], hi[6];
  int n;  // 4 or 6
  double vb[8], z[8], y[8], rho[8];
  // target of each coupling value: the residual is r_k = a_k - cv_k with
  // cv_k = v_k - z_k (formed once per ADMM iteration, by the bus step's
  // data; the textbook path uses a_k - v_k + z_k instead)
  double cv[8];
  double ltil[2], rtil;
};

// Values a_k(x) of the eight branch-side coupling quantities: flows p_ij,
// q_ij, p_ji, q_ji (eqs. pij-qji), then w_i = v_i^2, theta_i, w_j = v_j^2,
// theta_j. aux receives (cos, sin, w^R, w^I) when non-null.
template <class R>
void branch_values(const BranchData& d, const R* x, R* a, R* aux) {
  R vi = x[0], vj = x[1], ti = x[2], tj = x[3];
  R dt = ti - tj;
  R cs, sn;
  rsincos(dt, sn, cs);
  R vv = vi * vj;
  R WR = vv * cs, WI = vv * sn;
  R wi = vi * vi, wj = vj * vj;
  R gii = d.gii, bii = d.bii, gij = d.gij, bij = d.bij, gji = d.gji,
    bji = d.bji, gjj = d.gjj, bjj = d.bjj;
  a[0] = rfma(bij, WI, rfma(gij, WR, gii * wi));
  a[1] = rfma(gij, WI, rfma(-bij, WR, -bii * wi));
  a[2] = rfma(-bji, WI, rfma(gji, WR, gjj * wj));
  a[3] = rfma(-gji, WI, rfma(-bji, WR, -bjj * wj));
  a[4] = wi;
  a[5] = ti;
  a[6] = wj;
  a[7] = tj;
  if (aux) {
    aux[0] = cs;
    aux[1] = sn;
    aux[2] = WR;
    aux[3] = WI;
  }
}

// Upper triangle of a symmetric 4x4 matrix, row by row.
constexpr int UT_P[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
constexpr int UT_Q[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};

// Derivatives over (v_i, v_j, theta_i, theta_j). Each flow is linear in
// three quantities: a_k = cw_k w_own + cR_k w^R + cI_k w^I, with
// w^R = v_i v_j cos(theta_i - theta_j), w^I = v_i v_j sin(...) and w_own the
// squared magnitude at the flow's own end (v_i^2 for p_ij, q_ij; v_j^2 for
// p_ji, q_ji). W holds the gradients of w^R, w^I (dWR, dWI) and their
// upper-triangular Hessians (hWR, hWI, entries ordered as UT_P/UT_Q); ga the
// flow gradients.
template <class R>
struct WDerivs {
  R dWR[4], dWI[4], hWR[10], hWI[10];
  R cw[4], cR[4], cI[4];
};

template <class R>
void flow_derivs(const BranchData& d, const R* x, const R* aux, WDerivs<R>& W, R (*ga)[4]) {
  R vi = x[0], vj = x[1];
  R cs = aux[0], sn = aux[1], WR = aux[2], WI = aux[3];
  R jc = vj * cs, ic = vi * cs, js = vj * sn, is = vi * sn;
  R twvi = R(2.0) * vi, twvj = R(2.0) * vj;
  const R dWR[4] = {jc, ic, -WI, WI};
  const R dWI[4] = {js, is, WR, -WR};
  const R hWR[10] = {R(0.0), cs, -js, js, R(0.0), -is, is, -WR, WR, -WR};
  const R hWI[10] = {R(0.0), sn, jc, -jc, R(0.0), ic, -ic, -WI, WI, -WI};
  const R cw[4] = {R(d.gii), -R(d.bii), R(d.gjj), -R(d.bjj)};
  const R cR[4] = {R(d.gij), -R(d.bij), R(d.gji), -R(d.bji)};
  const R cI[4] = {R(d.bij), R(d.gij), -R(d.bji), -R(d.gji)};
  for (int p = 0; p < 4; ++p) { W.dWR[p] = dWR[p]; W.dWI[p] = dWI[p]; }
  for (int t = 0; t < 10; ++t) { W.hWR[t] = hWR[t]; W.hWI[t] = hWI[t]; }
  for (int k = 0; k < 4; ++k) { W.cw[k] = cw[k]; W.cR[k] = cR[k]; W.cI[k] = cI[k]; }
  for (int k = 0; k < 4; ++k) {
    int own = k < 2 ? 0 : 1;
    R tw = k < 2 ? twvi : twvj;
    for (int p = 0; p < 4; ++p) {
      if (p == own)
        ga[k][p] = rfma(cI[k], dWI[p], rfma(cR[k], dWR[p], cw[k] * tw));
      else
        ga[k][p] = rfma(cI[k], dWI[p], cR[k] * dWR[p]);
    }
  }
}

template <class R>
struct BranchProblem {
  const BranchData& d;
  explicit BranchProblem(const BranchData& dd) : d(dd) {}

  // F(x) = sum_k y_k r_k + rho_k/2 r_k^2 + sum_e ltil_e c_e + rtil/2 c_e^2
  // with r_k = a_k(x) - v_k + z_k, formed as a_k - (v_k - z_k), and
  // c_e = p_e^2 + q_e^2 + s_e.
  R f(const R* x) {
    R a[8];
    branch_values<R>(d, x, a, nullptr);
    R F = R(0.0);
    for (int k = 0; k < 8; ++k) {
      R r = a[k] - R(d.cv[k]);
      F = rfma(R(0.5) * R(d.rho[k]) * r, r, rfma(R(d.y[k]), r, F));
    }
    if (d.n == 6) {
      for (int e = 0; e < 2; ++e) {
        R c = rfma(a[2 * e], a[2 * e], a[2 * e + 1] * a[2 * e + 1]) + x[4 + e];
        F = rfma(R(0.5) * R(d.rtil) * c, c, rfma(R(d.ltil[e]), c, F));
      }
    }
    return F;
  }

  // F, its gradient and its Hessian (dense row-major n x n), by the chain
  // rule through the coupling values. With m_k = y_k + rho_k r_k for the
  // flows and, on rated branches, m_e = ltil_e + rtil c_e for the two line
  // limits (c_e = p_e^2 + q_e^2 + s_e, whose gradient is
  // 2 p_e grad p_e + 2 q_e grad q_e + e_s):
  //   grad F = sum_k mu_k grad a_k + (w, theta couplings) + m_e e_s,
  //   hess F = sum_k nu_k grad a_k grad a_k' + sum_k mu_k hess a_k
  //            + rtil grad c_e grad c_e' + (w, theta couplings),
  // where mu_k = m_k + 2 m_e a_k and nu_k = rho_k + 2 m_e for a flow k at
  // end e (mu_k = m_k, nu_k = rho_k without line limits). As the flows are
  // linear in (w_own, w^R, w^I), sum_k mu_k grad a_k and sum_k mu_k hess a_k
  // reduce to MR (grad, hess) w^R + MI (grad, hess) w^I + the w_own terms,
  // with MR = sum_k mu_k cR_k, MI = sum_k mu_k cI_k, O_i = mu_0 cw_0 +
  // mu_1 cw_1 (end i), O_j = mu_2 cw_2 + mu_3 cw_3 (end j).
  void fgh(const R* x, R& F, R* g, R* H) {
    const int n = d.n;
    R a[8], aux[4], ga[4][4];
    WDerivs<R> W;
    branch_values<R>(d, x, a, aux);
    flow_derivs<R>(d, x, aux, W, ga);
    F = R(0.0);
    // the four flow couplings
    R mu[4], nu[4];
    for (int k = 0; k < 4; ++k) {
      R r = a[k] - R(d.cv[k]);
      F = rfma(R(0.5) * R(d.rho[k]) * r, r, rfma(R(d.y[k]), r, F));
      mu[k] = rfma(R(d.rho[k]), r, R(d.y[k]));
      nu[k] = R(d.rho[k]);
    }
    // w_i = v_i^2 (variable 0), theta_i (2), w_j = v_j^2 (1), theta_j (3)
    const int var[4] = {0, 2, 1, 3};
    R mv[4];
    for (int k = 4; k < 8; ++k) {
      R r = a[k] - R(d.cv[k]);
      F = rfma(R(0.5) * R(d.rho[k]) * r, r, rfma(R(d.y[k]), r, F));
      mv[k - 4] = rfma(R(d.rho[k]), r, R(d.y[k]));
    }
    // augmented Lagrangian on the line limits (eq. branch, last two lines)
    R gc[2][4], me[2];
    if (n == 6) {
      for (int e = 0; e < 2; ++e) {
        int kp = 2 * e, kq = 2 * e + 1, s = 4 + e;
        R c = rfma(a[kp], a[kp], a[kq] * a[kq]) + x[s];
        F = rfma(R(0.5) * R(d.rtil) * c, c, rfma(R(d.ltil[e]), c, F));
        me[e] = rfma(R(d.rtil), c, R(d.ltil[e]));
        R tm = R(2.0) * me[e];
        mu[kp] = rfma(tm, a[kp], mu[kp]);
        mu[kq] = rfma(tm, a[kq], mu[kq]);
        nu[kp] = nu[kp] + tm;
        nu[kq] = nu[kq] + tm;
        for (int p = 0; p < 4; ++p)
          gc[e][p] = R(2.0) * rfma(a[kp], ga[kp][p], a[kq] * ga[kq][p]);
      }
    }
    R MR = rfma(mu[3], W.cR[3], rfma(mu[2], W.cR[2], rfma(mu[1], W.cR[1], mu[0] * W.cR[0])));
    R MI = rfma(mu[3], W.cI[3], rfma(mu[2], W.cI[2], rfma(mu[1], W.cI[1], mu[0] * W.cI[0])));
    R Oi = rfma(mu[1], W.cw[1], mu[0] * W.cw[0]);
    R Oj = rfma(mu[3], W.cw[3], mu[2] * W.cw[2]);
    for (int i = 0; i < n; ++i) {
      g[i] = R(0.0);
      for (int j = 0; j < n; ++j) H[i * n + j] = R(0.0);
    }
    for (int p = 0; p < 4; ++p) g[p] = rfma(MI, W.dWI[p], MR * W.dWR[p]);
    g[0] = rfma(R(2.0) * x[0], Oi, g[0]);
    g[1] = rfma(R(2.0) * x[1], Oj, g[1]);
    // Hessian block over (v_i, v_j, theta_i, theta_j), upper triangle
    R ng[4][4];
    for (int k = 0; k < 4; ++k)
      for (int p = 0; p < 4; ++p) ng[k][p] = nu[k] * ga[k][p];
    R rg[2][4];
    if (n == 6)
      for (int e = 0; e < 2; ++e)
        for (int p = 0; p < 4; ++p) rg[e][p] = R(d.rtil) * gc[e][p];
    for (int t = 0; t < 10; ++t) {
      int p = UT_P[t], q = UT_Q[t];
      R h;
      if (t == 0) h = R(2.0) * Oi;          // d2 w_i / dv_i^2 = 2
      else if (t == 4) h = R(2.0) * Oj;     // d2 w_j / dv_j^2 = 2
      else h = rfma(MI, W.hWI[t], MR * W.hWR[t]);
      for (int k = 0; k < 4; ++k) h = rfma(ng[k][p], ga[k][q], h);
      if (n == 6)
        for (int e = 0; e < 2; ++e) h = rfma(rg[e][p], gc[e][q], h);
      H[p * n + q] = h;
    }
    if (n == 6) {
      for (int e = 0; e < 2; ++e) {
        int s = 4 + e;
        g[s] = me[e];
        for (int p = 0; p < 4; ++p) H[p * 6 + s] = rg[e][p];
        H[s * 6 + s] = R(d.rtil);
      }
    }
    // the w and theta couplings act on single variables
    for (int k = 4; k < 8; ++k) {
      int p = var[k - 4];
      R m = mv[k - 4];
      if (k == 4 || k == 6) {  // d(v^2)/dv = 2v, d2(v^2)/dv2 = 2
        R gv = R(2.0) * x[p];
        g[p] = rfma(m, gv, g[p]);
        H[p * n + p] = rfma(m, R(2.0), rfma(R(d.rho[k]) * gv, gv, H[p * n + p]));
      } else {  // angle copy: gradient 1, no curvature
        g[p] = g[p] + m;
        H[p * n + p] = H[p * n + p] + R(d.rho[k]);
      }
    }
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) H[q * n + p] = H[p * n + q];
  }
};

// Branch solve (Sec. II-C, III-B): one TRON solve for unrated branches; for
// rated ones an augmented-Lagrangian loop on p^2 + q^2 + s = 0 around TRON.
// x (6), ltil (2), rtil and alpha are the persistent branch state; u (8)
// receives the branch-side coupling values a_k(x). alpha is the Cauchy step
// length of TRON's projected search: each TRON call starts from the length
// the branch's previous call ended with (1 after a cold start), which TRON
// itself already does from one iteration to the next within a call.
template <class R>
void branch_solve_t(BranchData& d, double* x6, double* ltil, double* rtil,
                    double* alpha, double* u8, const ora_params& prm, ora_stats* st) {
  TronConst C;
  ++st->branch_solves;
  R x[NMAX];
  for (int i = 0; i < d.n; ++i) x[i] = R(x6[i]);
  if (d.n == 4) {
    BranchProblem<R> P(d);
    tron<R>(P, 4, x, d.lo, d.hi, prm, st, C, alpha);
  } else {
    d.ltil[0] = ltil[0];
    d.ltil[1] = ltil[1];
    d.rtil = *rtil;
    R cprev = R(INF);
    for (int t = 0; t < prm.al_maxit; ++t) {
      ++st->al_iters;
      BranchProblem<R> P(d);
      tron<R>(P, 6, x, d.lo, d.hi, prm, st, C, alpha);
      R a[8];
      branch_values<R>(d, x, a, nullptr);
      R c0 = rfma(a[0], a[0], a[1] * a[1]) + x[4];
      R c1 = rfma(a[2], a[2], a[3] * a[3]) + x[5];
      R cn = rmax(rabs(c0), rabs(c1));
      // first-order multiplier estimate after every round, the last one
      // included, so that the persisted ltil is the multiplier of the
      // subproblem just solved
      d.ltil[0] = val(R(d.ltil[0]) + R(d.rtil) * c0);
      d.ltil[1] = val(R(d.ltil[1]) + R(d.rtil) * c1);
      if (cn <= R(prm.al_tol)) break;
      if (cn > R(prm.al_shrink) * cprev)
        d.rtil = val(rmin(R(d.rtil) * R(prm.al_rho_growth), R(prm.al_rho_max)));
      cprev = cn;
    }
    ltil[0] = d.ltil[0];
    ltil[1] = d.ltil[1];
    *rtil = d.rtil;
  }
  R a[8];
  branch_values<R>(d, x, a, nullptr);
  for (int k = 0; k < 8; ++k) u8[k] = val(a[k]);
  for (int i = 0; i < d.n; ++i) x6[i] = val(x[i]);
}

// ---------------------------------------------------------------------------
// Textbook path: the same method evaluated a second way, in the form in which
// the paper and Lin & More state it, so that the path above (which fixes one
// IEEE operation sequence) can be checked against it by the CPU tests:
//   * eq. (branch) summed term by term: F = sum_k y_k r_k + rho_k/2 r_k^2
//     + sum_e ltil_e c_e + rtil/2 c_e^2, with the gradient and Hessian of
//     each coupling value a_k written out from eqs. (pij)-(qji) and the chain
//     rule applied per term (no grouping of terms);
//   * sin and cos from the C library;
//   * plain products and sums (no fused multiply-adds; the library is built
//     without contraction), divisions, and square roots in the norm tests;
//   * the full quadratic model g's + s'(Hs)/2;
//   * the Lin & More preconditioner as they define it: the Cholesky factor
//     L L' = D H_FF D + alpha I with D = diag(|H_ii|^(-1/2)) (1 where
//     H_ii = 0), applied as z = D L'^-1 L^-1 D r.
// The decisions of the method (Cauchy extrapolation or interpolation,
// free sets, CG exits, the ratio test, the augmented-Lagrangian rounds) are
// the same rules; only the arithmetic that feeds them differs, by rounding.
// ---------------------------------------------------------------------------
namespace tb {

// Value, gradient and Hessian of one coupling quantity over the four voltage
// variables (v_i, v_j, theta_i, theta_j).
struct Quantity {
  double a;
  double g[4];
  double H[4][4];
};

// One flow of eqs. (pij)-(qji) in the form
//   a = alpha v_own^2 + v_i v_j (beta cos(theta_i - theta_j)
//                                + gamma sin(theta_i - theta_j)),
// own = 0 (v_i) or 1 (v_j): p_ij = g_ii w_i + g_ij w^R + b_ij w^I, etc.
void flow(double alpha, double beta, double gamma, int own, const double* x,
          Quantity& q) {
  const double vi = x[0], vj = x[1];
  const double d = x[2] - x[3];
  const double c = std::cos(d), s = std::sin(d);
  const double T = beta * c + gamma * s;    // d-part of the bracket
  const double Td = -beta * s + gamma * c;  // its derivative in d
  const double vo = own == 0 ? vi : vj;
  q.a = alpha * vo * vo + vi * vj * T;
  // first derivatives; d/dtheta_i = +d/dd, d/dtheta_j = -d/dd
  q.g[0] = vj * T;
  q.g[1] = vi * T;
  q.g[2] = vi * vj * Td;
  q.g[3] = -(vi * vj * Td);
  q.g[own] = q.g[own] + 2.0 * alpha * vo;
  // second derivatives (d2T/dd2 = -T)
  for (int p = 0; p < 4; ++p)
    for (int r = 0; r < 4; ++r) q.H[p][r] = 0.0;
  q.H[0][1] = T;
  q.H[0][2] = vj * Td;
  q.H[0][3] = -(vj * Td);
  q.H[1][2] = vi * Td;
  q.H[1][3] = -(vi * Td);
  q.H[2][2] = -(vi * vj * T);
  q.H[2][3] = vi * vj * T;
  q.H[3][3] = -(vi * vj * T);
  for (int p = 0; p < 4; ++p)
    for (int r = 0; r < p; ++r) q.H[p][r] = q.H[r][p];
  q.H[own][own] = q.H[own][own] + 2.0 * alpha;
}

// The eight coupling quantities of branch (i, j): p_ij, q_ij, p_ji, q_ji
// (eqs. pij-qji, with w^I_ji = -w^I_ij), then w_i = v_i^2, theta_i,
// w_j = v_j^2, theta_j.
void quantities(const BranchData& d, const double* x, Quantity* Q) {
  flow(d.gii, d.gij, d.bij, 0, x, Q[0]);
  flow(-d.bii, -d.bij, d.gij, 0, x, Q[1]);
  flow(d.gjj, d.gji, -d.bji, 1, x, Q[2]);
  flow(-d.bjj, -d.bji, -d.gji, 1, x, Q[3]);
  for (int k = 4; k < 8; ++k) {
    Q[k].a = 0.0;
    for (int p = 0; p < 4; ++p) {
      Q[k].g[p] = 0.0;
      for (int r = 0; r < 4; ++r) Q[k].H[p][r] = 0.0;
    }
  }
  Q[4].a = x[0] * x[0];
  Q[4].g[0] = 2.0 * x[0];
  Q[4].H[0][0] = 2.0;
  Q[5].a = x[2];
  Q[5].g[2] = 1.0;
  Q[6].a = x[1] * x[1];
  Q[6].g[1] = 2.0 * x[1];
  Q[6].H[1][1] = 2.0;
  Q[7].a = x[3];
  Q[7].g[3] = 1.0;
}

// Eq. (branch) and, when g is non-null, its gradient and Hessian (row-major
// n x n), summed term by term.
double branch_fgh(const BranchData& d, const double* x, double* g, double* H) {
  const int n = d.n;
  Quantity Q[8];
  quantities(d, x, Q);
  double F = 0.0;
  if (g)
    for (int i = 0; i < n; ++i) {
      g[i] = 0.0;
      for (int j = 0; j < n; ++j) H[i * n + j] = 0.0;
    }
  // ADMM terms y_k r_k + rho_k/2 r_k^2, r_k = a_k - v_k + z_k
  for (int k = 0; k < 8; ++k) {
    const double r = Q[k].a - d.vb[k] + d.z[k];
    F = F + d.y[k] * r + 0.5 * d.rho[k] * r * r;
    if (!g) continue;
    const double m = d.y[k] + d.rho[k] * r;  // dF/da_k
    for (int p = 0; p < 4; ++p) {
      g[p] = g[p] + m * Q[k].g[p];
      for (int q = 0; q < 4; ++q)
        H[p * n + q] = H[p * n + q] + d.rho[k] * Q[k].g[p] * Q[k].g[q] + m * Q[k].H[p][q];
    }
  }
  if (n == 6) {
    // line limits: c_e = p_e^2 + q_e^2 + s_e with ltil_e c_e + rtil/2 c_e^2
    for (int e = 0; e < 2; ++e) {
      const Quantity& P = Q[2 * e];
      const Quantity& R = Q[2 * e + 1];
      const int sv = 4 + e;
      const double c = P.a * P.a + R.a * R.a + x[sv];
      F = F + d.ltil[e] * c + 0.5 * d.rtil * c * c;
      if (!g) continue;
      const double m = d.ltil[e] + d.rtil * c;  // dF/dc_e
      double gc[6] = {0, 0, 0, 0, 0, 0};
      for (int p = 0; p < 4; ++p) gc[p] = 2.0 * P.a * P.g[p] + 2.0 * R.a * R.g[p];
      gc[sv] = 1.0;
      for (int p = 0; p < 6; ++p) {
        g[p] = g[p] + m * gc[p];
        for (int q = 0; q < 6; ++q) {
          double hc = 0.0;  // Hessian of c_e (zero in the slack rows)
          if (p < 4 && q < 4)
            hc = 2.0 * P.g[p] * P.g[q] + 2.0 * P.a * P.H[p][q] +
                 2.0 * R.g[p] * R.g[q] + 2.0 * R.a * R.H[p][q];
          H[p * 6 + q] = H[p * 6 + q] + d.rtil * gc[p] * gc[q] + m * hc;
        }
      }
    }
  }
  return F;
}

double proj(double t, double lo, double hi) { return t < lo ? lo : (t > hi ? hi : t); }

double dot(int n, const double* a, const double* b) {
  double t = 0.0;
  for (int i = 0; i < n; ++i) t = t + a[i] * b[i];
  return t;
}

double norm2(int n, const double* a) { return std::sqrt(dot(n, a, a)); }

// q(s) = g's + s'(Hs)/2
double model(int n, const double* g, const double* H, const double* s) {
  double Hs[NMAX];
  for (int i = 0; i < n; ++i) Hs[i] = dot(n, &H[i * n], s);
  return dot(n, g, s) + 0.5 * dot(n, s, Hs);
}

// tau >= 0 with ||a + tau p|| = delta, in the cancellation-free form of
// Lin & More's trust-region CG
double to_boundary(int n, const double* a, const double* p, double delta) {
  const double ap = dot(n, a, p), pp = dot(n, p, p), aa = dot(n, a, a);
  double dd = delta * delta - aa;
  if (dd < 0.0) dd = 0.0;
  const double sq = std::sqrt(ap * ap + pp * dd);
  if (ap >= 0.0) return ap + sq > 0.0 ? dd / (ap + sq) : 0.0;
  return (sq - ap) / pp;
}

// Cholesky A = L L' (L lower, row-major m x m); false at a non-positive pivot.
bool cholesky(int m, const double* A, double* L) {
  for (int i = 0; i < m * m; ++i) L[i] = 0.0;
  for (int j = 0; j < m; ++j) {
    double d = A[j * m + j];
    for (int k = 0; k < j; ++k) d = d - L[j * m + k] * L[j * m + k];
    if (!(d > 0.0)) return false;
    const double ljj = std::sqrt(d);
    L[j * m + j] = ljj;
    for (int i = j + 1; i < m; ++i) {
      double t = A[i * m + j];
      for (int k = 0; k < j; ++k) t = t - L[i * m + k] * L[j * m + k];
      L[i * m + j] = t / ljj;
    }
  }
  return true;
}

// z = M^-1 r for M = D^-1 L L' D^-1: z = D L'^-1 L^-1 D r.
void precondition(int m, const double* L, const double* Dg, const double* r, double* z) {
  double t[NMAX];
  for (int i = 0; i < m; ++i) {
    double a = Dg[i] * r[i];
    for (int k = 0; k < i; ++k) a = a - L[i * m + k] * t[k];
    t[i] = a / L[i * m + i];
  }
  for (int i = m - 1; i >= 0; --i) {
    double a = t[i];
    for (int k = i + 1; k < m; ++k) a = a - L[k * m + i] * z[k];
    z[i] = a / L[i * m + i];
  }
  for (int i = 0; i < m; ++i) z[i] = Dg[i] * z[i];
}

void cauchy(int n, const double* x, const double* g, const double* H, const double* lo,
            const double* hi, double delta, double& alpha, double* w, ora_stats* st,
            const TronConst& C) {
  // the projected path x(alpha) = P(x - alpha g) bends at its breakpoints;
  // extrapolation stops beyond the largest one
  double brpt = 0.0;
  for (int i = 0; i < n; ++i) {
    double bp = 0.0;
    if (g[i] > 0.0) bp = lo[i] == -INF ? INF : (x[i] - lo[i]) / g[i];
    else if (g[i] < 0.0) bp = hi[i] == INF ? INF : (x[i] - hi[i]) / g[i];
    if (bp > brpt) brpt = bp;
  }
  auto step = [&](double a, double* wo, double* so) {
    for (int i = 0; i < n; ++i) {
      wo[i] = proj(x[i] - a * g[i], lo[i], hi[i]);
      so[i] = wo[i] - x[i];
    }
  };
  // sufficient decrease of the model inside the trust region
  auto ok = [&](const double* s) {
    if (norm2(n, s) > delta) return false;
    return model(n, g, H, s) <= C.mu0 * dot(n, g, s);
  };
  double s[NMAX], wt[NMAX], s2[NMAX];
  step(alpha, w, s);
  ++st->cauchy_trials;
  if (ok(s)) {
    for (int t = 0; t < C.max_trials; ++t) {
      if (alpha > brpt) break;
      const double a2 = alpha * C.extrapf;
      step(a2, wt, s2);
      ++st->cauchy_trials;
      if (!ok(s2)) break;
      alpha = a2;
      for (int i = 0; i < n; ++i) w[i] = wt[i];
    }
  } else {
    for (int t = 0; t < C.max_trials; ++t) {
      alpha = alpha * C.interpf;
      step(alpha, w, s);
      ++st->cauchy_trials;
      if (ok(s)) break;
    }
  }
}

void subspace(int n, const double* x, const double* g, const double* H, const double* lo,
              const double* hi, double delta, double* w, ora_stats* st, const TronConst& C) {
  double s[NMAX];
  for (int i = 0; i < n; ++i) s[i] = w[i] - x[i];
  for (int pass = 0; pass < n; ++pass) {
    int F[NMAX], nf = 0;
    for (int i = 0; i < n; ++i)
      if (w[i] > lo[i] && w[i] < hi[i]) F[nf++] = i;
    if (nf == 0) break;
    // gradient of the model at w: g + H s
    double gq[NMAX];
    for (int i = 0; i < n; ++i) gq[i] = g[i] + dot(n, &H[i * n], s);
    double r[NMAX], B[NMAX * NMAX];
    for (int a = 0; a < nf; ++a) {
      r[a] = -gq[F[a]];
      for (int b = 0; b < nf; ++b) B[a * nf + b] = H[F[a] * n + F[b]];
    }
    const double r0 = norm2(nf, r);
    if (!(r0 > 0.0)) break;
    // Lin & More: L L' = D B D + shift I, D = diag(|B_aa|^(-1/2))
    double Dg[NMAX], DBD[NMAX * NMAX], L[NMAX * NMAX];
    for (int a = 0; a < nf; ++a) {
      const double baa = B[a * nf + a];
      Dg[a] = baa == 0.0 ? 1.0 : 1.0 / std::sqrt(std::fabs(baa));
    }
    double mind = INF;
    for (int a = 0; a < nf; ++a)
      for (int b = 0; b < nf; ++b) DBD[a * nf + b] = Dg[a] * B[a * nf + b] * Dg[b];
    for (int a = 0; a < nf; ++a) mind = std::min(mind, DBD[a * nf + a]);
    double shift = mind > 0.0 ? 0.0 : C.shift_min - mind;
    bool fact = false;
    for (int att = 0; att < C.max_chol; ++att) {
      double A[NMAX * NMAX];
      for (int q = 0; q < nf * nf; ++q) A[q] = DBD[q];
      for (int a = 0; a < nf; ++a) A[a * nf + a] = A[a * nf + a] + shift;
      ++st->chol_attempts;
      if (cholesky(nf, A, L)) { fact = true; break; }
      shift = std::max(2.0 * shift, C.shift_min);
    }
    if (!fact) {  // no factorization: unpreconditioned CG
      for (int q = 0; q < nf * nf; ++q) L[q] = 0.0;
      for (int a = 0; a < nf; ++a) { L[a * nf + a] = 1.0; Dg[a] = 1.0; }
    }
    // Steihaug's preconditioned CG on min d'Bd/2 - r'd within ||s + d|| <= delta
    double d[NMAX], res[NMAX], zz[NMAX], p[NMAX], Bp[NMAX];
    for (int a = 0; a < nf; ++a) { d[a] = 0.0; res[a] = r[a]; }
    precondition(nf, L, Dg, res, zz);
    for (int a = 0; a < nf; ++a) p[a] = zz[a];
    double rz = dot(nf, res, zz);
    bool boundary = false;
    for (int k = 0; k < nf; ++k) {
      ++st->cg_iters;
      for (int a = 0; a < nf; ++a) Bp[a] = dot(nf, &B[a * nf], p);
      const double pBp = dot(nf, p, Bp);
      double sd[NMAX], pf[NMAX];  // s + d and p in the full space
      for (int i = 0; i < n; ++i) { sd[i] = s[i]; pf[i] = 0.0; }
      for (int a = 0; a < nf; ++a) { sd[F[a]] = s[F[a]] + d[a]; pf[F[a]] = p[a]; }
      if (!(pBp > 0.0)) {  // negative curvature: to the boundary
        const double tau = to_boundary(n, sd, pf, delta);
        for (int a = 0; a < nf; ++a) d[a] = d[a] + tau * p[a];
        boundary = true;
        break;
      }
      const double alpha = rz / pBp;
      double tr[NMAX];
      for (int i = 0; i < n; ++i) tr[i] = sd[i] + alpha * pf[i];
      if (norm2(n, tr) >= delta) {  // leaves the region: stop on the boundary
        const double tau = to_boundary(n, sd, pf, delta);
        for (int a = 0; a < nf; ++a) d[a] = d[a] + tau * p[a];
        boundary = true;
        break;
      }
      for (int a = 0; a < nf; ++a) {
        d[a] = d[a] + alpha * p[a];
        res[a] = res[a] - alpha * Bp[a];
      }
      if (norm2(nf, res) <= C.cgtol * r0) break;
      precondition(nf, L, Dg, res, zz);
      const double rzn = dot(nf, res, zz);
      const double bcg = rzn / rz;
      rz = rzn;
      for (int a = 0; a < nf; ++a) p[a] = zz[a] + bcg * p[a];
    }
    // projected search along d from w, backtracking by halves
    const double qw = model(n, g, H, s);
    double beta = 1.0;
    bool acc = false;
    double wt[NMAX], stv[NMAX];
    for (int t = 0; t < C.max_trials; ++t) {
      ++st->ps_trials;
      for (int i = 0; i < n; ++i) wt[i] = w[i];
      for (int a = 0; a < nf; ++a) wt[F[a]] = proj(w[F[a]] + beta * d[a], lo[F[a]], hi[F[a]]);
      double dw[NMAX];
      for (int i = 0; i < n; ++i) { stv[i] = wt[i] - x[i]; dw[i] = wt[i] - w[i]; }
      if (model(n, g, H, stv) <= qw + C.mu0 * dot(n, gq, dw)) { acc = true; break; }
      beta = beta * 0.5;
    }
    if (!acc) break;
    bool hit = false;  // a new bound became active
    for (int a = 0; a < nf; ++a)
      if (wt[F[a]] == lo[F[a]] || wt[F[a]] == hi[F[a]]) hit = true;
    for (int i = 0; i < n; ++i) { w[i] = wt[i]; s[i] = stv[i]; }
    if (boundary || !hit) break;
  }
}

// Lin & More's trust-region Newton method for a bound-constrained problem
// with f and (f, g, H) callbacks; alpha0 carries the Cauchy step length.
template <class P>
int tron(P& prob, int n, double* x, const double* lo, const double* hi,
         const ora_params& prm, ora_stats* st, const TronConst& C, double* alpha0) {
  ++st->tron_calls;
  for (int i = 0; i < n; ++i) x[i] = proj(x[i], lo[i], hi[i]);
  double f, g[NMAX], H[NMAX * NMAX];
  prob.fgh(x, f, g, H);
  ++st->n_fgh;
  double pg[NMAX];
  for (int i = 0; i < n; ++i) pg[i] = proj(x[i] - g[i], lo[i], hi[i]) - x[i];
  double delta = norm2(n, pg);
  if (!(delta > 0.0)) delta = 1.0;
  double alphac = *alpha0;
  int status = TRON_MAXIT;
  for (int it = 0; it < prm.tron_maxit; ++it) {
    double pginf = 0.0;  // infinity norm of the projected gradient
    for (int i = 0; i < n; ++i)
      pginf = std::max(pginf, std::fabs(proj(x[i] - g[i], lo[i], hi[i]) - x[i]));
    if (pginf <= prm.tron_gtol) { status = TRON_CONVERGED; break; }
    ++st->tron_iters;
    double w[NMAX], s[NMAX];
    cauchy(n, x, g, H, lo, hi, delta, alphac, w, st, C);
    subspace(n, x, g, H, lo, hi, delta, w, st, C);
    for (int i = 0; i < n; ++i) s[i] = w[i] - x[i];
    const double prered = -model(n, g, H, s);
    const double snorm = norm2(n, s);
    if (!(prered > 0.0)) { status = TRON_STALL; break; }
    if (snorm < delta && prered <= prm.tron_ftol * (1.0 + std::fabs(f))) {
      for (int i = 0; i < n; ++i) x[i] = w[i];
      status = TRON_CONVERGED;
      break;
    }
    const double fw = prob.f(w);
    ++st->n_f;
    const double ratio = (f - fw) / prered;
    if (ratio <= C.eta0) delta = C.sigma2 * std::min(snorm, delta);
    else if (ratio <= C.eta1) delta = std::max(C.sigma1 * delta, C.sigma2 * std::min(snorm, delta));
    else if (ratio >= C.eta2) delta = std::min(C.sigma3 * delta, std::max(delta, C.sigma3 * snorm));
    if (ratio > C.eta0) {
      for (int i = 0; i < n; ++i) x[i] = w[i];
      prob.fgh(x, f, g, H);
      ++st->n_fgh;
    }
    if (delta <= 1e-15 * std::max(1.0, norm2(n, x))) { status = TRON_STALL; break; }
  }
  *alpha0 = alphac;
  if (status == TRON_CONVERGED) ++st->tron_converged;
  else if (status == TRON_MAXIT) ++st->tron_maxit;
  else ++st->tron_stall;
  return status;
}

struct Problem {
  const BranchData& d;
  double f(const double* x) { return branch_fgh(d, x, nullptr, nullptr); }
  void fgh(const double* x, double& F, double* g, double* H) { F = branch_fgh(d, x, g, H); }
};

// The branch solve of Sec. II-C and III-B as above (one trust-region solve,
// or the augmented-Lagrangian rounds on the line limits around it).
void branch_solve(BranchData& d, double* x6, double* ltil, double* rtil, double* alpha,
                  double* u8, const ora_params& prm, ora_stats* st) {
  TronConst C;
  ++st->branch_solves;
  double x[NMAX];
  for (int i = 0; i < d.n; ++i) x[i] = x6[i];
  if (d.n == 4) {
    Problem P{d};
    tron(P, 4, x, d.lo, d.hi, prm, st, C, alpha);
  } else {
    d.ltil[0] = ltil[0];
    d.ltil[1] = ltil[1];
    d.rtil = *rtil;
    double cprev = INF;
    for (int t = 0; t < prm.al_maxit; ++t) {
      ++st->al_iters;
      Problem P{d};
      tron(P, 6, x, d.lo, d.hi, prm, st, C, alpha);
      Quantity Q[8];
      quantities(d, x, Q);
      const double c0 = Q[0].a * Q[0].a + Q[1].a * Q[1].a + x[4];
      const double c1 = Q[2].a * Q[2].a + Q[3].a * Q[3].a + x[5];
      const double cn = std::max(std::fabs(c0), std::fabs(c1));
      d.ltil[0] = d.ltil[0] + d.rtil * c0;
      d.ltil[1] = d.ltil[1] + d.rtil * c1;
      if (cn <= prm.al_tol) break;
      if (cn > prm.al_shrink * cprev) d.rtil = std::min(d.rtil * prm.al_rho_growth, prm.al_rho_max);
      cprev = cn;
    }
    ltil[0] = d.ltil[0];
    ltil[1] = d.ltil[1];
    *rtil = d.rtil;
  }
  Quantity Q[8];
  quantities(d, x, Q);
  for (int k = 0; k < 8; ++k) u8[k] = Q[k].a;
  for (int i = 0; i < d.n; ++i) x6[i] = x[i];
}

}  // namespace tb

// ---------------------------------------------------------------------------
// Whole-grid state
// ---------------------------------------------------------------------------
struct Oracle {
  ora_params p;
  int nb, ng, nl, ref, m;
  double base;
  std::vector<double> pd, qd, gs, bs, vmin, vmax;
  std::vector<int> gbus;
  std::vector<double> pmin, pmax, qmin, qmax, c2, c1, c0;
  std::vector<int> from, to;
  // admittances (Sec. II-A, below eq. acopf) and squared scaled ratings
  std::vector<double> gii, bii, gij, bij, gji, bji, gjj, bjj, rate2;
  std::vector<double> rate;  // unscaled rating (p.u.), <= 0 unlimited
  std::vector<int> rated;
  // couplings
  std::vector<double> u, v, z, y, lam, rho, vprev;
  // branch state
  std::vector<double> bx, ltil, rtil, calpha;
  // per-bus incidence: gens, branches as from, branches as to
  std::vector<std::vector<int>> bus_gens, bus_from, bus_to;
  // outer-level scalars (Algorithm 1)
  double beta = 0, znorm_prev = INF, r_pri = 0, r_dual = 0, r_z = 0;
  int outer = 0, inner_total = 0, inner_in_outer = 0, status = 1;
  bool solved_once = false;
  std::vector<double> hist;  // per inner iteration: r_pri r_dual r_z obj beta outer
  ora_stats st{};
  bool count_flops = false;
  bool textbook = false;  // branch solves by the textbook path (namespace tb)
  int threads = 1;        // OpenMP threads of the per-element loops (1: serial)
};

int coupling_gen(int g, int k) { return 2 * g + k; }

}  // namespace

extern "C" {

typedef struct {
  int32_t n_bus, n_gen, n_branch, ref_bus;
  double base_mva;
  const double *pd, *qd, *gs, *bs, *vmin, *vmax;
  const int32_t* gen_bus;
  const double *pmin, *pmax, *qmin, *qmax, *c2, *c1, *c0;
  const int32_t *br_from, *br_to;
  const double *r, *x, *b, *tap, *shift, *rate;
} ora_grid;

void ora_sincos(double x, double* s, double* c) { series_sincos(x, s, c); }

// Returns nullptr on invalid input.
void* ora_create(const ora_grid* G, const ora_params* P) {
  auto* o = new Oracle();
  o->p = *P;
  o->nb = G->n_bus;
  o->ng = G->n_gen;
  o->nl = G->n_branch;
  o->ref = G->ref_bus;
  o->base = G->base_mva;
  o->m = 2 * o->ng + 8 * o->nl;
  auto cp = [](const double* s, int n) { return std::vector<double>(s, s + n); };
  o->pd = cp(G->pd, o->nb); o->qd = cp(G->qd, o->nb);
  o->gs = cp(G->gs, o->nb); o->bs = cp(G->bs, o->nb);
  o->vmin = cp(G->vmin, o->nb); o->vmax = cp(G->vmax, o->nb);
  o->gbus.assign(G->gen_bus, G->gen_bus + o->ng);
  o->pmin = cp(G->pmin, o->ng); o->pmax = cp(G->pmax, o->ng);
  o->qmin = cp(G->qmin, o->ng); o->qmax = cp(G->qmax, o->ng);
  o->c2 = cp(G->c2, o->ng); o->c1 = cp(G->c1, o->ng); o->c0 = cp(G->c0, o->ng);
  o->from.assign(G->br_from, G->br_from + o->nl);
  o->to.assign(G->br_to, G->br_to + o->nl);
  const int nl = o->nl;
  o->gii.resize(nl); o->bii.resize(nl); o->gij.resize(nl); o->bij.resize(nl);
  o->gji.resize(nl); o->bji.resize(nl); o->gjj.resize(nl); o->bjj.resize(nl);
  o->rate2.resize(nl); o->rated.resize(nl); o->rate.resize(nl);
  for (int l = 0; l < nl; ++l) {
    // series admittance y = 1/(r + jx), shunt j b/2 per end, a = tap e^{j shift}
    double r = G->r[l], xx = G->x[l];
    double den = r * r + xx * xx;
    double yr = r / den, yi = -xx / den;
    double tap = G->tap[l], sh = G->shift[l];
    double ar = tap * std::cos(sh), ai = tap * std::sin(sh);
    double a2 = tap * tap;
    // (y + j b/2)/|a|^2
    o->gii[l] = yr / a2;
    o->bii[l] = (yi + 0.5 * G->b[l]) / a2;
    // -y / conj(a) = -y a / |a|^2
    o->gij[l] = -(yr * ar - yi * ai) / a2;
    o->bij[l] = -(yr * ai + yi * ar) / a2;
    // -y / a = -y conj(a) / |a|^2
    o->gji[l] = -(yr * ar + yi * ai) / a2;
    o->bji[l] = -(yi * ar - yr * ai) / a2;
    // y + j b/2
    o->gjj[l] = yr;
    o->bjj[l] = yi + 0.5 * G->b[l];
    double rs = G->rate[l] * P->rate_scale;
    o->rated[l] = G->rate[l] > 0.0 ? 1 : 0;
    o->rate2[l] = o->rated[l] ? rs * rs : 0.0;
    o->rate[l] = G->rate[l];
  }
  o->bus_gens.assign(o->nb, {});
  o->bus_from.assign(o->nb, {});
  o->bus_to.assign(o->nb, {});
  for (int g = 0; g < o->ng; ++g) o->bus_gens[o->gbus[g]].push_back(g);
  for (int l = 0; l < nl; ++l) {
    o->bus_from[o->from[l]].push_back(l);
    o->bus_to[o->to[l]].push_back(l);
  }
  o->u.assign(o->m, 0.0); o->v.assign(o->m, 0.0); o->z.assign(o->m, 0.0);
  o->y.assign(o->m, 0.0); o->lam.assign(o->m, 0.0); o->rho.assign(o->m, 0.0);
  o->vprev.assign(o->m, 0.0);
  for (int g = 0; g < o->ng; ++g) {
    o->rho[2 * g] = P->rho_pq;
    o->rho[2 * g + 1] = P->rho_pq;
  }
  for (int l = 0; l < nl; ++l) {
    int b0 = 2 * o->ng + 8 * l;
    for (int k = 0; k < 4; ++k) o->rho[b0 + k] = P->rho_pq;
    for (int k = 4; k < 8; ++k) o->rho[b0 + k] = P->rho_va;
  }
  o->bx.assign(6 * nl, 0.0);
  o->ltil.assign(2 * nl, 0.0);
  o->rtil.assign(nl, P->al_rho0);
  o->calpha.assign(nl, 1.0);
  return o;
}

void ora_destroy(void* h) { delete static_cast<Oracle*>(h); }

static void fill_branch_data(const Oracle* o, int l, BranchData& d) {
  d.gii = o->gii[l]; d.bii = o->bii[l]; d.gij = o->gij[l]; d.bij = o->bij[l];
  d.gji = o->gji[l]; d.bji = o->bji[l]; d.gjj = o->gjj[l]; d.bjj = o->bjj[l];
  int i = o->from[l], j = o->to[l];
  d.lo[0] = o->vmin[i]; d.hi[0] = o->vmax[i];
  d.lo[1] = o->vmin[j]; d.hi[1] = o->vmax[j];
  d.lo[2] = -TWO_PI; d.hi[2] = TWO_PI;
  d.lo[3] = -TWO_PI; d.hi[3] = TWO_PI;
  d.lo[4] = -o->rate2[l]; d.hi[4] = 0.0;
  d.lo[5] = -o->rate2[l]; d.hi[5] = 0.0;
  d.n = o->rated[l] ? 6 : 4;
  int b0 = 2 * o->ng + 8 * l;
  for (int k = 0; k < 8; ++k) {
    d.vb[k] = o->v[b0 + k];
    d.z[k] = o->z[b0 + k];
    d.cv[k] = d.vb[k] - d.z[k];
    d.y[k] = o->y[b0 + k];
    d.rho[k] = o->rho[b0 + k];
  }
  d.ltil[0] = o->ltil[2 * l];
  d.ltil[1] = o->ltil[2 * l + 1];
  d.rtil = o->rtil[l];
}

// Cold start (Sec. IV-B): p, q, v at the midpoints of their bounds, angles
// zero, flows from the initial voltages; bus copies equal the component
// values; z = y = lambda = 0; beta = beta0.
void ora_cold_init(void* h) {
  auto* o = static_cast<Oracle*>(h);
  for (int g = 0; g < o->ng; ++g) {
    o->u[2 * g] = 0.5 * (o->pmin[g] + o->pmax[g]);
    o->u[2 * g + 1] = 0.5 * (o->qmin[g] + o->qmax[g]);
  }
  for (int l = 0; l < o->nl; ++l) {
    int i = o->from[l], j = o->to[l];
    double* x = &o->bx[6 * l];
    x[0] = 0.5 * (o->vmin[i] + o->vmax[i]);
    x[1] = 0.5 * (o->vmin[j] + o->vmax[j]);
    x[2] = 0.0;
    x[3] = 0.0;
    BranchData d;
    fill_branch_data(o, l, d);
    double a[8];
    branch_values<double>(d, x, a, nullptr);
    if (o->rated[l]) {
      double f0 = -(a[0] * a[0] + a[1] * a[1]);
      double f1 = -(a[2] * a[2] + a[3] * a[3]);
      x[4] = f0 < -o->rate2[l] ? -o->rate2[l] : (f0 > 0.0 ? 0.0 : f0);
      x[5] = f1 < -o->rate2[l] ? -o->rate2[l] : (f1 > 0.0 ? 0.0 : f1);
    } else {
      x[4] = 0.0;
      x[5] = 0.0;
    }
    int b0 = 2 * o->ng + 8 * l;
    for (int k = 0; k < 8; ++k) o->u[b0 + k] = a[k];
    o->ltil[2 * l] = 0.0;
    o->ltil[2 * l + 1] = 0.0;
    o->rtil[l] = o->p.al_rho0;
    o->calpha[l] = 1.0;
  }
  for (int k = 0; k < o->m; ++k) {
    o->v[k] = o->u[k];
    o->z[k] = 0.0;
    o->y[k] = 0.0;
    o->lam[k] = 0.0;
  }
  // the bus angle copies start at zero; the reference angle is zero
  o->beta = o->p.beta0;
  o->znorm_prev = INF;
  o->outer = 0;
  o->inner_total = 0;
  o->inner_in_outer = 0;
  o->status = 1;
  o->hist.clear();
}

// Generator step, eq. (qp-bound): min 1/2 Q x^2 - c x on [l, u] gives
// x = max(l, min(u, c/Q)); Q and c collect the scaled quadratic cost
// (MW based) and the coupling penalty terms.
void ora_gen_step(void* h) {
  auto* o = static_cast<Oracle*>(h);
  const double B = o->base, s = o->p.obj_scale;
#pragma omp parallel for num_threads(o->threads) if (o->threads > 1) schedule(static)
  for (int g = 0; g < o->ng; ++g) {
    int kp = 2 * g, kq = 2 * g + 1;
    double Qp = 2.0 * s * o->c2[g] * B * B + o->rho[kp];
    double cpv = o->rho[kp] * (o->v[kp] - o->z[kp]) - o->y[kp] - s * o->c1[g] * B;
    double xp = cpv / Qp;
    o->u[kp] = std::max(o->pmin[g], std::min(o->pmax[g], xp));
    double Qq = o->rho[kq];
    double cq = o->rho[kq] * (o->v[kq] - o->z[kq]) - o->y[kq];
    double xq = cq / Qq;
    o->u[kq] = std::max(o->qmin[g], std::min(o->qmax[g], xq));
  }
}

static void add_stats(ora_stats& a, const ora_stats& b) {
  a.branch_solves += b.branch_solves; a.tron_calls += b.tron_calls;
  a.tron_iters += b.tron_iters; a.n_fgh += b.n_fgh; a.n_f += b.n_f;
  a.cauchy_trials += b.cauchy_trials; a.cg_iters += b.cg_iters;
  a.chol_attempts += b.chol_attempts; a.ps_trials += b.ps_trials;
  a.al_iters += b.al_iters; a.tron_converged += b.tron_converged;
  a.tron_maxit += b.tron_maxit; a.tron_stall += b.tron_stall;
  a.flops += b.flops; a.trig += b.trig;
}

void ora_branch_step(void* h) {
  auto* o = static_cast<Oracle*>(h);
  if (o->threads > 1 && !o->count_flops) {
    // branches are independent: each thread keeps its own event counters,
    // which are integer sums (the same totals in any order)
    std::vector<ora_stats> part(o->threads, ora_stats{});
#pragma omp parallel num_threads(o->threads)
    {
#ifdef _OPENMP
      ora_stats& st = part[omp_get_thread_num()];
#else
      ora_stats& st = part[0];
#endif
#pragma omp for schedule(dynamic, 64)
      for (int l = 0; l < o->nl; ++l) {
        BranchData d;
        fill_branch_data(o, l, d);
        double* u8 = &o->u[2 * o->ng + 8 * l];
        if (o->textbook)
          tb::branch_solve(d, &o->bx[6 * l], &o->ltil[2 * l], &o->rtil[l], &o->calpha[l], u8,
                           o->p, &st);
        else
          branch_solve_t<double>(d, &o->bx[6 * l], &o->ltil[2 * l], &o->rtil[l],
                                 &o->calpha[l], u8, o->p, &st);
      }
    }
    for (const ora_stats& st : part) add_stats(o->st, st);
    return;
  }
  for (int l = 0; l < o->nl; ++l) {
    BranchData d;
    fill_branch_data(o, l, d);
    double* u8 = &o->u[2 * o->ng + 8 * l];
    if (o->textbook) {
      tb::branch_solve(d, &o->bx[6 * l], &o->ltil[2 * l], &o->rtil[l], &o->calpha[l], u8,
                       o->p, &o->st);
    } else if (o->count_flops) {
      FlopTally before = g_tally;
      branch_solve_t<CR>(d, &o->bx[6 * l], &o->ltil[2 * l], &o->rtil[l],
                         &o->calpha[l], u8, o->p, &o->st);
      o->st.flops += g_tally.total() - before.total();
      o->st.trig += g_tally.trig - before.trig;
    } else {
      branch_solve_t<double>(d, &o->bx[6 * l], &o->ltil[2 * l], &o->rtil[l],
                             &o->calpha[l], u8, o->p, &o->st);
    }
  }
}

// Bus step, eq. (qp-bus): min 1/2 x'Qx - c'x s.t. Ax = b with the two rows of
// eqs. (pg)-(qg); mu = (A Q^-1 A')^-1 (A Q^-1 c - b), x = Q^-1 (c - A' mu).
// x holds the bus copies of generator outputs, the bus copies of the flows
// leaving the bus (p_ij, q_ij on from-ends, p_ji, q_ji on to-ends) and w_i.
// The angle theta_i enters no constraint: theta = c_theta / Q_theta, and the
// reference angle is fixed at zero.
void ora_bus_step(void* h) {
  auto* o = static_cast<Oracle*>(h);
  const int ng = o->ng;
#pragma omp parallel for num_threads(o->threads) if (o->threads > 1) schedule(dynamic, 256)
  for (int i = 0; i < o->nb; ++i) {
    // variable list: index into couplings, row-P coefficient, row-Q coefficient
    std::vector<int> kidx;
    std::vector<double> aP, aQ, Qd, cv;
    for (int g : o->bus_gens[i]) {
      int kp = coupling_gen(g, 0), kq = coupling_gen(g, 1);
      kidx.push_back(kp); aP.push_back(1.0); aQ.push_back(0.0);
      kidx.push_back(kq); aP.push_back(0.0); aQ.push_back(1.0);
    }
    for (int l : o->bus_from[i]) {
      int b0 = 2 * ng + 8 * l;
      kidx.push_back(b0 + 0); aP.push_back(-1.0); aQ.push_back(0.0);
      kidx.push_back(b0 + 1); aP.push_back(0.0); aQ.push_back(-1.0);
    }
    for (int l : o->bus_to[i]) {
      int b0 = 2 * ng + 8 * l;
      kidx.push_back(b0 + 2); aP.push_back(-1.0); aQ.push_back(0.0);
      kidx.push_back(b0 + 3); aP.push_back(0.0); aQ.push_back(-1.0);
    }
    const int K = static_cast<int>(kidx.size());
    for (int t = 0; t < K; ++t) {
      int k = kidx[t];
      Qd.push_back(o->rho[k]);
      cv.push_back(o->rho[k] * (o->u[k] + o->z[k]) + o->y[k]);
    }
    // w_i: one shared variable over all w-couplings of the incident branches
    double Qw = 0.0, cw = 0.0;
    double Qt = 0.0, ct = 0.0;
    for (int l : o->bus_from[i]) {
      int kw = 2 * ng + 8 * l + 4, kt = kw + 1;
      Qw += o->rho[kw]; cw += o->rho[kw] * (o->u[kw] + o->z[kw]) + o->y[kw];
      Qt += o->rho[kt]; ct += o->rho[kt] * (o->u[kt] + o->z[kt]) + o->y[kt];
    }
    for (int l : o->bus_to[i]) {
      int kw = 2 * ng + 8 * l + 6, kt = kw + 1;
      Qw += o->rho[kw]; cw += o->rho[kw] * (o->u[kw] + o->z[kw]) + o->y[kw];
      Qt += o->rho[kt]; ct += o->rho[kt] * (o->u[kt] + o->z[kt]) + o->y[kt];
    }
    double awP = -o->gs[i], awQ = o->bs[i];
    // M = A Q^-1 A'
    double M00 = awP * awP / Qw, M01 = awP * awQ / Qw, M11 = awQ * awQ / Qw;
    // A Q^-1 c - b
    double r0 = awP * cw / Qw - o->pd[i], r1 = awQ * cw / Qw - o->qd[i];
    for (int t = 0; t < K; ++t) {
      M00 += aP[t] * aP[t] / Qd[t];
      M01 += aP[t] * aQ[t] / Qd[t];
      M11 += aQ[t] * aQ[t] / Qd[t];
      r0 += aP[t] * cv[t] / Qd[t];
      r1 += aQ[t] * cv[t] / Qd[t];
    }
    double det = M00 * M11 - M01 * M01;
    double mu0 = (M11 * r0 - M01 * r1) / det;
    double mu1 = (M00 * r1 - M01 * r0) / det;
    for (int t = 0; t < K; ++t)
      o->v[kidx[t]] = (cv[t] - aP[t] * mu0 - aQ[t] * mu1) / Qd[t];
    double w = (cw - awP * mu0 - awQ * mu1) / Qw;
    double th = (i == o->ref) ? 0.0 : ct / Qt;
    for (int l : o->bus_from[i]) {
      int kw = 2 * ng + 8 * l + 4;
      o->v[kw] = w;
      o->v[kw + 1] = th;
    }
    for (int l : o->bus_to[i]) {
      int kw = 2 * ng + 8 * l + 6;
      o->v[kw] = w;
      o->v[kw + 1] = th;
    }
  }
}

// z step, eq. (qp-bound) with (l, u) = (-inf, inf): minimizer of
// lambda z + beta/2 z^2 + y (u - v + z) + rho/2 (u - v + z)^2.
void ora_z_step(void* h) {
  auto* o = static_cast<Oracle*>(h);
#pragma omp parallel for num_threads(o->threads) if (o->threads > 1) schedule(static)
  for (int k = 0; k < o->m; ++k)
    o->z[k] = -(o->lam[k] + o->y[k] + o->rho[k] * (o->u[k] - o->v[k])) /
              (o->beta + o->rho[k]);
}

// Inner multiplier update y <- y + rho (Ax + B xbar + z) (Sec. III-B).
void ora_y_step(void* h) {
  auto* o = static_cast<Oracle*>(h);
#pragma omp parallel for num_threads(o->threads) if (o->threads > 1) schedule(static)
  for (int k = 0; k < o->m; ++k)
    o->y[k] = o->y[k] + o->rho[k] * (o->u[k] - o->v[k] + o->z[k]);
}

// Infinity norms: primal ||u - v + z||, dual ||v - v_prev||, ||z||.
void ora_residuals(void* h) {
  auto* o = static_cast<Oracle*>(h);
  double rp = 0.0, rd = 0.0, rz = 0.0;
  // maxima: the same value in any order
#pragma omp parallel for num_threads(o->threads) if (o->threads > 1) schedule(static) \
    reduction(max : rp, rd, rz)
  for (int k = 0; k < o->m; ++k) {
    rp = std::max(rp, std::fabs(o->u[k] - o->v[k] + o->z[k]));
    rd = std::max(rd, std::fabs(o->v[k] - o->vprev[k]));
    rz = std::max(rz, std::fabs(o->z[k]));
  }
  o->r_pri = rp;
  o->r_dual = rd;
  o->r_z = rz;
}

// Outer update (Algorithm 1): lambda <- proj(lambda + beta z) onto
// [-lambda_max, lambda_max]; beta grows by gamma when ||z|| did not shrink by
// the factor omega since the previous outer update.
void ora_outer_step(void* h) {
  auto* o = static_cast<Oracle*>(h);
  for (int k = 0; k < o->m; ++k) {
    double t = o->lam[k] + o->beta * o->z[k];
    o->lam[k] = std::max(-o->p.lambda_max, std::min(o->p.lambda_max, t));
  }
  if (o->r_z > o->p.beta_omega * o->znorm_prev)
    o->beta = std::min(o->p.beta_gamma * o->beta, o->p.beta_max);
  o->znorm_prev = o->r_z;
  o->outer += 1;
  o->inner_in_outer = 0;
}

// Solution quality, Sec. IV-A: the ADMM solution is the generator outputs of
// the generator problems and w_i, theta_i of the bus problems (taken from the
// bus's first branch end: from-ends, then to-ends, in input order); the flows
// are recomputed from w, theta with eqs. (pij)-(qji), w^R = v_i v_j cos,
// w^I = v_i v_j sin, v = sqrt(w). out6 receives ||c(x)||_inf over eq. acopf
// and its parts: max |residual of (pg)|, of (qg), max excess of the line
// limits (ij-limit)-(ji-limit) on the unscaled rating, of the voltage limits
// (v = sqrt(w) within [vmin, vmax]) and of |theta| <= 2 pi. Generator
// outputs are within their bounds by construction (projection).
// maximum that keeps a NaN once one appears, so that a broken state shows
static inline double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

// The solution itself: bus w, theta and the recomputed flows.
struct Recovered {
  std::vector<double> bw, bt, pij, qij, pji, qji;
};

static void recover(const Oracle* o, Recovered& R) {
  const int ng = o->ng;
  R.bw.resize(o->nb);
  R.bt.resize(o->nb);
  for (int i = 0; i < o->nb; ++i) {
    const int k = !o->bus_from[i].empty() ? 2 * ng + 8 * o->bus_from[i][0] + 4
                                          : 2 * ng + 8 * o->bus_to[i][0] + 6;
    R.bw[i] = o->v[k];
    R.bt[i] = o->v[k + 1];
  }
  R.pij.resize(o->nl);
  R.qij.resize(o->nl);
  R.pji.resize(o->nl);
  R.qji.resize(o->nl);
  for (int l = 0; l < o->nl; ++l) {
    const int i = o->from[l], j = o->to[l];
    const double wi = R.bw[i], wj = R.bw[j];
    double sn, cs;
    series_sincos(R.bt[i] - R.bt[j], &sn, &cs);
    const double vv = std::sqrt(wi) * std::sqrt(wj);
    const double WR = vv * cs, WI = vv * sn;
    R.pij[l] = std::fma(o->bij[l], WI, std::fma(o->gij[l], WR, o->gii[l] * wi));
    R.qij[l] = std::fma(o->gij[l], WI, std::fma(-o->bij[l], WR, -o->bii[l] * wi));
    R.pji[l] = std::fma(-o->bji[l], WI, std::fma(o->gji[l], WR, o->gjj[l] * wj));
    R.qji[l] = std::fma(-o->gji[l], WI, std::fma(-o->bji[l], WR, -o->bjj[l] * wj));
  }
}

// out[2 ng + 2 nb + 4 nl]: p_g, q_g, |V| = sqrt(w), theta, p_ij, q_ij, p_ji,
// q_ji (input order).
void ora_solution(void* h, double* out) {
  auto* o = static_cast<Oracle*>(h);
  Recovered R;
  recover(o, R);
  double* p = out;
  for (int g = 0; g < o->ng; ++g) p[g] = o->u[2 * g];
  p += o->ng;
  for (int g = 0; g < o->ng; ++g) p[g] = o->u[2 * g + 1];
  p += o->ng;
  for (int i = 0; i < o->nb; ++i) p[i] = R.bw[i] > 0.0 ? std::sqrt(R.bw[i]) : 0.0;
  p += o->nb;
  for (int i = 0; i < o->nb; ++i) p[i] = R.bt[i];
  p += o->nb;
  const std::vector<double>* fl[4] = {&R.pij, &R.qij, &R.pji, &R.qji};
  for (int k = 0; k < 4; ++k, p += o->nl)
    for (int l = 0; l < o->nl; ++l) p[l] = (*fl[k])[l];
}

void ora_quality(void* h, double* out6) {
  auto* o = static_cast<Oracle*>(h);
  Recovered R;
  recover(o, R);
  const std::vector<double>&bw = R.bw, &bt = R.bt, &pij = R.pij, &qij = R.qij, &pji = R.pji,
                           &qji = R.qji;
  double line = 0.0;
  for (int l = 0; l < o->nl; ++l) {
    if (o->rate[l] > 0.0) {
      const double sf = std::sqrt(std::fma(pij[l], pij[l], qij[l] * qij[l]));
      const double st = std::sqrt(std::fma(pji[l], pji[l], qji[l] * qji[l]));
      line = nanmax(line, nanmax(sf - o->rate[l], st - o->rate[l]));
    }
  }
  double balp = 0.0, balq = 0.0, volt = 0.0, ang = 0.0;
  for (int i = 0; i < o->nb; ++i) {
    double sp = 0.0, sq = 0.0;
    for (int g : o->bus_gens[i]) {
      sp = sp + o->u[2 * g];
      sq = sq + o->u[2 * g + 1];
    }
    sp = std::fma(-o->gs[i], bw[i], sp - o->pd[i]);
    sq = std::fma(o->bs[i], bw[i], sq - o->qd[i]);
    for (int l : o->bus_from[i]) {
      sp = sp - pij[l];
      sq = sq - qij[l];
    }
    for (int l : o->bus_to[i]) {
      sp = sp - pji[l];
      sq = sq - qji[l];
    }
    balp = nanmax(balp, std::fabs(sp));
    balq = nanmax(balq, std::fabs(sq));
    const double vm = bw[i] > 0.0 ? std::sqrt(bw[i]) : 0.0;
    volt = nanmax(volt, nanmax(o->vmin[i] - vm, vm - o->vmax[i]));
    ang = nanmax(ang, std::fabs(bt[i]) - TWO_PI);
  }
  out6[1] = balp;
  out6[2] = balq;
  out6[3] = line;
  out6[4] = volt;
  out6[5] = ang;
  out6[0] = nanmax(nanmax(nanmax(balp, balq), nanmax(line, volt)), ang);
}

double ora_objective(void* h) {
  auto* o = static_cast<Oracle*>(h);
  double f = 0.0;
  for (int g = 0; g < o->ng; ++g) {
    double P = o->base * o->u[2 * g];
    f += o->c2[g] * P * P + o->c1[g] * P + o->c0[g];
  }
  return f;
}

// One inner iteration of Algorithm 1 plus its control. Returns 1 when the
// whole solve has terminated (never in fixed-iteration mode).
int ora_iterate(void* h, int fixed) {
  auto* o = static_cast<Oracle*>(h);
  o->vprev = o->v;
  ora_gen_step(h);
  ora_branch_step(h);
  ora_bus_step(h);
  ora_z_step(h);
  ora_y_step(h);
  ora_residuals(h);
  o->inner_total += 1;
  o->inner_in_outer += 1;
  double obj = ora_objective(h);
  o->hist.push_back(o->r_pri);
  o->hist.push_back(o->r_dual);
  o->hist.push_back(o->r_z);
  o->hist.push_back(obj);
  o->hist.push_back(o->beta);
  o->hist.push_back(static_cast<double>(o->outer));
  bool inner_ok = o->r_pri <= o->p.eps_pri && o->r_dual <= o->p.eps_dual;
  if (!fixed && inner_ok && o->r_z <= o->p.eps_z) {
    o->status = 0;
    return 1;
  }
  if (inner_ok || o->inner_in_outer >= o->p.max_inner) {
    ora_outer_step(h);
    if (!fixed && o->outer >= o->p.max_outer) {
      o->status = 1;
      return 1;
    }
  }
  return 0;
}

// Warm start (Sec. IV-C): new loads, all primal and dual state kept; beta,
// the outer counter and the ||z|| history restart.
void ora_update_loads(void* h, const double* pd, const double* qd) {
  auto* o = static_cast<Oracle*>(h);
  for (int i = 0; i < o->nb; ++i) {
    o->pd[i] = pd[i];
    o->qd[i] = qd[i];
  }
}

// New real-power bounds of the generators (tracking with ramp limits,
// Sec. IV-C); the generator step projects onto them.
void ora_update_gen_bounds(void* h, const double* pmin, const double* pmax) {
  auto* o = static_cast<Oracle*>(h);
  for (int g = 0; g < o->ng; ++g) {
    o->pmin[g] = pmin[g];
    o->pmax[g] = pmax[g];
  }
}

void ora_warm_reset(void* h) {
  auto* o = static_cast<Oracle*>(h);
  o->beta = o->p.beta0;
  o->znorm_prev = INF;
  o->outer = 0;
  o->inner_in_outer = 0;
  o->inner_total = 0;
  o->status = 1;
  o->hist.clear();
}

// Runs Algorithm 1: fixed > 0 runs exactly that many inner iterations.
int ora_solve(void* h, int fixed) {
  auto* o = static_cast<Oracle*>(h);
  if (fixed > 0) {
    for (int t = 0; t < fixed; ++t) ora_iterate(h, 1);
    o->status = 1;
    return o->inner_total;
  }
  const long long cap = static_cast<long long>(o->p.max_outer) * o->p.max_inner;
  for (long long t = 0; t < cap; ++t)
    if (ora_iterate(h, 0)) break;
  return o->inner_total;
}

// --- state access (copies) -------------------------------------------------
// what: 0 u, 1 v, 2 z, 3 y, 4 lam, 5 rho, 6 bx (6 nl), 7 ltil (2 nl),
// 8 rtil (nl), 9 vprev, 10 pd, 11 qd, 12 calpha (nl)
static std::vector<double>* pick(Oracle* o, int what) {
  switch (what) {
    case 0: return &o->u;
    case 1: return &o->v;
    case 2: return &o->z;
    case 3: return &o->y;
    case 4: return &o->lam;
    case 5: return &o->rho;
    case 6: return &o->bx;
    case 7: return &o->ltil;
    case 8: return &o->rtil;
    case 9: return &o->vprev;
    case 10: return &o->pd;
    case 11: return &o->qd;
    case 12: return &o->calpha;
    default: return nullptr;
  }
}

int ora_get(void* h, int what, double* out, int64_t n) {
  auto* v = pick(static_cast<Oracle*>(h), what);
  if (!v || static_cast<int64_t>(v->size()) != n) return -1;
  std::memcpy(out, v->data(), sizeof(double) * n);
  return 0;
}

int ora_set(void* h, int what, const double* in, int64_t n) {
  auto* v = pick(static_cast<Oracle*>(h), what);
  if (!v || static_cast<int64_t>(v->size()) != n) return -1;
  std::memcpy(v->data(), in, sizeof(double) * n);
  return 0;
}

// scalars: [beta, znorm_prev, r_pri, r_dual, r_z, outer, inner_total,
// inner_in_outer, status]
void ora_get_scalars(void* h, double* out9) {
  auto* o = static_cast<Oracle*>(h);
  out9[0] = o->beta; out9[1] = o->znorm_prev; out9[2] = o->r_pri;
  out9[3] = o->r_dual; out9[4] = o->r_z; out9[5] = o->outer;
  out9[6] = o->inner_total; out9[7] = o->inner_in_outer; out9[8] = o->status;
}

void ora_set_scalars(void* h, const double* in9) {
  auto* o = static_cast<Oracle*>(h);
  o->beta = in9[0]; o->znorm_prev = in9[1]; o->r_pri = in9[2];
  o->r_dual = in9[3]; o->r_z = in9[4];
  o->outer = static_cast<int>(in9[5]);
  o->inner_total = static_cast<int>(in9[6]);
  o->inner_in_outer = static_cast<int>(in9[7]);
  o->status = static_cast<int>(in9[8]);
}

int64_t ora_hist_len(void* h) {
  return static_cast<int64_t>(static_cast<Oracle*>(h)->hist.size());
}

void ora_get_hist(void* h, double* out) {
  auto* o = static_cast<Oracle*>(h);
  std::memcpy(out, o->hist.data(), sizeof(double) * o->hist.size());
}

void ora_get_admittance(void* h, double* out9nl) {
  auto* o = static_cast<Oracle*>(h);
  for (int l = 0; l < o->nl; ++l) {
    double* t = out9nl + 9 * l;
    t[0] = o->gii[l]; t[1] = o->bii[l]; t[2] = o->gij[l]; t[3] = o->bij[l];
    t[4] = o->gji[l]; t[5] = o->bji[l]; t[6] = o->gjj[l]; t[7] = o->bjj[l];
    t[8] = o->rate2[l];
  }
}

void ora_get_stats(void* h, ora_stats* out) { *out = static_cast<Oracle*>(h)->st; }
void ora_reset_stats(void* h) { static_cast<Oracle*>(h)->st = ora_stats{}; }
void ora_set_count_flops(void* h, int on) { static_cast<Oracle*>(h)->count_flops = on != 0; }
// Threads of the per-element loops (generators, branches, buses, couplings);
// 1 runs them serially. Results do not depend on it: the elements are
// independent and the only reductions are maxima and integer counts.
void ora_set_threads(void* h, int n) { static_cast<Oracle*>(h)->threads = n < 1 ? 1 : n; }

// Branch solves of the whole-grid iteration by the textbook path (on != 0) or
// by the fixed-sequence path (0, the default).
void ora_set_textbook(void* h, int on) { static_cast<Oracle*>(h)->textbook = on != 0; }

// --- single-branch entry points for tests ----------------------------------
// data layout (doubles): [gii bii gij bij gji bji gjj bjj, lo[6], hi[6],
// vb[8], z[8], y[8], rho[8]] ; n = 4 or 6
static void unpack_branch(const double* in, int n, BranchData& d) {
  d.gii = in[0]; d.bii = in[1]; d.gij = in[2]; d.bij = in[3];
  d.gji = in[4]; d.bji = in[5]; d.gjj = in[6]; d.bjj = in[7];
  for (int i = 0; i < 6; ++i) { d.lo[i] = in[8 + i]; d.hi[i] = in[14 + i]; }
  for (int k = 0; k < 8; ++k) {
    d.vb[k] = in[20 + k];
    d.z[k] = in[28 + k];
    d.cv[k] = d.vb[k] - d.z[k];
    d.y[k] = in[36 + k];
    d.rho[k] = in[44 + k];
  }
  d.n = n;
}

// f, g (n), H (n*n) of the branch objective at x with multipliers ltil, rtil.
void ora_branch_eval(const double* data, int n, const double* ltil,
                     double rtil, const double* x, double* f, double* g,
                     double* H, double* a8) {
  BranchData d;
  unpack_branch(data, n, d);
  d.ltil[0] = ltil[0];
  d.ltil[1] = ltil[1];
  d.rtil = rtil;
  BranchProblem<double> P(d);
  double F;
  P.fgh(x, F, g, H);
  *f = F;
  if (a8) branch_values<double>(d, x, a8, nullptr);
}

// The same two entry points on the textbook path.
void ora_branch_eval_textbook(const double* data, int n, const double* ltil, double rtil,
                              const double* x, double* f, double* g, double* H, double* a8) {
  BranchData d;
  unpack_branch(data, n, d);
  d.ltil[0] = ltil[0];
  d.ltil[1] = ltil[1];
  d.rtil = rtil;
  *f = tb::branch_fgh(d, x, g, H);
  if (a8) {
    tb::Quantity Q[8];
    tb::quantities(d, x, Q);
    for (int k = 0; k < 8; ++k) a8[k] = Q[k].a;
  }
}

void ora_branch_solve_textbook(const double* data, int n, double* x6, double* ltil,
                               double* rtil, double* alpha, double* u8, const ora_params* P,
                               ora_stats* st) {
  BranchData d;
  unpack_branch(data, n, d);
  tb::branch_solve(d, x6, ltil, rtil, alpha, u8, *P, st);
}

void ora_branch_solve(const double* data, int n, double* x6, double* ltil,
                      double* rtil, double* alpha, double* u8, const ora_params* P,
                      ora_stats* st, int count) {
  BranchData d;
  unpack_branch(data, n, d);
  d.ltil[0] = ltil[0];
  d.ltil[1] = ltil[1];
  d.rtil = *rtil;
  if (count) {
    FlopTally before = g_tally;
    branch_solve_t<CR>(d, x6, ltil, rtil, alpha, u8, *P, st);
    st->flops += g_tally.total() - before.total();
    st->trig += g_tally.trig - before.trig;
  } else {
    branch_solve_t<double>(d, x6, ltil, rtil, alpha, u8, *P, st);
  }
}

// Generic bound-constrained TRON through callbacks (tests on quadratics,
// Rosenbrock and other closed-form problems).
typedef double (*ora_f_cb)(const double* x, void* ctx);
typedef void (*ora_fgh_cb)(const double* x, double* f, double* g, double* H,
                           void* ctx);

struct CbProblem {
  ora_f_cb fcb;
  ora_fgh_cb gcb;
  void* ctx;
  double f(const double* x) { return fcb(x, ctx); }
  void fgh(const double* x, double& F, double* g, double* H) { gcb(x, &F, g, H, ctx); }
};

// Building blocks of the trust-region method, for the CPU tests: the L E L'
// factorization (returns 1, or 0 at a non-positive pivot), the solve with it,
// and the quadratic model q(s) = g's + s'Hs/2. Matrices are dense row-major
// n x n (1 <= n <= 8).
int ora_ldlt(int n, const double* A, double* L, double* rd) {
  if (n < 1 || n > NMAX) return -1;
  return ldlt<double>(n, A, L, rd) ? 1 : 0;
}

int ora_ldlt_solve(int n, const double* L, const double* rd, const double* r, double* z) {
  if (n < 1 || n > NMAX) return -1;
  precond<double>(n, L, rd, r, z);
  return 0;
}

double ora_model(int n, const double* g, const double* H, const double* s) {
  return model_q<double>(n, g, H, s);
}

// The textbook path's Cholesky factor (returns 1, or 0 at a non-positive
// pivot) and its preconditioner z = D L'^-1 L^-1 D r.
int ora_chol_textbook(int n, const double* A, double* L) {
  if (n < 1 || n > NMAX) return -1;
  return tb::cholesky(n, A, L) ? 1 : 0;
}

int ora_precond_textbook(int n, const double* L, const double* D, const double* r, double* z) {
  if (n < 1 || n > NMAX) return -1;
  tb::precondition(n, L, D, r, z);
  return 0;
}

int ora_tron(int n, double* x, const double* lo, const double* hi,
             ora_f_cb fcb, ora_fgh_cb gcb, void* ctx, const ora_params* P,
             ora_stats* st) {
  if (n < 1 || n > NMAX) return -1;
  CbProblem prob{fcb, gcb, ctx};
  TronConst C;
  double alpha = 1.0;
  return tron<double>(prob, n, x, lo, hi, *P, st, C, &alpha);
}

int ora_tron_textbook(int n, double* x, const double* lo, const double* hi, ora_f_cb fcb,
                      ora_fgh_cb gcb, void* ctx, const ora_params* P, ora_stats* st) {
  if (n < 1 || n > NMAX) return -1;
  CbProblem prob{fcb, gcb, ctx};
  TronConst C;
  double alpha = 1.0;
  return tb::tron(prob, n, x, lo, hi, *P, st, C, &alpha);
}

}  // extern "C"
