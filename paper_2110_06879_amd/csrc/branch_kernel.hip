// Branch x-step of the component ADMM on gfx950: every branch subproblem
// (eq. branch, Sec. II-C) solved by a trust-region Newton method (Lin & More
// 1999) inside an augmented-Lagrangian loop on the line limits, all in FP64.
//
// Launch layout: one lane per branch solve, 64 per wavefront. The whole
// solve state of a branch (x, gradient, Hessian, Cholesky factor, trust
// region) lives in that lane's registers; the variable count N (4 for
// unlimited lines, 6 for rated lines with the two slacks) is a template
// constant so every small dense loop unrolls into register code. Rated and
// unlimited branches sit in separate contiguous ranges, so a wavefront never
// mixes the two shapes; a lane of the unlimited range may solve several
// branches one after another, so that every branch wavefront is resident on
// the device from the start. Branch data are structure-of-arrays (lane l
// reads element l); the values of a branch's eight couplings (v - z and y)
// come as one 128-byte record per branch that the bus step writes in branch
// order, and only the coupling values u go back to the bus-major vectors.
//
// Besides x and the AL multipliers and penalty, a branch keeps the Cauchy
// step length of its trust-region solves between ADMM iterations: a solve
// starts its projected search from the length the branch's previous solve
// ended with (1 after a cold start) rather than from 1, which halves the
// Cauchy trials once the iterates settle.
//
// Arithmetic is a fixed IEEE operation sequence that the CPU oracle follows
// too: no implicit contraction, fused multiply-adds written out where the
// oracle writes them, a square-root-free Cholesky factor with reciprocal
// pivots, norm tests in squares, and a series sin/cos. The oracle's textbook
// evaluation of the same subproblem (the terms of eq. (branch) one by one,
// Lin & More's scaled Cholesky, libm sin/cos) pins each of these transforms.
//
// The free set of a subspace step is handled with a mask over all N
// variables instead of compressed indices (fixed rows and columns act as
// identity), which keeps indexing static; the nonzero arithmetic is the same
// as on the compressed system. A pass in which every variable is free runs
// an instantiation without the mask.
//
// The heavy solves run alone in their wavefront at the end of a launch, one
// wavefront per SIMD, so a lane's time is its instruction count: values the
// lane already holds are not formed again (the model value at the current
// point, the coupling values of an accepted trial point, g's in the Cauchy
// test), with the flops counted as the algorithm performs them.
//
// Each lane can also count the algorithmic flops of the method as the plain
// serial algorithm performs them (+ - * / sqrt one each, sin and cos apart),
// step by step, so that achieved FP64 throughput can be reported exactly;
// the counter type is a template parameter, and the default kernels carry
// counters that do nothing.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "device_common.h"

namespace acopf_dev {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Trust-region constants (Lin & More 1999, Sec. 2-4 and the choices of the
// branch solver): acceptance and radius thresholds, Cauchy search factors,
// projected-search backtracking, CG tolerance, Cholesky shift.
constexpr double kEta0 = 1e-4, kEta1 = 0.25, kEta2 = 0.75;
constexpr double kSig1 = 0.25, kSig2 = 0.5, kSig3 = 4.0;
constexpr double kMu0 = 0.01, kInterp = 0.1, kExtrap = 10.0;
constexpr int kMaxTrials = 20;
constexpr double kCgTol = 0.1;
constexpr double kShiftMin = 1e-3;
constexpr int kMaxChol = 20;

// A counter that counts nothing: the uncounted kernels use it in place of
// uint32_t, so that no counting arithmetic is left in their code.
struct NoTally {
  __device__ NoTally& operator+=(uint32_t) { return *this; }
  __device__ NoTally& operator++() { return *this; }
  __device__ NoTally& operator=(uint32_t) { return *this; }
  __device__ operator uint32_t() const { return 0u; }
};

// Per-lane event and flop counters; CountersT<false> holds NoTally members.
template <bool kOn>
struct CountersT {
  using T = typename std::conditional<kOn, uint32_t, NoTally>::type;
  T flops, trig;  // per branch solve: far below 2^32
  T tron_calls, tron_iters, n_fgh, n_f, cauchy, cg, chol, ps, al, conv, maxit, stall;
};

#define FL(n) (cnt.flops += (uint32_t)(n))

// Symmetric N x N matrix, or a lower-triangular factor, in packed lower
// storage; (i, j) and (j, i) name the same element. Indices are compile-time
// constants after unrolling, so the storage stays in registers.
template <int N>
struct Sym {
  double t[N * (N + 1) / 2];
  __device__ static constexpr int idx(int i, int j) {
    return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
  }
  __device__ double& operator()(int i, int j) { return t[idx(i, j)]; }
  __device__ double operator()(int i, int j) const { return t[idx(i, j)]; }
};

template <int N>
struct BranchIn {
  double gii, bii, gij, bij, gji, bji, gjj, bjj;
  double cv[8], yc[8];  // per coupling: target v_k - z_k and multiplier y_k
  double rpq, rva;
  double lt0, lt1, rt;
  __device__ double rho(int k) const { return k < 4 ? rpq : rva; }
};

// sin and cos of an angle difference as a fixed sequence of IEEE operations
// (the library is built without floating-point contraction; every fused
// multiply-add is written out): reduction by pi/2 with a two-part constant
// (33-bit head), then the Taylor series of sin and cos on |r| <= pi/4 in
// Horner form with fused multiply-adds, truncated after r^17 and r^18
// (truncation error below 1e-19 there).
__device__ inline void series_sincos(double x, double* s, double* c) {
  constexpr double kHead = 1.5707963267341256;      // 0x1.921fb544p+0
  constexpr double kTail = 6.077100506506192e-11;   // pi/2 - kHead
  constexpr double kInvPio2 = 0.6366197723675814;   // 2/pi
  const double k = rint(x * kInvPio2);
  const double r = fma(-k, kTail, fma(-k, kHead, x));
  const double r2 = r * r;
  // odd coefficients (-1)^j/(2j+1)!, even coefficients (-1)^j/(2j)!
  double ps = 2.8114572543455206e-15;
  ps = fma(r2, ps, -7.647163731819816e-13);
  ps = fma(r2, ps, 1.6059043836821613e-10);
  ps = fma(r2, ps, -2.505210838544172e-08);
  ps = fma(r2, ps, 2.7557319223985893e-06);
  ps = fma(r2, ps, -0.0001984126984126984);
  ps = fma(r2, ps, 0.008333333333333333);
  ps = fma(r2, ps, -0.16666666666666666);
  double pc = -1.5619206968586225e-16;
  pc = fma(r2, pc, 4.779477332387385e-14);
  pc = fma(r2, pc, -1.1470745597729725e-11);
  pc = fma(r2, pc, 2.08767569878681e-09);
  pc = fma(r2, pc, -2.755731922398589e-07);
  pc = fma(r2, pc, 2.48015873015873e-05);
  pc = fma(r2, pc, -0.001388888888888889);
  pc = fma(r2, pc, 0.041666666666666664);
  pc = fma(r2, pc, -0.5);
  const double sr = fma(r, r2 * ps, r);
  const double cr = fma(r2, pc, 1.0);
  const int q = (int)(((long long)k) & 3);
  const double sv[4] = {sr, cr, -sr, -cr};
  const double cv[4] = {cr, -sr, -cr, sr};
  *s = q == 0 ? sv[0] : q == 1 ? sv[1] : q == 2 ? sv[2] : sv[3];
  *c = q == 0 ? cv[0] : q == 1 ? cv[1] : q == 2 ? cv[2] : cv[3];
}

// Projection onto [lo, hi] (lo <= hi) as max then min: two instructions.
// A NaN t gives lo, as in the oracle.
__device__ inline double clampd(double t, double lo, double hi) {
  return fmin(fmax(t, lo), hi);
}

// Flows and coupling values a_k(x); aux = (cos, sin, w^R, w^I).
template <int N, class Cnt>
__device__ inline void values(const BranchIn<N>& B, const double* x, double* a,
                              double* aux, Cnt& cnt) {
  const double vi = x[0], vj = x[1], ti = x[2], tj = x[3];
  const double dt = ti - tj;
  double sn, cs;
  series_sincos(dt, &sn, &cs);
  const double vv = vi * vj;
  const double WR = vv * cs, WI = vv * sn;
  const double wi = vi * vi, wj = vj * vj;
  a[0] = fma(B.bij, WI, fma(B.gij, WR, B.gii * wi));
  a[1] = fma(B.gij, WI, fma(-B.bij, WR, -B.bii * wi));
  a[2] = fma(-B.bji, WI, fma(B.gji, WR, B.gjj * wj));
  a[3] = fma(-B.gji, WI, fma(-B.bji, WR, -B.bjj * wj));
  a[4] = wi;
  a[5] = ti;
  a[6] = wj;
  a[7] = tj;
  aux[0] = cs;
  aux[1] = sn;
  aux[2] = WR;
  aux[3] = WI;
  FL(26);
  cnt.trig += 2;
}

// F alone; the coupling values and (cos, sin, w^R, w^I) at x are left in a
// and aux for an f/g/H evaluation at the same point.
template <int N, class Cnt>
__device__ double fval(const BranchIn<N>& B, const double* x, double* a, double* aux,
                       Cnt& cnt) {
  values<N>(B, x, a, aux, cnt);
  double F = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double r = a[k] - B.cv[k];
    F = fma(0.5 * B.rho(k) * r, r, fma(B.yc[k], r, F));
  }
  FL(56);
  if (N == 6) {
    const double c0 = fma(a[0], a[0], a[1] * a[1]) + x[4];
    F = fma(0.5 * B.rt * c0, c0, fma(B.lt0, c0, F));
    const double c1 = fma(a[2], a[2], a[3] * a[3]) + x[5];
    F = fma(0.5 * B.rt * c1, c1, fma(B.lt1, c1, F));
    FL(20);
  }
  ++cnt.n_f;
  return F;
}

// Upper-triangle enumeration of a 4x4 block.
__device__ constexpr int kUP[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
__device__ constexpr int kUQ[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};

// F, gradient and Hessian by the chain rule through the coupling values.
// m_k = y_k + rho_k r_k for every coupling and, on rated branches,
// m_e = ltil_e + rtil c_e for the line limit at end e. The flow terms are
// gathered per flow k (at end e) as mu_k = m_k + 2 m_e a_k (gradient and
// curvature weight) and nu_k = rho_k + 2 m_e (weight of grad a_k grad a_k').
// Every flow is linear in (w_own, w^R, w^I), so sum_k mu_k grad a_k and
// sum_k mu_k hess a_k reduce to MR, MI times the derivatives of w^R, w^I plus
// the w_own terms O_i, O_j. F is accumulated in the order of fval.
template <int N, class Cnt>
__device__ void fgh_at(const BranchIn<N>& B, const double* x, const double* a,
                       const double* aux, double& F, double* g, Sym<N>& H, Cnt& cnt) {
  const double vi = x[0], vj = x[1];
  const double cs = aux[0], sn = aux[1], WR = aux[2], WI = aux[3];
  const double jc = vj * cs, ic = vi * cs, js = vj * sn, is = vi * sn;
  const double twvi = 2.0 * vi, twvj = 2.0 * vj;
  const double dWR[4] = {jc, ic, -WI, WI};
  const double dWI[4] = {js, is, WR, -WR};
  const double hWR[10] = {0.0, cs, -js, js, 0.0, -is, is, -WR, WR, -WR};
  const double hWI[10] = {0.0, sn, jc, -jc, 0.0, ic, -ic, -WI, WI, -WI};
  const double cw[4] = {B.gii, -B.bii, B.gjj, -B.bjj};
  const double cR[4] = {B.gij, -B.bij, B.gji, -B.bji};
  const double cI[4] = {B.bij, B.gij, -B.bji, -B.gji};
  double ga[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int own = k < 2 ? 0 : 1;
    const double tw = k < 2 ? twvi : twvj;
#pragma unroll
    for (int p = 0; p < 4; ++p)
      ga[k][p] = p == own ? fma(cI[k], dWI[p], fma(cR[k], dWR[p], cw[k] * tw))
                          : fma(cI[k], dWI[p], cR[k] * dWR[p]);
  }
  FL(62);
  F = 0.0;
  double mu[4], nu[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double rk = B.rho(k);
    const double r = a[k] - B.cv[k];
    F = fma(0.5 * rk * r, r, fma(B.yc[k], r, F));
    mu[k] = fma(rk, r, B.yc[k]);
    nu[k] = rk;
  }
  double mv[4];  // voltage-magnitude and angle couplings: w_i, th_i, w_j, th_j
#pragma unroll
  for (int k = 4; k < 8; ++k) {
    const double rk = B.rva;
    const double r = a[k] - B.cv[k];
    F = fma(0.5 * rk * r, r, fma(B.yc[k], r, F));
    mv[k - 4] = fma(rk, r, B.yc[k]);
  }
  FL(72);
  double gc[2][4], me[2];
  if (N == 6) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int kp = 2 * e, kq = 2 * e + 1, s = 4 + e;
      const double lt = e == 0 ? B.lt0 : B.lt1;
      const double c = fma(a[kp], a[kp], a[kq] * a[kq]) + x[s];
      F = fma(0.5 * B.rt * c, c, fma(lt, c, F));
      me[e] = fma(B.rt, c, lt);
      const double tm = 2.0 * me[e];
      mu[kp] = fma(tm, a[kp], mu[kp]);
      mu[kq] = fma(tm, a[kq], mu[kq]);
      nu[kp] = nu[kp] + tm;
      nu[kq] = nu[kq] + tm;
#pragma unroll
      for (int p = 0; p < 4; ++p) gc[e][p] = 2.0 * fma(a[kp], ga[kp][p], a[kq] * ga[kq][p]);
    }
    FL(70);
  }
  const double MR = fma(mu[3], cR[3], fma(mu[2], cR[2], fma(mu[1], cR[1], mu[0] * cR[0])));
  const double MI = fma(mu[3], cI[3], fma(mu[2], cI[2], fma(mu[1], cI[1], mu[0] * cI[0])));
  const double Oi = fma(mu[1], cw[1], mu[0] * cw[0]);
  const double Oj = fma(mu[3], cw[3], mu[2] * cw[2]);
#pragma unroll
  for (int p = 0; p < 4; ++p) g[p] = fma(MI, dWI[p], MR * dWR[p]);
  g[0] = fma(2.0 * x[0], Oi, g[0]);
  g[1] = fma(2.0 * x[1], Oj, g[1]);
  double ng[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int p = 0; p < 4; ++p) ng[k][p] = nu[k] * ga[k][p];
  FL(54);
  double rg[2][4];
  if (N == 6) {
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int p = 0; p < 4; ++p) rg[e][p] = B.rt * gc[e][p];
    FL(8);
  }
#pragma unroll
  for (int t = 0; t < 10; ++t) {
    const int p = kUP[t], q = kUQ[t];
    double h;
    if (t == 0)
      h = 2.0 * Oi;
    else if (t == 4)
      h = 2.0 * Oj;
    else
      h = fma(MI, hWI[t], MR * hWR[t]);
#pragma unroll
    for (int k = 0; k < 4; ++k) h = fma(ng[k][p], ga[k][q], h);
    if (N == 6) {
#pragma unroll
      for (int e = 0; e < 2; ++e) h = fma(rg[e][p], gc[e][q], h);
    }
    H(p, q) = h;
  }
  FL(106);
  if (N == 6) {
    FL(40);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int s = 4 + e;
      g[s] = me[e];
#pragma unroll
      for (int p = 0; p < 4; ++p) H(p, s) = rg[e][p];
      H(s, s) = B.rt;
    }
    H(4, 5) = 0.0;
  }
  {
    const int var[4] = {0, 2, 1, 3};
#pragma unroll
    for (int k = 4; k < 8; ++k) {
      const int p = var[k - 4];
      const double m = mv[k - 4];
      if (k == 4 || k == 6) {
        const double gv = 2.0 * x[p];
        g[p] = fma(m, gv, g[p]);
        H(p, p) = fma(m, 2.0, fma(B.rva * gv, gv, H(p, p)));
      } else {
        g[p] = g[p] + m;
        H(p, p) = H(p, p) + B.rva;
      }
    }
    FL(20);
  }
  ++cnt.n_fgh;
}

// f/g/H at x. fgh_reuse does the same from the values an f evaluation at x
// left behind, and counts the skipped evaluation of the values, which the
// algorithm performs again.
template <int N, class Cnt>
__device__ void fgh(const BranchIn<N>& B, const double* x, double& F, double* g, Sym<N>& H,
                    Cnt& cnt) {
  double a[8], aux[4];
  values<N>(B, x, a, aux, cnt);
  fgh_at<N>(B, x, a, aux, F, g, H, cnt);
}

template <int N, class Cnt>
__device__ void fgh_reuse(const BranchIn<N>& B, const double* x, const double* a,
                          const double* aux, double& F, double* g, Sym<N>& H, Cnt& cnt) {
  FL(26);
  cnt.trig += 2;
  fgh_at<N>(B, x, a, aux, F, g, H, cnt);
}

template <int N>
__device__ inline double dotN(const double* a, const double* b) {
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) t = fma(a[i], b[i], t);
  return t;
}

// q(s) = g's + 1/2 s'Hs ; counted as 2N^2 + 4N + 2
template <int N, class Cnt>
__device__ inline double model(const double* g, const Sym<N>& H, const double* s,
                               Cnt& cnt, double* gs_out = nullptr) {
  // s'Hs = sum_i s_i (H_ii s_i + sum_{j<i} H_ij (2 s_j)): the lower triangle
  // only, doubling being exact. g's is returned in gs_out when asked for.
  double t[N];
#pragma unroll
  for (int j = 0; j < N; ++j) t[j] = 2.0 * s[j];
  double gs = 0.0, sHs = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    gs = fma(g[i], s[i], gs);
    double hi = H(i, i) * s[i];
#pragma unroll
    for (int j = 0; j < i; ++j) hi = fma(H(i, j), t[j], hi);
    sHs = fma(s[i], hi, sHs);
  }
  FL(N * N + 5 * N + 2);
  if (gs_out) *gs_out = gs;
  return fma(0.5, sHs, gs);
}

// tau >= 0 with ||a + tau p|| = delta
template <int N, class Cnt>
__device__ inline double to_boundary(const double* a, const double* p, double delta,
                                     Cnt& cnt) {
  const double ap = dotN<N>(a, p), pp = dotN<N>(p, p), aa = dotN<N>(a, a);
  double dd = delta * delta - aa;
  if (dd < 0.0) dd = 0.0;
  const double rad = ap * ap + pp * dd;
  const double sq = sqrt(rad);
  FL(6 * N + 6);
  double tau;
  if (ap >= 0.0) {
    const double den = ap + sq;
    FL(1);
    if (den > 0.0) {
      tau = dd / den;
      FL(1);
    } else {
      tau = 0.0;
    }
  } else {
    tau = (sq - ap) / pp;
    FL(2);
  }
  return tau;
}

// Cauchy-search acceptance: ||s|| <= delta and q(s) <= mu0 g's. q receives
// q(s) whenever it is evaluated (always, when the trial is accepted).
template <int N, class Cnt>
__device__ inline bool cauchy_ok(const double* g, const Sym<N>& H, const double* s,
                                 double delta, double& q, Cnt& cnt) {
  const double ss = dotN<N>(s, s);  // ||s|| <= delta, compared in squares
  FL(2 * N + 1);
  if (ss > delta * delta) return false;
  // g's is the dot product the model forms first, in the same order
  double gts;
  q = model<N>(g, H, s, cnt, &gts);
  FL(2 * N + 1);
  return q <= kMu0 * gts;
}

// The model's flops, counted where the algorithm evaluates q(s) again at a
// point whose value the kernel already holds.
template <int N, class Cnt>
__device__ inline void count_model(Cnt& cnt) {
  FL(N * N + 5 * N + 2);
}

template <int N, class Cnt>
__device__ inline void cauchy_trial(const double* x, const double* g, const double* lo,
                                    const double* hi, double a, double* w, double* s,
                                    Cnt& cnt) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    w[i] = clampd(fma(-a, g[i], x[i]), lo[i], hi[i]);
    s[i] = w[i] - x[i];
  }
  FL(3 * N);
}

template <int N, class Cnt>
__device__ void cauchy(const double* x, const double* g, const Sym<N>& H,
                       const double* lo, const double* hi, double delta,
                       double& alpha, double* w, double& qw, bool& qok, Cnt& cnt) {
  // On return qw = q(w - x) and qok is true, unless no trial was accepted.
  // The largest breakpoint of the projected path is only needed to stop an
  // extrapolation, so it is formed on that branch; the other branch counts
  // its flops all the same, as the algorithm forms it before the first trial.
  double s[N], wt[N], st[N];
  cauchy_trial<N>(x, g, lo, hi, alpha, w, s, cnt);
  ++cnt.cauchy;
  double q;
  qok = false;
  if (cauchy_ok<N>(g, H, s, delta, q, cnt)) {
    qw = q;
    qok = true;
    double brpt = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double bp = 0.0;
      if (g[i] > 0.0) {
        bp = (x[i] - lo[i]) / g[i];
        FL(2);
      } else if (g[i] < 0.0) {
        bp = (x[i] - hi[i]) / g[i];
        FL(2);
      }
      brpt = brpt < bp ? bp : brpt;
    }
    // extrapolate while the conditions hold and the path still bends
    for (int t = 0; t < kMaxTrials; ++t) {
      if (alpha > brpt) break;
      const double a2 = alpha * kExtrap;
      FL(1);
      cauchy_trial<N>(x, g, lo, hi, a2, wt, st, cnt);
      ++cnt.cauchy;
      if (!cauchy_ok<N>(g, H, st, delta, q, cnt)) break;
      alpha = a2;
      qw = q;
#pragma unroll
      for (int i = 0; i < N; ++i) w[i] = wt[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (g[i] > 0.0 || g[i] < 0.0) FL(2);
    for (int t = 0; t < kMaxTrials; ++t) {
      alpha = alpha * kInterp;
      FL(1);
      cauchy_trial<N>(x, g, lo, hi, alpha, w, s, cnt);
      ++cnt.cauchy;
      if (cauchy_ok<N>(g, H, s, delta, q, cnt)) {
        qw = q;
        qok = true;
        break;
      }
    }
  }
}

// Preconditioner application on the free variables (mask fr):
// z = L^-T E^-1 L^-1 r with L unit lower and the reciprocal pivots rd = 1/E;
// counted as 2 nf^2 - nf.
template <int N, bool kAll>
__device__ inline void precond(const Sym<N>& L, const double* rd, const bool* fr,
                               const double* r, double* z) {
  double t[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double a = r[i];
#pragma unroll
    for (int k = 0; k < i; ++k) a = fma(-L(i, k), t[k], a);
    t[i] = (kAll || fr[i]) ? a : 0.0;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) t[i] = t[i] * rd[i];
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    double a = t[i];
#pragma unroll
    for (int k = i + 1; k < N; ++k) a = fma(-L(k, i), z[k], a);
    z[i] = (kAll || fr[i]) ? a : 0.0;
  }
}

// Square-root-free Cholesky factorization L E L' (L unit lower, E diagonal)
// of the shifted free Hessian H + shift diag(Sd) (fixed rows/columns act as
// identity), formed element by element as the factorization needs it.
// Column j: v_k = L_jk e_k, pivot e_j = a_jj - sum_k L_jk v_k, and
// L_ij = (a_ij - sum_k L_ik v_k) times the reciprocal pivot, which is kept in
// rd for the solves. Returns false at the first non-positive free pivot;
// flops are counted as on the compressed nf x nf matrix.
template <int N, bool kAll, class Cnt>
__device__ inline bool ldlt(const Sym<N>& H, const double* Sd, double shift,
                            const bool* fr, int nf, Sym<N>& L, double* rd,
                            Cnt& cnt) {
#pragma unroll
  for (int q = 0; q < N * (N + 1) / 2; ++q) L.t[q] = 0.0;
  double e[N];
  int jc = 0;  // compressed column index
#pragma unroll
  for (int j = 0; j < N; ++j) {
    L(j, j) = 1.0;
    if (!(kAll || fr[j])) {
      e[j] = 1.0;
      rd[j] = 1.0;
      continue;
    }
    double v[N];
#pragma unroll
    for (int k = 0; k < j; ++k) v[k] = L(j, k) * e[k];
    double d = fma(shift, Sd[j], H(j, j));
#pragma unroll
    for (int k = 0; k < j; ++k) d = fma(-L(j, k), v[k], d);
    FL(3 * jc);
    if (!(d > 0.0)) return false;
    e[j] = d;
    const double rj = 1.0 / d;
    rd[j] = rj;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      if (!(kAll || fr[i])) continue;
      double t = H(i, j);
#pragma unroll
      for (int k = 0; k < j; ++k) t = fma(-L(i, k), v[k], t);
      L(i, j) = t * rj;
    }
    FL(1 + (nf - 1 - jc) * (2 * jc + 1));
    ++jc;
  }
  return true;
}

// Subspace steps from the Cauchy point w (in/out), Lin & More Sec. 4:
// Steihaug PCG on the free variables, projected search, repeat while a new
// bound becomes active and CG ended inside the trust region.
// One pass on the free set fr (nf free variables) at the current Cauchy or
// search point w, with s = w - x; returns true when the passes end. With
// kAll every variable is free, and the free-set tests compile away.
template <int N, bool kAll, class Cnt>
__device__ bool subspace_pass(const double* x, const double* g, const Sym<N>& H,
                              const double* lo, const double* hi, double delta, double* w,
                              double* s, const bool* fr, int nf, double& qcur, bool& qok,
                              Cnt& cnt) {
    double gq[N], r[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double t = g[i];
#pragma unroll
      for (int j = 0; j < N; ++j) t = fma(H(i, j), s[j], t);
      gq[i] = t;
      r[i] = (kAll || fr[i]) ? -t : 0.0;
    }
    FL(2 * N * N);
    const double rr0 = dotN<N>(r, r);  // squared norm of the initial residual
    FL(2 * nf);
    if (!(rr0 > 0.0)) return true;
    // Lin & More's scaled matrix D H D + shift I, D = diag(|H_ii|^(-1/2)),
    // gives the preconditioner H + shift D^-2; it is factored in that form,
    // H + shift Sd with Sd = |H_ii| (1 where H_ii = 0). The scaled diagonal
    // entries are the signs of H_ii; their minimum sets the shift.
    double Sd[N];
    double mind = 1.0 / 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double b = H(i, i);
      Sd[i] = b == 0.0 ? 1.0 : fabs(b);
      if ((kAll || fr[i])) {
        const double sgn = b > 0.0 ? 1.0 : (b < 0.0 ? -1.0 : 0.0);
        mind = sgn < mind ? sgn : mind;
      }
    }
    double shift = 0.0;
    if (!(mind > 0.0)) {
      shift = kShiftMin - mind;
      FL(1);
    }
    Sym<N> L;
    double rd[N];
    bool ok = false;
    for (int att = 0; att < kMaxChol; ++att) {
      FL(2 * nf);
      ++cnt.chol;
      if (ldlt<N, kAll>(H, Sd, shift, fr, nf, L, rd, cnt)) {
        ok = true;
        break;
      }
      shift = 2.0 * shift > kShiftMin ? 2.0 * shift : kShiftMin;
      FL(1);
    }
    if (!ok) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        rd[i] = 1.0;
#pragma unroll
        for (int j = 0; j <= i; ++j) L(i, j) = i == j ? 1.0 : 0.0;
      }
    }
    // Steihaug PCG on min 1/2 d'Bd - r'd s.t. ||s + d|| <= delta
    double d[N], res[N], zz[N], p[N], Bp[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      d[i] = 0.0;
      res[i] = r[i];
    }
    precond<N, kAll>(L, rd, fr, res, zz);
    FL(2 * nf * nf - nf);
#pragma unroll
    for (int i = 0; i < N; ++i) p[i] = zz[i];
    double rz = dotN<N>(res, zz);
    FL(2 * nf);
    bool boundary = false;
    for (int k = 0; k < nf; ++k) {
      ++cnt.cg;
      // p is exactly zero on the fixed variables, so their columns add
      // zeros and the free terms accumulate in the compressed order
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) t = fma(H(i, j), p[j], t);
        Bp[i] = (kAll || fr[i]) ? t : 0.0;
      }
      const double pBp = dotN<N>(p, Bp);
      FL(2 * nf * nf + 2 * nf);
      double sd[N];
#pragma unroll
      for (int i = 0; i < N; ++i) sd[i] = s[i] + d[i];
      FL(nf);
      if (!(pBp > 0.0)) {
        const double tau = to_boundary<N>(sd, p, delta, cnt);
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = fma(tau, p[i], d[i]);
        FL(2 * nf);
        boundary = true;
        break;
      }
      const double alpha = rz / pBp;
      double tr[N];
#pragma unroll
      for (int i = 0; i < N; ++i) tr[i] = fma(alpha, p[i], sd[i]);
      const double trr = dotN<N>(tr, tr);  // ||s + d|| >= delta, in squares
      FL(1 + 2 * N + 2 * N + 1);
      if (trr >= delta * delta) {
        const double tau = to_boundary<N>(sd, p, delta, cnt);
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = fma(tau, p[i], d[i]);
        FL(2 * nf);
        boundary = true;
        break;
      }
#pragma unroll
      for (int i = 0; i < N; ++i) {
        d[i] = fma(alpha, p[i], d[i]);
        res[i] = fma(-alpha, Bp[i], res[i]);
      }
      const double rr = dotN<N>(res, res);  // ||r|| <= tol ||r0||, in squares
      FL(4 * nf + 2 * nf + 1);
      if (rr <= (kCgTol * kCgTol) * rr0) break;
      precond<N, kAll>(L, rd, fr, res, zz);
      const double rzn = dotN<N>(res, zz);
      const double bcg = rzn / rz;
      rz = rzn;
#pragma unroll
      for (int i = 0; i < N; ++i) p[i] = (kAll || fr[i]) ? fma(bcg, p[i], zz[i]) : 0.0;
      FL(2 * nf * nf - nf + 2 * nf + 1 + 2 * nf);
    }
    // projected search along d from w
    // q(s) at the pass's start point: known when that point was accepted by
    // the Cauchy search or by the previous pass's search
    double qw;
    if (qok) {
      qw = qcur;
      count_model<N>(cnt);
    } else {
      qw = model<N>(g, H, s, cnt);
    }
    double beta = 1.0;
    bool acc = false;
    double qt_acc = 0.0;
    double wt[N], stv[N];
    for (int t = 0; t < kMaxTrials; ++t) {
      ++cnt.ps;
#pragma unroll
      for (int i = 0; i < N; ++i)
        wt[i] = (kAll || fr[i]) ? clampd(fma(beta, d[i], w[i]), lo[i], hi[i]) : w[i];
      double dw[N];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        stv[i] = wt[i] - x[i];
        dw[i] = wt[i] - w[i];
      }
      FL(2 * nf + 2 * N);
      const double qt = model<N>(g, H, stv, cnt);
      const double lhs = fma(kMu0, dotN<N>(gq, dw), qw);
      FL(2 * N + 2);
      if (qt <= lhs) {
        acc = true;
        qt_acc = qt;
        break;
      }
      beta = beta * 0.5;
      FL(1);
    }
    if (!acc) return true;
    bool hit = false;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if ((kAll || fr[i]) && (wt[i] == lo[i] || wt[i] == hi[i])) hit = true;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      w[i] = wt[i];
      s[i] = stv[i];
    }
    qcur = qt_acc;
    qok = true;
    if (boundary || !hit) return true;
    return false;
}

template <int N, class Cnt>
__device__ void subspace(const double* x, const double* g, const Sym<N>& H,
                         const double* lo, const double* hi, double delta,
                         double* w, double& qcur, bool& qok, Cnt& cnt) {
  double s[N];
#pragma unroll
  for (int i = 0; i < N; ++i) s[i] = w[i] - x[i];
  FL(N);
  for (int pass = 0; pass < N; ++pass) {
    bool fr[N];
    int nf = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      fr[i] = w[i] > lo[i] && w[i] < hi[i];
      nf += fr[i] ? 1 : 0;
    }
    if (nf == 0) break;
    const bool stop =
        nf == N ? subspace_pass<N, true>(x, g, H, lo, hi, delta, w, s, fr, nf, qcur, qok, cnt)
                : subspace_pass<N, false>(x, g, H, lo, hi, delta, w, s, fr, nf, qcur, qok, cnt);
    if (stop) break;
  }
}

enum { kConv = 0, kMaxit = 1, kStall = 2 };

template <int N, class Cnt>
__device__ int tron(const BranchIn<N>& B, double* x, const double* lo, const double* hi,
                    double gtol, double ftol, int maxit, double& alphac, Cnt& cnt) {
  ++cnt.tron_calls;
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = clampd(x[i], lo[i], hi[i]);
  double f, g[N];
  Sym<N> H;
  fgh<N>(B, x, f, g, H, cnt);
  double pg2 = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double t = clampd(x[i] - g[i], lo[i], hi[i]) - x[i];
    pg2 = fma(t, t, pg2);
  }
  double delta = sqrt(pg2);
  FL(4 * N + 1);
  if (!(delta > 0.0)) delta = 1.0;
  int status = kMaxit;
  for (int it = 0; it < maxit; ++it) {
    double pginf = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double t = fabs(clampd(x[i] - g[i], lo[i], hi[i]) - x[i]);
      pginf = fmax(pginf, t);  // t >= 0 or NaN; a NaN t leaves pginf, as comparing does
    }
    FL(2 * N);
    if (pginf <= gtol) {
      status = kConv;
      break;
    }
    ++cnt.tron_iters;
    double w[N], s[N];
    double qcur = 0.0;
    bool qok = false;
    cauchy<N>(x, g, H, lo, hi, delta, alphac, w, qcur, qok, cnt);
    subspace<N>(x, g, H, lo, hi, delta, w, qcur, qok, cnt);
#pragma unroll
    for (int i = 0; i < N; ++i) s[i] = w[i] - x[i];
    FL(N);
    double qs;
    if (qok) {
      qs = qcur;
      count_model<N>(cnt);
    } else {
      qs = model<N>(g, H, s, cnt);
    }
    const double prered = -qs;
    const double snorm = sqrt(dotN<N>(s, s));
    FL(2 * N + 1);
    if (!(prered > 0.0)) {
      status = kStall;
      break;
    }
    if (snorm < delta) {
      FL(2);
      if (prered <= ftol * (1.0 + fabs(f))) {
#pragma unroll
        for (int i = 0; i < N; ++i) x[i] = w[i];
        status = kConv;
        break;
      }
    }
    double aw[8], auxw[4];
    const double fw = fval<N>(B, w, aw, auxw, cnt);
    const double actred = f - fw;
    const double ratio = actred / prered;
    FL(2);
    if (ratio <= kEta0) {
      delta = kSig2 * (snorm < delta ? snorm : delta);
      FL(1);
    } else if (ratio <= kEta1) {
      const double a = kSig1 * delta, b = kSig2 * (snorm < delta ? snorm : delta);
      delta = a < b ? b : a;
      FL(2);
    } else if (ratio >= kEta2) {
      const double a = kSig3 * delta, b0 = kSig3 * snorm;
      const double b = delta < b0 ? b0 : delta;
      delta = b < a ? b : a;
      FL(2);
    }
    if (ratio > kEta0) {
#pragma unroll
      for (int i = 0; i < N; ++i) x[i] = w[i];
      fgh_reuse<N>(B, x, aw, auxw, f, g, H, cnt);
    }
    const double xx = dotN<N>(x, x);  // delta <= 1e-15 max(1, ||x||), in squares
    FL(2 * N + 2);
    if (delta * delta <= 1e-30 * (xx > 1.0 ? xx : 1.0)) {
      status = kStall;
      break;
    }
  }
  if (status == kConv) ++cnt.conv;
  else if (status == kMaxit) ++cnt.maxit;
  else ++cnt.stall;
  return status;
}

// ---------------------------------------------------------------------------
// Resumable TRON for the persistent x-step: the same iteration, split so a
// lane can advance its solve by one iteration per trip of a loop that all
// lanes of the wavefront share. tron_begin + repeated tron_advance performs
// exactly the operations of tron() in the same order.
// ---------------------------------------------------------------------------
template <int N>
struct TronState {
  double x[N];
  double f, g[N];
  Sym<N> H;
  double delta, alphac;
  int it, status;
  bool eval, first;
};

template <int N, class Cnt>
__device__ inline void tron_begin(TronState<N>& S, const double* lo, const double* hi,
                                  Cnt& cnt) {
  ++cnt.tron_calls;
#pragma unroll
  for (int i = 0; i < N; ++i) S.x[i] = clampd(S.x[i], lo[i], hi[i]);
  S.it = 0;
  S.status = kMaxit;
  S.eval = true;
  S.first = true;
  S.delta = 1.0;
}

// Returns true when the solve has ended (S.status is then set).
template <int N, class Cnt>
__device__ bool tron_advance(TronState<N>& S, const BranchIn<N>& B, const double* lo,
                             const double* hi, double gtol, double ftol, int maxit,
                             Cnt& cnt) {
  if (S.eval) {
    fgh<N>(B, S.x, S.f, S.g, S.H, cnt);
    S.eval = false;
    if (S.first) {
      double pg2 = 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const double t = clampd(S.x[i] - S.g[i], lo[i], hi[i]) - S.x[i];
        pg2 = fma(t, t, pg2);
      }
      S.delta = sqrt(pg2);
      FL(4 * N + 1);
      if (!(S.delta > 0.0)) S.delta = 1.0;
      S.first = false;
    }
  }
  if (S.it > 0) {
    const double xx = dotN<N>(S.x, S.x);
    FL(2 * N + 2);
    if (S.delta * S.delta <= 1e-30 * (xx > 1.0 ? xx : 1.0)) {
      S.status = kStall;
      return true;
    }
  }
  if (S.it >= maxit) {
    S.status = kMaxit;
    return true;
  }
  double pginf = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double t = fabs(clampd(S.x[i] - S.g[i], lo[i], hi[i]) - S.x[i]);
    pginf = fmax(pginf, t);
  }
  FL(2 * N);
  if (pginf <= gtol) {
    S.status = kConv;
    return true;
  }
  ++cnt.tron_iters;
  double w[N], s[N];
  double qcur = 0.0;
  bool qok = false;
  cauchy<N>(S.x, S.g, S.H, lo, hi, S.delta, S.alphac, w, qcur, qok, cnt);
  subspace<N>(S.x, S.g, S.H, lo, hi, S.delta, w, qcur, qok, cnt);
#pragma unroll
  for (int i = 0; i < N; ++i) s[i] = w[i] - S.x[i];
  FL(N);
  double qs;
  if (qok) {
    qs = qcur;
    count_model<N>(cnt);
  } else {
    qs = model<N>(S.g, S.H, s, cnt);
  }
  const double prered = -qs;
  const double snorm = sqrt(dotN<N>(s, s));
  FL(2 * N + 1);
  if (!(prered > 0.0)) {
    S.status = kStall;
    return true;
  }
  if (snorm < S.delta) {
    FL(2);
    if (prered <= ftol * (1.0 + fabs(S.f))) {
#pragma unroll
      for (int i = 0; i < N; ++i) S.x[i] = w[i];
      S.status = kConv;
      return true;
    }
  }
  double aw[8], auxw[4];
  const double fw = fval<N>(B, w, aw, auxw, cnt);
  const double actred = S.f - fw;
  const double ratio = actred / prered;
  FL(2);
  double delta = S.delta;
  if (ratio <= kEta0) {
    delta = kSig2 * (snorm < delta ? snorm : delta);
    FL(1);
  } else if (ratio <= kEta1) {
    const double a = kSig1 * delta, b = kSig2 * (snorm < delta ? snorm : delta);
    delta = a < b ? b : a;
    FL(2);
  } else if (ratio >= kEta2) {
    const double a = kSig3 * delta, b0 = kSig3 * snorm;
    const double b = delta < b0 ? b0 : delta;
    delta = b < a ? b : a;
    FL(2);
  }
  S.delta = delta;
  if (ratio > kEta0) {
#pragma unroll
    for (int i = 0; i < N; ++i) S.x[i] = w[i];
    S.eval = true;
  }
  ++S.it;
  return false;
}

#undef FL

// Coupling positions k = 0..7 of branch l: p_ij q_ij p_ji q_ji w_i th_i w_j th_j.
__device__ inline void branch_couplings(const BranchArgs& A, int64_t l, int64_t* cidx) {
  const int64_t ef = A.ef[l], et = A.et[l];
  cidx[0] = end_coupling(A.ng, A.ne, 0, ef);
  cidx[1] = end_coupling(A.ng, A.ne, 1, ef);
  cidx[2] = end_coupling(A.ng, A.ne, 0, et);
  cidx[3] = end_coupling(A.ng, A.ne, 1, et);
  cidx[4] = end_coupling(A.ng, A.ne, 2, ef);
  cidx[5] = end_coupling(A.ng, A.ne, 3, ef);
  cidx[6] = end_coupling(A.ng, A.ne, 2, et);
  cidx[7] = end_coupling(A.ng, A.ne, 3, et);
}

// The branch's record (written by the bus step, 128 bytes): per end (from,
// to) and per coupling kind (p, q, w, theta) the pair (v_k - z_k, y_k),
// read as eight 16-byte loads of one 128-byte line.
template <int N>
__device__ inline void load_record(const BranchArgs& A, int64_t l, BranchIn<N>& B) {
  const double2* rec = reinterpret_cast<const double2*>(A.brec) + 8 * l;
  double2 q[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) q[t] = rec[t];
  // record slot (end * 4 + kind) -> coupling k = 0..7: p_ij q_ij p_ji q_ji
  // w_i th_i w_j th_j
  constexpr int kOf[8] = {0, 1, 4, 5, 2, 3, 6, 7};
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    B.cv[kOf[t]] = q[t].x;
    B.yc[kOf[t]] = q[t].y;
  }
}

// Branch l of the device order with N variables: solve, write u and state.
// Every input load (branch data, its record, its state and the grid's done
// flag) is issued before the flag is tested, so that the lane waits for one
// round of memory accesses before it computes; the end positions are needed
// only for the stores of u. Returns false, without solving, when the grid has
// finished.
template <int N, bool kLanes, class Cnt>
__device__ bool solve_branch(const BranchArgs& A, int64_t l, Cnt& cnt) {
  {
    const int64_t nl = A.nl;
    const int grid = A.br_grid[l];
    BranchIn<N> B;
    B.gii = A.adm[0 * nl + l];
    B.bii = A.adm[1 * nl + l];
    B.gij = A.adm[2 * nl + l];
    B.bij = A.adm[3 * nl + l];
    B.gji = A.adm[4 * nl + l];
    B.bji = A.adm[5 * nl + l];
    B.gjj = A.adm[6 * nl + l];
    B.bjj = A.adm[7 * nl + l];
    double lo[N], hi[N];
    lo[0] = A.vlo_i[l];
    hi[0] = A.vhi_i[l];
    lo[1] = A.vlo_j[l];
    hi[1] = A.vhi_j[l];
    lo[2] = -kTwoPi;
    hi[2] = kTwoPi;
    lo[3] = -kTwoPi;
    hi[3] = kTwoPi;
    if (N == 6) {
      lo[4] = -A.rate2[l];
      hi[4] = 0.0;
      lo[5] = -A.rate2[l];
      hi[5] = 0.0;
    }
    load_record(A, l, B);
    B.rpq = A.rho_pq;
    B.rva = A.rho_va;
    double x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = A.bx_in[i * nl + l];
    B.lt0 = 0.0;
    B.lt1 = 0.0;
    B.rt = 0.0;
    double alphac = A.calpha_in[l];
    if (N == 6) {
      B.lt0 = A.ltil_in[l];
      B.lt1 = A.ltil_in[nl + l];
      B.rt = A.rtil_in[l];
    }
    if (A.ctl[grid].done != 0 || (kLanes && A.lane_of[grid] != A.lane)) return false;
    int failures = 0;
    if (N == 4) {
      failures +=
          tron<N>(B, x, lo, hi, A.tron_gtol, A.tron_ftol, A.tron_maxit, alphac, cnt) != kConv;
    } else {
      double cprev = 1.0 / 0.0;
      for (int t = 0; t < A.al_maxit; ++t) {
        ++cnt.al;
        failures +=
            tron<N>(B, x, lo, hi, A.tron_gtol, A.tron_ftol, A.tron_maxit, alphac, cnt) != kConv;
        double a[8], aux[4];
        values<N>(B, x, a, aux, cnt);
        const double c0 = fma(a[0], a[0], a[1] * a[1]) + x[4];
        const double c1 = fma(a[2], a[2], a[3] * a[3]) + x[5];
        cnt.flops += 8;
        const double cn = fabs(c0) > fabs(c1) ? fabs(c0) : fabs(c1);
        // multiplier estimate after every round, the last one included
        B.lt0 = B.lt0 + B.rt * c0;
        B.lt1 = B.lt1 + B.rt * c1;
        cnt.flops += 4;
        if (cn <= A.al_tol) break;
        cnt.flops += 1;
        if (cn > A.al_shrink * cprev) {
          const double gr = B.rt * A.al_rho_growth;
          B.rt = gr < A.al_rho_max ? gr : A.al_rho_max;
          cnt.flops += 1;
        }
        cprev = cn;
      }
      A.ltil[l] = B.lt0;
      A.ltil[nl + l] = B.lt1;
      A.rtil[l] = B.rt;
    }
    double a[8], aux[4];
    values<N>(B, x, a, aux, cnt);
    int64_t cidx[8];
    branch_couplings(A, l, cidx);
#pragma unroll
    for (int k = 0; k < 8; ++k) A.u[cidx[k]] = a[k];
#pragma unroll
    for (int i = 0; i < N; ++i) A.bx[i * nl + l] = x[i];
    A.calpha[l] = alphac;
    if (failures) atomicAdd(&A.failures[grid], failures);
  }
  return true;
}

// eq. (qp-bound) for generator g: p and q are couplings g and n_gen + g.
__device__ inline void solve_generator(const BranchArgs& A, int64_t g) {
  const int64_t kp = g, kq = A.ng + g;
  const double rho = A.rho_pq;
  const double Qp = A.c2q[g] + rho;
  const double cp = rho * (A.v[kp] - A.z[kp]) - A.y[kp] - A.c1l[g];
  const double xp = cp / Qp;
  A.u[kp] = fmax(A.pmin[g], fmin(A.pmax[g], xp));
  const double cq = rho * (A.v[kq] - A.z[kq]) - A.y[kq];
  const double xq = cq / rho;
  A.u[kq] = fmax(A.qmin[g], fmin(A.qmax[g], xq));
}


// Loads branch l: data, bounds, coupling values and the persistent state.
template <int N>
__device__ inline void load_branch(const BranchArgs& A, int64_t l, BranchIn<N>& B, double* lo,
                                   double* hi, double* x) {
  const int64_t nl = A.nl;
  B.gii = A.adm[0 * nl + l];
  B.bii = A.adm[1 * nl + l];
  B.gij = A.adm[2 * nl + l];
  B.bij = A.adm[3 * nl + l];
  B.gji = A.adm[4 * nl + l];
  B.bji = A.adm[5 * nl + l];
  B.gjj = A.adm[6 * nl + l];
  B.bjj = A.adm[7 * nl + l];
  lo[0] = A.vlo_i[l];
  hi[0] = A.vhi_i[l];
  lo[1] = A.vlo_j[l];
  hi[1] = A.vhi_j[l];
  lo[2] = -kTwoPi;
  hi[2] = kTwoPi;
  lo[3] = -kTwoPi;
  hi[3] = kTwoPi;
  if (N == 6) {
    lo[4] = -A.rate2[l];
    hi[4] = 0.0;
    lo[5] = -A.rate2[l];
    hi[5] = 0.0;
  }
  load_record(A, l, B);
  B.rpq = A.rho_pq;
  B.rva = A.rho_va;
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = A.bx_in[i * nl + l];
  B.lt0 = 0.0;
  B.lt1 = 0.0;
  B.rt = 0.0;
  if (N == 6) {
    B.lt0 = A.ltil_in[l];
    B.lt1 = A.ltil_in[nl + l];
    B.rt = A.rtil_in[l];
  }
}

// Persistent lanes over the branch pool [begin, end): every lane owns at most
// one branch solve at a time, advances it by one TRON iteration per trip and,
// when it ends, takes the next branch index from the pool counter (one atomic
// per wavefront per trip). The loop ends when the pool is exhausted and every
// lane of the wavefront has finished.
template <int N, class Cnt>
__device__ void run_pool(const BranchArgs& A, int64_t begin, int64_t end, unsigned* ctr,
                         Cnt& cnt, uint32_t& solves, uint64_t& flops) {
  const int lane = threadIdx.x & 63;
  enum { kFetch = 0, kRun = 1, kDone = 2 };
  int phase = kFetch;
  int64_t l = -1;
  int grid = 0, failures = 0, t_al = 0;
  double cprev = 0.0;
  BranchIn<N> B;
  double lo[N], hi[N];
  TronState<N> S;
  while (true) {
    const bool need = phase == kFetch;
    const unsigned long long m = __ballot(need);
    if (m) {
      const int leader = __ffsll((long long)m) - 1;
      unsigned base = 0;
      if (lane == leader) base = atomicAdd(ctr, (unsigned)__popcll(m));
      base = __shfl(base, leader, 64);
      if (need) {
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        const int64_t idx = begin + (int64_t)base + rank;
        if (idx >= end) {
          phase = kDone;
        } else {
          l = idx;
          grid = A.br_grid[l];
          if (A.ctl[grid].done == 0) {
            load_branch<N>(A, l, B, lo, hi, S.x);
            S.alphac = A.calpha_in[l];
            failures = 0;
            t_al = 0;
            cprev = 1.0 / 0.0;
            if (N == 6) ++cnt.al;
            tron_begin<N>(S, lo, hi, cnt);
            phase = kRun;
          }
        }
      }
    }
    if (__ballot(phase != kDone) == 0ull) break;
    if (phase != kRun) continue;
    if (!tron_advance<N>(S, B, lo, hi, A.tron_gtol, A.tron_ftol, A.tron_maxit, cnt)) continue;
    if (S.status == kConv) ++cnt.conv;
    else if (S.status == kMaxit) ++cnt.maxit;
    else ++cnt.stall;
    failures += S.status != kConv;
    bool finished = true;
    if (N == 6) {
      double a[8], aux[4];
      values<N>(B, S.x, a, aux, cnt);
      const double c0 = fma(a[0], a[0], a[1] * a[1]) + S.x[4];
      const double c1 = fma(a[2], a[2], a[3] * a[3]) + S.x[5];
      cnt.flops += 8;
      const double cn = fabs(c0) > fabs(c1) ? fabs(c0) : fabs(c1);
      B.lt0 = B.lt0 + B.rt * c0;
      B.lt1 = B.lt1 + B.rt * c1;
      cnt.flops += 4;
      if (!(cn <= A.al_tol)) {
        cnt.flops += 1;
        if (cn > A.al_shrink * cprev) {
          const double gr = B.rt * A.al_rho_growth;
          B.rt = gr < A.al_rho_max ? gr : A.al_rho_max;
          cnt.flops += 1;
        }
        cprev = cn;
        ++t_al;
        if (t_al < A.al_maxit) {
          ++cnt.al;
          tron_begin<N>(S, lo, hi, cnt);
          finished = false;
        }
      }
    }
    if (!finished) continue;
    const int64_t nl = A.nl;
    if (N == 6) {
      A.ltil[l] = B.lt0;
      A.ltil[nl + l] = B.lt1;
      A.rtil[l] = B.rt;
    }
    double a[8], aux[4];
    values<N>(B, S.x, a, aux, cnt);
    int64_t cidx[8];
    branch_couplings(A, l, cidx);
#pragma unroll
    for (int k = 0; k < 8; ++k) A.u[cidx[k]] = a[k];
#pragma unroll
    for (int i = 0; i < N; ++i) A.bx[i * nl + l] = S.x[i];
    A.calpha[l] = S.alphac;
    if (failures) atomicAdd(&A.failures[grid], failures);
    ++solves;
    flops += cnt.flops;  // a lane may solve many branches: keep the sum in 64 bits
    cnt.flops = 0;
    phase = kFetch;
  }
}

// Persistent x-step: a fixed number of 64-lane blocks drain the rated pool,
// then the unlimited pool, then the generators; the last block to finish
// rearms the pool counters. With kStats the lanes also count algorithmic
// flops and TRON events into A.stats; without it the counters are never read
// and the compiler drops their arithmetic.
template <bool kStats>
__global__ __launch_bounds__(64) void xstep_persistent_kernel(BranchArgs A, int64_t n6) {
  CountersT<kStats> cnt = {};
  uint32_t solves = 0;
  uint64_t flops = 0;
  run_pool<6>(A, 0, n6, &A.pool[0], cnt, solves, flops);
  run_pool<4>(A, n6, A.nl, &A.pool[1], cnt, solves, flops);
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < A.ng; g += nthreads)
    if (A.ctl[A.gen_grid[g]].done == 0) solve_generator(A, g);
  if (kStats) {
    uint64_t v[15] = {(uint64_t)solves, flops + cnt.flops, (uint64_t)cnt.trig, cnt.tron_calls,
                      cnt.tron_iters, cnt.n_fgh, cnt.n_f, cnt.cauchy, cnt.cg, cnt.chol,
                      cnt.ps, cnt.al, cnt.conv, cnt.maxit, cnt.stall};
#pragma unroll
    for (int q = 0; q < 15; ++q) {
      uint64_t t = v[q];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
      v[q] = t;
    }
    if (threadIdx.x == 0 && v[0] != 0) {
#pragma unroll
      for (int q = 0; q < 15; ++q) atomicAdd(&A.stats[q], (unsigned long long)v[q]);
    }
  }
  if (threadIdx.x == 0) {
    // the last block to finish rearms the pools for the next launch: every
    // other block has taken its final index before it counted itself done
    __threadfence();
    if (atomicAdd(&A.pool[2], 1u) == gridDim.x - 1) {
      atomicExch(&A.pool[0], 0u);
      atomicExch(&A.pool[1], 0u);
      atomicExch(&A.pool[2], 0u);
    }
  }
}

void launch_xstep_persistent(const BranchArgs& A, int64_t n6, int blocks, bool stats,
                             hipStream_t s) {
  if (blocks < 1) blocks = 1;
  if (stats)
    hipLaunchKernelGGL(xstep_persistent_kernel<true>, dim3(blocks), dim3(64), 0, s, A, n6);
  else
    hipLaunchKernelGGL(xstep_persistent_kernel<false>, dim3(blocks), dim3(64), 0, s, A, n6);
}

#ifndef ACOPF_XSTEP_WAVES_PER_EU
#define ACOPF_XSTEP_WAVES_PER_EU 1
#endif

// Lane-per-branch x-step. Blocks [0, b6) of the layout take one rated branch
// per lane, the next b4 blocks k4 unlimited branches per lane, one after the
// other (branch base + j * b4 * blockDim for j < k4), and the last bg blocks
// the generators. With k4 chosen so that every branch wavefront is resident
// from the start, the cheap unlimited branches finish inside the span of the
// expensive rated ones instead of waiting for a second round of SIMD slots;
// the short generator blocks come last, so that they take the SIMD slots the
// branch wavefronts leave free instead of delaying some of those wavefronts.
// When only some grids run, the launch has one block per layout block that
// touches them (vblock); lanes on branches of finished grids return at once.
// At chunk positions pos >= 1 the first n_dec blocks take the previous
// iteration's control decision of the running grids while the others solve
// (the state is double-buffered, so that branch solves that run past a
// grid's finish overwrite only the older buffer).
// kStats: as for the persistent kernel. kLanes: the handle's grids are split
// into launch lanes; a layout block can hold branches or generators of grids
// of several lanes, and each lane's launch solves only its own grids' ones.
template <bool kStats, bool kLanes>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ACOPF_XSTEP_WAVES_PER_EU)))
void xstep_kernel(BranchArgs A, int64_t n6, int bg, int b6, int b4, int k4,
                  const int* __restrict__ vblock, const DecideArgs* __restrict__ dec, int n_dec,
                  int pos) {
  if ((int)blockIdx.x < n_dec) {  // the previous iteration's decision for one grid
    decide_grid(*dec, blockIdx.x, pos & 1);
    return;
  }
  CountersT<kStats> cnt = {};
  uint32_t solves = 0;
  const int k = (int)blockIdx.x - n_dec;
  const int b = vblock ? vblock[k] : k;
  const int bs = blockDim.x;
  if (b >= b6 + b4) {
    const int64_t g = (int64_t)(b - b6 - b4) * bs + threadIdx.x;
    if (g < A.ng) {
      const int grid = A.gen_grid[g];
      if (A.ctl[grid].done == 0 && (!kLanes || A.lane_of[grid] == A.lane))
        solve_generator(A, g);
    }
    return;  // whole block is generators: no branch counters
  }
  if (b < b6) {
    const int64_t l = (int64_t)b * bs + threadIdx.x;
    if (l < n6 && solve_branch<6, kLanes>(A, l, cnt)) ++solves;
  } else {
    const int64_t base = n6 + (int64_t)(b - b6) * bs + threadIdx.x;
    const int64_t stride = (int64_t)b4 * bs;
    for (int j = 0; j < k4; ++j) {
      const int64_t l = base + j * stride;
      if (l >= A.nl) break;
      if (solve_branch<4, kLanes>(A, l, cnt)) ++solves;
    }
  }
  if (!kStats) return;
  // wave-level reduction of the counters, one atomic per counter per wavefront
  uint64_t v[15] = {(uint64_t)solves, (uint64_t)cnt.flops, (uint64_t)cnt.trig, cnt.tron_calls,
                    cnt.tron_iters, cnt.n_fgh, cnt.n_f, cnt.cauchy, cnt.cg, cnt.chol,
                    cnt.ps, cnt.al, cnt.conv, cnt.maxit, cnt.stall};
#pragma unroll
  for (int q = 0; q < 15; ++q) {
    uint64_t t = v[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    v[q] = t;
  }
  if ((threadIdx.x & 63) == 0 && v[0] != 0) {
#pragma unroll
    for (int q = 0; q < 15; ++q) atomicAdd(&A.stats[q], (unsigned long long)v[q]);
  }
}

void launch_xstep(const BranchArgs& A, const XLayout& L, const int* vblock, int n_blocks,
                  const DecideArgs* dec, int n_dec, int pos, int block, bool stats,
                  hipStream_t s) {
  if (n_blocks + n_dec <= 0) return;
  // the lane test is compiled only into the variants for several lanes
  auto kernel = stats ? (A.lane_of ? xstep_kernel<true, true> : xstep_kernel<true, false>)
                      : (A.lane_of ? xstep_kernel<false, true> : xstep_kernel<false, false>);
  hipLaunchKernelGGL(kernel, dim3(n_dec + n_blocks), dim3(block), 0, s, A, L.n6, L.bg, L.b6,
                     L.b4, L.k4, vblock, dec, n_dec, pos);
}

bool is_xstep_kernel(const void* f) {
  return f == reinterpret_cast<const void*>(&xstep_kernel<false, false>) ||
         f == reinterpret_cast<const void*>(&xstep_kernel<true, false>) ||
         f == reinterpret_cast<const void*>(&xstep_kernel<false, true>) ||
         f == reinterpret_cast<const void*>(&xstep_kernel<true, true>);
}

// ---------------------------------------------------------------------------
// Solution quality, Sec. IV-A: the ADMM solution is the generator outputs of
// the generator problems (u) and w_i, theta_i of the bus problems (v of the
// bus's first branch end in the bus CSR order: from-ends, then to-ends);
// flows are recomputed from w, theta with eqs. (pij)-(qji), w^R = v_i v_j cos,
// w^I = v_i v_j sin, v = sqrt(w), with the same operations as the branch
// evaluation. Maxima per grid (slot order): ||c||_inf, |residual of (pg)|,
// |of (qg)|, line-limit excess on the unscaled rating, voltage-limit excess,
// |theta| - 2 pi excess.
// ---------------------------------------------------------------------------
__device__ inline double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

// maximum into qmax[grid][slot]: one atomic per wavefront when its lanes share
// the grid, else one per lane
__device__ void quality_max(unsigned long long* qmax, int grid, int slot, double val) {
  const int g0 = __shfl(grid, 0, 64);
  const bool uniform = __ballot(grid != g0) == 0ull;
  if (uniform) {
    for (int off = 32; off > 0; off >>= 1) val = nanmax(val, __shfl_xor(val, off, 64));
    if ((threadIdx.x & 63) == 0 && g0 >= 0)
      atomicMax(&qmax[6 * g0 + slot], (unsigned long long)__double_as_longlong(val));
  } else if (grid >= 0) {
    atomicMax(&qmax[6 * grid + slot], (unsigned long long)__double_as_longlong(val));
  }
}

__global__ __launch_bounds__(256) void quality_values_kernel(QualityArgs Q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Q.nb) return;
  const int64_t e = Q.eptr[i];
  Q.bw[i] = Q.v[end_coupling(Q.ng, Q.ne, 2, e)];
  Q.bt[i] = Q.v[end_coupling(Q.ng, Q.ne, 3, e)];
}

__global__ __launch_bounds__(256) void quality_flow_kernel(QualityArgs Q) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int grid = -1;
  double line = 0.0;
  if (l < Q.nl) {
    grid = Q.br_grid[l];
    const int64_t ef = Q.ef[l], et = Q.et[l];
    const int i = Q.end_bus[ef], j = Q.end_bus[et];
    const int64_t nl = Q.nl;
    const double gii = Q.adm[0 * nl + l], bii = Q.adm[1 * nl + l], gij = Q.adm[2 * nl + l],
                 bij = Q.adm[3 * nl + l], gji = Q.adm[4 * nl + l], bji = Q.adm[5 * nl + l],
                 gjj = Q.adm[6 * nl + l], bjj = Q.adm[7 * nl + l];
    const double wi = Q.bw[i], wj = Q.bw[j];
    double sn, cs;
    series_sincos(Q.bt[i] - Q.bt[j], &sn, &cs);
    const double vv = sqrt(wi) * sqrt(wj);
    const double WR = vv * cs, WI = vv * sn;
    const double pij = fma(bij, WI, fma(gij, WR, gii * wi));
    const double qij = fma(gij, WI, fma(-bij, WR, -bii * wi));
    const double pji = fma(-bji, WI, fma(gji, WR, gjj * wj));
    const double qji = fma(-gji, WI, fma(-bji, WR, -bjj * wj));
    Q.pe[ef] = pij;
    Q.qe[ef] = qij;
    Q.pe[et] = pji;
    Q.qe[et] = qji;
    const double r = Q.rate[l];
    if (r > 0.0) {
      const double sf = sqrt(fma(pij, pij, qij * qij));
      const double st = sqrt(fma(pji, pji, qji * qji));
      line = nanmax(line, nanmax(sf - r, st - r));
    }
  }
  quality_max(Q.qmax, grid, 3, line);
}

__global__ __launch_bounds__(256) void quality_bus_kernel(QualityArgs Q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int grid = -1;
  double balp = 0.0, balq = 0.0, volt = 0.0, ang = 0.0;
  if (i < Q.nb) {
    grid = Q.bus_grid[i];
    double sp = 0.0, sq = 0.0;
    for (int g = Q.gptr[i]; g < Q.gptr[i + 1]; ++g) {
      sp = sp + Q.u[g];
      sq = sq + Q.u[Q.ng + g];
    }
    const double w = Q.bw[i];
    sp = fma(-Q.gs[i], w, sp - Q.pd[i]);
    sq = fma(Q.bs[i], w, sq - Q.qd[i]);
    for (int e = Q.eptr[i]; e < Q.eptr[i + 1]; ++e) {
      sp = sp - Q.pe[e];
      sq = sq - Q.qe[e];
    }
    balp = nanmax(balp, fabs(sp));
    balq = nanmax(balq, fabs(sq));
    const double vm = w > 0.0 ? sqrt(w) : 0.0;
    volt = nanmax(volt, nanmax(Q.vmin[i] - vm, vm - Q.vmax[i]));
    ang = nanmax(ang, fabs(Q.bt[i]) - kTwoPi);
  }
  quality_max(Q.qmax, grid, 1, balp);
  quality_max(Q.qmax, grid, 2, balq);
  quality_max(Q.qmax, grid, 4, volt);
  quality_max(Q.qmax, grid, 5, ang);
}

__global__ __launch_bounds__(256) void fill_u64_kernel(unsigned long long* p, int64_t n) {
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

void launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(256), 0, s, p, n);
}

void launch_quality(const QualityArgs& Q, hipStream_t s) {
  const int bs = 256;
  hipLaunchKernelGGL(quality_values_kernel, dim3((Q.nb + bs - 1) / bs), dim3(bs), 0, s, Q);
  hipLaunchKernelGGL(quality_flow_kernel, dim3((Q.nl + bs - 1) / bs), dim3(bs), 0, s, Q);
  hipLaunchKernelGGL(quality_bus_kernel, dim3((Q.nb + bs - 1) / bs), dim3(bs), 0, s, Q);
}

}  // namespace acopf_dev
