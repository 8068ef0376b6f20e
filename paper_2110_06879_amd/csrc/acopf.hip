// Host runtime and the closed-form kernels of the two-level component ADMM
// for ACOPF (Kim & Kim, PSCC 2022) on gfx950, behind the C ABI of acopf.h.
//
// One inner iteration of Algorithm 1 is two launches on one stream, and a
// chunk of iterations ends with a third:
//   xstep_kernel    branch subproblems, eq. (branch), TRON + AL     lane/branch
//                   and the generator closed form, eq. (qp-bound);  lane/gen
//                   in its first blocks, the previous iteration's   block/grid
//                   control decision (tests, outer step, beta rule)
//   bus_kernel      a pending outer multiplier step lambda <-      block/tile
//                   proj(lambda + beta z), the bus closed form     of buses,
//                   eq. (qp-bus), then z and y and the residual    lane/pair
//                   maxima of every coupling it owns (tiles of a
//                   bus too large for one block in a second
//                   launch, only when there are such buses)
//   ctl_kernel      the decision of the chunk's last iteration      block/grid
// The generator and branch steps read only the previous iteration's v, z, y
// and so could run in any order; the bus step owns each coupling exactly once
// (every coupling has one bus side), which makes the z and y updates and the
// residual maxima a fused, race-free pass. Each bus tile writes its residual
// maxima to a slot of its own and the decision takes the maximum over a
// grid's tiles: exact and independent of order, with no atomics contending
// on one address. The decision of iteration t runs beside the branch solves
// of iteration t + 1, which read their state from one of two buffers and
// write the other: if it finishes the grid, those solves overwrite only the
// older buffer, the bus step of t + 1 skips the grid, and the host moves the
// grid's state to the first buffer after the chunk. An outer step decided at
// iteration t is applied by the bus step of iteration t + 1 before it uses
// lambda (the branch step does not read lambda); one still pending when the
// host regains control (the grid finished, or the run stopped) is applied
// then. Kernels return at once for grids that have finished, so a chunk of
// launches can overshoot convergence harmlessly; the host reads the per-grid
// control words once per chunk.
//
// Device layout (structure of arrays, FP64), chosen for the HBM-bound bus
// step: every bus owns a contiguous range of generators and of branch ends,
// so the bus kernel streams its couplings. The branch step reads its inputs
// as one 128-byte record per branch (v - z and y of its eight couplings),
// which the bus step writes in branch order, and does the scattered accesses
// itself: the eight stores of its coupling values u.
//   generators: sorted by (grid, bus, input index), range gptr[b]..gptr[b+1];
//   branch ends: bus CSR order (per bus: from-ends, then to-ends, each in
//     input order), range eptr[b]..eptr[b+1];
//   couplings [m]: generator p [n_gen], generator q [n_gen], then the four
//     couplings p, q, w, theta of each branch end, end after end;
//   branches: rated (6-variable) first, then unlimited (4-variable), each by
//     (grid, from bus, input index); ef[l], et[l] locate their two ends.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/acopf.h"
#include "device_common.h"

using acopf_dev::BranchArgs;
using acopf_dev::DecideArgs;
using acopf_dev::GridCtl;
using acopf_dev::GridItem;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                        \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return fail(ACOPF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kHistCap = 1 << 15;  // per grid, inner iterations kept in history
constexpr int kStats = 16;
constexpr int kEvPerIter = 4;   // events per profiled iteration
constexpr int kTimed = 3;       // kernels timed per iteration (x-step, bus, ctl)
constexpr int kChunk = 16;      // iterations between control readbacks (default)
constexpr int kMaxChunk = 64;   // largest chunk acopf_set_tuning accepts
constexpr int kMaxLanes = 4;    // largest number of launch lanes

// Device-resident scratch of acopf_quality_noalloc: 2^20 eight-byte words
// (8 MiB) per device, held until the process ends. Host code never uses the
// array's name as an address: each device's address comes from
// hipGetSymbolAddress (noalloc_scratch below).
constexpr int64_t kNoAllocWords = int64_t(1) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocWords];

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// One bus tile: buses [b0, b1) of grid `grid`, their branch ends [e0, e1)
// and generators [g0, g1) in the device orders.
struct TileDesc {
  int b0, b1, e0, e1, g0, g1, grid, id;  // id: tile index (tmax slot), -1: none
};

struct BusArgs {
  int64_t nb, ng, ne;
  const TileDesc* tile_list;  // tiles of the launch (of running grids); a tile
                              // never spans two grids
  const TileDesc* hub_list;   // tiles of the hub launch
  const int* bus_grid;
  GridCtl* ctl;
  const int *gptr, *eptr;
  const double *pd, *qd, *gs, *bs;
  const int* isref;
  const double* u;
  double* lam;               // written by the outer multiplier step
  double *v, *z, *y;
  double rho_pq, rho_va;
  double* tmax;              // [n_tiles][3] residual maxima of each tile
  const int* erec;           // [ne] record half of each end: 2 l + (0 from, 1 to)
  double* brec;              // [nl][16] branch records for the next x-step
  double lambda_max;         // projection bound of the outer multiplier step
};

// Half of a branch record (64 bytes): the pairs (v_k - z_k, y_k) of one
// end's four couplings p, q, w, theta, written by the step that produced
// v, z and y, so that the branch step reads its inputs as one line.
__device__ inline void store_record_half(double* brec, int half, const double2* rec) {
  double2* dst = reinterpret_cast<double2*>(brec) + 4 * (int64_t)half;
#pragma unroll
  for (int t = 0; t < 4; ++t) dst[t] = rec[t];
}

// LDS bytes of one bus tile of `nt` lanes: per coupling (two per lane) its
// target and its quotient by rho_pq, per lane the local bus of its pair, per
// bus (at most nt / 2) four results.
__host__ __device__ inline size_t bus_lds_bytes(int nt) {
  return sizeof(double) * (4 * (size_t)nt + 4 * (size_t)(nt / 2)) + sizeof(unsigned short) * (size_t)nt;
}

// Phase 2 of the bus step for one bus (lane per bus): the sums over its
// couplings in their fixed order and the 2x2 solve. Slot 2 j and 2 j + 1 of
// `val` and `quo` are the two couplings of pair j (generator g is pair
// 2 n_ends + g: slots nce + 2 g for p, nce + 2 g + 1 for q). kHub: the tile is a
// single bus with more couplings than its LDS holds, and values past the
// LDS are recomputed from global memory by `val` and `quo`.
template <bool kHub, class Val, class Quo>
__device__ inline void bus_solve(int tid, int be0, int be1, int bg0, int bg1, int nce, int ngt,
                                 double bgs, double bbs, double bpd, double bqd, int bref,
                                 double rpq, double rva, const Val& val, const Quo& quo,
                                 unsigned short* cb, int ncap, double* bv, int tb) {
  // Each loop reads four terms at a time (a clamped index reads a valid slot
  // whose value is not used), so that the reads overlap; the sums still add
  // one term at a time in their fixed order.
  double Qw = 0.0, cw = 0.0, Qt = 0.0, ctt = 0.0;
  for (int e = be0; e < be1; e += 4) {
    double w4[4], t4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int ek = e + k < be1 ? e + k : e;
      w4[k] = val(4 * ek + 2);
      t4[k] = val(4 * ek + 3);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (e + k < be1) {
        Qw += rva;
        cw += w4[k];
        Qt += rva;
        ctt += t4[k];
        if (!kHub || 2 * (e + k) + 1 < ncap) {
          cb[2 * (e + k)] = (unsigned short)tid;
          cb[2 * (e + k) + 1] = (unsigned short)tid;
        }
      }
    }
  }
  const double awP = -bgs, awQ = bbs;
  double M00 = awP * awP / Qw, M01 = awP * awQ / Qw, M11 = awQ * awQ / Qw;
  double r0 = awP * cw / Qw - bpd, r1 = awQ * cw / Qw - bqd;
  const double inv_pq = 1.0 / rpq;
  for (int g = bg0; g < bg1; ++g) {
    M00 += inv_pq;
    r0 += quo(nce + 2 * g);
    M11 += inv_pq;
    r1 += quo(nce + 2 * g + 1);
    if (!kHub || nce / 2 + g < ncap) cb[nce / 2 + g] = (unsigned short)tid;
  }
  for (int e = be0; e < be1; e += 4) {
    double p4[4], q4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int ek = e + k < be1 ? e + k : e;
      p4[k] = quo(4 * ek);
      q4[k] = quo(4 * ek + 1);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (e + k < be1) {
        M00 += inv_pq;
        r0 += -p4[k];
        M11 += inv_pq;
        r1 += -q4[k];
      }
    }
  }
  const double det = M00 * M11 - M01 * M01;
  const double mu0 = (M11 * r0 - M01 * r1) / det;
  const double mu1 = (M00 * r1 - M01 * r0) / det;
  bv[tid] = mu0;
  bv[tb + tid] = mu1;
  bv[2 * tb + tid] = (cw - awP * mu0 - awQ * mu1) / Qw;
  bv[3 * tb + tid] = bref ? 0.0 : ctt / Qt;
}

// eq. (qp-bus) for every bus of one tile of consecutive buses: minimize
// sum_k rho_k/2 (x_k - x0_k)^2 over the bus copies (generator outputs, flows
// leaving the bus, w) subject to the two balance rows of eqs. (pg)-(qg);
// closed form through the 2x2 matrix M = A Q^-1 A'. Then z (eq. qp-bound
// with no bounds) and y for every coupling of the tile, and their residual
// maxima. A tile's couplings are its end couplings (contiguous, p q w theta
// per end) followed by its generators' p and q couplings; each lane owns a
// pair of couplings: an end's (p, q) or (w, theta), or a generator's (p, q).
//   0. lane per pair: the outer multiplier step, when the previous
//      iteration's decision left one pending;
//   1. lane per pair: the prox targets c_k = rho_k (u_k + z_k) + y_k and,
//      for p and q couplings, c_k / rho_pq, into LDS (16-byte loads);
//   2. lane per bus: the sums over its couplings in their fixed order, read
//      from LDS, and the 2x2 solve;
//   3. lane per pair: new v, z, y, the branch record pairs and the residuals.
// Every load a lane needs is issued before the grid's done flag is tested.
// A single bus with more couplings than the tile holds (a hub) gets a tile of
// its own; pairs past the lane count are recomputed from global memory with
// the same operations.
template <bool kHub>
__global__ __launch_bounds__(1024) void bus_kernel(BusArgs A) {
  extern __shared__ double sm[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const TileDesc D = (kHub ? A.hub_list : A.tile_list)[blockIdx.x];
  const int t = D.id;
  if (t < 0) return;  // the placeholder of an empty list
  const int b0 = D.b0, nbt = D.b1 - D.b0, grid = D.grid;
  const int tb = nt >> 1, ncap = nt;  // buses and pairs held in LDS
  double* cT = sm;                 // [2 nt] targets
  double* cQ = cT + 2 * nt;        // [2 nt] targets / rho_pq (p and q couplings)
  double* bv = cQ + 2 * nt;        // [4][tb] mu0, mu1, w, theta per bus
  unsigned short* cb = reinterpret_cast<unsigned short*>(bv + 4 * tb);  // [nt] local bus per pair
  const int64_t ng = A.ng;
  const double rpq = A.rho_pq, rva = A.rho_va;
  const int E0 = D.e0, G0 = D.g0;
  const int net = D.e1 - D.e0, ngt = D.g1 - D.g0;
  const int nce = 4 * net, npe = 2 * net, np = npe + ngt;
  // ---- loads: bus data (phase 2), the lane's pair, the grid's control word
  int be0 = 0, be1 = 0, bg0 = 0, bg1 = 0, bref = 0;
  double bgs = 0.0, bbs = 0.0, bpd = 0.0, bqd = 0.0;
  if (tid < nbt) {
    const int i = b0 + tid;
    be0 = A.eptr[i] - E0;
    be1 = A.eptr[i + 1] - E0;
    bg0 = A.gptr[i] - G0;
    bg1 = A.gptr[i + 1] - G0;
    bgs = A.gs[i];
    bbs = A.bs[i];
    bpd = A.pd[i];
    bqd = A.qd[i];
    bref = A.isref[i];
  }
  // pair j: j < npe end pair (end j / 2, kinds 2 (j & 1) and 2 (j & 1) + 1),
  // else generator j - npe (p and q)
  double2 cu{0.0, 0.0}, cz{0.0, 0.0}, cy{0.0, 0.0}, cv{0.0, 0.0}, cl{0.0, 0.0};
  int half = 0;
  auto load_pair = [&](int j, double2& u_, double2& z_, double2& y_, double2& v_, double2& l_, int& hf) {
    if (j < npe) {
      const int64_t k = 2 * ng + 4 * (int64_t)E0 + 2 * j;
      u_ = *reinterpret_cast<const double2*>(A.u + k);
      z_ = *reinterpret_cast<const double2*>(A.z + k);
      y_ = *reinterpret_cast<const double2*>(A.y + k);
      v_ = *reinterpret_cast<const double2*>(A.v + k);
      l_ = *reinterpret_cast<const double2*>(A.lam + k);
      hf = A.erec[E0 + (j >> 1)];
    } else {
      const int64_t kp = (int64_t)G0 + (j - npe), kq = ng + kp;
      u_ = make_double2(A.u[kp], A.u[kq]);
      z_ = make_double2(A.z[kp], A.z[kq]);
      y_ = make_double2(A.y[kp], A.y[kq]);
      v_ = make_double2(A.v[kp], A.v[kq]);
      l_ = make_double2(A.lam[kp], A.lam[kq]);
    }
  };
  const bool own = tid < np;
  if (own) load_pair(tid, cu, cz, cy, cv, cl, half);
  const GridCtl* C = A.ctl + grid;
  const int done = C->done;
  const double beta = C->beta;
  const int do_outer = C->do_outer;
  const double bl = C->beta_lam, lm = A.lambda_max;
  if (done) return;  // uniform: the tile lies in one grid
  // The previous iteration ended an outer step (Sec. III-B): the multiplier
  // step lambda <- proj_[-lmax, lmax](lambda + beta z) on this tile's
  // couplings, with the z that iteration produced, before z is updated.
  auto outer_step = [&](int j, double2& l_, const double2& z_) {
    l_.x = fmax(-lm, fmin(lm, l_.x + bl * z_.x));
    l_.y = fmax(-lm, fmin(lm, l_.y + bl * z_.y));
    if (j < npe) {
      *reinterpret_cast<double2*>(A.lam + 2 * ng + 4 * (int64_t)E0 + 2 * j) = l_;
    } else {
      const int64_t kp = (int64_t)G0 + (j - npe);
      A.lam[kp] = l_.x;
      A.lam[ng + kp] = l_.y;
    }
  };
  if (do_outer && own) outer_step(tid, cl, cz);
  // ---- phase 1
  auto is_va = [&](int j) { return j < npe && (j & 1); };  // (w, theta) pair
  if (own) {
    const double rho = is_va(tid) ? rva : rpq;
    const double c0 = rho * (cu.x + cz.x) + cy.x, c1 = rho * (cu.y + cz.y) + cy.y;
    // LDS slots 2 j and 2 j + 1 hold the targets of pair j
    cT[2 * tid] = c0;
    cT[2 * tid + 1] = c1;
    if (!is_va(tid)) {
      cQ[2 * tid] = c0 / rpq;
      cQ[2 * tid + 1] = c1 / rpq;
    }
  }
  __syncthreads();
  // ---- phase 2
  if (tid < nbt) {
    if (!kHub) {
      auto val = [&](int i) { return cT[i]; };
      auto quo = [&](int i) { return cQ[i]; };
      bus_solve<false>(tid, be0, be1, bg0, bg1, nce, ngt, bgs, bbs, bpd, bqd, bref, rpq, rva,
                       val, quo, cb, ncap, bv, tb);
    } else {
      // a hub: slot i (pair i / 2) is held in LDS when its pair is below ncap
      auto pair_of = [&](int i) { return i >> 1; };
      auto gidx = [&](int i) -> int64_t {
        if (i < nce) return 2 * ng + 4 * (int64_t)E0 + i;
        const int j = i - nce;
        return (int64_t)G0 + (j >> 1) + ((j & 1) ? ng : 0);
      };
      auto val = [&](int i) {
        if (pair_of(i) < ncap) return cT[i];
        const int64_t k = gidx(i);
        const double rho = (i < nce && (i & 3) >= 2) ? rva : rpq;
        return rho * (A.u[k] + A.z[k]) + A.y[k];
      };
      auto quo = [&](int i) {
        if (pair_of(i) < ncap) return cQ[i];
        const int64_t k = gidx(i);
        return (rpq * (A.u[k] + A.z[k]) + A.y[k]) / rpq;
      };
      bus_solve<true>(tid, be0, be1, bg0, bg1, nce, ngt, bgs, bbs, bpd, bqd, bref, rpq, rva,
                      val, quo, cb, ncap, bv, tb);
    }
  }
  __syncthreads();
  // ---- phase 3
  double rp = 0.0, rd = 0.0, rz = 0.0;
  auto fin = [&](double vnew, double rho, double vold, double uk, double yold, double lamk,
                 double& zk, double& yk) {
    zk = -(lamk + yold + rho * (uk - vnew)) / (beta + rho);
    yk = yold + rho * (uk - vnew + zk);
    rp = fmax(rp, fabs(uk - vnew + zk));
    rd = fmax(rd, fabs(vnew - vold));
    rz = fmax(rz, fabs(zk));
  };
  for (int j = tid; j < np; j += (kHub ? nt : np)) {
    double2 u_ = cu, z_ = cz, y_ = cy, v_ = cv, l_ = cl;
    int hf = half;
    if (kHub && j != tid) {  // hub overflow
      load_pair(j, u_, z_, y_, v_, l_, hf);
      if (do_outer) outer_step(j, l_, z_);
    }
    const int b = !kHub || j < ncap ? cb[j] : 0;
    const bool va = is_va(j);
    const double rho = va ? rva : rpq;
    // the targets of phase 1 (the same operations again for a hub's overflow)
    const double c0 = (kHub && j != tid) ? rho * (u_.x + z_.x) + y_.x : cT[2 * j];
    const double c1 = (kHub && j != tid) ? rho * (u_.y + z_.y) + y_.y : cT[2 * j + 1];
    double n0, n1;
    if (j < npe) {
      if (va) {
        n0 = bv[2 * tb + b];
        n1 = bv[3 * tb + b];
      } else {
        n0 = (c0 + bv[b]) / rpq;
        n1 = (c1 + bv[tb + b]) / rpq;
      }
    } else {
      n0 = (c0 - bv[b]) / rpq;
      n1 = (c1 - bv[tb + b]) / rpq;
    }
    double z0, y0, z1, y1;
    fin(n0, rho, v_.x, u_.x, y_.x, l_.x, z0, y0);
    fin(n1, rho, v_.y, u_.y, y_.y, l_.y, z1, y1);
    if (j < npe) {
      const int64_t k = 2 * ng + 4 * (int64_t)E0 + 2 * j;
      *reinterpret_cast<double2*>(A.v + k) = make_double2(n0, n1);
      *reinterpret_cast<double2*>(A.z + k) = make_double2(z0, z1);
      *reinterpret_cast<double2*>(A.y + k) = make_double2(y0, y1);
      double2* rec = reinterpret_cast<double2*>(A.brec) + 4 * (int64_t)hf + 2 * (j & 1);
      rec[0] = make_double2(n0 - z0, y0);
      rec[1] = make_double2(n1 - z1, y1);
    } else {
      const int64_t kp = (int64_t)G0 + (j - npe), kq = ng + kp;
      A.v[kp] = n0;
      A.z[kp] = z0;
      A.y[kp] = y0;
      A.v[kq] = n1;
      A.z[kq] = z1;
      A.y[kq] = y1;
    }
  }
  // tile maxima (wavefront, then across the block's wavefronts), written to
  // the tile's own slot: no atomics, and the control kernel reduces a grid's
  // tiles. Maxima are exact, so the order of reduction does not matter.
  __shared__ double red[3][16];
  for (int off = 32; off > 0; off >>= 1) {
    rp = fmax(rp, __shfl_xor(rp, off, 64));
    rd = fmax(rd, __shfl_xor(rd, off, 64));
    rz = fmax(rz, __shfl_xor(rz, off, 64));
  }
  const int wv = tid >> 6, nw = (nt + 63) >> 6;
  if ((tid & 63) == 0) {
    red[0][wv] = rp;
    red[1][wv] = rd;
    red[2][wv] = rz;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < nw; ++w) {
      rp = fmax(rp, red[0][w]);
      rd = fmax(rd, red[1][w]);
      rz = fmax(rz, red[2][w]);
    }
    A.tmax[3 * t + 0] = rp;
    A.tmax[3 * t + 1] = rd;
    A.tmax[3 * t + 2] = rz;
  }
}

// Branch records of the ends [e0, e1) from the current v, z and y (after a
// cold start or any change of the state from the host): the same values the
// bus step writes.
__global__ __launch_bounds__(256) void record_kernel(int64_t ng, int64_t e0, int64_t e1,
                                                     const int* erec, const double* v,
                                                     const double* z, const double* y,
                                                     double* brec) {
  const int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= e1) return;
  double2 rec[4];
#pragma unroll
  for (int kind = 0; kind < 4; ++kind) {
    const int64_t k = 2 * ng + 4 * e + kind;
    rec[kind] = make_double2(v[k] - z[k], y[k]);
  }
  store_record_half(brec, erec[e], rec);
}

// Control of Algorithm 1 per grid, one block of kCtlBlock lanes per running
// grid: the decision of decide_grid for x-step results in buffer cur. It
// takes the last decision of a chunk (the decision blocks of the x-step take
// the others), or every decision when the x-step runs without decision
// blocks (the persistent kernel, and with counting on).
constexpr int kCtlBlock = 256;
__global__ __launch_bounds__(kCtlBlock) void ctl_kernel(DecideArgs A, int cur) {
  acopf_dev::decide_grid(A, blockIdx.x, cur);
}

// An outer multiplier step of grid g (Sec. III-B) still pending when the
// host regains control: lambda <- proj_[-lmax, lmax](lambda + beta z), with
// the beta of the step (bl), over the grid's generator couplings [g0, g1) (p,
// and q at ng + k) and end couplings [c0, c1); the flag is cleared. Grid-
// stride, so any number of blocks covers the grid.
__global__ __launch_bounds__(256) void outer_step_kernel(GridCtl* ctl, int g, int64_t ng,
                                                         int64_t g0, int64_t g1, int64_t c0,
                                                         int64_t c1, double bl, double lm,
                                                         const double* z, double* lam) {
  const int64_t n_gen = g1 - g0, n = 2 * n_gen + (c1 - c0);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int64_t k = i < n_gen ? g0 + i
                                : (i < 2 * n_gen ? ng + g0 + (i - n_gen) : c0 + (i - 2 * n_gen));
    lam[k] = fmax(-lm, fmin(lm, lam[k] + bl * z[k]));
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl[g].do_outer = 0;
}

struct ColdArgs {
  int only;  // grid to initialize, or -1 for all
  int64_t ng, nl, ne, m;
  const int *ef, *et;
  const int *gen_grid, *br_grid;
  const double *pmin, *pmax, *qmin, *qmax;
  const double* adm;
  const double *vlo_i, *vhi_i, *vlo_j, *vhi_j, *rate2;
  int64_t n6;
  double *u, *v, *z, *y, *lam, *bx, *ltil, *rtil, *calpha;
  double al_rho0;
};

// Cold start (Sec. IV-B): p, q, |V| at the midpoints of their bounds, angles
// 0, flows from the initial voltages, bus copies equal to the component
// values, z = y = lambda = 0. Slacks start at -(p^2 + q^2) clipped to range.
__global__ __launch_bounds__(256) void cold_kernel(ColdArgs A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  auto setk = [&](int64_t k, double val) {
    A.u[k] = val;
    A.v[k] = val;
    A.z[k] = 0.0;
    A.y[k] = 0.0;
    A.lam[k] = 0.0;
  };
  if (t < A.ng) {
    if (A.only >= 0 && A.gen_grid[t] != A.only) return;
    setk(t, 0.5 * (A.pmin[t] + A.pmax[t]));
    setk(A.ng + t, 0.5 * (A.qmin[t] + A.qmax[t]));
    return;
  }
  const int64_t l = t - A.ng;
  if (l >= A.nl) return;
  if (A.only >= 0 && A.br_grid[l] != A.only) return;
  const int64_t nl = A.nl;
  const double vi = 0.5 * (A.vlo_i[l] + A.vhi_i[l]);
  const double vj = 0.5 * (A.vlo_j[l] + A.vhi_j[l]);
  // angles are zero: w^R = vi vj, w^I = 0
  const double* Y = A.adm;
  const double wi = vi * vi, wj = vj * vj, WR = vi * vj * 1.0, WI = vi * vj * 0.0;
  // flows as in the branch evaluation (fused multiply-adds in the same places)
  const double a0 = fma(Y[3 * nl + l], WI, fma(Y[2 * nl + l], WR, Y[0 * nl + l] * wi));
  const double a1 = fma(Y[2 * nl + l], WI, fma(-Y[3 * nl + l], WR, -Y[1 * nl + l] * wi));
  const double a2 = fma(-Y[5 * nl + l], WI, fma(Y[4 * nl + l], WR, Y[6 * nl + l] * wj));
  const double a3 = fma(-Y[4 * nl + l], WI, fma(-Y[5 * nl + l], WR, -Y[7 * nl + l] * wj));
  const double a[8] = {a0, a1, a2, a3, wi, 0.0, wj, 0.0};
  const int64_t ef = A.ef[l], et = A.et[l];
  setk(acopf_dev::end_coupling(A.ng, A.ne, 0, ef), a0);
  setk(acopf_dev::end_coupling(A.ng, A.ne, 1, ef), a1);
  setk(acopf_dev::end_coupling(A.ng, A.ne, 0, et), a2);
  setk(acopf_dev::end_coupling(A.ng, A.ne, 1, et), a3);
  setk(acopf_dev::end_coupling(A.ng, A.ne, 2, ef), a[4]);
  setk(acopf_dev::end_coupling(A.ng, A.ne, 3, ef), a[5]);
  setk(acopf_dev::end_coupling(A.ng, A.ne, 2, et), a[6]);
  setk(acopf_dev::end_coupling(A.ng, A.ne, 3, et), a[7]);
  A.bx[0 * nl + l] = vi;
  A.bx[1 * nl + l] = vj;
  A.bx[2 * nl + l] = 0.0;
  A.bx[3 * nl + l] = 0.0;
  double s0 = 0.0, s1 = 0.0;
  if (l < A.n6) {
    const double r2 = A.rate2[l];
    const double f0 = -(a0 * a0 + a1 * a1), f1 = -(a2 * a2 + a3 * a3);
    s0 = f0 < -r2 ? -r2 : (f0 > 0.0 ? 0.0 : f0);
    s1 = f1 < -r2 ? -r2 : (f1 > 0.0 ? 0.0 : f1);
  }
  A.bx[4 * nl + l] = s0;
  A.bx[5 * nl + l] = s1;
  A.ltil[l] = 0.0;
  A.ltil[nl + l] = 0.0;
  A.rtil[l] = A.al_rho0;
  A.calpha[l] = 1.0;
}

// Reset of the per-grid control words at the start of a solve of grid `only`
// (all grids when only < 0).
__global__ void ctl_start_kernel(GridCtl* ctl, int G, int only, int mode, int fixed,
                                 double beta0, int* failures, int* failures_it) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G || (only >= 0 && g != only)) return;
  GridCtl& c = ctl[g];
  if (mode != ACOPF_CONTINUE) {
    c.beta = beta0;
    c.beta_lam = beta0;
    c.znorm_prev = __longlong_as_double(0x7ff0000000000000ll);
    c.outer = 0;
    c.inner_total = 0;
    c.inner_in_outer = 0;
  }
  c.status = ACOPF_MAX_ITER;
  c.done = 0;
  c.do_outer = 0;
  c.cur = 0;
  c.fixed_mode = fixed > 0 ? 1 : 0;
  c.fixed_target = fixed > 0 ? c.inner_total + fixed : 0x7fffffff;
  failures[g] = 0;
  failures_it[g] = 0;
  failures_it[G + g] = 0;
}

// Marks every grid idle (done) without touching its state.
__global__ void ctl_idle_kernel(GridCtl* ctl, int G) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < G) {
    ctl[g].done = 1;
    ctl[g].do_outer = 0;
  }
}

// Device-side copy of up to kCopySegs ranges of doubles and one control
// block in one launch: a grid's state into another instance of the same grid.
// Block row y copies range y; the control block arrives marked idle.
constexpr int kCopySegs = 40;
struct CopySegs {
  int n;
  const double* src[kCopySegs];
  double* dst[kCopySegs];
  int64_t len[kCopySegs];
  const GridCtl* csrc;  // with cdst: the control block, arriving marked idle
  GridCtl* cdst;
  GridCtl* cur_clear;   // or: a control block whose state is now in buffer 0
};
__global__ __launch_bounds__(256) void copy_kernel(CopySegs C) {
  const int s = blockIdx.y;
  const double* src = C.src[0];
  double* dst = C.dst[0];
  int64_t n = C.len[0];
#pragma unroll
  for (int q = 1; q < kCopySegs; ++q)  // selects, so the argument is not indexed
    if (q == s) {
      src = C.src[q];
      dst = C.dst[q];
      n = C.len[q];
    }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
  if (s == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    if (C.csrc) {
      GridCtl c = *C.csrc;
      c.done = 1;
      c.do_outer = 0;
      *C.cdst = c;
    }
    if (C.cur_clear) C.cur_clear->cur = 0;
  }
}

// Objective sum_g c2 P^2 + c1 P + c0 with P = base p_g (Sec. IV-A), one block
// of kObjBlock lanes per grid (a 70k grid's 10,000 generators take each lane
// ten strided steps), fixed-order tree reduction.
constexpr int kObjBlock = 1024;
__global__ __launch_bounds__(kObjBlock) void objective_kernel(const int64_t* gen_off,
                                                             const double* c2, const double* c1,
                                                             const double* c0, const double* u,
                                                             const double* base, double* out) {
  __shared__ double sh[kObjBlock];
  const int g = blockIdx.x;
  const int64_t a = gen_off[g], b = gen_off[g + 1];
  const double bg = base[g];
  double t = 0.0;
  for (int64_t k = a + threadIdx.x; k < b; k += kObjBlock) {
    const double P = bg * u[k];
    t += c2[k] * P * P + c1[k] * P + c0[k];
  }
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int s = kObjBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[g] = sh[0];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct HostGrid {
  int64_t nb, ng, nl;
  int64_t bus_off, gen_off;
  std::vector<int64_t> br_dev;   // input branch -> device branch index
  std::vector<int64_t> gen_dev;  // input generator -> device generator index
  std::vector<int64_t> end_f, end_t;  // input branch -> device end positions
  int64_t e0 = 0, e1 = 0;             // device end range
  int64_t r6b = 0, r6e = 0, r4b = 0, r4e = 0;  // device branch ranges per class
  int ref;
};

struct DevBuf {
  std::vector<void*> ptrs;
  template <class T>
  hipError_t alloc(T** p, size_t n) {
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

bool finite_all(const double* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

}  // namespace

namespace acopf_dev {
// The thread's last error message for codes returned by other translation
// units of the library (the tracking server).
int report_error(int code, const char* msg) { return fail(code, msg); }
}  // namespace acopf_dev

// A launch lane: a subset of the handle's grids with its own stream, work
// lists and captured chunk. The chunks of all lanes are launched back to back
// and run concurrently, so that the issue-bound x-step of one lane overlaps
// the memory-bound bus step of another; the grids of different lanes share
// no data, so the results are those of one launch for all of them.
struct Lane {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t end = nullptr;          // end of the lane's chunk, for the handle's stream
  // Work lists of the lane's grids that run: x-step items, bus tiles, hub
  // tiles and grid items, in one device block filled from a pinned copy.
  char* lists = nullptr;
  char* stage = nullptr;
  int n_x = 0, n_t = 0, n_hl = 0, n_gl = 0;
  acopf_dev::XLayout xlay{};         // x-step block layout (kernel arguments)
  const int* xlist = nullptr;        // x-step blocks to run (null: all of them)
  DecideArgs* dec = nullptr;         // device copy of the decision arguments
  unsigned* pool = nullptr;          // persistent x-step pool counters [3]
  BranchArgs xba[2] = {};            // the x-step's other argument at even and odd positions
  std::vector<char> active_for;      // the running set the lists describe
  bool lists_dirty = true;
  // the captured chunk and its kernel nodes, with the list each one's grid
  // size follows (0 x-step, 1 bus tiles, 2 hub tiles, 3 grids, -1 fixed)
  hipGraph_t gtmpl = nullptr;
  hipGraphExec_t graph = nullptr;
  int graph_chunk = 0;
  std::vector<hipGraphNode_t> gnode;
  std::vector<int> grole;
  std::vector<hipKernelNodeParams> gparam;
};

struct acopf_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  acopf_params P{};
  int G = 0;
  int64_t nb = 0, ng = 0, nl = 0, n6 = 0, m = 0;
  std::vector<HostGrid> grids;
  DevBuf buf;
  // device arrays
  int64_t ne = 0;
  int *gen_grid = nullptr, *br_grid = nullptr, *bus_grid = nullptr;
  int *ef = nullptr, *et = nullptr;
  double *pmin, *pmax, *qmin, *qmax, *c2q, *c1l, *c2, *c1, *c0;
  double *adm, *vlo_i, *vhi_i, *vlo_j, *vhi_j, *rate2;
  double* rate = nullptr;     // [nl] unscaled ratings (solution quality)
  int* end_bus = nullptr;     // [2 nl] bus of each branch end
  double* qscratch = nullptr; // [2 nb + 4 nl] quality scratch (lazy)
  unsigned long long* qual = nullptr;  // [6 G] quality maxima (lazy)
  double *u, *v, *z, *y, *lam, *bx, *ltil, *rtil;
  double* calpha;  // [nl] TRON Cauchy step length of each branch's last solve
  // the second buffer of the x-step's results (u, branch state); between
  // chunks every grid's state is in the first
  double *u1 = nullptr, *bx1 = nullptr, *ltil1 = nullptr, *rtil1 = nullptr;
  double* calpha1 = nullptr;
  int* failures_it = nullptr;  // [2][G] branch failures of the results in each buffer
  double* brec = nullptr;  // [nl][16] branch records (v - z, y per coupling)
  int* erec = nullptr;     // [ne] record half of each branch end
  int *gptr, *eptr, *isref;
  std::vector<int> gptr_h, eptr_h;  // host copies, for the bus tiles
  std::vector<TileDesc> tiles_h;     // every bus tile of the handle
  std::vector<char> tile_hub;        // tile with more pairs than lanes
  int n_hub = 0;                     // hub tiles of the handle
  // layout of a lane's work lists (byte offsets of the tile, hub and grid
  // lists; room for xcap x-step items), the same for every lane
  size_t off_t = 0, off_h = 0, off_g = 0, list_bytes = 0;
  int64_t xcap = 0;
  std::vector<Lane> lanes;           // tune.lanes of them; lane 0 runs on `stream`
  std::vector<int> lane_of;          // [G] lane of each grid
  int* lane_of_d = nullptr;          // its device copy
  hipEvent_t join = nullptr;         // orders the lanes after work on `stream`
  int n_tiles = 0, tile_block = 0;
  double *pd, *qd, *gs, *bs;
  double *vmin_b, *vmax_b;  // [nb] voltage limits (solution quality)
  GridCtl* ctl;
  GridCtl* h_ctl = nullptr;  // pinned
  // pinned copies for results: every grid's control word, objective and
  // branch-failure count, read together (fetch_results)
  GridCtl* r_ctl = nullptr;
  double* r_obj = nullptr;
  int* r_fail = nullptr;
  unsigned long long* stats;
  double* tmax;          // [nb + 1][3] residual maxima per bus tile
  std::vector<int> grid_tile_h;  // [G + 1] tile range of each grid
  int* failures;
  int n_cu = 0;
  double* hist;
  int64_t* gen_off_d;
  int64_t* end_off_d;  // [G + 1] branch-end range of each grid
  double *base_d, *obj_d;
  bool solved = false;
  bool profile = false;
  bool count_stats = false;  // branch kernels count flops and events (slower)
  acopf_tuning tune{64, 256, kChunk, 1, 0, 0, 1};
  std::vector<double> t_start;         // host clock at each grid's start
  std::vector<double> t_end;           // host clock when it finished
  std::vector<char> running;           // started and not yet seen finished
  std::vector<char> started_once;
  std::vector<void*> snap;             // device snapshot buffers (lazy)
  std::vector<hipEvent_t> ev;
  double t_ms[kTimed] = {0, 0, 0};
  bool ev_ctl[kMaxLanes][kMaxChunk] = {};  // a control kernel ran in the profiled slot
  int64_t t_iters = 0;
};

namespace {

// The x-step's arguments for a lane, reading the branch state from buffer
// `in` and writing u and the branch state to buffer `out` (0 or 1).
BranchArgs branch_args(const acopf_s* h, const Lane& L, int in, int out) {
  BranchArgs A{};
  A.nl = h->nl;
  A.ne = h->ne;
  A.ef = h->ef;
  A.et = h->et;
  A.br_grid = h->br_grid;
  A.lane_of = h->lanes.size() > 1 ? h->lane_of_d : nullptr;
  A.lane = (int)(&L - h->lanes.data());
  A.ctl = h->ctl;
  A.adm = h->adm;
  A.vlo_i = h->vlo_i;
  A.vhi_i = h->vhi_i;
  A.vlo_j = h->vlo_j;
  A.vhi_j = h->vhi_j;
  A.rate2 = h->rate2;
  A.v = h->v;
  A.z = h->z;
  A.y = h->y;
  A.brec = h->brec;
  A.u = out ? h->u1 : h->u;
  A.bx_in = in ? h->bx1 : h->bx;
  A.ltil_in = in ? h->ltil1 : h->ltil;
  A.rtil_in = in ? h->rtil1 : h->rtil;
  A.calpha_in = in ? h->calpha1 : h->calpha;
  A.bx = out ? h->bx1 : h->bx;
  A.ltil = out ? h->ltil1 : h->ltil;
  A.rtil = out ? h->rtil1 : h->rtil;
  A.calpha = out ? h->calpha1 : h->calpha;
  A.rho_pq = h->P.rho_pq;
  A.rho_va = h->P.rho_va;
  A.tron_gtol = h->P.tron_gtol;
  A.tron_ftol = h->P.tron_ftol;
  A.al_tol = h->P.al_tol;
  A.al_shrink = h->P.al_shrink;
  A.al_rho_growth = h->P.al_rho_growth;
  A.al_rho_max = h->P.al_rho_max;
  A.tron_maxit = h->P.tron_maxit;
  A.al_maxit = h->P.al_maxit;
  A.failures = h->failures_it + (size_t)out * h->G;
  A.stats = h->stats;
  A.pool = L.pool;
  A.ng = h->ng;
  A.gen_grid = h->gen_grid;
  A.pmin = h->pmin;
  A.pmax = h->pmax;
  A.qmin = h->qmin;
  A.qmax = h->qmax;
  A.c2q = h->c2q;
  A.c1l = h->c1l;
  return A;
}

int blocks_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Bus tiles for workgroups of `block` lanes: runs of consecutive buses of one
// grid, at most block / 2 buses, whose coupling pairs (two per branch end,
// one per generator) fit the block's lanes. A single bus with more pairs
// than lanes (a hub) gets a tile of its own, flagged for the hub launch, which
// recomputes the pairs past the lanes from global memory. LDS per tile is
// 50 bytes per lane (51,200 at 1,024 lanes).
int build_tiles(acopf_s* h, int block) {
  const int tb = std::max(1, block / 2);
  std::vector<TileDesc> tiles;
  std::vector<int> grid_tile, hubs;
  tiles.reserve(h->nb / 8 + h->G + 1);
  for (int g = 0; g < h->G; ++g) {
    const HostGrid& H = h->grids[g];
    grid_tile.push_back((int)tiles.size());
    int64_t b = H.bus_off;
    const int64_t bend = H.bus_off + H.nb;
    while (b < bend) {
      int64_t c = b;
      while (c < bend && c - b < tb &&
             2 * (int64_t)(h->eptr_h[c + 1] - h->eptr_h[b]) +
                     (int64_t)(h->gptr_h[c + 1] - h->gptr_h[b]) <= block)
        ++c;
      c = std::max(c, b + 1);
      const int64_t pairs = 2 * (int64_t)(h->eptr_h[c] - h->eptr_h[b]) +
                            (int64_t)(h->gptr_h[c] - h->gptr_h[b]);
      if (pairs > block) hubs.push_back((int)tiles.size());
      tiles.push_back(TileDesc{(int)b, (int)c, h->eptr_h[b], h->eptr_h[c], h->gptr_h[b],
                               h->gptr_h[c], g, (int)tiles.size()});
      b = c;
    }
  }
  grid_tile.push_back((int)tiles.size());
  h->grid_tile_h = std::move(grid_tile);
  h->tile_hub.assign(tiles.size(), 0);
  for (int t : hubs) h->tile_hub[t] = 1;
  h->tiles_h = std::move(tiles);
  h->n_hub = (int)hubs.size();
  h->n_tiles = (int)h->tiles_h.size();
  h->tile_block = block;
  for (Lane& L : h->lanes) L.lists_dirty = true;
  return ACOPF_OK;
}

// A lane's control decision arguments (its device copy is the lane's `dec`).
DecideArgs decide_args(const acopf_s* h, const Lane& L) {
  return DecideArgs{h->ctl, h->tmax, reinterpret_cast<const GridItem*>(L.lists + h->off_g),
                    h->hist, h->failures, h->failures_it, h->P.eps_pri, h->P.eps_dual,
                    h->P.eps_z, h->P.beta_gamma, h->P.beta_omega, h->P.beta_max,
                    h->P.max_outer, h->P.max_inner, kHistCap, h->G};
}

// Whether the x-step takes the control decisions inside a chunk (its
// decision blocks); otherwise the control kernel takes every one. Counting
// mode keeps the control kernel, so that no branch solve past a grid's
// finish enters the counters.
bool fused_control(const acopf_s* h) { return h->tune.xstep_waves == 0 && !h->count_stats; }

// Launch inner iteration `slot` of a chunk (its position) for the grids of
// one lane, on the lane's stream; with profiling, events bracket each launch. The lane-per-branch x-step at position q reads
// the branch state from buffer q & 1 and writes its results to the other;
// with fused control it takes the previous iteration's decision in its first
// blocks at positions >= 1, and the control kernel takes the chunk's last one
// (`last`). The persistent x-step works in place (buffer 0), with the control
// kernel after every iteration.
void launch_iteration(acopf_s* h, int lane, int slot, bool last) {
  Lane& L = h->lanes[lane];
  hipStream_t s = L.stream;
  hipEvent_t* E =
      h->profile ? &h->ev[((size_t)lane * kMaxChunk + slot) * kEvPerIter] : nullptr;
  auto mark = [&](int k) {
    if (E) (void)hipEventRecord(E[k], s);
  };
  const bool persistent = h->tune.xstep_waves > 0, fused = fused_control(h);
  const int in = persistent ? 0 : (slot & 1), out = persistent ? 0 : ((slot + 1) & 1);
  BranchArgs ba = branch_args(h, L, in, out);
  mark(0);
  if (persistent)
    acopf_dev::launch_xstep_persistent(ba, h->n6, h->tune.xstep_waves * 4 * h->n_cu,
                                       h->count_stats, s);
  else
    acopf_dev::launch_xstep(ba, L.xlay, L.xlist, L.n_x, L.dec,
                            fused && slot > 0 ? L.n_gl : 0, slot, h->tune.xstep_block,
                            h->count_stats, s);
  mark(1);
  BusArgs bu{h->nb, h->ng, h->ne, reinterpret_cast<const TileDesc*>(L.lists + h->off_t),
             reinterpret_cast<const TileDesc*>(L.lists + h->off_h), h->bus_grid, h->ctl,
             h->gptr, h->eptr, h->pd, h->qd, h->gs, h->bs, h->isref, out ? h->u1 : h->u, h->lam,
             h->v, h->z, h->y, h->P.rho_pq, h->P.rho_va, h->tmax, h->erec, h->brec,
             h->P.lambda_max};
  const int bb = h->tile_block;
  hipLaunchKernelGGL(bus_kernel<false>, dim3(L.n_t), dim3(bb), bus_lds_bytes(h->tile_block), s,
                     bu);
  if (h->n_hub > 0)
    hipLaunchKernelGGL(bus_kernel<true>, dim3(L.n_hl), dim3(bb), bus_lds_bytes(h->tile_block),
                       s, bu);
  mark(2);
  const bool ctl = last || !fused;
  if (ctl)
    hipLaunchKernelGGL(ctl_kernel, dim3(L.n_gl), dim3(kCtlBlock), 0, s, decide_args(h, L), out);
  mark(3);
  if (E) h->ev_ctl[lane][slot] = ctl;
}

int validate_grid(const acopf_grid& g, int idx) {
  std::string p = "grid " + std::to_string(idx) + ": ";
  if (g.n_bus < 1 || g.n_branch < 1 || g.n_gen < 0)
    return fail(ACOPF_EINVAL, p + "need n_bus >= 1, n_branch >= 1, n_gen >= 0");
  if (!(g.base_mva > 0.0) || !std::isfinite(g.base_mva))
    return fail(ACOPF_EINVAL, p + "base_mva must be positive");
  if (g.ref_bus < 0 || g.ref_bus >= g.n_bus) return fail(ACOPF_EINVAL, p + "ref_bus out of range");
  const void* need[] = {g.pd, g.qd, g.gs, g.bs, g.vmin, g.vmax, g.br_from, g.br_to,
                        g.r, g.x, g.b, g.tap, g.shift, g.rate};
  for (const void* q : need)
    if (!q) return fail(ACOPF_EINVAL, p + "null array");
  if (g.n_gen > 0) {
    const void* needg[] = {g.gen_bus, g.pmin, g.pmax, g.qmin, g.qmax, g.c2, g.c1, g.c0};
    for (const void* q : needg)
      if (!q) return fail(ACOPF_EINVAL, p + "null generator array");
  }
  const double* bus_arrs[] = {g.pd, g.qd, g.gs, g.bs, g.vmin, g.vmax};
  for (const double* a : bus_arrs)
    if (!finite_all(a, g.n_bus)) return fail(ACOPF_EINVAL, p + "non-finite bus data");
  for (int i = 0; i < g.n_bus; ++i)
    if (!(g.vmin[i] > 0.0) || g.vmin[i] > g.vmax[i])
      return fail(ACOPF_EINVAL, p + "need 0 < vmin <= vmax at bus " + std::to_string(i));
  if (g.n_gen > 0) {
    const double* gen_arrs[] = {g.pmin, g.pmax, g.qmin, g.qmax, g.c2, g.c1, g.c0};
    for (const double* a : gen_arrs)
      if (!finite_all(a, g.n_gen)) return fail(ACOPF_EINVAL, p + "non-finite generator data");
    for (int k = 0; k < g.n_gen; ++k) {
      if (g.gen_bus[k] < 0 || g.gen_bus[k] >= g.n_bus)
        return fail(ACOPF_EINVAL, p + "gen_bus out of range");
      if (g.pmin[k] > g.pmax[k] || g.qmin[k] > g.qmax[k])
        return fail(ACOPF_EINVAL, p + "empty generator bound interval");
      if (g.c2[k] < 0.0) return fail(ACOPF_EINVAL, p + "negative quadratic cost");
    }
  }
  const double* br_arrs[] = {g.r, g.x, g.b, g.tap, g.shift, g.rate};
  for (const double* a : br_arrs)
    if (!finite_all(a, g.n_branch)) return fail(ACOPF_EINVAL, p + "non-finite branch data");
  std::vector<int> deg(g.n_bus, 0);
  for (int l = 0; l < g.n_branch; ++l) {
    const int i = g.br_from[l], j = g.br_to[l];
    if (i < 0 || i >= g.n_bus || j < 0 || j >= g.n_bus || i == j)
      return fail(ACOPF_EINVAL, p + "bad branch end at branch " + std::to_string(l));
    if (g.r[l] == 0.0 && g.x[l] == 0.0)
      return fail(ACOPF_EINVAL, p + "r = x = 0 at branch " + std::to_string(l));
    if (!(g.tap[l] > 0.0)) return fail(ACOPF_EINVAL, p + "tap must be positive");
    ++deg[i];
    ++deg[j];
  }
  for (int i = 0; i < g.n_bus; ++i)
    if (deg[i] == 0) return fail(ACOPF_EINVAL, p + "isolated bus " + std::to_string(i));
  return ACOPF_OK;
}

int validate_params(const acopf_params& P) {
  if (!(P.rho_pq > 0) || !(P.rho_va > 0)) return fail(ACOPF_EINVAL, "rho must be positive");
  if (!(P.beta0 > 0) || !(P.beta_max >= P.beta0) || !(P.beta_gamma >= 1.0))
    return fail(ACOPF_EINVAL, "need beta0 > 0, beta_max >= beta0, beta_gamma >= 1");
  if (!(P.obj_scale >= 0) || !(P.rate_scale > 0)) return fail(ACOPF_EINVAL, "bad scales");
  if (P.max_outer < 1 || P.max_inner < 1 || P.tron_maxit < 1 || P.al_maxit < 1)
    return fail(ACOPF_EINVAL, "iteration caps must be >= 1");
  if (!(P.al_rho0 > 0) || !(P.al_rho_max >= P.al_rho0) || !(P.lambda_max > 0))
    return fail(ACOPF_EINVAL, "bad AL or lambda parameters");
  return ACOPF_OK;
}

}  // namespace

extern "C" {

void acopf_default_params(acopf_params* p) {
  if (!p) return;
  p->rho_pq = 400.0;
  p->rho_va = 4000.0;
  p->obj_scale = 0.01;
  p->rate_scale = 0.99;
  p->beta0 = 1e4;
  p->beta_gamma = 6.0;
  p->beta_omega = 0.8;
  p->beta_max = 1e5;
  p->lambda_max = 1e12;
  p->eps_pri = 1e-4;
  p->eps_dual = 1e-4;
  p->eps_z = 1e-4;
  p->max_outer = 20;
  p->max_inner = 1000;
  p->tron_gtol = 1e-6;
  p->tron_ftol = 1e-12;
  p->tron_maxit = 50;
  p->al_rho0 = 10.0;
  p->al_rho_growth = 10.0;
  p->al_rho_max = 1e8;
  p->al_tol = 1e-6;
  p->al_shrink = 0.25;
  p->al_maxit = 20;
}

const char* acopf_last_error(void) { return g_err.c_str(); }

// Releases the last lane (its graph, lists, stream).
static void free_lane(acopf_s* h) {
  Lane& L = h->lanes.back();
  if (L.stream) (void)hipStreamSynchronize(L.stream);
  if (L.graph) (void)hipGraphExecDestroy(L.graph);
  if (L.gtmpl) (void)hipGraphDestroy(L.gtmpl);
  if (L.lists) (void)hipFree(L.lists);
  if (L.stage) (void)hipHostFree(L.stage);
  if (L.dec) (void)hipFree(L.dec);
  if (L.pool) (void)hipFree(L.pool);
  if (L.end) (void)hipEventDestroy(L.end);
  if (L.own_stream && L.stream) (void)hipStreamDestroy(L.stream);
  h->lanes.pop_back();
}

// A new lane: the first runs on the handle's stream, the others on streams
// of their own (default priority); each has its work lists, decision
// arguments and pool counters.
static int add_lane(acopf_s* h) {
  h->lanes.emplace_back();
  Lane& L = h->lanes.back();
  if (h->lanes.size() == 1) {
    L.stream = h->stream;
  } else {
    HIP_TRY(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
    L.own_stream = true;
    HIP_TRY(hipEventCreateWithFlags(&L.end, hipEventDisableTiming));
  }
  HIP_TRY(hipMalloc(reinterpret_cast<void**>(&L.lists), h->list_bytes));
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&L.stage), h->list_bytes, hipHostMallocDefault));
  HIP_TRY(hipMalloc(reinterpret_cast<void**>(&L.dec), sizeof(DecideArgs)));
  HIP_TRY(hipMalloc(reinterpret_cast<void**>(&L.pool), 3 * sizeof(unsigned)));
  const DecideArgs dv = decide_args(h, L);
  HIP_TRY(hipMemcpyAsync(L.dec, &dv, sizeof(dv), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemsetAsync(L.pool, 0, 3 * sizeof(unsigned), h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return ACOPF_OK;
}

// Grids to lanes: largest first (by branches, then buses) to the lane with
// the fewest branches so far.
static int assign_lanes(acopf_s* h) {
  const int nlanes = (int)h->lanes.size();
  std::vector<int> order(h->G);
  for (int g = 0; g < h->G; ++g) order[g] = g;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const HostGrid &A = h->grids[a], &B = h->grids[b];
    return A.nl != B.nl ? A.nl > B.nl : A.nb > B.nb;
  });
  std::vector<int64_t> load(nlanes, 0);
  h->lane_of.assign(h->G, 0);
  for (int g : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    h->lane_of[g] = k;
    load[k] += h->grids[g].nl + 1;
  }
  for (Lane& L : h->lanes) L.lists_dirty = true;
  HIP_TRY(hipMemcpyAsync(h->lane_of_d, h->lane_of.data(), sizeof(int) * h->G,
                         hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return ACOPF_OK;
}

// Sets the number of lanes (at most the number of grids) and reassigns the
// grids to them.
static int set_lanes(acopf_s* h, int n) {
  n = std::max(1, std::min(n, h->G));
  while ((int)h->lanes.size() > n) free_lane(h);
  while ((int)h->lanes.size() < n) {
    int rc = add_lane(h);
    if (rc) return rc;
  }
  return assign_lanes(h);
}

void acopf_destroy(acopf_handle h) {
  if (!h) return;
  if (h->device >= 0) (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  while (!h->lanes.empty()) free_lane(h);
  if (h->join) (void)hipEventDestroy(h->join);
  for (void* p : h->snap) (void)hipFree(p);
  if (h->qscratch) (void)hipFree(h->qscratch);
  if (h->qual) (void)hipFree(h->qual);
  h->buf.release();
  if (h->h_ctl) (void)hipHostFree(h->h_ctl);
  if (h->r_ctl) (void)hipHostFree(h->r_ctl);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

static int create_impl(const acopf_grid* grids, int32_t n_grids, const acopf_params* params,
                       int32_t device, void* hip_stream, acopf_s* h) {
  if (!grids || n_grids < 1 || !params) return fail(ACOPF_EINVAL, "need grids, n_grids >= 1, params");
  int rc = validate_params(*params);
  if (rc) return rc;
  for (int g = 0; g < n_grids; ++g) {
    rc = validate_grid(grids[g], g);
    if (rc) return rc;
  }
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(ACOPF_EINVAL, "device index out of range");
  HIP_TRY(hipSetDevice(device));
  h->device = device;
  HIP_TRY(hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, device));
  if (h->n_cu < 1) h->n_cu = 1;
  h->P = *params;
  h->G = n_grids;
  if (hip_stream) {
    h->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    HIP_TRY(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    h->own_stream = true;
  }

  // ---- sizes and orders
  h->grids.resize(n_grids);
  int64_t nb = 0, ng = 0, nl = 0, n6 = 0;
  for (int g = 0; g < n_grids; ++g) {
    const acopf_grid& G = grids[g];
    HostGrid& H = h->grids[g];
    H.nb = G.n_bus;
    H.ng = G.n_gen;
    H.nl = G.n_branch;
    H.bus_off = nb;
    H.gen_off = ng;
    H.ref = G.ref_bus;
    nb += G.n_bus;
    ng += G.n_gen;
    nl += G.n_branch;
    for (int l = 0; l < G.n_branch; ++l) n6 += G.rate[l] > 0.0 ? 1 : 0;
  }
  h->nb = nb;
  h->ng = ng;
  h->nl = nl;
  h->ne = 2 * nl;
  h->n6 = n6;
  h->m = 2 * ng + 8 * nl;
  if (nl >= (int64_t(1) << 30) || nb >= (int64_t(1) << 31))
    return fail(ACOPF_EINVAL, "problem too large for 32-bit element indices");
  // ---- per-bus counts -> CSR offsets of generators and branch ends
  std::vector<int> gptr(nb + 1, 0), eptr(nb + 1, 0);
  std::vector<int> fcount(nb, 0), tcount(nb, 0);
  for (int g = 0; g < n_grids; ++g) {
    const acopf_grid& G = grids[g];
    const HostGrid& H = h->grids[g];
    for (int k = 0; k < G.n_gen; ++k) ++gptr[H.bus_off + G.gen_bus[k] + 1];
    for (int l = 0; l < G.n_branch; ++l) {
      ++fcount[H.bus_off + G.br_from[l]];
      ++tcount[H.bus_off + G.br_to[l]];
    }
  }
  for (int64_t b = 0; b < nb; ++b) {
    gptr[b + 1] += gptr[b];
    eptr[b + 1] = eptr[b] + fcount[b] + tcount[b];
  }
  // generators: device order sorted by (grid, bus, input index); ends: per bus,
  // from-ends then to-ends, each in input order
  {
    std::vector<int> gpos(gptr.begin(), gptr.end() - 1), fpos(nb), tpos(nb);
    for (int64_t b = 0; b < nb; ++b) {
      fpos[b] = eptr[b];
      tpos[b] = eptr[b] + fcount[b];
    }
    for (int g = 0; g < n_grids; ++g) {
      const acopf_grid& G = grids[g];
      HostGrid& H = h->grids[g];
      H.gen_dev.resize(G.n_gen);
      for (int k = 0; k < G.n_gen; ++k) H.gen_dev[k] = gpos[H.bus_off + G.gen_bus[k]]++;
      H.end_f.resize(G.n_branch);
      H.end_t.resize(G.n_branch);
      for (int l = 0; l < G.n_branch; ++l) {
        H.end_f[l] = fpos[H.bus_off + G.br_from[l]]++;
        H.end_t[l] = tpos[H.bus_off + G.br_to[l]]++;
      }
      // each grid's generators occupy [gen_off, gen_off + ng) of the device order
    }
  }
  // branches: rated first, then unlimited; each by (grid, from bus, input index)
  std::vector<int> dev_grid(nl), ef(nl), et(nl);
  {
    std::vector<std::pair<int64_t, std::pair<int, int>>> r6, r4;  // (key, (grid, l))
    for (int g = 0; g < n_grids; ++g) {
      const acopf_grid& G = grids[g];
      const HostGrid& H = h->grids[g];
      for (int l = 0; l < G.n_branch; ++l) {
        const int64_t key = (H.bus_off + G.br_from[l]) * (int64_t)(1 << 30) + l;
        (G.rate[l] > 0.0 ? r6 : r4).push_back({key, {g, l}});
      }
    }
    std::sort(r6.begin(), r6.end());
    std::sort(r4.begin(), r4.end());
    int64_t d = 0;
    for (int cls = 0; cls < 2; ++cls) {
      auto& lst = cls == 0 ? r6 : r4;
      for (int g = 0; g < n_grids; ++g) {
        HostGrid& H = h->grids[g];
        (cls == 0 ? H.r6b : H.r4b) = d;
        (cls == 0 ? H.r6e : H.r4e) = d;
      }
      for (auto& it : lst) {
        const int g = it.second.first, l = it.second.second;
        HostGrid& H = h->grids[g];
        if (H.br_dev.empty()) H.br_dev.assign(H.nl, -1);
        if ((cls == 0 ? H.r6e : H.r4e) == (cls == 0 ? H.r6b : H.r4b)) (cls == 0 ? H.r6b : H.r4b) = d;
        H.br_dev[l] = d;
        dev_grid[d] = g;
        ef[d] = (int)H.end_f[l];
        et[d] = (int)H.end_t[l];
        ++d;
        (cls == 0 ? H.r6e : H.r4e) = d;
      }
    }
    for (int g = 0; g < n_grids; ++g) {
      HostGrid& H = h->grids[g];
      H.e0 = eptr[H.bus_off];
      H.e1 = eptr[H.bus_off + H.nb];
    }
  }
  // ---- host arrays in device order
  std::vector<int> gen_grid(ng), bus_grid(nb), isref(nb, 0);
  std::vector<double> pmin(ng), pmax(ng), qmin(ng), qmax(ng), c2q(ng), c1l(ng), c2(ng),
      c1(ng), c0(ng);
  std::vector<double> adm(8 * nl), vlo_i(nl), vhi_i(nl), vlo_j(nl), vhi_j(nl), rate2(nl),
      rate(nl);
  std::vector<double> pd(nb), qd(nb), gs(nb), bs(nb), vmin_b(nb), vmax_b(nb);
  std::vector<int64_t> gen_off(n_grids + 1, 0);
  std::vector<double> base(n_grids);
  const double s = params->obj_scale;
  for (int g = 0; g < n_grids; ++g) {
    const acopf_grid& G = grids[g];
    const HostGrid& H = h->grids[g];
    const double B = G.base_mva;
    base[g] = B;
    gen_off[g] = H.gen_off;
    gen_off[g + 1] = H.gen_off + H.ng;
    for (int k = 0; k < G.n_gen; ++k) {
      const int64_t d = H.gen_dev[k];
      gen_grid[d] = g;
      pmin[d] = G.pmin[k];
      pmax[d] = G.pmax[k];
      qmin[d] = G.qmin[k];
      qmax[d] = G.qmax[k];
      c2[d] = G.c2[k];
      c1[d] = G.c1[k];
      c0[d] = G.c0[k];
      c2q[d] = 2.0 * s * G.c2[k] * B * B;
      c1l[d] = s * G.c1[k] * B;
    }
    for (int i = 0; i < G.n_bus; ++i) {
      const int64_t d = H.bus_off + i;
      bus_grid[d] = g;
      pd[d] = G.pd[i];
      qd[d] = G.qd[i];
      gs[d] = G.gs[i];
      vmin_b[d] = G.vmin[i];
      vmax_b[d] = G.vmax[i];
      bs[d] = G.bs[i];
      isref[d] = i == G.ref_bus;
    }
    for (int l = 0; l < G.n_branch; ++l) {
      const int64_t d = H.br_dev[l];
      // pi model (below eq. acopf): series y = 1/(r + jx) = yr + j yi,
      // charging j b/2 at each end, turns ratio a = tap e^{j shift} = ar + j ai:
      //   (y + j b/2)/|a|^2,  -y/conj(a) = -y a/|a|^2,  -y/a = -y conj(a)/|a|^2,
      //   y + j b/2, expanded in real arithmetic.
      const double r = G.r[l], xx = G.x[l];
      const double den = r * r + xx * xx;
      const double yr = r / den, yi = -xx / den;
      const double ar = G.tap[l] * std::cos(G.shift[l]);
      const double ai = G.tap[l] * std::sin(G.shift[l]);
      const double a2 = G.tap[l] * G.tap[l];
      const double hb = 0.5 * G.b[l];
      adm[0 * nl + d] = yr / a2;
      adm[1 * nl + d] = (yi + hb) / a2;
      adm[2 * nl + d] = -(yr * ar - yi * ai) / a2;
      adm[3 * nl + d] = -(yr * ai + yi * ar) / a2;
      adm[4 * nl + d] = -(yr * ar + yi * ai) / a2;
      adm[5 * nl + d] = -(yi * ar - yr * ai) / a2;
      adm[6 * nl + d] = yr;
      adm[7 * nl + d] = yi + hb;
      const int i = G.br_from[l], j = G.br_to[l];
      vlo_i[d] = G.vmin[i];
      vhi_i[d] = G.vmax[i];
      vlo_j[d] = G.vmin[j];
      vhi_j[d] = G.vmax[j];
      const double rs = G.rate[l] * params->rate_scale;
      rate2[d] = G.rate[l] > 0.0 ? rs * rs : 0.0;
      rate[d] = G.rate[l];
    }
  }
  // ---- device allocation and upload
  DevBuf& D = h->buf;
  const int64_t m = h->m;
  HIP_TRY(D.alloc(&h->gen_grid, ng));
  HIP_TRY(D.alloc(&h->br_grid, nl));
  HIP_TRY(D.alloc(&h->bus_grid, nb));
  HIP_TRY(D.alloc(&h->ef, nl));
  HIP_TRY(D.alloc(&h->et, nl));
  double** gen_d[] = {&h->pmin, &h->pmax, &h->qmin, &h->qmax, &h->c2q, &h->c1l, &h->c2, &h->c1, &h->c0};
  for (double** p : gen_d) HIP_TRY(D.alloc(p, ng));
  HIP_TRY(D.alloc(&h->adm, 8 * nl));
  double** br_d[] = {&h->vlo_i, &h->vhi_i, &h->vlo_j, &h->vhi_j, &h->rate2, &h->rtil,
                     &h->calpha, &h->rate};
  for (double** p : br_d) HIP_TRY(D.alloc(p, nl));
  HIP_TRY(D.alloc(&h->end_bus, 2 * nl));
  HIP_TRY(D.alloc(&h->bx, 6 * nl));
  HIP_TRY(D.alloc(&h->brec, 16 * nl));
  HIP_TRY(D.alloc(&h->erec, 2 * nl));
  HIP_TRY(D.alloc(&h->ltil, 2 * nl));
  double** cp_d[] = {&h->u, &h->v, &h->z, &h->y, &h->lam, &h->u1};
  for (double** p : cp_d) HIP_TRY(D.alloc(p, m));
  HIP_TRY(D.alloc(&h->bx1, 6 * nl));
  HIP_TRY(D.alloc(&h->ltil1, 2 * nl));
  HIP_TRY(D.alloc(&h->rtil1, nl));
  HIP_TRY(D.alloc(&h->calpha1, nl));
  HIP_TRY(D.alloc(&h->gptr, nb + 1));
  {
    // work lists: x-step blocks (at least 64 lanes per block, plus a partial
    // block per class), bus and hub tiles (at most one tile per bus, plus a
    // placeholder), grids
    auto up16 = [](size_t b) { return (b + 15) & ~size_t(15); };
    h->xcap = (ng + nl) / 64 + 3 * (int64_t)n_grids + 8;
    h->off_t = up16(sizeof(int) * (size_t)h->xcap);
    h->off_h = h->off_t + up16(sizeof(TileDesc) * (size_t)(nb + 1));
    h->off_g = h->off_h + up16(sizeof(TileDesc) * (size_t)(nb + 1));
    h->list_bytes = h->off_g + up16(sizeof(GridItem) * (size_t)n_grids);
  }
  HIP_TRY(D.alloc(&h->eptr, nb + 1));
  HIP_TRY(D.alloc(&h->isref, nb));
  double** bus_d[] = {&h->pd, &h->qd, &h->gs, &h->bs, &h->vmin_b, &h->vmax_b};
  for (double** p : bus_d) HIP_TRY(D.alloc(p, nb));
  HIP_TRY(D.alloc(&h->ctl, n_grids));
  HIP_TRY(D.alloc(&h->tmax, 3 * (nb + 1)));
  HIP_TRY(D.alloc(&h->stats, kStats));
  HIP_TRY(D.alloc(&h->failures, n_grids));
  HIP_TRY(D.alloc(&h->failures_it, 2 * (size_t)n_grids));
  HIP_TRY(D.alloc(&h->lane_of_d, n_grids));
  HIP_TRY(D.alloc(&h->hist, (size_t)n_grids * kHistCap * 6));
  HIP_TRY(D.alloc(&h->gen_off_d, n_grids + 1));
  HIP_TRY(D.alloc(&h->end_off_d, n_grids + 1));
  HIP_TRY(D.alloc(&h->base_d, n_grids));
  HIP_TRY(D.alloc(&h->obj_d, n_grids));
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->h_ctl), sizeof(GridCtl) * n_grids,
                        hipHostMallocDefault));
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->r_ctl),
                        (sizeof(GridCtl) + sizeof(double) + sizeof(int)) * n_grids,
                        hipHostMallocDefault));
  h->r_obj = reinterpret_cast<double*>(h->r_ctl + n_grids);
  h->r_fail = reinterpret_cast<int*>(h->r_obj + n_grids);
  hipStream_t st = h->stream;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  };
  HIP_TRY(up(h->gen_grid, gen_grid.data(), sizeof(int) * ng));
  HIP_TRY(up(h->br_grid, dev_grid.data(), sizeof(int) * nl));
  HIP_TRY(up(h->bus_grid, bus_grid.data(), sizeof(int) * nb));
  HIP_TRY(up(h->ef, ef.data(), sizeof(int) * nl));
  HIP_TRY(up(h->et, et.data(), sizeof(int) * nl));
  std::vector<int> erec(2 * nl);
  for (int64_t d = 0; d < nl; ++d) {
    erec[ef[d]] = (int)(2 * d);
    erec[et[d]] = (int)(2 * d + 1);
  }
  HIP_TRY(up(h->erec, erec.data(), sizeof(int) * 2 * nl));
  const std::vector<double>* gen_h[] = {&pmin, &pmax, &qmin, &qmax, &c2q, &c1l, &c2, &c1, &c0};
  for (int q = 0; q < 9; ++q) HIP_TRY(up(*gen_d[q], gen_h[q]->data(), sizeof(double) * ng));
  HIP_TRY(up(h->adm, adm.data(), sizeof(double) * 8 * nl));
  HIP_TRY(up(h->vlo_i, vlo_i.data(), sizeof(double) * nl));
  HIP_TRY(up(h->vhi_i, vhi_i.data(), sizeof(double) * nl));
  HIP_TRY(up(h->vlo_j, vlo_j.data(), sizeof(double) * nl));
  HIP_TRY(up(h->vhi_j, vhi_j.data(), sizeof(double) * nl));
  HIP_TRY(up(h->rate2, rate2.data(), sizeof(double) * nl));
  HIP_TRY(up(h->rate, rate.data(), sizeof(double) * nl));
  {
    std::vector<int> end_bus(2 * nl);
    for (int64_t b = 0; b < nb; ++b)
      for (int e = eptr[b]; e < eptr[b + 1]; ++e) end_bus[e] = (int)b;
    HIP_TRY(up(h->end_bus, end_bus.data(), sizeof(int) * 2 * nl));
  }
  HIP_TRY(up(h->gptr, gptr.data(), sizeof(int) * (nb + 1)));
  h->gptr_h = gptr;
  h->eptr_h = eptr;
  HIP_TRY(up(h->eptr, eptr.data(), sizeof(int) * (nb + 1)));
  HIP_TRY(up(h->isref, isref.data(), sizeof(int) * nb));
  HIP_TRY(up(h->pd, pd.data(), sizeof(double) * nb));
  HIP_TRY(up(h->qd, qd.data(), sizeof(double) * nb));
  HIP_TRY(up(h->gs, gs.data(), sizeof(double) * nb));
  HIP_TRY(up(h->bs, bs.data(), sizeof(double) * nb));
  HIP_TRY(up(h->vmin_b, vmin_b.data(), sizeof(double) * nb));
  HIP_TRY(up(h->vmax_b, vmax_b.data(), sizeof(double) * nb));
  HIP_TRY(up(h->gen_off_d, gen_off.data(), sizeof(int64_t) * (n_grids + 1)));
  std::vector<int64_t> end_off(n_grids + 1);
  for (int g = 0; g < n_grids; ++g) end_off[g] = h->grids[g].e0;
  end_off[n_grids] = 2 * nl;
  HIP_TRY(up(h->end_off_d, end_off.data(), sizeof(int64_t) * (n_grids + 1)));
  HIP_TRY(up(h->base_d, base.data(), sizeof(double) * n_grids));
  HIP_TRY(hipMemsetAsync(h->stats, 0, sizeof(unsigned long long) * kStats, st));
  HIP_TRY(hipMemsetAsync(h->hist, 0, sizeof(double) * (size_t)n_grids * kHistCap * 6, st));
  HIP_TRY(hipMemsetAsync(h->ctl, 0, sizeof(GridCtl) * n_grids, st));
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipEventCreateWithFlags(&h->join, hipEventDisableTiming));
  // two lanes for a handle of several grids, one for a single grid
  h->tune.lanes = n_grids > 1 ? 2 : 1;
  int rc2 = set_lanes(h, h->tune.lanes);
  if (rc2) return rc2;
  return build_tiles(h, h->tune.bus_block);
}

static int ensure_graph(acopf_s* h);

// Address of `scratch` on each device, resolved once per device with that
// device current (at the first acopf_create on it).
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

static int noalloc_scratch(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return fail(ACOPF_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != device) HIP_TRY(hipSetDevice(device));
    double* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&ptr), HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr)
      return fail(ACOPF_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return ACOPF_OK;
}

int acopf_create(const acopf_grid* grids, int32_t n_grids, const acopf_params* params,
                 int32_t device, void* hip_stream, acopf_handle* out) {
  if (!out) return fail(ACOPF_EINVAL, "out is null");
  *out = nullptr;
  auto* h = new (std::nothrow) acopf_s();
  if (!h) return fail(ACOPF_ENOMEM, "host allocation failed");
  h->device = -1;
  int rc = create_impl(grids, n_grids, params, device, hip_stream, h);
  if (rc) {
    std::string msg = g_err;
    acopf_destroy(h);
    g_err = msg;
    return rc == ACOPF_EDEVICE && msg.find("hipMalloc") != std::string::npos ? ACOPF_ENOMEM : rc;
  }
  // cold state so that get_state is meaningful before the first solve
  ColdArgs ca{-1, h->ng, h->nl, h->ne, h->m, h->ef, h->et, h->gen_grid, h->br_grid, h->pmin, h->pmax, h->qmin, h->qmax,
              h->adm, h->vlo_i, h->vhi_i, h->vlo_j, h->vhi_j, h->rate2, h->n6,
              h->u, h->v, h->z, h->y, h->lam, h->bx, h->ltil, h->rtil, h->calpha,
              h->P.al_rho0};
  hipLaunchKernelGGL(cold_kernel, dim3(blocks_for(h->ng + h->nl, 256)), dim3(256), 0, h->stream, ca);
  hipLaunchKernelGGL(ctl_start_kernel, dim3(blocks_for(h->G, 64)), dim3(64), 0, h->stream,
                     h->ctl, h->G, -1, (int)ACOPF_COLD, 0, h->P.beta0, h->failures,
                     h->failures_it);
  hipLaunchKernelGGL(ctl_idle_kernel, dim3(blocks_for(h->G, 64)), dim3(64), 0, h->stream,
                     h->ctl, h->G);
  h->t_start.assign(h->G, 0.0);
  h->t_end.assign(h->G, 0.0);
  h->running.assign(h->G, 0);
  h->started_once.assign(h->G, 0);
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    acopf_destroy(h);
    return fail(ACOPF_EDEVICE, std::string("cold start: ") + hipGetErrorString(e));
  }
  double* sp = nullptr;
  rc = noalloc_scratch(h->device, &sp);
  if (!rc) rc = ensure_graph(h);
  if (rc) {
    std::string msg = g_err;
    acopf_destroy(h);
    g_err = msg;
    return rc;
  }
  *out = h;
  return ACOPF_OK;
}

// Adds the profiled launches of a chunk of `used` iterations of the lanes
// that ran (one after another): per iteration, the sum over those lanes.
static void accumulate_timing(acopf_s* h, int used, const std::vector<int>& ran) {
  for (int lane : ran)
    for (int s = 0; s < used; ++s) {
      hipEvent_t* E = &h->ev[((size_t)lane * kMaxChunk + s) * kEvPerIter];
      for (int k = 0; k < kTimed; ++k) {
        if (k == 2 && !h->ev_ctl[lane][s]) continue;  // no control kernel after this iteration
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, E[k], E[k + 1]) == hipSuccess) h->t_ms[k] += ms;
      }
    }
  h->t_iters += used;
}

static void drop_graph(Lane& L) {
  if (L.graph) (void)hipGraphExecDestroy(L.graph);
  if (L.gtmpl) (void)hipGraphDestroy(L.gtmpl);
  L.graph = nullptr;
  L.gtmpl = nullptr;
  L.graph_chunk = 0;
  L.gnode.clear();
  L.grole.clear();
  L.gparam.clear();
}

static void drop_graph(acopf_s* h) {
  for (Lane& L : h->lanes) drop_graph(L);
}

// Grid size of a captured kernel node of the given role under the lane's
// current work lists.
static unsigned role_blocks(const Lane& L, int role) {
  switch (role) {
    case 0: return (unsigned)L.n_x;
    case 1: return (unsigned)L.n_t;
    case 2: return (unsigned)L.n_hl;
    default: return (unsigned)L.n_gl;
  }
}

// Work lists of a lane's grids that are running (of all its grids when none
// is: the shape a chunk is captured with): x-step items over the generator, rated
// and unlimited ranges of those grids (adjacent ranges merged, so that with
// every grid running the items are those of one contiguous range per class),
// their bus tiles and hub tiles, and the grids themselves. The kernel nodes of
// a captured chunk take the new grid sizes in place; their arguments point to
// the lists and do not change.
static int build_active(acopf_s* h, int lane) {
  Lane& LN = h->lanes[lane];
  std::vector<char> act(h->G, 0);
  for (int g = 0; g < h->G; ++g) act[g] = h->running[g] && h->lane_of[g] == lane;
  if (std::find(act.begin(), act.end(), 1) == act.end())
    for (int g = 0; g < h->G; ++g) act[g] = h->lane_of[g] == lane;
  if (!LN.lists_dirty && act == LN.active_for) return ACOPF_OK;
  HIP_TRY(hipStreamSynchronize(LN.stream));  // the last copy from `stage` has landed
  // x-step: the block layout over the handle's ranges, with the unlimited
  // branches per lane chosen for the running grids (as many as it takes for
  // every branch wavefront to be resident at once, one per SIMD slot, unless
  // tuned), and the layout blocks that touch a running grid
  const int bs = h->tune.xstep_block;
  const int64_t n4_all = h->nl - h->n6;
  int64_t waves6 = 0, n4 = 0;
  bool all = true;
  for (int g = 0; g < h->G; ++g) {
    if (!act[g]) {
      all = false;
      continue;
    }
    const HostGrid& H = h->grids[g];
    waves6 += (H.r6e - H.r6b + bs - 1) / bs * ((bs + 63) / 64);
    n4 += H.r4e - H.r4b;
  }
  const int64_t slots = 4 * (int64_t)h->n_cu;
  int k4 = h->tune.xstep_per_lane;
  if (k4 <= 0) {
    // two per lane when that makes every branch wavefront resident at once;
    // otherwise one (more per lane would make the unlimited wavefronts longer
    // than the rated ones: on two 70k grids, eight per lane took 63 µs per
    // grid-iteration against 36 with one or two)
    const int64_t free_lanes = (slots - waves6) * 64;
    k4 = 1;
    if (free_lanes > 0 && (n4 + free_lanes - 1) / free_lanes == 2) k4 = 2;
  }
  acopf_dev::XLayout& L = LN.xlay;
  L.n6 = h->n6;
  L.bg = (int)((h->ng + bs - 1) / bs);
  L.b6 = (int)((h->n6 + bs - 1) / bs);
  L.b4 = (int)((n4_all + (int64_t)bs * k4 - 1) / ((int64_t)bs * k4));
  L.k4 = k4;
  int nx = L.bg + L.b6 + L.b4;
  LN.xlist = nullptr;
  if (!all) {
    std::vector<char> use((size_t)nx, 0);
    auto mark = [&](int64_t off, int64_t a, int64_t e) {  // blocks off + [a / bs, (e - 1) / bs]
      for (int64_t k = a / bs; a < e && k <= (e - 1) / bs; ++k) use[(size_t)(off + k)] = 1;
    };
    const int64_t span = (int64_t)L.b4 * bs;  // branches between a lane's unlimited solves
    for (int g = 0; g < h->G; ++g) {
      if (!act[g]) continue;
      const HostGrid& H = h->grids[g];
      mark(L.b6 + L.b4, H.gen_off, H.gen_off + H.ng);
      mark(0, H.r6b, H.r6e);
      // unlimited offsets o = l - n6: block u holds o = u bs + [0, bs) + j span
      int64_t a = H.r4b - h->n6, e = H.r4e - h->n6;
      if (e - a >= span) a = 0, e = span;
      for (int64_t o = a; o < e;) {
        const int64_t q = o % span, stop = std::min(e, o + (span - q));
        mark(L.b6, q, q + (stop - o));
        o = stop;
      }
    }
    int* xl = reinterpret_cast<int*>(LN.stage);
    nx = 0;
    for (size_t k = 0; k < use.size(); ++k)
      if (use[k]) xl[nx++] = (int)k;
    LN.xlist = reinterpret_cast<const int*>(LN.lists);
  }
  if (nx > h->xcap) return fail(ACOPF_EDEVICE, "x-step block list overflow");
  TileDesc* tl = reinterpret_cast<TileDesc*>(LN.stage + h->off_t);
  TileDesc* hl = reinterpret_cast<TileDesc*>(LN.stage + h->off_h);
  GridItem* gl = reinterpret_cast<GridItem*>(LN.stage + h->off_g);
  int nt = 0, nh = 0, ngl = 0;
  for (int g = 0; g < h->G; ++g) {
    if (!act[g]) continue;
    gl[ngl++] = GridItem{g, h->grid_tile_h[g], h->grid_tile_h[g + 1], 0};
  }
  for (int t = 0; t < h->n_tiles; ++t) {
    const TileDesc& D = h->tiles_h[t];
    if (!act[D.grid]) continue;
    if (h->tile_hub[t]) hl[nh++] = D;
    else tl[nt++] = D;
  }
  const TileDesc none{0, 0, 0, 0, 0, 0, 0, -1};
  if (nt == 0) tl[nt++] = none;  // a launch needs one block; it returns at once
  if (nh == 0) hl[nh++] = none;
  hipStream_t st = LN.stream;
  if (LN.xlist)
    HIP_TRY(hipMemcpyAsync(LN.lists, LN.stage, sizeof(int) * nx, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(LN.lists + h->off_t, tl, sizeof(TileDesc) * nt, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(LN.lists + h->off_h, hl, sizeof(TileDesc) * nh, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(LN.lists + h->off_g, gl, sizeof(GridItem) * ngl, hipMemcpyHostToDevice,
                         st));
  LN.n_x = nx;
  LN.n_t = nt;
  LN.n_hl = nh;
  LN.n_gl = ngl;
  LN.active_for = act;
  LN.lists_dirty = false;
  LN.xba[0] = branch_args(h, LN, 0, 1);
  LN.xba[1] = branch_args(h, LN, 1, 0);
  for (size_t i = 0; LN.graph && i < LN.gnode.size(); ++i) {
    if (LN.grole[i] < 0) continue;
    hipKernelNodeParams p = LN.gparam[i];
    p.gridDim = dim3(role_blocks(LN, LN.grole[i]));
    // an x-step node keeps its chunk position; its decision blocks follow
    // the running grids
    int pos = 0, n_dec = 0;
    void* xargs[10] = {nullptr, &L.n6, &L.bg, &L.b6, &L.b4, &L.k4, &LN.xlist, &LN.dec, &n_dec,
                       &pos};
    if (LN.grole[i] == 0) {
      pos = *static_cast<const int*>(LN.gparam[i].kernelParams[9]);
      n_dec = pos > 0 && fused_control(h) ? LN.n_gl : 0;
      xargs[0] = &LN.xba[pos & 1];
      p.gridDim = dim3((unsigned)(n_dec + LN.n_x));
      p.kernelParams = xargs;
    }
    HIP_TRY(hipGraphExecKernelNodeSetParams(LN.graph, LN.gnode[i], &p));
  }
  return ACOPF_OK;
}

// Captures one chunk of the tuned length of a lane as a hipGraph (without
// per-launch timing events) if graphs are on and none is held. Called when
// the launch shape or the kernel variant changes, so that capture and
// instantiation happen outside the solves that replay the graph. Its kernel
// nodes are kept so that build_active can resize them to the running grids.
static int ensure_graph(acopf_s* h, int lane) {
  Lane& L = h->lanes[lane];
  const int k = h->tune.chunk;
  if (!h->tune.use_graph || (L.graph && L.graph_chunk == k)) return ACOPF_OK;
  drop_graph(L);
  int rc = build_active(h, lane);
  if (rc) return rc;
  const bool prof = h->profile;
  h->profile = false;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(L.stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int c = 0; c < k; ++c) launch_iteration(h, lane, c, c == k - 1);
    e = hipStreamEndCapture(L.stream, &g);
  }
  h->profile = prof;
  if (e != hipSuccess) return fail(ACOPF_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  size_t n = 0;
  e = hipGraphGetNodes(g, nullptr, &n);
  std::vector<hipGraphNode_t> nodes(n);
  if (e == hipSuccess && n) e = hipGraphGetNodes(g, nodes.data(), &n);
  for (size_t i = 0; e == hipSuccess && i < n; ++i) {
    hipGraphNodeType ty;
    e = hipGraphNodeGetType(nodes[i], &ty);
    if (e != hipSuccess || ty != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams p;
    e = hipGraphKernelNodeGetParams(nodes[i], &p);
    if (e != hipSuccess) break;
    int role = -1;
    if (acopf_dev::is_xstep_kernel(p.func)) role = 0;
    else if (p.func == reinterpret_cast<void*>(&bus_kernel<false>)) role = 1;
    else if (p.func == reinterpret_cast<void*>(&bus_kernel<true>)) role = 2;
    else if (p.func == reinterpret_cast<void*>(&ctl_kernel)) role = 3;
    L.gnode.push_back(nodes[i]);
    L.grole.push_back(role);
    L.gparam.push_back(p);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&L.graph, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    L.graph = nullptr;
    drop_graph(L);
    return fail(ACOPF_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  }
  L.gtmpl = g;
  L.graph_chunk = k;
  return ACOPF_OK;
}

static int ensure_graph(acopf_s* h) {
  for (int lane = 0; lane < (int)h->lanes.size(); ++lane) {
    int rc = ensure_graph(h, lane);
    if (rc) return rc;
  }
  return ACOPF_OK;
}

// k inner iterations of a lane: one replay of its captured chunk when k
// equals the tuned chunk and timing is off, else plain launches.
static int launch_chunk(acopf_s* h, int lane, int k) {
  Lane& L = h->lanes[lane];
  if (!h->profile && h->tune.use_graph && k == h->tune.chunk) {
    int rc = ensure_graph(h, lane);
    if (rc) return rc;
    HIP_TRY(hipGraphLaunch(L.graph, L.stream));
    return ACOPF_OK;
  }
  for (int c = 0; c < k; ++c) launch_iteration(h, lane, c, c == k - 1);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

static int start_impl(acopf_s* h, int grid, int mode, int fixed_iters) {
  hipStream_t st = h->stream;
  if (mode == ACOPF_COLD) {
    ColdArgs ca{grid, h->ng, h->nl, h->ne, h->m, h->ef, h->et, h->gen_grid, h->br_grid,
                h->pmin, h->pmax, h->qmin, h->qmax, h->adm, h->vlo_i, h->vhi_i, h->vlo_j,
                h->vhi_j, h->rate2, h->n6, h->u, h->v, h->z, h->y, h->lam, h->bx, h->ltil,
                h->rtil, h->calpha, h->P.al_rho0};
    hipLaunchKernelGGL(cold_kernel, dim3(blocks_for(h->ng + h->nl, 256)), dim3(256), 0, st, ca);
  }
  // branch records from the state the solve starts from (the host may have
  // changed v, z or y since the last bus step)
  const int64_t e0 = grid < 0 ? 0 : h->grids[grid].e0, e1 = grid < 0 ? h->ne : h->grids[grid].e1;
  if (e1 > e0)
    hipLaunchKernelGGL(record_kernel, dim3(blocks_for(e1 - e0, 256)), dim3(256), 0, st, h->ng,
                       e0, e1, h->erec, h->v, h->z, h->y, h->brec);
  hipLaunchKernelGGL(ctl_start_kernel, dim3(blocks_for(h->G, 64)), dim3(64), 0, st, h->ctl,
                     h->G, grid, mode, fixed_iters, h->P.beta0, h->failures, h->failures_it);
  HIP_TRY(hipGetLastError());
  const double t = now_s();
  for (int g = 0; g < h->G; ++g)
    if (grid < 0 || g == grid) {
      h->running[g] = 1;
      h->started_once[g] = 1;
      h->t_start[g] = t;
    }
  return ACOPF_OK;
}

// Iterate until some running grid finishes (stop_on_first) or all have
// finished, or max_iters iterations ran. Returns the iterations issued.
// Applies the outer multiplier steps still pending after a run (decided by
// a grid's last iteration before it finished or the run stopped), so that
// between calls no step is pending and lambda is what Algorithm 1 holds. The
// control words were read after the run's last chunk.
static int settle_outer(acopf_s* h) {
  bool any = false;
  for (int g = 0; g < h->G; ++g) {
    const GridCtl& c = h->h_ctl[g];
    if (!c.do_outer) continue;
    const HostGrid& H = h->grids[g];
    const int64_t c0 = 2 * h->ng + 4 * H.e0, c1 = 2 * h->ng + 4 * H.e1;
    const int64_t n = 2 * H.ng + (c1 - c0);
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4 * (int64_t)h->n_cu);
    hipLaunchKernelGGL(outer_step_kernel, dim3(blocks), dim3(256), 0, h->stream, h->ctl, g,
                       h->ng, H.gen_off, H.gen_off + H.ng, c0, c1, c.beta_lam, h->P.lambda_max,
                       h->z, h->lam);
    any = true;
  }
  if (!any) return ACOPF_OK;
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (int g = 0; g < h->G; ++g) h->h_ctl[g].do_outer = 0;
  return ACOPF_OK;
}

// Moves the x-step results (u and the branch state) of every grid whose last
// accepted iteration wrote the second buffer (a grid that finished at an odd
// chunk position, or every running grid after a chunk of odd length) into
// the first, where the next chunk and every other part of the library read
// them. The control words were read after the chunk.
static int settle_buffers(acopf_s* h) {
  for (int g = 0; g < h->G; ++g) {
    if (!h->h_ctl[g].cur) continue;
    const HostGrid& H = h->grids[g];
    CopySegs C{};
    int64_t longest = 0;
    auto cp = [&](const double* src, double* dst, int64_t from, int64_t n) {
      if (n <= 0) return;
      C.src[C.n] = src + from;
      C.dst[C.n] = dst + from;
      C.len[C.n] = n;
      longest = std::max(longest, n);
      ++C.n;
    };
    const int64_t ng = h->ng, nl = h->nl;
    cp(h->u1, h->u, H.gen_off, H.ng);
    cp(h->u1, h->u, ng + H.gen_off, H.ng);
    cp(h->u1, h->u, 2 * ng + 4 * H.e0, 4 * (H.e1 - H.e0));
    for (int r = 0; r < 6; ++r) {  // the slacks (rows 4, 5) of rated branches only
      cp(h->bx1, h->bx, r * nl + H.r6b, H.r6e - H.r6b);
      if (r < 4) cp(h->bx1, h->bx, r * nl + H.r4b, H.r4e - H.r4b);
    }
    for (int r = 0; r < 2; ++r) cp(h->ltil1, h->ltil, r * nl + H.r6b, H.r6e - H.r6b);
    cp(h->rtil1, h->rtil, H.r6b, H.r6e - H.r6b);
    cp(h->calpha1, h->calpha, H.r6b, H.r6e - H.r6b);
    cp(h->calpha1, h->calpha, H.r4b, H.r4e - H.r4b);
    C.cur_clear = h->ctl + g;
    const int bx = (int)std::min<int64_t>(256, std::max<int64_t>(1, (longest + 255) / 256));
    hipLaunchKernelGGL(copy_kernel, dim3(bx, std::max(1, C.n)), dim3(256), 0, h->stream, C);
    HIP_TRY(hipGetLastError());
    h->h_ctl[g].cur = 0;
  }
  return ACOPF_OK;
}

static int run_impl(acopf_s* h, int64_t max_iters, bool stop_on_first, int64_t* issued_out) {
  int64_t issued = 0;
  while (issued < max_iters) {
    int nrun = 0;
    for (int g = 0; g < h->G; ++g) nrun += h->running[g];
    if (nrun == 0) break;
    const int k = (int)std::min<int64_t>(h->tune.chunk, max_iters - issued);
    // every lane with a running grid launches its chunk after the work queued
    // on the handle's stream (starts, copies, the last chunk's settling); with
    // profiling the lanes run one after another, so that events time each
    std::vector<int> ran;
    int rc = ACOPF_OK;
    std::vector<char> busy(h->lanes.size(), 0);
    bool other = false;  // a lane on a stream of its own runs
    for (int g = 0; g < h->G; ++g)
      if (h->running[g]) busy[h->lane_of[g]] = 1;
    for (size_t lane = 0; lane < busy.size(); ++lane)
      other = other || (busy[lane] && h->lanes[lane].stream != h->stream);
    if (other) HIP_TRY(hipEventRecord(h->join, h->stream));
    for (int lane = 0; lane < (int)h->lanes.size(); ++lane) {
      if (!busy[lane]) continue;
      Lane& L = h->lanes[lane];
      if (L.stream != h->stream) HIP_TRY(hipStreamWaitEvent(L.stream, h->join, 0));
      rc = build_active(h, lane);
      if (rc) return rc;
      rc = launch_chunk(h, lane, k);
      if (rc) return rc;
      if (h->profile) HIP_TRY(hipStreamSynchronize(L.stream));
      ran.push_back(lane);
    }
    // the control words are read on the handle's stream after every lane's
    // chunk (queued behind them, so that the copy starts as the chunks end)
    for (int lane : ran) {
      Lane& L = h->lanes[lane];
      if (L.stream == h->stream) continue;
      HIP_TRY(hipEventRecord(L.end, L.stream));
      HIP_TRY(hipStreamWaitEvent(h->stream, L.end, 0));
    }
    issued += k;
    HIP_TRY(hipMemcpyAsync(h->h_ctl, h->ctl, sizeof(GridCtl) * h->G, hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    rc = settle_buffers(h);
    if (rc) return rc;
    if (h->profile) accumulate_timing(h, k, ran);
    const double t = now_s();
    bool finished_one = false;
    for (int g = 0; g < h->G; ++g)
      if (h->running[g] && h->h_ctl[g].done) {
        h->running[g] = 0;
        h->t_end[g] = t;
        finished_one = true;
      }
    if (stop_on_first && finished_one) break;
  }
  if (issued_out) *issued_out = issued;
  return settle_outer(h);
}

// Every grid's objective (eq. (acopf)'s generation cost at u), control word
// and branch-failure count into the pinned result copies: one launch, three
// copies and one wait, whatever the number of grids asked for.
static int fetch_results(acopf_s* h) {
  hipStream_t st = h->stream;
  hipLaunchKernelGGL(objective_kernel, dim3(h->G), dim3(kObjBlock), 0, st, h->gen_off_d, h->c2,
                     h->c1, h->c0, h->u, h->base_d, h->obj_d);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(h->r_obj, h->obj_d, sizeof(double) * h->G, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(h->r_fail, h->failures, sizeof(int) * h->G, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(h->r_ctl, h->ctl, sizeof(GridCtl) * h->G, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return ACOPF_OK;
}

static void fill_result(const acopf_s* h, int g, acopf_result* r) {
  const GridCtl& c = h->r_ctl[g];
  r->status = c.done ? c.status : ACOPF_MAX_ITER;
  r->inner_iters = c.inner_total;
  r->outer_iters = c.outer;
  r->branch_failures = h->r_fail[g];
  r->objective = h->r_obj[g];
  r->r_pri = c.r_pri;
  r->r_dual = c.r_dual;
  r->r_z = c.r_z;
  r->beta = c.beta;
  r->seconds = (h->running[g] ? now_s() : h->t_end[g]) - h->t_start[g];
}

static int result_impl(acopf_s* h, int g, acopf_result* r) {
  const int rc = fetch_results(h);
  if (!rc) fill_result(h, g, r);
  return rc;
}

int acopf_solve(acopf_handle h, int32_t mode, int32_t fixed_iters, acopf_result* results) {
  if (!h) return fail(ACOPF_EINVAL, "null handle");
  if (mode != ACOPF_COLD && mode != ACOPF_WARM && mode != ACOPF_CONTINUE)
    return fail(ACOPF_EINVAL, "mode must be COLD, WARM or CONTINUE");
  if (fixed_iters < 0) return fail(ACOPF_EINVAL, "fixed_iters must be >= 0");
  if (mode != ACOPF_COLD && !h->solved)
    return fail(ACOPF_ESTATE, "warm or continued solve before any solve");
  HIP_TRY(hipSetDevice(h->device));
  int rc = start_impl(h, -1, mode, fixed_iters);
  if (rc) return rc;
  if (h->profile) {
    for (double& t : h->t_ms) t = 0.0;
    h->t_iters = 0;
  }
  const int64_t cap = fixed_iters > 0
                          ? fixed_iters
                          : (int64_t)h->P.max_outer * h->P.max_inner + 1;
  rc = run_impl(h, cap, false, nullptr);
  if (rc) return rc;
  h->solved = true;
  if (results) {
    rc = fetch_results(h);
    if (rc) return rc;
    for (int g = 0; g < h->G; ++g) fill_result(h, g, &results[g]);
  }
  return ACOPF_OK;
}

int acopf_start(acopf_handle h, int32_t grid, int32_t mode, int32_t fixed_iters) {
  if (!h) return fail(ACOPF_EINVAL, "null handle");
  if (grid < 0 || grid >= h->G) return fail(ACOPF_EINVAL, "grid index out of range");
  if (mode != ACOPF_COLD && mode != ACOPF_WARM && mode != ACOPF_CONTINUE)
    return fail(ACOPF_EINVAL, "mode must be COLD, WARM or CONTINUE");
  if (fixed_iters < 0) return fail(ACOPF_EINVAL, "fixed_iters must be >= 0");
  if (mode != ACOPF_COLD && !h->started_once[grid] && !h->solved)
    return fail(ACOPF_ESTATE, "warm or continued start of a grid never solved");
  if (h->running[grid]) return fail(ACOPF_ESTATE, "grid is already running");
  HIP_TRY(hipSetDevice(h->device));
  return start_impl(h, grid, mode, fixed_iters);
}

int acopf_run(acopf_handle h, int32_t max_iters, int32_t* running) {
  if (!h) return fail(ACOPF_EINVAL, "null handle");
  if (max_iters < 1) return fail(ACOPF_EINVAL, "max_iters must be >= 1");
  HIP_TRY(hipSetDevice(h->device));
  int rc = run_impl(h, max_iters, true, nullptr);
  if (rc) return rc;
  if (running) {
    int n = 0;
    for (int g = 0; g < h->G; ++g) n += h->running[g];
    *running = n;
  }
  return ACOPF_OK;
}

int acopf_poll(acopf_handle h, int32_t grid, int32_t* is_running, acopf_result* out) {
  if (!h) return fail(ACOPF_EINVAL, "null handle");
  if (grid < 0 || grid >= h->G) return fail(ACOPF_EINVAL, "grid index out of range");
  if (is_running) *is_running = h->running[grid];
  if (out) {
    HIP_TRY(hipSetDevice(h->device));
    return result_impl(h, grid, out);
  }
  return ACOPF_OK;
}

int acopf_update_loads(acopf_handle h, int32_t grid, const double* pd, const double* qd) {
  if (!h) return fail(ACOPF_EINVAL, "null handle");
  if (grid < 0 || grid >= h->G) return fail(ACOPF_EINVAL, "grid index out of range");
  if (!pd || !qd) return fail(ACOPF_EINVAL, "null load array");
  const HostGrid& H = h->grids[grid];
  if (!finite_all(pd, H.nb) || !finite_all(qd, H.nb))
    return fail(ACOPF_EINVAL, "non-finite load");
  HIP_TRY(hipSetDevice(h->device));
  HIP_TRY(hipMemcpyAsync(h->pd + H.bus_off, pd, sizeof(double) * H.nb, hipMemcpyHostToDevice,
                         h->stream));
  HIP_TRY(hipMemcpyAsync(h->qd + H.bus_off, qd, sizeof(double) * H.nb, hipMemcpyHostToDevice,
                         h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return ACOPF_OK;
}

int acopf_update_gen_bounds(acopf_handle h, int32_t grid, const double* pmin,
                            const double* pmax) {
  if (!h) return fail(ACOPF_EINVAL, "null handle");
  if (grid < 0 || grid >= h->G) return fail(ACOPF_EINVAL, "grid index out of range");
  const HostGrid& H = h->grids[grid];
  if (H.ng == 0) return ACOPF_OK;
  if (!pmin || !pmax) return fail(ACOPF_EINVAL, "null bound array");
  if (!finite_all(pmin, H.ng) || !finite_all(pmax, H.ng))
    return fail(ACOPF_EINVAL, "non-finite generator bound");
  std::vector<double> lo(H.ng), hi(H.ng);
  for (int64_t k = 0; k < H.ng; ++k) {
    if (pmin[k] > pmax[k]) return fail(ACOPF_EINVAL, "empty generator bound interval");
    lo[H.gen_dev[k] - H.gen_off] = pmin[k];
    hi[H.gen_dev[k] - H.gen_off] = pmax[k];
  }
  HIP_TRY(hipSetDevice(h->device));
  HIP_TRY(hipMemcpyAsync(h->pmin + H.gen_off, lo.data(), sizeof(double) * H.ng,
                         hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(h->pmax + H.gen_off, hi.data(), sizeof(double) * H.ng,
                         hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return ACOPF_OK;
}

static int64_t state_size(const HostGrid& H, int what) {
  const int64_t m = 2 * H.ng + 8 * H.nl;
  switch (what) {
    case ACOPF_U: case ACOPF_V: case ACOPF_Z: case ACOPF_Y: case ACOPF_LAMBDA: return m;
    case ACOPF_BRANCH_X: return 6 * H.nl;
    case ACOPF_BRANCH_LTIL: return 2 * H.nl;
    case ACOPF_BRANCH_RTIL: case ACOPF_BRANCH_ALPHA: return H.nl;
    case ACOPF_SCALARS: return 9;
    case ACOPF_PD: case ACOPF_QD: return H.nb;
    case ACOPF_STATS: return kStats;
    case ACOPF_SOLUTION: return 2 * H.ng + 2 * H.nb + 4 * H.nl;
    default: return -1;
  }
}

// Scratch of the solution recovery (bus w and theta, flows per branch end)
// and of the quality maxima, allocated on first use.
static int quality_scratch(acopf_s* h) {
  if (h->qscratch) return ACOPF_OK;
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(double) * (2 * h->nb + 2 * h->ne)) != hipSuccess)
    return fail(ACOPF_ENOMEM, "quality scratch allocation failed");
  h->qscratch = static_cast<double*>(p);
  if (hipMalloc(&p, sizeof(unsigned long long) * 6 * h->G) != hipSuccess)
    return fail(ACOPF_ENOMEM, "quality scratch allocation failed");
  h->qual = static_cast<unsigned long long*>(p);
  return ACOPF_OK;
}

// Recovers the solution of Sec. IV-A into the scratch (bus w, theta; flows
// of every branch end from the bus voltages) and the quality maxima per
// grid into h->qual (zeroed by a fill kernel first).
static int launch_recovery(acopf_s* h) {
  int rc = quality_scratch(h);
  if (rc) return rc;
  hipStream_t st = h->stream;
  acopf_dev::launch_fill_u64(h->qual, (int64_t)6 * h->G, st);
  acopf_dev::QualityArgs Q{h->nb, h->ng, h->nl, h->ne, h->bus_grid, h->br_grid, h->gen_grid,
                           h->gptr, h->eptr, h->ef, h->et, h->end_bus, h->adm, h->rate, h->u,
                           h->v, h->pd, h->qd, h->gs, h->bs, h->vmin_b, h->vmax_b,
                           h->qscratch, h->qscratch + h->nb, h->qscratch + 2 * h->nb,
                           h->qscratch + 2 * h->nb + h->ne, h->qual};
  acopf_dev::launch_quality(Q, st);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

// canonical <-> device permutations of the per-grid vectors
static int copy_state(acopf_s* h, int grid, int what, double* host, int64_t n, bool to_host) {
  const HostGrid& H = h->grids[grid];
  hipStream_t st = h->stream;
  auto pull = [&](const double* dsrc, int64_t count, std::vector<double>& tmp) {
    tmp.resize(count);
    return hipMemcpyAsync(tmp.data(), dsrc, sizeof(double) * count, hipMemcpyDeviceToHost, st);
  };
  auto push = [&](double* ddst, const std::vector<double>& tmp) {
    return hipMemcpyAsync(ddst, tmp.data(), sizeof(double) * tmp.size(), hipMemcpyHostToDevice, st);
  };
  const int64_t ng = h->ng, nl = h->nl;
  if (what <= ACOPF_LAMBDA) {
    double* base = what == ACOPF_U ? h->u : what == ACOPF_V ? h->v : what == ACOPF_Z ? h->z
                   : what == ACOPF_Y ? h->y : h->lam;
    std::vector<double> all;
    // whole vector round trip (state vectors are small next to HBM bandwidth)
    HIP_TRY(pull(base, h->m, all));
    HIP_TRY(hipStreamSynchronize(st));
    for (int64_t k = 0; k < H.ng; ++k) {
      double* p0 = &all[H.gen_dev[k]];
      double* p1 = &all[ng + H.gen_dev[k]];
      if (to_host) { host[2 * k] = *p0; host[2 * k + 1] = *p1; }
      else { *p0 = host[2 * k]; *p1 = host[2 * k + 1]; }
    }
    const int64_t ne = h->ne;
    for (int64_t l = 0; l < H.nl; ++l) {
      const int64_t ef = H.end_f[l], et = H.end_t[l];
      const int64_t pos[8] = {acopf_dev::end_coupling(ng, ne, 0, ef),
                              acopf_dev::end_coupling(ng, ne, 1, ef),
                              acopf_dev::end_coupling(ng, ne, 0, et),
                              acopf_dev::end_coupling(ng, ne, 1, et),
                              acopf_dev::end_coupling(ng, ne, 2, ef),
                              acopf_dev::end_coupling(ng, ne, 3, ef),
                              acopf_dev::end_coupling(ng, ne, 2, et),
                              acopf_dev::end_coupling(ng, ne, 3, et)};
      for (int k = 0; k < 8; ++k) {
        double* p = &all[pos[k]];
        double* q = &host[2 * H.ng + 8 * l + k];
        if (to_host) *q = *p; else *p = *q;
      }
    }
    if (!to_host) {
      HIP_TRY(push(base, all));
      HIP_TRY(hipStreamSynchronize(st));
    }
    return ACOPF_OK;
  }
  if (what == ACOPF_BRANCH_X || what == ACOPF_BRANCH_LTIL || what == ACOPF_BRANCH_RTIL ||
      what == ACOPF_BRANCH_ALPHA) {
    const int rows = what == ACOPF_BRANCH_X ? 6 : what == ACOPF_BRANCH_LTIL ? 2 : 1;
    double* base = what == ACOPF_BRANCH_X      ? h->bx
                   : what == ACOPF_BRANCH_LTIL ? h->ltil
                   : what == ACOPF_BRANCH_RTIL ? h->rtil
                                               : h->calpha;
    std::vector<double> all;
    HIP_TRY(pull(base, rows * nl, all));
    HIP_TRY(hipStreamSynchronize(st));
    for (int64_t l = 0; l < H.nl; ++l) {
      const int64_t d = H.br_dev[l];
      for (int r = 0; r < rows; ++r) {
        double* p = &all[r * nl + d];
        double* q = &host[rows * l + r];
        if (to_host) *q = *p; else *p = *q;
      }
    }
    if (!to_host) {
      HIP_TRY(push(base, all));
      HIP_TRY(hipStreamSynchronize(st));
    }
    return ACOPF_OK;
  }
  if (what == ACOPF_PD || what == ACOPF_QD) {
    double* base = (what == ACOPF_PD ? h->pd : h->qd) + H.bus_off;
    if (to_host)
      HIP_TRY(hipMemcpyAsync(host, base, sizeof(double) * H.nb, hipMemcpyDeviceToHost, st));
    else
      HIP_TRY(hipMemcpyAsync(base, host, sizeof(double) * H.nb, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return ACOPF_OK;
  }
  if (what == ACOPF_SCALARS) {
    GridCtl c;
    HIP_TRY(hipMemcpyAsync(&c, h->ctl + grid, sizeof(GridCtl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (to_host) {
      const double vals[9] = {c.beta, c.znorm_prev, c.r_pri, c.r_dual, c.r_z, (double)c.outer,
                              (double)c.inner_total, (double)c.inner_in_outer, (double)c.status};
      std::memcpy(host, vals, sizeof(vals));
    } else {
      c.beta = host[0];
      c.znorm_prev = host[1];
      c.r_pri = host[2];
      c.r_dual = host[3];
      c.r_z = host[4];
      c.outer = (int)host[5];
      c.inner_total = (int)host[6];
      c.inner_in_outer = (int)host[7];
      c.status = (int)host[8];
      HIP_TRY(hipMemcpyAsync(h->ctl + grid, &c, sizeof(GridCtl), hipMemcpyHostToDevice, st));
      HIP_TRY(hipStreamSynchronize(st));
    }
    return ACOPF_OK;
  }
  if (what == ACOPF_SOLUTION && to_host) {
    // generator outputs from the generator problems, |V| = sqrt(w) and
    // theta from the bus problems, flows recomputed from those voltages
    int rc = launch_recovery(h);
    if (rc) return rc;
    std::vector<double> uu, bw, bt, pe, qe;
    HIP_TRY(pull(h->u, 2 * ng, uu));
    HIP_TRY(pull(h->qscratch + H.bus_off, H.nb, bw));
    HIP_TRY(pull(h->qscratch + h->nb + H.bus_off, H.nb, bt));
    HIP_TRY(pull(h->qscratch + 2 * h->nb, h->ne, pe));
    HIP_TRY(pull(h->qscratch + 2 * h->nb + h->ne, h->ne, qe));
    HIP_TRY(hipStreamSynchronize(st));
    double* pg = host;
    double* qg = pg + H.ng;
    double* vm = qg + H.ng;
    double* va = vm + H.nb;
    double* fl = va + H.nb;
    for (int64_t k = 0; k < H.ng; ++k) {
      pg[k] = uu[H.gen_dev[k]];
      qg[k] = uu[ng + H.gen_dev[k]];
    }
    for (int64_t i = 0; i < H.nb; ++i) {
      vm[i] = bw[i] > 0.0 ? std::sqrt(bw[i]) : 0.0;
      va[i] = bt[i];
    }
    for (int64_t l = 0; l < H.nl; ++l) {
      fl[l] = pe[H.end_f[l]];
      fl[H.nl + l] = qe[H.end_f[l]];
      fl[2 * H.nl + l] = pe[H.end_t[l]];
      fl[3 * H.nl + l] = qe[H.end_t[l]];
    }
    return ACOPF_OK;
  }
  if (what == ACOPF_STATS && to_host) {
    unsigned long long s[kStats];
    HIP_TRY(hipMemcpyAsync(s, h->stats, sizeof(s), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int q = 0; q < kStats; ++q) host[q] = (double)s[q];
    return ACOPF_OK;
  }
  return fail(ACOPF_EINVAL, "unsupported state code for this direction");
}

int acopf_get_state(acopf_handle h, int32_t grid, int32_t what, double* out, int64_t n) {
  if (!h) return fail(ACOPF_EINVAL, "null handle");
  if (grid < 0 || grid >= h->G) return fail(ACOPF_EINVAL, "grid index out of range");
  if (!out) return fail(ACOPF_EINVAL, "null output");
  HIP_TRY(hipSetDevice(h->device));
  if (what == ACOPF_HISTORY) {
    GridCtl c;
    HIP_TRY(hipMemcpy(&c, h->ctl + grid, sizeof(GridCtl), hipMemcpyDeviceToHost));
    const int64_t len = (int64_t)std::min(c.inner_total, kHistCap) * 6;
    if (n != len) return fail(ACOPF_EINVAL, "history size must be 6 * min(inner_total, cap) = " + std::to_string(len));
    HIP_TRY(hipMemcpy(out, h->hist + (int64_t)grid * kHistCap * 6, sizeof(double) * len,
                      hipMemcpyDeviceToHost));
    return ACOPF_OK;
  }
  const int64_t need = state_size(h->grids[grid], what);
  if (need < 0) return fail(ACOPF_EINVAL, "unknown state code");
  if (n != need) return fail(ACOPF_EINVAL, "buffer size mismatch: need " + std::to_string(need));
  return copy_state(h, grid, what, out, n, true);
}

int acopf_set_state(acopf_handle h, int32_t grid, int32_t what, const double* in, int64_t n) {
  if (!h) return fail(ACOPF_EINVAL, "null handle");
  if (grid < 0 || grid >= h->G) return fail(ACOPF_EINVAL, "grid index out of range");
  if (!in) return fail(ACOPF_EINVAL, "null input");
  if (what == ACOPF_HISTORY || what == ACOPF_STATS || what == ACOPF_SOLUTION)
    return fail(ACOPF_EINVAL, "read-only state");
  const int64_t need = state_size(h->grids[grid], what);
  if (need < 0) return fail(ACOPF_EINVAL, "unknown state code");
  if (n != need) return fail(ACOPF_EINVAL, "buffer size mismatch: need " + std::to_string(need));
  if (!finite_all(in, n) && what != ACOPF_SCALARS) return fail(ACOPF_EINVAL, "non-finite state");
  if (what == ACOPF_BRANCH_ALPHA)
    for (int64_t i = 0; i < n; ++i)
      if (!(in[i] > 0.0)) return fail(ACOPF_EINVAL, "Cauchy step lengths must be positive");
  HIP_TRY(hipSetDevice(h->device));
  if (h->running[grid]) return fail(ACOPF_ESTATE, "grid is running");
  h->solved = true;
  h->started_once[grid] = 1;
  return copy_state(h, grid, what, const_cast<double*>(in), n, false);
}

int acopf_get_sizes(acopf_handle h, int32_t grid, int64_t* out4) {
  if (!h || !out4) return fail(ACOPF_EINVAL, "null argument");
  if (grid < 0 || grid >= h->G) return fail(ACOPF_EINVAL, "grid index out of range");
  const HostGrid& H = h->grids[grid];
  out4[0] = h->G;
  out4[1] = H.nb;
  out4[2] = H.ng;
  out4[3] = H.nl;
  return ACOPF_OK;
}

// Device arrays that make up the iteration state, with their lengths.
static std::vector<std::pair<void*, size_t>> state_arrays(acopf_s* h) {
  const size_t d = sizeof(double);
  return {{h->u, h->m * d},      {h->v, h->m * d},      {h->z, h->m * d},
          {h->y, h->m * d},      {h->lam, h->m * d},    {h->bx, 6 * h->nl * d},
          {h->ltil, 2 * h->nl * d}, {h->rtil, h->nl * d}, {h->calpha, h->nl * d},
          {h->brec, 16 * h->nl * d}, {h->pd, h->nb * d},
          {h->qd, h->nb * d},    {h->ctl, h->G * sizeof(GridCtl)}};
}

int acopf_snapshot(acopf_handle h, int32_t what) {
  if (!h) return fail(ACOPF_EINVAL, "null handle");
  if (what != 0 && what != 1) return fail(ACOPF_EINVAL, "what must be 0 (save) or 1 (restore)");
  HIP_TRY(hipSetDevice(h->device));
  auto arrs = state_arrays(h);
  if (what == 1 && h->snap.empty()) return fail(ACOPF_ESTATE, "restore without a saved snapshot");
  if (h->snap.empty()) {
    for (auto& a : arrs) {
      void* p = nullptr;
      if (hipMalloc(&p, a.second) != hipSuccess) {
        for (void* q : h->snap) (void)hipFree(q);
        h->snap.clear();
        return fail(ACOPF_ENOMEM, "snapshot allocation failed");
      }
      h->snap.push_back(p);
    }
  }
  for (size_t i = 0; i < arrs.size(); ++i) {
    if (what == 0)
      HIP_TRY(hipMemcpyAsync(h->snap[i], arrs[i].first, arrs[i].second, hipMemcpyDeviceToDevice,
                             h->stream));
    else
      HIP_TRY(hipMemcpyAsync(arrs[i].first, h->snap[i], arrs[i].second, hipMemcpyDeviceToDevice,
                             h->stream));
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (what == 1) {
    // the restored control blocks decide which grids are running
    HIP_TRY(hipMemcpy(h->h_ctl, h->ctl, sizeof(GridCtl) * h->G, hipMemcpyDeviceToHost));
    for (int g = 0; g < h->G; ++g) h->running[g] = h->h_ctl[g].done ? 0 : 1;
  }
  return ACOPF_OK;
}

int acopf_copy_grid(acopf_handle h, int32_t src, int32_t dst) {
  if (!h) return fail(ACOPF_EINVAL, "null handle");
  if (src < 0 || src >= h->G || dst < 0 || dst >= h->G)
    return fail(ACOPF_EINVAL, "grid index out of range");
  if (src == dst) return ACOPF_OK;
  const HostGrid& A = h->grids[src];
  const HostGrid& B = h->grids[dst];
  if (A.nb != B.nb || A.ng != B.ng || A.nl != B.nl || A.r6e - A.r6b != B.r6e - B.r6b)
    return fail(ACOPF_EINVAL, "grids differ in size");
  if (h->running[dst]) return fail(ACOPF_ESTATE, "destination grid is running");
  HIP_TRY(hipSetDevice(h->device));
  CopySegs C{};
  int64_t longest = 0;
  auto cp = [&](double* base, int64_t from, int64_t to, int64_t n) {
    if (n <= 0) return;
    C.src[C.n] = base + from;
    C.dst[C.n] = base + to;
    C.len[C.n] = n;
    longest = std::max(longest, n);
    ++C.n;
  };
  const int64_t ng = h->ng, nl = h->nl;
  double* vecs[] = {h->u, h->v, h->z, h->y, h->lam};
  for (double* v : vecs) {
    cp(v, A.gen_off, B.gen_off, A.ng);
    cp(v, ng + A.gen_off, ng + B.gen_off, A.ng);
    cp(v, 2 * ng + 4 * A.e0, 2 * ng + 4 * B.e0, 4 * (A.e1 - A.e0));
  }
  for (int r = 0; r < 6; ++r) {
    cp(h->bx, r * nl + A.r6b, r * nl + B.r6b, A.r6e - A.r6b);
    cp(h->bx, r * nl + A.r4b, r * nl + B.r4b, A.r4e - A.r4b);
  }
  for (int r = 0; r < 2; ++r) {
    cp(h->ltil, r * nl + A.r6b, r * nl + B.r6b, A.r6e - A.r6b);
    cp(h->ltil, r * nl + A.r4b, r * nl + B.r4b, A.r4e - A.r4b);
  }
  cp(h->rtil, A.r6b, B.r6b, A.r6e - A.r6b);
  cp(h->rtil, A.r4b, B.r4b, A.r4e - A.r4b);
  cp(h->calpha, A.r6b, B.r6b, A.r6e - A.r6b);
  cp(h->calpha, A.r4b, B.r4b, A.r4e - A.r4b);
  cp(h->pd, A.bus_off, B.bus_off, A.nb);
  cp(h->qd, A.bus_off, B.bus_off, A.nb);
  C.csrc = h->ctl + src;
  C.cdst = h->ctl + dst;
  const int bx = (int)std::min<int64_t>(256, std::max<int64_t>(1, (longest + 255) / 256));
  hipLaunchKernelGGL(copy_kernel, dim3(bx, std::max(1, C.n)), dim3(256), 0, h->stream, C);
  HIP_TRY(hipGetLastError());
  h->started_once[dst] = h->started_once[src] || h->solved;
  return ACOPF_OK;
}

static int check_tuning(const acopf_tuning& t) {
  if (t.xstep_block != 64 && t.xstep_block != 128 && t.xstep_block != 256)
    return fail(ACOPF_EINVAL, "xstep_block must be 64, 128 or 256");
  if (t.bus_block < 64 || t.bus_block > 1024 || t.bus_block % 64)
    return fail(ACOPF_EINVAL, "bus_block must be a multiple of 64 in [64, 1024]");
  if (t.chunk < 1 || t.chunk > kMaxChunk) return fail(ACOPF_EINVAL, "chunk must be in [1, 64]");
  if (t.xstep_waves < 0 || t.xstep_waves > 4)
    return fail(ACOPF_EINVAL, "xstep_waves must be in [0, 4]");
  if (t.xstep_per_lane < 0 || t.xstep_per_lane > 8)
    return fail(ACOPF_EINVAL, "xstep_per_lane must be in [0, 8]");
  if (t.lanes < 1 || t.lanes > kMaxLanes) return fail(ACOPF_EINVAL, "lanes must be in [1, 4]");
  return ACOPF_OK;
}

static int apply_tuning(acopf_s* h, const acopf_tuning& t) {
  drop_graph(h);
  if (t.bus_block != h->tile_block) {
    int rc = build_tiles(h, t.bus_block);
    if (rc) return rc;
  }
  // the persistent branch kernel pools every branch of the handle: one lane
  const int lanes = t.xstep_waves > 0 ? 1 : std::min(t.lanes, h->G);
  if (lanes != (int)h->lanes.size()) {
    int rc = set_lanes(h, lanes);
    if (rc) return rc;
  }
  h->tune = t;
  h->tune.lanes = (int)h->lanes.size();
  for (Lane& L : h->lanes) L.lists_dirty = true;  // x-step items depend on the block and per-lane count
  return ACOPF_OK;
}

int acopf_set_tuning(acopf_handle h, const acopf_tuning* t) {
  if (!h || !t) return fail(ACOPF_EINVAL, "null argument");
  int rc = check_tuning(*t);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(h->device));
  rc = apply_tuning(h, *t);
  return rc ? rc : ensure_graph(h);
}

int acopf_get_tuning(acopf_handle h, acopf_tuning* t) {
  if (!h || !t) return fail(ACOPF_EINVAL, "null argument");
  *t = h->tune;
  return ACOPF_OK;
}

int acopf_autotune(acopf_handle h, int32_t iters, acopf_tuning* out) {
  if (!h) return fail(ACOPF_EINVAL, "null handle");
  if (iters < 1) return fail(ACOPF_EINVAL, "iters must be >= 1");
  HIP_TRY(hipSetDevice(h->device));
  const bool prof = h->profile;
  h->profile = false;
  int rc = acopf_snapshot(h, 0);
  if (rc) return rc;
  const std::vector<char> run0 = h->running, once0 = h->started_once;
  const std::vector<double> ts0 = h->t_start, te0 = h->t_end;
  acopf_tuning best = h->tune;
  double best_t = 1e300;
  // x-step variants {block, persistent waves, unlimited branches per lane}:
  // lane per branch at three block sizes (branches per lane automatic, or
  // one), or the persistent kernel at one or two wavefronts per SIMD
  const int xs[7][3] = {{64, 0, 0}, {64, 0, 1}, {128, 0, 0}, {256, 0, 0},
                        {64, 1, 0}, {64, 2, 0}, {128, 0, 1}};
  const int bs[4] = {128, 256, 512, 1024}, cs[3] = {8, 16, 32};
  // best of two timed runs of `iters` iterations from the saved state
  auto measure = [&](const acopf_tuning& t, double* secs) -> int {
    int r = apply_tuning(h, t);
    if (r) return r;
    double tmin = 1e300;
    for (int rep = 0; rep < 2; ++rep) {  // first pass also captures the graphs
      r = acopf_snapshot(h, 1);
      if (r) return r;
      r = start_impl(h, -1, ACOPF_CONTINUE, iters);
      if (r) return r;
      HIP_TRY(hipStreamSynchronize(h->stream));
      const double t0 = now_s();
      r = run_impl(h, iters, false, nullptr);
      if (r) return r;
      tmin = std::min(tmin, now_s() - t0);
    }
    *secs = tmin;
    return ACOPF_OK;
  };
  for (const auto& xi : xs)
    for (int bi : bs)
      for (int ci : cs) {
        acopf_tuning t{xi[0], bi, ci, 1, xi[1], xi[2], h->tune.lanes};
        double secs = 0.0;
        rc = measure(t, &secs);
        if (rc) return rc;
        if (secs < best_t) {
          best_t = secs;
          best = t;
        }
      }
  // then the number of launch lanes for the best shape
  const acopf_tuning shape = best;
  for (int nl : {1, 2, 4}) {
    if (nl > h->G || nl == shape.lanes) continue;
    acopf_tuning t = shape;
    t.lanes = nl;
    double secs = 0.0;
    rc = measure(t, &secs);
    if (rc) return rc;
    if (secs < best_t) {
      best_t = secs;
      best = t;
    }
  }
  rc = apply_tuning(h, best);
  if (rc) return rc;
  rc = acopf_snapshot(h, 1);
  if (rc) return rc;
  h->running = run0;
  h->started_once = once0;
  h->t_start = ts0;
  h->t_end = te0;
  h->profile = prof;
  if (out) *out = best;
  return ACOPF_OK;
}

int acopf_set_counting(acopf_handle h, int32_t on) {
  if (!h) return fail(ACOPF_EINVAL, "null handle");
  if ((on != 0) != h->count_stats) {
    HIP_TRY(hipSetDevice(h->device));
    drop_graph(h);
    h->count_stats = on != 0;
    return ensure_graph(h);
  }
  return ACOPF_OK;
}

int acopf_set_profiling(acopf_handle h, int32_t on) {
  if (!h) return fail(ACOPF_EINVAL, "null handle");
  HIP_TRY(hipSetDevice(h->device));
  if (on && h->ev.empty()) {
    h->ev.resize((size_t)kEvPerIter * kMaxChunk * kMaxLanes);  // per lane and iteration
    for (auto& e : h->ev) HIP_TRY(hipEventCreate(&e));
  }
  h->profile = on != 0;
  return ACOPF_OK;
}

int acopf_quality(acopf_handle h, int32_t grid, double* out6) {
  if (!h || !out6) return fail(ACOPF_EINVAL, "null argument");
  if (grid < 0 || grid >= h->G) return fail(ACOPF_EINVAL, "grid index out of range");
  HIP_TRY(hipSetDevice(h->device));
  int rc = launch_recovery(h);
  if (rc) return rc;
  hipStream_t st = h->stream;
  unsigned long long bits[6];
  HIP_TRY(hipMemcpyAsync(bits, h->qual + 6 * grid, sizeof(bits), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double q[6];
  for (int k = 0; k < 6; ++k) std::memcpy(&q[k], &bits[k], sizeof(double));
  auto nanmax = [](double a, double b) { return (b > a || b != b) ? b : a; };
  out6[0] = nanmax(nanmax(nanmax(q[1], q[2]), nanmax(q[3], q[4])), q[5]);
  for (int k = 1; k < 6; ++k) out6[k] = q[k];
  return ACOPF_OK;
}

int acopf_quality_noalloc(acopf_handle h, int32_t grid, double* out6) {
  if (!h || !out6) return fail(ACOPF_EINVAL, "null argument");
  if (grid < 0 || grid >= h->G) return fail(ACOPF_EINVAL, "grid index out of range");
  // bus w and theta [2 nb], flows per branch end [2 ne], then 6 maxima per
  // grid of the handle, in eight-byte words
  const int64_t words = 2 * h->nb + 2 * h->ne + 6 * (int64_t)h->G;
  if (words > kNoAllocWords)
    return fail(ACOPF_EINVAL, "handle too large for the fixed scratch: needs " +
                                  std::to_string(words) + " words (2 n_bus + 4 n_branch + 6 "
                                  "n_grids over the handle), the maximum is " +
                                  std::to_string(kNoAllocWords));
  HIP_TRY(hipSetDevice(h->device));
  double* sp = nullptr;
  int rc = noalloc_scratch(h->device, &sp);
  if (rc) return rc;
  hipStream_t st = h->stream;
  unsigned long long* qmax = reinterpret_cast<unsigned long long*>(sp + 2 * h->nb + 2 * h->ne);
  acopf_dev::launch_fill_u64(qmax, (int64_t)6 * h->G, st);
  acopf_dev::QualityArgs Q{h->nb, h->ng, h->nl, h->ne, h->bus_grid, h->br_grid, h->gen_grid,
                           h->gptr, h->eptr, h->ef, h->et, h->end_bus, h->adm, h->rate, h->u,
                           h->v, h->pd, h->qd, h->gs, h->bs, h->vmin_b, h->vmax_b,
                           sp, sp + h->nb, sp + 2 * h->nb, sp + 2 * h->nb + h->ne, qmax};
  acopf_dev::launch_quality(Q, st);
  HIP_TRY(hipGetLastError());
  unsigned long long bits[6];
  HIP_TRY(hipMemcpyAsync(bits, qmax + 6 * grid, sizeof(bits), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double q[6];
  for (int k = 0; k < 6; ++k) std::memcpy(&q[k], &bits[k], sizeof(double));
  auto nanmax = [](double a, double b) { return (b > a || b != b) ? b : a; };
  out6[0] = nanmax(nanmax(nanmax(q[1], q[2]), nanmax(q[3], q[4])), q[5]);
  for (int k = 1; k < 6; ++k) out6[k] = q[k];
  return ACOPF_OK;
}

int acopf_get_timing(acopf_handle h, double* out5) {
  if (!h || !out5) return fail(ACOPF_EINVAL, "null argument");
  const double n = h->t_iters > 0 ? (double)h->t_iters : 1.0;
  for (int k = 0; k < kTimed; ++k) out5[k] = h->t_ms[k] / n;
  out5[3] = 0.0;  // the outer multiplier step runs inside the bus step
  out5[4] = (double)h->t_iters;
  return ACOPF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Measurement helpers: the device's achievable streaming bandwidth and FP64
// vector rate, reported beside the published peaks. Not part of the method.
// ---------------------------------------------------------------------------
namespace {

// Streaming copy in 16-byte vectors, grid-stride.
__global__ __launch_bounds__(256) void peak_copy_kernel(const double2* __restrict__ src,
                                                        double2* __restrict__ dst, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride)
    dst[i] = src[i];
}

// Eight independent FP64 fused multiply-add chains per lane. Each chain
// a <- a*b + (1 - b) contracts towards 1, so nothing overflows or becomes
// subnormal; b differs per lane so the chains cannot be folded.
__global__ __launch_bounds__(256) void peak_fma_kernel(double* out, int iters) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const double b = 0.999999 + 1e-9 * (double)(t & 7);
  const double c = 1.0 - b;
  double a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = 1.0 + 0.001 * k + 1e-7 * (double)(t & 63);
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = fma(a[k], b, c);
  }
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) sum += a[k];
  out[t] = sum;
}

// Buffers, stream and events of one measurement, released on every exit.
struct PeakScratch {
  void* a = nullptr;
  void* b = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~PeakScratch() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
  }
};

int peak_setup(PeakScratch& P, int* n_cu) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_TRY(hipStreamCreate(&P.s));
  HIP_TRY(hipEventCreate(&P.e0));
  HIP_TRY(hipEventCreate(&P.e1));
  return ACOPF_OK;
}

}  // namespace

extern "C" {

int acopf_peak_hbm(int64_t bytes, int32_t iters, double* gbs) {
  if (!gbs || bytes < (int64_t)1 << 20 || iters < 1)
    return fail(ACOPF_EINVAL, "peak_hbm: needs bytes >= 1 MiB, iters >= 1 and an output");
  PeakScratch P;
  int n_cu = 0;
  const int rc = peak_setup(P, &n_cu);
  if (rc != ACOPF_OK) return rc;
  const int64_t n2 = bytes / 16;
  if (hipMalloc(&P.a, (size_t)n2 * 16) != hipSuccess || hipMalloc(&P.b, (size_t)n2 * 16) != hipSuccess)
    return fail(ACOPF_ENOMEM, "peak_hbm: buffer allocation failed");
  HIP_TRY(hipMemsetAsync(P.a, 0, (size_t)n2 * 16, P.s));
  const dim3 grid(8 * n_cu), block(256);
  const double2* src = static_cast<const double2*>(P.a);
  double2* dst = static_cast<double2*>(P.b);
  hipLaunchKernelGGL(peak_copy_kernel, grid, block, 0, P.s, src, dst, n2);  // warm-up
  HIP_TRY(hipEventRecord(P.e0, P.s));
  for (int i = 0; i < iters; ++i) hipLaunchKernelGGL(peak_copy_kernel, grid, block, 0, P.s, src, dst, n2);
  HIP_TRY(hipEventRecord(P.e1, P.s));
  HIP_TRY(hipEventSynchronize(P.e1));
  HIP_TRY(hipGetLastError());
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, P.e0, P.e1));
  if (!(ms > 0.0f)) return fail(ACOPF_EDEVICE, "peak_hbm: no elapsed time");
  *gbs = 2.0 * 16.0 * (double)n2 * iters / (ms * 1e-3) / 1e9;
  return ACOPF_OK;
}

int acopf_device_memory(int32_t device, int64_t* out2) {
  if (!out2) return fail(ACOPF_EINVAL, "device_memory: null output");
  HIP_TRY(hipSetDevice(device));
  size_t fr = 0, tot = 0;
  HIP_TRY(hipMemGetInfo(&fr, &tot));
  out2[0] = (int64_t)fr;
  out2[1] = (int64_t)tot;
  return ACOPF_OK;
}

int acopf_peak_fp64(int32_t iters, double* tflops) {
  if (!tflops || iters < 1) return fail(ACOPF_EINVAL, "peak_fp64: needs iters >= 1 and an output");
  PeakScratch P;
  int n_cu = 0;
  const int rc = peak_setup(P, &n_cu);
  if (rc != ACOPF_OK) return rc;
  const int blocks = 8 * n_cu, threads = 256;  // 8 wavefronts per SIMD
  if (hipMalloc(&P.a, sizeof(double) * (size_t)blocks * threads) != hipSuccess)
    return fail(ACOPF_ENOMEM, "peak_fp64: output allocation failed");
  double* out = static_cast<double*>(P.a);
  // warm-up of the same length, so the timed run starts at a steady clock
  hipLaunchKernelGGL(peak_fma_kernel, dim3(blocks), dim3(threads), 0, P.s, out, iters);
  HIP_TRY(hipEventRecord(P.e0, P.s));
  hipLaunchKernelGGL(peak_fma_kernel, dim3(blocks), dim3(threads), 0, P.s, out, iters);
  HIP_TRY(hipEventRecord(P.e1, P.s));
  HIP_TRY(hipEventSynchronize(P.e1));
  HIP_TRY(hipGetLastError());
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, P.e0, P.e1));
  if (!(ms > 0.0f)) return fail(ACOPF_EDEVICE, "peak_fp64: no elapsed time");
  *tflops = 2.0 * 8.0 * (double)blocks * threads * (double)iters / (ms * 1e-3) / 1e12;
  return ACOPF_OK;
}

}  // extern "C"
