// Device-side data shared by the host runtime and the kernels of the ADMM
// library (internal; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace acopf_dev {

// Per-grid control block of Algorithm 1. Within a chunk of iterations the
// decision of iteration t is taken by a decision block of the x-step launch
// of iteration t + 1, concurrently with that launch's branch solves, and the
// control kernel takes the chunk's last one. The x-step therefore writes its
// results (u and the branch state) to the other of two buffers than the one
// it reads: when a decision finishes a grid, the x-step running beside it
// overwrites only the older buffer, and the grid's state stays in buffer
// `cur`, which the host moves to buffer 0 after the chunk.
struct GridCtl {
  double beta;        // outer penalty
  double beta_lam;    // beta used by a pending lambda update
  double znorm_prev;  // ||z||_inf at the previous outer update (inf at start)
  double r_pri, r_dual, r_z;
  int outer, inner_total, inner_in_outer, status;
  int done, do_outer, fixed_target, fixed_mode;  // fixed_mode: stop only at fixed_target
  int cur, pad0, pad1, pad2;  // cur: buffer of the last x-step results a decision accepted
};

// A grid of a control launch or of the decision blocks of an x-step: its
// index and the range [t0, t1) of its bus tiles' residual slots.
struct GridItem {
  int g, t0, t1, pad;
};

// What a control decision reads and writes besides the control block.
struct DecideArgs {
  GridCtl* ctl;           // [G]
  const double* tmax;     // [n_tiles][3] residual maxima per bus tile
  const GridItem* items;  // the running grids, one decision each
  double* hist;           // [G][hist_cap][6]
  int* failures;          // [G] branch solves that did not converge, per solve
  int* failures_it;       // [2][G] the same for the x-step results in each buffer
  double eps_pri, eps_dual, eps_z, beta_gamma, beta_omega, beta_max;
  int max_outer, max_inner, hist_cap, G;
};

// Termination tests, outer step decision and beta rule of Algorithm 1 for
// grid g, given its residual maxima; returns whether the outer step is due.
__device__ inline int ctl_decide(const DecideArgs& A, int g, GridCtl& c, double rp, double rd,
                                 double rz) {
  c.do_outer = 0;
  c.r_pri = rp;
  c.r_dual = rd;
  c.r_z = rz;
  if (c.inner_total < A.hist_cap) {
    double* h = A.hist + ((int64_t)g * A.hist_cap + c.inner_total) * 6;
    h[0] = rp;
    h[1] = rd;
    h[2] = rz;
    h[3] = 0.0;
    h[4] = c.beta;
    h[5] = (double)c.outer;
  }
  c.inner_total += 1;
  c.inner_in_outer += 1;
  if (!isfinite(rp) || !isfinite(rd) || !isfinite(rz)) {
    c.status = 2;  // ACOPF_NUMERICAL
    c.done = 1;
    return 0;
  }
  const bool inner_ok = rp <= A.eps_pri && rd <= A.eps_dual;
  const bool fixed = c.fixed_mode != 0;
  if (!fixed && inner_ok && rz <= A.eps_z) {
    c.status = 0;  // ACOPF_CONVERGED
    c.done = 1;
    return 0;
  }
  if (inner_ok || c.inner_in_outer >= A.max_inner) {
    c.do_outer = 1;
    c.beta_lam = c.beta;
    if (rz > A.beta_omega * c.znorm_prev) {
      const double b = A.beta_gamma * c.beta;
      c.beta = b < A.beta_max ? b : A.beta_max;
    }
    c.znorm_prev = rz;
    c.outer += 1;
    c.inner_in_outer = 0;
    if (!fixed && c.outer >= A.max_outer) {
      c.status = 1;  // ACOPF_MAX_ITER
      c.done = 1;
    }
  }
  if (fixed && c.inner_total >= c.fixed_target) {
    c.status = 1;  // ACOPF_MAX_ITER
    c.done = 1;
  }
  return c.do_outer;
}

// The control decision of items[i] by one whole block (a multiple of 64
// lanes, at most 1024) for the iteration whose x-step results are in buffer
// `cur`: the residual maxima over the grid's bus tiles (exact, so
// independent of the order of reduction), then ctl_decide by lane 0, which
// accepts the iteration (its branch failures count, its buffer becomes the
// grid's) and writes the control block. A grid that had already finished
// stays as it is, with an outer step that its last decision left pending
// (the host applies that one); the failures of the x-step that ran past its
// finish are dropped.
__device__ inline void decide_grid(const DecideArgs& A, int i, int cur) {
  const GridItem it = A.items[i];
  const int g = it.g;
  const int tid = threadIdx.x, nt = blockDim.x;
  // The tile maxima and lane 0's copy of the control block are loaded
  // together, so that their latencies overlap (a finished grid's maxima are
  // read and ignored); each lane issues the loads of up to kU tiles before it
  // combines them, so that one round covers kU nt tiles.
  GridCtl c;
  if (tid == 0) c = A.ctl[g];
  double rp = 0.0, rd = 0.0, rz = 0.0;
  constexpr int kU = 8;
  for (int t = it.t0 + tid; t < it.t1; t += kU * nt) {
    double m[kU][3];
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int tk = t + k * nt;
      const bool in = tk < it.t1;
      m[k][0] = in ? A.tmax[3 * tk + 0] : 0.0;
      m[k][1] = in ? A.tmax[3 * tk + 1] : 0.0;
      m[k][2] = in ? A.tmax[3 * tk + 2] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      rp = fmax(rp, m[k][0]);
      rd = fmax(rd, m[k][1]);
      rz = fmax(rz, m[k][2]);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    rp = fmax(rp, __shfl_xor(rp, off, 64));
    rd = fmax(rd, __shfl_xor(rd, off, 64));
    rz = fmax(rz, __shfl_xor(rz, off, 64));
  }
  __shared__ double red[3][16];
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = rp;
    red[1][tid >> 6] = rd;
    red[2][tid >> 6] = rz;
  }
  __syncthreads();
  if (tid != 0) return;
  int* fit = A.failures_it + (int64_t)cur * A.G + g;
  const int f = *fit;
  *fit = 0;
  if (c.done) return;
  for (int w = 1; w < (nt >> 6); ++w) {
    rp = fmax(rp, red[0][w]);
    rd = fmax(rd, red[1][w]);
    rz = fmax(rz, red[2][w]);
  }
  if (f) A.failures[g] += f;
  ctl_decide(A, g, c, rp, rd, rz);
  c.cur = cur;
  A.ctl[g] = c;
}

// Coupling vectors (u, v, z, y, lambda) are laid out bus-major: generator
// p [n_gen], generator q [n_gen] (generators sorted by bus), then the
// 2 n_branch branch ends in bus CSR order, four consecutive couplings per
// end (p, q, w, theta), so that the couplings of one end share 32 bytes of
// each vector. A branch finds its eight couplings through the positions ef
// (from end) and et (to end) of its two ends.
__host__ __device__ inline int64_t end_coupling(int64_t ng, int64_t ne, int kind, int64_t e) {
  (void)ne;
  return 2 * ng + 4 * e + kind;  // kind 0 p, 1 q, 2 w, 3 theta
}

struct BranchArgs {
  int64_t nl;                // branches in the handle
  int64_t ne;                // branch ends, 2 nl
  const int *ef, *et;        // [nl] end positions of each branch
  const int* br_grid;
  const int* lane_of;        // [G] launch lane of each grid, or null (one lane): a layout
                             // block can span grids of several lanes, and a lane
                             // solves only its own grids' branches and generators
  int lane;
  const GridCtl* ctl;
  const double* adm;         // [8][nl] gii bii gij bij gji bji gjj bjj
  const double *vlo_i, *vhi_i, *vlo_j, *vhi_j, *rate2;
  const double *v, *z, *y;
  const double* brec;        // [nl][16] branch records written by the bus step
  double* u;
  // branch state read (_in) and written: [6][nl], [2][nl], [nl], and the TRON
  // Cauchy step length [nl], carried between solves (two buffers, or one)
  const double *bx_in, *ltil_in, *rtil_in, *calpha_in;
  double *bx, *ltil, *rtil;
  double* calpha;
  double rho_pq, rho_va, tron_gtol, tron_ftol;
  double al_tol, al_shrink, al_rho_growth, al_rho_max;
  int tron_maxit, al_maxit;
  int* failures;             // [G] for the buffer written
  unsigned long long* stats; // [16]
  unsigned* pool;            // [3] next rated / unlimited branch, finished blocks
                             //     (persistent x-step; zero between launches)
  // generator step, fused into the same launch
  int64_t ng;
  const int* gen_grid;
  const double *pmin, *pmax, *qmin, *qmax, *c2q, *c1l;
};

// One launch for the whole x-step with `block` threads per block (a multiple
// of 64): blocks [0, b6) solve rated branches [0, n6), blocks [b6, b6 + b4)
// unlimited branches [n6, nl), the remaining blocks the generators.
// Solution quality (||c(x)||_inf over eq. acopf at the ADMM solution): see
// launch_quality. qmax holds six maxima per grid as bit patterns of
// non-negative doubles (or NaN), combined with integer atomicMax.
struct QualityArgs {
  int64_t nb, ng, nl, ne;
  const int *bus_grid, *br_grid, *gen_grid, *gptr, *eptr, *ef, *et, *end_bus;
  const double *adm, *rate, *u, *v, *pd, *qd, *gs, *bs, *vmin, *vmax;
  double *bw, *bt, *pe, *qe;  // scratch [nb], [nb], [ne], [ne]
  unsigned long long* qmax;   // [G][6], zeroed before the launch
};
void launch_quality(const QualityArgs& Q, hipStream_t s);
// Zeroes n 64-bit words with one block (a kernel rather than hipMemset).
void launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t s);

// Block layout of the lane-per-branch x-step over a handle's index ranges:
// blocks [0, b6) take rated branches [0, n6), one per lane; the next b4
// blocks unlimited branches [n6, nl), k4 per lane, block u's lane i taking
// branch n6 + u bs + i + j b4 bs for j < k4 (bs lanes per block); the last bg
// blocks generators [0, ng), one per lane.
struct XLayout {
  int64_t n6;
  int bg, b6, b4, k4;
};

// Lane-per-branch x-step: n_blocks blocks of `block` lanes. With vblock null
// every block of the layout runs (n_blocks = bg + b6 + b4); otherwise block
// k runs layout block vblock[k] (the blocks that touch running grids).
// stats: also count algorithmic flops and TRON events into A.stats.
// At chunk position pos >= 1 the launch starts with n_dec more blocks, which
// take the previous iteration's control decision of the running grids (one
// block each, dec in device memory, for the results in buffer pos & 1),
// concurrently with the branch solves; A then reads one buffer of the
// branch state and writes the other.
void launch_xstep(const BranchArgs& A, const XLayout& L, const int* vblock, int n_blocks,
                  const DecideArgs* dec, int n_dec, int pos, int block, bool stats,
                  hipStream_t s);
// Whether f is one of the kernels launch_xstep launches (graph node updates).
bool is_xstep_kernel(const void* f);

// Persistent x-step on `blocks` 64-lane blocks; the pool counters must be
// zero at launch and are zero again when it ends.
void launch_xstep_persistent(const BranchArgs& A, int64_t n6, int blocks, bool stats,
                             hipStream_t s);

}  // namespace acopf_dev
