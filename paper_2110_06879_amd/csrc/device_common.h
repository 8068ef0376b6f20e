// Device-side data shared by the host runtime and the kernels of the ADMM
// library (internal; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace acopf_dev {

// Per-grid control block of Algorithm 1, updated by the control kernel.
struct GridCtl {
  double beta;        // outer penalty
  double beta_lam;    // beta used by a pending lambda update
  double znorm_prev;  // ||z||_inf at the previous outer update (inf at start)
  double r_pri, r_dual, r_z;
  int outer, inner_total, inner_in_outer, status;
  int done, do_outer, fixed_target, branch_failures;
  int numerical, fixed_mode, running, pad2;  // fixed_mode: stop only at fixed_target
};

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
  const GridCtl* ctl;
  const double* adm;         // [8][nl] gii bii gij bij gji bji gjj bjj
  const double *vlo_i, *vhi_i, *vlo_j, *vhi_j, *rate2;
  const double *v, *z, *y;
  const double* brec;        // [nl][16] branch records written by the bus step
  double* u;
  double *bx, *ltil, *rtil;  // [6][nl], [2][nl], [nl]
  double* calpha;            // [nl] TRON Cauchy step length, carried between solves
  double rho_pq, rho_va, tron_gtol, tron_ftol;
  double al_tol, al_shrink, al_rho_growth, al_rho_max;
  int tron_maxit, al_maxit;
  int* failures;             // [G]
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
void launch_xstep(const BranchArgs& A, const XLayout& L, const int* vblock, int n_blocks,
                  int block, bool stats, hipStream_t s);
// Whether f is one of the kernels launch_xstep launches (graph node updates).
bool is_xstep_kernel(const void* f);

// Persistent x-step on `blocks` 64-lane blocks; the pool counters must be
// zero at launch and are zero again when it ends.
void launch_xstep_persistent(const BranchArgs& A, int64_t n6, int blocks, bool stats,
                             hipStream_t s);

}  // namespace acopf_dev
