// Batched Gauss-Newton step over many image pairs of uneven sizes.  Every phase of the
// step (brick passes, gathers, curvature, CG vector updates, line search, reductions) is
// ONE persistent launch over the work items of all pairs: a workgroup walks the items
// (pair, block) of a flattened list in which the pairs are ordered largest first, and
// runs the same device body as the single-pair kernel with that pair's descriptor and
// block coordinates, so each pair gets the single-pair arithmetic (up to the rounding of
// multiply-adds, which the compiler may fuse differently in the two kernels).  The whole
// sequence contains no host synchronisation and can be captured in one graph.
#pragma once
#include "kernels.hpp"
#include "solver.hpp"

namespace disco {

// what the finish reduction of a phase reads (up to three sources) and which
// post-operation it runs
struct FinishArgs {
  RedSrc s0, s1, s2;
  int nsrc, post;
  PostArgs pa;
  const double *stop;
};

// Everything one pair needs for a GN step; built on the host, stored in device memory.
template <class ST>
struct PairDesc {
  Geo g;
  BrickArgs<ST> lin;    // linearisation pass (M_GRAD) at u
  BrickArgs<ST> hv[2];  // GN product passes with v = p[0] / p[1]
  BrickArgs<ST> eval;   // line-search trial pass (M_EVAL) at ut, skipped once accepted
  GatherArgs glin;      // after the linearisation pass: g, diag + curvature, partials
  GatherArgs ghv[2];    // after the product passes: Hv + curvature + tau v, <v, Hv> partials
  FinishArgs fin_lin, fin_pcg, fin_lsb, fin_trial;
  float *u, *u_ref, *u_lin, *Lw, *grad, *diag, *x, *r, *z, *p[2], *q, *ut, *invM;
  double *sc, *blk_node, *blk_curv, *blk_upd;
  int *status;
  double *report;       // this pair's 16 report slots (nullable)
  int32_t *status_out;  // this pair's status word (nullable)
  int64_t n3, nodeblocks;
  float tau;
  double tol;
  double CH;
};

// the pair holding item `item` of a flattened work list (start[p] = first item of pair p,
// start[npairs] = total): largest p with start[p] <= item; uniform over the workgroup
__device__ __forceinline__ int find_pair(const int *start, int npairs, int item) {
  int lo = 0, hi = npairs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// block coordinates of local item `l` in a 3-D grid (nx, ny) x nz
__device__ __forceinline__ Blk grid_blk(int64_t l, int nx, int ny) {
  const int x = (int)(l % nx);
  const int64_t r = l / nx;
  return Blk{x, (int)(r % ny), (int)(r / ny), l};
}

__device__ __forceinline__ int node_gx(const Geo &g) { return (g.px + 63) / 64; }
__device__ __forceinline__ int node_gy(const Geo &g) { return (g.py + 3) / 4; }

// ---- brick passes -------------------------------------------------------------------
// sel: 0 = linearisation, 1/2 = GN product with p[0]/p[1], 3 = line-search trial; ZC: cell
// layers per brick (the batch's tile; the descriptors' geometry carries the matching
// brick counts)
template <class ST, int MODE, bool NGF, bool VCC, bool KP, int ZC>
__global__ __launch_bounds__(256, 1) void k_b_brick(const PairDesc<ST> *D,
                                                                                   const int *start, int npairs,
                                                                                   int sel, int acc) {
  const int total = start[npairs];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int pr = find_pair(start, npairs, item);
    const PairDesc<ST> &P = D[pr];
    const BrickArgs<ST> &A = sel == 0 ? P.lin : (sel == 3 ? P.eval : P.hv[sel - 1]);
    brick_body<ST, MODE, NGF, VCC, KP, ZC, false, true>(A, grid_blk(item - start[pr], A.g.nbx, A.g.nby), acc);
    __syncthreads();  // the next item reuses the workgroup's LDS
  }
}

// A brick pass with one workgroup per work item (grid = the items): the same body as
// k_b_brick without its work-item loop, whose addressing costs registers.
template <class ST, int MODE, bool NGF, bool VCC, bool KP, int ZC>
__global__ __launch_bounds__(256, (MODE == M_EVAL && NGF) ? 4 : 1) void k_b_brick_item(const PairDesc<ST> *D, const int *start, int npairs, int sel,
                                                     int acc) {
  const int item = blockIdx.x;
  if (item >= start[npairs]) return;
  const int pr = find_pair(start, npairs, item);
  const PairDesc<ST> &P = D[pr];
  const BrickArgs<ST> &A = sel == 0 ? P.lin : (sel == 3 ? P.eval : P.hv[sel - 1]);
  brick_body<ST, MODE, NGF, VCC, KP, ZC, false, true>(A, grid_blk(item - start[pr], A.g.nbx, A.g.nby), acc);
}

// GN product pass with one workgroup per work item in the role split of the single-pair
// kernel (four waves stream the voxels, four compute the cell terms): 8-wave workgroups
// that fit two to a compute unit.  The same brick body, so the same sums as k_b_brick.
template <class ST, bool VCC, bool KP, int ZC>
__global__ __launch_bounds__(512) void k_b_brick_split(const PairDesc<ST> *D, const int *start, int npairs, int sel,
                                                      int acc) {
  const int item = blockIdx.x;
  if (item >= start[npairs]) return;
  const int pr = find_pair(start, npairs, item);
  const PairDesc<ST> &P = D[pr];
  const BrickArgs<ST> &A = P.hv[sel - 1];
  brick_body<ST, M_HV, true, VCC, KP, ZC, false, false>(A, grid_blk(item - start[pr], A.g.nbx, A.g.nby), acc);
}

// ---- node-parallel passes -----------------------------------------------------------
// sel: 0 = after linearisation, 1/2 = after the product with p[0]/p[1]; ZC as in k_b_brick
template <class ST, int F, int NF, bool CURV, int ZC>
__global__ __launch_bounds__(256) void k_b_gather(const PairDesc<ST> *D, const int *start, int npairs, int sel) {
  const int total = start[npairs];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int pr = find_pair(start, npairs, item);
    const PairDesc<ST> &P = D[pr];
    const GatherArgs &A = sel == 0 ? P.glin : P.ghv[sel - 1];
    gather_body<ZC, F, NF, CURV>(A, grid_blk(item - start[pr], node_gx(P.g), node_gy(P.g)));
    __syncthreads();
  }
}

// sel: 0 = L(u - uhat) with energy (linearisation), 1 = L p[0] (first CG product),
// 2 = L(ut - uhat) with energy, skipped once the line search accepted
template <class ST>
__global__ __launch_bounds__(256) void k_b_curv_L(const PairDesc<ST> *D, const int *start, int npairs, int sel) {
  const int total = start[npairs];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int pr = find_pair(start, npairs, item);
    const PairDesc<ST> &P = D[pr];
    const Blk B = grid_blk(item - start[pr], node_gx(P.g), node_gy(P.g));
    if (sel == 0)
      curv_L_body(P.g, P.u, P.u_ref, P.Lw, P.blk_curv, nullptr, B);
    else if (sel == 1)
      curv_L_body(P.g, P.p[0], nullptr, P.Lw, nullptr, P.sc + SC_STOP, B);
    else
      curv_L_body(P.g, P.ut, P.u_ref, P.Lw, P.blk_curv, P.sc + SC_ACCEPT, B);
    __syncthreads();
  }
}

template <class ST>
__global__ __launch_bounds__(256) void k_b_curv_Lp(const PairDesc<ST> *D, const int *start, int npairs, int it) {
  const int total = start[npairs];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int pr = find_pair(start, npairs, item);
    const PairDesc<ST> &P = D[pr];
    const int64_t nbu = (P.n3 + 256 * kUpdK - 1) / (256 * kUpdK);
    curv_Lp_body<1>(P.g, it, P.sc, P.tol, P.blk_upd, nbu, P.z, P.p[(it - 1) & 1], P.p[it & 1], P.Lw,
                 grid_blk(item - start[pr], node_gx(P.g), node_gy(P.g)));
    __syncthreads();
  }
}

// ---- node-vector passes (256 elements per item) -------------------------------------
// op: 0 = u_lin = u, 1 = PCG start, 2 = <g, x> partials, 3 = trial point, 4 = accept
template <class ST>
__global__ __launch_bounds__(256) void k_b_vec(const PairDesc<ST> *D, const int *start, int npairs, int op,
                                               int trial) {
  const int total = start[npairs];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int pr = find_pair(start, npairs, item);
    const PairDesc<ST> &P = D[pr];
    const int64_t bid = item - start[pr];
    if (op == 0)
      copy_body(P.n3, P.u, P.u_lin, bid);
    else if (op == 1)
      pcg_init_body(P.n3, P.grad, P.diag, P.sc, P.tau, -1.0f, P.x, P.r, P.z, P.p[0], P.invM, P.blk_node, bid);
    else if (op == 2)
      dot_body(P.n3, P.grad, P.x, P.blk_node, bid);
    else if (op == 3)
      ls_point_body(P.n3, P.sc, trial, P.u, P.x, P.ut, bid);
    else
      ls_finish_body(P.n3, P.sc, P.ut, P.u, bid);
    __syncthreads();
  }
}

// CG update (256 * kUpdK elements per item)
template <class ST>
__global__ __launch_bounds__(256) void k_b_pcg_update(const PairDesc<ST> *D, const int *start, int npairs, int it) {
  const int total = start[npairs];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int pr = find_pair(start, npairs, item);
    const PairDesc<ST> &P = D[pr];
    pcg_update_body(P.n3, P.sc, it, P.blk_node, P.nodeblocks, P.invM, P.p[it & 1], P.q, P.x, P.r, P.z, P.blk_upd,
                    P.status, item - start[pr]);
    __syncthreads();
  }
}

// ---- per-pair scalar work (one workgroup per pair) ----------------------------------
// which: 0 = linearisation, 1 = PCG start, 2 = line-search begin, 3 = trial
template <class ST>
__global__ __launch_bounds__(1024) void k_b_finish(const PairDesc<ST> *D, int npairs, int which) {
  for (int pr = blockIdx.x; pr < npairs; pr += gridDim.x) {
    const PairDesc<ST> &P = D[pr];
    const FinishArgs &F = which == 0 ? P.fin_lin : (which == 1 ? P.fin_pcg : (which == 2 ? P.fin_lsb : P.fin_trial));
    finish_body(F.s0, F.s1, F.s2, F.nsrc, F.post, F.pa, F.stop);
    __syncthreads();
  }
}

// begin (clear the status word) or end (report) of the step, one thread per pair
template <class ST>
__global__ void k_b_status(const PairDesc<ST> *D, int npairs, int end) {
  const int pr = blockIdx.x * blockDim.x + threadIdx.x;
  if (pr >= npairs) return;
  const PairDesc<ST> &P = D[pr];
  if (end)
    report_body(P.sc, P.CH, P.report, P.status, P.status_out);
  else
    *P.status = 0;
}

}  // namespace disco
