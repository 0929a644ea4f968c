// Device kernels of the Gauss-Newton step: Jacobi-PCG vector updates and the Armijo
// line search, driven by device scalars (SC_* slots) so that a whole step runs without
// host round trips.  Inside the CG loop every workgroup of a consumer kernel reduces
// the producer's per-block partials itself (same fixed order everywhere); the other
// scalar bookkeeping runs in the single-workgroup k_finish (run_post).
#pragma once
#include "kernels.hpp"

namespace disco {

// the stop flag read once per workgroup (another workgroup of the same launch may set
// it), so that the whole workgroup takes the same branch before any barrier
__device__ inline bool block_stopped(const double *sc) {
  __shared__ int s_stop;
  if (threadIdx.x == 0) s_stop = sc[SC_STOP] != 0.0;
  __syncthreads();
  return s_stop != 0;
}

// per-block sums of two values over 256 threads (fixed tree)
__device__ inline void block_pair_sum(double x, double y, double *blocks, int64_t bid) {
  __shared__ double red[2][256];
  const int t = threadIdx.x;
  red[0][t] = x;
  red[1][t] = y;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      red[0][t] += red[0][t + s];
      red[1][t] += red[1][t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    blocks[2 * bid] = red[0][0];
    blocks[2 * bid + 1] = red[1][0];
  }
}

// x = 0, r = -g, z = r / M, p = z; per-block <r,z>, <r,r>
__global__ __launch_bounds__(256) void k_pcg_init(int64_t n, const float *g, const float *diag, const double *sc,
                                                  float tau, float *x, float *r, float *z, float *p,
                                                  double *blocks) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (i < n) {
    const float M = diag[i] + tau + (float)(1e-12 * sc[SC_MAXDIAG]);
    const float ri = -g[i];
    const float zi = ri / M;
    x[i] = 0.0f;
    r[i] = ri;
    z[i] = zi;
    p[i] = zi;
    rz = (double)ri * (double)zi;
    rr = (double)ri * (double)ri;
  }
  block_pair_sum(rz, rr, blocks, blockIdx.x);
}

// CG iteration, part 1 (grid-stride, few workgroups): every workgroup reduces the
// per-block <p, H p> of the product pass itself (same fixed order everywhere), so no
// separate reduction launch is needed.  alpha = <r,z> / <p,Hp>; x += alpha p,
// r -= alpha q, z = r / M; per-workgroup <r,z>, <r,r>.  <r,z> of this iteration is in
// slot SC_RZ + (it & 1).
__global__ __launch_bounds__(256) void k_pcg_update(int64_t n, double *sc, int it, const double *pq_blocks,
                                                    int64_t pq_nb, const float *diag, float tau, const float *p,
                                                    const float *q, float *x, float *r, float *z, double *blocks,
                                                    int *status) {
  __shared__ double red[256];
  if (block_stopped(sc)) return;
  const double pq = block_sum_all(pq_blocks, pq_nb, 3, 0, red);
  if (!(pq > 0.0)) {
    // breakdown: every workgroup sees the same pq and skips the update
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc[SC_STOP] = 1.0;
      sc[SC_BREAK] = 1.0;
      *status |= 2;
    }
    return;
  }
  const double alpha = sc[SC_RZ + (it & 1)] / pq;
  const float a = (float)alpha;
  const float M0 = tau + (float)(1e-12 * sc[SC_MAXDIAG]);
  double rz = 0.0, rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float M = diag[i] + M0;
    x[i] += a * p[i];
    const float ri = r[i] - a * q[i];
    r[i] = ri;
    const float zi = ri / M;
    z[i] = zi;
    rz += (double)ri * (double)zi;
    rr += (double)ri * (double)ri;
  }
  block_pair_sum(rz, rr, blocks, blockIdx.x);
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[SC_ALPHA] = alpha;
}

// CG iteration, part 2: every workgroup reduces the <r,z>, <r,r> partials of part 1;
// beta = <r,z>_new / <r,z>; p = z + beta p unless this was the last iteration or the
// tolerance is met.  Workgroup 0 records the scalars for the next iteration.
__global__ __launch_bounds__(256) void k_pcg_p(int64_t n, double *sc, int it, int last, double tol,
                                               const double *blocks, int64_t nb, const float *z, float *p) {
  __shared__ double red[256];
  if (block_stopped(sc)) return;
  const double rz_new = block_sum_all(blocks, nb, 2, 0, red);
  const double rr = block_sum_all(blocks, nb, 2, 1, red);
  const double beta = rz_new / sc[SC_RZ + (it & 1)];
  const bool conv = tol > 0.0 && sqrt(rr) <= tol * sqrt(sc[SC_BB]);
  if (!last && !conv) {
    const float b = (float)beta;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
      p[i] = z[i] + b * p[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[SC_RZ + ((it + 1) & 1)] = rz_new;
    sc[SC_RR] = rr;
    sc[SC_BETA] = beta;
    sc[SC_ITERS] = (double)(it + 1);
    if (conv) sc[SC_STOP] = 1.0;
  }
}

// per-block <a, b>
__global__ __launch_bounds__(256) void k_dot(int64_t n, const float *a, const float *b, double *blocks) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double x = i < n ? (double)a[i] * (double)b[i] : 0.0;
  block_pair_sum(x, 0.0, blocks, blockIdx.x);
}

// trial point ut = u + t x with t = 2^-trial
__global__ __launch_bounds__(256) void k_ls_point(int64_t n, double *sc, int trial, const float *u, const float *x,
                                                  float *ut) {
  if (sc[SC_ACCEPT] != 0.0) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const float t = ldexpf(1.0f, -trial);
  if (i < n) ut[i] = u[i] + t * x[i];
  if (i == 0) sc[SC_TTRY] = (double)t;
}

// accept: u = ut
__global__ __launch_bounds__(256) void k_ls_finish(int64_t n, const double *sc, const float *ut, float *u) {
  if (sc[SC_ACCEPT] == 0.0) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) u[i] = ut[i];
}

__global__ void k_report(const double *sc, double CH, double *rep, int *status, int *status_out) {
  if (rep) {
    rep[0] = sc[SC_J];
    rep[1] = sc[SC_D];
    rep[2] = 0.5 * CH * sc[SC_SRAW];
    rep[3] = sc[SC_NFOLD] > 0.0 ? INFINITY : sc[SC_V];
    rep[4] = sc[SC_K];
    rep[5] = sqrt(sc[SC_GG]);
    rep[6] = sc[SC_TACC];
    rep[7] = sc[SC_ITERS];
    rep[8] = sqrt(sc[SC_RR]);
    rep[9] = sc[SC_GTP];
    rep[10] = sc[SC_JT];
    rep[11] = sc[SC_DT];
    rep[12] = sc[SC_ST];
    rep[13] = sc[SC_TNFOLD] > 0.0 ? INFINITY : sc[SC_VT];
    rep[14] = sc[SC_KT];
    rep[15] = sc[SC_TRIALS];
  }
  if (sc[SC_ACCEPT] == 0.0) *status |= 4;
  if (status_out) *status_out = *status;
}

__global__ void k_clear_status(int *status) { *status = 0; }

}  // namespace disco
