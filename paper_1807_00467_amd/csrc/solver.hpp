// Device kernels of the Gauss-Newton step: Jacobi-PCG vector updates, scalar
// bookkeeping and the Armijo line search, all driven by device scalars so that a
// whole step can run without host round trips.
#pragma once
#include "kernels.hpp"

namespace disco {

// slots of the device scalar array
enum {
  SC_D = 0, SC_SRAW, SC_V, SC_K, SC_NFOLD,      // linearisation: D, sum (Lw)^2, C sum psi, sum |res|^2, folds
  SC_DOT, SC_MAXDIAG, SC_GG,                   // gather reductions: <dotv,out>, max diag, |out|^2
  SC_J, SC_RZ, SC_PQ, SC_ALPHA, SC_BETA, SC_RR, SC_BB, SC_STOP, SC_ITERS, SC_BREAK,
  SC_GTP, SC_TTRY, SC_ACCEPT, SC_TACC, SC_TRIALS,
  SC_TD, SC_TSRAW, SC_TV, SC_TK, SC_TNFOLD,    // trial point reductions
  SC_JT, SC_DT, SC_ST, SC_VT, SC_KT,           // accepted (or last) trial values
  SC_TMP0, SC_TMP1, SC_TMP2,
  SC_COUNT = 48
};

struct Weights {
  double alpha, gamma, delta, CH;  // CH = H_x H_y H_z
};

// J from the reduced terms; a fold counts only when gamma > 0
__device__ inline double total_J(const Weights &w, double D, double Sraw, double V, double K, double nfold) {
  if (w.gamma != 0.0 && nfold > 0.0) return INFINITY;
  return D + w.alpha * 0.5 * w.CH * Sraw + (w.gamma != 0.0 ? w.gamma * V : 0.0) + w.delta * K;
}

__global__ void k_lin_post(double *sc, Weights w, int *status) {
  sc[SC_J] = total_J(w, sc[SC_D], sc[SC_SRAW], sc[SC_V], sc[SC_K], sc[SC_NFOLD]);
  if (status && w.gamma != 0.0 && sc[SC_NFOLD] > 0.0) *status |= 1;
}

// x = 0, r = -g, z = r / M, p = z; per-block <r,z>, <r,r>
__global__ __launch_bounds__(256) void k_pcg_init(int64_t n, const float *g, const float *diag, const double *sc,
                                                  float tau, float *x, float *r, float *z, float *p,
                                                  double *blocks) {
  __shared__ double red[2][256];
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
  const int t = threadIdx.x;
  red[0][t] = rz;
  red[1][t] = rr;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      red[0][t] += red[0][t + s];
      red[1][t] += red[1][t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    blocks[2 * blockIdx.x] = red[0][0];
    blocks[2 * blockIdx.x + 1] = red[1][0];
  }
}

// after reducing <r,z>, <r,r> of the initial residual
__global__ void k_pcg_start(double *sc) {
  sc[SC_RZ] = sc[SC_TMP0];
  sc[SC_BB] = sc[SC_TMP1];
  sc[SC_RR] = sc[SC_TMP1];
  sc[SC_STOP] = 0.0;
  sc[SC_ITERS] = 0.0;
  sc[SC_BREAK] = 0.0;
}

// alpha = rz / pq, or breakdown
__global__ void k_pcg_alpha(double *sc, int *status) {
  if (sc[SC_STOP] != 0.0) return;
  const double pq = sc[SC_DOT];
  if (!(pq > 0.0)) {
    sc[SC_STOP] = 1.0;
    sc[SC_BREAK] = 1.0;
    if (status) *status |= 2;
    return;
  }
  sc[SC_ALPHA] = sc[SC_RZ] / pq;
}

// x += a p; r -= a q; z = r / M; per-block <r,z>, <r,r>
__global__ __launch_bounds__(256) void k_pcg_update(int64_t n, const double *sc, const float *diag, float tau,
                                                    const float *p, const float *q, float *x, float *r, float *z,
                                                    double *blocks) {
  __shared__ double red[2][256];
  if (sc[SC_STOP] != 0.0) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const float a = (float)sc[SC_ALPHA];
  double rz = 0.0, rr = 0.0;
  if (i < n) {
    const float M = diag[i] + tau + (float)(1e-12 * sc[SC_MAXDIAG]);
    x[i] += a * p[i];
    const float ri = r[i] - a * q[i];
    r[i] = ri;
    const float zi = ri / M;
    z[i] = zi;
    rz = (double)ri * (double)zi;
    rr = (double)ri * (double)ri;
  }
  const int t = threadIdx.x;
  red[0][t] = rz;
  red[1][t] = rr;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      red[0][t] += red[0][t + s];
      red[1][t] += red[1][t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    blocks[2 * blockIdx.x] = red[0][0];
    blocks[2 * blockIdx.x + 1] = red[1][0];
  }
}

// beta = rz_new / rz; convergence test
__global__ void k_pcg_beta(double *sc, double tol) {
  if (sc[SC_STOP] != 0.0) return;
  const double rz_new = sc[SC_TMP0];
  sc[SC_RR] = sc[SC_TMP1];
  sc[SC_ITERS] += 1.0;
  sc[SC_BETA] = rz_new / sc[SC_RZ];
  sc[SC_RZ] = rz_new;
  if (tol > 0.0 && sqrt(sc[SC_RR]) <= tol * sqrt(sc[SC_BB])) sc[SC_STOP] = 1.0;
}

__global__ __launch_bounds__(256) void k_pcg_p(int64_t n, const double *sc, const float *z, float *p) {
  if (sc[SC_STOP] != 0.0) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = z[i] + (float)sc[SC_BETA] * p[i];
}

// per-block <a, b>
__global__ __launch_bounds__(256) void k_dot(int64_t n, const float *a, const float *b, double *blocks) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int t = threadIdx.x;
  red[t] = i < n ? (double)a[i] * (double)b[i] : 0.0;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  if (t == 0) blocks[blockIdx.x] = red[0];
}

__global__ void k_ls_begin(double *sc) {
  sc[SC_GTP] = sc[SC_TMP0];
  sc[SC_ACCEPT] = 0.0;
  sc[SC_TACC] = 0.0;
  sc[SC_TRIALS] = 0.0;
  sc[SC_JT] = INFINITY;
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

// Armijo test of the trial just evaluated (reductions in SC_TD..SC_TNFOLD)
__global__ void k_ls_decide(double *sc, Weights w, double c1) {
  if (sc[SC_ACCEPT] != 0.0) return;
  const double t = sc[SC_TTRY];
  const double Jt = total_J(w, sc[SC_TD], sc[SC_TSRAW], sc[SC_TV], sc[SC_TK], sc[SC_TNFOLD]);
  sc[SC_TRIALS] += 1.0;
  sc[SC_JT] = Jt;
  sc[SC_DT] = sc[SC_TD];
  sc[SC_ST] = 0.5 * w.CH * sc[SC_TSRAW];
  sc[SC_VT] = sc[SC_TV];
  sc[SC_KT] = sc[SC_TK];
  if (isfinite(Jt) && Jt <= sc[SC_J] + c1 * t * sc[SC_GTP]) {
    sc[SC_ACCEPT] = 1.0;
    sc[SC_TACC] = t;
  }
}

// accept: u = ut; report and status
__global__ __launch_bounds__(256) void k_ls_finish(int64_t n, const double *sc, const float *ut, float *u) {
  if (sc[SC_ACCEPT] == 0.0) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) u[i] = ut[i];
}

__global__ void k_report(const double *sc, Weights w, double *rep, int *status, int *status_out) {
  if (rep) {
    rep[0] = sc[SC_J];
    rep[1] = sc[SC_D];
    rep[2] = 0.5 * w.CH * sc[SC_SRAW];
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

// brick reductions (SC_TMP0 + BS_*) -> linearisation slots
__global__ void k_lin_move(double *sc, double h3) {
  sc[SC_D] = sc[SC_TMP0 + BS_D] * h3;
  sc[SC_V] = sc[SC_TMP0 + BS_V];
  sc[SC_K] = sc[SC_TMP0 + BS_K];
  sc[SC_NFOLD] = sc[SC_TMP0 + BS_FOLD];
}

// brick reductions -> trial slots (skipped once a trial was accepted)
__global__ void k_ls_move(double *sc, double h3) {
  if (sc[SC_ACCEPT] != 0.0) return;
  sc[SC_TD] = sc[SC_TMP0 + BS_D] * h3;
  sc[SC_TV] = sc[SC_TMP0 + BS_V];
  sc[SC_TK] = sc[SC_TMP0 + BS_K];
  sc[SC_TNFOLD] = sc[SC_TMP0 + BS_FOLD];
}

__global__ void k_clear_status(int *status) { *status = 0; }

// small scalar helpers for the single-term entry points
__global__ void k_write_scalar(const double *src, double scale, double *dst, const double *fold, int fold_inf) {
  double v = *src * scale;
  if (fold_inf && fold && *fold > 0.0) v = INFINITY;
  *dst = v;
}
__global__ void k_write_int(const double *src, int32_t *dst) { *dst = (int32_t)(*src); }

}  // namespace disco
