// Device kernels of the Gauss-Newton step: Jacobi-PCG vector updates and the Armijo
// line search, driven by device scalars (SC_* slots) so that a whole step runs without
// host round trips.  Inside the CG loop every workgroup of a consumer kernel reduces
// the producer's per-block partials itself (same fixed order everywhere); the other
// scalar bookkeeping runs in the single-workgroup k_finish (run_post).
#pragma once
#include "kernels.hpp"

namespace disco {

// per-block sums of two values over 256 threads (fixed order)
__device__ inline void block_pair_sum(double x, double y, double *blocks, int64_t bid) {
  const double v[2] = {x, y};
  block_write<2>(v, blocks + 2 * bid);
}

// x = 0, r = sgn g (sgn = -1: the GN system H x = -g; +1: a system A x = g), z = r / M,
// p = z, invM = 1 / M; per-block <r,z>, <r,r>
__device__ __forceinline__ void pcg_init_body(int64_t n, const float *__restrict__ g, const float *__restrict__ diag,
                                              const double *sc, float tau, float sgn, float *__restrict__ x,
                                              float *__restrict__ r, float *__restrict__ z, float *__restrict__ p,
                                              float *__restrict__ invM, double *blocks, int64_t bid) {
  const int64_t i = bid * 256 + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (i < n) {
    const float M = diag[i] + tau + (float)(1e-12 * sc[SC_MAXDIAG]);
    const float iM = 1.0f / M;
    const float ri = sgn * g[i];
    const float zi = ri * iM;
    x[i] = 0.0f;
    r[i] = ri;
    z[i] = zi;
    p[i] = zi;
    invM[i] = iM;
    rz = (double)ri * (double)zi;
    rr = (double)ri * (double)ri;
  }
  block_pair_sum(rz, rr, blocks, bid);
}
__global__ __launch_bounds__(256) void k_pcg_init(int64_t n, const float *__restrict__ g,
                                                  const float *__restrict__ diag, const double *sc, float tau,
                                                  float sgn, float *__restrict__ x, float *__restrict__ r,
                                                  float *__restrict__ z, float *__restrict__ p, float *__restrict__ invM,
                                                  double *blocks) {
  pcg_init_body(n, g, diag, sc, tau, sgn, x, r, z, p, invM, blocks, blockIdx.x);
}

// elements per thread of the CG vector update (workgroup covers 256 * kUpdK elements)
constexpr int kUpdK = 16;

// CG iteration, vector part: every workgroup reduces the per-block <p, H p> of the
// product pass itself (same fixed order everywhere).  alpha = <r,z> / <p,Hp>;
// x += alpha p, r -= alpha q, z = r / M; per-workgroup <r,z>, <r,r>.  <r,z> of this
// iteration is in slot SC_RZ + (it & 1).  The vector loads, the partials and the stop
// flag are all requested before the first wait.
__device__ __forceinline__ void pcg_update_body(int64_t n, double *sc, int it, const double *pq_blocks, int64_t pq_nb,
                                                const float *__restrict__ invM, const float *__restrict__ p,
                                                const float *__restrict__ q, float *__restrict__ x,
                                                float *__restrict__ r, float *__restrict__ z, double *blocks,
                                                int *status, int64_t bid) {
  const int64_t base = bid * (256 * kUpdK) + threadIdx.x;
  float vp[kUpdK], vq[kUpdK], vx[kUpdK], vr[kUpdK], vm[kUpdK];
#pragma unroll
  for (int k = 0; k < kUpdK; ++k) {
    const int64_t i = base + k * 256;
    const bool in = i < n;
    const int64_t j = in ? i : 0;
    vp[k] = p[j];
    vq[k] = q[j];
    vx[k] = x[j];
    vr[k] = r[j];
    vm[k] = in ? invM[j] : 0.0f;
  }
  const double rz_old = sc[SC_RZ + (it & 1)];
  double pq, stop;
  block_sums<1>(pq_blocks, pq_nb, 3, 0, &pq, sc + SC_STOP, &stop);
  if (stop != 0.0) return;
  if (!(pq > 0.0)) {
    // breakdown: every workgroup sees the same pq and skips the update
    if (bid == 0 && threadIdx.x == 0) {
      sc[SC_STOP] = 1.0;
      sc[SC_BREAK] = 1.0;
      *status |= 2;
    }
    return;
  }
  const double alpha = rz_old / pq;
  const float a = (float)alpha;
  double rz = 0.0, rr = 0.0;
#pragma unroll
  for (int k = 0; k < kUpdK; ++k) {
    const int64_t i = base + k * 256;
    const float ri = vr[k] - a * vq[k];
    const float zi = ri * vm[k];
    if (i < n) {
      x[i] = vx[k] + a * vp[k];
      r[i] = ri;
      z[i] = zi;
      rz += (double)ri * (double)zi;
      rr += (double)ri * (double)ri;
    }
  }
  block_pair_sum(rz, rr, blocks, bid);
  if (bid == 0 && threadIdx.x == 0) {
    sc[SC_ALPHA] = alpha;
    sc[SC_ITERS] = (double)(it + 1);
  }
}
__global__ __launch_bounds__(256) void k_pcg_update(int64_t n, double *sc, int it, const double *pq_blocks,
                                                    int64_t pq_nb, const float *__restrict__ invM,
                                                    const float *__restrict__ p, const float *__restrict__ q,
                                                    float *__restrict__ x, float *__restrict__ r,
                                                    float *__restrict__ z, double *blocks, int *status) {
  pcg_update_body(n, sc, it, pq_blocks, pq_nb, invM, p, q, x, r, z, blocks, status, blockIdx.x);
}

// Start of CG iteration it >= 1: every workgroup reduces the <r,z>, <r,r> partials of
// the previous update; beta = <r,z>_new / <r,z>_old; stop when the tolerance is met.
// Otherwise p_new = z + beta p_old (written to p_new) and L p_new (the curvature
// operator of the next product) in the same pass: L at node m needs p_new at the
// 6 neighbours, which are formed from z and p_old there.  A workgroup takes a 64 x 4 node
// tile of NZ consecutive planes, walking up in z with the -z, centre and +z values rolled
// in registers, so that each plane is read once per tile; the first plane's loads are
// requested before the first wait.  Stencil neighbours outside the interior (chi = 0)
// carry weight zero.
template <int NZ>
__device__ __forceinline__ void curv_Lp_body(const Geo &g, int it, double *sc, double tol, const double *upd_blocks,
                                             int64_t upd_nb, const float *__restrict__ z,
                                             const float *__restrict__ p_old, float *__restrict__ p_new,
                                             float *__restrict__ Lw, const Blk &B) {
  const int px = B.x * 64 + (threadIdx.x & 63), py = B.y * 4 + (threadIdx.x >> 6), z0 = B.z * NZ;
  const bool in = px < g.px && py < g.py && z0 < g.pz;
  const int qx = in ? px : 0, qy = in ? py : 0, qz = in ? z0 : 0;
  const int64_t sy = g.px, sz = (int64_t)g.px * g.py;
  const bool ux = chi(qx, g.px) != 0, uy = chi(qy, g.py) != 0;
  const int64_t oxm = ux ? -1 : 0, oxp = ux ? 1 : 0, oym = uy ? -sy : 0, oyp = uy ? sy : 0;
  const float wx = ux ? 1.0f : 0.0f, wy = uy ? 1.0f : 0.0f;
  // [component][centre, -x, +x, -y, +y, -z, +z] of z and p_old at plane qz; -z and +z
  // clamped to the volume
  float zc[3][7], pc[3][7];
  int64_t nidx = ((int64_t)qz * g.py + qy) * g.px + qx;
  {
    const int64_t ozm = qz > 0 ? -sz : 0, ozp = qz < g.pz - 1 ? sz : 0;
    const int64_t offs[7] = {0, oxm, oxp, oym, oyp, ozm, ozp};
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < 7; ++m) {
        const int64_t off = c * g.nnodes + nidx + offs[m];
        zc[c][m] = z[off];
        pc[c][m] = p_old[off];
      }
  }
  const double rz_prev = sc[SC_RZ + ((it - 1) & 1)];
  double sums[2], stop;
  block_sums<2>(upd_blocks, upd_nb, 2, 0, sums, sc + SC_STOP, &stop);
  if (stop != 0.0) return;
  const double rz_new = sums[0], rr = sums[1];
  const double beta = rz_new / rz_prev;
  const bool conv = tol > 0.0 && sqrt(rr) <= tol * sqrt(sc[SC_BB]);
  if (B.lin == 0 && threadIdx.x == 0) {
    sc[SC_RZ + (it & 1)] = rz_new;
    sc[SC_RR] = rr;
    sc[SC_BETA] = beta;
    if (conv) sc[SC_STOP] = 1.0;
  }
  if (conv || !in) return;
  const float b = (float)beta;
  const float ih2[3] = {g.iHx * g.iHx, g.iHy * g.iHy, g.iHz * g.iHz};
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    const int pz = z0 + k;
    if (pz >= g.pz) break;
    // the next plane's x, y neighbours and +z centre are requested before this plane's
    // arithmetic; its -z and centre values are this plane's centre and +z
    const bool more = k + 1 < NZ && pz + 1 < g.pz;
    float zn[3][5], pn[3][5];
    if (more) {
      const int64_t ozp = pz + 1 < g.pz - 1 ? sz : 0;
      const int64_t offs[5] = {oxm, oxp, oym, oyp, ozp};
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int m = 0; m < 5; ++m) {
          const int64_t off = c * g.nnodes + nidx + sz + offs[m];
          zn[c][m] = z[off];
          pn[c][m] = p_old[off];
        }
    }
    const float wz = chi(pz, g.pz) ? 1.0f : 0.0f;
    const float wgt[3] = {wx, wy, wz};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float w[7];
#pragma unroll
      for (int m = 0; m < 7; ++m) w[m] = zc[c][m] + b * pc[c][m];
      float acc = 0.0f;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) acc += wgt[ax] * (w[1 + 2 * ax] - 2.0f * w[0] + w[2 + 2 * ax]) * ih2[ax];
      const int64_t off = c * g.nnodes + nidx;
      p_new[off] = w[0];
      Lw[off] = acc;
    }
    if (more) {
      nidx += sz;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        zc[c][5] = zc[c][0];
        pc[c][5] = pc[c][0];
        zc[c][0] = zc[c][6];
        pc[c][0] = pc[c][6];
#pragma unroll
        for (int m = 0; m < 5; ++m) {
          zc[c][m < 4 ? 1 + m : 6] = zn[c][m];
          pc[c][m < 4 ? 1 + m : 6] = pn[c][m];
        }
      }
    }
  }
}

constexpr int kLpZ = 4;  // node planes per workgroup of k_curv_Lp
__global__ __launch_bounds__(256) void k_curv_Lp(Geo g, int it, double *sc, double tol, const double *upd_blocks,
                                                 int64_t upd_nb, const float *__restrict__ z,
                                                 const float *__restrict__ p_old, float *__restrict__ p_new,
                                                 float *__restrict__ Lw) {
  curv_Lp_body<kLpZ>(g, it, sc, tol, upd_blocks, upd_nb, z, p_old, p_new, Lw, hw_blk());
}

// per-block <a, b>
__device__ __forceinline__ void dot_body(int64_t n, const float *a, const float *b, double *blocks, int64_t bid) {
  const int64_t i = bid * 256 + threadIdx.x;
  const double x = i < n ? (double)a[i] * (double)b[i] : 0.0;
  block_pair_sum(x, 0.0, blocks, bid);
}
__global__ __launch_bounds__(256) void k_dot(int64_t n, const float *a, const float *b, double *blocks) {
  dot_body(n, a, b, blocks, blockIdx.x);
}

// trial point ut = u + t x with t = 2^-trial
__device__ __forceinline__ void ls_point_body(int64_t n, double *sc, int trial, const float *u, const float *x,
                                              float *ut, int64_t bid) {
  if (sc[SC_ACCEPT] != 0.0) return;
  const int64_t i = bid * 256 + threadIdx.x;
  const float t = ldexpf(1.0f, -trial);
  if (i < n) ut[i] = u[i] + t * x[i];
  if (i == 0) sc[SC_TTRY] = (double)t;
}
__global__ __launch_bounds__(256) void k_ls_point(int64_t n, double *sc, int trial, const float *u, const float *x,
                                                  float *ut) {
  ls_point_body(n, sc, trial, u, x, ut, blockIdx.x);
}

// accept: u = ut
__device__ __forceinline__ void ls_finish_body(int64_t n, const double *sc, const float *ut, float *u, int64_t bid) {
  if (sc[SC_ACCEPT] == 0.0) return;
  const int64_t i = bid * 256 + threadIdx.x;
  if (i < n) u[i] = ut[i];
}
__global__ __launch_bounds__(256) void k_ls_finish(int64_t n, const double *sc, const float *ut, float *u) {
  ls_finish_body(n, sc, ut, u, blockIdx.x);
}

// copy of a node field (the linearisation point)
__device__ __forceinline__ void copy_body(int64_t n, const float *src, float *dst, int64_t bid) {
  const int64_t i = bid * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__device__ __forceinline__ void report_body(const double *sc, double CH, double *rep, int *status, int *status_out) {
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
    rep[16] = sc[SC_B];
    rep[17] = sc[SC_TB];
  }
  if (sc[SC_ACCEPT] == 0.0) *status |= 4;
  if (status_out) *status_out = *status;
}
__global__ void k_report(const double *sc, double CH, double *rep, int *status, int *status_out) {
  report_body(sc, CH, rep, status, status_out);
}

__global__ void k_clear_status(int *status) { *status = 0; }

// the terms of the last linearisation: J, D, S, V (+inf on a fold), K, B, folds, |grad J|
__global__ void k_terms(const double *sc, double CH, double *out) {
  out[0] = sc[SC_J];
  out[1] = sc[SC_D];
  out[2] = 0.5 * CH * sc[SC_SRAW];
  out[3] = sc[SC_NFOLD] > 0.0 ? INFINITY : sc[SC_V];
  out[4] = sc[SC_K];
  out[5] = sc[SC_B];
  out[6] = sc[SC_NFOLD];
  out[7] = sqrt(sc[SC_GG]);
}

// ---- L-BFGS vector operations (node fields) ----------------------------------------
// out = sa a + c b with c = f0 + fa sc[ka] + fb sc[kb] sc[kc] (a term whose first slot
// index is negative vanishes; b nullable); out may alias a.  With `blocks`, per-block
// <d, out> (stride 2, second value 0).
__global__ __launch_bounds__(256) void k_lb_axpy(int64_t n, float sa, const float *a, const float *b, float *out,
                                                 const double *sc, double f0, int ka, double fa, int kb, int kc,
                                                 double fb, const float *d, double *blocks) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double dot = 0.0;
  if (i < n) {
    double c = f0;
    if (ka >= 0) c += fa * sc[ka];
    if (kb >= 0) c += fb * sc[kb] * sc[kc];
    float v = sa * a[i];
    if (b) v += (float)c * b[i];
    out[i] = v;
    if (blocks) dot = (double)d[i] * (double)v;
  }
  if (blocks) block_pair_sum(dot, 0.0, blocks, blockIdx.x);
}

// completes a stored pair: y = Y + g (Y held -g_old), written back; per-block s.y, s.s,
// y.y (stride 3)
__global__ __launch_bounds__(256) void k_lb_pair(int64_t n, const float *S, float *Y, const float *g,
                                                 double *blocks) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (i < n) {
    const float y = Y[i] + g[i];
    Y[i] = y;
    const double s = S[i];
    v[0] = s * (double)y;
    v[1] = s * s;
    v[2] = (double)y * (double)y;
  }
  block_write<3>(v, blocks + 3 * (int64_t)blockIdx.x);
}

// starts a pair at the end of a step: S = ut - u if the line search accepted ut, else 0;
// Y = -g (the next linearisation adds its gradient)
__global__ __launch_bounds__(256) void k_lb_save(int64_t n, const double *sc, const float *u, const float *ut,
                                                 const float *g, float *S, float *Y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const bool acc = sc[SC_ACCEPT] != 0.0;
  S[i] = acc ? ut[i] - u[i] : 0.0f;
  Y[i] = -g[i];
}

}  // namespace disco
