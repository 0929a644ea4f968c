// Derivative of the NGF distance (eq. 1) with respect to the moving image T, for the
// differentiable loss.  D depends on T through a_v = G(y_v), the trilinear sample of
// grad T at the warped voxel centre, and grad T is the central-difference stencil of T:
//   dD/d(grad T)[p] = sum_v w_{v,p} (-2 h^3 r_v dr/da_v),   dD/dT = stencil^T(dD/d grad T).
// The first step scatters to warped positions, so it uses float atomics: the result is
// exact up to FP32 rounding, but its summation order (hence its last bits) is not fixed.
// W (the derivative with respect to grad T) is held component-planar, [3][Nz][Ny][Nx].
#pragma once
#include "kernels.hpp"

namespace disco {

__global__ __launch_bounds__(256) void k_fill(int64_t n, float *p, float v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// One thread per voxel (rows of 256 along x).  W is component-planar ([3][nvox]), so the
// lanes of a wave add to consecutive addresses.  The neighbouring voxels of a row sample
// neighbouring cells wherever the displacement varies slowly, so the +x corner of lane l
// is usually the -x corner of lane l + 1: lane l + 1 then adds both contributions with
// one atomic (found with wave shuffles), which halves the atomics of the pass.
template <class ST>
__global__ __launch_bounds__(256) void k_adjT_scatter(Geo g, const typename ST::elem *gR, const typename ST::elem *gT,
                                                      float sR, float sT, const float *u, float eta2, float h3x2,
                                                      float *W) {
  const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  const int lane = threadIdx.x & 63;
  // lanes past the row end take part in the shuffles with no contribution
  const bool act = i < g.nx;
  const int ic = act ? i : g.nx - 1;
  const int64_t v = ((int64_t)k * g.ny + j) * g.nx + ic;
  // displacement at the voxel: node values interpolated along x, then z, then y (one
  // fused multiply-add each), as in the brick kernel, so the sample cell is identical
  const int cx = ic >> 2, cy = j >> 2, cz = k >> 2;
  const float wx = ((ic & 3) + 0.5f) * 0.25f, wy = ((j & 3) + 0.5f) * 0.25f, wz = ((k & 3) + 0.5f) * 0.25f;
  const int64_t pxy = (int64_t)g.px * g.py;
  const int64_t n0 = (int64_t)cz * pxy + (int64_t)cy * g.px + cx;
  float f3[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float *f = u + c * g.nnodes + n0;
    float fx[2][2];
#pragma unroll
    for (int kz = 0; kz < 2; ++kz)
#pragma unroll
      for (int jy = 0; jy < 2; ++jy) {
        const float a0 = f[kz * pxy + jy * g.px], a1 = f[kz * pxy + jy * g.px + 1];
        fx[kz][jy] = __builtin_fmaf(wx, a1 - a0, a0);
      }
    float fz[2];
#pragma unroll
    for (int jy = 0; jy < 2; ++jy) fz[jy] = __builtin_fmaf(wz, fx[1][jy] - fx[0][jy], fx[0][jy]);
    f3[c] = __builtin_fmaf(wy, fz[1] - fz[0], fz[0]);
  }
  const float uh[3] = {f3[0] * g.ihx, f3[1] * g.ihy, f3[2] * g.ihz};
  float a[3], JG[3][3], b[3];
  sample_grad<ST, false>(gT, sT, g, ic, j, k, uh, a, JG);
  ST::loadp(gR + v * ST::W, sR, b);
  const float Da = eta2 + a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
  const float Db = eta2 + b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
  const float P = eta2 + a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
  const float isq = rsqrtf(Da * Db);
  const float r = P * isq;
  const float pda = P * frcp(Da);
  float w[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) w[c] = act ? -h3x2 * r * (b[c] - pda * a[c]) * isq : 0.0f;
  // the same corners and weights as the sample (zero outside the volume)
  const int idx[3] = {ic, j, k};
  const int n[3] = {g.nx, g.ny, g.nz};
  int i0[3];
  float t[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const float d = fminf(fmaxf(uh[ax], (float)(-2 - idx[ax])), (float)(n[ax] + 1 - idx[ax]));
    const float fl = floorf(d);
    t[ax] = d - fl;
    i0[ax] = idx[ax] + (int)fl;
  }
  const int64_t nv = g.nvox;
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
      const int yi = i0[1] + dy, zi = i0[2] + dz;
      const bool row = act && (unsigned)yi < (unsigned)g.ny && (unsigned)zi < (unsigned)g.nz;
      const bool ok0 = row && (unsigned)i0[0] < (unsigned)g.nx;
      const bool ok1 = row && (unsigned)(i0[0] + 1) < (unsigned)g.nx;
      // linear index of the -x corner (voxel counts stay below 2^31)
      const int key0 = row ? (int)(((int64_t)zi * g.ny + yi) * g.nx + i0[0]) : -2;
      const float wyz = (dy ? t[1] : 1.0f - t[1]) * (dz ? t[2] : 1.0f - t[2]);
      const float w0 = (1.0f - t[0]) * wyz, w1 = t[0] * wyz;
      // the left lane's +x corner is this lane's -x corner: add it here
      const int keyL = __shfl_up(key0, 1, 64);
      const int okL = __shfl_up((int)ok1, 1, 64);
      const bool take = lane > 0 && okL && ok0 && keyL + 1 == key0;
      // the right lane takes this lane's +x corner by the same test
      const int keyR = __shfl_down(key0, 1, 64);
      const int okR = __shfl_down((int)ok0, 1, 64);
      const bool given = lane < 63 && okR && ok1 && key0 + 1 == keyR;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float c1 = w1 * w[c];
        const float fromL = __shfl_up(c1, 1, 64);
        if (ok0) atomicAdd(W + c * nv + key0, w0 * w[c] + (take ? fromL : 0.0f));
        if (ok1 && !given) atomicAdd(W + c * nv + key0 + 1, c1);
      }
    }
}

// dT = transpose of (grad I)_a[i] = (I[clamp(i+e_a)] - I[clamp(i-e_a)]) / (2 h_a) applied to W
__global__ __launch_bounds__(256) void k_adjT_stencil(Geo g, const float *W, float *dT) {
  const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i >= g.nx) return;
  const int64_t v = ((int64_t)k * g.ny + j) * g.nx + i;
  const int idx[3] = {i, j, k};
  const int n[3] = {g.nx, g.ny, g.nz};
  const int64_t st[3] = {1, g.nx, (int64_t)g.nx * g.ny};
  const float ih2[3] = {0.5f * g.ihx, 0.5f * g.ihy, 0.5f * g.ihz};
  float acc = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float s = 0.0f;
    const float *Wa = W + a * g.nvox;
    if (idx[a] > 0) s += Wa[v - st[a]];          // voxel i - e_a reads I[i] as its "+" neighbour
    if (idx[a] == n[a] - 1) s += Wa[v];          // replicated border: i's "+" neighbour is i itself
    if (idx[a] < n[a] - 1) s -= Wa[v + st[a]];   // voxel i + e_a reads I[i] as its "-" neighbour
    if (idx[a] == 0) s -= Wa[v];                 // replicated border: i's "-" neighbour is i itself
    acc += s * ih2[a];
  }
  dT[v] = acc;
}

}  // namespace disco
