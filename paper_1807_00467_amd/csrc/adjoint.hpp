// Derivative of the NGF distance (eq. 1) with respect to the moving image T, for the
// differentiable loss.  D depends on T through a_v = G(y_v), the trilinear sample of
// grad T at the warped voxel centre, and grad T is the central-difference stencil of T:
//   dD/d(grad T)[p] = sum_v w_{v,p} (-2 h^3 r_v dr/da_v),   dD/dT = stencil^T(dD/d grad T).
// The first step scatters to warped positions, so it uses float atomics: the result is
// exact up to FP32 rounding, but its summation order (hence its last bits) is not fixed.
// W (the derivative with respect to grad T) is held component-planar, [3][Nz][Ny][Nx].
#pragma once
#include <climits>
#include "kernels.hpp"

namespace disco {

__global__ __launch_bounds__(256) void k_fill(int64_t n, float *p, float v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// The scatter works on tiles of 16 x 4 x 8 voxels (a workgroup of 256 threads; a thread
// takes one voxel column (x, y) through half a cell layer, 2 voxels along z).  A first pass
// finds the box of sample corners the tile's voxels reach.  When it holds at most
// kAdjBoxPts points, the tile adds its contributions into that box in LDS and then adds
// each touched point to W with one atomic (a smooth warp touches about 1.5 points per
// voxel instead of 8 corners).  Otherwise (a displacement that varies by several voxels
// across the tile) each voxel adds its corners to W directly.
//
// The LDS box holds 64-bit fixed point (integer LDS atomics run at the full LDS rate,
// float ones far slower).  Every contribution is bounded: with r = P / sqrt(Da Db) in
// [-1, 1], |b - (P / Da) a| <= 2 sqrt(Db) and Da >= eta^2, each component of the voxel
// factor w obeys |w_c| <= 2 h3x2 / eta, and a corner weight is at most 1.  A point takes at
// most one contribution per voxel of the tile, so with the scale
// qs = 2^62 / (1.01 * 512 * 2 h3x2 / eta) no partial sum reaches 2^63; the conversions
// truncate at 1 / qs, about 1e-16 of the bound.
constexpr int kAdjTX = 16, kAdjTY = 4, kAdjTZ = 8;
constexpr int kAdjBoxPts = 1600;  // points of a tile's corner box held in LDS (3 x 8 bytes each)

// sample cell (lower corner i0, fractions t) of a voxel, as the trilinear sampler takes it
__device__ __forceinline__ void adj_cell(const Geo &g, int i, int j, int k, const float uh[3], int i0[3],
                                         float t[3]) {
  const int idx[3] = {i, j, k};
  const int n[3] = {g.nx, g.ny, g.nz};
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const float d = fminf(fmaxf(uh[ax], (float)(-2 - idx[ax])), (float)(n[ax] + 1 - idx[ax]));
    const float fl = floorf(d);
    t[ax] = d - fl;
    i0[ax] = idx[ax] + (int)fl;
  }
}

// corners of one voxel added to W with global atomics.  W is component-planar ([3][nvox]),
// so the lanes of a wave add to consecutive addresses.  The neighbouring voxels of a row
// sample neighbouring cells wherever the displacement varies slowly, so the +x corner of
// lane l is usually the -x corner of lane l + 1: lane l + 1 then adds both contributions
// with one atomic (found with wave shuffles), which halves the atomics.  Every lane of the
// wave takes part (inactive ones with act = false).
__device__ __forceinline__ void adj_scatter_global(const Geo &g, float *W, int lane, bool act, const int i0[3],
                                                   const float t[3], const float w[3]) {
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

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

template <class ST>
__global__ __launch_bounds__(256) void k_adjT_scatter(Geo g, const typename ST::elem *gR, const typename ST::elem *gT,
                                                      float sR, float sT, const float *u, float eta2, float h3x2,
                                                      float qs, float iqs, float *W) {
  __shared__ unsigned long long box[3 * kAdjBoxPts];
  __shared__ int wlo[4][3], whi[4][3];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = blockIdx.x * kAdjTX + (tid & 15), j = blockIdx.y * kAdjTY + ((tid >> 4) & 3);
  const int kb = blockIdx.z * kAdjTZ + 2 * wave;  // first of the thread's two voxels along z
  // threads past the volume take part in the shuffles and barriers with no contribution
  const bool col = i < g.nx && j < g.ny;
  const int ic = min(i, g.nx - 1), jc = min(j, g.ny - 1);
  const int nk = max(0, min(2, g.nz - kb));
  // displacement along the column: node values interpolated along x for the two node
  // planes of the cell layer (kb and kb + 1 share it), then along z and y per voxel (one
  // fused multiply-add each, as in the brick kernel, so that the sample cell is identical)
  const int cx = ic >> 2, cy = jc >> 2, cz = min(kb >> 2, g.cz - 1);
  const float wx = ((ic & 3) + 0.5f) * 0.25f, wy = ((jc & 3) + 0.5f) * 0.25f;
  const int64_t pxy = (int64_t)g.px * g.py;
  float fx[2][2][3];  // [node plane cz + pl][jy][c]
#pragma unroll
  for (int pl = 0; pl < 2; ++pl)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int jy = 0; jy < 2; ++jy) {
        const float *f = u + c * g.nnodes + (cz + pl) * pxy + (int64_t)(cy + jy) * g.px + cx;
        fx[pl][jy][c] = __builtin_fmaf(wx, f[1] - f[0], f[0]);
      }
  auto disp = [&](int k, float uh[3]) {
    const float wz = ((k & 3) + 0.5f) * 0.25f;
    const float ih[3] = {g.ihx, g.ihy, g.ihz};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float fz0 = __builtin_fmaf(wz, fx[1][0][c] - fx[0][0][c], fx[0][0][c]);
      const float fz1 = __builtin_fmaf(wz, fx[1][1][c] - fx[0][1][c], fx[0][1][c]);
      uh[c] = __builtin_fmaf(wy, fz1 - fz0, fz0) * ih[c];
    }
  };

  // pass 1: the box of sample corners of the tile's voxels
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    if (col && kk < nk) {
      const int k = kb + kk;
      float uh[3], t[3];
      int i0[3];
      disp(k, uh);
      adj_cell(g, ic, jc, k, uh, i0, t);
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        lo[ax] = min(lo[ax], i0[ax]);
        hi[ax] = max(hi[ax], i0[ax] + 1);
      }
    }
  }
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    lo[ax] = wave_min_i(lo[ax]);
    hi[ax] = wave_max_i(hi[ax]);
  }
  if (lane == 0) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      wlo[wave][ax] = lo[ax];
      whi[wave][ax] = hi[ax];
    }
  }
  __syncthreads();
  // the box, cut to the volume (corners outside it add nothing); the tile's first voxel
  // is inside the volume, so it has at least one active voxel
  const int n[3] = {g.nx, g.ny, g.nz};
  int o[3], dim[3];
  bool empty = false;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int l = min(min(wlo[0][ax], wlo[1][ax]), min(wlo[2][ax], wlo[3][ax]));
    const int h = max(max(whi[0][ax], whi[1][ax]), max(whi[2][ax], whi[3][ax]));
    o[ax] = max(l, 0);
    dim[ax] = min(h, n[ax] - 1) - o[ax] + 1;
    empty = empty || dim[ax] <= 0;
  }
  // (qs = 0 when eta = 0, which bounds nothing: then the direct form)
  const bool in_lds = !empty && qs > 0.0f && (int64_t)dim[0] * dim[1] * dim[2] <= kAdjBoxPts;
  const int npts = in_lds ? dim[0] * dim[1] * dim[2] : 0;
  if (in_lds)
    for (int p = threadIdx.x; p < 3 * npts; p += 256) box[p] = 0ull;
  __syncthreads();

  // pass 2: dD/d(grad T) of each voxel, added to its sample corners
#pragma unroll 1
  for (int kk = 0; kk < 2; ++kk) {
    const bool act = col && kk < nk;
    const int k = min(kb + kk, g.nz - 1);
    float uh[3];
    disp(k, uh);
    const int64_t v = ((int64_t)k * g.ny + jc) * g.nx + ic;
    float a[3], JG[3][3], b[3];
    sample_grad<ST, false>(gT, sT, g, ic, jc, k, uh, a, JG);
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
    int i0[3];
    float t[3];
    adj_cell(g, ic, jc, k, uh, i0, t);
    if (in_lds) {
      if (act) {
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
          for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
              const int xi = i0[0] + dx, yi = i0[1] + dy, zi = i0[2] + dz;
              if ((unsigned)xi < (unsigned)g.nx && (unsigned)yi < (unsigned)g.ny && (unsigned)zi < (unsigned)g.nz) {
                const float wc = (dx ? t[0] : 1.0f - t[0]) * (dy ? t[1] : 1.0f - t[1]) * (dz ? t[2] : 1.0f - t[2]);
                const int q = ((zi - o[2]) * dim[1] + (yi - o[1])) * dim[0] + (xi - o[0]);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                  atomicAdd(&box[c * npts + q], (unsigned long long)(long long)(wc * w[c] * qs));
              }
            }
      }
    } else {
      adj_scatter_global(g, W, lane, act, i0, t, w);
    }
  }

  // the box's touched points to W, one atomic per point and component (consecutive
  // threads take consecutive x)
  if (in_lds) {
    __syncthreads();
    const float inv0 = 1.0f / (float)dim[0], inv1 = 1.0f / (float)dim[1];
    for (int p = threadIdx.x; p < npts; p += 256) {
      // p = (z dim1 + y) dim0 + x; the float quotients are exact for p < 2^20
      const int r = (int)(((float)p + 0.5f) * inv0);
      const int x = p - r * dim[0];
      const int z = (int)(((float)r + 0.5f) * inv1);
      const int y = r - z * dim[1];
      const int64_t key = ((int64_t)(o[2] + z) * g.ny + (o[1] + y)) * g.nx + (o[0] + x);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long acc = (long long)box[c * npts + p];
        if (acc != 0) atomicAdd(W + c * g.nvox + key, (float)acc * iqs);
      }
    }
  }
}

// dT = transpose of (grad I)_a[i] = (I[clamp(i+e_a)] - I[clamp(i-e_a)]) / (2 h_a) applied to W,
// times *scale when given
__global__ __launch_bounds__(256) void k_adjT_stencil(Geo g, const float *W, const double *scale, float *dT) {
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
  dT[v] = scale ? (float)((double)acc * *scale) : acc;
}

}  // namespace disco
