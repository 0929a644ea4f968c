// Multilevel scheme (Sec. II-D3): image pyramid levels by Gaussian smoothing and
// downsampling, and prolongation of the displacement from a coarse control grid to the
// next finer one.  These run once per level, not inside the optimiser: plain coalesced
// streaming kernels, one thread per output element.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace disco {

// combined taps of one downsampling pass along an axis: Gaussian smoothing (7 taps)
// followed by the mean of the two finer voxels a coarse voxel covers, i.e.
// out(i) = sum_{m=-3..4} c[m + 3] in(clamp(2 i + m))
struct DownTaps {
  float c[8];
};

// halves axis AX (0 = x, 1 = y, 2 = z) of a volume [nz][ny][nx]; the output has the
// same layout with that axis halved.  Border voxels are replicated.
template <int AX>
__global__ __launch_bounds__(256) void k_down_axis(const float *__restrict__ src, int nx, int ny, int nz,
                                                   float *__restrict__ dst, DownTaps t) {
  const int ox = AX == 0 ? nx / 2 : nx, oy = AX == 1 ? ny / 2 : ny;
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= ox) return;
  const int n = AX == 0 ? nx : (AX == 1 ? ny : nz);
  const int i = AX == 0 ? x : (AX == 1 ? y : z);
  const int64_t stride = AX == 0 ? 1 : (AX == 1 ? (int64_t)nx : (int64_t)nx * ny);
  // the voxel at index 0 along AX, the other coordinates fixed
  const int64_t base = AX == 0 ? ((int64_t)z * ny + y) * nx
                               : (AX == 1 ? (int64_t)z * nx * ny + x : (int64_t)y * nx + x);
  float v[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int j = min(max(2 * i + m - 3, 0), n - 1);
    v[m] = src[base + j * stride];
  }
  float acc = 0.0f;
#pragma unroll
  for (int m = 0; m < 8; ++m) acc += t.c[m] * v[m];
  dst[((int64_t)z * oy + y) * ox + x] = acc;
}

// fine node field [3][fz][fy][fx] from the coarse one [3][cz][cy][cx]: along a halved
// axis fine node q lies at coarse coordinate q / 2 (even q: a coarse node; odd q: the
// midpoint of two); other axes map one to one
__global__ __launch_bounds__(256) void k_prolong(const float *__restrict__ uc, int cx, int cy, int cz, int hx, int hy,
                                                 int hz, float *__restrict__ uf, int fx, int fy, int fz) {
  const int qx = blockIdx.x * 256 + threadIdx.x, qy = blockIdx.y, qz = blockIdx.z;
  if (qx >= fx) return;
  const int q[3] = {qx, qy, qz};
  const int hv[3] = {hx, hy, hz};
  int lo[3], hi[3];
  float w1[3];  // weight of the upper coarse node
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (hv[a]) {
      lo[a] = q[a] >> 1;
      hi[a] = (q[a] + 1) >> 1;
      w1[a] = (q[a] & 1) ? 0.5f : 0.0f;
    } else {
      lo[a] = hi[a] = q[a];
      w1[a] = 0.0f;
    }
  }
  const int64_t cn = (int64_t)cx * cy * cz, fn = (int64_t)fx * fy * fz;
  const int64_t fi = ((int64_t)qz * fy + qy) * fx + qx;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float *u = uc + c * cn;
    auto at = [&](int x, int y, int z) { return u[((int64_t)z * cy + y) * cx + x]; };
    // x, then y, then z
    const float a00 = at(lo[0], lo[1], lo[2]) + w1[0] * (at(hi[0], lo[1], lo[2]) - at(lo[0], lo[1], lo[2]));
    const float a10 = at(lo[0], hi[1], lo[2]) + w1[0] * (at(hi[0], hi[1], lo[2]) - at(lo[0], hi[1], lo[2]));
    const float a01 = at(lo[0], lo[1], hi[2]) + w1[0] * (at(hi[0], lo[1], hi[2]) - at(lo[0], lo[1], hi[2]));
    const float a11 = at(lo[0], hi[1], hi[2]) + w1[0] * (at(hi[0], hi[1], hi[2]) - at(lo[0], hi[1], hi[2]));
    const float b0 = a00 + w1[1] * (a10 - a00);
    const float b1 = a01 + w1[1] * (a11 - a01);
    uf[c * fn + fi] = b0 + w1[2] * (b1 - b0);
  }
}

}  // namespace disco
