// Device code of the dense registration objective (gfx950, wave64).
//
// Layout (see include/disco.h): volumes [Nz][Ny][Nx], per-voxel 3-vectors [N][3],
// node fields [3][nz][ny][nx], 4 voxels per control-grid cell and axis.
//
// The voxel-brick kernel `k_brick` is the hot path.  A workgroup of 4 waves owns a
// brick of 16 x 4 x ZC cells: lane l of wave w handles voxel column x = 64*bx + l of cell
// row y = 4*by + w and walks the ZC cell layers of the brick along z.  The transpose onto
// the nodes (P^T) is done without atomics:
//   * along z by rolling register accumulators (a node plane is finished after the two
//     cell layers that touch it);
//   * along x by quad-wide DPP sums (the 4 lanes of a quad are the 4 voxels of one cell);
//   * along y by a fixed-order LDS combine of the 4 waves;
//   * across bricks by writing the shared face nodes to a partial buffer that the
//     node-parallel `k_gather` sums in a fixed order.
// Every floating-point sum therefore has a fixed order: results are bitwise
// reproducible run to run.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace disco {

constexpr int kWG = 256;   // threads of a brick workgroup (4 waves)
constexpr int kBXC = 16;   // cells per brick along x (64 voxels = one wave)
constexpr int kBYC = 4;    // cells per brick along y (one wave per cell row)
constexpr int kNBOX = (kBXC + 1) * (kBYC + 1);  // nodes of one brick plane (17 x 5)

enum { M_EVAL = 0, M_GRAD = 1, M_HV = 2 };

// block scalar slots written by k_brick (doubles per workgroup)
enum { BS_D = 0, BS_V = 1, BS_K = 2, BS_FOLD = 3, BS_N = 4 };

struct Geo {
  int nx, ny, nz;        // voxels
  int cx, cy, cz;        // cells
  int px, py, pz;        // nodes per axis
  int nbx, nby, nbz, zc; // bricks and cells per brick along z
  float hx, hy, hz;      // voxel spacing (mm)
  float ihx, ihy, ihz;   // 1/h
  float Hx, Hy, Hz;      // cell size (mm)
  float iHx, iHy, iHz;   // 1/H
  float C;               // cell volume H_x H_y H_z
  int64_t nvox, nnodes;
};

// Storage of the per-voxel 3-vectors (image gradients, GN vectors s).
struct F32x3 {
  typedef float elem;
  __device__ static inline void load(const float *p, int64_t i, float s, float o[3]) {
    const float *q = p + 3 * i;
    o[0] = q[0];
    o[1] = q[1];
    o[2] = q[2];
    (void)s;
  }
  __device__ static inline void store(float *p, int64_t i, float s, const float v[3]) {
    float *q = p + 3 * i;
    q[0] = v[0];
    q[1] = v[1];
    q[2] = v[2];
    (void)s;
  }
};

// half precision, 4 halfs (8 B) per voxel, value = stored * s (s: per-volume power of two)
struct F16x4 {
  typedef __half elem;
  __device__ static inline void load(const __half *p, int64_t i, float s, float o[3]) {
    const uint2 w = *reinterpret_cast<const uint2 *>(p + 4 * i);
    __half2 a = *reinterpret_cast<const __half2 *>(&w.x);
    __half2 b = *reinterpret_cast<const __half2 *>(&w.y);
    float2 fa = __half22float2(a);
    float2 fb = __half22float2(b);
    o[0] = fa.x * s;
    o[1] = fa.y * s;
    o[2] = fb.x * s;
  }
  __device__ static inline void store(__half *p, int64_t i, float s, const float v[3]) {
    __half2 a = __floats2half2_rn(v[0] * s, v[1] * s);
    __half2 b = __floats2half2_rn(v[2] * s, 0.0f);
    uint2 w;
    w.x = *reinterpret_cast<const uint32_t *>(&a);
    w.y = *reinterpret_cast<const uint32_t *>(&b);
    *reinterpret_cast<uint2 *>(p + 4 * i) = w;
  }
};

template <class ST>
struct BrickArgs {
  Geo g;
  const typename ST::elem *gR;  // grad R  (M_EVAL / M_GRAD)
  const typename ST::elem *gT;  // grad T  (M_EVAL / M_GRAD)
  typename ST::elem *sc;        // s cache (written in M_GRAD, read in M_HV)
  float sR, sT;                 // dequantisation scales of gR, gT
  float sS_load, sS_store;      // s cache: value = stored * sS_load; stored = value * sS_store
  const float *u;               // displacement (M_EVAL/M_GRAD) or linearisation point (M_HV)
  const float *v;               // direction (M_HV)
  const float *kloc;            // keypoints relative to their cell origin [n][3]
  const float *ktgt;            // targets relative to the same origin [n][3]
  const int *kstart;            // CSR over cells [ncells + 1]
  float eta2;                   // eta^2
  float ngf_scale;              // 2 h_x h_y h_z
  float gamma, delta;           // weights of the cell terms folded into the node outputs
  float *out0, *out1;           // node fields: field 0 (g or Hv), field 1 (GN diagonal)
  float *part;                  // face partials
  double *blocks;               // BS_N doubles per workgroup
  const double *stop;           // if non-null and *stop != 0 the launch does nothing
};

// ---------------------------------------------------------------------------------
// quad (4-lane) sums with DPP quad permutations: xor 1 = [1,0,3,2], xor 2 = [2,3,0,1]
// ---------------------------------------------------------------------------------
__device__ __forceinline__ float dpp_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_xor2(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
}
__device__ __forceinline__ float quad_sum(float v) {
  v = v + dpp_xor1(v);
  return v + dpp_xor2(v);
}

__device__ __forceinline__ bool is_face(int l, int b, int nb, int B) {
  return (l == 0 && b > 0) || (l == B && b + 1 < nb);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// node plane pz of the 2 x 2 corner nodes (cx..cx+1, cy..cy+1) of a cell, [j][i][c]
__device__ __forceinline__ void load_plane(const float *f, const Geo &g, int cx, int cy, int pz, bool ok,
                                           float o[2][2][3]) {
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int64_t n = ((int64_t)pz * g.py + cy + j) * g.px + cx + i;
#pragma unroll
      for (int c = 0; c < 3; ++c) o[j][i][c] = ok ? f[c * g.nnodes + n] : 0.0f;
    }
}

// ---------------------------------------------------------------------------------
// trilinear sample of a 3-vector volume at continuous index q (zero padding): value G
// and Jacobian JG[c][a] = dG_c / dy_a.  q is split as (integer voxel index) + (u/h)
// so that the fraction keeps full precision.
// ---------------------------------------------------------------------------------
template <class ST>
__device__ __forceinline__ void sample_grad(const typename ST::elem *gT, float sT, const Geo &g, int ix, int iy,
                                            int iz, const float uh[3], float G[3], float JG[3][3]) {
  const int idx[3] = {ix, iy, iz};
  const int n[3] = {g.nx, g.ny, g.nz};
  int i0[3];
  float t[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // outside [-2, N+1] every corner is outside the volume: clamp (also avoids overflow)
    float d = fminf(fmaxf(uh[a], (float)(-2 - idx[a])), (float)(n[a] + 1 - idx[a]));
    float f = floorf(d);
    t[a] = d - f;
    i0[a] = idx[a] + (int)f;
  }
  const bool vx0 = (unsigned)i0[0] < (unsigned)g.nx, vx1 = (unsigned)(i0[0] + 1) < (unsigned)g.nx;
  const bool vy0 = (unsigned)i0[1] < (unsigned)g.ny, vy1 = (unsigned)(i0[1] + 1) < (unsigned)g.ny;
  const bool vz0 = (unsigned)i0[2] < (unsigned)g.nz, vz1 = (unsigned)(i0[2] + 1) < (unsigned)g.nz;
  float cv[2][2][2][3];  // [z][y][x][c]
#pragma unroll
  for (int cz = 0; cz < 2; ++cz)
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) {
        const bool ok = (cz ? vz1 : vz0) && (cy ? vy1 : vy0) && (cx ? vx1 : vx0);
        if (ok) {
          const int64_t vi = ((int64_t)(i0[2] + cz) * g.ny + (i0[1] + cy)) * g.nx + (i0[0] + cx);
          ST::load(gT, vi, sT, cv[cz][cy][cx]);
        } else {
          cv[cz][cy][cx][0] = cv[cz][cy][cx][1] = cv[cz][cy][cx][2] = 0.0f;
        }
      }
  // x, then y, then z; derivatives from differences of the lower-order interpolants
  float gx[2][2][3], dx[2][2][3];
#pragma unroll
  for (int cz = 0; cz < 2; ++cz)
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        gx[cz][cy][c] = cv[cz][cy][0][c] + t[0] * (cv[cz][cy][1][c] - cv[cz][cy][0][c]);
        dx[cz][cy][c] = cv[cz][cy][1][c] - cv[cz][cy][0][c];
      }
  float gxy[2][3], dxy[2][3], dyy[2][3];
#pragma unroll
  for (int cz = 0; cz < 2; ++cz)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      gxy[cz][c] = gx[cz][0][c] + t[1] * (gx[cz][1][c] - gx[cz][0][c]);
      dxy[cz][c] = dx[cz][0][c] + t[1] * (dx[cz][1][c] - dx[cz][0][c]);
      dyy[cz][c] = gx[cz][1][c] - gx[cz][0][c];
    }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    G[c] = gxy[0][c] + t[2] * (gxy[1][c] - gxy[0][c]);
    JG[c][0] = (dxy[0][c] + t[2] * (dxy[1][c] - dxy[0][c])) * g.ihx;
    JG[c][1] = (dyy[0][c] + t[2] * (dyy[1][c] - dyy[0][c])) * g.ihy;
    JG[c][2] = (gxy[1][c] - gxy[0][c]) * g.ihz;
  }
}

// ---------------------------------------------------------------------------------
// Per-cell terms: volume change control (eq. 7-9) and keypoints (eq. 10).
// Lane q of a quad handles the 16 coefficients d_abc with c = q (e3 edge (i,j) =
// (q & 1, q >> 1)) and the keypoints q, q+4, ... of the cell.  Results are corner
// contributions cc[f][k][j][i][comp] of this lane (summed over the quad by the caller).
// ---------------------------------------------------------------------------------
struct CellCorners {
  float u[2][2][2][3];  // [k][j][i][c] displacement at the 8 corners
  float v[2][2][2][3];  // direction (M_HV)
};

__device__ __forceinline__ void cross3(const float a[3], const float b[3], float o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ float dot3(const float a[3], const float b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

template <int MODE>
__device__ __forceinline__ void vcc_cell(const Geo &g, int q, const CellCorners &cc, float w,
                                         float out[2][2][2][2][3], double &sV, int &nfold) {
  // edge vectors of y = X + u: e1_(j,k) = y_1jk - y_0jk = H_x e_x + u_1jk - u_0jk, etc.
  float e1[4][3], e2[4][3], e3[3];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int c = 0; c < 3; ++c) e1[j + 2 * k][c] = cc.u[k][j][1][c] - cc.u[k][j][0][c] + (c == 0 ? g.Hx : 0.0f);
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) e2[i + 2 * k][c] = cc.u[k][1][i][c] - cc.u[k][0][i][c] + (c == 1 ? g.Hy : 0.0f);
  const int qi = q & 1, qj = q >> 1;
  // this lane's e3 edge, selected without dynamic register indexing
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float e[4];
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int ii = 0; ii < 2; ++ii) e[ii + 2 * jj] = cc.u[1][jj][ii][c] - cc.u[0][jj][ii][c];
    e3[c] = (q == 0 ? e[0] : q == 1 ? e[1] : q == 2 ? e[2] : e[3]) + (c == 2 ? g.Hz : 0.0f);
  }

  float de1[4][3], de2[4][3], de3[3];
  if (MODE == M_HV) {
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) de1[j + 2 * k][c] = cc.v[k][j][1][c] - cc.v[k][j][0][c];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) de2[i + 2 * k][c] = cc.v[k][1][i][c] - cc.v[k][0][i][c];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float e[4];
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) e[ii + 2 * jj] = cc.v[1][jj][ii][c] - cc.v[0][jj][ii][c];
      de3[c] = q == 0 ? e[0] : q == 1 ? e[1] : q == 2 ? e[2] : e[3];
    }
  }

  const float iC = 1.0f / g.C;
  float x23[4][3], x31[4][3];
#pragma unroll
  for (int b = 0; b < 4; ++b) cross3(e2[b], e3, x23[b]);
#pragma unroll
  for (int a = 0; a < 4; ++a) cross3(e3, e1[a], x31[a]);

  float G1[4][3] = {}, G2[4][3] = {}, G3[3] = {};
  // GN diagonal contributions go straight to the corners
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      float x12[3];
      cross3(e1[a], e2[b], x12);
      const float d = dot3(e1[a], x23[b]) * iC;
      if (!(d > 0.0f)) {
        if (MODE != M_HV) ++nfold;
        continue;
      }
      const float id = 1.0f / d;
      if (MODE == M_EVAL || MODE == M_GRAD) sV += (double)(d - 2.0f + id);
      if (MODE == M_GRAD) {
        const float p1 = 1.0f - id * id;  // psi'
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          G1[a][c] += p1 * x23[b][c];
          G2[b][c] += p1 * x31[a][c];
          G3[c] += p1 * x12[c];
        }
        // diag: C psi'' (dd/dy_n)^2 with dd/dy_n the signed sum of the cross products of
        // the edges of this term that contain corner n, divided by C
        const float p2 = 2.0f * id * id * id * w * iC;  // psi''/C, times the weight
        const int ja = a & 1, ka = a >> 1, ib = b & 1, kb = b >> 1;
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
              const bool in1 = (j == ja) && (k == ka);
              const bool in2 = (i == ib) && (k == kb);
              const bool in3 = (i == qi) && (j == qj);
              if (!(in1 || in2 || in3)) continue;
              const float s1 = in1 ? (i ? 1.0f : -1.0f) : 0.0f;
              const float s2 = in2 ? (j ? 1.0f : -1.0f) : 0.0f;
              const float s3 = in3 ? (k ? 1.0f : -1.0f) : 0.0f;
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                const float dd = s1 * x23[b][c] + s2 * x31[a][c] + s3 * x12[c];
                out[1][k][j][i][c] += p2 * dd * dd;
              }
            }
      }
      if (MODE == M_HV) {
        const float jv = (dot3(de1[a], x23[b]) + dot3(de2[b], x31[a]) + dot3(de3, x12)) * iC;
        const float coef = 2.0f * id * id * id * jv;  // psi''(d) (grad d . v)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          G1[a][c] += coef * x23[b][c];
          G2[b][c] += coef * x31[a][c];
          G3[c] += coef * x12[c];
        }
      }
    }
  if (MODE == M_GRAD || MODE == M_HV) {
    // edges -> corners: +G on the far node of the edge, -G on the near node
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            float acc = (i ? G1[j + 2 * k][c] : -G1[j + 2 * k][c]) + (j ? G2[i + 2 * k][c] : -G2[i + 2 * k][c]);
            if (i == qi && j == qj) acc += k ? G3[c] : -G3[c];
            out[0][k][j][i][c] += w * acc;
          }
  }
}

template <int MODE>
__device__ __forceinline__ void kp_cell(const Geo &g, int q, int ks, int ke, const float *kloc, const float *ktgt,
                                        const CellCorners &cc, float w, float out[2][2][2][2][3], double &sK) {
  for (int kk = ks + q; kk < ke; kk += 4) {
    float xl[3], tl[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xl[c] = kloc[3 * kk + c];
      tl[c] = ktgt[3 * kk + c];
    }
    const float t0 = xl[0] * g.iHx, t1 = xl[1] * g.iHy, t2 = xl[2] * g.iHz;
    float wt[2][2][2];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
          wt[k][j][i] = (i ? t0 : 1.0f - t0) * (j ? t1 : 1.0f - t1) * (k ? t2 : 1.0f - t2);
    float val[3];
    if (MODE == M_HV) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float pv = 0.0f;
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 2; ++i) pv += wt[k][j][i] * cc.v[k][j][i][c];
        val[c] = 2.0f * w * pv;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float y = xl[c];
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 2; ++i) y += wt[k][j][i] * cc.u[k][j][i][c];
        const float res = y - tl[c];
        sK += (double)res * (double)res;
        val[c] = 2.0f * w * res;
      }
    }
    if (MODE == M_GRAD || MODE == M_HV) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              out[0][k][j][i][c] += wt[k][j][i] * val[c];
              if (MODE == M_GRAD) out[1][k][j][i][c] += 2.0f * w * wt[k][j][i] * wt[k][j][i];
            }
    }
  }
}

// ---------------------------------------------------------------------------------
// The voxel-brick kernel.
// ---------------------------------------------------------------------------------
template <class ST, int MODE, bool NGF, bool VCC, bool KP, int ZC>
__global__ __launch_bounds__(kWG) void k_brick(BrickArgs<ST> A) {
  constexpr int F = (MODE == M_GRAD) ? 2 : ((MODE == M_HV) ? 1 : 0);
  constexpr int FS = F > 0 ? F : 1;
  constexpr bool CELLT = VCC || KP;
  __shared__ float lds[4][2][FS * 3][2][16];  // [wave][jn][field*3+c][A/B][quad]
  __shared__ double lred[4][BS_N];

  if (A.stop && *A.stop != 0.0) return;
  const Geo &g = A.g;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane & 3, xq = lane >> 2;
  const int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  const int ix = bx * 64 + lane;
  const int cx = ix >> 2;
  const int cy = by * kBYC + wave;
  const int cz0 = bz * ZC;
  const int cz1 = min(cz0 + ZC, g.cz);
  const bool ok = (cx < g.cx) && (cy < g.cy);
  const float xi = (q + 0.5f) * 0.25f;
  const int64_t brick = ((int64_t)bz * g.nby + by) * g.nbx + bx;

  // corner values of this lane's cell, rolled along z: [k][j][i][c]
  CellCorners cc;
  float tmp[2][2][3];
  const float *U = A.u;
  const float *V = A.v;
  const bool need_u = (MODE != M_HV) || VCC;
  const bool need_v = (MODE == M_HV);
  if (need_u) {
    load_plane(U, g, cx, cy, cz0, ok, tmp);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) cc.u[0][j][i][c] = tmp[j][i][c];
  }
  if (need_v) {
    load_plane(V, g, cx, cy, cz0, ok, tmp);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) cc.v[0][j][i][c] = tmp[j][i][c];
  }

  float carN[FS][2][3] = {};          // NGF, per lane before the x reduction: [f][jn][c]
  float carC[FS][2][2][3] = {};       // cell terms, quad-uniform: [f][jn][i][c]
  double sD = 0.0, sV = 0.0, sK = 0.0;
  int nfold = 0;
  const float sc_ngf = A.ngf_scale;

  auto emit = [&](int zl, const float nv[FS][2][3], const float cv[FS][2][2][3]) {
    if constexpr (F > 0) {
#pragma unroll
      for (int f = 0; f < F; ++f) {
        // field 1 (diagonal) uses squared weights
        const float wA = (f == 0) ? (1.0f - xi) : (1.0f - xi) * (1.0f - xi);
        const float wB = (f == 0) ? xi : xi * xi;
        const float s = (MODE == M_GRAD && f == 0) ? -sc_ngf : sc_ngf;
#pragma unroll
        for (int jn = 0; jn < 2; ++jn)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            float a = 0.0f, b = 0.0f;
            if (NGF) {
              a = quad_sum(nv[f][jn][c] * (wA * s));
              b = quad_sum(nv[f][jn][c] * (wB * s));
            }
            if (CELLT) {
              a += cv[f][jn][0][c];
              b += cv[f][jn][1][c];
            }
            if (q == 0) {
              lds[wave][jn][f * 3 + c][0][xq] = a;
              lds[wave][jn][f * 3 + c][1][xq] = b;
            }
          }
      }
      __syncthreads();
      const int pzn = cz0 + zl;
      const bool zface = is_face(zl, bz, g.nbz, ZC);
      for (int e = threadIdx.x; e < F * 3 * kNBOX; e += kWG) {
        const int xl = e % 17, yl = (e / 17) % 5, fc = e / kNBOX;
        float val = 0.0f;
        if (yl < 4) {
          if (xl < 16) val += lds[yl][0][fc][0][xl];
          if (xl > 0) val += lds[yl][0][fc][1][xl - 1];
        }
        if (yl > 0) {
          if (xl < 16) val += lds[yl - 1][1][fc][0][xl];
          if (xl > 0) val += lds[yl - 1][1][fc][1][xl - 1];
        }
        const int pxn = bx * kBXC + xl, pyn = by * kBYC + yl;
        if (pxn > g.cx || pyn > g.cy) continue;
        const bool face = zface || is_face(xl, bx, g.nbx, kBXC) || is_face(yl, by, g.nby, kBYC);
        if (face) {
          A.part[((brick * (ZC + 1) + zl) * (F * 3) + fc) * kNBOX + yl * 17 + xl] = val;
        } else {
          const int f = fc / 3, c = fc - 3 * f;
          float *o = f == 0 ? A.out0 : A.out1;
          o[c * g.nnodes + ((int64_t)pzn * g.py + pyn) * g.px + pxn] = val;
        }
      }
      __syncthreads();
    }
  };

  for (int czi = cz0; czi < cz1; ++czi) {
    // corners of the next node plane
    if (need_u) {
      load_plane(U, g, cx, cy, czi + 1, ok, tmp);
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) cc.u[1][j][i][c] = tmp[j][i][c];
    }
    if (need_v) {
      load_plane(V, g, cx, cy, czi + 1, ok, tmp);
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) cc.v[1][j][i][c] = tmp[j][i][c];
    }

    float accN[FS][2][2][3] = {};  // [f][kn][jn][c]
    if (NGF && ok) {
      // node values interpolated along x at this lane's voxel: fx[k][j][c]
      float fx[2][2][3];
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float a0 = (MODE == M_HV) ? cc.v[k][j][0][c] : cc.u[k][j][0][c];
            const float a1 = (MODE == M_HV) ? cc.v[k][j][1][c] : cc.u[k][j][1][c];
            fx[k][j][c] = a0 + xi * (a1 - a0);
          }
      auto zrow = [&](const int kv) {
        const float wz = (kv + 0.5f) * 0.25f;
        const int iz = czi * 4 + kv;
        float fz[2][3];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int c = 0; c < 3; ++c) fz[j][c] = fx[0][j][c] + wz * (fx[1][j][c] - fx[0][j][c]);
        float accY[FS][2][3] = {};
#pragma unroll
        for (int jv = 0; jv < 4; ++jv) {
          const float wy = (jv + 0.5f) * 0.25f;
          const int iy = cy * 4 + jv;
          const int64_t vox = ((int64_t)iz * g.ny + iy) * g.nx + ix;
          float f3[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) f3[c] = fz[0][c] + wy * (fz[1][c] - fz[0][c]);
          if (MODE == M_HV) {
            float s[3];
            ST::load(A.sc, vox, A.sS_load, s);
            const float w = s[0] * f3[0] + s[1] * f3[1] + s[2] * f3[2];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const float t = w * s[c];
              accY[0][0][c] += (1.0f - wy) * t;
              accY[0][1][c] += wy * t;
            }
          } else {
            // displacement in voxel units: q = index + u/h
            const float uh[3] = {f3[0] * g.ihx, f3[1] * g.ihy, f3[2] * g.ihz};
            float a[3], JG[3][3], b[3];
            sample_grad<ST>(A.gT, A.sT, g, ix, iy, iz, uh, a, JG);
            ST::load(A.gR, vox, A.sR, b);
            const float e2 = A.eta2;
            const float Da = e2 + a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
            const float Db = e2 + b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
            const float P = e2 + a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
            const float dab[3] = {a[0] - b[0], a[1] - b[1], a[2] - b[2]};
            float axb[3];
            cross3(a, b, axb);
            const float DD = Da * Db;
            const float cvox = (e2 * dot3(dab, dab) + dot3(axb, axb)) / DD;
            sD += (double)cvox;
            if (MODE == M_GRAD) {
              const float isq = rsqrtf(DD);
              const float r = P * isq;
              const float pda = P / Da;
              float dr[3], s[3];
#pragma unroll
              for (int c = 0; c < 3; ++c) dr[c] = (b[c] - pda * a[c]) * isq;
#pragma unroll
              for (int c = 0; c < 3; ++c) s[c] = JG[0][c] * dr[0] + JG[1][c] * dr[1] + JG[2][c] * dr[2];
              ST::store(A.sc, vox, A.sS_store, s);
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                const float t = r * s[c];
                accY[0][0][c] += (1.0f - wy) * t;
                accY[0][1][c] += wy * t;
                const float t2 = s[c] * s[c];
                accY[FS - 1][0][c] += (1.0f - wy) * (1.0f - wy) * t2;
                accY[FS - 1][1][c] += wy * wy * t2;
              }
            }
          }
        }
        if (F > 0) {
#pragma unroll
          for (int jn = 0; jn < 2; ++jn)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              accN[0][0][jn][c] += (1.0f - wz) * accY[0][jn][c];
              accN[0][1][jn][c] += wz * accY[0][jn][c];
              if (F == 2) {
                accN[FS - 1][0][jn][c] += (1.0f - wz) * (1.0f - wz) * accY[FS - 1][jn][c];
                accN[FS - 1][1][jn][c] += wz * wz * accY[FS - 1][jn][c];
              }
            }
        }
      };
      if constexpr (MODE == M_HV) {
#pragma unroll
        for (int kv = 0; kv < 4; ++kv) zrow(kv);
      } else {
#pragma unroll 1
        for (int kv = 0; kv < 4; ++kv) zrow(kv);
      }
    }

    // per-cell terms of this layer: corner contributions [f][k][j][i][c]
    float cterm[FS][2][2][2][3] = {};
    if (CELLT) {
      float ct[2][2][2][2][3] = {};
      if (ok) {
        if (VCC) vcc_cell<MODE>(g, q, cc, A.gamma, ct, sV, nfold);
        if (KP) {
          const int64_t cell = ((int64_t)czi * g.cy + cy) * g.cx + cx;
          const int ks = A.kstart[cell], ke = A.kstart[cell + 1];
          if (ke > ks) kp_cell<MODE>(g, q, ks, ke, A.kloc, A.ktgt, cc, A.delta, ct, sK);
        }
      }
      if (F > 0) {
#pragma unroll
        for (int f = 0; f < F; ++f)
#pragma unroll
          for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
              for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int c = 0; c < 3; ++c) cterm[f][k][j][i][c] = quad_sum(ct[f][k][j][i][c]);
      }
    }

    if (F > 0) {
      // node plane czi is complete: carried part + this layer's lower plane
      float nv[FS][2][3], cv[FS][2][2][3];
#pragma unroll
      for (int f = 0; f < FS; ++f)
#pragma unroll
        for (int jn = 0; jn < 2; ++jn)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            nv[f][jn][c] = carN[f][jn][c] + accN[f][0][jn][c];
            carN[f][jn][c] = accN[f][1][jn][c];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
              cv[f][jn][i][c] = carC[f][jn][i][c] + cterm[f][0][jn][i][c];
              carC[f][jn][i][c] = cterm[f][1][jn][i][c];
            }
          }
      emit(czi - cz0, nv, cv);
    }
    // roll the corners
    if (need_u) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) cc.u[0][j][i][c] = cc.u[1][j][i][c];
    }
    if (need_v) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) cc.v[0][j][i][c] = cc.v[1][j][i][c];
    }
  }
  if (F > 0) emit(cz1 - cz0, carN, carC);

  // workgroup scalars in a fixed order
  if (MODE != M_HV) {
    double vals[BS_N] = {sD, sV * (double)g.C, sK, (double)nfold};
#pragma unroll
    for (int t = 0; t < BS_N; ++t) {
      const double s = wave_sum_d(vals[t]);
      if (lane == 0) lred[wave][t] = s;
    }
    __syncthreads();
    if (threadIdx.x < BS_N) {
      const int t = threadIdx.x;
      const int64_t wg = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
      A.blocks[wg * BS_N + t] = ((lred[0][t] + lred[1][t]) + lred[2][t]) + lred[3][t];
    }
  }
}

// ---------------------------------------------------------------------------------
// Node-parallel gather: finishes brick-face nodes from the partial buffer, adds the
// curvature term alpha C_H L^T L w from a precomputed L w, the damping tau v, and
// optionally a per-block dot product <dotv, out> (FP64).
// ---------------------------------------------------------------------------------
struct GatherArgs {
  Geo g;
  int F;                 // fields written by the brick kernel (0: none ran)
  int nf;                // fields to produce (1 or 2)
  const float *part;
  float *out0, *out1;
  const float *Lw;       // L w (nullable): adds alpha C_H L^T L w to field 0
  float curv_scale;      // alpha C_H
  int curv_diag;         // add alpha C_H diag(L^T L) to field 1
  const float *tauv;     // adds tau * tauv to field 0 (nullable)
  float tau;
  const float *dotv;     // per-block <dotv, out0> (nullable)
  double *blocks;        // [nblocks][2]: <dotv,out0>, and for nf = 2: max(out1), <out0,out0>
  const double *stop;
};

__device__ __forceinline__ int chi(int p, int n) { return (p >= 1 && p <= n - 2) ? 1 : 0; }

__device__ __forceinline__ int brick_cands(int p, int B, int nb, int b[2], int l[2]) {
  int n = 0;
  const int b0 = p / B;
  for (int bb = b0 - 1; bb <= b0; ++bb) {
    if (bb < 0 || bb >= nb) continue;
    const int ll = p - bb * B;
    if (ll < 0 || ll > B) continue;
    b[n] = bb;
    l[n] = ll;
    ++n;
  }
  return n;
}

template <int ZC>
__global__ __launch_bounds__(256) void k_gather(GatherArgs A) {
  __shared__ double red[256];
  if (A.stop && *A.stop != 0.0) return;
  const Geo &g = A.g;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double dsum = 0.0, dmax = 0.0, gsq = 0.0;
  if (n < g.nnodes) {
    const int px = (int)(n % g.px), py = (int)((n / g.px) % g.py), pz = (int)(n / ((int64_t)g.px * g.py));
    int bxs[2], lxs[2], bys[2], lys[2], bzs[2], lzs[2];
    int nbx = 0, nby = 0, nbz = 0;
    bool shared = false;
    if (A.F > 0) {
      nbx = brick_cands(px, kBXC, g.nbx, bxs, lxs);
      nby = brick_cands(py, kBYC, g.nby, bys, lys);
      nbz = brick_cands(pz, ZC, g.nbz, bzs, lzs);
      shared = nbx > 1 || nby > 1 || nbz > 1;
    }
    for (int f = 0; f < A.nf; ++f) {
      float *o = f == 0 ? A.out0 : A.out1;
      for (int c = 0; c < 3; ++c) {
        const int64_t oi = c * g.nnodes + n;
        float val = 0.0f;
        if (A.F > f) {
          if (shared) {
            for (int iz = 0; iz < nbz; ++iz)
              for (int iy = 0; iy < nby; ++iy)
                for (int ixx = 0; ixx < nbx; ++ixx) {
                  const int64_t brick = ((int64_t)bzs[iz] * g.nby + bys[iy]) * g.nbx + bxs[ixx];
                  val += A.part[((brick * (ZC + 1) + lzs[iz]) * (A.F * 3) + f * 3 + c) * kNBOX + lys[iy] * 17 +
                                lxs[ixx]];
                }
          } else {
            val = o[oi];
          }
        }
        if (f == 0 && A.Lw) {
          // (L^T z)(p) = sum_a [chi_a(p-e_a) z(p-e_a) - 2 chi_a(p) z(p) + chi_a(p+e_a) z(p+e_a)] / H_a^2
          const float *z = A.Lw + c * g.nnodes;
          const int pp[3] = {px, py, pz};
          const int nn[3] = {g.px, g.py, g.pz};
          const int64_t st[3] = {1, g.px, (int64_t)g.px * g.py};
          const float ih2[3] = {g.iHx * g.iHx, g.iHy * g.iHy, g.iHz * g.iHz};
          float acc = 0.0f;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            float t = -2.0f * chi(pp[a], nn[a]) * z[n];
            if (pp[a] > 0 && chi(pp[a] - 1, nn[a])) t += z[n - st[a]];
            if (pp[a] < nn[a] - 1 && chi(pp[a] + 1, nn[a])) t += z[n + st[a]];
            acc += t * ih2[a];
          }
          val += A.curv_scale * acc;
        }
        if (f == 1 && A.curv_diag) {
          const int pp[3] = {px, py, pz};
          const int nn[3] = {g.px, g.py, g.pz};
          const float ih2[3] = {g.iHx * g.iHx, g.iHy * g.iHy, g.iHz * g.iHz};
          float centre = 0.0f, side = 0.0f;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            centre += 2.0f * chi(pp[a], nn[a]) * ih2[a];
            const int nb = (pp[a] > 0 ? chi(pp[a] - 1, nn[a]) : 0) + (pp[a] < nn[a] - 1 ? chi(pp[a] + 1, nn[a]) : 0);
            side += nb * ih2[a] * ih2[a];
          }
          val += A.curv_scale * (centre * centre + side);
        }
        if (f == 0 && A.tauv) val += A.tau * A.tauv[oi];
        o[oi] = val;
        if (f == 0 && A.dotv) dsum += (double)A.dotv[oi] * (double)val;
        if (f == 0) gsq += (double)val * (double)val;
        if (f == 1) dmax = fmax(dmax, (double)val);
      }
    }
  }
  if (A.blocks) {
    // fixed-order tree reductions
    const int t = threadIdx.x;
    double vals[3] = {dsum, dmax, gsq};
    for (int k = 0; k < 3; ++k) {
      red[t] = vals[k];
      __syncthreads();
      for (int s = 128; s > 0; s >>= 1) {
        if (t < s) red[t] = (k == 1) ? fmax(red[t], red[t + s]) : red[t] + red[t + s];
        __syncthreads();
      }
      if (t == 0) A.blocks[blockIdx.x * 3 + k] = red[0];
      __syncthreads();
    }
  }
}

// L w for w = a - b (b nullable), and per-block sum of (L w)^2
__global__ __launch_bounds__(256) void k_curv_L(Geo g, const float *a, const float *b, float *Lw, double *blocks,
                                                const double *stop) {
  __shared__ double red[256];
  if (stop && *stop != 0.0) return;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double e = 0.0;
  if (n < g.nnodes) {
    const int px = (int)(n % g.px), py = (int)((n / g.px) % g.py), pz = (int)(n / ((int64_t)g.px * g.py));
    const int pp[3] = {px, py, pz};
    const int nn[3] = {g.px, g.py, g.pz};
    const int64_t st[3] = {1, g.px, (int64_t)g.px * g.py};
    const float ih2[3] = {g.iHx * g.iHx, g.iHy * g.iHy, g.iHz * g.iHz};
    for (int c = 0; c < 3; ++c) {
      const float *ac = a + c * g.nnodes;
      const float *bc = b ? b + c * g.nnodes : nullptr;
      auto w = [&](int64_t m) { return bc ? ac[m] - bc[m] : ac[m]; };
      float acc = 0.0f;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
        if (chi(pp[ax], nn[ax])) acc += (w(n - st[ax]) - 2.0f * w(n) + w(n + st[ax])) * ih2[ax];
      Lw[c * g.nnodes + n] = acc;
      e += (double)acc * (double)acc;
    }
  }
  if (blocks) {
    const int t = threadIdx.x;
    red[t] = e;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) red[t] += red[t + s];
      __syncthreads();
    }
    if (t == 0) blocks[blockIdx.x] = red[0];
  }
}

// central-difference image gradient with replicated border, stored as ST
template <class ST>
__global__ __launch_bounds__(256) void k_imgrad(Geo g, const float *img, typename ST::elem *out, float sq) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= g.nvox) return;
  const int i = (int)(v % g.nx), j = (int)((v / g.nx) % g.ny), k = (int)(v / ((int64_t)g.nx * g.ny));
  const int64_t sx = 1, sy = g.nx, sz = (int64_t)g.nx * g.ny;
  const int64_t xm = i > 0 ? v - sx : v, xp = i < g.nx - 1 ? v + sx : v;
  const int64_t ym = j > 0 ? v - sy : v, yp = j < g.ny - 1 ? v + sy : v;
  const int64_t zm = k > 0 ? v - sz : v, zp = k < g.nz - 1 ? v + sz : v;
  float o[3];
  o[0] = (img[xp] - img[xm]) * (0.5f * g.ihx);
  o[1] = (img[yp] - img[ym]) * (0.5f * g.ihy);
  o[2] = (img[zp] - img[zm]) * (0.5f * g.ihz);
  ST::store(out, v, sq, o);
}

// max |grad| of a volume in blocks (for the FP16 scale)
__global__ __launch_bounds__(256) void k_absmax_grad(Geo g, const float *img, double *blocks) {
  __shared__ double red[256];
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double m = 0.0;
  if (v < g.nvox) {
    const int i = (int)(v % g.nx), j = (int)((v / g.nx) % g.ny), k = (int)(v / ((int64_t)g.nx * g.ny));
    const int64_t sx = 1, sy = g.nx, sz = (int64_t)g.nx * g.ny;
    const int64_t xm = i > 0 ? v - sx : v, xp = i < g.nx - 1 ? v + sx : v;
    const int64_t ym = j > 0 ? v - sy : v, yp = j < g.ny - 1 ? v + sy : v;
    const int64_t zm = k > 0 ? v - sz : v, zp = k < g.nz - 1 ? v + sz : v;
    m = fmax(fabs((double)((img[xp] - img[xm]) * (0.5f * g.ihx))),
             fmax(fabs((double)((img[yp] - img[ym]) * (0.5f * g.ihy))),
                  fabs((double)((img[zp] - img[zm]) * (0.5f * g.ihz)))));
  }
  const int t = threadIdx.x;
  red[t] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] = fmax(red[t], red[t + s]);
    __syncthreads();
  }
  if (t == 0) blocks[blockIdx.x] = red[0];
}

// convert a stored 3-vector volume to float32 [N][3]
template <class ST>
__global__ __launch_bounds__(256) void k_unpack3(Geo g, const typename ST::elem *in, float s, float *out) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= g.nvox) return;
  float o[3];
  ST::load(in, v, s, o);
  out[3 * v] = o[0];
  out[3 * v + 1] = o[1];
  out[3 * v + 2] = o[2];
}

// ---------------------------------------------------------------------------------
// Deterministic single-workgroup reduction of per-block values:
// out[k] = sum (or max) over b of blocks[b * stride + k], k < nvals.
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce(const double *blocks, int64_t nb, int stride, int nvals,
                                                uint32_t max_mask, double *out, const double *stop) {
  __shared__ double red[256];
  if (stop && *stop != 0.0) return;
  const int t = threadIdx.x;
  for (int k = 0; k < nvals; ++k) {
    const bool mx = (max_mask >> k) & 1u;
    double acc = mx ? -INFINITY : 0.0;
    for (int64_t b = t; b < nb; b += 256) {
      const double x = blocks[b * stride + k];
      acc = mx ? fmax(acc, x) : acc + x;
    }
    red[t] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) red[t] = mx ? fmax(red[t], red[t + s]) : red[t] + red[t + s];
      __syncthreads();
    }
    if (t == 0) out[k] = red[0];
    __syncthreads();
  }
}

}  // namespace disco
