// Keypoint stage (Sec. II-C2, II-C3): the NGF matching cost of eq. 2 over a grid of
// displacements, and min-sum belief propagation (eq. 4 with the regulariser of eq. 3)
// on a tree over the keypoints.
//
// The patch offsets {-3,-1,1,3} are odd and the displacements (step 2) even, so every
// voxel a keypoint's cost reads from the moving image, and every patch voxel of the fixed
// image, has the parity (k + 1) mod 2 per axis.  The normalised gradient 4-vectors
// (eta, grad I) / |(eta, grad I)| are therefore stored split by voxel parity: the voxels a
// keypoint needs form a dense (2R + 4)^3 block of one parity sub-volume, staged through
// LDS row by row with coalesced loads.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace disco {

// parity-split volume of float4: sub-volume (px, py, pz) holds voxels (2x + px, 2y + py,
// 2z + pz) at [((pz * 2 + py) * 2 + px)][z][y][x], each sub-volume hz x hy x hx with
// h_a = (n_a + 1) / 2; entries past the volume hold the vector of a zero gradient.
struct KpGeo {
  int nx, ny, nz;
  int hx, hy, hz;
  float ihx2, ihy2, ihz2;  // 1 / (2 h_a): central differences in HU/mm
};

__device__ __forceinline__ int64_t kp_par_index(const KpGeo &g, int px, int py, int pz, int x, int y, int z) {
  return ((((int64_t)((pz * 2 + py) * 2 + px) * g.hz + z) * g.hy + y) * g.hx + x);
}

// normalised 4-vectors of one image: thread per parity-split entry
__global__ __launch_bounds__(256) void k_kp_normalize(KpGeo g, const float *__restrict__ img, float eta,
                                                      float4 *__restrict__ out) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  const int zp = blockIdx.z;  // z + hz * parity index
  if (x >= g.hx) return;
  const int par = zp / g.hz, z = zp - par * g.hz;
  const int px = par & 1, py = (par >> 1) & 1, pz = par >> 2;
  const int vx = 2 * x + px, vy = 2 * y + py, vz = 2 * z + pz;
  float4 r = make_float4(1.0f, 0.0f, 0.0f, 0.0f);
  if (vx < g.nx && vy < g.ny && vz < g.nz) {
    auto at = [&](int i, int j, int k) { return img[((int64_t)k * g.ny + j) * g.nx + i]; };
    const float gx = (at(min(vx + 1, g.nx - 1), vy, vz) - at(max(vx - 1, 0), vy, vz)) * g.ihx2;
    const float gy = (at(vx, min(vy + 1, g.ny - 1), vz) - at(vx, max(vy - 1, 0), vz)) * g.ihy2;
    const float gz = (at(vx, vy, min(vz + 1, g.nz - 1)) - at(vx, vy, max(vz - 1, 0))) * g.ihz2;
    const float inv = rsqrtf(eta * eta + gx * gx + gy * gy + gz * gz);
    r = make_float4(eta * inv, gx * inv, gy * inv, gz * inv);
  }
  out[kp_par_index(g, px, py, pz, x, y, z)] = r;
}

constexpr int kKpRmax = 16;  // label radius: 2R + 1 <= 33 labels per axis
#ifndef DISCO_KP_ROWS
#define DISCO_KP_ROWS 11
#endif
#ifndef DISCO_KP_CHUNK
#define DISCO_KP_CHUNK 4
#endif
constexpr int kKpRows = DISCO_KP_ROWS;    // label rows (y) per workgroup
constexpr int kKpChunk = DISCO_KP_CHUNK;  // labels along x per thread
#ifndef DISCO_KP_PAD
#define DISCO_KP_PAD 1
#endif
#ifndef DISCO_KP_OYU
#define DISCO_KP_OYU 2
#endif
#ifndef DISCO_KP_OZU
#define DISCO_KP_OZU 1
#endif
// (LDS padding 1, oy unrolled by 2: measured best of the variants tried)
constexpr int kKpW = 2 * kKpRmax + 4;     // staged block width: 36
constexpr int kKpWP = kKpW + DISCO_KP_PAD;  // LDS row stride (float4)
constexpr int kKpNch = (2 * kKpRmax + 1 + kKpChunk - 1) / kKpChunk;
constexpr int kKpThreads = ((kKpRows * kKpNch + 63) / 64) * 64;

// the 64 fixed-image patch vectors of every keypoint, [nkp][64] (o = (ox, oy, oz) with
// index (oz * 4 + oy) * 4 + ox)
__global__ __launch_bounds__(64) void k_kp_patch(KpGeo g, const float4 *__restrict__ nF, int nkp,
                                                 const int *__restrict__ kp, float4 *__restrict__ patch) {
  const int k = blockIdx.x, t = threadIdx.x;
  const int kx = kp[3 * k], ky = kp[3 * k + 1], kz = kp[3 * k + 2];
  const int px = (kx + 1) & 1, py = (ky + 1) & 1, pz = (kz + 1) & 1;
  const int ox = t & 3, oy = (t >> 2) & 3, oz = t >> 4;
  // patch voxel k + o (o = 2 oi - 3): lattice (k + 1 - p) / 2 - 2 + oi
  const int x = (kx + 1 - px) / 2 - 2 + ox, y = (ky + 1 - py) / 2 - 2 + oy, z = (kz + 1 - pz) / 2 - 2 + oz;
  float4 v = make_float4(1.0f, 0.0f, 0.0f, 0.0f);
  if ((unsigned)x < (unsigned)g.hx && (unsigned)y < (unsigned)g.hy && (unsigned)z < (unsigned)g.hz)
    v = nF[kp_par_index(g, px, py, pz, x, y, z)];
  patch[(int64_t)k * 64 + t] = v;
}

// D_KP(k, d) for one keypoint k and up to kKpRows label rows iy, all label planes iz in
// turn.  The moving-image vectors the labels need lie in a (2R + 4)^3 block of one parity
// sub-volume; the workgroup keeps a ring of kKpRing lattice planes (rows + 3 rows of
// 2R + 4 vectors each) in LDS: plane iz + 4 is loaded into registers while the labels of
// plane iz are computed from planes iz .. iz + 3, then stored into the ring slot that is no
// longer needed.  Each thread accumulates sum r^2 for kKpChunk labels along x (every staged
// vector serves up to 4 labels); the keypoint's 64 patch vectors are read from LDS by
// broadcast.  Work items are ordered keypoint-major and dealt to the 8 XCDs in contiguous
// runs.
constexpr int kKpRing = 5;
constexpr int kKpPlane = (kKpRows + 3) * kKpW;                        // vectors per staged plane
constexpr int kKpPre = (kKpPlane + kKpThreads - 1) / kKpThreads;      // prefetched vectors per thread

__global__ __launch_bounds__(kKpThreads) void k_kp_cost(KpGeo g, const float4 *__restrict__ nM,
                                                        const float4 *__restrict__ patch, int nkp,
                                                        const int *__restrict__ kp, int R, int items, int run,
                                                        float *__restrict__ cost) {
  __shared__ float4 sM[kKpRing][kKpRows + 3][kKpWP];
  __shared__ float4 sP[64];  // the keypoint's patch vectors, read by all threads at one address
  const int hw = blockIdx.x;
  const int item = (hw & 7) * run + (hw >> 3);
  if (item >= items) return;
  const int nl = 2 * R + 1, W = 2 * R + 4;
  const int nh = (nl + kKpRows - 1) / kKpRows;
  const int k = item / nh, iy0 = (item - k * nh) * kKpRows;
  const int nrow = min(kKpRows, nl - iy0);
  const int kx = kp[3 * k], ky = kp[3 * k + 1], kz = kp[3 * k + 2];
  const int px = (kx + 1) & 1, py = (ky + 1) & 1, pz = (kz + 1) & 1;
  // lattice coordinate of voxel k + o + d: base + oi + i (oi = patch index, i = label index)
  const int bx = (kx + 1 - px) / 2 - 2 - R, by = (ky + 1 - py) / 2 - 2 - R, bz = (kz + 1 - pz) / 2 - 2 - R;
  const int t = threadIdx.x;
  const int npl = (nrow + 3) * W;  // vectors of one staged plane
  auto fetch = [&](int e, int zl) {
    const int xx = e % W, rr = e / W;
    const int x = bx + xx, y = by + iy0 + rr, z = bz + zl;
    float4 v = make_float4(1.0f, 0.0f, 0.0f, 0.0f);
    if ((unsigned)x < (unsigned)g.hx && (unsigned)y < (unsigned)g.hy && (unsigned)z < (unsigned)g.hz)
      v = nM[kp_par_index(g, px, py, pz, x, y, z)];
    return v;
  };
  // planes 0..3 of the window into ring slots 0..3
  for (int e = t; e < 4 * npl; e += kKpThreads) {
    const int pl = e / npl, r = e - pl * npl;
    sM[pl][r / W][r % W] = fetch(r, pl);
  }
  if (t < 64) sP[t] = patch[(int64_t)k * 64 + t];
  __syncthreads();
  const int nch = (nl + kKpChunk - 1) / kKpChunk;
  const int row = t / nch, ch = t - row * nch;
  const bool active = row < nrow;
  const int ix0 = ch * kKpChunk;
  const int64_t L = (int64_t)nl * nl * nl;
  for (int iz = 0; iz < nl; ++iz) {
    // prefetch window plane iz + 4 (the last label plane needs planes up to nl + 2)
    const bool pre = iz + 4 < nl + 3;
    float4 nxt[kKpPre];
#pragma unroll
    for (int q = 0; q < kKpPre; ++q) {
      const int e = t + q * kKpThreads;
      nxt[q] = (pre && e < npl) ? fetch(e, iz + 4) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    if (active) {
      float acc[kKpChunk];
#pragma unroll
      for (int c = 0; c < kKpChunk; ++c) acc[c] = 0.0f;
#pragma unroll 1
      for (int oz = 0; oz < 4; ++oz) {
        const int slot = (iz + oz) % kKpRing;
#pragma unroll DISCO_KP_OYU
        for (int oy = 0; oy < 4; ++oy) {
          float4 b[4];
#pragma unroll
          for (int ox = 0; ox < 4; ++ox) b[ox] = sP[(oz * 4 + oy) * 4 + ox];
          float4 a[kKpChunk + 3];
#pragma unroll
          for (int j = 0; j < kKpChunk + 3; ++j) a[j] = sM[slot][row + oy][min(ix0 + j, W - 1)];
#pragma unroll
          for (int c = 0; c < kKpChunk; ++c)
#pragma unroll
            for (int ox = 0; ox < 4; ++ox) {
              const float4 &u = a[c + ox];
              const float r = u.x * b[ox].x + u.y * b[ox].y + u.z * b[ox].z + u.w * b[ox].w;
              acc[c] = __builtin_fmaf(r, r, acc[c]);
            }
        }
      }
      float *o = cost + (int64_t)k * L + ((int64_t)iz * nl + iy0 + row) * nl;
#pragma unroll
      for (int c = 0; c < kKpChunk; ++c)
        if (ix0 + c < nl) o[ix0 + c] = 1.0f - acc[c] * (1.0f / 64.0f);
    }
    // plane iz + 4 goes to the slot of plane iz - 1, which no thread reads any more
    if (pre) {
      const int slot = (iz + 4) % kKpRing;
#pragma unroll
      for (int q = 0; q < kKpPre; ++q) {
        const int e = t + q * kKpThreads;
        if (e < npl) sM[slot][e / W][e % W] = nxt[q];
      }
    }
    __syncthreads();
  }
}

// (weight, index) minimum with ties to the lowest index
__device__ __forceinline__ void argmin_pair(double &v, int &i, double ov, int oi) {
  if (ov < v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}

// ---- minimum spanning tree by Boruvka rounds ------------------------------------------
// One round: for every keypoint i, the cheapest edge (i, j) to a keypoint of another
// component (comp[j] != comp[i]), ties to the lowest j; one wave per keypoint.  Edge
// costs |x_i - x_j| + |I_i - I_j| / sigma_I in double precision from the float inputs, in
// a fixed order without fused multiply-adds, so they are symmetric.
__global__ __launch_bounds__(256) void k_kp_boruvka(int n, const float *__restrict__ x,
                                                    const float *__restrict__ inten, double sigma_I,
                                                    const int *__restrict__ comp, double *__restrict__ best_w,
                                                    int *__restrict__ best_j) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= n) return;
  const double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2], ii = inten[i];
  const int ci = comp[i];
  double bw = INFINITY;
  int bj = 0x7fffffff;
  for (int j = lane; j < n; j += 64) {
    if (comp[j] == ci) continue;
    const double dx = (double)x[3 * j] - xi, dy = (double)x[3 * j + 1] - yi, dz = (double)x[3 * j + 2] - zi;
    const double ss = (dx * dx + dy * dy) + dz * dz;
    const double w = sqrt(ss) + fabs((double)inten[j] - ii) / sigma_I;
    argmin_pair(bw, bj, w, j);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double ov = __shfl_xor(bw, o, 64);
    const int oj = __shfl_xor(bj, o, 64);
    argmin_pair(bw, bj, ov, oj);
  }
  if (lane == 0) {
    best_w[i] = bw;
    best_j[i] = bj;
  }
}

// ---- belief propagation on the tree, one tree level per launch ---------------------
// The work buffers (h, inward messages m, temporaries) are indexed by breadth-first
// position from the root, so a level is a contiguous range of positions and so are the
// children of a node. Per position: KpNode {keypoint id, parent's keypoint id (-1 at the
// root), first child's position, child count} and the pairwise weight cw of the edge to
// the parent. The data cost D and the min-marginals M are indexed by keypoint id.
struct KpNode {
  int kid, pkid, cfirst, ccount;
};

// The min-convolution of a label volume with the quadratic pairwise cost,
//   out(d) = min_d' in(d') + cw |d - d'|^2   (d in mm, labels [iz][iy][ix]),
// is separable: three passes of the 1-D form out(i) = min_j in(j) + p (i - j)^2 with
// p = cw step_a^2, x and y on a label plane of fixed iz, z on a plane of fixed iy. A
// workgroup takes one (node, plane) and holds the plane in LDS (row pitch 33 whatever the
// label count), so even a tree level with few nodes spreads over many workgroups.
// Expanding the square, out(i) = min_j (in(j) + p j^2 - 2 p i j) + p i^2: one fused
// multiply-add and a minimum per candidate, each candidate shared by the five outputs of
// a line that one thread computes (seven threads per line).
constexpr int kKpNl = 2 * kKpRmax + 1;                // 33
constexpr int kKpPer = (kKpNl * kKpNl + 255) / 256;  // plane entries per thread when loading: 5
constexpr int kKpG = 7;                               // threads per line
constexpr int kKpR = (kKpNl + kKpG - 1) / kKpG;       // outputs per thread: 5

// The 1-D pass over the nl lines of a plane in LDS, line l holding src[l * LS + j * ES]
// (j < nl); thread (l, g) computes the outputs i = g + 7 r and hands them to
// store(l, i, value). NL = 33 fixes nl at compile time (R = 16), NL = 0 takes it at run time.
template <int LS, int ES, int NL, class Store>
__device__ __forceinline__ void kp_mincon_lines(const float *src, int nl, float p, Store store) {
  const int tid = threadIdx.x;
  if (tid >= nl * kKpG) return;
  const int l = tid / kKpG, g = tid - l * kKpG;
  float s[kKpR], best[kKpR];
#pragma unroll
  for (int r = 0; r < kKpR; ++r) {
    s[r] = -2.0f * p * (float)(g + kKpG * r);
    best[r] = INFINITY;
  }
#pragma unroll
  for (int j = 0; j < kKpNl; ++j) {
    if (NL == kKpNl || j < nl) {
      const float A = src[l * LS + j * ES] + p * (float)(j * j);
#pragma unroll
      for (int r = 0; r < kKpR; ++r) best[r] = fminf(best[r], fmaf(s[r], (float)j, A));
    }
  }
#pragma unroll
  for (int r = 0; r < kKpR; ++r) {
    const int i = g + kKpG * r;
    if (i < nl) store(l, i, r, best[r] + p * (float)(i * i));
  }
}

// x and y passes on the plane iz = blockIdx.y of the node at position base + blockIdx.x.
// The plane's input is, inward (OUT = false), h = D + the inward messages of the node's
// children (h is also stored), outward (OUT = true), M_parent - m.
template <bool OUT, int NL>
__global__ __launch_bounds__(256) void k_kp_plane_xy(int nl_rt, int base, const KpNode *__restrict__ node,
                                                     const float *__restrict__ cw, const float *src,
                                                     const float *__restrict__ msg, float sx, float sy,
                                                     float *__restrict__ h, float *__restrict__ out) {
  __shared__ float a[kKpNl * kKpNl], b[kKpNl * kKpNl];
  const int nl = NL ? NL : nl_rt;
  const int pos = base + blockIdx.x;
  const KpNode nd = node[pos];
  const int nl2 = nl * nl;
  const int64_t L = (int64_t)nl2 * nl, po = (int64_t)blockIdx.y * nl2;
  float v[kKpPer];
  if constexpr (OUT) {
    const float *pp = src + (int64_t)nd.pkid * L + po, *m = msg + (int64_t)pos * L + po;
#pragma unroll
    for (int u = 0; u < kKpPer; ++u) {
      const int t = threadIdx.x + 256 * u;
      v[u] = t < nl2 ? pp[t] - m[t] : 0.0f;
    }
  } else {
    const float *d = src + (int64_t)nd.kid * L + po;
#pragma unroll
    for (int u = 0; u < kKpPer; ++u) {
      const int t = threadIdx.x + 256 * u;
      v[u] = t < nl2 ? d[t] : 0.0f;
    }
    for (int c = 0; c < nd.ccount; ++c) {
      const float *m = msg + (int64_t)(nd.cfirst + c) * L + po;
#pragma unroll
      for (int u = 0; u < kKpPer; ++u) {
        const int t = threadIdx.x + 256 * u;
        if (t < nl2) v[u] += m[t];
      }
    }
    float *hp = h + (int64_t)pos * L + po;
#pragma unroll
    for (int u = 0; u < kKpPer; ++u) {
      const int t = threadIdx.x + 256 * u;
      if (t < nl2) hp[t] = v[u];
    }
  }
#pragma unroll
  for (int u = 0; u < kKpPer; ++u) {
    const int t = threadIdx.x + 256 * u;
    if (t < nl2) {
      const int iy = t / nl, ix = t - iy * nl;
      a[iy * kKpNl + ix] = v[u];
    }
  }
  __syncthreads();
  const float w = cw[pos];
  // x: line iy, outputs ix
  kp_mincon_lines<kKpNl, 1, NL>(a, nl, w * sx * sx, [&](int iy, int ix, int, float val) { b[iy * kKpNl + ix] = val; });
  __syncthreads();
  // y: line ix, outputs iy
  float *o = out + (int64_t)pos * L + po;
  kp_mincon_lines<1, kKpNl, NL>(b, nl, w * sy * sy, [&](int ix, int iy, int, float val) { o[iy * nl + ix] = val; });
}

// z pass on the plane iy = blockIdx.y of the node at position base + blockIdx.x, input
// in[position]. Inward (OUT = false) the result is the node's message m[position];
// outward (OUT = true) M[keypoint id] = h[position] + the result.
template <bool OUT, int NL>
__global__ __launch_bounds__(256) void k_kp_plane_z(int nl_rt, int base, const KpNode *__restrict__ node,
                                                    const float *__restrict__ cw, float sz, const float *__restrict__ in,
                                                    const float *__restrict__ h, float *__restrict__ out) {
  __shared__ float a[kKpNl * kKpNl];  // a[iz][ix] = in(iz, iy, ix)
  const int nl = NL ? NL : nl_rt;
  const int pos = base + blockIdx.x;
  const int nl2 = nl * nl;
  const int64_t L = (int64_t)nl2 * nl, po = (int64_t)pos * L + (int64_t)blockIdx.y * nl;
  float v[kKpPer];
#pragma unroll
  for (int u = 0; u < kKpPer; ++u) {
    const int t = threadIdx.x + 256 * u;
    const int iz = t / nl, ix = t - iz * nl;
    v[u] = t < nl2 ? in[po + (int64_t)iz * nl2 + ix] : 0.0f;
  }
  // outward: the h values this thread's outputs add to (line ix = l, outputs iz = g + 7 r)
  float hv[kKpR];
  {
    const int tid = threadIdx.x, l = tid / kKpG, g = tid - l * kKpG;
#pragma unroll
    for (int r = 0; r < kKpR; ++r) {
      const int iz = g + kKpG * r;
      hv[r] = OUT && tid < nl * kKpG && iz < nl ? h[po + (int64_t)iz * nl2 + l] : 0.0f;
    }
  }
#pragma unroll
  for (int u = 0; u < kKpPer; ++u) {
    const int t = threadIdx.x + 256 * u;
    if (t < nl2) {
      const int iz = t / nl, ix = t - iz * nl;
      a[iz * kKpNl + ix] = v[u];
    }
  }
  __syncthreads();
  const int64_t oo = OUT ? (int64_t)node[pos].kid * L + (int64_t)blockIdx.y * nl : po;
  // z: line ix, outputs iz
  kp_mincon_lines<1, kKpNl, NL>(a, nl, cw[pos] * sz * sz, [&](int ix, int iz, int r, float val) {
    out[oo + (int64_t)iz * nl2 + ix] = OUT ? hv[r] + val : val;
  });
}

// root (position 0): h = D + its children's inward messages, and M = h; thread per label
__global__ __launch_bounds__(256) void k_kp_root(int64_t L, const KpNode *__restrict__ node, const float *__restrict__ D,
                                                 const float *__restrict__ msg, float *__restrict__ h,
                                                 float *__restrict__ M) {
  const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (l >= L) return;
  const KpNode nd = node[0];
  float v = D[(int64_t)nd.kid * L + l];
  for (int c = 0; c < nd.ccount; ++c) v += msg[(int64_t)(nd.cfirst + c) * L + l];
  h[l] = v;
  M[(int64_t)nd.kid * L + l] = v;
}

// label of the smallest min-marginal per keypoint (lowest index on ties): one workgroup
// per keypoint
__global__ __launch_bounds__(256) void k_kp_argmin(int64_t L, const float *__restrict__ marg, int *__restrict__ lab) {
  __shared__ float sv[256];
  __shared__ int si[256];
  const int k = blockIdx.x, t = threadIdx.x;
  const float *m = marg + (int64_t)k * L;
  float bv = INFINITY;
  int bi = 0x7fffffff;
  for (int64_t l = t; l < L; l += 256) {
    const float v = m[l];
    if (v < bv) {
      bv = v;
      bi = (int)l;
    }
  }
  sv[t] = bv;
  si[t] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      const float ov = sv[t + s];
      const int oi = si[t + s];
      if (ov < sv[t] || (ov == sv[t] && oi < si[t])) {
        sv[t] = ov;
        si[t] = oi;
      }
    }
    __syncthreads();
  }
  if (t == 0) lab[k] = si[0];
}

}  // namespace disco
