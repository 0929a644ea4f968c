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
#include <cfloat>
#include <stdint.h>

namespace disco {

constexpr int kWG = 256;   // threads of a brick workgroup (4 waves)

// The GN product pass with cell terms runs workgroups of 4 + kCellWaves waves: waves 0-3
// stream the voxels (NGF, memory-bound), the others compute the cell terms of the brick's
// layers (volume change, keypoints; VALU-bound), so that the SIMDs hold waves of both
// kinds and the two overlap.  All other passes use 4 waves that do both in turn.
#ifndef DISCO_CELL_WAVES
#define DISCO_CELL_WAVES 4
#endif
constexpr int kCellWaves = DISCO_CELL_WAVES;  // cell-term waves per GN product workgroup
template <int MODE, bool NGF, bool CELLT>
__host__ __device__ constexpr int brick_threads() {
  return (MODE == 2 && NGF && CELLT) ? 64 * (4 + kCellWaves) : 256;
}
constexpr int kBXC = 16;   // cells per brick along x (64 voxels = one wave)
constexpr int kBYC = 4;    // cells per brick along y (one wave per cell row)
constexpr int kNBOX = (kBXC + 1) * (kBYC + 1);  // nodes of one brick plane (17 x 5)

enum { M_EVAL = 0, M_GRAD = 1, M_HV = 2 };

// Block coordinates of a work item: the hardware block index for single-pair launches,
// or a (pair, block) item of a batched launch.  lin is the linear block index within the
// pair's grid (x fastest), which also indexes the pair's per-block partials.
struct Blk {
  int x, y, z;
  int64_t lin;
};
__device__ __forceinline__ Blk hw_blk() {
  return Blk{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z,
             ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x};
}

// block scalar slots written by k_brick (doubles per workgroup)
enum { BS_D = 0, BS_V = 1, BS_K = 2, BS_FOLD = 3, BS_B = 4, BS_N = 5 };
constexpr int kRedVals = 5;  // values per source of the single-workgroup reduction (>= BS_N)

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
  static constexpr int W = 3;  // elements per voxel
  static constexpr bool kScaled = false;  // stored values are the values
  // a voxel's stored words, loaded now and converted later (lets a pass request many
  // loads before it uses the first)
  struct raw {
    float x, y, z;
  };
  __device__ static inline raw fetch(const float *q) { return raw{q[0], q[1], q[2]}; }
  __device__ static inline void unpack(const raw &r, const float *q, float s, float o[3]) {
    o[0] = r.x;
    o[1] = r.y;
    o[2] = r.z;
    (void)q;
    (void)s;
  }
  __device__ static inline void loadp(const float *q, float s, float o[3]) {
    o[0] = q[0];
    o[1] = q[1];
    o[2] = q[2];
    (void)s;
  }
  __device__ static inline void storep(float *q, float s, const float v[3]) {
    q[0] = v[0];
    q[1] = v[1];
    q[2] = v[2];
    (void)s;
  }
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

// half precision, value = stored * s (s: per-volume power of two).  A voxel takes 4 halfs
// (8 B, the fourth zero): every voxel is one aligned 8-byte word, read with one load
// and converted from the two 32-bit halves of the word.
struct F16x3 {
  typedef __half elem;
  static constexpr int W = 4;  // elements per voxel (3 components and a zero)
  static constexpr bool kScaled = true;  // stored values times the volume's scale
  struct raw {
    uint2 w;
  };
  __device__ static inline float lo(uint32_t x) { return __half2float(__ushort_as_half((unsigned short)(x & 0xFFFFu))); }
  __device__ static inline float hi(uint32_t x) { return __half2float(__ushort_as_half((unsigned short)(x >> 16))); }
  // component c of a raw voxel word as a half (converted by the instruction that uses it)
  __device__ static inline _Float16 comp(const raw &r, int c) {
    const uint32_t w = c < 2 ? r.w.x : r.w.y;
    return __builtin_bit_cast(_Float16, (unsigned short)((c & 1) ? (w >> 16) : (w & 0xFFFFu)));
  }
  __device__ static inline raw fetch(const __half *q) { return raw{*reinterpret_cast<const uint2 *>(q)}; }
  __device__ static inline void unpack(const raw &r, const __half *q, float s, float o[3]) {
    o[0] = lo(r.w.x) * s;
    o[1] = hi(r.w.x) * s;
    o[2] = lo(r.w.y) * s;
    (void)q;
  }
  __device__ static inline void loadp(const __half *q, float s, float o[3]) { unpack(fetch(q), q, s, o); }
  __device__ static inline void storep(__half *q, float s, const float v[3]) {
    const uint32_t h0 = __half_as_ushort(__float2half_rn(v[0] * s));
    const uint32_t h1 = __half_as_ushort(__float2half_rn(v[1] * s));
    const uint32_t h2 = __half_as_ushort(__float2half_rn(v[2] * s));
    *reinterpret_cast<uint2 *>(q) = make_uint2(h0 | (h1 << 16), h2);
  }
  __device__ static inline void load(const __half *p, int64_t i, float s, float o[3]) { loadp(p + 4 * i, s, o); }
  __device__ static inline void store(__half *p, int64_t i, float s, const float v[3]) { storep(p + 4 * i, s, v); }
};


// ---------------------------------------------------------------------------------
// quad (4-lane) sums with DPP quad permutations: xor 1 = [1,0,3,2], xor 2 = [2,3,0,1]
// ---------------------------------------------------------------------------------
__device__ __forceinline__ float dpp_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_xor2(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
}
__device__ __forceinline__ float quad_sum(float v) {
  v = v + dpp_xor1(v);
  return v + dpp_xor2(v);
}

// hardware reciprocal (about 1 ulp); the IEEE division sequence is not needed here
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ bool is_face(int l, int b, int nb, int B) {
  return (l == 0 && b > 0) || (l == B && b + 1 < nb);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------------
// Scalar post-operations run after a reduction (solver bookkeeping on device scalars)
// ---------------------------------------------------------------------------------
enum {
  POST_NONE = 0,
  POST_WRITE,      // dst = out[idx] * scale (+inf if fold_inf and out[fold_idx] > 0); idst = out[fold_idx]
  POST_LIN_BRICK,  // linearisation: D, V, K, folds -> sc; J; fold status
  POST_LS_BRICK,   // line-search trial: D, V, K, folds -> sc; Armijo decision
  POST_PCG_START,  // <r,z>, <r,r> of the initial residual
  POST_LS_BEGIN,   // g^T p -> start of the line search
  POST_STORE,      // out values only
  POST_LB_PAIR,    // s.y, s.s, y.y of a new L-BFGS pair -> rho (0 if s.y <= eps |s||y|)
  POST_LB_ALPHA,   // alpha_idx = rho_idx * (s_idx . q)
  POST_EVAL        // objective only: J and its terms -> dst[0..7] (J, D, S, V, K, B, folds, NaN)
};

struct PostArgs {
  double *sc;         // device scalar slots (solver state)
  int *status;        // device status word
  double alpha, gamma, delta, CH, h3;  // objective weights, C_H, voxel volume
  double beta;                        // lung-boundary weight
  double c1, tol;     // Armijo constant, CG tolerance
  double *dst;        // POST_WRITE destination (nullable)
  int32_t *idst;      // POST_WRITE fold-count destination (nullable)
  double scale;
  int idx, fold_idx, fold_inf;
};


// the objective from reduced terms; a fold counts only when gamma > 0 (then J = +inf)
__device__ inline double total_J(const PostArgs &w, double D, double Sraw, double V, double K, double nfold,
                                 double B) {
  if (w.gamma != 0.0 && nfold > 0.0) return INFINITY;
  return D + w.alpha * 0.5 * w.CH * Sraw + w.beta * B + (w.gamma != 0.0 ? w.gamma * V : 0.0) + w.delta * K;
}

// slots of the device scalar array used by the Gauss-Newton step
enum {
  SC_D = 0, SC_SRAW, SC_V, SC_K, SC_NFOLD,      // linearisation: D, sum (Lw)^2, C sum psi, sum |res|^2, folds
  SC_DOT, SC_MAXDIAG, SC_GG,                   // gather reductions: <dotv,out>, max diag, |out|^2
  SC_J, SC_RZ, SC_RZ1, SC_ALPHA, SC_BETA, SC_RR, SC_BB, SC_STOP, SC_ITERS, SC_BREAK,
  SC_GTP, SC_TTRY, SC_ACCEPT, SC_TACC, SC_TRIALS,
  SC_TD, SC_TSRAW, SC_TV, SC_TK, SC_TNFOLD,    // trial point reductions
  SC_JT, SC_DT, SC_ST, SC_VT, SC_KT,           // accepted (or last) trial values
  SC_TMP0, SC_TMP1, SC_TMP2, SC_TMP3, SC_TMP4,
  SC_B, SC_TB,                                 // lung-boundary term B at the linearisation / trial point
  SC_ESRAW,                                    // sum (L(u - uhat))^2 of an objective-only evaluation
  SC_LB_RHO = 48,     // L-BFGS: rho_i = 1 / s_i.y_i of the stored pairs (0: pair skipped)
  SC_LB_ALPHA = 56,   // L-BFGS: alpha_i of the first loop
  SC_LB_DOT = 64,     // L-BFGS: dot product scratch
  SC_COUNT = 72
};
constexpr int kLbfgsMax = 8;  // longest L-BFGS history
static_assert(SC_ESRAW < SC_LB_RHO && SC_TMP0 + kRedVals - 1 == SC_TMP4 && SC_LB_RHO + kLbfgsMax <= SC_LB_ALPHA && SC_LB_ALPHA + kLbfgsMax <= SC_LB_DOT &&
                  SC_LB_DOT < SC_COUNT,
              "scalar slots overlap");

__device__ inline void run_post(int post, const PostArgs &a, const double *r) {
  double *sc = a.sc;
  switch (post) {
    case POST_WRITE: {
      double v = r[a.idx] * a.scale;
      if (a.fold_inf && r[a.fold_idx] > 0.0) v = INFINITY;
      if (a.dst) *a.dst = v;
      if (a.idst) *a.idst = (int32_t)r[a.fold_idx];
      break;
    }
    case POST_LIN_BRICK:
      sc[SC_D] = r[0] * a.h3;
      sc[SC_V] = r[1];
      sc[SC_K] = r[2];
      sc[SC_NFOLD] = r[3];
      sc[SC_B] = 0.5 * a.h3 * r[4];
      sc[SC_J] = total_J(a, sc[SC_D], sc[SC_SRAW], sc[SC_V], sc[SC_K], sc[SC_NFOLD], sc[SC_B]);
      if (a.status && a.gamma != 0.0 && sc[SC_NFOLD] > 0.0) *a.status |= 1;
      break;
    case POST_LS_BRICK: {
      if (sc[SC_ACCEPT] != 0.0) break;
      sc[SC_TD] = r[0] * a.h3;
      sc[SC_TV] = r[1];
      sc[SC_TK] = r[2];
      sc[SC_TNFOLD] = r[3];
      sc[SC_TB] = 0.5 * a.h3 * r[4];
      const double t = sc[SC_TTRY];
      const double Jt = total_J(a, sc[SC_TD], sc[SC_TSRAW], sc[SC_TV], sc[SC_TK], sc[SC_TNFOLD], sc[SC_TB]);
      sc[SC_TRIALS] += 1.0;
      sc[SC_JT] = Jt;
      sc[SC_DT] = sc[SC_TD];
      sc[SC_ST] = 0.5 * a.CH * sc[SC_TSRAW];
      sc[SC_VT] = sc[SC_TV];
      sc[SC_KT] = sc[SC_TK];
      if (isfinite(Jt) && Jt <= sc[SC_J] + a.c1 * t * sc[SC_GTP]) {
        sc[SC_ACCEPT] = 1.0;
        sc[SC_TACC] = t;
      }
      break;
    }
    case POST_PCG_START:
      sc[SC_RZ] = r[0];
      sc[SC_BB] = r[1];
      sc[SC_RR] = r[1];
      sc[SC_STOP] = 0.0;
      sc[SC_ITERS] = 0.0;
      sc[SC_BREAK] = 0.0;
      break;
    case POST_LB_PAIR: {
      const double sy = r[0], ss = r[1], yy = r[2];
      sc[SC_LB_RHO + a.idx] = (sy > a.tol * sqrt(ss * yy) && sy > 0.0) ? 1.0 / sy : 0.0;
      break;
    }
    case POST_LB_ALPHA:
      sc[SC_LB_ALPHA + a.idx] = sc[SC_LB_RHO + a.idx] * r[0];
      break;
    case POST_EVAL: {
      const double D = r[0] * a.h3, B = 0.5 * a.h3 * r[4];
      a.dst[0] = total_J(a, D, sc[SC_ESRAW], r[1], r[2], r[3], B);
      a.dst[1] = D;
      a.dst[2] = 0.5 * a.CH * sc[SC_ESRAW];
      a.dst[3] = r[3] > 0.0 ? INFINITY : r[1];
      a.dst[4] = r[2];
      a.dst[5] = B;
      a.dst[6] = r[3];
      a.dst[7] = NAN;
      break;
    }
    case POST_LS_BEGIN:
      // residual of the last completed CG update (its partials were reduced into SC_TMP1)
      if (sc[SC_ITERS] > 0.0) sc[SC_RR] = sc[SC_TMP1 + 1];
      sc[SC_GTP] = r[0];
      sc[SC_ACCEPT] = 0.0;
      sc[SC_TACC] = 0.0;
      sc[SC_TRIALS] = 0.0;
      sc[SC_JT] = INFINITY;
      break;
    default:
      break;
  }
}

// One source of a single-workgroup reduction: out[k] = sum (or max) over b of
// blocks[b * stride + k], k < nvals <= kRedVals.
struct RedSrc {
  const double *blocks;
  int64_t nb;
  int stride, nvals;
  unsigned max_mask;  // bit k: value k is a maximum instead of a sum
  double *out;
};

// butterfly over the 64 lanes of a wave: every lane gets the same sum (or maximum)
__device__ __forceinline__ double wave_red_d(double v, bool mx) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double w = __shfl_xor(v, o, 64);
    v = mx ? fmax(v, w) : v + w;
  }
  return v;
}

// Reduce up to three sources of at most kRedVals values each in a fixed order (one workgroup of
// 1024 threads: per-thread sums over strided partials, a butterfly per wave, then the 16
// wave results in order), then run the scalar post-operation.  The first 2048 partials
// of every source are requested together.  Deterministic; no inter-workgroup
// communication.
__device__ __forceinline__ void finish_body(const RedSrc s0, const RedSrc s1, const RedSrc s2, int nsrc, int post,
                                            const PostArgs &pa, const double *stop) {
  __shared__ double wred[16][3 * kRedVals];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // sources selected by value (no addressable local array: it would live in scratch memory)
  auto src = [&](int q) -> RedSrc { return q == 0 ? s0 : (q == 1 ? s1 : s2); };
  const double stopv = stop ? *stop : 0.0;  // no workgroup writes it here: uniform
  double x[3][2][kRedVals];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const RedSrc S = src(q);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t b = u * 1024 + t;
#pragma unroll
      for (int k = 0; k < kRedVals; ++k) x[q][u][k] = (q < nsrc && b < S.nb && k < S.nvals) ? S.blocks[b * S.stride + k] : 0.0;
    }
  }
  if (stopv != 0.0) return;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const RedSrc S = src(q);
    if (q < nsrc) {
#pragma unroll
      for (int k = 0; k < kRedVals; ++k) {
        const bool mx = (S.max_mask >> k) & 1u;
        double acc = mx ? -INFINITY : 0.0;
#pragma unroll
        for (int u = 0; u < 2; ++u)
          if (u * 1024 + t < S.nb) acc = mx ? fmax(acc, x[q][u][k]) : acc + x[q][u][k];
        for (int64_t b = 2048 + t; b < S.nb; b += 1024) {
          const double y = k < S.nvals ? S.blocks[b * S.stride + k] : 0.0;
          acc = mx ? fmax(acc, y) : acc + y;
        }
        const double r = wave_red_d(acc, mx);
        if (lane == 0) wred[w][q * kRedVals + k] = r;
      }
    }
  }
  __syncthreads();
  // thread kRedVals q + k finishes value k of source q (q static in each unrolled pass)
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const RedSrc S = src(q);
    const int k = t - kRedVals * q;
    if (q < nsrc && k >= 0 && k < kRedVals && k < S.nvals) {
      const bool mx = (S.max_mask >> k) & 1u;
      double r = wred[0][t];
      for (int i = 1; i < 16; ++i) r = mx ? fmax(r, wred[i][t]) : r + wred[i][t];
      S.out[k] = r;
    }
  }
  __syncthreads();
  if (t == 0) run_post(post, pa, s0.out);
}

__global__ __launch_bounds__(1024) void k_finish(RedSrc s0, RedSrc s1, RedSrc s2, int nsrc, int post, PostArgs pa,
                                                 const double *stop) {
  finish_body(s0, s1, s2, nsrc, post, pa, stop);
}

// Sums of NV values over n partials, blocks[b * stride + k0 + k], computed identically by
// every 256-thread workgroup that calls it (fixed order: per-thread sums over b = t,
// t + 256, ... with sixteen loads in flight, a butterfly per wave, then the four wave
// sums in order).  Every thread receives the sums.  If flagp is given, thread 0 reads
// *flagp together with its partials and every thread receives that value in *flag (one
// read per workgroup, so all its threads take the same branch on it).
template <int NV>
__device__ inline void block_sums(const double *blocks, int64_t n, int stride, int k0, double out[NV],
                                  const double *flagp = nullptr, double *flag = nullptr) {
  __shared__ double wsum[4][NV];
  __shared__ double sflag;
  const int t = threadIdx.x;
  const double fl = (flagp && t == 0) ? *flagp : 0.0;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  for (int64_t b0 = 0; b0 < n; b0 += 16 * 256) {
    double x[16][NV];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t b = b0 + u * 256 + t;
#pragma unroll
      for (int k = 0; k < NV; ++k) x[u][k] = b < n ? blocks[b * stride + k0 + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int k = 0; k < NV; ++k) acc[k] += x[u][k];
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double r = wave_red_d(acc[k], false);
    if ((t & 63) == 0) wsum[t >> 6][k] = r;
  }
  if (t == 0) sflag = fl;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = ((wsum[0][k] + wsum[1][k]) + wsum[2][k]) + wsum[3][k];
  if (flag) *flag = sflag;
  __syncthreads();
}

// Per-workgroup sums (or maxima, bit k of max_mask) of NV values over 256 threads in a
// fixed order (butterfly per wave, then the four waves in order); thread 0 writes them to
// out[k].  All threads of the workgroup must call it.
template <int NV>
__device__ inline void block_write(const double v[NV], double *out, unsigned max_mask = 0u) {
  __shared__ double wsum[4][NV];
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double r = wave_red_d(v[k], (max_mask >> k) & 1u);
    if ((t & 63) == 0) wsum[t >> 6][k] = r;
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const bool mx = (max_mask >> k) & 1u;
      double r = wsum[0][k];
#pragma unroll
      for (int i = 1; i < 4; ++i) r = mx ? fmax(r, wsum[i][k]) : r + wsum[i][k];
      out[k] = r;
    }
  }
}

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
  const uint8_t *mF, *mM;       // lung masks b_F, b_M [N] (lung-boundary term)
  float *sbc;                   // boundary-term GN vectors sqrt(beta/2) grad b_M(y) [N][3], rows with rflag set
  uint8_t *rflag;               // per 64-voxel row: 1 if its boundary-term vectors are not all 0; 16 rows
                                // (4 z x 4 y voxel rows) of a wave's cell row per cell layer, together:
                                // [cz][brick x][cy][kv * 4 + jv]
  const float *zb;              // 64 x 3 zeros: read instead of sbc for rows without vectors
  float mscale, mroot;          // beta / 2, sqrt(beta / 2)
  const double *stop;           // if non-null and *stop != 0 the launch does nothing
  int acc;                      // add to out0/out1, part and blocks instead of writing them
                                // (a second pass over the same bricks, fixed order)
};

// node plane of the 2 x 2 corner nodes of a lane's cell, [j][i][c]: fb points at the
// lane's (cx, cy) node of plane 0 (node 0 for lanes outside the grid, whose values are
// discarded), poff is the uniform offset of the plane.  No branches, no 64-bit products.
__device__ __forceinline__ void load_plane(const float *fb, int64_t poff, const Geo &g, bool ok, float o[2][2][3]) {
  const float *p = fb + poff;
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float x = p[c * g.nnodes + j * g.px + i];
        o[j][i][c] = ok ? x : 0.0f;
      }
}

// ---------------------------------------------------------------------------------
// trilinear interpolation of the 8 corner values cv[z][y][x][c] at fractions t: value G
// and (JGW) the Jacobian JG[c][a] = dG_c / dy_a.  x, then y, then z; derivatives from
// differences of the lower-order interpolants.
template <bool JGW>
__device__ __forceinline__ void interp_corners(const float cv[2][2][2][3], const float t[3], const Geo &g, float G[3],
                                               float JG[3][3]) {
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
    if (JGW) {
      JG[c][0] = (dxy[0][c] + t[2] * (dxy[1][c] - dxy[0][c])) * g.ihx;
      JG[c][1] = (dyy[0][c] + t[2] * (dyy[1][c] - dyy[0][c])) * g.ihy;
      JG[c][2] = (gxy[1][c] - gxy[0][c]) * g.ihz;
    }
  }
}

// ---------------------------------------------------------------------------------
// trilinear sample of a 3-vector volume at continuous index q (zero padding): value G
// and (JGW) Jacobian JG[c][a] = dG_c / dy_a.  q is split as (integer voxel index) +
// (u/h) so that the fraction keeps full precision.  When the 8 corners of every active
// lane of the wave lie inside the volume, the corners are addressed from one 32-bit
// element offset and uniform strides without clamping or masking; otherwise corners
// outside read a clamped voxel and are discarded.
// ---------------------------------------------------------------------------------
// interp_corners for half-precision corners given as stored words: the first level (along
// x) takes the halves straight into mixed-precision multiply-adds (one rounding each, as
// in FP32 after an exact conversion), the rest is interp_corners' arithmetic
template <bool JGW>
__device__ __forceinline__ void interp_corners_h(const F16x3::raw cw[2][2][2], const float t[3], const Geo &g,
                                                 float G[3], float JG[3][3]) {
  float gx[2][2][3], dx[2][2][3];
#pragma unroll
  for (int cz = 0; cz < 2; ++cz)
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float c0 = (float)F16x3::comp(cw[cz][cy][0], c), c1 = (float)F16x3::comp(cw[cz][cy][1], c);
        dx[cz][cy][c] = c1 - c0;
        gx[cz][cy][c] = __builtin_fmaf(t[0], c1, __builtin_fmaf(-t[0], c0, c0));
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
    if (JGW) {
      JG[c][0] = (dxy[0][c] + t[2] * (dxy[1][c] - dxy[0][c])) * g.ihx;
      JG[c][1] = (dyy[0][c] + t[2] * (dyy[1][c] - dyy[0][c])) * g.ihy;
      JG[c][2] = (gxy[1][c] - gxy[0][c]) * g.ihz;
    }
  }
}

// Scaled storage: the samplers interpolate the stored values and apply the volume's
// power-of-two scale once to the result (exact, and the same as scaling every corner).
template <class ST, bool JGW>
__device__ __forceinline__ void scale_sample(float s, float G[3], float JG[3][3]) {
  if constexpr (ST::kScaled) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      G[c] *= s;
      if (JGW) {
#pragma unroll
        for (int a = 0; a < 3; ++a) JG[c][a] *= s;
      }
    }
  }
}

template <class ST, bool JGW = true>
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
  float cv[2][2][2][3];  // [z][y][x][c]
  const bool inside = (unsigned)i0[0] < (unsigned)(g.nx - 1) && (unsigned)i0[1] < (unsigned)(g.ny - 1) &&
                      (unsigned)i0[2] < (unsigned)(g.nz - 1);
  if (__all(inside)) {
    const uint32_t sy = (uint32_t)g.nx * ST::W, sz = (uint32_t)g.nx * (uint32_t)g.ny * ST::W;
    const uint32_t off = ((uint32_t)i0[2] * (uint32_t)g.ny + (uint32_t)i0[1]) * (uint32_t)g.nx * ST::W +
                         (uint32_t)i0[0] * ST::W;
    if constexpr (ST::kScaled && !JGW) {
      // value only: the halves go straight into mixed-precision multiply-adds (with the
      // Jacobian, converting each corner once for both uses measured faster)
      typename ST::raw cw[2][2][2];
#pragma unroll
      for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
          for (int cx = 0; cx < 2; ++cx)
            cw[cz][cy][cx] = ST::fetch(gT + (off + (cz ? sz : 0u) + (cy ? sy : 0u) + (cx ? (uint32_t)ST::W : 0u)));
      interp_corners_h<JGW>(cw, t, g, G, JG);
      scale_sample<ST, JGW>(sT, G, JG);
      return;
    }
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx)
          ST::loadp(gT + (off + (cz ? sz : 0u) + (cy ? sy : 0u) + (cx ? (uint32_t)ST::W : 0u)), 1.0f, cv[cz][cy][cx]);
  } else {
    const bool vx0 = (unsigned)i0[0] < (unsigned)g.nx, vx1 = (unsigned)(i0[0] + 1) < (unsigned)g.nx;
    const bool vy0 = (unsigned)i0[1] < (unsigned)g.ny, vy1 = (unsigned)(i0[1] + 1) < (unsigned)g.ny;
    const bool vz0 = (unsigned)i0[2] < (unsigned)g.nz, vz1 = (unsigned)(i0[2] + 1) < (unsigned)g.nz;
    // zero padding: corners outside the volume read a clamped voxel and are discarded
    const int X[2] = {min(max(i0[0], 0), g.nx - 1), min(max(i0[0] + 1, 0), g.nx - 1)};
    const int Y[2] = {min(max(i0[1], 0), g.ny - 1) * g.nx, min(max(i0[1] + 1, 0), g.ny - 1) * g.nx};
    const int Z[2] = {min(max(i0[2], 0), g.nz - 1) * (g.nx * g.ny), min(max(i0[2] + 1, 0), g.nz - 1) * (g.nx * g.ny)};
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
          const bool ok = (cz ? vz1 : vz0) && (cy ? vy1 : vy0) && (cx ? vx1 : vx0);
          const unsigned vi = (unsigned)(Z[cz] + Y[cy] + X[cx]);
          float t3[3];
          ST::loadp(gT + (uint64_t)vi * ST::W, 1.0f, t3);
#pragma unroll
          for (int c = 0; c < 3; ++c) cv[cz][cy][cx][c] = ok ? t3[c] : 0.0f;
        }
  }
  interp_corners<JGW>(cv, t, g, G, JG);
  scale_sample<ST, JGW>(sT, G, JG);
}

// wave-wide shift: lane i receives the value of lane i + 1; lane 63 and lanes whose
// source lane is inactive keep `old`
__device__ __forceinline__ int wave_next(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ float wave_next(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x130, 0xF, 0xF, false));
}

// corners of the previous voxel row of the same lane (rows advance by one voxel in y)
struct RowCache {
  int i0[3];
  float up[2][2][3];  // [z][x][c] at y = i0[1] + 1
  bool valid;
};

// trilinear sample for consecutive voxel rows of a lane (same x and z, y increasing):
// the same FP32 sample-cell decision and interpolation as sample_grad.  On the fast
// path (all corners of all active lanes inside the volume):
//  * the lower y row of corners is the previous row's upper one when the lane's cell
//    moved by exactly one voxel in y;
//  * lanes sample consecutive x, so lane i+1's corner x is usually lane i's corner x+1:
//    it is taken from the neighbour when the voxel indices say so.
// Which corners must be loaded depends on indices only, so every load is issued before
// any loaded value is used; the neighbour exchange follows.
template <class ST, bool JGW>
__device__ __forceinline__ void sample_grad_row(const typename ST::elem *gT, float sT, const Geo &g, int ix, int iy,
                                                int iz, const float uh[3], RowCache &rc, float G[3], float JG[3][3]) {
  const int idx[3] = {ix, iy, iz};
  const int n[3] = {g.nx, g.ny, g.nz};
  int i0[3];
  float t[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float d = fminf(fmaxf(uh[a], (float)(-2 - idx[a])), (float)(n[a] + 1 - idx[a]));
    float f = floorf(d);
    t[a] = d - f;
    i0[a] = idx[a] + (int)f;
  }
  const bool inside = (unsigned)i0[0] < (unsigned)(g.nx - 1) && (unsigned)i0[1] < (unsigned)(g.ny - 1) &&
                      (unsigned)i0[2] < (unsigned)(g.nz - 1);
  if (!__all(inside)) {
    rc.valid = false;
    sample_grad<ST, JGW>(gT, sT, g, ix, iy, iz, uh, G, JG);
    return;
  }
  const uint32_t W = ST::W;
  const int nxy = g.nx * g.ny;
  const int vid = (i0[2] * g.ny + i0[1]) * g.nx + i0[0];
  // corner rows r = y + 2 z: voxel index of corner x
  const int key[4] = {vid, vid + g.nx, vid + nxy, vid + g.nx + nxy};
  const bool reuse = rc.valid && i0[0] == rc.i0[0] && i0[1] == rc.i0[1] + 1 && i0[2] == rc.i0[2];
  bool share[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) share[r] = wave_next(key[r], key[r]) == key[r] + 1;
  float cx0[4][3], cx1[4][3];  // corners x and x+1 of row r
  // loads: rows y0 only without reuse; corner x+1 only when the neighbour cannot give it
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const bool need = (r & 1) || !reuse;
    if (need) ST::loadp(gT + (uint32_t)key[r] * W, 1.0f, cx0[r]);
    if (need && !share[r]) ST::loadp(gT + ((uint32_t)key[r] * W + W), 1.0f, cx1[r]);
  }
  float cv[2][2][2][3];  // [z][y][x][c]
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int y = r & 1, z = r >> 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float x0 = (y == 0 && reuse) ? rc.up[z][0][c] : cx0[r][c];
      const float nb = wave_next(0.0f, x0);  // neighbour's corner x (its own final value)
      const float x1 = (y == 0 && reuse) ? rc.up[z][1][c] : (share[r] ? nb : cx1[r][c]);
      cv[z][y][0][c] = x0;
      cv[z][y][1][c] = x1;
    }
  }
#pragma unroll
  for (int z = 0; z < 2; ++z)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int c = 0; c < 3; ++c) rc.up[z][x][c] = cv[z][1][x][c];
#pragma unroll
  for (int a = 0; a < 3; ++a) rc.i0[a] = i0[a];
  rc.valid = true;
  interp_corners<JGW>(cv, t, g, G, JG);
  scale_sample<ST, JGW>(sT, G, JG);
}

// ---------------------------------------------------------------------------------
// Per-cell terms, one thread per cell: volume change control (eq. 7-9, all 64
// coefficients of eq. 8) and keypoints (eq. 10).  Corner values are [k][j][i][c];
// results are corner contributions out[f][k][j][i][c] (f = 0: gradient or GN product,
// f = 1: GN diagonal), already multiplied by the term weight w.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ void cross3(const float a[3], const float b[3], float o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ float dot3(const float a[3], const float b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// edge vectors of a trilinear cell from its corner values x (+ the cell size h on the
// edge's own axis): e1[j+2k] = x_1jk - x_0jk, e2[i+2k] = x_i1k - x_i0k, e3[i+2j] = x_ij1 - x_ij0
__device__ __forceinline__ void cell_edges(const float x[2][2][2][3], float hx, float hy, float hz, float e1[4][3],
                                           float e2[4][3], float e3[4][3]) {
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        // the other components add -0, which x + (-0) = x lets the compiler drop
        e1[t + 2 * r][c] = x[r][t][1][c] - x[r][t][0][c] + (c == 0 ? hx : -0.0f);
        e2[t + 2 * r][c] = x[r][1][t][c] - x[r][0][t][c] + (c == 1 ? hy : -0.0f);
        e3[t + 2 * r][c] = x[1][r][t][c] - x[0][r][t][c] + (c == 2 ? hz : -0.0f);
      }
}

template <int MODE>
__device__ __forceinline__ void vcc_cell(const Geo &g, const float u[2][2][2][3], const float v[2][2][2][3], float w,
                                         float out[2][2][2][2][3], double &sV, int &nfold) {
  // y = X + u on the cell: e1_(j,k) = H_x e_x + u_1jk - u_0jk, and alike
  float e1[4][3], e2[4][3], e3[4][3];
  cell_edges(u, g.Hx, g.Hy, g.Hz, e1, e2, e3);
  float de1[4][3], de2[4][3], de3[4][3];
  if (MODE == M_HV) cell_edges(v, -0.0f, -0.0f, -0.0f, de1, de2, de3);
  const float iC = frcp(g.C);
  float G1[4][3] = {}, G2[4][3] = {}, G3[4][3] = {};  // dVhat/d(edge) or GN product per edge
  float D1[MODE == M_GRAD ? 4 : 1][3] = {}, D2[MODE == M_GRAD ? 4 : 1][3] = {}, D3[MODE == M_GRAD ? 4 : 1][3] = {};
#pragma unroll
  for (int c3 = 0; c3 < 4; ++c3) {
    float x23[4][3], x31[4][3];
#pragma unroll
    for (int b = 0; b < 4; ++b) cross3(e2[b], e3[c3], x23[b]);
#pragma unroll
    for (int a = 0; a < 4; ++a) cross3(e3[c3], e1[a], x31[a]);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        float x12[3];
        cross3(e1[a], e2[b], x12);
        // d_abc = det[e1_a, e2_b, e3_c] / C; terms with d <= 0 (a fold) only count
        const float d = dot3(e1[a], x23[b]) * iC;
        const bool pos = d > 0.0f;
        if (MODE != M_HV) nfold += pos ? 0 : 1;
        const float id = pos ? frcp(d) : 0.0f;
        if (MODE == M_EVAL || MODE == M_GRAD) {
          const float dm1 = d - 1.0f;
          sV += (double)(pos ? dm1 * dm1 * id : 0.0f);  // psi(d) = (d - 1)^2 / d
        }
        float coef = 0.0f;
        if (MODE == M_GRAD) coef = pos ? 1.0f - id * id : 0.0f;  // psi'(d)
        if (MODE == M_HV) {
          // psi''(d) (grad d . v), grad d . v = (de1.x23 + de2.x31 + de3.x12) / C
          const float jv = (dot3(de1[a], x23[b]) + dot3(de2[b], x31[a]) + dot3(de3[c3], x12)) * iC;
          coef = 2.0f * id * id * id * jv;
        }
        if (MODE == M_GRAD || MODE == M_HV) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            G1[a][c] += coef * x23[b][c];
            G2[b][c] += coef * x31[a][c];
            G3[c3][c] += coef * x12[c];
          }
        }
        if (MODE == M_GRAD) {
          // GN diagonal: C psi''(d) (dd/dy_n)^2, dd/dy_n = (sum over the edges of this term
          // through corner n of +-(cross product of the other two edges)) / C.  The square
          // splits into per-edge squares (accumulated per edge) and cross products of two
          // edges at their shared corner (which exists iff the indices below agree).
          const float p2 = 2.0f * id * id * id * w * iC;
          const int ja = a & 1, ka = a >> 1, ib = b & 1, kb = b >> 1, ic = c3 & 1, jc = c3 >> 1;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            D1[a][c] += p2 * x23[b][c] * x23[b][c];
            D2[b][c] += p2 * x31[a][c] * x31[a][c];
            D3[c3][c] += p2 * x12[c] * x12[c];
          }
          if (ka == kb) {  // e1_a and e2_b meet at corner (ib, ja, ka)
            const float sg = (ib ? 2.0f : -2.0f) * (ja ? 1.0f : -1.0f) * p2;
#pragma unroll
            for (int c = 0; c < 3; ++c) out[1][ka][ja][ib][c] += sg * x23[b][c] * x31[a][c];
          }
          if (ja == jc) {  // e1_a and e3_c meet at corner (ic, ja, ka)
            const float sg = (ic ? 2.0f : -2.0f) * (ka ? 1.0f : -1.0f) * p2;
#pragma unroll
            for (int c = 0; c < 3; ++c) out[1][ka][ja][ic][c] += sg * x23[b][c] * x12[c];
          }
          if (ib == ic) {  // e2_b and e3_c meet at corner (ib, jc, kb)
            const float sg = (jc ? 2.0f : -2.0f) * (kb ? 1.0f : -1.0f) * p2;
#pragma unroll
            for (int c = 0; c < 3; ++c) out[1][kb][jc][ib][c] += sg * x31[a][c] * x12[c];
          }
        }
      }
  }
  if (MODE == M_GRAD) {
    // per-edge squares to both corners of the edge
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) out[1][k][j][i][c] += D1[j + 2 * k][c] + D2[i + 2 * k][c] + D3[i + 2 * j][c];
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
            const float acc = (i ? G1[j + 2 * k][c] : -G1[j + 2 * k][c]) + (j ? G2[i + 2 * k][c] : -G2[i + 2 * k][c]) +
                              (k ? G3[i + 2 * j][c] : -G3[i + 2 * j][c]);
            out[0][k][j][i][c] += w * acc;
          }
  }
}

// GN product of the volume-change term for one cell: out = w C sum_t psi''(d_t)
// (grad d_t . v) grad d_t over the 64 coefficients d_abc = det[e1_a, e2_b, e3_c] / C.
// For fixed (b, c) the cross product x = e2_b x e3_c / C is shared by the four a, and
// grad d . v = de1_a . x + e1_a . y with y = (de2_b x e3_c + e2_b x de3_c) / C.  The
// derivatives with respect to e2_b and e3_c are (e3_c x e1_a) / C and (e1_a x e2_b) / C,
// so their sums over a collapse to one cross product with z = sum_a k_a e1_a.
__device__ __forceinline__ void vcc_cell_hv(const Geo &g, const float u[2][2][2][3], const float v[2][2][2][3],
                                            float w, float out[2][2][2][3]) {
  float e1[4][3], e2[4][3], e3[4][3];
  cell_edges(u, g.Hx, g.Hy, g.Hz, e1, e2, e3);
  float de1[4][3], de2[4][3], de3[4][3];
  cell_edges(v, -0.0f, -0.0f, -0.0f, de1, de2, de3);
  const float iC = frcp(g.C);
  // k = w C psi''(d) (grad d . v) = 2 w C id^3 jv.  The factor w2 = 2 w C is put into the
  // v edges and 1/C into the z edges, so that x = e2 x e3' and y = de2' x e3' + e2 x de3'
  // come out scaled as needed without per-term multiplications.
  const float w2 = 2.0f * w * g.C;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      de1[a][c] *= w2;
      de2[a][c] *= w2;
      de3[a][c] *= w2 * iC;
      e3[a][c] *= iC;
    }
  // accumulators start at -0, for which x + (-0) = x exactly: the first multiply-add of each
  // then compiles to a plain multiply (a +0 start costs an extra addition)
  float G1[4][3], G2[4][3], G3[4][3];  // G3 is accumulated times C
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) G1[a][c] = G2[a][c] = G3[a][c] = -0.0f;
#pragma unroll
  for (int c3 = 0; c3 < 4; ++c3)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      float x[3], y[3];
      cross3(e2[b], e3[c3], x);  // e2 x e3 / C
      // y = w2 (de2 x e3 + e2 x de3) / C, as one fused chain per component
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        float acc = de2[b][c1] * e3[c3][c2];
        acc = __builtin_fmaf(-de2[b][c2], e3[c3][c1], acc);
        acc = __builtin_fmaf(e2[b][c1], de3[c3][c2], acc);
        y[c] = __builtin_fmaf(-e2[b][c2], de3[c3][c1], acc);
      }
      float z[3] = {-0.0f, -0.0f, -0.0f};
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        // d less the smallest normal float, so that d <= 0 (a fold, whose term does not
        // count) gives a negative reciprocal and the maximum with zero drops it; for
        // 0 < d < 1e-13 the cube of 1/d overflows in FP32 either way
        const float d = __builtin_fmaf(e1[a][2], x[2], __builtin_fmaf(e1[a][1], x[1], __builtin_fmaf(e1[a][0], x[0], -FLT_MIN)));
        float jv = dot3(de1[a], x);
#pragma unroll
        for (int c = 0; c < 3; ++c) jv = __builtin_fmaf(e1[a][c], y[c], jv);
        const float id = fmaxf(frcp(d), 0.0f);
        const float k = id * id * id * jv;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          G1[a][c] = __builtin_fmaf(k, x[c], G1[a][c]);
          z[c] = __builtin_fmaf(k, e1[a][c], z[c]);
        }
      }
      // G2 += e3' x z, G3 += z x e2 (fused into the accumulators)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        G2[b][c] = __builtin_fmaf(e3[c3][c1], z[c2], G2[b][c]);
        G2[b][c] = __builtin_fmaf(-e3[c3][c2], z[c1], G2[b][c]);
        G3[c3][c] = __builtin_fmaf(z[c1], e2[b][c2], G3[c3][c]);
        G3[c3][c] = __builtin_fmaf(-z[c2], e2[b][c1], G3[c3][c]);
      }
    }
  // edges -> corners: +G on the far node of the edge, -G on the near node
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          out[k][j][i][c] = (i ? G1[j + 2 * k][c] : -G1[j + 2 * k][c]) + (j ? G2[i + 2 * k][c] : -G2[i + 2 * k][c]) +
                            (k ? iC * G3[i + 2 * j][c] : -iC * G3[i + 2 * j][c]);
}

template <int MODE>
__device__ __forceinline__ void kp_cell(const Geo &g, int ks, int ke, const float *kloc, const float *ktgt,
                                        const float u[2][2][2][3], const float v[2][2][2][3], float w,
                                        float out[2][2][2][2][3], double &sK) {
  for (int kk = ks; kk < ke; ++kk) {
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
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float acc = MODE == M_HV ? 0.0f : xl[c];
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int i = 0; i < 2; ++i) acc += wt[k][j][i] * (MODE == M_HV ? v[k][j][i][c] : u[k][j][i][c]);
      if (MODE == M_HV) {
        val[c] = 2.0f * w * acc;  // 2 delta (P v)(x_i)
      } else {
        const float res = acc - tl[c];  // y(x_i) - y_KP(x_i), relative to the cell origin
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

// the 8 corner values of a cell, [k][j][i][c]; fb points at the cell's (0,0,0) corner
// (node 0 for threads outside the grid, whose values are discarded)
__device__ __forceinline__ void load_corners(const float *fb, const Geo &g, bool ok, float o[2][2][2][3]) {
  const int64_t pxy = (int64_t)g.px * g.py;
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float x = fb[c * g.nnodes + k * pxy + j * g.px + i];
          o[k][j][i][c] = ok ? x : 0.0f;
        }
}

// ---------------------------------------------------------------------------------
// The voxel-brick kernel.
// ---------------------------------------------------------------------------------
// unrolling of the voxel rows (y) and layers (z) of a cell in the objective pass
#ifndef DISCO_EVAL_JV
#define DISCO_EVAL_JV 4
#endif
#ifndef DISCO_EVAL_KV
#define DISCO_EVAL_KV 1
#endif
#ifndef DISCO_HV_WAVES
#define DISCO_HV_WAVES 1
#endif
// Trilinear sample of the moving lung mask (uint8 0/1, zero outside the volume) at the
// warped voxel, in the same cell as the gradient sample (same FP32 decision), and the
// gradient of the interpolant in mm.
__device__ __forceinline__ void sample_mask(const uint8_t *__restrict__ mM, const Geo &g, int ix, int iy, int iz,
                                            const float uh[3], float &val, float grad[3]) {
  const int idx[3] = {ix, iy, iz};
  const int n[3] = {g.nx, g.ny, g.nz};
  int i0[3];
  float t[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float d = fminf(fmaxf(uh[a], (float)(-2 - idx[a])), (float)(n[a] + 1 - idx[a]));
    const float f = floorf(d);
    t[a] = d - f;
    i0[a] = idx[a] + (int)f;
  }
  float m[2][2][2];  // [z][y][x]
#pragma unroll
  for (int cz = 0; cz < 2; ++cz)
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) {
        const int ii = i0[0] + cx, jj = i0[1] + cy, kk = i0[2] + cz;
        const bool in = (unsigned)ii < (unsigned)g.nx && (unsigned)jj < (unsigned)g.ny && (unsigned)kk < (unsigned)g.nz;
        const int64_t off = in ? ((int64_t)kk * g.ny + jj) * g.nx + ii : 0;
        const uint8_t b = mM[off];
        m[cz][cy][cx] = in ? (float)b : 0.0f;
      }
  // along x, then y, then z
  float ax[2][2], dx[2][2];
#pragma unroll
  for (int cz = 0; cz < 2; ++cz)
#pragma unroll
    for (int cy = 0; cy < 2; ++cy) {
      dx[cz][cy] = m[cz][cy][1] - m[cz][cy][0];
      ax[cz][cy] = m[cz][cy][0] + t[0] * dx[cz][cy];
    }
  float ay[2], dyv[2], dxy[2];
#pragma unroll
  for (int cz = 0; cz < 2; ++cz) {
    dyv[cz] = ax[cz][1] - ax[cz][0];
    ay[cz] = ax[cz][0] + t[1] * dyv[cz];
    dxy[cz] = dx[cz][0] + t[1] * (dx[cz][1] - dx[cz][0]);
  }
  val = ay[0] + t[2] * (ay[1] - ay[0]);
  grad[0] = (dxy[0] + t[2] * (dxy[1] - dxy[0])) * g.ihx;
  grad[1] = (dyv[0] + t[2] * (dyv[1] - dyv[0])) * g.ihy;
  grad[2] = (ay[1] - ay[0]) * g.ihz;
}

// MASK adds the lung-boundary term (eq. 6) to the voxel pass: it needs NGF (the voxel
// pass of the data terms)
template <class ST, int MODE, bool NGF, bool VCC, bool KP, int ZC, bool MASK = false, bool NOSPLIT = false>
__device__ __forceinline__ void brick_body(const BrickArgs<ST> &A, const Blk &B, int acc) {
  static_assert(!MASK || NGF, "the boundary term rides on the voxel pass");
  constexpr int F = (MODE == M_GRAD) ? 2 : ((MODE == M_HV) ? 1 : 0);
  constexpr int FS = F > 0 ? F : 1;
  constexpr bool CELLT = VCC || KP;
  constexpr bool NGF_OUT = NGF && F > 0;
  constexpr bool CELL_OUT = CELLT && F > 0;
  // NGF node planes of the brick, staged per wave: [plane][wave][jn][field*3+c][A/B][quad]
  __shared__ float lds[NGF_OUT ? ZC + 1 : 1][4][2][FS * 3][2][16];
  // per-cell corner contributions: [field*24 + corner*3 + c][cell of the brick]
  __shared__ float cbuf[CELL_OUT ? FS * 24 : 1][CELL_OUT ? 64 * ZC : 1];
  __shared__ double lred[4][BS_N];

  if (A.stop && *A.stop != 0.0) return;
  const Geo &g = A.g;
  constexpr int WGS = NOSPLIT ? 256 : brick_threads<MODE, NGF, CELLT>();
  constexpr bool SPLIT = WGS != 256;
  constexpr int NCW = SPLIT ? kCellWaves : 4;  // waves that take cell layers
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cw = SPLIT ? wave - 4 : wave;  // index among the waves that compute cell terms
  const int q = lane & 3, xq = lane >> 2;
  const int bx = B.x, by = B.y, bz = B.z;
  const int ix = bx * 64 + lane;
  const int cx = ix >> 2;
  const int cy = by * kBYC + wave;
  const int cz0 = bz * ZC;
  const int cz1 = min(cz0 + ZC, g.cz);
  const bool ok = (cx < g.cx) && (cy < g.cy);
  const float xi = (q + 0.5f) * 0.25f;
  const int64_t brick = ((int64_t)bz * g.nby + by) * g.nbx + bx;
  const int64_t pxy = (int64_t)g.px * g.py;
  const int64_t nxy = (int64_t)g.nx * g.ny;

  double sD = 0.0, sV = 0.0, sK = 0.0, sB = 0.0;
  int nfold = 0;
  const float sc_ngf = A.ngf_scale;
  const float sg0 = (MODE == M_GRAD) ? -sc_ngf : sc_ngf;  // field 0: -2h^3 r s (gradient) or 2h^3 (GN)
  const float wA0 = (1.0f - xi) * sg0, wB0 = xi * sg0;
  const float wA1 = (1.0f - xi) * (1.0f - xi) * sc_ngf, wB1 = xi * xi * sc_ngf;

  // stage NGF node plane zl of this wave: x-reduce over the quad (A: node cx, B: node cx+1)
  auto stage = [&](int zl, const float nv[FS][2][3]) {
    if constexpr (NGF_OUT) {
#pragma unroll
      for (int f = 0; f < F; ++f) {
        const float wA = f == 0 ? wA0 : wA1;  // field 1 (diagonal) uses squared weights
        const float wB = f == 0 ? wB0 : wB1;
#pragma unroll
        for (int jn = 0; jn < 2; ++jn)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float a = quad_sum(nv[f][jn][c] * wA);
            const float b = quad_sum(nv[f][jn][c] * wB);
            if (q == 0) {
              lds[zl][wave][jn][f * 3 + c][0][xq] = a;
              lds[zl][wave][jn][f * 3 + c][1][xq] = b;
            }
          }
      }
    }
  };

  // voxel part (NGF): node values rolled along z, layer by layer
  auto ngf_phase = [&]() {
    if constexpr (NGF) {
      // NGF: node values of this lane's cell, rolled along z: [k][j][i][c] (u, or v for M_HV)
      float nc[2][2][2][3];
      const float *NF = (MODE == M_HV) ? A.v : A.u;
      const float *NB = NF + (ok ? (int64_t)cy * g.px + cx : 0);
      if (NGF) {
        float tmp[2][2][3];
        load_plane(NB, (int64_t)cz0 * pxy, g, ok, tmp);
    #pragma unroll
        for (int j = 0; j < 2; ++j)
    #pragma unroll
          for (int i = 0; i < 2; ++i)
    #pragma unroll
            for (int c = 0; c < 3; ++c) nc[0][j][i][c] = tmp[j][i][c];
      }

      float carN[FS][2][3] = {};  // NGF, per lane before the x reduction: [f][jn][c]
      for (int czi = cz0; czi < cz1; ++czi) {
        const int zl = czi - cz0;
        float accN[FS][2][2][3] = {};  // [f][kn][jn][c]
        if (NGF) {
          {
            float tmp[2][2][3];
            load_plane(NB, (int64_t)(czi + 1) * pxy, g, ok, tmp);
    #pragma unroll
            for (int j = 0; j < 2; ++j)
    #pragma unroll
              for (int i = 0; i < 2; ++i)
    #pragma unroll
                for (int c = 0; c < 3; ++c) nc[1][j][i][c] = tmp[j][i][c];
          }
          if (ok) {
            // node values interpolated along x at this lane's voxel: fx[k][j][c]
            float fx[2][2][3];
    #pragma unroll
            for (int k = 0; k < 2; ++k)
    #pragma unroll
              for (int j = 0; j < 2; ++j)
    #pragma unroll
                for (int c = 0; c < 3; ++c) fx[k][j][c] = __builtin_fmaf(xi, nc[k][j][1][c] - nc[k][j][0][c], nc[k][j][0][c]);
            // first voxel of this lane in the layer; voxel (kv, jv) is vbase + kv*nx*ny + jv*nx,
            // the offset being the same for the whole wave
            const int64_t vbase = ((int64_t)(czi * 4) * g.ny + cy * 4) * g.nx + ix;
            // boundary-term row flags of this layer (16 bytes, one load)
            uint32_t mflags[4] = {0u, 0u, 0u, 0u};
            if constexpr (MASK && MODE == M_HV) {
              const uint4 f4 = *reinterpret_cast<const uint4 *>(A.rflag + (((int64_t)czi * g.nbx + bx) * g.cy + cy) * 16);
              mflags[0] = f4.x;
              mflags[1] = f4.y;
              mflags[2] = f4.z;
              mflags[3] = f4.w;
            }
            const typename ST::elem *sp = A.sc + vbase * ST::W;
            const typename ST::elem *rp = A.gR + vbase * ST::W;
            // GN product: the layer's 16 s rows are requested before the first is used, so
            // that a wave keeps 12 KB in flight (the scheduler otherwise interleaves loads and
            // arithmetic and keeps only a few rows outstanding)
            typename ST::raw srow[(MODE == M_HV && !MASK) ? 4 : 1][4];
            if constexpr (MODE == M_HV && !MASK) {
    #pragma unroll
              for (int kv = 0; kv < 4; ++kv)
    #pragma unroll
                for (int jv = 0; jv < 4; ++jv) srow[kv][jv] = ST::fetch(sp + (kv * nxy + jv * g.nx) * ST::W);
              __builtin_amdgcn_sched_barrier(0);
            }
            auto zrow = [&](const int kv) {
              const float wz = (kv + 0.5f) * 0.25f;
              const int iz = czi * 4 + kv;
              float fz[2][3];
    #pragma unroll
              for (int j = 0; j < 2; ++j)
    #pragma unroll
                for (int c = 0; c < 3; ++c) fz[j][c] = __builtin_fmaf(wz, fx[1][j][c] - fx[0][j][c], fx[0][j][c]);
              float accY[FS][2][3] = {};
              RowCache rc;
              rc.valid = false;
    #pragma unroll (MODE == M_HV ? 4 : (MODE == M_EVAL ? DISCO_EVAL_JV : 1))
              for (int jv = 0; jv < 4; ++jv) {
                const float wy = (jv + 0.5f) * 0.25f;
                const int iy = cy * 4 + jv;
                const int64_t voff = (kv * nxy + jv * g.nx) * ST::W;  // wave-uniform
                float f3[3];
    #pragma unroll
                for (int c = 0; c < 3; ++c) f3[c] = __builtin_fmaf(wy, fz[1][c] - fz[0][c], fz[0][c]);
                if (MODE == M_HV) {
                  float s[3];
                  if constexpr (MASK)
                    ST::loadp(sp + voff, A.sS_load, s);
                  else
                    ST::unpack(srow[kv][jv], sp + voff, A.sS_load, s);
                  // moments over the row's voxels: accY[0][0] collects sum w s and accY[0][1]
                  // sum wy w s; the lower node's share, sum (1 - wy) w s, is their difference
                  const float w = s[0] * f3[0] + s[1] * f3[1] + s[2] * f3[2];
                  const float ww = wy * w;
    #pragma unroll
                  for (int c = 0; c < 3; ++c) {
                    accY[0][0][c] = __builtin_fmaf(w, s[c], accY[0][0][c]);
                    accY[0][1][c] = __builtin_fmaf(ww, s[c], accY[0][1][c]);
                  }
                  if constexpr (MASK) {
                    // boundary term: only rows that touch the mask boundary carry vectors; the
                    // others read a small zero buffer (cache hits), so that the loads need no
                    // branch and issue with the s loads
                    const bool fl = ((mflags[kv] >> (8 * jv)) & 0xffu) != 0u;
                    const float *bp = fl ? A.sbc + (vbase + kv * nxy + jv * g.nx) * 3 : A.zb + lane * 3;
                    const float sb[3] = {bp[0], bp[1], bp[2]};
                    const float wb = sb[0] * f3[0] + sb[1] * f3[1] + sb[2] * f3[2];
                    const float wwb = wy * wb;
    #pragma unroll
                    for (int c = 0; c < 3; ++c) {
                      accY[0][0][c] = __builtin_fmaf(wb, sb[c], accY[0][0][c]);
                      accY[0][1][c] = __builtin_fmaf(wwb, sb[c], accY[0][1][c]);
                    }
                  }
                } else {
                  // displacement in voxel units: q = index + u/h.  The displacement is interpolated
                  // in a fixed order (x, then z, then y, one fused multiply-add each) so that the
                  // cell holding the sample point is a reproducible FP32 decision.
                  const float uh[3] = {f3[0] * g.ihx, f3[1] * g.ihy, f3[2] * g.ihz};
                  float a[3], JG[3][3], b[3];
                  // objective pass: row sampler (shared corners) in FP32 storage; gradient pass
                  // and half-precision storage: plain sampler (measured faster there)
                  if constexpr (MODE == M_EVAL && !ST::kScaled)
                    sample_grad_row<ST, false>(A.gT, A.sT, g, ix, iy, iz, uh, rc, a, JG);
                  else if constexpr (MODE == M_EVAL)
                    sample_grad<ST, false>(A.gT, A.sT, g, ix, iy, iz, uh, a, JG);
                  else
                    sample_grad<ST, true>(A.gT, A.sT, g, ix, iy, iz, uh, a, JG);
                  ST::loadp(rp + voff, A.sR, b);
                  const float e2 = A.eta2;
                  const float Da = e2 + a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
                  const float Db = e2 + b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
                  const float P = e2 + a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
                  const float dab[3] = {a[0] - b[0], a[1] - b[1], a[2] - b[2]};
                  float axb[3];
                  cross3(a, b, axb);
                  const float DD = Da * Db;
                  // 1 - r^2 without cancellation (Lagrange's identity)
                  const float cvox = (e2 * dot3(dab, dab) + dot3(axb, axb)) * frcp(DD);
                  sD += (double)cvox;
                  if (MODE == M_GRAD) {
                    const float isq = rsqrtf(DD);
                    const float r = P * isq;
                    const float pda = P * frcp(Da);
                    float dr[3], s[3];
    #pragma unroll
                    for (int c = 0; c < 3; ++c) dr[c] = (b[c] - pda * a[c]) * isq;
    #pragma unroll
                    for (int c = 0; c < 3; ++c) s[c] = JG[0][c] * dr[0] + JG[1][c] * dr[1] + JG[2][c] * dr[2];
                    ST::storep(const_cast<typename ST::elem *>(sp) + voff, A.sS_store, s);
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
                  if constexpr (MASK) {
                    // lung-boundary term: res = b_M(y) - b_F(x), B += res^2 (times h^3 / 2 later)
                    float bm, gb[3];
                    sample_mask(A.mM, g, ix, iy, iz, uh, bm, gb);
                    const int64_t vi = vbase + kv * nxy + jv * g.nx;
                    const float res = bm - (float)A.mF[vi];
                    sB += (double)(res * res);
                    if (MODE == M_GRAD) {
                      // in units of the NGF fields: gradient -2h^3 (-(beta/2) res grad b),
                      // diagonal 2h^3 (beta/2) grad b^2, GN vector sqrt(beta/2) grad b
                      const bool nz = gb[0] != 0.0f || gb[1] != 0.0f || gb[2] != 0.0f;
                      const bool row = __any(nz);
                      if (row) {
                        float *bp = A.sbc + vi * 3;
    #pragma unroll
                        for (int c = 0; c < 3; ++c) bp[c] = A.mroot * gb[c];
                      }
                      if (lane == 0) A.rflag[(((int64_t)czi * g.nbx + bx) * g.cy + cy) * 16 + kv * 4 + jv] = row ? 1 : 0;
    #pragma unroll
                      for (int c = 0; c < 3; ++c) {
                        const float t = -A.mscale * res * gb[c];
                        accY[0][0][c] += (1.0f - wy) * t;
                        accY[0][1][c] += wy * t;
                        const float t2 = A.mscale * gb[c] * gb[c];
                        accY[FS - 1][0][c] += (1.0f - wy) * (1.0f - wy) * t2;
                        accY[FS - 1][1][c] += wy * wy * t2;
                      }
                    }
                  }
                }
              }
              if constexpr (MODE == M_HV) {
    #pragma unroll
                for (int c = 0; c < 3; ++c) accY[0][0][c] -= accY[0][1][c];
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
    #pragma unroll (MODE == M_EVAL ? DISCO_EVAL_KV : 1)
              for (int kv = 0; kv < 4; ++kv) zrow(kv);
            }
          }
        }

        if (NGF_OUT) {
          // node plane czi is complete: carried part + this layer's lower plane
          float nv[FS][2][3];
    #pragma unroll
          for (int f = 0; f < FS; ++f)
    #pragma unroll
            for (int jn = 0; jn < 2; ++jn)
    #pragma unroll
              for (int c = 0; c < 3; ++c) {
                nv[f][jn][c] = carN[f][jn][c] + accN[f][0][jn][c];
                carN[f][jn][c] = accN[f][1][jn][c];
              }
          stage(zl, nv);
        }
        if (NGF) {
          // roll the node values
    #pragma unroll
          for (int j = 0; j < 2; ++j)
    #pragma unroll
            for (int i = 0; i < 2; ++i)
    #pragma unroll
              for (int c = 0; c < 3; ++c) nc[0][j][i][c] = nc[1][j][i][c];
        }
      }

      // last node plane of the brick: the carried part alone
      if constexpr (NGF_OUT) stage(cz1 - cz0, carN);
    }
  };

  auto cell_phase = [&]() {
    // cell terms (volume change, keypoints), after the voxel layers so that their registers
    // do not add to the rolling NGF state: wave w takes cell layers w, w + 4, ..., one cell
    // per lane
    if (CELLT) {
      for (int zl = cw; zl < cz1 - cz0; zl += NCW) {
        const int czi = cz0 + zl;
        const int lx = lane & 15, ly = lane >> 4;
        const int ccx = bx * kBXC + lx, ccy = by * kBYC + ly;
        const bool cok = ccx < g.cx && ccy < g.cy;
        const int64_t cbase = cok ? (int64_t)czi * pxy + (int64_t)ccy * g.px + ccx : 0;
        float *cb = &cbuf[0][0] + zl * 64 + lane;  // this cell's column of cbuf (stride 64 * ZC)
        constexpr int CS = CELL_OUT ? 64 * ZC : 0;
        if constexpr (MODE == M_HV) {
          // the product: volume change first, written out, then the (rare) keypoint cells
          // add to it, so that no accumulator is live across the volume-change code
          {
            float ct[2][2][2][3] = {};
            if (VCC) {
              float ucor[2][2][2][3], vcor[2][2][2][3];
              load_corners(A.u + cbase, g, cok, ucor);
              load_corners(A.v + cbase, g, cok, vcor);
              if (cok) vcc_cell_hv(g, ucor, vcor, A.gamma, ct);
            }
  #pragma unroll
            for (int k = 0; k < 2; ++k)
  #pragma unroll
              for (int j = 0; j < 2; ++j)
  #pragma unroll
                for (int i = 0; i < 2; ++i)
  #pragma unroll
                  for (int c = 0; c < 3; ++c) cb[((i + 2 * j + 4 * k) * 3 + c) * CS] = ct[k][j][i][c];
          }
        } else {
          float ucor[2][2][2][3], vcor[2][2][2][3];
          load_corners(A.u + cbase, g, cok, ucor);
          float ct[FS][2][2][2][3] = {};
          if (cok) {
            if (VCC) vcc_cell<MODE>(g, ucor, vcor, A.gamma, ct, sV, nfold);
            if (KP) {
              const int64_t cell = ((int64_t)czi * g.cy + ccy) * g.cx + ccx;
              const int ks = A.kstart[cell], ke = A.kstart[cell + 1];
              if (ke > ks) kp_cell<MODE>(g, ks, ke, A.kloc, A.ktgt, ucor, vcor, A.delta, ct, sK);
            }
          }
          if constexpr (CELL_OUT) {
  #pragma unroll
            for (int f = 0; f < F; ++f)
  #pragma unroll
              for (int k = 0; k < 2; ++k)
  #pragma unroll
                for (int j = 0; j < 2; ++j)
  #pragma unroll
                  for (int i = 0; i < 2; ++i)
  #pragma unroll
                    for (int c = 0; c < 3; ++c) cb[(f * 24 + (i + 2 * j + 4 * k) * 3 + c) * CS] = ct[f][k][j][i][c];
          }
        }
      }
    }

    // HV keypoint cells (rare) in a pass of their own, adding to the volume-change result
    if constexpr (MODE == M_HV && KP) {
      for (int zl = cw; zl < cz1 - cz0; zl += NCW) {
        const int czi = cz0 + zl;
        const int ccx = bx * kBXC + (lane & 15), ccy = by * kBYC + (lane >> 4);
        if (ccx < g.cx && ccy < g.cy) {
          const int64_t cell = ((int64_t)czi * g.cy + ccy) * g.cx + ccx;
          const int ks = A.kstart[cell], ke = A.kstart[cell + 1];
          if (ke > ks) {
            float vcor[2][2][2][3];
            load_corners(A.v + (int64_t)czi * pxy + (int64_t)ccy * g.px + ccx, g, true, vcor);
            float kt[1][2][2][2][3] = {};
            kp_cell<MODE>(g, ks, ke, A.kloc, A.ktgt, vcor, vcor, A.delta, kt, sK);
            float *cb = &cbuf[0][0] + zl * 64 + lane;
  #pragma unroll
            for (int k = 0; k < 2; ++k)
  #pragma unroll
              for (int j = 0; j < 2; ++j)
  #pragma unroll
                for (int i = 0; i < 2; ++i)
  #pragma unroll
                  for (int c = 0; c < 3; ++c) cb[((i + 2 * j + 4 * k) * 3 + c) * 64 * ZC] += kt[0][k][j][i][c];
          }
        }
      }
    }

  };

  if constexpr (SPLIT) {
    if (wave < 4)
      ngf_phase();
    else
      cell_phase();
  } else {
    ngf_phase();
    cell_phase();
  }

  if constexpr (F > 0) {
    const int nl = cz1 - cz0;  // cell layers of this brick
    __syncthreads();
    // combine in a fixed order and write every node plane of the brick: interior nodes
    // directly, brick-face nodes to the partial buffer.  One thread per node of the brick's
    // (nl + 1) x 5 x 17 box, all fields and components in turn, so that the node's position,
    // its neighbour tests and its destination are worked out once.
    for (int e = threadIdx.x; e < (nl + 1) * kNBOX; e += WGS) {
      const int zl = e / kNBOX, pos = e - zl * kNBOX;
      const int yl = pos / 17, xl = pos - yl * 17;
      const int pxn = bx * kBXC + xl, pyn = by * kBYC + yl, pzn = cz0 + zl;
      if (pxn > g.cx || pyn > g.cy) continue;
      const bool face = is_face(zl, bz, g.nbz, ZC) || is_face(xl, bx, g.nbx, kBXC) || is_face(yl, by, g.nby, kBYC);
      float *pp = A.part + (brick * (ZC + 1) + zl) * (F * 3) * kNBOX + pos;
      const int64_t node = ((int64_t)pzn * g.py + pyn) * g.px + pxn;
#pragma unroll
      for (int fc = 0; fc < F * 3; ++fc) {
        const int f = fc / 3, c = fc - 3 * f;
        float val = 0.0f;
        if (NGF_OUT) {
          if (yl < 4) {
            if (xl < 16) val += lds[zl][yl][0][fc][0][xl];
            if (xl > 0) val += lds[zl][yl][0][fc][1][xl - 1];
          }
          if (yl > 0) {
            if (xl < 16) val += lds[zl][yl - 1][1][fc][0][xl];
            if (xl > 0) val += lds[zl][yl - 1][1][fc][1][xl - 1];
          }
        }
        if (CELL_OUT) {
#pragma unroll
          for (int dk = 0; dk < 2; ++dk)
#pragma unroll
            for (int dj = 0; dj < 2; ++dj)
#pragma unroll
              for (int di = 0; di < 2; ++di) {
                // cell (xl-1+di, yl-1+dj, zl-1+dk) touches this node at its corner (1-di, 1-dj, 1-dk)
                const int ci = xl - 1 + di, cj = yl - 1 + dj, ck = zl - 1 + dk;
                if (ci < 0 || ci >= 16 || cj < 0 || cj >= 4 || ck < 0 || ck >= nl) continue;
                const int corner = (1 - di) + 2 * (1 - dj) + 4 * (1 - dk);
                val += cbuf[f * 24 + corner * 3 + c][ck * 64 + cj * 16 + ci];
              }
        }
        if (face) {
          float *q = pp + fc * kNBOX;
          *q = acc ? *q + val : val;
        } else {
          float *po = (f == 0 ? A.out0 : A.out1) + c * g.nnodes + node;
          *po = acc ? *po + val : val;
        }
      }
    }
  }

  // workgroup scalars in a fixed order
  if (MODE != M_HV) {
    double vals[BS_N] = {sD, sV * (double)g.C, sK, (double)nfold, sB};
#pragma unroll
    for (int t = 0; t < BS_N; ++t) {
      const double s = wave_sum_d(vals[t]);
      if (lane == 0) lred[wave][t] = s;
    }
    __syncthreads();
    if (threadIdx.x < BS_N) {
      const int t = threadIdx.x;
      const int64_t wg = B.lin;
      const double v = ((lred[0][t] + lred[1][t]) + lred[2][t]) + lred[3][t];
      A.blocks[wg * BS_N + t] = acc ? A.blocks[wg * BS_N + t] + v : v;
    }
  }
}

template <class ST, int MODE, bool NGF, bool VCC, bool KP, int ZC, bool MASK = false>
__global__ __launch_bounds__((brick_threads<MODE, NGF, VCC || KP>()), MODE == M_HV ? DISCO_HV_WAVES : 1) void k_brick(
    BrickArgs<ST> A) {
  brick_body<ST, MODE, NGF, VCC, KP, ZC, MASK>(A, hw_blk(), A.acc);
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
  double *blocks;        // [nblocks][3]: <dotv,out0>, max(out1), <out0,out0>
  const double *stop;
};

__device__ __forceinline__ int chi(int p, int n) { return (p >= 1 && p <= n - 2) ? 1 : 0; }


// F: fields the brick kernel wrote (0: none ran), NF: fields produced (1 or 2),
// CURV: add curvature (field 0, and its diagonal to field 1 when NF = 2)
template <int ZC, int F, int NF, bool CURV>
__device__ __forceinline__ void gather_body(const GatherArgs &A, const Blk &B) {
  // read with the other loads; only the writes wait for it (no workgroup writes it here)
  const bool stopped = A.stop && *A.stop != 0.0;
  const Geo &g = A.g;
  const float *__restrict__ part = A.part;
  const float *__restrict__ Lw = A.Lw;
  const float *__restrict__ tauv = A.tauv;
  const float *__restrict__ dotv = A.dotv;
  float *__restrict__ out0 = A.out0;
  float *__restrict__ out1 = A.out1;
  // block (64 x 4 threads) covers nodes x in [64 bx, 64 bx + 64), y in [4 by, 4 by + 4), plane bz
  const int px = B.x * 64 + (threadIdx.x & 63), py = B.y * 4 + (threadIdx.x >> 6), pz = B.z;
  const int64_t bid = B.lin;
  double dsum = 0.0, dmax = 0.0, gsq = 0.0;
  if (px < g.px && py < g.py) {
    const int64_t n = ((int64_t)pz * g.py + py) * g.px + px;
    float val[NF][3];
    // brick kernel part: interior nodes were written directly, face nodes are summed here
    if (F > 0) {
      // the (at most two) bricks per axis whose box holds this node, in increasing order;
      // fixed-size candidate lists so that nothing is indexed dynamically
      const int pcoord[3] = {px, py, pz};
      const int BB[3] = {kBXC, kBYC, ZC};
      const int NB[3] = {g.nbx, g.nby, g.nbz};
      int cb[3][2], cl[3][2];
      bool cok[3][2];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int bb = pcoord[a] / BB[a] - 1 + k;
          const int ll = pcoord[a] - bb * BB[a];
          cb[a][k] = bb;
          cl[a][k] = ll;
          cok[a][k] = bb >= 0 && bb < NB[a] && ll >= 0 && ll <= BB[a];
        }
      const bool face = (cok[0][0] && cok[0][1]) || (cok[1][0] && cok[1][1]) || (cok[2][0] && cok[2][1]);
      if (face) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int c = 0; c < 3; ++c) val[f][c] = 0.0f;
#pragma unroll
        for (int iz = 0; iz < 2; ++iz)
#pragma unroll
          for (int iy = 0; iy < 2; ++iy)
#pragma unroll
            for (int ixx = 0; ixx < 2; ++ixx) {
              if (!(cok[2][iz] && cok[1][iy] && cok[0][ixx])) continue;
              const int64_t brick = ((int64_t)cb[2][iz] * g.nby + cb[1][iy]) * g.nbx + cb[0][ixx];
              const float *pp = part + (brick * (ZC + 1) + cl[2][iz]) * (F * 3) * kNBOX + cl[1][iy] * 17 + cl[0][ixx];
#pragma unroll
              for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int c = 0; c < 3; ++c) val[f][c] += (f < F) ? pp[(f * 3 + c) * kNBOX] : 0.0f;
            }
      } else {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int c = 0; c < 3; ++c) val[f][c] = (f < F) ? (f == 0 ? out0 : out1)[c * g.nnodes + n] : 0.0f;
      }
    } else {
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int c = 0; c < 3; ++c) val[f][c] = 0.0f;
    }
    if (CURV) {
      // alpha C_H (L^T z)(p), (L^T z)(p) = sum_a [chi_a(p-e_a) z(p-e_a) - 2 chi_a(p) z(p) + chi_a(p+e_a) z(p+e_a)] / H_a^2
      const int pp[3] = {px, py, pz};
      const int nn[3] = {g.px, g.py, g.pz};
      const int64_t st[3] = {1, g.px, (int64_t)g.px * g.py};
      const float ih2[3] = {g.iHx * g.iHx, g.iHy * g.iHy, g.iHz * g.iHz};
      float wc = 0.0f, wm[3], wp[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        wc += -2.0f * chi(pp[a], nn[a]) * ih2[a];
        wm[a] = (pp[a] > 0 && chi(pp[a] - 1, nn[a])) ? ih2[a] : 0.0f;
        wp[a] = (pp[a] < nn[a] - 1 && chi(pp[a] + 1, nn[a])) ? ih2[a] : 0.0f;
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float *z = Lw + c * g.nnodes + n;
        float acc = wc * z[0];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          // neighbours outside the grid have zero weight; read the centre instead
          acc += wm[a] * z[wm[a] != 0.0f ? -st[a] : 0];
          acc += wp[a] * z[wp[a] != 0.0f ? st[a] : 0];
        }
        val[0][c] += A.curv_scale * acc;
      }
      if (NF == 2 && A.curv_diag) {
        float side = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) side += (wm[a] + wp[a]) * ih2[a];
        const float d = A.curv_scale * (wc * wc + side);
#pragma unroll
        for (int c = 0; c < 3; ++c) val[NF - 1][c] += d;
      }
    }
    if (tauv) {
#pragma unroll
      for (int c = 0; c < 3; ++c) val[0][c] += A.tau * tauv[c * g.nnodes + n];
    }
    if (!stopped) {
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int c = 0; c < 3; ++c) (f == 0 ? out0 : out1)[c * g.nnodes + n] = val[f][c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (dotv) dsum += (double)dotv[c * g.nnodes + n] * (double)val[0][c];
      gsq += (double)val[0][c] * (double)val[0][c];
      if (NF == 2) dmax = fmax(dmax, (double)val[NF - 1][c]);
    }
  }
  if (A.blocks && !stopped) {
    const double v[3] = {dsum, dmax, gsq};
    block_write<3>(v, A.blocks + bid * 3, 2u);
  }
}

template <int ZC, int F, int NF, bool CURV>
__global__ __launch_bounds__(256) void k_gather(GatherArgs A) {
  gather_body<ZC, F, NF, CURV>(A, hw_blk());
}

// L w for w = a - b (b nullable), and per-block sum of (L w)^2.  Branch-free: stencil
// neighbours that L does not use (chi = 0) read the centre with weight zero, so every
// load is requested before the first wait.
__device__ __forceinline__ void curv_L_body(const Geo &g, const float *__restrict__ a, const float *__restrict__ b,
                                            float *__restrict__ Lw, double *blocks, const double *stop, const Blk &B) {
  // read with the other loads; only the writes wait for it (no workgroup writes it here)
  const bool stopped = stop && *stop != 0.0;
  const int px = B.x * 64 + (threadIdx.x & 63), py = B.y * 4 + (threadIdx.x >> 6), pz = B.z;
  const bool in = px < g.px && py < g.py;
  const int pp[3] = {in ? px : 0, in ? py : 0, pz};
  const int64_t n = ((int64_t)pp[2] * g.py + pp[1]) * g.px + pp[0];
  const int64_t bid = B.lin;
  const int nn[3] = {g.px, g.py, g.pz};
  const int64_t st[3] = {1, g.px, (int64_t)g.px * g.py};
  const float ih2[3] = {g.iHx * g.iHx, g.iHy * g.iHy, g.iHz * g.iHz};
  int64_t om[3], op[3];
  float wgt[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const bool use = chi(pp[ax], nn[ax]);
    om[ax] = use ? -st[ax] : 0;
    op[ax] = use ? st[ax] : 0;
    wgt[ax] = use ? ih2[ax] : 0.0f;
  }
  float w[3][7];  // [component][centre, -x, +x, -y, +y, -z, +z]
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t off = c * g.nnodes + n;
    const int64_t o[7] = {0, om[0], op[0], om[1], op[1], om[2], op[2]};
#pragma unroll
    for (int m = 0; m < 7; ++m) w[c][m] = b ? a[off + o[m]] - b[off + o[m]] : a[off + o[m]];
  }
  double e = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float acc = 0.0f;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) acc += (w[c][1 + 2 * ax] - 2.0f * w[c][0] + w[c][2 + 2 * ax]) * wgt[ax];
    if (in && !stopped) Lw[c * g.nnodes + n] = acc;
    if (in) e += (double)acc * (double)acc;
  }
  if (blocks && !stopped) block_write<1>(&e, blocks + bid);
}

__global__ __launch_bounds__(256) void k_curv_L(Geo g, const float *__restrict__ a, const float *__restrict__ b,
                                                float *__restrict__ Lw, double *blocks, const double *stop) {
  curv_L_body(g, a, b, Lw, blocks, stop, hw_blk());
}

// central-difference image gradient with replicated border, stored as ST.  A workgroup
// takes a 64 x kImgY voxel tile of kImgZ consecutive planes and walks up in z with the -z and
// +z values rolled in registers, so that each plane of the tile is read from memory once;
// the x and y neighbours lie in the plane just read (cache hits).
constexpr int kImgZ = 16, kImgY = 16;
template <class ST>
__global__ __launch_bounds__(64 * kImgY) void k_imgrad(Geo g, const float *__restrict__ img, typename ST::elem *__restrict__ out,
                                                float sq) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63), j = blockIdx.y * kImgY + (threadIdx.x >> 6);
  const int z0 = blockIdx.z * kImgZ, z1 = min(z0 + kImgZ, g.nz);
  if (i >= g.nx || j >= g.ny || z0 >= g.nz) return;
  const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny, col = (int64_t)j * g.nx + i;
  const int64_t dxm = i > 0 ? -1 : 0, dxp = i < g.nx - 1 ? 1 : 0;
  const int64_t dym = j > 0 ? -sy : 0, dyp = j < g.ny - 1 ? sy : 0;
  const float cx = 0.5f * g.ihx, cy = 0.5f * g.ihy, cz = 0.5f * g.ihz;
  float zm = img[(int64_t)(z0 > 0 ? z0 - 1 : 0) * sz + col];  // plane k - 1 (replicated at 0)
  float zc = img[(int64_t)z0 * sz + col];                     // plane k
#pragma unroll 4
  for (int k = z0; k < z1; ++k) {
    const int64_t v = (int64_t)k * sz + col;
    const float zp = k < g.nz - 1 ? img[v + sz] : zc;  // plane k + 1 (replicated at the top)
    float o[3];
    o[0] = (img[v + dxp] - img[v + dxm]) * cx;
    o[1] = (img[v + dyp] - img[v + dym]) * cy;
    o[2] = (zp - zm) * cz;
    ST::store(out, v, sq, o);
    zm = zc;
    zc = zp;
  }
}

// max |grad component| of a volume per tile (for the FP16 scale): the traversal and the
// gradient values of k_imgrad (before scaling), one maximum per 64 x kImgY x kImgZ tile
__global__ __launch_bounds__(64 * kImgY) void k_absmax_grad(Geo g, const float *__restrict__ img, double *blocks) {
  __shared__ float wmax[kImgY];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane, j = blockIdx.y * kImgY + wave;
  const int z0 = blockIdx.z * kImgZ, z1 = min(z0 + kImgZ, g.nz);
  float m = 0.0f;
  if (i < g.nx && j < g.ny && z0 < g.nz) {
    const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny, col = (int64_t)j * g.nx + i;
    const int64_t dxm = i > 0 ? -1 : 0, dxp = i < g.nx - 1 ? 1 : 0;
    const int64_t dym = j > 0 ? -sy : 0, dyp = j < g.ny - 1 ? sy : 0;
    const float cx = 0.5f * g.ihx, cy = 0.5f * g.ihy, cz = 0.5f * g.ihz;
    float zm = img[(int64_t)(z0 > 0 ? z0 - 1 : 0) * sz + col];
    float zc = img[(int64_t)z0 * sz + col];
#pragma unroll 4
    for (int k = z0; k < z1; ++k) {
      const int64_t v = (int64_t)k * sz + col;
      const float zp = k < g.nz - 1 ? img[v + sz] : zc;
      m = fmaxf(m, fabsf((img[v + dxp] - img[v + dxm]) * cx));
      m = fmaxf(m, fabsf((img[v + dyp] - img[v + dym]) * cy));
      m = fmaxf(m, fabsf((zp - zm) * cz));
      zm = zc;
      zc = zp;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if (lane == 0) wmax[wave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float r = wmax[0];
#pragma unroll
    for (int w = 1; w < kImgY; ++w) r = fmaxf(r, wmax[w]);
    blocks[((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = (double)r;
  }
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
