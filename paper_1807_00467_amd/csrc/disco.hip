// Host side of the C ABI declared in include/disco.h: context and workspace
// management, argument validation, kernel launches on the caller's stream.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <numeric>
#include <mutex>
#include <unordered_map>
#include <utility>
#include <vector>

#include "disco.h"
#include "kernels.hpp"
#include "solver.hpp"
#include "adjoint.hpp"
#include "batch.hpp"
#include "pyramid.hpp"
#include "keypoint.hpp"

using namespace disco;

namespace {

constexpr int kZC = 4;          // cells per brick along z

struct EventPair {
  hipEvent_t a, b;
};

struct Arena {
  void *ptr = nullptr;
};

}  // namespace

struct disco_ctx {
  int device = 0;
  int storage = DISCO_STORAGE_FP32;
  Geo g{};
  int64_t ncells = 0;
  int64_t nwg = 0;         // brick workgroups
  int64_t nodeblocks = 0;  // blocks of node-parallel kernels
  // derived volumes
  void *gR = nullptr, *gT = nullptr, *scache = nullptr;
  float sR = 1.f, sT = 1.f;                 // dequantisation scales (FP16)
  float sS_load = 1.f, sS_store = 1.f;      // s cache scales (FP16)
  double max_gT = 0.0;                      // max |grad T| component (FP16 storage)
  bool images = false;
  bool lin = false;
  double lin_eta = 0.0;
  // node workspaces
  float *u_lin = nullptr, *u_ref = nullptr, *Lw = nullptr;
  float *vg = nullptr, *vdiag = nullptr, *vx = nullptr, *vr = nullptr, *vz = nullptr, *vp = nullptr, *vq = nullptr,
        *vut = nullptr, *tmp0 = nullptr, *tmp1 = nullptr, *vp2 = nullptr, *vinvm = nullptr;
  float *part = nullptr;
  double *blk_brick = nullptr, *blk_node = nullptr, *sc = nullptr;
  double *blk_curv = nullptr, *blk_upd = nullptr;
  double *blk_img = nullptr;  // FP16 scale search: per-block maxima (allocated at first use)
  float *adjW = nullptr;  // dD/d(grad T) accumulator of ngf_grad_T, [N][3] (allocated on first use)
  // lung masks and the boundary term's GN vectors (allocated by disco_set_masks)
  uint8_t *mF = nullptr, *mM = nullptr, *rflag = nullptr;
  float *sbc = nullptr, *zb = nullptr;
  bool masks = false;
  bool lin_mask = false;  // the last linearisation wrote the boundary term's GN vectors
  // L-BFGS history (allocated on first use): a ring of lb_m pairs (s, y)
  float *lbS = nullptr, *lbY = nullptr;  // [lb_m][3][nodes]
  int lb_m = 0;
  int lb_count = 0;      // complete pairs in the ring
  int lb_next = 0;       // slot of the next pair
  bool lb_pending = false;  // the last step started a pair in slot lb_next
  int *status = nullptr;
  double *host_sc = nullptr;  // pinned
  hipEvent_t ls_ev[2] = {nullptr, nullptr};  // line search: trial flags copied to host_sc[0..1]
  // keypoints
  int32_t nkp = 0;
  float *kloc = nullptr, *ktgt = nullptr;
  int *kstart = nullptr;
  // profiling
  bool prof = false;
  std::vector<EventPair> ev[5];
};

// keypoint stage: normalised gradient 4-vectors of F and M, split by voxel parity
struct disco_kp {
  int device = 0;
  KpGeo g{};
  double h[3] = {1.0, 1.0, 1.0};
  float4 *nF = nullptr, *nM = nullptr;
  float4 *patch = nullptr;  // [cap][64] patch vectors of the keypoints of the last cost call
  int patch_cap = 0;
  float *bp = nullptr;  // belief-propagation work memory, grown as needed
  size_t bp_cap = 0;    // floats
  char *th = nullptr;   // tree set-up buffers for up to tcap keypoints: pinned host staging
  char *td = nullptr;   // and their device copies (see KpTreeBuf)
  int tcap = 0;
  bool images = false;
};

// a group of contexts stepped together (see batch.hpp)
struct disco_batch {
  int device = 0;
  int storage = DISCO_STORAGE_FP32;
  std::vector<disco_ctx *> ctx;  // in work order (largest pair first)
  std::vector<int> order;        // order[i] = caller index of ctx[i]
  void *desc = nullptr;          // PairDesc<ST>[npairs] on the device
  int *start = nullptr;          // work lists on the device: 4 x (npairs + 1)
  bool prepared = false;
  bool vcc = false, kp = false, curv = false;
  int pcg_iters = 0, ls_max = 0;
  int ncu = 0;
  int wpc[3] = {4, 8, 8};        // workgroups per compute unit: brick, node, vector passes
  int zc = kZC;                  // brick tile of the batched passes: cell layers per brick (2 or 4)
  std::unordered_map<const void *, int> occ;  // resident workgroups per compute unit, per kernel
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

inline int hip_err(hipError_t e) { return DISCO_ERR_HIP - (int)e; }

#define HIP_TRY(x)                      \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return hip_err(e_); \
  } while (0)

inline bool aligned4(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }
inline bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

inline hipStream_t S(disco_stream s) { return reinterpret_cast<hipStream_t>(s); }

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// 3-D grid of 64 x 4 thread blocks over the node grid
inline dim3 node_grid(const Geo &g) { return dim3((g.px + 63) / 64, (g.py + 3) / 4, g.pz); }
// geometry for bricks of zc cell layers (the batched passes' tile); bricks of that tile
inline Geo tile_geo(Geo g, int zc) {
  g.zc = zc;
  g.nbz = (g.cz + zc - 1) / zc;
  return g;
}
inline int64_t tile_bricks(const Geo &g, int zc) { return (int64_t)g.nbx * g.nby * ((g.cz + zc - 1) / zc); }
constexpr int kTileZ[2] = {4, 2};  // brick tiles of the batched passes
inline int64_t node_blocks(const Geo &g) { return (int64_t)((g.px + 63) / 64) * ((g.py + 3) / 4) * g.pz; }
// workgroups of the CG vector update, and the grid of the fused p update + L p pass
inline int64_t upd_blocks(const Geo &g) { return (3 * g.nnodes + 256 * kUpdK - 1) / (256 * kUpdK); }
inline dim3 lp_grid(const Geo &g) { return dim3((g.px + 63) / 64, (g.py + 3) / 4, (g.pz + kLpZ - 1) / kLpZ); }
// 3-D grid over the voxels (rows of 256)
inline dim3 vox_grid(const Geo &g) { return dim3((g.nx + 255) / 256, g.ny, g.nz); }
// k_imgrad: 64 x kImgY voxel tiles of kImgZ planes, 64 kImgY threads
inline dim3 imgrad_grid(const Geo &g) {
  return dim3((g.nx + 63) / 64, (g.ny + kImgY - 1) / kImgY, (g.nz + kImgZ - 1) / kImgZ);
}
inline size_t image_tiles(const Geo &g) {
  const dim3 t = imgrad_grid(g);
  return (size_t)t.x * t.y * t.z;
}

// event stamps of a profiled brick pass, taken by the kernels' own dispatches (as a kernel
// trace records them, without the event packets' own dispatch): the first kernel of the
// pass stamps its start, the last one its end
struct Stamp {
  hipEvent_t a = nullptr, b = nullptr;
  bool first = true;  // no kernel launched yet
};

template <class K, class A>
void brick_go(K kernel, dim3 grid, dim3 block, hipStream_t s, Stamp *st, bool last, const A &a) {
  if (st && st->a) {
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, st->first ? st->a : nullptr, last ? st->b : nullptr, 0u, a);
    st->first = false;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, 0, s, a);
  }
}

// times one pass of kind k while profiling is on: with a Stamp, by the kernels' own
// dispatch stamps; otherwise by events recorded around the pass on its stream
struct ProfScope {
  disco_ctx *c;
  int k;
  hipStream_t s;
  Stamp *st;
  EventPair e{};
  bool on;
  ProfScope(disco_ctx *c_, int k_, hipStream_t s_, Stamp *st_ = nullptr) : c(c_), k(k_), s(s_), st(st_), on(c_->prof) {
    if (on) {
      (void)hipEventCreate(&e.a);
      (void)hipEventCreate(&e.b);
      if (st) {
        st->a = e.a;
        st->b = e.b;
      } else {
        (void)hipEventRecord(e.a, s);
      }
    }
  }
  ~ProfScope() {
    if (!on) return;
    if (st && st->first) {  // the pass launched nothing
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
      return;
    }
    if (!st) (void)hipEventRecord(e.b, s);
    c->ev[k].push_back(e);
  }
};

void clear_profile(disco_ctx *c) {
  for (auto &v : c->ev) {
    for (auto &p : v) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    v.clear();
  }
}

// ------------------------------------------------------------------------------
// brick kernel dispatch
// ------------------------------------------------------------------------------
template <class ST, int MODE>
void launch_brick_mode(disco_ctx *c, bool ngf, bool vcc, bool kp, bool mask, const BrickArgs<ST> &a,
                       hipStream_t s, Stamp *st = nullptr, bool last = true) {
  dim3 grid(c->g.nbx, c->g.nby, c->g.nbz);
  const int key = (ngf ? 4 : 0) | (vcc ? 2 : 0) | (kp ? 1 : 0);
  if (MODE != M_HV && ngf && (vcc || kp)) {
    // objective and gradient passes: the cell terms (VALU-heavy, many registers) and the
    // NGF voxel pass (memory-bound) run as two launches with their own occupancy; the
    // second adds to the outputs of the first
    launch_brick_mode<ST, MODE>(c, false, vcc, kp, false, a, s, st, false);
    BrickArgs<ST> b = a;
    b.acc = 1;
    if (mask)
      brick_go((k_brick<ST, MODE, true, false, false, kZC, true>), grid, dim3(brick_threads<MODE, true, false>()), s, st, last, b);
    else
      brick_go((k_brick<ST, MODE, true, false, false, kZC>), grid, dim3(brick_threads<MODE, true, false>()), s, st, last, b);
    return;
  }
  if (mask && ngf) {
    // the lung-boundary term rides on the voxel pass
    switch (key) {
      case 7: if constexpr (MODE == M_HV) { brick_go((k_brick<ST, MODE, true, true, true, kZC, true>), grid, dim3(brick_threads<MODE, true, true>()), s, st, last, a); return; } break;
      case 6: if constexpr (MODE == M_HV) { brick_go((k_brick<ST, MODE, true, true, false, kZC, true>), grid, dim3(brick_threads<MODE, true, true>()), s, st, last, a); return; } break;
      case 5: if constexpr (MODE == M_HV) { brick_go((k_brick<ST, MODE, true, false, true, kZC, true>), grid, dim3(brick_threads<MODE, true, true>()), s, st, last, a); return; } break;
      case 4: brick_go((k_brick<ST, MODE, true, false, false, kZC, true>), grid, dim3(brick_threads<MODE, true, false>()), s, st, last, a); return;
      default: break;
    }
  }
  if constexpr (MODE == M_HV) {
    switch (key) {
      case 7: brick_go((k_brick<ST, MODE, true, true, true, kZC>), grid, dim3(brick_threads<MODE, true, true || true>()), s, st, last, a); return;
      case 6: brick_go((k_brick<ST, MODE, true, true, false, kZC>), grid, dim3(brick_threads<MODE, true, true || false>()), s, st, last, a); return;
      case 5: brick_go((k_brick<ST, MODE, true, false, true, kZC>), grid, dim3(brick_threads<MODE, true, false || true>()), s, st, last, a); return;
      default: break;
    }
  }
  switch (key) {
    case 4: brick_go((k_brick<ST, MODE, true, false, false, kZC>), grid, dim3(brick_threads<MODE, true, false || false>()), s, st, last, a); break;
    case 3: brick_go((k_brick<ST, MODE, false, true, true, kZC>), grid, dim3(brick_threads<MODE, false, true || true>()), s, st, last, a); break;
    case 2: brick_go((k_brick<ST, MODE, false, true, false, kZC>), grid, dim3(brick_threads<MODE, false, true || false>()), s, st, last, a); break;
    case 1: brick_go((k_brick<ST, MODE, false, false, true, kZC>), grid, dim3(brick_threads<MODE, false, false || true>()), s, st, last, a); break;
    default: break;
  }
}

struct BrickCall {
  int mode;
  bool ngf, vcc, kp;
  float eta2;
  float gamma, delta;
  const float *u, *v;
  float *out0, *out1;
  const double *stop;
  double beta = 0.0;  // lung-boundary weight (needs masks; rides on the NGF voxel pass)
};

template <class ST>
BrickArgs<ST> make_args(disco_ctx *c, const BrickCall &b) {
  BrickArgs<ST> a{};
  a.g = c->g;
  a.gR = reinterpret_cast<const typename ST::elem *>(c->gR);
  a.gT = reinterpret_cast<const typename ST::elem *>(c->gT);
  a.sc = reinterpret_cast<typename ST::elem *>(c->scache);
  a.sR = c->sR;
  a.sT = c->sT;
  a.sS_load = c->sS_load;
  a.sS_store = c->sS_store;
  a.u = b.u;
  a.v = b.v;
  a.kloc = c->kloc;
  a.ktgt = c->ktgt;
  a.kstart = c->kstart;
  a.eta2 = b.eta2;
  a.ngf_scale = (float)(2.0 * (double)c->g.hx * (double)c->g.hy * (double)c->g.hz);
  a.gamma = b.gamma;
  a.delta = b.delta;
  a.out0 = b.out0;
  a.out1 = b.out1;
  a.part = c->part;
  a.blocks = c->blk_brick;
  a.stop = b.stop;
  a.mF = c->mF;
  a.mM = c->mM;
  a.sbc = c->sbc;
  a.rflag = c->rflag;
  a.zb = c->zb;
  a.mscale = (float)(0.5 * b.beta);
  a.mroot = (float)std::sqrt(0.5 * b.beta);
  return a;
}

void launch_brick(disco_ctx *c, const BrickCall &b, hipStream_t s) {
  const int pk = b.mode == M_HV ? 0 : (b.mode == M_GRAD ? 1 : 2);
  Stamp st;
  ProfScope ps(c, pk, s, &st);
  Stamp *sp = c->prof ? &st : nullptr;
  const bool mask = b.ngf && b.beta != 0.0 && c->masks;
  if (c->storage == DISCO_STORAGE_FP16) {
    auto a = make_args<F16x3>(c, b);
    if (b.mode == M_EVAL) launch_brick_mode<F16x3, M_EVAL>(c, b.ngf, b.vcc, b.kp, mask, a, s, sp);
    if (b.mode == M_GRAD) launch_brick_mode<F16x3, M_GRAD>(c, b.ngf, b.vcc, b.kp, mask, a, s, sp);
    if (b.mode == M_HV) launch_brick_mode<F16x3, M_HV>(c, b.ngf, b.vcc, b.kp, mask, a, s, sp);
  } else {
    auto a = make_args<F32x3>(c, b);
    if (b.mode == M_EVAL) launch_brick_mode<F32x3, M_EVAL>(c, b.ngf, b.vcc, b.kp, mask, a, s, sp);
    if (b.mode == M_GRAD) launch_brick_mode<F32x3, M_GRAD>(c, b.ngf, b.vcc, b.kp, mask, a, s, sp);
    if (b.mode == M_HV) launch_brick_mode<F32x3, M_HV>(c, b.ngf, b.vcc, b.kp, mask, a, s, sp);
  }
}

double ch_of(const disco_ctx *c) { return (double)c->g.Hx * (double)c->g.Hy * (double)c->g.Hz; }
double h3_of(const disco_ctx *c) { return (double)c->g.hx * (double)c->g.hy * (double)c->g.hz; }

PostArgs post_args(disco_ctx *c, double alpha = 0.0, double gamma = 0.0, double delta = 0.0) {
  PostArgs a{};
  a.sc = c->sc;
  a.status = c->status;
  a.alpha = alpha;
  a.gamma = gamma;
  a.delta = delta;
  a.CH = ch_of(c);
  a.h3 = h3_of(c);
  a.beta = 0.0;
  return a;
}

RedSrc src_brick(disco_ctx *c, double *out) { return RedSrc{c->blk_brick, c->nwg, BS_N, BS_N, 0u, out}; }
RedSrc src_curv(disco_ctx *c, double *out) { return RedSrc{c->blk_curv, c->nodeblocks, 1, 1, 0u, out}; }
// gather blocks: <dotv,out0>, max out1, |out0|^2
RedSrc src_gather(disco_ctx *c, double *out) { return RedSrc{c->blk_node, c->nodeblocks, 3, 3, 2u, out}; }
RedSrc src_pairs(const double *blocks, int64_t nb, int nvals, double *out) { return RedSrc{blocks, nb, 2, nvals, 0u, out}; }

void launch_finish(int post, const PostArgs &pa, const double *stop, hipStream_t s, RedSrc s0, RedSrc s1 = RedSrc{},
                   RedSrc s2 = RedSrc{}) {
  const int n = s2.blocks ? 3 : (s1.blocks ? 2 : 1);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, s0, s1, s2, n, post, pa, stop);
}

void launch_reduce(const double *blocks, int64_t nb, int stride, int nvals, uint32_t max_mask, double *out,
                   const double *stop, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, blocks, nb, stride, nvals, max_mask, out, stop);
}

// gather after a brick pass (F fields written by the brick kernel, nf produced); with
// `reduce` it writes per-block <dotv, out0>, max out1, |out0|^2 to blk_node
void launch_gather(disco_ctx *c, int F, int nf, float *out0, float *out1, const float *Lw, float curv_scale,
                   int curv_diag, const float *tauv, float tau, const float *dotv, bool reduce, const double *stop,
                   hipStream_t s) {
  GatherArgs a{};
  a.g = c->g;
  a.F = F;
  a.nf = nf;
  a.part = c->part;
  a.out0 = out0;
  a.out1 = out1;
  a.Lw = Lw;
  a.curv_scale = curv_scale;
  a.curv_diag = curv_diag;
  a.tauv = tauv;
  a.tau = tau;
  a.dotv = dotv;
  a.blocks = reduce ? c->blk_node : nullptr;
  a.stop = stop;
  const dim3 grid = node_grid(c->g);
  const bool curv = Lw != nullptr;
#define GATHER(Fv, NFv, CV) hipLaunchKernelGGL((k_gather<kZC, Fv, NFv, CV>), grid, dim3(256), 0, s, a)
  if (F == 2 && nf == 2) {
    if (curv) GATHER(2, 2, true); else GATHER(2, 2, false);
  } else if (F == 1 && nf == 1) {
    if (curv) GATHER(1, 1, true); else GATHER(1, 1, false);
  } else if (F == 0 && nf == 2) {
    if (curv) GATHER(0, 2, true); else GATHER(0, 2, false);
  } else {
    if (curv) GATHER(0, 1, true); else GATHER(0, 1, false);
  }
#undef GATHER
}

// L w with w = a - b; with `energy` it writes per-block sum (L w)^2 to blk_curv
void launch_curv_L(disco_ctx *c, const float *a, const float *b, float *Lw, bool energy, const double *stop,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_curv_L, node_grid(c->g), dim3(256), 0, s, c->g, a, b, Lw, energy ? c->blk_curv : nullptr,
                     stop);
}

// FP16 s cache: |s_c| <= sum_a |JG[a][c]| |dr/da_a| <= sqrt(3) (2 max|grad T| / h_min) (2 / eta),
// since |dr/da| <= 2 / sqrt(eta^2 + |a|^2); the power-of-two scale keeps that bound below
// 2^15 (largest half is 65504), so no value overflows and typical values stay normal.
void set_s_scale(disco_ctx *c, double eta) {
  if (c->storage != DISCO_STORAGE_FP16) return;
  const double hmin = std::min((double)c->g.hx, std::min((double)c->g.hy, (double)c->g.hz));
  const double bound = 4.0 * std::sqrt(3.0) * c->max_gT / (hmin * eta);
  int ex = 0;
  if (bound > 0.0 && std::isfinite(bound)) ex = (int)std::floor(std::log2(32768.0 / bound));
  ex = std::max(-100, std::min(100, ex));
  c->sS_store = std::ldexp(1.0f, ex);
  c->sS_load = std::ldexp(1.0f, -ex);
}

int check_field(const void *p) {
  if (!p) return DISCO_ERR_ARG;
  if (!aligned4(p)) return DISCO_ERR_SHAPE;
  return DISCO_OK;
}

int set_device(disco_ctx *c) {
  HIP_TRY(hipSetDevice(c->device));
  return DISCO_OK;
}

// ------------------------------------------------------------------------------
// batched GN step (all pairs, one launch per phase)
// ------------------------------------------------------------------------------
template <class ST>
GatherArgs gather_args(disco_ctx *c, int F, int nf, float *out0, float *out1, const float *Lw, float curv_scale,
                       int curv_diag, const float *tauv, float tau, const float *dotv, const double *stop) {
  GatherArgs a{};
  a.g = c->g;
  a.F = F;
  a.nf = nf;
  a.part = c->part;
  a.out0 = out0;
  a.out1 = out1;
  a.Lw = Lw;
  a.curv_scale = curv_scale;
  a.curv_diag = curv_diag;
  a.tauv = tauv;
  a.tau = tau;
  a.dotv = dotv;
  a.blocks = c->blk_node;
  a.stop = stop;
  return a;
}

FinishArgs finish_args(int post, const PostArgs &pa, const double *stop, RedSrc s0, RedSrc s1 = RedSrc{},
                       RedSrc s2 = RedSrc{}) {
  FinishArgs f{};
  f.s0 = s0;
  f.s1 = s1;
  f.s2 = s2;
  f.nsrc = s2.blocks ? 3 : (s1.blocks ? 2 : 1);
  f.post = post;
  f.pa = pa;
  f.stop = stop;
  return f;
}

template <class ST>
PairDesc<ST> pair_desc(disco_ctx *c, const disco_params *p, float *u, double *report, int32_t *status_out, int zc) {
  PairDesc<ST> d{};
  const Geo &g = c->g;
  const Geo tg = tile_geo(g, zc);  // the batch's brick tile
  const bool vcc = p->gamma != 0.0;
  const bool kp = p->delta != 0.0 && c->nkp > 0;
  const bool curv = p->alpha != 0.0;
  const float eta2 = (float)(p->eta * p->eta);
  const double CH = ch_of(c);
  set_s_scale(c, p->eta);
  d.g = g;
  d.u = u;
  d.u_ref = c->u_ref;
  d.u_lin = c->u_lin;
  d.Lw = c->Lw;
  d.grad = c->vg;
  d.diag = c->vdiag;
  d.x = c->vx;
  d.r = c->vr;
  d.z = c->vz;
  d.p[0] = c->vp;
  d.p[1] = c->vp2;
  d.q = c->vq;
  d.ut = c->vut;
  d.invM = c->vinvm;
  d.sc = c->sc;
  d.blk_node = c->blk_node;
  d.blk_curv = c->blk_curv;
  d.blk_upd = c->blk_upd;
  d.status = c->status;
  d.report = report;
  d.status_out = status_out;
  d.n3 = 3 * g.nnodes;
  d.nodeblocks = c->nodeblocks;
  d.tau = (float)p->tau;
  d.tol = p->pcg_tol;
  d.CH = CH;
  PairDesc<ST> &D = d;
  D.lin = make_args<ST>(c, BrickCall{M_GRAD, true, vcc, kp, eta2, (float)p->gamma, (float)p->delta, u, nullptr,
                                     c->vg, c->vdiag, nullptr});
  for (int k = 0; k < 2; ++k)
    D.hv[k] = make_args<ST>(c, BrickCall{M_HV, true, vcc, kp, 0.f, (float)p->gamma, (float)p->delta, c->u_lin,
                                         D.p[k], c->vq, nullptr, c->sc + SC_STOP});
  D.eval = make_args<ST>(c, BrickCall{M_EVAL, true, vcc, kp, eta2, (float)p->gamma, (float)p->delta, c->vut,
                                      nullptr, nullptr, nullptr, c->sc + SC_ACCEPT});
  D.glin = gather_args<ST>(c, 2, 2, c->vg, c->vdiag, curv ? c->Lw : nullptr, (float)(p->alpha * CH), curv ? 1 : 0,
                           nullptr, 0.f, nullptr, nullptr);
  for (int k = 0; k < 2; ++k)
    D.ghv[k] = gather_args<ST>(c, 1, 1, c->vq, nullptr, curv ? c->Lw : nullptr, (float)(p->alpha * CH), 0,
                               p->tau != 0.0 ? D.p[k] : nullptr, (float)p->tau, D.p[k], c->sc + SC_STOP);
  // the brick passes and the gathers of their partials work on the batch's brick tile
  D.lin.g = D.eval.g = D.hv[0].g = D.hv[1].g = tg;
  D.glin.g = D.ghv[0].g = D.ghv[1].g = tg;
  const RedSrc bricks{c->blk_brick, tile_bricks(g, zc), BS_N, BS_N, 0u, nullptr};
  PostArgs pa = post_args(c, p->alpha, p->gamma, p->delta);
  pa.c1 = p->armijo_c1;
  pa.tol = p->pcg_tol;
  double *sc = c->sc;
  const int64_t nb3 = nblk(3 * g.nnodes);
  RedSrc b_lin = bricks, b_trial = bricks;
  b_lin.out = sc + SC_TMP0;
  b_trial.out = sc + SC_TMP0;
  D.fin_lin = finish_args(POST_LIN_BRICK, pa, nullptr, b_lin, src_curv(c, sc + SC_SRAW), src_gather(c, sc + SC_DOT));
  D.fin_pcg = finish_args(POST_PCG_START, pa, nullptr, src_pairs(c->blk_node, nb3, 2, sc + SC_TMP0));
  D.fin_lsb = finish_args(POST_LS_BEGIN, pa, nullptr, src_pairs(c->blk_node, nb3, 1, sc + SC_TMP0),
                          src_pairs(c->blk_upd, upd_blocks(g), 2, sc + SC_TMP1));
  D.fin_trial = finish_args(POST_LS_BRICK, pa, sc + SC_ACCEPT, b_trial, src_curv(c, sc + SC_TSRAW));
  return d;
}

}  // namespace

// ==============================================================================
// C ABI
// ==============================================================================
extern "C" {

const char *disco_status_string(int code) {
  switch (code) {
    case DISCO_OK: return "ok";
    case DISCO_ERR_ARG: return "invalid argument (null pointer, bad enum or count)";
    case DISCO_ERR_SHAPE: return "shape error (size not a positive multiple of 4, keypoint outside the image box, or misaligned pointer)";
    case DISCO_ERR_STATE: return "state error (images not set or no linearisation yet)";
    case DISCO_ERR_NONFINITE: return "non-finite or out-of-range scalar parameter";
    case DISCO_ERR_NOMEM: return "device allocation failed";
    case DISCO_ERR_LIMIT: return "volume exceeds the static scratch of disco_set_images_noalloc (FP16 storage: at most 2^14 tiles of 64 x 16 x 16 voxels)";
    default:
      if (code <= DISCO_ERR_HIP) return hipGetErrorString((hipError_t)(DISCO_ERR_HIP - code));
      return "unknown code";
  }
}

void disco_destroy(disco_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  clear_profile(c);
  void *ptrs[] = {c->gR,  c->gT,  c->scache, c->u_lin, c->u_ref, c->Lw,   c->vg,   c->vdiag, c->vx,   c->vr,
                  c->vz,  c->vp,  c->vq,     c->vut,   c->tmp0,  c->tmp1, c->part, c->blk_brick, c->blk_node,
                  c->sc,  c->status, c->kloc, c->ktgt, c->kstart, c->blk_curv, c->blk_upd, c->blk_img, c->adjW, c->vp2, c->vinvm,
                  c->lbS, c->lbY, c->mF, c->mM, c->rflag, c->sbc, c->zb};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (c->host_sc) (void)hipHostFree(c->host_sc);
  for (hipEvent_t e : c->ls_ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

int disco_create(const disco_geom *geom, int32_t storage, disco_ctx **out) {
  if (!out) return DISCO_ERR_ARG;
  *out = nullptr;
  if (!geom) return DISCO_ERR_ARG;
  if (storage != DISCO_STORAGE_FP32 && storage != DISCO_STORAGE_FP16) return DISCO_ERR_ARG;
  for (int a = 0; a < 3; ++a) {
    if (geom->n[a] < 4 || geom->n[a] % 4 != 0) return DISCO_ERR_SHAPE;
    if (!std::isfinite(geom->h[a]) || !(geom->h[a] > 0.0)) return DISCO_ERR_NONFINITE;
  }
  // 32-bit node/voxel coordinates, 64-bit linear indices; the sampling addresses the
  // 3-vector volumes with 32-bit element offsets (3 N < 2^32 in FP32, 4 N in FP16)
  const int64_t nvox = (int64_t)geom->n[0] * geom->n[1] * geom->n[2];
  if ((storage == DISCO_STORAGE_FP16 ? 4 : 3) * nvox >= ((int64_t)1 << 32)) return DISCO_ERR_SHAPE;

  disco_ctx *c = new (std::nothrow) disco_ctx();
  if (!c) return DISCO_ERR_NOMEM;
  (void)hipGetDevice(&c->device);
  c->storage = storage;
  Geo &g = c->g;
  g.nx = geom->n[0];
  g.ny = geom->n[1];
  g.nz = geom->n[2];
  g.cx = g.nx / 4;
  g.cy = g.ny / 4;
  g.cz = g.nz / 4;
  g.px = g.cx + 1;
  g.py = g.cy + 1;
  g.pz = g.cz + 1;
  g.zc = kZC;
  g.nbx = (g.cx + kBXC - 1) / kBXC;
  g.nby = (g.cy + kBYC - 1) / kBYC;
  g.nbz = (g.cz + kZC - 1) / kZC;
  g.hx = (float)geom->h[0];
  g.hy = (float)geom->h[1];
  g.hz = (float)geom->h[2];
  g.ihx = (float)(1.0 / geom->h[0]);
  g.ihy = (float)(1.0 / geom->h[1]);
  g.ihz = (float)(1.0 / geom->h[2]);
  g.Hx = (float)(4.0 * geom->h[0]);
  g.Hy = (float)(4.0 * geom->h[1]);
  g.Hz = (float)(4.0 * geom->h[2]);
  g.iHx = (float)(0.25 / geom->h[0]);
  g.iHy = (float)(0.25 / geom->h[1]);
  g.iHz = (float)(0.25 / geom->h[2]);
  g.C = (float)(64.0 * geom->h[0] * geom->h[1] * geom->h[2]);
  g.nvox = nvox;
  g.nnodes = (int64_t)g.px * g.py * g.pz;
  c->ncells = (int64_t)g.cx * g.cy * g.cz;
  c->nwg = (int64_t)g.nbx * g.nby * g.nbz;
  c->nodeblocks = node_blocks(g);

  const size_t vec3 = storage == DISCO_STORAGE_FP16 ? 8 : 12;  // bytes per voxel 3-vector
  const size_t nf = 3 * (size_t)g.nnodes * sizeof(float);
  bool okm = true;
  auto alloc = [&](void **p, size_t bytes) {
    if (!okm) return;
    if (hipMalloc(p, bytes) != hipSuccess) {
      *p = nullptr;
      okm = false;
    }
  };
  // 16 bytes of padding: the FP16 layout reads each voxel with an aligned 8-byte load
  alloc(&c->gR, vec3 * (size_t)nvox + 16);
  alloc(&c->gT, vec3 * (size_t)nvox + 16);
  alloc(&c->scache, vec3 * (size_t)nvox + 16);
  float **nodebufs[] = {&c->u_lin, &c->Lw, &c->vg, &c->vdiag, &c->vx, &c->vr, &c->vz, &c->vp, &c->vq, &c->vut,
                        &c->tmp0, &c->tmp1, &c->vp2, &c->vinvm};
  for (float **p : nodebufs) alloc(reinterpret_cast<void **>(p), nf);
  // brick partials and per-brick sums, sized for every brick tile (the batched passes may
  // use bricks of 2 cell layers)
  size_t part_planes = 0, nbrick = 0;
  for (int zc : kTileZ) {
    part_planes = std::max(part_planes, (size_t)tile_bricks(g, zc) * (zc + 1));
    nbrick = std::max(nbrick, (size_t)tile_bricks(g, zc));
  }
  alloc(reinterpret_cast<void **>(&c->part), sizeof(float) * part_planes * 6 * kNBOX);
  alloc(reinterpret_cast<void **>(&c->blk_brick), sizeof(double) * nbrick * BS_N);
  // node-parallel reductions: 3 values per block over nnodes, or 3 per 256 elements of 3 nnodes
  alloc(reinterpret_cast<void **>(&c->blk_node),
        sizeof(double) * ((size_t)std::max<int64_t>(c->nodeblocks * 6, 3 * (int64_t)nblk(3 * g.nnodes)) + 16));
  alloc(reinterpret_cast<void **>(&c->sc), sizeof(double) * SC_COUNT);
  alloc(reinterpret_cast<void **>(&c->status), sizeof(int));
  alloc(reinterpret_cast<void **>(&c->blk_curv), sizeof(double) * (size_t)c->nodeblocks);
  alloc(reinterpret_cast<void **>(&c->blk_upd), sizeof(double) * 2 * (size_t)upd_blocks(g));
  alloc(reinterpret_cast<void **>(&c->kstart), sizeof(int) * (size_t)(c->ncells + 1));
  if (okm && hipHostMalloc(reinterpret_cast<void **>(&c->host_sc), sizeof(double) * SC_COUNT) != hipSuccess) {
    c->host_sc = nullptr;
    okm = false;
  }
  for (hipEvent_t &e : c->ls_ev)
    if (okm && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      e = nullptr;
      okm = false;
    }
  if (!okm) {
    disco_destroy(c);
    return DISCO_ERR_NOMEM;
  }
  if (hipMemset(c->kstart, 0, sizeof(int) * (size_t)(c->ncells + 1)) != hipSuccess ||
      hipMemset(c->sc, 0, sizeof(double) * SC_COUNT) != hipSuccess ||
      hipMemset(c->status, 0, sizeof(int)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    disco_destroy(c);
    return DISCO_ERR_NOMEM;
  }
  *out = c;
  return DISCO_OK;
}

}  // extern "C"

// Static device scratch for disco_set_images_noalloc: the per-tile maxima of the FP16
// scale search (one double per 64 x 16 x 16 voxel tile), enough for 2^14 tiles
// (512 x 512 x 1024 voxels).
// Every device the library runs on holds its own copy until the process ends.  In host
// code the array's name is not a device address: kernels and copies take the address
// returned by hipGetSymbolAddress, fetched once per device (scratch_ptr).
constexpr size_t kScratchDoubles = (size_t)1 << 14;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static int scratch_ptr(int device, double **out) {
  static std::mutex mu;
  static double *addr[kMaxDevices] = {};  // fixed table: no heap allocation
  if (device < 0 || device >= kMaxDevices) return DISCO_ERR_ARG;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    // the caller has made `device` current
    double *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(reinterpret_cast<void **>(&p), HIP_SYMBOL(scratch)));
    if (!p) return DISCO_ERR_NOMEM;
    addr[device] = p;
  }
  *out = addr[device];
  return DISCO_OK;
}

// Central-difference gradient volumes of R (into gR) and/or T (into gT); null images are
// skipped.  FP16 storage first finds each image's power-of-two scale (max |grad| x scale
// <= 2^14) from per-tile maxima in `blk` (image_tiles(g) doubles, reused by the two
// images in stream order), with one host wait for both.
static int build_gradients(disco_ctx *c, const float *R, const float *T, hipStream_t s, double *blk) {
  const Geo &g = c->g;
  const float *img[2] = {R, T};
  if (c->storage == DISCO_STORAGE_FP16) {
    const dim3 tiles = imgrad_grid(g);
    const unsigned nb = tiles.x * tiles.y * tiles.z;
    for (int k = 0; k < 2; ++k) {
      if (!img[k]) continue;
      hipLaunchKernelGGL(k_absmax_grad, tiles, dim3(64 * kImgY), 0, s, g, img[k], blk);
      launch_reduce(blk, nb, 1, 1, 1u, c->sc + SC_TMP0 + k, nullptr, s);
    }
    HIP_TRY(hipMemcpyAsync(c->host_sc, c->sc + SC_TMP0, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < 2; ++k) {
      if (!img[k]) continue;
      const double mx = c->host_sc[k];
      int ex = 0;
      if (mx > 0.0 && std::isfinite(mx)) ex = (int)std::floor(std::log2(16384.0 / mx));
      ex = std::max(-100, std::min(100, ex));
      const float scale = std::ldexp(1.0f, ex);
      if (k == 0) {
        c->sR = 1.0f / scale;
      } else {
        c->sT = 1.0f / scale;
        c->max_gT = mx;
      }
      hipLaunchKernelGGL(k_imgrad<F16x3>, imgrad_grid(g), dim3(64 * kImgY), 0, s, g, img[k],
                         reinterpret_cast<__half *>(k == 0 ? c->gR : c->gT), scale);
    }
  } else {
    for (int k = 0; k < 2; ++k)
      if (img[k])
        hipLaunchKernelGGL(k_imgrad<F32x3>, imgrad_grid(g), dim3(64 * kImgY), 0, s, g, img[k],
                           reinterpret_cast<float *>(k == 0 ? c->gR : c->gT), 1.0f);
  }
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

// the context's buffer for the FP16 scale search, allocated at its first use
static int image_scratch(disco_ctx *c, hipStream_t s, double **blk) {
  *blk = nullptr;
  if (c->storage != DISCO_STORAGE_FP16) return DISCO_OK;
  if (!c->blk_img) {
    HIP_TRY(hipStreamSynchronize(s));
    if (hipMalloc(reinterpret_cast<void **>(&c->blk_img), sizeof(double) * image_tiles(c->g)) != hipSuccess) {
      c->blk_img = nullptr;
      return DISCO_ERR_NOMEM;
    }
  }
  *blk = c->blk_img;
  return DISCO_OK;
}

extern "C" {

int disco_set_images(disco_ctx *c, const float *R, const float *T, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  int e;
  if ((e = check_field(R)) || (e = check_field(T))) return e;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  double *blk = nullptr;
  if ((e = image_scratch(c, s, &blk))) return e;
  ProfScope ps(c, 3, s);
  c->images = false;
  c->lin = false;
  if ((e = build_gradients(c, R, T, s, blk))) return e;
  c->images = true;
  return DISCO_OK;
}

int disco_set_images_noalloc(disco_ctx *c, const float *R, const float *T, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  int e;
  if ((e = check_field(R)) || (e = check_field(T))) return e;
  if (c->storage == DISCO_STORAGE_FP16 && image_tiles(c->g) > kScratchDoubles) return DISCO_ERR_LIMIT;
  if ((e = set_device(c))) return e;
  double *blk = nullptr;
  if ((e = scratch_ptr(c->device, &blk))) return e;
  hipStream_t s = S(stream);
  c->images = false;
  c->lin = false;
  // every block writes its maximum before the reduction reads it: nothing to clear
  // (no profiling scope here: it creates events)
  if ((e = build_gradients(c, R, T, s, blk))) return e;
  c->images = true;
  return DISCO_OK;
}

int disco_set_moving(disco_ctx *c, const float *T, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  int e;
  if ((e = check_field(T))) return e;
  if (!c->images) return DISCO_ERR_STATE;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  double *blk = nullptr;
  if ((e = image_scratch(c, s, &blk))) return e;
  ProfScope ps(c, 3, s);
  c->lin = false;
  if ((e = build_gradients(c, nullptr, T, s, blk))) {
    c->images = false;
    return e;
  }
  return DISCO_OK;
}

int disco_set_keypoints(disco_ctx *c, int32_t n, const float *x_mm, const float *t_mm, disco_stream stream) {
  if (!c || n < 0) return DISCO_ERR_ARG;
  if (n > 0 && (!x_mm || !t_mm)) return DISCO_ERR_ARG;
  int e;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  const Geo &g = c->g;
  const double H[3] = {4.0 * (double)g.hx, 4.0 * (double)g.hy, 4.0 * (double)g.hz};
  const int ncell[3] = {g.cx, g.cy, g.cz};
  std::vector<int64_t> cell(n);
  std::vector<float> loc(3 * (size_t)n), tgt(3 * (size_t)n);
  std::vector<int> order(n);
  for (int32_t i = 0; i < n; ++i) {
    int cidx[3];
    for (int a = 0; a < 3; ++a) {
      const double x = (double)x_mm[3 * i + a];
      const double xi = x / H[a];
      if (!(xi >= 0.0 && xi <= (double)ncell[a])) return DISCO_ERR_SHAPE;
      int ci = (int)std::floor(xi);
      if (ci > ncell[a] - 1) ci = ncell[a] - 1;
      cidx[a] = ci;
    }
    if (!std::isfinite((double)t_mm[3 * i]) || !std::isfinite((double)t_mm[3 * i + 1]) ||
        !std::isfinite((double)t_mm[3 * i + 2]))
      return DISCO_ERR_NONFINITE;
    cell[i] = ((int64_t)cidx[2] * g.cy + cidx[1]) * g.cx + cidx[0];
    for (int a = 0; a < 3; ++a) {
      const double origin = (double)cidx[a] * H[a];
      loc[3 * i + a] = (float)((double)x_mm[3 * i + a] - origin);
      tgt[3 * i + a] = (float)((double)t_mm[3 * i + a] - origin);
    }
  }
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cell[a] < cell[b]; });
  std::vector<float> sloc(3 * (size_t)n), stgt(3 * (size_t)n);
  std::vector<int> start((size_t)c->ncells + 1, 0);
  for (int32_t k = 0; k < n; ++k) {
    const int i = order[k];
    for (int a = 0; a < 3; ++a) {
      sloc[3 * k + a] = loc[3 * i + a];
      stgt[3 * k + a] = tgt[3 * i + a];
    }
    start[cell[i] + 1]++;
  }
  for (int64_t q = 0; q < c->ncells; ++q) start[q + 1] += start[q];
  HIP_TRY(hipStreamSynchronize(s));
  if (c->kloc) (void)hipFree(c->kloc);
  if (c->ktgt) (void)hipFree(c->ktgt);
  c->kloc = c->ktgt = nullptr;
  c->nkp = 0;
  if (n > 0) {
    if (hipMalloc(reinterpret_cast<void **>(&c->kloc), sizeof(float) * 3 * (size_t)n) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&c->ktgt), sizeof(float) * 3 * (size_t)n) != hipSuccess)
      return DISCO_ERR_NOMEM;
    HIP_TRY(hipMemcpy(c->kloc, sloc.data(), sizeof(float) * 3 * (size_t)n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->ktgt, stgt.data(), sizeof(float) * 3 * (size_t)n, hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMemcpy(c->kstart, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice));
  c->nkp = n;
  return DISCO_OK;
}

int disco_set_reference(disco_ctx *c, const float *u_ref, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  int e;
  if ((e = set_device(c))) return e;
  if (!u_ref) {
    if (c->u_ref) {
      HIP_TRY(hipStreamSynchronize(S(stream)));
      (void)hipFree(c->u_ref);
    }
    c->u_ref = nullptr;
    return DISCO_OK;
  }
  if ((e = check_field(u_ref))) return e;
  if (!c->u_ref && hipMalloc(reinterpret_cast<void **>(&c->u_ref), 3 * sizeof(float) * (size_t)c->g.nnodes) != hipSuccess)
    return DISCO_ERR_NOMEM;
  HIP_TRY(hipMemcpyAsync(c->u_ref, u_ref, 3 * sizeof(float) * (size_t)c->g.nnodes, hipMemcpyDeviceToDevice,
                         S(stream)));
  return DISCO_OK;
}

int disco_set_masks(disco_ctx *c, const uint8_t *bF, const uint8_t *bM, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  if ((bF == nullptr) != (bM == nullptr)) return DISCO_ERR_ARG;
  int e;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  const Geo &g = c->g;
  if (!bF) {
    c->masks = false;
    c->lin_mask = false;
    return DISCO_OK;
  }
  if (!c->mF) {
    HIP_TRY(hipStreamSynchronize(s));
    const size_t nrow = (size_t)g.nz * g.ny * g.nbx;
    bool okm = hipMalloc(reinterpret_cast<void **>(&c->mF), (size_t)g.nvox) == hipSuccess &&
               hipMalloc(reinterpret_cast<void **>(&c->mM), (size_t)g.nvox) == hipSuccess &&
               hipMalloc(reinterpret_cast<void **>(&c->rflag), nrow) == hipSuccess &&
               hipMalloc(reinterpret_cast<void **>(&c->sbc), sizeof(float) * 3 * (size_t)g.nvox) == hipSuccess &&
               hipMalloc(reinterpret_cast<void **>(&c->zb), sizeof(float) * 3 * 64) == hipSuccess &&
               hipMemset(c->zb, 0, sizeof(float) * 3 * 64) == hipSuccess &&
               hipMemset(c->rflag, 0, nrow) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    if (!okm) {
      void *ps[] = {c->mF, c->mM, c->rflag, c->sbc, c->zb};
      for (void *q : ps)
        if (q) (void)hipFree(q);
      c->mF = c->mM = c->rflag = nullptr;
      c->sbc = c->zb = nullptr;
      return DISCO_ERR_NOMEM;
    }
  }
  HIP_TRY(hipMemcpyAsync(c->mF, bF, (size_t)g.nvox, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(c->mM, bM, (size_t)g.nvox, hipMemcpyDeviceToDevice, s));
  c->masks = true;
  c->lin_mask = false;
  return DISCO_OK;
}

int ngf_eval(disco_ctx *c, double eta, const float *u, double *D_dev, disco_stream stream) {
  if (!c || !D_dev) return DISCO_ERR_ARG;
  int e;
  if ((e = check_field(u))) return e;
  if (!std::isfinite(eta) || !(eta > 0.0)) return DISCO_ERR_NONFINITE;
  if (!c->images) return DISCO_ERR_STATE;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  PostArgs pa = post_args(c);
  pa.dst = D_dev;
  pa.idx = BS_D;
  pa.scale = h3_of(c);
  BrickCall b{M_EVAL, true, false, false, (float)(eta * eta), 0.f, 0.f, u, nullptr, nullptr, nullptr, nullptr};
  launch_brick(c, b, s);
  launch_finish(POST_WRITE, pa, nullptr, s, src_brick(c, c->sc + SC_TMP0));
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

int ngf_grad(disco_ctx *c, double eta, const float *u, double *D_dev, float *g, float *diag, disco_stream stream) {
  if (!c || !D_dev) return DISCO_ERR_ARG;
  int e;
  if ((e = check_field(u)) || (e = check_field(g))) return e;
  if (diag && !aligned4(diag)) return DISCO_ERR_SHAPE;
  if (!std::isfinite(eta) || !(eta > 0.0)) return DISCO_ERR_NONFINITE;
  if (!c->images) return DISCO_ERR_STATE;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  float *d1 = diag ? diag : c->tmp1;
  set_s_scale(c, eta);
  PostArgs pa = post_args(c);
  pa.dst = D_dev;
  pa.idx = BS_D;
  pa.scale = h3_of(c);
  BrickCall b{M_GRAD, true, false, false, (float)(eta * eta), 0.f, 0.f, u, nullptr, g, d1, nullptr};
  launch_brick(c, b, s);
  launch_finish(POST_WRITE, pa, nullptr, s, src_brick(c, c->sc + SC_TMP0));
  launch_gather(c, 2, 2, g, d1, nullptr, 0.f, 0, nullptr, 0.f, nullptr, false, nullptr, s);
  HIP_TRY(hipMemcpyAsync(c->u_lin, u, 3 * sizeof(float) * (size_t)c->g.nnodes, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipGetLastError());
  c->lin = true;
  c->lin_eta = eta;
  c->lin_mask = false;
  return DISCO_OK;
}

int ngf_hessvec(disco_ctx *c, const float *v, float *Hv, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  int e;
  if ((e = check_field(v)) || (e = check_field(Hv))) return e;
  if (!c->lin) return DISCO_ERR_STATE;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  BrickCall b{M_HV, true, false, false, 0.f, 0.f, 0.f, c->u_lin, v, Hv, nullptr, nullptr};
  launch_brick(c, b, s);
  launch_gather(c, 1, 1, Hv, nullptr, nullptr, 0.f, 0, nullptr, 0.f, nullptr, false, nullptr, s);
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

int curvature_apply(disco_ctx *c, double alpha, const float *u, const float *u_ref, double *S_dev, float *out,
                    float *diag, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  int e;
  if ((e = check_field(u))) return e;
  if ((u_ref && !aligned4(u_ref)) || (out && !aligned4(out)) || (diag && !aligned4(diag))) return DISCO_ERR_SHAPE;
  if (!finite_nonneg(alpha)) return DISCO_ERR_NONFINITE;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  const double CH = ch_of(c);
  PostArgs pa = post_args(c);
  pa.dst = S_dev;
  pa.idx = 0;
  pa.scale = 0.5 * CH * alpha;
  launch_curv_L(c, u, u_ref, c->Lw, S_dev != nullptr, nullptr, s);
  if (S_dev) launch_finish(POST_WRITE, pa, nullptr, s, src_curv(c, c->sc + SC_TMP0));
  if (out || diag) {
    float *o0 = out ? out : c->tmp0;
    float *o1 = diag ? diag : c->tmp1;
    launch_gather(c, 0, diag ? 2 : 1, o0, o1, c->Lw, (float)(alpha * CH), diag ? 1 : 0, nullptr, 0.f, nullptr,
                  false, nullptr, s);
  }
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

static int cell_term(disco_ctx *c, bool vcc, double w, const float *u, double *E_dev, float *g, float *diag,
                     const float *v, float *Hv, int32_t *nfold_dev, hipStream_t s) {
  int e;
  if ((e = check_field(u))) return e;
  if ((g && !aligned4(g)) || (diag && !aligned4(diag)) || (v && !aligned4(v)) || (Hv && !aligned4(Hv)))
    return DISCO_ERR_SHAPE;
  if ((v == nullptr) != (Hv == nullptr)) return DISCO_ERR_ARG;
  if (!finite_nonneg(w)) return DISCO_ERR_NONFINITE;
  if ((e = set_device(c))) return e;
  const float wf = (float)w;
  if (E_dev || nfold_dev || g || diag) {
    const bool grad = g || diag;
    PostArgs pa = post_args(c);
    pa.dst = E_dev;
    pa.idst = nfold_dev;
    pa.idx = vcc ? BS_V : BS_K;
    pa.fold_idx = BS_FOLD;
    pa.fold_inf = vcc ? 1 : 0;
    pa.scale = w;
    BrickCall b{grad ? M_GRAD : M_EVAL, false, vcc, !vcc, 0.f, vcc ? wf : 0.f, vcc ? 0.f : wf, u, nullptr,
                g ? g : c->tmp0, diag ? diag : c->tmp1, nullptr};
    launch_brick(c, b, s);
    launch_finish(POST_WRITE, pa, nullptr, s, src_brick(c, c->sc + SC_TMP0));
    if (grad)
      launch_gather(c, 2, 2, g ? g : c->tmp0, diag ? diag : c->tmp1, nullptr, 0.f, 0, nullptr, 0.f, nullptr, false,
                    nullptr, s);
  }
  if (v) {
    BrickCall b{M_HV, false, vcc, !vcc, 0.f, vcc ? wf : 0.f, vcc ? 0.f : wf, u, v, Hv, nullptr, nullptr};
    launch_brick(c, b, s);
    launch_gather(c, 1, 1, Hv, nullptr, nullptr, 0.f, 0, nullptr, 0.f, nullptr, false, nullptr, s);
  }
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

int volchange_eval(disco_ctx *c, double gamma, const float *u, double *V_dev, float *g, float *diag, const float *v,
                   float *Hv, int32_t *nfold_dev, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  return cell_term(c, true, gamma, u, V_dev, g, diag, v, Hv, nfold_dev, S(stream));
}

int keypoint_penalty(disco_ctx *c, double delta, const float *u, double *K_dev, float *g, float *diag,
                     const float *v, float *Hv, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  return cell_term(c, false, delta, u, K_dev, g, diag, v, Hv, nullptr, S(stream));
}

static int check_params(const disco_params *p) {
  if (!p) return DISCO_ERR_ARG;
  if (!std::isfinite(p->eta) || !(p->eta > 0.0)) return DISCO_ERR_NONFINITE;
  if (!finite_nonneg(p->alpha) || !finite_nonneg(p->gamma) || !finite_nonneg(p->delta) || !finite_nonneg(p->tau) ||
      !finite_nonneg(p->pcg_tol) || !finite_nonneg(p->beta))
    return DISCO_ERR_NONFINITE;
  if (!std::isfinite(p->armijo_c1) || !(p->armijo_c1 > 0.0 && p->armijo_c1 < 1.0)) return DISCO_ERR_NONFINITE;
  if (p->pcg_iters < 1 || p->ls_max < 1 || p->ls_max > 60) return DISCO_ERR_ARG;
  return DISCO_OK;
}

// H v at the context's linearisation, all terms of eq. 11; with `dot` the gather also
// writes per-block <v, Hv> (blk_node, stride 3)
// GN product after L v is in c->Lw: brick pass (NGF, VCC, keypoints), then the gather
// (face nodes, curvature, damping, optional per-block <v, Hv>)
static void gn_hv_body(disco_ctx *c, const disco_params *p, const float *v, float *Hv, bool dot,
                       const double *stop, hipStream_t s) {
  const bool vcc = p->gamma != 0.0;
  const bool kp = p->delta != 0.0 && c->nkp > 0;
  const bool curv = p->alpha != 0.0;
  BrickCall b{M_HV, true, vcc, kp, 0.f, (float)p->gamma, (float)p->delta, c->u_lin, v, Hv, nullptr, stop};
  b.beta = p->beta;
  launch_brick(c, b, s);
  launch_gather(c, 1, 1, Hv, nullptr, curv ? c->Lw : nullptr, (float)(p->alpha * ch_of(c)), 0,
                p->tau != 0.0 ? v : nullptr, (float)p->tau, dot ? v : nullptr, dot, stop, s);
}

static void gn_hv_launch(disco_ctx *c, const disco_params *p, const float *v, float *Hv, bool dot,
                         const double *stop, hipStream_t s) {
  if (p->alpha != 0.0) launch_curv_L(c, v, nullptr, c->Lw, false, stop, s);
  gn_hv_body(c, p, v, Hv, dot, stop, s);
}

int gn_hessvec(disco_ctx *c, const disco_params *p, const float *v, float *Hv, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  int e;
  if ((e = check_params(p))) return e;
  if ((e = check_field(v)) || (e = check_field(Hv))) return e;
  if (!c->lin) return DISCO_ERR_STATE;
  // the boundary term's GN vectors come from a linearisation with the term
  if (p->beta != 0.0 && c->masks && !c->lin_mask) return DISCO_ERR_STATE;
  if ((e = set_device(c))) return e;
  gn_hv_launch(c, p, v, Hv, false, nullptr, S(stream));
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

// linearisation of a step at u: J and its parts (device scalars), grad J (vg), diag of
// the GN matrix (vdiag), s cache; u_lin = u
static int linearise(disco_ctx *c, const disco_params *p, const float *u, const PostArgs &pa, hipStream_t s) {
  const bool vcc = p->gamma != 0.0;
  const bool kp = p->delta != 0.0 && c->nkp > 0;
  const bool curv = p->alpha != 0.0;
  const float eta2 = (float)(p->eta * p->eta);
  double *sc = c->sc;
  set_s_scale(c, p->eta);
  launch_curv_L(c, u, c->u_ref, c->Lw, true, nullptr, s);
  BrickCall b{M_GRAD, true, vcc, kp, eta2, (float)p->gamma, (float)p->delta, u, nullptr, c->vg, c->vdiag, nullptr};
  b.beta = p->beta;
  launch_brick(c, b, s);
  launch_gather(c, 2, 2, c->vg, c->vdiag, curv ? c->Lw : nullptr, (float)(p->alpha * ch_of(c)), curv ? 1 : 0, nullptr,
                0.f, nullptr, true, nullptr, s);
  // D, V, K, folds; sum (L(u - uhat))^2; max diag, |g|^2 -> J
  launch_finish(POST_LIN_BRICK, pa, nullptr, s, src_brick(c, sc + SC_TMP0), src_curv(c, sc + SC_SRAW),
                src_gather(c, sc + SC_DOT));
  HIP_TRY(hipMemcpyAsync(c->u_lin, u, sizeof(float) * 3 * c->g.nnodes, hipMemcpyDeviceToDevice, s));
  c->lin = true;
  c->lin_eta = p->eta;
  c->lin_mask = p->beta != 0.0 && c->masks;
  return DISCO_OK;
}

// Armijo backtracking along vx from u (t = 1, 1/2, ...); before u is replaced, `pre`
// runs (it may read u, vut and the acceptance flag); then the report
extern "C++" {
template <class Pre>
static int line_search(disco_ctx *c, const disco_params *p, float *u, const PostArgs &pa, double *report_dev,
                       int32_t *status_dev, hipStream_t s, Pre pre) {
  const Geo &g = c->g;
  const int64_t n3 = 3 * g.nnodes;
  const unsigned nb3 = nblk(n3);
  double *sc = c->sc;
  const bool vcc = p->gamma != 0.0;
  const bool kp = p->delta != 0.0 && c->nkp > 0;
  const float eta2 = (float)(p->eta * p->eta);
  hipLaunchKernelGGL(k_dot, dim3(nb3), dim3(256), 0, s, n3, c->vg, c->vx, c->blk_node);
  launch_finish(POST_LS_BEGIN, pa, nullptr, s, src_pairs(c->blk_node, nb3, 1, sc + SC_TMP0),
                src_pairs(c->blk_upd, upd_blocks(g), 2, sc + SC_TMP1));
  const double *acc = sc + SC_ACCEPT;
  const bool dev_ls = (p->flags & DISCO_FLAG_LS_DEVICE) != 0;
  for (int t = 0; t < p->ls_max; ++t) {
    hipLaunchKernelGGL(k_ls_point, dim3(nb3), dim3(256), 0, s, n3, sc, t, u, c->vx, c->vut);
    launch_curv_L(c, c->vut, c->u_ref, c->Lw, true, acc, s);
    BrickCall b{M_EVAL, true, vcc, kp, eta2, (float)p->gamma, (float)p->delta, c->vut, nullptr, nullptr, nullptr, acc};
    b.beta = p->beta;
    launch_brick(c, b, s);
    launch_finish(POST_LS_BRICK, pa, acc, s, src_brick(c, sc + SC_TMP0), src_curv(c, sc + SC_TSRAW));
    if (!dev_ls) {
      // the acceptance flag of trial t is copied to the host and read once trial t + 1 is
      // enqueued, so the GPU runs the next trial while the host waits; a trial enqueued
      // after the accepted one does nothing (its kernels test the flag first)
      HIP_TRY(hipMemcpyAsync(c->host_sc + (t & 1), sc + SC_ACCEPT, sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipEventRecord(c->ls_ev[t & 1], s));
      if (t > 0) {
        HIP_TRY(hipEventSynchronize(c->ls_ev[(t - 1) & 1]));
        if (c->host_sc[(t - 1) & 1] != 0.0) break;
      }
    }
  }
  pre();
  hipLaunchKernelGGL(k_ls_finish, dim3(nb3), dim3(256), 0, s, n3, sc, c->vut, u);
  hipLaunchKernelGGL(k_report, dim3(1), dim3(1), 0, s, sc, ch_of(c), report_dev, c->status, status_dev);
  return DISCO_OK;
}
}  // extern "C++"

static int check_lbfgs(const disco_lbfgs *lb) {
  if (!lb) return DISCO_ERR_ARG;
  if (lb->m < 1 || lb->m > kLbfgsMax || lb->h0_iters < 1) return DISCO_ERR_ARG;
  if (!std::isfinite(lb->tau) || !(lb->tau > 0.0) || !finite_nonneg(lb->curv_eps) || !finite_nonneg(lb->h0_tol))
    return DISCO_ERR_NONFINITE;
  return DISCO_OK;
}

int lbfgs_reset(disco_ctx *c) {
  if (!c) return DISCO_ERR_ARG;
  c->lb_count = 0;
  c->lb_next = 0;
  c->lb_pending = false;
  return DISCO_OK;
}

int lbfgs_step(disco_ctx *c, const disco_params *p, const disco_lbfgs *lb, float *u, double *report_dev,
               int32_t *status_dev, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  int e;
  if ((e = check_params(p)) || (e = check_lbfgs(lb))) return e;
  if ((e = check_field(u))) return e;
  if ((report_dev && ((reinterpret_cast<uintptr_t>(report_dev) & 7u) != 0)) ||
      (status_dev && !aligned4(status_dev)))
    return DISCO_ERR_SHAPE;
  if (!c->images) return DISCO_ERR_STATE;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  const Geo &g = c->g;
  const int64_t n3 = 3 * g.nnodes;
  const unsigned nb3 = nblk(n3);
  double *sc = c->sc;
  if (c->lb_m != lb->m) {
    // new history length: fresh history in new buffers
    HIP_TRY(hipStreamSynchronize(s));
    if (c->lbS) (void)hipFree(c->lbS);
    if (c->lbY) (void)hipFree(c->lbY);
    c->lbS = c->lbY = nullptr;
    c->lb_m = 0;
    lbfgs_reset(c);
    const size_t bytes = sizeof(float) * (size_t)lb->m * (size_t)n3;
    if (hipMalloc(reinterpret_cast<void **>(&c->lbS), bytes) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&c->lbY), bytes) != hipSuccess) {
      if (c->lbS) (void)hipFree(c->lbS);
      c->lbS = c->lbY = nullptr;
      return DISCO_ERR_NOMEM;
    }
    c->lb_m = lb->m;
  }
  const int m = c->lb_m;
  auto Sv = [&](int k) { return c->lbS + (size_t)k * n3; };
  auto Yv = [&](int k) { return c->lbY + (size_t)k * n3; };
  const bool curv = p->alpha != 0.0;
  PostArgs pa = post_args(c, p->alpha, p->gamma, p->delta);
  pa.beta = c->masks ? p->beta : 0.0;
  pa.c1 = p->armijo_c1;
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, s, c->status);

  // ---- J and grad J at u --------------------------------------------------------------
  if ((e = linearise(c, p, u, pa, s))) return e;

  // ---- complete the pair of the previous step: y = g - g_old, rho ---------------------
  if (c->lb_pending) {
    const int k = c->lb_next;
    hipLaunchKernelGGL(k_lb_pair, dim3(nb3), dim3(256), 0, s, n3, Sv(k), Yv(k), c->vg, c->blk_node);
    PostArgs pp = pa;
    pp.idx = k;
    pp.tol = lb->curv_eps;
    launch_finish(POST_LB_PAIR, pp, nullptr, s, RedSrc{c->blk_node, (int64_t)nb3, 3, 3, 0u, sc + SC_TMP0});
    c->lb_count = std::min(c->lb_count + 1, m);
    c->lb_next = (k + 1) % m;
    c->lb_pending = false;
  }
  const int cnt = c->lb_count;
  auto slot = [&](int age) { return ((c->lb_next - 1 - age) % m + m) % m; };  // age 0 = newest

  // ---- first loop, newest to oldest: alpha_i = rho_i s_i.q, q -= alpha_i y_i ---------
  const float *q = c->vg;
  if (cnt > 0) {
    hipLaunchKernelGGL(k_dot, dim3(nb3), dim3(256), 0, s, n3, Sv(slot(0)), c->vg, c->blk_node);
    for (int age = 0; age < cnt; ++age) {
      const int k = slot(age);
      PostArgs pp = pa;
      pp.idx = k;
      launch_finish(POST_LB_ALPHA, pp, nullptr, s, src_pairs(c->blk_node, nb3, 1, sc + SC_TMP0));
      const bool more = age + 1 < cnt;
      hipLaunchKernelGGL(k_lb_axpy, dim3(nb3), dim3(256), 0, s, n3, 1.0f, q, Yv(k), c->tmp1, sc, 0.0,
                         SC_LB_ALPHA + k, -1.0, -1, 0, 0.0, more ? Sv(slot(age + 1)) : nullptr,
                         more ? c->blk_node : nullptr);
      q = c->tmp1;
    }
  }

  // ---- x = -H0^{-1} q by Jacobi-PCG, H0 = alpha C_H L^T L + tau I -----------------------
  // diagonal of alpha C_H L^T L (the tau part is added by the CG start)
  launch_gather(c, 0, 2, c->tmp0, c->vdiag, curv ? c->Lw : nullptr, (float)(p->alpha * ch_of(c)), curv ? 1 : 0,
                nullptr, 0.f, nullptr, false, nullptr, s);
  hipLaunchKernelGGL(k_pcg_init, dim3(nb3), dim3(256), 0, s, n3, q, c->vdiag, sc, (float)lb->tau, -1.0f, c->vx, c->vr,
                     c->vz, c->vp, c->vinvm, c->blk_node);
  launch_finish(POST_PCG_START, pa, nullptr, s, src_pairs(c->blk_node, nb3, 2, sc + SC_TMP0));
  {
    const double *stop = sc + SC_STOP;
    const int64_t nbu = upd_blocks(g);
    float *P[2] = {c->vp, c->vp2};
    for (int it = 0; it < lb->h0_iters; ++it) {
      float *pv = P[it & 1];
      if (it == 0) {
        if (curv) launch_curv_L(c, pv, nullptr, c->Lw, false, stop, s);
      } else {
        hipLaunchKernelGGL(k_curv_Lp, lp_grid(g), dim3(256), 0, s, g, it, sc, lb->h0_tol, c->blk_upd, nbu, c->vz,
                           P[(it - 1) & 1], pv, c->Lw);
      }
      launch_gather(c, 0, 1, c->vq, nullptr, curv ? c->Lw : nullptr, (float)(p->alpha * ch_of(c)), 0, pv,
                    (float)lb->tau, pv, true, stop, s);
      hipLaunchKernelGGL(k_pcg_update, dim3((unsigned)nbu), dim3(256), 0, s, n3, sc, it, c->blk_node, c->nodeblocks,
                         c->vinvm, pv, c->vq, c->vx, c->vr, c->vz, c->blk_upd, c->status);
    }
  }

  // ---- second loop, oldest to newest on x = -r: x += (-alpha_i - rho_i y_i.x) s_i -------
  if (cnt > 0) {
    hipLaunchKernelGGL(k_dot, dim3(nb3), dim3(256), 0, s, n3, Yv(slot(cnt - 1)), c->vx, c->blk_node);
    for (int age = cnt - 1; age >= 0; --age) {
      const int k = slot(age);
      launch_finish(POST_STORE, pa, nullptr, s, src_pairs(c->blk_node, nb3, 1, sc + SC_LB_DOT));
      const bool more = age > 0;
      hipLaunchKernelGGL(k_lb_axpy, dim3(nb3), dim3(256), 0, s, n3, 1.0f, c->vx, Sv(k), c->vx, sc, 0.0,
                         SC_LB_ALPHA + k, -1.0, SC_LB_RHO + k, SC_LB_DOT, -1.0, more ? Yv(slot(age - 1)) : nullptr,
                         more ? c->blk_node : nullptr);
    }
  }

  // ---- Armijo line search along x; the accepted step starts the next pair --------------
  float *Snext = Sv(c->lb_next), *Ynext = Yv(c->lb_next);
  if ((e = line_search(c, p, u, pa, report_dev, status_dev, s, [&] {
         hipLaunchKernelGGL(k_lb_save, dim3(nb3), dim3(256), 0, s, n3, sc, u, c->vut, c->vg, Snext, Ynext);
       })))
    return e;
  c->lb_pending = true;
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

int gn_pcg_step(disco_ctx *c, const disco_params *p, float *u, double *report_dev, int32_t *status_dev,
                disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  int e;
  if ((e = check_params(p))) return e;
  if ((e = check_field(u))) return e;
  if ((report_dev && ((reinterpret_cast<uintptr_t>(report_dev) & 7u) != 0)) ||
      (status_dev && !aligned4(status_dev)))
    return DISCO_ERR_SHAPE;
  if (!c->images) return DISCO_ERR_STATE;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  const Geo &g = c->g;
  const int64_t n3 = 3 * g.nnodes;
  const unsigned nb3 = nblk(n3);
  double *sc = c->sc;
  const bool curv = p->alpha != 0.0;
  PostArgs pa = post_args(c, p->alpha, p->gamma, p->delta);
  pa.beta = c->masks ? p->beta : 0.0;
  pa.c1 = p->armijo_c1;
  pa.tol = p->pcg_tol;
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, s, c->status);

  // ---- linearise at u: J, grad J, diag of the GN matrix, s cache --------------------
  if ((e = linearise(c, p, u, pa, s))) return e;

  // ---- Jacobi-PCG on (H + tau I) x = -g ----------------------------------------------
  hipLaunchKernelGGL(k_pcg_init, dim3(nb3), dim3(256), 0, s, n3, c->vg, c->vdiag, sc, (float)p->tau, -1.0f, c->vx,
                     c->vr, c->vz, c->vp, c->vinvm, c->blk_node);
  launch_finish(POST_PCG_START, pa, nullptr, s, src_pairs(c->blk_node, nb3, 2, sc + SC_TMP0));
  const double *stop = sc + SC_STOP;
  const int64_t nbu = upd_blocks(g);
  float *P[2] = {c->vp, c->vp2};  // search direction, alternating between iterations
  for (int it = 0; it < p->pcg_iters; ++it) {
    float *pv = P[it & 1];
    if (it == 0) {
      if (curv) launch_curv_L(c, pv, nullptr, c->Lw, false, stop, s);
    } else {
      // beta, convergence test, p = z + beta p and L p in one pass
      hipLaunchKernelGGL(k_curv_Lp, lp_grid(g), dim3(256), 0, s, g, it, sc, p->pcg_tol, c->blk_upd, nbu, c->vz,
                         P[(it - 1) & 1], pv, c->Lw);
    }
    gn_hv_body(c, p, pv, c->vq, true, stop, s);
    hipLaunchKernelGGL(k_pcg_update, dim3((unsigned)nbu), dim3(256), 0, s, n3, sc, it, c->blk_node, c->nodeblocks,
                       c->vinvm, pv, c->vq, c->vx, c->vr, c->vz, c->blk_upd, c->status);
  }

  // ---- Armijo line search on J(u + t x) ------------------------------------------------
  if ((e = line_search(c, p, u, pa, report_dev, status_dev, s, [] {}))) return e;
  HIP_TRY(hipGetLastError());
  // the s cache and u_lin now describe the linearisation point of this step
  return DISCO_OK;
}

int objective_linearise(disco_ctx *c, const disco_params *p, const float *u, double *terms_dev, float *g,
                        float *diag, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  int e;
  if ((e = check_params(p))) return e;
  if ((e = check_field(u))) return e;
  if ((g && !aligned4(g)) || (diag && !aligned4(diag)) ||
      (terms_dev && (reinterpret_cast<uintptr_t>(terms_dev) & 7u) != 0))
    return DISCO_ERR_SHAPE;
  if (!c->images) return DISCO_ERR_STATE;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  PostArgs pa = post_args(c, p->alpha, p->gamma, p->delta);
  pa.beta = c->masks ? p->beta : 0.0;
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, s, c->status);
  if ((e = linearise(c, p, u, pa, s))) return e;
  const size_t nf = sizeof(float) * 3 * (size_t)c->g.nnodes;
  if (g) HIP_TRY(hipMemcpyAsync(g, c->vg, nf, hipMemcpyDeviceToDevice, s));
  if (diag) HIP_TRY(hipMemcpyAsync(diag, c->vdiag, nf, hipMemcpyDeviceToDevice, s));
  if (terms_dev) hipLaunchKernelGGL(k_terms, dim3(1), dim3(1), 0, s, c->sc, ch_of(c), terms_dev);
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

int objective_eval(disco_ctx *c, const disco_params *p, const float *u, double *terms_dev, disco_stream stream) {
  if (!c || !terms_dev) return DISCO_ERR_ARG;
  int e;
  if ((e = check_params(p))) return e;
  if ((e = check_field(u))) return e;
  if ((reinterpret_cast<uintptr_t>(terms_dev) & 7u) != 0) return DISCO_ERR_SHAPE;
  if (!c->images) return DISCO_ERR_STATE;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  PostArgs pa = post_args(c, p->alpha, p->gamma, p->delta);
  pa.beta = c->masks ? p->beta : 0.0;
  pa.dst = terms_dev;
  const bool vcc = p->gamma != 0.0;
  const bool kp = p->delta != 0.0 && c->nkp > 0;
  launch_curv_L(c, u, c->u_ref, c->Lw, true, nullptr, s);
  BrickCall b{M_EVAL, true, vcc, kp, (float)(p->eta * p->eta), (float)p->gamma, (float)p->delta, u, nullptr, nullptr,
              nullptr, nullptr};
  b.beta = p->beta;
  launch_brick(c, b, s);
  launch_finish(POST_EVAL, pa, nullptr, s, src_brick(c, c->sc + SC_TMP0), src_curv(c, c->sc + SC_ESRAW));
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

int ngf_grad_T(disco_ctx *c, double eta, const float *u, const double *scale, float *dT, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  int e;
  if ((e = check_field(u)) || (e = check_field(dT))) return e;
  if (!std::isfinite(eta) || !(eta > 0.0)) return DISCO_ERR_NONFINITE;
  if (!c->images) return DISCO_ERR_STATE;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  const Geo &g = c->g;
  if (!c->adjW) {
    HIP_TRY(hipStreamSynchronize(s));
    if (hipMalloc(reinterpret_cast<void **>(&c->adjW), sizeof(float) * 3 * (size_t)g.nvox) != hipSuccess) {
      c->adjW = nullptr;
      return DISCO_ERR_NOMEM;
    }
  }
  ProfScope ps(c, 4, s);
  hipLaunchKernelGGL(k_fill, dim3(nblk(3 * g.nvox)), dim3(256), 0, s, 3 * g.nvox, c->adjW, 0.0f);
  const float h3x2 = (float)(2.0 * h3_of(c));
  // tiles of kAdjTX x kAdjTY x kAdjTZ voxels; fixed-point scale of the LDS box (the
  // kernel's header derives the bound; no scale when eta = 0)
  const dim3 adj_grid((g.nx + kAdjTX - 1) / kAdjTX, (g.ny + kAdjTY - 1) / kAdjTY, (g.nz + kAdjTZ - 1) / kAdjTZ);
  const double wbound = eta > 0.0 ? 2.0 * (double)h3x2 / eta : 0.0;
  double qs = wbound > 0.0 ? std::ldexp(1.0, 62) / (1.01 * kAdjTX * kAdjTY * kAdjTZ * wbound) : 0.0;
  if (!(qs > 0.0 && qs < 1e38 && 1.0 / qs > 1e-38)) qs = 0.0;
  const float fqs = (float)qs, fiqs = qs > 0.0 ? (float)(1.0 / qs) : 0.0f;
  if (c->storage == DISCO_STORAGE_FP16)
    hipLaunchKernelGGL(k_adjT_scatter<F16x3>, adj_grid, dim3(256), 0, s, g,
                       reinterpret_cast<const __half *>(c->gR), reinterpret_cast<const __half *>(c->gT), c->sR, c->sT,
                       u, (float)(eta * eta), h3x2, fqs, fiqs, c->adjW);
  else
    hipLaunchKernelGGL(k_adjT_scatter<F32x3>, adj_grid, dim3(256), 0, s, g,
                       reinterpret_cast<const float *>(c->gR), reinterpret_cast<const float *>(c->gT), 1.0f, 1.0f, u,
                       (float)(eta * eta), h3x2, fqs, fiqs, c->adjW);
  hipLaunchKernelGGL(k_adjT_stencil, vox_grid(g), dim3(256), 0, s, g, c->adjW, scale, dT);
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

int disco_copy_buffer(disco_ctx *c, int32_t which, float *dst, disco_stream stream) {
  if (!c) return DISCO_ERR_ARG;
  int e;
  if ((e = check_field(dst))) return e;
  if (which < 0 || which > 2) return DISCO_ERR_ARG;
  if (which < 2 && !c->images) return DISCO_ERR_STATE;
  if (which == 2 && !c->lin) return DISCO_ERR_STATE;
  if ((e = set_device(c))) return e;
  hipStream_t s = S(stream);
  const void *src = which == 0 ? c->gR : (which == 1 ? c->gT : c->scache);
  const float sc = which == 0 ? c->sR : (which == 1 ? c->sT : c->sS_load);
  if (c->storage == DISCO_STORAGE_FP16)
    hipLaunchKernelGGL(k_unpack3<F16x3>, dim3(nblk(c->g.nvox)), dim3(256), 0, s, c->g,
                       reinterpret_cast<const __half *>(src), sc, dst);
  else
    hipLaunchKernelGGL(k_unpack3<F32x3>, dim3(nblk(c->g.nvox)), dim3(256), 0, s, c->g,
                       reinterpret_cast<const float *>(src), 1.0f, dst);
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

int disco_profile(disco_ctx *c, int32_t enable) {
  if (!c) return DISCO_ERR_ARG;
  if (enable) {
    (void)hipDeviceSynchronize();
    clear_profile(c);
  }
  c->prof = enable != 0;
  return DISCO_OK;
}

int disco_profile_read(disco_ctx *c, int32_t kernel, int64_t *launches, double *ms_total) {
  if (!c || !launches || !ms_total || kernel < 0 || kernel > 4) return DISCO_ERR_ARG;
  double tot = 0.0;
  for (auto &p : c->ev[kernel]) {
    HIP_TRY(hipEventSynchronize(p.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p.a, p.b));
    tot += ms;
  }
  *launches = (int64_t)c->ev[kernel].size();
  *ms_total = tot;
  return DISCO_OK;
}

// ------------------------------------------------------------------------------
// batched GN step
// ------------------------------------------------------------------------------
enum { WL_BRICK = 0, WL_NODE = 1, WL_VEC = 2, WL_UPD = 3 };

// work lists of the batch (bricks of its tile, node blocks, 256-element vector blocks, CG
// update blocks): item offsets of every pair, copied to the device (synchronous)
static int batch_worklists(disco_batch *b) {
  const int npairs = (int)b->ctx.size();
  std::vector<int> st(4 * (size_t)(npairs + 1), 0);
  int64_t acc[4] = {0, 0, 0, 0};
  for (int i = 0; i < npairs; ++i) {
    const disco_ctx *c = b->ctx[i];
    const int64_t cnt[4] = {tile_bricks(c->g, b->zc), c->nodeblocks, (int64_t)nblk(3 * c->g.nnodes), upd_blocks(c->g)};
    for (int w = 0; w < 4; ++w) {
      st[w * (npairs + 1) + i] = (int)acc[w];
      acc[w] += cnt[w];
    }
  }
  for (int w = 0; w < 4; ++w) {
    if (acc[w] >= ((int64_t)1 << 31)) return DISCO_ERR_SHAPE;
    st[w * (npairs + 1) + npairs] = (int)acc[w];
  }
  if (hipMemcpy(b->start, st.data(), sizeof(int) * st.size(), hipMemcpyHostToDevice) != hipSuccess) return DISCO_ERR_NOMEM;
  return DISCO_OK;
}

static void batch_free_graph(disco_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

int disco_batch_create(int32_t npairs, disco_ctx *const *ctxs, disco_batch **out) {
  if (!out) return DISCO_ERR_ARG;
  *out = nullptr;
  if (npairs < 1 || !ctxs) return DISCO_ERR_ARG;
  for (int i = 0; i < npairs; ++i) {
    if (!ctxs[i]) return DISCO_ERR_ARG;
    if (ctxs[i]->device != ctxs[0]->device || ctxs[i]->storage != ctxs[0]->storage) return DISCO_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return DISCO_ERR_ARG;
  }
  disco_batch *b = new (std::nothrow) disco_batch();
  if (!b) return DISCO_ERR_NOMEM;
  b->device = ctxs[0]->device;
  b->storage = ctxs[0]->storage;
  // work order: largest pair first (balances the persistent loops)
  b->order.resize(npairs);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int a, int c) { return ctxs[a]->g.nvox > ctxs[c]->g.nvox; });
  for (int i = 0; i < npairs; ++i) b->ctx.push_back(ctxs[b->order[i]]);
  if (hipSetDevice(b->device) != hipSuccess) {
    delete b;
    return DISCO_ERR_ARG;
  }
  hipDeviceProp_t prop;
  b->ncu = hipGetDeviceProperties(&prop, b->device) == hipSuccess ? prop.multiProcessorCount : 256;
  const size_t dsz = b->storage == DISCO_STORAGE_FP16 ? sizeof(PairDesc<F16x3>) : sizeof(PairDesc<F32x3>);
  if (hipMalloc(&b->desc, dsz * (size_t)npairs) != hipSuccess ||
      hipMalloc(reinterpret_cast<void **>(&b->start), sizeof(int) * 4 * (size_t)(npairs + 1)) != hipSuccess) {
    (void)hipFree(b->desc);
    delete b;
    return DISCO_ERR_NOMEM;
  }
  const int e = batch_worklists(b);
  if (e) {
    (void)hipFree(b->desc);
    (void)hipFree(b->start);
    delete b;
    return e;
  }
  *out = b;
  return DISCO_OK;
}

void disco_batch_destroy(disco_batch *b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  batch_free_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  (void)hipFree(b->desc);
  (void)hipFree(b->start);
  delete b;
}

extern "C++" {
template <class ST>
static int batch_prepare_t(disco_batch *b, const disco_params *params, float *const *u, double *report_dev,
                           int32_t *status_dev) {
  const int n = (int)b->ctx.size();
  std::vector<PairDesc<ST>> d(n);
  for (int i = 0; i < n; ++i) {
    const int ci = b->order[i];
    d[i] = pair_desc<ST>(b->ctx[i], &params[ci], u[ci], report_dev ? report_dev + DISCO_REP_SIZE * (size_t)ci : nullptr,
                         status_dev ? status_dev + ci : nullptr, b->zc);
  }
  HIP_TRY(hipMemcpy(b->desc, d.data(), sizeof(PairDesc<ST>) * (size_t)n, hipMemcpyHostToDevice));
  return DISCO_OK;
}

}  // extern "C++"

int disco_batch_prepare(disco_batch *b, const disco_params *params, float *const *u, double *report_dev,
                        int32_t *status_dev) {
  if (!b || !params || !u) return DISCO_ERR_ARG;
  const int n = (int)b->ctx.size();
  int e;
  for (int i = 0; i < n; ++i) {
    if ((e = check_params(&params[i]))) return e;
    if ((e = check_field(u[i]))) return e;
    if (!(params[i].flags & DISCO_FLAG_LS_DEVICE)) return DISCO_ERR_ARG;  // no host round trips in a batch
    if (params[i].beta != 0.0) return DISCO_ERR_ARG;  // the batched passes have no boundary term
  }
  if ((report_dev && ((reinterpret_cast<uintptr_t>(report_dev) & 7u) != 0)) || (status_dev && !aligned4(status_dev)))
    return DISCO_ERR_SHAPE;
  // the terms present, the CG iteration count and the trial count are shared by the batch
  const disco_params &p0 = params[0];
  const bool vcc = p0.gamma != 0.0, curv = p0.alpha != 0.0;
  const bool kp = p0.delta != 0.0 && b->ctx[0]->nkp > 0;
  for (int i = 0; i < n; ++i) {
    const disco_ctx *c = b->ctx[i];
    const disco_params &pi = params[b->order[i]];
    if (!c->images) return DISCO_ERR_STATE;
    if ((pi.gamma != 0.0) != vcc || (pi.alpha != 0.0) != curv || ((pi.delta != 0.0 && c->nkp > 0) != kp) ||
        pi.pcg_iters != p0.pcg_iters || pi.ls_max != p0.ls_max)
      return DISCO_ERR_ARG;
  }
  if ((e = set_device(b->ctx[0]))) return e;
  batch_free_graph(b);
  b->prepared = false;
  b->vcc = vcc;
  b->kp = kp;
  b->curv = curv;
  b->pcg_iters = p0.pcg_iters;
  b->ls_max = p0.ls_max;
  e = b->storage == DISCO_STORAGE_FP16 ? batch_prepare_t<F16x3>(b, params, u, report_dev, status_dev)
                                       : batch_prepare_t<F32x3>(b, params, u, report_dev, status_dev);
  if (e) return e;
  b->prepared = true;
  return DISCO_OK;
}

int disco_batch_set_launch(disco_batch *b, int32_t pass, int32_t wg_per_cu) {
  if (!b || pass < 0 || pass > 2 || wg_per_cu < 0 || wg_per_cu > 64) return DISCO_ERR_ARG;
  b->wpc[pass] = wg_per_cu;
  batch_free_graph(b);  // a captured graph keeps the old launch shape
  return DISCO_OK;
}

int disco_batch_set_tile(disco_batch *b, int32_t cells_z) {
  if (!b || (cells_z != 2 && cells_z != 4)) return DISCO_ERR_ARG;
  int e;
  if ((e = set_device(b->ctx[0]))) return e;
  batch_free_graph(b);
  b->prepared = false;  // the descriptors carry the tile's brick geometry
  b->zc = cells_z;
  b->occ.clear();
  return batch_worklists(b);
}

extern "C++" {
// With a persistent grid (wpc > 0) the workgroups loop over the items, so a workgroup that
// is not resident from the start would begin only once a resident one has finished all of
// its items: such grids are capped at the kernel's residency (workgroups per compute unit
// for its register and LDS use, queried once per kernel and batch).  wpc = 0 launches one
// workgroup per item.
template <class F>
static unsigned b_cap(disco_batch *b, int pass, F f, int threads, unsigned grid) {
  if (b->wpc[pass] == 0) return grid;  // one workgroup per item
  const void *key = reinterpret_cast<const void *>(f);
  int o = 0;
  const auto it = b->occ.find(key);
  if (it != b->occ.end())
    o = it->second;
  else if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, f, threads, 0) == hipSuccess && o > 0)
    b->occ[key] = o;
  else
    o = 0;
  return o > 0 ? std::min(grid, (unsigned)(b->ncu * o)) : grid;
}

template <class ST, int MODE, bool NGF, bool VCC, bool KP>
static void b_brick_go(disco_batch *b, unsigned grid, const PairDesc<ST> *D, const int *st, int n, int sel, int acc,
                       hipStream_t s) {
  constexpr int threads = 256;
  if constexpr (MODE == M_HV && NGF && (VCC || KP)) {
    if (b->wpc[0] == 0) {  // one workgroup per item (grid = the items): the role-split product pass
      if (b->zc == 2)
        hipLaunchKernelGGL((k_b_brick_split<ST, VCC, KP, 2>), dim3(grid), dim3(512), 0, s, D, st, n, sel, acc);
      else
        hipLaunchKernelGGL((k_b_brick_split<ST, VCC, KP, 4>), dim3(grid), dim3(512), 0, s, D, st, n, sel, acc);
      return;
    }
  }
  if (b->wpc[0] == 0) {  // one workgroup per item (grid = the items): no work-item loop
    if (b->zc == 2)
      hipLaunchKernelGGL((k_b_brick_item<ST, MODE, NGF, VCC, KP, 2>), dim3(grid), dim3(threads), 0, s, D, st, n, sel, acc);
    else
      hipLaunchKernelGGL((k_b_brick_item<ST, MODE, NGF, VCC, KP, 4>), dim3(grid), dim3(threads), 0, s, D, st, n, sel, acc);
    return;
  }
  if (b->zc == 2) {
    const unsigned gr = b_cap(b, 0, k_b_brick<ST, MODE, NGF, VCC, KP, 2>, threads, grid);
    hipLaunchKernelGGL((k_b_brick<ST, MODE, NGF, VCC, KP, 2>), dim3(gr), dim3(threads), 0, s, D, st, n, sel, acc);
  } else {
    const unsigned gr = b_cap(b, 0, k_b_brick<ST, MODE, NGF, VCC, KP, 4>, threads, grid);
    hipLaunchKernelGGL((k_b_brick<ST, MODE, NGF, VCC, KP, 4>), dim3(gr), dim3(threads), 0, s, D, st, n, sel, acc);
  }
}

// gather of the batch's brick partials (sel as in k_b_gather), on the batch's tile
template <class ST, int F, int NF, bool CURV>
static void b_gather_go(disco_batch *b, unsigned grid, const PairDesc<ST> *D, const int *st, int n, int sel,
                        hipStream_t s) {
  if (b->zc == 2) {
    const unsigned gr = b_cap(b, 1, k_b_gather<ST, F, NF, CURV, 2>, 256, grid);
    hipLaunchKernelGGL((k_b_gather<ST, F, NF, CURV, 2>), dim3(gr), dim3(256), 0, s, D, st, n, sel);
  } else {
    const unsigned gr = b_cap(b, 1, k_b_gather<ST, F, NF, CURV, 4>, 256, grid);
    hipLaunchKernelGGL((k_b_gather<ST, F, NF, CURV, 4>), dim3(gr), dim3(256), 0, s, D, st, n, sel);
  }
}

template <class ST, int MODE, bool NGF>
static void launch_b_brick(disco_batch *b, unsigned grid, const int *st, int n, int sel, int acc, hipStream_t s) {
  const PairDesc<ST> *D = reinterpret_cast<const PairDesc<ST> *>(b->desc);
  const int key = (b->vcc ? 2 : 0) | (b->kp ? 1 : 0);
  if constexpr (NGF && MODE != M_HV) {
    b_brick_go<ST, MODE, true, false, false>(b, grid, D, st, n, sel, acc, s);
  } else if constexpr (NGF) {
    switch (key) {
      case 3: b_brick_go<ST, MODE, true, true, true>(b, grid, D, st, n, sel, acc, s); break;
      case 2: b_brick_go<ST, MODE, true, true, false>(b, grid, D, st, n, sel, acc, s); break;
      case 1: b_brick_go<ST, MODE, true, false, true>(b, grid, D, st, n, sel, acc, s); break;
      default: b_brick_go<ST, MODE, true, false, false>(b, grid, D, st, n, sel, acc, s); break;
    }
  } else {
    switch (key) {
      case 3: b_brick_go<ST, MODE, false, true, true>(b, grid, D, st, n, sel, acc, s); break;
      case 2: b_brick_go<ST, MODE, false, true, false>(b, grid, D, st, n, sel, acc, s); break;
      case 1: b_brick_go<ST, MODE, false, false, true>(b, grid, D, st, n, sel, acc, s); break;
      default: break;
    }
  }
}

template <class ST>
static void batch_step_t(disco_batch *b, hipStream_t s) {
  const int n = (int)b->ctx.size();
  const PairDesc<ST> *D = reinterpret_cast<const PairDesc<ST> *>(b->desc);
  const int *wl[4];
  int tot[4];
  for (int w = 0; w < 4; ++w) wl[w] = b->start + w * (n + 1);
  for (int w = 0; w < 4; ++w) {
    int64_t t = 0;
    for (auto *c : b->ctx)
      t += w == WL_BRICK ? tile_bricks(c->g, b->zc)
                         : (w == WL_NODE ? c->nodeblocks : (w == WL_VEC ? (int64_t)nblk(3 * c->g.nnodes) : upd_blocks(c->g)));
    tot[w] = (int)t;
  }
  // wpc 0: one workgroup per item (the hardware schedules them); else a persistent grid of
  // wpc workgroups per compute unit, capped at each kernel's residency
  auto grid = [&](int w, int pass) {
    return (unsigned)std::max(1, b->wpc[pass] == 0 ? tot[w] : std::min(tot[w], b->ncu * b->wpc[pass]));
  };
  const unsigned gb = grid(WL_BRICK, 0), gn = grid(WL_NODE, 1), gv = grid(WL_VEC, 2), gu = grid(WL_UPD, 2);
  const bool cells = b->vcc || b->kp;
  const unsigned pairs_grid = (unsigned)std::min(n, b->ncu * 4);

  hipLaunchKernelGGL(k_b_status<ST>, dim3((n + 63) / 64), dim3(64), 0, s, D, n, 0);
  // linearisation: objective, gradient, GN diagonal, s cache
  if (b->curv) hipLaunchKernelGGL(k_b_curv_L<ST>, dim3(b_cap(b, 1, k_b_curv_L<ST>, 256, gn)), dim3(256), 0, s, D, wl[WL_NODE], n, 0);
  if (cells) launch_b_brick<ST, M_GRAD, false>(b, gb, wl[WL_BRICK], n, 0, 0, s);
  launch_b_brick<ST, M_GRAD, true>(b, gb, wl[WL_BRICK], n, 0, cells ? 1 : 0, s);
  if (b->curv)
    b_gather_go<ST, 2, 2, true>(b, gn, D, wl[WL_NODE], n, 0, s);
  else
    b_gather_go<ST, 2, 2, false>(b, gn, D, wl[WL_NODE], n, 0, s);
  hipLaunchKernelGGL(k_b_finish<ST>, dim3(pairs_grid), dim3(1024), 0, s, D, n, 0);
  hipLaunchKernelGGL(k_b_vec<ST>, dim3(b_cap(b, 2, k_b_vec<ST>, 256, gv)), dim3(256), 0, s, D, wl[WL_VEC], n, 0, 0);  // u_lin = u
  // Jacobi-PCG
  hipLaunchKernelGGL(k_b_vec<ST>, dim3(b_cap(b, 2, k_b_vec<ST>, 256, gv)), dim3(256), 0, s, D, wl[WL_VEC], n, 1, 0);
  hipLaunchKernelGGL(k_b_finish<ST>, dim3(pairs_grid), dim3(1024), 0, s, D, n, 1);
  for (int it = 0; it < b->pcg_iters; ++it) {
    if (it == 0) {
      if (b->curv) hipLaunchKernelGGL(k_b_curv_L<ST>, dim3(b_cap(b, 1, k_b_curv_L<ST>, 256, gn)), dim3(256), 0, s, D, wl[WL_NODE], n, 1);
    } else {
      hipLaunchKernelGGL(k_b_curv_Lp<ST>, dim3(b_cap(b, 1, k_b_curv_Lp<ST>, 256, gn)), dim3(256), 0, s, D, wl[WL_NODE], n, it);
    }
    launch_b_brick<ST, M_HV, true>(b, gb, wl[WL_BRICK], n, 1 + (it & 1), 0, s);
    if (b->curv)
      b_gather_go<ST, 1, 1, true>(b, gn, D, wl[WL_NODE], n, 1 + (it & 1), s);
    else
      b_gather_go<ST, 1, 1, false>(b, gn, D, wl[WL_NODE], n, 1 + (it & 1), s);
    hipLaunchKernelGGL(k_b_pcg_update<ST>, dim3(b_cap(b, 2, k_b_pcg_update<ST>, 256, gu)), dim3(256), 0, s, D, wl[WL_UPD], n, it);
  }
  // Armijo line search on the device (ls_max trials, skipped once accepted)
  hipLaunchKernelGGL(k_b_vec<ST>, dim3(b_cap(b, 2, k_b_vec<ST>, 256, gv)), dim3(256), 0, s, D, wl[WL_VEC], n, 2, 0);
  hipLaunchKernelGGL(k_b_finish<ST>, dim3(pairs_grid), dim3(1024), 0, s, D, n, 2);
  for (int t = 0; t < b->ls_max; ++t) {
    hipLaunchKernelGGL(k_b_vec<ST>, dim3(b_cap(b, 2, k_b_vec<ST>, 256, gv)), dim3(256), 0, s, D, wl[WL_VEC], n, 3, t);
    hipLaunchKernelGGL(k_b_curv_L<ST>, dim3(b_cap(b, 1, k_b_curv_L<ST>, 256, gn)), dim3(256), 0, s, D, wl[WL_NODE], n, 2);
    if (cells) launch_b_brick<ST, M_EVAL, false>(b, gb, wl[WL_BRICK], n, 3, 0, s);
    launch_b_brick<ST, M_EVAL, true>(b, gb, wl[WL_BRICK], n, 3, cells ? 1 : 0, s);
    hipLaunchKernelGGL(k_b_finish<ST>, dim3(pairs_grid), dim3(1024), 0, s, D, n, 3);
  }
  hipLaunchKernelGGL(k_b_vec<ST>, dim3(b_cap(b, 2, k_b_vec<ST>, 256, gv)), dim3(256), 0, s, D, wl[WL_VEC], n, 4, 0);
  hipLaunchKernelGGL(k_b_status<ST>, dim3((n + 63) / 64), dim3(64), 0, s, D, n, 1);
}

}  // extern "C++"

static int batch_step(disco_batch *b, hipStream_t s) {
  if (b->storage == DISCO_STORAGE_FP16)
    batch_step_t<F16x3>(b, s);
  else
    batch_step_t<F32x3>(b, s);
  for (auto *c : b->ctx) {
    c->lin = true;
    c->lin_mask = false;
  }
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

int disco_batch_gn_step(disco_batch *b, disco_stream stream) {
  if (!b) return DISCO_ERR_ARG;
  if (!b->prepared) return DISCO_ERR_STATE;
  int e;
  if ((e = set_device(b->ctx[0]))) return e;
  return batch_step(b, S(stream));
}

int disco_batch_graph_capture(disco_batch *b, int32_t nsteps) {
  if (!b || nsteps < 1) return DISCO_ERR_ARG;
  if (!b->prepared) return DISCO_ERR_STATE;
  int e;
  if ((e = set_device(b->ctx[0]))) return e;
  batch_free_graph(b);
  if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  int err = DISCO_OK;
  for (int k = 0; k < nsteps && !err; ++k) err = batch_step(b, b->cap_stream);
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(b->cap_stream, &graph);
  if (err) {
    if (graph) (void)hipGraphDestroy(graph);
    return err;
  }
  if (ce != hipSuccess) return hip_err(ce);
  b->graph = graph;
  const hipError_t ie = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    batch_free_graph(b);
    return hip_err(ie);
  }
  return DISCO_OK;
}

int disco_batch_graph_launch(disco_batch *b, disco_stream stream) {
  if (!b) return DISCO_ERR_ARG;
  if (!b->exec) return DISCO_ERR_STATE;
  int e;
  if ((e = set_device(b->ctx[0]))) return e;
  HIP_TRY(hipGraphLaunch(b->exec, S(stream)));
  return DISCO_OK;
}

// ---- multilevel scheme (Sec. II-D3) ----------------------------------------------------

// the axes halved to go one level coarser: the valid non-empty subset (halved sizes
// divisible by 8, coarse size >= 8) with the most nearly isotropic coarse spacing; ties:
// more axes, then x before y before z.  false if none is valid.
static bool pyr_halving(const int32_t n[3], const double h[3], int32_t S[3]) {
  bool found = false;
  double best_ratio = 0.0;
  int best_cnt = 0;
  for (int mask = 1; mask < 8; ++mask) {
    bool ok = true;
    double hh[3];
    int cnt = 0;
    for (int a = 0; a < 3; ++a) {
      const bool s = (mask >> a) & 1;
      if (s && (n[a] % 8 != 0 || n[a] / 2 < 8)) ok = false;
      hh[a] = s ? h[a] * 2.0 : h[a];
      cnt += s;
    }
    if (!ok) continue;
    const double ratio = std::max(hh[0], std::max(hh[1], hh[2])) / std::min(hh[0], std::min(hh[1], hh[2]));
    if (!found || ratio < best_ratio || (ratio == best_ratio && cnt > best_cnt)) {
      found = true;
      best_ratio = ratio;
      best_cnt = cnt;
      for (int a = 0; a < 3; ++a) S[a] = (mask >> a) & 1;
    }
  }
  return found;
}

int pyramid_plan(const int32_t n[3], const double h[3], int32_t levels, int32_t *levels_out, int32_t *n_out,
                 double *h_out, int32_t *halve_out) {
  if (!n || !h || !levels_out || !n_out || !h_out || !halve_out) return DISCO_ERR_ARG;
  if (levels < 1 || levels > DISCO_MAX_LEVELS) return DISCO_ERR_ARG;
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 4 || n[a] % 4 != 0) return DISCO_ERR_SHAPE;
    if (!std::isfinite(h[a]) || !(h[a] > 0.0)) return DISCO_ERR_NONFINITE;
  }
  int L = 1;
  for (int a = 0; a < 3; ++a) {
    n_out[a] = n[a];
    h_out[a] = h[a];
    halve_out[a] = 0;
  }
  while (L < levels) {
    int32_t S[3];
    if (!pyr_halving(n_out + 3 * (L - 1), h_out + 3 * (L - 1), S)) break;
    for (int a = 0; a < 3; ++a) {
      n_out[3 * L + a] = S[a] ? n_out[3 * (L - 1) + a] / 2 : n_out[3 * (L - 1) + a];
      h_out[3 * L + a] = S[a] ? h_out[3 * (L - 1) + a] * 2.0 : h_out[3 * (L - 1) + a];
      halve_out[3 * L + a] = S[a];
    }
    ++L;
  }
  *levels_out = L;
  return DISCO_OK;
}

// combined taps of one downsampling pass: Gaussian (sigma = 1 finer voxel, taps -3..3,
// renormalised), then the mean of the two finer voxels a coarse voxel covers
static DownTaps down_taps() {
  double w[7], sum = 0.0;
  for (int k = -3; k <= 3; ++k) {
    w[k + 3] = std::exp(-0.5 * (double)(k * k));
    sum += w[k + 3];
  }
  DownTaps t;
  for (int m = -3; m <= 4; ++m) {
    const double a = (m <= 3) ? w[m + 3] / sum : 0.0;
    const double b = (m - 1 >= -3) ? w[m - 1 + 3] / sum : 0.0;
    t.c[m + 3] = (float)(0.5 * (a + b));
  }
  return t;
}

int pyramid_downsample(const float *src, const int32_t n[3], const int32_t halve[3], float *dst, float *work,
                       disco_stream stream) {
  if (!src || !n || !halve || !dst) return DISCO_ERR_ARG;
  int nh = 0;
  for (int a = 0; a < 3; ++a) {
    if (halve[a] != 0 && halve[a] != 1) return DISCO_ERR_ARG;
    if (n[a] < 1 || (halve[a] && (n[a] < 2 || n[a] % 2 != 0))) return DISCO_ERR_SHAPE;
    nh += halve[a];
  }
  if (nh == 0) return DISCO_ERR_ARG;
  if (nh >= 2 && !work) return DISCO_ERR_ARG;
  if (!aligned4(src) || !aligned4(dst) || (work && !aligned4(work))) return DISCO_ERR_SHAPE;
  hipStream_t s = S(stream);
  const DownTaps t = down_taps();
  int dims[3] = {n[0], n[1], n[2]};
  const int64_t N = (int64_t)n[0] * n[1] * n[2];
  // pass outputs: work[0, N/2), then work[N/2, 3N/4), the last pass into dst
  float *outs[2] = {work, work ? work + N / 2 : nullptr};
  const float *in = src;
  int done = 0;
  for (int a = 0; a < 3; ++a) {
    if (!halve[a]) continue;
    float *out = (done == nh - 1) ? dst : outs[done];
    int od[3] = {dims[0], dims[1], dims[2]};
    od[a] /= 2;
    const dim3 grid((unsigned)((od[0] + 255) / 256), (unsigned)od[1], (unsigned)od[2]);
    if (a == 0)
      hipLaunchKernelGGL(k_down_axis<0>, grid, dim3(256), 0, s, in, dims[0], dims[1], dims[2], out, t);
    else if (a == 1)
      hipLaunchKernelGGL(k_down_axis<1>, grid, dim3(256), 0, s, in, dims[0], dims[1], dims[2], out, t);
    else
      hipLaunchKernelGGL(k_down_axis<2>, grid, dim3(256), 0, s, in, dims[0], dims[1], dims[2], out, t);
    dims[a] = od[a];
    in = out;
    ++done;
  }
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

int pyramid_prolong(const float *uc, const int32_t nodes[3], const int32_t halve[3], float *uf, disco_stream stream) {
  if (!uc || !nodes || !halve || !uf) return DISCO_ERR_ARG;
  int f[3];
  for (int a = 0; a < 3; ++a) {
    if (halve[a] != 0 && halve[a] != 1) return DISCO_ERR_ARG;
    if (nodes[a] < 2) return DISCO_ERR_SHAPE;
    f[a] = halve[a] ? 2 * (nodes[a] - 1) + 1 : nodes[a];
  }
  if (!aligned4(uc) || !aligned4(uf)) return DISCO_ERR_SHAPE;
  const dim3 grid((unsigned)((f[0] + 255) / 256), (unsigned)f[1], (unsigned)f[2]);
  hipLaunchKernelGGL(k_prolong, grid, dim3(256), 0, S(stream), uc, nodes[0], nodes[1], nodes[2], halve[0], halve[1],
                     halve[2], uf, f[0], f[1], f[2]);
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

// device buffers of a multilevel run, freed together
extern "C++" {
struct MlBuffers {
  std::vector<void *> p;
  ~MlBuffers() {
    for (void *q : p)
      if (q) (void)hipFree(q);
  }
  template <class T>
  bool alloc(T **out, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) return false;
    p.push_back(q);
    *out = static_cast<T *>(q);
    return true;
  }
};
}  // extern "C++"

int multilevel_register(const disco_geom *geom, const float *R, const float *T, int32_t nkp, const float *kp_x,
                        const float *kp_t, const disco_multilevel *cfg, float *u_out, double *report_dev,
                        int32_t *levels_out, double *delta_out, disco_stream stream) {
  if (!geom || !R || !T || !cfg || !u_out) return DISCO_ERR_ARG;
  if (nkp < 0 || (nkp > 0 && (!kp_x || !kp_t))) return DISCO_ERR_ARG;
  int e;
  if ((e = check_params(&cfg->params))) {
    // a negative delta is allowed when it is replaced by the adaptive one
    disco_params q = cfg->params;
    if (cfg->adaptive_delta) q.delta = 0.0;
    if ((e = check_params(&q))) return e;
  }
  if (cfg->optimizer != DISCO_OPT_GN && cfg->optimizer != DISCO_OPT_LBFGS) return DISCO_ERR_ARG;
  if (cfg->optimizer == DISCO_OPT_LBFGS && (e = check_lbfgs(&cfg->lbfgs))) return e;
  if (cfg->storage != DISCO_STORAGE_FP32 && cfg->storage != DISCO_STORAGE_FP16) return DISCO_ERR_ARG;
  if (!aligned4(R) || !aligned4(T) || !aligned4(u_out) ||
      (report_dev && (reinterpret_cast<uintptr_t>(report_dev) & 7u) != 0))
    return DISCO_ERR_SHAPE;
  int32_t L = 0, ns[3 * DISCO_MAX_LEVELS], hv[3 * DISCO_MAX_LEVELS];
  double hs[3 * DISCO_MAX_LEVELS];
  if ((e = pyramid_plan(geom->n, geom->h, cfg->levels, &L, ns, hs, hv))) return e;
  for (int l = 0; l < L; ++l)
    if (cfg->iters[L - 1 - l] < 0) return DISCO_ERR_ARG;
  int64_t rows = 0;
  for (int l = 0; l < L; ++l) rows += cfg->iters[l];
  hipStream_t s = S(stream);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  MlBuffers B;
  // level images (level 0 is the caller's), one work buffer for the downsampling passes
  std::vector<const float *> Rl(L), Tl(L);
  std::vector<float *> ul(L);
  Rl[0] = R;
  Tl[0] = T;
  const int64_t N0 = (int64_t)ns[0] * ns[1] * ns[2];
  float *work = nullptr;
  if (L > 1 && !B.alloc(&work, (size_t)(N0 / 2 + N0 / 4 + 1))) return DISCO_ERR_NOMEM;
  for (int l = 1; l < L; ++l) {
    const int64_t Nl = (int64_t)ns[3 * l] * ns[3 * l + 1] * ns[3 * l + 2];
    float *r = nullptr, *t = nullptr;
    if (!B.alloc(&r, (size_t)Nl) || !B.alloc(&t, (size_t)Nl)) return DISCO_ERR_NOMEM;
    if ((e = pyramid_downsample(Rl[l - 1], ns + 3 * (l - 1), hv + 3 * l, r, work, stream)) ||
        (e = pyramid_downsample(Tl[l - 1], ns + 3 * (l - 1), hv + 3 * l, t, work, stream)))
      return e;
    Rl[l] = r;
    Tl[l] = t;
  }
  for (int l = 0; l < L; ++l) {
    const int64_t nn = 3LL * (ns[3 * l] / 4 + 1) * (ns[3 * l + 1] / 4 + 1) * (ns[3 * l + 2] / 4 + 1);
    if (l == 0)
      ul[0] = u_out;
    else if (!B.alloc(&ul[l], (size_t)nn))
      return DISCO_ERR_NOMEM;
  }
  double *scal = nullptr;  // D(0), K(0) of the adaptive keypoint weight
  int32_t *st_dev = nullptr;
  if (!B.alloc(&scal, 2) || !B.alloc(&st_dev, 1)) return DISCO_ERR_NOMEM;
  // rows of iterations that are not run read as NaN
  if (report_dev && rows > 0) HIP_TRY(hipMemsetAsync(report_dev, 0xFF, sizeof(double) * DISCO_REP_SIZE * (size_t)rows, s));

  disco_params prm = cfg->params;
  double delta = cfg->adaptive_delta ? 0.0 : prm.delta;
  int64_t row = 0;
  disco_ctx *prev = nullptr;
  for (int l = L - 1; l >= 0; --l) {
    disco_geom gl;
    for (int a = 0; a < 3; ++a) {
      gl.n[a] = ns[3 * l + a];
      gl.h[a] = hs[3 * l + a];
    }
    disco_ctx *c = nullptr;
    HIP_TRY(hipSetDevice(dev));
    if ((e = disco_create(&gl, cfg->storage, &c))) {
      disco_destroy(prev);
      return e;
    }
    auto fail = [&](int code) {
      disco_destroy(c);
      disco_destroy(prev);
      return code;
    };
    const int64_t n3 = 3 * c->g.nnodes;
    if ((e = disco_set_images(c, Rl[l], Tl[l], stream)) || (e = disco_set_keypoints(c, nkp, kp_x, kp_t, stream)))
      return fail(e);
    if (l == L - 1) {
      hipLaunchKernelGGL(k_fill, dim3(nblk(n3)), dim3(256), 0, s, n3, ul[l], 0.0f);
      if (cfg->adaptive_delta) {
        // delta with D = delta K at the start of the registration (Sec. II-D2)
        if ((e = ngf_eval(c, prm.eta, ul[l], scal, stream))) return fail(e);
        if (nkp > 0 && (e = keypoint_penalty(c, 1.0, ul[l], scal + 1, nullptr, nullptr, nullptr, nullptr, stream)))
          return fail(e);
        double hsc[2] = {0.0, 0.0};
        if (hipMemcpyAsync(hsc, scal, sizeof(double) * (nkp > 0 ? 2 : 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return fail(DISCO_ERR_HIP);
        delta = (nkp > 0 && hsc[1] > 0.0) ? hsc[0] / hsc[1] : 0.0;
      }
    } else {
      const int32_t nc[3] = {prev->g.px, prev->g.py, prev->g.pz};
      if ((e = pyramid_prolong(ul[l + 1], nc, hv + 3 * (l + 1), ul[l], stream))) return fail(e);
    }
    disco_destroy(prev);
    prev = nullptr;
    prm.delta = delta;
    const int iters = cfg->iters[L - 1 - l];
    for (int it = 0; it < iters; ++it) {
      double *rep = report_dev ? report_dev + DISCO_REP_SIZE * (row + it) : nullptr;
      e = cfg->optimizer == DISCO_OPT_GN ? gn_pcg_step(c, &prm, ul[l], rep, st_dev, stream)
                                         : lbfgs_step(c, &prm, &cfg->lbfgs, ul[l], rep, st_dev, stream);
      if (e) return fail(e);
      int32_t st = 0;
      if (hipMemcpyAsync(&st, st_dev, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(DISCO_ERR_HIP);
      if (st & DISCO_STATUS_LS_FAIL) break;  // no descent along this direction: next level
    }
    row += iters;
    prev = c;
  }
  disco_destroy(prev);
  if (levels_out) *levels_out = L;
  if (delta_out) *delta_out = delta;
  HIP_TRY(hipStreamSynchronize(s));
  return DISCO_OK;
}

// ---- keypoint stage (Sec. II-C2, II-C3) ---------------------------------------------------

int disco_kp_create(const int32_t n[3], const double h[3], disco_kp **out) {
  if (!out) return DISCO_ERR_ARG;
  *out = nullptr;
  if (!n || !h) return DISCO_ERR_ARG;
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1) return DISCO_ERR_SHAPE;
    if (!std::isfinite(h[a]) || !(h[a] > 0.0)) return DISCO_ERR_NONFINITE;
  }
  const int64_t nvox = (int64_t)n[0] * n[1] * n[2];
  if (nvox >= ((int64_t)1 << 31)) return DISCO_ERR_SHAPE;
  disco_kp *k = new (std::nothrow) disco_kp();
  if (!k) return DISCO_ERR_NOMEM;
  (void)hipGetDevice(&k->device);
  KpGeo &g = k->g;
  g.nx = n[0];
  g.ny = n[1];
  g.nz = n[2];
  g.hx = (n[0] + 1) / 2;
  g.hy = (n[1] + 1) / 2;
  g.hz = (n[2] + 1) / 2;
  g.ihx2 = (float)(0.5 / h[0]);
  g.ihy2 = (float)(0.5 / h[1]);
  g.ihz2 = (float)(0.5 / h[2]);
  for (int a = 0; a < 3; ++a) k->h[a] = h[a];
  const size_t entries = (size_t)8 * g.hx * g.hy * g.hz;
  if (hipMalloc(reinterpret_cast<void **>(&k->nF), sizeof(float4) * entries) != hipSuccess ||
      hipMalloc(reinterpret_cast<void **>(&k->nM), sizeof(float4) * entries) != hipSuccess) {
    if (k->nF) (void)hipFree(k->nF);
    delete k;
    return DISCO_ERR_NOMEM;
  }
  *out = k;
  return DISCO_OK;
}

void disco_kp_destroy(disco_kp *k) {
  if (!k) return;
  (void)hipSetDevice(k->device);
  (void)hipDeviceSynchronize();
  if (k->nF) (void)hipFree(k->nF);
  if (k->nM) (void)hipFree(k->nM);
  if (k->patch) (void)hipFree(k->patch);
  if (k->bp) (void)hipFree(k->bp);
  if (k->th) (void)hipHostFree(k->th);
  if (k->td) (void)hipFree(k->td);
  delete k;
}

int disco_kp_set_images(disco_kp *k, const float *F, const float *M, double eta, disco_stream stream) {
  if (!k || !F || !M) return DISCO_ERR_ARG;
  if (!aligned4(F) || !aligned4(M)) return DISCO_ERR_SHAPE;
  if (!std::isfinite(eta) || !(eta > 0.0)) return DISCO_ERR_NONFINITE;
  HIP_TRY(hipSetDevice(k->device));
  const KpGeo &g = k->g;
  const dim3 grid((unsigned)((g.hx + 255) / 256), (unsigned)g.hy, (unsigned)(8 * g.hz));
  hipLaunchKernelGGL(k_kp_normalize, grid, dim3(256), 0, S(stream), g, F, (float)eta, k->nF);
  hipLaunchKernelGGL(k_kp_normalize, grid, dim3(256), 0, S(stream), g, M, (float)eta, k->nM);
  HIP_TRY(hipGetLastError());
  k->images = true;
  return DISCO_OK;
}

int disco_kp_cost(disco_kp *k, int32_t nkp, const int32_t *kp_vox, int32_t R, float *cost, disco_stream stream) {
  if (!k || nkp < 0 || (nkp > 0 && (!kp_vox || !cost))) return DISCO_ERR_ARG;
  if (R < 1 || R > kKpRmax) return DISCO_ERR_ARG;
  if (!k->images) return DISCO_ERR_STATE;
  if (nkp == 0) return DISCO_OK;
  if (!aligned4(kp_vox) || !aligned4(cost)) return DISCO_ERR_SHAPE;
  HIP_TRY(hipSetDevice(k->device));
  hipStream_t s = S(stream);
  if (nkp > k->patch_cap) {
    HIP_TRY(hipStreamSynchronize(s));
    if (k->patch) (void)hipFree(k->patch);
    k->patch = nullptr;
    k->patch_cap = 0;
    if (hipMalloc(reinterpret_cast<void **>(&k->patch), sizeof(float4) * 64 * (size_t)nkp) != hipSuccess) {
      k->patch = nullptr;
      return DISCO_ERR_NOMEM;
    }
    k->patch_cap = nkp;
  }
  hipLaunchKernelGGL(k_kp_patch, dim3((unsigned)nkp), dim3(64), 0, s, k->g, k->nF, nkp, kp_vox, k->patch);
  const int nl = 2 * R + 1;
  const int64_t items = (int64_t)nkp * ((nl + kKpRows - 1) / kKpRows);
  if (items >= ((int64_t)1 << 31) - 8) return DISCO_ERR_SHAPE;
  const int run = (int)((items + 7) / 8);  // contiguous items per XCD
  hipLaunchKernelGGL(k_kp_cost, dim3((unsigned)(8 * run)), dim3(kKpThreads), 0, s, k->g, k->nM, k->patch, nkp,
                     kp_vox, R, (int)items, run, cost);
  HIP_TRY(hipGetLastError());
  return DISCO_OK;
}

extern "C++" {
// inward pass, deepest level first: h, then m = min-convolution of h (x, y, z); root:
// M_root = h_root; outward pass: M = h + min-convolution of (M_parent - m)
template <int NL>
static void kp_messages(int nl, int maxd, const std::vector<int> &lstart, const KpNode *nodes, const float *cw,
                        const float *cost, int64_t L, float sx, float sy, float sz, float *h, float *msg, float *t1,
                        float *mg, hipStream_t s) {
  for (int d = maxd; d >= 1; --d) {
    const dim3 grid((unsigned)(lstart[d + 1] - lstart[d]), (unsigned)nl);
    hipLaunchKernelGGL((k_kp_plane_xy<false, NL>), grid, dim3(256), 0, s, nl, lstart[d], nodes, cw, cost, msg, sx, sy,
                       h, t1);
    hipLaunchKernelGGL((k_kp_plane_z<false, NL>), grid, dim3(256), 0, s, nl, lstart[d], nodes, cw, sz, t1, h, msg);
  }
  hipLaunchKernelGGL(k_kp_root, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, s, L, nodes, cost, msg, h, mg);
  for (int d = 1; d <= maxd; ++d) {
    const dim3 grid((unsigned)(lstart[d + 1] - lstart[d]), (unsigned)nl);
    hipLaunchKernelGGL((k_kp_plane_xy<true, NL>), grid, dim3(256), 0, s, nl, lstart[d], nodes, cw, mg, msg, sx, sy,
                       nullptr, t1);
    hipLaunchKernelGGL((k_kp_plane_z<true, NL>), grid, dim3(256), 0, s, nl, lstart[d], nodes, cw, sz, t1, h, mg);
  }
}

}  // extern "C++"

// Tree set-up arrays of n keypoints carved from one block (host staging or device copy):
// Boruvka round results w, j and components comp, keypoint positions x and intensities
// i, node descriptors and edge weights of the message schedule.
struct KpTreeBuf {
  double *w;
  KpNode *nodes;
  float *x, *i, *cw;
  int *comp, *j;
};
static size_t kp_tree_layout(int n, char *base, KpTreeBuf *b) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  b->w = reinterpret_cast<double *>(take(sizeof(double) * n));
  b->nodes = reinterpret_cast<KpNode *>(take(sizeof(KpNode) * n));
  b->x = reinterpret_cast<float *>(take(sizeof(float) * 3 * n));
  b->i = reinterpret_cast<float *>(take(sizeof(float) * n));
  b->cw = reinterpret_cast<float *>(take(sizeof(float) * n));
  b->comp = reinterpret_cast<int *>(take(sizeof(int) * n));
  b->j = reinterpret_cast<int *>(take(sizeof(int) * n));
  return off;
}

// breadth-first rooting of a tree given as sorted adjacency lists
static void bfs_tree(const std::vector<std::vector<int>> &adj, int root, std::vector<int> &parent, std::vector<int> &order) {
  const int n = (int)adj.size();
  parent.assign(n, -1);
  order.clear();
  order.push_back(root);
  std::vector<char> seen(n, 0);
  seen[root] = 1;
  for (size_t h = 0; h < order.size(); ++h)
    for (int b : adj[order[h]])
      if (!seen[b]) {
        seen[b] = 1;
        parent[b] = order[h];
        order.push_back(b);
      }
}

int disco_kp_regularise(disco_kp *k, int32_t nkp, const float *x_mm, const float *inten, int32_t R,
                        const float *cost, double alpha_kp, double sigma_I, float *marg, int32_t *labels,
                        int32_t *parent_out, disco_stream stream) {
  if (!k || nkp < 1 || !x_mm || !inten || !cost || !labels) return DISCO_ERR_ARG;
  if (R < 1 || R > kKpRmax) return DISCO_ERR_ARG;
  if (!finite_nonneg(alpha_kp) || !std::isfinite(sigma_I) || !(sigma_I > 0.0)) return DISCO_ERR_NONFINITE;
  if (!aligned4(cost) || !aligned4(labels) || (marg && !aligned4(marg))) return DISCO_ERR_SHAPE;
  HIP_TRY(hipSetDevice(k->device));
  hipStream_t s = S(stream);
  const int n = nkp, nl = 2 * R + 1;
  const int64_t L = (int64_t)nl * nl * nl;
  // tree, levels (depth from the root), children lists, per-edge weights (host)
  std::vector<int> parent(n), order(n), tree_out;
  // set-up buffers kept in the handle; the previous call on it has finished
  if (n > k->tcap) {
    if (k->th) (void)hipHostFree(k->th);
    if (k->td) (void)hipFree(k->td);
    k->th = k->td = nullptr;
    k->tcap = 0;
    KpTreeBuf sz;
    const size_t bytes = kp_tree_layout(n, nullptr, &sz);
    if (hipHostMalloc(reinterpret_cast<void **>(&k->th), bytes) != hipSuccess) {
      k->th = nullptr;
      return DISCO_ERR_NOMEM;
    }
    if (hipMalloc(reinterpret_cast<void **>(&k->td), bytes) != hipSuccess) {
      k->td = nullptr;
      return DISCO_ERR_NOMEM;
    }
    k->tcap = n;
  }
  KpTreeBuf H, D;
  kp_tree_layout(n, k->th, &H);
  kp_tree_layout(n, k->td, &D);
  std::vector<std::vector<int>> adj(n);
  {
    // Boruvka rounds on the device (cheapest outgoing edge per keypoint), components merged
    // on the host; the tree is then rooted at keypoint 0 (breadth first, neighbours in
    // increasing order)
    std::vector<int> uf(n);
    std::iota(uf.begin(), uf.end(), 0);
    auto find = [&](int a) {
      while (uf[a] != a) a = uf[a] = uf[uf[a]];
      return a;
    };
    std::memcpy(H.x, x_mm, sizeof(float) * 3 * n);
    std::memcpy(H.i, inten, sizeof(float) * n);
    HIP_TRY(hipMemcpyAsync(D.x, H.x, sizeof(float) * 3 * n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(D.i, H.i, sizeof(float) * n, hipMemcpyHostToDevice, s));
    const double *bw = H.w;
    const int *bj = H.j;
    int *comp = H.comp;
    int ncomp = n;
    while (ncomp > 1) {
      for (int q = 0; q < n; ++q) comp[q] = find(q);
      HIP_TRY(hipMemcpyAsync(D.comp, comp, sizeof(int) * n, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_kp_boruvka, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, D.x, D.i, sigma_I, D.comp,
                         D.w, D.j);
      HIP_TRY(hipMemcpyAsync(H.w, D.w, sizeof(double) * n, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(H.j, D.j, sizeof(int) * n, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      // cheapest edge per component under the order (w, min(i, j), max(i, j))
      std::vector<int> ce(n, -1);
      auto less = [&](int a, int b) {
        if (bw[a] != bw[b]) return bw[a] < bw[b];
        const int la = std::min(a, bj[a]), lb = std::min(b, bj[b]);
        if (la != lb) return la < lb;
        return std::max(a, bj[a]) < std::max(b, bj[b]);
      };
      for (int q = 0; q < n; ++q) {
        const int c = comp[q];
        if (ce[c] < 0 || less(q, ce[c])) ce[c] = q;
      }
      for (int c = 0; c < n; ++c) {
        if (ce[c] < 0) continue;
        const int a = ce[c], b = bj[a];
        const int ra = find(a), rb = find(b);
        if (ra == rb) continue;  // the same edge chosen from both sides
        uf[std::max(ra, rb)] = std::min(ra, rb);
        adj[a].push_back(b);
        adj[b].push_back(a);
        --ncomp;
      }
    }
    // root at keypoint 0 (the tree returned), breadth first with neighbours in increasing
    // order; the messages are scheduled from the tree's centre (below)
    for (auto &a : adj) std::sort(a.begin(), a.end());
    bfs_tree(adj, 0, parent, order);
    tree_out = parent;
    // centre: the middle of a longest path (ends: the farthest node from 0, then the
    // farthest from that one); rooted there the tree has half the levels, and the
    // min-marginals do not depend on the root
    const int a = order.back();
    bfs_tree(adj, a, parent, order);
    std::vector<int> path;
    for (int q = order.back(); q >= 0; q = parent[q]) path.push_back(q);
    bfs_tree(adj, path[path.size() / 2], parent, order);
  }
  // breadth-first positions: levels and each node's children are contiguous ranges
  std::vector<int> pos_of(n), lstart(1, 0), depth(n, 0);
  for (int p = 0; p < n; ++p) pos_of[order[p]] = p;
  KpNode *nodes = H.nodes;
  float *cw = H.cw;
  for (int p = 0; p < n; ++p) {
    const int q = order[p];
    nodes[p] = KpNode{q, parent[q], 0, 0};
    cw[p] = 0.0f;
    if (p > 0) {
      depth[q] = depth[parent[q]] + 1;
      if (depth[q] != depth[order[p - 1]]) lstart.push_back(p);
      KpNode &pn = nodes[pos_of[parent[q]]];
      if (pn.ccount++ == 0) pn.cfirst = p;
      const int r = parent[q];
      const double dx = (double)x_mm[3 * q] - x_mm[3 * r], dy = (double)x_mm[3 * q + 1] - x_mm[3 * r + 1],
                   dz = (double)x_mm[3 * q + 2] - x_mm[3 * r + 2];
      const double w = std::sqrt(dx * dx + dy * dy + dz * dz) + std::fabs((double)inten[q] - inten[r]) / sigma_I;
      cw[p] = (float)(alpha_kp / w);
    }
  }
  lstart.push_back(n);
  const int maxd = (int)lstart.size() - 2;
  KpNode *d_nodes = D.nodes;
  float *d_cw = D.cw;
  // h, m and a temporary per node (and the min-marginals when marg is null), kept in the
  // handle; the previous call on the handle has finished (each call waits for its stream)
  const size_t need = (size_t)(marg ? 3 : 4) * n * L;
  if (need > k->bp_cap) {
    if (k->bp) (void)hipFree(k->bp);
    k->bp = nullptr;
    k->bp_cap = 0;
    if (hipMalloc(reinterpret_cast<void **>(&k->bp), sizeof(float) * need) != hipSuccess) {
      k->bp = nullptr;
      return DISCO_ERR_NOMEM;
    }
    k->bp_cap = need;
  }
  float *h = k->bp, *msg = h + (size_t)n * L, *t1 = msg + (size_t)n * L, *mg = marg ? marg : t1 + (size_t)n * L;
  HIP_TRY(hipMemcpyAsync(d_nodes, nodes, sizeof(KpNode) * n, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_cw, cw, sizeof(float) * n, hipMemcpyHostToDevice, s));
  const float sx = (float)(2.0 * k->h[0]), sy = (float)(2.0 * k->h[1]), sz = (float)(2.0 * k->h[2]);
  if (nl == kKpNl)
    kp_messages<kKpNl>(nl, maxd, lstart, d_nodes, d_cw, cost, L, sx, sy, sz, h, msg, t1, mg, s);
  else
    kp_messages<0>(nl, maxd, lstart, d_nodes, d_cw, cost, L, sx, sy, sz, h, msg, t1, mg, s);
  hipLaunchKernelGGL(k_kp_argmin, dim3((unsigned)n), dim3(256), 0, s, L, mg, labels);
  HIP_TRY(hipGetLastError());
  if (parent_out)
    for (int q = 0; q < n; ++q) parent_out[q] = tree_out[q];
  // the work buffers are freed on return: wait for the kernels that use them
  HIP_TRY(hipStreamSynchronize(s));
  return DISCO_OK;
}

}  // extern "C"
