// lks_api.hip -- host layer of the C ABI declared in include/lks.h: problem
// validation, workspace layout, the forward time loop with checkpoints every
// K steps, the reverse sweep with segment recomputation, hipGraph capture of
// both time loops, the stand-alone stage entry points, per-kernel event
// timing and the batched graph of independent instances.
//
// The time loops contain launches only: every per-step quantity (rigid
// motion, support box) lives in a device table filled by the prelude, so a
// loop captured once per (plan, workspace) is replayed unchanged on later
// calls.  No host synchronisation happens inside a loop.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <cmath>
#include <vector>

#include "../../include/lks.h"
#include "lks_internal.h"

using namespace lks;

namespace {

thread_local std::string g_err;

lks_status fail(lks_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(expr)                                                                \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(LKS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ---------------------------------------------------------------- profiling
struct ProfRec {
  int cls;
  hipEvent_t a, b;
};
struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<std::string> names;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  int cls_id(const char* n) {
    for (size_t i = 0; i < names.size(); ++i)
      if (names[i] == n) return (int)i;
    names.push_back(n);
    return (int)names.size() - 1;
  }
  hipEvent_t ev() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Profiler g_prof;

// Times one launch while profiling.  A single-kernel scope hands its event
// pair to the launch itself (recorded in the dispatch, so the pair brackets
// the kernel's execution only); other scopes record the pair on the stream
// around their launches.
struct Scope {
  int cls = -1;
  bool single = false;
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  Scope(const char* name, hipStream_t st, bool single_kernel = false) : s(st) {
    if (!g_prof.on) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    cls = g_prof.cls_id(name);
    a = g_prof.ev();
    b = g_prof.ev();
    if (!a || !b) return;
    single = single_kernel;
    if (single)
      launch_events() = {a, b};
    else
      (void)hipEventRecord(a, s);
  }
  ~Scope() {
    if (cls < 0 || !a || !b) return;
    LaunchEvents& le = launch_events();
    if (single && le.start) {  // the launch did not take the pair
      le = {};
      (void)hipEventRecord(a, s);
      (void)hipEventRecord(b, s);
    } else if (!single) {
      (void)hipEventRecord(b, s);
    }
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.recs.push_back({cls, a, b});
  }
};

struct GraphCache {
  hipGraphExec_t exec = nullptr;
  void* ws = nullptr;
  int key = 0;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    ws = nullptr;
    key = 0;
  }
};

}  // namespace

namespace lks {
void device_counts(int* ncu, int* nxcd) {
  int dev = 0, cu = 0, xcc = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
    *ncu = cu;
  if (hipDeviceGetAttribute(&xcc, hipDeviceAttributeNumberOfXccs, dev) == hipSuccess && xcc > 0)
    *nxcd = xcc;
  (void)hipGetLastError();
}
}  // namespace lks

struct lks_plan {
  lks_problem prob;
  Geo g;
  int prec;
  size_t es;
  long long S;  // state elements
  int K, nck;
  int kmt;      // reverse steps whose map transposes share one launch (min(K, 256))
  bool full_btape;  // body fields of every step kept (else of one segment)
  bool store_all;   // K = nt: the march writes every state into the tape and
                    // the reverse sweep recomputes nothing
  bool alks;        // reverse sweep by the paper's ALKS instead of the exact adjoint
  bool j2;          // objective J2 (Eq. objective2) instead of J1
  int nblk_step, nblk_map;
  int nblk_j2;      // J2 design-point blocks (0 without J2)
  int mrow;         // block slots per step of the motion partials: map transpose, then J2
  Box bmax;     // strides, volume and launch extents of the body buffers
  // workspace offsets (bytes)
  size_t o_mot, o_tab, o_info, o_kref, o_flags, o_J3, o_seed, o_opart, o_ck, o_pp, o_tape, o_tape2,
      o_body, o_btape, o_badj, o_lam, o_xadj, o_acarry, o_inp, o_cmot, o_badjt, o_kpart, o_badjt2,
      o_kpart2, o_krefbar, o_mpart, o_mbar, o_den, o_kz, o_geo, o_j2acc, o_j2seed, total;
  int first_lazy = 1;
  void* fwd_ws = nullptr;
  bool use_graphs = true;
  hipStream_t cap = nullptr;  // private stream used for graph capture
  GraphCache gfwd, gadj, gbatch;
  std::vector<const void*> bkey;       // pointer tables the batch graph was captured for
  std::vector<hipStream_t> bstreams;   // capture branches of the batch graph
  // 2D reverse sweep: the next segment's recompute on a side stream, into the
  // second of two state tapes (tsel picks the tape tape_slot() addresses)
  bool ovl = false;
  int tsel = 0;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // 2D J1: each chunk's map transposes on a second side stream beside the
  // next chunk's reverse steps, the body-adjoint and kappa_ref-partial
  // buffers doubled (bsel picks the pair)
  bool ovt = false;
  int bsel = 0;
  hipStream_t side2 = nullptr;
  hipEvent_t ev_chunk = nullptr, ev_tr[2] = {nullptr, nullptr};
  ~lks_plan() {
    gfwd.reset();
    gadj.reset();
    gbatch.reset();
    for (hipStream_t b : bstreams) (void)hipStreamDestroy(b);
    if (cap) (void)hipStreamDestroy(cap);
    if (side) (void)hipStreamDestroy(side);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side2) (void)hipStreamDestroy(side2);
    if (ev_chunk) (void)hipEventDestroy(ev_chunk);
    for (hipEvent_t e : ev_tr)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

lks_status validate(const lks_problem* p) {
  if (!p) return fail(LKS_EINVAL, "null problem");
  if (p->d != 2 && p->d != 3) return fail(LKS_EINVAL, "d must be 2 or 3");
  if (p->precision != LKS_FP32 && p->precision != LKS_FP64)
    return fail(LKS_EINVAL, "precision must be LKS_FP32 or LKS_FP64");
  for (int a = 0; a < p->d; ++a) {
    if (p->n[a] < 1) return fail(LKS_EINVAL, "n must be positive");
    if (p->bc[a] != 0 && p->bc[a] != 1) return fail(LKS_EINVAL, "bc must be 0 or 1");
    if (p->bc[a] == 1 && p->n[a] < 4) return fail(LKS_EINVAL, "a wall axis needs >= 4 nodes");
    if (p->m[a] < 0) return fail(LKS_EINVAL, "m must be >= 0");
  }
  if (p->d == 2 && p->n[2] != 1) return fail(LKS_EINVAL, "n[2] must be 1 in 2D");
  if (p->d == 3 && p->bc[2] != 0) return fail(LKS_EINVAL, "3D requires a periodic z axis");
  if (p->margin < 0) return fail(LKS_EINVAL, "margin must be >= 0");
  if (p->nt < 1) return fail(LKS_EINVAL, "nt must be >= 1");
  if (p->r_t < 1 || p->r_w < 1) return fail(LKS_EINVAL, "filter radii must be >= 1");
  if (p->ckpt_k < 0 || p->ckpt_k > p->nt) return fail(LKS_EINVAL, "ckpt_k must be in 0..nt");
  if (p->body_tape < -1 || p->body_tape > 1) return fail(LKS_EINVAL, "body_tape must be -1, 0 or 1");
  if (p->scheme != LKS_ADJ_EXACT && p->scheme != LKS_ADJ_ALKS)
    return fail(LKS_EINVAL, "scheme must be LKS_ADJ_EXACT or LKS_ADJ_ALKS");
  if (p->objective != LKS_OBJ_J1 && p->objective != LKS_OBJ_J2)
    return fail(LKS_EINVAL, "objective must be LKS_OBJ_J1 or LKS_OBJ_J2");
  if (p->objective == LKS_OBJ_J2 &&
      (p->d != 2 || !(p->l_m > 0.0) || !(p->xg_max[1] > p->xg_min[1])))
    return fail(LKS_EINVAL, "J2 needs d = 2, l_m > 0 and xg_max[1] > xg_min[1]");
  if (p->rot != LKS_ROT_Z && p->rot != LKS_ROT_EULER)
    return fail(LKS_EINVAL, "rot must be LKS_ROT_Z or LKS_ROT_EULER");
  if (p->rot == LKS_ROT_EULER && p->d != 3)
    return fail(LKS_EINVAL, "three rotation angles need d = 3");
  if (!(p->nu >= 0.0) || !(p->kappa_max >= 0.0) || !(p->q > 0.0))
    return fail(LKS_EINVAL, "need nu >= 0, kappa_max >= 0, q > 0");
  long long N = 1;
  for (int a = 0; a < p->d; ++a) N *= p->n[a];
  // node offsets inside the (d+1)-plane state are 32-bit in the kernels
  if (N > (1LL << 29)) return fail(LKS_EINVAL, "grid too large (at most 2^29 nodes)");
  // the 3D step kernels address the whole (p, u) state through one buffer
  // resource with 32-bit byte offsets
  const long long es = p->precision == LKS_FP32 ? 4 : 8;
  if (p->d == 3 && 4 * N * es > 0xFFFFFFFFLL)
    return fail(LKS_EINVAL, "3D grid too large (the (p, u) state must stay below 4 GiB: fewer than 2^28 nodes in FP32, 2^27 in FP64)");
  return LKS_OK;
}

void fill_geo(const lks_problem& p, Geo& g) {
  memset(&g, 0, sizeof(g));
  g.d = p.d;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = (a < p.d) ? p.n[a] : 1;
    g.bc[a] = (a < p.d) ? p.bc[a] : 0;
    g.D[a] = (a < p.d) ? p.m[a] + 2 * p.margin : 1;
    g.m[a] = (a < p.d) ? p.m[a] : 1;
    g.xiG[a] = 0.5 * (g.D[a] - 1);
    g.tlo[a] = p.tgt_lo[a];
    g.thi[a] = p.tgt_hi[a];
    g.ndir[a] = p.ndir[a];
    g.xmin[a] = p.xg_min[a];
    g.xmax[a] = p.xg_max[a];
  }
  memcpy(g.uw, p.u_wall, sizeof(g.uw));
  g.N = (long long)g.n[0] * g.n[1] * g.n[2];
  g.A = 0.75 - 4.5 * p.nu;
  g.margin = p.margin;
  g.Mtot = (long long)g.D[0] * g.D[1] * g.D[2];
  g.kmax = p.kappa_max;
  g.q = p.q;
  g.phi = p.phi;
  g.nt = p.nt;
  g.r_t = p.r_t;
  g.r_w = p.r_w;
  g.thmin = p.th_min;
  g.thmax = p.th_max;
  long long T = 1;
  for (int a = 0; a < p.d; ++a) T *= std::max(0, p.tgt_hi[a] - p.tgt_lo[a]);
  g.NTinv = T > 0 ? 1.0 / ((double)p.nt * (double)T) : 0.0;
  g.obj = p.objective;
  g.rot = p.rot == LKS_ROT_EULER ? 1 : 0;
  g.mw = g.rot ? 12 : 8;
  g.nmc = g.rot ? 6 : 4;
  for (int k = 0; k < 2; ++k) {
    g.tmin[k] = p.tilt_min[k];
    g.tmax[k] = p.tilt_max[k];
  }
  if (p.objective == LKS_OBJ_J2) {
    double Min = 1.0;
    for (int a = 0; a < p.d; ++a) Min *= p.m[a];
    g.j2s[0] = 1.0 / ((double)p.nt * Min);
    g.j2s[1] = 1.0 / ((p.xg_max[1] - p.xg_min[1]) * Min);
    g.j2s[2] = 1.0 / (2.0 * M_PI * p.l_m * Min);
    g.j2w[0] = p.w_d;
    g.j2w[1] = p.w_t;
  }
  // tile-grid origin: keeps every node's wall-stencil partners within one tile halo
  g.ty3 = p.d == 3 ? tile3_y(p.precision) : TILE_Y;
  g.prec = p.precision;
  const int tile[2] = {TILE_X, g.ty3};
  for (int a = 0; a < 2; ++a) g.org[a] = (g.bc[a] == 1 && g.n[a] % tile[a] == 2) ? -1 : 0;
  // z segments: enough blocks to fill every CU with the resident block count
  // of each 3D step kernel, but no segment shorter than 4 planes (each
  // segment re-reads 2 halo planes)
  int ncu = 256, nxcd = 8;
  device_counts(&ncu, &nxcd);
  g.nxcd = nxcd;
  g.zseg = g.zseg_f = 1;
  if (g.d == 3) {
    const long long tiles = (long long)((g.n[0] - g.org[0] + TILE_X - 1) / TILE_X) *
                            ((g.n[1] - g.org[1] + g.ty3 - 1) / g.ty3);
    auto seg_for = [&](int resident) {
      const long long want = (long long)resident * ncu;
      long long nseg = std::max(1LL, (want + tiles - 1) / tiles);
      int zs = (int)((g.n[2] + nseg - 1) / nseg);
      return std::max(std::min(zs, g.n[2]), std::min(4, g.n[2]));
    };
    g.zseg = seg_for(step_resident_adj(p.precision));
    g.zseg_f = seg_for(STEP_RESIDENT_FWD);
  }
}

char* wsp(void* ws, size_t off) { return (char*)ws + off; }

const StepInfo* tab(lks_plan* P, void* ws, int n) {
  return (const StepInfo*)wsp(ws, P->o_tab) + (n - 1);
}
void* ck_slot(lks_plan* P, void* ws, int j) { return wsp(ws, P->o_ck) + (size_t)j * P->S * P->es; }
void* pp_slot(lks_plan* P, void* ws, int j) { return wsp(ws, P->o_pp) + (size_t)j * P->S * P->es; }
void* tape_slot(lks_plan* P, void* ws, int j) {
  return wsp(ws, P->tsel ? P->o_tape2 : P->o_tape) + (size_t)j * P->S * P->es;
}
void* lam_slot(lks_plan* P, void* ws, int j) { return wsp(ws, P->o_lam) + (size_t)j * P->S * P->es; }
void* xadj_slot(lks_plan* P, void* ws, int j) {
  return wsp(ws, P->o_xadj) + (size_t)j * P->g.d * P->g.N * P->es;
}
size_t body_bytes(const lks_plan* P) { return (size_t)(1 + P->g.d) * P->bmax.vol * P->es; }
// Body adjoint (dJ/dkappa, dJ/du_s on the box) of segment step j.
void* badj_slot(lks_plan* P, void* ws, int j) {
  return wsp(ws, P->bsel ? P->o_badjt2 : P->o_badjt) + (size_t)j * body_bytes(P);
}
double* kpart_buf(lks_plan* P, void* ws) {
  return (double*)wsp(ws, P->bsel ? P->o_kpart2 : P->o_kpart);
}
void* btape_slot(lks_plan* P, void* ws, int j) {
  return wsp(ws, P->o_btape) + (size_t)j * body_bytes(P);
}
// Body fields of step n in the reverse sweep of segment sg: the full tape's
// slot n - 1, or the segment tape's slot n - nb.
void* rev_body(lks_plan* P, void* ws, int n, int sg) {
  return btape_slot(P, ws, P->full_btape ? n - 1 : n - (sg * P->K + 1));
}
// Body fields the forward march maps step n into.
void* fwd_body(lks_plan* P, void* ws, int n) {
  return P->full_btape ? btape_slot(P, ws, n - 1) : wsp(ws, P->o_body);
}
// State the forward march writes at step n: with one segment (K = nt) the
// tape slot the reverse sweep reads, else a checkpoint every K steps and a
// ping-pong pair in between.
void* fwd_out(lks_plan* P, void* ws, int n) {
  if (P->store_all) return tape_slot(P, ws, n - 1);
  return (n % P->K == 0 && n / P->K < P->nck) ? ck_slot(P, ws, n / P->K) : pp_slot(P, ws, n & 1);
}

// Body fields (kappa, u_s) of step n into `body` (layout [1+d][bmax.vol]).
lks_status map_step(lks_plan* P, void* ws, int n, void* body, hipStream_t s) {
  Scope sc("map", s, true);
  HIPCHK(launch_map(P->g, P->prec, wsp(ws, P->o_kref), wsp(ws, P->o_kz), P->bmax.ext[2], nullptr,
                    tab(P, ws, n), P->bmax, body, (char*)body + P->bmax.vol * P->es, 0, s));
  return LKS_OK;
}

FwdArgs fwd_args(lks_plan* P, void* ws, int n, const void* in, void* out, const void* body,
                 int lazy, int obj) {
  FwdArgs a;
  memset(&a, 0, sizeof a);
  a.in = in;
  a.out = out;
  a.bk = body;
  a.bu = (const char*)body + P->bmax.vol * P->es;
  a.box = P->bmax;
  a.si = tab(P, ws, n);
  a.opart = obj ? (double*)wsp(ws, P->o_opart) : nullptr;
  a.flags = (int*)wsp(ws, P->o_flags);
  a.lazy_wall = lazy;
  return a;
}

lks_status fwd_step(lks_plan* P, void* ws, int n, const void* in, void* out, const void* body,
                    int lazy, int obj, hipStream_t s) {
  const FwdArgs a = fwd_args(P, ws, n, in, out, body, lazy, obj);
  Scope sc("fwd_step", s, true);
  HIPCHK(launch_forward_step(P->g, P->prec, a, s));
  return LKS_OK;
}

// Motion prelude, kappa_ref, the per-step table and the domain check
// (synchronises the stream once).
lks_status prelude(lks_plan* P, const double* gamma, const double* chi, const double* psi,
                   void* ws, hipStream_t s) {
  if (!gamma || !chi || !psi || !ws) return fail(LKS_EINVAL, "null input pointer");
  double* mot = (double*)wsp(ws, P->o_mot);
  int* info = (int*)wsp(ws, P->o_info);
  {
    // the inputs the march is run for (lks_adjoint checks its own against them)
    double* inp = (double*)wsp(ws, P->o_inp);
    const size_t M = (size_t)inner_points(P->g), nt = (size_t)P->g.nt;
    HIPCHK(hipMemcpyAsync(inp, gamma, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(inp + M, chi, 3 * nt * sizeof(double), hipMemcpyDeviceToDevice, s));
    const size_t np = P->g.rot ? 3 : 1;  // rotation design variables per step
    HIPCHK(hipMemcpyAsync(inp + M + 3 * nt, psi, np * nt * sizeof(double), hipMemcpyDeviceToDevice,
                          s));
  }
  {
    Scope sc("prelude", s);
    HIPCHK(launch_zero(info, 64 * sizeof(int), s));
    HIPCHK(launch_kappa_ref(P->g, P->prec, gamma, wsp(ws, P->o_kref), s));
    HIPCHK(launch_kref_t(P->g, P->prec, wsp(ws, P->o_kref), wsp(ws, P->o_kz), s));
    HIPCHK(launch_motion(P->g, chi, psi, mot, s));
    HIPCHK(launch_steps(P->g, mot, (StepInfo*)wsp(ws, P->o_tab), info, s));
  }
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, info, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (flag) {
    std::vector<StepInfo> t(P->g.nt);
    HIPCHK(hipMemcpy(t.data(), wsp(ws, P->o_tab), t.size() * sizeof(StepInfo),
                     hipMemcpyDeviceToHost));
    int step = 0;
    for (int k = 0; k < P->g.nt && !step; ++k)
      if (t[k].flag == flag) step = k + 1;
    char buf[192];
    snprintf(buf, sizeof buf,
             flag == 1 ? "step %d: the body's kernel support reaches a wall node"
                       : "step %d: the body's support exceeds a periodic extent",
             step);
    return fail(LKS_EDOMAIN, buf);
  }
  return LKS_OK;
}

// Forward time loop: launches only.
lks_status forward_loop(lks_plan* P, void* ws, hipStream_t s) {
  HIPCHK(launch_zero(wsp(ws, P->o_flags), 64 * sizeof(int), s));
  HIPCHK(launch_zero(wsp(ws, P->o_opart), (size_t)P->nblk_step * 2 * sizeof(double), s));
  if (P->j2) HIPCHK(launch_zero(wsp(ws, P->o_j2acc), (size_t)P->nblk_j2 * 3 * sizeof(double), s));
  const void* in = ck_slot(P, ws, 0);
  // Each step's map runs right before its step, which then reads the body
  // fields from cache.  (Mapping every step up front in a few wide launches
  // costs as much per step: the map is bound by its stores, not by how well
  // one step fills the GPU.)  In 2D with a body slot per step, step n, the
  // map of step n + 1 and (J2) the step sums of state n - 1 share one launch.
  if (P->g.d == 2 && P->full_btape) {
    if (lks_status e = map_step(P, ws, 1, fwd_body(P, ws, 1), s)) return e;
    const int nt = P->g.nt;
    double* jacc = (double*)wsp(ws, P->o_j2acc);
    for (int n = 1; n <= nt; ++n) {
      void* out = fwd_out(P, ws, n);
      const FwdArgs a = fwd_args(P, ws, n, in, out, fwd_body(P, ws, n),
                                 n == 1 ? P->first_lazy : 1, !P->j2);
      char* nb = n < nt ? (char*)fwd_body(P, ws, n + 1) : nullptr;
      const bool j2 = P->j2 && n > 1;
      Scope sc("fwd_step", s, true);
      HIPCHK(launch_forward_step_map(P->g, P->prec, a, wsp(ws, P->o_kref),
                                     nb ? tab(P, ws, n + 1) : nullptr, P->bmax, nb,
                                     nb ? nb + P->bmax.vol * P->es : nullptr,
                                     j2 ? tab(P, ws, n - 1) : nullptr, j2 ? in : nullptr, jacc, s));
      in = out;
    }
    if (P->j2) {
      {
        Scope sc("j2_fwd", s, true);
        HIPCHK(launch_j2_forward(P->g, P->prec, wsp(ws, P->o_kref), tab(P, ws, nt), in, jacc, s));
      }
      HIPCHK(launch_j2_final(P->g, jacc, (double*)wsp(ws, P->o_J3), s));
    } else {
      HIPCHK(launch_objective_final(P->g, (const double*)wsp(ws, P->o_opart), step_blocks(P->g),
                                    (double*)wsp(ws, P->o_J3), s));
    }
    return LKS_OK;
  }
  // 3D about z with a body slot per step: the maps of MAP_BATCH steps run as
  // one launch ahead of their steps (a one-step map is a few thousand short
  // waves, all resident at once, so its latency is not hidden)
  const bool mbatch = P->g.d == 3 && !P->g.rot && P->full_btape && !P->j2;
  for (int n = 1; n <= P->g.nt; ++n) {
    void* out = fwd_out(P, ws, n);
    void* body = fwd_body(P, ws, n);
    if (mbatch) {
      if ((n - 1) % MAP_BATCH == 0) {
        const int cnt = std::min(MAP_BATCH, P->g.nt - n + 1);
        Scope sc("map", s, true);
        HIPCHK(launch_map(P->g, P->prec, wsp(ws, P->o_kref), wsp(ws, P->o_kz), P->bmax.ext[2],
                          nullptr, tab(P, ws, n), P->bmax, body,
                          (char*)body + P->bmax.vol * P->es, 0, s, cnt,
                          (long long)(body_bytes(P) / P->es)));
      }
    } else if (P->j2 && n > 1) {
      // J2: the step sums of state n - 1 ride along with this step's map
      Scope sc("map", s, true);
      HIPCHK(launch_map_j2(P->g, P->prec, wsp(ws, P->o_kref), tab(P, ws, n), P->bmax, body,
                           (char*)body + P->bmax.vol * P->es, tab(P, ws, n - 1), in,
                           (double*)wsp(ws, P->o_j2acc), s));
    } else if (lks_status e = map_step(P, ws, n, body, s)) {
      return e;
    }
    if (lks_status e = fwd_step(P, ws, n, in, out, body, n == 1 ? P->first_lazy : 1, !P->j2, s))
      return e;
    in = out;
  }
  if (P->j2) {
    Scope sc("j2_fwd", s, true);
    HIPCHK(launch_j2_forward(P->g, P->prec, wsp(ws, P->o_kref), tab(P, ws, P->g.nt), in,
                             (double*)wsp(ws, P->o_j2acc), s));
  }
  if (P->j2)
    HIPCHK(launch_j2_final(P->g, (const double*)wsp(ws, P->o_j2acc), (double*)wsp(ws, P->o_J3), s));
  else
    HIPCHK(launch_objective_final(P->g, (const double*)wsp(ws, P->o_opart), step_blocks(P->g),
                                  (double*)wsp(ws, P->o_J3), s));
  return LKS_OK;
}

const void* final_state(lks_plan* P, void* ws) { return fwd_out(P, ws, P->g.nt); }

// Reverse sweep with segment recomputation: launches only.  The recompute
// keeps each step's body fields, which the reverse steps then reuse (with the
// full body tape the forward march's are reused and the recompute maps
// nothing).
// Adjoint step n of segment sg (first step nb = sg K + 1), reading the
// adjoint state from lambda slot `cur`.
AdjArgs adj_args(lks_plan* P, void* ws, int n, int sg, int cur) {
  const int nb = sg * P->K + 1;
  const void* body = rev_body(P, ws, n, sg);
  AdjArgs a;
  memset(&a, 0, sizeof a);
  a.lam = lam_slot(P, ws, cur);
  a.lam_prev = lam_slot(P, ws, 1 - cur);
  a.u_prev = (n == nb) ? ck_slot(P, ws, sg) : tape_slot(P, ws, n - nb - 1);
  a.u_cur = tape_slot(P, ws, n - nb);
  a.bk = body;
  a.bu = (const char*)body + P->bmax.vol * P->es;
  a.bkbar = wsp(ws, P->o_badj);
  a.bubar = wsp(ws, P->o_badj) + P->bmax.vol * P->es;
  a.box = P->bmax;
  a.si = tab(P, ws, n);
  a.seed = (const double*)wsp(ws, P->o_seed);
  a.E = (const double*)wsp(ws, P->o_J3) + 1;
  if (P->alks) {
    a.xin = xadj_slot(P, ws, cur);
    a.xout = xadj_slot(P, ws, 1 - cur);
    a.si_next = n > 1 ? tab(P, ws, n - 1) : nullptr;
    a.xall = n == 1;  // the raw part of state 0 goes out with adj_initial
    a.mout = n == 1 ? wsp(ws, P->o_acarry) : nullptr;  // and its ALKS state
  }
  return a;
}

// Map transpose of step n: the per-step motion partials go to row n - 1.
MapAdjArgs mapadj_args(lks_plan* P, void* ws, int n) {
  MapAdjArgs m;
  memset(&m, 0, sizeof m);
  m.kref = wsp(ws, P->o_kref);
  m.si = tab(P, ws, n);
  m.box = P->bmax;
  m.bkbar = wsp(ws, P->o_badj);
  m.bubar = wsp(ws, P->o_badj) + P->bmax.vol * P->es;
  m.kref_bar = (double*)wsp(ws, P->o_krefbar);
  m.mpart = (double*)wsp(ws, P->o_mpart) + (size_t)(n - 1) * P->mrow * P->g.mw;
  m.overwrite = n == P->g.nt ? 1 : 0;
  return m;
}

// fork_ok: the loop may fork a side stream from `s`.  Off where `s` is itself
// a branch forked inside a capture (lks_batch_run): a second-level fork under
// capture has crashed the HIP runtime on the host.
lks_status adjoint_loop(lks_plan* P, void* ws, hipStream_t s, bool fork_ok = true) {
  const int nt = P->g.nt, K = P->K;
  int cur = 0;
  const bool ovl = P->ovl && fork_ok;
  const bool ovt = P->ovt && fork_ok;
  P->tsel = 0;
  P->bsel = 0;
  int chunk = 0;  // chunks so far (their parity picks the transposes' buffers)
  if (ovt) {
    if (!P->side2) HIPCHK(hipStreamCreateWithFlags(&P->side2, hipStreamNonBlocking));
    if (!P->ev_chunk) HIPCHK(hipEventCreateWithFlags(&P->ev_chunk, hipEventDisableTiming));
    for (hipEvent_t& e : P->ev_tr)
      if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  // recompute segment sg into the tape: tape[n - nb] holds state n (with one
  // segment the forward march has written it already)
  auto recompute = [&](int sg, hipStream_t st) -> lks_status {
    const int nb = sg * K + 1, ne = std::min((sg + 1) * K, nt);
    for (int n = nb; n <= ne; ++n) {
      const void* in = (n == nb) ? ck_slot(P, ws, sg) : tape_slot(P, ws, n - nb - 1);
      const int lazy = (n == 1) ? P->first_lazy : 1;
      void* body = rev_body(P, ws, n, sg);
      if (!P->full_btape)
        if (lks_status e = map_step(P, ws, n, body, st)) return e;
      if (lks_status e = fwd_step(P, ws, n, in, tape_slot(P, ws, n - nb), body, lazy, 0, st))
        return e;
    }
    return LKS_OK;
  };
  // 2D launches are latency-bound and leave most of the GPU idle: the
  // recompute of segment sg - 1 (into the other tape) then runs on a side
  // stream beside the reverse steps of segment sg, forked from and joined to
  // the loop's stream (graph branches under capture)
  if (ovl) {
    if (!P->side) HIPCHK(hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking));
    if (!P->ev_fork) HIPCHK(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming));
    if (!P->ev_join) HIPCHK(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming));
    P->tsel = (P->nck - 1) & 1;
    if (lks_status e = recompute(P->nck - 1, s)) return e;
  }
  for (int sg = P->nck - 1; sg >= 0; --sg) {
    const int nb = sg * K + 1, ne = std::min((sg + 1) * K, nt);
    const bool fork = ovl && sg > 0;
    if (ovl) {
      if (fork) {
        HIPCHK(hipEventRecord(P->ev_fork, s));
        HIPCHK(hipStreamWaitEvent(P->side, P->ev_fork, 0));
        P->tsel = (sg - 1) & 1;
        if (lks_status e = recompute(sg - 1, P->side)) return e;
        HIPCHK(hipEventRecord(P->ev_join, P->side));
      }
      P->tsel = sg & 1;
    } else if (!P->store_all) {
      if (lks_status e = recompute(sg, s)) return e;
    }
    // J2: the segment's seeds on the fluid velocity in one launch (they
    // depend on the motion and kappa_ref only)
    const size_t js_bytes = 2 * (size_t)P->bmax.vol * P->es;
    if (P->j2) {
      Scope sc("j2_seed", s, true);
      HIPCHK(launch_j2_seed(P->g, P->prec, wsp(ws, P->o_kref), tab(P, ws, nb), P->bmax,
                            (const double*)wsp(ws, P->o_seed), wsp(ws, P->o_j2seed), ne - nb + 1,
                            s));
    }
    // reverse steps in chunks of at most kmt, each step keeping its body
    // adjoint in a slot of its own; then the chunk's map transposes in one
    // launch (one step alone fills the GPU poorly) and its kappa_ref
    // partials summed, latest step first, as a transpose per step would
    for (int chi = ne; chi >= nb; chi -= P->kmt, ++chunk) {
     const int clo = std::max(nb, chi - P->kmt + 1);
     if (ovt) {
       // the buffers of two chunks back are free once their transposes ran
       P->bsel = chunk & 1;
       if (chunk >= 2) HIPCHK(hipStreamWaitEvent(s, P->ev_tr[chunk & 1], 0));
     }
     for (int n = chi; n >= clo; --n) {
      AdjArgs a = adj_args(P, ws, n, sg, cur);
      a.bkbar = badj_slot(P, ws, n - clo);
      a.bubar = (char*)a.bkbar + P->bmax.vol * P->es;
      if (P->j2) {
        // J2 seeds the fluid velocity on the body box instead of the target box
        a.seed = nullptr;
        a.j2s = wsp(ws, P->o_j2seed) + (size_t)(n - nb) * js_bytes;
      }
      {
        Scope sc("adj_step", s, true);
        HIPCHK(launch_adjoint_step(P->g, P->prec, a, s));
      }
      cur = 1 - cur;
     }
     {
      // with ovt on the second side stream, in chunk order (the kappa_ref
      // partials are summed in the same order either way)
      hipStream_t ts = s;
      if (ovt) {
        HIPCHK(hipEventRecord(P->ev_chunk, s));
        HIPCHK(hipStreamWaitEvent(P->side2, P->ev_chunk, 0));
        ts = P->side2;
      }
      const int cnt = chi - clo + 1;
      const MapAdjArgs m = mapadj_args(P, ws, clo);
      double* kp = kpart_buf(P, ws);
      void* b0 = badj_slot(P, ws, 0);
      const StepBatch sb{(long long)(body_bytes(P) / P->es), P->g.Mtot,
                         (long long)P->mrow * P->g.mw};
      {
        Scope sc("map_adj", ts, true);
        HIPCHK(launch_map_adjoint(P->g, P->prec, m.kref, nullptr, m.si, m.box, b0,
                                  (char*)b0 + P->bmax.vol * P->es, kp, 1, m.mpart, ts, cnt, sb));
      }
      // J2's direct terms join the same rows, in their own block slots
      if (P->j2) {
        Scope sc("j2_adj", ts, true);
        HIPCHK(launch_j2_adjoint(P->g, P->prec, m.kref, m.si, tape_slot(P, ws, clo - nb), P->S,
                                 (const double*)wsp(ws, P->o_seed), kp, P->g.Mtot, m.mpart,
                                 (long long)P->mrow * P->g.mw, P->nblk_map, cnt, ts));
      }
      HIPCHK(launch_kref_accum(P->g.Mtot, cnt, kp, (double*)wsp(ws, P->o_krefbar), ts));
      if (ovt) HIPCHK(hipEventRecord(P->ev_tr[chunk & 1], P->side2));
     }
    }
    if (fork) HIPCHK(hipStreamWaitEvent(s, P->ev_join, 0));
  }
  // the last transposes join the loop's stream (the side stream runs them in
  // order, so the last event covers all)
  if (ovt && chunk > 0) HIPCHK(hipStreamWaitEvent(s, P->ev_tr[(chunk - 1) & 1], 0));
  P->tsel = 0;
  P->bsel = 0;
  return LKS_OK;
}

lks_status sens(lks_plan* P, const double* gamma, const void* ws, double* dg, double* dchi,
                double* dpsi, hipStream_t s) {
  Scope sc("sensitivities", s);
  double* den = (double*)wsp((void*)ws, P->o_den);
  HIPCHK(launch_sens(P->g, P->prec, gamma, (const double*)wsp((void*)ws, P->o_krefbar),
                     (const double*)wsp((void*)ws, P->o_mpart), P->mrow,
                     (double*)wsp((void*)ws, P->o_mbar), den, den + P->g.nt, dg, dchi, dpsi, s));
  return LKS_OK;
}

// Runs `body` on `s`: eagerly while profiling (per-launch events) or when
// graphs are off, otherwise through a graph captured on the plan's private
// stream on first use for this (workspace, key) and replayed afterwards.
template <class F>
lks_status run_loop(lks_plan* P, GraphCache& gc, void* ws, int key, hipStream_t s, F body) {
  if (!P->use_graphs || g_prof.on) return body(s);
  if (!(gc.exec && gc.ws == ws && gc.key == key)) {
    gc.reset();
    if (!P->cap) HIPCHK(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal));
    lks_status e = body(P->cap);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(P->cap, &graph);
    if (e) {
      if (graph) (void)hipGraphDestroy(graph);
      return e;
    }
    if (ce != hipSuccess) return fail(LKS_EHIP, std::string("capture: ") + hipGetErrorString(ce));
    hipError_t ie = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      gc.exec = nullptr;
      return fail(LKS_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
    }
    gc.ws = ws;
    gc.key = key;
  }
  HIPCHK(hipGraphLaunch(gc.exec, s));
  return LKS_OK;
}

Box full_box(const lks_plan* P) {
  Box b;
  memset(&b, 0, sizeof b);
  for (int a = 0; a < 3; ++a) b.ext[a] = P->g.n[a];
  b.sx = P->g.n[0];
  b.sy = P->g.n[1];
  b.vol = P->g.N;
  return b;
}

lks_status host_box(lks_plan* P, const double* motion8_dev, double* m8, Box& box, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(m8, motion8_dev, P->g.mw * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int b[8];
  body_box(P->g, m8, b);
  if (b[6] == 2) return fail(LKS_EINVAL, "the body's support exceeds a periodic extent");
  memset(&box, 0, sizeof box);
  for (int a = 0; a < 3; ++a) {
    box.lo[a] = b[a];
    box.ext[a] = b[3 + a];
  }
  return LKS_OK;
}

}  // namespace

extern "C" {

const char* lks_last_error(void) { return g_err.c_str(); }

#ifndef LKS_SOURCE_DIGEST
#define LKS_SOURCE_DIGEST "unknown"
#endif
const char* lks_source_digest(void) { return LKS_SOURCE_DIGEST; }

lks_status lks_plan_create(const lks_problem* prob, lks_plan** out, size_t* workspace_bytes) {
  if (!out) return fail(LKS_EINVAL, "null out");
  if (lks_status e = validate(prob)) return e;
  lks_plan* P = new lks_plan();
  P->prob = *prob;
  fill_geo(*prob, P->g);
  P->prec = prob->precision;
  P->es = prob->precision == LKS_FP32 ? 4 : 8;
  const Geo& g = P->g;
  P->S = (long long)(g.d + 1) * g.N;
  P->K = prob->ckpt_k == 0 ? g.nt : prob->ckpt_k;
  P->nck = (g.nt + P->K - 1) / P->K;
  P->kmt = std::min(P->K, 256);
  P->nblk_step = step_blocks(g);
  if (g.d == 3) {
    Geo g4 = g;
    g4.zseg = g4.zseg_f = std::min(4, g.n[2]);
    P->nblk_step = std::max(P->nblk_step, step_blocks(g4));
  }
  P->nblk_map = mapadj_blocks(g);
  P->j2 = prob->objective == LKS_OBJ_J2;
  P->nblk_j2 = P->j2 ? j2_blocks(g) : 0;
  P->mrow = P->nblk_map + P->nblk_j2;
  // body-box bound over any rotation about z (or, with three angles, any
  // rotation) and any translation
  const double diag = sqrt((double)(g.D[0] - 1) * (g.D[0] - 1) + (double)(g.D[1] - 1) * (g.D[1] - 1));
  const double diag3 = sqrt(diag * diag + (double)(g.D[2] - 1) * (g.D[2] - 1));
  int ext[3];
  for (int a = 0; a < 3; ++a) {
    if (a >= g.d) {
      ext[a] = 1;
      continue;
    }
    int e = g.rot ? (int)ceil(diag3) + 6 : (a < 2) ? (int)ceil(diag) + 6 : g.D[2] + 5;
    ext[a] = std::min(e, g.n[a]);
  }
  memset(&P->bmax, 0, sizeof(Box));
  P->bmax.sx = ext[0];
  P->bmax.sy = ext[1];
  P->bmax.vol = (long long)ext[0] * ext[1] * ext[2];
  for (int a = 0; a < 3; ++a) P->bmax.ext[a] = ext[a];
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t Sb = (size_t)P->S * P->es;
  P->o_mot = take((size_t)g.nt * g.mw * sizeof(double));
  P->o_tab = take((size_t)g.nt * sizeof(StepInfo));
  P->o_info = take(64 * sizeof(int));
  P->o_kref = take((size_t)g.Mtot * P->es);
  P->o_flags = take(64 * sizeof(int));
  P->o_J3 = take(4 * sizeof(double));
  P->o_seed = take(sizeof(double));
  P->o_opart = take((size_t)P->nblk_step * 2 * sizeof(double));
  P->o_ck = take((size_t)P->nck * Sb);
  P->o_pp = take(2 * Sb);
  P->o_tape = take((size_t)P->K * Sb);
  // 2D (latency-bound launches) with a body slot per step and more than one
  // segment: a second tape lets the next segment's recompute run beside the
  // reverse steps (set below, once the body-tape mode is known)
  P->o_tape2 = 0;
  const size_t full_tape = (size_t)g.nt * body_bytes(P);
  // one segment (K = nt): the march keeps every state in the tape, and the
  // segment's body tape is the full one
  P->store_all = P->K == g.nt;
  P->full_btape = P->store_all || prob->body_tape == 1 ||
                  (prob->body_tape == 0 && full_tape <= LKS_BODY_TAPE_AUTO_MAX);
  P->o_body = take(P->full_btape ? 0 : body_bytes(P));
  P->o_btape = take(P->full_btape ? full_tape : (size_t)P->K * body_bytes(P));
  P->ovl = g.d == 2 && !P->store_all && P->full_btape && P->nck > 1;
  if (P->ovl) P->o_tape2 = take((size_t)P->K * Sb);
  P->o_badj = take(body_bytes(P));
  // the reverse sweep keeps the body adjoint of each step of a chunk (at most
  // kmt steps) and transposes the chunk's maps in one launch, each step's
  // kappa_ref partials apart
  P->o_badjt = take((size_t)P->kmt * body_bytes(P));
  P->o_kpart = take((size_t)P->kmt * g.Mtot * sizeof(double));
  P->ovt = P->ovl && !P->j2;
  P->o_badjt2 = P->ovt ? take((size_t)P->kmt * body_bytes(P)) : 0;
  P->o_kpart2 = P->ovt ? take((size_t)P->kmt * g.Mtot * sizeof(double)) : 0;
  P->o_lam = take(2 * Sb);
  P->alks = prob->scheme == LKS_ADJ_ALKS;
  // ALKS: raw first-moment part of the adjoint velocity, two slots like lambda
  P->o_xadj = take(P->alks ? 2 * (size_t)g.d * g.N * P->es : 0);
  // ALKS: the state (p~, u~, s~) of level 0, written by the sweep's last step
  P->o_acarry = take(P->alks ? (size_t)alks_carry_planes(g.d) * g.N * P->es : 0);
  P->o_krefbar = take((size_t)g.Mtot * sizeof(double));
  P->o_mpart = take((size_t)g.nt * P->mrow * g.mw * sizeof(double));
  // J2: per-block step sums, and the reverse-step seeds of one segment on the body box
  P->o_j2acc = take((size_t)P->nblk_j2 * 3 * sizeof(double));
  P->o_j2seed = take(P->j2 ? (size_t)P->K * 2 * P->bmax.vol * P->es : 0);
  P->o_mbar = take((size_t)g.nt * g.mw * sizeof(double));
  // filter normalisers (2 nt) and the chain rule's per-component totals (nmc nt)
  P->o_den = take((size_t)g.nt * (2 + g.nmc) * sizeof(double));
  // lks_constraints: its own motion table and a discarded chi-gradient
  P->o_cmot = take((size_t)g.nt * (g.mw + 3) * sizeof(double));
  P->o_kz = take(kz_bytes(g, P->bmax.ext[2], P->prec));
  P->o_geo = take(sizeof(Geo));
  // copies of the last lks_forward's gamma, chi, psi (lks_adjoint checks its own against them)
  P->o_inp = take(((size_t)inner_points(g) + 6 * (size_t)g.nt) * sizeof(double));
  P->total = off;
  *out = P;
  if (workspace_bytes) *workspace_bytes = P->total;
  return LKS_OK;
}

lks_status lks_plan_destroy(lks_plan* plan) {
  delete plan;
  return LKS_OK;
}

lks_status lks_plan_set_graphs(lks_plan* P, int32_t on) {
  if (!P) return fail(LKS_EINVAL, "null plan");
  P->use_graphs = on != 0;
  return LKS_OK;
}

lks_status lks_plan_set_zseg(lks_plan* P, int32_t zseg) {
  if (!P) return fail(LKS_EINVAL, "null plan");
  if (P->g.d != 3) return LKS_OK;
  if (zseg < 0) return fail(LKS_EINVAL, "zseg must be >= 0");
  // zseg > 0 sets both step kernels' segment length; 0 restores the defaults
  Geo g2 = P->g;
  if (zseg == 0) {
    Geo gd;
    fill_geo(P->prob, gd);
    g2.zseg = gd.zseg;
    g2.zseg_f = gd.zseg_f;
  } else {
    g2.zseg = g2.zseg_f = std::min(zseg, P->g.n[2]);
  }
  if (g2.zseg != P->g.zseg || g2.zseg_f != P->g.zseg_f) {
    // the step grid (and with it the objective partial slots) changes
    if (step_blocks(g2) > P->nblk_step) return fail(LKS_EINVAL, "zseg too small for this plan");
    P->g.zseg = g2.zseg;
    P->g.zseg_f = g2.zseg_f;
    P->gfwd.reset();
    P->gadj.reset();
  }
  return LKS_OK;
}

lks_status lks_forward(lks_plan* P, const double* gamma, const double* chi, const double* psi,
                       const void* state0, void* state_final, void* ws, double* J_out,
                       hipStream_t s) {
  if (!P || !J_out) return fail(LKS_EINVAL, "null plan or J_out");
  if (lks_status e = prelude(P, gamma, chi, psi, ws, s)) return e;
  if (state0) {
    HIPCHK(hipMemcpyAsync(ck_slot(P, ws, 0), state0, (size_t)P->S * P->es,
                          hipMemcpyDeviceToDevice, s));
  } else {
    HIPCHK(launch_state_init(P->g, P->prec, ck_slot(P, ws, 0), s));
  }
  P->first_lazy = state0 ? 0 : 1;
  P->fwd_ws = nullptr;
  if (lks_status e = run_loop(P, P->gfwd, ws, P->first_lazy, s,
                              [&](hipStream_t st) { return forward_loop(P, ws, st); }))
    return e;
  HIPCHK(hipMemcpyAsync(J_out, wsp(ws, P->o_J3), 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (state_final) {
    HIPCHK(hipMemcpyAsync(state_final, final_state(P, ws), (size_t)P->S * P->es,
                          hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_wall_fixup(P->g, P->prec, state_final, s));
  }
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, wsp(ws, P->o_flags), sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  P->fwd_ws = ws;
  if (flag) return fail(LKS_EUNSTABLE, "the march produced |u| >= 0.5 or a non-finite value");
  return LKS_OK;
}

lks_status lks_adjoint(lks_plan* P, const double* gamma, const double* chi, const double* psi,
                       void* ws, const double* dJ, const void* adj_terminal, void* adj_initial,
                       double* dJ_dgamma, double* dJ_dchi, double* dJ_dpsi, hipStream_t s) {
  if (!P || !ws || !dJ || !gamma || !chi || !psi || !dJ_dgamma || !dJ_dchi || !dJ_dpsi)
    return fail(LKS_EINVAL, "null argument");
  if (P->fwd_ws != ws)
    return fail(LKS_EINVAL, "lks_adjoint needs a preceding lks_forward on this plan and workspace");
  {
    // the sweep reverses the last forward march: its inputs must be these
    const double* inp = (const double*)wsp(ws, P->o_inp);
    const long long M = inner_points(P->g), nt = P->g.nt;
    int* flag = (int*)wsp(ws, P->o_info) + 1;
    HIPCHK(launch_zero(flag, sizeof(int), s));
    HIPCHK(launch_differ(gamma, inp, M, flag, s));
    HIPCHK(launch_differ(chi, inp + M, 3 * nt, flag, s));
    HIPCHK(launch_differ(psi, inp + M + 3 * nt, (P->g.rot ? 3 : 1) * nt, flag, s));
    int differ = 0;
    HIPCHK(hipMemcpyAsync(&differ, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (differ)
      return fail(LKS_EINVAL,
                  "lks_adjoint: gamma, chi or psi differ from those of the preceding lks_forward");
  }
  const size_t Sb = (size_t)P->S * P->es;
  const size_t Xb = (size_t)P->g.d * P->g.N * P->es;  // ALKS raw-moment part
  HIPCHK(hipMemcpyAsync(wsp(ws, P->o_seed), dJ, sizeof(double), hipMemcpyDeviceToDevice, s));
  if (P->alks && adj_terminal) {
    // the carried ALKS state stands for the moments of the last level; its
    // adjoint equilibrium is formed with this run's velocity there
    HIPCHK(launch_alks_carry_in(P->g, P->prec, (const char*)adj_terminal + Sb, final_state(P, ws),
                                lam_slot(P, ws, 0), xadj_slot(P, ws, 0), s));
  } else {
    if (P->alks) HIPCHK(launch_zero(xadj_slot(P, ws, 0), Xb, s));
    if (adj_terminal)
      HIPCHK(hipMemcpyAsync(lam_slot(P, ws, 0), adj_terminal, Sb, hipMemcpyDeviceToDevice, s));
    else
      HIPCHK(launch_zero(lam_slot(P, ws, 0), Sb, s));
  }
  HIPCHK(launch_zero(wsp(ws, P->o_badj), body_bytes(P), s));
  HIPCHK(launch_zero(wsp(ws, P->o_krefbar), (size_t)P->g.Mtot * sizeof(double), s));
  // the z-fastest kappa_ref copy may have been reused by a stand-alone map call
  HIPCHK(launch_kref_t(P->g, P->prec, wsp(ws, P->o_kref), wsp(ws, P->o_kz), s));
  if (lks_status e = run_loop(P, P->gadj, ws, P->first_lazy, s,
                              [&](hipStream_t st) { return adjoint_loop(P, ws, st); }))
    return e;
  const int fin = P->g.nt % 2;  // lambda slot holding dJ/d state0
  if (adj_initial) {
    HIPCHK(hipMemcpyAsync(adj_initial, lam_slot(P, ws, fin), Sb, hipMemcpyDeviceToDevice, s));
    if (P->alks)
      HIPCHK(hipMemcpyAsync((char*)adj_initial + Sb, wsp(ws, P->o_acarry),
                            (size_t)alks_carry_planes(P->g.d) * P->g.N * P->es,
                            hipMemcpyDeviceToDevice, s));
  }
  return sens(P, gamma, ws, dJ_dgamma, dJ_dchi, dJ_dpsi, s);
}

lks_status lks_sensitivities(lks_plan* P, const double* gamma, const void* ws, double* dJ_dgamma,
                             double* dJ_dchi, double* dJ_dpsi, hipStream_t s) {
  if (!P || !ws || !gamma || !dJ_dgamma || !dJ_dchi || !dJ_dpsi)
    return fail(LKS_EINVAL, "null argument");
  return sens(P, gamma, ws, dJ_dgamma, dJ_dchi, dJ_dpsi, s);
}

lks_status lks_design_filter(lks_plan* P, const double* gamma, double radius, double beta,
                             double eta, double* gamma_phys, hipStream_t s) {
  if (!P || !gamma || !gamma_phys) return fail(LKS_EINVAL, "null argument");
  if (!(radius > 0.0 && radius <= 64.0)) return fail(LKS_EINVAL, "filter radius must be in (0, 64]");
  if (!(eta >= 0.0 && eta <= 1.0) || !std::isfinite(beta))
    return fail(LKS_EINVAL, "projection needs 0 <= eta <= 1 and a finite beta");
  Scope sc("design", s);
  HIPCHK(launch_design_filter(P->g, gamma, radius, beta, eta, gamma_phys, s));
  return LKS_OK;
}

lks_status lks_design_filter_adjoint(lks_plan* P, const double* gamma, double radius, double beta,
                                     double eta, const double* dJ_dphys, double* work,
                                     double* dJ_dgamma, hipStream_t s) {
  if (!P || !gamma || !dJ_dphys || !work || !dJ_dgamma) return fail(LKS_EINVAL, "null argument");
  if (!(radius > 0.0 && radius <= 64.0)) return fail(LKS_EINVAL, "filter radius must be in (0, 64]");
  if (!(eta >= 0.0 && eta <= 1.0) || !std::isfinite(beta))
    return fail(LKS_EINVAL, "projection needs 0 <= eta <= 1 and a finite beta");
  Scope sc("design", s);
  HIPCHK(launch_design_filter_adjoint(P->g, gamma, radius, beta, eta, dJ_dphys, work, dJ_dgamma, s));
  return LKS_OK;
}

lks_status lks_design_filter_adjoint_noalloc(lks_plan* P, const double* gamma, double radius,
                                             double beta, double eta, const double* dJ_dphys,
                                             double* dJ_dgamma, hipStream_t s) {
  if (!P || !gamma || !dJ_dphys || !dJ_dgamma) return fail(LKS_EINVAL, "null argument");
  if (!(radius > 0.0 && radius <= 64.0)) return fail(LKS_EINVAL, "filter radius must be in (0, 64]");
  if (!(eta >= 0.0 && eta <= 1.0) || !std::isfinite(beta))
    return fail(LKS_EINVAL, "projection needs 0 <= eta <= 1 and a finite beta");
  const long long M = inner_points(P->g);
  if (M > NOALLOC_MAX_POINTS)
    return fail(LKS_EINVAL, "lks_design_filter_adjoint_noalloc: " + std::to_string(M) +
                                " design points exceed its scratch of " +
                                std::to_string(NOALLOC_MAX_POINTS));
  double* work = nullptr;
  HIPCHK(noalloc_scratch(&work));
  HIPCHK(launch_design_filter_adjoint(P->g, gamma, radius, beta, eta, dJ_dphys, work, dJ_dgamma, s));
  return LKS_OK;
}

lks_status lks_constraints(lks_plan* P, void* ws, const double* gamma_phys, const double* chi,
                           const double* psi, double vmax, double omega_max, double p_omega,
                           double* G_out, double* dG1, double* dG2, double* dG3_dpsi,
                           hipStream_t s) {
  if (!P || !ws || !gamma_phys || !chi || !psi || !G_out) return fail(LKS_EINVAL, "null argument");
  if (!(vmax > 0.0) || !(omega_max > 0.0) || !(p_omega >= 1.0 && std::isfinite(p_omega)))
    return fail(LKS_EINVAL, "constraints need vmax > 0, omega_max > 0 and 1 <= p finite");
  double* cm = (double*)wsp(ws, P->o_cmot);
  Scope sc("constraints", s);
  HIPCHK(launch_constraints(P->g, gamma_phys, chi, psi, vmax, omega_max, p_omega, G_out, dG1, dG2,
                            dG3_dpsi, cm, (double*)wsp(ws, P->o_mbar),
                            (double*)wsp(ws, P->o_den), cm + (size_t)P->g.nt * P->g.mw, s));
  return LKS_OK;
}

lks_status lks_motion(lks_plan* P, const double* chi, const double* psi, double* motion,
                      hipStream_t s) {
  if (!P || !chi || !psi || !motion) return fail(LKS_EINVAL, "null argument");
  HIPCHK(launch_motion(P->g, chi, psi, motion, s));
  return LKS_OK;
}

lks_status lks_kappa_ref(lks_plan* P, const double* gamma, void* kappa_ref, hipStream_t s) {
  if (!P || !gamma || !kappa_ref) return fail(LKS_EINVAL, "null argument");
  HIPCHK(launch_kappa_ref(P->g, P->prec, gamma, kappa_ref, s));
  return LKS_OK;
}

lks_status lks_map_design_to_grid(lks_plan* P, const void* kappa_ref, const double* motion8,
                                  void* kappa, void* u_s, void* ws, hipStream_t s) {
  if (!P || !kappa_ref || !motion8 || !kappa || !u_s || !ws)
    return fail(LKS_EINVAL, "null argument");
  double m8[12];
  Box box;
  if (lks_status e = host_box(P, motion8, m8, box, s)) return e;
  HIPCHK(launch_zero(kappa, (size_t)P->g.N * P->es, s));
  HIPCHK(launch_zero(u_s, (size_t)P->g.d * P->g.N * P->es, s));
  HIPCHK(launch_kref_t(P->g, P->prec, kappa_ref, wsp(ws, P->o_kz), s));
  Scope sc("map", s, true);
  HIPCHK(launch_map(P->g, P->prec, kappa_ref, wsp(ws, P->o_kz), P->bmax.ext[2], m8, nullptr, box,
                    kappa, u_s, 1, s));
  return LKS_OK;
}

lks_status lks_step(lks_plan* P, const void* state_in, const void* kappa, const void* u_s,
                    void* state_out, hipStream_t s) {
  if (!P || !state_in || !kappa || !u_s || !state_out) return fail(LKS_EINVAL, "null argument");
  if (state_in == state_out) return fail(LKS_EINVAL, "state_in and state_out must not alias");
  FwdArgs a;
  memset(&a, 0, sizeof a);
  a.in = state_in;
  a.out = state_out;
  a.bk = kappa;
  a.bu = u_s;
  a.box = full_box(P);
  a.lazy_wall = 0;
  {
    Scope sc("fwd_step", s, true);
    HIPCHK(launch_forward_step(P->g, P->prec, a, s));
  }
  HIPCHK(launch_wall_fixup(P->g, P->prec, state_out, s));
  return LKS_OK;
}

lks_status lks_step_adjoint(lks_plan* P, const void* state_in, const void* state_out,
                            const void* kappa, const void* u_s, const void* lam, void* lam_prev,
                            void* kbar, void* usbar, hipStream_t s) {
  if (!P || !state_in || !state_out || !kappa || !u_s || !lam || !lam_prev || !kbar || !usbar)
    return fail(LKS_EINVAL, "null argument");
  HIPCHK(launch_zero(kbar, (size_t)P->g.N * P->es, s));
  HIPCHK(launch_zero(usbar, (size_t)P->g.d * P->g.N * P->es, s));
  AdjArgs a;
  memset(&a, 0, sizeof a);
  a.lam = lam;
  a.lam_prev = lam_prev;
  a.u_prev = state_in;
  a.u_cur = state_out;
  a.bk = kappa;
  a.bu = u_s;
  a.bkbar = kbar;
  a.bubar = usbar;
  a.box = full_box(P);
  Scope sc("adj_step", s, true);
  HIPCHK(launch_adjoint_step(P->g, P->prec, a, s));
  return LKS_OK;
}

// The stand-alone map transpose reduces its per-block partials in a second
// fixed-order pass; motion_bar8 must hold W * (blocks + 1) doubles (W the
// motion row width, 8 or 12): the first W receive the result, the rest serve
// as the partial store.
lks_status lks_map_adjoint(lks_plan* P, const void* kappa_ref, const double* motion8,
                           const void* kbar, const void* usbar, double* kref_bar,
                           double* motion_bar8, hipStream_t s) {
  if (!P || !kappa_ref || !motion8 || !kbar || !usbar || !kref_bar || !motion_bar8)
    return fail(LKS_EINVAL, "null argument");
  double m8[12];
  Box box;
  if (lks_status e = host_box(P, motion8, m8, box, s)) return e;
  double* part = motion_bar8 + P->g.mw;
  {
    Scope sc("map_adj", s, true);
    HIPCHK(launch_map_adjoint(P->g, P->prec, kappa_ref, m8, nullptr, full_box(P), kbar, usbar,
                              kref_bar, 1, part, s));
  }
  HIPCHK(launch_reduce_parts(P->g, part, P->nblk_map, motion_bar8, s));
  return LKS_OK;
}

int32_t lks_map_adjoint_blocks(lks_plan* P) { return P ? P->nblk_map : 0; }

// Forward + adjoint of up to BATCH_MAX 2D instances with equal step count,
// checkpoint interval and precision: every kernel of a step is ONE launch
// covering all instances (instance k owns a block range), so the per-step
// launch count does not grow with the number of instances.  The argument
// construction is the single-instance loops' own (fwd_args, adj_args,
// mapadj_args), so each instance computes exactly what it computes alone.
lks_status batched_march(int count, lks_plan* const* plans, void* const* ws,
                         const double* const* gamma, double* const* J_out, double* const* dg,
                         double* const* dchi, double* const* dpsi, hipStream_t s) {
  const int prec = plans[0]->prec, nt = plans[0]->g.nt, K = plans[0]->K;
  const int kmt = plans[0]->kmt;
  const int nck = plans[0]->nck;
  auto round8 = [](int v) { return (v + 7) / 8 * 8; };
  Batch<FwdArgs> fb;
  Batch<AdjArgs> ab;
  Batch<MapArgs> mb;
  Batch<MapAdjArgs> qb;
  memset(&fb, 0, sizeof fb);
  memset(&ab, 0, sizeof ab);
  memset(&mb, 0, sizeof mb);
  memset(&qb, 0, sizeof qb);
  fb.count = ab.count = mb.count = qb.count = count;
  for (int k = 0; k < count; ++k) {
    lks_plan* P = plans[k];
    const Geo* gp = (const Geo*)wsp(ws[k], P->o_geo);
    fb.geo[k] = ab.geo[k] = mb.geo[k] = qb.geo[k] = gp;
    fb.start[k + 1] = fb.start[k] + round8(step_blocks_2d(P->g));
    ab.start[k + 1] = ab.start[k] + round8(adj2d_blocks(P->g));
    int bxn = 0;
    mb.start[k + 1] = mb.start[k] + round8(map_blocks_2d(P->bmax, &bxn));
    mb.a[k].kref = wsp(ws[k], P->o_kref);
    mb.a[k].box = P->bmax;
    mb.a[k].bxn = bxn;
    qb.start[k + 1] = qb.start[k] + round8(mapadj_blocks(P->g));
  }
  const bool full = plans[0]->full_btape;
  auto set_map = [&](int n, int sg_body) {
    // sg_body < 0: the forward march's body buffer; else the tape slot of step n
    for (int k = 0; k < count; ++k) {
      lks_plan* P = plans[k];
      void* body = sg_body < 0 ? fwd_body(P, ws[k], n) : rev_body(P, ws[k], n, sg_body);
      mb.a[k].si = tab(P, ws[k], n);
      mb.a[k].bk = body;
      mb.a[k].bu = (char*)body + P->bmax.vol * P->es;
    }
  };
  auto map_all = [&](int n, int sg_body) -> lks_status {
    set_map(n, sg_body);
    {
      Scope sc("map", s, true);
      HIPCHK(launch_map_batch(prec, mb, s));
    }
    return LKS_OK;
  };
  // forward march
  std::vector<const void*> in(count);
  for (int k = 0; k < count; ++k) {
    lks_plan* P = plans[k];
    HIPCHK(launch_zero(wsp(ws[k], P->o_flags), 64 * sizeof(int), s));
    HIPCHK(launch_zero(wsp(ws[k], P->o_opart), (size_t)P->nblk_step * 2 * sizeof(double), s));
    in[k] = ck_slot(P, ws[k], 0);
  }
  // with a body slot per step, step n and the map of step n + 1 share a
  // launch (they touch different slots), as in a single plan's march
  if (full)
    if (lks_status e = map_all(1, -1)) return e;
  for (int n = 1; n <= nt; ++n) {
    if (!full)
      if (lks_status e = map_all(n, -1)) return e;
    for (int k = 0; k < count; ++k) {
      lks_plan* P = plans[k];
      void* out = fwd_out(P, ws[k], n);
      fb.a[k] = fwd_args(P, ws[k], n, in[k], out, fwd_body(P, ws[k], n),
                         n == 1 ? P->first_lazy : 1, 1);
      in[k] = out;
    }
    {
      Scope sc("fwd_step", s, true);
      if (full && n < nt) {
        set_map(n + 1, -1);
        HIPCHK(launch_forward_step_map_batch(prec, fb, mb, s));
      } else {
        HIPCHK(launch_forward_step_batch(prec, fb, s));
      }
    }
  }
  for (int k = 0; k < count; ++k) {
    lks_plan* P = plans[k];
    HIPCHK(launch_objective_final(P->g, (const double*)wsp(ws[k], P->o_opart),
                                  step_blocks(P->g), (double*)wsp(ws[k], P->o_J3), s));
    HIPCHK(hipMemcpyAsync(J_out[k], wsp(ws[k], P->o_J3), 3 * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
  }
  // adjoint march, segment by segment
  int cur = 0;
  for (int sg = nck - 1; sg >= 0; --sg) {
    const int nb = sg * K + 1, ne = std::min((sg + 1) * K, nt);
    for (int n = nb; n <= ne && !plans[0]->store_all; ++n) {
      if (!full)
        if (lks_status e = map_all(n, sg)) return e;
      for (int k = 0; k < count; ++k) {
        lks_plan* P = plans[k];
        const void* src = (n == nb) ? ck_slot(P, ws[k], sg) : tape_slot(P, ws[k], n - nb - 1);
        fb.a[k] = fwd_args(P, ws[k], n, src, tape_slot(P, ws[k], n - nb),
                           rev_body(P, ws[k], n, sg), (n == 1) ? P->first_lazy : 1, 0);
      }
      {
        Scope sc("fwd_step", s, true);
        HIPCHK(launch_forward_step_batch(prec, fb, s));
      }
    }
    // reverse steps, each keeping its body adjoint in a slot of its own;
    // then the segment's map transposes of every instance in one launch, as
    // in the single-instance sweep (adjoint_loop)
    for (int n = ne; n >= nb; --n) {
      const int clo = std::max(nb, n - (n - nb) % kmt);  // first step of n's chunk
      for (int k = 0; k < count; ++k) {
        lks_plan* P = plans[k];
        ab.a[k] = adj_args(P, ws[k], n, sg, cur);
        ab.a[k].bkbar = badj_slot(P, ws[k], n - clo);
        ab.a[k].bubar = (char*)ab.a[k].bkbar + P->bmax.vol * P->es;
      }
      {
        Scope sc("adj_step", s, true);
        HIPCHK(launch_adjoint_step_batch(prec, ab, s));
      }
      cur = 1 - cur;
      if (n != clo) continue;
      // the chunk's map transposes of every instance in one launch
      const int cnt = std::min(ne, clo + kmt - 1) - clo + 1;
      for (int k = 0; k < count; ++k) {
        lks_plan* P = plans[k];
        MapAdjArgs m = mapadj_args(P, ws[k], clo);
        m.bkbar = badj_slot(P, ws[k], 0);
        m.bubar = (const char*)m.bkbar + P->bmax.vol * P->es;
        m.kref_bar = (double*)wsp(ws[k], P->o_kpart);
        m.overwrite = 1;
        m.sb = StepBatch{(long long)(body_bytes(P) / P->es), P->g.Mtot,
                         (long long)P->mrow * 8};
        qb.a[k] = m;
      }
      Scope sc("map_adj", s, true);
      HIPCHK(launch_map_adjoint_batch(prec, qb, s, cnt));
      for (int k = 0; k < count; ++k) {
        lks_plan* P = plans[k];
        HIPCHK(launch_kref_accum(P->g.Mtot, cnt, (const double*)wsp(ws[k], P->o_kpart),
                                 (double*)wsp(ws[k], P->o_krefbar), s));
      }
    }
  }
  for (int k = 0; k < count; ++k)
    if (lks_status e = sens(plans[k], gamma[k], ws[k], dg[k], dchi[k], dpsi[k], s)) return e;
  return LKS_OK;
}

lks_status lks_batch_run(int32_t count, lks_plan* const* plans, const double* const* gamma,
                         const double* const* chi, const double* const* psi,
                         void* const* workspace, double* const* J_out, const double* dJ,
                         double* const* dJ_dgamma, double* const* dJ_dchi,
                         double* const* dJ_dpsi, hipStream_t s) {
  if (count < 1 || !plans || !gamma || !chi || !psi || !workspace || !J_out || !dJ_dgamma ||
      !dJ_dchi || !dJ_dpsi)
    return fail(LKS_EINVAL, "lks_batch_run: null table or count < 1");
  for (int k = 0; k < count; ++k) {
    if (!plans[k] || !gamma[k] || !chi[k] || !psi[k] || !workspace[k] || !J_out[k] ||
        !dJ_dgamma[k] || !dJ_dchi[k] || !dJ_dpsi[k])
      return fail(LKS_EINVAL, "lks_batch_run: null entry " + std::to_string(k));
    for (int j = 0; j < k; ++j)
      if (plans[j] == plans[k] || workspace[j] == workspace[k])
        return fail(LKS_EINVAL, "lks_batch_run: instances must not share a plan or workspace");
  }
  lks_plan* P0 = plans[0];
  // Per-instance set-up, eagerly on `s`: prelude with its domain check, the
  // initial state, the seed and the zeroed adjoint accumulators.
  for (int k = 0; k < count; ++k) {
    lks_plan* P = plans[k];
    void* ws = workspace[k];
    if (lks_status e = prelude(P, gamma[k], chi[k], psi[k], ws, s)) {
      return fail(e, "instance " + std::to_string(k) + ": " + lks_last_error());
    }
    HIPCHK(launch_state_init(P->g, P->prec, ck_slot(P, ws, 0), s));
    P->first_lazy = 1;
    if (dJ) {
      HIPCHK(hipMemcpyAsync(wsp(ws, P->o_seed), dJ + k, sizeof(double), hipMemcpyDeviceToDevice,
                            s));
    } else {
      const double one = 1.0;
      HIPCHK(hipMemcpyAsync(wsp(ws, P->o_seed), &one, sizeof(double), hipMemcpyHostToDevice, s));
    }
    HIPCHK(launch_zero(lam_slot(P, ws, 0), (size_t)P->S * P->es, s));
    if (P->alks) HIPCHK(launch_zero(xadj_slot(P, ws, 0), (size_t)P->g.d * P->g.N * P->es, s));
    HIPCHK(launch_zero(wsp(ws, P->o_badj), body_bytes(P), s));
    HIPCHK(launch_zero(wsp(ws, P->o_krefbar), (size_t)P->g.Mtot * sizeof(double), s));
    HIPCHK(hipMemcpyAsync(wsp(ws, P->o_geo), &P->g, sizeof(Geo), hipMemcpyHostToDevice, s));
  }
  // 2D J1 instances with a common step count, checkpoint interval, precision,
  // body-tape mode and adjoint scheme share every launch (groups of
  // BATCH_MAX); others run as graph branches
  bool shared = true;
  for (int k = 0; k < count; ++k)
    shared = shared && plans[k]->g.d == 2 && plans[k]->prec == P0->prec &&
             plans[k]->g.nt == P0->g.nt && plans[k]->K == P0->K && plans[k]->nck == P0->nck &&
             plans[k]->full_btape == P0->full_btape && plans[k]->alks == P0->alks &&
             !plans[k]->j2;
  // one graph: instance k's forward march, objective copy, adjoint march and
  // epilogue form branch k, forked from and joined to the launch stream
  std::vector<const void*> key;
  key.push_back((const void*)(intptr_t)count);
  for (int k = 0; k < count; ++k) {
    key.insert(key.end(), {plans[k], gamma[k], workspace[k], J_out[k], dJ_dgamma[k], dJ_dchi[k],
                           dJ_dpsi[k]});
  }
  auto shared_march = [&](hipStream_t st) -> lks_status {
    for (int k0 = 0; k0 < count; k0 += BATCH_MAX) {
      const int c = std::min(BATCH_MAX, count - k0);
      if (lks_status e = batched_march(c, plans + k0, workspace + k0, gamma + k0, J_out + k0,
                                       dJ_dgamma + k0, dJ_dchi + k0, dJ_dpsi + k0, st))
        return e;
    }
    return LKS_OK;
  };
  auto branch = [&](int k, hipStream_t st) -> lks_status {
    lks_plan* P = plans[k];
    void* ws = workspace[k];
    if (lks_status e = forward_loop(P, ws, st)) return e;
    HIPCHK(hipMemcpyAsync(J_out[k], wsp(ws, P->o_J3), 3 * sizeof(double),
                          hipMemcpyDeviceToDevice, st));
    if (lks_status e = adjoint_loop(P, ws, st, false)) return e;
    return sens(P, gamma[k], ws, dJ_dgamma[k], dJ_dchi[k], dJ_dpsi[k], st);
  };
  key.push_back((const void*)(intptr_t)(shared ? 1 : 0));
  if (!P0->use_graphs || g_prof.on) {
    if (shared) {
      if (lks_status e = shared_march(s)) return e;
    } else {
      for (int k = 0; k < count; ++k)
        if (lks_status e = branch(k, s)) return e;
    }
  } else if (shared) {
    GraphCache& gc = P0->gbatch;
    if (!(gc.exec && P0->bkey == key)) {
      gc.reset();
      P0->bkey.clear();
      if (lks_status e = run_loop(P0, gc, workspace[0], 0, s, shared_march)) return e;
      P0->bkey = key;
    } else {
      HIPCHK(hipGraphLaunch(gc.exec, s));
    }
  } else {
    GraphCache& gc = P0->gbatch;
    if (!(gc.exec && P0->bkey == key)) {
      gc.reset();
      P0->bkey.clear();
      if (!P0->cap) HIPCHK(hipStreamCreateWithFlags(&P0->cap, hipStreamNonBlocking));
      while ((int)P0->bstreams.size() < count) {
        hipStream_t b;
        HIPCHK(hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
        P0->bstreams.push_back(b);
      }
      std::vector<hipEvent_t> evs(count + 1, nullptr);
      for (auto& e : evs) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      auto destroy = [&]() {
        for (auto& e : evs) (void)hipEventDestroy(e);
      };
      HIPCHK(hipStreamBeginCapture(P0->cap, hipStreamCaptureModeThreadLocal));
      lks_status err = LKS_OK;
      hipError_t he = hipEventRecord(evs[count], P0->cap);
      for (int k = 0; k < count && !err && he == hipSuccess; ++k) {
        hipStream_t b = P0->bstreams[k];
        he = hipStreamWaitEvent(b, evs[count], 0);
        if (he == hipSuccess) err = branch(k, b);
        if (!err && he == hipSuccess) he = hipEventRecord(evs[k], b);
        if (!err && he == hipSuccess) he = hipStreamWaitEvent(P0->cap, evs[k], 0);
      }
      hipGraph_t graph = nullptr;
      hipError_t ce = hipStreamEndCapture(P0->cap, &graph);
      destroy();
      if (err || he != hipSuccess || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (err) return err;
        return fail(LKS_EHIP, std::string("batch capture: ") +
                                  hipGetErrorString(he != hipSuccess ? he : ce));
      }
      hipError_t ie = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        gc.exec = nullptr;
        return fail(LKS_EHIP, std::string("batch graph instantiate: ") + hipGetErrorString(ie));
      }
      P0->bkey = key;
    }
    HIPCHK(hipGraphLaunch(gc.exec, s));
  }
  // instability flags of every instance (one synchronisation)
  std::vector<int> flags(count, 0);
  for (int k = 0; k < count; ++k)
    HIPCHK(hipMemcpyAsync(&flags[k], wsp(workspace[k], plans[k]->o_flags), sizeof(int),
                          hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int k = 0; k < count; ++k) plans[k]->fwd_ws = workspace[k];
  for (int k = 0; k < count; ++k)
    if (flags[k])
      return fail(LKS_EUNSTABLE, "instance " + std::to_string(k) +
                                     ": the march produced |u| >= 0.5 or a non-finite value");
  return LKS_OK;
}

// ---- Algorithm 1 driver
namespace {
struct OptScratch {
  double *phys, *dphys, *dg, *dchi, *dpsi, *work, *dG1p, *dG2p, *dG1, *dG2, *dG3, *J3, *G;
  void *st_a, *st_b, *adj_a, *adj_b;
  size_t total;
};
OptScratch opt_layout(const lks_plan* P, void* base) {
  OptScratch o;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    void* p = base ? (char*)base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const size_t M = (size_t)inner_points(P->g), nt = (size_t)P->g.nt;
  const size_t np = P->g.rot ? 3 : 1;
  const size_t Sb = (size_t)P->S * P->es;
  const size_t Ab = P->alks ? (size_t)(P->g.d + 1 + alks_carry_planes(P->g.d)) * P->g.N * P->es : Sb;
  o.phys = (double*)take(M * 8);
  o.dphys = (double*)take(M * 8);
  o.dg = (double*)take(M * 8);
  o.dchi = (double*)take(nt * 3 * 8);
  o.dpsi = (double*)take(nt * np * 8);
  o.work = (double*)take(M * 8);
  o.dG1p = (double*)take(M * 8);
  o.dG2p = (double*)take(M * 8);
  o.dG1 = (double*)take(M * 8);
  o.dG2 = (double*)take(M * 8);
  o.dG3 = (double*)take(nt * np * 8);
  o.J3 = (double*)take(4 * 8);
  o.G = (double*)take(4 * 8);
  o.st_a = take(Sb);
  o.st_b = take(Sb);
  o.adj_a = take(Ab);
  o.adj_b = take(Ab);
  o.total = off;
  return o;
}
}  // namespace

size_t lks_optimize_scratch_bytes(const lks_plan* P) {
  if (!P) return 0;
  return opt_layout(P, nullptr).total;
}

lks_status lks_optimize(lks_plan* P, void* ws, const lks_opt_options* opt, double* gamma,
                        double* chi, double* psi, void* scratch, lks_update_fn update, void* user,
                        double* history, lks_opt_result* result, hipStream_t s) {
  if (!P || !ws || !opt || !gamma || !chi || !psi || !scratch || !update)
    return fail(LKS_EINVAL, "null argument");
  if (opt->n_cont < 1 || opt->n_opt < 1 || !opt->beta)
    return fail(LKS_EINVAL, "lks_optimize needs n_cont >= 1, n_opt >= 1 and a beta schedule");
  if (!(opt->tol >= 0.0)) return fail(LKS_EINVAL, "tol must be >= 0");
  const OptScratch o = opt_layout(P, scratch);
  const double one = 1.0;
  double* seed = o.J3 + 3;
  HIPCHK(hipMemcpyAsync(seed, &one, sizeof(double), hipMemcpyHostToDevice, s));
  lks_opt_result res;
  memset(&res, 0, sizeof res);
  bool have_state = false, have_adj = false;
  void* st_cur = o.st_a;   // final state of the last march
  void* adj_cur = o.adj_a; // adj_initial of the last sweep
  int total = 0;
  for (int l = 0; l < opt->n_cont; ++l) {
    res.levels = l + 1;
    const double beta = opt->beta[l];
    double J_prev = 0.0;
    for (int k = 0; k < opt->n_opt; ++k) {
      // filter and project the density, march, objective and constraints
      if (lks_status e = lks_design_filter(P, gamma, opt->radius, beta, opt->eta, o.phys, s))
        return e;
      void* st_next = st_cur == o.st_a ? o.st_b : o.st_a;
      const bool carry = opt->periodic && have_state;
      if (lks_status e = lks_forward(P, o.phys, chi, psi, carry ? st_cur : nullptr, st_next, ws,
                                     o.J3, s))
        return e;
      st_cur = st_next;
      have_state = true;
      if (lks_status e = lks_constraints(P, ws, o.phys, chi, psi, opt->vmax, opt->omega_max,
                                         opt->p_omega, o.G, o.dG1p, o.dG2p, o.dG3, s))
        return e;
      double JG[4];
      HIPCHK(hipMemcpyAsync(JG, o.J3, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(JG + 1, o.G, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (history) memcpy(history + 4 * (size_t)total, JG, sizeof JG);
      ++total;
      res.iterations = total;
      res.J_last = JG[0];
      // Sec. 3.2: the level ends once J settles with the constraints met
      bool feasible = true;
      for (int j = 0; j < 3; ++j)
        if ((opt->g_active >> j) & 1) feasible = feasible && JG[1 + j] <= 0.0;
      const bool settled = k > 0 && std::fabs(JG[0] - J_prev) <= opt->tol * std::fabs(J_prev);
      J_prev = JG[0];
      if (settled && feasible) break;
      // reverse sweep and the chain rule back to the design variables
      void* adj_next = adj_cur == o.adj_a ? o.adj_b : o.adj_a;
      const bool acarry = opt->periodic && have_adj;
      if (lks_status e = lks_adjoint(P, o.phys, chi, psi, ws, seed, acarry ? adj_cur : nullptr,
                                     adj_next, o.dphys, o.dchi, o.dpsi, s))
        return e;
      adj_cur = adj_next;
      have_adj = true;
      if (lks_status e = lks_design_filter_adjoint(P, gamma, opt->radius, beta, opt->eta, o.dphys,
                                                   o.work, o.dg, s))
        return e;
      if (lks_status e = lks_design_filter_adjoint(P, gamma, opt->radius, beta, opt->eta, o.dG1p,
                                                   o.work, o.dG1, s))
        return e;
      if (lks_status e = lks_design_filter_adjoint(P, gamma, opt->radius, beta, opt->eta, o.dG2p,
                                                   o.work, o.dG2, s))
        return e;
      lks_opt_state st;
      st.level = l;
      st.iter = k;
      st.total = total;
      st.beta = beta;
      st.J = JG[0];
      for (int j = 0; j < 3; ++j) st.G[j] = JG[1 + j];
      st.gamma = gamma;
      st.chi = chi;
      st.psi = psi;
      st.dJ_dgamma = o.dg;
      st.dJ_dchi = o.dchi;
      st.dJ_dpsi = o.dpsi;
      st.dG1_dgamma = o.dG1;
      st.dG2_dgamma = o.dG2;
      st.dG3_dpsi = o.dG3;
      if (update(user, &st, s) != 0) {
        res.stopped = 1;
        if (result) *result = res;
        return LKS_OK;
      }
    }
  }
  if (result) *result = res;
  return LKS_OK;
}

lks_status lks_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (auto& r : g_prof.recs) {
    g_prof.pool.push_back(r.a);
    g_prof.pool.push_back(r.b);
  }
  g_prof.recs.clear();
  g_prof.on = on != 0;
  return LKS_OK;
}

int32_t lks_profile_read(const char** names, double* total_ms, int64_t* launches, int32_t cap) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  std::vector<double> tot(g_prof.names.size(), 0.0);
  std::vector<int64_t> cnt(g_prof.names.size(), 0);
  for (auto& r : g_prof.recs) {
    (void)hipEventSynchronize(r.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      tot[r.cls] += ms;
      cnt[r.cls] += 1;
    }
  }
  int32_t k = 0;
  for (size_t i = 0; i < g_prof.names.size() && k < cap; ++i, ++k) {
    if (names) names[k] = g_prof.names[i].c_str();
    if (total_ms) total_ms[k] = tot[i];
    if (launches) launches[k] = cnt[i];
  }
  return k;
}

}  // extern "C"
