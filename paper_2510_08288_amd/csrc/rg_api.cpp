// Host side of the C ABI declared in include/rg.h: argument validation,
// workspace layout, and the enqueue order of one RG step (see rg_kernels.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/rg.h"
#include "rg_async.hpp"
#include "rg_internal.hpp"

using namespace rg;

struct rg_handle {
  Problem pr;
  rg_options opt;
  LaunchCfg cfg;
  // device memory
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  bool ws_ready = false;
  DevBuffers b{};
  // host mirrors
  uint32_t t = 0;
  long long gen_t = -1;  // RG step whose draws are in the streamed buffer
  std::string err;
  // captured generic closed-loop rounds: kGraphRounds of them, and one
  hipGraphExec_t round_graph[2] = {};
  // host copy of a fresh search record (uploaded by ensure_workspace and by
  // every allocation-free step); allocated with the handle
  DevSearch* srch_tmpl = nullptr;
  // profiling
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  rg_profile prof{};
};

namespace {

thread_local std::string g_create_error;

int fail(rg_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  else g_create_error = msg;
  return code;
}

int fail_hip(rg_handle* h, const char* what, hipError_t e) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(h, RG_E_HIP, m);
}

#define HIPCHK(h, call)                              \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return fail_hip(h, #call, e_); \
  } while (0)

// How many later steps' probes a probe-only round may also run (closed loop,
// bisection with first-round prediction, FP32 quad rollouts on streamed draws).
int32_t spec_allowed(const rg_handle* h) {
  const bool ok = h->opt.search == RG_SEARCH_BISECT && h->opt.predict &&
                  h->pr.s.rng_mode == RG_RNG_STREAM &&
                  rollout_uses_quad(h->pr, h->cfg, h->opt.precision);
  return ok ? h->opt.speculate : 0;
}

// Later steps a held step speculates on: each adds a whole first round (the
// probe and K midpoints) within the candidates of one round.  Held rounds are
// already two-thirds throughput-bound (many candidates die early, the small
// ones run long), so one step ahead pays and more do not (200-update bench
// loop: 0.292 ms per update without, 0.276 with one step, 0.283 with two,
// 0.286 with three).
constexpr int32_t kHoldMax = 1;
int32_t hold_allowed(const rg_handle* h) {
  int32_t d = spec_allowed(h);
  if (d > kHoldMax) d = kHoldMax;
  while (d > 0 && (1 + h->opt.K) * (1 + d) > kCMax) --d;
  return d;
}

void drop_graphs(rg_handle* h) {
  for (hipGraphExec_t& g : h->round_graph) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

bool finite_array(const double* a, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Both Newton searches: the adjoint-driven one and the forward-tangent one.
bool is_newton(int search) { return search == RG_SEARCH_NEWTON || search == RG_SEARCH_NEWTON_TAN; }

// Alg. 2 tabulates the steady-state margins of the 2^K bisection-tree nodes.
constexpr int kAlg2MaxK = 16;

// Workspace layout: offsets of each buffer inside one allocation.
struct Layout {
  size_t st, srch, res, r_seq, x_hist, wpair[kPairs], thpair[kPairs], rlist, per_m, per_j, per_key;
  size_t alg2_mss, tan_dv, scratch;
  size_t grad, adj_k, adj_w, adj_m, adj_dv, adj_dth, adj_ckpt, adj_seg;
  size_t seg_m, seg_j, seg_r, seg_x, seg_a, seg_cv, seg_ct, seg_scr, total;
};

Layout layout_of(const rg_handle* h) {
  const Problem& pr = h->pr;
  const size_t N = (size_t)pr.s.N;
  const size_t T = (size_t)h->opt.max_T;
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.st = take(sizeof(DevState));
  L.srch = take(sizeof(DevSearch));
  L.res = take(sizeof(DevResult) * T);
  L.r_seq = take(sizeof(double) * T);
  L.x_hist = take(sizeof(double) * (T + 1) * kMaxN);
  const size_t wbytes =
      pr.s.rng_mode == RG_RNG_STREAM ? sizeof(float) * (size_t)(pr.H + kQuadGroup) * pr.p.nw * N : 0;
  const size_t thbytes = pr.s.rng_mode == RG_RNG_STREAM ? sizeof(float) * (size_t)pr.p.nth * N : 0;
  for (int i = 0; i < kPairs; ++i) {
    L.wpair[i] = take(wbytes);
    L.thpair[i] = take(thbytes);
  }
  L.rlist = take(sizeof(int2) * (size_t)kCMax * N);
  L.per_m = take(sizeof(float) * (size_t)kCMax * N);
  L.per_j = take(sizeof(int32_t) * (size_t)kCMax * N);
  L.per_key = take(h->opt.chance_q > 0 ? sizeof(unsigned long long) * (size_t)kCMax * N : 0);
  L.alg2_mss = take(h->opt.search == RG_SEARCH_ALG2 ? sizeof(double) << h->opt.K : 0);
  L.tan_dv = take(sizeof(float) * N);
  L.scratch = take(sizeof(double) * kCMax * 4);
  const size_t n = (size_t)pr.p.n, Kc = (size_t)h->opt.Kc;
  L.grad = take(sizeof(DevGrad));
  L.adj_k = take(sizeof(int32_t) * N);
  L.adj_w = take(sizeof(float) * N);
  L.adj_m = take(sizeof(float) * N);
  L.adj_dv = take(sizeof(double) * N);
  L.adj_dth = take(sizeof(double) * kMaxTh * N);
  L.adj_ckpt = take(sizeof(float) * ((size_t)pr.H / Kc + 1) * n * N);
  L.adj_seg = take(sizeof(float) * Kc * n * N);
  const size_t S = (size_t)pr.H / Kc + 1;
  L.seg_m = take(sizeof(float) * S);
  L.seg_j = take(sizeof(int32_t) * S);
  L.seg_r = take(sizeof(int32_t) * S);
  L.seg_x = take(sizeof(float) * S * n);
  L.seg_a = take(sizeof(float) * S * n * n);
  L.seg_cv = take(sizeof(double) * S * n);
  L.seg_ct = take(sizeof(double) * S * n * kMaxTh);
  L.seg_scr = take(sizeof(float) * Kc * n * S * n);
  L.total = off;
  return L;
}

// Scenario-candidate pairs of one round up to which the 9-state FP32 rollouts
// run one scenario per group of 16 lanes (auto lanes): one lane per scenario
// leaves the chip mostly idle there and each round is bound by the latency of
// a whole RK4 step on one lane; with more pairs the groups' extra instructions
// (exchanges, lanes 9..15) cost more than the latency they save (measured:
// the 32-point grid at H = 1024 is 2.7x faster with groups at 16384 pairs,
// 2.0x at 32768, slower from about 100000; the adjoint Newton search 1.7x
// faster at N = 4096 and 10 % slower at N = 16384).
constexpr double kGroupPairsMax = 32768;

int lanes_for(const rg_handle* h) {
  const bool f32_robust = h->opt.precision == RG_PREC_F32_RECHECK && h->opt.chance_q == 0;
  // the quad kernel: FP32 rollouts, robust or chance-constrained verdict
  const bool quad_ok = h->pr.p.kind == RG_PLANT_LQ4 && h->opt.precision == RG_PREC_F32_RECHECK;
  // the 9-state groups: robust verdict; the forward tangent runs on one lane
  const bool group_ok =
      h->pr.p.kind == RG_PLANT_FC9 && f32_robust && h->opt.search != RG_SEARCH_NEWTON_TAN;
  if (h->opt.lanes == 4) return quad_ok ? 4 : 1;
  if (h->opt.lanes == 16) return group_ok ? 16 : 1;
  if (h->opt.lanes == 1) return 1;
  return quad_ok ? 4 : (group_ok ? 16 : 1);
}

int depth_for(const rg_handle* h, int lanes) {
  if (h->opt.depth > 0) return h->opt.depth;
  // Enough candidates per round to give every SIMD of the chip up to four
  // wavefronts (a round of few candidates is bound by one wave's latency, so
  // more waves per SIMD come almost free), then the smallest depth that needs
  // no more rounds.
  const int goal = h->opt.search == RG_SEARCH_GRID ? h->opt.refine : h->opt.K;
  const double lanes_budget = 4.0 * 256 * 4 * 64;
  const double per_cand = (double)h->pr.s.N * lanes;
  int dmax = 1;
  while (dmax < 6 && ((1 << (dmax + 1)) - 1) * per_cand <= lanes_budget) ++dmax;
  if (goal <= 0) return 1;
  const int rounds = (goal + dmax - 1) / dmax;
  return (goal + rounds - 1) / rounds;
}

void plan_with(rg_handle* h, int lanes);

void plan(rg_handle* h) {
  const bool auto_lanes = h->opt.lanes == 0;
  const int depth0 = h->opt.depth;  // 0: auto
  plan_with(h, lanes_for(h));
  // auto: 9-state groups only for rounds of few scenario-candidate pairs
  if (auto_lanes && h->cfg.lanes == 16 &&
      (double)h->cfg.cmax_round * h->pr.s.N > kGroupPairsMax) {
    h->opt.depth = depth0;
    plan_with(h, 1);
  }
}

void plan_with(rg_handle* h, int lanes) {
  const int d = depth_for(h, lanes);
  h->opt.depth = d;
  h->opt.lanes = lanes;
  LaunchCfg c;
  c.lanes = lanes;
  c.block = h->opt.block > 0 ? h->opt.block : 256;
  c.chance = h->opt.chance_q > 0 ? 1 : 0;
  const int tree = (1 << d) - 1;
  c.tan = h->opt.search == RG_SEARCH_NEWTON_TAN ? 1 : 0;
  if (is_newton(h->opt.search)) {
    // four candidates per Newton round; with prediction, round 0 after a held
    // step holds the probe and the K midpoints towards 0
    c.cmax_round = h->opt.predict && 1 + h->opt.K > 4 ? 1 + h->opt.K : 4;
    c.rounds = h->opt.K + 2;
  } else if (h->opt.search == RG_SEARCH_GRID) {
    c.cmax_round = h->opt.M > tree ? h->opt.M : tree;
    c.rounds = 1 + (h->opt.refine + d - 1) / d;
  } else {
    const int d0 = h->opt.K < d ? h->opt.K : d;
    const int r0 = 1 << d0;
    c.cmax_round = r0 > tree ? r0 : tree;
    c.rounds = 1 + (h->opt.K - d0 + d - 1) / d;
    if (h->opt.predict) {  // round 0: probe + the predicted path (K midpoints), or the probe alone
      if (1 + h->opt.K > c.cmax_round) c.cmax_round = 1 + h->opt.K;
      c.rounds = 1 + (h->opt.K + d - 1) / d;
    }
  }
  h->cfg = c;
  // a probe-only round 0 holds the probe and the probes of the next steps
  const int sp = spec_allowed(h);
  if (1 + sp > h->cfg.cmax_round) h->cfg.cmax_round = 1 + sp;
  // a held step's round 0 holds its own first round and those of the next steps
  const int hd = hold_allowed(h);
  if (hd > 0 && (1 + h->opt.K) * (1 + hd) > h->cfg.cmax_round)
    h->cfg.cmax_round = (1 + h->opt.K) * (1 + hd);
}

// Search record of a fresh handle: configuration, no step in progress, no
// prediction, empty steady-state cache.
void fill_search(const rg_handle* h, DevSearch* S, int32_t spec_depth, int32_t spec_hold) {
  memset(S, 0, sizeof(DevSearch));
  S->mode = h->opt.search == RG_SEARCH_GRID ? kGrid
            : is_newton(h->opt.search) ? kNewton : kBisect;
  S->delta = std::ldexp(1.0, -h->opt.K);
  S->predict = h->opt.search == RG_SEARCH_BISECT || is_newton(h->opt.search) ? h->opt.predict : 0;
  S->pred = std::nan("");
  S->K = h->opt.K;
  S->depth = h->opt.depth;
  S->M = h->opt.M;
  S->refine = h->opt.refine;
  S->precision = h->opt.precision;
  S->ss_check = h->pr.c.ss_check;
  S->n_c = h->pr.c.n_c;
  S->ny = h->pr.p.ny;
  S->eps = h->pr.c.eps;
  for (int r = 0; r < kNC; ++r) S->g[r] = h->pr.c.g[r];
  for (int i = 0; i < kNC * kMaxY; ++i) S->F[i] = h->pr.c.F[i];
  S->done = 1;
  for (int i = 0; i < kMssCache; ++i) S->mss_v[i] = std::nan("");  // empty cache
  S->spec_depth = spec_depth;
  S->spec_hold = spec_hold;
  S->spec_n = 0;
  S->spec_used = 0;
  S->band = h->opt.band;
  S->q = h->opt.chance_q;
}

int ensure_workspace(rg_handle* h) {
  if (h->ws_ready) return RG_OK;
  const Layout L = layout_of(h);
  if (!h->ws) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, L.total);
    if (e != hipSuccess) return fail(h, RG_E_NOMEM, std::string("hipMalloc workspace: ") + hipGetErrorString(e));
    h->ws = p;
    h->ws_bytes = L.total;
    h->ws_owned = true;
  }
  char* base = (char*)h->ws;
  DevBuffers& b = h->b;
  b.st = (DevState*)(base + L.st);
  b.srch = (DevSearch*)(base + L.srch);
  b.res = (DevResult*)(base + L.res);
  b.r_seq = (double*)(base + L.r_seq);
  b.x_hist = (double*)(base + L.x_hist);
  for (int i = 0; i < kPairs; ++i) {
    b.wpair[i] = (float*)(base + L.wpair[i]);
    b.thpair[i] = (float*)(base + L.thpair[i]);
  }
  b.wbuf = b.wpair[0];  // single steps, rg_margin, rg_grad, rg_draws
  b.thbuf = b.thpair[0];
  b.rlist = (int2*)(base + L.rlist);
  b.per_m = (float*)(base + L.per_m);
  b.per_j = (int32_t*)(base + L.per_j);
  b.per_key = h->opt.chance_q > 0 ? (unsigned long long*)(base + L.per_key) : nullptr;
  b.alg2_mss = h->opt.search == RG_SEARCH_ALG2 ? (double*)(base + L.alg2_mss) : nullptr;
  b.tan_dv = (float*)(base + L.tan_dv);
  b.scratch = (double*)(base + L.scratch);
  b.scratch_bytes = sizeof(double) * kCMax * 4;
  b.grad = (DevGrad*)(base + L.grad);
  b.adj_k = (int32_t*)(base + L.adj_k);
  b.adj_w = (float*)(base + L.adj_w);
  b.adj_m = (float*)(base + L.adj_m);
  b.adj_dv = (double*)(base + L.adj_dv);
  b.adj_dth = (double*)(base + L.adj_dth);
  b.adj_ckpt = (float*)(base + L.adj_ckpt);
  b.adj_seg = (float*)(base + L.adj_seg);
  b.seg_m = (float*)(base + L.seg_m);
  b.seg_j = (int32_t*)(base + L.seg_j);
  b.seg_r = (int32_t*)(base + L.seg_r);
  b.seg_x = (float*)(base + L.seg_x);
  b.seg_a = (float*)(base + L.seg_a);
  b.seg_cv = (double*)(base + L.seg_cv);
  b.seg_ct = (double*)(base + L.seg_ct);
  b.seg_scr = (float*)(base + L.seg_scr);
  // Search configuration.
  fill_search(h, h->srch_tmpl, spec_allowed(h), hold_allowed(h));
  hipError_t e =
      hipMemcpyAsync(b.srch, h->srch_tmpl, sizeof(DevSearch), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(h, "upload search configuration", e);
  h->ws_ready = true;
  return RG_OK;
}

int upload_state(rg_handle* h, const double* x, double r, double v_prev) {
  DevState s;
  memset(&s, 0, sizeof(s));
  for (int i = 0; i < h->pr.p.n; ++i) s.x[i] = x[i];
  s.v_prev = v_prev;
  s.r = r;
  s.t = h->t;
  s.cl_index = 0;
  HIPCHK(h, hipMemcpyAsync(h->b.st, &s, sizeof(s), hipMemcpyHostToDevice, h->stream));
  // The copy reads a stack object: wait for it before returning.
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return RG_OK;
}

// Draws for the current t into the streamed buffer (no-op in inline mode or if current).
int ensure_draws(rg_handle* h) {
  if (h->pr.s.rng_mode != RG_RNG_STREAM) return RG_OK;
  if (h->gen_t == (long long)h->t) return RG_OK;
  HIPCHK(h, launch_gen(h->pr, h->b, h->stream));
  h->gen_t = (long long)h->t;
  return RG_OK;
}

hipError_t next_event(rg_handle* h, hipEvent_t* ev) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    h->ev_pool.push_back(e);
  }
  *ev = h->ev_pool[h->ev_used++];
  return hipSuccess;
}

// Read back the event pairs recorded since the last harvest.
hipError_t harvest_events(rg_handle* h) {
  for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, h->ev_pool[i], h->ev_pool[i + 1]);
    if (e != hipSuccess) return e;
    h->prof.rollout_ms += ms;
    h->prof.rollout_launches += 1;
  }
  h->ev_used = 0;
  return hipSuccess;
}

// Draw pair i of the closed loop (step s uses pair s % kPairs).
void draw_pair(const rg_handle* h, int i, float** w, float** th) {
  *w = h->b.wpair[i % kPairs];
  *th = h->b.thpair[i % kPairs];
}

// Enqueue one RG step of rg_step: draws and round-0 setup, the planned rounds,
// the result record.
// pr and b default to the handle's own problem and workspace; the
// allocation-free step passes its inline-draw problem and static scratch (and
// profiling off, which would create events).
hipError_t enqueue_step(rg_handle* h, const Problem& pr, const DevBuffers& b, bool profile) {
  hipError_t e;
  const int prec = h->opt.precision;
  const double band = prec == RG_PREC_F32_RECHECK ? h->opt.band : 0.0;
  const bool streamed = pr.s.rng_mode == RG_RNG_STREAM;
  // draws and round-0 setup share a launch in stream mode
  e = streamed ? launch_gen_setup(pr, b, 0, h->stream) : launch_setup(pr, b, 0, h->stream);
  if (e != hipSuccess) return e;
  const bool newton = is_newton(h->opt.search);
  // with FP32 rollouts the recheck launch ends with the decision (the Newton
  // decision needs the derivative first)
  const bool chance = h->opt.chance_q > 0;
  const bool fused_decide = prec == RG_PREC_F32_RECHECK && !newton && !chance;
  for (int r = 0; r < h->cfg.rounds; ++r) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (profile) {
      if ((e = next_event(h, &e0)) != hipSuccess || (e = next_event(h, &e1)) != hipSuccess) return e;
      if ((e = hipEventRecord(e0, h->stream)) != hipSuccess) return e;
    }
    // the Newton iterate keeps checkpoints for its derivative
    if ((e = launch_rollout(pr, band, prec, h->opt.early_exit, 0, h->cfg, b, h->stream,
                            newton ? -1 : -2, h->opt.Kc)) != hipSuccess)
      return e;
    if (profile && (e = hipEventRecord(e1, h->stream)) != hipSuccess) return e;
    if (prec == RG_PREC_F32_RECHECK &&
        (e = launch_recheck(pr, h->opt.early_exit, h->cfg, b, h->stream, fused_decide)) !=
            hipSuccess)
      return e;
    if (newton && h->cfg.tan) {  // derivative from the tangent the rollout carried
      if ((e = launch_tan_grad(pr, b, -1, h->stream)) != hipSuccess) return e;
    } else if (newton) {  // derivative of the Newton iterate's worst margin (segment adjoint)
      if ((e = launch_grad_prepare(pr, b, -1, 1, h->stream)) != hipSuccess) return e;
      if ((e = launch_seg_grad(pr, h->opt.Kc, -1, b, h->stream)) != hipSuccess) return e;
      if ((e = launch_grad_reduce(b, 1, pr.p.nth, -1, h->stream)) != hipSuccess) return e;
    }
    if (chance && (e = launch_select_q(b, pr.s.N, h->cfg.cmax_round, 0, h->stream)) != hipSuccess)
      return e;
    if (!fused_decide && (e = launch_decide(pr, b, h->stream)) != hipSuccess) return e;
  }
  return launch_finalize(pr, 0, b, h->stream);
}

// Enqueue one generic round of the closed loop: whatever round the current
// step's search is at.  The kernels take the step from the device state and
// select its draw buffers themselves (pair t % kPairs; the speculative probe of
// step t + j reads pair (t + j) % kPairs); the first round of each step also
// generates the draws of step t + kSpecMax + 1.  The result launch records the
// step only once its search has ended, applies the true-plant step and
// prepares round 0 of the next step, so a step costs the rounds it needs and a
// step decided ahead costs one round of launches that return at once.
hipError_t enqueue_round(rg_handle* h) {
  hipError_t e;
  const int prec = h->opt.precision;
  const double band = prec == RG_PREC_F32_RECHECK ? h->opt.band : 0.0;
  const bool streamed = h->pr.s.rng_mode == RG_RNG_STREAM;
  DevBuffers b = h->b;
  b.ring = 1;
  // any non-null target switches the draw workgroups on; the kernel picks the buffer
  float* gen_w = streamed ? b.wpair[0] : nullptr;
  float* gen_th = streamed ? b.thpair[0] : nullptr;
  const bool newton = is_newton(h->opt.search);
  const bool chance = h->opt.chance_q > 0;
  const bool fused_decide = prec == RG_PREC_F32_RECHECK && !newton && !chance;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->profiling) {
    if ((e = next_event(h, &e0)) != hipSuccess || (e = next_event(h, &e1)) != hipSuccess) return e;
    if ((e = hipEventRecord(e0, h->stream)) != hipSuccess) return e;
  }
  if ((e = launch_rollout(h->pr, band, prec, h->opt.early_exit, 0, h->cfg, b, h->stream,
                          newton ? -1 : -2, h->opt.Kc, gen_w, gen_th)) != hipSuccess)
    return e;
  if (h->profiling && (e = hipEventRecord(e1, h->stream)) != hipSuccess) return e;
  if (prec == RG_PREC_F32_RECHECK &&
      (e = launch_recheck(h->pr, h->opt.early_exit, h->cfg, b, h->stream, fused_decide)) !=
          hipSuccess)
    return e;
  if (newton && h->cfg.tan) {
    if ((e = launch_tan_grad(h->pr, b, -1, h->stream)) != hipSuccess) return e;
  } else if (newton) {
    if ((e = launch_grad_prepare(h->pr, b, -1, 1, h->stream)) != hipSuccess) return e;
    if ((e = launch_seg_grad(h->pr, h->opt.Kc, -1, b, h->stream)) != hipSuccess) return e;
    if ((e = launch_grad_reduce(b, 1, h->pr.p.nth, -1, h->stream)) != hipSuccess) return e;
  }
  if (chance && (e = launch_select_q(b, h->pr.s.N, h->cfg.cmax_round, 0, h->stream)) != hipSuccess)
    return e;
  if (!fused_decide && (e = launch_decide(h->pr, b, h->stream)) != hipSuccess) return e;
  return launch_finalize(h->pr, 1, b, h->stream, 1, 1);
}

// One RG step under Alg. 2: this step's draws (streamed mode), then the
// per-scenario bisections and the result record.
hipError_t enqueue_alg2(rg_handle* h) {
  hipError_t e;
  if (h->pr.s.rng_mode == RG_RNG_STREAM && (e = launch_gen(h->pr, h->b, h->stream)) != hipSuccess)
    return e;
  const int prec = h->opt.precision;
  const double band = prec == RG_PREC_F32_RECHECK ? h->opt.band : 0.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->profiling) {
    if ((e = next_event(h, &e0)) != hipSuccess || (e = next_event(h, &e1)) != hipSuccess) return e;
    if ((e = hipEventRecord(e0, h->stream)) != hipSuccess) return e;
  }
  if ((e = launch_alg2(h->pr, band, prec, h->opt.early_exit, h->opt.K, h->cfg.block, h->b,
                       h->stream)) != hipSuccess)
    return e;
  if (h->profiling && (e = hipEventRecord(e1, h->stream)) != hipSuccess) return e;
  return hipSuccess;
}

int reset_search_schedule(rg_handle* h);

void fill_info(const DevResult& R, rg_step_info* info) {
  if (!info) return;
  info->kappa = R.kappa;
  info->v = R.v;
  info->worst_margin = R.worst;
  info->status = R.status;
  info->rounds = R.rounds;
  info->candidates = R.candidates;
  info->rechecks = R.rechecks;
  info->bisect_passes = R.passes_alg1;
  info->t = R.t;
  info->lane_steps = R.lane_steps;
  info->flags = R.flags;
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free RG step (rg_step_noalloc)
// ---------------------------------------------------------------------------
// Its search state, result record and recheck list live in this file-scope
// device array instead of a workspace: one copy per GPU, held until the process
// ends and shared by every allocation-free call on that GPU.  In host code the
// name `scratch` is only a stand-in for the symbol; kernels receive the device
// address that hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;  // 8 MiB
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device

// Device address of the current device's copy of `scratch` (looked up once per
// device, with that device current).
hipError_t noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

// Offsets inside `scratch`: state, search record, result, recheck list (one
// entry per candidate and scenario of the largest round at most).
struct NoAllocLayout {
  size_t st, srch, res, rlist, total;
};

NoAllocLayout noalloc_layout(const rg_handle* h) {
  NoAllocLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.st = take(sizeof(DevState));
  L.srch = take(sizeof(DevSearch));
  L.res = take(sizeof(DevResult));
  L.rlist = take(sizeof(int2) * (size_t)h->cfg.cmax_round * (size_t)h->pr.s.N);
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

int rg_step_noalloc(rg_handle* h, const double* x, double r, double v_prev, double* v_out,
                    double* kappa_out, rg_step_info* info) {
  if (!h) return RG_E_INVAL;
  if (!x || !v_out) return fail(h, RG_E_INVAL, "NULL x or v_out");
  if (!finite_array(x, h->pr.p.n) || !std::isfinite(r) || !std::isfinite(v_prev))
    return fail(h, RG_E_INVAL, "non-finite input");
  if (h->opt.search != RG_SEARCH_BISECT && h->opt.search != RG_SEARCH_GRID)
    return fail(h, RG_E_NOTSUP, "the allocation-free step runs bisection or the grid search");
  if (h->opt.chance_q > 0)
    return fail(h, RG_E_NOTSUP, "the allocation-free step runs the robust verdict");
  if (h->profiling) return fail(h, RG_E_STATE, "the allocation-free step does not profile");
  const NoAllocLayout L = noalloc_layout(h);
  if (L.total > kNoAllocScratchBytes)
    return fail(h, RG_E_NOTSUP,
                "the allocation-free step needs " + std::to_string(L.total) +
                    " bytes of device scratch (recheck list: 8 B x N x candidates per round), "
                    "more than its " + std::to_string(kNoAllocScratchBytes) + " bytes");
  void* base = nullptr;
  hipError_t e = noalloc_scratch(&base);
  if (e != hipSuccess) return fail_hip(h, "device scratch address", e);
  char* p = (char*)base;
  DevBuffers b{};
  b.st = (DevState*)(p + L.st);
  b.srch = (DevSearch*)(p + L.srch);
  b.res = (DevResult*)(p + L.res);
  b.rlist = (int2*)(p + L.rlist);
  // draws regenerated inside the kernels (no draw buffer); bit-identical to
  // the streamed draws
  Problem pr = h->pr;
  pr.s.rng_mode = RG_RNG_INLINE;
  // every call starts from a fresh search record: the array keeps whatever the
  // last call on this GPU (any handle) left in it
  fill_search(h, h->srch_tmpl, 0, 0);
  DevState s;
  memset(&s, 0, sizeof(s));
  for (int i = 0; i < h->pr.p.n; ++i) s.x[i] = x[i];
  s.v_prev = v_prev;
  s.r = r;
  s.t = h->t;
  HIPCHK(h, hipMemcpyAsync(b.srch, h->srch_tmpl, sizeof(DevSearch), hipMemcpyHostToDevice,
                           h->stream));
  HIPCHK(h, hipMemcpyAsync(b.st, &s, sizeof(s), hipMemcpyHostToDevice, h->stream));
  e = enqueue_step(h, pr, b, false);
  if (e != hipSuccess) return fail_hip(h, "enqueue allocation-free RG step", e);
  DevResult R;
  HIPCHK(h, hipMemcpyAsync(&R, b.res, sizeof(R), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->t += 1;
  *v_out = R.v;
  if (kappa_out) *kappa_out = R.kappa;
  fill_info(R, info);
  return R.status == 0 ? RG_OK : RG_S_INFEASIBLE;
}

int rg_default_options(rg_options* opt) {
  if (!opt) return RG_E_INVAL;
  opt->precision = RG_PREC_F32_RECHECK;
  opt->band = 1e-4;
  opt->K = 12;
  opt->search = RG_SEARCH_BISECT;
  opt->depth = 0;
  opt->M = 64;
  opt->refine = 6;
  opt->early_exit = 1;
  opt->block = 0;
  opt->max_T = 256;
  opt->lanes = 0;
  opt->Kc = 50;
  opt->persistent_wgs = 0;
  opt->predict = 1;
  opt->speculate = kSpecMax;
  opt->chance_q = 0;
  return RG_OK;
}

int rg_create(const rg_plant* plant, const rg_scenarios* scen, const rg_constraints* cons,
              int32_t H, double dt, const rg_options* opt, rg_handle** out) {
  if (!out) return fail(nullptr, RG_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!plant || !scen || !cons) return fail(nullptr, RG_E_INVAL, "NULL descriptor");
  rg_options o;
  rg_default_options(&o);
  if (opt) o = *opt;
  // plant
  int n, nw, ny, nth, ncoef;
  if (plant->kind == RG_PLANT_LQ4) {
    n = 4; nw = 2; ny = 2; nth = 0; ncoef = 52;
  } else if (plant->kind == RG_PLANT_FC9) {
    n = 9; nw = 9; ny = 3; nth = 20; ncoef = 115;
  } else {
    return fail(nullptr, RG_E_INVAL, "unknown plant kind");
  }
  if (plant->n != n || plant->n_w != nw || plant->n_y != ny || plant->n_theta != nth)
    return fail(nullptr, RG_E_INVAL, "plant dimensions do not match the kind");
  if (!plant->coeffs || plant->n_coeffs != ncoef)
    return fail(nullptr, RG_E_INVAL, "plant coefficient count does not match the kind");
  if (!finite_array(plant->coeffs, ncoef)) return fail(nullptr, RG_E_INVAL, "non-finite coefficient");
  // scenarios
  if (scen->N < 1) return fail(nullptr, RG_E_INVAL, "N must be >= 1");
  if ((size_t)scen->N * kCMax > (size_t)INT32_MAX) return fail(nullptr, RG_E_NOTSUP, "N too large");
  if (!scen->w_lo || !scen->w_hi) return fail(nullptr, RG_E_INVAL, "NULL disturbance box");
  if (!finite_array(scen->w_lo, nw) || !finite_array(scen->w_hi, nw))
    return fail(nullptr, RG_E_INVAL, "non-finite disturbance box");
  for (int c = 0; c < nw; ++c)
    if (scen->w_hi[c] < scen->w_lo[c]) return fail(nullptr, RG_E_INVAL, "w_hi < w_lo");
  if (!(scen->theta_rel >= 0.0 && scen->theta_rel < 1.0))
    return fail(nullptr, RG_E_INVAL, "theta_rel must be in [0, 1)");
  if (scen->inject != RG_INJECT_ODE && scen->inject != RG_INJECT_POST)
    return fail(nullptr, RG_E_INVAL, "bad inject mode");
  if (scen->rng_mode != RG_RNG_STREAM && scen->rng_mode != RG_RNG_INLINE)
    return fail(nullptr, RG_E_INVAL, "bad rng mode");
  // constraints
  if (cons->n_c < 1) return fail(nullptr, RG_E_INVAL, "n_c must be >= 1");
  if (cons->n_c > kNC) return fail(nullptr, RG_E_NOTSUP, "at most 4 constraint rows");
  if (!cons->F || !cons->g) return fail(nullptr, RG_E_INVAL, "NULL constraint arrays");
  if (!finite_array(cons->F, cons->n_c * ny) || !finite_array(cons->g, cons->n_c))
    return fail(nullptr, RG_E_INVAL, "non-finite constraint data");
  if (!(cons->eps >= 0.0 && cons->eps < 1.0)) return fail(nullptr, RG_E_INVAL, "eps must be in [0, 1)");
  // horizon and options
  if (H < 1) return fail(nullptr, RG_E_INVAL, "H must be >= 1");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(nullptr, RG_E_INVAL, "dt must be > 0");
  if (o.precision != RG_PREC_F32_RECHECK && o.precision != RG_PREC_F64)
    return fail(nullptr, RG_E_INVAL, "bad precision");
  if (!(o.band >= 0.0) || !std::isfinite(o.band)) return fail(nullptr, RG_E_INVAL, "bad band");
  if (o.K < 0 || o.K > 40) return fail(nullptr, RG_E_INVAL, "K must be in [0, 40]");
  if (o.search != RG_SEARCH_BISECT && o.search != RG_SEARCH_GRID && o.search != RG_SEARCH_NEWTON &&
      o.search != RG_SEARCH_ALG2 && o.search != RG_SEARCH_NEWTON_TAN)
    return fail(nullptr, RG_E_INVAL, "bad search");
  if (o.search == RG_SEARCH_ALG2 && o.K > kAlg2MaxK)
    return fail(nullptr, RG_E_NOTSUP, "Alg. 2 keeps K <= 16 (steady-state table of 2^K nodes)");
  if (is_newton(o.search) && o.precision != RG_PREC_F32_RECHECK)
    return fail(nullptr, RG_E_NOTSUP, "Newton search runs on the FP32 rollouts and adjoint");
  if (o.depth < 0 || o.depth > 6) return fail(nullptr, RG_E_INVAL, "depth must be in [0, 6]");
  if (o.search == RG_SEARCH_GRID && (o.M < 2 || o.M > kCMax - 1))
    return fail(nullptr, RG_E_INVAL, "M must be in [2, 127]");
  if (o.refine < 0 || o.refine > 40) return fail(nullptr, RG_E_INVAL, "refine must be in [0, 40]");
  if (o.block != 0 && (o.block < 64 || o.block > 256 || (o.block & 63)))
    return fail(nullptr, RG_E_INVAL, "block must be a multiple of 64 in [64, 256]");
  if (o.max_T < 1 || o.max_T > 65536) return fail(nullptr, RG_E_INVAL, "max_T must be in [1, 65536]");
  if (o.lanes != 0 && o.lanes != 1 && o.lanes != 4 && o.lanes != 16)
    return fail(nullptr, RG_E_INVAL, "lanes must be 0, 1, 4 or 16");
  if (o.Kc < 1 || o.Kc > 4096) return fail(nullptr, RG_E_INVAL, "Kc must be in [1, 4096]");
  if (o.predict != 0 && o.predict != 1) return fail(nullptr, RG_E_INVAL, "predict must be 0 or 1");
  if (o.speculate < 0 || o.speculate > kSpecMax)
    return fail(nullptr, RG_E_INVAL, "speculate must be 0.." + std::to_string(kSpecMax));
  if (o.chance_q < 0) return fail(nullptr, RG_E_INVAL, "chance_q must be >= 0");
  if (o.chance_q > 0 && is_newton(o.search))
    return fail(nullptr, RG_E_NOTSUP, "the chance-constrained verdict has no Newton search");
  if (o.chance_q > 0 && o.search == RG_SEARCH_ALG2)
    return fail(nullptr, RG_E_NOTSUP, "Alg. 2 bisects each scenario on the robust verdict");

  rg_handle* h = new (std::nothrow) rg_handle;
  if (!h) return fail(nullptr, RG_E_NOMEM, "host allocation");
  h->srch_tmpl = new (std::nothrow) DevSearch;
  if (!h->srch_tmpl) {
    delete h;
    return fail(nullptr, RG_E_NOMEM, "host allocation");
  }
  memset(&h->pr, 0, sizeof(h->pr));
  PlantDesc& p = h->pr.p;
  p.kind = plant->kind; p.n = n; p.nw = nw; p.ny = ny; p.nth = nth;
  for (int i = 0; i < ncoef; ++i) p.coeffs[i] = plant->coeffs[i];
  ScenDesc& s = h->pr.s;
  s.N = scen->N; s.seed = scen->seed; s.instance = scen->instance;
  for (int c = 0; c < nw; ++c) { s.wlo[c] = scen->w_lo[c]; s.whi[c] = scen->w_hi[c]; }
  s.theta_rel = scen->theta_rel; s.inject = scen->inject; s.rng_mode = scen->rng_mode;
  ConsDesc& c = h->pr.c;
  c.n_c = cons->n_c;
  for (int r = 0; r < kNC; ++r) {
    for (int i = 0; i < ny; ++i) c.F[r * ny + i] = r < cons->n_c ? cons->F[r * ny + i] : 0.0;
    c.g[r] = r < cons->n_c ? cons->g[r] : INFINITY;
  }
  c.eps = cons->eps; c.ss_check = cons->ss_check ? 1 : 0;
  h->pr.H = H;
  h->pr.dt = dt;
  h->opt = o;
  plan(h);
  *out = h;
  return RG_OK;
}

int rg_destroy(rg_handle* h) {
  if (!h) return RG_OK;
  drop_graphs(h);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  if (h->ws_owned && h->ws) (void)hipFree(h->ws);
  delete h->srch_tmpl;
  delete h;
  return RG_OK;
}

int rg_workspace_size(const rg_handle* h, size_t* bytes) {
  if (!h || !bytes) return RG_E_INVAL;
  *bytes = layout_of(h).total;
  return RG_OK;
}

int rg_bind_workspace(rg_handle* h, void* device_ptr, size_t bytes) {
  if (!h || !device_ptr) return RG_E_INVAL;
  if (h->ws) return fail(h, RG_E_STATE, "workspace already present");
  if (((uintptr_t)device_ptr & 255) != 0) return fail(h, RG_E_INVAL, "workspace not 256-byte aligned");
  if (bytes < layout_of(h).total) return fail(h, RG_E_NOMEM, "workspace too small");
  h->ws = device_ptr;
  h->ws_bytes = bytes;
  h->ws_owned = false;
  return RG_OK;
}

int rg_set_stream(rg_handle* h, void* hip_stream) {
  if (!h) return RG_E_INVAL;
  if (h->stream != (hipStream_t)hip_stream) drop_graphs(h);
  h->stream = (hipStream_t)hip_stream;
  return RG_OK;
}

int rg_set_step(rg_handle* h, uint32_t t) {
  if (!h) return RG_E_INVAL;
  h->t = t;
  return RG_OK;
}

int rg_get_step(const rg_handle* h, uint32_t* t) {
  if (!h || !t) return RG_E_INVAL;
  *t = h->t;
  return RG_OK;
}

int rg_reset(rg_handle* h) {
  if (!h) return RG_E_INVAL;
  if (!h->ws_ready) return RG_OK;
  // prediction and speculation fields first (also used by the autotuner)
  if (int rc = reset_search_schedule(h)) return rc;
  double none[kMssCache];
  for (double& x : none) x = std::nan("");
  const int32_t next = 0;
  HIPCHK(h, hipMemcpyAsync((char*)h->b.srch + offsetof(DevSearch, mss_v), none, sizeof(none),
                           hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync((char*)h->b.srch + offsetof(DevSearch, mss_next), &next, sizeof(next),
                           hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return RG_OK;
}

int rg_step(rg_handle* h, const double* x, double r, double v_prev, double* v_out,
            double* kappa_out, rg_step_info* info) {
  if (!h) return RG_E_INVAL;
  if (!x || !v_out) return fail(h, RG_E_INVAL, "NULL x or v_out");
  if (!finite_array(x, h->pr.p.n) || !std::isfinite(r) || !std::isfinite(v_prev))
    return fail(h, RG_E_INVAL, "non-finite input");
  int rc = ensure_workspace(h);
  if (rc) return rc;
  if ((rc = upload_state(h, x, r, v_prev))) return rc;
  hipError_t e = h->opt.search == RG_SEARCH_ALG2 ? enqueue_alg2(h) : enqueue_step(h, h->pr, h->b, h->profiling);
  if (e != hipSuccess) return fail_hip(h, "enqueue RG step", e);
  h->gen_t = (long long)h->t;
  DevResult R;
  HIPCHK(h, hipMemcpyAsync(&R, h->b.res, sizeof(R), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (h->profiling) {
    HIPCHK(h, harvest_events(h));
    h->prof.lane_steps += R.lane_steps;
    h->prof.steps += 1;
  }
  h->t += 1;
  *v_out = R.v;
  if (kappa_out) *kappa_out = R.kappa;
  fill_info(R, info);
  return R.status == 0 ? RG_OK : (R.status == 2 ? RG_S_FALLBACK : RG_S_INFEASIBLE);
}

int rg_step_async(rg_handle* h, const double* x, const double* r, const double* v_prev,
                  uint32_t* t, double* v_out, double* kappa_out, int32_t* status_out) {
  if (!h) return RG_E_INVAL;
  if (!x || !r || !v_prev || !t || !v_out) return fail(h, RG_E_INVAL, "NULL device pointer");
  if (h->opt.search == RG_SEARCH_ALG2)
    return fail(h, RG_E_NOTSUP, "Alg. 2 runs single RG steps (rg_step)");
  if (h->profiling) return fail(h, RG_E_STATE, "the asynchronous step does not profile");
  if (!h->ws_ready) {
    // setting up the workspace allocates and synchronises: not under capture
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(h, hipStreamIsCapturing(h->stream, &cs));
    if (cs != hipStreamCaptureStatusNone)
      return fail(h, RG_E_STATE,
                  "workspace not set up: run one step (or bind a workspace and step once) "
                  "before capturing");
    int rc = ensure_workspace(h);
    if (rc) return rc;
  }
  hipError_t e = launch_async_in(h->b, x, r, v_prev, t, h->pr.p.n, h->stream);
  if (e == hipSuccess) e = enqueue_step(h, h->pr, h->b, false);
  if (e == hipSuccess) e = launch_async_out(h->b, v_out, kappa_out, status_out, t, h->stream);
  if (e != hipSuccess) return fail_hip(h, "enqueue asynchronous RG step", e);
  h->gen_t = -1;  // the streamed draw buffer holds the draws of a step only the device knows
  return RG_OK;
}

int rg_margin(rg_handle* h, const double* x, double r, double v_prev, const double* kappa,
              int32_t M, double* margins, float* per_scenario, int32_t* per_scenario_j) {
  if (!h) return RG_E_INVAL;
  if (!x || !kappa || !margins || M < 1) return fail(h, RG_E_INVAL, "bad arguments");
  if (!finite_array(x, h->pr.p.n) || !std::isfinite(r) || !std::isfinite(v_prev))
    return fail(h, RG_E_INVAL, "non-finite input");
  for (int i = 0; i < M; ++i)
    if (!(kappa[i] >= 0.0 && kappa[i] <= 1.0)) return fail(h, RG_E_INVAL, "kappa outside [0, 1]");
  int rc = ensure_workspace(h);
  if (rc) return rc;
  if ((rc = upload_state(h, x, r, v_prev))) return rc;
  if ((rc = ensure_draws(h))) return rc;
  const int prec = h->opt.precision;
  const double band = prec == RG_PREC_F32_RECHECK ? h->opt.band : 0.0;
  const size_t N = (size_t)h->pr.s.N;
  std::vector<double> out(kCMax);
  for (int base = 0; base < M; base += kCMax) {
    const int m = (M - base) < kCMax ? (M - base) : kCMax;
    HIPCHK(h, hipMemcpyAsync((char*)h->b.srch + offsetof(DevSearch, kappa), kappa + base, sizeof(double) * m,
                             hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, launch_setup_list(h->pr, h->b, m, h->stream));
    LaunchCfg cfg = h->cfg;
    cfg.cmax_round = m;
    HIPCHK(h, launch_rollout(h->pr, band, prec, 0, 1, cfg, h->b, h->stream));
    if (prec == RG_PREC_F32_RECHECK) HIPCHK(h, launch_recheck(h->pr, 0, cfg, h->b, h->stream));
    if (h->opt.chance_q > 0) HIPCHK(h, launch_select_q(h->b, (int)N, m, 1, h->stream));
    HIPCHK(h, launch_collect(h->b, m, h->b.scratch, h->stream));
    HIPCHK(h, hipMemcpyAsync(out.data(), h->b.scratch, sizeof(double) * m, hipMemcpyDeviceToHost,
                             h->stream));
    if (per_scenario)
      HIPCHK(h, hipMemcpyAsync(per_scenario + (size_t)base * N, h->b.per_m, sizeof(float) * m * N,
                               hipMemcpyDeviceToHost, h->stream));
    if (per_scenario_j)
      HIPCHK(h, hipMemcpyAsync(per_scenario_j + (size_t)base * N, h->b.per_j,
                               sizeof(int32_t) * m * N, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int i = 0; i < m; ++i) margins[base + i] = out[i];
  }
  return RG_OK;
}

int rg_closed_loop(rg_handle* h, const double* x0, double v0, const double* r_seq, int32_t T,
                   double* v_out, double* kappa_out, double* x_out, rg_step_info* info_out,
                   int32_t use_graph) {
  if (!h) return RG_E_INVAL;
  if (!x0 || !r_seq || !v_out || T < 1) return fail(h, RG_E_INVAL, "bad arguments");
  if (!finite_array(x0, h->pr.p.n) || !std::isfinite(v0) || !finite_array(r_seq, T))
    return fail(h, RG_E_INVAL, "non-finite input");
  if (h->opt.search == RG_SEARCH_ALG2)
    return fail(h, RG_E_NOTSUP, "Alg. 2 runs single RG steps (rg_step)");
  int rc = ensure_workspace(h);
  if (rc) return rc;
  const int n = h->pr.p.n;
  const bool graph = use_graph && !h->profiling;
  if ((rc = upload_state(h, x0, r_seq[0], v0))) return rc;
  if (x_out)
    for (int i = 0; i < n; ++i) x_out[i] = x0[i];
  // generic rounds captured as graphs: kGraphRounds rounds, and one round
  constexpr int kGraphRounds = 4;
  auto capture = [&](int len, hipGraphExec_t* out) -> int {
    hipGraph_t g = nullptr;
    HIPCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int i = 0; i < len && e == hipSuccess; ++i) e = enqueue_round(h);
    hipError_t e2 = hipStreamEndCapture(h->stream, &g);
    if (e != hipSuccess) return fail_hip(h, "capture closed-loop rounds", e);
    if (e2 != hipSuccess) return fail_hip(h, "hipStreamEndCapture", e2);
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail_hip(h, "hipGraphInstantiate", e);
    return RG_OK;
  };
  if (graph && !h->round_graph[0] && (rc = capture(kGraphRounds, &h->round_graph[0]))) return rc;
  if (graph && !h->round_graph[1] && (rc = capture(1, &h->round_graph[1]))) return rc;
  std::vector<DevResult> R;
  std::vector<double> xs;
  int32_t done = 0;
  while (done < T) {
    const int chunk = (T - done) < h->opt.max_T ? (T - done) : h->opt.max_T;
    const int32_t cl[2] = {0, chunk};  // cl_index, cl_len
    static_assert(offsetof(DevState, cl_len) == offsetof(DevState, cl_index) + sizeof(int32_t),
                  "cl_index and cl_len are adjacent");
    HIPCHK(h, hipMemcpyAsync(h->b.r_seq, r_seq + done, sizeof(double) * chunk,
                             hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync((char*)h->b.st + offsetof(DevState, cl_index), cl, sizeof(cl),
                             hipMemcpyHostToDevice, h->stream));
    // prologue of the chunk: draws of its first kSpecMax + 1 steps and round 0
    // of its first step
    if (h->pr.s.rng_mode == RG_RNG_STREAM) {
      for (uint32_t d = 0; d <= (uint32_t)kSpecMax; ++d) {
        DevBuffers bd = h->b;
        draw_pair(h, (int)((h->t + d) % (uint32_t)kPairs), &bd.wbuf, &bd.thbuf);
        HIPCHK(h, launch_gen(h->pr, bd, h->stream, d));
      }
    }
    HIPCHK(h, launch_setup(h->pr, h->b, 1, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    // Every step takes at least one round: enqueue one round per step not yet
    // recorded, then read how many are recorded, until all are.  A step needs
    // at most cfg.rounds rounds, which bounds the loop.
    int32_t recorded = 0;
    long long issued = 0;
    const long long max_rounds = (long long)chunk * (h->cfg.rounds + 1) + kGraphRounds;
    while (recorded < chunk) {
      int need = chunk - recorded;
      if (issued + need > max_rounds)
        return fail(h, RG_E_STATE, "closed loop: steps not recorded after the maximum rounds");
      issued += need;
      while (need > 0) {
        hipError_t e = hipSuccess;
        if (graph) {
          const bool big = need >= kGraphRounds;
          e = hipGraphLaunch(h->round_graph[big ? 0 : 1], h->stream);
          need -= big ? kGraphRounds : 1;
        } else {
          e = enqueue_round(h);
          need -= 1;
        }
        if (e != hipSuccess) return fail_hip(h, "enqueue closed-loop round", e);
      }
      HIPCHK(h, hipMemcpyAsync(&recorded, (char*)h->b.st + offsetof(DevState, cl_index),
                               sizeof(recorded), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    R.resize(chunk);
    xs.resize((size_t)(chunk + 1) * n);
    HIPCHK(h, hipMemcpyAsync(R.data(), h->b.res, sizeof(DevResult) * chunk, hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipMemcpyAsync(xs.data(), h->b.x_hist, sizeof(double) * (chunk + 1) * n,
                             hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (h->profiling) HIPCHK(h, harvest_events(h));
    for (int s = 0; s < chunk; ++s) {
      v_out[done + s] = R[s].v;
      if (kappa_out) kappa_out[done + s] = R[s].kappa;
      if (info_out) fill_info(R[s], info_out + done + s);
      if (x_out)
        for (int i = 0; i < n; ++i) x_out[(size_t)(done + s + 1) * n + i] = xs[(size_t)(s + 1) * n + i];
      if (h->profiling) {
        h->prof.lane_steps += R[s].lane_steps;
        h->prof.steps += 1;
      }
    }
    done += chunk;
    h->t += (uint32_t)chunk;
  }
  h->gen_t = -1;  // the single-step draw pair no longer holds a known step
  return RG_OK;
}

int rg_grad(rg_handle* h, const double* x, double r, double v_prev, double kappa,
            const float* upstream, double* margin_out, double* dkappa_out, double* dtheta_out) {
  if (!h) return RG_E_INVAL;
  if (!x || !dkappa_out) return fail(h, RG_E_INVAL, "NULL x or dkappa_out");
  if (!finite_array(x, h->pr.p.n) || !std::isfinite(r) || !std::isfinite(v_prev))
    return fail(h, RG_E_INVAL, "non-finite input");
  if (!(kappa >= 0.0 && kappa <= 1.0)) return fail(h, RG_E_INVAL, "kappa outside [0, 1]");
  if (h->opt.chance_q > 0)
    return fail(h, RG_E_NOTSUP, "rg_grad differentiates the robust worst margin (chance_q = 0)");
  const int N = h->pr.s.N;
  std::vector<int32_t> ks;
  std::vector<float> ws;
  if (upstream) {
    for (int k = 0; k < N; ++k) {
      if (!std::isfinite(upstream[k])) return fail(h, RG_E_INVAL, "non-finite upstream gradient");
      if (upstream[k] != 0.f) {
        ks.push_back(k);
        ws.push_back(upstream[k]);
      }
    }
  }
  int rc = ensure_workspace(h);
  if (rc) return rc;
  if ((rc = upload_state(h, x, r, v_prev))) return rc;
  if ((rc = ensure_draws(h))) return rc;
  LaunchCfg cfg = h->cfg;
  cfg.cmax_round = 1;
  cfg.tan = 0;  // reverse mode: the rollout keeps checkpoints
  HIPCHK(h, hipMemcpyAsync((char*)h->b.srch + offsetof(DevSearch, kappa), &kappa, sizeof(double),
                           hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, launch_setup_list(h->pr, h->b, 1, h->stream));
  // arg-min scenario from the FP32 rollouts (keys carry the scenario index)
  HIPCHK(h, launch_rollout(h->pr, h->opt.band, RG_PREC_F32_RECHECK, 0, 1, cfg, h->b, h->stream,
                           upstream ? -2 : 0, h->opt.Kc));
  HIPCHK(h, launch_recheck(h->pr, 0, cfg, h->b, h->stream));
  int max_entries = 1;
  if (upstream) {
    const int32_t cnt = (int32_t)ks.size();
    max_entries = cnt > 0 ? cnt : 1;
    if (cnt > 0) {
      HIPCHK(h, hipMemcpyAsync(h->b.adj_k, ks.data(), sizeof(int32_t) * cnt, hipMemcpyHostToDevice,
                               h->stream));
      HIPCHK(h, hipMemcpyAsync(h->b.adj_w, ws.data(), sizeof(float) * cnt, hipMemcpyHostToDevice,
                               h->stream));
    }
    HIPCHK(h, hipMemcpyAsync((char*)h->b.grad + offsetof(DevGrad, n_entries), &cnt, sizeof(cnt),
                             hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, launch_grad_prepare(h->pr, h->b, 0, 0, h->stream));
  } else {
    HIPCHK(h, launch_grad_prepare(h->pr, h->b, 0, 1, h->stream));
  }
  if (upstream)  // weighted scenarios: one sequential reverse sweep per scenario
    HIPCHK(h, launch_adjoint(h->pr, h->opt.Kc, max_entries, h->b, 0, h->stream));
  else  // the arg-min scenario: segment-parallel reverse sweep
    HIPCHK(h, launch_seg_grad(h->pr, h->opt.Kc, 0, h->b, h->stream));
  HIPCHK(h, launch_grad_reduce(h->b, max_entries, h->pr.p.nth, 0, h->stream));
  DevGrad G;
  HIPCHK(h, hipMemcpyAsync(&G, h->b.grad, sizeof(G), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (margin_out) *margin_out = G.M;
  *dkappa_out = G.dM_dkappa;
  if (dtheta_out)
    for (int c = 0; c < h->pr.p.nth; ++c) dtheta_out[c] = G.dM_dth[c];
  return RG_OK;
}

int rg_tangent(rg_handle* h, const double* x, double r, double v_prev, double kappa,
               float* m_out, float* dm_dv_out, int32_t* j_out, double* margin_out,
               double* dkappa_out) {
  if (!h) return RG_E_INVAL;
  if (!x || !dkappa_out) return fail(h, RG_E_INVAL, "NULL x or dkappa_out");
  if (!finite_array(x, h->pr.p.n) || !std::isfinite(r) || !std::isfinite(v_prev))
    return fail(h, RG_E_INVAL, "non-finite input");
  if (!(kappa >= 0.0 && kappa <= 1.0)) return fail(h, RG_E_INVAL, "kappa outside [0, 1]");
  if (h->opt.chance_q > 0)
    return fail(h, RG_E_NOTSUP, "rg_tangent differentiates the robust worst margin (chance_q = 0)");
  if (h->opt.precision != RG_PREC_F32_RECHECK)
    return fail(h, RG_E_NOTSUP, "the tangent rollout runs in FP32 (precision F32_RECHECK)");
  const int N = h->pr.s.N;
  int rc = ensure_workspace(h);
  if (rc) return rc;
  if ((rc = upload_state(h, x, r, v_prev))) return rc;
  if ((rc = ensure_draws(h))) return rc;
  LaunchCfg cfg = h->cfg;
  cfg.cmax_round = 1;
  cfg.tan = 1;
  HIPCHK(h, hipMemcpyAsync((char*)h->b.srch + offsetof(DevSearch, kappa), &kappa, sizeof(double),
                           hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, launch_setup_list(h->pr, h->b, 1, h->stream));
  // candidate 0 carries the tangent over the full horizon; near-band lanes are
  // re-simulated in FP64 for the margin value
  HIPCHK(h, launch_rollout(h->pr, h->opt.band, RG_PREC_F32_RECHECK, 0, 0, cfg, h->b, h->stream, 0,
                           h->opt.Kc));
  HIPCHK(h, launch_recheck(h->pr, 0, cfg, h->b, h->stream));
  HIPCHK(h, launch_tan_grad(h->pr, h->b, 0, h->stream));
  DevGrad G;
  HIPCHK(h, hipMemcpyAsync(&G, h->b.grad, sizeof(G), hipMemcpyDeviceToHost, h->stream));
  if (m_out)
    HIPCHK(h, hipMemcpyAsync(m_out, h->b.per_m, sizeof(float) * N, hipMemcpyDeviceToHost, h->stream));
  if (dm_dv_out)
    HIPCHK(h, hipMemcpyAsync(dm_dv_out, h->b.tan_dv, sizeof(float) * N, hipMemcpyDeviceToHost,
                             h->stream));
  if (j_out)
    HIPCHK(h, hipMemcpyAsync(j_out, h->b.per_j, sizeof(int32_t) * N, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (margin_out) *margin_out = G.M;
  *dkappa_out = G.dM_dkappa;
  return RG_OK;
}

int rg_set_theta(rg_handle* h, const double* theta_nom) {
  if (!h) return RG_E_INVAL;
  if (h->pr.p.nth == 0) return fail(h, RG_E_NOTSUP, "this plant has no uncertain coefficients");
  if (!theta_nom || !finite_array(theta_nom, h->pr.p.nth)) return fail(h, RG_E_INVAL, "bad theta");
  for (int c = 0; c < h->pr.p.nth; ++c) h->pr.p.coeffs[90 + c] = theta_nom[c];
  drop_graphs(h);  // kernel arguments changed
  if (h->ws_ready) {  // cached steady-state margins belong to the old coefficients
    double none[kMssCache];
    for (double& x : none) x = std::nan("");
    HIPCHK(h, hipMemcpyAsync((char*)h->b.srch + offsetof(DevSearch, mss_v), none, sizeof(none),
                             hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
  }
  return RG_OK;
}

int rg_equilibrium(rg_handle* h, double v, double* x_out) {
  if (!h) return RG_E_INVAL;
  if (!x_out || !std::isfinite(v)) return fail(h, RG_E_INVAL, "bad arguments");
  int rc = ensure_workspace(h);
  if (rc) return rc;
  double out[kMaxN + 1];
  HIPCHK(h, launch_equilibrium(h->pr, h->b, v, h->b.scratch, h->stream));
  HIPCHK(h, hipMemcpyAsync(out, h->b.scratch, sizeof(double) * (h->pr.p.n + 1),
                           hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (out[h->pr.p.n] != 1.0) return fail(h, RG_E_STATE, "equilibrium iteration did not converge");
  for (int i = 0; i < h->pr.p.n; ++i) x_out[i] = out[i];
  return RG_OK;
}

}  // extern "C"

namespace {

// Switch the launch schedule (lanes, block, depth, prediction) of a handle:
// re-plan, drop the captured step graph, update the device search record.
// Reset the device search record's schedule fields and prediction state.
int reset_search_schedule(rg_handle* h) {
  if (h->ws_ready) {
    // spec_depth, spec_hold, spec_kind, spec_base, spec_per, spec_n, spec_used
    const int32_t spec[7] = {spec_allowed(h), hold_allowed(h), 0, 0, 0, 0, 0};
    static_assert(offsetof(DevSearch, spec_used) == offsetof(DevSearch, spec_depth) + 24,
                  "the speculation fields are adjacent");
    HIPCHK(h, hipMemcpyAsync((char*)h->b.srch + offsetof(DevSearch, spec_depth), spec, sizeof(spec),
                             hipMemcpyHostToDevice, h->stream));
    const int32_t depth = h->opt.depth;
    const int32_t predict =
        h->opt.search == RG_SEARCH_BISECT || is_newton(h->opt.search) ? h->opt.predict : 0;
    const double none = std::nan("");
    HIPCHK(h, hipMemcpyAsync((char*)h->b.srch + offsetof(DevSearch, depth), &depth, sizeof(depth),
                             hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync((char*)h->b.srch + offsetof(DevSearch, predict), &predict,
                             sizeof(predict), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync((char*)h->b.srch + offsetof(DevSearch, pred), &none, sizeof(none),
                             hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
  }
  return RG_OK;
}

int apply_schedule(rg_handle* h, const rg_options& o) {
  h->opt.lanes = o.lanes;
  h->opt.block = o.block;
  h->opt.depth = o.depth;
  h->opt.predict = o.predict;
  h->opt.speculate = o.speculate;
  plan(h);
  drop_graphs(h);
  return reset_search_schedule(h);
}

}  // namespace

extern "C" {

int rg_autotune(rg_handle* h, const double* x0, double v0, const double* r_seq, int32_t T,
                int32_t apply, rg_options* best_out, double* best_ms_out) {
  if (!h) return RG_E_INVAL;
  if (!x0 || !r_seq || T < 1) return fail(h, RG_E_INVAL, "bad arguments");
  if (h->profiling) return fail(h, RG_E_STATE, "autotune with profiling enabled");
  if (h->opt.search == RG_SEARCH_ALG2)
    return fail(h, RG_E_NOTSUP, "Alg. 2 has no launch schedule to tune");
  int rc = ensure_workspace(h);
  if (rc) return rc;
  const rg_options own = h->opt;
  const uint32_t t0 = h->t;
  const bool f32_robust = h->opt.precision == RG_PREC_F32_RECHECK && h->opt.chance_q == 0;
  const bool quad_ok = h->pr.p.kind == RG_PLANT_LQ4 && f32_robust;
  const bool group_ok =
      h->pr.p.kind == RG_PLANT_FC9 && f32_robust && h->opt.search != RG_SEARCH_NEWTON_TAN;
  std::vector<rg_options> cands;
  for (int lanes : {4, 16, 1}) {
    if (lanes == 4 && !quad_ok) continue;
    if (lanes == 16 && !group_ok) continue;
    for (int block : {256, 128}) {
      const bool grid = h->opt.search == RG_SEARCH_GRID;
      const int dlo = grid ? 1 : 2, dhi = grid ? 3 : 5;
      for (int depth = dlo; depth <= dhi; ++depth) {
        for (int predict : {1, 0}) {
          if (predict && h->opt.search != RG_SEARCH_BISECT && !is_newton(h->opt.search)) continue;
          if (is_newton(h->opt.search) && depth != dlo) continue;  // depth unused
          for (int speculate : {kSpecMax, 3, 1, 0}) {
            if (speculate && !(predict && lanes == 4)) continue;
            rg_options o = own;
            o.lanes = lanes;
            o.block = block;
            o.depth = depth;
            o.predict = predict;
            o.speculate = speculate;
            cands.push_back(o);
          }
        }
      }
    }
  }
  std::vector<double> v(T), kap(T), ref;
  double best_ms = INFINITY;
  rg_options best = own;
  for (const rg_options& o : cands) {
    if ((rc = apply_schedule(h, o))) break;
    // the first run captures the graphs; the faster of the next two counts
    double ms = INFINITY;
    for (int rep = 0; rep < 3 && rc == RG_OK; ++rep) {
      if ((rc = reset_search_schedule(h))) break;  // fresh prediction state for each run
      h->t = t0;
      const auto c0 = std::chrono::steady_clock::now();
      rc = rg_closed_loop(h, x0, v0, r_seq, T, v.data(), kap.data(), nullptr, nullptr, 1);
      const auto c1 = std::chrono::steady_clock::now();
      if (rep > 0) ms = std::min(ms, std::chrono::duration<double, std::milli>(c1 - c0).count() / T);
    }
    if (rc) break;
    if (ref.empty()) {
      ref = kap;
    } else if (ref != kap) {
      rc = fail(h, RG_E_STATE, "schedules disagree on kappa (lanes " + std::to_string(o.lanes) +
                                   ", block " + std::to_string(o.block) + ", depth " +
                                   std::to_string(o.depth) + ")");
      break;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = h->opt;  // as planned (depth and lanes resolved)
    }
  }
  h->t = t0;
  h->gen_t = -1;  // the streamed draws no longer match the step counter
  const int rc2 = apply_schedule(h, (rc == RG_OK && apply) ? best : own);
  if (rc) return rc;
  if (rc2) return rc2;
  if (best_out) *best_out = best;
  if (best_ms_out) *best_ms_out = best_ms;
  return RG_OK;
}

int rg_get_options(const rg_handle* h, rg_options* out) {
  if (!h || !out) return RG_E_INVAL;
  *out = h->opt;
  return RG_OK;
}

int rg_set_profiling(rg_handle* h, int32_t enable) {
  if (!h) return RG_E_INVAL;
  h->profiling = enable != 0;
  h->prof = rg_profile{};
  h->ev_used = 0;
  return RG_OK;
}

int rg_get_profile(const rg_handle* h, rg_profile* out) {
  if (!h || !out) return RG_E_INVAL;
  *out = h->prof;
  return RG_OK;
}

int rg_draws(rg_handle* h, uint32_t t, int32_t k0, int32_t nk, int32_t j0, int32_t nj,
             float* w_out, double* theta_out) {
  if (!h) return RG_E_INVAL;
  if (!w_out || k0 < 0 || nk < 1 || j0 < 0 || nj < 1) return fail(h, RG_E_INVAL, "bad arguments");
  int rc = ensure_workspace(h);
  if (rc) return rc;
  const size_t wb = sizeof(float) * (size_t)nk * nj * h->pr.p.nw;
  const size_t tb = sizeof(double) * (size_t)nk * (h->pr.p.nth > 0 ? h->pr.p.nth : 1);
  float* wd = nullptr;
  double* td = nullptr;
  HIPCHK(h, hipMalloc(&wd, wb));
  hipError_t e = hipMalloc(&td, tb);
  if (e != hipSuccess) {
    (void)hipFree(wd);
    return fail_hip(h, "hipMalloc", e);
  }
  e = launch_draws(h->pr, t, k0, nk, j0, nj, wd, theta_out ? td : nullptr, h->b, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(w_out, wd, wb, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess && theta_out && h->pr.p.nth > 0)
    e = hipMemcpyAsync(theta_out, td, sizeof(double) * (size_t)nk * h->pr.p.nth,
                       hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(wd);
  (void)hipFree(td);
  if (e != hipSuccess) return fail_hip(h, "rg_draws", e);
  return RG_OK;
}

int rg_trajectory(rg_handle* h, const double* x, double v, const int32_t* k_list, int32_t nk,
                  int32_t precision, double* traj) {
  if (!h) return RG_E_INVAL;
  if (!x || !k_list || !traj || nk < 1) return fail(h, RG_E_INVAL, "bad arguments");
  if (precision != RG_PREC_F32_RECHECK && precision != RG_PREC_F64)
    return fail(h, RG_E_INVAL, "bad precision");
  if (!finite_array(x, h->pr.p.n) || !std::isfinite(v)) return fail(h, RG_E_INVAL, "non-finite input");
  for (int i = 0; i < nk; ++i)
    if (k_list[i] < 0 || k_list[i] >= h->pr.s.N) return fail(h, RG_E_INVAL, "scenario out of range");
  int rc = ensure_workspace(h);
  if (rc) return rc;
  if ((rc = upload_state(h, x, v, v))) return rc;
  if ((rc = ensure_draws(h))) return rc;
  const size_t tb = sizeof(double) * (size_t)nk * (h->pr.H + 1) * h->pr.p.n;
  double* td = nullptr;
  int32_t* kd = nullptr;
  HIPCHK(h, hipMalloc(&td, tb));
  hipError_t e = hipMalloc(&kd, sizeof(int32_t) * nk);
  if (e != hipSuccess) {
    (void)hipFree(td);
    return fail_hip(h, "hipMalloc", e);
  }
  e = hipMemcpyAsync(kd, k_list, sizeof(int32_t) * nk, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = launch_trajectory(h->pr, v, kd, nk, precision, td, h->b, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(traj, td, tb, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(td);
  (void)hipFree(kd);
  if (e != hipSuccess) return fail_hip(h, "rg_trajectory", e);
  return RG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched serving
// ---------------------------------------------------------------------------
// Many independent governors stepped together.  Each instance keeps its own
// search record, result record and recheck list, carved from one device
// allocation, and its draws are regenerated inside the kernels (a batch of a
// thousand instances could not hold draw buffers).  One search round of the
// whole batch is one flat rollout launch per group of instances with the same
// plant kind and disturbance injection (every instance's scenario tiles side by
// side in one grid, each workgroup reading its instance's argument block from
// device memory), then one flat launch per group for the FP64 recheck and the
// round's decision (one workgroup per instance).  A batched step starts with
// the instances' round-0 setup and ends with their result records (one launch
// per group each); it is captured once as a HIP graph and replayed.
struct BatchGroup {
  int kind = 0, inject = 0, tiles = 0, cmax = 0;
  std::vector<int> members;     // batch indices of the group's instances
  void* args = nullptr;         // device: the members' FP32 rollout argument blocks
  void* args64 = nullptr;       // device: their FP64 recheck argument blocks
  void* ctl = nullptr;          // device: their control blocks (setup, decision)
  DevResult** resptr = nullptr; // device [members]: their result records
  int32_t* tile_inst = nullptr; // device [tiles]: member of each workgroup column
  int32_t* tile_first = nullptr;// device [members]: first tile of each member
};

struct rg_batch {
  int count = 0;
  rg_options opt{};
  std::vector<rg_handle*> inst;  // per instance: problem, plan and carved buffers
  std::vector<int> noff;         // offset of each instance's state in the packed x array
  std::vector<uint32_t> t;       // per-instance RG step counters
  std::vector<BatchGroup> groups;
  int tile = 256;                // scenarios per rollout workgroup
  int rounds = 0;                // device rounds per batched step (the largest plan)
  hipStream_t stream = nullptr;  // the caller's stream (NULL: own_stream)
  hipStream_t own_stream = nullptr;
  void* mem = nullptr;
  DevState* st = nullptr;   // [count]
  DevResult* res = nullptr; // [count]
  hipGraphExec_t graph = nullptr;
  std::string err;
};

namespace {

int bfail(rg_batch* bt, int code, const std::string& msg) {
  if (bt) bt->err = msg;
  else g_create_error = msg;
  return code;
}

void batch_release(rg_batch* bt) {
  if (bt->graph) (void)hipGraphExecDestroy(bt->graph);
  bt->graph = nullptr;
  if (bt->own_stream) (void)hipStreamDestroy(bt->own_stream);
  bt->own_stream = nullptr;
  if (bt->mem) (void)hipFree(bt->mem);
  bt->mem = nullptr;
  for (rg_handle* h : bt->inst) rg_destroy(h);  // no workspace of their own
  bt->inst.clear();
}

// Device memory, argument blocks and tile tables, on the first step.
int batch_ensure_memory(rg_batch* bt) {
  if (bt->mem) return RG_OK;
  const int count = bt->count;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t o_st = take(sizeof(DevState) * count);
  const size_t o_srch = take(sizeof(DevSearch) * count);
  const size_t o_res = take(sizeof(DevResult) * count);
  std::vector<size_t> o_rl(count);
  for (int i = 0; i < count; ++i) {
    const rg_handle* h = bt->inst[i];
    o_rl[i] = take(sizeof(int2) * (size_t)h->cfg.cmax_round * (size_t)h->pr.s.N);
  }
  const size_t ng = bt->groups.size();
  std::vector<size_t> o_args(ng), o_a64(ng), o_ctl(ng), o_rp(ng), o_ti(ng), o_tf(ng);
  for (size_t g = 0; g < ng; ++g) {
    const BatchGroup& G = bt->groups[g];
    const size_t nm = G.members.size();
    o_args[g] = take(flat_args_size(G.kind) * nm);
    o_a64[g] = take(flat_args64_size(G.kind) * nm);
    o_ctl[g] = take(flat_ctl_size(G.kind) * nm);
    o_rp[g] = take(sizeof(DevResult*) * nm);
    o_ti[g] = take(sizeof(int32_t) * (size_t)G.tiles);
    o_tf[g] = take(sizeof(int32_t) * nm);
  }
  hipError_t e = hipMalloc(&bt->mem, off);
  if (e != hipSuccess) {
    bt->mem = nullptr;
    return bfail(bt, RG_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  if (!bt->own_stream) e = hipStreamCreateWithFlags(&bt->own_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return bfail(bt, RG_E_HIP, std::string("batch stream: ") + hipGetErrorString(e));
  char* base = (char*)bt->mem;
  bt->st = (DevState*)(base + o_st);
  bt->res = (DevResult*)(base + o_res);
  DevSearch* srch = (DevSearch*)(base + o_srch);
  std::vector<DevSearch> tmpl(count);
  for (int i = 0; i < count; ++i) {
    rg_handle* h = bt->inst[i];
    DevBuffers b{};
    b.st = bt->st + i;
    b.srch = srch + i;
    b.res = bt->res + i;
    b.rlist = (int2*)(base + o_rl[i]);
    h->b = b;
    h->ws = bt->mem;  // carved from the batch's allocation: never freed by the handle
    h->ws_owned = false;
    h->ws_ready = true;
    fill_search(h, &tmpl[i], 0, 0);
  }
  const hipStream_t ms = bt->stream ? bt->stream : bt->own_stream;
  e = hipMemcpyAsync(srch, tmpl.data(), sizeof(DevSearch) * count, hipMemcpyHostToDevice, ms);
  // argument blocks and tables of each group (host staging kept until the copies end)
  std::vector<std::vector<char>> st_a(ng), st_a64(ng), st_c(ng);
  std::vector<std::vector<DevResult*>> st_rp(ng);
  std::vector<std::vector<int32_t>> st_ti(ng), st_tf(ng);
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ms);
  };
  for (size_t g = 0; g < ng; ++g) {
    BatchGroup& G = bt->groups[g];
    const size_t nm = G.members.size();
    const size_t asz = flat_args_size(G.kind), a64 = flat_args64_size(G.kind),
                 csz = flat_ctl_size(G.kind);
    st_a[g].assign(asz * nm, 0);
    st_a64[g].assign(a64 * nm, 0);
    st_c[g].assign(csz * nm, 0);
    st_rp[g].resize(nm);
    st_tf[g].resize(nm);
    st_ti[g].reserve(G.tiles);
    for (size_t m = 0; m < nm; ++m) {
      const rg_handle* h = bt->inst[G.members[m]];
      flat_fill_args(h->pr, bt->opt.band, bt->opt.early_exit, h->b, st_a[g].data() + m * asz);
      flat_fill_args64(h->pr, bt->opt.early_exit, h->b, st_a64[g].data() + m * a64);
      flat_fill_ctl(h->pr, h->b, st_c[g].data() + m * csz);
      st_rp[g][m] = h->b.res;
      st_tf[g][m] = (int32_t)st_ti[g].size();
      const int nt = (h->pr.s.N + bt->tile - 1) / bt->tile;
      for (int q = 0; q < nt; ++q) st_ti[g].push_back((int32_t)m);
    }
    G.args = base + o_args[g];
    G.args64 = base + o_a64[g];
    G.ctl = base + o_ctl[g];
    G.resptr = (DevResult**)(base + o_rp[g]);
    G.tile_inst = (int32_t*)(base + o_ti[g]);
    G.tile_first = (int32_t*)(base + o_tf[g]);
    up(G.args, st_a[g].data(), st_a[g].size());
    up(G.args64, st_a64[g].data(), st_a64[g].size());
    up(G.ctl, st_c[g].data(), st_c[g].size());
    up(G.resptr, st_rp[g].data(), sizeof(DevResult*) * nm);
    up(G.tile_inst, st_ti[g].data(), sizeof(int32_t) * st_ti[g].size());
    up(G.tile_first, st_tf[g].data(), sizeof(int32_t) * nm);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ms);
  if (e != hipSuccess) return bfail(bt, RG_E_HIP, std::string("batch upload: ") + hipGetErrorString(e));
  return RG_OK;
}

// One batched step on stream ms.
hipError_t batch_enqueue(rg_batch* bt, hipStream_t ms) {
  hipError_t e = hipSuccess;
  for (const BatchGroup& G : bt->groups)
    if (e == hipSuccess) e = launch_flat_setup(G.kind, G.ctl, (int)G.members.size(), ms);
  for (int r = 0; r < bt->rounds && e == hipSuccess; ++r) {
    for (const BatchGroup& G : bt->groups)
      if (e == hipSuccess)
        e = launch_flat_rollout(G.kind, G.inject, G.args, G.tile_inst, G.tile_first, G.tiles,
                                G.cmax, bt->tile, ms);
    for (const BatchGroup& G : bt->groups)
      if (e == hipSuccess)
        e = launch_flat_recheck(G.kind, G.inject, G.args64, G.ctl, (int)G.members.size(), ms);
  }
  for (const BatchGroup& G : bt->groups)
    if (e == hipSuccess)
      e = launch_flat_finalize(G.kind, G.ctl, G.resptr, (int)G.members.size(), ms);
  return e;
}

}  // namespace

extern "C" {

int rg_batch_create(const rg_instance_desc* descs, int32_t count, const rg_options* opt,
                    rg_batch** out) {
  if (!out) return bfail(nullptr, RG_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!descs || count < 1) return bfail(nullptr, RG_E_INVAL, "no instances");
  rg_options o;
  rg_default_options(&o);
  // A batch's rounds are throughput-bound: one candidate per instance and round
  // does the least work (measured: first-round prediction or deeper trees only
  // add candidates), so the defaults differ from a single handle's.
  o.predict = 0;
  o.block = 64;
  if (opt) o = *opt;
  if (o.precision != RG_PREC_F32_RECHECK)
    return bfail(nullptr, RG_E_NOTSUP, "batches run FP32 rollouts with the FP64 recheck");
  if (o.search != RG_SEARCH_BISECT && o.search != RG_SEARCH_GRID)
    return bfail(nullptr, RG_E_NOTSUP, "batches use bisection or the grid search");
  if (o.chance_q != 0) return bfail(nullptr, RG_E_NOTSUP, "batches use the robust verdict");
  if (o.block != 0 && o.block != 64 && o.block != 128 && o.block != 256)
    return bfail(nullptr, RG_E_INVAL, "block must be 64, 128 or 256");
  if (o.persistent_wgs < 0) return bfail(nullptr, RG_E_INVAL, "persistent_wgs must be >= 0");
  // search plan shared by the instances: a round already holds sum_i N_i lanes
  // per candidate, so speculative levels only while that is below the chip's
  // capacity (about two waves per SIMD)
  double lanes = 0.0;
  for (int i = 0; i < count; ++i) lanes += descs[i].scen.N > 0 ? descs[i].scen.N : 0;
  int d = o.depth;
  const int goal = o.search == RG_SEARCH_GRID ? o.refine : o.K;
  if (d == 0) {
    const double budget = 2.0 * 256 * 4 * 64;
    int dmax = 1;
    while (dmax < 6 && ((1 << (dmax + 1)) - 1) * lanes <= budget) ++dmax;
    const int rounds = goal > 0 ? (goal + dmax - 1) / dmax : 1;
    d = goal > 0 ? (goal + rounds - 1) / rounds : 1;
  }
  rg_batch* bt = new (std::nothrow) rg_batch;
  if (!bt) return bfail(nullptr, RG_E_NOMEM, "host allocation");
  bt->count = count;
  bt->opt = o;
  bt->opt.depth = d;
  bt->tile = o.block ? o.block : 64;
  int noff = 0;
  for (int i = 0; i < count; ++i) {
    rg_scenarios s = descs[i].scen;
    s.rng_mode = RG_RNG_INLINE;
    rg_options oi = o;
    oi.depth = d;
    oi.lanes = 1;       // the flat rollout runs one lane per scenario
    oi.speculate = 0;
    oi.max_T = 1;
    oi.block = bt->tile;
    rg_handle* h = nullptr;
    const int rc = rg_create(&descs[i].plant, &s, &descs[i].cons, descs[i].H, descs[i].dt, &oi, &h);
    if (rc != RG_OK) {
      std::string m = std::string("instance ") + std::to_string(i) + ": " + g_create_error;
      batch_release(bt);
      delete bt;
      return bfail(nullptr, rc, m);
    }
    bt->inst.push_back(h);
    bt->noff.push_back(noff);
    noff += h->pr.p.n;
    if (h->cfg.rounds > bt->rounds) bt->rounds = h->cfg.rounds;
    // group by plant kind and injection
    BatchGroup* G = nullptr;
    for (BatchGroup& g : bt->groups)
      if (g.kind == h->pr.p.kind && g.inject == h->pr.s.inject) G = &g;
    if (!G) {
      bt->groups.emplace_back();
      G = &bt->groups.back();
      G->kind = h->pr.p.kind;
      G->inject = h->pr.s.inject;
    }
    G->members.push_back(i);
    G->tiles += (h->pr.s.N + bt->tile - 1) / bt->tile;
    if (h->cfg.cmax_round > G->cmax) G->cmax = h->cfg.cmax_round;
  }
  bt->t.assign(count, 0u);
  *out = bt;
  return RG_OK;
}

int rg_fp64_tanh(const double* x, double* y, int32_t n) {
  if (!x || !y || n < 1) return fail(nullptr, RG_E_INVAL, "bad arguments");
  double* d = nullptr;
  hipError_t e = hipMalloc(&d, sizeof(double) * 2 * (size_t)n);
  if (e != hipSuccess) return fail(nullptr, RG_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  e = hipMemcpy(d, x, sizeof(double) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_eval_tanh64(d, d + n, n, nullptr);
  if (e == hipSuccess) e = hipMemcpy(y, d + n, sizeof(double) * n, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(nullptr, RG_E_HIP, std::string("rg_fp64_tanh: ") + hipGetErrorString(e));
  return RG_OK;
}

int rg_batch_destroy(rg_batch* bt) {
  if (!bt) return RG_OK;
  batch_release(bt);
  delete bt;
  return RG_OK;
}

int rg_batch_set_stream(rg_batch* bt, void* hip_stream) {
  if (!bt) return RG_E_INVAL;
  if (bt->stream != (hipStream_t)hip_stream && bt->graph) {
    (void)hipGraphExecDestroy(bt->graph);
    bt->graph = nullptr;
  }
  bt->stream = (hipStream_t)hip_stream;
  return RG_OK;
}

int rg_batch_set_step(rg_batch* bt, int32_t i, uint32_t t) {
  if (!bt || i < 0 || i >= bt->count) return RG_E_INVAL;
  bt->t[i] = t;
  return RG_OK;
}

int rg_batch_step(rg_batch* bt, const double* x, const double* r, const double* v_prev,
                  double* v_out, double* kappa_out, rg_step_info* info_out, int32_t use_graph) {
  if (!bt) return RG_E_INVAL;
  if (!x || !r || !v_prev || !v_out) return bfail(bt, RG_E_INVAL, "NULL argument");
  const int count = bt->count;
  for (int i = 0; i < count; ++i) {
    if (!finite_array(x + bt->noff[i], bt->inst[i]->pr.p.n) || !std::isfinite(r[i]) ||
        !std::isfinite(v_prev[i]))
      return bfail(bt, RG_E_INVAL, "non-finite input");
  }
  int rc = batch_ensure_memory(bt);
  if (rc) return rc;
  const hipStream_t ms = bt->stream ? bt->stream : bt->own_stream;
  std::vector<DevState> st(count);
  for (int i = 0; i < count; ++i) {
    memset(&st[i], 0, sizeof(DevState));
    for (int q = 0; q < bt->inst[i]->pr.p.n; ++q) st[i].x[q] = x[bt->noff[i] + q];
    st[i].v_prev = v_prev[i];
    st[i].r = r[i];
    st[i].t = bt->t[i];
  }
  hipError_t e = hipMemcpyAsync(bt->st, st.data(), sizeof(DevState) * count,
                                hipMemcpyHostToDevice, ms);
  if (e != hipSuccess) return bfail(bt, RG_E_HIP, std::string("upload: ") + hipGetErrorString(e));
  if (use_graph) {
    if (!bt->graph) {
      hipGraph_t g = nullptr;
      e = hipStreamBeginCapture(ms, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return bfail(bt, RG_E_HIP, std::string("capture: ") + hipGetErrorString(e));
      hipError_t e1 = batch_enqueue(bt, ms);
      hipError_t e2 = hipStreamEndCapture(ms, &g);
      if (e1 != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bfail(bt, RG_E_HIP, std::string("capture batch step: ") +
                                       hipGetErrorString(e1 != hipSuccess ? e1 : e2));
      }
      e = hipGraphInstantiate(&bt->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        bt->graph = nullptr;
        return bfail(bt, RG_E_HIP, std::string("instantiate: ") + hipGetErrorString(e));
      }
    }
    e = hipGraphLaunch(bt->graph, ms);
  } else {
    e = batch_enqueue(bt, ms);
  }
  if (e != hipSuccess) return bfail(bt, RG_E_HIP, std::string("batch step: ") + hipGetErrorString(e));
  std::vector<DevResult> R(count);
  e = hipMemcpyAsync(R.data(), bt->res, sizeof(DevResult) * count, hipMemcpyDeviceToHost, ms);
  if (e == hipSuccess) e = hipStreamSynchronize(ms);
  if (e != hipSuccess) return bfail(bt, RG_E_HIP, std::string("batch results: ") + hipGetErrorString(e));
  for (int i = 0; i < count; ++i) {
    v_out[i] = R[i].v;
    if (kappa_out) kappa_out[i] = R[i].kappa;
    if (info_out) fill_info(R[i], info_out + i);
    bt->t[i] += 1;
  }
  return RG_OK;
}

int rg_batch_autotune(const rg_instance_desc* descs, int32_t count, const rg_options* opt,
                      const double* x, const double* r, const double* v_prev,
                      rg_options* best_out, double* best_ms_out) {
  if (!descs || count < 1 || !x || !r || !v_prev)
    return bfail(nullptr, RG_E_INVAL, "bad arguments");
  rg_options base;
  rg_default_options(&base);
  base.predict = 0;
  base.block = 64;
  if (opt) base = *opt;
  std::vector<double> v(count), kap(count);
  std::vector<std::vector<double>> kref;  // kappa of steps 0..2 under the first schedule
  double best_ms = INFINITY;
  rg_options best = base;
  constexpr int kRuns = 3;  // steps t = 0, 1, 2: the first captures the graph
  for (int block : {64, 128, 256}) {
    for (int depth : {1, 2, 3}) {
      for (int predict : {0, 1}) {
        rg_options o = base;
        o.block = block;
        o.depth = depth;
        o.predict = predict;
        rg_batch* bt = nullptr;
        int rc = rg_batch_create(descs, count, &o, &bt);
        if (rc != RG_OK) return rc;  // message set by rg_batch_create
        double ms = INFINITY;
        std::vector<std::vector<double>> ks;
        for (int run = 0; run < kRuns && rc == RG_OK; ++run) {
          const auto t0 = std::chrono::steady_clock::now();
          rc = rg_batch_step(bt, x, r, v_prev, v.data(), kap.data(), nullptr, 1);
          const double el =
              std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                  .count();
          if (run > 0 && el < ms) ms = el;
          ks.push_back(kap);
        }
        rg_options got{};
        (void)rg_batch_get_options(bt, &got);
        const std::string err = bt->err;
        rg_batch_destroy(bt);
        if (rc != RG_OK) return bfail(nullptr, rc, err);
        if (kref.empty()) {
          kref = ks;
        } else if (ks != kref) {
          return bfail(nullptr, RG_E_STATE,
                       "batch schedules disagree on kappa (block " + std::to_string(block) +
                           ", depth " + std::to_string(depth) + ", predict " +
                           std::to_string(predict) + ")");
        }
        if (ms < best_ms) {
          best_ms = ms;
          best = got;
        }
      }
    }
  }
  if (best_out) *best_out = best;
  if (best_ms_out) *best_ms_out = best_ms;
  return RG_OK;
}

int rg_batch_get_options(const rg_batch* bt, rg_options* out) {
  if (!bt || !out) return RG_E_INVAL;
  *out = bt->opt;
  return RG_OK;
}

const char* rg_batch_last_error(const rg_batch* bt) {
  if (!bt) return g_create_error.c_str();
  return bt->err.c_str();
}

const char* rg_status_string(int status) {
  switch (status) {
    case RG_OK: return "ok";
    case RG_S_INFEASIBLE: return "no admissible candidate (kappa = 0, v = v_prev)";
    case RG_S_FALLBACK: return "Newton search fell back to bisection";
    case RG_E_INVAL: return "invalid argument";
    case RG_E_NOMEM: return "out of memory";
    case RG_E_HIP: return "HIP runtime error";
    case RG_E_NOTSUP: return "not supported";
    case RG_E_STATE: return "invalid handle state";
    default: return "unknown status";
  }
}

const char* rg_last_error(const rg_handle* h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

}  // extern "C"
