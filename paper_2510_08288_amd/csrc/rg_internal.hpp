// Internal layout shared by the HIP kernels and the host side of librg.
// Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rg {

constexpr int kCMax = 128;   // candidates per device round
constexpr int kMaxN = 9;     // state dimension
constexpr int kMaxW = 9;     // disturbance dimension
constexpr int kMaxY = 3;     // output dimension
constexpr int kNC = 4;       // constraint rows evaluated per step (unused rows padded)
constexpr int kMaxTh = 20;   // uncertain coefficients
// Steps per prefetch group of the LQ4 quad rollout; the streamed draw buffer
// holds this many spare rows past the horizon so whole groups load unclamped.
constexpr int kQuadGroup = 16;
constexpr int kMaxCoef = 115;

enum Mode { kBisect = 0, kGrid = 1, kNewton = 2 };

// Per-handle control state kept in device memory so that whole RG steps (and
// closed loops) can be enqueued or graph-captured without host round trips.
// Closed-loop speculation: a probe-only round may also run the kappa = 1
// probes of up to kSpecMax later steps; draws are kept for kPairs steps.
constexpr int kSpecMax = 7;
constexpr int kMssCache = 64;
constexpr int kPairs = kSpecMax + 2;

struct DevState {
  double x[kMaxN];      // x_t
  double v_prev;        // v_{t-1}
  double r;             // r_t
  uint32_t t;           // RG step counter (selects the draws)
  int32_t cl_index;     // closed loop: index of the current step in the chunk
  int32_t cl_len;       // closed loop: steps in the chunk
};

// Search state of one RG step.  Candidate c of the current round has set-point
// v[c]; tree nodes of a speculative bisection round keep their bracket in
// a_lo/a_hi so that node kappa = (a_lo + a_hi) / 2 reproduces the arithmetic
// of sequential bisection exactly.
struct DevSearch {
  // configuration
  int32_t mode, K, depth, M, refine, precision;
  int32_t ss_check, n_c, ny;
  double eps;
  double g[kNC];        // constraint right-hand sides (padded rows +inf)
  double F[kNC * kMaxY];
  // per-step state
  double lo, hi;
  int32_t round, halvings, goal, done, found, status;
  int32_t n_cand, probe, tree_base, tree_depth;
  double kappa_res, v_res, worst_res;
  int32_t cand_total, rechecks_total, rounds_total, passes_alg1;
  // per candidate of the current round
  double kappa[kCMax];
  double v[kCMax];
  double mss[kCMax];
  double a_lo[kCMax], a_hi[kCMax];
  unsigned long long key_all[kCMax];  // min over lanes of the FP32/FP64 rollout margin key
  unsigned long long key_far[kCMax];  // same, over lanes outside the recheck band
  unsigned long long key64[kCMax];    // min over FP64-rechecked lanes (ordered double)
  int32_t dead[kCMax];                // a lane fell below -band or went non-finite
  int32_t fail64[kCMax];              // a rechecked lane has an FP64 margin < 0
  int32_t n_recheck;                  // entries in the recheck list this round
  unsigned long long lane_steps;      // RK4 steps executed by rollout lanes this RG step
  int32_t full[kCMax];                // 1: no early exit / steady-state refusal (Newton iterate)
  // Newton search
  int32_t nk_idx;                     // candidate carrying the Newton iterate this round
  int32_t fallbacks;                  // rounds that used the midpoint instead of a Newton step
  double delta;                       // 2^-K
  // Bisection: round 0 speculates along the path to the previous step's kappa
  int32_t predict;                    // 1: enabled
  double pred;                        // previous step's kappa (NaN: none yet)
  // Workgroups of the current recheck launch that have finished; the last one
  // takes the round's decision and resets the count.
  uint32_t blocks_done;
  // Closed loop, round 0 speculating on the next spec_n steps: candidates
  // spec_base + (j - 1) * spec_per .. + spec_per - 1 belong to step t + j,
  // simulated from x_spec[j - 1] under the draws of step t + j.  spec_kind 1:
  // the previous kappa was 1, step t + j's kappa = 1 probe alone (spec_per = 1),
  // from the state it starts in if steps t..t + j - 1 all take kappa = 1.
  // spec_kind 2: the previous kappa was 0 (the governor holds v), step t + j's
  // whole first round (the probe and the K midpoints towards 0, spec_per =
  // 1 + K), from the state it starts in if steps t..t + j - 1 all hold v.  The
  // following steps consume them in order while the assumption holds.
  int32_t spec_depth;                 // allowed depth of kappa = 1 speculation (set by the host)
  int32_t spec_hold;                  // allowed depth of hold speculation (set by the host)
  int32_t spec_kind;                  // 1: kappa = 1 probes, 2: holds
  int32_t spec_base;                  // first speculative candidate
  int32_t spec_per;                   // speculative candidates per later step
  int32_t spec_n;                     // later steps speculated on in the last live round
  int32_t spec_used;                  // of those, consumed by the steps since
  double r_spec[kSpecMax];            // their references
  double x_spec[kSpecMax][kMaxN];     // their start states
  double band;                        // FP32 recheck band (a speculative verdict must be outside it)
  // Steady-state margins of recent set-points (a pure function of v for fixed
  // plant coefficients; NaN keys are empty entries, cleared when the nominal
  // coefficients change)
  double mss_v[kMssCache];
  double mss_m[kMssCache];
  int32_t mss_next;
  // Chance-constrained verdict (q > 0): a candidate is admissible when at most
  // q scenarios violate.  nviol counts the certain violations of the rollouts
  // (FP32 margin below -band, FP64 margin below 0), nviol64 the FP64-rechecked
  // ones; dead / fail64 are raised once the count exceeds q.  keyq is the
  // (q + 1)-th smallest per-scenario margin key of the candidate (~0: none).
  int32_t q;
  int32_t nviol[kCMax];
  int32_t nviol64[kCMax];
  unsigned long long keyq[kCMax];
  // Diagnostics of the current step (bit 0: the grid of Alg. 3 refused a row
  // below the row it returns, so feasibility was not monotone in kappa there)
  int32_t flags;
};

// Result record of one RG step.
struct DevResult {
  double kappa, v, worst;
  int32_t status, rounds, candidates, rechecks, passes_alg1;
  uint32_t t;
  unsigned long long lane_steps;
  int32_t flags;
};

// Gradient of a candidate's margin (rg_grad, Newton search).
struct DevGrad {
  int32_t n_entries;       // adjoint entries (0: the steady-state term is active)
  int32_t k_star;          // arg-min scenario (-1: steady state)
  double M;                // candidate worst margin
  double dM_dv;            // derivative w.r.t. the set-point
  double dM_dkappa;        // dM_dv * (r - v_prev)
  double dM_dth[kMaxTh];   // derivative w.r.t. the nominal coefficients
  int32_t j_star, r_star;  // minimising step and row of k_star
};

struct PlantDesc {
  int32_t kind, n, nw, ny, nth;
  double coeffs[kMaxCoef];
};

struct ConsDesc {
  int32_t n_c;
  double F[kNC * kMaxY];  // row-major n_c x n_y, rows >= n_c zero
  double g[kNC];          // rows >= n_c are +inf (never binding)
  double eps;
  int32_t ss_check;
};

struct ScenDesc {
  int32_t N;
  uint32_t seed, instance;
  double wlo[kMaxW], whi[kMaxW];
  double theta_rel;
  int32_t inject, rng_mode;
};

// Device buffers of one handle (all inside one workspace allocation).
struct DevBuffers {
  DevState* st;
  DevSearch* srch;
  DevResult* res;          // [max_T] results of a closed-loop chunk (entry 0 for rg_step)
  double* r_seq;           // [max_T]
  double* x_hist;          // [(max_T + 1) * n]
  float* wbuf;             // [H][nw][N] streamed draws
  float* thbuf;            // [nth][N] per-scenario coefficient factors
  // closed loop: step s reads pair s % kPairs (the speculative probe of step
  // t + j reads pair (t + j) % kPairs), and the first round of step t
  // generates the draws of step t + kSpecMax + 1
  float* wpair[kPairs];     // closed-loop draw pairs (step s uses pair s % kPairs)
  float* thpair[kPairs];
  int32_t ring;            // 1: kernels select pair t % kPairs themselves (generic closed-loop rounds)
  int2* rlist;             // [cmax_round * N] recheck list (candidate, scenario)
  float* per_m;            // [cmax_round * N] per-scenario margins (rg_margin)
  int32_t* per_j;          // [cmax_round * N]
  // [cmax_round * N] ordered keys of the per-scenario margins (chance-constrained
  // verdict only: the FP32 or FP64 rollout margin, replaced by the FP64 value
  // for rechecked scenarios)
  unsigned long long* per_key;
  double* alg2_mss;        // [2^K] steady-state margins of the bisection tree's nodes (Alg. 2)
  float* tan_dv;           // [N] forward tangent dm/dv of the tangent candidate's scenarios
  double* scratch;         // small staging area (trajectories, draws)
  size_t scratch_bytes;
  // adjoint
  DevGrad* grad;           // result of the last gradient request
  int32_t* adj_k;          // [N] scenario of each adjoint entry
  float* adj_w;            // [N] upstream weight of each entry
  float* adj_m;            // [N] margin of each entry
  double* adj_dv;          // [N] weighted dm/dv of each entry
  double* adj_dth;         // [N * kMaxTh] weighted dm/dtheta_nom of each entry
  float* adj_ckpt;         // [(H / Kc + 1) * n * N] forward checkpoints (SoA by entry)
  float* adj_seg;          // [Kc * n * N] recomputed segment states
  // segment-parallel derivative (S = H / Kc + 1 segments)
  float* seg_m;            // [S]
  int32_t* seg_j;          // [S]
  int32_t* seg_r;          // [S]
  float* seg_x;            // [S * n]
  float* seg_a;            // [S * n * n]
  double* seg_cv;          // [S * n]
  double* seg_ct;          // [S * n * kMaxTh]
  float* seg_scr;          // [Kc * n * S * n]
};

struct LaunchCfg {
  int lanes;               // lanes per scenario in FP32 LQ4 rollouts (1 or 4)
  int block;               // threads per rollout workgroup
  int cmax_round;          // largest candidate count of any round
  int rounds;              // device rounds per RG step
  int chance;              // 1: chance-constrained verdict (q > 0), its own rollout kernels
  int tan;                 // 1: derivatives by the forward tangent fused into the rollout
};

// Everything a launch needs about the problem (host copy).
struct Problem {
  PlantDesc p;
  ScenDesc s;
  ConsDesc c;
  int H;
  double dt;
};

// ---- launchers implemented in rg_kernels.hip --------------------------------
// Draws of step t + t_ofs (t: the device step counter) into b.wbuf / b.thbuf.
hipError_t launch_gen(const Problem& pr, const DevBuffers& b, hipStream_t st, uint32_t t_ofs = 0);
// Whether launch_rollout runs the LQ4 quad kernel for this configuration.
bool rollout_uses_quad(const Problem& pr, const LaunchCfg& cfg, int precision);
// Draws plus the round-0 setup in one launch (workgroup 0 runs the setup).
hipError_t launch_gen_setup(const Problem& pr, const DevBuffers& b, int closed_loop, hipStream_t st);
hipError_t launch_setup(const Problem& pr, const DevBuffers& b, int closed_loop, hipStream_t st);
hipError_t launch_setup_list(const Problem& pr, const DevBuffers& b, int M, hipStream_t st);
// ckpt_cand >= 0 (or -1 for the Newton iterate) keeps that candidate's
// checkpoints every Kc steps for the segment derivative; -2 keeps none.
// gen_w (non-null, streamed draws, closed loop): the launch also has
// workgroups of its own that generate, in a step's first round, the draws of
// step t + kSpecMax + 1 into the buffer pair the step counter selects.
hipError_t launch_rollout(const Problem& pr, double band, int precision, int early_exit, int record,
                          const LaunchCfg& cfg, const DevBuffers& b, hipStream_t st,
                          int ckpt_cand = -2, int Kc = 0, float* gen_w = nullptr,
                          float* gen_th = nullptr);
// decide != 0: the last workgroup to finish also takes the round's decision
// (the work of launch_decide), so no separate decision launch follows.
hipError_t launch_recheck(const Problem& pr, int early_exit, const LaunchCfg& cfg,
                          const DevBuffers& b, hipStream_t st, int decide = 0);
hipError_t launch_decide(const Problem& pr, const DevBuffers& b, hipStream_t st);
// setup_next (closed loop): the same launch prepares round 0 of the next step
// of the chunk, if there is one.
// when_done: only once the step's search has ended (generic closed-loop rounds).
hipError_t launch_finalize(const Problem& pr, int closed_loop, const DevBuffers& b,
                           hipStream_t st, int setup_next = 0, int when_done = 0);
hipError_t launch_collect(const DevBuffers& b, int M, double* out_dev, hipStream_t st);
// Alg. 2: per-scenario bisection (K halvings after the kappa = 1 probe) in one
// lane per scenario, the minimum over scenarios, and the result record.
hipError_t launch_alg2(const Problem& pr, double band, int precision, int early_exit, int K,
                       int block, const DevBuffers& b, hipStream_t st);
// Chance-constrained verdict: (q + 1)-th smallest margin key of each candidate
// (all = 0: only candidates still admissible).
hipError_t launch_select_q(const DevBuffers& b, int N, int cmax_round, int all, hipStream_t st);
hipError_t launch_draws(const Problem& pr, uint32_t t, int k0, int nk, int j0, int nj,
                        float* w_dev, double* th_dev, const DevBuffers& b, hipStream_t st);
hipError_t launch_equilibrium(const Problem& pr, const DevBuffers& b, double v, double* out_dev,
                              hipStream_t st);
hipError_t launch_grad_prepare(const Problem& pr, const DevBuffers& b, int cand, int use_keys,
                               hipStream_t st);
hipError_t launch_adjoint(const Problem& pr, int Kc, int max_entries, const DevBuffers& b,
                          int cand, hipStream_t st);
// Derivative of the worst margin of one scenario (k_star of the gradient
// record) from the checkpoints the rollout kept: segment kernels.
hipError_t launch_seg_grad(const Problem& pr, int Kc, int cand, const DevBuffers& b,
                           hipStream_t st);
// dM/dkappa of candidate cand (-1: the Newton iterate) from the forward tangent
// its rollout kept (or the steady-state term), into b.grad.
hipError_t launch_tan_grad(const Problem& pr, const DevBuffers& b, int cand, hipStream_t st);
hipError_t launch_grad_reduce(const DevBuffers& b, int max_entries, int nth, int cand,
                              hipStream_t st);
// Batched serving: per-instance FP32 rollout argument blocks (host side), and
// the flat rollout launch over a group of instances of one plant kind and
// injection (grid: tiles x cmax, workgroup `block` = the tile size).
hipError_t launch_eval_tanh64(const double* x_dev, double* y_dev, int n, hipStream_t st);
size_t flat_args_size(int kind);
void flat_fill_args(const Problem& pr, double band, int early, const DevBuffers& b, void* out);
hipError_t launch_flat_rollout(int kind, int inject, const void* args_dev, const int* tile_inst,
                               const int* tile_first, int tiles, int cmax, int block,
                               hipStream_t st);
// FP64 recheck argument blocks and control blocks of the instances, and the
// flat launches over a group: recheck + decision (one workgroup per instance),
// round-0 setup (one workgroup per instance), result records (res_dev: the
// instances' result record addresses, device array).
size_t flat_args64_size(int kind);
size_t flat_ctl_size(int kind);
void flat_fill_args64(const Problem& pr, int early, const DevBuffers& b, void* out);
void flat_fill_ctl(const Problem& pr, const DevBuffers& b, void* out);
hipError_t launch_flat_recheck(int kind, int inject, const void* args64_dev, const void* ctl_dev,
                               int count, hipStream_t st);
hipError_t launch_flat_setup(int kind, const void* ctl_dev, int count, hipStream_t st);
hipError_t launch_flat_finalize(int kind, const void* ctl_dev, DevResult* const* res_dev, int count,
                                hipStream_t st);
hipError_t launch_trajectory(const Problem& pr, double v, const int32_t* k_list_dev, int nk,
                             int precision, double* traj_dev, const DevBuffers& b,
                             hipStream_t st);

}  // namespace rg
