/*
 * rg.h -- C ABI of the MI355X (gfx950) scenario-based robust reference governor.
 *
 * The method is that of Ossareh, Shayne and Chevalier, "CPU- and GPU-Based
 * Parallelization of the Robust Reference Governor" (arXiv 2510.08288):
 *
 *   * the closed loop x_{t+1} = f(x_t, v_t) (+ d_t), y_t = h(x_t, v_t)
 *     (Eq. (1), Eq. (4)) is integrated with fixed-step fourth-order Runge-Kutta
 *     (Sec. IV-A);
 *   * a candidate kappa in [0, 1] gives the set-point v = v_{t-1} +
 *     kappa (r_t - v_{t-1}) (Eq. (2)); it is admissible when, for every one of N
 *     sampled disturbance scenarios, the predicted outputs stay in Y over
 *     j = 0..H and the steady-state output lies in (1 - eps) Y (Eq. (3); Alg. 2;
 *     Alg. 3 parallel steps 1-3);
 *   * the governor returns the largest admissible kappa found by bisection
 *     (Alg. 1, Alg. 2) or by the grid search of Alg. 3 / Eq. (5).
 *
 * Conventions for every entry point:
 *   - All pointers are HOST pointers unless stated otherwise.  Input arrays are
 *     copied before the call returns; the caller keeps ownership.
 *   - Every function returns an int status: RG_OK (0), a positive status that
 *     comes with valid outputs, or a negative error, in which case no output
 *     was written.  No function throws or aborts across the ABI.
 *   - Calls that produce results are blocking: they enqueue work on the
 *     handle's stream and synchronise that stream before returning.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Constraint sets are polytopes Y = {y : F y <= g}; a margin is
 *     min_r (g_r - F_r y), >= 0 iff y is in Y (Sec. II-A).
 */
#ifndef RG_H
#define RG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define RG_OK 0
#define RG_S_INFEASIBLE 1  /* valid output: no evaluated candidate was admissible;
                              kappa = 0 and v = v_prev (Alg. 1 starts from kappa_opt = 0) */
#define RG_S_FALLBACK 2    /* valid output: the Newton search took at least one midpoint step */
#define RG_E_INVAL (-1)    /* null pointer, non-positive size, non-finite input, bad shape */
#define RG_E_NOMEM (-2)    /* device or host allocation failed / workspace too small */
#define RG_E_HIP (-3)      /* a HIP runtime call failed (message in rg_last_error) */
#define RG_E_NOTSUP (-4)   /* valid request outside what this build supports */
#define RG_E_STATE (-5)    /* call not allowed in the handle's current state */

/* ---- enumerations --------------------------------------------------------- */
enum rg_plant_kind {
    RG_PLANT_LQ4 = 1, /* n=4, n_w=2, n_y=2, n_theta=0; coeffs A[16] B[4] G[16] E[8] C[8]:
                         xdot = A x + B v + G (x.*x) + E w,  y = C x */
    RG_PLANT_FC9 = 2  /* n=9, n_w=9, n_y=3, n_theta=20; coeffs W[81] xbar[9] theta_nom[20]
                         c_q0 p_amb d0 d1 p1ref (115 values); with z = x - xbar, p7 = p_amb,
                         theta = (a[9], k[6], b[3], mu[2]), q0 = c_q0 x7,
                         q_l = k_l sqrt(max(x_l - x_{l+1}, 0)) (l = 1..6, x_7 read as p7):
                           xdot_i = -a_i z_i + (W tanh z)_i + w_i + phi_i,
                           phi_l = q_{l-1} - q_l (l = 1..6),
                           phi_7 = b1 v - mu1 x7 (x1 - p1ref), phi_8 = b2 v x7,
                           phi_9 = b3 v - mu2 (x9 - 1) v;
                           y = (c_q0 x7 / (d0 + d1 x9), x1, x7)  (1-based indices) */
};
enum rg_inject {
    RG_INJECT_ODE = 0, /* w enters the continuous dynamics, held over each RK4 step */
    RG_INJECT_POST = 1 /* Eq. (4): x+ = RK4(x, v) + D w (D = E for LQ4, I for FC9) */
};
enum rg_rng_mode {
    RG_RNG_STREAM = 0, /* draws generated once per RG step into device memory, read coalesced */
    RG_RNG_INLINE = 1  /* draws regenerated inside the rollout kernel from the counter */
};
enum rg_precision {
    RG_PREC_F32_RECHECK = 0, /* FP32 rollouts; lanes with |margin| < band re-simulated in FP64 */
    RG_PREC_F64 = 1          /* FP64 rollouts throughout */
};
enum rg_search {
    RG_SEARCH_BISECT = 0, /* Alg. 1 on the worst margin: kappa = 1 probe, then K halvings */
    RG_SEARCH_GRID = 1,   /* Alg. 3 / Eq. (5): M-point grid, then `refine` halvings */
    RG_SEARCH_NEWTON = 2, /* safeguarded Newton on the worst margin M(kappa), derivative from
                             the adjoint of the arg-min rollout (or the steady-state term):
                             each device round tests the iterate kappa_N, kappa_N -/+ 2^-K and
                             the bracket midpoint; a step at or past a bracket end moves
                             2^-K inside that end, a non-negative or non-finite slope falls
                             back to the midpoint (status RG_S_FALLBACK); stops at a bracket
                             of 2^-K (at most K+2 rounds).  FP32 precision only. */
    RG_SEARCH_NEWTON_TAN = 4, /* the same safeguarded Newton search, its derivative from the
                             forward tangent dx/dv carried by the iterate's FP32 rollout lanes
                             (full horizon, no checkpoints, no reverse sweep; rg_tangent):
                             about twice the iterate row's forward work instead of the
                             adjoint's separate launches.  FP32 precision only. */
    RG_SEARCH_ALG2 = 3    /* Alg. 2: every scenario runs Alg. 1 (kappa = 1 probe, K halvings)
                             on its own verdict (its rollout margin and the steady-state test),
                             one GPU lane per scenario with no barrier between candidates;
                             kappa = the smallest per-scenario result.  Equals BISECT when
                             feasibility is monotone in kappa.  FP32 verdicts within the band
                             are re-simulated in FP64 by the same lane.  rg_step only
                             (rg_closed_loop, rg_autotune: RG_E_NOTSUP); K <= 16 (the
                             steady-state margins of the 2^K tree nodes are tabulated first);
                             chance_q must be 0.  The result's worst_margin is NaN (no
                             candidate is evaluated over all scenarios; -inf if infeasible),
                             candidates = bisect_passes = the single-scenario evaluations
                             summed over scenarios. */
};
/* rg_step_info.flags */
#define RG_FLAG_GRID_NONMONOTONE 1 /* RG_SEARCH_GRID: a grid row below the returned row i* was
                                      refused (Eq. (5) takes the largest all-admissible row
                                      regardless), i.e. feasibility is not monotone in kappa
                                      on the grid */

/* ---- descriptors -------------------------------------------------------------- */
typedef struct rg_plant {
    int32_t kind;          /* enum rg_plant_kind */
    int32_t n, n_w, n_y;   /* must match the kind */
    int32_t n_theta;       /* uncertain coefficients: 0 (LQ4) or 20 (FC9) */
    const double* coeffs;  /* n_coeffs values, layout per kind */
    int32_t n_coeffs;
} rg_plant;

/* Scenario distribution (Sec. II-C: N_sim sequences drawn at each time step).
 * Draw c of scenario k at prediction step j of RG step t is the Philox4x32-10
 * word (counter (k, j, t, (0<<16) | c/4), key (seed, instance)), word c%4,
 * mapped to fl32(fl32(hi-lo) * ((word>>8) 2^-24) + fl32(lo)) by one binary32
 * fused multiply-add.  Per-scenario coefficients use tag 1 (j = 0) and the box
 * [1 - theta_rel, 1 + theta_rel) as a factor on theta_nom; the true-plant
 * disturbance of the closed loop uses tag 2 with k = j = 0. */
typedef struct rg_scenarios {
    int32_t N;             /* scenarios, >= 1 */
    uint32_t seed;         /* key word 0 */
    uint32_t instance;     /* key word 1 */
    const double* w_lo;    /* [n_w] lower box corner */
    const double* w_hi;    /* [n_w] upper box corner (>= w_lo) */
    double theta_rel;      /* relative spread of theta, in [0, 1) */
    int32_t inject;        /* enum rg_inject */
    int32_t rng_mode;      /* enum rg_rng_mode */
} rg_scenarios;

typedef struct rg_constraints {
    int32_t n_c;           /* rows, 1..4 */
    const double* F;       /* [n_c x n_y] row-major */
    const double* g;       /* [n_c] */
    double eps;            /* steady-state tightening: rows g_r - eps |g_r| - F_r y_ss >= 0 */
    int32_t ss_check;      /* 0 disables the steady-state test */
} rg_constraints;

typedef struct rg_options {
    int32_t precision;     /* enum rg_precision (default F32_RECHECK) */
    double band;           /* recheck band on |FP32 margin| (default 1e-4) */
    int32_t K;             /* halvings after the kappa = 1 probe (default 12) */
    int32_t search;        /* enum rg_search (default BISECT) */
    int32_t depth;         /* bisection levels evaluated per device round (1..6; 0 = auto) */
    int32_t M;             /* grid points for RG_SEARCH_GRID (2..127) */
    int32_t refine;        /* halvings after the grid */
    int32_t early_exit;    /* 1: a candidate stops once one lane is below -band */
    int32_t block;         /* threads per workgroup for rollouts (64..256, multiple of 64; 0 = auto) */
    int32_t max_T;         /* closed-loop steps kept on the device per chunk (default 256) */
    int32_t lanes;         /* lanes per scenario of FP32 rollouts: 1; 4 for LQ4 (one
                              scenario per quad, state split across lanes; robust or
                              chance-constrained verdict); 16 for FC9 (one scenario per group
                              of 16 lanes, one lane per state component; robust verdict, not
                              with the tangent-driven Newton search); 0 = auto (LQ4: 4; FC9:
                              16 while a round holds at most 32768 scenario-candidate pairs,
                              else 1).  kappa is the same in every layout; the 9-state
                              groups' margins are bit-identical to one lane's */
    int32_t Kc;            /* adjoint checkpoint interval in RK4 steps (default 50) */
    int32_t persistent_wgs;/* batches: workgroups of the persistent rollout kernel (0 = auto) */
    int32_t predict;       /* bisection: 1 (default) makes the first device round of a step
                              evaluate the kappa = 1 probe plus every midpoint on the bisection
                              path to the previous step's kappa (the probe alone when that was
                              1); later rounds use the speculative tree.  Only which
                              candidates are evaluated early changes: the result is that of
                              sequential bisection either way.  0: tree from round 0.
                              Newton searches: after a step that held v (kappa = 0), 1 makes
                              the first round test the kappa = 1 probe and the bisection path
                              2^-1 .. 2^-K towards 0, every candidate stopping at its first
                              violation, with no Newton iterate and no derivative; a step whose
                              candidates are all refused ends there with kappa = 0, otherwise
                              Newton continues from the bracket bisection has after that path.
                              kappa stays within 2^-K of bisection's either way. */
    int32_t speculate;     /* closed loop, bisection with prediction, FP32 LQ4 rollouts on 4 lanes
                              per scenario, streamed draws: s in 0..7 (default 7) lets a round
                              that runs the kappa = 1 probe alone also run the probes of the next
                              s steps, step t + j from the state it starts in if steps t..t+j-1
                              all have kappa = 1.  When that holds and every scenario of step
                              t + j's probe keeps a margin of at least the band, step t + j is
                              decided (kappa = 1) without a round of its own.  The results are
                              those of sequential bisection either way.  0: off. */
    int32_t chance_q;      /* chance-constrained verdict (scenario approach with discarded
                              samples, Sec. II-C): a candidate is admissible when the
                              steady-state test passes and at most chance_q of the N scenario
                              rollouts leave Y; its worst margin is then the (chance_q + 1)-th
                              smallest scenario margin (or m_ss if smaller).  0 (default): the
                              robust verdict, every scenario.  > 0: LQ4 FP32 rollouts on
                              quads of lanes (a wave runs until all its scenarios violated
                              or the candidate died), otherwise one lane per scenario; a
                              later step is decided ahead only on certain verdicts (every
                              scenario at least the band away, or more than chance_q
                              violating); bisection or grid search (Newton: RG_E_NOTSUP),
                              per-scenario margin keys in the workspace (8 B x 128 x N). */
} rg_options;

typedef struct rg_step_info {
    double kappa;          /* chosen kappa */
    double v;              /* chosen set-point */
    double worst_margin;   /* M(kappa) of the chosen candidate (-inf if none admissible) */
    int32_t status;        /* RG_OK or RG_S_INFEASIBLE */
    int32_t rounds;        /* device rounds executed */
    int32_t candidates;    /* candidate evaluations executed (incl. speculative ones) */
    int32_t rechecks;      /* (candidate, scenario) pairs re-simulated in FP64 */
    int32_t bisect_passes; /* candidate evaluations plain sequential Alg. 1 would make */
    uint32_t t;            /* RG step counter used for the draws */
    uint64_t lane_steps;   /* RK4 steps executed by FP32/FP64 rollout lanes (speculative
                              candidates and early exits included; rechecks excluded) */
    int32_t flags;         /* RG_FLAG_* diagnostics of the step */
} rg_step_info;

/* Kernel timing collected while profiling is on (rg_set_profiling). */
typedef struct rg_profile {
    int64_t rollout_launches;  /* rollout kernel launches timed */
    double rollout_ms;         /* summed HIP-event time of those launches */
    uint64_t lane_steps;       /* RK4 steps executed by those launches */
    int64_t steps;             /* RG steps covered */
} rg_profile;

typedef struct rg_handle rg_handle;
typedef struct rg_batch rg_batch;

/* One independent governor of a batch. */
typedef struct rg_instance_desc {
    rg_plant plant;
    rg_scenarios scen;     /* rng_mode is ignored: batches draw inline */
    rg_constraints cons;
    int32_t H;
    double dt;
} rg_instance_desc;

/* ---- lifecycle ---------------------------------------------------------------- */

/* Fill *opt with defaults.  Returns RG_E_INVAL if opt is NULL. */
int rg_default_options(rg_options* opt);

/* Create a governor for one problem (Eq. (3) fixes f, h, Y, eps and j* = H;
 * Sec. II-C fixes N_sim and the distribution).  H >= 1 steps of length dt > 0.
 * opt may be NULL (defaults).  All descriptor arrays are copied.  No device
 * memory is allocated here: see rg_workspace_size / rg_bind_workspace. */
int rg_create(const rg_plant* plant, const rg_scenarios* scen, const rg_constraints* cons,
              int32_t H, double dt, const rg_options* opt, rg_handle** out);

/* Release the handle and whatever device memory the library allocated itself.
 * A bound workspace is not freed.  Accepts NULL. */
int rg_destroy(rg_handle* h);

/* Bytes of device memory one handle needs. */
int rg_workspace_size(const rg_handle* h, size_t* bytes);

/* Give the handle caller-owned device memory (e.g. a torch tensor), >= the size
 * above and 256-byte aligned; it must outlive the handle.  Without a bound
 * workspace the first compute call allocates one with hipMalloc. */
int rg_bind_workspace(rg_handle* h, void* device_ptr, size_t bytes);

/* Stream (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream) that
 * all work of this handle is enqueued on; NULL = the default stream. */
int rg_set_stream(rg_handle* h, void* hip_stream);

/* RG step counter t (selects fresh scenario draws, Sec. II-C).  rg_step and
 * rg_closed_loop advance it by one per step; setting it allows exact resume. */
int rg_set_step(rg_handle* h, uint32_t t);
int rg_get_step(const rg_handle* h, uint32_t* t);

/* Forget what earlier RG steps left in the handle's device search state: the
 * previous kappa that first-round prediction follows, the speculative probes
 * of later steps, and the cache of steady-state margins by set-point.  No
 * result depends on this state (it only decides which candidates run early,
 * and a cached margin equals a recomputed one); after the call the next step
 * runs exactly as the first step of a new handle would.  t is unchanged.
 * Blocking.  RG_OK also before any device memory exists (nothing to reset). */
int rg_reset(rg_handle* h);

/* ---- the governor --------------------------------------------------------------- */

/* One RG update (Alg. 1-3 inputs x_t, v_{t-1}, r_t; output kappa_opt, v_t).
 * x: [n].  v_out required; kappa_out and info nullable.  Advances t.  Returns
 * RG_OK or RG_S_INFEASIBLE (then kappa = 0, v = v_prev). */
int rg_step(rg_handle* h, const double* x, double r, double v_prev, double* v_out,
            double* kappa_out, rg_step_info* info);

/* rg_step with its inputs and outputs in device memory, enqueued on the
 * handle's stream without waiting: one RG update (Alg. 1-3 inputs x_t,
 * v_{t-1}, r_t; output kappa_opt, v_t) that a caller can capture into a HIP
 * graph of its own and replay, or chain behind its own kernels.  All pointers
 * are device memory on the handle's device, owned by the caller, and must stay
 * valid until the step has run: x [n] (FP64), r, v_prev (one FP64 each), t
 * (one uint32: the step index that selects the scenario draws; the step reads
 * it and writes t + 1, so replays of a captured step advance it), v_out
 * (FP64), kappa_out (FP64, nullable), status_out (int32, nullable: 0 admitted,
 * 1 infeasible with kappa = 0 and v = v_prev, 2 Newton fell back to bisection).
 * Inputs are not checked for finiteness (they are never read on the host).
 * Same kappa, v and status as rg_step at the same x, r, v_prev and t; the
 * handle's own step counter (rg_set_step, rg_get_step) is neither read nor
 * advanced.  No host copies, synchronisation or allocation once the workspace
 * is in place: the first call on a handle sets it up (allocating unless one is
 * bound, and synchronising), so make one call (or one rg_step) before
 * capturing; under capture without it, RG_E_STATE.  RG_E_NOTSUP for Alg. 2,
 * RG_E_STATE while profiling is on.  Steps on one handle run in stream order;
 * overlapping steps of one handle on different streams race. */
int rg_step_async(rg_handle* h, const double* x, const double* r, const double* v_prev,
                  uint32_t* t, double* v_out, double* kappa_out, int32_t* status_out);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, tight serving loops): rg_step without a workspace.  Same
 * arguments, outputs, status and effect on t as rg_step, and the same kappa, v
 * and worst margin.  It allocates nothing: the search record, the result
 * record and the FP64 recheck list live in one static device array of 8 MiB
 * per GPU (held until the process ends), and the scenario draws are
 * regenerated inside the kernels (bit-identical to the streamed draws).  Runs
 * on the current device; the handle's stream must belong to it.  Every call
 * starts from a fresh search record (no first-round prediction from earlier
 * steps; results do not depend on it).  All calls on one GPU share the array,
 * so calls that overlap in time on one GPU (threads, streams, handles) race:
 * serialise them.  RG_E_NOTSUP when the recheck list, 8 B x N x (candidates
 * per device round), does not fit beside the 14 KB of records (for example
 * N = 4096 at the default 13 candidates per round needs 0.43 MB; the limit is
 * about 1e6 scenario-candidate pairs), and for the Newton search, Alg. 2 and
 * the chance-constrained verdict; RG_E_STATE while profiling is on. */
int rg_step_noalloc(rg_handle* h, const double* x, double r, double v_prev, double* v_out,
                    double* kappa_out, rg_step_info* info);

/* Worst margins of explicit candidates without searching (Alg. 3 step 5 for a
 * given list): margins[i] = min(min_k m^k(v_i), m_ss(v_i)) with v_i from
 * kappa[i] (each in [0, 1]), full horizon, t unchanged.  per_scenario
 * (nullable) receives the [M x N] FP32 (or FP64-rounded, in F64 precision)
 * rollout margins before any recheck; per_scenario_j (nullable) the first step
 * attaining each.  In F32_RECHECK precision, margins[] uses the FP64 value of
 * every lane with |m32| < band. */
int rg_margin(rg_handle* h, const double* x, double r, double v_prev, const double* kappa,
              int32_t M, double* margins, float* per_scenario, int32_t* per_scenario_j);

/* T closed-loop steps on the device (Fig. 1): at step s the governor picks
 * v_s from (x_s, v_{s-1}, r_seq[s]), then the true plant advances
 * x_{s+1} = RK4(x_s, v_s) under the tag-2 disturbance.  x0: [n]; r_seq: [T];
 * v_out, kappa_out: [T]; x_out: [(T+1) x n]; info_out: [T]; outputs nullable
 * except v_out.  Advances t by T.  The device runs generic search rounds (the
 * current step's next round; a step's result is recorded, and the next step
 * prepared, once its search has ended); the host enqueues one round per step
 * not yet recorded and reads the device's count of recorded steps, a few
 * times per chunk of max_T steps.  use_graph = 1 replays the rounds from HIP
 * graphs captured once per handle and stream; profiling forces plain launches.
 * RG_E_STATE if steps stay unrecorded after the planned number of rounds per
 * step. */
int rg_closed_loop(rg_handle* h, const double* x0, double v0, const double* r_seq, int32_t T,
                   double* v_out, double* kappa_out, double* x_out, rg_step_info* info_out,
                   int32_t use_graph);

/* The options in force, with auto fields (depth, lanes) resolved. */
int rg_get_options(const rg_handle* h, rg_options* out);

/* Autotuner of the launch schedule.  Runs the closed loop of T RG updates from
 * (x0, v0) under r_seq (as rg_closed_loop, graph replay, starting at the
 * handle's step counter, which is restored afterwards) for every candidate
 * schedule (three runs: the first captures the graphs, the faster of the other
 * two counts): lanes per scenario (FP32 rollouts: 1 or 4 for LQ4, 1 or 16 for
 * FC9 with the robust verdict), rollout workgroup (128 or 256 threads), device
 * search depth (2..5; 1..3 for the grid refinement), first-round prediction
 * (on/off, bisection only) and the
 * speculation depth (7, 3, 1, 0; with prediction and 4 lanes).  Schedules
 * change only which candidates run when, so every one must give the same kappa
 * sequence; a mismatch returns RG_E_STATE.  best_out (nullable) receives the
 * fastest schedule's options, best_ms_out (nullable) its time per update; with
 * apply = 1 the handle keeps that schedule, else its own.  The first-round
 * prediction state is reset.  Host-blocking; allocates nothing beyond the
 * workspace. */
int rg_autotune(rg_handle* h, const double* x0, double v0, const double* r_seq, int32_t T,
                int32_t apply, rg_options* best_out, double* best_ms_out);

/* Profiling: with enable = 1, every rollout launch is bracketed by HIP events
 * on the handle's stream and the totals accumulate until reset (enable = 1
 * again resets).  rg_get_profile copies the totals. */
int rg_set_profiling(rg_handle* h, int32_t enable);
int rg_get_profile(const rg_handle* h, rg_profile* out);

/* Derivatives of the candidate kappa's margins (not in the paper; they back the
 * Newton search).  Reverse mode through the discrete RK4 map of each selected
 * scenario: a forward pass keeps the state every Kc steps, the reverse sweep
 * recomputes one segment at a time.  States and adjoints are FP32, parameter
 * sums FP64, and the sum over scenarios has a fixed order (deterministic).
 *   upstream == NULL: derivative of the worst margin M(kappa) = min(min_k m^k,
 *     m_ss): the first minimising scenario's rollout term, or the steady-state
 *     term (implicit-function derivative, FP64) when that is smaller;
 *   upstream [N]: sum_k upstream[k] * d m^k, over scenarios with a nonzero weight.
 * Outputs: margin_out (nullable) = M(kappa); dkappa_out = d/dkappa (through
 * v = v_prev + kappa (r - v_prev)); dtheta_out (nullable, [n_theta]) =
 * d/d(nominal coefficients) through theta^k = theta_nom * factor_k.  The margin
 * is not differentiable where the minimiser changes; the derivative returned
 * there is that of the first minimiser.  t is not advanced.  RG_E_NOTSUP for a
 * handle with the chance-constrained verdict (chance_q > 0). */
int rg_grad(rg_handle* h, const double* x, double r, double v_prev, double kappa,
            const float* upstream, double* margin_out, double* dkappa_out, double* dtheta_out);

/* Forward-mode counterpart of rg_grad (not in the paper; it backs
 * RG_SEARCH_NEWTON_TAN): one FP32 rollout of every scenario under the candidate
 * kappa carries the tangent dx/dv of the discrete RK4 map (draws held fixed)
 * over the full horizon.  Outputs (nullable except dkappa_out), each [N]:
 * m_out = the scenario's FP32 margin m^k, dm_dv_out = dm^k/dv at its first
 * minimising step and row, j_out = that step; margin_out = M(kappa) (FP64
 * recheck within the band, steady-state term included); dkappa_out = dM/dkappa
 * = dM/dv (r - v_prev) of the active term (the arg-min scenario's tangent, or
 * the steady-state implicit derivative when that term is smaller).  FP32
 * precision only (else RG_E_NOTSUP); t is not advanced. */
int rg_tangent(rg_handle* h, const double* x, double r, double v_prev, double kappa,
               float* m_out, float* dm_dv_out, int32_t* j_out, double* margin_out,
               double* dkappa_out);

/* Replace the nominal uncertain coefficients theta_nom ([n_theta], FC9 only);
 * scenario k then uses theta_nom * factor_k with unchanged factors.
 * RG_E_NOTSUP for plants without coefficients. */
int rg_set_theta(rg_handle* h, const double* theta_nom);

/* Equilibrium of the nominal closed loop under constant set-point v (w = 0):
 * the state behind y_ss(v), from the Newton iteration of the steady-state test
 * (Sec. II-A).  x_out: [n].  RG_E_STATE if it does not converge. */
int rg_equilibrium(rg_handle* h, double v, double* x_out);

/* ---- batched serving (many independent governors per launch) ---------------------- */

/* A batch of `count` independent governors (own plant, scenarios, constraints,
 * H and dt each; the paper notes one small governor gains little from a GPU,
 * Sec. IV-B).  Each instance keeps its own search record and FP64 recheck list
 * in one device allocation, and its draws are regenerated inside the kernels
 * (the scenarios' rng_mode is ignored).  One search round of the whole batch is
 * one flat rollout launch per group of instances with the same plant kind and
 * injection (all their scenario tiles in one grid, FP32, one lane per
 * scenario), then each instance's FP64 recheck and decision.  All instances
 * use one search depth (opt.depth = 0: from the sum of N over the batch; large
 * batches evaluate one candidate per round).  opt: precision F32_RECHECK,
 * search BISECT or GRID, chance_q 0 (else RG_E_NOTSUP); block is the scenario
 * tile (64, 128, 256); predict as for rg_create; persistent_wgs is accepted
 * and unused.  opt = NULL: the defaults of rg_default_options except block =
 * 64 and predict = 0 (a batch's rounds are throughput-bound, so the least
 * candidates per round is fastest).  Every descriptor is validated as by rg_create (error
 * names the instance; message via rg_batch_last_error(NULL)).  No device
 * memory is allocated here. */
int rg_batch_create(const rg_instance_desc* descs, int32_t count, const rg_options* opt,
                    rg_batch** out);
int rg_batch_destroy(rg_batch* b);
/* Stream the batch's steps are ordered on (NULL: a stream of the batch's own). */
int rg_batch_set_stream(rg_batch* b, void* hip_stream);
/* Per-instance RG step counter (draw selection); starts at 0, +1 per rg_batch_step. */
int rg_batch_set_step(rg_batch* b, int32_t instance, uint32_t t);
/* The options in force (depth resolved). */
int rg_batch_get_options(const rg_batch* b, rg_options* out);
/* Autotuner of a batch's launch schedule (not in the paper; serving
 * throughput).  For every candidate schedule — scenario tile, i.e. waves per
 * workgroup column of an instance (opt.block 64, 128, 256), search depth (1, 2,
 * 3) and first-round prediction (off, on) — creates the batch of `count`
 * instances described by descs (other options from opt, NULL: the defaults of
 * rg_batch_create), runs its steps t = 0, 1, 2 from the states x and references r,
 * v_prev (as rg_batch_step, graph replay; the first step allocates and
 * captures) and times the faster of the last two; the batch is then
 * destroyed.  Lanes per scenario are not a choice: batches run one lane per
 * scenario.  Schedules change only which candidates run when, so every one must
 * give the same kappa at every step; a mismatch returns RG_E_STATE.  best_out
 * (nullable) receives the fastest schedule's options (depth resolved),
 * best_ms_out (nullable) its time per batched step in ms.  Errors as
 * rg_batch_create and rg_batch_step (message via rg_batch_last_error(NULL)).
 * Allocates and frees one batch's device memory per schedule; host-blocking. */
int rg_batch_autotune(const rg_instance_desc* descs, int32_t count, const rg_options* opt,
                      const double* x, const double* r, const double* v_prev,
                      rg_options* best_out, double* best_ms_out);
/* One RG step of every instance.  x: the instances' states packed in order
 * (n_i values each); r, v_prev, v_out: [count]; kappa_out and info_out
 * ([count]) nullable.  use_graph = 1 captures the step once as a HIP graph
 * and replays it.  The first call allocates the batch's device memory.
 * Blocking. */
int rg_batch_step(rg_batch* b, const double* x, const double* r, const double* v_prev,
                  double* v_out, double* kappa_out, rg_step_info* info_out, int32_t use_graph);
const char* rg_batch_last_error(const rg_batch* b);

/* ---- inspection ----------------------------------------------------------------- */

/* Scenario draws as the device sees them: w_out[(j - j0) * nk * n_w + (k - k0) * n_w + c]
 * for k in [k0, k0+nk), j in [j0, j0+nj), at RG step t; theta_out (nullable)
 * [nk x n_theta] per-scenario coefficients (FP64 value theta_nom * factor). */
int rg_draws(rg_handle* h, uint32_t t, int32_t k0, int32_t nk, int32_t j0, int32_t nj,
             float* w_out, double* theta_out);

/* Predicted states of scenarios k_list[0..nk) under set-point v at the current
 * t, starting from x: traj[(i * (H + 1) + j) * n + s].  precision selects the
 * FP32 or FP64 rollout code path of the governor's kernels. */
int rg_trajectory(rg_handle* h, const double* x, double v, const int32_t* k_list, int32_t nk,
                  int32_t precision, double* traj);

/* The FP64 tanh the FP64 rollouts, rechecks and steady-state solves of the
 * 9-state plant use, evaluated on the current device for x[0..n) into y
 * (host arrays; for tests of its accuracy).  Blocking; allocates and frees
 * device memory. */
int rg_fp64_tanh(const double* x, double* y, int32_t n);

/* Static text for a status code. */
const char* rg_status_string(int status);

/* Last error message of a handle (empty string if none); NULL handle gives the
 * last error of a failed rg_create in this thread. */
const char* rg_last_error(const rg_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* RG_H */
