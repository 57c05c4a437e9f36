/*
 * rg_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, sequential, FP64 CPU reference of the scenario-based robust reference
 * governor (RG) of "CPU- and GPU-Based Parallelization of the Robust Reference
 * Governor" (Ossareh, Shayne, Chevalier; arXiv 2510.08288).  It exists to check
 * the GPU library against; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may call it.  It shares no code, header, table or constant
 * with the GPU library.
 *
 * Every function states the passage of the paper it follows.  Where the paper
 * is silent the reading used is stated next to the code.
 *
 * Parity status:
 *   pinned   : Philox (published known-answer vectors), LQ4 rollout (RK4
 *              matrix-polynomial closed form), LQ4 steady state (fixed point of
 *              the closed form), FC9 right-hand side and outputs (values worked
 *              out by hand at x = xbar and at chosen states, flow telescoping,
 *              single coupling entries, the closed check valve), FC9 steady
 *              state (closed-form equilibrium with W = 0 and a_1..a_6 = 0),
 *              RK4 order on both plants (against an independent solver),
 *              bisection / Alg. 2 / Alg. 3 search (exact linear ratio test,
 *              brute-force grids, invariants), closed loop (recursive
 *              feasibility), tangent gradients (central FD, linear closed form).
 *   not pinned by a closed form: FC9 trajectories under disturbance and
 *              coefficient spread (checked through the pinned right-hand side,
 *              RK4 order, equilibrium convergence and FD gradients).
 */
#ifndef RG_ORACLE_H
#define RG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXN 9      /* largest state dimension (FC9) */
#define ORC_MAXW 9      /* largest disturbance dimension */
#define ORC_MAXY 4      /* largest output dimension */
#define ORC_MAXC 8      /* largest number of constraint rows */
#define ORC_MAXTH 20    /* largest number of uncertain coefficients */
#define ORC_MAXCOEF 128 /* plant coefficient storage */

enum { ORC_LQ4 = 1, ORC_FC9 = 2 };
enum { ORC_INJECT_ODE = 0, ORC_INJECT_POST = 1 };

/*
 * Problem description (plant, constraints, scenario distribution, horizon).
 *
 * LQ4 coefficients (row-major):  A[16] B[4] G[16] E[8] C[8]
 *   f(x,v,w) = A x + B v + G (x.*x) + E w ,   y = C x
 * FC9 coefficients:  W[81] xbar[9] theta_nom[20] c_q0 p_amb d0 d1 p1ref
 *   theta = (a[9], k[6], b[3], mu[2]); the equations are in rg_oracle.c.
 */
typedef struct {
    int32_t kind;
    int32_t n, n_w, n_y, n_theta;
    double coeffs[ORC_MAXCOEF];
    int32_t n_c;
    double F[ORC_MAXC * ORC_MAXY]; /* n_c x n_y, row-major */
    double g[ORC_MAXC];
    double eps;                    /* steady-state tightening */
    int32_t ss_check;              /* 0: skip the steady-state test */
    int32_t N;                     /* scenarios */
    uint32_t seed, instance;       /* Philox key */
    double w_lo[ORC_MAXW], w_hi[ORC_MAXW];
    double theta_rel;              /* per-scenario relative spread of theta */
    int32_t inject;                /* ORC_INJECT_ODE or ORC_INJECT_POST */
    int32_t H;                     /* prediction horizon j* (RK4 steps) */
    double dt;
    int32_t nthreads;              /* threads over scenarios (timing driver) */
} orc_problem;

/* ---- random numbers --------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float orc_uniform_box(uint32_t word, double lo, double hi);
void orc_draw_w(const orc_problem* p, uint32_t t, uint32_t k, uint32_t j, double* w);
void orc_draw_theta(const orc_problem* p, uint32_t t, uint32_t k, double* theta);
void orc_draw_true_w(const orc_problem* p, uint32_t t, double* w);

/* ---- plant ------------------------------------------------------------- */
void orc_rhs(const orc_problem* p, const double* theta, const double* x, double v,
             const double* w, double* xdot);
void orc_output(const orc_problem* p, const double* x, double v, double* y);
void orc_rk4(const orc_problem* p, const double* theta, const double* x, double v,
             const double* w, double* xn);
void orc_step(const orc_problem* p, const double* theta, const double* x, double v,
              const double* w, double* xn);
double orc_margin(const orc_problem* p, const double* y, int32_t* r_arg);

/* ---- prediction and verdict ------------------------------------------- */
double orc_candidate_v(double kappa, double r, double v_prev);
double orc_rollout(const orc_problem* p, const double* x0, double v, uint32_t t, uint32_t k,
                   int32_t* j_arg, int32_t* r_arg, double* traj);
double orc_steady_margin(const orc_problem* p, double v, double* x_ss, int32_t* iters);
double orc_candidate(const orc_problem* p, const double* x0, double v, uint32_t t,
                     double* per_scen, int32_t* k_arg, double* m_ss_out);

/* ---- kappa searches ----------------------------------------------------- */
typedef struct {
    double kappa, v, worst;   /* result, set-point, worst margin at the result */
    int32_t passes;           /* candidate evaluations performed */
    int32_t status;           /* 0 ok, 1 no admissible candidate found (kappa=0) */
} orc_result;

orc_result orc_bisect(const orc_problem* p, const double* x0, double r, double v_prev,
                      uint32_t t, int32_t K, double* trace_kappa, double* trace_margin);
orc_result orc_alg2(const orc_problem* p, const double* x0, double r, double v_prev,
                    uint32_t t, int32_t K);
orc_result orc_grid(const orc_problem* p, const double* x0, double r, double v_prev,
                    uint32_t t, int32_t M, int32_t refine, uint8_t* Pmat);

/* ---- chance-constrained verdict (at most q violating scenarios) --------- */
double orc_candidate_q(const orc_problem* p, const double* x0, double v, uint32_t t, int32_t q,
                       double* per_scen, int32_t* n_viol);
orc_result orc_bisect_q(const orc_problem* p, const double* x0, double r, double v_prev,
                        uint32_t t, int32_t K, int32_t q);

/* ---- closed loop ------------------------------------------------------- */
void orc_plant_step(const orc_problem* p, const double* x, double v, uint32_t t, double* xn);
int32_t orc_closed_loop(const orc_problem* p, const double* x0, double v0, const double* r_seq,
                        int32_t T, uint32_t t0, int32_t search, int32_t K, int32_t M,
                        int32_t refine, double* v_out, double* kappa_out, double* x_out);

/* ---- sensitivities (back the adjoint / Newton search) ------------------ */
double orc_rollout_tangent(const orc_problem* p, const double* x0, double v, uint32_t t,
                           uint32_t k, double* dm_dv, double* dm_dtheta_nom,
                           int32_t* j_arg, int32_t* r_arg);
double orc_steady_tangent(const orc_problem* p, double v, double* dmss_dv, double* dmss_dtheta);
double orc_candidate_grad(const orc_problem* p, const double* x0, double kappa, double r,
                          double v_prev, uint32_t t, double* dM_dkappa, double* dM_dtheta,
                          int32_t* k_arg);
orc_result orc_newton(const orc_problem* p, const double* x0, double r, double v_prev,
                      uint32_t t, int32_t K, int32_t* rounds_out, int32_t* fallbacks_out);

#ifdef __cplusplus
}
#endif
#endif
