/*
 * rg_oracle.c -- TEST INFRASTRUCTURE ONLY (see rg_oracle.h).
 *
 * Plain sequential FP64 reference of the scenario-based robust reference
 * governor.  Build: gcc -O2 -ffp-contract=off -std=c99 (no fast-math), so every
 * expression below is evaluated exactly as written, one IEEE rounding per
 * operation.  Threads (orc_problem.nthreads) only split the scenario loop of one
 * candidate evaluation; the minimum is order-free, so results do not depend on
 * the thread count.
 */
#define _POSIX_C_SOURCE 200809L
#include "rg_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ========================================================================= *
 * Random numbers.  The paper draws N_sim disturbance sequences d_j^k,
 * j = 0..j*, at every RG time step (Sec. II-C; Alg. 2 and Alg. 3 draw them once
 * and reuse them for every candidate kappa).  Reading: the draws are a pure
 * function of (seed, instance, t, k, j, component), produced by the
 * counter-based generator Philox4x32-10 of Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3" (SC'11), which the GPU library
 * implements separately from the same definition.
 * ========================================================================= */

/* Philox4x32 with 10 rounds, as defined by Salmon et al. (SC'11, Sec. 4.2):
 * each round multiplies counter words 0 and 2 by two fixed 32-bit multipliers,
 * forms the 64-bit products, and permutes/XORs the halves with the other words
 * and the round key; the key is advanced by the two Weyl increments between
 * rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t MUL0 = 0xD2511F53u, MUL1 = 0xCD9E8D57u;
    const uint32_t WEYL0 = 0x9E3779B9u, WEYL1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += WEYL0;
            k1 += WEYL1;
        }
        uint64_t p0 = (uint64_t)MUL0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)MUL1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Canonical uniform draw on [lo, hi): the top 24 bits of a Philox word give
 * u = (word >> 8) * 2^-24, exactly representable in binary32; the value is then
 * one correctly rounded binary32 fused multiply-add, fl32(span32 * u + lo32),
 * with lo32 = fl32(lo) and span32 = fl32(hi - lo).  Both the FP32 and FP64
 * computations consume this binary32 value, so they see identical inputs. */
float orc_uniform_box(uint32_t word, double lo, double hi)
{
    float u = (float)(word >> 8) * 0x1p-24f;
    float lo32 = (float)lo;
    float span32 = (float)(hi - lo);
    return fmaf(span32, u, lo32);
}

static void orc_counter_words(const orc_problem* p, uint32_t k, uint32_t j, uint32_t t,
                              uint32_t tag, uint32_t block, uint32_t out[4])
{
    uint32_t ctr[4] = {k, j, t, (tag << 16) | block};
    uint32_t key[2] = {p->seed, p->instance};
    orc_philox4x32_10(ctr, key, out);
}

/* Disturbance of scenario k at prediction step j of RG step t (tag 0). */
void orc_draw_w(const orc_problem* p, uint32_t t, uint32_t k, uint32_t j, double* w)
{
    uint32_t words[4];
    for (int c = 0; c < p->n_w; ++c) {
        if ((c & 3) == 0) orc_counter_words(p, k, j, t, 0u, (uint32_t)(c >> 2), words);
        w[c] = (double)orc_uniform_box(words[c & 3], p->w_lo[c], p->w_hi[c]);
    }
}

/* Uncertain coefficients of scenario k at RG step t (tag 1, j = 0):
 * theta^k = theta_nom * (1 + theta_rel * s), s uniform on [-1, 1); the factor
 * is the canonical binary32 draw on [1 - theta_rel, 1 + theta_rel). */
void orc_draw_theta(const orc_problem* p, uint32_t t, uint32_t k, double* theta)
{
    const double* nom = NULL;
    if (p->kind == ORC_FC9) nom = p->coeffs + 90;
    uint32_t words[4];
    for (int q = 0; q < p->n_theta; ++q) {
        if ((q & 3) == 0) orc_counter_words(p, k, 0u, t, 1u, (uint32_t)(q >> 2), words);
        double factor = (double)orc_uniform_box(words[q & 3], 1.0 - p->theta_rel,
                                                1.0 + p->theta_rel);
        theta[q] = nom[q] * factor;
    }
}

/* Disturbance acting on the true plant between RG steps t and t+1 (tag 2). */
void orc_draw_true_w(const orc_problem* p, uint32_t t, double* w)
{
    uint32_t words[4];
    for (int c = 0; c < p->n_w; ++c) {
        if ((c & 3) == 0) orc_counter_words(p, 0u, 0u, t, 2u, (uint32_t)(c >> 2), words);
        w[c] = (double)orc_uniform_box(words[c & 3], p->w_lo[c], p->w_hi[c]);
    }
}

/* ========================================================================= *
 * Plant.  The closed loop is x_{t+1} = f(x_t, v_t), y_t = h(x_t, v_t)
 * (Eq. (1)); the paper discretises its continuous-time model with fixed-step
 * fourth-order Runge-Kutta (Sec. IV-A).  Two synthetic closed loops stand in
 * for the paper's fuel-cell model, whose equations are not in the paper.
 * ========================================================================= */

/* LQ4: xdot = A x + B v + G (x .* x) + E w. */
static void lq4_rhs(const double* c, const double* x, double v, const double* w, double* xd)
{
    const double* A = c;
    const double* B = c + 16;
    const double* G = c + 20;
    const double* E = c + 36;
    for (int i = 0; i < 4; ++i) {
        double s = B[i] * v;
        for (int j = 0; j < 4; ++j) s += A[4 * i + j] * x[j];
        for (int j = 0; j < 4; ++j) s += G[4 * i + j] * (x[j] * x[j]);
        for (int j = 0; j < 2; ++j) s += E[2 * i + j] * w[j];
        xd[i] = s;
    }
}

/* FC9 (air-supply-like chain of six volumes p1..p6 fed by a compressor of
 * speed w1, an auxiliary speed w2 and a fast demand state w3):
 *   z = x - xbar, p7 = p_amb,
 *   q0 = c_q0 * w1,  q_l = k_l * sqrt(max(p_l - p_{l+1}, 0)), l = 1..6,
 *   xdot_i = -a_i z_i + sum_j W_ij tanh(z_j) + w_i + phi_i,
 *   phi_l = q_{l-1} - q_l (l = 1..6),
 *   phi_7 = b1 v - mu1 w1 (p1 - p1ref),  phi_8 = b2 v w1,
 *   phi_9 = b3 v - mu2 (w3 - 1) v.
 * theta = (a[9], k[6], b[3], mu[2]). */
static void fc9_rhs(const double* c, const double* th, const double* x, double v,
                    const double* w, double* xd)
{
    const double* W = c;
    const double* xbar = c + 81;
    const double c_q0 = c[110], p_amb = c[111], p1ref = c[114];
    const double* a = th;
    const double* kq = th + 9;
    const double* b = th + 15;
    const double* mu = th + 18;
    double z[9], s[9], q[7];
    for (int i = 0; i < 9; ++i) {
        z[i] = x[i] - xbar[i];
        s[i] = tanh(z[i]);
    }
    q[0] = c_q0 * x[6];
    for (int l = 0; l < 6; ++l) {
        double downstream = (l < 5) ? x[l + 1] : p_amb;
        double dp = x[l] - downstream;
        q[l + 1] = kq[l] * sqrt(dp > 0.0 ? dp : 0.0);
    }
    for (int i = 0; i < 9; ++i) {
        double acc = -a[i] * z[i];
        for (int j = 0; j < 9; ++j) acc += W[9 * i + j] * s[j];
        acc += w[i];
        double phi;
        if (i < 6) phi = q[i] - q[i + 1];
        else if (i == 6) phi = b[0] * v - mu[0] * x[6] * (x[0] - p1ref);
        else if (i == 7) phi = b[1] * v * x[6];
        else phi = b[2] * v - mu[1] * (x[8] - 1.0) * v;
        xd[i] = acc + phi;
    }
}

static const double* nominal_theta(const orc_problem* p)
{
    return (p->kind == ORC_FC9) ? p->coeffs + 90 : NULL;
}

void orc_rhs(const orc_problem* p, const double* theta, const double* x, double v,
             const double* w, double* xdot)
{
    if (p->kind == ORC_LQ4) lq4_rhs(p->coeffs, x, v, w, xdot);
    else fc9_rhs(p->coeffs, theta ? theta : nominal_theta(p), x, v, w, xdot);
}

/* Constrained outputs y = h(x, v).  LQ4: y = C x.  FC9: y1 = c_q0 w1 / (d0 + d1 w3)
 * (ratio of supplied flow to demand, kept above a floor like the paper's
 * oxygen excess ratio, Sec. IV-A), y2 = p1, y3 = w1. */
void orc_output(const orc_problem* p, const double* x, double v, double* y)
{
    if (p->kind == ORC_LQ4) {
        const double* C = p->coeffs + 44;
        for (int i = 0; i < 2; ++i) {
            double s = 0.0;
            for (int j = 0; j < 4; ++j) s += C[4 * i + j] * x[j];
            y[i] = s;
        }
    } else {
        const double* c = p->coeffs;
        (void)v;
        y[0] = c[110] * x[6] / (c[112] + c[113] * x[8]);
        y[1] = x[0];
        y[2] = x[6];
    }
}

/* Classical fourth-order Runge-Kutta step of length dt with v, w, theta held
 * over the step (Sec. IV-A: "4th order Runge Kutta", fixed step):
 *   k1 = f(x), k2 = f(x + dt/2 k1), k3 = f(x + dt/2 k2), k4 = f(x + dt k3),
 *   x+ = x + dt/6 (k1 + 2 k2 + 2 k3 + k4). */
void orc_rk4(const orc_problem* p, const double* theta, const double* x, double v,
             const double* w, double* xn)
{
    const int n = p->n;
    const double h = p->dt;
    double k1[ORC_MAXN], k2[ORC_MAXN], k3[ORC_MAXN], k4[ORC_MAXN], xs[ORC_MAXN];
    orc_rhs(p, theta, x, v, w, k1);
    for (int i = 0; i < n; ++i) xs[i] = x[i] + (h / 2.0) * k1[i];
    orc_rhs(p, theta, xs, v, w, k2);
    for (int i = 0; i < n; ++i) xs[i] = x[i] + (h / 2.0) * k2[i];
    orc_rhs(p, theta, xs, v, w, k3);
    for (int i = 0; i < n; ++i) xs[i] = x[i] + h * k3[i];
    orc_rhs(p, theta, xs, v, w, k4);
    for (int i = 0; i < n; ++i)
        xn[i] = x[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

/* One prediction step under disturbance w.  ORC_INJECT_ODE: w enters the
 * continuous dynamics, held over the step.  ORC_INJECT_POST: the literal
 * form of Eq. (4), x+ = f(x, v) + d with d = D w added after the step
 * (D = E for LQ4, the identity for FC9). */
void orc_step(const orc_problem* p, const double* theta, const double* x, double v,
              const double* w, double* xn)
{
    if (p->inject == ORC_INJECT_ODE) {
        orc_rk4(p, theta, x, v, w, xn);
        return;
    }
    double zero[ORC_MAXW] = {0};
    orc_rk4(p, theta, x, v, zero, xn);
    if (p->kind == ORC_LQ4) {
        const double* E = p->coeffs + 36;
        for (int i = 0; i < 4; ++i) xn[i] = xn[i] + (E[2 * i] * w[0] + E[2 * i + 1] * w[1]);
    } else {
        for (int i = 0; i < p->n; ++i) xn[i] = xn[i] + w[i];
    }
}

/* Constraint margin of y for Y = {y : F y <= g} (Sec. II-A: y_t in Y, Y convex):
 * m = min_r (g_r - F_r y); m >= 0 iff y in Y.  r_arg = first minimising row. */
double orc_margin(const orc_problem* p, const double* y, int32_t* r_arg)
{
    double best = INFINITY;
    int32_t arg = 0;
    for (int r = 0; r < p->n_c; ++r) {
        double fy = 0.0;
        for (int i = 0; i < p->n_y; ++i) fy += p->F[r * p->n_y + i] * y[i];
        double m = p->g[r] - fy;
        if (isnan(m)) m = -INFINITY;
        if (r == 0 || m < best) {
            best = m;
            arg = r;
        }
    }
    if (r_arg) *r_arg = arg;
    return best;
}

/* ========================================================================= *
 * Prediction and verdict (Eq. (3); the candidate test of Alg. 1; the parallel evaluation of Alg. 3).
 * ========================================================================= */

/* Candidate set-point, Eq. (2): v = v_{t-1} + kappa (r_t - v_{t-1}).
 * Reading: at kappa = 1 the candidate is r_t itself (Alg. 1 stops there). */
double orc_candidate_v(double kappa, double r, double v_prev)
{
    if (kappa == 1.0) return r;
    return v_prev + kappa * (r - v_prev);
}

static int all_finite(const double* x, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

/* Worst constraint margin of one scenario rollout: xhat_0 = x_t,
 * xhat_{j+1} = step(xhat_j, v, d_j^k), margins checked at j = 0..j* (Eq. (3)
 * constraint rows; Alg. 3 parallel step 2-3).  Returns min_j m_j with the
 * first minimising (j, r); a non-finite state or margin returns -inf at the
 * first such j.  traj (nullable) receives the (H+1) x n states. */
double orc_rollout(const orc_problem* p, const double* x0, double v, uint32_t t, uint32_t k,
                   int32_t* j_arg, int32_t* r_arg, double* traj)
{
    const int n = p->n;
    double x[ORC_MAXN], xn[ORC_MAXN], y[ORC_MAXY], w[ORC_MAXW], theta[ORC_MAXTH];
    if (p->n_theta > 0) orc_draw_theta(p, t, k, theta);
    memcpy(x, x0, sizeof(double) * (size_t)n);
    double best = INFINITY;
    int32_t bj = 0, br = 0;
    for (int32_t j = 0; j <= p->H; ++j) {
        if (traj) memcpy(traj + (size_t)j * (size_t)n, x, sizeof(double) * (size_t)n);
        int32_t r = 0;
        double m;
        if (!all_finite(x, n)) {
            m = -INFINITY;
        } else {
            orc_output(p, x, v, y);
            m = orc_margin(p, y, &r);
            if (!isfinite(m) && m != INFINITY) m = -INFINITY;
        }
        if (m < best || j == 0) {
            best = m;
            bj = j;
            br = r;
        }
        if (best == -INFINITY) break;
        if (j == p->H) break;
        orc_draw_w(p, t, k, (uint32_t)j, w);
        orc_step(p, theta, x, v, w, xn);
        memcpy(x, xn, sizeof(double) * (size_t)n);
    }
    if (j_arg) *j_arg = bj;
    if (r_arg) *r_arg = br;
    return best;
}

/* Dense solve of J d = b by Gaussian elimination with partial pivoting.
 * Returns 0 on success, -1 if a pivot vanishes. */
static int dense_solve(int n, double* J, double* b)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(J[r * n + c]) > fabs(J[piv * n + c])) piv = r;
        if (!(fabs(J[piv * n + c]) > 1e-300)) return -1;
        if (piv != c) {
            for (int q = 0; q < n; ++q) {
                double tmp = J[c * n + q];
                J[c * n + q] = J[piv * n + q];
                J[piv * n + q] = tmp;
            }
            double tmp = b[c];
            b[c] = b[piv];
            b[piv] = tmp;
        }
        for (int r = c + 1; r < n; ++r) {
            double f = J[r * n + c] / J[c * n + c];
            for (int q = c; q < n; ++q) J[r * n + q] -= f * J[c * n + q];
            b[r] -= f * b[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        double s = b[c];
        for (int q = c + 1; q < n; ++q) s -= J[c * n + q] * b[q];
        b[c] = s / J[c * n + c];
    }
    return 0;
}

/* Jacobian df/dx of the continuous dynamics at (x, v), nominal theta, w = 0. */
static void orc_jacobian(const orc_problem* p, const double* x, double v, double* J)
{
    if (p->kind == ORC_LQ4) {
        const double* A = p->coeffs;
        const double* G = p->coeffs + 20;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) J[4 * i + j] = A[4 * i + j] + 2.0 * G[4 * i + j] * x[j];
        return;
    }
    const double* c = p->coeffs;
    const double* W = c;
    const double* xbar = c + 81;
    const double* th = c + 90;
    const double* a = th;
    const double* kq = th + 9;
    const double* b = th + 15;
    const double* mu = th + 18;
    const double c_q0 = c[110], p_amb = c[111], p1ref = c[114];
    (void)b;
    for (int i = 0; i < 9; ++i) {
        for (int j = 0; j < 9; ++j) {
            double sj = tanh(x[j] - xbar[j]);
            J[9 * i + j] = W[9 * i + j] * (1.0 - sj * sj);
        }
        J[9 * i + i] += -a[i];
    }
    /* dq_l/dp: q_l = k_l sqrt(max(dp_l, 0)); derivative 0 where dp_l <= 0. */
    double dq_up[6], dq_dn[6];
    for (int l = 0; l < 6; ++l) {
        double downstream = (l < 5) ? x[l + 1] : p_amb;
        double dp = x[l] - downstream;
        double d = (dp > 0.0) ? kq[l] / (2.0 * sqrt(dp)) : 0.0;
        dq_up[l] = d;   /* d q_{l+1} / d p_l       */
        dq_dn[l] = -d;  /* d q_{l+1} / d p_{l+1}   */
    }
    /* phi_1 = q0 - q1; phi_l = q_{l-1} - q_l */
    J[9 * 0 + 6] += c_q0;
    for (int l = 0; l < 6; ++l) {
        /* -q_{l+1} in phi_l */
        J[9 * l + l] += -dq_up[l];
        if (l < 5) J[9 * l + (l + 1)] += -dq_dn[l];
        /* +q_{l+1} in phi_{l+1} */
        if (l < 5) {
            J[9 * (l + 1) + l] += dq_up[l];
            J[9 * (l + 1) + (l + 1)] += dq_dn[l];
        }
    }
    /* phi_7 = b1 v - mu1 w1 (p1 - p1ref) */
    J[9 * 6 + 6] += -mu[0] * (x[0] - p1ref);
    J[9 * 6 + 0] += -mu[0] * x[6];
    /* phi_8 = b2 v w1 */
    J[9 * 7 + 6] += b[1] * v;
    /* phi_9 = b3 v - mu2 (w3 - 1) v */
    J[9 * 8 + 8] += -mu[1] * v;
}

/* Tightened steady-state test (Sec. II-A): y_ss(v) in (1 - eps) Y.  The
 * equilibrium manifold is "assumed known"; reading: y_ss(v) = h(x_ss, v) with
 * x_ss the equilibrium f(x_ss, v, w = 0, theta_nom) = 0 reached by Newton's
 * method from x = -A^{-1} B v (LQ4, the linear part's DC solution) or x = xbar
 * (FC9), stopped at ||f||_inf <= 1e-12 within 50 iterations; failure gives
 * -inf.  (1 - eps) Y is read row-wise as g_r - eps |g_r| - F_r y >= 0, which
 * equals (1 - eps) g_r - F_r y whenever 0 is in Y.  ss_check = 0 returns +inf. */
double orc_steady_margin(const orc_problem* p, double v, double* x_ss, int32_t* iters)
{
    const int n = p->n;
    double x[ORC_MAXN], f[ORC_MAXN], J[ORC_MAXN * ORC_MAXN], zero[ORC_MAXW] = {0};
    if (iters) *iters = 0;
    if (!p->ss_check) return INFINITY;
    if (p->kind == ORC_LQ4) {
        double A[16];
        memcpy(A, p->coeffs, sizeof A);
        for (int i = 0; i < 4; ++i) x[i] = -(p->coeffs[16 + i] * v);
        if (dense_solve(4, A, x) != 0) return -INFINITY;
    } else {
        memcpy(x, p->coeffs + 81, sizeof(double) * 9);
    }
    int converged = 0;
    for (int it = 0; it <= 50; ++it) {
        orc_rhs(p, NULL, x, v, zero, f);
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) {
            if (!isfinite(f[i])) return -INFINITY;
            if (fabs(f[i]) > nrm) nrm = fabs(f[i]);
        }
        if (nrm <= 1e-12) {
            converged = 1;
            if (iters) *iters = it;
            break;
        }
        if (it == 50) break;
        orc_jacobian(p, x, v, J);
        for (int i = 0; i < n; ++i) f[i] = -f[i];
        if (dense_solve(n, J, f) != 0) return -INFINITY;
        for (int i = 0; i < n; ++i) x[i] += f[i];
    }
    if (!converged) return -INFINITY;
    if (x_ss) memcpy(x_ss, x, sizeof(double) * (size_t)n);
    double y[ORC_MAXY];
    orc_output(p, x, v, y);
    double best = INFINITY;
    for (int r = 0; r < p->n_c; ++r) {
        double fy = 0.0;
        for (int i = 0; i < p->n_y; ++i) fy += p->F[r * p->n_y + i] * y[i];
        double m = (p->g[r] - p->eps * fabs(p->g[r])) - fy;
        if (isnan(m)) m = -INFINITY;
        if (m < best) best = m;
    }
    return best;
}

typedef struct {
    const orc_problem* p;
    const double* x0;
    double v;
    uint32_t t;
    int32_t k_begin, k_end;
    double* per_scen;
} orc_chunk;

static void* orc_chunk_run(void* arg)
{
    orc_chunk* c = (orc_chunk*)arg;
    for (int32_t k = c->k_begin; k < c->k_end; ++k)
        c->per_scen[k] = orc_rollout(c->p, c->x0, c->v, c->t, (uint32_t)k, NULL, NULL, NULL);
    return NULL;
}

/* Candidate worst margin M(v) = min( min_k m^k(v), m_ss(v) ); the candidate is
 * admissible iff M(v) >= 0 (the verdict of Alg. 2 and of Alg. 3: robust means
 * every sampled scenario).  per_scen (nullable) receives m^k; k_arg the first
 * minimising scenario; m_ss_out the steady-state margin. */
double orc_candidate(const orc_problem* p, const double* x0, double v, uint32_t t,
                     double* per_scen, int32_t* k_arg, double* m_ss_out)
{
    const int32_t N = p->N;
    double* m = per_scen;
    double* owned = NULL;
    if (!m) {
        owned = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
        m = owned;
    }
    int T = p->nthreads > 1 ? p->nthreads : 1;
    if (T > N) T = N > 0 ? N : 1;
    if (T == 1) {
        for (int32_t k = 0; k < N; ++k)
            m[k] = orc_rollout(p, x0, v, t, (uint32_t)k, NULL, NULL, NULL);
    } else {
        pthread_t th[256];
        orc_chunk ch[256];
        if (T > 256) T = 256;
        for (int i = 0; i < T; ++i) {
            ch[i].p = p; ch[i].x0 = x0; ch[i].v = v; ch[i].t = t;
            ch[i].k_begin = (int32_t)(((int64_t)N * i) / T);
            ch[i].k_end = (int32_t)(((int64_t)N * (i + 1)) / T);
            ch[i].per_scen = m;
            pthread_create(&th[i], NULL, orc_chunk_run, &ch[i]);
        }
        for (int i = 0; i < T; ++i) pthread_join(th[i], NULL);
    }
    double worst = INFINITY;
    int32_t ka = 0;
    for (int32_t k = 0; k < N; ++k) {
        if (k == 0 || m[k] < worst) {
            worst = m[k];
            ka = k;
        }
    }
    double mss = orc_steady_margin(p, v, NULL, NULL);
    if (m_ss_out) *m_ss_out = mss;
    if (k_arg) *k_arg = ka;
    free(owned);
    return worst < mss ? worst : mss;
}

/* ========================================================================= *
 * Kappa searches.
 * ========================================================================= */

/* Alg. 1 (bisection) on the robust verdict M(v) >= 0 over all scenarios.
 * Definition used here: the search first asks whether kappa = 1 is admissible
 * and returns it if so.  Otherwise it holds a bracket [lo, hi] with hi refused
 * and lo the largest admissible candidate found so far (0, not evaluated, at
 * the start) and halves it K times at its midpoint, keeping that property; the
 * result is lo.  At most K + 1 candidate evaluations, and the bracket closes to
 * 2^-K (reading of the iteration count: K counts the halvings after the
 * kappa = 1 probe).  Alg. 2 computes the same value when feasibility is
 * monotone in kappa (the minimum over scenarios commutes with the dyadic
 * floor); orc_alg2 is the per-scenario form.  trace_* (nullable) receive the
 * evaluated candidates and their worst margins in order. */
orc_result orc_bisect(const orc_problem* p, const double* x0, double r, double v_prev,
                      uint32_t t, int32_t K, double* trace_kappa, double* trace_margin)
{
    orc_result res = {0.0, v_prev, -INFINITY, 0, 1};
    double M = orc_candidate(p, x0, orc_candidate_v(1.0, r, v_prev), t, NULL, NULL, NULL);
    if (trace_kappa) trace_kappa[0] = 1.0;
    if (trace_margin) trace_margin[0] = M;
    res.passes = 1;
    if (M >= 0.0) {
        res.kappa = 1.0;
        res.v = r;
        res.worst = M;
        res.status = 0;
        return res;
    }
    double lo = 0.0, hi = 1.0;
    for (int32_t h = 0; h < K; ++h) {
        const double mid = (lo + hi) / 2.0;
        M = orc_candidate(p, x0, orc_candidate_v(mid, r, v_prev), t, NULL, NULL, NULL);
        if (trace_kappa) trace_kappa[res.passes] = mid;
        if (trace_margin) trace_margin[res.passes] = M;
        res.passes += 1;
        if (M >= 0.0) {
            lo = mid;
            res.worst = M;
            res.status = 0;
        } else {
            hi = mid;
        }
    }
    res.kappa = res.status == 0 ? lo : 0.0;
    res.v = res.status == 0 ? orc_candidate_v(lo, r, v_prev) : v_prev;
    return res;
}

/* Verdict of one scenario alone (Alg. 2 runs Alg. 1 once per scenario): its
 * rollout margin and the steady-state margin both non-negative. */
static int orc_scenario_admits(const orc_problem* p, const double* x0, double v, uint32_t t,
                               uint32_t k)
{
    const double mk = orc_rollout(p, x0, v, t, k, NULL, NULL, NULL);
    const double ms = orc_steady_margin(p, v, NULL, NULL);
    return mk >= 0.0 && ms >= 0.0;
}

/* Alg. 2: the bisection defined at orc_bisect applied to each scenario's own
 * verdict, then the smallest of the per-scenario results.  A scenario with no
 * admissible candidate contributes 0 and makes the status 1 (kappa = 0,
 * v = v_prev) when the minimum is 0. */
orc_result orc_alg2(const orc_problem* p, const double* x0, double r, double v_prev,
                    uint32_t t, int32_t K)
{
    orc_result res = {1.0, r, -INFINITY, 0, 0};
    double kmin = 1.0;
    int any_none = 0;
    for (int32_t k = 0; k < p->N; ++k) {
        double kk;
        res.passes += 1;
        if (orc_scenario_admits(p, x0, orc_candidate_v(1.0, r, v_prev), t, (uint32_t)k)) {
            kk = 1.0;
        } else {
            double lo = 0.0, hi = 1.0;
            int found = 0;
            for (int32_t h = 0; h < K; ++h) {
                const double mid = (lo + hi) / 2.0;
                res.passes += 1;
                if (orc_scenario_admits(p, x0, orc_candidate_v(mid, r, v_prev), t, (uint32_t)k)) {
                    lo = mid;
                    found = 1;
                } else {
                    hi = mid;
                }
            }
            if (!found) any_none = 1;
            kk = lo;
        }
        if (kk < kmin) kmin = kk;
    }
    res.kappa = kmin;
    res.status = (kmin == 0.0 && any_none) ? 1 : 0;
    res.v = res.status ? v_prev : orc_candidate_v(kmin, r, v_prev);
    return res;
}

/* Alg. 3 / Eq. (5): grid kappa_i = (i-1)/(M-1), P_ik = 1 iff scenario k and
 * the steady-state test admit kappa_i, i* = the largest row of all ones (even
 * if a smaller row fails), kappa_opt = kappa_{i*}; then `refine` bisection
 * halvings inside [kappa_{i*}, kappa_{i*+1}] (0 for the plain Alg. 3).  No
 * admissible row returns kappa = 0 with status 1.  Pmat (nullable) receives the
 * M x N boolean array P. */
orc_result orc_grid(const orc_problem* p, const double* x0, double r, double v_prev,
                    uint32_t t, int32_t M, int32_t refine, uint8_t* Pmat)
{
    orc_result res = {0.0, v_prev, -INFINITY, 0, 1};
    double* m = (double*)malloc(sizeof(double) * (size_t)(p->N > 0 ? p->N : 1));
    int32_t istar = -1;
    double worst_star = -INFINITY;
    for (int32_t i = 0; i < M; ++i) {
        double kappa = (M > 1) ? (double)i / (double)(M - 1) : 1.0;
        double v = orc_candidate_v(kappa, r, v_prev);
        double mss = 0.0;
        double W = orc_candidate(p, x0, v, t, m, NULL, &mss);
        res.passes++;
        int row_ok = 1;
        for (int32_t k = 0; k < p->N; ++k) {
            int ok = (m[k] >= 0.0 && mss >= 0.0);
            if (Pmat) Pmat[(size_t)i * (size_t)p->N + (size_t)k] = (uint8_t)ok;
            if (!ok) row_ok = 0;
        }
        if (p->N == 0 && !(mss >= 0.0)) row_ok = 0;
        if (row_ok) {
            istar = i;
            worst_star = W;
        }
    }
    free(m);
    if (istar < 0) return res;
    double kappa = (M > 1) ? (double)istar / (double)(M - 1) : 1.0;
    double worst = worst_star;
    if (istar < M - 1 && refine > 0) {
        double lo = kappa, hi = (double)(istar + 1) / (double)(M - 1);
        for (int32_t s = 0; s < refine; ++s) {
            double mid = (lo + hi) / 2.0;
            double W = orc_candidate(p, x0, orc_candidate_v(mid, r, v_prev), t, NULL, NULL, NULL);
            res.passes++;
            if (W >= 0.0) {
                lo = mid;
                worst = W;
            } else {
                hi = mid;
            }
        }
        kappa = lo;
    }
    res.kappa = kappa;
    res.v = orc_candidate_v(kappa, r, v_prev);
    res.worst = worst;
    res.status = 0;
    return res;
}

/* ========================================================================= *
 * Chance-constrained verdict (scenario approach with discarded scenarios).
 * Sec. II-C builds the robust governor on N sampled disturbance sequences and
 * states its guarantee probabilistically; the scenario method it draws on also
 * allows a candidate whose predictions leave Y in a few of the samples.  Reading
 * used here: a candidate is admissible when the steady-state test passes and at
 * most q of the N scenario rollouts violate (m^k < 0).  Its worst margin is
 * M_q(v) = min(m_(q+1), m_ss), with m_(q+1) the (q+1)-th smallest scenario
 * margin (order statistic, +inf when q >= N), so that admissible <=> M_q >= 0
 * and q = 0 is the robust verdict.
 * ========================================================================= */

static int orc_cmp_double(const void* a, const void* b)
{
    const double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* M_q(v); n_viol (nullable) receives the number of scenarios with m^k < 0. */
double orc_candidate_q(const orc_problem* p, const double* x0, double v, uint32_t t, int32_t q,
                       double* per_scen, int32_t* n_viol)
{
    const int32_t N = p->N;
    double* m = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double mss = 0.0;
    orc_candidate(p, x0, v, t, m, NULL, &mss);
    int32_t viol = 0;
    for (int32_t k = 0; k < N; ++k) {
        if (per_scen) per_scen[k] = m[k];
        if (m[k] < 0.0) viol++;
    }
    qsort(m, (size_t)N, sizeof(double), orc_cmp_double);
    const double mq = (q < N) ? m[q] : INFINITY;
    free(m);
    if (n_viol) *n_viol = viol;
    return mq < mss ? mq : mss;
}

/* Alg. 1 (as defined at orc_bisect) on the chance-constrained verdict M_q >= 0. */
orc_result orc_bisect_q(const orc_problem* p, const double* x0, double r, double v_prev,
                        uint32_t t, int32_t K, int32_t q)
{
    orc_result res = {0.0, v_prev, -INFINITY, 0, 1};
    double M = orc_candidate_q(p, x0, orc_candidate_v(1.0, r, v_prev), t, q, NULL, NULL);
    res.passes = 1;
    if (M >= 0.0) {
        res.kappa = 1.0;
        res.v = r;
        res.worst = M;
        res.status = 0;
        return res;
    }
    double lo = 0.0, hi = 1.0;
    for (int32_t h = 0; h < K; ++h) {
        const double mid = (lo + hi) / 2.0;
        M = orc_candidate_q(p, x0, orc_candidate_v(mid, r, v_prev), t, q, NULL, NULL);
        res.passes += 1;
        if (M >= 0.0) {
            lo = mid;
            res.worst = M;
            res.status = 0;
        } else {
            hi = mid;
        }
    }
    res.kappa = res.status == 0 ? lo : 0.0;
    res.v = res.status == 0 ? orc_candidate_v(lo, r, v_prev) : v_prev;
    return res;
}

/* ========================================================================= *
 * Closed loop (Fig. 1): the RG picks v_t from (x_t, v_{t-1}, r_t), the plant
 * advances one step under v_t and the true disturbance (Eq. (4)).
 * ========================================================================= */

/* True plant: one step of the nominal model under the tag-2 disturbance. */
void orc_plant_step(const orc_problem* p, const double* x, double v, uint32_t t, double* xn)
{
    double w[ORC_MAXW];
    orc_draw_true_w(p, t, w);
    orc_step(p, NULL, x, v, w, xn);
}

/* T closed-loop steps from (x0, v0) at RG step t0.  search: 0 = bisection
 * (K halvings), 1 = grid (M points, `refine` halvings), 2 = Alg. 2.  x_out
 * receives (T+1) x n states.  Returns the number of steps whose search found
 * no admissible candidate. */
int32_t orc_closed_loop(const orc_problem* p, const double* x0, double v0, const double* r_seq,
                        int32_t T, uint32_t t0, int32_t search, int32_t K, int32_t M,
                        int32_t refine, double* v_out, double* kappa_out, double* x_out)
{
    const int n = p->n;
    double x[ORC_MAXN], xn[ORC_MAXN];
    memcpy(x, x0, sizeof(double) * (size_t)n);
    if (x_out) memcpy(x_out, x, sizeof(double) * (size_t)n);
    double v_prev = v0;
    int32_t infeasible = 0;
    for (int32_t s = 0; s < T; ++s) {
        uint32_t t = t0 + (uint32_t)s;
        orc_result res;
        if (search == 1) res = orc_grid(p, x, r_seq[s], v_prev, t, M, refine, NULL);
        else if (search == 2) res = orc_alg2(p, x, r_seq[s], v_prev, t, K);
        else res = orc_bisect(p, x, r_seq[s], v_prev, t, K, NULL, NULL);
        if (res.status) infeasible++;
        if (v_out) v_out[s] = res.v;
        if (kappa_out) kappa_out[s] = res.kappa;
        orc_plant_step(p, x, res.v, t, xn);
        memcpy(x, xn, sizeof(double) * (size_t)n);
        if (x_out) memcpy(x_out + (size_t)(s + 1) * (size_t)n, x, sizeof(double) * (size_t)n);
        v_prev = res.v;
    }
    return infeasible;
}

/* ========================================================================= *
 * Sensitivities (not in the paper; they back the adjoint/Newton search).
 * Forward-mode tangents of the discrete RK4 map, propagated alongside the
 * state: S_v = dx/dv and S_p = dx/dtheta_p (theta = the scenario's
 * coefficients).  The margin's derivative is that of the minimising term
 * (j*, r*) (first minimiser on ties); d/dtheta_nom = d/dtheta * factor_p.
 * ========================================================================= */

/* df/dx at (x, v, theta); w enters additively and drops out. */
static void orc_jac_theta(const orc_problem* p, const double* th, const double* x, double v,
                          double* J)
{
    if (p->kind == ORC_LQ4) {
        orc_jacobian(p, x, v, J);
        return;
    }
    /* FC9 with the scenario's theta: same structure as orc_jacobian. */
    orc_problem q = *p;
    for (int i = 0; i < 20; ++i) q.coeffs[90 + i] = th[i];
    orc_jacobian(&q, x, v, J);
}

/* df/dv at (x, v, theta). */
static void orc_dfdv(const orc_problem* p, const double* th, const double* x, double* fv)
{
    if (p->kind == ORC_LQ4) {
        for (int i = 0; i < 4; ++i) fv[i] = p->coeffs[16 + i];
        return;
    }
    const double* b = th + 15;
    const double* mu = th + 18;
    for (int i = 0; i < 9; ++i) fv[i] = 0.0;
    fv[6] = b[0];
    fv[7] = b[1] * x[6];
    fv[8] = b[2] - mu[1] * (x[8] - 1.0);
}

/* df/dtheta (n x n_theta, row-major) at (x, v, theta); FC9 only. */
static void orc_dfdtheta(const orc_problem* p, const double* th, const double* x, double v,
                         double* Ft)
{
    const int n = p->n, nt = p->n_theta;
    for (int i = 0; i < n * nt; ++i) Ft[i] = 0.0;
    if (p->kind != ORC_FC9) return;
    (void)th;
    const double* xbar = p->coeffs + 81;
    const double p_amb = p->coeffs[111], p1ref = p->coeffs[114];
    for (int i = 0; i < 9; ++i) Ft[i * nt + i] = -(x[i] - xbar[i]);          /* a_i */
    for (int l = 0; l < 6; ++l) {                                            /* k_l */
        double downstream = (l < 5) ? x[l + 1] : p_amb;
        double dp = x[l] - downstream;
        double s = sqrt(dp > 0.0 ? dp : 0.0);
        Ft[l * nt + 9 + l] += -s;
        if (l < 5) Ft[(l + 1) * nt + 9 + l] += s;
    }
    Ft[6 * nt + 15] = v;                          /* b1 */
    Ft[7 * nt + 16] = v * x[6];                   /* b2 */
    Ft[8 * nt + 17] = v;                          /* b3 */
    Ft[6 * nt + 18] = -x[6] * (x[0] - p1ref);     /* mu1 */
    Ft[8 * nt + 19] = -(x[8] - 1.0) * v;          /* mu2 */
}

/* dy/dx (n_y x n) at x; the outputs of both plants do not depend on v. */
static void orc_dhdx(const orc_problem* p, const double* x, double* Hx)
{
    const int n = p->n;
    for (int i = 0; i < p->n_y * n; ++i) Hx[i] = 0.0;
    if (p->kind == ORC_LQ4) {
        for (int i = 0; i < 8; ++i) Hx[i] = p->coeffs[44 + i];
        return;
    }
    const double* c = p->coeffs;
    double den = c[112] + c[113] * x[8];
    Hx[0 * n + 6] = c[110] / den;
    Hx[0 * n + 8] = -c[110] * x[6] * c[113] / (den * den);
    Hx[1 * n + 0] = 1.0;
    Hx[2 * n + 6] = 1.0;
}

/* Tangent of one RK4 step: given x and tangent columns T (n x m), advance both. */
static void orc_rk4_tangent(const orc_problem* p, const double* th, const double* x, double v,
                            const double* w, double* T, int m, const double* T_force,
                            double* xn)
{
    /* T_force(xs) supplies df/dparam at the stage state: column 0 = d/dv, columns
     * 1.. = d/dtheta; recomputed inside for each stage. */
    (void)T_force;
    const int n = p->n;
    const double h = p->dt;
    double xs[ORC_MAXN], k[4][ORC_MAXN];
    double dk[4][ORC_MAXN * (1 + ORC_MAXTH)];
    double dxs[ORC_MAXN * (1 + ORC_MAXTH)];
    double J[ORC_MAXN * ORC_MAXN], fv[ORC_MAXN], Ft[ORC_MAXN * ORC_MAXTH];
    const double c[4] = {0.0, 0.5, 0.5, 1.0};
    double zero[ORC_MAXW] = {0};
    const double* wu = (p->inject == ORC_INJECT_ODE) ? w : zero;
    for (int s = 0; s < 4; ++s) {
        for (int i = 0; i < n; ++i) xs[i] = (s == 0) ? x[i] : x[i] + (c[s] * h) * k[s - 1][i];
        for (int i = 0; i < n * m; ++i)
            dxs[i] = (s == 0) ? T[i] : T[i] + (c[s] * h) * dk[s - 1][i];
        orc_rhs(p, th, xs, v, wu, k[s]);
        orc_jac_theta(p, th, xs, v, J);
        orc_dfdv(p, th, xs, fv);
        orc_dfdtheta(p, th, xs, v, Ft);
        for (int i = 0; i < n; ++i) {
            for (int col = 0; col < m; ++col) {
                double acc = 0.0;
                for (int q = 0; q < n; ++q) acc += J[i * n + q] * dxs[q * m + col];
                if (col == 0) acc += fv[i];
                else acc += Ft[i * p->n_theta + (col - 1)];
                dk[s][i * m + col] = acc;
            }
        }
    }
    for (int i = 0; i < n; ++i)
        xn[i] = x[i] + (h / 6.0) * (k[0][i] + 2.0 * k[1][i] + 2.0 * k[2][i] + k[3][i]);
    for (int i = 0; i < n * m; ++i)
        T[i] = T[i] + (h / 6.0) * (dk[0][i] + 2.0 * dk[1][i] + 2.0 * dk[2][i] + dk[3][i]);
    if (p->inject == ORC_INJECT_POST) {
        if (p->kind == ORC_LQ4) {
            const double* E = p->coeffs + 36;
            for (int i = 0; i < 4; ++i) xn[i] = xn[i] + (E[2 * i] * w[0] + E[2 * i + 1] * w[1]);
        } else {
            for (int i = 0; i < n; ++i) xn[i] = xn[i] + w[i];
        }
    }
}

/* Worst margin of scenario k with its derivatives: dm/dv and dm/dtheta_nom
 * (n_theta values; zero-length for LQ4).  Same margin, minimiser and
 * non-finite rules as orc_rollout. */
double orc_rollout_tangent(const orc_problem* p, const double* x0, double v, uint32_t t,
                           uint32_t k, double* dm_dv, double* dm_dtheta_nom,
                           int32_t* j_arg, int32_t* r_arg)
{
    const int n = p->n, nt = p->n_theta, m = 1 + nt;
    double x[ORC_MAXN], xn[ORC_MAXN], y[ORC_MAXY], w[ORC_MAXW], theta[ORC_MAXTH];
    double T[ORC_MAXN * (1 + ORC_MAXTH)] = {0};
    double Hx[ORC_MAXY * ORC_MAXN];
    double factor[ORC_MAXTH];
    if (nt > 0) {
        orc_draw_theta(p, t, k, theta);
        for (int q = 0; q < nt; ++q) factor[q] = theta[q] / p->coeffs[90 + q];
    }
    memcpy(x, x0, sizeof(double) * (size_t)n);
    double best = INFINITY;
    double best_dv = 0.0, best_dth[ORC_MAXTH] = {0};
    int32_t bj = 0, br = 0;
    for (int32_t j = 0; j <= p->H; ++j) {
        int32_t r = 0;
        double mj;
        if (!all_finite(x, n)) {
            mj = -INFINITY;
        } else {
            orc_output(p, x, v, y);
            mj = orc_margin(p, y, &r);
            if (!isfinite(mj) && mj != INFINITY) mj = -INFINITY;
        }
        if (mj < best || j == 0) {
            best = mj;
            bj = j;
            br = r;
            /* dm_j/d. = -F_r Hx dx/d. */
            orc_dhdx(p, x, Hx);
            double g[ORC_MAXN];
            for (int i = 0; i < n; ++i) {
                double a = 0.0;
                for (int yy = 0; yy < p->n_y; ++yy) a += p->F[r * p->n_y + yy] * Hx[yy * n + i];
                g[i] = -a;
            }
            best_dv = 0.0;
            for (int i = 0; i < n; ++i) best_dv += g[i] * T[i * m + 0];
            for (int q = 0; q < nt; ++q) {
                double a = 0.0;
                for (int i = 0; i < n; ++i) a += g[i] * T[i * m + 1 + q];
                best_dth[q] = a;
            }
        }
        if (best == -INFINITY) break;
        if (j == p->H) break;
        orc_draw_w(p, t, k, (uint32_t)j, w);
        orc_rk4_tangent(p, nt > 0 ? theta : NULL, x, v, w, T, m, NULL, xn);
        memcpy(x, xn, sizeof(double) * (size_t)n);
    }
    if (dm_dv) *dm_dv = best_dv;
    if (dm_dtheta_nom)
        for (int q = 0; q < nt; ++q) dm_dtheta_nom[q] = best_dth[q] * factor[q];
    if (j_arg) *j_arg = bj;
    if (r_arg) *r_arg = br;
    return best;
}

/* Steady-state margin with its derivatives by the implicit function theorem:
 * f(x_ss, v, theta_nom) = 0 => dx_ss/d. = -J^{-1} df/d. */
double orc_steady_tangent(const orc_problem* p, double v, double* dmss_dv, double* dmss_dtheta)
{
    const int n = p->n, nt = p->n_theta;
    double xs[ORC_MAXN];
    double mss = orc_steady_margin(p, v, xs, NULL);
    if (dmss_dv) *dmss_dv = 0.0;
    if (dmss_dtheta)
        for (int q = 0; q < nt; ++q) dmss_dtheta[q] = 0.0;
    if (!isfinite(mss)) return mss;
    const double* thn = nominal_theta(p);
    double J[ORC_MAXN * ORC_MAXN], rhs[ORC_MAXN], fv[ORC_MAXN], Ft[ORC_MAXN * ORC_MAXTH];
    double y[ORC_MAXY], Hx[ORC_MAXY * ORC_MAXN];
    orc_output(p, xs, v, y);
    int r_arg = 0;
    double best = INFINITY;
    for (int r = 0; r < p->n_c; ++r) {
        double fy = 0.0;
        for (int i = 0; i < p->n_y; ++i) fy += p->F[r * p->n_y + i] * y[i];
        double m = (p->g[r] - p->eps * fabs(p->g[r])) - fy;
        if (r == 0 || m < best) {
            best = m;
            r_arg = r;
        }
    }
    orc_dhdx(p, xs, Hx);
    double gr[ORC_MAXN];
    for (int i = 0; i < n; ++i) {
        double a = 0.0;
        for (int yy = 0; yy < p->n_y; ++yy) a += p->F[r_arg * p->n_y + yy] * Hx[yy * n + i];
        gr[i] = -a;
    }
    orc_dfdv(p, thn, xs, fv);
    orc_dfdtheta(p, thn, xs, v, Ft);
    /* dx/dv */
    orc_jacobian(p, xs, v, J);
    for (int i = 0; i < n; ++i) rhs[i] = -fv[i];
    if (dense_solve(n, J, rhs) != 0) return mss;
    double dv = 0.0;
    for (int i = 0; i < n; ++i) dv += gr[i] * rhs[i];
    if (dmss_dv) *dmss_dv = dv;
    if (dmss_dtheta) {
        for (int q = 0; q < nt; ++q) {
            orc_jacobian(p, xs, v, J);
            for (int i = 0; i < n; ++i) rhs[i] = -Ft[i * nt + q];
            if (dense_solve(n, J, rhs) != 0) return mss;
            double a = 0.0;
            for (int i = 0; i < n; ++i) a += gr[i] * rhs[i];
            dmss_dtheta[q] = a;
        }
    }
    return mss;
}

/* Candidate worst margin M(kappa) with dM/dkappa and dM/dtheta_nom: the
 * derivative of the active term (the first minimising scenario, or the
 * steady-state margin when it is the smaller).  dv/dkappa = r - v_prev. */
double orc_candidate_grad(const orc_problem* p, const double* x0, double kappa, double r,
                          double v_prev, uint32_t t, double* dM_dkappa, double* dM_dtheta,
                          int32_t* k_arg)
{
    const int nt = p->n_theta;
    double v = orc_candidate_v(kappa, r, v_prev);
    int32_t ka = 0;
    double mss = 0.0;
    double* per = (double*)malloc(sizeof(double) * (size_t)(p->N > 0 ? p->N : 1));
    double M = orc_candidate(p, x0, v, t, per, &ka, &mss);
    double worst_roll = p->N > 0 ? per[ka] : INFINITY;
    free(per);
    double dv = 0.0, dth[ORC_MAXTH] = {0};
    if (mss < worst_roll) {          /* the steady-state term is active */
        orc_steady_tangent(p, v, &dv, dth);
        ka = -1;
    } else {                          /* ties go to the rollout term */
        orc_rollout_tangent(p, x0, v, t, (uint32_t)ka, &dv, dth, NULL, NULL);
    }
    if (dM_dkappa) *dM_dkappa = dv * (r - v_prev);
    if (dM_dtheta)
        for (int q = 0; q < nt; ++q) dM_dtheta[q] = dth[q];
    if (k_arg) *k_arg = ka;
    return M;
}

/* ========================================================================= *
 * Safeguarded Newton search on phi(kappa) = M(kappa) (an alternative to the
 * bisection of Alg. 1; not in the paper).  Round 0 evaluates kappa = 1 (stop
 * if admissible) and the midpoint 1/2.  Each later round evaluates the Newton
 * iterate kappa_N, its neighbours kappa_N -/+ delta (delta = 2^-K) and the
 * bracket midpoint; every verdict tightens the bracket [lo, hi] (lo admissible
 * or 0, hi refused).  kappa_N = kappa_c - phi(kappa_c) / phi'(kappa_c) from the
 * last iterate kappa_c (derivative of the active term); a step at or past a
 * bracket end moves delta inside that end, and a non-negative or non-finite
 * slope falls back to the midpoint.  Stops when hi - lo <= delta and returns lo.  The midpoint makes the
 * bracket at least halve per round, so at most K + 1 rounds.
 * ========================================================================= */
orc_result orc_newton(const orc_problem* p, const double* x0, double r, double v_prev,
                      uint32_t t, int32_t K, int32_t* rounds_out, int32_t* fallbacks_out)
{
    orc_result res = {0.0, v_prev, -INFINITY, 0, 1};
    const double delta = ldexp(1.0, -K);
    double lo = 0.0, hi = 1.0;
    int found = 0, rounds = 0, fallbacks = 0;
    double worst_lo = -INFINITY;
    double kc = 1.0, phi = 0.0, dphi = 0.0;
    /* round 0 */
    phi = orc_candidate_grad(p, x0, 1.0, r, v_prev, t, &dphi, NULL, NULL);
    res.passes++;
    rounds = 1;
    if (phi >= 0.0) {
        res.kappa = 1.0;
        res.v = r;
        res.worst = phi;
        res.status = 0;
        if (rounds_out) *rounds_out = rounds;
        if (fallbacks_out) *fallbacks_out = 0;
        return res;
    }
    {
        double Mm = orc_candidate(p, x0, orc_candidate_v(0.5, r, v_prev), t, NULL, NULL, NULL);
        res.passes++;
        if (Mm >= 0.0) { lo = 0.5; found = 1; worst_lo = Mm; }
        else hi = 0.5;
    }
    while (hi - lo > delta && rounds < K + 2) {
        double kn;
        int newton_ok = isfinite(phi) && isfinite(dphi) && dphi < 0.0;
        kn = newton_ok ? kc - phi / dphi : 0.5 * (lo + hi);
        /* A step at or past a bracket end is moved just inside that end: the
         * root lies next to it (hi - lo > delta keeps lo + delta and hi - delta
         * strictly inside). */
        if (newton_ok && kn <= lo) kn = lo + delta;
        else if (newton_ok && kn >= hi) kn = hi - delta;
        if (!(kn > lo && kn < hi)) {
            kn = 0.5 * (lo + hi);
            newton_ok = 0;
        }
        if (!newton_ok) fallbacks++;
        double cand[4] = {kn - delta, kn, kn + delta, 0.5 * (lo + hi)};
        double M[4];
        double dn = 0.0;
        for (int c = 0; c < 4; ++c) {
            if (!(cand[c] > lo && cand[c] < hi)) { M[c] = NAN; continue; }
            if (c == 1) M[c] = orc_candidate_grad(p, x0, cand[c], r, v_prev, t, &dn, NULL, NULL);
            else M[c] = orc_candidate(p, x0, orc_candidate_v(cand[c], r, v_prev), t, NULL, NULL, NULL);
            res.passes++;
        }
        for (int c = 0; c < 4; ++c) {
            if (M[c] != M[c]) continue;
            if (M[c] >= 0.0) {
                if (cand[c] > lo) { lo = cand[c]; found = 1; worst_lo = M[c]; }
            } else if (cand[c] < hi) {
                hi = cand[c];
            }
        }
        kc = kn;
        phi = M[1];
        dphi = dn;
        rounds++;
    }
    res.kappa = found ? lo : 0.0;
    res.v = found ? orc_candidate_v(lo, r, v_prev) : v_prev;
    res.worst = worst_lo;
    res.status = found ? 0 : 1;
    if (rounds_out) *rounds_out = rounds;
    if (fallbacks_out) *fallbacks_out = fallbacks;
    return res;
}
