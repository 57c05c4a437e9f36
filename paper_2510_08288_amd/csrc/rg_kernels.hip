// HIP kernels of the robust reference governor for gfx950 (wave64).
//
// Per RG step the host enqueues (or replays from a graph):
//   gen       scenario draws d_j^k for this step into device memory (Sec. II-C:
//             one draw set per time step, shared by every candidate)
//   setup     round-0 candidates: kappa = 1 and the first levels of the
//             bisection tree (Alg. 1), or the M-point grid (Alg. 3)
//   R x { rollout   one lane per (candidate, scenario): RK4 prediction over
//                   j = 0..H with the constraint margin folded into a running
//                   minimum (Eq. (3) constraint rows; Alg. 3 parallel steps 2-3)
//         recheck   FP64 re-simulation of lanes whose FP32 margin is within
//                   the band of zero
//         decide    verdicts, bracket update, next round's candidates }
//   finalize  result record; in closed loop the true-plant step x_{t+1}
//
// No step reads back to the host.  All search state lives in DevSearch.
#include <hip/hip_runtime.h>

#include <cstring>
#include <type_traits>

#include "rg_device.hpp"

namespace rg {

// ---------------------------------------------------------------------------
// Argument blocks
// ---------------------------------------------------------------------------
template <int KIND, class T>
struct RollArgs {
  using P = Plant<KIND, T>;
  typename P::Coef pc;
  T F[kNC * P::ny];
  T g[kNC];
  T h, hh, h6;
  T band;
  int H, N;
  int early, record, inject;
  uint32_t seed, inst;
  float wlo[P::nw], wspan[P::nw];
  float thlo, thspan;
  const float* wbuf;
  const float* thbuf;
  const DevState* st;
  DevSearch* srch;
  float* per_m;
  int32_t* per_j;
  unsigned long long* per_key;  // chance-constrained verdict: per-scenario margin keys
  int2* rlist;
  // checkpoints of one candidate's scenarios for the segment derivative:
  // ckpt[(s * n + i) * N + k] = state component i of scenario k at step s * Kc
  float* ckpt;
  int Kc;
  int ckpt_cand;  // that candidate (-1: the Newton iterate of the round)
  // gen_row0 > 0: rows blockIdx.y >= gen_row0 of the launch generate the
  // draws of step t + 1 into gen_w / gen_th instead of simulating
  int gen_row0;
  uint32_t gen_ofs;  // the draws generated are those of step t + gen_ofs
  float* gen_w;
  float* gen_th;
  // forward tangent (CKPT = 2): per scenario of the tangent candidate, dm/dv
  // (tan_dv[k]), the margin (per_m[k]) and its minimising step (per_j[k])
  float* tan_dv;
  // ring != 0 (closed loop): the draws of step s are in wring[s % kPairs],
  // selected from the step counter on the device (wbuf, gen_w and gen_th are
  // then unused; gen_w != nullptr only switches the draw workgroups on)
  int ring;
  float* wring[kPairs];
  float* thring[kPairs];
};

// Draws of step t (streamed mode).
template <class A>
__device__ __forceinline__ const float* step_w(const A& a, uint32_t t) {
  return a.ring ? a.wring[t % kPairs] : a.wbuf;
}
template <class A>
__device__ __forceinline__ const float* step_th(const A& a, uint32_t t) {
  return a.ring ? a.thring[t % kPairs] : a.thbuf;
}

template <int KIND>
struct CtlArgs {
  typename Plant<KIND, double>::Coef pc;
  DevState* st;
  DevSearch* srch;
  const double* r_seq;
  int closed_loop;
  DevGrad* grad;
};

// ---------------------------------------------------------------------------
// Draws
// ---------------------------------------------------------------------------
template <int NW>
__device__ __forceinline__ void draw_w(uint32_t seed, uint32_t inst, uint32_t t, uint32_t tag,
                                       uint32_t k, uint32_t j, const float* lo, const float* span,
                                       float* w) {
#pragma unroll
  for (int blk = 0; blk < (NW + 3) / 4; ++blk) {
    const Words r = philox10(k, j, t, (tag << 16) | (uint32_t)blk, seed, inst);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = 4 * blk + q;
      if (c < NW) w[c] = box_draw(r.v[q], lo[c], span[c]);
    }
  }
}

template <int NTH>
__device__ __forceinline__ void draw_theta_factor(uint32_t seed, uint32_t inst, uint32_t t,
                                                  uint32_t k, float lo, float span, float* f) {
#pragma unroll
  for (int blk = 0; blk < (NTH + 3) / 4; ++blk) {
    const Words r = philox10(k, 0u, t, (1u << 16) | (uint32_t)blk, seed, inst);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = 4 * blk + q;
      if (c < NTH) f[c] = box_draw(r.v[q], lo, span);
    }
  }
}

// Streamed draws: w[(j * nw + c) * N + k] (consecutive scenarios contiguous, so
// a wave's loads of one step coalesce), theta factors f[c * N + k].
template <int KIND, class A>
__device__ __forceinline__ void gen_body(const A& a, float* wbuf, float* thbuf, size_t gid,
                                         uint32_t t, bool streaming = false) {
  using P = Plant<KIND, float>;
  const size_t nwork = (size_t)a.H * a.N;
  if (gid < nwork) {
    const int j = (int)(gid / a.N);
    const int k = (int)(gid - (size_t)j * a.N);
    float w[P::nw];
    draw_w<P::nw>(a.seed, a.inst, t, 0u, (uint32_t)k, (uint32_t)j, a.wlo, a.wspan, w);
#pragma unroll
    for (int c = 0; c < P::nw; ++c) {
      float* dst = &wbuf[((size_t)j * P::nw + c) * a.N + k];
      if (streaming) __builtin_nontemporal_store(w[c], dst);
      else *dst = w[c];
    }
  } else if (P::nth > 0 && gid < nwork + (size_t)a.N) {
    const int k = (int)(gid - nwork);
    float f[P::nth > 0 ? P::nth : 1];
    draw_theta_factor<P::nth>(a.seed, a.inst, t, (uint32_t)k, a.thlo, a.thspan, f);
#pragma unroll
    for (int c = 0; c < P::nth; ++c) {
      float* dst = &thbuf[(size_t)c * a.N + k];
      if (streaming) __builtin_nontemporal_store(f[c], dst);
      else *dst = f[c];
    }
  }
}

template <int KIND>
__global__ void __launch_bounds__(256) k_gen(RollArgs<KIND, float> a, float* wbuf, float* thbuf,
                                             uint32_t t_ofs) {
  gen_body<KIND>(a, wbuf, thbuf, (size_t)blockIdx.x * blockDim.x + threadIdx.x, a.st->t + t_ofs);
}

// Draw rows of a rollout launch (grid-stride over the rows' threads): the
// draws of step t + gen_ofs, or in the closed loop (ring) those of the steps
// the step's setup chose (gen_lo .. gen_lo + gen_n - 1, in its first round
// only).  Returns true in those rows.
template <int KIND, class A>
__device__ __forceinline__ bool gen_rows(const A& a) {
  if (a.gen_row0 <= 0 || (int)blockIdx.y < a.gen_row0) return false;
  uint32_t t1 = a.st->t + a.gen_ofs;
  int nsteps = 1;
  if (a.ring) {  // while the chunk has steps left
    if (a.srch->round != 0 || a.st->cl_index >= a.st->cl_len) return true;
    t1 = a.st->gen_lo;
    nsteps = a.st->gen_n;
  }
  const size_t nth = (size_t)(gridDim.y - a.gen_row0) * gridDim.x * blockDim.x;
  const size_t work = (size_t)a.H * a.N + (Plant<KIND, float>::nth > 0 ? (size_t)a.N : 0);
  const size_t i0 =
      ((size_t)(blockIdx.y - a.gen_row0) * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
  for (int g = 0; g < nsteps; ++g, ++t1) {
    float* gw = a.ring ? a.wring[t1 % kPairs] : a.gen_w;
    float* gth = a.ring ? a.thring[t1 % kPairs] : a.gen_th;
    // streaming stores: these draws are read steps later, and lines left dirty
    // in L2 would have to be written back by the device-scope fences in between
    for (size_t i = i0; i < work; i += nth) gen_body<KIND>(a, gw, gth, i, t1, true);
  }
  return true;
}

// A float or double moved between lanes by DPP (CTRL: quad permutations, row
// shifts), 0 where the source lane lies outside the row.
template <int CTRL>
__device__ __forceinline__ float dpp_row(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL,
                                                               0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp64(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <int CTRL>
__device__ __forceinline__ double dpp_row(double x) {
  return dpp64<CTRL>(x);
}

// 9-state plant: a copy of the coupling matrix W in vector registers (identity
// DPP moves make the copies lane values), which the derivative then reads: 81
// uniform values beside the other coefficients exceed the scalar registers, and
// spilled scalars are restored at every use (a sixth of the one-lane FP32 loop).
template <int KIND, class T, class Coef, class Lane>
__device__ __forceinline__ void w_in_vgprs(const Coef& pc, T* wv, Lane& L) {
  if constexpr (KIND == 2) {
#pragma unroll
    for (int c = 0; c < 81; ++c) wv[c] = dpp_row<0xE4>(pc.W[c]);
    L.W = wv;
  }
}

// Forward declarations: the recheck kernels end with the round's decision.
template <int KIND>
__device__ void decide_body(const typename Plant<KIND, double>::Coef& pc, const DevState* st,
                            DevSearch* S, const DevGrad* grad);
template <int KIND>
__device__ void last_block_decides(const CtlArgs<KIND>& ctl);
template <int KIND>
__device__ void true_plant_step(const RollArgs<KIND, double>& a, const double* x_in, double v,
                                uint32_t t, double* x_out);

// ---------------------------------------------------------------------------
// One scenario rollout with the fused running-minimum margin.
// stop_flag (nullable) is polled every 32 steps; early != 0 also stops the
// lane once its minimum is below -band.  traj (nullable) receives states.
// ---------------------------------------------------------------------------
// With WAVE set the whole wave evaluates one candidate and stop_flag is that
// candidate's dead flag: one violation anywhere ends the candidate, so the
// wave stops as soon as any of its lanes sees one, and raises the flag at once
// for the other waves (which read it every 8 steps).  Without WAVE, lanes
// stop on their own and stop_flag is only read.
template <int KIND, class T, int RNG, int INJ, class A, int CKPT = 0, bool WAVE = false,
          bool WREG = false>
__device__ __forceinline__ T rollout_lane(const A& a, int early, T v, int k, uint32_t t,
                                          int32_t* stop_flag, int& jbest, int& nsteps,
                                          double* traj, bool ck = false,
                                          bool* stopped = nullptr) {
  using P = Plant<KIND, T>;
  T th[P::nth > 0 ? P::nth : 1];
  if constexpr (P::nth > 0) {
    float f[P::nth];
    if (RNG == 0) {
      const float* tb = step_th(a, t);
#pragma unroll
      for (int c = 0; c < P::nth; ++c) f[c] = tb[(size_t)c * a.N + k];
    } else {
      draw_theta_factor<P::nth>(a.seed, a.inst, t, (uint32_t)k, a.thlo, a.thspan, f);
    }
#pragma unroll
    for (int c = 0; c < P::nth; ++c) th[c] = a.pc.thnom[c] * (T)f[c];
  }
  typename P::Lane L;
  P::lane_init(a.pc, th, v, L);
  // WREG (the FP32 rollout kernels): W in vector registers
  T wv[KIND == 2 && WREG ? 81 : 1];
  if constexpr (WREG) w_in_vgprs<KIND>(a.pc, wv, L);
  T x[P::n];
#pragma unroll
  for (int i = 0; i < P::n; ++i) x[i] = (T)a.st->x[i];
  T y[P::ny];
  P::output(a.pc, L, x, y);
  T best = margin_rows<P::ny>(a.F, a.g, y);
  if (best != best) best = -t_inf<T>();
  jbest = 0;
  if (traj) {
    for (int i = 0; i < P::n; ++i) traj[i] = (double)x[i];
  }
  int ck_left = 0, ck_seg = 0;  // steps to the next checkpoint, its index
  if constexpr (CKPT) {
    if (ck) {
      for (int i = 0; i < P::n; ++i) a.ckpt[(size_t)i * a.N + k] = (float)x[i];
      ck_left = a.Kc;
    }
  }
  float wc[P::nw], wn[P::nw];
  const float* wb = RNG == 0 ? step_w(a, t) : nullptr;
  auto load = [&](int j, float* w) {
    if (RNG == 0) {
#pragma unroll
      for (int c = 0; c < P::nw; ++c) w[c] = wb[((size_t)j * P::nw + c) * a.N + k];
    } else {
      draw_w<P::nw>(a.seed, a.inst, t, 0u, (uint32_t)k, (uint32_t)j, a.wlo, a.wspan, w);
    }
  };
  if (a.H > 0) load(0, wc);
  int j = 0;
  int stop_seen = 0;  // dead flag read at the start of an 8-step block, tested at its end
  for (; j < a.H; ++j) {
    if (j + 1 < a.H) load(j + 1, wn);
    if (WAVE && early && (j & 7) == 0)
      stop_seen = __hip_atomic_load(stop_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    T s[P::n];
    if (INJ == 0) {
      T wt[P::nw];
#pragma unroll
      for (int c = 0; c < P::nw; ++c) wt[c] = (T)wc[c];
      P::force(a.pc, L, wt, s);
    } else {
      P::force0(a.pc, L, s);
    }
    rk4_step<KIND, T>(a.pc, L, s, a.h, a.hh, a.h6, x);
    if (INJ == 1) {
      T wt[P::nw];
#pragma unroll
      for (int c = 0; c < P::nw; ++c) wt[c] = (T)wc[c];
      P::post(a.pc, wt, x);
    }
    P::output(a.pc, L, x, y);
    T m = margin_rows<P::ny>(a.F, a.g, y);
    m = (m == m) ? m : -t_inf<T>();
    if (m < best) {
      best = m;
      jbest = j + 1;
    }
    if (traj) {
      for (int i = 0; i < P::n; ++i) traj[(size_t)(j + 1) * P::n + i] = (double)x[i];
    }
    if constexpr (CKPT) {
      if (ck && --ck_left == 0) {
        ck_left = a.Kc;
        ++ck_seg;
        for (int i = 0; i < P::n; ++i)
          a.ckpt[((size_t)ck_seg * P::n + i) * a.N + k] = (float)x[i];
      }
    }
    if (early) {
      if constexpr (WAVE) {
        const bool viol = best < -a.band;
        if (__builtin_amdgcn_ballot_w64(viol) != 0) {
          if (viol) __hip_atomic_store(stop_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          *stopped = true;
          ++j;
          break;
        }
        if ((j & 7) == 7 && stop_seen) {
          *stopped = true;
          ++j;
          break;
        }
      } else {
        if (best < -a.band) {
          ++j;
          break;
        }
        if ((j & 31) == 31 && stop_flag &&
            __hip_atomic_load(stop_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ++j;
          break;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < P::nw; ++c) wc[c] = wn[c];
  }
  nsteps = j;
  bool finite = true;
#pragma unroll
  for (int i = 0; i < P::n; ++i) finite = finite && (x[i] - x[i] == (T)0);
  if (!finite) best = -t_inf<T>();
  return best;
}

// ---------------------------------------------------------------------------
// Rollout of one 9-state scenario by a group of 16 lanes (a DPP row), for the
// FP64 recheck of a few near-band scenarios and for FP32 rounds with few
// scenarios: one lane per scenario would leave every serial RK4 step on one
// lane while most of the chip idles.  Lane i of the group owns state
// component i; lanes 9..15 repeat component 8 and nothing reads them.  At every
// derivative evaluation each lane computes its own tanh and orifice factors,
// the group exchanges (x_i, tanh z_i) through its 16 LDS slots (the orifice
// factors through DPP row shifts), and each lane forms its component with
// Plant<2>::comp, the arithmetic of the one-lane rollout; every lane computes
// the margin from the exchanged state.  The result equals that of
// rollout_lane<2, T> bit for bit.  Control flow is uniform over the group
// (over the wave with WAVE): every branch depends on exchanged values or on a
// ballot.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void group_sync() {
  // The group is part of one wave, whose LDS accesses complete in program
  // order; this only keeps the compiler from moving them across.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T>
struct Pair;
template <>
struct Pair<float> {
  using type = float2;
};
template <>
struct Pair<double> {
  using type = double2;
};

// WAVE (FP32 rollouts of one candidate): the whole wave stops at the first
// violation of any of its groups, as rollout_lane's WAVE form, and stop_flag
// is that candidate's dead flag; otherwise (FP64 rechecks) the group stops on
// its own and stop_flag is only read.  CKPT with ck: checkpoints as
// rollout_lane's (lane i stores component i).  jbest and nsteps as
// rollout_lane's.
template <class T, int RNG, int INJ, bool WAVE = false, int CKPT = 0>
__device__ T rollout_fc9_group(const RollArgs<2, T>& a, int early, T v, int k, uint32_t t,
                               int32_t* stop_flag, typename Pair<T>::type* xch, int li,
                               unsigned long long gmask, int& jbest, int& nsteps, bool ck = false,
                               bool* stopped = nullptr) {
  using P = Plant<2, T>;
  const int i = li < 9 ? li : 8;
  T th[P::nth];
  {
    float f[P::nth];
    if (RNG == 0) {
      const float* tb = step_th(a, t);
#pragma unroll
      for (int c = 0; c < P::nth; ++c) f[c] = tb[(size_t)c * a.N + k];
    } else {
      draw_theta_factor<P::nth>(a.seed, a.inst, t, (uint32_t)k, a.thlo, a.thspan, f);
    }
#pragma unroll
    for (int c = 0; c < P::nth; ++c) th[c] = a.pc.thnom[c] * (T)f[c];
  }
  typename P::Lane L;
  P::lane_init(a.pc, th, v, L);
  // this lane's coefficients: a_i, xbar_i (and its tanh exponent shift), a_i
  // xbar_i, row i of W, k_{i-1} and k_i of the orifice flows q_i and q_{i+1},
  // the draw bounds of w_i
  T ai = L.a[0], xb = a.pc.xbar[0], nkxb = a.pc.nkxbar[0], axb = L.axb[0], kql = (T)0,
    kqh = L.kq[0], wrow[9];
  float wlo = a.wlo[0], wsp = a.wspan[0];
#pragma unroll
  for (int j = 0; j < 9; ++j) wrow[j] = a.pc.W[j];
#pragma unroll
  for (int r = 1; r < 9; ++r) {
    const bool on = i == r;
    ai = on ? L.a[r] : ai;
    xb = on ? a.pc.xbar[r] : xb;
    nkxb = on ? a.pc.nkxbar[r] : nkxb;
    axb = on ? L.axb[r] : axb;
    wlo = on ? a.wlo[r] : wlo;
    wsp = on ? a.wspan[r] : wsp;
#pragma unroll
    for (int j = 0; j < 9; ++j) wrow[j] = on ? a.pc.W[9 * r + j] : wrow[j];
    if (r < 6) kqh = on ? L.kq[r] : kqh;
    if (r < 6) kql = on ? L.kq[r - 1] : kql;
  }
  // exchange of the evaluation point: X and TZ receive (x_j, tanh z_j) of
  // every component; rh = r_i and rl = r_{i-1}, the orifice factors of q_{i+1}
  // and q_i, come from the neighbouring lanes by DPP row shifts
  T X[9], TZ[9], rl, rh;
  auto exch = [&](T xv) {
    const T xn = dpp_row<0x101>(xv);  // row_shl:1, x_{i+1}
    rh = P::orifice(xv, i < 5 ? xn : a.pc.p_amb);
    rl = dpp_row<0x111>(rh);  // row_shr:1, r_{i-1}
    typename Pair<T>::type e;
    e.x = xv;
    e.y = P::tanh_at(xv, xb, nkxb);
    xch[li] = e;
    group_sync();
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const typename Pair<T>::type f = xch[j];
      X[j] = f.x;
      TZ[j] = f.y;
    }
    group_sync();
  };
  // component i of the derivative at the exchanged point (own component xv)
  auto eval = [&](T xv, T si) {
    const T qa = i == 0 ? a.pc.c_q0 : kql;
    const T qb = i == 0 ? X[6] : rl;
    return P::comp(i, ai, wrow, si, xv, TZ, qa, qb, kqh, rh, X[0], X[6], X[8], L, a.pc.p1ref);
  };
  const float* wb = RNG == 0 ? step_w(a, t) : nullptr;
  const int wq = i & 3;
  auto load = [&](int j) -> float {
    if (RNG == 0) return wb[((size_t)j * P::nw + i) * a.N + k];
    const Words r = philox10((uint32_t)k, (uint32_t)j, t, (uint32_t)(i >> 2), a.seed, a.inst);
    const uint32_t word = wq == 0 ? r.v[0] : (wq == 1 ? r.v[1] : (wq == 2 ? r.v[2] : r.v[3]));
    return box_draw(word, wlo, wsp);
  };
  T xv = (T)a.st->x[i];
  exch(xv);
  T y[P::ny];
  P::output(a.pc, L, X, y);
  T best = margin_rows<P::ny>(a.F, a.g, y);
  if (best != best) best = -t_inf<T>();
  jbest = 0;
  int ck_left = 0, ck_seg = 0;  // steps to the next checkpoint, its index
  if constexpr (CKPT) {
    if (ck) {
      if (li < 9) a.ckpt[(size_t)i * a.N + k] = (float)xv;
      ck_left = a.Kc;
    }
  }
  float wc = a.H > 0 ? load(0) : 0.0f, wn = 0.0f;
  int j = 0;
  bool stop_seen = false;  // dead flag read at the start of an 8-step block, tested at its end
  for (; j < a.H; ++j) {
    if (j + 1 < a.H) wn = load(j + 1);
    if (WAVE && early && (j & 7) == 0)
      stop_seen = __hip_atomic_load(stop_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    const T si = INJ == 0 ? (T)wc + axb : axb;  // P::force / P::force0 of component i
    T kk = eval(xv, si);
    T acc = kk;
    T xs = t_fma(a.hh, kk, xv);
    exch(xs);
    kk = eval(xs, si);
    acc = t_fma((T)2, kk, acc);
    xs = t_fma(a.hh, kk, xv);
    exch(xs);
    kk = eval(xs, si);
    acc = t_fma((T)2, kk, acc);
    xs = t_fma(a.h, kk, xv);
    exch(xs);
    kk = eval(xs, si);
    xv = t_fma(a.h6, acc + kk, xv);
    if (INJ == 1) xv = xv + (T)wc;
    exch(xv);
    P::output(a.pc, L, X, y);
    T m = margin_rows<P::ny>(a.F, a.g, y);
    m = (m == m) ? m : -t_inf<T>();
    if (m < best) {
      best = m;
      jbest = j + 1;
    }
    if constexpr (CKPT) {
      if (ck && --ck_left == 0) {
        ck_left = a.Kc;
        ++ck_seg;
        if (li < 9) a.ckpt[((size_t)ck_seg * P::n + i) * a.N + k] = (float)xv;
      }
    }
    if (early) {
      if constexpr (WAVE) {
        // every group of the wave evaluates the same candidate
        const bool viol = best < -a.band;
        if (__builtin_amdgcn_ballot_w64(viol) != 0) {
          if (viol && li == 0)
            __hip_atomic_store(stop_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          *stopped = true;
          ++j;
          break;
        }
        if ((j & 7) == 7 && __builtin_amdgcn_ballot_w64(stop_seen) != 0) {
          *stopped = true;
          ++j;
          break;
        }
      } else {
        if (best < -a.band) {
          ++j;
          break;
        }
        if ((j & 31) == 31 && stop_flag) {
          const bool f =
              __hip_atomic_load(stop_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
          if (__builtin_amdgcn_ballot_w64(f) & gmask) {
            ++j;
            break;
          }
        }
      }
    }
    wc = wn;
  }
  nsteps = j;
  bool finite = true;
#pragma unroll
  for (int jj = 0; jj < 9; ++jj) finite = finite && (X[jj] - X[jj] == (T)0);
  if (!finite) best = -t_inf<T>();
  return best;
}

// The FP64 recheck of near-band entries [g0, n) with stride gstride over
// groups of 16 lanes (rollout_fc9_group), with the verdict updates of
// k_recheck made by the group's first lane.  blockDim.x is a multiple of 16
// and at most 64.
template <int RNG, int INJ>
__device__ void recheck_fc9_groups(const RollArgs<2, double>& a, DevSearch* S, int n, uint32_t t,
                                   int g0, int gstride) {
  __shared__ double2 xch[64];
  const int li = threadIdx.x & 15;
  double2* slot = xch + (threadIdx.x & ~15);
  const unsigned long long gmask = 0xffffull << (threadIdx.x & 48);
  const int q = S->q;
  for (int e = g0; e < n; e += gstride) {
    const int2 en = a.rlist[e];
    const int c = en.x, k = en.y;
    const bool skip =
        a.early && (__hip_atomic_load(&S->dead[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                    __hip_atomic_load(&S->fail64[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (__builtin_amdgcn_ballot_w64(skip) & gmask) continue;
    int jb = 0, ns = 0;
    const double m = rollout_fc9_group<double, RNG, INJ>(
        a, a.early, S->v[c], k, t, a.early && q == 0 ? &S->fail64[c] : nullptr, slot, li, gmask,
        jb, ns);
    if (li != 0) continue;
    atomicMin(&S->key64[c], ord64(m));
    if (q > 0) {
      a.per_key[(size_t)c * a.N + k] = ord64(m);
      if (m < 0.0 && S->nviol[c] + atomicAdd(&S->nviol64[c], 1) >= q)
        __hip_atomic_store(&S->fail64[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (m < 0.0) {
      __hip_atomic_store(&S->fail64[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// One scenario rollout in FP32 over the full horizon with the forward tangent
// of the state with respect to the set-point carried along (not in the paper:
// it gives the derivative the Newton search needs in the same pass).  Returns
// the running-minimum margin as rollout_lane does; dm receives the derivative
// of that minimum: -F_r* (dh/dx) dx/dv at its first minimising step j* (jbest)
// and row r*.  The state update is that of rollout_lane.
template <int KIND, int RNG, int INJ, class A>
__device__ __forceinline__ float rollout_lane_tan(const A& a, float v, int k, uint32_t t,
                                                  float& dm, int& jbest, int& nsteps) {
  using P = Plant<KIND, float>;
  float th[P::nth > 0 ? P::nth : 1];
  if constexpr (P::nth > 0) {
    float f[P::nth];
    if (RNG == 0) {
      const float* tb = step_th(a, t);
#pragma unroll
      for (int c = 0; c < P::nth; ++c) f[c] = tb[(size_t)c * a.N + k];
    } else {
      draw_theta_factor<P::nth>(a.seed, a.inst, t, (uint32_t)k, a.thlo, a.thspan, f);
    }
#pragma unroll
    for (int c = 0; c < P::nth; ++c) th[c] = a.pc.thnom[c] * f[c];
  }
  typename P::Lane L;
  P::lane_init(a.pc, th, v, L);
  float x[P::n], dx[P::n], y[P::ny], dy[P::ny];
#pragma unroll
  for (int i = 0; i < P::n; ++i) {
    x[i] = (float)a.st->x[i];
    dx[i] = 0.f;  // x_t does not depend on the candidate
  }
  // margin at a step and its derivative through the minimising row
  auto margin_tan = [&](float& m, float& dmj) {
    int r = 0;
    P::output(a.pc, L, x, y);
    m = margin_rows_arg<P::ny>(a.F, a.g, y, r);
    P::output_tan(a.pc, x, dx, dy);
    // row r of F by selection (a per-lane index into the argument block would
    // place the block in scratch memory)
    float fr[P::ny];
#pragma unroll
    for (int i = 0; i < P::ny; ++i) fr[i] = a.F[i];
#pragma unroll
    for (int rr = 1; rr < kNC; ++rr)
#pragma unroll
      for (int i = 0; i < P::ny; ++i) fr[i] = rr == r ? a.F[rr * P::ny + i] : fr[i];
    float fy = fr[0] * dy[0];
#pragma unroll
    for (int i = 1; i < P::ny; ++i) fy = __builtin_fmaf(fr[i], dy[i], fy);
    dmj = -fy;
  };
  float best, dbest;
  margin_tan(best, dbest);
  if (best != best) best = -INFINITY;
  jbest = 0;
  const float* wb = RNG == 0 ? step_w(a, t) : nullptr;
  auto load = [&](int jj, float* w) {
    if (RNG == 0) {
#pragma unroll
      for (int c = 0; c < P::nw; ++c) w[c] = wb[((size_t)jj * P::nw + c) * a.N + k];
    } else {
      draw_w<P::nw>(a.seed, a.inst, t, 0u, (uint32_t)k, (uint32_t)jj, a.wlo, a.wspan, w);
    }
  };
  // the next step's draws are in flight while this step computes
  float w[P::nw], wn[P::nw];
  if (a.H > 0) load(0, w);
  int j = 0;
  for (; j < a.H; ++j) {
    if (j + 1 < a.H) load(j + 1, wn);
    float s[P::n];
    if (INJ == 0) P::force(a.pc, L, w, s);
    else P::force0(a.pc, L, s);
    rk4_step_tan<KIND, float>(a.pc, L, s, a.h, a.hh, a.h6, x, dx);
    if (INJ == 1) P::post(a.pc, w, x);
    float m, dmj;
    margin_tan(m, dmj);
    m = (m == m) ? m : -INFINITY;
    if (m < best) {
      best = m;
      dbest = dmj;
      jbest = j + 1;
    }
#pragma unroll
    for (int c = 0; c < P::nw; ++c) w[c] = wn[c];
  }
  nsteps = j;
  bool finite = true;
#pragma unroll
  for (int i = 0; i < P::n; ++i) finite = finite && (x[i] - x[i] == 0.f);
  if (!finite) best = -INFINITY;
  dm = dbest;
  return best;
}

// Wave64 + workgroup minimum of a 64-bit key; returns the minimum in thread 0.
__device__ __forceinline__ unsigned long long block_min_u64(unsigned long long v,
                                                             unsigned long long* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)v, off);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), off);
    const unsigned long long o = ((unsigned long long)hi << 32) | lo;
    v = o < v ? o : v;
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 1; i < nw; ++i) v = sh[i] < v ? sh[i] : v;
  }
  __syncthreads();
  return v;
}

// Step offset of candidate c: 0 for the step's own candidates, j for a
// speculative candidate of step t + j (closed loop, round 0).
__device__ __forceinline__ int cand_step(const DevSearch* S, int c) {
  const int r = c - S->spec_base;
  return (S->spec_n > 0 && r >= 0 && r < S->spec_n * S->spec_per) ? 1 + r / S->spec_per : 0;
}

// In decision mode a candidate whose FP64 steady-state test already fails is
// refused without simulating it (the verdict of Alg. 1 needs both tests).
// bx: the workgroup's scenario tile (tile 0 raises the flag).
__device__ __forceinline__ bool refused_by_steady_state(int early, DevSearch* S, int c,
                                                        int bx = -1) {
  if (!early || !(S->mss[c] < 0.0)) return false;
  if ((bx < 0 ? (int)blockIdx.x : bx) == 0 && threadIdx.x == 0)
    __hip_atomic_store(&S->dead[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// Main rollout kernel: blockIdx.y = candidate of the round, blockIdx.x * block
// + threadIdx.x = scenario.  CHANCE = 1 is the chance-constrained verdict
// (handles with q > 0): lanes stop on their own and every lane's margin key is
// kept.  It is a separate instantiation so that the robust kernel carries one
// rollout body only (two bodies double the 9-state kernel's registers).
// Body of one rollout workgroup: candidate row c, scenario tile bx (scenarios
// bx * blockDim.x + threadIdx.x).
template <int KIND, class T, int RNG, int INJ, int CKPT, int CHANCE>
__device__ __forceinline__ void rollout_block(const RollArgs<KIND, T>& a, const int c,
                                              const int bx, unsigned long long* sh) {
  DevSearch* S = a.srch;
  if (S->done || c >= S->n_cand) return;  // uniform over the workgroup
  // CKPT = 1: that candidate keeps checkpoints (adjoint); CKPT = 2: its lanes
  // carry the forward tangent instead (full horizon, no early exit)
  const bool ck = CKPT == 1 && c == (a.ckpt_cand >= 0 ? a.ckpt_cand : S->nk_idx);
  const bool tan_row = CKPT == 2 && c == (a.ckpt_cand >= 0 ? a.ckpt_cand : S->nk_idx);
  const int early = a.early && !S->full[c] && !tan_row;
  if (refused_by_steady_state(early, S, c, bx)) return;
  const int k = bx * blockDim.x + threadIdx.x;
  const uint32_t t = a.st->t;
  const int q = CHANCE ? S->q : 0;  // chance-constrained verdict: up to q violating scenarios
  T m = t_inf<T>();
  int jb = 0, ns = 0;
  if (k < a.N) {
    bool stopped = false;  // the candidate died while this wave ran (no recheck needed)
    if (CKPT == 2 && std::is_same<T, float>::value && tan_row) {
      if constexpr (CKPT == 2 && std::is_same<T, float>::value) {
        float dm = 0.f;
        m = rollout_lane_tan<KIND, RNG, INJ>(a, (float)S->v[c], k, t, dm, jb, ns);
        a.tan_dv[k] = dm;
        a.per_m[k] = (float)m;
        a.per_j[k] = jb;
      }
    } else if constexpr (CHANCE) {
      // a violating lane stops alone; the candidate dies once more than q did
      m = rollout_lane<KIND, T, RNG, INJ, RollArgs<KIND, T>, CKPT, false,
                       std::is_same<T, float>::value>(
          a, early, (T)S->v[c], k, t, early ? &S->dead[c] : nullptr, jb, ns, nullptr, ck);
      a.per_key[(size_t)c * a.N + k] = ord64((double)m);
    } else {
      m = rollout_lane<KIND, T, RNG, INJ, RollArgs<KIND, T>, CKPT, true,
                       std::is_same<T, float>::value>(
          a, early, (T)S->v[c], k, t, &S->dead[c], jb, ns, nullptr, ck, &stopped);
    }
    if (a.record) {
      a.per_m[(size_t)c * a.N + k] = (float)m;
      a.per_j[(size_t)c * a.N + k] = jb;
    }
    if (m < -a.band) {
      if (q == 0 || atomicAdd(&S->nviol[c], 1) >= q)
        __hip_atomic_store(&S->dead[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (m < a.band && !stopped) {
      const int idx = atomicAdd(&S->n_recheck, 1);
      a.rlist[idx] = make_int2(c, k);
    }
  }
  const unsigned long long key = lane_key(m, k);
  const unsigned long long kall = block_min_u64(key, sh);
  const unsigned long long kfar = block_min_u64((m >= a.band) ? key : ~0ull, sh);
  // executed steps: wave sum, one atomic per wave
  int wsum = ns;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(&S->lane_steps, (unsigned long long)wsum);
  if (threadIdx.x == 0) {
    atomicMin(&S->key_all[c], kall);
    if (kfar != ~0ull) atomicMin(&S->key_far[c], kfar);
  }
}

template <int KIND, class T, int RNG, int INJ, int CKPT, int CHANCE = 0>
__global__ void __launch_bounds__(256) k_rollout(const RollArgs<KIND, T> a) {
  if (gen_rows<KIND>(a)) return;
  __shared__ unsigned long long sh[16];
  rollout_block<KIND, T, RNG, INJ, CKPT, CHANCE>(a, blockIdx.y, blockIdx.x, sh);
}

// 9-state FP32 rollouts with one scenario per group of 16 lanes
// (rollout_fc9_group), robust verdict: blockIdx.y = candidate, 16 scenarios
// per 256 lanes.  The per-scenario bookkeeping is rollout_block's, made by the
// group's first lane; the margins equal the one-lane kernel's bit for bit.
// CKPT = 1: the checkpoint candidate's groups store the adjoint's checkpoints.
template <int RNG, int INJ, int CKPT>
__global__ void __launch_bounds__(256) k_rollout_fc9_group(const RollArgs<2, float> a) {
  if (gen_rows<2>(a)) return;
  __shared__ unsigned long long sh[16];
  __shared__ float2 xch[256];
  DevSearch* S = a.srch;
  const int c = blockIdx.y;
  if (S->done || c >= S->n_cand) return;  // uniform over the workgroup
  const bool ck = CKPT == 1 && c == (a.ckpt_cand >= 0 ? a.ckpt_cand : S->nk_idx);
  const int early = a.early && !S->full[c];
  if (refused_by_steady_state(early, S, c)) return;
  const int li = threadIdx.x & 15;
  const int k = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 4);
  const unsigned long long gmask = 0xffffull << (threadIdx.x & 48);
  const uint32_t t = a.st->t;
  float m = INFINITY;
  int jb = 0, ns = 0;
  if (k < a.N) {  // whole groups are active or inactive together
    bool stopped = false;  // the candidate died while this wave ran (no recheck needed)
    m = rollout_fc9_group<float, RNG, INJ, true, CKPT>(a, early, (float)S->v[c], k, t, &S->dead[c],
                                                       xch + (threadIdx.x & ~15u), li, gmask, jb,
                                                       ns, ck, &stopped);
    if (li == 0) {
      if (a.record) {
        a.per_m[(size_t)c * a.N + k] = m;
        a.per_j[(size_t)c * a.N + k] = jb;
      }
      if (m < -a.band) {
        __hip_atomic_store(&S->dead[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if (m < a.band && !stopped) {
        const int idx = atomicAdd(&S->n_recheck, 1);
        a.rlist[idx] = make_int2(c, k);
      }
    }
  }
  const bool own = li == 0 && k < a.N;
  const unsigned long long key = own ? lane_key(m, k) : ~0ull;
  const unsigned long long kall = block_min_u64(key, sh);
  const unsigned long long kfar = block_min_u64((own && m >= a.band) ? key : ~0ull, sh);
  int wsum = li == 0 ? ns : 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(&S->lane_steps, (unsigned long long)wsum);
  if (threadIdx.x == 0) {
    atomicMin(&S->key_all[c], kall);
    if (kfar != ~0ull) atomicMin(&S->key_far[c], kfar);
  }
}

// Batched serving: one launch per search round covers every instance of a
// (plant, disturbance injection) group.  Workgroup g of the flat grid takes
// scenario tile g - tile_first[i] of instance i = tile_inst[g], with the
// instance's own argument block from device memory; row blockIdx.y is the
// candidate (instances with fewer candidates in the round return at once).
// FP32, robust verdict, draws regenerated in the lanes.
template <int KIND, int INJ>
__global__ void __launch_bounds__(256) k_flat_rollout(const RollArgs<KIND, float>* __restrict__ args,
                                                      const int* __restrict__ tile_inst,
                                                      const int* __restrict__ tile_first) {
  __shared__ unsigned long long sh[16];
  const int i = tile_inst[blockIdx.x];
  rollout_block<KIND, float, 1, INJ, 0, 0>(args[i], blockIdx.y, (int)blockIdx.x - tile_first[i], sh);
}

// ---------------------------------------------------------------------------
// LQ4 in FP32 with one scenario per quad of lanes.  Lane q of the quad holds
// state component x_q.  Every derivative evaluation forms the contributions of
// x_q to the four rows in lane-relative order (slot s <-> row q XOR s), so two
// DPP butterflies (partner q^2, then q^1) leave row q's sum in lane q with no
// selects.  The margin rows use D = F C the same way: lane q keeps the running
// minimum of row q, and the quad minimum is formed once per group of steps
// (for the exit test) and at the end.  All control decisions are quad-uniform,
// which the DPP exchanges require.
// ---------------------------------------------------------------------------
struct QuadCoef {
  float a[4][4];  // a[q][s] = A[q^s][q]
  float g[4][4];  // g[q][s] = G[q^s][q]
  float d[4][4];  // d[q][s] = -(F C)[q^s][q]
  float b[4];     // B[q]
  float e[4][2];  // E[q][.]
  float grow[4];  // g_q (constraint row q; +inf for padding rows)
};

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL,
                                                               0xf, 0xf, true));
}
constexpr int kSwap2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);  // quad_perm [2,3,0,1]
constexpr int kSwap1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);  // quad_perm [1,0,3,2]

struct QuadLane {
  float a0, a1, a2, a3, g0, g1, g2, g3;
};

// Row q of f(x) = s + A x + G (x.*x), summed over the quad.  Lane q forms
// x_q's contribution to row q^s as c_s = (A[q^s][q] + G[q^s][q] x_q) x_q (slot
// s); two DPP butterflies (partner q^2, then q^1) leave row q's sum in lane q.
__device__ __forceinline__ float quad_deriv(const QuadLane& L, float s, float x) {
  const float c2 = __builtin_fmaf(L.g2, x, L.a2) * x;
  const float c3 = __builtin_fmaf(L.g3, x, L.a3) * x;
  float c0 = __builtin_fmaf(__builtin_fmaf(L.g0, x, L.a0), x, s);
  float c1 = __builtin_fmaf(L.g1, x, L.a1) * x;
  c1 = c1 + dpp<kSwap2>(c3);
  c0 = c0 + dpp<kSwap2>(c2);
  return c0 + dpp<kSwap1>(c1);
}

__device__ __forceinline__ float min2(float a, float b) { return b < a ? b : a; }

// Minimum over the four lanes of a quad (every lane gets it).
__device__ __forceinline__ float quad_min(float m) {
  m = min2(m, dpp<kSwap1>(m));
  return min2(m, dpp<kSwap2>(m));
}

// Forward tangent in the quad layout: lane q carries dx_q/dv beside x_q.  A
// stage's tangent row i is B_i + sum_q (A[i][q] + 2 G[i][q] x_q) dx_q, formed
// in the same slots and butterflies as the state.
__device__ __forceinline__ float quad_tan(const QuadLane& L, float b, float x, float d) {
  const float x2 = x + x;
  const float c2 = __builtin_fmaf(L.g2, x2, L.a2) * d;
  const float c3 = __builtin_fmaf(L.g3, x2, L.a3) * d;
  float c0 = __builtin_fmaf(__builtin_fmaf(L.g0, x2, L.a0), d, b);
  float c1 = __builtin_fmaf(L.g1, x2, L.a1) * d;
  c1 = c1 + dpp<kSwap2>(c3);
  c0 = c0 + dpp<kSwap2>(c2);
  return c0 + dpp<kSwap1>(c1);
}

// Quad minimum of (margin, derivative, step) over the lanes' rows: the smallest
// margin, ties to the earlier step, then to the lower row (lane).
__device__ __forceinline__ void quad_min_tan(float& m, float& d, int& j, int q) {
  int r = q;
  auto take = [&](float m2, float d2, int j2, int r2) {
    if (m2 < m || (m2 == m && (j2 < j || (j2 == j && r2 < r)))) {
      m = m2;
      d = d2;
      j = j2;
      r = r2;
    }
  };
  {
    const float m2 = dpp<kSwap1>(m), d2 = dpp<kSwap1>(d);
    const int j2 = __builtin_amdgcn_update_dpp(0, j, kSwap1, 0xf, 0xf, true);
    const int r2 = __builtin_amdgcn_update_dpp(0, r, kSwap1, 0xf, 0xf, true);
    take(m2, d2, j2, r2);
  }
  {
    const float m2 = dpp<kSwap2>(m), d2 = dpp<kSwap2>(d);
    const int j2 = __builtin_amdgcn_update_dpp(0, j, kSwap2, 0xf, 0xf, true);
    const int r2 = __builtin_amdgcn_update_dpp(0, r, kSwap2, 0xf, 0xf, true);
    take(m2, d2, j2, r2);
  }
}

// CHANCE = 1: the chance-constrained verdict (handles with q > 0, no record,
// no checkpoints): a quad that violates counts itself once and the candidate
// dies once more than q did; a wave stops when all its quads have violated or
// the candidate died, and every scenario's margin key is kept for the order
// statistic.
template <int RNG, int INJ, int RECORD, int CKPT, int CHANCE = 0>
__global__ void __launch_bounds__(256) k_rollout_lq4_quad(const RollArgs<1, float> a,
                                                         const QuadCoef qc) {
  constexpr int U = kQuadGroup;  // steps per group: one prefetch, one exit test per group
  if (gen_rows<1>(a)) return;
  DevSearch* S = a.srch;
  const int c = blockIdx.y;
  if (S->done || c >= S->n_cand) return;  // uniform over the workgroup
  // CKPT = 1: that candidate keeps checkpoints (adjoint); CKPT = 2: its lanes
  // carry the forward tangent instead (full horizon, no early exit)
  const bool ck = CKPT == 1 && c == (a.ckpt_cand >= 0 ? a.ckpt_cand : S->nk_idx);
  const bool tan_row = CKPT == 2 && c == (a.ckpt_cand >= 0 ? a.ckpt_cand : S->nk_idx);
  const int early = a.early && !S->full[c] && !tan_row;
  if (refused_by_steady_state(early, S, c)) return;
  __shared__ unsigned long long sh[16];
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = gid >> 2, q = gid & 3;
  // speculative candidate of step t + sj (sj >= 1): its own start state and draws
  const int sj = cand_step(S, c);
  const bool spec = sj > 0;
  const uint32_t t = a.st->t + (uint32_t)sj;
  const float* wsrc = step_w(a, t);  // speculative probes exist only in the closed loop (ring)
  float best = INFINITY;
  int jb = 0, ns = 0;
  bool stopped = false;  // the candidate died while this wave ran (no recheck needed)
  bool counted = false;  // CHANCE: this quad's violation is counted in nviol
  if (CKPT == 2 && tan_row && k < a.N) {
    // tangent candidate: state and dx/dv over the full horizon; each lane
    // keeps its row's running minimum with derivative and first step
    QuadLane L;
    L.a0 = qc.a[q][0]; L.a1 = qc.a[q][1]; L.a2 = qc.a[q][2]; L.a3 = qc.a[q][3];
    L.g0 = qc.g[q][0]; L.g1 = qc.g[q][1]; L.g2 = qc.g[q][2]; L.g3 = qc.g[q][3];
    const float d0 = qc.d[q][0], d1 = qc.d[q][1], d2 = qc.d[q][2], d3 = qc.d[q][3];
    const float e0 = qc.e[q][0], e1 = qc.e[q][1], grow = qc.grow[q], bq0 = qc.b[q];
    const float bv = bq0 * (float)S->v[c];
    const float h = a.h, hh = a.hh, h6 = a.h6;
    float x = (float)a.st->x[q], dx = 0.f;
    auto row_sum = [&](float xv, float g0v) {
      const float c2 = d2 * xv, c3 = d3 * xv;
      float c0 = __builtin_fmaf(d0, xv, g0v);
      float c1 = d1 * xv;
      c1 = c1 + dpp<kSwap2>(c3);
      c0 = c0 + dpp<kSwap2>(c2);
      return c0 + dpp<kSwap1>(c1);
    };
    float bq = row_sum(x, grow), dbq = row_sum(dx, 0.f);
    int jq = 0;
    const float* wsrc_t = step_w(a, t);
    auto ld = [&](int j, float& u0, float& u1) {
      if (RNG == 0) {
        u0 = wsrc_t[(size_t)(2 * j) * a.N + k];
        u1 = wsrc_t[(size_t)(2 * j + 1) * a.N + k];
      } else {
        const Words r = philox10((uint32_t)k, (uint32_t)j, t, 0u, a.seed, a.inst);
        u0 = box_draw(r.v[0], a.wlo[0], a.wspan[0]);
        u1 = box_draw(r.v[1], a.wlo[1], a.wspan[1]);
      }
    };
    // draws of steps j + 1 and j + 2 are in flight while step j computes
    float w0 = 0.f, w1 = 0.f, n0 = 0.f, n1 = 0.f, f0 = 0.f, f1 = 0.f;
    if (a.H > 0) ld(0, w0, w1);
    if (a.H > 1) ld(1, n0, n1);
    for (int j = 0; j < a.H; ++j) {
      if (j + 2 < a.H) ld(j + 2, f0, f1);
      const float sf = INJ == 0 ? __builtin_fmaf(e1, w1, __builtin_fmaf(e0, w0, bv)) : bv;
      const float k1 = quad_deriv(L, sf, x), t1 = quad_tan(L, bq0, x, dx);
      float acc = k1, dacc = t1;
      float xs = __builtin_fmaf(hh, k1, x), ds = __builtin_fmaf(hh, t1, dx);
      const float k2 = quad_deriv(L, sf, xs), t2 = quad_tan(L, bq0, xs, ds);
      acc = __builtin_fmaf(2.f, k2, acc);
      dacc = __builtin_fmaf(2.f, t2, dacc);
      xs = __builtin_fmaf(hh, k2, x);
      ds = __builtin_fmaf(hh, t2, dx);
      const float k3 = quad_deriv(L, sf, xs), t3 = quad_tan(L, bq0, xs, ds);
      acc = __builtin_fmaf(2.f, k3, acc);
      dacc = __builtin_fmaf(2.f, t3, dacc);
      xs = __builtin_fmaf(h, k3, x);
      ds = __builtin_fmaf(h, t3, dx);
      const float k4 = quad_deriv(L, sf, xs), t4 = quad_tan(L, bq0, xs, ds);
      x = __builtin_fmaf(h6, acc + k4, x);
      dx = __builtin_fmaf(h6, dacc + t4, dx);
      if (INJ == 1) x = x + (e0 * w0 + e1 * w1);
      const float mr = row_sum(x, grow);
      const float dmr = row_sum(dx, 0.f);
      if (mr < bq) {
        bq = mr;
        dbq = dmr;
        jq = j + 1;
      }
      w0 = n0;
      w1 = n1;
      n0 = f0;
      n1 = f1;
    }
    ns = a.H;
    quad_min_tan(bq, dbq, jq, q);
    best = bq;
    float bad = x - x;
    bad = bad + dpp<kSwap1>(bad);
    bad = bad + dpp<kSwap2>(bad);
    if (!(bad == 0.f) || best != best) best = -INFINITY;
    if (q == 0) {
      a.tan_dv[k] = dbq;
      a.per_m[k] = best;
      a.per_j[k] = jq;
    }
  } else if (k < a.N) {  // whole quads are active or inactive together
    QuadLane L;
    L.a0 = qc.a[q][0]; L.a1 = qc.a[q][1]; L.a2 = qc.a[q][2]; L.a3 = qc.a[q][3];
    L.g0 = qc.g[q][0]; L.g1 = qc.g[q][1]; L.g2 = qc.g[q][2]; L.g3 = qc.g[q][3];
    const float d0 = qc.d[q][0], d1 = qc.d[q][1], d2 = qc.d[q][2], d3 = qc.d[q][3];
    const float e0 = qc.e[q][0], e1 = qc.e[q][1], grow = qc.grow[q];
    const float bv = qc.b[q] * (float)S->v[c];
    const float h = a.h, hh = a.hh, h6 = a.h6;
    const int H = a.H;
    float x = (float)(spec ? S->x_spec[sj - 1][q] : a.st->x[q]);
    // lane q: margin of constraint row q (g_q - (F C x)_q); padding rows are +inf
    auto row_margin = [&](float xv) {
      const float c2 = d2 * xv, c3 = d3 * xv;
      float c0 = __builtin_fmaf(d0, xv, grow);
      float c1 = d1 * xv;
      c1 = c1 + dpp<kSwap2>(c3);
      c0 = c0 + dpp<kSwap2>(c2);
      return c0 + dpp<kSwap1>(c1);
    };
    // Without a recorded arg-min step each lane keeps the running minimum of
    // its own row; the quad minimum is taken once per group (exit test) and
    // at the end, which gives the same minimum over rows and steps.
    float bq = row_margin(x);
    if (RECORD) best = quad_min(bq);
    int ck_left = 0, ck_seg = 0;  // steps to the next checkpoint, its index
    if (CKPT && ck) {
      a.ckpt[(size_t)q * a.N + k] = x;
      ck_left = a.Kc;
    }
    auto step = [&](float w0, float w1, int jnext) {
      const float s = INJ == 0 ? __builtin_fmaf(e1, w1, __builtin_fmaf(e0, w0, bv)) : bv;
      const float k1 = quad_deriv(L, s, x);
      float acc = k1;
      float xs = __builtin_fmaf(hh, k1, x);
      const float k2 = quad_deriv(L, s, xs);
      acc = __builtin_fmaf(2.f, k2, acc);
      xs = __builtin_fmaf(hh, k2, x);
      const float k3 = quad_deriv(L, s, xs);
      acc = __builtin_fmaf(2.f, k3, acc);
      xs = __builtin_fmaf(h, k3, x);
      const float k4 = quad_deriv(L, s, xs);
      x = __builtin_fmaf(h6, acc + k4, x);
      if (INJ == 1) x = x + (e0 * w0 + e1 * w1);
      if (CKPT && ck && --ck_left == 0) {
        ck_left = a.Kc;
        ++ck_seg;
        a.ckpt[((size_t)ck_seg * 4 + q) * a.N + k] = x;
      }
      const float mr = row_margin(x);
      if (RECORD) {
        const float m = quad_min(mr);
        if (m < best) {
          best = m;
          jb = jnext;
        }
      } else {
        bq = fminf(bq, mr);
      }
    };
    // Draws of steps j..j+U-1.  Streamed: raw buffer loads with the row's byte
    // offset in a scalar register and the lane's offset in a vector register
    // (no per-lane address arithmetic); the buffer holds U spare rows past H and
    // its byte size fits the 32-bit offsets (checked by the launcher).
    const uint32_t row_bytes = 8u * (uint32_t)a.N;  // one step: n_w = 2 floats x N
    const uint32_t vo0 = 4u * (uint32_t)k, vo1 = vo0 + 4u * (uint32_t)a.N;
    const __amdgpu_buffer_rsrc_t wres = __builtin_amdgcn_make_buffer_rsrc(
        (void*)wsrc, (short)0, (int)(row_bytes * (uint32_t)(H + U)), 0x00020000);
    uint32_t so = 0;  // byte offset of the next group's first row
    auto load_group = [&](int j, float* w) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (RNG == 0) {
          const uint32_t sr = so + (uint32_t)u * row_bytes;
          w[2 * u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(wres, vo0, sr, 0));
          w[2 * u + 1] =
              __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(wres, vo1, sr, 0));
        } else {
          const Words r = philox10((uint32_t)k, (uint32_t)(j + u), t, 0u, a.seed, a.inst);
          w[2 * u] = box_draw(r.v[0], a.wlo[0], a.wspan[0]);
          w[2 * u + 1] = box_draw(r.v[1], a.wlo[1], a.wspan[1]);
        }
      }
      if (RNG == 0) so += (uint32_t)U * row_bytes;
    };
    // Two draw buffers in turn: a group of U steps runs on one while the next
    // group's draws stream into the other.
    float wa[2 * U], wb[2 * U];
    load_group(0, wa);
    const int full = H / U;
    int g = 0;
    // One violation anywhere ends the candidate: the wave stops as soon as any
    // of its quads sees one and raises the dead flag at once; the flag is read
    // at the start of every group and tested at its end.  Returns true to stop.
    auto run_group = [&](const float* wc, float* wn) -> bool {
      load_group((g + 1) * U, wn);
      const int dead_seen =
          early ? __hip_atomic_load(&S->dead[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
#pragma unroll
      for (int u = 0; u < U; ++u) step(wc[2 * u], wc[2 * u + 1], g * U + u + 1);
      ++g;
      if (early) {
        const float bg = RECORD ? best : quad_min(bq);
        const bool viol = bg < -a.band;
        if constexpr (CHANCE) {
          if (viol && !counted) {
            counted = true;
            if (q == 0 && atomicAdd(&S->nviol[c], 1) >= S->q)
              __hip_atomic_store(&S->dead[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          if (__builtin_amdgcn_ballot_w64(!viol) == 0) return true;  // every quad violated
        } else if (__builtin_amdgcn_ballot_w64(viol) != 0) {
          if (viol && q == 0)
            __hip_atomic_store(&S->dead[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          stopped = true;
          return true;
        }
        if (dead_seen) {
          stopped = true;
          return true;
        }
      }
      return false;
    };
    bool tail_in_b = false;  // which buffer holds the draws after the last full group
    while (g < full) {
      if (run_group(wa, wb)) break;
      if (g == full) {
        tail_in_b = true;
        break;
      }
      if (run_group(wb, wa)) break;
    }
    ns = g * U;
    if (g == full && !stopped) {  // ragged tail of the horizon
      if (tail_in_b) {
#pragma unroll
        for (int u = 0; u < 2 * U; ++u) wa[u] = wb[u];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (u < H - full * U) step(wa[2 * u], wa[2 * u + 1], full * U + u + 1);
      ns = H;
    }
    if (!RECORD) best = quad_min(bq);
    // non-finite state in any lane of the quad -> -inf
    float bad = x - x;
    bad = bad + dpp<kSwap1>(bad);
    bad = bad + dpp<kSwap2>(bad);
    if (!(bad == 0.f) || best != best) best = -INFINITY;
  }
  const bool lead = (q == 0) && (k < a.N);
  if (lead) {
    if (RECORD) {
      a.per_m[(size_t)c * a.N + k] = best;
      a.per_j[(size_t)c * a.N + k] = jb;
    }
    if (CHANCE) a.per_key[(size_t)c * a.N + k] = ord64((double)best);
    if (best < -a.band) {
      if (!CHANCE || (!counted && atomicAdd(&S->nviol[c], 1) >= S->q))
        __hip_atomic_store(&S->dead[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (best < a.band && !stopped && !spec) {  // a speculative probe is never rechecked
      const int idx = atomicAdd(&S->n_recheck, 1);
      a.rlist[idx] = make_int2(c, k);
    }
  }
  const unsigned long long key = lead ? lane_key(best, k) : ~0ull;
  const unsigned long long kall = block_min_u64(key, sh);
  const unsigned long long kfar = block_min_u64((lead && best >= a.band) ? key : ~0ull, sh);
  int wsum = lead ? ns : 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(&S->lane_steps, (unsigned long long)wsum);
  if (threadIdx.x == 0) {
    atomicMin(&S->key_all[c], kall);
    if (kfar != ~0ull) atomicMin(&S->key_far[c], kfar);
  }
}

// FP64 re-simulation of the near-band list, LQ4 with one entry per quad of
// lanes (the layout of the FP32 quad rollout, in double precision: a 64-bit
// DPP exchange is two 32-bit ones).  Same verdict as the one-lane recheck.
struct QuadCoef64 {
  double a[4][4], g[4][4], d[4][4];
  double b[4];
  double e[4][2];
  double grow[4];
};

__device__ __forceinline__ double min2d(double a, double b) { return b < a ? b : a; }

__device__ __forceinline__ double quad_min64(double m) {
  m = min2d(m, dpp64<kSwap1>(m));
  return min2d(m, dpp64<kSwap2>(m));
}

template <int RNG, int INJ>
__global__ void __launch_bounds__(256) k_recheck_lq4_quad(const RollArgs<1, double> a,
                                                         const QuadCoef64 qc,
                                                         const CtlArgs<1> ctl, int decide) {
  constexpr int U = kQuadGroup;
  DevSearch* S = a.srch;
  if (S->done) return;
  const int n = S->n_recheck;
  const uint32_t t = a.st->t;
  const int q = threadIdx.x & 3;
  const double A0 = qc.a[q][0], A1 = qc.a[q][1], A2 = qc.a[q][2], A3 = qc.a[q][3];
  const double G0 = qc.g[q][0], G1 = qc.g[q][1], G2 = qc.g[q][2], G3 = qc.g[q][3];
  const double d0 = qc.d[q][0], d1 = qc.d[q][1], d2 = qc.d[q][2], d3 = qc.d[q][3];
  const double e0 = qc.e[q][0], e1 = qc.e[q][1], grow = qc.grow[q], bq = qc.b[q];
  const double h = a.h, hh = a.hh, h6 = a.h6;
  const int H = a.H;
  const uint32_t row_bytes = 8u * (uint32_t)a.N;
  const __amdgpu_buffer_rsrc_t wres = __builtin_amdgcn_make_buffer_rsrc(
      (void*)step_w(a, t), (short)0, (int)(row_bytes * (uint32_t)(H + U)), 0x00020000);
  const int stride = (int)((gridDim.x * blockDim.x) >> 2);
  // chance-constrained verdict (qv > 0): one FP64 violation refuses the
  // candidate only once more than qv scenarios violate, so an entry does not
  // stop on another's, and every entry keeps its margin key
  const int qv = S->q;
  // every lane of a quad holds the same entry, so all exits are quad-uniform
  for (int i = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 2); i < n; i += stride) {
    const int2 en = a.rlist[i];
    const int c = en.x, k = en.y;
    if (a.early &&
        (__hip_atomic_load(&S->dead[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
         __hip_atomic_load(&S->fail64[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)))
      continue;
    const double bv = bq * S->v[c];
    double x = a.st->x[q];
    auto deriv = [&](double s, double xv) {
      const double c2 = __builtin_fma(G2, xv, A2) * xv;
      const double c3 = __builtin_fma(G3, xv, A3) * xv;
      double c0 = __builtin_fma(__builtin_fma(G0, xv, A0), xv, s);
      double c1 = __builtin_fma(G1, xv, A1) * xv;
      c1 = c1 + dpp64<kSwap2>(c3);
      c0 = c0 + dpp64<kSwap2>(c2);
      return c0 + dpp64<kSwap1>(c1);
    };
    auto row_margin = [&](double xv) {
      const double c2 = d2 * xv, c3 = d3 * xv;
      double c0 = __builtin_fma(d0, xv, grow);
      double c1 = d1 * xv;
      c1 = c1 + dpp64<kSwap2>(c3);
      c0 = c0 + dpp64<kSwap2>(c2);
      return c0 + dpp64<kSwap1>(c1);
    };
    double bm = row_margin(x);  // lane q: running minimum of row q
    const uint32_t vo0 = 4u * (uint32_t)k, vo1 = vo0 + 4u * (uint32_t)a.N;
    uint32_t so = 0;
    auto load_group = [&](int j, float* w) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (RNG == 0) {
          const uint32_t sr = so + (uint32_t)u * row_bytes;
          w[2 * u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(wres, vo0, sr, 0));
          w[2 * u + 1] =
              __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(wres, vo1, sr, 0));
        } else {
          const Words r = philox10((uint32_t)k, (uint32_t)(j + u), t, 0u, a.seed, a.inst);
          w[2 * u] = box_draw(r.v[0], a.wlo[0], a.wspan[0]);
          w[2 * u + 1] = box_draw(r.v[1], a.wlo[1], a.wspan[1]);
        }
      }
      if (RNG == 0) so += (uint32_t)U * row_bytes;
    };
    auto step = [&](float w0f, float w1f) {
      const double w0 = (double)w0f, w1 = (double)w1f;
      const double s = INJ == 0 ? __builtin_fma(e1, w1, __builtin_fma(e0, w0, bv)) : bv;
      const double k1 = deriv(s, x);
      double acc = k1;
      double xs = __builtin_fma(hh, k1, x);
      const double k2 = deriv(s, xs);
      acc = __builtin_fma(2.0, k2, acc);
      xs = __builtin_fma(hh, k2, x);
      const double k3 = deriv(s, xs);
      acc = __builtin_fma(2.0, k3, acc);
      xs = __builtin_fma(h, k3, x);
      const double k4 = deriv(s, xs);
      x = __builtin_fma(h6, acc + k4, x);
      if (INJ == 1) x = x + (e0 * w0 + e1 * w1);
      bm = fmin(bm, row_margin(x));
    };
    float wcur[2 * U], wnext[2 * U];
    load_group(0, wcur);
    const int full = H / U;
    int g = 0;
    for (; g < full; ++g) {
      load_group((g + 1) * U, wnext);
#pragma unroll
      for (int u = 0; u < U; ++u) step(wcur[2 * u], wcur[2 * u + 1]);
#pragma unroll
      for (int u = 0; u < 2 * U; ++u) wcur[u] = wnext[u];
      if (a.early) {
        if (quad_min64(bm) < 0.0) {
          ++g;
          break;
        }
        if ((g & 7) == 7 && qv == 0 &&
            __hip_atomic_load(&S->fail64[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          break;
      }
    }
    if (g == full)
      for (int u = 0; u < H - full * U; ++u) step(wcur[2 * u], wcur[2 * u + 1]);
    double m = quad_min64(bm);
    double bad = x - x;
    bad = bad + dpp64<kSwap1>(bad);
    bad = bad + dpp64<kSwap2>(bad);
    if (!(bad == 0.0) || m != m) m = -INFINITY;
    if (q == 0) {
      atomicMin(&S->key64[c], ord64(m));
      if (qv > 0) {
        a.per_key[(size_t)c * a.N + k] = ord64(m);
        if (m < 0.0 && S->nviol[c] + atomicAdd(&S->nviol64[c], 1) >= qv)
          __hip_atomic_store(&S->fail64[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if (m < 0.0) {
        __hip_atomic_store(&S->fail64[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  if (decide) last_block_decides<1>(ctl);
}

// FP64 re-simulation of the near-band list.
template <int KIND, int RNG, int INJ>
__global__ void __launch_bounds__(64) k_recheck(const RollArgs<KIND, double> a,
                                                const CtlArgs<KIND> ctl, int decide) {
  DevSearch* S = a.srch;
  if (S->done) return;
  const int n = S->n_recheck;
  const uint32_t t = a.st->t;
  if constexpr (KIND == 2) {
    // up to two entries per group of 16 lanes: the cooperative rollout
    const int groups = (int)(gridDim.x * blockDim.x) >> 4;
    if (n <= 2 * groups) {
      recheck_fc9_groups<RNG, INJ>(a, S, n, t, (int)(blockIdx.x * blockDim.x + threadIdx.x) >> 4,
                                   groups);
      if (decide) last_block_decides<KIND>(ctl);
      return;
    }
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int2 e = a.rlist[i];
    const int c = e.x, k = e.y;
    // The verdict needs one failing lane only, also for a candidate whose FP32
    // rollout ran in full (the Newton iterate): its rechecks stop at the first
    // FP64 violation too.
    if (a.early &&
        (__hip_atomic_load(&S->dead[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
         __hip_atomic_load(&S->fail64[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)))
      continue;
    int jb = 0, ns = 0;
    const int early = a.early;
    const int q = S->q;
    // chance-constrained verdict: one FP64 violation refuses the candidate only
    // once more than q scenarios violate, so the lane does not stop on others'
    const double m = rollout_lane<KIND, double, RNG, INJ>(
        a, early, S->v[c], k, t, early && q == 0 ? &S->fail64[c] : nullptr, jb, ns, nullptr);
    atomicMin(&S->key64[c], ord64(m));
    if (q > 0) {
      a.per_key[(size_t)c * a.N + k] = ord64(m);
      if (m < 0.0 && S->nviol[c] + atomicAdd(&S->nviol64[c], 1) >= q)
        __hip_atomic_store(&S->fail64[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (m < 0.0) {
      __hip_atomic_store(&S->fail64[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (decide) last_block_decides<KIND>(ctl);
}

// Batched serving: the FP64 recheck of every instance of a group in one launch,
// one workgroup per instance (its own near-band list, as k_recheck), which then
// takes that instance's decision for the round (as the last workgroup of
// k_recheck does).  The workgroup's own rechecks are published by a
// device-scope fence before the decision reads the verdicts.
template <int KIND, int INJ>
__global__ void __launch_bounds__(64) k_flat_recheck(const RollArgs<KIND, double>* __restrict__ args,
                                                     const CtlArgs<KIND>* __restrict__ ctl) {
  const RollArgs<KIND, double>& a = args[blockIdx.x];
  DevSearch* S = a.srch;
  if (S->done) return;  // uniform: nothing writes it before the decision below
  const int n = S->n_recheck;
  const uint32_t t = a.st->t;
  if constexpr (KIND == 2) {
    // few entries: the cooperative rollout, four groups of 16 lanes
    if (n <= 8) {
      recheck_fc9_groups<1, INJ>(a, S, n, t, (int)threadIdx.x >> 4, (int)blockDim.x >> 4);
      __threadfence();
      __syncthreads();
      const CtlArgs<KIND>& cl = ctl[blockIdx.x];
      decide_body<KIND>(cl.pc, cl.st, cl.srch, cl.grad);
      return;
    }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int2 e = a.rlist[i];
    const int c = e.x, k = e.y;
    if (a.early &&
        (__hip_atomic_load(&S->dead[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
         __hip_atomic_load(&S->fail64[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)))
      continue;
    int jb = 0, ns = 0;
    const double m = rollout_lane<KIND, double, 1, INJ>(
        a, a.early, S->v[c], k, t, a.early ? &S->fail64[c] : nullptr, jb, ns, nullptr);
    atomicMin(&S->key64[c], ord64(m));
    if (m < 0.0) __hip_atomic_store(&S->fail64[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __threadfence();
  __syncthreads();
  const CtlArgs<KIND>& cl = ctl[blockIdx.x];
  decide_body<KIND>(cl.pc, cl.st, cl.srch, cl.grad);
}

// Batched serving: round-0 setup of every instance of a group, one workgroup
// per instance (as k_setup).
template <int KIND>
__global__ void __launch_bounds__(128) k_flat_setup(const CtlArgs<KIND>* __restrict__ ctl) {
  const CtlArgs<KIND>& a = ctl[blockIdx.x];
  setup_body<KIND>(a.pc, a.st, a.srch, a.r_seq, a.closed_loop);
}

// Batched serving: the result record of every instance of a group (as
// k_finalize outside the closed loop), one thread per instance.
template <int KIND>
__global__ void k_flat_finalize(const CtlArgs<KIND>* __restrict__ ctl, DevResult* const* __restrict__ res,
                                int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const DevSearch* S = ctl[i].srch;
  DevState* st = ctl[i].st;
  DevResult R;
  R.kappa = S->kappa_res;
  R.v = S->v_res;
  R.worst = S->worst_res;
  R.status = S->status;
  R.rounds = S->rounds_total;
  R.candidates = S->cand_total;
  R.rechecks = S->rechecks_total;
  R.passes_alg1 = S->passes_alg1;
  R.t = st->t;
  R.lane_steps = S->lane_steps;
  R.flags = S->flags;
  *res[i] = R;
  st->t = st->t + 1;
}

// ---------------------------------------------------------------------------
// Candidates, steady state, verdicts
// ---------------------------------------------------------------------------

// Eq. (2) with v = r exactly at kappa = 1.  Contraction is off here: the value
// is the three-rounding expression v_prev + kappa (r - v_prev), never an FMA.
__device__ __forceinline__ double cand_v(double kappa, double r, double v_prev) {
#pragma clang fp contract(off)
  if (kappa == 1.0) return r;
  const double d = r - v_prev;
  const double p = kappa * d;
  return v_prev + p;
}

__device__ __forceinline__ double midpoint(double a, double b) {
#pragma clang fp contract(off)
  return (a + b) * 0.5;
}

// Tightened right-hand side g - eps |g| (two roundings, no FMA).
__device__ __forceinline__ double tightened_rhs(double g, double eps) {
#pragma clang fp contract(off)
  const double e = eps * fabs(g);
  return g - e;
}

template <int NN>
__device__ bool dense_solve(double* J, double* b) {
  for (int c = 0; c < NN; ++c) {
    int piv = c;
    for (int r = c + 1; r < NN; ++r)
      if (fabs(J[r * NN + c]) > fabs(J[piv * NN + c])) piv = r;
    if (!(fabs(J[piv * NN + c]) > 1e-300)) return false;
    if (piv != c) {
      for (int q = 0; q < NN; ++q) {
        const double tmp = J[c * NN + q];
        J[c * NN + q] = J[piv * NN + q];
        J[piv * NN + q] = tmp;
      }
      const double tmp = b[c];
      b[c] = b[piv];
      b[piv] = tmp;
    }
    for (int r = c + 1; r < NN; ++r) {
      const double f = J[r * NN + c] / J[c * NN + c];
      for (int q = c; q < NN; ++q) J[r * NN + q] -= f * J[c * NN + q];
      b[r] -= f * b[c];
    }
  }
  for (int c = NN - 1; c >= 0; --c) {
    double s = b[c];
    for (int q = c + 1; q < NN; ++q) s -= J[c * NN + q] * b[q];
    b[c] = s / J[c * NN + c];
  }
  return true;
}

// Tightened steady-state margin min_r (g_r - eps |g_r| - F_r y_ss(v)) with the
// equilibrium from Newton's method (nominal coefficients, w = 0); failure to
// reach ||f||_inf <= 1e-12 within 50 iterations gives -inf.
template <int KIND>
__device__ double steady_margin(const typename Plant<KIND, double>::Coef& pc, const DevSearch* S,
                                double v) {
  using P = Plant<KIND, double>;
  if (!S->ss_check) return INFINITY;
  double x[P::n], f[P::n], J[P::n * P::n], s0[P::n];
  P::eq_guess(pc, v, x, J);
  if (P::eq_guess_needs_solve()) {
    if (!dense_solve<P::n>(J, x)) return -INFINITY;
  }
  typename P::Lane L;
  P::lane_init(pc, P::nominal_theta(pc), v, L);
  P::force0(pc, L, s0);
  bool ok = false;
  for (int it = 0; it <= 50; ++it) {
    P::deriv(pc, L, s0, x, f);
    double nrm = 0.0;
    for (int i = 0; i < P::n; ++i) {
      if (!isfinite(f[i])) return -INFINITY;
      nrm = fmax(nrm, fabs(f[i]));
    }
    if (nrm <= 1e-12) {
      ok = true;
      break;
    }
    if (it == 50) break;
    P::jacobian(pc, x, v, J);
    for (int i = 0; i < P::n; ++i) f[i] = -f[i];
    if (!dense_solve<P::n>(J, f)) return -INFINITY;
    for (int i = 0; i < P::n; ++i) x[i] += f[i];
  }
  if (!ok) return -INFINITY;
  double y[P::ny];
  P::output(pc, L, x, y);
  double best = INFINITY;
  for (int r = 0; r < S->n_c; ++r) {
    double fy = 0.0;
    for (int i = 0; i < P::ny; ++i) fy += S->F[r * P::ny + i] * y[i];
    const double gt = tightened_rhs(S->g[r], S->eps);
    const double m = gt - fy;
    best = (m < best || m != m) ? m : best;
  }
  return (best == best) ? best : -INFINITY;
}

__device__ __forceinline__ bool cand_feasible(const DevSearch* S, int c) {
  return !S->dead[c] && !S->fail64[c] && S->mss[c] >= 0.0;
}

__device__ __forceinline__ double cand_worst_p(const DevSearch* S, int c, int precision) {
  if (S->q > 0) {  // chance-constrained: the (q + 1)-th smallest scenario margin
    const double wq = S->keyq[c] == ~0ull ? INFINITY : unord64(S->keyq[c]);
    return (S->mss[c] < wq) ? S->mss[c] : wq;
  }
  double w;
  const double kall = S->key_all[c] == ~0ull ? INFINITY : key_margin(S->key_all[c], precision);
  if (S->dead[c] || S->key64[c] == ~0ull) {
    w = kall;
  } else {
    const double far = S->key_far[c] == ~0ull ? INFINITY : key_margin(S->key_far[c], precision);
    const double r64 = unord64(S->key64[c]);
    w = far < r64 ? far : r64;
  }
  const double ms = S->mss[c];
  return (ms < w) ? ms : w;
}

__device__ __forceinline__ double cand_worst(const DevSearch* S, int c) {
  return cand_worst_p(S, c, S->precision);
}

// Lay out a speculative bisection tree of `depth` levels over (lo, hi) at
// candidates base.. (breadth-first; node q has children 2q+1 and 2q+2).
__device__ void build_tree(DevSearch* S, int base, int depth, double lo, double hi) {
  const int nn = (1 << depth) - 1;
  S->a_lo[base] = lo;
  S->a_hi[base] = hi;
  S->kappa[base] = midpoint(lo, hi);
  for (int q = 0; q < nn; ++q) {
    const int c = base + q;
    const double kq = S->kappa[c];
    const int l = 2 * q + 1, r = 2 * q + 2;
    if (l < nn) {
      S->a_lo[base + l] = S->a_lo[c];
      S->a_hi[base + l] = kq;
      S->kappa[base + l] = midpoint(S->a_lo[c], kq);
    }
    if (r < nn) {
      S->a_lo[base + r] = kq;
      S->a_hi[base + r] = S->a_hi[c];
      S->kappa[base + r] = midpoint(kq, S->a_hi[c]);
    }
  }
  S->tree_base = base;
  S->tree_depth = depth;
}

// Thread-parallel per-candidate preparation: set-points, steady-state margins,
// reduction accumulators.
// Steady-state margins come from a small cache of recent set-points when
// possible (the same v recurs from one RG step to the next while the governor
// holds v or has reached r).
template <int KIND>
__device__ void prepare_candidates(const typename Plant<KIND, double>::Coef& pc, const DevState* st,
                                   DevSearch* S) {
  const double r = st->r, vp = st->v_prev;
  __shared__ double s_cv[kMssCache], s_cm[kMssCache], s_v[kCMax];
  __shared__ int s_miss[kCMax];
  for (int i = threadIdx.x; i < kMssCache; i += blockDim.x) {
    s_cv[i] = S->mss_v[i];
    s_cm[i] = S->mss_m[i];
  }
  __syncthreads();
  const int n = S->n_cand;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    if (S->mode != kNewton) S->full[c] = 0;
    // a speculative candidate of step t + j: that step's reference; its v_prev
    // is this step's (holds), or any (kappa = 1 gives v = r)
    const int sj = cand_step(S, c);
    const double v = cand_v(S->kappa[c], sj ? S->r_spec[sj - 1] : r, vp);
    S->v[c] = v;
    int hit = -1;
    for (int i = 0; i < kMssCache; ++i) {
      if (s_cv[i] == v) {
        hit = i;
        break;
      }
    }
    S->mss[c] = hit >= 0 ? s_cm[hit] : steady_margin<KIND>(pc, S, v);
    if (c < kCMax) {
      s_miss[c] = hit < 0;
      s_v[c] = v;
    }
    S->key_all[c] = ~0ull;
    S->key_far[c] = ~0ull;
    S->key64[c] = ~0ull;
    S->dead[c] = 0;
    S->fail64[c] = 0;
    S->nviol[c] = 0;
    S->nviol64[c] = 0;
    S->keyq[c] = ~0ull;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    S->n_recheck = 0;
    int next = S->mss_next;
    for (int c = 0; c < n && c < kCMax; ++c) {
      if (!s_miss[c]) continue;
      const double v = s_v[c];
      bool dup = false;  // the same set-point twice in one round
      for (int e = 0; e < c; ++e) dup = dup || (s_miss[e] && s_v[e] == v);
      if (dup) continue;
      S->mss_v[next] = v;
      S->mss_m[next] = S->mss[c];
      next = (next + 1) % kMssCache;
    }
    S->mss_next = next;
  }
}

// Start of one RG step: round-0 candidates.
template <int KIND>
__device__ void setup_body(const typename Plant<KIND, double>::Coef& pc, DevState* st,
                           DevSearch* S, const double* r_seq, int closed_loop,
                           const RollArgs<KIND, double>* pa = nullptr) {
  if (threadIdx.x == 0) {
    if (closed_loop) st->r = r_seq[st->cl_index];
    // Was this step's first round already evaluated by an earlier round
    // (speculatively, from the state this step starts in if the steps before
    // it did as assumed)?  A speculative candidate never gets an FP64 recheck,
    // so its verdict counts only when it is certain without one: refused by a
    // lane below -band or by the steady-state test, or admitted with every
    // scenario's FP32 margin at least the band.  The result is then the one
    // Alg. 1 reaches from those verdicts: kappa = 1 if the probe is admitted;
    // after holds, kappa = 0 if the probe and every midpoint towards 0 are
    // refused, or 2^-K if only the last is admitted.
    bool decided = false;
    int spec_found = 0, spec_passes = 0;
    double spec_kappa = 0.0, spec_worst = -INFINITY;
    if (closed_loop && S->done && S->spec_used < S->spec_n) {
      const int base = S->spec_base + S->spec_used * S->spec_per;
      auto kall_of = [&](int c) {
        return S->key_all[c] == ~0ull ? INFINITY : key_margin(S->key_all[c], S->precision);
      };
      auto verdict = [&](int c) {  // 1 admitted, 0 refused, -1 not certain
        if (S->fail64[c]) return -1;
        if (S->dead[c] || S->mss[c] < 0.0) return 0;
        return kall_of(c) >= S->band ? 1 : -1;
      };
      // certain admission: every scenario's FP32 margin at least the band, so
      // no scenario violates (also under the chance-constrained verdict, whose
      // worst margin is the order statistic the round selected)
      auto admit = [&](int c, int passes) {
        decided = true;
        spec_found = 1;
        spec_kappa = S->kappa[c];
        const double kall = kall_of(c);
        spec_worst = S->q > 0 ? cand_worst(S, c) : (kall < S->mss[c] ? kall : S->mss[c]);
        spec_passes = passes;
      };
      if (S->spec_kind == 1) {
        if (S->kappa_res == 1.0 && verdict(base) == 1) admit(base, 1);
      } else if (S->kappa_res == 0.0) {  // the previous step held v
        const int vb = verdict(base);
        if (vb == 1) {
          admit(base, 1);
        } else if (vb == 0) {
          const int K = S->K;
          int l = 1;
          while (l <= K && verdict(base + l) == 0) ++l;
          if (l > K) {
            decided = true;
            spec_passes = 1 + K;
          } else if (l == K && verdict(base + K) == 1) {
            admit(base + K, 1 + K);
          }
        }
      }
      if (decided) S->spec_used += 1;
    }
    if (!decided) {
      S->spec_n = 0;
      S->spec_used = 0;
    }
    S->done = 0;
    S->found = 0;
    S->status = 0;
    S->round = 0;
    S->halvings = 0;
    S->lo = 0.0;
    S->hi = 1.0;
    S->kappa_res = 0.0;
    S->v_res = st->v_prev;
    S->worst_res = -INFINITY;
    S->cand_total = 0;
    S->rechecks_total = 0;
    S->rounds_total = 0;
    S->passes_alg1 = 0;
    S->lane_steps = 0ull;
    S->fallbacks = 0;
    S->flags = 0;
    if (decided) {
      S->done = 1;
      S->found = spec_found;
      S->status = spec_found ? 0 : 1;
      S->lo = spec_kappa;
      S->kappa_res = spec_kappa;
      S->pred = spec_kappa;
      S->v_res = spec_found ? cand_v(spec_kappa, st->r, st->v_prev) : st->v_prev;
      S->worst_res = spec_worst;
      S->passes_alg1 = spec_passes;
      S->n_cand = 0;
    } else if (S->mode == kNewton) {
      S->kappa[0] = 1.0;  // probe, carries the first derivative
      S->kappa[1] = 0.5;
      S->full[0] = 1;
      S->full[1] = 0;
      int n = 2;
      // Prediction after a step that held v (kappa = 0): the round also runs
      // the midpoints 2^-2 .. 2^-K of the bisection path towards 0.  When they
      // are all refused, as every candidate of that path, the result is
      // kappa = 0, the result of bisection itself; otherwise their verdicts
      // narrow the bracket the Newton steps start from.  Such a round has no
      // iterate (index -1) and takes no derivative: the probe stops at its
      // first violation like the others, and the next round, if any, starts
      // from the bracket's midpoint.
      const double pr = S->pred;
      const bool held = S->predict && pr == 0.0;
      if (held) {
        double m = 0.5;
        for (int l = 2; l <= S->K && n < kCMax; ++l) {
          m = midpoint(0.0, m);
          S->kappa[n] = m;
          S->full[n++] = 0;
        }
        S->full[0] = 0;
      }
      S->n_cand = n;
      S->nk_idx = held ? -1 : 0;
      S->probe = 1;
      S->tree_depth = 0;
      S->goal = S->K;
    } else if (S->mode == kGrid) {
      const int M = S->M;
      for (int i = 0; i < M; ++i) S->kappa[i] = (M > 1) ? (double)i / (double)(M - 1) : 1.0;
      S->n_cand = M;
      S->probe = 0;
      S->tree_depth = 0;
      S->goal = S->refine;
    } else {
      S->kappa[0] = 1.0;
      S->probe = 1;
      S->goal = S->K;
      const double pr = S->pred;
      if (S->predict && pr == pr && S->K > 0) {
        // Speculate along the previous step's result: the kappa = 1 probe alone
        // when it was 1, else every midpoint on the bisection path towards it.
        // The decision still takes each level's verdict from its own midpoint,
        // so the result is that of sequential bisection whatever the guess.
        S->tree_depth = 0;
        if (pr >= 1.0) {
          S->n_cand = 1;
          // The probe alone fills few SIMDs: the round also runs the next
          // step's probe, from the state the next step starts in if this
          // step's kappa is 1 (the same FP64 true-plant step as the result
          // launch), under the next step's draws.
          int d = pa && closed_loop ? S->spec_depth : 0;
          if (d > st->cl_len - 1 - st->cl_index) d = st->cl_len - 1 - st->cl_index;
          for (int j = 1; j <= d; ++j) {
            const double* xp = j == 1 ? st->x : S->x_spec[j - 2];
            const double rp = j == 1 ? st->r : S->r_spec[j - 2];
            true_plant_step<KIND>(*pa, xp, rp, st->t + (uint32_t)(j - 1), S->x_spec[j - 1]);
            S->r_spec[j - 1] = r_seq[st->cl_index + j];
            S->kappa[j] = 1.0;  // a later step's probe (the walk reads own candidates only)
          }
          if (d > 0) {
            S->spec_kind = 1;
            S->spec_base = 1;
            S->spec_per = 1;
            S->spec_n = d;
            S->spec_used = 0;
            S->n_cand = 1 + d;
          }
        } else {
          double lo = 0.0, hi = 1.0;
          for (int l = 0; l < S->K; ++l) {
            const double m = midpoint(lo, hi);
            S->kappa[1 + l] = m;
            if (pr >= m) lo = m;
            else hi = m;
          }
          S->n_cand = 1 + S->K;
          // The governor held v (kappa = 0): the round also runs the first
          // rounds of the next steps (probe and midpoints towards 0), from the
          // states they start in if they hold v too (the same FP64 true-plant
          // steps as the result launch), under their draws.  Their tails run
          // beside this step's on SIMDs the step alone leaves idle.
          int d = pa && closed_loop && pr == 0.0 ? S->spec_hold : 0;
          if (d > st->cl_len - 1 - st->cl_index) d = st->cl_len - 1 - st->cl_index;
          const int per = 1 + S->K;
          for (int j = 1; j <= d; ++j) {
            const double* xp = j == 1 ? st->x : S->x_spec[j - 2];
            true_plant_step<KIND>(*pa, xp, st->v_prev, st->t + (uint32_t)(j - 1), S->x_spec[j - 1]);
            S->r_spec[j - 1] = r_seq[st->cl_index + j];
            const int b = per * j;
            double h = 1.0;
            S->kappa[b] = 1.0;
            for (int l = 1; l <= S->K; ++l) {
              h = midpoint(0.0, h);
              S->kappa[b + l] = h;
            }
          }
          if (d > 0) {
            S->spec_kind = 2;
            S->spec_base = per;
            S->spec_per = per;
            S->spec_n = d;
            S->spec_used = 0;
            S->n_cand = per * (1 + d);
          }
        }
      } else {
        const int d0 = S->K < S->depth ? S->K : S->depth;
        if (d0 > 0) build_tree(S, 1, d0, 0.0, 1.0);
        else S->tree_depth = 0;
        S->n_cand = 1 + ((1 << d0) - 1);
      }
    }
    if (closed_loop) {
      // Draws of the ring.  Rounds of step t read steps t .. t + kSpecMax, so
      // its first round must leave step t + kSpecMax + 1 generated for the
      // next step.  A round with candidates (long, with SIMDs idle in its
      // tail) generates as far as the ring allows, t + kPairs - 1; a step
      // decided ahead, whose launch has nothing else to do, only what is
      // missing.  Nothing past the chunk's last step.  The chunk's prologue
      // generated t .. t + kSpecMax.
      const uint32_t t = st->t;
      if (st->cl_index == 0) st->gen_hi = t + (uint32_t)kSpecMax;
      uint32_t want = t + (uint32_t)(S->n_cand > 0 ? kPairs - 1 : kSpecMax + 1);
      const uint32_t last = t + (uint32_t)(st->cl_len - 1 - st->cl_index);
      if (want > last) want = last;
      const uint32_t lo = st->gen_hi + 1u;
      st->gen_lo = lo;
      st->gen_n = want >= lo ? (int32_t)(want - lo + 1u) : 0;
      if (want >= lo) st->gen_hi = want;
    }
  }
  __syncthreads();
  prepare_candidates<KIND>(pc, st, S);
}

template <int KIND>
__global__ void __launch_bounds__(128) k_setup(const CtlArgs<KIND> a) {
  setup_body<KIND>(a.pc, a.st, a.srch, a.r_seq, a.closed_loop);
}

// rg_margin: explicit candidate list (kappa[] already uploaded).
template <int KIND>
__global__ void __launch_bounds__(128) k_setup_list(const CtlArgs<KIND> a, int M) {
  DevSearch* S = a.srch;
  if (threadIdx.x == 0) {
    S->done = 0;
    S->n_cand = M;
    S->round = 0;
  }
  __syncthreads();
  prepare_candidates<KIND>(a.pc, a.st, S);
}

// Safeguarded Newton on phi(kappa) = M(kappa): the verdicts of round 0 give
// the bracket bisection has after them, every later verdict tightens
// [lo, hi]; the next iterate is kappa_c - phi/phi' from this round's iterate
// (adjoint derivative), moved to lo + delta or hi - delta when it lands at or
// past that end, and the midpoint when the slope is not negative or not
// finite; candidates kappa_N -/+ delta and the midpoint go with it.
// Returns true when hi - lo <= delta (or the round cap K + 2 is reached).
__device__ bool newton_decide(DevSearch* S, const DevGrad* G) {
  const double delta = S->delta;
  S->passes_alg1 += S->n_cand;
  if (S->round == 0 && cand_feasible(S, 0)) {
    S->found = 1;
    S->lo = 1.0;
    S->worst_res = cand_worst(S, 0);
    return true;
  }
  if (S->round == 0) {
    // Round 0 holds the probe and midpoints of the bisection path (0.5, and
    // after a held step every midpoint towards 0): walk them as bisection does,
    // each level taking the verdict of its own midpoint, which needs no
    // monotonicity of the verdicts.
    double lo = S->lo, hi = S->hi;
    for (;;) {
      const double m = midpoint(lo, hi);
      int c = -1;
      for (int i = 1; i < S->n_cand; ++i) {
        if (S->kappa[i] == m) {
          c = i;
          break;
        }
      }
      if (c < 0) break;
      if (cand_feasible(S, c)) {
        lo = m;
        S->found = 1;
        S->worst_res = cand_worst(S, c);
      } else {
        hi = m;
      }
      if (hi - lo <= delta) break;
    }
    S->lo = lo;
    S->hi = hi;
  } else {
    for (int c = 0; c < S->n_cand; ++c) {
      const double kc = S->kappa[c];
      if (cand_feasible(S, c)) {
        if (kc > S->lo || (!S->found && kc >= S->lo)) {
          S->lo = kc;
          S->found = 1;
          S->worst_res = cand_worst(S, c);
        }
      } else if (kc < S->hi) {
        S->hi = kc;
      }
    }
  }
  if (S->hi - S->lo <= delta || S->round + 1 >= S->K + 2) return true;
  // no iterate this round (a held step's first round): a midpoint step,
  // which is no fallback
  const bool iterate = S->nk_idx >= 0;
  const double kap_c = iterate ? S->kappa[S->nk_idx] : 0.0;
  const double phi = G->M, dphi = G->dM_dkappa;
  bool ok = iterate && (phi == phi) && (dphi == dphi) && isfinite(phi) && isfinite(dphi) &&
            dphi < 0.0;
  double kn = ok ? kap_c - phi / dphi : 0.5 * (S->lo + S->hi);
  // a step at or past a bracket end moves just inside that end (the root is next to it)
  if (ok && kn <= S->lo) kn = S->lo + delta;
  else if (ok && kn >= S->hi) kn = S->hi - delta;
  if (!(kn > S->lo && kn < S->hi)) {
    kn = 0.5 * (S->lo + S->hi);
    ok = false;
  }
  if (!ok && iterate) S->fallbacks += 1;
  const double cand[4] = {kn, kn - delta, kn + delta, 0.5 * (S->lo + S->hi)};
  int n = 0;
  for (int i = 0; i < 4; ++i) {
    if (i > 0 && !(cand[i] > S->lo && cand[i] < S->hi)) continue;
    S->kappa[n] = cand[i];
    S->full[n] = (i == 0);
    ++n;
  }
  S->n_cand = n;
  S->nk_idx = 0;
  return false;
}

// Verdicts of the finished round, bracket update, next round.
template <int KIND>
__device__ void decide_body(const typename Plant<KIND, double>::Coef& pc, const DevState* st,
                            DevSearch* S, const DevGrad* grad) {
  // Thread 0 may set S->done below: take the entry decision once, for the whole
  // workgroup, so every wave reaches the same barriers.  The verdicts and worst
  // margins of the round's candidates are staged in LDS by all threads first,
  // so the sequential walk below reads no global memory in its loop.
  __shared__ int s_done, s_n;
  __shared__ double s_kappa[kCMax], s_worst[kCMax];
  __shared__ unsigned char s_ok[kCMax], s_own[kCMax];
  if (threadIdx.x == 0) {
    s_done = S->done;
    s_n = S->n_cand < kCMax ? S->n_cand : kCMax;
  }
  __syncthreads();
  if (s_done) return;
  if (S->mode != kNewton) {
    for (int c = threadIdx.x; c < s_n; c += blockDim.x) {
      s_kappa[c] = S->kappa[c];
      s_ok[c] = cand_feasible(S, c) ? 1 : 0;
      s_worst[c] = cand_worst(S, c);
      s_own[c] = cand_step(S, c) == 0 ? 1 : 0;  // not a later step's speculative candidate
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    S->rounds_total += 1;
    S->cand_total += S->n_cand;
    S->rechecks_total += S->n_recheck;
    bool finished = false;
    if (S->mode == kNewton) {
      finished = newton_decide(S, grad);
    } else if (S->mode == kGrid && S->round == 0) {
      const int M = S->M;
      int istar = -1;
      for (int i = 0; i < M; ++i)
        if (s_ok[i]) istar = i;
      // Eq. (5) takes the largest all-admissible row even when a row below it
      // was refused; say so in the step's diagnostics
      for (int i = 0; i < istar; ++i)
        if (!s_ok[i]) S->flags |= 1;
      S->passes_alg1 += M;
      if (istar < 0) {
        finished = true;
      } else {
        S->found = 1;
        S->worst_res = s_worst[istar];
        S->lo = s_kappa[istar];
        if (istar == M - 1) {
          finished = true;
        } else {
          S->hi = s_kappa[istar + 1];
          if (S->goal <= 0) finished = true;
        }
      }
    } else {
      double lo = S->lo, hi = S->hi, worst = S->worst_res;
      int halvings = S->halvings, passes = S->passes_alg1, found = S->found;
      const int probe = S->probe, goal = S->goal, n = s_n;
      if (probe) {
        passes += 1;
        if (s_ok[0]) {
          found = 1;
          lo = 1.0;
          worst = s_worst[0];
          finished = true;
        }
      }
      if (!finished) {
        // Sequential bisection over this round's candidates: each level takes
        // the verdict of the candidate equal to the current midpoint (dyadic
        // midpoints are exact, so equality identifies the node), until a
        // midpoint was not evaluated this round.
        while (halvings < goal) {
          const double m = midpoint(lo, hi);
          int c = -1;
          for (int i = probe; i < n; ++i) {
            if (s_kappa[i] == m && s_own[i]) {
              c = i;
              break;
            }
          }
          if (c < 0) break;
          passes += 1;
          if (s_ok[c]) {
            lo = m;
            found = 1;
            worst = s_worst[c];
          } else {
            hi = m;
          }
          halvings += 1;
        }
        if (halvings >= goal) finished = true;
      }
      S->lo = lo;
      S->hi = hi;
      S->worst_res = worst;
      S->halvings = halvings;
      S->passes_alg1 = passes;
      S->found = found;
    }
    if (finished) {
      S->done = 1;
      S->status = S->found ? (S->mode == kNewton && S->fallbacks > 0 ? 2 : 0) : 1;
      S->kappa_res = S->found ? S->lo : 0.0;
      S->pred = S->kappa_res;
      S->v_res = S->found ? cand_v(S->kappa_res, st->r, st->v_prev) : st->v_prev;
      if (!S->found) S->worst_res = -INFINITY;
    } else if (S->mode != kNewton) {
      const int rem = S->goal - S->halvings;
      const int d = rem < S->depth ? rem : S->depth;
      S->probe = 0;
      S->spec_n = 0;  // the slots are reused; this step's kappa is below 1 anyway
      S->spec_used = 0;
      build_tree(S, 0, d, S->lo, S->hi);
      S->n_cand = (1 << d) - 1;
      S->round += 1;
    } else {
      S->round += 1;
    }
  }
  __shared__ int s_more;
  if (threadIdx.x == 0) s_more = !S->done;
  __syncthreads();
  if (s_more) prepare_candidates<KIND>(pc, st, S);  // uniform: it has barriers
}

template <int KIND>
__global__ void __launch_bounds__(128) k_decide(const CtlArgs<KIND> a) {
  decide_body<KIND>(a.pc, a.st, a.srch, a.grad);
}

// End of a recheck launch: the last workgroup to finish takes the round's
// decision.  Each workgroup publishes its verdict updates (device-scope
// fence) before it counts itself; the last one fences again before reading
// them, resets the count for the next launch and runs the decision.  No
// workgroup waits for another.
template <int KIND>
__device__ void last_block_decides(const CtlArgs<KIND>& ctl) {
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t prev = atomicAdd(&ctl.srch->blocks_done, 1u);
    s_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  if (threadIdx.x == 0) ctl.srch->blocks_done = 0u;
  decide_body<KIND>(ctl.pc, ctl.st, ctl.srch, ctl.grad);
}

// Draws and the round-0 setup in one launch: workgroup 0 runs the setup (it
// needs no draws), the others generate the draws.
template <int KIND>
__global__ void __launch_bounds__(256) k_gen_setup(RollArgs<KIND, float> a, float* wbuf,
                                                   float* thbuf, const CtlArgs<KIND> ctl) {
  if (blockIdx.x == 0) {
    setup_body<KIND>(ctl.pc, ctl.st, ctl.srch, ctl.r_seq, ctl.closed_loop);
    return;
  }
  gen_body<KIND>(a, wbuf, thbuf, (size_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x, a.st->t);
}

// Result record; in closed loop also the true-plant step (Eq. (4)) in FP64
// under the tag-2 disturbance, and the hand-over v_prev <- v_t.  With
// setup_next the launch then prepares round 0 of the chunk's next step.
// True-plant step of the closed loop in FP64 (Eq. (4)) from x under set-point
// v and the tag-2 disturbance of step t.
template <int KIND>
__device__ void true_plant_step(const RollArgs<KIND, double>& a, const double* x_in, double v,
                                uint32_t t, double* x_out) {
  using P = Plant<KIND, double>;
  float w32[P::nw];
  draw_w<P::nw>(a.seed, a.inst, t, 2u, 0u, 0u, a.wlo, a.wspan, w32);
  double w[P::nw];
  for (int c = 0; c < P::nw; ++c) w[c] = (double)w32[c];
  typename P::Lane L;
  P::lane_init(a.pc, P::nominal_theta(a.pc), v, L);
  double x[P::n], s[P::n];
  for (int i = 0; i < P::n; ++i) x[i] = x_in[i];
  if (a.inject == 0) {
    P::force(a.pc, L, w, s);
    rk4_step<KIND, double>(a.pc, L, s, a.h, a.hh, a.h6, x);
  } else {
    P::force0(a.pc, L, s);
    rk4_step<KIND, double>(a.pc, L, s, a.h, a.hh, a.h6, x);
    P::post(a.pc, w, x);
  }
  for (int i = 0; i < P::n; ++i) x_out[i] = x[i];
}

template <int KIND>
__device__ void finalize_body(const RollArgs<KIND, double>& a, DevResult* res, double* x_hist,
                              int closed_loop) {
  using P = Plant<KIND, double>;
  DevSearch* S = a.srch;
  DevState* st = const_cast<DevState*>(a.st);
  const int idx = closed_loop ? st->cl_index : 0;
  DevResult R;
  R.kappa = S->kappa_res;
  R.v = S->v_res;
  R.worst = S->worst_res;
  R.status = S->status;
  R.rounds = S->rounds_total;
  R.candidates = S->cand_total;
  R.rechecks = S->rechecks_total;
  R.passes_alg1 = S->passes_alg1;
  R.t = st->t;
  R.lane_steps = S->lane_steps;
  R.flags = S->flags;
  res[idx] = R;
  if (closed_loop) {
    double x[P::n];
    true_plant_step<KIND>(a, st->x, R.v, st->t, x);
    for (int i = 0; i < P::n; ++i) {
      st->x[i] = x[i];
      x_hist[(size_t)(idx + 1) * P::n + i] = x[i];
    }
    st->v_prev = R.v;
    st->cl_index = idx + 1;
  }
  st->t = st->t + 1;
}

template <int KIND>
__global__ void __launch_bounds__(64) k_finalize(const RollArgs<KIND, double> a, DevResult* res,
                                                 double* x_hist, int closed_loop,
                                                 const CtlArgs<KIND> ctl, int setup_next,
                                                 int when_done) {
  // when_done: a launch of a generic closed-loop round, which records the
  // result only once the step's search has ended (and never past the chunk)
  __shared__ int s_next;
  if (threadIdx.x == 0) {
    const bool skip = when_done && (!a.srch->done || a.st->cl_index >= a.st->cl_len);
    if (!skip) finalize_body<KIND>(a, res, x_hist, closed_loop);
    s_next = !skip && setup_next && a.st->cl_index < a.st->cl_len;
  }
  if (!setup_next) return;
  __syncthreads();
  if (s_next) setup_body<KIND>(ctl.pc, ctl.st, ctl.srch, ctl.r_seq, 1, &a);
}

// rg_margin: worst margin of each listed candidate.
__global__ void k_collect(const DevSearch* S, int M, double* out) {
  for (int c = threadIdx.x; c < M; c += blockDim.x) out[c] = cand_worst(S, c);
}

// Chance-constrained verdict: the (q + 1)-th smallest of a candidate's N
// per-scenario margin keys (one workgroup per candidate), by radix selection
// on the 64-bit ordered keys, eight bits per pass from the top: each pass
// counts the keys that share the prefix found so far into 256 bins and keeps
// the bin holding the wanted rank.  Exact, duplicates included.  In decision
// mode (all == 0) only candidates still admissible are selected: every one of
// their lanes ran (violating lanes only up to their first violation, which
// keeps them below every admissible lane).
__global__ void __launch_bounds__(256) k_select_q(DevSearch* S, const unsigned long long* per_key,
                                                  int N, int all) {
  const int c = blockIdx.x;
  __shared__ int hist[256];
  __shared__ unsigned long long s_prefix;
  __shared__ int s_rank;
  if (S->done || c >= S->n_cand) return;  // uniform over the workgroup
  const int q = S->q;
  if (q <= 0) return;
  if ((!all && !cand_feasible(S, c)) || q >= N) {
    if (threadIdx.x == 0) S->keyq[c] = ~0ull;
    return;
  }
  const unsigned long long* keys = per_key + (size_t)c * N;
  if (threadIdx.x == 0) {
    s_prefix = 0ull;
    s_rank = q;
  }
  unsigned long long mask = 0ull;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const unsigned long long prefix = s_prefix;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      const unsigned long long key = keys[i];
      if ((key & mask) == prefix) atomicAdd(&hist[(int)((key >> shift) & 255ull)], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int rank = s_rank, bin = 0;
      while (bin < 255 && rank >= hist[bin]) {
        rank -= hist[bin];
        ++bin;
      }
      s_rank = rank;
      s_prefix = prefix | ((unsigned long long)bin << shift);
    }
    mask |= 255ull << shift;
    __syncthreads();
  }
  if (threadIdx.x == 0) S->keyq[c] = s_prefix;
}

// ---------------------------------------------------------------------------
// Alg. 2: each scenario runs the bisection of Alg. 1 on its own verdict (its
// rollout margin together with the steady-state test): the kappa = 1 probe,
// then K halvings; the result is the smallest per-scenario kappa.  One lane per
// scenario walks its own path through the bisection tree with no barrier
// between lanes, then one minimum over the grid.
//
// Tree nodes: node 0 is the kappa = 1 probe; heap node i >= 1 at depth
// d = floor(log2 i) is the midpoint bisection reaches there,
// kappa = (2 (i - 2^d) + 1) / 2^(d + 1) (exact: every bracket end is dyadic);
// an admitted node continues at 2i + 1, a refused one at 2i.  The steady-state
// margins of all 2^K nodes are computed first, one thread per node, so a lane
// reads its node's margin instead of running Newton's method itself.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double alg2_node_kappa(int i) {
  if (i == 0) return 1.0;
  const int d = 31 - __builtin_clz((unsigned)i);
  return ldexp((double)(2 * (i - (1 << d)) + 1), -(d + 1));
}

template <int KIND>
__global__ void __launch_bounds__(64) k_alg2_setup(const CtlArgs<KIND> ctl, double* mss_tab,
                                                   int nodes) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  DevSearch* S = ctl.srch;
  if (i == 0) {
    S->key_all[0] = ~0ull;
    S->n_recheck = 0;
    S->lane_steps = 0ull;
    S->passes_alg1 = 0;
    S->flags = 0;
  }
  if (i < nodes) {
    const double v = cand_v(alg2_node_kappa(i), ctl.st->r, ctl.st->v_prev);
    mss_tab[i] = steady_margin<KIND>(ctl.pc, S, v);
  }
}

// One lane per scenario.  T = float: a verdict whose FP32 margin lies within
// the band of zero is re-simulated in FP64 by the same lane (a64); T = double:
// FP64 throughout (a64 unused).
template <int KIND, class T, int RNG, int INJ>
__global__ void __launch_bounds__(256) k_alg2(const RollArgs<KIND, T> a,
                                              const RollArgs<KIND, double> a64,
                                              const double* mss_tab, int K) {
  __shared__ unsigned long long sh[16];
  DevSearch* S = a.srch;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t t = a.st->t;
  const double r = a.st->r, vp = a.st->v_prev;
  unsigned long long key = ~0ull;
  int passes = 0, rechecks = 0;
  unsigned long long steps = 0ull;
  if (k < a.N) {
    auto admits = [&](int node, double kap) -> bool {
      passes += 1;
      if (!(mss_tab[node] >= 0.0)) return false;  // refused by the steady-state test
      const double v = cand_v(kap, r, vp);
      int jb = 0, ns = 0;
      const T m = rollout_lane<KIND, T, RNG, INJ>(a, a.early, (T)v, k, t, nullptr, jb, ns, nullptr);
      steps += (unsigned long long)ns;
      if constexpr (std::is_same<T, double>::value) {
        return m >= 0.0;
      } else {
        if (m >= a.band) return true;
        if (m < -a.band) return false;
        rechecks += 1;
        const double m64 =
            rollout_lane<KIND, double, RNG, INJ>(a64, a64.early, v, k, t, nullptr, jb, ns, nullptr);
        return m64 >= 0.0;
      }
    };
    double kap = 1.0;
    if (!admits(0, 1.0)) {
      double lo = 0.0, hi = 1.0;
      int node = 1;
      for (int h = 0; h < K; ++h) {
        const double mid = midpoint(lo, hi);
        if (admits(node, mid)) {
          lo = mid;
          node = 2 * node + 1;
        } else {
          hi = mid;
          node = 2 * node;
        }
      }
      kap = lo;  // 0 when no candidate of this scenario was admitted
    }
    // kappa >= 0: its bit pattern orders like the value
    key = (unsigned long long)__double_as_longlong(kap);
  }
  const unsigned long long kmin = block_min_u64(key, sh);
  int wp = passes, wr = rechecks;
  unsigned long long ws = steps;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    wp += __shfl_xor(wp, off);
    wr += __shfl_xor(wr, off);
    const uint32_t lo = __shfl_xor((uint32_t)ws, off);
    const uint32_t hi = __shfl_xor((uint32_t)(ws >> 32), off);
    ws += ((unsigned long long)hi << 32) | lo;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&S->passes_alg1, wp);
    atomicAdd(&S->n_recheck, wr);
    atomicAdd(&S->lane_steps, ws);
  }
  if (threadIdx.x == 0) atomicMin(&S->key_all[0], kmin);
}

// Result record of an Alg. 2 step: kappa = 0 means some scenario admitted no
// candidate (status infeasible, v = v_prev).  No candidate is evaluated over
// all scenarios, so the worst margin is not defined (NaN; -inf when
// infeasible).
__global__ void k_alg2_finalize(DevSearch* S, DevState* st, DevResult* res) {
  if (threadIdx.x != 0) return;
  const double kap = __longlong_as_double((long long)S->key_all[0]);
  const int status = kap == 0.0 ? 1 : 0;
  DevResult R;
  R.kappa = kap;
  R.v = status ? st->v_prev : cand_v(kap, st->r, st->v_prev);
  R.worst = status ? -INFINITY : __longlong_as_double(0x7ff8000000000000ll);
  R.status = status;
  R.rounds = 1;
  R.candidates = S->passes_alg1;
  R.rechecks = S->n_recheck;
  R.passes_alg1 = S->passes_alg1;
  R.t = st->t;
  R.lane_steps = S->lane_steps;
  R.flags = 0;
  res[0] = R;
  S->kappa_res = kap;
  S->v_res = R.v;
  S->done = 1;
  st->t = st->t + 1;
}

struct ThetaNominal {
  double v[kMaxTh];
};

template <int KIND>
__global__ void k_draws(RollArgs<KIND, float> a, uint32_t t, int k0, int nk, int j0, int nj,
                        float* w_out, double* th_out, ThetaNominal thnom) {
  using P = Plant<KIND, float>;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < nk * nj) {
    const int jj = gid / nk, kk = gid - jj * nk;
    float w[P::nw];
    draw_w<P::nw>(a.seed, a.inst, t, 0u, (uint32_t)(k0 + kk), (uint32_t)(j0 + jj), a.wlo, a.wspan,
                  w);
    for (int c = 0; c < P::nw; ++c) w_out[((size_t)jj * nk + kk) * P::nw + c] = w[c];
  } else if (P::nth > 0 && th_out && gid < nk * nj + nk) {
    const int kk = gid - nk * nj;
    float f[P::nth > 0 ? P::nth : 1];
    draw_theta_factor<P::nth>(a.seed, a.inst, t, (uint32_t)(k0 + kk), a.thlo, a.thspan, f);
    for (int c = 0; c < P::nth; ++c) th_out[(size_t)kk * P::nth + c] = thnom.v[c] * (double)f[c];
  }
}

template <int KIND, class T, int RNG, int INJ>
__global__ void k_traj(const RollArgs<KIND, T> a, T v, const int32_t* k_list, int nk,
                       double* traj) {
  using P = Plant<KIND, T>;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nk) return;
  int jb, ns;
  rollout_lane<KIND, T, RNG, INJ>(a, 0, v, k_list[i], a.st->t, nullptr, jb, ns,
                                  traj + (size_t)i * (a.H + 1) * P::n);
}


// ---------------------------------------------------------------------------
// Gradients of a candidate's margin.
//
// Reverse mode through the discrete RK4 map: forward pass with checkpoints
// every Kc steps (tracking the minimiser j*, r*), then segment by segment from
// j* back to 0: recompute the segment's states from its checkpoint, sweep them
// in reverse with rk4_vjp.  States and adjoints in FP32, parameter sums in
// FP64.  One lane per (scenario, upstream weight) entry.
// ---------------------------------------------------------------------------
struct AdjArgs {
  int Kc;
  int lmax;                // stride of the SoA scratch (= N)
  int cand;                // candidate index whose v is used
  const int32_t* k_list;
  const float* w_list;
  float* out_m;
  double* out_dv;
  double* out_dth;
  float* ckpt;
  float* seg;
  DevGrad* grad;
};

template <int KIND, int RNG, int INJ>
__global__ void __launch_bounds__(64) k_adjoint(const RollArgs<KIND, float> a, const AdjArgs g) {
  using P = Plant<KIND, float>;
  constexpr int n = P::n;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.grad->n_entries) return;
  const int k = g.k_list[e];
  const float wgt = g.w_list[e];
  const uint32_t t = a.st->t;
  const int cand = g.cand >= 0 ? g.cand : a.srch->nk_idx;
  if ((a.srch->done || cand < 0) && g.cand < 0) return;
  const float v = (float)a.srch->v[cand];
  const size_t L = (size_t)g.lmax;
  float th[P::nth > 0 ? P::nth : 1], fac[P::nth > 0 ? P::nth : 1];
  if constexpr (P::nth > 0) {
    if (RNG == 0) {
      const float* tb = step_th(a, t);
      for (int c = 0; c < P::nth; ++c) fac[c] = tb[(size_t)c * a.N + k];
    } else {
      draw_theta_factor<P::nth>(a.seed, a.inst, t, (uint32_t)k, a.thlo, a.thspan, fac);
    }
    for (int c = 0; c < P::nth; ++c) th[c] = a.pc.thnom[c] * fac[c];
  }
  typename P::Lane Ln;
  P::lane_init(a.pc, th, v, Ln);
  float wv[KIND == 2 ? 81 : 1];
  w_in_vgprs<KIND>(a.pc, wv, Ln);
  const float* wb = RNG == 0 ? step_w(a, t) : nullptr;
  auto load_w = [&](int j, float* w) {
    if (RNG == 0) {
      for (int c = 0; c < P::nw; ++c) w[c] = wb[((size_t)j * P::nw + c) * a.N + k];
    } else {
      draw_w<P::nw>(a.seed, a.inst, t, 0u, (uint32_t)k, (uint32_t)j, a.wlo, a.wspan, w);
    }
  };
  auto forcing = [&](const float* w, float* s) {
    if (INJ == 0) P::force(a.pc, Ln, w, s);
    else P::force0(a.pc, Ln, s);
  };
  auto step = [&](float* x, const float* w) {
    float s[n];
    forcing(w, s);
    rk4_step<KIND, float>(a.pc, Ln, s, a.h, a.hh, a.h6, x);
    if (INJ == 1) P::post(a.pc, w, x);
  };
  // forward: minimiser and checkpoints
  float x[n], xbest[n], y[P::ny], w[P::nw];
  for (int i = 0; i < n; ++i) x[i] = (float)a.st->x[i];
  int rb = 0, jb = 0;
  P::output(a.pc, Ln, x, y);
  float best = margin_rows_arg<P::ny>(a.F, a.g, y, rb);
  for (int i = 0; i < n; ++i) {
    xbest[i] = x[i];
    g.ckpt[(size_t)i * L + e] = x[i];
  }
  for (int j = 0; j < a.H; ++j) {
    load_w(j, w);
    step(x, w);
    int r = 0;
    P::output(a.pc, Ln, x, y);
    const float m = margin_rows_arg<P::ny>(a.F, a.g, y, r);
    if (m < best) {
      best = m;
      jb = j + 1;
      rb = r;
      for (int i = 0; i < n; ++i) xbest[i] = x[i];
    }
    if ((j + 1) % g.Kc == 0 && j + 1 < a.H)
      for (int i = 0; i < n; ++i) g.ckpt[((size_t)((j + 1) / g.Kc) * n + i) * L + e] = x[i];
  }
  bool finite = best == best;
  for (int i = 0; i < n; ++i) finite = finite && (x[i] - x[i] == 0.f);
  double vb = 0.0;
  double tb[P::nth > 0 ? P::nth : 1];
  for (int c = 0; c < (P::nth > 0 ? P::nth : 1); ++c) tb[c] = 0.0;
  if (finite) {
    float lam[n];
    P::out_grad(a.pc, a.F + rb * P::ny, xbest, lam);
    for (int seg = (jb - 1) / g.Kc; jb > 0 && seg >= 0; --seg) {
      const int j0 = seg * g.Kc;
      const int j1 = (j0 + g.Kc) < jb ? (j0 + g.Kc) : jb;
      float xs[n];
      for (int i = 0; i < n; ++i) xs[i] = g.ckpt[((size_t)seg * n + i) * L + e];
      for (int j = j0; j < j1; ++j) {
        for (int i = 0; i < n; ++i) g.seg[((size_t)(j - j0) * n + i) * L + e] = xs[i];
        load_w(j, w);
        step(xs, w);
      }
      for (int j = j1 - 1; j >= j0; --j) {
        for (int i = 0; i < n; ++i) xs[i] = g.seg[((size_t)(j - j0) * n + i) * L + e];
        load_w(j, w);
        float s[n];
        forcing(w, s);
        rk4_vjp<KIND, float>(a.pc, Ln, s, a.h, a.hh, a.h6, xs, lam, vb, tb);
      }
    }
  } else {
    best = -INFINITY;
  }
  g.out_m[e] = best;
  g.out_dv[e] = (double)wgt * vb;
  for (int c = 0; c < P::nth; ++c) g.out_dth[(size_t)e * kMaxTh + c] = (double)wgt * tb[c] * (double)fac[c];
  if (e == 0) {
    g.grad->j_star = jb;
    g.grad->r_star = rb;
  }
}

// ---------------------------------------------------------------------------
// Segment-parallel derivative of one scenario's worst margin.
//
// The rollout keeps the state of every scenario of one candidate at steps
// s * Kc.  For the chosen scenario k*:
//   k_seg_min      one lane per segment: recompute the segment, its margin
//                  minimum, first minimising step and row, and that state;
//   k_seg_vjp      one lane per (segment s, state component o), segments up to
//                  the first minimising step j*: recompute the segment, then
//                  run the RK4 reverse sweep from lambda = e_o at its end.  The
//                  lane leaves row o of the segment's state transfer matrix and
//                  the derivative of component o at the segment end with
//                  respect to v and theta over that segment;
//   k_seg_combine  one thread: lambda = dm/dx at j*, then for the segments
//                  from the last to the first, add lambda . (v, theta columns)
//                  and apply the transposed transfer matrix.
// The result equals the reverse sweep over all j* steps (chain rule over the
// segments); the sequential part is one short loop per segment instead of
// one RK4 step per time step.
// ---------------------------------------------------------------------------
struct SegArgs {
  int Kc, S;          // checkpoint interval; segments covering steps 0..H
  int cand;           // candidate (-1: the Newton iterate)
  int lanes;          // stride of the state scratch (= S * n)
  float* seg_m;       // [S] segment minimum (NaN: non-finite trajectory)
  int32_t* seg_j;     // [S] its first minimising step
  int32_t* seg_r;     // [S] its constraint row
  float* seg_x;       // [S * n] state at that step
  float* seg_a;       // [(s * n + o) * n + i] row o of the segment's transfer matrix
  double* seg_cv;     // [s * n + o] d x_o(segment end) / d v over the segment
  double* seg_ct;     // [(s * n + o) * kMaxTh + c] same for theta^k_c
  float* scratch;     // [(jj * n + i) * lanes + lane] states of a lane's segment
  float* out_m;       // entry 0 outputs, as the sequential adjoint writes them
  double* out_dv;
  double* out_dth;
  DevGrad* grad;
};

// Per-lane scenario model shared by the segment kernels.
template <int KIND, int RNG, int INJ>
struct SegLane {
  using P = Plant<KIND, float>;
  const RollArgs<KIND, float>& a;
  int k;
  uint32_t t;
  typename P::Lane L;
  float fac[P::nth > 0 ? P::nth : 1];
  __device__ SegLane(const RollArgs<KIND, float>& a_, int k_, float v) : a(a_), k(k_) {
    t = a.st->t;
    float th[P::nth > 0 ? P::nth : 1];
    if constexpr (P::nth > 0) {
      if (RNG == 0) {
        const float* tb = step_th(a, t);
        for (int c = 0; c < P::nth; ++c) fac[c] = tb[(size_t)c * a.N + k];
      } else {
        draw_theta_factor<P::nth>(a.seed, a.inst, t, (uint32_t)k, a.thlo, a.thspan, fac);
      }
      for (int c = 0; c < P::nth; ++c) th[c] = a.pc.thnom[c] * fac[c];
    } else {
      fac[0] = 1.f;
    }
    P::lane_init(a.pc, th, v, L);
  }
  __device__ void draws(int j, float* w) const {
    if (RNG == 0) {
      const float* wb = step_w(a, t);
      for (int c = 0; c < P::nw; ++c) w[c] = wb[((size_t)j * P::nw + c) * a.N + k];
    } else {
      draw_w<P::nw>(a.seed, a.inst, t, 0u, (uint32_t)k, (uint32_t)j, a.wlo, a.wspan, w);
    }
  }
  __device__ void forcing(const float* w, float* s) const {
    if (INJ == 0) P::force(a.pc, L, w, s);
    else P::force0(a.pc, L, s);
  }
  __device__ void step(float* x, int j) const {
    float w[P::nw], s[P::n];
    draws(j, w);
    forcing(w, s);
    rk4_step<KIND, float>(a.pc, L, s, a.h, a.hh, a.h6, x);
    if (INJ == 1) P::post(a.pc, w, x);
  }
  __device__ float margin(const float* x, int& r) const {
    float y[P::ny];
    P::output(a.pc, L, x, y);
    return margin_rows_arg<P::ny>(a.F, a.g, y, r);
  }
};

// Which candidate and scenario the segment kernels work on; false when there
// is nothing to do (search finished, or the steady-state term is active).
__device__ __forceinline__ bool seg_target(const DevSearch* S, const SegArgs& g, int& cand,
                                           int& ks) {
  if (g.cand < 0 && S->done) return false;
  cand = g.cand >= 0 ? g.cand : S->nk_idx;
  if (cand < 0) return false;  // no iterate this round
  ks = g.grad->k_star;
  return ks >= 0 && g.grad->n_entries > 0;
}

// First minimiser over the segment minima; false if any segment is non-finite.
__device__ __forceinline__ bool seg_argmin(const SegArgs& g, float& best, int& sb) {
  best = INFINITY;
  sb = 0;
  for (int s = 0; s < g.S; ++s) {
    const float m = g.seg_m[s];
    if (m != m) return false;
    if (m < best) {
      best = m;
      sb = s;
    }
  }
  return true;
}

template <int KIND, int RNG, int INJ>
__global__ void __launch_bounds__(64) k_seg_min(const RollArgs<KIND, float> a, const SegArgs g,
                                                const float* ckpt) {
  using P = Plant<KIND, float>;
  constexpr int n = P::n;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.S) return;
  int cand, ks;
  if (!seg_target(a.srch, g, cand, ks)) return;
  const SegLane<KIND, RNG, INJ> M(a, ks, (float)a.srch->v[cand]);
  float x[n], xb[n];
  for (int i = 0; i < n; ++i) x[i] = ckpt[((size_t)s * n + i) * a.N + ks];
  const int j0 = s * g.Kc, j1 = (j0 + g.Kc < a.H) ? j0 + g.Kc : a.H;
  float best = INFINITY;
  int jb = j0, rb = 0;
  if (s == 0) {  // the initial state belongs to the first segment
    best = M.margin(x, rb);
    jb = 0;
  }
  for (int i = 0; i < n; ++i) xb[i] = x[i];
  for (int j = j0; j < j1; ++j) {
    M.step(x, j);
    int r = 0;
    const float m = M.margin(x, r);
    if (m < best || m != m) {
      best = m;
      jb = j + 1;
      rb = r;
      for (int i = 0; i < n; ++i) xb[i] = x[i];
    }
  }
  bool finite = true;
  for (int i = 0; i < n; ++i) finite = finite && (x[i] - x[i] == 0.f);
  g.seg_m[s] = finite ? best : NAN;
  g.seg_j[s] = jb;
  g.seg_r[s] = rb;
  for (int i = 0; i < n; ++i) g.seg_x[(size_t)s * n + i] = xb[i];
}

template <int KIND, int RNG, int INJ>
__global__ void __launch_bounds__(64) k_seg_vjp(const RollArgs<KIND, float> a, const SegArgs g,
                                                const float* ckpt) {
  using P = Plant<KIND, float>;
  constexpr int n = P::n;
  const int lane = blockIdx.x * blockDim.x + threadIdx.x;
  if (lane >= g.S * n) return;
  int cand, ks;
  if (!seg_target(a.srch, g, cand, ks)) return;
  float best;
  int sb;
  if (!seg_argmin(g, best, sb)) return;
  const int js = g.seg_j[sb];
  const int s = lane / n, o = lane - s * n;
  const int j0 = s * g.Kc;
  if (j0 >= js) return;  // segment after the minimising step
  const int j1 = (j0 + g.Kc < js) ? j0 + g.Kc : js;
  const SegLane<KIND, RNG, INJ> M(a, ks, (float)a.srch->v[cand]);
  float x[n];
  for (int i = 0; i < n; ++i) x[i] = ckpt[((size_t)s * n + i) * a.N + ks];
  const size_t L = (size_t)g.lanes;
  for (int j = j0; j < j1; ++j) {
    for (int i = 0; i < n; ++i) g.scratch[((size_t)(j - j0) * n + i) * L + lane] = x[i];
    M.step(x, j);
  }
  float lam[n];
  for (int i = 0; i < n; ++i) lam[i] = (i == o) ? 1.f : 0.f;
  double vb = 0.0;
  double tb[P::nth > 0 ? P::nth : 1];
  for (int c = 0; c < (P::nth > 0 ? P::nth : 1); ++c) tb[c] = 0.0;
  for (int j = j1 - 1; j >= j0; --j) {
    for (int i = 0; i < n; ++i) x[i] = g.scratch[((size_t)(j - j0) * n + i) * L + lane];
    float w[P::nw], sf[n];
    M.draws(j, w);
    M.forcing(w, sf);
    rk4_vjp<KIND, float>(a.pc, M.L, sf, a.h, a.hh, a.h6, x, lam, vb, tb);
  }
  for (int i = 0; i < n; ++i) g.seg_a[((size_t)s * n + o) * n + i] = lam[i];
  g.seg_cv[(size_t)s * n + o] = vb;
  for (int c = 0; c < P::nth; ++c) g.seg_ct[((size_t)s * n + o) * kMaxTh + c] = tb[c];
}

template <int KIND, int RNG, int INJ>
__global__ void k_seg_combine(const RollArgs<KIND, float> a, const SegArgs g) {
  using P = Plant<KIND, float>;
  constexpr int n = P::n;
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int cand, ks;
  if (!seg_target(a.srch, g, cand, ks)) return;
  float best;
  int sb;
  double dv = 0.0, dth[P::nth > 0 ? P::nth : 1];
  for (int c = 0; c < (P::nth > 0 ? P::nth : 1); ++c) dth[c] = 0.0;
  int js = 0, rs = 0;
  if (!seg_argmin(g, best, sb)) {
    best = -INFINITY;
  } else {
    js = g.seg_j[sb];
    rs = g.seg_r[sb];
    float xs[n], gx[n];
    for (int i = 0; i < n; ++i) xs[i] = g.seg_x[(size_t)sb * n + i];
    P::out_grad(a.pc, a.F + rs * P::ny, xs, gx);
    double lam[n], nl[n];
    for (int i = 0; i < n; ++i) lam[i] = (double)gx[i];
    for (int s = (js + g.Kc - 1) / g.Kc - 1; js > 0 && s >= 0; --s) {
      for (int i = 0; i < n; ++i) nl[i] = 0.0;
      for (int o = 0; o < n; ++o) {
        const double lo = lam[o];
        dv += lo * g.seg_cv[(size_t)s * n + o];
        for (int c = 0; c < P::nth; ++c) dth[c] += lo * g.seg_ct[((size_t)s * n + o) * kMaxTh + c];
        for (int i = 0; i < n; ++i) nl[i] += lo * (double)g.seg_a[((size_t)s * n + o) * n + i];
      }
      for (int i = 0; i < n; ++i) lam[i] = nl[i];
    }
  }
  // theta^k = theta_nom * factor_k
  const SegLane<KIND, RNG, INJ> M(a, ks, (float)a.srch->v[cand]);
  g.out_m[0] = best;
  g.out_dv[0] = dv;
  for (int c = 0; c < P::nth; ++c) g.out_dth[c] = dth[c] * (double)M.fac[c];
  g.grad->j_star = js;
  g.grad->r_star = rs;
}

// Steady-state margin gradient by the adjoint of the equilibrium condition:
// f(x_ss, v) = 0, m = g_r - eps|g_r| - F_r h(x_ss):  solve J^T mu = dm/dx, then
// dm/dv = -mu . df/dv and dm/dtheta_nom = -mu . df/dtheta (FP64).
template <int KIND>
__device__ double steady_grad(const typename Plant<KIND, double>::Coef& pc, const DevSearch* S,
                              double v, double* dmdv, double* dth) {
  using P = Plant<KIND, double>;
  constexpr int n = P::n;
  *dmdv = 0.0;
  for (int c = 0; c < kMaxTh; ++c) dth[c] = 0.0;
  if (!S->ss_check) return INFINITY;
  double x[n], f[n], J[n * n], s0[n];
  P::eq_guess(pc, v, x, J);
  if (P::eq_guess_needs_solve()) {
    if (!dense_solve<n>(J, x)) return -INFINITY;
  }
  typename P::Lane L;
  P::lane_init(pc, P::nominal_theta(pc), v, L);
  P::force0(pc, L, s0);
  bool ok = false;
  for (int it = 0; it <= 50; ++it) {
    P::deriv(pc, L, s0, x, f);
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) nrm = fmax(nrm, fabs(f[i]));
    if (!(nrm == nrm)) return -INFINITY;
    if (nrm <= 1e-12) {
      ok = true;
      break;
    }
    if (it == 50) break;
    P::jacobian(pc, x, v, J);
    for (int i = 0; i < n; ++i) f[i] = -f[i];
    if (!dense_solve<n>(J, f)) return -INFINITY;
    for (int i = 0; i < n; ++i) x[i] += f[i];
  }
  if (!ok) return -INFINITY;
  double y[P::ny];
  P::output(pc, L, x, y);
  double best = INFINITY;
  int rb = 0;
  for (int r = 0; r < S->n_c; ++r) {
    double fy = 0.0;
    for (int i = 0; i < P::ny; ++i) fy += S->F[r * P::ny + i] * y[i];
    const double m = tightened_rhs(S->g[r], S->eps) - fy;
    if (r == 0 || m < best) {
      best = m;
      rb = r;
    }
  }
  double Fr[P::ny], gx[n], mu[n];
  for (int i = 0; i < P::ny; ++i) Fr[i] = S->F[rb * P::ny + i];
  P::out_grad(pc, Fr, x, gx);
  P::jacobian(pc, x, v, J);
  double Jt[n * n];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Jt[i * n + j] = J[j * n + i];
  for (int i = 0; i < n; ++i) mu[i] = gx[i];
  if (!dense_solve<n>(Jt, mu)) return best;
  double xb[n], vb = 0.0, tb[kMaxTh];
  for (int c = 0; c < kMaxTh; ++c) tb[c] = 0.0;
  P::vjp(pc, L, x, mu, xb, vb, tb);
  *dmdv = -vb;
  for (int c = 0; c < P::nth; ++c) dth[c] = -tb[c];
  return best;
}

// Choose the active term of M(kappa) for candidate `cand`: the arg-min
// scenario (one adjoint entry) or the steady-state margin (gradient here).
// use_keys = 0 keeps the entries the host uploaded (weighted sum).
template <int KIND>
__global__ void k_grad_prepare(const CtlArgs<KIND> a, DevGrad* G, int32_t* adj_k, float* adj_w,
                               int cand, int use_keys) {
  if (threadIdx.x != 0) return;
  DevSearch* S = a.srch;
  if (cand < 0) {
    if (S->done) return;
    cand = S->nk_idx;
    if (cand < 0) {  // no iterate this round: nothing to differentiate
      G->k_star = -1;
      G->n_entries = 0;
      return;
    }
  }
  const double worst = cand_worst_p(S, cand, 0);  // gradients use the FP32 rollouts
  G->M = worst;
  G->dM_dv = 0.0;
  for (int c = 0; c < kMaxTh; ++c) G->dM_dth[c] = 0.0;
  if (!use_keys) {
    G->k_star = -1;
    return;
  }
  const unsigned long long key = S->key_all[cand];
  const double roll = key == ~0ull ? INFINITY : key_margin(key, 0);
  if (S->mss[cand] < roll) {
    double dv, dth[kMaxTh];
    steady_grad<KIND>(a.pc, S, S->v[cand], &dv, dth);
    G->dM_dv = dv;
    for (int c = 0; c < kMaxTh; ++c) G->dM_dth[c] = dth[c];
    G->n_entries = 0;
    G->k_star = -1;
  } else {
    const int ks = (int)(uint32_t)(key & 0xffffffffu);
    G->n_entries = 1;
    G->k_star = ks;
    adj_k[0] = ks;
    adj_w[0] = 1.f;
  }
}

// Deterministic sum of the entries' weighted derivatives (fixed order per
// thread, then a fixed LDS tree), then dM/dkappa = dM/dv (r - v_prev).
__global__ void __launch_bounds__(256) k_grad_reduce(DevGrad* G, const double* dv, const double* dth,
                                                     int nth, const DevState* st,
                                                     const DevSearch* S, int cand) {
  if (cand < 0 && (S->done || S->nk_idx < 0)) return;  // finished, or no iterate this round
  __shared__ double sh[256];
  const int n = G->n_entries;
  const int tid = threadIdx.x;
  for (int c = -1; c < nth; ++c) {
    double acc = 0.0;
    for (int e = tid; e < n; e += 256) acc += c < 0 ? dv[e] : dth[(size_t)e * kMaxTh + c];
    sh[tid] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) sh[tid] += sh[tid + s];
      __syncthreads();
    }
    if (tid == 0 && n > 0) {
      if (c < 0) G->dM_dv += sh[0];
      else G->dM_dth[c] += sh[0];
    }
    __syncthreads();
  }
  if (tid == 0) {  // v = r exactly at kappa = 1; dv/dkappa = r - v_prev on both sides
    G->dM_dkappa = G->dM_dv * (st->r - st->v_prev);
  }
}


// Derivative of the worst margin M(kappa) of candidate `cand` (-1: the Newton
// iterate) from the forward tangent the rollout left: the active term is the
// arg-min scenario's rollout margin (its tangent) or, when smaller, the
// steady-state margin (implicit derivative in FP64); then dM/dkappa =
// dM/dv (r - v_prev).
template <int KIND>
__global__ void k_tan_grad(const CtlArgs<KIND> a, DevGrad* G, const float* tan_dv, int cand) {
  if (threadIdx.x != 0) return;
  DevSearch* S = a.srch;
  if (cand < 0) {
    if (S->done) return;
    cand = S->nk_idx;
    if (cand < 0) return;  // no iterate this round
  }
  G->M = cand_worst_p(S, cand, 0);
  for (int c = 0; c < kMaxTh; ++c) G->dM_dth[c] = 0.0;
  G->n_entries = 0;
  const unsigned long long key = S->key_all[cand];
  const double roll = key == ~0ull ? INFINITY : key_margin(key, 0);
  if (S->mss[cand] < roll || key == ~0ull) {
    double dv, dth[kMaxTh];
    steady_grad<KIND>(a.pc, S, S->v[cand], &dv, dth);
    G->dM_dv = dv;
    for (int c = 0; c < kMaxTh; ++c) G->dM_dth[c] = dth[c];
    G->k_star = -1;
  } else {
    const int ks = (int)(uint32_t)(key & 0xffffffffu);
    G->k_star = ks;
    G->dM_dv = (double)tan_dv[ks];
  }
  G->dM_dkappa = G->dM_dv * (a.st->r - a.st->v_prev);
}

// Equilibrium f(x, v, 0, theta_nom) = 0 by the steady-state Newton iteration;
// out[0..n) = x_ss, out[n] = 1 if converged.
template <int KIND>
__global__ void k_equilibrium(const CtlArgs<KIND> a, double v, double* out) {
  using P = Plant<KIND, double>;
  constexpr int n = P::n;
  if (threadIdx.x != 0) return;
  double x[n], f[n], J[n * n], s0[n];
  P::eq_guess(a.pc, v, x, J);
  bool ok = !P::eq_guess_needs_solve() || dense_solve<n>(J, x);
  typename P::Lane L;
  P::lane_init(a.pc, P::nominal_theta(a.pc), v, L);
  P::force0(a.pc, L, s0);
  bool conv = false;
  for (int it = 0; ok && it <= 50; ++it) {
    P::deriv(a.pc, L, s0, x, f);
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) nrm = fmax(nrm, fabs(f[i]));
    if (!(nrm == nrm)) break;
    if (nrm <= 1e-12) {
      conv = true;
      break;
    }
    P::jacobian(a.pc, x, v, J);
    for (int i = 0; i < n; ++i) f[i] = -f[i];
    if (!dense_solve<n>(J, f)) break;
    for (int i = 0; i < n; ++i) x[i] += f[i];
  }
  for (int i = 0; i < n; ++i) out[i] = x[i];
  out[n] = conv ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
// Host-side argument filling and launchers
// ---------------------------------------------------------------------------
template <int KIND, class T>
static RollArgs<KIND, T> make_args(const Problem& pr, double band, int early, int record,
                                   const DevBuffers& b) {
  using P = Plant<KIND, T>;
  RollArgs<KIND, T> a;
  memset(&a, 0, sizeof(a));
  P::load(a.pc, pr.p.coeffs);
  for (int r = 0; r < kNC; ++r) {
    for (int i = 0; i < P::ny; ++i) a.F[r * P::ny + i] = (T)pr.c.F[r * P::ny + i];
    a.g[r] = (T)pr.c.g[r];
  }
  a.h = (T)pr.dt;
  a.hh = (T)(pr.dt * 0.5);
  a.h6 = (T)(pr.dt / 6.0);
  a.band = (T)band;
  a.H = pr.H;
  a.N = pr.s.N;
  a.early = early;
  a.record = record;
  a.inject = pr.s.inject;
  a.seed = pr.s.seed;
  a.inst = pr.s.instance;
  for (int c = 0; c < P::nw; ++c) {
    a.wlo[c] = (float)pr.s.wlo[c];
    a.wspan[c] = (float)(pr.s.whi[c] - pr.s.wlo[c]);
  }
  a.thlo = (float)(1.0 - pr.s.theta_rel);
  a.thspan = (float)(2.0 * pr.s.theta_rel);
  a.wbuf = b.wbuf;
  a.thbuf = b.thbuf;
  a.ring = b.ring;
  for (int j = 0; j < kPairs; ++j) {
    a.wring[j] = b.wpair[j];
    a.thring[j] = b.thpair[j];
  }
  a.st = b.st;
  a.srch = b.srch;
  a.per_m = b.per_m;
  a.per_j = b.per_j;
  a.per_key = b.per_key;
  a.rlist = b.rlist;
  a.tan_dv = b.tan_dv;
  return a;
}

template <int KIND>
static CtlArgs<KIND> make_ctl(const Problem& pr, const DevBuffers& b, int closed_loop) {
  CtlArgs<KIND> a;
  memset(&a, 0, sizeof(a));
  Plant<KIND, double>::load(a.pc, pr.p.coeffs);
  a.st = b.st;
  a.srch = b.srch;
  a.r_seq = b.r_seq;
  a.closed_loop = closed_loop;
  a.grad = b.grad;
  return a;
}

template <int V>
using IC = std::integral_constant<int, V>;

template <class F>
static hipError_t by_kind(int kind, F&& f) {
  if (kind == 1) return f(IC<1>{});
  if (kind == 2) return f(IC<2>{});
  return hipErrorInvalidValue;
}
template <class F>
static hipError_t by_bit(int v, F&& f) {
  return v ? f(IC<1>{}) : f(IC<0>{});
}

static int div_up(size_t a, size_t b) { return (int)((a + b - 1) / b); }

hipError_t launch_gen(const Problem& pr, const DevBuffers& b, hipStream_t st, uint32_t t_ofs) {
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    auto a = make_args<K, float>(pr, 0.0, 0, 0, b);
    const size_t work = (size_t)pr.H * pr.s.N + (Plant<K, float>::nth > 0 ? pr.s.N : 0);
    hipLaunchKernelGGL(k_gen<K>, dim3(div_up(work, 256)), dim3(256), 0, st, a, b.wbuf, b.thbuf,
                       t_ofs);
    return hipGetLastError();
  });
}

hipError_t launch_gen_setup(const Problem& pr, const DevBuffers& b, int closed_loop,
                            hipStream_t st) {
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    auto a = make_args<K, float>(pr, 0.0, 0, 0, b);
    const size_t work = (size_t)pr.H * pr.s.N + (Plant<K, float>::nth > 0 ? pr.s.N : 0);
    hipLaunchKernelGGL(k_gen_setup<K>, dim3(1 + div_up(work, 256)), dim3(256), 0, st, a, b.wbuf,
                       b.thbuf, make_ctl<K>(pr, b, closed_loop));
    return hipGetLastError();
  });
}

hipError_t launch_setup(const Problem& pr, const DevBuffers& b, int closed_loop, hipStream_t st) {
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    hipLaunchKernelGGL(k_setup<K>, dim3(1), dim3(128), 0, st, make_ctl<K>(pr, b, closed_loop));
    return hipGetLastError();
  });
}

hipError_t launch_setup_list(const Problem& pr, const DevBuffers& b, int M, hipStream_t st) {
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    hipLaunchKernelGGL(k_setup_list<K>, dim3(1), dim3(128), 0, st, make_ctl<K>(pr, b, 0), M);
    return hipGetLastError();
  });
}

static QuadCoef make_quad_coef(const Problem& pr) {
  QuadCoef qc;
  memset(&qc, 0, sizeof(qc));
  const double* A = pr.p.coeffs;
  const double* B = pr.p.coeffs + 16;
  const double* G = pr.p.coeffs + 20;
  const double* E = pr.p.coeffs + 36;
  const double* Cm = pr.p.coeffs + 44;
  double D[4][4];
  for (int r = 0; r < 4; ++r)
    for (int i = 0; i < 4; ++i) {
      double acc = 0.0;
      for (int y = 0; y < 2; ++y) acc += pr.c.F[r * 2 + y] * Cm[y * 4 + i];
      D[r][i] = acc;
    }
  for (int q = 0; q < 4; ++q) {
    for (int s = 0; s < 4; ++s) {
      const int row = q ^ s;
      qc.a[q][s] = (float)A[row * 4 + q];
      qc.g[q][s] = (float)G[row * 4 + q];
      qc.d[q][s] = (float)(-D[row][q]);
    }
    qc.b[q] = (float)B[q];
    qc.e[q][0] = (float)E[q * 2 + 0];
    qc.e[q][1] = (float)E[q * 2 + 1];
    qc.grow[q] = (float)pr.c.g[q];
  }
  return qc;
}

// The quad kernel addresses the streamed draws with 32-bit byte offsets.
static bool quad_draws_addressable(const Problem& pr) {
  const double bytes = 8.0 * (double)pr.s.N * (double)(pr.H + kQuadGroup);
  return pr.s.rng_mode != 0 || bytes < 4294967296.0;  // rng_mode 1: inline draws
}

bool rollout_uses_quad(const Problem& pr, const LaunchCfg& cfg, int precision) {
  return cfg.lanes == 4 && precision == 0 && pr.p.kind == 1 && quad_draws_addressable(pr);
}

hipError_t launch_rollout(const Problem& pr, double band, int precision, int early_exit, int record,
                          const LaunchCfg& cfg, const DevBuffers& b, hipStream_t st, int ckpt_cand,
                          int Kc, float* gen_w, float* gen_th) {
  const bool ckpt = ckpt_cand >= -1 && precision == 0;
  const bool gen = gen_w != nullptr && pr.s.rng_mode == 0;
  // rows of draw workgroups after the candidate rows: up to about 2^19 threads
  // (measured when an update decided ahead ran these rows alone; 4-state bench
  // loop: 0.277 ms per update with 2^17 threads, 0.271 with 2^18 or 2^19, 0.270
  // with 2^20)
  auto gen_rows_for = [&](size_t row_threads) {
    if (!gen) return 0;
    size_t work = (size_t)pr.H * pr.s.N + (size_t)pr.s.N;
    if (work > (size_t(1) << 19)) work = size_t(1) << 19;
    return (int)((work + row_threads - 1) / row_threads);
  };
  auto set_gen = [&](auto& a) {
    if (!gen) return;
    a.gen_row0 = cfg.cmax_round;
    a.gen_ofs = kSpecMax + 1;
    a.gen_w = gen_w;
    a.gen_th = gen_th;
  };
  if (cfg.lanes == 4 && precision == 0 && pr.p.kind == 1 && quad_draws_addressable(pr) &&
      !(cfg.chance && (record || ckpt))) {
    const int gx = div_up((size_t)pr.s.N * 4, (size_t)cfg.block);
    const dim3 grid(gx, cfg.cmax_round + gen_rows_for((size_t)gx * cfg.block));
    const QuadCoef qc = make_quad_coef(pr);
    auto a = make_args<1, float>(pr, band, early_exit, record, b);
    a.ckpt = b.adj_ckpt;
    a.Kc = Kc;
    a.ckpt_cand = ckpt_cand;
    set_gen(a);
    return by_bit(pr.s.rng_mode, [&](auto rc) {
      constexpr int R = decltype(rc)::value;
      return by_bit(pr.s.inject, [&](auto ic) {
        constexpr int I = decltype(ic)::value;
        return by_bit(record, [&](auto dc) {
          constexpr int D = decltype(dc)::value;
          if (cfg.chance)
            hipLaunchKernelGGL((k_rollout_lq4_quad<R, I, 0, 0, 1>), grid, dim3(cfg.block), 0, st, a,
                               qc);
          else if (ckpt && cfg.tan)
            hipLaunchKernelGGL((k_rollout_lq4_quad<R, I, D, 2>), grid, dim3(cfg.block), 0, st, a, qc);
          else if (ckpt)
            hipLaunchKernelGGL((k_rollout_lq4_quad<R, I, D, 1>), grid, dim3(cfg.block), 0, st, a, qc);
          else
            hipLaunchKernelGGL((k_rollout_lq4_quad<R, I, D, 0>), grid, dim3(cfg.block), 0, st, a, qc);
          return hipGetLastError();
        });
      });
    });
  }
  if (cfg.lanes == 16 && precision == 0 && pr.p.kind == 2 && !cfg.chance && !(ckpt && cfg.tan)) {
    // 9-state plant, one scenario per group of 16 lanes
    const int gx = div_up((size_t)pr.s.N * 16, (size_t)cfg.block);
    const dim3 grid(gx, cfg.cmax_round + gen_rows_for((size_t)gx * cfg.block));
    auto a = make_args<2, float>(pr, band, early_exit, record, b);
    a.ckpt = b.adj_ckpt;
    a.Kc = Kc;
    a.ckpt_cand = ckpt_cand;
    set_gen(a);
    return by_bit(pr.s.rng_mode, [&](auto rc) {
      constexpr int R = decltype(rc)::value;
      return by_bit(pr.s.inject, [&](auto ic) {
        constexpr int I = decltype(ic)::value;
        if (ckpt)
          hipLaunchKernelGGL((k_rollout_fc9_group<R, I, 1>), grid, dim3(cfg.block), 0, st, a);
        else
          hipLaunchKernelGGL((k_rollout_fc9_group<R, I, 0>), grid, dim3(cfg.block), 0, st, a);
        return hipGetLastError();
      });
    });
  }
  const int gx = div_up((size_t)pr.s.N, (size_t)cfg.block);
  const dim3 grid(gx, cfg.cmax_round + gen_rows_for((size_t)gx * cfg.block));
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    return by_bit(pr.s.rng_mode, [&](auto rc) {
      constexpr int R = decltype(rc)::value;
      return by_bit(pr.s.inject, [&](auto ic) {
        constexpr int I = decltype(ic)::value;
        if (precision == 0) {
          auto a = make_args<K, float>(pr, band, early_exit, record, b);
          a.ckpt = b.adj_ckpt;
          a.Kc = Kc;
          a.ckpt_cand = ckpt_cand;
          set_gen(a);
          if (cfg.chance)  // no Newton search, hence no checkpoints
            hipLaunchKernelGGL((k_rollout<K, float, R, I, 0, 1>), grid, dim3(cfg.block), 0, st, a);
          else if (ckpt && cfg.tan)
            hipLaunchKernelGGL((k_rollout<K, float, R, I, 2>), grid, dim3(cfg.block), 0, st, a);
          else if (ckpt)
            hipLaunchKernelGGL((k_rollout<K, float, R, I, 1>), grid, dim3(cfg.block), 0, st, a);
          else
            hipLaunchKernelGGL((k_rollout<K, float, R, I, 0>), grid, dim3(cfg.block), 0, st, a);
        } else {
          auto a = make_args<K, double>(pr, 0.0, early_exit, record, b);
          set_gen(a);
          if (cfg.chance)
            hipLaunchKernelGGL((k_rollout<K, double, R, I, 0, 1>), grid, dim3(cfg.block), 0, st, a);
          else
            hipLaunchKernelGGL((k_rollout<K, double, R, I, 0>), grid, dim3(cfg.block), 0, st, a);
        }
        return hipGetLastError();
      });
    });
  });
}

// The FP64 counterpart of make_quad_coef (same slot layout).
static QuadCoef64 make_quad_coef64(const Problem& pr) {
  QuadCoef64 qc;
  memset(&qc, 0, sizeof(qc));
  const double* A = pr.p.coeffs;
  const double* B = pr.p.coeffs + 16;
  const double* G = pr.p.coeffs + 20;
  const double* E = pr.p.coeffs + 36;
  const double* Cm = pr.p.coeffs + 44;
  double D[4][4];
  for (int r = 0; r < 4; ++r)
    for (int i = 0; i < 4; ++i) {
      double acc = 0.0;
      for (int y = 0; y < 2; ++y) acc += pr.c.F[r * 2 + y] * Cm[y * 4 + i];
      D[r][i] = acc;
    }
  for (int q = 0; q < 4; ++q) {
    for (int s = 0; s < 4; ++s) {
      const int row = q ^ s;
      qc.a[q][s] = A[row * 4 + q];
      qc.g[q][s] = G[row * 4 + q];
      qc.d[q][s] = -D[row][q];
    }
    qc.b[q] = B[q];
    qc.e[q][0] = E[q * 2 + 0];
    qc.e[q][1] = E[q * 2 + 1];
    qc.grow[q] = pr.c.g[q];
  }
  return qc;
}

hipError_t launch_recheck(const Problem& pr, int early_exit, const LaunchCfg& cfg,
                          const DevBuffers& b, hipStream_t st, int decide) {
  const size_t cap = (size_t)cfg.cmax_round * pr.s.N;
  // Few workgroups: each of them counts itself on one device-scope counter at
  // the end (the last one decides), and near-band entries are rare; a
  // grid-stride loop takes any excess.
  if (cfg.lanes == 4 && pr.p.kind == 1 && quad_draws_addressable(pr)) {
    const int qblocks = div_up((cap < 4096 ? cap : 4096) * 4, 256);
    const QuadCoef64 qc = make_quad_coef64(pr);
    auto a = make_args<1, double>(pr, 0.0, early_exit, 0, b);
    return by_bit(pr.s.rng_mode, [&](auto rc) {
      constexpr int R = decltype(rc)::value;
      return by_bit(pr.s.inject, [&](auto ic) {
        constexpr int I = decltype(ic)::value;
        hipLaunchKernelGGL((k_recheck_lq4_quad<R, I>), dim3(qblocks), dim3(256), 0, st, a, qc,
                           make_ctl<1>(pr, b, 0), decide);
        return hipGetLastError();
      });
    });
  }
  // 9-state plant: up to one group of 16 lanes per possible entry (four per
  // workgroup, at most 256 workgroups), for the cooperative FP64 rollout
  const int blocks = pr.p.kind == 2 ? (int)(div_up(cap, 4) < 256 ? div_up(cap, 4) : 256)
                                    : (int)div_up(cap < 16384 ? cap : 16384, 64);
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    return by_bit(pr.s.rng_mode, [&](auto rc) {
      constexpr int R = decltype(rc)::value;
      return by_bit(pr.s.inject, [&](auto ic) {
        constexpr int I = decltype(ic)::value;
        auto a = make_args<K, double>(pr, 0.0, early_exit, 0, b);
        hipLaunchKernelGGL((k_recheck<K, R, I>), dim3(blocks), dim3(64), 0, st, a,
                           make_ctl<K>(pr, b, 0), decide);
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_decide(const Problem& pr, const DevBuffers& b, hipStream_t st) {
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    hipLaunchKernelGGL(k_decide<K>, dim3(1), dim3(128), 0, st, make_ctl<K>(pr, b, 0));
    return hipGetLastError();
  });
}

hipError_t launch_finalize(const Problem& pr, int closed_loop, const DevBuffers& b,
                           hipStream_t st, int setup_next, int when_done) {
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    auto a = make_args<K, double>(pr, 0.0, 0, 0, b);
    hipLaunchKernelGGL(k_finalize<K>, dim3(1), dim3(64), 0, st, a, b.res, b.x_hist, closed_loop,
                       make_ctl<K>(pr, b, closed_loop), setup_next, when_done);
    return hipGetLastError();
  });
}

hipError_t launch_select_q(const DevBuffers& b, int N, int cmax_round, int all, hipStream_t st) {
  hipLaunchKernelGGL(k_select_q, dim3(cmax_round), dim3(256), 0, st, b.srch, b.per_key, N, all);
  return hipGetLastError();
}

hipError_t launch_collect(const DevBuffers& b, int M, double* out_dev, hipStream_t st) {
  hipLaunchKernelGGL(k_collect, dim3(1), dim3(128), 0, st, b.srch, M, out_dev);
  return hipGetLastError();
}

hipError_t launch_draws(const Problem& pr, uint32_t t, int k0, int nk, int j0, int nj,
                        float* w_dev, double* th_dev, const DevBuffers& b, hipStream_t st) {
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    auto a = make_args<K, float>(pr, 0.0, 0, 0, b);
    ThetaNominal thn;
    memset(&thn, 0, sizeof(thn));
    if (K == 2)
      for (int i = 0; i < kMaxTh; ++i) thn.v[i] = pr.p.coeffs[90 + i];
    const size_t work = (size_t)nk * nj + nk;
    hipLaunchKernelGGL(k_draws<K>, dim3(div_up(work, 256)), dim3(256), 0, st, a, t, k0, nk, j0, nj,
                       w_dev, th_dev, thn);
    return hipGetLastError();
  });
}

hipError_t launch_grad_prepare(const Problem& pr, const DevBuffers& b, int cand, int use_keys,
                               hipStream_t st) {
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    hipLaunchKernelGGL(k_grad_prepare<K>, dim3(1), dim3(64), 0, st, make_ctl<K>(pr, b, 0), b.grad,
                       b.adj_k, b.adj_w, cand, use_keys);
    return hipGetLastError();
  });
}

hipError_t launch_adjoint(const Problem& pr, int Kc, int max_entries, const DevBuffers& b,
                          int cand, hipStream_t st) {
  AdjArgs g;
  g.Kc = Kc;
  g.lmax = pr.s.N;
  g.cand = cand;
  g.k_list = b.adj_k;
  g.w_list = b.adj_w;
  g.out_m = b.adj_m;
  g.out_dv = b.adj_dv;
  g.out_dth = b.adj_dth;
  g.ckpt = b.adj_ckpt;
  g.seg = b.adj_seg;
  g.grad = b.grad;
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    return by_bit(pr.s.rng_mode, [&](auto rc) {
      constexpr int R = decltype(rc)::value;
      return by_bit(pr.s.inject, [&](auto ic) {
        constexpr int I = decltype(ic)::value;
        auto a = make_args<K, float>(pr, 0.0, 0, 0, b);
        hipLaunchKernelGGL((k_adjoint<K, R, I>), dim3(div_up(max_entries, 64)), dim3(64), 0, st, a,
                           g);
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_seg_grad(const Problem& pr, int Kc, int cand, const DevBuffers& b,
                           hipStream_t st) {
  SegArgs g;
  g.Kc = Kc;
  g.S = pr.H / Kc + 1;
  g.cand = cand;
  g.lanes = g.S * pr.p.n;
  g.seg_m = b.seg_m;
  g.seg_j = b.seg_j;
  g.seg_r = b.seg_r;
  g.seg_x = b.seg_x;
  g.seg_a = b.seg_a;
  g.seg_cv = b.seg_cv;
  g.seg_ct = b.seg_ct;
  g.scratch = b.seg_scr;
  g.out_m = b.adj_m;
  g.out_dv = b.adj_dv;
  g.out_dth = b.adj_dth;
  g.grad = b.grad;
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    return by_bit(pr.s.rng_mode, [&](auto rc) {
      constexpr int R = decltype(rc)::value;
      return by_bit(pr.s.inject, [&](auto ic) {
        constexpr int I = decltype(ic)::value;
        auto a = make_args<K, float>(pr, 0.0, 0, 0, b);
        hipLaunchKernelGGL((k_seg_min<K, R, I>), dim3(div_up(g.S, 64)), dim3(64), 0, st, a, g,
                           (const float*)b.adj_ckpt);
        hipLaunchKernelGGL((k_seg_vjp<K, R, I>), dim3(div_up(g.lanes, 64)), dim3(64), 0, st, a, g,
                           (const float*)b.adj_ckpt);
        hipLaunchKernelGGL((k_seg_combine<K, R, I>), dim3(1), dim3(64), 0, st, a, g);
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_tan_grad(const Problem& pr, const DevBuffers& b, int cand, hipStream_t st) {
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    hipLaunchKernelGGL(k_tan_grad<K>, dim3(1), dim3(64), 0, st, make_ctl<K>(pr, b, 0), b.grad,
                       (const float*)b.tan_dv, cand);
    return hipGetLastError();
  });
}

hipError_t launch_grad_reduce(const DevBuffers& b, int max_entries, int nth, int cand,
                              hipStream_t st) {
  (void)max_entries;
  hipLaunchKernelGGL(k_grad_reduce, dim3(1), dim3(256), 0, st, b.grad, b.adj_dv, b.adj_dth, nth,
                     b.st, b.srch, cand);
  return hipGetLastError();
}

hipError_t launch_equilibrium(const Problem& pr, const DevBuffers& b, double v, double* out_dev,
                              hipStream_t st) {
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    hipLaunchKernelGGL(k_equilibrium<K>, dim3(1), dim3(64), 0, st, make_ctl<K>(pr, b, 0), v, out_dev);
    return hipGetLastError();
  });
}

hipError_t launch_alg2(const Problem& pr, double band, int precision, int early_exit, int K,
                       int block, const DevBuffers& b, hipStream_t st) {
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int KD = decltype(kc)::value;
    const int nodes = 1 << K;
    hipLaunchKernelGGL(k_alg2_setup<KD>, dim3(div_up(nodes, 64)), dim3(64), 0, st,
                       make_ctl<KD>(pr, b, 0), b.alg2_mss, nodes);
    const dim3 grid(div_up((size_t)pr.s.N, (size_t)block));
    auto a64 = make_args<KD, double>(pr, 0.0, early_exit, 0, b);
    hipError_t e = by_bit(pr.s.rng_mode, [&](auto rc) {
      constexpr int R = decltype(rc)::value;
      return by_bit(pr.s.inject, [&](auto ic) {
        constexpr int I = decltype(ic)::value;
        if (precision == 0) {
          auto a = make_args<KD, float>(pr, band, early_exit, 0, b);
          hipLaunchKernelGGL((k_alg2<KD, float, R, I>), grid, dim3(block), 0, st, a, a64,
                             (const double*)b.alg2_mss, K);
        } else {
          hipLaunchKernelGGL((k_alg2<KD, double, R, I>), grid, dim3(block), 0, st, a64, a64,
                             (const double*)b.alg2_mss, K);
        }
        return hipGetLastError();
      });
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_alg2_finalize, dim3(1), dim3(64), 0, st, b.srch, b.st, b.res);
    return hipGetLastError();
  });
}

// The FP64 tanh of the FP64 rollouts, evaluated on the device (tests).
__global__ void k_eval_tanh64(const double* x, double* y, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = t_tanh(x[i]);
}

hipError_t launch_eval_tanh64(const double* x_dev, double* y_dev, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_eval_tanh64, dim3(div_up((size_t)n, 256)), dim3(256), 0, st, x_dev, y_dev, n);
  return hipGetLastError();
}

size_t flat_args_size(int kind) {
  return kind == 1 ? sizeof(RollArgs<1, float>) : sizeof(RollArgs<2, float>);
}

void flat_fill_args(const Problem& pr, double band, int early, const DevBuffers& b, void* out) {
  if (pr.p.kind == 1) {
    const RollArgs<1, float> a = make_args<1, float>(pr, band, early, 0, b);
    memcpy(out, &a, sizeof(a));
  } else {
    const RollArgs<2, float> a = make_args<2, float>(pr, band, early, 0, b);
    memcpy(out, &a, sizeof(a));
  }
}

size_t flat_args64_size(int kind) {
  return kind == 1 ? sizeof(RollArgs<1, double>) : sizeof(RollArgs<2, double>);
}
size_t flat_ctl_size(int kind) { return kind == 1 ? sizeof(CtlArgs<1>) : sizeof(CtlArgs<2>); }

void flat_fill_args64(const Problem& pr, int early, const DevBuffers& b, void* out) {
  if (pr.p.kind == 1) {
    const RollArgs<1, double> a = make_args<1, double>(pr, 0.0, early, 0, b);
    memcpy(out, &a, sizeof(a));
  } else {
    const RollArgs<2, double> a = make_args<2, double>(pr, 0.0, early, 0, b);
    memcpy(out, &a, sizeof(a));
  }
}

void flat_fill_ctl(const Problem& pr, const DevBuffers& b, void* out) {
  if (pr.p.kind == 1) {
    const CtlArgs<1> a = make_ctl<1>(pr, b, 0);
    memcpy(out, &a, sizeof(a));
  } else {
    const CtlArgs<2> a = make_ctl<2>(pr, b, 0);
    memcpy(out, &a, sizeof(a));
  }
}

hipError_t launch_flat_recheck(int kind, int inject, const void* args64_dev, const void* ctl_dev,
                               int count, hipStream_t st) {
  return by_kind(kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    return by_bit(inject, [&](auto ic) {
      constexpr int I = decltype(ic)::value;
      hipLaunchKernelGGL((k_flat_recheck<K, I>), dim3(count), dim3(64), 0, st,
                         (const RollArgs<K, double>*)args64_dev, (const CtlArgs<K>*)ctl_dev);
      return hipGetLastError();
    });
  });
}

hipError_t launch_flat_setup(int kind, const void* ctl_dev, int count, hipStream_t st) {
  return by_kind(kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    hipLaunchKernelGGL(k_flat_setup<K>, dim3(count), dim3(128), 0, st, (const CtlArgs<K>*)ctl_dev);
    return hipGetLastError();
  });
}

hipError_t launch_flat_finalize(int kind, const void* ctl_dev, DevResult* const* res_dev, int count,
                                hipStream_t st) {
  return by_kind(kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    hipLaunchKernelGGL(k_flat_finalize<K>, dim3(div_up(count, 64)), dim3(64), 0, st,
                       (const CtlArgs<K>*)ctl_dev, res_dev, count);
    return hipGetLastError();
  });
}

hipError_t launch_flat_rollout(int kind, int inject, const void* args_dev, const int* tile_inst,
                               const int* tile_first, int tiles, int cmax, int block,
                               hipStream_t st) {
  const dim3 grid(tiles, cmax);
  return by_kind(kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    return by_bit(inject, [&](auto ic) {
      constexpr int I = decltype(ic)::value;
      hipLaunchKernelGGL((k_flat_rollout<K, I>), grid, dim3(block), 0, st,
                         (const RollArgs<K, float>*)args_dev, tile_inst, tile_first);
      return hipGetLastError();
    });
  });
}

hipError_t launch_trajectory(const Problem& pr, double v, const int32_t* k_list_dev, int nk,
                             int precision, double* traj_dev, const DevBuffers& b,
                             hipStream_t st) {
  return by_kind(pr.p.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    return by_bit(pr.s.rng_mode, [&](auto rc) {
      constexpr int R = decltype(rc)::value;
      return by_bit(pr.s.inject, [&](auto ic) {
        constexpr int I = decltype(ic)::value;
        if (precision == 0) {
          auto a = make_args<K, float>(pr, 0.0, 0, 0, b);
          hipLaunchKernelGGL((k_traj<K, float, R, I>), dim3(div_up(nk, 64)), dim3(64), 0, st, a,
                             (float)v, k_list_dev, nk, traj_dev);
        } else {
          auto a = make_args<K, double>(pr, 0.0, 0, 0, b);
          hipLaunchKernelGGL((k_traj<K, double, R, I>), dim3(div_up(nk, 64)), dim3(64), 0, st, a,
                             v, k_list_dev, nk, traj_dev);
        }
        return hipGetLastError();
      });
    });
  });
}

}  // namespace rg
