// nbx_bs_device.h -- per-particle work of the block time-step integrator: Hermite corrector,
// interpolated derivatives, time-step criteria and power-of-two quantisation (the formulas are
// listed in nbx_blockstep.hip).  Shared by the corrector kernel and the split-combine kernel,
// which runs it directly on the combined forces of a block step.
#pragma once

#include "nbx_internal.h"
#include "nbx_predict.h"

namespace nbx {

__device__ __forceinline__ double norm3(const double v[3]) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

// Step level k of a power-of-two step dt = 2^-k (0 <= k < kBsLevels), from the exponent bits.
__device__ __forceinline__ int bs_level(double dt) {
  return 1023 - (int)((__double_as_longlong(dt) >> 52) & 0x7ff);
}

// A step clamped at dt_min (or a criterion that is not a number): counted for the host.
__device__ inline void report_clamp(const BlockStepParams &bp) {
  atomicAdd(&bp.err[3], 1);
  atomicAdd(&bp.sched->clamped, 1);
}

// Power-of-two step for the criterion `crit`, from the current step dt_old ending at t1.
__device__ inline double quantise(double crit, double dt_old, double t1, const BlockStepParams &bp) {
  if (!(crit >= 0.0)) {  // NaN or negative: keep the step and report it
    report_clamp(bp);
    return dt_old;
  }
  double dn = dt_old;
  if (crit < dt_old) {
    while (dn > crit && dn > bp.dt_min) dn *= 0.5;
    if (dn > crit) report_clamp(bp);  // clamped at dt_min
  } else if (crit >= 2.0 * dt_old && 2.0 * dt_old <= bp.dt_max && fmod(t1, 2.0 * dt_old) == 0.0) {
    dn = 2.0 * dt_old;
  }
  return dn;
}

// Ratio guard: a zero denominator (e.g. a particle far from everything) allows the largest step.
__device__ __forceinline__ double safe_ratio(double num, double den, double big) {
  return den > 0.0 ? num / den : big;
}

// State of particle i at the start of its step: the source record and the step.
struct BsState {
  Raw r;
  double dt;
};

template <int Order>
__device__ __forceinline__ void bs_load_state(const BlockStepParams &bp, int i, BsState &st) {
  load_raw<Order>(bp.src, i, st.r);
  st.dt = bp.dt[i];
}

// Correct particle i, whose state at t0 is st and whose forces at t1 are a1, j1 (and s1 for
// order 6): Hermite corrector, interpolated higher derivatives, step criterion and quantisation;
// the state at t1 is written back into the source arrays.  Called by k_bs_correct and, fused, by
// the split-combine kernel (which loads st before it sums the partial forces).
template <int Order>
__device__ inline void bs_correct_particle(const BlockStepParams &bp, int i, const BsState &st, double t1,
                                           const double a1[3], const double j1[3], const double s1[3]) {
  const Raw &r = st.r;
  const double dt = st.dt;
  const double h = 0.5 * dt;
  const double h2 = h * h;
  double x1[3], v1[3];
  double d2[3], d3[3], d4[3] = {0.0, 0.0, 0.0}, d5[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double am = a1[c] - r.a[c], ap = a1[c] + r.a[c];
    const double jm = j1[c] - r.j[c], jp = j1[c] + r.j[c];
    if constexpr (Order == 4) {
      v1[c] = r.v[c] + h * ap - (h2 / 3.0) * jm;
      x1[c] = r.x[c] + h * (r.v[c] + v1[c]) - (h2 / 3.0) * am;
      const double c2 = jm / (4.0 * h);
      const double c3 = (h * jp - am) / (4.0 * h2 * h);
      d2[c] = 2.0 * c2 + 6.0 * c3 * h;
      d3[c] = 6.0 * c3;
    } else {
      const double sm = s1[c] - r.s[c], sp = s1[c] + r.s[c];
      v1[c] = r.v[c] + h * ap - (0.4 * h2) * jm + (h2 * h / 15.0) * sp;
      x1[c] = r.x[c] + h * (r.v[c] + v1[c]) - (0.4 * h2) * am + (h2 * h / 15.0) * jp;
      const double w4 = (h2 * sp - h * jm) / 16.0;               // c4 h^4
      const double w5 = (h2 * sm - 3.0 * h * jp + 3.0 * am) / 16.0;  // c5 h^5
      const double w3 = (5.0 * h * jp - 5.0 * am - h2 * sm) / 8.0;   // c3 h^3
      const double h3 = h2 * h, h4 = h2 * h2, h5 = h4 * h;
      d2[c] = s1[c];
      d3[c] = (6.0 * w3 + 24.0 * w4 + 60.0 * w5) / h3;
      d4[c] = (24.0 * w4 + 120.0 * w5) / h4;
      d5[c] = 120.0 * w5 / h5;
    }
  }
  const double na = norm3(a1), nj = norm3(j1), n2 = norm3(d2), n3 = norm3(d3);
  const double big = bp.dt_max * bp.dt_max * 4.0;
  const double num = na * n2 + nj * nj;
  double crit = sqrt(bp.eta4 * safe_ratio(num, nj * n3 + n2 * n2, big / bp.eta4));
  if constexpr (Order == 6) {
    const double n4 = norm3(d4), n5 = norm3(d5);
    const double q = safe_ratio(num, n3 * n5 + n4 * n4, -1.0);
    const double dt6 = q < 0.0 ? 2.0 * bp.dt_max : bp.eta6 * pow(q, 1.0 / 6.0);
    crit = 0.5 * (crit + dt6);
  }
  const double dn = quantise(crit, dt, t1, bp);
  if (dn != dt) {  // the particle changes step level
    atomicAdd(&bp.level_count[bs_level(dt)], -1);
    atomicAdd(&bp.level_count[bs_level(dn)], 1);
  }
  bp.src.pos_mass[i] = make_double4(x1[0], x1[1], x1[2], r.m);
  bp.src.vel_time[i] = make_double4(v1[0], v1[1], v1[2], t1);
  double *aj = bp.src.acc_jrk + 6 * (size_t)i;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    aj[c] = a1[c];
    aj[3 + c] = j1[c];
  }
  if constexpr (Order == 6) {
    double *sc = bp.src.snp_crk + 6 * (size_t)i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sc[c] = s1[c];
      sc[3 + c] = d3[c];  // crackle at t1 for the next prediction
    }
  }
  bp.dt[i] = dn;
  bp.tnext[i] = t1 + dn;
}


}  // namespace nbx
