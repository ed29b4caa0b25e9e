// nbx_predict.h -- the FP64 Taylor predictor of the sources, shared by every kernel that needs a
// predicted state (the gravity kernel's tile staging and sink set-up, the standalone predictor,
// the block time-step corrector), so that all of them compute the same bits for the same source.
#pragma once

#include "nbx_internal.h"

namespace nbx {

// ---------------------------------------------------------------------------------------------
// Source state and the FP64 Taylor predictor
// ---------------------------------------------------------------------------------------------
struct Raw {
  double x[3], m, v[3], tj, a[3], j[3], s[3], c[3];
};

template <int Order>
__device__ __forceinline__ void load_raw(const SourceArrays &src, int addr, Raw &r) {
  const double4 pm = src.pos_mass[addr];
  const double4 vt = src.vel_time[addr];
  r.x[0] = pm.x; r.x[1] = pm.y; r.x[2] = pm.z; r.m = pm.w;
  r.v[0] = vt.x; r.v[1] = vt.y; r.v[2] = vt.z; r.tj = vt.w;
  const double2 *aj = reinterpret_cast<const double2 *>(src.acc_jrk + 6 * (size_t)addr);
  const double2 q0 = aj[0], q1 = aj[1], q2 = aj[2];
  r.a[0] = q0.x; r.a[1] = q0.y; r.a[2] = q1.x;
  r.j[0] = q1.y; r.j[1] = q2.x; r.j[2] = q2.y;
  if constexpr (Order >= 6) {
    const double2 *sc = reinterpret_cast<const double2 *>(src.snp_crk + 6 * (size_t)addr);
    const double2 s0 = sc[0], s1 = sc[1], s2 = sc[2];
    r.s[0] = s0.x; r.s[1] = s0.y; r.s[2] = s1.x;
    r.c[0] = s1.y; r.c[1] = s2.x; r.c[2] = s2.y;
  }
}

// Taylor polynomial about t_j in Horner form with explicit FMAs and contraction disabled, so
// that every call site computes the same bits for the same source.  Order 8 predicts x, v and a
// as order 6 does and in addition the jerk (to second order in dt, from snap and crackle), which
// it returns in ap[3..5]; ap has 6 entries there, 3 otherwise.
template <int Order>
__device__ __forceinline__ void predict_raw(const Raw &r, double t, double xp[3], double vp[3],
                                            double *ap) {
#pragma clang fp contract(off)
  const double dt = t - r.tj;
  const double h2 = dt * 0.5;
  const double h3 = dt * (1.0 / 3.0);
  if constexpr (Order == 2) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      xp[k] = fma(dt, fma(h2, r.a[k], r.v[k]), r.x[k]);
      vp[k] = fma(dt, r.a[k], r.v[k]);
      ap[k] = r.a[k];
    }
  } else if constexpr (Order == 4) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      xp[k] = fma(dt, fma(h2, fma(h3, r.j[k], r.a[k]), r.v[k]), r.x[k]);
      vp[k] = fma(dt, fma(h2, r.j[k], r.a[k]), r.v[k]);
      ap[k] = fma(dt, r.j[k], r.a[k]);
    }
  } else {
    const double h4 = dt * 0.25;
    const double h5 = dt * 0.2;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      xp[k] = fma(dt, fma(h2, fma(h3, fma(h4, fma(h5, r.c[k], r.s[k]), r.j[k]), r.a[k]), r.v[k]), r.x[k]);
      vp[k] = fma(dt, fma(h2, fma(h3, fma(h4, r.c[k], r.s[k]), r.j[k]), r.a[k]), r.v[k]);
      ap[k] = fma(dt, fma(h2, fma(h3, r.c[k], r.s[k]), r.j[k]), r.a[k]);
      if constexpr (Order == 8) ap[3 + k] = fma(dt, fma(h2, r.c[k], r.s[k]), r.j[k]);
    }
  }
}

template <int Order>
__device__ __forceinline__ void predict_addr(const SourceArrays &src, int addr, double t,
                                             double xp[3], double vp[3], double *ap, double &m) {
  Raw r;
  load_raw<Order>(src, addr, r);
  predict_raw<Order>(r, t, xp, vp, ap);
  m = r.m;
}

}  // namespace nbx
