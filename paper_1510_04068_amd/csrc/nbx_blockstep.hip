// nbx_blockstep.hip -- device-resident block time-step Hermite integrator (4th and 6th order).
//
// The paper's library leaves the integrator to the host code (Results > Block time-step
// simulations: between force calls the host corrects the particles, picks their next steps and
// copies them back; the GPU predicts and computes gravity).  Here those host steps run as kernels on the same
// stream, so a block step moves no particle data over PCIe: the particle state lives in the
// library's FP64 source arrays, and only (t_next, N_active) comes back to the host each block step
// (the force launch shape depends on N_active).
//
// One block step:
//   1. schedule: t_next = min_i (t_i + dt_i), found from the occupied step levels, and the list
//      of the particles with t_i + dt_i == t_next (k_bs_list);
//   2. forces on the active particles at t_next: the gravity kernel (fused predictor);
//   3. correct, choose the next step and write the new state back into the source arrays
//      (k_bs_correct, or the split-combine kernel of step 2 when the force launch has splits).
//
// Hermite corrector (Makino & Aarseth 1992 for 4th order; Nitadori & Makino 2008 for 6th), with
// h = dt/2.  Each line is the integral over the step of the Hermite interpolant of the integrand
// through its values and derivatives at both ends:
//   4th: v1 = v0 + h (a0 + a1) - h^2/3 (j1 - j0)
//        x1 = x0 + h (v0 + v1) - h^2/3 (a1 - a0)
//   6th: v1 = v0 + h (a0 + a1) - 2h^2/5 (j1 - j0) + h^3/15 (s0 + s1)
//        x1 = x0 + h (v0 + v1) - 2h^2/5 (a1 - a0) + h^3/15 (j0 + j1)
// The higher derivatives at t1 come from the same interpolant of the acceleration (cubic through
// a, j; quintic through a, j, s) written about the mid-point, tau in [-h, h]:
//   cubic:   c2 = (j1 - j0) / (4h),                 c3 h^3 = (h (j0 + j1) - (a1 - a0)) / 4
//   quintic: c4 h^4 = (h^2 (s0 + s1) - h (j1 - j0)) / 16
//            c5 h^5 = (h^2 (s1 - s0) - 3h (j0 + j1) + 3 (a1 - a0)) / 16
//            c3 h^3 = (5h (j0 + j1) - 5 (a1 - a0) - h^2 (s1 - s0)) / 8
// and a^(k)(h) follows by differentiating sum c_m tau^m.
//
// Time-step criteria (Results > Block time-step simulations; the paper prints no formula):
//   Aarseth:      dt4 = sqrt(eta4 (|a||a2| + |a1|^2) / (|a1||a3| + |a2|^2))
//   6th order:    dt6 = eta6 ((|a||a2| + |a1|^2) / (|a3||a5| + |a4|^2))^(1/6)
//   order 4 uses dt4; order 6 uses the average (dt4 + dt6) / 2, the choice the paper makes for
//   both its DS and DP runs because dt6 alone can collapse when jerk and snap carry rounding noise.
// Block quantisation: steps are powers of two; a particle halves its step until it is at most the
// criterion, and doubles it (once per step, up to dt_max) only when the criterion allows twice the
// step and the new time is a multiple of twice the step, so that blocks stay synchronised.  A step
// that would fall below dt_min is clamped there and counted; the host stops integrating once the
// count is non-zero (the interpolated derivatives are dominated by force rounding noise, which the
// paper observed for the 6th-order criterion with double-single forces).

#include "nbx.h"
#include "nbx_internal.h"
#include "nbx_predict.h"
#include "nbx_bs_device.h"

namespace nbx {

constexpr int kBsPer = kBsChunk / kThreads;  // particles per thread in the scheduling kernel

// Exclusive prefix sum over the workgroup in thread order; *total receives the sum.
__device__ int block_exclusive_scan(int v, int *red, int *total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int inc = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(inc, off);
    if (lane >= off) inc += o;
  }
  if (lane == 63) red[wave] = inc;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wave) before += red[w];
    all += red[w];
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

// Schedule.  Every particle sits on the grid of its own step: t_i is a multiple of dt_i and
// t_i <= T < t_i + dt_i at the last block time T, so t_i + dt_i is the first multiple of dt_i after
// T.  The smallest of these belongs to the finest occupied step level kmax (dt = 2^-kmax), so
// t_next = (floor(T / dt) + 1) dt with no pass over the particles: the per-level counts, kept by
// the start and corrector kernels, name kmax.  The active particles are those with
// t_i + dt_i == t_next.  Each workgroup collects its chunk of kBsChunk particles in address order
// (prefix scan) and reserves their slots in the list with one atomic add on count[parity], which
// the previous schedule zeroed; the chunks land in the list in arrival order.  Every result of a
// block step depends only on the set of active particles, not on their order, because each sink's
// sum order is fixed by the launch shape.  Workgroup 0 publishes t_next and zeroes the other
// counter for the next schedule.
// DD (device-driven runs): the last block time is sched->tnow[parity] and the schedule itself
// decides whether the step is taken (not when the run is stopped, a step has clamped, or t_next
// passes t_end; then the count stays zero and every kernel of the step returns at once).
// Workgroup 0 also counts the step before this schedule and publishes the new block time.  Every
// workgroup reaches the same decision from inputs no kernel of this step writes, except stop,
// which workgroup 0 sets only when the decision is to stop.
template <bool DD>
__global__ __launch_bounds__(kThreads) void k_bs_list(BlockStepParams bp, double t_now, int parity) {
  __shared__ int redi[kThreads / 64];
  __shared__ int base;
  __shared__ double tn_sh;
  __shared__ int go_sh;
  if (DD) t_now = bp.sched->tnow[parity];
  if (threadIdx.x < 64) {
    const bool occ = bp.level_count[threadIdx.x] > 0;
    const uint64_t m = __ballot(occ);
    if (threadIdx.x == 0) {
      double tn = __builtin_huge_val();
      if (m != 0) {
        const int kmax = 63 - __clzll(m);
        const double dt = ldexp(1.0, -kmax);
        tn = (floor(t_now / dt) + 1.0) * dt;
      }
      bool go = m != 0;
      if (DD) go = go && bp.sched->stop == 0 && bp.sched->clamped == 0 && tn <= bp.sched->t_end;
      tn_sh = tn;
      go_sh = go ? 1 : 0;
    }
  }
  __syncthreads();
  const double tn = tn_sh;
  if (DD) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      const int prev = bp.sched->count[parity ^ 1];  // the step before this schedule, now complete
      if (prev > 0) {
        bp.sched->blocks += 1;
        bp.sched->steps += prev;
      }
      bp.sched->count[parity ^ 1] = 0;
      bp.sched->tnow[parity ^ 1] = go_sh ? tn : t_now;
      if (go_sh) bp.sched->t_next = tn;
      else bp.sched->stop = 1;
    }
    if (!go_sh) return;
  }
  // thread t owns the kBsPer consecutive particles b0 + t*kBsPer ... (address order = thread order)
  const int i0 = blockIdx.x * kBsChunk + threadIdx.x * kBsPer;
  bool act[kBsPer];
  int mine = 0;
#pragma unroll
  for (int r = 0; r < kBsPer; ++r) {
    const int i = i0 + r;
    act[r] = i < bp.n && bp.tnext[i] == tn;
    mine += act[r] ? 1 : 0;
  }
  int total = 0;
  const int pos0 = block_exclusive_scan(mine, redi, &total);
  if (threadIdx.x == 0) {
    base = total > 0 ? atomicAdd(&bp.sched->count[parity], total) : 0;
    if (!DD && blockIdx.x == 0) {
      bp.sched->t_next = tn;
      bp.sched->count[parity ^ 1] = 0;
    }
  }
  __syncthreads();
  int pos = base + pos0;
#pragma unroll
  for (int r = 0; r < kBsPer; ++r)
    if (act[r]) bp.list[pos++] = i0 + r;
}

template <int Order>
__global__ __launch_bounds__(kThreads) void k_bs_correct(BlockStepParams bp, int ni, double t1) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k >= ni) return;
  const int i = bp.list[k];
  BsState st;
  bs_load_state<Order>(bp, i, st);
  double a1[3], j1[3], s1[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    a1[c] = bp.acc[3 * (size_t)k + c];
    j1[c] = bp.jrk[3 * (size_t)k + c];
    if constexpr (Order == 6) s1[c] = bp.snp[3 * (size_t)k + c];
  }
  bs_correct_particle<Order>(bp, i, st, t1, a1, j1, s1);
}

// Start: particles at t = 0 with no derivatives yet; list = 0..n-1.
template <int Order>
__global__ __launch_bounds__(kThreads) void k_bs_load(BlockStepParams bp, const int64_t *id, const double *m,
                                                      const double *x, const double *v) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= bp.n) return;
  const size_t b = 3 * (size_t)i;
  bp.src.pos_mass[i] = make_double4(x[b], x[b + 1], x[b + 2], m[i]);
  bp.src.vel_time[i] = make_double4(v[b], v[b + 1], v[b + 2], 0.0);
  double *aj = bp.src.acc_jrk + 6 * (size_t)i;
#pragma unroll
  for (int c = 0; c < 6; ++c) aj[c] = 0.0;
  if constexpr (Order == 6) {
    double *sc = bp.src.snp_crk + 6 * (size_t)i;
#pragma unroll
    for (int c = 0; c < 6; ++c) sc[c] = 0.0;
  }
  bp.src.id[i] = id[i];
  bp.list[i] = i;
  if (i == 0) {
    bp.sched->t_next = 0.0;
    bp.sched->count[0] = bp.sched->count[1] = 0;
    bp.sched->clamped = 0;
    bp.sched->stop = 0;
    bp.sched->tnow[0] = bp.sched->tnow[1] = 0.0;
    bp.sched->t_end = 0.0;
    bp.sched->blocks = bp.sched->steps = 0;
  }
}

// Start, after a force pass on every particle (row i = particle i): store a and j (the 6th-order
// snap needs the sources' accelerations, so order 6 runs a second pass after this).
__global__ __launch_bounds__(kThreads) void k_bs_seed(BlockStepParams bp) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= bp.n) return;
  double *aj = bp.src.acc_jrk + 6 * (size_t)i;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    aj[c] = bp.acc[3 * (size_t)i + c];
    aj[3 + c] = bp.jrk[3 * (size_t)i + c];
  }
}

// Start: first step dt0 = eta_start |a|/|j| (order 6: the smaller of that and
// eta_start sqrt(|a|/|s|)), rounded down to a power of two <= dt_max; crackle starts at zero.
template <int Order>
__global__ __launch_bounds__(kThreads) void k_bs_start(BlockStepParams bp) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= bp.n) return;
  double a[3], j[3], s[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    a[c] = bp.acc[3 * (size_t)i + c];
    j[c] = bp.jrk[3 * (size_t)i + c];
    s[c] = Order == 6 ? bp.snp[3 * (size_t)i + c] : 0.0;
  }
  const double na = norm3(a), nj = norm3(j), ns = norm3(s);
  double d0 = nj > 0.0 ? bp.eta_start * na / nj : bp.dt_max;
  if (Order == 6 && ns > 0.0) d0 = fmin(d0, bp.eta_start * sqrt(na / ns));
  double dn = bp.dt_max;
  while (dn > d0 && dn > bp.dt_min) dn *= 0.5;
  // clamped at dt_min (or NaN): reported by nbx_bs_init, but a crude first estimate does not stop
  // the integration the way a collapsing criterion does
  if (!(dn <= d0) && !(d0 >= bp.dt_max)) atomicAdd(&bp.err[3], 1);
  if constexpr (Order == 6) {
    double *sc = bp.src.snp_crk + 6 * (size_t)i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sc[c] = s[c];
      sc[3 + c] = 0.0;
    }
  }
  bp.dt[i] = dn;
  bp.tnext[i] = dn;
  atomicAdd(&bp.level_count[bs_level(dn)], 1);
}

__global__ __launch_bounds__(kThreads) void k_iota(int32_t *p, int n) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < n) p[i] = i;
}

static inline int grid_for(int n) { return (n + kThreads - 1) / kThreads; }

hipError_t launch_iota(int32_t *p, int n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(kThreads), 0, stream, p, n);
  return hipGetLastError();
}

int bs_groups(int n) { return (n + kBsChunk - 1) / kBsChunk; }

hipError_t launch_bs_schedule(const BlockStepParams &bp, double t_now, int parity, hipStream_t stream) {
  const int g = bs_groups(bp.n);
  hipLaunchKernelGGL(k_bs_list<false>, dim3(g), dim3(kThreads), 0, stream, bp, t_now, parity);
  return hipGetLastError();
}

hipError_t launch_bs_schedule_dd(const BlockStepParams &bp, int parity, hipStream_t stream) {
  const int g = bs_groups(bp.n);
  hipLaunchKernelGGL(k_bs_list<true>, dim3(g), dim3(kThreads), 0, stream, bp, 0.0, parity);
  return hipGetLastError();
}

hipError_t launch_bs_correct(int order, const BlockStepParams &bp, int ni, double t1, hipStream_t stream) {
  if (ni <= 0) return hipSuccess;
  if (order == 6)
    hipLaunchKernelGGL(k_bs_correct<6>, dim3(grid_for(ni)), dim3(kThreads), 0, stream, bp, ni, t1);
  else
    hipLaunchKernelGGL(k_bs_correct<4>, dim3(grid_for(ni)), dim3(kThreads), 0, stream, bp, ni, t1);
  return hipGetLastError();
}

hipError_t launch_bs_load(int order, const BlockStepParams &bp, const int64_t *id, const double *m, const double *x,
                          const double *v, hipStream_t stream) {
  if (order == 6)
    hipLaunchKernelGGL(k_bs_load<6>, dim3(grid_for(bp.n)), dim3(kThreads), 0, stream, bp, id, m, x, v);
  else
    hipLaunchKernelGGL(k_bs_load<4>, dim3(grid_for(bp.n)), dim3(kThreads), 0, stream, bp, id, m, x, v);
  return hipGetLastError();
}

hipError_t launch_bs_seed(const BlockStepParams &bp, hipStream_t stream) {
  hipLaunchKernelGGL(k_bs_seed, dim3(grid_for(bp.n)), dim3(kThreads), 0, stream, bp);
  return hipGetLastError();
}

hipError_t launch_bs_start(int order, const BlockStepParams &bp, hipStream_t stream) {
  if (order == 6)
    hipLaunchKernelGGL(k_bs_start<6>, dim3(grid_for(bp.n)), dim3(kThreads), 0, stream, bp);
  else
    hipLaunchKernelGGL(k_bs_start<4>, dim3(grid_for(bp.n)), dim3(kThreads), 0, stream, bp);
  return hipGetLastError();
}

}  // namespace nbx
