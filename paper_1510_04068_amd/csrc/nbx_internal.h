// nbx_internal.h -- definitions shared by the HIP kernels and the host runtime of libnbx.
//
// Device layout of the source ("j-particle") state.  Sources are always stored in FP64
// (Methods > Numerical Accuracy); the arithmetic precision is chosen per force call.
// Records are structure-of-arrays so that one thread per source reads them with coalesced
// 16-byte loads:
//   pos_mass[a] = (x, y, z, m)            32 B
//   vel_time[a] = (vx, vy, vz, t_j)       32 B
//   acc_jrk[a]  = (ax, ay, az, jx, jy, jz) 48 B
//   snp_crk[a]  = (sx, sy, sz, cx, cy, cz) 48 B   (orders 6 and 8 only)
//   id[a]       int64
// The arrays hold nj_max entries; entries never written hold a massless source at
// (1e18, 1e18, 1e18) with id -1.  The force kernel reads addresses [0, nj) and substitutes
// the same massless far-away source for the tail [nj, nj_pad) of the last LDS tile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nbx {

constexpr int kThreads = 256;  // workgroup size: 4 wave64s
constexpr int kTile = 256;     // sources per LDS tile (one per thread when staging)
// Position of padding sources: far enough that every term is negligible, near enough that R^2
// (~3e36) stays finite in FP32, so R^-1 (and any Newton step on it) stays finite too.
constexpr double kPadPos = 1e18;

struct SourceArrays {
  double4 *pos_mass;
  double4 *vel_time;
  double *acc_jrk;
  double *snp_crk;
  int64_t *id;
};

// Block time-step integrator (device resident).  The particle state is the source arrays; the
// force rows acc/jrk/snp are those of the active list (row k = particle list[k]).
constexpr int kBsChunk = 4 * kThreads;  // particles per workgroup in the scheduling kernel
constexpr int kBsLevels = 64;            // step levels k, dt = 2^-k (dt_min >= 2^-63)
struct BsSched {
  double t_next;  // next block time
  int count[2];   // active particles at t_next; schedules alternate between the two counters
  int clamped;    // steps clamped at dt_min (or with a criterion that is not a number) since the start
  int stop;       // device-driven runs: set once the next block time passes t_end or a step clamped
  // device-driven runs: the block time before the schedule of parity p is tnow[p], after it
  // tnow[p ^ 1]; t_end of the run; block steps and particle steps taken (each schedule counts the
  // step before it)
  double tnow[2];
  double t_end;
  long long blocks, steps;
};
struct BlockStepParams {
  SourceArrays src;
  int n;
  double eta4, eta6, eta_start, dt_max, dt_min;
  double *dt;       // [n] current step of each particle (power of two)
  double *tnext;    // [n] t_i + dt_i
  int32_t *list;    // [n] active particles of the current block step (address order within chunks)
  int *level_count;  // [kBsLevels] particles per step level k (dt = 2^-k)
  BsSched *sched;
  const double *acc, *jrk, *snp;  // forces of the active list at the block time
  int *err;                       // [3]: steps clamped at dt_min or criteria that were not numbers
};

// One force launch.  Sinks are either taken by address from the predicted sources (i_addr) or
// given explicitly (ext_*, with self-exclusion by id).
struct ForceParams {
  SourceArrays src;
  int nj;      // sources in use
  int nj_pad;  // nj rounded up to kTile
  double t;    // prediction time
  double eps2;
  int ni;
  const int32_t *i_addr;  // by-address sinks [ni]
  const int32_t *ext_self;  // explicit sinks: address of the source with the sink's id, or -1
  const int64_t *ext_id;    // explicit sinks: id [ni], x/v/a [ni][3] (ext_x == nullptr: by address)
  const double *ext_x;
  const double *ext_v;
  const double *ext_a;  // order 6 and 8: sink accelerations
  const double *ext_j;  // order 8: sink jerks
  const double *h2;  // [ni] squared neighbour radii, or nullptr
  int nbr_max;
  int nn;  // nonzero: nearest-neighbour search (nn_id, nn_r2 written); 0: skipped, outputs untouched
  // launch shape
  int lanes_log2;  // lanes per sink = 1 << lanes_log2 (1..256)
  int splits;      // source splits S (workgroups per sink block)
  // outputs (device)
  double *acc;
  double *jrk;
  double *snp;
  double *crk;  // order 8: crackle of the sinks
  double *pot;
  int64_t *nn_id;
  double *nn_r2;
  int32_t *nbr_count;
  int64_t *nbr_ids;
  // split-combine scratch (S > 1), written by k_force and read by k_combine: split-major
  // part[(s*K + k)*ni + q], part_key/part_idx[s*ni + q], or with part_sm sink-major
  // part[(q*K + k)*S + s], part_key/part_idx[q*S + s]
  int part_sm;
  double *part;
  uint64_t *part_key;
  int32_t *part_idx;
  // with the nearest-neighbour search and S > 1: the FP64 predicted position of each sink,
  // part_xi[3*q + k], written by the split-0 workgroups during their sink set-up so that the
  // combine's exact |r|^2 needs no second load of the sink's address and state (null: not kept)
  double *part_xi;
  int *err;  // device-side error counters: [0] bad sink address, [1] bad source address, [2] list overflow
  // block time-step step (bs_fuse != 0, only with S > 1): the combine kernel corrects particle
  // bs.list[q] at time bs_t1 instead of writing sink q's outputs
  int bs_fuse;
  double bs_t1;
  BlockStepParams bs;
  // device-driven block steps (k_force_dd / k_combine_dd): N_i = *dd_count and the prediction time
  // *dd_t are read on the device; dd_shape[k] = (lanes_log2, splits) for N_i in (2^(k-1), 2^k]
  const int *dd_count;
  const double *dd_t;
  int2 dd_shape[32];
};

// Batched few-body systems: particles of system s are [offset[s], offset[s+1]); items[k] =
// (system, lanes_log2, first sink, end sink), one wave per item, in schedule order.
constexpr int kBatchMax = 128;  // largest system of a batch
struct BatchParams {
  int n_items;
  const int4 *items;  // (system, lanes_log2, first sink, end sink), the costliest first
  const int32_t *offset;
  const double *m;
  const double *x;
  const double *v;
  double eps2;
  double *acc;
  double *jrk;
  double *pot;
};

// Adjoint of the 4th-order forces of a closed system (every particle a sink and a source).
struct VjpParams {
  int n;
  int n_pad;   // n rounded up to kTile
  int splits;  // source splits S; partials part[(s*7 + k)*n + p] when S > 1
  double eps2;
  const double *m;
  const double *x;
  const double *v;
  const double *g_acc;
  const double *g_jerk;
  const double *g_pot;
  double *grad_x;
  double *grad_v;
  double *grad_m;
  double *part;
};

// Combine kernel: sinks per workgroup W = 2^wlog, with R = 256 / W threads per sink: R =
// nextpow2(S) (at most 256), but at least min(nextpow2(N_i), kCombineQ) sinks per workgroup, so
// that a load instruction covers whole cache lines of partials.  Shared by the host launchers and
// the device-driven kernel.
constexpr int kCombineQ = 16;
__host__ __device__ inline int combine_wlog(int ni, int S) {
  int qmin = 1;
  while (qmin < ni && qmin < kCombineQ) qmin *= 2;
  int rlog = 0;
  while ((1 << rlog) < S && (1 << rlog) < kThreads / qmin) ++rlog;
  return 8 - rlog;
}

// Sink-major partials (small N_i, many splits): one workgroup per sink or few sinks, R =
// nextpow2(S) threads per sink (at most 256) reading consecutive splits.
constexpr int kSinkMajorMaxNi = 256;  // largest N_i combined sink-major (A/B: -13% at N_i = 64, -6% at 256, neutral at 512, +4% at 1024)
constexpr int kSinkMajorMinS = 64;     // fewest splits combined sink-major
__host__ __device__ inline int combine_wlog_sink_major(int S) {
  int rlog = 0;
  while ((1 << rlog) < S && rlog < 8) ++rlog;
  return 8 - rlog;
}

struct LaunchShape {
  int lanes_log2;
  int sinks_per_lane;
  int splits;
  int blocks;  // sink blocks
};

// Kernel entry points (defined in nbx_kernels.hip).
hipError_t launch_force(int order, int precision, const ForceParams &fp, const LaunchShape &ls,
                        hipStream_t stream);
// Device-driven block step (orders 4 and 6): gravity with force_groups workgroups, then the
// combine + corrector with combine_groups workgroups; both loop over their work.
hipError_t launch_force_dd(int order, int precision, const ForceParams &fp, int force_groups, int combine_groups,
                           hipStream_t stream);
hipError_t launch_jupdate(int order, const SourceArrays &src, int nj_cap, int n, const int32_t *addr,
                          const int64_t *id, const double *m, const double *t, const double *x,
                          const double *v, const double *a, const double *jerk, const double *snap,
                          const double *crackle, int *err, hipStream_t stream);
hipError_t launch_pad(int order, const SourceArrays &src, int from, int to, hipStream_t stream);
hipError_t launch_predict_out(int order, const SourceArrays &src, int nj, double t, int n,
                              const int32_t *addr, double *xp, double *vp, double *ap, int *err,
                              hipStream_t stream);
hipError_t launch_gather_j(int order, const SourceArrays &src, int n, const int32_t *addr,
                           int64_t *id, double *m, double *t, double *x, double *v, double *a,
                           double *jerk, double *snap, double *crackle, hipStream_t stream);
hipError_t launch_fill_i32(int32_t *p, int n, int value, hipStream_t stream);
hipError_t launch_clock_sample(int n_groups, int64_t *out, hipStream_t stream);
hipError_t launch_vjp(int precision, const VjpParams &vp, hipStream_t stream);
hipError_t launch_batch(int precision, const BatchParams &bp, int grid, hipStream_t stream);
// Workgroups of the batch kernel resident on the device at once (occupancy x CUs), 0 if unknown.
int batch_resident_groups(int precision, int device);
hipError_t launch_selfmap(const SourceArrays &src, int nj, int ni, const int64_t *ext_id, int32_t *self,
                          hipStream_t stream);

// Block time-step kernels (defined in nbx_blockstep.hip).
int bs_groups(int n);
// Schedules the block step after the last block time t_now, counting into sched->count[parity].
hipError_t launch_bs_schedule(const BlockStepParams &bp, double t_now, int parity, hipStream_t stream);
// Device-driven schedule: the block time and t_end come from bp.sched (see BsSched).
hipError_t launch_bs_schedule_dd(const BlockStepParams &bp, int parity, hipStream_t stream);
hipError_t launch_bs_correct(int order, const BlockStepParams &bp, int ni, double t1, hipStream_t stream);
hipError_t launch_bs_load(int order, const BlockStepParams &bp, const int64_t *id, const double *m, const double *x,
                          const double *v, hipStream_t stream);
hipError_t launch_bs_seed(const BlockStepParams &bp, hipStream_t stream);
hipError_t launch_bs_start(int order, const BlockStepParams &bp, hipStream_t stream);
hipError_t launch_iota(int32_t *p, int n, hipStream_t stream);

// Launch-shape rule (defined in nbx_kernels.hip).
LaunchShape choose_shape(int ni, int nj_pad, int prec, int order);
int values_per_sink(int order);  // doubles per sink in the split-combine scratch

}  // namespace nbx
