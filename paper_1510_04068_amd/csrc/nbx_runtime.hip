// nbx_runtime.hip -- host runtime and C ABI of libnbx (declared in include/nbx.h).
//
// A context owns: the FP64 source arrays (Methods > Numerical Accuracy: data always stored in
// double precision), the sink-side buffers of the host-pointer path, the split-combine scratch
// of the gravity kernel, and one HIP stream at default priority.  Every entry point validates
// its arguments, maps HIP failures to NBX_ERR_DEVICE with a message, and never throws.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "nbx.h"
#include "nbx_internal.h"

using namespace nbx;

namespace {

constexpr int kVersion = 10300;  // 1.3.0: want_nn (kernels without the nearest-neighbour search)

std::string g_open_error;  // message of the last failed nbx_open

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Pinned host staging for the host-pointer path: host arrays are packed into it with memcpy and
// move in one asynchronous copy; `ev` marks the end of the last copy that used it.
struct Pinned {
  void *h = nullptr;
  size_t bytes = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};

constexpr int kBatchMaxGroups = 8 * 256;  // batched launch: at most 8 workgroups per CU
constexpr size_t kErrDoubles = 8;  // the error counters head the output block (64 bytes)
// Host transfers up to this size go through pinned staging (one copy, no per-array overhead);
// larger ones copy straight from / to the caller's pageable arrays, which the runtime pipelines
// better than a host memcpy followed by one DMA.
constexpr size_t kStageMax = size_t(1) << 20;

// Split partials of the allocation-free entry point (nbx_force_dev_noalloc) live in this
// file-scope device array, one copy per GPU for the life of the process.  Host code never uses
// its name as an address: nbx_open looks up its device address once per device (scratch_setup)
// and every launch takes that pointer.
constexpr size_t kNoallocScratchBytes = size_t(NBX_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` on each device

}  // namespace

struct nbx_ctx {
  nbx_config cfg{};
  int precision = NBX_FP64;
  hipStream_t stream = nullptr;
  int nj = 0;
  bool predicted = false;
  double t_pred = 0.0;
  SourceArrays src{};
  // host-pointer path: sink inputs and results
  int32_t *d_iaddr = nullptr;
  double *d_h2 = nullptr;
  int64_t *d_ext_id = nullptr;
  double *d_ext_x = nullptr, *d_ext_v = nullptr, *d_ext_a = nullptr, *d_ext_j = nullptr;
  int32_t *d_ext_self = nullptr;
  // results of the last host-path force call, laid out for its ni in one block behind the error
  // counters (d_out), so that nbx_get_force moves counters and results in one copy
  double *d_out = nullptr;
  size_t out_doubles = 0;
  double *d_acc = nullptr, *d_jrk = nullptr, *d_snp = nullptr, *d_crk = nullptr, *d_pot = nullptr,
         *d_nnr2 = nullptr;
  int64_t *d_nnid = nullptr;
  Pinned stage_j, stage_i, stage_out;  // staging of nbx_set_j, of the sink inputs, of the results
  int32_t *d_nbr_cnt = nullptr;
  int64_t *d_nbr_ids = nullptr;
  // split-combine scratch
  DevBuf part, part_key, part_idx, part_xi;
  void *noalloc_scratch = nullptr;  // this device's static scratch (nbx_force_dev_noalloc)
  int *d_err = nullptr;  // [0] bad sink address, [1] bad source address, [2] nbr overflow, [3] dt clamped
                         // (the first 16 bytes of d_out)
  // set_j staging (host path), grown on demand
  DevBuf up;
  int up_cap = 0;
  // batched few-body systems
  std::vector<int32_t> batch_sizes;
  int32_t *d_batch_offset = nullptr;
  DevBuf batch_items;
  int batch_n_items = 0;
  int batch_lg[8] = {-1, -1, -1, -1, -1, -1, -1, -1};  // lanes_log2 per size class (-1: default)
  // block time-step integrator: particle state in the source arrays, addresses 0..n-1
  struct {
    bool ready = false;
    int n = 0;
    nbx_bs_params p{};
    double t = 0.0;
    int64_t blocks = 0, steps = 0;
    DevBuf dt, tnext, list, acc, jrk, snp, pot, level_count, sched;
    int parity = 0;  // counter of the next schedule
    BsSched *h_sched = nullptr;  // pinned host copy of the schedule
  } bs;
  // launch-shape tables from nbx_tune, per precision: per N_i class k (ni in (2^(k-1), 2^k]),
  // valid while the number of source tiles is tune_ntiles[precision]; force_shape overrides
  // everything while tuning
  struct TunedShape {
    int lanes_log2 = -1, sinks_per_lane = 1, splits = 1;
  } tuned[3][32];
  int tune_ntiles[3] = {0, 0, 0};
  const LaunchShape *force_shape = nullptr;
  // state of the last force call (host path)
  int last_ni = -1;
  bool last_nbr = false;
  bool last_nn = false;
  std::vector<void *> owned;
  std::string err;
};

namespace {

int fail(nbx_ctx *c, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c)
    c->err = buf;
  else
    g_open_error = buf;
  return code;
}

int hip_fail(nbx_ctx *c, hipError_t e, const char *what) {
  return fail(c, NBX_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(c, expr)                                   \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return hip_fail((c), e_, #expr); \
  } while (0)

int alloc(nbx_ctx *c, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return NBX_OK;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(c, NBX_ERR_OOM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
  }
  c->owned.push_back(*p);
  return NBX_OK;
}

template <typename T>
int alloc_n(nbx_ctx *c, T **p, size_t n) {
  return alloc(c, reinterpret_cast<void **>(p), n * sizeof(T));
}

// Grow a scratch buffer to at least `bytes` (contents are not preserved).
int grow(nbx_ctx *c, DevBuf &b, size_t bytes) {
  if (b.bytes >= bytes) return NBX_OK;
  if (b.p) {
    auto it = std::find(c->owned.begin(), c->owned.end(), b.p);
    if (it != c->owned.end()) c->owned.erase(it);
    hipError_t e = hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    if (e != hipSuccess) return hip_fail(c, e, "hipFree");
  }
  int rc = alloc(c, &b.p, bytes);
  if (rc == NBX_OK) b.bytes = bytes;
  return rc;
}

int set_device(nbx_ctx *c) {
  HIP_TRY(c, hipSetDevice(c->cfg.device));
  return NBX_OK;
}

// Device address of the static scratch on the context's device (current): looked up once per
// device and kept for the life of the process.
int scratch_setup(nbx_ctx *c) {
  const int d = c->cfg.device;
  if (d < 0 || d >= kMaxDevices) return fail(c, NBX_ERR_NO_DEVICE, "device %d beyond %d", d, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[d]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(c, NBX_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[d] = ptr;
  }
  c->noalloc_scratch = g_scratch_ptr[d];
  return NBX_OK;
}

int ensure_scratch(nbx_ctx *c, int ni, const LaunchShape &ls) {
  if (ls.splits <= 1) return NBX_OK;
  const size_t K = (size_t)values_per_sink(c->cfg.order);
  const size_t n = (size_t)ls.splits * (size_t)ni;
  int rc = grow(c, c->part, n * K * sizeof(double));
  if (rc) return rc;
  rc = grow(c, c->part_key, n * sizeof(uint64_t));
  if (rc) return rc;
  rc = grow(c, c->part_idx, n * sizeof(int32_t));
  if (rc) return rc;
  return grow(c, c->part_xi, (size_t)ni * 3 * sizeof(double));
}

// Wait until the last copy through the staging buffer has finished, then make it hold `bytes`.
int pinned_acquire(nbx_ctx *c, Pinned &p, size_t bytes) {
  if (p.pending) {
    HIP_TRY(c, hipEventSynchronize(p.ev));
    p.pending = false;
  }
  if (!p.ev) HIP_TRY(c, hipEventCreateWithFlags(&p.ev, hipEventDisableTiming));
  if (p.bytes < bytes) {
    if (p.h) (void)hipHostFree(p.h);
    p.h = nullptr;
    p.bytes = 0;
    const size_t nb = (bytes + 65535) / 65536 * 65536;
    void *h = nullptr;
    HIP_TRY(c, hipHostMalloc(&h, nb, hipHostMallocDefault));
    p.h = h;
    p.bytes = nb;
  }
  return NBX_OK;
}

// The copy just enqueued on `s` reads (or writes) the staging buffer.
int pinned_release(nbx_ctx *c, Pinned &p, hipStream_t s) {
  HIP_TRY(c, hipEventRecord(p.ev, s));
  p.pending = true;
  return NBX_OK;
}

void pinned_free(Pinned &p) {
  if (p.ev) (void)hipEventDestroy(p.ev);
  if (p.h) (void)hipHostFree(p.h);
  p = Pinned{};
}

size_t align16(size_t bytes) { return (bytes + 15) / 16 * 16; }

// Point the host-path result arrays at consecutive pieces of d_out for ni sinks.
void out_layout(nbx_ctx *c, int ni) {
  const size_t n = (size_t)ni;
  double *p = c->d_out + kErrDoubles;
  c->d_acc = p;
  p += 3 * n;
  c->d_jrk = nullptr;
  c->d_snp = nullptr;
  c->d_crk = nullptr;
  if (c->cfg.order != 2) {
    c->d_jrk = p;
    p += 3 * n;
  }
  if (c->cfg.order >= 6) {
    c->d_snp = p;
    p += 3 * n;
  }
  if (c->cfg.order == 8) {
    c->d_crk = p;
    p += 3 * n;
  }
  c->d_pot = p;
  p += n;
  c->d_nnid = reinterpret_cast<int64_t *>(p);
  p += n;
  c->d_nnr2 = p;
  p += n;
  c->out_doubles = (size_t)(p - c->d_out);
}

// NBX_DS exists for the gravity kernels of orders 4 and 6.
bool valid_prec(int p, int order) {
  return p == NBX_FP64 || p == NBX_MIXED || (p == NBX_DS && (order == 4 || order == 6));
}

int check_ctx(nbx_ctx *c) {
  if (!c) return NBX_ERR_ARG;
  c->err.clear();
  return set_device(c);
}

int ni_class(int ni) {  // smallest k with 2^k >= ni
  int k = 0;
  while ((1 << k) < ni && k < 30) ++k;
  return k;
}

// Launch shape for ni sinks: the shape under test while tuning, else the tuned table entry of the
// N_i class (when the source tile count still matches), else the static rule.  NBX_SHAPE in the
// environment goes to the static rule, which honours it.
LaunchShape ctx_shape(const nbx_ctx *c, int ni, int nj_pad) {
  const int ntiles = nj_pad / kTile > 0 ? nj_pad / kTile : 1;
  const nbx_ctx::TunedShape *t = nullptr;
  nbx_ctx::TunedShape forced;
  if (c->force_shape) {
    forced.lanes_log2 = c->force_shape->lanes_log2;
    forced.sinks_per_lane = c->force_shape->sinks_per_lane;
    forced.splits = c->force_shape->splits;
    t = &forced;
  } else if (!getenv("NBX_SHAPE") && c->tune_ntiles[c->precision] == ntiles &&
             c->tuned[c->precision][ni_class(ni)].lanes_log2 >= 0) {
    t = &c->tuned[c->precision][ni_class(ni)];
  }
  if (!t) return choose_shape(ni, nj_pad, c->precision, c->cfg.order);
  LaunchShape ls;
  ls.lanes_log2 = t->lanes_log2;
  ls.sinks_per_lane = t->sinks_per_lane;
  const int Q = (kThreads >> ls.lanes_log2) * ls.sinks_per_lane;
  ls.blocks = (ni + Q - 1) / Q;
  int S = t->splits < ntiles ? t->splits : ntiles;
  const int64_t scap = ((int64_t)1 << 21) / (ni > 0 ? ni : 1);
  if (S > scap) S = (int)scap;
  ls.splits = S < 1 ? 1 : S;
  return ls;
}

// Shared by the host and device force paths.
// With bs given, a launch with source splits lets the combine kernel run the block-step corrector
// (at time bs_t1) instead of writing the outputs; *fused tells the caller whether that happened.
int enqueue_force(nbx_ctx *c, hipStream_t stream, int ni, const int32_t *d_iaddr, const int32_t *ext_self,
                  const int64_t *ext_id, const double *ext_x, const double *ext_v, const double *ext_a,
                  double eps2, const double *d_h2, double *acc, double *jrk, double *snp, double *crk, double *pot,
                  int64_t *nn_id, double *nn_r2, int32_t *nbr_cnt, int64_t *nbr_ids,
                  const BlockStepParams *bs = nullptr, double bs_t1 = 0.0, bool *fused = nullptr,
                  const double *ext_j = nullptr, void *fixed_scratch = nullptr) {
  if (fused) *fused = false;
  if (!c->predicted) return fail(c, NBX_ERR_STATE, "nbx_force before nbx_predict");
  if (!(eps2 >= 0.0)) return fail(c, NBX_ERR_ARG, "eps2 must be >= 0 (got %g)", eps2);
  if (ni == 0) return NBX_OK;
  // every force path, explicit sinks included: sinks with no sources are a caller's slip
  if (c->nj < 1) return fail(c, NBX_ERR_STATE, "no sources in use (nbx_set_nj)");
  const int nj_pad = (c->nj + kTile - 1) / kTile * kTile;
  LaunchShape ls = ctx_shape(c, ni, nj_pad);
  double *part = nullptr;
  uint64_t *part_key = nullptr;
  int32_t *part_idx = nullptr;
  double *part_xi = nullptr;
  if (fixed_scratch) {
    // the partials go to the fixed area: fewer source splits when the shape needs more room
    const size_t K = (size_t)values_per_sink(c->cfg.order);
    const size_t per_split = align16((size_t)ni * K * 8) + align16((size_t)ni * 8) + align16((size_t)ni * 4);
    const size_t xi_bytes = align16((size_t)ni * 3 * 8);
    const size_t smax = kNoallocScratchBytes > xi_bytes ? (kNoallocScratchBytes - xi_bytes) / per_split : 0;
    if ((size_t)ls.splits > smax) ls.splits = smax >= 1 ? (int)smax : 1;
    if (ls.splits > 1) {
      char *p = static_cast<char *>(fixed_scratch);
      part = reinterpret_cast<double *>(p);
      p += align16((size_t)ls.splits * (size_t)ni * K * 8);
      part_key = reinterpret_cast<uint64_t *>(p);
      p += align16((size_t)ls.splits * (size_t)ni * 8);
      part_idx = reinterpret_cast<int32_t *>(p);
      p += align16((size_t)ls.splits * (size_t)ni * 4);
      part_xi = reinterpret_cast<double *>(p);
    }
  } else {
    if (int rc = ensure_scratch(c, ni, ls)) return rc;
    part = static_cast<double *>(c->part.p);
    part_key = static_cast<uint64_t *>(c->part_key.p);
    part_idx = static_cast<int32_t *>(c->part_idx.p);
    part_xi = static_cast<double *>(c->part_xi.p);
  }
  ForceParams fp{};
  fp.src = c->src;
  fp.nj = c->nj;
  fp.nj_pad = nj_pad;
  fp.t = c->t_pred;
  fp.eps2 = eps2;
  fp.ni = ni;
  fp.i_addr = d_iaddr;
  fp.ext_self = ext_self;
  fp.ext_id = ext_id;
  fp.ext_x = ext_x;
  fp.ext_v = ext_v;
  fp.ext_a = ext_a;
  fp.ext_j = ext_j;
  fp.h2 = d_h2;
  fp.nbr_max = c->cfg.nbr_max;
  fp.lanes_log2 = ls.lanes_log2;
  fp.splits = ls.splits;
  fp.acc = acc;
  fp.jrk = jrk;
  fp.snp = snp;
  fp.crk = crk;
  fp.pot = pot;
  fp.nn_id = nn_id;
  fp.nn_r2 = nn_r2;
  fp.nn = nn_id != nullptr && nn_r2 != nullptr;  // no outputs: the kernels without the search
  fp.nbr_count = nbr_cnt;
  fp.nbr_ids = nbr_ids;
  fp.part = part;
  fp.part_key = part_key;
  fp.part_idx = part_idx;
  fp.part_xi = fp.nn && ls.splits > 1 ? part_xi : nullptr;
  fp.part_sm = ls.splits >= kSinkMajorMinS && ni <= kSinkMajorMaxNi ? 1 : 0;
  fp.err = c->d_err;
  if (bs && ls.splits > 1 && !d_h2) {
    fp.bs_fuse = 1;
    fp.bs_t1 = bs_t1;
    fp.bs = *bs;
  }
  hipError_t e = launch_force(c->cfg.order, c->precision, fp, ls, stream);
  if (e != hipSuccess) return hip_fail(c, e, "force kernel launch");
  if (fused) *fused = fp.bs_fuse != 0;
  return NBX_OK;
}

// Workgroups of the persistent batch launch: as many as are resident at once for the context's
// precision (occupancy times CUs, from the runtime), else 8 per CU.
int batch_groups(nbx_ctx *c) {
  const int g = batch_resident_groups(c->precision, c->cfg.device);
  return g > 0 ? std::min(g, kBatchMaxGroups) : kBatchMaxGroups;
}

// Size class of a batched system of n particles: smallest c with n <= 2^c.
int batch_class(int n) {
  int c = 0;
  while ((1 << c) < n) ++c;
  return c;
}

int batch_default_lg(int c) {  // L = 64 / 2^c, at least 1
  return c >= 6 ? 0 : 6 - c;
}

// Build and upload the schedule of the selected size classes (mask): items (system, lanes_log2,
// first sink, end sink), one wave each.  A system's sinks go in rounds of 64 / L; its rounds are
// split into items of about the mean cost per wave of the whole batch (cost = rounds x the
// sources each lane visits per round), so that the largest systems do not set the launch time.
// Items are ordered by cost, the costliest first (ties by system index), and the waves take them
// round-robin.  Each sink is computed by exactly one item, with the same arithmetic as unsplit.
int batch_upload(nbx_ctx *c, unsigned class_mask, const int *lg_override, hipStream_t stream) {
  const int n_sys = (int)c->batch_sizes.size();
  struct Sys {
    int k, lg, n, per_round, rounds;
    int64_t round_cost;
  };
  std::vector<Sys> sys;
  int64_t total = 0;
  for (int k = 0; k < n_sys; ++k) {
    const int n = c->batch_sizes[k];
    const int cl = batch_class(n);
    if (!(class_mask & (1u << cl))) continue;
    int lg = lg_override ? lg_override[cl] : c->batch_lg[cl];
    if (lg < 0) lg = batch_default_lg(cl);
    Sys q;
    q.k = k;
    q.lg = lg;
    q.n = n;
    q.per_round = 64 >> lg;
    q.rounds = (n + q.per_round - 1) / q.per_round;
    q.round_cost = (n + (1 << lg) - 1) >> lg;
    total += q.rounds * q.round_cost;
    sys.push_back(q);
  }
  const int64_t waves = (int64_t)batch_groups(c) * (kThreads / 64);
  const int64_t target = std::max<int64_t>(1, (total + waves - 1) / waves);
  struct Item {
    int4 v;
    int64_t cost;
  };
  std::vector<Item> items;
  for (const Sys &q : sys) {
    const int per_item = (int)std::max<int64_t>(1, target / q.round_cost);  // rounds per item
    for (int r0 = 0; r0 < q.rounds; r0 += per_item) {
      const int r1 = std::min(q.rounds, r0 + per_item);
      items.push_back({make_int4(q.k, q.lg, r0 * q.per_round, std::min(q.n, r1 * q.per_round)),
                       (r1 - r0) * q.round_cost});
    }
  }
  std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) { return a.cost > b.cost; });
  std::vector<int4> packed(items.size());
  for (size_t k = 0; k < items.size(); ++k) packed[k] = items[k].v;
  if (int rc = grow(c, c->batch_items, std::max<size_t>(1, packed.size()) * sizeof(int4))) return rc;
  if (!packed.empty())
    HIP_TRY(c, hipMemcpyAsync(c->batch_items.p, packed.data(), packed.size() * sizeof(int4), hipMemcpyHostToDevice,
                              stream));
  HIP_TRY(c, hipStreamSynchronize(stream));
  c->batch_n_items = (int)packed.size();
  return NBX_OK;
}

int batch_enqueue(nbx_ctx *c, hipStream_t stream, const double *d_m, const double *d_x, const double *d_v,
                  double eps2, double *d_acc, double *d_jerk, double *d_pot) {
  BatchParams bp{};
  bp.n_items = c->batch_n_items;
  bp.items = static_cast<const int4 *>(c->batch_items.p);
  bp.offset = c->d_batch_offset;
  bp.m = d_m;
  bp.x = d_x;
  bp.v = d_v;
  bp.eps2 = eps2;
  bp.acc = d_acc;
  bp.jrk = d_jerk;
  bp.pot = d_pot;
  const int waves_per_wg = kThreads / 64;
  int grid = (bp.n_items + waves_per_wg - 1) / waves_per_wg;
  if (grid > batch_groups(c)) grid = batch_groups(c);  // persistent: waves loop over items
  if (grid < 1) grid = 1;
  hipError_t e = launch_batch(c->precision, bp, grid, stream);
  if (e != hipSuccess) return hip_fail(c, e, "batch kernel launch");
  return NBX_OK;
}

// Status from error counters read back from the device (stream idle); clears them when set.
int errors_from(nbx_ctx *c, const int h[4]) {
  if (h[0] || h[1] || h[2] || h[3]) {
    HIP_TRY(c, launch_fill_i32(c->d_err, 4, 0, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  if (h[0]) return fail(c, NBX_ERR_ARG, "%d sink address(es) outside [0, nj) were skipped", h[0]);
  if (h[1]) return fail(c, NBX_ERR_ARG, "%d source address(es) out of range were skipped", h[1]);
  if (h[2]) return NBX_WARN_NBR_OVERFLOW;
  if (h[3]) {
    fail(c, NBX_OK, "%d block time-step(s) clamped at dt_min or with a criterion that is not a number", h[3]);
    return NBX_WARN_DT_MIN;
  }
  return NBX_OK;
}

// Read and clear the device error counters (stream must be idle).
int collect_errors(nbx_ctx *c) {
  int h[4] = {0, 0, 0, 0};
  HIP_TRY(c, hipMemcpy(h, c->d_err, sizeof h, hipMemcpyDeviceToHost));
  return errors_from(c, h);
}

// Shared by nbx_force_dev, nbx_force8_dev (d_crackle: order 8 only) and nbx_force_dev_noalloc
// (fixed_scratch: the static scratch instead of the context's split buffers).
int force_dev(nbx_ctx *c, void *stream, int ni, const int32_t *d_i_addr, double eps2, const double *d_h2,
              double *d_acc, double *d_jerk, double *d_snap, double *d_crackle, double *d_pot, int64_t *d_nn_id,
              double *d_nn_r2, int32_t *d_nbr_count, int64_t *d_nbr_ids, void *fixed_scratch = nullptr) {
  if (ni < 0) return fail(c, NBX_ERR_ARG, "ni < 0");
  if (ni > c->cfg.ni_max) return fail(c, NBX_ERR_CAPACITY, "ni=%d > ni_max=%d", ni, c->cfg.ni_max);
  if (ni == 0) return NBX_OK;
  if (!d_i_addr || !d_acc || (!d_jerk && c->cfg.order != 2) || !d_pot ||
      (c->cfg.want_nn && (!d_nn_id || !d_nn_r2)))
    return fail(c, NBX_ERR_ARG, "NULL device array");
  if (c->cfg.order >= 6 && !d_snap) return fail(c, NBX_ERR_ARG, "orders 6 and 8 need d_snap");
  if (c->cfg.order == 8 && !d_crackle) return fail(c, NBX_ERR_ARG, "order 8 needs d_crackle");
  if (d_h2 && (c->cfg.nbr_max == 0 || !d_nbr_count || !d_nbr_ids))
    return fail(c, NBX_ERR_ARG, "neighbour lists need nbr_max > 0 and count/id arrays");
  if (c->nj < 1) return fail(c, NBX_ERR_STATE, "no sources in use (nbx_set_nj)");
  const bool nn = c->cfg.want_nn != 0;
  return enqueue_force(c, static_cast<hipStream_t>(stream), ni, d_i_addr, nullptr, nullptr, nullptr, nullptr, nullptr,
                       eps2, d_h2, d_acc, d_jerk, d_snap, d_crackle, d_pot, nn ? d_nn_id : nullptr,
                       nn ? d_nn_r2 : nullptr, d_nbr_count, d_nbr_ids, nullptr, 0.0, nullptr, nullptr,
                       fixed_scratch);
}

}  // namespace

extern "C" {

int nbx_version(void) { return kVersion; }

int nbx_device_count(int *count) {
  if (!count) return NBX_ERR_ARG;
  *count = 0;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return NBX_ERR_NO_DEVICE;
  }
  *count = n;
  return NBX_OK;
}

int nbx_open(nbx_ctx **out, const nbx_config *cfg) {
  if (!out) return fail(nullptr, NBX_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(nullptr, NBX_ERR_ARG, "cfg is NULL");
  if (cfg->order != 2 && cfg->order != 4 && cfg->order != 6 && cfg->order != 8)
    return fail(nullptr, NBX_ERR_ARG, "order must be 2, 4, 6 or 8");
  if (!valid_prec(cfg->precision, cfg->order))
    return fail(nullptr, NBX_ERR_ARG, "precision must be NBX_FP64, NBX_MIXED or (orders 4 and 6) NBX_DS");
  if (cfg->nj_max < 1 || cfg->ni_max < 1 || cfg->nbr_max < 0)
    return fail(nullptr, NBX_ERR_ARG, "nj_max and ni_max must be >= 1, nbr_max >= 0");
  int ndev = 0;
  if (nbx_device_count(&ndev) != NBX_OK) return fail(nullptr, NBX_ERR_NO_DEVICE, "no HIP device available");
  if (cfg->device < 0 || cfg->device >= ndev)
    return fail(nullptr, NBX_ERR_NO_DEVICE, "device %d does not exist (%d visible)", cfg->device, ndev);

  nbx_ctx *c = new (std::nothrow) nbx_ctx;
  if (!c) return fail(nullptr, NBX_ERR_OOM, "host allocation failed");
  c->cfg = *cfg;
  c->precision = cfg->precision;
  auto bail = [&](int rc) {
    g_open_error = c->err;
    nbx_close(c);
    return rc;
  };
  if (int rc = set_device(c)) return bail(rc);
  if (int rc = scratch_setup(c)) return bail(rc);
  {
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(hip_fail(c, e, "hipStreamCreate"));
  }
  const size_t nj = (size_t)cfg->nj_max, ni = (size_t)cfg->ni_max;
  int rc = NBX_OK;
  rc = rc ? rc : alloc_n(c, &c->src.pos_mass, nj);
  rc = rc ? rc : alloc_n(c, &c->src.vel_time, nj);
  rc = rc ? rc : alloc_n(c, &c->src.acc_jrk, 6 * nj);
  if (cfg->order >= 6) rc = rc ? rc : alloc_n(c, &c->src.snp_crk, 6 * nj);
  rc = rc ? rc : alloc_n(c, &c->src.id, nj);
  rc = rc ? rc : alloc_n(c, &c->d_iaddr, ni);
  rc = rc ? rc : alloc_n(c, &c->d_out, kErrDoubles + 15 * ni);
  if (cfg->nbr_max > 0) {
    rc = rc ? rc : alloc_n(c, &c->d_h2, ni);
    rc = rc ? rc : alloc_n(c, &c->d_nbr_cnt, ni);
    rc = rc ? rc : alloc_n(c, &c->d_nbr_ids, ni * (size_t)cfg->nbr_max);
  }
  if (rc) return bail(rc);
  c->d_err = reinterpret_cast<int *>(c->d_out);
  out_layout(c, cfg->ni_max);
  hipError_t e = launch_pad(cfg->order, c->src, 0, cfg->nj_max, c->stream);
  if (e == hipSuccess) e = launch_fill_i32(c->d_err, 4, 0, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return bail(hip_fail(c, e, "context initialisation"));
  *out = c;
  return NBX_OK;
}

int nbx_close(nbx_ctx *c) {
  if (!c) return NBX_OK;
  (void)hipSetDevice(c->cfg.device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (void *p : c->owned) (void)hipFree(p);
  if (c->bs.h_sched) (void)hipHostFree(c->bs.h_sched);
  pinned_free(c->stage_j);
  pinned_free(c->stage_i);
  pinned_free(c->stage_out);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return NBX_OK;
}

const char *nbx_last_error(const nbx_ctx *c) { return c ? c->err.c_str() : g_open_error.c_str(); }

int nbx_set_precision(nbx_ctx *c, int precision) {
  if (!c) return NBX_ERR_ARG;
  c->err.clear();
  if (!valid_prec(precision, c->cfg.order))
    return fail(c, NBX_ERR_ARG, "precision must be NBX_FP64, NBX_MIXED or (orders 4 and 6) NBX_DS");
  c->precision = precision;
  return NBX_OK;
}

int nbx_set_nj(nbx_ctx *c, int nj) {
  if (!c) return NBX_ERR_ARG;
  c->err.clear();
  if (nj < 0 || nj > c->cfg.nj_max) return fail(c, NBX_ERR_CAPACITY, "nj=%d outside [0, %d]", nj, c->cfg.nj_max);
  c->nj = nj;
  return NBX_OK;
}

int nbx_set_j(nbx_ctx *c, int n, const int32_t *addr, const int64_t *id, const double *m, const double *t,
              const double *x, const double *v, const double *a, const double *jerk, const double *snap,
              const double *crackle) {
  if (int rc = check_ctx(c)) return rc;
  if (n < 0) return fail(c, NBX_ERR_ARG, "n < 0");
  if (n == 0) return NBX_OK;
  if (n > c->cfg.nj_max) return fail(c, NBX_ERR_CAPACITY, "n=%d > nj_max=%d", n, c->cfg.nj_max);
  const bool two = c->cfg.order == 2;
  if (!addr || !id || !m || !t || !x || (!two && (!v || !a || !jerk)))
    return fail(c, NBX_ERR_ARG, "NULL input array");
  const bool six = c->cfg.order >= 6;
  if (six && (!snap || !crackle)) return fail(c, NBX_ERR_ARG, "orders 6 and 8 need snap and crackle");
  int hi = -1;
  for (int k = 0; k < n; ++k) {
    if (addr[k] < 0 || addr[k] >= c->cfg.nj_max)
      return fail(c, NBX_ERR_ARG, "addr[%d]=%d outside [0, %d)", k, addr[k], c->cfg.nj_max);
    hi = std::max(hi, addr[k]);
  }
  // device staging layout (16-byte aligned pieces): addr | id | m | t | x v a [jerk [snap crackle]],
  // then the copy kernel scatters them.  Small updates are packed into pinned memory and move in
  // one copy, and nothing waits: later work on the context stream is ordered after the scatter.
  const size_t nv = six ? 6 : (two ? 3 : 4);
  const size_t N = (size_t)n;
  const double *h_vec[6] = {x, v, a, jerk, snap, crackle};
  size_t off_vec[6] = {0, 0, 0, 0, 0, 0};
  const size_t off_id = align16(N * 4), off_m = off_id + align16(N * 8), off_t = off_m + align16(N * 8);
  size_t bytes = off_t + align16(N * 8);
  for (size_t k = 0; k < nv; ++k) {
    if (!h_vec[k]) continue;  // optional for order 2 (v, a): the copy kernel takes NULL as zero
    off_vec[k] = bytes;
    bytes += align16(N * 24);
  }
  if (int rc = grow(c, c->up, bytes)) return rc;
  hipStream_t s = c->stream;
  char *base = static_cast<char *>(c->up.p);
  const bool staged = bytes <= kStageMax;
  if (staged) {
    if (int rc = pinned_acquire(c, c->stage_j, bytes)) return rc;
    char *h = static_cast<char *>(c->stage_j.h);
    std::memcpy(h, addr, N * 4);
    std::memcpy(h + off_id, id, N * 8);
    std::memcpy(h + off_m, m, N * 8);
    std::memcpy(h + off_t, t, N * 8);
    for (size_t k = 0; k < nv; ++k)
      if (h_vec[k]) std::memcpy(h + off_vec[k], h_vec[k], N * 24);
    HIP_TRY(c, hipMemcpyAsync(base, h, bytes, hipMemcpyHostToDevice, s));
    if (int rc = pinned_release(c, c->stage_j, s)) return rc;
  } else {
    HIP_TRY(c, hipMemcpyAsync(base, addr, N * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(base + off_id, id, N * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(base + off_m, m, N * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(base + off_t, t, N * 8, hipMemcpyHostToDevice, s));
    for (size_t k = 0; k < nv; ++k)
      if (h_vec[k]) HIP_TRY(c, hipMemcpyAsync(base + off_vec[k], h_vec[k], N * 24, hipMemcpyHostToDevice, s));
  }
  const double *d_vec[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  for (size_t k = 0; k < nv; ++k)
    if (h_vec[k]) d_vec[k] = reinterpret_cast<const double *>(base + off_vec[k]);
  HIP_TRY(c, launch_jupdate(c->cfg.order, c->src, c->cfg.nj_max, n, reinterpret_cast<const int32_t *>(base),
                            reinterpret_cast<const int64_t *>(base + off_id),
                            reinterpret_cast<const double *>(base + off_m),
                            reinterpret_cast<const double *>(base + off_t), d_vec[0], d_vec[1], d_vec[2], d_vec[3],
                            d_vec[4], d_vec[5], c->d_err, s));
  if (!staged) HIP_TRY(c, hipStreamSynchronize(s));  // the caller's arrays have been read
  c->nj = std::max(c->nj, hi + 1);
  c->bs.ready = false;  // the block time-step state lives in the same arrays
  return NBX_OK;
}

int nbx_predict(nbx_ctx *c, double t) {
  if (!c) return NBX_ERR_ARG;
  c->err.clear();
  c->t_pred = t;
  c->predicted = true;
  return NBX_OK;
}

int nbx_force(nbx_ctx *c, int ni, const int32_t *i_addr, double eps2, const double *h2) {
  if (int rc = check_ctx(c)) return rc;
  if (ni < 0) return fail(c, NBX_ERR_ARG, "ni < 0");
  if (ni > c->cfg.ni_max) return fail(c, NBX_ERR_CAPACITY, "ni=%d > ni_max=%d", ni, c->cfg.ni_max);
  if (ni > 0 && !i_addr) return fail(c, NBX_ERR_ARG, "i_addr is NULL");
  if (ni > 0 && c->nj < 1) return fail(c, NBX_ERR_STATE, "no sources in use (nbx_set_nj)");
  for (int k = 0; k < ni; ++k)
    if (i_addr[k] < 0 || i_addr[k] >= c->nj)
      return fail(c, NBX_ERR_ARG, "i_addr[%d]=%d outside [0, nj=%d)", k, i_addr[k], c->nj);
  if (h2 && c->cfg.nbr_max == 0) return fail(c, NBX_ERR_ARG, "neighbour lists need nbr_max > 0");
  const size_t n_i = (size_t)ni, off_h2_i = align16(n_i * 4);
  if (ni > 0 && off_h2_i + (h2 ? n_i * 8 : 0) > kStageMax) {  // large: straight from the caller's arrays
    HIP_TRY(c, hipMemcpyAsync(c->d_iaddr, i_addr, n_i * 4, hipMemcpyHostToDevice, c->stream));
    if (h2) HIP_TRY(c, hipMemcpyAsync(c->d_h2, h2, n_i * 8, hipMemcpyHostToDevice, c->stream));
  } else if (ni > 0) {  // small: addresses (and radii) through the pinned staging buffer
    const size_t n = n_i, off_h2 = off_h2_i;
    if (int rc = pinned_acquire(c, c->stage_i, off_h2 + (h2 ? n * 8 : 0))) return rc;
    char *h = static_cast<char *>(c->stage_i.h);
    std::memcpy(h, i_addr, n * 4);
    HIP_TRY(c, hipMemcpyAsync(c->d_iaddr, h, n * 4, hipMemcpyHostToDevice, c->stream));
    if (h2) {
      std::memcpy(h + off_h2, h2, n * 8);
      HIP_TRY(c, hipMemcpyAsync(c->d_h2, h + off_h2, n * 8, hipMemcpyHostToDevice, c->stream));
    }
    if (int rc = pinned_release(c, c->stage_i, c->stream)) return rc;
  }
  out_layout(c, ni);
  const bool nn = c->cfg.want_nn != 0;
  int rc = enqueue_force(c, c->stream, ni, c->d_iaddr, nullptr, nullptr, nullptr, nullptr, nullptr, eps2,
                         h2 ? c->d_h2 : nullptr, c->d_acc, c->d_jrk, c->d_snp, c->d_crk, c->d_pot,
                         nn ? c->d_nnid : nullptr, nn ? c->d_nnr2 : nullptr, c->d_nbr_cnt, c->d_nbr_ids);
  if (rc < 0) return rc;
  c->last_ni = ni;
  c->last_nbr = h2 != nullptr;
  c->last_nn = nn;
  return rc;
}

// Explicit sinks at every order: a (orders 6 and 8) and jerk (order 8) as the order needs them.
static int force_ext_impl(nbx_ctx *c, int ni, const int64_t *id, const double *x, const double *v, const double *a,
                          const double *jerk, double eps2, const double *h2) {
  const int order = c->cfg.order;
  if (ni < 0) return fail(c, NBX_ERR_ARG, "ni < 0");
  if (ni > c->cfg.ni_max) return fail(c, NBX_ERR_CAPACITY, "ni=%d > ni_max=%d", ni, c->cfg.ni_max);
  if (ni > 0 && (!id || !x || (!v && order != 2))) return fail(c, NBX_ERR_ARG, "NULL sink array");
  if (ni > 0 && order >= 6 && !a) return fail(c, NBX_ERR_ARG, "orders 6 and 8 need the sink accelerations");
  if (ni > 0 && order == 8 && !jerk) return fail(c, NBX_ERR_ARG, "order 8 needs the sink jerks");
  if (h2 && c->cfg.nbr_max == 0) return fail(c, NBX_ERR_ARG, "neighbour lists need nbr_max > 0");
  if (!c->d_ext_id) {  // explicit-sink buffers, allocated on first use
    const size_t n = (size_t)c->cfg.ni_max;
    int rc = alloc_n(c, &c->d_ext_id, n);
    rc = rc ? rc : alloc_n(c, &c->d_ext_x, 3 * n);
    if (order != 2) rc = rc ? rc : alloc_n(c, &c->d_ext_v, 3 * n);
    if (order >= 6) rc = rc ? rc : alloc_n(c, &c->d_ext_a, 3 * n);
    if (order == 8) rc = rc ? rc : alloc_n(c, &c->d_ext_j, 3 * n);
    rc = rc ? rc : alloc_n(c, &c->d_ext_self, n);
    if (rc) return rc;
  }
  const size_t n = (size_t)ni;
  hipStream_t s = c->stream;
  const bool hv = order != 2, ha = order >= 6, hj = order == 8;
  const size_t off_x = align16(n * 8), off_v = off_x + align16(n * 24), off_a = off_v + (hv ? align16(n * 24) : 0);
  const size_t off_j = off_a + (ha ? align16(n * 24) : 0);
  const size_t off_h2 = off_j + (hj ? align16(n * 24) : 0), bytes = off_h2 + (h2 ? n * 8 : 0);
  if (ni > 0 && bytes > kStageMax) {  // large: straight from the caller's arrays
    HIP_TRY(c, hipMemcpyAsync(c->d_ext_id, id, n * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(c->d_ext_x, x, n * 24, hipMemcpyHostToDevice, s));
    if (hv) HIP_TRY(c, hipMemcpyAsync(c->d_ext_v, v, n * 24, hipMemcpyHostToDevice, s));
    if (ha) HIP_TRY(c, hipMemcpyAsync(c->d_ext_a, a, n * 24, hipMemcpyHostToDevice, s));
    if (hj) HIP_TRY(c, hipMemcpyAsync(c->d_ext_j, jerk, n * 24, hipMemcpyHostToDevice, s));
    if (h2) HIP_TRY(c, hipMemcpyAsync(c->d_h2, h2, n * 8, hipMemcpyHostToDevice, s));
    if (c->predicted) HIP_TRY(c, launch_selfmap(c->src, c->nj, ni, c->d_ext_id, c->d_ext_self, s));
  } else if (ni > 0) {  // small: sink states through the pinned staging buffer: id | x | v | a | jerk | h2
    if (int rc = pinned_acquire(c, c->stage_i, bytes)) return rc;
    char *h = static_cast<char *>(c->stage_i.h);
    std::memcpy(h, id, n * 8);
    std::memcpy(h + off_x, x, n * 24);
    HIP_TRY(c, hipMemcpyAsync(c->d_ext_id, h, n * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(c->d_ext_x, h + off_x, n * 24, hipMemcpyHostToDevice, s));
    if (hv) {
      std::memcpy(h + off_v, v, n * 24);
      HIP_TRY(c, hipMemcpyAsync(c->d_ext_v, h + off_v, n * 24, hipMemcpyHostToDevice, s));
    }
    if (ha) {
      std::memcpy(h + off_a, a, n * 24);
      HIP_TRY(c, hipMemcpyAsync(c->d_ext_a, h + off_a, n * 24, hipMemcpyHostToDevice, s));
    }
    if (hj) {
      std::memcpy(h + off_j, jerk, n * 24);
      HIP_TRY(c, hipMemcpyAsync(c->d_ext_j, h + off_j, n * 24, hipMemcpyHostToDevice, s));
    }
    if (h2) {
      std::memcpy(h + off_h2, h2, n * 8);
      HIP_TRY(c, hipMemcpyAsync(c->d_h2, h + off_h2, n * 8, hipMemcpyHostToDevice, s));
    }
    if (int rc = pinned_release(c, c->stage_i, s)) return rc;
    if (c->predicted) HIP_TRY(c, launch_selfmap(c->src, c->nj, ni, c->d_ext_id, c->d_ext_self, s));
  }
  out_layout(c, ni);
  const bool nn = c->cfg.want_nn != 0;
  int rc = enqueue_force(c, s, ni, nullptr, c->d_ext_self, c->d_ext_id, c->d_ext_x, c->d_ext_v,
                         ha ? c->d_ext_a : nullptr, eps2, h2 ? c->d_h2 : nullptr, c->d_acc, c->d_jrk, c->d_snp,
                         c->d_crk, c->d_pot, nn ? c->d_nnid : nullptr, nn ? c->d_nnr2 : nullptr, c->d_nbr_cnt,
                         c->d_nbr_ids, nullptr, 0.0, nullptr, hj ? c->d_ext_j : nullptr);
  if (rc < 0) return rc;
  c->last_ni = ni;
  c->last_nbr = h2 != nullptr;
  c->last_nn = nn;
  return rc;
}

int nbx_force_ext(nbx_ctx *c, int ni, const int64_t *id, const double *x, const double *v, const double *a,
                  double eps2, const double *h2) {
  if (int rc = check_ctx(c)) return rc;
  if (c->cfg.order == 8) return fail(c, NBX_ERR_ARG, "order 8 explicit sinks go through nbx_force_ext8");
  return force_ext_impl(c, ni, id, x, v, a, nullptr, eps2, h2);
}

int nbx_force_ext8(nbx_ctx *c, int ni, const int64_t *id, const double *x, const double *v, const double *a,
                   const double *jerk, double eps2, const double *h2) {
  if (int rc = check_ctx(c)) return rc;
  if (c->cfg.order != 8) return fail(c, NBX_ERR_ARG, "nbx_force_ext8 needs an order-8 context");
  return force_ext_impl(c, ni, id, x, v, a, jerk, eps2, h2);
}

int nbx_get_force(nbx_ctx *c, double *acc, double *jerk, double *snap, double *pot, int64_t *nn_id,
                  double *nn_r2) {
  if (int rc = check_ctx(c)) return rc;
  if (c->last_ni < 0) return fail(c, NBX_ERR_STATE, "nbx_get_force before nbx_force");
  const size_t bytes = c->out_doubles * sizeof(double);
  if (bytes > kStageMax) {  // large: straight into the caller's arrays
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int rc = collect_errors(c);
    if (rc < 0) return rc;
    const size_t n = (size_t)c->last_ni;
    if (acc) HIP_TRY(c, hipMemcpy(acc, c->d_acc, n * 24, hipMemcpyDeviceToHost));
    if (jerk && c->d_jrk) HIP_TRY(c, hipMemcpy(jerk, c->d_jrk, n * 24, hipMemcpyDeviceToHost));
    if (snap && c->d_snp) HIP_TRY(c, hipMemcpy(snap, c->d_snp, n * 24, hipMemcpyDeviceToHost));
    if (pot) HIP_TRY(c, hipMemcpy(pot, c->d_pot, n * 8, hipMemcpyDeviceToHost));
    if (nn_id && c->last_nn) HIP_TRY(c, hipMemcpy(nn_id, c->d_nnid, n * 8, hipMemcpyDeviceToHost));
    if (nn_r2 && c->last_nn) HIP_TRY(c, hipMemcpy(nn_r2, c->d_nnr2, n * 8, hipMemcpyDeviceToHost));
    return rc;
  }
  // small: one copy of the error counters and the results (laid out for last_ni by the force call)
  if (int rc = pinned_acquire(c, c->stage_out, bytes)) return rc;
  HIP_TRY(c, hipMemcpyAsync(c->stage_out.h, c->d_out, bytes, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const char *h = static_cast<const char *>(c->stage_out.h);
  int err[4];
  std::memcpy(err, h, sizeof err);
  const int rc = errors_from(c, err);
  if (rc < 0) return rc;
  const size_t n = (size_t)c->last_ni;
  if (n == 0) return rc;
  auto from = [&](const void *d) { return h + (static_cast<const char *>(d) - reinterpret_cast<const char *>(c->d_out)); };
  if (acc) std::memcpy(acc, from(c->d_acc), n * 24);
  if (jerk && c->d_jrk) std::memcpy(jerk, from(c->d_jrk), n * 24);
  if (snap && c->d_snp) std::memcpy(snap, from(c->d_snp), n * 24);
  if (pot) std::memcpy(pot, from(c->d_pot), n * 8);
  if (nn_id && c->last_nn) std::memcpy(nn_id, from(c->d_nnid), n * 8);
  if (nn_r2 && c->last_nn) std::memcpy(nn_r2, from(c->d_nnr2), n * 8);
  return rc;
}

int nbx_get_crackle(nbx_ctx *c, double *crackle) {
  if (int rc = check_ctx(c)) return rc;
  if (c->cfg.order != 8) return fail(c, NBX_ERR_ARG, "crackle is computed at order 8 only");
  if (c->last_ni < 0) return fail(c, NBX_ERR_STATE, "nbx_get_crackle before nbx_force");
  if (!crackle) return fail(c, NBX_ERR_ARG, "crackle is NULL");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int rc = collect_errors(c);
  if (rc < 0) return rc;
  if (c->last_ni > 0) HIP_TRY(c, hipMemcpy(crackle, c->d_crk, (size_t)c->last_ni * 24, hipMemcpyDeviceToHost));
  return rc;
}

int nbx_get_nbr(nbx_ctx *c, int32_t *count, int64_t *ids) {
  if (int rc = check_ctx(c)) return rc;
  if (c->last_ni < 0 || !c->last_nbr) return fail(c, NBX_ERR_STATE, "the last force call computed no neighbour lists");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t n = (size_t)c->last_ni;
  if (n == 0) return NBX_OK;
  std::vector<int32_t> cnt(n);
  HIP_TRY(c, hipMemcpy(cnt.data(), c->d_nbr_cnt, n * 4, hipMemcpyDeviceToHost));
  if (count) std::memcpy(count, cnt.data(), n * 4);
  if (ids) HIP_TRY(c, hipMemcpy(ids, c->d_nbr_ids, n * (size_t)c->cfg.nbr_max * 8, hipMemcpyDeviceToHost));
  const int rc = collect_errors(c);
  if (rc < 0) return rc;
  for (size_t k = 0; k < n; ++k)
    if (cnt[k] > c->cfg.nbr_max) return NBX_WARN_NBR_OVERFLOW;
  return rc;
}

int nbx_get_predicted(nbx_ctx *c, int n, const int32_t *addr, double *xp, double *vp, double *ap) {
  if (int rc = check_ctx(c)) return rc;
  if (n < 0) return fail(c, NBX_ERR_ARG, "n < 0");
  if (n == 0) return NBX_OK;
  if (!addr || !xp || !vp) return fail(c, NBX_ERR_ARG, "NULL argument");
  if (!c->predicted) return fail(c, NBX_ERR_STATE, "nbx_get_predicted before nbx_predict");
  for (int k = 0; k < n; ++k)
    if (addr[k] < 0 || addr[k] >= c->nj)
      return fail(c, NBX_ERR_ARG, "addr[%d]=%d outside [0, nj=%d)", k, addr[k], c->nj);
  const size_t bytes = (size_t)n * (16 + 72);
  if (int rc = grow(c, c->up, bytes)) return rc;
  char *base = static_cast<char *>(c->up.p);
  int32_t *d_addr = reinterpret_cast<int32_t *>(base);
  double *d_x = reinterpret_cast<double *>(base + ((size_t)n * 4 + 15) / 16 * 16);
  double *d_v = d_x + 3 * (size_t)n;
  double *d_a = d_v + 3 * (size_t)n;
  HIP_TRY(c, hipMemcpyAsync(d_addr, addr, (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_predict_out(c->cfg.order, c->src, c->nj, c->t_pred, n, d_addr, d_x, d_v, d_a, c->d_err,
                                c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(xp, d_x, (size_t)n * 24, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(vp, d_v, (size_t)n * 24, hipMemcpyDeviceToHost));
  if (ap) HIP_TRY(c, hipMemcpy(ap, d_a, (size_t)n * 24, hipMemcpyDeviceToHost));
  return collect_errors(c);
}

int nbx_get_j(nbx_ctx *c, int n, const int32_t *addr, int64_t *id, double *m, double *t, double *x, double *v,
              double *a, double *jerk, double *snap, double *crackle) {
  if (int rc = check_ctx(c)) return rc;
  if (n < 0) return fail(c, NBX_ERR_ARG, "n < 0");
  if (n == 0) return NBX_OK;
  if (!addr) return fail(c, NBX_ERR_ARG, "addr is NULL");
  for (int k = 0; k < n; ++k)
    if (addr[k] < 0 || addr[k] >= c->cfg.nj_max)
      return fail(c, NBX_ERR_ARG, "addr[%d]=%d outside [0, %d)", k, addr[k], c->cfg.nj_max);
  const bool six = c->cfg.order >= 6;
  // staging: addr | id | m | t | x v a jerk snap crackle
  const size_t bytes = (size_t)n * (16 + 8 + 8 + 8 + 6 * 24);
  if (int rc = grow(c, c->up, bytes)) return rc;
  char *base = static_cast<char *>(c->up.p);
  int32_t *d_addr = reinterpret_cast<int32_t *>(base);
  size_t off = ((size_t)n * 4 + 15) / 16 * 16;
  int64_t *d_id = reinterpret_cast<int64_t *>(base + off);
  off += (size_t)n * 8;
  double *d_m = reinterpret_cast<double *>(base + off);
  off += (size_t)n * 8;
  double *d_t = reinterpret_cast<double *>(base + off);
  off += (size_t)n * 8;
  double *d_vec[6];
  for (int k = 0; k < 6; ++k) {
    d_vec[k] = reinterpret_cast<double *>(base + off);
    off += (size_t)n * 24;
  }
  HIP_TRY(c, hipMemcpyAsync(d_addr, addr, (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_gather_j(c->cfg.order, c->src, n, d_addr, d_id, d_m, d_t, d_vec[0], d_vec[1], d_vec[2],
                             d_vec[3], six ? d_vec[4] : nullptr, six ? d_vec[5] : nullptr, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  double *h_vec[6] = {x, v, a, jerk, snap, crackle};
  if (id) HIP_TRY(c, hipMemcpy(id, d_id, (size_t)n * 8, hipMemcpyDeviceToHost));
  if (m) HIP_TRY(c, hipMemcpy(m, d_m, (size_t)n * 8, hipMemcpyDeviceToHost));
  if (t) HIP_TRY(c, hipMemcpy(t, d_t, (size_t)n * 8, hipMemcpyDeviceToHost));
  for (int k = 0; k < (six ? 6 : 4); ++k)
    if (h_vec[k]) HIP_TRY(c, hipMemcpy(h_vec[k], d_vec[k], (size_t)n * 24, hipMemcpyDeviceToHost));
  return NBX_OK;
}

int nbx_set_j_dev(nbx_ctx *c, void *stream, int n, const int32_t *d_addr, const int64_t *d_id, const double *d_m,
                  const double *d_t, const double *d_x, const double *d_v, const double *d_a,
                  const double *d_jerk, const double *d_snap, const double *d_crackle) {
  if (int rc = check_ctx(c)) return rc;
  if (n < 0) return fail(c, NBX_ERR_ARG, "n < 0");
  if (n == 0) return NBX_OK;
  if (n > c->cfg.nj_max) return fail(c, NBX_ERR_CAPACITY, "n=%d > nj_max=%d", n, c->cfg.nj_max);
  if (!d_addr || !d_id || !d_m || !d_t || !d_x || (c->cfg.order != 2 && (!d_v || !d_a || !d_jerk)))
    return fail(c, NBX_ERR_ARG, "NULL input array");
  if (c->cfg.order >= 6 && (!d_snap || !d_crackle))
    return fail(c, NBX_ERR_ARG, "orders 6 and 8 need snap and crackle");
  HIP_TRY(c, launch_jupdate(c->cfg.order, c->src, c->cfg.nj_max, n, d_addr, d_id, d_m, d_t, d_x, d_v, d_a, d_jerk,
                            d_snap, d_crackle, c->d_err, static_cast<hipStream_t>(stream)));
  c->bs.ready = false;
  return NBX_OK;
}

int nbx_force_dev(nbx_ctx *c, void *stream, int ni, const int32_t *d_i_addr, double eps2, const double *d_h2,
                  double *d_acc, double *d_jerk, double *d_snap, double *d_pot, int64_t *d_nn_id, double *d_nn_r2,
                  int32_t *d_nbr_count, int64_t *d_nbr_ids) {
  if (int rc = check_ctx(c)) return rc;
  if (c->cfg.order == 8) return fail(c, NBX_ERR_ARG, "order 8 forces go through nbx_force8_dev");
  return force_dev(c, stream, ni, d_i_addr, eps2, d_h2, d_acc, d_jerk, d_snap, nullptr, d_pot, d_nn_id, d_nn_r2,
                   d_nbr_count, d_nbr_ids);
}

int nbx_force_dev_noalloc(nbx_ctx *c, void *stream, int ni, const int32_t *d_i_addr, double eps2,
                          const double *d_h2, double *d_acc, double *d_jerk, double *d_snap, double *d_pot,
                          int64_t *d_nn_id, double *d_nn_r2, int32_t *d_nbr_count, int64_t *d_nbr_ids) {
  if (int rc = check_ctx(c)) return rc;
  if (c->cfg.order == 8) return fail(c, NBX_ERR_ARG, "order 8 forces go through nbx_force8_dev");
  if (!c->noalloc_scratch) return fail(c, NBX_ERR_STATE, "static scratch not set up for this device");
  return force_dev(c, stream, ni, d_i_addr, eps2, d_h2, d_acc, d_jerk, d_snap, nullptr, d_pot, d_nn_id, d_nn_r2,
                   d_nbr_count, d_nbr_ids, c->noalloc_scratch);
}

int nbx_force8_dev(nbx_ctx *c, void *stream, int ni, const int32_t *d_i_addr, double eps2, const double *d_h2,
                   double *d_acc, double *d_jerk, double *d_snap, double *d_crackle, double *d_pot,
                   int64_t *d_nn_id, double *d_nn_r2, int32_t *d_nbr_count, int64_t *d_nbr_ids) {
  if (int rc = check_ctx(c)) return rc;
  if (c->cfg.order != 8) return fail(c, NBX_ERR_ARG, "nbx_force8_dev needs an order-8 context");
  return force_dev(c, stream, ni, d_i_addr, eps2, d_h2, d_acc, d_jerk, d_snap, d_crackle, d_pot, d_nn_id, d_nn_r2,
                   d_nbr_count, d_nbr_ids);
}

int nbx_force_vjp_dev(nbx_ctx *c, void *stream, int n, const double *d_m, const double *d_x, const double *d_v,
                      double eps2, const double *d_g_acc, const double *d_g_jerk, const double *d_g_pot,
                      double *d_grad_x, double *d_grad_v, double *d_grad_m) {
  if (int rc = check_ctx(c)) return rc;
  if (c->precision == NBX_DS) return fail(c, NBX_ERR_ARG, "the adjoint runs in NBX_FP64 or NBX_MIXED");
  if (n < 0) return fail(c, NBX_ERR_ARG, "n < 0");
  if (n == 0) return NBX_OK;
  if (!d_m || !d_x || !d_v || !d_g_acc || !d_g_jerk || !d_g_pot || !d_grad_x || !d_grad_v || !d_grad_m)
    return fail(c, NBX_ERR_ARG, "NULL device array");
  if (!(eps2 >= 0.0)) return fail(c, NBX_ERR_ARG, "eps2 must be >= 0");
  VjpParams vp{};
  vp.n = n;
  vp.n_pad = (n + kTile - 1) / kTile * kTile;
  const int blocks = (n + kThreads - 1) / kThreads;
  const int ntiles = vp.n_pad / kTile;
  int S = (2048 + blocks - 1) / blocks;
  const int scap = (int)std::max<int64_t>(1, ((int64_t)1 << 21) / n);
  S = std::min(std::min(S, ntiles), scap);
  vp.splits = std::max(S, 1);
  if (vp.splits > 1)
    if (int rc = grow(c, c->part, (size_t)vp.splits * 7 * (size_t)n * sizeof(double))) return rc;
  vp.eps2 = eps2;
  vp.m = d_m;
  vp.x = d_x;
  vp.v = d_v;
  vp.g_acc = d_g_acc;
  vp.g_jerk = d_g_jerk;
  vp.g_pot = d_g_pot;
  vp.grad_x = d_grad_x;
  vp.grad_v = d_grad_v;
  vp.grad_m = d_grad_m;
  vp.part = static_cast<double *>(c->part.p);
  hipError_t e = launch_vjp(c->precision, vp, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "adjoint kernel launch");
  return NBX_OK;
}

int nbx_batch_setup(nbx_ctx *c, int n_sys, const int32_t *offsets) {
  if (int rc = check_ctx(c)) return rc;
  if (n_sys < 1 || !offsets) return fail(c, NBX_ERR_ARG, "need n_sys >= 1 and offsets");
  if (offsets[0] != 0) return fail(c, NBX_ERR_ARG, "offsets[0] must be 0");
  std::vector<int32_t> sizes(n_sys);
  for (int k = 0; k < n_sys; ++k) {
    sizes[k] = offsets[k + 1] - offsets[k];
    if (sizes[k] < 1 || sizes[k] > NBX_BATCH_NMAX)
      return fail(c, NBX_ERR_ARG, "system %d has %d particles (allowed 1..%d)", k, sizes[k], NBX_BATCH_NMAX);
  }
  if (c->d_batch_offset) {
    auto it = std::find(c->owned.begin(), c->owned.end(), (void *)c->d_batch_offset);
    if (it != c->owned.end()) c->owned.erase(it);
    HIP_TRY(c, hipFree(c->d_batch_offset));
    c->d_batch_offset = nullptr;
  }
  if (int rc = alloc_n(c, &c->d_batch_offset, (size_t)n_sys + 1)) return rc;
  HIP_TRY(c, hipMemcpyAsync(c->d_batch_offset, offsets, ((size_t)n_sys + 1) * 4, hipMemcpyHostToDevice, c->stream));
  c->batch_sizes = sizes;
  for (int k = 0; k < 8; ++k) c->batch_lg[k] = -1;
  return batch_upload(c, 0xffu, nullptr, c->stream);
}

int nbx_batch_force_dev(nbx_ctx *c, void *stream, const double *d_m, const double *d_x, const double *d_v,
                        double eps2, double *d_acc, double *d_jerk, double *d_pot) {
  if (int rc = check_ctx(c)) return rc;
  if (c->precision == NBX_DS) return fail(c, NBX_ERR_ARG, "batched systems run in NBX_FP64 or NBX_MIXED");
  if (c->batch_sizes.empty()) return fail(c, NBX_ERR_STATE, "nbx_batch_force_dev before nbx_batch_setup");
  if (!d_m || !d_x || !d_v || !d_acc || !d_jerk || !d_pot) return fail(c, NBX_ERR_ARG, "NULL device array");
  if (!(eps2 >= 0.0)) return fail(c, NBX_ERR_ARG, "eps2 must be >= 0");
  return batch_enqueue(c, static_cast<hipStream_t>(stream), d_m, d_x, d_v, eps2, d_acc, d_jerk, d_pot);
}

int nbx_batch_tune(nbx_ctx *c, void *stream, const double *d_m, const double *d_x, const double *d_v, double eps2,
                   double *d_acc, double *d_jerk, double *d_pot, int32_t *lanes_per_class) {
  if (int rc = check_ctx(c)) return rc;
  if (c->precision == NBX_DS) return fail(c, NBX_ERR_ARG, "batched systems run in NBX_FP64 or NBX_MIXED");
  if (c->batch_sizes.empty()) return fail(c, NBX_ERR_STATE, "nbx_batch_tune before nbx_batch_setup");
  if (!d_m || !d_x || !d_v || !d_acc || !d_jerk || !d_pot) return fail(c, NBX_ERR_ARG, "NULL device array");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned present = 0;
  for (int32_t n : c->batch_sizes) present |= 1u << batch_class(n);
  struct Events {  // destroyed on every return path
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } ev;
  HIP_TRY(c, hipEventCreate(&ev.e0));
  HIP_TRY(c, hipEventCreate(&ev.e1));
  hipEvent_t e0 = ev.e0, e1 = ev.e1;
  int best[8];
  for (int cl = 0; cl < 8; ++cl) {
    best[cl] = -1;
    if (!(present & (1u << cl))) continue;
    float best_ms = 1e30f;
    for (int lg = 0; lg <= 6; ++lg) {
      int lgs[8];
      for (int k = 0; k < 8; ++k) lgs[k] = lg;
      int rc = batch_upload(c, 1u << cl, lgs, s);
      for (int rep = 0; rc == NBX_OK && rep < 2; ++rep)
        rc = batch_enqueue(c, s, d_m, d_x, d_v, eps2, d_acc, d_jerk, d_pot);
      if (rc) return rc;
      constexpr int reps = 10;
      HIP_TRY(c, hipEventRecord(e0, s));
      for (int rep = 0; rc == NBX_OK && rep < reps; ++rep)
        rc = batch_enqueue(c, s, d_m, d_x, d_v, eps2, d_acc, d_jerk, d_pot);
      HIP_TRY(c, hipEventRecord(e1, s));
      HIP_TRY(c, hipEventSynchronize(e1));
      if (rc) return rc;
      float ms = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) {
        best_ms = ms;
        best[cl] = lg;
      }
    }
  }
  for (int cl = 0; cl < 8; ++cl) {
    c->batch_lg[cl] = best[cl];
    if (lanes_per_class) lanes_per_class[cl] = best[cl] < 0 ? 0 : 1 << best[cl];
  }
  int rc = batch_upload(c, 0xffu, nullptr, s);
  if (rc) return rc;
  return batch_enqueue(c, s, d_m, d_x, d_v, eps2, d_acc, d_jerk, d_pot);
}

}  // extern "C"

// ---- block time-step integrator ------------------------------------------------------------------

namespace {

bool pow2(double x) {
  if (!(x > 0.0) || !(x <= 1.0)) return false;
  int e = 0;
  return std::frexp(x, &e) == 0.5;
}

BlockStepParams bs_params(nbx_ctx *c) {
  BlockStepParams bp{};
  bp.src = c->src;
  bp.n = c->bs.n;
  bp.eta4 = c->bs.p.eta4;
  bp.eta6 = c->bs.p.eta6;
  bp.eta_start = c->bs.p.eta_start;
  bp.dt_max = c->bs.p.dt_max;
  bp.dt_min = c->bs.p.dt_min;
  bp.dt = static_cast<double *>(c->bs.dt.p);
  bp.tnext = static_cast<double *>(c->bs.tnext.p);
  bp.list = static_cast<int32_t *>(c->bs.list.p);
  bp.level_count = static_cast<int *>(c->bs.level_count.p);
  bp.sched = static_cast<BsSched *>(c->bs.sched.p);
  bp.acc = static_cast<const double *>(c->bs.acc.p);
  bp.jrk = static_cast<const double *>(c->bs.jrk.p);
  bp.snp = static_cast<const double *>(c->bs.snp.p);
  bp.err = c->d_err;
  return bp;
}

// Forces on the first ni particles of the list at time t into the integrator's force rows (the
// kernels without the nearest-neighbour search: the integrator never uses it).  With
// step != nullptr (a block step) the corrector may be fused into the combine kernel (*fused).
int bs_force(nbx_ctx *c, int ni, double t, const BlockStepParams *step = nullptr, bool *fused = nullptr) {
  c->t_pred = t;
  c->predicted = true;
  return enqueue_force(c, c->stream, ni, static_cast<const int32_t *>(c->bs.list.p), nullptr, nullptr, nullptr,
                       nullptr, nullptr, c->bs.p.eps2, nullptr, static_cast<double *>(c->bs.acc.p),
                       static_cast<double *>(c->bs.jrk.p), static_cast<double *>(c->bs.snp.p), nullptr,
                       static_cast<double *>(c->bs.pot.p), nullptr, nullptr, nullptr, nullptr, step, t, fused);
}

// Schedule the next block step; returns (t_next, count, clamped so far) through the pinned copy.
int bs_schedule(nbx_ctx *c, double *t_next, int *count, int *clamped) {
  const BlockStepParams bp = bs_params(c);
  const int parity = c->bs.parity;
  HIP_TRY(c, launch_bs_schedule(bp, c->bs.t, parity, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->bs.h_sched, bp.sched, sizeof(BsSched), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->bs.parity = parity ^ 1;
  *t_next = c->bs.h_sched->t_next;
  *count = c->bs.h_sched->count[parity];
  *clamped = c->bs.h_sched->clamped;
  return NBX_OK;
}

// Device-driven run: the host enqueues kDdBatch block steps at a time (schedule, gravity, combine
// with the corrector; each kernel reads N_active and the block time from the schedule record) and
// synchronises once per batch.  Launch shapes per N_i class come from ctx_shape (tuned table or
// static rule) with one sink per lane and at least two source splits, so that the corrector
// always runs in the combine kernel.  Needs at least two source tiles; returns NBX_ERR_STATE
// otherwise (the caller then takes the host loop).
constexpr int kDdBatch = 32;

int bs_run_dd(nbx_ctx *c, double t_end, int *status) {
  const int n = c->bs.n;
  const int nj_pad = (c->nj + kTile - 1) / kTile * kTile;
  const int ntiles = nj_pad / kTile;
  if (ntiles < 2) return NBX_ERR_STATE;
  ForceParams fp{};
  int kmax = 0;
  while ((1 << kmax) < n && kmax < 31) ++kmax;
  size_t part_slots = 0;
  int force_groups = 1, combine_groups = 1;
  for (int k = 0; k <= kmax; ++k) {
    const int ni = std::min(1 << k, n);
    LaunchShape ls = ctx_shape(c, ni, nj_pad);
    if (ls.sinks_per_lane == 2) ls.sinks_per_lane = 1;  // one sink per lane: blocks of 256 / L sinks
    int S = std::max(2, std::min(ls.splits, ntiles));
    const int64_t scap = ((int64_t)1 << 21) / ni;
    if (S > scap) S = std::max<int64_t>(2, scap);
    const int Q = kThreads >> ls.lanes_log2;
    const int blocks = (ni + Q - 1) / Q;
    fp.dd_shape[k] = make_int2(ls.lanes_log2, S);
    part_slots = std::max(part_slots, (size_t)S * (size_t)ni);
    force_groups = std::max(force_groups, blocks * S);
    combine_groups = std::max(combine_groups, (ni + (1 << combine_wlog(ni, S)) - 1) >> combine_wlog(ni, S));
  }
  for (int k = kmax + 1; k < 32; ++k) fp.dd_shape[k] = fp.dd_shape[kmax];
  force_groups = std::min(force_groups, 2048);  // 8 per CU; larger steps loop over their work items
  combine_groups = std::min(combine_groups, 512);
  {
    const size_t K = (size_t)values_per_sink(c->cfg.order);
    if (int rc = grow(c, c->part, part_slots * K * sizeof(double))) return rc;
    if (int rc = grow(c, c->part_key, part_slots * sizeof(uint64_t))) return rc;
    if (int rc = grow(c, c->part_idx, part_slots * sizeof(int32_t))) return rc;
  }
  const BlockStepParams bp = bs_params(c);
  fp.src = c->src;
  fp.nj = c->nj;
  fp.nj_pad = nj_pad;
  fp.eps2 = c->bs.p.eps2;
  fp.i_addr = bp.list;
  fp.acc = static_cast<double *>(c->bs.acc.p);
  fp.jrk = static_cast<double *>(c->bs.jrk.p);
  fp.snp = static_cast<double *>(c->bs.snp.p);
  fp.pot = static_cast<double *>(c->bs.pot.p);
  fp.part = static_cast<double *>(c->part.p);
  fp.part_key = static_cast<uint64_t *>(c->part_key.p);
  fp.part_idx = static_cast<int32_t *>(c->part_idx.p);
  fp.err = c->d_err;
  fp.nn = 0;
  fp.bs_fuse = 1;
  fp.bs = bp;
  ForceParams fpp[2] = {fp, fp};
  for (int p = 0; p < 2; ++p) {
    fpp[p].dd_count = &bp.sched->count[p];
    fpp[p].dd_t = &bp.sched->tnow[p ^ 1];
  }
  // the run's fields of the schedule record (stop .. steps) from the host, and the counter of the
  // step before the first schedule, which the host has already counted, cleared
  int parity = c->bs.parity;
  BsSched *h = c->bs.h_sched;
  h->stop = 0;
  h->tnow[0] = h->tnow[1] = c->bs.t;
  h->t_end = t_end;
  h->blocks = c->bs.blocks;
  h->steps = c->bs.steps;
  const size_t off = offsetof(BsSched, stop);
  hipStream_t s = c->stream;
  HIP_TRY(c, hipMemcpyAsync(reinterpret_cast<char *>(bp.sched) + off, reinterpret_cast<char *>(h) + off,
                            sizeof(BsSched) - off, hipMemcpyHostToDevice, s));
  HIP_TRY(c, launch_fill_i32(&bp.sched->count[parity ^ 1], 1, 0, s));
  for (;;) {
    for (int k = 0; k < kDdBatch; ++k) {
      HIP_TRY(c, launch_bs_schedule_dd(bp, parity, s));
      HIP_TRY(c, launch_force_dd(c->cfg.order, c->precision, fpp[parity], force_groups, combine_groups, s));
      parity ^= 1;
    }
    HIP_TRY(c, hipMemcpyAsync(h, bp.sched, sizeof(BsSched), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (h->stop) break;
  }
  c->bs.parity = parity;
  c->bs.t = h->tnow[parity];
  c->bs.blocks = h->blocks;
  c->bs.steps = h->steps;
  c->t_pred = c->bs.t;
  c->predicted = true;
  *status = h->clamped > 0 ? NBX_WARN_DT_MIN : NBX_OK;
  return NBX_OK;
}

int bs_check(nbx_ctx *c) {
  if (int rc = check_ctx(c)) return rc;
  if (!c->bs.ready) return fail(c, NBX_ERR_STATE, "no block time-step state (nbx_bs_init, and no nbx_set_j since)");
  return NBX_OK;
}

}  // namespace

extern "C" {

int nbx_bs_init(nbx_ctx *c, int n, const int64_t *id, const double *m, const double *x, const double *v,
                const nbx_bs_params *p) {
  if (int rc = check_ctx(c)) return rc;
  if (c->cfg.order != 4 && c->cfg.order != 6) return fail(c, NBX_ERR_ARG, "the integrator needs order 4 or 6");
  if (n < 1 || !id || !m || !x || !v || !p) return fail(c, NBX_ERR_ARG, "need n >= 1 and every array");
  if (n > c->cfg.nj_max || n > c->cfg.ni_max)
    return fail(c, NBX_ERR_CAPACITY, "n=%d exceeds nj_max=%d or ni_max=%d", n, c->cfg.nj_max, c->cfg.ni_max);
  if (!(p->eps2 >= 0.0) || !(p->eta4 > 0.0) || !(p->eta_start > 0.0) || (c->cfg.order == 6 && !(p->eta6 > 0.0)))
    return fail(c, NBX_ERR_ARG, "need eps2 >= 0 and positive eta4, eta_start (and eta6 for order 6)");
  if (!pow2(p->dt_max) || !pow2(p->dt_min) || p->dt_min > p->dt_max ||
      p->dt_min < std::ldexp(1.0, -(kBsLevels - 1)))
    return fail(c, NBX_ERR_ARG, "dt_max and dt_min must be powers of two with 2^-%d <= dt_min <= dt_max <= 1",
                kBsLevels - 1);
  c->bs.ready = false;
  const size_t N = (size_t)n;
  int rc = NBX_OK;
  rc = rc ? rc : grow(c, c->bs.dt, N * 8);
  rc = rc ? rc : grow(c, c->bs.tnext, N * 8);
  rc = rc ? rc : grow(c, c->bs.list, N * 4);
  rc = rc ? rc : grow(c, c->bs.acc, N * 24);
  rc = rc ? rc : grow(c, c->bs.jrk, N * 24);
  if (c->cfg.order == 6) rc = rc ? rc : grow(c, c->bs.snp, N * 24);
  rc = rc ? rc : grow(c, c->bs.pot, N * 8);
  rc = rc ? rc : grow(c, c->bs.level_count, kBsLevels * sizeof(int));
  rc = rc ? rc : grow(c, c->bs.sched, sizeof(BsSched));
  rc = rc ? rc : grow(c, c->up, N * (8 + 8 + 24 + 24) + 256);
  if (rc) return rc;
  if (!c->bs.h_sched) {
    void *h = nullptr;
    HIP_TRY(c, hipHostMalloc(&h, sizeof(BsSched)));
    c->bs.h_sched = static_cast<BsSched *>(h);
  }
  c->bs.n = n;
  c->bs.p = *p;
  c->bs.t = 0.0;
  c->bs.parity = 0;
  c->bs.blocks = c->bs.steps = 0;
  c->nj = n;
  char *base = static_cast<char *>(c->up.p);
  int64_t *d_id = reinterpret_cast<int64_t *>(base);
  double *d_m = reinterpret_cast<double *>(base + N * 8);
  double *d_x = d_m + N;
  double *d_v = d_x + 3 * N;
  hipStream_t s = c->stream;
  HIP_TRY(c, hipMemcpyAsync(d_id, id, N * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(d_m, m, N * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(d_x, x, N * 24, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(d_v, v, N * 24, hipMemcpyHostToDevice, s));
  const BlockStepParams bp = bs_params(c);
  HIP_TRY(c, launch_fill_i32(bp.level_count, kBsLevels, 0, s));  // counted by the start kernel
  HIP_TRY(c, launch_bs_load(c->cfg.order, bp, d_id, d_m, d_x, d_v, s));
  // acc and jerk at t = 0; order 6 needs a second pass for the snap, which uses the accelerations
  if ((rc = bs_force(c, n, 0.0))) return rc;
  if (c->cfg.order == 6) {
    HIP_TRY(c, launch_bs_seed(bp, s));
    if ((rc = bs_force(c, n, 0.0))) return rc;
  }
  HIP_TRY(c, launch_bs_seed(bp, s));
  HIP_TRY(c, launch_bs_start(c->cfg.order, bp, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  c->bs.ready = true;
  return collect_errors(c);
}

int nbx_bs_step(nbx_ctx *c, double t_end, int *n_active) {
  if (int rc = bs_check(c)) return rc;
  if (n_active) *n_active = 0;
  double tn = 0.0;
  int ni = 0, clamped = 0;
  if (int rc = bs_schedule(c, &tn, &ni, &clamped)) return rc;
  if (clamped > 0) {  // a step hit dt_min: stop rather than crawl on at the smallest step
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int rc = collect_errors(c);
    return rc == NBX_OK ? NBX_WARN_DT_MIN : rc;
  }
  if (!(tn <= t_end) || ni < 1) return NBX_OK;
  const BlockStepParams bp = bs_params(c);
  bool fused = false;
  if (int rc = bs_force(c, ni, tn, &bp, &fused)) return rc;
  if (!fused) HIP_TRY(c, launch_bs_correct(c->cfg.order, bp, ni, tn, c->stream));
  c->bs.t = tn;
  c->bs.blocks += 1;
  c->bs.steps += ni;
  if (n_active) *n_active = ni;
  return NBX_OK;
}

int nbx_bs_run(nbx_ctx *c, double t_end, nbx_bs_stats *stats) {
  if (int rc = bs_check(c)) return rc;
  int rc = NBX_OK;
  int dd_status = NBX_OK;
  const int dd = getenv("NBX_BS_HOST_LOOP") ? NBX_ERR_STATE : bs_run_dd(c, t_end, &dd_status);
  if (dd == NBX_OK) {
    rc = dd_status;
  } else if (dd != NBX_ERR_STATE) {
    return dd;
  } else {
    for (;;) {  // one source tile, or the host loop asked for: one synchronised block step at a time
      int ni = 0;
      rc = nbx_bs_step(c, t_end, &ni);
      if (rc != NBX_OK || ni == 0) break;
    }
  }
  if (rc < 0) return rc;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int rc2 = collect_errors(c);
  if (rc2 < 0) return rc2;
  if (rc == NBX_OK) rc = rc2;
  if (stats) {
    stats->t = c->bs.t;
    stats->block_steps = c->bs.blocks;
    stats->particle_steps = c->bs.steps;
  }
  return rc;
}

int nbx_bs_get_state(nbx_ctx *c, double *t, double *x, double *v, double *dt, double *t_i, nbx_bs_stats *stats) {
  if (int rc = bs_check(c)) return rc;
  const size_t N = (size_t)c->bs.n;
  if (t) *t = c->bs.t;
  if (stats) {
    stats->t = c->bs.t;
    stats->block_steps = c->bs.blocks;
    stats->particle_steps = c->bs.steps;
  }
  if (x || v) {
    if (int rc = grow(c, c->up, N * 48 + 256)) return rc;
    double *d_x = static_cast<double *>(c->up.p);
    double *d_v = d_x + 3 * N;
    int32_t *list = static_cast<int32_t *>(c->bs.list.p);
    HIP_TRY(c, launch_iota(list, c->bs.n, c->stream));
    HIP_TRY(c, launch_predict_out(c->cfg.order, c->src, c->nj, c->bs.t, c->bs.n, list, d_x, d_v, nullptr, c->d_err,
                                  c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (x) HIP_TRY(c, hipMemcpy(x, d_x, N * 24, hipMemcpyDeviceToHost));
    if (v) HIP_TRY(c, hipMemcpy(v, d_v, N * 24, hipMemcpyDeviceToHost));
  }
  if (dt) HIP_TRY(c, hipMemcpy(dt, c->bs.dt.p, N * 8, hipMemcpyDeviceToHost));
  if (t_i) {
    std::vector<double> tn(N), d(N);
    HIP_TRY(c, hipMemcpy(tn.data(), c->bs.tnext.p, N * 8, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(d.data(), c->bs.dt.p, N * 8, hipMemcpyDeviceToHost));
    for (size_t k = 0; k < N; ++k) t_i[k] = tn[k] - d[k];
  }
  return collect_errors(c);
}

int nbx_bs_energy(nbx_ctx *c, double *ekin, double *epot) {
  if (int rc = bs_check(c)) return rc;
  const int n = c->bs.n;
  const size_t N = (size_t)n;
  int32_t *list = static_cast<int32_t *>(c->bs.list.p);
  HIP_TRY(c, launch_iota(list, n, c->stream));
  if (int rc = bs_force(c, n, c->bs.t)) return rc;
  if (int rc = grow(c, c->up, N * 56 + 256)) return rc;
  double *d_x = static_cast<double *>(c->up.p);
  double *d_v = d_x + 3 * N;
  double *d_m = d_v + 3 * N;
  HIP_TRY(c, launch_predict_out(c->cfg.order, c->src, c->nj, c->bs.t, n, list, d_x, d_v, nullptr, c->d_err,
                                c->stream));
  HIP_TRY(c, launch_gather_j(c->cfg.order, c->src, n, list, nullptr, d_m, nullptr, nullptr, nullptr, nullptr, nullptr,
                             nullptr, nullptr, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::vector<double> v(3 * N), m(N), pot(N);
  HIP_TRY(c, hipMemcpy(v.data(), d_v, N * 24, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(m.data(), d_m, N * 8, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(pot.data(), c->bs.pot.p, N * 8, hipMemcpyDeviceToHost));
  long double k = 0.0L, w = 0.0L;
  for (size_t i = 0; i < N; ++i) {
    k += 0.5L * m[i] * ((long double)v[3 * i] * v[3 * i] + (long double)v[3 * i + 1] * v[3 * i + 1] +
                        (long double)v[3 * i + 2] * v[3 * i + 2]);
    w += 0.5L * m[i] * pot[i];
  }
  if (ekin) *ekin = (double)k;
  if (epot) *epot = (double)w;
  return collect_errors(c);
}

}  // extern "C"

// ---- launch-shape tuner ------------------------------------------------------------------------

namespace {

// Candidate shapes for ni sinks against ntiles source tiles: every lanes-per-sink L (two sinks per
// lane only with L = 1) whose sink slots are not mostly idle, and every power-of-two split count
// (and ntiles itself) that gives at most 8192 workgroups and at most 2^21 partial sums; shapes with
// fewer than 64 workgroups are dropped unless no shape reaches 64 (few sources).
std::vector<LaunchShape> tune_candidates(int ni, int ntiles) {
  std::vector<LaunchShape> out;
  int64_t wmax = 0;
  int cover = 1;
  while (cover < ni) cover *= 2;
  for (int lg = 0; lg <= 8; ++lg) {
    for (int P = 1; P <= 2; ++P) {
      if (P == 2 && lg != 0) continue;
      const int Q = (kThreads >> lg) * P;
      if (Q > 1 && Q > 2 * cover) continue;
      const int blocks = (ni + Q - 1) / Q;
      for (int S = 1; S <= ntiles; S = (S * 2 <= ntiles || S == ntiles) ? S * 2 : ntiles) {
        const int64_t W = (int64_t)blocks * S;
        if (W <= 8192 && (int64_t)S * ni <= ((int64_t)1 << 21)) {
          LaunchShape ls;
          ls.lanes_log2 = lg;
          ls.sinks_per_lane = P;
          ls.splits = S;
          ls.blocks = blocks;
          out.push_back(ls);
          wmax = std::max(wmax, W);
        }
        if (S == ntiles) break;
      }
    }
  }
  const int64_t wmin = std::min<int64_t>(64, wmax);
  std::vector<LaunchShape> keep;
  for (const LaunchShape &ls : out)
    if ((int64_t)ls.blocks * ls.splits >= wmin) keep.push_back(ls);
  return keep;
}

}  // namespace

extern "C" {

int nbx_tune(nbx_ctx *c, int ni_max, int32_t *shapes_out, int n_classes) {
  if (int rc = check_ctx(c)) return rc;
  if (!c->predicted) return fail(c, NBX_ERR_STATE, "nbx_tune before nbx_predict");
  if (c->nj < 1) return fail(c, NBX_ERR_STATE, "no sources in use");
  if (ni_max < 1) return fail(c, NBX_ERR_ARG, "ni_max must be >= 1");
  if (shapes_out && n_classes < 0) return fail(c, NBX_ERR_ARG, "n_classes < 0");
  ni_max = std::min(std::min(ni_max, c->cfg.ni_max), c->nj);
  const int nj_pad = (c->nj + kTile - 1) / kTile * kTile;
  const int ntiles = nj_pad / kTile;
  struct Events {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } ev;
  HIP_TRY(c, hipEventCreate(&ev.e0));
  HIP_TRY(c, hipEventCreate(&ev.e1));
  struct Reset {  // leave no shape override behind on any return path
    nbx_ctx *c;
    ~Reset() { c->force_shape = nullptr; }
  } reset{c};
  const int pr = c->precision;
  // the kernels later calls use: without the nearest-neighbour search while the device integrator
  // runs (it never needs it) or when the context does not want it
  const bool nn = !c->bs.ready && c->cfg.want_nn != 0;
  c->tune_ntiles[pr] = 0;
  for (auto &t : c->tuned[pr]) t = nbx_ctx::TunedShape{};
  const int kmax = ni_class(ni_max);
  std::vector<int32_t> addr;
  for (int k = 0; k <= kmax; ++k) {
    const int ni = std::min(1 << k, ni_max);
    addr.resize(ni);
    for (int i = 0; i < ni; ++i) addr[i] = (int32_t)((int64_t)i * c->nj / ni);  // evenly strided sinks
    HIP_TRY(c, hipStreamSynchronize(c->stream));  // the previous class's launches read d_iaddr
    HIP_TRY(c, hipMemcpy(c->d_iaddr, addr.data(), (size_t)ni * 4, hipMemcpyHostToDevice));
    out_layout(c, ni);
    float best_ms = 1e30f;
    nbx_ctx::TunedShape best;
    for (const LaunchShape &cand : tune_candidates(ni, ntiles)) {
      c->force_shape = &cand;
      auto launch = [&]() {
        return enqueue_force(c, c->stream, ni, c->d_iaddr, nullptr, nullptr, nullptr, nullptr, nullptr, 0.0, nullptr,
                             c->d_acc, c->d_jrk ? c->d_jrk : c->d_acc, c->d_snp, c->d_crk, c->d_pot,
                             nn ? c->d_nnid : nullptr, nn ? c->d_nnr2 : nullptr, nullptr, nullptr);
      };
      if (int rc = launch()) return rc;  // warm-up, and an estimate of the launch time
      HIP_TRY(c, hipEventRecord(ev.e0, c->stream));
      if (int rc = launch()) return rc;
      HIP_TRY(c, hipEventRecord(ev.e1, c->stream));
      HIP_TRY(c, hipEventSynchronize(ev.e1));
      float ms = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&ms, ev.e0, ev.e1));
      const int reps = std::max(2, std::min(20, (int)(2.0f / std::max(ms, 1e-3f))));
      HIP_TRY(c, hipEventRecord(ev.e0, c->stream));
      for (int r = 0; r < reps; ++r)
        if (int rc = launch()) return rc;
      HIP_TRY(c, hipEventRecord(ev.e1, c->stream));
      HIP_TRY(c, hipEventSynchronize(ev.e1));
      HIP_TRY(c, hipEventElapsedTime(&ms, ev.e0, ev.e1));
      ms /= reps;
      if (ms < best_ms) {
        best_ms = ms;
        best.lanes_log2 = cand.lanes_log2;
        best.sinks_per_lane = cand.sinks_per_lane;
        best.splits = cand.splits;
      }
    }
    c->force_shape = nullptr;
    c->tuned[pr][k] = best;
    if (shapes_out && k < n_classes) {
      shapes_out[3 * k] = best.lanes_log2 < 0 ? 0 : 1 << best.lanes_log2;
      shapes_out[3 * k + 1] = best.sinks_per_lane;
      shapes_out[3 * k + 2] = best.splits;
    }
  }
  c->tune_ntiles[pr] = ntiles;
  c->last_ni = -1;  // the host-path result buffers hold tuning output
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return collect_errors(c);
}

int nbx_sync(nbx_ctx *c, void *stream) {
  if (int rc = check_ctx(c)) return rc;
  if (stream) HIP_TRY(c, hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipDeviceSynchronize());
  return collect_errors(c);
}

int nbx_clock_sample(nbx_ctx *c, void *stream, int n_groups, int64_t *d_out) {
  if (int rc = check_ctx(c)) return rc;
  if (n_groups < 1 || !d_out) return fail(c, NBX_ERR_ARG, "need n_groups >= 1 and an output array");
  HIP_TRY(c, launch_clock_sample(n_groups, d_out, static_cast<hipStream_t>(stream)));
  return NBX_OK;
}

int nbx_clock_rates(nbx_ctx *c, int *wall_khz, int *sclk_max_khz) {
  if (int rc = check_ctx(c)) return rc;
  int w = 0, s = 0;
  HIP_TRY(c, hipDeviceGetAttribute(&w, hipDeviceAttributeWallClockRate, c->cfg.device));
  HIP_TRY(c, hipDeviceGetAttribute(&s, hipDeviceAttributeClockRate, c->cfg.device));
  if (wall_khz) *wall_khz = w;
  if (sclk_max_khz) *sclk_max_khz = s;
  return NBX_OK;
}

int nbx_launch_shape(nbx_ctx *c, int ni, int *lanes_per_sink, int *sinks_per_lane, int *splits, int *workgroups) {
  if (!c || ni < 1) return NBX_ERR_ARG;
  const int nj_pad = (c->nj + kTile - 1) / kTile * kTile;
  const LaunchShape ls = ctx_shape(c, ni, nj_pad);
  if (lanes_per_sink) *lanes_per_sink = 1 << ls.lanes_log2;
  if (sinks_per_lane) *sinks_per_lane = ls.sinks_per_lane;
  if (splits) *splits = ls.splits;
  if (workgroups) *workgroups = ls.blocks * ls.splits;
  return NBX_OK;
}

}  // extern "C"
