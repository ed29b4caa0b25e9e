// nbx_kernels.hip -- gfx950 kernels of the direct N-body force path.
//
// The three GPU steps of one force evaluation are the ones the paper lists (Methods > Other
// differences): a copy kernel that scatters updated sources into the device arrays, a
// predictor, and the gravity kernel.  Here the predictor is fused into the gravity kernel: each
// workgroup predicts the sources of the LDS tile it is about to use, in FP64, while staging
// them (Background, Yebisu paragraph: prediction on the GPU), and predicts its by-address sinks
// with the same code so that a sink and its own source copy agree bit for bit.
//
// Work decomposition (Methods > Parallelisation method; Results > Block-size / active-particles):
//   * a workgroup (256 threads, four wave64s) owns a block of Q sinks and one of S contiguous
//     source ranges ("j-split"), so that a handful of active sinks still fills the 256 CUs;
//   * inside the workgroup each sink is handled by L lanes (L = 1..256, "2D thread-blocks")
//     that stride over the LDS tile, and each lane may hold P = 1 or 2 sinks so that one LDS
//     broadcast read of a source feeds P interactions;
//   * partial sums are combined deterministically: a butterfly over the L lanes (all lanes end
//     with bit-identical values), an LDS pass across waves when L > 64, and, when S > 1, a
//     second kernel that sums the S partials of each sink in a fixed order (the paper folded
//     the subsets with atomics inside the gravity kernel, Methods > Other differences; on
//     gfx950 the device-scope fence that would need per workgroup is the expensive part).
//
// Orders: 2 (the GRAPE-5 / leapfrog mode of the Background section: acceleration and potential
// from positions and masses), 4 (adds the jerk), 6 (adds the snap, from predicted
// accelerations) and 8 (adds the crackle, from predicted jerks: the higher-order expansion that
// Methods > Numerical Accuracy and the Conclusion name).  All four share the staging, the loop,
// the reductions and the combine.
//
// Arithmetic per interaction (the pair terms of nbx.h):
//   MIXED: dx = (xh_j - xh_i) + (xl_j - xl_i) in FP32 from double-single positions, FP32
//          velocities/masses, R^-1 straight from v_rsq_f32 (a Newton step measured no better
//          in the median, 2x better only in the worst sink, for 10% of the issue slots), FP32
//          chunk sums folded into FP64 totals (acceleration every 16 terms, the rest every 64).
//          FP32 add/mul/fma issue at twice the FP64 rate on gfx950.
//   FP64:  all IEEE double; R^-1 from v_rsq_f64 plus one third-order Newton correction; FP64
//          chunk sums folded with TwoSum.
// Self-interaction (by-address sinks): a sink and its own source copy are predicted by the same
// code, so r = 0 exactly.  A wave checks per tile whether the tile holds the own source of one of its sinks
// (1-2 tiles of nj/256 when the active sinks are consecutive) and only then runs the loop variant
// that forces R^-1 = 0 and the nearest-neighbour key to its maximum for j == self: the self pair
// never enters a sum, so no -m_i/eps term has to be removed later, and eps2 = 0 needs no special
// case.  A distinct source at the sink's position (r = 0) is an ordinary candidate.

#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "nbx_internal.h"
#include "nbx_predict.h"
#include "nbx_bs_device.h"

#include "nbx.h"

namespace nbx {

constexpr int kChunkAcc = 16;  // acceleration terms summed in plain FP32/FP64 before a fold
constexpr int kChunk = 64;     // same for jerk, pot and snap (a multiple of kChunkAcc)
// The gravity kernel's long-chunk variant (workgroups that run several source tiles with one lane
// per sink) sums Tr::kLongChunk acceleration terms per chunk: fewer folds per interaction, while
// the one-off re-scan of a nearest-neighbour group (one chunk long) stays small next to the loop.

// ---------------------------------------------------------------------------------------------
// Compensated accumulation: K running values, each a plain chunk sum that is folded every
// kChunkAcc terms (the acceleration, values 0..2; Tr::kLongChunk in the gravity kernel's long-chunk
// variant) or kChunk terms (the others) into a running total: the summation error of a chunk grows
// with its length, and the acceleration carries the tightest bound.  FP64 chunks fold into a (hi, lo) pair with TwoSum (Knuth), i.e. a double-double
// total; FP32 chunks fold into an FP64 total (a convert and an FP64 add, cheaper in issue slots
// than a single-single TwoSum and more accurate).
// ---------------------------------------------------------------------------------------------
template <typename T, int K>
struct Comp {
  T part[K], hi[K], lo[K];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int k = 0; k < K; ++k) part[k] = hi[k] = lo[k] = T(0);
  }
  template <int K0, int K1>
  __device__ __forceinline__ void fold() {
#pragma clang fp contract(off)
#pragma unroll
    for (int k = K0; k < K1; ++k) {
      const T s = hi[k] + part[k];
      const T bp = s - hi[k];
      const T e = (hi[k] - (s - bp)) + (part[k] - bp);
      hi[k] = s;
      lo[k] += e;
      part[k] = T(0);
    }
  }
  __device__ __forceinline__ double value(int k) const { return (double)hi[k] + (double)lo[k]; }
};

template <int K>
struct Comp<float, K> {
  float part[K];
  double sum[K];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      part[k] = 0.0f;
      sum[k] = 0.0;
    }
  }
  template <int K0, int K1>
  __device__ __forceinline__ void fold() {
#pragma unroll
    for (int k = K0; k < K1; ++k) {
      sum[k] += (double)part[k];
      part[k] = 0.0f;
    }
  }
  __device__ __forceinline__ double value(int k) const { return sum[k]; }
};

// value slots: 0..2 acc, 3..5 jerk, 6 pot, 7..9 snap, 10..12 crackle (order 2: 0..2 acc, 3 pot)
template <int Order>
constexpr int kValues = Order == 8 ? 13 : (Order == 6 ? 10 : (Order == 4 ? 7 : 4));
template <int Order>
constexpr int kPotSlot = Order == 2 ? 3 : 6;

// ---------------------------------------------------------------------------------------------
// Precision traits: LDS tile layout, sink representation and the pair interaction
// ---------------------------------------------------------------------------------------------
template <int Order>
struct MixedTile;
template <>
struct MixedTile<2> {  // 32 B per source
  float4 t0[kTile];    // xh.x xh.y xh.z m
  float4 t1[kTile];    // xl.x xl.y xl.z (unused)
};
template <>
struct MixedTile<4> {  // 40 B per source
  float4 t0[kTile];    // xh.x xh.y xh.z m
  float4 t1[kTile];    // xl.x xl.y xl.z vx
  float2 t2[kTile];    // vy vz
};
template <>
struct MixedTile<6> {  // 52 B per source
  float4 t0[kTile];    // xh.x xh.y xh.z m
  float4 t1[kTile];    // xl.x xl.y xl.z vx
  float4 t2[kTile];    // vy vz ax ay
  float t3[kTile];     // az
};
template <>
struct MixedTile<8> {  // 64 B per source
  float4 t0[kTile];    // xh.x xh.y xh.z m
  float4 t1[kTile];    // xl.x xl.y xl.z vx
  float4 t2[kTile];    // vy vz ax ay
  float4 t3[kTile];    // az jx jy jz
};

__device__ __forceinline__ void ds_split(double x, float &hi, float &lo) {
  hi = (float)x;
  lo = (float)(x - (double)hi);
}

template <int Order>
struct Mixed {
  using Real = float;
  using Key = uint32_t;
  static constexpr int kK = kValues<Order>;
  // long chunks: acceleration terms per FP32 chunk before the fold into FP64 (the chunk's own
  // rounding stays a small part of the error: measured 1.8e-8 against ~1e-7 condition-normalised)
  static constexpr int kLongChunk = 32;
  using Tile = MixedTile<Order>;
  struct Sink {
    float xh[3], xl[3], v[3], a[3], j[3];  // j: order 8
    float m;
    int64_t id;
  };
  struct J {
    float xh[3], m, xl[3], v[3], a[3], j[3];
  };

  // A sink whose state is exactly a staged source record (batched systems).
  __device__ static __forceinline__ Sink sink_from_j(const J &j) {
    Sink s;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s.xh[k] = j.xh[k];
      s.xl[k] = j.xl[k];
      s.v[k] = j.v[k];
      s.a[k] = j.a[k];
      s.j[k] = j.j[k];
    }
    s.m = j.m;
    s.id = -1;
    return s;
  }

  // ap: the acceleration [3], followed for order 8 by the jerk [3]
  __device__ static __forceinline__ Sink make_sink(const double xp[3], const double vp[3],
                                                   const double ap[6], double m) {
    Sink s;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ds_split(xp[k], s.xh[k], s.xl[k]);
      s.v[k] = (float)vp[k];
      s.a[k] = (float)ap[k];
      s.j[k] = Order == 8 ? (float)ap[3 + k] : 0.0f;
    }
    s.m = (float)m;
    s.id = -1;
    return s;
  }

  __device__ static __forceinline__ void store(Tile &tl, int e, const double xp[3], const double vp[3],
                                               const double ap[6], double m) {
    float xh[3], xl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) ds_split(xp[k], xh[k], xl[k]);
    tl.t0[e] = make_float4(xh[0], xh[1], xh[2], (float)m);
    if constexpr (Order == 2) {
      tl.t1[e] = make_float4(xl[0], xl[1], xl[2], 0.0f);
    } else if constexpr (Order == 4) {
      tl.t1[e] = make_float4(xl[0], xl[1], xl[2], (float)vp[0]);
      tl.t2[e] = make_float2((float)vp[1], (float)vp[2]);
    } else if constexpr (Order == 6) {
      tl.t1[e] = make_float4(xl[0], xl[1], xl[2], (float)vp[0]);
      tl.t2[e] = make_float4((float)vp[1], (float)vp[2], (float)ap[0], (float)ap[1]);
      tl.t3[e] = (float)ap[2];
    } else {
      tl.t1[e] = make_float4(xl[0], xl[1], xl[2], (float)vp[0]);
      tl.t2[e] = make_float4((float)vp[1], (float)vp[2], (float)ap[0], (float)ap[1]);
      tl.t3[e] = make_float4((float)ap[2], (float)ap[3], (float)ap[4], (float)ap[5]);
    }
  }

  __device__ static __forceinline__ J load(const Tile &tl, int e) {
    J j;
    const float4 a = tl.t0[e];
    const float4 b = tl.t1[e];
    j.xh[0] = a.x; j.xh[1] = a.y; j.xh[2] = a.z; j.m = a.w;
    j.xl[0] = b.x; j.xl[1] = b.y; j.xl[2] = b.z;
    if constexpr (Order == 2) {
      // positions and mass are all the 2nd-order terms use
    } else if constexpr (Order == 4) {
      const float2 c = tl.t2[e];
      j.v[0] = b.w; j.v[1] = c.x; j.v[2] = c.y;
    } else if constexpr (Order == 6) {
      const float4 c = tl.t2[e];
      j.v[0] = b.w;
      j.v[1] = c.x; j.v[2] = c.y; j.a[0] = c.z; j.a[1] = c.w;
      j.a[2] = tl.t3[e];
    } else {
      const float4 c = tl.t2[e];
      const float4 d = tl.t3[e];
      j.v[0] = b.w;
      j.v[1] = c.x; j.v[2] = c.y; j.a[0] = c.z; j.a[1] = c.w;
      j.a[2] = d.x; j.j[0] = d.y; j.j[1] = d.z; j.j[2] = d.w;
    }
    return j;
  }

  // The source record as the force loop sees it after staging (same conversions as store/load).
  __device__ static __forceinline__ J make_j(const double xp[3], const double vp[3], const double ap[6], double m) {
    J j;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ds_split(xp[k], j.xh[k], j.xl[k]);
      j.v[k] = (float)vp[k];
      j.a[k] = (float)ap[k];
      j.j[k] = Order == 8 ? (float)ap[3 + k] : 0.0f;
    }
    j.m = (float)m;
    return j;
  }

  // Position difference and a squared distance: with Fold (the kernels without neighbour lists)
  // the softened R^2 = |r|^2 + eps2 in one fma chain that starts from eps2, else the unsoftened
  // |r|^2.  The nearest-neighbour key is taken on this value (an increasing function of |r|^2), and
  // the one definition serves the force loop and the nearest-neighbour re-scan, so both produce
  // the same bits.
  template <bool Fold>
  __device__ static __forceinline__ float diff_d2(const J &j, const Sink &s, float eps2, float &dx, float &dy,
                                                  float &dz) {
    dx = (j.xh[0] - s.xh[0]) + (j.xl[0] - s.xl[0]);
    dy = (j.xh[1] - s.xh[1]) + (j.xl[1] - s.xl[1]);
    dz = (j.xh[2] - s.xh[2]) + (j.xl[2] - s.xl[2]);
    if constexpr (Fold) return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
    else return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
  }

  // Nearest-neighbour key: the bit pattern of |r|^2 >= 0, whose unsigned order is the order of
  // |r|^2 (the self pair is given the maximum key by the guarded loop).  The minimum over a group
  // of sources is kept on the keys themselves (one min3 per two keys).
  __device__ static __forceinline__ Key key_of(float r2) { return __float_as_uint(r2); }
  using GKey = Key;
  __device__ static __forceinline__ GKey gkey_none() { return ~Key(0); }
  __device__ static __forceinline__ Key group_key(GKey g) { return g; }
  // the group minimum as a value (a NaN for an empty group, so that no comparison holds); the
  // neighbour-list test runs once per group on it (tile_compute)
  static constexpr bool kChunkLists = true;
  __device__ static __forceinline__ float group_r2(GKey g) { return __uint_as_float(g); }

  template <bool Nbr>
  __device__ static __forceinline__ float pair_r2(const J &j, const Sink &s, float eps2) {
    float dx, dy, dz;
    return diff_d2<!Nbr>(j, s, eps2, dx, dy, dz);
  }
  template <bool Nbr>
  __device__ static __forceinline__ Key nn_key(const J &j, const Sink &s, float eps2) {
    return key_of(pair_r2<Nbr>(j, s, eps2));
  }

  // One pair; returns the unsoftened |r|^2 for the neighbour-list test (Nbr), else R^2.  NN: keep
  // the nearest-neighbour group minimum (the kernels without it leave gmin untouched), on |r|^2
  // with lists and on R^2 without.
  template <bool Guard, bool NN, bool Nbr>
  __device__ static __forceinline__ float interact(const J &j, const Sink &s, float eps2, int jidx, int self,
                                                  Comp<float, kValues<Order>> &A, GKey &gmin) {
    float dx, dy, dz;
    const float r2 = diff_d2<!Nbr>(j, s, eps2, dx, dy, dz);
    const float R2 = Nbr ? r2 + eps2 : r2;
    float rinv = __builtin_amdgcn_rsqf(R2);  // v_rsq_f32
    if constexpr (Guard) rinv = jidx != self ? rinv : 0.0f;
    const float rinv2 = rinv * rinv;
    const float mr = j.m * rinv;
    const float mr3 = mr * rinv2;
    if constexpr (Order == 2) {
      A.part[0] = __builtin_fmaf(mr3, dx, A.part[0]);
      A.part[1] = __builtin_fmaf(mr3, dy, A.part[1]);
      A.part[2] = __builtin_fmaf(mr3, dz, A.part[2]);
      A.part[3] -= mr;
    } else {
      const float dvx = j.v[0] - s.v[0];
      const float dvy = j.v[1] - s.v[1];
      const float dvz = j.v[2] - s.v[2];
      const float rv = __builtin_fmaf(dz, dvz, __builtin_fmaf(dy, dvy, dx * dvx));
      const float al = rv * rinv2;
      if constexpr (Order == 4) {
        const float am3 = al * -3.0f;
        const float wx = __builtin_fmaf(am3, dx, dvx);
        const float wy = __builtin_fmaf(am3, dy, dvy);
        const float wz = __builtin_fmaf(am3, dz, dvz);
        A.part[0] = __builtin_fmaf(mr3, dx, A.part[0]);
        A.part[1] = __builtin_fmaf(mr3, dy, A.part[1]);
        A.part[2] = __builtin_fmaf(mr3, dz, A.part[2]);
        A.part[3] = __builtin_fmaf(mr3, wx, A.part[3]);
        A.part[4] = __builtin_fmaf(mr3, wy, A.part[4]);
        A.part[5] = __builtin_fmaf(mr3, wz, A.part[5]);
        A.part[6] -= mr;
      } else {
        const float dax = j.a[0] - s.a[0];
        const float day = j.a[1] - s.a[1];
        const float daz = j.a[2] - s.a[2];
        const float vv = __builtin_fmaf(dvz, dvz, __builtin_fmaf(dvy, dvy, dvx * dvx));
        const float ra = __builtin_fmaf(dz, daz, __builtin_fmaf(dy, day, dx * dax));
        const float be = __builtin_fmaf(al, al, (vv + ra) * rinv2);
        const float am3 = al * -3.0f;
        const float am6 = al * -6.0f;
        const float bm3 = be * -3.0f;
        const float a0x = mr3 * dx, a0y = mr3 * dy, a0z = mr3 * dz;
        const float a1x = __builtin_fmaf(am3, a0x, mr3 * dvx);
        const float a1y = __builtin_fmaf(am3, a0y, mr3 * dvy);
        const float a1z = __builtin_fmaf(am3, a0z, mr3 * dvz);
        const float a2x = __builtin_fmaf(am6, a1x, __builtin_fmaf(bm3, a0x, mr3 * dax));
        const float a2y = __builtin_fmaf(am6, a1y, __builtin_fmaf(bm3, a0y, mr3 * day));
        const float a2z = __builtin_fmaf(am6, a1z, __builtin_fmaf(bm3, a0z, mr3 * daz));
        A.part[0] += a0x; A.part[1] += a0y; A.part[2] += a0z;
        A.part[3] += a1x; A.part[4] += a1y; A.part[5] += a1z;
        A.part[6] -= mr;
        A.part[7] += a2x; A.part[8] += a2y; A.part[9] += a2z;
        if constexpr (Order == 8) {
          // crackle: gamma = (3 v.a + r.j) / R^2 + alpha (3 beta - 4 alpha^2),
          // A3 = m j / R^3 - 9 alpha A2 - 9 beta A1 - 3 gamma A0
          const float djx = j.j[0] - s.j[0];
          const float djy = j.j[1] - s.j[1];
          const float djz = j.j[2] - s.j[2];
          const float va = __builtin_fmaf(dvz, daz, __builtin_fmaf(dvy, day, dvx * dax));
          const float rj = __builtin_fmaf(dz, djz, __builtin_fmaf(dy, djy, dx * djx));
          const float ga = __builtin_fmaf(__builtin_fmaf(3.0f, va, rj), rinv2,
                                          al * __builtin_fmaf(-4.0f * al, al, 3.0f * be));
          const float am9 = al * -9.0f;
          const float bm9 = be * -9.0f;
          const float gm3 = ga * -3.0f;
          A.part[10] += __builtin_fmaf(am9, a2x, __builtin_fmaf(bm9, a1x, __builtin_fmaf(gm3, a0x, mr3 * djx)));
          A.part[11] += __builtin_fmaf(am9, a2y, __builtin_fmaf(bm9, a1y, __builtin_fmaf(gm3, a0y, mr3 * djy)));
          A.part[12] += __builtin_fmaf(am9, a2z, __builtin_fmaf(bm9, a1z, __builtin_fmaf(gm3, a0z, mr3 * djz)));
        }
      }
    }
    if constexpr (NN) {
      Key key = key_of(r2);
      if constexpr (Guard) key = jidx != self ? key : ~Key(0);
      gmin = key < gmin ? key : gmin;
    }
    return r2;
  }
};

template <int Order>
struct F64Tile;
template <>
struct F64Tile<2> {   // 32 B per source
  double2 t0[kTile];  // x y
  double2 t1[kTile];  // z m
};
template <>
struct F64Tile<4> {  // 56 B per source
  double2 t0[kTile];  // x y
  double2 t1[kTile];  // z m
  double2 t2[kTile];  // vx vy
  double t3[kTile];   // vz
};
template <>
struct F64Tile<6> {  // 80 B per source
  double2 t0[kTile];  // x y
  double2 t1[kTile];  // z m
  double2 t2[kTile];  // vx vy
  double2 t3[kTile];  // vz ax
  double2 t4[kTile];  // ay az
};
template <>
struct F64Tile<8> {  // 104 B per source
  double2 t0[kTile];  // x y
  double2 t1[kTile];  // z m
  double2 t2[kTile];  // vx vy
  double2 t3[kTile];  // vz ax
  double2 t4[kTile];  // ay az
  double2 t5[kTile];  // jx jy
  double t6[kTile];   // jz
};

// R^-1 in FP64: v_rsq_f64 estimate y, e = 1 - x y^2, y (1 + e/2 + 3e^2/8) (third-order Newton).
__device__ __forceinline__ double rsqrt64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double xy = x * y;
  const double e = fma(-xy, y, 1.0);
  const double c = fma(e, 0.375, 0.5);
  return fma(y * e, c, y);
}

template <int Order>
struct F64 {
  using Real = double;
  using Key = uint64_t;
  static constexpr int kK = kValues<Order>;
  static constexpr int kLongChunk = kChunk;  // long chunks: every FP64 sum folds (TwoSum) every 64 terms
  using Tile = F64Tile<Order>;
  struct Sink {
    double x[3], v[3], a[3], j[3];  // j: order 8
    double m;
    int64_t id;
  };
  struct J {
    double x[3], m, v[3], a[3], j[3];
  };

  __device__ static __forceinline__ Sink sink_from_j(const J &j) {
    Sink s;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s.x[k] = j.x[k];
      s.v[k] = j.v[k];
      s.a[k] = j.a[k];
      s.j[k] = j.j[k];
    }
    s.m = j.m;
    s.id = -1;
    return s;
  }

  // ap: the acceleration [3], followed for order 8 by the jerk [3]
  __device__ static __forceinline__ Sink make_sink(const double xp[3], const double vp[3],
                                                   const double ap[6], double m) {
    Sink s;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s.x[k] = xp[k];
      s.v[k] = vp[k];
      s.a[k] = ap[k];
      s.j[k] = Order == 8 ? ap[3 + k] : 0.0;
    }
    s.m = m;
    s.id = -1;
    return s;
  }

  __device__ static __forceinline__ void store(Tile &tl, int e, const double xp[3], const double vp[3],
                                               const double ap[6], double m) {
    tl.t0[e] = make_double2(xp[0], xp[1]);
    tl.t1[e] = make_double2(xp[2], m);
    if constexpr (Order == 2) {
    } else if constexpr (Order == 4) {
      tl.t2[e] = make_double2(vp[0], vp[1]);
      tl.t3[e] = vp[2];
    } else {
      tl.t2[e] = make_double2(vp[0], vp[1]);
      tl.t3[e] = make_double2(vp[2], ap[0]);
      tl.t4[e] = make_double2(ap[1], ap[2]);
      if constexpr (Order == 8) {
        tl.t5[e] = make_double2(ap[3], ap[4]);
        tl.t6[e] = ap[5];
      }
    }
  }

  __device__ static __forceinline__ J load(const Tile &tl, int e) {
    J j;
    const double2 a = tl.t0[e];
    const double2 b = tl.t1[e];
    j.x[0] = a.x; j.x[1] = a.y; j.x[2] = b.x; j.m = b.y;
    if constexpr (Order == 2) {
    } else if constexpr (Order == 4) {
      const double2 c = tl.t2[e];
      j.v[0] = c.x; j.v[1] = c.y; j.v[2] = tl.t3[e];
    } else {
      const double2 c = tl.t2[e];
      j.v[0] = c.x; j.v[1] = c.y;
      const double2 d = tl.t3[e];
      const double2 f = tl.t4[e];
      j.v[2] = d.x; j.a[0] = d.y; j.a[1] = f.x; j.a[2] = f.y;
      if constexpr (Order == 8) {
        const double2 g = tl.t5[e];
        j.j[0] = g.x; j.j[1] = g.y; j.j[2] = tl.t6[e];
      }
    }
    return j;
  }

  __device__ static __forceinline__ J make_j(const double xp[3], const double vp[3], const double ap[6], double m) {
    J j;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      j.x[k] = xp[k];
      j.v[k] = vp[k];
      j.a[k] = ap[k];
      j.j[k] = Order == 8 ? ap[3 + k] : 0.0;
    }
    j.m = m;
    return j;
  }

  // As Mixed::diff_d2.
  template <bool Fold>
  __device__ static __forceinline__ double diff_d2(const J &j, const Sink &s, double eps2, double &dx, double &dy,
                                                   double &dz) {
    dx = j.x[0] - s.x[0];
    dy = j.x[1] - s.x[1];
    dz = j.x[2] - s.x[2];
    if constexpr (Fold) return fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
    else return fma(dz, dz, fma(dy, dy, dx * dx));
  }

  __device__ static __forceinline__ Key key_of(double r2) { return (Key)__double_as_longlong(r2); }
  // Orders 2 and 4 keep the minimum over a group of sources on the FP64 values (one min per pair
  // instead of a 64-bit compare and two selects); the self pair counts as +inf, and a group with
  // no other source maps to the "none" key.  Orders 6 and 8 keep it on the keys: there the FP64
  // form needs two more registers and the launch would lose half its waves (256 -> 258 per lane).
  static constexpr bool kFloatMin = Order <= 4;
  using GKey = std::conditional_t<kFloatMin, double, Key>;
  __device__ static __forceinline__ GKey gkey_none() {
    if constexpr (kFloatMin) return __builtin_huge_val();
    else return ~Key(0);
  }
  __device__ static __forceinline__ Key group_key(GKey g) {
    if constexpr (kFloatMin) return g < __builtin_huge_val() ? key_of(g) : ~Key(0);
    else return g;
  }
  // the group minimum as a value (+inf or a NaN for an empty group, so that no comparison holds);
  // the neighbour-list test runs once per group on it (tile_compute)
  static constexpr bool kChunkLists = true;
  __device__ static __forceinline__ double group_r2(GKey g) {
    if constexpr (kFloatMin) return g;
    else return __longlong_as_double((long long)g);
  }

  template <bool Nbr>
  __device__ static __forceinline__ double pair_r2(const J &j, const Sink &s, double eps2) {
    double dx, dy, dz;
    return diff_d2<!Nbr>(j, s, eps2, dx, dy, dz);
  }
  template <bool Nbr>
  __device__ static __forceinline__ Key nn_key(const J &j, const Sink &s, double eps2) {
    return key_of(pair_r2<Nbr>(j, s, eps2));
  }

  // One pair; as Mixed::interact.
  template <bool Guard, bool NN, bool Nbr>
  __device__ static __forceinline__ double interact(const J &j, const Sink &s, double eps2, int jidx, int self,
                                                  Comp<double, kValues<Order>> &A, GKey &gmin) {
    double dx, dy, dz;
    const double r2 = diff_d2<!Nbr>(j, s, eps2, dx, dy, dz);
    const double R2 = Nbr ? r2 + eps2 : r2;
    double rinv = rsqrt64(R2);
    if constexpr (Guard) rinv = jidx != self ? rinv : 0.0;
    const double rinv2 = rinv * rinv;
    const double mr = j.m * rinv;
    const double mr3 = mr * rinv2;
    if constexpr (Order == 2) {
      A.part[0] = fma(mr3, dx, A.part[0]);
      A.part[1] = fma(mr3, dy, A.part[1]);
      A.part[2] = fma(mr3, dz, A.part[2]);
      A.part[3] -= mr;
    } else {
      const double dvx = j.v[0] - s.v[0];
      const double dvy = j.v[1] - s.v[1];
      const double dvz = j.v[2] - s.v[2];
      const double rv = fma(dz, dvz, fma(dy, dvy, dx * dvx));
      const double al = rv * rinv2;
      if constexpr (Order == 4) {
        const double am3 = al * -3.0;
        const double wx = fma(am3, dx, dvx);
        const double wy = fma(am3, dy, dvy);
        const double wz = fma(am3, dz, dvz);
        A.part[0] = fma(mr3, dx, A.part[0]);
        A.part[1] = fma(mr3, dy, A.part[1]);
        A.part[2] = fma(mr3, dz, A.part[2]);
        A.part[3] = fma(mr3, wx, A.part[3]);
        A.part[4] = fma(mr3, wy, A.part[4]);
        A.part[5] = fma(mr3, wz, A.part[5]);
        A.part[6] -= mr;
      } else {
        const double dax = j.a[0] - s.a[0];
        const double day = j.a[1] - s.a[1];
        const double daz = j.a[2] - s.a[2];
        const double vv = fma(dvz, dvz, fma(dvy, dvy, dvx * dvx));
        const double ra = fma(dz, daz, fma(dy, day, dx * dax));
        const double be = fma(al, al, (vv + ra) * rinv2);
        const double am3 = al * -3.0;
        const double am6 = al * -6.0;
        const double bm3 = be * -3.0;
        const double a0x = mr3 * dx, a0y = mr3 * dy, a0z = mr3 * dz;
        const double a1x = fma(am3, a0x, mr3 * dvx);
        const double a1y = fma(am3, a0y, mr3 * dvy);
        const double a1z = fma(am3, a0z, mr3 * dvz);
        const double a2x = fma(am6, a1x, fma(bm3, a0x, mr3 * dax));
        const double a2y = fma(am6, a1y, fma(bm3, a0y, mr3 * day));
        const double a2z = fma(am6, a1z, fma(bm3, a0z, mr3 * daz));
        A.part[0] += a0x; A.part[1] += a0y; A.part[2] += a0z;
        A.part[3] += a1x; A.part[4] += a1y; A.part[5] += a1z;
        A.part[6] -= mr;
        A.part[7] += a2x; A.part[8] += a2y; A.part[9] += a2z;
        if constexpr (Order == 8) {
          // crackle: gamma = (3 v.a + r.j) / R^2 + alpha (3 beta - 4 alpha^2),
          // A3 = m j / R^3 - 9 alpha A2 - 9 beta A1 - 3 gamma A0
          const double djx = j.j[0] - s.j[0];
          const double djy = j.j[1] - s.j[1];
          const double djz = j.j[2] - s.j[2];
          const double va = fma(dvz, daz, fma(dvy, day, dvx * dax));
          const double rj = fma(dz, djz, fma(dy, djy, dx * djx));
          const double ga = fma(fma(3.0, va, rj), rinv2, al * fma(-4.0 * al, al, 3.0 * be));
          const double am9 = al * -9.0;
          const double bm9 = be * -9.0;
          const double gm3 = ga * -3.0;
          A.part[10] += fma(am9, a2x, fma(bm9, a1x, fma(gm3, a0x, mr3 * djx)));
          A.part[11] += fma(am9, a2y, fma(bm9, a1y, fma(gm3, a0y, mr3 * djy)));
          A.part[12] += fma(am9, a2z, fma(bm9, a1z, fma(gm3, a0z, mr3 * djz)));
        }
      }
    }
    if constexpr (!NN) {
      // no nearest-neighbour search
    } else if constexpr (kFloatMin) {
      double gk = r2;
      if constexpr (Guard) gk = jidx != self ? gk : __builtin_huge_val();
      gmin = fmin(gk, gmin);
    } else {
      Key key = key_of(r2);
      if constexpr (Guard) key = jidx != self ? key : ~Key(0);
      gmin = key < gmin ? key : gmin;
    }
    return r2;
  }
};


// ---------------------------------------------------------------------------------------------
// Double-single arithmetic (the paper's DS precision: a value is an unevaluated sum hi + lo of
// two FP32 numbers, |lo| <= ulp(hi)/2, about 48 significant bits; Background, footnote on the
// Yebisu library).  Error-free transformations: Knuth's TwoSum, Dekker's FastTwoSum (|a| >= |b|),
// and the FMA product error; every operation renormalises.  Contraction is off inside each of
// them so that the compiler keeps every rounding where it is written.
// ---------------------------------------------------------------------------------------------
struct dsf {
  float hi, lo;
};

__device__ __forceinline__ dsf ds_of(double x) {
  const float h = (float)x;
  return {h, (float)(x - (double)h)};
}
__device__ __forceinline__ double ds_to_double(dsf a) { return (double)a.hi + (double)a.lo; }  // exact

__device__ __forceinline__ dsf ds_fast_two_sum(float a, float b) {
#pragma clang fp contract(off)
  const float s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ dsf ds_two_sum(float a, float b) {
#pragma clang fp contract(off)
  const float s = a + b;
  const float bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dsf ds_add(dsf a, dsf b) {
#pragma clang fp contract(off)
  const dsf s = ds_two_sum(a.hi, b.hi);
  return ds_fast_two_sum(s.hi, s.lo + (a.lo + b.lo));
}
__device__ __forceinline__ dsf ds_neg(dsf a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dsf ds_sub(dsf a, dsf b) { return ds_add(a, ds_neg(b)); }
__device__ __forceinline__ dsf ds_mul(dsf a, dsf b) {
#pragma clang fp contract(off)
  const float p = a.hi * b.hi;
  float e = __builtin_fmaf(a.hi, b.hi, -p);
  e = __builtin_fmaf(a.hi, b.lo, __builtin_fmaf(a.lo, b.hi, e));
  return ds_fast_two_sum(p, e);
}
__device__ __forceinline__ dsf ds_mulf(dsf a, float f) {  // by an FP32 number (exact small constants)
#pragma clang fp contract(off)
  const float p = a.hi * f;
  const float e = __builtin_fmaf(a.lo, f, __builtin_fmaf(a.hi, f, -p));
  return ds_fast_two_sum(p, e);
}
__device__ __forceinline__ dsf ds_sqr(dsf a) {
#pragma clang fp contract(off)
  const float p = a.hi * a.hi;
  const float e = __builtin_fmaf(a.hi + a.hi, a.lo, __builtin_fmaf(a.hi, a.hi, -p));
  return ds_fast_two_sum(p, e);
}
__device__ __forceinline__ dsf ds_dot3(const dsf a[3], const dsf b[3]) {
  return ds_add(ds_add(ds_mul(a[0], b[0]), ds_mul(a[1], b[1])), ds_mul(a[2], b[2]));
}
// 1/sqrt(x): the hardware estimate y (about 1 ulp of FP32) and one Newton step evaluated in DS,
// y1 = y + y (1 - x y^2) / 2, whose error is about (3/2) (2^-23)^2, below the DS rounding.
__device__ __forceinline__ dsf ds_rsqrt(dsf x) {
#pragma clang fp contract(off)
  const float y = __builtin_amdgcn_rsqf(x.hi);
  const dsf yy = ds_fast_two_sum(y * y, __builtin_fmaf(y, y, -(y * y)));
  const dsf d = ds_sub(dsf{1.0f, 0.0f}, ds_mul(x, yy));  // small: |d| ~ 2^-22
  const float c = 0.5f * y * d.hi;
  return ds_add(dsf{y, 0.0f}, ds_fast_two_sum(c, __builtin_fmaf(0.5f * y, d.hi, -c)));
}

template <int Order>
struct DSTile;
template <>
struct DSTile<4> {   // 56 B per source
  float4 t0[kTile];  // x.hi m.hi
  float4 t1[kTile];  // x.lo m.lo
  float4 t2[kTile];  // v.hi vx.lo
  float2 t3[kTile];  // vy.lo vz.lo
};
template <>
struct DSTile<6> {   // 80 B per source
  float4 t0[kTile];  // x.hi m.hi
  float4 t1[kTile];  // x.lo m.lo
  float4 t2[kTile];  // v.hi vx.lo
  float2 t3[kTile];  // vy.lo vz.lo
  float4 t4[kTile];  // a.hi ax.lo
  float2 t5[kTile];  // ay.lo az.lo
};

// DS precision (orders 4 and 6): every pair quantity in double-single arithmetic from the FP64
// predicted state; the pair terms convert exactly to FP64 and sum in FP64 chunks folded with
// TwoSum (as the FP64 kernels do).  R^-1 from the hardware estimate refined once in DS.
template <int Order>
struct DS {
  static_assert(Order == 4 || Order == 6, "double-single arithmetic is built for orders 4 and 6");
  using Real = double;  // sums, eps2 and list radii
  using Key = uint32_t;
  static constexpr int kK = kValues<Order>;
  static constexpr int kLongChunk = kChunk;
  using Tile = DSTile<Order>;
  struct Sink {
    dsf x[3], v[3], a[3];
    int64_t id;
  };
  struct J {
    dsf x[3], m, v[3], a[3];
  };

  __device__ static __forceinline__ Sink sink_from_j(const J &j) {
    Sink s;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s.x[k] = j.x[k];
      s.v[k] = j.v[k];
      s.a[k] = j.a[k];
    }
    s.id = -1;
    return s;
  }
  __device__ static __forceinline__ Sink make_sink(const double xp[3], const double vp[3], const double ap[6],
                                                   double) {
    Sink s;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s.x[k] = ds_of(xp[k]);
      s.v[k] = ds_of(vp[k]);
      s.a[k] = ds_of(ap[k]);
    }
    s.id = -1;
    return s;
  }
  __device__ static __forceinline__ J make_j(const double xp[3], const double vp[3], const double ap[6], double m) {
    J j;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      j.x[k] = ds_of(xp[k]);
      j.v[k] = ds_of(vp[k]);
      j.a[k] = ds_of(ap[k]);
    }
    j.m = ds_of(m);
    return j;
  }
  __device__ static __forceinline__ void store(Tile &tl, int e, const double xp[3], const double vp[3],
                                               const double ap[6], double m) {
    const J j = make_j(xp, vp, ap, m);
    tl.t0[e] = make_float4(j.x[0].hi, j.x[1].hi, j.x[2].hi, j.m.hi);
    tl.t1[e] = make_float4(j.x[0].lo, j.x[1].lo, j.x[2].lo, j.m.lo);
    tl.t2[e] = make_float4(j.v[0].hi, j.v[1].hi, j.v[2].hi, j.v[0].lo);
    tl.t3[e] = make_float2(j.v[1].lo, j.v[2].lo);
    if constexpr (Order == 6) {
      tl.t4[e] = make_float4(j.a[0].hi, j.a[1].hi, j.a[2].hi, j.a[0].lo);
      tl.t5[e] = make_float2(j.a[1].lo, j.a[2].lo);
    }
  }
  __device__ static __forceinline__ J load(const Tile &tl, int e) {
    J j;
    const float4 a = tl.t0[e], b = tl.t1[e], c = tl.t2[e];
    const float2 d = tl.t3[e];
    j.x[0] = {a.x, b.x};
    j.x[1] = {a.y, b.y};
    j.x[2] = {a.z, b.z};
    j.m = {a.w, b.w};
    j.v[0] = {c.x, c.w};
    j.v[1] = {c.y, d.x};
    j.v[2] = {c.z, d.y};
    if constexpr (Order == 6) {
      const float4 f = tl.t4[e];
      const float2 g = tl.t5[e];
      j.a[0] = {f.x, f.w};
      j.a[1] = {f.y, g.x};
      j.a[2] = {f.z, g.y};
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k) j.a[k] = {0.0f, 0.0f};
    }
    return j;
  }

  // Unsoftened |r|^2 in DS (the nearest-neighbour key is taken on its leading part).
  __device__ static __forceinline__ dsf diff_r2(const J &j, const Sink &s, dsf (&d)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = ds_sub(j.x[k], s.x[k]);
    return ds_add(ds_add(ds_sqr(d[0]), ds_sqr(d[1])), ds_sqr(d[2]));
  }
  __device__ static __forceinline__ Key key_of(float r2) { return __float_as_uint(r2); }
  using GKey = Key;
  __device__ static __forceinline__ GKey gkey_none() { return ~Key(0); }
  __device__ static __forceinline__ Key group_key(GKey g) { return g; }
  // the key is the leading FP32 part of |r|^2 while the list test takes its FP64 value: lists keep
  // the test per pair
  static constexpr bool kChunkLists = false;
  template <bool Nbr>
  __device__ static __forceinline__ Key nn_key(const J &j, const Sink &s, double) {
    dsf d[3];
    return key_of(diff_r2(j, s, d).hi);
  }

  // One pair; returns the unsoftened |r|^2 (its FP64 value) for the neighbour-list test.
  template <bool Guard, bool NN, bool Nbr>
  __device__ static __forceinline__ double interact(const J &j, const Sink &s, double eps2, int jidx, int self,
                                                  Comp<double, kValues<Order>> &A, GKey &gmin) {
    dsf d[3], w[3];
    const dsf r2 = diff_r2(j, s, d);
    dsf rinv = ds_rsqrt(ds_add(r2, ds_of(eps2)));
    if constexpr (Guard) {
      if (jidx == self) rinv = {0.0f, 0.0f};
    }
    const dsf rinv2 = ds_sqr(rinv);
    const dsf mr = ds_mul(j.m, rinv);
    const dsf mr3 = ds_mul(mr, rinv2);
#pragma unroll
    for (int k = 0; k < 3; ++k) w[k] = ds_sub(j.v[k], s.v[k]);
    const dsf al = ds_mul(ds_dot3(d, w), rinv2);
    dsf a0[3], a1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a0[k] = ds_mul(mr3, d[k]);
      a1[k] = ds_add(ds_mul(mr3, w[k]), ds_mul(ds_mulf(al, -3.0f), a0[k]));
      A.part[k] += ds_to_double(a0[k]);
      A.part[3 + k] += ds_to_double(a1[k]);
    }
    A.part[6] -= ds_to_double(mr);
    if constexpr (Order == 6) {
      dsf u[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) u[k] = ds_sub(j.a[k], s.a[k]);
      const dsf be = ds_add(ds_mul(ds_add(ds_dot3(w, w), ds_dot3(d, u)), rinv2), ds_sqr(al));
      const dsf am6 = ds_mulf(al, -6.0f), bm3 = ds_mulf(be, -3.0f);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const dsf a2 = ds_add(ds_add(ds_mul(mr3, u[k]), ds_mul(am6, a1[k])), ds_mul(bm3, a0[k]));
        A.part[7 + k] += ds_to_double(a2);
      }
    }
    if constexpr (NN) {
      Key key = key_of(r2.hi);
      if constexpr (Guard) key = jidx != self ? key : ~Key(0);
      gmin = key < gmin ? key : gmin;
    }
    return ds_to_double(r2);
  }
};

template <int Order, int Prec>
struct TraitsSel;
template <int Order>
struct TraitsSel<Order, NBX_MIXED> {
  using type = Mixed<Order>;
};
template <int Order>
struct TraitsSel<Order, NBX_FP64> {
  using type = F64<Order>;
};
template <int Order>
struct TraitsSel<Order, NBX_DS> {
  using type = DS<Order>;
};

// ---------------------------------------------------------------------------------------------
// Deterministic reduction over contiguous groups of `gs` threads (power of two, <= 256):
// butterfly inside each wave (every lane ends with the same bits), then, for groups spanning
// several waves, a sum in wave order through LDS.  Must be called by the whole workgroup.
// NN candidates combine lexicographically on (key, index) with index compared unsigned.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ bool nn_better(uint64_t k1, int i1, uint64_t k2, int i2) {
  return k1 < k2 || (k1 == k2 && (unsigned)i1 < (unsigned)i2);
}

// Butterfly exchange in VALU (DPP and the row / half-wave swaps) instead of LDS-routed permutes:
// stage Off returns the value of the partner lane, lane ^ 1 and lane ^ 2 (quad permutes),
// lane ^ 7 (half-row mirror), lane ^ 15 (row mirror), lane ^ 16 and lane ^ 32 (swaps).  Stages run
// in increasing order over aligned groups of contiguous lanes: before stage Off every aligned group
// of Off lanes holds equal values, so the mirror partners stand for the xor partners, and each pair
// adds a + b on one side and b + a on the other, which IEEE addition makes the same bits.
template <int Off>
__device__ __forceinline__ uint32_t lane_xchg32(uint32_t v) {
  if constexpr (Off == 1) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (Off == 2) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else if constexpr (Off == 4) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  } else if constexpr (Off == 8) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);  // row_mirror
  } else if constexpr (Off == 16) {
    const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);  // [0]: even rows, [1]: odd
    return ((threadIdx.x >> 4) & 1) ? p[0] : p[1];
  } else {
    static_assert(Off == 32, "butterfly stages are 1, 2, 4, 8, 16, 32");
    const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);  // [0]: low half, [1]: high
    return (threadIdx.x & 32) ? p[0] : p[1];
  }
}

template <int Off>
__device__ __forceinline__ uint64_t lane_xchg64(uint64_t v) {
  return ((uint64_t)lane_xchg32<Off>((uint32_t)(v >> 32)) << 32) | lane_xchg32<Off>((uint32_t)v);
}

template <int Off, int P, int K, bool NN>
__device__ __forceinline__ void lane_stage(double (&v)[P][K], uint64_t (&kk)[P], int (&ii)[P]) {
#pragma unroll
  for (int p = 0; p < P; ++p) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint64_t bits = (uint64_t)__double_as_longlong(v[p][k]);
      v[p][k] += __longlong_as_double((long long)lane_xchg64<Off>(bits));
    }
    if constexpr (NN) {
      const uint64_t ok = lane_xchg64<Off>(kk[p]);
      const int oi = (int)lane_xchg32<Off>((uint32_t)ii[p]);
      if (nn_better(ok, oi, kk[p], ii[p])) {
        kk[p] = ok;
        ii[p] = oi;
      }
    }
  }
}

// Reduction over aligned groups of `width` contiguous lanes (a power of two, <= 64).
template <int P, int K, bool NN>
__device__ __forceinline__ void lane_butterfly(int width, double (&v)[P][K], uint64_t (&kk)[P], int (&ii)[P]) {
  if (width > 1) lane_stage<1, P, K, NN>(v, kk, ii);
  if (width > 2) lane_stage<2, P, K, NN>(v, kk, ii);
  if (width > 4) lane_stage<4, P, K, NN>(v, kk, ii);
  if (width > 8) lane_stage<8, P, K, NN>(v, kk, ii);
  if (width > 16) lane_stage<16, P, K, NN>(v, kk, ii);
  if (width > 32) lane_stage<32, P, K, NN>(v, kk, ii);
}

template <int P, int K>
struct RedLds {
  double v[4][P][K];
  uint64_t k[4][P];
  int i[4][P];
};

template <int P, int K, bool NN = true, bool Valu = true>
__device__ __forceinline__ void group_reduce(int gs, double (&v)[P][K], uint64_t (&kk)[P], int (&ii)[P],
                                             RedLds<P, K> &red) {
  const int wl = gs < 64 ? gs : 64;
  if constexpr (Valu) {
    lane_butterfly<P, K, NN>(wl, v, kk, ii);
  } else {  // the same butterfly through LDS-routed permutes, largest offset first
    for (int off = wl >> 1; off > 0; off >>= 1) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[p][k] += __shfl_xor(v[p][k], off);
        if constexpr (NN) {
          const uint64_t ok = __shfl_xor(kk[p], off);
          const int oi = __shfl_xor(ii[p], off);
          if (nn_better(ok, oi, kk[p], ii[p])) {
            kk[p] = ok;
            ii[p] = oi;
          }
        }
      }
    }
  }
  if (gs > 64) {
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int k = 0; k < K; ++k) red.v[wave][p][k] = v[p][k];
        red.k[wave][p] = kk[p];
        red.i[wave][p] = ii[p];
      }
    }
    __syncthreads();
    const int wpg = gs >> 6;
    const int w0 = (wave / wpg) * wpg;
#pragma unroll
    for (int p = 0; p < P; ++p) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        double s = red.v[w0][p][k];
        for (int w = 1; w < wpg; ++w) s += red.v[w0 + w][p][k];
        v[p][k] = s;
      }
      if constexpr (NN) {
        uint64_t bk = red.k[w0][p];
        int bi = red.i[w0][p];
        for (int w = 1; w < wpg; ++w) {
          if (nn_better(red.k[w0 + w][p], red.i[w0 + w][p], bk, bi)) {
            bk = red.k[w0 + w][p];
            bi = red.i[w0 + w][p];
          }
        }
        kk[p] = bk;
        ii[p] = bi;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// Exact FP64 |r|^2 between sink q and source idx (inf when idx is no source): the sink is its own
// predicted source addr, or its explicit position, or the position xi_pre the caller already has
// (the same bits: the gravity kernel's set-up predicted it with this predictor).  Same predictor
// as the staging, so the value is the one the oracle computes from the predicted positions.
// ---------------------------------------------------------------------------------------------
template <int Order>
__device__ double nn_exact_r2(const ForceParams &fp, int q, int addr, int idx, const double *xi_pre) {
  if (idx < 0 || idx >= fp.nj) return __builtin_huge_val();
  double xi[3], vi[3], ai[6], mi, xj[3], vj[3], aj[6], mj;
  if (xi_pre) {
#pragma unroll
    for (int k = 0; k < 3; ++k) xi[k] = xi_pre[k];
  } else if (fp.ext_x) {
#pragma unroll
    for (int k = 0; k < 3; ++k) xi[k] = fp.ext_x[3 * (size_t)q + k];
  } else {
    predict_addr<Order>(fp.src, addr, fp.t, xi, vi, ai, mi);
  }
  predict_addr<Order>(fp.src, idx, fp.t, xj, vj, aj, mj);
  {
#pragma clang fp contract(off)
    const double dx = xj[0] - xi[0], dy = xj[1] - xi[1], dz = xj[2] - xi[2];
    return dx * dx + dy * dy + dz * dz;
  }
}

// Final write of one sink: results, nearest neighbour id and its exact FP64 |r|^2 (xi: the sink's
// predicted position when the caller has it, else null).
template <int Order, bool NN = true>
__device__ void finalize_sink(const ForceParams &fp, int q, const double *v, int idx, const double *xi) {
  const bool ext = fp.ext_x != nullptr;
  const int addr = ext ? -1 : fp.i_addr[q];
  if (!ext && (addr < 0 || addr >= fp.nj)) {
    atomicAdd(&fp.err[0], 1);
    return;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    fp.acc[3 * (size_t)q + k] = v[k];
    if constexpr (Order != 2) fp.jrk[3 * (size_t)q + k] = v[3 + k];
    if constexpr (Order >= 6) fp.snp[3 * (size_t)q + k] = v[7 + k];
    if constexpr (Order == 8) fp.crk[3 * (size_t)q + k] = v[10 + k];
  }
  fp.pot[q] = v[kPotSlot<Order>];
  if constexpr (!NN) return;  // the nearest-neighbour outputs are left untouched
  if (idx >= 0 && idx < fp.nj) {
    fp.nn_id[q] = fp.src.id[idx];
    fp.nn_r2[q] = nn_exact_r2<Order>(fp, q, addr, idx, xi);
  } else {
    fp.nn_id[q] = -1;
    fp.nn_r2[q] = __builtin_huge_val();
  }
}

// One LDS tile against the lane's P sinks.  Guard = true is used only for tiles that hold the
// own source of some sink of the wave: there R^-1 is forced to 0 for j == self, so the self pair
// adds exact zeros everywhere and its nearest-neighbour key is the maximum.
// The lane's sources are taken in groups of one chunk (kChunkAcc, or Tr::kLongChunk with Long);
// the acceleration sums fold after each group, the others every kChunk.  Inside a group only the minimum
// nearest-neighbour key is kept, and after the group the (key, first source of the group) pair
// replaces the running best if the key is smaller.  The exact source is found afterwards by
// re-scanning that one group (nn_rescan).  L1: one lane per sink (compile-time offsets).
// Nbr: neighbour lists; each source with |r|^2 < h2 (strict, never the sink's own source, never
// padding) is appended to the sink's list through an atomic counter.  Sinks without a list slot
// carry h2 = -1 and never append.  NN = false: no nearest-neighbour search (no keys, no groups).
__device__ __forceinline__ void nbr_append(const ForceParams &fp, int q, int jj) {
  const int k = atomicAdd(&fp.nbr_count[q], 1);
  if (k < fp.nbr_max) fp.nbr_ids[(size_t)q * fp.nbr_max + k] = fp.src.id[jj];
}

template <class Tr, int P, bool Guard, bool L1, bool Nbr, bool NN, bool Long>
__device__ __forceinline__ void tile_compute(const ForceParams &fp, const typename Tr::Tile &tl, int slot, int lg,
                                             int jb, const typename Tr::Sink (&sink)[P], const int (&self)[P],
                                             const int (&q)[P], const typename Tr::Real (&h2)[P],
                                             typename Tr::Real eps2,
                                             Comp<typename Tr::Real, Tr::kK> (&acc)[P],
                                             typename Tr::Key (&nnk)[P], int (&nng)[P]) {
  using Key = typename Tr::Key;
  // lists: the test r^2 < h^2 runs once per group on the group's minimum |r|^2 (which the search
  // keeps anyway), and only a group whose minimum passes is scanned again, with the same
  // arithmetic, for its members; the pair loop carries no branch and no atomic
  constexpr bool kChunkNbr = Nbr && Tr::kChunkLists;
  constexpr bool kMin = NN || kChunkNbr;  // the group keeps its minimum
  const int per = L1 ? kTile : kTile >> lg;
  constexpr int kCA = Long ? Tr::kLongChunk : kChunkAcc;
  for (int c = 0; c < per; c += kCA) {
    const int ce = per < c + kCA ? per : c + kCA;
    typename Tr::GKey gmin[P];
#pragma unroll
    for (int p = 0; p < P; ++p) gmin[p] = Tr::gkey_none();
#pragma unroll 2
    for (int u = c; u < ce; ++u) {
      const int e = L1 ? u : slot + (u << lg);
      const typename Tr::J j = Tr::load(tl, e);
      const int jidx = L1 ? jb + u : jb + (u << lg);
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const typename Tr::Real r2 =
            Tr::template interact<Guard, kMin, Nbr>(j, sink[p], eps2, jidx, self[p], acc[p], gmin[p]);
        if constexpr (Nbr && !kChunkNbr) {
          if (r2 < h2[p] && jidx < fp.nj && (!Guard || jidx != self[p])) nbr_append(fp, q[p], jidx);
        }
      }
    }
    if constexpr (kChunkNbr) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        if (Tr::group_r2(gmin[p]) < h2[p]) {  // some source of the group may lie within h
          for (int u = c; u < ce; ++u) {
            const int e = L1 ? u : slot + (u << lg);
            const int jidx = L1 ? jb + u : jb + (u << lg);
            const typename Tr::Real r2 = Tr::template pair_r2<true>(Tr::load(tl, e), sink[p], eps2);
            if (r2 < h2[p] && jidx < fp.nj && (!Guard || jidx != self[p])) nbr_append(fp, q[p], jidx);
          }
        }
      }
    }
    if constexpr (NN) {
      const int g0 = L1 ? jb + c : jb + (c << lg);
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const Key gk = Tr::group_key(gmin[p]);
        if (gk < nnk[p]) {
          nnk[p] = gk;
          nng[p] = g0;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) acc[p].template fold<0, 3>();
    if (ce == per || (ce % kChunk) == 0) {
#pragma unroll
      for (int p = 0; p < P; ++p) acc[p].template fold<3, Tr::kK>();
    }
  }
}

// Source record of address j exactly as staged by the gravity kernel (padding beyond nj).
template <class Tr, int Order>
__device__ __forceinline__ typename Tr::J staged_j(const ForceParams &fp, int jj) {
  double xp[3], vp[3], ap[6], m;
  if (jj < fp.nj) {
    predict_addr<Order>(fp.src, jj, fp.t, xp, vp, ap, m);
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      xp[k] = kPadPos;
      vp[k] = 0.0;
      ap[k] = 0.0;
      ap[3 + k] = 0.0;
    }
    m = 0.0;
  }
  return Tr::make_j(xp, vp, ap, m);
}

// Find the first source of the winning group whose key equals the best key (the group start g0
// and lane stride L identify the group; its length is min(chunk, 256 / L)).
// When the group lies in the tile still resident in LDS after the loop (the workgroup's last
// tile: always the case when a workgroup has one tile, i.e. at small and medium N_i), its records
// are read back from LDS; otherwise they are staged again from global memory.  Either way they are
// the records the loop used, so the keys match bit for bit.  With four or more lanes per sink
// (N_i <= 256: one tile per workgroup, read back from LDS) every source of the group is tested,
// last to first, and the earliest match survives: no early exit, so the reads of several sources
// are in flight together.  With fewer lanes per sink the extra bank-conflicted reads of that form
// slow the waves still in their loops (measured 6% slower at N_i = 512, two lanes per sink), so
// there, and for groups staged again from global memory, the scan stops at the first match.
template <class Tr, int Order, bool Nbr, bool Long, bool L1>
__device__ __forceinline__ int nn_rescan(const ForceParams &fp, const typename Tr::Tile &last, int last_tile,
                                         const typename Tr::Sink &s, typename Tr::Key key, int g0, int lg,
                                         int self, typename Tr::Real eps2) {
  if (g0 < 0) return -1;
  const int per = kTile >> lg;
  constexpr int kCA = Long ? Tr::kLongChunk : kChunkAcc;
  const int len = per < kCA ? per : kCA;
  if ((g0 >> 8) == last_tile) {  // kTile == 256
    if (!L1 && lg >= 2) {
      int found = -1;
#pragma unroll 8
      for (int k = len - 1; k >= 0; --k) {
        const int jj = g0 + (k << lg);
        const bool hit = Tr::template nn_key<Nbr>(Tr::load(last, jj & (kTile - 1)), s, eps2) == key;
        found = (hit && jj != self) ? jj : found;
      }
      return found;
    }
    for (int k = 0; k < len; ++k) {
      const int jj = g0 + (k << lg);
      if (jj != self && Tr::template nn_key<Nbr>(Tr::load(last, jj & (kTile - 1)), s, eps2) == key) return jj;
    }
    return -1;
  }
  for (int k = 0; k < len; ++k) {
    const int jj = g0 + (k << lg);
    if (jj != self && Tr::template nn_key<Nbr>(staged_j<Tr, Order>(fp, jj), s, eps2) == key) return jj;
  }
  return -1;  // not reached: the group's minimum key comes from one of its sources
}

// ---------------------------------------------------------------------------------------------
// The gravity kernel.  Grid: blocks * S workgroups; workgroup w handles sink block w / S and
// source split w % S (split-fastest, so with S a multiple of 8 every split stays on one XCD and
// its sources stay in that XCD's L2).
// ---------------------------------------------------------------------------------------------
// Waves per SIMD the FP64 gravity kernel with one sink per lane is held to: order 6 with
// neighbour lists needs 258-286 registers per lane and order 8 326-380, which leaves one wave per
// SIMD; capped at 256 (two waves) they spill a few values instead.  Order 4 needs 176-204 (two
// waves); capped at 168 it runs three.  Measured with old and new library alternating on one box:
// faster for orders 4 and 6 at every N_i timed; for order 8 faster with one lane per sink (N_i >=
// 1024) but slower with several lanes per sink at N_i <= 64, where each workgroup runs one tile
// and the spills of its set-up and reduction are not amortised, so order 8 caps only the former.
// The mixed 4th-order kernel with two sinks per lane (the many-sink case) takes 156-176 registers
// (three waves, two with lists and search); capped at 128 it runs four, its spills stay out of the
// pair loops, and it ran 5% faster at N_i = 65536 and 131072.  The same cap on the 6th-order one
// (three waves instead of two) gained nothing.  The other mixed kernels keep the compiler's choice.
template <int Order, int Prec, int P, bool L1>
constexpr int kForceWaves =
    (Prec == NBX_MIXED && P == 2 && Order == 4)
        ? 4
        : (Prec != NBX_FP64 || P != 1 || (Order == 8 && !L1)) ? 1 : (Order >= 6 ? 2 : (Order == 4 ? 3 : 1));

// Index of value k (of nv per sink) of split s for sink q in the split-partial arrays: split-major
// (the partials of one split and value are contiguous over the sinks: coalesced for many sinks)
// or, with part_sm, sink-major (the splits of one sink and value are contiguous: coalesced when
// the combine gives each sink a whole workgroup, at small N_i).
__device__ __forceinline__ size_t part_at(const ForceParams &fp, int s, int k, int q, int nv) {
  return fp.part_sm ? ((size_t)q * nv + k) * fp.splits + s : ((size_t)s * nv + k) * fp.ni + q;
}

// One work item of the gravity kernel: sink block w / S against source split w % S.  Run by the
// whole workgroup; tiles and red are its LDS.
template <int Order, int Prec, int P, bool L1, bool Nbr, bool NN, bool Long>
__device__ __forceinline__ void force_item(const ForceParams &fp, int w,
                                           typename TraitsSel<Order, Prec>::type::Tile (&tiles)[2],
                                           RedLds<P, kValues<Order>> &red) {
  using Tr = typename TraitsSel<Order, Prec>::type;
  using T = typename Tr::Real;
  using Key = typename Tr::Key;
  constexpr int K = kValues<Order>;

  const int tid = threadIdx.x;
  const int lg = fp.lanes_log2;
  const int L = 1 << lg;
  const int G = kThreads >> lg;
  const int slot = tid & (L - 1);
  const int grp = tid >> lg;
  const int S = fp.splits;
  const int split = w % S;
  const int ib = w / S;
  const int Q = G * P;
  const int ntiles = fp.nj_pad / kTile;
  const int t0 = (int)(((int64_t)split * ntiles) / S);
  const int t1 = (int)(((int64_t)(split + 1) * ntiles) / S);

  // Tile staging with the fused predictor.  Addresses >= nj (the tail of the last tile) get a
  // padding source: massless, at rest, at (kPadPos, kPadPos, kPadPos); all its terms are exact
  // zeros in both precisions and its address marks "no neighbour".
  auto stage = [&](int tile, int buf) {
    const int jj = tile * kTile + tid;
    double xp[3], vp[3], ap[6], m;
    if (jj < fp.nj) {
      predict_addr<Order>(fp.src, jj, fp.t, xp, vp, ap, m);
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        xp[k] = kPadPos;
        vp[k] = 0.0;
        ap[k] = 0.0;
        ap[3 + k] = 0.0;
      }
      m = 0.0;
    }
    Tr::store(tiles[buf], tid, xp, vp, ap, m);
  };

  // the first tile's loads go out before the sink set-up's (an address, then the sink's state),
  // so that the two latencies overlap
  if (t0 < t1) stage(t0, 0);
  typename Tr::Sink sink[P];
  Comp<T, K> acc[P];
  Key nnk[P];
  int nng[P];  // first source of the group holding the best key (-1: none yet)
  int q[P];
  int self[P];  // own source address of each sink (-1: none, or no sink in this slot)
  T h2[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    q[p] = ib * Q + p * G + grp;
    const bool live = q[p] < fp.ni;
    double xp[3], vp[3], ap[6], m = 0.0;
    if (fp.ext_x) {  // explicit sink state, used as given
      const int qq = live ? q[p] : 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        xp[k] = fp.ext_x[3 * (size_t)qq + k];
        vp[k] = (Order != 2) ? fp.ext_v[3 * (size_t)qq + k] : 0.0;
        ap[k] = (Order >= 6) ? fp.ext_a[3 * (size_t)qq + k] : 0.0;
        ap[3 + k] = (Order == 8) ? fp.ext_j[3 * (size_t)qq + k] : 0.0;
      }
      self[p] = live ? fp.ext_self[qq] : -1;
    } else {  // by address: the sink's own predicted source state
      int addr = live ? fp.i_addr[q[p]] : -1;
      if (addr < 0 || addr >= fp.nj) addr = -1;  // bad addresses are reported by finalize_sink
      self[p] = addr;
      predict_addr<Order>(fp.src, addr < 0 ? 0 : addr, fp.t, xp, vp, ap, m);
    }
    if constexpr (NN) {  // the combine's exact |r|^2 reads the sink's position from here
      if (fp.part_xi && split == 0 && slot == 0 && live) {
#pragma unroll
        for (int k = 0; k < 3; ++k) fp.part_xi[3 * (size_t)q[p] + k] = xp[k];
      }
    }
    sink[p] = Tr::make_sink(xp, vp, ap, m);
    h2[p] = (Nbr && live) ? (T)fp.h2[q[p]] : T(-1);
    acc[p].init();
    nnk[p] = ~Key(0);
    nng[p] = -1;
  }
  const T eps2 = (T)fp.eps2;

  __syncthreads();
  for (int tile = t0; tile < t1; ++tile) {
    const int buf = (tile - t0) & 1;
    bool mine = false;
#pragma unroll
    for (int p = 0; p < P; ++p) mine |= (self[p] >> 8) == tile;  // kTile == 256
    if (__any(mine))
      tile_compute<Tr, P, true, L1, Nbr, NN, Long>(fp, tiles[buf], slot, lg, tile * kTile + slot, sink, self, q, h2,
                                                   eps2, acc, nnk, nng);
    else
      tile_compute<Tr, P, false, L1, Nbr, NN, Long>(fp, tiles[buf], slot, lg, tile * kTile + slot, sink, self, q, h2,
                                                    eps2, acc, nnk, nng);
    if (tile + 1 < t1) stage(tile + 1, buf ^ 1);
    __syncthreads();
  }

  // exact nearest-neighbour source of each lane, then lanes of a sink -> one value (identical in
  // every lane of the group)
  double v[P][K];
  uint64_t kk[P];
  int ii[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[p][k] = acc[p].value(k);
    kk[p] = (uint64_t)nnk[p];
    ii[p] = NN ? nn_rescan<Tr, Order, Nbr, Long, L1>(fp, tiles[(t1 - 1 - t0) & 1], t1 - 1, sink[p], nnk[p], nng[p],
                                                     lg, self[p], eps2)
               : -1;
  }
  // the kernels with one lane per sink never combine lanes (L = 1) but keep the permute form of
  // the call: without it, or with the VALU form, the compiler placed the spills of the 128-register
  // many-sink kernel differently and that kernel ran 2.7-4.4% slower at N_i = 131072
  group_reduce<P, K, NN, !L1>(L, v, kk, ii, red);

  if (S == 1) {
    if (slot == 0) {
#pragma unroll
      for (int p = 0; p < P; ++p)
        if (q[p] < fp.ni) finalize_sink<Order, NN>(fp, q[p], v[p], ii[p], nullptr);
    }
    return;
  }

  // S > 1: publish this split's partials; k_combine sums them in a fixed order.
  if (slot == 0) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      if (q[p] < fp.ni) {
#pragma unroll
        for (int k = 0; k < K; ++k) fp.part[part_at(fp, split, k, q[p], K)] = v[p][k];
        if constexpr (NN) {
          fp.part_key[part_at(fp, split, 0, q[p], 1)] = kk[p];
          fp.part_idx[part_at(fp, split, 0, q[p], 1)] = ii[p];
        }
      }
    }
  }
}

template <int Order, int Prec, int P, bool L1, bool Nbr, bool NN, bool Long>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kForceWaves<Order, Prec, P, L1>)))
void k_force(const ForceParams fp) {
  __shared__ typename TraitsSel<Order, Prec>::type::Tile tiles[2];
  __shared__ RedLds<P, kValues<Order>> red;
  force_item<Order, Prec, P, L1, Nbr, NN, Long>(fp, blockIdx.x, tiles, red);
}

// Launch shape of a device-driven block step for ni sinks: lanes per sink and splits from the
// per-class table (class k: ni in (2^(k-1), 2^k]), sink blocks of 256 / L sinks.
__device__ __forceinline__ void dd_shape(const ForceParams &fp, int ni, int &lg, int &S, int &blocks) {
  int k = 0;
  while ((1 << k) < ni && k < 31) ++k;
  lg = fp.dd_shape[k].x;
  S = fp.dd_shape[k].y;
  blocks = (ni + (kThreads >> lg) - 1) / (kThreads >> lg);
}

// Device-driven block step (the integrator's run loop): the number of active sinks and the
// prediction time are read from device memory, which the scheduling kernel just wrote, so that
// the host enqueues many block steps without waiting for each schedule.  Several lanes per sink
// (runtime L, one sink per lane), no lists, no nearest neighbour; the workgroups loop over the
// work items.
template <int Order, int Prec>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kForceWaves<Order, Prec, 1, false>)))
void k_force_dd(const ForceParams fp0) {
  __shared__ typename TraitsSel<Order, Prec>::type::Tile tiles[2];
  __shared__ RedLds<1, kValues<Order>> red;
  const int ni = *fp0.dd_count;
  if (ni <= 0) return;
  ForceParams fp = fp0;
  fp.ni = ni;
  fp.t = *fp0.dd_t;
  int blocks = 0;
  dd_shape(fp0, ni, fp.lanes_log2, fp.splits, blocks);
  const int items = blocks * fp.splits;
  for (int w = blockIdx.x; w < items; w += gridDim.x) {
    force_item<Order, Prec, 1, false, false, false, false>(fp, w, tiles, red);
    __syncthreads();  // the next item restages the tiles
  }
}

// ---------------------------------------------------------------------------------------------
// Combine kernel for S > 1: a workgroup takes W = 2^wlog consecutive sinks with R = 256 / W threads
// each; thread t serves sink t mod W as its lane r = t / W, so that neighbouring lanes read
// neighbouring sinks' partials (the partials of one split and value are contiguous over the
// sinks).  Lane r sums splits s = r, r + R, ... in order; the lanes of a sink inside a wave
// combine by a butterfly (offsets W .. 32), and the at most four wave partials of a sink in wave
// order through LDS.  The sum order depends only on S and W, so results are bit-reproducible.
// The nearest neighbour is the best (key, address) over the splits; the final write predicts the
// pair for its exact |r|^2.  The paper merged this step into the gravity kernel with atomics
// (Methods > Other differences); on this multi-XCD part the device-scope fence each workgroup
// would need costs more than a second launch.
// ---------------------------------------------------------------------------------------------
template <int K>
struct CombineLds {
  double v[kThreads][K];
  uint64_t k[kThreads];
  int i[kThreads];
};

// One workgroup's share of the combine: sinks blk * W .. blk * W + W - 1.
template <int Order, bool NN>
__device__ __forceinline__ void combine_block(const ForceParams &fp, int wlog, int blk, CombineLds<kValues<Order>> &red) {
  constexpr int K = kValues<Order>;
  const int t = threadIdx.x;
  const int W = 1 << wlog;
  const int R = kThreads >> wlog;
  const int ql = t & (W - 1);
  const int r = t >> wlog;
  const int qg = blk * W + ql;
  const int S = fp.splits;
  double w[1][K];
  uint64_t wk[1] = {~0ull};
  int wi[1] = {-1};
#pragma unroll
  for (int k = 0; k < K; ++k) w[0][k] = 0.0;
  // block time-step: the particle's state at t0 is loaded first, so that its latency overlaps the
  // loads of the partials
  BsState st;
  int bs_i = -1;
  if constexpr (Order == 4 || Order == 6) {  // the integrator runs at orders 4 and 6
    if (fp.bs_fuse && r == 0 && qg < fp.ni) {
      bs_i = fp.bs.list[qg];
      bs_load_state<Order>(fp.bs, bs_i, st);
    }
  }
  // the sink's predicted position for the exact nearest-neighbour |r|^2, likewise loaded first
  double xi[3] = {0.0, 0.0, 0.0};
  if constexpr (NN) {
    if (fp.part_xi && r == 0 && qg < fp.ni) {
#pragma unroll
      for (int k = 0; k < 3; ++k) xi[k] = fp.part_xi[3 * (size_t)qg + k];
    }
  }
  if (qg < fp.ni) {
#pragma unroll 4
    for (int s = r; s < S; s += R) {
#pragma unroll
      for (int k = 0; k < K; ++k) w[0][k] += fp.part[part_at(fp, s, k, qg, K)];
      if constexpr (NN) {
        const uint64_t pk = fp.part_key[part_at(fp, s, 0, qg, 1)];
        const int pi = fp.part_idx[part_at(fp, s, 0, qg, 1)];
        if (nn_better(pk, pi, wk[0], wi[0])) {
          wk[0] = pk;
          wi[0] = pi;
        }
      }
    }
  }
  // lanes of one sink inside a wave (W < 64): butterfly over offsets W .. 32; every lane ends
  // with the same bits.  With one sink per workgroup (W = 1) the whole wave is one aligned group
  // and the exchange runs in VALU; with W > 1 a sink's lanes are strided and use permutes.
  if (W == 1) {
    lane_butterfly<1, K, NN>(64, w, wk, wi);
  } else {
    for (int off = 32; off >= W; off >>= 1) {
#pragma unroll
      for (int k = 0; k < K; ++k) w[0][k] += __shfl_xor(w[0][k], off);
      if constexpr (NN) {
        const uint64_t ok = __shfl_xor(wk[0], off);
        const int oi = __shfl_xor(wi[0], off);
        if (nn_better(ok, oi, wk[0], wi[0])) {
          wk[0] = ok;
          wi[0] = oi;
        }
      }
    }
  }
  if (R > 1) {
    // wave partials of a sink: for W < 64 one per wave at thread 64 w + ql (4 in all); for
    // W >= 64 lane r sits at thread r W + ql (R <= 4 in all)
#pragma unroll
    for (int k = 0; k < K; ++k) red.v[t][k] = w[0][k];
    red.k[t] = wk[0];
    red.i[t] = wi[0];
    __syncthreads();
    if (r == 0) {
      const int stride = W < 64 ? 64 : W;
      const int parts = W < 64 ? kThreads / 64 : R;
      for (int j = 1; j < parts; ++j) {
        const int o = j * stride + ql;
#pragma unroll
        for (int k = 0; k < K; ++k) w[0][k] += red.v[o][k];
        if (NN && nn_better(red.k[o], red.i[o], wk[0], wi[0])) {
          wk[0] = red.k[o];
          wi[0] = red.i[o];
        }
      }
    }
  }
  if (r != 0 || qg >= fp.ni) return;
  if constexpr (Order == 4 || Order == 6) {
    if (fp.bs_fuse) {  // block time-step: correct the particle right away
      bs_correct_particle<Order>(fp.bs, bs_i, st, fp.bs_t1, &w[0][0], &w[0][3], Order == 6 ? &w[0][7] : &w[0][0]);
      return;
    }
  }
  finalize_sink<Order, NN>(fp, qg, w[0], wi[0], NN && fp.part_xi ? xi : nullptr);
}

template <int Order, bool NN>
__global__ __launch_bounds__(kThreads) void k_combine(const ForceParams fp, int wlog) {
  __shared__ CombineLds<kValues<Order>> red;
  combine_block<Order, NN>(fp, wlog, blockIdx.x, red);
}

// Device-driven block step: the combine and corrector for the sinks of k_force_dd's launch.
template <int Order>
__global__ __launch_bounds__(kThreads) void k_combine_dd(const ForceParams fp0) {
  __shared__ CombineLds<kValues<Order>> red;
  const int ni = *fp0.dd_count;
  if (ni <= 0) return;
  ForceParams fp = fp0;
  fp.ni = ni;
  fp.t = *fp0.dd_t;
  fp.bs_t1 = fp.t;
  int blocks = 0;
  dd_shape(fp0, ni, fp.lanes_log2, fp.splits, blocks);
  const int wlog = combine_wlog(ni, fp.splits);
  const int nblk = (ni + (1 << wlog) - 1) >> wlog;
  for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
    combine_block<Order, false>(fp, wlog, b, red);
    __syncthreads();  // the next block reuses the LDS
  }
}

// ---------------------------------------------------------------------------------------------
// Batched few-body systems (4th order: acc, jerk, pot).  One persistent launch; each wave takes
// the work items w, w + W, w + 2W, ... of a cost-sorted schedule (W = waves in the grid).  An
// item is a range of sinks of one system of n <= kBatchMax particles: the wave stages the whole
// system in its own LDS slice, then covers its sinks 64/L at a time with L lanes per sink, each
// lane summing every L-th source (self excluded by index), and a butterfly over the L lanes.  L
// comes per item from the schedule (chosen per size class by nbx_batch_tune).
// ---------------------------------------------------------------------------------------------
// The batch stages the 4th-order part of each source record only (position, mass, velocity):
// 40 B (mixed) or 56 B (FP64) per particle instead of the full record, so that more workgroups fit
// a CU's LDS.
template <int Prec>
struct BatchRec;
template <>
struct BatchRec<NBX_MIXED> {
  float xh[3], m, xl[3], v[3];
  __device__ static __forceinline__ BatchRec of(const Mixed<4>::J &j) {
    BatchRec r;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r.xh[c] = j.xh[c];
      r.xl[c] = j.xl[c];
      r.v[c] = j.v[c];
    }
    r.m = j.m;
    return r;
  }
  __device__ __forceinline__ Mixed<4>::J j() const {
    Mixed<4>::J o;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      o.xh[c] = xh[c];
      o.xl[c] = xl[c];
      o.v[c] = v[c];
      o.a[c] = o.j[c] = 0.0f;
    }
    o.m = m;
    return o;
  }
};
template <>
struct BatchRec<NBX_FP64> {
  double x[3], m, v[3];
  __device__ static __forceinline__ BatchRec of(const F64<4>::J &j) {
    BatchRec r;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r.x[c] = j.x[c];
      r.v[c] = j.v[c];
    }
    r.m = j.m;
    return r;
  }
  __device__ __forceinline__ F64<4>::J j() const {
    F64<4>::J o;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      o.x[c] = x[c];
      o.v[c] = v[c];
      o.a[c] = o.j[c] = 0.0;
    }
    o.m = m;
    return o;
  }
};

template <int Prec>
__global__ __launch_bounds__(kThreads) void k_batch(const BatchParams bp) {
  using Tr = typename TraitsSel<4, Prec>::type;
  using T = typename Tr::Real;
  constexpr int K = kValues<4>;
  __shared__ BatchRec<Prec> lds_all[kThreads / 64][kBatchMax];
  __shared__ RedLds<1, K> red_unused;
  const int lane = threadIdx.x & 63;
  const int wslot = threadIdx.x >> 6;
  BatchRec<Prec> *lds = lds_all[wslot];
  const int nwaves = gridDim.x * (kThreads / 64);
  const T eps2 = (T)bp.eps2;
  for (int it = blockIdx.x * (kThreads / 64) + wslot; it < bp.n_items; it += nwaves) {
    const int4 item = bp.items[it];  // (system, lanes_log2, first sink, end sink)
    const int b = bp.offset[item.x];
    const int n = bp.offset[item.x + 1] - b;
    const int s_end = item.w < n ? item.w : n;
    const double zero[3] = {0.0, 0.0, 0.0};
    for (int k = lane; k < n; k += 64) {
      double x[3], v[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        x[c] = bp.x[3 * (size_t)(b + k) + c];
        v[c] = bp.v[3 * (size_t)(b + k) + c];
      }
      lds[k] = BatchRec<Prec>::of(Tr::make_j(x, v, zero, bp.m[b + k]));
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int lg = item.y;
    const int L = 1 << lg;
    for (int base = item.z; base < s_end; base += 64 >> lg) {
      const int i = base + (lane >> lg);
      const int slot = lane & (L - 1);
      const bool live = i < s_end;
      const typename Tr::Sink si = Tr::sink_from_j(lds[live ? i : 0].j());
      Comp<T, K> acc;
      acc.init();
      typename Tr::GKey dummy = Tr::gkey_none();
      for (int j0 = slot; j0 < n; j0 += kChunkAcc << lg) {
        const int je = n < j0 + (kChunkAcc << lg) ? n : j0 + (kChunkAcc << lg);
        for (int j = j0; j < je; j += L)
          Tr::template interact<true, false, false>(lds[j].j(), si, eps2, j, i, acc, dummy);
        acc.template fold<0, K>();
      }
      double w[1][K];
      uint64_t wk[1] = {0};
      int wi[1] = {0};
#pragma unroll
      for (int k = 0; k < K; ++k) w[0][k] = acc.value(k);
      group_reduce<1, K, false>(L, w, wk, wi, red_unused);  // L <= 64: within the wave
      if (slot == 0 && live) {
        const size_t q = (size_t)(b + i);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          bp.acc[3 * q + k] = w[0][k];
          bp.jrk[3 * q + k] = w[0][3 + k];
        }
        bp.pot[q] = w[0][6];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// ---------------------------------------------------------------------------------------------
// Adjoint (vector-Jacobian product) of the 4th-order outputs of a closed system.  For a pair
// with r = x_q - x_p, w = v_q - v_p, q = 1/R, s = r.w and the sink's upstream gradients
// (g_a, g_j, g_p), the pair term f = g_a.A0 + g_j.A1 + g_p.P has (Ga = g_a.r, G1 = g_j.w,
// G2 = g_j.r)
//   df/dr = m_src [q^3 g_a - 3 q^5 s g_j - 3 q^5 G2 w + (-3 q^5 (Ga + G1) + 15 q^7 s G2 + g_p q^3) r]
//   df/dw = m_src [q^3 g_j - 3 q^5 G2 r],   df/dm_src = q^3 (Ga + G1) - 3 q^5 s G2 - g_p q.
// Particle p gathers, over every other particle o, the pair (p sink, o source) with -df/dr,
// -df/dw and the pair (o sink, p source) with +df/dr, +df/dw, +df/dm at r -> -r, w -> -w.  One
// particle per lane, LDS tiles of the other particles, source splits combined in fixed order.
// ---------------------------------------------------------------------------------------------
template <int Prec>
struct VjpRec;
template <>
struct alignas(16) VjpRec<NBX_MIXED> {
  float xh[3], m, xl[3], gp, v[3], pad0, ga[3], pad1, gj[3], pad2;
};
template <>
struct alignas(16) VjpRec<NBX_FP64> {
  double x[3], m, v[3], gp, ga[3], pad0, gj[3], pad1;
};

template <int Prec>
__device__ __forceinline__ VjpRec<Prec> vjp_rec(const VjpParams &vp, int o) {
  VjpRec<Prec> r{};
  const bool live = o < vp.n;
  const size_t b = 3 * (size_t)(live ? o : 0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double x = live ? vp.x[b + k] : kPadPos;
    if constexpr (Prec == NBX_MIXED) {
      ds_split(x, r.xh[k], r.xl[k]);
      r.v[k] = live ? (float)vp.v[b + k] : 0.0f;
      r.ga[k] = live ? (float)vp.g_acc[b + k] : 0.0f;
      r.gj[k] = live ? (float)vp.g_jerk[b + k] : 0.0f;
    } else {
      r.x[k] = x;
      r.v[k] = live ? vp.v[b + k] : 0.0;
      r.ga[k] = live ? vp.g_acc[b + k] : 0.0;
      r.gj[k] = live ? vp.g_jerk[b + k] : 0.0;
    }
  }
  r.m = live ? vp.m[o] : 0.0;
  r.gp = live ? vp.g_pot[o] : 0.0;
  return r;
}

// One pair (p, o), o != p guarded; A[0..2] += d/dx_p, A[3..5] += d/dv_p, A[6] += d/dm_p, with the
// source part accumulated without the factor m_p (applied once at the end): values 7..12.
template <int Prec, typename T>
__device__ __forceinline__ void vjp_pair(const VjpRec<Prec> &P, const VjpRec<Prec> &O, T eps2, bool self,
                                         T (&acc)[13]) {
  T r[3], w[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if constexpr (Prec == NBX_MIXED) {
      r[k] = (O.xh[k] - P.xh[k]) + (O.xl[k] - P.xl[k]);
    } else {
      r[k] = O.x[k] - P.x[k];
    }
    w[k] = O.v[k] - P.v[k];
  }
  const T R2 = r[2] * r[2] + (r[1] * r[1] + (r[0] * r[0] + eps2));
  T q;
  if constexpr (Prec == NBX_MIXED) {
    q = __builtin_amdgcn_rsqf(R2);
    q = q * __builtin_fmaf(-0.5f * R2, q * q, 1.5f);
  } else {
    q = rsqrt64(R2);
  }
  q = self ? T(0) : q;
  const T q2 = q * q, q3 = q * q2, q5 = q3 * q2, q7 = q5 * q2;
  const T s = r[0] * w[0] + r[1] * w[1] + r[2] * w[2];
  // p as the sink of o (gradients of p, mass of o): subtract df/dr, df/dw
  {
    const T Ga = P.ga[0] * r[0] + P.ga[1] * r[1] + P.ga[2] * r[2];
    const T G1 = P.gj[0] * w[0] + P.gj[1] * w[1] + P.gj[2] * w[2];
    const T G2 = P.gj[0] * r[0] + P.gj[1] * r[1] + P.gj[2] * r[2];
    const T cr = T(-3) * q5 * (Ga + G1) + T(15) * q7 * s * G2 + P.gp * q3;
    const T mo = O.m;
    const T t1 = mo * q3, t2 = mo * T(3) * q5 * s, t3 = mo * T(3) * q5 * G2, t4 = mo * cr;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      acc[k] -= t1 * P.ga[k] - t2 * P.gj[k] - t3 * w[k] + t4 * r[k];
      acc[3 + k] -= t1 * P.gj[k] - t3 * r[k];
    }
  }
  // p as the source of o (gradients of o, mass of p), r -> -r, w -> -w
  {
    const T Ha = O.ga[0] * r[0] + O.ga[1] * r[1] + O.ga[2] * r[2];
    const T H1 = O.gj[0] * w[0] + O.gj[1] * w[1] + O.gj[2] * w[2];
    const T H2 = O.gj[0] * r[0] + O.gj[1] * r[1] + O.gj[2] * r[2];
    const T crp = T(3) * q5 * (Ha + H1) - T(15) * q7 * s * H2 + O.gp * q3;
    const T u2 = T(3) * q5 * s, u3 = T(3) * q5 * H2;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      acc[7 + k] += q3 * O.ga[k] - u2 * O.gj[k] - u3 * w[k] - crp * r[k];
      acc[10 + k] += q3 * O.gj[k] - u3 * r[k];
    }
    acc[6] += -q3 * (Ha + H1) + u2 * H2 - O.gp * q;
  }
}

template <int Prec>
__global__ __launch_bounds__(kThreads) void k_vjp(const VjpParams vp) {
  using T = typename std::conditional<Prec == NBX_MIXED, float, double>::type;
  __shared__ VjpRec<Prec> tile[kTile];
  const int S = vp.splits;
  const int split = blockIdx.x % S;
  const int ib = blockIdx.x / S;
  const int p = ib * kThreads + threadIdx.x;
  const int ntiles = vp.n_pad / kTile;
  const int t0 = (int)(((int64_t)split * ntiles) / S);
  const int t1 = (int)(((int64_t)(split + 1) * ntiles) / S);
  const VjpRec<Prec> P = vjp_rec<Prec>(vp, p);
  const T eps2 = (T)vp.eps2;
  Comp<T, 13> acc;
  acc.init();
  for (int tl = t0; tl < t1; ++tl) {
    __syncthreads();
    tile[threadIdx.x] = vjp_rec<Prec>(vp, tl * kTile + threadIdx.x);
    __syncthreads();
    for (int c = 0; c < kTile; c += kChunkAcc) {
#pragma unroll 2
      for (int e = c; e < c + kChunkAcc; ++e) {
        const int o = tl * kTile + e;
        vjp_pair<Prec, T>(P, tile[e], eps2, o == p || o >= vp.n, acc.part);
      }
      acc.template fold<0, 13>();
    }
  }
  double g[7];
  const double mp = P.m;
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = acc.value(k) + mp * acc.value(7 + k);
  g[6] = acc.value(6);
  if (p >= vp.n) return;
  if (S == 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      vp.grad_x[3 * (size_t)p + k] = g[k];
      vp.grad_v[3 * (size_t)p + k] = g[3 + k];
    }
    vp.grad_m[p] = g[6];
  } else {
#pragma unroll
    for (int k = 0; k < 7; ++k) vp.part[((size_t)split * 7 + k) * vp.n + p] = g[k];
  }
}

__global__ __launch_bounds__(256) void k_vjp_combine(const VjpParams vp) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= vp.n) return;
  double g[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int s = 0; s < vp.splits; ++s) {
#pragma unroll
    for (int k = 0; k < 7; ++k) g[k] += vp.part[((size_t)s * 7 + k) * vp.n + p];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    vp.grad_x[3 * (size_t)p + k] = g[k];
    vp.grad_v[3 * (size_t)p + k] = g[3 + k];
  }
  vp.grad_m[p] = g[6];
}

// ---------------------------------------------------------------------------------------------
// Explicit sinks: address of the source carrying each sink's id (first match), or -1.  Sources
// are scanned in LDS tiles of 256 ids.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_selfmap(SourceArrays src, int nj, int ni, const int64_t *ext_id,
                                                      int32_t *self) {
  __shared__ int64_t ids[kTile];
  const int q = blockIdx.x * kThreads + threadIdx.x;
  const int64_t mine = q < ni ? ext_id[q] : 0;
  int found = -1;
  for (int base = 0; base < nj; base += kTile) {
    const int jj = base + (int)threadIdx.x;
    __syncthreads();
    ids[threadIdx.x] = jj < nj ? src.id[jj] : 0;
    __syncthreads();
    const int n = nj - base < kTile ? nj - base : kTile;
    if (found < 0) {
      for (int k = 0; k < n; ++k) {
        if (ids[k] == mine) {
          found = base + k;
          break;
        }
      }
    }
  }
  if (q < ni) self[q] = found;
}

// Neighbour-list overflow: any count above nbr_max raises err[2].
__global__ __launch_bounds__(256) void k_nbr_check(const int32_t *count, int ni, int nbr_max, int *err) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < ni && count[q] > nbr_max) atomicAdd(&err[2], 1);
}

// ---------------------------------------------------------------------------------------------
// Copy kernel: scatter n updated sources (AoS [n][3] FP64) to their addresses.
// ---------------------------------------------------------------------------------------------
template <int Order>
__global__ __launch_bounds__(256) void k_jupdate(SourceArrays src, int nj_max, int n, const int32_t *addr,
                                                 const int64_t *id, const double *m, const double *t,
                                                 const double *x, const double *v, const double *a,
                                                 const double *jk, const double *sn, const double *cr,
                                                 int *err) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int ad = addr[k];
  if (ad < 0 || ad >= nj_max) {
    atomicAdd(&err[1], 1);
    return;
  }
  const size_t b = 3 * (size_t)k;
  src.pos_mass[ad] = make_double4(x[b], x[b + 1], x[b + 2], m[k]);
  double *aj = src.acc_jrk + 6 * (size_t)ad;
  if constexpr (Order == 2) {  // velocity and acceleration optional (NULL: zero), no jerk
    if (v)
      src.vel_time[ad] = make_double4(v[b], v[b + 1], v[b + 2], t[k]);
    else
      src.vel_time[ad] = make_double4(0.0, 0.0, 0.0, t[k]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      aj[c] = a ? a[b + c] : 0.0;
      aj[3 + c] = 0.0;
    }
  } else {
    src.vel_time[ad] = make_double4(v[b], v[b + 1], v[b + 2], t[k]);
    aj[0] = a[b]; aj[1] = a[b + 1]; aj[2] = a[b + 2];
    aj[3] = jk[b]; aj[4] = jk[b + 1]; aj[5] = jk[b + 2];
  }
  if constexpr (Order == 6) {
    double *sc = src.snp_crk + 6 * (size_t)ad;
    sc[0] = sn[b]; sc[1] = sn[b + 1]; sc[2] = sn[b + 2];
    sc[3] = cr[b]; sc[4] = cr[b + 1]; sc[5] = cr[b + 2];
  }
  src.id[ad] = id[k];
}

// Padding sources for addresses [from, to): massless, at rest, far away.
template <int Order>
__global__ __launch_bounds__(256) void k_pad(SourceArrays src, int from, int to) {
  const int ad = from + blockIdx.x * blockDim.x + threadIdx.x;
  if (ad >= to) return;
  src.pos_mass[ad] = make_double4(kPadPos, kPadPos, kPadPos, 0.0);
  src.vel_time[ad] = make_double4(0.0, 0.0, 0.0, 0.0);
  double *aj = src.acc_jrk + 6 * (size_t)ad;
#pragma unroll
  for (int k = 0; k < 6; ++k) aj[k] = 0.0;
  if constexpr (Order == 6) {
    double *sc = src.snp_crk + 6 * (size_t)ad;
#pragma unroll
    for (int k = 0; k < 6; ++k) sc[k] = 0.0;
  }
  src.id[ad] = -1;
}

// Predicted FP64 state of n sources (the force kernel's predictor, written out).
template <int Order>
__global__ __launch_bounds__(256) void k_predict_out(SourceArrays src, int nj, double t, int n,
                                                     const int32_t *addr, double *xp, double *vp,
                                                     double *ap, int *err) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int ad = addr[k];
  if (ad < 0 || ad >= nj) {
    atomicAdd(&err[1], 1);
    return;
  }
  double x[3], v[3], a[3], m;
  predict_addr<Order>(src, ad, t, x, v, a, m);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    xp[3 * (size_t)k + c] = x[c];
    vp[3 * (size_t)k + c] = v[c];
    if (ap) ap[3 * (size_t)k + c] = a[c];
  }
}

// Read back stored (unpredicted) state; any output may be null.
template <int Order>
__global__ __launch_bounds__(256) void k_gather_j(SourceArrays src, int n, const int32_t *addr, int64_t *id,
                                                  double *m, double *t, double *x, double *v, double *a,
                                                  double *jk, double *sn, double *cr) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int ad = addr[k];
  const double4 pm = src.pos_mass[ad];
  const double4 vt = src.vel_time[ad];
  const double *aj = src.acc_jrk + 6 * (size_t)ad;
  const size_t b = 3 * (size_t)k;
  if (id) id[k] = src.id[ad];
  if (m) m[k] = pm.w;
  if (t) t[k] = vt.w;
  if (x) { x[b] = pm.x; x[b + 1] = pm.y; x[b + 2] = pm.z; }
  if (v) { v[b] = vt.x; v[b + 1] = vt.y; v[b + 2] = vt.z; }
  if (a) { a[b] = aj[0]; a[b + 1] = aj[1]; a[b + 2] = aj[2]; }
  if (jk) { jk[b] = aj[3]; jk[b + 1] = aj[4]; jk[b + 2] = aj[5]; }
  if constexpr (Order == 6) {
    const double *sc = src.snp_crk + 6 * (size_t)ad;
    if (sn) { sn[b] = sc[0]; sn[b + 1] = sc[1]; sn[b + 2] = sc[2]; }
    if (cr) { cr[b] = sc[3]; cr[b + 1] = sc[4]; cr[b + 2] = sc[5]; }
  }
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t *p, int n, int value) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = value;
}

// Clock sample (measurement): the first lane of workgroup g records the accelerator complex die
// (XCD) it runs on (hardware register XCC_ID, low 16 bits), the shader-clock cycle counter and the
// constant-rate counter.  Two samples around a timed region give the mean shader clock per XCD.
__global__ __launch_bounds__(64) void k_clock_sample(int64_t *out) {
  if (threadIdx.x != 0) return;
  const int g = blockIdx.x;
  out[3 * g + 0] = (int64_t)(__builtin_amdgcn_s_getreg(20 | (15 << 11)) & 0xffff);  // HW_REG_XCC_ID
  out[3 * g + 1] = (int64_t)clock64();
  out[3 * g + 2] = (int64_t)wall_clock64();
}

// ---------------------------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------------------------
int values_per_sink(int order) { return order == 8 ? 13 : (order == 6 ? 10 : (order == 4 ? 7 : 4)); }

// Launch shape (static rule; nbx_tune replaces it by measured choices per N_i class).  A
// workgroup holds Q = (256 / L) * P sinks and one of S source ranges.
//   * About 8 workgroups per CU (2048) fill the 256 CUs; 16 per CU (4096) from N_i = 2048 on,
//     where every workgroup runs several tiles and a finer split evens out the last round of
//     workgroups on the CUs (5-7 are resident per CU; 2-3% faster at N_i = 2048 and 8192 than
//     2048 workgroups); few sinks take 512 (below 128) or 1024 (128 to 256).
//   * Partials cost S * ni * 72 bytes of scratch traffic: S * ni <= 2^21, and S <= 512 (more
//     splits only add partial traffic: measured slower at every N_i).
//   * Staging a tile costs one FP64 prediction per thread, so a thread should get at least 16
//     interactions per tile: Q >= 16 unless there are fewer sinks than that.
//   * Two sinks per lane (Q = 512) pay off only at large N_i (>= 65536), where each workgroup
//     sees many tiles: mixed precision at orders 2 to 6, FP64 at order 4.
// Q runs from ni rounded up to a power of two (at most 256, or 512 at large N_i) down to that
// floor and the first Q that reaches the workgroup target wins (the largest reuse of each staged
// source); if none does, the floor is used with the largest S allowed.  NBX_SHAPE="L,P,S" in the
// environment overrides the rule.
static int ilog2(int v) {
  int l = 0;
  while ((1 << (l + 1)) <= v) ++l;
  return l;
}

LaunchShape choose_shape(int ni, int nj_pad, int prec, int order) {
  LaunchShape ls;
  const int ntiles = nj_pad / kTile > 0 ? nj_pad / kTile : 1;
  // workgroups to aim for: few sinks take ~512 (two per CU) so that each staged, predicted source
  // feeds as many sinks as possible; many sinks take more, to even out the last round.  Between
  // 128 and 256 sinks 1024 won over 512 and 2048 (4-5% at N_i = 128 and 256, both precisions)
  const int target = ni >= 2048 ? 4096 : (ni > 256 ? 2048 : (ni >= 128 ? 1024 : 512));
  const int64_t part_cap = (int64_t)1 << 21;
  int scap = (int)(part_cap / (ni > 0 ? ni : 1));
  if (scap > ntiles) scap = ntiles;
  if (scap > 512) scap = 512;
  if (scap < 1) scap = 1;
  if (const char *env = getenv("NBX_SHAPE")) {
    int L = 0, P = 0, S = 0;
    // two sinks per lane exist only with one lane per sink
    if (sscanf(env, "%d,%d,%d", &L, &P, &S) == 3 && L >= 1 && L <= kThreads && (L & (L - 1)) == 0 &&
        (P == 1 || (P == 2 && L == 1)) && S >= 1) {
      ls.lanes_log2 = ilog2(L);
      ls.sinks_per_lane = P;
      const int Q = (kThreads >> ls.lanes_log2) * P;
      ls.blocks = (ni + Q - 1) / Q;
      ls.splits = S < ntiles ? S : ntiles;
      return ls;
    }
  }
  int qmin = 1;
  while (qmin < ni && qmin < 16) qmin *= 2;
  int qcover = 1;  // never more sink slots than the next power of two of ni
  // two sinks per lane from N_i = 65536: in FP32 arithmetic at orders 2-6, and in FP64 at order 4,
  // where the long-chunk kernel holds two sinks' FP64 sums at two waves per SIMD (2.4% and 2.8%
  // faster at N_i = 65536 and 131072; 1-10% slower with this rule's splits from 4096 to 32768);
  // not at order 8, where the second sink's 13 sums and jerk push the lane past 256 registers and
  // the launch loses half its waves
  const bool two = ni >= 65536 && ((prec == NBX_MIXED && order <= 6) || (prec == NBX_FP64 && order == 4));
  const int qtop = two ? 2 * kThreads : kThreads;
  while (qcover < ni && qcover < qtop) qcover *= 2;
  int Q = qcover > qmin ? qcover : qmin;
  for (; Q >= qmin; Q /= 2) {
    const int64_t blocks = (ni + Q - 1) / Q;
    if (blocks * scap >= target) break;
  }
  if (Q < qmin) Q = qmin;
  ls.sinks_per_lane = Q > kThreads ? 2 : 1;
  ls.lanes_log2 = ilog2(kThreads * ls.sinks_per_lane / Q);
  ls.blocks = (ni + Q - 1) / Q;
  int S = (target + ls.blocks - 1) / ls.blocks;
  if (S > scap) S = scap;
  if (S < 1) S = 1;
  ls.splits = S;
  return ls;
}

template <int Order, int Prec, int P, bool L1, bool NN, bool Long>
static hipError_t launch_force_t(const ForceParams &fp, const LaunchShape &ls, hipStream_t stream) {
  const dim3 grid(ls.blocks * ls.splits), block(kThreads);
  if (fp.h2) {
    hipError_t e = launch_fill_i32(fp.nbr_count, fp.ni, 0, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_force<Order, Prec, P, L1, true, NN, Long>), grid, block, 0, stream, fp);
  } else {
    hipLaunchKernelGGL((k_force<Order, Prec, P, L1, false, NN, Long>), grid, block, 0, stream, fp);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && fp.h2) {
    hipLaunchKernelGGL(k_nbr_check, dim3((fp.ni + 255) / 256), dim3(256), 0, stream, fp.nbr_count, fp.ni, fp.nbr_max,
                       fp.err);
    e = hipGetLastError();
  }
  if (e != hipSuccess || ls.splits <= 1) return e;
  const int wlog = fp.part_sm ? combine_wlog_sink_major(ls.splits) : combine_wlog(fp.ni, ls.splits);
  const int W = 1 << wlog;
  hipLaunchKernelGGL((k_combine<Order, NN>), dim3((fp.ni + W - 1) / W), dim3(kThreads), 0, stream, fp, wlog);
  return hipGetLastError();
}

// Long chunks where a workgroup runs at least kLongTiles source tiles with one lane per sink (two
// sinks per lane only occur there); several lanes per sink always take the short chunks.
constexpr int kLongTiles = 8;

template <int Order, int Prec, bool NN>
static hipError_t launch_force_nn(const ForceParams &fp, const LaunchShape &ls, hipStream_t stream) {
  const bool long_chunks = fp.nj_pad / kTile >= kLongTiles * ls.splits;
  if (ls.sinks_per_lane == 2) return launch_force_t<Order, Prec, 2, true, NN, true>(fp, ls, stream);
  if (ls.lanes_log2 == 0)
    return long_chunks ? launch_force_t<Order, Prec, 1, true, NN, true>(fp, ls, stream)
                       : launch_force_t<Order, Prec, 1, true, NN, false>(fp, ls, stream);
  return launch_force_t<Order, Prec, 1, false, NN, false>(fp, ls, stream);
}

template <int Order, int Prec>
static hipError_t launch_force_op(const ForceParams &fp, const LaunchShape &ls, hipStream_t stream) {
  return fp.nn ? launch_force_nn<Order, Prec, true>(fp, ls, stream) : launch_force_nn<Order, Prec, false>(fp, ls, stream);
}

hipError_t launch_force(int order, int precision, const ForceParams &fp, const LaunchShape &ls,
                        hipStream_t stream) {
  if (order == 2)
    return precision == NBX_MIXED ? launch_force_op<2, NBX_MIXED>(fp, ls, stream)
                                  : launch_force_op<2, NBX_FP64>(fp, ls, stream);
  if (order == 4)
    return precision == NBX_MIXED ? launch_force_op<4, NBX_MIXED>(fp, ls, stream)
           : precision == NBX_DS  ? launch_force_op<4, NBX_DS>(fp, ls, stream)
                                  : launch_force_op<4, NBX_FP64>(fp, ls, stream);
  if (order == 6)
    return precision == NBX_MIXED ? launch_force_op<6, NBX_MIXED>(fp, ls, stream)
           : precision == NBX_DS  ? launch_force_op<6, NBX_DS>(fp, ls, stream)
                                  : launch_force_op<6, NBX_FP64>(fp, ls, stream);
  return precision == NBX_MIXED ? launch_force_op<8, NBX_MIXED>(fp, ls, stream)
                                : launch_force_op<8, NBX_FP64>(fp, ls, stream);
}

template <int Order, int Prec>
static hipError_t launch_force_dd_t(const ForceParams &fp, int force_groups, int combine_groups, hipStream_t stream) {
  hipLaunchKernelGGL((k_force_dd<Order, Prec>), dim3(force_groups), dim3(kThreads), 0, stream, fp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_combine_dd<Order>, dim3(combine_groups), dim3(kThreads), 0, stream, fp);
  return hipGetLastError();
}

hipError_t launch_force_dd(int order, int precision, const ForceParams &fp, int force_groups, int combine_groups,
                           hipStream_t stream) {
  if (order == 4)
    return precision == NBX_MIXED ? launch_force_dd_t<4, NBX_MIXED>(fp, force_groups, combine_groups, stream)
           : precision == NBX_DS  ? launch_force_dd_t<4, NBX_DS>(fp, force_groups, combine_groups, stream)
                                  : launch_force_dd_t<4, NBX_FP64>(fp, force_groups, combine_groups, stream);
  if (order == 6)
    return precision == NBX_MIXED ? launch_force_dd_t<6, NBX_MIXED>(fp, force_groups, combine_groups, stream)
           : precision == NBX_DS  ? launch_force_dd_t<6, NBX_DS>(fp, force_groups, combine_groups, stream)
                                  : launch_force_dd_t<6, NBX_FP64>(fp, force_groups, combine_groups, stream);
  return hipErrorInvalidValue;
}

static inline int grid_for(int n) { return (n + 255) / 256; }

// Source storage, padding, read-back and the x, v, a predictor are the same at orders 6 and 8
// (order 8 adds only the predicted jerk, used inside the force kernel).
hipError_t launch_jupdate(int order, const SourceArrays &src, int nj_max, int n, const int32_t *addr,
                          const int64_t *id, const double *m, const double *t, const double *x,
                          const double *v, const double *a, const double *jerk, const double *snap,
                          const double *crackle, int *err, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (order == 2)
    hipLaunchKernelGGL(k_jupdate<2>, dim3(grid_for(n)), dim3(256), 0, stream, src, nj_max, n, addr, id, m, t,
                       x, v, a, jerk, snap, crackle, err);
  else if (order == 4)
    hipLaunchKernelGGL(k_jupdate<4>, dim3(grid_for(n)), dim3(256), 0, stream, src, nj_max, n, addr, id, m, t,
                       x, v, a, jerk, snap, crackle, err);
  else
    hipLaunchKernelGGL(k_jupdate<6>, dim3(grid_for(n)), dim3(256), 0, stream, src, nj_max, n, addr, id, m, t,
                       x, v, a, jerk, snap, crackle, err);
  return hipGetLastError();
}

hipError_t launch_pad(int order, const SourceArrays &src, int from, int to, hipStream_t stream) {
  if (to <= from) return hipSuccess;
  if (order < 6)
    hipLaunchKernelGGL(k_pad<4>, dim3(grid_for(to - from)), dim3(256), 0, stream, src, from, to);
  else
    hipLaunchKernelGGL(k_pad<6>, dim3(grid_for(to - from)), dim3(256), 0, stream, src, from, to);
  return hipGetLastError();
}

hipError_t launch_predict_out(int order, const SourceArrays &src, int nj, double t, int n, const int32_t *addr,
                              double *xp, double *vp, double *ap, int *err, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (order == 2)
    hipLaunchKernelGGL(k_predict_out<2>, dim3(grid_for(n)), dim3(256), 0, stream, src, nj, t, n, addr, xp, vp,
                       ap, err);
  else if (order == 4)
    hipLaunchKernelGGL(k_predict_out<4>, dim3(grid_for(n)), dim3(256), 0, stream, src, nj, t, n, addr, xp, vp,
                       ap, err);
  else
    hipLaunchKernelGGL(k_predict_out<6>, dim3(grid_for(n)), dim3(256), 0, stream, src, nj, t, n, addr, xp, vp,
                       ap, err);
  return hipGetLastError();
}

hipError_t launch_gather_j(int order, const SourceArrays &src, int n, const int32_t *addr, int64_t *id,
                           double *m, double *t, double *x, double *v, double *a, double *jerk,
                           double *snap, double *crackle, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (order < 6)
    hipLaunchKernelGGL(k_gather_j<4>, dim3(grid_for(n)), dim3(256), 0, stream, src, n, addr, id, m, t, x, v, a,
                       jerk, snap, crackle);
  else
    hipLaunchKernelGGL(k_gather_j<6>, dim3(grid_for(n)), dim3(256), 0, stream, src, n, addr, id, m, t, x, v, a,
                       jerk, snap, crackle);
  return hipGetLastError();
}

hipError_t launch_vjp(int precision, const VjpParams &vp, hipStream_t stream) {
  if (vp.n <= 0) return hipSuccess;
  const int blocks = (vp.n + kThreads - 1) / kThreads;
  const dim3 grid(blocks * vp.splits), block(kThreads);
  if (precision == NBX_MIXED)
    hipLaunchKernelGGL(k_vjp<NBX_MIXED>, grid, block, 0, stream, vp);
  else
    hipLaunchKernelGGL(k_vjp<NBX_FP64>, grid, block, 0, stream, vp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || vp.splits <= 1) return e;
  hipLaunchKernelGGL(k_vjp_combine, dim3(grid_for(vp.n)), dim3(256), 0, stream, vp);
  return hipGetLastError();
}

hipError_t launch_batch(int precision, const BatchParams &bp, int grid, hipStream_t stream) {
  if (bp.n_items <= 0) return hipSuccess;
  if (precision == NBX_MIXED)
    hipLaunchKernelGGL(k_batch<NBX_MIXED>, dim3(grid), dim3(kThreads), 0, stream, bp);
  else
    hipLaunchKernelGGL(k_batch<NBX_FP64>, dim3(grid), dim3(kThreads), 0, stream, bp);
  return hipGetLastError();
}

int batch_resident_groups(int precision, int device) {
  int per_cu = 0, cus = 0;
  const hipError_t e = precision == NBX_MIXED
                           ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<NBX_MIXED>, kThreads, 0)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<NBX_FP64>, kThreads, 0);
  if (e != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      per_cu < 1 || cus < 1) {
    (void)hipGetLastError();
    return 0;
  }
  return per_cu * cus;
}

hipError_t launch_selfmap(const SourceArrays &src, int nj, int ni, const int64_t *ext_id, int32_t *self,
                          hipStream_t stream) {
  if (ni <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_selfmap, dim3(grid_for(ni)), dim3(kThreads), 0, stream, src, nj, ni, ext_id, self);
  return hipGetLastError();
}

hipError_t launch_clock_sample(int n_groups, int64_t *out, hipStream_t stream) {
  if (n_groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_clock_sample, dim3(n_groups), dim3(64), 0, stream, out);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int n, int value, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, stream, p, n, value);
  return hipGetLastError();
}

}  // namespace nbx
