/*
 * nbx.h -- C ABI of the nbx direct N-body force library (MI355X / gfx950).
 *
 * The library is the GPU half of a GRAPE-style direct N-body code, as in
 * Bedorf, Gaburov & Portegies Zwart, "Sapporo2: A versatile direct N-body
 * library" (arXiv:1510.04068).  In the paper the integrator (block
 * time-steps, Hermite corrector, time-step choice) stays with the host code
 * (Background; Results > Block time-step simulations); here it may, or it can
 * run on the device through the nbx_bs_* entry points below.  One force
 * evaluation is:
 *
 *   1. nbx_set_j      copy updated sources ("j-particles") into the library
 *                     (the copy kernel of Methods > Other differences);
 *   2. nbx_predict    choose the time t every source is predicted to (the
 *                     predict kernel; prediction runs on the GPU, which cuts
 *                     host traffic, Background, Yebisu paragraph);
 *   3. nbx_force      forces on N_i active sinks ("i-particles") from all
 *                     nj sources (the gravity kernel; Methods >
 *                     Parallelisation method);
 *   4. nbx_get_force  read the results back.
 *
 * Force law (the paper prints none; this is the reading used): Newtonian
 * gravity, G = 1, Plummer softening R^2 = |r|^2 + eps2, r = x_j - x_i,
 * v = v_j - v_i, a = a_j - a_i, j = j_j - j_i (predicted), alpha = r.v / R^2,
 * beta = (v.v + r.a) / R^2 + alpha^2,
 * gamma = (3 v.a + r.j) / R^2 + alpha (3 beta - 4 alpha^2):
 *     acc     += m_j r / R^3                                           (= A0)
 *     jerk    += m_j v / R^3 - 3 alpha A0                              (= A1)
 *     snap    += m_j a / R^3 - 6 alpha A1 - 3 beta A0      (orders 6, 8; = A2)
 *     crackle += m_j j / R^3 - 9 alpha A2 - 9 beta A1 - 3 gamma A0   (order 8)
 *     pot     -= m_j / R
 * Sources with the sink's own id are excluded from every output.  Jerk, snap
 * and crackle are the time derivatives of the softened acceleration along the
 * predicted motion, as a 4th/6th/8th-order Hermite integrator needs them
 * (Results; Results > Sixth order performance; order 8 is the expansion that
 * Methods > Numerical Accuracy and the Conclusion name for the double-precision
 * storage: it predicts the jerk of every source and sink as well,
 * j + s dt + c dt^2/2).  Order 2 is the GRAPE-5 mode
 * for a 2nd-order leapfrog (Background; Conclusion): acc and pot only, from
 * positions and masses; its predictor stops at the acceleration term.
 *
 * Nearest neighbour (Results; Discussion > CPU: particle id and distance):
 * the other source with the smallest |r|^2, returned as (id, |r|^2 in FP64);
 * none: id -1, r2 +inf.  In NBX_FP64 the choice is made on the exact FP64
 * |r|^2 (ties to the lower source address); in NBX_MIXED it is made on the
 * FP32 value of |r|^2, so sources whose |r|^2 agree to FP32 rounding may be
 * returned in either order.  A distinct source at the sink's position is a
 * valid nearest neighbour (r2 = 0).  Neighbour list (Background; Results, perturber
 * lists): every other source with |r|^2 < h2_i, at most nbr_max per sink;
 * the count is exact, and when it exceeds nbr_max the stored ids are an
 * unspecified subset and the call returns NBX_WARN_NBR_OVERFLOW.
 *
 * Precision (Methods > Numerical Accuracy; chosen at run time, Background):
 * sources are always stored in FP64.
 *   NBX_FP64   every operation in IEEE double.
 *   NBX_MIXED  predictor in FP64; positions split into double-single
 *              (hi = fl32(x), lo = fl32(x - hi)) and differenced as
 *              (hi_j - hi_i) + (lo_j - lo_i); everything else in FP32, with
 *              FP32 chunk sums folded into FP64 totals.  Results are FP64 arrays.
 *   NBX_DS     the paper's double-single precision (about 14 significant digits):
 *              predictor in FP64, then every pair quantity in double-single
 *              arithmetic (TwoSum / FMA products, R^-1 from the hardware estimate
 *              and one Newton step in double-single), pair terms summed in FP64.
 *              Orders 4 and 6 only (nbx_open / nbx_set_precision return
 *              NBX_ERR_ARG otherwise); the batched and adjoint entry points take
 *              NBX_FP64 or NBX_MIXED.
 *
 * Conventions shared by every entry point:
 *   - Return value: NBX_OK (0), a negative NBX_ERR_* code, or a positive
 *     NBX_WARN_* code.  Nothing aborts and no C++ exception crosses the ABI;
 *     nbx_last_error gives a per-context message for the last failure.
 *   - Vectors are FP64 row-major [n][3] (a contiguous (n, 3) array).
 *   - Host pointers: inputs are read and copied before the call returns, so
 *     the caller may reuse them at once; outputs are caller-owned and written
 *     only by nbx_get_*.
 *   - Device pointers (the *_dev entry points): the caller owns the memory,
 *     which must be device memory of the context's device, and the stream
 *     (a hipStream_t passed as void*, NULL = the null stream).  Those calls
 *     only enqueue work; the caller keeps every buffer alive until the stream
 *     has finished it.
 *   - A context is not thread-safe: use one context per host thread.
 *   - NaN and inf in inputs propagate as IEEE values; they are not checked.
 *   - eps2 = 0 is allowed.  A sink's own source is always excluded, but a distinct source
 *     at exactly the sink's position then gives inf/NaN (the unsoftened pair force).
 */
#ifndef NBX_H
#define NBX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NBX_OK 0
#define NBX_WARN_NBR_OVERFLOW 1 /* a neighbour list was truncated to nbr_max (counts stay exact) */
#define NBX_WARN_DT_MIN 2       /* a block time-step was clamped at dt_min (or its criterion was not a number) */
#define NBX_ERR_ARG (-1)        /* NULL pointer, negative size, bad order/precision, address out of range */
#define NBX_ERR_CAPACITY (-2)   /* n > nj_max or ni > ni_max */
#define NBX_ERR_STATE (-3)      /* call out of order (force before predict, get before force, ...) */
#define NBX_ERR_DEVICE (-4)     /* a HIP call failed; see nbx_last_error */
#define NBX_ERR_NO_DEVICE (-5)  /* no usable GPU (or the requested device does not exist) */
#define NBX_ERR_OOM (-6)        /* device memory allocation failed */

#define NBX_FP64 0
#define NBX_MIXED 1
#define NBX_DS 2 /* double-single arithmetic, orders 4 and 6 (the gravity kernels only) */

typedef struct nbx_ctx nbx_ctx; /* opaque; owns every device buffer it allocates */

typedef struct nbx_config {
  int device;    /* HIP device ordinal */
  int order;     /* 2: acc, pot (GRAPE-5 mode);  4: acc, jerk, pot;  6: also snap (needs snap and
                    crackle of the sources);  8: also crackle (same source data as order 6) */
  int precision; /* NBX_FP64, NBX_MIXED or (orders 4, 6) NBX_DS; can be changed with nbx_set_precision */
  int nj_max;    /* source capacity (addresses 0 .. nj_max-1) */
  int ni_max;    /* largest number of sinks in one nbx_force call */
  int nbr_max;   /* neighbour-list capacity per sink; 0 disables neighbour lists */
  int want_nn;   /* nonzero: force calls return the nearest neighbour (nn_id, nn_r2); 0: the gravity
                    kernels skip the search (the paper makes it a compile-time option of its kernel,
                    Results) and leave every nearest-neighbour output untouched, which may then be
                    NULL; acc, jerk, snap, crackle, pot and lists are bit-identical either way */
} nbx_config;

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int nbx_version(void);

/* Number of visible HIP devices; NBX_ERR_NO_DEVICE (and *count = 0) when none. */
int nbx_device_count(int *count);

/* Create a context on cfg->device and allocate its source/sink buffers.
 * Errors: NBX_ERR_ARG (NULL, order not 2/4/6/8, bad precision, nj_max < 1,
 * ni_max < 1, nbr_max < 0), NBX_ERR_NO_DEVICE, NBX_ERR_OOM, NBX_ERR_DEVICE.
 * On error *out is NULL. */
int nbx_open(nbx_ctx **out, const nbx_config *cfg);

/* Release the context and all its device memory (waits for its own stream). NULL is a no-op. */
int nbx_close(nbx_ctx *ctx);

/* Message describing the last failure on this context (never NULL; "" if none).  Valid until the
 * next call on the same context.  With ctx NULL: the message of the last failed nbx_open. */
const char *nbx_last_error(const nbx_ctx *ctx);

/* Switch the arithmetic of later nbx_force calls (NBX_FP64, NBX_MIXED, or NBX_DS at orders 4 and 6). */
int nbx_set_precision(nbx_ctx *ctx, int precision);

/* Set the number of sources in use: addresses 0 .. nj-1 take part in every force evaluation.
 * 0 <= nj <= nj_max, else NBX_ERR_CAPACITY. */
int nbx_set_nj(nbx_ctx *ctx, int nj);

/* Copy n sources from host arrays into addresses addr[k] (the copy step).  id[n], m[n], t[n]
 * (the time the Taylor data refers to), x, v, a, jerk [n][3]; snap and crackle [n][3] for orders
 * 6 and 8 (NULL for order 4).  Order 2: v and a may be NULL (taken as zero) and jerk is ignored (may be
 * NULL); the predictor uses x + v dt + a dt^2/2.  Every addr must be in [0, nj_max) (else
 * NBX_ERR_ARG, nothing copied); the number of sources in use grows to cover the highest address
 * written.  The host arrays are read before the call returns (packed into pinned staging memory
 * and moved in one copy); the scatter into the source arrays is enqueued on the context's stream
 * and ordered before every later call on the context. */
int nbx_set_j(nbx_ctx *ctx, int n, const int32_t *addr, const int64_t *id, const double *m,
              const double *t, const double *x, const double *v, const double *a,
              const double *jerk, const double *snap, const double *crackle);

/* Select the prediction time: every later force evaluation first predicts each source, and each
 * by-address sink, from its own time t_j to t with its Taylor polynomial (FP64, fused into the
 * force kernel).  Must be called after the sources are set and before nbx_force. */
int nbx_predict(nbx_ctx *ctx, double t);

/* Forces on ni sinks taken by address from the source set (the sink's state is its own
 * predicted source state, so the self pair has r = 0 exactly and is excluded).
 * i_addr[ni] host array, each in [0, nj); eps2 >= 0; h2[ni] squared neighbour radii or NULL
 * (no lists).  Results stay on the device until nbx_get_force / nbx_get_nbr.  Enqueued on the
 * context's stream; returns without waiting for the GPU.  ni = 0 is a no-op; with ni > 0 and no
 * sources in use (nj = 0) every force call, this one and the explicit-sink and device-memory
 * forms, returns NBX_ERR_STATE. */
int nbx_force(nbx_ctx *ctx, int ni, const int32_t *i_addr, double eps2, const double *h2);

/* Forces on ni sinks given explicitly (they need not be sources): id[ni], x, v [ni][3] (v may be
 * NULL for order 2), a [ni][3] for order 6 (else NULL).  A source with the sink's id is excluded.  The sink state is used as
 * given (no prediction).  Otherwise as nbx_force.  An order-8 context returns NBX_ERR_ARG: use
 * nbx_force_ext8. */
int nbx_force_ext(nbx_ctx *ctx, int ni, const int64_t *id, const double *x, const double *v,
                  const double *a, double eps2, const double *h2);

/* Order 8 (Methods > Numerical Accuracy; Conclusion): as nbx_force_ext, with the sink
 * accelerations a and jerks jerk [ni][3] both required (the crackle needs the relative jerk).
 * NBX_ERR_ARG on a context of another order. */
int nbx_force_ext8(nbx_ctx *ctx, int ni, const int64_t *id, const double *x, const double *v,
                   const double *a, const double *jerk, double eps2, const double *h2);

/* Wait for the last nbx_force / nbx_force_ext and copy its results to caller-owned host arrays:
 * acc, jerk [ni][3] (orders 4, 6, 8; never written for order 2), snap [ni][3] (orders 6, 8), pot [ni],
 * nn_id [ni], nn_r2 [ni] (not written when the context has want_nn = 0).  Any pointer may be NULL to
 * skip that output.  The results and the
 * error counters come back in one copy.  Returns NBX_WARN_NBR_OVERFLOW if a neighbour list
 * overflowed, NBX_ERR_ARG if an address was out of range in a copy or force call since the last
 * check. */
int nbx_get_force(nbx_ctx *ctx, double *acc, double *jerk, double *snap, double *pot,
                  int64_t *nn_id, double *nn_r2);

/* Order 8 (Conclusion: the next expansion of the double-precision storage): wait for the last
 * nbx_force and copy its crackle [ni][3] to a caller-owned host array.  NBX_ERR_ARG for another
 * order or NULL; NBX_ERR_STATE before the first force call; error counters as nbx_get_force. */
int nbx_get_crackle(nbx_ctx *ctx, double *crackle);

/* Neighbour lists of the last force call: count[ni] (exact) and ids[ni][nbr_max] (the first
 * min(count, nbr_max) entries of each row are valid, in no particular order). */
int nbx_get_nbr(nbx_ctx *ctx, int32_t *count, int64_t *ids);

/* Predicted FP64 state of n sources at the current prediction time: xp, vp [n][3]; ap [n][3]
 * (NULL to skip).  addr[n] in [0, nj).  Synchronous.  Uses the same predictor as the
 * force kernel. */
int nbx_get_predicted(nbx_ctx *ctx, int n, const int32_t *addr, double *xp, double *vp, double *ap);

/* Read back the stored (unpredicted) state of n sources, e.g. to checkpoint: any output may be
 * NULL.  addr[n] in [0, nj_max).  Synchronous. */
int nbx_get_j(nbx_ctx *ctx, int n, const int32_t *addr, int64_t *id, double *m, double *t,
              double *x, double *v, double *a, double *jerk, double *snap, double *crackle);

/* ---- device-pointer variants (caller-owned device memory and stream; enqueue only) ---------- */

/* As nbx_set_j, from device arrays (order 2: d_v, d_a, d_jerk may be NULL, as there).  Out-of-range
 * addresses are skipped and counted; the next
 * nbx_sync reports them as NBX_ERR_ARG.  The number of sources in use is not changed: call
 * nbx_set_nj. */
int nbx_set_j_dev(nbx_ctx *ctx, void *stream, int n, const int32_t *d_addr, const int64_t *d_id,
                  const double *d_m, const double *d_t, const double *d_x, const double *d_v,
                  const double *d_a, const double *d_jerk, const double *d_snap,
                  const double *d_crackle);

/* As nbx_force, with the sink addresses and every output in caller device memory:
 * d_acc, d_jerk [ni][3] (required; d_jerk may be NULL for order 2 and is not written there),
 * d_snap [ni][3] (order 6, else may be NULL), d_pot [ni],
 * d_nn_id [ni], d_nn_r2 [ni] (required with want_nn; with want_nn = 0 they may be NULL and are never
 * written); d_nbr_count [ni] and d_nbr_ids [ni][nbr_max] when d_h2
 * is given.  Sink addresses outside [0, nj) make the kernel skip that sink (its outputs are left
 * untouched) and are counted for nbx_sync.  An order-8 context returns NBX_ERR_ARG: use
 * nbx_force8_dev. */
int nbx_force_dev(nbx_ctx *ctx, void *stream, int ni, const int32_t *d_i_addr, double eps2,
                  const double *d_h2, double *d_acc, double *d_jerk, double *d_snap,
                  double *d_pot, int64_t *d_nn_id, double *d_nn_r2, int32_t *d_nbr_count,
                  int64_t *d_nbr_ids);

/* For callers that cannot allocate device memory while they run (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): nbx_force_dev without any allocation.
 * nbx_force_dev grows the context's split-partial buffers with hipMalloc when a call needs more;
 * this variant keeps the partials in a static device area of NBX_NOALLOC_SCRATCH_BYTES that every
 * GPU the library runs on holds for the life of the process (its address is looked up once per
 * device by nbx_open), and calls no hipMalloc, hipFree or allocating library routine.  Same
 * arguments, orders (2, 4, 6; order 8 is NBX_ERR_ARG), want_nn behaviour and errors as
 * nbx_force_dev: ni > ni_max is NBX_ERR_CAPACITY.  Sizes: the partials of S source splits take
 * S * ni * (8 * values + 12) bytes (values: 4, 7 or 10 for orders 2, 4, 6; each of the three
 * arrays rounded up to 16 bytes), after 24 bytes per sink (rounded up to 16) for the sinks'
 * predicted positions that the split combine reads; when the launch shape
 * nbx_force_dev would use needs more than the area holds, the call lowers S until they fit (down to
 * one split, which needs none), so results then differ from nbx_force_dev by summation order only,
 * and are bit-identical where the shape fits.  Every call on one GPU shares its area, which keeps
 * the last call's partials: calls that overlap on one GPU (other streams, other contexts, other
 * host threads) race and must be ordered by the caller. */
#define NBX_NOALLOC_SCRATCH_BYTES (64u << 20)
int nbx_force_dev_noalloc(nbx_ctx *ctx, void *stream, int ni, const int32_t *d_i_addr, double eps2,
                          const double *d_h2, double *d_acc, double *d_jerk, double *d_snap,
                          double *d_pot, int64_t *d_nn_id, double *d_nn_r2, int32_t *d_nbr_count,
                          int64_t *d_nbr_ids);

/* Order 8 (Methods > Numerical Accuracy; Conclusion): as nbx_force_dev, with d_snap and d_crackle
 * [ni][3] both required.
 * NBX_ERR_ARG on a context of another order. */
int nbx_force8_dev(nbx_ctx *ctx, void *stream, int ni, const int32_t *d_i_addr, double eps2,
                   const double *d_h2, double *d_acc, double *d_jerk, double *d_snap,
                   double *d_crackle, double *d_pot, int64_t *d_nn_id, double *d_nn_r2,
                   int32_t *d_nbr_count, int64_t *d_nbr_ids);

/* ---- adjoint -----------------------------------------------------------------------------------
 * Gradients of L = sum_i (g_acc_i . acc_i + g_jerk_i . jerk_i + g_pot_i pot_i) with respect to the
 * positions, velocities and masses of a closed system of n particles, where acc, jerk, pot are the
 * 4th-order outputs of nbx_force with every particle a sink and a source (state used as given, no
 * prediction, self excluded).  This is the vector-Jacobian product of that force evaluation, for
 * reverse-mode differentiation through an integrator.  d_m [n], d_x, d_v [n][3], upstream
 * d_g_acc, d_g_jerk [n][3], d_g_pot [n] in; d_grad_x, d_grad_v [n][3], d_grad_m [n] out.  eps2 >= 0.
 * Precision follows the context (NBX_MIXED needs every softened distance above ~1e-5 so that R^-7
 * stays finite in FP32).  Uses the context's split scratch.  Enqueue only. */
int nbx_force_vjp_dev(nbx_ctx *ctx, void *stream, int n, const double *d_m, const double *d_x,
                      const double *d_v, double eps2, const double *d_g_acc, const double *d_g_jerk,
                      const double *d_g_pot, double *d_grad_x, double *d_grad_v, double *d_grad_m);

/* ---- batched few-body systems (4th order: acc, jerk, pot) -------------------------------------
 * Many independent small systems in one persistent launch.  System s holds the particles
 * [offsets[s], offsets[s+1]) of flat device arrays; every particle is a sink and a source of its
 * own system only, its own term excluded; the state is used as given (no prediction).  eps2 >= 0
 * (0 is allowed: coincident distinct particles give inf/NaN).  Precision follows the context.
 * This extends the paper's aim of keeping the GPU busy when only a few particles are integrated
 * (Abstract; Discussion > CPU: small N favours the CPU). */
#define NBX_BATCH_NMAX 128 /* largest system of a batch */

/* Describe the batch: n_sys >= 1 systems, host offsets[n_sys + 1] with offsets[0] = 0 and every
 * size offsets[s+1] - offsets[s] in [1, NBX_BATCH_NMAX] (else NBX_ERR_ARG).  Builds the wave
 * schedule on the host (largest systems first) and uploads it.  Synchronous. */
int nbx_batch_setup(nbx_ctx *ctx, int n_sys, const int32_t *offsets);

/* Autotuner: for every size class present (n in (2^(c-1), 2^c], c = 0..7) time each
 * lanes-per-sink option L = 1..64 on the given device data with HIP events, keep the fastest in
 * the context and rebuild the schedule.  Writes the outputs as a side effect.  Synchronous.
 * lanes_per_class[8] (may be NULL) receives the chosen L per class (0: class absent). */
int nbx_batch_tune(nbx_ctx *ctx, void *stream, const double *d_m, const double *d_x, const double *d_v,
                   double eps2, double *d_acc, double *d_jerk, double *d_pot, int32_t *lanes_per_class);

/* Forces within every system: d_m [n], d_x, d_v [n][3] in, d_acc, d_jerk [n][3] and d_pot [n]
 * out (n = offsets[n_sys]).  Enqueue only.  Without nbx_batch_tune a default L per class is used
 * (L = 64 / next power of two of the class's largest size, at least 1). */
int nbx_batch_force_dev(nbx_ctx *ctx, void *stream, const double *d_m, const double *d_x, const double *d_v,
                        double eps2, double *d_acc, double *d_jerk, double *d_pot);

/* ---- block time-step Hermite integrator ---------------------------------------------------------
 * The integrator the paper runs on top of the library (Results > Block time-step simulations):
 * 4th- or 6th-order Hermite (the context's order) with individual power-of-two time steps, kept
 * resident on the device.  The particles are the context's sources 0..n-1 (nbx_bs_init loads
 * them; any later nbx_set_j / nbx_set_j_dev ends the integration), every block step predicts all
 * of them to the block time, computes the forces on the particles due at that time (the gravity
 * kernel at the context's precision), corrects them and picks their next steps, all on the GPU;
 * only the block time and N_active return to the host.  Corrector (h = dt/2):
 *   order 4: v1 = v0 + h (a0 + a1) - h^2/3 (j1 - j0),  x1 = x0 + h (v0 + v1) - h^2/3 (a1 - a0)
 *   order 6: v1 = v0 + h (a0 + a1) - 2h^2/5 (j1 - j0) + h^3/15 (s0 + s1),
 *            x1 = x0 + h (v0 + v1) - 2h^2/5 (a1 - a0) + h^3/15 (j0 + j1)
 * (the integrals of the Hermite interpolants).  Higher derivatives a2..a5 at the end of a step come
 * from the interpolant of the acceleration (cubic through a, j; quintic through a, j, s).
 * Step criteria: Aarseth dt4 = sqrt(eta4 (|a||a2| + |a1|^2) / (|a1||a3| + |a2|^2)); order 6 takes
 * the average of dt4 and dt6 = eta6 ((|a||a2| + |a1|^2) / (|a3||a5| + |a4|^2))^(1/6), as the paper
 * does for its DS and DP runs (the 6th-order criterion alone can collapse when jerk and snap carry
 * rounding noise).  A step halves until it is at most the criterion and doubles, at most once per
 * step and up to dt_max, when the criterion allows it and the new time is a multiple of the doubled
 * step.  The first step is eta_start |a|/|j| (order 6: at most eta_start sqrt(|a|/|s|)) rounded
 * down to a power of two; the crackle starts at zero. */
typedef struct nbx_bs_params {
  double eps2;      /* softening */
  double eta4;      /* Aarseth accuracy parameter (the paper: 0.01) */
  double eta6;      /* 6th-order accuracy parameter (the paper: 0.1; order 6 only) */
  double eta_start; /* first-step parameter (e.g. 0.01) */
  double dt_max;    /* largest step, a power of two <= 1 */
  double dt_min;    /* smallest step, a power of two, 2^-63 <= dt_min <= dt_max (smaller requests are clamped) */
} nbx_bs_params;

typedef struct nbx_bs_stats {
  double t;               /* current block time */
  int64_t block_steps;    /* block steps since nbx_bs_init */
  int64_t particle_steps; /* sum of N_active over those steps (interactions = particle_steps * n) */
} nbx_bs_stats;

/* Start an integration at t = 0 from host arrays id[n], m[n], x, v [n][3] (1 <= n <= nj_max and
 * <= ni_max; order 4 or 6).  Computes the starting forces (order 6: two passes, the snap needs the
 * accelerations) and first steps.  Synchronous.  NBX_WARN_DT_MIN if a first step was clamped at
 * dt_min (the integration can still proceed; only clamps in later steps stop it). */
int nbx_bs_init(nbx_ctx *ctx, int n, const int64_t *id, const double *m, const double *x,
                const double *v, const nbx_bs_params *p);

/* One block step, if the next block time is <= t_end; *n_active (may be NULL) receives N_active
 * (0: no step taken).  Returns after enqueueing the corrector (waits only for the schedule).  Once
 * any step has been clamped at dt_min it takes no further step and returns NBX_WARN_DT_MIN: the
 * step criterion has collapsed (the paper sees this for the 6th-order criterion when the forces
 * are not accurate enough); the state stays valid and readable. */
int nbx_bs_step(nbx_ctx *ctx, double t_end, int *n_active);

/* Block steps until the next block time would pass t_end; stats (may be NULL) as after the run.
 * Stops early with NBX_WARN_DT_MIN as soon as a step has been clamped at dt_min (stats.t then
 * shows how far it got).  With two or more 256-source tiles the steps are device-driven: the
 * schedule, gravity and combine kernels of each step read N_active and the block time from device
 * memory and the host synchronises once per 32 steps (launch shapes per N_active class as
 * nbx_force would choose them, one sink per lane, at least two source splits); with one tile, or
 * with NBX_BS_HOST_LOOP set in the environment, it runs nbx_bs_step in a loop. */
int nbx_bs_run(nbx_ctx *ctx, double t_end, nbx_bs_stats *stats);

/* State at the current block time: x, v [n][3] (predicted for particles between their steps), dt
 * [n] current steps, t_i [n] the particles' own times, stats; every output may be NULL. */
int nbx_bs_get_state(nbx_ctx *ctx, double *t, double *x, double *v, double *dt, double *t_i,
                     nbx_bs_stats *stats);

/* Kinetic and potential energy at the current block time (positions and velocities predicted;
 * the potential from a force evaluation on all particles; sums in long double).  Synchronous. */
int nbx_bs_energy(nbx_ctx *ctx, double *ekin, double *epot);

/* Wait for all work this context enqueued (on its own stream and on stream) and report
 * device-side argument errors (NBX_ERR_ARG) or neighbour-list overflow (NBX_WARN_NBR_OVERFLOW)
 * recorded since the last nbx_sync. */
int nbx_sync(nbx_ctx *ctx, void *stream);

/* Launch-shape tuner.  The paper's library ships tuning runs that pick the block configuration per
 * GPU (Results > Thread-block configuration; Conclusion).  For every N_i class 2^k up to ni_max
 * (capped at ni_max of the context and the sources in use) this times candidate shapes of the
 * gravity kernel (lanes per sink, sinks per lane, source splits) on the current sources at the
 * current prediction time and precision, with ni evenly strided source addresses as sinks, and
 * keeps the fastest per class.  Later force calls at that precision use the table while the
 * number of 256-source tiles stays the same; otherwise, and before tuning, a static rule applies.
 * shapes_out (may be NULL) receives lanes per sink, sinks per lane and splits for classes
 * k = 0 .. n_classes-1 (3 ints each).  Requires nbx_predict.  Synchronous; overwrites the results
 * of the last nbx_force.  Results of every shape agree to rounding; a fixed table keeps runs
 * bit-reproducible. */
int nbx_tune(nbx_ctx *ctx, int ni_max, int32_t *shapes_out, int n_classes);

/* Launch shape the library would use for ni sinks against the current sources (tuned table or
 * static rule): lanes per sink, sinks per lane, source splits, workgroups.  Lets callers and
 * benchmarks report it. */
int nbx_launch_shape(nbx_ctx *ctx, int ni, int *lanes_per_sink, int *sinks_per_lane,
                     int *splits, int *workgroups);

/* ---- measurement ---------------------------------------------------------------------------
 * Throughput is only comparable with a roofline at a known shader clock, and the clock under load
 * varies from board to board (Results: the paper states its clocks with every GPU).  Enqueue on
 * stream one tiny kernel of n_groups >= 1 workgroups; the first lane of workgroup g writes
 * d_out[3g .. 3g+2] = (XCD the workgroup runs on, shader-clock cycle counter, constant-rate counter).
 * Two samples around a timed region give the mean shader clock of each XCD over that region:
 * (cycles after - cycles before) / (constant ticks after - before) * the constant rate.  d_out is
 * caller device memory of at least 3 n_groups int64.  Enqueue only. */
int nbx_clock_sample(nbx_ctx *ctx, void *stream, int n_groups, int64_t *d_out);

/* The constant rate of the counter above and the shader clock's nominal maximum, in kHz (either
 * pointer may be NULL). */
int nbx_clock_rates(nbx_ctx *ctx, int *wall_khz, int *sclk_max_khz);

#ifdef __cplusplus
}
#endif

#endif /* NBX_H */
