/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the direct N-body force path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library; neither includes the other.
 *
 * What it computes (Bedorf, Gaburov & Portegies Zwart, "Sapporo2: A versatile
 * direct N-body library", arXiv:1510.04068):
 *
 *  - oracle_predict: the source ("j-particle") predictor run before every
 *    force evaluation (Background, Yebisu paragraph; Methods > Other
 *    differences: copy, predict and gravity kernels).  The paper does not
 *    print the predictor; it is the Taylor polynomial of the particle's orbit
 *    about its own time t_j, truncated at the integrator's order: position and
 *    velocity through the acceleration for the 2nd-order (GRAPE-5, leapfrog)
 *    mode, through the jerk for 4th order, and position, velocity and
 *    acceleration through the crackle for 6th.
 *
 *  - oracle_force: direct summation of the forces exerted by the sources on
 *    the sinks ("i-particles") (Methods > Parallelisation method), with the
 *    quantities the Results section lists: acceleration, its time derivative
 *    (jerk) for 4th-order Hermite, the second derivative (snap) for 6th order
 *    (Results > Sixth order performance), the potential (the 2nd-order mode
 *    of the Background section returns acceleration and potential only), the nearest
 *    neighbour (particle id and distance, Discussion > CPU) and the list of
 *    particles within a radius (Background; Results, NBODY4/Kira perturber
 *    lists).  The paper prints no force law; the reading used is Newtonian
 *    gravity with G = 1 and Plummer softening, R^2 = |r|^2 + eps^2, with jerk
 *    and snap the exact time derivatives of the softened acceleration along
 *    the predicted motion:
 *        r = x_j - x_i,  v = v_j - v_i,  a = a_j - a_i
 *        A0 = m_j r / R^3
 *        alpha = (r.v) / R^2
 *        A1 = m_j v / R^3 - 3 alpha A0
 *        beta = (v.v + r.a) / R^2 + alpha^2
 *        A2 = m_j a / R^3 - 6 alpha A1 - 3 beta A0
 *        acc = sum A0, jerk = sum A1, snap = sum A2, pot = -sum m_j / R
 *    Sources whose id equals the sink's id are left out of every output.
 *
 *  - oracle_force8, oracle_predict_jerk: the 8th-order mode.  The paper keeps
 *    its data in double precision so that higher-order Hermite integrators,
 *    6th and 8th order (Nitadori & Makino 2008), can be added without
 *    changing the host code (Methods > Numerical Accuracy; Conclusion: the
 *    library could be expanded with an 8th-order integrator).  That needs the
 *    third derivative of the pair acceleration (crackle) along the predicted
 *    motion, which also uses the relative jerk j = j_j - j_i:
 *        gamma = (3 v.a + r.j) / R^2 + alpha (3 beta - 4 alpha^2)
 *        A3 = m_j j / R^3 - 9 alpha A2 - 9 beta A1 - 3 gamma A0
 *    (d/dt R^-3 = -3 alpha R^-3, d alpha/dt = beta - 3 alpha^2 and
 *    d beta/dt = (3 v.a + r.j) / R^2 - 4 alpha^3 give it from A2), crackle =
 *    sum A3.  Sources carry x, v, a, jerk, snap and crackle as in 6th order;
 *    the predictor adds the jerk, jerk_p = jerk + snap dt + crackle dt^2/2.
 *
 * Arithmetic: every per-pair term is evaluated in IEEE double exactly as
 * written above (1/sqrt for R^-1, no fused multiply-add, no reassociation);
 * the sums over sources run in source index order and are kept in
 * long double (x87 80-bit) so that their rounding is negligible next to the
 * GPU's.  Sinks are independent and are spread over OpenMP threads; a sink's
 * result does not depend on the thread count.
 *
 * Nearest neighbour: the source j != i with the smallest unsoftened |r|^2,
 * ties to the smallest source index; none -> id -1, r^2 = +inf.
 * Neighbour list: every source j != i with |r|^2 < h_i^2 (strict,
 * unsoftened), in source index order, the first nbr_max stored, the count
 * exact.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_ERR_ARG -1

/* Taylor predictor: for each particle, dt = t - t_j and
 *   order 2:  x_p = x + v dt + a dt^2/2,  v_p = v + a dt,  a_p = a
 *   order 4:  x_p = x + v dt + a dt^2/2 + jerk dt^3/6
 *             v_p = v + a dt + jerk dt^2/2,  a_p = a + jerk dt
 *   order 6 (and 8):
 *             x_p = x + v dt + a dt^2/2 + jerk dt^3/6 + snap dt^4/24 + crackle dt^5/120
 *             v_p = v + a dt + jerk dt^2/2 + snap dt^3/6 + crackle dt^4/24
 *             a_p = a + jerk dt + snap dt^2/2 + crackle dt^3/6
 * Arrays are [n][3] row-major; tj is [n].  ap may be NULL for orders 2 and 4; jerk may be NULL
 * for order 2 (it is not used). */
int oracle_predict(int n, int order, double t, const double *tj, const double *x, const double *v,
                   const double *a, const double *jerk, const double *snap, const double *crackle,
                   double *xp, double *vp, double *ap) {
  if (n < 0 || (order != 2 && order != 4 && order != 6 && order != 8) || !tj || !x || !v || !a || !xp ||
      !vp)
    return ORACLE_ERR_ARG;
  if (order != 2 && !jerk) return ORACLE_ERR_ARG;
  if (order >= 6 && (!snap || !crackle || !ap)) return ORACLE_ERR_ARG;
  for (int p = 0; p < n; ++p) {
    const double dt = t - tj[p];
    const double dt2 = dt * dt, dt3 = dt2 * dt, dt4 = dt3 * dt, dt5 = dt4 * dt;
    for (int k = 0; k < 3; ++k) {
      const int q = 3 * p + k;
      if (order == 2) {
        xp[q] = x[q] + v[q] * dt + a[q] * dt2 / 2.0;
        vp[q] = v[q] + a[q] * dt;
        if (ap) ap[q] = a[q];
      } else if (order == 4) {
        xp[q] = x[q] + v[q] * dt + a[q] * dt2 / 2.0 + jerk[q] * dt3 / 6.0;
        vp[q] = v[q] + a[q] * dt + jerk[q] * dt2 / 2.0;
        if (ap) ap[q] = a[q] + jerk[q] * dt;
      } else {
        xp[q] = x[q] + v[q] * dt + a[q] * dt2 / 2.0 + jerk[q] * dt3 / 6.0 + snap[q] * dt4 / 24.0 +
                crackle[q] * dt5 / 120.0;
        vp[q] = v[q] + a[q] * dt + jerk[q] * dt2 / 2.0 + snap[q] * dt3 / 6.0 + crackle[q] * dt4 / 24.0;
        ap[q] = a[q] + jerk[q] * dt + snap[q] * dt2 / 2.0 + crackle[q] * dt3 / 6.0;
      }
    }
  }
  return ORACLE_OK;
}

/* Direct summation.  Sources: nj, idj[nj], mj[nj], xj/vj[nj][3], aj[nj][3]
 * (6th order only).  Sinks: ni, idi[ni], xi/vi[ni][3], ai[ni][3] (6th only),
 * h2[ni] (NULL: no neighbour lists).  Outputs (any may be NULL except acc):
 * acc/jerk/snap[ni][3], pot[ni], nn_id[ni], nn_r2[ni], nbr_count[ni],
 * nbr_ids[ni][nbr_max], cond[ni][3] = (sum |A0|, sum |A1|, sum |A2|) for
 * condition-normalised error measures.  Order 2: acceleration and potential
 * only; vj and vi may be NULL and jerk is not written.  nthreads <= 0: OpenMP
 * default. */
int oracle_force(int order, double eps2, int nj, const int64_t *idj, const double *mj, const double *xj,
                 const double *vj, const double *aj, int ni, const int64_t *idi, const double *xi,
                 const double *vi, const double *ai, const double *h2, int nbr_max, double *acc,
                 double *jerk, double *snap, double *pot, int64_t *nn_id, double *nn_r2,
                 int32_t *nbr_count, int64_t *nbr_ids, double *cond, int nthreads) {
  if ((order != 2 && order != 4 && order != 6) || nj < 0 || ni < 0 || !idj || !mj || !xj || !idi ||
      !xi || !acc)
    return ORACLE_ERR_ARG;
  if (order != 2 && (!vj || !vi)) return ORACLE_ERR_ARG;
  if (order == 6 && (!aj || !ai)) return ORACLE_ERR_ARG;
  if (h2 && (nbr_max < 0 || !nbr_count || (nbr_max > 0 && !nbr_ids))) return ORACLE_ERR_ARG;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif

#pragma omp parallel for schedule(static)
  for (int i = 0; i < ni; ++i) {
    long double s_acc[3] = {0, 0, 0}, s_jerk[3] = {0, 0, 0}, s_snap[3] = {0, 0, 0}, s_pot = 0;
    long double s_c0 = 0, s_c1 = 0, s_c2 = 0;
    double best_r2 = INFINITY;
    int64_t best_id = -1;
    int32_t count = 0;
    const double *x0 = xi + 3 * (size_t)i, *v0 = (order == 2) ? NULL : vi + 3 * (size_t)i;
    const double *a0 = (order == 6) ? ai + 3 * (size_t)i : NULL;
    for (int j = 0; j < nj; ++j) {
      if (idj[j] == idi[i]) continue;
      double r[3], v[3] = {0, 0, 0}, a[3] = {0, 0, 0};
      for (int k = 0; k < 3; ++k) {
        r[k] = xj[3 * (size_t)j + k] - x0[k];
        if (order != 2) v[k] = vj[3 * (size_t)j + k] - v0[k];
        if (order == 6) a[k] = aj[3 * (size_t)j + k] - a0[k];
      }
      const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      const double R2 = r2 + eps2;
      const double Rinv = 1.0 / sqrt(R2);
      const double Rinv2 = Rinv * Rinv;
      const double mR3 = mj[j] * Rinv * Rinv2;
      const double alpha = (r[0] * v[0] + r[1] * v[1] + r[2] * v[2]) * Rinv2;
      double A0[3], A1[3], A2[3];
      for (int k = 0; k < 3; ++k) {
        A0[k] = mR3 * r[k];
        A1[k] = mR3 * v[k] - 3.0 * alpha * A0[k];
      }
      if (order == 6) {
        const double beta =
            (v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + r[0] * a[0] + r[1] * a[1] + r[2] * a[2]) * Rinv2 +
            alpha * alpha;
        for (int k = 0; k < 3; ++k) A2[k] = mR3 * a[k] - 6.0 * alpha * A1[k] - 3.0 * beta * A0[k];
      }
      for (int k = 0; k < 3; ++k) {
        s_acc[k] += A0[k];
        s_jerk[k] += A1[k];
        if (order == 6) s_snap[k] += A2[k];
      }
      s_pot -= mj[j] * Rinv;
      s_c0 += sqrt(A0[0] * A0[0] + A0[1] * A0[1] + A0[2] * A0[2]);
      s_c1 += sqrt(A1[0] * A1[0] + A1[1] * A1[1] + A1[2] * A1[2]);
      if (order == 6) s_c2 += sqrt(A2[0] * A2[0] + A2[1] * A2[1] + A2[2] * A2[2]);
      if (r2 < best_r2) { /* strict: an equal r^2 later in index order loses */
        best_r2 = r2;
        best_id = idj[j];
      }
      if (h2 && r2 < h2[i]) {
        if (count < nbr_max) nbr_ids[(size_t)i * nbr_max + count] = idj[j];
        ++count;
      }
    }
    for (int k = 0; k < 3; ++k) {
      acc[3 * (size_t)i + k] = (double)s_acc[k];
      if (jerk && order != 2) jerk[3 * (size_t)i + k] = (double)s_jerk[k];
      if (snap && order == 6) snap[3 * (size_t)i + k] = (double)s_snap[k];
    }
    if (pot) pot[i] = (double)s_pot;
    if (nn_id) nn_id[i] = best_id;
    if (nn_r2) nn_r2[i] = best_r2;
    if (h2) nbr_count[i] = count;
    if (cond) {
      cond[3 * (size_t)i + 0] = (double)s_c0;
      cond[3 * (size_t)i + 1] = (order == 2) ? 0.0 : (double)s_c1;
      cond[3 * (size_t)i + 2] = (double)s_c2;
    }
  }
  return ORACLE_OK;
}

/* 8th-order mode, predicted jerk: jp = jerk + snap dt + crackle dt^2/2, dt = t - tj. */
int oracle_predict_jerk(int n, double t, const double *tj, const double *jerk, const double *snap,
                        const double *crackle, double *jp) {
  if (n < 0 || !tj || !jerk || !snap || !crackle || !jp) return ORACLE_ERR_ARG;
  for (int p = 0; p < n; ++p) {
    const double dt = t - tj[p];
    for (int k = 0; k < 3; ++k) {
      const int q = 3 * p + k;
      jp[q] = jerk[q] + snap[q] * dt + crackle[q] * dt * dt / 2.0;
    }
  }
  return ORACLE_OK;
}

/* 8th-order mode: as oracle_force at order 6, plus the sources' and sinks' jerks jj[nj][3],
 * ji[ni][3] and the output crackle[ni][3]; cond is [ni][4] (sum |A0|, |A1|, |A2|, |A3|). */
int oracle_force8(double eps2, int nj, const int64_t *idj, const double *mj, const double *xj,
                  const double *vj, const double *aj, const double *jj, int ni, const int64_t *idi,
                  const double *xi, const double *vi, const double *ai, const double *ji, const double *h2,
                  int nbr_max, double *acc, double *jerk, double *snap, double *crackle, double *pot,
                  int64_t *nn_id, double *nn_r2, int32_t *nbr_count, int64_t *nbr_ids, double *cond,
                  int nthreads) {
  if (nj < 0 || ni < 0 || !idj || !mj || !xj || !vj || !aj || !jj || !idi || !xi || !vi || !ai || !ji ||
      !acc)
    return ORACLE_ERR_ARG;
  if (h2 && (nbr_max < 0 || !nbr_count || (nbr_max > 0 && !nbr_ids))) return ORACLE_ERR_ARG;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif

#pragma omp parallel for schedule(static)
  for (int i = 0; i < ni; ++i) {
    long double s[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, s_pot = 0, s_c[4] = {0, 0, 0, 0};
    double best_r2 = INFINITY;
    int64_t best_id = -1;
    int32_t count = 0;
    const double *x0 = xi + 3 * (size_t)i, *v0 = vi + 3 * (size_t)i, *a0 = ai + 3 * (size_t)i;
    const double *j0 = ji + 3 * (size_t)i;
    for (int j = 0; j < nj; ++j) {
      if (idj[j] == idi[i]) continue;
      double r[3], v[3], a[3], jr[3];
      for (int k = 0; k < 3; ++k) {
        r[k] = xj[3 * (size_t)j + k] - x0[k];
        v[k] = vj[3 * (size_t)j + k] - v0[k];
        a[k] = aj[3 * (size_t)j + k] - a0[k];
        jr[k] = jj[3 * (size_t)j + k] - j0[k];
      }
      const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      const double Rinv = 1.0 / sqrt(r2 + eps2);
      const double Rinv2 = Rinv * Rinv;
      const double mR3 = mj[j] * Rinv * Rinv2;
      const double va = v[0] * a[0] + v[1] * a[1] + v[2] * a[2];
      const double rj = r[0] * jr[0] + r[1] * jr[1] + r[2] * jr[2];
      const double alpha = (r[0] * v[0] + r[1] * v[1] + r[2] * v[2]) * Rinv2;
      const double beta =
          (v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + r[0] * a[0] + r[1] * a[1] + r[2] * a[2]) * Rinv2 +
          alpha * alpha;
      const double gamma = (3.0 * va + rj) * Rinv2 + alpha * (3.0 * beta - 4.0 * alpha * alpha);
      double A[4][3];
      for (int k = 0; k < 3; ++k) {
        A[0][k] = mR3 * r[k];
        A[1][k] = mR3 * v[k] - 3.0 * alpha * A[0][k];
        A[2][k] = mR3 * a[k] - 6.0 * alpha * A[1][k] - 3.0 * beta * A[0][k];
        A[3][k] = mR3 * jr[k] - 9.0 * alpha * A[2][k] - 9.0 * beta * A[1][k] - 3.0 * gamma * A[0][k];
      }
      for (int d = 0; d < 4; ++d) {
        for (int k = 0; k < 3; ++k) s[d][k] += A[d][k];
        s_c[d] += sqrt(A[d][0] * A[d][0] + A[d][1] * A[d][1] + A[d][2] * A[d][2]);
      }
      s_pot -= mj[j] * Rinv;
      if (r2 < best_r2) { /* strict: an equal r^2 later in index order loses */
        best_r2 = r2;
        best_id = idj[j];
      }
      if (h2 && r2 < h2[i]) {
        if (count < nbr_max) nbr_ids[(size_t)i * nbr_max + count] = idj[j];
        ++count;
      }
    }
    for (int k = 0; k < 3; ++k) {
      acc[3 * (size_t)i + k] = (double)s[0][k];
      if (jerk) jerk[3 * (size_t)i + k] = (double)s[1][k];
      if (snap) snap[3 * (size_t)i + k] = (double)s[2][k];
      if (crackle) crackle[3 * (size_t)i + k] = (double)s[3][k];
    }
    if (pot) pot[i] = (double)s_pot;
    if (nn_id) nn_id[i] = best_id;
    if (nn_r2) nn_r2[i] = best_r2;
    if (h2) nbr_count[i] = count;
    if (cond)
      for (int d = 0; d < 4; ++d) cond[4 * (size_t)i + d] = (double)s_c[d];
  }
  return ORACLE_OK;
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Vector-Jacobian product of the 4th-order outputs (acc, jerk, pot) of a closed system (every
 * particle is a sink and a source, self excluded) with respect to the inputs (x, v, m).
 * Upstream gradients g_acc, g_jerk [n][3] and g_pot [n].  For one pair with
 * r = x_j - x_i, v = v_j - v_i, q = 1/R, s = r.v and the sink's gradients (g_a, g_j, g_p), the
 * contribution f = g_a.A0 + g_j.A1 + g_p.P (A0 = m_j r q^3, A1 = m_j (v q^3 - 3 s r q^5),
 * P = -m_j q) has, writing Ga = g_a.r, G1 = g_j.v, G2 = g_j.r:
 *   df/dr = m_j [q^3 g_a - 3 q^5 s g_j - 3 q^5 G2 v + (-3 q^5 (Ga + G1) + 15 q^7 s G2 + g_p q^3) r]
 *   df/dv = m_j [q^3 g_j - 3 q^5 G2 r]
 *   df/dm_j = q^3 (Ga + G1) - 3 q^5 s G2 - g_p q
 * and r, v enter x_j, v_j with + and x_i, v_i with -.  Outputs grad_x, grad_v [nsel][3] and
 * grad_m [nsel] for the particles sel[nsel] (all if sel is NULL and nsel == n). */
int oracle_force_vjp(double eps2, int n, const double *m, const double *x, const double *v,
                     const double *g_acc, const double *g_jerk, const double *g_pot, int nsel,
                     const int32_t *sel, double *grad_x, double *grad_v, double *grad_m, int nthreads) {
  if (n < 0 || nsel < 0 || !m || !x || !v || !g_acc || !g_jerk || !g_pot || !grad_x || !grad_v || !grad_m)
    return ORACLE_ERR_ARG;
  if (!sel && nsel != n) return ORACLE_ERR_ARG;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(static)
  for (int a = 0; a < nsel; ++a) {
    const int p = sel ? sel[a] : a;
    long double gx[3] = {0, 0, 0}, gv[3] = {0, 0, 0}, gm = 0;
    for (int o = 0; o < n; ++o) {
      if (o == p) continue;
      /* p as the sink of source o: r = x_o - x_p; d/dx_p = -df/dr, d/dv_p = -df/dv */
      /* p as the source of sink o: r = x_p - x_o; d/dx_p = +df/dr, d/dv_p = +df/dv, d/dm_p = df/dm */
      for (int role = 0; role < 2; ++role) {
        const int sink = role == 0 ? p : o, src = role == 0 ? o : p;
        double r[3], w[3];
        for (int k = 0; k < 3; ++k) {
          r[k] = x[3 * (size_t)src + k] - x[3 * (size_t)sink + k];
          w[k] = v[3 * (size_t)src + k] - v[3 * (size_t)sink + k];
        }
        const double *ga = g_acc + 3 * (size_t)sink, *gj = g_jerk + 3 * (size_t)sink;
        const double gp = g_pot[sink], mj = m[src];
        const double R2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
        const double q = 1.0 / sqrt(R2);
        const double q3 = q * q * q, q5 = q3 * q * q, q7 = q5 * q * q;
        const double s = r[0] * w[0] + r[1] * w[1] + r[2] * w[2];
        const double Ga = ga[0] * r[0] + ga[1] * r[1] + ga[2] * r[2];
        const double G1 = gj[0] * w[0] + gj[1] * w[1] + gj[2] * w[2];
        const double G2 = gj[0] * r[0] + gj[1] * r[1] + gj[2] * r[2];
        const double cr = -3.0 * q5 * (Ga + G1) + 15.0 * q7 * s * G2 + gp * q3;
        const double sign = role == 0 ? -1.0 : 1.0;
        for (int k = 0; k < 3; ++k) {
          const double dr = mj * (q3 * ga[k] - 3.0 * q5 * s * gj[k] - 3.0 * q5 * G2 * w[k] + cr * r[k]);
          const double dv = mj * (q3 * gj[k] - 3.0 * q5 * G2 * r[k]);
          gx[k] += sign * dr;
          gv[k] += sign * dv;
        }
        if (role == 1) gm += q3 * (Ga + G1) - 3.0 * q5 * s * G2 - gp * q;
      }
    }
    for (int k = 0; k < 3; ++k) {
      grad_x[3 * (size_t)a + k] = (double)gx[k];
      grad_v[3 * (size_t)a + k] = (double)gv[k];
    }
    grad_m[a] = (double)gm;
  }
  return ORACLE_OK;
}
