/*
 * lbm_oracle.c -- plain, slow FP64 CPU oracle for the D2Q9 MRT lattice
 * Boltzmann time step with the absorbing-layer damping term of
 * H. Xu and P. Sagaut, "Analysis of the absorbing layers for the
 * weakly-compressible lattice Boltzmann schemes" (arXiv:1203.6350).
 *
 * TEST INFRASTRUCTURE. This file exists to check the HIP implementation.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it. It shares no code, header, table or helper with the HIP path,
 * and the HIP path never calls it.
 *
 * What it computes (notation of the paper, Section 2):
 *   state f_i(x,t): pre-collision populations, i = 0..8, on a periodic
 *   nx-by-ny lattice (lattice closure, Section 2.1), delta t = 1.
 *   One step, for every cell x:
 *     1. m = M f with the D2Q9 transform matrix M of Appendix A.1 (eq. q-macro)
 *     2. shifted macroscopic quantities rho*, rho* u* defined implicitly by the
 *        Guo-type sums of Sections 2.2.1-2.2.3; since every damping force F has
 *        sum_i F_i = chi (rho^f - rho*) and sum_i c_i F_i = chi (j^f - j*)
 *        (Appendix B.1), the implicit definition is solved exactly:
 *        rho* = (rho + n chi rho^f)/(1 + n chi), j* = (j + m chi j^f)/(1 + m chi)
 *     3. f^eq(rho*, j*) in velocity space and m^eq* = M f^eq(rho*, j*)
 *     4. damping vector d in moment space, Gamma = chi I (eq. eq:gamma):
 *          NONE : d = 0
 *          I    : d = chi (M f^eq(rho^f, j^f) - m)          (Section 2.2.1)
 *          II   : d = chi (M f^eq(rho^f, j^f) - m^eq*)      (Section 2.2.2)
 *          III  : d = chi (M f^L(rho^f, j^f) - M f^L(rho*, j*)) (Section 2.2.3)
 *        plus, for checking only, Type I in its rewritten form of eq.
 *        app:newbgka (relaxation S + chi I towards m^eq*, force F).
 *     5. m' = m + S o (m^eq* - m) + d   (Lambda = M^-1 S M, eq. blbs-abc-1)
 *     6. f' = M^-1 m', with M^-1 from Gauss-Jordan elimination
 *     7. a separate streaming pass: f_i(x, t+1) = f'_i(x - c_i)   (eq. blbs)
 *
 * Readings where the paper is silent (the equilibrium form, the weights and
 * the velocity order) follow the standard second-order D2Q9 model with
 * c_s^2 = 1/3, which the paper's wavelength lambda = c_s/2 = 0.288675
 * (Section 4.2) confirms:
 *   f^eq_i = w_i [rho + 3 c_i.j + 9/2 (c_i.j)^2/rho - 3/2 |j|^2/rho]
 *   f^L_i  = w_i [rho + 3 c_i.j]   (the part linear in j)
 * Velocities follow the column order of M's rows 1 and 2 (Appendix A.1).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 9

/* Appendix A.1, D2Q9 transform matrix; rows (rho, jx, jy, e, eps, qx, qy,
 * pxx, pxy). */
static const double M_D2Q9[Q][Q] = {
    { 1,  1,  1,  1,  1, 1,  1,  1,  1},
    { 0,  1,  0, -1,  0, 1, -1, -1,  1},
    { 0,  0,  1,  0, -1, 1,  1, -1, -1},
    {-4, -1, -1, -1, -1, 2,  2,  2,  2},
    { 4, -2, -2, -2, -2, 1,  1,  1,  1},
    { 0, -2,  0,  2,  0, 1, -1, -1,  1},
    { 0,  0, -2,  0,  2, 1,  1, -1, -1},
    { 0,  1, -1,  1, -1, 0,  0,  0,  0},
    { 0,  0,  0,  0,  0, 1, -1,  1, -1}};

/* Velocity set: c_j = (M[1][j], M[2][j]) (the condition M_{alpha j} = v_j^alpha
 * of Section 2.1). */
static int CX[Q], CY[Q];
/* Standard D2Q9 weights (reading: not printed in the paper). */
static const double W[Q] = {4.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9, 1.0 / 9,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static double MINV[Q][Q];
static int g_ready = 0;

/* Gauss-Jordan elimination with partial pivoting on a 9x9 system. */
static int invert9(const double A[Q][Q], double R[Q][Q]) {
  double a[Q][2 * Q];
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < 2 * Q; ++j)
      a[i][j] = j < Q ? A[i][j] : (j - Q == i ? 1.0 : 0.0);
  for (int c = 0; c < Q; ++c) {
    int p = c;
    for (int r = c + 1; r < Q; ++r)
      if (fabs(a[r][c]) > fabs(a[p][c])) p = r;
    if (a[p][c] == 0.0) return -1;
    if (p != c)
      for (int j = 0; j < 2 * Q; ++j) {
        double t = a[c][j];
        a[c][j] = a[p][j];
        a[p][j] = t;
      }
    double piv = a[c][c];
    for (int j = 0; j < 2 * Q; ++j) a[c][j] /= piv;
    for (int r = 0; r < Q; ++r) {
      if (r == c) continue;
      double fac = a[r][c];
      if (fac == 0.0) continue;
      for (int j = 0; j < 2 * Q; ++j) a[r][j] -= fac * a[c][j];
    }
  }
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j) R[i][j] = a[i][j + Q];
  return 0;
}

static void setup(void) {
  if (g_ready) return;
  for (int j = 0; j < Q; ++j) {
    CX[j] = (int)M_D2Q9[1][j];
    CY[j] = (int)M_D2Q9[2][j];
  }
  invert9(M_D2Q9, MINV);
  g_ready = 1;
}

/* y = A x for a 9x9 matrix. */
static void matvec(const double A[Q][Q], const double *x, double *y) {
  for (int i = 0; i < Q; ++i) {
    double acc = 0.0;
    for (int j = 0; j < Q; ++j) acc += A[i][j] * x[j];
    y[i] = acc;
  }
}

/* Second-order equilibrium in velocity space from (rho, jx, jy). */
static void feq(double rho, double jx, double jy, double *out) {
  for (int i = 0; i < Q; ++i) {
    double cj = CX[i] * jx + CY[i] * jy;
    out[i] = W[i] * (rho + 3.0 * cj + 4.5 * cj * cj / rho -
                     1.5 * (jx * jx + jy * jy) / rho);
  }
}

/* Linear part f^(L,eq) of the equilibrium (Section 2.1). */
static void flin(double rho, double jx, double jy, double *out) {
  for (int i = 0; i < Q; ++i)
    out[i] = W[i] * (rho + 3.0 * (CX[i] * jx + CY[i] * jy));
}

/* V_VISC: the comparison strategy of Section 4.1 (no damping term; the
 * relaxation rates of the non-conserved moments decrease linearly towards 1
 * inside the layer): the chi argument then carries the ramp coordinate
 * xi in [0, 1], and s_k becomes s_k + (1 - s_k) xi for k >= 3. */
enum { V_NONE = 0, V_I = 1, V_II = 2, V_III = 3, V_I_REWRITTEN = 4, V_VISC = 5 };

/* Collision with the damping term at one cell.
 * fin: pre-collision populations; chi: sponge strength at the cell;
 * rf, uxf, uyf: reference (far-field) state q_ref = (rho^f, u^f);
 * s[9]: diagonal of S; n, m: shift parameters of rho* and rho* u*. */
static void collide_cell(const double *fin, double chi, double rf, double uxf,
                         double uyf, const double *s, double n, double m,
                         int variant, double *fout) {
  double mom[Q], f_eqs[Q], meqs[Q], tmp[Q], tmp2[Q], d[Q], mp[Q];
  /* without an absorbing term the force vanishes and rho* = rho, j* = j */
  const double xi = chi;
  if (variant == V_NONE || variant == V_VISC) chi = 0.0;
  matvec(M_D2Q9, fin, mom);
  const double rho = mom[0], jx = mom[1], jy = mom[2];
  const double jxf = rf * uxf, jyf = rf * uyf;
  /* exact solution of the implicit rho*, j* definition */
  const double rhos = (rho + n * chi * rf) / (1.0 + n * chi);
  const double jxs = (jx + m * chi * jxf) / (1.0 + m * chi);
  const double jys = (jy + m * chi * jyf) / (1.0 + m * chi);
  feq(rhos, jxs, jys, f_eqs);
  matvec(M_D2Q9, f_eqs, meqs);

  for (int k = 0; k < Q; ++k) d[k] = 0.0;
  double sk[Q];
  for (int k = 0; k < Q; ++k) sk[k] = s[k];
  switch (variant) {
    case V_NONE:
      break;
    case V_I: /* f^ref = f^eq(rho^f,u^f), f* = f */
      feq(rf, jxf, jyf, tmp);
      matvec(M_D2Q9, tmp, tmp2);
      for (int k = 0; k < Q; ++k) d[k] = chi * (tmp2[k] - mom[k]);
      break;
    case V_II: /* f^ref = f^eq(rho^f,u^f), f* = f^eq(rho*,u*) */
      feq(rf, jxf, jyf, tmp);
      matvec(M_D2Q9, tmp, tmp2);
      for (int k = 0; k < Q; ++k) d[k] = chi * (tmp2[k] - meqs[k]);
      break;
    case V_III: { /* f^ref = f^L(rho^f,u^f), f* = f^L(rho*,u*) */
      double a[Q], b[Q];
      flin(rf, jxf, jyf, tmp);
      matvec(M_D2Q9, tmp, a);
      flin(rhos, jxs, jys, tmp);
      matvec(M_D2Q9, tmp, b);
      for (int k = 0; k < Q; ++k) d[k] = chi * (a[k] - b[k]);
      break;
    }
    case V_VISC:
      for (int k = 3; k < Q; ++k) sk[k] = s[k] + (1.0 - s[k]) * xi;
      break;
    case V_I_REWRITTEN: { /* eq. app:newbgka: S' = S + chi I, force F */
      double a[Q];
      feq(rf, jxf, jyf, tmp);
      matvec(M_D2Q9, tmp, a);
      for (int k = 0; k < Q; ++k) {
        sk[k] = s[k] + chi;
        d[k] = chi * (a[k] - meqs[k]);
      }
      break;
    }
    default:
      break;
  }
  for (int k = 0; k < Q; ++k) mp[k] = mom[k] + sk[k] * (meqs[k] - mom[k]) + d[k];
  matvec(MINV, mp, fout);
}

static inline int64_t wrap(int64_t a, int64_t n) {
  a %= n;
  return a < 0 ? a + n : a;
}

/*
 * oracle_step -- advance the pre-collision state f by nsteps steps.
 *   f      : [9][ny][nx] FP64, x fastest; updated in place.
 *   chi    : [ny][nx] sponge strength, or NULL for chi = 0 everywhere.
 *   qref   : [3][ny][nx] (rho^f, u^f_x, u^f_y) per cell, or NULL to use
 *            qref_uniform[3].
 *   s      : 9 relaxation rates (diagonal of S).
 *   srel   : [ny][nx] per-cell rate replacing s[3..8], or NULL.
 *   n, m   : shift parameters (0.5 in the paper).
 *   variant: 0 none, 1 Type I, 2 Type II, 3 Type III, 4 Type I rewritten,
 *            5 viscosity ramp (chi then holds the ramp coordinate xi).
 *   nthreads: OpenMP threads (<= 0: library default).
 * Returns 0, or -1 on bad arguments.
 */
int oracle_step(int64_t nx, int64_t ny, double *f, const double *chi,
                const double *qref, const double *qref_uniform,
                const double *s, const double *srel, double n, double m,
                int variant, int64_t nsteps, int nthreads) {
  setup();
  if (nx < 1 || ny < 1 || !f || !s || nsteps < 0) return -1;
  if (!qref && !qref_uniform) return -1;
  const int64_t N = nx * ny;
  double *post = (double *)malloc(sizeof(double) * Q * N);
  if (!post) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  for (int64_t t = 0; t < nsteps; ++t) {
    /* collision, cell by cell */
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < ny; ++y) {
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t c = y * nx + x;
        double fin[Q], fo[Q], sl[Q];
        for (int i = 0; i < Q; ++i) fin[i] = f[i * N + c];
        const double ch = chi ? chi[c] : 0.0;
        const double rf = qref ? qref[c] : qref_uniform[0];
        const double uxf = qref ? qref[N + c] : qref_uniform[1];
        const double uyf = qref ? qref[2 * N + c] : qref_uniform[2];
        for (int i = 0; i < Q; ++i) sl[i] = s[i];
        if (srel)
          for (int i = 3; i < Q; ++i) sl[i] = srel[c];
        collide_cell(fin, ch, rf, uxf, uyf, sl, n, m, variant, fo);
        for (int i = 0; i < Q; ++i) post[i * N + c] = fo[i];
      }
    }
    /* streaming: f_i(x) <- f'_i(x - c_i), periodic */
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < ny; ++y) {
      for (int64_t x = 0; x < nx; ++x) {
        for (int i = 0; i < Q; ++i) {
          const int64_t xs = wrap(x - CX[i], nx), ys = wrap(y - CY[i], ny);
          f[i * N + y * nx + x] = post[i * N + ys * nx + xs];
        }
      }
    }
  }
  free(post);
  return 0;
}

/*
 * oracle_step_avg -- like oracle_step with a time-dependent reference state
 * (Sec. 1 and Sec. 2.2: q_ref may be a time-dependent mean of the
 * macroscopic quantities). The mean is kept in conserved form:
 *   cf : [3][ny][nx] (rho^f, j^f_x, j^f_y), updated in place.
 * Each step, every cell collides with q_ref = (rho^f, j^f / rho^f), then the
 * mean follows the cell's pre-collision moments c = (rho, j) as an
 * exponential running mean, c^f <- c^f + alpha (c - c^f), before streaming.
 * alpha = 0 keeps the field fixed.
 */
int oracle_step_avg(int64_t nx, int64_t ny, double *f, const double *chi, double *cf,
                    const double *s, double n, double m, int variant, double alpha,
                    int64_t nsteps, int nthreads) {
  setup();
  if (nx < 1 || ny < 1 || !f || !cf || !s || nsteps < 0) return -1;
  const int64_t N = nx * ny;
  double *post = (double *)malloc(sizeof(double) * Q * N);
  if (!post) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  for (int64_t t = 0; t < nsteps; ++t) {
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < ny; ++y) {
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t c = y * nx + x;
        double fin[Q], fo[Q], mom[Q];
        for (int i = 0; i < Q; ++i) fin[i] = f[i * N + c];
        const double rf = cf[c], jxf = cf[N + c], jyf = cf[2 * N + c];
        collide_cell(fin, chi ? chi[c] : 0.0, rf, jxf / rf, jyf / rf, s, n, m, variant, fo);
        for (int i = 0; i < Q; ++i) post[i * N + c] = fo[i];
        matvec(M_D2Q9, fin, mom);  /* pre-collision moments: rho = mom[0], j = mom[1..2] */
        cf[c] = rf + alpha * (mom[0] - rf);
        cf[N + c] = jxf + alpha * (mom[1] - jxf);
        cf[2 * N + c] = jyf + alpha * (mom[2] - jyf);
      }
    }
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < ny; ++y) {
      for (int64_t x = 0; x < nx; ++x) {
        for (int i = 0; i < Q; ++i) {
          const int64_t xs = wrap(x - CX[i], nx), ys = wrap(y - CY[i], ny);
          f[i * N + y * nx + x] = post[i * N + ys * nx + xs];
        }
      }
    }
  }
  free(post);
  return 0;
}

/*
 * oracle_step_line_source -- like oracle_step (uniform q_ref) on a channel
 * with the acoustic line source of Sec. 4.2: after each step's collision
 * the column x = 0 is replaced by the source's equilibrium
 * f^eq(rho_src(t + 1), u_src), rho_src(t) = rho0 + amp sin(2 pi freq t + phase)
 * (t counted in steps, t0 the step index of the input state), and, if
 * outflow != 0, the column x = nx - 1 by a copy of column nx - 2
 * (zero-gradient outflow); streaming then proceeds as on the periodic
 * lattice, which these two columns' overrides cut in x.
 *   src: {rho0, amp, freq, phase, ux, uy}.
 */
int oracle_step_line_source(int64_t nx, int64_t ny, double *f, const double *chi,
                            const double *qref_uniform, const double *s, double n, double m,
                            int variant, const double *src, int outflow, int64_t t0,
                            int64_t nsteps, int nthreads) {
  setup();
  if (nx < 3 || ny < 1 || !f || !s || !qref_uniform || !src || nsteps < 0) return -1;
  const int64_t N = nx * ny;
  double *post = (double *)malloc(sizeof(double) * Q * N);
  if (!post) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  const double PI = 3.14159265358979323846;
  for (int64_t t = 0; t < nsteps; ++t) {
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < ny; ++y) {
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t c = y * nx + x;
        double fin[Q], fo[Q];
        for (int i = 0; i < Q; ++i) fin[i] = f[i * N + c];
        collide_cell(fin, chi ? chi[c] : 0.0, qref_uniform[0], qref_uniform[1], qref_uniform[2],
                     s, n, m, variant, fo);
        for (int i = 0; i < Q; ++i) post[i * N + c] = fo[i];
      }
    }
    /* boundary columns */
    const double tn = (double)(t0 + t + 1);
    const double rs = src[0] + src[1] * sin(2.0 * PI * src[2] * tn + src[3]);
    double fs[Q];
    feq(rs, rs * src[4], rs * src[5], fs);
    for (int64_t y = 0; y < ny; ++y) {
      for (int i = 0; i < Q; ++i) {
        post[i * N + y * nx] = fs[i];
        if (outflow) post[i * N + y * nx + nx - 1] = post[i * N + y * nx + nx - 2];
      }
    }
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < ny; ++y) {
      for (int64_t x = 0; x < nx; ++x) {
        for (int i = 0; i < Q; ++i) {
          const int64_t xs = wrap(x - CX[i], nx), ys = wrap(y - CY[i], ny);
          f[i * N + y * nx + x] = post[i * N + ys * nx + xs];
        }
      }
    }
  }
  free(post);
  return 0;
}

/* One collision (no streaming) for a batch of independent cells, used by the
 * Von Neumann cross-checks.  fin, fout: [ncell][9]. */
int oracle_collide(int64_t ncell, const double *fin, const double *chi,
                   const double *qref /* [ncell][3] */, const double *s,
                   double n, double m, int variant, double *fout) {
  setup();
  if (ncell < 0 || !fin || !fout || !s || !qref) return -1;
  for (int64_t c = 0; c < ncell; ++c)
    collide_cell(fin + 9 * c, chi ? chi[c] : 0.0, qref[3 * c], qref[3 * c + 1],
                 qref[3 * c + 2], s, n, m, variant, fout + 9 * c);
  return 0;
}

/* Equilibrium populations f^eq(rho, u) on a field: out [9][N]. */
int oracle_feq_field(int64_t N, const double *rho, const double *ux,
                     const double *uy, double *out) {
  setup();
  for (int64_t c = 0; c < N; ++c) {
    double e[Q];
    feq(rho[c], rho[c] * ux[c], rho[c] * uy[c], e);
    for (int i = 0; i < Q; ++i) out[i * N + c] = e[i];
  }
  return 0;
}

/* Linear equilibrium f^L(rho, u) on a field: out [9][N]. */
int oracle_flin_field(int64_t N, const double *rho, const double *ux,
                      const double *uy, double *out) {
  setup();
  for (int64_t c = 0; c < N; ++c) {
    double e[Q];
    flin(rho[c], rho[c] * ux[c], rho[c] * uy[c], e);
    for (int i = 0; i < Q; ++i) out[i * N + c] = e[i];
  }
  return 0;
}

/*
 * oracle_diagnostics -- the monitored quantities of a pre-collision state
 * f[9][ny][nx] relative to the base state (rho_b, u_b). The density
 * deviation delta rho = rho - rho_b is what the L2 error of Section 4.1 sums
 * (E_L2 = sqrt(sum delta rho^2 / N) with rho_b = rho_0), and the momentum
 * deviation delta j = j - rho_b u_b its counterpart for the flow.
 *   out[0] = sum over cells of delta rho       (rho = sum_i f_i)
 *   out[1] = sum of delta j_x                  (j = sum_i c_i f_i)
 *   out[2] = sum of delta j_y
 *   out[3] = sum of delta rho^2
 *   out[4] = sum of |delta j|^2
 *   out[5] = max over finite cells of max_i |f_i - f^eq_i(rho_b, rho_b u_b)|
 *            (0 when no cell is finite)
 *   out[6] = number of cells with a non-finite population
 * The sums run over every cell, so a non-finite cell makes them non-finite;
 * a cell is finite when all nine of its populations are.
 */
int oracle_diagnostics(int64_t nx, int64_t ny, const double *f, double rho_b,
                       double ux_b, double uy_b, double *out) {
  setup();
  if (nx < 1 || ny < 1 || !f || !out) return -1;
  const int64_t N = nx * ny;
  double fb[Q];
  feq(rho_b, rho_b * ux_b, rho_b * uy_b, fb);
  double s_r = 0.0, s_jx = 0.0, s_jy = 0.0, s_r2 = 0.0, s_j2 = 0.0, mx = 0.0, bad = 0.0;
  for (int64_t c = 0; c < N; ++c) {
    double rho = 0.0, jx = 0.0, jy = 0.0, dmax = 0.0;
    int finite = 1;
    for (int i = 0; i < Q; ++i) {
      const double v = f[i * N + c];
      rho += v;
      jx += CX[i] * v;
      jy += CY[i] * v;
      if (!isfinite(v)) finite = 0;
      const double d = fabs(v - fb[i]);
      if (d > dmax) dmax = d;
    }
    const double dr = rho - rho_b, djx = jx - rho_b * ux_b, djy = jy - rho_b * uy_b;
    s_r += dr;
    s_jx += djx;
    s_jy += djy;
    s_r2 += dr * dr;
    s_j2 += djx * djx + djy * djy;
    if (finite) {
      if (dmax > mx) mx = dmax;
    } else {
      bad += 1.0;
    }
  }
  out[0] = s_r;
  out[1] = s_jx;
  out[2] = s_jy;
  out[3] = s_r2;
  out[4] = s_j2;
  out[5] = mx;
  out[6] = bad;
  return 0;
}

/* Copies of the oracle's matrices, velocities and weights for the tests. */
int oracle_tables(double *M_out, double *Minv_out, int *cx, int *cy,
                  double *w) {
  setup();
  for (int i = 0; i < Q; ++i) {
    for (int j = 0; j < Q; ++j) {
      M_out[i * Q + j] = M_D2Q9[i][j];
      Minv_out[i * Q + j] = MINV[i][j];
    }
    cx[i] = CX[i];
    cy[i] = CY[i];
    w[i] = W[i];
  }
  return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
