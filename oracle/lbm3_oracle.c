/*
 * lbm3_oracle.c -- plain, slow FP64 CPU oracle for the three-dimensional
 * D3Q15 MRT lattice Boltzmann time step with the absorbing-layer damping
 * term of H. Xu and P. Sagaut, "Analysis of the absorbing layers for the
 * weakly-compressible lattice Boltzmann schemes" (arXiv:1203.6350): the
 * scheme of Section 2 with the 15-velocity transform matrix of Appendix A.2.
 *
 * TEST INFRASTRUCTURE. This file exists to check the HIP implementation.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it. It shares no code, header, table or helper with the HIP path
 * (nor with the D2Q9 oracle), and the HIP path never calls it.
 *
 * One step, for every cell x of a periodic nx-by-ny-by-nz lattice, state
 * f_i(x,t) pre-collision, i = 0..14:
 *   1. m = M f (Appendix A.2)
 *   2. rho* = (rho + n chi rho^f)/(1 + n chi), j* = (j + m chi j^f)/(1 + m chi)
 *      (the implicit shifted quantities of Sections 2.2.1-2.2.3, solved
 *      exactly because every damping force has sum F = chi (rho^f - rho*) and
 *      sum c F = chi (j^f - j*))
 *   3. m^eq* = M f^eq(rho*, j*), f^eq in velocity space
 *   4. d = 0 (none); chi (M f^eq(c^f) - m) (I); chi (M f^eq(c^f) - m^eq*) (II);
 *      chi (M f^L(c^f) - M f^L(c*)) (III); variant 4 = the viscosity ramp of
 *      Section 4.1 (rates k >= 4 ramped to 1 by xi, carried in chi)
 *   5. m' = m + S o (m^eq* - m) + d
 *   6. f' = M^-1 m', M^-1 by Gauss-Jordan elimination
 *   7. streaming f_i(x, t+1) = f'_i(x - c_i), periodic
 *
 * Readings where the paper is silent: the standard second-order equilibrium
 * with c_s^2 = 1/3, f^eq_i = w_i [rho + 3 c.j + 9/2 (c.j)^2/rho - 3/2 |j|^2/rho],
 * f^L_i = w_i [rho + 3 c.j], with the D3Q15 weights 2/9 (rest), 1/9 (the six
 * axis velocities), 1/72 (the eight diagonals); velocities follow rows 1-3 of
 * M. The conserved rows are 0-3; the viscosity ramp acts on rows 4-14.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q3 15

/* Appendix A.2: rows (rho, jx, jy, jz, e, eps, qx, qy, qz, 3pxx, pww, pxy,
 * pyz, pzx, mxyz). */
static const double M3[Q3][Q3] = {
    { 1,  1,  1,  1,  1,  1,  1, 1,  1,  1,  1,  1,  1,  1,  1},
    { 0,  1, -1,  0,  0,  0,  0, 1, -1,  1, -1,  1, -1,  1, -1},
    { 0,  0,  0,  1, -1,  0,  0, 1,  1, -1, -1,  1,  1, -1, -1},
    { 0,  0,  0,  0,  0,  1, -1, 1,  1,  1,  1, -1, -1, -1, -1},
    {-2, -1, -1, -1, -1, -1, -1, 1,  1,  1,  1,  1,  1,  1,  1},
    {16, -4, -4, -4, -4, -4, -4, 1,  1,  1,  1,  1,  1,  1,  1},
    { 0, -4,  4,  0,  0,  0,  0, 1, -1,  1, -1,  1, -1,  1, -1},
    { 0,  0,  0, -4,  4,  0,  0, 1,  1, -1, -1,  1,  1, -1, -1},
    { 0,  0,  0,  0,  0, -4,  4, 1,  1,  1,  1, -1, -1, -1, -1},
    { 0,  2,  2, -1, -1, -1, -1, 0,  0,  0,  0,  0,  0,  0,  0},
    { 0,  0,  0,  1,  1, -1, -1, 0,  0,  0,  0,  0,  0,  0,  0},
    { 0,  0,  0,  0,  0,  0,  0, 1, -1, -1,  1,  1, -1, -1,  1},
    { 0,  0,  0,  0,  0,  0,  0, 1,  1, -1, -1, -1, -1,  1,  1},
    { 0,  0,  0,  0,  0,  0,  0, 1, -1,  1, -1, -1,  1, -1,  1},
    { 0,  0,  0,  0,  0,  0,  0, 1, -1, -1,  1, -1,  1,  1, -1}};

static int C3X[Q3], C3Y[Q3], C3Z[Q3];
static const double W3[Q3] = {2.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,
                              1.0 / 9,  1.0 / 9,  1.0 / 72, 1.0 / 72, 1.0 / 72,
                              1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72};
static double M3INV[Q3][Q3];
static int g3_ready = 0;

static void setup3(void) {
  if (g3_ready) return;
  for (int j = 0; j < Q3; ++j) {
    C3X[j] = (int)M3[1][j];
    C3Y[j] = (int)M3[2][j];
    C3Z[j] = (int)M3[3][j];
  }
  /* Gauss-Jordan elimination with partial pivoting on [M | I] */
  double a[Q3][2 * Q3];
  for (int i = 0; i < Q3; ++i)
    for (int j = 0; j < 2 * Q3; ++j) a[i][j] = j < Q3 ? M3[i][j] : (j - Q3 == i ? 1.0 : 0.0);
  for (int col = 0; col < Q3; ++col) {
    int piv = col;
    for (int r = col + 1; r < Q3; ++r)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (piv != col)
      for (int j = 0; j < 2 * Q3; ++j) {
        double t = a[col][j];
        a[col][j] = a[piv][j];
        a[piv][j] = t;
      }
    const double p = a[col][col];
    for (int j = 0; j < 2 * Q3; ++j) a[col][j] /= p;
    for (int r = 0; r < Q3; ++r) {
      if (r == col || a[r][col] == 0.0) continue;
      const double fct = a[r][col];
      for (int j = 0; j < 2 * Q3; ++j) a[r][j] -= fct * a[col][j];
    }
  }
  for (int i = 0; i < Q3; ++i)
    for (int j = 0; j < Q3; ++j) M3INV[i][j] = a[i][Q3 + j];
  g3_ready = 1;
}

static void mv3(const double A[Q3][Q3], const double *x, double *y) {
  for (int i = 0; i < Q3; ++i) {
    double acc = 0.0;
    for (int j = 0; j < Q3; ++j) acc += A[i][j] * x[j];
    y[i] = acc;
  }
}

static void feq3(double rho, double jx, double jy, double jz, double *out) {
  for (int i = 0; i < Q3; ++i) {
    const double cj = C3X[i] * jx + C3Y[i] * jy + C3Z[i] * jz;
    out[i] = W3[i] * (rho + 3.0 * cj + 4.5 * cj * cj / rho -
                      1.5 * (jx * jx + jy * jy + jz * jz) / rho);
  }
}

static void flin3(double rho, double jx, double jy, double jz, double *out) {
  for (int i = 0; i < Q3; ++i)
    out[i] = W3[i] * (rho + 3.0 * (C3X[i] * jx + C3Y[i] * jy + C3Z[i] * jz));
}

enum { V3_NONE = 0, V3_I = 1, V3_II = 2, V3_III = 3, V3_VISC = 4 };

/* One collision of one cell. rf, uf[3]: reference state. */
static void collide3(const double *fin, double chi, double rf, const double *uf,
                     const double *s, double n, double m, int variant, double *fout) {
  double mom[Q3], meq[Q3], d[Q3], tmp[Q3], a[Q3], b[Q3], mp[Q3], sk[Q3];
  const double xi = chi;
  if (variant == V3_NONE || variant == V3_VISC) chi = 0.0;
  mv3(M3, fin, mom);
  const double rho = mom[0], jx = mom[1], jy = mom[2], jz = mom[3];
  const double jfx = rf * uf[0], jfy = rf * uf[1], jfz = rf * uf[2];
  const double rs = (rho + n * chi * rf) / (1.0 + n * chi);
  const double jsx = (jx + m * chi * jfx) / (1.0 + m * chi);
  const double jsy = (jy + m * chi * jfy) / (1.0 + m * chi);
  const double jsz = (jz + m * chi * jfz) / (1.0 + m * chi);
  feq3(rs, jsx, jsy, jsz, tmp);
  mv3(M3, tmp, meq);
  for (int k = 0; k < Q3; ++k) d[k] = 0.0;
  if (variant == V3_I || variant == V3_II) {
    feq3(rf, jfx, jfy, jfz, tmp);
    mv3(M3, tmp, a);
    for (int k = 0; k < Q3; ++k) d[k] = chi * (a[k] - (variant == V3_I ? mom[k] : meq[k]));
  } else if (variant == V3_III) {
    flin3(rf, jfx, jfy, jfz, tmp);
    mv3(M3, tmp, a);
    flin3(rs, jsx, jsy, jsz, tmp);
    mv3(M3, tmp, b);
    for (int k = 0; k < Q3; ++k) d[k] = chi * (a[k] - b[k]);
  }
  for (int k = 0; k < Q3; ++k) sk[k] = s[k];
  if (variant == V3_VISC)
    for (int k = 4; k < Q3; ++k) sk[k] = s[k] + (1.0 - s[k]) * xi;
  for (int k = 0; k < Q3; ++k) mp[k] = mom[k] + sk[k] * (meq[k] - mom[k]) + d[k];
  mv3(M3INV, mp, fout);
}

static inline int64_t wrap3(int64_t a, int64_t n) {
  a %= n;
  return a < 0 ? a + n : a;
}

/*
 * oracle3_step -- advance the pre-collision state f by nsteps steps.
 *   f    : [15][nz][ny][nx] FP64, x fastest; updated in place.
 *   chi  : [nz][ny][nx] sponge strength (or the ramp coordinate of the
 *          viscosity strategy), or NULL for 0.
 *   qref : {rho^f, u^f_x, u^f_y, u^f_z}, uniform.
 *   s    : 15 relaxation rates; n, m: shift parameters.
 */
int oracle3_step(int64_t nx, int64_t ny, int64_t nz, double *f, const double *chi,
                 const double *qref, const double *s, double n, double m, int variant,
                 int64_t nsteps, int nthreads) {
  setup3();
  if (nx < 1 || ny < 1 || nz < 1 || !f || !qref || !s || nsteps < 0) return -1;
  const int64_t N = nx * ny * nz;
  double *post = (double *)malloc(sizeof(double) * Q3 * N);
  if (!post) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  for (int64_t t = 0; t < nsteps; ++t) {
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
      double fin[Q3], fo[Q3];
      for (int i = 0; i < Q3; ++i) fin[i] = f[i * N + c];
      collide3(fin, chi ? chi[c] : 0.0, qref[0], qref + 1, s, n, m, variant, fo);
      for (int i = 0; i < Q3; ++i) post[i * N + c] = fo[i];
    }
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
      for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x)
          for (int i = 0; i < Q3; ++i) {
            const int64_t xs = wrap3(x - C3X[i], nx), ys = wrap3(y - C3Y[i], ny),
                          zs = wrap3(z - C3Z[i], nz);
            f[i * N + (z * ny + y) * nx + x] = post[i * N + (zs * ny + ys) * nx + xs];
          }
  }
  free(post);
  return 0;
}

/* Equilibrium populations of a field: rho, ux, uy, uz [ncell]; out [15][ncell]. */
int oracle3_feq_field(int64_t ncell, const double *rho, const double *ux, const double *uy,
                      const double *uz, double *out) {
  setup3();
  if (ncell < 0 || !rho || !ux || !uy || !uz || !out) return -1;
  for (int64_t c = 0; c < ncell; ++c) {
    double e[Q3];
    feq3(rho[c], rho[c] * ux[c], rho[c] * uy[c], rho[c] * uz[c], e);
    for (int i = 0; i < Q3; ++i) out[i * ncell + c] = e[i];
  }
  return 0;
}

/* One collision (no streaming) for independent cells: fin, fout [ncell][15];
 * chi [ncell] or NULL. */
int oracle3_collide(int64_t ncell, const double *fin, const double *chi, const double *qref,
                    const double *s, double n, double m, int variant, double *fout) {
  setup3();
  if (ncell < 0 || !fin || !fout || !qref || !s) return -1;
  for (int64_t c = 0; c < ncell; ++c)
    collide3(fin + Q3 * c, chi ? chi[c] : 0.0, qref[0], qref + 1, s, n, m, variant,
             fout + Q3 * c);
  return 0;
}

/* Tables for the tests: M, M^-1 (row-major 15x15), velocities, weights. */
void oracle3_tables(double *m_out, double *minv_out, int *cx, int *cy, int *cz, double *w) {
  setup3();
  for (int i = 0; i < Q3; ++i) {
    for (int j = 0; j < Q3; ++j) {
      m_out[i * Q3 + j] = M3[i][j];
      minv_out[i * Q3 + j] = M3INV[i][j];
    }
    cx[i] = C3X[i];
    cy[i] = C3Y[i];
    cz[i] = C3Z[i];
    w[i] = W3[i];
  }
}
