/*
 * lbm3.h -- C ABI of the three-dimensional D3Q15 lattice of liblbm.so: the
 * MRT scheme with the absorbing-layer damping term of Xu & Sagaut,
 * "Analysis of the absorbing layers for the weakly-compressible lattice
 * Boltzmann schemes" (arXiv:1203.6350), Section 2, with the 15-velocity
 * transform matrix of Appendix A.2.
 *
 * Conventions as in lbm.h (status codes, storage modes, damping variants
 * LBM_VARIANT_*, combine modes, the thread-local lbm_last_error, one thread
 * per handle at a time). Host arrays are FP64 [nz][ny][nx], x fastest;
 * populations [15][nz][ny][nx] in the velocity order of the columns of M's
 * rows 1-3: 0 rest; 1, 2 = +x, -x; 3, 4 = +y, -y; 5, 6 = +z, -z; 7..14 the
 * diagonals (sx, sy, sz) = (+++), (-++), (+-+), (--+), (++-), (-+-), (+--),
 * (---). Relaxation rates s[15] follow M's rows (rho, jx, jy, jz, e, eps,
 * qx, qy, qz, 3pxx, pww, pxy, pyz, pzx, mxyz). The lattice is periodic in
 * all three directions. The step runs one cell per thread, reading and
 * writing every stored element once per step.
 */
#ifndef LBM3_H
#define LBM3_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3_config {
  int64_t nx, ny, nz;   /* >= 1 each, nx * ny * nz < 2^31                    */
  double rho_base;      /* deviation base f^eq(rho_base, u_base), > 0        */
  double ux_base, uy_base, uz_base;
  double s[15];         /* diagonal of S, each in [0, 2]                      */
  double shift_n, shift_m; /* shifts of rho*, j* (Sec. 2.2; 0.5 in the paper) */
  int32_t storage;      /* LBM_STORAGE_F64 / F32 / F16                        */
  int32_t variant;      /* LBM_VARIANT_NONE / I / II / III / VISC             */
  double f16_scale;     /* F16 only: amplitude of the deviations, > 0         */
  void *stream;         /* hipStream_t for all work of the handle, or NULL    */
} lbm3_config;

/* Reference (far-field) state q_ref = (rho^f, u^f), uniform (eq. eq:reff). */
typedef struct lbm3_qref {
  double rho_f, ux_f, uy_f, uz_f;
} lbm3_qref;

typedef struct lbm3_handle lbm3_handle;

/* Allocate the two lattices and set f = f^eq(rho, u) from host fields
 * [nz][ny][nx] (each may be NULL: the base value). Synchronises. */
int lbm3_create(const lbm3_config *cfg, const double *rho, const double *ux,
                const double *uy, const double *uz, lbm3_handle **out);

/* Sponge strength chi >= 0 (finite; the viscosity variant: the ramp
 * coordinate in [0, 1]) as a field [nz][ny][nx] (NULL: 0 everywhere), and
 * the reference state (NULL: keep). Copied, not retained. */
int lbm3_set_sponge(lbm3_handle *h, const double *chi, const lbm3_qref *q);

/* Separable sponge: chi(x, y, z) = max or sum (combine = LBM_COMBINE_*) of
 * chi_x[nx], chi_y[ny], chi_z[nz] (a NULL profile counts as 0). */
int lbm3_set_sponge_separable(lbm3_handle *h, const double *chi_x, const double *chi_y,
                              const double *chi_z, int32_t combine, const lbm3_qref *q);

/* Enqueue n >= 0 steps on the handle's stream. */
int lbm3_step(lbm3_handle *h, int64_t n);
int lbm3_sync(lbm3_handle *h);

/* Full FP64 pre-collision populations [15][nz][ny][nx] (synchronises). */
int lbm3_get_populations(lbm3_handle *h, double *f);
int lbm3_set_populations(lbm3_handle *h, const double *f);

/* rho and u = j / rho of the pre-collision state, host [nz][ny][nx] (any
 * may be NULL); synchronises. */
int lbm3_moments(lbm3_handle *h, double *rho, double *ux, double *uy, double *uz);

/* Launch shape of the step: kernel 0 = one cell per thread (a workgroup
 * covers consecutive cells of one row); kernel 1 = two consecutive cells of
 * a row per thread (nx even); block = threads per workgroup, 64..512 in
 * steps of 64. Default: kernel 1 for FP16 storage when nx is even, else
 * kernel 0; block 256. Every shape gives bit-identical results. LBM_EINVAL
 * for an unavailable shape. */
int lbm3_set_tuning(lbm3_handle *h, int32_t kernel, int32_t block);
int lbm3_get_tuning(lbm3_handle *h, int32_t *kernel, int32_t *block);

/* Time every available launch shape on the handle's own lattice (reps >= 1
 * steps each, after one untimed step; the state is left as it was: each
 * candidate reads the current lattice and writes the other one), keep the
 * fastest and report it (any output may be NULL). Synchronises. */
int lbm3_autotune(lbm3_handle *h, int32_t reps, int32_t *kernel, int32_t *block,
                  double *ms_per_step);

/* Number of steps taken since creation or the last lbm3_set_populations. */
int lbm3_steps_done(lbm3_handle *h, int64_t *steps);

/* Free the handle (NULL is ignored). */
void lbm3_destroy(lbm3_handle *h);

#ifdef __cplusplus
}
#endif

#endif
