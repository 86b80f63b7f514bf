/*
 * lbm.h -- C ABI of liblbm.so: a D2Q9 multi-relaxation-time lattice
 * Boltzmann time stepper with the absorbing-layer damping terms of
 * H. Xu and P. Sagaut, "Analysis of the absorbing layers for the
 * weakly-compressible lattice Boltzmann schemes" (arXiv:1203.6350),
 * running on AMD Instinct MI355X (gfx950) through HIP.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Velocities are ordered as the columns of the paper's D2Q9 transform
 *   matrix M (Appendix A.1): c0=(0,0) c1=(1,0) c2=(0,1) c3=(-1,0) c4=(0,-1)
 *   c5=(1,1) c6=(-1,1) c7=(-1,-1) c8=(1,-1); delta t = 1; c_s^2 = 1/3.
 * - Fields are row-major [ny][nx] (x fastest); populations are [9][ny][nx].
 * - The lattice is periodic in x and y (lattice closure, Section 2.1).
 * - The state observed through this API is the pre-collision population
 *   f(x, t) of eq. blbs; one step is collision (with damping) followed by
 *   streaming, f_i(x + c_i, t + 1) = f'_i(x, t).
 * - Host pointers are read or written during the call only; the library
 *   never keeps them. Device pointers (the *_dev calls) are used on the
 *   handle's stream and must stay valid until that work completes.
 * - Every function returns LBM_OK (0) or a negative status; no C++ exception
 *   crosses the ABI. lbm_last_error() returns a thread-local description of
 *   the last failure on the calling thread.
 * - A handle must be used by one thread at a time; distinct handles may run
 *   concurrently on distinct streams.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define LBM_OK 0
#define LBM_EINVAL (-1)    /* bad argument (size, range, NULL, non-finite) */
#define LBM_ENOMEM (-2)    /* device or host allocation failed             */
#define LBM_EDEVICE (-3)   /* HIP runtime error or no usable gfx950 device */
#define LBM_EUNSTABLE (-4) /* the instability detector tripped             */
#define LBM_ESTATE (-5)    /* call not valid in the handle's current state */

/* ---- population storage ---------------------------------------------- */
/* All modes store deviations g_i = f_i - f_i^base from the base state
 * f^base = f^eq(rho_base, u_base) (u_base = 0 gives the rest weights
 * w_i rho_base). */
#define LBM_STORAGE_F64 0 /* FP64 storage, FP64 arithmetic                */
#define LBM_STORAGE_F32 1 /* FP32 storage, FP32 arithmetic                */
#define LBM_STORAGE_F16 2 /* FP16 storage of g_i / 2^e_i with 2^e_i the power
                             of two nearest to w_i f16_scale, FP32 arithmetic */

/* ---- damping variants (Section 2.2, Gamma = chi I, eq. eq:gamma) ------ */
#define LBM_VARIANT_NONE 0 /* plain scheme, eq. blbs                       */
#define LBM_VARIANT_I 1    /* f^ref = f^eq(q_ref), f* = f (Sec. 2.2.1)     */
#define LBM_VARIANT_II 2   /* f^ref = f^eq(q_ref), f* = f^eq(rho*,u*) (2.2.2) */
#define LBM_VARIANT_III 3  /* f^ref = f^L(q_ref), f* = f^L(rho*,u*) (2.2.3) */
#define LBM_VARIANT_VISC 4 /* comparison strategy of Sec. 4.1: no damping
                              term; the non-conserved rates ramp linearly to
                              1 in the layer, s_k + (1 - s_k) xi, where the
                              sponge arrays hold xi in [0, 1] instead of chi */

/* ---- separable sponge combination ------------------------------------ */
#define LBM_COMBINE_MAX 0 /* chi(x,y) = max(chi_x[x], chi_y[y]) */
#define LBM_COMBINE_SUM 1 /* chi(x,y) = chi_x[x] + chi_y[y]     */

typedef struct lbm_config {
  int64_t nx, ny;      /* lattice size, each >= 1; nx * ny * 9 < 2^31     */
  double rho_base;     /* base state of the stored deviations, > 0         */
  double ux_base, uy_base;
  double s[9];         /* diagonal of S in moment order (rho, jx, jy, e,
                          eps, qx, qy, pxx, pxy), each in [0, 2]
                          (Section 2.1); BGK is s[k] = s for all k         */
  double shift_n;      /* n of rho* = sum f + n dt sum F (Sec. 2.2)       */
  double shift_m;      /* m of rho* u* = sum c f + m dt sum c F            */
  int32_t storage;     /* LBM_STORAGE_*                                    */
  int32_t variant;     /* LBM_VARIANT_*                                    */
  double f16_scale;    /* amplitude scale sigma of LBM_STORAGE_F16, > 0    */
  void *stream;        /* hipStream_t for all work of the handle; NULL =
                          the default stream                               */
} lbm_config;

/* Reference (far-field) state q_ref = (rho^f, u^f), eqs. eq:reff, Sec. 3.2. */
typedef struct lbm_qref {
  double rho_f, ux_f, uy_f;
} lbm_qref;

typedef struct lbm_info {
  int64_t nx, ny;
  int64_t pitch;        /* elements between rows                            */
  int64_t plane_stride; /* elements between population planes               */
  int64_t steps_done;   /* steps taken since create / set_populations       */
  int32_t storage, variant;
  int32_t elem_bytes;   /* bytes per stored population element              */
  int32_t chi_mode;     /* 0 none, 1 2-D field, 2 separable                 */
  size_t device_bytes;  /* device memory held for both lattices + sponge    */
} lbm_info;

typedef struct lbm_handle lbm_handle;

/* Create a lattice and set f = f^eq(rho, u) (the initial state of the
 * pulse set-up, eq. pulseprofile). rho, ux, uy: host [ny][nx] FP64, or NULL
 * for the uniform base state. The library allocates and owns the device
 * memory. The sponge starts at chi = 0 with q_ref = base state.
 * Errors: EINVAL (sizes, rates outside [0,2], rho_base <= 0, non-finite or
 * non-positive rho), EDEVICE, ENOMEM. */
int lbm_create(const lbm_config *cfg, const double *rho, const double *ux,
               const double *uy, lbm_handle **out);

/* Re-initialise to f = f^eq(rho, u) from device FP64 fields [ny][nx], each
 * of which may be NULL for the base value (rho_base, ux_base, uy_base).
 * Asynchronous on the handle's stream; the fields are not validated and must
 * stay valid until the work completes. Resets steps_done to 0. */
int lbm_init_fields_dev(lbm_handle *h, const double *rho, const double *ux,
                        const double *uy);

/* Bytes of device memory one lattice pair needs (both lattices, padded). */
int lbm_required_bytes(const lbm_config *cfg, size_t *bytes);

/* As lbm_create, but the two population buffers are caller-owned device
 * memory (for instance torch tensors), each at least
 * lbm_required_bytes()/2 bytes and 256-byte aligned; they must outlive the
 * handle. */
int lbm_create_ext(const lbm_config *cfg, const double *rho, const double *ux,
                   const double *uy, void *dev_buf_a, void *dev_buf_b,
                   size_t bytes_each, lbm_handle **out);

/* Sponge strength chi(x) >= 0 as a full host field [ny][nx] (NULL means
 * chi = 0 everywhere) and the uniform reference state q (NULL keeps the
 * current one). Values are copied. sigma = chi sigma~ profiles of eq.
 * normalizedsigma and Table tab:sigma are built by the caller.
 * Errors: EINVAL (negative or non-finite chi, rho_f <= 0). */
int lbm_set_sponge(lbm_handle *h, const double *chi, const lbm_qref *q);

/* Separable sponge chi(x, y) = combine(chi_x[x], chi_y[y]) with host arrays
 * chi_x[nx], chi_y[ny] (either may be NULL for zeros); adds no per-cell
 * memory traffic. combine: LBM_COMBINE_*. */
int lbm_set_sponge_separable(lbm_handle *h, const double *chi_x,
                             const double *chi_y, int32_t combine,
                             const lbm_qref *q);

/* As lbm_set_sponge_separable with the profiles in device memory (FP64
 * chi_x[nx], chi_y[ny], either may be NULL for zeros), for callers that set
 * up lattices on a busy stream (a server admitting requests): everything is
 * enqueued on the handle's stream and the call does not wait. The profiles
 * are not validated (they must be finite and >= 0, and in [0, 1] for the
 * viscosity ramp) and must stay valid until the enqueued work completes. */
int lbm_set_sponge_separable_dev(lbm_handle *h, const double *chi_x,
                                 const double *chi_y, int32_t combine,
                                 const lbm_qref *q);

/* Enqueue n >= 0 time steps (collision with the damping term of the
 * handle's variant, then streaming) on the handle's stream and return
 * without waiting. */
int lbm_step(lbm_handle *h, int64_t n);

/* Wait for all work of the handle. Returns LBM_EUNSTABLE once the
 * instability detector (below) has tripped. */
int lbm_sync(lbm_handle *h);

/* ---- instability detector ---------------------------------------------
 * Type I relaxes its non-conserved moments at the effective rate s + chi
 * (Sec. 2.2.1, eq. effectrelax), so wherever s + chi > 2 the layer itself
 * amplifies the solution (the Von Neumann threshold of Sec. 3.3), and a run
 * past a stability limit grows until it overflows. The detector catches
 * this during lbm_step: with every_n >= 1, after each kernel launch that
 * brings the handle's step count to or past the next multiple of every_n,
 * a check kernel reads the stored state on the handle's stream and trips if
 * any cell holds a non-finite population or a deviation |f_i - f_i^base|
 * larger than max_dev: the same condition as lbm_diagnostics reporting
 * out[6] > 0 or out[5] > max_dev. (Launches of the K-step kernels advance K
 * steps, so a check can land up to K - 1 steps after the multiple.) Batch
 * ticks check their members the same way at the end of the tick. The first
 * trip keeps the step count at which it was seen; from then on lbm_sync,
 * lbm_moments and lbm_diagnostics complete their work (outputs written)
 * and return LBM_EUNSTABLE, until the detector is set again or the state is
 * replaced (lbm_set_populations, lbm_load_state, lbm_init_fields_dev).
 *
 * every_n: 0 switches the detector off (the default), otherwise the check
 *          period in steps. max_dev: > 0, or +INFINITY to check for
 *          non-finite values only. Errors: EINVAL (every_n < 0, max_dev
 *          not > 0 or NaN), ENOMEM (the 8-byte device trip word).
 *          Synchronises the handle's stream.
 * Cost: one read of the nine planes per check (about one step's reads). */
int lbm_set_detector(lbm_handle *h, int64_t every_n, double max_dev);

/* Step count of the first trip, or -1 while the detector has not tripped
 * (or is off). Synchronises; returns LBM_OK either way. */
int lbm_detector_status(lbm_handle *h, int64_t *tripped_at);

/* Raw pre-collision moments rho = sum_i f_i, u = sum_i c_i f_i / rho
 * (eq. q-macro) into host arrays [ny][nx] FP64 (any may be NULL).
 * Synchronises; LBM_EUNSTABLE once the detector has tripped (the arrays
 * are written all the same). */
int lbm_moments(lbm_handle *h, double *rho, double *ux, double *uy);

/* As lbm_moments into device arrays [ny][nx] FP64, asynchronous. */
int lbm_moments_dev(lbm_handle *h, double *rho, double *ux, double *uy);

/* FP64 reductions over the lattice of the pre-collision state, with
 * deviations taken from the base state:
 *   out[0] = sum drho, out[1] = sum djx, out[2] = sum djy,
 *   out[3] = sum drho^2, out[4] = sum |dj|^2,
 *   out[5] = max over the finite cells of max_i |f_i - f_i^base| (0 when no
 *   cell is finite), out[6] = number of cells holding a non-finite
 *   population (a non-finite cell also makes the sums non-finite).
 * E_L2 of Section 4.1 with rho_ref = rho_base is sqrt(out[3] / sum rho_ref^2).
 * Deterministic (fixed reduction order). Synchronises; LBM_EUNSTABLE once
 * the detector has tripped (out is written all the same). */
int lbm_diagnostics(lbm_handle *h, double out[7]);

/* As lbm_diagnostics into a device array of 7 doubles, asynchronous on the
 * handle's stream. */
int lbm_diagnostics_dev(lbm_handle *h, double *out7_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * lbm_diagnostics_dev without any allocation. lbm_diagnostics_dev
 * allocates its per-block partials (56 KiB) at its first call on a handle;
 * this variant takes them from a static device array of that fixed size
 * instead (one per device, held until the process ends, its address looked
 * up at the first call on each device). Same kernels and results, bit for
 * bit. Every call on one device shares that array: calls that overlap on
 * one device (different streams, or different host threads) race and must
 * be ordered by the caller. Errors: EINVAL (NULL argument, or a reduction
 * whose partials would exceed the array's size), EDEVICE. Asynchronous;
 * does not report the detector. */
int lbm_diagnostics_dev_noalloc(lbm_handle *h, double *out7_dev);

/* Full pre-collision populations f = f^base + g in FP64, host [9][ny][nx].
 * Synchronises. */
int lbm_get_populations(lbm_handle *h, double *f);

/* Replace the state by host populations f [9][ny][nx] FP64 (checkpoint
 * restore); resets steps_done to 0. Synchronises. */
int lbm_set_populations(lbm_handle *h, const double *f);

/* Raw checkpoint of the stored state: the nine planes of the current lattice
 * exactly as held on the device (storage precision, pull layout) plus the
 * step count. lbm_state_bytes gives the size; lbm_save_state copies into a
 * host buffer of that size, lbm_load_state restores it, so that a resumed
 * run continues bit for bit. Both synchronise. */
int lbm_state_bytes(lbm_handle *h, size_t *bytes);
int lbm_save_state(lbm_handle *h, void *host, size_t bytes);
int lbm_load_state(lbm_handle *h, const void *host, size_t bytes);

int lbm_get_info(lbm_handle *h, lbm_info *info);

/* ---- per-cell and time-averaged reference state ----------------------
 * The paper lets q_ref depend on space and time: a far field, or a
 * time-dependent mean of the macroscopic quantities (Sec. 1, eq. eq:sponge;
 * Sec. 2.2, eq. eq:reff and the discussion after it).
 *
 * lbm_set_qref_field: per-cell reference state, host [ny][nx] arrays
 * (rho_f > 0, all finite), copied to the device as the conserved moments
 * (rho^f, rho^f u^f) in the compute precision; it replaces the uniform q_ref
 * of lbm_set_sponge until cleared with three NULL arrays (which also sets
 * the averaging rate back to 0). While a field is set, the K-step kernels
 * of the tuning run only with the default-form parameters (conserved rates
 * s0 = s1 = s2 = 0 and shift_n = shift_m; for a running mean also a damped
 * variant I, II or III), lbm_step takes the one-cell-per-thread kernel
 * otherwise (same results either way); the handle cannot join a batch, and
 * the field is not part of lbm_save_state (read it with
 * lbm_get_qref_field). A running mean in the K-step kernels keeps a second
 * field buffer (allocated at the first such step).
 *
 * lbm_set_qref_average: after each step's collision the field follows the
 * cell's pre-collision conserved moments c = (rho, j) as an exponential
 * running mean, c^f <- c^f + alpha (c - c^f), alpha in [0, 1] (0: fixed
 * field, the default). Needs a field (LBM_ESTATE otherwise).
 *
 * lbm_get_qref_field: the current field as (rho^f, u^f = j^f / rho^f),
 * host [ny][nx]; synchronises. */
int lbm_set_qref_field(lbm_handle *h, const double *rho_f, const double *ux_f,
                       const double *uy_f);
int lbm_set_qref_average(lbm_handle *h, double alpha);
int lbm_get_qref_field(lbm_handle *h, double *rho_f, double *ux_f, double *uy_f);

/* ---- acoustic line source with outflow (Sec. 4.2) ---------------------
 * Turns the lattice into a channel in x: after each step's collision the
 * column x = 0 holds the source's equilibrium f^eq(rho_src(t), u_src),
 * rho_src(t) = rho0 + amp sin(2 pi freq t + phase), t = the step index the
 * step ends at (the handle's step count), freq in cycles per step; with
 * outflow = 1 the column x = nx - 1 holds a copy of column nx - 2 after the
 * collision (zero-gradient outflow). y stays periodic. Needs nx >= 3 and
 * rho0 - |amp| > 0; src = NULL (with outflow = 0) makes x periodic again.
 * While set, lbm_step runs the one-cell-per-thread kernel whatever the
 * tuning, and the handle cannot join a batch or take a reference field. */
typedef struct lbm_line_source {
  double rho0, amp, freq, phase, ux, uy;
} lbm_line_source;
int lbm_set_line_source(lbm_handle *h, const lbm_line_source *src, int32_t outflow);

/* ---- kernel tuning ----------------------------------------------------
 * Launch shape of the step kernel. Every choice computes the same per-cell
 * arithmetic, so results are bit-identical across tunings. */
typedef struct lbm_tuning {
  int32_t kernel;      /* 0: one cell per thread; 1: 16-byte vector rows
                          (4 cells FP32, 2 FP64, 8 FP16; needs nx % cells == 0,
                          otherwise the library falls back to 0);
                          2, 3, 4: that many time steps per launch (each
                          64-lane wave owns a strip of 64 - 2 * kernel
                          columns of a chunk of rows, the block's waves take
                          adjacent strips; the lattice is read and written
                          once per launch; a shorter remainder of steps
                          runs as one launch of that many steps, a single
                          remaining step with kernel 0; rows of 2^32
                          bytes or more (FP64 with nx >= 2^29, FP32 with
                          nx = 2^30) always run with kernel 0: the strips
                          address a row with 32-bit byte offsets and
                          ranges)                                            */
  int32_t block;       /* threads per block: 64, 128, 256 or 512 (FP64
                          storage with kernel 4: at most 256)               */
  int32_t nontemporal; /* 1: streaming stores (vector kernel only)           */
  int32_t rows;        /* kernels 2-4: rows per chunk, 1..4096, or 0 for
                          the height at which all blocks are resident at
                          once; ignored by kernels 0 and 1                  */
} lbm_tuning;

int lbm_set_tuning(lbm_handle *h, const lbm_tuning *t);
int lbm_get_tuning(lbm_handle *h, lbm_tuning *t);

/* Time every candidate launch shape on the handle's own lattice (reps
 * launches each, after two warm-up launches; the state is not advanced),
 * keep the fastest and return it with its mean time per time step in ms.
 * best and best_ms may be NULL. Synchronises. The timings depend on the
 * current state: a field whose deviations are still mostly exact zeros
 * (just initialised from localised pulses) runs faster and can rank the
 * shapes differently from the developed field, so tune after some steps. */
int lbm_autotune(lbm_handle *h, int32_t reps, lbm_tuning *best, double *best_ms);

/* Release all resources of the handle; NULL is accepted. */
void lbm_destroy(lbm_handle *h);

const char *lbm_last_error(void);

/* ---- batched stepping of many lattices --------------------------------
 * A batch steps many independent lattices (each an lbm_handle with its own
 * size, relaxation rates, damping variant, sponge and reference state) with
 * persistent launches captured in HIP graphs: by default each launch
 * advances every member by K steps (the strip kernel over a table of work
 * items, which its workgroups take one by one, tallest first; K = 4 for
 * FP32 storage, 3 for FP64 and FP16) and a member's
 * remainder of fewer than K steps in a tick runs as one-step launches over
 * a table of 256-cell tiles. A batch whose work items do not fill the
 * device once (few or small members) runs its ticks as one-step tile
 * launches only, which spread it over the whole device. All members must
 * share the storage mode and the device. Members may carry a fixed per-cell
 * reference state (lbm_set_qref_field; Sec. 2.2); members with a running-
 * mean reference (lbm_set_qref_average with alpha != 0), a line source or
 * rows of 2^32 bytes or more are refused (LBM_EINVAL), at creation and,
 * for the first two, which can be set on a member later, at every tick
 * before it enqueues anything. Each member's result is bit-identical to
 * stepping it alone with lbm_step.
 * While a batch has work in flight its members must not be used on their
 * own; lbm_batch_sync makes them usable again. Member parameters (sponge,
 * q_ref and its per-cell field, tuning) are read at every tick, so they may
 * change between ticks.
 * The batch keeps pointers to the members: destroy the batch before them. */
typedef struct lbm_batch lbm_batch;

/* members: count >= 1 distinct handles; stream: hipStream_t for the batch
 * (NULL: the batch creates its own stream). */
int lbm_batch_create(lbm_handle *const *members, int32_t count, void *stream,
                     lbm_batch **out);

/* Advance every member by n >= 0 steps (enqueued; returns without waiting). */
int lbm_batch_step(lbm_batch *b, int64_t n);

/* One tick of `tick` >= 1 launches in which member i takes member_steps[i]
 * steps (0 <= member_steps[i] <= tick; NULL means tick for all). Members
 * that finish early keep their state for the rest of the tick. */
int lbm_batch_tick(lbm_batch *b, int32_t tick, const int32_t *member_steps);

/* Replace the member list (same rules as lbm_batch_create) for the ticks
 * enqueued after this call. Stream-ordered: the tile and item tables are
 * copied on the batch stream behind the work already enqueued there and
 * rewritten in place when they fit, so graphs captured earlier stay valid
 * and the call does not wait for the device; it waits only when a table
 * outgrows its buffer, and for a member whose own stream is not the batch
 * stream (so that work enqueued for it there is done). A handle dropped
 * from the list may be destroyed once the ticks that still advance it have
 * completed. */
int lbm_batch_set_members(lbm_batch *b, lbm_handle *const *members,
                          int32_t count);

/* Persistent workgroups per compute unit of the one-step tile kernel
 * (1..64, default 8). */
int lbm_batch_set_grid(lbm_batch *b, int32_t blocks_per_cu);

/* Launch shape of the batch (see lbm_tuning): kernel 0 or 1 = one-step
 * launches over 256-cell tiles only (block and rows ignored); kernel 2, 3
 * or 4 = that many steps per launch of the strip kernel, `block` threads per
 * workgroup (64, 128, 256 or 512, at most 256 for FP64 storage with 4 steps:
 * adjacent strips of one member; LBM_EINVAL otherwise), `rows`
 * rows per work item (1..4096, or 0 for an automatic height: the member
 * rows over the resident workgroups, so that a launch has an item for each,
 * clamped to 8..64 rows). Default: K as above, block 128, rows 0. Rebuilds
 * the work-item table; synchronises the batch stream. Results are
 * bit-identical for every shape. */
int lbm_batch_set_tuning(lbm_batch *b, const lbm_tuning *t);
int lbm_batch_get_tuning(lbm_batch *b, lbm_tuning *t);

/* Smallest number of strip work items for which a tick uses K-step launches
 * (fewer: one-step tile launches only). -1 (default): the number of
 * strip-kernel workgroups resident on the device at once; 0: always. */
int lbm_batch_set_min_items(lbm_batch *b, int32_t min_items);

/* Wait for the batch's work. Returns LBM_EUNSTABLE when the detector of a
 * member (set with lbm_set_detector before the tick) has tripped; which
 * ones and when is given by lbm_batch_detector_status. */
int lbm_batch_sync(lbm_batch *b);

/* Per member (in member-list order): the step count of its detector's first
 * trip, or -1 (not tripped, or no detector). tripped_at: host array of the
 * member count. Synchronises; returns LBM_OK either way. */
int lbm_batch_detector_status(lbm_batch *b, int64_t *tripped_at);

void lbm_batch_destroy(lbm_batch *b);

/* ---- Von Neumann analysis (Section 3.2, eqs. eq:linearized, sec:matrix) --
 * For the scheme linearised about f^eq(q_ref) with uniform chi, computes per
 * wavenumber k = (kx, ky) the amplification matrix with the streaming phase
 * restored, G(k) = diag(exp(-i k.c_j)) M^-1 A_m M, where
 * A_m = I + S (J D P - I) - chi X is the moment-space Jacobian of the
 * collision (P: projection on rho, jx, jy; D: derivative of rho*, j*;
 * J: derivative of m^eq; X = I for Type I, J D P for Type II, L D P for
 * Type III with L the derivative of m^L), and its eigenvalues
 * lambda = exp(-i omega), sorted by (-|lambda|, arg lambda).
 * All arithmetic is FP64 on the device. */
typedef struct lbm_vn_params {
  double s[9];
  double shift_n, shift_m;
  double chi;
  double rho_f, ux_f, uy_f;
  int32_t variant;
  int32_t pad_;
} lbm_vn_params;

/* kx, ky: nk wavenumbers; eig: [nk][9][2] (re, im); G: NULL or
 * [nk][9][9][2]. Pointers are host memory. Synchronous. */
int vn_amplification(const lbm_vn_params *p, int64_t nk, const double *kx,
                     const double *ky, double *eig, double *G);

/* Device-pointer variant, asynchronous on stream (hipStream_t, may be NULL):
 * nparams parameter sets, each evaluated on the same nk wavenumbers;
 * params is host memory, kx/ky/eig/G are device memory with eig
 * [nparams][nk][9][2] and G NULL or [nparams][nk][9][9][2]. */
int vn_amplification_dev(const lbm_vn_params *params, int64_t nparams,
                         int64_t nk, const double *kx, const double *ky,
                         double *eig, double *G, void *stream);

/* ---- device bandwidth probe ------------------------------------------
 * Copies `bytes` (multiple of 16) from src to dst device memory with the
 * library's streaming copy kernel on `stream`; used to calibrate the
 * achievable HBM bandwidth and the traffic counters. */
int lbm_device_copy(void *dst, const void *src, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
