// lbm_internal.h -- host-side structures shared by the C ABI and the kernel
// launchers of liblbm. Not installed; the public interface is include/lbm.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbm {

// Everything a step kernel needs, in FP64; launchers convert to the compute
// precision of the storage mode.
struct StepConfig {
  int nx, ny;
  int64_t pitch;         // elements between rows
  int64_t plane_stride;  // elements between population planes
  int storage;           // LBM_STORAGE_*
  int variant;           // LBM_VARIANT_*
  int chi_mode;          // ChiMode
  double s[9];
  double n, m;
  double rho_b, ubx, uby;
  double dcf[3];         // q_ref - base, conserved moments
  double f16_scale;
  const void *chi_field; // [ny][pitch] compute type, CHI_FIELD
  const void *chi_x;     // [nx] compute type
  const void *chi_y;     // [ny] compute type
  int kernel;            // KERNEL_GENERIC, KERNEL_VEC, or 2..4 time steps per launch
  int block;             // threads per block: 64, 128, 256 or 512
  int nontemporal;       // 1: streaming (non-temporal) stores (vector kernel)
  int rows;              // rows per chunk of the multi-step kernel (0: fit the device)
  // per-cell reference state: three planes [3][qps] of (d rho^f, d j^f_x,
  // d j^f_y), each [ny][pitch], compute type; NULL: uniform dcf above
  void *qfield;
  void *qfield_out;      // second field buffer of the strip kernels' running mean
  int64_t qps;
  double qalpha;         // running-mean rate of the reference (0: fixed)
  // channel in x (line source at x = 0, optional outflow at x = nx - 1)
  int channel;           // 0: periodic in x
  int outflow;
  double src_dev[9];     // post-collision deviations stored at x = 0 this step
};

enum { KERNEL_GENERIC = 0, KERNEL_VEC = 1, KERNEL_MULTI_MIN = 2, KERNEL_MULTI_MAX = 4 };

// Largest workgroup of the single-lattice K-step kernel: FP64 storage with
// four steps per launch is built for one wave per SIMD (its registers do
// not fit two), so its workgroups take at most 256 threads.
constexpr int multi_step_max_block(int storage, int k) { return storage == 0 && k == 4 ? 256 : 512; }

// The strip kernels address a lane's column within a row as a 32-bit byte
// offset and read a row through a buffer range of the row's byte count (a
// 32-bit field), so they take rows of fewer than 2^32 bytes (FP64 rows of
// 2^29 cells or more, FP32 rows of 2^30, run in the one-cell kernels).
inline bool strip_row_fits(int64_t nx, int storage) {
  const int64_t eb = storage == 0 ? 8 : (storage == 1 ? 4 : 2);
  return nx * eb < (int64_t(1) << 32);
}

// The multi-step strip kernels take this configuration: rows that fit
// their byte offsets, no channel, and a
// per-cell reference state only when the collision has its default form
// (conserved rates 0, n = m in the compute precision). A fixed reference is
// ignored by the undamped and viscosity-ramp variants; a running mean (which
// needs the second field buffer qfield_out) is taken by the damped variants.
inline bool multi_step_supports(const StepConfig &c) {
  if (c.channel || !strip_row_fits(c.nx, c.storage)) return false;
  if (!c.qfield) return true;
  const bool damped = c.variant >= 1 && c.variant <= 3;
  if (c.qalpha == 0.0 && !damped) return true;
  if (!damped) return false;
  if (c.storage == 0)
    return c.s[0] == 0.0 && c.s[1] == 0.0 && c.s[2] == 0.0 && c.n == c.m;
  return (float)c.s[0] == 0.0f && (float)c.s[1] == 0.0f && (float)c.s[2] == 0.0f &&
         (float)c.n == (float)c.m;
}
// k = 2..4 time steps in one launch (src at t -> dst at t + k).
hipError_t launch_multi_steps(const StepConfig &c, int k, const void *src, void *dst,
                              hipStream_t stream);
// per storage type (lbm_strip_f64/f32/f16.hip)
// Per storage type and step count (lbm_strip_f64/f32/f16.hip, one object
// per K): the single-lattice strip launch, the batched one and its
// resident workgroups per CU.
#define LBM_STRIP_DECL(ST, K)                                                                    \
  hipError_t launch_multi_##ST##_k##K(const StepConfig &c, const void *src, void *dst,          \
                                      hipStream_t stream);                                       \
  hipError_t launch_batch_multi_##ST##_k##K(int nw, int form, const BatchDomain *doms,          \
                                            const int4 *items, int *nitems, int grid,     \
                                            int j, hipStream_t stream);                          \
  int batch_multi_per_cu_##ST##_k##K(int nw, int form);
#define LBM_STRIP_DECL_K(ST) LBM_STRIP_DECL(ST, 2) LBM_STRIP_DECL(ST, 3) LBM_STRIP_DECL(ST, 4)
bool vec_supported(const StepConfig &c);
// FP16 mode: stored value = deviation / storage_scale (a power of two).
double storage_scale(const StepConfig &c, int i);

// Launchers (lbm_kernels.hip). All enqueue on `stream` and return the HIP
// status of the launch.
hipError_t launch_step(const StepConfig &c, const void *src, void *dst,
                       hipStream_t stream);
hipError_t launch_init(const StepConfig &c, const double *rho,
                       const double *ux, const double *uy, void *dst,
                       hipStream_t stream);
hipError_t launch_set_populations(const StepConfig &c, const double *f,
                                  void *dst, hipStream_t stream);
hipError_t launch_get_populations(const StepConfig &c, const void *src,
                                  double *f, hipStream_t stream);
hipError_t launch_moments(const StepConfig &c, const void *src, double *rho,
                          double *ux, double *uy, hipStream_t stream);
// partials: device scratch of at least diag_partials_bytes(c) bytes;
// out7: device array of 7 doubles.
size_t diag_partials_bytes(const StepConfig &c);
// Device address and size of the static partials workspace of the
// allocation-free diagnostics call on `device` (looked up once per device).
hipError_t diag_scratch(int device, double **ptr, size_t *bytes);
hipError_t launch_diagnostics(const StepConfig &c, const void *src,
                              double *partials, double *out7,
                              hipStream_t stream);
hipError_t launch_copy(void *dst, const void *src, size_t bytes,
                       hipStream_t stream);

// Instability detector: scans the nine stored planes of one lattice and, if
// any deviation is non-finite or larger than max_dev in magnitude, lowers
// *trip (and *trip2 when not NULL) to `step` (atomic minimum; "not tripped"
// is ~0ull).
struct CheckDesc {
  const void *lat;
  unsigned long long *trip;
  unsigned long long *trip2;
  int64_t n;               // cells per plane (nx * ny; rows are contiguous)
  int64_t ps;              // elements between planes
  unsigned long long step;
  double max_dev;
  double scale[9];         // storage scale of each plane (FP16 mode)
};
constexpr unsigned long long TRIP_NONE = ~0ull;
void fill_check_desc(const StepConfig &c, const void *lat, CheckDesc &d);
hipError_t launch_check(int storage, const CheckDesc &d, hipStream_t stream);
// descs_dev: device array of ndesc descriptors (one member each); max_cells:
// the largest n among them.
hipError_t launch_check_batch(int storage, const CheckDesc *descs_dev, int ndesc,
                              int64_t max_cells, hipStream_t stream);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v,
                           hipStream_t stream);
hipError_t launch_fill_i32(int *p, int64_t n, int v, hipStream_t stream);
// FP64 device profile (or NULL: zeros) -> n values of the storage's compute
// type (FP64 for FP64 storage, FP32 otherwise).
hipError_t launch_convert_profile(int storage, const double *src, void *dst, int64_t n,
                                  hipStream_t stream);
int elem_bytes_of(int storage);

// Batched stepping (lbm_batch.hip). One descriptor per member domain.
constexpr int BATCH_TILE = 256;  // cells per tile = threads per workgroup
struct BatchDomain {
  void *lat[2];          // lat[parity] is current at the start of a tick
  const void *chi_field; // compute type, CHI_FIELD
  const void *chi_x, *chi_y;
  int64_t pitch, ps;
  int nx, ny, variant, chi_mode;
  int parity;            // current lattice at the start of the tick
  int stop_at;           // steps this domain takes in the tick
  double s[9];
  double n, m, rho_b, ubx, uby;
  double dcf[3];
  double scale[9], inv_scale[9];
  // fixed per-cell reference state (compute type, [3][qps], rows of pitch),
  // set for the damped variants when the member has one, else NULL
  const void *qf;
  int64_t qps;
};
// Forms of the batched strip kernel (bit mask): BATCH_DEF, every member has
// the default form's parameters (conserved rates 0, n = m in the compute
// precision); BATCH_QF, some member has a per-cell reference state;
// BATCH_SEPMAX, every member's sponge is the separable max form (compiled
// in, where otherwise the form is chosen per item at run time).
constexpr int BATCH_DEF = 1;
constexpr int BATCH_QF = 2;
constexpr int BATCH_SEPMAX = 4;
// One step (launch k of a tick) over the tile table. kmulti = 0: the tick
// runs as one-step launches only; kmulti = K: the tick's bulk ran as K-step
// launches and this launch takes step k of each member's remainder.
hipError_t launch_batch(int storage, const BatchDomain *doms, const int2 *tiles,
                        const int *ntiles_dev, int grid, int k, int kmulti,
                        hipStream_t stream);
// K = k steps (launch j of a tick) over the strip work items (int4: member,
// first strip of the group, first row, rows), workgroups of nw waves.
// nitems: device ints, [0] the item count, [1 + j] the item ticket of
// launch j (zeroed before the launch).
// form: BATCH_DEF, BATCH_QF and BATCH_SEPMAX bits, which select that form of
// the kernel.
hipError_t launch_batch_multi(int storage, int k, int nw, int form, const BatchDomain *doms,
                              const int4 *items, int *nitems, int grid, int j,
                              hipStream_t stream);
int batch_multi_per_cu(int storage, int k, int nw, int form);
LBM_STRIP_DECL_K(f64)
LBM_STRIP_DECL_K(f32)
LBM_STRIP_DECL_K(f16)

// Three-dimensional D3Q15 step (lbm3_kernels.hip): everything a kernel
// needs in FP64, converted per launch to the compute precision.
struct Step3Config {
  int nx, ny, nz;
  int64_t pitch;         // elements between rows (slices are ny rows)
  int64_t plane_stride;  // elements between population planes
  int storage, variant, chi_mode;
  double s[15];
  double n, m;
  double rho_b, ub[3];
  double dcf[4];         // q_ref - base, conserved moments
  double f16_scale;
  const void *chi_field; // [nz][ny][pitch] compute type
  const void *chi_x, *chi_y, *chi_z;
  int kernel;            // 0: one cell per thread; 1: two cells of a row per thread (nx even)
  int block;             // threads per workgroup, 64..512, a multiple of 64
};
hipError_t launch_step3(const Step3Config &c, const void *src, void *dst, hipStream_t stream);
hipError_t launch_init3(const Step3Config &c, const double *rho, const double *ux,
                        const double *uy, const double *uz, void *dst, hipStream_t stream);
hipError_t launch_setpop3(const Step3Config &c, const double *f, void *dst, hipStream_t stream);
hipError_t launch_getpop3(const Step3Config &c, const void *src, double *f, double *rho,
                          double *ux, double *uy, double *uz, hipStream_t stream);

// Von Neumann (lbm_vn.hip).
struct VnParamsDev {
  double s[9];
  double n, m, chi, rho_f, ux_f, uy_f;
  int variant;
  int pad_;
};
hipError_t launch_vn(const VnParamsDev *params_dev, int nparams, int64_t nk,
                     const double *kx, const double *ky, double *eig,
                     double *G, hipStream_t stream);

}  // namespace lbm
