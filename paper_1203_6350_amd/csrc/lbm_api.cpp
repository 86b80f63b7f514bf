// lbm_api.cpp -- C ABI of liblbm (declared in include/lbm.h).
//
// Owns the device state of one lattice (two population lattices, the sponge
// arrays, diagnostic scratch), validates arguments, and enqueues the kernels
// of lbm_kernels.hip / lbm_vn.hip on the handle's stream. No arithmetic of
// the method runs on the host: the host only converts parameters and copies
// inputs and outputs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lbm.h"
#include "../../include/lbm3.h"
#include "lbm_device.h"
#include "lbm_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  (void)hipGetLastError();  // clear the sticky launch error
  return e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE;
}

#define HIP_TRY(expr, what)                  \
  do {                                       \
    hipError_t _e = (expr);                  \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

int check_device(int *dev_out) {
  // the architecture of a device is looked up once (hipGetDeviceProperties
  // takes milliseconds, and lattices are created per request when serving)
  constexpr int MAXDEV = 64;
  static std::atomic<int> arch_ok[MAXDEV] = {};  // 0 unknown, 1 gfx950, -1 other
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const int known = dev >= 0 && dev < MAXDEV ? arch_ok[dev].load(std::memory_order_relaxed) : 0;
  if (known == 0) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    const bool ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    if (dev >= 0 && dev < MAXDEV) arch_ok[dev].store(ok ? 1 : -1, std::memory_order_relaxed);
    if (!ok)
      return fail(LBM_EDEVICE, std::string("liblbm is built for gfx950, device is ") +
                                   prop.gcnArchName);
  } else if (known < 0) {
    return fail(LBM_EDEVICE, "liblbm is built for gfx950; the current device is not one");
  }
  if (dev_out) *dev_out = dev;
  return LBM_OK;
}

bool is_fin(double v) { return std::isfinite(v); }

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct lbm_handle {
  lbm_config user;
  lbm::StepConfig cfg;
  lbm_qref q;
  hipStream_t stream = nullptr;
  void *lat[2] = {nullptr, nullptr};
  bool own_lat = true;
  int cur = 0;
  void *chi_field = nullptr;  // compute type [ny][pitch]
  void *chi_x = nullptr;      // compute type [nx]
  void *chi_y = nullptr;      // compute type [ny]
  void *qf = nullptr;         // compute type [3][qps]: per-cell reference, or NULL
  void *qf2 = nullptr;        // second buffer for the strip kernels' running mean
  int64_t qps = 0;
  double qalpha = 0.0;        // running-mean rate of the reference
  int channel = 0;            // line source at x = 0 (Sec. 4.2)
  int outflow = 0;            // zero-gradient outflow at x = nx - 1
  lbm_line_source src = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double *diag_partials = nullptr;
  double *diag_out = nullptr;
  int64_t steps = 0;
  size_t lat_bytes = 0;
  int device = 0;
  // instability detector (lbm_set_detector)
  int64_t det_every = 0;      // 0: off
  double det_max = 0.0;
  int64_t det_next = 0;       // step count at which the next check is due
  unsigned long long *det_word = nullptr;  // device: first tripping step, or TRIP_NONE
  int64_t tripped_at = -1;    // host copy of the trip, once read
};

namespace {

int validate_config(const lbm_config *c) {
  if (!c) return fail(LBM_EINVAL, "config is NULL");
  if (c->nx < 1 || c->ny < 1) return fail(LBM_EINVAL, "nx and ny must be >= 1");
  if (c->nx > (1 << 30) || c->ny > (1 << 30) || c->nx * c->ny >= (int64_t(1) << 31))
    return fail(LBM_EINVAL, "nx * ny must be below 2^31");
  if (!(c->rho_base > 0) || !is_fin(c->rho_base))
    return fail(LBM_EINVAL, "rho_base must be finite and > 0");
  if (!is_fin(c->ux_base) || !is_fin(c->uy_base))
    return fail(LBM_EINVAL, "base velocity must be finite");
  for (int k = 0; k < 9; ++k)
    if (!(c->s[k] >= 0.0 && c->s[k] <= 2.0))
      return fail(LBM_EINVAL, "relaxation rates must lie in [0, 2]");
  if (!is_fin(c->shift_n) || !is_fin(c->shift_m) || c->shift_n < 0 || c->shift_m < 0)
    return fail(LBM_EINVAL, "shift parameters must be finite and >= 0");
  if (c->storage < LBM_STORAGE_F64 || c->storage > LBM_STORAGE_F16)
    return fail(LBM_EINVAL, "unknown storage mode");
  if (c->variant < LBM_VARIANT_NONE || c->variant > LBM_VARIANT_VISC)
    return fail(LBM_EINVAL, "unknown damping variant");
  if (c->storage == LBM_STORAGE_F16 && !(c->f16_scale > 0 && is_fin(c->f16_scale)))
    return fail(LBM_EINVAL, "f16_scale must be finite and > 0");
  return LBM_OK;
}

void layout(const lbm_config *c, int64_t *pitch, int64_t *ps, size_t *lat_bytes) {
  const int eb = lbm::elem_bytes_of(c->storage);
  *pitch = c->nx;
  // planes start on 256-byte boundaries
  *ps = round_up(c->nx * c->ny, 256 / eb);
  *lat_bytes = (size_t)(*ps) * 9 * eb;
}

void fill_cfg(lbm_handle *h) {
  lbm::StepConfig &s = h->cfg;
  const lbm_config &u = h->user;
  s.nx = (int)u.nx;
  s.ny = (int)u.ny;
  s.storage = u.storage;
  s.variant = u.variant;
  for (int k = 0; k < 9; ++k) s.s[k] = u.s[k];
  s.n = u.shift_n;
  s.m = u.shift_m;
  s.rho_b = u.rho_base;
  s.ubx = u.ux_base;
  s.uby = u.uy_base;
  s.f16_scale = u.storage == LBM_STORAGE_F16 ? u.f16_scale : 1.0;
  // q_ref - base in FP64 (argument conversion)
  s.dcf[0] = h->q.rho_f - u.rho_base;
  s.dcf[1] = (h->q.rho_f - u.rho_base) * h->q.ux_f + u.rho_base * (h->q.ux_f - u.ux_base);
  s.dcf[2] = (h->q.rho_f - u.rho_base) * h->q.uy_f + u.rho_base * (h->q.uy_f - u.uy_base);
  s.chi_field = h->chi_field;
  s.chi_x = h->chi_x;
  s.chi_y = h->chi_y;
  s.qfield = h->qf;
  s.qfield_out = h->qf2;
  s.qps = h->qps;
  s.qalpha = h->qf ? h->qalpha : 0.0;
  s.channel = h->channel;
  s.outflow = h->outflow;
}

// Equilibrium deviation f^eq_i(rho_b + dr, j_b + dj) - f^eq_i(rho_b, j_b) in
// FP64, every term O(dr, dj): the same expression the device's
// initialisation evaluates.
void feq_dev_host(double dr, double djx, double djy, double rho_b, double ubx, double uby,
                  double out[9]) {
  const double rho = rho_b + dr;
  for (int i = 0; i < 9; ++i) {
    const double cx = lbm::cx_of(i), cy = lbm::cy_of(i);
    const double dJ = cx * djx + cy * djy;
    const double Ub = cx * ubx + cy * uby;
    const double vJ = dJ - Ub * dr;
    const double dq_c = 2.0 * Ub * dJ - Ub * Ub * dr + vJ * vJ / rho;
    const double vx = djx - ubx * dr, vy = djy - uby * dr;
    const double dq_x = 2.0 * ubx * djx - ubx * ubx * dr + vx * vx / rho;
    const double dq_y = 2.0 * uby * djy - uby * uby * dr + vy * vy / rho;
    out[i] = lbm::w_of(i) * (dr + 3.0 * dJ + 4.5 * dq_c - 1.5 * (dq_x + dq_y));
  }
}

// Source deviations stored at x = 0 by the step that ends at step index t.
void source_dev(const lbm_handle *h, int64_t t, double out[9]) {
  const double PI = 3.14159265358979323846;
  const lbm_line_source &q = h->src;
  const double rs = q.rho0 + q.amp * std::sin(2.0 * PI * q.freq * (double)t + q.phase);
  const double rb = h->user.rho_base, ubx = h->user.ux_base, uby = h->user.uy_base;
  const double dr = rs - rb;
  feq_dev_host(dr, dr * q.ux + rb * (q.ux - ubx), dr * q.uy + rb * (q.uy - uby), rb, ubx, uby,
               out);
}

// Upload an FP64 host array converted to the compute type of the handle.
int upload_compute(lbm_handle *h, const double *src, size_t n, void **dst) {
  const bool f64 = h->user.storage == LBM_STORAGE_F64;
  const size_t eb = f64 ? 8 : 4;
  if (!*dst) HIP_TRY(hipMallocAsync(dst, n * eb, h->stream), "hipMallocAsync(sponge)");
  std::vector<float> tmp;
  const void *p = src;
  if (!f64) {
    tmp.resize(n);
    for (size_t i = 0; i < n; ++i) tmp[i] = (float)src[i];
    p = tmp.data();
  }
  HIP_TRY(hipMemcpyAsync(*dst, p, n * eb, hipMemcpyHostToDevice, h->stream),
          "hipMemcpy(sponge)");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  return LBM_OK;
}

// Auxiliary buffers (sponge arrays, staging, diagnostics) use stream-ordered
// allocation on the handle's stream, so creating and destroying handles
// never waits for the whole device.
void free_sponge(lbm_handle *h) {
  if (h->chi_field) (void)hipFreeAsync(h->chi_field, h->stream);
  if (h->chi_x) (void)hipFreeAsync(h->chi_x, h->stream);
  if (h->chi_y) (void)hipFreeAsync(h->chi_y, h->stream);
  h->chi_field = h->chi_x = h->chi_y = nullptr;
}

int ensure_diag(lbm_handle *h) {
  if (h->diag_partials) return LBM_OK;
  HIP_TRY(hipMallocAsync((void **)&h->diag_partials, lbm::diag_partials_bytes(h->cfg), h->stream),
          "hipMallocAsync(diagnostics)");
  HIP_TRY(hipMallocAsync((void **)&h->diag_out, 8 * sizeof(double), h->stream),
          "hipMallocAsync(diagnostics)");
  return LBM_OK;
}

// Enqueue a detector check of the current lattice at the handle's step
// count when one is due (called after every launch that advances it).
int detector_after_launch(lbm_handle *h, hipStream_t stream, unsigned long long *trip2) {
  if (!h->det_every || h->steps < h->det_next) return LBM_OK;
  lbm::CheckDesc d;
  lbm::fill_check_desc(h->cfg, h->lat[h->cur], d);
  d.trip = h->det_word;
  d.trip2 = trip2;
  d.step = (unsigned long long)h->steps;
  d.max_dev = h->det_max;
  h->det_next = (h->steps / h->det_every + 1) * h->det_every;
  HIP_TRY(lbm::launch_check(h->user.storage, d, stream), "detector kernel");
  return LBM_OK;
}

// Forget any trip (new state or new settings); stream-ordered.
int detector_reset(lbm_handle *h) {
  h->tripped_at = -1;
  if (h->det_every) h->det_next = (h->steps / h->det_every + 1) * h->det_every;
  if (h->det_word)
    HIP_TRY(lbm::launch_fill_u64(h->det_word, 1, lbm::TRIP_NONE, h->stream), "detector reset");
  return LBM_OK;
}

// After the handle's stream has drained: fold the device trip word into the
// host copy and report it.
int detector_result(lbm_handle *h) {
  if (!h->det_word) return LBM_OK;
  unsigned long long w = lbm::TRIP_NONE;
  HIP_TRY(hipMemcpyAsync(&w, h->det_word, sizeof(w), hipMemcpyDeviceToHost, h->stream),
          "hipMemcpy(detector)");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (w != lbm::TRIP_NONE && (h->tripped_at < 0 || (int64_t)w < h->tripped_at))
    h->tripped_at = (int64_t)w;
  if (h->tripped_at >= 0)
    return fail(LBM_EUNSTABLE, "instability detector tripped at step " +
                                   std::to_string(h->tripped_at));
  return LBM_OK;
}

int check_qref(const lbm_qref *q) {
  if (!q) return LBM_OK;
  if (!(q->rho_f > 0) || !is_fin(q->rho_f) || !is_fin(q->ux_f) || !is_fin(q->uy_f))
    return fail(LBM_EINVAL, "q_ref must be finite with rho_f > 0");
  return LBM_OK;
}

int check_chi(const double *a, size_t n, int variant) {
  if (!a) return LBM_OK;
  for (size_t i = 0; i < n; ++i) {
    if (!(a[i] >= 0.0) || !is_fin(a[i]))
      return fail(LBM_EINVAL, "chi must be finite and >= 0");
    if (variant == LBM_VARIANT_VISC && a[i] > 1.0)
      return fail(LBM_EINVAL, "the viscosity ramp coordinate must lie in [0, 1]");
  }
  return LBM_OK;
}

int init_state(lbm_handle *h, const double *rho, const double *ux,
               const double *uy) {
  const int64_t N = h->user.nx * h->user.ny;
  double *d = nullptr;
  if (rho) {
    for (int64_t i = 0; i < N; ++i)
      if (!(rho[i] > 0) || !is_fin(rho[i]) || (ux && !is_fin(ux[i])) || (uy && !is_fin(uy[i])))
        return fail(LBM_EINVAL, "initial fields must be finite with rho > 0");
    HIP_TRY(hipMallocAsync((void **)&d, sizeof(double) * 3 * N, h->stream), "hipMallocAsync(init)");
    std::vector<double> zero;
    if (!ux || !uy) zero.assign(N, 0.0);
    hipError_t e = hipMemcpyAsync(d, rho, sizeof(double) * N, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d + N, ux ? ux : zero.data(), sizeof(double) * N, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d + 2 * N, uy ? uy : zero.data(), sizeof(double) * N, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) {
      (void)hipFreeAsync(d, h->stream);
      return hip_fail(e, "hipMemcpy(init)");
    }
  }
  hipError_t e = lbm::launch_init(h->cfg, d, d ? d + N : nullptr, d ? d + 2 * N : nullptr,
                                  h->lat[0], h->stream);
  if (d) (void)hipFreeAsync(d, h->stream);
  // the host arrays (and the zero vector) must outlive the copies; without
  // them nothing waits (a server creates lattices on a busy stream)
  if (e == hipSuccess && d) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "init kernel");
  h->cur = 0;
  h->steps = 0;
  return LBM_OK;
}

int create_common(const lbm_config *cfg, const double *rho, const double *ux,
                  const double *uy, void *buf_a, void *buf_b, size_t bytes_each,
                  lbm_handle **out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_config(cfg);
  if (rc) return rc;
  int dev = 0;
  rc = check_device(&dev);
  if (rc) return rc;
  lbm_handle *h = new (std::nothrow) lbm_handle();
  if (!h) return fail(LBM_ENOMEM, "host allocation failed");
  h->user = *cfg;
  h->device = dev;
  h->stream = (hipStream_t)cfg->stream;
  h->q = lbm_qref{cfg->rho_base, cfg->ux_base, cfg->uy_base};
  int64_t pitch, ps;
  layout(cfg, &pitch, &ps, &h->lat_bytes);
  h->cfg.pitch = pitch;
  h->cfg.plane_stride = ps;
  h->cfg.chi_mode = lbm::CHI_ZERO;
  h->cfg.kernel = lbm::KERNEL_VEC;
  h->cfg.block = 256;
  h->cfg.nontemporal = 0;
  h->cfg.rows = 64;
  if (buf_a) {
    if (!buf_b || bytes_each < h->lat_bytes || ((uintptr_t)buf_a & 255) ||
        ((uintptr_t)buf_b & 255)) {
      delete h;
      return fail(LBM_EINVAL, "caller buffers too small or not 256-byte aligned");
    }
    h->lat[0] = buf_a;
    h->lat[1] = buf_b;
    h->own_lat = false;
  } else {
    for (int k = 0; k < 2; ++k) {
      hipError_t e = hipMalloc(&h->lat[k], h->lat_bytes);
      if (e != hipSuccess) {
        lbm_destroy(h);
        return hip_fail(e, "hipMalloc(lattice)");
      }
    }
  }
  // zero both lattices so that plane padding is deterministic
  for (int k = 0; k < 2; ++k) {
    hipError_t ez = hipMemsetAsync(h->lat[k], 0, h->lat_bytes, h->stream);
    if (ez != hipSuccess) {
      lbm_destroy(h);
      return hip_fail(ez, "hipMemset(lattice)");
    }
  }
  fill_cfg(h);
  rc = init_state(h, rho, ux, uy);
  if (rc) {
    lbm_destroy(h);
    return rc;
  }
  *out = h;
  return LBM_OK;
}

}  // namespace

namespace {
// The second reference-field buffer of the strip kernels' running mean.
int ensure_qf2(lbm_handle *h) {
  if (h->qf2) return LBM_OK;
  const size_t eb = h->user.storage == LBM_STORAGE_F64 ? 8 : 4;
  HIP_TRY(hipMallocAsync(&h->qf2, (size_t)(3 * h->qps) * eb, h->stream), "hipMallocAsync(reference)");
  h->cfg.qfield_out = h->qf2;
  return LBM_OK;
}
}  // namespace

extern "C" {

int lbm_required_bytes(const lbm_config *cfg, size_t *bytes) {
  int rc = validate_config(cfg);
  if (rc) return rc;
  if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
  int64_t pitch, ps;
  size_t lb;
  layout(cfg, &pitch, &ps, &lb);
  *bytes = 2 * lb;
  return LBM_OK;
}

int lbm_create(const lbm_config *cfg, const double *rho, const double *ux,
               const double *uy, lbm_handle **out) {
  return create_common(cfg, rho, ux, uy, nullptr, nullptr, 0, out);
}

int lbm_create_ext(const lbm_config *cfg, const double *rho, const double *ux,
                   const double *uy, void *dev_buf_a, void *dev_buf_b,
                   size_t bytes_each, lbm_handle **out) {
  if (!dev_buf_a || !dev_buf_b) return fail(LBM_EINVAL, "device buffers are NULL");
  return create_common(cfg, rho, ux, uy, dev_buf_a, dev_buf_b, bytes_each, out);
}

int lbm_set_sponge(lbm_handle *h, const double *chi, const lbm_qref *q) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  int rc = check_qref(q);
  if (rc) return rc;
  const size_t N = (size_t)(h->user.nx * h->user.ny);
  rc = check_chi(chi, N, h->user.variant);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  free_sponge(h);
  if (chi) {
    // field stored with the lattice row pitch
    std::vector<double> padded((size_t)(h->cfg.pitch * h->user.ny), 0.0);
    for (int64_t y = 0; y < h->user.ny; ++y)
      std::memcpy(&padded[(size_t)(y * h->cfg.pitch)], chi + y * h->user.nx,
                  sizeof(double) * h->user.nx);
    rc = upload_compute(h, padded.data(), padded.size(), &h->chi_field);
    if (rc) return rc;
    h->cfg.chi_mode = lbm::CHI_FIELD;
  } else {
    h->cfg.chi_mode = lbm::CHI_ZERO;
  }
  if (q) h->q = *q;
  fill_cfg(h);
  return LBM_OK;
}

int lbm_set_sponge_separable(lbm_handle *h, const double *chi_x,
                             const double *chi_y, int32_t combine,
                             const lbm_qref *q) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (combine != LBM_COMBINE_MAX && combine != LBM_COMBINE_SUM)
    return fail(LBM_EINVAL, "unknown combine mode");
  int rc = check_qref(q);
  if (rc) return rc;
  rc = check_chi(chi_x, (size_t)h->user.nx, h->user.variant);
  if (!rc) rc = check_chi(chi_y, (size_t)h->user.ny, h->user.variant);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  free_sponge(h);
  if (chi_x || chi_y) {
    std::vector<double> ax(h->user.nx, 0.0), ay(h->user.ny, 0.0);
    if (chi_x) std::memcpy(ax.data(), chi_x, sizeof(double) * h->user.nx);
    if (chi_y) std::memcpy(ay.data(), chi_y, sizeof(double) * h->user.ny);
    rc = upload_compute(h, ax.data(), ax.size(), &h->chi_x);
    if (!rc) rc = upload_compute(h, ay.data(), ay.size(), &h->chi_y);
    if (rc) return rc;
    h->cfg.chi_mode = combine == LBM_COMBINE_MAX ? lbm::CHI_SEP_MAX : lbm::CHI_SEP_SUM;
  } else {
    h->cfg.chi_mode = lbm::CHI_ZERO;
  }
  if (q) h->q = *q;
  fill_cfg(h);
  return LBM_OK;
}

int lbm_set_sponge_separable_dev(lbm_handle *h, const double *chi_x, const double *chi_y,
                                 int32_t combine, const lbm_qref *q) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (combine != LBM_COMBINE_MAX && combine != LBM_COMBINE_SUM)
    return fail(LBM_EINVAL, "unknown combine mode");
  int rc = check_qref(q);
  if (rc) return rc;
  // stream-ordered throughout: the old arrays are freed behind the work
  // that reads them, the new ones converted behind that
  free_sponge(h);
  if (chi_x || chi_y) {
    const size_t eb = h->user.storage == LBM_STORAGE_F64 ? 8 : 4;
    HIP_TRY(hipMallocAsync(&h->chi_x, eb * h->user.nx, h->stream), "hipMallocAsync(sponge)");
    HIP_TRY(hipMallocAsync(&h->chi_y, eb * h->user.ny, h->stream), "hipMallocAsync(sponge)");
    HIP_TRY(lbm::launch_convert_profile(h->user.storage, chi_x, h->chi_x, h->user.nx, h->stream),
            "sponge conversion");
    HIP_TRY(lbm::launch_convert_profile(h->user.storage, chi_y, h->chi_y, h->user.ny, h->stream),
            "sponge conversion");
    h->cfg.chi_mode = combine == LBM_COMBINE_MAX ? lbm::CHI_SEP_MAX : lbm::CHI_SEP_SUM;
  } else {
    h->cfg.chi_mode = lbm::CHI_ZERO;
  }
  if (q) h->q = *q;
  fill_cfg(h);
  return LBM_OK;
}

int lbm_step(lbm_handle *h, int64_t n) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  int64_t k = 0;
  const int per = h->cfg.kernel;  // time steps per launch of the multi-step kernel
  // a channel, rows of 2^32 bytes or more, a running-mean reference state,
  // or a per-cell one with parameters other than the default form run in the
  // one-step kernel only
  if (per >= lbm::KERNEL_MULTI_MIN && lbm::multi_step_supports(h->cfg)) {
    // a running-mean reference: each launch writes the updated field to the
    // second buffer, which then becomes the current one
    const bool qa = h->qf && h->qalpha != 0.0;
    if (qa && n - k >= 2) {
      int rc = ensure_qf2(h);
      if (rc) return rc;
    }
    while (n - k >= 2) {
      const int m = n - k >= per ? per : (int)(n - k);
      hipError_t e = lbm::launch_multi_steps(h->cfg, m, h->lat[h->cur], h->lat[1 - h->cur], h->stream);
      if (e != hipSuccess) return hip_fail(e, "multi-step kernel");
      h->cur = 1 - h->cur;
      h->steps += m;
      k += m;
      if (qa) {
        std::swap(h->qf, h->qf2);
        h->cfg.qfield = h->qf;
        h->cfg.qfield_out = h->qf2;
      }
      int rc = detector_after_launch(h, h->stream, nullptr);
      if (rc) return rc;
    }
  }
  for (; k < n; ++k) {
    if (h->channel) source_dev(h, h->steps + 1, h->cfg.src_dev);
    hipError_t e = lbm::launch_step(h->cfg, h->lat[h->cur], h->lat[1 - h->cur], h->stream);
    if (e != hipSuccess) return hip_fail(e, "step kernel");
    h->cur = 1 - h->cur;
    h->steps += 1;
    int rc = detector_after_launch(h, h->stream, nullptr);
    if (rc) return rc;
  }
  return LBM_OK;
}

int lbm_set_detector(lbm_handle *h, int64_t every_n, double max_dev) {
  // arguments first, so that their checks need no device
  if (every_n < 0) return fail(LBM_EINVAL, "every_n must be >= 0");
  if (every_n > 0 && !(max_dev > 0.0)) return fail(LBM_EINVAL, "max_dev must be > 0 (may be infinite)");
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (every_n > 0 && !h->det_word)
    HIP_TRY(hipMallocAsync((void **)&h->det_word, sizeof(unsigned long long), h->stream),
            "hipMallocAsync(detector)");
  h->det_every = every_n;
  h->det_max = every_n > 0 ? max_dev : 0.0;
  int rc = detector_reset(h);
  if (rc) return rc;
  // the word is now ready for any stream (a batch checks on its own)
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  return LBM_OK;
}

int lbm_detector_status(lbm_handle *h, int64_t *tripped_at) {
  if (!h || !tripped_at) return fail(LBM_EINVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  const int rc = detector_result(h);
  if (rc != LBM_OK && rc != LBM_EUNSTABLE) return rc;
  *tripped_at = h->tripped_at;
  return LBM_OK;
}

int lbm_sync(lbm_handle *h) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  return detector_result(h);
}

int lbm_moments_dev(lbm_handle *h, double *rho, double *ux, double *uy) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  hipError_t e = lbm::launch_moments(h->cfg, h->lat[h->cur], rho, ux, uy, h->stream);
  if (e != hipSuccess) return hip_fail(e, "moments kernel");
  return LBM_OK;
}

int lbm_moments(lbm_handle *h, double *rho, double *ux, double *uy) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  const int64_t N = h->user.nx * h->user.ny;
  double *d = nullptr;
  HIP_TRY(hipMallocAsync((void **)&d, sizeof(double) * 3 * N, h->stream), "hipMallocAsync(moments)");
  hipError_t e = lbm::launch_moments(h->cfg, h->lat[h->cur], d, d + N, d + 2 * N, h->stream);
  if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, d, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess && ux) e = hipMemcpyAsync(ux, d + N, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess && uy) e = hipMemcpyAsync(uy, d + 2 * N, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
  (void)hipFreeAsync(d, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "moments");
  return detector_result(h);
}

int lbm_diagnostics(lbm_handle *h, double out[7]) {
  if (!h || !out) return fail(LBM_EINVAL, "NULL argument");
  int rc = ensure_diag(h);
  if (rc) return rc;
  hipError_t e = lbm::launch_diagnostics(h->cfg, h->lat[h->cur], h->diag_partials,
                                         h->diag_out, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, h->diag_out, 7 * sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics");
  return detector_result(h);
}

int lbm_diagnostics_dev(lbm_handle *h, double *out7_dev) {
  if (!h || !out7_dev) return fail(LBM_EINVAL, "NULL argument");
  int rc = ensure_diag(h);
  if (rc) return rc;
  hipError_t e = lbm::launch_diagnostics(h->cfg, h->lat[h->cur], h->diag_partials,
                                         out7_dev, h->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics");
  return LBM_OK;
}

int lbm_diagnostics_dev_noalloc(lbm_handle *h, double *out7_dev) {
  if (!h || !out7_dev) return fail(LBM_EINVAL, "NULL argument");
  double *ws = nullptr;
  size_t ws_bytes = 0;
  HIP_TRY(lbm::diag_scratch(h->device, &ws, &ws_bytes), "diagnostics workspace");
  if (lbm::diag_partials_bytes(h->cfg) > ws_bytes)
    return fail(LBM_EINVAL, "the reduction needs " + std::to_string(lbm::diag_partials_bytes(h->cfg)) +
                                " bytes of partials, above the static workspace of " +
                                std::to_string(ws_bytes));
  hipError_t e = lbm::launch_diagnostics(h->cfg, h->lat[h->cur], ws, out7_dev, h->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics");
  return LBM_OK;
}

int lbm_get_populations(lbm_handle *h, double *f) {
  if (!h || !f) return fail(LBM_EINVAL, "NULL argument");
  const int64_t N = h->user.nx * h->user.ny;
  double *d = nullptr;
  HIP_TRY(hipMallocAsync((void **)&d, sizeof(double) * 9 * N, h->stream), "hipMallocAsync(populations)");
  hipError_t e = lbm::launch_get_populations(h->cfg, h->lat[h->cur], d, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(f, d, sizeof(double) * 9 * N, hipMemcpyDeviceToHost, h->stream);
  (void)hipFreeAsync(d, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "get_populations");
  return LBM_OK;
}

int lbm_set_populations(lbm_handle *h, const double *f) {
  if (!h || !f) return fail(LBM_EINVAL, "NULL argument");
  const int64_t N = h->user.nx * h->user.ny;
  for (int64_t i = 0; i < 9 * N; ++i)
    if (!is_fin(f[i])) return fail(LBM_EINVAL, "populations must be finite");
  double *d = nullptr;
  HIP_TRY(hipMallocAsync((void **)&d, sizeof(double) * 9 * N, h->stream), "hipMallocAsync(populations)");
  hipError_t e = hipMemcpyAsync(d, f, sizeof(double) * 9 * N, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = lbm::launch_set_populations(h->cfg, d, h->lat[0], h->stream);
  (void)hipFreeAsync(d, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "set_populations");
  h->cur = 0;
  h->steps = 0;
  return detector_reset(h);
}

int lbm_state_bytes(lbm_handle *h, size_t *bytes) {
  if (!h || !bytes) return fail(LBM_EINVAL, "NULL argument");
  *bytes = h->lat_bytes + sizeof(int64_t);
  return LBM_OK;
}

int lbm_save_state(lbm_handle *h, void *host, size_t bytes) {
  if (!h || !host) return fail(LBM_EINVAL, "NULL argument");
  if (bytes != h->lat_bytes + sizeof(int64_t)) return fail(LBM_EINVAL, "state buffer size mismatch");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  HIP_TRY(hipMemcpy(host, h->lat[h->cur], h->lat_bytes, hipMemcpyDeviceToHost), "hipMemcpy(state)");
  std::memcpy((char *)host + h->lat_bytes, &h->steps, sizeof(int64_t));
  return LBM_OK;
}

int lbm_load_state(lbm_handle *h, const void *host, size_t bytes) {
  if (!h || !host) return fail(LBM_EINVAL, "NULL argument");
  if (bytes != h->lat_bytes + sizeof(int64_t)) return fail(LBM_EINVAL, "state buffer size mismatch");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  HIP_TRY(hipMemcpy(h->lat[0], host, h->lat_bytes, hipMemcpyHostToDevice), "hipMemcpy(state)");
  h->cur = 0;
  std::memcpy(&h->steps, (const char *)host + h->lat_bytes, sizeof(int64_t));
  return detector_reset(h);
}

int lbm_get_info(lbm_handle *h, lbm_info *info) {
  if (!h || !info) return fail(LBM_EINVAL, "NULL argument");
  info->nx = h->user.nx;
  info->ny = h->user.ny;
  info->pitch = h->cfg.pitch;
  info->plane_stride = h->cfg.plane_stride;
  info->steps_done = h->steps;
  info->storage = h->user.storage;
  info->variant = h->user.variant;
  info->elem_bytes = lbm::elem_bytes_of(h->user.storage);
  info->chi_mode = h->cfg.chi_mode;
  info->device_bytes = 2 * h->lat_bytes;
  return LBM_OK;
}

int lbm_set_tuning(lbm_handle *h, const lbm_tuning *t) {
  if (!h || !t) return fail(LBM_EINVAL, "NULL argument");
  if (t->kernel < 0 || t->kernel > lbm::KERNEL_MULTI_MAX)
    return fail(LBM_EINVAL, "kernel must be 0, 1, 2, 3 or 4");
  if (t->block != 64 && t->block != 128 && t->block != 256 && t->block != 512)
    return fail(LBM_EINVAL, "block must be 64, 128, 256 or 512");
  if (t->nontemporal != 0 && t->nontemporal != 1) return fail(LBM_EINVAL, "nontemporal must be 0 or 1");
  if (t->kernel >= 2 && (t->rows < 0 || t->rows > 4096))
    return fail(LBM_EINVAL, "rows must be 0 (fit the device) or 1..4096");
  if (t->kernel >= 2 && t->block > lbm::multi_step_max_block(h->user.storage, t->kernel))
    return fail(LBM_EINVAL, "FP64 storage with four steps per launch takes blocks of at most 256");
  h->cfg.kernel = t->kernel;
  h->cfg.block = t->block;
  h->cfg.nontemporal = t->kernel == 1 ? t->nontemporal : 0;
  if (t->kernel >= 2) h->cfg.rows = t->rows;
  return LBM_OK;
}

int lbm_get_tuning(lbm_handle *h, lbm_tuning *t) {
  if (!h || !t) return fail(LBM_EINVAL, "NULL argument");
  if (h->cfg.kernel >= lbm::KERNEL_MULTI_MIN)
    t->kernel = h->cfg.kernel;
  else
    t->kernel = h->cfg.kernel == lbm::KERNEL_VEC && lbm::vec_supported(h->cfg) ? 1 : 0;
  t->block = h->cfg.block;
  t->nontemporal = t->kernel == 1 ? h->cfg.nontemporal : 0;
  t->rows = t->kernel >= 2 ? h->cfg.rows : 0;
  return LBM_OK;
}

int lbm_autotune(lbm_handle *h, int32_t reps, lbm_tuning *best, double *best_ms) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (reps < 1) return fail(LBM_EINVAL, "reps must be >= 1");
  std::vector<lbm_tuning> cands;
  const int blocks[4] = {64, 128, 256, 512};
  for (int b : blocks) cands.push_back(lbm_tuning{0, b, 0, 0});
  if (lbm::vec_supported(h->cfg))
    for (int nt = 0; nt < 2; ++nt)
      for (int b : blocks) cands.push_back(lbm_tuning{1, b, nt, 0});
  const int rows[4] = {0, 8, 16, 32};
  if (lbm::multi_step_supports(h->cfg))  // lbm_step would not run them otherwise
    for (int kk = lbm::KERNEL_MULTI_MIN; kk <= lbm::KERNEL_MULTI_MAX; ++kk)
      for (int b : blocks)
        if (b <= lbm::multi_step_max_block(h->user.storage, kk))
          for (int r : rows) cands.push_back(lbm_tuning{kk, b, 0, r});
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  // the running mean would advance during the timing: keep a copy
  void *qf_keep = nullptr;
  const size_t qf_bytes = h->qf ? (size_t)(3 * h->qps) * (h->user.storage == LBM_STORAGE_F64 ? 8 : 4) : 0;
  if (h->qf && h->qalpha != 0.0) {
    int rc = ensure_qf2(h);
    if (rc) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return rc;
    }
    e = hipMallocAsync(&qf_keep, qf_bytes, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(qf_keep, h->qf, qf_bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) {
      if (qf_keep) (void)hipFreeAsync(qf_keep, h->stream);
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return hip_fail(e, "autotune reference copy");
    }
  }
  const lbm::StepConfig saved = h->cfg;
  double best_t = 1e300;
  lbm_tuning best_c = cands[0];
  for (const lbm_tuning &c : cands) {
    h->cfg.kernel = c.kernel;
    h->cfg.block = c.block;
    h->cfg.nontemporal = c.nontemporal;
    h->cfg.rows = c.kernel >= 2 ? c.rows : saved.rows;
    // the candidate reads the current lattice and overwrites the other one,
    // whose contents the next step replaces anyway
    for (int k = 0; k < 2 + reps && e == hipSuccess; ++k) {
      if (k == 2) e = hipEventRecord(e0, h->stream);
      if (e == hipSuccess)
        e = c.kernel >= 2 ? lbm::launch_multi_steps(h->cfg, c.kernel, h->lat[h->cur],
                                                    h->lat[1 - h->cur], h->stream)
                          : lbm::launch_step(h->cfg, h->lat[h->cur], h->lat[1 - h->cur], h->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) break;
    const double per = ms / reps / (c.kernel >= 2 ? (double)c.kernel : 1.0);  // per time step
    if (per < best_t) {
      best_t = per;
      best_c = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->cfg = saved;
  if (qf_keep) {
    const hipError_t e2 = hipMemcpyAsync(h->qf, qf_keep, qf_bytes, hipMemcpyDeviceToDevice, h->stream);
    (void)hipFreeAsync(qf_keep, h->stream);
    if (e == hipSuccess) e = e2;
  }
  if (e != hipSuccess) return hip_fail(e, "autotune");
  h->cfg.kernel = best_c.kernel;
  h->cfg.block = best_c.block;
  h->cfg.nontemporal = best_c.nontemporal;
  if (best_c.kernel >= 2) h->cfg.rows = best_c.rows;
  if (best) *best = best_c;
  if (best_ms) *best_ms = best_t;
  return LBM_OK;
}

void lbm_destroy(lbm_handle *h) {
  if (!h) return;
  free_sponge(h);
  if (h->qf) (void)hipFreeAsync(h->qf, h->stream);
  if (h->qf2) (void)hipFreeAsync(h->qf2, h->stream);
  if (h->diag_partials) (void)hipFreeAsync(h->diag_partials, h->stream);
  if (h->diag_out) (void)hipFreeAsync(h->diag_out, h->stream);
  if (h->det_word) (void)hipFreeAsync(h->det_word, h->stream);
  if (h->own_lat) {
    (void)hipStreamSynchronize(h->stream);
    for (int k = 0; k < 2; ++k)
      if (h->lat[k]) (void)hipFree(h->lat[k]);
  }
  delete h;
}

int lbm_set_qref_field(lbm_handle *h, const double *rho_f, const double *ux_f,
                       const double *uy_f) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (!rho_f && !ux_f && !uy_f) {
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    if (h->qf) (void)hipFreeAsync(h->qf, h->stream);
    if (h->qf2) (void)hipFreeAsync(h->qf2, h->stream);
    h->qf = h->qf2 = nullptr;
    h->qalpha = 0.0;
    fill_cfg(h);
    return LBM_OK;
  }
  if (!rho_f || !ux_f || !uy_f) return fail(LBM_EINVAL, "give all three reference fields or none");
  if (h->channel) return fail(LBM_ESTATE, "a reference field cannot be combined with a line source");
  const int64_t nx = h->user.nx, ny = h->user.ny, pitch = h->cfg.pitch;
  for (int64_t c = 0; c < nx * ny; ++c)
    if (!(rho_f[c] > 0) || !is_fin(rho_f[c]) || !is_fin(ux_f[c]) || !is_fin(uy_f[c]))
      return fail(LBM_EINVAL, "reference fields must be finite with rho_f > 0");
  // conserved moments as deviations from the base, formed in FP64 without
  // cancellation: d j = (rho^f - rho_b) u^f + rho_b (u^f - u_b)
  const double rb = h->user.rho_base, ubx = h->user.ux_base, uby = h->user.uy_base;
  const int64_t qps = round_up(ny * pitch, 64);
  std::vector<double> host((size_t)(3 * qps), 0.0);
  for (int64_t y = 0; y < ny; ++y)
    for (int64_t x = 0; x < nx; ++x) {
      const int64_t c = y * nx + x, d = y * pitch + x;
      const double dr = rho_f[c] - rb;
      host[(size_t)d] = dr;
      host[(size_t)(qps + d)] = dr * ux_f[c] + rb * (ux_f[c] - ubx);
      host[(size_t)(2 * qps + d)] = dr * uy_f[c] + rb * (uy_f[c] - uby);
    }
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (h->qf && h->qps != qps) {
    (void)hipFreeAsync(h->qf, h->stream);
    if (h->qf2) (void)hipFreeAsync(h->qf2, h->stream);
    h->qf = h->qf2 = nullptr;
  }
  h->qps = qps;
  int rc = upload_compute(h, host.data(), host.size(), &h->qf);
  if (rc) return rc;
  fill_cfg(h);
  return LBM_OK;
}

int lbm_get_qref_field(lbm_handle *h, double *rho_f, double *ux_f, double *uy_f) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (!h->qf) return fail(LBM_ESTATE, "no per-cell reference state is set");
  if (!rho_f || !ux_f || !uy_f) return fail(LBM_EINVAL, "output arrays are NULL");
  const bool f64 = h->user.storage == LBM_STORAGE_F64;
  const size_t n = (size_t)(3 * h->qps);
  std::vector<double> host(n);
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (f64) {
    HIP_TRY(hipMemcpy(host.data(), h->qf, n * 8, hipMemcpyDeviceToHost), "hipMemcpy(reference)");
  } else {
    std::vector<float> tmp(n);
    HIP_TRY(hipMemcpy(tmp.data(), h->qf, n * 4, hipMemcpyDeviceToHost), "hipMemcpy(reference)");
    for (size_t i = 0; i < n; ++i) host[i] = tmp[i];
  }
  const double rb = h->user.rho_base, ubx = h->user.ux_base, uby = h->user.uy_base;
  const int64_t nx = h->user.nx, ny = h->user.ny, pitch = h->cfg.pitch, qps = h->qps;
  for (int64_t y = 0; y < ny; ++y)
    for (int64_t x = 0; x < nx; ++x) {
      const int64_t c = y * nx + x, d = y * pitch + x;
      const double rho = rb + host[(size_t)d];
      rho_f[c] = rho;
      ux_f[c] = (rb * ubx + host[(size_t)(qps + d)]) / rho;
      uy_f[c] = (rb * uby + host[(size_t)(2 * qps + d)]) / rho;
    }
  return LBM_OK;
}

int lbm_set_line_source(lbm_handle *h, const lbm_line_source *src, int32_t outflow) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (!src) {
    if (outflow) return fail(LBM_EINVAL, "an outflow boundary needs the line source");
    h->channel = h->outflow = 0;
    fill_cfg(h);
    return LBM_OK;
  }
  if (h->qf) return fail(LBM_ESTATE, "a line source cannot be combined with a reference field");
  if (h->user.nx < 3) return fail(LBM_EINVAL, "a channel needs nx >= 3");
  if (outflow != 0 && outflow != 1) return fail(LBM_EINVAL, "outflow must be 0 or 1");
  const double *v = &src->rho0;
  for (int i = 0; i < 6; ++i)
    if (!is_fin(v[i])) return fail(LBM_EINVAL, "line source parameters must be finite");
  if (!(src->rho0 - std::fabs(src->amp) > 0)) return fail(LBM_EINVAL, "source density must stay > 0");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  h->src = *src;
  h->channel = 1;
  h->outflow = outflow;
  fill_cfg(h);
  return LBM_OK;
}

int lbm_set_qref_average(lbm_handle *h, double alpha) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(LBM_EINVAL, "alpha must lie in [0, 1]");
  if (!h->qf) return fail(LBM_ESTATE, "set a per-cell reference state first");
  h->qalpha = alpha;
  fill_cfg(h);
  return LBM_OK;
}

int lbm_init_fields_dev(lbm_handle *h, const double *rho, const double *ux,
                        const double *uy) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  hipError_t e = lbm::launch_init(h->cfg, rho, ux, uy, h->lat[0], h->stream);
  if (e != hipSuccess) return hip_fail(e, "init kernel");
  h->cur = 0;
  h->steps = 0;
  return detector_reset(h);
}

const char *lbm_last_error(void) { return g_err.c_str(); }

}  // extern "C"

struct lbm_batch {
  std::vector<lbm_handle *> members;
  int storage = 1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  lbm::BatchDomain *d_doms = nullptr;
  lbm::BatchDomain *h_doms[2] = {nullptr, nullptr};  // pinned staging, alternating
  hipEvent_t copied[2] = {nullptr, nullptr};         // staging buffer free again
  int slot = 0;
  int2 *d_tiles = nullptr;
  int *d_ntiles = nullptr;
  int ntiles = 0;
  size_t dom_cap = 0, tile_cap = 0;
  int cus = 1;
  int blocks_per_cu = 8;
  // K-step strip launches (multi_k = 0: one-step tile launches only)
  int multi_k = 0;
  int multi_nw = 2;    // waves per workgroup
  int multi_rows = 0;  // rows per work item, 0: automatic (8..64, an item per resident workgroup)
  int multi_grid = 0;  // persistent workgroups of the strip kernel
  int min_items = -1;  // strip launches need this many items (-1: multi_grid)
  int4 *d_items = nullptr;
  int *d_nitems = nullptr;
  int nitems = 0;
  size_t item_cap = 0;
  int multi_form = 0;  // BATCH_DEF / BATCH_QF of the member list when the items were made
  // instability detector: per-member trip slots (one copy at lbm_batch_sync)
  // and the descriptors of one tick's checks, staged like the members'
  unsigned long long *d_trip = nullptr;            // [dom_cap]
  lbm::CheckDesc *d_chk = nullptr;                 // [dom_cap]
  lbm::CheckDesc *h_chk[2] = {nullptr, nullptr};   // pinned staging, alternating
  hipEvent_t chk_copied[2] = {nullptr, nullptr};
  // pinned staging of the tile and item tables (member changes are
  // stream-ordered: no wait for the device unless a table outgrows its buffer)
  char *h_tab[2] = {nullptr, nullptr};
  size_t tab_cap[2] = {0, 0};
  hipEvent_t tab_copied[2] = {nullptr, nullptr};
  int tab_slot = 0;
  int chk_slot = 0;
  bool any_detector = false;  // some check ran since the member list was set
  // graphs keyed by (K or 0, K-step launches or ticks, remainder launches,
  // tile workgroups per CU, strip workgroup waves, default form)
  std::map<std::tuple<int, int, int, int, int, int>, hipGraphExec_t> graphs;
};

namespace {

void fill_domain(const lbm_handle *h, int stop_at, lbm::BatchDomain &d) {
  const lbm::StepConfig &c = h->cfg;
  d.lat[0] = h->lat[0];
  d.lat[1] = h->lat[1];
  d.chi_field = c.chi_field;
  d.chi_x = c.chi_x;
  d.chi_y = c.chi_y;
  d.pitch = c.pitch;
  d.ps = c.plane_stride;
  d.nx = c.nx;
  d.ny = c.ny;
  d.variant = c.variant;
  d.chi_mode = c.chi_mode;
  d.parity = h->cur;
  d.stop_at = stop_at;
  for (int k = 0; k < 9; ++k) d.s[k] = c.s[k];
  d.n = c.n;
  d.m = c.m;
  d.rho_b = c.rho_b;
  d.ubx = c.ubx;
  d.uby = c.uby;
  for (int k = 0; k < 3; ++k) d.dcf[k] = c.dcf[k];
  for (int i = 0; i < 9; ++i) {
    d.scale[i] = lbm::storage_scale(c, i);
    d.inv_scale[i] = 1.0 / d.scale[i];
  }
  // a fixed per-cell reference; the undamped and viscosity-ramp variants
  // ignore it, as alone
  const bool damped = c.variant == LBM_VARIANT_I || c.variant == LBM_VARIANT_II ||
                      c.variant == LBM_VARIANT_III;
  d.qf = h->qf && damped ? h->qf : nullptr;
  d.qps = h->qps;
}

// The member's parameters allow the collision's default form: conserved
// rates 0 and n = m, compared in the compute precision as the kernels see
// them (FP64 storage computes in FP64, the others in FP32).
bool default_form(const lbm::StepConfig &c) {
  if (c.storage == LBM_STORAGE_F64)
    return c.s[0] == 0.0 && c.s[1] == 0.0 && c.s[2] == 0.0 && c.n == c.m;
  return (float)c.s[0] == 0.0f && (float)c.s[1] == 0.0f && (float)c.s[2] == 0.0f &&
         (float)c.n == (float)c.m;
}

// What a batch cannot step: a line source (its per-step column override),
// a running-mean reference (its second buffer follows the member's own
// launches). Checked when the members are set and before every tick, since
// both can be set on a member afterwards.
int check_batchable(const lbm_handle *h, size_t i) {
  if (h->channel)
    return fail(LBM_EINVAL, "member " + std::to_string(i) + " has a line source; it is not batched");
  if (h->qf && h->qalpha != 0.0)
    return fail(LBM_EINVAL, "member " + std::to_string(i) +
                                " has a running-mean reference state; batches take fixed ones");
  return LBM_OK;
}

// The strip kernel's form for the current members.
int batch_form(const std::vector<lbm_handle *> &members) {
  bool def = true, qf = false, mx = true;
  for (const lbm_handle *h : members) {
    def = def && default_form(h->cfg);
    const int v = h->cfg.variant;
    qf = qf || (h->qf && (v == LBM_VARIANT_I || v == LBM_VARIANT_II || v == LBM_VARIANT_III));
    mx = mx && h->cfg.chi_mode == lbm::CHI_SEP_MAX;
  }
  return (def ? lbm::BATCH_DEF : 0) | (qf ? lbm::BATCH_QF : 0) | (mx ? lbm::BATCH_SEPMAX : 0);
}

void free_graphs(lbm_batch *b) {
  for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

// Instantiated graph of one tick: `nmulti` K-step strip launches
// (j = 0 .. nmulti-1, strip kernel form `form`) then `nsingle` one-step
// tile launches (k = 0 .. nsingle-1; with K-step launches these take the
// members' remainders).
int batch_graph(lbm_batch *b, int K, int nmulti, int nsingle, int form, hipGraphExec_t *out) {
  const int grid = b->cus * b->blocks_per_cu;
  const auto key = std::make_tuple(K, nmulti, nsingle, b->blocks_per_cu, K ? b->multi_nw : 0,
                                   K ? form : 0);
  auto it = b->graphs.find(key);
  if (it != b->graphs.end()) {
    *out = it->second;
    return LBM_OK;
  }
  HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  hipError_t e = hipSuccess;
  // zero the item tickets of the tick's strip launches (a kernel node: the
  // graph is replayed every tick)
  if (nmulti > 0) e = lbm::launch_fill_i32(b->d_nitems + 1, nmulti, 0, b->stream);
  for (int j = 0; j < nmulti && e == hipSuccess; ++j)
    e = lbm::launch_batch_multi(b->storage, K, b->multi_nw, form, b->d_doms,
                                b->d_items, b->d_nitems, b->multi_grid, j, b->stream);
  for (int k = 0; k < nsingle && e == hipSuccess; ++k)
    e = lbm::launch_batch(b->storage, b->d_doms, b->d_tiles, b->d_ntiles, grid, k, K, b->stream);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(e != hipSuccess ? e : e2, "graph capture");
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  b->graphs[key] = ex;
  *out = ex;
  return LBM_OK;
}

}  // namespace

extern "C" {

void lbm_batch_destroy(lbm_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  free_graphs(b);
  if (b->d_doms) (void)hipFree(b->d_doms);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  if (b->d_ntiles) (void)hipFree(b->d_ntiles);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_nitems) (void)hipFree(b->d_nitems);
  if (b->d_trip) (void)hipFree(b->d_trip);
  if (b->d_chk) (void)hipFree(b->d_chk);
  for (int k = 0; k < 2; ++k) {
    if (b->h_doms[k]) (void)hipHostFree(b->h_doms[k]);
    if (b->copied[k]) (void)hipEventDestroy(b->copied[k]);
    if (b->h_chk[k]) (void)hipHostFree(b->h_chk[k]);
    if (b->chk_copied[k]) (void)hipEventDestroy(b->chk_copied[k]);
    if (b->h_tab[k]) (void)hipHostFree(b->h_tab[k]);
    if (b->tab_copied[k]) (void)hipEventDestroy(b->tab_copied[k]);
  }
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"

namespace {

int validate_members(lbm_handle *const *members, int32_t count) {
  if (!members || count < 1) return fail(LBM_EINVAL, "a batch needs at least one member");
  for (int32_t i = 0; i < count; ++i) {
    if (!members[i]) return fail(LBM_EINVAL, "NULL member");
    if (members[i]->user.storage != members[0]->user.storage)
      return fail(LBM_EINVAL, "all members must share the storage mode");
    if (members[i]->device != members[0]->device)
      return fail(LBM_EINVAL, "all members must live on one device");
    for (int32_t j = 0; j < i; ++j)
      if (members[j] == members[i]) return fail(LBM_EINVAL, "members must be distinct");
    int rc = check_batchable(members[i], (size_t)i);
    if (rc) return rc;
    if (!lbm::strip_row_fits(members[i]->user.nx, members[i]->user.storage))
      return fail(LBM_EINVAL, "members with rows of 2^32 bytes or more are not batched");
  }
  return LBM_OK;
}

// Copy the tile table (optional) and the item table to the device through
// the next pinned staging slot, in stream order on the batch stream: the
// copies land after every launch enqueued before them.
int upload_tables(lbm_batch *b, const std::vector<int2> *tiles, const std::vector<int4> *items) {
  const int sl = b->tab_slot;
  b->tab_slot ^= 1;
  HIP_TRY(hipEventSynchronize(b->tab_copied[sl]), "hipEventSynchronize");  // slot free again
  const size_t tb = tiles ? sizeof(int2) * tiles->size() : 0;
  const size_t ib = items ? sizeof(int4) * items->size() : 0;
  const size_t need = tb + ib + 16;
  if (need > b->tab_cap[sl]) {
    if (b->h_tab[sl]) (void)hipHostFree(b->h_tab[sl]);
    b->h_tab[sl] = nullptr;
    b->tab_cap[sl] = 0;
    const size_t cap = std::max<size_t>(need, (size_t)(1.5 * need));
    HIP_TRY(hipHostMalloc((void **)&b->h_tab[sl], cap, hipHostMallocDefault), "batch table staging");
    b->tab_cap[sl] = cap;
  }
  char *h = b->h_tab[sl];
  size_t off = 0;
  if (tiles) {
    std::memcpy(h, tiles->data(), tb);
    std::memcpy(h + tb, &b->ntiles, sizeof(int));
    HIP_TRY(hipMemcpyAsync(b->d_tiles, h, tb, hipMemcpyHostToDevice, b->stream), "copy(tiles)");
    HIP_TRY(hipMemcpyAsync(b->d_ntiles, h + tb, sizeof(int), hipMemcpyHostToDevice, b->stream),
            "copy(ntiles)");
    off = tb + 8;
  }
  if (items) {
    std::memcpy(h + off, items->data(), ib);
    std::memcpy(h + off + ib, &b->nitems, sizeof(int));
    if (ib)
      HIP_TRY(hipMemcpyAsync(b->d_items, h + off, ib, hipMemcpyHostToDevice, b->stream), "copy(items)");
    HIP_TRY(hipMemcpyAsync(b->d_nitems, h + off + ib, sizeof(int), hipMemcpyHostToDevice, b->stream),
            "copy(nitems)");
  }
  HIP_TRY(hipEventRecord(b->tab_copied[sl], b->stream), "hipEventRecord");
  return LBM_OK;
}

// The strip work-item table for the batch's members and K-step shape
// (empty without K-step launches); reallocates the device table, after
// waiting for the batch stream, only when it outgrows its buffer.
int make_items(lbm_batch *b, std::vector<int4> &items) {
  items.clear();
  if (!b->multi_k) {
    b->nitems = 0;
    return LBM_OK;
  }
  const int W = 64 - 2 * b->multi_k;
  const int nw = b->multi_nw;
  b->multi_form = batch_form(b->members);
  const int per_cu = lbm::batch_multi_per_cu(b->storage, b->multi_k, nw, b->multi_form);
  if (per_cu < 1) return fail(LBM_EDEVICE, "the strip kernel does not fit on a compute unit");
  b->multi_grid = b->cus * per_cu;
  int64_t group_rows = 0;
  for (lbm_handle *h : b->members) {
    const int64_t ngroups = ((h->user.nx + W - 1) / W + nw - 1) / nw;
    group_rows += ngroups * h->user.ny;
  }
  // automatic height: at least one item per resident workgroup (so that
  // the K-step launches fill the device even for a few small members),
  // at most 64 rows (the best height on large batches), at least 8 rows
  const int64_t rows =
      b->multi_rows > 0 ? b->multi_rows
                        : std::min<int64_t>(64, std::max<int64_t>(8, group_rows / b->multi_grid));
  for (size_t i = 0; i < b->members.size(); ++i) {
    const lbm_handle *h = b->members[i];
    const int nstrips = (h->user.nx + W - 1) / W;
    for (int64_t y0 = 0; y0 < h->user.ny; y0 += rows)
      for (int s0 = 0; s0 < nstrips; s0 += nw)
        items.push_back(make_int4((int)i, s0, (int)y0, (int)std::min<int64_t>(rows, h->user.ny - y0)));
  }
  // tallest items first: the workgroups take them in this order, so the
  // short ones (members' last chunks) fill the end of a launch
  std::stable_sort(items.begin(), items.end(),
                   [](const int4 &a, const int4 &c) { return a.w > c.w; });
  if (items.size() > (size_t)0x7fffffff) return fail(LBM_EINVAL, "too many work items");
  if (items.size() > b->item_cap) {
    // the old table (and every graph that points at it) goes away
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    free_graphs(b);
    if (b->d_items) (void)hipFree(b->d_items);
    b->d_items = nullptr;
    b->item_cap = 0;
    const size_t cap = std::max<size_t>(items.size(), (size_t)(1.5 * items.size()));
    HIP_TRY(hipMalloc((void **)&b->d_items, sizeof(int4) * cap), "batch work items");
    b->item_cap = cap;
  }
  b->nitems = (int)items.size();
  return LBM_OK;
}

int build_items(lbm_batch *b) {
  std::vector<int4> items;
  int rc = make_items(b, items);
  if (rc) return rc;
  return upload_tables(b, nullptr, &items);
}

// Rebuild the tile table for a new member list; reuses the device buffers
// (and so the captured graphs) whenever they are large enough.
int batch_set_members_impl(lbm_batch *b, lbm_handle *const *members, int32_t count) {
  int rc = validate_members(members, count);
  if (rc) return rc;
  if (!b->members.empty() && members[0]->user.storage != b->storage)
    return fail(LBM_EINVAL, "members must keep the batch's storage mode");
  std::vector<int2> tiles;
  for (int32_t i = 0; i < count; ++i) {
    const int64_t cells = members[i]->user.nx * members[i]->user.ny;
    for (int64_t c0 = 0; c0 < cells; c0 += lbm::BATCH_TILE) tiles.push_back(make_int2(i, (int)c0));
  }
  if (tiles.size() > (size_t)0x7fffffff) return fail(LBM_EINVAL, "too many tiles");
  // work a member enqueued on another stream (its initialisation) must be
  // done before the batch reads it; on the batch's own stream the order of
  // the stream takes care of it
  for (int32_t i = 0; i < count; ++i)
    if (members[i]->stream != b->stream)
      HIP_TRY(hipStreamSynchronize(members[i]->stream), "hipStreamSynchronize");
  if ((size_t)count > b->dom_cap || tiles.size() > b->tile_cap) {
    // grow: the old buffers (and every graph that points at them) go away
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    free_graphs(b);
    if (b->d_doms) (void)hipFree(b->d_doms);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_trip) (void)hipFree(b->d_trip);
    if (b->d_chk) (void)hipFree(b->d_chk);
    for (int k = 0; k < 2; ++k) {
      if (b->h_doms[k]) (void)hipHostFree(b->h_doms[k]);
      if (b->h_chk[k]) (void)hipHostFree(b->h_chk[k]);
    }
    b->d_doms = nullptr;
    b->d_tiles = nullptr;
    b->d_trip = nullptr;
    b->d_chk = nullptr;
    b->h_doms[0] = b->h_doms[1] = nullptr;
    b->h_chk[0] = b->h_chk[1] = nullptr;
    b->dom_cap = b->tile_cap = 0;
    const size_t dc = std::max<size_t>((size_t)count, 2 * b->members.size());
    const size_t tc = std::max<size_t>(tiles.size(), (size_t)(1.5 * tiles.size()));
    hipError_t e = hipMalloc((void **)&b->d_doms, sizeof(lbm::BatchDomain) * dc);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_tiles, sizeof(int2) * tc);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_trip, sizeof(unsigned long long) * dc);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_chk, sizeof(lbm::CheckDesc) * dc);
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
      e = hipHostMalloc((void **)&b->h_doms[k], sizeof(lbm::BatchDomain) * dc, hipHostMallocDefault);
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
      e = hipHostMalloc((void **)&b->h_chk[k], sizeof(lbm::CheckDesc) * dc, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "batch buffers");
    b->dom_cap = dc;
    b->tile_cap = tc;
  }
  b->ntiles = (int)tiles.size();
  b->members.assign(members, members + count);
  b->storage = members[0]->user.storage;
  // fresh trip slots for the new member list (stream-ordered)
  HIP_TRY(lbm::launch_fill_u64(b->d_trip, count, lbm::TRIP_NONE, b->stream), "detector slots");
  b->any_detector = false;
  std::vector<int4> items;
  rc = make_items(b, items);
  if (rc) return rc;
  return upload_tables(b, &tiles, &items);
}

// After a tick: one launch checks every member whose detector is due at
// its new step count (its own trip word and the batch's slot).
int batch_detector_checks(lbm_batch *b) {
  const int sl = b->chk_slot;
  lbm::CheckDesc *hc = b->h_chk[sl];
  int nd = 0;
  int64_t max_cells = 0;
  bool waited = false;
  for (size_t i = 0; i < b->members.size(); ++i) {
    lbm_handle *h = b->members[i];
    if (!h->det_every || h->steps < h->det_next) continue;
    if (!waited) {  // the copy that last read this staging buffer has finished
      HIP_TRY(hipEventSynchronize(b->chk_copied[sl]), "hipEventSynchronize");
      waited = true;
    }
    lbm::CheckDesc &d = hc[nd++];
    lbm::fill_check_desc(h->cfg, h->lat[h->cur], d);
    d.trip = h->det_word;
    d.trip2 = b->d_trip + i;
    d.step = (unsigned long long)h->steps;
    d.max_dev = h->det_max;
    h->det_next = (h->steps / h->det_every + 1) * h->det_every;
    max_cells = std::max(max_cells, d.n);
  }
  if (!nd) return LBM_OK;
  b->chk_slot ^= 1;
  b->any_detector = true;
  HIP_TRY(hipMemcpyAsync(b->d_chk, hc, sizeof(lbm::CheckDesc) * nd, hipMemcpyHostToDevice,
                         b->stream), "hipMemcpy(detector descriptors)");
  HIP_TRY(hipEventRecord(b->chk_copied[sl], b->stream), "hipEventRecord");
  for (int off = 0; off < nd; off += 65535)
    HIP_TRY(lbm::launch_check_batch(b->storage, b->d_chk + off, std::min(65535, nd - off),
                                    max_cells, b->stream), "detector kernel");
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_create(lbm_handle *const *members, int32_t count, void *stream,
                     lbm_batch **out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_members(members, count);
  if (rc) return rc;
  lbm_batch *b = new (std::nothrow) lbm_batch();
  if (!b) return fail(LBM_ENOMEM, "host allocation failed");
  hipError_t e = hipSuccess;
  if (stream) {
    b->stream = (hipStream_t)stream;
  } else {
    e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    b->own_stream = e == hipSuccess;
  }
  int dev = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipMalloc((void **)&b->d_ntiles, sizeof(int));
  // item count and one ticket per strip launch of a tick (at most 4096 / 2)
  if (e == hipSuccess) e = hipMalloc((void **)&b->d_nitems, sizeof(int) * (1 + 4096 / 2));
  // default shape: K-step strip launches (K = 4 for FP32, 3 for FP64 and FP16)
  b->storage = members[0]->user.storage;
  b->multi_k = b->storage == LBM_STORAGE_F32 ? 4 : 3;
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = hipEventCreateWithFlags(&b->copied[k], hipEventDisableTiming);
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = hipEventCreateWithFlags(&b->chk_copied[k], hipEventDisableTiming);
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = hipEventCreateWithFlags(&b->tab_copied[k], hipEventDisableTiming);
  if (e != hipSuccess) {
    lbm_batch_destroy(b);
    return hip_fail(e, "lbm_batch_create");
  }
  rc = batch_set_members_impl(b, members, count);
  if (rc) {
    lbm_batch_destroy(b);
    return rc;
  }
  *out = b;
  return LBM_OK;
}

int lbm_batch_set_members(lbm_batch *b, lbm_handle *const *members, int32_t count) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  return batch_set_members_impl(b, members, count);
}

int lbm_batch_set_grid(lbm_batch *b, int32_t blocks_per_cu) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (blocks_per_cu < 1 || blocks_per_cu > 64) return fail(LBM_EINVAL, "blocks_per_cu must be 1..64");
  b->blocks_per_cu = blocks_per_cu;
  return LBM_OK;
}

int lbm_batch_set_tuning(lbm_batch *b, const lbm_tuning *t) {
  if (!b || !t) return fail(LBM_EINVAL, "NULL argument");
  if (t->kernel < 0 || t->kernel > lbm::KERNEL_MULTI_MAX)
    return fail(LBM_EINVAL, "kernel must be 0, 1, 2, 3 or 4");
  if (t->kernel >= 2) {
    if (t->block != 64 && t->block != 128 && t->block != 256 && t->block != 512)
      return fail(LBM_EINVAL, "block must be 64, 128, 256 or 512");
    if (t->block > lbm::multi_step_max_block(b->storage, t->kernel))
      return fail(LBM_EINVAL, "block must be at most " +
                                  std::to_string(lbm::multi_step_max_block(b->storage, t->kernel)) +
                                  " for this storage and step count");
    if (t->rows < 0 || t->rows > 4096) return fail(LBM_EINVAL, "rows must be 0 or 1..4096");
  }
  HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  b->multi_k = t->kernel >= 2 ? t->kernel : 0;
  if (b->multi_k) {
    b->multi_nw = t->block / 64;
    b->multi_rows = t->rows;
  }
  return build_items(b);
}

int lbm_batch_set_min_items(lbm_batch *b, int32_t min_items) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (min_items < -1) return fail(LBM_EINVAL, "min_items must be -1 or >= 0");
  b->min_items = min_items;
  return LBM_OK;
}

int lbm_batch_get_tuning(lbm_batch *b, lbm_tuning *t) {
  if (!b || !t) return fail(LBM_EINVAL, "NULL argument");
  t->kernel = b->multi_k;
  t->block = b->multi_k ? 64 * b->multi_nw : lbm::BATCH_TILE;
  t->nontemporal = 0;
  t->rows = b->multi_k ? b->multi_rows : 0;
  return LBM_OK;
}

int lbm_batch_tick(lbm_batch *b, int32_t tick, const int32_t *member_steps) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (tick < 1 || tick > 4096) return fail(LBM_EINVAL, "tick must be 1..4096");
  const size_t n = b->members.size();
  if (member_steps)
    for (size_t i = 0; i < n; ++i)
      if (member_steps[i] < 0 || member_steps[i] > tick)
        return fail(LBM_EINVAL, "member steps must lie in [0, tick]");
  for (size_t i = 0; i < n; ++i) {
    int rc = check_batchable(b->members[i], i);
    if (rc) return rc;
  }
  // a reference field set on a member after the items were made selects
  // that form now (the persistent grid, sized for the earlier form, takes
  // its items by ticket whatever its residency)
  const int form = batch_form(b->members);
  // descriptors go through one of two pinned staging buffers; the copy that
  // last read this buffer (two ticks ago) must have finished
  const int sl = b->slot;
  b->slot ^= 1;
  HIP_TRY(hipEventSynchronize(b->copied[sl]), "hipEventSynchronize");
  lbm::BatchDomain *hd = b->h_doms[sl];
  for (size_t i = 0; i < n; ++i)
    fill_domain(b->members[i], member_steps ? member_steps[i] : tick, hd[i]);
  // stream order puts this copy after the previous tick's launches, which are
  // the last readers of d_doms
  HIP_TRY(hipMemcpyAsync(b->d_doms, hd, sizeof(lbm::BatchDomain) * n,
                         hipMemcpyHostToDevice, b->stream), "hipMemcpy(descriptors)");
  HIP_TRY(hipEventRecord(b->copied[sl], b->stream), "hipEventRecord");
  // K-step strip launches need enough work items to fill the persistent
  // grid (each item marches its rows in sequence); a smaller batch runs as
  // one-step tile launches, which spread it over the whole device. With
  // K-step launches, member i takes st / K of them and then st mod K
  // one-step launches; every launch flips its current lattice once. The
  // graph holds tick / K K-step launches (members needing fewer skip the
  // rest) and as many one-step launches as the largest remainder, so one
  // tick length needs at most K graphs whatever the members' step counts.
  const int need = b->min_items >= 0 ? b->min_items : b->multi_grid;
  const int K = b->multi_k && b->nitems >= need ? b->multi_k : 0;
  int nmulti = 0, nsingle = tick;
  if (K) {
    nmulti = tick / K;
    nsingle = 0;
    for (size_t i = 0; i < n; ++i) {
      const int st = member_steps ? member_steps[i] : tick;
      nsingle = std::max(nsingle, st % K);
    }
  }
  hipGraphExec_t ex = nullptr;
  int rc = batch_graph(b, K, nmulti, nsingle, form, &ex);
  if (rc) return rc;
  HIP_TRY(hipGraphLaunch(ex, b->stream), "hipGraphLaunch");
  for (size_t i = 0; i < n; ++i) {
    const int st = member_steps ? member_steps[i] : tick;
    const int launches = K ? st / K + st % K : st;
    b->members[i]->cur ^= launches & 1;
    b->members[i]->steps += st;
  }
  return batch_detector_checks(b);
}

int lbm_batch_step(lbm_batch *b, int64_t n) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  const int64_t chunk = 4096;
  while (n > 0) {
    const int32_t t = (int32_t)(n < chunk ? n : chunk);
    int rc = lbm_batch_tick(b, t, nullptr);
    if (rc) return rc;
    n -= t;
  }
  return LBM_OK;
}

namespace {
// Fold the batch's trip slots into the members' host copies; the batch
// stream must be idle. Returns the number of members that have tripped.
int batch_fold_trips(lbm_batch *b, int *tripped) {
  *tripped = 0;
  if (b->any_detector) {
    std::vector<unsigned long long> w(b->members.size());
    HIP_TRY(hipMemcpy(w.data(), b->d_trip, sizeof(unsigned long long) * w.size(),
                      hipMemcpyDeviceToHost), "hipMemcpy(detector slots)");
    for (size_t i = 0; i < w.size(); ++i) {
      lbm_handle *h = b->members[i];
      if (w[i] != lbm::TRIP_NONE && (h->tripped_at < 0 || (int64_t)w[i] < h->tripped_at))
        h->tripped_at = (int64_t)w[i];
    }
  }
  for (const lbm_handle *h : b->members) *tripped += h->det_every && h->tripped_at >= 0;
  return LBM_OK;
}
}  // namespace

int lbm_batch_sync(lbm_batch *b) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  int tripped = 0;
  int rc = batch_fold_trips(b, &tripped);
  if (rc) return rc;
  if (tripped)
    return fail(LBM_EUNSTABLE, std::to_string(tripped) + " member(s) tripped the instability detector");
  return LBM_OK;
}

int lbm_batch_detector_status(lbm_batch *b, int64_t *tripped_at) {
  if (!b || !tripped_at) return fail(LBM_EINVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  int tripped = 0;
  int rc = batch_fold_trips(b, &tripped);
  if (rc) return rc;
  for (size_t i = 0; i < b->members.size(); ++i)
    tripped_at[i] = b->members[i]->det_every ? b->members[i]->tripped_at : -1;
  return LBM_OK;
}

int lbm_device_copy(void *dst, const void *src, size_t bytes, void *stream) {
  if (!dst || !src || (bytes & 15)) return fail(LBM_EINVAL, "copy needs non-NULL pointers and bytes % 16 == 0");
  hipError_t e = lbm::launch_copy(dst, src, bytes, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "copy kernel");
  return LBM_OK;
}

}  // extern "C"

namespace {
int validate_vn(const lbm_vn_params *params, int64_t nparams) {
  if (nparams > 65535) return fail(LBM_EINVAL, "at most 65535 parameter sets per call");
  for (int64_t p = 0; p < nparams; ++p) {
    const lbm_vn_params &v = params[p];
    for (int k = 0; k < 9; ++k)
      if (!(v.s[k] >= 0 && v.s[k] <= 2)) return fail(LBM_EINVAL, "rates must lie in [0, 2]");
    if (!(v.chi >= 0) || !is_fin(v.chi) || !(v.rho_f > 0) || !is_fin(v.ux_f) ||
        !is_fin(v.uy_f) || !is_fin(v.shift_n) || !is_fin(v.shift_m))
      return fail(LBM_EINVAL, "bad Von Neumann parameters");
    if (v.variant < 0 || v.variant > 3) return fail(LBM_EINVAL, "unknown variant");
  }
  return LBM_OK;
}
}  // namespace

extern "C" {

int vn_amplification_dev(const lbm_vn_params *params, int64_t nparams, int64_t nk,
                         const double *kx, const double *ky, double *eig,
                         double *G, void *stream) {
  if (!params || nparams < 1 || nk < 0 || (nk > 0 && (!kx || !ky || !eig)))
    return fail(LBM_EINVAL, "bad Von Neumann arguments");
  int rc0 = validate_vn(params, nparams);
  if (rc0) return rc0;
  if (nk == 0) return LBM_OK;
  int rc = check_device(nullptr);
  if (rc) return rc;
  std::vector<lbm::VnParamsDev> hp(nparams);
  for (int64_t p = 0; p < nparams; ++p) {
    for (int k = 0; k < 9; ++k) hp[p].s[k] = params[p].s[k];
    hp[p].n = params[p].shift_n;
    hp[p].m = params[p].shift_m;
    hp[p].chi = params[p].chi;
    hp[p].rho_f = params[p].rho_f;
    hp[p].ux_f = params[p].ux_f;
    hp[p].uy_f = params[p].uy_f;
    hp[p].variant = params[p].variant;
    hp[p].pad_ = 0;
  }
  hipStream_t s = (hipStream_t)stream;
  lbm::VnParamsDev *dp = nullptr;
  HIP_TRY(hipMallocAsync((void **)&dp, sizeof(lbm::VnParamsDev) * nparams, s), "hipMallocAsync(vn params)");
  // a pageable source makes this copy complete before the call returns
  hipError_t e = hipMemcpyAsync(dp, hp.data(), sizeof(lbm::VnParamsDev) * nparams,
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = lbm::launch_vn(dp, (int)nparams, nk, kx, ky, eig, G, s);
  (void)hipFreeAsync(dp, s);
  if (e != hipSuccess) return hip_fail(e, "Von Neumann kernel");
  return LBM_OK;
}

int vn_amplification(const lbm_vn_params *p, int64_t nk, const double *kx,
                     const double *ky, double *eig, double *G) {
  if (!p || nk < 0 || (nk > 0 && (!kx || !ky || !eig)))
    return fail(LBM_EINVAL, "bad Von Neumann arguments");
  int rc = validate_vn(p, 1);
  if (rc) return rc;
  if (nk == 0) return LBM_OK;
  rc = check_device(nullptr);
  if (rc) return rc;
  double *d = nullptr;
  const size_t nkb = sizeof(double) * nk;
  const size_t eb = nkb * 18, gb = G ? nkb * 162 : 0;
  HIP_TRY(hipMalloc((void **)&d, 2 * nkb + eb + gb), "hipMalloc(vn)");
  hipError_t e = hipMemcpy(d, kx, nkb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d + nk, ky, nkb, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e, "hipMemcpy(vn)");
  }
  double *de = d + 2 * nk, *dg = G ? de + 18 * nk : nullptr;
  rc = vn_amplification_dev(p, 1, nk, d, d + nk, de, dg, nullptr);
  if (rc == LBM_OK) {
    e = hipMemcpy(eig, de, eb, hipMemcpyDeviceToHost);
    if (e == hipSuccess && G) e = hipMemcpy(G, dg, gb, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy(vn)");
  }
  (void)hipFree(d);
  return rc;
}

}  // extern "C"

// ---------------------------------------------------------------- D3Q15 lattice

struct lbm3_handle {
  lbm3_config user;
  lbm::Step3Config cfg;
  lbm3_qref q;
  hipStream_t stream = nullptr;
  void *lat[2] = {nullptr, nullptr};
  int cur = 0;
  void *chi_field = nullptr, *chi_x = nullptr, *chi_y = nullptr, *chi_z = nullptr;
  int64_t steps = 0;
  size_t lat_bytes = 0;
  int64_t ncell = 0;
};

namespace {

int validate3(const lbm3_config *c) {
  if (!c) return fail(LBM_EINVAL, "config is NULL");
  if (c->nx < 1 || c->ny < 1 || c->nz < 1) return fail(LBM_EINVAL, "nx, ny and nz must be >= 1");
  if (c->nx > (1 << 30) || c->ny > (1 << 30) || c->nz > (1 << 30) ||
      (double)c->nx * (double)c->ny * (double)c->nz >= 2147483648.0)
    return fail(LBM_EINVAL, "nx * ny * nz must be below 2^31");
  if (!(c->rho_base > 0) || !is_fin(c->rho_base))
    return fail(LBM_EINVAL, "rho_base must be finite and > 0");
  if (!is_fin(c->ux_base) || !is_fin(c->uy_base) || !is_fin(c->uz_base))
    return fail(LBM_EINVAL, "base velocity must be finite");
  for (int k = 0; k < 15; ++k)
    if (!(c->s[k] >= 0.0 && c->s[k] <= 2.0)) return fail(LBM_EINVAL, "relaxation rates must lie in [0, 2]");
  if (!is_fin(c->shift_n) || !is_fin(c->shift_m) || c->shift_n < 0 || c->shift_m < 0)
    return fail(LBM_EINVAL, "shift parameters must be finite and >= 0");
  if (c->storage < LBM_STORAGE_F64 || c->storage > LBM_STORAGE_F16)
    return fail(LBM_EINVAL, "unknown storage mode");
  if (c->variant < LBM_VARIANT_NONE || c->variant > LBM_VARIANT_VISC)
    return fail(LBM_EINVAL, "unknown damping variant");
  if (c->storage == LBM_STORAGE_F16 && !(c->f16_scale > 0 && is_fin(c->f16_scale)))
    return fail(LBM_EINVAL, "f16_scale must be finite and > 0");
  return LBM_OK;
}

void fill_cfg3(lbm3_handle *h) {
  lbm::Step3Config &s = h->cfg;
  const lbm3_config &u = h->user;
  s.nx = (int)u.nx;
  s.ny = (int)u.ny;
  s.nz = (int)u.nz;
  s.storage = u.storage;
  s.variant = u.variant;
  for (int k = 0; k < 15; ++k) s.s[k] = u.s[k];
  s.n = u.shift_n;
  s.m = u.shift_m;
  s.rho_b = u.rho_base;
  s.ub[0] = u.ux_base;
  s.ub[1] = u.uy_base;
  s.ub[2] = u.uz_base;
  s.f16_scale = u.storage == LBM_STORAGE_F16 ? u.f16_scale : 1.0;
  const double dr = h->q.rho_f - u.rho_base;
  s.dcf[0] = dr;
  s.dcf[1] = dr * h->q.ux_f + u.rho_base * (h->q.ux_f - u.ux_base);
  s.dcf[2] = dr * h->q.uy_f + u.rho_base * (h->q.uy_f - u.uy_base);
  s.dcf[3] = dr * h->q.uz_f + u.rho_base * (h->q.uz_f - u.uz_base);
  s.chi_field = h->chi_field;
  s.chi_x = h->chi_x;
  s.chi_y = h->chi_y;
  s.chi_z = h->chi_z;
}

void free_sponge3(lbm3_handle *h) {
  for (void **p : {&h->chi_field, &h->chi_x, &h->chi_y, &h->chi_z}) {
    if (*p) (void)hipFreeAsync(*p, h->stream);
    *p = nullptr;
  }
}

// FP64 host array -> device buffer of the compute type of the handle.
int upload3(lbm3_handle *h, const double *src, size_t n, void **dst) {
  const bool f64 = h->user.storage == LBM_STORAGE_F64;
  const size_t eb = f64 ? 8 : 4;
  HIP_TRY(hipMallocAsync(dst, n * eb, h->stream), "hipMallocAsync(sponge)");
  std::vector<float> tmp;
  const void *p = src;
  if (!f64) {
    tmp.resize(n);
    for (size_t i = 0; i < n; ++i) tmp[i] = (float)src[i];
    p = tmp.data();
  }
  HIP_TRY(hipMemcpyAsync(*dst, p, n * eb, hipMemcpyHostToDevice, h->stream), "hipMemcpy(sponge)");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  return LBM_OK;
}

int check_q3(const lbm3_qref *q) {
  if (!q) return LBM_OK;
  if (!(q->rho_f > 0) || !is_fin(q->rho_f) || !is_fin(q->ux_f) || !is_fin(q->uy_f) ||
      !is_fin(q->uz_f))
    return fail(LBM_EINVAL, "q_ref must be finite with rho_f > 0");
  return LBM_OK;
}

int check_chi3(const double *chi, size_t n, int variant) {
  if (!chi) return LBM_OK;
  for (size_t i = 0; i < n; ++i) {
    if (!is_fin(chi[i]) || chi[i] < 0) return fail(LBM_EINVAL, "chi must be finite and >= 0");
    if (variant == LBM_VARIANT_VISC && chi[i] > 1)
      return fail(LBM_EINVAL, "the viscosity ramp coordinate must lie in [0, 1]");
  }
  return LBM_OK;
}

// FP64 device copy of a host array of n doubles (NULL stays NULL).
int dev_copy3(lbm3_handle *h, const double *src, size_t n, double **dst) {
  *dst = nullptr;
  if (!src) return LBM_OK;
  HIP_TRY(hipMallocAsync((void **)dst, n * 8, h->stream), "hipMallocAsync(fields)");
  HIP_TRY(hipMemcpyAsync(*dst, src, n * 8, hipMemcpyHostToDevice, h->stream), "hipMemcpy(fields)");
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm3_create(const lbm3_config *cfg, const double *rho, const double *ux, const double *uy,
                const double *uz, lbm3_handle **out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate3(cfg);
  if (rc) return rc;
  rc = check_device(nullptr);
  if (rc) return rc;
  lbm3_handle *h = new (std::nothrow) lbm3_handle();
  if (!h) return fail(LBM_ENOMEM, "host allocation failed");
  h->user = *cfg;
  h->stream = (hipStream_t)cfg->stream;
  h->q = lbm3_qref{cfg->rho_base, cfg->ux_base, cfg->uy_base, cfg->uz_base};
  const int eb = lbm::elem_bytes_of(cfg->storage);
  h->ncell = cfg->nx * cfg->ny * cfg->nz;
  h->cfg.pitch = cfg->nx;
  h->cfg.plane_stride = round_up(h->ncell, 256 / eb);
  h->cfg.chi_mode = lbm::CHI_ZERO;
  h->lat_bytes = (size_t)h->cfg.plane_stride * 15 * eb;
  // FP16: two cells per thread halve the accesses per byte (+13% at 256^3)
  h->cfg.kernel = cfg->storage == LBM_STORAGE_F16 && cfg->nx % 2 == 0 ? 1 : 0;
  h->cfg.block = 256;
  fill_cfg3(h);
  for (int k = 0; k < 2; ++k) {
    hipError_t e = hipMalloc(&h->lat[k], h->lat_bytes);
    if (e == hipSuccess) e = hipMemsetAsync(h->lat[k], 0, h->lat_bytes, h->stream);
    if (e != hipSuccess) {
      lbm3_destroy(h);
      return hip_fail(e, "lattice allocation");
    }
  }
  double *d[4];
  const double *src[4] = {rho, ux, uy, uz};
  for (int k = 0; k < 4; ++k) {
    rc = dev_copy3(h, src[k], (size_t)h->ncell, &d[k]);
    if (rc) {
      for (int j = 0; j < k; ++j)
        if (d[j]) (void)hipFreeAsync(d[j], h->stream);
      lbm3_destroy(h);
      return rc;
    }
  }
  hipError_t e = lbm::launch_init3(h->cfg, d[0], d[1], d[2], d[3], h->lat[0], h->stream);
  for (int k = 0; k < 4; ++k)
    if (d[k]) (void)hipFreeAsync(d[k], h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    lbm3_destroy(h);
    return hip_fail(e, "init kernel");
  }
  *out = h;
  return LBM_OK;
}

int lbm3_set_sponge(lbm3_handle *h, const double *chi, const lbm3_qref *q) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  int rc = check_q3(q);
  if (!rc) rc = check_chi3(chi, (size_t)h->ncell, h->user.variant);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  free_sponge3(h);
  h->cfg.chi_mode = lbm::CHI_ZERO;
  if (chi) {
    rc = upload3(h, chi, (size_t)h->ncell, &h->chi_field);
    if (rc) return rc;
    h->cfg.chi_mode = lbm::CHI_FIELD;
  }
  if (q) h->q = *q;
  fill_cfg3(h);
  return LBM_OK;
}

int lbm3_set_sponge_separable(lbm3_handle *h, const double *chi_x, const double *chi_y,
                              const double *chi_z, int32_t combine, const lbm3_qref *q) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (combine != LBM_COMBINE_MAX && combine != LBM_COMBINE_SUM)
    return fail(LBM_EINVAL, "unknown combine mode");
  int rc = check_q3(q);
  const int64_t len[3] = {h->user.nx, h->user.ny, h->user.nz};
  const double *prof[3] = {chi_x, chi_y, chi_z};
  for (int a = 0; a < 3 && !rc; ++a) rc = check_chi3(prof[a], (size_t)len[a], h->user.variant);
  if (rc) return rc;
  if (h->user.variant == LBM_VARIANT_VISC && combine == LBM_COMBINE_SUM)
    return fail(LBM_EINVAL, "the viscosity ramp combines its profiles by max");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  free_sponge3(h);
  void **dst[3] = {&h->chi_x, &h->chi_y, &h->chi_z};
  for (int a = 0; a < 3; ++a) {
    std::vector<double> v(prof[a] ? prof[a] : nullptr, prof[a] ? prof[a] + len[a] : nullptr);
    if (!prof[a]) v.assign((size_t)len[a], 0.0);
    rc = upload3(h, v.data(), v.size(), dst[a]);
    if (rc) return rc;
  }
  h->cfg.chi_mode = combine == LBM_COMBINE_MAX ? lbm::CHI_SEP_MAX : lbm::CHI_SEP_SUM;
  if (q) h->q = *q;
  fill_cfg3(h);
  return LBM_OK;
}

int lbm3_step(lbm3_handle *h, int64_t n) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  for (int64_t k = 0; k < n; ++k) {
    hipError_t e = lbm::launch_step3(h->cfg, h->lat[h->cur], h->lat[1 - h->cur], h->stream);
    if (e != hipSuccess) return hip_fail(e, "step kernel");
    h->cur = 1 - h->cur;
    h->steps += 1;
  }
  return LBM_OK;
}

int lbm3_sync(lbm3_handle *h) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  return LBM_OK;
}

int lbm3_get_populations(lbm3_handle *h, double *f) {
  if (!h || !f) return fail(LBM_EINVAL, "NULL argument");
  const size_t bytes = (size_t)h->ncell * 15 * 8;
  double *d = nullptr;
  HIP_TRY(hipMallocAsync((void **)&d, bytes, h->stream), "hipMallocAsync(populations)");
  hipError_t e = lbm::launch_getpop3(h->cfg, h->lat[h->cur], d, nullptr, nullptr, nullptr,
                                     nullptr, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(f, d, bytes, hipMemcpyDeviceToHost, h->stream);
  (void)hipFreeAsync(d, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "get populations");
  return LBM_OK;
}

int lbm3_set_populations(lbm3_handle *h, const double *f) {
  if (!h || !f) return fail(LBM_EINVAL, "NULL argument");
  const size_t bytes = (size_t)h->ncell * 15 * 8;
  double *d = nullptr;
  HIP_TRY(hipMallocAsync((void **)&d, bytes, h->stream), "hipMallocAsync(populations)");
  hipError_t e = hipMemcpyAsync(d, f, bytes, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = lbm::launch_setpop3(h->cfg, d, h->lat[h->cur], h->stream);
  (void)hipFreeAsync(d, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "set populations");
  h->steps = 0;
  return LBM_OK;
}

int lbm3_moments(lbm3_handle *h, double *rho, double *ux, double *uy, double *uz) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  const size_t bytes = (size_t)h->ncell * 8;
  double *d = nullptr;
  HIP_TRY(hipMallocAsync((void **)&d, 4 * bytes, h->stream), "hipMallocAsync(moments)");
  double *dd[4] = {d, d + h->ncell, d + 2 * h->ncell, d + 3 * h->ncell};
  double *outs[4] = {rho, ux, uy, uz};
  hipError_t e = lbm::launch_getpop3(h->cfg, h->lat[h->cur], nullptr, dd[0], dd[1], dd[2], dd[3],
                                     h->stream);
  for (int k = 0; k < 4 && e == hipSuccess; ++k)
    if (outs[k]) e = hipMemcpyAsync(outs[k], dd[k], bytes, hipMemcpyDeviceToHost, h->stream);
  (void)hipFreeAsync(d, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "moments");
  return LBM_OK;
}

int lbm3_set_tuning(lbm3_handle *h, int32_t kernel, int32_t block) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (kernel != 0 && kernel != 1) return fail(LBM_EINVAL, "kernel must be 0 or 1");
  if (block < 64 || block > 512 || block % 64)
    return fail(LBM_EINVAL, "block must be 64..512 in steps of 64");
  if (kernel == 1 && h->user.nx % 2)
    return fail(LBM_EINVAL, "two cells per thread need an even nx");
  h->cfg.kernel = kernel;
  h->cfg.block = block;
  return LBM_OK;
}

int lbm3_autotune(lbm3_handle *h, int32_t reps, int32_t *kernel, int32_t *block,
                  double *ms_per_step) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (reps < 1) return fail(LBM_EINVAL, "reps must be >= 1");
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  const int saved_k = h->cfg.kernel, saved_b = h->cfg.block;
  double best_t = 1e300;
  int best_k = saved_k, best_b = saved_b;
  for (int k = 0; k <= 1 && e == hipSuccess; ++k) {
    if (k == 1 && h->user.nx % 2) break;
    for (int b = 64; b <= 512 && e == hipSuccess; b *= 2) {
      h->cfg.kernel = k;
      h->cfg.block = b;
      for (int r = 0; r < 1 + reps && e == hipSuccess; ++r) {
        if (r == 1) e = hipEventRecord(e0, h->stream);
        if (e == hipSuccess)
          e = lbm::launch_step3(h->cfg, h->lat[h->cur], h->lat[1 - h->cur], h->stream);
      }
      if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && ms / reps < best_t) {
        best_t = ms / reps;
        best_k = k;
        best_b = b;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->cfg.kernel = saved_k;
  h->cfg.block = saved_b;
  if (e != hipSuccess) return hip_fail(e, "autotune");
  h->cfg.kernel = best_k;
  h->cfg.block = best_b;
  if (kernel) *kernel = best_k;
  if (block) *block = best_b;
  if (ms_per_step) *ms_per_step = best_t;
  return LBM_OK;
}

int lbm3_get_tuning(lbm3_handle *h, int32_t *kernel, int32_t *block) {
  if (!h || !kernel || !block) return fail(LBM_EINVAL, "NULL argument");
  *kernel = h->cfg.kernel;
  *block = h->cfg.block;
  return LBM_OK;
}

int lbm3_steps_done(lbm3_handle *h, int64_t *steps) {
  if (!h || !steps) return fail(LBM_EINVAL, "NULL argument");
  *steps = h->steps;
  return LBM_OK;
}

void lbm3_destroy(lbm3_handle *h) {
  if (!h) return;
  free_sponge3(h);
  (void)hipStreamSynchronize(h->stream);
  for (int k = 0; k < 2; ++k)
    if (h->lat[k]) (void)hipFree(h->lat[k]);
  delete h;
}

}  // extern "C"
