// lbm_kernels.hip -- HIP kernels of the D2Q9 MRT + absorbing-layer step for
// gfx950 (Xu & Sagaut, arXiv:1203.6350) and their launchers.
//
// Memory layout (HBM): two lattices A and B, each nine population planes of
// ny rows x pitch elements (x fastest), planes plane_stride elements apart.
// A lattice holds post-collision deviations g'(x, t) at the cell where they
// were produced; a step pulls g_i(x, t+1) = g'_i(x - c_i, t) (streaming),
// collides at x and writes g'(x, t+1) into the other lattice at x. So every
// element is read once and written once per step, the writes are fully
// coalesced and the reads of the six x-shifted planes are offset by one
// element.
#include <cmath>
#include <mutex>
#include <type_traits>

#include "lbm_device.h"
#include "lbm_internal.h"
#include "lbm_launch.h"

namespace lbm {

// Per-direction scale of the FP16 mode: the power of two nearest to
// w_i * f16_scale. A power of two makes the scaling exact, so the stored half
// is the single rounding of the FP32 deviation whichever instruction sequence
// the compiler picks for scale-and-convert.
double storage_scale(const StepConfig &c, int i) {
  if (c.storage != 2) return 1.0;
  return std::exp2(std::nearbyint(std::log2(w_of(i) * c.f16_scale)));
}

__device__ __forceinline__ int wrapi(int a, int n) {
  return a < 0 ? a + n : (a >= n ? a - n : a);
}

// ---------------------------------------------------------------- step
// Generic kernel: one cell per thread, a block covers BX consecutive cells of
// one row; blocks are numbered row-major so consecutive blocks (which the
// hardware spreads over the XCDs) stream consecutive memory.
template <typename S, int VAR, int CHI, int BX>
__global__ __launch_bounds__(BX) void step_generic(
    const S *__restrict__ src, S *__restrict__ dst, Lat<S> L,
    CollideParams<typename Store<S>::C> p,
    const typename Store<S>::C *__restrict__ chi_field,
    const typename Store<S>::C *__restrict__ chix,
    const typename Store<S>::C *__restrict__ chiy) {
  typedef typename Store<S>::C C;
  const int bpr = (L.nx + BX - 1) / BX;
  const int y = blockIdx.x / bpr;
  const int x = (blockIdx.x - y * bpr) * BX + threadIdx.x;
  if (x >= L.nx) return;
  const int xm = x == 0 ? L.nx - 1 : x - 1;
  const int xp = x == L.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? L.ny - 1 : y - 1;
  const int yp = y == L.ny - 1 ? 0 : y + 1;
  const int64_t r0 = (int64_t)y * L.pitch, rm = (int64_t)ym * L.pitch,
                rp = (int64_t)yp * L.pitch;
  const int64_t ps = L.ps;
  C g[9];
  // pull: g_i(x) <- g'_i(x - c_i)
  g[0] = Store<S>::load(src + 0 * ps + r0 + x, L.scale[0]);
  g[1] = Store<S>::load(src + 1 * ps + r0 + xm, L.scale[1]);
  g[2] = Store<S>::load(src + 2 * ps + rm + x, L.scale[2]);
  g[3] = Store<S>::load(src + 3 * ps + r0 + xp, L.scale[3]);
  g[4] = Store<S>::load(src + 4 * ps + rp + x, L.scale[4]);
  g[5] = Store<S>::load(src + 5 * ps + rm + xm, L.scale[5]);
  g[6] = Store<S>::load(src + 6 * ps + rm + xp, L.scale[6]);
  g[7] = Store<S>::load(src + 7 * ps + rp + xp, L.scale[7]);
  g[8] = Store<S>::load(src + 8 * ps + rp + xm, L.scale[8]);
  const C chi = chi_at<C, CHI>(chi_field, chix, chiy, r0 + x, x, y);
  collide<C, VAR>(g, chi, p);
#pragma unroll
  for (int i = 0; i < 9; ++i)
    Store<S>::store(dst + i * ps + r0 + x, g[i], L.inv_scale[i]);
}

// Vector kernel: each thread owns V = 16 / sizeof(S) consecutive cells of one
// row and moves every plane with one 16-byte load and one 16-byte store. The
// three planes with c_x = 0 are read aligned; the six x-shifted planes are
// read one element to the left or right (element-aligned 16-byte loads, which
// the HSA unaligned access mode serves). The first and last thread of a row
// take the periodic wrap with element loads. Requires nx % V == 0.
template <typename S>
struct Vec16 {
  S v[16 / sizeof(S)];
};

template <typename S>
__device__ __forceinline__ void load16(Vec16<S> &d, const S *p) {
  __builtin_memcpy(&d, p, 16);
}

template <bool NT, typename S>
__device__ __forceinline__ void store16(S *p, const Vec16<S> &d) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  u4 w;
  __builtin_memcpy(&w, &d, 16);
  if (NT)
    __builtin_nontemporal_store(w, (u4 *)p);
  else
    *(u4 *)p = w;
}

template <typename S, int VAR, int CHI, int BX, bool NT>
__global__ __launch_bounds__(BX) void step_vec(
    const S *__restrict__ src, S *__restrict__ dst, Lat<S> L,
    CollideParams<typename Store<S>::C> p,
    const typename Store<S>::C *__restrict__ chi_field,
    const typename Store<S>::C *__restrict__ chix,
    const typename Store<S>::C *__restrict__ chiy) {
  typedef typename Store<S>::C C;
  constexpr int V = 16 / sizeof(S);
  const int vpr = L.nx / V;
  const int bpr = (vpr + BX - 1) / BX;
  const int y = blockIdx.x / bpr;
  const int xv = (blockIdx.x - y * bpr) * BX + threadIdx.x;
  if (xv >= vpr) return;
  const int x0 = xv * V;
  const int ym = y == 0 ? L.ny - 1 : y - 1;
  const int yp = y == L.ny - 1 ? 0 : y + 1;
  const int64_t r0 = (int64_t)y * L.pitch, rm = (int64_t)ym * L.pitch,
                rp = (int64_t)yp * L.pitch;
  const int64_t ps = L.ps;
  Vec16<S> in[9];
  // c_x = 0: aligned
  load16(in[0], src + 0 * ps + r0 + x0);
  load16(in[2], src + 2 * ps + rm + x0);
  load16(in[4], src + 4 * ps + rp + x0);
  // c_x = +1 (1, 5, 8) pull from x - 1; c_x = -1 (3, 6, 7) pull from x + 1
  if (x0 > 0) {
    load16(in[1], src + 1 * ps + r0 + x0 - 1);
    load16(in[5], src + 5 * ps + rm + x0 - 1);
    load16(in[8], src + 8 * ps + rp + x0 - 1);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int xs = v == 0 ? L.nx - 1 : v - 1;
      in[1].v[v] = src[1 * ps + r0 + xs];
      in[5].v[v] = src[5 * ps + rm + xs];
      in[8].v[v] = src[8 * ps + rp + xs];
    }
  }
  if (x0 + V < L.nx) {
    load16(in[3], src + 3 * ps + r0 + x0 + 1);
    load16(in[6], src + 6 * ps + rm + x0 + 1);
    load16(in[7], src + 7 * ps + rp + x0 + 1);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int xs = x0 + v + 1 == L.nx ? 0 : x0 + v + 1;
      in[3].v[v] = src[3 * ps + r0 + xs];
      in[6].v[v] = src[6 * ps + rm + xs];
      in[7].v[v] = src[7 * ps + rp + xs];
    }
  }
  Vec16<S> out[9];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    C g[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = Store<S>::load(&in[i].v[v], L.scale[i]);
    const C chi = chi_at<C, CHI>(chi_field, chix, chiy, r0 + x0 + v, x0 + v, y);
    collide<C, VAR>(g, chi, p);
#pragma unroll
    for (int i = 0; i < 9; ++i) Store<S>::store(&out[i].v[v], g[i], L.inv_scale[i]);
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) store16<NT>(dst + i * ps + r0 + x0, out[i]);
}

// One step with a per-cell reference state (the paper lets q_ref depend on
// space and time: a far field, or a time-dependent mean of the macroscopic
// quantities, Sec. 1 and Sec. 2.2). qf holds three planes, qps elements
// apart, of the reference's conserved moments as deviations from the base,
// (d rho^f, d j^f_x, d j^f_y), each [ny][pitch]. The cell's reference moments
// dm^ref = m^eq(c^f) - m^eq(c_b) are formed per cell. With alpha != 0 the
// reference then follows the cell's pre-collision conserved moments as an
// exponential running mean, c^f <- c^f + alpha (c - c^f), in place (every
// cell reads and writes only its own entry).
template <typename S, int VAR, int CHI>
__global__ __launch_bounds__(256) void step_qfield(
    const S *__restrict__ src, S *__restrict__ dst, Lat<S> L,
    CollideParams<typename Store<S>::C> p,
    const typename Store<S>::C *__restrict__ chi_field,
    const typename Store<S>::C *__restrict__ chix,
    const typename Store<S>::C *__restrict__ chiy,
    typename Store<S>::C *__restrict__ qf, int64_t qps, typename Store<S>::C alpha) {
  typedef typename Store<S>::C C;
  const int bpr = (L.nx + 255) / 256;
  const int y = blockIdx.x / bpr;
  const int x = (blockIdx.x - y * bpr) * 256 + threadIdx.x;
  if (x >= L.nx) return;
  const int xm = x == 0 ? L.nx - 1 : x - 1;
  const int xp = x == L.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? L.ny - 1 : y - 1;
  const int yp = y == L.ny - 1 ? 0 : y + 1;
  const int64_t r0 = (int64_t)y * L.pitch, rm = (int64_t)ym * L.pitch,
                rp = (int64_t)yp * L.pitch;
  const int64_t ps = L.ps;
  C g[9];
  g[0] = Store<S>::load(src + 0 * ps + r0 + x, L.scale[0]);
  g[1] = Store<S>::load(src + 1 * ps + r0 + xm, L.scale[1]);
  g[2] = Store<S>::load(src + 2 * ps + rm + x, L.scale[2]);
  g[3] = Store<S>::load(src + 3 * ps + r0 + xp, L.scale[3]);
  g[4] = Store<S>::load(src + 4 * ps + rp + x, L.scale[4]);
  g[5] = Store<S>::load(src + 5 * ps + rm + xm, L.scale[5]);
  g[6] = Store<S>::load(src + 6 * ps + rm + xp, L.scale[6]);
  g[7] = Store<S>::load(src + 7 * ps + rp + xp, L.scale[7]);
  g[8] = Store<S>::load(src + 8 * ps + rp + xm, L.scale[8]);
  const int64_t cell = r0 + x;
  const C chi = chi_at<C, CHI>(chi_field, chix, chiy, cell, x, y);
  CollideParams<C> pc = p;
  pc.dcf0 = qf[cell];
  pc.dcf1 = qf[qps + cell];
  pc.dcf2 = qf[2 * qps + cell];
  // pre-collision conserved moments (rows 0-2 of M)
  const C dr = g[0] + ((g[1] + g[3]) + (g[2] + g[4])) + ((g[5] + g[7]) + (g[6] + g[8]));
  const C djx = (g[1] - g[3]) + ((g[5] - g[7]) + (g[8] - g[6]));
  const C djy = (g[2] - g[4]) + ((g[5] - g[7]) + (g[6] - g[8]));
  C mref[9];
  if (VAR == V_I || VAR == V_II) ref_moments(pc, mref);
  collide<C, VAR>(g, chi, pc, mref);
#pragma unroll
  for (int i = 0; i < 9; ++i) Store<S>::store(dst + i * ps + r0 + x, g[i], L.inv_scale[i]);
  if (alpha != C(0)) {
    qf[cell] = fmaC(alpha, dr - pc.dcf0, pc.dcf0);
    qf[qps + cell] = fmaC(alpha, djx - pc.dcf1, pc.dcf1);
    qf[2 * qps + cell] = fmaC(alpha, djy - pc.dcf2, pc.dcf2);
  }
}

// One step on a channel (the acoustic line source of Sec. 4.2): the column
// x = 0 stores the source's equilibrium (deviations given per step in sdev)
// in place of its collision result; with outflow, the column x = nx - 1
// stores the update of column nx - 2 (zero-gradient outflow), which its
// thread computes again from the same inputs. All other cells step as on the
// periodic lattice; the two overridden columns cut it in x.
template <typename S>
struct SrcDev {
  typename Store<S>::C v[9];
};

template <typename S, int VAR, int CHI>
__global__ __launch_bounds__(256) void step_channel(
    const S *__restrict__ src, S *__restrict__ dst, Lat<S> L,
    CollideParams<typename Store<S>::C> p,
    const typename Store<S>::C *__restrict__ chi_field,
    const typename Store<S>::C *__restrict__ chix,
    const typename Store<S>::C *__restrict__ chiy, SrcDev<S> sdev, int outflow) {
  typedef typename Store<S>::C C;
  const int bpr = (L.nx + 255) / 256;
  const int y = blockIdx.x / bpr;
  const int xo = (blockIdx.x - y * bpr) * 256 + threadIdx.x;  // column written
  if (xo >= L.nx) return;
  const int64_t r0 = (int64_t)y * L.pitch;
  const int64_t ps = L.ps;
  if (xo == 0) {
#pragma unroll
    for (int i = 0; i < 9; ++i) Store<S>::store(dst + i * ps + r0, sdev.v[i], L.inv_scale[i]);
    return;
  }
  const int x = outflow && xo == L.nx - 1 ? L.nx - 2 : xo;  // column updated
  const int xm = x == 0 ? L.nx - 1 : x - 1;
  const int xp = x == L.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? L.ny - 1 : y - 1;
  const int yp = y == L.ny - 1 ? 0 : y + 1;
  const int64_t rm = (int64_t)ym * L.pitch, rp = (int64_t)yp * L.pitch;
  C g[9];
  g[0] = Store<S>::load(src + 0 * ps + r0 + x, L.scale[0]);
  g[1] = Store<S>::load(src + 1 * ps + r0 + xm, L.scale[1]);
  g[2] = Store<S>::load(src + 2 * ps + rm + x, L.scale[2]);
  g[3] = Store<S>::load(src + 3 * ps + r0 + xp, L.scale[3]);
  g[4] = Store<S>::load(src + 4 * ps + rp + x, L.scale[4]);
  g[5] = Store<S>::load(src + 5 * ps + rm + xm, L.scale[5]);
  g[6] = Store<S>::load(src + 6 * ps + rm + xp, L.scale[6]);
  g[7] = Store<S>::load(src + 7 * ps + rp + xp, L.scale[7]);
  g[8] = Store<S>::load(src + 8 * ps + rp + xm, L.scale[8]);
  const C chi = chi_at<C, CHI>(chi_field, chix, chiy, r0 + x, x, y);
  collide<C, VAR>(g, chi, p);
#pragma unroll
  for (int i = 0; i < 9; ++i) Store<S>::store(dst + i * ps + r0 + xo, g[i], L.inv_scale[i]);
}

template <typename S, int VAR, int CHI>
static hipError_t launch_channel(const StepConfig &c, const void *src, void *dst,
                                 hipStream_t stream) {
  typedef typename Store<S>::C C;
  Lat<S> L = make_lat<S>(c);
  CollideParams<C> p = make_params<C>(c);
  SrcDev<S> sd;
  for (int i = 0; i < 9; ++i) sd.v[i] = C(c.src_dev[i]);
  const int64_t blocks = (int64_t)((c.nx + 255) / 256) * c.ny;
  step_channel<S, VAR, CHI><<<dim3((unsigned)blocks), dim3(256), 0, stream>>>(
      (const S *)src, (S *)dst, L, p, (const C *)c.chi_field, (const C *)c.chi_x,
      (const C *)c.chi_y, sd, c.outflow);
  return hipGetLastError();
}

template <typename S, int VAR, int CHI>
static hipError_t launch_qfield(const StepConfig &c, const void *src, void *dst,
                                hipStream_t stream) {
  typedef typename Store<S>::C C;
  Lat<S> L = make_lat<S>(c);
  CollideParams<C> p = make_params<C>(c);
  const int64_t blocks = (int64_t)((c.nx + 255) / 256) * c.ny;
  step_qfield<S, VAR, CHI><<<dim3((unsigned)blocks), dim3(256), 0, stream>>>(
      (const S *)src, (S *)dst, L, p, (const C *)c.chi_field, (const C *)c.chi_x,
      (const C *)c.chi_y, (C *)c.qfield, c.qps, C(c.qalpha));
  return hipGetLastError();
}

template <typename S, int VAR, int CHI, int BX>
static hipError_t launch_generic(const StepConfig &c, const void *src, void *dst,
                                 hipStream_t stream) {
  typedef typename Store<S>::C C;
  Lat<S> L = make_lat<S>(c);
  CollideParams<C> p = make_params<C>(c);
  const int64_t blocks = (int64_t)((c.nx + BX - 1) / BX) * c.ny;
  step_generic<S, VAR, CHI, BX><<<dim3((unsigned)blocks), dim3(BX), 0, stream>>>(
      (const S *)src, (S *)dst, L, p, (const C *)c.chi_field,
      (const C *)c.chi_x, (const C *)c.chi_y);
  return hipGetLastError();
}

template <typename S, int VAR, int CHI, int BX, bool NT>
static hipError_t launch_vec(const StepConfig &c, const void *src, void *dst,
                             hipStream_t stream) {
  typedef typename Store<S>::C C;
  constexpr int V = 16 / sizeof(S);
  Lat<S> L = make_lat<S>(c);
  CollideParams<C> p = make_params<C>(c);
  const int vpr = c.nx / V;
  const int64_t blocks = (int64_t)((vpr + BX - 1) / BX) * c.ny;
  step_vec<S, VAR, CHI, BX, NT><<<dim3((unsigned)blocks), dim3(BX), 0, stream>>>(
      (const S *)src, (S *)dst, L, p, (const C *)c.chi_field,
      (const C *)c.chi_x, (const C *)c.chi_y);
  return hipGetLastError();
}

bool vec_supported(const StepConfig &c) {
  const int V = 16 / elem_bytes_of(c.storage);
  return c.nx % V == 0 && c.nx >= V && c.pitch % V == 0;
}


template <typename S, int VAR, int CHI>
static hipError_t launch_step_t(const StepConfig &c, const void *src,
                                void *dst, hipStream_t stream) {
  if (c.qfield) return launch_qfield<S, VAR, CHI>(c, src, dst, stream);
  if (c.channel) return launch_channel<S, VAR, CHI>(c, src, dst, stream);
  const int kernel = c.kernel == KERNEL_VEC && vec_supported(c) ? KERNEL_VEC : KERNEL_GENERIC;
  if (kernel == KERNEL_GENERIC) {
    switch (c.block) {
      case 64: return launch_generic<S, VAR, CHI, 64>(c, src, dst, stream);
      case 128: return launch_generic<S, VAR, CHI, 128>(c, src, dst, stream);
      case 512: return launch_generic<S, VAR, CHI, 512>(c, src, dst, stream);
      default: return launch_generic<S, VAR, CHI, 256>(c, src, dst, stream);
    }
  }
  if (c.nontemporal) {
    switch (c.block) {
      case 64: return launch_vec<S, VAR, CHI, 64, true>(c, src, dst, stream);
      case 128: return launch_vec<S, VAR, CHI, 128, true>(c, src, dst, stream);
      case 512: return launch_vec<S, VAR, CHI, 512, true>(c, src, dst, stream);
      default: return launch_vec<S, VAR, CHI, 256, true>(c, src, dst, stream);
    }
  }
  switch (c.block) {
    case 64: return launch_vec<S, VAR, CHI, 64, false>(c, src, dst, stream);
    case 128: return launch_vec<S, VAR, CHI, 128, false>(c, src, dst, stream);
    case 512: return launch_vec<S, VAR, CHI, 512, false>(c, src, dst, stream);
    default: return launch_vec<S, VAR, CHI, 256, false>(c, src, dst, stream);
  }
}

template <typename S, int VAR>
static hipError_t dispatch_chi(const StepConfig &c, const void *src, void *dst,
                               hipStream_t s) {
  switch (c.chi_mode) {
    case CHI_ZERO: return launch_step_t<S, VAR, CHI_ZERO>(c, src, dst, s);
    case CHI_FIELD: return launch_step_t<S, VAR, CHI_FIELD>(c, src, dst, s);
    case CHI_SEP_MAX: return launch_step_t<S, VAR, CHI_SEP_MAX>(c, src, dst, s);
    case CHI_SEP_SUM: return launch_step_t<S, VAR, CHI_SEP_SUM>(c, src, dst, s);
  }
  return hipErrorInvalidValue;
}

template <typename S>
static hipError_t dispatch_var(const StepConfig &c, const void *src, void *dst,
                               hipStream_t s) {
  switch (c.variant) {
    case V_NONE: return dispatch_chi<S, V_NONE>(c, src, dst, s);
    case V_I: return dispatch_chi<S, V_I>(c, src, dst, s);
    case V_II: return dispatch_chi<S, V_II>(c, src, dst, s);
    case V_III: return dispatch_chi<S, V_III>(c, src, dst, s);
    case V_VISC: return dispatch_chi<S, V_VISC>(c, src, dst, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_step(const StepConfig &c, const void *src, void *dst,
                       hipStream_t stream) {
  switch (c.storage) {
    case 0: return dispatch_var<double>(c, src, dst, stream);
    case 1: return dispatch_var<float>(c, src, dst, stream);
    case 2: return dispatch_var<__half>(c, src, dst, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_multi_steps(const StepConfig &c, int k, const void *src, void *dst,
                              hipStream_t stream) {
#define LBM_MULTI_K(ST)                                                \
  switch (k) {                                                         \
    case 2: return launch_multi_##ST##_k2(c, src, dst, stream);        \
    case 3: return launch_multi_##ST##_k3(c, src, dst, stream);        \
    case 4: return launch_multi_##ST##_k4(c, src, dst, stream);        \
  }                                                                    \
  return hipErrorInvalidValue;
  switch (c.storage) {
    case 0: { LBM_MULTI_K(f64) }
    case 1: { LBM_MULTI_K(f32) }
    case 2: { LBM_MULTI_K(f16) }
  }
#undef LBM_MULTI_K
  return hipErrorInvalidValue;
}

int elem_bytes_of(int storage) {
  return storage == 0 ? 8 : (storage == 1 ? 4 : 2);
}

// ---------------------------------------------------------------- FP64 helpers
// f^eq_i(rho, j) - f^eq_i(rho_b, j_b) in FP64, every term O(drho, dj).
// f^eq_i = w_i [rho + 3 c.j + 9/2 (c.j)^2/rho - 3/2 |j|^2/rho].
__device__ __forceinline__ double feq_dev_i(int i, double dr, double djx,
                                            double djy, double rho_b,
                                            double ubx, double uby) {
  const double rho = rho_b + dr;
  const double cx = cx_of(i), cy = cy_of(i);
  const double dJ = cx * djx + cy * djy;   // d(c.j)
  const double Ub = cx * ubx + cy * uby;   // c.u_b
  const double vJ = dJ - Ub * dr;
  const double dq_c = 2.0 * Ub * dJ - Ub * Ub * dr + vJ * vJ / rho;  // d((c.j)^2/rho)
  const double vx = djx - ubx * dr, vy = djy - uby * dr;
  const double dq_x = 2.0 * ubx * djx - ubx * ubx * dr + vx * vx / rho;
  const double dq_y = 2.0 * uby * djy - uby * uby * dr + vy * vy / rho;
  return w_of(i) * (dr + 3.0 * dJ + 4.5 * dq_c - 1.5 * (dq_x + dq_y));
}

__device__ __forceinline__ double fbase_i(int i, double rho_b, double ubx,
                                          double uby) {
  const double cu = cx_of(i) * ubx + cy_of(i) * uby;
  const double u2 = ubx * ubx + uby * uby;
  return w_of(i) * rho_b * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * u2);
}

template <typename S>
__device__ __forceinline__ void store_dev(S *p, double v, double inv_scale);
template <>
__device__ __forceinline__ void store_dev<double>(double *p, double v, double) {
  *p = v;
}
template <>
__device__ __forceinline__ void store_dev<float>(float *p, double v, double) {
  *p = (float)v;
}
template <>
__device__ __forceinline__ void store_dev<__half>(__half *p, double v,
                                                  double inv_scale) {
  // FP64 -> FP32 -> FP16; the scale keeps values in the normal range
  *p = __float2half_rn((float)(v * inv_scale));
}

template <typename S>
__device__ __forceinline__ double load_dev(const S *p, double scale);
template <>
__device__ __forceinline__ double load_dev<double>(const double *p, double) {
  return *p;
}
template <>
__device__ __forceinline__ double load_dev<float>(const float *p, double) {
  return (double)*p;
}
template <>
__device__ __forceinline__ double load_dev<__half>(const __half *p,
                                                   double scale) {
  return (double)((float)__half2float(*p) * (float)scale);
}

struct DevLat {
  int nx, ny;
  int64_t pitch, ps;
  double rho_b, ubx, uby;
  double scale[9], inv_scale[9];
};

static DevLat make_devlat(const StepConfig &c) {
  DevLat d;
  d.nx = c.nx;
  d.ny = c.ny;
  d.pitch = c.pitch;
  d.ps = c.plane_stride;
  d.rho_b = c.rho_b;
  d.ubx = c.ubx;
  d.uby = c.uby;
  for (int i = 0; i < 9; ++i) {
    d.scale[i] = storage_scale(c, i);
    d.inv_scale[i] = 1.0 / d.scale[i];
  }
  return d;
}

// ---------------------------------------------------------------- init
// Storage location x holds, for direction i, the deviation that the next pull
// brings to cell x + c_i: g'_i(x) = f^eq_i(rho, u at x + c_i) - f^base_i.
template <typename S>
__global__ void init_kernel(DevLat L, const double *__restrict__ rho,
                            const double *__restrict__ ux,
                            const double *__restrict__ uy, S *__restrict__ dst) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= (int64_t)L.nx * L.ny) return;
  const int y = (int)(cell / L.nx), x = (int)(cell - (int64_t)y * L.nx);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int xs = wrapi(x + cx_of(i), L.nx), ys = wrapi(y + cy_of(i), L.ny);
    const int64_t src = (int64_t)ys * L.nx + xs;
    // missing fields take the base value
    const double dr = rho ? rho[src] - L.rho_b : 0.0;
    const double u = ux ? ux[src] : L.ubx, w = uy ? uy[src] : L.uby;
    // j - j_b = drho u + rho_b (u - u_b)
    const double djx = dr * u + L.rho_b * (u - L.ubx);
    const double djy = dr * w + L.rho_b * (w - L.uby);
    const double v = feq_dev_i(i, dr, djx, djy, L.rho_b, L.ubx, L.uby);
    store_dev<S>(dst + i * L.ps + (int64_t)y * L.pitch + x, v, L.inv_scale[i]);
  }
}

// f: [9][ny][nx] full FP64 populations (pre-collision) -> storage.
template <typename S>
__global__ void setpop_kernel(DevLat L, const double *__restrict__ f,
                              S *__restrict__ dst) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)L.nx * L.ny;
  if (cell >= N) return;
  const int y = (int)(cell / L.nx), x = (int)(cell - (int64_t)y * L.nx);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int xs = wrapi(x + cx_of(i), L.nx), ys = wrapi(y + cy_of(i), L.ny);
    const double v = f[i * N + (int64_t)ys * L.nx + xs] -
                     fbase_i(i, L.rho_b, L.ubx, L.uby);
    store_dev<S>(dst + i * L.ps + (int64_t)y * L.pitch + x, v, L.inv_scale[i]);
  }
}

template <typename S>
__global__ void getpop_kernel(DevLat L, const S *__restrict__ src,
                              double *__restrict__ f) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)L.nx * L.ny;
  if (cell >= N) return;
  const int y = (int)(cell / L.nx), x = (int)(cell - (int64_t)y * L.nx);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int xs = wrapi(x - cx_of(i), L.nx), ys = wrapi(y - cy_of(i), L.ny);
    const double g = load_dev<S>(src + i * L.ps + (int64_t)ys * L.pitch + xs,
                                 L.scale[i]);
    f[i * N + cell] = fbase_i(i, L.rho_b, L.ubx, L.uby) + g;
  }
}

template <typename S>
__device__ __forceinline__ void gather_dev(const DevLat &L, const S *src,
                                           int x, int y, double g[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int xs = wrapi(x - cx_of(i), L.nx), ys = wrapi(y - cy_of(i), L.ny);
    g[i] = load_dev<S>(src + i * L.ps + (int64_t)ys * L.pitch + xs, L.scale[i]);
  }
}

template <typename S>
__global__ void moments_kernel(DevLat L, const S *__restrict__ src,
                               double *__restrict__ rho, double *__restrict__ ux,
                               double *__restrict__ uy) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= (int64_t)L.nx * L.ny) return;
  const int y = (int)(cell / L.nx), x = (int)(cell - (int64_t)y * L.nx);
  double g[9];
  gather_dev<S>(L, src, x, y, g);
  double dr = 0.0, djx = 0.0, djy = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    dr += g[i];
    djx += cx_of(i) * g[i];
    djy += cy_of(i) * g[i];
  }
  const double r = L.rho_b + dr;
  if (rho) rho[cell] = r;
  if (ux) ux[cell] = (L.rho_b * L.ubx + djx) / r;
  if (uy) uy[cell] = (L.rho_b * L.uby + djy) / r;
}

// ---------------------------------------------------------------- diagnostics
constexpr int DIAG_BLOCKS = 1024;
constexpr int DIAG_THREADS = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <typename S>
__global__ __launch_bounds__(DIAG_THREADS) void diag_kernel(
    DevLat L, const S *__restrict__ src, double *__restrict__ partials) {
  const int64_t N = (int64_t)L.nx * L.ny;
  const int64_t stride = (int64_t)DIAG_BLOCKS * DIAG_THREADS;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t cell = (int64_t)blockIdx.x * DIAG_THREADS + threadIdx.x;
       cell < N; cell += stride) {
    const int y = (int)(cell / L.nx), x = (int)(cell - (int64_t)y * L.nx);
    double g[9];
    gather_dev<S>(L, src, x, y, g);
    double dr = 0.0, djx = 0.0, djy = 0.0, mx = 0.0;
    bool finite = true;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      dr += g[i];
      djx += cx_of(i) * g[i];
      djy += cy_of(i) * g[i];
      finite = finite && __builtin_isfinite(g[i]);
      mx = fmax(mx, fabs(g[i]));
    }
    acc[0] += dr;
    acc[1] += djx;
    acc[2] += djy;
    acc[3] += dr * dr;
    acc[4] += djx * djx + djy * djy;
    // the largest deviation is taken over the finite cells; non-finite
    // cells are counted instead
    if (finite) acc[5] = fmax(acc[5], mx);
    acc[6] += finite ? 0.0 : 1.0;
  }
  __shared__ double red[DIAG_THREADS / 64][7];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const double v = k == 5 ? wave_max(acc[k]) : wave_sum(acc[k]);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int k = threadIdx.x;
    double v = red[0][k];
    for (int w = 1; w < DIAG_THREADS / 64; ++w)
      v = k == 5 ? fmax(v, red[w][k]) : v + red[w][k];
    partials[(int64_t)blockIdx.x * 7 + k] = v;
  }
}

__global__ __launch_bounds__(64) void diag_final_kernel(
    const double *__restrict__ partials, double *__restrict__ out) {
  // one wave; lane l sums blocks l, l + 64, ... in order, then a fixed tree
  const int lane = threadIdx.x;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = lane; b < DIAG_BLOCKS; b += 64)
#pragma unroll
    for (int k = 0; k < 7; ++k)
      acc[k] = k == 5 ? fmax(acc[k], partials[b * 7 + k]) : acc[k] + partials[b * 7 + k];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const double v = k == 5 ? wave_max(acc[k]) : wave_sum(acc[k]);
    if (lane == 0) out[k] = v;
  }
}

size_t diag_partials_bytes(const StepConfig &) {
  return sizeof(double) * 7 * DIAG_BLOCKS;
}

// Workspace of the allocation-free diagnostics call: the per-block partials
// of one reduction (56 KiB). Each device holds its own copy until the
// process ends; every call on a device shares it, so calls that overlap on
// one device race. Host code never passes the array's name to a kernel: it
// takes the device address from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[7 * DIAG_BLOCKS];

constexpr int SCRATCH_MAX_DEVICES = 64;

hipError_t diag_scratch(int device, double **ptr, size_t *bytes) {
  static std::mutex mu;
  static void *addr[SCRATCH_MAX_DEVICES] = {};
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *ptr = (double *)addr[device];
  *bytes = sizeof(scratch);
  return hipSuccess;
}

// ---------------------------------------------------------------- launchers
template <typename F>
static hipError_t by_storage(int storage, F &&f) {
  switch (storage) {
    case 0: return f((double *)nullptr);
    case 1: return f((float *)nullptr);
    case 2: return f((__half *)nullptr);
  }
  return hipErrorInvalidValue;
}

static unsigned cell_blocks(const StepConfig &c) {
  return (unsigned)(((int64_t)c.nx * c.ny + 255) / 256);
}

hipError_t launch_init(const StepConfig &c, const double *rho,
                       const double *ux, const double *uy, void *dst,
                       hipStream_t stream) {
  DevLat L = make_devlat(c);
  return by_storage(c.storage, [&](auto tag) {
    typedef std::remove_pointer_t<decltype(tag)> S;
    init_kernel<S><<<cell_blocks(c), 256, 0, stream>>>(L, rho, ux, uy, (S *)dst);
    return hipGetLastError();
  });
}

hipError_t launch_set_populations(const StepConfig &c, const double *f,
                                  void *dst, hipStream_t stream) {
  DevLat L = make_devlat(c);
  return by_storage(c.storage, [&](auto tag) {
    typedef std::remove_pointer_t<decltype(tag)> S;
    setpop_kernel<S><<<cell_blocks(c), 256, 0, stream>>>(L, f, (S *)dst);
    return hipGetLastError();
  });
}

hipError_t launch_get_populations(const StepConfig &c, const void *src,
                                  double *f, hipStream_t stream) {
  DevLat L = make_devlat(c);
  return by_storage(c.storage, [&](auto tag) {
    typedef std::remove_pointer_t<decltype(tag)> S;
    getpop_kernel<S><<<cell_blocks(c), 256, 0, stream>>>(L, (const S *)src, f);
    return hipGetLastError();
  });
}

hipError_t launch_moments(const StepConfig &c, const void *src, double *rho,
                          double *ux, double *uy, hipStream_t stream) {
  DevLat L = make_devlat(c);
  return by_storage(c.storage, [&](auto tag) {
    typedef std::remove_pointer_t<decltype(tag)> S;
    moments_kernel<S><<<cell_blocks(c), 256, 0, stream>>>(L, (const S *)src, rho, ux, uy);
    return hipGetLastError();
  });
}

hipError_t launch_diagnostics(const StepConfig &c, const void *src,
                              double *partials, double *out7,
                              hipStream_t stream) {
  DevLat L = make_devlat(c);
  hipError_t e = by_storage(c.storage, [&](auto tag) {
    typedef std::remove_pointer_t<decltype(tag)> S;
    diag_kernel<S><<<DIAG_BLOCKS, DIAG_THREADS, 0, stream>>>(L, (const S *)src, partials);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  diag_final_kernel<<<1, 64, 0, stream>>>(partials, out7);
  return hipGetLastError();
}

// ---------------------------------------------------------------- detector
// Trips when any stored deviation is non-finite or exceeds max_dev in
// magnitude: every element of the nine planes is one of the cells'
// pre-collision deviations (the pull layout permutes them), so this is
// exactly "non-finite count > 0 or max |f - f^base| over finite cells >
// max_dev" of the diagnostics. The planes are streamed linearly (coalesced);
// a block that finds a tripping element lowers the trip word(s) to the step
// count with one atomic minimum.
template <typename S>
__device__ __forceinline__ bool check_planes(const CheckDesc &d, int64_t t, int64_t nt) {
  bool bad = false;
  const S *base = (const S *)d.lat;
#pragma unroll 1
  for (int i = 0; i < 9; ++i) {
    const S *p = base + (int64_t)i * d.ps;
    const double sc = d.scale[i];
    for (int64_t c = t; c < d.n; c += nt) bad |= !(fabs(load_dev<S>(p + c, sc)) <= d.max_dev);
  }
  return bad;
}

__device__ __forceinline__ void check_report(const CheckDesc &d, bool bad) {
  if (__syncthreads_or(bad) && threadIdx.x == 0) {
    atomicMin(d.trip, d.step);
    if (d.trip2) atomicMin(d.trip2, d.step);
  }
}

template <typename S>
__global__ __launch_bounds__(256) void check_kernel(CheckDesc d) {
  const bool bad = check_planes<S>(d, (int64_t)blockIdx.x * 256 + threadIdx.x,
                                   (int64_t)gridDim.x * 256);
  check_report(d, bad);
}

// Batch form: blockIdx.y selects the member's descriptor.
template <typename S>
__global__ __launch_bounds__(256) void check_batch_kernel(const CheckDesc *__restrict__ ds) {
  const CheckDesc d = ds[blockIdx.y];
  const bool bad = check_planes<S>(d, (int64_t)blockIdx.x * 256 + threadIdx.x,
                                   (int64_t)gridDim.x * 256);
  check_report(d, bad);
}

__global__ void fill_u64_kernel(unsigned long long *p, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_i32_kernel(int *p, int64_t n, int v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int *p, int64_t n, int v, hipStream_t stream) {
  if (n < 1) return hipSuccess;
  fill_i32_kernel<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(p, n, v);
  return hipGetLastError();
}

template <typename C>
__global__ void convert_profile_kernel(const double *src, C *dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src ? C(src[i]) : C(0);
}

hipError_t launch_convert_profile(int storage, const double *src, void *dst, int64_t n,
                                  hipStream_t stream) {
  if (n < 1) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (storage == 0)
    convert_profile_kernel<double><<<blocks, 256, 0, stream>>>(src, (double *)dst, n);
  else
    convert_profile_kernel<float><<<blocks, 256, 0, stream>>>(src, (float *)dst, n);
  return hipGetLastError();
}

void fill_check_desc(const StepConfig &c, const void *lat, CheckDesc &d) {
  d.lat = lat;
  d.n = (int64_t)c.nx * c.ny;  // pitch == nx: the cells of a plane are contiguous
  d.ps = c.plane_stride;
  for (int i = 0; i < 9; ++i) d.scale[i] = storage_scale(c, i);
}

static unsigned check_blocks(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

hipError_t launch_check(int storage, const CheckDesc &d, hipStream_t stream) {
  return by_storage(storage, [&](auto tag) {
    typedef std::remove_pointer_t<decltype(tag)> S;
    check_kernel<S><<<check_blocks(d.n), 256, 0, stream>>>(d);
    return hipGetLastError();
  });
}

hipError_t launch_check_batch(int storage, const CheckDesc *descs_dev, int ndesc,
                              int64_t max_cells, hipStream_t stream) {
  if (ndesc < 1) return hipSuccess;
  if (ndesc > 65535) return hipErrorInvalidValue;
  const unsigned bx = check_blocks(max_cells) < 64 ? check_blocks(max_cells) : 64;
  return by_storage(storage, [&](auto tag) {
    typedef std::remove_pointer_t<decltype(tag)> S;
    check_batch_kernel<S><<<dim3(bx, (unsigned)ndesc), 256, 0, stream>>>(descs_dev);
    return hipGetLastError();
  });
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v,
                           hipStream_t stream) {
  if (n < 1) return hipSuccess;
  fill_u64_kernel<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(p, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------- copy probe
// One 16-byte element per thread, exact grid, non-temporal stores: the plain
// streaming copy used to calibrate bandwidth and traffic counters.
__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ src,
                                                   uint4 *__restrict__ dst,
                                                   int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    u4 w;
    __builtin_memcpy(&w, &src[i], 16);
    __builtin_nontemporal_store(w, (u4 *)&dst[i]);
  }
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes,
                       hipStream_t stream) {
  const int64_t n = (int64_t)(bytes / 16);
  const int64_t blocks = (n + 255) / 256;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  copy_kernel<<<dim3((unsigned)blocks), 256, 0, stream>>>((const uint4 *)src, (uint4 *)dst, n);
  return hipGetLastError();
}

}  // namespace lbm
