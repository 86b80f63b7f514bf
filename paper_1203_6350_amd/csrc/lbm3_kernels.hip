// lbm3_kernels.hip -- HIP kernels of the three-dimensional D3Q15 MRT +
// absorbing-layer step for gfx950 (Xu & Sagaut, arXiv:1203.6350: Section 2
// with the transform matrix of Appendix A.2) and their launchers.
//
// Memory layout (HBM): two lattices, each 15 population planes of nz slices
// of ny rows of `pitch` elements (x fastest); planes `ps` elements apart,
// starting on 256-byte boundaries. A lattice holds post-collision deviations
// g'_i(x) = f'_i(x) - f^eq_i(rho_b, j_b) at the cell that produced them; a
// step pulls g_i(x) = g'_i(x - c_i) (periodic), collides and writes the
// other lattice at x: every element is read and written once per step
// (120 B per cell update in FP32).
#include <hip/hip_fp16.h>

#include <cmath>

#include "lbm3_device.h"
#include "lbm_internal.h"

namespace lbm {

template <typename S>
struct Lat3 {
  typedef typename Store<S>::C C;
  int nx, ny, nz;
  int64_t pitch, slice, ps;  // elements between rows, slices and planes
  C scale[15], inv_scale[15];
};

// FP16 mode: the power of two nearest to w_i * f16_scale (exact scaling).
static double storage_scale3(const Step3Config &c, int i) {
  if (c.storage != 2) return 1.0;
  return std::exp2(std::nearbyint(std::log2(w3_of(i) * c.f16_scale)));
}

template <typename S>
static Lat3<S> make_lat3(const Step3Config &c) {
  typedef typename Store<S>::C C;
  Lat3<S> L;
  L.nx = c.nx;
  L.ny = c.ny;
  L.nz = c.nz;
  L.pitch = c.pitch;
  L.slice = c.pitch * c.ny;
  L.ps = c.plane_stride;
  for (int i = 0; i < 15; ++i) {
    const double sc = storage_scale3(c, i);
    L.scale[i] = C(sc);
    L.inv_scale[i] = C(1.0 / sc);
  }
  return L;
}

template <typename C>
static CollideParams3<C> make_params3(const Step3Config &c) {
  CollideParams3<C> p;
  for (int k = 0; k < 15; ++k) p.s[k] = C(c.s[k]);
  p.n = C(c.n);
  p.m = C(c.m);
  p.rho_b = C(c.rho_b);
  p.ubx = C(c.ub[0]);
  p.uby = C(c.ub[1]);
  p.ubz = C(c.ub[2]);
  p.dcf0 = C(c.dcf[0]);
  p.dcf1 = C(c.dcf[1]);
  p.dcf2 = C(c.dcf[2]);
  p.dcf3 = C(c.dcf[3]);
  return p;
}

__device__ __forceinline__ int wrap3i(int a, int n) {
  return a < 0 ? a + n : (a >= n ? a - n : a);
}

// Sponge strength at a cell: CHI_FIELD a [nz][ny][pitch] field; the
// separable forms combine chi_x[x], chi_y[y], chi_z[z] by max or sum.
template <typename C, int CHI>
__device__ __forceinline__ C chi3_at(const C *field, const C *cx, const C *cy, const C *cz,
                                     int64_t cell, int x, int y, int z) {
  if (CHI == CHI_ZERO) return C(0);
  if (CHI == CHI_FIELD) return field[cell];
  const C a = cx[x], b = cy[y], d = cz[z];
  if (CHI == CHI_SEP_MAX) {
    const C ab = a > b ? a : b;
    return ab > d ? ab : d;
  }
  return (a + b) + d;
}

// One step, one cell per thread; a block covers consecutive cells of one row
// (64..512), blocks are numbered row-major (x, then y, then z) so
// consecutive blocks stream consecutive memory.
template <typename S, int VAR, int CHI>
__global__ __launch_bounds__(512) void step3_kernel(
    const S *__restrict__ src, S *__restrict__ dst, Lat3<S> L,
    CollideParams3<typename Store<S>::C> p, const typename Store<S>::C *__restrict__ chi_field,
    const typename Store<S>::C *__restrict__ chix, const typename Store<S>::C *__restrict__ chiy,
    const typename Store<S>::C *__restrict__ chiz) {
  typedef typename Store<S>::C C;
  const int bx = blockDim.x;
  const int bpr = (L.nx + bx - 1) / bx;
  const int row = blockIdx.x / bpr;  // y + ny z
  const int x = (blockIdx.x - row * bpr) * bx + threadIdx.x;
  if (x >= L.nx) return;
  const int z = row / L.ny, y = row - z * L.ny;
  const int xm = x == 0 ? L.nx - 1 : x - 1, xp = x == L.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? L.ny - 1 : y - 1, yp = y == L.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? L.nz - 1 : z - 1, zp = z == L.nz - 1 ? 0 : z + 1;
  // pull g_i(x) <- g'_i(x - c_i): offsets of the source rows
  const int64_t sz0 = (int64_t)z * L.slice, szm = (int64_t)zm * L.slice,
                szp = (int64_t)zp * L.slice;
  const int64_t ry0 = (int64_t)y * L.pitch, rym = (int64_t)ym * L.pitch,
                ryp = (int64_t)yp * L.pitch;
  const int64_t ps = L.ps;
  C g[15];
  g[0] = Store<S>::load(src + 0 * ps + sz0 + ry0 + x, L.scale[0]);
  g[1] = Store<S>::load(src + 1 * ps + sz0 + ry0 + xm, L.scale[1]);   // c = +x
  g[2] = Store<S>::load(src + 2 * ps + sz0 + ry0 + xp, L.scale[2]);   // c = -x
  g[3] = Store<S>::load(src + 3 * ps + sz0 + rym + x, L.scale[3]);    // c = +y
  g[4] = Store<S>::load(src + 4 * ps + sz0 + ryp + x, L.scale[4]);    // c = -y
  g[5] = Store<S>::load(src + 5 * ps + szm + ry0 + x, L.scale[5]);    // c = +z
  g[6] = Store<S>::load(src + 6 * ps + szp + ry0 + x, L.scale[6]);    // c = -z
  g[7] = Store<S>::load(src + 7 * ps + szm + rym + xm, L.scale[7]);   // (+ + +)
  g[8] = Store<S>::load(src + 8 * ps + szm + rym + xp, L.scale[8]);   // (- + +)
  g[9] = Store<S>::load(src + 9 * ps + szm + ryp + xm, L.scale[9]);   // (+ - +)
  g[10] = Store<S>::load(src + 10 * ps + szm + ryp + xp, L.scale[10]);  // (- - +)
  g[11] = Store<S>::load(src + 11 * ps + szp + rym + xm, L.scale[11]);  // (+ + -)
  g[12] = Store<S>::load(src + 12 * ps + szp + rym + xp, L.scale[12]);  // (- + -)
  g[13] = Store<S>::load(src + 13 * ps + szp + ryp + xm, L.scale[13]);  // (+ - -)
  g[14] = Store<S>::load(src + 14 * ps + szp + ryp + xp, L.scale[14]);  // (- - -)
  const int64_t cell = sz0 + ry0 + x;
  const C chi = chi3_at<C, CHI>(chi_field, chix, chiy, chiz, cell, x, y, z);
  collide3<C, VAR>(g, chi, p);
#pragma unroll
  for (int i = 0; i < 15; ++i) Store<S>::store(dst + i * ps + cell, g[i], L.inv_scale[i]);
}

// Row kernel: each thread owns V consecutive cells of one row and moves
// every plane with one V-element access where the alignment allows it (the
// five planes with c_x = 0; the ten x-shifted ones are read one element to
// the left or right); the first and last thread of a row take the periodic
// wrap with element loads. Threads are numbered over all rows
// (nx % V == 0), so a wave covers 64 V consecutive cells. With V = 2 it
// halves the FP16 accesses per byte.
template <typename S, int V>
struct RowV {
  S v[V];
};

// One access of V * sizeof(S) bytes at element alignment.
template <int B>
struct RowWord;
template <>
struct RowWord<4> {
  typedef unsigned int T __attribute__((aligned(2)));
};
template <>
struct RowWord<8> {
  typedef unsigned int T __attribute__((ext_vector_type(2), aligned(2)));
};
template <>
struct RowWord<16> {
  typedef unsigned int T __attribute__((ext_vector_type(4), aligned(2)));
};

template <typename S, int V>
__device__ __forceinline__ void row_load(RowV<S, V> &d, const S *p) {
  typedef typename RowWord<V * sizeof(S)>::T W;
  const W w = *(const W *)p;
  __builtin_memcpy(&d, &w, sizeof(d));
}

template <typename S, int VAR, int CHI, int V>
__global__ __launch_bounds__(512) void step3_rows(
    const S *__restrict__ src, S *__restrict__ dst, Lat3<S> L,
    CollideParams3<typename Store<S>::C> p, const typename Store<S>::C *__restrict__ chi_field,
    const typename Store<S>::C *__restrict__ chix, const typename Store<S>::C *__restrict__ chiy,
    const typename Store<S>::C *__restrict__ chiz) {
  typedef typename Store<S>::C C;
  const int vpr = L.nx / V;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)vpr * L.ny * L.nz) return;
  const int row = (int)(gid / vpr);  // y + ny z
  const int x0 = (int)(gid - (int64_t)row * vpr) * V;
  const int z = row / L.ny, y = row - z * L.ny;
  const int ym = y == 0 ? L.ny - 1 : y - 1, yp = y == L.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? L.nz - 1 : z - 1, zp = z == L.nz - 1 ? 0 : z + 1;
  const int64_t sz0 = (int64_t)z * L.slice, szm = (int64_t)zm * L.slice,
                szp = (int64_t)zp * L.slice;
  const int64_t ry0 = (int64_t)y * L.pitch, rym = (int64_t)ym * L.pitch,
                ryp = (int64_t)yp * L.pitch;
  const int64_t ps = L.ps;
  // source row of each plane (pull g_i(x) <- g'_i(x - c_i)), before the x shift
  const int64_t base[15] = {sz0 + ry0, sz0 + ry0, sz0 + ry0, sz0 + rym, sz0 + ryp,
                            szm + ry0, szp + ry0, szm + rym, szm + rym, szm + ryp,
                            szm + ryp, szp + rym, szp + rym, szp + ryp, szp + ryp};
  RowV<S, V> in[15];
#pragma unroll
  for (int i = 0; i < 15; ++i) {
    const S *rowp = src + i * ps + base[i];
    if (c3x(i) == 0) {
      row_load(in[i], rowp + x0);
    } else if (c3x(i) > 0) {  // pull from x - 1
      if (x0 > 0) {
        row_load(in[i], rowp + x0 - 1);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) in[i].v[v] = rowp[v == 0 ? L.nx - 1 : v - 1];
      }
    } else {  // pull from x + 1
      if (x0 + V < L.nx) {
        row_load(in[i], rowp + x0 + 1);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) in[i].v[v] = rowp[x0 + v + 1 == L.nx ? 0 : x0 + v + 1];
      }
    }
  }
  const int64_t cell0 = sz0 + ry0 + x0;
  RowV<S, V> out[15];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    C g[15];
#pragma unroll
    for (int i = 0; i < 15; ++i) g[i] = Store<S>::load(&in[i].v[v], L.scale[i]);
    const C chi = chi3_at<C, CHI>(chi_field, chix, chiy, chiz, cell0 + v, x0 + v, y, z);
    collide3<C, VAR>(g, chi, p);
#pragma unroll
    for (int i = 0; i < 15; ++i) Store<S>::store(&out[i].v[v], g[i], L.inv_scale[i]);
  }
#pragma unroll
  for (int i = 0; i < 15; ++i) __builtin_memcpy(dst + i * ps + cell0, &out[i], sizeof(out[i]));
}

template <typename S, int VAR, int CHI, int V>
static hipError_t launch_rows3(const Step3Config &c, const Lat3<S> &L,
                               const CollideParams3<typename Store<S>::C> &p, const void *src,
                               void *dst, hipStream_t stream) {
  typedef typename Store<S>::C C;
  if constexpr (V < 2) {
    return hipErrorInvalidValue;
  } else {
    if (c.nx % V) return hipErrorInvalidValue;
    const int64_t n = (int64_t)(c.nx / V) * c.ny * c.nz;
    const int64_t blocks = (n + c.block - 1) / c.block;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    step3_rows<S, VAR, CHI, V><<<dim3((unsigned)blocks), dim3(c.block), 0, stream>>>(
        (const S *)src, (S *)dst, L, p, (const C *)c.chi_field, (const C *)c.chi_x,
        (const C *)c.chi_y, (const C *)c.chi_z);
    return hipGetLastError();
  }
}

template <typename S, int VAR, int CHI>
static hipError_t launch_step3_t(const Step3Config &c, const void *src, void *dst,
                                 hipStream_t stream) {
  typedef typename Store<S>::C C;
  const Lat3<S> L = make_lat3<S>(c);
  const CollideParams3<C> p = make_params3<C>(c);
  const int bx = c.block;
  if (bx < 64 || bx > 512 || bx % 64) return hipErrorInvalidValue;
  if (c.kernel == 1) return launch_rows3<S, VAR, CHI, 2>(c, L, p, src, dst, stream);
  if (c.kernel != 0) return hipErrorInvalidValue;
  const int64_t blocks = (int64_t)((c.nx + bx - 1) / bx) * c.ny * c.nz;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  step3_kernel<S, VAR, CHI><<<dim3((unsigned)blocks), dim3(bx), 0, stream>>>(
      (const S *)src, (S *)dst, L, p, (const C *)c.chi_field, (const C *)c.chi_x,
      (const C *)c.chi_y, (const C *)c.chi_z);
  return hipGetLastError();
}

template <typename S, int VAR>
static hipError_t step3_chi(const Step3Config &c, const void *src, void *dst, hipStream_t s) {
  switch (c.chi_mode) {
    case CHI_ZERO: return launch_step3_t<S, VAR, CHI_ZERO>(c, src, dst, s);
    case CHI_FIELD: return launch_step3_t<S, VAR, CHI_FIELD>(c, src, dst, s);
    case CHI_SEP_MAX: return launch_step3_t<S, VAR, CHI_SEP_MAX>(c, src, dst, s);
    case CHI_SEP_SUM: return launch_step3_t<S, VAR, CHI_SEP_SUM>(c, src, dst, s);
  }
  return hipErrorInvalidValue;
}

template <typename S>
static hipError_t step3_var(const Step3Config &c, const void *src, void *dst, hipStream_t s) {
  switch (c.variant) {
    case V_NONE: return step3_chi<S, V_NONE>(c, src, dst, s);
    case V_I: return step3_chi<S, V_I>(c, src, dst, s);
    case V_II: return step3_chi<S, V_II>(c, src, dst, s);
    case V_III: return step3_chi<S, V_III>(c, src, dst, s);
    case V_VISC: return step3_chi<S, V_VISC>(c, src, dst, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_step3(const Step3Config &c, const void *src, void *dst, hipStream_t stream) {
  switch (c.storage) {
    case 0: return step3_var<double>(c, src, dst, stream);
    case 1: return step3_var<float>(c, src, dst, stream);
    case 2: return step3_var<__half>(c, src, dst, stream);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- FP64 helpers
struct DevLat3 {
  int nx, ny, nz;
  int64_t pitch, slice, ps;
  double rho_b, ub[3];
  double scale[15], inv_scale[15];
};

static DevLat3 make_devlat3(const Step3Config &c) {
  DevLat3 d;
  d.nx = c.nx;
  d.ny = c.ny;
  d.nz = c.nz;
  d.pitch = c.pitch;
  d.slice = c.pitch * c.ny;
  d.ps = c.plane_stride;
  d.rho_b = c.rho_b;
  for (int k = 0; k < 3; ++k) d.ub[k] = c.ub[k];
  for (int i = 0; i < 15; ++i) {
    d.scale[i] = storage_scale3(c, i);
    d.inv_scale[i] = 1.0 / d.scale[i];
  }
  return d;
}

// f^eq_i(rho_b + dr, j_b + dj) - f^eq_i(rho_b, j_b), every term O(dr, dj).
__device__ __forceinline__ double feq3_dev_i(int i, double dr, const double dj[3],
                                             const DevLat3 &L) {
  const double rho = L.rho_b + dr;
  const double c[3] = {(double)c3x(i), (double)c3y(i), (double)c3z(i)};
  double dJ = 0.0, Ub = 0.0, dq = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dJ += c[a] * dj[a];
    Ub += c[a] * L.ub[a];
    const double va = dj[a] - L.ub[a] * dr;
    dq += 2.0 * L.ub[a] * dj[a] - L.ub[a] * L.ub[a] * dr + va * va / rho;
  }
  const double vJ = dJ - Ub * dr;
  const double dq_c = 2.0 * Ub * dJ - Ub * Ub * dr + vJ * vJ / rho;
  return w3_of(i) * (dr + 3.0 * dJ + 4.5 * dq_c - 1.5 * dq);
}

__device__ __forceinline__ double fbase3_i(int i, const DevLat3 &L) {
  const double cu = c3x(i) * L.ub[0] + c3y(i) * L.ub[1] + c3z(i) * L.ub[2];
  const double u2 = L.ub[0] * L.ub[0] + L.ub[1] * L.ub[1] + L.ub[2] * L.ub[2];
  return w3_of(i) * L.rho_b * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * u2);
}

template <typename S>
__device__ __forceinline__ void store3_dev(S *p, double v, double inv_scale) {
  if constexpr (sizeof(S) == 8)
    *p = v;
  else if constexpr (sizeof(S) == 4)
    *p = (float)v;
  else
    *p = __float2half_rn((float)(v * inv_scale));
}
template <typename S>
__device__ __forceinline__ double load3_dev(const S *p, double scale) {
  if constexpr (sizeof(S) == 8)
    return *p;
  else if constexpr (sizeof(S) == 4)
    return (double)*p;
  else
    return (double)((float)__half2float(*p) * (float)scale);
}

__device__ __forceinline__ void cell3_of(const DevLat3 &L, int64_t cell, int &x, int &y, int &z) {
  const int64_t r = cell / L.nx;
  x = (int)(cell - r * L.nx);
  z = (int)(r / L.ny);
  y = (int)(r - (int64_t)z * L.ny);
}

// Storage location x holds, for direction i, the deviation the next pull
// brings to x + c_i: the equilibrium of the fields (FP64 host arrays
// [nz][ny][nx], NULL = base value) at x + c_i.
template <typename S>
__global__ void init3_kernel(DevLat3 L, const double *__restrict__ rho,
                             const double *__restrict__ ux, const double *__restrict__ uy,
                             const double *__restrict__ uz, S *__restrict__ dst) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= (int64_t)L.nx * L.ny * L.nz) return;
  int x, y, z;
  cell3_of(L, cell, x, y, z);
  const int64_t out = (int64_t)z * L.slice + (int64_t)y * L.pitch + x;
#pragma unroll
  for (int i = 0; i < 15; ++i) {
    const int xs = wrap3i(x + c3x(i), L.nx), ys = wrap3i(y + c3y(i), L.ny),
              zs = wrap3i(z + c3z(i), L.nz);
    const int64_t s = ((int64_t)zs * L.ny + ys) * L.nx + xs;
    const double dr = rho ? rho[s] - L.rho_b : 0.0;
    const double u[3] = {ux ? ux[s] : L.ub[0], uy ? uy[s] : L.ub[1], uz ? uz[s] : L.ub[2]};
    double dj[3];
    for (int a = 0; a < 3; ++a) dj[a] = dr * u[a] + L.rho_b * (u[a] - L.ub[a]);
    store3_dev<S>(dst + i * L.ps + out, feq3_dev_i(i, dr, dj, L), L.inv_scale[i]);
  }
}

// f: [15][nz][ny][nx] full FP64 pre-collision populations -> storage.
template <typename S>
__global__ void setpop3_kernel(DevLat3 L, const double *__restrict__ f, S *__restrict__ dst) {
  const int64_t N = (int64_t)L.nx * L.ny * L.nz;
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= N) return;
  int x, y, z;
  cell3_of(L, cell, x, y, z);
  const int64_t out = (int64_t)z * L.slice + (int64_t)y * L.pitch + x;
#pragma unroll
  for (int i = 0; i < 15; ++i) {
    const int xs = wrap3i(x + c3x(i), L.nx), ys = wrap3i(y + c3y(i), L.ny),
              zs = wrap3i(z + c3z(i), L.nz);
    const double v = f[i * N + ((int64_t)zs * L.ny + ys) * L.nx + xs] - fbase3_i(i, L);
    store3_dev<S>(dst + i * L.ps + out, v, L.inv_scale[i]);
  }
}

// storage -> f [15][nz][ny][nx] full FP64 pre-collision populations, and/or
// the moments rho, u (NULL outputs skipped).
template <typename S>
__global__ void getpop3_kernel(DevLat3 L, const S *__restrict__ src, double *__restrict__ f,
                               double *__restrict__ rho, double *__restrict__ ux,
                               double *__restrict__ uy, double *__restrict__ uz) {
  const int64_t N = (int64_t)L.nx * L.ny * L.nz;
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= N) return;
  int x, y, z;
  cell3_of(L, cell, x, y, z);
  double dr = 0.0, dj[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 15; ++i) {
    const int xs = wrap3i(x - c3x(i), L.nx), ys = wrap3i(y - c3y(i), L.ny),
              zs = wrap3i(z - c3z(i), L.nz);
    const double g =
        load3_dev<S>(src + i * L.ps + (int64_t)zs * L.slice + (int64_t)ys * L.pitch + xs,
                     L.scale[i]);
    if (f) f[i * N + cell] = fbase3_i(i, L) + g;
    dr += g;
    dj[0] += c3x(i) * g;
    dj[1] += c3y(i) * g;
    dj[2] += c3z(i) * g;
  }
  const double r = L.rho_b + dr;
  if (rho) rho[cell] = r;
  if (ux) ux[cell] = (L.rho_b * L.ub[0] + dj[0]) / r;
  if (uy) uy[cell] = (L.rho_b * L.ub[1] + dj[1]) / r;
  if (uz) uz[cell] = (L.rho_b * L.ub[2] + dj[2]) / r;
}

static unsigned cell_blocks3(const Step3Config &c) {
  return (unsigned)(((int64_t)c.nx * c.ny * c.nz + 255) / 256);
}

hipError_t launch_init3(const Step3Config &c, const double *rho, const double *ux,
                        const double *uy, const double *uz, void *dst, hipStream_t stream) {
  const DevLat3 L = make_devlat3(c);
  switch (c.storage) {
    case 0: init3_kernel<double><<<cell_blocks3(c), 256, 0, stream>>>(L, rho, ux, uy, uz, (double *)dst); break;
    case 1: init3_kernel<float><<<cell_blocks3(c), 256, 0, stream>>>(L, rho, ux, uy, uz, (float *)dst); break;
    case 2: init3_kernel<__half><<<cell_blocks3(c), 256, 0, stream>>>(L, rho, ux, uy, uz, (__half *)dst); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_setpop3(const Step3Config &c, const double *f, void *dst, hipStream_t stream) {
  const DevLat3 L = make_devlat3(c);
  switch (c.storage) {
    case 0: setpop3_kernel<double><<<cell_blocks3(c), 256, 0, stream>>>(L, f, (double *)dst); break;
    case 1: setpop3_kernel<float><<<cell_blocks3(c), 256, 0, stream>>>(L, f, (float *)dst); break;
    case 2: setpop3_kernel<__half><<<cell_blocks3(c), 256, 0, stream>>>(L, f, (__half *)dst); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_getpop3(const Step3Config &c, const void *src, double *f, double *rho,
                          double *ux, double *uy, double *uz, hipStream_t stream) {
  const DevLat3 L = make_devlat3(c);
  switch (c.storage) {
    case 0: getpop3_kernel<double><<<cell_blocks3(c), 256, 0, stream>>>(L, (const double *)src, f, rho, ux, uy, uz); break;
    case 1: getpop3_kernel<float><<<cell_blocks3(c), 256, 0, stream>>>(L, (const float *)src, f, rho, ux, uy, uz); break;
    case 2: getpop3_kernel<__half><<<cell_blocks3(c), 256, 0, stream>>>(L, (const __half *)src, f, rho, ux, uy, uz); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lbm
