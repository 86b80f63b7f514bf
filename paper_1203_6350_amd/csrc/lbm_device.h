// lbm_device.h -- per-cell arithmetic of the D2Q9 MRT step with the
// absorbing-layer damping term (Xu & Sagaut, arXiv:1203.6350, Section 2),
// shared by every kernel of the library.
//
// The state is stored as deviations g_i = f_i - f_i^base from a uniform base
// equilibrium f^base = f^eq(rho_b, u_b). Everything below works on
// deviations of moments, so the weak acoustic signal never has to be
// recovered from the difference of two O(1) numbers:
//
//   dm       = M g                       (transform of Appendix A.1; integer
//                                         coefficients, adds only)
//   dc*      = (dc + n chi dc^f)/(1 + n chi)   (exact solution of the implicit
//                                         rho*, rho* u* of Sections 2.2.1-2.2.3;
//                                         every damping force has
//                                         sum F = chi (rho^f - rho*) and
//                                         sum c F = chi (j^f - j*))
//   dm^eq*   = m^eq(c_b + dc*) - m^eq(c_b)   (moment equilibria, written so
//                                         that every term is O(dc))
//   d        = chi (dm^ref - dm)          Type I   (f* = f)
//              chi (dm^ref - dm^eq*)      Type II  (f* = f^eq(rho*, u*))
//              chi L (dc^f - dc*)         Type III (f* = f^L(rho*, u*))
//   dm'      = dm + S o (dm^eq* - dm) + d (Lambda = M^-1 S M, Gamma = chi I;
//                                         d enters as fma(chi, e, .))
//   g'       = M^-1 dm' = M^T diag(1/9,1/6,1/6,1/36,1/36,1/12,1/12,1/4,1/4) dm'
//
// m^eq(rho, j) = (rho, jx, jy, -2 rho + 3|j|^2/rho, rho - 3|j|^2/rho, -jx, -jy,
//                 (jx^2 - jy^2)/rho, jx jy/rho) is the moment image of the
// standard second-order D2Q9 equilibrium (c_s^2 = 1/3); its part linear in
// (rho, j) is m^L = L c = (rho, jx, jy, -2 rho, rho, -jx, -jy, 0, 0).
// With u_b the base velocity, v = dj - u_b drho and rho = rho_b + drho, the
// quadratic moments change by
//   d(j_a j_b / rho) = u_ba dj_b + u_bb dj_a - u_ba u_bb drho + v_a v_b / rho.
//
// All floating-point operations are written explicitly (fma where used) and
// the library is compiled without automatic contraction, so a cell gives the
// same bits in every kernel and launch shape.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace lbm {

// V_VISC is the comparison strategy of Section 4.1: no damping term; the
// non-conserved relaxation rates ramp linearly to 1 inside the layer,
// s_k(x) = s_k + (1 - s_k) xi(x), with xi in [0, 1] supplied where the other
// variants take chi.
enum Variant { V_NONE = 0, V_I = 1, V_II = 2, V_III = 3, V_VISC = 4 };
enum ChiMode { CHI_ZERO = 0, CHI_FIELD = 1, CHI_SEP_MAX = 2, CHI_SEP_SUM = 3 };

// Velocity set in the column order of M (Appendix A.1).
__host__ __device__ constexpr int cx_of(int i) {
  return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cy_of(int i) {
  return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}
__host__ __device__ constexpr double w_of(int i) {
  return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}

// Parameters of the collision in compute precision C.
template <typename C>
struct CollideParams {
  C s[9];          // diagonal of S
  C n, m;          // shift parameters of rho* and j*
  C rho_b, ubx, uby;  // base state
  C dcf0, dcf1, dcf2; // q_ref - base: (rho^f - rho_b, j^f - j_b)
};

template <typename C>
__device__ __forceinline__ C fmaC(C a, C b, C c);
template <>
__device__ __forceinline__ float fmaC<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
template <>
__device__ __forceinline__ double fmaC<double>(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

// Reciprocal: the hardware FP32 reciprocal (within 1 ulp) in FP32; exact
// division in FP64.
template <typename C>
__device__ __forceinline__ C recip(C x);
template <>
__device__ __forceinline__ float recip<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}
template <>
__device__ __forceinline__ double recip<double>(double x) {
  return 1.0 / x;
}

// Deviation of the moment equilibria, dm^eq = m^eq(c_b + dc) - m^eq(c_b).
template <typename C>
__device__ __forceinline__ void meq_delta(C dr, C djx, C djy, C rho_b, C ubx,
                                          C uby, C out[9]) {
  const C rho = rho_b + dr;
  const C inv = recip(rho);
  const C vx = djx - ubx * dr;
  const C vy = djy - uby * dr;
  // d(jx^2/rho), d(jy^2/rho), d(jx jy/rho)
  const C qxx = fmaC(vx * vx, inv, ubx * (C(2) * djx - ubx * dr));
  const C qyy = fmaC(vy * vy, inv, uby * (C(2) * djy - uby * dr));
  const C qxy = fmaC(vx * vy, inv, ubx * djy + uby * djx - ubx * uby * dr);
  const C tr = qxx + qyy;
  out[0] = dr;
  out[1] = djx;
  out[2] = djy;
  out[3] = C(3) * tr - C(2) * dr;
  out[4] = dr - C(3) * tr;
  out[5] = -djx;
  out[6] = -djy;
  out[7] = qxx - qyy;
  out[8] = qxy;
}

// Reference moments dm^ref = m^eq(c^f) - m^eq(c_b) of the damping Types I
// and II. They depend on the launch parameters only, so a kernel that
// collides many cells per thread computes them once.
template <typename C>
__device__ __forceinline__ void ref_moments(const CollideParams<C> &p, C mref[9]) {
  meq_delta(p.dcf0, p.dcf1, p.dcf2, p.rho_b, p.ubx, p.uby, mref);
}

// One collision in deviation form; g holds the pre-collision deviations on
// entry and the post-collision deviations on return. mref comes from
// ref_moments (read by Types I and II only).
//
// A conserved moment (k < 3) whose rate is exactly 0 skips the relaxation
// (its value passes unchanged), in every kernel; SC0 = true states at
// compile time that all three conserved rates are 0 (the paper's MRT
// default), which drops the run-time test and the relaxation arithmetic of
// those moments.
template <typename C, int VAR, bool SC0 = false>
__device__ __forceinline__ void collide(C g[9], C chi, const CollideParams<C> &p,
                                        const C mref[9]) {
  // ---- dm = M g (Appendix A.1)
  const C ax = g[1] + g[3], ay = g[2] + g[4];
  const C sa = ax + ay;                     // axis populations
  const C sd = (g[5] + g[7]) + (g[6] + g[8]);  // diagonal populations
  const C ex = g[1] - g[3], ey = g[2] - g[4];
  const C dx = (g[5] - g[7]) + (g[8] - g[6]);  // g5 - g6 - g7 + g8
  const C dy = (g[5] - g[7]) + (g[6] - g[8]);  // g5 + g6 - g7 - g8
  C dm[9];
  dm[0] = g[0] + sa + sd;
  dm[1] = ex + dx;
  dm[2] = ey + dy;
  dm[3] = C(2) * sd - sa - C(4) * g[0];
  dm[4] = C(4) * g[0] - C(2) * sa + sd;
  dm[5] = dx - C(2) * ex;
  dm[6] = dy - C(2) * ey;
  dm[7] = ax - ay;
  dm[8] = (g[5] + g[7]) - (g[6] + g[8]);

  // ---- shifted conserved quantities dc*
  C dr = dm[0], djx = dm[1], djy = dm[2];
  if (VAR != V_NONE && VAR != V_VISC) {
    const C nchi = p.n * chi, mchi = p.m * chi;
    const C inv_n = recip(C(1) + nchi);
    const C inv_m = p.n == p.m ? inv_n : recip(C(1) + mchi);
    dr = fmaC(nchi, p.dcf0, dm[0]) * inv_n;
    djx = fmaC(mchi, p.dcf1, dm[1]) * inv_m;
    djy = fmaC(mchi, p.dcf2, dm[2]) * inv_m;
  }

  // ---- equilibrium moments at the shifted state
  C meq[9];
  meq_delta(dr, djx, djy, p.rho_b, p.ubx, p.uby, meq);

  // ---- relaxation, then the damping d = chi e (Gamma = chi I) added with
  // one fused multiply-add per moment
  C mp[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    C sk = p.s[k];
    if (VAR == V_VISC && k >= 3) sk = fmaC(C(1) - sk, chi, sk);
    if (k < 3)
      mp[k] = (SC0 || sk == C(0)) ? dm[k] : fmaC(sk, meq[k] - dm[k], dm[k]);
    else
      mp[k] = fmaC(sk, meq[k] - dm[k], dm[k]);
  }
  if (VAR == V_I) {
#pragma unroll
    for (int k = 0; k < 9; ++k) mp[k] = fmaC(chi, mref[k] - dm[k], mp[k]);
  } else if (VAR == V_II) {
    // rows 5 and 6 of m^eq (and of m^ref) are -jx and -jy: their damping
    // differences are those of rows 1 and 2 with the sign flipped
    C e[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) e[k] = mref[k] - meq[k];
    e[5] = -e[1];
    e[6] = -e[2];
#pragma unroll
    for (int k = 0; k < 9; ++k) mp[k] = fmaC(chi, e[k], mp[k]);
  } else if (VAR == V_III) {
    // e = L (dc^f - dc*), L c = (rho, jx, jy, -2 rho, rho, -jx, -jy, 0, 0)
    const C a = p.dcf0 - dr, bx = p.dcf1 - djx, by = p.dcf2 - djy;
    mp[0] = fmaC(chi, a, mp[0]);
    mp[1] = fmaC(chi, bx, mp[1]);
    mp[2] = fmaC(chi, by, mp[2]);
    mp[3] = fmaC(chi, C(-2) * a, mp[3]);
    mp[4] = fmaC(chi, a, mp[4]);
    mp[5] = fmaC(chi, -bx, mp[5]);
    mp[6] = fmaC(chi, -by, mp[6]);
  }

  // ---- g' = M^-1 dm'
  const C a0 = mp[0] * C(1.0 / 9.0);
  const C a1 = mp[1] * C(1.0 / 6.0), a2 = mp[2] * C(1.0 / 6.0);
  const C a3 = mp[3] * C(1.0 / 36.0), a4 = mp[4] * C(1.0 / 36.0);
  const C a5 = mp[5] * C(1.0 / 12.0), a6 = mp[6] * C(1.0 / 12.0);
  const C a7 = mp[7] * C(0.25), a8 = mp[8] * C(0.25);
  const C pa = a0 - a3 - C(2) * a4;   // shared by the axis directions
  const C pd = a0 + C(2) * a3 + a4;   // shared by the diagonal directions
  const C tx = a1 - C(2) * a5, ty = a2 - C(2) * a6;
  const C bx = a1 + a5, by = a2 + a6;
  g[0] = a0 - C(4) * a3 + C(4) * a4;
  g[1] = (pa + tx) + a7;
  g[2] = (pa + ty) - a7;
  g[3] = (pa - tx) + a7;
  g[4] = (pa - ty) - a7;
  g[5] = (pd + bx) + (by + a8);
  g[6] = (pd - bx) + (by - a8);
  g[7] = (pd - bx) - (by - a8);
  g[8] = (pd + bx) - (by + a8);
}

// The same collision for a thread that collides one cell.
template <typename C, int VAR>
__device__ __forceinline__ void collide(C g[9], C chi, const CollideParams<C> &p) {
  C mref[9];
  if (VAR == V_I || VAR == V_II) ref_moments(p, mref);
  collide<C, VAR, false>(g, chi, p, mref);
}

// Storage traits: load/store one population element with the per-direction
// scale of the FP16 mode.
template <typename S>
struct Store;
template <>
struct Store<double> {
  typedef double C;
  static __device__ __forceinline__ double load(const double *p, double) {
    return *p;
  }
  static __device__ __forceinline__ void store(double *p, double v, double) {
    *p = v;
  }
};
template <>
struct Store<float> {
  typedef float C;
  static __device__ __forceinline__ float load(const float *p, float) {
    return *p;
  }
  static __device__ __forceinline__ void store(float *p, float v, float) {
    *p = v;
  }
};
template <>
struct Store<__half> {
  typedef float C;
  static __device__ __forceinline__ float load(const __half *p, float scale) {
    return __half2float(*p) * scale;
  }
  static __device__ __forceinline__ void store(__half *p, float v,
                                               float inv_scale) {
    *p = __float2half_rn(v * inv_scale);
  }
};

// Sponge strength at a cell.
template <typename C, int CHI>
__device__ __forceinline__ C chi_at(const C *field, const C *chix,
                                    const C *chiy, int64_t cell, int x,
                                    int y) {
  if (CHI == CHI_ZERO) return C(0);
  if (CHI == CHI_FIELD) return field[cell];
  const C a = chix[x], b = chiy[y];
  if (CHI == CHI_SEP_MAX) return a > b ? a : b;
  return a + b;
}

}  // namespace lbm
