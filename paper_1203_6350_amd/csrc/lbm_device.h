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
  C sig[9], tau[9];   // rows k >= 3: (1 - s_k)/D_k and s_k/D_k (set_relax_coeffs)
};

// 1/D_k, D = diag(9, 6, 6, 36, 36, 12, 12, 4, 4): M's rows are orthogonal,
// M^-1 = M^T D^-1.
__host__ __device__ constexpr double dinv_of(int k) {
  return k == 0 ? 1.0 / 9.0 : (k <= 2 ? 1.0 / 6.0 : (k <= 4 ? 1.0 / 36.0 : (k <= 6 ? 1.0 / 12.0 : 0.25)));
}

// The FP32 relaxation's per-row coefficients from the rates, in the compute
// precision; host and device evaluate the same two IEEE operations, so
// every construction of the parameters gives the same bits.
template <typename C>
__host__ __device__ inline void set_relax_coeffs(CollideParams<C> &p) {
  for (int k = 0; k < 9; ++k) {
    p.sig[k] = (C(1) - p.s[k]) * C(dinv_of(k));
    p.tau[k] = p.s[k] * C(dinv_of(k));
  }
}

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

// m * (1/D) for a conserved moment (mass or momentum row) with D an integer
// row norm. In FP32 a product with the rounded 1/D would scale the moment by
// the same factor at every collision (1 + 7.5e-9 for D = 9, 1 + 3.0e-8 for
// D = 6), which amplifies the acoustic field linearly in time; the
// two-term constant hi + lo = 1/D (to 2^-48) makes the result the correctly
// rounded quotient, whose rounding error varies in sign from value to
// value. FP64 keeps the plain product (its bias, about 1e-16 per step, stays
// far below its bars).
template <typename C>
__device__ __forceinline__ C scale_conserved(C m, double inv_d) {
  if (sizeof(C) == 4) {
    const float hi = (float)inv_d, lo = (float)(inv_d - (double)hi);
    return fmaC(m, C(hi), m * C(lo));
  }
  return m * C(inv_d);
}

// Deviation of the moment equilibria, dm^eq = m^eq(c_b + dc) - m^eq(c_b).
template <typename C>
__device__ __forceinline__ void meq_delta(C dr, C djx, C djy, C rho_b, C ubx,
                                          C uby, C out[9]) {
  const C rho = rho_b + dr;
  const C inv = recip(rho);
  // v = dj - u_b dr, so that j = u_b rho + v and
  //   d(jx^2/rho) = ubx (djx + vx) + vx^2/rho
  //   d(jy^2/rho) = uby (djy + vy) + vy^2/rho
  //   d(jx jy/rho) = ubx djy + uby vx + vx vy/rho
  const C vx = fmaC(-ubx, dr, djx);
  const C vy = fmaC(-uby, dr, djy);
  const C qxx = fmaC(vx * vx, inv, ubx * (djx + vx));
  const C qyy = fmaC(vy * vy, inv, uby * (djy + vy));
  const C qxy = fmaC(vx * vy, inv, fmaC(ubx, djy, uby * vx));
  const C tr = qxx + qyy;
  out[0] = dr;
  out[1] = djx;
  out[2] = djy;
  out[3] = fmaC(C(3), tr, C(-2) * dr);
  out[4] = fmaC(C(-3), tr, dr);
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
// (its value passes unchanged), in every kernel. DEF = true states at
// compile time that the launch has the paper's MRT defaults in this
// respect: all three conserved rates are 0 and the two shift parameters are
// equal (n = m). That drops the run-time rate test, the relaxation
// arithmetic of those moments and the second reciprocal; the results are
// the same bits as without it.
template <typename C, int VAR, bool DEF = false>
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
  dm[3] = fmaC(C(-4), g[0], fmaC(C(2), sd, -sa));
  dm[4] = fmaC(C(4), g[0], fmaC(C(-2), sa, sd));
  dm[5] = fmaC(C(-2), ex, dx);
  dm[6] = fmaC(C(-2), ey, dy);
  dm[7] = ax - ay;
  dm[8] = (g[5] + g[7]) - (g[6] + g[8]);

  // ---- shifted conserved quantities dc* = (dc + n chi dc^f)/(1 + n chi)
  // (m for j), written as dc + (n chi/(1 + n chi)) (dc^f - dc); the
  // remainder dc^f - dc* = (dc^f - dc)/(1 + n chi) is what the damping of
  // the conserved rows needs.
  C dr = dm[0], djx = dm[1], djy = dm[2];
  C d0 = C(0), d1 = C(0), d2 = C(0), inv_n = C(1), inv_m = C(1);
  if (VAR != V_NONE && VAR != V_VISC) {
    d0 = p.dcf0 - dm[0];
    d1 = p.dcf1 - dm[1];
    d2 = p.dcf2 - dm[2];
    const C nchi = p.n * chi, mchi = DEF ? nchi : p.m * chi;
    inv_n = recip(C(1) + nchi);
    inv_m = (DEF || p.n == p.m) ? inv_n : recip(C(1) + mchi);
    const C fn = nchi * inv_n, fm = mchi * inv_m;
    dr = fmaC(fn, d0, dm[0]);
    djx = fmaC(fm, d1, dm[1]);
    djy = fmaC(fm, d2, dm[2]);
  }

  // ---- equilibrium moments at the shifted state
  C meq[9];
  meq_delta(dr, djx, djy, p.rho_b, p.ubx, p.uby, meq);

  // ---- relaxation and damping, m' = dm + S o (dm^eq* - dm) + chi e
  // (Gamma = chi I), delivered as a_k = m'_k / D_k for the back-transform
  // M^-1 = M^T D^-1, D = diag(9, 6, 6, 36, 36, 12, 12, 4, 4).
  constexpr double DINV[9] = {dinv_of(0), dinv_of(1), dinv_of(2), dinv_of(3), dinv_of(4),
                              dinv_of(5), dinv_of(6), dinv_of(7), dinv_of(8)};
  C a[9];
  // conserved rows: a zero rate leaves the moment as it is
  {
    C mc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const C sk = p.s[k];
      mc[k] = (DEF || sk == C(0)) ? dm[k] : fmaC(sk, meq[k] - dm[k], dm[k]);
    }
    if (VAR == V_I) {
      // rows 0-2 of m^ref - m are dc^f - dc
      mc[0] = fmaC(chi, d0, mc[0]);
      mc[1] = fmaC(chi, d1, mc[1]);
      mc[2] = fmaC(chi, d2, mc[2]);
    } else if (VAR == V_II || VAR == V_III) {
      // rows 0-2 of m^ref - m^eq* (II) and of L (dc^f - dc*) (III) are
      // dc^f - dc* = (dc^f - dc)/(1 + n chi) (m for j)
      mc[0] = fmaC(chi * inv_n, d0, mc[0]);
      mc[1] = fmaC(chi * inv_m, d1, mc[1]);
      mc[2] = fmaC(chi * inv_m, d2, mc[2]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) a[k] = scale_conserved(mc[k], DINV[k]);
  }
  // non-conserved rows, one rate per row (the viscosity ramp raises it per
  // cell). In FP32: a_k = ((1 - s_k)/D_k) dm_k + (s_k/D_k) dm^eq*_k +
  // chi e_k / D_k, which saves the separate scaling; in FP64 (twice the
  // registers per value) the relaxed moment is formed first and then
  // scaled. Within a precision every variant takes the same form, so that
  // where chi = 0 they all give the bits of the undamped scheme.
  if (sizeof(C) == 8) {
#pragma unroll
    for (int k = 3; k < 9; ++k) {
      C sk = p.s[k];
      if (VAR == V_VISC) sk = fmaC(C(1) - sk, chi, sk);
      C m = fmaC(sk, meq[k] - dm[k], dm[k]);
      if (VAR == V_I) {
        m = fmaC(chi, mref[k] - dm[k], m);
      } else if (VAR == V_II) {
        if (k == 5) m = fmaC(-chi * inv_m, d1, m);
        else if (k == 6) m = fmaC(-chi * inv_m, d2, m);
        else m = fmaC(chi, mref[k] - meq[k], m);
      } else if (VAR == V_III) {
        if (k == 3) m = fmaC(C(-2) * chi * inv_n, d0, m);
        else if (k == 4) m = fmaC(chi * inv_n, d0, m);
        else if (k == 5) m = fmaC(-chi * inv_m, d1, m);
        else if (k == 6) m = fmaC(-chi * inv_m, d2, m);
      }
      a[k] = m * C(DINV[k]);
    }
  } else {
    C e[9];
#pragma unroll
    for (int k = 3; k < 9; ++k) e[k] = C(0);
    if (VAR == V_I) {
      const C c36 = chi * C(DINV[3]), c12 = chi * C(DINV[5]), c4 = chi * C(DINV[7]);
      e[3] = c36 * (mref[3] - dm[3]);
      e[4] = c36 * (mref[4] - dm[4]);
      e[5] = c12 * (mref[5] - dm[5]);
      e[6] = c12 * (mref[6] - dm[6]);
      e[7] = c4 * (mref[7] - dm[7]);
      e[8] = c4 * (mref[8] - dm[8]);
    } else if (VAR == V_II) {
      // rows 5 and 6 of m^eq and m^ref are -jx and -jy: their differences
      // are those of rows 1 and 2 with the sign flipped
      const C c36 = chi * C(DINV[3]), c4 = chi * C(DINV[7]), cm12 = chi * inv_m * C(DINV[5]);
      e[3] = c36 * (mref[3] - meq[3]);
      e[4] = c36 * (mref[4] - meq[4]);
      e[5] = -cm12 * d1;
      e[6] = -cm12 * d2;
      e[7] = c4 * (mref[7] - meq[7]);
      e[8] = c4 * (mref[8] - meq[8]);
    } else if (VAR == V_III) {
      // L (dc^f - dc*), L c = (rho, jx, jy, -2 rho, rho, -jx, -jy, 0, 0)
      const C c36 = chi * inv_n * C(DINV[3]), cm12 = chi * inv_m * C(DINV[5]);
      e[3] = C(-2) * c36 * d0;
      e[4] = c36 * d0;
      e[5] = -cm12 * d1;
      e[6] = -cm12 * d2;
    }
#pragma unroll
    for (int k = 3; k < 9; ++k) {
      C sig = p.sig[k], tau = p.tau[k];
      if (VAR == V_VISC) {
        const C sk = fmaC(C(1) - p.s[k], chi, p.s[k]);
        sig = (C(1) - sk) * C(DINV[k]);
        tau = sk * C(DINV[k]);
      }
      a[k] = fmaC(sig, dm[k], fmaC(tau, meq[k], e[k]));
    }
  }

  // ---- g' = M^-1 dm' = M^T a
  const C a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3], a4 = a[4], a5 = a[5], a6 = a[6],
          a7 = a[7], a8 = a[8];
  const C pa = fmaC(C(-2), a4, a0 - a3);  // shared by the axis directions
  const C pd = fmaC(C(2), a3, a0 + a4);   // shared by the diagonal directions
  const C tx = fmaC(C(-2), a5, a1), ty = fmaC(C(-2), a6, a2);
  const C bx = a1 + a5, by = a2 + a6;
  const C pxa = pa + a7, pya = pa - a7;
  g[0] = fmaC(C(4), a4 - a3, a0);
  g[1] = pxa + tx;
  g[2] = pya + ty;
  g[3] = pxa - tx;
  g[4] = pya - ty;
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
