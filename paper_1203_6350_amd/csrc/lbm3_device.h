// lbm3_device.h -- per-cell arithmetic of the three-dimensional D3Q15 MRT step
// with the absorbing-layer damping term (Xu & Sagaut, arXiv:1203.6350:
// Section 2 with the transform matrix of Appendix A.2), in the deviation form
// of lbm_device.h: g_i = f_i - f^eq_i(rho_b, j_b).
//
// Velocity order of the columns of M's rows 1-3: 0 rest; 1, 2 = +x, -x;
// 3, 4 = +y, -y; 5, 6 = +z, -z; 7..14 = the diagonals (sx, sy, sz) with
// (+++), (-++), (+-+), (--+), (++-), (-+-), (+--), (---).
// Moment rows: rho, jx, jy, jz, e, eps, qx, qy, qz, 3pxx, pww, pxy, pyz, pzx,
// mxyz; row norms D = (15, 10, 10, 10, 18, 360, 40, 40, 40, 12, 4, 8, 8, 8, 8),
// the rows being orthogonal, so M^-1 = M^T D^-1.
// Equilibrium moments of the second-order equilibrium (c_s^2 = 1/3):
//   m^eq = (rho, j, -rho + |j|^2/rho, rho - 5 |j|^2/rho, -7/3 j,
//           (2 jx^2 - jy^2 - jz^2)/rho, (jy^2 - jz^2)/rho, jx jy/rho,
//           jy jz/rho, jz jx/rho, 0);
// its part linear in (rho, j): m^L = (rho, j, -rho, rho, -7/3 j, 0, ..., 0).
#pragma once

#include "lbm_device.h"

namespace lbm {

template <typename C>
struct CollideParams3 {
  C s[15];
  C n, m;
  C rho_b, ubx, uby, ubz;
  C dcf0, dcf1, dcf2, dcf3;  // q_ref - base: (rho^f - rho_b, j^f - j_b)
};

__host__ __device__ constexpr int c3x(int i) {
  return i == 1 ? 1 : i == 2 ? -1 : (i >= 7 ? ((i - 7) % 2 == 0 ? 1 : -1) : 0);
}
__host__ __device__ constexpr int c3y(int i) {
  return i == 3 ? 1 : i == 4 ? -1 : (i >= 7 ? (((i - 7) / 2) % 2 == 0 ? 1 : -1) : 0);
}
__host__ __device__ constexpr int c3z(int i) {
  return i == 5 ? 1 : i == 6 ? -1 : (i >= 7 ? (i < 11 ? 1 : -1) : 0);
}
__host__ __device__ constexpr double w3_of(int i) {
  return i == 0 ? 2.0 / 9.0 : (i <= 6 ? 1.0 / 9.0 : 1.0 / 72.0);
}

// Deviation of the equilibrium moments, dm^eq = m^eq(c_b + dc) - m^eq(c_b).
// d(j_a j_b / rho) = u_ba dj_b + u_bb dj_a - u_ba u_bb drho + v_a v_b / rho,
// v = dj - u_b drho, rho = rho_b + drho.
template <typename C>
__device__ __forceinline__ void meq3_delta(C dr, C djx, C djy, C djz, const CollideParams3<C> &p,
                                           C out[15]) {
  const C rho = p.rho_b + dr;
  const C inv = recip(rho);
  const C vx = djx - p.ubx * dr, vy = djy - p.uby * dr, vz = djz - p.ubz * dr;
  const C qxx = fmaC(vx * vx, inv, p.ubx * (C(2) * djx - p.ubx * dr));
  const C qyy = fmaC(vy * vy, inv, p.uby * (C(2) * djy - p.uby * dr));
  const C qzz = fmaC(vz * vz, inv, p.ubz * (C(2) * djz - p.ubz * dr));
  const C qxy = fmaC(vx * vy, inv, p.ubx * djy + p.uby * djx - p.ubx * p.uby * dr);
  const C qyz = fmaC(vy * vz, inv, p.uby * djz + p.ubz * djy - p.uby * p.ubz * dr);
  const C qzx = fmaC(vz * vx, inv, p.ubz * djx + p.ubx * djz - p.ubz * p.ubx * dr);
  const C tr = (qxx + qyy) + qzz;
  out[0] = dr;
  out[1] = djx;
  out[2] = djy;
  out[3] = djz;
  out[4] = tr - dr;
  out[5] = dr - C(5) * tr;
  out[6] = C(-7.0 / 3.0) * djx;
  out[7] = C(-7.0 / 3.0) * djy;
  out[8] = C(-7.0 / 3.0) * djz;
  out[9] = C(2) * qxx - (qyy + qzz);
  out[10] = qyy - qzz;
  out[11] = qxy;
  out[12] = qyz;
  out[13] = qzx;
  out[14] = C(0);
}

template <typename C>
__device__ __forceinline__ void ref_moments3(const CollideParams3<C> &p, C mref[15]) {
  meq3_delta(p.dcf0, p.dcf1, p.dcf2, p.dcf3, p, mref);
}

// One D3Q15 collision in deviation form; g: pre-collision deviations in,
// post-collision deviations out. mref from ref_moments3 (Types I and II).
template <typename C, int VAR>
__device__ __forceinline__ void collide3(C g[15], C chi, const CollideParams3<C> &p,
                                         const C mref[15]) {
  // ---- dm = M g
  const C ax = g[1] + g[2], ay = g[3] + g[4], az = g[5] + g[6];
  const C sa = (ax + ay) + az;
  const C dx = g[1] - g[2], dy = g[3] - g[4], dz = g[5] - g[6];
  // diagonals: sums and signed sums over the (sx, sy, sz) pattern
  const C p78 = g[7] + g[8], m78 = g[7] - g[8];
  const C p910 = g[9] + g[10], m910 = g[9] - g[10];
  const C p1112 = g[11] + g[12], m1112 = g[11] - g[12];
  const C p1314 = g[13] + g[14], m1314 = g[13] - g[14];
  const C zp = p78 + p910, zm = p1112 + p1314;  // z = +1 and z = -1 diagonals
  const C sd = zp + zm;
  const C Dx = (m78 + m910) + (m1112 + m1314);
  const C Dy = (p78 - p910) + (p1112 - p1314);
  const C Dz = zp - zm;
  const C Dxy = (m78 - m910) + (m1112 - m1314);
  const C Dyz = (p78 - p910) - (p1112 - p1314);
  const C Dzx = (m78 + m910) - (m1112 + m1314);
  const C Dxyz = (m78 - m910) - (m1112 - m1314);
  C dm[15];
  dm[0] = (g[0] + sa) + sd;
  dm[1] = dx + Dx;
  dm[2] = dy + Dy;
  dm[3] = dz + Dz;
  dm[4] = (sd - sa) - C(2) * g[0];
  dm[5] = fmaC(C(16), g[0], sd) - C(4) * sa;
  dm[6] = Dx - C(4) * dx;
  dm[7] = Dy - C(4) * dy;
  dm[8] = Dz - C(4) * dz;
  dm[9] = C(2) * ax - (ay + az);
  dm[10] = ay - az;
  dm[11] = Dxy;
  dm[12] = Dyz;
  dm[13] = Dzx;
  dm[14] = Dxyz;

  // ---- shifted conserved quantities
  C dr = dm[0], djx = dm[1], djy = dm[2], djz = dm[3];
  if (VAR != V_NONE && VAR != V_VISC) {
    const C nchi = p.n * chi, mchi = p.m * chi;
    const C inv_n = recip(C(1) + nchi);
    const C inv_m = p.n == p.m ? inv_n : recip(C(1) + mchi);
    dr = fmaC(nchi, p.dcf0, dm[0]) * inv_n;
    djx = fmaC(mchi, p.dcf1, dm[1]) * inv_m;
    djy = fmaC(mchi, p.dcf2, dm[2]) * inv_m;
    djz = fmaC(mchi, p.dcf3, dm[3]) * inv_m;
  }
  C meq[15];
  meq3_delta(dr, djx, djy, djz, p, meq);

  // ---- relaxation and damping
  C mp[15];
#pragma unroll
  for (int k = 0; k < 15; ++k) {
    C sk = p.s[k];
    if (VAR == V_VISC && k >= 4) sk = fmaC(C(1) - sk, chi, sk);
    mp[k] = fmaC(sk, meq[k] - dm[k], dm[k]);
  }
  if (VAR == V_I || VAR == V_II) {
#pragma unroll
    for (int k = 0; k < 15; ++k)
      mp[k] = fmaC(chi, mref[k] - (VAR == V_I ? dm[k] : meq[k]), mp[k]);
  } else if (VAR == V_III) {
    // e = L (dc^f - dc*), L c = (rho, j, -rho, rho, -7/3 j, 0, ...)
    const C a = p.dcf0 - dr, bx = p.dcf1 - djx, by = p.dcf2 - djy, bz = p.dcf3 - djz;
    mp[0] = fmaC(chi, a, mp[0]);
    mp[1] = fmaC(chi, bx, mp[1]);
    mp[2] = fmaC(chi, by, mp[2]);
    mp[3] = fmaC(chi, bz, mp[3]);
    mp[4] = fmaC(chi, -a, mp[4]);
    mp[5] = fmaC(chi, a, mp[5]);
    mp[6] = fmaC(chi, C(-7.0 / 3.0) * bx, mp[6]);
    mp[7] = fmaC(chi, C(-7.0 / 3.0) * by, mp[7]);
    mp[8] = fmaC(chi, C(-7.0 / 3.0) * bz, mp[8]);
  }

  // ---- g' = M^T D^-1 m'
  const C a0 = scale_conserved(mp[0], 1.0 / 15.0);
  const C a1 = scale_conserved(mp[1], 0.1), a2 = scale_conserved(mp[2], 0.1),
          a3 = scale_conserved(mp[3], 0.1);
  const C a4 = mp[4] * C(1.0 / 18.0), a5 = mp[5] * C(1.0 / 360.0);
  const C a6 = mp[6] * C(0.025), a7 = mp[7] * C(0.025), a8 = mp[8] * C(0.025);
  const C a9 = mp[9] * C(1.0 / 12.0), a10 = mp[10] * C(0.25);
  const C a11 = mp[11] * C(0.125), a12 = mp[12] * C(0.125), a13 = mp[13] * C(0.125),
          a14 = mp[14] * C(0.125);
  g[0] = fmaC(C(16), a5, a0 - C(2) * a4);
  const C A = (a0 - a4) - C(4) * a5;  // shared by the axis directions
  const C ex = a1 - C(4) * a6, ey = a2 - C(4) * a7, ez = a3 - C(4) * a8;
  const C bxx = A + C(2) * a9, byy = (A - a9) + a10, bzz = (A - a9) - a10;
  g[1] = bxx + ex;
  g[2] = bxx - ex;
  g[3] = byy + ey;
  g[4] = byy - ey;
  g[5] = bzz + ez;
  g[6] = bzz - ez;
  const C P = (a0 + a4) + a5;
  const C X = a1 + a6, Y = a2 + a7, Z = a3 + a8;
  const C T1 = P + Z, T2 = P - Z;  // z = +1 and z = -1 diagonals
  const C Xp = X + a13, Yp = Y + a12, Rp = a11 + a14;
  const C Xm = X - a13, Ym = Y - a12, Rm = a11 - a14;
  const C u1 = T1 + Rp, u2 = T1 - Rp, w1 = Xp + Yp, w2 = Xp - Yp;
  g[7] = u1 + w1;   // (+ + +)
  g[10] = u1 - w1;  // (- - +)
  g[9] = u2 + w2;   // (+ - +)
  g[8] = u2 - w2;   // (- + +)
  const C v1 = T2 + Rm, v2 = T2 - Rm, z1 = Xm + Ym, z2 = Xm - Ym;
  g[11] = v1 + z1;  // (+ + -)
  g[14] = v1 - z1;  // (- - -)
  g[13] = v2 + z2;  // (+ - -)
  g[12] = v2 - z2;  // (- + -)
}

template <typename C, int VAR>
__device__ __forceinline__ void collide3(C g[15], C chi, const CollideParams3<C> &p) {
  C mref[15];
  if (VAR == V_I || VAR == V_II) ref_moments3(p, mref);
  collide3<C, VAR>(g, chi, p, mref);
}

}  // namespace lbm
