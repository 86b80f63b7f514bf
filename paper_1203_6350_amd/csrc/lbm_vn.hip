// lbm_vn.hip -- batched Von Neumann analysis of the linearised scheme with
// the absorbing term (Xu & Sagaut, arXiv:1203.6350, Section 3.2, eqs.
// eq:linearized, perturb-w-f, sec:matrix), FP64 on gfx950.
//
// For each parameter set the block first forms the real 9x9 Jacobian of the
// collision at f^eq(q_ref) in moment space,
//   A_m = I + S (J D P - I) - chi X,
// (P: picks rho, jx, jy; D = diag(1/(1+n chi), 1/(1+m chi), 1/(1+m chi)) is
// the derivative of the shifted rho*, j*; J = d m^eq/d(rho, j) at q_ref;
// X = I for Type I, J D P for Type II, L D P for Type III with
// L = d m^L/d(rho, j); X = 0 and D = I without damping), then
// A = M^-1 A_m M. Each thread takes one wavenumber k and
//   G(k) = diag(exp(-i k.c_j)) A
// (the streaming phase, pull form), reduces G to upper Hessenberg form with
// complex Householder reflections and finds its eigenvalues with single-shift
// complex QR (Wilkinson shifts, deflation on negligible subdiagonals,
// exceptional shifts after 10 and 20 stalled sweeps). Eigenvalues are
// returned sorted by (-|lambda|, arg lambda).
//
// Each lane holds its wavenumber's matrix in registers (81 complex values,
// every index fixed at compile time: the loops are fully unrolled), so the
// solve runs from the register file at the VALU rate. The QR sweeps are
// wave-wide: every lane runs the same instruction stream over the full
// 9 x 9 matrix, and a lane's own state (the bottom row of its active window,
// its shift, its stall counter) enters only through predicates: rotations
// outside its window are the identity. A wave ends when all its lanes have
// converged.
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx mk(double r, double i) { return cplx{r, i}; }
__device__ __forceinline__ cplx add(cplx a, cplx b) { return mk(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ cplx sub(cplx a, cplx b) { return mk(a.re - b.re, a.im - b.im); }
__device__ __forceinline__ cplx mul(cplx a, cplx b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__device__ __forceinline__ cplx conjc(cplx a) { return mk(a.re, -a.im); }
__device__ __forceinline__ cplx scal(double s, cplx a) { return mk(s * a.re, s * a.im); }
__device__ __forceinline__ double abs1(cplx a) { return fabs(a.re) + fabs(a.im); }
__device__ __forceinline__ double absc(cplx a) { return hypot(a.re, a.im); }
__device__ __forceinline__ cplx divc(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return mk((a.re + a.im * r) / d, (a.im - a.re * r) / d);
  }
  const double r = b.re / b.im, d = b.re * r + b.im;
  return mk((a.re * r + a.im) / d, (a.im * r - a.re) / d);
}
__device__ __forceinline__ cplx sqrtc(cplx z) {
  const double r = absc(z);
  if (r == 0.0) return mk(0.0, 0.0);
  if (z.re >= 0.0) {
    const double t = sqrt(0.5 * (r + z.re));
    return mk(t, z.im / (2.0 * t));
  }
  const double t = sqrt(0.5 * (r - z.re));
  return mk(fabs(z.im) / (2.0 * t), copysign(t, z.im));
}

constexpr int N = 9;

// The D2Q9 transform of Appendix A.1, row-major; rows (rho, jx, jy, e, eps,
// qx, qy, pxx, pxy).
__constant__ double kM[81] = {
     1,  1,  1,  1,  1, 1,  1,  1,  1,
     0,  1,  0, -1,  0, 1, -1, -1,  1,
     0,  0,  1,  0, -1, 1,  1, -1, -1,
    -4, -1, -1, -1, -1, 2,  2,  2,  2,
     4, -2, -2, -2, -2, 1,  1,  1,  1,
     0, -2,  0,  2,  0, 1, -1, -1,  1,
     0,  0, -2,  0,  2, 1,  1, -1, -1,
     0,  1, -1,  1, -1, 0,  0,  0,  0,
     0,  0,  0,  0,  0, 1, -1,  1, -1};
// Squared row norms (M M^T)_kk; the rows are orthogonal, so
// (M^-1)_{ik} = M_{ki} / (M M^T)_kk.
__constant__ double kMnorm[9] = {9, 6, 6, 36, 36, 12, 12, 4, 4};

// Moment-space Jacobian A_m (row-major 81) for one parameter set.
__device__ void build_Am(const VnParamsDev &p, double *Am) {
  const double chi = p.variant == V_NONE ? 0.0 : p.chi;
  const double ux = p.ux_f, uy = p.uy_f, u2 = ux * ux + uy * uy;
  const double J[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                          {-2.0 - 3.0 * u2, 6.0 * ux, 6.0 * uy},
                          {1.0 + 3.0 * u2, -6.0 * ux, -6.0 * uy},
                          {0, -1, 0}, {0, 0, -1},
                          {-(ux * ux - uy * uy), 2.0 * ux, -2.0 * uy},
                          {-ux * uy, uy, ux}};
  const double L[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {-2, 0, 0}, {1, 0, 0},
                          {0, -1, 0}, {0, 0, -1}, {0, 0, 0}, {0, 0, 0}};
  const double D[3] = {1.0 / (1.0 + p.n * chi), 1.0 / (1.0 + p.m * chi),
                       1.0 / (1.0 + p.m * chi)};
  for (int k = 0; k < 9; ++k) {
    for (int l = 0; l < 9; ++l) {
      const double JDP = l < 3 ? J[k][l] * D[l] : 0.0;
      const double LDP = l < 3 ? L[k][l] * D[l] : 0.0;
      const double id = k == l ? 1.0 : 0.0;
      double X = 0.0;
      if (p.variant == V_I) X = id;
      else if (p.variant == V_II) X = JDP;
      else if (p.variant == V_III) X = LDP;
      Am[k * 9 + l] = id + p.s[k] * (JDP - id) - chi * X;
    }
  }
}

// Eigenvalues of the 2x2 block [a b; c d].
__device__ void eig2(cplx a, cplx b, cplx c, cplx d, cplx &l1, cplx &l2) {
  const cplx p = scal(0.5, sub(a, d));
  const cplx bc = mul(b, c);
  cplx y = sqrtc(add(mul(p, p), bc));
  if (p.re * y.re + p.im * y.im < 0.0) y = scal(-1.0, y);
  const cplx z1 = add(p, y);
  if (abs1(z1) == 0.0) {
    l1 = d;
    l2 = d;
    return;
  }
  l1 = add(d, z1);
  l2 = sub(d, divc(bc, z1));
}

__device__ __forceinline__ bool before(cplx a, cplx b) {
  const double ma = absc(a), mb = absc(b);
  if (ma != mb) return ma > mb;
  return atan2(a.im, a.re) < atan2(b.im, b.re);
}

}  // namespace

// 1/sqrt(x) for x > 0 to about one ulp: the hardware estimate refined by
// two Newton steps (each doubles the correct bits).
__device__ __forceinline__ double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * __builtin_fma(-hx * y, y, 1.5);
  y = y * __builtin_fma(-hx * y, y, 1.5);
  return y;
}

// One lane's matrix: H = R + i I, row-major, static indices only.
struct RegMat {
  double r[N][N], m[N][N];
  __device__ __forceinline__ cplx at(int i, int j) const { return mk(r[i][j], m[i][j]); }
  __device__ __forceinline__ void put(int i, int j, cplx v) {
    r[i][j] = v.re;
    m[i][j] = v.im;
  }
};

// Element (i, j) of the tridiagonal band (|i - j| <= 1) at the lane's own
// (run-time) indices, read by selecting over the static positions.
__device__ __forceinline__ cplx pick(const RegMat &H, int i, int j) {
  cplx v = mk(0.0, 0.0);
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = 0; b < N; ++b)
      if (b >= a - 1 && b <= a + 1) {  // the sub-, main and superdiagonal are all we read
        const bool hit = a == i && b == j;
        v.re = hit ? H.r[a][b] : v.re;
        v.im = hit ? H.m[a][b] : v.im;
      }
  return v;
}

// Householder reduction to upper Hessenberg form, H <- Q^H H Q.
__device__ __forceinline__ void hessenberg_reg(RegMat &H) {
#pragma unroll
  for (int k = 0; k < N - 2; ++k) {
    double xn2 = 0.0;
#pragma unroll
    for (int i = k + 1; i < N; ++i) xn2 += H.r[i][k] * H.r[i][k] + H.m[i][k] * H.m[i][k];
    const double xn = sqrt(xn2);
    const cplx x0 = H.at(k + 1, k);
    const double ax0 = absc(x0);
    const cplx ph = ax0 > 0.0 ? scal(1.0 / ax0, x0) : mk(1.0, 0.0);
    const cplx alpha = scal(-xn, ph);  // -e^{i arg x0} ||x||
    // v = x - alpha e1, normalised (v = 0, the identity, for a zero column)
    cplx v[N];
    double vn2 = 0.0;
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      v[i] = i == k + 1 ? sub(x0, alpha) : H.at(i, k);
      vn2 += v[i].re * v[i].re + v[i].im * v[i].im;
    }
    const double inv = vn2 > 0.0 ? rsqrt_f64(vn2) : 0.0;
#pragma unroll
    for (int i = k + 1; i < N; ++i) v[i] = scal(inv, v[i]);
    // left: rows k+1.., columns k+1..
#pragma unroll
    for (int j = k + 1; j < N; ++j) {
      cplx w = mk(0.0, 0.0);
#pragma unroll
      for (int i = k + 1; i < N; ++i) w = add(w, mul(conjc(v[i]), H.at(i, j)));
      w = scal(2.0, w);
#pragma unroll
      for (int i = k + 1; i < N; ++i) H.put(i, j, sub(H.at(i, j), mul(v[i], w)));
    }
    // column k below the subdiagonal: the reflection maps x to alpha e1
    // (with v = 0 the column was zero below x0 already); the entries below
    // the subdiagonal become compile-time zeros, which frees their registers
    // for the QR sweeps (they never read them)
    H.put(k + 1, k, vn2 > 0.0 ? alpha : x0);
#pragma unroll
    for (int i = k + 2; i < N; ++i) H.put(i, k, mk(0.0, 0.0));
    // right: all rows, columns k+1..
#pragma unroll
    for (int i = 0; i < N; ++i) {
      cplx w = mk(0.0, 0.0);
#pragma unroll
      for (int j = k + 1; j < N; ++j) w = add(w, mul(H.at(i, j), v[j]));
      w = scal(2.0, w);
#pragma unroll
      for (int j = k + 1; j < N; ++j) H.put(i, j, sub(H.at(i, j), mul(w, conjc(v[j]))));
    }
  }
}

// Rotation [c s; -conj(s) conj(c)] with c = conj(x)/r, s = conj(y)/r,
// r = sqrt(|x|^2 + |y|^2), which maps (x, y) to (r, 0); the identity when
// inactive or when x = y = 0.
__device__ __forceinline__ void givens(cplx x, cplx y, bool act, cplx &c, cplx &s) {
  const double n2 = x.re * x.re + x.im * x.im + y.re * y.re + y.im * y.im;
  const bool on = act && n2 > 0.0;
  const double ir = on ? rsqrt_f64(n2) : 0.0;
  c = on ? mk(x.re * ir, -x.im * ir) : mk(1.0, 0.0);
  s = on ? mk(y.re * ir, -y.im * ir) : mk(0.0, 0.0);
}

// H <- H G^H on columns q, q + 1 for rows 0..rmax, G = [c s; -conj(s) conj(c)].
__device__ __forceinline__ void right_rot(RegMat &H, int q, int rmax, cplx c, cplx s) {
#pragma unroll
  for (int i = 0; i <= rmax; ++i) {
    const cplx t1 = H.at(i, q), t2 = H.at(i, q + 1);
    H.put(i, q, add(mul(t1, conjc(c)), mul(t2, conjc(s))));
    H.put(i, q + 1, sub(mul(t2, c), mul(t1, s)));
  }
}

constexpr int VN_MAX_SWEEPS = 40 * N;

// Eigenvalues of the upper Hessenberg H by single-shift QR sweeps on the
// lane's active window 0..hi (Wilkinson shift from its trailing 2 x 2,
// exceptional shifts after 10 and 20 stalled sweeps; the bottom eigenvalue
// deflates when its subdiagonal is negligible). Returns false if the lane
// did not converge within VN_MAX_SWEEPS sweeps.
__device__ __forceinline__ bool qr_reg(RegMat &H, double2 *ev, int stride) {
  const double eps = 2.220446049250313e-16;
  int hi = N - 1, it = 0;
  bool done = false;
  for (int sweep = 0; sweep < VN_MAX_SWEEPS; ++sweep) {
    // deflate converged eigenvalues at the bottom (two checks per sweep)
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
      if (!done) {
        if (hi <= 0) {
          ev[0] = make_double2(H.r[0][0], H.m[0][0]);
          done = true;
        } else {
          const cplx d = pick(H, hi, hi - 1);
          const cplx a = pick(H, hi - 1, hi - 1), b = pick(H, hi, hi);
          if (abs1(d) <= eps * (abs1(a) + abs1(b))) {
            ev[hi * stride] = make_double2(b.re, b.im);
            --hi;
            it = 0;
          } else if (hi == 1) {
            cplx l0, l1;
            eig2(a, pick(H, 0, 1), d, b, l0, l1);
            ev[0] = make_double2(l0.re, l0.im);
            ev[stride] = make_double2(l1.re, l1.im);
            done = true;
          }
        }
      }
    }
    if (__all(done)) break;
    // shift of the active window
    cplx mu = mk(0.0, 0.0);
    if (!done) {
      const cplx a = pick(H, hi - 1, hi - 1), b = pick(H, hi - 1, hi);
      const cplx c = pick(H, hi, hi - 1), d = pick(H, hi, hi);
      if (it == 10 || it == 20) {
        const double e2 = hi >= 2 ? fabs(pick(H, hi - 1, hi - 2).re) : 0.0;
        mu = add(d, mk(0.75 * fabs(c.re) + e2, 0.0));
      } else {
        cplx l1, l2;
        eig2(a, b, c, d, l1, l2);
        mu = abs1(sub(l1, d)) <= abs1(sub(l2, d)) ? l1 : l2;
      }
      ++it;
    }
    // H - mu I on the window
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const bool in = !done && i <= hi;
      H.r[i][i] -= in ? mu.re : 0.0;
      H.m[i][i] -= in ? mu.im : 0.0;
    }
    // R = G_{hi-1} ... G_0 (H - mu I), then R G_0^H ... G_{hi-1}^H, with
    // each right rotation applied once the next left one is: the left
    // rotation k reads H(k, k) before the right rotation k - 1 changes it.
    // Rotations that no lane of the wave needs (k >= hi in every lane) are
    // skipped as a whole; a pending right rotation is applied first.
    cplx cp = mk(1.0, 0.0), sp = mk(0.0, 0.0);
    bool pend = false;
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
      if (__any(!done && k < hi)) {
        cplx c, s;
        givens(H.at(k, k), H.at(k + 1, k), !done && k < hi, c, s);
#pragma unroll
        for (int j = k; j < N; ++j) {
          const cplx t1 = H.at(k, j), t2 = H.at(k + 1, j);
          H.put(k, j, add(mul(c, t1), mul(s, t2)));
          H.put(k + 1, j, sub(mul(conjc(c), t2), mul(conjc(s), t1)));
        }
        if (k > 0) right_rot(H, k - 1, k, cp, sp);
        cp = c;
        sp = s;
        pend = true;
      } else if (pend) {
        right_rot(H, k - 1, k, cp, sp);
        pend = false;
      }
    }
    if (pend) right_rot(H, N - 2, N - 1, cp, sp);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const bool in = !done && i <= hi;
      H.r[i][i] += in ? mu.re : 0.0;
      H.m[i][i] += in ? mu.im : 0.0;
    }
  }
  return done;
}

// One wavenumber per lane, 64 lanes per workgroup (one wave); blockIdx.y
// is the parameter set.
__global__ __launch_bounds__(64) void vn_kernel(const VnParamsDev *__restrict__ params,
                                                int64_t nk,
                                                const double *__restrict__ kx,
                                                const double *__restrict__ ky,
                                                double *__restrict__ eig,
                                                double *__restrict__ G) {
  __shared__ double Are[81];  // A = M^-1 A_m M
  __shared__ double Am[81];
  __shared__ double2 evs[N * 64];  // eigenvalues as they deflate, [index][lane]
  const int pset = blockIdx.y;
  const int t = threadIdx.x;
  if (t == 0) build_Am(params[pset], Am);
  __syncthreads();
  for (int e = t; e < 81; e += 64) {
    const int i = e / 9, j = e % 9;
    double acc = 0.0;
    for (int k = 0; k < 9; ++k) {
      double inner = 0.0;
      for (int l = 0; l < 9; ++l) inner += Am[k * 9 + l] * kM[l * 9 + j];
      acc += kM[k * 9 + i] / kMnorm[k] * inner;
    }
    Are[e] = acc;
  }
  __syncthreads();
  const int64_t kidx = (int64_t)blockIdx.x * 64 + t;
  // lanes past the end solve a copy of the last wavenumber and store nothing,
  // so that every lane of the wave runs the same sweeps
  const int64_t kk = kidx < nk ? kidx : nk - 1;
  const double k1 = kx[kk], k2 = ky[kk];
  RegMat H;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double ph = -(k1 * cx_of(i) + k2 * cy_of(i));
    double sp, cp;
    sincos(ph, &sp, &cp);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const double a = Are[i * 9 + j];
      H.r[i][j] = cp * a;
      H.m[i][j] = sp * a;
    }
  }
  const int64_t out = (int64_t)pset * nk + kidx;
  if (G && kidx < nk) {
#pragma unroll
    for (int e = 0; e < 81; ++e) {
      G[(out * 81 + e) * 2] = H.r[e / 9][e % 9];
      G[(out * 81 + e) * 2 + 1] = H.m[e / 9][e % 9];
    }
  }
  hessenberg_reg(H);
  const bool ok = qr_reg(H, evs + t, 64);
  if (kidx >= nk) return;
  cplx ev[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double2 v = evs[i * 64 + t];
    ev[i] = ok ? mk(v.x, v.y) : mk(__builtin_nan(""), __builtin_nan(""));
  }
  // insertion sort by (-|lambda|, arg lambda)
  for (int i = 1; i < N; ++i) {
    const cplx v = ev[i];
    int j = i - 1;
    while (j >= 0 && before(v, ev[j])) {
      ev[j + 1] = ev[j];
      --j;
    }
    ev[j + 1] = v;
  }
  for (int i = 0; i < N; ++i) {
    eig[(out * 9 + i) * 2] = ev[i].re;
    eig[(out * 9 + i) * 2 + 1] = ev[i].im;
  }
}

hipError_t launch_vn(const VnParamsDev *params_dev, int nparams, int64_t nk,
                     const double *kx, const double *ky, double *eig, double *G,
                     hipStream_t stream) {
  if (nk < 1) return hipSuccess;
  const int64_t bx = (nk + 63) / 64;
  if (bx > 0x7fffffff) return hipErrorInvalidValue;
  vn_kernel<<<dim3((unsigned)bx, (unsigned)nparams), dim3(64), 0, stream>>>(
      params_dev, nk, kx, ky, eig, G);
  return hipGetLastError();
}

}  // namespace lbm
