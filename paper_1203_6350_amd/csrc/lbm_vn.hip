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
// Each thread's matrix lives in LDS, laid out [element][thread] (16-byte
// complex pairs) so that the lanes touch consecutive pairs. The solve is
// bound by LDS latency with few waves resident (1.3 KB of LDS per
// wavenumber), so workgroups are 16 threads: more of them fit on a CU
// (measured: 16 threads 56, 32 threads 54, 64 threads 40 M wavenumbers/s).
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

// Matrix element (i, j) of this thread; NT threads share the block's LDS,
// one 16-byte (re, im) pair per element.
template <int NT>
struct Mat {
  double2 *a;
  int t;
  __device__ __forceinline__ cplx get(int i, int j) const {
    const double2 v = a[(i * N + j) * NT + t];
    return mk(v.x, v.y);
  }
  __device__ __forceinline__ void set(int i, int j, cplx v) const {
    a[(i * N + j) * NT + t] = make_double2(v.re, v.im);
  }
};

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

template <int NT>
__device__ void hessenberg(const Mat<NT> &H) {
  for (int k = 0; k < N - 2; ++k) {
    double xn2 = 0.0;
    for (int i = k + 1; i < N; ++i) {
      const cplx v = H.get(i, k);
      xn2 += v.re * v.re + v.im * v.im;
    }
    const double xn = sqrt(xn2);
    const cplx x0 = H.get(k + 1, k);
    double tail = 0.0;
    for (int i = k + 2; i < N; ++i) tail += abs1(H.get(i, k));
    if (tail == 0.0) continue;  // already reduced in this column
    const double ax0 = absc(x0);
    const cplx ph = ax0 > 0.0 ? scal(1.0 / ax0, x0) : mk(1.0, 0.0);
    const cplx alpha = scal(-xn, ph);  // -e^{i arg x0} ||x||
    // v = x - alpha e1, normalised
    cplx v[N];
    double vn2 = 0.0;
    for (int i = k + 1; i < N; ++i) {
      cplx vi = H.get(i, k);
      if (i == k + 1) vi = sub(vi, alpha);
      v[i] = vi;
      vn2 += vi.re * vi.re + vi.im * vi.im;
    }
    const double inv = 1.0 / sqrt(vn2);
    for (int i = k + 1; i < N; ++i) v[i] = scal(inv, v[i]);
    // left: H <- (I - 2 v v^H) H on rows k+1.., columns k+1..
    for (int j = k + 1; j < N; ++j) {
      cplx w = mk(0.0, 0.0);
      for (int i = k + 1; i < N; ++i) w = add(w, mul(conjc(v[i]), H.get(i, j)));
      for (int i = k + 1; i < N; ++i) H.set(i, j, sub(H.get(i, j), scal(2.0, mul(v[i], w))));
    }
    H.set(k + 1, k, alpha);
    for (int i = k + 2; i < N; ++i) H.set(i, k, mk(0.0, 0.0));
    // right: H <- H (I - 2 v v^H) on all rows, columns k+1..
    for (int i = 0; i < N; ++i) {
      cplx w = mk(0.0, 0.0);
      for (int j = k + 1; j < N; ++j) w = add(w, mul(H.get(i, j), v[j]));
      for (int j = k + 1; j < N; ++j)
        H.set(i, j, sub(H.get(i, j), scal(2.0, mul(w, conjc(v[j])))));
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

template <int NT>
__device__ bool hqr(const Mat<NT> &H, cplx *ev) {
  const double eps = 2.220446049250313e-16;
  int hi = N - 1, iter = 0, total = 0;
  while (hi >= 0) {
    if (hi == 0) {
      ev[0] = H.get(0, 0);
      break;
    }
    int l = hi;
    for (; l > 0; --l) {
      const double tst = abs1(H.get(l - 1, l - 1)) + abs1(H.get(l, l));
      if (abs1(H.get(l, l - 1)) <= eps * tst) {
        H.set(l, l - 1, mk(0.0, 0.0));
        break;
      }
    }
    if (l == hi) {
      ev[hi] = H.get(hi, hi);
      --hi;
      iter = 0;
      continue;
    }
    if (l == hi - 1) {
      eig2(H.get(hi - 1, hi - 1), H.get(hi - 1, hi), H.get(hi, hi - 1), H.get(hi, hi),
           ev[hi - 1], ev[hi]);
      hi -= 2;
      iter = 0;
      continue;
    }
    if (++total > 40 * N) return false;
    cplx mu;
    if (iter == 10 || iter == 20) {
      // exceptional shift
      mu = add(H.get(hi, hi), mk(0.75 * fabs(H.get(hi, hi - 1).re) + fabs(H.get(hi - 1, hi - 2).re), 0.0));
    } else {
      cplx l1, l2;
      eig2(H.get(hi - 1, hi - 1), H.get(hi - 1, hi), H.get(hi, hi - 1), H.get(hi, hi), l1, l2);
      const cplx hh = H.get(hi, hi);
      mu = abs1(sub(l1, hh)) <= abs1(sub(l2, hh)) ? l1 : l2;  // Wilkinson
    }
    ++iter;
    // QR sweep of the active block l..hi: H - mu I = Q R, H <- R Q + mu I
    for (int k = l; k <= hi; ++k) H.set(k, k, sub(H.get(k, k), mu));
    double cs[N];
    cplx sn[N];
    for (int k = l; k < hi; ++k) {
      const cplx x = H.get(k, k), y = H.get(k + 1, k);
      const double ax = absc(x), r = hypot(ax, absc(y));
      double c;
      cplx s;
      if (r == 0.0) {
        c = 1.0;
        s = mk(0.0, 0.0);
      } else if (ax == 0.0) {
        c = 0.0;
        s = scal(1.0 / absc(y), conjc(y));
      } else {
        c = ax / r;
        s = scal(1.0 / (ax * r), mul(x, conjc(y)));
      }
      cs[k] = c;
      sn[k] = s;
      for (int j = k; j <= hi; ++j) {
        const cplx t1 = H.get(k, j), t2 = H.get(k + 1, j);
        H.set(k, j, add(scal(c, t1), mul(s, t2)));
        H.set(k + 1, j, sub(scal(c, t2), mul(conjc(s), t1)));
      }
    }
    for (int k = l; k < hi; ++k) {
      const double c = cs[k];
      const cplx s = sn[k];
      for (int i = l; i <= k + 1; ++i) {
        const cplx t1 = H.get(i, k), t2 = H.get(i, k + 1);
        H.set(i, k, add(scal(c, t1), mul(t2, conjc(s))));
        H.set(i, k + 1, sub(scal(c, t2), mul(t1, s)));
      }
    }
    for (int k = l; k <= hi; ++k) H.set(k, k, add(H.get(k, k), mu));
  }
  return true;
}

__device__ __forceinline__ bool before(cplx a, cplx b) {
  const double ma = absc(a), mb = absc(b);
  if (ma != mb) return ma > mb;
  return atan2(a.im, a.re) < atan2(b.im, b.re);
}

}  // namespace

template <int NT>
__global__ __launch_bounds__(NT) void vn_kernel(const VnParamsDev *__restrict__ params,
                                                int64_t nk,
                                                const double *__restrict__ kx,
                                                const double *__restrict__ ky,
                                                double *__restrict__ eig,
                                                double *__restrict__ G) {
  extern __shared__ double smem[];
  double *Are = smem;                  // 81: A = M^-1 A_m M
  double *Am = smem + 81;              // 81
  double2 *Hm = (double2 *)(smem + 162);  // 81 * NT (re, im) pairs
  const int pset = blockIdx.y;
  const VnParamsDev p = params[pset];
  const int t = threadIdx.x;
  if (t == 0) build_Am(p, Am);
  __syncthreads();
  for (int e = t; e < 81; e += NT) {
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
  const int64_t kidx = (int64_t)blockIdx.x * NT + t;
  if (kidx >= nk) return;
  const double k1 = kx[kidx], k2 = ky[kidx];
  Mat<NT> H{Hm, t};
  for (int i = 0; i < 9; ++i) {
    const double ph = -(k1 * cx_of(i) + k2 * cy_of(i));
    double sp, cp;
    sincos(ph, &sp, &cp);
    for (int j = 0; j < 9; ++j) {
      const double a = Are[i * 9 + j];
      H.set(i, j, mk(cp * a, sp * a));
    }
  }
  const int64_t out = (int64_t)pset * nk + kidx;
  if (G) {
    for (int e = 0; e < 81; ++e) {
      const cplx v = H.get(e / 9, e % 9);
      G[(out * 81 + e) * 2] = v.re;
      G[(out * 81 + e) * 2 + 1] = v.im;
    }
  }
  hessenberg(H);
  cplx ev[N];
  const bool ok = hqr(H, ev);
  if (!ok)
    for (int i = 0; i < N; ++i) ev[i] = mk(__builtin_nan(""), __builtin_nan(""));
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

template <int NT>
static hipError_t launch_vn_t(const VnParamsDev *params_dev, int nparams, int64_t nk,
                              const double *kx, const double *ky, double *eig,
                              double *G, hipStream_t stream) {
  const size_t shmem = sizeof(double) * (162 + 2 * 81 * NT);
  const int64_t bx = (nk + NT - 1) / NT;
  if (bx > 0x7fffffff) return hipErrorInvalidValue;
  vn_kernel<NT><<<dim3((unsigned)bx, (unsigned)nparams), dim3(NT), shmem, stream>>>(
      params_dev, nk, kx, ky, eig, G);
  return hipGetLastError();
}

hipError_t launch_vn(const VnParamsDev *params_dev, int nparams, int64_t nk,
                     const double *kx, const double *ky, double *eig, double *G,
                     hipStream_t stream) {
  return launch_vn_t<16>(params_dev, nparams, nk, kx, ky, eig, G, stream);
}

}  // namespace lbm
