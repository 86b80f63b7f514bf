// lbm_launch.h -- launch-side helpers shared by the kernel translation
// units of liblbm: the per-launch lattice description and the collision
// parameters in compute precision, both built from a StepConfig.
#pragma once

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

template <typename S>
struct Lat {
  typedef typename Store<S>::C C;
  int nx, ny;
  int64_t pitch, ps;
  C scale[9], inv_scale[9];
};

template <typename S>
inline Lat<S> make_lat(const StepConfig &c) {
  typedef typename Store<S>::C C;
  Lat<S> L;
  L.nx = c.nx;
  L.ny = c.ny;
  L.pitch = c.pitch;
  L.ps = c.plane_stride;
  for (int i = 0; i < 9; ++i) {
    const double sc = storage_scale(c, i);
    L.scale[i] = C(sc);
    L.inv_scale[i] = C(1.0 / sc);
  }
  return L;
}

template <typename C>
inline CollideParams<C> make_params(const StepConfig &c) {
  CollideParams<C> p;
  for (int k = 0; k < 9; ++k) p.s[k] = C(c.s[k]);
  p.n = C(c.n);
  p.m = C(c.m);
  p.rho_b = C(c.rho_b);
  p.ubx = C(c.ubx);
  p.uby = C(c.uby);
  p.dcf0 = C(c.dcf[0]);
  p.dcf1 = C(c.dcf[1]);
  p.dcf2 = C(c.dcf[2]);
  set_relax_coeffs(p);
  return p;
}

}  // namespace lbm
