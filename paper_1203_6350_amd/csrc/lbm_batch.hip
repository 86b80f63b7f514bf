// lbm_batch.hip -- one persistent launch per time step over many independent
// lattices of uneven size (Xu & Sagaut, arXiv:1203.6350: the same step as
// lbm_kernels.hip, per domain its own relaxation rates, damping variant,
// sponge and reference state).
//
// Work decomposition: the cells of every member domain, flattened row-major,
// are cut into tiles of TILE consecutive cells; the tile table lists
// (domain, first cell) pairs. A fixed grid of workgroups (a few per CU) walks
// the table with a static stride, so small and large domains share one launch
// and no workgroup is left with a partial row of a 64-cell domain. The tile
// count and the per-domain descriptors live in device memory: a captured
// graph of launches stays valid while the host rewrites them between
// replays. Each domain carries its own parity (which of its two lattices is
// current) and the number of steps it takes in the current tick; launch k of
// a tick advances the domains with k < stop_at. When the tick's bulk runs as
// launches of kmulti steps each (the strip kernel), these launches take the
// remainder: a domain has taken stop_at / kmulti multi-step launches and
// launch k advances it if k < stop_at mod kmulti.
//
// The per-cell arithmetic is the collide() of lbm_device.h, so a domain
// stepped here is bit-identical to the same domain stepped alone.
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

template <typename S, int BX>
__global__ __launch_bounds__(BX) void batch_step_kernel(
    const BatchDomain *__restrict__ doms, const int2 *__restrict__ tiles,
    const int *__restrict__ ntiles_dev, int k, int kmulti) {
  typedef typename Store<S>::C C;
  const int nt = *ntiles_dev;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const int2 tile = tiles[t];
    const BatchDomain &d = doms[tile.x];
    const int done = kmulti > 0 ? d.stop_at / kmulti : 0;  // multi-step launches taken
    if (k >= d.stop_at - done * kmulti) continue;
    const int nx = d.nx, ny = d.ny;
    const int c = tile.y + threadIdx.x;
    if (c >= nx * ny) continue;
    const int y = c / nx, x = c - y * nx;
    const int par = (d.parity + done + k) & 1;
    const S *__restrict__ src = (const S *)d.lat[par];
    S *__restrict__ dst = (S *)d.lat[par ^ 1];
    const int xm = x == 0 ? nx - 1 : x - 1;
    const int xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1;
    const int yp = y == ny - 1 ? 0 : y + 1;
    const int64_t r0 = (int64_t)y * d.pitch, rm = (int64_t)ym * d.pitch,
                  rp = (int64_t)yp * d.pitch;
    const int64_t ps = d.ps;
    C scale[9], inv_scale[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      scale[i] = C(d.scale[i]);
      inv_scale[i] = C(d.inv_scale[i]);
    }
    C g[9];
    g[0] = Store<S>::load(src + 0 * ps + r0 + x, scale[0]);
    g[1] = Store<S>::load(src + 1 * ps + r0 + xm, scale[1]);
    g[2] = Store<S>::load(src + 2 * ps + rm + x, scale[2]);
    g[3] = Store<S>::load(src + 3 * ps + r0 + xp, scale[3]);
    g[4] = Store<S>::load(src + 4 * ps + rp + x, scale[4]);
    g[5] = Store<S>::load(src + 5 * ps + rm + xm, scale[5]);
    g[6] = Store<S>::load(src + 6 * ps + rm + xp, scale[6]);
    g[7] = Store<S>::load(src + 7 * ps + rp + xp, scale[7]);
    g[8] = Store<S>::load(src + 8 * ps + rp + xm, scale[8]);
    C chi = C(0);
    switch (d.chi_mode) {
      case CHI_FIELD: chi = chi_at<C, CHI_FIELD>((const C *)d.chi_field, nullptr, nullptr, r0 + x, x, y); break;
      case CHI_SEP_MAX: chi = chi_at<C, CHI_SEP_MAX>(nullptr, (const C *)d.chi_x, (const C *)d.chi_y, 0, x, y); break;
      case CHI_SEP_SUM: chi = chi_at<C, CHI_SEP_SUM>(nullptr, (const C *)d.chi_x, (const C *)d.chi_y, 0, x, y); break;
      default: break;
    }
    CollideParams<C> p;
#pragma unroll
    for (int i = 0; i < 9; ++i) p.s[i] = C(d.s[i]);
    p.n = C(d.n);
    p.m = C(d.m);
    p.rho_b = C(d.rho_b);
    p.ubx = C(d.ubx);
    p.uby = C(d.uby);
    p.dcf0 = C(d.dcf[0]);
    p.dcf1 = C(d.dcf[1]);
    p.dcf2 = C(d.dcf[2]);
    if (d.qf) {  // the cell's own reference state (damped variants only)
      const C *q = (const C *)d.qf;
      const int64_t cell = r0 + x;
      p.dcf0 = q[cell];
      p.dcf1 = q[d.qps + cell];
      p.dcf2 = q[2 * d.qps + cell];
    }
    set_relax_coeffs(p);
    switch (d.variant) {
      case V_I: collide<C, V_I>(g, chi, p); break;
      case V_II: collide<C, V_II>(g, chi, p); break;
      case V_III: collide<C, V_III>(g, chi, p); break;
      case V_VISC: collide<C, V_VISC>(g, chi, p); break;
      default: collide<C, V_NONE>(g, chi, p); break;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) Store<S>::store(dst + i * ps + r0 + x, g[i], inv_scale[i]);
  }
}

template <typename S>
static hipError_t launch_batch_t(const BatchDomain *doms, const int2 *tiles,
                                 const int *ntiles_dev, int grid, int k, int kmulti,
                                 hipStream_t stream) {
  batch_step_kernel<S, BATCH_TILE><<<dim3(grid), dim3(BATCH_TILE), 0, stream>>>(
      doms, tiles, ntiles_dev, k, kmulti);
  return hipGetLastError();
}

hipError_t launch_batch(int storage, const BatchDomain *doms, const int2 *tiles,
                        const int *ntiles_dev, int grid, int k, int kmulti,
                        hipStream_t stream) {
  switch (storage) {
    case 0: return launch_batch_t<double>(doms, tiles, ntiles_dev, grid, k, kmulti, stream);
    case 1: return launch_batch_t<float>(doms, tiles, ntiles_dev, grid, k, kmulti, stream);
    case 2: return launch_batch_t<__half>(doms, tiles, ntiles_dev, grid, k, kmulti, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_multi(int storage, int k, int nw, int form, const BatchDomain *doms,
                              const int4 *items, int *nitems, int grid, int j,
                              hipStream_t stream) {
#define LBM_BMULTI_K(ST)                                                                      \
  switch (k) {                                                                                \
    case 2: return launch_batch_multi_##ST##_k2(nw, form, doms, items, nitems, grid, j, stream); \
    case 3: return launch_batch_multi_##ST##_k3(nw, form, doms, items, nitems, grid, j, stream); \
    case 4: return launch_batch_multi_##ST##_k4(nw, form, doms, items, nitems, grid, j, stream); \
  }                                                                                           \
  return hipErrorInvalidValue;
  switch (storage) {
    case 0: { LBM_BMULTI_K(f64) }
    case 1: { LBM_BMULTI_K(f32) }
    case 2: { LBM_BMULTI_K(f16) }
  }
#undef LBM_BMULTI_K
  return hipErrorInvalidValue;
}

int batch_multi_per_cu(int storage, int k, int nw, int form) {
#define LBM_BPERCU_K(ST)                                        \
  switch (k) {                                                  \
    case 2: return batch_multi_per_cu_##ST##_k2(nw, form);       \
    case 3: return batch_multi_per_cu_##ST##_k3(nw, form);       \
    case 4: return batch_multi_per_cu_##ST##_k4(nw, form);       \
  }                                                             \
  return 0;
  switch (storage) {
    case 0: { LBM_BPERCU_K(f64) }
    case 1: { LBM_BPERCU_K(f32) }
    case 2: { LBM_BPERCU_K(f16) }
  }
#undef LBM_BPERCU_K
  return 0;
}

}  // namespace lbm
