// lbm_strip.h -- the multi-step strip kernel of liblbm (Xu & Sagaut,
// arXiv:1203.6350: K applications of the step of Section 2 per launch) and
// its launcher. Instantiated once per storage type, in lbm_strip_f64.hip,
// lbm_strip_f32.hip and lbm_strip_f16.hip.
#pragma once

#include <atomic>
#include <type_traits>

#include "lbm_device.h"
#include "lbm_internal.h"
#include "lbm_launch.h"

namespace lbm {

// ---------------------------------------------------------------- several steps per launch
// Temporal blocking: one launch advances the lattice by K = 2, 3 or 4 time
// steps, reading and writing it once.
//
// Each wave owns a strip of STRIP = 64 - 2K output columns of one chunk of
// rows: lane l holds column X0 - K + l (mod nx), so the 64 lanes cover the
// strip plus K halo columns on each side. The wave marches down the rows.
// When row a of the input lattice arrives, the lanes compute step 1 at row
// a - 1, step 2 at row a - 2, ..., step K at row a - K, each from the rows
// the step before produced. Pulls along x come from the neighbouring lanes
// (DPP wave shifts); pulls along y from registers carried over rows. A row's
// populations are consumed in three groups, each by one step at one row:
// {4, 7, 8} (c_y = -1) at the row above, {0, 1, 3} (c_y = 0) at the row
// itself, {2, 5, 6} (c_y = +1) at the row below. After step j a lane's result
// is valid on lanes j..63-j; step K's lanes K..63-K are the strip's outputs.
//
// Every intermediate result is rounded through the storage format before
// the next step reads it, exactly as a stored and reloaded value would be,
// so the result is bit-identical to K launches of the one-step kernels.
//
// Everything that indexes rows is uniform across the wave (scalar
// registers); per lane only the column offset differs. The row loop is
// unrolled over six phases (the row position mod 6) so that each carried
// group keeps a fixed register per phase, which leaves no register moves.
//
// A workgroup of nw waves takes nw adjacent strips of one chunk (a strip
// group) and its waves pass a barrier at every row, so their row accesses
// reach memory together as one contiguous run of nw * STRIP elements per
// plane. Strips past the right edge repeat the last strip and store nothing,
// so every wave of a workgroup runs the same number of rows and barriers.

// Sponge form chosen per launch item at run time (the batched kernel, whose
// members may each use another form); the other values are ChiMode.
constexpr int CHI_RUNTIME = 4;

// The VAR parameter of the strip kernels is a Variant, optionally with
// V_DEF set: in the compute precision the launch's conserved rates s_0,
// s_1, s_2 are all 0 and its shift parameters n and m are equal (collide's
// DEF).
// V_QF: a per-cell reference state (fixed in time) replaces the uniform
// q_ref: three planes of the reference's conserved-moment deviations, read
// per row like a sponge field (only with V_DEF and the damped variants).
// V_QA (with V_QF): the reference follows the cells' pre-collision
// conserved moments as a running mean, c^f <- c^f + alpha (c - c^f), after
// each step's collision; a launch reads the field and writes the updated
// one to a second buffer (strips read their neighbours' entries as halo).
constexpr int V_MASK = 7;
constexpr int V_DEF = 8;
constexpr int V_QF = 16;
constexpr int V_QA = 32;

template <int K>
constexpr int strip_width() {
  return 64 - 2 * K;
}
template <int M>
__device__ constexpr int md(int x) {  // x mod M in [0, M)
  return ((x % M) + M) % M;
}

template <typename S>
__device__ __forceinline__ typename Store<S>::C roundtrip(typename Store<S>::C v,
                                                          typename Store<S>::C scale,
                                                          typename Store<S>::C inv_scale) {
  S t;
  Store<S>::store(&t, v, inv_scale);
  return Store<S>::load(&t, scale);
}

// DPP wave shifts: wave_shr:1 gives lane l the value of lane l - 1,
// wave_shl:1 the value of lane l + 1 (lanes 0 and 63 receive 0; their
// results are never stored).
__device__ __forceinline__ int wave_shr1(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ int wave_shl1(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true);
}
__device__ __forceinline__ float lane_up(float v) {  // value of lane - 1
  return __builtin_bit_cast(float, wave_shr1(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float lane_down(float v) {  // value of lane + 1
  return __builtin_bit_cast(float, wave_shl1(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_up(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const unsigned lo = (unsigned)wave_shr1((int)b), hi = (unsigned)wave_shr1((int)(b >> 32));
  return __builtin_bit_cast(double, (long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double lane_down(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const unsigned lo = (unsigned)wave_shl1((int)b), hi = (unsigned)wave_shl1((int)(b >> 32));
  return __builtin_bit_cast(double, (long long)(((unsigned long long)hi << 32) | lo));
}

// Pull at one row: rm = the row above's {2, 5, 6}, r0 = this row's
// {0, 1, 3}, rp = the row below (all nine, only 4, 7, 8 read).
template <typename C>
__device__ __forceinline__ void pull(const C rm[3], const C r0[3], C rp4, C rp7, C rp8,
                                     C g[9]) {
  g[0] = r0[0];
  g[1] = lane_up(r0[1]);
  g[3] = lane_down(r0[2]);
  g[2] = rm[0];
  g[5] = lane_up(rm[1]);
  g[6] = lane_down(rm[2]);
  g[4] = rp4;
  g[7] = lane_down(rp7);
  g[8] = lane_up(rp8);
}

// Carried state of one wave. Ring slots are indexed by the row's position
// q = row - (Y0 - K) within the chunk (q >= 0): a group live over two
// iterations sits in slot q % 2, one live over three in slot q % 3.
template <typename C, int K>
struct StripState {
  C a478[3][3];         // input rows: populations 4, 7, 8 (loaded two rows ahead)
  C a013[3][3];         // input rows: populations 0, 1, 3
  C a256[3][3];         // input rows: populations 2, 5, 6
  C craw[6];            // sponge input (chi_raw) of the rows, slot q % 6
  C qraw[6][3];         // reference-state deviations of the rows (V_QF), slot q % 6
  C b013[K - 1][2][3];  // results of steps 1..K-1: populations 0, 1, 3
  C b256[K - 1][3][3];  // results of steps 1..K-1: populations 2, 5, 6
};

template <typename S, int VAR, int CHI, int K>
struct StripCtx {
  typedef typename Store<S>::C C;
  const S *src;
  S *dst;
  int64_t ps, pitch;
  unsigned col;        // this lane's column
  unsigned col_bytes;  // col * sizeof(S)
  unsigned out_bytes;  // (lane - K) * sizeof(S): output offset from the strip start
  unsigned row_bytes;  // bytes of a row's cells (the range of a row's loads)
  unsigned out_range;  // bytes of the strip's outputs in a row (0: an idle wave)
  bool store_lane;
  int nw;              // waves per workgroup
  int nx, ny, Y0, X0;
  C cx_chi;
  const C *chi_field, *chiy;
  int chi_mode;        // ChiMode, read when CHI == CHI_RUNTIME
  C scale[9], inv_scale[9];
  CollideParams<C> p;
  C mref[9];
  const C *qf;         // V_QF: [3][qps] reference-state deviations, rows of `pitch`
  C *qf_out;           // V_QA: the field after the launch's K steps
  int64_t qps;
  C alpha;             // V_QA: running-mean rate

  static constexpr bool QF = (VAR & V_QF) != 0;
  static constexpr bool QA = (VAR & V_QA) != 0;

  __device__ __forceinline__ int wrap_row(int r) const {
    r %= ny;
    return r < 0 ? r + ny : r;
  }
  // Rows are read and written through buffer resources: a scalar
  // descriptor (the row's address and byte range) plus the lane's 32-bit
  // byte offset, which is never modified and so needs no copy per access
  // (a global access with the scalar-base form needed one per load). An
  // access at or past the range reads 0 or is dropped: a row's loads cover
  // its nx cells, a row's stores the strip's own output columns. Stores are
  // also lane-masked (store_lane): left to the range check alone, the halo
  // lanes' addresses cost the memory-leaning two- and three-step shapes 4%.
  // Elements move as same-size integers (the FP16 element type is a class).
  typedef typename std::conditional<
      sizeof(S) == 2, uint16_t,
      typename std::conditional<sizeof(S) == 4, uint32_t, uint64_t>::type>::type Bits;
  static __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base,
                                                                unsigned bytes) {
    // raw access (stride 0); the third word is the gfx9-family default
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes,
                                             0x00020000);
  }
  __device__ __forceinline__ C ld(int i, int r) const {
    const __amdgpu_buffer_rsrc_t rs = rsrc(src + i * ps + (int64_t)r * pitch, row_bytes);
    Bits b;
    if constexpr (sizeof(S) == 2) {
      b = __builtin_amdgcn_raw_buffer_load_b16(rs, (int)col_bytes, 0, 0);
    } else if constexpr (sizeof(S) == 4) {
      b = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)col_bytes, 0, 0);
    } else {
      const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)col_bytes, 0, 0);
      __builtin_memcpy(&b, &w, sizeof(b));
    }
    S v;
    __builtin_memcpy(&v, &b, sizeof(S));
    return Store<S>::load(&v, scale[i]);
  }
  // store of population i at this lane's output column of row y (only
  // lanes with store_lane call it; the range drops anything else)
  __device__ __forceinline__ void st_out(int i, int y, C v) const {
    const __amdgpu_buffer_rsrc_t rs = rsrc(dst + i * ps + (int64_t)y * pitch + X0, out_range);
    S t;
    Store<S>::store(&t, v, inv_scale[i]);
    Bits b;
    __builtin_memcpy(&b, &t, sizeof(S));
    if constexpr (sizeof(S) == 2) {
      __builtin_amdgcn_raw_buffer_store_b16(b, rs, (int)out_bytes, 0, 0);
    } else if constexpr (sizeof(S) == 4) {
      __builtin_amdgcn_raw_buffer_store_b32(b, rs, (int)out_bytes, 0, 0);
    } else {
      // the 64-bit form takes a vector of two words
      decltype(__builtin_amdgcn_raw_buffer_load_b64(rs, 0, 0, 0)) w;
      __builtin_memcpy(&w, &b, sizeof(w));
      __builtin_amdgcn_raw_buffer_store_b64(w, rs, (int)out_bytes, 0, 0);
    }
  }
  // Sponge input of row r: the field value at this lane, or chi_y[r] of a
  // separable profile (combined with chi_x by chi_of when used).
  __device__ __forceinline__ int mode() const { return CHI == CHI_RUNTIME ? chi_mode : CHI; }
  __device__ __forceinline__ C chi_raw(int r) const {
    const int m = mode();
    if (m == CHI_ZERO) return C(0);
    if (m == CHI_FIELD) return chi_field[(int64_t)r * pitch + col];
    return chiy[r];
  }
  // Per-row cell inputs of row r into ring slot Q: the sponge input and,
  // with a reference field, the cell's reference-state deviations.
  template <int Q>
  __device__ __forceinline__ void row_inputs(StripState<C, K> &st, int r) const {
    st.craw[md<6>(Q)] = chi_raw(r);
    if constexpr (QF) {
      const int64_t cell = (int64_t)r * pitch + col;
      st.qraw[md<6>(Q)][0] = qf[cell];
      st.qraw[md<6>(Q)][1] = qf[qps + cell];
      st.qraw[md<6>(Q)][2] = qf[2 * qps + cell];
    }
  }
  // The collision of a cell of the row in ring slot Q; with a running-mean
  // reference the slot then holds the cell's updated reference.
  template <int Q>
  __device__ __forceinline__ void collide_at(StripState<C, K> &st, C g[9]) const {
    const C chi = chi_of(st.craw[md<6>(Q)]);
    if constexpr (QF) {
      CollideParams<C> pc = p;
      pc.dcf0 = st.qraw[md<6>(Q)][0];
      pc.dcf1 = st.qraw[md<6>(Q)][1];
      pc.dcf2 = st.qraw[md<6>(Q)][2];
      // pre-collision conserved moments (rows 0-2 of M, summed as the
      // collision sums them)
      C dr = C(0), djx = C(0), djy = C(0);
      if constexpr (QA) {
        dr = g[0] + ((g[1] + g[3]) + (g[2] + g[4])) + ((g[5] + g[7]) + (g[6] + g[8]));
        djx = (g[1] - g[3]) + ((g[5] - g[7]) + (g[8] - g[6]));
        djy = (g[2] - g[4]) + ((g[5] - g[7]) + (g[6] - g[8]));
      }
      C mr[9];
      if ((VAR & V_MASK) == V_I || (VAR & V_MASK) == V_II) ref_moments(pc, mr);
      collide<C, VAR & V_MASK, (VAR & V_DEF) != 0>(g, chi, pc, mr);
      if constexpr (QA) {
        st.qraw[md<6>(Q)][0] = fmaC(alpha, dr - pc.dcf0, pc.dcf0);
        st.qraw[md<6>(Q)][1] = fmaC(alpha, djx - pc.dcf1, pc.dcf1);
        st.qraw[md<6>(Q)][2] = fmaC(alpha, djy - pc.dcf2, pc.dcf2);
      }
    } else {
      collide<C, VAR & V_MASK, (VAR & V_DEF) != 0>(g, chi, p, mref);
    }
  }
  __device__ __forceinline__ C chi_of(C raw) const {
    const int m = mode();
    if (m == CHI_SEP_MAX) return cx_chi > raw ? cx_chi : raw;
    if (m == CHI_SEP_SUM) return cx_chi + raw;
    return raw;
  }
  // Loads of input row r (position Q).
  template <int Q>
  __device__ __forceinline__ void load_478(StripState<C, K> &st, int r) const {
    st.a478[md<3>(Q)][0] = ld(4, r);
    st.a478[md<3>(Q)][1] = ld(7, r);
    st.a478[md<3>(Q)][2] = ld(8, r);
  }
  template <int Q>
  __device__ __forceinline__ void load_013(StripState<C, K> &st, int r) const {
    st.a013[md<3>(Q)][0] = ld(0, r);
    st.a013[md<3>(Q)][1] = ld(1, r);
    st.a013[md<3>(Q)][2] = ld(3, r);
  }
  template <int Q>
  __device__ __forceinline__ void load_256(StripState<C, K> &st, int r) const {
    st.a256[md<3>(Q)][0] = ld(2, r);
    st.a256[md<3>(Q)][1] = ld(5, r);
    st.a256[md<3>(Q)][2] = ld(6, r);
  }
  // Keep the result of step JJ at row position Q for the rows below.
  template <int JJ, int Q>
  __device__ __forceinline__ void keep(StripState<C, K> &st, const C g[9]) const {
    st.b013[JJ - 1][md<2>(Q)][0] = g[0];
    st.b013[JJ - 1][md<2>(Q)][1] = g[1];
    st.b013[JJ - 1][md<2>(Q)][2] = g[3];
    st.b256[JJ - 1][md<3>(Q)][0] = g[2];
    st.b256[JJ - 1][md<3>(Q)][1] = g[5];
    st.b256[JJ - 1][md<3>(Q)][2] = g[6];
  }

  // Iteration at input row a (position P, taken mod 6): load what later
  // steps read of rows a + 1 (periodic row index r_next) and a + 2 (r_next2,
  // populations 4, 7, 8, which step 1 needs soonest), then steps 1..J at rows
  // a - 1 .. a - J.
  //
  // The loads are unconditional: near the end of the chunk they fetch up
  // to three rows that no step reads (valid rows, the index wraps), but
  // every iteration then issues the same memory operations, so each wait
  // for a row's data waits for that row alone and not for the loads issued
  // after it (a load behind a branch makes the wait drain them all).
  template <int P, int J>
  __device__ __forceinline__ void iter(StripState<C, K> &st, int a, int r_next,
                                       int r_next2) const {
    if (nw > 1) __builtin_amdgcn_s_barrier();  // rows of the strip group in step
    load_478<P + 2>(st, r_next2);
    load_013<P + 1>(st, r_next);
    // step 1 at row a - 1 from input rows a - 2, a - 1, a
    C g[9];
    {
      const C *rp = st.a478[md<3>(P)];
      pull<C>(st.a256[md<3>(P - 2)], st.a013[md<3>(P - 1)], rp[0], rp[1], rp[2], g);
    }
    // row a - 2's {2, 5, 6} are consumed: its slot takes row a + 1's
    load_256<P + 1>(st, r_next);
    // the cell inputs of row a + 1 go to another ring slot than row a - 1's,
    // and are first needed in the next iteration
    row_inputs<P + 1>(st, r_next);
    collide_at<P - 1>(st, g);
    chain<P, J, 2>(st, g, a);
  }

  // g = result of step j - 1 at row a - (j - 1); run steps j..J.
  template <int P, int J, int j>
  __device__ __forceinline__ void chain(StripState<C, K> &st, C g[9], int a) const {
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = roundtrip<S>(g[i], scale[i], inv_scale[i]);
    if constexpr (j > J) {
      keep<j - 1, P - (j - 1)>(st, g);
    } else {
      // step j at row a - j from step j - 1 rows a - j - 1, a - j, a - j + 1
      C o[9];
      pull<C>(st.b256[j - 2][md<3>(P - j - 1)], st.b013[j - 2][md<2>(P - j)], g[4], g[7], g[8],
              o);
      keep<j - 1, P - (j - 1)>(st, g);
      collide_at<P - j>(st, o);
      if constexpr (j == K) {
        if (store_lane) {
#pragma unroll
          for (int i = 0; i < 9; ++i) st_out(i, a - K, o[i]);
        }
        if constexpr (QA) {
          if (store_lane) {
            const int64_t cell = (int64_t)(a - K) * pitch + X0 + (threadIdx.x & 63) - K;
            qf_out[cell] = st.qraw[md<6>(P - K)][0];
            qf_out[qps + cell] = st.qraw[md<6>(P - K)][1];
            qf_out[2 * qps + cell] = st.qraw[md<6>(P - K)][2];
          }
        }
      } else {
        chain<P, J, j + 1>(st, o, a);
      }
    }
  }
};

// Lane geometry and launch constants of one strip: the wave's lane column,
// the sponge's x part and the collision parameters.
template <typename S, int VAR, int CHI, int K>
__device__ __forceinline__ void strip_setup(StripCtx<S, VAR, CHI, K> &c, const S *src, S *dst,
                                            int nx, int ny, int64_t pitch, int64_t ps, int strip,
                                            bool idle, int Y0, int nw,
                                            const typename Store<S>::C *chi_field,
                                            const typename Store<S>::C *chix,
                                            const typename Store<S>::C *chiy, int chi_mode,
                                            const typename Store<S>::C scale[9],
                                            const typename Store<S>::C inv_scale[9],
                                            const CollideParams<typename Store<S>::C> &p,
                                            const typename Store<S>::C *qf = nullptr,
                                            int64_t qps = 0,
                                            typename Store<S>::C *qf_out = nullptr,
                                            typename Store<S>::C alpha = 0) {
  typedef typename Store<S>::C C;
  constexpr int W = strip_width<K>();
  c.qf = qf;
  c.qps = qps;
  c.qf_out = qf_out;
  c.alpha = alpha;
  const int lane = threadIdx.x & 63;
  c.src = src;
  c.dst = dst;
  c.ps = ps;
  c.pitch = pitch;
  c.nx = nx;
  c.ny = ny;
  c.nw = nw;
  c.X0 = strip * W;
  c.Y0 = Y0;
  int col = (c.X0 - K + lane) % nx;
  if (col < 0) col += nx;
  c.col = (unsigned)col;
  c.col_bytes = (unsigned)col * (unsigned)sizeof(S);
  c.out_bytes = (unsigned)(lane - K) * (unsigned)sizeof(S);
  // a row holds fewer than 2^32 bytes (strip_row_fits): its byte count is
  // the range
  c.row_bytes = (unsigned)((uint64_t)nx * sizeof(S));
  c.out_range = idle ? 0u : (unsigned)(min(W, nx - c.X0) * (int)sizeof(S));
  c.store_lane = !idle && lane >= K && lane < K + W && c.X0 + lane - K < nx;
  c.chi_mode = chi_mode;
  const int m = c.mode();
  c.cx_chi = (m == CHI_SEP_MAX || m == CHI_SEP_SUM) ? chix[col] : C(0);
  c.chi_field = chi_field;
  c.chiy = chiy;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    c.scale[i] = scale[i];
    c.inv_scale[i] = inv_scale[i];
  }
  c.p = p;
  if (!StripCtx<S, VAR, CHI, K>::QF && ((VAR & V_MASK) == V_I || (VAR & V_MASK) == V_II))
    ref_moments(p, c.mref);
}

// The row loop of one strip over R output rows from Y0 on.
template <typename S, int VAR, int CHI, int K>
__device__ __forceinline__ void strip_run(const StripCtx<S, VAR, CHI, K> &c, int R) {
  typedef typename Store<S>::C C;
  const int ny = c.ny;
  StripState<C, K> st;
  // Positions q = 0, 1, 2, 3 (rows Y0 - K .. Y0 - K + 3): step 1 starts at
  // q = 1, so row q = 0 supplies only {2, 5, 6}; {4, 7, 8} run two rows ahead.
  auto next = [&](int rr) { return rr + 1 == ny ? 0 : rr + 1; };
  int r = c.wrap_row(c.Y0 - K);
  c.template load_256<0>(st, r);
  r = next(r);
  c.template load_256<1>(st, r);
  c.template load_013<1>(st, r);
  c.template row_inputs<1>(st, r);
  r = next(r);
  c.template load_478<2>(st, r);
  c.template load_013<2>(st, r);
  c.template load_256<2>(st, r);
  c.template row_inputs<2>(st, r);
  c.template load_478<3>(st, next(r));
  // Iterations q = 2 .. R + 2K - 1 at input rows a = Y0 - K + q. Step j runs
  // from q = 2j on: q = 2, 3 run step 1, q = 4, 5 steps 1-2, q = 6, 7 steps
  // 1-3, and from q = 2K on all K steps run (R iterations).
  int a = c.Y0 - K + 2;
  r = next(r);
  c.template iter<2, 1>(st, a, r, next(r));
  ++a;
  r = next(r);
  c.template iter<3, 1>(st, a, r, next(r));
  if constexpr (K >= 3) {
    ++a;
    r = next(r);
    c.template iter<4, 2>(st, a, r, next(r));
    ++a;
    r = next(r);
    c.template iter<5, 2>(st, a, r, next(r));
  }
  if constexpr (K >= 4) {
    ++a;
    r = next(r);
    c.template iter<0, 3>(st, a, r, next(r));
    ++a;
    r = next(r);
    c.template iter<1, 3>(st, a, r, next(r));
  }
  int left = R;  // iterations with all K steps
#define LBM_STRIP_ITER(PH)                                          \
  ++a;                                                              \
  r = next(r);                                                      \
  c.template iter<(2 * K + PH) % 6, K>(st, a, r, next(r));          \
  if (--left == 0) break;
  for (;;) {
    LBM_STRIP_ITER(0)
    LBM_STRIP_ITER(1)
    LBM_STRIP_ITER(2)
    LBM_STRIP_ITER(3)
    LBM_STRIP_ITER(4)
    LBM_STRIP_ITER(5)
  }
#undef LBM_STRIP_ITER
}

// Waves per SIMD the single-lattice kernel may run: the FP64 four-step form
// one (its 253 registers would fit two, but the fitted chunks then halve in
// height and the extra warm-up rows cost more than the second wave gains:
// 0.530 against 0.539 ms per launch at 4096^2), the others unconstrained.
template <typename S, int K>
constexpr int strip_max_waves() {
  return sizeof(S) == 8 && K == 4 ? 1 : 8;
}
template <typename S, int VAR, int CHI, int K>
__global__ __launch_bounds__(multi_step_max_block(sizeof(S) == 8 ? 0 : 1, K))
__attribute__((amdgpu_waves_per_eu(1, strip_max_waves<S, K>())))
void step_multi_strip(
    const S *__restrict__ src, S *__restrict__ dst, Lat<S> L,
    CollideParams<typename Store<S>::C> p,
    const typename Store<S>::C *__restrict__ chi_field,
    const typename Store<S>::C *__restrict__ chix,
    const typename Store<S>::C *__restrict__ chiy, const typename Store<S>::C *__restrict__ qf,
    typename Store<S>::C *__restrict__ qf_out, int64_t qps, typename Store<S>::C alpha,
    int rows_per_chunk, int nstrips, int ngroups, int wg_per_xcd, int nwg) {
  // XCD-aware order: workgroup i runs on XCD i % 8; give each XCD a
  // contiguous range of work (a band of chunk rows) so neighbouring strips
  // and chunks share an L2
  const int v = (blockIdx.x & 7) * wg_per_xcd + (blockIdx.x >> 3);
  if (v >= nwg) return;
  const int nw = blockDim.x >> 6;
  const int chunk = v / ngroups, group = v - chunk * ngroups;
  int strip = group * nw + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool idle = strip >= nstrips;
  if (idle) strip = nstrips - 1;
  const int Y0 = chunk * rows_per_chunk;
  StripCtx<S, VAR, CHI, K> c;
  strip_setup(c, src, dst, L.nx, L.ny, L.pitch, L.ps, strip, idle, Y0, nw, chi_field, chix, chiy,
              CHI, L.scale, L.inv_scale, p, qf, qps, qf_out, alpha);
  strip_run(c, min(rows_per_chunk, L.ny - Y0));
}

// Batched form: a persistent grid works through a table of work items
// (member domain, first strip of a strip group, first row, rows); each
// workgroup takes the next item with an atomic ticket (work[1 + j], zeroed
// before the launch; work[0] holds the item count) and runs the strip loop
// of its item with the member's own size, rates, variant, sponge and
// parity. The table lists the tallest items first, so the short ones fill
// the end of the launch. Launch j of a tick advances the members that take
// at least (j + 1) K steps in it.
// Workgroups take at most multi_step_max_block threads, as the single-lattice
// kernel. Waves per SIMD the registers are budgeted for: FP32 three (the
// run-time variant and rate switches would otherwise take it to two), two
// with per-cell references; FP16 (its round trips through the storage
// format hold more values) two; FP64 one.
// DEF: every member has the default form's parameters (collide's DEF).
// QF: members may carry a fixed per-cell reference state (BatchDomain::qf,
// set for the damped variants only); the form without it keeps the
// registers of the uniform reference (18 fewer carried values).
// MAXF: every member's sponge is the separable max form, compiled in. The
// run-time choice of the form costs a test at every collision, which cuts
// the loop into blocks and keeps the compiler from sharing 1/(1 + n chi)
// between the steps of a row: 116.7 against 127 VALU per collision (Type
// II), 166 against 160 GLUPS on 256 uneven members although the compiled-in
// form spills 48-65 registers at three waves per SIMD.
template <typename S, bool QF>
constexpr int batch_waves_per_simd() {
  return sizeof(S) == 8 ? 1 : (sizeof(S) == 2 || QF ? 2 : 3);
}
template <typename S, int K, bool DEF, bool QF, bool MAXF>
__global__ __launch_bounds__(multi_step_max_block(sizeof(S) == 8 ? 0 : 1, K))
__attribute__((amdgpu_waves_per_eu(batch_waves_per_simd<S, QF>())))
void batch_multi_strip(const BatchDomain *__restrict__ doms, const int4 *__restrict__ items,
                       int *__restrict__ work, int j) {
  typedef typename Store<S>::C C;
  const int nitems = work[0];
  int *ticket = work + 1 + j;
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __shared__ int s_ticket;
  for (;;) {
    int t;
    if (nw == 1) {
      int v = 0;
      if ((threadIdx.x & 63) == 0) v = atomicAdd(ticket, 1);
      t = __builtin_amdgcn_readfirstlane(v);
    } else {
      if (threadIdx.x == 0) s_ticket = atomicAdd(ticket, 1);
      __syncthreads();
      t = s_ticket;
      __syncthreads();  // everyone has read it before the next ticket replaces it
    }
    if (t >= nitems) break;
    const int4 it = items[t];
    const BatchDomain &d = doms[it.x];
    if (j >= d.stop_at / K) continue;
    const int nstrips = (d.nx + strip_width<K>() - 1) / strip_width<K>();
    int strip = it.y + wave;
    const bool idle = strip >= nstrips;
    if (idle) strip = nstrips - 1;
    const int par = (d.parity + j) & 1;
    C scale[9], inv_scale[9];
    CollideParams<C> p;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      scale[i] = C(d.scale[i]);
      inv_scale[i] = C(d.inv_scale[i]);
      p.s[i] = C(d.s[i]);
    }
    p.n = C(d.n);
    p.m = C(d.m);
    p.rho_b = C(d.rho_b);
    p.ubx = C(d.ubx);
    p.uby = C(d.uby);
    p.dcf0 = C(d.dcf[0]);
    p.dcf1 = C(d.dcf[1]);
    p.dcf2 = C(d.dcf[2]);
    set_relax_coeffs(p);
#define LBM_BATCH_RUN(VAR, QFP)                                                              \
  {                                                                                          \
    StripCtx<S, VAR | (DEF ? V_DEF : 0), MAXF ? CHI_SEP_MAX : CHI_RUNTIME, K> c;           \
    strip_setup(c, (const S *)d.lat[par], (S *)d.lat[par ^ 1], d.nx, d.ny, d.pitch, d.ps,   \
                strip, idle, it.z, nw, (const C *)d.chi_field, (const C *)d.chi_x,           \
                (const C *)d.chi_y, d.chi_mode, scale, inv_scale, p, QFP, d.qps);            \
    strip_run(c, it.w);                                                                      \
  }
    bool ran = false;
    if constexpr (QF) {
      if (d.qf) {
        const C *q = (const C *)d.qf;
        ran = true;
        switch (d.variant) {
          case V_I: LBM_BATCH_RUN(V_I | V_QF, q) break;
          case V_II: LBM_BATCH_RUN(V_II | V_QF, q) break;
          default: LBM_BATCH_RUN(V_III | V_QF, q) break;
        }
      }
    }
    if (!ran) {
      switch (d.variant) {
        case V_I: LBM_BATCH_RUN(V_I, nullptr) break;
        case V_II: LBM_BATCH_RUN(V_II, nullptr) break;
        case V_III: LBM_BATCH_RUN(V_III, nullptr) break;
        case V_VISC: LBM_BATCH_RUN(V_VISC, nullptr) break;
        default: LBM_BATCH_RUN(V_NONE, nullptr) break;
      }
    }
#undef LBM_BATCH_RUN
    // the next item may belong to another member: no wave of this
    // workgroup starts it before all have finished this one's rows
    if (nw > 1) __builtin_amdgcn_s_barrier();
  }
}

// Workgroups of the multi-step kernel that fit on the device at once, for
// workgroups of nw waves (nw = 1, 2, 4 or 8).
template <typename S, int VAR, int CHI, int K>
static int64_t multi_step_capacity(int nw) {
  static std::atomic<int64_t> cache[4] = {{-1}, {-1}, {-1}, {-1}};
  const int slot = nw == 1 ? 0 : (nw == 2 ? 1 : (nw == 4 ? 2 : 3));
  int64_t cap = cache[slot].load(std::memory_order_relaxed);
  if (cap >= 0) return cap;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, step_multi_strip<S, VAR, CHI, K>,
                                                   64 * nw, 0) != hipSuccess)
    return 0;
  cap = (int64_t)cus * per_cu;
  cache[slot].store(cap, std::memory_order_relaxed);
  return cap;
}

template <typename S, int VAR, int CHI, int K>
static hipError_t launch_multi_t(const StepConfig &c, const void *src, void *dst,
                                 hipStream_t stream) {
  typedef typename Store<S>::C C;
  Lat<S> L = make_lat<S>(c);
  CollideParams<C> p = make_params<C>(c);
  if (c.block > multi_step_max_block(sizeof(S) == 8 ? 0 : 1, K)) return hipErrorInvalidValue;
  const int nw = c.block == 64 ? 1 : (c.block == 128 ? 2 : (c.block == 256 ? 4 : 8));
  const int nstrips = (c.nx + strip_width<K>() - 1) / strip_width<K>();
  const int ngroups = (nstrips + nw - 1) / nw;
  int rows = c.rows;
  if (rows <= 0) {
    // chunk height that lets every workgroup be resident at once
    const int64_t cap = multi_step_capacity<S, VAR, CHI, K>(nw);
    const int64_t chunks = cap > ngroups ? cap / ngroups : 1;
    rows = (int)((c.ny + chunks - 1) / chunks);
  }
  const int nchunks = (c.ny + rows - 1) / rows;
  const int64_t nwg = (int64_t)ngroups * nchunks;
  const int64_t per_xcd = (nwg + 7) / 8;
  if (8 * per_xcd > 0x7fffffff) return hipErrorInvalidValue;
  step_multi_strip<S, VAR, CHI, K><<<dim3((unsigned)(8 * per_xcd)), dim3(64 * nw), 0, stream>>>(
      (const S *)src, (S *)dst, L, p, (const C *)c.chi_field, (const C *)c.chi_x,
      (const C *)c.chi_y, (const C *)c.qfield, (C *)c.qfield_out, c.qps, C(c.qalpha), rows,
      nstrips, ngroups, (int)per_xcd, (int)nwg);
  return hipGetLastError();
}

// A translation unit may instantiate the kernels of one step count only
// (LBM_STRIP_ONLY_K), so that the step counts compile side by side.
template <int K>
static constexpr bool strip_k_built() {
#ifdef LBM_STRIP_ONLY_K
  return K == LBM_STRIP_ONLY_K;
#else
  return true;
#endif
}

template <typename S, int VAR, int CHI, int K>
static hipError_t launch_multi_k(const StepConfig &c, const void *src, void *dst,
                                 hipStream_t stream) {
  if constexpr (strip_k_built<K>()) return launch_multi_t<S, VAR, CHI, K>(c, src, dst, stream);
  return hipErrorInvalidValue;
}

template <typename S, int VAR, int CHI>
static hipError_t launch_multi(const StepConfig &c, int k, const void *src, void *dst,
                               hipStream_t stream) {
  switch (k) {
    case 2: return launch_multi_k<S, VAR, CHI, 2>(c, src, dst, stream);
    case 3: return launch_multi_k<S, VAR, CHI, 3>(c, src, dst, stream);
    case 4: return launch_multi_k<S, VAR, CHI, 4>(c, src, dst, stream);
  }
  return hipErrorInvalidValue;
}

template <typename S, int K, bool DEF, bool QF, bool MAXF>
static hipError_t launch_batch_multi_k(int nw, const BatchDomain *doms, const int4 *items,
                                       int *nitems, int grid, int j, hipStream_t s) {
  if constexpr (strip_k_built<K>()) {
    batch_multi_strip<S, K, DEF, QF, MAXF>
        <<<dim3(grid), dim3(64 * nw), 0, s>>>(doms, items, nitems, j);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <typename S, bool DEF, bool QF, bool MAXF>
static hipError_t launch_batch_multi_t(int k, int nw, const BatchDomain *doms, const int4 *items,
                                       int *nitems, int grid, int j, hipStream_t s) {
  switch (k) {
    case 2: return launch_batch_multi_k<S, 2, DEF, QF, MAXF>(nw, doms, items, nitems, grid, j, s);
    case 3: return launch_batch_multi_k<S, 3, DEF, QF, MAXF>(nw, doms, items, nitems, grid, j, s);
    case 4: return launch_batch_multi_k<S, 4, DEF, QF, MAXF>(nw, doms, items, nitems, grid, j, s);
  }
  return hipErrorInvalidValue;
}

template <typename S, bool DEF, bool QF>
static hipError_t launch_batch_multi_m(int k, int nw, bool mx, const BatchDomain *doms,
                                       const int4 *items, int *nitems, int grid, int j,
                                       hipStream_t s) {
  return mx ? launch_batch_multi_t<S, DEF, QF, true>(k, nw, doms, items, nitems, grid, j, s)
            : launch_batch_multi_t<S, DEF, QF, false>(k, nw, doms, items, nitems, grid, j, s);
}

// (Internal linkage: each translation unit builds its own step counts.)
template <typename S>
static hipError_t launch_batch_multi_storage(int k, int nw, int form, const BatchDomain *doms,
                                             const int4 *items, int *nitems, int grid, int j,
                                             hipStream_t s) {
  const bool mx = form & BATCH_SEPMAX;
  switch (form & (BATCH_DEF | BATCH_QF)) {
    case BATCH_DEF:
      return launch_batch_multi_m<S, true, false>(k, nw, mx, doms, items, nitems, grid, j, s);
    case BATCH_DEF | BATCH_QF:
      return launch_batch_multi_m<S, true, true>(k, nw, mx, doms, items, nitems, grid, j, s);
    case BATCH_QF:
      return launch_batch_multi_m<S, false, true>(k, nw, mx, doms, items, nitems, grid, j, s);
  }
  return launch_batch_multi_m<S, false, false>(k, nw, mx, doms, items, nitems, grid, j, s);
}

template <typename S, int K, bool DEF, bool QF, bool MAXF>
static int batch_multi_per_cu_k(int nw) {
  int per_cu = 0;
  if constexpr (strip_k_built<K>()) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, batch_multi_strip<S, K, DEF, QF, MAXF>, 64 * nw, 0) != hipSuccess)
      return 0;
  }
  return per_cu;
}

template <typename S, bool DEF, bool QF, bool MAXF>
static int batch_multi_per_cu_t(int k, int nw) {
  switch (k) {
    case 2: return batch_multi_per_cu_k<S, 2, DEF, QF, MAXF>(nw);
    case 3: return batch_multi_per_cu_k<S, 3, DEF, QF, MAXF>(nw);
    case 4: return batch_multi_per_cu_k<S, 4, DEF, QF, MAXF>(nw);
  }
  return 0;
}

template <typename S, bool DEF, bool QF>
static int batch_multi_per_cu_m(int k, int nw, bool mx) {
  return mx ? batch_multi_per_cu_t<S, DEF, QF, true>(k, nw)
            : batch_multi_per_cu_t<S, DEF, QF, false>(k, nw);
}

// Workgroups of nw waves of the batched multi-step kernel resident per CU.
template <typename S>
static int batch_multi_per_cu(int k, int nw, int form) {
  const bool mx = form & BATCH_SEPMAX;
  switch (form & (BATCH_DEF | BATCH_QF)) {
    case BATCH_DEF: return batch_multi_per_cu_m<S, true, false>(k, nw, mx);
    case BATCH_DEF | BATCH_QF: return batch_multi_per_cu_m<S, true, true>(k, nw, mx);
    case BATCH_QF: return batch_multi_per_cu_m<S, false, true>(k, nw, mx);
  }
  return batch_multi_per_cu_m<S, false, false>(k, nw, mx);
}

// All variants, sponge forms and step counts of one storage type.
template <typename S>
static hipError_t launch_multi_storage(const StepConfig &c, int k, const void *src, void *dst,
                                hipStream_t s) {
#define LBM_CHI(VAR)                                                          \
  switch (c.chi_mode) {                                                       \
    case CHI_ZERO: return launch_multi<S, VAR, CHI_ZERO>(c, k, src, dst, s);   \
    case CHI_FIELD: return launch_multi<S, VAR, CHI_FIELD>(c, k, src, dst, s); \
    case CHI_SEP_MAX: return launch_multi<S, VAR, CHI_SEP_MAX>(c, k, src, dst, s); \
    case CHI_SEP_SUM: return launch_multi<S, VAR, CHI_SEP_SUM>(c, k, src, dst, s); \
  }                                                                           \
  return hipErrorInvalidValue;
  typedef typename Store<S>::C C;
  const bool def = C(c.s[0]) == C(0) && C(c.s[1]) == C(0) && C(c.s[2]) == C(0) &&
                   C(c.n) == C(c.m);
  if (c.qfield && (c.variant == V_I || c.variant == V_II || c.variant == V_III)) {
    // a per-cell reference state: the default form only (multi_step_supports)
    if (!def) return hipErrorInvalidValue;
    if (c.qalpha != 0.0) {
      if (!c.qfield_out) return hipErrorInvalidValue;
      switch (c.variant) {
        case V_I: { LBM_CHI(V_I | V_DEF | V_QF | V_QA) }
        case V_II: { LBM_CHI(V_II | V_DEF | V_QF | V_QA) }
        case V_III: { LBM_CHI(V_III | V_DEF | V_QF | V_QA) }
      }
    }
    switch (c.variant) {
      case V_I: { LBM_CHI(V_I | V_DEF | V_QF) }
      case V_II: { LBM_CHI(V_II | V_DEF | V_QF) }
      case V_III: { LBM_CHI(V_III | V_DEF | V_QF) }
    }
  }
  if (def) {
    switch (c.variant) {
      case V_NONE: { LBM_CHI(V_NONE | V_DEF) }
      case V_I: { LBM_CHI(V_I | V_DEF) }
      case V_II: { LBM_CHI(V_II | V_DEF) }
      case V_III: { LBM_CHI(V_III | V_DEF) }
      case V_VISC: { LBM_CHI(V_VISC | V_DEF) }
    }
  } else {
    switch (c.variant) {
      case V_NONE: { LBM_CHI(V_NONE) }
      case V_I: { LBM_CHI(V_I) }
      case V_II: { LBM_CHI(V_II) }
      case V_III: { LBM_CHI(V_III) }
      case V_VISC: { LBM_CHI(V_VISC) }
    }
  }
#undef LBM_CHI
  return hipErrorInvalidValue;
}

}  // namespace lbm
