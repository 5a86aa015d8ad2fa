// Per-cell pieces of the forward advance shared by the forward kernels and
// the adjoint kernels (which re-evaluate them to freeze the same branches).
#pragma once
#include "amr_internal.hpp"
#include "mhd_device.hpp"

namespace amr {

template <int NDIM> struct Idx {
  int64_t base;  // element of cell (0,0,0)
  int32_t sy, sz;
  __host__ __device__ __forceinline__ Idx(const GridDesc& G) {
    sy = G.P[0];
    sz = G.P[0] * G.P[1];
    base = G.off + G.g + (int64_t)G.g * sy + (NDIM == 3 ? (int64_t)G.g * sz : 0);
  }
  __host__ __device__ __forceinline__ int64_t operator()(int i, int j, int k) const {
    return base + i + (int64_t)j * sy + (NDIM == 3 ? (int64_t)k * sz : 0);
  }
};

// Addressing by 32-bit byte offsets from the start of the level arrays (a
// field's array holds under 2^32 bytes; the hierarchy's set-up checks): the
// array pointers stay in scalar registers and each lane carries one 32-bit
// offset, so loads and stores take the scalar-base form instead of 64-bit
// lane addresses.  IdxB gives the byte offset of interior cell (i, j, k) of a
// grid (i, j, k >= -g); the sums wrap modulo 2^32 to the exact offset.
template <int NDIM, class T> struct IdxB {
  using B = typename ByteOffset<T>::type;
  B b0;            // cell (0,0,0)
  int32_t sy, sz;  // row and plane strides
  __host__ __device__ __forceinline__ IdxB(const GridDesc& G) {
    sy = G.P[0] * (int32_t)sizeof(T);
    sz = G.P[0] * G.P[1] * (int32_t)sizeof(T);
    const int64_t e0 = G.off + G.g + (int64_t)G.g * G.P[0] + (NDIM == 3 ? (int64_t)G.g * G.P[0] * G.P[1] : 0);
    b0 = (B)(e0 * (int64_t)sizeof(T));
  }
  __host__ __device__ __forceinline__ B operator()(int i, int j, int k) const {
    return b0 + (B)(i * (int32_t)sizeof(T) + j * sy + (NDIM == 3 ? k * sz : 0));
  }
};

// load_prim / load_prim_faces at byte offset b (strides sy, sz in bytes).
template <class T, int NDIM, class B>
__device__ __forceinline__ void load_prim_b(const DevState<T>& U, B b, int32_t sy, int32_t sz, T gm1,
                                            T (&w)[8]) {
  T u[8];
#pragma unroll
  for (int q = 0; q < 5; ++q) u[q] = ldb(U.f[q], b);
  u[5] = T(0.5) * (ldb(U.f[5], b) + ldb(U.f[5], b, (int)sizeof(T)));
  u[6] = T(0.5) * (ldb(U.f[6], b) + ldb(U.f[6], b + sy));
  if (NDIM == 3)
    u[7] = T(0.5) * (ldb(U.f[7], b) + ldb(U.f[7], b + sz));
  else
    u[7] = ldb(U.f[7], b);
  to_primitive(u, w, gm1);
}

template <class T, int NDIM, class B>
__device__ __forceinline__ void load_prim_faces_b(const DevState<T>& U, B b, int32_t sy, int32_t sz, T gm1,
                                                  T (&w)[8], T (&fb)[3][2]) {
  T u[8];
#pragma unroll
  for (int q = 0; q < 5; ++q) u[q] = ldb(U.f[q], b);
  fb[0][0] = ldb(U.f[5], b);
  fb[0][1] = ldb(U.f[5], b, (int)sizeof(T));
  fb[1][0] = ldb(U.f[6], b);
  fb[1][1] = ldb(U.f[6], b + sy);
  u[5] = T(0.5) * (fb[0][0] + fb[0][1]);
  u[6] = T(0.5) * (fb[1][0] + fb[1][1]);
  if (NDIM == 3) {
    fb[2][0] = ldb(U.f[7], b);
    fb[2][1] = ldb(U.f[7], b + sz);
    u[7] = T(0.5) * (fb[2][0] + fb[2][1]);
  } else {
    fb[2][0] = T(0);
    fb[2][1] = T(0);
    u[7] = ldb(U.f[7], b);
  }
  to_primitive(u, w, gm1);
}

// Primitive state of cell e (element index) from the conserved state and
// the bounding faces.
template <class T, int NDIM>
__device__ __forceinline__ void load_prim(const DevState<T>& U, int64_t e, int32_t sy, int32_t sz, T gm1, T (&w)[8]) {
  T u[8];
  u[0] = U.f[0][e];
  u[1] = U.f[1][e];
  u[2] = U.f[2][e];
  u[3] = U.f[3][e];
  u[4] = U.f[4][e];
  u[5] = T(0.5) * (U.f[5][e] + U.f[5][e + 1]);
  u[6] = T(0.5) * (U.f[6][e] + U.f[6][e + sy]);
  if (NDIM == 3)
    u[7] = T(0.5) * (U.f[7][e] + U.f[7][e + sz]);
  else
    u[7] = U.f[7][e];
  to_primitive(u, w, gm1);
}

// load_prim that also returns the cell's six face fields (low/high along
// x, y, z; zero along z in 2D), which the predictor needs as the normal B of
// its face states.
template <class T, int NDIM>
__device__ __forceinline__ void load_prim_faces(const DevState<T>& U, int64_t e, int32_t sy, int32_t sz, T gm1,
                                                T (&w)[8], T (&fb)[3][2]) {
  T u[8];
  u[0] = U.f[0][e];
  u[1] = U.f[1][e];
  u[2] = U.f[2][e];
  u[3] = U.f[3][e];
  u[4] = U.f[4][e];
  fb[0][0] = U.f[5][e];
  fb[0][1] = U.f[5][e + 1];
  fb[1][0] = U.f[6][e];
  fb[1][1] = U.f[6][e + sy];
  u[5] = T(0.5) * (fb[0][0] + fb[0][1]);
  u[6] = T(0.5) * (fb[1][0] + fb[1][1]);
  if (NDIM == 3) {
    fb[2][0] = U.f[7][e];
    fb[2][1] = U.f[7][e + sz];
    u[7] = T(0.5) * (fb[2][0] + fb[2][1]);
  } else {
    fb[2][0] = T(0);
    fb[2][1] = T(0);
    u[7] = U.f[7][e];
  }
  to_primitive(u, w, gm1);
}

// load_prim_faces_b in two halves, so the loads can be issued a plane ahead
// of the arithmetic: the raw conserved fields and face fields of the cell at
// byte offset b (3-D), then the same conversion.
template <class T, class B>
__device__ __forceinline__ void load_raw3(const DevState<T>& U, B b, int32_t sy, int32_t sz, T (&u)[5],
                                          T (&fb)[3][2]) {
#pragma unroll
  for (int q = 0; q < 5; ++q) u[q] = ldb(U.f[q], b);
  fb[0][0] = ldb(U.f[5], b);
  fb[0][1] = ldb(U.f[5], b, (int)sizeof(T));
  fb[1][0] = ldb(U.f[6], b);
  fb[1][1] = ldb(U.f[6], b + sy);
  fb[2][0] = ldb(U.f[7], b);
  fb[2][1] = ldb(U.f[7], b + sz);
}

template <class T>
__device__ __forceinline__ void raw3_to_prim(const T (&r)[5], const T (&fb)[3][2], T gm1, T (&w)[8]) {
  T u[8];
#pragma unroll
  for (int q = 0; q < 5; ++q) u[q] = r[q];
  u[5] = T(0.5) * (fb[0][0] + fb[0][1]);
  u[6] = T(0.5) * (fb[1][0] + fb[1][1]);
  u[7] = T(0.5) * (fb[2][0] + fb[2][1]);
  to_primitive(u, w, gm1);
}

__device__ __forceinline__ void flag_bad(ErrBlock* err, int64_t e) {
  unsigned old = atomicOr(&err->flags, 1u);
  if ((old & 1u) == 0u) atomicExch((unsigned long long*)&err->first_bad, (unsigned long long)e);
}

// Direction-d face states of one cell, Hancock-evolved to the half step and
// returned as rotated primitives (rho, u_n, u_t1, u_t2, p, B_t1, B_t2).
template <int D, class T>
__device__ __forceinline__ void rotate7(const T (&w)[8], T (&q)[7]) {
  q[0] = w[0];
  q[1] = w[1 + D];
  q[2] = w[1 + (D + 1) % 3];
  q[3] = w[1 + (D + 2) % 3];
  q[4] = w[4];
  q[5] = w[5 + (D + 1) % 3];
  q[6] = w[5 + (D + 2) % 3];
}

template <class T, int NDIM>
struct Pred {
  T m[3][7];  // low-side (minus) states per direction
  T p[3][7];  // high-side (plus) states per direction
};

// Slopes, face states, Hancock increment and predicted states of one cell.
// wx/wy/wz hold the neighbours (minus, plus) along each axis; fb[d][0/1] are
// the cell's low/high face fields along d.  Each predicted state is handed to
// emit(d, side, q) as soon as it is formed (side 0 low, 1 high), so callers
// that store it right away never hold all 2*NDIM states in registers.
// Returns false if a predicted density or pressure is not positive.
// When WANT_DU, du_out receives the Hancock increment of the cell's
// conserved state.
template <class T, int NDIM, bool WANT_DU = false, class Emit>
__device__ __forceinline__ bool predict_emit(const T (&w)[8], const T (&wxm)[8], const T (&wxp)[8],
                                             const T (&wym)[8], const T (&wyp)[8], const T (&wzm)[8],
                                             const T (&wzp)[8], const T (&fb)[3][2], T hdt, const T (&idx)[3], T gam,
                                             Emit&& emit, T (&du_out)[8]) {
  const T gm1 = gam - T(1);
  const T gm1_inv = drcp(gm1);
  T sl[3][8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    sl[0][q] = limiter_minmod(w[q] - wxm[q], wxp[q] - w[q]);
    sl[1][q] = limiter_minmod(w[q] - wym[q], wyp[q] - w[q]);
    if (NDIM == 3) sl[2][q] = limiter_minmod(w[q] - wzm[q], wzp[q] - w[q]);
  }
  T du[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) du[q] = T(0);
#pragma unroll
  for (int d = 0; d < NDIM; ++d) {
    T wl[8], wr[8], fl[8], fr[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      wl[q] = w[q] - T(0.5) * sl[d][q];
      wr[q] = w[q] + T(0.5) * sl[d][q];
    }
    wl[5 + d] = fb[d][0];
    wr[5 + d] = fb[d][1];
    if (d == 0) {
      flux_along<0>(wl, fl, gm1_inv);
      flux_along<0>(wr, fr, gm1_inv);
    } else if (d == 1) {
      flux_along<1>(wl, fl, gm1_inv);
      flux_along<1>(wr, fr, gm1_inv);
    } else {
      flux_along<2>(wl, fl, gm1_inv);
      flux_along<2>(wr, fr, gm1_inv);
    }
    const T c = hdt * idx[d];
#pragma unroll
    for (int q = 0; q < 8; ++q) du[q] -= c * (fr[q] - fl[q]);
  }
  if constexpr (WANT_DU) {
#pragma unroll
    for (int q = 0; q < 8; ++q) du_out[q] = du[q];
  }
  bool ok = true;
#pragma unroll
  for (int d = 0; d < NDIM; ++d) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      T ws[8], us[8], wb[8];
      const T h = side ? T(0.5) : T(-0.5);
#pragma unroll
      for (int q = 0; q < 8; ++q) ws[q] = w[q] + h * sl[d][q];
      ws[5 + d] = fb[d][side];
      to_conserved(ws, us, gm1_inv);
#pragma unroll
      for (int q = 0; q < 8; ++q) us[q] += du[q];
      to_primitive(us, wb, gm1);
      ok = ok && (wb[0] > T(0)) && (wb[4] > T(0));
      T q7[7];
      if (d == 0) rotate7<0>(wb, q7);
      else if (d == 1) rotate7<1>(wb, q7);
      else rotate7<2>(wb, q7);
      emit(d, side, q7);
    }
  }
  return ok;
}

template <class T, int NDIM>
__device__ __forceinline__ bool predict(const T (&w)[8], const T (&wxm)[8], const T (&wxp)[8], const T (&wym)[8],
                                        const T (&wyp)[8], const T (&wzm)[8], const T (&wzp)[8],
                                        const T (&fb)[3][2], T hdt, const T (&idx)[3], T gam,
                                        Pred<T, NDIM>& out) {
  T unused[8];
  return predict_emit<T, NDIM>(w, wxm, wxp, wym, wyp, wzm, wzp, fb, hdt, idx, gam,
                               [&](int d, int side, const T (&q)[7]) {
#pragma unroll
                                 for (int c = 0; c < 7; ++c) (side ? out.p[d] : out.m[d])[c] = q[c];
                               }, unused);
}

// predict() that also returns the Hancock increment du of the cell.
template <class T, int NDIM>
__device__ __forceinline__ bool predict_du(const T (&w)[8], const T (&wxm)[8], const T (&wxp)[8], const T (&wym)[8],
                                           const T (&wyp)[8], const T (&wzm)[8], const T (&wzp)[8],
                                           const T (&fb)[3][2], T hdt, const T (&idx)[3], T gam,
                                           Pred<T, NDIM>& out, T (&du)[8]) {
  return predict_emit<T, NDIM, true>(w, wxm, wxp, wym, wyp, wzm, wzp, fb, hdt, idx, gam,
                                     [&](int d, int side, const T (&q)[7]) {
#pragma unroll
                                       for (int c = 0; c < 7; ++c) (side ? out.p[d] : out.m[d])[c] = q[c];
                                     }, du);
}

template <class T>
__device__ __forceinline__ void hlld7(const T (&l)[7], const T (&r)[7], T bn, T gam, T (&f)[7]) {
  T ql[8] = {l[0], l[1], l[2], l[3], l[4], bn, l[5], l[6]};
  T qr[8] = {r[0], r[1], r[2], r[3], r[4], bn, r[5], r[6]};
  riemann_hlld(ql, qr, bn, gam, f);
}


}  // namespace amr
