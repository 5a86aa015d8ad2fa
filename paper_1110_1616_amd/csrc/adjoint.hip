// Discrete adjoint of the single-level advance (band 2, refilled by the copy
// map every step) for gfx950.  One reverse step maps the adjoint of the
// output state, lambda' (interior cells and own faces), to the adjoint of the
// input state, with every branch frozen at the recomputed forward values.
// It is a sequence of gathers (each output element has one writer):
//   k_adj_pred   forward: predicted face states of every cell   -> PS
//   k_adj_face   per face: flux adjoint from lambda' (cell updates and edge
//                EMFs), then the HLLD adjoint                   -> AF
//   k_adj_cell   per cell: adjoint of the Hancock predictor, face states and
//                slopes' use                                    -> AC
//   k_adj_prim   per cell: adjoint of the minmod slopes (frozen choices) and
//                of the primitive recovery                      -> AU
//   k_adj_assemble  per element: identity part of the update plus every
//                contribution above                             -> TMP
//   k_adj_fold   transpose of the band copy: band adjoints are added to the
//                interior elements they were copied from        -> lambda
#include "adjoint_internal.hpp"
#include "advance_common.hpp"
#include "emf.hpp"
#include "mhd_adjoint.hpp"

namespace amr {

namespace {

// Decode the element of a flat item: grid and local (i, j, k) in [-g, n+g].
struct ElemPos {
  int i, j, k;
  int64_t e;
  bool ok;
};

template <int NDIM>
__device__ __forceinline__ ElemPos elem_pos(const GridDesc& G, int local) {
  ElemPos p;
  const int box = G.P[0] * G.P[1] * G.P[2];
  p.ok = local < box;
  const int i = local % G.P[0];
  const int j = (local / G.P[0]) % G.P[1];
  const int k = local / (G.P[0] * G.P[1]);
  p.i = i - G.g;
  p.j = j - G.g;
  p.k = NDIM == 3 ? k - G.g : 0;
  p.e = G.off + local;
  return p;
}

__device__ __forceinline__ bool in_range(int x, int lo, int hi) { return x >= lo && x < hi; }

template <int NDIM> struct Reg {
  // cell regions for band-2 steps: W [-2, n+2), predicted [-1, n+1), own [0, n)
  __device__ static bool cells(const GridDesc& G, int i, int j, int k, int w) {
    return in_range(i, -w, G.n[0] + w) && in_range(j, -w, G.n[1] + w) && (NDIM == 2 || in_range(k, -w, G.n[2] + w));
  }
};

template <class T> struct AdjArrays {
  T* ps;  // predicted states: [(d*2+side)*7 + q] arrays
  T* af;  // per face direction: [d*15 + 0..6] a_WL, [+7..13] a_WR, [+14] a_Bn
  T* ac;  // per cell: [0..7] a_Wpred, [8 + d*8 + q] a_slope, [32 + d*2 + side] a_face
  T* au;  // per cell: [0..4] a_U hydro, [5] a_Bz cell (2D), [6 + d] a_Bbar
  T* tmp; // 8 assembled adjoint arrays
  int64_t stride;  // elements per array
  int64_t e0;      // pool element of array index 0
  __device__ T& PS(int d, int side, int q, int64_t e) const {
    return ps[(int64_t)((d * 2 + side) * 7 + q) * stride + (e - e0)];
  }
  __device__ T& AF(int d, int c, int64_t e) const { return af[(int64_t)(d * 15 + c) * stride + (e - e0)]; }
  __device__ T& AC(int c, int64_t e) const { return ac[(int64_t)c * stride + (e - e0)]; }
  __device__ T& AU(int c, int64_t e) const { return au[(int64_t)c * stride + (e - e0)]; }
  __device__ T& TMP(int c, int64_t e) const { return tmp[(int64_t)c * stride + (e - e0)]; }
};

// Step size and 1/dx of a grid's level, evaluated as the forward kernels do.
template <class T, int NDIM> struct LevelStep {
  T dt, hdt, idx[3];
  __device__ __forceinline__ LevelStep(const GridDesc& G, const Phys& ph, double dt0) {
    double rl = 1.0;
    for (int l = 0; l < G.level; ++l) rl *= (double)ph.ratio;
    dt = T(dt0 / rl);
    hdt = T(0.5) * dt;
    idx[0] = T(rl / ph.dx0[0]);
    idx[1] = T(rl / ph.dx0[1]);
    idx[2] = T(NDIM == 3 ? rl / ph.dx0[2] : 0.0);
  }
};

template <class T> __device__ __forceinline__ T ldz(const T* p, int64_t e, bool ok) { return ok ? p[e] : T(0); }

// ------------------------------------------------------------- K1 forward
template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_adj_pred(const GridDesc* __restrict__ grids, const int2* __restrict__ items,
                                                  int nitems, DevState<T> U, AdjArrays<T> A, double dt0, Phys ph) {
  const T gam = T(ph.gamma), gm1 = gam - T(1);
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const GridDesc G = grids[item.x];
    const ElemPos p = elem_pos<NDIM>(G, item.y + threadIdx.x);
    if (!p.ok || !Reg<NDIM>::cells(G, p.i, p.j, p.k, 1)) continue;
    const Idx<NDIM> ix(G);
    const LevelStep<T, NDIM> ls(G, ph, dt0);
    const int64_t st[3] = {1, ix.sy, NDIM == 3 ? ix.sz : 0};
    T w[8], wxm[8], wxp[8], wym[8], wyp[8], wzm[8], wzp[8];
    load_prim<T, NDIM>(U, p.e, ix.sy, ix.sz, gm1, w);
    load_prim<T, NDIM>(U, p.e - st[0], ix.sy, ix.sz, gm1, wxm);
    load_prim<T, NDIM>(U, p.e + st[0], ix.sy, ix.sz, gm1, wxp);
    load_prim<T, NDIM>(U, p.e - st[1], ix.sy, ix.sz, gm1, wym);
    load_prim<T, NDIM>(U, p.e + st[1], ix.sy, ix.sz, gm1, wyp);
    if (NDIM == 3) {
      load_prim<T, NDIM>(U, p.e - st[2], ix.sy, ix.sz, gm1, wzm);
      load_prim<T, NDIM>(U, p.e + st[2], ix.sy, ix.sz, gm1, wzp);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) { wzm[q] = w[q]; wzp[q] = w[q]; }
    }
    T fb[3][2];
    fb[0][0] = U.f[5][p.e];
    fb[0][1] = U.f[5][p.e + 1];
    fb[1][0] = U.f[6][p.e];
    fb[1][1] = U.f[6][p.e + st[1]];
    fb[2][0] = NDIM == 3 ? U.f[7][p.e] : T(0);
    fb[2][1] = NDIM == 3 ? U.f[7][p.e + st[2]] : T(0);
    Pred<T, NDIM> pr;
    (void)predict<T, NDIM>(w, wxm, wxp, wym, wyp, wzm, wzp, fb, ls.hdt, ls.idx, gam, pr);
#pragma unroll
    for (int d = 0; d < NDIM; ++d)
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        A.PS(d, 0, q, p.e) = pr.m[d][q];
        A.PS(d, 1, q, p.e) = pr.p[d][q];
      }
  }
}

// ------------------------------------------------------------- K2 faces
template <class T, int NDIM>
__device__ __forceinline__ bool own_face(const GridDesc& G, int d, int i, int j, int k) {
  const int x[3] = {i, j, k};
#pragma unroll
  for (int a = 0; a < NDIM; ++a) {
    const int hi = a == d ? G.n[a] + 1 : G.n[a];
    if (x[a] < 0 || x[a] >= hi) return false;
  }
  return true;
}

template <class T, int NDIM>
__device__ __forceinline__ bool own_cell(const GridDesc& G, int i, int j, int k) {
  return Reg<NDIM>::cells(G, i, j, k, 0);
}

// adjoint of the EMF along axis a at the edge with high-side cell (i,j,k):
// the face updates that use it (lambda' on own faces only)
template <class T, int NDIM>
__device__ __forceinline__ T edge_lambda(const GridDesc& G, const DevState<T>& Lp, int a, int i, int j, int k,
                                         const int64_t (&st)[3], const T (&cdt)[3]) {
  const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
  const int64_t e = G.off + (i + G.g) + (int64_t)(j + G.g) * st[1] + (NDIM == 3 ? (int64_t)(k + G.g) * st[2] : 0);
  T v = T(0);
  int x[3] = {i, j, k};
  // faces normal a1: lambda(E_a) += cdt[a2] (lam_{a1}(e) - lam_{a1}(e - e_{a2}))
  if (a2 < NDIM) {
    int y[3] = {x[0], x[1], x[2]};
    y[a2] -= 1;
    const T l0 = own_face<T, NDIM>(G, a1, x[0], x[1], x[2]) ? Lp.f[5 + a1][e] : T(0);
    const T l1 = own_face<T, NDIM>(G, a1, y[0], y[1], y[2]) ? Lp.f[5 + a1][e - st[a2]] : T(0);
    v += cdt[a2] * (l0 - l1);
  }
  // faces normal a2: lambda(E_a) -= cdt[a1] (lam_{a2}(e) - lam_{a2}(e - e_{a1}))
  if (a1 < NDIM) {
    int y[3] = {x[0], x[1], x[2]};
    y[a1] -= 1;
    const T l0 = own_face<T, NDIM>(G, a2, x[0], x[1], x[2]) ? Lp.f[5 + a2][e] : T(0);
    const T l1 = own_face<T, NDIM>(G, a2, y[0], y[1], y[2]) ? Lp.f[5 + a2][e - st[a1]] : T(0);
    v -= cdt[a1] * (l0 - l1);
  }
  return v;
}

template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_adj_face(const GridDesc* __restrict__ grids, const int2* __restrict__ items,
                                                  int nitems, DevState<T> U, DevState<T> Lp, AdjArrays<T> A,
                                                  double dt0, Phys ph) {
  const T gam = T(ph.gamma);
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const GridDesc G = grids[item.x];
    const ElemPos p = elem_pos<NDIM>(G, item.y + threadIdx.x);
    if (!p.ok) continue;
    const LevelStep<T, NDIM> ls(G, ph, dt0);
    // dU/dF and dB/dE coefficients of the update: dt / dx per axis
    const T cdt[3] = {ls.dt * ls.idx[0], ls.dt * ls.idx[1], ls.dt * ls.idx[2]};
    const int64_t st[3] = {1, G.P[0], NDIM == 3 ? (int64_t)G.P[0] * G.P[1] : 0};
    const int x[3] = {p.i, p.j, p.k};
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      // flux faces: normal index [0, n], transverse [-1, n]
      bool ok = true;
#pragma unroll
      for (int a = 0; a < NDIM; ++a) {
        const int lo = a == d ? 0 : -1;
        const int hi = G.n[a] + 1;
        ok = ok && x[a] >= lo && x[a] < hi;
      }
      if (!ok) continue;
      int xm[3] = {x[0], x[1], x[2]};
      xm[d] -= 1;
      const bool oc = own_cell<T, NDIM>(G, x[0], x[1], x[2]);
      const bool om = own_cell<T, NDIM>(G, xm[0], xm[1], xm[2]);
      T af[7];
      // hydro slots (and the cell Bz of 2D): dU(c)/dF = +dt/dx, dU(c-e_d)/dF = -dt/dx
      const int slots[6] = {0, 1, 2, 3, 4, 7};
      const int ns = NDIM == 2 ? 6 : 5;
#pragma unroll
      for (int q = 0; q < 7; ++q) af[q] = T(0);
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        if (t >= ns) break;
        const int s = slots[t];
        const T lc = ldz(Lp.f[s], p.e, oc);
        const T lm = ldz(Lp.f[s], p.e - st[d], om);
        af[flux_comp(s, d)] += cdt[d] * (lc - lm);
      }
      if (NDIM == 3) {
        // component 5 (B_{d+1}) enters E_{d+2} at this edge and at +e_{d+1}
        const int a5 = (d + 2) % 3, o5 = (d + 1) % 3;
        int y[3] = {x[0], x[1], x[2]};
        y[o5] += 1;
        af[5] += -T(0.25) * (edge_lambda<T, NDIM>(G, Lp, a5, x[0], x[1], x[2], st, cdt) +
                             edge_lambda<T, NDIM>(G, Lp, a5, y[0], y[1], y[2], st, cdt));
        // component 6 (B_{d+2}) enters E_{d+1} at this edge and at +e_{d+2}
        const int a6 = (d + 1) % 3, o6 = (d + 2) % 3;
        int z[3] = {x[0], x[1], x[2]};
        z[o6] += 1;
        af[6] += T(0.25) * (edge_lambda<T, NDIM>(G, Lp, a6, x[0], x[1], x[2], st, cdt) +
                            edge_lambda<T, NDIM>(G, Lp, a6, z[0], z[1], z[2], st, cdt));
      } else {
        if (d == 0) {  // B_y flux -> E_z at this corner and +y
          int y[3] = {x[0], x[1] + 1, 0};
          af[5] += -T(0.25) * (edge_lambda<T, NDIM>(G, Lp, 2, x[0], x[1], 0, st, cdt) +
                               edge_lambda<T, NDIM>(G, Lp, 2, y[0], y[1], 0, st, cdt));
        } else {  // B_x flux -> E_z at this corner and +x
          int y[3] = {x[0] + 1, x[1], 0};
          af[6] += T(0.25) * (edge_lambda<T, NDIM>(G, Lp, 2, x[0], x[1], 0, st, cdt) +
                              edge_lambda<T, NDIM>(G, Lp, 2, y[0], y[1], 0, st, cdt));
        }
      }
      // HLLD adjoint: L = (d,+) state of cell c - e_d, R = (d,-) state of c
      T ql[8], qr[8], aql[8], aqr[8];
      const T bn = U.f[5 + d][p.e];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        ql[q] = A.PS(d, 1, q, p.e - st[d]);
        qr[q] = A.PS(d, 0, q, p.e);
      }
      ql[5] = bn;
      qr[5] = bn;
      ql[6] = A.PS(d, 1, 5, p.e - st[d]);
      ql[7] = A.PS(d, 1, 6, p.e - st[d]);
      qr[6] = A.PS(d, 0, 5, p.e);
      qr[7] = A.PS(d, 0, 6, p.e);
#pragma unroll
      for (int q = 0; q < 8; ++q) { aql[q] = T(0); aqr[q] = T(0); }
      T abn = T(0);
      riemann_hlld_adj(ql, qr, bn, gam, af, aql, aqr, abn);
      // the face B_n enters both states (slot 5) and the solver directly
      abn += aql[5] + aqr[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        A.AF(d, q, p.e) = aql[q];
        A.AF(d, 7 + q, p.e) = aqr[q];
      }
      A.AF(d, 5, p.e) = aql[6];
      A.AF(d, 6, p.e) = aql[7];
      A.AF(d, 12, p.e) = aqr[6];
      A.AF(d, 13, p.e) = aqr[7];
      A.AF(d, 14, p.e) = abn;
    }
  }
}

// --------------------------------------------------- K3 cell predictor
// unrotate a 7-component rotated adjoint of direction D into the lab frame
template <int D, class T>
__device__ __forceinline__ void unrotate7(const T (&q)[7], T (&w)[8]) {
  w[0] = q[0];
  w[1 + D] = q[1];
  w[1 + (D + 1) % 3] = q[2];
  w[1 + (D + 2) % 3] = q[3];
  w[4] = q[4];
  w[5 + D] = T(0);
  w[5 + (D + 1) % 3] = q[5];
  w[5 + (D + 2) % 3] = q[6];
}

template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_adj_cell(const GridDesc* __restrict__ grids, const int2* __restrict__ items,
                                                  int nitems, DevState<T> U, AdjArrays<T> A, double dt0, Phys ph) {
  const T gam = T(ph.gamma), gm1 = gam - T(1), gm1_inv = T(1) / gm1;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const GridDesc G = grids[item.x];
    const ElemPos p = elem_pos<NDIM>(G, item.y + threadIdx.x);
    if (!p.ok || !Reg<NDIM>::cells(G, p.i, p.j, p.k, 1)) continue;
    const LevelStep<T, NDIM> ls(G, ph, dt0);
    const T cd[3] = {ls.hdt * ls.idx[0], ls.hdt * ls.idx[1], ls.hdt * ls.idx[2]};
    const Idx<NDIM> ix(G);
    const int64_t st[3] = {1, ix.sy, NDIM == 3 ? ix.sz : 0};
    const int x[3] = {p.i, p.j, p.k};
    // forward recompute: W, slopes, face states, increment
    T w[8], nb[3][2][8];
    load_prim<T, NDIM>(U, p.e, ix.sy, ix.sz, gm1, w);
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      load_prim<T, NDIM>(U, p.e - st[d], ix.sy, ix.sz, gm1, nb[d][0]);
      load_prim<T, NDIM>(U, p.e + st[d], ix.sy, ix.sz, gm1, nb[d][1]);
    }
    T sl[3][8], ws[3][2][8], fb[3][2];
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      fb[d][0] = U.f[5 + d][p.e];
      fb[d][1] = U.f[5 + d][p.e + st[d]];
#pragma unroll
      for (int q = 0; q < 8; ++q) sl[d][q] = limiter_minmod(w[q] - nb[d][0][q], nb[d][1][q] - w[q]);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        ws[d][0][q] = w[q] - T(0.5) * sl[d][q];
        ws[d][1][q] = w[q] + T(0.5) * sl[d][q];
      }
      ws[d][0][5 + d] = fb[d][0];
      ws[d][1][5 + d] = fb[d][1];
    }
    T du[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) du[q] = T(0);
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      T fl[8], fr[8];
      if (d == 0) { flux_along<0>(ws[d][0], fl, gm1_inv); flux_along<0>(ws[d][1], fr, gm1_inv); }
      else if (d == 1) { flux_along<1>(ws[d][0], fl, gm1_inv); flux_along<1>(ws[d][1], fr, gm1_inv); }
      else { flux_along<2>(ws[d][0], fl, gm1_inv); flux_along<2>(ws[d][1], fr, gm1_inv); }
      const T c = cd[d];
#pragma unroll
      for (int q = 0; q < 8; ++q) du[q] -= c * (fr[q] - fl[q]);
    }
    // reverse: predicted states
    T a_ws[3][2][8], a_du[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a_du[q] = T(0);
#pragma unroll
    for (int d = 0; d < NDIM; ++d)
#pragma unroll
      for (int side = 0; side < 2; ++side) {
#pragma unroll
        for (int q = 0; q < 8; ++q) a_ws[d][side][q] = T(0);
        // adjoint of the predicted state (d, side) from its face
        int y[3] = {x[0], x[1], x[2]};
        if (side == 1) y[d] += 1;
        bool okf = true;
#pragma unroll
        for (int a = 0; a < NDIM; ++a) {
          const int lo = a == d ? 0 : -1;
          okf = okf && y[a] >= lo && y[a] < G.n[a] + 1;
        }
        T a7[7];
        const int64_t fe = side == 1 ? p.e + st[d] : p.e;
        const int off = side == 1 ? 0 : 7;  // (d,+) is the L state of the face above
#pragma unroll
        for (int q = 0; q < 7; ++q) a7[q] = okf ? A.AF(d, off + q, fe) : T(0);
        T a_wb[8];
        if (d == 0) unrotate7<0>(a7, a_wb);
        else if (d == 1) unrotate7<1>(a7, a_wb);
        else unrotate7<2>(a7, a_wb);
        T us[8], ubar[8];
        to_conserved(ws[d][side], us, gm1_inv);
#pragma unroll
        for (int q = 0; q < 8; ++q) ubar[q] = us[q] + du[q];
        T a_ub[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) a_ub[q] = T(0);
        to_primitive_adj(ubar, gm1, a_wb, a_ub);
#pragma unroll
        for (int q = 0; q < 8; ++q) a_du[q] += a_ub[q];
        to_conserved_adj(ws[d][side], gm1_inv, a_ub, a_ws[d][side]);
      }
    // reverse: increment du = -sum_d c_d (F_d(w+) - F_d(w-))
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      T afr[8], afl[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        afr[q] = -cd[d] * a_du[q];
        afl[q] = cd[d] * a_du[q];
      }
      if (d == 0) { flux_along_adj<0>(ws[d][1], gm1_inv, afr, a_ws[d][1]); flux_along_adj<0>(ws[d][0], gm1_inv, afl, a_ws[d][0]); }
      else if (d == 1) { flux_along_adj<1>(ws[d][1], gm1_inv, afr, a_ws[d][1]); flux_along_adj<1>(ws[d][0], gm1_inv, afl, a_ws[d][0]); }
      else { flux_along_adj<2>(ws[d][1], gm1_inv, afr, a_ws[d][1]); flux_along_adj<2>(ws[d][0], gm1_inv, afl, a_ws[d][0]); }
    }
    // reverse: face states W +- slope/2 (normal B from the faces)
    T a_w[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a_w[q] = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int q = 0; q < 8; ++q) A.AC(8 + d * 8 + q, p.e) = T(0);
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (q == 5 + d) continue;
        a_w[q] += a_ws[d][0][q] + a_ws[d][1][q];
        A.AC(8 + d * 8 + q, p.e) = T(0.5) * (a_ws[d][1][q] - a_ws[d][0][q]);
      }
      A.AC(32 + d * 2 + 0, p.e) = a_ws[d][0][5 + d];
      A.AC(32 + d * 2 + 1, p.e) = a_ws[d][1][5 + d];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) A.AC(q, p.e) = a_w[q];
  }
}

// ------------------------------------------------ K4 slopes + primitives
template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_adj_prim(const GridDesc* __restrict__ grids, const int2* __restrict__ items,
                                                  int nitems, DevState<T> U, AdjArrays<T> A, Phys ph) {
  const T gam = T(ph.gamma), gm1 = gam - T(1);
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const GridDesc G = grids[item.x];
    const ElemPos p = elem_pos<NDIM>(G, item.y + threadIdx.x);
    if (!p.ok || !Reg<NDIM>::cells(G, p.i, p.j, p.k, 2)) continue;
    const Idx<NDIM> ix(G);
    const int64_t st[3] = {1, ix.sy, NDIM == 3 ? ix.sz : 0};
    const int x[3] = {p.i, p.j, p.k};
    T a_w[8];
    const bool pred_here = Reg<NDIM>::cells(G, x[0], x[1], x[2], 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) a_w[q] = pred_here ? A.AC(q, p.e) : T(0);
    // slopes of the cells c' = c - e_d, c, c + e_d use W(c)
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
#pragma unroll
      for (int o = -1; o <= 1; ++o) {
        int y[3] = {x[0], x[1], x[2]};
        y[d] += o;
        if (!Reg<NDIM>::cells(G, y[0], y[1], y[2], 1)) continue;
        const int64_t ec = p.e + o * st[d];
        T wm[8], wc[8], wp[8];
        load_prim<T, NDIM>(U, ec - st[d], ix.sy, ix.sz, gm1, wm);
        load_prim<T, NDIM>(U, ec, ix.sy, ix.sz, gm1, wc);
        load_prim<T, NDIM>(U, ec + st[d], ix.sy, ix.sz, gm1, wp);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (q == 5 + d) continue;
          const T a = wc[q] - wm[q], b = wp[q] - wc[q];
          if (!(a * b > T(0))) continue;
          const bool pick_b = dabs(b) < dabs(a);
          const T as = A.AC(8 + d * 8 + q, ec);
          // slope = a = W(c') - W(c'-e_d), or b = W(c'+e_d) - W(c')
          if (!pick_b) {
            if (o == 0) a_w[q] += as;       // c' = c
            else if (o == 1) a_w[q] -= as;  // c = c' - e_d
          } else {
            if (o == -1) a_w[q] += as;      // c = c' + e_d
            else if (o == 0) a_w[q] -= as;  // c' = c
          }
        }
      }
    }
    // primitive recovery with cell-centred B
    T u[8], a_u[8];
    u[0] = U.f[0][p.e];
    u[1] = U.f[1][p.e];
    u[2] = U.f[2][p.e];
    u[3] = U.f[3][p.e];
    u[4] = U.f[4][p.e];
    u[5] = T(0.5) * (U.f[5][p.e] + U.f[5][p.e + 1]);
    u[6] = T(0.5) * (U.f[6][p.e] + U.f[6][p.e + st[1]]);
    u[7] = NDIM == 3 ? T(0.5) * (U.f[7][p.e] + U.f[7][p.e + st[2]]) : U.f[7][p.e];
#pragma unroll
    for (int q = 0; q < 8; ++q) a_u[q] = T(0);
    to_primitive_adj(u, gm1, a_w, a_u);
#pragma unroll
    for (int q = 0; q < 5; ++q) A.AU(q, p.e) = a_u[q];
    A.AU(5, p.e) = NDIM == 2 ? a_u[7] : T(0);
    A.AU(6, p.e) = a_u[5];
    A.AU(7, p.e) = a_u[6];
    A.AU(8, p.e) = NDIM == 3 ? a_u[7] : T(0);
  }
}

// ------------------------------------------------------- K5 assemble
template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_adj_assemble(const GridDesc* __restrict__ grids,
                                                      const int2* __restrict__ items, int nitems, DevState<T> Lp,
                                                      AdjArrays<T> A) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const GridDesc G = grids[item.x];
    const ElemPos p = elem_pos<NDIM>(G, item.y + threadIdx.x);
    if (!p.ok) continue;
    const int64_t st[3] = {1, G.P[0], NDIM == 3 ? (int64_t)G.P[0] * G.P[1] : 0};
    const int x[3] = {p.i, p.j, p.k};
    const bool oc = own_cell<T, NDIM>(G, x[0], x[1], x[2]);
    const bool wc = Reg<NDIM>::cells(G, x[0], x[1], x[2], 2);
    // cell fields
    const int slots[6] = {0, 1, 2, 3, 4, 7};
    const int ns = NDIM == 2 ? 6 : 5;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      if (t >= ns) break;
      const int s = slots[t];
      T v = oc ? Lp.f[s][p.e] : T(0);
      if (wc) v += A.AU(t, p.e);
      A.TMP(s, p.e) = v;
    }
    // faces
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      int xm[3] = {x[0], x[1], x[2]};
      xm[d] -= 1;
      // inside the padded box the face index runs to n+g
      T v = own_face<T, NDIM>(G, d, x[0], x[1], x[2]) ? Lp.f[5 + d][p.e] : T(0);
      bool flux = true;
#pragma unroll
      for (int a = 0; a < NDIM; ++a) {
        const int lo = a == d ? 0 : -1;
        flux = flux && x[a] >= lo && x[a] < G.n[a] + 1;
      }
      if (flux) v += A.AF(d, 14, p.e);
      if (Reg<NDIM>::cells(G, x[0], x[1], x[2], 1)) v += A.AC(32 + d * 2 + 0, p.e);
      if (Reg<NDIM>::cells(G, xm[0], xm[1], xm[2], 1)) v += A.AC(32 + d * 2 + 1, p.e - st[d]);
      if (Reg<NDIM>::cells(G, x[0], x[1], x[2], 2)) v += T(0.5) * A.AU(6 + d, p.e);
      if (Reg<NDIM>::cells(G, xm[0], xm[1], xm[2], 2)) v += T(0.5) * A.AU(6 + d, p.e - st[d]);
      A.TMP(5 + d, p.e) = v;
    }
  }
}

// ----------------------------------------------------------- K6 fold
template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_adj_own(const GridDesc* __restrict__ grids, const int2* __restrict__ items,
                                                 int nitems, AdjArrays<T> A, DevState<T> Lout) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const GridDesc G = grids[item.x];
    const ElemPos p = elem_pos<NDIM>(G, item.y + threadIdx.x);
    if (!p.ok) continue;
    const bool oc = own_cell<T, NDIM>(G, p.i, p.j, p.k);
    const int slots[6] = {0, 1, 2, 3, 4, 7};
    const int ns = NDIM == 2 ? 6 : 5;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      if (t >= ns) break;
      Lout.f[slots[t]][p.e] = oc ? A.TMP(slots[t], p.e) : T(0);
    }
#pragma unroll
    for (int d = 0; d < NDIM; ++d)
      Lout.f[5 + d][p.e] = own_face<T, NDIM>(G, d, p.i, p.j, p.k) ? A.TMP(5 + d, p.e) : T(0);
  }
}

template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_adj_fold(const InvCopy* __restrict__ inv, int n,
                                                  const int32_t* __restrict__ dsts, AdjArrays<T> A,
                                                  DevState<T> Lout) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const InvCopy c = inv[t];
    if (c.cls == 0) {
      const int slots[6] = {0, 1, 2, 3, 4, 7};
      const int ns = NDIM == 2 ? 6 : 5;
      for (int q = 0; q < ns; ++q) {
        T acc = T(0);
        for (int i = c.begin; i < c.end; ++i) acc += A.TMP(slots[q], dsts[i]);
        Lout.f[slots[q]][c.src] += acc;
      }
    } else {
      const int s = 4 + c.cls;
      T acc = T(0);
      for (int i = c.begin; i < c.end; ++i) acc += A.TMP(s, dsts[i]);
      Lout.f[s][c.src] += acc;
    }
  }
}

// ----------------------------------------- store / load-primitive adjoints
template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_store_adj(GridDesc G, Ptr8 g, DevState<T> L) {
  // own elements of L <- g (interior layout: cells nx*ny*nz, faces along d
  // with n_d + 1 entries on that axis)
  const int nx = G.n[0], ny = G.n[1], nz = NDIM == 3 ? G.n[2] : 1;
  const int64_t sy = G.P[0], sz = (int64_t)G.P[0] * G.P[1];
  const int64_t base = G.off + G.g + G.g * sy + (NDIM == 3 ? (int64_t)G.g * sz : 0);
  const int ex = nx + 1, ey = ny + 1, ez = nz + (NDIM == 3 ? 1 : 0);
  const int64_t total = (int64_t)ex * ey * ez;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % ex), j = (int)((t / ex) % ey), k = (int)(t / ((int64_t)ex * ey));
    const int64_t e = base + i + j * sy + (int64_t)k * sz;
    const bool ci = i < nx, cj = j < ny, ck = k < nz;
    if (ci && cj && ck) {
      const int64_t c = ((int64_t)k * ny + j) * nx + i;
      for (int s = 0; s < 5; ++s) L.f[s][e] = T(g.p[s][c]);
      if (NDIM == 2) L.f[7][e] = T(g.p[7][c]);
    }
    if (cj && ck) L.f[5][e] = T(g.p[5][((int64_t)k * ny + j) * (nx + 1) + i]);
    if (ci && ck) L.f[6][e] = T(g.p[6][((int64_t)k * (ny + 1) + j) * nx + i]);
    if (NDIM == 3 && ci && cj) L.f[7][e] = T(g.p[7][((int64_t)k * ny + j) * nx + i]);
  }
}

template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_load_prim_adj(GridDesc G, Ptr8 prim, DevState<T> L, MutPtr8 out) {
  // U(rho, v) = (rho, rho v, p/(gamma-1) + rho |v|^2 / 2 + |B|^2 / 2), so
  // dJ/drho = l_rho + l_m . v + l_E |v|^2 / 2 and dJ/dv = rho (l_m + l_E v)
  const int nx = G.n[0], ny = G.n[1], nz = NDIM == 3 ? G.n[2] : 1;
  const int64_t sy = G.P[0], sz = (int64_t)G.P[0] * G.P[1];
  const int64_t base = G.off + G.g + G.g * sy + (NDIM == 3 ? (int64_t)G.g * sz : 0);
  const int64_t total = (int64_t)nx * ny * nz;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % nx), j = (int)((t / nx) % ny), k = (int)(t / ((int64_t)nx * ny));
    const int64_t e = base + i + j * sy + (int64_t)k * sz;
    const double r = prim.p[0][t], vx = prim.p[1][t], vy = prim.p[2][t], vz = prim.p[3][t];
    const double lr = (double)L.f[0][e], lx = (double)L.f[1][e], ly = (double)L.f[2][e], lz = (double)L.f[3][e],
                 le = (double)L.f[4][e];
    out.p[0][t] = lr + lx * vx + ly * vy + lz * vz + 0.5 * le * (vx * vx + vy * vy + vz * vz);
    out.p[1][t] = r * (lx + le * vx);
    out.p[2][t] = r * (ly + le * vy);
    out.p[3][t] = r * (lz + le * vz);
  }
}

struct Values32 {
  double v[32];
};

__global__ void k_put_values(double* __restrict__ dst, Values32 vals, int n) {
  const int t = threadIdx.x;
  if (t < n) dst[t] = vals.v[t];
}

inline int blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65535) b = 65535;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

template <class T>
void launch_adjoint_step(int ndim, const GridDesc* grids, const int2* items, int nitems, const InvCopy* inv, int ninv,
                         const int32_t* dsts, DevState<T> U, DevState<T> Lp, DevState<T> Lout, AdjBuffers buf,
                         double dt0, Phys ph, hipStream_t s) {
  if (nitems <= 0) return;
  AdjArrays<T> A;
  A.ps = (T*)buf.ps;
  A.af = (T*)buf.af;
  A.ac = (T*)buf.ac;
  A.au = (T*)buf.au;
  A.tmp = (T*)buf.tmp;
  A.stride = buf.stride;
  A.e0 = buf.e0;
  const dim3 grid(nitems), block(256);
  if (ndim == 3) {
    hipLaunchKernelGGL((k_adj_pred<T, 3>), grid, block, 0, s, grids, items, nitems, U, A, dt0, ph);
    hipLaunchKernelGGL((k_adj_face<T, 3>), grid, block, 0, s, grids, items, nitems, U, Lp, A, dt0, ph);
    hipLaunchKernelGGL((k_adj_cell<T, 3>), grid, block, 0, s, grids, items, nitems, U, A, dt0, ph);
    hipLaunchKernelGGL((k_adj_prim<T, 3>), grid, block, 0, s, grids, items, nitems, U, A, ph);
    hipLaunchKernelGGL((k_adj_assemble<T, 3>), grid, block, 0, s, grids, items, nitems, Lp, A);
    hipLaunchKernelGGL((k_adj_own<T, 3>), grid, block, 0, s, grids, items, nitems, A, Lout);
    if (ninv > 0)
      hipLaunchKernelGGL((k_adj_fold<T, 3>), dim3(blocks_for(ninv)), block, 0, s, inv, ninv, dsts, A, Lout);
  } else {
    hipLaunchKernelGGL((k_adj_pred<T, 2>), grid, block, 0, s, grids, items, nitems, U, A, dt0, ph);
    hipLaunchKernelGGL((k_adj_face<T, 2>), grid, block, 0, s, grids, items, nitems, U, Lp, A, dt0, ph);
    hipLaunchKernelGGL((k_adj_cell<T, 2>), grid, block, 0, s, grids, items, nitems, U, A, dt0, ph);
    hipLaunchKernelGGL((k_adj_prim<T, 2>), grid, block, 0, s, grids, items, nitems, U, A, ph);
    hipLaunchKernelGGL((k_adj_assemble<T, 2>), grid, block, 0, s, grids, items, nitems, Lp, A);
    hipLaunchKernelGGL((k_adj_own<T, 2>), grid, block, 0, s, grids, items, nitems, A, Lout);
    if (ninv > 0)
      hipLaunchKernelGGL((k_adj_fold<T, 2>), dim3(blocks_for(ninv)), block, 0, s, inv, ninv, dsts, A, Lout);
  }
}

template <class T>
void launch_store_adj(int ndim, const GridDesc& G, Ptr8 g, DevState<T> L, hipStream_t s) {
  int64_t n = (int64_t)(G.n[0] + 1) * (G.n[1] + 1) * (ndim == 3 ? G.n[2] + 1 : 1);
  if (ndim == 3)
    hipLaunchKernelGGL((k_store_adj<T, 3>), dim3(blocks_for(n)), dim3(256), 0, s, G, g, L);
  else
    hipLaunchKernelGGL((k_store_adj<T, 2>), dim3(blocks_for(n)), dim3(256), 0, s, G, g, L);
}

template <class T>
void launch_load_prim_adj(int ndim, const GridDesc& G, Ptr8 prim, DevState<T> L, MutPtr8 out, hipStream_t s) {
  int64_t n = (int64_t)G.n[0] * G.n[1] * (ndim == 3 ? G.n[2] : 1);
  if (ndim == 3)
    hipLaunchKernelGGL((k_load_prim_adj<T, 3>), dim3(blocks_for(n)), dim3(256), 0, s, G, prim, L, out);
  else
    hipLaunchKernelGGL((k_load_prim_adj<T, 2>), dim3(blocks_for(n)), dim3(256), 0, s, G, prim, L, out);
}

void launch_put_values(double* dst, const double* host, int n, hipStream_t s) {
  for (int i = 0; i < n; i += 32) {
    Values32 v{};
    const int m = n - i < 32 ? n - i : 32;
    for (int j = 0; j < m; ++j) v.v[j] = host[i + j];
    hipLaunchKernelGGL(k_put_values, dim3(1), dim3(32), 0, s, dst + i, v, m);
  }
}

#define AMR_ADJ_INST(T)                                                                                             \
  template void launch_adjoint_step<T>(int, const GridDesc*, const int2*, int, const InvCopy*, int, const int32_t*, \
                                       DevState<T>, DevState<T>, DevState<T>, AdjBuffers, double, Phys,             \
                                       hipStream_t);                                                                \
  template void launch_store_adj<T>(int, const GridDesc&, Ptr8, DevState<T>, hipStream_t);                       \
  template void launch_load_prim_adj<T>(int, const GridDesc&, Ptr8, DevState<T>, MutPtr8, hipStream_t);
AMR_ADJ_INST(float)
AMR_ADJ_INST(double)
#undef AMR_ADJ_INST

}  // namespace amr
