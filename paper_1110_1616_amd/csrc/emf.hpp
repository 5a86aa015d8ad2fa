// Edge EMF of constrained transport from stored face fluxes (shared by the
// update kernel and the synchronisation registers so both see the same
// value bit for bit).
#pragma once
#include "amr_internal.hpp"

namespace amr {

// The update's arithmetic, shared by the update kernel, the fused
// flux-update kernel and the registers so that all of them produce the same
// bits: no multiply-add contraction here (it would otherwise depend on the
// code each is inlined into).  Edge EMF from the four face values around the
// edge: b_lo, b_hi the B_t1 flux component on the two b-faces, c_lo, c_hi
// the B_t2 component on the two c-faces (low side first).
template <class T> __device__ __forceinline__ T emf_mean(T b_lo, T b_hi, T c_lo, T c_hi) {
#pragma clang fp contract(off)
  const T s1 = b_lo + b_hi;
  const T s2 = c_lo + c_hi;
  return T(0.25) * (s2 - s1);
}
// Flux difference of a cell field over its faces: cdx (F_x,high - F_x,low) +
// cdy (...) [+ cdz (...) in 3-D].
template <class T, int NDIM>
__device__ __forceinline__ T flux_delta(T cdx, T xh, T xl, T cdy, T yh, T yl, T cdz, T zh, T zl) {
#pragma clang fp contract(off)
  T acc = cdx * (xh - xl) + cdy * (yh - yl);
  if (NDIM == 3) acc += cdz * (zh - zl);
  return acc;
}
// Curl term of a face update: c1 (a1 - a0) - c2 (b1 - b0); in 2-D the
// single term c (a1 - a0).
template <class T> __device__ __forceinline__ T curl_delta(T c1, T a1, T a0, T c2, T b1, T b0) {
#pragma clang fp contract(off)
  return c1 * (a1 - a0) - c2 * (b1 - b0);
}
template <class T> __device__ __forceinline__ T face_delta2(T c, T a1, T a0) {
#pragma clang fp contract(off)
  return c * (a1 - a0);
}
// Updated value u - d (kept apart from the products above).
template <class T> __device__ __forceinline__ T sub_nc(T u, T d) {
#pragma clang fp contract(off)
  return u - d;
}
// Rotated flux component of direction d that carries lab conserved slot s
// (0..4): density and energy keep their slot; momentum a = s - 1 is the
// normal (1), first (2) or second (3) tangential component.
__host__ __device__ __forceinline__ int hydro_comp(int s, int d) {
  return (s == 0 || s == 4) ? s : 1 + (s - 1 + 3 - d) % 3;
}

// EMF along axis A at the edge whose high-side cell (in the two other axes)
// has element e: the mean of the four adjacent face values, E_A = -F_b(B_c)
// on b-faces and +F_c(B_b) on c-faces (b = A+1, c = A+2; rotated flux
// components 5 = B_t1 and 6 = B_t2).  st: element strides of the grid.
template <int A, class T>
__device__ __forceinline__ T edge_emf(const DevFlux<T>& F, int64_t e, const int64_t (&st)[3]) {
  constexpr int B = (A + 1) % 3, C = (A + 2) % 3;
  return emf_mean(F.f[B][5][e - st[C]], F.f[B][5][e], F.f[C][6][e - st[B]], F.f[C][6][e]);
}

// Upwinded EMF (Gardiner & Stone 2005, J. Comput. Phys. 205, 509) at the
// same edge: the mean above plus half-cell differences between face values
// and the cell-centred reference EMF F.e[A] of the four cells around the
// edge, each difference taken on the upwind side of the mass flux (rotated
// component 0) through the face it starts from, their mean when that flux is
// zero.  Names: bS/bN the b-faces below/above the edge along c, cW/cE the
// c-faces below/above along b, eSW..eNE the cells (b low/high, c low/high).
template <int A, class T>
__device__ __forceinline__ T edge_emf_upwind(const DevFlux<T>& F, int64_t e, const int64_t (&st)[3]) {
  constexpr int B = (A + 1) % 3, C = (A + 2) % 3;
  const T bS = -F.f[B][5][e - st[C]], bN = -F.f[B][5][e];
  const T cW = F.f[C][6][e - st[B]], cE = F.f[C][6][e];
  const T eSW = F.e[A][e - st[B] - st[C]], eSE = F.e[A][e - st[C]];
  const T eNW = F.e[A][e - st[B]], eNE = F.e[A][e];
  auto upw = [](T flux, T lo, T hi) { return flux > T(0) ? lo : (flux < T(0) ? hi : T(0.5) * (lo + hi)); };
  const T dc_hi = upw(F.f[B][0][e], eNW - cW, eNE - cE);
  const T dc_lo = upw(F.f[B][0][e - st[C]], cW - eSW, cE - eSE);
  const T db_hi = upw(F.f[C][0][e], eSE - bS, eNE - bN);
  const T db_lo = upw(F.f[C][0][e - st[B]], bS - eSW, bN - eNW);
  return T(0.25) * ((bS + bN) + (cW + cE)) + T(0.25) * ((dc_lo - dc_hi) + (db_lo - db_hi));
}

// Edge EMF as the update and the registers read it: the mean from the face
// fluxes, or the upwinded value stored per edge by the EMF kernel.
template <int A, bool UPWIND, class T>
__device__ __forceinline__ T emf_at(const DevFlux<T>& F, int64_t e, const int64_t (&st)[3]) {
  if constexpr (UPWIND) return F.edge[A][e];
  else return edge_emf<A>(F, e, st);
}

// edge_emf_upwind at byte offset b (byte strides sb): identical arithmetic,
// so identical values.
template <int A, class T, class Off>
__device__ __forceinline__ T edge_emf_upwind_b(const DevFlux<T>& F, Off b, const int32_t (&sb)[3]) {
  constexpr int B = (A + 1) % 3, C = (A + 2) % 3;
  const T bS = -ldb(F.f[B][5], b - sb[C]), bN = -ldb(F.f[B][5], b);
  const T cW = ldb(F.f[C][6], b - sb[B]), cE = ldb(F.f[C][6], b);
  const T eSW = ldb(F.e[A], b - sb[B] - sb[C]), eSE = ldb(F.e[A], b - sb[C]);
  const T eNW = ldb(F.e[A], b - sb[B]), eNE = ldb(F.e[A], b);
  auto upw = [](T flux, T lo, T hi) { return flux > T(0) ? lo : (flux < T(0) ? hi : T(0.5) * (lo + hi)); };
  const T dc_hi = upw(ldb(F.f[B][0], b), eNW - cW, eNE - cE);
  const T dc_lo = upw(ldb(F.f[B][0], b - sb[C]), cW - eSW, cE - eSE);
  const T db_hi = upw(ldb(F.f[C][0], b), eSE - bS, eNE - bN);
  const T db_lo = upw(ldb(F.f[C][0], b - sb[B]), bS - eSW, bN - eNW);
  return T(0.25) * ((bS + bN) + (cW + cE)) + T(0.25) * ((dc_lo - dc_hi) + (db_lo - db_hi));
}

// Rotated flux component of direction d that carries lab conserved slot s
// (0 rho, 1..3 momentum, 4 energy, 7 the cell-centred Bz of 2D).
__device__ __forceinline__ int flux_comp(int s, int d) {
  if (s == 0 || s == 4) return s;
  if (s == 7) return d == 0 ? 6 : 5;
  return 1 + ((s - 1) - d + 3) % 3;
}

}  // namespace amr
