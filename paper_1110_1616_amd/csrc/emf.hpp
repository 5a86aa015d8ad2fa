// Edge EMF of constrained transport from stored face fluxes (shared by the
// update kernel and the synchronisation registers so both see the same
// value bit for bit).
#pragma once
#include "amr_internal.hpp"

namespace amr {

// EMF along axis A at the edge whose high-side cell (in the two other axes)
// has element e: the mean of the four adjacent face values, E_A = -F_b(B_c)
// on b-faces and +F_c(B_b) on c-faces (b = A+1, c = A+2; rotated flux
// components 5 = B_t1 and 6 = B_t2).  st: element strides of the grid.
template <int A, class T>
__device__ __forceinline__ T edge_emf(const DevFlux<T>& F, int64_t e, const int64_t (&st)[3]) {
  constexpr int B = (A + 1) % 3, C = (A + 2) % 3;
  T s1 = F.f[B][5][e - st[C]] + F.f[B][5][e];
  T s2 = F.f[C][6][e - st[B]] + F.f[C][6][e];
  return T(0.25) * (s2 - s1);
}

// Rotated flux component of direction d that carries lab conserved slot s
// (0 rho, 1..3 momentum, 4 energy, 7 the cell-centred Bz of 2D).
__device__ __forceinline__ int flux_comp(int s, int d) {
  if (s == 0 || s == 4) return s;
  if (s == 7) return d == 0 ? 6 : 5;
  return 1 + ((s - 1) - d + 3) % 3;
}

}  // namespace amr
