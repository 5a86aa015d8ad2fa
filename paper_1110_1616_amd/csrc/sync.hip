// Level synchronisation kernels for gfx950: coarse/fine registers, reflux,
// EMF correction and restriction (the (S)ynchronise and (R)estrict steps of
// the paper's level cycle, Sec. 4).  Every kernel is a gather over tables
// built by the host runtime: one thread per register, cell or face copy, so
// each output has exactly one writer and no atomics are used.
#include "amr_internal.hpp"
#include "emf.hpp"
#include "sync_internal.hpp"

namespace amr {

namespace {

inline int blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65535) b = 65535;
  return (int)(b < 1 ? 1 : b);
}

// The refinement ratio of a synchronised hierarchy (the runtime refuses any
// other): the gathers below are unrolled over it, so each thread issues all
// of its loads before the first use and sums them in the order the
// definition states (one memory latency per thread instead of one per term).
constexpr int kR = 2;

// Coarse/fine registers of one substep, both kinds in one launch: entries
// [0, nf) are face registers, [nf, nf + ne) edge registers.
template <class T, int NDIM>
__device__ __forceinline__ void reg_face(const FaceRegEntry& e, const DevFlux<T>& F, T* __restrict__ reg, int nreg,
                                         int slot, T dt) {
  constexpr int ns = NDIM == 2 ? 6 : 5;
  constexpr int nmax = NDIM == 3 ? kR * kR : kR;
  T* out = reg + ((int64_t)slot * nreg + e.reg) * 6;
  T v[ns][nmax];
#pragma unroll
  for (int q = 0; q < ns; ++q) {
    const int s = q < 5 ? q : 7;
    const T* f = F.f[e.d][flux_comp(s, e.d)];
#pragma unroll
    for (int i = 0; i < nmax; ++i) v[q][i] = i < e.n ? f[e.e[i]] : T(0);
  }
#pragma unroll
  for (int q = 0; q < ns; ++q) {
    T m = T(0);
#pragma unroll
    for (int i = 0; i < nmax; ++i)
      if (i < e.n) m += v[q][i];
    out[q] = dt * (m / T(e.n));
  }
}

template <class T, int NDIM, bool UPWIND>
__device__ __forceinline__ void reg_edge(const EdgeRegEntry& e, const GridDesc* __restrict__ grids,
                                         const DevFlux<T>& F, T* __restrict__ reg, int nreg, int slot, T dt) {
  const GridDesc G = grids[e.grid];
  const int64_t st[3] = {1, G.P[0], NDIM == 3 ? (int64_t)G.P[0] * G.P[1] : 0};
  T v[kR];
#pragma unroll
  for (int i = 0; i < kR; ++i) {
    v[i] = T(0);
    if (i < e.n) {
      if (e.a == 0) v[i] = emf_at<0, UPWIND>(F, e.e[i], st);
      else if (e.a == 1) v[i] = emf_at<1, UPWIND>(F, e.e[i], st);
      else v[i] = emf_at<2, UPWIND>(F, e.e[i], st);
    }
  }
  T m = T(0);
#pragma unroll
  for (int i = 0; i < kR; ++i)
    if (i < e.n) m += v[i];
  reg[(int64_t)slot * nreg + e.reg] = dt * (m / T(e.n));
}

// The face and edge registers of one fine step in one launch: threads
// [0, nf) take face entries, [nf, nf + ne) edge entries.
template <class T, int NDIM, bool UPWIND>
__global__ __launch_bounds__(256) void k_registers(const FaceRegEntry* __restrict__ fe, int nf,
                                                   const EdgeRegEntry* __restrict__ ee, int ne,
                                                   const GridDesc* __restrict__ grids, DevFlux<T> F,
                                                   T* __restrict__ freg, int nfreg, T* __restrict__ ereg, int nereg,
                                                   int slot, const double* __restrict__ dt0p, double dt_div) {
  const T dt = T(dt0p[0] / dt_div);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nf + ne; t += gridDim.x * blockDim.x) {
    if (t < nf) reg_face<T, NDIM>(fe[t], F, freg, nfreg, slot, dt);
    else reg_edge<T, NDIM, UPWIND>(ee[t - nf], grids, F, ereg, nereg, slot, dt);
  }
}

template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_reflux(const RefluxEntry* __restrict__ ent, int n, const T* __restrict__ reg,
                                                int nreg, DevState<T> U) {
  constexpr int ns = NDIM == 2 ? 6 : 5;
  constexpr int imax = 6;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const RefluxEntry e = ent[t];
#pragma unroll
    for (int q = 0; q < ns; ++q) {
      const int s = q < 5 ? q : 7;
      T acc = U.f[s][e.cell];
      T rc[imax], rf[imax][kR];
#pragma unroll
      for (int i = 0; i < imax; ++i) {
        rc[i] = T(0);
#pragma unroll
        for (int k = 0; k < kR; ++k) rf[i][k] = T(0);
        if (i < e.n) {
          const T* r = reg + (int64_t)e.reg[i] * 6 + q;
          rc[i] = r[0];
#pragma unroll
          for (int k = 0; k < kR; ++k) rf[i][k] = r[(int64_t)(k + 1) * nreg * 6];
        }
      }
#pragma unroll
      for (int i = 0; i < imax; ++i)
        if (i < e.n) {
          T fine = T(0);
#pragma unroll
          for (int k = 0; k < kR; ++k) fine += rf[i][k];
          const T delta = rc[i] - fine;
          acc += T(e.coef[i]) * delta;
        }
      U.f[s][e.cell] = acc;
    }
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_emffix(const EmfFixEntry* __restrict__ ent, int n, const T* __restrict__ reg,
                                                int nreg, DevState<T> U) {
  constexpr int imax = 4;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const EmfFixEntry e = ent[t];
    T rc[imax], rf[imax][kR];
#pragma unroll
    for (int i = 0; i < imax; ++i) {
      rc[i] = T(0);
#pragma unroll
      for (int k = 0; k < kR; ++k) rf[i][k] = T(0);
      if (i < e.n) {
        const T* r = reg + e.reg[i];
        rc[i] = r[0];
#pragma unroll
        for (int k = 0; k < kR; ++k) rf[i][k] = r[(int64_t)(k + 1) * nreg];
      }
    }
    T corr = T(0);
#pragma unroll
    for (int i = 0; i < imax; ++i)
      if (i < e.n) {
        T fine = T(0);
#pragma unroll
        for (int k = 0; k < kR; ++k) fine += rf[i][k];
        corr += T(e.coef[i]) * (fine - rc[i]);
      }
    U.f[5 + e.d][e.face] -= corr;
  }
}

template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_restrict(const RestrictEntry* __restrict__ ent, int n,
                                                  const GridDesc* __restrict__ grids, DevState<T> Uf,
                                                  DevState<T> Uc) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const RestrictEntry e = ent[t];
    const GridDesc G = grids[e.fgrid];
    const int64_t st[3] = {1, G.P[0], (int64_t)G.P[0] * G.P[1]};
    if (e.d < 0) {
      constexpr int ns = NDIM == 2 ? 6 : 5;
      constexpr int nz = NDIM == 3 ? kR : 1;
      T v[ns][nz * kR * kR];
#pragma unroll
      for (int q = 0; q < ns; ++q) {
        const int s = q < 5 ? q : 7;
#pragma unroll
        for (int kz = 0; kz < nz; ++kz)
#pragma unroll
          for (int ky = 0; ky < kR; ++ky)
#pragma unroll
            for (int kx = 0; kx < kR; ++kx)
              v[q][(kz * kR + ky) * kR + kx] = Uf.f[s][e.src + kx + ky * st[1] + kz * st[2]];
      }
#pragma unroll
      for (int q = 0; q < ns; ++q) {
        const int s = q < 5 ? q : 7;
        T m = T(0);
#pragma unroll
        for (int c = 0; c < nz * kR * kR; ++c) m += v[q][c];
        Uc.f[s][e.dst] = m / T(kR * kR * nz);
      }
    } else {
      const int d = e.d;
      const int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
      const int n1 = a1 < NDIM ? kR : 1, n2 = a2 < NDIM ? kR : 1;
      T v[kR * kR];
#pragma unroll
      for (int i1 = 0; i1 < kR; ++i1)
#pragma unroll
        for (int i2 = 0; i2 < kR; ++i2)
          v[i1 * kR + i2] = (i1 < n1 && i2 < n2) ? Uf.f[5 + d][e.src + i1 * st[a1] + i2 * st[a2]] : T(0);
      T m = T(0);
#pragma unroll
      for (int i1 = 0; i1 < kR; ++i1)
#pragma unroll
        for (int i2 = 0; i2 < kR; ++i2)
          if (i1 < n1 && i2 < n2) m += v[i1 * kR + i2];
      Uc.f[5 + d][e.dst] = m / T(n1 * n2);
    }
  }
}

}  // namespace

template <class T>
void launch_registers(int ndim, const GridDesc* grids, const FaceRegEntry* fe, int nf, const EdgeRegEntry* ee, int ne,
                      DevFlux<T> F, T* freg, T* ereg, int nfreg, int nereg, int slot, const double* dt0,
                      double dt_div, bool upwind_emf, hipStream_t s) {
  if (nf + ne <= 0) return;
#define AMR_REGS(ND, U)                                                                                            \
  hipLaunchKernelGGL((k_registers<T, ND, U>), dim3(blocks_for((int64_t)nf + ne)), dim3(256), 0, s, fe, nf, ee, ne, \
                     grids, F, freg, nfreg, ereg, nereg, slot, dt0, dt_div)
  if (ndim == 3) {
    if (upwind_emf) AMR_REGS(3, true);
    else AMR_REGS(3, false);
  } else {
    if (upwind_emf) AMR_REGS(2, true);
    else AMR_REGS(2, false);
  }
#undef AMR_REGS
}

template <class T>
void launch_sync(int ndim, int R, const GridDesc* grids, const SyncTables& t, const T* freg, const T* ereg,
                 DevState<T> Uf, DevState<T> Uc, hipStream_t s) {
  (void)R;  // the kernels are unrolled over kR; the caller checks R == kR
  if (t.n_reflux > 0) {
    if (ndim == 3)
      hipLaunchKernelGGL((k_reflux<T, 3>), dim3(blocks_for(t.n_reflux)), dim3(256), 0, s, t.d_reflux, t.n_reflux, freg,
                         t.nfreg, Uc);
    else
      hipLaunchKernelGGL((k_reflux<T, 2>), dim3(blocks_for(t.n_reflux)), dim3(256), 0, s, t.d_reflux, t.n_reflux, freg,
                         t.nfreg, Uc);
  }
  if (t.n_emffix > 0)
    hipLaunchKernelGGL((k_emffix<T>), dim3(blocks_for(t.n_emffix)), dim3(256), 0, s, t.d_emffix, t.n_emffix, ereg,
                       t.nereg, Uc);
  if (t.n_restrict > 0) {
    if (ndim == 3)
      hipLaunchKernelGGL((k_restrict<T, 3>), dim3(blocks_for(t.n_restrict)), dim3(256), 0, s, t.d_restrict,
                         t.n_restrict, grids, Uf, Uc);
    else
      hipLaunchKernelGGL((k_restrict<T, 2>), dim3(blocks_for(t.n_restrict)), dim3(256), 0, s, t.d_restrict,
                         t.n_restrict, grids, Uf, Uc);
  }
}

template void launch_registers<float>(int, const GridDesc*, const FaceRegEntry*, int, const EdgeRegEntry*, int,
                                      DevFlux<float>, float*, float*, int, int, int, const double*, double, bool,
                                      hipStream_t);
template void launch_registers<double>(int, const GridDesc*, const FaceRegEntry*, int, const EdgeRegEntry*, int,
                                       DevFlux<double>, double*, double*, int, int, int, const double*, double, bool,
                                       hipStream_t);
template void launch_sync<float>(int, int, const GridDesc*, const SyncTables&, const float*, const float*,
                                 DevState<float>, DevState<float>, hipStream_t);
template void launch_sync<double>(int, int, const GridDesc*, const SyncTables&, const double*, const double*,
                                  DevState<double>, DevState<double>, hipStream_t);

}  // namespace amr
