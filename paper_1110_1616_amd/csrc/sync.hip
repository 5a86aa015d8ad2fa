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

// The face and edge registers of every job of a launch cycle in one launch:
// thread t takes entry t - begin of the job whose range holds it, face
// entries first, then edge entries.
template <class T, int NDIM, bool UPWIND>
__global__ __launch_bounds__(256) void k_registers(RegJobs<T> jobs, const GridDesc* __restrict__ grids, DevFlux<T> F,
                                                   const double* __restrict__ dt0p) {
  const double dt0 = dt0p[0];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < jobs.total; t += gridDim.x * blockDim.x) {
    int j = 0;
    while (j + 1 < jobs.n && t >= jobs.j[j + 1].begin) ++j;
    const RegJob<T>& J = jobs.j[j];
    const T dt = T(dt0 / J.dt_div);
    const int i = t - J.begin;
    if (i < J.nf) reg_face<T, NDIM>(J.fe[i], F, J.freg, J.nfreg, J.slot, dt);
    else reg_edge<T, NDIM, UPWIND>(J.ee[i - J.nf], grids, F, J.ereg, J.nereg, J.slot, dt);
  }
}

// Reflux of one uncovered coarse cell.
template <class T, int NDIM>
__device__ __forceinline__ void reflux_one(const RefluxEntry& e, const T* __restrict__ reg, int nreg,
                                           const DevState<T>& U) {
  constexpr int ns = NDIM == 2 ? 6 : 5;
  constexpr int imax = 6;
  {
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

// EMF correction of one copy of an uncovered coarse face.
template <class T>
__device__ __forceinline__ void emffix_one(const EmfFixEntry& e, const T* __restrict__ reg, int nreg,
                                           const DevState<T>& U) {
  constexpr int imax = 4;
  {
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

// Restriction of one covered coarse cell or coarse face copy.
template <class T, int NDIM>
__device__ __forceinline__ void restrict_one(const RestrictEntry& e, const GridDesc* __restrict__ grids,
                                             const DevState<T>& Uf, const DevState<T>& Uc) {
  {
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

// One synchronisation in one launch: threads [0, nr) reflux uncovered
// coarse cells, the next ne correct uncovered coarse faces, the rest
// restrict covered cells and faces.  The three sets of outputs are disjoint
// and none reads another's outputs, so the order inside the launch is free.
template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_sync(const RefluxEntry* __restrict__ rfx, int nr,
                                              const EmfFixEntry* __restrict__ efx, int ne,
                                              const RestrictEntry* __restrict__ rst, int nrs,
                                              const GridDesc* __restrict__ grids, const T* __restrict__ freg,
                                              int nfreg, const T* __restrict__ ereg, int nereg, DevState<T> Uf,
                                              DevState<T> Uc) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nr + ne + nrs; t += gridDim.x * blockDim.x) {
    if (t < nr) reflux_one<T, NDIM>(rfx[t], freg, nfreg, Uc);
    else if (t < nr + ne) emffix_one<T>(efx[t - nr], ereg, nereg, Uc);
    else restrict_one<T, NDIM>(rst[t - nr - ne], grids, Uf, Uc);
  }
}

}  // namespace

template <class T>
void launch_register_jobs(int ndim, const GridDesc* grids, const RegJobs<T>& jobs, DevFlux<T> F, const double* dt0,
                          bool upwind_emf, hipStream_t s) {
  if (jobs.total <= 0) return;
#define AMR_REGS(ND, U) \
  hipLaunchKernelGGL((k_registers<T, ND, U>), dim3(blocks_for(jobs.total)), dim3(256), 0, s, jobs, grids, F, dt0)
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
  const int n = t.n_reflux + t.n_emffix + t.n_restrict;
  if (n <= 0) return;
#define AMR_SYNC(ND)                                                                                              \
  hipLaunchKernelGGL((k_sync<T, ND>), dim3(blocks_for(n)), dim3(256), 0, s, t.d_reflux, t.n_reflux, t.d_emffix,   \
                     t.n_emffix, t.d_restrict, t.n_restrict, grids, freg, t.nfreg, ereg, t.nereg, Uf, Uc)
  if (ndim == 3) AMR_SYNC(3);
  else AMR_SYNC(2);
#undef AMR_SYNC
}

template void launch_register_jobs<float>(int, const GridDesc*, const RegJobs<float>&, DevFlux<float>,
                                          const double*, bool, hipStream_t);
template void launch_register_jobs<double>(int, const GridDesc*, const RegJobs<double>&, DevFlux<double>,
                                           const double*, bool, hipStream_t);
template void launch_sync<float>(int, int, const GridDesc*, const SyncTables&, const float*, const float*,
                                 DevState<float>, DevState<float>, hipStream_t);
template void launch_sync<double>(int, int, const GridDesc*, const SyncTables&, const double*, const double*,
                                  DevState<double>, DevState<double>, hipStream_t);

}  // namespace amr
