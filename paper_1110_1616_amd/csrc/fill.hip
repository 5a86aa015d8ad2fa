// Ghost-band fill, CFL reduction and state marshalling kernels for gfx950.
//
// Band fills are gathers over precomputed element maps built by the host
// runtime at hierarchy creation: a copy map (same-level interiors, periodic
// images and outflow boundaries) and, for FULL fills above level 0,
// prolongation maps that name the coarse cell or face each band element is
// reconstructed from.  Every band element has exactly one writer.
#include <algorithm>

#include "amr_internal.hpp"
#include "fill_internal.hpp"
#include "frozen.hpp"
#include "mhd_device.hpp"

namespace amr {

namespace {

// ------------------------------------------------------------------ copies
// entries [0, nc[0]) cells, then x-, y-, z-face entries.
template <class T, int NDIM>
__device__ __forceinline__ void copy_one(int t, const CopyEntry& e, int4 cls, const DevState<T>& U) {
  {
    if (t < cls.x) {
      U.f[0][e.dst] = U.f[0][e.src];
      U.f[1][e.dst] = U.f[1][e.src];
      U.f[2][e.dst] = U.f[2][e.src];
      U.f[3][e.dst] = U.f[3][e.src];
      U.f[4][e.dst] = U.f[4][e.src];
      if (NDIM == 2) U.f[7][e.dst] = U.f[7][e.src];
    } else if (t < cls.y) {
      U.f[5][e.dst] = U.f[5][e.src];
    } else if (t < cls.z) {
      U.f[6][e.dst] = U.f[6][e.src];
    } else {
      U.f[7][e.dst] = U.f[7][e.src];
    }
  }
}

// -------------------------------------------------------------- prolongation
// Cells: U_f = U_c + sum_d (s_d / 4) minmod(U_c - U_{c-e_d}, U_{c+e_d} - U_c)
// for the conserved cell fields (R = 2, s_d = +-1 the fine half).
template <class T, int NDIM>
__device__ __forceinline__ void prolong_cell_one(const ProlongEntry& e, const GridDesc* __restrict__ grids,
                                                 const DevState<T>& Us, const DevState<T>& Ud) {
  {
    const GridDesc P = grids[e.pgrid];
    const int64_t st[3] = {1, P.P[0], (int64_t)P.P[0] * P.P[1]};
    const int nfield = NDIM == 2 ? 6 : 5;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      if (q >= nfield) break;
      const int s = q < 5 ? q : 7;
      const T* f = Us.f[s];
      const T c = f[e.src];
      T v = c;
#pragma unroll
      for (int d = 0; d < NDIM; ++d) {
        T sl = limiter_minmod(c - f[e.src - st[d]], f[e.src + st[d]] - c);
        const T sg = ((e.code >> d) & 1) ? T(0.25) : T(-0.25);
        v += sg * sl;
      }
      Ud.f[s][e.dst] = v;
    }
  }
}

// Faces: divergence-free reconstruction (Balsara 2001) inside each coarse
// cell, R = 2.  code bits: 0-1 face axis d; 2 = fine face lies inside the
// coarse cell (mid-plane) rather than on a coarse face; 3,4 = fine half
// (+1 if set) along the transverse axes d+1, d+2.  e.src is the coarse
// element of the coarse face (on-face) or of the coarse cell (mid-plane).
template <class T, int NDIM>
__device__ __forceinline__ T tslope(const T* f, int64_t e, int64_t s) {
  const T c = f[e];
  return limiter_minmod(c - f[e - s], f[e + s] - c);
}

template <class T, int NDIM>
__device__ __forceinline__ void prolong_face_one(const ProlongEntry& e, const GridDesc* __restrict__ grids,
                                                 const DevState<T>& Us, const DevState<T>& Ud, const Phys& ph) {
  {
    const GridDesc P = grids[e.pgrid];
    const int64_t st[3] = {1, P.P[0], (int64_t)P.P[0] * P.P[1]};
    const int d = e.code & 3;
    const bool mid = (e.code >> 2) & 1;
    const T s1 = ((e.code >> 3) & 1) ? T(1) : T(-1);
    const T s2 = ((e.code >> 4) & 1) ? T(1) : T(-1);
    const int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
    const bool act1 = a1 < NDIM, act2 = a2 < NDIM;
    const T* fd = Us.f[5 + d];
    T v;
    if (!mid) {
      v = fd[e.src];
      if (act1) v += T(0.25) * s1 * tslope<T, NDIM>(fd, e.src, st[a1]);
      if (act2) v += T(0.25) * s2 * tslope<T, NDIM>(fd, e.src, st[a2]);
    } else {
      // coarse cell widths of the parent level
      double rl = 1.0;
      for (int l = 0; l < P.level; ++l) rl *= (double)ph.ratio;
      const T wdt[3] = {T(ph.dx0[0] / rl), T(ph.dx0[1] / rl), T(NDIM == 3 ? ph.dx0[2] / rl : 1.0)};
      const int64_t lo = e.src, hi = e.src + st[d];
      const T bm = fd[lo], bp = fd[hi];
      T ay = T(0), az = T(0);
      if (act1) ay = T(0.25) * (tslope<T, NDIM>(fd, hi, st[a1]) + tslope<T, NDIM>(fd, lo, st[a1]));
      if (act2) az = T(0.25) * (tslope<T, NDIM>(fd, hi, st[a2]) + tslope<T, NDIM>(fd, lo, st[a2]));
      // a_dd = -(w_d / 2) sum_t (slope_d(B_t^+) - slope_d(B_t^-)) / (4 w_t)
      T add = T(0);
#pragma unroll
      for (int tt = 1; tt <= 2; ++tt) {
        const int ta = (d + tt) % 3;
        if (ta >= NDIM) continue;
        const T* ft = Us.f[5 + ta];
        const T sp = tslope<T, NDIM>(ft, e.src + st[ta], st[d]);
        const T sm = tslope<T, NDIM>(ft, e.src, st[d]);
        add += T(0.25) * (sp - sm) / wdt[ta];
      }
      add *= -T(0.5) * wdt[d];
      const T a0 = T(0.5) * (bp + bm) - add;
      v = a0 + T(0.5) * s1 * ay + T(0.5) * s2 * az;
    }
    Ud.f[5 + d][e.dst] = v;
  }
}

template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_copy(const CopyEntry* __restrict__ ent, int n, int4 cls, DevState<T> U) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) copy_one<T, NDIM>(t, ent[t], cls, U);
}

template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_prolong_cells(const ProlongEntry* __restrict__ ent, int n,
                                                       const GridDesc* __restrict__ grids, DevState<T> Us,
                                                       DevState<T> Ud) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    prolong_cell_one<T, NDIM>(ent[t], grids, Us, Ud);
}

template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_prolong_faces(const ProlongEntry* __restrict__ ent, int n,
                                                       const GridDesc* __restrict__ grids, DevState<T> Us,
                                                       DevState<T> Ud, Phys ph) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    prolong_face_one<T, NDIM>(ent[t], grids, Us, Ud, ph);
}

// A full band fill in one launch: threads [0, nc) copy same-level band
// elements, the next npc prolong band cells from the parent level, the rest
// band faces.  The three write disjoint band elements, the copies read the
// level's interiors and the prolongations the parent level only, so the
// order inside the launch is free.
template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_fill(const CopyEntry* __restrict__ cp, int nc, int4 cls,
                                              const ProlongEntry* __restrict__ pc, int npc,
                                              const ProlongEntry* __restrict__ pf, int npf,
                                              const GridDesc* __restrict__ grids, DevState<T> Us, DevState<T> Ud,
                                              Phys ph) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nc + npc + npf; t += gridDim.x * blockDim.x) {
    if (t < nc) copy_one<T, NDIM>(t, cp[t], cls, Ud);
    else if (t < nc + npc) prolong_cell_one<T, NDIM>(pc[t - nc], grids, Us, Ud);
    else prolong_face_one<T, NDIM>(pf[t - nc - npc], grids, Us, Ud, ph);
  }
}

// ------------------------------------------------------------------- CFL
// Max over interior cells of sum_d (|v_d| + c_f,d) / dx0_d; blocks stride
// over (grid, plane, rows) items.  Wavefront max by lane exchange, then LDS
// across the four waves, then one atomic max per block on the bit pattern of
// the non-negative double (order independent, hence deterministic).
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_cfl(const GridDesc* __restrict__ grids, const int4* __restrict__ items,
                                             int nitems, DevState<T> S0, DevState<T> S1, uint32_t parity, Phys ph,
                                             unsigned long long* acc, ErrBlock* err) {
  __shared__ double red[4];
  const T gam = T(ph.gamma);
  const T gm1 = gam - T(1);
  // a few blocks per CU stride over the items; each thread keeps its
  // running max and the block reduces once at the end (one atomic per block)
  double m = 0.0;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    // item: (grid, plane k, first row j0, rows)
    const int4 item = items[it];
    const GridDesc G = grids[item.x];
    const DevState<T> U = ((parity >> G.level) & 1u) ? S1 : S0;
    const int k = item.y;
    const int64_t sy = G.P[0], sz = (int64_t)G.P[0] * G.P[1];
    const int64_t base = G.off + G.g + G.g * sy + (NDIM == 3 ? (int64_t)G.g * sz : 0) + (int64_t)k * sz +
                         (int64_t)item.z * sy;
    const int ncell = G.n[0] * item.w;
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
      const int i = c % G.n[0], j = c / G.n[0];
      const int64_t e = base + i + j * sy;
      T u[8], w[8];
      u[0] = U.f[0][e];
      u[1] = U.f[1][e];
      u[2] = U.f[2][e];
      u[3] = U.f[3][e];
      u[4] = U.f[4][e];
      u[5] = T(0.5) * (U.f[5][e] + U.f[5][e + 1]);
      u[6] = T(0.5) * (U.f[6][e] + U.f[6][e + sy]);
      u[7] = NDIM == 3 ? T(0.5) * (U.f[7][e] + U.f[7][e + sz]) : U.f[7][e];
      to_primitive(u, w, gm1);
      if (!(w[0] > T(0)) || !(w[4] > T(0))) {
        unsigned old = atomicOr(&err->flags, 1u);
        if ((old & 1u) == 0u) atomicExch((unsigned long long*)&err->first_bad, (unsigned long long)e);
      }
      const T b2 = w[5] * w[5] + w[6] * w[6] + w[7] * w[7];
      double s = 0.0;
#pragma unroll
      for (int d = 0; d < NDIM; ++d) {
        T cf = fast_magnetosonic(w[0], w[4], b2, w[5 + d], gam);
        s += (double)((dabs(w[1 + d]) + cf) / T(ph.dx0[d]));
      }
      m = fmax(m, s);
    }
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(acc, (unsigned long long)__double_as_longlong(b));
  }
}

__global__ void k_dt_finalize(unsigned long long* acc, double cfl, double* dt0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double m = __longlong_as_double((long long)*acc);
    dt0[0] = cfl / m;
    *acc = 0ull;
  }
}

// ------------------------------------------------------------ marshalling
template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_load_prim(GridDesc G, const double* __restrict__ r,
                                                   const double* __restrict__ vx, const double* __restrict__ vy,
                                                   const double* __restrict__ vz, const double* __restrict__ p,
                                                   const double* __restrict__ bx, const double* __restrict__ by,
                                                   const double* __restrict__ bz, DevState<T> U, double gamma) {
  const int nx = G.n[0], ny = G.n[1], nz = NDIM == 3 ? G.n[2] : 1;
  const int64_t sy = G.P[0], sz = (int64_t)G.P[0] * G.P[1];
  const int64_t base = G.off + G.g + G.g * sy + (NDIM == 3 ? (int64_t)G.g * sz : 0);
  const int64_t total = (int64_t)nx * ny * nz;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % nx);
    const int j = (int)((t / nx) % ny);
    const int k = (int)(t / ((int64_t)nx * ny));
    const int64_t e = base + i + j * sy + (int64_t)k * sz;
    // interior-layout indices of this cell's low faces and the high ones
    const int64_t ibx = ((int64_t)k * ny + j) * (nx + 1) + i;
    const int64_t iby = ((int64_t)k * (ny + 1) + j) * nx + i;
    const int64_t ibz = ((int64_t)k * ny + j) * nx + i;
    const double bxl = bx[ibx], bxh = bx[ibx + 1];
    const double byl = by[iby], byh = by[iby + nx];
    const double bzl = bz[ibz], bzh = NDIM == 3 ? bz[ibz + (int64_t)nx * ny] : bzl;
    const double bcx = 0.5 * (bxl + bxh), bcy = 0.5 * (byl + byh), bcz = NDIM == 3 ? 0.5 * (bzl + bzh) : bzl;
    const double rho = r[t];
    const double v2 = vx[t] * vx[t] + vy[t] * vy[t] + vz[t] * vz[t];
    const double en = p[t] / (gamma - 1.0) + 0.5 * rho * v2 + 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz);
    U.f[0][e] = T(rho);
    U.f[1][e] = T(rho * vx[t]);
    U.f[2][e] = T(rho * vy[t]);
    U.f[3][e] = T(rho * vz[t]);
    U.f[4][e] = T(en);
    U.f[5][e] = T(bxl);
    U.f[6][e] = T(byl);
    U.f[7][e] = T(bzl);
    if (i == nx - 1) U.f[5][e + 1] = T(bxh);
    if (j == ny - 1) U.f[6][e + sy] = T(byh);
    if (NDIM == 3 && k == nz - 1) U.f[7][e + sz] = T(bzh);
  }
}

template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_store(GridDesc G, DevState<T> U, double* o0, double* o1, double* o2,
                                               double* o3, double* o4, double* o5, double* o6, double* o7) {
  const int nx = G.n[0], ny = G.n[1], nz = NDIM == 3 ? G.n[2] : 1;
  const int64_t sy = G.P[0], sz = (int64_t)G.P[0] * G.P[1];
  const int64_t base = G.off + G.g + G.g * sy + (NDIM == 3 ? (int64_t)G.g * sz : 0);
  // iterate over the (nx+1)(ny+1)(nz+1) superset and write what each array holds
  const int ex = nx + 1, ey = ny + 1, ez = nz + (NDIM == 3 ? 1 : 0);
  const int64_t total = (int64_t)ex * ey * ez;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % ex);
    const int j = (int)((t / ex) % ey);
    const int k = (int)(t / ((int64_t)ex * ey));
    const int64_t e = base + i + j * sy + (int64_t)k * sz;
    const bool ci = i < nx, cj = j < ny, ck = k < nz;
    if (ci && cj && ck) {
      const int64_t c = ((int64_t)k * ny + j) * nx + i;
      o0[c] = (double)U.f[0][e];
      o1[c] = (double)U.f[1][e];
      o2[c] = (double)U.f[2][e];
      o3[c] = (double)U.f[3][e];
      o4[c] = (double)U.f[4][e];
      if (NDIM == 2) o7[c] = (double)U.f[7][e];
    }
    if (cj && ck) o5[((int64_t)k * ny + j) * (nx + 1) + i] = (double)U.f[5][e];
    if (ci && ck) o6[((int64_t)k * (ny + 1) + j) * nx + i] = (double)U.f[6][e];
    if (NDIM == 3 && ci && cj) o7[((int64_t)k * ny + j) * nx + i] = (double)U.f[7][e];
  }
}

inline int blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65535) b = 65535;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

template <class T>
void launch_copy(int ndim, const CopyEntry* ent, int n, int4 cls, DevState<T> U, hipStream_t s) {
  if (n <= 0) return;
  if (ndim == 3)
    hipLaunchKernelGGL((k_copy<T, 3>), dim3(blocks_for(n)), dim3(256), 0, s, ent, n, cls, U);
  else
    hipLaunchKernelGGL((k_copy<T, 2>), dim3(blocks_for(n)), dim3(256), 0, s, ent, n, cls, U);
}

template <class T>
void launch_prolong(int ndim, const ProlongEntry* cells, int ncells, const ProlongEntry* faces, int nfaces,
                    const GridDesc* grids, DevState<T> Us, DevState<T> Ud, Phys ph, hipStream_t s) {
  if (ncells > 0) {
    if (ndim == 3)
      hipLaunchKernelGGL((k_prolong_cells<T, 3>), dim3(blocks_for(ncells)), dim3(256), 0, s, cells, ncells, grids, Us,
                         Ud);
    else
      hipLaunchKernelGGL((k_prolong_cells<T, 2>), dim3(blocks_for(ncells)), dim3(256), 0, s, cells, ncells, grids, Us,
                         Ud);
  }
  if (nfaces > 0) {
    if (ndim == 3)
      hipLaunchKernelGGL((k_prolong_faces<T, 3>), dim3(blocks_for(nfaces)), dim3(256), 0, s, faces, nfaces, grids, Us,
                         Ud, ph);
    else
      hipLaunchKernelGGL((k_prolong_faces<T, 2>), dim3(blocks_for(nfaces)), dim3(256), 0, s, faces, nfaces, grids, Us,
                         Ud, ph);
  }
}

template <class T>
void launch_fill_full(int ndim, const CopyEntry* cp, int nc, int4 cls, const ProlongEntry* cells, int ncells,
                      const ProlongEntry* faces, int nfaces, const GridDesc* grids, DevState<T> Us, DevState<T> Ud,
                      Phys ph, hipStream_t s) {
  const int64_t n = (int64_t)nc + ncells + nfaces;
  if (n <= 0) return;
  if (ndim == 3)
    hipLaunchKernelGGL((k_fill<T, 3>), dim3(blocks_for(n)), dim3(256), 0, s, cp, nc, cls, cells, ncells, faces, nfaces,
                       grids, Us, Ud, ph);
  else
    hipLaunchKernelGGL((k_fill<T, 2>), dim3(blocks_for(n)), dim3(256), 0, s, cp, nc, cls, cells, ncells, faces, nfaces,
                       grids, Us, Ud, ph);
}

constexpr int kCflBlocks = 2048;  // 8 per CU on 256 CUs

template <class T>
void launch_cfl(int ndim, const GridDesc* grids, const int4* items, int nitems, DevState<T> S0, DevState<T> S1,
                uint32_t parity, Phys ph, unsigned long long* acc, ErrBlock* err, double cfl, double* dt0,
                hipStream_t s) {
  if (nitems > 0) {
    if (ndim == 3)
      hipLaunchKernelGGL((k_cfl<T, 3>), dim3(std::min(nitems, kCflBlocks)), dim3(256), 0, s, grids, items, nitems, S0,
                         S1, parity, ph, acc, err);
    else
      hipLaunchKernelGGL((k_cfl<T, 2>), dim3(std::min(nitems, kCflBlocks)), dim3(256), 0, s, grids, items, nitems, S0,
                         S1, parity, ph, acc, err);
  }
  hipLaunchKernelGGL(k_dt_finalize, dim3(1), dim3(64), 0, s, acc, cfl, dt0);
}

template <class T>
void launch_load_prim(int ndim, const GridDesc& G, const double* const* prim, const double* const* b,
                      DevState<T> U, double gamma, hipStream_t s) {
  int64_t n = (int64_t)G.n[0] * G.n[1] * (ndim == 3 ? G.n[2] : 1);
  if (ndim == 3)
    hipLaunchKernelGGL((k_load_prim<T, 3>), dim3(blocks_for(n)), dim3(256), 0, s, G, prim[0], prim[1], prim[2],
                       prim[3], prim[4], b[0], b[1], b[2], U, gamma);
  else
    hipLaunchKernelGGL((k_load_prim<T, 2>), dim3(blocks_for(n)), dim3(256), 0, s, G, prim[0], prim[1], prim[2],
                       prim[3], prim[4], b[0], b[1], b[2], U, gamma);
}

template <class T>
void launch_store(int ndim, const GridDesc& G, DevState<T> U, double* const* out, hipStream_t s) {
  int64_t n = (int64_t)(G.n[0] + 1) * (G.n[1] + 1) * (ndim == 3 ? G.n[2] + 1 : 1);
  if (ndim == 3)
    hipLaunchKernelGGL((k_store<T, 3>), dim3(blocks_for(n)), dim3(256), 0, s, G, U, out[0], out[1], out[2], out[3],
                       out[4], out[5], out[6], out[7]);
  else
    hipLaunchKernelGGL((k_store<T, 2>), dim3(blocks_for(n)), dim3(256), 0, s, G, U, out[0], out[1], out[2], out[3],
                       out[4], out[5], out[6], out[7]);
}

#define AMR_INST(T)                                                                                              \
  template void launch_copy<T>(int, const CopyEntry*, int, int4, DevState<T>, hipStream_t);                       \
  template void launch_prolong<T>(int, const ProlongEntry*, int, const ProlongEntry*, int, const GridDesc*,       \
                                  DevState<T>, DevState<T>, Phys, hipStream_t);                                   \
  template void launch_fill_full<T>(int, const CopyEntry*, int, int4, const ProlongEntry*, int,                   \
                                    const ProlongEntry*, int, const GridDesc*, DevState<T>, DevState<T>, Phys,    \
                                    hipStream_t);                                                                 \
  template void launch_cfl<T>(int, const GridDesc*, const int4*, int, DevState<T>, DevState<T>, uint32_t, Phys,   \
                              unsigned long long*, ErrBlock*, double, double*, hipStream_t);                      \
  template void launch_load_prim<T>(int, const GridDesc&, const double* const*, const double* const*,            \
                                    DevState<T>, double, hipStream_t);                                            \
  template void launch_store<T>(int, const GridDesc&, DevState<T>, double* const*, hipStream_t);
AMR_INST(float)
AMR_INST(double)
#undef AMR_INST
template void launch_copy<FrozenD>(int, const CopyEntry*, int, int4, DevState<FrozenD>, hipStream_t);
template void launch_copy<FrozenF>(int, const CopyEntry*, int, int4, DevState<FrozenF>, hipStream_t);

}  // namespace amr
