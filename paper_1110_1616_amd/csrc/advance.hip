// Patch advance kernels for gfx950: the hot path of the hyperbolic step.
//
// One substep of a set of grids is two launches over a batched work list:
//   k_flux   - per 16x16-thread column tile marching along z: primitive
//              recovery, minmod slopes, Hancock half-step and HLLD fluxes on
//              the tile's faces (a wave64 holds four 16-cell rows; x is the
//              fastest index so global loads and stores are coalesced);
//   k_update - conservative update of cells and CT update of faces from the
//              face fluxes, with the edge EMFs formed from them.
// Work lists hold tiles of any number of grids of any level; the kernels
// read each tile's grid descriptor, so one launch covers every grid that
// steps in a launch cycle.
#include <algorithm>
#include <type_traits>

#include "advance_common.hpp"
#include "launch_common.hpp"
#include "amr_internal.hpp"
#include "emf.hpp"
#include "frozen.hpp"
#include "mhd_device.hpp"

namespace amr {

namespace {

template <class T, int NDIM, bool PERSIST, bool UPWIND>
__global__ __launch_bounds__(256) void k_flux(const GridDesc* __restrict__ grids, const FluxItem* __restrict__ items,
                                              int nitems, DevState<T> S0, DevState<T> S1, uint32_t parity,
                                              DevFlux<T> F, const double* __restrict__ dt0p, Phys ph, ErrBlock* err,
                                              WorkQueue* q, bool xcd, int claim) {
  __shared__ T sW[8][kMaxPlane];
  __shared__ int s_claim[2], s_c;
  if (threadIdx.x == 0) s_c = 0;
  __shared__ T sX[7][256];
  __shared__ T sY[7][256];

  const int tid = threadIdx.x;
  const T gam = T(ph.gamma);
  const T gm1 = gam - T(1);

  ItemRange rng = first_claim<PERSIST>(nitems, claim, xcd);
  for (;;) {
    const int it = next_item<PERSIST>(rng, nitems, claim, q, s_claim, &s_c, xcd);
    if (it < 0) break;
    const FluxItem item = items[it];
    const GridDesc G = grids[item.grid];
    // each level's current data lives in S0 or S1 (bit `level` of parity)
    const DevState<T> U = ((parity >> G.level) & 1u) ? S1 : S0;
    const Idx<NDIM> ix(G);  // element index, for error reports only
    const IdxB<NDIM, T> bx(G);
    const int gv = item.gv;
    const int cl = -gv + 1;
    const int chx = G.n[0] + gv - 1, chy = G.n[1] + gv - 1;
    const int wlo = -gv, whix = G.n[0] + gv, whiy = G.n[1] + gv;  // valid input cells [wlo, whi)
    const int x0 = item.x0, y0 = item.y0;
    const int tw = item.tw, th = 256 / tw, kW = tw + 2;
    const int tx = tid % tw, ty = tid / tw;
    const bool live = ty < th;
    const int cx = x0 - 1 + tx, cy = y0 - 1 + ty;
    const bool act = live && cx >= cl && cx < chx && cy >= cl && cy < chy;
    const bool own = act && tx >= 1 && ty >= 1;

    // time step of this grid's level and 1/dx
    double rl = 1.0;
    for (int l = 0; l < G.level; ++l) rl *= (double)ph.ratio;
    const T dt = T(dt0p[0] / rl);
    const T hdt = T(0.5) * dt;
    T idx[3];
    idx[0] = T(rl / ph.dx0[0]);
    idx[1] = T(rl / ph.dx0[1]);
    idx[2] = T(NDIM == 3 ? rl / ph.dx0[2] : 0.0);

    // own LDS entry and (for the first nring threads) one ring entry
    const int eo = (ty + 1) * kW + tx + 1;
    const int nring = 2 * (tw + th);
    int rex = 0, rey = 0;
    if (tid < nring) ring_entry(tid, tw, th, rex, rey);
    const int rcx = x0 - 2 + rex, rcy = y0 - 2 + rey;
    const bool rok = tid < nring && rcx >= wlo && rcx < whix && rcy >= wlo && rcy < whiy;
    const bool ook = live && cx >= wlo && cx < whix && cy >= wlo && cy < whiy;

    const int kstart = NDIM == 3 ? max(item.z0 - 1, cl) : 0;
    const int kend = NDIM == 3 ? item.z1 : 1;

    T wprev[8], wcur[8], wnext[8], wring[8];
    T fbcur[3][2], fbnext[3][2];  // face fields of the current / next plane's cell
    T zcarry[7];
#pragma unroll
    for (int q = 0; q < 8; ++q) { wprev[q] = T(1); wcur[q] = T(1); wnext[q] = T(1); wring[q] = T(1); }
#pragma unroll
    for (int q = 0; q < 7; ++q) zcarry[q] = T(0);

    // prologue: W(kstart-1) and W(kstart+1) own (3D), W(kstart) own + ring
    // into LDS; in 3-D the own cell's loads then run two planes ahead (the
    // predictor of plane k needs W(k+1))
    if (NDIM == 3 && ook) load_prim_b<T, NDIM>(U, bx(cx, cy, kstart - 1), bx.sy, bx.sz, gm1, wprev);
#pragma unroll
    for (int d = 0; d < 3; ++d) fbcur[d][0] = fbcur[d][1] = fbnext[d][0] = fbnext[d][1] = T(0);
    if (ook) load_prim_faces_b<T, NDIM>(U, bx(cx, cy, kstart), bx.sy, bx.sz, gm1, wcur, fbcur);
    if (NDIM == 3 && ook) load_prim_faces_b<T, NDIM>(U, bx(cx, cy, kstart + 1), bx.sy, bx.sz, gm1, wnext, fbnext);
    if (rok) load_prim_b<T, NDIM>(U, bx(rcx, rcy, kstart), bx.sy, bx.sz, gm1, wring);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (live) sW[q][eo] = wcur[q];
      if (tid < nring) sW[q][rey * kW + rex] = wring[q];
    }
    __syncthreads();

    for (int k = kstart; k < kend; ++k) {
      // raw fields of the own cell two planes up and of the ring cell one
      // plane up, converted once the predictor is done and before any flux
      // store of this plane: the loads have the predictor to arrive in, and
      // waiting for them does not wait for this plane's stores
      T rnext[5], rfb[3][2], rring[5], rrfb[3][2];
      const bool pf = NDIM == 3 && ook && k + 2 <= kend;
      if (NDIM == 3) {
        if (pf) load_raw3<T>(U, bx(cx, cy, k + 2), bx.sy, bx.sz, rnext, rfb);
        if (rok) load_raw3<T>(U, bx(rcx, rcy, k + 1), bx.sy, bx.sz, rring, rrfb);
      }
      Pred<T, NDIM> pr;
      if (act) {
        T wxm[8], wxp[8], wym[8], wyp[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          wxm[q] = sW[q][eo - 1];
          wxp[q] = sW[q][eo + 1];
          wym[q] = sW[q][eo - kW];
          wyp[q] = sW[q][eo + kW];
        }
        if ((wcur[0] <= T(0)) || (wcur[4] <= T(0))) flag_bad(err, ix(cx, cy, k));
        bool ok;
        if constexpr (UPWIND) {
          T du[8];
          ok = predict_du<T, NDIM>(wcur, wxm, wxp, wym, wyp, wprev, wnext, fbcur, hdt, idx, gam, pr, du);
          // reference EMF of the upwinded CT: -v x B with v of the half-step
          // cell state U + du and B at time n; one writer per cell (the
          // tile's own cells, plus the grid's first column / row / plane)
          if (k >= item.z0 && (tx >= 1 || cx == cl) && (ty >= 1 || cy == cl)) {
            const T ir = drcp(wcur[0] + du[0]);
            const T vx = (wcur[0] * wcur[1] + du[1]) * ir;
            const T vy = (wcur[0] * wcur[2] + du[2]) * ir;
            const T vz = (wcur[0] * wcur[3] + du[3]) * ir;
            const auto eb = bx(cx, cy, k);
            if (NDIM == 3) {
              stb(F.e[0], eb, vz * wcur[6] - vy * wcur[7]);
              stb(F.e[1], eb, vx * wcur[7] - vz * wcur[5]);
            }
            stb(F.e[2], eb, vy * wcur[5] - vx * wcur[6]);
          }
        } else {
          ok = predict<T, NDIM>(wcur, wxm, wxp, wym, wyp, wprev, wnext, fbcur, hdt, idx, gam, pr);
        }
        if (!ok) flag_bad(err, ix(cx, cy, k));
#pragma unroll
        for (int q = 0; q < 7; ++q) {
          sX[q][tid] = pr.p[0][q];
          sY[q][tid] = pr.p[1][q];
        }
      }
      __syncthreads();
      // every read of this plane's W is done: the next plane's W (own cell
      // and ring) goes into LDS while the Riemann problems run, and the
      // own-cell planes move up by one (the Riemann problems read only the
      // low-face normal fields bn of this plane)
      T bn[3] = {fbcur[0][0], fbcur[1][0], fbcur[2][0]};
      if (NDIM == 3) {
        if (rok) raw3_to_prim<T>(rring, rrfb, gm1, wring);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (live) sW[q][eo] = wnext[q];
          if (tid < nring) sW[q][rey * kW + rex] = wring[q];
          wprev[q] = wcur[q];
          wcur[q] = wnext[q];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          fbcur[d][0] = fbnext[d][0];
          fbcur[d][1] = fbnext[d][1];
        }
        if (pf) {
          raw3_to_prim<T>(rnext, rfb, gm1, wnext);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            fbnext[d][0] = rfb[d][0];
            fbnext[d][1] = rfb[d][1];
          }
        }
      }
      if (own && k >= item.z0) {
        const auto eb = bx(cx, cy, k);
        T f[7];
        if (cx > cl) {
          T l[7];
#pragma unroll
          for (int q = 0; q < 7; ++q) l[q] = sX[q][tid - 1];
          hlld7(l, pr.m[0], bn[0], gam, f);
#pragma unroll
          for (int q = 0; q < 7; ++q) stb(F.f[0][q], eb, f[q]);
        }
        if (cy > cl) {
          T l[7];
#pragma unroll
          for (int q = 0; q < 7; ++q) l[q] = sY[q][tid - tw];
          hlld7(l, pr.m[1], bn[1], gam, f);
#pragma unroll
          for (int q = 0; q < 7; ++q) stb(F.f[1][q], eb, f[q]);
        }
        if (NDIM == 3 && k > cl) {
          hlld7(zcarry, pr.m[2], bn[2], gam, f);
#pragma unroll
          for (int q = 0; q < 7; ++q) stb(F.f[2][q], eb, f[q]);
        }
      }
      if (NDIM == 3) {
#pragma unroll
        for (int q = 0; q < 7; ++q) zcarry[q] = pr.p[2][q];
      }
      __syncthreads();
    }
  }
  retire<PERSIST>(q);
}

template <class T, int NDIM, bool PERSIST, bool UPWIND>
__global__ __launch_bounds__(256) void k_update(const GridDesc* __restrict__ grids, const UpdItem* __restrict__ items,
                                                int nitems, DevState<T> S0, DevState<T> S1, uint32_t parity,
                                                DevFlux<T> F, const double* __restrict__ dt0p, Phys ph, WorkQueue* q,
                                                bool xcd, int claim) {
  __shared__ int s_claim[2], s_c;
  if (threadIdx.x == 0) s_c = 0;
  const int tid = threadIdx.x;
  ItemRange rng = first_claim<PERSIST>(nitems, claim, xcd);
  for (;;) {
    const int it = next_item<PERSIST>(rng, nitems, claim, q, s_claim, &s_c, xcd);
    if (it < 0) break;
    const UpdItem item = items[it];
    const GridDesc G = grids[item.grid];
    const bool odd = (parity >> G.level) & 1u;
    const DevState<T> Uin = odd ? S1 : S0;
    const DevState<T> Uout = odd ? S0 : S1;
    const Idx<NDIM> ix(G);
    const int gv = item.gv;
    const int uhx = G.n[0] + gv - 2, uhy = G.n[1] + gv - 2, uhz = NDIM == 3 ? G.n[2] + gv - 2 : 0;
    const int tw = item.tw, th = 256 / tw;
    const int tx = tid % tw, ty = tid / tw;
    if (ty >= th) continue;
    const int cx = item.x0 + tx, cy = item.y0 + ty;
    if (cx > uhx || cy > uhy) continue;

    double rl = 1.0;
    for (int l = 0; l < G.level; ++l) rl *= (double)ph.ratio;
    const T dt = T(dt0p[0] / rl);
    T idx[3];
    idx[0] = T(rl / ph.dx0[0]);
    idx[1] = T(rl / ph.dx0[1]);
    idx[2] = T(NDIM == 3 ? rl / ph.dx0[2] : 0.0);
    const T cdx = dt * idx[0], cdy = dt * idx[1], cdz = dt * idx[2];
    const int64_t st[3] = {1, ix.sy, NDIM == 3 ? ix.sz : 0};

    for (int k = item.z0; k < item.z1; ++k) {
      const int64_t e = ix(cx, cy, k);
      const bool cell = cx < uhx && cy < uhy && (NDIM == 2 || k < uhz);
      if (cell) {
        // lab conserved slot -> rotated component of direction d
#pragma unroll
        for (int s = 0; s < 5; ++s) {
          // lab conserved slot s -> rotated component of each direction
          const int qx = hydro_comp(s, 0), qy = hydro_comp(s, 1), qz = hydro_comp(s, 2);
          const T acc = flux_delta<T, NDIM>(cdx, F.f[0][qx][e + 1], F.f[0][qx][e], cdy, F.f[1][qy][e + st[1]],
                                            F.f[1][qy][e], cdz, NDIM == 3 ? F.f[2][qz][e + st[2]] : T(0),
                                            NDIM == 3 ? F.f[2][qz][e] : T(0));
          Uout.f[s][e] = Uin.f[s][e] - acc;
        }
        if (NDIM == 2) {
          // cell-centred Bz: x-flux component t2 (index 6), y-flux component t1 (index 5)
          const T acc = flux_delta<T, 2>(cdx, F.f[0][6][e + 1], F.f[0][6][e], cdy, F.f[1][5][e + st[1]],
                                         F.f[1][5][e], T(0), T(0), T(0));
          Uout.f[7][e] = Uin.f[7][e] - acc;
        }
      }
      if (NDIM == 3) {
        // faces: dB_d/dt = -(curl E)_d
        if (cy < uhy && k < uhz) {  // Bx face (cx, cy, k)
          T ez0 = emf_at<2, UPWIND>(F, e, st), ez1 = emf_at<2, UPWIND>(F, e + st[1], st);
          T ey0 = emf_at<1, UPWIND>(F, e, st), ey1 = emf_at<1, UPWIND>(F, e + st[2], st);
          Uout.f[5][e] = Uin.f[5][e] - curl_delta(cdy, ez1, ez0, cdz, ey1, ey0);
        }
        if (cx < uhx && k < uhz) {  // By face
          T ex0 = emf_at<0, UPWIND>(F, e, st), ex1 = emf_at<0, UPWIND>(F, e + st[2], st);
          T ez0 = emf_at<2, UPWIND>(F, e, st), ez1 = emf_at<2, UPWIND>(F, e + st[0], st);
          Uout.f[6][e] = Uin.f[6][e] - curl_delta(cdz, ex1, ex0, cdx, ez1, ez0);
        }
        if (cx < uhx && cy < uhy) {  // Bz face
          T ey0 = emf_at<1, UPWIND>(F, e, st), ey1 = emf_at<1, UPWIND>(F, e + st[0], st);
          T ex0 = emf_at<0, UPWIND>(F, e, st), ex1 = emf_at<0, UPWIND>(F, e + st[1], st);
          Uout.f[7][e] = Uin.f[7][e] - curl_delta(cdx, ey1, ey0, cdy, ex1, ex0);
        }
      } else {
        // 2D: only E_z; edges are cell corners.
        auto ez = [&](int64_t ee) { return emf_at<2, UPWIND>(F, ee, st); };
        if (cy < uhy) {  // Bx face
          T e0 = ez(e), e1 = ez(e + st[1]);
          Uout.f[5][e] = Uin.f[5][e] - face_delta2(cdy, e1, e0);
        }
        if (cx < uhx) {  // By face
          T e0 = ez(e), e1 = ez(e + st[0]);
          Uout.f[6][e] = Uin.f[6][e] + face_delta2(cdx, e1, e0);
        }
      }
    }
  }
  retire<PERSIST>(q);
}

// Upwinded edge EMFs (one thread per (x, y) column of an update tile one
// column and row wider than the update's, marching its planes): E_x, E_y, E_z
// of the edges at the low corner of each element (E_z only in 2D).
template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_emf(const GridDesc* __restrict__ grids, const UpdItem* __restrict__ items,
                                             DevFlux<T> F) {
  const UpdItem item = items[blockIdx.x];
  const int tw = item.tw, th = 256 / tw;
  const int tx = (int)threadIdx.x % tw, ty = (int)threadIdx.x / tw;
  if (ty >= th) return;
  const GridDesc G = grids[item.grid];
  const int ehx = G.n[0] + item.gv - 1, ehy = G.n[1] + item.gv - 1;  // last edge index (inclusive)
  const int cx = item.x0 + tx, cy = item.y0 + ty;
  if (cx > ehx || cy > ehy) return;
  const IdxB<NDIM, T> bx(G);
  const int32_t sb[3] = {(int32_t)sizeof(T), bx.sy, NDIM == 3 ? bx.sz : 0};
  for (int k = item.z0; k < item.z1; ++k) {
    const auto e = bx(cx, cy, k);
    if (NDIM == 3) {
      stb(F.edge[0], e, edge_emf_upwind_b<0>(F, e, sb));
      stb(F.edge[1], e, edge_emf_upwind_b<1>(F, e, sb));
    }
    stb(F.edge[2], e, edge_emf_upwind_b<2>(F, e, sb));
  }
}

}  // namespace

template <class T>
void launch_flux(int ndim, const GridDesc* grids, const FluxItem* items, int nitems, DevState<T> S0, DevState<T> S1,
                 uint32_t parity, DevFlux<T> F, const double* dt0, Phys ph, ErrBlock* err, WorkQueue* q, int pblocks,
                 bool xcd, int claim, bool upwind_emf, hipStream_t s) {
  if (nitems <= 0) return;
  const bool per = pblocks > 0 && q != nullptr;
  const dim3 grid(per ? std::min(pblocks, nitems) : claim_blocks(nitems, claim, xcd)), block(256);
#define AMR_FLUX_LAUNCH(ND, P, U)                                                                                  \
  hipLaunchKernelGGL((k_flux<T, ND, P, U>), grid, block, 0, s, grids, items, nitems, S0, S1, parity, F, dt0, ph, err, \
                     q, xcd, claim)
  if constexpr (std::is_same<T, float>::value || std::is_same<T, double>::value) {
    if (upwind_emf) {
      if (ndim == 3) {
        if (per) AMR_FLUX_LAUNCH(3, true, true);
        else AMR_FLUX_LAUNCH(3, false, true);
      } else {
        if (per) AMR_FLUX_LAUNCH(2, true, true);
        else AMR_FLUX_LAUNCH(2, false, true);
      }
      return;
    }
  }
  if (ndim == 3) {
    if (per) AMR_FLUX_LAUNCH(3, true, false);
    else AMR_FLUX_LAUNCH(3, false, false);
  } else {
    if (per) AMR_FLUX_LAUNCH(2, true, false);
    else AMR_FLUX_LAUNCH(2, false, false);
  }
#undef AMR_FLUX_LAUNCH
}

template <class T>
void launch_update(int ndim, const GridDesc* grids, const UpdItem* items, int nitems, DevState<T> S0, DevState<T> S1,
                   uint32_t parity, DevFlux<T> F, const double* dt0, Phys ph, WorkQueue* q, int pblocks,
                   bool xcd, int claim, bool upwind_emf, hipStream_t s) {
  if (nitems <= 0) return;
  const bool per = pblocks > 0 && q != nullptr;
  const dim3 grid(per ? std::min(pblocks, nitems) : claim_blocks(nitems, claim, xcd)), block(256);
#define AMR_UPD_LAUNCH(ND, P, U)                                                                                   \
  hipLaunchKernelGGL((k_update<T, ND, P, U>), grid, block, 0, s, grids, items, nitems, S0, S1, parity, F, dt0, ph, q, \
                     xcd, claim)
  if constexpr (std::is_same<T, float>::value || std::is_same<T, double>::value) {
    if (upwind_emf) {
      if (ndim == 3) {
        if (per) AMR_UPD_LAUNCH(3, true, true);
        else AMR_UPD_LAUNCH(3, false, true);
      } else {
        if (per) AMR_UPD_LAUNCH(2, true, true);
        else AMR_UPD_LAUNCH(2, false, true);
      }
      return;
    }
  }
  if (ndim == 3) {
    if (per) AMR_UPD_LAUNCH(3, true, false);
    else AMR_UPD_LAUNCH(3, false, false);
  } else {
    if (per) AMR_UPD_LAUNCH(2, true, false);
    else AMR_UPD_LAUNCH(2, false, false);
  }
#undef AMR_UPD_LAUNCH
}

template <class T>
void launch_emf(int ndim, const GridDesc* grids, const UpdItem* items, int nitems, DevFlux<T> F, hipStream_t s) {
  if (nitems <= 0) return;
  if (ndim == 3)
    hipLaunchKernelGGL((k_emf<T, 3>), dim3(nitems), dim3(256), 0, s, grids, items, F);
  else
    hipLaunchKernelGGL((k_emf<T, 2>), dim3(nitems), dim3(256), 0, s, grids, items, F);
}
template void launch_emf<float>(int, const GridDesc*, const UpdItem*, int, DevFlux<float>, hipStream_t);
template void launch_emf<double>(int, const GridDesc*, const UpdItem*, int, DevFlux<double>, hipStream_t);

// Resident 256-thread blocks per CU of each kernel (for persistent launches).
template <class T>
void kernel_occupancy(int ndim, int* flux_blocks_per_cu, int* update_blocks_per_cu) {
  int a = 0, b = 0;
  if (ndim == 3) {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_flux<T, 3, true, false>, 256, 0);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_update<T, 3, true, false>, 256, 0);
  } else {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_flux<T, 2, true, false>, 256, 0);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_update<T, 2, true, false>, 256, 0);
  }
  *flux_blocks_per_cu = a > 0 ? a : 1;
  *update_blocks_per_cu = b > 0 ? b : 1;
}

#define AMR_ADV_INST(T)                                                                                             \
  template void launch_flux<T>(int, const GridDesc*, const FluxItem*, int, DevState<T>, DevState<T>, uint32_t,     \
                               DevFlux<T>, const double*, Phys, ErrBlock*, WorkQueue*, int, bool, int, bool,          \
                               hipStream_t);                                                                       \
  template void launch_update<T>(int, const GridDesc*, const UpdItem*, int, DevState<T>, DevState<T>, uint32_t,   \
                                 DevFlux<T>, const double*, Phys, WorkQueue*, int, bool, int, bool, hipStream_t);
AMR_ADV_INST(float)
AMR_ADV_INST(double)
// frozen-branch instances (finite-difference verification of the adjoint)
AMR_ADV_INST(FrozenD)
AMR_ADV_INST(FrozenF)
#undef AMR_ADV_INST
template void kernel_occupancy<float>(int, int*, int*);
template void kernel_occupancy<double>(int, int*, int*);

}  // namespace amr
