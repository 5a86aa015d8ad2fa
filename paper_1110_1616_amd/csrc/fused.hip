// Fused advance kernel for gfx950: the flux kernel's work (primitive
// recovery, minmod slopes, Hancock predictor, HLLD on every face) and the
// update kernel's work (edge EMFs, conservative and constrained-transport
// update) in one launch, so the face fluxes never travel through HBM.
//
// A work item is a column tile of tw x th threads over cells
// (x0-1+tx, y0-1+ty) marching along z.  Per plane k every active lane forms
// its cell's predicted face states; lanes then solve the Riemann problems of
// their cell's low x-face (tx >= 1), low y-face (ty >= 1) and low z-face
// (from the state carried from plane k-1), and the fluxes go to LDS, double
// buffered over two planes.  From them come the edge EMFs E_z of plane k and
// E_x, E_y at z = k - 1/2, and the update of plane k-1 (cells and their x-
// and y-faces) and of the z-faces at k - 1/2.  A plane takes two barriers in
// 3-D: the update reads E_z of the plane below (from the iteration before)
// and forms the neighbours' E_x, E_y again from their inputs in LDS.  A tile updates the cells of
// lanes tx in [1, tw-2], ty in [1, th-2] (their high faces and the edges
// around them are computed in the tile); tiles overlap by two columns and
// rows (the last x- and y-face of the update region go to the lane that
// holds them).  Every flux, EMF and update is formed with the same source
// expressions as the two-kernel path (the update's arithmetic is shared, in
// emf.hpp), and the library is compiled with multiply-add contraction
// inside single expressions only, so the results equal the two-kernel
// path's bit for bit.
//
// Face fluxes that the coarse/fine registers read afterwards are still
// stored: a per-element mask marks them (bit d for the face normal to d) and
// one owning lane per face writes them.
#include <algorithm>
#include <type_traits>

#include "advance_common.hpp"
#include "amr_internal.hpp"
#include "emf.hpp"
#include "launch_common.hpp"
#include "mhd_device.hpp"

namespace amr {

namespace {

// Both state sets, indexed by level parity per work item (a kernel-argument
// block read where an item starts, not held in registers across items).
template <class T> struct StatePair {
  DevState<T> s[2];
};
// A masked store of a face's seven flux components forms the arrays'
// addresses from the base and stride where it stores (the empty asm keeps
// the 21 addresses from being formed once and held in scalar registers
// through the plane loop, which spilled them).
template <class T, class B>
__device__ __forceinline__ void st_flux7(const DevFlux<T>& F, int d, B b, const T (&v)[7]) {
  uint64_t p = reinterpret_cast<uint64_t>(F.base), st = F.stride;
  asm volatile("" : "+s"(p), "+s"(st));
  p += (uint64_t)(7 * d) * st;
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    *reinterpret_cast<__attribute__((address_space(1))) T*>(p + b) = v[c];
    p += st;
  }
}

// Lane t of a tile dimension tdim is the one that stores (for the
// registers) coordinate c of a computed range [clo, chi]: tiles overlap by
// two, so interior lanes [1, tdim-2] own their coordinate and the edge lanes
// only the range's end points.
__device__ __forceinline__ bool owns(int t, int tdim, int c, int clo, int chi) {
  return (t >= 1 && t <= tdim - 2) || (t == 0 && c == clo) || (t == tdim - 1 && c == chi);
}

template <class T, int NDIM, bool PERSIST>
__global__ __launch_bounds__(256) void k_fused(const GridDesc* __restrict__ grids, const FluxItem* __restrict__ items,
                                               int nitems, StatePair<T> S, uint32_t parity,
                                               DevFlux<T> F, const uint8_t* __restrict__ fmask,
                                               const double* __restrict__ dt0p, Phys ph, ErrBlock* err, WorkQueue* q,
                                               bool xcd, int claim) {
  __shared__ T sW[8][kMaxPlane];
  __shared__ T sX[7][256];
  __shared__ T sY[7][256];
  __shared__ T sH[2][10][256];  // hydro components 0..4 of the x- (0..4) and y-face (5..9) fluxes, by plane parity
  __shared__ T sB[4][256];      // EMF inputs of this plane: F_x c5, F_y c6, F_z c5, F_z c6 (2-D: F_x c6, F_y c5)
  __shared__ T sEz[2][256];     // E_z at each lane's (x, y) low corner, by plane parity
  __shared__ T sX6[2][256];     // 3-D: F_x c6 and F_y c5 of each lane, by plane parity (the inputs of
  __shared__ T sY5[2][256];     // the neighbours' E_x, E_y, formed again where the z-faces need them)
  __shared__ int s_claim[2], s_c;
  if (threadIdx.x == 0) s_c = 0;

  const int tid = threadIdx.x;
  const T gam = T(ph.gamma);
  const T gm1 = gam - T(1);

  ItemRange rng = first_claim<PERSIST>(nitems, claim, xcd);
  for (;;) {
    const int it = next_item<PERSIST>(rng, nitems, claim, q, s_claim, &s_c, xcd);
    if (it < 0) break;
    const FluxItem item = items[it];
    const GridDesc G = grids[item.grid];
    const bool odd = (parity >> G.level) & 1u;
    const DevState<T> U = S.s[odd ? 1 : 0];
    const DevState<T> V = S.s[odd ? 0 : 1];
    const Idx<NDIM> ix(G);
    const IdxB<NDIM, T> bx(G);
    const int gv = item.gv;
    const int cl = -gv + 1;
    const int chx = G.n[0] + gv - 1, chy = G.n[1] + gv - 1;
    const int wlo = -gv, whix = G.n[0] + gv, whiy = G.n[1] + gv;
    const int ul = -gv + 2;
    const int uhx = G.n[0] + gv - 2, uhy = G.n[1] + gv - 2, uhz = NDIM == 3 ? G.n[2] + gv - 2 : 1;
    const int x0 = item.x0, y0 = item.y0;
    const int tw = item.tw, th = 256 / tw, kW = tw + 2;
    const int tx = tid % tw, ty = tid / tw;
    const bool live = ty < th;
    const int cx = x0 - 1 + tx, cy = y0 - 1 + ty;
    const bool act = live && cx >= cl && cx < chx && cy >= cl && cy < chy;
    const bool xf = act && tx >= 1 && cx > cl;  // solves its cell's low x-face
    const bool yf = act && ty >= 1 && cy > cl;  // low y-face
    // update ownership: cells and z-faces at interior lanes; x- and y-faces
    // also the update region's last face (uh), wherever it falls
    const bool ucol = tx >= 1 && tx <= tw - 2 && cx >= ul && cx < uhx;
    const bool urow = ty >= 1 && ty <= th - 2 && cy >= ul && cy < uhy;
    const bool ucell = live && ucol && urow;
    const bool ubx = live && urow && (ucol || (tx >= 1 && cx == uhx));
    const bool uby = live && ucol && (urow || (ty >= 1 && cy == uhy));
    // flux stores for the registers: one owning lane per computed face
    const bool sxy_x = owns(tx, tw, cx, cl, chx - 1), sxy_y = owns(ty, th, cy, cl, chy - 1);

    double rl = 1.0;
    for (int l = 0; l < G.level; ++l) rl *= (double)ph.ratio;
    const T dt = T(dt0p[0] / rl);
    const T hdt = T(0.5) * dt;
    T idx[3];
    idx[0] = T(rl / ph.dx0[0]);
    idx[1] = T(rl / ph.dx0[1]);
    idx[2] = T(NDIM == 3 ? rl / ph.dx0[2] : 0.0);
    const T cdx = dt * idx[0], cdy = dt * idx[1], cdz = dt * idx[2];

    const int eo = (ty + 1) * kW + tx + 1;
    const int nring = 2 * (tw + th);
    int rex = 0, rey = 0;
    if (tid < nring) ring_entry(tid, tw, th, rex, rey);
    const int rcx = x0 - 2 + rex, rcy = y0 - 2 + rey;
    const bool rok = tid < nring && rcx >= wlo && rcx < whix && rcy >= wlo && rcy < whiy;
    const bool ook = live && cx >= wlo && cx < whix && cy >= wlo && cy < whiy;

    // planes: update planes [z0, z1) (cells below uhz; z-faces up to uhz);
    // predicted states from z0 - 1 to the last plane whose fluxes they need
    const int z0 = NDIM == 3 ? item.z0 : 0, z1 = NDIM == 3 ? item.z1 : 1;
    const int kstart = NDIM == 3 ? z0 - 1 : 0;
    const int kend = NDIM == 3 ? min(z1, uhz) : 0;  // inclusive

    T wprev[8], wcur[8], wnext[8], wring[8];
    T fbcur[3][2], fbnext[3][2];
    T zcarry[7];
#pragma unroll
    for (int c = 0; c < 8; ++c) { wprev[c] = T(1); wcur[c] = T(1); wnext[c] = T(1); wring[c] = T(1); }
#pragma unroll
    for (int c = 0; c < 7; ++c) zcarry[c] = T(0);
    // carried from the previous plane: z-flux hydro components at k - 1/2,
    // E_x and E_y at the low z-edges, F_y c5 and F_x c6 of the plane
    T fzp[5] = {T(0), T(0), T(0), T(0), T(0)};
    T exp_ = T(0), eyp_ = T(0), fy5p = T(0), fx6p = T(0);

#pragma unroll
    for (int d = 0; d < 3; ++d) fbcur[d][0] = fbcur[d][1] = fbnext[d][0] = fbnext[d][1] = T(0);
    if (NDIM == 3) {
      // the item's first planes: every load issued before any conversion
      T r0[5], r1[5], r2[5], rr[5], f0[3][2], fr[3][2];
      if (ook) {
        load_raw3<T>(U, bx(cx, cy, kstart - 1), bx.sy, bx.sz, r0, f0);
        load_raw3<T>(U, bx(cx, cy, kstart), bx.sy, bx.sz, r1, fbcur);
        load_raw3<T>(U, bx(cx, cy, kstart + 1), bx.sy, bx.sz, r2, fbnext);
      }
      if (rok) load_raw3<T>(U, bx(rcx, rcy, kstart), bx.sy, bx.sz, rr, fr);
      if (ook) {
        raw3_to_prim<T>(r0, f0, gm1, wprev);
        raw3_to_prim<T>(r1, fbcur, gm1, wcur);
        raw3_to_prim<T>(r2, fbnext, gm1, wnext);
      }
      if (rok) raw3_to_prim<T>(rr, fr, gm1, wring);
    } else {
      if (ook) load_prim_faces_b<T, NDIM>(U, bx(cx, cy, kstart), bx.sy, bx.sz, gm1, wcur, fbcur);
      if (rok) load_prim_b<T, NDIM>(U, bx(rcx, rcy, kstart), bx.sy, bx.sz, gm1, wring);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (live) sW[c][eo] = wcur[c];
      if (tid < nring) sW[c][rey * kW + rex] = wring[c];
    }
    __syncthreads();

    uint8_t mknext = (fmask && act) ? fmask[ix(cx, cy, kstart)] : uint8_t(0);
    for (int k = kstart; k <= kend; ++k) {
      const int pb = k & 1;
      // this plane's face mask was loaded an iteration ago; the next one's
      // load is in flight through this iteration
      const uint8_t mk = mknext;
      if (fmask && act && k + 1 <= kend) mknext = fmask[ix(cx, cy, k + 1)];
      T rnext[5], rfb[3][2], rring[5], rrfb[3][2];
      const bool pf = NDIM == 3 && ook && k + 2 <= kend + 1;
      if (NDIM == 3) {
        if (pf) load_raw3<T>(U, bx(cx, cy, k + 2), bx.sy, bx.sz, rnext, rfb);
        if (rok && k + 1 <= kend) load_raw3<T>(U, bx(rcx, rcy, k + 1), bx.sy, bx.sz, rring, rrfb);
      }
      Pred<T, NDIM> pr;
      if (act) {
        T wxm[8], wxp[8], wym[8], wyp[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          wxm[c] = sW[c][eo - 1];
          wxp[c] = sW[c][eo + 1];
          wym[c] = sW[c][eo - kW];
          wyp[c] = sW[c][eo + kW];
        }
        if ((wcur[0] <= T(0)) || (wcur[4] <= T(0))) flag_bad(err, ix(cx, cy, k));
        const bool ok = predict<T, NDIM>(wcur, wxm, wxp, wym, wyp, wprev, wnext, fbcur, hdt, idx, gam, pr);
        if (!ok) flag_bad(err, ix(cx, cy, k));
#pragma unroll
        for (int c = 0; c < 7; ++c) {
          sX[c][tid] = pr.p[0][c];
          sY[c][tid] = pr.p[1][c];
        }
      }
      __syncthreads();
      // this plane's W has been read: the next plane's goes into LDS while
      // the Riemann problems run
      T bn[3] = {fbcur[0][0], fbcur[1][0], fbcur[2][0]};
      if (NDIM == 3) {
        if (rok && k + 1 <= kend) raw3_to_prim<T>(rring, rrfb, gm1, wring);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          if (live) sW[c][eo] = wnext[c];
          if (tid < nring) sW[c][rey * kW + rex] = wring[c];
          wprev[c] = wcur[c];
          wcur[c] = wnext[c];
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
      const bool zf = NDIM == 3 && act && k >= z0;
      const auto eb = bx(cx, cy, k);
      T fx[7], fy[7], fz[7];
#pragma unroll
      for (int c = 0; c < 7; ++c) { fx[c] = T(0); fy[c] = T(0); fz[c] = T(0); }
      if (xf) {
        T l[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) l[c] = sX[c][tid - 1];
        hlld7(l, pr.m[0], bn[0], gam, fx);
        if ((mk & 1u) && sxy_x && sxy_y && (NDIM == 2 || (k >= z0 && k < z1) || (k == kstart && z0 == ul)))
          st_flux7(F, 0, eb, fx);
      }
      if (yf) {
        T l[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) l[c] = sY[c][tid - tw];
        hlld7(l, pr.m[1], bn[1], gam, fy);
        if ((mk & 2u) && sxy_x && sxy_y && (NDIM == 2 || (k >= z0 && k < z1) || (k == kstart && z0 == ul)))
          st_flux7(F, 1, eb, fy);
      }
      if (zf) {
        hlld7(zcarry, pr.m[2], bn[2], gam, fz);
        if ((mk & 4u) && sxy_x && sxy_y && k < z1)
          st_flux7(F, 2, eb, fz);
      }
      if (NDIM == 3) {
#pragma unroll
        for (int c = 0; c < 7; ++c) zcarry[c] = pr.p[2][c];
      }
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        sH[pb][c][tid] = fx[c];
        sH[pb][5 + c][tid] = fy[c];
      }
      sB[0][tid] = fx[5];
      sB[1][tid] = fy[6];
      if (NDIM == 3) {
        sB[2][tid] = fz[5];
        sB[3][tid] = fz[6];
        sX6[pb][tid] = fx[6];
        sY5[pb][tid] = fy[5];
      } else {
        sB[2][tid] = fx[6];
        sB[3][tid] = fy[5];
      }
      __syncthreads();
      // edge EMFs: E_z at (cx - 1/2, cy - 1/2) of plane k; E_x at
      // (cx, cy - 1/2) and E_y at (cx - 1/2, cy), both at z = k - 1/2
      if (xf && yf) sEz[pb][tid] = emf_mean(sB[0][tid - tw], fx[5], sB[1][tid - 1], fy[6]);
      T ex = T(0), ey = T(0);
      if (NDIM == 3 && k >= z0) {
        if (yf) ex = emf_mean(fy5p, fy[5], sB[3][tid - tw], fz[6]);
        if (xf) ey = emf_mean(sB[2][tid - 1], fz[5], fx6p, fx[6]);
      }
      // 2-D: the faces read E_z of the neighbours' corners, formed above; in
      // 3-D every input of this plane's update is in LDS already (E_z of the
      // plane below, and the inputs of the neighbours' E_x, E_y)
      if (NDIM == 2) __syncthreads();
      if (NDIM == 3) {
        // the old values of everything this plane updates are loaded before
        // any store, so their latencies overlap
        const int kk = k - 1;
        const bool zup = ucell && k >= z0 && k < z1;
        const bool cup = kk >= z0 && kk < z1 && kk < uhz;
        const auto ec = bx(cx, cy, kk);
        T uo[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) uo[s] = T(0);
        if (zup) uo[7] = ldb(U.f[7], eb);
        if (cup && ucell)
#pragma unroll
          for (int s = 0; s < 5; ++s) uo[s] = ldb(U.f[s], ec);
        if (cup && ubx) uo[5] = ldb(U.f[5], ec);
        if (cup && uby) uo[6] = ldb(U.f[6], ec);
        // z-faces at k - 1/2 (element of plane k)
        if (zup) {
          // E_y of the next lane's and E_x of the next row's low z-edge,
          // from the same inputs as those lanes form them
          const int qb = kk & 1;
          const T ey1 = emf_mean(sB[2][tid], sB[2][tid + 1], sX6[qb][tid + 1], sX6[pb][tid + 1]);
          const T ex1 = emf_mean(sY5[qb][tid + tw], sY5[pb][tid + tw], sB[3][tid], sB[3][tid + tw]);
          stb(V.f[7], eb, uo[7] - curl_delta(cdx, ey1, ey, cdy, ex1, ex));
        }
        // cells and x-, y-faces of plane k - 1
        if (cup) {
          const int qb = kk & 1;
          if (ucell) {
#pragma unroll
            for (int s = 0; s < 5; ++s) {
              const int qx = hydro_comp(s, 0), qy = hydro_comp(s, 1), qz = hydro_comp(s, 2);
              const T acc = flux_delta<T, 3>(cdx, sH[qb][qx][tid + 1], sH[qb][qx][tid], cdy, sH[qb][5 + qy][tid + tw],
                                             sH[qb][5 + qy][tid], cdz, fz[qz], fzp[qz]);
              stb(V.f[s], ec, uo[s] - acc);
            }
          }
          if (ubx) {
            const T ez0 = sEz[qb][tid], ez1 = sEz[qb][tid + tw];
            stb(V.f[5], ec, uo[5] - curl_delta(cdy, ez1, ez0, cdz, ey, eyp_));
          }
          if (uby) {
            const T ez0 = sEz[qb][tid], ez1 = sEz[qb][tid + 1];
            stb(V.f[6], ec, uo[6] - curl_delta(cdz, ex, exp_, cdx, ez1, ez0));
          }
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) fzp[c] = fz[c];
        exp_ = ex;
        eyp_ = ey;
        fy5p = fy[5];
        fx6p = fx[6];
      } else {
        // 2-D: the single plane's cells (B_z cell-centred) and faces
        if (ucell) {
#pragma unroll
          for (int s = 0; s < 5; ++s) {
            const int qx = hydro_comp(s, 0), qy = hydro_comp(s, 1);
            const T acc = flux_delta<T, 2>(cdx, sH[0][qx][tid + 1], sH[0][qx][tid], cdy, sH[0][5 + qy][tid + tw],
                                           sH[0][5 + qy][tid], T(0), T(0), T(0));
            stb(V.f[s], eb, ldb(U.f[s], eb) - acc);
          }
          const T acc = flux_delta<T, 2>(cdx, sB[2][tid + 1], sB[2][tid], cdy, sB[3][tid + tw], sB[3][tid], T(0), T(0),
                                         T(0));
          stb(V.f[7], eb, ldb(U.f[7], eb) - acc);
        }
        if (ubx) {
          const T e0 = sEz[0][tid], e1 = sEz[0][tid + tw];
          stb(V.f[5], eb, ldb(U.f[5], eb) - face_delta2(cdy, e1, e0));
        }
        if (uby) {
          const T e0 = sEz[0][tid], e1 = sEz[0][tid + 1];
          stb(V.f[6], eb, ldb(U.f[6], eb) + face_delta2(cdx, e1, e0));
        }
      }
    }
    __syncthreads();
  }
  retire<PERSIST>(q);
}

}  // namespace

template <class T>
void launch_fused(int ndim, const GridDesc* grids, const FluxItem* items, int nitems, DevState<T> S0, DevState<T> S1,
                  uint32_t parity, DevFlux<T> F, const uint8_t* fmask, const double* dt0, Phys ph, ErrBlock* err,
                  WorkQueue* q, int pblocks, bool xcd, int claim, hipStream_t s) {
  if (nitems <= 0) return;
  const bool per = pblocks > 0 && q != nullptr;
  const dim3 grid(per ? std::min(pblocks, nitems) : claim_blocks(nitems, claim, xcd)), block(256);
  StatePair<T> SP;
  SP.s[0] = S0;
  SP.s[1] = S1;
#define AMR_FUSED_LAUNCH(ND, P) \
  hipLaunchKernelGGL((k_fused<T, ND, P>), grid, block, 0, s, grids, items, nitems, SP, parity, F, fmask, dt0, ph, err, q, \
                     xcd, claim)
  if (ndim == 3) {
    if (per) AMR_FUSED_LAUNCH(3, true);
    else AMR_FUSED_LAUNCH(3, false);
  } else {
    if (per) AMR_FUSED_LAUNCH(2, true);
    else AMR_FUSED_LAUNCH(2, false);
  }
#undef AMR_FUSED_LAUNCH
}

template <class T> int fused_occupancy(int ndim) {
  int a = 0;
  if (ndim == 3)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_fused<T, 3, true>, 256, 0);
  else
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_fused<T, 2, true>, 256, 0);
  return a > 0 ? a : 1;
}

#define AMR_FUSED_INST(T)                                                                                           \
  template void launch_fused<T>(int, const GridDesc*, const FluxItem*, int, DevState<T>, DevState<T>, uint32_t,    \
                                DevFlux<T>, const uint8_t*, const double*, Phys, ErrBlock*, WorkQueue*, int, bool, \
                                int, hipStream_t);                                                                      \
  template int fused_occupancy<T>(int);
AMR_FUSED_INST(float)
AMR_FUSED_INST(double)
#undef AMR_FUSED_INST

}  // namespace amr
