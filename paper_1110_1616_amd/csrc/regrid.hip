// Regridding support for gfx950: refinement flags, the (O)verlap transfer
// from a previous iteration of grids, and the host-side Berger-Rigoutsos
// clustering.
//
// The paper's mesh is adaptive: every level has successive iterations of
// grids and the fluid variables move from the previous iteration to the
// current one (Sec. 2, the (O) of the level cycle in Sec. 4).  Flags mark
// level-l cells whose relative centred density jump along some axis exceeds
// theta; the host clusters them into the next iteration's level-(l+1) boxes.
// The transfer is a gather over host-built maps: same-level copies from the
// old pool, prolongation from the new parent level (the band-fill kernels),
// and a projection that completes the faces inside each prolonged coarse
// cell so every fine cell is divergence-free.
#include <algorithm>
#include <cmath>

#include "regrid_internal.hpp"

namespace amr {

namespace {

// ------------------------------------------------------------------ flags
// flag(c) = any_d |rho(c + e_d) - rho(c - e_d)| > theta (rho(c + e_d) +
// rho(c - e_d)), evaluated in FP64 on the (filled) level.
template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_flag(const GridDesc* __restrict__ grids, const FlagItem* __restrict__ items,
                                              DevState<T> U, double theta, uint8_t* __restrict__ out) {
  const FlagItem it = items[blockIdx.x];
  const int t = it.first + (int)threadIdx.x;
  if (t >= it.last) return;
  const GridDesc G = grids[it.grid];
  const int i = t % G.n[0];
  const int r = t / G.n[0];
  const int j = r % G.n[1];
  const int k = NDIM == 3 ? r / G.n[1] : 0;
  const int64_t sy = G.P[0], sz = (int64_t)G.P[0] * G.P[1];
  const int64_t e = G.off + (i + G.g) + (int64_t)(j + G.g) * sy + (NDIM == 3 ? (int64_t)(k + G.g) * sz : 0);
  const int64_t st[3] = {1, sy, sz};
  bool f = false;
#pragma unroll
  for (int d = 0; d < NDIM; ++d) {
    const double rp = (double)U.f[0][e + st[d]];
    const double rm = (double)U.f[0][e - st[d]];
    f = f || (fabs(rp - rm) > theta * (rp + rm));
  }
  out[it.out + t] = f ? 1 : 0;
}

// ----------------------------------------------------- copies across pools
template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_copy2(const CopyEntry* __restrict__ ent, int n, int4 cls, DevState<T> Us,
                                               DevState<T> Ud) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const CopyEntry e = ent[t];
    if (t < cls.x) {
      Ud.f[0][e.dst] = Us.f[0][e.src];
      Ud.f[1][e.dst] = Us.f[1][e.src];
      Ud.f[2][e.dst] = Us.f[2][e.src];
      Ud.f[3][e.dst] = Us.f[3][e.src];
      Ud.f[4][e.dst] = Us.f[4][e.src];
      if (NDIM == 2) Ud.f[7][e.dst] = Us.f[7][e.src];
    } else if (t < cls.y) {
      Ud.f[5][e.dst] = Us.f[5][e.src];
    } else if (t < cls.z) {
      Ud.f[6][e.dst] = Us.f[6][e.src];
    } else {
      Ud.f[7][e.dst] = Us.f[7][e.src];
    }
  }
}

// ------------------------------------------------------------- projection
// Faces inside one prolonged coarse cell (R = 2): each starts as the mean
// of the two boundary faces in line with it; r(c) is then the divergence of
// fine cell c (bits of c = its half along x, y, z); the correction is the
// smallest one that zeroes every r: potentials p = L^+ r of the fine-cell
// graph Laplacian (edge weight 1/dx_d^2), whose eigenvectors are the sign
// patterns chi_s(c) = (-1)^popcount(s & c) with eigenvalue
// 2 sum_{d in s} 1/dx_d^2; the face between c (low) and c + e_d then loses
// (p(c) - p(c + e_d)) / dx_d.
template <class T, int NDIM>
__global__ __launch_bounds__(256) void k_project(const ProjEntry* __restrict__ ent, int n,
                                                 const GridDesc* __restrict__ grids, DevState<T> U, Phys ph) {
  constexpr int NC = 1 << NDIM;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const ProjEntry pe = ent[t];
    const GridDesc G = grids[pe.grid];
    const int64_t st[3] = {1, G.P[0], (int64_t)G.P[0] * G.P[1]};
    double rl = 1.0;
    for (int l = 0; l < G.level; ++l) rl *= (double)ph.ratio;
    double dxd[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) dxd[d] = ph.dx0[d] / rl;
    T dx[3] = {T(dxd[0]), T(dxd[1]), T(dxd[2])};
    int64_t ec[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      ec[c] = pe.e0;
#pragma unroll
      for (int a = 0; a < NDIM; ++a)
        if ((c >> a) & 1) ec[c] += st[a];
    }
    // lo[d][c], hi[d][c]: faces of cell c along d (interior ones filled below)
    T lo[NDIM][NC], hi[NDIM][NC];
#pragma unroll
    for (int d = 0; d < NDIM; ++d)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if ((c >> d) & 1) continue;
        const int c1 = c | (1 << d);
        const T bl = U.f[5 + d][ec[c]];
        const T bh = U.f[5 + d][ec[c1] + st[d]];
        const T m = T(0.5) * (bl + bh);
        lo[d][c] = bl;
        hi[d][c] = m;
        lo[d][c1] = m;
        hi[d][c1] = bh;
      }
    T r[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      r[c] = T(0);
#pragma unroll
      for (int d = 0; d < NDIM; ++d) r[c] += (hi[d][c] - lo[d][c]) / dx[d];
    }
    T pot[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) pot[c] = T(0);
#pragma unroll
    for (int s = 1; s < NC; ++s) {
      double lamd = 0.0;
#pragma unroll
      for (int d = 0; d < NDIM; ++d)
        if ((s >> d) & 1) lamd += 2.0 / (dxd[d] * dxd[d]);
      const T lam = T(lamd);
      T dot = T(0);
#pragma unroll
      for (int c = 0; c < NC; ++c) dot += ((__builtin_popcount(s & c) & 1) ? T(-1) : T(1)) * r[c];
#pragma unroll
      for (int c = 0; c < NC; ++c) pot[c] += ((__builtin_popcount(s & c) & 1) ? T(-1) : T(1)) * dot / (T(NC) * lam);
    }
#pragma unroll
    for (int d = 0; d < NDIM; ++d)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if ((c >> d) & 1) continue;
        const int c1 = c | (1 << d);
        U.f[5 + d][ec[c1]] = hi[d][c] - (pot[c] - pot[c1]) / dx[d];
      }
  }
}

int blocks_for(int n) { return std::max(1, std::min((n + 255) / 256, 8192)); }

}  // namespace

template <class T>
void launch_flag(int ndim, const GridDesc* grids, const FlagItem* items, int nitems, DevState<T> U, double theta,
                 uint8_t* out, hipStream_t s) {
  if (nitems <= 0) return;
  if (ndim == 3)
    hipLaunchKernelGGL((k_flag<T, 3>), dim3(nitems), dim3(256), 0, s, grids, items, U, theta, out);
  else
    hipLaunchKernelGGL((k_flag<T, 2>), dim3(nitems), dim3(256), 0, s, grids, items, U, theta, out);
}

template <class T>
void launch_copy2(int ndim, const CopyEntry* ent, int n, int4 cls, DevState<T> Us, DevState<T> Ud, hipStream_t s) {
  if (n <= 0) return;
  if (ndim == 3)
    hipLaunchKernelGGL((k_copy2<T, 3>), dim3(blocks_for(n)), dim3(256), 0, s, ent, n, cls, Us, Ud);
  else
    hipLaunchKernelGGL((k_copy2<T, 2>), dim3(blocks_for(n)), dim3(256), 0, s, ent, n, cls, Us, Ud);
}

template <class T>
void launch_project(int ndim, const ProjEntry* ent, int n, const GridDesc* grids, DevState<T> U, Phys ph,
                    hipStream_t s) {
  if (n <= 0) return;
  if (ndim == 3)
    hipLaunchKernelGGL((k_project<T, 3>), dim3(blocks_for(n)), dim3(256), 0, s, ent, n, grids, U, ph);
  else
    hipLaunchKernelGGL((k_project<T, 2>), dim3(blocks_for(n)), dim3(256), 0, s, ent, n, grids, U, ph);
}

#define AMR_REGRID_INST(T)                                                                                       \
  template void launch_flag<T>(int, const GridDesc*, const FlagItem*, int, DevState<T>, double, uint8_t*,        \
                               hipStream_t);                                                                     \
  template void launch_copy2<T>(int, const CopyEntry*, int, int4, DevState<T>, DevState<T>, hipStream_t);       \
  template void launch_project<T>(int, const ProjEntry*, int, const GridDesc*, DevState<T>, Phys, hipStream_t);
AMR_REGRID_INST(float)
AMR_REGRID_INST(double)
#undef AMR_REGRID_INST

// ------------------------------------------------------------ clustering
// Cut preference: (1) a hole of the signature (no point across the box),
// axes by decreasing extent (ties: lower axis), the hole nearest the
// middle (ties: lower); (2) the strongest sign change of the signature's
// second difference, cut between the two cells where it changes (ties:
// nearer the middle, longer axis, lower axis, then the first found); (3)
// halve the longest axis (ties: lower axis).
namespace {

struct Cut {
  int axis, at;
};

Cut choose_cut(int nd, const IBox& B, const std::vector<int64_t> (&sig)[3]) {
  int ext[3];
  for (int a = 0; a < 3; ++a) ext[a] = B.hi[a] - B.lo[a];
  int by_len[3] = {0, 1, 2};
  std::stable_sort(by_len, by_len + nd, [&](int x, int y) { return ext[x] > ext[y]; });
  for (int q = 0; q < nd; ++q) {
    const int a = by_len[q];
    const double mid = ext[a] / 2.0;
    int best = -1;
    double bd = 0.0;
    for (int i = 0; i < ext[a]; ++i) {
      if (sig[a][i] != 0) continue;
      const double dd = std::fabs(i + 0.5 - mid);
      if (best < 0 || dd < bd) {
        best = i;
        bd = dd;
      }
    }
    if (best >= 0) return Cut{a, B.lo[a] + best};
  }
  bool have = false;
  int64_t bs = 0;
  double bmid = 0.0;
  int bn = 0, ba = 0;
  Cut bc{0, 0};
  for (int a = 0; a < nd; ++a) {
    const int n = ext[a];
    if (n < 4) continue;
    const double mid = n / 2.0;
    for (int i = 2; i < n - 1; ++i) {
      const int64_t x = sig[a][i - 2] - 2 * sig[a][i - 1] + sig[a][i];
      const int64_t y = sig[a][i - 1] - 2 * sig[a][i] + sig[a][i + 1];
      if (!((x < 0 && y > 0) || (y < 0 && x > 0))) continue;
      const int64_t st = y > x ? y - x : x - y;
      const double md = -std::fabs(i - mid);
      // lexicographic (strength, -|i - mid|, n, -axis), strictly greater wins
      bool better = !have;
      if (have) {
        if (st != bs) better = st > bs;
        else if (md != bmid) better = md > bmid;
        else if (n != bn) better = n > bn;
        else better = -a > -ba;
      }
      if (better) {
        have = true;
        bs = st;
        bmid = md;
        bn = n;
        ba = a;
        bc = Cut{a, B.lo[a] + i};
      }
    }
  }
  if (have) return bc;
  const int a = by_len[0];
  return Cut{a, B.lo[a] + ext[a] / 2};
}

}  // namespace

std::vector<IBox> cluster_boxes(int ndim, const int (&N)[3], const std::vector<std::array<int, 3>>& pts, double eff,
                                int maxbox, const std::function<bool(const IBox&)>& admissible) {
  std::vector<IBox> out;
  struct Job {
    IBox B;
    std::vector<int> idx;
  };
  std::vector<Job> stack;
  {
    Job j;
    for (int a = 0; a < 3; ++a) {
      j.B.lo[a] = 0;
      j.B.hi[a] = a < ndim ? N[a] : 1;
    }
    j.idx.resize(pts.size());
    for (size_t i = 0; i < pts.size(); ++i) j.idx[i] = (int)i;
    stack.push_back(std::move(j));
  }
  while (!stack.empty()) {
    Job job = std::move(stack.back());
    stack.pop_back();
    if (job.idx.empty()) continue;
    IBox B;
    for (int a = 0; a < 3; ++a) {
      B.lo[a] = a < ndim ? INT32_MAX : 0;
      B.hi[a] = a < ndim ? INT32_MIN : 1;
    }
    for (int i : job.idx)
      for (int a = 0; a < ndim; ++a) {
        B.lo[a] = std::min(B.lo[a], pts[i][a]);
        B.hi[a] = std::max(B.hi[a], pts[i][a] + 1);
      }
    int64_t vol = 1;
    int emax = 0;
    for (int a = 0; a < ndim; ++a) {
      vol *= B.hi[a] - B.lo[a];
      emax = std::max(emax, B.hi[a] - B.lo[a]);
    }
    const int64_t count = (int64_t)job.idx.size();
    if (vol == 1 || ((double)count >= eff * (double)vol && emax <= maxbox && admissible(B))) {
      out.push_back(B);
      continue;
    }
    std::vector<int64_t> sig[3];
    for (int a = 0; a < ndim; ++a) sig[a].assign(B.hi[a] - B.lo[a], 0);
    for (int i : job.idx)
      for (int a = 0; a < ndim; ++a) sig[a][pts[i][a] - B.lo[a]] += 1;
    const Cut c = choose_cut(ndim, B, sig);
    Job lo, hi;
    lo.B = B;
    hi.B = B;
    lo.B.hi[c.axis] = c.at;
    hi.B.lo[c.axis] = c.at;
    for (int i : job.idx) (pts[i][c.axis] < c.at ? lo.idx : hi.idx).push_back(i);
    stack.push_back(std::move(hi));  // taken second
    stack.push_back(std::move(lo));  // taken first
  }
  return out;
}

}  // namespace amr
