// Host-side self-check of the hand-written adjoints (no GPU needed): the
// pointwise device functions are also host functions, so each reverse-mode
// piece is compared, on random physical states, with the exact directional
// derivative of its forward piece evaluated in a forward-mode dual number
// (the dot-product test <a_out, J d> = <J^T a_out, d>).
#include <cmath>
#include <cstdint>
#include <random>

#include "../../include/amr.h"
#include "mhd_adjoint.hpp"

// Forward-mode dual number for exact directional derivatives of the host
// instances of the pointwise functions.
struct HDual {
  __host__ __device__ HDual(const HDual&) = default;
  __host__ __device__ HDual& operator=(const HDual&) = default;
  double v, d;
  __host__ __device__ HDual(double x = 0.0) : v(x), d(0.0) {}
  __host__ __device__ HDual(double x, double dx) : v(x), d(dx) {}
};
__host__ __device__ inline HDual operator+(HDual a, HDual b) { return HDual(a.v + b.v, a.d + b.d); }
__host__ __device__ inline HDual operator-(HDual a, HDual b) { return HDual(a.v - b.v, a.d - b.d); }
__host__ __device__ inline HDual operator-(HDual a) { return HDual(-a.v, -a.d); }
__host__ __device__ inline HDual operator*(HDual a, HDual b) { return HDual(a.v * b.v, a.d * b.v + a.v * b.d); }
__host__ __device__ inline HDual operator/(HDual a, HDual b) {
  const double q = a.v / b.v;
  return HDual(q, (a.d - q * b.d) / b.v);
}
__host__ __device__ inline HDual& operator+=(HDual& a, HDual b) { return a = a + b; }
__host__ __device__ inline HDual& operator-=(HDual& a, HDual b) { return a = a - b; }
__host__ __device__ inline HDual& operator*=(HDual& a, HDual b) { return a = a * b; }
__host__ __device__ inline bool operator<(HDual a, HDual b) { return a.v < b.v; }
__host__ __device__ inline bool operator>(HDual a, HDual b) { return a.v > b.v; }
__host__ __device__ inline bool operator<=(HDual a, HDual b) { return a.v <= b.v; }
__host__ __device__ inline bool operator>=(HDual a, HDual b) { return a.v >= b.v; }
namespace amr {
template <> __host__ __device__ inline HDual dsqrt<HDual>(HDual x) {
  const double s = __builtin_sqrt(x.v);
  return HDual(s, x.d / (2.0 * s));
}
}  // namespace amr

using namespace amr;

namespace {

struct Rng {
  std::mt19937_64 g;
  explicit Rng(uint64_t s) : g(s) {}
  double u(double a, double b) { return std::uniform_real_distribution<double>(a, b)(g); }
  double n() { return std::normal_distribution<double>(0.0, 1.0)(g); }
};

void rand_prim(Rng& r, double (&w)[8]) {
  w[0] = r.u(0.5, 2.0);
  w[1] = 0.4 * r.n();
  w[2] = 0.4 * r.n();
  w[3] = 0.4 * r.n();
  w[4] = r.u(0.3, 2.0);
  w[5] = 0.6 * r.n();
  w[6] = 0.6 * r.n();
  w[7] = 0.6 * r.n();
}

double rel(double a, double b) { return std::fabs(a - b) / (std::fabs(a) + std::fabs(b) + 1e-300); }

}  // namespace

extern "C" {

// which: 0 to_primitive, 1 to_conserved, 2..4 flux_along<0..2>, 5 fast speed,
// 6 HLLD.  Returns the largest relative mismatch over ntrials.
double amr_selfcheck_adjoint(int32_t which, int32_t ntrials, uint64_t seed) {
  if (which < 0 || which > 6 || ntrials < 1) return -1.0;
  Rng r(seed);
  const double gam = 5.0 / 3.0, gm1 = gam - 1.0, gi = 1.0 / gm1;
  double worst = 0.0;
  for (int t = 0; t < ntrials; ++t) {
    double x[17], dx[17];
    int nin = 0, nout = 0;
    double w[8];
    rand_prim(r, w);
    double w2[8];
    rand_prim(r, w2);
    if (which == 0) {  // input U
      to_conserved(w, *(double(*)[8])x, gi);
      nin = 8;
      nout = 8;
    } else if (which <= 4) {
      for (int q = 0; q < 8; ++q) x[q] = w[q];
      nin = 8;
      nout = which == 1 ? 8 : 8;
    } else if (which == 5) {
      x[0] = w[0]; x[1] = w[4]; x[2] = w[5] * w[5] + w[6] * w[6] + w[7] * w[7]; x[3] = w[5];
      nin = 4;
      nout = 1;
    } else {
      for (int q = 0; q < 8; ++q) x[q] = w[q];
      for (int q = 0; q < 8; ++q) x[8 + q] = w2[q];
      x[16] = w[5];
      nin = 17;
      nout = 7;
    }
    for (int i = 0; i < nin; ++i) dx[i] = r.n();
    if (which == 6) { dx[5] = 0.0; dx[13] = 0.0; }
    double lam[8];
    for (int i = 0; i < nout; ++i) lam[i] = r.n();
    auto fwd = [&](const double* xx, double* out) {
      if (which == 0) {
        double u[8], o[8];
        for (int q = 0; q < 8; ++q) u[q] = xx[q];
        to_primitive(u, o, gm1);
        for (int q = 0; q < 8; ++q) out[q] = o[q];
      } else if (which == 1) {
        double ww[8], o[8];
        for (int q = 0; q < 8; ++q) ww[q] = xx[q];
        to_conserved(ww, o, gi);
        for (int q = 0; q < 8; ++q) out[q] = o[q];
      } else if (which <= 4) {
        double ww[8], o[8];
        for (int q = 0; q < 8; ++q) ww[q] = xx[q];
        if (which == 2) flux_along<0>(ww, o, gi);
        if (which == 3) flux_along<1>(ww, o, gi);
        if (which == 4) flux_along<2>(ww, o, gi);
        for (int q = 0; q < 8; ++q) out[q] = o[q];
        out[which - 2 + 5] = 0.0;
      } else if (which == 5) {
        out[0] = fast_magnetosonic(xx[0], xx[1], xx[2], xx[3], gam);
      } else {
        double ql[8], qr[8], f[7];
        for (int q = 0; q < 8; ++q) {
          ql[q] = xx[q];
          qr[q] = xx[8 + q];
        }
        riemann_hlld(ql, qr, xx[16], gam, f);
        for (int q = 0; q < 7; ++q) out[q] = f[q];
      }
    };
    // exact directional derivative <lam, J dx> by forward-mode duals
    (void)fwd;
    double fd = 0.0;
    {
      HDual xd[17];
      for (int i = 0; i < nin; ++i) xd[i] = HDual(x[i], dx[i]);
      HDual od[8];
      if (which == 0) {
        HDual u[8], o[8];
        for (int q = 0; q < 8; ++q) u[q] = xd[q];
        to_primitive(u, o, HDual(gm1));
        for (int q = 0; q < 8; ++q) od[q] = o[q];
      } else if (which == 1) {
        HDual ww[8], o[8];
        for (int q = 0; q < 8; ++q) ww[q] = xd[q];
        to_conserved(ww, o, HDual(gi));
        for (int q = 0; q < 8; ++q) od[q] = o[q];
      } else if (which <= 4) {
        HDual ww[8], o[8];
        for (int q = 0; q < 8; ++q) ww[q] = xd[q];
        if (which == 2) flux_along<0>(ww, o, HDual(gi));
        if (which == 3) flux_along<1>(ww, o, HDual(gi));
        if (which == 4) flux_along<2>(ww, o, HDual(gi));
        for (int q = 0; q < 8; ++q) od[q] = o[q];
        od[which - 2 + 5] = HDual(0.0);
      } else if (which == 5) {
        od[0] = fast_magnetosonic(xd[0], xd[1], xd[2], xd[3], HDual(gam));
      } else {
        HDual ql[8], qr[8], f[7];
        for (int q = 0; q < 8; ++q) {
          ql[q] = xd[q];
          qr[q] = xd[8 + q];
        }
        riemann_hlld(ql, qr, xd[16], HDual(gam), f);
        for (int q = 0; q < 7; ++q) od[q] = f[q];
      }
      for (int i = 0; i < nout; ++i) fd += lam[i] * od[i].d;
    }
    // adjoint
    double ad[17] = {0};
    if (which == 0) {
      double u[8], aw[8], au[8] = {0};
      for (int q = 0; q < 8; ++q) { u[q] = x[q]; aw[q] = lam[q]; }
      to_primitive_adj(u, gm1, aw, au);
      for (int q = 0; q < 8; ++q) ad[q] = au[q];
    } else if (which == 1) {
      double ww[8], au[8], aw[8] = {0};
      for (int q = 0; q < 8; ++q) { ww[q] = x[q]; au[q] = lam[q]; }
      to_conserved_adj(ww, gi, au, aw);
      for (int q = 0; q < 8; ++q) ad[q] = aw[q];
    } else if (which <= 4) {
      double ww[8], af[8], aw[8] = {0};
      for (int q = 0; q < 8; ++q) { ww[q] = x[q]; af[q] = lam[q]; }
      if (which == 2) flux_along_adj<0>(ww, gi, af, aw);
      if (which == 3) flux_along_adj<1>(ww, gi, af, aw);
      if (which == 4) flux_along_adj<2>(ww, gi, af, aw);
      for (int q = 0; q < 8; ++q) ad[q] = aw[q];
    } else if (which == 5) {
      double ar = 0, ap = 0, ab2 = 0, abn = 0;
      fast_magnetosonic_adj(x[0], x[1], x[2], x[3], gam, lam[0], ar, ap, ab2, abn);
      ad[0] = ar; ad[1] = ap; ad[2] = ab2; ad[3] = abn;
    } else {
      double ql[8], qr[8], af[7], aql[8] = {0}, aqr[8] = {0}, abn = 0;
      for (int q = 0; q < 8; ++q) { ql[q] = x[q]; qr[q] = x[8 + q]; }
      for (int q = 0; q < 7; ++q) af[q] = lam[q];
      riemann_hlld_adj(ql, qr, x[16], gam, af, aql, aqr, abn);
      for (int q = 0; q < 8; ++q) { ad[q] = aql[q]; ad[8 + q] = aqr[q]; }
      ad[16] = abn;
    }
    double adot = 0.0;
    for (int i = 0; i < nin; ++i) adot += ad[i] * dx[i];
    const double e = rel(adot, fd);
    if (e > worst) worst = e;
  }
  return worst;
}

}  // extern "C"
