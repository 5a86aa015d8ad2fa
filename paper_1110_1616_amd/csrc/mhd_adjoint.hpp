// Reverse-mode (adjoint) versions of the pointwise pieces of the advance,
// written by hand from the forward code in mhd_device.hpp.  Each function
// re-evaluates its forward pass, then propagates output adjoints back to its
// inputs with every branch (min/max choices, clamps, HLLD region and
// degeneracy tests, sign of B_n) frozen at the forward values.  Adjoints are
// accumulated (+=) into the caller's input-adjoint arrays.
#pragma once
#include "mhd_device.hpp"

namespace amr {

// fast_magnetosonic(r, p, b2, bn): adjoint of the returned speed.
template <class T>
__host__ __device__ __forceinline__ void fast_magnetosonic_adj(T r, T p, T b2, T bn, T gam, T a_cf, T& a_r, T& a_p,
                                                               T& a_b2, T& a_bn) {
  const T ir = drcp(r);
  const T gp = gam * p;
  const T a = (gp + b2) * ir;
  const T d0 = a * a - T(4) * gp * bn * bn * ir * ir;
  const bool pos = d0 > T(0);
  const T d = pos ? d0 : T(0);
  const T sd = psqrt(d);
  const T cf = psqrt(T(0.5) * (a + sd));
  const T a_cf2 = a_cf * T(0.5) * drcp(cf);
  T a_a = T(0.5) * a_cf2;
  const T a_sd = T(0.5) * a_cf2;
  const T a_d0 = (pos && sd > T(0)) ? a_sd * T(0.5) * drcp(sd) : T(0);
  a_a += T(2) * a * a_d0;
  T a_gp = -T(4) * bn * bn * ir * ir * a_d0;
  a_bn += -T(8) * gp * bn * ir * ir * a_d0;
  T a_ir = -T(8) * gp * bn * bn * ir * a_d0;
  a_gp += ir * a_a;
  a_b2 += ir * a_a;
  a_ir += (gp + b2) * a_a;
  a_p += gam * a_gp;
  a_r += -ir * ir * a_ir;
}

// to_primitive(u -> w): a_u += (dw/du)^T a_w.
template <class T>
__host__ __device__ __forceinline__ void to_primitive_adj(const T (&u)[8], T gm1, const T (&a_w)[8], T (&a_u)[8]) {
  const T ir = drcp(u[0]);
  const T w1 = u[1] * ir, w2 = u[2] * ir, w3 = u[3] * ir;
  const T v2 = w1 * w1 + w2 * w2 + w3 * w3;
  a_u[4] += gm1 * a_w[4];
  a_u[0] += a_w[0] - T(0.5) * gm1 * v2 * a_w[4];
  const T a_v2 = -T(0.5) * gm1 * u[0] * a_w[4];
  const T a_b2 = -T(0.5) * gm1 * a_w[4];
  const T a1 = a_w[1] + T(2) * w1 * a_v2;
  const T a2 = a_w[2] + T(2) * w2 * a_v2;
  const T a3 = a_w[3] + T(2) * w3 * a_v2;
  a_u[1] += ir * a1;
  a_u[2] += ir * a2;
  a_u[3] += ir * a3;
  const T a_ir = u[1] * a1 + u[2] * a2 + u[3] * a3;
  a_u[0] += -ir * ir * a_ir;
  a_u[5] += a_w[5] + T(2) * u[5] * a_b2;
  a_u[6] += a_w[6] + T(2) * u[6] * a_b2;
  a_u[7] += a_w[7] + T(2) * u[7] * a_b2;
}

// to_conserved(w -> u): a_w += (du/dw)^T a_u.
template <class T>
__host__ __device__ __forceinline__ void to_conserved_adj(const T (&w)[8], T gm1_inv, const T (&a_u)[8], T (&a_w)[8]) {
  const T v2 = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
  a_w[0] += a_u[0] + w[1] * a_u[1] + w[2] * a_u[2] + w[3] * a_u[3] + T(0.5) * v2 * a_u[4];
  a_w[1] += w[0] * a_u[1] + w[0] * w[1] * a_u[4];
  a_w[2] += w[0] * a_u[2] + w[0] * w[2] * a_u[4];
  a_w[3] += w[0] * a_u[3] + w[0] * w[3] * a_u[4];
  a_w[4] += gm1_inv * a_u[4];
  a_w[5] += a_u[5] + w[5] * a_u[4];
  a_w[6] += a_u[6] + w[6] * a_u[4];
  a_w[7] += a_u[7] + w[7] * a_u[4];
}

// flux_along<D>(w -> f): a_w += (df/dw)^T a_f (a_f[5+D] is ignored).
template <int D, class T>
__host__ __device__ __forceinline__ void flux_along_adj(const T (&w)[8], T gm1_inv, const T (&a_f)[8], T (&a_w)[8]) {
  const T r = w[0];
  const T vn = w[1 + D];
  const T bn = w[5 + D];
  const T v2 = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
  const T b2 = w[5] * w[5] + w[6] * w[6] + w[7] * w[7];
  const T pt = w[4] + T(0.5) * b2;
  const T e = w[4] * gm1_inv + T(0.5) * r * v2 + T(0.5) * b2;
  const T vb = w[1] * w[5] + w[2] * w[6] + w[3] * w[7];
  const T rvn = r * vn;
  T a_rvn = a_f[0];
  T a_vn = T(0), a_bn = T(0), a_pt = T(0), a_e = T(0), a_vb = T(0), a_r = T(0), a_v2 = T(0), a_b2 = T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    a_rvn += w[1 + a] * a_f[1 + a];
    a_w[1 + a] += rvn * a_f[1 + a];
    a_bn += -w[5 + a] * a_f[1 + a];
    a_w[5 + a] += -bn * a_f[1 + a];
  }
  a_pt += a_f[1 + D];
  a_e += vn * a_f[4];
  a_pt += vn * a_f[4];
  a_vn += (e + pt) * a_f[4];
  a_bn += -vb * a_f[4];
  a_vb += -bn * a_f[4];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a == D) continue;
    a_w[5 + a] += vn * a_f[5 + a];
    a_vn += w[5 + a] * a_f[5 + a];
    a_bn += -w[1 + a] * a_f[5 + a];
    a_w[1 + a] += -bn * a_f[5 + a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    a_w[1 + a] += w[5 + a] * a_vb;
    a_w[5 + a] += w[1 + a] * a_vb;
  }
  a_w[4] += gm1_inv * a_e;
  a_r += T(0.5) * v2 * a_e;
  a_v2 += T(0.5) * r * a_e;
  a_b2 += T(0.5) * a_e;
  a_w[4] += a_pt;
  a_b2 += T(0.5) * a_pt;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    a_w[1 + a] += T(2) * w[1 + a] * a_v2;
    a_w[5 + a] += T(2) * w[5 + a] * a_b2;
  }
  a_r += vn * a_rvn;
  a_vn += r * a_rvn;
  a_w[1 + D] += a_vn;
  a_w[5 + D] += a_bn;
  a_w[0] += a_r;
}

// HLLD adjoint: given a_f (7), accumulate into a_ql, a_qr (slots 0..4, 6, 7
// of the rotated states; slot 5 unused) and a_bn.
template <class T>
__host__ __device__ void riemann_hlld_adj(const T (&ql)[8], const T (&qr)[8], T bn, T gam, const T (&a_f)[7],
                                          T (&a_ql)[8], T (&a_qr)[8], T& a_bn) {
  // ---------------- forward (same arithmetic as riemann_hlld) ----------------
  const T g1i = drcp(gam - T(1));
  const T bn2 = bn * bn;
  const T rl = ql[0], ul = ql[1], vl = ql[2], wl = ql[3], pl = ql[4], byl = ql[6], bzl = ql[7];
  const T rr = qr[0], ur = qr[1], vr = qr[2], wr = qr[3], pr = qr[4], byr = qr[6], bzr = qr[7];
  const T b2l = bn2 + byl * byl + bzl * bzl;
  const T b2r = bn2 + byr * byr + bzr * bzr;
  const T ptl = pl + T(0.5) * b2l;
  const T ptr = pr + T(0.5) * b2r;
  const T kl = ul * ul + vl * vl + wl * wl;
  const T kr = ur * ur + vr * vr + wr * wr;
  const T el = pl * g1i + T(0.5) * rl * kl + T(0.5) * b2l;
  const T er = pr * g1i + T(0.5) * rr * kr + T(0.5) * b2r;
  const T cfl = fast_magnetosonic(rl, pl, b2l, bn, gam);
  const T cfr = fast_magnetosonic(rr, pr, b2r, bn, gam);
  const bool cl_big = cfl > cfr;
  const T cmx = cl_big ? cfl : cfr;
  const bool ul_lt = ul < ur;
  const bool ul_gt = ul > ur;
  const T sl = (ul_lt ? ul : ur) - cmx;
  const T sr = (ul_gt ? ul : ur) + cmx;
  const T dl = sl - ul, dr = sr - ur;
  const T rdl = rl * dl, rdr = rr * dr;
  const T num = rdr * ur - rdl * ul - ptr + ptl;
  const T den = rdr - rdl;
  const T sm = num * drcp(den);
  const T pts = ptl + rdl * (sm - ul);
  const T tiny = T(1e-12) * pts;

  struct Side {
    T d, rd, dsm, idsm, rs, dn, idn, smu, fv, qq, fb, vs, ws, bys, bzs, vb, vbs, x, es;
    bool deg;
  };
  auto star = [&](T r, T u, T v, T w, T by, T bz, T e, T pt, T s, T rd) {
    Side o;
    o.d = s - u;
    o.rd = rd;
    o.dsm = s - sm;
    o.idsm = drcp(o.dsm);
    o.rs = rd * o.idsm;
    o.dn = rd * o.dsm - bn2;
    o.deg = dabs(o.dn) <= tiny;
    o.idn = o.deg ? T(0) : drcp(o.dn);
    o.smu = sm - u;
    o.fv = bn * o.smu * o.idn;
    o.qq = rd * o.d - bn2;
    o.fb = o.qq * o.idn;
    o.vs = o.deg ? v : v - by * o.fv;
    o.ws = o.deg ? w : w - bz * o.fv;
    o.bys = o.deg ? by : by * o.fb;
    o.bzs = o.deg ? bz : bz * o.fb;
    o.vb = u * bn + v * by + w * bz;
    o.vbs = sm * bn + o.vs * o.bys + o.ws * o.bzs;
    o.x = o.d * e - pt * u + pts * sm + bn * (o.vb - o.vbs);
    o.es = o.x * o.idsm;
    (void)r;
    return o;
  };
  const Side L = star(rl, ul, vl, wl, byl, bzl, el, ptl, sl, rdl);
  const Side R = star(rr, ur, vr, wr, byr, bzr, er, ptr, sr, rdr);
  const T sql = psqrt(L.rs), sqr = psqrt(R.rs);
  const T sb = bn < T(0) ? T(-1) : T(1);  // d|bn|/dbn
  const T abn = dabs(bn);
  const T ssl = sm - abn * drcp(sql);
  const T ssr = sm + abn * drcp(sqr);
  const bool ddeg = T(0.5) * bn2 <= tiny;
  const T sg = bn > T(0) ? T(1) : T(-1);
  const T isum = drcp(sql + sqr);
  const T nv = sql * L.vs + sqr * R.vs + (R.bys - L.bys) * sg;
  const T nw = sql * L.ws + sqr * R.ws + (R.bzs - L.bzs) * sg;
  const T nby = sql * R.bys + sqr * L.bys + sql * sqr * (R.vs - L.vs) * sg;
  const T nbz = sql * R.bzs + sqr * L.bzs + sql * sqr * (R.ws - L.ws) * sg;
  const T vss = nv * isum, wss = nw * isum, byss = nby * isum, bzss = nbz * isum;
  const T vbss = sm * bn + vss * byss + wss * bzss;
  // essl = esl - sql (vbsl - vbss) sg ; essr = esr + sqr (vbsr - vbss) sg
  int region;
  if (sl > T(0)) region = 0;
  else if (ssl >= T(0)) region = 1;
  else if (sm >= T(0)) region = 2;
  else if (ssr >= T(0)) region = 3;
  else if (sr >= T(0)) region = 4;
  else region = 5;
  const bool left = region <= 2;

  // ---------------- reverse ----------------
  // adjoints of shared intermediates
  T a_sm = T(0), a_pts = T(0), a_sql = T(0), a_sqr = T(0);
  T a_vss = T(0), a_wss = T(0), a_byss = T(0), a_bzss = T(0);
  T a_sl = T(0), a_sr = T(0), a_ssl = T(0), a_ssr = T(0);
  // per side star adjoints
  T aL_rs = T(0), aL_vs = T(0), aL_ws = T(0), aL_bys = T(0), aL_bzs = T(0), aL_es = T(0);
  T aR_rs = T(0), aR_vs = T(0), aR_ws = T(0), aR_bys = T(0), aR_bzs = T(0), aR_es = T(0);
  // outer state adjoints (side of the base flux)
  T a_r0 = T(0), a_u0 = T(0), a_v0 = T(0), a_w0 = T(0), a_by0 = T(0), a_bz0 = T(0), a_e0 = T(0), a_pt0 = T(0);
  T a_bnl = T(0);  // local accumulator of a_bn
  T a_bn2 = T(0);

  const T r0 = left ? rl : rr, u0 = left ? ul : ur, v0 = left ? vl : vr, w0 = left ? wl : wr;
  const T by0 = left ? byl : byr, bz0 = left ? bzl : bzr, e0 = left ? el : er, pt0 = left ? ptl : ptr;
  const T ru = r0 * u0;

  // f += ss * (U** - U*) for regions 2, 3
  if (region == 2 || region == 3) {
    const bool lft = region == 2;
    const Side& S = lft ? L : R;
    const T ss = lft ? ssl : ssr;
    T a_vssx = T(0), a_wssx = T(0), a_byssx = T(0), a_bzssx = T(0), a_essx = T(0);
    // f2 += ss*rs*(vss2 - vs); f3 += ss*rs*(wss2 - ws); f4 += ss*(ess2 - es);
    // f5 += ss*(byss2 - bys); f6 += ss*(bzss2 - bzs)
    const T vss2 = ddeg ? S.vs : vss, wss2 = ddeg ? S.ws : wss, byss2 = ddeg ? S.bys : byss,
            bzss2 = ddeg ? S.bzs : bzss;
    const T essx = ddeg ? S.es
                        : (lft ? S.es - sql * (S.vbs - vbss) * sg : S.es + sqr * (S.vbs - vbss) * sg);
    T a_ss = a_f[2] * S.rs * (vss2 - S.vs) + a_f[3] * S.rs * (wss2 - S.ws) + a_f[4] * (essx - S.es) +
             a_f[5] * (byss2 - S.bys) + a_f[6] * (bzss2 - S.bzs);
    T a_rs = a_f[2] * ss * (vss2 - S.vs) + a_f[3] * ss * (wss2 - S.ws);
    a_vssx += a_f[2] * ss * S.rs;
    a_wssx += a_f[3] * ss * S.rs;
    a_essx += a_f[4] * ss;
    a_byssx += a_f[5] * ss;
    a_bzssx += a_f[6] * ss;
    T a_vs = -a_f[2] * ss * S.rs, a_ws = -a_f[3] * ss * S.rs, a_es = -a_f[4] * ss, a_bys = -a_f[5] * ss,
      a_bzs = -a_f[6] * ss;
    T a_vbs = T(0);
    if (ddeg) {
      a_vs += a_vssx;
      a_ws += a_wssx;
      a_bys += a_byssx;
      a_bzs += a_bzssx;
      a_es += a_essx;
    } else {
      a_vss += a_vssx;
      a_wss += a_wssx;
      a_byss += a_byssx;
      a_bzss += a_bzssx;
      // essx = es -+ sq (vbs - vbss) sg
      a_es += a_essx;
      const T sgn = lft ? T(-1) : T(1);
      const T sq = lft ? sql : sqr;
      const T a_sq = sgn * a_essx * (S.vbs - vbss) * sg;
      if (lft) a_sql += a_sq;
      else a_sqr += a_sq;
      a_vbs += sgn * a_essx * sq * sg;
      const T a_vbss = -sgn * a_essx * sq * sg;
      // vbss = sm bn + vss byss + wss bzss
      a_sm += a_vbss * bn;
      a_bnl += a_vbss * sm;
      a_vss += a_vbss * byss;
      a_byss += a_vbss * vss;
      a_wss += a_vbss * bzss;
      a_bzss += a_vbss * wss;
    }
    // ss = sm -+ |bn| / sq
    a_sm += a_ss;
    if (lft) {
      a_ssl += a_ss;
    } else {
      a_ssr += a_ss;
    }
    if (lft) {
      aL_rs += a_rs; aL_vs += a_vs; aL_ws += a_ws; aL_es += a_es; aL_bys += a_bys; aL_bzs += a_bzs;
    } else {
      aR_rs += a_rs; aR_vs += a_vs; aR_ws += a_ws; aR_es += a_es; aR_bys += a_bys; aR_bzs += a_bzs;
    }
    // apply vbs adjoint now (vbs depends on sm, bn, vs, bys, ws, bzs of the side)
    a_sm += a_vbs * bn;
    a_bnl += a_vbs * sm;
    if (lft) {
      aL_vs += a_vbs * S.bys; aL_bys += a_vbs * S.vs; aL_ws += a_vbs * S.bzs; aL_bzs += a_vbs * S.ws;
    } else {
      aR_vs += a_vbs * S.bys; aR_bys += a_vbs * S.vs; aR_ws += a_vbs * S.bzs; aR_bzs += a_vbs * S.ws;
    }
  }
  // ss adjoints: ssl = sm - |bn|/sql ; ssr = sm + |bn|/sqr  (the a_sm part is
  // already added above; here the |bn| and sq parts)
  if (a_ssl != T(0)) {
    a_bnl += -a_ssl * sb / sql;
    a_sql += a_ssl * abn / (sql * sql);
  }
  if (a_ssr != T(0)) {
    a_bnl += a_ssr * sb / sqr;
    a_sqr += -a_ssr * abn / (sqr * sqr);
  }
  // double-star averages (only if used)
  if (a_vss != T(0) || a_wss != T(0) || a_byss != T(0) || a_bzss != T(0)) {
    const T a_nv = a_vss * isum, a_nw = a_wss * isum, a_nby = a_byss * isum, a_nbz = a_bzss * isum;
    const T a_isum = a_vss * nv + a_wss * nw + a_byss * nby + a_bzss * nbz;
    // isum = 1/(sql + sqr)
    const T a_den2 = -a_isum * isum * isum;
    a_sql += a_den2;
    a_sqr += a_den2;
    // nv = sql vsl + sqr vsr + (bysr - bysl) sg
    a_sql += a_nv * L.vs;
    aL_vs += a_nv * sql;
    a_sqr += a_nv * R.vs;
    aR_vs += a_nv * sqr;
    aR_bys += a_nv * sg;
    aL_bys += -a_nv * sg;
    a_sql += a_nw * L.ws;
    aL_ws += a_nw * sql;
    a_sqr += a_nw * R.ws;
    aR_ws += a_nw * sqr;
    aR_bzs += a_nw * sg;
    aL_bzs += -a_nw * sg;
    // nby = sql bysr + sqr bysl + sql sqr (vsr - vsl) sg
    a_sql += a_nby * (R.bys + sqr * (R.vs - L.vs) * sg);
    a_sqr += a_nby * (L.bys + sql * (R.vs - L.vs) * sg);
    aR_bys += a_nby * sql;
    aL_bys += a_nby * sqr;
    aR_vs += a_nby * sql * sqr * sg;
    aL_vs += -a_nby * sql * sqr * sg;
    a_sql += a_nbz * (R.bzs + sqr * (R.ws - L.ws) * sg);
    a_sqr += a_nbz * (L.bzs + sql * (R.ws - L.ws) * sg);
    aR_bzs += a_nbz * sql;
    aL_bzs += a_nbz * sqr;
    aR_ws += a_nbz * sql * sqr * sg;
    aL_ws += -a_nbz * sql * sqr * sg;
  }
  // f += s * (U* - U) for regions 1..4, and the base physical flux
  if (region >= 1 && region <= 4) {
    const bool lft = left;
    const Side& S = lft ? L : R;
    const T s = lft ? sl : sr;
    const T j0 = S.rs - r0, j1 = S.rs * sm - ru, j2 = S.rs * S.vs - r0 * v0, j3 = S.rs * S.ws - r0 * w0,
            j4 = S.es - e0, j5 = S.bys - by0, j6 = S.bzs - bz0;
    const T a_s = a_f[0] * j0 + a_f[1] * j1 + a_f[2] * j2 + a_f[3] * j3 + a_f[4] * j4 + a_f[5] * j5 + a_f[6] * j6;
    if (lft) a_sl += a_s;
    else a_sr += a_s;
    T a_rs = a_f[0] * s + a_f[1] * s * sm + a_f[2] * s * S.vs + a_f[3] * s * S.ws;
    a_sm += a_f[1] * s * S.rs;
    T a_ru_j = -a_f[1] * s;
    a_r0 += -a_f[0] * s - a_f[2] * s * v0 - a_f[3] * s * w0;
    a_v0 += -a_f[2] * s * r0;
    a_w0 += -a_f[3] * s * r0;
    a_e0 += -a_f[4] * s;
    a_by0 += -a_f[5] * s;
    a_bz0 += -a_f[6] * s;
    if (lft) {
      aL_rs += a_rs; aL_vs += a_f[2] * s * S.rs; aL_ws += a_f[3] * s * S.rs; aL_es += a_f[4] * s;
      aL_bys += a_f[5] * s; aL_bzs += a_f[6] * s;
    } else {
      aR_rs += a_rs; aR_vs += a_f[2] * s * S.rs; aR_ws += a_f[3] * s * S.rs; aR_es += a_f[4] * s;
      aR_bys += a_f[5] * s; aR_bzs += a_f[6] * s;
    }
    // ru = r0 u0
    a_r0 += a_ru_j * u0;
    a_u0 += a_ru_j * r0;
  }
  {
    // base flux: f0 = ru; f1 = ru u0 + pt0 - bn2; f2 = ru v0 - bn by0; f3 = ru w0 - bn bz0;
    // f4 = (e0 + pt0) u0 - bn vb0; f5 = by0 u0 - bn v0; f6 = bz0 u0 - bn w0
    const T vb0 = u0 * bn + v0 * by0 + w0 * bz0;
    T a_ru = a_f[0] + a_f[1] * u0 + a_f[2] * v0 + a_f[3] * w0;
    a_u0 += a_f[1] * ru;
    a_pt0 += a_f[1];
    a_bn2 += -a_f[1];
    a_v0 += a_f[2] * ru;
    a_bnl += -a_f[2] * by0 - a_f[3] * bz0;
    a_by0 += -a_f[2] * bn;
    a_w0 += a_f[3] * ru;
    a_bz0 += -a_f[3] * bn;
    a_e0 += a_f[4] * u0;
    a_pt0 += a_f[4] * u0;
    a_u0 += a_f[4] * (e0 + pt0);
    a_bnl += -a_f[4] * vb0;
    const T a_vb0 = -a_f[4] * bn;
    a_u0 += a_vb0 * bn;
    a_bnl += a_vb0 * u0;
    a_v0 += a_vb0 * by0;
    a_by0 += a_vb0 * v0;
    a_w0 += a_vb0 * bz0;
    a_bz0 += a_vb0 * w0;
    a_by0 += a_f[5] * u0;
    a_u0 += a_f[5] * by0;
    a_bnl += -a_f[5] * v0 - a_f[6] * w0;
    a_v0 += -a_f[5] * bn;
    a_bz0 += a_f[6] * u0;
    a_u0 += a_f[6] * bz0;
    a_w0 += -a_f[6] * bn;
    a_r0 += a_ru * u0;
    a_u0 += a_ru * r0;
  }
  // sqrt of the star densities
  aL_rs += a_sql * T(0.5) / sql;
  aR_rs += a_sqr * T(0.5) / sqr;

  // outer-state adjoints to accumulate (side of the base flux)
  T aLq[8] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
  T aRq[8] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
  T a_el = T(0), a_er = T(0), a_ptl = T(0), a_ptr = T(0);
  {
    T(&aq)[8] = left ? aLq : aRq;
    aq[0] += a_r0;
    aq[1] += a_u0;
    aq[2] += a_v0;
    aq[3] += a_w0;
    aq[6] += a_by0;
    aq[7] += a_bz0;
    if (left) {
      a_el += a_e0;
      a_ptl += a_pt0;
    } else {
      a_er += a_e0;
      a_ptr += a_pt0;
    }
  }

  // star states, reverse of `star` for each side
  auto star_adj = [&](const Side& o, T r, T u, T v, T w, T by, T bz, T e, T pt, T a_rs, T a_vs, T a_ws, T a_bys,
                      T a_bzs, T a_es, T (&aq)[8], T& a_e, T& a_pt, T& a_s, T& a_rd) {
    (void)r;
    // es = x idsm
    T a_x = a_es * o.idsm;
    T a_idsm = a_es * o.x;
    // x = d e - pt u + pts sm + bn (vb - vbs)
    T a_d = a_x * e;
    a_e += a_x * o.d;
    a_pt += -a_x * u;
    aq[1] += -a_x * pt;
    a_pts += a_x * sm;
    a_sm += a_x * pts;
    a_bnl += a_x * (o.vb - o.vbs);
    T a_vb = a_x * bn;
    T a_vbs = -a_x * bn;
    // vbs = sm bn + vs bys + ws bzs
    a_sm += a_vbs * bn;
    a_bnl += a_vbs * sm;
    a_vs += a_vbs * o.bys;
    a_bys += a_vbs * o.vs;
    a_ws += a_vbs * o.bzs;
    a_bzs += a_vbs * o.ws;
    // vb = u bn + v by + w bz
    aq[1] += a_vb * bn;
    a_bnl += a_vb * u;
    aq[2] += a_vb * by;
    aq[6] += a_vb * v;
    aq[3] += a_vb * bz;
    aq[7] += a_vb * w;
    // tangential star values
    T a_fv = T(0), a_fb = T(0);
    if (o.deg) {
      aq[2] += a_vs;
      aq[3] += a_ws;
      aq[6] += a_bys;
      aq[7] += a_bzs;
    } else {
      aq[2] += a_vs;
      aq[6] += -a_vs * o.fv;
      a_fv += -a_vs * by;
      aq[3] += a_ws;
      aq[7] += -a_ws * o.fv;
      a_fv += -a_ws * bz;
      aq[6] += a_bys * o.fb;
      a_fb += a_bys * by;
      aq[7] += a_bzs * o.fb;
      a_fb += a_bzs * bz;
    }
    // fb = qq idn, qq = rd d - bn2; fv = bn smu idn
    T a_idn = a_fb * o.qq + a_fv * bn * o.smu;
    T a_qq = a_fb * o.idn;
    a_bnl += a_fv * o.smu * o.idn;
    T a_smu = a_fv * bn * o.idn;
    a_rd += a_qq * o.d;
    a_d += a_qq * o.rd;
    a_bn2 += -a_qq;
    // smu = sm - u
    a_sm += a_smu;
    aq[1] += -a_smu;
    // idn = 1/dn (0 when degenerate)
    T a_dn = o.deg ? T(0) : -a_idn * o.idn * o.idn;
    // dn = rd dsm - bn2
    a_rd += a_dn * o.dsm;
    T a_dsm = a_dn * o.rd;
    a_bn2 += -a_dn;
    // rs = rd idsm
    a_rd += a_rs * o.idsm;
    a_idsm += a_rs * o.rd;
    // idsm = 1/dsm
    a_dsm += -a_idsm * o.idsm * o.idsm;
    // dsm = s - sm
    a_s += a_dsm;
    a_sm += -a_dsm;
    // d = s - u
    a_s += a_d;
    aq[1] += -a_d;
  };
  T a_rdl = T(0), a_rdr = T(0);
  star_adj(L, rl, ul, vl, wl, byl, bzl, el, ptl, aL_rs, aL_vs, aL_ws, aL_bys, aL_bzs, aL_es, aLq, a_el, a_ptl, a_sl,
           a_rdl);
  star_adj(R, rr, ur, vr, wr, byr, bzr, er, ptr, aR_rs, aR_vs, aR_ws, aR_bys, aR_bzs, aR_es, aRq, a_er, a_ptr, a_sr,
           a_rdr);
  // pts = ptl + rdl (sm - ul)
  a_ptl += a_pts;
  a_rdl += a_pts * (sm - ul);
  a_sm += a_pts * rdl;
  aLq[1] += -a_pts * rdl;
  // sm = num / den
  const T a_num = a_sm / den;
  const T a_den = -a_sm * sm / den;
  // num = rdr ur - rdl ul - ptr + ptl ; den = rdr - rdl
  a_rdr += a_num * ur + a_den;
  aRq[1] += a_num * rdr;
  a_rdl += -a_num * ul - a_den;
  aLq[1] += -a_num * rdl;
  a_ptr += -a_num;
  a_ptl += a_num;
  // rdl = rl dl, dl = sl - ul ; rdr = rr dr, dr = sr - ur
  aLq[0] += a_rdl * dl;
  const T a_dl = a_rdl * rl;
  aRq[0] += a_rdr * dr;
  const T a_dr = a_rdr * rr;
  a_sl += a_dl;
  aLq[1] += -a_dl;
  a_sr += a_dr;
  aRq[1] += -a_dr;
  // sl = min(ul, ur) - cmx ; sr = max(ul, ur) + cmx
  if (ul_lt) aLq[1] += a_sl;
  else aRq[1] += a_sl;
  if (ul_gt) aLq[1] += a_sr;
  else aRq[1] += a_sr;
  const T a_cmx = -a_sl + a_sr;
  T a_b2l = T(0), a_b2r = T(0);
  if (cl_big)
    fast_magnetosonic_adj(rl, pl, b2l, bn, gam, a_cmx, aLq[0], aLq[4], a_b2l, a_bnl);
  else
    fast_magnetosonic_adj(rr, pr, b2r, bn, gam, a_cmx, aRq[0], aRq[4], a_b2r, a_bnl);
  // el = pl g1i + 0.5 rl kl + 0.5 b2l
  aLq[4] += a_el * g1i;
  aLq[0] += a_el * T(0.5) * kl;
  aLq[1] += a_el * rl * ul;
  aLq[2] += a_el * rl * vl;
  aLq[3] += a_el * rl * wl;
  a_b2l += a_el * T(0.5);
  aRq[4] += a_er * g1i;
  aRq[0] += a_er * T(0.5) * kr;
  aRq[1] += a_er * rr * ur;
  aRq[2] += a_er * rr * vr;
  aRq[3] += a_er * rr * wr;
  a_b2r += a_er * T(0.5);
  // ptl = pl + 0.5 b2l
  aLq[4] += a_ptl;
  a_b2l += T(0.5) * a_ptl;
  aRq[4] += a_ptr;
  a_b2r += T(0.5) * a_ptr;
  // b2 = bn2 + by^2 + bz^2
  a_bn2 += a_b2l + a_b2r;
  aLq[6] += T(2) * byl * a_b2l;
  aLq[7] += T(2) * bzl * a_b2l;
  aRq[6] += T(2) * byr * a_b2r;
  aRq[7] += T(2) * bzr * a_b2r;
  a_bnl += T(2) * bn * a_bn2;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    a_ql[q] += aLq[q];
    a_qr[q] += aRq[q];
  }
  a_bn += a_bnl;
}

}  // namespace amr
