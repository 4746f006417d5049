// Device-side building blocks of the staggered (Kogut-Susskind) operator:
//   (D chi)(x) = m chi(x) + H chi(x),
//   (H chi)(x) = 1/2 sum_mu eta_mu(x) [ s+ U_mu(x) chi(x+mu) - s- U_mu(x-mu)^dag chi(x-mu) ]
// with eta_1 = 1, eta_2 = (-1)^x, eta_3 = (-1)^(x+y), eta_4 = (-1)^(x+y+z) and
// the boundary signs s+/s- of the Wilson operator.  H is anti-Hermitian and
// connects even and odd sites only, so D^dag D = m^2 - H^2 is block-diagonal
// and the even block M_e = m^2 - H_eo H_oe is Hermitian positive definite.
// Flop count per output site: 8 SU(3) x vector products (66 each) and 7
// vector sums (6 each) = 570 (the 1/2 folds into the epilogue coefficient).
#pragma once

#include "wd_device.h"

namespace wd {

template <typename T> struct cvec { cplx<T> c[3]; };

// One parity block of nrhs colour vectors over n sites: [colour][site][rhs]
// chunks of one complex each (double2 at FP64, float2 at FP32), so that
// consecutive lanes make coalesced accesses.  FP16 is not provided.
template <int P> struct SFmt;

template <> struct SFmt<F64> {
  WD_HD static size_t bytes(size_t ne) { return ne * 3 * 16; }
  WD_HD static void load(const void* base, size_t ne, size_t e, cvec<double>& v) {
    const double2* p = (const double2*)base;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double2 d = p[k * ne + e];
      v.c[k] = {d.x, d.y};
    }
  }
  WD_HD static void store(void* base, size_t ne, size_t e, const cvec<double>& v) {
    double2* p = (double2*)base;
#pragma unroll
    for (int k = 0; k < 3; ++k) p[k * ne + e] = make_double2(v.c[k].re, v.c[k].im);
  }
};

template <> struct SFmt<F32> {
  WD_HD static size_t bytes(size_t ne) { return ne * 3 * 8; }
  WD_HD static void load(const void* base, size_t ne, size_t e, cvec<float>& v) {
    const float2* p = (const float2*)base;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float2 d = p[k * ne + e];
      v.c[k] = {d.x, d.y};
    }
  }
  WD_HD static void store(void* base, size_t ne, size_t e, const cvec<float>& v) {
    float2* p = (float2*)base;
#pragma unroll
    for (int k = 0; k < 3; ++k) p[k * ne + e] = make_float2(v.c[k].re, v.c[k].im);
  }
};

template <typename T> WD_HD void cvec_zero(cvec<T>& v) {
#pragma unroll
  for (int k = 0; k < 3; ++k) v.c[k] = {T(0), T(0)};
}

template <typename T> WD_HD double cvec_norm2(const cvec<T>& v) {
  double a = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) a += (double)v.c[k].re * (double)v.c[k].re + (double)v.c[k].im * (double)v.c[k].im;
  return a;
}

// eta_mu(x) as +1 / -1.
WD_HD int stag_phase(const Coord& k, int mu) {
  int s = 0;
  if (mu > 0) s += k.c[0];
  if (mu > 1) s += k.c[1];
  if (mu > 2) s += k.c[2];
  return (s & 1) ? -1 : 1;
}

// acc += sign * (U v) (DIR > 0) or sign * (U^dag v) (DIR < 0); sign = +-1
// applied by choosing the add or the subtract.
template <typename T, int DIR>
WD_HD void stag_accumulate(const su3<T>& u, const cvec<T>& v, bool neg, cvec<T>& acc) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<T> s;
    if (DIR > 0) {
      s = cmul(u.e[3 * a], v.c[0]);
      s = cadd(s, cmul(u.e[3 * a + 1], v.c[1]));
      s = cadd(s, cmul(u.e[3 * a + 2], v.c[2]));
    } else {
      s = cjmul(u.e[a], v.c[0]);
      s = cadd(s, cjmul(u.e[3 + a], v.c[1]));
      s = cadd(s, cjmul(u.e[6 + a], v.c[2]));
    }
    acc.c[a] = neg ? csub(acc.c[a], s) : cadd(acc.c[a], s);
  }
}

// acc += eta_mu(x) * (+- boundary sign) * (U chi(x+mu) or -U^dag chi(x-mu)),
// without the factor 1/2.
template <int P, int R, int MU, int DIR, bool NT>
WD_HD void stag_dir(const Geom& g, const Coord& k, int parity, int s, int rhs, int nrhs, const char* gauge,
                    const void* in, float bc_sign, cvec<typename RealOf<P>::T>& acc) {
  using T = typename RealOf<P>::T;
  const size_t n = (size_t)g.n;
  const size_t ne = n * (size_t)nrhs;
  const int nb = neighbour_cb(g, k, MU, DIR);
  cvec<T> v;
  SFmt<P>::load(in, ne, (size_t)nb * nrhs + rhs, v);
  const int lp = DIR > 0 ? parity : 1 - parity;
  const size_t ls = DIR > 0 ? (size_t)s : (size_t)nb;
  su3<T> u;
  const char* lbase = gauge + (size_t)(lp * 4 + MU) * link_dir_bytes<P, R>(n);
  if constexpr (NT) LinkFmt<P, R>::load_nt(lbase, n, ls, u);
  else LinkFmt<P, R>::load(lbase, n, ls, u);
  const bool crosses = DIR > 0 ? (k.c[MU] == g.L[MU] - 1) : (k.c[MU] == 0);
  int sign = stag_phase(k, MU) * (DIR > 0 ? 1 : -1);
  if (crosses && bc_sign < 0.f) sign = -sign;
  stag_accumulate<T, DIR>(u, v, sign < 0, acc);
}

// Hops H0 .. H0 + NH - 1 of 2 (H in)(x), accumulated in hop order (hop h is
// direction h / 2, forward for even h and backward for odd h).
template <int P, int R, int H0, int NH, bool NT>
WD_HD void stag_hops(const Geom& g, const Coord& k, int parity, int s, int rhs, int nrhs, const char* gauge,
                     const void* in, const float bc[4], cvec<typename RealOf<P>::T>& acc) {
  if constexpr (NH > 0) {
    constexpr int MU = H0 >> 1;
    constexpr int DIR = (H0 & 1) ? -1 : 1;
    stag_dir<P, R, MU, DIR, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc[MU], acc);
    stag_hops<P, R, H0 + 1, NH - 1, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, acc);
  }
}

// Share `part` of the D shares (8 / D consecutive hops each) of 2 (H in)(x)
// at output site (parity, s) for one rhs; D = 1 is the whole sum.
template <int P, int R, int D, bool NT>
WD_HD void stag_site(const Geom& g, int parity, int s, int rhs, int nrhs, const char* gauge, const void* in,
                     const float bc[4], int part, cvec<typename RealOf<P>::T>& acc) {
  const Coord k = site_coord(g, parity, s);
  cvec_zero(acc);
  if constexpr (D == 1) {
    stag_hops<P, R, 0, 8, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, acc);
  } else if constexpr (D == 2) {
    if (part == 0) stag_hops<P, R, 0, 4, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, acc);
    else stag_hops<P, R, 4, 4, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, acc);
  } else {
    switch (part) {
      case 0: stag_hops<P, R, 0, 2, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, acc); break;
      case 1: stag_hops<P, R, 2, 2, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, acc); break;
      case 2: stag_hops<P, R, 4, 2, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, acc); break;
      default: stag_hops<P, R, 6, 2, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, acc); break;
    }
  }
}

}  // namespace wd
