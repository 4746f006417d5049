// Device-side building blocks of the Wilson-Dirac stencil: storage formats,
// checkerboard geometry, spin projection and SU(3) products.
//
// Every function here is __host__ __device__ so that the per-site arithmetic
// can also be driven from a plain CPU loop when checking indexing.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <utility>

#define WD_HD __host__ __device__ __forceinline__

#include "wd_fastdiv.h"

// Native vector type for non-temporal loads (the builtin takes clang vectors).
typedef double wd_nt_d2 __attribute__((ext_vector_type(2)));
typedef float wd_nt_f2 __attribute__((ext_vector_type(2)));
typedef float wd_nt_f4 __attribute__((ext_vector_type(4)));
typedef unsigned int wd_nt_u2 __attribute__((ext_vector_type(2)));
typedef unsigned int wd_nt_u4 __attribute__((ext_vector_type(4)));

namespace wd {

enum Prec : int { F64 = 0, F32 = 1, F16 = 2 };

template <int P> struct RealOf { using T = float; };
template <> struct RealOf<F64> { using T = double; };

template <typename T> struct cplx { T re, im; };

template <typename T> WD_HD cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename T> WD_HD cplx<T> cjmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T> WD_HD cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> WD_HD cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
// a + i b, a - i b
template <typename T> WD_HD cplx<T> cadd_i(cplx<T> a, cplx<T> b) { return {a.re - b.im, a.im + b.re}; }
template <typename T> WD_HD cplx<T> csub_i(cplx<T> a, cplx<T> b) { return {a.re + b.im, a.im - b.re}; }
template <typename T> WD_HD cplx<T> cneg(cplx<T> a) { return {-a.re, -a.im}; }
template <typename T> WD_HD cplx<T> ctimes_i(cplx<T> a) { return {-a.im, a.re}; }     // i a
template <typename T> WD_HD cplx<T> ctimes_mi(cplx<T> a) { return {a.im, -a.re}; }    // -i a
template <typename T> WD_HD cplx<T> cconj(cplx<T> a) { return {a.re, -a.im}; }
template <typename T> WD_HD cplx<T> cscale(cplx<T> a, T s) { return {a.re * s, a.im * s}; }

// A complex as a pair of halves (re, im), for the FP16 stencil.
typedef _Float16 wd_h2 __attribute__((ext_vector_type(2)));
typedef __fp16 wd_hp2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ wd_h2 cadd(wd_h2 a, wd_h2 b) { return a + b; }
__device__ __forceinline__ wd_h2 csub(wd_h2 a, wd_h2 b) { return a - b; }
__device__ __forceinline__ wd_h2 cadd_i(wd_h2 a, wd_h2 b) { return a + (wd_h2){-b.y, b.x}; }  // a + i b
__device__ __forceinline__ wd_h2 csub_i(wd_h2 a, wd_h2 b) { return a + (wd_h2){b.y, -b.x}; }  // a - i b
__device__ __forceinline__ wd_h2 h2_conj(wd_h2 v) {
  return __builtin_bit_cast(wd_h2, __builtin_bit_cast(uint32_t, v) ^ 0x80000000u);
}
__device__ __forceinline__ wd_h2 h2_swap(wd_h2 v) { return v.yx; }
__device__ __forceinline__ wd_h2 h2_bits(uint32_t u) { return __builtin_bit_cast(wd_h2, u); }
__device__ __forceinline__ float dot2h(wd_h2 a, wd_h2 b, float c) {
  return __builtin_amdgcn_fdot2(__builtin_bit_cast(wd_hp2, a), __builtin_bit_cast(wd_hp2, b), c, false);
}

// A full spinor: 4 spins x 3 colours; component k = 3*spin + colour.
template <typename T> struct spinor { cplx<T> c[12]; };
// A half spinor after spin projection: 2 spins x 3 colours.
template <typename T> struct half_spinor { cplx<T> c[6]; };
template <typename T> struct su3 { cplx<T> e[9]; };  // row-major e[3*row + col]

// ---------------------------------------------------------------------------
// Spinor vectors.  One parity block of nrhs fields over n sites is stored as
// [chunk][site][rhs] of 16-byte chunks (consecutive lanes -> consecutive
// (site, rhs) -> coalesced 16-byte accesses):
//   F64: 12 chunks of double2 (one complex each)
//   F32:  6 chunks of float4  (two complexes each)
//   F16:  3 chunks of 8 halves (four complexes each), followed by one float
//         scale per (site, rhs): stored value = component / scale, where the
//         scale is the largest |real or imaginary part| of the site's 24 reals.
// ---------------------------------------------------------------------------
template <int P> struct SpinorFmt;

template <> struct SpinorFmt<F64> {
  static constexpr int chunks = 12;
  WD_HD static size_t bytes(size_t ne) { return ne * 12 * 16; }
  WD_HD static void load(const void* base, size_t ne, size_t e, spinor<double>& s) {
    const double2* v = (const double2*)base;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      double2 d = v[k * ne + e];
      s.c[k] = {d.x, d.y};
    }
  }
  WD_HD static void store(void* base, size_t ne, size_t e, const spinor<double>& s) {
    double2* v = (double2*)base;
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k * ne + e] = make_double2(s.c[k].re, s.c[k].im);
  }
  // components c0 .. c0+NK-1 only
  template <int NK> WD_HD static void load_comps(const void* base, size_t ne, size_t e, int c0, cplx<double>* s) {
    const double2* v = (const double2*)base;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const double2 d = v[(size_t)(c0 + k) * ne + e];
      s[k] = {d.x, d.y};
    }
  }
  template <int NK> WD_HD static void store_comps(void* base, size_t ne, size_t e, int c0, const cplx<double>* s) {
    double2* v = (double2*)base;
#pragma unroll
    for (int k = 0; k < NK; ++k) v[(size_t)(c0 + k) * ne + e] = make_double2(s[k].re, s[k].im);
  }
};

template <> struct SpinorFmt<F32> {
  static constexpr int chunks = 6;
  WD_HD static size_t bytes(size_t ne) { return ne * 6 * 16; }
  WD_HD static void load(const void* base, size_t ne, size_t e, spinor<float>& s) {
    const float4* v = (const float4*)base;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float4 d = v[k * ne + e];
      s.c[2 * k] = {d.x, d.y};
      s.c[2 * k + 1] = {d.z, d.w};
    }
  }
  WD_HD static void store(void* base, size_t ne, size_t e, const spinor<float>& s) {
    float4* v = (float4*)base;
#pragma unroll
    for (int k = 0; k < 6; ++k)
      v[k * ne + e] = make_float4(s.c[2 * k].re, s.c[2 * k].im, s.c[2 * k + 1].re, s.c[2 * k + 1].im);
  }
  // components c0 .. c0+NK-1 only (c0 and NK even: whole chunks)
  template <int NK> WD_HD static void load_comps(const void* base, size_t ne, size_t e, int c0, cplx<float>* s) {
    static_assert(NK % 2 == 0, "whole chunks");
    const float4* v = (const float4*)base;
#pragma unroll
    for (int k = 0; k < NK / 2; ++k) {
      const float4 d = v[(size_t)(c0 / 2 + k) * ne + e];
      s[2 * k] = {d.x, d.y};
      s[2 * k + 1] = {d.z, d.w};
    }
  }
  template <int NK> WD_HD static void store_comps(void* base, size_t ne, size_t e, int c0, const cplx<float>* s) {
    static_assert(NK % 2 == 0, "whole chunks");
    float4* v = (float4*)base;
#pragma unroll
    for (int k = 0; k < NK / 2; ++k)
      v[(size_t)(c0 / 2 + k) * ne + e] = make_float4(s[2 * k].re, s[2 * k].im, s[2 * k + 1].re, s[2 * k + 1].im);
  }
};

union h8 {
  uint4 u;
  __half2 h[4];
};

template <> struct SpinorFmt<F16> {
  static constexpr int chunks = 3;
  WD_HD static size_t data_bytes(size_t ne) { return ne * 3 * 16; }
  WD_HD static size_t bytes(size_t ne) { return data_bytes(ne) + ne * 4; }
  WD_HD static void load(const void* base, size_t ne, size_t e, spinor<float>& s) {
    const uint4* v = (const uint4*)base;
    const float* sc = (const float*)((const char*)base + data_bytes(ne));
    float a = sc[e];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      h8 d;
      d.u = v[k * ne + e];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float2 f = __half22float2(d.h[j]);
        s.c[4 * k + j] = {f.x * a, f.y * a};
      }
    }
  }
  WD_HD static void store(void* base, size_t ne, size_t e, const spinor<float>& s) {
    uint4* v = (uint4*)base;
    float* sc = (float*)((char*)base + data_bytes(ne));
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(s.c[k].re), fabsf(s.c[k].im)));
    // A site whose largest component is below the smallest normal float is
    // stored as zero: 1/m would overflow to infinity and poison the site
    // (such sites appear at the edge of a point source's support).
    if (m < 1.17549435e-38f) m = 0.f;
    const float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      h8 d;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        d.h[j] = __floats2half2_rn(s.c[4 * k + j].re * inv, s.c[4 * k + j].im * inv);
      v[k * ne + e] = d.u;
    }
    sc[e] = m;
  }
};

// ---------------------------------------------------------------------------
// Links.  One store holds [parity][mu][chunk][site] for the links rooted at
// each site (U_mu(x) lives with site x), n sites per parity.
//   recon 18: all nine complexes; recon 12: rows 0 and 1, the third row is
//   rebuilt as conj(row0 x row1), exact for SU(3).
//   F64: double2 per complex.  F32-18: float2 per complex; F32-12: float4 per
//   complex pair.  F16-18: half2 per complex; F16-12: 8 halves (complexes
//   0..3) plus 4 halves (complexes 4..5).
// ---------------------------------------------------------------------------
template <int P, int R> struct LinkFmt;

template <typename T> WD_HD void reconstruct_row2(su3<T>& u) {
  // row2 = conj(row0 x row1)
  u.e[6] = cconj(csub(cmul(u.e[1], u.e[5]), cmul(u.e[2], u.e[4])));
  u.e[7] = cconj(csub(cmul(u.e[2], u.e[3]), cmul(u.e[0], u.e[5])));
  u.e[8] = cconj(csub(cmul(u.e[0], u.e[4]), cmul(u.e[1], u.e[3])));
}

// FP64 and FP32 links: `load` is an ordinary load; `load_nt` carries the
// non-temporal hint.  Each link is used once per stencil launch; the launcher
// picks the hinted loads when the links cannot stay in the Infinity Cache
// until the next launch (stream_links), so that they do not evict the
// neighbour spinors that are reused.
template <int R> struct LinkFmt<F64, R> {
  static constexpr int ncplx = R == 18 ? 9 : 6;
  static constexpr int chunk_bytes = 16;
  static constexpr int chunks = ncplx;
  WD_HD static void load(const void* base, size_t n, size_t s, su3<double>& u) {
    const double2* v = (const double2*)base;
#pragma unroll
    for (int k = 0; k < ncplx; ++k) {
      const double2 d = v[k * n + s];
      u.e[k] = {d.x, d.y};
    }
    if (R == 12) reconstruct_row2(u);
  }
  WD_HD static void load_nt(const void* base, size_t n, size_t s, su3<double>& u) {
    const double2* v = (const double2*)base;
#pragma unroll
    for (int k = 0; k < ncplx; ++k) {
      const wd_nt_d2 d = __builtin_nontemporal_load((const wd_nt_d2*)&v[k * n + s]);
      u.e[k] = {d.x, d.y};
    }
    if (R == 12) reconstruct_row2(u);
  }
  WD_HD static void store(void* base, size_t n, size_t s, const su3<double>& u) {
    double2* v = (double2*)base;
#pragma unroll
    for (int k = 0; k < ncplx; ++k) v[k * n + s] = make_double2(u.e[k].re, u.e[k].im);
  }
};

template <> struct LinkFmt<F32, 18> {
  static constexpr int chunks = 9;
  static constexpr int chunk_bytes = 8;
  WD_HD static void load(const void* base, size_t n, size_t s, su3<float>& u) {
    const float2* v = (const float2*)base;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float2 d = v[k * n + s];
      u.e[k] = {d.x, d.y};
    }
  }
  WD_HD static void load_nt(const void* base, size_t n, size_t s, su3<float>& u) {
    const float2* v = (const float2*)base;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const wd_nt_f2 d = __builtin_nontemporal_load((const wd_nt_f2*)&v[k * n + s]);
      u.e[k] = {d.x, d.y};
    }
  }
  WD_HD static void store(void* base, size_t n, size_t s, const su3<float>& u) {
    float2* v = (float2*)base;
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k * n + s] = make_float2(u.e[k].re, u.e[k].im);
  }
};

template <> struct LinkFmt<F32, 12> {
  static constexpr int chunks = 3;
  static constexpr int chunk_bytes = 16;
  WD_HD static void load(const void* base, size_t n, size_t s, su3<float>& u) {
    const float4* v = (const float4*)base;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float4 d = v[k * n + s];
      u.e[2 * k] = {d.x, d.y};
      u.e[2 * k + 1] = {d.z, d.w};
    }
    reconstruct_row2(u);
  }
  WD_HD static void load_nt(const void* base, size_t n, size_t s, su3<float>& u) {
    const float4* v = (const float4*)base;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const wd_nt_f4 d = __builtin_nontemporal_load((const wd_nt_f4*)&v[k * n + s]);
      u.e[2 * k] = {d.x, d.y};
      u.e[2 * k + 1] = {d.z, d.w};
    }
    reconstruct_row2(u);
  }
  WD_HD static void store(void* base, size_t n, size_t s, const su3<float>& u) {
    float4* v = (float4*)base;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      v[k * n + s] = make_float4(u.e[2 * k].re, u.e[2 * k].im, u.e[2 * k + 1].re, u.e[2 * k + 1].im);
  }
};

template <> struct LinkFmt<F16, 18> {
  static constexpr int chunks = 9;
  static constexpr int chunk_bytes = 4;
  WD_HD static void load(const void* base, size_t n, size_t s, su3<float>& u) {
    const __half2* v = (const __half2*)base;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float2 d = __half22float2(v[k * n + s]);
      u.e[k] = {d.x, d.y};
    }
  }
  WD_HD static void store(void* base, size_t n, size_t s, const su3<float>& u) {
    __half2* v = (__half2*)base;
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k * n + s] = __floats2half2_rn(u.e[k].re, u.e[k].im);
  }
};

union h4 {
  uint2 u;
  __half2 h[2];
};

// FP16-12: complexes 0..3 in one 16-byte chunk array, complexes 4..5 in one
// 8-byte chunk array (two loads per link instead of three).
template <> struct LinkFmt<F16, 12> {
  static constexpr int chunks = 3;        // in 8-byte units: link_dir_bytes = 24 n
  static constexpr int chunk_bytes = 8;
  WD_HD static void load(const void* base, size_t n, size_t s, su3<float>& u) {
    const uint4* a = (const uint4*)base;
    const uint2* b = (const uint2*)((const char*)base + 16 * n);
    h8 d;
    d.u = a[s];
    h4 e;
    e.u = b[s];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float2 f = __half22float2(d.h[k]);
      u.e[k] = {f.x, f.y};
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const float2 f = __half22float2(e.h[k]);
      u.e[4 + k] = {f.x, f.y};
    }
    reconstruct_row2(u);
  }
  WD_HD static void store(void* base, size_t n, size_t s, const su3<float>& u) {
    uint4* a = (uint4*)base;
    uint2* b = (uint2*)((char*)base + 16 * n);
    h8 d;
#pragma unroll
    for (int k = 0; k < 4; ++k) d.h[k] = __floats2half2_rn(u.e[k].re, u.e[k].im);
    h4 e;
#pragma unroll
    for (int k = 0; k < 2; ++k) e.h[k] = __floats2half2_rn(u.e[4 + k].re, u.e[4 + k].im);
    a[s] = d.u;
    b[s] = e.u;
  }
};

template <int P, int R> WD_HD size_t link_dir_bytes(size_t n) {
  return (size_t)LinkFmt<P, R>::chunks * LinkFmt<P, R>::chunk_bytes * n;
}

// ---------------------------------------------------------------------------
// Checkerboard geometry.  Lexicographic index i = x + Lx (y + Ly (z + Lz t));
// the checkerboard index of a site within its parity is i / 2 (Lx even).
// ---------------------------------------------------------------------------
struct Geom {
  int L[4];   // Lx, Ly, Lz, Lt
  int hx;     // Lx / 2
  int n;      // sites per parity (below 2^30)
  FastDiv dhx, dy, dz;  // division by hx, Ly and Lz (set_divisors)
};

// Host: the divisors site_coord uses, from hx and L.
inline void set_divisors(Geom& g) {
  g.dhx = make_fastdiv(g.hx);
  g.dy = make_fastdiv(g.L[1]);
  g.dz = make_fastdiv(g.L[2]);
}

struct Coord {
  int c[4];
  int rest;   // y + Ly (z + Lz t): the cb index is x/2 + hx * rest
};

WD_HD Coord site_coord(const Geom& g, int parity, int s) {
  Coord k;
  const int rest = fdiv(s, g.dhx);
  const int xh = s - rest * g.hx;
  const int r2 = fdiv(rest, g.dy);
  const int y = rest - r2 * g.L[1];
  const int t = fdiv(r2, g.dz);
  const int z = r2 - t * g.L[2];
  k.c[0] = 2 * xh + ((parity + y + z + t) & 1);
  k.c[1] = y;
  k.c[2] = z;
  k.c[3] = t;
  k.rest = rest;
  return k;
}

// cb index of the neighbour x + dir*mu_hat (dir = +1 or -1), with wrap.
WD_HD int neighbour_cb(const Geom& g, const Coord& k, int mu, int dir) {
  int c = k.c[mu] + dir;
  if (c == g.L[mu]) c = 0;
  if (c < 0) c = g.L[mu] - 1;
  int x = mu == 0 ? c : k.c[0];
  int y = mu == 1 ? c : k.c[1];
  int z = mu == 2 ? c : k.c[2];
  int t = mu == 3 ? c : k.c[3];
  return (x >> 1) + g.hx * (y + g.L[1] * (z + g.L[2] * t));
}

// ---------------------------------------------------------------------------
// Spin projection in the chiral basis.  For the forward hop the projector is
// (1 - g_mu), for the backward hop (1 + g_mu).  Writing g_mu = [[0, A],[A^dag, 0]]
// with A_k = -i sigma_k, A_4 = 1, the projected spinor is fixed by its upper
// two spins h = psi_up -/+ A psi_low; its lower two spins are -/+ A^dag h.
// The colour product commutes with the spin projection, so only h is
// multiplied by the link and the lower spins are rebuilt afterwards.
// ---------------------------------------------------------------------------
// The 4 spin components s0..s3 (colour a) of p map to the 2 of h; C is a
// complex type with cadd/csub/cadd_i/csub_i (cplx<T>, or a pair of halves).
template <int MU, int DIR, typename C>
WD_HD void project_c(const C* p, C* h) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    C s0 = p[a], s1 = p[3 + a], s2 = p[6 + a], s3 = p[9 + a];
    if (DIR > 0) {  // 1 - g_mu
      if (MU == 0) { h[a] = cadd_i(s0, s3); h[3 + a] = cadd_i(s1, s2); }
      if (MU == 1) { h[a] = cadd(s0, s3);   h[3 + a] = csub(s1, s2); }
      if (MU == 2) { h[a] = cadd_i(s0, s2); h[3 + a] = csub_i(s1, s3); }
      if (MU == 3) { h[a] = csub(s0, s2);   h[3 + a] = csub(s1, s3); }
    } else {        // 1 + g_mu
      if (MU == 0) { h[a] = csub_i(s0, s3); h[3 + a] = csub_i(s1, s2); }
      if (MU == 1) { h[a] = csub(s0, s3);   h[3 + a] = cadd(s1, s2); }
      if (MU == 2) { h[a] = csub_i(s0, s2); h[3 + a] = cadd_i(s1, s3); }
      if (MU == 3) { h[a] = cadd(s0, s2);   h[3 + a] = cadd(s1, s3); }
    }
  }
}

template <int MU, int DIR, typename T>
WD_HD void project(const spinor<T>& p, half_spinor<T>& h) {
  project_c<MU, DIR>(p.c, h.c);
}

// Lower spin components of the rebuilt spinor from the upper ones g0, g1.
template <int MU, int DIR, typename T>
WD_HD void lower_from_upper(cplx<T> g0, cplx<T> g1, cplx<T>& l2, cplx<T>& l3) {
  if (DIR > 0) {  // lower = -A^dag g
    if (MU == 0) { l2 = ctimes_mi(g1); l3 = ctimes_mi(g0); }
    if (MU == 1) { l2 = cneg(g1);      l3 = g0; }
    if (MU == 2) { l2 = ctimes_mi(g0); l3 = ctimes_i(g1); }
    if (MU == 3) { l2 = cneg(g0);      l3 = cneg(g1); }
  } else {        // lower = +A^dag g
    if (MU == 0) { l2 = ctimes_i(g1);  l3 = ctimes_i(g0); }
    if (MU == 1) { l2 = g1;            l3 = cneg(g0); }
    if (MU == 2) { l2 = ctimes_i(g0);  l3 = ctimes_mi(g1); }
    if (MU == 3) { l2 = g0;            l3 = g1; }
  }
}

// acc += full spinor rebuilt from the link-multiplied half spinor g.
template <int MU, int DIR, typename T>
WD_HD void accumulate(spinor<T>& acc, const half_spinor<T>& g) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<T> g0 = g.c[a], g1 = g.c[3 + a];
    acc.c[a] = cadd(acc.c[a], g0);
    acc.c[3 + a] = cadd(acc.c[3 + a], g1);
    cplx<T> l2, l3;
    lower_from_upper<MU, DIR>(g0, g1, l2, l3);
    acc.c[6 + a] = cadd(acc.c[6 + a], l2);
    acc.c[9 + a] = cadd(acc.c[9 + a], l3);
  }
}

// acc += w * (full spinor rebuilt from g), one FMA per real.
template <int MU, int DIR>
WD_HD void accumulate_scaled(spinor<float>& acc, const half_spinor<float>& g, float w) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<float> g0 = g.c[a], g1 = g.c[3 + a];
    cplx<float> l2, l3;
    lower_from_upper<MU, DIR>(g0, g1, l2, l3);
    acc.c[a] = {fmaf(w, g0.re, acc.c[a].re), fmaf(w, g0.im, acc.c[a].im)};
    acc.c[3 + a] = {fmaf(w, g1.re, acc.c[3 + a].re), fmaf(w, g1.im, acc.c[3 + a].im)};
    acc.c[6 + a] = {fmaf(w, l2.re, acc.c[6 + a].re), fmaf(w, l2.im, acc.c[6 + a].im)};
    acc.c[9 + a] = {fmaf(w, l3.re, acc.c[9 + a].re), fmaf(w, l3.im, acc.c[9 + a].im)};
  }
}

// g = U h  (colour matrix on both spins)
template <typename T>
WD_HD void mul_link(const su3<T>& u, const half_spinor<T>& h, half_spinor<T>& g) {
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cplx<T> s = cmul(u.e[3 * a], h.c[3 * sp]);
      s = cadd(s, cmul(u.e[3 * a + 1], h.c[3 * sp + 1]));
      s = cadd(s, cmul(u.e[3 * a + 2], h.c[3 * sp + 2]));
      g.c[3 * sp + a] = s;
    }
  }
}

// g = U^dag h
template <typename T>
WD_HD void mul_link_dag(const su3<T>& u, const half_spinor<T>& h, half_spinor<T>& g) {
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cplx<T> s = cjmul(u.e[a], h.c[3 * sp]);
      s = cadd(s, cjmul(u.e[3 + a], h.c[3 * sp + 1]));
      s = cadd(s, cjmul(u.e[6 + a], h.c[3 * sp + 2]));
      g.c[3 * sp + a] = s;
    }
  }
}

template <typename T> WD_HD void gamma5_inplace(spinor<T>& s) {
#pragma unroll
  for (int k = 6; k < 12; ++k) s.c[k] = cneg(s.c[k]);
}

template <typename T> WD_HD void spinor_zero(spinor<T>& s) {
#pragma unroll
  for (int k = 0; k < 12; ++k) s.c[k] = {T(0), T(0)};
}

template <typename T> WD_HD double spinor_norm2(const spinor<T>& s) {
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < 12; ++k) acc += (double)s.c[k].re * (double)s.c[k].re + (double)s.c[k].im * (double)s.c[k].im;
  return acc;
}

template <typename TO, typename TI> WD_HD void spinor_convert(spinor<TO>& o, const spinor<TI>& i) {
#pragma unroll
  for (int k = 0; k < 12; ++k) o.c[k] = {(TO)i.c[k].re, (TO)i.c[k].im};
}

// ---------------------------------------------------------------------------
// The hopping term at one output site: acc = H in (optionally gamma5 on in).
// gauge points at the start of the store; in points at the input parity
// block.  ne = n * nrhs is the chunk stride of the spinor block.
//
// Hop h (0..7) is direction mu = h / 2, forward for even h and backward for
// odd h.  FP64 and FP32 run each hop in turn (hop_dir: spinor and link
// loads, projection, product; 18-real links loaded after the projection),
// relying on the waves in flight to hide the latency.  FP16, whose stencil is
// bound by instruction issue rather than memory, fetches the spinors and links of 4 hops first (all their loads in
// flight together, no branch between them) and then computes them.  Measured
// on one box with the same launch shapes: the grouped form was 2-4 % faster
// for FP16 (24^3x48, 32^3x64), but 4 % slower for the FP64 CG-residual
// stencil (19.8 against 19.0 us at 16^3x32) and 1 % slower for FP32; at
// FP64 a group of 2 hops took the 2-way split to one wave per SIMD.
// ---------------------------------------------------------------------------
template <int P, int R, int MU, int DIR, bool NT>
WD_HD void hop_dir(const Geom& g, const Coord& k, int parity, int s, int rhs, int nrhs,
                   const char* gauge, const void* in, float bc_sign, bool g5in,
                   spinor<typename RealOf<P>::T>& acc) {
  using T = typename RealOf<P>::T;
  const size_t n = (size_t)g.n;
  const size_t ne = n * (size_t)nrhs;
  int nb = neighbour_cb(g, k, MU, DIR);
  spinor<T> p;
  SpinorFmt<P>::load(in, ne, (size_t)nb * nrhs + rhs, p);
  su3<T> u;
  // forward: U_mu(x), rooted at the output site (parity `parity`);
  // backward: U_mu(x - mu), rooted at the neighbour (other parity).
  const int lp = DIR > 0 ? parity : 1 - parity;
  const size_t ls = DIR > 0 ? (size_t)s : (size_t)nb;
  const char* lbase = gauge + (size_t)(lp * 4 + MU) * link_dir_bytes<P, R>(n);
  // 12-real links are loaded right after the spinor, so that both are in
  // flight together; 18-real ones after the projection, since loading their
  // 36 registers early cost waves per SIMD (FP64 with 2 parts: 2 -> 1).
  if constexpr (R == 12) {
    if constexpr (NT) LinkFmt<P, R>::load_nt(lbase, n, ls, u);
    else LinkFmt<P, R>::load(lbase, n, ls, u);
  }
  if (g5in) gamma5_inplace(p);
  half_spinor<T> h, gh;
  project<MU, DIR>(p, h);
  bool crosses = DIR > 0 ? (k.c[MU] == g.L[MU] - 1) : (k.c[MU] == 0);
  if (crosses && bc_sign < 0.f) {
#pragma unroll
    for (int j = 0; j < 6; ++j) h.c[j] = cneg(h.c[j]);
  }
  if constexpr (R != 12) {
    if constexpr (NT) LinkFmt<P, R>::load_nt(lbase, n, ls, u);
    else LinkFmt<P, R>::load(lbase, n, ls, u);
  }
  if (DIR > 0) mul_link(u, h, gh);
  else mul_link_dag(u, h, gh);
  accumulate<MU, DIR>(acc, gh);
}

// ---------------------------------------------------------------------------
// FP16 hops in packed half arithmetic.  The neighbour spinor stays in its
// stored halves (component / site scale): the spin projection adds pairs of
// halves (one v_pk_add_f16 per complex), the colour product takes dot
// products of half pairs with FP32 accumulation (v_dot2_f32_f16; the half
// products are exact in FP32), and the neighbour's scale, with the boundary
// sign, multiplies the FP32 product as it is accumulated (one FMA per real).
// Links are used as stored; the third row of a 12-real link is rebuilt from
// half dot products accumulated in FP32 and rounded to halves like the
// stored rows.  A complex is a pair of halves (re, im):
//   Re(U h) = sum dot2((U.re, -U.im), h)       Im(U h) = sum dot2(U, (h.im, h.re))
//   Re(U^dag h) = sum dot2(U, h)               Im(U^dag h) = sum dot2((U.re, -U.im), (h.im, h.re))
// ---------------------------------------------------------------------------
struct HopBuf16 {
  wd_h2 s[12];  // neighbour spinor as stored (component / scale)
  float w;      // its scale
  wd_h2 u[9];   // link as stored (12-real links: rows 0 and 1)
  bool flip;    // the hop crosses a boundary with sign -1
};

template <int R, int H, bool NT>
__device__ __forceinline__ void hop_fetch16(const Geom& g, const Coord& k, int parity, int s, int rhs, int nrhs,
                                            const char* gauge, const void* in, const float bc[4], HopBuf16& b) {
  constexpr int MU = H >> 1;
  constexpr int DIR = (H & 1) ? -1 : 1;
  const size_t n = (size_t)g.n;
  const size_t ne = n * (size_t)nrhs;
  const int nb = neighbour_cb(g, k, MU, DIR);
  const size_t e = (size_t)nb * nrhs + rhs;
  const uint4* v = (const uint4*)in;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const uint4 d = v[c * ne + e];
    b.s[4 * c] = h2_bits(d.x);
    b.s[4 * c + 1] = h2_bits(d.y);
    b.s[4 * c + 2] = h2_bits(d.z);
    b.s[4 * c + 3] = h2_bits(d.w);
  }
  b.w = ((const float*)((const char*)in + SpinorFmt<F16>::data_bytes(ne)))[e];
  // forward: U_mu(x), rooted at the output site (parity `parity`);
  // backward: U_mu(x - mu), rooted at the neighbour (other parity).
  const int lp = DIR > 0 ? parity : 1 - parity;
  const size_t ls = DIR > 0 ? (size_t)s : (size_t)nb;
  const char* lbase = gauge + (size_t)(lp * 4 + MU) * link_dir_bytes<F16, R>(n);
  // The non-temporal loads take integer vectors: loaded as float vectors and
  // bit-cast to half pairs, some of a link's words were dropped by the compiled
  // code (their registers reused while the load was in flight).
  if constexpr (R == 12 && NT) {
    const wd_nt_u4 d = __builtin_nontemporal_load((const wd_nt_u4*)lbase + ls);
    const wd_nt_u2 f = __builtin_nontemporal_load((const wd_nt_u2*)(lbase + 16 * n) + ls);
    b.u[0] = h2_bits(d.x);
    b.u[1] = h2_bits(d.y);
    b.u[2] = h2_bits(d.z);
    b.u[3] = h2_bits(d.w);
    b.u[4] = h2_bits(f.x);
    b.u[5] = h2_bits(f.y);
  } else if constexpr (R == 12) {
    const uint4 d = ((const uint4*)lbase)[ls];
    const uint2 f = ((const uint2*)(lbase + 16 * n))[ls];
    b.u[0] = h2_bits(d.x);
    b.u[1] = h2_bits(d.y);
    b.u[2] = h2_bits(d.z);
    b.u[3] = h2_bits(d.w);
    b.u[4] = h2_bits(f.x);
    b.u[5] = h2_bits(f.y);
  } else if constexpr (NT) {
    const uint32_t* lv = (const uint32_t*)lbase;
#pragma unroll
    for (int q = 0; q < 9; ++q) b.u[q] = h2_bits(__builtin_nontemporal_load(&lv[q * n + ls]));
  } else {
    const uint32_t* lv = (const uint32_t*)lbase;
#pragma unroll
    for (int q = 0; q < 9; ++q) b.u[q] = h2_bits(lv[q * n + ls]);
  }
  const bool crosses = DIR > 0 ? (k.c[MU] == g.L[MU] - 1) : (k.c[MU] == 0);
  b.flip = crosses && bc[MU] < 0.f;
}

template <int R, int H>
__device__ __forceinline__ void hop_finish16(HopBuf16& b, bool g5in, spinor<float>& acc) {
  constexpr int MU = H >> 1;
  constexpr int DIR = (H & 1) ? -1 : 1;
  wd_h2 uc[9];  // (U.re, -U.im)
#pragma unroll
  for (int q = 0; q < 6; ++q) uc[q] = h2_conj(b.u[q]);
  if constexpr (R == 12) {
    // Third row = conj(row0 x row1), from half dot products accumulated in
    // FP32 (the products of halves are exact there), rounded to halves like
    // the stored rows.  For e = conj(a d - b' c) with b' the negated row-0
    // entry:  Re e = dot(a, (d.re, -d.im)) + dot(b', (c.re, -c.im)),
    //         Im e = dot(a, (-d.im, -d.re)) + dot(b', (-c.im, -c.re)).
    wd_h2 ng[3], sw[3];  // -row0 entries; (-x.im, -x.re) of the row-1 entries
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      ng[q] = -b.u[q];
      const uint32_t v = __builtin_bit_cast(uint32_t, b.u[3 + q]);
      sw[q] = h2_bits(((v >> 16) | (v << 16)) ^ 0x80008000u);  // (-x.im, -x.re)
    }
    // (a, b', d, c) row indices: e6 = conj(u1 u5 - u2 u4), e7 = conj(u2 u3 - u0 u5), e8 = conj(u0 u4 - u1 u3)
    constexpr int A_[3] = {1, 2, 0}, B_[3] = {2, 0, 1}, D_[3] = {5, 3, 4}, C_[3] = {4, 5, 3};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float re = dot2h(b.u[A_[q]], uc[D_[q]], dot2h(ng[B_[q]], uc[C_[q]], 0.f));
      const float im = dot2h(b.u[A_[q]], sw[D_[q] - 3], dot2h(ng[B_[q]], sw[C_[q] - 3], 0.f));
      b.u[6 + q] = (wd_h2){(_Float16)re, (_Float16)im};
    }
  }
#pragma unroll
  for (int q = 6; q < 9; ++q) uc[q] = h2_conj(b.u[q]);
  if (g5in) {
#pragma unroll
    for (int q = 6; q < 12; ++q) b.s[q] = -b.s[q];
  }
  wd_h2 h[6], hs[6];
  project_c<MU, DIR>(b.s, h);
#pragma unroll
  for (int j = 0; j < 6; ++j) hs[j] = h2_swap(h[j]);
  half_spinor<float> gh;
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float re = 0.f, im = 0.f;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if (DIR > 0) {  // U h: U_aj
          re = dot2h(uc[3 * a + j], h[3 * sp + j], re);
          im = dot2h(b.u[3 * a + j], hs[3 * sp + j], im);
        } else {        // U^dag h: conj(U_ja)
          re = dot2h(b.u[3 * j + a], h[3 * sp + j], re);
          im = dot2h(uc[3 * j + a], hs[3 * sp + j], im);
        }
      }
      gh.c[3 * sp + a] = {re, im};
    }
  }
  accumulate_scaled<MU, DIR>(acc, gh, b.flip ? -b.w : b.w);
}

template <int R, int H0, bool NT, int... J>
__device__ __forceinline__ void hop_fetch_group16(std::integer_sequence<int, J...>, const Geom& g, const Coord& k,
                                                  int parity, int s, int rhs, int nrhs, const char* gauge,
                                                  const void* in, const float bc[4], HopBuf16* b) {
  (hop_fetch16<R, H0 + J, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, b[J]), ...);
}

template <int R, int H0, int... J>
__device__ __forceinline__ void hop_finish_group16(std::integer_sequence<int, J...>, HopBuf16* b, bool g5in,
                                                   spinor<float>& acc) {
  (hop_finish16<R, H0 + J>(b[J], g5in, acc), ...);
}

// Hops H0 .. H0 + NH - 1, accumulated in hop order (FP16 in groups of 4).
template <int P, int R, int H0, int NH, bool NT>
WD_HD void hop_range(const Geom& g, const Coord& k, int parity, int s, int rhs, int nrhs, const char* gauge,
                     const void* in, const float bc[4], bool g5in, spinor<typename RealOf<P>::T>& acc) {
  if constexpr (NH > 0 && P != F16) {
    constexpr int MU = H0 >> 1;
    constexpr int DIR = (H0 & 1) ? -1 : 1;
    hop_dir<P, R, MU, DIR, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc[MU], g5in, acc);
    hop_range<P, R, H0 + 1, NH - 1, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc);
  } else if constexpr (NH > 0) {
    constexpr int M = NH < 4 ? NH : 4;
    HopBuf16 b[M];
    hop_fetch_group16<R, H0, NT>(std::make_integer_sequence<int, M>{}, g, k, parity, s, rhs, nrhs, gauge, in, bc, b);
    hop_finish_group16<R, H0>(std::make_integer_sequence<int, M>{}, b, g5in, acc);
    hop_range<P, R, H0 + M, NH - M, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc);
  }
}

// Hops H... in the order given (FP64 and FP32: hop_dir one after the other).
template <int P, int R, bool NT, int... H>
WD_HD void hop_list(const Geom& g, const Coord& k, int parity, int s, int rhs, int nrhs, const char* gauge,
                    const void* in, const float bc[4], bool g5in, spinor<typename RealOf<P>::T>& acc) {
  (hop_dir<P, R, (H >> 1), ((H & 1) ? -1 : 1), NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc[H >> 1], g5in, acc),
   ...);
}

// The share `part` of the 8 hops when they are split over D threads:
// D = 1 all directions, D = 2 (x,y) / (z,t), D = 4 one direction each,
// D = 8 one hop each.  Parts are whole waves, so the branch on `part` is
// uniform.  At FP64 the parts of D = 2 and D = 4 pair a near hop (x or y,
// whose neighbour spinors mostly come from the L1) with a far one (z or t,
// from the L2 or memory): D = 4 takes {x+, t+}, {x-, t-}, {y+, z+}, {y-, z-}
// and D = 2 {x+, t+, y+, z+}, {x-, t-, y-, z-}.  All waves of a
// workgroup then wait about as long for their loads, and none holds the
// workgroup at the combine step (24^3x48 FP64 stencil, 4 parts: 1-3 %
// faster than one direction per part).
template <int P, int R, int D, bool NT>
WD_HD void hop_part(const Geom& g, int parity, int s, int rhs, int nrhs, const char* gauge, const void* in,
                    const float bc[4], bool g5in, int part, spinor<typename RealOf<P>::T>& acc) {
  Coord k = site_coord(g, parity, s);
  spinor_zero(acc);
  if constexpr (P == F64 && D == 4) {
    switch (part) {
      case 0: hop_list<P, R, NT, 0, 6>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
      case 1: hop_list<P, R, NT, 1, 7>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
      case 2: hop_list<P, R, NT, 2, 4>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
      default: hop_list<P, R, NT, 3, 5>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
    }
  } else if constexpr (P == F64 && D == 2) {
    if (part == 0) hop_list<P, R, NT, 0, 6, 2, 4>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc);
    else hop_list<P, R, NT, 1, 7, 3, 5>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc);
  } else if constexpr (D == 1) {
    hop_range<P, R, 0, 8, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc);
  } else if constexpr (D == 2) {
    if (part == 0) hop_range<P, R, 0, 4, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc);
    else hop_range<P, R, 4, 4, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc);
  } else if constexpr (D == 4) {
    switch (part) {
      case 0: hop_range<P, R, 0, 2, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
      case 1: hop_range<P, R, 2, 2, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
      case 2: hop_range<P, R, 4, 2, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
      default: hop_range<P, R, 6, 2, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
    }
  } else {
    switch (part) {
      case 0: hop_range<P, R, 0, 1, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
      case 1: hop_range<P, R, 1, 1, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
      case 2: hop_range<P, R, 2, 1, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
      case 3: hop_range<P, R, 3, 1, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
      case 4: hop_range<P, R, 4, 1, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
      case 5: hop_range<P, R, 5, 1, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
      case 6: hop_range<P, R, 6, 1, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
      default: hop_range<P, R, 7, 1, NT>(g, k, parity, s, rhs, nrhs, gauge, in, bc, g5in, acc); break;
    }
  }
}

}  // namespace wd
