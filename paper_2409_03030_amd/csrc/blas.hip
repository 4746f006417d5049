// CG vector kernels (one thread per site and rhs, all 24 reals of the site
// in registers so FP16 per-site scales are formed in place) and the layout
// conversions between the complex128 boundary arrays and the internal
// parity blocks.
#include "wd_kcommon.h"
#include "wd_kernels.h"

namespace wd {

template <int P> struct AccOfB { static constexpr int value = P == F16 ? F32 : P; };

// The inner solution x (accumulation precision, FP64 or FP32) in the vector
// update of a launch whose inner vectors exceed kStreamVecBytes, read and
// written with the non-temporal hint: no stencil reads it, so it need not take
// Infinity Cache space from the vectors the stencils gather.
template <typename TA>
__device__ __forceinline__ void load_x_nt(const void* base, size_t ne, size_t e, spinor<TA>& s) {
  if constexpr (sizeof(TA) == 8) {
    const double2* v = (const double2*)base;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const wd_nt_d2 d = __builtin_nontemporal_load((const wd_nt_d2*)&v[k * ne + e]);
      s.c[k] = {d.x, d.y};
    }
  } else {
    const float4* v = (const float4*)base;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const wd_nt_f4 d = __builtin_nontemporal_load((const wd_nt_f4*)&v[k * ne + e]);
      s.c[2 * k] = {d.x, d.y};
      s.c[2 * k + 1] = {d.z, d.w};
    }
  }
}

template <typename TA>
__device__ __forceinline__ void store_x_nt(void* base, size_t ne, size_t e, const spinor<TA>& s) {
  if constexpr (sizeof(TA) == 8) {
    double2* v = (double2*)base;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const wd_nt_d2 d = {s.c[k].re, s.c[k].im};
      __builtin_nontemporal_store(d, (wd_nt_d2*)&v[k * ne + e]);
    }
  } else {
    float4* v = (float4*)base;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const wd_nt_f4 d = {s.c[2 * k].re, s.c[2 * k].im, s.c[2 * k + 1].re, s.c[2 * k + 1].im};
      __builtin_nontemporal_store(d, (wd_nt_f4*)&v[k * ne + e]);
    }
  }
}

// BLAS_INIT  : x_h = 0, x = 0, r = low(b), p = low(b);   ||b||^2 -> FIN_INIT
// BLAS_CGUPD : x += alpha p (active rhs); p = r + beta p (running rhs); with
//              prefin = FIN_CG every block first finishes the |r|^2 reduction
// BLAS_RU_ACC: x_h += x, x = 0                            (held rhs)
// BLAS_RU_FIN: r = low(r_h), p = r + beta p               (resumed rhs)
template <int P, int MODE, bool XNT>
__global__ void __launch_bounds__(kBlock) blas_kernel(const Launch L) {
  using T = typename RealOf<P>::T;
  constexpr int A = AccOfB<P>::value;
  using TA = typename RealOf<A>::T;
  const Tile t = make_tile(L);
  const Slot& S = L.s[t.slot];
  // Launches with a reduction run every block: every block partial of the
  // slot must be written for the finalize step.
  if (L.fin == FIN_NONE && !slot_selected(L, S)) return;
  const bool both = L.parity == 2;
  const size_t pv = both ? (size_t)t.parity * S.vstride : 0;
  const size_t pa = both ? (size_t)t.parity * S.astride : 0;
  const size_t ph = both ? (size_t)t.parity * S.hstride : 0;
  const size_t ne = (size_t)S.g.n * L.nrhs;
  const size_t e = (size_t)t.site * L.nrhs + t.rhs;
  double v = 0.0;
  if (MODE == BLAS_CGUPD) {
    const bool on = t.valid && rhs_selected(S.st, L.mask, t.rhs);
    spinor<T> p;
    spinor<TA> x, r;
    if (on) {  // issued before stage 2 so that both sets of loads are in flight together
      SpinorFmt<P>::load((const char*)S.out + pv, ne, e, p);
      if constexpr (XNT) load_x_nt((const char*)S.x + pa, ne, e, x);
      else SpinorFmt<A>::load((const char*)S.x + pa, ne, e, x);
      SpinorFmt<A>::load((const char*)S.r + pa, ne, e, r);
    }
    __shared__ double s_beta[kBlock / 2];
    __shared__ int s_state[kBlock / 2];
    double beta_d;
    int state;
    if (L.prefin == FIN_CG) {
      fold_finalize_cg(L, S, t, s_beta, s_state);
      beta_d = s_beta[t.rhs];
      state = s_state[t.rhs];
    } else {
      beta_d = S.st[t.rhs].beta;
      state = S.st[t.rhs].state;
    }
    if (on) {
      const TA alpha = (TA)S.st[t.rhs].alpha;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        x.c[k].re += alpha * (TA)p.c[k].re;
        x.c[k].im += alpha * (TA)p.c[k].im;
      }
      if constexpr (XNT) store_x_nt((char*)S.x + pa, ne, e, x);
      else SpinorFmt<A>::store((char*)S.x + pa, ne, e, x);
      if (state == ST_RUN) {
        const TA beta = (TA)beta_d;
        spinor<T> np;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          np.c[k].re = (T)(r.c[k].re + beta * (TA)p.c[k].re);
          np.c[k].im = (T)(r.c[k].im + beta * (TA)p.c[k].im);
        }
        SpinorFmt<P>::store((char*)S.out + pv, ne, e, np);
      }
    }
    return;
  }
  if (t.valid && rhs_selected(S.st, L.mask, t.rhs)) {
    if (MODE == BLAS_INIT) {
      spinor<double> b;
      SpinorFmt<F64>::load((const char*)S.b + ph, ne, e, b);
      v = spinor_norm2(b);
      spinor<double> z;
      spinor_zero(z);
      SpinorFmt<F64>::store((char*)S.xh + ph, ne, e, z);
      spinor<TA> ra, xa;
      spinor_convert(ra, b);
      spinor_zero(xa);
      SpinorFmt<A>::store((char*)S.r + pa, ne, e, ra);
      SpinorFmt<A>::store((char*)S.x + pa, ne, e, xa);
      spinor<T> pp;
      spinor_convert(pp, b);
      SpinorFmt<P>::store((char*)S.out + pv, ne, e, pp);
    } else if (MODE == BLAS_RU_ACC) {
      spinor<double> xh;
      spinor<TA> x;
      SpinorFmt<F64>::load((const char*)S.xh + ph, ne, e, xh);
      SpinorFmt<A>::load((const char*)S.x + pa, ne, e, x);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        xh.c[k].re += (double)x.c[k].re;
        xh.c[k].im += (double)x.c[k].im;
      }
      SpinorFmt<F64>::store((char*)S.xh + ph, ne, e, xh);
      spinor_zero(x);
      SpinorFmt<A>::store((char*)S.x + pa, ne, e, x);
    } else {  // BLAS_RU_FIN
      const TA beta = (TA)S.st[t.rhs].beta;
      spinor<double> rh;
      SpinorFmt<F64>::load((const char*)S.rh + ph, ne, e, rh);
      spinor<TA> r;
      spinor_convert(r, rh);
      SpinorFmt<A>::store((char*)S.r + pa, ne, e, r);
      spinor<T> p;
      SpinorFmt<P>::load((const char*)S.out + pv, ne, e, p);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        p.c[k].re = (T)(r.c[k].re + beta * (TA)p.c[k].re);
        p.c[k].im = (T)(r.c[k].im + beta * (TA)p.c[k].im);
      }
      SpinorFmt<P>::store((char*)S.out + pv, ne, e, p);
    }
  }
  if (L.fin != FIN_NONE) block_reduce_store(L, S, t, v);
}

// Stage 2 of a reduction: one block per slot (see gather_and_finalize).
__global__ void __launch_bounds__(kBlock) finalize_kernel(const Launch L) {
  const Slot& S = L.s[blockIdx.x];
  gather_and_finalize(L, S, L.fin);
}

hipError_t launch_finalize(const Launch& L, hipStream_t stream) {
  if (L.nslots <= 0 || L.fin == FIN_NONE) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)L.nslots), dim3(kBlock), 0, stream, L);
  return hipGetLastError();
}

template <int P>
static hipError_t blas_mode(const Launch& L, int mode, bool xnt, hipStream_t stream) {
  dim3 grid((unsigned)L.total_blocks), block((unsigned)(L.sblk * L.nrhs));
  switch (mode) {
    case BLAS_INIT: hipLaunchKernelGGL((blas_kernel<P, BLAS_INIT, false>), grid, block, 0, stream, L); break;
    case BLAS_CGUPD:
      if (xnt) hipLaunchKernelGGL((blas_kernel<P, BLAS_CGUPD, true>), grid, block, 0, stream, L);
      else hipLaunchKernelGGL((blas_kernel<P, BLAS_CGUPD, false>), grid, block, 0, stream, L);
      break;
    case BLAS_RU_ACC: hipLaunchKernelGGL((blas_kernel<P, BLAS_RU_ACC, false>), grid, block, 0, stream, L); break;
    case BLAS_RU_FIN: hipLaunchKernelGGL((blas_kernel<P, BLAS_RU_FIN, false>), grid, block, 0, stream, L); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Bytes of the inner CG's vectors in the launch's slots (p, t1, t2 at the inner
// precision; x and r at the accumulation precision; both parities unless even-odd).
static double inner_vector_bytes(const Launch& L) {
  double b = 0.0;
  for (int k = 0; k < L.nslots; ++k) b += 3.0 * (double)L.s[k].vstride + 2.0 * (double)L.s[k].astride;
  return L.parity == 2 ? 2.0 * b : b;
}

hipError_t launch_blas(const Launch& L0, int prec, int mode, hipStream_t stream) {
  if (L0.total_blocks <= 0) return hipSuccess;
  Launch L = L0;
  L.split = 1;  // one thread per (site, rhs)
  const bool xnt = mode == BLAS_CGUPD && inner_vector_bytes(L) > kStreamVecBytes;
  if (prec == F64) return blas_mode<F64>(L, mode, xnt, stream);
  if (prec == F32) return blas_mode<F32>(L, mode, xnt, stream);
  if (prec == F16) return blas_mode<F16>(L, mode, xnt, stream);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// layout conversion
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lex_coord(const Geom& g, int i, int c[4]) {
  c[0] = i % g.L[0];
  int r = i / g.L[0];
  c[1] = r % g.L[1];
  r /= g.L[1];
  c[2] = r % g.L[2];
  c[3] = r / g.L[2];
}

template <int P, int R>
__global__ void gauge_import_kernel(const double2* __restrict__ U, char* __restrict__ store, Geom g) {
  using T = typename RealOf<P>::T;
  const int V = 2 * g.n;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 4L * V) return;
  const int mu = (int)(idx / V);
  const int i = (int)(idx % V);
  int c[4];
  lex_coord(g, i, c);
  const int parity = (c[0] + c[1] + c[2] + c[3]) & 1;
  su3<T> u;
  const double2* src = U + ((size_t)mu * V + i) * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double2 d = src[k];
    u.e[k] = {(T)d.x, (T)d.y};
  }
  char* base = store + (size_t)(parity * 4 + mu) * link_dir_bytes<P, R>((size_t)g.n);
  LinkFmt<P, R>::store(base, (size_t)g.n, (size_t)(i >> 1), u);
}

template <int P>
__global__ void spinor_import_kernel(const double2* __restrict__ src, char* __restrict__ dst, size_t pstride,
                                     Geom g, int nrhs, int parities) {
  using T = typename RealOf<P>::T;
  const int V = 2 * g.n;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)V * nrhs) return;
  const int r = (int)(idx / V);
  const int i = (int)(idx % V);
  int c[4];
  lex_coord(g, i, c);
  const int parity = (c[0] + c[1] + c[2] + c[3]) & 1;
  if (parities == 1 && parity == 1) return;
  spinor<T> s;
  const double2* p = src + ((size_t)r * V + i) * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    double2 d = p[k];
    s.c[k] = {(T)d.x, (T)d.y};
  }
  const size_t ne = (size_t)g.n * nrhs;
  SpinorFmt<P>::store(dst + (parities == 2 ? parity * pstride : 0), ne, (size_t)(i >> 1) * nrhs + r, s);
}

template <int P>
__global__ void spinor_export_kernel(const char* __restrict__ src, size_t pstride, double2* __restrict__ dst,
                                     Geom g, int nrhs, int parities) {
  using T = typename RealOf<P>::T;
  const int V = 2 * g.n;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)V * nrhs) return;
  const int r = (int)(idx / V);
  const int i = (int)(idx % V);
  int c[4];
  lex_coord(g, i, c);
  const int parity = (c[0] + c[1] + c[2] + c[3]) & 1;
  double2* p = dst + ((size_t)r * V + i) * 12;
  if (parities == 1 && parity == 1) {
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = make_double2(0.0, 0.0);
    return;
  }
  spinor<T> s;
  const size_t ne = (size_t)g.n * nrhs;
  SpinorFmt<P>::load(src + (parities == 2 ? parity * pstride : 0), ne, (size_t)(i >> 1) * nrhs + r, s);
#pragma unroll
  for (int k = 0; k < 12; ++k) p[k] = make_double2((double)s.c[k].re, (double)s.c[k].im);
}

hipError_t launch_gauge_import(const void* U, void* store, const Geom& g, int prec, int recon, hipStream_t stream) {
  const long total = 8L * g.n;
  const unsigned grid = (unsigned)((total + 255) / 256);
  const double2* u = (const double2*)U;
  char* s = (char*)store;
#define WD_GI(P_, R_) hipLaunchKernelGGL((gauge_import_kernel<P_, R_>), dim3(grid), dim3(256), 0, stream, u, s, g)
  if (prec == F64 && recon == 18) WD_GI(F64, 18);
  else if (prec == F64 && recon == 12) WD_GI(F64, 12);
  else if (prec == F32 && recon == 18) WD_GI(F32, 18);
  else if (prec == F32 && recon == 12) WD_GI(F32, 12);
  else if (prec == F16 && recon == 18) WD_GI(F16, 18);
  else if (prec == F16 && recon == 12) WD_GI(F16, 12);
  else return hipErrorInvalidValue;
#undef WD_GI
  return hipGetLastError();
}

hipError_t launch_spinor_import(const void* src, void* dst, size_t pstride, const Geom& g, int nrhs, int parities,
                                int prec, hipStream_t stream) {
  const long total = 2L * g.n * nrhs;
  const unsigned grid = (unsigned)((total + 255) / 256);
  const double2* s = (const double2*)src;
  char* d = (char*)dst;
  if (prec == F64) hipLaunchKernelGGL((spinor_import_kernel<F64>), dim3(grid), dim3(256), 0, stream, s, d, pstride, g, nrhs, parities);
  else if (prec == F32) hipLaunchKernelGGL((spinor_import_kernel<F32>), dim3(grid), dim3(256), 0, stream, s, d, pstride, g, nrhs, parities);
  else if (prec == F16) hipLaunchKernelGGL((spinor_import_kernel<F16>), dim3(grid), dim3(256), 0, stream, s, d, pstride, g, nrhs, parities);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_spinor_export(const void* src, size_t pstride, void* dst, const Geom& g, int nrhs, int parities,
                                int prec, hipStream_t stream) {
  const long total = 2L * g.n * nrhs;
  const unsigned grid = (unsigned)((total + 255) / 256);
  const char* s = (const char*)src;
  double2* d = (double2*)dst;
  if (prec == F64) hipLaunchKernelGGL((spinor_export_kernel<F64>), dim3(grid), dim3(256), 0, stream, s, pstride, d, g, nrhs, parities);
  else if (prec == F32) hipLaunchKernelGGL((spinor_export_kernel<F32>), dim3(grid), dim3(256), 0, stream, s, pstride, d, g, nrhs, parities);
  else if (prec == F16) hipLaunchKernelGGL((spinor_export_kernel<F16>), dim3(grid), dim3(256), 0, stream, s, pstride, d, g, nrhs, parities);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace wd
