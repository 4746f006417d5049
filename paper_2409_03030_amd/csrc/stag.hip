// The staggered stencil with fused CG epilogues, its CG vector kernels and
// the colour-vector layout conversions.  Same launch descriptors, masks and
// deterministic two-stage reductions as the Wilson kernels; one, two or four
// threads per (output site, rhs), which split its 8 hops.  The CG runs on the
// even block
// M_e = m^2 - H_eo H_oe (Hermitian positive definite):
//   t = H_oe p ; <p, M_e p> = m^2 |p|^2 + |t|^2        S_NORM  (alpha partials)
//   alpha ; r -= alpha (m^2 p - H_eo t) ; |r|^2        S_CGR   (alpha folded in, FIN_CG)
//   x += alpha p ; p = r + beta p                      sblas CGUPD
#include "wd_kcommon.h"
#include "wd_kernels.h"
#include "wd_stag.h"

namespace wd {

// NT: links read with the non-temporal hint (stag_kernel_nt), for launches
// whose links cannot stay in the Infinity Cache (as in the Wilson stencil).
template <int P, int R, int MODE, int D, bool NT>
__device__ __forceinline__ void stag_body(const Launch& L) {
  using T = typename RealOf<P>::T;
  const Tile t = make_tile(L);
  const Slot& S = L.s[t.slot];
  // alpha folded into every block (the residual update needs it everywhere);
  // the mask then uses the block's own copy of `active`
  __shared__ double s_alpha[kBlock / 2];
  __shared__ int s_active[kBlock / 2];
  const bool fold_alpha = MODE == S_CGR && L.prefin == FIN_ALPHA_ALL;
  if (fold_alpha) fold_finalize_alpha(L, S, t, s_alpha, s_active);
  else if (L.prefin != FIN_NONE && t.lblk == 0) gather_and_finalize(L, S, L.prefin);
  // Launches with a reduction run every block: every block partial of the
  // slot must be written for the finalize step.
  if (L.fin == FIN_NONE && !slot_selected(L, S)) return;
  if (L.work_flag != nullptr && t.lblk == 0 && threadIdx.x == 0 && slot_selected(L, S)) *L.work_flag = 1;
  const bool both = L.parity == 2;
  const int par = t.parity;
  const size_t ne = (size_t)S.g.n * L.nrhs;
  const size_t e = (size_t)t.site * L.nrhs + t.rhs;
  const bool sel = t.valid && (fold_alpha ? s_active[t.rhs] != 0 : rhs_selected(S.st, L.mask, t.rhs));
  cvec<T> h;
  if (sel) {
    const char* in = (const char*)S.in + (both ? (size_t)(1 - par) * S.vstride : 0);
    stag_site<P, R, D, NT>(S.g, par, t.site, t.rhs, L.nrhs, S.gauge, in, S.bc, t.part, h);  // (share of) 2 H in
  }
  if constexpr (D > 1) {
    // parts 1..D-1 hand their sums to part 0, which adds them in part order
    // and alone runs the epilogue
    __shared__ T lds_h[(D - 1) * 6 * (kBlock / D)];
    const int per = L.sblk * L.nrhs;
    const int loc = (int)threadIdx.x - t.part * per;
    if (sel && t.part > 0) {
      T* q = lds_h + (size_t)(t.part - 1) * 6 * per + loc;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        q[(2 * k) * per] = h.c[k].re;
        q[(2 * k + 1) * per] = h.c[k].im;
      }
    }
    __syncthreads();
    if (sel && t.part == 0) {
#pragma unroll
      for (int pp = 1; pp < D; ++pp) {
        const T* q = lds_h + (size_t)(pp - 1) * 6 * per + loc;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          h.c[k].re += q[(2 * k) * per];
          h.c[k].im += q[(2 * k + 1) * per];
        }
      }
    }
  }
  double v = 0.0;
  if (sel && t.part == 0) {
    const size_t pv = both ? (size_t)par * S.vstride : 0;
    if (MODE == S_PLAIN || MODE == S_NORM) {
#pragma unroll
      for (int k = 0; k < 3; ++k) h.c[k] = cscale(h.c[k], T(0.5));
      SFmt<P>::store((char*)S.out + pv, ne, e, h);
      if (MODE == S_NORM) {
        cvec<T> p;
        SFmt<P>::load((const char*)S.aux + pv, ne, e, p);
        v = cvec_norm2(h) + S.st[t.rhs].c * cvec_norm2(p);
      }
    } else if (MODE == S_XPAY) {
      const T c = (T)(S.st ? S.st[t.rhs].c : L.coef);
      const T a = (T)(0.5 * (S.st ? S.st[t.rhs].alpha : L.coef2));
      cvec<T> x, y;
      SFmt<P>::load((const char*)S.aux + pv, ne, e, x);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        y.c[k].re = c * x.c[k].re + a * h.c[k].re;
        y.c[k].im = c * x.c[k].im + a * h.c[k].im;
      }
      SFmt<P>::store((char*)S.out + pv, ne, e, y);
    } else {
      const T c = (T)S.st[t.rhs].c;
      cvec<T> p, q;
      SFmt<P>::load((const char*)S.aux + pv, ne, e, p);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        q.c[k].re = c * p.c[k].re - T(0.5) * h.c[k].re;
        q.c[k].im = c * p.c[k].im - T(0.5) * h.c[k].im;
      }
      if (MODE == S_CGR) {
        const T alpha = (T)(fold_alpha ? s_alpha[t.rhs] : S.st[t.rhs].alpha);
        char* r = (char*)S.r + (both ? (size_t)par * S.astride : 0);
        cvec<T> rv;
        SFmt<P>::load(r, ne, e, rv);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          rv.c[k].re -= alpha * q.c[k].re;
          rv.c[k].im -= alpha * q.c[k].im;
        }
        SFmt<P>::store(r, ne, e, rv);
        v = cvec_norm2(rv);
      } else {  // S_RESID, FP64
        const char* b = (const char*)S.b + (both ? (size_t)par * S.hstride : 0);
        char* rh = (char*)S.rh + (both ? (size_t)par * S.hstride : 0);
        cvec<double> bv, res;
        SFmt<F64>::load(b, ne, e, bv);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          res.c[k].re = bv.c[k].re - (double)q.c[k].re;
          res.c[k].im = bv.c[k].im - (double)q.c[k].im;
        }
        SFmt<F64>::store(rh, ne, e, res);
        v = cvec_norm2(res);
      }
    }
  }
  if (L.fin != FIN_NONE) block_reduce_store(L, S, t, v);
}

template <int P, int R, int MODE, int D>
__global__ void __launch_bounds__(kBlock) stag_kernel(const Launch L) {
  stag_body<P, R, MODE, D, false>(L);
}

template <int P, int R, int MODE, int D>
__global__ void __launch_bounds__(kBlock) stag_kernel_nt(const Launch L) {
  stag_body<P, R, MODE, D, true>(L);
}

template <int P, int R, int MODE, int D>
static hipError_t stag_one(const Launch& L, bool nt, hipStream_t stream) {
  const dim3 grid((unsigned)L.total_blocks), block((unsigned)(D * L.sblk * L.nrhs));
  {
    if (nt) {
      hipLaunchKernelGGL((stag_kernel_nt<P, R, MODE, D>), grid, block, 0, stream, L);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((stag_kernel<P, R, MODE, D>), grid, block, 0, stream, L);
  return hipGetLastError();
}

template <int P, int R, int MODE>
static hipError_t stag_split(const Launch& L, bool nt, hipStream_t stream) {
  switch (L.split) {
    case 1: return stag_one<P, R, MODE, 1>(L, nt, stream);
    case 2: return stag_one<P, R, MODE, 2>(L, nt, stream);
    case 4: return stag_one<P, R, MODE, 4>(L, nt, stream);
  }
  return hipErrorInvalidValue;
}

template <int P, int R>
static hipError_t stag_mode(const Launch& L, int mode, bool nt, hipStream_t stream) {
  switch (mode) {
    case S_PLAIN: return stag_split<P, R, S_PLAIN>(L, nt, stream);
    case S_XPAY: return stag_split<P, R, S_XPAY>(L, nt, stream);
    case S_NORM: return stag_split<P, R, S_NORM>(L, nt, stream);
    case S_CGR: return stag_split<P, R, S_CGR>(L, nt, stream);
    case S_RESID:
      if constexpr (P == F64) return stag_split<P, R, S_RESID>(L, nt, stream);
      return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

// L.split threads per (site, rhs): 1, 2 or 4, each taking 8 / split hops.
// Links take the non-temporal hint when the launch's link fields exceed
// kStreamLinkBytes, or when an FP64 launch moves more than kStreamLaunchBytes.
hipError_t launch_stag(const Launch& L0, int prec, int recon, int mode, hipStream_t stream) {
  if (L0.total_blocks <= 0) return hipSuccess;
  const Launch& L = L0;
  if (L.split != 1 && L.split != 2 && L.split != 4) return hipErrorInvalidValue;
  if (L.split * L.sblk * L.nrhs > kBlock) return hipErrorInvalidValue;
  // every slot has the same decision (see item_streams_links)
  const bool nt = item_streams_links(L.s[0].g.n, L.parity, L.nrhs, prec, recon, mode, true);
  if (prec == F64)
    return recon == 12 ? stag_mode<F64, 12>(L, mode, nt, stream) : stag_mode<F64, 18>(L, mode, nt, stream);
  if (prec == F32)
    return recon == 12 ? stag_mode<F32, 12>(L, mode, nt, stream) : stag_mode<F32, 18>(L, mode, nt, stream);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// CG vector kernels on colour vectors (the accumulation precision equals the
// inner precision: FP64 or FP32).
//   BLAS_INIT  : x_h = 0, x = 0, r = low(b), p = low(b);   |b|^2 -> FIN_INIT
//   BLAS_CGUPD : x += alpha p (active rhs); p = r + beta p (running rhs); with
//                prefin = FIN_CG every block first finishes the |r|^2 reduction
//   BLAS_RU_ACC: x_h += x, x = 0                            (held rhs)
//   BLAS_RU_FIN: r = low(r_h), p = r + beta p               (resumed rhs)
// ---------------------------------------------------------------------------
template <int P, int MODE>
__global__ void __launch_bounds__(kBlock) sblas_kernel(const Launch L) {
  using T = typename RealOf<P>::T;
  const Tile t = make_tile(L);
  const Slot& S = L.s[t.slot];
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
    cvec<T> p, x, r;
    if (on) {
      SFmt<P>::load((const char*)S.out + pv, ne, e, p);
      SFmt<P>::load((const char*)S.x + pa, ne, e, x);
      SFmt<P>::load((const char*)S.r + pa, ne, e, r);
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
      const T alpha = (T)S.st[t.rhs].alpha;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        x.c[k].re += alpha * p.c[k].re;
        x.c[k].im += alpha * p.c[k].im;
      }
      SFmt<P>::store((char*)S.x + pa, ne, e, x);
      if (state == ST_RUN) {
        const T beta = (T)beta_d;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          p.c[k].re = r.c[k].re + beta * p.c[k].re;
          p.c[k].im = r.c[k].im + beta * p.c[k].im;
        }
        SFmt<P>::store((char*)S.out + pv, ne, e, p);
      }
    }
    return;
  }
  if (t.valid && rhs_selected(S.st, L.mask, t.rhs)) {
    if (MODE == BLAS_INIT) {
      cvec<double> b;
      SFmt<F64>::load((const char*)S.b + ph, ne, e, b);
      v = cvec_norm2(b);
      cvec<double> z;
      cvec_zero(z);
      SFmt<F64>::store((char*)S.xh + ph, ne, e, z);
      cvec<T> lb, xz;
#pragma unroll
      for (int k = 0; k < 3; ++k) lb.c[k] = {(T)b.c[k].re, (T)b.c[k].im};
      cvec_zero(xz);
      SFmt<P>::store((char*)S.r + pa, ne, e, lb);
      SFmt<P>::store((char*)S.x + pa, ne, e, xz);
      SFmt<P>::store((char*)S.out + pv, ne, e, lb);
    } else if (MODE == BLAS_RU_ACC) {
      cvec<double> xh;
      cvec<T> x;
      SFmt<F64>::load((const char*)S.xh + ph, ne, e, xh);
      SFmt<P>::load((const char*)S.x + pa, ne, e, x);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        xh.c[k].re += (double)x.c[k].re;
        xh.c[k].im += (double)x.c[k].im;
      }
      SFmt<F64>::store((char*)S.xh + ph, ne, e, xh);
      cvec_zero(x);
      SFmt<P>::store((char*)S.x + pa, ne, e, x);
    } else {  // BLAS_RU_FIN
      const T beta = (T)S.st[t.rhs].beta;
      cvec<double> rh;
      SFmt<F64>::load((const char*)S.rh + ph, ne, e, rh);
      cvec<T> r, p;
#pragma unroll
      for (int k = 0; k < 3; ++k) r.c[k] = {(T)rh.c[k].re, (T)rh.c[k].im};
      SFmt<P>::store((char*)S.r + pa, ne, e, r);
      SFmt<P>::load((const char*)S.out + pv, ne, e, p);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        p.c[k].re = r.c[k].re + beta * p.c[k].re;
        p.c[k].im = r.c[k].im + beta * p.c[k].im;
      }
      SFmt<P>::store((char*)S.out + pv, ne, e, p);
    }
  }
  if (L.fin != FIN_NONE) block_reduce_store(L, S, t, v);
}

template <int P>
static hipError_t sblas_mode(const Launch& L, int mode, hipStream_t stream) {
  dim3 grid((unsigned)L.total_blocks), block((unsigned)(L.sblk * L.nrhs));
  switch (mode) {
    case BLAS_INIT: hipLaunchKernelGGL((sblas_kernel<P, BLAS_INIT>), grid, block, 0, stream, L); break;
    case BLAS_CGUPD: hipLaunchKernelGGL((sblas_kernel<P, BLAS_CGUPD>), grid, block, 0, stream, L); break;
    case BLAS_RU_ACC: hipLaunchKernelGGL((sblas_kernel<P, BLAS_RU_ACC>), grid, block, 0, stream, L); break;
    case BLAS_RU_FIN: hipLaunchKernelGGL((sblas_kernel<P, BLAS_RU_FIN>), grid, block, 0, stream, L); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sblas(const Launch& L0, int prec, int mode, hipStream_t stream) {
  if (L0.total_blocks <= 0) return hipSuccess;
  Launch L = L0;
  L.split = 1;
  if (prec == F64) return sblas_mode<F64>(L, mode, stream);
  if (prec == F32) return sblas_mode<F32>(L, mode, stream);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// complex128 [rhs][t][z][y][x][3] <-> internal parity blocks.  parities = 1:
// even sites only (block at dst; the export writes zeros at odd sites);
// 2: both (even block at dst, odd block at dst + pstride).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int stag_parity_of(const Geom& g, int i) {
  const int x = i % g.L[0];
  int r = i / g.L[0];
  const int y = r % g.L[1];
  r /= g.L[1];
  const int z = r % g.L[2];
  const int t = r / g.L[2];
  return (x + y + z + t) & 1;
}

template <int P>
__global__ void stag_import_kernel(const double2* __restrict__ src, char* __restrict__ dst, size_t pstride, Geom g,
                                   int nrhs, int parities) {
  using T = typename RealOf<P>::T;
  const int V = 2 * g.n;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)V * nrhs) return;
  const int r = (int)(idx / V);
  const int i = (int)(idx % V);
  const int parity = stag_parity_of(g, i);
  if (parities == 1 && parity == 1) return;
  const double2* p = src + ((size_t)r * V + i) * 3;
  cvec<T> v;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double2 d = p[k];
    v.c[k] = {(T)d.x, (T)d.y};
  }
  const size_t ne = (size_t)g.n * nrhs;
  SFmt<P>::store(dst + (parities == 2 ? parity * pstride : 0), ne, (size_t)(i >> 1) * nrhs + r, v);
}

template <int P>
__global__ void stag_export_kernel(const char* __restrict__ src, size_t pstride, double2* __restrict__ dst, Geom g,
                                   int nrhs, int parities) {
  using T = typename RealOf<P>::T;
  const int V = 2 * g.n;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)V * nrhs) return;
  const int r = (int)(idx / V);
  const int i = (int)(idx % V);
  const int parity = stag_parity_of(g, i);
  double2* p = dst + ((size_t)r * V + i) * 3;
  if (parities == 1 && parity == 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) p[k] = make_double2(0.0, 0.0);
    return;
  }
  cvec<T> v;
  const size_t ne = (size_t)g.n * nrhs;
  SFmt<P>::load(src + (parities == 2 ? parity * pstride : 0), ne, (size_t)(i >> 1) * nrhs + r, v);
#pragma unroll
  for (int k = 0; k < 3; ++k) p[k] = make_double2((double)v.c[k].re, (double)v.c[k].im);
}

hipError_t launch_stag_import(const void* src, void* dst, size_t pstride, const Geom& g, int nrhs, int parities,
                              int prec, hipStream_t stream) {
  const long long total = 2LL * g.n * nrhs;
  const unsigned grid = (unsigned)((total + 255) / 256);
  const double2* s = (const double2*)src;
  char* d = (char*)dst;
  if (prec == F64)
    hipLaunchKernelGGL((stag_import_kernel<F64>), dim3(grid), dim3(256), 0, stream, s, d, pstride, g, nrhs, parities);
  else if (prec == F32)
    hipLaunchKernelGGL((stag_import_kernel<F32>), dim3(grid), dim3(256), 0, stream, s, d, pstride, g, nrhs, parities);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_stag_export(const void* src, size_t pstride, void* dst, const Geom& g, int nrhs, int parities,
                              int prec, hipStream_t stream) {
  const long long total = 2LL * g.n * nrhs;
  const unsigned grid = (unsigned)((total + 255) / 256);
  const char* s = (const char*)src;
  double2* d = (double2*)dst;
  if (prec == F64)
    hipLaunchKernelGGL((stag_export_kernel<F64>), dim3(grid), dim3(256), 0, stream, s, pstride, d, g, nrhs, parities);
  else if (prec == F32)
    hipLaunchKernelGGL((stag_export_kernel<F32>), dim3(grid), dim3(256), 0, stream, s, pstride, d, g, nrhs, parities);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace wd
