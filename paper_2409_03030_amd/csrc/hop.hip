// The Wilson hopping stencil with fused epilogues.
//
// One thread computes (H in)(x) for one output site x and one rhs: for each
// of the 8 directions it loads the neighbour spinor, spin-projects it to a
// half spinor (adds and i-swaps only), multiplies the half spinor by the
// link (U or U^dag), applies the boundary sign, and accumulates the rebuilt
// full spinor: 8 x (12 + 132) + 7 x 24 = 1320 flop per output site.
// The epilogue then forms one of
//   HOP_PLAIN : out = [g5] H [g5] in
//   HOP_XPAY  : out = aux - c [g5] H [g5] in          (+ ||out||^2, FIN_ALPHA)
//   HOP_CGR   : r  -= alpha (aux - c [g5] H [g5] in)  (+ ||r||^2,  FIN_CG)
//   HOP_RESID : rh  = b - (aux - c [g5] H [g5] in)    (+ ||rh||^2, FIN_RESID)
// so that the CG on D_hat^dag D_hat never stores A p separately and its dot
// products ride on the stencil's own output.
#include "wd_kcommon.h"
#include "wd_kernels.h"

namespace wd {

template <int P> struct AccOf { static constexpr int value = P == F16 ? F32 : P; };

// NT: links read with the non-temporal hint (hop_kernel_nt, FP64 and FP32),
// for launches whose links cannot stay in the Infinity Cache (stream_links).
template <int P, int R, int MODE, int D, bool NT>
__device__ __forceinline__ void hop_body(const Launch& L) {
  using T = typename RealOf<P>::T;
  constexpr int A = AccOf<P>::value;
  using TA = typename RealOf<A>::T;
  // The previous launch's reduction is finished by nslots extra workgroups at
  // the start of the grid, one per slot, while the others run the stencil:
  // this launch's own work must not depend on it (its mask reads only states
  // that the finalize step leaves unchanged for the selected rhs).
  const int lead = L.prefin != FIN_NONE ? L.nslots : 0;
  if ((int)blockIdx.x < lead) {
    gather_and_finalize(L, L.s[blockIdx.x], L.prefin);
    return;
  }
  const Tile t = make_tile(L, lead);
  const Slot& S = L.s[t.slot];
  // A slot with no selected rhs does nothing, not even its block partials:
  // stage 2 changes no state of an unselected rhs whatever the sums (FIN_ALPHA
  // leaves only running rhs active, FIN_CG acts on active rhs, FIN_RESID on
  // held ones), and the mask of a reducing launch reads states that no block
  // of it changes.  Masked iterations after convergence then cost a launch.
  if (!slot_selected(L, S)) return;
  const bool both = L.parity == 2;
  const int par = t.parity;
  const size_t ne = (size_t)S.g.n * L.nrhs;
  const size_t e = (size_t)t.site * L.nrhs + t.rhs;
  const bool sel = t.valid && rhs_selected(S.st, L.mask, t.rhs);
  spinor<T> acc;
  if (sel) {
    const char* in = (const char*)S.in + (both ? (size_t)(1 - par) * S.vstride : 0);
    hop_part<P, R, D, NT>(S.g, par, t.site, t.rhs, L.nrhs, S.gauge, in, S.bc, L.g5in != 0, t.part, acc);
  }
  if (D > 1) {
    // parts 1..D-1 hand their sums to part 0, which adds them in part order
    constexpr int kLds = D > 1 ? (D - 1) * 24 * ((D == 8 ? kMaxBlock : kBlock) / D) : 1;
    __shared__ T lds_acc[kLds];
    const int per = L.sblk * L.nrhs;
    const int loc = (int)threadIdx.x - t.part * per;
    if (sel && t.part > 0) {
      T* q = lds_acc + (size_t)(t.part - 1) * 24 * per + loc;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        q[(2 * k) * per] = acc.c[k].re;
        q[(2 * k + 1) * per] = acc.c[k].im;
      }
    }
    __syncthreads();
    if (sel && t.part == 0) {
#pragma unroll
      for (int pp = 1; pp < D; ++pp) {
        const T* q = lds_acc + (size_t)(pp - 1) * 24 * per + loc;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          acc.c[k].re += q[(2 * k) * per];
          acc.c[k].im += q[(2 * k + 1) * per];
        }
      }
    }
  }
  double v = 0.0;
  if (sel && t.part == 0) {
    if (L.g5out) gamma5_inplace(acc);
    if (MODE == HOP_PLAIN) {
      char* out = (char*)S.out + (both ? (size_t)par * S.vstride : 0);
      SpinorFmt<P>::store(out, ne, e, acc);
    } else {
      const T c = (T)(S.st ? S.st[t.rhs].c : L.coef);
      const char* aux = (const char*)S.aux + (both ? (size_t)par * S.vstride : 0);
      spinor<T> a;
      SpinorFmt<P>::load(aux, ne, e, a);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        a.c[k].re -= c * acc.c[k].re;
        a.c[k].im -= c * acc.c[k].im;
      }
      if (MODE == HOP_XPAY) {
        char* out = (char*)S.out + (both ? (size_t)par * S.vstride : 0);
        SpinorFmt<P>::store(out, ne, e, a);
        v = spinor_norm2(a);
      } else if (MODE == HOP_CGR) {
        const TA alpha = (TA)S.st[t.rhs].alpha;
        char* r = (char*)S.r + (both ? (size_t)par * S.astride : 0);
        spinor<TA> rv;
        SpinorFmt<A>::load(r, ne, e, rv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          rv.c[k].re -= alpha * (TA)a.c[k].re;
          rv.c[k].im -= alpha * (TA)a.c[k].im;
        }
        SpinorFmt<A>::store(r, ne, e, rv);
        v = spinor_norm2(rv);
      } else {  // HOP_RESID, FP64 only
        const char* b = (const char*)S.b + (both ? (size_t)par * S.hstride : 0);
        char* rh = (char*)S.rh + (both ? (size_t)par * S.hstride : 0);
        spinor<double> bv, res;
        SpinorFmt<F64>::load(b, ne, e, bv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          res.c[k].re = bv.c[k].re - (double)a.c[k].re;
          res.c[k].im = bv.c[k].im - (double)a.c[k].im;
        }
        SpinorFmt<F64>::store(rh, ne, e, res);
        v = spinor_norm2(res);
      }
    }
  }
  if (L.fin != FIN_NONE) block_reduce_store(L, S, t, v);
}

template <int P, int R, int MODE, int D>
__global__ void __launch_bounds__(D == 8 ? kMaxBlock : kBlock) hop_kernel(const Launch L) {
  hop_body<P, R, MODE, D, false>(L);
}

template <int P, int R, int MODE, int D>
__global__ void __launch_bounds__(D == 8 ? kMaxBlock : kBlock) hop_kernel_nt(const Launch L) {
  hop_body<P, R, MODE, D, true>(L);
}

template <int P, int R, int MODE, int D>
static hipError_t launch_one(const Launch& L, bool nt, hipStream_t stream) {
  const int lead = L.prefin != FIN_NONE ? L.nslots : 0;  // finalize-only workgroups
  dim3 grid((unsigned)(L.total_blocks + lead)), block((unsigned)(D * L.sblk * L.nrhs));
  if constexpr (P != F16) {
    if (nt) {
      hipLaunchKernelGGL((hop_kernel_nt<P, R, MODE, D>), grid, block, 0, stream, L);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((hop_kernel<P, R, MODE, D>), grid, block, 0, stream, L);
  return hipGetLastError();
}

template <int P, int R, int MODE>
static hipError_t launch_split(const Launch& L, bool nt, hipStream_t stream) {
  switch (L.split) {
    case 1: return launch_one<P, R, MODE, 1>(L, nt, stream);
    case 2: return launch_one<P, R, MODE, 2>(L, nt, stream);
    case 4: return launch_one<P, R, MODE, 4>(L, nt, stream);
    case 8:  // one hop per thread; its LDS combine would exceed 64 KB at FP64
      if constexpr (P != F64) return launch_one<P, R, MODE, 8>(L, nt, stream);
      return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

template <int P, int R>
static hipError_t launch_mode(const Launch& L, int mode, bool nt, hipStream_t stream) {
  if (L.split * L.sblk * L.nrhs > (L.split == 8 ? kMaxBlock : kBlock)) return hipErrorInvalidValue;
  switch (mode) {
    case HOP_PLAIN: return launch_split<P, R, HOP_PLAIN>(L, nt, stream);
    case HOP_XPAY: return launch_split<P, R, HOP_XPAY>(L, nt, stream);
    case HOP_CGR: return launch_split<P, R, HOP_CGR>(L, nt, stream);
    case HOP_RESID:
      if constexpr (P == F64) return launch_split<P, R, HOP_RESID>(L, nt, stream);
      return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

// Links take the non-temporal hint when the launch's link fields exceed
// kStreamLinkBytes, or when an FP64 launch moves more than kStreamLaunchBytes
// (FP64 and FP32; the FP16 stencil always loads them ordinarily).
static bool stream_links(const Launch& L, int prec, int recon, int mode) {
  if (prec == F16) return false;
  long long sites = 0;
  for (int k = 0; k < L.nslots; ++k) sites += (long long)L.s[k].g.n * (L.parity == 2 ? 2 : 1) * L.nrhs;
  return link_field_bytes(L, prec, recon) > kStreamLinkBytes ||
         (prec == F64 && hop_launch_bytes(prec, recon, mode, sites, L.nrhs) > kStreamLaunchBytes);
}

hipError_t launch_hop(const Launch& L, int prec, int recon, int mode, hipStream_t stream) {
  if (L.total_blocks <= 0) return hipSuccess;
  const bool nt = stream_links(L, prec, recon, mode);
  if (prec == F64)
    return recon == 12 ? launch_mode<F64, 12>(L, mode, nt, stream) : launch_mode<F64, 18>(L, mode, nt, stream);
  if (prec == F32)
    return recon == 12 ? launch_mode<F32, 12>(L, mode, nt, stream) : launch_mode<F32, 18>(L, mode, nt, stream);
  if (prec == F16)
    return recon == 12 ? launch_mode<F16, 12>(L, mode, nt, stream) : launch_mode<F16, 18>(L, mode, nt, stream);
  return hipErrorInvalidValue;
}

}  // namespace wd
