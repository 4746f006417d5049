// The Wilson hopping stencil with fused epilogues.
//
// One thread computes (H in)(x) for one output site x and one rhs (or a
// share of its 8 hops, when `split` threads take one site): for each
// direction it loads the neighbour spinor, spin-projects it to a half spinor
// (adds and i-swaps only), multiplies the half spinor by the link (U or
// U^dag), applies the boundary sign, and accumulates the rebuilt full
// spinor: 8 x (12 + 132) + 7 x 24 = 1320 flop per output site.
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

// The split stencil's parts finish the output together when each part's
// share (12 / D components) is whole 16-byte chunks: FP64 with 2 or 4 parts,
// FP32 with 2.  Otherwise part 0 finishes the whole site: FP16, whose
// per-site scale needs all 24 reals (a variant exchanging each half's largest
// component through LDS was 5 % slower), FP32 with 4 parts (half-chunk
// accesses: faster at 24^3x48, slower at 16^3x32), and 8 parts.
template <int P, int D> struct SplitEpilogue {
  static constexpr bool value = (P == F64 && (D == 2 || D == 4)) || (P == F32 && D == 2);
};

// Components c0 .. c0+NK-1 of a spinor (NK = 12: the whole spinor, any format).
template <int P, int NK, typename T>
__device__ __forceinline__ void load_comps(const void* base, size_t ne, size_t e, int c0, cplx<T>* s) {
  if constexpr (NK == 12) {
    spinor<T> sp;
    SpinorFmt<P>::load(base, ne, e, sp);
#pragma unroll
    for (int k = 0; k < 12; ++k) s[k] = sp.c[k];
  } else {
    SpinorFmt<P>::template load_comps<NK>(base, ne, e, c0, s);
  }
}

template <int P, int NK, typename T>
__device__ __forceinline__ void store_comps(void* base, size_t ne, size_t e, int c0, const cplx<T>* s) {
  if constexpr (NK == 12) {
    spinor<T> sp;
#pragma unroll
    for (int k = 0; k < 12; ++k) sp.c[k] = s[k];
    SpinorFmt<P>::store(base, ne, e, sp);
  } else {
    SpinorFmt<P>::template store_comps<NK>(base, ne, e, c0, s);
  }
}

// The epilogue on components c0 .. c0+NK-1 of the site's H in (h, after the
// optional gamma5): stores them and returns their part of the launch's norm.
template <int P, int A, int MODE, int NK, typename T>
__device__ __forceinline__ double hop_epilogue_comps(const Launch& L, const Slot& S, const Tile& t, bool both,
                                                     int par, size_t ne, size_t e, int c0, const cplx<T>* h) {
  using TA = typename RealOf<A>::T;
  if constexpr (MODE == HOP_PLAIN) {
    char* out = (char*)S.out + (both ? (size_t)par * S.vstride : 0);
    store_comps<P, NK>(out, ne, e, c0, h);
    return 0.0;
  } else {
    const T c = (T)(S.st ? S.st[t.rhs].c : L.coef);
    const char* aux = (const char*)S.aux + (both ? (size_t)par * S.vstride : 0);
    cplx<T> a[NK];
    load_comps<P, NK>(aux, ne, e, c0, a);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      a[k].re -= c * h[k].re;
      a[k].im -= c * h[k].im;
    }
    double v = 0.0;
    if constexpr (MODE == HOP_XPAY) {
      char* out = (char*)S.out + (both ? (size_t)par * S.vstride : 0);
      store_comps<P, NK>(out, ne, e, c0, a);
#pragma unroll
      for (int k = 0; k < NK; ++k) v += (double)a[k].re * (double)a[k].re + (double)a[k].im * (double)a[k].im;
    } else if constexpr (MODE == HOP_CGR) {
      const TA alpha = (TA)S.st[t.rhs].alpha;
      char* r = (char*)S.r + (both ? (size_t)par * S.astride : 0);
      cplx<TA> rv[NK];
      load_comps<A, NK>(r, ne, e, c0, rv);
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        rv[k].re -= alpha * (TA)a[k].re;
        rv[k].im -= alpha * (TA)a[k].im;
      }
      store_comps<A, NK>(r, ne, e, c0, rv);
#pragma unroll
      for (int k = 0; k < NK; ++k) v += (double)rv[k].re * (double)rv[k].re + (double)rv[k].im * (double)rv[k].im;
    } else {  // HOP_RESID, FP64 only
      const char* b = (const char*)S.b + (both ? (size_t)par * S.hstride : 0);
      char* rh = (char*)S.rh + (both ? (size_t)par * S.hstride : 0);
      cplx<double> bv[NK], res[NK];
      load_comps<F64, NK>(b, ne, e, c0, bv);
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        res[k].re = bv[k].re - (double)a[k].re;
        res[k].im = bv[k].im - (double)a[k].im;
      }
      store_comps<F64, NK>(rh, ne, e, c0, res);
#pragma unroll
      for (int k = 0; k < NK; ++k) v += res[k].re * res[k].re + res[k].im * res[k].im;
    }
    return v;
  }
}

// NT: links read with the non-temporal hint (hop_kernel_nt), for launches
// whose links cannot stay in the Infinity Cache (stream_links).
template <int P, int R, int MODE, int D, bool NT>
__device__ __forceinline__ void hop_body(const Launch& L) {
  using T = typename RealOf<P>::T;
  constexpr int A = AccOf<P>::value;
  // The previous launch's reduction is finished by nslots extra workgroups at
  // the start of the grid, one per slot, while the others run the stencil:
  // this launch's own work must not depend on it (its mask reads only states
  // that the finalize step leaves unchanged for the selected rhs).
  // LDS: the parts' exchange of sums, which the finalize-only workgroups use
  // for their stage-2 sums instead, and the block reduction's buffer.
  constexpr int kThreads = D == 8 ? kMaxBlock : kBlock;
  constexpr size_t kAccBytes = D > 1 ? (size_t)(D - 1) * 24 * (kThreads / D) * sizeof(T) : 0;
  constexpr size_t kRawBytes = kAccBytes > kRedSlots * sizeof(double) ? kAccBytes : kRedSlots * sizeof(double);
  __shared__ __align__(16) unsigned char lds_raw[kRawBytes];
  __shared__ double lds_red[kThreads];
  const int lead = L.prefin != FIN_NONE ? L.nslots : 0;
  if ((int)blockIdx.x < lead) {
    gather_and_finalize_buf(L, L.s[blockIdx.x], L.prefin, (double*)lds_raw);
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
  if (L.work_flag != nullptr && t.lblk == 0 && threadIdx.x == 0) *L.work_flag = 1;
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
  double v = 0.0;
  if constexpr (SplitEpilogue<P, D>::value) {
    // Each part finishes 12/D of the site's components: part p takes the
    // other parts' sums of its components from LDS and adds all D in part
    // order (the same sums as one thread adding whole spinors), then loads,
    // combines and stores only its own chunks.
    constexpr int NK = 12 / D;
    T* lds_acc = (T*)lds_raw;
    const int per = L.sblk * L.nrhs;
    const int p = t.part;
    const int loc = (int)threadIdx.x - p * per;
    // writer q, owner o != q: block q * (D - 1) + (o < q ? o : o - 1) of 2 NK reals
    auto blk = [&](int q, int o) { return lds_acc + (size_t)((q * (D - 1) + (o < q ? o : o - 1)) * 2 * NK) * per + loc; };
    if (sel) {
#pragma unroll
      for (int o = 0; o < D; ++o) {
        if (o == p) continue;
        T* d = blk(p, o);
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          d[(2 * k) * per] = acc.c[o * NK + k].re;
          d[(2 * k + 1) * per] = acc.c[o * NK + k].im;
        }
      }
    }
    __syncthreads();
    if (sel) {
      cplx<T> mine[NK], h[NK];
#pragma unroll
      for (int o = 0; o < D; ++o)
        if (o == p) {
#pragma unroll
          for (int k = 0; k < NK; ++k) mine[k] = acc.c[o * NK + k];
        }
#pragma unroll
      for (int q = 0; q < D; ++q) {
        cplx<T> x[NK];
        if (q == p) {
#pragma unroll
          for (int k = 0; k < NK; ++k) x[k] = mine[k];
        } else {
          const T* src = blk(q, p);
#pragma unroll
          for (int k = 0; k < NK; ++k) x[k] = {src[(2 * k) * per], src[(2 * k + 1) * per]};
        }
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          if (q == 0) h[k] = x[k];
          else h[k] = cadd(h[k], x[k]);
        }
      }
      const int c0 = p * NK;
      if (L.g5out) {
#pragma unroll
        for (int k = 0; k < NK; ++k)
          if (c0 + k >= 6) h[k] = cneg(h[k]);
      }
      v = hop_epilogue_comps<P, A, MODE, NK>(L, S, t, both, par, ne, e, c0, h);
    }
    if (L.fin != FIN_NONE) block_reduce_store_buf(L, S, t, v, D, lds_red);
  } else {
    if (D > 1) {
      // parts 1..D-1 hand their sums to part 0, which adds them in part order
      T* lds_acc = (T*)lds_raw;
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
    if (sel && t.part == 0) {
      if (L.g5out) gamma5_inplace(acc);
      v = hop_epilogue_comps<P, A, MODE, 12>(L, S, t, both, par, ne, e, 0, acc.c);
    }
    if (L.fin != FIN_NONE) block_reduce_store_buf(L, S, t, v, 1, lds_red);
  }
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
  if (nt) {
    hipLaunchKernelGGL((hop_kernel_nt<P, R, MODE, D>), grid, block, 0, stream, L);
    return hipGetLastError();
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

// Links take the non-temporal hint when an item's link field exceeds
// kStreamLinkBytes, or when its FP64 launch alone would move more than
// kStreamLaunchBytes.  Every slot of a launch has the same decision (the
// engine groups only such items), so slot 0 decides.
static bool stream_links(const Launch& L, int prec, int recon, int mode) {
  return item_streams_links(L.s[0].g.n, L.parity, L.nrhs, prec, recon, mode, false);
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
