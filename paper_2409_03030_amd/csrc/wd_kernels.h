// Host-callable launchers of the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "wd_launch.h"

namespace wd {

// Epilogues of the staggered stencil (H = the hopping part, anti-Hermitian):
//   S_PLAIN: out = H in
//   S_XPAY : out = c aux + a H in        (c, a) = (st.c, st.alpha) or (coef, coef2)
//   S_NORM : out = H in; |out|^2 + c |aux|^2 (aux at the output site's index) -> FIN_ALPHA
//   S_CGR  : r -= alpha (c aux - H in); |r|^2 -> FIN_CG
//   S_RESID: r_h = b - (c aux - H in); |r_h|^2 -> FIN_RESID (FP64)
enum StagMode : int { S_PLAIN = 0, S_XPAY = 1, S_NORM = 2, S_CGR = 3, S_RESID = 4 };

// Stencil with epilogue `mode` (HopMode) at precision prec and link recon.
hipError_t launch_hop(const Launch& L, int prec, int recon, int mode, hipStream_t stream);

// Algorithmic bytes of one stencil launch over `sites` output sites with
// nrhs fields: 8 links per site (shared by the rhs), the input spinor once,
// and the epilogue vectors of the mode once each.
double hop_launch_bytes(int prec, int recon, int mode, long long sites, int nrhs);
// The same for the staggered stencil (StagMode).
double stag_launch_bytes(int prec, int recon, int mode, long long sites, int nrhs);

// A stencil reads each link once.  Its links take the non-temporal hint when
// they cannot stay in the 256 MB Infinity Cache until the next launch: when
// the link field exceeds three quarters of it (kStreamLinkBytes), or, at FP64,
// when the launch itself moves more than three times its size
// (kStreamLaunchBytes), so that nothing it reads survives to the next launch
// anyway.  Otherwise ordinary loads leave the links resident there.
// (Measured, hinted against ordinary: FP64 links of 50-75 MB (16^3x32) 8 %
// slower solves; FP32 links of 127 MB (24^3x48) a 26 % slower stencil; FP64
// links of 127-191 MB (24^3x24) 11-15 % slower stencils; 12 FP64 fields at
// 16^3x32 (launches up to 0.65 GB) 4 % slower propagators; FP64 links of
// 255-382 MB (24^3x48) and FP32 links of 402 MB (32^3x64) 8-13 % and 10 %
// faster stencils; FP16 links of 201 and 302 MB (32^3x64, recon 12 and 18)
// the four stencils of a CG iteration 8 % and 12 % faster.  The launch-size
// condition keeps FP64 items that move more than three times the Infinity
// Cache per launch on the hinted loads.)
constexpr double kStreamLinkBytes = 192e6;
constexpr double kStreamLaunchBytes = 768e6;

// The decision is taken for each item (lattice and its nrhs fields) on its own,
// as if it ran alone, and the solve engine puts only items with the same
// decisions into one launch: the streamed and the ordinary kernels may round
// differently (their code is scheduled apart), so an item's results would
// otherwise depend on what shares its launches.  n sites per parity; parity 2
// = both; stag: the staggered stencil's byte count.
inline bool item_streams_links(long long n, int parity, int nrhs, int prec, int recon, int mode, bool stag) {
  const double link = (prec == F64 ? 16.0 : prec == F32 ? 8.0 : 4.0) * (recon == 12 ? 6 : 9);
  const long long sites = n * (parity == 2 ? 2 : 1) * nrhs;
  if ((double)n * 8 * link > kStreamLinkBytes) return true;
  if (prec != F64) return false;
  const double b = stag ? stag_launch_bytes(prec, recon, mode, sites, nrhs) : hop_launch_bytes(prec, recon, mode, sites, nrhs);
  return b > kStreamLaunchBytes;
}

// The CG vector update reads and writes the inner solution x, which no
// stencil reads, with the non-temporal hint when the launch's inner vectors
// exceed half the Infinity Cache.  (Measured, hinted against ordinary: the
// 24^3x48 plain FP64 solve, 318 MB of vectors, 29.3 against 28.4 ms and the
// FP32-inner one, 160 MB, 16.8 against 16.5 ms; 12 FP32 sources at 16^3x32,
// 378 MB, 6-7 % faster batched solves; single 16^3x32 FP32-inner solves,
// 32 MB, 2 % slower.)  Unlike the links' hint this one is taken per launch:
// it changes only the loads and stores of x, while each component's update is
// the same single FMA in both kernels, so an item's results do not depend on
// what shares its launches.
constexpr double kStreamVecBytes = 128e6;

// CG vector kernel `mode` (BlasMode); prec is the precision of p (the
// accumulation vectors x, r are F32 when prec is F16, else prec).
hipError_t launch_blas(const Launch& L, int prec, int mode, hipStream_t stream);

// Stage 2 of the reductions of a launch that had fin != FIN_NONE: one block
// per slot sums the block partials and runs the CG scalar update.
hipError_t launch_finalize(const Launch& L, hipStream_t stream);

// complex128 boundary gauge field [mu][t][z][y][x][3][3] -> store.
hipError_t launch_gauge_import(const void* U, void* store, const Geom& g, int prec, int recon,
                               hipStream_t stream);

// complex128 boundary spinors [rhs][t][z][y][x][4][3] <-> internal parity
// blocks.  parities = 1: even sites only (block at dst); 2: both (even block
// at dst, odd block at dst + pstride).
hipError_t launch_spinor_import(const void* src, void* dst, size_t pstride, const Geom& g, int nrhs,
                                int parities, int prec, hipStream_t stream);
hipError_t launch_spinor_export(const void* src, size_t pstride, void* dst, const Geom& g, int nrhs,
                                int parities, int prec, hipStream_t stream);

// v <- g5 v on `parities` FP64 parity blocks (pstride bytes apart) of ne
// elements each.
hipError_t launch_gamma5_f64(void* v, size_t pstride, size_t ne, int parities, hipStream_t stream);

// Pion correlator of nsrc propagator columns S (complex128 boundary layout,
// nc complex values per site: 12 Wilson, 3 staggered): block partials
// (Lt * pion_shares(Lt) doubles) then corr[Lt] (device).
int pion_shares(int Lt);
hipError_t launch_pion(const void* S, const Geom& g, int nsrc, int t0, int nc, double* partial, double* corr,
                       hipStream_t stream);

// Streaming read of `bytes` (a multiple of 16) by `blocks` blocks of 256
// threads; one double per block is written to out.
hipError_t launch_read_probe(const void* buf, size_t bytes, double* out, int blocks, hipStream_t stream);

// Pseudofermion force F_mu(x) = U dS_f/dU from X = (D^dag D)^{-1} eta and
// Y = D X (FP64 internal fields, one rhs, parity blocks pstride bytes apart)
// and the FP64 link store; F complex128 [mu][t][z][y][x][3][3].
hipError_t launch_force(const void* X, const void* Y, size_t pstride, const void* gauge, int recon, const Geom& g,
                        const float bc[4], double kappa, void* F, hipStream_t stream);

// p += factor * TA(F) over nmat 3x3 complex128 matrices.
hipError_t launch_ta_add(void* p, const void* F, double factor, long long nmat, hipStream_t stream);

// Staggered stencil (StagMode) and CG vector kernels (BlasMode) at FP64 or
// FP32; colour-vector layout conversions to and from complex128
// [rhs][t][z][y][x][3].
hipError_t launch_stag(const Launch& L, int prec, int recon, int mode, hipStream_t stream);
hipError_t launch_sblas(const Launch& L, int prec, int mode, hipStream_t stream);
hipError_t launch_stag_import(const void* src, void* dst, size_t pstride, const Geom& g, int nrhs, int parities,
                              int prec, hipStream_t stream);
hipError_t launch_stag_export(const void* src, size_t pstride, void* dst, const Geom& g, int nrhs, int parities,
                              int prec, hipStream_t stream);

}  // namespace wd
