// Launch descriptors shared by the host driver and the kernels.
//
// One launch covers up to kMaxSlots "slots"; a slot is one lattice with nrhs
// right-hand sides (all slots of a launch have the same nrhs).  Work is tiled
// as (slot, parity, block of sblk sites) x nrhs threads: thread t of a block
// handles site t / nrhs of the block and rhs t % nrhs, so the nrhs threads of
// a site sit in adjacent lanes, read the same links (one memory request per
// wave) and adjacent 16-byte spinor chunks.  The stencil may also split the
// 8 hops of a site over `split` threads (part-major: part p is threads
// [p*sblk*nrhs, (p+1)*sblk*nrhs)), which multiplies the waves in flight.
#pragma once

#include "wd_device.h"

namespace wd {

constexpr int kMaxSlots = 8;
constexpr int kBlock = 256;     // threads per block, except the 8-way split stencil
constexpr int kMaxBlock = 512;  // threads per block of the 8-way split stencil

// Per right-hand-side solver state.  Lives in device memory; written by the
// host before a solve and afterwards only by the last block of a reduction.
struct RhsState {
  double rho;        // <r, r> of the current residual
  double rho_prev;   // rho at the start of the last iteration (for beta after an update)
  double alpha, beta;
  double max_rho;    // largest rho since the last reliable update
  double bnorm2;     // ||b||^2 (FP64)
  double stop2;      // host writes tol^2; INIT turns it into tol^2 ||b||^2
  double delta2;     // reliable-update trigger, squared
  double c;          // epilogue coefficient of the inner operator (kappa or kappa^2)
  double true_res2;  // last true ||b - A x||^2
  double iter_res2;  // last iterated ||r||^2
  int state;         // ST_*
  int active;        // 1 if the current iteration updates this rhs
  int ru;            // 1 if the last reliable update resumed this rhs
  int iters, maxiter, reliable;
  int pad[2];
};

enum State : int { ST_RUN = 0, ST_HOLD = 1, ST_DONE = 2, ST_NOTCONV = 3, ST_NONFINITE = 4 };
enum Mask : int { MASK_NONE = 0, MASK_RUN = 1, MASK_HOLD = 2, MASK_RU = 3, MASK_ACTIVE = 4 };
enum HopMode : int { HOP_PLAIN = 0, HOP_XPAY = 1, HOP_CGR = 2, HOP_RESID = 3 };
enum BlasMode : int { BLAS_INIT = 0, BLAS_CGUPD = 1, BLAS_RU_ACC = 2, BLAS_RU_FIN = 3 };
enum Fin : int { FIN_NONE = 0, FIN_ALPHA = 1, FIN_CG = 2, FIN_RESID = 3, FIN_INIT = 4, FIN_ALPHA_ALL = 5 };

struct Slot {
  Geom g;
  float bc[4];
  int blk0;             // first block of the slot in the launch
  int nblk;             // blocks of the slot over all parities of the launch
  int npart;            // partials finished by this launch (prefin / fold): the producing launch's nblk
  const char* gauge;    // link store of the launch's precision
  const void* in;       // stencil input (P precision), parity block of the input parity
  void* out;            // output (P precision; F64 in HOP_RESID)
  const void* aux;      // epilogue operand (P precision)
  void* r;              // residual (accumulation precision)
  const void* b;        // source (F64)
  void* x;              // low-precision solution (accumulation precision)
  void* xh;             // FP64 solution
  void* rh;             // FP64 residual
  size_t vstride;       // bytes between parity blocks of a P-precision vector
  size_t astride;       // ... of an accumulation-precision vector
  size_t hstride;       // ... of an F64 vector
  RhsState* st;
  double* partial;      // [nblk][nrhs] block partial sums
};

struct Launch {
  Slot s[kMaxSlots];
  int nslots;
  int nrhs;
  int sblk;             // sites per block (power of two)
  int split;            // threads per (site, rhs) in the stencil: 1, 2, 4 or 8 (each takes 8/split hops)
  int parity;           // output parity 0 / 1, or 2 = both (input = the other one)
  int g5in, g5out;
  int mask;             // Mask
  int fin;              // Fin
  int prefin;           // Fin of the previous launch's partials, run alongside or before this launch's own
                        // work: by one extra workgroup per slot at the start of a Wilson stencil's grid, by
                        // block 0 of each slot in a staggered stencil, by every block for FIN_CG (CG vector
                        // update) and FIN_ALPHA_ALL (staggered residual update)
  int swz;              // block order: 0 plain, 1 XCD-aware, 2 XCD-aware with the t-slices of an XCD's range
                        // visited innermost (see logical_block)
  int bt;               // swz 2: logical blocks per t-slice (of the only slot, or of all interleaved groups);
                        // 0 = order as swz 1
  int ilv;              // 1: the slots are right-hand-side groups of one lattice (same geometry, links and
                        // block count); logical block b is block b / nslots of slot b % nslots, so the
                        // groups' blocks for the same sites run next to each other (links read from the L2)
  int total_blocks;
  int tsS[2];           // swz 2: t-slices in an XCD's range of q + 1 (index 1) or q (index 0) blocks, q =
                        // total_blocks / 8, where that range is at least two whole slices; else 0
  FastDiv dts[2];       // division by tsS[i]
  FastDiv dpart, drhs, dslots;  // division by sblk * nrhs, nrhs and nslots (finish_launch)
  int* work_flag;       // timed launches: set to 1 by a block of a slot that does its work; else null
  double coef;          // epilogue coefficient when no RhsState is attached
  double coef2;         // second coefficient (staggered XPAY) when no RhsState is attached
};

}  // namespace wd
