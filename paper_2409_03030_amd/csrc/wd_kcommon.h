// Kernel-side plumbing shared by the stencil and vector kernels: block to
// (slot, parity, sites) mapping, per-rhs masks, and the deterministic
// two-stage FP64 reduction whose last block runs the CG scalar updates.
#pragma once

#include "wd_launch.h"

namespace wd {

struct Tile {
  int slot;
  int parity;   // output parity of this block
  int site;     // checkerboard index of this thread's site (may be >= n: idle)
  int rhs;
  int lblk;     // block index within the slot
  int part;     // which share of the hops this thread computes (stencil split)
  bool valid;   // site < n
};

// Workgroups are dealt to the 8 XCDs round robin (w -> XCD w % 8).  With
// swizzling, XCD x receives a contiguous range of logical blocks so that
// neighbouring sites share that XCD's L2.
__device__ __forceinline__ int logical_block(int w, int nb, int swz) {
  if (!swz) return w;
  const int q = nb >> 3, rem = nb & 7;
  const int x = w & 7;
  const int start = x * q + (x < rem ? x : rem);
  return start + (w >> 3);
}

__device__ __forceinline__ Tile make_tile(const Launch& L) {
  Tile t;
  const int b = logical_block((int)blockIdx.x, L.total_blocks, L.swz);
  int sl = 0;
#pragma unroll 1
  for (int i = 1; i < L.nslots; ++i)
    if (b >= L.s[i].blk0) sl = i;
  const Slot& S = L.s[sl];
  int lb = b - S.blk0;
  t.slot = sl;
  t.lblk = lb;
  if (L.parity == 2) {
    const int half = S.nblk >> 1;
    t.parity = lb >= half ? 1 : 0;
    lb -= t.parity * half;
  } else {
    t.parity = L.parity;
  }
  const int per_part = L.sblk * L.nrhs;
  const int tid = (int)threadIdx.x;
  t.part = tid / per_part;
  const int loc = tid - t.part * per_part;
  t.site = lb * L.sblk + loc / L.nrhs;
  t.rhs = loc % L.nrhs;
  t.valid = (t.part < (L.split > 0 ? L.split : 1)) && (t.site < S.g.n);
  return t;
}

__device__ __forceinline__ bool rhs_selected(const RhsState* st, int mask, int r) {
  if (mask == MASK_NONE || st == nullptr) return true;
  const RhsState& s = st[r];
  switch (mask) {
    case MASK_RUN: return s.state == ST_RUN;
    case MASK_HOLD: return s.state == ST_HOLD;
    case MASK_RU: return s.ru != 0;
    case MASK_ACTIVE: return s.active != 0;
  }
  return true;
}

// True if any rhs of the slot is selected.  Every block of a slot sees the
// same answer: states only change in the last block of a reduction, after
// every block has passed this point.
__device__ __forceinline__ bool slot_selected(const Launch& L, const Slot& S) {
  if (L.mask == MASK_NONE || S.st == nullptr) return true;
  for (int r = 0; r < L.nrhs; ++r)
    if (rhs_selected(S.st, L.mask, r)) return true;
  return false;
}

__device__ __forceinline__ bool finite_d(double v) { return v == v && v - v == 0.0; }

// CG scalar updates, one thread per rhs, run by the last block of a reduction.
__device__ void finalize_rhs(int fin, RhsState& s, double sum) {
  switch (fin) {
    case FIN_INIT: {
      s.bnorm2 = sum;
      s.rho = sum;
      s.rho_prev = sum;
      s.max_rho = sum;
      s.stop2 = s.stop2 * sum;
      s.true_res2 = sum;
      s.iter_res2 = sum;
      s.alpha = 0.0;
      s.beta = 0.0;
      s.iters = 0;
      s.reliable = 0;
      s.active = 0;
      s.ru = 0;
      if (!finite_d(sum)) s.state = ST_NONFINITE;
      else if (sum == 0.0) s.state = ST_DONE;
      else s.state = ST_RUN;
      break;
    }
    case FIN_ALPHA: {  // sum = <p, A p> = ||D p||^2
      if (s.state == ST_RUN) {
        if (finite_d(sum) && sum > 0.0) {
          s.alpha = s.rho / sum;
          s.active = 1;
        } else {
          s.alpha = 0.0;
          s.active = 0;
          s.state = ST_NONFINITE;
        }
      } else {
        s.alpha = 0.0;
        s.active = 0;
      }
      break;
    }
    case FIN_CG: {  // sum = ||r_new||^2
      if (s.active) {
        s.iters += 1;
        s.iter_res2 = sum;
        if (!finite_d(sum)) {
          s.state = ST_NONFINITE;
          s.beta = 0.0;
          break;
        }
        s.beta = sum / s.rho;
        s.rho_prev = s.rho;
        s.rho = sum;
        if (sum > s.max_rho) s.max_rho = sum;
        if (sum <= s.stop2 || sum <= s.delta2 * s.max_rho || s.iters >= s.maxiter) s.state = ST_HOLD;
      }
      break;
    }
    case FIN_RESID: {  // sum = ||b - A x_h||^2 in FP64
      if (s.state == ST_HOLD) {
        s.reliable += 1;
        s.true_res2 = sum;
        if (!finite_d(sum)) {
          s.state = ST_NONFINITE;
          s.ru = 0;
        } else if (sum <= s.stop2) {
          s.state = ST_DONE;
          s.ru = 0;
        } else if (s.iters >= s.maxiter) {
          s.state = ST_NOTCONV;
          s.ru = 0;
        } else {
          s.beta = sum / s.rho_prev;
          s.rho = sum;
          s.max_rho = sum;
          s.iter_res2 = sum;
          s.state = ST_RUN;
          s.ru = 1;
        }
      } else {
        s.ru = 0;
      }
      break;
    }
    default: break;
  }
}

// Two-stage FP64 reduction with a fixed summation order (deterministic:
// independent of block scheduling).
//
// Stage 1 (here, in the producing kernel): the block sums v per rhs (wave
// butterfly shuffles for nrhs = 1, else a tree over the block's sites) and
// writes its partial with an ordinary store.  Stage 2 runs in a separate
// one-block-per-slot kernel (finalize_kernel) after the kernel boundary has
// made every partial visible; it sums the partials in a fixed order and runs
// the CG scalar update.  (Finishing inside the producer needs either a
// device-scope release fence per block -- on gfx950 a write-back of the
// XCD's whole L2 -- or coherent stores, waits and atomics whose round trips
// serialise at the end of every block; both cost more than a small kernel.)
// All threads of the block must call this.
__device__ void block_reduce_store(const Launch& L, const Slot& S, const Tile& t, double v) {
  __shared__ double lds[kMaxBlock];
  const int tid = (int)threadIdx.x;
  const int nr = L.nrhs;
  const int sb = L.sblk;
  const int nthr = sb * nr;
  const int sl = tid / nr;
  if (nr == 1) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0) lds[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      const int nw = (nthr + 63) >> 6;
      for (int w = 0; w < nw; ++w) s += lds[w];
      S.partial[t.lblk] = s;
    }
    return;
  }
  if (tid < nthr) lds[tid] = v;
  __syncthreads();
  for (int w = sb >> 1; w > 0; w >>= 1) {
    if (sl < w) lds[tid] += lds[tid + w * nr];
    __syncthreads();
  }
  if (tid < nr) S.partial[(size_t)t.lblk * nr + tid] = lds[tid];
}

// Stage 2: block b handles slot b.  G groups of nr threads, group g summing
// partials g, g+G, ... in order with 8 loads in flight, then a fixed-order
// tree over the groups, then finalize_rhs per rhs.
__device__ void gather_and_finalize(const Launch& L, const Slot& S, int fin) {
  __shared__ double lds[kMaxBlock];
  const int tid = (int)threadIdx.x;
  const int nr = L.nrhs;
  const int T = (int)blockDim.x;
  int G = 1;
  while (2 * G * nr <= T) G *= 2;
  double acc = 0.0;
  const int g = tid / nr;
  if (g < G) {
    const int r = tid - g * nr;
    const double* part = S.partial + r;
    int b = g;
    for (; b + 7 * G < S.nblk; b += 8 * G) {
      double q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = part[(size_t)(b + u * G) * nr];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += q[u];
    }
    for (; b < S.nblk; b += G) acc += part[(size_t)b * nr];
    lds[tid] = acc;
  }
  __syncthreads();
  for (int w = G >> 1; w > 0; w >>= 1) {
    if (g < w) lds[tid] += lds[tid + w * nr];
    __syncthreads();
  }
  if (tid < nr && S.st != nullptr) finalize_rhs(fin, S.st[tid], lds[tid]);
  __syncthreads();
}

}  // namespace wd
