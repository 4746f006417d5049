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
// swz = 1, XCD x receives a contiguous range of logical blocks so that
// neighbouring sites share that XCD's L2.  With swz = 2 the XCD keeps the same
// range (so vectors written by one kernel are read from the same L2 by the
// next) but visits it in another order: the range spans S whole t-slices of bt
// blocks, and the k-th block the XCD runs is block k / S of slice k % S.  The
// t-neighbours of a site are then read within a few dozen blocks of each
// other rather than a whole slice apart, which keeps them in the L2 between
// their uses (at 24^3x48 it cut the FP64 stencil's fetched bytes from 1.37 to
// 1.10 times the algorithmic ones).  A range that is not whole slices keeps
// the swz = 1 order.
__device__ __forceinline__ int logical_block(int w, const Launch& L) {
  if (!L.swz) return w;
  const int q = L.total_blocks >> 3, rem = L.total_blocks & 7;
  const int x = w & 7;
  const int start = x * q + (x < rem ? x : rem);
  const int k = w >> 3;
  if (L.swz == 2) {
    const int hi = x < rem ? 1 : 0;  // the range holds q + 1 blocks
    const int S = L.tsS[hi];
    if (S > 0) {
      const int a = fdiv(k, L.dts[hi]);  // k / S
      return start + (k - a * S) * L.bt + a;
    }
  }
  return start + k;
}

// lead: workgroups at the start of the grid that take no tile (they finish the
// previous launch's reduction).
__device__ __forceinline__ Tile make_tile(const Launch& L, int lead = 0) {
  Tile t;
  const int b = logical_block((int)blockIdx.x - lead, L);
  int sl = 0, lb;
  if (L.ilv) {
    lb = fdiv(b, L.dslots);
    sl = b - lb * L.nslots;
  } else {
#pragma unroll 1
    for (int i = 1; i < L.nslots; ++i)
      if (b >= L.s[i].blk0) sl = i;
    lb = b - L.s[sl].blk0;
  }
  const Slot& S = L.s[sl];
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
  t.part = fdiv(tid, L.dpart);
  const int loc = tid - t.part * per_part;
  const int sr = fdiv(loc, L.drhs);
  t.site = lb * L.sblk + sr;
  t.rhs = loc - sr * L.nrhs;
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
    case FIN_ALPHA:      // sum = <p, A p> = ||D p||^2
    case FIN_ALPHA_ALL: {  // the same, without counting the iteration (see fold_finalize_alpha)
      if (s.state == ST_RUN) {
        if (finite_d(sum) && sum > 0.0) {
          s.alpha = s.rho / sum;
          s.active = 1;
          if (fin == FIN_ALPHA) s.iters += 1;
          s.rho_prev = s.rho;
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
      // Reads only fields that it leaves unchanged (active, rho_prev, iters,
      // the limits) or changes idempotently (max_rho), so running it again
      // on its own output gives the same state: every block of the next
      // vector kernel may run it while the first block stores the result.
      if (s.active) {
        s.iter_res2 = sum;
        if (!finite_d(sum)) {
          s.state = ST_NONFINITE;
          s.beta = 0.0;
          break;
        }
        s.beta = sum / s.rho_prev;
        s.rho = sum;
        if (sum > s.max_rho) s.max_rho = sum;
        s.state = (sum <= s.stop2 || sum <= s.delta2 * s.max_rho || s.iters >= s.maxiter) ? ST_HOLD : ST_RUN;
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
// writes its partial with an ordinary store.  Stage 2 runs after the kernel
// boundary has made every partial visible: in a separate one-block-per-slot
// kernel (finalize_kernel), in the first block of the next stencil, or (for
// FIN_CG with few partials) in every block of the next vector kernel; it
// sums the partials in a fixed order and runs the CG scalar update.
// (Finishing inside the producer needs either a
// device-scope release fence per block -- on gfx950 a write-back of the
// XCD's whole L2 -- or coherent stores, waits and atomics whose round trips
// serialise at the end of every block; both cost more than a small kernel.)
// parts: how many part-major groups of sblk * nrhs threads hold values (a
// stencil whose split parts each finish a share of the output components);
// the tree then runs over parts * sblk "sites".
// lds: blockDim.x doubles of LDS.  All threads of the block must call this.
__device__ void block_reduce_store_buf(const Launch& L, const Slot& S, const Tile& t, double v, int parts,
                                       double* lds) {
  const int tid = (int)threadIdx.x;
  const int nr = L.nrhs;
  const int sb = L.sblk * parts;
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

__device__ void block_reduce_store(const Launch& L, const Slot& S, const Tile& t, double v, int parts = 1) {
  __shared__ double lds[kMaxBlock];
  block_reduce_store_buf(L, S, t, v, parts, lds);
}

// Stage 2 summation order, fixed by nrhs alone so that every kernel that
// runs stage 2 (whatever its block size) gets bitwise the same sums: for
// each rhs, G groups (G = the largest power of two with G * nrhs <= 256);
// group g sums partials g, g+G, g+2G, ... in increasing order, then a
// pairwise tree combines the groups.  Threads take several groups when the
// block has fewer than G * nrhs threads.  On return red[g * nr + r] holds
// nothing useful except red[r] = the sum for rhs r.  All threads of the
// block must call this.
constexpr int kRedSlots = 256;

__device__ __forceinline__ int red_groups(int nr) {
  int G = 1;
  while (2 * G * nr <= kRedSlots) G *= 2;
  return G;
}

__device__ void reduce_partials(const double* __restrict__ part, int npart, int nr, double* red) {
  const int tid = (int)threadIdx.x;
  const int G = red_groups(nr);
  const int per = (int)blockDim.x / nr;  // groups worked on at once, per rhs
  const int r = tid % nr;
  const bool on = tid < per * nr;
  if (on) {
    for (int g = tid / nr; g < G; g += per) {
      const double* q0 = part + r;
      double acc = 0.0;
      int b = g;
      for (; b + 7 * G < npart; b += 8 * G) {
        double q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] = q0[(size_t)(b + u * G) * nr];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += q[u];
      }
      for (; b < npart; b += G) acc += q0[(size_t)b * nr];
      red[g * nr + r] = acc;
    }
  }
  __syncthreads();
  for (int w = G >> 1; w > 0; w >>= 1) {
    if (on)
      for (int g = tid / nr; g < w; g += per) red[g * nr + r] += red[(g + w) * nr + r];
    __syncthreads();
  }
}

// Stage 2 in its own kernel (block b handles slot b) or in the first block of
// the next stencil: sum the partials and run the CG scalar update.
// red: kRedSlots doubles of LDS.
__device__ void gather_and_finalize_buf(const Launch& L, const Slot& S, int fin, double* red) {
  reduce_partials(S.partial, S.npart, L.nrhs, red);
  const int tid = (int)threadIdx.x;
  if (tid < L.nrhs && S.st != nullptr) finalize_rhs(fin, S.st[tid], red[tid]);
  __syncthreads();
}

__device__ void gather_and_finalize(const Launch& L, const Slot& S, int fin) {
  __shared__ double red[kRedSlots];
  gather_and_finalize_buf(L, S, fin, red);
}

// Stage 2 of FIN_ALPHA run by every block of the stencil that needs alpha
// (the staggered residual update): each block sums the same partials in the
// same order and applies the alpha update to a private copy of the states;
// the first block of the slot stores the states and counts the iteration.
// Without the count the update reads only fields it leaves unchanged (rho,
// the state of a running rhs) or sets idempotently (alpha, active, rho_prev,
// a non-finite state), so a block that reads a state after the first block
// stored it computes the same result.
__device__ void fold_finalize_alpha(const Launch& L, const Slot& S, const Tile& t, double* alpha, int* active) {
  __shared__ double red[kRedSlots];
  reduce_partials(S.partial, S.npart, L.nrhs, red);
  const int tid = (int)threadIdx.x;
  if (tid < L.nrhs) {
    RhsState s = S.st[tid];
    const int iters = s.iters;
    finalize_rhs(FIN_ALPHA_ALL, s, red[tid]);
    alpha[tid] = s.alpha;
    active[tid] = s.active;
    if (t.lblk == 0) {
      RhsState& d = S.st[tid];
      d.alpha = s.alpha;
      d.active = s.active;
      d.rho_prev = s.rho_prev;
      d.state = s.state;
      d.iters = iters + (s.active ? 1 : 0);
    }
  }
  __syncthreads();
}

// Stage 2 of FIN_CG run by every block of the vector kernel that follows the
// reducing stencil: each block sums the same partials in the same order and
// applies FIN_CG to a private copy of the states, handing beta and the new
// state to its threads; the first block of the slot also stores the states.
// Sound because FIN_CG is idempotent (see finalize_rhs): a block that reads
// a state after the first block stored it computes the same result.
__device__ void fold_finalize_cg(const Launch& L, const Slot& S, const Tile& t, double* beta, int* state) {
  __shared__ double red[kRedSlots];
  reduce_partials(S.partial, S.npart, L.nrhs, red);
  const int tid = (int)threadIdx.x;
  if (tid < L.nrhs) {
    RhsState s = S.st[tid];
    finalize_rhs(FIN_CG, s, red[tid]);
    beta[tid] = s.beta;
    state[tid] = s.state;
    if (t.lblk == 0 && s.active) {
      RhsState& d = S.st[tid];
      d.iter_res2 = s.iter_res2;
      d.beta = s.beta;
      d.rho = s.rho;
      d.max_rho = s.max_rho;
      d.state = s.state;
    }
  }
  __syncthreads();
}

}  // namespace wd
