// CG engine: conjugate gradient on D^dag D (full lattice) or on the even-odd
// Schur complement D_hat^dag D_hat, with the inner iteration in FP64, FP32 or
// FP16 and FP64 reliable updates, for a set of solve items that may change
// between poll blocks.
//
// One inner iteration (even-odd; FULL mode fuses the parities):
//   t1 = H_oe p                               stencil, odd output
//   t2 = p - c H_eo t1 ; alpha = rho/|t2|^2   stencil + reduction  (<p,A p> = |D_hat p|^2)
//   t1 = H_oe g5 t2                           stencil
//   r -= alpha (t2 - c g5 H_eo t1) ; |r|^2    stencil + reduction  (A p never stored)
//   x += alpha p ; p = r + beta p             vector kernel
// with c = kappa^2.  A reliable update (Sleijpen and van der Vorst; held rhs
// only) does x_h += x, r_h = b - A x_h with the FP64 store, and resumes with
// r = r_h, p = r + beta p.  All scalars stay on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "wd_host.h"

namespace wd {

int min_sblk(int nrhs) {
  int s = 1;
  while (s * nrhs < 32) s *= 2;
  return s;
}

size_t states_bytes(size_t nstates) { return align_up(nstates * sizeof(RhsState)); }

size_t field_bytes(int op, int prec, size_t n, int nrhs) {
  if (op == OP_WILSON) return vec_bytes(prec, n, nrhs);
  return align_up(n * (size_t)nrhs * 3 * (prec == F64 ? 16 : 8));  // colour vectors, FP64 or FP32
}

ItemLayout item_layout(const wd_lattice_s* lat, const wd_solve_params& p, int nrhs, int op) {
  ItemLayout l;
  const size_t n = (size_t)lat->g.n;
  const int np = p.precond == WD_EO ? 1 : 2;
  const int P = p.inner, A = op == OP_WILSON ? acc_prec(P) : P;
  const size_t vh = field_bytes(op, F64, n, nrhs), va = field_bytes(op, A, n, nrhs), vp = field_bytes(op, P, n, nrhs);
  size_t o = 0;
  l.off_partial = o;
  o += align_up((size_t)np * ((n + min_sblk(nrhs) - 1) / min_sblk(nrhs)) * nrhs * sizeof(double));
  l.off_bh = o; o += np * vh;
  l.off_xh = o; o += np * vh;
  l.off_rh = o; o += np * vh;
  l.off_h1 = o; o += np * vh;
  l.off_h2 = o; o += np * vh;
  l.off_x = o; o += np * va;
  l.off_r = o; o += np * va;
  l.off_p = o; o += np * vp;
  l.off_t1 = o; o += np * vp;
  l.off_t2 = o; o += np * vp;
  l.hstride = vh;
  l.astride = va;
  l.vstride = vp;
  l.total = o;
  return l;
}

enum Role { R_NONE, R_P, R_T1, R_T2, R_BH, R_XH, R_H1, R_H2 };

static void* role_ptr(const EItem* it, int role) {
  const ItemLayout& l = it->lay;
  char* b = it->base;
  switch (role) {
    case R_P: return b + l.off_p;
    case R_T1: return b + l.off_t1;
    case R_T2: return b + l.off_t2;
    case R_BH: return b + l.off_bh;
    case R_XH: return b + l.off_xh;
    case R_H1: return b + l.off_h1;
    case R_H2: return b + l.off_h2;
  }
  return nullptr;
}

static uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
  const unsigned char* c = (const unsigned char*)data;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

struct Engine::Phase {
  bool hop;
  int prec;  // -1 = the inner precision
  int mode;
  int parity;
  int g5in, g5out;
  int mask, fin;
  int in, out, aux;
  int prefin;       // finalize of the previous phase's reduction, folded into this launch
  bool fin_folded;  // this phase's reduction is finished by the next phase (prefin)
  bool fold_small;  // FIN_CG producer / consumer pair: fold when every slot has few partials
};

// A reduction is finished by every block of the launch that consumes it
// (FIN_CG in the vector update, the staggered alpha in its residual update)
// when each slot has at most kFoldPartials block partials and the consumer's
// blocks together read at most kFoldReads of them (wd_host.h).

// Consumer blocks of a slot: the stencil's own block count, or the vector
// kernels' (blas_sblk sites per block).
static int blas_sblk(int nrhs);

static bool fold_ok(const Launch& L, bool consumer_is_blas) {
  for (int k = 0; k < L.nslots; ++k) {
    const Slot& S = L.s[k];
    const long long parts = (long long)S.npart * L.nrhs;
    if (parts > kFoldPartials) return false;
    const int sb = consumer_is_blas ? std::max(blas_sblk(L.nrhs), L.sblk) : L.sblk;
    const long long blocks = ((long long)S.g.n + sb - 1) / sb * (L.parity == 2 ? 2 : 1);
    if (blocks * parts > kFoldReads) return false;
  }
  return true;
}

// Sites per block of the vector kernels, whatever the stencil's shape, so that
// a folded stage 2 (every block reading all the stencil's partials) is not
// repeated by many small blocks: 256 threads for one right-hand side, else
// the fewest sites (a power of two) that give a block more than 64 threads.
// (Measured at 16^3x32: with 256 threads rather than 128 the single-field
// staggered FP64 and FP32 solves ran 1.6 % and 2.5 % faster and the Wilson
// solves the same; the 12-field batched Wilson solves at 192 threads rather
// than 96 ran 0.5 % slower.  FP32 stencil blocks of 64 sites, once used for
// the vector kernels too, made the solve 4 % slower.)
static int blas_sblk(int nrhs) {
  if (nrhs == 1) return kBlock;
  int s = 1;
  while (2 * s * nrhs <= kBlock / 2) s *= 2;
  return s;
}

wd_status Engine::run_phase(const std::vector<EItem*>& list, const Phase& ph0) {
  Phase ph = ph0;
  if (ph.prec < 0) ph.prec = p_.inner;
  size_t i = 0;
  while (i < list.size()) {
    // a launch: consecutive items with the same nrhs, the same link recon of
    // the store this phase reads (the kernel decodes every slot's links with
    // one recon), the same tuned launch shape and the same link-load
    // decisions (item_streams_links), at most kMaxSlots.  The
    // shape fixes each slot's arithmetic (the hop split orders the sum over
    // the 8 hops, the block size the first stage of every reduction), so an
    // item computes the same bits whatever shares its launches.  Producer and
    // consumer phases of a folded reduction read the same precision, so they
    // split alike.
    const int nrhs = list[i]->nrhs;
    const wd_lattice_s* lat0 = list[i]->lat;
    const int recon = lat0->store[ph.prec].recon;
    auto lookup = [&](const wd_lattice_s* lat) {
      return op_ == OP_STAG ? stag_tune_lookup(lat, ph.prec, recon, nrhs) : tune_lookup(lat, ph.prec, recon, nrhs);
    };
    const Tune t = lookup(lat0);
    // the items' link-load decisions in every stencil mode at this precision
    // (taken for each item on its own): equal within a launch
    auto streams = [&](const wd_lattice_s* lat) {
      int mask = 0;
      for (int m = 0; m < (op_ == OP_STAG ? 5 : 4); ++m)
        if (item_streams_links(lat->g.n, ph.parity, nrhs, ph.prec, recon, m, op_ == OP_STAG)) mask |= 1 << m;
      return mask;
    };
    const int st0 = streams(lat0);
    size_t j = i + 1;
    while (j < list.size() && j - i < (size_t)kMaxSlots && list[j]->nrhs == nrhs &&
           list[j]->lat->store[ph.prec].recon == recon) {
      const Tune tj = lookup(list[j]->lat);
      if (tj.sblk != t.sblk || tj.split != t.split || tj.swz != t.swz) break;
      if (streams(list[j]->lat) != st0) break;
      ++j;
    }
    Launch L = base_launch(nrhs, t, ph.parity);
    L.g5in = ph.g5in;
    L.g5out = ph.g5out;
    L.mask = ph.mask;
    L.fin = ph.fin;
    L.prefin = ph.prefin;
    L.nslots = (int)(j - i);
    long long sites = 0;
    for (size_t k = i; k < j; ++k) {
      const EItem* it = list[k];
      Slot& S = L.s[k - i];
      fill_slot_geometry(S, it->lat, t.sblk, ph.parity);
      S.gauge = (const char*)it->lat->store[ph.prec].ptr;
      S.in = role_ptr(it, ph.in);
      S.out = role_ptr(it, ph.out);
      S.aux = role_ptr(it, ph.aux);
      const ItemLayout& l = it->lay;
      S.r = it->base + l.off_r;
      S.x = it->base + l.off_x;
      S.b = it->base + l.off_bh;
      S.xh = it->base + l.off_xh;
      S.rh = it->base + l.off_rh;
      S.vstride = ph.prec == F64 ? l.hstride : l.vstride;
      S.astride = l.astride;
      S.hstride = l.hstride;
      S.st = it->st;
      S.partial = (double*)(it->base + l.off_partial);
      sites += (long long)it->lat->g.n * (ph.parity == 2 ? 2 : 1) * nrhs;
    }
    if (!ph.hop) {
      // vector kernel: its own block shape; a folded stage 2 still reads the
      // partials of the stencil launch before it
      const int sb = std::max(blas_sblk(nrhs), t.sblk);
      L.sblk = sb;
      for (size_t k2 = i; k2 < j; ++k2) {
        Slot& S = L.s[k2 - i];
        const int npart = S.nblk;
        fill_slot_geometry(S, list[k2]->lat, sb, ph.parity);
        if (ph.prefin != FIN_NONE) S.npart = npart;
      }
    }
    finish_launch(L);
    // Fold decisions, taken alike by the producing and the consuming launch:
    // the consumer of a FIN_CG fold is a vector kernel, that of the staggered
    // alpha fold the residual-update stencil (the producer's geometry).
    const bool folded = ph.fold_small && ph.fin != FIN_NONE && fold_ok(L, ph.fin == FIN_CG);
    if (ph.fold_small && ph.prefin != FIN_NONE && !fold_ok(L, !ph.hop)) L.prefin = FIN_NONE;
    if (hash_) {
      // key of a captured block: every launch's kernel choice and arguments
      const int id[5] = {ph.hop ? 1 : 0, ph.prec, recon, ph.mode, op_};
      *hash_ = fnv1a(*hash_, id, sizeof id);
      *hash_ = fnv1a(*hash_, &L, sizeof L);
      i = j;
      continue;
    }
    if (ph.hop) {
      L.work_flag = timer_ ? timer_->next_flag() : nullptr;
      hipError_t e = timer_ ? timer_->begin(stream_) : hipSuccess;
      if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
      e = op_ == OP_STAG ? launch_stag(L, ph.prec, recon, ph.mode, stream_)
                         : launch_hop(L, ph.prec, recon, ph.mode, stream_);
      if (e != hipSuccess) return hip_fail(e, "stencil launch");
      const double bytes = op_ == OP_STAG ? stag_launch_bytes(ph.prec, recon, ph.mode, sites, nrhs)
                                          : hop_launch_bytes(ph.prec, recon, ph.mode, sites, nrhs);
      e = timer_ ? timer_->end(stream_, sites, bytes, (op_ == OP_STAG ? 0 : ph.mode) + 4 * ph.prec) : hipSuccess;
      if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    } else {
      hipError_t e = op_ == OP_STAG ? launch_sblas(L, ph.prec, ph.mode, stream_)
                                    : launch_blas(L, ph.prec, ph.mode, stream_);
      if (e != hipSuccess) return hip_fail(e, "vector kernel launch");
    }
    if (ph.fin != FIN_NONE && !ph.fin_folded && !folded) {
      hipError_t e = launch_finalize(L, stream_);
      if (e != hipSuccess) return hip_fail(e, "finalize launch");
    }
    i = j;
  }
  return WD_OK;
}

wd_status Engine::run_iteration() {
  // EO: the alpha reduction of the second stencil is finished by the first
  // block of the third, which selects running rhs (alpha only changes the
  // state of a running rhs when <p, A p> is not positive and finite).
  static const Phase eo[5] = {
      {true, -1, HOP_PLAIN, 1, 0, 0, MASK_RUN, FIN_NONE, R_P, R_T1, R_NONE, FIN_NONE, false},
      {true, -1, HOP_XPAY, 0, 0, 0, MASK_RUN, FIN_ALPHA, R_T1, R_T2, R_P, FIN_NONE, true},
      {true, -1, HOP_PLAIN, 1, 1, 0, MASK_RUN, FIN_NONE, R_T2, R_T1, R_NONE, FIN_ALPHA, false},
      {true, -1, HOP_CGR, 0, 0, 1, MASK_ACTIVE, FIN_CG, R_T1, R_NONE, R_T2, FIN_NONE, false, true},
      {false, -1, BLAS_CGUPD, 0, 0, 0, MASK_ACTIVE, FIN_NONE, R_NONE, R_P, R_NONE, FIN_CG, false, true},
  };
  static const Phase full[3] = {
      {true, -1, HOP_XPAY, 2, 0, 0, MASK_RUN, FIN_ALPHA, R_P, R_T2, R_P, FIN_NONE, false},
      {true, -1, HOP_CGR, 2, 1, 1, MASK_ACTIVE, FIN_CG, R_T2, R_NONE, R_T2, FIN_NONE, false, true},
      {false, -1, BLAS_CGUPD, 2, 0, 0, MASK_ACTIVE, FIN_NONE, R_NONE, R_P, R_NONE, FIN_CG, false, true},
  };
  // Staggered (even block M_e = m^2 - H_eo H_oe, c = m^2): alpha needs the
  // whole <p, M_e p> before the residual update, so every block of that
  // update finishes the alpha reduction itself when the partials are few (else
  // a finalize kernel runs between the two stencils).
  static const Phase st[3] = {
      {true, -1, S_NORM, 1, 0, 0, MASK_RUN, FIN_ALPHA, R_P, R_T1, R_P, FIN_NONE, false, true},
      {true, -1, S_CGR, 0, 0, 0, MASK_ACTIVE, FIN_CG, R_T1, R_NONE, R_P, FIN_ALPHA_ALL, false, true},
      {false, -1, BLAS_CGUPD, 0, 0, 0, MASK_ACTIVE, FIN_NONE, R_NONE, R_P, R_NONE, FIN_CG, false, true},
  };
  const Phase* k = op_ == OP_STAG ? st : eo_ ? eo : full;
  const int nk = op_ == OP_STAG ? 3 : eo_ ? 5 : 3;
  for (int q = 0; q < nk; ++q) {
    wd_status s = run_phase(items, k[q]);
    if (s != WD_OK) return s;
  }
  return WD_OK;
}

wd_status Engine::run_reliable() {
  static const Phase eo[6] = {
      {false, -1, BLAS_RU_ACC, 0, 0, 0, MASK_HOLD, FIN_NONE, R_NONE, R_P, R_NONE, FIN_NONE, false},
      {true, F64, HOP_PLAIN, 1, 0, 0, MASK_HOLD, FIN_NONE, R_XH, R_H1, R_NONE, FIN_NONE, false},
      {true, F64, HOP_XPAY, 0, 0, 0, MASK_HOLD, FIN_NONE, R_H1, R_H2, R_XH, FIN_NONE, false},
      {true, F64, HOP_PLAIN, 1, 1, 0, MASK_HOLD, FIN_NONE, R_H2, R_H1, R_NONE, FIN_NONE, false},
      {true, F64, HOP_RESID, 0, 0, 1, MASK_HOLD, FIN_RESID, R_H1, R_NONE, R_H2, FIN_NONE, false},
      {false, -1, BLAS_RU_FIN, 0, 0, 0, MASK_RU, FIN_NONE, R_NONE, R_P, R_NONE, FIN_NONE, false},
  };
  static const Phase full[4] = {
      {false, -1, BLAS_RU_ACC, 2, 0, 0, MASK_HOLD, FIN_NONE, R_NONE, R_P, R_NONE, FIN_NONE, false},
      {true, F64, HOP_XPAY, 2, 0, 0, MASK_HOLD, FIN_NONE, R_XH, R_H2, R_XH, FIN_NONE, false},
      {true, F64, HOP_RESID, 2, 1, 1, MASK_HOLD, FIN_RESID, R_H2, R_NONE, R_H2, FIN_NONE, false},
      {false, -1, BLAS_RU_FIN, 2, 0, 0, MASK_RU, FIN_NONE, R_NONE, R_P, R_NONE, FIN_NONE, false},
  };
  static const Phase st[4] = {
      {false, -1, BLAS_RU_ACC, 0, 0, 0, MASK_HOLD, FIN_NONE, R_NONE, R_P, R_NONE, FIN_NONE, false},
      {true, F64, S_PLAIN, 1, 0, 0, MASK_HOLD, FIN_NONE, R_XH, R_H1, R_NONE, FIN_NONE, false},
      {true, F64, S_RESID, 0, 0, 0, MASK_HOLD, FIN_RESID, R_H1, R_NONE, R_XH, FIN_NONE, false},
      {false, -1, BLAS_RU_FIN, 0, 0, 0, MASK_RU, FIN_NONE, R_NONE, R_P, R_NONE, FIN_NONE, false},
  };
  const Phase* k = op_ == OP_STAG ? st : eo_ ? eo : full;
  const int nk = op_ == OP_STAG ? 4 : eo_ ? 6 : 4;
  for (int q = 0; q < nk; ++q) {
    wd_status s = run_phase(items, k[q]);
    if (s != WD_OK) return s;
  }
  return WD_OK;
}

wd_status Engine::start_item(EItem* it) {
  it->h_init.assign(it->nrhs, RhsState{});
  for (int r = 0; r < it->nrhs; ++r) {
    RhsState& s = it->h_init[r];
    memset(&s, 0, sizeof s);
    const double k = it->kappa[r];
    s.stop2 = p_.tol * p_.tol;
    s.delta2 = p_.delta * p_.delta;
    s.c = (eo_ || op_ == OP_STAG) ? k * k : k;  // kappa^2, kappa, or the staggered m^2
    s.maxiter = p_.maxiter;
    s.state = ST_RUN;
  }
  WD_HIP(hipMemcpyAsync(it->st, it->h_init.data(), it->nrhs * sizeof(RhsState), hipMemcpyHostToDevice, stream_));
  if (op_ == OP_STAG)
    WD_HIP(launch_stag_import(it->b, it->base + it->lay.off_bh, it->lay.hstride, it->lat->g, it->nrhs, eo_ ? 1 : 2,
                              F64, stream_));
  else
    WD_HIP(launch_spinor_import(it->b, it->base + it->lay.off_bh, it->lay.hstride, it->lat->g, it->nrhs,
                                eo_ ? 1 : 2, F64, stream_));
  const Phase init = {false, -1, BLAS_INIT, eo_ ? 0 : 2, 0, 0, MASK_NONE, FIN_INIT, R_NONE, R_P, R_NONE, FIN_NONE,
                      false};
  std::vector<EItem*> one{it};
  it->started_block = blocks;
  return run_phase(one, init);
}

wd_status Engine::export_item(EItem* it) {
  if (op_ == OP_STAG)
    WD_HIP(launch_stag_export(it->base + it->lay.off_xh, it->lay.hstride, it->x, it->lat->g, it->nrhs, eo_ ? 1 : 2,
                              F64, stream_));
  else
    WD_HIP(launch_spinor_export(it->base + it->lay.off_xh, it->lay.hstride, it->x, it->lat->g, it->nrhs,
                                eo_ ? 1 : 2, F64, stream_));
  return WD_OK;
}

int Engine::max_block() const {
  long long work = 0;
  for (auto* it : items) work += (long long)it->lat->g.n * it->nrhs * (eo_ ? 1 : 2);
  int K = p_.poll_every;
  if (K <= 0) K = (int)std::max(4LL, std::min(32LL, (1LL << 22) / std::max(1LL, work)));
  return K;
}

// Block sizes used for captured graphs: a small set keeps the cache small.
static int round_block(int k, int kmax) {
  static const int sizes[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};
  int best = 1;
  for (int s : sizes)
    if (s <= k) best = s;
  return std::min(best, kmax);
}

constexpr double kEstShrink = 0.8;

// Iterations until the next event (convergence or a reliable update) of a
// running rhs, extrapolated from the decrease of its iterated residual.
// With one rhs running, a late block end costs masked iterations (a launch
// each) and an early one an extra poll, so the estimate leans early: the
// faster of the rate since the previous poll and the rate since the first
// poll, shortened by kEstShrink (CG converges faster than its recent rate
// towards the end, and after a reliable update the recent rate can be near
// zero), and a short probe block of kmax / 4 where neither rate shows a
// decrease.  With several rhs in the launches a held rhs only idles while the
// others run, so blocks follow the recent rate and stay long (measured with
// 12 and 36 point sources: the early-leaning rule made the batched solves
// 5-9 % slower through extra polls).
int BlockPlanner::next(const RhsState* hs, size_t n, int inflight, const int* idx) {
  double best = 1e30, best_full = 1e30;
  bool any = false;
  nrun = 0;
  for (size_t j = 0; j < n; ++j) {
    const size_t q = idx ? (size_t)idx[j] : j;
    const RhsState& s = hs[q];
    if (!(s.state == ST_DONE || s.state == ST_NOTCONV || s.state == ST_NONFINITE)) ++nrun;
  }
  const bool lean = nrun == 1;
  for (size_t j = 0; j < n; ++j) {
    const size_t q = idx ? (size_t)idx[j] : j;
    if (snap.size() <= q) snap.resize(q + 1, Snap{-1, 0.0, -1, 0.0});
    const RhsState& s = hs[q];
    if (s.state == ST_DONE || s.state == ST_NOTCONV || s.state == ST_NONFINITE) continue;
    any = true;
    if (s.state == ST_HOLD) {  // its update runs at the end of the block in flight
      best = std::min(best, 1.0);
      best_full = std::min(best_full, 1.0);
      continue;
    }
    const double rho = s.iter_res2 > 0.0 ? s.iter_res2 : s.rho;
    double target = s.stop2;
    if (s.delta2 > 0.0) target = std::max(target, s.delta2 * s.max_rho);
    Snap& sn = snap[q];
    double est = (sn.iters0 < 0 || !lean) ? (double)kmax : std::max(1.0, kmax / 4.0);
    double rate = 0.0;  // log decrease per iteration (negative when decreasing)
    if (sn.iters >= 0 && s.iters > sn.iters && sn.rho > 0.0 && rho > 0.0)
      rate = std::min(rate, std::log(rho / sn.rho) / (s.iters - sn.iters));
    if (lean && sn.iters0 >= 0 && s.iters > sn.iters0 && sn.rho0 > 0.0 && rho > 0.0)
      rate = std::min(rate, std::log(rho / sn.rho0) / (s.iters - sn.iters0));
    double est_full = est;
    if (rate < -1e-6) {
      est_full = std::log(target / rho) / rate;
      est = (lean ? kEstShrink : 1.0) * est_full;
    }
    if (sn.iters0 < 0 && rho > 0.0) {
      sn.iters0 = s.iters;
      sn.rho0 = rho;
    }
    sn.iters = s.iters;
    sn.rho = rho;
    est = std::max(0.0, est);
    best = std::min(best, est);
    best_full = std::min(best_full, std::max(0.0, est_full));
  }
  if (!any) return 0;
  left = best - inflight;  // iterations still needed after the blocks in flight
  left_full = best_full - inflight;
  if (left < 0.5) return -1;  // the event falls in a block in flight: wait for it
  return round_block((int)std::ceil(left), kmax);
}

int Engine::reliable_every() const { return 0; }

// K inner iterations, then (ru) one reliable-update sequence: held rhs
// (converged iterate, delta drop, or maxiter) get their FP64 true residual
// there.  The host sizes K so that a block ends where the next such event is
// expected, and leaves the sequence out of a block not expected to reach one
// (it would run masked).
wd_status Engine::enqueue_direct(int K, bool ru) {
  for (int j = 0; j < K; ++j) {
    wd_status s = run_iteration();
    if (s != WD_OK) return s;
  }
  return ru ? run_reliable() : WD_OK;
}

// Instantiated graphs, shared by every engine of the process and keyed by the
// exact launches they contain, so repeated solves on the same buffers replay
// without capturing again.  An entry is destroyed only after the last replay
// recorded on it has completed.
namespace {
struct GraphEntry {
  uint64_t key;
  hipGraphExec_t exec;
  hipEvent_t last;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;  // most recently used last
constexpr size_t kGraphCap = 48;
}  // namespace

// A block is K copies of one iteration's launches plus, or not, one
// reliable-update sequence, so its key is the hash of those launches, K and ru.
uint64_t Engine::block_key(int K, bool ru) {
  if (base_key_ == 0) {
    uint64_t h = 1469598103934665603ull;
    hash_ = &h;
    (void)run_iteration();
    (void)run_reliable();
    hash_ = nullptr;
    base_key_ = h | 1;
  }
  const int kr[2] = {K, ru ? 1 : 0};
  return fnv1a(base_key_, kr, sizeof kr);
}

wd_status Engine::enqueue_block(int K, bool ru) {
  if (items.empty()) return WD_OK;
  const int every = reliable_every();
  if (K < 1) K = 1;
  if (every > 0 && K % every) K = (K / every + 1) * every;
  ++blocks;
  if (!p_.use_graph || timer_) return enqueue_direct(K, ru);
  const uint64_t key = block_key(K, ru);
  std::lock_guard<std::mutex> lk(g_graph_mu);
  GraphEntry ent{0, nullptr, nullptr};
  for (size_t i = 0; i < g_graphs.size(); ++i)
    if (g_graphs[i].key == key) {
      ent = g_graphs[i];
      g_graphs.erase(g_graphs.begin() + i);
      break;
    }
  if (!ent.exec) {
    // capture only blocks that repeat: the first use of a key launches
    // directly (a changing set of served requests rarely repeats a block)
    bool seen = false;
    for (uint64_t k : seen_)
      if (k == key) seen = true;
    if (!seen) {
      if (seen_.size() >= 256) seen_.erase(seen_.begin());
      seen_.push_back(key);
      return enqueue_direct(K, ru);
    }
    WD_HIP(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
    wd_status s = enqueue_direct(K, ru);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(stream_, &g);
    if (s != WD_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&ent.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    e = hipEventCreateWithFlags(&ent.last, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipGraphExecDestroy(ent.exec);
      return hip_fail(e, "hipEventCreate");
    }
    ent.key = key;
  }
  hipError_t e = hipGraphLaunch(ent.exec, stream_);
  if (e == hipSuccess) e = hipEventRecord(ent.last, stream_);
  g_graphs.push_back(ent);
  while (g_graphs.size() > kGraphCap) {
    GraphEntry old = g_graphs.front();
    g_graphs.erase(g_graphs.begin());
    (void)hipEventSynchronize(old.last);
    (void)hipGraphExecDestroy(old.exec);
    (void)hipEventDestroy(old.last);
  }
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return WD_OK;
}

wd_status stats_from_state(const RhsState& s, double seconds, const HopTimer* t, wd_solve_stats& o) {
  memset(&o, 0, sizeof o);
  o.iters = s.iters;
  o.reliable_updates = s.reliable;
  const double bn = s.bnorm2 > 0.0 ? s.bnorm2 : 1.0;
  o.true_resid = std::sqrt(s.true_res2 / bn);
  o.iter_resid = std::sqrt(s.iter_res2 / bn);
  o.seconds = seconds;
  if (t && t->on) {
    o.hop_launches = (long long)(t->dur.size()) - t->nskipped;
    o.hop_skipped = (int32_t)t->nskipped;
    o.hop_site_updates = t->site_updates;
    o.hop_bytes = t->bytes;
  }
  if (s.state == ST_DONE) o.status = WD_OK;
  else if (s.state == ST_NONFINITE) o.status = WD_ENONFINITE;
  else o.status = WD_ENOTCONVERGED;
  return o.status;
}

static bool finished(int st) { return st == ST_DONE || st == ST_NOTCONV || st == ST_NONFINITE; }

// The legacy null stream cannot be captured into a graph.  Solves given it run
// on a per-thread blocking stream instead, which the null stream orders with
// the caller's other work (legacy default-stream semantics).
static hipStream_t solve_stream(hipStream_t s, wd_status* st) {
  *st = WD_OK;
  if (s) return s;
  static thread_local hipStream_t own = nullptr;
  if (!own) {
    hipError_t e = hipStreamCreate(&own);
    if (e != hipSuccess) {
      *st = hip_fail(e, "hipStreamCreate");
      own = nullptr;
      return nullptr;
    }
  }
  return own;
}

// The work flags of timed stencil launches (HopTimer): a ring per device,
// shared by the timed solves running on it at the same time (their skipped
// counts are then unreliable).  Its address is looked up once per device.
static __device__ int timing_flags[kTimingFlags];
static std::mutex g_flags_mu;
static int* g_flags_ptr[64];

static wd_status timing_flags_address(int** out) {
  int dev = -1;
  WD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(WD_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_flags_mu);
  if (!g_flags_ptr[dev]) {
    void* q = nullptr;
    const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(timing_flags));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(timing_flags)");
    g_flags_ptr[dev] = (int*)q;
  }
  *out = g_flags_ptr[dev];
  return WD_OK;
}

wd_status run_batch(std::vector<EItem>& items, const wd_solve_params& p, RhsState* states, hipStream_t stream_in,
                    wd_solve_stats* stats, int op) {
  auto t0 = std::chrono::steady_clock::now();
  wd_status sst;
  hipStream_t stream = solve_stream(stream_in, &sst);
  if (sst != WD_OK) return sst;
  HopTimer timer;
  timer.on = p.timing != 0;
  if (timer.on) {
    wd_status fs = timing_flags_address(&timer.flags);
    if (fs != WD_OK) return fs;
    const hipError_t e = hipMemsetAsync(timer.flags, 0, kTimingFlags * sizeof(int), stream);
    if (e != hipSuccess) return hip_fail(e, "timing flags clear");
  }
  Engine eng(p, stream, states, timer.on ? &timer : nullptr, op);
  size_t nst = 0;
  for (auto& it : items) nst += (size_t)it.nrhs;
  wd_status result = WD_OK;
  for (auto& it : items) {
    eng.items.push_back(&it);
    if ((result = eng.start_item(&it)) != WD_OK) return result;
  }
  RhsState* hs[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  do {
    hipError_t e;
    if ((e = hipHostMalloc((void**)&hs[0], nst * sizeof(RhsState), hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&hs[1], nst * sizeof(RhsState), hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&ev[0], hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&ev[1], hipEventDisableTiming)) != hipSuccess) {
      result = hip_fail(e, "poll buffers");
      break;
    }
    // Up to two blocks in flight: while the GPU runs one block the host reads
    // the states copied after the previous one and sizes the next block so
    // that it ends where the next reliable update or convergence is expected.
    BlockPlanner plan;
    plan.kmax = eng.max_block();
    struct Posted {
      int buf, K;
    };
    std::vector<Posted> fly;
    int next_buf = 0;
    auto post = [&](int K, bool ru) -> wd_status {
      wd_status s = eng.enqueue_block(K, ru);
      if (s != WD_OK) return s;
      const int k = next_buf;
      next_buf ^= 1;
      hipError_t e2 = hipMemcpyAsync(hs[k], states, nst * sizeof(RhsState), hipMemcpyDeviceToHost, stream);
      if (e2 != hipSuccess) return hip_fail(e2, "state copy");
      e2 = hipEventRecord(ev[k], stream);
      if (e2 != hipSuccess) return hip_fail(e2, "hipEventRecord");
      fly.push_back({k, K});
      return WD_OK;
    };
    const int k0 = std::min(plan.kmax, 8);
    if ((result = post(k0, true)) != WD_OK) break;
    if ((result = post(k0, true)) != WD_OK) break;
    long long iters_posted = 2LL * k0;
    for (;;) {
      const Posted done = fly.front();
      fly.erase(fly.begin());
      e = hipEventSynchronize(ev[done.buf]);
      if (e != hipSuccess) {
        result = hip_fail(e, "hipEventSynchronize");
        break;
      }
      int inflight = 0;
      for (auto& f : fly) inflight += f.K;
      const int K = plan.next(hs[done.buf], nst, inflight);
      if (K == 0) break;  // every rhs finished
      if (iters_posted > (long long)p.maxiter + 64LL * plan.kmax) break;  // device caps iterations; bounds the host loop
      if (K < 0) {
        if (fly.empty() && (result = post(1, true)) != WD_OK) break;
        continue;
      }
      // the reliable-update sequence only in a block expected to reach the
      // next event by the unshrunk extrapolation (a block sized to the
      // early-leaning estimate usually ends short of it, and its sequence
      // would run masked; a rhs that gets there early waits for the next
      // block's sequence)
      if ((result = post(K, K + 0.5 >= plan.left_full)) != WD_OK) break;
      iters_posted += K;
      if (fly.size() < 2 && K >= plan.kmax && (plan.nrun > 1 || plan.left >= 2.0 * K)) {
        // far from any event: keep a second block queued so the GPU never waits
        if ((result = post(K, 2 * K + 0.5 >= plan.left_full)) != WD_OK) break;
        iters_posted += K;
      }
    }
  } while (false);
  hipError_t es = hipStreamSynchronize(stream);
  if (result == WD_OK && es != hipSuccess) result = hip_fail(es, "hipStreamSynchronize");
  std::vector<RhsState> fin(nst);
  if (result == WD_OK) {
    hipError_t e = hipMemcpy(fin.data(), states, nst * sizeof(RhsState), hipMemcpyDeviceToHost);
    if (e != hipSuccess) result = hip_fail(e, "final state copy");
  }
  if (result == WD_OK) {
    for (auto& it : items)
      if ((result = eng.export_item(&it)) != WD_OK) break;
    hipError_t e = hipStreamSynchronize(stream);
    if (result == WD_OK && e != hipSuccess) result = hip_fail(e, "hipStreamSynchronize");
  }
  for (int k = 0; k < 2; ++k) {
    if (hs[k]) (void)hipHostFree(hs[k]);
    if (ev[k]) (void)hipEventDestroy(ev[k]);
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (result != WD_OK) {
    timer.release();
    return result;
  }
  if (timer.on) {
    const hipError_t e = timer.classify();
    if (e != hipSuccess) {
      timer.release();
      return hip_fail(e, "timing flags copy");
    }
  }
  const double hop_ms = timer.on ? timer.total_ms() : 0.0;
  double mms[4], mb[4], ims[4], ib[4];
  long long mn[4], in[4];
  timer.by_mode(mms, mn, mb);
  timer.by_mode(ims, in, ib, p.inner);
  wd_status worst = WD_OK;
  for (size_t q = 0; q < nst; ++q) {
    wd_status st = stats_from_state(fin[q], secs, &timer, stats[q]);
    stats[q].hop_ms = hop_ms;
    for (int m = 0; m < 4; ++m) {
      stats[q].hop_mode_ms[m] = mms[m];
      stats[q].hop_mode_launches[m] = mn[m];
      stats[q].hop_mode_bytes[m] = mb[m];
      stats[q].hop_inner_mode_ms[m] = ims[m];
      stats[q].hop_inner_mode_launches[m] = in[m];
      stats[q].hop_inner_mode_bytes[m] = ib[m];
    }
    if (worst == WD_OK && st != WD_OK) worst = st;
  }
  timer.release();
  if (worst == WD_ENONFINITE) set_error("non-finite value met in the solve");
  if (worst == WD_ENOTCONVERGED) set_error("solve did not reach the tolerance within maxiter");
  return worst;
}

}  // namespace wd
