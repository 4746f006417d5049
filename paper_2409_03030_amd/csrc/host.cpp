// Host driver and C ABI of the Wilson-Dirac library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "wd_host.h"

namespace wd {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

wd_status fail(wd_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

wd_status hip_fail(hipError_t e, const char* what) {
  return fail(WD_EDEVICE, "%s failed: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// sizes
// ---------------------------------------------------------------------------
size_t vec_bytes(int prec, size_t n, int nrhs) {
  const size_t ne = n * (size_t)nrhs;
  switch (prec) {
    case F64: return align_up(SpinorFmt<F64>::bytes(ne));
    case F32: return align_up(SpinorFmt<F32>::bytes(ne));
    case F16: return align_up(SpinorFmt<F16>::bytes(ne));
  }
  return 0;
}

size_t gauge_bytes(const Geom& g, int prec, int recon) {
  const size_t n = (size_t)g.n;
  size_t dir = 0;
  if (recon != 18 && recon != 12) return 0;
  if (prec == F64) dir = recon == 18 ? link_dir_bytes<F64, 18>(n) : link_dir_bytes<F64, 12>(n);
  else if (prec == F32) dir = recon == 18 ? link_dir_bytes<F32, 18>(n) : link_dir_bytes<F32, 12>(n);
  else if (prec == F16) dir = recon == 18 ? link_dir_bytes<F16, 18>(n) : link_dir_bytes<F16, 12>(n);
  else return 0;
  return 8 * dir;
}

// ---------------------------------------------------------------------------
// tuning table
// ---------------------------------------------------------------------------
using TuneKey = std::tuple<int, int, int, int, int, int, int>;
static std::mutex g_tune_mu;
static std::map<TuneKey, Tune> g_tune;

static TuneKey tkey(const wd_lattice_s* lat, int prec, int recon, int nrhs) {
  return TuneKey(lat->L[0], lat->L[1], lat->L[2], lat->L[3], prec, recon, nrhs);
}

int default_sblk(int nrhs) {
  int s = 1;
  while (s * 2 * nrhs <= kBlock) s *= 2;
  if (nrhs == 1) s = 128;
  return s;
}

// A block holds split * sblk * nrhs threads (at most kBlock, or kMaxBlock for
// the 8-way split, which exists below FP64 only); a part of the split covers
// whole waves; the reduction needs at least one full wave.
bool valid_tune(const Tune& t, int nrhs, int prec) {
  if (t.split == 8 && prec == F64) return false;
  const int sb = t.sblk;
  if (sb < 1 || (sb & (sb - 1)) != 0) return false;
  if (t.split != 1 && t.split != 2 && t.split != 4 && t.split != 8) return false;
  if (t.swz < 0 || t.swz > 2) return false;
  const int per = sb * nrhs;
  if (per < 64 || t.split * per > (t.split == 8 ? kMaxBlock : kBlock)) return false;
  if (t.split > 1 && per % 64 != 0) return false;
  return true;
}

Tune tune_lookup(const wd_lattice_s* lat, int prec, int recon, int nrhs) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(tkey(lat, prec, recon, nrhs));
  if (it != g_tune.end()) return it->second;
  return Tune{default_sblk(nrhs), 1, 1};
}

void tune_store(const wd_lattice_s* lat, int prec, int recon, int nrhs, Tune t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[tkey(lat, prec, recon, nrhs)] = t;
}

// Staggered stencil shapes (one thread per site and rhs), filled by
// wd_stag_autotune; without an entry the Wilson entry's block shape is used.
static std::map<TuneKey, Tune> g_stag_tune;

Tune stag_tune_lookup(const wd_lattice_s* lat, int prec, int recon, int nrhs) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_stag_tune.find(tkey(lat, prec, recon, nrhs));
    if (it != g_stag_tune.end()) return it->second;
  }
  Tune t = tune_lookup(lat, prec, recon, nrhs);
  t.split = 1;
  return t;
}

void stag_tune_store(const wd_lattice_s* lat, int prec, int recon, int nrhs, Tune t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_stag_tune[tkey(lat, prec, recon, nrhs)] = t;
}

// ---------------------------------------------------------------------------
// launch assembly
// ---------------------------------------------------------------------------
void fill_slot_geometry(Slot& S, const wd_lattice_s* lat, int sblk, int parity) {
  S.g = lat->g;
  for (int mu = 0; mu < 4; ++mu) S.bc[mu] = (float)lat->bc[mu];
  const int nbp = (lat->g.n + sblk - 1) / sblk;
  S.nblk = parity == 2 ? 2 * nbp : nbp;
  S.npart = S.nblk;
}

void finish_launch(Launch& L) {
  int b = 0;
  for (int i = 0; i < L.nslots; ++i) {
    L.s[i].blk0 = b;
    b += L.s[i].nblk;
  }
  L.total_blocks = b;
  // Right-hand-side groups of one lattice (slots with the same geometry, links
  // and block count) take interleaved block order (Launch::ilv): measured, the
  // 36-source solve at 16^3x32 (9 groups of 4 in launches of 8 and 1 slots)
  // went from 214 to 193 ms; the 12-source solves did not change.
  L.ilv = 0;
  if (L.nslots > 1) {
    bool same = true;
    for (int i = 1; i < L.nslots; ++i) {
      const Slot& a = L.s[0];
      const Slot& c = L.s[i];
      same = same && c.nblk == a.nblk && c.gauge == a.gauge && c.g.n == a.g.n && c.g.hx == a.g.hx &&
             c.g.L[1] == a.g.L[1] && c.g.L[2] == a.g.L[2] && c.g.L[3] == a.g.L[3];
    }
    L.ilv = same ? 1 : 0;
  }
  // t-slice order: one slot, or interleaved groups, whose logical blocks of a
  // t-slice are the slice's blocks of every group
  L.bt = 0;
  if (L.swz == 2 && (L.nslots == 1 || L.ilv) && L.parity != 2) {
    const Geom& g = L.s[0].g;
    const int per_slice = g.n / g.L[3];  // sites of one parity in a t-slice
    if (per_slice % L.sblk == 0) L.bt = per_slice / L.sblk * L.nslots;
  }
  // the t-slices of an XCD's range, for ranges of q and q + 1 blocks
  const int q = L.total_blocks >> 3;
  for (int hi = 0; hi < 2; ++hi) {
    const int cnt = q + hi, S = L.bt > 0 ? cnt / L.bt : 0;
    L.tsS[hi] = S >= 2 && S * L.bt == cnt ? S : 0;
    L.dts[hi] = make_fastdiv(L.tsS[hi]);
  }
  L.dpart = make_fastdiv(L.sblk * L.nrhs);
  L.drhs = make_fastdiv(L.nrhs);
  L.dslots = make_fastdiv(L.nslots);
}

Launch base_launch(int nrhs, const Tune& t, int parity) {
  Launch L;
  memset(&L, 0, sizeof L);
  L.nrhs = nrhs;
  L.sblk = t.sblk;
  L.swz = t.swz;
  L.split = t.split;
  L.parity = parity;
  // the divisors of a one-slot launch; finish_launch sets them for the final shape
  L.dpart = make_fastdiv(L.sblk * L.nrhs);
  L.drhs = make_fastdiv(L.nrhs);
  L.dslots = make_fastdiv(1);
  L.dts[0] = L.dts[1] = make_fastdiv(1);
  return L;
}

// ---------------------------------------------------------------------------
// timing
// ---------------------------------------------------------------------------
hipError_t HopTimer::begin(hipStream_t s) {
  if (!on) return hipSuccess;
  if (used + 2 > ev.size()) {
    for (int i = 0; i < 256; ++i) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      ev.push_back(e);
    }
  }
  return hipEventRecord(ev[used], s);
}

hipError_t HopTimer::end(hipStream_t s, long long sites, double b, int m) {
  if (!on) return hipSuccess;
  hipError_t r = hipEventRecord(ev[used + 1], s);
  used += 2;
  mode.push_back(m);
  mode_bytes.push_back(b);
  mode_sites.push_back(sites);
  return r;
}

hipError_t HopTimer::classify() {
  const size_t nl = std::min(used / 2, mode.size());
  dur.assign(nl, -1.f);
  skipped.assign(nl, 0);
  for (size_t i = 0; i < nl; ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) == hipSuccess) dur[i] = t;
  }
  if (flags) {
    std::vector<int> f(std::min(nl, (size_t)kTimingFlags));
    if (!f.empty()) {
      const hipError_t e = hipMemcpy(f.data(), flags, f.size() * sizeof(int), hipMemcpyDeviceToHost);
      if (e != hipSuccess) return e;
    }
    for (size_t i = 0; i < f.size(); ++i) skipped[i] = f[i] == 0;
  }
  site_updates = 0;
  bytes = 0.0;
  nskipped = 0;
  for (size_t i = 0; i < nl; ++i) {
    if (dur[i] < 0.f) continue;
    if (skipped[i]) {
      ++nskipped;
      continue;
    }
    site_updates += mode_sites[i];
    bytes += mode_bytes[i];
  }
  return hipSuccess;
}

void HopTimer::by_mode(double ms[4], long long n[4], double b[4], int prec) {
  for (int m = 0; m < 4; ++m) {
    ms[m] = 0.0;
    n[m] = 0;
    b[m] = 0.0;
  }
  for (size_t i = 0; i < dur.size(); ++i) {
    if (dur[i] < 0.f || skipped[i]) continue;
    const int m = mode[i] & 3;
    if (prec >= 0 && (mode[i] >> 2) != prec) continue;
    ms[m] += dur[i];
    n[m] += 1;
    b[m] += mode_bytes[i];
  }
}

double hop_launch_bytes(int prec, int recon, int mode, long long sites, int nrhs) {
  const double link = (prec == F64 ? 16.0 : prec == F32 ? 8.0 : 4.0) * (recon == 12 ? 6 : 9);
  const double sp = prec == F64 ? 192.0 : prec == F32 ? 96.0 : 52.0;  // F16: 48 B data + 4 B scale
  const int A = acc_prec(prec);
  const double sa = A == F64 ? 192.0 : 96.0;
  double vec = 0.0;
  switch (mode) {
    case HOP_PLAIN: vec = 2 * sp; break;                  // in, out
    case HOP_XPAY: vec = 3 * sp; break;                   // in, aux, out
    case HOP_CGR: vec = 2 * sp + 2 * sa; break;           // in, aux, r read + write
    case HOP_RESID: vec = 2 * sp + 2 * 192.0; break;      // in, aux, b, r_h
  }
  const double site_sets = (double)sites / nrhs;           // sites counts site x rhs
  return site_sets * 8 * link + (double)sites * vec;
}

double stag_launch_bytes(int prec, int recon, int mode, long long sites, int nrhs) {
  const double link = (prec == F64 ? 16.0 : 8.0) * (recon == 12 ? 6 : 9);
  const double sv = prec == F64 ? 48.0 : 24.0;
  double vec = 0.0;
  switch (mode) {
    case S_PLAIN: vec = 2 * sv; break;               // in, out
    case S_XPAY: case S_NORM: vec = 3 * sv; break;   // in, aux, out
    case S_CGR: vec = 4 * sv; break;                 // in, aux, r read + write
    case S_RESID: vec = 2 * sv + 2 * 48.0; break;    // in, aux, b, r_h
  }
  return (double)sites / nrhs * 8 * link + (double)sites * vec;
}

double HopTimer::total_ms() {
  double t = 0.0;
  for (size_t i = 0; i < dur.size(); ++i)
    if (dur[i] >= 0.f && !skipped[i]) t += dur[i];
  return t;
}

void HopTimer::release() {
  for (auto e : ev) (void)hipEventDestroy(e);
  ev.clear();
  mode.clear();
  mode_bytes.clear();
  mode_sites.clear();
  dur.clear();
  skipped.clear();
  used = 0;
}

// ---------------------------------------------------------------------------
// argument checks
// ---------------------------------------------------------------------------
wd_status check_params(const wd_solve_params& p) {
  if (!(p.tol > 0.0) || !std::isfinite(p.tol)) return fail(WD_EINVAL, "tol must be positive and finite");
  if (p.maxiter <= 0) return fail(WD_EINVAL, "maxiter must be positive");
  if (p.inner < F64 || p.inner > F16) return fail(WD_EINVAL, "inner precision %d unknown", p.inner);
  if (p.recon != 0 && p.recon != 12 && p.recon != 18) return fail(WD_EINVAL, "recon must be 0, 12 or 18");
  if (!(p.delta >= 0.0 && p.delta < 1.0)) return fail(WD_EINVAL, "delta must be in [0, 1)");
  if (p.precond != WD_FULL && p.precond != WD_EO) return fail(WD_EINVAL, "precond %d unknown", p.precond);
  if (p.poll_every < 0 || p.poll_every > 4096) return fail(WD_EINVAL, "poll_every out of range");
  if (p.rhs_group < 0 || p.rhs_group > kBlock / 2) return fail(WD_EINVAL, "rhs_group out of range");
  return WD_OK;
}

wd_status check_lattice_for(const wd_lattice_s* lat, int prec, int precond) {
  if (!lat) return fail(WD_EINVAL, "null lattice");
  if (prec < F64 || prec > F16) return fail(WD_EINVAL, "precision %d unknown", prec);
  if (precond != WD_FULL && precond != WD_EO) return fail(WD_EINVAL, "precond %d unknown", precond);
  if (!lat->store[prec].ptr) return fail(WD_ENOGAUGE, "no gauge store of precision %d registered", prec);
  return WD_OK;
}

// Measured at 16^3x32, FP32: 256-thread blocks gave the same stencil time as
// 128-thread blocks (10.3 against 10.4 us inside the solve) but a 3 % faster
// solve (11.0 against 11.4 ms) with half the partials; the staggered FP32
// stencil's fastest shape (1024 blocks of 4 threads per site) lost both folds
// and made its solve 25 % slower.  Between equal block counts the XCD-aware
// order wins: with it every kernel of the CG (whatever its block size) gives
// each XCD the same contiguous eighth of the sites, so a vector written by
// one kernel is read from the same L2 by the next (staggered FP32 solve 5.6
// against 5.9 ms, FP16-inner Wilson solve 10.1 against 10.5 ms, with bare
// stencil times within noise of each other).
// The swz = 2 order differs from swz = 1 only when the blocks of a parity
// split over the 8 XCDs into ranges of at least two whole t-slices.
bool tslice_order_applies(const Geom& g, int sblk) {
  const int per_slice = g.n / g.L[3];
  if (per_slice % sblk) return false;
  const int bt = per_slice / sblk, nb = (g.n + sblk - 1) / sblk;
  if (nb % 8) return false;
  const int q = nb / 8;
  return q % bt == 0 && q / bt >= 2;
}

Tune pick_shape(const std::vector<std::pair<Tune, double>>& timed_all, long long n, int nrhs, int per_iter,
                double vec_bytes, Tune fallback) {
  constexpr double kTuneSlack = 1.03;
  // For each (sblk, split) one candidate goes on: the faster of the XCD-aware
  // orders (swz 1 and 2, which give every XCD the same range of sites), kept
  // unless it is more than swz_slack slower than the plain order in the bare
  // stencil.  The bare stencil times one kernel alone and so misses the
  // cross-kernel L2 reuse of the XCD-aware orders; that reuse needs a vector to
  // fit in half of the XCDs' L2s (8 x 4 MB), otherwise only a tie goes to them.
  const double swz_slack = vec_bytes <= 16.0e6 ? 1.10 : 1.0;
  std::vector<std::pair<Tune, double>> timed;
  for (const auto& c : timed_all) {
    bool first = true;  // first candidate of its (sblk, split) in the list
    for (const auto& d : timed_all) {
      if (&d == &c) break;
      if (d.first.sblk == c.first.sblk && d.first.split == c.first.split) first = false;
    }
    if (!first) continue;
    const std::pair<Tune, double>* plain = nullptr;
    const std::pair<Tune, double>* xcd = nullptr;
    for (const auto& d : timed_all) {
      if (d.first.sblk != c.first.sblk || d.first.split != c.first.split) continue;
      if (d.first.swz == 0) plain = &d;
      else if (!xcd || d.second < xcd->second) xcd = &d;
    }
    if (!xcd) timed.push_back(*plain);
    else if (!plain) timed.push_back(*xcd);
    else if (xcd->second <= swz_slack * plain->second) timed.push_back({xcd->first, std::min(xcd->second, plain->second)});
    else timed.push_back(*plain);
  }
  auto blocks_of = [&](const Tune& t) { return (n + t.sblk - 1) / t.sblk; };
  auto folds = [&](const Tune& t) {
    const long long b = blocks_of(t), parts = b * nrhs;
    return parts <= kFoldPartials && b * parts <= kFoldReads;
  };
  // cost of a CG iteration: its per_iter stencil launches, plus a finalize
  // kernel (about 5 us) for each of the two reductions that cannot be folded
  auto cost = [&](const std::pair<Tune, double>& c) {
    return per_iter * c.second + (folds(c.first) ? 0.0 : 2 * 0.005);
  };
  double best = 1e30;
  for (const auto& c : timed) best = std::min(best, cost(c));
  Tune bt = fallback;
  long long bt_blocks = -1;
  double bt_cost = 1e30;
  for (const auto& c : timed) {
    const double cc = cost(c);
    if (cc > kTuneSlack * best) continue;
    const long long b = blocks_of(c.first);
    const bool cx = c.first.swz != 0, bx = bt.swz != 0;
    const bool better = bt_blocks < 0 || b < bt_blocks || (b == bt_blocks && (cx > bx || (cx == bx && cc < bt_cost)));
    if (better) {
      bt = c.first;
      bt_blocks = b;
      bt_cost = cc;
    }
  }
  return bt;
}

// First item of each wave (kWaveBytes): one wave unless a single request's
// groups exceed the budget and at least two of its largest groups fit in it.
static std::vector<size_t> wave_starts(const std::vector<EItem>& items, int32_t nreq) {
  std::vector<size_t> w{0};
  if (nreq != 1 || items.size() < 2) return w;
  auto inner = [](const EItem& it) { return it.lay.total - it.lay.off_x; };
  size_t tot = 0, big = 0;
  for (const EItem& it : items) {
    tot += inner(it);
    big = std::max(big, inner(it));
  }
  if (tot <= kWaveBytes || 2 * big > kWaveBytes) return w;
  size_t acc = 0;
  for (size_t k = 0; k < items.size(); ++k) {
    if (acc > 0 && acc + inner(items[k]) > kWaveBytes) {
      w.push_back(k);
      acc = 0;
    }
    acc += inner(items[k]);
  }
  return w;
}

}  // namespace wd

using namespace wd;

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* wd_version(void) { return "wdirac 0.1 (gfx950)"; }

const char* wd_last_error(void) { return g_last_error.c_str(); }

const char* wd_status_string(wd_status s) {
  switch (s) {
    case WD_OK: return "ok";
    case WD_EINVAL: return "invalid argument";
    case WD_EBUFSIZE: return "buffer too small";
    case WD_ENOGAUGE: return "no gauge field of that precision";
    case WD_ENOTCONVERGED: return "not converged";
    case WD_ENONFINITE: return "non-finite value";
    case WD_EDEVICE: return "device error";
    case WD_EBUSY: return "busy";
    case WD_ENOTFOUND: return "not found";
  }
  return "unknown status";
}

wd_status wd_lattice_create(wd_lattice* out, const int32_t L[4], const int32_t bc[4]) {
  if (!out || !L || !bc) return fail(WD_EINVAL, "null argument");
  *out = nullptr;
  long long V = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (L[mu] < 2 || (L[mu] & 1)) return fail(WD_EINVAL, "extent L[%d] = %d must be even and >= 2", mu, L[mu]);
    if (bc[mu] != 1 && bc[mu] != -1) return fail(WD_EINVAL, "bc[%d] = %d must be +1 or -1", mu, bc[mu]);
    V *= L[mu];
  }
  if (V > (1LL << 30)) return fail(WD_EINVAL, "lattice volume %lld too large", V);
  wd_lattice_s* lat = new wd_lattice_s();
  for (int mu = 0; mu < 4; ++mu) {
    lat->L[mu] = L[mu];
    lat->bc[mu] = bc[mu];
    lat->g.L[mu] = L[mu];
  }
  lat->g.hx = L[0] / 2;
  lat->g.n = (int)(V / 2);
  set_divisors(lat->g);
  *out = lat;
  return WD_OK;
}

wd_status wd_lattice_destroy(wd_lattice lat) {
  delete lat;
  return WD_OK;
}

size_t wd_gauge_bytes(wd_lattice lat, int32_t prec, int32_t recon) {
  if (!lat) return 0;
  return gauge_bytes(lat->g, prec, recon);
}

wd_status wd_set_gauge(wd_lattice lat, const void* U, void* store, size_t store_bytes, int32_t prec, int32_t recon,
                       void* stream) {
  if (!lat || !U || !store) return fail(WD_EINVAL, "null argument");
  if (prec < F64 || prec > F16) return fail(WD_EINVAL, "precision %d unknown", prec);
  if (recon != 18 && recon != 12) return fail(WD_EINVAL, "recon must be 18 or 12");
  const size_t need = gauge_bytes(lat->g, prec, recon);
  if (store_bytes < need) return fail(WD_EBUFSIZE, "gauge store holds %zu bytes, %zu needed", store_bytes, need);
  WD_HIP(launch_gauge_import(U, store, lat->g, prec, recon, (hipStream_t)stream));
  lat->store[prec].ptr = store;
  lat->store[prec].recon = recon;
  return WD_OK;
}

// Four full-lattice vectors, then (for the timing calls) a scratch solver
// state and block partials.
static size_t timing_tail_bytes(const wd_lattice_s* lat, int nrhs) {
  const size_t n = (size_t)lat->g.n;
  return align_up((size_t)nrhs * sizeof(RhsState)) +
         align_up(((n + min_sblk(nrhs) - 1) / min_sblk(nrhs)) * nrhs * sizeof(double));
}

size_t wd_apply_workspace_bytes(wd_lattice lat, int32_t prec, int32_t nrhs) {
  if (!lat || prec < F64 || prec > F16 || nrhs < 1) return 0;
  return 4 * 2 * vec_bytes(prec, (size_t)lat->g.n, nrhs) + timing_tail_bytes(lat, nrhs);
}

static wd_status apply_common(wd_lattice lat, void* y, const void* x, int32_t nrhs, double kappa, int32_t precond,
                              int32_t prec, void* ws, size_t ws_bytes, void* stream, bool normal, int dagger) {
  wd_status s = check_lattice_for(lat, prec, precond);
  if (s != WD_OK) return s;
  if (!y || !x || !ws) return fail(WD_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > kBlock / 2) return fail(WD_EINVAL, "nrhs = %d out of range [1, %d]", nrhs, kBlock / 2);
  if (!std::isfinite(kappa)) return fail(WD_EINVAL, "kappa not finite");
  const size_t need = wd_apply_workspace_bytes(lat, prec, nrhs);
  if (ws_bytes < need) return fail(WD_EBUFSIZE, "workspace holds %zu bytes, %zu needed", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  const size_t vb = vec_bytes(prec, (size_t)lat->g.n, nrhs);
  char* w = (char*)ws;
  char* vin = w;
  char* vt = w + 2 * vb;
  char* vout = w + 4 * vb;
  char* vout2 = w + 6 * vb;
  const int recon = lat->store[prec].recon;
  const Tune t = tune_lookup(lat, prec, recon, nrhs);
  const bool eo = precond == WD_EO;
  auto hop = [&](int mode, int parity, const void* in, void* out, const void* aux, double coef, int g5in,
                 int g5out) -> wd_status {
    Launch L = base_launch(nrhs, t, parity);
    L.nslots = 1;
    L.g5in = g5in;
    L.g5out = g5out;
    L.mask = MASK_NONE;
    L.fin = FIN_NONE;
    L.coef = coef;
    Slot& S = L.s[0];
    fill_slot_geometry(S, lat, t.sblk, parity);
    S.gauge = (const char*)lat->store[prec].ptr;
    S.in = in;
    S.out = out;
    S.aux = aux;
    S.vstride = vb;
    finish_launch(L);
    WD_HIP(launch_hop(L, prec, recon, mode, st));
    return WD_OK;
  };
  WD_HIP(launch_spinor_import(x, vin, vb, lat->g, nrhs, eo ? 1 : 2, prec, st));
  // first operator: D (or D^dag)
  const int d1 = normal ? 0 : dagger;
  if (eo) {
    if ((s = hop(HOP_PLAIN, 1, vin, vt, nullptr, 0.0, d1, 0)) != WD_OK) return s;
    if ((s = hop(HOP_XPAY, 0, vt, vout, vin, kappa * kappa, 0, d1)) != WD_OK) return s;
  } else {
    if ((s = hop(HOP_XPAY, 2, vin, vout, vin, kappa, d1, d1)) != WD_OK) return s;
  }
  char* res = vout;
  if (normal) {  // then D^dag = g5 D g5
    if (eo) {
      if ((s = hop(HOP_PLAIN, 1, vout, vt, nullptr, 0.0, 1, 0)) != WD_OK) return s;
      if ((s = hop(HOP_XPAY, 0, vt, vout2, vout, kappa * kappa, 0, 1)) != WD_OK) return s;
    } else {
      if ((s = hop(HOP_XPAY, 2, vout, vout2, vout, kappa, 1, 1)) != WD_OK) return s;
    }
    res = vout2;
  }
  WD_HIP(launch_spinor_export(res, vb, y, lat->g, nrhs, eo ? 1 : 2, prec, st));
  return WD_OK;
}

wd_status wd_apply_D(wd_lattice lat, void* y, const void* x, int32_t nrhs, double kappa, int32_t dagger,
                     int32_t precond, int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  if (dagger != 0 && dagger != 1) return fail(WD_EINVAL, "dagger must be 0 or 1");
  return apply_common(lat, y, x, nrhs, kappa, precond, prec, ws, ws_bytes, stream, false, dagger);
}

wd_status wd_apply_DdagD(wd_lattice lat, void* y, const void* x, int32_t nrhs, double kappa, int32_t precond,
                         int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  return apply_common(lat, y, x, nrhs, kappa, precond, prec, ws, ws_bytes, stream, true, 0);
}

// The allocation-free variant of wd_apply_D takes its workspace from this
// file-scope array instead of a caller buffer.  In host code the array's name
// is only a stand-in for the symbol: each device holds its own copy, whose
// address hipGetSymbolAddress returns with that device current; only that
// address ever reaches a kernel.  Every call on one device shares its copy.
static __device__ __align__(256) unsigned char scratch[WD_NOALLOC_SCRATCH_BYTES];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];  // per device: the address of its copy of scratch

// Device address of the current device's scratch array, looked up on the
// first call on that device.
static wd_status scratch_address(void** out) {
  int dev = -1;
  WD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(WD_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(WD_EDEVICE, "hipGetSymbolAddress(scratch) gave a null address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return WD_OK;
}

wd_status wd_apply_D_noalloc(wd_lattice lat, void* y, const void* x, int32_t nrhs, double kappa, int32_t dagger,
                             int32_t precond, int32_t prec, void* stream) {
  if (dagger != 0 && dagger != 1) return fail(WD_EINVAL, "dagger must be 0 or 1");
  wd_status s = check_lattice_for(lat, prec, precond);
  if (s != WD_OK) return s;
  if (nrhs < 1 || nrhs > kBlock / 2) return fail(WD_EINVAL, "nrhs = %d out of range [1, %d]", nrhs, kBlock / 2);
  const size_t need = wd_apply_workspace_bytes(lat, prec, nrhs);
  if (need > (size_t)WD_NOALLOC_SCRATCH_BYTES)
    return fail(WD_EBUFSIZE, "the call needs %zu bytes of scratch; the allocation-free call holds %zu", need,
                (size_t)WD_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  if ((s = scratch_address(&ws)) != WD_OK) return s;
  return apply_common(lat, y, x, nrhs, kappa, precond, prec, ws, (size_t)WD_NOALLOC_SCRATCH_BYTES, stream, false,
                      dagger);
}

void wd_solve_params_default(wd_solve_params* p) {
  if (!p) return;
  memset(p, 0, sizeof *p);
  p->tol = 1e-10;
  p->maxiter = 100000;
  p->inner = WD_F64;
  p->recon = 0;
  p->delta = 0.0;
  p->precond = WD_EO;
  p->poll_every = 0;
  p->use_graph = 1;
  p->timing = 0;
  p->rhs_group = 0;
}

static wd_status check_item(wd_lattice lat, const wd_solve_params& p) {
  if (!lat) return fail(WD_EINVAL, "null lattice");
  if (!lat->store[F64].ptr) return fail(WD_ENOGAUGE, "the FP64 gauge store is needed for the true residual");
  if (!lat->store[p.inner].ptr) return fail(WD_ENOGAUGE, "no gauge store of the inner precision %d", p.inner);
  if (p.recon != 0 && lat->store[p.inner].recon != p.recon)
    return fail(WD_ENOGAUGE, "inner gauge store has recon %d, %d requested", lat->store[p.inner].recon, p.recon);
  return WD_OK;
}

size_t wd_solver_workspace_bytes(wd_lattice lat, const wd_solve_params* params, int32_t nrhs) {
  if (!lat || !params || nrhs < 1) return 0;
  wd_solve_request r;
  memset(&r, 0, sizeof r);
  r.lat = lat;
  r.nrhs = nrhs;
  return wd_batch_workspace_bytes(1, &r, params);
}

// Groups of consecutive rhs of one request: (request, first rhs, count).
struct RhsGroup {
  int req, r0, n;
};
static std::vector<RhsGroup> rhs_groups(int32_t nreq, const wd_solve_request* reqs, const wd_solve_params& p) {
  const int G = p.rhs_group > 0 ? p.rhs_group : 4;
  std::vector<RhsGroup> out;
  for (int i = 0; i < nreq; ++i)
    for (int r0 = 0; r0 < reqs[i].nrhs; r0 += G) out.push_back({i, r0, std::min(G, reqs[i].nrhs - r0)});
  return out;
}

size_t wd_batch_workspace_bytes(int32_t nreq, const wd_solve_request* reqs, const wd_solve_params* params) {
  if (nreq < 1 || !reqs || !params) return 0;
  size_t nst = 0, tot = 0;
  for (int i = 0; i < nreq; ++i) {
    if (!reqs[i].lat || reqs[i].nrhs < 1) return 0;
    nst += (size_t)reqs[i].nrhs;
  }
  for (const RhsGroup& g : rhs_groups(nreq, reqs, *params)) tot += item_layout(reqs[g.req].lat, *params, g.n).total;
  return states_bytes(nst) + tot;
}

wd_status wd_solve_batch(int32_t nreq, const wd_solve_request* reqs, const wd_solve_params* params, void* ws,
                         size_t ws_bytes, wd_solve_stats* stats, void* stream) {
  if (nreq < 1 || !reqs || !params || !ws || !stats) return fail(WD_EINVAL, "null argument or empty batch");
  wd_status s = check_params(*params);
  if (s != WD_OK) return s;
  for (int i = 0; i < nreq; ++i) {
    const int nrhs = reqs[i].nrhs;
    if (nrhs < 1 || nrhs > kBlock / 2) return fail(WD_EINVAL, "request %d: nrhs = %d out of range [1, %d]", i, nrhs, kBlock / 2);
    if (!reqs[i].x || !reqs[i].b || !reqs[i].kappa) return fail(WD_EINVAL, "request %d has a null pointer", i);
    if ((s = check_item(reqs[i].lat, *params)) != WD_OK) return s;
    for (int r = 0; r < nrhs; ++r)
      if (!std::isfinite(reqs[i].kappa[r])) return fail(WD_EINVAL, "request %d: kappa[%d] not finite", i, r);
  }
  const size_t need = wd_batch_workspace_bytes(nreq, reqs, params);
  if (ws_bytes < need) return fail(WD_EBUFSIZE, "workspace holds %zu bytes, %zu needed", ws_bytes, need);
  size_t nst = 0;
  for (int i = 0; i < nreq; ++i) nst += (size_t)reqs[i].nrhs;
  char* w = (char*)ws;
  RhsState* states = (RhsState*)w;
  size_t off = states_bytes(nst);
  int si = 0;
  const std::vector<RhsGroup> groups = rhs_groups(nreq, reqs, *params);
  std::vector<EItem> items(groups.size());
  for (size_t k = 0; k < groups.size(); ++k) {
    const RhsGroup& gr = groups[k];
    const wd_solve_request& rq = reqs[gr.req];
    // field r of a request starts at r * V * 12 complex128 values
    const size_t field = (size_t)2 * rq.lat->g.n * 12 * 16;
    EItem& it = items[k];
    it.lat = rq.lat;
    it.x = (char*)rq.x + gr.r0 * field;
    it.b = (const char*)rq.b + gr.r0 * field;
    it.nrhs = gr.n;
    it.kappa.assign(rq.kappa + gr.r0, rq.kappa + gr.r0 + gr.n);
    it.lay = item_layout(it.lat, *params, it.nrhs);
    it.base = w + off;
    off += it.lay.total;
    it.st = states + si;
    it.state_index = si;
    si += it.nrhs;
  }
  const std::vector<size_t> waves = wave_starts(items, nreq);
  if (waves.size() == 1) return run_batch(items, *params, states, (hipStream_t)stream, stats);
  // consecutive waves: each solves its groups to the end (states and stats of
  // a wave are the contiguous entries of its rhs)
  wd_status worst = WD_OK;
  for (size_t k = 0; k < waves.size(); ++k) {
    const size_t a = waves[k], e = k + 1 < waves.size() ? waves[k + 1] : items.size();
    std::vector<EItem> sub(items.begin() + (long)a, items.begin() + (long)e);
    const int s0 = items[a].state_index;
    const wd_status r = run_batch(sub, *params, states + s0, (hipStream_t)stream, stats + s0);
    if (r != WD_OK && r != WD_ENOTCONVERGED && r != WD_ENONFINITE) return r;
    if (worst == WD_OK) worst = r;
  }
  if (worst == WD_ENONFINITE) set_error("non-finite value met in the solve");
  if (worst == WD_ENOTCONVERGED) set_error("solve did not reach the tolerance within maxiter");
  return worst;
}

wd_status wd_solve_DdagD(wd_lattice lat, void* x, const void* b, int32_t nrhs, const double* kappa,
                         const wd_solve_params* params, void* ws, size_t ws_bytes, wd_solve_stats* stats,
                         void* stream) {
  wd_solve_request r;
  memset(&r, 0, sizeof r);
  r.lat = lat;
  r.x = x;
  r.b = b;
  r.nrhs = nrhs;
  r.kappa = kappa;
  if (!lat) return fail(WD_EINVAL, "null lattice");
  return wd_solve_batch(1, &r, params, ws, ws_bytes, stats, stream);
}

// ---------------------------------------------------------------------------
// measurement and tuning
// ---------------------------------------------------------------------------
// Mode of wd_time_hop: the four stencil launches of one CG iteration in order.
constexpr int kTimeCgStencils = 4;

static wd_status time_hop_shape(wd_lattice lat, int prec, int nrhs, int mode, int n, const Tune& t, char* ws,
                                double* ms, hipStream_t st) {
  const size_t vb = vec_bytes(prec, (size_t)lat->g.n, nrhs);
  const int recon = lat->store[prec].recon;
  char* tail = ws + 8 * vb;
  // Workspace blocks of both parities: 0 at ws, 1 at ws + 2 vb, 2 at ws + 4 vb,
  // the residual at ws + 6 vb; solver states and partials after them.
  auto make = [&](int m, int parity, const char* in, char* out, const char* aux, int g5in, int g5out) {
    Launch L = base_launch(nrhs, t, parity);
    L.nslots = 1;
    L.g5in = g5in;
    L.g5out = g5out;
    Slot& S = L.s[0];
    fill_slot_geometry(S, lat, t.sblk, L.parity);
    S.gauge = (const char*)lat->store[prec].ptr;
    S.in = in;
    S.out = out;
    S.aux = aux;
    S.r = ws + 6 * vb;
    S.vstride = vb;
    S.astride = vec_bytes(acc_prec(prec), (size_t)lat->g.n, nrhs);
    if (m != HOP_PLAIN) {
      L.fin = m == HOP_XPAY ? FIN_ALPHA : FIN_CG;
      L.mask = MASK_NONE;
      S.st = (RhsState*)tail;
      S.partial = (double*)(tail + align_up((size_t)nrhs * sizeof(RhsState)));
    }
    finish_launch(L);
    return L;
  };
  std::vector<std::pair<Launch, int>> seq;
  if (mode == kTimeCgStencils) {
    // t1 = H_oe p; t2 = p - c H_eo t1 with |t2|^2; t3 = H_oe g5 t2;
    // r -= alpha (t2 - c g5 H_eo t3) with |r|^2 (p, t2, r even; t1, t3 odd)
    seq.push_back({make(HOP_PLAIN, 1, ws, ws + 2 * vb, nullptr, 0, 0), HOP_PLAIN});
    seq.push_back({make(HOP_XPAY, 0, ws + 2 * vb, ws + 4 * vb, ws, 0, 0), HOP_XPAY});
    seq.push_back({make(HOP_PLAIN, 1, ws + 4 * vb, ws + 2 * vb, nullptr, 1, 0), HOP_PLAIN});
    seq.push_back({make(HOP_CGR, 0, ws + 2 * vb, ws + 4 * vb, ws + 4 * vb, 0, 1), HOP_CGR});
  } else {
    seq.push_back({make(mode, mode == HOP_PLAIN ? 1 : 0, ws, ws + 2 * vb, ws + 4 * vb, 0, 0), mode});
  }
  auto run = [&]() {
    hipError_t e = hipSuccess;
    for (size_t k = 0; k < seq.size() && e == hipSuccess; ++k) e = launch_hop(seq[k].first, prec, recon, seq[k].second, st);
    return e;
  };
  hipEvent_t e0, e1;
  WD_HIP(hipEventCreate(&e0));
  WD_HIP(hipEventCreate(&e1));
  wd_status res = WD_OK;
  hipError_t e = hipSuccess;
  for (int i = 0; i < 3 && e == hipSuccess; ++i) e = run();
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int i = 0; i < n && e == hipSuccess; ++i) e = run();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float f = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
  if (e != hipSuccess) res = hip_fail(e, "timed stencil launches");
  else *ms = (double)f / n;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return res;
}

wd_status wd_time_hop(wd_lattice lat, int32_t prec, int32_t nrhs, int32_t mode, int32_t n, void* ws, size_t ws_bytes,
                      double* ms_per_launch, void* stream) {
  wd_status s = check_lattice_for(lat, prec, WD_EO);
  if (s != WD_OK) return s;
  if (!ws || !ms_per_launch || n < 1) return fail(WD_EINVAL, "bad argument");
  if (mode != HOP_PLAIN && mode != HOP_XPAY && mode != HOP_CGR && mode != kTimeCgStencils)
    return fail(WD_EINVAL, "mode %d not timed (0, 1, 2 or 4)", mode);
  if (nrhs < 1 || nrhs > kBlock / 2) return fail(WD_EINVAL, "nrhs out of range");
  const size_t need = wd_apply_workspace_bytes(lat, prec, nrhs);
  if (ws_bytes < need) return fail(WD_EBUFSIZE, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  // zeroed scratch: finite inputs, zero solver state (alpha = c = 0)
  WD_HIP(hipMemsetAsync(ws, 0, need, st));
  const Tune t = tune_lookup(lat, prec, lat->store[prec].recon, nrhs);
  return time_hop_shape(lat, prec, nrhs, mode, n, t, (char*)ws, ms_per_launch, st);
}

wd_status wd_time_read(const void* buf, size_t bytes, int32_t n, void* out, size_t out_bytes, double* ms_per_read,
                       void* stream) {
  if (!buf || !out || !ms_per_read || n < 1) return fail(WD_EINVAL, "bad argument");
  if (bytes < 16 || bytes % 16) return fail(WD_EINVAL, "bytes must be a positive multiple of 16");
  const int blocks = 2048;
  if (out_bytes < blocks * sizeof(double)) return fail(WD_EBUFSIZE, "out holds %zu bytes, %zu needed", out_bytes,
                                                        blocks * sizeof(double));
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  WD_HIP(hipEventCreate(&e0));
  WD_HIP(hipEventCreate(&e1));
  hipError_t e = hipSuccess;
  for (int i = 0; i < 3 && e == hipSuccess; ++i) e = launch_read_probe(buf, bytes, (double*)out, blocks, st);
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int i = 0; i < n && e == hipSuccess; ++i) e = launch_read_probe(buf, bytes, (double*)out, blocks, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float f = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "timed reads");
  *ms_per_read = (double)f / n;
  return WD_OK;
}

wd_status wd_autotune(wd_lattice lat, int32_t prec, int32_t nrhs, void* ws, size_t ws_bytes,
                      int32_t* best_sites_per_block, int32_t* best_swizzle, int32_t* best_split, void* stream) {
  wd_status s = check_lattice_for(lat, prec, WD_EO);
  if (s != WD_OK) return s;
  if (!ws) return fail(WD_EINVAL, "null workspace");
  if (nrhs < 1 || nrhs > kBlock / 2) return fail(WD_EINVAL, "nrhs out of range");
  if (ws_bytes < wd_apply_workspace_bytes(lat, prec, nrhs)) return fail(WD_EBUFSIZE, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  const size_t vb = vec_bytes(prec, (size_t)lat->g.n, nrhs);
  char* w = (char*)ws;
  // a deterministic input: the workspace's input block filled with a pattern
  std::vector<unsigned char> pat(vb);
  for (size_t i = 0; i < vb; ++i) pat[i] = (unsigned char)((i * 2654435761u) >> 13) & 0x3f;
  WD_HIP(hipMemcpyAsync(w, pat.data(), vb, hipMemcpyHostToDevice, st));
  // the rest zeroed: finite epilogue operands and solver states (alpha = c = 0)
  // for the timed CG-residual launches
  WD_HIP(hipMemsetAsync(w + vb, 0, wd_apply_workspace_bytes(lat, prec, nrhs) - vb, st));
  WD_HIP(hipStreamSynchronize(st));
  std::vector<unsigned char> ref[9], got;
  std::vector<std::pair<Tune, double>> timed;
  for (int split = 1; split <= 8; split *= 2) {
    for (int sblk = 1; sblk <= kMaxBlock; sblk *= 2) {
      for (int swz = 0; swz <= 2; ++swz) {
        Tune t{sblk, swz, split};
        if (!valid_tune(t, nrhs, prec)) continue;
        // the t-slice order exists only where the XCD ranges are whole t-slices
        if (swz == 2 && !tslice_order_applies(lat->g, sblk)) continue;
        WD_HIP(hipMemsetAsync(w + 2 * vb, 0, vb, st));
        // one plain hop for the output check below
        double m1 = 0.0;
        if ((s = time_hop_shape(lat, prec, nrhs, HOP_PLAIN, 1, t, w, &m1, st)) != WD_OK) return s;
        // within one split the per-site arithmetic does not depend on the tiling:
        // every shape must produce the same bytes
        got.resize(vb);
        WD_HIP(hipMemcpy(got.data(), w + 2 * vb, vb, hipMemcpyDeviceToHost));
        if (ref[split].empty()) ref[split] = got;
        else if (memcmp(ref[split].data(), got.data(), vb) != 0)
          return fail(WD_EDEVICE, "tuning candidate sblk=%d swz=%d split=%d changed the stencil output", sblk, swz,
                      split);
        // Timed: the four stencil launches of one CG iteration in order (two
        // plain hops and the two epilogue stencils, as the solve runs them),
        // the best of 3 timings of 5 iterations: the shapes of a small lattice
        // differ by a few percent, about the run-to-run spread of one timing.
        double mq = 1e30;
        for (int rep = 0; rep < 3; ++rep) {
          if ((s = time_hop_shape(lat, prec, nrhs, kTimeCgStencils, 5, t, w, &m1, st)) != WD_OK) return s;
          mq = std::min(mq, m1);
        }
        timed.push_back({t, 0.25 * mq});  // per launch
      }
    }
  }
  const Tune bt = pick_shape(timed, lat->g.n, nrhs, 4, (double)vb, Tune{default_sblk(nrhs), 1, 1});
  tune_store(lat, prec, lat->store[prec].recon, nrhs, bt);
  if (best_sites_per_block) *best_sites_per_block = bt.sblk;
  if (best_swizzle) *best_swizzle = bt.swz;
  if (best_split) *best_split = bt.split;
  return WD_OK;
}

size_t wd_tune_export(char* buf, size_t cap) {
  std::ostringstream os;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& kv : g_tune) {
      const TuneKey& k = kv.first;
      os << std::get<0>(k) << ' ' << std::get<1>(k) << ' ' << std::get<2>(k) << ' ' << std::get<3>(k) << ' '
         << std::get<4>(k) << ' ' << std::get<5>(k) << ' ' << std::get<6>(k) << ' ' << kv.second.sblk << ' '
         << kv.second.swz << ' ' << kv.second.split << '\n';
    }
  }
  const std::string s = os.str();
  if (buf && cap > 0) {
    const size_t m = std::min(cap - 1, s.size());
    memcpy(buf, s.data(), m);
    buf[m] = 0;
  }
  return s.size() + 1;
}

wd_status wd_tune_import(const char* text) {
  if (!text) return fail(WD_EINVAL, "null text");
  std::istringstream is(text);
  std::string line;
  std::vector<std::pair<TuneKey, Tune>> rows;
  while (std::getline(is, line)) {
    if (line.empty()) continue;
    std::istringstream ls(line);
    int v[10];
    for (int i = 0; i < 10; ++i)
      if (!(ls >> v[i])) return fail(WD_EINVAL, "malformed tuning line '%s'", line.c_str());
    const Tune t{v[7], v[8], v[9]};
    if (!valid_tune(t, v[6], v[4])) return fail(WD_EINVAL, "invalid tuning values in '%s'", line.c_str());
    rows.push_back({TuneKey(v[0], v[1], v[2], v[3], v[4], v[5], v[6]), t});
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& r : rows) g_tune[r.first] = r.second;
  return WD_OK;
}

}  // extern "C"
