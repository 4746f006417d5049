// C ABI of the staggered operator: apply D or D^dag, and solve D x = b (or
// D^dag x = b) through the even-odd decomposition
//   b'_e = m b_e - s H_eo b_o,   M_e x_e = b'_e  (CG, M_e = m^2 - H_eo H_oe),
//   x_o = (b_o - s H_oe x_e) / m,
// with s = +1 for D = m + H and s = -1 for D^dag = m - H.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "wd_host.h"

namespace wd {
namespace {

struct SLayout {
  size_t st_a, st_b;  // per-rhs coefficients of the pre- and post-steps
  size_t B, Y;        // FP64 internal fields, two parity blocks each
  size_t BB;          // complex128 boundary fields: the even-block source
  size_t items;       // engine workspace (states + items)
  size_t total;
  size_t vb;
};

int group_size(const wd_solve_params& p) { return p.rhs_group > 0 ? p.rhs_group : 4; }

size_t engine_bytes(wd_lattice_s* lat, const wd_solve_params& p, int nrhs) {
  size_t tot = states_bytes((size_t)nrhs);
  const int G = group_size(p);
  for (int r0 = 0; r0 < nrhs; r0 += G) tot += item_layout(lat, p, std::min(G, nrhs - r0), OP_STAG).total;
  return tot;
}

SLayout s_layout(wd_lattice_s* lat, const wd_solve_params& p, int nrhs) {
  SLayout l;
  const size_t n = (size_t)lat->g.n;
  l.vb = field_bytes(OP_STAG, F64, n, nrhs);
  size_t o = 0;
  l.st_a = o;
  o += states_bytes((size_t)nrhs);
  l.st_b = o;
  o += states_bytes((size_t)nrhs);
  l.B = o;
  o += 2 * l.vb;
  l.Y = o;
  o += 2 * l.vb;
  l.BB = o;
  o += align_up(2 * n * 3 * 16 * (size_t)nrhs);
  l.items = o;
  o += engine_bytes(lat, p, nrhs);
  l.total = o;
  return l;
}

wd_status stag64(wd_lattice_s* lat, int nrhs, int mode, int parity, const void* in, void* out, const void* aux,
                 RhsState* st, double coef, double coef2, size_t vb, hipStream_t s) {
  const int recon = lat->store[F64].recon;
  const Tune t = stag_tune_lookup(lat, F64, recon, nrhs);
  Launch L = base_launch(nrhs, t, parity);
  L.nslots = 1;
  L.mask = MASK_NONE;
  L.fin = FIN_NONE;
  L.coef = coef;
  L.coef2 = coef2;
  Slot& S = L.s[0];
  fill_slot_geometry(S, lat, t.sblk, parity);
  S.gauge = (const char*)lat->store[F64].ptr;
  S.in = in;
  S.out = out;
  S.aux = aux;
  S.vstride = vb;
  S.st = st;
  finish_launch(L);
  WD_HIP(launch_stag(L, F64, recon, mode, s));
  return WD_OK;
}

}  // namespace
}  // namespace wd

using namespace wd;

extern "C" {

size_t wd_stag_apply_workspace_bytes(wd_lattice lat, int32_t prec, int32_t nrhs) {
  if (!lat || (prec != F64 && prec != F32) || nrhs < 1) return 0;
  return 4 * field_bytes(OP_STAG, prec, (size_t)lat->g.n, nrhs);
}

wd_status wd_stag_apply(wd_lattice lat, void* y, const void* x, int32_t nrhs, double mass, int32_t dagger,
                        int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  if (!lat || !y || !x || !ws) return fail(WD_EINVAL, "null argument");
  if (prec != F64 && prec != F32) return fail(WD_EINVAL, "the staggered operator runs at FP64 or FP32");
  if (dagger != 0 && dagger != 1) return fail(WD_EINVAL, "dagger must be 0 or 1");
  if (nrhs < 1 || nrhs > kBlock / 2) return fail(WD_EINVAL, "nrhs = %d out of range [1, %d]", nrhs, kBlock / 2);
  if (!std::isfinite(mass)) return fail(WD_EINVAL, "mass not finite");
  if (!lat->store[prec].ptr) return fail(WD_ENOGAUGE, "no gauge store of precision %d registered", prec);
  const size_t need = wd_stag_apply_workspace_bytes(lat, prec, nrhs);
  if (ws_bytes < need) return fail(WD_EBUFSIZE, "workspace holds %zu bytes, %zu needed", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  const size_t vb = field_bytes(OP_STAG, prec, (size_t)lat->g.n, nrhs);
  char* vin = (char*)ws;
  char* vout = vin + 2 * vb;
  WD_HIP(launch_stag_import(x, vin, vb, lat->g, nrhs, 2, prec, st));
  const int recon = lat->store[prec].recon;
  const Tune t = stag_tune_lookup(lat, prec, recon, nrhs);
  Launch L = base_launch(nrhs, t, 2);
  L.nslots = 1;
  L.mask = MASK_NONE;
  L.fin = FIN_NONE;
  L.coef = mass;
  L.coef2 = dagger ? -1.0 : 1.0;
  Slot& S = L.s[0];
  fill_slot_geometry(S, lat, t.sblk, 2);
  S.gauge = (const char*)lat->store[prec].ptr;
  S.in = vin;
  S.out = vout;
  S.aux = vin;
  S.vstride = vb;
  finish_launch(L);
  WD_HIP(launch_stag(L, prec, recon, S_XPAY, st));
  WD_HIP(launch_stag_export(vout, vb, y, lat->g, nrhs, 2, prec, st));
  return WD_OK;
}

wd_status wd_stag_autotune(wd_lattice lat, int32_t prec, int32_t nrhs, void* ws, size_t ws_bytes,
                           int32_t* best_sites_per_block, int32_t* best_swizzle, int32_t* best_split,
                           void* stream) {
  if (!lat || !ws) return fail(WD_EINVAL, "null argument");
  if (prec != F64 && prec != F32) return fail(WD_EINVAL, "the staggered operator runs at FP64 or FP32");
  if (nrhs < 1 || nrhs > kBlock / 2) return fail(WD_EINVAL, "nrhs out of range");
  if (!lat->store[prec].ptr) return fail(WD_ENOGAUGE, "no gauge store of precision %d registered", prec);
  const size_t need = wd_stag_apply_workspace_bytes(lat, prec, nrhs);
  if (ws_bytes < need) return fail(WD_EBUFSIZE, "workspace holds %zu bytes, %zu needed", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  const size_t vb = field_bytes(OP_STAG, prec, (size_t)lat->g.n, nrhs);
  char* vin = (char*)ws;
  char* vout = vin + 2 * vb;
  // a deterministic input: the even block filled with a byte pattern of small values
  std::vector<unsigned char> pat(vb);
  for (size_t i = 0; i < vb; ++i) pat[i] = (unsigned char)((i * 2654435761u) >> 13) & 0x3f;
  WD_HIP(hipMemcpyAsync(vin, pat.data(), vb, hipMemcpyHostToDevice, st));
  WD_HIP(hipStreamSynchronize(st));
  const int recon = lat->store[prec].recon;
  std::vector<unsigned char> ref[5], got;
  std::vector<std::pair<Tune, double>> timed;
  hipEvent_t e0, e1;
  WD_HIP(hipEventCreate(&e0));
  WD_HIP(hipEventCreate(&e1));
  wd_status res = WD_OK;
  // blocks of 128 to 256 threads: below that the per-block fixed costs of the
  // CG kernels (the folded reductions) outweigh what the bare stencil gains;
  // split threads share the 8 hops of a site
  for (int split = 1; split <= 4 && res == WD_OK; split *= 2) {
    for (int sblk = 1; sblk <= kBlock && res == WD_OK; sblk *= 2) {
      const int threads = split * sblk * nrhs;
      if (threads < kBlock / 2 || threads > kBlock) continue;
      for (int swz = 0; swz <= 1 && res == WD_OK; ++swz) {
        const Tune tn{sblk, swz, split};
        Launch L = base_launch(nrhs, tn, 1);
        L.nslots = 1;
        L.mask = MASK_NONE;
        L.fin = FIN_NONE;
        Slot& S = L.s[0];
        fill_slot_geometry(S, lat, sblk, 1);
        S.gauge = (const char*)lat->store[prec].ptr;
        S.in = vin;
        S.out = vout;
        S.vstride = vb;
        finish_launch(L);
        hipError_t e = hipSuccess;
        for (int i = 0; i < 2 && e == hipSuccess; ++i) e = launch_stag(L, prec, recon, S_PLAIN, st);
        // the best of 3 timings of 20 launches (shapes differ by a few percent)
        float ms = 1e30f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
          e = hipEventRecord(e0, st);
          for (int i = 0; i < 20 && e == hipSuccess; ++i) e = launch_stag(L, prec, recon, S_PLAIN, st);
          if (e == hipSuccess) e = hipEventRecord(e1, st);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float m1 = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&m1, e0, e1);
          ms = std::min(ms, m1 / 20.0f);  // per launch
        }
        // within one split the sums do not depend on the tiling: every shape
        // must produce the same bytes
        std::vector<unsigned char>& dst = ref[split].empty() ? ref[split] : got;
        dst.resize(vb);
        if (e == hipSuccess) e = hipMemcpy(dst.data(), vout, vb, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
          res = hip_fail(e, "staggered autotune launch");
          break;
        }
        if (&dst == &got && got != ref[split]) {
          res = fail(WD_EDEVICE, "staggered stencil output differs between launch shapes (sblk %d swz %d split %d)",
                     sblk, swz, split);
          break;
        }
        timed.push_back({tn, (double)ms});
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (res != WD_OK) return res;
  const Tune bt = pick_shape(timed, lat->g.n, nrhs, 2, (double)vb, stag_tune_lookup(lat, prec, recon, nrhs));
  stag_tune_store(lat, prec, recon, nrhs, bt);
  if (best_sites_per_block) *best_sites_per_block = bt.sblk;
  if (best_swizzle) *best_swizzle = bt.swz;
  if (best_split) *best_split = bt.split;
  return WD_OK;
}

wd_status wd_stag_set_shape(wd_lattice lat, int32_t prec, int32_t nrhs, int32_t sites_per_block, int32_t swizzle,
                            int32_t split) {
  if (!lat) return fail(WD_EINVAL, "null lattice");
  if (prec != F64 && prec != F32) return fail(WD_EINVAL, "the staggered operator runs at FP64 or FP32");
  if (nrhs < 1 || nrhs > kBlock / 2) return fail(WD_EINVAL, "nrhs out of range");
  if (!lat->store[prec].ptr) return fail(WD_ENOGAUGE, "no gauge store of precision %d registered", prec);
  if (split != 1 && split != 2 && split != 4) return fail(WD_EINVAL, "split = %d must be 1, 2 or 4", split);
  if (swizzle != 0 && swizzle != 1) return fail(WD_EINVAL, "swizzle must be 0 or 1");
  if (sites_per_block < 1 || (sites_per_block & (sites_per_block - 1)) != 0)
    return fail(WD_EINVAL, "sites_per_block = %d must be a power of two", sites_per_block);
  if ((long long)split * sites_per_block * nrhs > kBlock)
    return fail(WD_EINVAL, "split * sites_per_block * nrhs = %lld exceeds %d threads",
                (long long)split * sites_per_block * nrhs, kBlock);
  stag_tune_store(lat, prec, lat->store[prec].recon, nrhs, Tune{sites_per_block, swizzle, split});
  return WD_OK;
}

size_t wd_stag_solve_workspace_bytes(wd_lattice lat, const wd_solve_params* params, int32_t nrhs) {
  if (!lat || !params || nrhs < 1) return 0;
  return s_layout(lat, *params, nrhs).total;
}

wd_status wd_stag_solve(wd_lattice lat, void* x, const void* b, int32_t nrhs, const double* mass, int32_t dagger,
                        const wd_solve_params* params, void* ws, size_t ws_bytes, wd_solve_stats* stats,
                        void* stream) {
  if (!lat || !x || !b || !mass || !params || !ws || !stats) return fail(WD_EINVAL, "null argument");
  if (dagger != 0 && dagger != 1) return fail(WD_EINVAL, "dagger must be 0 or 1");
  wd_status s = check_params(*params);
  if (s != WD_OK) return s;
  if (params->precond != WD_EO) return fail(WD_EINVAL, "the staggered solve is even-odd only");
  if (params->inner != F64 && params->inner != F32) return fail(WD_EINVAL, "the staggered solve runs at FP64 or FP32");
  if (nrhs < 1 || nrhs > kBlock / 2) return fail(WD_EINVAL, "nrhs = %d out of range [1, %d]", nrhs, kBlock / 2);
  if (!lat->store[F64].ptr) return fail(WD_ENOGAUGE, "the FP64 gauge store is needed");
  if (!lat->store[params->inner].ptr) return fail(WD_ENOGAUGE, "no gauge store of the inner precision");
  if (params->recon != 0 && lat->store[params->inner].recon != params->recon)
    return fail(WD_ENOGAUGE, "inner gauge store has recon %d, %d requested", lat->store[params->inner].recon,
                params->recon);
  for (int r = 0; r < nrhs; ++r)
    if (!std::isfinite(mass[r]) || mass[r] == 0.0) return fail(WD_EINVAL, "mass[%d] must be finite and nonzero", r);
  const SLayout l = s_layout(lat, *params, nrhs);
  if (ws_bytes < l.total) return fail(WD_EBUFSIZE, "workspace holds %zu bytes, %zu needed", ws_bytes, l.total);
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  char* B = w + l.B;
  char* Y = w + l.Y;
  void* BB = w + l.BB;
  RhsState* sa = (RhsState*)(w + l.st_a);
  RhsState* sb = (RhsState*)(w + l.st_b);
  const size_t vb = l.vb;
  const Geom& g = lat->g;
  const double sg = dagger ? -1.0 : 1.0;
  // pre-step: out = m b_e - s H_eo b_o  (c = m, alpha = -s)
  // post-step: out = (1/m) b_o - (s/m) H_oe x_e  (c = 1/m, alpha = -s/m)
  // The host staging stays alive until the stream has drained.
  std::vector<RhsState> ha((size_t)nrhs), hb((size_t)nrhs);
  memset(ha.data(), 0, ha.size() * sizeof(RhsState));
  memset(hb.data(), 0, hb.size() * sizeof(RhsState));
  for (int r = 0; r < nrhs; ++r) {
    ha[r].c = mass[r];
    ha[r].alpha = -sg;
    hb[r].c = 1.0 / mass[r];
    hb[r].alpha = -sg / mass[r];
  }
  auto pre = [&]() -> wd_status {
    WD_HIP(hipMemcpyAsync(sa, ha.data(), nrhs * sizeof(RhsState), hipMemcpyHostToDevice, st));
    WD_HIP(hipMemcpyAsync(sb, hb.data(), nrhs * sizeof(RhsState), hipMemcpyHostToDevice, st));
    WD_HIP(launch_stag_import(b, B, vb, g, nrhs, 2, F64, st));
    wd_status e = stag64(lat, nrhs, S_XPAY, 0, B + vb, Y, B, sa, 0.0, 0.0, vb, st);
    if (e != WD_OK) return e;
    WD_HIP(launch_stag_export(Y, vb, BB, g, nrhs, 1, F64, st));
    return WD_OK;
  };
  if ((s = pre()) != WD_OK) {
    (void)hipStreamSynchronize(st);
    return s;
  }
  // the engine: one item per group of rhs, CG on M_e
  char* iw = w + l.items;
  RhsState* states = (RhsState*)iw;
  size_t off = states_bytes((size_t)nrhs);
  const int G = group_size(*params);
  const size_t field = (size_t)2 * g.n * 3 * 16;
  std::vector<EItem> items;
  int si = 0;
  for (int r0 = 0; r0 < nrhs; r0 += G) {
    EItem it;
    it.lat = lat;
    it.x = (char*)x + r0 * field;
    it.b = (const char*)BB + r0 * field;
    it.nrhs = std::min(G, nrhs - r0);
    it.kappa.assign(mass + r0, mass + r0 + it.nrhs);
    it.lay = item_layout(lat, *params, it.nrhs, OP_STAG);
    it.base = iw + off;
    off += it.lay.total;
    it.st = states + si;
    it.state_index = si;
    si += it.nrhs;
    items.push_back(it);
  }
  const wd_status cg = run_batch(items, *params, states, st, stats, OP_STAG);
  if (cg != WD_OK && cg != WD_ENOTCONVERGED && cg != WD_ENONFINITE) {
    (void)hipStreamSynchronize(st);
    return cg;
  }
  const std::string msg = wd_last_error();
  auto post = [&]() -> wd_status {
    WD_HIP(launch_stag_import(x, Y, vb, g, nrhs, 1, F64, st));
    wd_status e = stag64(lat, nrhs, S_XPAY, 1, Y, Y + vb, B + vb, sb, 0.0, 0.0, vb, st);
    if (e != WD_OK) return e;
    WD_HIP(launch_stag_export(Y, vb, x, g, nrhs, 2, F64, st));
    WD_HIP(hipStreamSynchronize(st));
    return WD_OK;
  };
  if ((s = post()) != WD_OK) {
    (void)hipStreamSynchronize(st);
    return s;
  }
  if (cg != WD_OK) set_error("%s", msg.c_str());
  return cg;
}

}  // extern "C"
