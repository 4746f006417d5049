// Solving D x = b and D^dag x = b on top of the D^dag D solver, the pion
// contraction of point-source propagators, and the pseudofermion action,
// force and momentum update (C ABI).
//
// Even-odd (Schur complement; D = [[1, -k H_eo], [-k H_oe, 1]] in the
// (even, odd) blocks):
//   b'_e = b_e + k H_eo b_o
//   D_hat x_e = b'_e, solved as D_hat^dag D_hat x_e = D_hat^dag b'_e by CG
//   x_o = b_o + k H_oe x_e
// Full lattice: D^dag D x = D^dag b.  The adjoint system D^dag x = b is
// D (g5 x) = g5 b, since D^dag = g5 D g5.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "wd_host.h"

namespace wd {
namespace {

struct DLayout {
  size_t st_a, st_b;  // per-rhs coefficient states of the pre- and post-steps
  size_t B, T, Y;     // FP64 internal fields, two parity blocks each
  size_t BB;          // complex128 boundary fields: the normal-equation source
  size_t solver;      // workspace of the D^dag D solve
  size_t total;
  size_t vb;          // bytes of one FP64 parity block
};

DLayout d_layout(wd_lattice_s* lat, const wd_solve_params& p, int nrhs) {
  DLayout l;
  const size_t n = (size_t)lat->g.n;
  l.vb = vec_bytes(F64, n, nrhs);
  size_t o = 0;
  l.st_a = o;
  o += states_bytes((size_t)nrhs);
  l.st_b = o;
  o += states_bytes((size_t)nrhs);
  l.B = o;
  o += 2 * l.vb;
  l.T = o;
  o += 2 * l.vb;
  l.Y = o;
  o += 2 * l.vb;
  l.BB = o;
  o += align_up(2 * n * 12 * 16 * (size_t)nrhs);
  l.solver = o;
  o += wd_solver_workspace_bytes(lat, &p, nrhs);
  l.total = o;
  return l;
}

// One FP64 stencil launch over a single lattice with per-rhs coefficients
// st[r].c (no mask, no reduction).
wd_status hop64(wd_lattice_s* lat, int nrhs, int mode, int parity, const void* in, void* out, const void* aux,
                RhsState* st, int g5in, int g5out, size_t vb, hipStream_t s) {
  const int recon = lat->store[F64].recon;
  const Tune t = tune_lookup(lat, F64, recon, nrhs);
  Launch L = base_launch(nrhs, t, parity);
  L.nslots = 1;
  L.g5in = g5in;
  L.g5out = g5out;
  L.mask = MASK_NONE;
  L.fin = FIN_NONE;
  Slot& S = L.s[0];
  fill_slot_geometry(S, lat, t.sblk, parity);
  S.gauge = (const char*)lat->store[F64].ptr;
  S.in = in;
  S.out = out;
  S.aux = aux;
  S.vstride = vb;
  S.st = st;
  finish_launch(L);
  WD_HIP(launch_hop(L, F64, recon, mode, s));
  return WD_OK;
}

struct FLayout {
  size_t yb, xb;   // complex128 boundary fields Y = D^-dag eta, X = D^-1 Y
  size_t xi, yi;   // the same in the FP64 internal layout (two parity blocks each)
  size_t pion;     // time-slice sums of |Y|^2 for the action
  size_t solve;    // workspace of one wd_solve_D
  size_t total;
  size_t vb;
};

FLayout f_layout(wd_lattice_s* lat, const wd_solve_params& p) {
  FLayout l;
  const size_t n = (size_t)lat->g.n;
  l.vb = vec_bytes(F64, n, 1);
  const size_t field = align_up(2 * n * 12 * 16);
  size_t o = 0;
  l.yb = o;
  o += field;
  l.xb = o;
  o += field;
  l.xi = o;
  o += 2 * l.vb;
  l.yi = o;
  o += 2 * l.vb;
  l.pion = o;
  o += align_up(wd_pion_workspace_bytes(lat));
  l.solve = o;
  o += wd_solve_D_workspace_bytes(lat, &p, 1);
  l.total = o;
  return l;
}

}  // namespace
}  // namespace wd

using namespace wd;

extern "C" {

size_t wd_solve_D_workspace_bytes(wd_lattice lat, const wd_solve_params* params, int32_t nrhs) {
  if (!lat || !params || nrhs < 1) return 0;
  return d_layout(lat, *params, nrhs).total;
}

wd_status wd_solve_D(wd_lattice lat, void* x, const void* b, int32_t nrhs, const double* kappa, int32_t dagger,
                     const wd_solve_params* params, void* ws, size_t ws_bytes, wd_solve_stats* stats,
                     void* stream) {
  if (!lat || !x || !b || !kappa || !params || !ws || !stats) return fail(WD_EINVAL, "null argument");
  if (dagger != 0 && dagger != 1) return fail(WD_EINVAL, "dagger must be 0 or 1");
  wd_status s = check_params(*params);
  if (s != WD_OK) return s;
  if (nrhs < 1 || nrhs > kBlock / 2) return fail(WD_EINVAL, "nrhs = %d out of range [1, %d]", nrhs, kBlock / 2);
  if (!lat->store[F64].ptr) return fail(WD_ENOGAUGE, "the FP64 gauge store is needed");
  for (int r = 0; r < nrhs; ++r)
    if (!std::isfinite(kappa[r])) return fail(WD_EINVAL, "kappa[%d] not finite", r);
  const DLayout l = d_layout(lat, *params, nrhs);
  if (l.total == 0 || ws_bytes < l.total)
    return fail(WD_EBUFSIZE, "workspace holds %zu bytes, %zu needed", ws_bytes, l.total);
  const bool eo = params->precond == WD_EO;
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  char* B = w + l.B;
  char* T = w + l.T;
  char* Y = w + l.Y;
  void* BB = w + l.BB;
  RhsState* sa = (RhsState*)(w + l.st_a);
  RhsState* sb = (RhsState*)(w + l.st_b);
  const size_t vb = l.vb;
  const size_t ne = (size_t)lat->g.n * nrhs;
  const Geom& g = lat->g;

  // c = -kappa for the pre/post steps (aux - c H in = aux + kappa H in);
  // c = kappa^2 (EO) or kappa (full) for the adjoint operator.  The host
  // staging stays alive until the stream has drained (every path below ends
  // with a synchronisation).
  std::vector<RhsState> ha((size_t)nrhs), hb((size_t)nrhs);
  memset(ha.data(), 0, ha.size() * sizeof(RhsState));
  memset(hb.data(), 0, hb.size() * sizeof(RhsState));
  for (int r = 0; r < nrhs; ++r) {
    ha[r].c = -kappa[r];
    hb[r].c = eo ? kappa[r] * kappa[r] : kappa[r];
  }
  auto pre = [&]() -> wd_status {
    WD_HIP(hipMemcpyAsync(sa, ha.data(), nrhs * sizeof(RhsState), hipMemcpyHostToDevice, st));
    WD_HIP(hipMemcpyAsync(sb, hb.data(), nrhs * sizeof(RhsState), hipMemcpyHostToDevice, st));
    WD_HIP(launch_spinor_import(b, B, vb, g, nrhs, 2, F64, st));
    if (dagger) WD_HIP(launch_gamma5_f64(B, vb, ne, 2, st));
    wd_status e;
    if (eo) {
      // T_e = b_e + k H_eo b_o
      if ((e = hop64(lat, nrhs, HOP_XPAY, 0, B + vb, T, B, sa, 0, 0, vb, st)) != WD_OK) return e;
      // T_o = H_oe g5 T_e ; Y_e = T_e - k^2 g5 H_eo T_o = D_hat^dag T_e
      if ((e = hop64(lat, nrhs, HOP_PLAIN, 1, T, T + vb, nullptr, sa, 1, 0, vb, st)) != WD_OK) return e;
      if ((e = hop64(lat, nrhs, HOP_XPAY, 0, T + vb, Y, T, sb, 0, 1, vb, st)) != WD_OK) return e;
      WD_HIP(launch_spinor_export(Y, vb, BB, g, nrhs, 1, F64, st));
    } else {
      // Y = D^dag b = b - k g5 H g5 b
      if ((e = hop64(lat, nrhs, HOP_XPAY, 2, B, Y, B, sb, 1, 1, vb, st)) != WD_OK) return e;
      WD_HIP(launch_spinor_export(Y, vb, BB, g, nrhs, 2, F64, st));
    }
    return WD_OK;
  };
  auto post = [&]() -> wd_status {
    wd_status e;
    if (eo) {
      // x_o = b_o + k H_oe x_e
      WD_HIP(launch_spinor_import(x, Y, vb, g, nrhs, 1, F64, st));
      if ((e = hop64(lat, nrhs, HOP_XPAY, 1, Y, Y + vb, B + vb, sa, 0, 0, vb, st)) != WD_OK) return e;
      if (dagger) WD_HIP(launch_gamma5_f64(Y, vb, ne, 2, st));
      WD_HIP(launch_spinor_export(Y, vb, x, g, nrhs, 2, F64, st));
    } else if (dagger) {
      WD_HIP(launch_spinor_import(x, Y, vb, g, nrhs, 2, F64, st));
      WD_HIP(launch_gamma5_f64(Y, vb, ne, 2, st));
      WD_HIP(launch_spinor_export(Y, vb, x, g, nrhs, 2, F64, st));
    }
    WD_HIP(hipStreamSynchronize(st));
    return WD_OK;
  };
  if ((s = pre()) != WD_OK) {
    (void)hipStreamSynchronize(st);
    return s;
  }
  wd_solve_request rq;
  memset(&rq, 0, sizeof rq);
  rq.lat = lat;
  rq.x = x;
  rq.b = BB;
  rq.nrhs = nrhs;
  rq.kappa = kappa;
  const wd_status cg = wd_solve_batch(1, &rq, params, w + l.solver, l.total - l.solver, stats, stream);
  if (cg != WD_OK && cg != WD_ENOTCONVERGED && cg != WD_ENONFINITE) {
    (void)hipStreamSynchronize(st);
    return cg;
  }
  const std::string msg = wd_last_error();
  if ((s = post()) != WD_OK) {
    (void)hipStreamSynchronize(st);
    return s;
  }
  if (cg != WD_OK) set_error("%s", msg.c_str());
  return cg;
}

size_t wd_fermion_force_workspace_bytes(wd_lattice lat, const wd_solve_params* params) {
  if (!lat || !params) return 0;
  return f_layout(lat, *params).total;
}

wd_status wd_pseudofermion_heatbath(wd_lattice lat, void* eta, const void* xi, double kappa, void* ws,
                                    size_t ws_bytes, void* stream) {
  return wd_apply_D(lat, eta, xi, 1, kappa, 1, WD_FULL, WD_F64, ws, ws_bytes, stream);
}

wd_status wd_fermion_force(wd_lattice lat, void* F, double* action, const void* eta, double kappa,
                           const wd_solve_params* params, void* ws, size_t ws_bytes, wd_solve_stats* stats,
                           void* stream) {
  if (!lat || !eta || !params || !ws || !stats) return fail(WD_EINVAL, "null argument");
  if (!F && !action) return fail(WD_EINVAL, "neither the force nor the action requested");
  if (!std::isfinite(kappa)) return fail(WD_EINVAL, "kappa not finite");
  wd_status s = check_params(*params);
  if (s != WD_OK) return s;
  if (!lat->store[F64].ptr) return fail(WD_ENOGAUGE, "the FP64 gauge store is needed");
  const FLayout l = f_layout(lat, *params);
  if (ws_bytes < l.total) return fail(WD_EBUFSIZE, "workspace holds %zu bytes, %zu needed", ws_bytes, l.total);
  memset(stats, 0, 2 * sizeof(wd_solve_stats));
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  void* Yb = w + l.yb;
  void* Xb = w + l.xb;
  const Geom& g = lat->g;
  // Y = D^-dag eta: the action is ||Y||^2 = eta^dag (D^dag D)^{-1} eta
  s = wd_solve_D(lat, Yb, eta, 1, &kappa, 1, params, w + l.solve, l.total - l.solve, &stats[0], stream);
  if (s != WD_OK) return s;
  if (action) {
    const int Lt = lat->L[3];
    std::vector<double> slices((size_t)Lt);
    if ((s = wd_pion_correlator(lat, slices.data(), Yb, 1, 0, w + l.pion, l.solve - l.pion, stream)) != WD_OK)
      return s;
    double a = 0.0;
    for (int t = 0; t < Lt; ++t) a += slices[(size_t)t];
    *action = a;
  }
  if (!F) return WD_OK;
  // X = D^-1 Y = (D^dag D)^{-1} eta
  s = wd_solve_D(lat, Xb, Yb, 1, &kappa, 0, params, w + l.solve, l.total - l.solve, &stats[1], stream);
  if (s != WD_OK) return s;
  WD_HIP(launch_spinor_import(Xb, w + l.xi, l.vb, g, 1, 2, F64, st));
  WD_HIP(launch_spinor_import(Yb, w + l.yi, l.vb, g, 1, 2, F64, st));
  float bc[4];
  for (int mu = 0; mu < 4; ++mu) bc[mu] = (float)lat->bc[mu];
  WD_HIP(launch_force(w + l.xi, w + l.yi, l.vb, lat->store[F64].ptr, lat->store[F64].recon, g, bc, kappa, F, st));
  WD_HIP(hipStreamSynchronize(st));
  return WD_OK;
}

wd_status wd_ta_add(wd_lattice lat, void* p, double factor, const void* F, void* stream) {
  if (!lat || !p || !F) return fail(WD_EINVAL, "null argument");
  if (!std::isfinite(factor)) return fail(WD_EINVAL, "factor not finite");
  WD_HIP(launch_ta_add(p, F, factor, 8LL * lat->g.n, (hipStream_t)stream));
  return WD_OK;
}

size_t wd_pion_workspace_bytes(wd_lattice lat) {
  if (!lat) return 0;
  const int Lt = lat->L[3];
  return align_up((size_t)Lt * pion_shares(Lt) * sizeof(double)) + align_up((size_t)Lt * sizeof(double));
}

static wd_status pion_common(wd_lattice lat, double* corr, const void* S, int32_t nsrc, int32_t t0, int nc, void* ws,
                             size_t ws_bytes, void* stream) {
  if (!lat || !corr || !S || !ws) return fail(WD_EINVAL, "null argument");
  const int Lt = lat->L[3];
  if (nsrc < 1) return fail(WD_EINVAL, "nsrc = %d must be positive", nsrc);
  if (t0 < 0 || t0 >= Lt) return fail(WD_EINVAL, "t0 = %d outside [0, %d)", t0, Lt);
  const size_t need = wd_pion_workspace_bytes(lat);
  if (ws_bytes < need) return fail(WD_EBUFSIZE, "workspace holds %zu bytes, %zu needed", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  double* partial = (double*)ws;
  double* dcorr = (double*)((char*)ws + align_up((size_t)Lt * pion_shares(Lt) * sizeof(double)));
  WD_HIP(launch_pion(S, lat->g, nsrc, t0, nc, partial, dcorr, st));
  WD_HIP(hipMemcpyAsync(corr, dcorr, (size_t)Lt * sizeof(double), hipMemcpyDeviceToHost, st));
  WD_HIP(hipStreamSynchronize(st));
  return WD_OK;
}

wd_status wd_pion_correlator(wd_lattice lat, double* corr, const void* S, int32_t nsrc, int32_t t0, void* ws,
                             size_t ws_bytes, void* stream) {
  return pion_common(lat, corr, S, nsrc, t0, 12, ws, ws_bytes, stream);
}

wd_status wd_stag_pion_correlator(wd_lattice lat, double* corr, const void* S, int32_t nsrc, int32_t t0, void* ws,
                                  size_t ws_bytes, void* stream) {
  return pion_common(lat, corr, S, nsrc, t0, 3, ws, ws_bytes, stream);
}

}  // extern "C"
