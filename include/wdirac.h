/*
 * wdirac.h -- C ABI of the MI355X (gfx950) Wilson-Dirac library.
 *
 * The calls follow the paper's statement of the fermion problem (App. C,
 * "Definition of Dirac operators"): build an operator from a gauge field and
 * a hopping parameter kappa, apply D (``mul!(y,D,x)``), its adjoint (``D'``)
 * or the normal operator D^dag D (``DdagD_operator``), and solve
 * D^dag D x = b iteratively to a tolerance (``solve_DinvX!`` with
 * ``eps_CG``).  Output arguments come first, as in the paper's mutating calls.
 *
 * Operator (the paper cites Wilson's formulation without printing it; the
 * library fixes the textbook hopping-parameter form, r = 1):
 *
 *   (D psi)(x) = psi(x) - kappa * sum_mu [ (1 - g_mu) U_mu(x) s+ psi(x+mu)
 *                                        + (1 + g_mu) U_mu(x-mu)^dag s- psi(x-mu) ]
 *
 * with the Euclidean chiral gamma basis g_k = [[0,-i sigma_k],[i sigma_k,0]],
 * g_4 = [[0,1],[1,0]], g_5 = diag(1,1,-1,-1), and s+/s- = bc[mu] for a hop
 * that crosses the lattice boundary in direction mu (else 1).
 * Even-odd mode (WD_EO) works with the Schur complement on the even sites,
 * D_hat = 1 - kappa^2 H_eo H_oe (D = 1 - kappa H); parity of a site is
 * (x+y+z+t) mod 2.
 *
 * Data at the boundary (all device pointers, complex128 = two doubles re,im):
 *   spinor field : [t][z][y][x][spin 4][colour 3]; colour fastest, matching
 *                  the paper's element x[ic,ix,iy,iz,it,ialpha] (App. C,
 *                  "Definition of pseudo-fermion fields").  nrhs fields are
 *                  stored back to back: [rhs][t][z][y][x][4][3].
 *   gauge field  : [mu = x,y,z,t][t][z][y][x][row 3][col 3] (the paper's
 *                  U[mu], App. B).  Boundary signs are NOT folded in.
 *   In WD_EO mode the odd sites of an input are ignored and the odd sites of
 *   an output are written as zero.
 *
 * Memory ownership: the library never allocates device memory.  The caller
 * allocates gauge stores and workspaces (size queries below) and keeps them
 * alive while in use; the library keeps no pointer to x, y or b after a call
 * returns.  A gauge store registered with wd_set_gauge must outlive every
 * call that uses that precision on the lattice.
 *
 * Streams: ``stream`` is a hipStream_t (0 = the null stream).  apply calls
 * are asynchronous on it; solve calls block the host until the solve ends.
 *
 * Errors: every call returns a wd_status; on error a thread-local message is
 * available from wd_last_error().  Arguments are checked before any work is
 * queued: on error nothing has been launched.
 *
 * Thread safety: calls on different lattices are independent; calls on one
 * lattice must be serialised by the caller.
 */
#ifndef WDIRAC_H
#define WDIRAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t wd_status;
enum {
  WD_OK = 0,
  WD_EINVAL = -1,         /* bad argument (shape, precision, null pointer, odd extent in EO) */
  WD_EBUFSIZE = -2,       /* caller buffer smaller than the size query requires */
  WD_ENOGAUGE = -3,       /* no gauge store of the requested precision registered */
  WD_ENOTCONVERGED = -4,  /* maxiter reached; x holds the last iterate, stats are filled */
  WD_ENONFINITE = -5,     /* NaN/Inf met in the source or during the iteration */
  WD_EDEVICE = -6,        /* a HIP runtime call failed */
  WD_EBUSY = -7,          /* server: request not admitted (no slot or memory) */
  WD_ENOTFOUND = -8       /* server: unknown ticket */
};

typedef enum { WD_F64 = 0, WD_F32 = 1, WD_F16 = 2 } wd_prec;
typedef enum { WD_FULL = 0, WD_EO = 1 } wd_precond;

typedef struct wd_lattice_s* wd_lattice;

/* Solver parameters (the paper's params dict: kappa, eps_CG, verbose). */
typedef struct {
  double tol;          /* stop when ||b - A x|| / ||b|| <= tol, true residual in FP64 */
  int32_t maxiter;     /* iteration cap (inner iterations) */
  int32_t inner;       /* wd_prec of the inner CG: F64 = plain FP64 CG, F32/F16 = mixed */
  int32_t recon;       /* 0: use the inner precision's gauge store whatever its recon; 18 or 12: that
                          store must hold this recon (else WD_ENOGAUGE).  Requests of a batch or
                          server may mix recons: launches are split by the recon of each store read */
  double delta;        /* reliable update when ||r|| < delta * max ||r|| since the last one;
                          0 = only at convergence (plain CG) */
  int32_t precond;     /* wd_precond */
  int32_t poll_every;  /* iterations between host convergence polls; 0 = automatic */
  int32_t use_graph;   /* 1: replay captured hipGraphs of poll_every iterations */
  int32_t timing;      /* 1: time every stencil launch with hipEvents (disables graphs) */
  int32_t rhs_group;   /* a request with more rhs is solved as consecutive groups of at most this
                          many rhs, each its own slot of the same launches (smaller per-site working
                          set in the L2); 0 = automatic (4) */
} wd_solve_params;

/* Per right-hand side result. */
typedef struct {
  int32_t status;            /* WD_OK, WD_ENOTCONVERGED or WD_ENONFINITE for this rhs */
  int32_t iters;             /* inner CG iterations */
  int32_t reliable_updates;  /* FP64 true-residual recomputations */
  int32_t hop_skipped;       /* with timing=1: stencil launches left out of the hop_* figures below
                                because every slot skipped its work (masked after convergence, or a
                                reliable-update sequence with nothing held), as the kernels flag it in
                                a ring of 65536 flags per device (a 256 KiB device array of the library;
                                timed solves running on one GPU at once share it, and their counts are
                                then unreliable; launches beyond the ring are counted as working) */
  double true_resid;         /* last FP64 true relative residual */
  double iter_resid;         /* last iterated relative residual */
  double seconds;            /* wall time of the whole solve call */
  double hop_ms;             /* with timing=1: summed duration of the stencil launches that worked */
  int64_t hop_launches;      /* with timing=1: number of those launches */
  int64_t hop_site_updates;  /* stencil output sites x rhs processed by those launches */
  double hop_bytes;          /* algorithmic bytes of those launches: each launch reads its 8 links per
                                output site once (shared by the rhs), its input spinor once per site and
                                rhs, and reads/writes its epilogue vectors once */
  /* the same three figures split by stencil epilogue: [0] plain H, [1] aux - c H
     (with |.|^2), [2] CG residual update r -= alpha (aux - c g5 H), [3] FP64 true residual */
  double hop_mode_ms[4];
  int64_t hop_mode_launches[4];
  double hop_mode_bytes[4];
  /* the same split, counting only the stencil launches at the inner precision (for a mixed solve:
     without the FP64 launches of the reliable updates) */
  double hop_inner_mode_ms[4];
  int64_t hop_inner_mode_launches[4];
  double hop_inner_mode_bytes[4];
} wd_solve_stats;

/* ---- lattice ---------------------------------------------------------- */

/* L = {Lx, Ly, Lz, Lt}, each >= 2 and even (needed for the even-odd split and
 * the checkerboard index); bc = per-direction boundary sign, +1 periodic or
 * -1 antiperiodic.  Host-only; allocates a small host object. */
wd_status wd_lattice_create(wd_lattice* out, const int32_t L[4], const int32_t bc[4]);
wd_status wd_lattice_destroy(wd_lattice lat);

/* Bytes of a gauge store of precision prec with recon = 18 (full 3x3) or 12
 * (two rows; the third is rebuilt as the conjugate cross product of the first
 * two, exact for SU(3)).  0 on bad arguments. */
size_t wd_gauge_bytes(wd_lattice lat, int32_t prec, int32_t recon);

/* Convert the complex128 gauge field U (device, boundary layout) into the
 * caller-owned device store (wd_gauge_bytes bytes) and register it as the
 * lattice's links of precision prec.  One store per precision; calling again
 * replaces the registration.  Asynchronous on stream. */
wd_status wd_set_gauge(wd_lattice lat, const void* U, void* store, size_t store_bytes,
                       int32_t prec, int32_t recon, void* stream);

/* ---- operator application -------------------------------------------- */

/* Workspace bytes needed by wd_apply_D / wd_apply_DdagD at precision prec. */
size_t wd_apply_workspace_bytes(wd_lattice lat, int32_t prec, int32_t nrhs);

/* y = D x (dagger = 0) or y = D^dag x (dagger = 1) for nrhs fields; in WD_EO
 * mode D_hat (resp. D_hat^dag) on the even sites.  The arithmetic runs in
 * precision prec with that precision's registered gauge store; x and y stay
 * complex128.  Asynchronous on stream. */
wd_status wd_apply_D(wd_lattice lat, void* y, const void* x, int32_t nrhs, double kappa,
                     int32_t dagger, int32_t precond, int32_t prec,
                     void* ws, size_t ws_bytes, void* stream);

/* y = D^dag D x (WD_FULL) or y = D_hat^dag D_hat x (WD_EO).  Asynchronous. */
wd_status wd_apply_DdagD(wd_lattice lat, void* y, const void* x, int32_t nrhs, double kappa,
                         int32_t precond, int32_t prec,
                         void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): wd_apply_D without
 * the workspace argument.  Its workspace is a file-scope device array of
 * WD_NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds until the
 * process ends; the call allocates nothing.  Calls that need more than that
 * (wd_apply_workspace_bytes(lat, prec, nrhs) > WD_NOALLOC_SCRATCH_BYTES; at
 * nrhs = 1 FP64 fits up to about 87000 sites, e.g. 16^3x16 or 12^3x24, FP32
 * and FP16 up to about 174000, e.g. 16^3x32) return WD_EBUFSIZE.  Nothing in
 * the array needs to start at zero: each call writes every part it reads.
 * All calls on one GPU share that GPU's array, so calls that overlap on one
 * GPU (other streams or host threads) race; order them on one stream.  The
 * first call on a device looks up the array's address there.  Otherwise as
 * wd_apply_D: asynchronous on stream, x and y complex128 device fields. */
#define WD_NOALLOC_SCRATCH_BYTES (64u << 20)
wd_status wd_apply_D_noalloc(wd_lattice lat, void* y, const void* x, int32_t nrhs, double kappa,
                             int32_t dagger, int32_t precond, int32_t prec, void* stream);

/* ---- solver ------------------------------------------------------------ */

/* Workspace bytes for wd_solve_DdagD with these parameters and nrhs fields. */
size_t wd_solver_workspace_bytes(wd_lattice lat, const wd_solve_params* params, int32_t nrhs);

/* Fill *params with defaults: tol 1e-10, maxiter 100000, inner F64, recon 0 (any),
 * delta 0, WD_EO, automatic polling, graphs on, timing off, automatic rhs groups. */
void wd_solve_params_default(wd_solve_params* params);

/* Solve D^dag D x = b (WD_FULL) or D_hat^dag D_hat x_e = b_e (WD_EO) for nrhs
 * right-hand sides at once; kappa[r] is the hopping parameter of rhs r.
 * CG from x0 = 0; inner arithmetic in params->inner with FP64 reliable
 * updates (x_h += x_l, r_h = b - A x_h recomputed with the FP64 store, FP64
 * norms).  Needs the FP64 gauge store, and the inner precision's store when
 * inner != F64.  stats has nrhs entries (host).  Blocks the host.  Returns
 * WD_OK when every rhs converged, else the first failing rhs status.  Many
 * rhs may run as consecutive waves (wd_solve_batch). */
wd_status wd_solve_DdagD(wd_lattice lat, void* x, const void* b, int32_t nrhs, const double* kappa,
                         const wd_solve_params* params, void* ws, size_t ws_bytes,
                         wd_solve_stats* stats, void* stream);

/* ---- solving D x = b, propagators and the pion correlator -------------- */

/* Workspace bytes for wd_solve_D with these parameters and nrhs fields. */
size_t wd_solve_D_workspace_bytes(wd_lattice lat, const wd_solve_params* params, int32_t nrhs);

/* Solve D x = b (dagger = 0) or D^dag x = b (dagger = 1) for nrhs full-lattice
 * fields; the paper's solve_DinvX!(y, D, x) and solve_DinvX!(y, D', x)
 * (App. C, "Definition of Dirac operators").  kappa[r] (host) is the hopping
 * parameter of rhs r.  x and b are device fields in the boundary layout with
 * every site used (both parities, whatever params->precond says).
 *   WD_EO  : Schur complement.  b'_e = b_e + kappa H_eo b_o; CG on
 *            D_hat^dag D_hat x_e = D_hat^dag b'_e; x_o = b_o + kappa H_oe x_e.
 *   WD_FULL: CG on the normal equations D^dag D x = D^dag b.
 * The adjoint system is solved as D (g5 x) = g5 b.  The pre- and post-steps
 * run in FP64 with the FP64 gauge store; the CG is wd_solve_DdagD's (mixed
 * precision and reliable updates per params).  stats (host, nrhs entries)
 * describe that CG: its residual is the one of the normal equations, to
 * params->tol.  Blocks the host.  Errors as wd_solve_DdagD; x is written only
 * when the CG ran (WD_OK, WD_ENOTCONVERGED, WD_ENONFINITE). */
wd_status wd_solve_D(wd_lattice lat, void* x, const void* b, int32_t nrhs, const double* kappa,
                     int32_t dagger, const wd_solve_params* params, void* ws, size_t ws_bytes,
                     wd_solve_stats* stats, void* stream);

/* Workspace bytes for wd_pion_correlator on this lattice. */
size_t wd_pion_workspace_bytes(wd_lattice lat);

/* Zero-momentum pion correlator of Wilson quarks (the paper's momentum-
 * projected Wilson pion correlator, Sec. 2 and App. D):
 *   corr[t] = sum over the spatial sites of time slice (t0 + t) mod Lt, over the
 *             nsrc propagator columns and over spin and colour, of |S|^2,
 * for t = 0 .. Lt-1.  S (device, boundary layout, nsrc fields back to back)
 * holds the solutions of D S_k = point source k, usually the 12 spin-colour
 * sources at a site of time slice t0; by gamma5-hermiticity the pion
 * contraction tr[g5 S g5 g5 S^dag g5] is this sum of squared moduli.  FP64
 * sums in a fixed order (deterministic).  corr is a host array of Lt doubles.
 * Blocks the host. */
wd_status wd_pion_correlator(wd_lattice lat, double* corr, const void* S, int32_t nsrc, int32_t t0,
                             void* ws, size_t ws_bytes, void* stream);

/* ---- pseudofermion action and force (molecular dynamics) -------------- */

/* eta = D^dag xi: the pseudofermion heatbath (the paper's
 * sample_pseudofermions! from a Gaussian xi, App. C, "Hybrid Monte Carlo"),
 * after which S_f(eta) = xi^dag xi.  One field, FP64, full lattice; needs
 * wd_apply_workspace_bytes(lat, WD_F64, 1).  Asynchronous. */
wd_status wd_pseudofermion_heatbath(wd_lattice lat, void* eta, const void* xi, double kappa,
                                    void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for wd_fermion_force with these parameters. */
size_t wd_fermion_force_workspace_bytes(wd_lattice lat, const wd_solve_params* params);

/* The pseudofermion action S_f = eta^dag (D^dag D)^{-1} eta and its
 * derivative "U dS_f/dU" (the paper's evaluate_FermiAction and calc_UdSfdU,
 * App. C, "Definition of fermion actions").  Solves D^dag Y = eta and D X = Y
 * with wd_solve_D (params; stats[0], stats[1] describe the two solves), then
 *   *action  = ||Y||^2                                         (host; may be NULL)
 *   F_mu(x)  = 2 kappa s_mu(x) U_mu(x) [ M + N^dag ]           (device; may be NULL)
 *   M = sum_s ((1 - g_mu) X(x+mu))_s Y(x)_s^dag,  N = sum_s ((1 + g_mu) X(x))_s Y(x+mu)_s^dag
 * (colour outer products summed over spin; s_mu(x) the boundary sign of the
 * link).  For U_mu(x) -> exp(eps T) U_mu(x), T traceless antihermitian,
 * dS_f/deps = Re tr[T F_mu(x)].  eta: one complex128 field, boundary layout;
 * F: complex128 [mu][t][z][y][x][3][3].  When only the action is requested the
 * second solve is skipped.  Blocks the host; errors as wd_solve_D. */
wd_status wd_fermion_force(wd_lattice lat, void* F, double* action, const void* eta, double kappa,
                           const wd_solve_params* params, void* ws, size_t ws_bytes,
                           wd_solve_stats* stats, void* stream);

/* p_mu(x) += factor * TA(F_mu(x)) with TA(M) = (M - M^dag)/2 - tr(M - M^dag)/6:
 * the momentum update of the paper's P_update_fermion
 * (Traceless_antihermitian_add!, factor = -eps * dtau).  p and F are device
 * complex128 [mu][t][z][y][x][3][3]; p may not overlap F.  Asynchronous. */
wd_status wd_ta_add(wd_lattice lat, void* p, double factor, const void* F, void* stream);

/* ---- staggered fermions ------------------------------------------------- */

/* The paper's second Dirac operator (App. C, "Definition of Dirac operators":
 * the staggered operator with a mass, applied with mul! and inverted with
 * solve_DinvX!), in the textbook Kogut-Susskind form on one colour vector per
 * site:
 *   (D chi)(x) = m chi(x) + 1/2 sum_mu eta_mu(x) [ s+ U_mu(x) chi(x+mu) - s- U_mu(x-mu)^dag chi(x-mu) ]
 * with eta_1 = 1, eta_2 = (-1)^x, eta_3 = (-1)^(x+y), eta_4 = (-1)^(x+y+z) and the
 * lattice's boundary signs s+/s-.  The hopping part is anti-Hermitian, so
 * D^dag = m - (hopping part).  Fields: complex128 [rhs][t][z][y][x][colour 3].
 * The gauge stores registered with wd_set_gauge serve both operators. */

/* Workspace bytes for wd_stag_apply. */
size_t wd_stag_apply_workspace_bytes(wd_lattice lat, int32_t prec, int32_t nrhs);

/* y = D x (dagger = 0) or D^dag x (dagger = 1) on the full lattice, at FP64 or
 * FP32 with that precision's gauge store.  Asynchronous. */
wd_status wd_stag_apply(wd_lattice lat, void* y, const void* x, int32_t nrhs, double mass, int32_t dagger,
                        int32_t prec, void* ws, size_t ws_bytes, void* stream);

/* Autotune the staggered stencil's launch shape (sites per workgroup, XCD-
 * aware block order, 1, 2 or 4 threads sharing the 8 hops of a site) for
 * this lattice, precision and nrhs by timing every candidate of 128 to 256
 * threads on stream (outputs with the same split must be bit-identical).
 * The choice follows the rule of wd_autotune and is kept in a process-wide
 * table used by later staggered
 * launches (not part of the exported text table).  Needs
 * wd_stag_apply_workspace_bytes.  Blocks the host.  The best_* outputs
 * receive the choice (may be NULL). */
wd_status wd_stag_autotune(wd_lattice lat, int32_t prec, int32_t nrhs, void* ws, size_t ws_bytes,
                           int32_t* best_sites_per_block, int32_t* best_swizzle, int32_t* best_split,
                           void* stream);

/* Set the staggered stencil's launch shape for this lattice, precision (of
 * its registered store) and nrhs, as wd_stag_autotune would: sites per
 * workgroup (a power of two), XCD-aware block order (0 / 1) and the number of
 * threads (1, 2, 4) sharing a site's 8 hops, with split * sites_per_block *
 * nrhs <= 256.  WD_EINVAL for any other shape, WD_ENOGAUGE without a store.
 * Host only. */
wd_status wd_stag_set_shape(wd_lattice lat, int32_t prec, int32_t nrhs, int32_t sites_per_block, int32_t swizzle,
                            int32_t split);

/* Workspace bytes for wd_stag_solve with these parameters and nrhs fields. */
size_t wd_stag_solve_workspace_bytes(wd_lattice lat, const wd_solve_params* params, int32_t nrhs);

/* Solve D x = b (dagger = 0) or D^dag x = b (dagger = 1) for nrhs fields with
 * per-rhs masses (host, finite and nonzero).  Even-odd: b'_e = m b_e - s H_eo b_o,
 * CG on the Hermitian positive definite even block M_e = m^2 - H_eo H_oe, then
 * x_o = (b_o - s H_oe x_e) / m (s = +1 for D, -1 for D^dag).  The CG is the
 * engine of wd_solve_DdagD: FP64 or FP32 inner iterations (params->inner) with
 * FP64 reliable updates, stopping on the true FP64 residual of M_e x_e = b'_e
 * at params->tol; params->precond must be WD_EO.  stats (host, nrhs entries)
 * describe that CG.  Blocks the host; errors as wd_solve_DdagD. */
wd_status wd_stag_solve(wd_lattice lat, void* x, const void* b, int32_t nrhs, const double* mass, int32_t dagger,
                        const wd_solve_params* params, void* ws, size_t ws_bytes, wd_solve_stats* stats,
                        void* stream);

/* Goldstone pion correlator of staggered quarks (the staggered entry of the
 * paper's pion correlators, Sec. 2 and App. D):
 *   corr[t] = sum over the spatial sites of time slice (t0 + t) mod Lt, over the
 *             nsrc propagator columns and over colour, of |S|^2,
 * for t = 0 .. Lt-1.  S (device, staggered layout [nsrc][t][z][y][x][colour 3]
 * complex128) holds the solutions of D S_a = point source a, usually the 3
 * colour sources at one site of slice t0; the staggered form of gamma5-
 * hermiticity, G(y, x) = eps(x) eps(y) G(x, y)^dag with eps = (-1)^(x+y+z+t),
 * turns the pion contraction into this sum of squared moduli.  Workspace:
 * wd_pion_workspace_bytes.  FP64 sums in a fixed order (deterministic); corr
 * is a host array of Lt doubles.  Blocks the host; errors as
 * wd_pion_correlator. */
wd_status wd_stag_pion_correlator(wd_lattice lat, double* corr, const void* S, int32_t nsrc, int32_t t0,
                                  void* ws, size_t ws_bytes, void* stream);

/* ---- batched solve over several lattices in one launch sequence ------- */

typedef struct {
  wd_lattice lat;
  void* x;              /* device, complex128 boundary layout, nrhs fields */
  const void* b;        /* device, complex128 boundary layout, nrhs fields */
  int32_t nrhs;         /* must be equal across the requests of one batch */
  int32_t pad;
  const double* kappa;  /* host, nrhs entries */
} wd_solve_request;

/* Workspace bytes for wd_solve_batch over these requests. */
size_t wd_batch_workspace_bytes(int32_t nreq, const wd_solve_request* reqs, const wd_solve_params* params);

/* Solve every request with one stencil launch per CG phase covering all of
 * them (uneven lattices in one grid).  stats holds sum(nrhs) entries, in
 * request order.  Blocks the host.  A single request whose rhs groups'
 * inner-loop vectors (the inner- and accumulation-precision vectors) exceed
 * 384 MB runs as consecutive waves of groups within that budget when a wave
 * holds at least two groups (each wave's results are those of its rhs solved
 * alone; its stats report that wave's time). */
wd_status wd_solve_batch(int32_t nreq, const wd_solve_request* reqs, const wd_solve_params* params,
                         void* ws, size_t ws_bytes, wd_solve_stats* stats, void* stream);

/* ---- measurement and tuning ------------------------------------------ */

/* Time n back-to-back launches of one stencil kernel of the CG iteration (one
 * even-odd hop, V/2 output sites x nrhs, precision prec, the tuned launch
 * shape) with hipEvents on stream; *ms_per_launch gets the mean duration.
 * mode selects the epilogue: 0 = plain H, 1 = aux - c H with |.|^2 reduction,
 * 2 = the CG residual update r -= alpha (aux - c g5 H) with |r|^2 reduction;
 * or 4 = the four stencil launches of one CG iteration on D_hat^dag D_hat
 * (App. C, "Definition of Dirac operators"), in order, repeated n times:
 * t1 = H p, t2 = p - c H t1 (mode 1), t3 = H g5 t2, then mode 2 on t3 and t2;
 * *ms_per_launch then gets the mean duration of the four together (the
 * reductions' stage 1 included; their stage 2 and the vector update are not).
 * Operates on scratch data in the workspace (wd_apply_workspace_bytes(lat,
 * prec, nrhs) bytes, zeroed first).  Blocks the host. */
wd_status wd_time_hop(wd_lattice lat, int32_t prec, int32_t nrhs, int32_t mode, int32_t n,
                      void* ws, size_t ws_bytes, double* ms_per_launch, void* stream);

/* Time n back-to-back launches of a plain streaming-read kernel over the
 * device buffer buf (bytes, a positive multiple of 16; 2048 blocks of 256
 * threads, 16-byte loads with a grid stride): the attainable read rate the
 * stencils are compared with.  out (device, >= 2048 doubles) receives the
 * block sums.  *ms_per_read gets the mean duration.  Blocks the host. */
wd_status wd_time_read(const void* buf, size_t bytes, int32_t n, void* out, size_t out_bytes, double* ms_per_read,
                       void* stream);

/* Autotune the stencil launch shape (sites per workgroup, block order: 0
 * plain, 1 each XCD a contiguous range of sites, 2 the same ranges visited
 * t-slice innermost; number of threads the 8 hops of a site are split over) for this
 * lattice, precision and nrhs by timing every candidate on stream (the four
 * stencil launches of one CG iteration in order, as wd_time_hop mode 4).  Among
 * the candidates whose workgroup count lets the CG fold its reductions (if
 * any do), of those within 3 % of the fastest, the one with the fewest
 * workgroups is chosen, XCD-aware order first (each reducing launch of the
 * CG leaves one partial sum per workgroup for stage 2 to gather).  The choice
 * is kept in a process-wide table keyed by (dims, prec, recon, nrhs) and used
 * by every later launch.  Candidates with the same split must produce
 * bit-identical output (checked).  Needs wd_apply_workspace_bytes(lat, prec,
 * nrhs).  Blocks the host.  The best_* outputs receive the choice (may be NULL). */
wd_status wd_autotune(wd_lattice lat, int32_t prec, int32_t nrhs, void* ws, size_t ws_bytes,
                      int32_t* best_sites_per_block, int32_t* best_swizzle, int32_t* best_split,
                      void* stream);

/* Read or write the tuning table as text ("Lx Ly Lz Lt prec recon nrhs sblk swz split"
 * lines; swz in {0,1,2}; split in {1,2,4,8} (8 not at FP64); split * sblk * nrhs <= 256, or <= 512
 * for split 8; sblk * nrhs >= 64).
 * wd_tune_export returns the bytes needed (including the NUL) and writes at
 * most cap bytes into buf (may be NULL). */
size_t wd_tune_export(char* buf, size_t cap);
wd_status wd_tune_import(const char* text);

/* ---- serving ------------------------------------------------------------ */

typedef struct wd_server_s* wd_server;

/* A server owns a caller-provided device pool of pool_bytes and admits solve
 * requests while their footprint (per-request workspace) fits in the pool and
 * a slot (of max_slots) is free.  Admitted requests are solved together by a
 * worker thread, one launch per CG phase over all running requests
 * (continuous batching: requests join and leave at poll boundaries).  Gauge
 * stores are the caller's (registered on each lattice) and stay resident. */
wd_status wd_server_create(wd_server* out, void* pool, size_t pool_bytes, int32_t max_slots,
                           const wd_solve_params* params, void* stream);
wd_status wd_server_destroy(wd_server srv);

/* Bytes of the pool a request of this lattice and nrhs would hold. */
size_t wd_server_footprint(wd_server srv, wd_lattice lat, int32_t nrhs);

/* Queue a solve of D^dag D x = b (nrhs fields, kappa[nrhs] host values
 * copied at submit).  x and b are caller device buffers that must stay alive
 * until the ticket completes.  Returns WD_EBUSY without queueing when the
 * footprint can never fit the pool.  Requests wait FIFO for memory/slots. */
wd_status wd_server_submit(wd_server srv, wd_lattice lat, void* x, const void* b, int32_t nrhs,
                           const double* kappa, uint64_t* ticket);

/* Non-blocking: returns 1 and fills stats[nrhs] (host) once the ticket has
 * completed, 0 while it is queued or running, <0 on error. */
int32_t wd_server_poll(wd_server srv, uint64_t ticket, wd_solve_stats* stats);

/* Block until the ticket completes (timeout_ms < 0: no limit); 1 done, 0 timed out. */
int32_t wd_server_wait(wd_server srv, uint64_t ticket, wd_solve_stats* stats, int32_t timeout_ms);

/* ---- diagnostics --------------------------------------------------------- */
const char* wd_status_string(wd_status s);
const char* wd_last_error(void);
const char* wd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WDIRAC_H */
