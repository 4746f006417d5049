// Host-side internals: lattice object, error reporting, tuning table and
// the batched CG driver shared by the C ABI and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/wdirac.h"
#include "wd_kernels.h"

struct wd_lattice_s {
  wd::Geom g;
  int32_t L[4];
  int32_t bc[4];
  struct Store {
    void* ptr = nullptr;
    int recon = 0;
  } store[3];
};

namespace wd {

void set_error(const char* fmt, ...);
wd_status fail(wd_status s, const char* fmt, ...);
wd_status hip_fail(hipError_t e, const char* what);

#define WD_HIP(call)                                  \
  do {                                                \
    hipError_t _e = (call);                           \
    if (_e != hipSuccess) return hip_fail(_e, #call); \
  } while (0)

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Bytes of one parity block of nrhs spinors over n sites at precision prec.
size_t vec_bytes(int prec, size_t n, int nrhs);
size_t gauge_bytes(const Geom& g, int prec, int recon);
inline int acc_prec(int prec) { return prec == F16 ? F32 : prec; }

struct Tune {
  int sblk;   // sites per block (power of two; see valid_tune)
  int swz;    // block order: 0 plain, 1 XCD-aware, 2 XCD-aware with t-slices innermost
  int split;  // threads per (site, rhs) in the stencil: 1, 2 or 4
};
bool valid_tune(const Tune& t, int nrhs, int prec);

// Fold limits of the CG reductions: a reduction is finished by every block
// of the launch that consumes it only when each slot has at most
// kFoldPartials block partials and the consumer's blocks together read at
// most kFoldReads of them; every block repeats the whole gather, so the fold
// only pays off while partials and blocks are few.  (Measured at 16^3x32:
// 1024 stencil blocks each gathering 1024 partials cost the staggered FP64 CG
// about 9 us per iteration, far more than a finalize kernel; 512
// vector-update blocks gathering 1024 partials were still 6 us per iteration
// faster than the finalize kernel in the FP32 Wilson CG.)
constexpr int kFoldPartials = 1024;
constexpr long long kFoldReads = 1LL << 19;

// Cache blocking of a single request's rhs groups: when the vectors that
// every CG iteration touches (the inner- and accumulation-precision vectors
// of all groups) exceed kWaveBytes, the groups run as consecutive waves of
// at most kWaveBytes each, provided a wave still holds two groups or more
// (the groups of one launch share the links' reads).  1.5 x the Infinity
// Cache: a 12-source FP32-inner request at 16^3x32 (378 MB) stays one wave.
constexpr size_t kWaveBytes = (size_t)384 << 20;

// The autotuners' choice among timed stencil shapes (ms per launch) for a
// lattice of n sites per parity: each shape is costed as per_iter of its
// launches plus a finalize kernel (about 5 us) for each of the two CG
// reductions its block count cannot fold; of the shapes within 3 % of the
// cheapest, the one with the fewest blocks (every reducing launch leaves one
// partial per block), preferring the XCD-aware order, which is also kept
// within 10 % of the plain order while a vector (vec_bytes) fits in half of
// the L2s.
// Whether the swz = 2 block order differs from swz = 1 on this lattice at sblk sites per block.
bool tslice_order_applies(const Geom& g, int sblk);
Tune pick_shape(const std::vector<std::pair<Tune, double>>& timed, long long n, int nrhs, int per_iter,
                double vec_bytes, Tune fallback);
Tune tune_lookup(const wd_lattice_s* lat, int prec, int recon, int nrhs);
void tune_store(const wd_lattice_s* lat, int prec, int recon, int nrhs, Tune t);
Tune stag_tune_lookup(const wd_lattice_s* lat, int prec, int recon, int nrhs);
void stag_tune_store(const wd_lattice_s* lat, int prec, int recon, int nrhs, Tune t);
int default_sblk(int nrhs);

// Slot of a launch for a lattice; blocks for `parity` (0/1 or 2 = both).
void fill_slot_geometry(Slot& S, const wd_lattice_s* lat, int sblk, int parity);
void finish_launch(Launch& L);
Launch base_launch(int nrhs, const Tune& t, int parity);
int min_sblk(int nrhs);  // smallest block size the partial buffers allow

// Events around stencil launches (timing mode).
// Event timing of every stencil launch of a solve (timing = 1).  A launch
// whose slots all skip their work (masked after convergence, or a reliable-
// update sequence with nothing held) returns at once: the kernels set the
// launch's work flag (Launch::work_flag, one int per timed launch in a ring
// of kTimingFlags per device) only when a slot did its work, and the figures
// below leave the other launches out, so that their algorithmic bytes are not
// counted against a few microseconds.  Launches beyond the ring are counted.
constexpr int kTimingFlags = 1 << 16;
struct HopTimer {
  bool on = false;
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  int* flags = nullptr;              // device ring of kTimingFlags work flags, zeroed at the start
  std::vector<int> mode;             // epilogue mode + 4 x precision of each timed launch
  std::vector<double> mode_bytes;    // its algorithmic bytes
  std::vector<long long> mode_sites;  // its output sites x rhs
  std::vector<float> dur;            // after classify(): ms of each launch
  std::vector<char> skipped;         // after classify(): 1 if it skipped its work
  long long site_updates = 0;        // after classify(): over the launches that worked
  double bytes = 0.0;
  long long nskipped = 0;
  int* next_flag() const { return flags && used / 2 < (size_t)kTimingFlags ? flags + used / 2 : nullptr; }
  hipError_t begin(hipStream_t s);
  hipError_t end(hipStream_t s, long long sites, double bytes, int mode);
  hipError_t classify();  // after the stream has finished
  double total_ms();
  // per epilogue mode; prec >= 0: only the launches at that precision
  void by_mode(double ms[4], long long n[4], double b[4], int prec = -1);
  void release();
};

// Workspace of one solve item (a lattice with nrhs fields), relative to the
// item's base.  The per-rhs states live in a separate array shared by every
// item of an engine so that one copy polls all of them.
struct ItemLayout {
  size_t off_partial;
  size_t off_bh, off_xh, off_rh, off_h1, off_h2;  // FP64 vectors
  size_t off_x, off_r;                            // accumulation precision
  size_t off_p, off_t1, off_t2;                   // inner precision
  size_t hstride, astride, vstride;               // parity strides (FULL mode)
  size_t total;
};
// Operator families the engine runs: the Wilson operator (CG on D^dag D or
// D_hat^dag D_hat) or the staggered operator (CG on its even block
// M_e = m^2 - H_eo H_oe; even-odd only, FP64 or FP32 inner).
enum Op : int { OP_WILSON = 0, OP_STAG = 1 };

// Bytes of one parity block of nrhs fields of the operator's vector type.
size_t field_bytes(int op, int prec, size_t n, int nrhs);

ItemLayout item_layout(const wd_lattice_s* lat, const wd_solve_params& p, int nrhs, int op = OP_WILSON);
size_t states_bytes(size_t nstates);

// One solve in an engine.
struct EItem {
  wd_lattice_s* lat = nullptr;
  void* x = nullptr;
  const void* b = nullptr;
  std::vector<double> kappa;
  int nrhs = 1;
  ItemLayout lay{};
  char* base = nullptr;             // device workspace of the item
  RhsState* st = nullptr;           // device states (nrhs entries)
  int state_index = 0;              // index of st[0] in the engine's state array
  std::vector<RhsState> h_init;     // host staging of the initial states
  long long started_block = 0;      // engine block count when the item was started
  // server bookkeeping
  uint64_t ticket = 0;
  double t_submit = 0.0, t_done = 0.0;
  size_t pool_off = 0, pool_len = 0;
  int slot = -1;
  std::vector<wd_solve_stats> stats;
};

// Runs CG for a changing set of items: one launch per CG phase covers every
// item (grouped by nrhs, at most kMaxSlots per launch).
class Engine {
 public:
  Engine(const wd_solve_params& p, hipStream_t s, RhsState* states, HopTimer* timer, int op = OP_WILSON)
      : p_(p), eo_(p.precond == WD_EO), op_(op), stream_(s), states_(states), timer_(timer) {}
  std::vector<EItem*> items;
  long long blocks = 0;  // poll blocks enqueued so far

  wd_status start_item(EItem* it);    // enqueue state init, source import, INIT
  // Enqueue K inner iterations (K a multiple of reliable_every()), with a
  // reliable-update sequence after every reliable_every() iterations.
  wd_status enqueue_block(int K, bool ru = true);
  wd_status export_item(EItem* it);   // x = x_h (boundary layout)
  void set_changed() { base_key_ = 0; }
  int max_block() const;              // block size for a cold start
  int reliable_every() const;
  RhsState* states() const { return states_; }

 private:
  struct Phase;
  wd_status run_phase(const std::vector<EItem*>& list, const Phase& ph);
  wd_status run_iteration();
  wd_status run_reliable();
  wd_status enqueue_direct(int K, bool ru);
  uint64_t block_key(int K, bool ru);
  wd_solve_params p_;
  bool eo_;
  int op_;
  hipStream_t stream_;
  RhsState* states_;
  HopTimer* timer_;
  uint64_t* hash_ = nullptr;          // when set, launches are hashed instead of issued
  uint64_t base_key_ = 0;             // hash of one iteration + reliable sequence for the current items
  std::vector<uint64_t> seen_;        // block keys launched once by this engine
};

// Sizes poll blocks from the residual history: the next block ends where the
// earliest rhs is expected to reach its next event (delta drop or tolerance).
struct BlockPlanner {
  struct Snap {
    int iters;    // at the previous poll
    double rho;
    int iters0;   // at the first poll
    double rho0;
  };
  std::vector<Snap> snap;
  int kmax = 32;
  double left = 0.0;  // iterations expected after the blocks in flight (last call of next)
  double left_full = 0.0;  // the same without the early-leaning shrink (whether a block reaches the event)
  int nrun = 0;       // rhs not yet finished (last call of next)
  // > 0: size of the next block; -1: wait for the blocks in flight; 0: all done.
  // idx (optional) lists the state entries to consider; else entries 0..n-1.
  int next(const RhsState* hs, size_t n, int inflight, const int* idx = nullptr);
};

// Fill stats from final device states (host copy).
wd_status stats_from_state(const RhsState& s, double seconds, const HopTimer* t, wd_solve_stats& o);

// Solve items to completion (no items join later).  Blocks the host.
wd_status run_batch(std::vector<EItem>& items, const wd_solve_params& p, RhsState* states, hipStream_t stream,
                    wd_solve_stats* stats, int op = OP_WILSON);

wd_status check_params(const wd_solve_params& p);
wd_status check_lattice_for(const wd_lattice_s* lat, int prec, int precond);

}  // namespace wd
