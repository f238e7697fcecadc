// Solver state machines for Sinkhorn (Section 4.1) and IBP barycenters (Appendix A),
// and the engine that advances any set of them together with batched launches.
#pragma once

#include <memory>
#include <vector>

#include "se2_internal.h"

namespace se2 {

// Stream-ordered device allocation with an optional arena (the serving queue's budget).
class DeviceArena;

struct DevBuf {
    double *p = nullptr;
    size_t n = 0;
};

// Solve kinds: the two public request kinds and the JKO step of a gradient flow.
constexpr int kKindJKO = 2;
// Largest share of recomputed groups a bulk phase on the matrix cores keeps running with:
// above it the exact engine is faster.  Against the pruned exact engine (measured on the
// eps-scaling stages of the paired lines: the matrix cores win at eps 1.6 and 0.8 and lose at
// 0.4 and 0.2) a quarter; against a dense exact visit, whose cost the recomputation of a
// share s approaches as s (plus the contraction, a few percent of it), three quarters.
constexpr double kBulkFallbackMaxPruned = 0.25;
constexpr double kBulkFallbackMaxDense = 0.75;

// One solve, resident on the device.  All potentials are base-2 log-scalings.
struct Solve {
    int kind = SE2_REQ_OT;           // SE2_REQ_OT or SE2_REQ_BARYCENTER
    const Kernel *k = nullptr;
    size_t E = 0;                    // elements per grid array
    int tiles = 0;                   // 8x8 output tiles per grid array
    se2_opts_t opts{};
    // OT
    double *lmu = nullptr, *lnu = nullptr, *phi[2] = {nullptr, nullptr}, *psi = nullptr;
    ListSet ls_phi, ls_psi;          // pruning state of the b-update (input phi) and a-update (input psi)
    const double *mu_lin = nullptr, *nu_lin = nullptr;  // FP64 inputs (dual, final checks)
    int cur = 0;
    // JKO step: lsum = log2 K^T a of the last b-update; prox constant c, exponent m, cell measure
    double *lsum = nullptr;
    double jko_c = 0.0, jko_m = 2.0, jko_ref = 1.0;
    // barycenter: only measures with lambda > 0
    int n = 0;
    std::vector<double> lam;
    std::vector<double *> lm, lv, lw, ld;
    std::vector<ListSet> ls_v, ls_w;  // pruning state of the w-update (input lv_i) and d-update (input lw_i)
    std::vector<const double *> m_lin;
    double *logbar = nullptr;
    double **d_lv = nullptr;         // device tables of lv[i], ld[i], lw[i] and the weights
    const double **d_ld = nullptr;
    const double **d_lw = nullptr;
    SumItem *d_cost_items = nullptr; // [2n] cost and mass sums of the finishing
    double *work_all = nullptr;      // [2n][tiles][2] work counters of every list, contiguous
    double *d_lam = nullptr;
    double *combine_part = nullptr;  // [combine_chunks(n)][E] chunk partials of the combine
    // common
    double *partial = nullptr;       // [job][tile][nt] error partials
    double *err = nullptr;           // 3 * max(1, n) + 8 result slots of the finishing (device)
    int32_t *offsets = nullptr;      // per-job partial offsets (device), max(1, n) + 1
    int iter = 0;                    // completed iterations
    bool done = false;
    int status = SE2_MAX_ITER;
    double last_err = -1.0;
    int convs = 0;
    double t_start = 0.0;
    // eps-scaling: the kernels of the stages (coarser eps first, the requested eps last)
    std::vector<double> stage_eps;
    std::vector<const Kernel *> stage_k;
    int stage = 0;
    int scaling_iters = 0;           // iterations run before the last stage began
    // phases: a solve with opts.polish runs its bulk engine (opts.bulk) over the coarse eps
    // stages and at the final eps until phase_after_check() moves it to opts.prec
    int phase = 0;                   // 0: bulk, 1: polish
    int phase_switch_iter = -1;      // iteration at which the polish phase began
    double prev_err = -1.0;          // error of the previous check of the current stage
    // bulk phase: recomputed groups (summed over the measures) at the last check, as read by
    // read_errors (-1: not read), and the count and iteration of the check before
    double fb_checked = -1.0;
    double fb_prev = 0.0;
    int fb_prev_iter = 0;
    uint64_t trace_range = 0;        // roctx range of the current phase (0: none open)
    int32_t *fb_count = nullptr;     // per job (measure): groups recomputed after a failed certificate (read as uint32)
    double terms_linear = 0.0;       // window terms evaluated by the matrix-core engines
    // memory
    void *block = nullptr;           // single allocation holding every buffer
    size_t bytes = 0;
};

// OT and JKO solves have one scaling pair (a, b) with a double-buffered a-potential.
inline bool ot_like(const Solve &s) { return s.kind != SE2_REQ_BARYCENTER; }

// Window entries inside the grid summed over all outputs: the algorithmic LSE
// terms of one convolution of a grid array with this kernel.
double conv_terms(const Kernel &k);

// Bytes one solve needs on the device (for admission against a budget).
size_t solve_bytes(int kind, const Kernel &k, int n_active, bool prune);
// Pruning applies to the exact FP32 engine only (the FP64 engine always visits every term,
// the matrix-core engines evaluate the whole window on the matrix cores).
inline bool prune_wanted(const se2_opts_t &o) { return o.prune != 0 && o.prec == SE2_F32; }
bool prune_enabled(const Solve &s);
// The engine a solve runs now: its bulk engine during the bulk phase, else opts.prec.
inline bool in_bulk_phase(const Solve &s) { return s.opts.polish && s.phase == 0; }
inline int engine_prec(const Solve &s) { return in_bulk_phase(s) ? s.opts.bulk : s.opts.prec; }
inline bool linear_engine(int prec) { return prec == SE2_BF16 || prec == SE2_F32_MFMA; }
// Options a solver accepts for this kernel (engines, phases, iteration limits, eps schedule).
bool valid_solver_opts(const se2_opts_t &o, const Kernel &k);
// Phase control after a check of a solve that goes on (error err).  A solve in its bulk phase
// moves to the polish engine (a) at any stage, once more than kBulkFallbackMax* of the
// (tile, orientation) groups its bulk engine visited since the previous check were recomputed
// exactly (the matrix-core engine no longer pays there), or (b) at its final eps stage, once
// err <= opts.switch_tol or the error did not fall since the stage's previous check.
void phase_after_check(Solve &s, double err);

// Carve the buffers of `s` out of `mem` (size solve_bytes()).
void solve_bind(Solve &s, void *mem);

// Upload inputs and initialise: log-marginals, potentials, the first half-step.
// mus/lams: for barycenters the active measures only.  Stream-ordered.
int solve_reset_lists(Solve &s, hipStream_t st);
int solve_setup_ot(Solve &s, const double *mu, const double *nu, const double *init_g_natural, hipStream_t st);
int solve_setup_bary(Solve &s, const std::vector<const double *> &mus, hipStream_t st);
// init (may be null: log b = 0) times init_scale gives the first log2 b.
int solve_setup_jko(Solve &s, const double *mu, const double *init, double init_scale, hipStream_t st);

// eps-scaling schedule of `o` for a kernel at `eps`: eps_start * factor^s while above eps,
// then eps itself (only eps when the scheme is off).  SE2_EINVAL for a bad schedule (factor
// outside (0, 1), stage_iters < 1, more than 32 coarse stages, coarse iterations >= max_iter).
int eps_schedule(const se2_opts_t &o, double eps, std::vector<double> &out);
// Resolves the stage kernels of `s` (from s.opts and the kernel of the requested eps) and
// starts the solve at the first stage.  Call before solve_bind.
int plan_stages(Solve &s, const Kernel &base);
inline bool final_stage(const Solve &s) { return s.stage + 1 >= static_cast<int>(s.stage_k.size()); }

// Kinds of batched convolution launches: the exact log-domain engine (dense visits, or
// certified sparse visits with their rebuilds), its FP64 form, and the certified linear-domain
// engines on the matrix cores (bfloat16 or FP32 operands) with their exact recomputation.
enum LaunchKind { LK_DENSE = 0, LK_SPARSE = 1, LK_F64 = 2, LK_LIN_BF16 = 3, LK_LIN_F32 = 4 };

// Debug checks, on when the environment variable SE2_DEBUG is set (and not "0") at the
// first launch: every job table is checked on the host against the invariants the kernels
// assume (grid and tile counts, block ranges, radius within the launch's, no output aliasing
// its input, the pruning state of sparse jobs), and every launch is synchronised, so that
// a failing kernel is reported by the launch that issued it.  Results are unchanged.
bool debug_checks();
int check_jobs(const std::vector<ConvJob> &jobs, int nblocks, int nt, int R_max, LaunchKind kind, int rpw);

// Advances a set of solves (same ntheta or not) by one iteration each, with batched
// launches: one launch per (stage, ntheta class, engine).  If `check` is true, also reduces
// each solve's marginal error into its device `err` slot.
class Engine {
public:
    Engine();
    ~Engine();
    int init_first_halfstep(const std::vector<Solve *> &solves, hipStream_t st);
    int step(const std::vector<Solve *> &solves, bool check, hipStream_t st);
    // One half of step(): half 0 is the b-update (d-update and combine for barycenters,
    // the proximal step for JKO), half 1 the a-update (w-update) with the iteration count,
    // and the error sums when `check`.
    int step_half(const std::vector<Solve *> &solves, int half, bool check, hipStream_t st);
    // Rebuilds of uncertified tiles at 16 waves per item while few are queued (the
    // default), or always at 8.  Outputs are identical either way; a wide workgroup
    // cannot share a CU with a sparse one, so engines whose streams run beside other
    // engines' work keep the narrow form.
    void set_wide_rebuild(bool on) { wide_rebuild_ = on; }
    // Copies err slots of the given solves to host (synchronises the stream).
    int read_errors(const std::vector<Solve *> &solves, std::vector<double> &max_err, hipStream_t st);
    // Optional event timing of every log-domain convolution launch.  With a reference event
    // (recorded before any profiled launch on this engine's stream), every launch's
    // [start, end] in ms after it is kept in prof_intervals, so the intervals of engines
    // on different streams can be merged.
    void set_profiling(bool on, hipEvent_t ref = nullptr);
    std::vector<std::pair<double, double>> prof_intervals;
    // FP64 check convolutions (dense, FP64 exp): one launch per ntheta class.
    int launch_checks(const std::vector<ConvJob> &jobs, const std::vector<int> &nts, hipStream_t st);
    // Folds the pending timing-event pairs into the totals, waiting for each; a check folds
    // those already known complete by itself, so call this before reading the totals.
    int collect_profile();
    // The caller has synchronised the engine's stream: everything launched so far is done.
    void mark_drained() { drained_ = clock_; }
    double prof_seconds = 0.0, prof_terms = 0.0, prof_outputs = 0.0;
    int64_t prof_launches = 0;

private:
    int launch_stage(const std::vector<Solve *> &solves, int stage, bool with_err, hipStream_t st);
    int stage_and_launch(std::vector<ConvJob> &jobs, int nblocks, int nt, int R_max, LaunchKind kind, int rpw,
                         hipStream_t st);
    int ensure(size_t njobs, size_t nblocks);
    // Device copies of job tables and block maps, kept while their content recurs (a
    // solve set cycles through a few tables: two stages x two buffer parities, and the
    // check variants); a table is uploaded only when it is not cached.
    struct TableSlot {
        std::vector<ConvJob> key;  // host copy of the table held
        ConvJob *d_jobs = nullptr;
        int32_t *d_map = nullptr;
        size_t cap_jobs = 0, cap_blocks = 0;
        uint64_t last = 0;  // clock of the last launch that read the slot
    };
    static constexpr int kTableSlots = 16;
    TableSlot tables_[kTableSlots];
    // Launch clock, and its value when the stream was last seen idle (after a host
    // synchronisation).  An engine issues all its work on one stream, so a table slot or item
    // table whose last use is not later than drained_ can be rewritten without waiting.
    uint64_t clock_ = 0;
    uint64_t drained_ = 0;
    int sync(hipStream_t st);  // hipStreamSynchronize, then drained_ = clock_
    int2 *d_rebuild_ = nullptr;      // tiles left to the wide rebuild kernel, one slot per block
    int *d_rebuild_count_ = nullptr;  // two counters, used alternately
    int *h_published_ = nullptr;      // pinned: rebuild items of the last launch per ntheta class
    int *d_published_ = nullptr;      // the same memory as the kernels address it
    bool wide_rebuild_ = true;
    int4 *d_fb_ = nullptr;           // tiles left to the exact recomputation by matrix-core launches
    size_t cap_fb_ = 0;
    int *d_fb_count_ = nullptr;      // two counters used alternately (each launch zeroes the other)
    int fb_flip_ = 0;
    int rc_flip_ = 0;
    size_t cap_rebuild_ = 0;
    ConvJob *h_jobs_ = nullptr;      // pinned staging (double-buffered)
    int32_t *h_map_ = nullptr;
    size_t cap_jobs_ = 0, cap_blocks_ = 0;
    int flip_ = 0;
    hipEvent_t staged_[2] = {nullptr, nullptr};
    // check results: pinned coherent memory that k_publish writes (flag word, then errors)
    static constexpr size_t kChkHeader = 256;
    static constexpr int kCheckPollMs = 5;
    char *h_chk_ = nullptr, *d_chk_ = nullptr;
    size_t cap_err_ = 0;
    int chk_seq_ = 0;
    // batched error sums of a check: one item per (solve, job), results contiguous
    std::vector<SumItem> items_key_;   // the item table on the device
    SumItem *h_items_ = nullptr, *d_items_ = nullptr;
    double *d_errs_ = nullptr;
    size_t cap_items_ = 0;
    uint64_t items_last_ = 0;  // clock of the last error-sum launch that read the item table
    int sum_errors(const std::vector<Solve *> &solves, hipStream_t st);
    bool prof_ = false;
    hipEvent_t prof_ref_ = nullptr;
    struct Pending {
        hipEvent_t a, b;
        double terms, outputs;
    };
    std::vector<Pending> pending_;
    size_t prof_ready_ = 0;  // leading entries of pending_ known to be complete
    int fold_profile(size_t count, bool wait);
    std::vector<hipEvent_t> spare_;
};

// Moves every solve of `solves` whose coarse eps stage has run its iterations to the next
// eps: its scalings are carried over in absolute units (log b times eps_old / eps_new), its
// pruning lists are dropped, and the next a-update (w-update) is taken with the new kernel,
// batched over the solves that move.  A solve's stage boundaries depend on its own iteration
// count only.  Stream-ordered.
int advance_stages(Engine &eng, const std::vector<Solve *> &solves, hipStream_t st);

// Finishing of a group of solves: potentials out (natural units), plan cost, mass,
// dual, optional FP64 re-check of the marginal error.  Every solve's GPU work is
// queued first (the FP64 checks batched over the group), then one synchronisation;
// each request's report and status are filled in.  Blocking on `st`.
struct FinishReq {
    Solve *s = nullptr;
    double *f_out = nullptr, *g_out = nullptr;  // OT and JKO outputs (may be null)
    double *bary_out = nullptr;                 // barycenter output, or the next measure of a JKO step
    se2_report_t rep{};
    int rc = SE2_OK;
};
int finish_solves(Engine &eng, std::vector<FinishReq> &reqs, hipStream_t st);

double now_seconds();

}  // namespace se2
