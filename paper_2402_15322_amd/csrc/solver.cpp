// Sinkhorn and IBP state machines on the device, and the batched stepping engine.
//
// Sinkhorn (Section 4.1), log form with phi = log a, psi = log b in base-2 units:
//     phi_{l+1} = log mu - LSE(L + psi_l),   psi_{l+1} = log nu - LSE(L + phi_{l+1}),
// psi_0 = 0 (or a warm start), K^T = K.  Iteration l = b-update then a-update; the
// a-update of iteration l+1 also yields the first-marginal L1 error of (phi_l, psi_l),
//     e_l = sum_x mu(x) |2^(phi_l(x) - phi_{l+1}(x)) - 1|,
// whose second marginal is exact.  phi is double-buffered so that the iterate
// whose error was measured is the one returned.
//
// IBP barycenter (Appendix A), log form, measures with lambda_i > 0 only:
//     w-update  lw_i = log mu_i - LSE(L + lv_i)
//     d-update  ld_i = lv_i + LSE(L + lw_i)
//     combine   log bar = sum_i lambda_i ld_i,  lv_i += log bar - ld_i
// The w-update of iteration j+1 yields max_i sum mu_i |2^(lw_i^(j) - lw_i^(j+1)) - 1|,
// the mu_i-side marginal error of iterate j (its barycenter side is exact).
#include "solver.h"
#include "launch.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <thread>

namespace se2 {

double now_seconds() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

namespace {

constexpr size_t kAlign = 256;

size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

struct Carver {
    char *p;
    size_t used = 0;
    template <typename T>
    T *take(size_t count) {
        T *r = p ? reinterpret_cast<T *>(p + used) : nullptr;
        used += up(count * sizeof(T));
        return r;
    }
};

ListSet carve_lists(Carver &c, const Kernel &k, size_t E, int tiles, bool prune, double *work = nullptr) {
    const int nt = k.grid.ntheta, HW = kTile + 2 * k.metric.radius;
    ListSet l;
    if (prune) {
        l.lists = c.take<ListEntry>(static_cast<size_t>(tiles) * nt * kListMax + kListPad);
        l.ref = c.take<float>(static_cast<size_t>(tiles) * nt * HW * HW);
        l.len = c.take<int32_t>(static_cast<size_t>(tiles) * nt);
        l.mref = c.take<float>(E);
    }
    l.dense_flag = c.take<int32_t>(static_cast<size_t>(tiles));
    l.work = work ? work : c.take<double>(2 * static_cast<size_t>(tiles));
    return l;
}

// Lays out every buffer of a solve; with mem == nullptr it only measures.
size_t carve(Solve &s, int kind, const Kernel &k, int n, bool prune, void *mem) {
    const size_t E = static_cast<size_t>(k.grid.nx) * k.grid.ny * k.grid.ntheta;
    const int tiles = tiles_of(k.grid.nx) * tiles_of(k.grid.ny);
    prune = prune && conv_lse_sparse_fits(k.grid.ntheta, k.metric.radius);
    const int nj = kind != SE2_REQ_BARYCENTER ? 1 : n;
    const size_t npart = static_cast<size_t>(tiles) * k.grid.ntheta * nj;
    const size_t ncost = 2 * static_cast<size_t>(plan_parts(k)) * nj + 512;
    Carver c{static_cast<char *>(mem)};
    if (kind != SE2_REQ_BARYCENTER) {
        s.lmu = c.take<double>(E);
        s.lnu = c.take<double>(E);
        s.phi[0] = c.take<double>(E);
        s.phi[1] = c.take<double>(E);
        s.psi = c.take<double>(E);
        s.ls_phi = carve_lists(c, k, E, tiles, prune);
        s.ls_psi = carve_lists(c, k, E, tiles, prune);
        if (kind == kKindJKO) s.lsum = c.take<double>(E);
    } else {
        s.lm.assign(n, nullptr);
        s.lv.assign(n, nullptr);
        s.lw.assign(n, nullptr);
        s.ld.assign(n, nullptr);
        for (int i = 0; i < n; ++i) {
            s.lm[i] = c.take<double>(E);
            s.lv[i] = c.take<double>(E);
            s.lw[i] = c.take<double>(E);
            s.ld[i] = c.take<double>(E);
        }
        s.logbar = c.take<double>(E);
        s.phi[0] = c.take<double>(E);  // scratch for the FP64 check
        s.d_lv = c.take<double *>(n);
        s.d_ld = c.take<const double *>(n);
        s.d_lw = c.take<const double *>(n);
        s.d_lam = c.take<double>(n);
        s.d_cost_items = c.take<SumItem>(2 * static_cast<size_t>(n));
        s.combine_part = combine_chunks(n) > 1 ? c.take<double>(static_cast<size_t>(combine_chunks(n)) * E) : nullptr;
        s.work_all = c.take<double>(4 * static_cast<size_t>(n) * tiles);
        s.ls_v.assign(n, ListSet());
        s.ls_w.assign(n, ListSet());
        for (int i = 0; i < n; ++i) {
            double *w = s.work_all ? s.work_all + 4 * static_cast<size_t>(i) * tiles : nullptr;
            s.ls_v[i] = carve_lists(c, k, E, tiles, prune, w);
            s.ls_w[i] = carve_lists(c, k, E, tiles, prune, w ? w + 2 * static_cast<size_t>(tiles) : nullptr);
        }
    }
    s.partial = c.take<double>(npart > ncost ? npart : ncost);
    s.err = c.take<double>(3 * static_cast<size_t>(nj) + 8);
    s.offsets = c.take<int32_t>(static_cast<size_t>(nj) + 1);
    s.fb_count = c.take<int32_t>(static_cast<size_t>(nj));
    return c.used;
}

}  // namespace

double conv_terms(const Kernel &k) {
    const int R = k.metric.radius, nt = k.grid.ntheta;
    double sx = 0.0, sy = 0.0;
    for (int d = -R; d <= R; ++d) {
        sx += (k.grid.nx - std::abs(d)) > 0 ? (k.grid.nx - std::abs(d)) : 0;
        sy += (k.grid.ny - std::abs(d)) > 0 ? (k.grid.ny - std::abs(d)) : 0;
    }
    return sx * sy * nt * nt;
}

size_t solve_bytes(int kind, const Kernel &k, int n_active, bool prune) {
    Solve tmp;
    return carve(tmp, kind, k, n_active, prune, nullptr);
}

bool prune_enabled(const Solve &s) {
    return prune_wanted(s.opts) && conv_lse_sparse_fits(s.k->grid.ntheta, s.k->metric.radius);
}

void solve_bind(Solve &s, void *mem) {
    s.E = static_cast<size_t>(s.k->grid.nx) * s.k->grid.ny * s.k->grid.ntheta;
    s.tiles = tiles_of(s.k->grid.nx) * tiles_of(s.k->grid.ny);
    s.bytes = carve(s, s.kind, *s.k, s.n, prune_wanted(s.opts), mem);
    s.block = mem;
}

namespace {
int reset_list(const ListSet &l, const Solve &s, hipStream_t st) {
    const size_t nt = s.k->grid.ntheta;
    int rc = SE2_OK;
    if (l.len) rc = launch_fill_i32(l.len, static_cast<size_t>(s.tiles) * nt, -1, st);
    if (rc == SE2_OK && l.dense_flag) rc = launch_fill_i32(l.dense_flag, static_cast<size_t>(s.tiles), 0, st);
    if (rc == SE2_OK && l.work) rc = launch_fill(l.work, 2 * static_cast<size_t>(s.tiles), 0.0, st);
    return rc;
}
}  // namespace

// roctx ranges of a solve's phases, for tools that record them (rocprofv3 --marker-trace):
// "se2 bulk" (the bulk engine of a solve with polish), "se2 solve" (a solve on one engine),
// "se2 polish" (after the switch) and "se2 check" (the FP64 check and the report).  Each
// solve has at most one range open; opening the next closes it.
static void trace_phase(Solve &s, const char *name) {
    if (s.trace_range != 0) roctxRangeStop(s.trace_range);
    s.trace_range = name ? roctxRangeStartA(name) : 0;
}

int solve_reset_lists(Solve &s, hipStream_t st) {
    int rc = SE2_OK;
    trace_phase(s, s.opts.polish ? "se2 bulk" : "se2 solve");
    s.phase = 0;
    s.phase_switch_iter = -1;
    s.prev_err = -1.0;
    s.fb_checked = -1.0;
    s.fb_prev = 0.0;
    s.fb_prev_iter = 0;
    s.terms_linear = 0.0;
    if (s.fb_count && (rc = launch_fill_i32(s.fb_count, ot_like(s) ? 1 : static_cast<size_t>(s.n), 0, st)))
        return rc;
    if (ot_like(s)) {
        if ((rc = reset_list(s.ls_phi, s, st))) return rc;
        return reset_list(s.ls_psi, s, st);
    }
    for (int i = 0; i < s.n; ++i) {
        if ((rc = reset_list(s.ls_v[i], s, st))) return rc;
        if ((rc = reset_list(s.ls_w[i], s, st))) return rc;
    }
    return rc;
}

int eps_schedule(const se2_opts_t &o, double eps, std::vector<double> &out) {
    out.clear();
    if (!(o.eps_start > eps)) {
        out.push_back(eps);
        return SE2_OK;
    }
    if (!std::isfinite(o.eps_start) || !(o.eps_factor > 0.0 && o.eps_factor < 1.0) || o.stage_iters < 1)
        return SE2_EINVAL;
    for (double e = o.eps_start; e > eps * (1.0 + 1e-12); e *= o.eps_factor) {
        if (out.size() >= 32) return SE2_EINVAL;
        out.push_back(e);
    }
    if (static_cast<long long>(out.size()) * o.stage_iters >= o.max_iter) return SE2_EINVAL;
    out.push_back(eps);
    return SE2_OK;
}

int plan_stages(Solve &s, const Kernel &base) {
    int rc = eps_schedule(s.opts, base.metric.eps, s.stage_eps);
    if (rc) return rc;
    s.stage_k.assign(s.stage_eps.size(), nullptr);
    for (size_t i = 0; i < s.stage_eps.size(); ++i)
        if ((rc = kernel_at_eps(base, s.stage_eps[i], &s.stage_k[i]))) return rc;
    s.stage = 0;
    s.scaling_iters = 0;
    s.k = s.stage_k[0];
    return SE2_OK;
}

namespace {
int drop_lists(const ListSet &l, const Solve &s, hipStream_t st) {
    return l.len ? launch_fill_i32(l.len, static_cast<size_t>(s.tiles) * s.k->grid.ntheta, -1, st) : SE2_OK;
}
}  // namespace

int advance_stages(Engine &eng, const std::vector<Solve *> &solves, hipStream_t st) {
    std::vector<Solve *> moved;
    int rc;
    for (Solve *s : solves) {
        if (s->done || final_stage(*s) || s->iter < (s->stage + 1) * s->opts.stage_iters) continue;
        const double r = s->stage_eps[s->stage] / s->stage_eps[s->stage + 1];
        if (ot_like(*s)) {
            if ((rc = launch_scale(s->psi, s->psi, s->E, r, st))) return rc;
            if ((rc = drop_lists(s->ls_phi, *s, st)) || (rc = drop_lists(s->ls_psi, *s, st))) return rc;
        } else {
            for (int i = 0; i < s->n; ++i) {
                if ((rc = launch_scale(s->lv[i], s->lv[i], s->E, r, st))) return rc;
                if ((rc = drop_lists(s->ls_v[i], *s, st)) || (rc = drop_lists(s->ls_w[i], *s, st))) return rc;
            }
        }
        s->stage += 1;
        s->k = s->stage_k[s->stage];
        s->scaling_iters = s->iter;
        s->prev_err = -1.0;
        moved.push_back(s);
    }
    return moved.empty() ? SE2_OK : eng.init_first_halfstep(moved, st);
}

namespace {
bool valid_engine(int prec, const Kernel &k) {
    switch (prec) {
        case SE2_F32:
        case SE2_F64:
            return true;
        case SE2_BF16:
            return lin_supported(k.grid.ntheta, true);
        case SE2_F32_MFMA:
            return lin_supported(k.grid.ntheta, false) && k.d_Fpack != nullptr;
        default:
            return false;
    }
}
}  // namespace

bool valid_solver_opts(const se2_opts_t &o, const Kernel &k) {
    if (!(o.max_iter >= 1 && o.check_every >= 1 && !std::isnan(o.tol_marg_l1) && !std::isnan(o.eps_start)))
        return false;
    if (!valid_engine(o.prec, k)) return false;
    if (o.polish != 0 && o.polish != 1) return false;
    if (o.polish && (!valid_engine(o.bulk, k) || std::isnan(o.switch_tol))) return false;
    std::vector<double> sched;
    return eps_schedule(o, k.metric.eps, sched) == SE2_OK;
}

void phase_after_check(Solve &s, double err) {
    if (in_bulk_phase(s)) {
        bool to_polish = false;
        // (a) the share of the bulk engine's groups that fell back since the previous check:
        // each iteration visits every (tile, orientation) group of every measure twice
        const int its = s.iter - s.fb_prev_iter;
        if (s.fb_checked >= 0.0 && its > 0) {
            const double groups = 2.0 * its * s.tiles * s.k->grid.ntheta * (ot_like(s) ? 1 : s.n);
            const bool pruned = s.opts.prune && conv_lse_sparse_fits(s.k->grid.ntheta, s.k->metric.radius);
            const double cap = pruned ? kBulkFallbackMaxPruned : kBulkFallbackMaxDense;
            to_polish = (s.fb_checked - s.fb_prev) > cap * groups;
            s.fb_prev = s.fb_checked;
            s.fb_prev_iter = s.iter;
        }
        // (b) at the final eps: the tolerance or the bulk engine's noise floor
        if (final_stage(s)) {
            const bool stalled = s.prev_err >= 0.0 && !(err < s.prev_err);
            to_polish = to_polish || err <= s.opts.switch_tol || stalled;
        }
        if (to_polish) {
            s.phase = 1;
            s.phase_switch_iter = s.iter;
            trace_phase(s, "se2 polish");
        }
    }
    s.prev_err = err;
}

int solve_setup_ot(Solve &s, const double *mu, const double *nu, const double *init_g, hipStream_t st) {
    s.mu_lin = mu;
    s.nu_lin = nu;
    int rc;
    if ((rc = launch_log2_measure(mu, s.lmu, s.E, st))) return rc;
    if ((rc = launch_log2_measure(nu, s.lnu, s.E, st))) return rc;
    // g/eps (natural) -> base-2 units: multiply by log2(e)
    if (init_g) {
        if ((rc = launch_scale(init_g, s.psi, s.E, kLog2e, st))) return rc;
    } else if ((rc = launch_fill(s.psi, s.E, 0.0, st))) {
        return rc;
    }
    if ((rc = solve_reset_lists(s, st))) return rc;
    std::vector<int32_t> off = {0, s.tiles * s.k->grid.ntheta};
    SE2_HIP(hipMemcpyAsync(s.offsets, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    SE2_HIP(hipStreamSynchronize(st));  // `off` is a host temporary
    s.cur = 0;
    s.iter = 0;
    s.done = false;
    return SE2_OK;
}

int solve_setup_jko(Solve &s, const double *mu, const double *init, double init_scale, hipStream_t st) {
    s.mu_lin = mu;
    int rc;
    if ((rc = launch_log2_measure(mu, s.lmu, s.E, st))) return rc;
    if (init) {
        if ((rc = launch_scale(init, s.psi, s.E, init_scale, st))) return rc;
    } else if ((rc = launch_fill(s.psi, s.E, 0.0, st))) {
        return rc;
    }
    if ((rc = solve_reset_lists(s, st))) return rc;
    const int32_t off[2] = {0, s.tiles * s.k->grid.ntheta};
    SE2_HIP(hipMemcpyAsync(s.offsets, off, sizeof(off), hipMemcpyHostToDevice, st));
    SE2_HIP(hipStreamSynchronize(st));  // `off` is a host temporary
    s.cur = 0;
    s.iter = 0;
    s.done = false;
    return SE2_OK;
}

int solve_setup_bary(Solve &s, const std::vector<const double *> &mus, hipStream_t st) {
    int rc;
    s.m_lin = mus;
    for (int i = 0; i < s.n; ++i) {
        if ((rc = launch_log2_measure(mus[i], s.lm[i], s.E, st))) return rc;
        if ((rc = launch_fill(s.lv[i], s.E, 0.0, st))) return rc;
    }
    if ((rc = solve_reset_lists(s, st))) return rc;
    std::vector<int32_t> off(s.n + 1);
    for (int i = 0; i <= s.n; ++i) off[i] = i * s.tiles * s.k->grid.ntheta;
    SE2_HIP(hipMemcpyAsync(s.offsets, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    SE2_HIP(hipMemcpyAsync(s.d_lv, s.lv.data(), s.n * sizeof(double *), hipMemcpyHostToDevice, st));
    SE2_HIP(hipMemcpyAsync(s.d_ld, s.ld.data(), s.n * sizeof(double *), hipMemcpyHostToDevice, st));
    SE2_HIP(hipMemcpyAsync(s.d_lw, s.lw.data(), s.n * sizeof(double *), hipMemcpyHostToDevice, st));
    const int nb = plan_parts(*s.k);
    std::vector<SumItem> items(2 * static_cast<size_t>(s.n));
    for (int j = 0; j < 2 * s.n; ++j) items[j] = SumItem{s.partial, j * nb, (j + 1) * nb};
    SE2_HIP(hipMemcpyAsync(s.d_cost_items, items.data(), items.size() * sizeof(SumItem), hipMemcpyHostToDevice, st));
    SE2_HIP(hipMemcpyAsync(s.d_lam, s.lam.data(), s.n * sizeof(double), hipMemcpyHostToDevice, st));
    SE2_HIP(hipStreamSynchronize(st));  // the host vectors are read by the copies
    s.iter = 0;
    s.done = false;
    return SE2_OK;
}

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------

Engine::Engine() {}

void Engine::set_profiling(bool on, hipEvent_t ref) {
    prof_ = on;
    prof_ref_ = ref;
    prof_seconds = prof_terms = prof_outputs = 0.0;
    prof_launches = 0;
    prof_intervals.clear();
}

int Engine::collect_profile() { return fold_profile(pending_.size(), true); }

int Engine::fold_profile(size_t count, bool wait) {
    if (count > pending_.size()) count = pending_.size();
    for (size_t i = 0; i < count; ++i) {
        Pending &p = pending_[i];
        if (wait) SE2_HIP(hipEventSynchronize(p.b));
        float t0 = 0.0f, t1 = 0.0f;
        if (prof_ref_) {
            SE2_HIP(hipEventElapsedTime(&t0, prof_ref_, p.a));
            SE2_HIP(hipEventElapsedTime(&t1, prof_ref_, p.b));
            prof_intervals.emplace_back(t0, t1);
        } else {
            SE2_HIP(hipEventElapsedTime(&t1, p.a, p.b));
        }
        prof_seconds += 1e-3 * static_cast<double>(t1 - t0);
        prof_terms += p.terms;
        prof_outputs += p.outputs;
        prof_launches += 1;
        spare_.push_back(p.a);
        spare_.push_back(p.b);
    }
    pending_.erase(pending_.begin(), pending_.begin() + static_cast<std::ptrdiff_t>(count));
    prof_ready_ = prof_ready_ > count ? prof_ready_ - count : 0;
    return SE2_OK;
}

Engine::~Engine() {
    if (d_fb_) (void)hipFree(d_fb_);
    if (d_fb_count_) (void)hipFree(d_fb_count_);
    if (d_rebuild_) (void)hipFree(d_rebuild_);
    if (d_rebuild_count_) (void)hipFree(d_rebuild_count_);
    for (Pending &p : pending_) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : spare_) (void)hipEventDestroy(e);
    for (TableSlot &t : tables_) {
        if (t.d_jobs) (void)hipFree(t.d_jobs);
        if (t.d_map) (void)hipFree(t.d_map);
    }
    if (h_jobs_) (void)hipHostFree(h_jobs_);
    if (h_map_) (void)hipHostFree(h_map_);
    if (h_chk_) (void)hipHostFree(h_chk_);
    if (h_published_) (void)hipHostFree(h_published_);
    if (h_items_) (void)hipHostFree(h_items_);
    if (d_items_) (void)hipFree(d_items_);
    if (d_errs_) (void)hipFree(d_errs_);
    for (auto &e : staged_)
        if (e) (void)hipEventDestroy(e);
}

int Engine::ensure(size_t njobs, size_t nblocks) {
    if (!staged_[0]) {
        SE2_HIP(hipEventCreateWithFlags(&staged_[0], hipEventDisableTiming));
        SE2_HIP(hipEventCreateWithFlags(&staged_[1], hipEventDisableTiming));
    }
    if (njobs > cap_jobs_ || nblocks > cap_blocks_) {
        // wait until both staging halves are free before reallocating
        SE2_HIP(hipEventSynchronize(staged_[0]));
        SE2_HIP(hipEventSynchronize(staged_[1]));
        size_t nj = njobs > cap_jobs_ ? njobs * 2 : cap_jobs_;
        size_t nb = nblocks > cap_blocks_ ? nblocks * 2 : cap_blocks_;
        if (h_jobs_) SE2_HIP(hipHostFree(h_jobs_));
        if (h_map_) SE2_HIP(hipHostFree(h_map_));
        SE2_HIP(hipHostMalloc(&h_jobs_, 2 * nj * sizeof(ConvJob), hipHostMallocDefault));
        SE2_HIP(hipHostMalloc(&h_map_, 2 * nb * sizeof(int32_t), hipHostMallocDefault));
        cap_jobs_ = nj;
        cap_blocks_ = nb;
    }
    return SE2_OK;
}

bool debug_checks() {
    static const bool on = [] {
        const char *v = std::getenv("SE2_DEBUG");
        return v != nullptr && v[0] != '\0' && std::strcmp(v, "0") != 0;
    }();
    return on;
}

namespace {

int job_error(size_t q, const char *what) {
    set_last_error(std::string("debug check of a launch, job ") + std::to_string(q) + ": " + what);
    return SE2_EINVAL;
}

}  // namespace

int check_jobs(const std::vector<ConvJob> &jobs, int nblocks, int nt, int R_max, LaunchKind kind, int rpw) {
    const bool sparse = kind == LK_SPARSE;
    const bool lin = kind == LK_LIN_BF16 || kind == LK_LIN_F32;
    if (nt != 8 && nt != 16 && nt != 32) return job_error(0, "ntheta of the launch");
    if (R_max < 0 || R_max > kMaxRadius) return job_error(0, "window radius of the launch");
    if (sparse && !conv_lse_sparse_fits(nt, R_max)) return job_error(0, "sparse halo does not fit the LDS");
    int next = 0;
    for (size_t q = 0; q < jobs.size(); ++q) {
        const ConvJob &j = jobs[q];
        if (!j.in || !j.L64) return job_error(q, "null input or kernel table");
        // an FP64 check writes no output: only the error partials against `old`
        if (!j.out && !(kind == LK_F64 && j.epi == EPI_SCALE && j.old && j.partial))
            return job_error(q, "null output");
        if (j.in == j.out) return job_error(q, "output aliases the input (other tiles read its halo)");
        if (j.nx < 1 || j.ny < 1) return job_error(q, "empty grid");
        if (j.R < 0 || j.R > R_max || (lin && j.R != R_max)) return job_error(q, "job radius outside the launch's");
        const int tx = (j.nx + kTile - 1) / kTile, ty = (j.ny + kTile - 1) / kTile;
        if (j.tiles_x != tx || j.tiles != tx * ty) return job_error(q, "tile counts do not match the grid");
        const int want = lin ? lin_blocks(j.nx, j.ny, rpw) : j.tiles;
        if (j.blocks != want || j.first_block != next) return job_error(q, "block range of the job");
        next += j.blocks;
        if (j.epi != EPI_RAW && j.epi != EPI_SCALE && j.epi != EPI_ADD) return job_error(q, "epilogue kind");
        if (j.epi != EPI_RAW && !j.aux) return job_error(q, "epilogue operand missing");
        if (sparse && (!j.lists || !j.ref || !j.len || !j.mref || !j.L32 || j.lmax != kListMax))
            return job_error(q, "pruning state of a sparse job");
        if (lin && !j.kop) return job_error(q, "packed kernel of a matrix-core job");
    }
    if (next != nblocks) return job_error(jobs.size(), "blocks of the launch");
    return SE2_OK;
}

int Engine::stage_and_launch(std::vector<ConvJob> &jobs, int nblocks, int nt, int R_max, LaunchKind kind, int rpw,
                             hipStream_t st) {
    const bool sparse = kind == LK_SPARSE, f64 = kind == LK_F64;
    const bool lin = kind == LK_LIN_BF16 || kind == LK_LIN_F32;
    const size_t nj = jobs.size();
    if (debug_checks()) {
        const int rc = check_jobs(jobs, nblocks, nt, R_max, kind, rpw);
        if (rc) return rc;
    }
    TableSlot *t = nullptr;
    for (TableSlot &c : tables_)
        if (c.key.size() == nj && std::memcmp(c.key.data(), jobs.data(), nj * sizeof(ConvJob)) == 0) {
            t = &c;
            break;
        }
    if (!t) {
        // least recently used slot; no launch still in flight may read it when it is rewritten
        t = &tables_[0];
        for (TableSlot &c : tables_)
            if (c.last < t->last) t = &c;
        if (t->last > drained_) {
            const int rc = sync(st);
            if (rc) return rc;
        }
        if (nj > t->cap_jobs || static_cast<size_t>(nblocks) > t->cap_blocks) {
            if (t->d_jobs) SE2_HIP(hipFree(t->d_jobs));
            if (t->d_map) SE2_HIP(hipFree(t->d_map));
            t->cap_jobs = nj * 2;
            t->cap_blocks = static_cast<size_t>(nblocks) * 2;
            SE2_HIP(hipMalloc(&t->d_jobs, t->cap_jobs * sizeof(ConvJob)));
            SE2_HIP(hipMalloc(&t->d_map, t->cap_blocks * sizeof(int32_t)));
        }
        int rc = ensure(nj, nblocks);
        if (rc) return rc;
        const int h = flip_;
        flip_ ^= 1;
        SE2_HIP(hipEventSynchronize(staged_[h]));  // the copy that last read this half is done
        ConvJob *hj = h_jobs_ + h * cap_jobs_;
        int32_t *hm = h_map_ + h * cap_blocks_;
        std::memcpy(hj, jobs.data(), nj * sizeof(ConvJob));
        for (size_t q = 0; q < nj; ++q)
            for (int b = 0; b < jobs[q].blocks; ++b) hm[jobs[q].first_block + b] = static_cast<int32_t>(q);
        SE2_HIP(hipMemcpyAsync(t->d_jobs, hj, nj * sizeof(ConvJob), hipMemcpyHostToDevice, st));
        SE2_HIP(hipMemcpyAsync(t->d_map, hm, static_cast<size_t>(nblocks) * sizeof(int32_t), hipMemcpyHostToDevice,
                               st));
        SE2_HIP(hipEventRecord(staged_[h], st));
        t->key = jobs;
    }
    t->last = ++clock_;
    if (sparse && static_cast<size_t>(nblocks) > cap_rebuild_) {
        // stream order: earlier launches that used the old buffers finish before it is freed
        const int rs = sync(st);
        if (rs) return rs;
        if (d_rebuild_) SE2_HIP(hipFree(d_rebuild_));
        if (!d_rebuild_count_) {
            // two counters used alternately: each sparse launch zeroes the other one
            SE2_HIP(hipMalloc(&d_rebuild_count_, 2 * sizeof(int)));
            SE2_HIP(hipMemsetAsync(d_rebuild_count_, 0, 2 * sizeof(int), st));
        }
        if (!h_published_) {
            // rebuild item counts the kernels publish, one per ntheta class; until the first
            // count arrives the narrow rebuild (suited to many items) is used
            SE2_HIP(hipHostMalloc(reinterpret_cast<void **>(&h_published_), 3 * sizeof(int), hipHostMallocCoherent));
            for (int c = 0; c < 3; ++c) h_published_[c] = INT_MAX;
            SE2_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&d_published_), h_published_, 0));
        }
        cap_rebuild_ = static_cast<size_t>(nblocks) * 2;
        SE2_HIP(hipMalloc(&d_rebuild_, cap_rebuild_ * sizeof(int2)));
    }
    size_t cap_tiles = 0;  // 8 x 8 tiles of a matrix-core launch: the capacity of its fallback list
    if (lin)
        for (const ConvJob &j : jobs) cap_tiles += static_cast<size_t>(j.tiles);
    if (lin && cap_tiles > cap_fb_) {
        const int rs = sync(st);  // earlier launches that used the old list are done
        if (rs) return rs;
        if (d_fb_) SE2_HIP(hipFree(d_fb_));
        if (!d_fb_count_) {
            SE2_HIP(hipMalloc(&d_fb_count_, 2 * sizeof(int)));
            SE2_HIP(hipMemsetAsync(d_fb_count_, 0, 2 * sizeof(int), st));
        }
        cap_fb_ = cap_tiles * 2;
        SE2_HIP(hipMalloc(&d_fb_, cap_fb_ * sizeof(int4)));
    }
    int rc;
    if (lin) {
        int *cnt = d_fb_count_ + fb_flip_, *next = d_fb_count_ + (1 - fb_flip_);
        fb_flip_ ^= 1;
        const int fb_grid = cap_tiles < 1024 ? static_cast<int>(cap_tiles) : 1024;
        rc = launch_conv_lin_log(t->d_jobs, nblocks, t->d_map, nt, R_max, rpw, kind == LK_LIN_BF16, d_fb_, cnt, next,
                                 fb_grid, st);
    } else if (!sparse) {
        rc = launch_conv_lse(t->d_jobs, static_cast<int>(nj), nblocks, t->d_map, nt, R_max, f64, false, nullptr, nullptr,
                             nullptr, 8, nullptr, st);
    } else {
        int *cnt = d_rebuild_count_ + rc_flip_, *next = d_rebuild_count_ + (1 - rc_flip_);
        rc_flip_ ^= 1;
        // rebuild width from the last count this class published (written by the GPU
        // asynchronously: a value some launches old; the results do not depend on it)
        const int cls = nt == 8 ? 0 : (nt == 16 ? 1 : 2);
        const int last = *reinterpret_cast<volatile int *>(h_published_ + cls);
        const int rb_waves = (wide_rebuild_ && last <= kRebuildWideItems) ? 16 : 8;
        rc = launch_conv_lse(t->d_jobs, static_cast<int>(nj), nblocks, t->d_map, nt, R_max, f64, true, d_rebuild_, cnt,
                             next, rb_waves, d_published_ + cls, st);
    }
    if (rc == SE2_OK && debug_checks()) {
        // debug: every launch completes (or reports its failure) before the next is issued
        SE2_HIP(hipStreamSynchronize(st));
        SE2_HIP(hipGetLastError());
        drained_ = clock_;
    }
    return rc;
}

LaunchEvents *&launch_events() {
    thread_local LaunchEvents *current = nullptr;
    return current;
}

namespace {

// Installs a LaunchEvents for the launches of one profiled group (no-op when `on` is false)
// and restores the previous one on exit.
class EventScope {
public:
    EventScope(bool on, hipEvent_t start) : on_(on), prev_(launch_events()) {
        if (!on_) return;
        ev_.start = start;
        launch_events() = &ev_;
    }
    ~EventScope() {
        if (on_) launch_events() = prev_;
    }
    EventScope(const EventScope &) = delete;
    EventScope &operator=(const EventScope &) = delete;
    void arm_stop(hipEvent_t stop) {
        if (on_) ev_.stop = stop;
    }
    int finish(hipStream_t st) {
        if (ev_.start) SE2_HIP(hipEventRecord(ev_.start, st));
        if (ev_.stop) SE2_HIP(hipEventRecord(ev_.stop, st));
        ev_.start = ev_.stop = nullptr;
        return SE2_OK;
    }

private:
    bool on_;
    LaunchEvents *prev_;
    LaunchEvents ev_;
};

}  // namespace

int Engine::sync(hipStream_t st) {
    SE2_HIP(hipStreamSynchronize(st));
    drained_ = clock_;
    return SE2_OK;
}

int Engine::launch_stage(const std::vector<Solve *> &solves, int stage, bool with_err, hipStream_t st) {
    // group jobs by ntheta (the kernels are specialised on it) and by engine: dense FP32,
    // pruned (certified sparse kernel and its rebuild), dense FP64, and the matrix-core engines
    // (bfloat16 or FP32 operands, per window radius)
    static const int kClasses[3] = {8, 16, 32};
    for (int nt : kClasses) {
        std::vector<ConvJob> jobs[3];
        int nblocks[3] = {0, 0, 0};
        int R_max = 0;
        bool present = false;
        // matrix-core jobs, by (bfloat16?, rows per wave, window radius): their tiling is specialised on all three
        std::vector<std::pair<std::pair<int, int>, std::vector<ConvJob>>> lin;
        for (Solve *s : solves) {
            if (s->k->grid.ntheta != nt) continue;
            present = true;
            const Kernel &k = *s->k;
            const int ep = engine_prec(*s);
            ConvJob base{};
            base.L64 = k.d_L64;
            base.L32 = k.d_L32;
            base.nx = k.grid.nx;
            base.ny = k.grid.ny;
            base.R = k.metric.radius;
            base.tiles_x = tiles_of(k.grid.nx);
            base.tiles = s->tiles;
            base.lmax = kListMax;
            auto attach = [&](ConvJob &j, const ListSet &l) {
                j.lists = l.lists;
                j.ref = l.ref;
                j.len = l.len;
                j.mref = l.mref;
                j.dense_flag = l.dense_flag;
                j.work = l.work;
            };
            const bool f64 = ep == SE2_F64;
            const bool is_lin = linear_engine(ep);
            auto push = [&](ConvJob &j) {
                if (is_lin) {
                    // the whole window on the matrix cores: no lists; the exact recomputation of
                    // rejected groups adds to the dense work counter and to the solve's fallbacks
                    j.lists = nullptr;
                    j.ref = nullptr;
                    j.len = nullptr;
                    j.mref = nullptr;
                    j.kop = ep == SE2_BF16 ? static_cast<const void *>(k.d_Bpack) : static_cast<const void *>(k.d_Fpack);
                    // key: (bfloat16?, radius, rows per wave)
                    const int rpw = lin_rows_per_wave(nt, ep == SE2_BF16, k.grid.ny);
                    const std::pair<int, int> key((ep == SE2_BF16 ? 1 : 0) + 2 * rpw, k.metric.radius);
                    size_t g = 0;
                    while (g < lin.size() && lin[g].first != key) ++g;
                    if (g == lin.size()) lin.emplace_back(key, std::vector<ConvJob>());
                    lin[g].second.push_back(j);
                    s->terms_linear += conv_terms(k);
                    return;
                }
                const int g = f64 ? 2 : (j.lists != nullptr ? 1 : 0);
                if (j.R > R_max) R_max = j.R;
                j.first_block = nblocks[g];
                j.blocks = j.tiles;
                nblocks[g] += j.tiles;
                jobs[g].push_back(j);
            };
            if (ot_like(*s)) {
                ConvJob j = base;
                j.fallbacks = s->fb_count;
                if (stage == 0 && s->kind == kKindJKO) {  // JKO: lsum = LSE(L + phi[cur]); the prox follows
                    j.in = s->phi[s->cur];
                    j.out = s->lsum;
                    j.epi = EPI_RAW;
                    attach(j, s->ls_phi);
                } else if (stage == 0) {  // b-update: psi = log nu - LSE(L + phi[cur])
                    j.in = s->phi[s->cur];
                    j.out = s->psi;
                    j.aux = s->lnu;
                    j.epi = EPI_SCALE;
                    attach(j, s->ls_phi);
                } else {  // a-update: phi[1-cur] = log mu - LSE(L + psi)
                    j.in = s->psi;
                    j.out = s->phi[1 - s->cur];
                    j.aux = s->lmu;
                    j.epi = EPI_SCALE;
                    attach(j, s->ls_psi);
                    if (with_err) {
                        j.old = s->phi[s->cur];
                        j.partial = s->partial;
                    }
                }
                push(j);
            } else {
                for (int i = 0; i < s->n; ++i) {
                    ConvJob j = base;
                    j.fallbacks = s->fb_count + i;
                    if (stage == 0) {  // d-update: ld_i = lv_i + LSE(L + lw_i)
                        j.in = s->lw[i];
                        j.out = s->ld[i];
                        j.aux = s->lv[i];
                        j.epi = EPI_ADD;
                        attach(j, s->ls_w[i]);
                    } else {  // w-update: lw_i = log mu_i - LSE(L + lv_i)
                        j.in = s->lv[i];
                        j.out = s->lw[i];
                        j.aux = s->lm[i];
                        j.epi = EPI_SCALE;
                        attach(j, s->ls_v[i]);
                        if (with_err) {
                            j.old = s->lw[i];
                            j.partial = s->partial + static_cast<size_t>(i) * s->tiles * s->k->grid.ntheta;
                        }
                    }
                    push(j);
                }
            }
        }
        if (!present) continue;
        Pending pe{};
        if (prof_) {
            for (int q = 0; q < 2; ++q) {
                hipEvent_t e = nullptr;
                if (!spare_.empty()) {
                    e = spare_.back();
                    spare_.pop_back();
                } else {
                    // timing only: a device-scope release (no system-scope cache writeback)
                    SE2_HIP(hipEventCreateWithFlags(&e, hipEventReleaseToDevice));
                }
                (q == 0 ? pe.a : pe.b) = e;
            }
            for (Solve *s : solves) {
                if (s->k->grid.ntheta != nt) continue;
                const double c = ot_like(*s) ? 1.0 : s->n;
                pe.terms += c * conv_terms(*s->k);
                pe.outputs += c * static_cast<double>(s->E);
            }
        }
        // the first kernel of the group takes pe.a as its start time and the last kernel of
        // the last launcher takes pe.b as its end time: no marker packets between half-steps
        EventScope scope(prof_, pe.a);
        int calls_left = static_cast<int>(lin.size());
        for (int g = 0; g < 3; ++g) calls_left += jobs[g].empty() ? 0 : 1;
        for (int g = 0; g < 3; ++g) {
            if (jobs[g].empty()) continue;
            const LaunchKind kind = g == 1 ? LK_SPARSE : (g == 2 ? LK_F64 : LK_DENSE);
            if (--calls_left == 0) scope.arm_stop(pe.b);
            const int rc = stage_and_launch(jobs[g], nblocks[g], nt, R_max, kind, 0, st);
            if (rc) return rc;
        }
        for (auto &grp : lin) {
            const bool bf16 = (grp.first.first & 1) != 0;
            const int rpw = grp.first.first >> 1;
            const int R = grp.first.second;
            std::vector<ConvJob> &js = grp.second;
            int nb = 0;
            for (ConvJob &j : js) {
                j.first_block = nb;
                j.blocks = lin_blocks(j.nx, j.ny, rpw);
                nb += j.blocks;
            }
            if (--calls_left == 0) scope.arm_stop(pe.b);
            const int rc = stage_and_launch(js, nb, nt, R, bf16 ? LK_LIN_BF16 : LK_LIN_F32, rpw, st);
            if (rc) return rc;
        }
        if (prof_) {
            const int rc = scope.finish(st);  // events no kernel took (nothing launched) as markers
            if (rc) return rc;
            pending_.push_back(pe);
        }
        for (Solve *s : solves) s->convs += (s->k->grid.ntheta == nt) ? (ot_like(*s) ? 1 : s->n) : 0;
    }
    return SE2_OK;
}

int Engine::init_first_halfstep(const std::vector<Solve *> &solves, hipStream_t st) {
    const int rc = launch_stage(solves, 1, false, st);
    if (rc) return rc;
    // the first a-update wrote phi[1 - cur]: that is the current a-potential now
    for (Solve *s : solves)
        if (ot_like(*s)) s->cur ^= 1;
    return SE2_OK;
}

int Engine::step(const std::vector<Solve *> &solves, bool check, hipStream_t st) {
    const int rc = step_half(solves, 0, false, st);
    return rc ? rc : step_half(solves, 1, check, st);
}

int Engine::step_half(const std::vector<Solve *> &solves, int half, bool check, hipStream_t st) {
    int rc;
    if (half == 1) {
        rc = launch_stage(solves, 1, check, st);
        if (rc) return rc;
        for (Solve *s : solves) {
            s->iter += 1;
            if (!check && ot_like(*s)) s->cur ^= 1;  // the new a-potential becomes current
        }
        return check ? sum_errors(solves, st) : SE2_OK;
    }
    rc = launch_stage(solves, 0, false, st);
    if (rc) return rc;
    for (Solve *s : solves) {
        if (s->kind == kKindJKO) {
            // b = prox(K^T a) / K^T a
            if ((rc = launch_porous_prox(s->lsum, s->psi, s->E, s->jko_c, s->jko_m, st))) return rc;
            continue;
        }
        if (s->kind != SE2_REQ_BARYCENTER) continue;
        rc = launch_ibp_combine(s->d_lv, s->d_ld, s->d_lam, s->n, s->E, s->combine_part, s->logbar, st);
        if (rc) return rc;
    }
    return SE2_OK;
}

int Engine::sum_errors(const std::vector<Solve *> &solves, hipStream_t st) {
    std::vector<SumItem> items;
    for (Solve *s : solves) {
        const int nj = ot_like(*s) ? 1 : s->n;
        const int per = s->tiles * s->k->grid.ntheta;
        for (int i = 0; i < nj; ++i) items.push_back(SumItem{s->partial, i * per, (i + 1) * per});
        // in the bulk phase also the solve's recomputed-group counters (for phase_after_check)
        if (in_bulk_phase(*s) && s->fb_count)
            items.push_back(SumItem{s->fb_count, 0, nj, 1});
    }
    const size_t n = items.size();
    const bool same = items_key_.size() == n &&
                      std::memcmp(items_key_.data(), items.data(), n * sizeof(SumItem)) == 0;
    if (!same) {
        if (items_last_ > drained_) {  // no copy or sum in flight may use the table
            const int rs = sync(st);
            if (rs) return rs;
        }
        if (n > cap_items_) {
            if (h_items_) SE2_HIP(hipHostFree(h_items_));
            if (d_items_) SE2_HIP(hipFree(d_items_));
            if (d_errs_) SE2_HIP(hipFree(d_errs_));
            cap_items_ = n * 2;
            SE2_HIP(hipHostMalloc(&h_items_, cap_items_ * sizeof(SumItem), hipHostMallocDefault));
            SE2_HIP(hipMalloc(&d_items_, cap_items_ * sizeof(SumItem)));
            SE2_HIP(hipMalloc(&d_errs_, cap_items_ * sizeof(double)));
        }
        std::memcpy(h_items_, items.data(), n * sizeof(SumItem));
        SE2_HIP(hipMemcpyAsync(d_items_, h_items_, n * sizeof(SumItem), hipMemcpyHostToDevice, st));
        items_key_ = items;
    }
    items_last_ = ++clock_;
    return launch_sum_items(d_items_, static_cast<int>(n), d_errs_, st);
}

int Engine::read_errors(const std::vector<Solve *> &solves, std::vector<double> &max_err, hipStream_t st) {
    // the errors of the last check, in the item order of sum_errors()
    size_t total = 0;
    for (Solve *s : solves) total += (ot_like(*s) ? 1 : s->n) + ((in_bulk_phase(*s) && s->fb_count) ? 1 : 0);
    if (total != items_key_.size() || !d_errs_) return SE2_EINVAL;
    if (total > cap_err_) {
        // coherent pinned memory the GPU writes directly: the flag word in its own 256 bytes,
        // then the errors
        if (h_chk_) {
            const int rs = sync(st);
            if (rs) return rs;
            SE2_HIP(hipHostFree(h_chk_));
            h_chk_ = nullptr;
        }
        const size_t bytes = kChkHeader + total * 2 * sizeof(double);
        SE2_HIP(hipHostMalloc(reinterpret_cast<void **>(&h_chk_), bytes, hipHostMallocCoherent));
        std::memset(h_chk_, 0, bytes);
        SE2_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&d_chk_), h_chk_, 0));
        cap_err_ = total * 2;
    }
    int *flag = reinterpret_cast<int *>(h_chk_);
    const double *h_err = reinterpret_cast<const double *>(h_chk_ + kChkHeader);
    chk_seq_ = chk_seq_ == INT_MAX ? 1 : chk_seq_ + 1;  // never 0, the word's initial value
    const int seq = chk_seq_;
    int rc = launch_publish(d_errs_, static_cast<int>(total), reinterpret_cast<double *>(d_chk_ + kChkHeader),
                            reinterpret_cast<int *>(d_chk_), seq, st);
    if (rc) return rc;
    // while the queued iterations run: fold the timing events known to be complete (those
    // recorded before the previous check's results arrived)
    if (prof_ && (rc = fold_profile(prof_ready_, false))) return rc;
    // Poll the flag (a lane waits here for the queued iterations to finish; polling answers
    // within a microsecond where a blocking synchronisation takes tens).  After kCheckPollMs
    // the wait blocks in hipStreamSynchronize, which also reports a failed launch.
    const auto t0 = std::chrono::steady_clock::now();
    for (int spins = 0; *reinterpret_cast<volatile int *>(flag) != seq; ++spins) {
        if ((spins & 255) == 255) {
            if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(kCheckPollMs)) {
                const int rs = sync(st);
                if (rs) return rs;
                if (*reinterpret_cast<volatile int *>(flag) != seq) {
                    set_last_error("the check results did not arrive although the stream drained");
                    return SE2_EHIP;
                }
                break;
            }
            std::this_thread::yield();
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    prof_ready_ = pending_.size();  // everything recorded before the results is complete
    max_err.assign(solves.size(), 0.0);
    size_t off = 0;
    for (size_t q = 0; q < solves.size(); ++q) {
        Solve &s = *solves[q];
        const size_t c = ot_like(s) ? 1 : s.n;
        double m = 0.0;
        for (size_t i = 0; i < c; ++i) {
            const double e = h_err[off + i];
            if (!(e <= m)) m = e;  // NaN propagates
        }
        max_err[q] = m;
        off += c;
        if (in_bulk_phase(s) && s.fb_count) s.fb_checked = h_err[off++];
    }
    return SE2_OK;
}

// ---------------------------------------------------------------------------
// finishing
// ---------------------------------------------------------------------------

namespace {

// FP64 re-check of one marginal: aux - LSE_f64(L + in) compared with old; the output
// itself is not stored, only the error partials [tile][nt] in `partial`.
ConvJob check_job(const Kernel &k, const double *in, const double *aux, const double *old, double *partial,
                  int tiles) {
    ConvJob j{};
    j.in = in;
    j.out = nullptr;
    j.aux = aux;
    j.old = old;
    j.partial = partial;
    j.L64 = k.d_L64;
    j.L32 = k.d_L32;
    j.nx = k.grid.nx;
    j.ny = k.grid.ny;
    j.R = k.metric.radius;
    j.epi = EPI_SCALE;
    j.tiles_x = tiles_of(k.grid.nx);
    j.tiles = tiles;
    j.lmax = kListMax;
    return j;
}

// Sum of the dense and sparse term counters of a list set (host copy, synchronous).
int read_work(const ListSet &l, int tiles, double *dense, double *sparse) {
    if (!l.work) return SE2_OK;
    std::vector<double> h(2 * static_cast<size_t>(tiles));
    SE2_HIP(hipMemcpy(h.data(), l.work, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int t = 0; t < tiles; ++t) {
        *dense += h[2 * t];
        *sparse += h[2 * t + 1];
    }
    return SE2_OK;
}

}  // namespace

int Engine::launch_checks(const std::vector<ConvJob> &jobs, const std::vector<int> &nts, hipStream_t st) {
    static const int kClasses[3] = {8, 16, 32};
    for (int nt : kClasses) {
        std::vector<ConvJob> group;
        int nblocks = 0, R_max = 0;
        for (size_t q = 0; q < jobs.size(); ++q) {
            if (nts[q] != nt) continue;
            ConvJob j = jobs[q];
            j.first_block = nblocks;
            j.blocks = j.tiles;
            nblocks += j.tiles;
            if (j.R > R_max) R_max = j.R;
            group.push_back(j);
        }
        if (group.empty()) continue;
        const int rc = stage_and_launch(group, nblocks, nt, R_max, LK_F64, 0, st);
        if (rc) return rc;
    }
    return SE2_OK;
}

int finish_solves(Engine &eng, std::vector<FinishReq> &reqs, hipStream_t st) {
    // 1. every GPU step of every solve, in stream order; results land in err slots
    //    OT:  [2] cost, [3] plan mass, [4] <f, mu>, [5] <g, nu> (base 2), [6] [7] FP64 checks
    //    IBP: [2+2i] cost and [3+2i] mass of plan i, [2+2n] barycenter mass, [3+2n+i] FP64 check i
    std::vector<ConvJob> chk_a, chk_b;
    std::vector<int> nt_a, nt_b;
    for (FinishReq &q : reqs) trace_phase(*q.s, "se2 check");
    for (FinishReq &q : reqs) {
        Solve &s = *q.s;
        const Kernel &k = *s.k;
        const int nb = plan_parts(k);
        double *part = s.partial;  // scratch: >= 2 * nb + 512 doubles
        int rc = SE2_OK;
        if (ot_like(s)) {
            const double scale = k.metric.eps * kLn2;  // base-2 log-scaling -> eps * natural log
            const double *phi = s.phi[s.cur];
            if (q.f_out && (rc = launch_scale(phi, q.f_out, s.E, scale, st))) return rc;
            if (q.g_out && (rc = launch_scale(s.psi, q.g_out, s.E, scale, st))) return rc;
            if ((rc = launch_plan_tiles(k, phi, s.psi, nullptr, nullptr, 1, part, st))) return rc;
            if ((rc = launch_reduce_fixed(part, nb, 2, s.err + 2, st))) return rc;
            const int dnb = 256;
            if (s.kind == kKindJKO) {
                // the next measure nu = b K^T a and its energy F(nu)
                if (q.bary_out && (rc = launch_exp2_sum(s.psi, s.lsum, q.bary_out, s.E, st))) return rc;
                if ((rc = launch_porous_energy(s.psi, s.lsum, s.E, s.jko_m, s.jko_ref, part, dnb, st))) return rc;
                if ((rc = launch_reduce_fixed(part, dnb, 1, s.err + 4, st))) return rc;
                if (s.opts.final_check) {
                    chk_a.push_back(check_job(k, s.psi, s.lmu, phi, s.partial, s.tiles));
                    nt_a.push_back(k.grid.ntheta);
                }
                continue;
            }
            if ((rc = launch_dot_exp(phi, s.mu_lin, s.E, part, dnb, st))) return rc;
            if ((rc = launch_reduce_fixed(part, dnb, 1, s.err + 4, st))) return rc;
            if ((rc = launch_dot_exp(s.psi, s.nu_lin, s.E, part, dnb, st))) return rc;
            if ((rc = launch_reduce_fixed(part, dnb, 1, s.err + 5, st))) return rc;
            if (s.opts.final_check) {
                // first marginal: the a-update from psi against phi; second: the b-update from phi against psi
                chk_a.push_back(check_job(k, s.psi, s.lmu, phi, s.partial, s.tiles));
                nt_a.push_back(k.grid.ntheta);
                chk_b.push_back(check_job(k, phi, s.lnu, s.psi, s.partial, s.tiles));
                nt_b.push_back(k.grid.ntheta);
            }
        } else {
            if ((rc = launch_exp2_out(s.logbar, q.bary_out, s.E, st))) return rc;
            // sum_i lambda_i <pi_i, rho^2> with pi_i = diag(w_i) K diag(v_i) (first marginal exact):
            // every plan in one launch, then the cost and mass sums of each in one launch
            if ((rc = launch_plan_tiles(k, nullptr, nullptr, s.d_lw, const_cast<const double *const *>(s.d_lv), s.n,
                                        part, st)))
                return rc;
            if ((rc = launch_sum_items(s.d_cost_items, 2 * s.n, s.err + 2, st))) return rc;
            // barycenter mass (FP64 fixed-order sum, the validation reduction)
            if ((rc = launch_validate(q.bary_out, s.E, part, st))) return rc;
            SE2_HIP(hipMemcpyAsync(s.err + 2 + 2 * s.n, part, sizeof(double), hipMemcpyDeviceToDevice, st));
            if (s.opts.final_check) {
                // barycenter side of pi_i in FP64: sum bar |v_i (K*w_i) / bar - 1| (its mu_i side is
                // exact by construction of the last w-update)
                const size_t per = static_cast<size_t>(s.tiles) * k.grid.ntheta;
                for (int i = 0; i < s.n; ++i) {
                    chk_a.push_back(check_job(k, s.lw[i], s.logbar, s.lv[i], s.partial + i * per, s.tiles));
                    nt_a.push_back(k.grid.ntheta);
                }
            }
        }
    }
    // 2. FP64 checks, batched over the solves: first marginals, then second marginals
    int rc;
    if (!chk_a.empty()) {
        if ((rc = eng.launch_checks(chk_a, nt_a, st))) return rc;
        for (FinishReq &q : reqs) {
            Solve &s = *q.s;
            if (!s.opts.final_check) continue;
            const bool ot = ot_like(s);
            if ((rc = launch_sum_partials(s.partial, s.offsets, ot ? 1 : s.n, s.err + (ot ? 6 : 3 + 2 * s.n), st)))
                return rc;
        }
    }
    if (!chk_b.empty()) {
        if ((rc = eng.launch_checks(chk_b, nt_b, st))) return rc;
        for (FinishReq &q : reqs) {
            Solve &s = *q.s;
            if (!s.opts.final_check || s.kind != SE2_REQ_OT) continue;
            if ((rc = launch_sum_partials(s.partial, s.offsets, 1, s.err + 7, st))) return rc;
        }
    }
    SE2_HIP(hipStreamSynchronize(st));
    eng.mark_drained();
    // 3. reports
    for (FinishReq &q : reqs) {
        Solve &s = *q.s;
        const int nj = ot_like(s) ? 1 : s.n;
        std::vector<double> e(3 * static_cast<size_t>(nj) + 8);
        SE2_HIP(hipMemcpy(e.data(), s.err, e.size() * sizeof(double), hipMemcpyDeviceToHost));
        se2_report_t r{};
        r.status = s.status;
        r.iters = s.iter;
        r.marg_l1 = s.last_err;
        r.marg_l1_f64 = -1.0;
        r.convs = s.convs;
        r.scaling_iters = s.scaling_iters;
        r.phase_switch_iter = s.phase_switch_iter;
        r.terms_linear = s.terms_linear;
        {
            // one unsigned 32-bit device counter per measure; the total saturates the int32 field
            std::vector<uint32_t> fb(static_cast<size_t>(nj));
            SE2_HIP(hipMemcpy(fb.data(), s.fb_count, fb.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
            uint64_t total = 0;
            for (uint32_t v : fb) total += v;
            r.fallbacks = static_cast<int32_t>(std::min<uint64_t>(total, INT32_MAX));
        }
        if (s.kind == kKindJKO) {
            r.cost = e[2];
            r.mass = e[3];
            r.dual = e[4];  // F(nu) of the next measure
            if (s.opts.final_check) r.marg_l1_f64 = e[6];
            if ((rc = read_work(s.ls_phi, s.tiles, &r.terms_dense, &r.terms_sparse))) return rc;
            if ((rc = read_work(s.ls_psi, s.tiles, &r.terms_dense, &r.terms_sparse))) return rc;
        } else if (ot_like(s)) {
            r.cost = e[2];
            r.mass = e[3];
            r.dual = s.k->metric.eps * kLn2 * (e[4] + e[5]);
            if (s.opts.final_check) r.marg_l1_f64 = e[6] + e[7];
            if ((rc = read_work(s.ls_phi, s.tiles, &r.terms_dense, &r.terms_sparse))) return rc;
            if ((rc = read_work(s.ls_psi, s.tiles, &r.terms_dense, &r.terms_sparse))) return rc;
        } else {
            double cost = 0.0, worst = 0.0;
            for (int i = 0; i < s.n; ++i) {
                cost += s.lam[i] * e[2 + 2 * i];
                const double c = e[3 + 2 * s.n + i];
                if (!(c <= worst)) worst = c;
            }
            r.cost = cost;
            r.mass = e[2 + 2 * s.n];
            r.dual = 0.0;
            if (s.opts.final_check) r.marg_l1_f64 = worst;
            // every list's counters in one copy ([measure][v, w][tile][dense, sparse])
            std::vector<double> h(4 * static_cast<size_t>(s.n) * s.tiles);
            SE2_HIP(hipMemcpy(h.data(), s.work_all, h.size() * sizeof(double), hipMemcpyDeviceToHost));
            for (size_t t = 0; t < h.size(); t += 2) {
                r.terms_dense += h[t];
                r.terms_sparse += h[t + 1];
            }
        }
        r.seconds = now_seconds() - s.t_start;
        q.rc = (std::isfinite(r.cost) && std::isfinite(r.marg_l1)) ? SE2_OK : SE2_ENUMERIC;
        q.rep = r;
        trace_phase(s, nullptr);
    }
    return SE2_OK;
}

}  // namespace se2
