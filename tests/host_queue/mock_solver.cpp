// Mock executor for the host build of the serving queue (tests/test_queue_host.py): the
// solver and engine calls that csrc/queue.cpp makes, implemented on the host with a fake
// clock, so that the queue's threads, admission, bookkeeping and profiling can run under the
// thread, address and undefined-behaviour sanitizers without a GPU.
//
// A mock solve converges at iteration N = round(1 / tol_marg_l1): its error at iteration i
// is 1 / i.  Every engine step advances the fake clock (now_seconds) by one millisecond and,
// while profiling, records the step as one launch interval [t, t + 1 ms] (also appended to a
// global log the test reads to recompute the union of all lanes' intervals).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <vector>

#include "../../paper_2402_15322_amd/csrc/solver.h"

namespace mock {
std::atomic<long long> ticks{0};
std::mutex log_mu;
std::vector<std::pair<double, double>> interval_log;
}  // namespace mock

extern "C" double mock_now_ms() { return static_cast<double>(mock::ticks.load()); }
extern "C" size_t mock_interval_count() {
    std::lock_guard<std::mutex> lk(mock::log_mu);
    return mock::interval_log.size();
}
extern "C" double mock_interval_union_ms() {
    std::vector<std::pair<double, double>> iv;
    {
        std::lock_guard<std::mutex> lk(mock::log_mu);
        iv = mock::interval_log;
    }
    std::sort(iv.begin(), iv.end());
    double busy = 0.0, a = 0.0, b = -1.0;
    for (const auto &x : iv) {
        if (x.first > b) {
            if (b > a) busy += b - a;
            a = x.first;
            b = x.second;
        } else if (x.second > b) {
            b = x.second;
        }
    }
    if (b > a) busy += b - a;
    return busy;
}
extern "C" void mock_reset_log() {
    std::lock_guard<std::mutex> lk(mock::log_mu);
    mock::interval_log.clear();
}

namespace se2 {

double now_seconds() { return 1e-3 * static_cast<double>(mock::ticks.load()); }
void set_last_hip_error(hipError_t, const char *, const char *, int) {}

size_t solve_bytes(int kind, const Kernel &k, int n_active, bool) {
    const size_t E = static_cast<size_t>(k.grid.nx) * k.grid.ny * k.grid.ntheta;
    return (kind == SE2_REQ_BARYCENTER ? 4 * static_cast<size_t>(n_active) : 5) * E * sizeof(double);
}

int eps_schedule(const se2_opts_t &, double eps, std::vector<double> &out) {
    out.assign(1, eps);
    return SE2_OK;
}

int kernel_at_eps(const Kernel &base, double, const Kernel **out) {
    *out = &base;
    return SE2_OK;
}

int plan_stages(Solve &s, const Kernel &base) {
    s.stage_eps.assign(1, base.metric.eps);
    s.stage_k.assign(1, &base);
    s.stage = 0;
    s.k = &base;
    return SE2_OK;
}

bool valid_solver_opts(const se2_opts_t &o, const Kernel &) {
    return o.max_iter >= 1 && o.check_every >= 1 && !std::isnan(o.tol_marg_l1);
}

void phase_after_check(Solve &s, double err) { s.prev_err = err; }

void solve_bind(Solve &s, void *mem) {
    s.block = mem;
    s.E = static_cast<size_t>(s.k->grid.nx) * s.k->grid.ny * s.k->grid.ntheta;
}

int validate_measures(const std::vector<const double *> &, size_t, double, hipStream_t) { return SE2_OK; }

int solve_setup_ot(Solve &s, const double *, const double *, const double *, hipStream_t) {
    s.iter = 0;
    s.cur = 0;
    s.done = false;
    return SE2_OK;
}

int solve_setup_bary(Solve &s, const std::vector<const double *> &, hipStream_t) {
    s.iter = 0;
    s.done = false;
    return SE2_OK;
}

int advance_stages(Engine &, const std::vector<Solve *> &, hipStream_t) { return SE2_OK; }

Engine::Engine() {}
Engine::~Engine() {}

void Engine::set_profiling(bool on, hipEvent_t ref) {
    prof_ = on;
    prof_ref_ = ref;
    prof_seconds = prof_terms = prof_outputs = 0.0;
    prof_launches = 0;
    prof_intervals.clear();
}

int Engine::collect_profile() { return SE2_OK; }

int Engine::init_first_halfstep(const std::vector<Solve *> &, hipStream_t) { return SE2_OK; }

int Engine::step(const std::vector<Solve *> &solves, bool, hipStream_t) {
    const long long t0 = mock::ticks.fetch_add(1);
    for (Solve *s : solves) s->iter += 1;
    if (prof_) {
        const std::pair<double, double> iv(static_cast<double>(t0), static_cast<double>(t0 + 1));
        for (int half = 0; half < 2; ++half) prof_intervals.push_back(iv);  // two half-steps, same interval
        prof_terms += 100.0 * solves.size();
        prof_outputs += 10.0 * solves.size();
        std::lock_guard<std::mutex> lk(mock::log_mu);
        mock::interval_log.push_back(iv);
    }
    return SE2_OK;
}

int Engine::read_errors(const std::vector<Solve *> &solves, std::vector<double> &max_err, hipStream_t) {
    max_err.assign(solves.size(), 0.0);
    for (size_t i = 0; i < solves.size(); ++i) max_err[i] = 1.0 / static_cast<double>(solves[i]->iter);
    return SE2_OK;
}

int finish_solves(Engine &, std::vector<FinishReq> &reqs, hipStream_t) {
    for (FinishReq &q : reqs) {
        se2_report_t r{};
        r.status = q.s->status;
        r.iters = q.s->iter;
        r.marg_l1 = q.s->last_err;
        r.marg_l1_f64 = -1.0;
        r.phase_switch_iter = -1;
        q.rep = r;
        q.rc = SE2_OK;
    }
    return SE2_OK;
}

}  // namespace se2
