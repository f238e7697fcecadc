// Serving queue: admission by HBM budget, continuous batching of resident solves.
//
// The queue owns one device arena of the budget size and three lanes; a lane is a
// worker thread with its own engine and HIP stream (three streams and the caller's
// stay within the four hardware queues a process gets by default).  Each request is placed at submit
// on the lane with less outstanding work and admitted, in arrival order within its
// lane, once a slot (counted over all lanes) and enough arena memory are free; its
// inputs are copied into its slot, its potentials stay resident, and every admitted
// solve of a lane advances one iteration per step of that lane's worker (one batched
// launch per half-step and ntheta class covering the lane's solves).  The lanes run
// independently, so their launches overlap on the GPU: the dense rebuild of one lane's
// uncertified tiles, which occupies few compute units, runs beside the other lanes'
// sparse evaluation, and one lane's convergence checks do not stall the others.  A
// solve only decides to stop at its own check iterations (multiples of its
// check_every, or its max_iter), and its tiles and reductions never mix with other
// solves', so its result is bitwise the same alone, in a mix, and on any lane.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "solver.h"

namespace se2 {
namespace {

// First-fit allocator over one device block (offsets in bytes, 256-byte granules).
class Arena {
public:
    bool init(size_t bytes) {
        size_ = (bytes / 256) * 256;
        if (size_ == 0) return true;
        if (hipMalloc(&base_, size_) != hipSuccess) return false;
        free_[0] = size_;
        return true;
    }
    ~Arena() {
        if (base_) (void)hipFree(base_);
    }
    void *alloc(size_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, sz = it->second;
                free_.erase(it);
                if (sz > bytes) free_[off + bytes] = sz - bytes;
                used_[off] = bytes;
                in_use_ += bytes;
                return static_cast<char *>(base_) + off;
            }
        }
        return nullptr;
    }
    void release(void *p) {
        const size_t off = static_cast<size_t>(static_cast<char *>(p) - static_cast<char *>(base_));
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t sz = u->second;
        used_.erase(u);
        in_use_ -= sz;
        size_t o = off;
        auto nx = free_.lower_bound(o);
        if (nx != free_.end() && nx->first == o + sz) {
            sz += nx->second;
            free_.erase(nx);
        }
        auto pv = free_.lower_bound(o);
        if (pv != free_.begin()) {
            --pv;
            if (pv->first + pv->second == o) {
                o = pv->first;
                sz += pv->second;
                free_.erase(pv);
            }
        }
        free_[o] = sz;
    }
    size_t size() const { return size_; }

private:
    void *base_ = nullptr;
    size_t size_ = 0, in_use_ = 0;
    std::map<size_t, size_t> free_, used_;
};

enum ReqState { WAITING = 0, ACTIVE = 1, DONE = 2 };

struct Req {
    uint64_t ticket = 0;
    se2_request_t r{};
    std::vector<double> lambdas_all;
    std::vector<const double *> mus_all;
    Solve s;
    int state = WAITING;
    int rc = SE2_OK;
    se2_report_t rep{};
    double t_submit = 0, t_admit = 0, t_done = 0;
    size_t bytes = 0;
    void *mem = nullptr;
    std::vector<double *> inputs;  // copies in slot memory
    int lane = 0;
};

#ifndef SE2_QUEUE_LANES
#define SE2_QUEUE_LANES 3
#endif
constexpr int kLanes = SE2_QUEUE_LANES;

// Work of one request per iteration, for balancing the lanes: output elements of its
// convolutions.
double request_load(const Req &q) {
    const Kernel &k = *reinterpret_cast<const Kernel *>(q.r.kernel);
    const double E = static_cast<double>(k.grid.nx) * k.grid.ny * k.grid.ntheta;
    return E * (q.r.kind == SE2_REQ_OT ? 1.0 : static_cast<double>(q.mus_all.size()));
}

}  // namespace
}  // namespace se2

struct se2_queue_s {
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::thread worker[se2::kLanes];
    hipStream_t st[se2::kLanes] = {};
    int device = 0;
    size_t budget = 0;
    int max_slots = 1;
    se2::Arena arena;
    std::deque<se2::Req *> waiting[se2::kLanes];
    std::vector<se2::Req *> active[se2::kLanes];
    double load[se2::kLanes] = {};  // work of the lane's waiting and active requests
    std::map<uint64_t, std::unique_ptr<se2::Req>> all;
    uint64_t next_ticket = 1;
    uint64_t gen = 0;  // bumped whenever a lane may find new work (submit, finish, profile, stop)
    bool stop = false;
    int64_t admitted = 0, completed = 0, rejected = 0, peak = 0, steps = 0;
    // profiling: each lane resets its engine when it sees its flag; at checks it appends the
    // launch intervals (ms after prof_ref) that its engine collected since its last check and
    // publishes its totals.  The union of the intervals is formed only when it is asked for
    // (se2_solve_queue_kernel_time), so a check costs time in the new intervals only.
    int prof_request = 0;
    bool prof_reset[se2::kLanes] = {};
    hipEvent_t prof_ref = nullptr;
    std::vector<std::pair<double, double>> prof_iv[se2::kLanes];
    double prof_terms[se2::kLanes] = {}, prof_outputs[se2::kLanes] = {};
    int64_t prof_rounds[se2::kLanes] = {};
    se2::Engine eng[se2::kLanes];
};

namespace se2 {
namespace {

size_t request_bytes(const Req &q) {
    const Kernel &k = *reinterpret_cast<const Kernel *>(q.r.kernel);
    const size_t E = static_cast<size_t>(k.grid.nx) * k.grid.ny * k.grid.ntheta;
    const bool prune = prune_wanted(q.r.opts);
    if (q.r.kind == SE2_REQ_OT)
        return solve_bytes(SE2_REQ_OT, k, 1, prune) + 2 * ((E * sizeof(double) + 255) / 256 * 256);
    const int n = static_cast<int>(q.mus_all.size());
    int npos = 0;
    for (double l : q.lambdas_all) npos += l > 0.0;
    return solve_bytes(SE2_REQ_BARYCENTER, k, npos, prune) + n * ((E * sizeof(double) + 255) / 256 * 256);
}

// Bind slot memory, copy inputs, validate, initialise.  Worker thread, queue stream.
int admit_one(se2_queue_s *Q, Req *q) {
    const Kernel *k = reinterpret_cast<const Kernel *>(q->r.kernel);
    const size_t E = static_cast<size_t>(k->grid.nx) * k->grid.ny * k->grid.ntheta;
    const size_t in_bytes = (E * sizeof(double) + 255) / 256 * 256;
    Solve &s = q->s;
    s.kind = q->r.kind;
    s.k = k;
    s.opts = q->r.opts;
    s.opts.init_g = nullptr;
    s.t_start = now_seconds();
    int rc = plan_stages(s, *k);  // the stage kernels were built at submit: found in the cache
    if (rc) return rc;
    char *p = static_cast<char *>(q->mem);
    const int nin = q->r.kind == SE2_REQ_OT ? 2 : static_cast<int>(q->mus_all.size());
    for (int i = 0; i < nin; ++i) {
        double *dst = reinterpret_cast<double *>(p + static_cast<size_t>(i) * in_bytes);
        const double *src = q->r.kind == SE2_REQ_OT ? (i == 0 ? q->r.mu : q->r.nu) : q->mus_all[i];
        SE2_HIP(hipMemcpyAsync(dst, src, E * sizeof(double), hipMemcpyDeviceToDevice, Q->st[q->lane]));
        q->inputs.push_back(dst);
    }
    char *solve_mem = p + static_cast<size_t>(nin) * in_bytes;
    if ((rc = validate_measures(std::vector<const double *>(q->inputs.begin(), q->inputs.end()), E, 1e-9,
                                Q->st[q->lane])))
        return rc;
    if (q->r.kind == SE2_REQ_OT) {
        s.n = 1;
        solve_bind(s, solve_mem);
        return solve_setup_ot(s, q->inputs[0], q->inputs[1], nullptr, Q->st[q->lane]);
    }
    std::vector<const double *> act;
    s.lam.clear();
    for (size_t i = 0; i < q->mus_all.size(); ++i) {
        if (q->lambdas_all[i] > 0.0) {
            act.push_back(q->inputs[i]);
            s.lam.push_back(q->lambdas_all[i]);
        }
    }
    s.n = static_cast<int>(act.size());
    solve_bind(s, solve_mem);
    rc = solve_setup_bary(s, act, Q->st[q->lane]);
    return rc;
}

// Finishes a group of requests of lane l that left the iteration together: the GPU
// finishing of the successful ones is batched, then every request is marked done.
void finish_group(se2_queue_s *Q, int l, const std::vector<Req *> &done) {
    std::vector<FinishReq> fin;
    std::vector<Req *> who;
    for (Req *q : done) {
        if (q->rc != SE2_OK) continue;
        FinishReq f;
        f.s = &q->s;
        f.f_out = q->r.f_out;
        f.g_out = q->r.g_out;
        f.bary_out = q->r.bary_out;
        fin.push_back(f);
        who.push_back(q);
    }
    if (!fin.empty()) {
        const int rc = finish_solves(Q->eng[l], fin, Q->st[l]);
        for (size_t i = 0; i < fin.size(); ++i) {
            who[i]->rc = rc ? rc : fin[i].rc;
            who[i]->rep = fin[i].rep;
        }
    }
    (void)hipStreamSynchronize(Q->st[l]);
    std::lock_guard<std::mutex> lk(Q->mu);
    for (Req *q : done) {
        Q->arena.release(q->mem);
        q->mem = nullptr;
        q->t_done = now_seconds();
        q->rep.seconds = q->t_done - q->t_submit;
        q->state = DONE;
        Q->completed += 1;
        Q->load[l] -= request_load(*q);
    }
    auto &act = Q->active[l];
    act.erase(std::remove_if(act.begin(), act.end(), [](Req *q) { return q->state == DONE; }), act.end());
    Q->done_cv.notify_all();
    Q->gen += 1;
    Q->cv.notify_all();  // freed slots and memory may let the other lane admit
}

// The union of all lanes' published launch intervals, in seconds (under Q->mu).  Called by
// se2_solve_queue_kernel_time only, never on a lane's iteration path.
double union_seconds(const se2_queue_s *Q) {
    std::vector<std::pair<double, double>> iv;
    for (int l = 0; l < kLanes; ++l) iv.insert(iv.end(), Q->prof_iv[l].begin(), Q->prof_iv[l].end());
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
    return 1e-3 * busy;
}

// Requests admitted on all lanes (under Q->mu).
int active_count(const se2_queue_s *Q) {
    size_t n = 0;
    for (int l = 0; l < kLanes; ++l) n += Q->active[l].size();
    return static_cast<int>(n);
}

void lane_main(se2_queue_s *Q, int l) {
    (void)hipSetDevice(Q->device);
    Engine &eng = Q->eng[l];
    eng.set_wide_rebuild(false);  // the lanes' kernels share the GPU
    hipStream_t st = Q->st[l];
    std::vector<double> errs;
    for (;;) {
        std::vector<Req *> fresh;
        {
            std::unique_lock<std::mutex> lk(Q->mu);
            for (;;) {
                if (Q->prof_reset[l]) {
                    Q->prof_reset[l] = false;
                    (void)eng.collect_profile();
                    eng.set_profiling(Q->prof_request != 0, Q->prof_request ? Q->prof_ref : nullptr);
                    Q->prof_iv[l].clear();
                    Q->prof_terms[l] = Q->prof_outputs[l] = 0.0;
                    Q->prof_rounds[l] = 0;
                }
                if (Q->stop && Q->waiting[l].empty() && Q->active[l].empty()) return;
                // admission in arrival order within the lane: stop at the first request that does not fit
                while (!Q->waiting[l].empty() &&
                       active_count(Q) < Q->max_slots) {
                    Req *q = Q->waiting[l].front();
                    void *m = Q->arena.alloc(q->bytes);
                    if (!m) break;
                    q->mem = m;
                    q->t_admit = now_seconds();
                    q->state = ACTIVE;
                    Q->waiting[l].pop_front();
                    fresh.push_back(q);
                    Q->active[l].push_back(q);
                }
                if (!fresh.empty() || !Q->active[l].empty()) break;
                // nothing to run: sleep until a submit, a finish (freed slots or memory), a
                // profiling change or the stop
                const uint64_t g = Q->gen;
                Q->cv.wait(lk, [&] { return Q->stop || Q->gen != g; });
            }
            Q->admitted += static_cast<int64_t>(fresh.size());
            const int64_t n_act = static_cast<int64_t>(active_count(Q));
            if (n_act > Q->peak) Q->peak = n_act;
        }
        std::vector<Solve *> init;
        for (Req *q : fresh) {
            q->rc = admit_one(Q, q);
            if (q->rc == SE2_OK) init.push_back(&q->s);
        }
        if (!init.empty()) {
            const int rc = eng.init_first_halfstep(init, st);
            for (Solve *s : init) s->convs = (s->kind == SE2_REQ_OT) ? 1 : s->n;
            if (rc)
                for (Req *q : fresh) q->rc = rc;
        }
        // the lane's requests (only this worker changes its lane's active list, apart from
        // the admissions above, so a copy taken under the lock stays valid)
        std::vector<Req *> mine;
        {
            std::lock_guard<std::mutex> lk(Q->mu);
            mine = Q->active[l];
        }
        // failed admissions finish immediately
        std::vector<Req *> run, failed;
        for (Req *q : mine) {
            if (q->rc != SE2_OK) failed.push_back(q);
            else run.push_back(q);
        }
        if (!failed.empty()) finish_group(Q, l, failed);
        if (run.empty()) continue;
        // one iteration for every running solve of the lane
        std::vector<Solve *> solves;
        bool check = false;
        for (Req *q : run) {
            Solve &s = q->s;
            solves.push_back(&s);
            const int next = s.iter + 1;
            if (next % s.opts.check_every == 0 || next >= s.opts.max_iter) check = true;
        }
        int rc = eng.step(solves, check, st);
        if (rc == SE2_OK && check) rc = eng.read_errors(solves, errs, st);
        std::vector<Req *> finished;
        for (size_t i = 0; i < run.size(); ++i) {
            Req *q = run[i];
            Solve &s = q->s;
            if (rc != SE2_OK) {
                q->rc = rc;
                finished.push_back(q);
                continue;
            }
            if (!check) continue;
            const bool own_check = (s.iter % s.opts.check_every == 0) || s.iter >= s.opts.max_iter;
            if (!own_check) {
                if (s.kind == SE2_REQ_OT) s.cur ^= 1;
                continue;
            }
            s.last_err = errs[i];
            if (!std::isfinite(errs[i])) {
                q->rc = SE2_ENUMERIC;
                finished.push_back(q);
            } else if (final_stage(s) && s.opts.tol_marg_l1 >= 0 && errs[i] <= s.opts.tol_marg_l1) {
                s.status = SE2_CONVERGED;
                finished.push_back(q);
            } else if (s.iter >= s.opts.max_iter) {
                s.status = SE2_MAX_ITER;
                finished.push_back(q);
            } else {
                if (s.kind == SE2_REQ_OT) s.cur ^= 1;
                phase_after_check(s, errs[i]);
            }
        }
        if (rc == SE2_OK) {
            // eps-scaling: solves whose coarse stage has ended move to the next eps
            std::vector<Req *> going;
            std::vector<Solve *> going_s;
            for (Req *q : run)
                if (std::find(finished.begin(), finished.end(), q) == finished.end()) {
                    going.push_back(q);
                    going_s.push_back(&q->s);
                }
            const int rc2 = advance_stages(eng, going_s, st);
            if (rc2)
                for (Req *q : going) {
                    q->rc = rc2;
                    finished.push_back(q);
                }
        }
        // a check folds the timing events of the interval before it; when solves finish here,
        // fold the rest too, so that the intervals are published before their tickets complete
        if (check && !finished.empty()) (void)eng.collect_profile();
        {
            std::lock_guard<std::mutex> lk(Q->mu);
            Q->steps += 1;
            if (Q->prof_request) Q->prof_rounds[l] += 2;
            if (check && Q->prof_request) {
                // publish the intervals collected since this lane's last check, and its totals
                Q->prof_iv[l].insert(Q->prof_iv[l].end(), eng.prof_intervals.begin(), eng.prof_intervals.end());
                eng.prof_intervals.clear();
                Q->prof_terms[l] = eng.prof_terms;
                Q->prof_outputs[l] = eng.prof_outputs;
            }
        }
        if (!finished.empty()) finish_group(Q, l, finished);
    }
}

}  // namespace
}  // namespace se2

using namespace se2;

extern "C" {

int se2_solve_queue_create(size_t hbm_budget_bytes, int32_t max_slots, se2_queue_t *out) {
    if (!out || max_slots < 1) return SE2_EINVAL;
    auto *Q = new (std::nothrow) se2_queue_s();
    if (!Q) return SE2_ENOMEM;
    Q->budget = hbm_budget_bytes;
    Q->max_slots = max_slots;
    // default-priority streams, one per lane
    bool ok = hipGetDevice(&Q->device) == hipSuccess;
    for (int l = 0; l < kLanes && ok; ++l) ok = hipStreamCreateWithFlags(&Q->st[l], hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        for (hipStream_t x : Q->st)
            if (x) (void)hipStreamDestroy(x);
        delete Q;
        return SE2_EHIP;
    }
    if (!Q->arena.init(hbm_budget_bytes)) {
        for (hipStream_t x : Q->st) (void)hipStreamDestroy(x);
        delete Q;
        return SE2_ENOMEM;
    }
    for (int l = 0; l < kLanes; ++l) Q->worker[l] = std::thread(lane_main, Q, l);
    *out = Q;
    return SE2_OK;
}

int se2_request_bytes(const se2_request_t *req, size_t *bytes) {
    if (!req || !bytes || !req->kernel) return SE2_EINVAL;
    Req q;
    q.r = *req;
    if (req->kind == SE2_REQ_BARYCENTER) {
        if (req->n < 1 || req->n > kMaxMeasures || !req->lambdas) return SE2_EINVAL;
        for (int i = 0; i < req->n; ++i) {
            q.mus_all.push_back(nullptr);
            q.lambdas_all.push_back(req->lambdas[i]);
        }
    } else if (req->kind != SE2_REQ_OT) {
        return SE2_EINVAL;
    }
    *bytes = request_bytes(q);
    return SE2_OK;
}

int se2_solve_queue_submit(se2_queue_t Q, const se2_request_t *req, uint64_t *ticket) {
    if (!Q || !req || !ticket || !req->kernel) return SE2_EINVAL;
    const se2_opts_t &o = req->opts;
    if (!valid_solver_opts(o, *reinterpret_cast<const Kernel *>(req->kernel))) return SE2_EINVAL;
    {
        // build the kernels of an eps-scaling schedule here, so admission only looks them up
        const Kernel &base = *reinterpret_cast<const Kernel *>(req->kernel);
        std::vector<double> sched;
        int rc = eps_schedule(o, base.metric.eps, sched);
        if (rc) return rc;
        for (double e : sched) {
            const Kernel *kk = nullptr;
            if ((rc = kernel_at_eps(base, e, &kk))) return rc;
        }
    }
    auto q = std::make_unique<Req>();
    q->r = *req;
    q->r.opts.init_g = nullptr;
    if (req->kind == SE2_REQ_OT) {
        if (!req->mu || !req->nu) return SE2_EINVAL;
    } else if (req->kind == SE2_REQ_BARYCENTER) {
        if (req->n < 1 || req->n > kMaxMeasures || !req->mus || !req->lambdas || !req->bary_out) return SE2_EINVAL;
        double lsum = 0.0;
        int npos = 0;
        for (int i = 0; i < req->n; ++i) {
            if (!req->mus[i] || !(req->lambdas[i] >= 0.0) || !std::isfinite(req->lambdas[i])) return SE2_EINVAL;
            lsum += req->lambdas[i];
            npos += req->lambdas[i] > 0.0;
            q->mus_all.push_back(req->mus[i]);
            q->lambdas_all.push_back(req->lambdas[i]);
        }
        if (!(std::fabs(lsum - 1.0) <= 1e-12) || npos == 0) return SE2_EINVAL;
        q->r.mus = nullptr;
        q->r.lambdas = nullptr;
    } else {
        return SE2_EINVAL;
    }
    q->bytes = request_bytes(*q);
    q->t_submit = now_seconds();
    std::lock_guard<std::mutex> lk(Q->mu);
    if (q->bytes > Q->arena.size()) {
        Q->rejected += 1;
        return SE2_ENOMEM;
    }
    q->ticket = Q->next_ticket++;
    *ticket = q->ticket;
    q->lane = 0;  // the lane with the least outstanding work
    for (int l = 1; l < kLanes; ++l)
        if (Q->load[l] < Q->load[q->lane]) q->lane = l;
    Q->load[q->lane] += request_load(*q);
    Q->waiting[q->lane].push_back(q.get());
    Q->all[q->ticket] = std::move(q);
    Q->gen += 1;
    Q->cv.notify_all();
    return SE2_OK;
}

int se2_solve_queue_poll(se2_queue_t Q, uint64_t ticket, se2_report_t *report) {
    if (!Q) return SE2_EINVAL;
    std::lock_guard<std::mutex> lk(Q->mu);
    auto it = Q->all.find(ticket);
    if (it == Q->all.end()) return SE2_EINVAL;
    Req *q = it->second.get();
    if (q->state != DONE) return SE2_PENDING;
    if (report) *report = q->rep;
    return q->rc;
}

int se2_solve_queue_wait(se2_queue_t Q, uint64_t ticket, se2_report_t *report) {
    if (!Q) return SE2_EINVAL;
    std::unique_lock<std::mutex> lk(Q->mu);
    auto it = Q->all.find(ticket);
    if (it == Q->all.end()) return SE2_EINVAL;
    Req *q = it->second.get();
    Q->done_cv.wait(lk, [&] { return q->state == DONE; });
    if (report) *report = q->rep;
    return q->rc;
}

int se2_solve_queue_times(se2_queue_t Q, uint64_t ticket, double *t_submit, double *t_admit, double *t_done) {
    if (!Q) return SE2_EINVAL;
    std::lock_guard<std::mutex> lk(Q->mu);
    auto it = Q->all.find(ticket);
    if (it == Q->all.end()) return SE2_EINVAL;
    Req *q = it->second.get();
    if (t_submit) *t_submit = q->t_submit;
    if (t_admit) *t_admit = q->t_admit;
    if (t_done) *t_done = q->t_done;
    return q->state == DONE ? SE2_OK : SE2_PENDING;
}

int se2_solve_queue_release(se2_queue_t Q, uint64_t ticket) {
    if (!Q) return SE2_EINVAL;
    std::lock_guard<std::mutex> lk(Q->mu);
    auto it = Q->all.find(ticket);
    if (it == Q->all.end()) return SE2_EINVAL;
    if (it->second->state != DONE) return SE2_PENDING;
    Q->all.erase(it);
    return SE2_OK;
}

int se2_solve_queue_stats(se2_queue_t Q, int64_t *out5) {
    if (!Q || !out5) return SE2_EINVAL;
    std::lock_guard<std::mutex> lk(Q->mu);
    out5[0] = Q->admitted;
    out5[1] = Q->completed;
    out5[2] = Q->rejected;
    out5[3] = Q->peak;
    out5[4] = Q->steps;
    return SE2_OK;
}

int se2_solve_queue_profile(se2_queue_t Q, int32_t enable) {
    if (!Q) return SE2_EINVAL;
    std::lock_guard<std::mutex> lk(Q->mu);
    if (enable) {
        // a common time origin for all lanes: recorded on lane 0, the others wait for it, and
        // the lanes start timing only after this call
        if (!Q->prof_ref) SE2_HIP(hipEventCreate(&Q->prof_ref));
        SE2_HIP(hipEventRecord(Q->prof_ref, Q->st[0]));
        for (int l = 1; l < kLanes; ++l) SE2_HIP(hipStreamWaitEvent(Q->st[l], Q->prof_ref, 0));
    }
    Q->prof_request = enable ? 1 : 0;
    for (bool &f : Q->prof_reset) f = true;
    for (auto &v : Q->prof_iv) v.clear();
    for (int l = 0; l < kLanes; ++l) {
        Q->prof_terms[l] = Q->prof_outputs[l] = 0.0;
        Q->prof_rounds[l] = 0;
    }
    Q->gen += 1;
    Q->cv.notify_all();
    return SE2_OK;
}

int se2_solve_queue_kernel_time(se2_queue_t Q, double *out4) {
    if (!Q || !out4) return SE2_EINVAL;
    std::lock_guard<std::mutex> lk(Q->mu);
    double terms = 0.0, outputs = 0.0;
    int64_t rounds = 0;
    for (int j = 0; j < kLanes; ++j) {
        terms += Q->prof_terms[j];
        outputs += Q->prof_outputs[j];
        rounds = std::max(rounds, Q->prof_rounds[j]);
    }
    out4[0] = union_seconds(Q);
    out4[1] = terms;
    out4[2] = static_cast<double>(rounds);
    out4[3] = outputs;
    return SE2_OK;
}

int se2_solve_queue_destroy(se2_queue_t Q) {
    if (!Q) return SE2_EINVAL;
    {
        std::lock_guard<std::mutex> lk(Q->mu);
        Q->stop = true;
        Q->gen += 1;
        Q->cv.notify_all();
    }
    for (std::thread &w : Q->worker)
        if (w.joinable()) w.join();
    for (hipStream_t x : Q->st) {
        (void)hipStreamSynchronize(x);
        (void)hipStreamDestroy(x);
    }
    if (Q->prof_ref) (void)hipEventDestroy(Q->prof_ref);
    delete Q;
    return SE2_OK;
}

}  // extern "C"
