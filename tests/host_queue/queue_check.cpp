// Host build of the serving queue (csrc/queue.cpp) against the mock executor: admission by
// budget and slot count in arrival order, latency bookkeeping on the fake clock, release of
// finished tickets, the kernel-time union against the intervals the executor recorded, and
// concurrent submitters.  Built with the thread sanitizer and with the address and
// undefined-behaviour sanitizers by tests/test_queue_host.py; exits non-zero on a failed check.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "../../paper_2402_15322_amd/csrc/solver.h"

extern "C" double mock_now_ms();
extern "C" double mock_interval_union_ms();
extern "C" size_t mock_interval_count();
extern "C" void mock_reset_log();

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

namespace {

se2::Kernel *make_kernel(int n, int nt) {
    auto *k = new se2::Kernel();
    k->grid = se2_grid_t{n, n, nt, 0};
    k->metric = se2_metric_t{1.0, 2.0, 1.0, 0.5, 2};
    k->W = 5;
    return k;
}

// An OT request whose mock solve converges at iteration n_iter (error 1 / i at iteration i).
se2_request_t ot_request(se2::Kernel *k, const double *mu, int n_iter, int check_every) {
    se2_request_t r{};
    r.kind = SE2_REQ_OT;
    r.n = 1;
    r.kernel = reinterpret_cast<se2_kernel_t>(k);
    r.mu = mu;
    r.nu = mu;
    r.opts.tol_marg_l1 = 1.0 / n_iter;
    r.opts.max_iter = 10 * n_iter;
    r.opts.check_every = check_every;
    r.opts.prec = SE2_F32;
    return r;
}

void admission_and_bookkeeping() {
    se2::Kernel *k = make_kernel(8, 8);
    std::vector<double> mu(8 * 8 * 8, 1.0 / 512);
    se2_request_t r = ot_request(k, mu.data(), 20, 10);
    size_t bytes = 0;
    CHECK(se2_request_bytes(&r, &bytes) == SE2_OK && bytes > 0);
    se2_queue_t q = nullptr;
    // room for two resident solves at a time
    CHECK(se2_solve_queue_create(bytes * 5 / 2, 16, &q) == SE2_OK);
    std::vector<uint64_t> t(8);
    for (auto &x : t) CHECK(se2_solve_queue_submit(q, &r, &x) == SE2_OK);
    std::vector<double> sub(8), adm(8), done(8);
    for (int i = 0; i < 8; ++i) {
        se2_report_t rep{};
        CHECK(se2_solve_queue_wait(q, t[i], &rep) == SE2_OK);
        CHECK(rep.status == SE2_CONVERGED && rep.iters == 20);
        CHECK(se2_solve_queue_times(q, t[i], &sub[i], &adm[i], &done[i]) == SE2_OK);
        CHECK(sub[i] <= adm[i] && adm[i] <= done[i]);
        // 20 iterations, each at least one step of the fake clock after admission
        CHECK(done[i] - adm[i] >= 20 * 1e-3 - 1e-12);
        CHECK(std::fabs(rep.seconds - (done[i] - sub[i])) <= 1e-12);
    }
    int64_t st[5];
    CHECK(se2_solve_queue_stats(q, st) == SE2_OK);
    CHECK(st[0] == 8 && st[1] == 8 && st[2] == 0);
    CHECK(st[3] >= 1 && st[3] <= 2);  // never more than the budget holds
    // a request larger than the whole budget is refused at submit
    se2::Kernel *big = make_kernel(64, 16);
    std::vector<double> mub(64 * 64 * 16, 1.0 / (64 * 64 * 16));
    se2_request_t rb = ot_request(big, mub.data(), 10, 10);
    uint64_t tb = 0;
    CHECK(se2_solve_queue_submit(q, &rb, &tb) == SE2_ENOMEM);
    CHECK(se2_solve_queue_stats(q, st) == SE2_OK && st[2] == 1);
    // release: a finished ticket is dropped and becomes invalid
    CHECK(se2_solve_queue_release(q, t[0]) == SE2_OK);
    CHECK(se2_solve_queue_poll(q, t[0], nullptr) == SE2_EINVAL);
    CHECK(se2_solve_queue_release(q, t[0]) == SE2_EINVAL);
    CHECK(se2_solve_queue_destroy(q) == SE2_OK);
    delete k;
    delete big;
}

void slots_and_arrival_order() {
    se2::Kernel *k = make_kernel(8, 8);
    std::vector<double> mu(512, 1.0 / 512);
    se2_queue_t q = nullptr;
    CHECK(se2_solve_queue_create(64 << 20, 1, &q) == SE2_OK);  // one slot over all lanes
    std::vector<uint64_t> t(6);
    for (int i = 0; i < 6; ++i) {
        se2_request_t r = ot_request(k, mu.data(), 10 + 10 * (i % 3), 10);
        CHECK(se2_solve_queue_submit(q, &r, &t[i]) == SE2_OK);
    }
    std::vector<double> adm(6), done(6);
    for (int i = 0; i < 6; ++i) {
        CHECK(se2_solve_queue_wait(q, t[i], nullptr) == SE2_OK);
        CHECK(se2_solve_queue_times(q, t[i], nullptr, &adm[i], &done[i]) == SE2_OK);
    }
    // one slot: the solves' resident intervals [admission, completion] never overlap
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j)
            if (i != j) CHECK(done[i] <= adm[j] || done[j] <= adm[i]);
    int64_t st[5];
    CHECK(se2_solve_queue_stats(q, st) == SE2_OK && st[3] == 1);
    CHECK(se2_solve_queue_destroy(q) == SE2_OK);
    delete k;
}

void profiling_union() {
    se2::Kernel *k = make_kernel(8, 8);
    std::vector<double> mu(512, 1.0 / 512);
    se2_queue_t q = nullptr;
    CHECK(se2_solve_queue_create(64 << 20, 32, &q) == SE2_OK);
    mock_reset_log();
    CHECK(se2_solve_queue_profile(q, 1) == SE2_OK);
    std::vector<uint64_t> t(12);
    for (int i = 0; i < 12; ++i) {
        se2_request_t r = ot_request(k, mu.data(), 10 * (1 + i % 3), 10);
        CHECK(se2_solve_queue_submit(q, &r, &t[i]) == SE2_OK);
    }
    for (auto x : t) CHECK(se2_solve_queue_wait(q, x, nullptr) == SE2_OK);
    double out4[4];
    CHECK(se2_solve_queue_kernel_time(q, out4) == SE2_OK);
    // every lane's last step is a check step, so every recorded interval is published; the
    // queue's union equals the union of the executor's intervals (disjoint 1 ms steps)
    const double expect = 1e-3 * mock_interval_union_ms();
    CHECK(mock_interval_count() > 0);
    CHECK(std::fabs(out4[0] - expect) <= 1e-12);
    CHECK(out4[0] <= 1e-3 * mock_now_ms());
    CHECK(out4[2] >= 60.0);  // the longest solve's 30 iterations, two half-steps each
    CHECK(se2_solve_queue_profile(q, 0) == SE2_OK);
    CHECK(se2_solve_queue_destroy(q) == SE2_OK);
    delete k;
}

void concurrent_submitters() {
    se2::Kernel *k = make_kernel(8, 8);
    std::vector<double> mu(512, 1.0 / 512);
    se2_queue_t q = nullptr;
    CHECK(se2_solve_queue_create(64 << 20, 8, &q) == SE2_OK);
    std::vector<std::thread> th;
    std::vector<int> bad(4, 0);
    for (int w = 0; w < 4; ++w)
        th.emplace_back([&, w] {
            for (int i = 0; i < 25; ++i) {
                se2_request_t r = ot_request(k, mu.data(), 10 + 10 * ((w + i) % 2), 10);
                uint64_t tk = 0;
                if (se2_solve_queue_submit(q, &r, &tk) != SE2_OK) {
                    ++bad[w];
                    continue;
                }
                se2_report_t rep{};
                int rc;
                if (i % 2) {
                    while ((rc = se2_solve_queue_poll(q, tk, &rep)) == SE2_PENDING) std::this_thread::yield();
                } else {
                    rc = se2_solve_queue_wait(q, tk, &rep);
                }
                double a, b, c;
                if (rc != SE2_OK || se2_solve_queue_times(q, tk, &a, &b, &c) != SE2_OK || !(a <= b && b <= c)) ++bad[w];
                if (se2_solve_queue_release(q, tk) != SE2_OK) ++bad[w];
            }
        });
    for (auto &x : th) x.join();
    for (int b : bad) CHECK(b == 0);
    int64_t st[5];
    CHECK(se2_solve_queue_stats(q, st) == SE2_OK && st[1] == 100);
    CHECK(se2_solve_queue_destroy(q) == SE2_OK);
    delete k;
}

}  // namespace

int main() {
    admission_and_bookkeeping();
    slots_and_arrival_order();
    profiling_union();
    concurrent_submitters();
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("queue host checks passed\n");
    return 0;
}
