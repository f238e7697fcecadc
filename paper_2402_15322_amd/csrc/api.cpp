// C ABI of the SE(2) entropic-OT library: argument checks, kernel handles,
// stream-ordered convolutions and the blocking Sinkhorn / barycenter drivers.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "solver.h"

namespace se2 {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string &msg) { g_last_error = msg; }

void set_last_hip_error(hipError_t e, const char *what, const char *file, int line) {
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    g_last_error = buf;
}

namespace {

bool valid_grid(const se2_grid_t *g) {
    return g && g->nx >= 1 && g->ny >= 1 && (g->ntheta == 8 || g->ntheta == 16 || g->ntheta == 32) &&
           (g->theta_axial == 0 || g->theta_axial == 1) &&
           static_cast<long long>(g->nx) * g->ny * g->ntheta <= (1LL << 31);
}

bool valid_metric(const se2_metric_t *m) {
    return m && std::isfinite(m->w1) && std::isfinite(m->w2) && std::isfinite(m->w3) && std::isfinite(m->eps) &&
           m->w1 > 0 && m->w2 > 0 && m->w3 > 0 && m->eps > 0 && m->radius >= 0 && m->radius <= kMaxRadius;
}

bool valid_opts(const se2_opts_t *o, const Kernel *k) { return o && k && valid_solver_opts(*o, *k); }

}  // namespace

void kernel_free(Kernel *k) {
    if (!k) return;
    for (auto &e : k->scaled) kernel_free(e.second);
    (void)hipFree(k->d_L64);
    (void)hipFree(k->d_L32);
    (void)hipFree(k->d_cost32);
    (void)hipFree(k->d_K32);
    (void)hipFree(k->d_Kbf16);
    (void)hipFree(k->d_K64);
    (void)hipFree(k->d_Bpack);
    (void)hipFree(k->d_Fpack);
    delete k;
}

int kernel_at_eps(const Kernel &base, double eps, const Kernel **out) {
    if (eps == base.metric.eps) {
        *out = &base;
        return SE2_OK;
    }
    std::lock_guard<std::mutex> lk(base.scaled_mu);
    for (auto &e : base.scaled)
        if (e.first == eps) {
            *out = e.second;
            return SE2_OK;
        }
    Kernel *k = new (std::nothrow) Kernel();
    if (!k) return SE2_ENOMEM;
    k->grid = base.grid;
    k->metric = base.metric;
    k->metric.eps = eps;
    k->device = base.device;
    int dev = 0;
    SE2_HIP(hipGetDevice(&dev));
    if (dev != base.device) SE2_HIP(hipSetDevice(base.device));
    const int rc = build_tables(*k);
    if (dev != base.device) SE2_HIP(hipSetDevice(dev));
    if (rc) {
        kernel_free(k);
        return rc;
    }
    base.scaled.emplace_back(eps, k);
    *out = k;
    return SE2_OK;
}

// Device-side FP64 validation of a probability vector: finite, >= 0, |sum - 1| <= tol.
int validate_measure(const double *m, size_t n, double tol, hipStream_t st) {
    double *stats = nullptr;
    SE2_HIP(hipMallocAsync(reinterpret_cast<void **>(&stats), (2 + 2 * 256) * sizeof(double), st));
    int rc = launch_validate(m, n, stats, st);
    double h[2] = {0, 0};
    if (rc == SE2_OK) {
        SE2_HIP(hipMemcpyAsync(h, stats, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        SE2_HIP(hipStreamSynchronize(st));
    }
    SE2_HIP(hipFreeAsync(stats, st));
    if (rc) return rc;
    if (h[1] != 0.0 || !(std::fabs(h[0] - 1.0) <= tol)) {
        g_last_error = "input measure is not a probability vector (negative, non-finite or |sum-1| > tol)";
        return SE2_EINVAL;
    }
    return SE2_OK;
}

int validate_measures(const std::vector<const double *> &ms, size_t n, double tol, hipStream_t st) {
    const int m = static_cast<int>(ms.size());
    if (m == 0) return SE2_OK;
    if (m == 1) return validate_measure(ms[0], n, tol, st);
    const size_t nb = static_cast<size_t>(validate_many_blocks(n));
    const size_t tab_bytes = (m * sizeof(double *) + 255) / 256 * 256;
    const size_t bytes = tab_bytes + (2 * static_cast<size_t>(m) + 2 * m * nb) * sizeof(double);
    char *mem = nullptr;
    SE2_HIP(hipMallocAsync(reinterpret_cast<void **>(&mem), bytes, st));
    const double **tab = reinterpret_cast<const double **>(mem);
    double *stats = reinterpret_cast<double *>(mem + tab_bytes);
    std::vector<double> h(2 * static_cast<size_t>(m));
    int rc = SE2_OK;
    if (hipMemcpyAsync(tab, ms.data(), m * sizeof(double *), hipMemcpyHostToDevice, st) != hipSuccess) rc = SE2_EHIP;
    if (rc == SE2_OK) rc = launch_validate_many(tab, m, n, stats, stats + 2 * m, st);
    if (rc == SE2_OK && hipMemcpyAsync(h.data(), stats, h.size() * sizeof(double), hipMemcpyDeviceToHost, st) !=
                            hipSuccess)
        rc = SE2_EHIP;
    SE2_HIP(hipStreamSynchronize(st));  // also keeps `ms` and `h` alive for the copies
    SE2_HIP(hipFreeAsync(mem, st));
    if (rc) return rc;
    for (int j = 0; j < m; ++j)
        if (h[2 * j + 1] != 0.0 || !(std::fabs(h[2 * j] - 1.0) <= tol)) {
            g_last_error = "input measure " + std::to_string(j) +
                           " is not a probability vector (negative, non-finite or |sum-1| > tol)";
            return SE2_EINVAL;
        }
    return SE2_OK;
}

namespace {

struct DeviceBlock {
    void *p = nullptr;
    hipStream_t st = nullptr;
    ~DeviceBlock() {
        if (p) (void)hipFreeAsync(p, st);
    }
};

}  // namespace
}  // namespace se2

namespace se2 {
namespace {

bool valid_flow(const Kernel *k, const se2_flow_t *flow, const se2_opts_t *opts) {
    return flow && valid_opts(opts, k) && std::isfinite(flow->tau) && flow->tau >= 0.0 &&
           std::isfinite(flow->m) && flow->m > 1.0 && std::isfinite(flow->ref) && flow->ref > 0.0 &&
           !(opts->eps_start > k->metric.eps) &&
           std::isfinite((flow->tau / k->metric.eps) * flow->m / (flow->m - 1.0) * std::pow(flow->ref, 1.0 - flow->m));
}

// One JKO step from the (validated) device measure mu: the scaling iterations of
// se2_jko_step, log b started from init * init_scale (init may be null: log b = 0).
// psi_out (device, may be null) receives the returned iterate's log b in base 2.
int jko_run(const Kernel *k, const double *mu, const double *init, double init_scale, const se2_flow_t &flow,
            const se2_opts_t &opts, double *mu_next, double *f_out, double *g_out, double *psi_out,
            se2_report_t *report, hipStream_t st) {
    Solve s;
    s.kind = kKindJKO;
    s.k = k;
    s.opts = opts;
    s.n = 1;
    s.t_start = now_seconds();
    // prox constant of min_q (tau/eps) F(q) + KL(q | p): log q + c q^(m-1) = log p
    const double m = flow.m;
    s.jko_m = m;
    s.jko_ref = flow.ref;
    s.jko_c = (flow.tau / k->metric.eps) * m / (m - 1.0) * std::pow(flow.ref, 1.0 - m);
    int rc;
    if ((rc = plan_stages(s, *k))) return rc;
    DeviceBlock mem;
    mem.st = st;
    SE2_HIP(hipMallocAsync(&mem.p, solve_bytes(kKindJKO, *k, 1, prune_wanted(opts)), st));
    solve_bind(s, mem.p);
    if ((rc = solve_setup_jko(s, mu, init, init_scale, st))) return rc;
    Engine eng;
    std::vector<Solve *> one = {&s};
    if ((rc = eng.init_first_halfstep(one, st))) return rc;
    s.convs = 1;
    std::vector<double> errs;
    while (!s.done) {
        const bool last = s.iter + 1 >= opts.max_iter;
        const bool check = last || ((s.iter + 1) % opts.check_every == 0);
        if ((rc = eng.step(one, check, st))) return rc;
        if (check) {
            if ((rc = eng.read_errors(one, errs, st))) return rc;
            s.last_err = errs[0];
            if (!std::isfinite(errs[0])) {
                g_last_error = "non-finite marginal error";
                return SE2_ENUMERIC;
            }
            if (opts.tol_marg_l1 >= 0 && errs[0] <= opts.tol_marg_l1) {
                s.done = true;
                s.status = SE2_CONVERGED;
            } else if (last) {
                s.done = true;
                s.status = SE2_MAX_ITER;
            } else {
                s.cur ^= 1;
                phase_after_check(s, errs[0]);
            }
        }
    }
    std::vector<FinishReq> fin(1);
    fin[0].s = &s;
    fin[0].f_out = f_out;
    fin[0].g_out = g_out;
    fin[0].bary_out = mu_next;
    if ((rc = finish_solves(eng, fin, st))) return rc;
    if (psi_out) SE2_HIP(hipMemcpyAsync(psi_out, s.psi, s.E * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (report) *report = fin[0].rep;
    return fin[0].rc;
}

}  // namespace
}  // namespace se2

using namespace se2;

extern "C" {

int se2_init(void) {
    int dev = 0;
    SE2_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    SE2_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_last_error = std::string("device is ") + prop.gcnArchName + ", library built for gfx950";
        return SE2_EINVAL;
    }
    // device address of the library's own scratch on this device (se2_split_signed_noalloc)
    double *scr = nullptr;
    return split_noalloc_scratch(&scr);
}

const char *se2_strerror(int code) {
    switch (code) {
        case SE2_OK: return "ok";
        case SE2_EINVAL: return g_last_error.empty() ? "invalid argument" : g_last_error.c_str();
        case SE2_ENOMEM: return "out of memory or over the queue budget";
        case SE2_EHIP: return g_last_error.empty() ? "HIP runtime error" : g_last_error.c_str();
        case SE2_ENUMERIC: return "non-finite value (mass without a partner inside the window?)";
        case SE2_PENDING: return "pending";
        default: return "unknown error";
    }
}

int se2_kernel_build(const se2_grid_t *grid, const se2_metric_t *metric, se2_kernel_t *out) {
    if (!out || !valid_grid(grid) || !valid_metric(metric)) return SE2_EINVAL;
    Kernel *k = new (std::nothrow) Kernel();
    if (!k) return SE2_ENOMEM;
    k->grid = *grid;
    k->metric = *metric;
    SE2_HIP(hipGetDevice(&k->device));
    int rc = build_tables(*k);
    if (rc) {
        se2_kernel_destroy(reinterpret_cast<se2_kernel_t>(k));
        return rc;
    }
    *out = reinterpret_cast<se2_kernel_t>(k);
    return SE2_OK;
}

int se2_kernel_destroy(se2_kernel_t h) {
    Kernel *k = reinterpret_cast<Kernel *>(h);
    if (!k) return SE2_EINVAL;
    kernel_free(k);
    return SE2_OK;
}

int se2_kernel_table(se2_kernel_t h, double *host_logk, double *host_cost) {
    const Kernel *k = reinterpret_cast<const Kernel *>(h);
    if (!k) return SE2_EINVAL;
    if (host_logk) std::memcpy(host_logk, k->logk.data(), k->entries * sizeof(double));
    if (host_cost) std::memcpy(host_cost, k->cost.data(), k->entries * sizeof(double));
    return SE2_OK;
}

int se2_kernel_info(se2_kernel_t h, se2_grid_t *grid, se2_metric_t *metric, int32_t *nz) {
    const Kernel *k = reinterpret_cast<const Kernel *>(h);
    if (!k) return SE2_EINVAL;
    if (grid) *grid = k->grid;
    if (metric) *metric = k->metric;
    if (nz) *nz = k->nonzero_bf16;
    return SE2_OK;
}

int se2_conv(se2_kernel_t h, se2_prec_t prec, const void *in, void *out, int32_t batch, se2_stream_t stream) {
    const Kernel *k = reinterpret_cast<const Kernel *>(h);
    if (!k || !in || !out || batch < 0 || in == out) return SE2_EINVAL;
    // the float paths stage the input with 16-byte loads
    if (prec != SE2_F64 && (reinterpret_cast<uintptr_t>(in) & 15)) return SE2_EINVAL;
    if (batch == 0) return SE2_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    switch (prec) {
        case SE2_BF16:
            return launch_conv_bf16(*k, static_cast<const float *>(in), static_cast<float *>(out), batch, st);
        case SE2_F32:
            return launch_conv_f32(*k, static_cast<const float *>(in), static_cast<float *>(out), batch, st);
        case SE2_F64:
            return launch_conv_f64(*k, static_cast<const double *>(in), static_cast<double *>(out), batch, st);
        default:
            return SE2_EINVAL;
    }
}

int se2_conv_log(se2_kernel_t h, se2_prec_t prec, const double *in, double *out, int32_t batch, int32_t *fallbacks,
                 se2_stream_t stream) {
    const Kernel *k = reinterpret_cast<const Kernel *>(h);
    if (!k || !in || !out || batch < 0 || in == out) return SE2_EINVAL;
    const bool lin = prec == SE2_BF16 || prec == SE2_F32_MFMA;
    if (prec != SE2_F32 && prec != SE2_F64 && !lin) return SE2_EINVAL;
    if (lin && !lin_supported(k->grid.ntheta, prec == SE2_BF16)) return SE2_EINVAL;
    if (batch == 0) {
        if (fallbacks) *fallbacks = 0;
        return SE2_OK;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int nt = k->grid.ntheta, R = k->metric.radius;
    const size_t E = static_cast<size_t>(k->grid.nx) * k->grid.ny * nt;
    const int tiles = tiles_of(k->grid.nx) * tiles_of(k->grid.ny);
    // the matrix-core engines' tiling (rows per wave from the grid, as in the solvers)
    const int rpw = lin ? lin_rows_per_wave(nt, prec == SE2_BF16, k->grid.ny) : 0;
    const int per = lin ? lin_blocks(k->grid.nx, k->grid.ny, rpw) : tiles;
    // scratch: base-2 copy of the input, job table, block map; for the matrix-core engines also
    // the list of tiles with rejected groups, two counters and the fallback counter
    const size_t cap_tiles = static_cast<size_t>(tiles) * batch;  // capacity of the fallback list
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t o_jobs = al(E * batch * sizeof(double));
    const size_t o_map = o_jobs + al(batch * sizeof(ConvJob));
    const size_t o_fb = o_map + al(static_cast<size_t>(per) * batch * sizeof(int32_t));
    const size_t o_cnt = o_fb + (lin ? al(cap_tiles * sizeof(int4)) : 0);
    const size_t total = o_cnt + (lin ? al(3 * sizeof(int32_t)) : 0);
    char *mem = nullptr;
    SE2_HIP(hipMallocAsync(reinterpret_cast<void **>(&mem), total, st));
    double *tmp = reinterpret_cast<double *>(mem);
    ConvJob *dj = reinterpret_cast<ConvJob *>(mem + o_jobs);
    int32_t *dm = reinterpret_cast<int32_t *>(mem + o_map);
    int4 *fb = lin ? reinterpret_cast<int4 *>(mem + o_fb) : nullptr;
    int32_t *cnt = lin ? reinterpret_cast<int32_t *>(mem + o_cnt) : nullptr;
    // natural -> base-2 log units on the scratch copy; results scaled back in place
    int rc = launch_scale(in, tmp, E * batch, kLog2e, st);
    std::vector<ConvJob> jobs(batch);
    std::vector<int32_t> map(static_cast<size_t>(per) * batch);
    for (int b = 0; b < batch; ++b) {
        ConvJob &j = jobs[b];
        j = ConvJob{};
        j.in = tmp + E * b;
        j.out = out + E * b;
        j.L64 = k->d_L64;
        j.L32 = k->d_L32;
        j.nx = k->grid.nx;
        j.ny = k->grid.ny;
        j.R = R;
        j.epi = EPI_RAW;
        j.tiles_x = tiles_of(k->grid.nx);
        j.tiles = tiles;
        j.first_block = b * per;
        j.blocks = per;
        if (lin) {
            j.kop = prec == SE2_BF16 ? static_cast<const void *>(k->d_Bpack) : static_cast<const void *>(k->d_Fpack);
            j.fallbacks = cnt + 2;
        }
        for (int t = 0; t < per; ++t) map[static_cast<size_t>(b) * per + t] = b;
    }
    if (rc == SE2_OK && hipMemcpyAsync(dj, jobs.data(), batch * sizeof(ConvJob), hipMemcpyHostToDevice, st) != hipSuccess)
        rc = SE2_EHIP;
    if (rc == SE2_OK && hipMemcpyAsync(dm, map.data(), map.size() * sizeof(int32_t), hipMemcpyHostToDevice, st) !=
                            hipSuccess)
        rc = SE2_EHIP;
    if (rc == SE2_OK && lin) rc = launch_fill_i32(cnt, 3, 0, st);
    if (rc == SE2_OK) {
        if (lin) {
            const int fb_grid = cap_tiles < 1024 ? static_cast<int>(cap_tiles) : 1024;
            rc = launch_conv_lin_log(dj, per * batch, dm, nt, R, rpw, prec == SE2_BF16, fb, cnt, cnt + 1, fb_grid, st);
        } else {
            rc = launch_conv_lse(dj, batch, tiles * batch, dm, nt, R, prec == SE2_F64, false, nullptr, nullptr, nullptr,
                                 8, nullptr, st);
        }
    }
    if (rc == SE2_OK) rc = launch_scale(out, out, E * batch, kLn2, st);
    int32_t h_fb = 0;
    if (rc == SE2_OK && lin && fallbacks &&
        hipMemcpyAsync(&h_fb, cnt + 2, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = SE2_EHIP;
    // host vectors are read by the async copies: wait before they go out of scope
    SE2_HIP(hipStreamSynchronize(st));
    SE2_HIP(hipFreeAsync(mem, st));
    if (rc == SE2_OK && fallbacks) *fallbacks = lin ? h_fb : 0;
    return rc;
}

int se2_lift_field(const se2_grid_t *grid, const double *mag, const double *angle, double *out, int32_t batch,
                   se2_stream_t stream) {
    if (!valid_grid(grid) || !mag || !angle || !out || batch < 0 || (reinterpret_cast<uintptr_t>(out) & 15))
        return SE2_EINVAL;
    const size_t npix = static_cast<size_t>(grid->nx) * grid->ny * static_cast<size_t>(batch);
    const double period = grid->theta_axial ? M_PI : 2.0 * M_PI;
    return launch_lift_field(mag, angle, out, npix, grid->ntheta, period, reinterpret_cast<hipStream_t>(stream));
}

int se2_project(const se2_grid_t *grid, const double *u, const double *u_minus, double *mass, int32_t *argmax,
                double *angle, int32_t batch, se2_stream_t stream) {
    if (!valid_grid(grid) || !u || !mass || batch < 0 || (reinterpret_cast<uintptr_t>(u) & 15) ||
        (reinterpret_cast<uintptr_t>(u_minus) & 15))
        return SE2_EINVAL;
    const size_t npix = static_cast<size_t>(grid->nx) * grid->ny * static_cast<size_t>(batch);
    const double period = grid->theta_axial ? M_PI : 2.0 * M_PI;
    return launch_project(u, u_minus, npix, grid->ntheta, period, mass, argmax, angle,
                          reinterpret_cast<hipStream_t>(stream));
}

int se2_split_signed(const double *u, size_t n, double *plus, double *minus, se2_stream_t stream) {
    if ((!u || !plus || !minus) && n > 0) return SE2_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double *scratch = nullptr;
    SE2_HIP(hipMallocAsync(reinterpret_cast<void **>(&scratch), (2 * static_cast<size_t>(split_blocks(n)) + 2) *
                                                                    sizeof(double), st));
    const int rc = launch_split_signed(u, n, plus, minus, scratch, st);
    SE2_HIP(hipFreeAsync(scratch, st));
    return rc;
}

int se2_split_signed_noalloc(const double *u, size_t n, double *plus, double *minus, se2_stream_t stream) {
    if ((!u || !plus || !minus) && n > 0) return SE2_EINVAL;
    if (split_blocks(n) > kSplitNoallocMaxBlocks) {
        g_last_error = "se2_split_signed_noalloc: n = " + std::to_string(n) + " exceeds the maximum of " +
                       std::to_string(static_cast<size_t>(kSplitNoallocMaxBlocks) * 16384) + " elements";
        return SE2_EINVAL;
    }
    double *scr = nullptr;
    const int rc = split_noalloc_scratch(&scr);
    if (rc) return rc;
    return launch_split_signed(u, n, plus, minus, scr, reinterpret_cast<hipStream_t>(stream));
}

int se2_sinkhorn(se2_kernel_t h, const double *mu, const double *nu, const se2_opts_t *opts, double *f_out,
                 double *g_out, se2_report_t *report, se2_stream_t stream) {
    const Kernel *k = reinterpret_cast<const Kernel *>(h);
    if (!k || !mu || !nu || !valid_opts(opts, k)) return SE2_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const double t0 = now_seconds();
    const size_t E = static_cast<size_t>(k->grid.nx) * k->grid.ny * k->grid.ntheta;
    int rc = validate_measure(mu, E, 1e-9, st);
    if (rc) return rc;
    if ((rc = validate_measure(nu, E, 1e-9, st))) return rc;
    Solve s;
    s.kind = SE2_REQ_OT;
    s.k = k;
    s.opts = *opts;
    s.n = 1;
    s.t_start = t0;
    if ((rc = plan_stages(s, *k))) return rc;
    DeviceBlock mem;
    mem.st = st;
    const size_t bytes = solve_bytes(SE2_REQ_OT, *k, 1, prune_wanted(*opts));
    SE2_HIP(hipMallocAsync(&mem.p, bytes, st));
    solve_bind(s, mem.p);
    if ((rc = solve_setup_ot(s, mu, nu, opts->init_g, st))) return rc;
    Engine eng;
    std::vector<Solve *> one = {&s};
    if ((rc = eng.init_first_halfstep(one, st))) return rc;
    s.convs = 1;
    std::vector<double> errs;
    while (!s.done) {
        const bool last = s.iter + 1 >= opts->max_iter;
        const bool check = last || ((s.iter + 1) % opts->check_every == 0);
        if ((rc = eng.step(one, check, st))) return rc;
        if (check) {
            if ((rc = eng.read_errors(one, errs, st))) return rc;
            s.last_err = errs[0];
            if (!std::isfinite(errs[0])) {
                g_last_error = "non-finite marginal error";
                return SE2_ENUMERIC;
            }
            if (final_stage(s) && opts->tol_marg_l1 >= 0 && errs[0] <= opts->tol_marg_l1) {
                s.done = true;
                s.status = SE2_CONVERGED;
            } else if (last) {
                s.done = true;
                s.status = SE2_MAX_ITER;
            } else {
                s.cur ^= 1;
                phase_after_check(s, errs[0]);
            }
        }
        if (!s.done && (rc = advance_stages(eng, one, st))) return rc;
    }
    std::vector<FinishReq> fin(1);
    fin[0].s = &s;
    fin[0].f_out = f_out;
    fin[0].g_out = g_out;
    if ((rc = finish_solves(eng, fin, st))) return rc;
    if (report) *report = fin[0].rep;
    return fin[0].rc;
}

int se2_jko_step(se2_kernel_t h, const double *mu, const se2_flow_t *flow, const se2_opts_t *opts, double *mu_next,
                 double *f_out, double *g_out, se2_report_t *report, se2_stream_t stream) {
    const Kernel *k = reinterpret_cast<const Kernel *>(h);
    if (!k || !mu || !mu_next || !valid_flow(k, flow, opts)) return SE2_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const size_t E = static_cast<size_t>(k->grid.nx) * k->grid.ny * k->grid.ntheta;
    int rc = validate_measure(mu, E, 1e-9, st);
    if (rc) return rc;
    return jko_run(k, mu, opts->init_g, kLog2e, *flow, *opts, mu_next, f_out, g_out, nullptr, report, st);
}

int se2_gradient_flow(se2_kernel_t h, const double *mu0, const se2_flow_t *flow, int32_t nsteps,
                      const se2_opts_t *opts, double *mu_out, double *traj, se2_report_t *reports,
                      se2_stream_t stream) {
    const Kernel *k = reinterpret_cast<const Kernel *>(h);
    if (!k || !mu0 || !mu_out || nsteps < 1 || !valid_flow(k, flow, opts)) return SE2_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const size_t E = static_cast<size_t>(k->grid.nx) * k->grid.ny * k->grid.ntheta;
    int rc = validate_measure(mu0, E, 1e-9, st);
    if (rc) return rc;
    // current measure, next measure, log b carried between steps (base 2), mass scratch
    const size_t Eb = (E * sizeof(double) + 255) / 256 * 256;
    DeviceBlock mem;
    mem.st = st;
    SE2_HIP(hipMallocAsync(&mem.p, 3 * Eb + (2 + 2 * 256) * sizeof(double), st));
    double *cur = reinterpret_cast<double *>(static_cast<char *>(mem.p));
    double *nxt = reinterpret_cast<double *>(static_cast<char *>(mem.p) + Eb);
    double *psi = reinterpret_cast<double *>(static_cast<char *>(mem.p) + 2 * Eb);
    double *stats = reinterpret_cast<double *>(static_cast<char *>(mem.p) + 3 * Eb);
    SE2_HIP(hipMemcpyAsync(cur, mu0, E * sizeof(double), hipMemcpyDeviceToDevice, st));
    for (int t = 0; t < nsteps; ++t) {
        se2_report_t rep{};
        const double *init = t == 0 ? opts->init_g : psi;
        const double scale = t == 0 ? kLog2e : 1.0;
        if ((rc = jko_run(k, cur, init, scale, *flow, *opts, nxt, nullptr, nullptr, psi, &rep, st))) return rc;
        if (reports) reports[t] = rep;
        // the next step starts from the step's measure scaled to mass one (the inner iterations
        // stop at a tolerance, so its mass is one to within that tolerance)
        if ((rc = launch_normalise(nxt, E, stats, st))) return rc;
        if (traj) SE2_HIP(hipMemcpyAsync(traj + E * t, nxt, E * sizeof(double), hipMemcpyDeviceToDevice, st));
        std::swap(cur, nxt);
    }
    SE2_HIP(hipMemcpyAsync(mu_out, cur, E * sizeof(double), hipMemcpyDeviceToDevice, st));
    SE2_HIP(hipStreamSynchronize(st));
    return SE2_OK;
}

int se2_barycenter(se2_kernel_t h, int32_t n, const double *const *mus, const double *lambdas,
                   const se2_opts_t *opts, double *bary_out, se2_report_t *report, se2_stream_t stream) {
    const Kernel *k = reinterpret_cast<const Kernel *>(h);
    if (!k || n < 1 || n > kMaxMeasures || !mus || !lambdas || !bary_out || !valid_opts(opts, k))
        return SE2_EINVAL;
    double lsum = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!(lambdas[i] >= 0.0) || !std::isfinite(lambdas[i]) || !mus[i]) return SE2_EINVAL;
        lsum += lambdas[i];
    }
    if (!(std::fabs(lsum - 1.0) <= 1e-12)) return SE2_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const double t0 = now_seconds();
    const size_t E = static_cast<size_t>(k->grid.nx) * k->grid.ny * k->grid.ntheta;
    std::vector<const double *> act;
    std::vector<double> lam;
    int rc;
    if ((rc = validate_measures(std::vector<const double *>(mus, mus + n), E, 1e-9, st))) return rc;
    for (int i = 0; i < n; ++i) {
        if (lambdas[i] > 0.0) {
            act.push_back(mus[i]);
            lam.push_back(lambdas[i]);
        }
    }
    Solve s;
    s.kind = SE2_REQ_BARYCENTER;
    s.k = k;
    s.opts = *opts;
    s.n = static_cast<int>(act.size());
    s.lam = lam;
    s.t_start = t0;
    if ((rc = plan_stages(s, *k))) return rc;
    DeviceBlock mem;
    mem.st = st;
    SE2_HIP(hipMallocAsync(&mem.p, solve_bytes(SE2_REQ_BARYCENTER, *k, s.n, prune_wanted(*opts)), st));
    solve_bind(s, mem.p);
    if ((rc = solve_setup_bary(s, act, st))) return rc;
    Engine eng;
    std::vector<Solve *> one = {&s};
    if ((rc = eng.init_first_halfstep(one, st))) return rc;
    s.convs = s.n;
    std::vector<double> errs;
    while (!s.done) {
        const bool last = s.iter + 1 >= opts->max_iter;
        const bool check = last || ((s.iter + 1) % opts->check_every == 0);
        if ((rc = eng.step(one, check, st))) return rc;
        if (check) {
            if ((rc = eng.read_errors(one, errs, st))) return rc;
            s.last_err = errs[0];
            if (!std::isfinite(errs[0])) {
                g_last_error = "non-finite marginal error";
                return SE2_ENUMERIC;
            }
            if (final_stage(s) && opts->tol_marg_l1 >= 0 && errs[0] <= opts->tol_marg_l1) {
                s.done = true;
                s.status = SE2_CONVERGED;
            } else if (last) {
                s.done = true;
                s.status = SE2_MAX_ITER;
            } else {
                phase_after_check(s, errs[0]);
            }
        }
        if (!s.done && (rc = advance_stages(eng, one, st))) return rc;
    }
    std::vector<FinishReq> fin(1);
    fin[0].s = &s;
    fin[0].bary_out = bary_out;
    if ((rc = finish_solves(eng, fin, st))) return rc;
    if (report) *report = fin[0].rep;
    return fin[0].rc;
}

}  // extern "C"
