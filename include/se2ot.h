/*
 * se2ot.h -- C ABI of the MI355X (gfx950) library for entropic optimal transport
 * on the roto-translation group SE(2) = R^2 x| SO(2).
 *
 * The operations follow "Optimal Transport on the Lie Group of Roto-translations"
 * (Bon, Pai, Bellaard, Mula, Duits; arXiv 2402.15322):
 *
 *   se2_kernel_build  Gibbs kernel K(g) = exp(-rho_b(g)^2 / eps) on a window of
 *                     grid offsets; rho_b is the half-angle distance approximation
 *                     of Section 4.3, eqs. (rhob) and (logcomp), with the
 *                     left-invariant metric diag(w1^2, w2^2, w3^2) of Section 2.3.
 *   se2_conv          the group convolution (K * f)(g) = sum_h K(h^-1 g) f(h) of
 *                     Section 4.2 (the operator K b of the scaling iterations).
 *   se2_conv_log      the same operator on log-values: log(K * exp(f)).
 *   se2_sinkhorn      entropic OT between two measures, the Sinkhorn iterations
 *                     a = mu / K b, b = nu / K^T a of Section 4.1 (in log form).
 *   se2_barycenter    the iterative Bregman projections of Appendix A.
 *   se2_solve_queue_* a serving queue that admits OT and barycenter solves by an
 *                     HBM budget and advances all admitted solves together.
 *
 * Discretisation: pixel (ix, iy) sits at (x, y) = (ix, iy) (unit spacing);
 * theta_k = k * Theta / ntheta with Theta = 2*pi, or pi when theta_axial = 1
 * (orientations without direction; the distance on the quotient by the half
 * turn is the smaller of its two lifts).  The kernel is truncated to a square
 * (2r+1)^2 window of grid offsets x_out - x_in with full theta support; the
 * spatial boundary is zero (no wrap) and theta is periodic.  The Haar cell
 * volume is dropped (a constant that the scalings absorb).
 *
 * Layout of every grid array: [batch][iy][ix][k], theta innermost, dense.
 *
 * Pointers: unless stated otherwise, array arguments are HIP DEVICE pointers
 * owned by the caller; the library never frees them and keeps no reference
 * after the call returns (queue requests excepted, see below).
 *
 * Errors: functions return 0 (SE2_OK) or a negative code; se2_strerror() names
 * it.  Invalid arguments are detected before any device work is queued.
 * Non-convergence is not an error: it is reported in se2_report_t.status.
 */
#ifndef SE2OT_H
#define SE2OT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SE2_OK 0
#define SE2_EINVAL (-1)   /* bad argument or input measure (NaN, negative, not normalised) */
#define SE2_ENOMEM (-2)   /* device or host allocation failed, or request exceeds the queue budget */
#define SE2_EHIP (-3)     /* a HIP runtime call failed */
#define SE2_ENUMERIC (-4) /* non-finite value produced (e.g. mass with no partner in the window) */
#define SE2_PENDING 1     /* queue ticket not finished yet */

/* Solve status in se2_report_t.status */
#define SE2_CONVERGED 0
#define SE2_MAX_ITER 1

typedef struct {
    int32_t nx, ny;      /* pixels, >= 1 */
    int32_t ntheta;      /* orientations: 8, 16 or 32 */
    int32_t theta_axial; /* 0: theta in [0, 2 pi); 1: theta in [0, pi) */
} se2_grid_t;

typedef struct {
    double w1, w2, w3; /* metric weights, > 0 (Section 2.3, eq. (metric_SE2)) */
    double eps;        /* entropic regularisation, > 0 (Section 4.1) */
    int32_t radius;    /* window half-width r: offsets |dx|, |dy| <= r, 0 <= r <= 12 */
} se2_metric_t;

/* Arithmetic of a convolution.
 *  SE2_BF16    : se2_conv -- input rounded to bfloat16 (RNE), kernel in bfloat16, products
 *                accumulated in FP32 on the matrix cores (MFMA); float in/out.
 *                Log-domain paths (se2_conv_log and the solvers) -- the certified linear-domain
 *                engine on the matrix cores: per workgroup tile the input is shifted by its
 *                maximum M over the tile's halo, 2^(in - M) is rounded to bfloat16 and
 *                contracted with the bfloat16 kernel (FP32 accumulation), and the log is
 *                M + log S.  An output whose sum S falls below 2^-87 in that frame (where
 *                underflowed terms could matter) has its (8 x 8 tile, orientation) group
 *                recomputed exactly in the log domain (counted in se2_report_t.fallbacks).
 *                Relative error of K * exp(in) about 2^-8 (bfloat16 operands).
 *  SE2_F32     : se2_conv -- FP32 kernel and accumulation (float in/out, on the matrix cores at
 *                ntheta = 16 and 32, on the vector ALUs at 8).  Log-domain paths -- the exact
 *                engine: exponent arguments formed in FP64, FP32 exp2 and FP32 partial sums
 *                combined in FP64 (certified pruning of negligible terms, see prune).
 *  SE2_F64     : FP64 throughout (se2_conv: double in/out).
 *  SE2_F32_MFMA: log-domain paths only, ntheta = 16 or 32 -- the certified linear-domain engine
 *                of SE2_BF16 with FP32 operands on the FP32 matrix cores, FP32 sums over one
 *                step of the contraction (at most 128 products) added in FP64; relative error
 *                of K * exp(in) about 1e-6 at most.                                          */
typedef enum { SE2_BF16 = 0, SE2_F32 = 1, SE2_F64 = 2, SE2_F32_MFMA = 3 } se2_prec_t;

typedef struct {
    double tol_marg_l1;   /* stop when the marginal L1 error <= tol; tol < 0 runs exactly max_iter */
    int32_t max_iter;     /* >= 1 */
    int32_t check_every;  /* iterations between convergence checks (>= 1) */
    se2_prec_t prec;      /* engine of the solve (of its polish phase when polish = 1): SE2_F32 (exact,
                             the default), SE2_F64 (FP64 exp, slow), SE2_BF16 or SE2_F32_MFMA (matrix
                             cores, certified; see se2_prec_t) */
    int32_t final_check;  /* 1: recompute the final marginal error with an FP64 convolution */
    int32_t prune;        /* 1: certified pruning of negligible window entries (results equal the dense
                             sum to 2^-48 relative per skipped entry); 0: every entry, every time */
    const double *init_g; /* device, may be NULL: warm start log b = g/eps (natural log units) at the
                             first eps of the schedule */
    /* eps-scaling (an outer loop around the scaling iterations; not in the paper, it is the
     * published warm-start scheme of Schmitzer, "Stabilized sparse scaling algorithms for
     * entropy regularized transport problems", SIAM J. Sci. Comput. 2019).  With
     * eps_start > eps the solve first runs stage_iters iterations at each of the coarser
     * values eps_start, eps_start*eps_factor, eps_start*eps_factor^2, ... that lie above
     * eps (at most 32 of them), then continues at eps.  Between stages the scalings are
     * carried over in absolute units (g kept, so log b is multiplied by eps_old/eps_new)
     * and the next a-update is taken with the new kernel.  Iterations of every stage count
     * towards max_iter, which must exceed the coarse ones; the stopping test applies at eps
     * only.  eps_start <= eps (e.g. 0) switches the scheme off and the other two fields are
     * ignored.  Kernels at the coarser values are built once per kernel handle and kept
     * with it. */
    double eps_start;
    double eps_factor;    /* in (0, 1) */
    int32_t stage_iters;  /* >= 1 */
    /* Phases.  polish = 0: the solve runs on `prec` throughout (bulk and switch_tol ignored).
     * polish = 1: a bulk phase on the engine `bulk` (typically SE2_BF16) comes first -- over
     * the coarse eps stages and at the final eps.  The solve moves to `prec` at the first
     * check after which more than a quarter (three quarters when `prec` visits whole
     * windows: prune = 0, or a halo beyond the pruned kernel's LDS) of the (tile, orientation)
     * groups the bulk engine visited since the previous check were recomputed exactly (any
     * stage), or, at the final eps, whose marginal L1 error is <= switch_tol or did not fall
     * since the previous check of that stage (the bulk engine's precision floor); the final
     * FP64 check (final_check) follows as usual.  se2_report_t.phase_switch_iter records the
     * move. */
    se2_prec_t bulk;
    int32_t polish;
    double switch_tol;
} se2_opts_t;

typedef struct {
    int32_t status;     /* SE2_CONVERGED, SE2_MAX_ITER */
    int32_t iters;      /* iterations done by the returned iterate (every eps stage) */
    double marg_l1;     /* L1 error of the non-exact marginal(s) of the returned iterate */
    double marg_l1_f64; /* same, from an FP64 convolution (final_check = 1), else -1 */
    double cost;        /* sum pi * rho_b^2 (OT) or sum_i lambda_i <pi_i, rho_b^2> (barycenter) */
    double mass;        /* total mass of the plan (OT) or of the barycenter */
    double dual;        /* <f, mu> + <g, nu> (OT only, diagnostic) */
    double seconds;     /* wall time of the solve on the host clock */
    double terms_dense;  /* in-grid window terms evaluated by dense convolution visits */
    double terms_sparse; /* list entries evaluated by certified sparse visits (per output) */
    int32_t convs;      /* group convolutions applied */
    int32_t scaling_iters; /* iterations run at coarser eps (eps-scaling), included in iters */
    int32_t fallbacks;  /* (8 x 8 tile, orientation) groups that the matrix-core engines recomputed in
                           the log domain after a failed certificate, summed over the measures;
                           saturates at 2^31 - 1 (each measure's count is kept modulo 2^32) */
    int32_t phase_switch_iter; /* iteration at which the polish phase began (-1: never) */
    double terms_linear; /* window terms evaluated on the matrix cores (SE2_BF16, SE2_F32_MFMA) */
} se2_report_t;

typedef struct se2_kernel_s *se2_kernel_t; /* library-owned, immutable, usable from any thread */
typedef struct se2_queue_s *se2_queue_t;
typedef void *se2_stream_t;                /* a hipStream_t; NULL = the default stream */

/* Library version and device check.  Returns 0 if a gfx950 device is current. */
int se2_init(void);
const char *se2_strerror(int code);

/*
 * se2_kernel_build -- tabulate the Gibbs kernel on the window (Sections 4.2, 4.3).
 * For each offset d = (dx, dy), |dx|,|dy| <= r, and orientation pair (ko, ki):
 *     logK[d][ko][ki] = -rho_b(h^-1 g)^2 / eps,   h = (x, theta_ki), g = (x + d, theta_ko),
 *     h^-1 g = (R_{-theta_ki} d, theta_ko - theta_ki)    (group law of Section 2.3).
 * Tables are built on the host in FP64 and uploaded once (FP64 log-kernel, FP64
 * cost rho_b^2, FP32 and bfloat16 kernels for se2_conv).  The handle is
 * immutable and may be shared by concurrent solves.  Uses the current device.
 */
int se2_kernel_build(const se2_grid_t *grid, const se2_metric_t *metric, se2_kernel_t *out);
int se2_kernel_destroy(se2_kernel_t k);

/* Copy the FP64 tables to HOST memory, layout [dy+r][dx+r][ko][ki], natural log
 * units: host_logk = -rho_b^2/eps, host_cost = rho_b^2 (either may be NULL).
 * Each must hold (2r+1)^2 * ntheta^2 doubles. */
int se2_kernel_table(se2_kernel_t k, double *host_logk, double *host_cost);

/* Grid and window of a kernel (any pointer may be NULL). */
int se2_kernel_info(se2_kernel_t k, se2_grid_t *grid, se2_metric_t *metric, int32_t *window_nonzero_bf16);

/*
 * se2_conv -- out[b] = K * in[b] for b < batch (Section 4.2), stream-ordered,
 * no host synchronisation.  SE2_BF16 and SE2_F32 read/write float arrays (in
 * 16-byte aligned, else SE2_EINVAL), SE2_F64 double arrays; each is
 * batch * nx * ny * ntheta elements.  in and out must not overlap.
 */
int se2_conv(se2_kernel_t k, se2_prec_t prec, const void *in, void *out, int32_t batch, se2_stream_t stream);

/*
 * se2_conv_log -- out[b] = log(K * exp(in[b])) in natural-log units, FP64 in and
 * out (-inf allowed: zero mass), the log form of the operator applied in every
 * Sinkhorn half-step.  prec SE2_F32: FP64 exponent arguments, FP32 exp2 and
 * partial sums, FP64 combination; SE2_F64: FP64 throughout; SE2_BF16 and
 * SE2_F32_MFMA: the certified linear-domain engines on the matrix cores (see
 * se2_prec_t; SE2_F32_MFMA needs ntheta = 16 or 32).  fallbacks (HOST, may be NULL)
 * receives the number of (8 x 8 tile, orientation) groups recomputed in the log domain
 * (0 for SE2_F32 and SE2_F64).  Takes a scratch with hipMallocAsync on `stream` and
 * synchronises the stream before it returns (its job tables are staged from the host).
 */
int se2_conv_log(se2_kernel_t k, se2_prec_t prec, const double *in, double *out, int32_t batch,
                 int32_t *fallbacks, se2_stream_t stream);

/*
 * se2_sinkhorn -- entropic OT between mu and nu (Section 4.1), log form:
 *     f/eps <- log mu - log K exp(g/eps),   g/eps <- log nu - log K exp(f/eps),
 * starting from g = init_g (0 if NULL); K^T = K because rho_b(g^-1) = rho_b(g).
 * mu, nu: device FP64 probability vectors (finite, >= 0, |sum - 1| <= 1e-9).
 * f_out, g_out: device FP64 (may be NULL) receive f = eps log a, g = eps log b
 * of the returned iterate (-inf where the mass is zero).  The plan is
 * pi(x, y) = exp((f(x) + g(y) - rho_b^2(x, y)) / eps) on the window; it is never
 * materialised.  Blocks the calling thread until the solve is done (the work is
 * queued on `stream`).  report may be NULL.
 */
int se2_sinkhorn(se2_kernel_t k, const double *mu, const double *nu, const se2_opts_t *opts,
                 double *f_out, double *g_out, se2_report_t *report, se2_stream_t stream);

/*
 * se2_barycenter -- entropic Wasserstein barycenter of n measures with weights
 * lambda (Appendix A, iterative Bregman projections), log form.  1 <= n <= 65535: the
 * convolutions of all measures go out in one batched launch per half-step, and the
 * product of the d_i^lambda_i is summed in index order within chunks of 64 measures,
 * then over the chunks in order.
 * mus: HOST array of n device pointers to FP64 probability vectors;
 * lambdas: HOST array of n weights on the simplex (>= 0, |sum - 1| <= 1e-12);
 * bary_out: device FP64 grid array receiving the barycenter.  Measures with
 * lambda_i = 0 do not enter the barycenter and are skipped.  Blocking.
 */
int se2_barycenter(se2_kernel_t k, int32_t n, const double *const *mus, const double *lambdas,
                   const se2_opts_t *opts, double *bary_out, se2_report_t *report, se2_stream_t stream);

/*
 * se2_jko_step -- one step of the entropic JKO scheme for the Wasserstein gradient flow of
 * the porous-medium energy (Section 5.4, eqs. (GF_JKO) and (cost_GF), with the equation
 * d mu / dt = Laplacian_G mu^m of eq. (pde_ndiff)):
 *     mu_next = argmin_nu  W_eps(mu, nu) + tau F(nu),   F(nu) = ref/(m-1) sum_x (nu(x)/ref)^m,
 * where W_eps is the entropic transport cost of Section 4.1 with this kernel's cost rho_b^2
 * and ref is the measure of one grid cell against which densities are taken (the paper's
 * integral of the density to the power m; e.g. 1/(nx ny ntheta) for a domain of volume 1).
 * Solved with the entropic scheme the paper cites (Peyre 2015): the scaling iterations
 *     a = mu / K b,   b = prox^KL_{tau F / eps}(K^T a) / K^T a,
 * in log form, the proximal step solved per element (see the kernels).  Stops as
 * se2_sinkhorn does on the L1 error of the first marginal (the second marginal is free: it
 * is mu_next).  opts->init_g warm-starts log b (e.g. from the previous step of a flow);
 * eps-scaling is not available here (eps_start must be <= eps).
 * mu: device FP64 probability vector; mu_next (device, required) receives
 * nu = b K^T a of the returned iterate; f_out, g_out as in se2_sinkhorn (may be NULL).
 * report->cost is the transport cost of the plan, report->mass its mass, report->dual
 * holds F(mu_next).  SE2_EINVAL for tau < 0, m <= 1, ref <= 0 or non-finite values.
 * Blocking.
 */
typedef struct {
    double tau; /* time step, >= 0 (0: the entropic blur of mu, K^T (mu / K 1)) */
    double m;   /* exponent, > 1 (the paper's experiments use 5) */
    double ref; /* reference cell measure, > 0 */
} se2_flow_t;
int se2_jko_step(se2_kernel_t k, const double *mu, const se2_flow_t *flow, const se2_opts_t *opts, double *mu_next,
                 double *f_out, double *g_out, se2_report_t *report, se2_stream_t stream);

/*
 * se2_gradient_flow -- nsteps JKO steps from mu0 (the time marching of Section 2.2,
 * eq. (GF_JKO), for the energy of se2_jko_step), all on the device: step t starts from the
 * measure of step t-1 scaled to mass one (the inner iterations stop at a tolerance) and from
 * its log b (step 0 from opts->init_g).  mu_out (device, required) receives the last
 * measure; traj (device, may be NULL) receives every step's measure, [nsteps][grid];
 * reports (HOST array of nsteps, may be NULL) one report per step.  Blocking.
 */
int se2_gradient_flow(se2_kernel_t k, const double *mu0, const se2_flow_t *flow, int32_t nsteps,
                      const se2_opts_t *opts, double *mu_out, double *traj, se2_report_t *reports,
                      se2_stream_t stream);

/*
 * Lift and projection around the transport path.  Grid arrays as above, 16-byte aligned
 * (SE2_EINVAL otherwise); images and fields are [batch][iy][ix].  Stream-ordered, no host
 * synchronisation.
 *
 * se2_lift_field -- the orientation-field lift of Section 5.3, eq. (lifting_vector_field):
 *   out(x, y, theta_k) = mag(x, y) in the orientation bin of angle(x, y), 0 in the others.
 *   The bin of an angle a is the k nearest to a on the circle of circumference Theta
 *   (theta_k = k Theta / ntheta; a at a bin edge goes to the upper bin), i.e. the bin
 *   with circular distance below half a step (the paper's pi/N for Theta = 2 pi).  mag
 *   (>= 0) and angle (radians, any finite value) are batch * nx * ny doubles; out holds
 *   batch * nx * ny * ntheta doubles.  Mass is preserved.
 *
 * se2_project -- the projection P(U) = integral of U over theta (Section 2.3, eq. (proj)),
 *   for arrays of mass per grid cell the sum over the orientation bins, and the argmax
 *   reconstruction of Section 5.3, eq. (reconstruction_vector_field):
 *     mass(x, y)   = sum_k u(x, y, k) - sum_k u_minus(x, y, k)   (u_minus may be NULL;
 *                    with both, the difference of projections b_t = P(U+) - P(U-) of
 *                    Section 5.2, eq. (final));
 *     argmax(x, y) = the k of the largest u(x, y, k), the lowest such k on ties (may be NULL);
 *     angle(x, y)  = theta_argmax = argmax * Theta / ntheta (may be NULL).
 *   The field is v = mass * (cos angle, sin angle).  u, u_minus: batch * nx * ny * ntheta
 *   doubles; mass, angle: batch * nx * ny doubles; argmax: batch * nx * ny int32.
 *
 * se2_split_signed -- step 2 of the image pipeline of Section 5.2: the positive and
 *   negative parts of a signed array u of n doubles, each normalised to sum 1 (FP64 sums
 *   in a fixed order): plus = max(u, 0) / sum max(u, 0), minus = max(-u, 0) / sum max(-u, 0);
 *   a part with zero sum is returned as zeros.  Allocates and frees a small scratch
 *   stream-ordered (hipMallocAsync / hipFreeAsync on `stream`).
 */
int se2_lift_field(const se2_grid_t *grid, const double *mag, const double *angle, double *out, int32_t batch,
                   se2_stream_t stream);
int se2_project(const se2_grid_t *grid, const double *u, const double *u_minus, double *mass, int32_t *argmax,
                double *angle, int32_t batch, se2_stream_t stream);
int se2_split_signed(const double *u, size_t n, double *plus, double *minus, se2_stream_t stream);

/*
 * se2_split_signed_noalloc -- se2_split_signed without any allocation, for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc.  Same arguments, kernels and results (bitwise) as
 * se2_split_signed; the partial sums go to a scratch array that the library holds on each
 * GPU it runs on (64 KiB, kept until the process ends; its address is looked up once per
 * device, by se2_init or by the first call on that device).  n is limited to
 * 4096 * 16384 = 67,108,864 elements: larger n returns SE2_EINVAL before any device work.
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one GPU (on
 * different streams, or from several threads without ordering) race and must not be
 * issued.  Nothing in the scratch needs clearing: each call writes every value it reads.
 * Stream-ordered, no host synchronisation.
 */
int se2_split_signed_noalloc(const double *u, size_t n, double *plus, double *minus, se2_stream_t stream);

/*
 * Serving queue.  Three lanes, each a worker thread with its own stream on the current
 * device.  A request goes at submit to the lane with the least outstanding work and is
 * admitted, in arrival order within its lane, while the HBM budget and the slot count
 * (shared by the lanes) allow; every admitted solve keeps its potentials resident and
 * the solves of a lane advance together, one batched launch per half-step and (ntheta)
 * class; the lanes run independently and their launches overlap on the GPU.
 * A solve's arithmetic (tiling, reduction order) does not depend on what else is
 * admitted, so its result is bitwise the same alone or in a mix.
 */
#define SE2_REQ_OT 0
#define SE2_REQ_BARYCENTER 1

typedef struct {
    int32_t kind;               /* SE2_REQ_OT or SE2_REQ_BARYCENTER */
    int32_t n;                  /* barycenter: number of measures, 1 ... 65535 */
    se2_kernel_t kernel;        /* must outlive the request */
    const double *mu, *nu;      /* OT: device inputs, copied into slot memory at admission */
    const double *const *mus;   /* barycenter: host array of n device pointers, copied at admission */
    const double *lambdas;      /* barycenter: host weights, copied at submit */
    se2_opts_t opts;            /* init_g ignored */
    double *f_out, *g_out;      /* OT outputs (device, may be NULL); must stay valid until done */
    double *bary_out;           /* barycenter output (device) */
} se2_request_t;

/* Device bytes a request occupies in the queue while it is resident (inputs, potentials,
 * pruning state); a request with more bytes than the budget is rejected at submit. */
int se2_request_bytes(const se2_request_t *req, size_t *bytes);
int se2_solve_queue_create(size_t hbm_budget_bytes, int32_t max_slots, se2_queue_t *out);
/* Non-blocking.  SE2_ENOMEM if the request alone exceeds the budget. */
int se2_solve_queue_submit(se2_queue_t q, const se2_request_t *req, uint64_t *ticket);
/* SE2_PENDING while running; 0 and the report once done; a negative code if the solve failed. */
int se2_solve_queue_poll(se2_queue_t q, uint64_t ticket, se2_report_t *report);
int se2_solve_queue_wait(se2_queue_t q, uint64_t ticket, se2_report_t *report);
/* Timestamps (host steady clock, seconds) of submit, admission and completion. */
int se2_solve_queue_times(se2_queue_t q, uint64_t ticket, double *t_submit, double *t_admit, double *t_done);
/* Forget a finished ticket: its report and times are dropped and the ticket becomes invalid
 * (SE2_EINVAL afterwards).  SE2_PENDING (nothing dropped) while the solve runs.  A queue keeps
 * every finished ticket until it is released or the queue is destroyed, so a long-running
 * serving loop releases each ticket once it has read the report and times; no other call
 * on the same ticket may be in progress. */
int se2_solve_queue_release(se2_queue_t q, uint64_t ticket);
/* Counters: admitted, completed, rejected, peak slots in use, batched steps run. */
int se2_solve_queue_stats(se2_queue_t q, int64_t *out5);
/* Kernel timing of the queue's log-domain convolutions, measured with HIP events on
 * the queue's own streams (diagnostics for benchmarks; recording adds two event records
 * per launch and event reads at every check).  enable = 1 starts recording (and zeroes
 * the totals), enable = 0 stops it; out4 receives, for the launches recorded up to the
 * last check of each lane, [seconds during which any convolution launch of the queue ran
 * (the union of the launch intervals of its streams, formed by this call), algorithmic
 * LSE terms (window entries inside the grid), batched half-steps issued (two per
 * iteration of the resident solves), output elements]. */
int se2_solve_queue_profile(se2_queue_t q, int32_t enable);
int se2_solve_queue_kernel_time(se2_queue_t q, double *out4);
/* Waits for all submitted work, then frees the queue. */
int se2_solve_queue_destroy(se2_queue_t q);

#ifdef __cplusplus
}
#endif
#endif /* SE2OT_H */
