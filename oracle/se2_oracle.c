/*
 * se2_oracle.c -- plain FP64 CPU oracle for entropic optimal transport on SE(2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; it exists so the tests, the smoke check and the CPU-baseline leg of
 * the benchmark can compare the GPU library against an obviously correct
 * reference.  It shares no source with the GPU path.
 *
 * Everything is FP64 and in the log domain (the paper's scaling iterations in
 * log form: identical in exact arithmetic, needed because exp(-rho^2/eps)
 * underflows FP64 for most window entries at the target eps).  The loops follow
 * the paper's definitions with no blocking, fusion or reordering:
 *
 *   group law, inverse          Section 2.3 (fixed coordinates, theta in [-pi,pi))
 *   half-angle distance rho_b   Section 4.3, eqs. (rhob) and (logcomp)
 *   group convolution K * f     Section 4.2, (K*f)(g) = sum_h K(h^-1 g) f(h)
 *   Sinkhorn                    Section 4.1, a = mu / K b, b = nu / K^T a
 *   IBP barycenter              Appendix A (SE(2) Wasserstein barycenter algorithm)
 *   plan and transport cost     Section 4.1 (pi = a K b) and Section 2.2 (L^{W_p})
 *
 * Discretisation (readings where the paper is silent):
 *   pixel (ix,iy) sits at (x,y) = (ix,iy); theta_k = k*Theta/nt, Theta = 2*pi, or
 *   pi for axial grids; zero spatial boundary; theta periodic; the Haar cell
 *   volume is dropped (a constant absorbed by the scalings); the kernel is
 *   truncated to a square (2R+1)^2 window on the grid offset x_out - x_in with
 *   full theta support.  For axial grids the distance on the quotient by the
 *   half-turn is the smaller of the two lifts of the angle difference.
 *
 * Arrays are [iy][ix][k] with k (theta) innermost.  Kernel tables are
 * [dy+R][dx+R][ko][ki] with (dx,dy) = output pixel minus input pixel.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI = 3.14159265358979323846;

/* Representative of an angle in the small-angle convention [-pi, pi). */
static double wrap_angle(double t)
{
    double r = fmod(t + PI, 2.0 * PI);
    if (r < 0.0) r += 2.0 * PI;
    return r - PI;
}

/* Half-angle coordinates b(g) of g = (x, y, theta), Section 4.3 eq. (logcomp). */
void oc_half_angle(double x, double y, double theta, double *b)
{
    double t = wrap_angle(theta);
    double c = cos(0.5 * t), s = sin(0.5 * t);
    b[0] = x * c + y * s;
    b[1] = -x * s + y * c;
    b[2] = t;
}

/* rho_b(g)^2 = sum_i (w_i b^i(g))^2, Section 4.3 eq. (rhob). */
double oc_rho2(double x, double y, double theta, double w1, double w2, double w3)
{
    double b[3];
    oc_half_angle(x, y, theta, b);
    return (w1 * b[0]) * (w1 * b[0]) + (w2 * b[1]) * (w2 * b[1]) + (w3 * b[2]) * (w3 * b[2]);
}

/* h^{-1} g for h = (xh, yh, th), g = (xg, yg, tg): (R_{-th}(xg - xh, yg - yh), tg - th),
 * from the group law and inverse of Section 2.3. */
static void rel_element(double dx, double dy, double th, double tg, double *out)
{
    double c = cos(th), s = sin(th);
    out[0] = c * dx + s * dy;
    out[1] = -s * dx + c * dy;
    out[2] = tg - th;
}

/* Squared distance between input h=(x_i, theta_ki) and output g=(x_i+delta, theta_ko). */
static double pair_rho2(int dx, int dy, int ko, int ki, int nt, int axial, double w1, double w2, double w3)
{
    double period = axial ? PI : 2.0 * PI;
    double th_i = period * ki / nt, th_o = period * ko / nt;
    double r[3];
    rel_element((double)dx, (double)dy, th_i, th_o, r);
    double d2 = oc_rho2(r[0], r[1], r[2], w1, w2, w3);
    if (axial) {
        double d2b = oc_rho2(r[0], r[1], r[2] + PI, w1, w2, w3);
        if (d2b < d2) d2 = d2b;
    }
    return d2;
}

/* Kernel tables over the window: logk = -rho^2/eps and cost = rho^2 (either may be NULL).
 * Gibbs kernel K = exp(-rho_b^2/eps), Section 4.2 and Appendix A. */
void oc_kernel_table(int nt, int axial, double w1, double w2, double w3, double eps, int R,
                     double *logk, double *cost)
{
    int W = 2 * R + 1;
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx)
            for (int ko = 0; ko < nt; ++ko)
                for (int ki = 0; ki < nt; ++ki) {
                    size_t idx = ((((size_t)(dy + R) * W + (dx + R)) * nt + ko) * nt + ki);
                    double d2 = pair_rho2(dx, dy, ko, ki, nt, axial, w1, w2, w3);
                    if (logk) logk[idx] = -d2 / eps;
                    if (cost) cost[idx] = d2;
                }
}

/* log-sum-exp of n terms (-inf terms contribute nothing; all -inf gives -inf). */
static double lse(const double *t, int n)
{
    double m = -INFINITY;
    for (int j = 0; j < n; ++j) if (t[j] > m) m = t[j];
    if (m == -INFINITY) return -INFINITY;
    double s = 0.0;
    for (int j = 0; j < n; ++j) if (t[j] != -INFINITY) s += exp(t[j] - m);
    return m + log(s);
}

/* out(x, ko) = log sum_{y in window, ki} exp(logk[x-y, ko, ki] + in(y, ki)):
 * the group convolution of Section 4.2 applied to exp(in), returned as a log. */
void oc_conv_log(int nx, int ny, int nt, int R, const double *logk, const double *in, double *out)
{
    int W = 2 * R + 1;
    int nterm = W * W * nt;
#pragma omp parallel
    {
        double *t = (double *)malloc(sizeof(double) * (size_t)nterm);
#pragma omp for collapse(2) schedule(static)
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix)
                for (int ko = 0; ko < nt; ++ko) {
                    int n = 0;
                    for (int dy = -R; dy <= R; ++dy) {
                        int jy = iy - dy;
                        if (jy < 0 || jy >= ny) continue;
                        for (int dx = -R; dx <= R; ++dx) {
                            int jx = ix - dx;
                            if (jx < 0 || jx >= nx) continue;
                            const double *kr = logk + ((((size_t)(dy + R) * W + (dx + R)) * nt + ko) * nt);
                            const double *fr = in + (((size_t)jy * nx + jx) * nt);
                            for (int ki = 0; ki < nt; ++ki) t[n++] = kr[ki] + fr[ki];
                        }
                    }
                    out[((size_t)iy * nx + ix) * nt + ko] = lse(t, n);
                }
        free(t);
    }
}

/* Linear group convolution out = K * in with K = exp(logk), for small pinned cases. */
void oc_conv_linear(int nx, int ny, int nt, int R, const double *logk, const double *in, double *out)
{
    int W = 2 * R + 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix)
            for (int ko = 0; ko < nt; ++ko) {
                double s = 0.0;
                for (int dy = -R; dy <= R; ++dy) {
                    int jy = iy - dy;
                    if (jy < 0 || jy >= ny) continue;
                    for (int dx = -R; dx <= R; ++dx) {
                        int jx = ix - dx;
                        if (jx < 0 || jx >= nx) continue;
                        const double *kr = logk + ((((size_t)(dy + R) * W + (dx + R)) * nt + ko) * nt);
                        const double *fr = in + (((size_t)jy * nx + jx) * nt);
                        for (int ki = 0; ki < nt; ++ki) s += exp(kr[ki]) * fr[ki];
                    }
                }
                out[((size_t)iy * nx + ix) * nt + ko] = s;
            }
}

/* sum_x mu(x) |exp(p_old(x) - p_new(x)) - 1|: the L1 distance between mu and the
 * first marginal of the plan built from p_old, given p_new = log mu - log(K b). */
static double marginal_gap(size_t n, const double *logmu, const double *p_old, const double *p_new)
{
    double e = 0.0;
    for (size_t i = 0; i < n; ++i) {
        if (logmu[i] == -INFINITY) continue;
        e += exp(logmu[i]) * fabs(expm1(p_old[i] - p_new[i]));
    }
    return e;
}

/* p = logm - c elementwise, with log 0 giving -inf whatever c is. */
static void scaling_update(size_t n, const double *logm, const double *c, double *p)
{
    for (size_t i = 0; i < n; ++i)
        p[i] = (logm[i] == -INFINITY) ? -INFINITY : logm[i] - c[i];
}

/*
 * Sinkhorn in log form (Section 4.1):
 *   phi_{l+1} = log mu - log K exp(psi_l),   psi_{l+1} = log nu - log K^T exp(phi_{l+1}),
 * with phi = f/eps = log a, psi = g/eps = log b, psi_0 = psi_init (0 if NULL) and
 * K^T = K (the distance is symmetric).  After iteration l the pair (phi_l, psi_l)
 * meets the second marginal exactly; err_l is its first-marginal L1 error, read off
 * the next a-update.  Stops at the first l with err_l <= tol, or at l = max_iter
 * (tol < 0 runs exactly max_iter iterations).  Returns (phi_l, psi_l), the
 * iteration count and err_l; err_hist (may be NULL) receives err_1..err_l.
 */
int oc_sinkhorn(int nx, int ny, int nt, int R, const double *logk,
                const double *logmu, const double *lognu, const double *psi_init,
                int max_iter, double tol, double *phi, double *psi,
                double *err_hist, double *err_out)
{
    size_t n = (size_t)nx * ny * nt;
    double *c = (double *)malloc(sizeof(double) * n);
    double *phi_next = (double *)malloc(sizeof(double) * n);
    if (!c || !phi_next) { free(c); free(phi_next); return -1; }
    for (size_t i = 0; i < n; ++i) psi[i] = psi_init ? psi_init[i] : 0.0;
    oc_conv_log(nx, ny, nt, R, logk, psi, c);
    scaling_update(n, logmu, c, phi);
    int l = 0;
    double err = INFINITY;
    while (l < max_iter) {
        ++l;
        oc_conv_log(nx, ny, nt, R, logk, phi, c);
        scaling_update(n, lognu, c, psi);
        oc_conv_log(nx, ny, nt, R, logk, psi, c);
        scaling_update(n, logmu, c, phi_next);
        err = marginal_gap(n, logmu, phi, phi_next);
        if (err_hist) err_hist[l - 1] = err;
        if (err <= tol || l == max_iter) break;
        memcpy(phi, phi_next, sizeof(double) * n);
    }
    if (err_out) *err_out = err;
    free(c);
    free(phi_next);
    return l;
}

/*
 * Iterative Bregman projections for the barycenter (Appendix A), in log form with
 * lv_i = log v_i, lw_i = log w_i, ld_i = log d_i:
 *   lw_i = log mu_i - log K*exp(lv_i)
 *   ld_i = lv_i + log K*exp(lw_i)
 *   log bar = sum_i lambda_i ld_i          (fixed i order)
 *   lv_i += log bar - ld_i                 (lv_i = -inf where bar = 0)
 * Measures with lambda_i = 0 never enter bar (d_i^0 = 1) and are skipped.
 * err_j = max_i sum_x mu_i |exp(lw_i^(j) - lw_i^(j+1)) - 1| is the mu_i-side
 * marginal error of iterate j (the barycenter side is exact after the v-update),
 * read off the next w-update.  Stops at the first j with err_j <= tol or at
 * j = max_iter.  logbar receives log of iterate j's barycenter.
 * logmus: the nmeas log-measures back to back.  lv_init (may be NULL: all zero, v = 1
 * as in Appendix A) starts the lv_i; lv_out (may be NULL) receives the lv_i of iterate j.
 * Returns the iteration count, or -1 when max_iter < 1 or memory runs out.
 */
int oc_ibp(int nx, int ny, int nt, int R, const double *logk, int nmeas,
           const double *logmus, const double *lambdas, int max_iter, double tol,
           double *logbar, double *err_hist, double *err_out,
           const double *lv_init, double *lv_out)
{
    size_t n = (size_t)nx * ny * nt;
    if (max_iter < 1) return -1;
    double *lv = (double *)malloc(sizeof(double) * n * nmeas);
    double *lw = (double *)malloc(sizeof(double) * n * nmeas);
    double *ld = (double *)malloc(sizeof(double) * n * nmeas);
    double *c = (double *)malloc(sizeof(double) * n);
    double *lw_new = (double *)malloc(sizeof(double) * n);
    if (!lv || !lw || !ld || !c || !lw_new) {
        free(lv); free(lw); free(ld); free(c); free(lw_new);
        return -1;
    }
    for (size_t i = 0; i < n * nmeas; ++i) { lv[i] = lv_init ? lv_init[i] : 0.0; lw[i] = 0.0; }
    int j = 0;
    double err = INFINITY;
    for (int it = 1; it <= max_iter + 1; ++it) {
        /* w-updates; for it > 1 they also measure the error of iterate it-1 */
        double e = 0.0;
        for (int m = 0; m < nmeas; ++m) {
            if (lambdas[m] == 0.0) continue;
            const double *lmu = logmus + n * m;
            oc_conv_log(nx, ny, nt, R, logk, lv + n * m, c);
            scaling_update(n, lmu, c, lw_new);
            if (it > 1) {
                double em = marginal_gap(n, lmu, lw + n * m, lw_new);
                if (!(em <= e)) e = em; /* the largest error; a NaN one is reported as NaN */
            }
            memcpy(lw + n * m, lw_new, sizeof(double) * n);
        }
        if (it > 1) {
            err = e;
            if (err_hist) err_hist[j - 1] = err;
            if (err <= tol || j == max_iter) break;
        }
        /* d-updates and the barycenter */
        for (size_t i = 0; i < n; ++i) logbar[i] = 0.0;
        for (int m = 0; m < nmeas; ++m) {
            if (lambdas[m] == 0.0) continue;
            oc_conv_log(nx, ny, nt, R, logk, lw + n * m, c);
            for (size_t i = 0; i < n; ++i) {
                double v = lv[n * m + i];
                ld[n * m + i] = (v == -INFINITY || c[i] == -INFINITY) ? -INFINITY : v + c[i];
                logbar[i] += lambdas[m] * ld[n * m + i];
            }
        }
        /* v-updates */
        for (int m = 0; m < nmeas; ++m) {
            if (lambdas[m] == 0.0) continue;
            for (size_t i = 0; i < n; ++i) {
                if (logbar[i] == -INFINITY) lv[n * m + i] = -INFINITY;
                else lv[n * m + i] += logbar[i] - ld[n * m + i];
            }
        }
        j = it;
    }
    if (err_out) *err_out = err;
    if (lv_out) memcpy(lv_out, lv, sizeof(double) * n * nmeas);
    free(lv); free(lw); free(ld); free(c); free(lw_new);
    return j;
}

/*
 * Plan diagnostics from log-scalings (phi, psi):
 *   pi(x,y) = exp(phi(x) + logk(x,y) + psi(y))  (Section 4.1, plan from the scalings),
 *   cost    = sum_{x,y} pi(x,y) rho^2(x,y)       (Section 2.2, L^{W_2} with c = rho_b^2),
 *   mass    = sum pi,  marg1 = sum_y pi(.,y),  marg2 = sum_x pi(x,.).
 * Any output pointer may be NULL.
 */
void oc_plan_stats(int nx, int ny, int nt, int R, const double *logk, const double *cost_tab,
                   const double *phi, const double *psi, double *cost, double *mass,
                   double *marg1, double *marg2)
{
    int W = 2 * R + 1;
    size_t n = (size_t)nx * ny * nt;
    double tc = 0.0, tm = 0.0;
    if (marg2) memset(marg2, 0, sizeof(double) * n);
    /* marg1 and the sums: rows are independent */
#pragma omp parallel for collapse(2) reduction(+ : tc, tm) schedule(static)
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix)
            for (int ko = 0; ko < nt; ++ko) {
                size_t xo = ((size_t)iy * nx + ix) * nt + ko;
                double row = 0.0, rc = 0.0;
                if (phi[xo] != -INFINITY) {
                    for (int dy = -R; dy <= R; ++dy) {
                        int jy = iy - dy;
                        if (jy < 0 || jy >= ny) continue;
                        for (int dx = -R; dx <= R; ++dx) {
                            int jx = ix - dx;
                            if (jx < 0 || jx >= nx) continue;
                            size_t kb = (((size_t)(dy + R) * W + (dx + R)) * nt + ko) * nt;
                            size_t yb = ((size_t)jy * nx + jx) * nt;
                            for (int ki = 0; ki < nt; ++ki) {
                                double p = exp(phi[xo] + logk[kb + ki] + psi[yb + ki]);
                                row += p;
                                if (cost_tab) rc += p * cost_tab[kb + ki];
                            }
                        }
                    }
                }
                if (marg1) marg1[xo] = row;
                tm += row;
                tc += rc;
            }
    if (marg2) {
        /* column sums, same terms, gathered per input element */
#pragma omp parallel for collapse(2) schedule(static)
        for (int jy = 0; jy < ny; ++jy)
            for (int jx = 0; jx < nx; ++jx)
                for (int ki = 0; ki < nt; ++ki) {
                    size_t yi = ((size_t)jy * nx + jx) * nt + ki;
                    double col = 0.0;
                    if (psi[yi] != -INFINITY) {
                        for (int dy = -R; dy <= R; ++dy) {
                            int iy = jy + dy;
                            if (iy < 0 || iy >= ny) continue;
                            for (int dx = -R; dx <= R; ++dx) {
                                int ix = jx + dx;
                                if (ix < 0 || ix >= nx) continue;
                                for (int ko = 0; ko < nt; ++ko) {
                                    size_t kb = (((size_t)(dy + R) * W + (dx + R)) * nt + ko) * nt;
                                    size_t xo = ((size_t)iy * nx + ix) * nt + ko;
                                    col += exp(phi[xo] + logk[kb + ki] + psi[yi]);
                                }
                            }
                        }
                    }
                    marg2[yi] = col;
                }
    }
    if (cost) *cost = tc;
    if (mass) *mass = tm;
}

/* sum_{x,y} |pi_a(x,y) - pi_b(x,y)| over the window for two pairs of log-scalings. */
double oc_plan_l1(int nx, int ny, int nt, int R, const double *logk,
                  const double *phi_a, const double *psi_a, const double *phi_b, const double *psi_b)
{
    int W = 2 * R + 1;
    double tot = 0.0;
#pragma omp parallel for collapse(2) reduction(+ : tot) schedule(static)
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix)
            for (int ko = 0; ko < nt; ++ko) {
                size_t xo = ((size_t)iy * nx + ix) * nt + ko;
                for (int dy = -R; dy <= R; ++dy) {
                    int jy = iy - dy;
                    if (jy < 0 || jy >= ny) continue;
                    for (int dx = -R; dx <= R; ++dx) {
                        int jx = ix - dx;
                        if (jx < 0 || jx >= nx) continue;
                        size_t kb = (((size_t)(dy + R) * W + (dx + R)) * nt + ko) * nt;
                        size_t yb = ((size_t)jy * nx + jx) * nt;
                        for (int ki = 0; ki < nt; ++ki) {
                            double pa = exp(phi_a[xo] + logk[kb + ki] + psi_a[yb + ki]);
                            double pb = exp(phi_b[xo] + logk[kb + ki] + psi_b[yb + ki]);
                            tot += fabs(pa - pb);
                        }
                    }
                }
            }
    return tot;
}

int oc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
