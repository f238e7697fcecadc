// Elementwise and reduction kernels around the convolutions (gfx950).
//
// Every reduction is two-level with a fixed order (per-block tree, then one
// block over the partials in index order), so a result depends only on the data
// and the array length, never on timing or on what else runs on the device.
#include <hip/hip_runtime.h>

#include <cmath>

#include "se2_internal.h"

namespace se2 {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double block_tree_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (static_cast<int>(threadIdx.x) < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// in == out allowed (each element is read and written by one thread)
__global__ __launch_bounds__(kThreads) void k_scale(const double *in, double *out, size_t n, double mul) {
    for (size_t i = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * kThreads)
        out[i] = in[i] * mul;
}

__global__ __launch_bounds__(kThreads) void k_log2m(const double *__restrict__ m, double *__restrict__ out, size_t n) {
    for (size_t i = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * kThreads) {
        const double v = m[i];
        out[i] = (v > 0.0) ? log2(v) : -INFINITY;
    }
}

__global__ __launch_bounds__(kThreads) void k_exp2(const double *__restrict__ in, double *__restrict__ out, size_t n) {
    for (size_t i = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * kThreads)
        out[i] = exp2(in[i]);
}

__global__ __launch_bounds__(kThreads) void k_fill(double *__restrict__ p, size_t n, double v) {
    for (size_t i = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * kThreads)
        p[i] = v;
}

__global__ __launch_bounds__(kThreads) void k_fill_i32(int32_t *__restrict__ p, size_t n, int32_t v) {
    for (size_t i = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * kThreads)
        p[i] = v;
}

// Per block: [sum m, count of bad entries (non-finite or negative)], over a
// fixed contiguous chunk of the array per block.
__global__ __launch_bounds__(kThreads) void k_validate_partial(const double *__restrict__ m, size_t n, size_t chunk,
                                                               double *__restrict__ part) {
    __shared__ double sh[kThreads];
    const size_t b0 = blockIdx.x * chunk;
    const size_t b1 = (b0 + chunk < n) ? b0 + chunk : n;
    double s = 0.0, bad = 0.0;
    for (size_t i = b0 + threadIdx.x; i < b1; i += kThreads) {
        const double v = m[i];
        if (!(v >= 0.0) || !isfinite(v)) bad += 1.0;
        else s += v;
    }
    s = block_tree_sum(s, sh);
    bad = block_tree_sum(bad, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s;
        part[2 * blockIdx.x + 1] = bad;
    }
}

// The same check for many arrays of one length (blockIdx.y = array, pointers from a
// device table): part[(j * gridDim.x + block) * 2 + {0, 1}].
__global__ __launch_bounds__(kThreads) void k_validate_partial_tab(const double *const *__restrict__ tab, size_t n,
                                                                   size_t chunk, double *__restrict__ part) {
    __shared__ double sh[kThreads];
    const double *m = tab[blockIdx.y];
    const size_t b0 = blockIdx.x * chunk;
    const size_t b1 = (b0 + chunk < n) ? b0 + chunk : n;
    double s = 0.0, bad = 0.0;
    for (size_t i = b0 + threadIdx.x; i < b1; i += kThreads) {
        const double v = m[i];
        if (!(v >= 0.0) || !isfinite(v)) bad += 1.0;
        else s += v;
    }
    s = block_tree_sum(s, sh);
    bad = block_tree_sum(bad, sh);
    if (threadIdx.x == 0) {
        const size_t o = (static_cast<size_t>(blockIdx.y) * gridDim.x + blockIdx.x) * 2;
        part[o] = s;
        part[o + 1] = bad;
    }
}

// One block per array j: out[2 j + c] = sum over p < count of part[(j count + p) 2 + c].
__global__ __launch_bounds__(kThreads) void k_reduce_pairs(const double *__restrict__ part, int count,
                                                           double *__restrict__ out) {
    __shared__ double sh[kThreads];
    const double *pj = part + static_cast<size_t>(blockIdx.x) * count * 2;
    for (int c = 0; c < 2; ++c) {
        double s = 0.0;
        for (int p = threadIdx.x; p < count; p += kThreads) s += pj[2 * static_cast<size_t>(p) + c];
        s = block_tree_sum(s, sh);
        if (threadIdx.x == 0) out[2 * static_cast<size_t>(blockIdx.x) + c] = s;
    }
}

// out[c] = sum over p < count of part[p * stride + c], c < stride, in index order.
__global__ __launch_bounds__(kThreads) void k_reduce_fixed(const double *__restrict__ part, int count, int stride,
                                                           double *__restrict__ out) {
    __shared__ double sh[kThreads];
    for (int c = 0; c < stride; ++c) {
        double s = 0.0;
        for (int p = threadIdx.x; p < count; p += kThreads) s += part[static_cast<size_t>(p) * stride + c];
        s = block_tree_sum(s, sh);
        if (threadIdx.x == 0) out[c] = s;
    }
}

// One block per job: out[j] = sum of partials[offsets[j] .. offsets[j+1]).
__global__ __launch_bounds__(kThreads) void k_sum_partials(const double *__restrict__ part,
                                                           const int32_t *__restrict__ offsets,
                                                           double *__restrict__ out) {
    __shared__ double sh[kThreads];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int p = offsets[j] + threadIdx.x; p < offsets[j + 1]; p += kThreads) s += part[p];
    s = block_tree_sum(s, sh);
    if (threadIdx.x == 0) out[j] = s;
}

// One workgroup per item, the same fixed-order reduction as k_sum_partials.
__global__ __launch_bounds__(kThreads) void k_sum_items(const SumItem *__restrict__ items, double *__restrict__ out) {
    __shared__ double sh[kThreads];
    const SumItem it = items[blockIdx.x];
    double s = 0.0;
    if (it.ints) {
        const uint32_t *v = static_cast<const uint32_t *>(it.part);  // counters that wrap at 2^32
        for (int p = it.begin + threadIdx.x; p < it.end; p += kThreads) s += static_cast<double>(v[p]);
    } else {
        const double *v = static_cast<const double *>(it.part);
        for (int p = it.begin + threadIdx.x; p < it.end; p += kThreads) s += v[p];
    }
    s = block_tree_sum(s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// Hands the n error sums of a check to the host: copies them into pinned host memory, then
// (after a system-scope fence) stores `seq` to the host's flag word, which the host polls.
// One workgroup; it runs after k_sum_items in stream order, so the sums are complete.
__global__ __launch_bounds__(kThreads) void k_publish(const double *__restrict__ errs, int n,
                                                      double *__restrict__ host_errs, int *host_flag, int seq) {
    for (int i = threadIdx.x; i < n; i += kThreads) host_errs[i] = errs[i];
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence_system();
        *reinterpret_cast<volatile int *>(host_flag) = seq;
    }
}

// IBP combine (Appendix A): log bar = sum_i lambda_i log d_i, then log v_i += log bar -
// log d_i (log v_i = -inf where the barycenter is 0).  The sum runs in a fixed order: in
// index order within chunks of kCombineChunk measures (one block row per chunk), then the
// chunk partials in chunk order; with one chunk the partial is the sum itself.
__device__ __forceinline__ double acc_log(double bar, double lam, double d) {
    return (d == -INFINITY || bar == -INFINITY) ? -INFINITY : bar + lam * d;
}

__global__ __launch_bounds__(kThreads) void k_ibp_bar_partial(const double *const *__restrict__ ld,
                                                              const double *__restrict__ lam, int n, size_t len,
                                                              double *__restrict__ part) {
    const int i0 = blockIdx.y * kCombineChunk;
    const int i1 = (i0 + kCombineChunk < n) ? i0 + kCombineChunk : n;
    for (size_t x = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; x < len;
         x += static_cast<size_t>(gridDim.x) * kThreads) {
        double bar = 0.0;
        for (int i = i0; i < i1; ++i) bar = acc_log(bar, lam[i], ld[i][x]);
        part[blockIdx.y * len + x] = bar;
    }
}

__global__ __launch_bounds__(kThreads) void k_ibp_bar_total(const double *__restrict__ part, int nchunks, size_t len,
                                                            double *__restrict__ logbar) {
    for (size_t x = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; x < len;
         x += static_cast<size_t>(gridDim.x) * kThreads) {
        double bar = part[x];
        for (int c = 1; c < nchunks; ++c) {
            const double p = part[c * len + x];
            bar = (p == -INFINITY || bar == -INFINITY) ? -INFINITY : bar + p;
        }
        logbar[x] = bar;
    }
}

__global__ __launch_bounds__(kThreads) void k_ibp_vupdate(double *const *__restrict__ lv,
                                                          const double *const *__restrict__ ld, int n, size_t len,
                                                          const double *__restrict__ logbar) {
    const int i0 = blockIdx.y * kCombineChunk;
    const int i1 = (i0 + kCombineChunk < n) ? i0 + kCombineChunk : n;
    for (size_t x = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; x < len;
         x += static_cast<size_t>(gridDim.x) * kThreads) {
        const double bar = logbar[x];
        for (int i = i0; i < i1; ++i) {
            const double v = lv[i][x];
            lv[i][x] = (bar == -INFINITY || v == -INFINITY) ? -INFINITY : v + (bar - ld[i][x]);
        }
    }
}

// Per block: sum over entries with m > 0 of f2 * m.
__global__ __launch_bounds__(kThreads) void k_dot_pos(const double *__restrict__ f2, const double *__restrict__ m,
                                                      size_t n, size_t chunk, double *__restrict__ part) {
    __shared__ double sh[kThreads];
    const size_t b0 = blockIdx.x * chunk;
    const size_t b1 = (b0 + chunk < n) ? b0 + chunk : n;
    double s = 0.0;
    for (size_t i = b0 + threadIdx.x; i < b1; i += kThreads) {
        const double w = m[i];
        if (w > 0.0) s += f2[i] * w;
    }
    s = block_tree_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// KL proximal step of the porous-medium energy (JKO step of the gradient flow of
// F(nu) = ref/(m-1) sum (nu/ref)^m): from s = ln K^T a, the log q with
// log q + c q^(m-1) = s, and the new b-potential log b = log q - s (base-2 units in and
// out).  With z = c (m-1) q^(m-1) the equation becomes z + ln z = A,
// A = (m-1) s + ln(c (m-1)) (Wright's omega function of A), solved by Newton's method in
// u = ln z from a start right of the root (e^u + u - A is increasing and convex, so the
// iterates decrease monotonically): u0 = A for A <= 1, else ln A.  Then
// ln q = s - z / (m-1), so ln b = -z / (m-1).
__global__ __launch_bounds__(kThreads) void k_porous_prox(const double *__restrict__ lsum, double *__restrict__ psi,
                                                          size_t n, double c, double m) {
    const double lc = (c > 0.0) ? log(c * (m - 1.0)) : 0.0;
    for (size_t i = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * kThreads) {
        const double s2 = lsum[i];
        if (s2 == -INFINITY) {
            psi[i] = -INFINITY;  // no mass reaches this element: b is arbitrary there
            continue;
        }
        double lb = 0.0;  // ln b = ln q - s; exactly 0 (b = 1) when the energy is off
        if (c > 0.0) {
            const double s = s2 * kLn2;
            const double A = (m - 1.0) * s + lc;
            double u = (A <= 1.0) ? A : log(A);
            for (int it = 0; it < 64; ++it) {
                const double e = exp(u);
                const double du = (e + u - A) / (e + 1.0);
                u -= du;
                if (!(fabs(du) > 1e-15 * (1.0 + fabs(u)))) break;
            }
            lb = -exp(u) / (m - 1.0);
        }
        psi[i] = lb * kLog2e;
    }
}

// p /= sums[0] (a measure scaled to mass one; the sum from the validation reduction).
__global__ __launch_bounds__(kThreads) void k_div_by(double *__restrict__ p, size_t n, const double *__restrict__ sums) {
    const double t = sums[0];
    for (size_t i = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * kThreads)
        p[i] = p[i] / t;
}

// out = 2^(a + b) (the next measure of a JKO step: nu = b K^T a).
__global__ __launch_bounds__(kThreads) void k_exp2_sum(const double *__restrict__ a, const double *__restrict__ b,
                                                       double *__restrict__ out, size_t n) {
    for (size_t i = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * kThreads)
        out[i] = exp2(a[i] + b[i]);
}

// Per block: sum of ref/(m-1) (nu/ref)^m with nu = 2^(a + b), fixed tree order.
__global__ __launch_bounds__(kThreads) void k_porous_energy(const double *__restrict__ a,
                                                            const double *__restrict__ b, size_t n, size_t chunk,
                                                            double m, double lref2, double scale,
                                                            double *__restrict__ part) {
    __shared__ double sh[kThreads];
    const size_t b0 = blockIdx.x * chunk;
    const size_t b1 = (b0 + chunk < n) ? b0 + chunk : n;
    double s = 0.0;
    for (size_t i = b0 + threadIdx.x; i < b1; i += kThreads) s += exp2(m * ((a[i] + b[i]) - lref2));
    s = block_tree_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s * scale;
}

int grid_for(size_t n) {
    size_t b = (n + kThreads - 1) / kThreads;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return static_cast<int>(b);
}

}  // namespace

int launch_scale(const double *in, double *out, size_t n, double mul, hipStream_t s) {
    if (n == 0) return SE2_OK;
    hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(kThreads), 0, s, in, out, n, mul);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_log2_measure(const double *m, double *logm, size_t n, hipStream_t s) {
    if (n == 0) return SE2_OK;
    hipLaunchKernelGGL(k_log2m, dim3(grid_for(n)), dim3(kThreads), 0, s, m, logm, n);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_exp2_out(const double *in2, double *out, size_t n, hipStream_t s) {
    if (n == 0) return SE2_OK;
    hipLaunchKernelGGL(k_exp2, dim3(grid_for(n)), dim3(kThreads), 0, s, in2, out, n);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_fill(double *p, size_t n, double v, hipStream_t s) {
    if (n == 0) return SE2_OK;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kThreads), 0, s, p, n, v);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_fill_i32(int32_t *p, size_t n, int32_t v, hipStream_t s) {
    if (n == 0) return SE2_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(kThreads), 0, s, p, n, v);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

// d_stats receives [sum, bad]; needs a scratch of 2 * 256 doubles after the first 2.
int launch_validate(const double *m, size_t n, double *d_stats, hipStream_t s) {
    const int nb = 256;
    const size_t chunk = (n + nb - 1) / nb;
    double *part = d_stats + 2;
    hipLaunchKernelGGL(k_validate_partial, dim3(nb), dim3(kThreads), 0, s, m, n, chunk == 0 ? 1 : chunk, part);
    SE2_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_fixed, dim3(1), dim3(kThreads), 0, s, part, nb, 2, d_stats);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int validate_many_blocks(size_t n) {
    const size_t b = (n + 4095) / 4096;
    return static_cast<int>(b < 1 ? 1 : (b > 256 ? 256 : b));
}

int launch_validate_many(const double *const *d_tab, int m, size_t n, double *d_stats, double *d_part, hipStream_t s) {
    if (m < 1) return SE2_OK;
    const int nb = validate_many_blocks(n);
    const size_t chunk = (n + nb - 1) / nb;
    hipLaunchKernelGGL(k_validate_partial_tab, dim3(nb, m), dim3(kThreads), 0, s, d_tab, n, chunk == 0 ? 1 : chunk,
                       d_part);
    SE2_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_pairs, dim3(m), dim3(kThreads), 0, s, d_part, nb, d_stats);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_reduce_fixed(const double *partials, int count, int stride, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_fixed, dim3(1), dim3(kThreads), 0, s, partials, count, stride, out);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_sum_partials(const double *partials, const int32_t *offsets, int njobs, double *out, hipStream_t s) {
    if (njobs <= 0) return SE2_OK;
    hipLaunchKernelGGL(k_sum_partials, dim3(njobs), dim3(kThreads), 0, s, partials, offsets, out);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_sum_items(const SumItem *d_items, int n, double *out, hipStream_t s) {
    if (n <= 0) return SE2_OK;
    hipLaunchKernelGGL(k_sum_items, dim3(n), dim3(kThreads), 0, s, d_items, out);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_publish(const double *errs, int n, double *host_errs, int *host_flag, int seq, hipStream_t s) {
    if (n < 0 || !host_errs || !host_flag) return SE2_EINVAL;
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(kThreads), 0, s, errs, n, host_errs, host_flag, seq);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_ibp_combine(double *const *d_lv, const double *const *d_ld, const double *d_lam, int n, size_t len,
                       double *part, double *logbar, hipStream_t s) {
    if (n < 1 || len == 0) return n < 1 ? SE2_EINVAL : SE2_OK;
    const int nchunks = combine_chunks(n);
    const int gx = grid_for(len);
    hipLaunchKernelGGL(k_ibp_bar_partial, dim3(gx, nchunks), dim3(kThreads), 0, s, d_ld, d_lam, n, len,
                       nchunks == 1 ? logbar : part);
    SE2_HIP(hipGetLastError());
    if (nchunks > 1) {
        hipLaunchKernelGGL(k_ibp_bar_total, dim3(gx), dim3(kThreads), 0, s, part, nchunks, len, logbar);
        SE2_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_ibp_vupdate, dim3(gx, nchunks), dim3(kThreads), 0, s, d_lv, d_ld, n, len, logbar);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_porous_prox(const double *lsum, double *psi, size_t n, double c, double m, hipStream_t s) {
    if (n == 0) return SE2_OK;
    hipLaunchKernelGGL(k_porous_prox, dim3(grid_for(n)), dim3(kThreads), 0, s, lsum, psi, n, c, m);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_normalise(double *p, size_t n, double *stats, hipStream_t s) {
    if (n == 0) return SE2_OK;
    int rc = launch_validate(p, n, stats, s);  // stats[0] = sum (fixed order)
    if (rc) return rc;
    hipLaunchKernelGGL(k_div_by, dim3(grid_for(n)), dim3(kThreads), 0, s, p, n, stats);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_exp2_sum(const double *a, const double *b, double *out, size_t n, hipStream_t s) {
    if (n == 0) return SE2_OK;
    hipLaunchKernelGGL(k_exp2_sum, dim3(grid_for(n)), dim3(kThreads), 0, s, a, b, out, n);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_porous_energy(const double *a, const double *b, size_t n, double m, double ref, double *partials,
                         int nblocks, hipStream_t s) {
    const size_t chunk = (n + nblocks - 1) / nblocks;
    hipLaunchKernelGGL(k_porous_energy, dim3(nblocks), dim3(kThreads), 0, s, a, b, n, chunk == 0 ? 1 : chunk, m,
                       std::log2(ref), ref / (m - 1.0), partials);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_dot_exp(const double *f2, const double *m, size_t n, double *partials, int nblocks, hipStream_t s) {
    const size_t chunk = (n + nblocks - 1) / nblocks;
    hipLaunchKernelGGL(k_dot_pos, dim3(nblocks), dim3(kThreads), 0, s, f2, m, n, chunk == 0 ? 1 : chunk, partials);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

}  // namespace se2
