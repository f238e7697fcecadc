// Lift and projection around the transport path (gfx950): the orientation-field lift
// of Section 5.3 (eq. (lifting_vector_field)), the projection P(U) = integral of U over
// theta of Section 2.3 (eq. (proj)) with the argmax reconstruction of eq.
// (reconstruction_vector_field), the difference of projections b_t = P(U+) - P(U-) of
// Section 5.2 (eq. (final)), and the split of a signed score into normalised positive
// and negative parts (Section 5.2, step 2).
//
// All of it is HBM-bound elementwise and segmented-reduction work: no contraction, so
// no matrix cores.  Arrays are [batch][iy][ix][k] with theta innermost; a pixel's
// ntheta values are contiguous, so one wave reads 64 consecutive doubles and reduces
// them in groups of ntheta lanes with cross-lane moves (fixed butterfly order).
#include <hip/hip_runtime.h>

#include <cmath>

#include "se2_internal.h"

namespace se2 {

namespace {

constexpr int kThreads = 256;

int blocks_for(size_t n) {
    const size_t b = (n + kThreads - 1) / kThreads;
    return static_cast<int>(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

// Orientation bin of an angle: the k whose centre theta_k = k * Theta / nt is nearest,
// on the circle of circumference Theta (ties at a bin edge go to the upper bin).
__device__ __forceinline__ int angle_bin(double psi, double inv_step, int nt) {
    const double u = floor(psi * inv_step + 0.5);
    long long b = static_cast<long long>(u) % nt;
    if (b < 0) b += nt;
    return static_cast<int>(b);
}

// One thread per output element (pixel, k): the lifted value is the pixel's magnitude in
// the bin of its angle and 0 elsewhere.
__global__ __launch_bounds__(kThreads) void k_lift_field(const double *__restrict__ mag,
                                                         const double *__restrict__ angle, double *__restrict__ out,
                                                         size_t n_out, int nt, double inv_step) {
    for (size_t i = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; i < n_out;
         i += static_cast<size_t>(gridDim.x) * kThreads) {
        const size_t p = i / nt;
        const int k = static_cast<int>(i - p * nt);
        const double a = angle[p];
        out[i] = (angle_bin(a, inv_step, nt) == k) ? mag[p] : 0.0;
    }
}

// Butterfly sum and (max, lowest index) over aligned groups of NT lanes.
template <int NT>
__device__ __forceinline__ void group_reduce(double &s, double &m, int &arg) {
#pragma unroll
    for (int off = 1; off < NT; off <<= 1) {
        const double so = __shfl_xor(s, off, 64);
        const double mo = __shfl_xor(m, off, 64);
        const int ao = __shfl_xor(arg, off, 64);
        s += so;
        // the larger value wins; on equal values the lower orientation index
        if (mo > m || (mo == m && ao < arg)) {
            m = mo;
            arg = ao;
        }
    }
}

// One thread per element, NT consecutive lanes per pixel: mass = sum_k u - sum_k u_minus,
// argmax_k u (lowest k on ties), its angle theta_argmax.
template <int NT>
__global__ __launch_bounds__(kThreads) void k_project(const double *__restrict__ u, const double *__restrict__ um,
                                                      size_t npix, double step, double *__restrict__ mass,
                                                      int32_t *__restrict__ argmax, double *__restrict__ ang) {
    const size_t n = npix * NT;
    const size_t stride = static_cast<size_t>(gridDim.x) * kThreads;
    // every lane of a wave runs the same number of rounds (the butterflies need all 64)
    const size_t rounds = (n + stride - 1) / stride;
    size_t i = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x;
    for (size_t r = 0; r < rounds; ++r, i += stride) {
        const bool in = i < n;
        const int k = static_cast<int>(i % NT);
        double v = in ? u[i] : 0.0;
        double s = v - ((in && um) ? um[i] : 0.0);
        double m = in ? v : -INFINITY;
        int a = k;
        group_reduce<NT>(s, m, a);
        if (in && k == 0) {
            const size_t p = i / NT;
            mass[p] = s;
            if (argmax) argmax[p] = a;
            if (ang) ang[p] = a * step;
        }
    }
}

// Sums of the positive and negative parts, per block (fixed tree order), then one block
// over the partials in index order.
__global__ __launch_bounds__(kThreads) void k_signed_partials(const double *__restrict__ u, size_t n, size_t chunk,
                                                              double *__restrict__ part) {
    __shared__ double sp[kThreads], sn[kThreads];
    const size_t b0 = blockIdx.x * chunk, b1 = (b0 + chunk < n) ? b0 + chunk : n;
    double p = 0.0, q = 0.0;
    for (size_t i = b0 + threadIdx.x; i < b1; i += kThreads) {
        const double v = u[i];
        if (v > 0.0) p += v;
        else q -= v;
    }
    sp[threadIdx.x] = p;
    sn[threadIdx.x] = q;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (static_cast<int>(threadIdx.x) < s) {
            sp[threadIdx.x] += sp[threadIdx.x + s];
            sn[threadIdx.x] += sn[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sp[0];
        part[2 * blockIdx.x + 1] = sn[0];
    }
}

__global__ __launch_bounds__(kThreads) void k_signed_total(double *__restrict__ part, int nblocks,
                                                           double *__restrict__ sums) {
    __shared__ double sp[kThreads], sn[kThreads];
    double p = 0.0, q = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kThreads) {
        p += part[2 * b];
        q += part[2 * b + 1];
    }
    sp[threadIdx.x] = p;
    sn[threadIdx.x] = q;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (static_cast<int>(threadIdx.x) < s) {
            sp[threadIdx.x] += sp[threadIdx.x + s];
            sn[threadIdx.x] += sn[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sums[0] = sp[0];
        sums[1] = sn[0];
    }
}

// plus = max(u, 0) / S+, minus = max(-u, 0) / S- (a part with zero sum stays zero).
__global__ __launch_bounds__(kThreads) void k_signed_split(const double *__restrict__ u, size_t n,
                                                           const double *__restrict__ sums, double *__restrict__ plus,
                                                           double *__restrict__ minus) {
    const double sp = sums[0], sn = sums[1];
    for (size_t i = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * kThreads) {
        const double v = u[i];
        plus[i] = v > 0.0 ? v / sp : 0.0;   // v > 0 implies sp > 0
        minus[i] = v < 0.0 ? -v / sn : 0.0;
    }
}

}  // namespace

int launch_lift_field(const double *mag, const double *angle, double *out, size_t npix, int nt, double period,
                      hipStream_t s) {
    const size_t n = npix * nt;
    if (n == 0) return SE2_OK;
    hipLaunchKernelGGL(k_lift_field, dim3(blocks_for(n)), dim3(kThreads), 0, s, mag, angle, out, n, nt, nt / period);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_project(const double *u, const double *um, size_t npix, int nt, double period, double *mass,
                   int32_t *argmax, double *ang, hipStream_t s) {
    if (npix == 0) return SE2_OK;
    const size_t n = npix * nt;
    const double step = period / nt;
    const dim3 g(blocks_for(n)), b(kThreads);
    switch (nt) {
        case 8: hipLaunchKernelGGL(k_project<8>, g, b, 0, s, u, um, npix, step, mass, argmax, ang); break;
        case 16: hipLaunchKernelGGL(k_project<16>, g, b, 0, s, u, um, npix, step, mass, argmax, ang); break;
        case 32: hipLaunchKernelGGL(k_project<32>, g, b, 0, s, u, um, npix, step, mass, argmax, ang); break;
        default: return SE2_EINVAL;
    }
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

// Blocks of the partial-sum pass of launch_split_signed (the scratch holds 2 per block + 2).
int split_blocks(size_t n) {
    const size_t chunk = 16384;
    const size_t b = (n + chunk - 1) / chunk;
    return static_cast<int>(b > 0 ? b : 1);
}

int launch_split_signed(const double *u, size_t n, double *plus, double *minus, double *scratch, hipStream_t s) {
    const int nb = split_blocks(n);
    const size_t chunk = 16384;
    hipLaunchKernelGGL(k_signed_partials, dim3(nb), dim3(kThreads), 0, s, u, n, chunk, scratch);
    SE2_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_signed_total, dim3(1), dim3(kThreads), 0, s, scratch, nb, scratch + 2 * nb);
    SE2_HIP(hipGetLastError());
    if (n > 0) {
        hipLaunchKernelGGL(k_signed_split, dim3(blocks_for(n)), dim3(kThreads), 0, s, u, n, scratch + 2 * nb, plus,
                           minus);
        SE2_HIP(hipGetLastError());
    }
    return SE2_OK;
}

}  // namespace se2
