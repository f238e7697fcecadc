// Lift and projection around the transport path (gfx950): the orientation-field lift
// of Section 5.3 (eq. (lifting_vector_field)), the projection P(U) = integral of U over
// theta of Section 2.3 (eq. (proj)) with the argmax reconstruction of eq.
// (reconstruction_vector_field), the difference of projections b_t = P(U+) - P(U-) of
// Section 5.2 (eq. (final)), and the split of a signed score into normalised positive
// and negative parts (Section 5.2, step 2).
//
// All of it is HBM-bound elementwise and segmented-reduction work: no contraction, so
// no matrix cores.  Arrays are [batch][iy][ix][k] with theta innermost; a pixel's
// ntheta values are contiguous and move as 16-byte vectors (grid arrays must be 16-byte
// aligned).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "se2_internal.h"

namespace se2 {

// Scratch of se2_split_signed_noalloc: the per-block partial sums of the positive and
// negative parts and their two totals, 2 * kSplitNoallocMaxBlocks + 2 doubles (64 KiB).
// Every GPU the library runs on holds its own copy until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is a stand-in, not a device
// address): it uses the address split_noalloc_scratch() obtained for the current device.
static __device__ __align__(256) double scratch[2 * kSplitNoallocMaxBlocks + 2];

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

// One thread per four consecutive outputs of a pixel (two 16-byte stores): the lifted
// value is the pixel's magnitude in the bin of its angle and 0 elsewhere.
template <int NT>
__global__ __launch_bounds__(kThreads) void k_lift_field(const double *__restrict__ mag,
                                                         const double *__restrict__ angle, double *__restrict__ out,
                                                         size_t nquads, double inv_step) {
    constexpr int Q = NT / 4;  // quads per pixel
    for (size_t j = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; j < nquads;
         j += static_cast<size_t>(gridDim.x) * kThreads) {
        const size_t p = j / Q;
        const int k0 = static_cast<int>(j - p * Q) * 4;
        const int b = angle_bin(angle[p], inv_step, NT);
        const double m = mag[p];
        double2 lo, hi;
        lo.x = (b == k0) ? m : 0.0;
        lo.y = (b == k0 + 1) ? m : 0.0;
        hi.x = (b == k0 + 2) ? m : 0.0;
        hi.y = (b == k0 + 3) ? m : 0.0;
        double2 *o = reinterpret_cast<double2 *>(out + 4 * j);
        o[0] = lo;
        o[1] = hi;
    }
}

// One thread per pixel, its NT values read with 16-byte loads: mass = sum_k u - sum_k
// u_minus (k in order), argmax_k u (the first maximum, i.e. the lowest k on ties) and its
// angle theta_argmax.  The lanes of a wave read 64 neighbouring pixels, so every fetched
// line is used by the wave's loads.
template <int NT>
__global__ __launch_bounds__(kThreads) void k_project(const double *__restrict__ u, const double *__restrict__ um,
                                                      size_t npix, double step, double *__restrict__ mass,
                                                      int32_t *__restrict__ argmax, double *__restrict__ ang) {
    for (size_t p = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; p < npix;
         p += static_cast<size_t>(gridDim.x) * kThreads) {
        const double2 *row = reinterpret_cast<const double2 *>(u + p * NT);
        double2 v[NT / 2];
#pragma unroll
        for (int q = 0; q < NT / 2; ++q) v[q] = row[q];
        double s = 0.0, m = v[0].x;
        int a = 0;
#pragma unroll
        for (int q = 0; q < NT / 2; ++q) {
            s += v[q].x;
            s += v[q].y;
            if (v[q].x > m) {
                m = v[q].x;
                a = 2 * q;
            }
            if (v[q].y > m) {
                m = v[q].y;
                a = 2 * q + 1;
            }
        }
        if (um) {
            const double2 *rm = reinterpret_cast<const double2 *>(um + p * NT);
#pragma unroll
            for (int q = 0; q < NT / 2; ++q) v[q] = rm[q];
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < NT / 2; ++q) {
                t += v[q].x;
                t += v[q].y;
            }
            s -= t;
        }
        mass[p] = s;
        if (argmax) argmax[p] = a;
        if (ang) ang[p] = a * step;
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
    const size_t nq = npix * nt / 4;
    if (nq == 0) return SE2_OK;
    const dim3 g(blocks_for(nq)), b(kThreads);
    const double inv = nt / period;
    switch (nt) {
        case 8: hipLaunchKernelGGL(k_lift_field<8>, g, b, 0, s, mag, angle, out, nq, inv); break;
        case 16: hipLaunchKernelGGL(k_lift_field<16>, g, b, 0, s, mag, angle, out, nq, inv); break;
        case 32: hipLaunchKernelGGL(k_lift_field<32>, g, b, 0, s, mag, angle, out, nq, inv); break;
        default: return SE2_EINVAL;
    }
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

int launch_project(const double *u, const double *um, size_t npix, int nt, double period, double *mass,
                   int32_t *argmax, double *ang, hipStream_t s) {
    if (npix == 0) return SE2_OK;
    const double step = period / nt;
    const dim3 g(blocks_for(npix)), b(kThreads);
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

int split_noalloc_scratch(double **out) {
    static std::mutex mu;
    static std::vector<double *> per_device;  // device address of `scratch` on each GPU, once known
    int dev = 0;
    SE2_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if (static_cast<size_t>(dev) >= per_device.size()) per_device.resize(static_cast<size_t>(dev) + 1, nullptr);
    if (per_device[dev] == nullptr) {
        void *p = nullptr;
        SE2_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (p == nullptr) return SE2_EHIP;
        per_device[dev] = static_cast<double *>(p);
    }
    *out = per_device[dev];
    return SE2_OK;
}

int launch_split_signed(const double *u, size_t n, double *plus, double *minus, double *part, hipStream_t s) {
    const int nb = split_blocks(n);
    const size_t chunk = 16384;
    hipLaunchKernelGGL(k_signed_partials, dim3(nb), dim3(kThreads), 0, s, u, n, chunk, part);
    SE2_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_signed_total, dim3(1), dim3(kThreads), 0, s, part, nb, part + 2 * nb);
    SE2_HIP(hipGetLastError());
    if (n > 0) {
        hipLaunchKernelGGL(k_signed_split, dim3(blocks_for(n)), dim3(kThreads), 0, s, u, n, part + 2 * nb, plus,
                           minus);
        SE2_HIP(hipGetLastError());
    }
    return SE2_OK;
}

}  // namespace se2
