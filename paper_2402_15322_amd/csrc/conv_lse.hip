// Log-domain SE(2) group convolution with fused scaling epilogues (gfx950).
//
// For every output element (x, ko) of a job:
//     LSE(x, ko) = log2 sum_{d in window, ki} 2^( L2[d][ko][ki] + in(x - d, ki) )
// i.e. log2 of (K * 2^in)(x, ko), the operator K b of the Sinkhorn updates
// (Section 4.1) written as the group convolution of Section 4.2, evaluated term
// by term in the log domain.
//
// Dense path (exact): every window entry is visited.  A first pass finds the
// per-output maximum M of the exponents in FP32; the second forms each exponent
// u = L2 + in - M in FP64 (the two addends are O(10^3) and nearly cancel for the
// terms that matter), rounds u to FP32 and takes a native exp2.  Partial sums
// over one window row are FP32 and are combined in FP64.  F64EXP uses an FP64
// exp2 and FP64 sums throughout (the checking path).
//
// Certified sparse path (SPARSE kernels, jobs that carry term lists): a dense
// visit of a tile also records, for each output orientation ko, the union over
// the tile's 64 pixels of the window entries (d, ki) whose exponent is within
// kListCut of that output's maximum, the maximum itself (mref) and the input
// halo it saw (ref).  A later visit measures the drift delta = in - ref over the
// halo, lo <= delta <= hi.  Every skipped entry had u <= -kListCut at reference
// time; its exponent grew by at most hi and the maximum fell by at most -lo, so
// now u <= -kListCut + (hi - lo).  While the spread hi - lo <= kDriftSpread the
// skipped entries sum to less than n 2^-(kListCut - kDriftSpread) = n 2^-48 of
// the result and the tile only visits its list, shifting exponents by
// mref + (lo + hi)/2 (within 2^+-spread/2 of the true maximum).  Otherwise the
// tile takes the dense path and rebuilds its list.  The decision is per tile, so results stay independent of
// any other job in the launch.
//
// Work layout: one workgroup = one 8 x 8 output tile of one job, all ntheta
// outputs; lane = pixel of the tile, wave w owns ko = w, w+4, ... .  The input
// halo (8+2R)^2 is staged in LDS as FP64, theta-major so that the 64 lanes of a
// wave read neighbouring addresses.  Kernel values and list entries are
// wave-uniform and read through the scalar cache.
#include <hip/hip_runtime.h>

#include <cmath>

#include "se2_internal.h"

namespace se2 {

namespace {

typedef const __attribute__((address_space(4))) double *cdptr;
typedef const __attribute__((address_space(4))) float *cfptr;
typedef const __attribute__((address_space(4))) int32_t *ciptr;

template <int KC>
__device__ __forceinline__ void load_halo(double *lds, const double *__restrict__ in, int nt, int k0, int x0, int y0,
                                          int R, int HW, int nx, int ny) {
    const int npix = HW * HW;
    const int total = npix * KC;
    for (int e = threadIdx.x; e < total; e += kConvThreads) {
        const int p = e / KC;
        const int kc = e - p * KC;
        const int hy = p / HW;
        const int hx = p - hy * HW;
        const int gy = y0 - R + hy, gx = x0 - R + hx;
        double v = -INFINITY;
        if (gy >= 0 && gy < ny && gx >= 0 && gx < nx) v = in[(static_cast<size_t>(gy) * nx + gx) * nt + k0 + kc];
        lds[kc * npix + p] = v;
    }
}

__device__ __forceinline__ double block_sum_fixed(double v, double *scratch) {
    // Fixed-order tree over the 256 threads: the result does not depend on timing.
    scratch[threadIdx.x] = v;
    __syncthreads();
    for (int s = kConvThreads / 2; s > 0; s >>= 1) {
        if (static_cast<int>(threadIdx.x) < s) scratch[threadIdx.x] += scratch[threadIdx.x + s];
        __syncthreads();
    }
    return scratch[0];
}

__device__ __forceinline__ float wave_max(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}

template <int NT, int KC, bool F64EXP, bool SPARSE>
__global__ __launch_bounds__(kConvThreads) void k_conv_lse(const ConvJob *__restrict__ jobs,
                                                           const int32_t *__restrict__ block_job) {
    extern __shared__ double lds[];
    __shared__ float s_red[kConvThreads / 64];
    __shared__ float s_red2[kConvThreads / 64];
    __shared__ int s_flag;
    __shared__ int s_list_off[NT + 1];
    static_assert(!SPARSE || KC == NT, "the sparse path keeps the whole halo in LDS");
    constexpr int NJ = NT / 4;
    const int j = block_job[blockIdx.x];
    const ConvJob job = jobs[j];
    const int tile = static_cast<int>(blockIdx.x) - job.first_block;
    const int ty = tile / job.tiles_x;
    const int tx = tile - ty * job.tiles_x;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int R = job.R, W = 2 * R + 1, HW = kTile + 2 * R, npix = HW * HW;
    const int nx = job.nx, ny = job.ny;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int px = lane & 7, py = lane >> 3;
    const int gx = x0 + px, gy = y0 + py;
    const bool valid = gx < nx && gy < ny;
    const size_t obase = (static_cast<size_t>(gy) * nx + gx) * NT;
    const cdptr L64 = (cdptr)(job.L64);
    const cfptr L32 = (cfptr)(job.L32);
    const bool lists = SPARSE && job.lists != nullptr;

    double lse[NJ];
    float mx[NJ];

    // ---------------- certified sparse path ----------------
    bool dense = true;
    float spread = 0.0f, shift = 0.0f;
    if constexpr (SPARSE) {
        if (lists) {
            load_halo<NT>(lds, job.in, NT, 0, x0, y0, R, HW, nx, ny);
            if (threadIdx.x == 0) {
                // list offsets of the tile's orientations; missing/overflowed lists or a total
                // beyond the LDS staging capacity force the dense path
                int acc = 0, ok = 1;
                for (int k = 0; k < NT; ++k) {
                    const int n = job.len[static_cast<size_t>(tile) * NT + k];
                    s_list_off[k] = acc;
                    if (n < 0) ok = 0;
                    else acc += n;
                }
                s_list_off[NT] = acc;
                s_flag = (ok && acc <= kListLds) ? 1 : 0;
            }
            __syncthreads();
            const double *ref = job.ref + static_cast<size_t>(tile) * NT * npix;
            // drift delta = in - ref over the halo; only its spread matters: a common shift of the
            // inputs moves every exponent and the maximum alike
            float dlo = INFINITY, dhi = -INFINITY;
            bool bad = false;
            for (int e = threadIdx.x; e < NT * npix; e += kConvThreads) {
                const double a = lds[e], b = ref[e];
                if (a == -INFINITY && b == -INFINITY) continue;
                const double de = a - b;  // +-inf or NaN when only one side is -inf
                if (!(fabs(de) < 1e30)) {
                    bad = true;
                    continue;
                }
                dlo = fminf(dlo, static_cast<float>(de));
                dhi = fmaxf(dhi, static_cast<float>(de));
            }
            if (bad) s_flag = 0;
            dlo = -wave_max(-dlo);
            dhi = wave_max(dhi);
            if (lane == 0) {
                s_red[wave] = dlo;
                s_red2[wave] = dhi;
            }
            __syncthreads();
            const float lo = fminf(fminf(s_red[0], s_red[1]), fminf(s_red[2], s_red[3]));
            const float hi = fmaxf(fmaxf(s_red2[0], s_red2[1]), fmaxf(s_red2[2], s_red2[3]));
            // all entries -inf on both sides: no spread at all
            spread = (hi >= lo) ? hi - lo : 0.0f;
            shift = (hi >= lo) ? 0.5f * (hi + lo) : 0.0f;
            // 1 ulp of the FP32 differences per unit of magnitude is far below kDriftSpread's slack
            dense = !(s_flag != 0 && spread <= kDriftSpread);
        }
    }
    int listed = 0;  // list entries visited by this wave (sparse path)
    if (!dense) {
        // Stage the tile's lists in LDS (one bulk copy), then lane = pixel, one ko at a time,
        // with the entries read as wave-wide broadcasts, 8 per step.
        ListEntry *lst_lds = reinterpret_cast<ListEntry *>(lds + static_cast<size_t>(NT) * npix);
        const int total = s_list_off[NT];
        const ListEntry *src = job.lists;
        for (int e = threadIdx.x; e < total; e += kConvThreads) {
            int ko = 0;
            while (e >= s_list_off[ko + 1]) ++ko;
            lst_lds[e] = src[(static_cast<size_t>(tile) * NT + ko) * job.lmax + (e - s_list_off[ko])];
        }
        __syncthreads();
        const int base = py * HW + px;
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
            const int ko = wave + 4 * q;
            const int e0 = s_list_off[ko], n = s_list_off[ko + 1] - e0;
            listed += n;
            const float mr = valid ? job.mref[obase + ko] : -INFINITY;
            // the reference maximum moved with the inputs by shift +- spread/2
            const double M = (mr == -INFINITY) ? 0.0 : static_cast<double>(mr) + static_cast<double>(shift);
            const ListEntry *L = lst_lds + e0;
            double S = 0.0;
            int e = 0;
            for (; e + 8 <= n; e += 8) {
                double v[8];
                double lv[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    lv[t] = L[e + t].L;
                    v[t] = lds[L[e + t].off + base];
                }
                float s8 = 0.0f;
#pragma unroll
                for (int t = 0; t < 8; ++t) s8 += __builtin_amdgcn_exp2f(static_cast<float>((lv[t] + v[t]) - M));
                S += static_cast<double>(s8);
            }
            float st = 0.0f;
            for (; e < n; ++e) st += __builtin_amdgcn_exp2f(static_cast<float>((L[e].L + lds[L[e].off + base]) - M));
            S += static_cast<double>(st);
            lse[q] = (mr == -INFINITY || !(S > 0.0)) ? -INFINITY : M + log2(S);
        }
    } else {
        // ---------------- dense path ----------------
#pragma unroll
        for (int q = 0; q < NJ; ++q) mx[q] = -INFINITY;
        for (int k0 = 0; k0 < NT; k0 += KC) {
            if (!(SPARSE && lists)) {
                if (k0 > 0) __syncthreads();
                load_halo<KC>(lds, job.in, NT, k0, x0, y0, R, HW, nx, ny);
                __syncthreads();
            }
            for (int dy = -R; dy <= R; ++dy) {
                for (int dx = -R; dx <= R; ++dx) {
                    const int hb = (py + R - dy) * HW + (px + R - dx);
                    const cfptr Lr = L32 + (static_cast<size_t>((dy + R) * W + (dx + R)) * NT) * NT + k0;
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc) {
                        const float v = static_cast<float>(lds[kc * npix + hb]);
#pragma unroll
                        for (int q = 0; q < NJ; ++q) mx[q] = fmaxf(mx[q], v + Lr[(wave + 4 * q) * NT + kc]);
                    }
                }
            }
        }
        double M[NJ], S[NJ];
        int cnt[NJ];
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
            M[q] = (mx[q] == -INFINITY) ? 0.0 : static_cast<double>(mx[q]);
            S[q] = 0.0;
            cnt[q] = 0;
        }
        for (int k0 = 0; k0 < NT; k0 += KC) {
            if (NT > KC) {
                __syncthreads();
                load_halo<KC>(lds, job.in, NT, k0, x0, y0, R, HW, nx, ny);
                __syncthreads();
            }
            for (int dy = -R; dy <= R; ++dy) {
                if constexpr (F64EXP) {
                    for (int dx = -R; dx <= R; ++dx) {
                        const int hb = (py + R - dy) * HW + (px + R - dx);
                        const cdptr Lr = L64 + (static_cast<size_t>((dy + R) * W + (dx + R)) * NT) * NT + k0;
#pragma unroll
                        for (int kc = 0; kc < KC; ++kc) {
                            const double v = lds[kc * npix + hb];
#pragma unroll
                            for (int q = 0; q < NJ; ++q) S[q] += exp2((v + Lr[(wave + 4 * q) * NT + kc]) - M[q]);
                        }
                    }
                } else {
                    float srow[NJ];
#pragma unroll
                    for (int q = 0; q < NJ; ++q) srow[q] = 0.0f;
                    for (int dx = -R; dx <= R; ++dx) {
                        const int hb = (py + R - dy) * HW + (px + R - dx);
                        const cdptr Lr = L64 + (static_cast<size_t>((dy + R) * W + (dx + R)) * NT) * NT + k0;
#pragma unroll
                        for (int kc = 0; kc < KC; ++kc) {
                            const double v = lds[kc * npix + hb];
#pragma unroll
                            for (int q = 0; q < NJ; ++q) {
                                const double Lv = Lr[(wave + 4 * q) * NT + kc];
                                const double u = (v + Lv) - M[q];
                                srow[q] += __builtin_amdgcn_exp2f(static_cast<float>(u));
                                if constexpr (SPARSE) {
                                    if (lists) {
                                        // union over the tile's pixels of the entries within the list cut
                                        const bool keep = valid && u >= -kListCut;
                                        if (__ballot(keep) != 0) {
                                            if (cnt[q] < job.lmax && lane == 0) {
                                                ListEntry *dst = job.lists +
                                                                 (static_cast<size_t>(tile) * NT + wave + 4 * q) *
                                                                     job.lmax +
                                                                 cnt[q];
                                                dst->L = Lv;
                                                dst->off = kc * npix + (R - dy) * HW + (R - dx);
                                                dst->pad = 0;
                                            }
                                            cnt[q] += 1;
                                        }
                                    }
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < NJ; ++q) S[q] += static_cast<double>(srow[q]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NJ; ++q) lse[q] = (S[q] > 0.0) ? M[q] + log2(S[q]) : -INFINITY;
        if constexpr (SPARSE) {
            if (lists) {
                // publish the rebuilt lists, the reference maxima and the reference halo
#pragma unroll
                for (int q = 0; q < NJ; ++q) {
                    if (lane == 0) job.len[static_cast<size_t>(tile) * NT + wave + 4 * q] =
                        (cnt[q] <= job.lmax) ? cnt[q] : -1;
                    if (valid) job.mref[obase + wave + 4 * q] = mx[q];
                }
                double *ref = job.ref + static_cast<size_t>(tile) * NT * npix;
                for (int e = threadIdx.x; e < NT * npix; e += kConvThreads) ref[e] = lds[e];
                if (job.dense_flag != nullptr && threadIdx.x == 0) job.dense_flag[tile] += 1;
            }
        }
    }

    // ---------------- work counters (diagnostics) ----------------
    if (job.work != nullptr) {
        // in-grid terms of this lane's outputs (dense) or the visited list entries (sparse)
        double w = 0.0;
        if (valid) {
            if (dense) {
                const int cx = min(R, gx) + min(R, nx - 1 - gx) + 1;
                const int cy = min(R, gy) + min(R, ny - 1 - gy) + 1;
                w = static_cast<double>(cx) * cy * NT * NJ;
            } else {
                w = static_cast<double>(listed);
            }
        }
        __syncthreads();
        const double t = block_sum_fixed(w, lds);
        if (threadIdx.x == 0) job.work[2 * tile + (dense ? 0 : 1)] += t;
        __syncthreads();
    }

    // ---------------- epilogue ----------------
    double err = 0.0;
    if (valid) {
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
            const size_t idx = obase + wave + 4 * q;
            double o;
            if (job.epi == EPI_RAW) {
                o = lse[q];
            } else if (job.epi == EPI_SCALE) {
                const double lm = job.aux[idx];
                o = (lm == -INFINITY) ? -INFINITY : lm - lse[q];
                if (job.old != nullptr && lm != -INFINITY)
                    err += exp2(lm) * fabs(expm1((job.old[idx] - o) * kLn2));
            } else {
                const double bse = job.aux[idx];
                o = (bse == -INFINITY || lse[q] == -INFINITY) ? -INFINITY : bse + lse[q];
            }
            job.out[idx] = o;
        }
    }
    if (job.epi == EPI_SCALE && job.partial != nullptr) {
        __syncthreads();
        const double t = block_sum_fixed(err, lds);
        if (threadIdx.x == 0) job.partial[tile] = t;
    }
}

template <int NT, int KC, bool F64EXP, bool SPARSE>
int launch_t(const ConvJob *d_jobs, int nblocks, const int32_t *d_block_job, int R_max, hipStream_t s) {
    const int HW = kTile + 2 * R_max;
    size_t lds = static_cast<size_t>(HW) * HW * KC * sizeof(double);
    if (SPARSE) lds += static_cast<size_t>(kListLds) * sizeof(ListEntry);  // staged lists of the sparse path
    if (lds < kConvThreads * sizeof(double)) lds = kConvThreads * sizeof(double);
    if (lds > 65536)
        SE2_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_conv_lse<NT, KC, F64EXP, SPARSE>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    hipLaunchKernelGGL((k_conv_lse<NT, KC, F64EXP, SPARSE>), dim3(nblocks), dim3(kConvThreads), lds, s, d_jobs,
                       d_block_job);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

}  // namespace

bool conv_lse_sparse_fits(int nt, int R) {
    const int HW = kTile + 2 * R;
    return static_cast<size_t>(HW) * HW * nt * sizeof(double) <= kSparseLdsMax;
}

int launch_conv_lse(const ConvJob *d_jobs, int njobs, int nblocks, const int32_t *d_block_job, int nt, int R_max,
                    bool f64exp, bool sparse, hipStream_t s) {
    (void)njobs;
    if (nblocks <= 0) return SE2_OK;
    if (R_max < 0 || R_max > kMaxRadius) return SE2_EINVAL;
    const int HW = kTile + 2 * R_max;
    if (sparse && !f64exp && conv_lse_sparse_fits(nt, R_max)) {
        switch (nt) {
            case 8: return launch_t<8, 8, false, true>(d_jobs, nblocks, d_block_job, R_max, s);
            case 16: return launch_t<16, 16, false, true>(d_jobs, nblocks, d_block_job, R_max, s);
            case 32: return launch_t<32, 32, false, true>(d_jobs, nblocks, d_block_job, R_max, s);
            default: return SE2_EINVAL;
        }
    }
    const bool kc16 = HW * HW * 16 * 8 <= 65536;
    switch (nt) {
        case 8:
            return f64exp ? launch_t<8, 8, true, false>(d_jobs, nblocks, d_block_job, R_max, s)
                          : launch_t<8, 8, false, false>(d_jobs, nblocks, d_block_job, R_max, s);
        case 16:
            if (kc16)
                return f64exp ? launch_t<16, 16, true, false>(d_jobs, nblocks, d_block_job, R_max, s)
                              : launch_t<16, 16, false, false>(d_jobs, nblocks, d_block_job, R_max, s);
            return f64exp ? launch_t<16, 8, true, false>(d_jobs, nblocks, d_block_job, R_max, s)
                          : launch_t<16, 8, false, false>(d_jobs, nblocks, d_block_job, R_max, s);
        case 32:
            if (kc16)
                return f64exp ? launch_t<32, 16, true, false>(d_jobs, nblocks, d_block_job, R_max, s)
                              : launch_t<32, 16, false, false>(d_jobs, nblocks, d_block_job, R_max, s);
            return f64exp ? launch_t<32, 8, true, false>(d_jobs, nblocks, d_block_job, R_max, s)
                          : launch_t<32, 8, false, false>(d_jobs, nblocks, d_block_job, R_max, s);
        default:
            return SE2_EINVAL;
    }
}

}  // namespace se2
