// Log-domain SE(2) group convolution with fused scaling epilogues (gfx950).
//
// For every output element (x, ko) of a job:
//     LSE(x, ko) = log2 sum_{d in window, ki} 2^( L2[d][ko][ki] + in(x - d, ki) )
// i.e. log2 of (K * 2^in)(x, ko), the operator K b of the Sinkhorn updates
// (Section 4.1) written as the group convolution of Section 4.2, evaluated term
// by term in the log domain.
//
// Dense evaluation (exact): every window entry is visited.  A first pass finds
// the per-output maximum M of the exponents in FP32; the second forms each
// exponent u = L2 + in - M in FP64 (the two addends are O(10^3) and nearly cancel
// for the terms that matter), rounds u to FP32 and takes a native exp2.  Partial
// sums over one window row are FP32 and are combined in FP64.  F64EXP uses an
// FP64 exp2 and FP64 sums throughout (the checking path).
//
// Certified pruning (jobs that carry term lists).  A dense visit of a tile records,
// for each output orientation ko, the union over the tile's 64 pixels of the window
// terms (d, ki) whose exponent is within kListCut of that output's maximum, the
// maximum itself (mref) and the input halo it saw (ref).  A later visit measures
// the drift delta = in - ref over the halo, lo <= delta <= hi.  Every unlisted term
// had u <= -kListCut at reference time; its exponent grew by at most hi and the
// maximum fell by at most -lo, so now u <= -kListCut + (hi - lo).  While the spread
// hi - lo <= kDriftSpread the unlisted terms are each below 2^-(kListCut -
// kDriftSpread) = 2^-48 of the largest term and the tile evaluates its lists only,
// shifting exponents by mref + (lo + hi)/2 (within 2^+-spread/2 of the true
// maximum).  Otherwise the tile is rebuilt densely.  Every decision is per tile and
// depends only on that job's data, so results are independent of the other jobs in
// a launch.
//
// Kernels.  k_conv_lse evaluates jobs without lists densely, one 8 x 8 output tile
// (all ko) per workgroup: lane = pixel of the tile, wave w owns ko = w, w+4, ... .
// Pruned jobs run k_sparse (certificate, then list evaluation; min(nt, 16) waves
// per tile) followed by k_rebuild, which takes the tiles whose certificate failed and
// spreads each over ntheta workgroups (one per ko, the window rows split over the
// four waves), so that a few rebuilds never hold a launch on one compute unit.
//
// The input halo (8+2R)^2 is staged in LDS as FP64, theta-major so that the 64 lanes
// of a wave read neighbouring addresses.  Kernel values of the dense visits are
// wave-uniform and read through the scalar cache.
#include <hip/hip_runtime.h>

#include <cmath>

#include "conv_dev.h"
#include "se2_internal.h"
#include "launch.h"

namespace se2 {

namespace {

typedef const __attribute__((address_space(4))) double *cdptr;
typedef const __attribute__((address_space(4))) float *cfptr;

constexpr int kHaloBatch = 4;        // halo items each thread loads before storing any
constexpr int kHaloBatchSparse = 2;  // the same in the sparse kernel (fewer registers)

// Stage the input halo (8+2R)^2 x KC orientations (from k0) in LDS as [kc][hy][hx],
// -inf outside the grid.  A thread takes 4 consecutive orientations of one halo pixel
// per item (two 16-byte loads), and issues the loads of kHaloBatch items (clamped
// addresses, no branches) before it stores any; hy = p / HW via a float reciprocal
// (exact for p < 2^20: the +0.5 keeps the rounding error far below the gap to an
// integer).
template <int KC, int NTH = kConvThreads, int BATCH = kHaloBatch>
__device__ __forceinline__ void load_halo(double *lds, const double *in_, int nt, int k0, int x0, int y0, int R,
                                          int HW, int nx, int ny) {
    static_assert(KC % 4 == 0, "orientations are staged in quads");
    constexpr int QK = KC / 4;
    const gdptr in = (gdptr)in_;
    const int npix = HW * HW;
    const int total = npix * QK;
    const float inv = 1.0f / static_cast<float>(HW);
    for (int e0 = 0; e0 < total; e0 += BATCH * NTH) {
        double v[BATCH][4];
        bool ok[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const int e = min(e0 + u * NTH + static_cast<int>(threadIdx.x), total - 1);
            const int p = e / QK;
            const int kq = e - p * QK;
            const int hy = static_cast<int>((static_cast<float>(p) + 0.5f) * inv);
            const int hx = p - hy * HW;
            const int gy = y0 - R + hy, gx = x0 - R + hx;
            ok[u] = gy >= 0 && gy < ny && gx >= 0 && gx < nx;
            const int cy = min(max(gy, 0), ny - 1), cx = min(max(gx, 0), nx - 1);
            const gdptr src = in + (static_cast<size_t>(cy * nx + cx)) * nt + k0 + 4 * kq;
#pragma unroll
            for (int c = 0; c < 4; ++c) v[u][c] = src[c];
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const int e = e0 + u * NTH + static_cast<int>(threadIdx.x);
            if (e < total) {
                const int p = e / QK;
                const int kq = e - p * QK;
#pragma unroll
                for (int c = 0; c < 4; ++c) lds[(4 * kq + c) * npix + p] = ok[u] ? v[u][c] : -INFINITY;
            }
        }
    }
}

// Sum over the 256 threads: butterflies within each wave, then the four wave sums in
// wave order (fixed order, independent of timing).  `scratch` holds 4 doubles.
__device__ __forceinline__ double block_sum_waves(double v, double *scratch) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((scratch[0] + scratch[1]) + scratch[2]) + scratch[3];
}

__device__ __forceinline__ float wave_max(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}


// LDS offset of list term j relative to the output pixel: ki*npix + (R-dy)*HW + (R-dx).
__device__ __forceinline__ int term_offset(uint32_t term, int nt, int R, int W, int HW, int npix) {
    const int kc = static_cast<int>(term) % nt, r = static_cast<int>(term) / nt;
    const int dyi = r / W, dxi = r - dyi * W;
    return kc * npix + (2 * R - dyi) * HW + (2 * R - dxi);
}

// Dense evaluation of one 8 x 8 tile of a job at NQ output orientations per wave: lse[q]
// receives the LSE of the lane's pixel at orientation ko(q) (wave-uniform; lane = pixel
// px + 8 py of the tile; rows and columns past the grid compute clamped garbage that the
// caller does not store).  The input halo is staged in LDS KC orientations at a time (twice
// when KC < NT: the max pass, then the sum).  With MAYIDLE, a wave with active == false takes
// part in the staging only.  Each output's maximum and sum run over the same terms in the same
// order whichever orientations share the wave, so the result of an output does not depend on
// NQ.  (ko is a callable rather than an array so that the dense engine's ko = wave + 4 q stays
// a compile-time stride: an array there cost the one-solve launches 1.5x.)
template <int NT, int KC, bool F64EXP, int NQ, bool MAYIDLE, class KoF>
__device__ __forceinline__ void dense_tile_at(const ConvJob &job, double *lds, int x0, int y0, int px, int py,
                                              KoF ko, bool active, double (&lse)[NQ]) {
    constexpr int NJ = NQ;
    const int R = job.R, W = 2 * R + 1, HW = kTile + 2 * R, npix = HW * HW;
    const int nx = job.nx, ny = job.ny;
    const cdptr L64 = (cdptr)(job.L64);
    const cfptr L32 = (cfptr)(job.L32);
    float mx[NJ];
#pragma unroll
    for (int q = 0; q < NJ; ++q) mx[q] = -INFINITY;
    for (int k0 = 0; k0 < NT; k0 += KC) {
        if (k0 > 0) __syncthreads();
        load_halo<KC>(lds, job.in, NT, k0, x0, y0, R, HW, nx, ny);
        __syncthreads();
        if (MAYIDLE && !active) continue;
        for (int dy = -R; dy <= R; ++dy) {
            for (int dx = -R; dx <= R; ++dx) {
                const int hb = (py + R - dy) * HW + (px + R - dx);
                const cfptr Lr = L32 + (static_cast<size_t>((dy + R) * W + (dx + R)) * NT) * NT + k0;
#pragma unroll
                for (int kc = 0; kc < KC; ++kc) {
                    const float v = static_cast<float>(lds[kc * npix + hb]);
#pragma unroll
                    for (int q = 0; q < NJ; ++q) mx[q] = fmaxf(mx[q], v + Lr[ko(q) * NT + kc]);
                }
            }
        }
    }
    double M[NJ], S[NJ];
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        M[q] = (mx[q] == -INFINITY) ? 0.0 : static_cast<double>(mx[q]);
        S[q] = 0.0;
    }
    for (int k0 = 0; k0 < NT; k0 += KC) {
        if (NT > KC) {
            __syncthreads();
            load_halo<KC>(lds, job.in, NT, k0, x0, y0, R, HW, nx, ny);
            __syncthreads();
        }
        if (MAYIDLE && !active) continue;
        for (int dy = -R; dy <= R; ++dy) {
            if constexpr (F64EXP) {
                for (int dx = -R; dx <= R; ++dx) {
                    const int hb = (py + R - dy) * HW + (px + R - dx);
                    const cdptr Lr = L64 + (static_cast<size_t>((dy + R) * W + (dx + R)) * NT) * NT + k0;
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc) {
                        const double v = lds[kc * npix + hb];
#pragma unroll
                        for (int q = 0; q < NJ; ++q) S[q] += exp2((v + Lr[ko(q) * NT + kc]) - M[q]);
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
                        for (int q = 0; q < NJ; ++q)
                            srow[q] += __builtin_amdgcn_exp2f(
                                static_cast<float>((v + Lr[ko(q) * NT + kc]) - M[q]));
                    }
                }
#pragma unroll
                for (int q = 0; q < NJ; ++q) S[q] += static_cast<double>(srow[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NJ; ++q) lse[q] = (S[q] > 0.0) ? M[q] + log2(S[q]) : -INFINITY;
}

// All NT orientations of the tile: wave w takes ko = w, w + 4, ... .
template <int NT, int KC, bool F64EXP>
__device__ __forceinline__ void dense_tile(const ConvJob &job, double *lds, int x0, int y0, int px, int py, int wave,
                                           double (&lse)[NT / 4]) {
    dense_tile_at<NT, KC, F64EXP, NT / 4, false>(job, lds, x0, y0, px, py, [wave](int q) { return wave + 4 * q; },
                                                 true, lse);
}

template <int NT, int KC, bool F64EXP>
__global__ __launch_bounds__(kConvThreads) void k_conv_lse(const ConvJob *__restrict__ jobs,
                                                           const int32_t *__restrict__ block_job) {
    extern __shared__ double lds[];
    __shared__ double s_sum[8];
    constexpr int NJ = NT / 4;
    const int j = block_job[blockIdx.x];
    const ConvJob job = jobs[j];
    const int tile = static_cast<int>(blockIdx.x) - job.first_block;
    const int ty = tile / job.tiles_x;
    const int tx = tile - ty * job.tiles_x;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int R = job.R;
    const int nx = job.nx, ny = job.ny;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int px = lane & 7, py = lane >> 3;
    const int gx = x0 + px, gy = y0 + py;
    const bool valid = gx < nx && gy < ny;
    const size_t obase = (static_cast<size_t>(gy) * nx + gx) * NT;

    double lse[NJ];
    dense_tile<NT, KC, F64EXP>(job, lds, x0, y0, px, py, wave, lse);

    // ---------------- work counters (diagnostics) ----------------
    if (job.work != nullptr) {
        // in-grid terms of this lane's outputs
        double w = 0.0;
        if (valid) {
            const int cx = min(R, gx) + min(R, nx - 1 - gx) + 1;
            const int cy = min(R, gy) + min(R, ny - 1 - gy) + 1;
            w = static_cast<double>(cx) * cy * NT * NJ;
        }
        const double t = block_sum_waves(w, s_sum);
        if (threadIdx.x == 0) job.work[2 * tile] += t;
    }

    // ---------------- epilogue ----------------
    double err = 0.0;
    if (valid) {
#pragma unroll
        for (int q = 0; q < NJ; ++q) err += epilogue(job, obase + wave + 4 * q, lse[q]);
    }
    if (job.epi == EPI_SCALE && job.partial != nullptr) {
        // partials are laid out [tile][nt]; a tile evaluated here fills slot 0
        const double t = block_sum_waves(err, s_sum + 4);
        if (static_cast<int>(threadIdx.x) < NT)
            job.partial[static_cast<size_t>(tile) * NT + threadIdx.x] = (threadIdx.x == 0) ? t : 0.0;
    }
}

// Workgroup i is dispatched to XCD i % 8; logical blocks are handed out so that each
// XCD gets a contiguous range (neighbouring tiles of a solve share that XCD's L2).
// Returns -1 for the padding blocks of a grid of 8 * ceil(nblocks / 8).
__device__ __forceinline__ int xcd_block(int nblocks) {
    const int per = (nblocks + 7) >> 3;
    const int i = static_cast<int>(blockIdx.x);
    const int lb = (i & 7) * per + (i >> 3);
    return lb < nblocks ? lb : -1;
}

__host__ __forceinline__ int xcd_grid(int nblocks) { return ((nblocks + 7) >> 3) << 3; }

// Scaling epilogue with the per-output operands already loaded (aux, old).
__device__ __forceinline__ double epilogue_pre(const ConvJob &job, size_t idx, double lse, double lm, double od) {
    double o, err = 0.0;
    if (job.epi == EPI_RAW) {
        o = lse;
    } else if (job.epi == EPI_SCALE) {
        o = (lm == -INFINITY) ? -INFINITY : lm - lse;
        if (job.old != nullptr && lm != -INFINITY) err = exp2(lm) * fabs(expm1((od - o) * kLn2));
    } else {
        o = (lm == -INFINITY || lse == -INFINITY) ? -INFINITY : lm + lse;
    }
    ((gdptr_w)job.out)[idx] = o;
    return err;
}

// Sum over the `len` packed list entries at Lp (wave-uniform) of 2^(L + in - M) for
// the lane's output, whose input halo starts at LDS offset `base`; groups of 8 entries
// are summed in FP32, the groups in FP64.  Groups alternate between two register sets, and the next group is
// requested only once the current group's gathers are back: lgkmcnt counts the scalar
// loads as well, and these return out of order, so a request issued before the
// gathers would be waited for together with them.  Reads run up to 8 entries past the
// list (loaded, never used).
__device__ __forceinline__ double eval_list(const cdptr Lp, int len, double M, const double *lds, int base) {
    constexpr uint32_t kMask = (1u << kOffBits) - 1u;
    double S = 0.0;
    auto step = [&](const double (&P)[8], double (&Q)[8], const cdptr nxt) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v[u] = lds[static_cast<int>(static_cast<uint32_t>(__double2loint(P[u])) & kMask) + base];
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the gathers
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 8; ++u) Q[u] = nxt[u];
        __builtin_amdgcn_sched_barrier(0);
        float s8 = 0.0f;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const unsigned int lo32 = static_cast<unsigned int>(__double2loint(P[u]));
            const double lv = __hiloint2double(__double2hiint(P[u]), static_cast<int>(lo32 & ~kMask));
            s8 += __builtin_amdgcn_exp2f(static_cast<float>((lv + v[u]) - M));
        }
        S += static_cast<double>(s8);
    };
    // the last r < 8 entries as a full group: the unused slots read the lane's own halo
    // corner with a kernel value of -inf, i.e. add exact zeros (selects on the scalar unit)
    auto tail = [&](const double (&P)[8], int r) {
        double T8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            T8[u] = (u < r) ? P[u] : __hiloint2double(static_cast<int>(0xfff00000u), 0);
        float st = 0.0f;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const unsigned int lo32 = static_cast<unsigned int>(__double2loint(T8[u]));
            const double lv = __hiloint2double(__double2hiint(T8[u]), static_cast<int>(lo32 & ~kMask));
            const double v = lds[static_cast<int>(lo32 & kMask) + base];
            st += __builtin_amdgcn_exp2f(static_cast<float>((lv + v) - M));
        }
        S += static_cast<double>(st);
    };
    const int n8 = len & ~7;
    double A[8], B[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) A[u] = Lp[u];
    int e = 0;
    for (; e + 16 <= n8; e += 16) {
        step(A, B, Lp + e + 8);
        step(B, A, Lp + e + 16);
    }
    if (e < n8) {
        step(A, B, Lp + e + 8);
        tail(B, len - n8);
    } else {
        tail(A, len - n8);
    }
    return S;
}

// Certified sparse evaluation of pruned jobs: one workgroup per 8 x 8 tile with
// NW = min(nt, 16) waves (wave w owns ko = w, w+NW, ...; lane = pixel).  Every global
// load of the tile's lanes (list lengths, per-output operands, the input halo and its
// reference) is issued before the certificate is decided.  A tile whose certificate
// fails is appended to the rebuild list and left to k_rebuild.
template <int NT>
__global__ __launch_bounds__(64 * (NT < 16 ? NT : 16)) void k_sparse(const ConvJob *__restrict__ jobs,
                                                                     const int32_t *__restrict__ block_job,
                                                                     int nblocks, int2 *__restrict__ rebuild,
                                                                     int *__restrict__ rebuild_count,
                                                                     int *__restrict__ next_count) {
    constexpr int NW = NT < 16 ? NT : 16;  // waves
    constexpr int NTH = 64 * NW;
    constexpr int NJ = NT / NW;             // orientations per wave
    static_assert(kListMax >= 16 && kListMax % 8 == 0, "list regions hold whole groups of 8");
    typedef const __attribute__((address_space(4))) int32_t *ciptr;
    extern __shared__ double lds[];
    __shared__ float s_lo[NW], s_hi[NW];
    __shared__ int s_bad[NW];
    __shared__ double s_err[NW], s_work[NW];
    // the counter of the following launch (idle now: the previous rebuild has finished)
    if (blockIdx.x == 0 && threadIdx.x == 0) *next_count = 0;
    const int lb = xcd_block(nblocks);
    if (lb < 0) return;
    const int j = block_job[lb];
    const ConvJob job = jobs[j];
    const int tile = lb - job.first_block;
    const int ty = tile / job.tiles_x;
    const int tx = tile - ty * job.tiles_x;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int R = job.R, HW = kTile + 2 * R, npix = HW * HW;
    const int nx = job.nx, ny = job.ny;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int px = lane & 7, py = lane >> 3;
    const int gx = x0 + px, gy = y0 + py;
    const bool valid = gx < nx && gy < ny;
    const size_t obase = (static_cast<size_t>(min(gy, ny - 1)) * nx + min(gx, nx - 1)) * NT;

    // ---------------- prefetch ----------------
    int n[NJ];
    float mr[NJ];
    double ax[NJ], od[NJ];
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        const int ko = wave + NW * q;
        n[q] = ((ciptr)(job.len))[static_cast<size_t>(tile) * NT + ko];
        mr[q] = ((gfptr)job.mref)[obase + ko];
        ax[q] = (job.epi != EPI_RAW) ? ((gdptr)job.aux)[obase + ko] : 0.0;
        od[q] = (job.old != nullptr) ? ((gdptr)job.old)[obase + ko] : 0.0;
    }

    // ---------------- halo and certificate ----------------
    // drift delta = in - ref over the halo; only its spread matters: a common shift of the
    // inputs moves every exponent and the maximum alike
    // reference halo, pixel-major [p][kc] in FP32
    const gfptr ref = (gfptr)(job.ref + static_cast<size_t>(tile) * NT * npix);
    const gdptr in = (gdptr)job.in;
    float dlo = INFINITY, dhi = -INFINITY;
    bool bad = false;
    int pf[NJ];
    {
        constexpr int QK = NT / 4;
        const float inv = 1.0f / static_cast<float>(HW);
        const int total = npix * QK;
        for (int e0 = 0; e0 < total; e0 += kHaloBatchSparse * NTH) {
            double va[kHaloBatchSparse][4];
            float vb[kHaloBatchSparse][4];
            bool ok[kHaloBatchSparse];
#pragma unroll
            for (int u = 0; u < kHaloBatchSparse; ++u) {
                const int e = min(e0 + u * NTH + static_cast<int>(threadIdx.x), total - 1);
                const int p = e / QK;
                const int kq = e - p * QK;
                const int hy = static_cast<int>((static_cast<float>(p) + 0.5f) * inv);
                const int hx = p - hy * HW;
                const int qy = y0 - R + hy, qx = x0 - R + hx;
                ok[u] = qy >= 0 && qy < ny && qx >= 0 && qx < nx;
                const int cy = min(max(qy, 0), ny - 1), cx = min(max(qx, 0), nx - 1);
                const gdptr src = in + static_cast<size_t>(cy * nx + cx) * NT + 4 * kq;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    va[u][c] = src[c];
                    vb[u][c] = ref[4 * e + c];
                }
            }
            if (e0 == 0) {
                // touch every 64-byte line of the lists the waves will read, so that the
                // scalar reads of the evaluation hit the L2 (lane = line)
#pragma unroll
                for (int q = 0; q < NJ; ++q) {
                    const int lines = (n[q] + 7) >> 3;
                    const giptr L32 = (giptr)(job.lists + (static_cast<size_t>(tile) * NT + wave + NW * q) * job.lmax);
                    pf[q] = L32[16 * min(lane, max(lines - 1, 0)) + 1];
                }
            }
#pragma unroll
            for (int u = 0; u < kHaloBatchSparse; ++u) {
                const int e = e0 + u * NTH + static_cast<int>(threadIdx.x);
                if (e < total) {
                    const int p = e / QK;
                    const int kq = e - p * QK;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const float b = vb[u][c];
                        const double a = ok[u] ? va[u][c] : -INFINITY;
                        lds[(4 * kq + c) * npix + p] = a;
                        // both -inf: NaN, which the min/max below skip; one side -inf: +-inf,
                        // which fails the certificate
                        const float df = static_cast<float>(a - static_cast<double>(b));
                        dlo = fminf(dlo, df);
                        dhi = fmaxf(dhi, df);
                        bad = bad || (fabsf(b) >= kRefMax && b != -INFINITY) || (a != a);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NJ; ++q) bad = bad || n[q] < 0;  // no list (never built or overflowed)
    dlo = -wave_max(-dlo);
    dhi = wave_max(dhi);
    const bool wbad = __ballot(bad) != 0ull;
    if (lane == 0) {
        s_lo[wave] = dlo;
        s_hi[wave] = dhi;
        s_bad[wave] = wbad ? 1 : 0;
    }
    __syncthreads();
    float lo = s_lo[0], hi = s_hi[0];
    int anybad = s_bad[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
        lo = fminf(lo, s_lo[w]);
        hi = fmaxf(hi, s_hi[w]);
        anybad |= s_bad[w];
    }
    // all entries -inf on both sides: no spread at all (an infinite spread fails)
    const float spread = (hi >= lo) ? hi - lo : 0.0f;
    const float shift = (hi >= lo) ? 0.5f * (hi + lo) : 0.0f;
    if (anybad != 0 || !(spread + kRefMargin <= kDriftSpread)) {
        // left to the rebuild kernel (block-uniform exit, nothing written here)
        if (threadIdx.x == 0) {
            const int slot = atomicAdd(rebuild_count, 1);
            rebuild[slot] = make_int2(j, tile);
        }
        return;
    }

    // ---------------- certified sparse evaluation ----------------
    // List entries are wave-uniform: they come through the scalar cache into SGPRs and
    // are unpacked on the scalar unit, so LDS bandwidth goes to the per-lane halo
    // gathers only.  The touch loads above brought the lists' lines into the L2.
    const int base = py * HW + px;
    double err = 0.0, work = 0.0;
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        const int ko = wave + NW * q;
        // the reference maximum moved with the inputs by shift +- spread/2
        const double M = (mr[q] == -INFINITY) ? 0.0 : static_cast<double>(mr[q]) + static_cast<double>(shift);
        const cdptr Lp = (cdptr)(job.lists + (static_cast<size_t>(tile) * NT + ko) * job.lmax);
        const int nq = n[q];
        const double S = eval_list(Lp, nq, M, lds, base);
        const double lse = (mr[q] == -INFINITY || !(S > 0.0)) ? -INFINITY : M + log2(S);
        if (valid) {
            err += epilogue_pre(job, obase + ko, lse, ax[q], od[q]);
            // the touched list word is the high half of a finite kernel value whenever
            // nq > 0, never this NaN pattern: the test only keeps the touch load alive
            work += static_cast<double>(nq) + ((nq > 0 && pf[q] == 0x7ff80001) ? 1.0 : 0.0);
        }
    }
    // error partial of the tile (slot 0 of [tile][nt]) and the work counter, in wave order
    err = wave_sum(err);
    work = wave_sum(work);
    if (lane == 0) {
        s_err[wave] = err;
        s_work[wave] = work;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double te = 0.0, tw = 0.0;
        for (int w = 0; w < NW; ++w) {
            te += s_err[w];
            tw += s_work[w];
        }
        if (job.epi == EPI_SCALE && job.partial != nullptr) job.partial[static_cast<size_t>(tile) * NT] = te;
        if (job.work != nullptr) job.work[2 * tile + 1] += tw;
    }
    if (job.epi == EPI_SCALE && job.partial != nullptr && threadIdx.x > 0 && static_cast<int>(threadIdx.x) < NT)
        job.partial[static_cast<size_t>(tile) * NT + threadIdx.x] = 0.0;
}

// Dense rebuild of the tiles listed by k_sparse: one workgroup of RBW (8 or 16) waves
// per (tile, ko) item, lane = pixel of the tile.  The window's (dy, dx) pairs are dealt
// to the waves round-robin; partial maxima and sums are combined in LDS.  Each wave
// records, per pair, a ballot mask of the orientations ki whose term is within
// kListCut (+1) of the maximum for some pixel; a block-wide prefix sum over the masks
// places every listed term, in (pair, ki) order, and the packed entries are written.
//
// The sum is split the same way for either width: pair r belongs to class r mod 16,
// each class is summed over its pairs in increasing r, classes c and c + 8 are added,
// and the eight results are summed in order of c.  A rebuild of 8 waves keeps two
// accumulators per wave (classes w and w + 8), one of 16 waves one per wave; both give
// bitwise identical outputs and lists, so the width is a free choice per launch.  Wide
// items finish sooner (half the pairs per wave); narrow workgroups pack two to a CU
// (~118 VGPRs: 4 waves per SIMD), against one wide one, and win when many tiles are
// queued.
constexpr int kRbClasses = 16;

template <int NT, int RBW>
__global__ __launch_bounds__(64 * RBW) void k_rebuild(const ConvJob *__restrict__ jobs,
                                                      const int2 *__restrict__ rebuild,
                                                      const int *__restrict__ rebuild_count,
                                                      int *__restrict__ published) {
    static_assert(RBW == 8 || RBW == 16, "8 or 16 waves per item");
    constexpr int NTH = 64 * RBW;
    extern __shared__ double lds[];
    __shared__ float s_mx[RBW][64];
    __shared__ double s_S[RBW][64];
    __shared__ int s_wsum[RBW];
    static_assert(NT <= 32, "masks hold up to 32 input orientations");
    const int nitems = *rebuild_count * NT;
    // the host reads this (pinned memory, a vector store) to size the next rebuild
    if (published != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *(volatile int *)published = nitems;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int px = lane & 7, py = lane >> 3;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int2 it = rebuild[item / NT];
        const int ko = item % NT;
        const ConvJob job = jobs[it.x];
        const int tile = it.y;
        const int ty = tile / job.tiles_x;
        const int tx = tile - ty * job.tiles_x;
        const int x0 = tx * kTile, y0 = ty * kTile;
        const int R = job.R, W = 2 * R + 1, HW = kTile + 2 * R, npix = HW * HW;
        const int nx = job.nx, ny = job.ny;
        const int gx = x0 + px, gy = y0 + py;
        const bool valid = gx < nx && gy < ny;
        const size_t idx = (static_cast<size_t>(gy) * nx + gx) * NT + ko;
        const cdptr L64 = (cdptr)(job.L64);
        const cfptr L32 = (cfptr)(job.L32);
        // LDS: halo, then W*W masks (one per window pair), then up to lmax term indices
        uint32_t *masks = reinterpret_cast<uint32_t *>(lds + static_cast<size_t>(NT) * npix);
        uint32_t *terms = masks + W * W;

        __syncthreads();  // LDS of the previous item is free
        load_halo<NT, NTH, 2>(lds, job.in, NT, 0, x0, y0, R, HW, nx, ny);
        __syncthreads();

        // pass 1: maximum over this wave's pairs
        float mx = -INFINITY;
        for (int r = wave; r < W * W; r += RBW) {
            const int dyi = r / W, dxi = r - dyi * W;  // dy = dyi - R, dx = dxi - R
            const int hb = (py + 2 * R - dyi) * HW + (px + 2 * R - dxi);
            const cfptr Lr = L32 + (static_cast<size_t>(r) * NT + ko) * NT;
#pragma unroll 8
            for (int kc = 0; kc < NT; ++kc) mx = fmaxf(mx, static_cast<float>(lds[kc * npix + hb]) + Lr[kc]);
        }
        s_mx[wave][lane] = mx;
        __syncthreads();
        mx = s_mx[0][lane];
#pragma unroll
        for (int w = 1; w < RBW; ++w) mx = fmaxf(mx, s_mx[w][lane]);
        const double M = (mx == -INFINITY) ? 0.0 : static_cast<double>(mx);

        // pass 2: sum (per class) and membership masks of this wave's pairs
        const unsigned long long vmask = __builtin_amdgcn_ballot_w64(valid);  // pixels inside the grid
        double Sc[2] = {0.0, 0.0};  // classes wave and wave + 8 (RBW = 8); class wave (RBW = 16)
        int half = 0;
        for (int r = wave; r < W * W; r += RBW) {
            const int dyi = r / W, dxi = r - dyi * W;
            const int hb = (py + 2 * R - dyi) * HW + (px + 2 * R - dxi);
            const cdptr Lr = L64 + (static_cast<size_t>(r) * NT + ko) * NT;
            float srow = 0.0f;
            uint32_t m = 0u;
#pragma unroll 4
            for (int kc = 0; kc < NT; ++kc) {
                const double u = (lds[kc * npix + hb] + Lr[kc]) - M;
                srow += __builtin_amdgcn_exp2f(static_cast<float>(u));
                // any lane inside the grid: the ballot of the bare compare, masked with
                // the valid lanes and tested by a select, keeps the mask on the scalar unit
                const unsigned long long b = __builtin_amdgcn_ballot_w64(u >= -(kListCut + 1.0)) & vmask;
                m |= (b != 0ull) ? (1u << kc) : 0u;
            }
            if (lane == 0) masks[r] = m;
            if (RBW == kRbClasses / 2 && half) Sc[1] += static_cast<double>(srow);
            else Sc[0] += static_cast<double>(srow);
            half ^= 1;
        }
        // slot w holds classes w and w + 8 added (RBW = 8) or class w alone (RBW = 16)
        s_S[wave][lane] = (RBW == kRbClasses / 2) ? Sc[0] + Sc[1] : Sc[0];
        __syncthreads();
        double S;
        if constexpr (RBW == kRbClasses / 2) {
            S = s_S[0][lane];
#pragma unroll
            for (int w = 1; w < RBW; ++w) S += s_S[w][lane];
        } else {
            S = s_S[0][lane] + s_S[8][lane];
#pragma unroll
            for (int w = 1; w < kRbClasses / 2; ++w) S += s_S[w][lane] + s_S[w + 8][lane];
        }
        const double lse = (S > 0.0) ? M + log2(S) : -INFINITY;

        // compaction: exclusive prefix sum of the mask popcounts over the pairs, in
        // rounds of NTH pairs
        int base = 0;
        for (int r0 = 0; r0 < W * W; r0 += NTH) {
            const int r = r0 + static_cast<int>(threadIdx.x);
            const uint32_t m = (r < W * W) ? masks[r] : 0u;
            const int c = __builtin_popcount(m);
            int incl = c;  // inclusive scan within the wave
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(incl, off);
                if (lane >= off) incl += t;
            }
            if (lane == 63) s_wsum[wave] = incl;
            __syncthreads();
            int wbase = base;
            for (int w = 0; w < wave; ++w) wbase += s_wsum[w];
            int total = base;
            for (int w = 0; w < RBW; ++w) total += s_wsum[w];
            int pos = wbase + incl - c;
            uint32_t mm = m;
            while (mm != 0u) {
                const int b = __builtin_ctz(mm);
                mm &= mm - 1u;
                if (pos < job.lmax) terms[pos] = static_cast<uint32_t>(r * NT + b);
                ++pos;
            }
            base = total;
            __syncthreads();  // s_wsum reused by the next round
        }
        const int cnt = base;
        if (threadIdx.x == 0) ((int32_t *)job.len)[static_cast<size_t>(tile) * NT + ko] = (cnt <= job.lmax) ? cnt : -1;

        if (wave == 0) {
            if (valid) ((gfptr_w)job.mref)[idx] = mx;
            // epilogue of the 64 outputs (pixel, ko) and this item's error partial
            const double err = valid ? epilogue(job, idx, lse) : 0.0;
            const double es = wave_sum(err);
            if (job.epi == EPI_SCALE && job.partial != nullptr && lane == 0)
                job.partial[static_cast<size_t>(tile) * NT + ko] = es;
            if (job.work != nullptr) {
                double w = 0.0;
                if (valid) {
                    const int cx = min(R, gx) + min(R, nx - 1 - gx) + 1;
                    const int cy = min(R, gy) + min(R, ny - 1 - gy) + 1;
                    w = static_cast<double>(cx) * cy * NT;
                }
                const double ws = wave_sum(w);
                if (lane == 0) atomicAdd(&job.work[2 * tile], ws);
            }
        }
        {
            // packed entries of (tile, ko), written by all threads
            const int n = cnt <= job.lmax ? cnt : 0;
            const gdptr_w dst = (gdptr_w)(job.lists + (static_cast<size_t>(tile) * NT + ko) * job.lmax);
            for (int e = threadIdx.x; e < n; e += NTH) {
                const uint32_t term = terms[e];
                const double Lv = ((gdptr)job.L64)[((term / NT) * NT + ko) * NT + term % NT];
                const uint32_t off = static_cast<uint32_t>(term_offset(term, NT, R, W, HW, npix));
                const unsigned long long b =
                    (static_cast<unsigned long long>(__double_as_longlong(Lv)) & ~((1ull << kOffBits) - 1ull)) | off;
                dst[e] = __longlong_as_double(static_cast<long long>(b));
            }
        }
        if (ko == 0) {
            // reference halo, pixel-major [p][kc]
            const gfptr_w ref = (gfptr_w)(job.ref + static_cast<size_t>(tile) * NT * npix);
            for (int e = threadIdx.x; e < NT * npix; e += NTH) {
                const int p = e / NT, kc = e - p * NT;
                ref[e] = static_cast<float>(lds[kc * npix + p]);
            }
            if (job.dense_flag != nullptr && threadIdx.x == 0) job.dense_flag[tile] += 1;
        }
    }
}

// Exact log-domain recomputation of the (tile, ko) groups that the certificate of the
// matrix-core engines rejected.  An item (job, tile, ko mask) is one 8 x 8 tile with the
// orientations to recompute.  A workgroup stages the tile's halo as k_conv_lse does and
// evaluates the masked orientations only, the j-th set bit of the mask on wave j mod 4
// (NQ = ceil(popcount / 4) per wave; a wave's spare slot repeats the lowest masked
// orientation and is not stored).  It writes the outputs, error partial slots [tile][ko] and
// counters of the masked orientations only: the others were written by the matrix-core
// kernel, which for in-place updates has already replaced their previous values.  The
// outputs are the same bits as a dense visit of the whole tile.
__device__ __forceinline__ int nth_set_bit(uint32_t m, int j) {
    for (int i = 0; i < j; ++i) m &= m - 1u;
    return __builtin_ctz(m);
}

template <int NT, int KC, int NQ>
__device__ __forceinline__ void lse_tile_item(const ConvJob &job, double *lds, int tile, uint32_t mask, int wave,
                                              int lane) {
    const int p = __popc(mask);
    const int px = lane & 7, py = lane >> 3;
    const int ty = tile / job.tiles_x;
    const int tx = tile - ty * job.tiles_x;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int R = job.R;
    const int nx = job.nx, ny = job.ny;
    const int gx = x0 + px, gy = y0 + py;
    const bool valid = gx < nx && gy < ny;
    const size_t obase = (static_cast<size_t>(min(gy, ny - 1)) * nx + min(gx, nx - 1)) * NT;
    int ko[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int j = wave + 4 * q;
        ko[q] = __builtin_amdgcn_readfirstlane(nth_set_bit(mask, j < p ? j : 0));
    }
    double lse[NQ];
    dense_tile_at<NT, KC, false, NQ, true>(job, lds, x0, y0, px, py, [&ko](int q) { return ko[q]; }, wave < p, lse);
    double work = 0.0;
    if (valid) {
        const int cx = min(R, gx) + min(R, nx - 1 - gx) + 1;
        const int cy = min(R, gy) + min(R, ny - 1 - gy) + 1;
        work = static_cast<double>(cx) * cy * NT;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (wave + 4 * q >= p) continue;  // wave-uniform
        const double err = valid ? epilogue(job, obase + ko[q], lse[q]) : 0.0;
        const double es = wave_sum(err);
        if (job.epi == EPI_SCALE && job.partial != nullptr && lane == 0)
            job.partial[static_cast<size_t>(tile) * NT + ko[q]] = es;
        const double ws = wave_sum(work);
        if (job.work != nullptr && lane == 0) atomicAdd(&job.work[2 * tile], ws);
    }
}

template <int NT, int KC, int NQ = 1>
__device__ __forceinline__ void lse_tile_item_nq(int nq, const ConvJob &job, double *lds, int tile, uint32_t mask,
                                                 int wave, int lane) {
    if constexpr (NQ <= NT / 4) {
        if (nq <= NQ)
            lse_tile_item<NT, KC, NQ>(job, lds, tile, mask, wave, lane);
        else
            lse_tile_item_nq<NT, KC, NQ + 1>(nq, job, lds, tile, mask, wave, lane);
    }
}

template <int NT, int KC>
__global__ __launch_bounds__(kConvThreads) void k_lse_tiles(const ConvJob *__restrict__ jobs,
                                                            const int4 *__restrict__ items,
                                                            const int *__restrict__ count) {
    extern __shared__ double lds[];
    const int n = *count;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 v = items[it];
        const ConvJob job = jobs[v.x];
        const uint32_t mask = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(v.z));
        __syncthreads();  // the LDS of the previous item is free
        if (mask != 0u) lse_tile_item_nq<NT, KC>((__popc(mask) + 3) >> 2, job, lds, v.y, mask, wave, lane);
        if (job.fallbacks != nullptr && threadIdx.x == 0) atomicAdd(job.fallbacks, __popc(mask));
    }
}

template <int NT, int KC>
int launch_tiles_t(const ConvJob *d_jobs, int grid, int R_max, const int4 *items, const int *count, hipStream_t s) {
    const int HW = kTile + 2 * R_max;
    const size_t lds = static_cast<size_t>(HW) * HW * KC * sizeof(double);
    if (lds > 65536)
        SE2_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_lse_tiles<NT, KC>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    return launch_kernel(&k_lse_tiles<NT, KC>, dim3(grid), dim3(kConvThreads), lds, s, true, d_jobs, items, count);
}

template <int NT, int KC, bool F64EXP>
int launch_dense_t(const ConvJob *d_jobs, int nblocks, const int32_t *d_block_job, int R_max, hipStream_t s) {
    const int HW = kTile + 2 * R_max;
    size_t lds = static_cast<size_t>(HW) * HW * KC * sizeof(double);
    if (lds < kConvThreads * sizeof(double)) lds = kConvThreads * sizeof(double);
    if (lds > 65536)
        SE2_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_conv_lse<NT, KC, F64EXP>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    return launch_kernel(&k_conv_lse<NT, KC, F64EXP>, dim3(nblocks), dim3(kConvThreads), lds, s, true, d_jobs,
                         d_block_job);
}

template <int NT, int RBW>
int launch_rebuild_t(const ConvJob *d_jobs, int nblocks, int R_max, const int2 *rebuild, const int *rebuild_count,
                     int *published, hipStream_t s) {
    const int HW = kTile + 2 * R_max, W = 2 * R_max + 1;
    const size_t lr = static_cast<size_t>(HW) * HW * NT * sizeof(double) +
                      (static_cast<size_t>(W) * W + kListMax) * sizeof(uint32_t);
    if (lr > 65536)
        SE2_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rebuild<NT, RBW>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lr)));
    const int cap = (RBW == 16) ? kRebuildGridWide : kRebuildGrid;
    const int grid = nblocks * NT < cap ? nblocks * NT : cap;
    return launch_kernel(&k_rebuild<NT, RBW>, dim3(grid), dim3(64 * RBW), lr, s, true, d_jobs, rebuild,
                         rebuild_count, published);
}

template <int NT>
int launch_sparse_t(const ConvJob *d_jobs, int nblocks, const int32_t *d_block_job, int R_max, int2 *rebuild,
                    int *rebuild_count, int *next_count, int rb_waves, int *published, hipStream_t s) {
    constexpr int NW = NT < 16 ? NT : 16;
    const int HW = kTile + 2 * R_max;
    const size_t lds = static_cast<size_t>(HW) * HW * NT * sizeof(double);
    if (lds > 65536)
        SE2_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sparse<NT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    const int rc = launch_kernel(&k_sparse<NT>, dim3(xcd_grid(nblocks)), dim3(64 * NW), lds, s, false, d_jobs,
                                 d_block_job, nblocks, rebuild, rebuild_count, next_count);
    if (rc) return rc;
    return rb_waves == 16 ? launch_rebuild_t<NT, 16>(d_jobs, nblocks, R_max, rebuild, rebuild_count, published, s)
                          : launch_rebuild_t<NT, 8>(d_jobs, nblocks, R_max, rebuild, rebuild_count, published, s);
}

// Plan statistics of pi(x, y) = 2^(phi2(x) + L2[x - y] + psi2(y)), the transport plan of the
// scalings (Section 4.1), for the transport cost sum pi rho_b^2 and the plan mass sum pi
// (Section 2.2).  Workgroup (tile, g) of plan j = blockIdx.y covers the outputs x of one 8 x 8
// tile at the 4 NQ orientations ko = 4 NQ g + wave + 4 q (lane = pixel, q < NQ) and their
// windows; the psi halo is staged in LDS KC orientations at a time, kernel and cost values are
// wave-uniform (scalar loads).  After an a-update the rows of pi sum to the first marginal, so
// every term is at most 1 and 2^u needs no shift.  Sums: FP32 over the KC orientations of one
// window offset, FP64 over the offsets, then over q, lanes (butterflies) and the four waves in
// order.  Partial b of plan j goes to part[2 b], part[2 b + 1] (one plan, interleaved) or
// part[2 j nb + b], part[(2 j + 1) nb + b] (plan tables, planar), nb = gridDim.x.
template <int NT, int KC, int NQ>
__global__ __launch_bounds__(kConvThreads) void k_plan_tiles(const double *__restrict__ phi1,
                                                             const double *__restrict__ psi1,
                                                             const double *const *__restrict__ phi_tab,
                                                             const double *const *__restrict__ psi_tab,
                                                             const double *__restrict__ L64_,
                                                             const float *__restrict__ cost_, int nx, int ny, int R,
                                                             int tiles_x, double *__restrict__ part) {
    extern __shared__ double lds[];
    __shared__ double s_sum[8];
    constexpr int NG = NT / (4 * NQ);
    const int j = blockIdx.y;
    const double *phi = phi_tab != nullptr ? phi_tab[j] : phi1;
    const double *psi = psi_tab != nullptr ? psi_tab[j] : psi1;
    const int tile = static_cast<int>(blockIdx.x) / NG;
    const int g = static_cast<int>(blockIdx.x) - tile * NG;
    const int ty = tile / tiles_x;
    const int tx = tile - ty * tiles_x;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int px = lane & 7, py = lane >> 3;
    const int gx = x0 + px, gy = y0 + py;
    const bool valid = gx < nx && gy < ny;
    double f[NQ];
    bool any = false;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int ko = 4 * NQ * g + wave + 4 * q;
        f[q] = valid ? phi[(static_cast<size_t>(gy) * nx + gx) * NT + ko] : -INFINITY;
        any = any || f[q] != -INFINITY;
    }
    const int W = 2 * R + 1, HW = kTile + 2 * R, npix = HW * HW;
    const cdptr L64 = (cdptr)L64_;
    const cfptr cost = (cfptr)cost_;
    double c[NQ], m[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) c[q] = m[q] = 0.0;
    for (int k0 = 0; k0 < NT; k0 += KC) {
        if (k0 > 0) __syncthreads();
        load_halo<KC>(lds, psi, NT, k0, x0, y0, R, HW, nx, ny);
        __syncthreads();
        if (!any) continue;
        for (int dy = -R; dy <= R; ++dy) {
            for (int dx = -R; dx <= R; ++dx) {
                const int hb = (py + R - dy) * HW + (px + R - dx);
                const size_t row = (static_cast<size_t>((dy + R) * W + (dx + R)) * NT + 4 * NQ * g + wave) * NT + k0;
                float rs[NQ], rc[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) rs[q] = rc[q] = 0.0f;
#pragma unroll
                for (int kc = 0; kc < KC; ++kc) {
                    const double v = lds[kc * npix + hb];
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        const size_t e = row + static_cast<size_t>(4 * q) * NT + kc;
                        const float p = __builtin_amdgcn_exp2f(static_cast<float>((f[q] + L64[e]) + v));
                        rs[q] += p;
                        rc[q] += p * cost[e];
                    }
                }
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    m[q] += static_cast<double>(rs[q]);
                    c[q] += static_cast<double>(rc[q]);
                }
            }
        }
    }
    double ct = 0.0, mt = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        ct += c[q];
        mt += m[q];
    }
    ct = block_sum_waves(ct, s_sum);
    mt = block_sum_waves(mt, s_sum + 4);
    if (threadIdx.x == 0) {
        const size_t nb = gridDim.x;
        if (phi_tab != nullptr) {
            part[(2 * static_cast<size_t>(j)) * nb + blockIdx.x] = ct;
            part[(2 * static_cast<size_t>(j) + 1) * nb + blockIdx.x] = mt;
        } else {
            part[2 * static_cast<size_t>(blockIdx.x)] = ct;
            part[2 * static_cast<size_t>(blockIdx.x) + 1] = mt;
        }
    }
}

// Orientations per lane of the plan statistics: four on grids whose one-per-lane launch would
// already have 4096 workgroups per plan or more (the halo is then staged once per 16
// orientations instead of once per 4, and a lane carries four independent sums), else one (a
// small grid needs the workgroups to fill the compute units).
int plan_nq(const Kernel &k) {
    const int tiles = ((k.grid.nx + kTile - 1) / kTile) * ((k.grid.ny + kTile - 1) / kTile);
    const int nt = k.grid.ntheta;
    return (tiles * (nt / 4) >= 4096 && nt >= 16) ? 4 : 1;
}

template <int NT, int KC, int NQ>
int launch_plan_t(const Kernel &k, const double *phi, const double *psi, const double *const *phi_tab,
                  const double *const *psi_tab, int nplans, double *part, hipStream_t s) {
    const int R = k.metric.radius, HW = kTile + 2 * R;
    const size_t lds = static_cast<size_t>(HW) * HW * KC * sizeof(double);
    if (lds > 65536)
        SE2_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_plan_tiles<NT, KC, NQ>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    const int tx = (k.grid.nx + kTile - 1) / kTile, ty = (k.grid.ny + kTile - 1) / kTile;
    hipLaunchKernelGGL((k_plan_tiles<NT, KC, NQ>), dim3(tx * ty * (NT / (4 * NQ)), nplans), dim3(kConvThreads), lds,
                       s, phi, psi, phi_tab, psi_tab, k.d_L64, k.d_cost32, k.grid.nx, k.grid.ny, R, tx, part);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

template <int NT, int KC>
int launch_plan_nq(const Kernel &k, const double *phi, const double *psi, const double *const *phi_tab,
                   const double *const *psi_tab, int nplans, double *part, hipStream_t s) {
    if constexpr (NT >= 16) {
        if (plan_nq(k) == 4) return launch_plan_t<NT, KC, 4>(k, phi, psi, phi_tab, psi_tab, nplans, part, s);
    }
    return launch_plan_t<NT, KC, 1>(k, phi, psi, phi_tab, psi_tab, nplans, part, s);
}

}  // namespace

int launch_lse_tiles(const ConvJob *d_jobs, int grid, int nt, int R_max, const int4 *items, const int *count,
                     hipStream_t s) {
    if (grid <= 0) return SE2_OK;
    if (R_max < 0 || R_max > kMaxRadius || !items || !count) return SE2_EINVAL;
    // the largest chunk of input orientations whose FP64 halo fits in 64 KiB (as k_conv_lse)
    const bool kc16 = (kTile + 2 * R_max) * (kTile + 2 * R_max) * 16 * 8 <= 65536;
    switch (nt) {
        case 8: return launch_tiles_t<8, 8>(d_jobs, grid, R_max, items, count, s);
        case 16:
            return kc16 ? launch_tiles_t<16, 16>(d_jobs, grid, R_max, items, count, s)
                        : launch_tiles_t<16, 8>(d_jobs, grid, R_max, items, count, s);
        case 32:
            return kc16 ? launch_tiles_t<32, 16>(d_jobs, grid, R_max, items, count, s)
                        : launch_tiles_t<32, 8>(d_jobs, grid, R_max, items, count, s);
        default: return SE2_EINVAL;
    }
}

int plan_parts(const Kernel &k) {
    const int tx = (k.grid.nx + kTile - 1) / kTile, ty = (k.grid.ny + kTile - 1) / kTile;
    return tx * ty * (k.grid.ntheta / (4 * plan_nq(k)));
}

int launch_plan_tiles(const Kernel &k, const double *phi, const double *psi, const double *const *phi_tab,
                      const double *const *psi_tab, int nplans, double *part, hipStream_t s) {
    if (nplans < 1) return SE2_OK;
    const int R = k.metric.radius;
    if (R < 0 || R > kMaxRadius || !part || (phi_tab == nullptr) != (psi_tab == nullptr) ||
        (phi_tab == nullptr && (!phi || !psi || nplans != 1)))
        return SE2_EINVAL;
    const bool kc16 = (kTile + 2 * R) * (kTile + 2 * R) * 16 * 8 <= 65536;
    switch (k.grid.ntheta) {
        case 8: return launch_plan_nq<8, 8>(k, phi, psi, phi_tab, psi_tab, nplans, part, s);
        case 16:
            return kc16 ? launch_plan_nq<16, 16>(k, phi, psi, phi_tab, psi_tab, nplans, part, s)
                        : launch_plan_nq<16, 8>(k, phi, psi, phi_tab, psi_tab, nplans, part, s);
        case 32:
            return kc16 ? launch_plan_nq<32, 16>(k, phi, psi, phi_tab, psi_tab, nplans, part, s)
                        : launch_plan_nq<32, 8>(k, phi, psi, phi_tab, psi_tab, nplans, part, s);
        default: return SE2_EINVAL;
    }
}

bool conv_lse_sparse_fits(int nt, int R) {
    const int HW = kTile + 2 * R;
    return static_cast<size_t>(HW) * HW * nt * sizeof(double) <= kSparseLdsMax;
}

int launch_conv_lse(const ConvJob *d_jobs, int njobs, int nblocks, const int32_t *d_block_job, int nt, int R_max,
                    bool f64exp, bool sparse, int2 *rebuild, int *rebuild_count, int *next_count, int rb_waves,
                    int *published, hipStream_t s) {
    (void)njobs;
    if (nblocks <= 0) return SE2_OK;
    if (R_max < 0 || R_max > kMaxRadius) return SE2_EINVAL;
    const int HW = kTile + 2 * R_max;
    if (sparse) {
        // every job of a sparse launch carries lists (the engine groups them apart)
        if (f64exp || !conv_lse_sparse_fits(nt, R_max) || !rebuild || !rebuild_count || !next_count ||
            rebuild_count == next_count || (rb_waves != 8 && rb_waves != 16))
            return SE2_EINVAL;
        switch (nt) {
            case 8:
                return launch_sparse_t<8>(d_jobs, nblocks, d_block_job, R_max, rebuild, rebuild_count, next_count,
                                             rb_waves, published, s);
            case 16:
                return launch_sparse_t<16>(d_jobs, nblocks, d_block_job, R_max, rebuild, rebuild_count, next_count,
                                             rb_waves, published, s);
            case 32:
                return launch_sparse_t<32>(d_jobs, nblocks, d_block_job, R_max, rebuild, rebuild_count, next_count,
                                             rb_waves, published, s);
            default: return SE2_EINVAL;
        }
    }
    const bool kc16 = HW * HW * 16 * 8 <= 65536;
    switch (nt) {
        case 8:
            return f64exp ? launch_dense_t<8, 8, true>(d_jobs, nblocks, d_block_job, R_max, s)
                          : launch_dense_t<8, 8, false>(d_jobs, nblocks, d_block_job, R_max, s);
        case 16:
            if (kc16)
                return f64exp ? launch_dense_t<16, 16, true>(d_jobs, nblocks, d_block_job, R_max, s)
                              : launch_dense_t<16, 16, false>(d_jobs, nblocks, d_block_job, R_max, s);
            return f64exp ? launch_dense_t<16, 8, true>(d_jobs, nblocks, d_block_job, R_max, s)
                          : launch_dense_t<16, 8, false>(d_jobs, nblocks, d_block_job, R_max, s);
        case 32:
            if (kc16)
                return f64exp ? launch_dense_t<32, 16, true>(d_jobs, nblocks, d_block_job, R_max, s)
                              : launch_dense_t<32, 16, false>(d_jobs, nblocks, d_block_job, R_max, s);
            return f64exp ? launch_dense_t<32, 8, true>(d_jobs, nblocks, d_block_job, R_max, s)
                          : launch_dense_t<32, 8, false>(d_jobs, nblocks, d_block_job, R_max, s);
        default:
            return SE2_EINVAL;
    }
}

}  // namespace se2
