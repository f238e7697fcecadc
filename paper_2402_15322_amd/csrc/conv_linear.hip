// Linear SE(2) group convolution out = K * in (Section 4.2) on gfx950.
//
//   BF16: implicit GEMM on the matrix cores.  For a fixed window row dy and a group
//         of window columns, the contraction over (dx, ki) is a 16 x 32 by 32 x 16
//         product: rows = 16 output pixels of one image row, columns = 16 output
//         orientations ko, K-dimension = (dx slot, ki); one
//         v_mfma_f32_16x16x32_bf16 each, FP32 accumulation over the whole window.
//         Reuse: a wave owns 8 (or 4) output rows and holds the kernel fragments of
//         up to 8 window rows in registers, so every input-row fragment read from
//         LDS feeds up to 8 MFMAs (output row oy and window row dy meet input row
//         oy - dy).
//         The input halo tile is rounded to bfloat16 (RNE) once while it is staged
//         in LDS; kernel fragments are pre-packed on the host in operand order (one
//         coalesced 16-byte load per lane) and zero-padded where a dx group
//         overhangs the window or a dy chunk runs past it.
//   F32, nt = 16 and 32: the same implicit GEMM on the FP32 matrix cores
//         (v_mfma_f32_16x16x4f32): per window offset (dy, dx) and 16 input orientations,
//         four 16 x 4 by 4 x 16 products per block of 16 output orientations; a lane's
//         four A operands are the four orientations it reads with one 16-byte LDS load,
//         and the B operand is packed on the host to match.  The halo is staged in FP32,
//         unrounded, 16 input orientations at a time.
//   F32 (nt = 8) / F64: an 8 x 8 tile per workgroup on the vector ALUs with FP32 / FP64
//         FMAs.
#include <hip/hip_runtime.h>

#include <cstring>

#include "conv_dev.h"
#include "se2_internal.h"
#include "launch.h"

namespace se2 {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

namespace {

constexpr int kSeg = 16;   // output pixels per MFMA row block
constexpr int kWaves = 4;  // a workgroup is kWaves * RPW output rows of kSeg pixels
constexpr int kNumCUs = 256;  // compute units of an MI355X
constexpr int kDYCMax = 8;  // most window rows whose kernel fragments a wave holds at once

// dy chunking of a window of W rows: the fewest chunks of at most kDYCMax rows, all of
// one size DYC >= 4 (rows past the window are zero fragments).
__host__ __device__ constexpr int dy_chunk(int W) {
    const int n = (W + kDYCMax - 1) / kDYCMax;
    const int d = (W + n - 1) / n;
    return d < 4 ? 4 : d;
}

__device__ __forceinline__ uint32_t f32x2_to_bf16x2_rne(float lo, float hi) {
    uint32_t a = __float_as_uint(lo), b = __float_as_uint(hi);
    a += 0x7fffu + ((a >> 16) & 1u);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (a >> 16) | (b & 0xffff0000u);
}

// Geometry of the packing: SPM dx slots per MFMA K-dimension, NB column blocks of 16 ko.
template <int NT>
struct Pack {
    static constexpr int SPM = (NT >= 32) ? 1 : 32 / NT;  // 8 -> 4, 16 -> 2, 32 -> 1
    static constexpr int KI = 32 / SPM;                   // ki per slot (== NT for NT <= 32)
    static constexpr int NB = (NT > 16) ? NT / 16 : 1;
};

// MFMAs of one dy chunk for one dx group: t runs over the input rows that the wave's
// output rows meet with the chunk's window rows; (r, c) with r - c = t - (DYC - 1) is
// output row r and window row dy0 + c.  Rows past the window carry zero fragments; the
// input row is clamped into the halo for them (the product is then 0).
template <int NT, int DYC, int RPW>
__device__ __forceinline__ void mfma_chunk(f32x4_t (&acc)[RPW][Pack<NT>::NB],
                                           const bf16x8_t (&bfr)[DYC][Pack<NT>::NB], const uint16_t *lds16,
                                           int hrow_t0, int HWX, int hx, int kio) {
    using P = Pack<NT>;
    constexpr int T = RPW + DYC - 1;
    const uint16_t *base = lds16 + hx * NT + kio;
    const int rstride = HWX * NT;
    auto read_a = [&](int t) {
        return *reinterpret_cast<const bf16x8_t *>(base + max(hrow_t0 + t, 0) * rstride);
    };
    // the read of input row t+1 is issued before the MFMAs of row t
    bf16x8_t a = read_a(0);
#pragma unroll
    for (int t = 0; t < T; ++t) {
        bf16x8_t an = a;
        if (t + 1 < T) an = read_a(t + 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int c = r - t + DYC - 1;
            if (c < 0 || c >= DYC) continue;
#pragma unroll
            for (int nb = 0; nb < P::NB; ++nb)
                acc[r][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bfr[c][nb], acc[r][nb], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
        a = an;
    }
}

// Kernel fragments of step `step` ((dx group, dy chunk) = (step / nchunks, step % nchunks))
// of the BF16 contraction, one 16-byte load per lane and fragment.
template <int NT, int DYC>
__device__ __forceinline__ void bf16_load_b(bf16x8_t (&dstb)[DYC][Pack<NT>::NB], const bf16x8_t *__restrict__ Bp,
                                            int step, int R, int lane) {
    using P = Pack<NT>;
    const int W = 2 * R + 1;
    const int G = (W + P::SPM - 1) / P::SPM;
    const int nchunks = (W + DYC - 1) / DYC;
    const int g = step / nchunks, ch = step - g * nchunks;
    const bf16x8_t *src = Bp + (static_cast<size_t>(ch * DYC) * G + g) * P::NB * 64 + lane;
#pragma unroll
    for (int c = 0; c < DYC; ++c)
#pragma unroll
        for (int nb = 0; nb < P::NB; ++nb) dstb[c][nb] = src[(static_cast<size_t>(c) * G * P::NB + nb) * 64];
}

// The first two fragment sets of the contraction (steps 0 and 1, or 0 twice when there is
// one step), requested by the caller right before bf16_contract.  (Requesting them before
// the halo staging gains nothing: the staging loop waits for every load in flight.)
template <int NT, int DYC>
__device__ __forceinline__ void bf16_first_b(bf16x8_t (&b0)[DYC][Pack<NT>::NB], bf16x8_t (&b1)[DYC][Pack<NT>::NB],
                                             const bf16x8_t *__restrict__ Bp, int R, int lane) {
    using P = Pack<NT>;
    const int W = 2 * R + 1;
    const int nsteps = ((W + P::SPM - 1) / P::SPM) * ((W + DYC - 1) / DYC);
    bf16_load_b<NT, DYC>(b0, Bp, 0, R, lane);
    bf16_load_b<NT, DYC>(b1, Bp, min(1, nsteps - 1), R, lane);
}

// All (dx group, dy chunk) steps of the BF16 contraction of one workgroup tile: acc[r][nb]
// receives output row row0 + r of the tile, column block nb.  lds16 holds the halo
// [hy][hx][ki] in bfloat16 with hx = 0 at pixel xl; b0 and b1 hold the fragments of the
// first two steps (bf16_first_b) and are used as buffers afterwards.
template <int NT, int DYC, int RPW>
__device__ __forceinline__ void bf16_contract(f32x4_t (&acc)[RPW][Pack<NT>::NB], const uint16_t *lds16,
                                              const bf16x8_t *__restrict__ Bp, int R, int x0, int xl, int row0,
                                              int lane, bf16x8_t (&b0)[DYC][Pack<NT>::NB],
                                              bf16x8_t (&b1)[DYC][Pack<NT>::NB]) {
    using P = Pack<NT>;
    const int W = 2 * R + 1;
    const int G = (W + P::SPM - 1) / P::SPM;
    const int HWX = kSeg + 2 * R + (G * P::SPM - W);
    const int i = lane & 15;   // output pixel within the segment (A row)
    const int kb = lane >> 4;  // 8-wide K block of this lane
    const int slot = (kb * 8) / P::KI;
    const int kio = (kb * 8) % P::KI;

#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int nb = 0; nb < P::NB; ++nb) acc[r][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    // (g, chunk) steps; the kernel fragments of the next step are loaded while the
    // current one runs on the matrix cores
    const int nchunks = (W + DYC - 1) / DYC;
    const int nsteps = G * nchunks;
    auto load_b = [&](bf16x8_t(&dstb)[DYC][P::NB], int step) { bf16_load_b<NT, DYC>(dstb, Bp, step, R, lane); };
    auto run = [&](const bf16x8_t(&bfr)[DYC][P::NB], int step) {
        const int g = step / nchunks, ch = step - g * nchunks;
        // this lane's dx: slots of group g run dx = -R + g*SPM + slot; input pixel
        // x0 + i - dx sits at halo column (x0 + i - dx) - xl
        const int hx = x0 + i - (-R + g * P::SPM + slot) - xl;
        const int dy0 = -R + ch * DYC;
        // halo row of (r, c): row0 + r - (dy0 + c) + R = hrow_t0 + t
        mfma_chunk<NT, DYC, RPW>(acc, bfr, lds16, row0 + R - dy0 - (DYC - 1), HWX, hx, kio);
    };
    if constexpr (P::NB == 1) {
        // three fragment buffers in rotation: the fragments of step s + 2 are requested while
        // step s runs (a step is ~24 MFMAs per wave at two waves per SIMD, about one L2
        // round trip), and no buffer is copied, so no wait falls on a load still in flight.
        // Prefetch indices are clamped (the last steps reload fragments they do not use) so
        // that the loads' wait counts stay exact; the last nsteps % 3 steps run after the loop.
        bf16x8_t b2[DYC][P::NB];
        int step = 0;
        for (; step + 3 <= nsteps; step += 3) {
            load_b(b2, min(step + 2, nsteps - 1));
            __builtin_amdgcn_sched_barrier(0);
            run(b0, step);
            __builtin_amdgcn_sched_barrier(0);
            load_b(b0, min(step + 3, nsteps - 1));
            __builtin_amdgcn_sched_barrier(0);
            run(b1, step + 1);
            __builtin_amdgcn_sched_barrier(0);
            load_b(b1, min(step + 4, nsteps - 1));
            __builtin_amdgcn_sched_barrier(0);
            run(b2, step + 2);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (step < nsteps) run(b0, step);
        if (step + 1 < nsteps) run(b1, step + 1);
    } else {
        // two column blocks (nt = 32): the fragments of the next step are loaded while the
        // current one runs (a third buffer would not fit the registers); the prefetch index is
        // clamped (the last step reloads its own fragments) so the loop body has no branch.
        // b1 already holds step 1 (or step 0 again): it is overwritten before its first use.
        for (int step = 0; step < nsteps; ++step) {
            load_b(b1, min(step + 1, nsteps - 1));
            __builtin_amdgcn_sched_barrier(0);
            run(b0, step);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = 0; c < DYC; ++c)
#pragma unroll
                for (int nb = 0; nb < P::NB; ++nb) b0[c][nb] = b1[c][nb];
        }
    }
}

template <int NT, int DYC, int RPW>
__global__ __launch_bounds__(256) void k_conv_bf16(const float *__restrict__ in, float *__restrict__ out,
                                                   const bf16x8_t *__restrict__ Bp, int nx, int ny, int R,
                                                   int tiles_x, int tiles_y) {
    using P = Pack<NT>;
    extern __shared__ uint16_t lds16[];
    const int W = 2 * R + 1;
    const int G = (W + P::SPM - 1) / P::SPM;
    const int HWX = kSeg + 2 * R + (G * P::SPM - W);  // halo width incl. overhang of the last dx group
    constexpr int kRows = RPW * kWaves;
    const int HWY = kRows + 2 * R;
    const int tiles = tiles_x * tiles_y;
    const int b = blockIdx.x / tiles;
    const int t = blockIdx.x - b * tiles;
    const int ty = t / tiles_x, tx = t - ty * tiles_x;
    const int x0 = tx * kSeg, y0 = ty * kRows;
    const float *img = in + static_cast<size_t>(b) * nx * ny * NT;
    float *dst = out + static_cast<size_t>(b) * nx * ny * NT;

    // stage halo [hy][hx][ki] as bfloat16, four orientations per thread and element;
    // hx = 0 is pixel x0 - R - (overhang).  Loads go out in batches of 8 per thread
    // (clamped indices, no branches) before any of them is converted and stored.
    const int xl = x0 - R - (G * P::SPM - W);
    {
        constexpr int Q = NT / 4;
        constexpr int NB8 = 8;
        const int total = HWY * HWX * Q;
        const float inv = 1.0f / static_cast<float>(HWX);
        for (int e0 = 0; e0 < total; e0 += NB8 * 256) {
            float4 v[NB8];
            bool ok[NB8];
#pragma unroll
            for (int u = 0; u < NB8; ++u) {
                const int e = min(e0 + u * 256 + static_cast<int>(threadIdx.x), total - 1);
                const int p = e / Q, q = e - p * Q;
                // p / HWX through a float reciprocal: exact for p < 2^20 (the +0.5 keeps
                // the rounding error far from an integer boundary)
                const int hy = static_cast<int>((static_cast<float>(p) + 0.5f) * inv), hx = p - hy * HWX;
                const int gy = y0 - R + hy, gx = xl + hx;
                ok[u] = gy >= 0 && gy < ny && gx >= 0 && gx < nx;
                const int cy = min(max(gy, 0), ny - 1), cx = min(max(gx, 0), nx - 1);
                v[u] = *reinterpret_cast<const float4 *>(&img[(static_cast<size_t>(cy) * nx + cx) * NT + 4 * q]);
            }
#pragma unroll
            for (int u = 0; u < NB8; ++u) {
                const int e = e0 + u * 256 + static_cast<int>(threadIdx.x);
                if (e < total)
                    *reinterpret_cast<uint2 *>(&lds16[4 * e]) =
                        ok[u] ? make_uint2(f32x2_to_bf16x2_rne(v[u].x, v[u].y), f32x2_to_bf16x2_rne(v[u].z, v[u].w))
                              : make_uint2(0u, 0u);
            }
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int row0 = wave * RPW;  // first output row of this wave within the tile
    f32x4_t acc[RPW][P::NB];
    bf16x8_t b0[DYC][P::NB], b1[DYC][P::NB];
    bf16_first_b<NT, DYC>(b0, b1, Bp, R, lane);
    bf16_contract<NT, DYC, RPW>(acc, lds16, Bp, R, x0, xl, row0, lane, b0, b1);

    // D: lane holds column j = lane % 16 (ko), rows 4*(lane/16) + q (pixels)
    const int j = lane & 15;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int gy = y0 + row0 + r;
        if (gy >= ny) continue;
#pragma unroll
        for (int nb = 0; nb < P::NB; ++nb) {
            const int ko = nb * 16 + j;
            if (ko >= NT) continue;  // nt = 8: columns 8..15 are padding
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gx = x0 + 4 * (lane >> 4) + q;
                if (gx < nx) dst[(static_cast<size_t>(gy) * nx + gx) * NT + ko] = acc[r][nb][q];
            }
        }
    }
}

// FP32 matrix-core steps (nt = 16 or 32): the tiling of k_conv_bf16 (kSeg output pixels by
// kWaves * RPW output rows per workgroup, window rows in chunks of DYC), one step per (dx, dy
// chunk), in NT / 16 passes over 16 input orientations each (the halo of one pass is staged
// in LDS in FP32, [hy][hx][16 ki], hx = 0 at pixel x0 - R).  For output row r and window row c
// of the chunk, the lane of pixel i = lane % 16 and quad kq = lane / 16 reads the pass's
// input orientations 4 kq .. 4 kq + 3 of its input pixel as one float4; MFMA e (e = 0..3) of
// column block nb multiplies element e by the packed B value
// K[ko = 16 nb + lane % 16][ki = 16 pass + 4 kq + e], so the four MFMAs sum the pass's 16
// orientations into the 16 output orientations of the block.
template <int NT, int DYC>
__device__ __forceinline__ void f32m_load_b(f32x4_t (&dstb)[DYC][NT / 16], const f32x4_t *__restrict__ Fp, int step,
                                            int pass, int nchunks, int W, int lane) {
    constexpr int NB = NT / 16, NP = NT / 16;
    const int dxi = step / nchunks, ch = step - dxi * nchunks;
#pragma unroll
    for (int c = 0; c < DYC; ++c)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
            dstb[c][nb] = Fp[((((static_cast<size_t>(ch * DYC + c) * W + dxi) * NP + pass) * NB + nb) * 64) + lane];
}

// Every step of one pass, with the first step's fragments already in b0.  With FLUSH the
// FP32 accumulators are added into FP64 ones after every step and cleared, so that no FP32
// sum runs over more than one step (16 DYC products).  With SCALE, fragment element e of
// column block nb is multiplied by 2^kx[nb][e] (exact: an exponent change) before it is used.
template <int NT, int DYC, int RPW, bool FLUSH, bool SCALE = false>
__device__ __forceinline__ void f32m_steps(f32x4_t (&acc)[RPW][NT / 16], double (&acc64)[RPW][NT / 16][4],
                                           f32x4_t (&b0)[DYC][NT / 16], const float *lds32,
                                           const f32x4_t *__restrict__ Fp, int pass, int R, int row0, int lane,
                                           const int (*kx)[4] = nullptr) {
    constexpr int NB = NT / 16;
    const int W = 2 * R + 1;
    const int HWX = kSeg + 2 * R;
    const int i = lane & 15;   // output pixel within the segment (A row)
    const int kq = lane >> 4;  // orientation quad of this lane
    const int nchunks = (W + DYC - 1) / DYC;
    const int nsteps = W * nchunks;
    f32x4_t b1[DYC][NB];
    auto run = [&](const f32x4_t(&bfr)[DYC][NB], int step) {
        const int dxi = step / nchunks, ch = step - dxi * nchunks;
        // input pixel x0 + i - dx (dx = dxi - R) sits at halo column i + 2R - dxi; output
        // row r and window row c = r - t + DYC - 1 of the chunk meet halo row hrow0 + t
        // (rows past the window carry zero fragments; their row index is clamped)
        const float *base = lds32 + (i + 2 * R - dxi) * 16 + 4 * kq;
        const int rstride = HWX * 16;
        const int hrow0 = row0 + 2 * R - ch * DYC - (DYC - 1);
        constexpr int T = RPW + DYC - 1;
        auto read_a = [&](int tt) { return *reinterpret_cast<const f32x4_t *>(base + max(hrow0 + tt, 0) * rstride); };
        f32x4_t a = read_a(0);
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            f32x4_t an = a;
            if (tt + 1 < T) an = read_a(tt + 1);
            __builtin_amdgcn_sched_barrier(0);
            // e outermost: consecutive MFMAs update different accumulators
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    const int c = r - tt + DYC - 1;
                    if (c < 0 || c >= DYC) continue;
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[r][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], bfr[c][nb][e], acc[r][nb], 0, 0, 0);
                }
            __builtin_amdgcn_sched_barrier(0);
            a = an;
        }
    };
    // a step is RPW * DYC * 4 * NB MFMAs of 32 cycles per wave: one step of lookahead
    // hides the fragment loads
    for (int step = 0; step < nsteps; ++step) {
        if constexpr (SCALE) {
            // b0 was requested a step ago: scale it now, before the next request goes out
#pragma unroll
            for (int c = 0; c < DYC; ++c)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int e = 0; e < 4; ++e) b0[c][nb][e] = __builtin_amdgcn_ldexpf(b0[c][nb][e], kx[nb][e]);
        }
        f32m_load_b<NT, DYC>(b1, Fp, min(step + 1, nsteps - 1), pass, nchunks, W, lane);
        __builtin_amdgcn_sched_barrier(0);
        run(b0, step);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (FLUSH) {
#pragma unroll
            for (int r = 0; r < RPW; ++r)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc64[r][nb][q] += static_cast<double>(acc[r][nb][q]);
                    acc[r][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
                }
        }
#pragma unroll
        for (int c = 0; c < DYC; ++c)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) b0[c][nb] = b1[c][nb];
    }
}

// FP32 convolution on the matrix cores, nt = 16 or 32 (steps above).
template <int NT, int DYC, int RPW>
__global__ __launch_bounds__(256) void k_conv_f32m(const float *__restrict__ in, float *__restrict__ out,
                                                   const f32x4_t *__restrict__ Fp, int nx, int ny, int R,
                                                   int tiles_x, int tiles_y) {
    static_assert(NT == 16 || NT == 32, "16 or 32 orientations");
    constexpr int NB = NT / 16;  // output column blocks
    constexpr int NP = NT / 16;  // passes over the input orientations
    extern __shared__ float lds32[];
    const int W = 2 * R + 1;
    const int HWX = kSeg + 2 * R;
    constexpr int kRows = RPW * kWaves;
    const int HWY = kRows + 2 * R;
    const int tiles = tiles_x * tiles_y;
    const int b = blockIdx.x / tiles;
    const int t = blockIdx.x - b * tiles;
    const int ty = t / tiles_x, tx = t - ty * tiles_x;
    const int x0 = tx * kSeg, y0 = ty * kRows;
    const float *img = in + static_cast<size_t>(b) * nx * ny * NT;
    float *dst = out + static_cast<size_t>(b) * nx * ny * NT;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int row0 = wave * RPW;  // first output row of this wave within the tile

    f32x4_t acc[RPW][NB];
    double unused[RPW][NB][4];
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[r][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    const int nchunks = (W + DYC - 1) / DYC;
    f32x4_t b0[DYC][NB];
    const int xl = x0 - R;
    for (int pass = 0; pass < NP; ++pass) {
        // the fragments of a pass's first step are loaded before its halo staging, so that
        // their latency overlaps it
        f32m_load_b<NT, DYC>(b0, Fp, 0, pass, nchunks, W, lane);
        if (pass > 0) __syncthreads();  // every wave is done with the previous pass's halo
        // stage the pass's halo [hy][hx][16 ki] in FP32, zero outside the grid; loads go
        // out in batches of 8 float4 per thread (clamped indices, no branches) before any
        // is stored
        {
            constexpr int Q = 4;
            constexpr int NB8 = 8;
            const int total = HWY * HWX * Q;
            const float inv = 1.0f / static_cast<float>(HWX);
            for (int e0 = 0; e0 < total; e0 += NB8 * 256) {
                float4 v[NB8];
                bool ok[NB8];
#pragma unroll
                for (int u = 0; u < NB8; ++u) {
                    const int e = min(e0 + u * 256 + static_cast<int>(threadIdx.x), total - 1);
                    const int p = e / Q, q = e - p * Q;
                    // p / HWX through a float reciprocal: exact for p < 2^20
                    const int hy = static_cast<int>((static_cast<float>(p) + 0.5f) * inv), hx = p - hy * HWX;
                    const int gy = y0 - R + hy, gx = xl + hx;
                    ok[u] = gy >= 0 && gy < ny && gx >= 0 && gx < nx;
                    const int cy = min(max(gy, 0), ny - 1), cx = min(max(gx, 0), nx - 1);
                    v[u] = *reinterpret_cast<const float4 *>(
                        &img[(static_cast<size_t>(cy) * nx + cx) * NT + 16 * pass + 4 * q]);
                }
#pragma unroll
                for (int u = 0; u < NB8; ++u) {
                    const int e = e0 + u * 256 + static_cast<int>(threadIdx.x);
                    if (e < total)
                        *reinterpret_cast<float4 *>(&lds32[4 * e]) = ok[u] ? v[u] : make_float4(0.f, 0.f, 0.f, 0.f);
                }
            }
        }
        __syncthreads();
        f32m_steps<NT, DYC, RPW, false>(acc, unused, b0, lds32, Fp, pass, R, row0, lane);
    }

    // D: lane holds column j = lane % 16 (ko within the block), rows 4 * (lane / 16) + q
    const int j = lane & 15;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int gy = y0 + row0 + r;
        if (gy >= ny) continue;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gx = x0 + 4 * (lane >> 4) + q;
                if (gx < nx) dst[(static_cast<size_t>(gy) * nx + gx) * NT + 16 * nb + j] = acc[r][nb][q];
            }
    }
}

// Vector-ALU linear convolution (FP32 or FP64): one 8 x 8 tile per workgroup,
// lane = pixel, wave w owns ko = w, w+4, ...; the halo of KC input orientations
// at a time is staged in LDS theta-major.
template <typename T, int NT, int KC>
__global__ __launch_bounds__(256) void k_conv_valu(const T *__restrict__ in, T *__restrict__ out,
                                                   const T *__restrict__ K, int nx, int ny, int R, int tiles_x,
                                                   int tiles_y) {
    extern __shared__ unsigned char lds_raw[];
    T *lds = reinterpret_cast<T *>(lds_raw);
    constexpr int NJ = NT / 4;
    const int W = 2 * R + 1, HW = kTile + 2 * R, npix = HW * HW;
    const int tiles = tiles_x * tiles_y;
    const int b = blockIdx.x / tiles;
    const int t = blockIdx.x - b * tiles;
    const int ty = t / tiles_x, tx = t - ty * tiles_x;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const T *img = in + static_cast<size_t>(b) * nx * ny * NT;
    T *dst = out + static_cast<size_t>(b) * nx * ny * NT;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int px = lane & 7, py = lane >> 3;
    T acc[NJ];
#pragma unroll
    for (int q = 0; q < NJ; ++q) acc[q] = T(0);
    for (int k0 = 0; k0 < NT; k0 += KC) {
        if (k0 > 0) __syncthreads();
        for (int e = threadIdx.x; e < npix * KC; e += 256) {
            const int p = e / KC, k = e - p * KC;
            const int hy = p / HW, hx = p - hy * HW;
            const int gy = y0 - R + hy, gx = x0 - R + hx;
            T v = T(0);
            if (gy >= 0 && gy < ny && gx >= 0 && gx < nx) v = img[(static_cast<size_t>(gy) * nx + gx) * NT + k0 + k];
            lds[k * npix + p] = v;
        }
        __syncthreads();
        for (int dy = -R; dy <= R; ++dy)
            for (int dx = -R; dx <= R; ++dx) {
                const int hb = (py + R - dy) * HW + (px + R - dx);
                const T *Kr = K + (static_cast<size_t>((dy + R) * W + (dx + R)) * NT) * NT + k0;
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    const T v = lds[k * npix + hb];
#pragma unroll
                    for (int q = 0; q < NJ; ++q) acc[q] += Kr[(wave + 4 * q) * NT + k] * v;
                }
            }
    }
    const int gx = x0 + px, gy = y0 + py;
    if (gx < nx && gy < ny) {
#pragma unroll
        for (int q = 0; q < NJ; ++q) dst[(static_cast<size_t>(gy) * nx + gx) * NT + wave + 4 * q] = acc[q];
    }
}

// ---------------------------------------------------------------------------------------
// Certified linear-domain evaluation of log-domain jobs (the solver's matrix-core engines)
// ---------------------------------------------------------------------------------------
//
// For a job with log2 input g (FP64, -inf for zero mass) a workgroup computes, for every
// output (x, ko) of its tile, LSE(x, ko) = log2 sum_{d, ki} K[d][ko][ki] 2^g(x - d, ki) as
//     M = max of g over the tile's input halo,   V = 2^(g - M) (in (0, 1], 0 for zero mass),
//     S = sum K V on the matrix cores,           LSE = M + log2 S.
// The halo is read twice from global memory: once for M, once (from the L2) to form V,
// which is rounded to bfloat16 (RNE) or kept in FP32 as it is staged in LDS.  The
// contraction is that of the linear kernels.  The epilogue checks the certificate
// S >= kLinCert per output; a group (8 x 8 tile, ko) all of whose outputs pass is written
// with the job's scaling epilogue and error partial, slot [tile][ko]; a group with a
// failing output is written nowhere here and appended to a list that k_lse_items then
// recomputes exactly (so that in-place updates keep their previous values for it).

// Maximum of the FP64 input over the halo rows [ylo, ylo + HWY) and columns [xl, xl + HWX)
// (-inf outside the grid), over all NT orientations; the block maximum is returned to
// every thread.  16-byte loads, BATCH items of 4 orientations per thread in flight.
template <int NT>
__device__ __forceinline__ double halo_max(const double *in_, int nx, int ny, int HWX, int HWY, int xl, int ylo,
                                           double *s_m) {
    constexpr int Q = NT / 4;
    constexpr int BATCH = 4;
    const gdptr in = (gdptr)in_;
    const int total = HWY * HWX * Q;
    const float inv = 1.0f / static_cast<float>(HWX);
    double m = -INFINITY;
    for (int e0 = 0; e0 < total; e0 += BATCH * 256) {
        double v[BATCH][4];
        bool ok[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const int e = min(e0 + u * 256 + static_cast<int>(threadIdx.x), total - 1);
            const int p = e / Q, q = e - p * Q;
            const int hy = static_cast<int>((static_cast<float>(p) + 0.5f) * inv), hx = p - hy * HWX;
            const int gy = ylo + hy, gx = xl + hx;
            ok[u] = gy >= 0 && gy < ny && gx >= 0 && gx < nx;
            const int cy = min(max(gy, 0), ny - 1), cx = min(max(gx, 0), nx - 1);
            const gdptr src = in + (static_cast<size_t>(cy) * nx + cx) * NT + 4 * q;
#pragma unroll
            for (int c = 0; c < 4; ++c) v[u][c] = src[c];
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u)
            if (ok[u]) m = fmax(m, fmax(fmax(v[u][0], v[u][1]), fmax(v[u][2], v[u][3])));
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    return fmax(fmax(s_m[0], s_m[1]), fmax(s_m[2], s_m[3]));
}

// Per-orientation maxima of the FP64 input over the halo (as halo_max), written to s_out[NT]
// (-inf where an orientation has no mass in the halo); s_w holds kWaves * NT doubles.  Item
// e = 4 orientations 4q .. 4q+3 of one pixel, q = e % (NT / 4); every thread keeps one q
// (256 is a multiple of NT / 4), lanes with the same q are combined by butterflies over
// multiples of NT / 4, then the waves in LDS.
template <int NT>
__device__ __forceinline__ void halo_max_per_k(const double *in_, int nx, int ny, int HWX, int HWY, int xl, int ylo,
                                               double *s_w, double *s_out) {
    constexpr int Q = NT / 4;
    constexpr int BATCH = 4;
    const gdptr in = (gdptr)in_;
    const int total = HWY * HWX * Q;
    const float inv = 1.0f / static_cast<float>(HWX);
    double m[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int e0 = 0; e0 < total; e0 += BATCH * 256) {
        double v[BATCH][4];
        bool ok[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const int eu = e0 + u * 256 + static_cast<int>(threadIdx.x);
            const int e = min(eu, total - 1);
            const int p = e / Q, q = e - p * Q;
            const int hy = static_cast<int>((static_cast<float>(p) + 0.5f) * inv), hx = p - hy * HWX;
            const int gy = ylo + hy, gx = xl + hx;
            // a clamped item repeats the last one, whose quad may differ from this thread's
            ok[u] = eu < total && gy >= 0 && gy < ny && gx >= 0 && gx < nx;
            const int cy = min(max(gy, 0), ny - 1), cx = min(max(gx, 0), nx - 1);
            const gdptr src = in + (static_cast<size_t>(cy) * nx + cx) * NT + 4 * q;
#pragma unroll
            for (int c = 0; c < 4; ++c) v[u][c] = src[c];
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u)
            if (ok[u])
#pragma unroll
                for (int c = 0; c < 4; ++c) m[c] = fmax(m[c], v[u][c]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 4; ++c)
        for (int off = 32; off >= Q; off >>= 1) m[c] = fmax(m[c], __shfl_xor(m[c], off));
    if (lane < Q)
#pragma unroll
        for (int c = 0; c < 4; ++c) s_w[wave * NT + 4 * lane + c] = m[c];
    __syncthreads();
    if (static_cast<int>(threadIdx.x) < NT) {
        const int k = threadIdx.x;
        s_out[k] = fmax(fmax(s_w[k], s_w[NT + k]), fmax(s_w[2 * NT + k], s_w[3 * NT + k]));
    }
    __syncthreads();
}

// Stage V = 2^(g - M) of orientations [k0, k0 + KS) of the halo in LDS, [hy][hx][KS], as
// bfloat16 (RNE) or FP32; zero outside the grid and for zero mass.
// With kshift (LDS, NT integers) the shift of orientation k is kshift[k] instead of M.
template <int NT, int KS, bool BF16>
__device__ __forceinline__ void stage_shifted(void *lds, const double *in_, double M, int k0, int nx, int ny, int HWX,
                                              int HWY, int xl, int ylo, const int *kshift = nullptr) {
    constexpr int Q = KS / 4;
    constexpr int BATCH = 4;
    const gdptr in = (gdptr)in_;
    const int total = HWY * HWX * Q;
    const float inv = 1.0f / static_cast<float>(HWX);
    for (int e0 = 0; e0 < total; e0 += BATCH * 256) {
        double v[BATCH][4];
        bool ok[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const int e = min(e0 + u * 256 + static_cast<int>(threadIdx.x), total - 1);
            const int p = e / Q, q = e - p * Q;
            const int hy = static_cast<int>((static_cast<float>(p) + 0.5f) * inv), hx = p - hy * HWX;
            const int gy = ylo + hy, gx = xl + hx;
            ok[u] = gy >= 0 && gy < ny && gx >= 0 && gx < nx;
            const int cy = min(max(gy, 0), ny - 1), cx = min(max(gx, 0), nx - 1);
            const gdptr src = in + (static_cast<size_t>(cy) * nx + cx) * NT + k0 + 4 * q;
#pragma unroll
            for (int c = 0; c < 4; ++c) v[u][c] = src[c];
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const int e = e0 + u * 256 + static_cast<int>(threadIdx.x);
            if (e < total) {
                float f[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    // 2^d with d = g - M split as dh + dl (dh = FP32(d), |dl| <= 2^-24 |d|):
                    // 2^dh (native exp2) times 1 + dl ln 2, so that the FP32 rounding of a
                    // large |d| does not enter the result
                    const int kk = k0 + 4 * ((e0 + u * 256 + static_cast<int>(threadIdx.x)) % Q) + c;
                    const double d = v[u][c] - (kshift != nullptr ? static_cast<double>(kshift[kk]) : M);
                    const float dh = static_cast<float>(d);
                    const float e = __builtin_amdgcn_exp2f(dh);
                    if constexpr (BF16) {
                        f[c] = ok[u] ? e : 0.0f;
                    } else {
                        const float dl = static_cast<float>(d - static_cast<double>(dh));
                        f[c] = (ok[u] && v[u][c] != -INFINITY) ? fmaf(e, dl * 0.693147180559945309f, e) : 0.0f;
                    }
                }
                if constexpr (BF16) {
                    *reinterpret_cast<uint2 *>(static_cast<uint16_t *>(lds) + 4 * e) =
                        make_uint2(f32x2_to_bf16x2_rne(f[0], f[1]), f32x2_to_bf16x2_rne(f[2], f[3]));
                } else {
                    *reinterpret_cast<float4 *>(static_cast<float *>(lds) + 4 * e) = make_float4(f[0], f[1], f[2], f[3]);
                }
            }
        }
    }
}

// Certificate, epilogue, error partials and the fallback list of a matrix-core tile.
// S[r][nb][q] is the shifted sum of the lane's output at pixel x0 + 4 (lane / 16) + q of row
// y0 + row0 + r, orientation ko = 16 nb + lane % 16, and Mk[nb] the log2 of its frame.  The group (8 x 8 tile, ko) of an output
// is held by lanes ko + 16 {2h, 2h + 1} (h = 8-pixel half of the segment) over 8 rows: one
// wave at 8 rows per wave, the wave pair (2m, 2m + 1) at 4 rows per wave.  Fixed-order sums:
// within a lane over (r, q), then the even lane's sum plus the odd lane's, then the even
// wave's plus the odd wave's.  An 8 x 8 tile with rejected groups is listed once, with the
// mask of its rejected orientations.
template <int NT, int RPW, int NB>
__device__ __forceinline__ void lin_log_epilogue(const ConvJob &job, int jb, const double (&S)[RPW][NB][4],
                                                 const double (&Mk)[NB],
                                                 int x0, int y0, int row0, int lane, int wave, int4 *__restrict__ fb,
                                                 int *__restrict__ fb_count, int *s_xi, double *s_xd) {
    const int nx = job.nx, ny = job.ny;
    const int kb = lane >> 4, jj = lane & 15;
    const int tx8 = (x0 >> 3) + (kb >> 1);
    const int ty8 = (y0 + row0) >> 3;
    const bool rep = ((kb & 1) == 0) && (RPW == 8 || (wave & 1) == 0);
    const size_t slot = static_cast<size_t>(ty8 * job.tiles_x + tx8) * NT;
    uint32_t rejected[2] = {0u, 0u};  // per 8-pixel half: orientations to recompute (wave-uniform)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int ko = 16 * nb + jj;
        int any = 0, bad = 0;
#pragma unroll
        for (int r = 0; r < RPW; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gx = x0 + 4 * kb + q, gy = y0 + row0 + r;
                if (ko < NT && gx < nx && gy < ny) {
                    any = 1;
                    if (!(S[r][nb][q] >= static_cast<double>(kLinCert))) bad = 1;
                }
            }
        any |= __shfl_xor(any, 16);
        bad |= __shfl_xor(bad, 16);
        if constexpr (RPW == 4) {
            __syncthreads();  // the previous round's reads of s_xi are done
            s_xi[wave * 64 + lane] = any | (bad << 1);
            __syncthreads();
            const int o = s_xi[(wave ^ 1) * 64 + lane];
            any |= o & 1;
            bad |= o >> 1;
        }
        double err = 0.0;
        if (any && !bad) {
#pragma unroll
            for (int r = 0; r < RPW; ++r)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int gx = x0 + 4 * kb + q, gy = y0 + row0 + r;
                    if (ko < NT && gx < nx && gy < ny) {
                        const double lse = Mk[nb] + log2(S[r][nb][q]);
                        err += epilogue(job, (static_cast<size_t>(gy) * nx + gx) * NT + ko, lse);
                    }
                }
        }
        if (job.epi == EPI_SCALE && job.partial != nullptr) {
            const double eo = __shfl_xor(err, 16);
            double e = ((kb & 1) == 0) ? err + eo : eo + err;
            if constexpr (RPW == 4) {
                s_xd[wave * 64 + lane] = e;
                __syncthreads();
                const double ow = s_xd[(wave ^ 1) * 64 + lane];
                e = ((wave & 1) == 0) ? e + ow : ow + e;
            }
            if (rep && any && !bad) job.partial[slot + ko] = e;
        }
        // rejected groups: lane 16 kb + jj with kb = 2h stands for (half h, ko)
        const unsigned long long m = __ballot(rep && any && bad);
        rejected[0] |= static_cast<uint32_t>(m & 0xffffull) << (16 * nb);
        rejected[1] |= static_cast<uint32_t>((m >> 32) & 0xffffull) << (16 * nb);
    }
    const int np = (rejected[0] != 0u ? 1 : 0) + (rejected[1] != 0u ? 1 : 0);
    if (np > 0 && lane == 0) {
        int base = atomicAdd(fb_count, np);
        const int row = ty8 * job.tiles_x + (x0 >> 3);
        if (rejected[0] != 0u) fb[base++] = make_int4(jb, row, static_cast<int>(rejected[0]), 0);
        if (rejected[1] != 0u) fb[base] = make_int4(jb, row + 1, static_cast<int>(rejected[1]), 0);
    }
}

// BF16 operands: V rounded to bfloat16, the kernel's bfloat16 table, FP32 accumulation.
template <int NT, int DYC, int RPW>
__global__ __launch_bounds__(256) void k_lin_log_bf16(const ConvJob *__restrict__ jobs,
                                                      const int32_t *__restrict__ block_job, int4 *__restrict__ fb,
                                                      int *__restrict__ fb_count, int *__restrict__ fb_next) {
    using P = Pack<NT>;
    extern __shared__ uint16_t lds16[];
    __shared__ double s_m[kWaves];
    __shared__ int s_xi[kWaves * 64];
    __shared__ double s_xd[kWaves * 64];
    // the list counter of the following launch (its readers have finished: stream order)
    if (blockIdx.x == 0 && threadIdx.x == 0) *fb_next = 0;
    const int jb = block_job[blockIdx.x];
    const ConvJob job = jobs[jb];
    const int lt = static_cast<int>(blockIdx.x) - job.first_block;
    const int nx = job.nx, ny = job.ny, R = job.R, W = 2 * R + 1;
    const int G = (W + P::SPM - 1) / P::SPM;
    const int HWX = kSeg + 2 * R + (G * P::SPM - W);
    constexpr int kRows = RPW * kWaves;
    const int HWY = kRows + 2 * R;
    const int ltx = (nx + kSeg - 1) / kSeg;
    const int ty = lt / ltx, tx = lt - ty * ltx;
    const int x0 = tx * kSeg, y0 = ty * kRows;
    const int xl = x0 - R - (G * P::SPM - W);
    double M = halo_max<NT>(job.in, nx, ny, HWX, HWY, xl, y0 - R, s_m);
    if (M == -INFINITY) M = 0.0;  // no mass in the halo: every V is 0, every group goes to the fallback
    stage_shifted<NT, NT, true>(lds16, job.in, M, 0, nx, ny, HWX, HWY, xl, y0 - R);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int row0 = wave * RPW;
    f32x4_t acc[RPW][P::NB];
    bf16x8_t b0[DYC][Pack<NT>::NB], b1[DYC][Pack<NT>::NB];
    bf16_first_b<NT, DYC>(b0, b1, reinterpret_cast<const bf16x8_t *>(job.kop), R, lane);
    bf16_contract<NT, DYC, RPW>(acc, lds16, reinterpret_cast<const bf16x8_t *>(job.kop), R, x0, xl, row0, lane, b0,
                                b1);
    double S[RPW][P::NB][4];
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int nb = 0; nb < P::NB; ++nb)
#pragma unroll
            for (int q = 0; q < 4; ++q) S[r][nb][q] = static_cast<double>(acc[r][nb][q]);
    double Mk[P::NB];
#pragma unroll
    for (int nb = 0; nb < P::NB; ++nb) Mk[nb] = M;
    lin_log_epilogue<NT, RPW, P::NB>(job, jb, S, Mk, x0, y0, row0, lane, wave, fb, fb_count, s_xi, s_xd);
}

// FP32 operands on the FP32 matrix cores (nt = 16, 32): V and the kernel in FP32, FP32 sums
// over one step added into FP64 accumulators.  Frames per orientation: input orientation ki is
// shifted by s_ki = ceil(max of g(., ki) over the halo), output orientation ko is reported in
// the frame t_ko = ceil(max_ki (s_ki + L2[0][ko][ki])), and the kernel value K[d][ko][ki]
// enters as K 2^(s_ki - t_ko) <= 1 (L2[d][ko][ki] <= L2[0][ko][ki]: the distance grows with the
// offset), an exact exponent change.  Every term is <= 1 in the frame of its output, so the
// certificate of kLinCert holds as for one shift per tile, while an orientation far from the
// dominant ones (the tails of a peaked angular profile) keeps its own scale.
constexpr int kNoMassShift = -(1 << 26);
template <int NT, int DYC, int RPW>
__global__ __launch_bounds__(256) void k_lin_log_f32(const ConvJob *__restrict__ jobs,
                                                     const int32_t *__restrict__ block_job, int4 *__restrict__ fb,
                                                     int *__restrict__ fb_count, int *__restrict__ fb_next) {
    static_assert(NT == 16 || NT == 32, "16 or 32 orientations");
    constexpr int NB = NT / 16, NP = NT / 16;
    extern __shared__ float lds32[];
    __shared__ double s_w[kWaves * NT];
    __shared__ double s_max[NT];
    __shared__ int s_sk[NT], s_tk[NT];
    __shared__ int s_xi[kWaves * 64];
    __shared__ double s_xd[kWaves * 64];
    if (blockIdx.x == 0 && threadIdx.x == 0) *fb_next = 0;
    const int jb = block_job[blockIdx.x];
    const ConvJob job = jobs[jb];
    const int lt = static_cast<int>(blockIdx.x) - job.first_block;
    const int nx = job.nx, ny = job.ny, R = job.R, W = 2 * R + 1;
    const int HWX = kSeg + 2 * R;
    constexpr int kRows = RPW * kWaves;
    const int HWY = kRows + 2 * R;
    const int ltx = (nx + kSeg - 1) / kSeg;
    const int ty = lt / ltx, tx = lt - ty * ltx;
    const int x0 = tx * kSeg, y0 = ty * kRows;
    const int xl = x0 - R;
    const f32x4_t *Fp = reinterpret_cast<const f32x4_t *>(job.kop);
    halo_max_per_k<NT>(job.in, nx, ny, HWX, HWY, xl, y0 - R, s_w, s_max);
    if (static_cast<int>(threadIdx.x) < NT) {
        const double m = s_max[threadIdx.x];
        s_sk[threadIdx.x] = (m == -INFINITY) ? kNoMassShift
                                             : static_cast<int>(ceil(fmin(fmax(m, -67108864.0), 67108864.0)));
    }
    __syncthreads();
    if (static_cast<int>(threadIdx.x) < NT) {
        const int ko = threadIdx.x;
        const gdptr L0 = (gdptr)(job.L64) + (static_cast<size_t>(R * W + R) * NT + ko) * NT;  // offset d = 0
        double t = -INFINITY;
        for (int ki = 0; ki < NT; ++ki) t = fmax(t, static_cast<double>(s_sk[ki]) + L0[ki]);
        s_tk[ko] = static_cast<int>(ceil(fmin(fmax(t, -67108864.0 * 2.0), 67108864.0)));
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int row0 = wave * RPW;
    f32x4_t acc[RPW][NB];
    double acc64[RPW][NB][4];
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            acc[r][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < 4; ++q) acc64[r][nb][q] = 0.0;
        }
    const int nchunks = (W + DYC - 1) / DYC;
    f32x4_t b0[DYC][NB];
    for (int pass = 0; pass < NP; ++pass) {
        f32m_load_b<NT, DYC>(b0, Fp, 0, pass, nchunks, W, lane);
        // exponent of fragment element e of block nb: s(ki) - t(ko), ki = 16 pass + 4 (lane / 16) + e,
        // ko = 16 nb + lane % 16 (clamped: K 2^x with x below -300 is zero either way)
        int kx[NB][4];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                kx[nb][e] = max(s_sk[16 * pass + 4 * (lane >> 4) + e] - s_tk[16 * nb + (lane & 15)], -300);
        if (pass > 0) __syncthreads();  // every wave is done with the previous pass's halo
        stage_shifted<NT, 16, false>(lds32, job.in, 0.0, 16 * pass, nx, ny, HWX, HWY, xl, y0 - R, s_sk);
        __syncthreads();
        f32m_steps<NT, DYC, RPW, true, true>(acc, acc64, b0, lds32, Fp, pass, R, row0, lane, kx);
    }
    double Mk[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) Mk[nb] = static_cast<double>(s_tk[16 * nb + (lane & 15)]);
    lin_log_epilogue<NT, RPW, NB>(job, jb, acc64, Mk, x0, y0, row0, lane, wave, fb, fb_count, s_xi, s_xd);
}

template <int NT, int DYC, int RPW, bool BF16>
int launch_lin_log_t(const ConvJob *d_jobs, int nblocks, const int32_t *d_map, int R, int4 *fb, int *fb_count,
                     int *fb_next, hipStream_t s) {
    const int rows = RPW * kWaves;
    size_t lds;
    const void *fn;
    if constexpr (BF16) {
        using P = Pack<NT>;
        const int W = 2 * R + 1, G = (W + P::SPM - 1) / P::SPM;
        lds = static_cast<size_t>(kSeg + 2 * R + (G * P::SPM - W)) * (rows + 2 * R) * NT * sizeof(uint16_t);
        fn = reinterpret_cast<const void *>(&k_lin_log_bf16<NT, DYC, RPW>);
    } else {
        lds = static_cast<size_t>(kSeg + 2 * R) * (rows + 2 * R) * 16 * sizeof(float);
        fn = reinterpret_cast<const void *>(&k_lin_log_f32<NT, DYC, RPW>);
    }
    if (lds > 65536) SE2_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    // the exact recomputation of rejected groups follows: this is not the group's last kernel
    if constexpr (BF16)
        return launch_kernel(&k_lin_log_bf16<NT, DYC, RPW>, dim3(nblocks), dim3(256), lds, s, false, d_jobs, d_map, fb,
                             fb_count, fb_next);
    else
        return launch_kernel(&k_lin_log_f32<NT, DYC, RPW>, dim3(nblocks), dim3(256), lds, s, false, d_jobs, d_map, fb,
                             fb_count, fb_next);
}

// nt = 32 has one row count per operand type (lin_rows_per_wave): 8 rows for bfloat16, 4 for
// FP32 (its two FP64 accumulator blocks); nt <= 16 has both.
template <int NT, int DYC, bool BF16>
int launch_lin_log_rpw(const ConvJob *d_jobs, int nblocks, const int32_t *d_map, int R, int rpw, int4 *fb,
                       int *fb_count, int *fb_next, hipStream_t s) {
    if constexpr (NT == 32) {
        constexpr int kR = BF16 ? 8 : 4;
        if (rpw != kR) return SE2_EINVAL;
        return launch_lin_log_t<NT, DYC, kR, BF16>(d_jobs, nblocks, d_map, R, fb, fb_count, fb_next, s);
    } else {
        if (rpw == 8) return launch_lin_log_t<NT, DYC, 8, BF16>(d_jobs, nblocks, d_map, R, fb, fb_count, fb_next, s);
        return launch_lin_log_t<NT, DYC, 4, BF16>(d_jobs, nblocks, d_map, R, fb, fb_count, fb_next, s);
    }
}

template <int NT, bool BF16>
int launch_lin_log_nt(const ConvJob *d_jobs, int nblocks, const int32_t *d_map, int R, int rpw, int4 *fb,
                      int *fb_count, int *fb_next, hipStream_t s) {
    switch (dy_chunk(2 * R + 1)) {
        case 4: return launch_lin_log_rpw<NT, 4, BF16>(d_jobs, nblocks, d_map, R, rpw, fb, fb_count, fb_next, s);
        case 5: return launch_lin_log_rpw<NT, 5, BF16>(d_jobs, nblocks, d_map, R, rpw, fb, fb_count, fb_next, s);
        case 6: return launch_lin_log_rpw<NT, 6, BF16>(d_jobs, nblocks, d_map, R, rpw, fb, fb_count, fb_next, s);
        case 7: return launch_lin_log_rpw<NT, 7, BF16>(d_jobs, nblocks, d_map, R, rpw, fb, fb_count, fb_next, s);
        case 8: return launch_lin_log_rpw<NT, 8, BF16>(d_jobs, nblocks, d_map, R, rpw, fb, fb_count, fb_next, s);
        default: return SE2_EINVAL;
    }
}

template <int NT, int DYC, int RPW>
int launch_bf16_t(const Kernel &k, const float *in, float *out, int batch, hipStream_t s) {
    using P = Pack<NT>;
    const int nx = k.grid.nx, ny = k.grid.ny, R = k.metric.radius, W = 2 * R + 1;
    const int G = (W + P::SPM - 1) / P::SPM;
    const int rows = RPW * kWaves;
    const int HWX = kSeg + 2 * R + (G * P::SPM - W), HWY = rows + 2 * R;
    const size_t lds = static_cast<size_t>(HWX) * HWY * NT * sizeof(uint16_t);
    const int tx = (nx + kSeg - 1) / kSeg, ty = (ny + rows - 1) / rows;
    if (lds > 65536)
        SE2_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_conv_bf16<NT, DYC, RPW>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    hipLaunchKernelGGL((k_conv_bf16<NT, DYC, RPW>), dim3(tx * ty * batch), dim3(256), lds, s, in, out,
                       reinterpret_cast<const bf16x8_t *>(k.d_Bpack), nx, ny, R, tx, ty);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

// 8 output rows per wave, or 4 (twice the workgroups, less reuse per LDS read) when
// 8 would leave fewer than 4 workgroups per compute unit.  nt = 32 keeps 8: its halo
// limits it to one workgroup per compute unit either way (measured: 8 rows faster).
template <int NT, int DYC>
int launch_bf16_rpw(const Kernel &k, const float *in, float *out, int batch, hipStream_t s) {
    const long tiles8 = static_cast<long>((k.grid.nx + kSeg - 1) / kSeg) * ((k.grid.ny + 8 * kWaves - 1) / (8 * kWaves));
    if (NT >= 32 || tiles8 * batch >= 4L * kNumCUs) return launch_bf16_t<NT, DYC, 8>(k, in, out, batch, s);
    if constexpr (NT < 32) return launch_bf16_t<NT, DYC, 4>(k, in, out, batch, s);
    return SE2_EINVAL;
}

template <int NT>
int launch_bf16_nt(const Kernel &k, const float *in, float *out, int batch, hipStream_t s) {
    switch (dy_chunk(2 * k.metric.radius + 1)) {
        case 4: return launch_bf16_rpw<NT, 4>(k, in, out, batch, s);
        case 5: return launch_bf16_rpw<NT, 5>(k, in, out, batch, s);
        case 6: return launch_bf16_rpw<NT, 6>(k, in, out, batch, s);
        case 7: return launch_bf16_rpw<NT, 7>(k, in, out, batch, s);
        case 8: return launch_bf16_rpw<NT, 8>(k, in, out, batch, s);
        default: return SE2_EINVAL;
    }
}

template <int NT, int DYC, int RPW>
int launch_f32m_t(const Kernel &k, const float *in, float *out, int batch, hipStream_t s) {
    const int nx = k.grid.nx, ny = k.grid.ny, R = k.metric.radius;
    const int rows = RPW * kWaves;
    const size_t lds = static_cast<size_t>(kSeg + 2 * R) * (rows + 2 * R) * 16 * sizeof(float);
    const int tx = (nx + kSeg - 1) / kSeg, ty = (ny + rows - 1) / rows;
    if (lds > 65536)
        SE2_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_conv_f32m<NT, DYC, RPW>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    hipLaunchKernelGGL((k_conv_f32m<NT, DYC, RPW>), dim3(tx * ty * batch), dim3(256), lds, s, in, out,
                       reinterpret_cast<const f32x4_t *>(k.d_Fpack), nx, ny, R, tx, ty);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

// nt = 16: 8 output rows per wave, or 4 when 8 would leave fewer than 4 workgroups per
// compute unit.  nt = 32: 4 rows per wave (one 83 KB halo per CU at the 21 x 21 window;
// measured at 256 x 256 x 32: 1852 us against 1995 us with 2 rows and two halos per CU).
template <int NT, int DYC>
int launch_f32m_rpw(const Kernel &k, const float *in, float *out, int batch, hipStream_t s) {
    if constexpr (NT == 32) {
        return launch_f32m_t<NT, DYC, 4>(k, in, out, batch, s);
    } else {
        const long tiles8 =
            static_cast<long>((k.grid.nx + kSeg - 1) / kSeg) * ((k.grid.ny + 8 * kWaves - 1) / (8 * kWaves));
        if (tiles8 * batch >= 4L * kNumCUs) return launch_f32m_t<NT, DYC, 8>(k, in, out, batch, s);
        return launch_f32m_t<NT, DYC, 4>(k, in, out, batch, s);
    }
}

template <int NT>
int launch_f32m_nt(const Kernel &k, const float *in, float *out, int batch, hipStream_t s) {
    switch (dy_chunk(2 * k.metric.radius + 1)) {
        case 4: return launch_f32m_rpw<NT, 4>(k, in, out, batch, s);
        case 5: return launch_f32m_rpw<NT, 5>(k, in, out, batch, s);
        case 6: return launch_f32m_rpw<NT, 6>(k, in, out, batch, s);
        case 7: return launch_f32m_rpw<NT, 7>(k, in, out, batch, s);
        case 8: return launch_f32m_rpw<NT, 8>(k, in, out, batch, s);
        default: return SE2_EINVAL;
    }
}

template <typename T, int NT, int KC>
int launch_valu_kc(const Kernel &k, const T *K, const T *in, T *out, int batch, hipStream_t s) {
    const int nx = k.grid.nx, ny = k.grid.ny, R = k.metric.radius;
    const int HW = kTile + 2 * R;
    const size_t lds = static_cast<size_t>(HW) * HW * KC * sizeof(T);
    const int tx = tiles_of(nx), ty = tiles_of(ny);
    hipLaunchKernelGGL((k_conv_valu<T, NT, KC>), dim3(tx * ty * batch), dim3(256), lds, s, in, out, K, nx, ny, R,
                       tx, ty);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
}

// Largest chunk of input orientations whose halo fits in 64 KiB of LDS.
template <typename T, int NT>
int launch_valu_t(const Kernel &k, const T *K, const T *in, T *out, int batch, hipStream_t s) {
    const int HW = kTile + 2 * k.metric.radius;
    const size_t per_k = static_cast<size_t>(HW) * HW * sizeof(T);
    if (per_k * NT <= 65536) return launch_valu_kc<T, NT, NT>(k, K, in, out, batch, s);
    if constexpr (NT > 8) {
        if (per_k * 8 <= 65536) return launch_valu_kc<T, NT, 8>(k, K, in, out, batch, s);
    }
    return launch_valu_kc<T, NT, 4>(k, K, in, out, batch, s);
}

}  // namespace

size_t conv_bf16_lds_bytes(int nt, int R) {
    const int W = 2 * R + 1;
    const int spm = (nt >= 32) ? 1 : 32 / nt;
    const int G = (W + spm - 1) / spm;
    return static_cast<size_t>(kSeg + 2 * R + (G * spm - W)) * (8 * kWaves + 2 * R) * nt * sizeof(uint16_t);
}

// Host packing of the bfloat16 kernel into MFMA B-operand order:
// Bp[dy][g][nb][lane][e] = K[dy][dx = -R + g*SPM + slot][ko = nb*16 + lane%16][ki], where
// lane/16 = kb selects K-rows 8*kb .. 8*kb+7 = (slot, ki); zero outside the window or
// ko >= NT.  The dy rows run on to a multiple of the dy chunk (zero rows).
std::vector<uint16_t> pack_bf16_operand(const std::vector<uint16_t> &Kb, int nt, int R) {
    const int W = 2 * R + 1;
    const int spm = (nt >= 32) ? 1 : 32 / nt;
    const int kis = 32 / spm;
    const int NB = (nt > 16) ? nt / 16 : 1;
    const int G = (W + spm - 1) / spm;
    const int DYC = dy_chunk(W);
    const int WP = (W + DYC - 1) / DYC * DYC;
    std::vector<uint16_t> Bp(static_cast<size_t>(WP) * G * NB * 64 * 8, 0);
    for (int dyi = 0; dyi < W; ++dyi)
        for (int g = 0; g < G; ++g)
            for (int nb = 0; nb < NB; ++nb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int e = 0; e < 8; ++e) {
                        const int krow = 8 * (lane >> 4) + e;
                        const int slot = krow / kis, ki = krow % kis;
                        const int dxi = g * spm + slot;
                        const int ko = nb * 16 + (lane & 15);
                        uint16_t v = 0;
                        if (dxi < W && ko < nt && ki < nt)
                            v = Kb[((static_cast<size_t>(dyi) * W + dxi) * nt + ko) * nt + ki];
                        Bp[((((static_cast<size_t>(dyi) * G + g) * NB + nb) * 64 + lane) * 8) + e] = v;
                    }
    return Bp;
}

// Host packing of the FP32 kernel (nt = 16 or 32) into the B operands of k_conv_f32m:
// Fp[dyp][dx][pass][nb][lane][e] = K[dy = dyp - R][dx - R][ko = 16 nb + lane % 16]
// [ki = 16 pass + 4 (lane / 16) + e], zero for the dy rows that run past the window to a
// multiple of the dy chunk.
std::vector<float> pack_f32_operand(const std::vector<float> &K32, int nt, int R) {
    if (nt != 16 && nt != 32) return {};
    const int W = 2 * R + 1;
    const int DYC = dy_chunk(W);
    const int WP = (W + DYC - 1) / DYC * DYC;
    const int NB = nt / 16, NP = nt / 16;
    std::vector<float> Fp(static_cast<size_t>(WP) * W * NP * NB * 64 * 4, 0.0f);
    for (int dyi = 0; dyi < W; ++dyi)
        for (int dxi = 0; dxi < W; ++dxi)
            for (int pass = 0; pass < NP; ++pass)
                for (int nb = 0; nb < NB; ++nb)
                    for (int lane = 0; lane < 64; ++lane)
                        for (int e = 0; e < 4; ++e) {
                            const int ko = 16 * nb + (lane & 15), ki = 16 * pass + 4 * (lane >> 4) + e;
                            Fp[(((((static_cast<size_t>(dyi) * W + dxi) * NP + pass) * NB + nb) * 64 + lane) * 4) + e] =
                                K32[((static_cast<size_t>(dyi) * W + dxi) * nt + ko) * nt + ki];
                        }
    return Fp;
}

int launch_conv_bf16(const Kernel &k, const float *in, float *out, int batch, hipStream_t s) {
    switch (k.grid.ntheta) {
        case 8: return launch_bf16_nt<8>(k, in, out, batch, s);
        case 16: return launch_bf16_nt<16>(k, in, out, batch, s);
        case 32: return launch_bf16_nt<32>(k, in, out, batch, s);
        default: return SE2_EINVAL;
    }
}

int launch_conv_f32(const Kernel &k, const float *in, float *out, int batch, hipStream_t s) {
    switch (k.grid.ntheta) {
        case 8: return launch_valu_t<float, 8>(k, k.d_K32, in, out, batch, s);
        case 16: return k.d_Fpack ? launch_f32m_nt<16>(k, in, out, batch, s)
                                  : launch_valu_t<float, 16>(k, k.d_K32, in, out, batch, s);
        case 32: return k.d_Fpack ? launch_f32m_nt<32>(k, in, out, batch, s)
                                  : launch_valu_t<float, 32>(k, k.d_K32, in, out, batch, s);
        default: return SE2_EINVAL;
    }
}

int lin_rows_per_wave(int nt, bool bf16, int ny) {
    if (nt == 32) return bf16 ? 8 : 4;
    return ny >= 128 ? 8 : 4;
}

int lin_blocks(int nx, int ny, int rpw) {
    const int rows = rpw * kWaves;
    return ((nx + kSeg - 1) / kSeg) * ((ny + rows - 1) / rows);
}

bool lin_supported(int nt, bool bf16) { return bf16 ? (nt == 8 || nt == 16 || nt == 32) : (nt == 16 || nt == 32); }

int launch_conv_lin_log(const ConvJob *d_jobs, int nblocks, const int32_t *d_block_job, int nt, int R, int rpw,
                        bool bf16, int4 *fb, int *fb_count, int *fb_next, int fb_grid, hipStream_t s) {
    if (nblocks <= 0) return SE2_OK;
    if (R < 0 || R > kMaxRadius || (rpw != 4 && rpw != 8) || !lin_supported(nt, bf16) || !fb || !fb_count ||
        !fb_next || fb_count == fb_next)
        return SE2_EINVAL;
    int rc;
    switch (nt) {
        case 8: rc = launch_lin_log_nt<8, true>(d_jobs, nblocks, d_block_job, R, rpw, fb, fb_count, fb_next, s); break;
        case 16:
            rc = bf16 ? launch_lin_log_nt<16, true>(d_jobs, nblocks, d_block_job, R, rpw, fb, fb_count, fb_next, s)
                      : launch_lin_log_nt<16, false>(d_jobs, nblocks, d_block_job, R, rpw, fb, fb_count, fb_next, s);
            break;
        case 32:
            rc = bf16 ? launch_lin_log_nt<32, true>(d_jobs, nblocks, d_block_job, R, rpw, fb, fb_count, fb_next, s)
                      : launch_lin_log_nt<32, false>(d_jobs, nblocks, d_block_job, R, rpw, fb, fb_count, fb_next, s);
            break;
        default: return SE2_EINVAL;
    }
    if (rc) return rc;
    return launch_lse_tiles(d_jobs, fb_grid, nt, R, fb, fb_count, s);
}

int launch_conv_f64(const Kernel &k, const double *in, double *out, int batch, hipStream_t s) {
    switch (k.grid.ntheta) {
        case 8: return launch_valu_t<double, 8>(k, k.d_K64, in, out, batch, s);
        case 16: return launch_valu_t<double, 16>(k, k.d_K64, in, out, batch, s);
        case 32: return launch_valu_t<double, 32>(k, k.d_K64, in, out, batch, s);
        default: return SE2_EINVAL;
    }
}

}  // namespace se2
