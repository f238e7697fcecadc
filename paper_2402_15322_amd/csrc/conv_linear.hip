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

#include "se2_internal.h"

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
    const int i = lane & 15;   // output pixel within the segment (A row)
    const int kb = lane >> 4;  // 8-wide K block of this lane
    const int slot = (kb * 8) / P::KI;
    const int kio = (kb * 8) % P::KI;
    const int row0 = wave * RPW;  // first output row of this wave within the tile

    f32x4_t acc[RPW][P::NB];
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int nb = 0; nb < P::NB; ++nb) acc[r][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    // (g, chunk) steps; the kernel fragments of the next step are loaded while the
    // current one runs on the matrix cores
    const int nchunks = (W + DYC - 1) / DYC;
    const int nsteps = G * nchunks;
    bf16x8_t b0[DYC][P::NB], b1[DYC][P::NB];
    auto load_b = [&](bf16x8_t(&dstb)[DYC][P::NB], int step) {
        const int g = step / nchunks, ch = step - g * nchunks;
        const bf16x8_t *src = Bp + (static_cast<size_t>(ch * DYC) * G + g) * P::NB * 64 + lane;
#pragma unroll
        for (int c = 0; c < DYC; ++c)
#pragma unroll
            for (int nb = 0; nb < P::NB; ++nb) dstb[c][nb] = src[(static_cast<size_t>(c) * G * P::NB + nb) * 64];
    };
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
        load_b(b0, 0);
        load_b(b1, min(1, nsteps - 1));
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
        // clamped (the last step reloads its own fragments) so the loop body has no branch
        load_b(b0, 0);
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

// FP32 convolution on the matrix cores, nt = 16 or 32: the tiling of k_conv_bf16 (kSeg
// output pixels by kWaves * RPW output rows per workgroup, window rows in chunks of
// DYC), one step per (dx, dy chunk), in NT / 16 passes over 16 input orientations each
// (the halo of one pass is staged in LDS in FP32).  For output row r and window row c of
// the chunk, the lane of pixel i = lane % 16 and quad kq = lane / 16 reads the pass's
// input orientations 4 kq .. 4 kq + 3 of its input pixel as one float4; MFMA e (e = 0..3)
// of column block nb multiplies element e by the packed B value
// K[ko = 16 nb + lane % 16][ki = 16 pass + 4 kq + e], so the four MFMAs sum the pass's 16
// orientations into the 16 output orientations of the block.
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
    const int i = lane & 15;      // output pixel within the segment (A row)
    const int kq = lane >> 4;     // orientation quad of this lane
    const int row0 = wave * RPW;  // first output row of this wave within the tile

    f32x4_t acc[RPW][NB];
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[r][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    // (dx, dy chunk) steps of a pass; the fragments of a step are loaded one step ahead,
    // those of a pass's first step before its halo staging, so that their latency overlaps it
    const int nchunks = (W + DYC - 1) / DYC;
    const int nsteps = W * nchunks;
    f32x4_t b0[DYC][NB], b1[DYC][NB];
    auto load_b = [&](f32x4_t(&dstb)[DYC][NB], int step, int pass) {
        const int dxi = step / nchunks, ch = step - dxi * nchunks;
#pragma unroll
        for (int c = 0; c < DYC; ++c)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                dstb[c][nb] = Fp[((((static_cast<size_t>(ch * DYC + c) * W + dxi) * NP + pass) * NB + nb) * 64) + lane];
    };
    const int xl = x0 - R;
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

    for (int pass = 0; pass < NP; ++pass) {
        load_b(b0, 0, pass);
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
        // a step is RPW * DYC * 4 * NB MFMAs of 32 cycles per wave: one step of lookahead
        // hides the fragment loads
        for (int step = 0; step < nsteps; ++step) {
            load_b(b1, min(step + 1, nsteps - 1), pass);
            __builtin_amdgcn_sched_barrier(0);
            run(b0, step);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = 0; c < DYC; ++c)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) b0[c][nb] = b1[c][nb];
        }
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

int launch_conv_f64(const Kernel &k, const double *in, double *out, int batch, hipStream_t s) {
    switch (k.grid.ntheta) {
        case 8: return launch_valu_t<double, 8>(k, k.d_K64, in, out, batch, s);
        case 16: return launch_valu_t<double, 16>(k, k.d_K64, in, out, batch, s);
        case 32: return launch_valu_t<double, 32>(k, k.d_K64, in, out, batch, s);
        default: return SE2_EINVAL;
    }
}

}  // namespace se2
