// Linear SE(2) group convolution out = K * in (Section 4.2) on gfx950.
//
//   BF16: implicit GEMM on the matrix cores.  For a fixed window row dy and a group
//         of window columns, the contraction over (dx, ki) is a 16 x 32 by 32 x 16
//         product: rows = 16 output pixels of one image row, columns = 16 output
//         orientations ko, K-dimension = (dx slot, ki).  One
//         v_mfma_f32_16x16x32_bf16 per (output row segment, dy, dx group); FP32
//         accumulation over the whole window.  The input halo tile is rounded to
//         bfloat16 (RNE) once while it is staged in LDS; kernel fragments are
//         pre-packed on the host in operand order (one coalesced 16-byte load per
//         lane) and zero-padded where the dx group overhangs the window.
//   F32 / F64: the same tiling on the vector ALUs with FP32 / FP64 FMAs.
#include <hip/hip_runtime.h>

#include <cstring>

#include "se2_internal.h"

namespace se2 {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

namespace {

constexpr int kSeg = 16;   // output pixels per MFMA row block
constexpr int kRowsPerWave = 4;
constexpr int kWaves = 4;
constexpr int kRows = kRowsPerWave * kWaves;  // output rows per workgroup

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

// Geometry of the packing: SPM dx slots per MFMA K-dimension, NB column blocks of 16 ko.
template <int NT>
struct Pack {
    static constexpr int SPM = (NT >= 32) ? 1 : 32 / NT;  // 8 -> 4, 16 -> 2, 32 -> 1
    static constexpr int KI = 32 / SPM;                   // ki per slot (== NT for NT <= 32)
    static constexpr int NB = (NT > 16) ? NT / 16 : 1;
};

template <int NT>
__global__ __launch_bounds__(256) void k_conv_bf16(const float *__restrict__ in, float *__restrict__ out,
                                                   const bf16x8_t *__restrict__ Bp, int nx, int ny, int R,
                                                   int tiles_x, int tiles_y) {
    using P = Pack<NT>;
    extern __shared__ uint16_t lds16[];
    const int W = 2 * R + 1;
    const int G = (W + P::SPM - 1) / P::SPM;
    const int HWX = kSeg + 2 * R + (G * P::SPM - W);  // halo width incl. overhang of the last dx group
    const int HWY = kRows + 2 * R;
    const int tiles = tiles_x * tiles_y;
    const int b = blockIdx.x / tiles;
    const int t = blockIdx.x - b * tiles;
    const int ty = t / tiles_x, tx = t - ty * tiles_x;
    const int x0 = tx * kSeg, y0 = ty * kRows;
    const float *img = in + static_cast<size_t>(b) * nx * ny * NT;
    float *dst = out + static_cast<size_t>(b) * nx * ny * NT;

    // stage halo [hy][hx][ki] as bfloat16; hx = 0 is pixel x0 - R - (overhang)
    const int xl = x0 - R - (G * P::SPM - W);
    const int total = HWY * HWX * NT;
    for (int e = threadIdx.x; e < total; e += 256) {
        const int k = e % NT;
        const int p = e / NT;
        const int hy = p / HWX, hx = p - hy * HWX;
        const int gy = y0 - R + hy, gx = xl + hx;
        float v = 0.0f;
        if (gy >= 0 && gy < ny && gx >= 0 && gx < nx) v = img[(static_cast<size_t>(gy) * nx + gx) * NT + k];
        lds16[e] = f32_to_bf16_rne(v);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int i = lane & 15;   // output pixel within the segment (A row)
    const int kb = lane >> 4;  // 8-wide K block of this lane
    const int slot = (kb * 8) / P::KI;
    const int kio = (kb * 8) % P::KI;

    f32x4_t acc[kRowsPerWave][P::NB];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r)
#pragma unroll
        for (int nb = 0; nb < P::NB; ++nb) acc[r][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    for (int dy = -R; dy <= R; ++dy) {
        for (int g = 0; g < G; ++g) {
            bf16x8_t bfr[P::NB];
#pragma unroll
            for (int nb = 0; nb < P::NB; ++nb)
                bfr[nb] = Bp[((static_cast<size_t>(dy + R) * G + g) * P::NB + nb) * 64 + lane];
            // this lane's dx: slots of group g run dx = -R + g*SPM + slot
            const int dxl = -R + g * P::SPM + slot;
            // input pixel x0 + i - dx  ->  halo column (x0 + i - dx) - xl
            const int hx = x0 + i - dxl - xl;
#pragma unroll
            for (int r = 0; r < kRowsPerWave; ++r) {
                const int oy = wave * kRowsPerWave + r;        // output row within the tile
                const int hy = oy + R - dy;                    // input row y0 + oy - dy
                const bf16x8_t a = *reinterpret_cast<const bf16x8_t *>(&lds16[(hy * HWX + hx) * NT + kio]);
#pragma unroll
                for (int nb = 0; nb < P::NB; ++nb)
                    acc[r][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bfr[nb], acc[r][nb], 0, 0, 0);
            }
        }
    }

    // D: lane holds column j = lane % 16 (ko), rows 4*(lane/16) + q (pixels)
    const int j = lane & 15;
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
        const int gy = y0 + wave * kRowsPerWave + r;
        if (gy >= ny) continue;
#pragma unroll
        for (int nb = 0; nb < P::NB; ++nb) {
            const int ko = nb * 16 + j;
            if (ko >= NT) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gx = x0 + 4 * (lane >> 4) + q;
                if (gx < nx) dst[(static_cast<size_t>(gy) * nx + gx) * NT + ko] = acc[r][nb][q];
            }
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

template <int NT>
int launch_bf16_t(const Kernel &k, const float *in, float *out, int batch, hipStream_t s) {
    using P = Pack<NT>;
    const int nx = k.grid.nx, ny = k.grid.ny, R = k.metric.radius, W = 2 * R + 1;
    const int G = (W + P::SPM - 1) / P::SPM;
    const int HWX = kSeg + 2 * R + (G * P::SPM - W), HWY = kRows + 2 * R;
    const size_t lds = static_cast<size_t>(HWX) * HWY * NT * sizeof(uint16_t);
    const int tx = (nx + kSeg - 1) / kSeg, ty = (ny + kRows - 1) / kRows;
    if (lds > 65536)
        SE2_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_conv_bf16<NT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    hipLaunchKernelGGL(k_conv_bf16<NT>, dim3(tx * ty * batch), dim3(256), lds, s, in, out,
                       reinterpret_cast<const bf16x8_t *>(k.d_Bpack), nx, ny, R, tx, ty);
    SE2_HIP(hipGetLastError());
    return SE2_OK;
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
    return static_cast<size_t>(kSeg + 2 * R + (G * spm - W)) * (kRows + 2 * R) * nt * sizeof(uint16_t);
}

// Host packing of the bfloat16 kernel into MFMA B-operand order:
// Bp[dy][g][nb][lane][e] = K[dy][dx = -R + g*SPM + slot][ko = nb*16 + lane%16][ki], where
// lane/16 = kb selects K-rows 8*kb .. 8*kb+7 = (slot, ki); zero outside the window or ko >= NT.
std::vector<uint16_t> pack_bf16_operand(const std::vector<uint16_t> &Kb, int nt, int R) {
    const int W = 2 * R + 1;
    const int spm = (nt >= 32) ? 1 : 32 / nt;
    const int kis = 32 / spm;
    const int NB = (nt > 16) ? nt / 16 : 1;
    const int G = (W + spm - 1) / spm;
    std::vector<uint16_t> Bp(static_cast<size_t>(W) * G * NB * 64 * 8, 0);
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

int launch_conv_bf16(const Kernel &k, const float *in, float *out, int batch, hipStream_t s) {
    switch (k.grid.ntheta) {
        case 8: return launch_bf16_t<8>(k, in, out, batch, s);
        case 16: return launch_bf16_t<16>(k, in, out, batch, s);
        case 32: return launch_bf16_t<32>(k, in, out, batch, s);
        default: return SE2_EINVAL;
    }
}

int launch_conv_f32(const Kernel &k, const float *in, float *out, int batch, hipStream_t s) {
    switch (k.grid.ntheta) {
        case 8: return launch_valu_t<float, 8>(k, k.d_K32, in, out, batch, s);
        case 16: return launch_valu_t<float, 16>(k, k.d_K32, in, out, batch, s);
        case 32: return launch_valu_t<float, 32>(k, k.d_K32, in, out, batch, s);
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
