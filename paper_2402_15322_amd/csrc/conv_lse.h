// Shared definitions of the log-domain convolution kernels and their host side: base-2
// units, tile sizes, the certified-pruning constants and the job descriptor.
#pragma once

#include <cstddef>
#include <cstdint>

namespace se2 {

// Everything on the device works in base-2 log units: a log-scaling phi2 =
// f / (eps ln 2) and a log-kernel L2 = -rho^2 / (eps ln 2), so every exponential
// is a native exp2.  The C ABI speaks natural logs and converts at the edges.
constexpr double kLn2 = 0.693147180559945309417232121458176568;
constexpr double kLog2e = 1.442695040888963407359924681001892137;

constexpr int kTile = 8;          // output tile of the log-domain kernels: 8 x 8 pixels
constexpr int kConvThreads = 256; // 4 waves of 64
constexpr int kMaxRadius = 12;

// Certified pruning of the log-domain convolution (base-2 units): the entries within
// kListCut of an output's maximum are listed (the criterion has one unit of slack
// for the FP32 rounding of the maximum it is measured from); a list stays in use
// while the drift of the input from the halo it was built on spreads over at most
// kDriftSpread (that halo is kept in FP32: |value| < kRefMax, rounding error below
// kRefMargin / 2, added to the measured spread), so every skipped entry is below
// 2^-(kListCut - kDriftSpread) = 2^-48 of the result's largest term.
#ifndef SE2_LIST_CUT
#define SE2_LIST_CUT 88
#endif
#ifndef SE2_DRIFT_SPREAD
#define SE2_DRIFT_SPREAD 40
#endif
constexpr double kListCut = SE2_LIST_CUT;
constexpr float kDriftSpread = SE2_DRIFT_SPREAD;
constexpr float kRefMax = 1048576.0f;  // 2^20: FP32 rounding error < 2^-4
constexpr float kRefMargin = 0.125f;
#ifndef SE2_LIST_MAX
#define SE2_LIST_MAX 512
#endif
constexpr int kListMax = SE2_LIST_MAX;      // entries per (tile, ko); longer lists fall back to dense
constexpr int kListPad = 8;                 // entries after the last list: reads run past a list by < 8
constexpr size_t kSparseLdsMax = 98304;     // the sparse path keeps the full FP64 halo in LDS

// A list entry is the FP64 log2 kernel value of a window term with its low kOffBits
// mantissa bits replaced by the LDS offset of the term's input relative to the output
// pixel, ki*npix + (R-dy)*HW + (R-dx) (< 2^15 whenever the halo fits kSparseLdsMax);
// the kernel value changes by less than 2^-37 relative, far below the FP32 rounding
// of the exponents it enters.
typedef double ListEntry;
constexpr uint32_t kOffBits = 15;
constexpr int kRebuildGrid = 2048;          // workgroups of the rebuild kernel at 8 waves per item
constexpr int kRebuildGridWide = 256;       // the same at 16 waves per item (one item per workgroup and CU)
constexpr int kRebuildWideItems = 256;      // at most this many queued items: rebuild at 16 waves per item

// Device-side description of one log-domain convolution applied to one grid array.
enum Epilogue : int32_t {
    EPI_RAW = 0,   // out = LSE
    EPI_SCALE = 1, // out = logm - LSE  (Sinkhorn half-step / IBP w-update), error partial vs old
    EPI_ADD = 2,   // out = base + LSE   (IBP d-update: log d = log v + log K*w)
};

struct ConvJob {
    const double *in;   // log2 input [ny][nx][nt]
    double *out;        // log2 output
    const double *aux;  // EPI_SCALE: log2 marginal; EPI_ADD: base array
    const double *old;  // EPI_SCALE: previous output for the marginal error (may be null)
    double *partial;    // EPI_SCALE: one FP64 error partial per tile (may be null)
    const double *L64;  // log2 kernel [W][W][nt][nt], FP64
    const float *L32;   // the same in FP32 (max pass only)
    // certified pruning state of this (solve, direction); lists == nullptr: dense only
    ListEntry *lists;   // [tiles][nt][lmax] packed entries
    float *ref;         // [tiles][npix][nt] input halo the lists were built on (FP32, pixel-major)
    int32_t *len;       // [tiles][nt], -1 = none
    float *mref;        // [E] per-output maximum exponent at build time
    int32_t *dense_flag; // [tiles] dense visits (diagnostics), may be null
    double *work;       // [tiles][2] in-grid LSE terms evaluated on the dense / sparse path, may be null
    // certified linear-domain engines (matrix cores): the kernel in MFMA operand order and a
    // counter of the (tile, ko) groups recomputed in the log domain (may be null)
    const void *kop;
    int32_t *fallbacks;
    int32_t nx, ny, R, epi;
    int32_t tiles_x, tiles, first_block, lmax;
    int32_t blocks;     // workgroups of this job in its launch (8 x 8 tiles, or matrix-core tiles)
    int32_t pad_;
};

// Certificate of the linear-domain engines.  A workgroup shifts its input halo by its
// maximum M (so every exponential is <= 1) and sums S = sum K 2^(in - M) in FP32 on the
// matrix cores.  Entries that underflow (an input, kernel value or product below 2^-126)
// are lost, at most 2^-126 each, and a window holds fewer than 2^15 of them, so while
// S >= kLinCert = 2^-87 the lost part is below 2^-24 of S: the output keeps the
// precision of its arithmetic.  A group (8 x 8 tile, output orientation) with any output
// below the bound (or with S = 0) is recomputed exactly in the log domain.
constexpr float kLinCert = 0x1p-87f;

}  // namespace se2
