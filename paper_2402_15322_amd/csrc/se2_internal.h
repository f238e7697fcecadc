// Internal declarations of the SE(2) entropic-OT library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/se2ot.h"
#include "conv_lse.h"

namespace se2 {

constexpr int kMaxMeasures = 65535;  // measures of one barycenter (a launch grid dimension)

#define SE2_HIP(call)                                                  \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) {                                        \
            se2::set_last_hip_error(e_, #call, __FILE__, __LINE__);    \
            return SE2_EHIP;                                           \
        }                                                              \
    } while (0)

void set_last_hip_error(hipError_t e, const char *what, const char *file, int line);
void set_last_error(const std::string &msg);  // the message se2_strerror() returns next

// Pruning state of one convolution direction of one solve.
struct ListSet {
    ListEntry *lists = nullptr;
    float *ref = nullptr;
    int32_t *len = nullptr;
    float *mref = nullptr;
    int32_t *dense_flag = nullptr;
    double *work = nullptr;
};

struct Kernel {
    se2_grid_t grid;
    se2_metric_t metric;
    int W = 0;                  // 2R+1
    size_t entries = 0;         // W*W*nt*nt
    std::vector<double> logk;   // natural-log kernel (host copy)
    std::vector<double> cost;   // rho^2 (host copy)
    double *d_L64 = nullptr;    // log2 kernel, FP64
    float *d_L32 = nullptr;     // log2 kernel, FP32
    float *d_cost32 = nullptr;  // rho^2, FP32 (plan statistics)
    float *d_K32 = nullptr;     // exp(logk) in FP32 (zero below the FP32 range)
    uint16_t *d_Kbf16 = nullptr; // exp(logk) in bfloat16 (RNE), table layout
    double *d_K64 = nullptr;    // exp(logk) in FP64
    uint16_t *d_Bpack = nullptr; // bfloat16 kernel packed in MFMA B-operand order
    float *d_Fpack = nullptr;    // FP32 kernel packed in FP32-MFMA B-operand order (nt = 16, 32)
    int nonzero_bf16 = 0;       // window offsets with any nonzero bfloat16 entry
    int device = 0;
    // eps-scaling: kernels of the same grid, weights and window at coarser eps, built on
    // first use and owned by this handle (the handle stays immutable for its callers)
    mutable std::mutex scaled_mu;
    mutable std::vector<std::pair<double, Kernel *>> scaled;
};

// The kernel of `base`'s grid, weights and window at `eps` (base itself when eps equals
// its own), built on first use and kept with `base`; thread-safe.
int kernel_at_eps(const Kernel &base, double eps, const Kernel **out);
void kernel_free(Kernel *k);

// kernel_table.cpp
int build_tables(Kernel &k);

// launchers (conv_lse.hip)
// Error partials of EPI_SCALE jobs are laid out [tile][nt]; `rebuild` must hold one
// int2 per block of the launch (sparse launches only).  A sparse launch rebuilds its
// uncertified tiles at rb_waves (8 or 16) waves per (tile, ko) item, with identical
// results either way, and stores the number of items it found to *published (pinned
// host memory, may be null) for the caller's next choice of width.
int launch_conv_lse(const ConvJob *d_jobs, int njobs, int nblocks, const int32_t *d_block_job, int nt, int R_max,
                    bool f64exp, bool sparse, int2 *rebuild, int *rebuild_count, int *next_count, int rb_waves,
                    int *published, hipStream_t s);
bool conv_lse_sparse_fits(int nt, int R);
// Exact log-domain recomputation of listed tiles (the fallback of the matrix-core engines):
// item (job, 8 x 8 tile, mask of the orientations to recompute, unused); `count` (device)
// holds the number of items, `grid` workgroups loop over them.
int launch_lse_tiles(const ConvJob *d_jobs, int grid, int nt, int R_max, const int4 *items, const int *count,
                     hipStream_t s);

// launchers (conv_linear.hip)
std::vector<uint16_t> pack_bf16_operand(const std::vector<uint16_t> &Kb, int nt, int R);
std::vector<float> pack_f32_operand(const std::vector<float> &K32, int nt, int R);  // empty unless nt = 16, 32
size_t conv_bf16_lds_bytes(int nt, int R);
int launch_conv_bf16(const Kernel &k, const float *in, float *out, int batch, hipStream_t s);
int launch_conv_f32(const Kernel &k, const float *in, float *out, int batch, hipStream_t s);
int launch_conv_f64(const Kernel &k, const double *in, double *out, int batch, hipStream_t s);
// Certified linear-domain log convolutions on the matrix cores (the solver's BF16 and FP32
// engines): jobs of one ntheta and window radius R, `rpw` output rows per wave (4 or 8, a
// function of the job's own grid, so that a job's tiles and results do not depend on what
// else is in the launch), workgroups of lin_blocks() per job.  The 8 x 8 tiles with groups
// (tile, ko) whose certificate fails are listed in fb (capacity: the jobs' tiles) with the
// count in *fb_count and recomputed exactly by fb_grid workgroups right after; *fb_next (the
// other of two counters) is zeroed for the following launch.  FP32 needs nt = 16 or 32.
bool lin_supported(int nt, bool bf16);
int lin_rows_per_wave(int nt, bool bf16, int ny);
int lin_blocks(int nx, int ny, int rpw);
int launch_conv_lin_log(const ConvJob *d_jobs, int nblocks, const int32_t *d_block_job, int nt, int R, int rpw,
                        bool bf16, int4 *fb, int *fb_count, int *fb_next, int fb_grid, hipStream_t s);

// elementwise.hip
int launch_scale(const double *in, double *out, size_t n, double mul, hipStream_t s);
int launch_log2_measure(const double *m, double *logm, size_t n, hipStream_t s);
int launch_validate(const double *m, size_t n, double *d_stats /* 2 + 2 * 256 doubles */, hipStream_t s);
int launch_fill(double *p, size_t n, double v, hipStream_t s);
int launch_fill_i32(int32_t *p, size_t n, int32_t v, hipStream_t s);
// One FP64 sum of part[begin, end): the marginal-error partials of one job.
struct SumItem {
    const void *part;  // double values, or uint32_t counters when ints != 0
    int32_t begin, end;
    int32_t ints = 0;
    int32_t pad = 0;
};
int launch_sum_items(const SumItem *d_items, int n, double *out, hipStream_t s);
// Copies errs[0, n) to host_errs (pinned, device-addressable) and then stores seq to
// *host_flag (the same memory kind) for a host that polls it.
int launch_publish(const double *errs, int n, double *host_errs, int *host_flag, int seq, hipStream_t s);
int launch_sum_partials(const double *partials, const int32_t *offsets, int njobs, double *out, hipStream_t s);
// IBP combine over device tables of the measures' log v_i and log d_i pointers and weights;
// `part` holds combine_chunks(n) * len doubles (unused when that is 1).
constexpr int kCombineChunk = 64;
inline int combine_chunks(int n) { return (n + kCombineChunk - 1) / kCombineChunk; }
int launch_ibp_combine(double *const *d_lv, const double *const *d_ld, const double *d_lam, int n, size_t len,
                       double *part, double *logbar, hipStream_t s);
// Plan statistics (transport cost sum pi rho^2 and mass sum pi) of pi = 2^(phi2 + L2 + psi2):
// one plan from phi/psi (tables null; partials [part][cost, mass]) or nplans plans from device
// pointer tables (partials [plan][cost | mass][part]); plan_parts(k) partials per plan.
int plan_parts(const Kernel &k);
int launch_plan_tiles(const Kernel &k, const double *phi, const double *psi, const double *const *phi_tab,
                      const double *const *psi_tab, int nplans, double *part, hipStream_t s);
// JKO step of the porous-medium flow: psi = prox(lsum) - lsum (base 2), nu = 2^(psi + lsum),
// and per-block partials of F(nu) = ref/(m-1) sum (nu/ref)^m.
int launch_porous_prox(const double *lsum, double *psi, size_t n, double c, double m, hipStream_t s);
int launch_exp2_sum(const double *a, const double *b, double *out, size_t n, hipStream_t s);
// p /= sum(p) on the device; stats holds 2 + 2 * 256 doubles.
int launch_normalise(double *p, size_t n, double *stats, hipStream_t s);
int launch_porous_energy(const double *a, const double *b, size_t n, double m, double ref, double *partials,
                         int nblocks, hipStream_t s);
int launch_reduce_fixed(const double *partials, int count, int stride, double *out, hipStream_t s);
int launch_exp2_out(const double *in2, double *out, size_t n, hipStream_t s);
int launch_dot_exp(const double *f2, const double *m, size_t n, double *partials, int nblocks, hipStream_t s);

// field.hip: lift and projection (period = Theta of the grid)
int launch_lift_field(const double *mag, const double *angle, double *out, size_t npix, int nt, double period,
                      hipStream_t s);
int launch_project(const double *u, const double *um, size_t npix, int nt, double period, double *mass,
                   int32_t *argmax, double *ang, hipStream_t s);
int split_blocks(size_t n);  // the scratch of launch_split_signed holds 2 * split_blocks(n) + 2 doubles
int launch_split_signed(const double *u, size_t n, double *plus, double *minus, double *part, hipStream_t s);
// The library's own split scratch on the current device (2 * kSplitNoallocMaxBlocks + 2 doubles,
// a file-scope device array of field.hip); its address is looked up once per device.
constexpr int kSplitNoallocMaxBlocks = 4096;
int split_noalloc_scratch(double **out);

// Sums and bad-entry counts of m arrays of length n (pointers in a device table): d_stats
// receives [m][2], d_part holds m * validate_many_blocks(n) * 2 doubles.
int validate_many_blocks(size_t n);
int launch_validate_many(const double *const *d_tab, int m, size_t n, double *d_stats, double *d_part, hipStream_t s);

// api.cpp: device-side FP64 check of a probability vector (finite, >= 0, |sum - 1| <= tol); syncs `st`.
int validate_measure(const double *m, size_t n, double tol, hipStream_t st);
// The same check for many vectors of one length with one launch and one synchronisation.
int validate_measures(const std::vector<const double *> &ms, size_t n, double tol, hipStream_t st);

// helpers
inline int tiles_of(int n) { return (n + kTile - 1) / kTile; }

}  // namespace se2
