// Gibbs-kernel tables on the window of grid offsets (built once per grid+metric, FP64 on the host).
//
// The squared distance between an input element h = (x, theta_i) and an output
// element g = (x + d, theta_o) is rho_b(h^-1 g)^2 (Section 4.3, eqs. (rhob) and
// (logcomp)), with h^-1 g = (R_{-theta_i} d, theta_o - theta_i) from the group law
// of Section 2.3 and the angle taken in [-pi, pi).  The kernel is
// K = exp(-rho_b^2 / eps) (Section 4.2; Appendix A).
#include <cmath>
#include <cstring>

#include "se2_internal.h"

namespace se2 {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Angle representative in [-pi, pi).
double small_angle(double t) {
    double r = std::fmod(t + kPi, 2.0 * kPi);
    if (r < 0.0) r += 2.0 * kPi;
    return r - kPi;
}

// rho_b^2 of the group element (u, v, a): half-angle coordinates, weighted squares.
double rho_b_sq(double u, double v, double a, double w1, double w2, double w3) {
    const double t = small_angle(a);
    const double ch = std::cos(0.5 * t), sh = std::sin(0.5 * t);
    const double b1 = ch * u + sh * v;
    const double b2 = ch * v - sh * u;
    return w1 * w1 * b1 * b1 + w2 * w2 * b2 * b2 + w3 * w3 * t * t;
}

// Round a non-negative double to the nearest bfloat16 (ties to even), returning the bit pattern.
uint16_t to_bf16_rne(double x) {
    if (!(x > 0.0)) return 0;
    if (x >= 3.3895313892515355e38) return 0x7f7f;  // largest finite bfloat16 (not reached: K <= 1)
    int ex = 0;
    std::frexp(x, &ex);                        // x = f * 2^ex, f in [0.5, 1)
    double q = std::ldexp(1.0, ex - 8);         // 8 significant bits
    const double qmin = std::ldexp(1.0, -133);  // subnormal quantum
    if (q < qmin) q = qmin;
    const double r = std::nearbyint(x / q);     // ties to even in the default rounding mode
    const float y = static_cast<float>(r * q);  // exact: r * q is a bfloat16 value
    uint32_t bits;
    std::memcpy(&bits, &y, 4);
    return static_cast<uint16_t>(bits >> 16);
}

}  // namespace

int build_tables(Kernel &k) {
    const int nt = k.grid.ntheta, R = k.metric.radius, W = 2 * R + 1;
    const double period = k.grid.theta_axial ? kPi : 2.0 * kPi;
    const double w1 = k.metric.w1, w2 = k.metric.w2, w3 = k.metric.w3, eps = k.metric.eps;
    k.W = W;
    k.entries = static_cast<size_t>(W) * W * nt * nt;
    k.logk.assign(k.entries, 0.0);
    k.cost.assign(k.entries, 0.0);
    std::vector<double> L2(k.entries), K64(k.entries);
    std::vector<float> L32(k.entries), K32(k.entries);
    std::vector<uint16_t> Kb(k.entries);
    std::vector<double> cosi(nt), sini(nt);
    for (int i = 0; i < nt; ++i) {
        cosi[i] = std::cos(period * i / nt);
        sini[i] = std::sin(period * i / nt);
    }
    int nz = 0;
    for (int dy = -R; dy <= R; ++dy) {
        for (int dx = -R; dx <= R; ++dx) {
            bool any = false;
            for (int ko = 0; ko < nt; ++ko) {
                for (int ki = 0; ki < nt; ++ki) {
                    // relative element h^-1 g: rotate the offset by -theta_i
                    const double u = cosi[ki] * dx + sini[ki] * dy;
                    const double v = cosi[ki] * dy - sini[ki] * dx;
                    const double a = period * (ko - ki) / nt;
                    double d2 = rho_b_sq(u, v, a, w1, w2, w3);
                    if (k.grid.theta_axial) {
                        const double d2h = rho_b_sq(u, v, a + kPi, w1, w2, w3);
                        if (d2h < d2) d2 = d2h;
                    }
                    const size_t idx = ((static_cast<size_t>(dy + R) * W + (dx + R)) * nt + ko) * nt + ki;
                    k.cost[idx] = d2;
                    k.logk[idx] = -d2 / eps;
                    L2[idx] = k.logk[idx] * kLog2e;
                    L32[idx] = static_cast<float>(L2[idx]);
                    K64[idx] = std::exp(k.logk[idx]);
                    K32[idx] = static_cast<float>(K64[idx]);
                    Kb[idx] = to_bf16_rne(K64[idx]);
                    any = any || Kb[idx] != 0;
                }
            }
            nz += any ? 1 : 0;
        }
    }
    k.nonzero_bf16 = nz;
    const size_t e = k.entries;
    SE2_HIP(hipMalloc(&k.d_L64, e * sizeof(double)));
    SE2_HIP(hipMalloc(&k.d_L32, e * sizeof(float)));
    SE2_HIP(hipMalloc(&k.d_cost32, e * sizeof(float)));
    SE2_HIP(hipMalloc(&k.d_K32, e * sizeof(float)));
    SE2_HIP(hipMalloc(&k.d_Kbf16, e * sizeof(uint16_t)));
    SE2_HIP(hipMalloc(&k.d_K64, e * sizeof(double)));
    const std::vector<uint16_t> Bp = pack_bf16_operand(Kb, nt, R);
    SE2_HIP(hipMalloc(&k.d_Bpack, Bp.size() * sizeof(uint16_t)));
    SE2_HIP(hipMemcpy(k.d_Bpack, Bp.data(), Bp.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    const std::vector<float> Fp = pack_f32_operand(K32, nt, R);
    if (!Fp.empty()) {
        SE2_HIP(hipMalloc(&k.d_Fpack, Fp.size() * sizeof(float)));
        SE2_HIP(hipMemcpy(k.d_Fpack, Fp.data(), Fp.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    SE2_HIP(hipMemcpy(k.d_L64, L2.data(), e * sizeof(double), hipMemcpyHostToDevice));
    SE2_HIP(hipMemcpy(k.d_L32, L32.data(), e * sizeof(float), hipMemcpyHostToDevice));
    const std::vector<float> C32(k.cost.begin(), k.cost.end());
    SE2_HIP(hipMemcpy(k.d_cost32, C32.data(), e * sizeof(float), hipMemcpyHostToDevice));
    SE2_HIP(hipMemcpy(k.d_K32, K32.data(), e * sizeof(float), hipMemcpyHostToDevice));
    SE2_HIP(hipMemcpy(k.d_Kbf16, Kb.data(), e * sizeof(uint16_t), hipMemcpyHostToDevice));
    SE2_HIP(hipMemcpy(k.d_K64, K64.data(), e * sizeof(double), hipMemcpyHostToDevice));
    return SE2_OK;
}

}  // namespace se2
