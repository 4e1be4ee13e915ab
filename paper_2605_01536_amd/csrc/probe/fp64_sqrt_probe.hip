// fp64_sqrt_probe.hip -- accuracy of gfx950's v_sqrt_f64, v_rsq_f64, v_rcp_f64 (raw
// hardware approximations) against the correctly rounded library sqrt, on
// 2^20 log-uniform arguments in [1e-12, 1e12], and of refinements built on
// them.  Prints the maximum error in units in the last place.  Not part of
// the library; build and run with
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         paper_2605_01536_amd/csrc/probe/fp64_sqrt_probe.hip -o /tmp/fp64_sqrt_probe && /tmp/fp64_sqrt_probe
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

constexpr int kN = 1 << 20;

__global__ void k_eval(const double* __restrict__ x, double* __restrict__ out, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double v = x[i];
    const double s = __builtin_amdgcn_sqrt(v);
    const double r = __builtin_amdgcn_rsq(v);
    // one Newton correction of the hardware square root: s + (v - s^2) / (2 s)
    const double h = 0.5 * __builtin_amdgcn_rcp(s);
    const double s1 = fma(fma(-s, s, v), h, s);
    // from the reciprocal square root: s0 = v r, one correction with h = r / 2
    const double y0 = v * r, hr = 0.5 * r;
    const double y1 = fma(fma(-y0, y0, v), hr, y0);
    // Goldschmidt: refine y and h together once, then the final correction
    const double g = fma(-y0, hr, 0.5);
    const double y2 = fma(y0, g, y0), h2 = fma(hr, g, hr);
    const double y3 = fma(fma(-y2, y2, v), h2, y2);
    // reciprocal: v_rcp_f64 with one and with two Newton steps
    const double q0 = __builtin_amdgcn_rcp(v);
    const double q1 = fma(q0, fma(-v, q0, 1.0), q0);
    const double q2 = fma(q1, fma(-v, q1, 1.0), q1);
    out[8 * i + 6] = q1;
    out[8 * i + 7] = q2;
    out[8 * i] = s;
    out[8 * i + 1] = r;
    out[8 * i + 2] = s1;
    out[8 * i + 3] = ::sqrt(v);
    out[8 * i + 4] = y1;
    out[8 * i + 5] = y3;
}

static double ulps(double a, double ref) { return std::fabs(a - ref) / (std::nextafter(ref, INFINITY) - ref); }

int main() {
    std::vector<double> hx(kN), ho(8 * (size_t)kN);
    unsigned long long st = 0x9e3779b97f4a7c15ull;
    for (int i = 0; i < kN; ++i) {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        const double u = (double)(st >> 11) * 0x1.0p-53;
        hx[i] = std::pow(10.0, -12.0 + 24.0 * u);
    }
    double *dx, *dout;
    if (hipMalloc(&dx, sizeof(double) * kN) != hipSuccess) return 1;
    if (hipMalloc(&dout, sizeof(double) * 8 * kN) != hipSuccess) return 1;
    (void)hipMemcpy(dx, hx.data(), sizeof(double) * kN, hipMemcpyHostToDevice);
    k_eval<<<kN / 256, 256>>>(dx, dout, kN);
    (void)hipMemcpy(ho.data(), dout, sizeof(double) * 8 * kN, hipMemcpyDeviceToHost);
    double e_sqrt = 0, e_rsq = 0, e_ref = 0, e_lib = 0, e_y1 = 0, e_y3 = 0, e_q1 = 0, e_q2 = 0;
    for (int i = 0; i < kN; ++i) {
        const double ref = std::sqrt(hx[i]);
        e_sqrt = std::fmax(e_sqrt, ulps(ho[8 * i], ref));
        e_rsq = std::fmax(e_rsq, ulps(ho[8 * i + 1], 1.0 / ref));
        e_ref = std::fmax(e_ref, ulps(ho[8 * i + 2], ref));
        e_lib = std::fmax(e_lib, ulps(ho[8 * i + 3], ref));
        e_y1 = std::fmax(e_y1, ulps(ho[8 * i + 4], ref));
        e_y3 = std::fmax(e_y3, ulps(ho[8 * i + 5], ref));
        e_q1 = std::fmax(e_q1, ulps(ho[8 * i + 6], 1.0 / hx[i]));
        e_q2 = std::fmax(e_q2, ulps(ho[8 * i + 7], 1.0 / hx[i]));
    }
    printf("max ulp: v_sqrt_f64 %.3g  v_rsq_f64 %.3g (vs 1/sqrt rounded)  v_sqrt_f64+1 Newton %.3g  library %.3g\n",
           e_sqrt, e_rsq, e_ref, e_lib);
    printf("max ulp: v_rsq_f64 + 1 correction %.3g  v_rsq_f64 + Goldschmidt step + correction %.3g\n", e_y1, e_y3);
    printf("max ulp: v_rcp_f64 + 1 Newton %.3g  + 2 Newton %.3g (vs 1/x rounded)\n", e_q1, e_q2);
    printf("status %s\n", hipGetErrorString(hipDeviceSynchronize()));
    return 0;
}
