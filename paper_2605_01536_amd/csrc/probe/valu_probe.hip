// valu_probe.hip -- VALU issue cost of the instruction classes the boundary
// kernels use (FP32 and FP64), measured as the time of 16 independent dependency chains per
// lane relative to v_fma_f32 in the same launch shape.  Also reports the shader
// clock of one wave (clock64 against the 100 MHz wall clock).  Not part of the
// library; build and run with
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         paper_2605_01536_amd/csrc/probe/valu_probe.hip -o /tmp/valu_probe && /tmp/valu_probe
#include <hip/hip_runtime.h>
#include <cstdio>

#define CH 16
template <int OP>
__global__ __launch_bounds__(256) void k(float* out, long long* clk, int iters, float seed) {
    float a[CH];
    int b[CH];
    for (int c = 0; c < CH; ++c) {
        a[c] = seed + threadIdx.x * 1e-3f + c;
        b[c] = threadIdx.x * 7 + c;
    }
    const long long c0 = clock64(), w0 = wall_clock64();
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (OP == 0) a[c] = __builtin_fmaf(a[c], 0.999f, 1e-3f);                       // v_fma_f32
            if (OP == 1) a[c] = a[c] * 0.999f;                                             // v_mul_f32
            if (OP == 2) a[c] = a[c] + 1e-3f;                                              // v_add_f32
            if (OP == 3) a[c] = __builtin_amdgcn_sqrtf(a[c]);                              // v_sqrt_f32
            if (OP == 4) a[c] = __builtin_amdgcn_rcpf(a[c]);                               // v_rcp_f32
            if (OP == 5) b[c] = b[c] - (int)threadIdx.x;                                   // v_sub_u32
            if (OP == 6) a[c] = (a[c] > 1.5f) ? a[c] * 0.5f : a[c] * 1.001f;               // cmp + mul + cndmask
            if (OP == 7) { b[c] += 3; a[c] = __builtin_fmaf(a[c], 0.5f, (float)b[c]); }     // add_u32 + cvt + fma
            if (OP == 8) a[c] = fminf(a[c] * 1.001f, 3.0f);                                // mul + min
        }
    }
    const long long c1 = clock64(), w1 = wall_clock64();
    float s = 0;
    for (int c = 0; c < CH; ++c) s += a[c] + (float)b[c];
    out[blockIdx.x * 256 + threadIdx.x] = s;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        clk[0] = c1 - c0;
        clk[1] = w1 - w0;
    }
}

// the same in FP64 (the all-FP64 boundary path): v_fma_f64, v_mul_f64,
// v_add_f64, v_rcp_f64, the library square root and v_sqrt_f64
template <int OP>
__global__ __launch_bounds__(256) void kd(float* out, long long* clk, int iters, float seed) {
    double a[CH];
    for (int c = 0; c < CH; ++c) a[c] = seed + threadIdx.x * 1e-3 + c;
    const long long c0 = clock64(), w0 = wall_clock64();
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (OP == 0) a[c] = __builtin_fma(a[c], 0.999, 1e-3);
            if (OP == 1) a[c] = a[c] * 0.999;
            if (OP == 2) a[c] = a[c] + 1e-3;
            if (OP == 3) a[c] = __builtin_amdgcn_rcp(a[c]);
            if (OP == 4) a[c] = ::sqrt(a[c]);
            if (OP == 5) a[c] = __builtin_amdgcn_sqrt(a[c]);
        }
    }
    const long long c1 = clock64(), w1 = wall_clock64();
    double s = 0;
    for (int c = 0; c < CH; ++c) s += a[c];
    out[blockIdx.x * 256 + threadIdx.x] = (float)s;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        clk[0] = c1 - c0;
        clk[1] = w1 - w0;
    }
}

typedef void (*KF)(float*, long long*, int, float);

int main() {
    const int blocks = 256 * 8, iters = 4000;
    float* o;
    long long* clk;
    if (hipMalloc(&o, sizeof(float) * blocks * 256) != hipSuccess) return 1;
    if (hipMalloc(&clk, sizeof(long long) * 2) != hipSuccess) return 1;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const char* names[] = {"fma_f32", "mul_f32", "add_f32", "sqrt_f32", "rcp_f32", "sub_u32",
                           "cmp+mul+cndmask", "add_u32+cvt+fma", "mul+min", "fma_f64", "mul_f64",
                           "add_f64", "rcp_f64", "sqrt_f64 (library)", "v_sqrt_f64"};
    KF ks[] = {k<0>, k<1>, k<2>, k<3>, k<4>, k<5>, k<6>, k<7>, k<8>, kd<0>, kd<1>, kd<2>, kd<3>, kd<4>, kd<5>};
    float base = 0;
    for (int op = 0; op < 15; ++op) {
        for (int rep = 0; rep < 3; ++rep) {
            (void)hipEventRecord(e0);
            ks[op]<<<blocks, 256>>>(o, clk, iters, 1.f);
            (void)hipEventRecord(e1);
            (void)hipEventSynchronize(e1);
            float ms;
            (void)hipEventElapsedTime(&ms, e0, e1);
            long long hc[2];
            (void)hipMemcpy(hc, clk, sizeof(hc), hipMemcpyDeviceToHost);
            if (op == 0 && rep == 2) base = ms;
            if (rep == 2)
                printf("%-18s %7.3f ms  %.3e lane-iterations/s  %.2f x fma  (wave clock %.2f GHz)\n", names[op], ms,
                       (double)blocks * 256 * iters * CH / (ms * 1e-3), ms / base, hc[0] / (hc[1] * 10.0));
        }
    }
    printf("status %s\n", hipGetErrorString(hipDeviceSynchronize()));
    return 0;
}
