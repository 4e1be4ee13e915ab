// mfma_probe.hip -- dense bf16 matrix-core throughput of one gfx950 GPU:
// v_mfma_f32_16x16x32_bf16 (the surrogate's inference instruction),
// v_mfma_f32_16x16x16bf16_1k (its training instruction) and
// v_mfma_f32_32x32x16_bf16, each wave issuing 8 independent accumulator chains,
// 4 (or 8) waves per SIMD on every CU.  Reports TFLOP/s (2 M N K per wave
// instruction) next to the wave clock.  Not
// part of the library; build and run with
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         paper_2605_01536_amd/csrc/probe/mfma_probe.hip -o /tmp/mfma_probe && /tmp/mfma_probe
#include <hip/hip_runtime.h>
#include <cstdio>

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kChains = 8;
constexpr int kChains32 = 4;   // 32x32 accumulators are 16 registers each

template <int OP>
__global__ __launch_bounds__(256) void k(float* out, long long* clk, int iters) {
    v4f acc[kChains];
    for (int c = 0; c < kChains; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
    v8bf a8, b8;
    v4s a4, b4;
    for (int e = 0; e < 8; ++e) {
        a8[e] = (__bf16)(0.001f * (threadIdx.x + e));
        b8[e] = (__bf16)(0.002f * (threadIdx.x - e));
    }
    for (int e = 0; e < 4; ++e) {
        a4[e] = (short)(threadIdx.x + e);
        b4[e] = (short)(threadIdx.x * 3 + e);
    }
    const long long c0 = clock64(), w0 = wall_clock64();
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if (OP == 0) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a8, b8, acc[c], 0, 0, 0);
            if (OP == 1) acc[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a4, b4, acc[c], 0, 0, 0);
        }
    }
    const long long c1 = clock64(), w1 = wall_clock64();
    float s = 0.f;
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        clk[0] = c1 - c0;
        clk[1] = w1 - w0;
    }
}

__global__ __launch_bounds__(256) void k32(float* out, long long* clk, int iters) {
    v16f acc[kChains32];
    for (int c = 0; c < kChains32; ++c)
        for (int e = 0; e < 16; ++e) acc[c][e] = 0.f;
    v8bf a8, b8;
    for (int e = 0; e < 8; ++e) {
        a8[e] = (__bf16)(0.001f * (threadIdx.x + e));
        b8[e] = (__bf16)(0.002f * (threadIdx.x - e));
    }
    const long long c0 = clock64(), w0 = wall_clock64();
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains32; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, b8, acc[c], 0, 0, 0);
    }
    const long long c1 = clock64(), w1 = wall_clock64();
    float s = 0.f;
    for (int c = 0; c < kChains32; ++c)
        for (int e = 0; e < 16; ++e) s += acc[c][e];
    out[blockIdx.x * 256 + threadIdx.x] = s;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        clk[0] = c1 - c0;
        clk[1] = w1 - w0;
    }
}

typedef void (*KF)(float*, long long*, int);

int main() {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, 0) != hipSuccess) return 1;
    const int ncu = prop.multiProcessorCount;
    const int blocks = ncu * 8, iters = 20000;   // output room for up to 8 waves per SIMD
    printf("device %s, %d CUs, max clock %d MHz\n", prop.name, ncu, prop.clockRate / 1000);
    float* o;
    long long* clk;
    if (hipMalloc(&o, sizeof(float) * blocks * 256) != hipSuccess) return 1;
    if (hipMalloc(&clk, sizeof(long long) * 2) != hipSuccess) return 1;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    struct Case {
        const char* name;
        KF fn;
        double flop;   // per wave instruction
        int per_simd;  // resident waves per SIMD
        int chains;    // instructions per iteration
    };
    const Case cases[] = {{"mfma_f32_16x16x32_bf16", k<0>, 2.0 * 16 * 16 * 32, 4, kChains},
                          {"mfma_f32_16x16x32_bf16", k<0>, 2.0 * 16 * 16 * 32, 8, kChains},
                          {"mfma_f32_16x16x16bf16_1k", k<1>, 2.0 * 16 * 16 * 16, 4, kChains},
                          {"mfma_f32_32x32x16_bf16", k32, 2.0 * 32 * 32 * 16, 2, kChains32},
                          {"mfma_f32_32x32x16_bf16", k32, 2.0 * 32 * 32 * 16, 4, kChains32}};
    for (const Case& cs : cases) {
        const int nb = ncu * cs.per_simd;   // blocks of 4 waves: per_simd waves on each SIMD
        if (nb > blocks) continue;
        for (int rep = 0; rep < 3; ++rep) {
            (void)hipEventRecord(e0);
            cs.fn<<<nb, 256>>>(o, clk, iters);
            (void)hipEventRecord(e1);
            (void)hipEventSynchronize(e1);
            float ms;
            (void)hipEventElapsedTime(&ms, e0, e1);
            long long hc[2];
            (void)hipMemcpy(hc, clk, sizeof(hc), hipMemcpyDeviceToHost);
            const double flop = (double)nb * 4 * iters * cs.chains * cs.flop;
            if (rep == 2)
                printf("%-26s %d waves/SIMD %8.3f ms  %7.1f TFLOP/s  (wave clock %.2f GHz)\n", cs.name, cs.per_simd, ms,
                       flop / (ms * 1e-3) / 1e12, hc[0] / (hc[1] * 10.0));
        }
    }
    printf("status %s\n", hipGetErrorString(hipDeviceSynchronize()));
    return 0;
}
