// mlp.hip -- learned surrogate for far-field winding-number queries:
// Fourier features gamma(p) = [sin 2piGp, cos 2piGp] (G: 32x3, fixed), four
// GELU layers 64->128->128->128->128 and a linear output 128->1.  Every matrix
// product of training runs on v_mfma_f32_32x32x16_bf16 (bf16 operands, fp32
// accumulation) in a transposed fragment layout where one layer's output registers are the
// next layer's operand: inference (k_infer) keeps the activations in
// registers; training runs the forward and backward passes in one kernel
// (k_tfb) and the weight gradients in another (k_twgrad).
// Inference runs its products on v_mfma_f32_32x32x16_f16 with half-precision
// activations and evaluates GELU by a minimax polynomial of Phi in packed half
// arithmetic (gelu_half2, within 2.4e-3 |z| of the erf form); training uses the
// erf form (Abramowitz & Stegun 7.1.26, 1.5e-7) on bf16 operands, which the
// inference kernel keeps as an option (GWN_INFER_GELU=erf).  FP32 master weights are updated by Adam and re-packed into
// the bf16 copies the kernels read.  The band query evaluates the network,
// re-evaluates every point whose prediction lies within `band` of 1/2 with the
// exact kernels, and scatters those results back.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "gwn_alloc.h"
#include "gwn_kernels.h"
#include "gwn_mesh.h"

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

namespace gwn {
namespace mlp {

constexpr int kFreq = 32, kIn = 64, kHid = 128;
constexpr int kNParams = 64 * 128 + 128 + 3 * (128 * 128 + 128) + 128 + 1;   // 57985
constexpr int kOffW[5] = {0, 8320, 24832, 41344, 57856};
constexpr int kOffB[5] = {8192, 24704, 41216, 57728, 57984};
// the same offsets as arithmetic, for run-time layer indices (a constant table
// indexed at run time would live in scratch memory)
__host__ __device__ constexpr int off_w(int l) { return l == 0 ? 0 : 8320 + (l - 1) * 16512; }
__host__ __device__ constexpr int off_b(int l) { return l == 4 ? 57984 : off_w(l) + (l == 0 ? 64 : 128) * 128; }
static_assert(off_w(0) == kOffW[0] && off_w(1) == kOffW[1] && off_w(2) == kOffW[2] && off_w(3) == kOffW[3] &&
              off_w(4) == kOffW[4], "weight offsets");
static_assert(off_b(0) == kOffB[0] && off_b(1) == kOffB[1] && off_b(2) == kOffB[2] && off_b(3) == kOffB[3] &&
              off_b(4) == kOffB[4], "bias offsets");
constexpr int kWf = 128 * 64 + 3 * 128 * 128 + 128;   // forward bf16 copy: Wt0..Wt3 ([out][in]) + w4
constexpr int kWb = 3 * 128 * 128;                    // backward copy: W1..W3 as MFMA A fragments
constexpr int kWi = 128 * 64 + 3 * 128 * 128;         // inference copy: W0..W3 as MFMA A fragments

struct Dev {
    float* master;   // kNParams
    float* m;        // Adam first moment
    float* v;        // Adam second moment
    float* G;        // 96
    unsigned short* wf;
    unsigned short* wb;
    unsigned short* wi;
    unsigned short* wh;   // the inference copy in half precision (same layout as wi)
};

struct Train {
    unsigned short* x;   // X: tiles x 36 K-blocks (fragment layout, bf16)
    unsigned short* dz;  // DZ: tiles x 32 K-blocks
    float* y;            // tiles x 32
    float* dy;           // tiles x 32: dL/dy, 0 beyond the batch
    float* tb;           // tiles x 32: the batch's targets, in batch order
    float* part;         // nchunk x (kNParams + 1)   (last entry: sum of (dL/dy)^2)
    float* grad;         // kNParams + 1
    long long cap;       // points (a multiple of 32)
};

__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
// half-precision bits of a bf16 weight: exact for |w| in [2^-14, 65504] (8
// significant bits into 11), rounded into the subnormals below, saturated above;
// a NaN stays NaN (so a diverged network reads NaN on both inference paths)
__device__ __forceinline__ unsigned short w2h(float w) {
    const float c = fabsf(w) > 65504.0f ? copysignf(65504.0f, w) : w;
    return __builtin_bit_cast(unsigned short, (_Float16)c);
}

// splitmix64's output function (Steele, Lea and Flood 2014): a bijective 64-bit
// mix.  Applied to a counter it is the splitmix64 generator; here it also
// drives the shuffle's round function and the training points.
__host__ __device__ inline unsigned long long smix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
constexpr unsigned long long kGolden = 0x9E3779B97F4A7C15ull;

// Where the rows of a training batch come from: row r is source point
// order(off + r), where order is the identity (half == 0) or a keyed random
// permutation of [0, ntot): a 4-round Feistel network on 2*half bits with
// cycle walking (re-apply until the value falls below ntot; the walk stays on
// the cycle of a bijection, so it ends, after fewer than 4 rounds on average
// since 2^(2 half) < 4 ntot).  Every epoch draws a new key.
struct Src {
    const float* qx;
    const float* qy;
    const float* qz;
    long long qs;
    const float* tgt;
    long long off;
    long long ntot;
    unsigned long long key;
    int half;
};

__host__ __device__ inline long long src_index(const Src& s, long long i) {
    if (s.half == 0) return i;
    const unsigned mask = (1u << s.half) - 1u;
    unsigned long long x = (unsigned long long)i;
    do {
        unsigned L = (unsigned)(x >> s.half), R = (unsigned)x & mask;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const unsigned F = (unsigned)smix64(s.key + (unsigned long long)(r + 1) * kGolden + R) & mask;
            const unsigned nr = L ^ F;
            L = R;
            R = nr;
        }
        x = ((unsigned long long)L << s.half) | R;
    } while (x >= (unsigned long long)s.ntot);
    return (long long)x;
}

// half-width of the shuffle's Feistel network for n points (2 half >= log2 n)
inline int shuffle_half(long long n) {
    int b = 1;
    while (b < 62 && (1ll << b) < n) ++b;
    return (b + 1) / 2;
}

// Training points: coordinate c of point i is lo_c + u (hi_c - lo_c) with
// u = (top 53 bits of splitmix64 at counter 3 i + c + 1) / 2^53, in FP64, rounded once.
__global__ void k_gen_points(unsigned long long seed, long long n, double lx, double ly, double lz, double ex,
                             double ey, double ez, float* __restrict__ X) {
    const long long i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= n) return;
    const double lo[3] = {lx, ly, lz}, ext[3] = {ex, ey, ez};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const unsigned long long h = smix64(seed + (unsigned long long)(3 * i + c + 1) * kGolden);
        const double u = (double)(h >> 11) * (1.0 / 9007199254740992.0);
        X[3 * i + c] = (float)(lo[c] + u * ext[c]);
    }
}

// erf by Abramowitz & Stegun 7.1.26 (|error| <= 1.5e-7); returns Phi(z) and
// exp(-z^2/2) so that gelu = z Phi and gelu' = Phi + z exp(-z^2/2)/sqrt(2 pi).
__device__ __forceinline__ void gelu_parts(float z, float& phi, float& e) {
    const float x = fabsf(z) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
    e = __builtin_amdgcn_exp2f(-x * x * 1.4426950408889634f);
    float p = fmaf(1.061405429f, t, -1.453152027f);
    p = fmaf(p, t, 1.421413741f);
    p = fmaf(p, t, -0.284496736f);
    p = fmaf(p, t, 0.254829592f);
    p *= t;
    const float erfa = fmaf(-p, e, 1.0f);
    phi = 0.5f + 0.5f * copysignf(erfa, z);
}
__device__ __forceinline__ float gelu(float z) {
    float phi, e;
    gelu_parts(z, phi, e);
    return z * phi;
}

// Inference GELU in packed half precision, two activations per instruction:
// t = z / (2c) + 1/2 clamped to [0, 1] (the FMA's output clamp), u = 2t - 1 =
// clamp(z / c, -1, 1), Phi(z) - 1/2 = u Q(u^2), GELU = z (u Q(u^2) + 1/2).  Q of
// degree 4 for c = 3.5 (kGeluHC), a minimax fit rounded to half-precision
// coefficients one at a time with the rest re-fitted (gen_gelu_poly.py 4 3.5):
// |Phi error| <= 1.2e-3 in exact arithmetic, 2.4e-3 as evaluated here, plus
// the clamp's 2.3e-4 beyond c -- the size of the bf16 rounding of an
// activation (2^-9 to 2^-8 relative).  10 VALU instructions per pair of
// activations (conversion, clamp, 2t - 1, square, four FMAs, the 1/2 term, the
// product) against 11.5 per activation for a degree-7 polynomial in float32.
// NaN stays NaN (the product with z); pre-activations beyond the half range
// (|z| > 65504) become infinite.
constexpr float kGeluHC = 3.5f;
constexpr float kGeluH[] = {0.900390625f, -2.86328125f, 3.705078125f, -2.62890625f, 1.3876953125f};
__device__ __forceinline__ h2 hsplat(float a) { return (h2){(_Float16)a, (_Float16)a}; }
__device__ __forceinline__ h2 gelu_half2(float a, float b) {
    const h2 z = (h2){(_Float16)a, (_Float16)b};   // one v_cvt_pk_f16_f32 (round to nearest even)
    const h2 t = __builtin_elementwise_min(
        __builtin_elementwise_max(__builtin_elementwise_fma(z, hsplat(0.5f / kGeluHC), hsplat(0.5f)), hsplat(0.0f)),
        hsplat(1.0f));
    const h2 u = __builtin_elementwise_fma(t, hsplat(2.0f), hsplat(-1.0f));
    const h2 v = u * u;
    h2 q = hsplat(kGeluH[0]);
#pragma unroll
    for (int i = 1; i < 5; ++i) q = __builtin_elementwise_fma(q, v, hsplat(kGeluH[i]));
    return z * __builtin_elementwise_fma(u, q, hsplat(0.5f));
}

// Sum of the chunks' partial gradients of parameter p: four running sums
// (chunk c goes to sum c % 4), sixteen loads in flight per round
__device__ __forceinline__ float chunk_sum(const float* __restrict__ part, int nchunk, int p) {
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    int c = 0;
    for (; c + 16 <= nchunk; c += 16) {
        float r[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) r[k] = part[(long long)(c + k) * (kNParams + 1) + p];
#pragma unroll
        for (int k = 0; k < 16; ++k) s[k & 3] += r[k];
    }
    for (; c + 4 <= nchunk; c += 4)
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] += part[(long long)(c + k) * (kNParams + 1) + p];
    for (; c < nchunk; ++c) s[0] += part[(long long)c * (kNParams + 1) + p];
    return (s[0] + s[1]) + (s[2] + s[3]);
}

__global__ void k_reduce(const float* __restrict__ part, int nchunk, float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNParams) return;
    grad[p] = chunk_sum(part, nchunk, p);
}

// Copy n16 16-byte words from global memory to LDS with NT threads, eight
// loads in flight per thread (a plain loop waits out every load in turn).
template <int NT>
__device__ __forceinline__ void stage_lds(uint4* __restrict__ dst, const uint4* __restrict__ src, int n16) {
    for (int base = threadIdx.x; base < n16; base += NT * 8) {
        uint4 r[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (base + k * NT < n16) r[k] = src[base + k * NT];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (base + k * NT < n16) dst[base + k * NT] = r[k];
    }
}

// ---- inference: the activations never leave registers
//
// Each hidden layer is computed transposed, H_out^T = W^T H_in^T, with
// v_mfma_f32_32x32x16_f16 (or its bf16 twin, which has the same operand
// layout): A = 32 output features x 16 input features of the
// weights, B = 16 input features x 32 points of the activations, D = 32 output
// features x 32 points.  Operand layout (wave64): lane l holds A[l%32][8(l/32)+i]
// and B[8(l/32)+i][l%32] (i = 0..7); D[8j + 4(l/32) + i][l%32] lands in
// accumulator component 4j + i (j, i = 0..3).  Which input feature sits in B
// slot (h = l/32, i) of K-block kb is free as long as A agrees, so the hidden
// layers number them
//   kappa(kb, h, i) = 16 kb + 8 (i / 4) + 4 h + i % 4,
// which makes a lane's accumulator components 0..7 of output tile T its B
// fragment of K-block 2T and components 8..15 that of K-block 2T+1: one layer's
// output is the next layer's operand without any data movement.  The Fourier
// features use kappa0(b, h, i) = 32 (b / 2) + 16 h + 8 (b % 2) + i (K-blocks 0
// and 1: sines, 2 and 3: cosines; lane half h computes frequencies 16h..16h+15
// of its point).  The weights are packed once per update into these A
// fragments, 16 bytes per lane, in the order the kernel reads them; the bias
// enters as the accumulator input of each output tile's first product.
__host__ __device__ inline int infer_slot(int l, int k, int o) {
    int kb, h, i;
    if (l == 0) {
        const int r = k % 32;
        kb = 2 * (k / 32) + (r % 16) / 8;
        h = r / 16;
        i = r % 8;
    } else {
        const int r = k % 16;
        kb = k / 16;
        h = (r % 8) / 4;
        i = 4 * (r / 8) + r % 4;
    }
    const int nkb = l == 0 ? 4 : 8;
    const int base = l == 0 ? 0 : 8192 + (l - 1) * 16384;
    const int frag = (o / 32) * nkb + kb, lane = o % 32 + 32 * h;
    return base + (frag * 64 + lane) * 8 + i;
}

// input feature held in slot i of K-block kb by lane half h (hidden layers)
__device__ __forceinline__ int kappa(int kb, int h, int i) { return 16 * kb + 8 * (i >> 2) + 4 * h + (i & 3); }

typedef float v16f __attribute__((ext_vector_type(16)));

// sin(2 pi t) and cos(2 pi t) from the hardware sine and cosine, which take
// their argument in revolutions, after reducing t to its fractional part
__device__ __forceinline__ void sincos_rev(float t, float& s, float& c) {
    const float f = __builtin_amdgcn_fractf(t);
    s = __builtin_amdgcn_sinf(f);
    c = __builtin_amdgcn_cosf(f);
}

__device__ __forceinline__ v16f mfma32(const v8bf& a, const v8bf& b, const v16f& c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v16f mfma32(const v8h& a, const v8h& b, const v16f& c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// One layer for NT tiles of 32 points: X (NKB K-blocks) -> Y (8 K-blocks).
// The output tiles are software-pipelined: the products of tile T are issued
// before the activations of tile T - 1 are evaluated, so the matrix core works
// while the vector unit evaluates GELU.
// V = v8h: half-precision operands and the packed half GELU; V = v8bf: bf16
// operands and the erf form of GELU (the training kernels' arithmetic).
template <int NKB, int NT, class V>
__device__ __forceinline__ void infer_layer(const V* __restrict__ W, const float* __restrict__ bias, int lane, int h,
                                            const V (&X)[NT][8], V (&Y)[NT][8]) {
    constexpr bool HALF = __is_same(V, v8h);
    v16f acc[2][NT];
#pragma unroll
    for (int T = 0; T <= 4; ++T) {
        // a scheduling fence per output tile: without it the scheduler hoists
        // every weight fragment of the layer and runs out of registers
        __builtin_amdgcn_sched_barrier(0);
        if (T < 4) {
            v16f b;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float4 v = *(const float4*)(bias + 32 * T + 8 * j + 4 * h);
                b[4 * j] = v.x;
                b[4 * j + 1] = v.y;
                b[4 * j + 2] = v.z;
                b[4 * j + 3] = v.w;
            }
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb) {
                const V A = W[(T * NKB + kb) * 64 + lane];
#pragma unroll
                for (int p = 0; p < NT; ++p) acc[T & 1][p] = mfma32(A, X[p][kb], kb == 0 ? b : acc[T & 1][p]);
            }
        }
        if (T > 0) {
            const int U = T - 1;
#pragma unroll
            for (int p = 0; p < NT; ++p)
#pragma unroll
                for (int e = 0; e < 16; e += 2) {
                    if constexpr (HALF) {
                        const h2 g = gelu_half2(acc[U & 1][p][e], acc[U & 1][p][e + 1]);
                        Y[p][2 * U + (e >> 3)][e & 7] = g[0];
                        Y[p][2 * U + (e >> 3)][(e & 7) + 1] = g[1];
                    } else {
                        Y[p][2 * U + (e >> 3)][e & 7] = (__bf16)gelu(acc[U & 1][p][e]);
                        Y[p][2 * U + (e >> 3)][(e & 7) + 1] = (__bf16)gelu(acc[U & 1][p][e + 1]);
                    }
                }
        }
    }
}

// NT tiles of 32 points per wave and step (each A fragment read from LDS
// serves NT tiles), NW waves per workgroup sharing one copy of the weights in
// LDS (one workgroup per CU).  POLY: half-precision operands (the wh copy of
// the weights) and the packed half GELU (gelu_half2); else bf16 operands (wi)
// and the erf form of the training kernels.
template <int NT, int NW, bool POLY>
__global__ __launch_bounds__(64 * NW) void k_infer(Dev P, const float* __restrict__ qx, const float* __restrict__ qy,
                                                   const float* __restrict__ qz, long long qs, long long n,
                                                   float* __restrict__ y) {
    constexpr int kPts = 32 * NT;   // points per wave per step
    using V = typename std::conditional<POLY, v8h, v8bf>::type;
    using E = typename std::conditional<POLY, _Float16, __bf16>::type;
    __shared__ V sWi[kWi / 8];
    __shared__ __attribute__((aligned(16))) float sB[4][128];
    __shared__ float sW4[128];
    __shared__ float sG[96];
    stage_lds<64 * NW>((uint4*)sWi, (const uint4*)(POLY ? P.wh : P.wi), kWi / 8);
    for (int i = threadIdx.x; i < 128; i += 64 * NW) {
        sW4[i] = bf2f(P.wf[8192 + 3 * 16384 + i]);
        for (int l = 0; l < 4; ++l) sB[l][i] = P.master[kOffB[l] + i];
    }
    if (threadIdx.x < 96) sG[threadIdx.x] = P.G[threadIdx.x];
    const float b4 = P.master[kOffB[4]];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, ln = lane & 31, h = lane >> 5;
    for (long long step = (long long)blockIdx.x * NW + wave; step * kPts < n; step += (long long)gridDim.x * NW) {
        V X[NT][8], Y[NT][8];
        long long pt[NT];
#pragma unroll
        for (int p = 0; p < NT; ++p) {   // Fourier features: frequencies 16h..16h+15 of point ln of tile p
            pt[p] = step * kPts + 32 * p + ln;
            const long long q = min(pt[p], n - 1);
            const float px = qx[q * qs], py = qy[q * qs], pz = qz[q * qs];
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int f = 16 * h + 8 * b + i;
                    float sn, cs;
                    sincos_rev(fmaf(sG[3 * f], px, fmaf(sG[3 * f + 1], py, sG[3 * f + 2] * pz)), sn, cs);
                    X[p][b][i] = (E)sn;
                    X[p][2 + b][i] = (E)cs;
                }
        }
        infer_layer<4, NT, V>(sWi, sB[0], lane, h, X, Y);
        infer_layer<8, NT, V>(sWi + 8192 / 8, sB[1], lane, h, Y, X);
        infer_layer<8, NT, V>(sWi + (8192 + 16384) / 8, sB[2], lane, h, X, Y);
        infer_layer<8, NT, V>(sWi + (8192 + 2 * 16384) / 8, sB[3], lane, h, Y, X);
        // output layer: each lane's 64 activations, then the two lane halves of a point
#pragma unroll
        for (int p = 0; p < NT; ++p) {
            float s = 0.f;
#pragma unroll
            for (int kb = 0; kb < 8; ++kb)
#pragma unroll
                for (int i = 0; i < 8; ++i) s = fmaf((float)X[p][kb][i], sW4[kappa(kb, h, i)], s);
            s += __shfl_xor(s, 32);
            if (h == 0 && pt[p] < n) y[pt[p]] = s + b4;
        }
    }
}
// ---- training: tiles of 32 points on the inference kernel's MFMA form
//
// The forward and backward passes compute every product as the inference
// kernel does (v_mfma_f32_32x32x16_bf16, transposed, operands in the fragment
// layout), in one kernel (k_tfb).  What the weight gradients need goes to HBM
// in the fragment layout, 16 bytes per lane and K-block (a contiguous
// kilobyte per wave and K-block):
//   X   the inputs of the five layers, bf16: the features (4 K-blocks), then
//       the four GELU outputs (8 K-blocks each)                    36 K-blocks
//   DZ  dL/dz of the four GELU layers, bf16                         32 K-blocks
// K-block kb of tile t of a tensor with nkb K-blocks per tile sits at element
// ((t nkb + kb) 64 + lane) 8; lane (n, h) holds slots i = 0..7 of point 32 t + n
// (features kappa0(kb, h, i) for the first layer's input, kappa(kb, h, i)
// otherwise).  Rows beyond the batch carry dL/dy = 0, so their terms vanish.
constexpr int kXkb = 36, kDzkb = 32;
__host__ __device__ constexpr int x_kb0(int l) { return l == 0 ? 0 : 4 + 8 * (l - 1); }

__device__ __forceinline__ void st_frag(unsigned short* base, long long t, int nkb, int kb, int lane, v8bf v) {
    *(v8bf*)(base + ((t * nkb + kb) * 64 + lane) * 8) = v;
}
__device__ __forceinline__ v8bf ld_frag(const unsigned short* base, long long t, int nkb, int kb, int lane) {
    return *(const v8bf*)(base + ((t * nkb + kb) * 64 + lane) * 8);
}

// the kappa0 feature of slot i of K-block kb for lane half h (first layer)
__host__ __device__ inline int kappa0(int kb, int h, int i) { return 32 * (kb >> 1) + 16 * h + 8 * (kb & 1) + i; }

// Backward A fragments (layers 1..3): A'[i][k] = W_l[i][o] with i an input
// feature of output tile i / 32 and o = kappa(kb, h, slot) the output feature
// in K-block kb, so dx^T = A' dz^T chains like the forward pass.
__host__ __device__ inline int bwd_slot(int l, int k, int o) {
    const int kb = o / 16, r = o % 16;
    const int h = (r % 8) / 4, i = 4 * (r / 8) + r % 4;
    return (l - 1) * 16384 + (((k / 32) * 8 + kb) * 64 + k % 32 + 32 * h) * 8 + i;
}

// One training pass over the tiles of a batch, forward and backward through
// the activations: wave q of a workgroup computes output tile q (32 features)
// of every layer of the workgroup's current tile, holding its own forward and
// backward weight fragments in registers (loaded once) and GELU'(z) of its
// features from the forward pass to the backward one.  The four waves
// exchange activations and dL/dz through LDS, one barrier per layer.  Writes
// X, DZ, y, dL/dy = 2 (y - t) / n (0 beyond the batch) and the batch targets;
// the backward pass ends at dz of the first layer (dx of the features is not
// needed).
__global__ __launch_bounds__(256) void k_tfb(Dev P, Src S, long long n, float inv_n, Train T) {
    __shared__ v8bf sX[2][8][64];   // activations, then dL/dz, ping-pong
    __shared__ float sP[4][64];     // output-layer partial sums of the four waves
    __shared__ float sDy[32];
    __shared__ __attribute__((aligned(16))) float sB[4][128];
    __shared__ float sW4[128];
    __shared__ float sG[96];
    for (int i = threadIdx.x; i < 128; i += 256) {
        sW4[i] = bf2f(P.wf[8192 + 3 * 16384 + i]);
        for (int l = 0; l < 4; ++l) sB[l][i] = P.master[kOffB[l] + i];
    }
    if (threadIdx.x < 96) sG[threadIdx.x] = P.G[threadIdx.x];
    const float b4 = P.master[kOffB[4]];
    const int lane = threadIdx.x & 63, ln = lane & 31, h = lane >> 5, q = threadIdx.x >> 6;
    // this wave's weight fragments: forward (4 + 3 x 8) and backward (3 x 8)
    const v8bf* wi = (const v8bf*)P.wi;
    const v8bf* wb = (const v8bf*)P.wb;
    v8bf Af[28], Ab[24];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) Af[kb] = wi[(q * 4 + kb) * 64 + lane];
#pragma unroll
    for (int l = 1; l < 4; ++l)
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
            Af[4 + 8 * (l - 1) + kb] = wi[(8192 + (l - 1) * 16384) / 8 + (q * 8 + kb) * 64 + lane];
            Ab[8 * (l - 1) + kb] = wb[(l - 1) * 16384 / 8 + (q * 8 + kb) * 64 + lane];
        }
    __syncthreads();
    const long long tiles = (n + 31) / 32;
    for (long long t = blockIdx.x; t < tiles; t += gridDim.x) {
        const long long row = t * 32 + ln;
        float tg;
        {   // features: wave q computes K-block q (sines for q < 2, cosines otherwise)
            const long long pi = src_index(S, S.off + min(row, n - 1));
            const float px = S.qx[pi * S.qs], py = S.qy[pi * S.qs], pz = S.qz[pi * S.qs];
            tg = S.tgt[pi];
            v8bf f;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int fr = 16 * h + 8 * (q & 1) + i;
                const float a = __builtin_amdgcn_fractf(
                    fmaf(sG[3 * fr], px, fmaf(sG[3 * fr + 1], py, sG[3 * fr + 2] * pz)));
                f[i] = (__bf16)(q < 2 ? __builtin_amdgcn_sinf(a) : __builtin_amdgcn_cosf(a));
            }
            sX[0][q][lane] = f;
            st_frag(T.x, t, kXkb, q, lane, f);
        }
        __syncthreads();
        v8bf gd[4][2];   // GELU'(z) of this wave's features, per layer
        float part = 0.f;
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int nkb = l == 0 ? 4 : 8, a0 = l == 0 ? 0 : 4 + 8 * (l - 1);
            v16f acc;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float4 v = *(const float4*)(&sB[l][32 * q + 8 * j + 4 * h]);
                acc[4 * j] = v.x;
                acc[4 * j + 1] = v.y;
                acc[4 * j + 2] = v.z;
                acc[4 * j + 3] = v.w;
            }
#pragma unroll
            for (int kb = 0; kb < nkb; ++kb)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Af[a0 + kb], sX[l & 1][kb][lane], acc, 0, 0, 0);
            v8bf y[2];
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                float phi, ex;
                gelu_parts(acc[e], phi, ex);
                y[e >> 3][e & 7] = (__bf16)(acc[e] * phi);
                gd[l][e >> 3][e & 7] = (__bf16)fmaf(acc[e] * 0.39894228040143268f, ex, phi);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                st_frag(T.x, t, kXkb, x_kb0(l + 1) + 2 * q + u, lane, y[u]);
                if (l < 3) sX[(l + 1) & 1][2 * q + u][lane] = y[u];
            }
            if (l == 3) {   // this wave's share of the output layer
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int i = 0; i < 8; ++i) part = fmaf((float)y[u][i], sW4[kappa(2 * q + u, h, i)], part);
                sP[q][lane] = part;
            }
            __syncthreads();
        }
        if (q == 0) {
            float s = sP[0][lane] + sP[1][lane] + sP[2][lane] + sP[3][lane];
            s += __shfl_xor(s, 32);
            const float yv = s + b4, dy = row < n ? 2.f * (yv - tg) * inv_n : 0.f;
            if (h == 0) {
                T.y[row] = yv;
                T.dy[row] = dy;
                T.tb[row] = tg;
                sDy[ln] = dy;
            }
        }
        __syncthreads();
        {   // dz of the last GELU layer, K-blocks 2q and 2q+1
            const float dy = sDy[ln];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int kb = 2 * q + u;
                v8bf d;
#pragma unroll
                for (int i = 0; i < 8; ++i) d[i] = (__bf16)(dy * sW4[kappa(kb, h, i)] * (float)gd[3][u][i]);
                sX[0][kb][lane] = d;
                st_frag(T.dz, t, kDzkb, 24 + kb, lane, d);
            }
        }
        __syncthreads();
        // dx_l^T = A'_l dz_l^T, then dz_{l-1} = dx_l GELU'(z_{l-1}), for l = 3, 2, 1
#pragma unroll
        for (int l = 3; l >= 1; --l) {
            const int src = (3 - l) & 1;
            v16f acc = {};
#pragma unroll
            for (int kb = 0; kb < 8; ++kb)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ab[8 * (l - 1) + kb], sX[src][kb][lane], acc, 0, 0, 0);
            v8bf d[2];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                d[0][e] = (__bf16)(acc[e] * (float)gd[l - 1][0][e]);
                d[1][e] = (__bf16)(acc[8 + e] * (float)gd[l - 1][1][e]);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                st_frag(T.dz, t, kDzkb, 8 * (l - 1) + 2 * q + u, lane, d[u]);
                if (l > 1) sX[src ^ 1][2 * q + u][lane] = d[u];
            }
            __syncthreads();
        }
    }
}

// Weight gradients dW_l[i][o] = sum over points of x_l[i] dz_l[o] (and the
// bias gradients as sums of dz) for the tiles of one chunk, on MFMA with the
// points as the contraction index.  A tensor's fragments hold points in
// lanes; one product with an identity operand transposes a pair of K-blocks
// (D = X I puts 32 features in the columns and the points in the rows of the
// result, which is the operand layout the point contraction needs).  Job
// (blockIdx.y): 0-1 the first layer's input tiles, 2-13 input tile (job - 2) % 4
// of layer (job - 2) / 4 + 1, 14 the output layer (and the loss).
__device__ __forceinline__ int xt_feature(int l, int I, int c) {
    const int kb = 2 * I + (c >> 4), r = c & 15;
    return l == 0 ? kappa0(kb, r >> 3, r & 7) : kappa(kb, r >> 3, r & 7);
}

// Four waves per workgroup take the chunk's tiles in turn and add their sums
// through LDS in a fixed order at the end.
constexpr int kWgW = 4;
__global__ __launch_bounds__(64 * kWgW) void k_twgrad(long long n, int chunk_tiles, Train T) {
    __shared__ float sAcc[kWgW - 1][68][64];   // per lane: 64 accumulator values, 4 more sums
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, c = lane & 31, kg = lane >> 5;
    const int job = blockIdx.y;
    const long long tiles = (n + 31) / 32;
    const long long ta = (long long)blockIdx.x * chunk_tiles, tb = min(tiles, ta + chunk_tiles);
    float* part = T.part + (long long)blockIdx.x * (kNParams + 1);
    v8bf ilo, ihi;   // B operands: ilo[k][n] = (k == n), ihi[k][n] = (k + 16 == n)
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        ilo[s] = (__bf16)(8 * kg + s == c ? 1.f : 0.f);
        ihi[s] = (__bf16)(8 * kg + s + 16 == c ? 1.f : 0.f);
    }
    const v16f zero = {};
    // transposed pair of K-blocks (a, b): raw fp32 values and their bf16 operands
    auto transpose = [&](const v8bf& a, const v8bf& b, v8bf (&out)[2], v16f& raw) {
        raw = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, ilo, zero, 0, 0, 0);
        raw = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b, ihi, raw, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 16; ++e) out[e >> 3][e & 7] = (__bf16)raw[e];
    };
    v16f acc[4] = {};
    float sums[4] = {0.f, 0.f, 0.f, 0.f};   // bias gradients, or sum dL/dy and sum (dL/dy)^2
    if (job < 14) {
        const int l = job < 2 ? 0 : (job - 2) / 4 + 1, I = job < 2 ? job : (job - 2) % 4;
        for (long long t = ta + wave; t < tb; t += kWgW) {
            v8bf cx[2], cd[8];
#pragma unroll
            for (int u = 0; u < 2; ++u) cx[u] = ld_frag(T.x, t, kXkb, x_kb0(l) + 2 * I + u, lane);
#pragma unroll
            for (int k = 0; k < 8; ++k) cd[k] = ld_frag(T.dz, t, kDzkb, 8 * l + k, lane);
            v8bf xt[2];
            v16f raw;
            transpose(cx[0], cx[1], xt, raw);
#pragma unroll
            for (int O = 0; O < 4; ++O) {
                v8bf dt[2];
                transpose(cd[2 * O], cd[2 * O + 1], dt, raw);
                if (I == 0)
#pragma unroll
                    for (int e = 0; e < 16; ++e) sums[O] += raw[e];
                acc[O] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xt[0], dt[0], acc[O], 0, 0, 0);
                acc[O] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xt[1], dt[1], acc[O], 0, 0, 0);
            }
        }
    } else {
        // output layer: dw4 = X_4^T dL/dy on MFMA (dL/dy in column 0 of B)
        for (long long t = ta + wave; t < tb; t += kWgW) {
            v8bf cx[8], dyb[2];
#pragma unroll
            for (int k = 0; k < 8; ++k) cx[k] = ld_frag(T.x, t, kXkb, x_kb0(4) + k, lane);
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int s = 0; s < 8; ++s)
                    dyb[u][s] = (__bf16)(c == 0 ? T.dy[t * 32 + 16 * u + 8 * (s >> 2) + 4 * kg + (s & 3)] : 0.f);
            const float d = lane < 32 ? T.dy[t * 32 + lane] : 0.f;
            sums[0] += d;
            sums[1] = fmaf(d, d, sums[1]);
#pragma unroll
            for (int I = 0; I < 4; ++I) {
                v8bf xt[2];
                v16f raw;
                transpose(cx[2 * I], cx[2 * I + 1], xt, raw);
                acc[I] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xt[0], dyb[0], acc[I], 0, 0, 0);
                acc[I] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xt[1], dyb[1], acc[I], 0, 0, 0);
            }
        }
    }
    // waves 1..3 hand their sums to wave 0, which adds them in order
    if (wave > 0) {
#pragma unroll
        for (int O = 0; O < 4; ++O) {
#pragma unroll
            for (int e = 0; e < 16; ++e) sAcc[wave - 1][16 * O + e][lane] = acc[O][e];
            sAcc[wave - 1][64 + O][lane] = sums[O];
        }
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < kWgW - 1; ++w)
#pragma unroll
        for (int O = 0; O < 4; ++O) {
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[O][e] += sAcc[w][16 * O + e][lane];
            sums[O] += sAcc[w][64 + O][lane];
        }
    // result: lane (column c, half kg) holds rows 8j + 4kg + i in component 4j + i
    if (job < 14) {
        const int l = job < 2 ? 0 : (job - 2) / 4 + 1, I = job < 2 ? job : (job - 2) % 4;
#pragma unroll
        for (int O = 0; O < 4; ++O) {
            const int fo = xt_feature(1, O, c);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int r = 8 * (e >> 2) + 4 * kg + (e & 3);
                part[off_w(l) + xt_feature(l, I, r) * 128 + fo] = acc[O][e];
            }
            if (I == 0) {
                const float s = sums[O] + __shfl_xor(sums[O], 32);
                if (kg == 0) part[off_b(l) + fo] = s;
            }
        }
    } else {
        if (c == 0)
#pragma unroll
            for (int I = 0; I < 4; ++I)
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    part[kOffW[4] + xt_feature(4, I, 8 * (e >> 2) + 4 * kg + (e & 3))] = acc[I][e];
        float sdy = sums[0], sdy2 = sums[1];
#pragma unroll
        for (int o = 16; o >= 1; o >>= 1) {
            sdy += __shfl_xor(sdy, o);
            sdy2 += __shfl_xor(sdy2, o);
        }
        if (lane == 0) {
            part[kOffB[4]] = sdy;
            part[kNParams] = sdy2;   // the host turns sum (dL/dy)^2 into the loss
        }
    }
}

// bf16 copies of one master parameter in the layouts the kernels read
__device__ __forceinline__ void pack_one(const Dev& P, int p, float w) {
    for (int l = 0; l < 4; ++l) {
        if (p >= kOffW[l] && p < kOffB[l]) {
            const int kin = l == 0 ? 64 : 128;
            const int k = (p - kOffW[l]) / 128, o = (p - kOffW[l]) % 128;
            const unsigned short b = f2bf(w);
            P.wf[(l == 0 ? 0 : 8192 + (l - 1) * 16384) + o * kin + k] = b;
            if (l >= 1) P.wb[bwd_slot(l, k, o)] = b;
            P.wi[infer_slot(l, k, o)] = b;
            P.wh[infer_slot(l, k, o)] = w2h(bf2f(b));
            return;
        }
    }
    if (p >= kOffW[4] && p < kOffB[4]) P.wf[8192 + 3 * 16384 + (p - kOffW[4])] = f2bf(w);
}

__global__ void k_pack(Dev P) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNParams) pack_one(P, p, P.master[p]);
}

// One Adam step: the chunks' partial gradients summed (as k_reduce does) and
// applied at once.  loss_slot (nullable) receives the batch's mean squared
// error, sum(dy^2) nb / 4 with dy = 2 (y - t) / nb.
__global__ void k_reduce_adam(Dev P, const float* __restrict__ part, int nchunk, float lr, float b1, float b2,
                              float eps, float c1, float c2, float* __restrict__ loss_slot, float nb) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNParams) return;
    const float g = chunk_sum(part, nchunk, p);
    if (p == kNParams) {
        if (loss_slot) *loss_slot = g * nb * 0.25f;
        return;
    }
    const float m = b1 * P.m[p] + (1.f - b1) * g;
    const float v = b2 * P.v[p] + (1.f - b2) * g * g;
    P.m[p] = m;
    P.v[p] = v;
    const float w = P.master[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    P.master[p] = w;
    pack_one(P, p, w);
}

// ---- band fallback: compaction by ballot / mbcnt, gather, scatter

// Stable two-pass compaction of the band points: per-block counts over
// contiguous segments, an exclusive scan, then each block writes its indices in
// order (one counter per block instead of one atomic per wave).
constexpr int kBandBlocks = 1024;

// rule 0: |y - 1/2| < band (the uncertain region between outside, w = 0, and
// inside, w = 1); rule 1: |frac(y) - 1/2| < band, i.e. y within band of the
// nearest half-integer (any jump between consecutive winding levels)
__device__ __forceinline__ bool in_band(const float* y, long long i, long long n, float band, int rule) {
    if (i >= n) return false;
    const float v = y[i];
    const float d = rule == 0 ? v - 0.5f : v - floorf(v) - 0.5f;
    return fabsf(d) < band;
}

__global__ __launch_bounds__(256) void k_band_count(const float* __restrict__ y, long long n, long long seg,
                                                    float band, int rule, int* __restrict__ bcnt) {
    __shared__ int wc[4];
    const long long a = blockIdx.x * seg, e = min(n, a + seg);
    int c = 0;
    for (long long i = a + threadIdx.x; i < e; i += 256) c += in_band(y, i, n, band, rule) ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) bcnt[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

// exclusive scan of the kBandBlocks counts (one block of kBandBlocks threads);
// the total goes to *count
__global__ __launch_bounds__(kBandBlocks) void k_band_scan(const int* __restrict__ bcnt, int* __restrict__ boff,
                                                          int* __restrict__ count) {
    __shared__ int sh[kBandBlocks];
    const int t = threadIdx.x;
    sh[t] = bcnt[t];
    __syncthreads();
    for (int o = 1; o < kBandBlocks; o <<= 1) {
        const int v = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    boff[t] = sh[t] - bcnt[t];
    if (t == kBandBlocks - 1) *count = sh[t];
}

__global__ __launch_bounds__(256) void k_band_write(const float* __restrict__ y, long long n, long long seg,
                                                    float band, int rule, const int* __restrict__ boff,
                                                    long long* __restrict__ idx, unsigned char* __restrict__ mask) {
    __shared__ int wc[4];
    const long long a = blockIdx.x * seg, e = min(n, a + seg);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int base = boff[blockIdx.x];
    for (long long c0 = a; c0 < e; c0 += 256) {
        const long long i = c0 + threadIdx.x;
        const bool f = i < e && in_band(y, i, n, band, rule);
        if (mask && i < e) mask[i] = f ? 1 : 0;
        const unsigned long long b = __builtin_amdgcn_ballot_w64(f);
        if (lane == 0) wc[wave] = __popcll(b);
        __syncthreads();
        int before = base;
        for (int w = 0; w < wave; ++w) before += wc[w];
        if (f) {
            const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)b, 0));
            idx[before + rank] = i;
        }
        base += wc[0] + wc[1] + wc[2] + wc[3];
        __syncthreads();
    }
}

__global__ void k_gather(const float* __restrict__ qx, const float* __restrict__ qy, const float* __restrict__ qz,
                         long long qs, const long long* __restrict__ idx, const int* __restrict__ count,
                         float* __restrict__ out) {
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j >= *count) return;
    const long long i = idx[j];
    out[3 * j] = qx[i * qs];
    out[3 * j + 1] = qy[i * qs];
    out[3 * j + 2] = qz[i * qs];
}

__global__ void k_scatter(const float* __restrict__ wc, const long long* __restrict__ idx, const int* __restrict__ count,
                          float* __restrict__ w) {
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j >= *count) return;
    w[idx[j]] = wc[j];
}

// host-side parameter initialisation: a splitmix64 stream, Box-Muller normals
struct Rng {
    unsigned long long s;
    unsigned long long next() { return smix64(s += kGolden); }
    double uni() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal() { return std::sqrt(-2.0 * std::log(uni())) * std::cos(6.283185307179586 * uni()); }
};

// The training data a handle generated for itself: n points uniform in the box,
// drawn from `seed`, labelled by the exact FP32 path on the mesh.
// The mesh's triangle and boundary-edge counts are kept as a fingerprint, so
// that a resumed run cannot silently relabel its points on another mesh.
struct Recipe {
    unsigned long long seed = 0;
    long long n = 0;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    long long mesh_nf = -1, mesh_nb = -1;
    bool operator==(const Recipe& o) const {
        return seed == o.seed && n == o.n && std::memcmp(lo, o.lo, sizeof(lo)) == 0 &&
               std::memcmp(hi, o.hi, sizeof(hi)) == 0 && mesh_nf == o.mesh_nf && mesh_nb == o.mesh_nb;
    }
};

// The schedule of a training run, recorded so that a resumed run (after
// gwn_surrogate_load, or a later gwn_surrogate_train call) continues it exactly.
struct Schedule {
    int epochs = 0, batch = 0;
    float lr = 0.f, lr_final = 0.f;
    int external = 0;          // 1: the caller supplied the points
    bool operator==(const Schedule& o) const {
        return epochs == o.epochs && batch == o.batch && lr == o.lr && lr_final == o.lr_final &&
               external == o.external;
    }
};

}  // namespace mlp
}  // namespace gwn

struct gwn_mlp_s {
    int device = 0;
    gwn::mlp::Dev d{};
    gwn::mlp::Train t{};
    long long step = 0;              // Adam steps taken
    double sigma = 0.0;              // Fourier-feature scale the network was created with
    unsigned long long init_seed = 0;
    // training run in progress (gwn_surrogate_train)
    gwn::mlp::Recipe recipe{};
    gwn::mlp::Schedule sched{};
    long long epochs_done = 0;
    float* data_x = nullptr;         // recipe.n x 3 generated points
    float* data_t = nullptr;         // their labels (or the labels of caller points, when only X is given)
    long long data_cap = 0;
    bool data_valid = false;         // data_x / data_t hold the recipe's points and labels
    float* loss_dev = nullptr;       // per-step batch losses of one call
    long long loss_cap = 0;
    // band query scratch
    float* scratch_w = nullptr;      // compacted fallback outputs
    float* scratch_q = nullptr;      // compacted fallback coordinates
    long long* scratch_idx = nullptr;
    int* scratch_cnt = nullptr;
    int* scratch_chi = nullptr;
    int* scratch_blk = nullptr;      // per-block band counts and offsets (2 x kBandBlocks)
    long long scratch_cap = 0;
};

namespace gwn {

using namespace mlp;

namespace {

void free_train(gwn_mlp_s* h) {
    (void)hipFree(h->t.x);
    (void)hipFree(h->t.dz);
    (void)hipFree(h->t.y);
    (void)hipFree(h->t.dy);
    (void)hipFree(h->t.tb);
    (void)hipFree(h->t.part);
    (void)hipFree(h->t.grad);
    h->t = Train{};
}

// tiles of 32 points per weight-gradient chunk: at least 8, and at most 64
// chunks (so the partial sums stay small next to the activations)
long long wgrad_chunk(long long tiles) { return std::max<long long>(8, (tiles + 63) / 64); }

gwn_status ensure_train(gwn_mlp_s* h, long long n) {
    if (h->t.cap >= n) return GWN_OK;
    if (h->t.x) (void)hipDeviceSynchronize();   // earlier steps may still use the buffers
    free_train(h);
    const long long tiles = (std::max<long long>(n, 1024) + 31) / 32, cap = tiles * 32;
    // a batch of at most `tiles` tiles has at most this many chunks (every chunk
    // but the last holds wgrad_chunk() >= 8 tiles, and there are at most 64)
    const long long nchunk = std::min<long long>(64, (tiles + 7) / 8);
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->t.x, sizeof(unsigned short) * tiles * kXkb * 512));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->t.dz, sizeof(unsigned short) * tiles * kDzkb * 512));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->t.y, sizeof(float) * cap));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->t.dy, sizeof(float) * cap));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->t.tb, sizeof(float) * cap));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->t.part, sizeof(float) * nchunk * (kNParams + 1)));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->t.grad, sizeof(float) * (kNParams + 1)));
    h->t.cap = cap;
    return GWN_OK;
}

gwn_status ensure_scratch(gwn_mlp_s* h, long long n) {
    if (h->scratch_cap >= n) return GWN_OK;
    if (h->scratch_w) (void)hipDeviceSynchronize();   // an earlier query may still use the buffers
    (void)hipFree(h->scratch_w);
    (void)hipFree(h->scratch_q);
    (void)hipFree(h->scratch_idx);
    (void)hipFree(h->scratch_chi);
    h->scratch_w = nullptr;
    h->scratch_q = nullptr;
    h->scratch_idx = nullptr;
    h->scratch_chi = nullptr;
    h->scratch_cap = 0;
    const long long cap = std::max<long long>(n, 1024);
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->scratch_w, sizeof(float) * cap));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->scratch_q, sizeof(float) * 3 * cap));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->scratch_idx, sizeof(long long) * cap));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->scratch_chi, sizeof(int) * cap));
    if (!h->scratch_cnt) GWN_HIP_TRY(gwn::dmalloc((void**)&h->scratch_cnt, sizeof(int)));
    if (!h->scratch_blk) GWN_HIP_TRY(gwn::dmalloc((void**)&h->scratch_blk, sizeof(int) * 2 * kBandBlocks));
    h->scratch_cap = cap;
    return GWN_OK;
}

gwn_status ensure_data(gwn_mlp_s* h, long long n) {
    if (h->data_cap >= n) return GWN_OK;
    if (h->data_x) (void)hipDeviceSynchronize();   // earlier training may still read the data
    (void)hipFree(h->data_x);
    (void)hipFree(h->data_t);
    h->data_x = nullptr;
    h->data_t = nullptr;
    h->data_cap = 0;
    h->data_valid = false;
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->data_x, sizeof(float) * 3 * (size_t)std::max<long long>(n, 1)));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->data_t, sizeof(float) * (size_t)std::max<long long>(n, 1)));
    h->data_cap = n;
    return GWN_OK;
}

gwn_status alloc_params(gwn_mlp_s* h) {
    GWN_HIP_TRY(hipGetDevice(&h->device));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->d.master, sizeof(float) * kNParams));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->d.m, sizeof(float) * kNParams));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->d.v, sizeof(float) * kNParams));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->d.G, sizeof(float) * 96));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->d.wf, sizeof(unsigned short) * kWf));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->d.wb, sizeof(unsigned short) * kWb));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->d.wi, sizeof(unsigned short) * kWi));
    GWN_HIP_TRY(gwn::dmalloc((void**)&h->d.wh, sizeof(unsigned short) * kWi));
    return GWN_OK;
}

// One optimisation step on the batch rows S.off .. S.off + n - 1: forward,
// backward, weight gradients, their sum, then Adam at learning rate lr.
gwn_status train_batch(gwn_mlp_s* h, const Src& S, long long n, float lr, float* loss_slot, hipStream_t st) {
    const long long tiles = (n + 31) / 32;
    // one workgroup of four waves per CU (each wave's weight fragments fill
    // its registers), persistent over the tiles
    k_tfb<<<(int)std::min<long long>(tiles, 256), 256, 0, st>>>(h->d, S, n, 1.0f / (float)n, h->t);
    GWN_HIP_TRY(hipGetLastError());
    const long long ct = wgrad_chunk(tiles);
    const int nchunk = (int)((tiles + ct - 1) / ct);
    k_twgrad<<<dim3(nchunk, 15), 64 * kWgW, 0, st>>>(n, (int)ct, h->t);
    GWN_HIP_TRY(hipGetLastError());
    if (lr < 0.f) {   // gradient only
        k_reduce<<<(kNParams + 1 + 255) / 256, 256, 0, st>>>(h->t.part, nchunk, h->t.grad);
        GWN_HIP_TRY(hipGetLastError());
        return GWN_OK;
    }
    h->step += 1;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)h->step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)h->step));
    k_reduce_adam<<<(kNParams + 1 + 255) / 256, 256, 0, st>>>(h->d, h->t.part, nchunk, lr, 0.9f, 0.999f, 1e-8f, c1,
                                                             c2, loss_slot, (float)n);
    GWN_HIP_TRY(hipGetLastError());
    return GWN_OK;
}

Src plain_src(const float* qx, const float* qy, const float* qz, int64_t qs, const float* tgt, int64_t n) {
    Src s{};
    s.qx = qx;
    s.qy = qy;
    s.qz = qz;
    s.qs = qs;
    s.tgt = tgt;
    s.off = 0;
    s.ntot = n;
    s.key = 0;
    s.half = 0;
    return s;
}

// ---- checkpoint file: a fixed little-endian header, the arrays, then an
// FNV-1a 64-bit checksum of every byte before it
constexpr char kMagic[8] = {'G', 'W', 'N', 'S', 'U', 'R', 'R', '1'};
constexpr uint32_t kVersion = 2;   // 2: the 32x32x16 fragment layouts of the bf16 copies

struct FileHeader {
    char magic[8];
    uint32_t version;
    uint32_t header_bytes;
    int64_t nparams;
    int64_t step;              // Adam steps taken (bias correction)
    int64_t epochs_done;       // epochs of the recorded schedule completed
    double sigma;
    uint64_t init_seed;
    uint64_t data_seed;        // the recipe of the generated training points
    int64_t data_n;
    double box_lo[3], box_hi[3];
    int32_t sched_epochs, sched_batch;
    float sched_lr, sched_lr_final;
    int32_t sched_external;
    int32_t data_generated;    // 1: the run trains on generated points (recipe above)
    int64_t mesh_nf, mesh_nb;  // fingerprint of the labelling mesh (-1: labels from the caller)
    int64_t n_wf, n_wb, n_wi;  // bf16 copies stored after the fp32 arrays
};

uint64_t fnv1a(const unsigned char* p, size_t n, uint64_t h) {
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

}  // namespace

int mlp_device(const gwn_mlp_s* h) { return h->device; }

void mlp_release(gwn_mlp_s* h) {
    if (!h) return;
    (void)hipDeviceSynchronize();   // nothing may still use the buffers
    (void)hipFree(h->d.master);
    (void)hipFree(h->d.m);
    (void)hipFree(h->d.v);
    (void)hipFree(h->d.G);
    (void)hipFree(h->d.wf);
    (void)hipFree(h->d.wb);
    (void)hipFree(h->d.wi);
    (void)hipFree(h->d.wh);
    free_train(h);
    (void)hipFree(h->data_x);
    (void)hipFree(h->data_t);
    (void)hipFree(h->loss_dev);
    (void)hipFree(h->scratch_w);
    (void)hipFree(h->scratch_q);
    (void)hipFree(h->scratch_idx);
    (void)hipFree(h->scratch_chi);
    (void)hipFree(h->scratch_cnt);
    (void)hipFree(h->scratch_blk);
    delete h;
}

gwn_status mlp_create(uint64_t seed, double sigma, gwn_mlp_s** out) {
    gwn_mlp_s* h = new (std::nothrow) gwn_mlp_s();
    if (!h) return GWN_E_OOM;
    struct Guard {
        gwn_mlp_s* h;
        ~Guard() { if (h) mlp_release(h); }
    } guard{h};
    gwn_status s = alloc_params(h);
    if (s != GWN_OK) return s;
    h->sigma = sigma;
    h->init_seed = seed;
    Rng r{seed};
    std::vector<float> G(96), theta(kNParams, 0.f);
    for (float& g : G) g = (float)(sigma * r.normal());
    const int fan_in[5] = {64, 128, 128, 128, 128};
    for (int l = 0; l < 5; ++l) {
        const double a = std::sqrt(6.0 / fan_in[l]);   // uniform He-style bound
        for (int p = kOffW[l]; p < kOffB[l]; ++p) theta[p] = (float)(a * (2.0 * r.uni() - 1.0));
    }
    std::vector<float> zeros(kNParams, 0.f);
    GWN_HIP_TRY(hipMemcpy(h->d.G, G.data(), sizeof(float) * 96, hipMemcpyHostToDevice));
    GWN_HIP_TRY(hipMemcpy(h->d.master, theta.data(), sizeof(float) * kNParams, hipMemcpyHostToDevice));
    GWN_HIP_TRY(hipMemcpy(h->d.m, zeros.data(), sizeof(float) * kNParams, hipMemcpyHostToDevice));
    GWN_HIP_TRY(hipMemcpy(h->d.v, zeros.data(), sizeof(float) * kNParams, hipMemcpyHostToDevice));
    k_pack<<<(kNParams + 255) / 256, 256>>>(h->d);
    GWN_HIP_TRY(hipGetLastError());
    GWN_HIP_TRY(hipDeviceSynchronize());
    guard.h = nullptr;
    *out = h;
    return GWN_OK;
}

gwn_status mlp_get_state(gwn_mlp_s* h, float* theta, float* m, float* v, float* G, int64_t* step) {
    GWN_HIP_TRY(hipDeviceSynchronize());
    if (theta) GWN_HIP_TRY(hipMemcpy(theta, h->d.master, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
    if (m) GWN_HIP_TRY(hipMemcpy(m, h->d.m, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
    if (v) GWN_HIP_TRY(hipMemcpy(v, h->d.v, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
    if (G) GWN_HIP_TRY(hipMemcpy(G, h->d.G, sizeof(float) * 96, hipMemcpyDeviceToHost));
    if (step) *step = h->step;
    return GWN_OK;
}

gwn_status mlp_set_state(gwn_mlp_s* h, const float* theta, const float* m, const float* v, const float* G,
                         int64_t step) {
    GWN_HIP_TRY(hipDeviceSynchronize());
    if (theta) GWN_HIP_TRY(hipMemcpy(h->d.master, theta, sizeof(float) * kNParams, hipMemcpyHostToDevice));
    if (m) GWN_HIP_TRY(hipMemcpy(h->d.m, m, sizeof(float) * kNParams, hipMemcpyHostToDevice));
    if (v) GWN_HIP_TRY(hipMemcpy(h->d.v, v, sizeof(float) * kNParams, hipMemcpyHostToDevice));
    if (G) GWN_HIP_TRY(hipMemcpy(h->d.G, G, sizeof(float) * 96, hipMemcpyHostToDevice));
    if (step >= 0) h->step = step;
    k_pack<<<(kNParams + 255) / 256, 256>>>(h->d);
    GWN_HIP_TRY(hipGetLastError());
    GWN_HIP_TRY(hipDeviceSynchronize());
    return GWN_OK;
}

gwn_status mlp_forward(gwn_mlp_s* h, const float* qx, const float* qy, const float* qz, int64_t qs, int64_t n,
                       float* y, hipStream_t st) {
    if (n == 0) return GWN_OK;
    // half path: k_infer<2, 8>, two tiles of 32 points per wave (each weight
    // fragment read from LDS serves both), 8 waves; erf path: one tile per wave
    // (its 150 VGPRs leave no room for a second)
    const long long nw = 8;
    auto blocks = [&](long long pts) {
        const long long steps = (n + pts - 1) / pts;
        return (unsigned)std::max<long long>(1, std::min<long long>((steps + nw - 1) / nw, 256));
    };
    // GWN_INFER_GELU=erf selects the erf form of GELU on bf16 operands (the training kernels' arithmetic)
    bool poly = true;
    if (const char* e = std::getenv("GWN_INFER_GELU")) poly = std::string(e) != "erf";
    if (poly) k_infer<2, 8, true><<<blocks(64), 64 * 8, 0, st>>>(h->d, qx, qy, qz, qs, n, y);
    else k_infer<1, 8, false><<<blocks(32), 64 * 8, 0, st>>>(h->d, qx, qy, qz, qs, n, y);
    GWN_HIP_TRY(hipGetLastError());
    return GWN_OK;
}

gwn_status mlp_loss_grad(gwn_mlp_s* h, const float* qx, const float* qy, const float* qz, int64_t qs,
                         const float* tgt, int64_t n, float* grad_out, float* loss_out, hipStream_t st) {
    gwn_status s = ensure_train(h, n);
    if (s != GWN_OK) return s;
    s = train_batch(h, plain_src(qx, qy, qz, qs, tgt, n), n, -1.f, nullptr, st);
    if (s != GWN_OK) return s;
    if (grad_out)
        GWN_HIP_TRY(hipMemcpyAsync(grad_out, h->t.grad, sizeof(float) * kNParams, hipMemcpyDeviceToDevice, st));
    if (loss_out) {   // sum(dy^2) = sum(4 d^2 / n^2)  ->  loss = mean(d^2) = sum(dy^2) n / 4
        float sdy2 = 0.f;
        GWN_HIP_TRY(hipMemcpyAsync(&sdy2, h->t.grad + kNParams, sizeof(float), hipMemcpyDeviceToHost, st));
        GWN_HIP_TRY(hipStreamSynchronize(st));
        *loss_out = sdy2 * (float)n / 4.0f;
    }
    return GWN_OK;
}

gwn_status mlp_train_step(gwn_mlp_s* h, const float* qx, const float* qy, const float* qz, int64_t qs,
                          const float* tgt, int64_t n, float lr, float* loss_out, hipStream_t st) {
    gwn_status s = ensure_train(h, n);
    if (s != GWN_OK) return s;
    if (!h->loss_dev) {
        GWN_HIP_TRY(gwn::dmalloc((void**)&h->loss_dev, sizeof(float) * 1024));
        h->loss_cap = 1024;
    }
    s = train_batch(h, plain_src(qx, qy, qz, qs, tgt, n), n, lr, h->loss_dev, st);
    if (s != GWN_OK) return s;
    if (loss_out) {
        GWN_HIP_TRY(hipMemcpyAsync(loss_out, h->loss_dev, sizeof(float), hipMemcpyDeviceToHost, st));
        GWN_HIP_TRY(hipStreamSynchronize(st));
    }
    return GWN_OK;
}

// World-frame bounding box of the mesh's vertices (the handle keeps it in the
// frame of its ray axis: frame component c is world component (c + axis) % 3).
static void world_bbox(const gwn_mesh_s* m, double lo[3], double hi[3]) {
    for (int c = 0; c < 3; ++c) {
        const int a = (c + m->axis) % 3;
        lo[a] = m->bbox[c];
        hi[a] = m->bbox[3 + c];
    }
}

gwn_status surrogate_train(gwn_mlp_s* h, const gwn_mesh_s* mesh, const gwn_surrogate_cfg& c, const float* X,
                           const float* T, int64_t n_given, float* epoch_loss, int64_t* epochs_run, hipStream_t st) {
    if (epochs_run) *epochs_run = 0;
    Schedule sc;
    sc.epochs = c.epochs;
    sc.batch = c.batch;
    sc.lr = c.lr;
    sc.lr_final = c.lr_final;
    sc.external = X ? 1 : 0;
    Recipe rc;
    if (!X) {
        rc.seed = c.seed;
        rc.n = c.n_train;
        const bool dflt = c.box_lo[0] == 0 && c.box_lo[1] == 0 && c.box_lo[2] == 0 && c.box_hi[0] == 0 &&
                          c.box_hi[1] == 0 && c.box_hi[2] == 0;
        if (dflt) world_bbox(mesh, rc.lo, rc.hi);
        else
            for (int a = 0; a < 3; ++a) {
                rc.lo[a] = c.box_lo[a];
                rc.hi[a] = c.box_hi[a];
            }
    } else {
        rc.seed = c.seed;
        rc.n = n_given;
    }
    if (!X || !T) {
        rc.mesh_nf = mesh->nf;
        rc.mesh_nb = mesh->nb;
    }
    // a run in progress continues only under the schedule and data it started with
    if (h->epochs_done > 0 && !(h->sched == sc && h->recipe == rc)) {
        set_error("gwn_surrogate_train: the handle has trained %lld epochs under another schedule or data recipe; "
                  "resume with the same configuration or start from a new handle", h->epochs_done);
        return GWN_E_INVALID;
    }
    const long long n = rc.n;
    const int stop = c.stop_epoch > 0 ? std::min(c.stop_epoch, c.epochs) : c.epochs;
    h->sched = sc;
    const float* dx = X;
    const float* dt = T;
    gwn_status s = GWN_OK;
    if (!X || !T) {
        // generated points, or caller points without labels: the library keeps
        // the points (when generated) and the labels
        if (!X && !(h->data_valid && h->recipe == rc)) {
            s = ensure_data(h, n);
            if (s != GWN_OK) return s;
            k_gen_points<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(rc.seed, n, rc.lo[0], rc.lo[1], rc.lo[2],
                                                                     rc.hi[0] - rc.lo[0], rc.hi[1] - rc.lo[1],
                                                                     rc.hi[2] - rc.lo[2], h->data_x);
            GWN_HIP_TRY(hipGetLastError());
            s = query_batch(mesh, h->data_x, h->data_x + 1, h->data_x + 2, 3, n, GWN_PREC_FP32, h->data_t, nullptr,
                            st);
            if (s != GWN_OK) return s;
            h->data_valid = true;
        } else if (X) {
            s = ensure_data(h, n);
            if (s != GWN_OK) return s;
            h->data_valid = false;   // holds labels of caller points, not the recipe
            s = query_batch(mesh, X, X + 1, X + 2, 3, n, GWN_PREC_FP32, h->data_t, nullptr, st);
            if (s != GWN_OK) return s;
        }
        if (!X) dx = h->data_x;
        dt = h->data_t;
    }
    h->recipe = rc;
    if (h->epochs_done >= stop) return GWN_OK;
    const long long batch = std::min<long long>(c.batch, n);
    const long long spe = (n + batch - 1) / batch;
    const long long total = (long long)c.epochs * spe;
    const long long nsteps = (stop - h->epochs_done) * spe;
    s = ensure_train(h, batch);
    if (s != GWN_OK) return s;
    if (h->loss_cap < nsteps) {
        if (h->loss_dev) (void)hipDeviceSynchronize();
        (void)hipFree(h->loss_dev);
        h->loss_dev = nullptr;
        h->loss_cap = 0;
        GWN_HIP_TRY(gwn::dmalloc((void**)&h->loss_dev, sizeof(float) * (size_t)nsteps));
        h->loss_cap = nsteps;
    }
    Src S{};
    S.qx = dx;
    S.qy = dx + 1;
    S.qz = dx + 2;
    S.qs = 3;
    S.tgt = dt;
    S.ntot = n;
    S.half = shuffle_half(n);
    const int first = (int)h->epochs_done;
    long long j = 0;
    for (int e = first; e < stop; ++e) {
        // the epoch's shuffle key: a pure function of the seed and the epoch
        S.key = smix64(rc.seed ^ smix64(0x5348554646ull + (unsigned long long)e * kGolden));
        for (long long b = 0; b < spe; ++b, ++j) {
            S.off = b * batch;
            const long long nb = std::min(batch, n - S.off);
            const long long k = (long long)e * spe + b;   // position in the whole schedule
            const double ph = 3.141592653589793 * (double)k / (double)std::max<long long>(1, total - 1);
            const float lr = (float)(c.lr_final + 0.5 * ((double)c.lr - c.lr_final) * (1.0 + std::cos(ph)));
            s = train_batch(h, S, nb, lr, h->loss_dev + j, st);
            if (s != GWN_OK) return s;
        }
        h->epochs_done = e + 1;
    }
    std::vector<float> losses((size_t)nsteps);
    GWN_HIP_TRY(hipMemcpyAsync(losses.data(), h->loss_dev, sizeof(float) * (size_t)nsteps, hipMemcpyDeviceToHost, st));
    GWN_HIP_TRY(hipStreamSynchronize(st));
    if (epoch_loss)
        for (int e = first; e < stop; ++e) {
            double acc = 0.0;
            for (long long b = 0; b < spe; ++b) acc += losses[(size_t)((e - first) * spe + b)];
            epoch_loss[e - first] = (float)(acc / (double)spe);
        }
    if (epochs_run) *epochs_run = stop - first;
    return GWN_OK;
}

gwn_status surrogate_save(gwn_mlp_s* h, const char* path) {
    FileHeader hd{};
    std::memcpy(hd.magic, kMagic, 8);
    hd.version = kVersion;
    hd.header_bytes = sizeof(FileHeader);
    hd.nparams = kNParams;
    hd.step = h->step;
    hd.epochs_done = h->epochs_done;
    hd.sigma = h->sigma;
    hd.init_seed = h->init_seed;
    hd.data_seed = h->recipe.seed;
    hd.data_n = h->recipe.n;
    for (int a = 0; a < 3; ++a) {
        hd.box_lo[a] = h->recipe.lo[a];
        hd.box_hi[a] = h->recipe.hi[a];
    }
    hd.sched_epochs = h->sched.epochs;
    hd.sched_batch = h->sched.batch;
    hd.sched_lr = h->sched.lr;
    hd.sched_lr_final = h->sched.lr_final;
    hd.sched_external = h->sched.external;
    hd.data_generated = h->sched.external ? 0 : 1;
    hd.mesh_nf = h->recipe.mesh_nf;
    hd.mesh_nb = h->recipe.mesh_nb;
    hd.n_wf = kWf;
    hd.n_wb = kWb;
    hd.n_wi = kWi;
    std::vector<float> G(96), th(kNParams), m(kNParams), v(kNParams);
    std::vector<unsigned short> wf(kWf), wb(kWb), wi(kWi);
    GWN_HIP_TRY(hipDeviceSynchronize());
    GWN_HIP_TRY(hipMemcpy(G.data(), h->d.G, sizeof(float) * 96, hipMemcpyDeviceToHost));
    GWN_HIP_TRY(hipMemcpy(th.data(), h->d.master, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
    GWN_HIP_TRY(hipMemcpy(m.data(), h->d.m, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
    GWN_HIP_TRY(hipMemcpy(v.data(), h->d.v, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
    GWN_HIP_TRY(hipMemcpy(wf.data(), h->d.wf, sizeof(unsigned short) * kWf, hipMemcpyDeviceToHost));
    GWN_HIP_TRY(hipMemcpy(wb.data(), h->d.wb, sizeof(unsigned short) * kWb, hipMemcpyDeviceToHost));
    GWN_HIP_TRY(hipMemcpy(wi.data(), h->d.wi, sizeof(unsigned short) * kWi, hipMemcpyDeviceToHost));
    std::vector<unsigned char> buf;
    auto put = [&buf](const void* p, size_t n) {
        const unsigned char* c = (const unsigned char*)p;
        buf.insert(buf.end(), c, c + n);
    };
    put(&hd, sizeof(hd));
    put(G.data(), sizeof(float) * 96);
    put(th.data(), sizeof(float) * kNParams);
    put(m.data(), sizeof(float) * kNParams);
    put(v.data(), sizeof(float) * kNParams);
    put(wf.data(), sizeof(unsigned short) * kWf);
    put(wb.data(), sizeof(unsigned short) * kWb);
    put(wi.data(), sizeof(unsigned short) * kWi);
    const uint64_t sum = fnv1a(buf.data(), buf.size(), 0xCBF29CE484222325ull);
    put(&sum, sizeof(sum));
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) {
        set_error("gwn_surrogate_save: cannot open %s for writing", tmp.c_str());
        return GWN_E_INVALID;
    }
    const size_t wrote = std::fwrite(buf.data(), 1, buf.size(), f);
    const bool ok = wrote == buf.size() && std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        set_error("gwn_surrogate_save: writing %s failed", path);
        return GWN_E_INVALID;
    }
    return GWN_OK;
}

gwn_status surrogate_load(const char* path, gwn_mlp_s** out) {
    FILE* f = std::fopen(path, "rb");
    if (!f) {
        set_error("gwn_surrogate_load: cannot open %s", path);
        return GWN_E_INVALID;
    }
    std::vector<unsigned char> buf;
    unsigned char tmp[1 << 16];
    size_t got;
    while ((got = std::fread(tmp, 1, sizeof(tmp), f)) > 0) buf.insert(buf.end(), tmp, tmp + got);
    std::fclose(f);
    const size_t arrays = sizeof(float) * (96 + 3 * (size_t)kNParams) + sizeof(unsigned short) * (kWf + kWb + kWi);
    const size_t want = sizeof(FileHeader) + arrays + sizeof(uint64_t);
    FileHeader hd;
    if (buf.size() < sizeof(FileHeader)) {
        set_error("gwn_surrogate_load: %s is too short for a checkpoint", path);
        return GWN_E_INVALID;
    }
    std::memcpy(&hd, buf.data(), sizeof(hd));
    if (std::memcmp(hd.magic, kMagic, 8) != 0 || hd.version != kVersion || hd.header_bytes != sizeof(FileHeader) ||
        hd.nparams != kNParams || hd.n_wf != kWf || hd.n_wb != kWb || hd.n_wi != kWi || buf.size() != want) {
        set_error("gwn_surrogate_load: %s is not a version-%u surrogate checkpoint of this network", path, kVersion);
        return GWN_E_INVALID;
    }
    uint64_t sum;
    std::memcpy(&sum, buf.data() + want - sizeof(uint64_t), sizeof(sum));
    if (fnv1a(buf.data(), want - sizeof(uint64_t), 0xCBF29CE484222325ull) != sum) {
        set_error("gwn_surrogate_load: checksum mismatch in %s", path);
        return GWN_E_INVALID;
    }
    if (!(hd.sigma > 0.0) || hd.step < 0 || hd.epochs_done < 0 || hd.data_n < 0) {
        set_error("gwn_surrogate_load: bad values in the header of %s", path);
        return GWN_E_INVALID;
    }
    gwn_mlp_s* h = new (std::nothrow) gwn_mlp_s();
    if (!h) return GWN_E_OOM;
    struct Guard {
        gwn_mlp_s* h;
        ~Guard() { if (h) mlp_release(h); }
    } guard{h};
    gwn_status s = alloc_params(h);
    if (s != GWN_OK) return s;
    const unsigned char* p = buf.data() + sizeof(FileHeader);
    auto dev = [&p](void* d, size_t n) -> hipError_t {
        const hipError_t e = hipMemcpy(d, p, n, hipMemcpyHostToDevice);
        p += n;
        return e;
    };
    GWN_HIP_TRY(dev(h->d.G, sizeof(float) * 96));
    GWN_HIP_TRY(dev(h->d.master, sizeof(float) * kNParams));
    GWN_HIP_TRY(dev(h->d.m, sizeof(float) * kNParams));
    GWN_HIP_TRY(dev(h->d.v, sizeof(float) * kNParams));
    // the bf16 copies are a function of the masters: re-pack them and require
    // the stored ones to agree, bit for bit
    k_pack<<<(kNParams + 255) / 256, 256>>>(h->d);
    GWN_HIP_TRY(hipGetLastError());
    std::vector<unsigned short> w((size_t)(kWf + kWb + kWi));
    GWN_HIP_TRY(hipMemcpy(w.data(), h->d.wf, sizeof(unsigned short) * kWf, hipMemcpyDeviceToHost));
    GWN_HIP_TRY(hipMemcpy(w.data() + kWf, h->d.wb, sizeof(unsigned short) * kWb, hipMemcpyDeviceToHost));
    GWN_HIP_TRY(hipMemcpy(w.data() + kWf + kWb, h->d.wi, sizeof(unsigned short) * kWi, hipMemcpyDeviceToHost));
    if (std::memcmp(w.data(), p, sizeof(unsigned short) * w.size()) != 0) {
        set_error("gwn_surrogate_load: the bf16 weights in %s do not match its fp32 masters", path);
        return GWN_E_INVALID;
    }
    h->step = hd.step;
    h->epochs_done = hd.epochs_done;
    h->sigma = hd.sigma;
    h->init_seed = hd.init_seed;
    h->recipe.seed = hd.data_seed;
    h->recipe.n = hd.data_n;
    h->recipe.mesh_nf = hd.mesh_nf;
    h->recipe.mesh_nb = hd.mesh_nb;
    for (int a = 0; a < 3; ++a) {
        h->recipe.lo[a] = hd.box_lo[a];
        h->recipe.hi[a] = hd.box_hi[a];
    }
    h->sched.epochs = hd.sched_epochs;
    h->sched.batch = hd.sched_batch;
    h->sched.lr = hd.sched_lr;
    h->sched.lr_final = hd.sched_lr_final;
    h->sched.external = hd.sched_external;
    guard.h = nullptr;
    *out = h;
    return GWN_OK;
}

gwn_status surrogate_query(gwn_mlp_s* h, const gwn_mesh_s* mesh, const float* qx, const float* qy, const float* qz,
                           int64_t qs, int64_t n, float band, int rule, float* w, unsigned char* mask,
                           int64_t* nfallback, hipStream_t st) {
    if (n == 0) {
        if (nfallback) *nfallback = 0;
        return GWN_OK;
    }
    gwn_status s = ensure_scratch(h, n);
    if (s != GWN_OK) return s;
    s = mlp_forward(h, qx, qy, qz, qs, n, w, st);
    if (s != GWN_OK) return s;
    const unsigned nb = (unsigned)((n + 255) / 256);
    const long long seg = ((n + kBandBlocks - 1) / kBandBlocks + 255) / 256 * 256;
    k_band_count<<<kBandBlocks, 256, 0, st>>>(w, n, seg, band, rule, h->scratch_blk);
    k_band_scan<<<1, kBandBlocks, 0, st>>>(h->scratch_blk, h->scratch_blk + kBandBlocks, h->scratch_cnt);
    k_band_write<<<kBandBlocks, 256, 0, st>>>(w, n, seg, band, rule, h->scratch_blk + kBandBlocks, h->scratch_idx,
                                              mask);
    k_gather<<<nb, 256, 0, st>>>(qx, qy, qz, qs, h->scratch_idx, h->scratch_cnt, h->scratch_q);
    GWN_HIP_TRY(hipGetLastError());
    // the fallback count sizes the exact evaluation (one synchronisation), which
    // then takes the ordinary batch path on the compacted points
    int c = 0;
    GWN_HIP_TRY(hipMemcpyAsync(&c, h->scratch_cnt, sizeof(int), hipMemcpyDeviceToHost, st));
    GWN_HIP_TRY(hipStreamSynchronize(st));
    if (nfallback) *nfallback = c;
    if (c == 0) return GWN_OK;
    s = query_batch(mesh, h->scratch_q, h->scratch_q + 1, h->scratch_q + 2, 3, c, GWN_PREC_FP32, h->scratch_w,
                    h->scratch_chi, st);
    if (s != GWN_OK) return s;
    k_scatter<<<(unsigned)((c + 255) / 256), 256, 0, st>>>(h->scratch_w, h->scratch_idx, h->scratch_cnt, w);
    GWN_HIP_TRY(hipGetLastError());
    return GWN_OK;
}

}  // namespace gwn
