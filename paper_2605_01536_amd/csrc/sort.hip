// sort.hip -- the library's own device radix sort and prefix scans (see
// gwn_sort.h).
//
// Radix sort: least significant digit first, 8-bit digits.  Each pass splits
// the keys into tiles of 4,096 (256 threads x 16 rounds, round j holding
// positions 256 j .. 256 j + 255 of the tile, so loads are coalesced):
//   1. k_rs_hist counts each tile's digits into hist[digit][tile];
//   2. an exclusive scan of hist, digit-major, gives every (digit, tile) its
//      first output position: all smaller digits, then the same digit in
//      earlier tiles;
//   3. k_rs_scatter ranks each key within its tile stably -- a wave finds the
//      lanes sharing its digit with 8 ballots (one per digit bit), a lane's
//      rank is the number of such lanes below it, the four waves' counts are
//      combined per digit in LDS, and a running count per digit carries over
//      from round to round -- and writes the key (and payload) to its position.
// Every step keeps input order among equal digits, so each pass is stable and
// the passes compose to a sort by all the bits.
//
// Scan: a tile of 4,096 ints is staged in LDS, each thread scans 16
// consecutive values, the 256 thread totals are scanned by wave shuffles and
// one LDS exchange across the four waves.  Longer inputs reduce each tile,
// scan the tile totals recursively, and add the tile's prefix.
#include <climits>

#include "gwn_alloc.h"
#include "gwn_sort.h"

namespace gwn {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;
constexpr int kRadix = 256;

// ------------------------------------------------------------------ scan

struct OpSum {
    static __device__ __forceinline__ int id() { return 0; }
    static __device__ __forceinline__ int f(int a, int b) { return a + b; }
};
struct OpMax {
    static __device__ __forceinline__ int id() { return INT_MIN; }
    static __device__ __forceinline__ int f(int a, int b) { return a > b ? a : b; }
};

// reduction of each tile of `in` into sums[tile]
template <class Op>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const int* __restrict__ in, int64_t n,
                                                          int* __restrict__ sums) {
    __shared__ int sw[kThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int acc = Op::id();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t p = base + j * kThreads + threadIdx.x;
        if (p < n) acc = Op::f(acc, in[p]);
    }
    for (int o = 32; o > 0; o >>= 1) acc = Op::f(acc, __shfl_xor(acc, o));
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = sw[0];
        for (int w = 1; w < kThreads / 64; ++w) r = Op::f(r, sw[w]);
        sums[blockIdx.x] = r;
    }
}

// scan of each tile, offset by prefix[tile] (exclusive prefix of the tiles
// before it; nullptr: identity); in-place safe (a tile is read before written)
template <class Op>
__global__ __launch_bounds__(kThreads) void k_scan_tile(const int* in, int* out, int64_t n,
                                                        const int* __restrict__ prefix, int inclusive) {
    // element e of the tile sits at e + e / 16: a thread's 16 values are
    // consecutive, and the padding spreads the threads over the banks
    __shared__ int s[kTile + kTile / kItems];
    __shared__ int swave[kThreads / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int e = j * kThreads + t;
        const int64_t p = base + e;
        s[e + e / kItems] = p < n ? in[p] : Op::id();
    }
    __syncthreads();
    int v[kItems];
    int run = Op::id();
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = s[t * (kItems + 1) + i];
        run = Op::f(run, v[i]);
    }
    // inclusive scan of the thread totals within the wave
    int inc = run;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(inc, o);
        if (lane >= o) inc = Op::f(inc, u);
    }
    if (lane == 63) swave[wave] = inc;
    __syncthreads();
    int carry = prefix ? prefix[blockIdx.x] : Op::id();
    for (int w = 0; w < wave; ++w) carry = Op::f(carry, swave[w]);
    int excl = __shfl_up(inc, 1);
    if (lane == 0) excl = Op::id();
    carry = Op::f(carry, excl);
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int nxt = Op::f(carry, v[i]);
        s[t * (kItems + 1) + i] = inclusive ? nxt : carry;
        carry = nxt;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int e = j * kThreads + t;
        const int64_t p = base + e;
        if (p < n) out[p] = s[e + e / kItems];
    }
}

int64_t tiles_of(int64_t n) { return (n + kTile - 1) / kTile; }

// ints of temporary storage for a scan of n values
int64_t scan_temp_ints(int64_t n) {
    if (n <= kTile) return 0;
    const int64_t nb = tiles_of(n);
    return nb + scan_temp_ints(nb);
}

template <class Op>
hipError_t scan_rec(const int* in, int* out, int64_t n, bool inclusive, int* tmp, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = tiles_of(n);
    if (nb == 1) {
        k_scan_tile<Op><<<1, kThreads, 0, st>>>(in, out, n, nullptr, inclusive ? 1 : 0);
        return hipGetLastError();
    }
    int* sums = tmp;
    k_scan_reduce<Op><<<(unsigned)nb, kThreads, 0, st>>>(in, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_rec<Op>(sums, sums, nb, false, tmp + nb, st);   // tile prefixes, in place
    if (e != hipSuccess) return e;
    k_scan_tile<Op><<<(unsigned)nb, kThreads, 0, st>>>(in, out, n, sums, inclusive ? 1 : 0);
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort

template <class K>
__device__ __forceinline__ unsigned digit_of(K key, int shift, unsigned mask) {
    return (unsigned)(key >> shift) & mask;
}

// hist[d * ntiles + tile] = number of keys of the tile with digit d; one
// counter set per wave keeps same-address LDS atomics to one wave
template <class K>
__global__ __launch_bounds__(kThreads) void k_rs_hist(const K* __restrict__ keys, int64_t n, int shift, unsigned mask,
                                                      int ntiles, int* __restrict__ hist) {
    __shared__ int h[kThreads / 64][kRadix];
    const int t = threadIdx.x, wave = t >> 6;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) h[w][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll 4
    for (int j = 0; j < kItems; ++j) {
        const int64_t p = base + j * kThreads + t;
        if (p < n) atomicAdd(&h[wave][digit_of(keys[p], shift, mask)], 1);
    }
    __syncthreads();
    int c = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) c += h[w][t];
    hist[(int64_t)t * ntiles + blockIdx.x] = c;
}

template <class K, bool kVals>
__global__ __launch_bounds__(kThreads) void k_rs_scatter(const K* __restrict__ kin, const int* __restrict__ vin,
                                                         K* __restrict__ kout, int* __restrict__ vout, int64_t n,
                                                         int shift, unsigned mask, int ntiles,
                                                         const int* __restrict__ offs) {
    __shared__ int s_next[kRadix];                 // next output position of each digit
    __shared__ int s_w[kThreads / 64][kRadix];     // per wave: count, then first position
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    s_next[t] = offs[(int64_t)t * ntiles + blockIdx.x];
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int j = 0; j < kItems; ++j) {
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) s_w[w][t] = 0;
        __syncthreads();
        const int64_t p = base + j * kThreads + t;
        const bool ok = p < n;
        const K key = ok ? kin[p] : K(0);
        const int val = (kVals && ok) ? vin[p] : 0;
        const unsigned d = digit_of(key, shift, mask);
        // lanes of this wave holding a key with the same digit
        unsigned long long same = __builtin_amdgcn_ballot_w64(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long bb = __builtin_amdgcn_ballot_w64(bit);
            same &= bit ? bb : ~bb;
        }
        const int rank = __popcll(same & below);
        if (ok && rank == 0) s_w[wave][d] = __popcll(same);
        __syncthreads();
        {   // thread t owns digit t: the first position of each wave's run, then advance
            const int c0 = s_w[0][t], c1 = s_w[1][t], c2 = s_w[2][t], c3 = s_w[3][t];
            const int o = s_next[t];
            s_w[0][t] = o;
            s_w[1][t] = o + c0;
            s_w[2][t] = o + c0 + c1;
            s_w[3][t] = o + c0 + c1 + c2;
            s_next[t] = o + c0 + c1 + c2 + c3;
        }
        __syncthreads();
        const int pos = s_w[wave][d] + rank;
        if (ok && pos >= 0 && (int64_t)pos < n) {   // always true for consistent counts
            kout[pos] = key;
            if (kVals) vout[pos] = val;
        }
        __syncthreads();
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

template <class K>
hipError_t radix_sort(const K* kin, K* kout, const int* vin, int* vout, int64_t n, int begin_bit, int end_bit,
                      void* temp, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const bool vals = vin != nullptr;
    char* p = (char*)temp;
    K* kalt = (K*)p;
    p += align256(sizeof(K) * (size_t)n);
    int* valt = nullptr;
    if (vals) {
        valt = (int*)p;
        p += align256(sizeof(int) * (size_t)n);
    }
    const int64_t ntiles = tiles_of(n);
    int* hist = (int*)p;
    p += align256(sizeof(int) * (size_t)(kRadix * ntiles));
    int* stmp = (int*)p;
    const int passes = end_bit > begin_bit ? (end_bit - begin_bit + 7) / 8 : 0;
    if (passes == 0) {
        hipError_t e = hipMemcpyAsync(kout, kin, sizeof(K) * (size_t)n, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && vals) e = hipMemcpyAsync(vout, vin, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, st);
        return e;
    }
    const K* ksrc = kin;
    const int* vsrc = vin;
    for (int ps = 0; ps < passes; ++ps) {
        // the last pass writes into kout: odd pass counts start there
        K* kdst = ((passes - 1 - ps) % 2 == 0) ? kout : kalt;
        int* vdst = ((passes - 1 - ps) % 2 == 0) ? vout : valt;
        const int shift = begin_bit + 8 * ps;
        const int width = end_bit - shift < 8 ? end_bit - shift : 8;
        const unsigned mask = (1u << width) - 1u;
        k_rs_hist<K><<<(unsigned)ntiles, kThreads, 0, st>>>(ksrc, n, shift, mask, (int)ntiles, hist);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = scan_rec<OpSum>(hist, hist, kRadix * ntiles, false, stmp, st);
        if (e != hipSuccess) return e;
        if (vals)
            k_rs_scatter<K, true><<<(unsigned)ntiles, kThreads, 0, st>>>(ksrc, vsrc, kdst, vdst, n, shift, mask,
                                                                        (int)ntiles, hist);
        else
            k_rs_scatter<K, false><<<(unsigned)ntiles, kThreads, 0, st>>>(ksrc, nullptr, kdst, nullptr, n, shift,
                                                                         mask, (int)ntiles, hist);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        ksrc = kdst;
        vsrc = vdst;
    }
    return hipSuccess;
}

}  // namespace

size_t scan_temp_bytes(int64_t n) { return align256(sizeof(int) * (size_t)(scan_temp_ints(n) + 1)); }

size_t sort_temp_bytes(int64_t n, int key_bytes, bool with_values) {
    const int64_t ntiles = tiles_of(n > 0 ? n : 1);
    size_t b = align256((size_t)key_bytes * (size_t)(n > 0 ? n : 1));
    if (with_values) b += align256(sizeof(int) * (size_t)(n > 0 ? n : 1));
    b += align256(sizeof(int) * (size_t)(kRadix * ntiles));
    b += scan_temp_bytes(kRadix * ntiles);
    return b;
}

hipError_t radix_sort_u32(const uint32_t* kin, uint32_t* kout, const int* vin, int* vout, int64_t n, int begin_bit,
                          int end_bit, void* temp, hipStream_t st) {
    return radix_sort<uint32_t>(kin, kout, vin, vout, n, begin_bit, end_bit, temp, st);
}

hipError_t radix_sort_u64(const uint64_t* kin, uint64_t* kout, const int* vin, int* vout, int64_t n, int begin_bit,
                          int end_bit, void* temp, hipStream_t st) {
    return radix_sort<uint64_t>(kin, kout, vin, vout, n, begin_bit, end_bit, temp, st);
}

hipError_t scan_exclusive_sum(const int* in, int* out, int64_t n, void* temp, hipStream_t st) {
    return scan_rec<OpSum>(in, out, n, false, (int*)temp, st);
}

hipError_t scan_inclusive_max(const int* in, int* out, int64_t n, void* temp, hipStream_t st) {
    return scan_rec<OpMax>(in, out, n, true, (int*)temp, st);
}

}  // namespace gwn

// ------------------------------------------------------------------ C ABI (include/gwn_prims.h)

#include "../../include/gwn_prims.h"

namespace gwn {
void set_error(const char* fmt, ...);
void clear_error();
}  // namespace gwn

namespace {

gwn_status prim_args(const char* fn, const void* in, const void* out, int64_t n) {
    if (n < 0 || n >= (1ll << 31) || (n > 0 && (!in || !out))) {
        gwn::set_error("%s: bad n=%lld or null array", fn, (long long)n);
        return GWN_E_INVALID;
    }
    return GWN_OK;
}

gwn_status prim_status(const char* fn, hipError_t e) {
    if (e == hipSuccess) return GWN_OK;
    gwn::set_error("%s: %s", fn, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? GWN_E_OOM : GWN_E_HIP;
}

// runs f(temp) with `bytes` of stream-ordered temporary memory
template <class F>
gwn_status with_async_temp(const char* fn, size_t bytes, hipStream_t st, F&& f) {
    void* tmp = nullptr;
    hipError_t e = gwn::dmalloc_async(&tmp, bytes, st);
    if (e != hipSuccess) return prim_status(fn, e);
    e = f(tmp);
    const hipError_t e2 = hipFreeAsync(tmp, st);
    return prim_status(fn, e != hipSuccess ? e : e2);
}

template <class K>
gwn_status sort_entry(const char* fn, const K* kin, K* kout, const int32_t* vin, int32_t* vout, int64_t n, int32_t b0,
                      int32_t b1, void* stream) {
    gwn::clear_error();
    gwn_status s = prim_args(fn, kin, kout, n);
    if (s != GWN_OK) return s;
    if (b0 < 0 || b0 > b1 || b1 > (int32_t)(8 * sizeof(K)) || (vin && !vout && n > 0)) {
        gwn::set_error("%s: bad bit range [%d, %d) or payload without output", fn, b0, b1);
        return GWN_E_INVALID;
    }
    if (n == 0) return GWN_OK;
    hipStream_t st = (hipStream_t)stream;
    return with_async_temp(fn, gwn::sort_temp_bytes(n, (int)sizeof(K), vin != nullptr), st, [&](void* tmp) {
        if (sizeof(K) == 4)
            return gwn::radix_sort_u32((const uint32_t*)kin, (uint32_t*)kout, vin, vout, n, b0, b1, tmp, st);
        return gwn::radix_sort_u64((const uint64_t*)kin, (uint64_t*)kout, vin, vout, n, b0, b1, tmp, st);
    });
}

}  // namespace

extern "C" {

gwn_status gwn_radix_sort_u32(const uint32_t* keys_in, uint32_t* keys_out, const int32_t* vals_in,
                              int32_t* vals_out, int64_t n, int32_t begin_bit, int32_t end_bit, void* stream) {
    return sort_entry("gwn_radix_sort_u32", keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, stream);
}

gwn_status gwn_radix_sort_u64(const uint64_t* keys_in, uint64_t* keys_out, const int32_t* vals_in,
                              int32_t* vals_out, int64_t n, int32_t begin_bit, int32_t end_bit, void* stream) {
    return sort_entry("gwn_radix_sort_u64", keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, stream);
}

gwn_status gwn_scan_exclusive_sum_i32(const int32_t* in, int32_t* out, int64_t n, void* stream) {
    gwn::clear_error();
    gwn_status s = prim_args("gwn_scan_exclusive_sum_i32", in, out, n);
    if (s != GWN_OK || n == 0) return s;
    hipStream_t st = (hipStream_t)stream;
    return with_async_temp("gwn_scan_exclusive_sum_i32", gwn::scan_temp_bytes(n), st,
                           [&](void* tmp) { return gwn::scan_exclusive_sum(in, out, n, tmp, st); });
}

gwn_status gwn_scan_inclusive_max_i32(const int32_t* in, int32_t* out, int64_t n, void* stream) {
    gwn::clear_error();
    gwn_status s = prim_args("gwn_scan_inclusive_max_i32", in, out, n);
    if (s != GWN_OK || n == 0) return s;
    hipStream_t st = (hipStream_t)stream;
    return with_async_temp("gwn_scan_inclusive_max_i32", gwn::scan_temp_bytes(n), st,
                           [&](void* tmp) { return gwn::scan_inclusive_max(in, out, n, tmp, st); });
}

}  // extern "C"
