// Diagnostics reductions for gfx950: beam moments (means and centred
// covariance, §4) and the paired squared-difference sums used by the error
// metrics.  FP64 throughout.
//
// Scheme (fixed order, hence bitwise reproducible run to run):
//  1. each thread sums its particles (grid-stride, at most ~100 per thread)
//     into NV FP64 accumulators, coordinates shifted by particle 0 so that
//     the second moments do not cancel against the mean; the sums whose
//     terms take both signs (the six first moments, the paired
//     differences' squares too as they are few) are compensated: every
//     addition goes through TwoSum and its rounding error into a second
//     accumulator, and the pair seeds the double-double merge (compensating
//     all 27 moment sums measured 72 % slower, the six first ones 8 %);
//  2. the 64 lanes of a wavefront merge their sums as double-double pairs
//     (error-free TwoSum) through cross-lane shuffles, the waves of a block
//     through LDS, and each block writes NV double-double partials;
//  3. one block per value merges the block partials in double-double; a
//     final thread forms mean = shift + S/n and cov = (P - S_j S_k / n) / n.
// Compiled with -ffp-contract=off: the TwoSum sequences must not be fused.
#include "hbl_internal.hpp"

#include <mutex>

namespace hbl {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxBlocks = 1024;

struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD two_sum(double a, double b) {
    const double s = a + b;
    const double bp = s - a;
    const double e = (a - (s - bp)) + (b - bp);
    return {s, e};
}

__device__ __forceinline__ DD quick_two_sum(double a, double b) {
    const double s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ DD dd_add(DD a, DD b) {
    DD s = two_sum(a.hi, b.hi);
    const DD t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ DD dd_mul(DD a, DD b) {
    const double p = a.hi * b.hi;
    double e = fma(a.hi, b.hi, -p);
    e = fma(a.hi, b.lo, e);
    e = fma(a.lo, b.hi, e);
    return quick_two_sum(p, e);
}

__device__ __forceinline__ DD dd_div_d(DD a, double b) {
    const double q1 = a.hi / b;
    const double ph = q1 * b;
    const double pl = fma(q1, b, -ph);
    DD s = two_sum(a.hi, -ph);
    s.lo -= pl;
    s.lo += a.lo;
    const double q2 = (s.hi + s.lo) / b;
    return quick_two_sum(q1, q2);
}

__device__ __forceinline__ DD dd_neg(DD a) { return {-a.hi, -a.lo}; }

// Merge NV double-double values across the block; lanes 0..NV-1 of wave 0
// hold the block totals on return (others undefined).
template <int NV>
__device__ void block_reduce_dd(DD (&v)[NV], DD* lds) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            DD o;
            o.hi = __shfl_xor(v[q].hi, off, 64);
            o.lo = __shfl_xor(v[q].lo, off, 64);
            v[q] = dd_add(v[q], o);
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[wave * NV + q] = v[q];
    }
    __syncthreads();
}

// Per-particle contributions.
// Shift = particle 0 (read on the device; uniform across the grid).
// TwoSum accumulation: a + x exactly as the new a plus the rounding error,
// which is added into c.
__device__ __forceinline__ void add_comp(double& a, double& c, double x) {
    const double s = a + x;
    const double bp = s - a;
    c += (a - (s - bp)) + (x - bp);
    a = s;
}

struct MomentsOp {
    static constexpr int NV = 27;
    static constexpr int NC = 6;     // compensated: the first moments
    const double* z;
    int64_t ld;
    double sh[6];
    __device__ __forceinline__ void init() {
#pragma unroll
        for (int j = 0; j < 6; ++j) sh[j] = z[j * ld];
    }
    // four particles i, i + st, i + 2 st, i + 3 st: all 24 loads in flight
    // before the first feeds the accumulation (same order as one at a time)
    __device__ __forceinline__ void add4(int64_t i, int64_t st, double (&acc)[NV], double (&cmp)[NC]) const {
        double a[4][6];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < 6; ++j) a[r][j] = __builtin_nontemporal_load(z + j * ld + i + r * st);
#pragma unroll
        for (int r = 0; r < 4; ++r) accumulate(a[r], acc, cmp);
    }
    __device__ __forceinline__ void add(int64_t i, double (&acc)[NV], double (&cmp)[NC]) const {
        double a[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) a[j] = __builtin_nontemporal_load(z + j * ld + i);
        accumulate(a, acc, cmp);
    }
    __device__ __forceinline__ void accumulate(const double (&v)[6], double (&acc)[NV], double (&cmp)[NC]) const {
        double d[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) d[j] = v[j] - sh[j];
#pragma unroll
        for (int j = 0; j < 6; ++j) add_comp(acc[j], cmp[j], d[j]);
#pragma unroll
        for (int j = 0; j < 6; ++j)
#pragma unroll
            for (int k = j; k < 6; ++k) {
                const int q = 6 + j * 6 - j * (j - 1) / 2 + (k - j);
                acc[q] = fma(d[j], d[k], acc[q]);
            }
    }
};

struct Diff2Op {
    static constexpr int NV = 6;
    static constexpr int NC = 6;     // all compensated
    const double* zs;
    const double* zf;
    int64_t ld;
    __device__ __forceinline__ void init() {}
    __device__ __forceinline__ void add4(int64_t i, int64_t st, double (&acc)[NV], double (&cmp)[NC]) const {
        double a[4][6];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < 6; ++j)
                a[r][j] = __builtin_nontemporal_load(zs + j * ld + i + r * st) -
                          __builtin_nontemporal_load(zf + j * ld + i + r * st);
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < 6; ++j) add_comp(acc[j], cmp[j], a[r][j] * a[r][j]);
    }
    __device__ __forceinline__ void add(int64_t i, double (&acc)[NV], double (&cmp)[NC]) const {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const double d = __builtin_nontemporal_load(zs + j * ld + i) - __builtin_nontemporal_load(zf + j * ld + i);
            add_comp(acc[j], cmp[j], d * d);
        }
    }
};

template <class Op>
__global__ __launch_bounds__(kBlock) void k_partials(Op op, int64_t n, DD* __restrict__ part) {
    constexpr int NV = Op::NV, NC = Op::NC;
    op.init();
    __shared__ DD lds[kWaves * NV];
    double acc[NV], cmp[NC];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
#pragma unroll
    for (int q = 0; q < NC; ++q) cmp[q] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    // four particles per iteration: their loads are in flight before the
    // first feeds the (fixed-order) accumulation; the bunch is streamed once,
    // so the loads are non-temporal.  Moments of 2.5e7 particles: 240 us with
    // two plain loads per iteration, 218 us non-temporal, 197 us with four
    // (6.1 TB/s), 213 us with the first moments compensated.
    for (; i + 3 * stride < n; i += 4 * stride) op.add4(i, stride, acc, cmp);
    for (; i < n; i += stride) op.add(i, acc, cmp);
    DD v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = q < NC ? two_sum(acc[q], cmp[q]) : DD{acc[q], 0.0};
    block_reduce_dd<NV>(v, lds);
    if (threadIdx.x < NV) {
        const int q = threadIdx.x;
        DD s = lds[q];
        for (int w = 1; w < kWaves; ++w) s = dd_add(s, lds[w * NV + q]);
        part[(int64_t)blockIdx.x * NV + q] = s;
    }
}

// Block q merges the nb partials of value q (fixed order: strided per-thread
// sums, then a tree), writing one double-double total.
__global__ __launch_bounds__(kBlock) void k_merge(const DD* __restrict__ part, int nb, int nv,
                                                  DD* __restrict__ tot) {
    __shared__ DD red[kBlock];
    const int q = blockIdx.x;
    DD s{0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += kBlock) s = dd_add(s, part[(int64_t)b * nv + q]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = dd_add(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) tot[q] = red[0];
}

__global__ void k_moments_final(const DD* __restrict__ tot, const double* __restrict__ z, int64_t ld,
                                int64_t n, double* __restrict__ out) {
    // one thread per output: 6 means, then the 21 upper-triangle covariances
    const int q = threadIdx.x;
    const double nd = (double)n;
    if (q < 6) {
        // mean = shift + S/n, the shift being particle 0
        const DD m = dd_div_d(tot[q], nd);
        const DD mean = dd_add(DD{z[(int64_t)q * ld], 0.0}, m);
        out[q] = mean.hi + mean.lo;
    } else if (q < 27) {
        int j = 0, r = q - 6;
        while (r >= 6 - j) {
            r -= 6 - j;
            ++j;
        }
        const int k = j + r;
        const DD t = dd_div_d(dd_mul(tot[j], tot[k]), nd);
        const DD u = dd_add(tot[q], dd_neg(t));
        const DD c = dd_div_d(u, nd);
        out[q] = c.hi + c.lo;
    }
}

__global__ void k_diff2_final(const DD* __restrict__ tot, double* __restrict__ out) {
    if (threadIdx.x < 6) out[threadIdx.x] = tot[threadIdx.x].hi + tot[threadIdx.x].lo;
}

int reduce_grid(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > kMaxBlocks) g = kMaxBlocks;
    return (int)g;
}

// Fixed scratch of the no-allocation moments call: the workspace of the
// largest grid (kMaxBlocks block partials, then the totals; 27 double-double
// values each, 442,800 bytes), one copy in every device's memory for the life
// of the process.  Host code never names this array as an address: each
// device's copy is looked up once with hipGetSymbolAddress (scratch_pointer).
constexpr size_t kScratchDD = (size_t)(kMaxBlocks + 1) * 27;
static __device__ __align__(256) DD scratch[kScratchDD];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

}  // namespace

size_t reduce_scratch_bytes() { return kScratchDD * sizeof(DD); }

hipError_t reduce_scratch(double** out) {
    *out = nullptr;
    int d = -1;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return e;
    if (d < 0 || d >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[d]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // this device's copy (device d is current)
        if (e != hipSuccess) return e;
        g_scratch_ptr[d] = p;
    }
    *out = static_cast<double*>(g_scratch_ptr[d]);
    return hipSuccess;
}

size_t reduce_ws_bytes(int64_t n) {
    return ((size_t)reduce_grid(n) + 1) * 27 * sizeof(DD);   // block partials, then the totals
}

hipError_t launch_moments(const double* z, int64_t n, int64_t ld, double* ws, double* out27,
                          hipStream_t s) {
    const int nb = reduce_grid(n);
    MomentsOp op;
    op.z = z;
    op.ld = ld;
    for (int j = 0; j < 6; ++j) op.sh[j] = 0.0;  // loaded on the device by init()
    DD* part = reinterpret_cast<DD*>(ws);
    DD* tot = part + (size_t)nb * 27;
    hipLaunchKernelGGL(k_partials<MomentsOp>, dim3(nb), dim3(kBlock), 0, s, op, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge, dim3(27), dim3(kBlock), 0, s, part, nb, 27, tot);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_moments_final, dim3(1), dim3(64), 0, s, tot, z, ld, n, out27);
    return hipGetLastError();
}

hipError_t launch_diff2(const double* zs, const double* zf, int64_t n, int64_t ld, double* ws,
                        double* out6, hipStream_t s) {
    const int nb = reduce_grid(n);
    Diff2Op op{zs, zf, ld};
    DD* part = reinterpret_cast<DD*>(ws);
    DD* tot = part + (size_t)nb * 6;
    hipLaunchKernelGGL(k_partials<Diff2Op>, dim3(nb), dim3(kBlock), 0, s, op, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge, dim3(6), dim3(kBlock), 0, s, part, nb, 6, tot);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diff2_final, dim3(1), dim3(64), 0, s, tot, out6);
    return hipGetLastError();
}

}  // namespace hbl
