// Kernels of the wide PReLU surrogate (the network shape the paper trains,
// §3 Eq. 2 and 3: several hidden layers of equal width W in the hundreds,
// PReLU with one learned slope per hidden layer).  At W = 700-900 a particle
// costs 2-6.5 MFLOP, so the dense layers are true matrix products and run as
// tiled bf16 GEMMs on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation), one launch per layer over a chunk of particles whose bf16
// activations stay in two ping-pong buffers.
//
// Layout.  Activations X: [rows][Wp] bf16, particle-major (a particle's
// features contiguous), Wp = W rounded up to 64; rows = the chunk rounded up
// to the 256-particle tile; padded features hold exact zeros, padded
// particles are computed from a zero input and never written back.  Weights
// of a W x W layer: [Wp][Wp] bf16 row-major ([out][in]) with zero padding;
// the output layer: [16][Wp] (rows 6..15 zero); biases FP32, padded.
//
// GEMM (layer l, D^T = W X^T): the out-features are the MFMA A operand
// (rows), particles the B operand (columns), so a lane's 4 accumulators are
// 4 consecutive out-features of one particle and the bf16 result row is
// written with 8-byte stores.  Workgroup = 4 waves; a wave owns NT x 16
// particles (NT = 4: a 256-particle tile per workgroup) and all MT x 16
// out-features of its workgroup's M block.  Both operands stream through LDS
// in K chunks of 32 with the direct-to-LDS load (no registers held for the
// chunks in flight) through a ring of 4 stages: chunks k + 1 .. k + 3 are in
// flight while chunk k feeds the matrix cores; the M block's weights are
// shared by the four waves, each wave stages its own particles.
//
// Matrix-core layout (16x16x32, lane l, g = l / 16, r = l % 16):
//   A (16 x 32): row r, k = 8g .. 8g+7;  B (32 x 16): column r, k = 8g .. 8g+7
//   D (16 x 16): column r, rows 4g .. 4g+3
#include "hbl_elements.hpp"

namespace hbl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;
constexpr int kNT = 4;                         // 16-particle MFMA tiles per wave
constexpr int kKc = 32;                        // K chunk staged in LDS

__device__ __forceinline__ uint32_t pack2(float a, float b) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    bf16x2 v;
    v[0] = (__bf16)a;                          // round to nearest even
    v[1] = (__bf16)b;
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ float prelu(float v, float a) { return v > 0.0f ? v : a * v; }

// XCD-aware tile order: workgroups are dealt to the 8 XCDs round-robin by
// id, so the M blocks of one particle tile are given ids on the same XCD
// and close in time (their shared activation rows then hit that XCD's L2).
__device__ __forceinline__ void tile_of(int id, int mblocks, int& m, int& tile) {
    const int xcd = id & 7, local = id >> 3;
    m = local % mblocks;
    tile = (local / mblocks) * 8 + xcd;
}

// ------------------------------------------------------------ packing
__global__ void k_pack_bf16(const float* __restrict__ src, int rows, int cols, uint16_t* __restrict__ dst,
                            int rows_p, int cols_p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)rows_p * cols_p) return;
    const int r = (int)(i / cols_p), c = (int)(i % cols_p);
    const float v = (r < rows && c < cols) ? src[(int64_t)r * cols + c] : 0.0f;
    dst[i] = __builtin_bit_cast(uint16_t, (__bf16)v);
}

__global__ void k_pack_f32(const float* __restrict__ src, int n, float* __restrict__ dst, int n_p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_p) dst[i] = i < n ? src[i] : 0.0f;
}

// ------------------------------------------------------------ input layer
// 6 -> W on the vector ALU in FP32 (the network input needs more than bf16's
// 8 bits).  Block of 256 particles: each thread forms one particle's
// normalised input into LDS; then thread t keeps the weights of feature
// group t % G (8 features, G = Wp/8) in registers and walks the particles
// of its set t / G, so consecutive threads write consecutive 16-B pieces of
// one activation row.
constexpr int kInP = 256;

template <bool GAPS, bool CHROM>
__global__ __launch_bounds__(kBlock) void k_dense_input(const double* __restrict__ z, int64_t nend, int64_t ld,
                                                        int64_t p0, DenseImage im, DenseNorm nm,
                                                        LatticeView pre, uint16_t* __restrict__ x) {
    __shared__ float xs[kInP][6];
    const int tid = threadIdx.x;
    {
        const int64_t i = p0 + (int64_t)blockIdx.x * kInP + tid;
        float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (i < nend) {
            P6 p;
            load6(z, ld, i, p);
            if (GAPS) apply_elements<CHROM>(p, pre);
            const double pv[6] = {p.x, p.y, p.t, p.px, p.py, p.pt};
#pragma unroll
            for (int j = 0; j < 6; ++j) v[j] = (float)((pv[j] - nm.mu_in[j]) / nm.sd_in[j]);
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) xs[tid][j] = v[j];
    }
    __syncthreads();
    const int groups = im.wp / 8, sets = kBlock / groups;
    const int gq = tid % groups, set = tid / groups;
    if (set >= sets) return;                  // no barrier follows
    float w[8][6], b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        b[j] = im.b0[gq * 8 + j];
#pragma unroll
        for (int c = 0; c < 6; ++c) w[j][c] = im.w0[(gq * 8 + j) * 6 + c];
    }
    const float a0 = im.slope[0];
    uint16_t* xb = x + (int64_t)blockIdx.x * kInP * im.wp + gq * 8;
    for (int q = set; q < kInP; q += sets) {
        float h[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float acc = b[j];
#pragma unroll
            for (int c = 0; c < 6; ++c) acc = fmaf(w[j][c], xs[q][c], acc);
            h[j] = prelu(acc, a0);
        }
        *(u32x4*)(xb + (int64_t)q * im.wp) = u32x4{pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]), pack2(h[6], h[7])};
    }
}

// ------------------------------------------------------------ dense layer
struct LayerArgs {
    const uint16_t* x;     // [rows][K]
    const uint16_t* w;     // [Mp][K]
    const float* bias;     // [Mp]
    const float* slope;    // this layer's PReLU slope (hidden layers)
    uint16_t* y;           // [rows][Mp] (hidden layers)
    int K, Mp, mblocks, tiles;
    // output layer: particles p0 + row for rows with p0 + row < nend
    double* z;
    int64_t ld, p0, nend;
};

enum { kEpiHidden = 0, kEpiOut = 1 };

// LDS tiles hold 64-byte rows (one K chunk of 32 bf16) with the 16-B
// pieces of row R stored at position piece ^ swz(R): any 16 consecutive rows
// read at one piece hit distinct 16-B bank groups, for 8 as well as for 16
// lanes per LDS cycle, so the matrix-core operand reads are conflict-free.
constexpr int kStages = 4;                     // LDS ring: chunks k+1..k+3 in flight
__device__ __forceinline__ int swz(int row) { return ((row >> 1) ^ (row >> 3)) & 3; }

// 16 rows x 64 B of a row-major bf16 matrix (row stride K elements) into
// 1 KB of LDS with the direct-to-LDS load: lane L fills position L % 4 of
// row L / 4, i.e. loads piece (L % 4) ^ swz(row) of that row.
__device__ __forceinline__ void dma_rows16(const uint16_t* src_row0, int K, int row_base, int k0,
                                           __attribute__((address_space(3))) void* lds, int lane) {
    const int rr = lane >> 2, piece = (lane & 3) ^ swz(row_base + rr);
    __builtin_amdgcn_global_load_lds(src_row0 + (int64_t)rr * K + k0 + piece * 8, lds, 16, 0, 0);
}

// s_waitcnt with only the vector-memory counter: at most n loads outstanding.
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <int MT, int EPI, bool GAPS, bool CHROM>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_dense_layer(LayerArgs a, DenseNorm nm,
                                                                                                LatticeView post) {
    constexpr int ROWS = MT * 16;                       // out-features of this M block
    constexpr int PROWS = kWaves * kNT * 16;            // particles of this tile
    constexpr int A_BYTES = ROWS * 64, B_BYTES = PROWS * 64, STAGE = A_BYTES + B_BYTES;
    // direct-to-LDS loads per wave per chunk: the M block's MT pieces of 1 KB
    // dealt over the waves (a wave past the last piece reloads it, so that
    // every wave issues the same count), and its own kNT pieces of particles
    constexpr int A_PER_WAVE = (MT + kWaves - 1) / kWaves, PER_CHUNK = A_PER_WAVE + kNT;
    __shared__ __attribute__((aligned(1024))) char smem[kStages * STAGE];
    int m, tile;
    tile_of(blockIdx.x, a.mblocks, m, tile);
    if (tile >= a.tiles) return;                        // whole workgroup: no barrier follows
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, r = lane & 15;
    const int K = a.K;
    const uint16_t* wblk = a.w + (int64_t)m * ROWS * K;
    const int64_t wrow0 = (int64_t)tile * PROWS + wave * (kNT * 16);   // this wave's first particle row
    const uint16_t* xw = a.x + wrow0 * K;
    typedef __attribute__((address_space(3))) char lds_char;
    lds_char* sm = (lds_char*)smem;

    auto issue = [&](int kc) {
        lds_char* A = sm + (kc % kStages) * STAGE;
        lds_char* B = A + A_BYTES + wave * (kNT * 16 * 64);
        const int k0 = kc * kKc;
#pragma unroll
        for (int i = 0; i < A_PER_WAVE; ++i) {
            const int j = min(wave + i * kWaves, MT - 1);
            dma_rows16(wblk + (int64_t)(j * 16) * K, K, j * 16, k0, A + j * 1024, lane);
        }
#pragma unroll
        for (int i = 0; i < kNT; ++i) dma_rows16(xw + (int64_t)(i * 16) * K, K, i * 16, k0, B + i * 1024, lane);
    };

    f32x4 acc[MT][kNT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

    // operands of one chunk, read from LDS into registers
    struct Ops {
        bf16x8 a[MT];
        bf16x8 b[kNT];
    };
    auto read_ops = [&](int kc, Ops& o) {
        const lds_char* A = sm + (kc % kStages) * STAGE;
        const lds_char* B = A + A_BYTES + wave * (kNT * 16 * 64);
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
            const int pr = nt * 16 + r;
            o.b[nt] = *(const __attribute__((address_space(3))) bf16x8*)(B + pr * 64 + ((g ^ swz(pr)) * 16));
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int ar = mt * 16 + r;
            o.a[mt] = *(const __attribute__((address_space(3))) bf16x8*)(A + ar * 64 + ((g ^ swz(ar)) * 16));
        }
    };
    auto products = [&](const Ops& o) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.a[mt], o.b[nt], acc[mt][nt], 0, 0, 0);
    };
    const int nk = K / kKc;                             // even: Wp is a multiple of 64
    // make chunk c readable: this wave's loads of it have landed (only the
    // loads of the chunks after it may be pending) and its reads of chunk
    // c - 1 are done; after the barrier the same holds for every wave, so
    // chunk c - 1's stage takes the loads of chunk c + 3.
    auto sync_for = [&](int c) {
        if (c + 2 < nk) wait_vm<2 * PER_CHUNK>();
        else if (c + 1 < nk) wait_vm<PER_CHUNK>();
        else wait_vm<0>();
        __builtin_amdgcn_s_waitcnt(0xC07F);             // lgkmcnt(0) only
        asm volatile("s_barrier" ::: "memory");        // a fence here would wait for every chunk in flight
        if (c + kStages - 1 < nk) issue(c + kStages - 1);
    };

#pragma unroll
    for (int kc = 0; kc < kStages - 1; ++kc)
        if (kc < nk) issue(kc);
    Ops o0, o1;
    sync_for(0);
    read_ops(0, o0);
    // chunk kc's operands are in flight into o0; the next chunk's reads
    // overlap chunk kc's products, and so on (the last pair is peeled so that
    // no branch joins reads in flight with reads completed)
    auto half = [&](int c, Ops& next, const Ops& cur) {
        sync_for(c);
        read_ops(c, next);
        products(cur);
        __builtin_amdgcn_sched_group_barrier(0x100, kNT + MT, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, MT * kNT, 0);
    };
    for (int kc = 0; kc + 2 < nk; kc += 2) {
        half(kc + 1, o1, o0);
        half(kc + 2, o0, o1);
    }
    half(nk - 1, o1, o0);
    products(o1);
    const int64_t row0 = wrow0 + r;

    if (EPI == kEpiHidden) {
        const float s = *a.slope;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int o = m * ROWS + mt * 16 + 4 * g;
            const f32x4 bb = *(const f32x4*)(a.bias + o);
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) {
                const f32x4 v = acc[mt][nt];
                const u32x2 st = {pack2(prelu(v[0] + bb[0], s), prelu(v[1] + bb[1], s)),
                                  pack2(prelu(v[2] + bb[2], s), prelu(v[3] + bb[3], s))};
                *(u32x2*)(a.y + (row0 + nt * 16) * a.Mp + o) = st;
            }
        }
    } else {
        // output layer: rows 4g + i, i < 4; outputs 0..5 live in lanes g = 0, 1
        const f32x4 bb = *(const f32x4*)(a.bias + 4 * g);
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
            const f32x4 v = acc[0][nt] + bb;
            const float o4 = __shfl(v[0], 16 + r, 64), o5 = __shfl(v[1], 16 + r, 64);
            const int64_t i = a.p0 + row0 + nt * 16;
            if (g == 0 && i < a.nend) {
                P6 q;
                q.x = fma(nm.sd_out[0], (double)v[0], nm.mu_out[0]);
                q.y = fma(nm.sd_out[1], (double)v[1], nm.mu_out[1]);
                q.t = fma(nm.sd_out[2], (double)v[2], nm.mu_out[2]);
                q.px = fma(nm.sd_out[3], (double)v[3], nm.mu_out[3]);
                q.py = fma(nm.sd_out[4], (double)o4, nm.mu_out[4]);
                q.pt = fma(nm.sd_out[5], (double)o5, nm.mu_out[5]);
                if (GAPS) apply_elements<CHROM>(q, post);
                store6(a.z, a.ld, i, q);
            }
        }
    }
}

template <int MT>
hipError_t launch_hidden_mt(const LayerArgs& a, hipStream_t s) {
    const LatticeView none{};
    const DenseNorm nm{};
    const int grid = a.mblocks * ((a.tiles + 7) / 8) * 8;
    hipLaunchKernelGGL((k_dense_layer<MT, kEpiHidden, false, false>), dim3(grid), dim3(kBlock), 0, s, a, nm, none);
    return hipGetLastError();
}

typedef hipError_t (*HiddenLauncher)(const LayerArgs&, hipStream_t);
constexpr int kMaxMT = 12;      // accumulators MT x NT x 4 <= 192 stay in the AGPR file
const HiddenLauncher kHidden[kMaxMT] = {
    launch_hidden_mt<1>, launch_hidden_mt<2>, launch_hidden_mt<3>, launch_hidden_mt<4>,
    launch_hidden_mt<5>, launch_hidden_mt<6>, launch_hidden_mt<7>, launch_hidden_mt<8>,
    launch_hidden_mt<9>, launch_hidden_mt<10>, launch_hidden_mt<11>, launch_hidden_mt<12>};

// M block of a W x W layer: the largest MT <= kMaxMT dividing Wp / 16 (Wp is
// a multiple of 64, so 4 always divides it).
int hidden_mt(int wp) {
    const int tiles = wp / 16;
    for (int mt = kMaxMT; mt >= 1; --mt)
        if (tiles % mt == 0) return mt;
    return 1;
}

}  // namespace

hipError_t launch_dense_pack(const float* params, const DenseShape& sh, const DenseImage& im, hipStream_t s) {
    const int W = sh.width, Wp = im.wp, H = sh.hidden;
    int64_t off = 0;
    for (int l = 0; l <= H; ++l) {
        const int ni = l == 0 ? 6 : W, no = l == H ? 6 : W;
        const float* A = params + off;
        const float* b = A + (int64_t)no * ni;
        if (l == 0) {
            hipLaunchKernelGGL(k_pack_f32, dim3((Wp * 6 + 255) / 256), dim3(256), 0, s, A, W * 6, im.w0, Wp * 6);
            hipLaunchKernelGGL(k_pack_f32, dim3((Wp + 255) / 256), dim3(256), 0, s, b, W, im.b0, Wp);
        } else {
            const int rows_p = l == H ? 16 : Wp;
            const int64_t cnt = (int64_t)rows_p * Wp;
            hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, A, no, ni,
                               im.w[l], rows_p, Wp);
            hipLaunchKernelGGL(k_pack_f32, dim3((rows_p + 255) / 256), dim3(256), 0, s, b, no, im.b[l], rows_p);
        }
        off += (int64_t)no * (ni + 1);
        if (l < H) {
            hipLaunchKernelGGL(k_pack_f32, dim3(1), dim3(64), 0, s, params + off, 1, im.slope + l, 1);
            off += 1;
        }
    }
    return hipGetLastError();
}

int dense_tile_rows() { return kWaves * kNT * 16; }

hipError_t launch_dense_infer(double* z, int64_t n, int64_t ld, const DenseShape& sh, const DenseImage& im,
                              const DenseNorm& nm, const LatticeView& pre, const LatticeView& post,
                              uint16_t* buf0, uint16_t* buf1, int64_t chunk, hipStream_t s) {
    const int Wp = im.wp, H = sh.hidden, MT = hidden_mt(Wp);
    const int tile = dense_tile_rows();
    const bool gaps = pre.n > 0 || post.n > 0;
    const bool chrom = pre.chromatic || post.chromatic;
    for (int64_t p0 = 0; p0 < n; p0 += chunk) {
        const int64_t nc = n - p0 < chunk ? n - p0 : chunk, nend = p0 + nc;
        const int tiles = (int)((nc + tile - 1) / tile);
        const int64_t rows = (int64_t)tiles * tile;
        const dim3 gin((unsigned)(rows / kInP));
        if (!gaps)
            hipLaunchKernelGGL((k_dense_input<false, false>), gin, dim3(kBlock), 0, s, z, nend, ld, p0, im, nm, pre, buf0);
        else if (!chrom)
            hipLaunchKernelGGL((k_dense_input<true, false>), gin, dim3(kBlock), 0, s, z, nend, ld, p0, im, nm, pre, buf0);
        else
            hipLaunchKernelGGL((k_dense_input<true, true>), gin, dim3(kBlock), 0, s, z, nend, ld, p0, im, nm, pre, buf0);
        uint16_t* xin = buf0;
        uint16_t* yout = buf1;
        for (int l = 1; l < H; ++l) {
            LayerArgs a{};
            a.x = xin; a.w = im.w[l]; a.bias = im.b[l]; a.slope = im.slope + l; a.y = yout;
            a.K = Wp; a.Mp = Wp; a.mblocks = Wp / (16 * MT); a.tiles = tiles;
            hipError_t e = kHidden[MT - 1](a, s);
            if (e != hipSuccess) return e;
            uint16_t* t = xin; xin = yout; yout = t;
        }
        LayerArgs a{};
        a.x = xin; a.w = im.w[H]; a.bias = im.b[H]; a.K = Wp; a.Mp = 16; a.mblocks = 1; a.tiles = tiles;
        a.z = z; a.ld = ld; a.p0 = p0; a.nend = nend;
        const dim3 gout((unsigned)(((tiles + 7) / 8) * 8));
        if (!gaps)
            hipLaunchKernelGGL((k_dense_layer<1, kEpiOut, false, false>), gout, dim3(kBlock), 0, s, a, nm, post);
        else if (!chrom)
            hipLaunchKernelGGL((k_dense_layer<1, kEpiOut, true, false>), gout, dim3(kBlock), 0, s, a, nm, post);
        else
            hipLaunchKernelGGL((k_dense_layer<1, kEpiOut, true, true>), gout, dim3(kBlock), 0, s, a, nm, post);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hbl
