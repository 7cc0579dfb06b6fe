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
// K-blocked layout (inference at 512 <= Wp <= 960, dense_blocked): the same
// matrices cut into K chunks of 32, [Wp/32][rows][32], so that the 64 bytes
// of one row in one chunk sit next to those of the following rows and the
// operand loads of a chunk read whole 128-byte lines (row-major rows put
// half a line in one chunk and the other half in the next).
//
// GEMM (layer l, D^T = W X^T): the out-features are the MFMA A operand
// (rows), particles the B operand (columns), so a lane's 4 accumulators are
// 4 consecutive out-features of one particle and the bf16 result row is
// written with 8-byte stores.  Workgroup = 4 waves; a wave owns NT x 16
// particles (NT = 4: a 256-particle tile per workgroup) and all MT x 16
// out-features of its workgroup's M block (or 8 waves, two per SIMD, each
// with half of them: the form used for 12-tile M blocks).  Both operands stream through LDS
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
                            int rows_p, int cols_p, int blocked) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)rows_p * cols_p) return;
    const int r = (int)(i / cols_p), c = (int)(i % cols_p);
    const float v = (r < rows && c < cols) ? src[(int64_t)r * cols + c] : 0.0f;
    const int64_t d = blocked ? (int64_t)(c >> 5) * rows_p * 32 + (int64_t)r * 32 + (c & 31) : i;
    dst[d] = __builtin_bit_cast(uint16_t, (__bf16)v);
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

template <bool GAPS, bool CHROM, bool BLK>
__global__ __launch_bounds__(kBlock) void k_dense_input(const double* __restrict__ z, int64_t nend, int64_t ld,
                                                        int64_t p0, DenseImage im, DenseNorm nm,
                                                        LatticeView pre, uint16_t* __restrict__ x, int64_t rows) {
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
    // row-major: row stride wp; K-blocked: features 8 gq .. 8 gq + 7 lie in
    // chunk gq / 4 at offset 8 (gq % 4), row stride 32
    const int64_t rstride = BLK ? 32 : im.wp;
    uint16_t* xb = BLK ? x + (int64_t)(gq >> 2) * rows * 32 + (int64_t)blockIdx.x * kInP * 32 + (gq & 3) * 8
                       : x + (int64_t)blockIdx.x * kInP * im.wp + gq * 8;
    for (int q = set; q < kInP; q += sets) {
        float h[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float acc = b[j];
#pragma unroll
            for (int c = 0; c < 6; ++c) acc = fmaf(w[j][c], xs[q][c], acc);
            h[j] = prelu(acc, a0);
        }
        *(u32x4*)(xb + (int64_t)q * rstride) = u32x4{pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]), pack2(h[6], h[7])};
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
    // training (rows = batch samples, ldt = padded batch)
    uint16_t* v;           // [rows][Mp] pre-activations (forward) / read (backward)
    uint16_t* yt;          // [Mp][ldt] transposed output, or nullptr
    int ldt;
    float* part;           // one partial sum per workgroup (backward: slope gradient)
    // gradient GEMM: rows o < W of the M operand; "particle" rows k < gcols are
    // weight columns (grad[o * gcols + k]), row bias_row carries the bias (gradb[o])
    float* grad;
    float* gradb;
    int W, gcols, bias_row;
};

// kEpiHidden: y = bf16(prelu(acc + b)).  kEpiOut: de-normalised FP64 output.
// kEpiTrain: kEpiHidden, also keeping v = bf16(acc + b) and the transposed y.
// kEpiBwd: acc = dL/dh of the layer below (weights transposed); writes its
//   dL/dv = acc * prelu'(v) as y and transposed, and the workgroup's share
//   of the slope gradient, sum of acc * v over v <= 0.
// kEpiGrad: acc = weight gradient [o][k] (o: rows, k: "particle" rows), FP32.
enum { kEpiHidden = 0, kEpiOut = 1, kEpiTrain = 2, kEpiBwd = 3, kEpiGrad = 4 };

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

// WM = 1: 4 waves, each with all MT row tiles of the M block and 64
// particles; WM = 2: 8 waves (two per SIMD, so one can issue products while
// the other waits), each with half the row tiles.
template <int MT, int WM, int EPI, bool GAPS, bool CHROM, bool BX = false>
__global__ __launch_bounds__(256 * WM) __attribute__((amdgpu_waves_per_eu(WM, WM))) void k_dense_layer(
    LayerArgs a, DenseNorm nm, LatticeView post) {
    static_assert(MT % WM == 0, "the M block splits evenly over the wave rows");
    constexpr int NW = 4 * WM, MTW = MT / WM;           // waves; MFMA row tiles per wave
    constexpr int ROWS = MT * 16;                       // out-features of this M block
    constexpr int PROWS = 4 * kNT * 16;                 // particles of this tile
    constexpr int A_BYTES = ROWS * 64, B_BYTES = PROWS * 64, STAGE = A_BYTES + B_BYTES;
    // direct-to-LDS loads per wave per chunk: the M block's MT pieces of 1 KB
    // dealt over the waves (a wave past the last piece reloads it, so that
    // every wave issues the same count), and an equal share of the tile's 16
    // pieces of particle rows
    constexpr int A_PER_WAVE = (MT + NW - 1) / NW, B_PER_WAVE = 4 * kNT / NW;
    constexpr int PER_CHUNK = A_PER_WAVE + B_PER_WAVE;
    __shared__ __attribute__((aligned(1024))) char smem[kStages * STAGE];
    int m, tile;
    tile_of(blockIdx.x, a.mblocks, m, tile);
    if (tile >= a.tiles) {                              // whole workgroup: no barrier follows
        if (EPI == kEpiBwd && threadIdx.x == 0) a.part[blockIdx.x] = 0.0f;
        return;
    }
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, r = lane & 15;
    const int wm = wave >> 2, wn = wave & 3;            // wave row (out-features) and column (particles)
    const int K = a.K;
    const uint16_t* wblk = a.w + (int64_t)m * ROWS * K;
    const int64_t wrow0 = (int64_t)tile * PROWS + wn * (kNT * 16);     // this wave's first particle row
    const uint16_t* xt = a.x + (int64_t)tile * PROWS * K;               // the tile's particle rows
    typedef __attribute__((address_space(3))) char lds_char;
    lds_char* sm = (lds_char*)smem;

    auto issue = [&](int kc) {
        lds_char* A = sm + (kc % kStages) * STAGE;
        lds_char* B = A + A_BYTES;
        const int k0 = kc * kKc;
#pragma unroll
        for (int i = 0; i < A_PER_WAVE; ++i) {
            const int j = min(wave + i * NW, MT - 1);
            dma_rows16(wblk + (int64_t)(j * 16) * K, K, j * 16, k0, A + j * 1024, lane);
        }
#pragma unroll
        for (int i = 0; i < B_PER_WAVE; ++i) {
            const int j = wave * B_PER_WAVE + i;       // tile rows 16j .. 16j+15
            if (BX)                                    // K-blocked X: 1 KB contiguous
                dma_rows16(a.x + ((int64_t)kc * a.tiles * PROWS + (int64_t)tile * PROWS + j * 16) * 32, 32,
                           (j * 16) & 63, 0, B + j * 1024, lane);
            else
                dma_rows16(xt + (int64_t)(j * 16) * K, K, (j * 16) & 63, k0, B + j * 1024, lane);
        }
    };

    f32x4 acc[MTW][kNT];
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

    // operands of one chunk, read from LDS into registers
    struct Ops {
        bf16x8 a[MTW];
        bf16x8 b[kNT];
    };
    auto read_ops = [&](int kc, Ops& o) {
        const lds_char* A = sm + (kc % kStages) * STAGE + wm * (MTW * 16 * 64);
        const lds_char* B = sm + (kc % kStages) * STAGE + A_BYTES + wn * (kNT * 16 * 64);
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
            const int pr = nt * 16 + r;
            o.b[nt] = *(const __attribute__((address_space(3))) bf16x8*)(B + pr * 64 + ((g ^ swz(pr)) * 16));
        }
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
            const int ar = mt * 16 + r;                 // row within this wave's rows; the
            const int arow = wm * (MTW * 16) + ar;      // swizzle follows the M-block row
            o.a[mt] = *(const __attribute__((address_space(3))) bf16x8*)(A + ar * 64 + ((g ^ swz(arow)) * 16));
        }
    };
    auto products = [&](const Ops& o) {
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt)
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
        __builtin_amdgcn_sched_group_barrier(0x100, kNT + MTW, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, MTW * kNT, 0);
    };
    for (int kc = 0; kc + 2 < nk; kc += 2) {
        half(kc + 1, o1, o0);
        half(kc + 2, o0, o1);
    }
    half(nk - 1, o1, o0);
    products(o1);
    const int64_t row0 = wrow0 + r;

    if (EPI == kEpiTrain) {
        const float s = *a.slope;
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
            const int o = m * ROWS + wm * (MTW * 16) + mt * 16 + 4 * g;
            const f32x4 bb = *(const f32x4*)(a.bias + o);
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) {
                const int64_t p = row0 + nt * 16;
                const f32x4 v = acc[mt][nt] + bb;
                const float h0 = prelu(v[0], s), h1 = prelu(v[1], s), h2 = prelu(v[2], s), h3 = prelu(v[3], s);
                *(u32x2*)(a.y + p * a.Mp + o) = u32x2{pack2(h0, h1), pack2(h2, h3)};
                *(u32x2*)(a.v + p * a.Mp + o) = u32x2{pack2(v[0], v[1]), pack2(v[2], v[3])};
                if (a.yt) {
                    const float hh[4] = {h0, h1, h2, h3};
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        a.yt[(int64_t)(o + i) * a.ldt + p] = __builtin_bit_cast(uint16_t, (__bf16)hh[i]);
                }
            }
        }
    } else if (EPI == kEpiBwd) {
        const float s = *a.slope;
        float sp = 0.0f;
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
            const int k = m * ROWS + wm * (MTW * 16) + mt * 16 + 4 * g;
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) {
                const int64_t p = row0 + nt * 16;
                const f32x4 dh = acc[mt][nt];
                const u32x2 vw = *(const u32x2*)(a.v + p * a.Mp + k);
                const float vv[4] = {__uint_as_float(vw[0] << 16), __uint_as_float(vw[0] & 0xffff0000u),
                                     __uint_as_float(vw[1] << 16), __uint_as_float(vw[1] & 0xffff0000u)};
                float dv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const bool pos = vv[i] > 0.0f;
                    dv[i] = pos ? dh[i] : s * dh[i];
                    sp += pos ? 0.0f : dh[i] * vv[i];
                    a.yt[(int64_t)(k + i) * a.ldt + p] = __builtin_bit_cast(uint16_t, (__bf16)dv[i]);
                }
                *(u32x2*)(a.y + p * a.Mp + k) = u32x2{pack2(dv[0], dv[1]), pack2(dv[2], dv[3])};
            }
        }
        // workgroup sum of the slope-gradient share (fixed order)
        for (int off = 32; off >= 1; off >>= 1) sp += __shfl_xor(sp, off, 64);
        __shared__ float red[NW];
        if (lane == 0) red[wave] = sp;
        __syncthreads();
        if (tid == 0) {
            float t = 0.0f;
            for (int w = 0; w < NW; ++w) t += red[w];
            a.part[blockIdx.x] = t;
        }
    } else if (EPI == kEpiGrad) {
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
            const int o = m * ROWS + wm * (MTW * 16) + mt * 16 + 4 * g;
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) {
                const int64_t k = row0 + nt * 16;
                const f32x4 gv = acc[mt][nt];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (o + i >= a.W) continue;
                    if (k < a.gcols) a.grad[(int64_t)(o + i) * a.gcols + k] = gv[i];
                    else if (k == a.bias_row) a.gradb[o + i] = gv[i];
                }
            }
        }
    } else if (EPI == kEpiHidden) {
        const float s = *a.slope;
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
            const int o = m * ROWS + wm * (MTW * 16) + mt * 16 + 4 * g;
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


// Hidden layer of inference on K-blocked X, W and Y, at MT = Wp/64 row tiles
// per M block (4 M blocks).  Each wave's 64 particles are its own, so the
// particle operand goes from global memory straight into registers (a ring
// of 5 chunks, loads 3 chunks ahead) and only the M block's weights go
// through LDS (direct-to-LDS, a ring of 4 stages shared by the four waves).
// NK = Wp/32 K chunks, fixed at compile time: the loop is unrolled and every
// ring slot is a constant.  Each accumulator takes its chunks in order, one
// 16x16x32 product per chunk, as in k_dense_layer: the two kernels give the
// same bits.  An item is one (M block, 256-particle tile).  PERSIST: a
// workgroup per CU walks items id, id + G, ...; after an item's last
// products it starts the next item's first three chunks, so that their
// loads fly during this item's epilogue (the biases come through LDS, so
// that the epilogue does not wait on the vector-memory counter behind
// them).  Without PERSIST (MT 14 and 15, whose register budget does not hold
// the next item's operands beside the epilogue) one item per workgroup.
constexpr int kBlkMinMT = 8, kBlkMaxMT = 15, kBlkPersistMaxMT = 13;
constexpr int kPersistGroups = 256;                  // one workgroup per compute unit (a multiple of the 8 XCDs)
template <int MT, bool PERSIST>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_dense_hidden_blk(LayerArgs a,
                                                                                                       int n_items) {
    constexpr int NK = 2 * MT, K = NK * kKc, ROWS = MT * 16, PROWS = kWaves * kNT * 16, A_BYTES = ROWS * 64;
    constexpr int A_PER_WAVE = (MT + kWaves - 1) / kWaves, PER_CHUNK = A_PER_WAVE + kNT, BR = kStages + 1;
    static_assert(MT <= kBlkMaxMT, "MT x 4 x 4 accumulators fit the 256 accumulator registers");
    static_assert(ROWS * 4 <= 1024, "an M block's biases fit one 1 KB LDS buffer");
    __shared__ __attribute__((aligned(1024))) char smem[kStages * A_BYTES + 2048];
    const int G = PERSIST ? (int)gridDim.x : n_items;   // item stride
    int id = blockIdx.x, m = 0, tile = 0;
    auto valid = [&](int i, int& mm, int& tt) {
        if (i >= n_items) return false;
        tile_of(i, a.mblocks, mm, tt);
        return tt < a.tiles;
    };
    while (id < n_items && !valid(id, m, tile)) id += G;
    if (id >= n_items) return;                          // whole workgroup: no barrier follows
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, r = lane & 15;
    const int64_t R = (int64_t)a.tiles * PROWS;         // rows of this launch's X and Y
    typedef __attribute__((address_space(3))) char lds_char;
    lds_char* sm = (lds_char*)smem;
    lds_char* bias_lds = sm + kStages * A_BYTES;        // two 1 KB buffers, by item parity
    bf16x8 bq[BR][kNT];                                 // particle operands, chunk kc in slot kc % BR
    bf16x8 aq[2][MT];                                   // weight operands of chunks kc (even/odd)
    f32x4 acc[MT][kNT];
    int par = 0;
    const uint16_t* xnext = nullptr;                    // the next chunk's particle rows (this lane)
    const uint16_t* wnext = nullptr;                    // the next chunk's weight rows (M block)
    // an item's biases into LDS (wave 0, before its chunk 0) and its chunk pointers
    auto start = [&](int im, int itile, int ipar) {
        if (wave == 0) {
            const float* src = a.bias + im * ROWS + min(lane * 4, ROWS - 4);
            __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(bias_lds + ipar * 1024),
                                             16, 0, 0);
        }
        wnext = a.w + (int64_t)im * ROWS * 32;
        xnext = a.x + ((int64_t)itile * PROWS + wave * (kNT * 16) + r) * 32 + 8 * g;
    };
    // chunk kc of the started item: weights into LDS stage kc % kStages, this
    // wave's particles into register slot kc % BR; chunks are issued in order
    auto issue = [&](int kc) {
        lds_char* A = sm + (kc % kStages) * A_BYTES;
#pragma unroll
        for (int i = 0; i < A_PER_WAVE; ++i) {
            const int j = min(wave + i * kWaves, MT - 1);
            dma_rows16(wnext + j * 16 * 32, 32, j * 16, 0, A + j * 1024, lane);
        }
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) bq[kc % BR][nt] = *(const bf16x8*)(xnext + nt * 16 * 32);
        wnext += (int64_t)K * 32;
        xnext += R * 32;
        asm volatile("" : "+s"(wnext));                 // one running pointer, not NK precomputed ones
        asm volatile("" : "+v"(xnext));
    };
    // LDS offset of this lane's operand piece in row tile mt: swz(16 mt + r) =
    // swz(r) ^ (2 mt & 3), so two lane offsets serve every tile (the tile and
    // stage parts are immediates of the LDS reads)
    const int a_off_even = r * 64 + ((g ^ swz(r)) * 16), a_off_odd = r * 64 + ((g ^ swz(r) ^ 2) * 16);
    auto read_a = [&](int kc) {
        const lds_char* A = sm + (kc % kStages) * A_BYTES;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            aq[kc & 1][mt] = *(const __attribute__((address_space(3))) bf16x8*)(A + mt * 1024 + ((mt & 1) ? a_off_odd
                                                                                                    : a_off_even));
    };
    auto products = [&](int kc) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq[kc & 1][mt], bq[kc % BR][nt], acc[mt][nt], 0, 0, 0);
    };
    start(m, tile, 0);
#pragma unroll
    for (int kc = 0; kc < kStages - 1; ++kc) issue(kc);
    const float s = *a.slope;
    for (;;) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            // chunk c readable: this wave's loads of it have landed (the loads
            // of the chunks after it, up to c + kStages - 2, may be pending)
            // and every wave's operand reads of chunk c - 1 are done, so its
            // stage and its register slot take chunk c + kStages - 1
            const int after = min(c + kStages - 2, NK - 1) - c;
            if (after >= 2) wait_vm<2 * PER_CHUNK>();
            else if (after == 1) wait_vm<PER_CHUNK>();
            else wait_vm<0>();
            __builtin_amdgcn_s_waitcnt(0xC07F);         // lgkmcnt(0) only
            asm volatile("s_barrier" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            const bool more = c + kStages - 1 < NK;
            if (more) issue(c + kStages - 1);
            read_a(c);
            if (c > 0) products(c - 1);
            // the loads first, then each operand read of chunk c beside the
            // kNT products of chunk c - 1 that use the register it replaces
            if (more) __builtin_amdgcn_sched_group_barrier(0x010, PER_CHUNK, 0);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                if (c > 0) __builtin_amdgcn_sched_group_barrier(0x008, kNT, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        products(NK - 1);
        int nid = id + G, nm = m, ntile = tile;
        while (nid < n_items && !valid(nid, nm, ntile)) nid += G;
        const bool last = nid >= n_items;
        if (PERSIST) {
            // every wave is done with this item's LDS stages; the next item's
            // first chunks (after the last item: this item's again, never read,
            // so that the loads and the counts below do not depend on a branch)
            __builtin_amdgcn_s_waitcnt(0xC07F);
            asm volatile("s_barrier" ::: "memory");
            if (last) { nm = m; ntile = tile; }
            start(nm, ntile, par ^ 1);
#pragma unroll
            for (int kc = 0; kc < kStages - 1; ++kc) issue(kc);
        } else {
            wait_vm<0>();                               // the biases
            asm volatile("s_barrier" ::: "memory");
        }
        const int64_t row0 = (int64_t)tile * PROWS + wave * (kNT * 16) + r;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int o = m * ROWS + mt * 16 + 4 * g;
            const f32x4 bb = *(const __attribute__((address_space(3))) f32x4*)(bias_lds + par * 1024 + (mt * 16 + 4 * g) * 4);
            uint16_t* yo = a.y + ((int64_t)(o >> 5) * R + row0) * 32 + (o & 31);
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) {
                const f32x4 v = acc[mt][nt];
                const u32x2 st = {pack2(prelu(v[0] + bb[0], s), prelu(v[1] + bb[1], s)),
                                  pack2(prelu(v[2] + bb[2], s), prelu(v[3] + bb[3], s))};
                *(u32x2*)(yo + nt * 16 * 32) = st;
            }
            __builtin_amdgcn_sched_barrier(0);          // one row of tiles at a time: registers
        }
        if (!PERSIST || last) break;
        id = nid; m = nm; tile = ntile; par ^= 1;
    }
    wait_vm<0>();                                       // no load in flight when the wave ends
}

// ------------------------------------------------------------ training
// Training kernels below work on one 256-row block of the batch and one
// chunk of 64 features (blockIdx.y): thread (f, pl) = (tid % 8, tid / 8) forms features
// 8f .. 8f+7 of rows pl, pl + 32, ... (16-B row-major stores), the same
// values go into a [64 features][256 rows] LDS tile, which the block then
// writes to the transposed array as whole 512-B rows.
constexpr int kFeatChunk = 64;
__device__ __forceinline__ void store_tile_t(const uint16_t (*tile)[kInP + 8], uint16_t* dst_t, int64_t ldt,
                                             int k0, int64_t p0) {
    // 64 rows x 256 columns of bf16: 2048 pieces of 16 B, 8 per thread
    for (int piece = threadIdx.x; piece < kFeatChunk * (kInP / 8); piece += kBlock) {
        const int kk = piece / (kInP / 8), c8 = (piece % (kInP / 8)) * 8;
        const u32x4 v = *(const u32x4*)&tile[kk][c8];
        *(u32x4*)(dst_t + (int64_t)(k0 + kk) * ldt + p0 + c8) = v;
    }
}

// Input layer of a training batch: sample p < B is pair idx[p] (rows >= B
// take a zero input); stores the transposed bf16 network input (rows 0..5 of
// x0t), the pre-activations, the activations and their transpose.
__global__ __launch_bounds__(kBlock) void k_train_input(const double* __restrict__ zin, int64_t ld,
                                                        DenseTrainBufs tb, DenseImage im, DenseNorm nm) {
    __shared__ float xs[kInP][6];
    __shared__ __attribute__((aligned(16))) uint16_t tile[kFeatChunk][kInP + 8];
    const int tid = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * kInP;
    {
        const int64_t p = p0 + tid;
        float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (p < tb.B) {
            P6 q;
            load6(zin, ld, tb.idx[p], q);
            const double pv[6] = {q.x, q.y, q.t, q.px, q.py, q.pt};
#pragma unroll
            for (int j = 0; j < 6; ++j) v[j] = (float)((pv[j] - nm.mu_in[j]) / nm.sd_in[j]);
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            xs[tid][j] = v[j];
            if (blockIdx.y == 0) tb.x0t[(int64_t)j * tb.bp + p] = __builtin_bit_cast(uint16_t, (__bf16)v[j]);
        }
    }
    const int f = tid % 8, pl = tid / 8;
    const float a0 = im.slope[0];
    {
        const int k0 = blockIdx.y * kFeatChunk;           // this block's 64 features
        __syncthreads();                                  // xs ready
        const int kf = k0 + 8 * f;
        float w[8][6], b[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            b[j] = im.b0[kf + j];
#pragma unroll
            for (int c = 0; c < 6; ++c) w[j][c] = im.w0[(kf + j) * 6 + c];
        }
        for (int q = pl; q < kInP; q += kBlock / 8) {
            float h[8], v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                float acc = b[j];
#pragma unroll
                for (int c = 0; c < 6; ++c) acc = fmaf(w[j][c], xs[q][c], acc);
                v[j] = acc;
                h[j] = prelu(acc, a0);
                tile[8 * f + j][q] = __builtin_bit_cast(uint16_t, (__bf16)h[j]);
            }
            const int64_t off = (p0 + q) * im.wp + kf;
            *(u32x4*)(tb.h[0] + off) = u32x4{pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]), pack2(h[6], h[7])};
            *(u32x4*)(tb.v[0] + off) = u32x4{pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), pack2(v[6], v[7])};
        }
        __syncthreads();
        store_tile_t(tile, tb.ht[0], tb.bp, k0, p0);
    }
}

// Output layer forward and its error (Eq. 4): one wave per sample; yhat =
// W_H h + b_H (bf16 weights and activations, FP32 sums), dy = scale (yhat -
// y) with y the normalised target; rows >= B give zero error.
__global__ __launch_bounds__(kBlock) void k_train_out_fwd(const double* __restrict__ zout, int64_t ld,
                                                          DenseTrainBufs tb, DenseImage im, DenseNorm nm,
                                                          const uint16_t* __restrict__ hlast, uint16_t* __restrict__ wH,
                                                          const float* __restrict__ bH, float scale) {
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * kWaves + (threadIdx.x >> 6);
    float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k = lane * 8; k < im.wp; k += 64 * 8) {
        const u32x4 hv = *(const u32x4*)(hlast + (int64_t)p * im.wp + k);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const u32x4 wv = *(const u32x4*)(wH + (int64_t)j * im.wp + k);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                acc[j] = fmaf(__uint_as_float(wv[e] << 16), __uint_as_float(hv[e] << 16), acc[j]);
                acc[j] = fmaf(__uint_as_float(wv[e] & 0xffff0000u), __uint_as_float(hv[e] & 0xffff0000u), acc[j]);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 6; ++j)
        for (int off = 32; off >= 1; off >>= 1) acc[j] += __shfl_xor(acc[j], off, 64);
    if (lane == 0) {
        float l2 = 0.0f;
        for (int j = 0; j < 6; ++j) {
            float d = 0.0f;
            if (p < tb.B) {
                const double y = (zout[(int64_t)j * ld + tb.idx[p]] - nm.mu_out[j]) / nm.sd_out[j];
                d = (acc[j] + bH[j]) - (float)y;
            }
            l2 = fmaf(d, d, l2);
            tb.dy[p * 8 + j] = scale * d;
            tb.dyt[(int64_t)j * tb.bp + p] = __builtin_bit_cast(uint16_t, (__bf16)(scale * d));
        }
        tb.lossp[p] = l2;
    }
}

// Back through the output layer and the last PReLU: dh = W_H^T dy, dv =
// dh prelu'(v); the workgroup's share of the slope gradient to part.
__global__ __launch_bounds__(kBlock) void k_train_out_bwd(DenseTrainBufs tb, DenseImage im,
                                                          const uint16_t* __restrict__ wH,
                                                          const uint16_t* __restrict__ vlast,
                                                          const float* __restrict__ slope, uint16_t* __restrict__ dv,
                                                          float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) uint16_t tile[kFeatChunk][kInP + 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int f = tid % 8, pl = tid / 8;
    const int64_t p0 = (int64_t)blockIdx.x * kInP;
    const float a = *slope;
    float sp = 0.0f;
    {
        const int k0 = blockIdx.y * kFeatChunk;           // this block's 64 features
        const int kf = k0 + 8 * f;
        float w[8][6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const u32x4 wv = *(const u32x4*)(wH + (int64_t)j * im.wp + kf);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                w[2 * e][j] = __uint_as_float(wv[e] << 16);
                w[2 * e + 1][j] = __uint_as_float(wv[e] & 0xffff0000u);
            }
        }
        for (int q = pl; q < kInP; q += kBlock / 8) {
            const int64_t p = p0 + q;
            const int64_t off = p * im.wp + kf;
            const u32x4 vv = *(const u32x4*)(vlast + off);
            float dy[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) dy[j] = tb.dy[p * 8 + j];
            float d[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                float dh = 0.0f;
#pragma unroll
                for (int j = 0; j < 6; ++j) dh = fmaf(w[e][j], dy[j], dh);
                const float v = (e & 1) ? __uint_as_float(vv[e >> 1] & 0xffff0000u) : __uint_as_float(vv[e >> 1] << 16);
                const bool pos = v > 0.0f;
                d[e] = pos ? dh : a * dh;
                sp += pos ? 0.0f : dh * v;
                tile[8 * f + e][q] = __builtin_bit_cast(uint16_t, (__bf16)d[e]);
            }
            *(u32x4*)(dv + off) = u32x4{pack2(d[0], d[1]), pack2(d[2], d[3]), pack2(d[4], d[5]), pack2(d[6], d[7])};
        }
        __syncthreads();
        store_tile_t(tile, tb.dvt, tb.bp, k0, p0);
    }
    for (int off = 32; off >= 1; off >>= 1) sp += __shfl_xor(sp, off, 64);
    __shared__ float red[kWaves];
    if (lane == 0) red[wave] = sp;
    __syncthreads();
    if (tid == 0) {
        float t = 0.0f;
        for (int w2 = 0; w2 < kWaves; ++w2) t += red[w2];
        part[blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
}

// Loss and slope gradients of one step: one workgroup, fixed summation order
// (thread t sums entries t, t + 256, ...; then a tree over the threads).
struct FinishArgs {
    int64_t slope_off[kDenseMaxHidden];
    int32_t nparts[kDenseMaxHidden];
    int32_t hidden;
};
__device__ float block_sum(float x, float* red) {
    red[threadIdx.x] = x;
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const float t = red[0];
    __syncthreads();
    return t;
}
__global__ __launch_bounds__(kBlock) void k_train_finish(DenseTrainBufs tb, FinishArgs fa, float* grad,
                                                         double* loss_acc, double scale) {
    __shared__ float red[kBlock];
    const int t = threadIdx.x;
    float l = 0.0f;
    for (int p = t; p < tb.B; p += kBlock) l += tb.lossp[p];
    l = block_sum(l, red);
    if (t == 0) *loss_acc += (double)l * scale;
    if (!grad) return;                                 // uniform: the whole block returns
    for (int h = 0; h < fa.hidden; ++h) {
        float x = 0.0f;
        for (int q = t; q < fa.nparts[h]; q += kBlock) x += tb.part[h * kDensePartMax + q];
        x = block_sum(x, red);
        if (t == 0) grad[fa.slope_off[h]] = x;
    }
}

__global__ void k_fill_row(uint16_t* row, int n, int valid, uint16_t one) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) row[i] = i < valid ? one : (uint16_t)0;
}

__global__ void k_pack_bf16_t(const float* __restrict__ src, int rows, int cols, uint16_t* __restrict__ dst,
                              int rows_p, int cols_p) {
    // dst[c][r] = src[r][c] (dst: cols_p x rows_p), zero padding
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)rows_p * cols_p) return;
    const int c = (int)(i / rows_p), r = (int)(i % rows_p);
    const float v = (r < rows && c < cols) ? src[(int64_t)r * cols + c] : 0.0f;
    dst[i] = __builtin_bit_cast(uint16_t, (__bf16)v);
}

// Adam (bias-corrected) on every parameter, writing the updated value
// straight into the operand images as well: first-layer FP32, biases and
// slopes FP32, W x W weights bf16 in both orientations, output layer bf16.
struct WtImages {
    uint16_t* w[kDenseMaxHidden + 1];
};
__global__ void k_dense_adam_pack(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                  const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps,
                                  float c1, float c2, DenseOffsets off, DenseImage im, WtImages wt, int H, int W) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    int l = 0;
    while (l < H && i >= off.A[l + 1]) ++l;            // i lies in layer l's tensors
    const int wp = im.wp;
    if (l < H && i == off.slope[l]) {
        im.slope[l] = pi;
    } else if (i >= off.b[l]) {
        const int o = (int)(i - off.b[l]);
        if (l == 0) im.b0[o] = pi;
        else im.b[l][o] = pi;
    } else {
        const int64_t q = i - off.A[l];
        const int ni = l == 0 ? 6 : W;
        const int o = (int)(q / ni), k = (int)(q % ni);
        if (l == 0) {
            im.w0[o * 6 + k] = pi;
        } else {
            const uint16_t b = __builtin_bit_cast(uint16_t, (__bf16)pi);
            im.w[l][(int64_t)o * wp + k] = b;
            if (l < H && wt.w[l]) wt.w[l][(int64_t)k * wp + o] = b;
            if (l < H && im.wb[l]) im.wb[l][(int64_t)(k >> 5) * wp * 32 + (int64_t)o * 32 + (k & 31)] = b;
        }
    }
}

int layer_grid(const LayerArgs& a) { return a.mblocks * ((a.tiles + 7) / 8) * 8; }

template <int MT, int EPI, int WM = 1>
hipError_t launch_layer_mt(const LayerArgs& a, hipStream_t s) {
    const LatticeView none{};
    const DenseNorm nm{};
    hipLaunchKernelGGL((k_dense_layer<MT, WM, EPI, false, false>), dim3(layer_grid(a)), dim3(256 * WM), 0, s, a, nm,
                       none);
    return hipGetLastError();
}

typedef hipError_t (*LayerLauncher)(const LayerArgs&, hipStream_t);
constexpr int kMaxMT = 12;      // accumulators MT x NT x 4 <= 192 stay in the AGPR file
template <int EPI>
struct LayerTable {
    static constexpr LayerLauncher f[kMaxMT] = {
        launch_layer_mt<1, EPI>, launch_layer_mt<2, EPI>, launch_layer_mt<3, EPI>, launch_layer_mt<4, EPI>,
        launch_layer_mt<5, EPI>, launch_layer_mt<6, EPI>, launch_layer_mt<7, EPI>, launch_layer_mt<8, EPI>,
        launch_layer_mt<9, EPI>, launch_layer_mt<10, EPI>, launch_layer_mt<11, EPI>, launch_layer_mt<12, EPI>};
};

// M block of a W x W layer: the largest MT <= kMaxMT dividing Wp / 16 (Wp is
// a multiple of 64, so 4 always divides it).
int hidden_mt(int wp) {
    const int tiles = wp / 16;
    for (int mt = kMaxMT; mt >= 1; --mt)
        if (tiles % mt == 0) return mt;
    return 1;
}

template <int MT>
hipError_t launch_hidden_blk(const LayerArgs& a, hipStream_t s) {
    const int items = layer_grid(a);
    constexpr bool P = MT <= kBlkPersistMaxMT;
    const int grid = P && items > kPersistGroups ? kPersistGroups : items;
    hipLaunchKernelGGL((k_dense_hidden_blk<MT, P>), dim3(grid), dim3(kBlock), 0, s, a, items);
    return hipGetLastError();
}
constexpr LayerLauncher kHiddenBlk[kBlkMaxMT - kBlkMinMT + 1] = {
    launch_hidden_blk<8>,  launch_hidden_blk<9>,  launch_hidden_blk<10>, launch_hidden_blk<11>,
    launch_hidden_blk<12>, launch_hidden_blk<13>, launch_hidden_blk<14>, launch_hidden_blk<15>};

}  // namespace

bool dense_blocked(int wp) { return wp % 64 == 0 && wp / 64 >= kBlkMinMT && wp / 64 <= kBlkMaxMT; }

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
                               im.w[l], rows_p, Wp, 0);
            if (l < H && im.wb[l])
                hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, A, no, ni,
                                   im.wb[l], rows_p, Wp, 1);
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
    // 512 <= W' <= 960: activations K-blocked, hidden layers on k_dense_hidden_blk
    const bool blk = dense_blocked(Wp);
    for (int l = 1; l < H; ++l)
        if (blk && !im.wb[l]) return hipErrorInvalidValue;
    for (int64_t p0 = 0; p0 < n; p0 += chunk) {
        const int64_t nc = n - p0 < chunk ? n - p0 : chunk, nend = p0 + nc;
        const int tiles = (int)((nc + tile - 1) / tile);
        const int64_t rows = (int64_t)tiles * tile;
        const dim3 gin((unsigned)(rows / kInP));
        if (blk) {
            if (!gaps)
                hipLaunchKernelGGL((k_dense_input<false, false, true>), gin, dim3(kBlock), 0, s, z, nend, ld, p0, im, nm,
                                   pre, buf0, rows);
            else if (!chrom)
                hipLaunchKernelGGL((k_dense_input<true, false, true>), gin, dim3(kBlock), 0, s, z, nend, ld, p0, im, nm,
                                   pre, buf0, rows);
            else
                hipLaunchKernelGGL((k_dense_input<true, true, true>), gin, dim3(kBlock), 0, s, z, nend, ld, p0, im, nm,
                                   pre, buf0, rows);
        } else {
            if (!gaps)
                hipLaunchKernelGGL((k_dense_input<false, false, false>), gin, dim3(kBlock), 0, s, z, nend, ld, p0, im,
                                   nm, pre, buf0, rows);
            else if (!chrom)
                hipLaunchKernelGGL((k_dense_input<true, false, false>), gin, dim3(kBlock), 0, s, z, nend, ld, p0, im,
                                   nm, pre, buf0, rows);
            else
                hipLaunchKernelGGL((k_dense_input<true, true, false>), gin, dim3(kBlock), 0, s, z, nend, ld, p0, im,
                                   nm, pre, buf0, rows);
        }
        uint16_t* xin = buf0;
        uint16_t* yout = buf1;
        for (int l = 1; l < H; ++l) {
            LayerArgs a{};
            a.x = xin; a.w = im.w[l]; a.bias = im.b[l]; a.slope = im.slope + l; a.y = yout;
            a.K = Wp; a.Mp = Wp; a.mblocks = Wp / (16 * MT); a.tiles = tiles;
            hipError_t e;
            if (blk) {
                a.w = im.wb[l];
                a.mblocks = 4;
                e = kHiddenBlk[Wp / 64 - kBlkMinMT](a, s);
            } else {
                // 12-tile M blocks (W' = 1024 and other multiples of 192 outside
                // the blocked range) take the 8-wave form: measured 9 % faster
                // than 4 waves
                e = MT == 12 ? launch_layer_mt<12, kEpiHidden, 2>(a, s) : LayerTable<kEpiHidden>::f[MT - 1](a, s);
            }
            if (e != hipSuccess) return e;
            uint16_t* t = xin; xin = yout; yout = t;
        }
        LayerArgs a{};
        a.x = xin; a.w = im.w[H]; a.bias = im.b[H]; a.K = Wp; a.Mp = 16; a.mblocks = 1; a.tiles = tiles;
        a.z = z; a.ld = ld; a.p0 = p0; a.nend = nend;
        const dim3 gout((unsigned)(((tiles + 7) / 8) * 8));
        if (blk) {
            if (!gaps)
                hipLaunchKernelGGL((k_dense_layer<1, 1, kEpiOut, false, false, true>), gout, dim3(kBlock), 0, s, a, nm,
                                   post);
            else if (!chrom)
                hipLaunchKernelGGL((k_dense_layer<1, 1, kEpiOut, true, false, true>), gout, dim3(kBlock), 0, s, a, nm,
                                   post);
            else
                hipLaunchKernelGGL((k_dense_layer<1, 1, kEpiOut, true, true, true>), gout, dim3(kBlock), 0, s, a, nm,
                                   post);
        } else if (!gaps)
            hipLaunchKernelGGL((k_dense_layer<1, 1, kEpiOut, false, false>), gout, dim3(kBlock), 0, s, a, nm, post);
        else if (!chrom)
            hipLaunchKernelGGL((k_dense_layer<1, 1, kEpiOut, true, false>), gout, dim3(kBlock), 0, s, a, nm, post);
        else
            hipLaunchKernelGGL((k_dense_layer<1, 1, kEpiOut, true, true>), gout, dim3(kBlock), 0, s, a, nm, post);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hbl

namespace hbl {

DenseOffsets dense_offsets(const DenseShape& sh) {
    DenseOffsets o{};
    int64_t off = 0;
    for (int l = 0; l <= sh.hidden; ++l) {
        const int64_t ni = l == 0 ? 6 : sh.width, no = l == sh.hidden ? 6 : sh.width;
        o.A[l] = off;
        o.b[l] = off + no * ni;
        off += no * (ni + 1);
        if (l < sh.hidden) o.slope[l] = off++;
    }
    return o;
}

hipError_t launch_dense_pack_t(const float* params, const DenseShape& sh, int32_t wp, uint16_t* const* wt,
                               hipStream_t s) {
    const DenseOffsets o = dense_offsets(sh);
    for (int l = 1; l < sh.hidden; ++l) {
        const int64_t cnt = (int64_t)wp * wp;
        hipLaunchKernelGGL(k_pack_bf16_t, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, params + o.A[l],
                           sh.width, sh.width, wt[l], wp, wp);
    }
    return hipGetLastError();
}

hipError_t launch_dense_fill_ones(const DenseTrainBufs& tb, int32_t wp, int32_t hidden, hipStream_t s) {
    const uint16_t one = 0x3F80;   // bf16 1.0
    const dim3 g((tb.bp + 255) / 256);
    hipLaunchKernelGGL(k_fill_row, g, dim3(256), 0, s, tb.x0t + (int64_t)6 * tb.bp, tb.bp, tb.B, one);
    for (int l = 0; l < hidden; ++l)
        hipLaunchKernelGGL(k_fill_row, g, dim3(256), 0, s, tb.ht[l] + (int64_t)wp * tb.bp, tb.bp, tb.B, one);
    return hipGetLastError();
}

hipError_t launch_dense_train_step(const double* zin, const double* zout, int64_t ld, const DenseShape& sh,
                                   const DenseImage& im, uint16_t* const* wt, const DenseNorm& nm,
                                   const DenseTrainBufs& tb, const float* params, float* grad,
                                   double* loss_acc, double loss_scale, hipStream_t s) {
    (void)params;
    // a training batch is only a few 256-row tiles: M blocks of 2 MFMA tiles
    // (32 rows) give the products enough workgroups to spread over the chip
    const int wp = im.wp, H = sh.hidden, MT = 2;
    const int tiles = tb.bp / dense_tile_rows();
    const DenseOffsets off = dense_offsets(sh);
    FinishArgs fa{};
    fa.hidden = H;
    // ---- forward, keeping what the backward pass needs
    const dim3 g2(tb.bp / kInP, wp / kFeatChunk);         // row blocks x feature chunks
    hipLaunchKernelGGL(k_train_input, g2, dim3(kBlock), 0, s, zin, ld, tb, im, nm);
    for (int l = 1; l < H; ++l) {
        LayerArgs a{};
        a.x = tb.h[l - 1]; a.w = im.w[l]; a.bias = im.b[l]; a.slope = im.slope + l; a.y = tb.h[l];
        a.v = tb.v[l]; a.yt = tb.ht[l]; a.ldt = tb.bp;
        a.K = wp; a.Mp = wp; a.mblocks = wp / (16 * MT); a.tiles = tiles;
        hipError_t e = LayerTable<kEpiTrain>::f[MT - 1](a, s);
        if (e != hipSuccess) return e;
    }
    const float scale = 2.0f / (float)(tb.B * 6);
    hipLaunchKernelGGL(k_train_out_fwd, dim3(tb.bp / kWaves), dim3(kBlock), 0, s, zout, ld, tb, im, nm,
                       tb.h[H - 1], im.w[H], im.b[H], scale);
    if (grad) {
        // ---- output layer: weight and bias gradients, then back into the last hidden layer
        {
            LayerArgs a{};
            a.x = tb.ht[H - 1]; a.w = tb.dyt; a.K = tb.bp; a.Mp = 16; a.mblocks = 1;
            a.tiles = tb.np / dense_tile_rows();
            a.grad = grad + off.A[H]; a.gradb = grad + off.b[H]; a.W = 6; a.gcols = sh.width; a.bias_row = wp;
            hipError_t e = LayerTable<kEpiGrad>::f[0](a, s);
            if (e != hipSuccess) return e;
        }
        int cur = 0;
        hipLaunchKernelGGL(k_train_out_bwd, g2, dim3(kBlock), 0, s, tb, im, im.w[H], tb.v[H - 1],
                           im.slope + (H - 1), tb.dv[cur], tb.part + (int64_t)(H - 1) * kDensePartMax);
        fa.nparts[H - 1] = (int)(g2.x * g2.y);
        // ---- hidden layers, top down
        for (int l = H - 1; l >= 1; --l) {
            LayerArgs g{};
            g.x = tb.ht[l - 1]; g.w = tb.dvt; g.K = tb.bp; g.Mp = wp; g.mblocks = wp / (16 * MT);
            g.tiles = tb.np / dense_tile_rows();
            g.grad = grad + off.A[l]; g.gradb = grad + off.b[l]; g.W = sh.width; g.gcols = sh.width; g.bias_row = wp;
            hipError_t e = LayerTable<kEpiGrad>::f[MT - 1](g, s);
            if (e != hipSuccess) return e;
            LayerArgs b{};
            b.x = tb.dv[cur]; b.w = wt[l]; b.slope = im.slope + (l - 1); b.y = tb.dv[cur ^ 1]; b.v = tb.v[l - 1];
            b.yt = tb.dvt; b.ldt = tb.bp; b.part = tb.part + (int64_t)(l - 1) * kDensePartMax;
            b.K = wp; b.Mp = wp; b.mblocks = wp / (16 * MT); b.tiles = tiles;
            fa.nparts[l - 1] = layer_grid(b);
            e = LayerTable<kEpiBwd>::f[MT - 1](b, s);
            if (e != hipSuccess) return e;
            cur ^= 1;
        }
        // ---- first layer: gradient against the transposed network input
        {
            LayerArgs a{};
            a.x = tb.x0t; a.w = tb.dvt; a.K = tb.bp; a.Mp = wp; a.mblocks = wp / (16 * MT); a.tiles = 1;
            a.grad = grad + off.A[0]; a.gradb = grad + off.b[0]; a.W = sh.width; a.gcols = 6; a.bias_row = 6;
            hipError_t e = LayerTable<kEpiGrad>::f[MT - 1](a, s);
            if (e != hipSuccess) return e;
        }
        for (int h = 0; h < H; ++h) fa.slope_off[h] = off.slope[h];
    }
    hipLaunchKernelGGL(k_train_finish, dim3(1), dim3(kBlock), 0, s, tb, fa, grad, loss_acc, loss_scale);
    return hipGetLastError();
}

hipError_t launch_dense_adam_pack(float* p, float* m, float* v, const float* g, int64_t n, int64_t t, float lr,
                                  float b1, float b2, float eps, const DenseShape& sh, const DenseImage& im,
                                  uint16_t* const* wt, hipStream_t s) {
    const float c1 = (float)(1.0 - pow((double)b1, (double)t)), c2 = (float)(1.0 - pow((double)b2, (double)t));
    WtImages w{};
    for (int l = 0; l <= kDenseMaxHidden; ++l) w.w[l] = wt ? wt[l] : nullptr;
    hipLaunchKernelGGL(k_dense_adam_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, m, v, g, n, lr, b1,
                       b2, eps, c1, c2, dense_offsets(sh), im, w, sh.hidden, sh.width);
    return hipGetLastError();
}

}  // namespace hbl
