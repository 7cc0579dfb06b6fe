// Tracking kernels for gfx950: Gaussian bunch fill, fused and per-element
// lattice push, fine-step plasma stage.  All FP64.  Bunch rows are SoA
// (x, y, t, px, py, pt at z + j*ld): every load and store below is a
// unit-stride access across the lanes of a wavefront.
//
// Compiled with -ffp-contract=off: every fused multiply-add is written out
// as fma(), so the fused and per-element lattice paths execute the same
// operations in the same order and agree bitwise.
#include "hbl_elements.hpp"

namespace hbl {
namespace {

constexpr int kBlock = 256;

// --------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products, key advanced by the Weyl constants each round.
// Each product is formed as one 64-bit value (a single v_mad_u64_u32 gives
// both halves; separate low and high multiplies issue twice as many
// quarter-rate instructions).
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// sin(2 pi u) and cos(2 pi u) for u in [0, 1): the octant reduction
// u = (k + 1/2)/8 + d is exact for a 53-bit u, theta = 2 pi d lies in
// [-pi/8, pi/8), sin and cos of theta come from their Taylor series
// (Horner form in theta^2 with the coefficients +-1/n!, truncation below
// 1e-17) and the octant centre (2k+1) pi/8 enters through the
// angle-addition formulas.  Error ~2e-16 absolute.
__device__ __forceinline__ void sincos_2pi(double u, double& s, double& c) {
    const double k = floor(u * 8.0);
    const double d = u - (k + 0.5) * 0.125;
    const double th = d * (2.0 * M_PI);
    const double t2 = th * th;
    double ps = 1.0 / 6227020800.0;                 // 1/13!
    ps = fma(ps, t2, -1.0 / 39916800.0);            // 1/11!
    ps = fma(ps, t2, 1.0 / 362880.0);               // 1/9!
    ps = fma(ps, t2, -1.0 / 5040.0);                // 1/7!
    ps = fma(ps, t2, 1.0 / 120.0);                  // 1/5!
    ps = fma(ps, t2, -1.0 / 6.0);                   // 1/3!
    const double st = fma(th * t2, ps, th);
    double pc = -1.0 / 87178291200.0;               // 1/14!
    pc = fma(pc, t2, 1.0 / 479001600.0);            // 1/12!
    pc = fma(pc, t2, -1.0 / 3628800.0);             // 1/10!
    pc = fma(pc, t2, 1.0 / 40320.0);                // 1/8!
    pc = fma(pc, t2, -1.0 / 720.0);                 // 1/6!
    pc = fma(pc, t2, 1.0 / 24.0);                   // 1/4!
    pc = fma(pc, t2, -0.5);                         // 1/2!
    const double ct = fma(t2, pc, 1.0);
    const int ki = (int)k;
    const double s1 = 0.38268343236508978, c1 = 0.92387953251128674;  // sin, cos of pi/8
    const bool a = ((ki ^ (ki >> 1)) & 1) == 0;
    double sp = a ? s1 : c1, cp = a ? c1 : s1;
    if (ki >= 4) sp = -sp;
    if ((ki + 2) & 4) cp = -cp;
    s = fma(sp, ct, cp * st);
    c = fma(cp, ct, -(sp * st));
}

// ln(u) for u in (0, 1] (the Box-Muller radius): u = m 2^e with m in
// [1/sqrt 2, sqrt 2), ln m = 2 atanh(s) with s = (m - 1)/(m + 1), |s| < 0.172,
// summed as 2s + s^3 (2/3 + s^2 (2/5 + ...)) through the s^25 term
// (truncation below 1e-19 relative), and e ln 2 added in two parts (ln 2 cut
// to 32 significant bits, so e ln2_hi is exact, plus the remainder).
// m - 1 is exact; s comes from the hardware reciprocal refined by two Newton
// steps and one residual correction.  Error below 1.5 ulp of ln u (checked
// against extended-precision logs over 3e7 arguments), i.e. ~2e-16
// relative on sqrt(-2 ln u); a third of the instructions of the library log.
__device__ __forceinline__ double log_unit(double u) {
    int e;
    double m = frexp(u, &e);
    if (m < 0.70710678118654752) {
        m *= 2.0;
        e -= 1;
    }
    const double f = m - 1.0, d = m + 1.0;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    double sq = f * r;
    sq = fma(fma(-sq, d, f), r, sq);
    const double s2 = sq * sq;
    double p = 2.0 / 25.0;
    p = fma(p, s2, 2.0 / 23.0);
    p = fma(p, s2, 2.0 / 21.0);
    p = fma(p, s2, 2.0 / 19.0);
    p = fma(p, s2, 2.0 / 17.0);
    p = fma(p, s2, 2.0 / 15.0);
    p = fma(p, s2, 2.0 / 13.0);
    p = fma(p, s2, 2.0 / 11.0);
    p = fma(p, s2, 2.0 / 9.0);
    p = fma(p, s2, 2.0 / 7.0);
    p = fma(p, s2, 2.0 / 5.0);
    p = fma(p, s2, 2.0 / 3.0);
    const double lm = fma(sq * s2, p, 2.0 * sq);
    const double ln2_hi = 0x1.62e42fee00000p-1, ln2_lo = 1.9082149292705877e-10;
    const double de = (double)e;
    return fma(de, ln2_hi, fma(de, ln2_lo, lm));
}

struct FillArgs {
    double mean[6];
    double sigma[6];
};

// One thread per particle.  Pair q of particle g: counter (g_lo, g_hi, q,
// "GAUS"), two 53-bit uniforms u1 in (0,1], u2 in [0,1), Box-Muller
// (Box & Muller 1958): r = sqrt(-2 ln u1), (r cos 2 pi u2, r sin 2 pi u2).
__global__ __launch_bounds__(kBlock) void k_fill_gaussian(double* __restrict__ z, int64_t n,
                                                          int64_t ld, uint32_t key0,
                                                          uint32_t key1, int64_t i0,
                                                          FillArgs a) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const uint64_t g = (uint64_t)(i0 + i);
#pragma unroll
        for (uint32_t q = 0; q < 3; ++q) {
            uint32_t c0 = (uint32_t)g, c1 = (uint32_t)(g >> 32), c2 = q, c3 = 0x47415553u;
            philox4x32_10(c0, c1, c2, c3, key0, key1);
            const uint64_t ua = ((uint64_t)(c0 >> 5) << 26) | (c1 >> 6);
            const uint64_t ub = ((uint64_t)(c2 >> 5) << 26) | (c3 >> 6);
            const double u1 = ((double)ua + 1.0) * 0x1.0p-53;
            const double u2 = (double)ub * 0x1.0p-53;
            const double r = sqrt(-2.0 * log_unit(u1));
            double sn, cs;
            sincos_2pi(u2, sn, cs);
            z[(2 * q) * ld + i] = a.mean[2 * q] + a.sigma[2 * q] * (r * cs);
            z[(2 * q + 1) * ld + i] = a.mean[2 * q + 1] + a.sigma[2 * q + 1] * (r * sn);
        }
    }
}

// --------------------------------------------------------------- lattice
// Fused lattice (this C form serves lattices with chromatic elements; the
// achromatic form is k_lattice_fused_asm below): each thread keeps kPer = 4
// particles in registers (four independent chains of FP64 operations per
// element) through the whole element sequence; drifts (the most common
// element) take their 3-FMA map, every other element its unified record
// (coefficients and kinds are wavefront-uniform scalar loads, the drift test
// a scalar branch).  One tile
// of kPer*kBlock particles per block (grid-stride beyond 2^20 blocks): a
// persistent, capped grid measured 20 % slower, and a switch over all the
// element kinds cost more in register copies than the FMAs it saves.  Reads
// the six rows and writes back the five an element can change (88 B per
// particle): no lattice element changes pt.
template <bool CHROM, int kPer>
__global__ __launch_bounds__(kBlock) void k_lattice_fused(double* __restrict__ z, int64_t n,
                                                          int64_t ld, const double* __restrict__ gen,
                                                          const int32_t* __restrict__ kinds, int32_t n_elem) {
    const int64_t tile = (int64_t)kPer * kBlock;
    for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile) {
        P6 p[kPer];
        bool live[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int64_t i = base + k * kBlock + threadIdx.x;
            live[k] = i < n;
            if (live[k]) load6_nt(z, ld, i, p[k]);
            else p[k] = P6{0, 0, 0, 0, 0, 0};
        }
#pragma unroll 2
        for (int32_t e = 0; e < n_elem; ++e) {
            const double* g = gen + (int64_t)e * kGen;
            const int32_t kind = kinds[e];
            if (kind == kDrift) {
#pragma unroll
                for (int k = 0; k < kPer; ++k) el_drift_gen(p[k], g);
            } else if (!CHROM && kind == kQuad) {
#pragma unroll
                for (int k = 0; k < kPer; ++k) el_quad_gen(p[k], g);
            } else {
#pragma unroll
                for (int k = 0; k < kPer; ++k) el_unified<CHROM>(p[k], g);
            }
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int64_t i = base + k * kBlock + threadIdx.x;
            if (live[k]) store5_nt(z, ld, i, p[k]);         // pt is never changed by a lattice element
        }
    }
}

// Achromatic fused lattice with the element loop as one inline-asm block
// (HBL_ELEMENT_LOOP, hbl_elements.hpp) over the four particles of each
// thread: no register copies at the kind-branch joins, results bitwise those
// of the per-element path.  The chromatic form is k_lattice_fused<true> above.
__global__ __launch_bounds__(kBlock) void k_lattice_fused_asm(double* __restrict__ z, int64_t n, int64_t ld,
                                                              const double* __restrict__ gen,
                                                              const int32_t* __restrict__ kinds, int32_t n_elem) {
    constexpr int kPer = 4;
    if (n_elem <= 0) return;
    const int64_t tile = (int64_t)kPer * kBlock;
    for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile) {
        P6 p[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int64_t i = base + k * kBlock + threadIdx.x;
            if (i < n) load6_nt(z, ld, i, p[k]);
            else p[k] = P6{0, 0, 0, 0, 0, 0};
        }
        double w[kPer];
        uint32_t off = 0, koff = 0;     // byte offsets of the current record and kind
        int32_t cnt = n_elem;
        asm volatile(HBL_ELEMENT_LOOP(HBL_OP4, HBL_MOV4)
                     : [x0] "+v"(p[0].x), [y0] "+v"(p[0].y), [t0] "+v"(p[0].t), [px0] "+v"(p[0].px),
                       [py0] "+v"(p[0].py), [x1] "+v"(p[1].x), [y1] "+v"(p[1].y), [t1] "+v"(p[1].t),
                       [px1] "+v"(p[1].px), [py1] "+v"(p[1].py), [x2] "+v"(p[2].x), [y2] "+v"(p[2].y),
                       [t2] "+v"(p[2].t), [px2] "+v"(p[2].px), [py2] "+v"(p[2].py), [x3] "+v"(p[3].x),
                       [y3] "+v"(p[3].y), [t3] "+v"(p[3].t), [px3] "+v"(p[3].px), [py3] "+v"(p[3].py),
                       [w0] "=&v"(w[0]), [w1] "=&v"(w[1]), [w2] "=&v"(w[2]), [w3] "=&v"(w[3]),
                       [off] "+s"(off), [koff] "+s"(koff), [cnt] "+s"(cnt)
                     : [pt0] "v"(p[0].pt), [pt1] "v"(p[1].pt), [pt2] "v"(p[2].pt), [pt3] "v"(p[3].pt),
                       [gp] "s"(gen), [kp] "s"(kinds)
                     : HBL_ELEMENT_LOOP_CLOBBERS);
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int64_t i = base + k * kBlock + threadIdx.x;
            if (i < n) store5_nt(z, ld, i, p[k]);           // pt is never changed by a lattice element
        }
    }
}


// One element through its unified record: the unfused push of a lattice
// with chromatic elements (the specialised kernels below are achromatic).
template <bool CHROM>
__global__ __launch_bounds__(kBlock) void k_lattice_gen(double* __restrict__ z, int64_t n, int64_t ld,
                                                        const double* __restrict__ g) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        P6 p;
        load6(z, ld, i, p);
        el_unified<CHROM>(p, g);
        store6(z, ld, i, p);
    }
}

// Per-element comparator: one launch per element, loading and storing only
// the rows that element reads and writes.
template <int KIND>
__global__ __launch_bounds__(kBlock) void k_lattice_one(double* __restrict__ z, int64_t n,
                                                        int64_t ld, ElemCoef ec) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        P6 p;
        if (KIND == kLens) {
            p.x = z[i];
            p.y = z[ld + i];
            p.px = z[3 * ld + i];
            p.py = z[4 * ld + i];
            el_lens(p, ec.c);
            z[3 * ld + i] = p.px;
            z[4 * ld + i] = p.py;
        } else {
            load6(z, ld, i, p);
            if (KIND == kDrift) {
                el_drift(p, ec.c);
                z[i] = p.x;
                z[ld + i] = p.y;
                z[2 * ld + i] = p.t;
            } else if (KIND == kQuad) {
                el_quad(p, ec.c);
                z[i] = p.x;
                z[ld + i] = p.y;
                z[2 * ld + i] = p.t;
                z[3 * ld + i] = p.px;
                z[4 * ld + i] = p.py;
            } else {
                el_sbend(p, ec.c);
                z[i] = p.x;
                z[ld + i] = p.y;
                z[2 * ld + i] = p.t;
                z[3 * ld + i] = p.px;
            }
        }
    }
}

// --------------------------------------------------------------- stage
// One thread per particle, the whole stage in registers.  Variables
// v = h u (u = p/(m c)) so a kick is v -= h^2 kappa x and a drift is
// x += v / gamma_i.  Adjacent half kicks are merged.  1/gamma_i(s_n) is
// refined from the previous substep's reciprocal by NEWTON Newton steps
// r <- r (2 - a r) (the relative change per substep is small, checked by the
// host); NEWTON == 0 divides every substep.  gmid[n] = gamma_ref at the
// middle of substep n (uniform across the wavefront: scalar loads).
// The transport gap before the stage (pre) and after it (post) are applied
// in registers in the same pass (empty sequences for a lone stage), and the
// recorded training input is the state after `pre`.
template <int NEWTON, bool CHIRP, bool CHROM>
__global__ __launch_bounds__(kBlock) void k_stage(double* __restrict__ z, int64_t n, int64_t ld,
                                                  double* __restrict__ rec, int64_t rld,
                                                  StageParams sp,
                                                  const double* __restrict__ gmid,
                                                  LatticeView pre, LatticeView post) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const double* __restrict__ gs = gmid + sp.nsub;   // gp * s_mid per substep (CHIRP)
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        P6 p;
        load6(z, ld, i, p);
        apply_elements<CHROM>(p, pre);
        if (rec) store6(rec, rld, i, p);
        const double t_in = p.t;
        const double dg = -p.pt * sp.bg_in;
        // particle gradient gp (1 + chirp t_in): gamma_i = gamma_mid + dg + chirp t_in gp s_mid
        const double cg = CHIRP ? sp.chirp * t_in : 0.0;
        // the host sized the Newton steps for a gain factor 1 + chirp t within [0, 2];
        // a particle outside divides (a per-lane branch, uniform in practice)
        const bool divide = CHIRP && fabs(cg) > 1.0;
        const double hb = sp.h * sp.bg_in;
        double x = p.x, y = p.y;
        double vx = p.px * hb, vy = p.py * hb;
        vx = fma(-sp.half_hk2, x, vx);
        vy = fma(-sp.half_hk2, y, vy);
        double a = CHIRP ? fma(cg, gs[0], gmid[0] + dg) : gmid[0] + dg;
        double r = 1.0 / a;
        x = fma(vx, r, x);
        y = fma(vy, r, y);
        auto substep = [&](double gm, double gsm) {
            vx = fma(-sp.hk2, x, vx);
            vy = fma(-sp.hk2, y, vy);
            a = CHIRP ? fma(cg, gsm, gm + dg) : gm + dg;
            if (NEWTON == 0 || divide) {
                r = 1.0 / a;
            } else {
#pragma unroll
                for (int q = 0; q < NEWTON; ++q) {
                    const double e = fma(-a, r, 1.0);
                    r = fma(r, e, r);
                }
            }
            x = fma(vx, r, x);
            y = fma(vy, r, y);
        };
        // Substeps in blocks of U whose table entries are read by one group of
        // scalar loads (one wait per block instead of one per substep;
        // 8 entries measured 3-4 % faster than one at a time), then the rest.
        constexpr int U = CHIRP ? 4 : 8;
        int32_t s = 1;
        for (; s + U <= sp.nsub; s += U) {
            double gm[U], gsm[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                gm[u] = gmid[s + u];
                gsm[u] = CHIRP ? gs[s + u] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) substep(gm[u], gsm[u]);
        }
        for (; s < sp.nsub; ++s) substep(gmid[s], CHIRP ? gs[s] : 0.0);
        vx = fma(-sp.half_hk2, x, vx);
        vy = fma(-sp.half_hk2, y, vy);
        p.x = x;
        p.y = y;
        p.px = vx * sp.inv_h_bgout;
        p.py = vy * sp.inv_h_bgout;
        p.t = fma(sp.r56, p.pt, p.t);
        if (CHIRP) {
            p.t = fma(-sp.chirp_t, t_in, p.t);
            p.pt = fma(-sp.chirp_gain, t_in, p.pt * sp.bg_in) * sp.inv_bgout;
        } else {
            p.pt = p.pt * sp.pt_scale;
        }
        apply_elements<CHROM>(p, post);
        store6(z, ld, i, p);
    }
}

int grid_for(int64_t n, int64_t per_block, int cap) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

hipError_t launch_fill_gaussian(double* z, int64_t n, int64_t ld, uint64_t seed,
                                const double* mean, const double* sigma, int64_t i0,
                                hipStream_t s) {
    if (n == 0) return hipSuccess;
    FillArgs a;
    for (int j = 0; j < 6; ++j) {
        a.mean[j] = mean[j];
        a.sigma[j] = sigma[j];
    }
    const int grid = grid_for(n, kBlock, 1 << 20);
    hipLaunchKernelGGL(k_fill_gaussian, dim3(grid), dim3(kBlock), 0, s, z, n, ld,
                       (uint32_t)seed, (uint32_t)(seed >> 32), i0, a);
    return hipGetLastError();
}

hipError_t launch_lattice_fused(double* z, int64_t n, int64_t ld, const double* gen, const int32_t* kinds,
                                int32_t n_elem, bool chromatic, hipStream_t s) {
    if (n == 0 || n_elem == 0) return hipSuccess;
    constexpr int P = 4;                      // particles per thread (measured: 2 -> 4 is 8-10 % faster)
    const int grid = grid_for(n, (int64_t)P * kBlock, 1 << 20);
    if (chromatic)
        hipLaunchKernelGGL((k_lattice_fused<true, P>), dim3(grid), dim3(kBlock), 0, s, z, n, ld, gen, kinds, n_elem);
    else
        hipLaunchKernelGGL(k_lattice_fused_asm, dim3(grid), dim3(kBlock), 0, s, z, n, ld, gen, kinds, n_elem);
    return hipGetLastError();
}

hipError_t launch_lattice_gen(double* z, int64_t n, int64_t ld, const double* gen1, bool chromatic,
                              hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int grid = grid_for(n, kBlock, 1 << 20);
    if (chromatic)
        hipLaunchKernelGGL(k_lattice_gen<true>, dim3(grid), dim3(kBlock), 0, s, z, n, ld, gen1);
    else
        hipLaunchKernelGGL(k_lattice_gen<false>, dim3(grid), dim3(kBlock), 0, s, z, n, ld, gen1);
    return hipGetLastError();
}

hipError_t launch_lattice_element(double* z, int64_t n, int64_t ld, int32_t kind,
                                  const ElemCoef& c, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int grid = grid_for(n, kBlock, 1 << 20);
    switch (kind) {
        case kDrift:
            hipLaunchKernelGGL(k_lattice_one<kDrift>, dim3(grid), dim3(kBlock), 0, s, z, n, ld, c);
            break;
        case kQuad:
            hipLaunchKernelGGL(k_lattice_one<kQuad>, dim3(grid), dim3(kBlock), 0, s, z, n, ld, c);
            break;
        case kSbend:
            hipLaunchKernelGGL(k_lattice_one<kSbend>, dim3(grid), dim3(kBlock), 0, s, z, n, ld, c);
            break;
        default:
            hipLaunchKernelGGL(k_lattice_one<kLens>, dim3(grid), dim3(kBlock), 0, s, z, n, ld, c);
            break;
    }
    return hipGetLastError();
}

namespace {
template <bool CHIRP, bool CHROM>
void launch_stage_t(int grid, double* z, int64_t n, int64_t ld, double* rec, int64_t rld,
                    const StageParams& p, const double* tab, const LatticeView& pre,
                    const LatticeView& post, hipStream_t s) {
#define HBL_STAGE_LAUNCH(K)                                                                         \
    hipLaunchKernelGGL((k_stage<K, CHIRP, CHROM>), dim3(grid), dim3(kBlock), 0, s, z, n, ld, rec, rld, \
                       p, tab, pre, post)
    switch (p.newton) {
        case 1: HBL_STAGE_LAUNCH(1); break;
        case 2: HBL_STAGE_LAUNCH(2); break;
        case 3: HBL_STAGE_LAUNCH(3); break;
        case 4: HBL_STAGE_LAUNCH(4); break;
        default: HBL_STAGE_LAUNCH(0); break;
    }
#undef HBL_STAGE_LAUNCH
}
}  // namespace

hipError_t launch_stage(double* z, int64_t n, int64_t ld, double* rec, int64_t rld,
                        const StageParams& p, const double* tab, const LatticeView& pre,
                        const LatticeView& post, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int grid = grid_for(n, kBlock, 1 << 20);
    const bool chirp = p.chirp != 0.0, chrom = pre.chromatic || post.chromatic;
    if (chirp && chrom) launch_stage_t<true, true>(grid, z, n, ld, rec, rld, p, tab, pre, post, s);
    else if (chirp) launch_stage_t<true, false>(grid, z, n, ld, rec, rld, p, tab, pre, post, s);
    else if (chrom) launch_stage_t<false, true>(grid, z, n, ld, rec, rld, p, tab, pre, post, s);
    else launch_stage_t<false, false>(grid, z, n, ld, rec, rld, p, tab, pre, post, s);
    return hipGetLastError();
}

}  // namespace hbl
