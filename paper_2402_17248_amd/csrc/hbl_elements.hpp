// Device-side first-order element maps shared by the tracking, stage and
// surrogate kernels (the coefficient records are built on the host, see
// ElemCoef in hbl_internal.hpp).  Every multiply-add is an explicit fma():
// the kernels are compiled with -ffp-contract=off, so every kernel that
// applies an element executes the same operations in the same order.
#pragma once

#include "hbl_internal.hpp"

namespace hbl {

struct P6 {
    double x, y, t, px, py, pt;
};

__device__ __forceinline__ void el_drift(P6& p, const double* c) {
    p.x = fma(c[0], p.px, p.x);
    p.y = fma(c[0], p.py, p.y);
    p.t = fma(c[1], p.pt, p.t);
}

__device__ __forceinline__ void el_quad(P6& p, const double* c) {
    const double x = p.x, px = p.px, y = p.y, py = p.py;
    p.x = fma(c[1], px, c[0] * x);
    p.px = fma(c[3], px, c[2] * x);
    p.y = fma(c[5], py, c[4] * y);
    p.py = fma(c[7], py, c[6] * y);
    p.t = fma(c[8], p.pt, p.t);
}

__device__ __forceinline__ void el_sbend(P6& p, const double* c) {
    const double x = p.x, px = p.px, pt = p.pt;
    p.x = fma(c[2], pt, fma(c[1], px, c[0] * x));
    p.px = fma(c[5], pt, fma(c[4], px, c[3] * x));
    p.y = fma(c[9], p.py, p.y);
    p.t = fma(c[8], pt, fma(c[7], px, fma(c[6], x, p.t)));
}

// A thin lens adds the rounded kick: px + round(c0 x), as the unified map does.
__device__ __forceinline__ void el_lens(P6& p, const double* c) {
    p.px = p.px + c[0] * p.x;
    p.py = p.py + c[0] * p.y;
}

// Any element through its unified record (GenCoef): branch-free, bitwise
// equal to the specialised map of its kind; CHROM adds the first-order
// chromatic terms of quads and lenses (zero for the other kinds).
template <bool CHROM = false>
__device__ __forceinline__ void el_unified(P6& p, const double* g) {
    const double x = p.x, px = p.px, y = p.y, py = p.py, pt = p.pt;
    p.x = fma(g[2], pt, fma(g[1], px, g[0] * x));
    p.px = fma(g[5], pt, fma(g[4], px, g[3] * x));
    p.y = fma(g[7], py, g[6] * y);
    p.py = fma(g[9], py, g[8] * y);
    p.t = fma(g[12], pt, fma(g[11], px, fma(g[10], x, p.t)));
    if (CHROM) {
        p.x = fma(fma(g[17], px, g[16] * x), pt, p.x);
        p.px = fma(fma(g[19], px, g[18] * x), pt, p.px);
        p.y = fma(fma(g[21], py, g[20] * y), pt, p.y);
        p.py = fma(fma(g[23], py, g[22] * y), pt, p.py);
    }
}

// A compiled element sequence (device coefficient tables), passed by value.
struct LatticeView {
    const int32_t* kinds;
    const double* coef;   // ElemCoef records
    const double* gen;    // GenCoef records
    int32_t n;
    int32_t chromatic;    // any element chromatic
};

// A drift through its unified record's three nonzero off-diagonal terms
// (g1 = g7 = L, g12 = L/(beta gamma)^2): the specialised drift map, bitwise.
__device__ __forceinline__ void el_drift_gen(P6& p, const double* g) {
    p.x = fma(g[1], p.px, p.x);
    p.y = fma(g[7], p.py, p.y);
    p.t = fma(g[12], p.pt, p.t);
}

// A thick quadrupole through its unified record's nonzero terms (the two
// plane matrices and the t-pt term): the specialised quad map, bitwise.
__device__ __forceinline__ void el_quad_gen(P6& p, const double* g) {
    const double x = p.x, px = p.px, y = p.y, py = p.py;
    p.x = fma(g[1], px, g[0] * x);
    p.px = fma(g[4], px, g[3] * x);
    p.y = fma(g[7], py, g[6] * y);
    p.py = fma(g[9], py, g[8] * y);
    p.t = fma(g[12], p.pt, p.t);
}

// Apply the sequence to one particle: the unified record of each element,
// read by scalar loads (uniform across the wavefront), no branches (inside
// the register-heavy stage and inference kernels a drift branch measured
// slower: its register copies cost more than the FMAs it saves).
template <bool CHROM = false>
__device__ __forceinline__ void apply_elements(P6& p, const LatticeView& lv) {
    for (int32_t e = 0; e < lv.n; ++e) el_unified<CHROM>(p, lv.gen + (int64_t)e * kGen);
}

__device__ __forceinline__ void load6(const double* __restrict__ z, int64_t ld, int64_t i, P6& p) {
    p.x = z[i];
    p.y = z[ld + i];
    p.t = z[2 * ld + i];
    p.px = z[3 * ld + i];
    p.py = z[4 * ld + i];
    p.pt = z[5 * ld + i];
}

// Streaming variants (non-temporal hint): the fused lattice reads and writes
// each particle exactly once.
__device__ __forceinline__ void load6_nt(const double* __restrict__ z, int64_t ld, int64_t i, P6& p) {
    p.x = __builtin_nontemporal_load(z + i);
    p.y = __builtin_nontemporal_load(z + ld + i);
    p.t = __builtin_nontemporal_load(z + 2 * ld + i);
    p.px = __builtin_nontemporal_load(z + 3 * ld + i);
    p.py = __builtin_nontemporal_load(z + 4 * ld + i);
    p.pt = __builtin_nontemporal_load(z + 5 * ld + i);
}

__device__ __forceinline__ void store6_nt(double* __restrict__ z, int64_t ld, int64_t i, const P6& p) {
    __builtin_nontemporal_store(p.x, z + i);
    __builtin_nontemporal_store(p.y, z + ld + i);
    __builtin_nontemporal_store(p.t, z + 2 * ld + i);
    __builtin_nontemporal_store(p.px, z + 3 * ld + i);
    __builtin_nontemporal_store(p.py, z + 4 * ld + i);
    __builtin_nontemporal_store(p.pt, z + 5 * ld + i);
}

// The five rows a lattice element can change: no drift, quadrupole, bend or
// thin lens (chromatic or not) changes pt, so a lattice pass stores 40 of
// the 48 bytes of a particle.
__device__ __forceinline__ void store5_nt(double* __restrict__ z, int64_t ld, int64_t i, const P6& p) {
    __builtin_nontemporal_store(p.x, z + i);
    __builtin_nontemporal_store(p.y, z + ld + i);
    __builtin_nontemporal_store(p.t, z + 2 * ld + i);
    __builtin_nontemporal_store(p.px, z + 3 * ld + i);
    __builtin_nontemporal_store(p.py, z + 4 * ld + i);
}

__device__ __forceinline__ void store6(double* __restrict__ z, int64_t ld, int64_t i, const P6& p) {
    z[i] = p.x;
    z[ld + i] = p.y;
    z[2 * ld + i] = p.t;
    z[3 * ld + i] = p.px;
    z[4 * ld + i] = p.py;
    z[5 * ld + i] = p.pt;
}

}  // namespace hbl
