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

// ---------------------------------------------------------------- asm element loop
// The element loop of an achromatic lattice as the text of one inline-asm
// block, shared by the kernels that apply lattices.  Written in C, a branch
// on the element kind is restructured by the compiler into flow blocks whose
// joins move the particle state between register sets (a 64-bit copy per
// coordinate and element); in the asm block the state is tied in place
// ("+v" operands x<k>, y<k>, t<k>, px<k>, py<k>; inputs pt<k>), each map
// updates it in place with one temporary w<k> per particle (a plane at a
// time), and the only copies left are the two a 2x2 plane map needs.  The
// operations and their order are those of el_drift_gen, el_quad_gen and
// el_unified<false>, so results are bitwise those of the C maps.
//
// Per element the kind (s90) and the 13 achromatic coefficients of its
// record (s[64:89]) are read with scalar loads and waited for inside the
// block (no load is left in flight at its end); there are no scalar stores.
// Operands: [gp] record table, [kp] kinds (SGPR pointers), [off] / [koff]
// byte offsets (start at 0), [cnt] element count (>= 1; the block runs a
// do-while loop).  OP applies "op dst, coef, src" to every particle of the
// block, MOV copies a coordinate.
static_assert(kGen == 24 && kDrift == 1 && kQuad == 2, "the asm loop hard-codes the record stride and kinds");

#define HBL_G0 "s[64:65]"
#define HBL_G1 "s[66:67]"
#define HBL_G2 "s[68:69]"
#define HBL_G3 "s[70:71]"
#define HBL_G4 "s[72:73]"
#define HBL_G5 "s[74:75]"
#define HBL_G6 "s[76:77]"
#define HBL_G7 "s[78:79]"
#define HBL_G8 "s[80:81]"
#define HBL_G9 "s[82:83]"
#define HBL_G10 "s[84:85]"
#define HBL_G11 "s[86:87]"
#define HBL_G12 "s[88:89]"

#define HBL_OP1(op, d, c, s) op " %[" d "0], " c ", %[" s "0]\n\t"
#define HBL_MOV1(d, s) "v_mov_b64 %[" d "0], %[" s "0]\n\t"
#define HBL_OP4(op, d, c, s)                                                         \
    op " %[" d "0], " c ", %[" s "0]\n\t" op " %[" d "1], " c ", %[" s "1]\n\t"      \
    op " %[" d "2], " c ", %[" s "2]\n\t" op " %[" d "3], " c ", %[" s "3]\n\t"
#define HBL_MOV4(d, s)                                                               \
    "v_mov_b64 %[" d "0], %[" s "0]\n\tv_mov_b64 %[" d "1], %[" s "1]\n\t"           \
    "v_mov_b64 %[" d "2], %[" s "2]\n\tv_mov_b64 %[" d "3], %[" s "3]\n\t"

#define HBL_ELEMENT_LOOP(OP, MOV)                                                                      \
    "L_elem_%=:\n\t"                                                                                   \
    "s_load_dword s90, %[kp], %[koff]\n\t"                                                             \
    "s_load_dwordx16 s[64:79], %[gp], %[off]\n\t"                                                      \
    "s_add_u32 s91, %[off], 0x40\n\t"                                                                  \
    "s_load_dwordx8 s[80:87], %[gp], s91\n\t"                                                          \
    "s_add_u32 s91, %[off], 0x60\n\t"                                                                  \
    "s_load_dwordx2 s[88:89], %[gp], s91\n\t"                                                          \
    "s_add_u32 %[off], %[off], 0xc0\n\t"                                                               \
    "s_add_u32 %[koff], %[koff], 4\n\t"                                                                \
    "s_waitcnt lgkmcnt(0)\n\t"                                                                         \
    "s_cmp_eq_u32 s90, 1\n\t"                                                                          \
    "s_cbranch_scc1 L_drift_%=\n\t"                                                                    \
    "s_cmp_eq_u32 s90, 2\n\t"                                                                          \
    "s_cbranch_scc1 L_quad_%=\n\t"                                                                     \
    /* unified record: t first (it reads the old x, px), then the x and y planes */                    \
    OP("v_fmac_f64", "t", HBL_G10, "x") OP("v_fmac_f64", "t", HBL_G11, "px")                           \
    OP("v_fmac_f64", "t", HBL_G12, "pt")                                                               \
    OP("v_mul_f64", "w", HBL_G3, "x") OP("v_mul_f64", "x", HBL_G0, "x")                                \
    OP("v_fmac_f64", "w", HBL_G4, "px") OP("v_fmac_f64", "x", HBL_G1, "px")                            \
    OP("v_fmac_f64", "w", HBL_G5, "pt") OP("v_fmac_f64", "x", HBL_G2, "pt") MOV("px", "w")             \
    OP("v_mul_f64", "w", HBL_G8, "y") OP("v_mul_f64", "y", HBL_G6, "y")                                \
    OP("v_fmac_f64", "w", HBL_G9, "py") OP("v_fmac_f64", "y", HBL_G7, "py") MOV("py", "w")             \
    "s_branch L_next_%=\n\t"                                                                           \
    "L_drift_%=:\n\t"                                                                                  \
    OP("v_fmac_f64", "x", HBL_G1, "px") OP("v_fmac_f64", "y", HBL_G7, "py")                            \
    OP("v_fmac_f64", "t", HBL_G12, "pt")                                                               \
    "s_branch L_next_%=\n\t"                                                                           \
    "L_quad_%=:\n\t"                                                                                   \
    OP("v_mul_f64", "w", HBL_G3, "x") OP("v_mul_f64", "x", HBL_G0, "x")                                \
    OP("v_fmac_f64", "w", HBL_G4, "px") OP("v_fmac_f64", "x", HBL_G1, "px") MOV("px", "w")             \
    OP("v_mul_f64", "w", HBL_G8, "y") OP("v_mul_f64", "y", HBL_G6, "y")                                \
    OP("v_fmac_f64", "w", HBL_G9, "py") OP("v_fmac_f64", "y", HBL_G7, "py") MOV("py", "w")             \
    OP("v_fmac_f64", "t", HBL_G12, "pt")                                                               \
    "L_next_%=:\n\t"                                                                                   \
    "s_sub_u32 %[cnt], %[cnt], 1\n\t"                                                                  \
    "s_cmp_lg_u32 %[cnt], 0\n\t"                                                                       \
    "s_cbranch_scc1 L_elem_%="

#define HBL_ELEMENT_LOOP_CLOBBERS                                                                      \
    "s64", "s65", "s66", "s67", "s68", "s69", "s70", "s71", "s72", "s73", "s74", "s75", "s76", "s77",  \
        "s78", "s79", "s80", "s81", "s82", "s83", "s84", "s85", "s86", "s87", "s88", "s89", "s90",     \
        "s91", "scc", "memory"

// One particle through an achromatic lattice with the asm element loop.
__device__ __forceinline__ void apply_elements_asm(P6& p, const LatticeView& lv) {
    if (lv.n <= 0) return;
    double w;
    uint32_t off = 0, koff = 0;
    int32_t cnt = lv.n;
    asm volatile(HBL_ELEMENT_LOOP(HBL_OP1, HBL_MOV1)
                 : [x0] "+v"(p.x), [y0] "+v"(p.y), [t0] "+v"(p.t), [px0] "+v"(p.px), [py0] "+v"(p.py),
                   [w0] "=&v"(w), [off] "+s"(off), [koff] "+s"(koff), [cnt] "+s"(cnt)
                 : [pt0] "v"(p.pt), [gp] "s"(lv.gen), [kp] "s"(lv.kinds)
                 : HBL_ELEMENT_LOOP_CLOBBERS);
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
