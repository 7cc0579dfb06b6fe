// Internal declarations shared by the libhbl translation units (not part of
// the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace hbl {

// ----------------------------------------------------------------- errors
void set_error(int code, const char* fmt, ...);
void clear_error();

// ------------------------------------------------------ compiled elements
// First-order transfer map coefficients of one linear element, computed on
// the host in FP64 for the reference particle the lattice was compiled for.
//  DRIFT : c[0] = L, c[1] = L/(beta gamma)^2
//  QUAD  : c[0..3] = x-plane m11 m12 m21 m22, c[4..7] = y-plane, c[8] = L/(beta gamma)^2
//  SBEND : c[0] m11, c[1] m12, c[2] m16, c[3] m21, c[4] m22, c[5] m26,
//          c[6] m51, c[7] m52, c[8] m56, c[9] L (vertical drift)
//  LENS  : c[0] = -1/f
constexpr int kCoef = 12;
enum ElemKind : int32_t { kDrift = 1, kQuad = 2, kSbend = 3, kLens = 4 };

struct ElemCoef {
    double c[kCoef];
};

// The same element as one unified sparse map (the union of the four kinds):
//   x'  = fma(g2,  pt, fma(g1,  px, g0 * x))
//   px' = fma(g5,  pt, fma(g4,  px, g3 * x))
//   y'  = fma(g7,  py, g6 * y)
//   py' = fma(g9,  py, g8 * y)
//   t'  = fma(g12, pt, fma(g11, px, fma(g10, x, t)))
// with unit and zero coefficients placed so that every kind gives exactly
// the same result as its specialised map (a multiply by 1, an fma with a 0
// factor and an fma adding +-0 are exact).  Chromatic quads and lenses add,
// with the old coordinates and pt (first order in delta = -pt/beta),
//   x'  = fma(fma(g17, px, g16 * x), pt, x'),  px' = fma(fma(g19, px, g18 * x), pt, px')
//   y'  = fma(fma(g21, py, g20 * y), pt, y'),  py' = fma(fma(g23, py, g22 * y), pt, py')
// 24 doubles, 13..15 unused.
constexpr int kGen = 24;
struct GenCoef {
    double g[kGen];
};
// chrom8: the eight chromatic coefficients (g16..g23) or nullptr.
GenCoef unify(int32_t kind, const ElemCoef& c, const double* chrom8);

// ----------------------------------------------------------- stage params
struct StageParams {
    double bg_in;          // (beta gamma)_ref at entry
    double h;              // substep length
    double hk2;            // h^2 kappa (merged full kick on v = h u)
    double half_hk2;       // h^2 kappa / 2
    double inv_h_bgout;    // 1/(h (beta gamma)_out)
    double pt_scale;       // (beta gamma)_in / (beta gamma)_out
    double r56;            // first-order flight-time coefficient
    // energy-correlated gain (chirp != 0): particle gain dE (1 + chirp t_entry)
    double chirp;          // [1/m]
    double chirp_gain;     // chirp (gamma_out - gamma_in)
    double chirp_t;        // chirp gp L^2 / (2 gamma_in gamma_out^2)
    double inv_bgout;      // 1/(beta gamma)_out
    int32_t nsub;
    int32_t newton;        // Newton steps per substep (0 = divide every substep)
};

// ------------------------------------------------------------- launchers
// All launchers validate nothing (the ABI layer does) and return the HIP
// launch status.
hipError_t launch_fill_gaussian(double* z, int64_t n, int64_t ld, uint64_t seed,
                                const double* mean, const double* sigma, int64_t i0,
                                hipStream_t s);
hipError_t launch_lattice_fused(double* z, int64_t n, int64_t ld, const double* gen, const int32_t* kinds,
                                int32_t n_elem, bool chromatic, hipStream_t s);
// One element through its unified record (unfused push of a chromatic lattice).
hipError_t launch_lattice_gen(double* z, int64_t n, int64_t ld, const double* gen1, bool chromatic,
                              hipStream_t s);
hipError_t launch_lattice_element(double* z, int64_t n, int64_t ld, int32_t kind,
                                  const ElemCoef& c, hipStream_t s);
struct LatticeView;
// tab: gamma_ref at the middle of each substep, then (chirp only) the ramp
// increment gp * s_mid of each substep.
hipError_t launch_stage(double* z, int64_t n, int64_t ld, double* rec, int64_t rld,
                        const StageParams& p, const double* tab, const LatticeView& pre,
                        const LatticeView& post, hipStream_t s);

// Reductions.  `ws` is device scratch of at least reduce_ws_bytes(n) bytes.
size_t reduce_ws_bytes(int64_t n);
// The library's fixed per-device reduction scratch (no allocation): its size,
// and its address on the current device (looked up once per device).
size_t reduce_scratch_bytes();
hipError_t reduce_scratch(double** out);
hipError_t launch_moments(const double* z, int64_t n, int64_t ld, double* ws, double* out27,
                          hipStream_t s);
hipError_t launch_diff2(const double* zs, const double* zf, int64_t n, int64_t ld, double* ws,
                        double* out6, hipStream_t s);

// Surrogate network (tanh MLP 6-64-64-64-6).
int mlp_nparams();
int mlp_image_words();
hipError_t launch_mlp_pack(const float* params, uint32_t* img, hipStream_t s);
// Lowest-test-loss parameter copy (info: 2 doubles, best: mlp_nparams() floats).
hipError_t launch_best_init(double* info, hipStream_t s);
hipError_t launch_keep_best(const double* loss, double* info, const float* params, float* best, int64_t epoch,
                            hipStream_t s);
// Emittance criterion: snapshot the parameters with {score, test loss} into
// rec (2 doubles), then select among nw snapshots and restore the choice.
hipError_t launch_snapshot(const double* pred27, const double* true27, const double* loss, const float* params,
                           float* snap, double* rec, hipStream_t s);
hipError_t launch_select_snapshot(const double* rec, int nw, double tol, const float* snap, float* params,
                                  double* info, hipStream_t s);
hipError_t launch_restore_best(const double* info, const float* best, float* params, hipStream_t s);
hipError_t launch_mlp_infer(double* z, int64_t n, int64_t ld, const uint32_t* img, const double* norm24,
                            const LatticeView& pre, const LatticeView& post, hipStream_t s);
hipError_t launch_train_step(const double* zin, const double* zout, int64_t ld, const int32_t* idx,
                             int32_t batch, const uint32_t* img, float* part, float* loss_part,
                             const double* norm24, hipStream_t s);
hipError_t launch_train_adam(float* p, float* m, float* v, const float* part, int32_t nb,
                             const float* loss_part, double* loss_acc, double loss_scale, int64_t t,
                             float lr, float b1, float b2, float eps, hipStream_t s);
hipError_t launch_grad_sum(const float* part, int32_t nb, float* grad, hipStream_t s);
int eval_loss_blocks(int64_t n);
hipError_t launch_eval_loss(const double* zin, const double* zout, int64_t ld, int64_t i0, int64_t n,
                            const uint32_t* img, const double* norm24, double* part, double* out,
                            hipStream_t s);

// Wide PReLU surrogate (hidden width W <= 1024, 1..7 hidden layers).
constexpr int kDenseMaxWidth = 1024;
constexpr int kDenseMaxHidden = 7;
struct DenseShape {
    int32_t width, hidden;
};
// Device image of the network, rebuilt from the FP32 master parameters.
struct DenseImage {
    int32_t wp;                          // width rounded up to 64
    float* w0;                           // [wp][6] first layer, FP32
    float* b0;                           // [wp]
    float* slope;                        // [hidden] PReLU slopes
    uint16_t* w[kDenseMaxHidden + 1];    // layer l >= 1: bf16 [wp][wp] (output layer [16][wp])
    float* b[kDenseMaxHidden + 1];       // layer l >= 1: [wp] (output layer [16])
    // hidden layers 1 <= l < hidden again, K-blocked: [wp/32][wp][32] (element
    // (o, k) at (k/32) wp 32 + 32 o + k % 32); nullptr unless dense_blocked(wp)
    uint16_t* wb[kDenseMaxHidden + 1];
};
// Widths whose inference runs on K-blocked activations and weights (the
// hidden layers as 4 M blocks of wp/4 rows on the direct-load kernel).
bool dense_blocked(int wp);
struct DenseNorm {
    double mu_in[6], sd_in[6], mu_out[6], sd_out[6];
};
int dense_tile_rows();
hipError_t launch_dense_pack(const float* params, const DenseShape& sh, const DenseImage& im, hipStream_t s);
// Inference over n particles in chunks of `chunk` (a multiple of
// dense_tile_rows()); buf0/buf1: chunk x wp bf16 each.
hipError_t launch_dense_infer(double* z, int64_t n, int64_t ld, const DenseShape& sh, const DenseImage& im,
                              const DenseNorm& nm, const LatticeView& pre, const LatticeView& post,
                              uint16_t* buf0, uint16_t* buf1, int64_t chunk, hipStream_t s);

// Training of the wide network (batch rows padded to bp, a multiple of the
// 256-row tile; rows >= B carry zero error).
constexpr int kDensePartMax = 4096;      // slope-gradient partial sums per layer
struct DenseTrainBufs {
    int32_t bp, B, np;                   // padded batch, batch, rows of the transposed activations
    const int32_t* idx;                  // [B] sample indices of this step
    uint16_t* x0t;                       // [256][bp] network input, transposed; row 6 = 1 (bias)
    uint16_t* h[kDenseMaxHidden];        // [bp][wp] hidden activations
    uint16_t* v[kDenseMaxHidden];        // [bp][wp] pre-activations
    uint16_t* ht[kDenseMaxHidden];       // [np][bp] activations transposed; row wp = 1 (bias)
    uint16_t* dv[2];                     // [bp][wp] dL/dv ping-pong
    uint16_t* dvt;                       // [wp][bp] dL/dv transposed
    uint16_t* dyt;                       // [16][bp] output error, transposed (bf16)
    float* dy;                           // [bp][8] output error
    float* lossp;                        // [bp] squared error per sample
    float* part;                         // [kDenseMaxHidden][kDensePartMax]
};
// Flat parameter offsets (as the public layout): A_l, b_l, slope_l.
struct DenseOffsets {
    int64_t A[kDenseMaxHidden + 1], b[kDenseMaxHidden + 1], slope[kDenseMaxHidden];
};
DenseOffsets dense_offsets(const DenseShape& sh);
hipError_t launch_dense_pack_t(const float* params, const DenseShape& sh, int32_t wp, uint16_t* const* wt,
                               hipStream_t s);
hipError_t launch_dense_fill_ones(const DenseTrainBufs& tb, int32_t wp, int32_t hidden, hipStream_t s);
// Forward with stored activations, loss and full gradient of one batch;
// adds sum(loss) * loss_scale to *loss_acc.  grad_out may be nullptr for a
// loss-only (evaluation) pass.
hipError_t launch_dense_train_step(const double* zin, const double* zout, int64_t ld, const DenseShape& sh,
                                   const DenseImage& im, uint16_t* const* wt, const DenseNorm& nm,
                                   const DenseTrainBufs& tb, const float* params, float* grad_out,
                                   double* loss_acc, double loss_scale, hipStream_t s);
// Adam on the FP32 parameters, the updated values also written into the
// operand images (im, and the transposed W x W images wt[1..H-1]).
hipError_t launch_dense_adam_pack(float* p, float* m, float* v, const float* g, int64_t n, int64_t t, float lr,
                                  float b1, float b2, float eps, const DenseShape& sh, const DenseImage& im,
                                  uint16_t* const* wt, hipStream_t s);

// The reduction workspace of stream s on the current device (one buffer per
// device and stream, grow-only, kept until the process ends).
double* workspace(size_t bytes, hipStream_t s);

}  // namespace hbl
