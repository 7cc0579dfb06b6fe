/*
 * orc.h -- CPU ORACLE for the hybrid beamline hot path (test infrastructure).
 *
 * Plain, serial, FP64 reference implementation written from the paper
 * (Sandberg et al., "Synthesizing Particle-in-Cell Simulations Through
 * Learning and GPU Computing for Hybrid Particle Accelerator Beamlines",
 * PASC '24) and textbook linear beam optics.  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no
 * source, header, table or helper with the GPU library.
 *
 * Bunch layout: six FP64 rows (x, y, t, px, py, pt), row j of particle i at
 * z[j*ld + i].  Units: x, y, t in m (t = c * (t_particle - t_ref), positive =
 * later); px = p_x/p_ref, py = p_y/p_ref, pt = -(E - E_ref)/(p_ref c).
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_DRIFT = 1, ORC_QUAD = 2, ORC_SBEND = 3, ORC_THIN_LENS = 4, ORC_STAGE = 5 };

typedef struct {
    int32_t kind;
    int32_t nsub;      /* stage substeps */
    double L;          /* length [m] */
    double k;          /* quad strength [m^-2] */
    double angle;      /* bend angle [rad] */
    double f;          /* thin-lens focal length [m] */
    double n0_m3;      /* stage plasma density [m^-3] */
    double dE_MeV;     /* stage energy gain [MeV] */
    double chirp;      /* stage: particle gain dE (1 + chirp t_entry), chirp [1/m]; 0 = uniform */
    int32_t chromatic; /* quad, thin lens: focusing scales as 1/(1 + delta), first order in delta */
    int32_t pad;
} orc_elem;

typedef struct {
    double mass_MeV;   /* rest energy */
    double gamma;      /* Lorentz factor of the reference particle */
    double s;          /* path length [m] */
} orc_ref;

/* Counter-based generator (Philox4x32-10, Salmon et al. SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Gaussian bunch: particle with global index g = (idx ? idx[i] : i0 + i). */
int orc_fill_gaussian(double* z, int64_t n, int64_t ld, uint64_t seed,
                      const double mean[6], const double sigma[6],
                      int64_t i0, const int64_t* idx);

/* Push through a sequence of elements (linear elements and stages). */
int orc_push(double* z, int64_t n, int64_t ld, const orc_elem* e, int32_t n_elem, orc_ref* ref);

/* Exact moments: means[6], centred population covariance, upper triangle
 * row-major (00,01,..,05,11,..,55) = 21 entries. */
int orc_moments(const double* z, int64_t n, int64_t ld, double mean6[6], double cov21[21]);
/* Geometric emittances of (x,px), (y,py), (t,pt) from the covariance. */
int orc_emittances(const double cov21[21], double eps3[3]);
/* Paired error metrics of a test bunch s against a reference bunch f. */
int orc_compare(const double* s, const double* f, int64_t n, int64_t ld,
                double rms6[6], double centroid6[6], double eps_rel3[3]);

/* bfloat16 round-to-nearest-even of an FP32 value, returned as FP32. */
float orc_bf16(float x);

/* ---- MLP surrogate (Eq. 3), MSE loss (Eq. 4), Adam ---- */
typedef struct { int32_t n_in, width, hidden, n_out; } orc_shape;
int64_t orc_mlp_nparams(const orc_shape* sh);
int orc_mlp_init(const orc_shape* sh, uint64_t seed, float* params);
/* norm: mu_in[6], sd_in[6], mu_out[6], sd_out[6] (FP64). mode 0 = FP64, the
 * network as defined (the parity reference, with the rounding-error models of
 * mlp_error.py); mode 1 = an emulation that FOLLOWS THE LIBRARY KERNEL's own
 * rounding points (its tanh scale fold and first-layer split included), kept
 * as a secondary, kernel-specific check only. */
int orc_mlp_apply(const orc_shape* sh, const float* params, const double* norm, int mode,
                  const double* zin, double* zout, int64_t n, int64_t ld);
/* Loss (Eq. 4, normalised coordinates) and gradient over the pairs idx[0..b). */
int orc_mlp_loss_grad(const orc_shape* sh, const float* params, const double* norm, int mode,
                      const double* zin, const double* zout, int64_t ld,
                      const int64_t* idx, int64_t b, double* grad, double* loss);
int orc_adam_step(int64_t np, float* params, double* m, double* v, const double* grad,
                  int64_t t, double lr, double b1, double b2, double eps);
/* Normalisation statistics of the first n_train pairs. */
int orc_norm_stats(const double* zin, const double* zout, int64_t n_train, int64_t ld, double* norm);
/* Epoch permutation (Fisher-Yates driven by Philox). */
int orc_epoch_perm(int64_t n, uint64_t seed, int64_t epoch, int64_t* perm);
/* PReLU network of the paper's shape (Eq. 2 and 3): one learned slope per
 * hidden layer; flat layout A_0, b_0, a_0, ..., A_{H-1}, b_{H-1}, a_{H-1},
 * A_H, b_H; slopes start at 0.25.  Mode 0 = FP64, mode 1 = the GPU rounding
 * points (FP32 first layer, bf16 weights and activations elsewhere). */
int64_t orc_prelu_nparams(const orc_shape* sh);
int orc_prelu_init(const orc_shape* sh, uint64_t seed, float* params);
int orc_prelu_apply(const orc_shape* sh, const float* params, const double* norm, int mode,
                    const double* zin, double* zout, int64_t n, int64_t ld);
/* Loss (Eq. 4) and exact FP64 gradient over the pairs idx[0..b). */
int orc_prelu_loss_grad(const orc_shape* sh, const float* params, const double* norm,
                        const double* zin, const double* zout, int64_t ld,
                        const int64_t* idx, int64_t b, double* grad, double* loss);
/* Learning rate of step t (1-based) of `planned`: half cosine lr -> lr_final. */
double orc_lr_at(int64_t t, int64_t planned, double lr, double lr_final);
/* Full training loop; loss_log[2*e] = mean train loss, [2*e+1] = test loss. */
int orc_mlp_train(const orc_shape* sh, float* params, double* norm, int mode,
                  const double* zin, const double* zout, int64_t n_pairs, int64_t ld,
                  int64_t batch, int64_t epochs, int64_t max_steps, double lr, double lr_final,
                  double b1, double b2, double eps, double train_frac, uint64_t shuffle_seed,
                  double* loss_log);

#ifdef __cplusplus
}
#endif
#endif
