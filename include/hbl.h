/*
 * hbl.h -- C ABI of libhbl, hybrid beamline tracking on one AMD MI355X.
 *
 * The library pushes an electron bunch in 6-D phase space through a beamline
 * of conventional elements (drift, thick quadrupole, sector bend, thin plasma
 * lens) and plasma-accelerator stages, each stage taken either by a fine-step
 * reference integrator or by a small neural-network surrogate, as in the
 * hybrid conventional + surrogate beamline of Sandberg et al., "Synthesizing
 * Particle-in-Cell Simulations Through Learning and GPU Computing for Hybrid
 * Particle Accelerator Beamlines", PASC '24 (§2).  Every element is a
 * per-particle map of R^6 with no collective effects (§1), so every call is
 * data parallel over particles.
 *
 * CONVENTIONS
 *  - Bunch: `z` is a DEVICE pointer to six FP64 rows of `n` particles, row j at
 *    z + j*ld: x, y, t, px, py, pt (row order 0..5) relative to the reference
 *    particle.  x, y, t in metres (t = c*(t_particle - t_ref), positive =
 *    later), px = p_x/p_ref, py = p_y/p_ref, pt = -(E - E_ref)/(p_ref c).
 *    `z` must be 16-byte aligned and `ld` even, ld >= n.  The caller owns the
 *    memory (e.g. a torch tensor of shape (6, ld)); the library never frees
 *    it.  n == 0 is a valid no-op.
 *  - Streams: `stream` is a hipStream_t (NULL = the null stream).  Calls
 *    marked ASYNC only enqueue work on it; calls marked SYNC wait for it.
 *    Particle data never leaves the device (§2, §4.3).
 *  - Errors: every call returns an hbl_status; arguments are validated before
 *    any GPU work is enqueued, and a rejected call has no effect.  Device
 *    arguments must be memory of the current HIP device (hipMalloc'd or
 *    managed) whose allocation holds every row they span; a host pointer,
 *    memory of another device or a range past its allocation is HBL_EINVAL.
 *    hbl_last_error() gives a message for the calling thread's last failure.
 *    A device fault in enqueued work surfaces at the next SYNC call.  No C++
 *    exception crosses this interface.
 *  - Handles (lattice, surrogate) own small device buffers on the device that
 *    was current when they were created; use them with that device current.
 *    A handle must not be used by two threads at once.
 *  - The reductions (hbl_moments, hbl_moments_async, hbl_compare, and the
 *    normalisation statistics of hbl_surrogate_train) use a workspace of
 *    the stream they are enqueued on (one per device and stream, grown on
 *    demand and kept until the process ends): reductions on one stream run
 *    in order on its workspace, reductions on different streams use
 *    different ones and may overlap.  Calls on one stream from several host
 *    threads must not overlap.
 */
#ifndef HBL_H
#define HBL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hbl_status;
#define HBL_OK 0
#define HBL_EINVAL (-1)     /* bad argument; nothing was enqueued */
#define HBL_EHIP (-2)       /* HIP runtime error */
#define HBL_ENOMEM (-3)     /* device or host allocation failed */
#define HBL_ENONFINITE (-4) /* a reduction met NaN or Inf particle data */
#define HBL_ESTATE (-5)     /* handle used in a state that does not allow it */
#define HBL_EIO (-6)        /* file I/O or format error */

/* Message of the calling thread's last failure ("" if none). */
const char* hbl_last_error(void);
/* Library version string. */
const char* hbl_version(void);

/* Reference particle (host POD).  gamma is its Lorentz factor; s the path
 * length along the beamline [m] (§1: s is the independent variable). */
typedef struct hbl_ref {
    double mass_MeV; /* rest energy, 0.51099895 for electrons */
    double gamma;
    double s;
} hbl_ref;

/* Element kinds. */
#define HBL_DRIFT 1
#define HBL_QUAD 2
#define HBL_SBEND 3
#define HBL_THIN_LENS 4
#define HBL_STAGE 5

/* One beamline element (host POD).  Fields not used by a kind must be zero.
 *  DRIFT     L
 *  QUAD      L, k [m^-2] (k > 0 focuses x, defocuses y), chromatic
 *  SBEND     L, angle [rad] (sector bend, hard edge, no edge focusing)
 *  THIN_LENS f [m] (plasma lens: px -= x/f, py -= y/f; §4, Fig. 1), chromatic
 *  STAGE     L, n0_m3 [m^-3], dE_MeV, nsub (plasma stage, §4), chirp
 * chromatic = 1: the focusing strength of a quad or lens scales as
 *   1/(1 + delta) for a particle of relative momentum deviation delta,
 *   taken to first order in delta = -pt/beta (drifts and px = dx/ds stay
 *   those of the reference); 0: achromatic.  Other kinds reject 1.
 * chirp [1/m]: a stage particle gains dE_MeV (1 + chirp t), t its entry
 *   t (energy correlated along the bunch, as in the longitudinal correlation
 *   of a plasma stage, §4.4); 0: uniform gain.  Other kinds reject nonzero. */
typedef struct hbl_element {
    int32_t kind;
    int32_t nsub;
    double L;
    double k;
    double angle;
    double f;
    double n0_m3;
    double dE_MeV;
    double chirp;
    int32_t chromatic;
    int32_t reserved;      /* must be 0 */
} hbl_element;

typedef void* hbl_stream;

/* ---------------------------------------------------------------- bunch */

/* ASYNC.  Fill particles [0, n) with independent Gaussians: coordinate j of
 * particle i is mean[j] + sigma[j]*N(0,1), drawn by Philox4x32-10 keyed by
 * `seed` with counter (i0 + i, pair, ...) and the Box-Muller transform; pairs
 * (x,y), (t,px), (py,pt).  The same (seed, i0 + i) always gives the same
 * particle, so a bunch can be filled in pieces.  Stands in for the Gaussian
 * bunches of the paper's simulations (§4.1).  mean, sigma: host arrays of 6. */
hbl_status hbl_bunch_fill_gaussian(double* z, int64_t n, int64_t ld, uint64_t seed,
                                   const double mean[6], const double sigma[6], int64_t i0,
                                   hbl_stream stream);

/* ---------------------------------------------------------------- lattice */

typedef struct hbl_lattice hbl_lattice;

/* Compile a sequence of linear elements (DRIFT, QUAD, SBEND, THIN_LENS; no
 * STAGE) for a reference particle of Lorentz factor ref->gamma into a device
 * coefficient table (first-order transfer maps of each element, §1).
 * Synchronous (uploads the table).  *out receives the handle. */
hbl_status hbl_lattice_create(const hbl_element* elems, int32_t n_elem, const hbl_ref* ref,
                              hbl_lattice** out);
hbl_status hbl_lattice_destroy(hbl_lattice* lat);
/* Total length [m] and element count of a compiled lattice. */
hbl_status hbl_lattice_info(const hbl_lattice* lat, double* length, int32_t* n_elem);

#define HBL_FUSED 0u   /* one kernel; each particle stays in registers through all elements */
#define HBL_UNFUSED 1u /* one kernel per element (comparator) */

/* ASYNC.  Push the bunch through the lattice in place.  ref->gamma must equal
 * the gamma the lattice was compiled for; ref->s advances by its length.
 * Fused and unfused paths give bitwise identical results. */
hbl_status hbl_push_lattice(double* z, int64_t n, int64_t ld, const hbl_lattice* lat,
                            hbl_ref* ref, uint32_t flags, hbl_stream stream);

/* ---------------------------------------------------------------- stage */

/* ASYNC.  Fine-step reference map of one plasma-accelerator stage (the LPA
 * stage of §4, a nonlinear per-particle map; the paper models it with PIC).
 * Model: linear ion-channel focusing du/ds = -(k_p^2/2) x on u = p_x/(m c),
 * drift dx/ds = u/gamma_i(s) with the particle's own gamma_i(s) =
 * gamma_ref(s) + dgamma_i, gamma_ref ramping linearly by dE over L, nsub
 * kick-drift-kick substeps; every particle gains the same energy.  ref->gamma
 * and ref->s advance.  If `record` is not NULL (rows at record + j*record_ld,
 * same alignment rules) it receives a copy of the input bunch, so the call
 * emits (input, output) training pairs (§3). */
hbl_status hbl_apply_stage(double* z, int64_t n, int64_t ld, const hbl_element* stage,
                           hbl_ref* ref, double* record, int64_t record_ld, hbl_stream stream);

/* Host only.  Newton steps per substep that hbl_apply_stage uses for the
 * particle's 1/gamma_i at the given entry reference: the reciprocal of the
 * previous substep has relative error at most d = |gamma ramp per substep| /
 * (0.9 min(gamma_in, gamma_out)) (twice that for a chirped stage), k steps
 * leave d^(2^k), and the fewest k in 1..4 with d^(2^k) < 1e-17 is taken;
 * *steps = 0 means every substep divides.  Validates like hbl_apply_stage. */
hbl_status hbl_stage_newton_steps(const hbl_element* stage, const hbl_ref* ref, int32_t* steps);

/* ASYNC.  One pass over the bunch equivalent to hbl_push_lattice(pre),
 * hbl_apply_stage(stage), hbl_push_lattice(post): the transport gaps before
 * and after the stage (§4, Fig. 1: stages joined by transport sections) are
 * applied in registers by the stage kernel.  pre and post are nullable; pre
 * must be compiled for ref->gamma, post for the stage's exit gamma.  record
 * (nullable) receives the stage input, i.e. the bunch after pre.  Results
 * are bitwise those of the three separate calls. */
hbl_status hbl_apply_stage_gaps(double* z, int64_t n, int64_t ld, const hbl_lattice* pre,
                                const hbl_element* stage, const hbl_lattice* post, hbl_ref* ref,
                                double* record, int64_t record_ld, hbl_stream stream);

/* ---------------------------------------------------------------- diagnostics */

/* SYNC.  Beam moments (§4): mean6[j] = <z_j>; cov21 = centred population
 * covariance <(z_j - <z_j>)(z_k - <z_k>)>, upper triangle row-major
 * (00,01,..,05,11,..,55).  Unweighted.  Compensated FP64 (double-double)
 * reduction in a fixed order: bitwise reproducible.  HBL_ENONFINITE if the
 * bunch holds NaN/Inf.  n >= 1. */
hbl_status hbl_moments(const double* z, int64_t n, int64_t ld, double mean6[6], double cov21[21],
                       hbl_stream stream);
/* ASYNC variant: writes the 27 doubles (mean6 then cov21) to DEVICE memory
 * out27 (8-byte aligned). */
hbl_status hbl_moments_async(const double* z, int64_t n, int64_t ld, double* out27,
                             hbl_stream stream);
/* ASYNC, allocates nothing.  For callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and kernels as hbl_moments_async, with
 * identical results, but the reduction's scratch is a fixed array of
 * 442,800 bytes that the library holds in each device's memory until the
 * process ends (looked up on a device's first call; no hipMalloc, hipFree or
 * allocating library call is made).  Every n >= 1 fits in it (the reduction
 * grid is capped); a size that did not would be rejected with HBL_EINVAL
 * before anything is enqueued.  All calls on one device share that device's
 * array and nothing in it needs clearing between calls: two calls that can
 * overlap on one device (different streams, or different threads) race on
 * it, so keep them on one stream.  The scratch is not shared with the other
 * reductions' workspaces. */
hbl_status hbl_moments_async_noalloc(const double* z, int64_t n, int64_t ld, double* out27,
                                     hbl_stream stream);
/* Host only.  Geometric RMS emittances of (x,px), (y,py), (t,pt),
 * eps = sqrt(<dx^2><dpx^2> - <dx dpx>^2) (§4). */
hbl_status hbl_emittances(const double cov21[21], double eps3[3]);
/* SYNC.  Error metrics of a test bunch zs against a reference bunch zf (same
 * n, ld): rms6[j] = sqrt(<(s_j - f_j)^2>)/sigma_f,j; centroid6[j] =
 * (<s_j> - <f_j>)/sigma_f,j; eps_rel3[p] = eps_s,p/eps_f,p - 1. */
hbl_status hbl_compare(const double* zs, const double* zf, int64_t n, int64_t ld, double rms6[6],
                       double centroid6[6], double eps_rel3[3], hbl_stream stream);

/* ---------------------------------------------------------------- surrogate */

/* Neural-network stage surrogate (§3): the feed-forward network of Eq. (3),
 * F = L_H o tanh o ... o tanh o L_0, L_i(x) = A_i x + b_i, acting on the six
 * coordinates normalised per direction by the mean and standard deviation of
 * the training inputs and outputs (§3); trained on the mean-squared error of
 * Eq. (4) with Adam.  The kernels support the shape {6, 64, 3, 6} (three
 * hidden layers of 64).  Dense layers run on the matrix cores in bf16 with
 * FP32 accumulation; tanh and normalisation in FP32/FP64; the output layer
 * result stays FP32 and is de-normalised in FP64.  Rounding points, which
 * bound how far results may lie from the FP64 network: hidden and output
 * layers take bf16 weights and bf16 activations (8 significant bits); the
 * first layer keeps 16 significant bits of its FP32 input and weights (a
 * bf16 hi + lo split); tanh has absolute error below 2^-20; in training, the
 * errors back-propagated into layers 1..3 and the weights they meet enter the
 * products in bf16, the first layer's weight gradient is FP32.  FP32 master parameters,
 * flat layout A_0 (64x6, row-major [out][in]), b_0, A_1, b_1, A_2, b_2, A_3
 * (6x64), b_3: 9158 floats. */
typedef struct hbl_surrogate hbl_surrogate;
typedef struct hbl_mlp_shape {
    int32_t n_in, width, hidden, n_out;
} hbl_mlp_shape;

/* Training recipe.  batch: multiple of 64; epochs >= 0; max_steps < 0 = no
 * limit, else training stops after that many optimizer steps.  Learning
 * rate: lr at the first step, annealed by a half cosine to lr_final at the
 * last of the T planned steps, lr_t = lr_final + (lr - lr_final)(1 +
 * cos(pi (t-1)/(T-1)))/2 (constant when lr_final == lr).  The first
 * round(train_frac * n_pairs) pairs train, the rest test (§3: 70/30); each
 * epoch visits the training pairs in a Fisher-Yates order (Philox4x32-10,
 * key shuffle_seed, counter (i/4, epoch, 'SHUF'), word i%4, j = floor(r (i+1)
 * / 2^32)) in batches, dropping the last partial batch.  keep_best selects,
 * when there is a test split, which epoch's parameters the training ends
 * with (model selection on the held-out pairs, tracked on the device with no
 * host synchronisation per epoch; the Adam moments and step stay those of the
 * last step): 0, the last epoch's; 1, those of the lowest test loss; 2, among
 * the epochs of the last quarter (at least the last) whose test loss is
 * within 10 % of the lowest test loss of those epochs, those whose predicted
 * test outputs have the emittances of (x, px) and (y, py) (§4) closest to
 * those of the true test outputs (the lowest max over the two planes of
 * |eps_pred / eps_true - 1|; keeps a 36.6 KB parameter snapshot per epoch of
 * that quarter in device memory during the call).  resume (0 or 1): with 1
 * the call continues an earlier training of this handle (or of the model it
 * was loaded from): the normalisation, the Adam moments and the step count
 * are kept, not reset; the step count must be a whole number E of epochs of
 * this call's recipe, and the epochs are numbered from E on (their
 * Fisher-Yates orders are those of epochs E, E + 1, ...); the learning-rate
 * schedule spans this call's steps.  With the same pairs, recipe and a
 * constant rate, training E epochs, saving, loading and resuming for F more
 * gives the parameters of one run of E + F epochs, bit for bit. */
typedef struct hbl_train_cfg {
    int32_t batch;
    int32_t epochs;
    int64_t max_steps;
    float lr, lr_final, beta1, beta2, eps;
    double train_frac;
    uint64_t shuffle_seed;
    int32_t keep_best;
    int32_t resume;
} hbl_train_cfg;

/* Create a surrogate with parameters U(-1/sqrt(fan_in), 1/sqrt(fan_in)):
 * parameter p takes word 0 of Philox4x32-10 block (p, 0, 0, 'MLPI') keyed by
 * init_seed, u = (word >> 8) 2^-24, value (2u - 1) / sqrt(fan_in).
 * Synchronous.  Only shape {6, 64, 3, 6} is accepted. */
hbl_status hbl_surrogate_create(const hbl_mlp_shape* shape, uint64_t init_seed, hbl_surrogate** out);
hbl_status hbl_surrogate_destroy(hbl_surrogate* m);
/* Number of FP32 parameters (9158). */
hbl_status hbl_surrogate_num_params(const hbl_surrogate* m, int64_t* n);
/* SYNC.  Copy the FP32 master parameters to / from host memory (n floats). */
hbl_status hbl_surrogate_get_params(const hbl_surrogate* m, float* host, int64_t n);
hbl_status hbl_surrogate_set_params(hbl_surrogate* m, const float* host, int64_t n);
/* Normalisation: norm24 = mean_in[6], sd_in[6], mean_out[6], sd_out[6]
 * (host FP64; sd > 0).  Training sets it from the training split. */
hbl_status hbl_surrogate_get_norm(const hbl_surrogate* m, double norm24[24]);
hbl_status hbl_surrogate_set_norm(hbl_surrogate* m, const double norm24[24]);
/* Declare the stage the surrogate replaces: applying it moves the reference
 * particle as the stage would (gamma by dE/mass, s by L).  at_entry->gamma is
 * the entry energy it was trained for. */
hbl_status hbl_surrogate_set_stage(hbl_surrogate* m, const hbl_element* stage, const hbl_ref* at_entry);

/* Train on n_pairs (input, output) pairs (zin, zout: DEVICE bunches, same
 * ld; e.g. recorded by hbl_apply_stage).  Computes the normalisation from the
 * training split, resets the Adam state, then runs cfg->epochs epochs
 * entirely on the device (forward, MSE, backward, Adam and the per-epoch test
 * loss are this library's kernels).  SYNC at the end.  loss_log (host,
 * nullable, 2*epochs floats): mean training-batch loss and test loss per
 * epoch, in normalised units.  Every buffer it uses is the handle's, its own
 * or its stream's, so trainings of different handles on different streams
 * (from different host threads) may run at the same time; each gives the
 * result it gives alone. */
hbl_status hbl_surrogate_train(hbl_surrogate* m, const double* zin, const double* zout, int64_t n_pairs,
                               int64_t ld, const hbl_train_cfg* cfg, float* loss_log, hbl_stream stream);

/* SYNC.  Loss and gradient of one batch at the current parameters and
 * normalisation, without updating: idx (host, batch int32 indices into the
 * pairs, batch a multiple of 64), grad (host, 9158 floats), loss (host). */
hbl_status hbl_surrogate_loss_grad(hbl_surrogate* m, const double* zin, const double* zout, int64_t ld,
                                   const int32_t* idx, int32_t batch, float* grad, double* loss,
                                   hbl_stream stream);

/* ASYNC.  Apply the surrogate to the bunch in place (inference, §4.3): the
 * stage it stands for, taken by the network; advances ref like the stage when
 * one was declared (ref->gamma must then equal the declared entry gamma).
 * Needs a normalisation (set or trained). */
hbl_status hbl_surrogate_apply(double* z, int64_t n, int64_t ld, const hbl_surrogate* m, hbl_ref* ref,
                               hbl_stream stream);

/* ASYNC.  hbl_push_lattice(pre), hbl_surrogate_apply, hbl_push_lattice(post)
 * in one pass over the bunch (the gaps applied in registers by the inference
 * kernel).  Needs a declared stage; pre compiled for ref->gamma, post for
 * the exit gamma; both nullable.  Bitwise equal to the separate calls. */
hbl_status hbl_surrogate_apply_gaps(double* z, int64_t n, int64_t ld, const hbl_lattice* pre,
                                    const hbl_surrogate* m, const hbl_lattice* post, hbl_ref* ref,
                                    hbl_stream stream);

/* Save / load the model (shape, normalisation, stage, FP32 parameters, Adam
 * moments and step) to a binary file with a checksum.  HBL_EIO on I/O or
 * format errors. */
hbl_status hbl_surrogate_save(const hbl_surrogate* m, const char* path);
hbl_status hbl_surrogate_load(const char* path, hbl_surrogate** out);

/* ------------------------------------------------------ wide PReLU surrogate */

/* The network shape the paper trains for its stages (§3 Eq. 2 and 3; §4.2:
 * three hidden layers of 700 for most stages, five of 900 for the first
 * ones): shape {6, W, H, 6} with 8 <= W <= 1024 and 1 <= H <= 7, hidden
 * layers h_{l+1} = PReLU_{a_l}(A_l h_l + b_l), PReLU_a(v) = v for v > 0 and
 * a v otherwise, one learned slope a_l per hidden layer; output A_H h_H + b_H;
 * the same per-direction normalisation as the tanh surrogate.  FP32 master
 * parameters, flat layout A_0 (W x 6, row-major [out][in]), b_0, a_0, A_1
 * (W x W), b_1, a_1, ..., A_{H-1}, b_{H-1}, a_{H-1}, A_H (6 x W), b_H:
 * 6W + W + 1 + (H - 1)(W^2 + W + 1) + 6W + 6 floats.
 * Arithmetic: the first layer in FP32 on the vector ALU (FP32 network input);
 * the W x W layers and the output layer as bf16 products with FP32
 * accumulation on the matrix cores, bias and PReLU in FP32, each hidden
 * activation rounded to bf16; output FP32, de-normalised in FP64.
 * Device memory held by a network: its parameters, their bf16 image (for
 * 512 <= W' <= 960 with a second, K-blocked copy of the W x W layers) and two
 * activation buffers of chunk x W' bf16 (W' = W rounded up to 64; 2 x 126 MB
 * at W = 900), allocated at creation.  Calls that use one network must be
 * ordered (one stream, or synchronised): they share those buffers. */
typedef struct hbl_prelu_net hbl_prelu_net;

/* Weights and biases U(-1/sqrt(fan_in), 1/sqrt(fan_in)), parameter p (flat
 * index) from word 0 of Philox4x32-10 block (p, 0, 0, 'MLPI') keyed by
 * init_seed, u = (word >> 8) 2^-24, value (2u - 1)/sqrt(fan_in); slopes 0.25.
 * Synchronous.  HBL_EINVAL for a shape outside the limits above. */
hbl_status hbl_prelu_create(const hbl_mlp_shape* shape, uint64_t init_seed, hbl_prelu_net** out);
hbl_status hbl_prelu_destroy(hbl_prelu_net* m);
hbl_status hbl_prelu_num_params(const hbl_prelu_net* m, int64_t* n);
/* SYNC.  Copy the FP32 parameters to / from host memory (n floats, finite). */
hbl_status hbl_prelu_get_params(const hbl_prelu_net* m, float* host, int64_t n);
hbl_status hbl_prelu_set_params(hbl_prelu_net* m, const float* host, int64_t n);
/* SYNC.  Particles per inference chunk (default 98304 at 512 <= W' <= 832,
 * 65536 otherwise; a multiple of 256 in
 * [256, 2^22]): the two activation buffers hold chunk x W' bf16 each.
 * Smaller chunks keep the activations in the last-level cache; larger ones
 * give each layer launch more workgroups.  HBL_ENOMEM leaves the old ones. */
hbl_status hbl_prelu_set_chunk(hbl_prelu_net* m, int64_t particles);
/* norm24 as for hbl_surrogate_set_norm (host FP64, sd > 0). */
hbl_status hbl_prelu_set_norm(hbl_prelu_net* m, const double norm24[24]);
hbl_status hbl_prelu_get_norm(const hbl_prelu_net* m, double norm24[24]);
/* Declare the stage the network replaces (as hbl_surrogate_set_stage). */
hbl_status hbl_prelu_set_stage(hbl_prelu_net* m, const hbl_element* stage, const hbl_ref* at_entry);
/* ASYNC.  Inference in place on n particles of the DEVICE bunch z (§4.3),
 * in chunks (hbl_prelu_set_chunk); advances ref like the declared stage. */
hbl_status hbl_prelu_apply(double* z, int64_t n, int64_t ld, const hbl_prelu_net* m, hbl_ref* ref,
                           hbl_stream stream);
/* ASYNC.  pre lattice, the network, post lattice in the same launches (pre
 * applied where the network input is formed, post where its output is
 * written); needs a declared stage; lattices as for hbl_surrogate_apply_gaps. */
hbl_status hbl_prelu_apply_gaps(double* z, int64_t n, int64_t ld, const hbl_lattice* pre,
                                const hbl_prelu_net* m, const hbl_lattice* post, hbl_ref* ref,
                                hbl_stream stream);

/* SYNC.  Loss (Eq. 4, normalised units) and gradient of one batch at the
 * current parameters and normalisation, without updating: idx (host, batch
 * indices into the pairs, 1 <= batch <= 16384), grad (host, num_params
 * floats, flat layout), loss (host).  Forward as inference, keeping the bf16
 * pre-activations and activations; the output error, every back-propagated
 * error and the activations enter bf16 matrix-core products with FP32
 * accumulation (weight gradients as products over the batch, including the
 * bias through a constant-one activation row); slope gradients are FP32
 * sums over the batch. */
hbl_status hbl_prelu_loss_grad(hbl_prelu_net* m, const double* zin, const double* zout, int64_t ld,
                               const int32_t* idx, int32_t batch, float* grad, double* loss,
                               hbl_stream stream);
/* Train as hbl_surrogate_train (normalisation from the training split, Adam
 * reset, half-cosine learning rate, Fisher-Yates epoch order, test loss per
 * epoch), entirely on the device; batch any size in [1, 16384] (§4.2 uses
 * 1200).  cfg->keep_best and cfg->resume must be 0 here (HBL_EINVAL
 * otherwise).  SYNC at the end; loss_log as for hbl_surrogate_train. */
hbl_status hbl_prelu_train(hbl_prelu_net* m, const double* zin, const double* zout, int64_t n_pairs,
                           int64_t ld, const hbl_train_cfg* cfg, float* loss_log, hbl_stream stream);

/* Save / load the network (shape, normalisation, stage, FP32 parameters,
 * Adam moments when it has trained, step) to a binary file with a checksum.
 * HBL_EIO on I/O or format errors. */
hbl_status hbl_prelu_save(const hbl_prelu_net* m, const char* path);
hbl_status hbl_prelu_load(const char* path, hbl_prelu_net** out);

#ifdef __cplusplus
}
#endif
#endif /* HBL_H */
