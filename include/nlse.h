/*
 * nlse.h -- C ABI of the MI355X (gfx950) 2SHOC-RK4 solver for the nonlinear
 * Schroedinger / Gross-Pitaevskii equation
 *
 *     i Psi_t + a Lap(Psi) - V(r) Psi + s |Psi|^2 Psi = 0,   a > 0      (Sec. 1, Eq. NLSE)
 *
 * on a uniform 1D, 2D or 3D grid with the same step h on every axis (Sec. 2).
 * Each RK4 step (Sec. 3.1, Eq. RK4) evaluates F(Psi) = i[a Lap + (s|Psi|^2 - V)Psi]
 * four times; Lap is the two-step high-order compact (2SHOC) Laplacian
 * (Sec. 2.1-2.3): step 1 a second difference D, step 2 a compact combination of
 * D that is fourth-order accurate.  Boundary closures follow Sec. 3.2 (Dirichlet
 * Eqs. dbc_lap / dbc_ut; modulus-squared Dirichlet, Eqs. msdbc_lap / msdbc_ut, in
 * 1D, 2D and 3D).  Every step runs in hand-written HIP kernels on the GPU.
 *
 * Conventions shared by every entry point
 *   - Grid: n[a] intervals per axis, n[a] + 1 nodes including both boundary
 *     nodes; node i on axis a sits at x_min + i h.
 *   - Fields: dense, C order [z][y][x] (x fastest), complex values interleaved
 *     (re, im).  Element type: complex128 (two doubles) for NLSE_F64 and
 *     NLSE_F32_MIXED, complex64 (two floats) for NLSE_F32.
 *   - Pointers flagged on_device are device pointers (e.g. from torch) and the
 *     copy is ordered on the context's stream; otherwise they are host pointers
 *     and the call returns when the copy is complete.  The library never keeps
 *     a caller pointer: inputs are copied in, outputs copied out.
 *   - Ownership: a context owns all its device memory; nlse_destroy frees it.
 *   - Streams: all GPU work of a context is enqueued on params.stream (a
 *     hipStream_t; NULL = the default stream).  nlse_step returns without
 *     waiting; nlse_mass / nlse_energy / nlse_max_dt and host-side
 *     get_field wait for the stream.
 *   - Errors: every call returns an nlse_status; on failure nlse_last_error()
 *     returns a thread-local message.  No exception crosses the ABI.  A context
 *     must not be used from two threads at once.
 */
#ifndef NLSE_H
#define NLSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nlse_ctx nlse_ctx;

typedef enum {
    NLSE_OK = 0,
    NLSE_E_INVAL = -1,         /* NULL pointer, bad size, a <= 0, h <= 0, ... */
    NLSE_E_DT_UNSTABLE = -2,   /* dt above the stability bound (see nlse_step) */
    NLSE_E_NONFINITE = -3,     /* a reduction met NaN or Inf in the field */
    NLSE_E_NOMEM = -4,         /* device allocation failed */
    NLSE_E_HIP = -5,           /* a HIP runtime call failed */
    NLSE_E_UNSUPPORTED = -6    /* valid but not implemented (e.g. a 1D field too large
                                  for the on-chip solver) */
} nlse_status;

typedef enum {
    NLSE_F64 = 0,        /* complex128 storage and arithmetic */
    NLSE_F32 = 1,        /* complex64 storage and arithmetic */
    NLSE_F32_MIXED = 2   /* complex64 stage fields, stencil and RK4 stage sums;
                            complex128 master Psi^n: the final RK4 accumulation
                            Psi^{n+1} = Psi^n + (k/6)(K_tot + K_4) adds an FP32
                            increment in FP64; mass / energy in FP64 */
} nlse_precision;

typedef enum {
    NLSE_BC_DIRICHLET = 0, /* boundary nodes keep their initial values (Eq. dbc_ut);
                              step-1 boundary value from Eq. dbc_lap */
    NLSE_BC_MSD = 1        /* |Psi_b|^2 constant (Eqs. msdbc_ut, msdbc_lap).  b-1 is the
                              closest interior node: the normal neighbour on a face, the
                              diagonal one on an edge or corner (2D/3D; Sec. 3.2 says the rule
                              carries over to several dimensions, the corner choice is ours).
                              1D needs n >= 4 intervals.  2D/3D run the stage kernels with one
                              small boundary launch before each stage */
} nlse_bc;

typedef enum {
    NLSE_STENCIL_2SHOC = 0,       /* the two-step compact scheme (Sec. 2), the default */
    NLSE_STENCIL_NONCOMPACT = 1,  /* non-compact fourth-order stencil per axis, the scheme 2SHOC
                                     is compared with (Sec. 2.1, Sec. 5); one node beyond a
                                     boundary node b it reads the ghost 2 Psi_b - Psi_{b+-1}
                                     + h^2 D^a_b, D^a_b the step-1 face value of Eq. dbc_lap,
                                     so it equals 2SHOC up to rounding for any Dirichlet data */
    NLSE_STENCIL_CD = 2           /* second-order central difference (Sec. 3.1's CD) */
} nlse_stencil;

typedef struct {
    int32_t ndim;          /* 1, 2 or 3 */
    int64_t n[3];          /* intervals per axis (n[a] >= 2 for a < ndim) */
    double h;              /* grid step, > 0, the same on every axis */
    double a;              /* dispersion coefficient, > 0 */
    double s;              /* nonlinearity coefficient */
    const double *V;       /* host array of (n+1)^ndim reals in field order, or NULL for V = 0;
                              copied at nlse_create */
    int32_t bc;            /* nlse_bc */
    int32_t prec;          /* nlse_precision */
    int32_t allow_unstable;/* nonzero: nlse_step skips the dt check */
    void *stream;          /* hipStream_t or NULL */
} nlse_params;

/* Create a context: validates params, allocates the resident device arrays
 * (Psi^n, two ping-pong stage fields, K_tot, V) and copies V.  The field is
 * zero until nlse_set_field.  Returns NLSE_E_INVAL for invalid params,
 * NLSE_E_UNSUPPORTED for a 1D field larger than the on-chip solver holds or a 3D
 * field of 2^31 or more padded elements (the 3D kernels use 32-bit offsets; about
 * 1290^3 nodes), and NLSE_E_NOMEM when the device arrays cannot be allocated. */
int nlse_create(nlse_ctx **out, const nlse_params *p);

/* Copy a full field (all (n+1)^ndim nodes, boundary included) into the context.
 * psi: contiguous, x fastest, the context's master type (complex128 for F64 and
 * F32_MIXED, complex64 for F32); on_device nonzero: a device pointer, copied on the
 * context stream; zero: host memory, copied through a temporary device buffer of the
 * field's size (allocated and freed within the call; the call waits for the stream).
 * Under Dirichlet the boundary values given here are held fixed from then on.
 * Also evaluates the stability bound of nlse_max_dt on this field (waits for
 * the stream) and stores it for nlse_step's check. */
int nlse_set_field(nlse_ctx *c, const void *psi, int on_device);

/* Advance nsteps classic RK4 steps of size dt (Sec. 3.1), enqueued on the
 * context stream (asynchronous).  Returns NLSE_E_DT_UNSTABLE, doing nothing,
 * when dt exceeds the bound stored by the last nlse_set_field and the context
 * was created with allow_unstable = 0; NLSE_E_INVAL for dt <= 0 or nsteps < 0. */
int nlse_step(nlse_ctx *c, int64_t nsteps, double dt);

/* Copy the current field out (same layout and element type as nlse_set_field; host
 * memory goes through a temporary device buffer as there, and the call waits for the
 * stream; a device pointer is filled asynchronously on the context stream). */
int nlse_get_field(nlse_ctx *c, void *out, int on_device);

/* Mass h^d sum_{all nodes} |Psi|^2, accumulated in FP64 in a fixed order
 * (bitwise reproducible run to run).  NLSE_E_NONFINITE if the sum is not finite. */
int nlse_mass(nlse_ctx *c, double *out);

/* Energy h^d sum_{interior} [ -a Re(conj(Psi) Lap Psi) + V|Psi|^2 - (s/2)|Psi|^4 ]
 * with the 2SHOC Laplacian, accumulated in FP64 (the Hamiltonian of Eq. NLSE). */
int nlse_energy(nlse_ctx *c, double *out);

/* Linearised stability bound on the current field (Sec. 3.3, Eq. kdfull):
 *   k_max = sqrt(8) h^2 / (a max(|B|_inf, G_max - L_min, L_max - G_min)),
 *   L_i = (h^2/a)(s|Psi_i|^2 - V_i) over interior nodes, (G_max, G_min) =
 *   (64, -4)/12, (128, -8)/12, (192, -12)/12 in 1D / 2D / 3D (Table
 *   t:sumresults), B_b = 0 for Dirichlet and (h^2/(i a)) F_{b-1}/Psi_{b-1} for
 *   MSD (Table t:bc2), over every node b-1 the MSD rule reads. */
int nlse_max_dt(nlse_ctx *c, double *out);

/* Wait until all work enqueued by the context has finished. */
int nlse_sync(nlse_ctx *c);

/* Free everything the context owns.  NULL is ignored. */
void nlse_destroy(nlse_ctx *c);

/* Message describing the last failure on the calling thread ("" if none). */
const char *nlse_last_error(void);

/* Number of kernel launches one RK4 step enqueues for this context with its current
 * variant: 4 for the 2D/3D stage kernels (8 under MSD: a boundary launch, face values
 * and boundary nodes, before each stage), 1 for the 2D whole-step kernels (Dirichlet and
 * MSD) and 2 for the 3D two-stage kernels (Dirichlet only); 1D contexts advance all steps in
 * one launch and report 0.  For throughput accounting. */
int nlse_launches_per_step(const nlse_ctx *c);

/* Kernel variants.  2D: 0-2 are the stage kernels (one launch per RK4 stage, tiles of
 * 64 columns x 8, 4 or 16 rows per wave); 3-9 the whole-step kernels (one launch per RK4
 * step, Sec. 3.1 with all four stages fused; a wave walks a 64-column strip down a segment
 * of 29, 20, 38, 56, 11, 47 or 29 rows, the last with two rows of Psi^n in flight instead
 * of one; offered when the padded field has fewer than 2^31 elements).  Under MSD (2D, at
 * least 2 intervals per axis) the whole-step kernels form the face values and the boundary
 * nodes of Eqs. msdbc_lap and msdbc_ut themselves, and the strips that hold a face column
 * take segments of about half as many rows; their results equal the MSD stage kernels' to the
 * last place except for rare one-unit differences of it that start on the face y = 0.
 * 3D: 0-3 stage kernels with 64 x 4 or 64 x 8 column tiles marching 16, 32 or 64 planes;
 * 4-6 (Dirichlet, fields below 2^31 elements) two launches per step, each fusing two stages
 * (1+2, 3+4) on 64 x 16 or 64 x 8 column tiles marching 32 or 64 planes.
 * 1D: the on-chip solver with 512 threads holding up to 10 (FP64) or 18 (FP32, mixed)
 * nodes each (0), 256 threads with as many (1), 512 threads with at most 4 (2) or 3 (3)
 * nodes each; a variant is offered only while it holds the field (5120 / 9216, 2560 /
 * 4608, 2048 and 1536 nodes), so the count is 1 to 4.
 * Every variant computes bit-identical fields; they differ only in speed. */
int nlse_variant_count(const nlse_ctx *c);
int nlse_set_variant(nlse_ctx *c, int variant);   /* NLSE_E_INVAL if out of range */
int nlse_get_variant(const nlse_ctx *c);

/* Laplacian of the right-hand side (Dirichlet boundaries; NLSE_E_UNSUPPORTED for the
 * alternatives under MSD, NLSE_E_INVAL for an unknown value).  The non-compact stencil
 * is one five-point difference per axis: the 1D stencil of Sec. 2.1, the 9-point cross of
 * Eq. 2dnonhoc in 2D, the 13-point cross in 3D (Sec. 2.3).  In 2D every variant runs them
 * (stage and whole-step kernels); in 3D they run in the stage kernels only, so the
 * two-stage variants disappear from the variant list while they are selected (such a
 * variant then reverts to variant 0); the 1D on-chip solver runs them in every variant.
 * nlse_max_dt keeps the 2SHOC bound of Eq. kdfull (the non-compact stencil has the
 * same spectral radius, CD a smaller one), and nlse_energy always uses the 2SHOC
 * Laplacian.  For the comparisons of Sec. 5 on this hardware. */
int nlse_set_stencil(nlse_ctx *c, int32_t stencil);
int nlse_get_stencil(const nlse_ctx *c);

/* Autotuner: times `reps` RK4 steps of every variant on this context's own arrays
 * (twice, keeping the fastest), selects the fastest and caches the choice for the
 * process under (ndim, precision, n, stencil, boundary rule).  Later calls reuse the cached choice unless
 * force != 0.  Needs a field (nlse_set_field).  The field is saved to a temporary
 * device buffer first and restored afterwards, so the integration state is unchanged;
 * NLSE_E_NOMEM if that buffer cannot be allocated.  Waits for the stream.  The chosen
 * variant is returned in *chosen (may be NULL). */
int nlse_autotune(nlse_ctx *c, int reps, int force, int *chosen);

/* ---------------------------------------------------------------- batches --
 * Many independent 1D / 2D problems of uneven size advanced together by one
 * persistent kernel launch (captured in a hipGraph).  Each instance has its own
 * grid, coefficients, potential, boundary rule (MSD for 1D only: 2D instances
 * with MSD give NLSE_E_UNSUPPORTED) and step dt; all
 * share the precision and the stream of items[0].  Workgroups take instances
 * longest-first from a device queue; a 1D instance (at most 8704 nodes in FP32 /
 * mixed, 5120 in FP64) runs entirely on chip, a 2D instance is swept tile by tile
 * by one workgroup.  Results are identical to advancing each instance alone. */
typedef struct nlse_batch nlse_batch;

/* items[i] as for nlse_create (ndim 1 or 2).  Allocates every instance. */
int nlse_batch_create(nlse_batch **out, const nlse_params *items, int32_t count);
int32_t nlse_batch_count(const nlse_batch *b);
/* Field of instance i (as nlse_set_field; also evaluates that instance's bound). */
int nlse_batch_set_field(nlse_batch *b, int32_t i, const void *psi, int on_device);
int nlse_batch_get_field(nlse_batch *b, int32_t i, void *out, int on_device);
/* Step size of instance i; NLSE_E_DT_UNSTABLE above its bound unless allow_unstable. */
int nlse_batch_set_dt(nlse_batch *b, int32_t i, double dt);
int nlse_batch_max_dt(nlse_batch *b, int32_t i, double *out);
int nlse_batch_mass(nlse_batch *b, int32_t i, double *out);
/* Every instance advances nsteps RK4 steps of its own dt: one graph launch on the
 * stream (asynchronous).  NLSE_E_INVAL if an instance lacks a field or a dt. */
int nlse_batch_step(nlse_batch *b, int64_t nsteps);
int nlse_batch_sync(nlse_batch *b);
/* Variants of the 2D instances (row segments of 56, 29 or 20 rows for the whole-step wave
 * body) and the autotuner: per variant one untimed call of nsteps (graph capture and first
 * launch), then the fastest of three timed launches of that graph; the state is restored
 * after every call.  A 1D instance always runs the on-chip solver body with the smallest
 * node bound per thread that holds it. */
int nlse_batch_variant_count(const nlse_batch *b);
int nlse_batch_set_variant(nlse_batch *b, int variant);
int nlse_batch_get_variant(const nlse_batch *b);
int nlse_batch_autotune(nlse_batch *b, int64_t nsteps, int force, int *chosen);
void nlse_batch_destroy(nlse_batch *b);

/* ------------------------------------------------------ learned corrector --
 * A 3-layer 3x3 convolutional network that corrects a coarse 2D field every few
 * RK4 steps: Psi <- Psi + scale (Y0 + i Y1) on interior nodes, with
 *   A0 = bf16(features(Psi)), 8 channels per node: Re Psi, Im Psi, 16 Re(h^2 L Psi),
 *        16 Im(h^2 L Psi), |Psi|^2, V/4, 0, 0  (L: five-point Laplacian, zero outside),
 *   A1 = bf16(silu(conv(A0, W1) + b1)), A2 = bf16(silu(conv(A1, W2) + b2)) (32 channels),
 *   Y  = conv(A2, W3) + b3 (2 channels, FP32), zero padding at the grid edge.
 * Weights are FP32 masters rounded to bf16 for the BF16 MFMA units (FP32 accumulate).
 * Parameter vector (nlse_corr_param_count() floats): W1[32][9][8] b1[32] W2[32][9][32]
 * b2[32] W3[2][9][32] b3[2], tap t = 3(dy+1) + (dx+1).  Dense field arguments are
 * device pointers to complex64 [batch][H][W], ordered on the corrector's stream.
 * A corrector is used on one stream at a time; its workspace is reused by every call. */
typedef struct nlse_corr nlse_corr;

int32_t nlse_corr_param_count(void);
/* Workspace for fields of H x W nodes and up to max_batch fields per call; V: host
 * potential [H][W] (the V channel of the features), may be NULL for V = 0. */
int nlse_corr_create(nlse_corr **out, int32_t H, int32_t W, int32_t max_batch, const double *V, void *stream);
/* Host FP32 parameters and the output scale; resets the Adam moments. */
int nlse_corr_set_params(nlse_corr *m, const float *params, double scale);
int nlse_corr_get_params(nlse_corr *m, float *params);
/* Network output Y (before scaling) for `batch` fields: y_out device FP32 [batch][H][W][2]. */
int nlse_corr_infer(nlse_corr *m, const void *psi, int32_t batch, float *y_out);
/* Training on pairs (pred, ref): pred = coarse field after the coarse steps, ref = the
 * reference (restricted fine) field at the same time.  Loss = mean over interior nodes
 * and both channels of (Y - (ref - pred)/scale)^2.  nlse_corr_grads returns the FP32
 * gradient of the loss (host array, may be NULL) and the loss; nlse_corr_train_step
 * also applies one Adam step (beta 0.9 / 0.999, eps 1e-8) with learning rate lr. */
int nlse_corr_grads(nlse_corr *m, const void *pred, const void *ref, int32_t batch, float *grads, double *loss);
int nlse_corr_train_step(nlse_corr *m, const void *pred, const void *ref, int32_t batch, double lr, double *loss);
/* smooth = R in 1..4: the training target is (ref - pred) filtered by the binomial
 * kernel of width 2R + 1 along each axis (C(2R, k) / 4^R: [1 2 1]/4, [1 4 6 4 1]/16, ...),
 * so the network learns only resolved-scale corrections; 0: unfiltered.
 * NLSE_E_INVAL outside 0..4. */
int nlse_corr_set_target_filter(nlse_corr *m, int32_t smooth);
/* Training-input augmentation: Gaussian noise of standard deviation sigma (per real and
 * imaginary part, interior nodes) added to pred before its features are formed; the
 * target still uses the unperturbed pred.  Counter-based (splitmix64 + Box-Muller) from
 * seed and the Adam step, so a training run is reproducible.  sigma = 0 disables it.
 * Inference (nlse_corr_infer / apply / step_corrected) never adds noise. */
int nlse_corr_set_augment(nlse_corr *m, double sigma, uint64_t seed);
/* Validation access to the training passes, layer by layer (tests compare each stage with a
 * CPU reference on the same inputs).  nlse_corr_tensor copies `bytes` bytes between a host
 * array and an internal tensor (to_device != 0: host -> tensor; waits for the stream).
 * Layouts are NHWC over the batch's pixels P = batch x H x W: X0 bf16 [P][8] (the features),
 * A1 / A2 bf16 [P][32], Z1 / Z2 FP32 [P][32] (pre-activations), Y FP32 [P][2], dY bf16 [P][8]
 * (channels 0-1 used), dZ2 / dZ1 bf16 [P][32], GRADS FP32 in the parameter vector's layout;
 * bf16 values are raw 16-bit patterns.  nlse_corr_stage runs one stage on them:
 *   FWD1: Z1 = conv(X0, W1) + b1, A1 = bf16(silu(Z1));  FWD2: the same from A1 to Z2, A2;
 *   FWD3: Y = conv(A2, W3) + b3;
 *   WGRAD3 / WGRAD2 / WGRAD1: gradients of W3, b3 (from A2, dY), W2, b2 (A1, dZ2), W1, b1
 *   (X0, dZ1) into GRADS;  BWD3: dZ2 = bf16(conv^T(dY, W3) silu'(Z2));
 *   BWD2: dZ1 = bf16(conv^T(dZ2, W2) silu'(Z1)).
 * Weights are the current parameters rounded to bf16.  NLSE_E_INVAL for an unknown tensor or
 * stage, more bytes than a tensor holds, or batch outside 1..max_batch. */
enum { NLSE_CORR_X0 = 0, NLSE_CORR_A1 = 1, NLSE_CORR_A2 = 2, NLSE_CORR_Z1 = 3, NLSE_CORR_Z2 = 4, NLSE_CORR_Y = 5,
       NLSE_CORR_DY = 6, NLSE_CORR_DZ2 = 7, NLSE_CORR_DZ1 = 8, NLSE_CORR_GRADS = 9 };
enum { NLSE_CORR_FWD1 = 1, NLSE_CORR_FWD2 = 2, NLSE_CORR_FWD3 = 3, NLSE_CORR_WGRAD3 = 4, NLSE_CORR_BWD3 = 5,
       NLSE_CORR_WGRAD2 = 6, NLSE_CORR_BWD2 = 7, NLSE_CORR_WGRAD1 = 8 };
int nlse_corr_tensor(nlse_corr *m, int32_t which, int32_t to_device, void *host, int64_t bytes);
int nlse_corr_stage(nlse_corr *m, int32_t op, int32_t batch);
/* One correction of a 2D context's current field (its grid must be H x W nodes and its
 * stream the corrector's). */
int nlse_corr_apply(nlse_corr *m, nlse_ctx *c);
/* nsteps RK4 steps of size dt with a correction after every `every` steps. */
int nlse_step_corrected(nlse_ctx *c, nlse_corr *m, int64_t nsteps, double dt, int32_t every);
void nlse_corr_destroy(nlse_corr *m);

/* Injection restriction of a dense square complex field (device pointers, stream-ordered):
 * dst[y][x] = src[f y][f x], src of src_n intervals (complex64 if src_prec = NLSE_F32,
 * else complex128), dst complex64 of dst_n = src_n / f intervals. */
int nlse_inject(const void *src, int32_t src_prec, int64_t src_n, void *dst, int64_t dst_n, int32_t factor,
                void *stream);

/* ---------------------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops that forbid hipMalloc): the mass of nlse_mass, h^ndim * sum over every node of
 * |Psi|^2 reduced in FP64 in the same fixed order (bitwise equal to nlse_mass of a context
 * holding the same field), for a caller's field.  Allocates nothing: the reduction's
 * partial sums live in a static device array of the library (1024 doubles per GPU, held
 * until the process ends; its size does not depend on the field, so every field size is
 * accepted).
 *   psi:    device pointer, dense [z][y][x] field of (n[a] + 1) nodes per axis a < ndim,
 *           interleaved complex128 (NLSE_F64, NLSE_F32_MIXED) or complex64 (NLSE_F32).
 *   out:    device pointer to one double, written by the last kernel of the call.
 *   stream: hipStream_t the kernels are enqueued on (NULL = default stream); the call
 *           returns without waiting.
 * The caller keeps ownership of psi and out.  Calls that overlap on one GPU share the
 * static array and race: serialise them (one stream, or wait between calls).  Returns
 * NLSE_E_INVAL for NULL pointers, ndim outside 1..3, n[a] < 1 or h <= 0. */
int nlse_mass_noalloc(int32_t ndim, const int64_t *n, double h, int32_t prec, const void *psi, double *out,
                      void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NLSE_H */
