/* firm.h -- C ABI of the MI355X (gfx950) FIRM library.
 *
 * FIRM (Wang, Shkolnisky & Singer, "A Fourier-based Approach for Iterative 3D
 * Reconstruction from Cryo-EM Images") reconstructs an N^3 volume V from M
 * Fourier slices b by solving the normal equations of the least-squares cost
 * (section 3.3, eq. cost1), here with a Tikhonov term:
 *
 *     (A*A + lambda I) V = A* b.
 *
 * A is the forward projector of eq. (forward-projector), A* the back-projector
 * of eq. (backprojection), and A*A is the convolution with the kernel Ker of
 * eq. (kernel) (eq. property), applied through a 2N-per-axis circulant
 * embedding and FFTs (eq. embedding_circulant, circ1).
 *
 * Conventions
 *   Volume:  float, C order V[i1][i2][i3], voxel n = i - N/2 (section 3.1).
 *   Slices:  complex64 (interleaved re, im), image-major, M x P(N): image m holds
 *            the P(N) disk points k with ||k|| <= N/2 (eq. truncation) in the
 *            canonical order k1 ascending, then k2 ascending.  Index P-1-j holds -k_j.
 *   Rotations: row-major 3x3 R_m; sample point xi = R_m^{-1}(2 pi k1/N, 2 pi k2/N, 0).
 *   CTF:     a table h_g(q), q = k1^2 + k2^2 in [0, N^2/4], per defocus group g; image m
 *            uses group ctf_group[m].  NULL table means h = 1.
 *   Shifts:  s_m in pixels; slices are re-centred by exp(+i <omega_k, s_m>) before
 *            back-projection (section 3.1, images re-shifted to their centres).
 *   Kernel:  Ker(n) for -N < n < N per axis, stored as a (2N)^3 float array in centred
 *            offset order ker[j1][j2][j3] = Ker(j - N); planes with some j_d = 0
 *            (offset -N, outside the kernel's domain) hold 0.
 *   Preconditioner diagonal d: float N^3, indexed by centred frequency q + N/2.
 *
 * Memory: every pointer argument named *_dev is a device pointer owned by the
 * caller; the library never frees it.  Host arrays are copied during the call.
 * The plan owns its workspaces (kernel spectrum, padded FFT buffers, gridding
 * grids) and frees them in firm_plan_destroy.
 *
 * Streams: every call is ordered on the plan's stream (firm_options.stream, or
 * the null stream).  Calls return once the work is enqueued unless stated;
 * firm_cg_solve synchronises for its stopping checks.
 *
 * Errors: functions return a firm_status; nothing aborts or throws across the
 * ABI.  firm_last_error(plan) (or firm_last_error(NULL) for errors raised
 * before a plan exists) returns the message of the latest failure.
 * A plan is not thread-safe.
 */
#ifndef FIRM_H
#define FIRM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct firm_plan_s* firm_plan;

typedef enum {
    FIRM_OK = 0,
    FIRM_ERR_ARG = 1,           /* invalid argument (message says which) */
    FIRM_ERR_ALLOC = 2,         /* device or host allocation failed */
    FIRM_ERR_HIP = 3,           /* a HIP runtime call failed */
    FIRM_ERR_STATE = 4,         /* call out of order, e.g. apply before a kernel exists */
    FIRM_ERR_BREAKDOWN = 5,     /* CG/PCG breakdown (non-positive or non-finite curvature) */
    FIRM_ERR_NOT_CONVERGED = 6  /* CG stopped at max_iter above tol; x is still valid */
} firm_status;

typedef struct {
    int kb_width;         /* Kaiser-Bessel window width in fine-grid cells, 4..8; 0 = 7 */
    int refine_every;     /* precision 0: residual replacement period in iterations; 0 = 50, <0 = never */
    int check_every;      /* CG iterations enqueued between host checks of the stop flag; 0 = 10 */
    int precision;        /* CG arithmetic: 0 = FP32 vectors and product, FP64 sums and scalars;
                             1 = FP64 iterative refinement (FP64 residual, product and solution,
                             FP32 (P)CG corrections); 2 = FP64 CG (no preconditioner) */
    int lambda_relative;  /* 0: lambda as given; 1: the lambda of every call is multiplied by
                             Ker(0) = sum_m sum_k h_m^2, the diagonal of A*A */
    int khat_bf16;        /* 16-bit kernel spectrum for the FP32 product (and FP32 (P)CG), half
                             the spectrum bytes, product error <= 1e-3; the FP64 product keeps
                             the FP32 kernel.  0 = FP32 K^; 1 = BF16 codes of (K^ - o_s) / s_s
                             with a per-shell offset o_s (shell mean) and scale s_s (largest
                             deviation), shell = rounded |q|; 2 = BF16 codes of K^ */
    double inner_tol;     /* precision 1: relative tolerance of each FP32 correction (never tighter
                             than half of what the remaining reduction to tol needs); 0 = the
                             first correction to sqrt(tol) (within [1e-4, 1e-2]), later ones to
                             half of the remaining reduction (at least 1e-4) */
    void* stream;         /* hipStream_t for all work; NULL = null stream */
    int stagnation_iters; /* preconditioned solves: restart as plain CG from the current x when the
                             residual norm has not halved in this many iterations (checked every
                             check_every iterations); 0 = 300, < 0 = never */
} firm_options;

typedef struct {
    int iters;            /* CG iterations performed (all corrections, precision 1) */
    int refinements;      /* precision 0: residual replacements; precision 1: FP64 corrections */
    int fell_back;        /* 1 if a preconditioned solve restarted as plain CG */
    int status;           /* firm_status of the solve */
    double rel_res;       /* residual / ||A*b|| that stopped the solver */
    double true_rel_res;  /* ||A*b - (A*A + lambda) x|| / ||A*b|| with the FP64 product, for the x
                             written out (FP32 x in firm_cg_solve, FP64 x in firm_cg_solve_f64) */
    double t_ms;          /* wall time of the solve in ms */
} firm_cg_report;

/* P(N): number of disk points per slice (eq. truncation). */
int64_t firm_slice_points(int N);

/* Create a plan for N^3 volumes (N a power of two, 8..256) and M images.
 * rotations: host M x 9 doubles (R_m row-major, orthonormal with det +1 to 1e-6).
 * shifts: host M x 2 doubles or NULL.  ctf_group: host M int32 in [0, G) or NULL
 * (group 0).  ctf_table: host G x (N*N/4 + 1) floats or NULL (h = 1).
 * opt may be NULL for defaults.  Errors: FIRM_ERR_ARG for bad sizes, rotations,
 * groups or options; FIRM_ERR_ALLOC / FIRM_ERR_HIP on device failure (*out = NULL). */
firm_status firm_plan_create(firm_plan* out, int N, int M, const double* rotations,
                             const double* shifts, const int32_t* ctf_group, int G,
                             const float* ctf_table, const firm_options* opt);

void firm_plan_destroy(firm_plan plan);

/* Set the stream used by later calls (hipStream_t, NULL = null stream). */
firm_status firm_plan_set_stream(firm_plan plan, void* stream);

/* Step 3 of the algorithm (section 3.4): compute Ker (eq. kernel) by gridding the
 * CTF^2-weighted sample points with a Kaiser-Bessel window onto a (4N)^3 grid,
 * FFT, deconvolution and crop, then the spectrum of its 2N circulant embedding
 * (eq. embedding_circulant).  Uses Ker(-n) = Ker(n) to spread half the disk. */
firm_status firm_kernel_precompute(firm_plan plan);

/* Copy Ker into ker_dev ((2N)^3 floats, centred offset order, see above). */
firm_status firm_kernel_get(firm_plan plan, float* ker_dev);

/* Replace the plan's kernel by ker_dev ((2N)^3 floats, centred offset order; the
 * j_d = 0 planes are ignored) and recompute its circulant spectrum.  Lets a caller
 * reuse a stored kernel or apply any Toeplitz kernel. */
firm_status firm_kernel_set(firm_plan plan, const float* ker_dev);

/* Fourier-space regularizer (section 5: damping of high frequencies).  Adds mu L_p to the operator
 * of every later product and solve, (A*A + lambda I + mu L_p) x = A*b, with
 *   L_p = crop F_2N^{-1} diag(w^p) F_2N pad,   w(q) = sum_d 4 sin^2(pi q_d / 2N),
 * the same zero-padded 2N embedding as the product (pad, crop: the N^3 volume inside (2N)^3 zeros).
 * w is the symbol of the 7-point negative Laplacian, so L_1 x is that stencil with zero values
 * outside the volume; L_p is positive semidefinite for every p.  It enters the product's spectrum
 * (no extra memory traffic), the FP64 product and T. Chan's spectrum (firm_chan_spectrum).  order:
 * 0 (none, the default) .. 3; mu >= 0 in the units of lambda (times Ker(0) with lambda_relative).
 * Takes effect at once if a kernel exists (the spectrum is rebuilt from the kernel), else when one
 * is computed or set.  firm_kernel_get still returns Ker. */
firm_status firm_set_regularizer(firm_plan plan, int order, double mu);

/* Step 2 (section 3.4): atb_dev (N^3 floats) = Re A*(re-centred b) (eq. backprojection)
 * for slices b_dev (device, M x P complex64, finite values).  Exact real part for any b: the
 * spread uses the pair (k, -k) as b(k) + conj(b(-k)).  The gridding accumulates exact
 * fixed-point sums whose unit follows the largest |component| of b (found on the device first),
 * so the result's accuracy is that of FP32 terms for any overall scale of b. */
firm_status firm_backproject(firm_plan plan, const void* b_dev, float* atb_dev);

/* The forward projector (eq. forward-projector) with the imaging model of section 3.1:
 * b_dev (device, M x P complex64, disk order) receives
 *   b(k, m) = h_m(|k|) exp(-i <omega_k, s_m>) sum_n V(n) exp(-i <n, xi_{k,m}>)
 * for V_dev (device, N^3 floats, centred order: voxel i is n = i - N/2), i.e. the slices
 * that images of V at the plan's rotations, shifts and CTFs would have.  It is the adjoint of
 * firm_backproject: for real V and any b, <V, firm_backproject(b)> = Re <forward(V), b>.
 * Evaluated as a type-2 non-uniform FFT with the plan's Kaiser-Bessel window on the (2N)^3
 * grid (relative error ~1e-6 at width 7).  Every element of b_dev is written; the result
 * satisfies b(-k) = conj b(k).  Uses the gridding workspaces (allocated on first use). */
firm_status firm_forward_project(firm_plan plan, const float* V_dev, void* b_dev);

/* y_dev = (A*A + lambda I) x_dev through the circulant embedding (eq. property,
 * embedding_circulant, circ1): pad to (2N)^3, FFT, multiply by the kernel
 * spectrum, inverse FFT, crop.  x_dev, y_dev: N^3 floats, must not alias.
 * FIRM_ERR_STATE if no kernel exists; FIRM_ERR_ARG if lambda < 0. */
firm_status firm_apply_AtA(firm_plan plan, const float* x_dev, float* y_dev, double lambda);

/* Instrumented firm_apply_AtA: runs it reps times on the plan stream, each of its five FFT
 * passes (rows along i3 with padding; columns along i2; the fused multiply pass along i1;
 * inverse along i2; inverse along i3 with crop and lambda x) launched with a pair of HIP
 * events in its own dispatch (hipExtLaunchKernelGGL), and writes the passes' average kernel
 * durations in ms to pass_ms[5] (host).  Synchronises after every product. */
firm_status firm_apply_AtA_timed(firm_plan plan, const float* x_dev, float* y_dev, double lambda, int reps,
                                 float* pass_ms);

/* FP64 form of firm_apply_AtA: x_dev, y_dev are N^3 doubles; the spectrum is computed in
 * FP64 from the FP32 kernel values (so it is exactly the Toeplitz product with them). */
firm_status firm_apply_AtA_f64(firm_plan plan, const double* x_dev, double* y_dev, double lambda);

/* Step 4 (section 3.3-3.4): CG on (A*A + lambda I) x = atb from the initial guess in
 * x_dev (pass zeros for the paper's x0 = 0), in the arithmetic of firm_options.precision.
 * atb_dev, x_dev: N^3 floats (device); x is FP32 on return in every mode, so with
 * precision 1 or 2 its residual can exceed the FP64 iterate's by the rounding of x
 * (about 6e-8 times the condition number): rep->true_rel_res is that of the FP32 x.
 * Precision 0 stops when the residual measured with the FP32 product is <= tol ||atb||
 * (a recursive residual below tol is confirmed by a recomputed one); precision 1 and 2
 * stop on the FP64 residual.  max_iter bounds the CG iterations.  precond_d_dev: NULL for plain CG, else a Fourier diagonal d
 * (N^3, centred frequency order, d > 0, d(q) = d(-q)) applied as
 * z = F^{-1}(d . F r) on the periodic N^3 grid; a breakdown of the preconditioned
 * recursion restarts plain CG from the current x.  rep may be NULL.
 * Returns FIRM_ERR_NOT_CONVERGED (x valid) if max_iter was reached above tol. */
firm_status firm_cg_solve(firm_plan plan, const float* atb_dev, float* x_dev, double lambda,
                          double tol, int max_iter, const float* precond_d_dev,
                          firm_cg_report* rep);

/* firm_cg_solve with an FP64 right-hand side and solution (atb_dev, x_dev: N^3 doubles,
 * device; x_dev holds the initial guess).  Needs precision 1 or 2 (FIRM_ERR_STATE for 0);
 * the FP64 iterate is x itself, so residuals below the FP32 rounding of x are reachable.
 * Precision 2 takes no preconditioner (FIRM_ERR_ARG), here and in firm_cg_solve. */
firm_status firm_cg_solve_f64(firm_plan plan, const double* atb_dev, double* x_dev, double lambda,
                              double tol, int max_iter, const float* precond_d_dev,
                              firm_cg_report* rep);

/* z_dev = F^{-1}(d . F r) on the periodic N^3 grid (circulant diagonalisation,
 * eq. circ1); d_dev, r_dev, z_dev: N^3 floats (d in centred frequency order). */
firm_status firm_precond_apply(firm_plan plan, const float* d_dev, const float* r_dev, float* z_dev);

/* Copy the kernel spectrum K^(q) = DFT_{2N}(c)(q) / (2N)^3 of the circulant first
 * column c for q3 in [0, N] into khat_dev ((2N) x (2N) x (N+1) floats, q in FFT
 * order).  It is real because Ker is real and even. */
firm_status firm_kernel_spectrum(firm_plan plan, float* khat_dev);

/* Step 1 of the algorithm (section 3.4): slices from images.  images_dev: device, M x N x N
 * floats (image m, row i1, column i2; pixel i sits at x = i - N/2).  b_dev (device, M x P
 * complex64, disk order) receives the centred 2D DFT of section 2.2 at the disk points,
 *   b(k, m) = sum_x J_m(x) exp(-2 pi i <k, x> / N),
 * with the periodic value at the boundary points k_d = +N/2.  The images are taken as
 * recorded (no CTF or shift correction; firm_backproject re-centres).  Batched real FFTs in
 * groups of images through a workspace of at most 1 GiB (allocated on first use). */
firm_status firm_images_to_slices(firm_plan plan, const float* images_dev, void* b_dev);

/* Synthetic real-space images: images_dev (M x N x N floats, layout of firm_images_to_slices)
 * = projections of a sum of B Gaussian blobs along the plan's views (section 3.1: each blob
 * a exp(-||x - c||^2 / (2 s^2)) projects to a sqrt(2 pi) s exp(-||x - p||^2 / (2 s^2)) with p
 * the first two coordinates of R_m c), translated by the plan's shifts (image J(x - s_m)),
 * plus white Gaussian pixel noise at the given SNR (mean clean pixel power / noise variance;
 * snr <= 0 or infinite: none).  No CTF.  sigma > 0 required; B in [1, 320].  Noise uses
 * Philox4x32-10 keyed by seed. */
firm_status firm_synth_images(firm_plan plan, int B, const double* centers, const double* sigmas,
                              const double* amps, double snr, uint64_t seed, float* images_dev);

/* Synthetic slices for benchmarks and tests: b_dev (M x P complex64) = CTF-filtered,
 * translated Fourier slices of a sum of B Gaussian blobs given in closed form by the
 * projection-slice theorem (eq. continuous_fps), plus complex white noise with the
 * symmetry of a real image's DFT at the given SNR (mean clean power / noise power;
 * snr <= 0 or infinite: no noise).  centers (B x 3), sigmas, amps: host doubles in
 * voxel units; sigma 0 is a point source.  Noise uses Philox4x32-10 keyed by seed. */
firm_status firm_synth_slices(firm_plan plan, int B, const double* centers, const double* sigmas,
                              const double* amps, double snr, uint64_t seed, void* b_dev);

/* Sampled blob volume for accuracy measurements: V_dev (N^3 floats, centred order) =
 * sum_b a_b exp(-||n - c_b||^2 / (2 s_b^2)) at the voxels n = i - N/2 (section 3.1's sampling of
 * the potential), the volume whose slices firm_synth_slices gives in closed form.  centers (B x 3),
 * sigmas (> 0), amps: host doubles in voxel units; B in [1, 320]. */
firm_status firm_synth_volume(firm_plan plan, int B, const double* centers, const double* sigmas,
                              const double* amps, float* V_dev);

/* Fourier shell correlation of section 4 between V1_dev and V2_dev (N^3 floats, device): for the
 * shells i = 1 .. N/2 - 1, Shell_i = {j : 0.5 + (i-1) + 1e-4 <= ||j|| < 0.5 + i + 1e-4},
 *   FSC(i) = sum_{Shell_i} F(V1) conj F(V2) / sqrt(sum |F(V1)|^2 sum |F(V2)|^2)
 * (against the true volume, the Fourier cross-resolution), and the modified forms restricted to
 * the frequencies outside / inside the cone of half-angle cone_deg about the third axis (the
 * missing cone of a random conical tilt series at tilt 90 - cone_deg degrees).  fsc_host (host,
 * 3 x (N/2 - 1) doubles): rows all, outside, inside; NaN where a shell region is empty. */
firm_status firm_fsc(firm_plan plan, const float* V1_dev, const float* V2_dev, double cone_deg, double* fsc_host);

/* ---- learned Fourier-diagonal preconditioner ----------------------------------------
 * A 3D conv net maps f = log(|K^| pooled to res^3 / Ker(0) + lam_rel) to a log floor on the
 * res^3 frequency grid: o = c4(relu(c3(relu(c2(relu(c1(f))))))) with 3^3 filters, circular
 * padding, 1 -> 32 -> 32 -> 32 -> 1 channels (c2, c3 on BF16 matrix cores, FP32 accumulation).
 * res is a power of two in [32, 256]; the network is fully convolutional, so weights trained
 * at one res apply at another.
 * The diagonal of z = F^{-1}(d . F r) is d = 1 / (t + Ker(0) exp(U sym(o))) on the N^3 grid, with
 * t the Fourier diagonal of A*A + lambda (firm_chan_spectrum, T. Chan's circulant spectrum), sym
 * o(u) + o(-u) halved and U periodic trilinear interpolation: the network sets a floor under the
 * analytic spectrum (a floor of 0 is Chan's 1 / t; a network whose last layer has zero weights
 * gives the constant floor exp(b4)).  |K^| is the unnormalised DFT_2N of the circulant column (the
 * Fourier multiplier of the embedded product).  Objectives (firm_pcnet_loss_grad):
 *   0  probe loss E ||P (A*A + lambda) z - z||^2 / E ||z||^2, a per-frequency quadratic in d by
 *      Parseval (statistics from firm_probe_stats);
 *   1  Kaporin: log(mean(d t)) - mean(log(d t)), the log of Kaporin's condition number of
 *      P (A*A + lambda) per unknown up to a constant; zero iff d is proportional to 1 / t;
 *   2  a loss whose gradient with respect to log d the caller supplies, e.g. the unrolled PCG
 *      error of firm_pcg_unrolled (the default training objective: section 3.3's CG minimises
 *      the energy-norm error over its Krylov space, and this loss measures what k steps leave). */
typedef struct firm_pcnet_s* firm_pcnet;

/* Number of network parameters; host parameter arrays hold w1 [32][1][27], b1 [32],
 * w2 [32][32][27], b2, w3, b3, w4 [1][32][27], b4 [1] in that order (tap = 9a + 3b + c for the
 * offset (a-1, b-1, c-1)). */
int64_t firm_pcnet_num_params(void);
firm_status firm_pcnet_create(firm_pcnet* out, int max_batch, void* stream);
void firm_pcnet_destroy(firm_pcnet net);
firm_status firm_pcnet_set_params(firm_pcnet net, const float* params_host);  /* resets Adam */
firm_status firm_pcnet_get_params(firm_pcnet net, float* params_host);
/* out_dev [B][res^3] = network output o for features feat_dev [B][res^3] (centred order).
 * Activation buffers grow on first use of a larger B x res^3 (24 bytes per voxel x 32 channels x
 * ... : about 1.6 GB at res 128, B 1). */
firm_status firm_pcnet_forward(firm_pcnet net, const float* feat_dev, int res, float* out_dev, int B);
/* Mean loss of B samples at size N (N <= 8 res) under `objective`, features [B][res^3], and (if
 * grad_host) the parameter gradients (host, NPARAM floats).  t_dev [B][N^3]: the Fourier
 * diagonals t of each sample (firm_chan_spectrum, t > 0).  objective 0: A_dev, B_dev [B][N^3]
 * probe statistics (centred order) from firm_probe_stats and sumc host [B]; objective 1: A_dev,
 * B_dev and sumc unused (may be NULL); objective 2: A_dev [B][N^3] the gradient of the caller's
 * loss with respect to log d, *loss set to 0 (loss may be NULL).  ker0: host [B], Ker(0) of each
 * sample's kernel.  FIRM_ERR_ARG for another objective. */
firm_status firm_pcnet_loss_grad(firm_pcnet net, const float* feat_dev, int res, int B, int N, int objective,
                                 const float* t_dev, const float* A_dev, const float* B_dev, const double* sumc,
                                 const double* ker0, double* loss, float* grad_host);
/* One Adam step (Kingma & Ba 2015) on the mean loss of firm_pcnet_loss_grad (same arguments): step
 * size lr for every parameter except the output bias b4 (the log of the floor's level), which
 * steps at lr_floor (the floor is exp of the output, so the weights move it through products of
 * many activations while b4 moves it directly). */
firm_status firm_pcnet_train_step(firm_pcnet net, const float* feat_dev, int res, int B, int N, int objective,
                                  const float* t_dev, const float* A_dev, const float* B_dev, const double* sumc,
                                  const double* ker0, double lr, double lr_floor, double* loss);
const char* firm_pcnet_last_error(firm_pcnet net);

/* Unrolled PCG objective for the preconditioner d_dev (N^3, centred frequency order, d > 0,
 * d(q) = d(-q)): for each probe z (probes_dev [nprobes][N^3]), b = (A*A + lambda) z and x_k the
 * k-th iterate of PCG from x0 = 0 (section 3.3, preconditioned by z = F^{-1}(d . F r));
 * *loss (host) = mean over the probes of ||z - x_k||_T^2 / ||z||_T^2 in the energy norm of
 * T = A*A + lambda (lambda read as by firm_apply_AtA).  grad_dev (N^3, centred; NULL: loss only) =
 * d loss / d log d, from the recursion's adjoint with its step lengths and ratios held fixed: x_k
 * minimises the error over its Krylov space, so that is the derivative of the minimum (the
 * envelope theorem).  FP32 vectors, FP64 scalars.  k in [1, 1000]; uses (k + 7) N^3 floats of
 * plan workspace (allocated on first use).  FIRM_ERR_BREAKDOWN if the loss is not finite. */
firm_status firm_pcg_unrolled(firm_plan plan, const float* d_dev, const float* probes_dev, int nprobes, int k,
                              double lambda, double* loss, float* grad_dev);

/* Features of the plan's kernel: feat_dev [res^3] = log(mean |K^| over (2N/res)^3 blocks /
 * Ker(0) + lam_rel), centred frequency order, with K^ the unnormalised DFT_2N of the circulant
 * column ((2N)^3 times the spectrum of firm_kernel_spectrum).  res: power of two in [32, 2N]
 * (and <= 256). */
firm_status firm_kernel_features(firm_plan plan, double lam_rel, int res, float* feat_dev);
/* d_dev [N^3] (centred) = 1 / (t + Ker(0) exp(U sym(out))) from a network output out_dev [res^3]
 * (N <= 8 res) and the Fourier diagonal t_dev [N^3] of A*A + lambda (firm_chan_spectrum).
 * Allocates res^3 floats of scratch for the call and synchronises the plan stream. */
firm_status firm_precond_from_output(firm_plan plan, const float* out_dev, int res, const float* t_dev,
                                     float* d_dev);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): firm_precond_from_output with its res^3 scratch (the
 * symmetrised network output) in a static device array of 128^3 floats (8 MiB on every GPU the
 * library runs on, held until the process ends) instead of a per-call allocation.  res <= 128
 * (FIRM_ERR_ARG beyond, checked before any device work); other arguments as firm_precond_from_output.
 * Enqueued on the plan stream; returns without synchronising.  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other threads) race, calls in order
 * on one stream do not.  Nothing needs clearing: each call writes the entries it reads. */
firm_status firm_precond_from_output_noalloc(firm_plan plan, const float* out_dev, int res, const float* t_dev,
                                             float* d_dev);
/* Probe statistics on the centred N^3 grid for nprobes real probes z (probes_dev [nprobes][N^3]):
 * A = sum |F u|^2, B = sum Re(conj(F u) F z) with u = (A*A + lambda) z (FP32 product), and
 * *sumc = sum ||F z||^2 (host). */
firm_status firm_probe_stats(firm_plan plan, const float* probes_dev, int nprobes, double lambda, float* A_dev,
                             float* B_dev, double* sumc);
/* t_dev [N^3] (centred frequency order) = the Fourier diagonal of A*A + lambda I on the periodic
 * N^3 grid: diag(F T F^H) / N^3 for the Toeplitz operator T of the plan's kernel, which is the
 * spectrum of T. Chan's optimal circulant (first column: the Fejer-weighted fold
 * c(j) = sum over o_d in {j_d, j_d - N} of prod_d (1 - |o_d| / N) Ker(o)), plus lambda.
 * 1 / t is the analytic Fourier-diagonal preconditioner; t is the target of the Kaporin
 * objective.  FP32, through one N^3 FFT. */
firm_status firm_chan_spectrum(firm_plan plan, double lambda, float* t_dev);
/* out_dev[i] = standard normal from Philox4x32-10 keyed by seed, counter (i, offset). */
firm_status firm_synth_normals(firm_plan plan, uint64_t seed, uint64_t offset, int64_t n, float* out_dev);

/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw, SC 2011), the source of
 * the synthetic noise: out = bijection(ctr) keyed by key.  Host function, no device work. */
void firm_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Message of the latest failure on plan (NULL: of the latest failure without a plan). */
const char* firm_last_error(firm_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* FIRM_H */
