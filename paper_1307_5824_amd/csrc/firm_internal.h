// Internal declarations shared by the HIP translation units of libfirm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/firm.h"

#define FIRM_TWN 1024  // twiddle table length: exp(-2 pi i m / 1024), m in [0, 1024)

struct firm_plan_s {
    int N = 0, M = 0, G = 0, P = 0, Q = 0;  // Q = N*N/4 + 1 (CTF table width)
    int QP = 0;                              // pitch of the half-spectrum axis (>= N+1)
    int kbw = 7;
    double beta = 0.0;
    int refine_every = 50, check_every = 10;
    int stagnation_iters = 300;  // preconditioned solves: plain-CG restart after this many iterations
                                 // without a halving of the residual norm (<= 0: never)
    int precision = 0;          // 0 FP32 CG, 1 FP64 iterative refinement, 2 FP64 CG
    int lambda_relative = 0;    // lambda multiplies Ker(0)
    double inner_tol = 0.0;     // relative tolerance of each FP32 correction (precision 1; 0 = per solve)
    double ker0 = 0.0;          // Ker(0) of the current kernel
    int reg_order = 0;          // Fourier-space damping: order p of mu L_p (0 = none)
    double reg_mu = 0.0;        // its weight as given (times Ker(0) with lambda_relative)
    double reg_mu_eff = 0.0;    // the weight in the operator's units, set when the spectrum is built
    hipStream_t stream = nullptr;
    std::string err;

    // geometry (device)
    double* c12 = nullptr;     // M x 6: columns 1 and 2 of R_m^{-1}
    float* nrm = nullptr;      // M x 4: plane normal (c1 x c2), float
    int32_t* group = nullptr;  // M
    float* table = nullptr;    // G x Q (h), or null
    double* shifts = nullptr;  // M x 2 or null
    // the same per-view arrays in the gridding's view order (normals folded to one hemisphere and
    // sorted along a space-filling curve of their direction), its map to the caller's order, and
    // per block of SP_VBLK views the box of the normals and the largest |n|_1
    double* c12s = nullptr;
    float* nrms = nullptr;
    int32_t* groups = nullptr;
    double* shiftss = nullptr;
    int32_t* vorder = nullptr;  // gridding position -> view index
    float4* vbox = nullptr;     // 2 per block: (min n, max |n|_1), (max n, 0)
    double ker_k0 = 0.0;       // sum_m h_m(0)^2: the k = 0 term of Ker

    // Kaiser-Bessel window (device)
    float* kb_poly = nullptr;  // w x (KB_DEG+1) polynomial coefficients on f in [0, 1]
    float fx_ker = 1.f;        // kernel gridding: integer units per unit (power of 2, terms < 2^31)
    float fx_atb_coef = 0.f;   // A*b gridding: units per unit times the largest |b component| may reach
    unsigned* fx_bmax = nullptr;  // device word: bits of the largest |b component| (inside dscal)
    float* deconv_ker = nullptr;  // 2N: 1/phihat at circulant position p (L = 4N)
    float* deconv_atb = nullptr;  // N: 1/phihat at centred index i (L = 2N)

    float2* tw = nullptr;      // FIRM_TWN twiddles

    // kernel and its spectrum (device)
    bool have_kernel = false;
    float* kerc = nullptr;     // (2N)^3 Ker in circulant order c[p1][p2][p3]
    float* khat = nullptr;     // real spectrum, q3 in [0, N], blocked as [q2][q3 group][q1][C]
    int khat_bf16 = 0;         // option: the FP32 product reads the 16-bit copy below
    uint16_t* khat16 = nullptr;  // BF16 codes of (K^ - offset) / scale per shell, blocked like khat
    float2* shtab = nullptr;     // per-shell (offset, scale), KSH_MAX entries

    // apply workspaces
    float2* T1 = nullptr;      // [N][N][QP]
    float2* T2 = nullptr;      // [N][2N][QP]

    // FP64 product (allocated on first use): spectrum, workspaces, twiddles, vectors
    bool khat64_valid = false;
    double* khat64 = nullptr;  // blocked like khat (double-precision pencil width)
    double2* T1d = nullptr;
    double2* T2d = nullptr;
    double2* tw64 = nullptr;
    double *x64 = nullptr, *r64 = nullptr, *p64 = nullptr, *q64 = nullptr, *y64 = nullptr, *atb64 = nullptr;
    float *rhs = nullptr, *dvec = nullptr;  // FP32 correction right-hand side and solution

    // CG workspaces
    float *r = nullptr, *p = nullptr, *z = nullptr, *tmp = nullptr;
    double* partials = nullptr;  // per-block FP64 partial sums
    int npart = 0;
    double* scal = nullptr;      // device scalars (see cg.hip)
    double* host_scal = nullptr; // pinned host mirror
    float* dhalf = nullptr;      // preconditioner diagonal / N^3, FFT order, blocked [q2][q3 group][q1][C]
    float2* S1 = nullptr;        // PCG FFT workspace [N][N][QPn]
    float2* S2 = nullptr;        // second half-spectrum workspace (probe statistics), on first use
    size_t s2_bytes = 0;
    int QPn = 0;

    // gridding workspaces (allocated on first use, kept)
    void* grid = nullptr; size_t grid_bytes = 0;
    void* ws1 = nullptr; size_t ws1_bytes = 0;
    void* ws2 = nullptr; size_t ws2_bytes = 0;
    int* tiles_ker = nullptr; int ntiles_ker = 0;   // work list for the kernel spread
    int* tiles_atb = nullptr; int ntiles_atb = 0;   // work list for the A*b spread
    double* dscal = nullptr;   // small device scratch for the A*b k=0 term
    int* rowstart = nullptr;   // N+1: disk index of (k1, 0), so idx(k1, k2) = rowstart[k1 + N/2] + k2
    int* flags = nullptr;      // CG control words on device (see cg.hip)
    int* host_flags = nullptr; // pinned mirror
    double* partials2 = nullptr;
    double* partials3 = nullptr;
    void* img_ws = nullptr; size_t img_ws_bytes = 0;  // image spectra workspace (Step 1), on first use
    float* uws = nullptr; size_t uws_bytes = 0;        // unrolled-PCG vectors, on first use
    double* usc = nullptr; size_t usc_bytes = 0;       // unrolled-PCG scalars, on first use
};

// status helpers (api.cpp)
firm_status firm_fail(firm_plan p, firm_status s, const std::string& msg);
#define FIRM_HIP(p, call)                                                                 \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return firm_fail((p), FIRM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---- fft.hip launchers (return hipError_t of the launch) ----
hipError_t fft_apply_AtA(firm_plan p, const float* x, float* y, float lam);
int fft_cols_per_block(int L, bool dbl);  // pencils per workgroup of the L-point pass
int64_t fft_t2_elems(int N, bool dbl);    // complex elements of the blocked T2 [2N][groups][N][C]
size_t blocked_spectrum_elems(int L, int nouter, int ncols, bool dbl);
hipError_t fft_khat_unblock(firm_plan p, float* out);
hipError_t fft_forward_r2c(firm_plan p, const float* x, float2* out);  // N^3 real -> [N][N][QPn] half spectrum
hipError_t chan_spectrum(firm_plan p, double lam, float* out);  // fft.hip: Chan spectrum + lam, centred N^3
hipError_t kernel_features(firm_plan p, float lam_rel, int res, float* feat);
hipError_t probe_accumulate(firm_plan p, const float2* zh, const float2* uh, float* A, float* B, double* partials,
                            int nblocks);
hipError_t synth_normals(firm_plan p, uint64_t seed, uint64_t offset, int64_t n, float* out);
// ev: 10 events, a start/end pair per pass carried by that pass's own dispatch
hipError_t fft_apply_AtA_events(firm_plan p, const float* x, float* y, float lam, hipEvent_t* ev);
hipError_t fft_khat_from_kerc(firm_plan p, float2* w1);        // kerc -> khat (w1: [2N][2N][QP])
hipError_t fft_ker_grid(firm_plan p, const float* grid, float2* h1, float2* h2, float* chalf);
hipError_t fft_atb_grid(firm_plan p, const float2* grid, float2* j1, float2* j2, float* atb,
                        const double* k0term);
hipError_t fft_project_grid(firm_plan p, const float* u, float2* t1, float2* w, float2* X);  // L x L x QP
hipError_t fft_images_r2c(firm_plan p, const float* img, int G, float2* out);  // G x N x QPn half spectra
// z = IFFT_N(dhalf . FFT_N(r)); partials: also fft_precond_partials(p) block partials of <r, z>.
// z == nullptr (N > 64 only): z is left as its half spectra along i3 in S1, for
// fft_apply_cg_front_pz
hipError_t fft_precond(firm_plan p, const float* dhalf, const float* r, float* z, const int* active = nullptr,
                       double* partials = nullptr);
int fft_precond_partials(firm_plan p);
hipError_t fft_apply_AtA64(firm_plan p, const double* x, double* y, double lam);
hipError_t fft_khat64_from_kerc64(firm_plan p, const double* kerc64, double2* w1);
// fused CG variants of the apply passes (cg.hip drives them)
// CG product in two parts: the front forms p = src + beta p (beta on the device), transforms it
// and multiplies by K^ + lam / (2N)^3, writing fft_apply_cg_partials(p) block partials of
// <p, (A*A + lam) p> to dotp; the step finishes the product q and, with alpha on the device,
// takes x += alpha p, r -= alpha q, writing fft_apply_cg_step_partials(p) partials of ||r||^2.
// Both do nothing while *active == 0.
hipError_t fft_apply_cg_front(firm_plan p, const float* src, float* pvec, float lam, const double* beta_dev,
                              const int* active, double* dotp);
hipError_t fft_apply_cg_step(firm_plan p, float* x, const float* pvec, float* r, const double* alpha_dev,
                             const int* active, double* partials);
// the front with z taken from the preconditioner's half spectra in S1 (N = 128, 256; see
// fft_precond with z == nullptr): p = z + beta p, z itself is never stored
hipError_t fft_apply_cg_front_pz(firm_plan p, float* pvec, float lam, const double* beta_dev, const int* active,
                                 double* dotp);
int fft_apply_cg_step_partials(firm_plan p);
int fft_apply_cg_partials(firm_plan p);

// ---- spread.hip ----
hipError_t spread_ker(firm_plan p, float* grid);
hipError_t spread_atb(firm_plan p, const float2* b, float2* grid);
hipError_t atb_k0_term(firm_plan p, const float2* b, double* out);
hipError_t kerc_from_half(firm_plan p, const float* chalf);
hipError_t kerc_to_centred(firm_plan p, float* out);
hipError_t kerc_from_centred(firm_plan p, const float* in);
hipError_t fill_zero(void* ptr, size_t bytes, hipStream_t s);
hipError_t kerc_to_double(firm_plan p, double* out);
firm_status ensure_fp64(firm_plan p);  // api.hip: FP64 buffers and khat64

// ---- project.hip ----
hipError_t forward_project(firm_plan p, const float* V, float2* b);

// ---- images.hip ----
hipError_t images_gather(firm_plan p, const float2* spec, int G, int m0, float2* b);
hipError_t synth_images(firm_plan p, int B, const double* blobs_dev, double snr, uint64_t seed, float* img,
                        double* partials, int64_t npart);
int64_t synth_images_scratch(int N, int M);  // doubles of device scratch synth_images needs

// ---- synth.hip ----
hipError_t synth_slices(firm_plan p, int B, const double* blobs_dev, double snr, uint64_t seed,
                        float2* b, double* power_dev);
hipError_t synth_volume(firm_plan p, int B, const double* blobs_dev, float* V);  // blobs B x (c, s, a)

// ---- pcnet.hip ----
hipError_t noalloc_scratch_setup();  // device address of the no-allocation scratch, current device

// ---- eval.hip ----
// per (region all / outside / inside the cone, quantity Re(F1 conj F2) / |F1|^2 / |F2|^2, shell)
// sums, 9 x fsc_max_shells() doubles at sums_dev (shell index i at offset i; i = 0 unused)
hipError_t fsc_sums(firm_plan p, const float* V1, const float* V2, double cone_deg, double* sums_dev);
int fsc_max_shells();

// ---- unroll.hip ----
int64_t unrolled_workspace_floats(int N, int k);
int unrolled_scalar_count(int k);
hipError_t pcg_unrolled(firm_plan p, const float* d, const float* probes, int nprobes, int k, float lam, float* ws,
                        double* sc, double* loss_host, float* grad);

// ---- cg.hip ----
firm_status cg_solve(firm_plan p, const float* atb, float* x, double lam, double tol, int max_iter,
                     const float* d, firm_cg_report* rep);
firm_status cg_solve64(firm_plan p, const double* atb, double* x, double lam, double tol, int max_iter,
                       const float* d, firm_cg_report* rep);
hipError_t precond_set(firm_plan p, const float* d_centred);

std::vector<int> spread_worklist(int L, int T, int M, double s);
int spread_tile_real();
int spread_tile_cplx();
constexpr int SP_VBLK = 512;  // views per block of the gridding's view order (its workgroup size)
void kb_tables(firm_plan p, std::vector<float>& poly, std::vector<float>& dker, std::vector<float>& datb);

// block count helper
static inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
