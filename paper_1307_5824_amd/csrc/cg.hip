// Conjugate gradients for (A*A + lambda I) x = A*b (section 3.3, step 4 of the
// algorithm in section 3.4), with an optional Fourier-diagonal preconditioner
// (circulant diagonalisation, eq. circ1).
//
// Precision modes:
//  0  FP32 CG: vectors and the FFT product in FP32; every inner product is
//     accumulated in FP64 (per-block partials, then a one-block reduction) and
//     the scalars alpha, beta and the residual norms live in FP64 on the device,
//     so an iteration needs no host round trip.  The direction update
//     p = z + beta p is fused into the first FFT pass of the product, <p, q> into
//     its middle pass (Parseval over the spectrum) and the step x += alpha p,
//     r -= alpha q with ||r||^2 into its last pass; for N > 64 the
//     preconditioner's last pass is fused into the product's first as well.
//     Every refine_every iterations the recursive residual is replaced by the
//     residual recomputed from the FP32 product.  The host reads a small flag
//     block every check_every iterations; kernels enqueued after convergence
//     see the flag and exit.
//  1  FP64 iterative refinement: the residual, the product that forms it and the
//     solution are FP64; each correction is an FP32 (P)CG solve of the residual
//     equation to a relative tolerance.  Reaches residuals below the FP32
//     product's accuracy at nearly FP32 cost.
//  2  FP64 CG: vectors, product and sums in FP64 (the kernel values themselves
//     are the FP32 ones).
// Every mode reports the true residual measured with the FP64 product.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "fft_core.h"
#include "firm_internal.h"

namespace {

enum { S_RZ = 0, S_PQ, S_ALPHA, S_BETA, S_RR, S_BB, S_TOL2, S_TRUE };
enum { F_ACTIVE = 0, F_ITER, F_REASON, F_MAXIT };
enum { R_RUN = 0, R_CONV = 1, R_MAXIT = 2, R_BREAK = 3 };

constexpr int VB = 1024;  // blocks of the vector kernels
constexpr int VT = 256;
constexpr int RT = 1024;  // threads of the one-block sums that form alpha and beta

// block sum of a double over NT threads; result valid in thread 0
template <int NT = VT>
__device__ __forceinline__ double block_reduce(double v) {
    __shared__ double red[NT / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}

// sum of n block partials by one block of NT threads; the unrolled loop has a thread's loads
// in flight together (the partials were just written by the blocks of another kernel, so each
// load waits on the memory behind L2)
template <int NT = VT>
__device__ __forceinline__ double sum_partials(const double* part, int n) {
    double a = 0.0;
#pragma unroll 8
    for (int i = threadIdx.x; i < n; i += NT) a += part[i];
    return block_reduce<NT>(a);
}

// r = atb - y in FP64, stored FP32; partial sums of r^2.
__global__ void __launch_bounds__(VT) k_resid(const float* __restrict__ atb, const float* __restrict__ y,
                                              float* __restrict__ r, int64_t n, double* partials,
                                              const int* flags) {
    if (flags && flags[F_ACTIVE] == 0) return;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
        const double v = (double)atb[i] - (double)y[i];
        const float f = (float)v;
        r[i] = f;
        acc += (double)f * (double)f;
    }
    const double s = block_reduce(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(VT) k_dot(const float* __restrict__ a, const float* __restrict__ b, int64_t n,
                                            double* partials) {
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
        acc += (double)a[i] * (double)b[i];
    const double s = block_reduce(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// scal[idx] = sum of partials; when copy_to >= 0 also scal[copy_to].
__global__ void __launch_bounds__(VT) k_reduce_to(const double* part, int n, double* scal, int idx, int copy_to,
                                                  const int* flags) {
    if (flags && flags[F_ACTIVE] == 0) return;
    const double s = sum_partials(part, n);
    if (threadIdx.x == 0) {
        scal[idx] = s;
        if (copy_to >= 0) scal[copy_to] = s;
    }
}

__global__ void k_init(double* scal, int* flags, double tol, int max_iter) {
    scal[S_TOL2] = tol * tol * scal[S_BB];
    scal[S_BETA] = 0.0;
    flags[F_ITER] = 0;
    flags[F_MAXIT] = max_iter;
    const bool done = !(scal[S_RR] > scal[S_TOL2]) || max_iter <= 0;
    flags[F_ACTIVE] = done ? 0 : 1;
    flags[F_REASON] = done ? (max_iter <= 0 && scal[S_RR] > scal[S_TOL2] ? R_MAXIT : R_CONV) : R_RUN;
}

__global__ void __launch_bounds__(RT) k_alpha(const double* part, int n, double* scal, int* flags) {
    if (flags[F_ACTIVE] == 0) return;
    const double pq = sum_partials<RT>(part, n);
    if (threadIdx.x == 0) {
        scal[S_PQ] = pq;
        const double a = scal[S_RZ] / pq;
        if (!(pq > 0.0) || !isfinite(a)) {
            flags[F_ACTIVE] = 0;
            flags[F_REASON] = R_BREAK;
        } else {
            scal[S_ALPHA] = a;
        }
    }
}

// rr = ||r||^2, rz = <r, z> (= rr without preconditioner), beta = rz_new / rz_old, stop tests.
__global__ void __launch_bounds__(RT) k_beta(const double* part_rr, int n_rr, const double* part_rz, int n_rz,
                                             double* scal, int* flags) {
    if (flags[F_ACTIVE] == 0) return;
    const double rr = sum_partials<RT>(part_rr, n_rr);
    __syncthreads();
    const double rz = part_rz ? sum_partials<RT>(part_rz, n_rz) : rr;
    if (threadIdx.x == 0) {
        const double b = rz / scal[S_RZ];
        scal[S_RR] = rr;
        scal[S_BETA] = b;
        scal[S_RZ] = rz;
        const int it = flags[F_ITER] + 1;
        flags[F_ITER] = it;
        if (!isfinite(rr) || (part_rz && (!(rz > 0.0) || !isfinite(b)))) {
            flags[F_ACTIVE] = 0;
            flags[F_REASON] = R_BREAK;
        } else if (rr <= scal[S_TOL2]) {
            flags[F_ACTIVE] = 0;
            flags[F_REASON] = R_CONV;
        } else if (it >= flags[F_MAXIT]) {
            flags[F_ACTIVE] = 0;
            flags[F_REASON] = R_MAXIT;
        }
    }
}

__global__ void k_set_active(int* flags, double* scal, int restart_dir) {
    flags[F_ACTIVE] = flags[F_ITER] < flags[F_MAXIT] ? 1 : 0;
    flags[F_REASON] = flags[F_ACTIVE] ? R_RUN : R_MAXIT;
    if (restart_dir) scal[S_BETA] = 0.0;
}

// d (centred order) -> dhalf = (d(q) + d(-q)) / (2 N^3) in FFT order for q3 in [0, N/2], in the
// blocked layout [q2][q3 group][q1][C] read by the preconditioner's middle pass.
__global__ void k_precond_set(const float* __restrict__ d, float* __restrict__ dh, int N, int C) {
    const int H = N / 2 + 1;
    const int ng = (H + C - 1) / C;
    const int64_t tot = (int64_t)N * N * H;
    const double inv = 1.0 / ((double)N * N * N);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int j3 = (int)(i % H), j2 = (int)((i / H) % N), j1 = (int)(i / ((int64_t)H * N));
        const int c1 = (j1 + N / 2) % N, c2 = (j2 + N / 2) % N, c3 = (j3 + N / 2) % N;
        const int m1 = (N - j1) % N, m2 = (N - j2) % N, m3 = (N - j3) % N;
        const int e1 = (m1 + N / 2) % N, e2 = (m2 + N / 2) % N, e3 = (m3 + N / 2) % N;
        const double v = 0.5 * ((double)d[((int64_t)c1 * N + c2) * N + c3] + (double)d[((int64_t)e1 * N + e2) * N + e3]);
        dh[(((int64_t)j2 * ng + j3 / C) * N + j1) * C + j3 % C] = (float)(v * inv);
    }
}

#define CK(e)                                                                              \
    do {                                                                                   \
        hipError_t e__ = (e);                                                              \
        if (e__ != hipSuccess) return firm_fail(p, FIRM_ERR_HIP, std::string(#e) + ": " + hipGetErrorString(e__)); \
    } while (0)

}  // namespace

hipError_t precond_set(firm_plan p, const float* d_centred) {
    const int N = p->N;
    const int64_t n = (int64_t)N * N * (N / 2 + 1);
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_precond_set, dim3(blocks), dim3(256), 0, p->stream, d_centred, p->dhalf, N,
                       fft_cols_per_block(N, false));
    return hipGetLastError();
}

// FP32 CG (FP64 sums and scalars) on (A*A + lam) x = atb from the guess in x.  Stops when the
// residual measured with the FP32 product is <= tol ||atb|| or after max_iter iterations.
static firm_status cg_core32(firm_plan p, const float* atb, float* x, double lam, double tol, int max_iter,
                             const float* d, firm_cg_report* rep) {
    auto t0 = std::chrono::steady_clock::now();
    const int N = p->N;
    const int64_t n = (int64_t)N * N * N;
    hipStream_t st = p->stream;
    double* scal = p->scal;
    int* flags = p->flags;
    const int nb_apply = fft_apply_cg_partials(p);     // partials of <p, q> per product
    const int nb_step = fft_apply_cg_step_partials(p);  // partials of ||r||^2 per CG step
    const int nb_prec = fft_precond_partials(p);        // partials of <r, z> per preconditioner step
    if (nb_apply <= 0 || nb_apply > p->npart || nb_step <= 0 || nb_step > p->npart || nb_prec <= 0 ||
        nb_prec > p->npart)
        CK(hipErrorInvalidValue);
    bool pc = (d != nullptr);
    int refinements = 0, fell_back = 0;

    if (pc) CK(precond_set(p, d));
    // r = atb - (A*A + lam) x, ||atb||^2
    CK(fft_apply_AtA(p, x, p->tmp, (float)lam));
    hipLaunchKernelGGL(k_resid, dim3(VB), dim3(VT), 0, st, atb, p->tmp, p->r, n, p->partials3, nullptr);
    hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(VT), 0, st, p->partials3, VB, scal, (int)S_RR, -1, nullptr);
    hipLaunchKernelGGL(k_dot, dim3(VB), dim3(VT), 0, st, atb, atb, n, p->partials3);
    hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(VT), 0, st, p->partials3, VB, scal, (int)S_BB, -1, nullptr);
    hipLaunchKernelGGL(k_init, dim3(1), dim3(1), 0, st, scal, flags, tol, max_iter);
    CK(fill_zero(p->p, n * sizeof(float), st));
    // N > 64: z stays as its row half spectra in S1 and the product's first pass finishes the
    // preconditioner (fft_apply_cg_front_pz), so that z is never written or read
    auto fused = [&]() { return pc && N > 64; };
    auto set_rz = [&](bool guarded) -> hipError_t {
        const int* fl = guarded ? flags : nullptr;
        if (pc) {
            hipError_t e = fft_precond(p, p->dhalf, p->r, fused() ? nullptr : p->z, fl, p->partials2);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(VT), 0, st, p->partials2, nb_prec, scal, (int)S_RZ, -1, fl);
        } else {
            hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(VT), 0, st, p->partials3, VB, scal, (int)S_RZ, -1, fl);
        }
        return hipGetLastError();
    };
    // rz from the initial residual (partials3 still holds ||r||^2 partials only if no
    // preconditioner; recompute them to be safe)
    hipLaunchKernelGGL(k_dot, dim3(VB), dim3(VT), 0, st, p->r, p->r, n, p->partials3);
    CK(set_rz(false));

    int it_host = 0;
    firm_status result = FIRM_OK;
    double stag_rr = INFINITY;  // squared residual norm at the last halving
    int stag_it = 0;            // iteration of the last halving
    for (;;) {
        for (int i = 0; i < p->check_every; ++i) {
            const float* src = pc ? p->z : p->r;
            // p = src + beta p and q = (A*A + lam) p, with alpha = rz / <p, q> formed between the
            // two halves of the product and the step x += alpha p, r -= alpha q in its last pass
            if (fused())
                CK(fft_apply_cg_front_pz(p, p->p, (float)lam, scal + S_BETA, flags + F_ACTIVE, p->partials));
            else
                CK(fft_apply_cg_front(p, src, p->p, (float)lam, scal + S_BETA, flags + F_ACTIVE, p->partials));
            hipLaunchKernelGGL(k_alpha, dim3(1), dim3(RT), 0, st, p->partials, nb_apply, scal, flags);
            CK(fft_apply_cg_step(p, x, p->p, p->r, scal + S_ALPHA, flags + F_ACTIVE, p->partials3));
            if (pc) CK(fft_precond(p, p->dhalf, p->r, fused() ? nullptr : p->z, flags + F_ACTIVE, p->partials2));
            hipLaunchKernelGGL(k_beta, dim3(1), dim3(RT), 0, st, p->partials3, nb_step, pc ? p->partials2 : nullptr,
                               nb_prec, scal, flags);
            ++it_host;
            if (p->refine_every > 0 && it_host % p->refine_every == 0) {
                // true residual replacement, skipped by the kernels once inactive
                CK(fft_apply_AtA(p, x, p->tmp, (float)lam));
                hipLaunchKernelGGL(k_resid, dim3(VB), dim3(VT), 0, st, atb, p->tmp, p->r, n, p->partials3, flags);
                hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(VT), 0, st, p->partials3, VB, scal, (int)S_RR,
                                   (int)S_TRUE, flags);
                CK(set_rz(true));
                ++refinements;
            }
        }
        CK(hipMemcpyAsync(p->host_flags, flags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
        if (pc && p->stagnation_iters > 0)
            CK(hipMemcpyAsync(p->host_scal, scal, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        // restart as plain CG from the current x (after a breakdown or a stagnation of the
        // preconditioned recursion)
        auto restart_plain = [&]() -> hipError_t {
            pc = false;
            fell_back = 1;
            hipError_t e = fft_apply_AtA(p, x, p->tmp, (float)lam);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_resid, dim3(VB), dim3(VT), 0, st, atb, p->tmp, p->r, n, p->partials3, nullptr);
            hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(VT), 0, st, p->partials3, VB, scal, (int)S_RR, (int)S_RZ,
                               nullptr);
            hipLaunchKernelGGL(k_set_active, dim3(1), dim3(1), 0, st, flags, scal, 1);
            return hipGetLastError();
        };
        if (p->host_flags[F_ACTIVE]) {
            if (pc && p->stagnation_iters > 0) {
                // stagnation: the residual norm has not halved (its square not quartered) within
                // stagnation_iters iterations of the last halving
                const double rr = p->host_scal[S_RR];
                const int it = p->host_flags[F_ITER];
                if (rr <= 0.25 * stag_rr) {
                    stag_rr = rr;
                    stag_it = it;
                } else if (it - stag_it >= p->stagnation_iters) {
                    CK(restart_plain());
                }
            }
            continue;
        }
        const int reason = p->host_flags[F_REASON];
        if (reason == R_BREAK) {
            if (pc) {
                CK(restart_plain());
                continue;
            }
            result = FIRM_ERR_BREAKDOWN;
            break;
        }
        // confirm with the true residual (FP64 sum of the FP32 product)
        CK(fft_apply_AtA(p, x, p->tmp, (float)lam));
        hipLaunchKernelGGL(k_resid, dim3(VB), dim3(VT), 0, st, atb, p->tmp, p->r, n, p->partials3, nullptr);
        hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(VT), 0, st, p->partials3, VB, scal, (int)S_TRUE,
                           (int)S_RR, nullptr);
        CK(hipMemcpyAsync(p->host_scal, scal, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
        CK(hipMemcpyAsync(p->host_flags, flags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        const bool ok = p->host_scal[S_TRUE] <= p->host_scal[S_TOL2];
        if (ok) { result = FIRM_OK; break; }
        if (p->host_flags[F_ITER] >= max_iter) { result = FIRM_ERR_NOT_CONVERGED; break; }
        // recursive residual drifted below tol: continue from the true residual
        CK(set_rz(false));
        hipLaunchKernelGGL(k_set_active, dim3(1), dim3(1), 0, st, flags, scal, 0);
        ++refinements;
    }
    CK(hipMemcpyAsync(p->host_scal, scal, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(p->host_flags, flags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (rep) {
        const double bb = p->host_scal[S_BB] > 0 ? p->host_scal[S_BB] : 1.0;
        rep->iters = p->host_flags[F_ITER];
        rep->refinements = refinements;
        rep->fell_back = fell_back;
        rep->status = result;
        rep->rel_res = std::sqrt(p->host_scal[S_RR] / bb);
        rep->true_rel_res = std::sqrt(p->host_scal[S_TRUE] / bb);
        rep->t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return result;
}

namespace {

__global__ void k_d_from_f(double* __restrict__ o, const float* __restrict__ a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) o[i] = a[i];
}
__global__ void k_f_from_d(float* __restrict__ o, const double* __restrict__ a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) o[i] = (float)a[i];
}
__global__ void k_add_f_to_d(double* __restrict__ x, const float* __restrict__ d, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) x[i] += (double)d[i];
}
// r = atb - y (FP64); partial sums of r^2
__global__ void __launch_bounds__(VT) k_resid64(const double* __restrict__ atb, const double* __restrict__ y,
                                                double* __restrict__ r, int64_t n, double* partials) {
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
        const double v = atb[i] - y[i];
        r[i] = v;
        acc += v * v;
    }
    const double s = block_reduce(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
__global__ void __launch_bounds__(VT) k_dot64(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                                              double* partials) {
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) acc += a[i] * b[i];
    const double s = block_reduce(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
__global__ void k_dir64(double* __restrict__ pv, const double* __restrict__ r, const double* scal, int64_t n) {
    const double b = scal[S_BETA];
    for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) pv[i] = r[i] + b * pv[i];
}
__global__ void __launch_bounds__(VT) k_update64(double* __restrict__ x, const double* __restrict__ pv,
                                                 double* __restrict__ r, const double* __restrict__ q, int64_t n,
                                                 const double* scal, double* partials) {
    const double a = scal[S_ALPHA];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
        x[i] += a * pv[i];
        const double rv = r[i] - a * q[i];
        r[i] = rv;
        acc += rv * rv;
    }
    const double s = block_reduce(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
__global__ void k_set_scalar(double* scal, int idx, double v) { scal[idx] = v; }
__global__ void k_alpha64(double* scal) {
    scal[S_ALPHA] = scal[S_RZ] / scal[S_PQ];
}
__global__ void k_beta64(double* scal) {
    scal[S_BETA] = scal[S_RR] / scal[S_RZ];
    scal[S_RZ] = scal[S_RR];
}

}  // namespace

#define L1(k, ...) hipLaunchKernelGGL(k, dim3(VB), dim3(VT), 0, st, __VA_ARGS__)
#define R1(...) hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(VT), 0, st, __VA_ARGS__)

// ||atb - (A*A + lam) x||^2 with the FP64 product, and ||atb||^2 (atb, x: FP64 device arrays;
// x must not be p->y64 or p->r64).
static firm_status residual64(firm_plan p, const double* atb, const double* x, double lam, double* rr,
                              double* bb) {
    const int64_t n = (int64_t)p->N * p->N * p->N;
    hipStream_t st = p->stream;
    CK(fft_apply_AtA64(p, x, p->y64, lam));
    L1(k_resid64, atb, p->y64, p->r64, n, p->partials3);
    R1(p->partials3, VB, p->scal, (int)S_TRUE, -1, nullptr);
    L1(k_dot64, atb, atb, n, p->partials3);
    R1(p->partials3, VB, p->scal, (int)S_BB, -1, nullptr);
    CK(hipMemcpyAsync(p->host_scal, p->scal, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    *rr = p->host_scal[S_TRUE];
    *bb = p->host_scal[S_BB] > 0 ? p->host_scal[S_BB] : 1.0;
    return FIRM_OK;
}

// FP64 CG: vectors, product and sums in double (khat64 from the FP32 kernel values); the
// iterate xw (FP64, device) holds the initial guess and receives the solution.
static firm_status cg_fp64(firm_plan p, const double* atb, double* xw, double lam, double tol, int max_iter,
                           firm_cg_report* rep) {
    const int64_t n = (int64_t)p->N * p->N * p->N;
    hipStream_t st = p->stream;
    double* sc = p->scal;
    CK(fft_apply_AtA64(p, xw, p->y64, lam));
    L1(k_resid64, atb, p->y64, p->r64, n, p->partials3);
    R1(p->partials3, VB, sc, (int)S_RR, (int)S_RZ, nullptr);
    L1(k_dot64, atb, atb, n, p->partials3);
    R1(p->partials3, VB, sc, (int)S_BB, -1, nullptr);
    hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, st, sc, (int)S_BETA, 0.0);
    CK(fill_zero(p->p64, n * sizeof(double), st));
    CK(hipMemcpyAsync(p->host_scal, sc, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    const double bb = p->host_scal[S_BB] > 0 ? p->host_scal[S_BB] : 1.0;
    double rr = p->host_scal[S_RR];
    int it = 0;
    firm_status result = FIRM_OK;
    while (rr > tol * tol * bb) {
        if (it >= max_iter) { result = FIRM_ERR_NOT_CONVERGED; break; }
        L1(k_dir64, p->p64, p->r64, sc, n);
        CK(fft_apply_AtA64(p, p->p64, p->q64, lam));
        L1(k_dot64, p->p64, p->q64, n, p->partials);
        R1(p->partials, VB, sc, (int)S_PQ, -1, nullptr);
        hipLaunchKernelGGL(k_alpha64, dim3(1), dim3(1), 0, st, sc);
        L1(k_update64, xw, p->p64, p->r64, p->q64, n, sc, p->partials3);
        R1(p->partials3, VB, sc, (int)S_RR, -1, nullptr);
        hipLaunchKernelGGL(k_beta64, dim3(1), dim3(1), 0, st, sc);
        CK(hipMemcpyAsync(p->host_scal, sc, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        ++it;
        rr = p->host_scal[S_RR];
        if (!(p->host_scal[S_PQ] > 0.0) || !std::isfinite(rr)) { result = FIRM_ERR_BREAKDOWN; break; }
    }
    if (rep) {
        rep->iters = it;
        rep->rel_res = std::sqrt(rr / bb);
    }
    return result;
}

// FP64 iterative refinement: r = atb - (A*A + lam) x with the FP64 product and FP64 x; each
// correction solves (A*A + lam) d = r with FP32 (P)CG to a relative tolerance, x += d.
static firm_status cg_refine64(firm_plan p, const double* atb, double* xw, double lam, double tol, int max_iter,
                               const float* d, firm_cg_report* rep) {
    const int64_t n = (int64_t)p->N * p->N * p->N;
    hipStream_t st = p->stream;
    L1(k_dot64, atb, atb, n, p->partials3);
    R1(p->partials3, VB, p->scal, (int)S_BB, -1, nullptr);
    // a zero initial guess (the usual case) has the residual atb itself: no first product
    L1(k_dot64, xw, xw, n, p->partials3);
    R1(p->partials3, VB, p->scal, (int)S_TRUE, -1, nullptr);
    CK(hipMemcpyAsync(p->host_scal, p->scal, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    const double bb0 = p->host_scal[S_BB];
    const double bb = bb0 > 0 ? bb0 : 1.0;
    bool xzero = p->host_scal[S_TRUE] == 0.0;
    int total = 0, outer = 0, fell_back = 0;
    double rr = 0.0;
    firm_status result = FIRM_OK;
    for (;;) {
        const double* res = p->r64;
        if (xzero) {
            rr = bb0;
            res = atb;
            xzero = false;
        } else {
            CK(fft_apply_AtA64(p, xw, p->y64, lam));
            L1(k_resid64, atb, p->y64, p->r64, n, p->partials3);
            R1(p->partials3, VB, p->scal, (int)S_TRUE, -1, nullptr);
            CK(hipMemcpyAsync(p->host_scal, p->scal, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
            CK(hipStreamSynchronize(st));
            rr = p->host_scal[S_TRUE];
        }
        if (!std::isfinite(rr)) { result = FIRM_ERR_BREAKDOWN; break; }
        if (rr <= tol * tol * bb) break;
        if (total >= max_iter) { result = FIRM_ERR_NOT_CONVERGED; break; }
        // correction with the FP32 solver; the rhs is the FP64 residual rounded to FP32
        L1(k_f_from_d, p->rhs, res, n);
        CK(fill_zero(p->dvec, n * sizeof(float), st));
        const double rel = std::sqrt(rr / bb);
        // an explicit inner tolerance bounds every correction, which then goes to half of the
        // reduction still needed; by default the first goes to sqrt(tol) and each later one to
        // 0.8 of the reduction still needed (the FP64 residual is checked after every
        // correction, so an overshoot below tol only costs iterations)
        const double floor_tol = p->inner_tol > 0 ? p->inner_tol
                                                  : (outer == 0 ? std::min(1e-2, std::max(1e-4, std::sqrt(tol))) : 1e-4);
        const double inner = std::max(floor_tol, (p->inner_tol > 0 ? 0.5 : 0.8) * tol / rel);
        firm_cg_report ir{};
        firm_status is = cg_core32(p, p->rhs, p->dvec, lam, std::min(inner, 0.5), max_iter - total, d, &ir);
        if (is != FIRM_OK && is != FIRM_ERR_NOT_CONVERGED && is != FIRM_ERR_BREAKDOWN) return is;
        total += ir.iters;
        fell_back |= ir.fell_back;
        L1(k_add_f_to_d, xw, p->dvec, n);
        ++outer;
        if (ir.iters == 0) { result = FIRM_ERR_NOT_CONVERGED; break; }  // no progress possible
    }
    if (rep) {
        rep->iters = total;
        rep->refinements = outer;
        rep->fell_back = fell_back;
        rep->rel_res = std::sqrt(rr / bb);
    }
    return result;
}

static firm_status finish(firm_plan p, firm_status r, firm_cg_report* rep) {
    if (rep) rep->status = r;
    if (r == FIRM_ERR_NOT_CONVERGED) return firm_fail(p, r, "CG reached max_iter above tol");
    if (r == FIRM_ERR_BREAKDOWN) return firm_fail(p, r, "CG breakdown (non-positive curvature)");
    return r;
}

static bool solver_ran(firm_status r) {
    return r == FIRM_OK || r == FIRM_ERR_NOT_CONVERGED || r == FIRM_ERR_BREAKDOWN;
}

// FP32 in and out: the solution returned is FP32 in every mode, and the reported true residual
// is that of the FP32 x written out (for precision 1 and 2 it can exceed the FP64 iterate's
// residual by the rounding of x, about 6e-8 times the condition number).
firm_status cg_solve(firm_plan p, const float* atb, float* x, double lam, double tol, int max_iter,
                     const float* d, firm_cg_report* rep) {
    auto t0 = std::chrono::steady_clock::now();
    firm_status fs = ensure_fp64(p);
    if (fs != FIRM_OK) return fs;
    const int64_t n = (int64_t)p->N * p->N * p->N;
    hipStream_t st = p->stream;
    L1(k_d_from_f, p->atb64, atb, n);
    firm_status r;
    if (p->precision == 0) {
        r = cg_core32(p, atb, x, lam, tol, max_iter, d, rep);
    } else {
        L1(k_d_from_f, p->x64, x, n);
        r = p->precision == 2 ? cg_fp64(p, p->atb64, p->x64, lam, tol, max_iter, rep)
                              : cg_refine64(p, p->atb64, p->x64, lam, tol, max_iter, d, rep);
        if (solver_ran(r)) L1(k_f_from_d, x, p->x64, n);
    }
    if (solver_ran(r)) {
        L1(k_d_from_f, p->x64, x, n);
        double trr = 0, tbb = 1;
        fs = residual64(p, p->atb64, p->x64, lam, &trr, &tbb);
        if (fs != FIRM_OK) return fs;
        if (rep) {
            rep->true_rel_res = std::sqrt(trr / tbb);
            rep->t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
    }
    return finish(p, r, rep);
}

// FP64 in and out (precision 1 or 2): x is the FP64 iterate itself.
firm_status cg_solve64(firm_plan p, const double* atb, double* x, double lam, double tol, int max_iter,
                       const float* d, firm_cg_report* rep) {
    auto t0 = std::chrono::steady_clock::now();
    firm_status fs = ensure_fp64(p);
    if (fs != FIRM_OK) return fs;
    firm_status r = p->precision == 2 ? cg_fp64(p, atb, x, lam, tol, max_iter, rep)
                                      : cg_refine64(p, atb, x, lam, tol, max_iter, d, rep);
    if (solver_ran(r)) {
        double trr = 0, tbb = 1;
        fs = residual64(p, atb, x, lam, &trr, &tbb);
        if (fs != FIRM_OK) return fs;
        if (rep) {
            rep->true_rel_res = std::sqrt(trr / tbb);
            rep->t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
    }
    return finish(p, r, rep);
}
