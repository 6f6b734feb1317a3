// Unrolled PCG objective of the learned preconditioner: the energy-norm error that k steps of
// preconditioned CG leave (CG minimises that norm over its Krylov space, section 3.3), and its
// gradient with respect to the log of the Fourier diagonal d.
//
// For a probe z and b = T z (T = A*A + lambda), PCG from x0 = 0 gives x_k; the loss is
// ||z - x_k||_T^2 / ||z||_T^2.  With the step lengths alpha_i and ratios beta_i held fixed, x_k is
// a fixed polynomial combination of (P T)^j P b, and since x_k minimises the error over that
// Krylov space, the derivative of the minimum is the derivative of the combination (envelope
// theorem).  The reverse pass therefore runs the recursion's adjoint with the stored scalars:
//   xbar = -2 T e / ||z||_T^2,
//   Pbar_i = alpha_i xbar + beta_i Pbar_{i+1} - alpha_i T Rbar_{i+1},   Sbar_i = Pbar_i,
//   Rbar_i = Rbar_{i+1} + P Sbar_i,
//   dL/dd(q) += Re(conj(F Sbar_i)(q) (F r_i)(q)) / N^3   (P = F^{-1} diag(d) F, Parseval),
// each step one product, one preconditioner application and two forward transforms.
#include <algorithm>

#include "firm_internal.h"

namespace {

constexpr int UT = 256;  // threads per block
constexpr int UB = 512;  // blocks of the grid-stride kernels

// device scalars: rho_0..rho_k, pi_0..pi_{k-1}, alpha, beta, then loss numerator and <z, b>
struct Slots {
    int k;
    __host__ __device__ int rho(int i) const { return i; }
    __host__ __device__ int pi(int i) const { return k + 1 + i; }
    __host__ __device__ int alpha(int i) const { return 2 * k + 1 + i; }
    __host__ __device__ int beta(int i) const { return 3 * k + 1 + i; }
    __host__ __device__ int num() const { return 4 * k + 1; }
    __host__ __device__ int nz() const { return 4 * k + 2; }
    __host__ __device__ int count() const { return 4 * k + 3; }
};

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[UT / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < UT / 64; ++i) s += red[i];
    return s;
}

__global__ void __launch_bounds__(UT) k_udot(const float* __restrict__ a, const float* __restrict__ b, int64_t n,
                                             double* __restrict__ part) {
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)UT + threadIdx.x; i < n; i += (int64_t)gridDim.x * UT)
        acc += (double)a[i] * (double)b[i];
    const double s = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// sc[slot] = sum of the nb partials
__global__ void __launch_bounds__(UT) k_ufinish(const double* __restrict__ part, int nb, double* sc, int slot) {
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += UT) a += part[i];
    const double s = block_sum(a);
    if (threadIdx.x == 0) sc[slot] = s;
}

__global__ void k_ualpha(double* sc, Slots sl, int i) { sc[sl.alpha(i)] = sc[sl.rho(i)] / sc[sl.pi(i)]; }
__global__ void k_ubeta(double* sc, Slots sl, int i) { sc[sl.beta(i)] = sc[sl.rho(i + 1)] / sc[sl.rho(i)]; }

// x += alpha p, rn = r - alpha q (FP64 arithmetic, FP32 storage)
__global__ void __launch_bounds__(UT) k_ustep(float* __restrict__ x, const float* __restrict__ p,
                                              const float* __restrict__ r, const float* __restrict__ q,
                                              float* __restrict__ rn, const double* __restrict__ sc, int slot,
                                              int64_t n) {
    const double a = sc[slot];
    for (int64_t i = blockIdx.x * (int64_t)UT + threadIdx.x; i < n; i += (int64_t)gridDim.x * UT) {
        x[i] = (float)((double)x[i] + a * p[i]);
        rn[i] = (float)((double)r[i] - a * q[i]);
    }
}

// p = s + beta p
__global__ void __launch_bounds__(UT) k_udir(float* __restrict__ p, const float* __restrict__ s,
                                             const double* __restrict__ sc, int slot, int64_t n) {
    const double bt = sc[slot];
    for (int64_t i = blockIdx.x * (int64_t)UT + threadIdx.x; i < n; i += (int64_t)gridDim.x * UT)
        p[i] = (float)((double)s[i] + bt * p[i]);
}

// e = z - x
__global__ void __launch_bounds__(UT) k_usub(float* __restrict__ e, const float* __restrict__ z,
                                             const float* __restrict__ x, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)UT + threadIdx.x; i < n; i += (int64_t)gridDim.x * UT) e[i] = z[i] - x[i];
}

// xbar = -2 u / <z, b>
__global__ void __launch_bounds__(UT) k_uxbar(float* __restrict__ xb, const float* __restrict__ u,
                                              const double* __restrict__ sc, int slot, int64_t n) {
    const double c = -2.0 / sc[slot];
    for (int64_t i = blockIdx.x * (int64_t)UT + threadIdx.x; i < n; i += (int64_t)gridDim.x * UT)
        xb[i] = (float)(c * u[i]);
}

// Pbar = alpha_i xbar + beta_i Pbar - alpha_i u (u = T Rbar_{i+1}; Pbar holds Pbar_{i+1});
// at the last step Pbar_{k} = Rbar_{k} = 0, so Pbar = alpha xbar
__global__ void __launch_bounds__(UT) k_upbar(float* __restrict__ pb, const float* __restrict__ xb,
                                              const float* __restrict__ u, const double* __restrict__ sc, Slots sl,
                                              int i, int last, int64_t n) {
    const double a = sc[sl.alpha(i)];
    if (last) {
        for (int64_t j = blockIdx.x * (int64_t)UT + threadIdx.x; j < n; j += (int64_t)gridDim.x * UT)
            pb[j] = (float)(a * xb[j]);
        return;
    }
    const double bt = sc[sl.beta(i)];
    for (int64_t j = blockIdx.x * (int64_t)UT + threadIdx.x; j < n; j += (int64_t)gridDim.x * UT)
        pb[j] = (float)(a * xb[j] + bt * pb[j] - a * u[j]);
}

// y += x
__global__ void __launch_bounds__(UT) k_uadd(float* __restrict__ y, const float* __restrict__ x, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)UT + threadIdx.x; i < n; i += (int64_t)gridDim.x * UT) y[i] += x[i];
}

// grad = acc d c (centred grid)
__global__ void __launch_bounds__(UT) k_ugrad(float* __restrict__ g, const float* __restrict__ acc,
                                              const float* __restrict__ d, float c, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)UT + threadIdx.x; i < n; i += (int64_t)gridDim.x * UT)
        g[i] = acc[i] * d[i] * c;
}

int ublocks(int64_t n) { return (int)std::min<int64_t>((n + UT - 1) / UT, UB); }

}  // namespace

int64_t unrolled_workspace_floats(int N, int k) { return (int64_t)(k + 7) * N * N * N; }
int unrolled_scalar_count(int k) { return Slots{k}.count(); }

// ws: unrolled_workspace_floats(N, k) floats; sc: unrolled_scalar_count(k) doubles; S1, S2 and
// the product workspaces of the plan.  loss_host: mean loss over the probes; grad (may be null).
hipError_t pcg_unrolled(firm_plan p, const float* d, const float* probes, int nprobes, int k, float lam, float* ws,
                        double* sc, double* loss_host, float* grad) {
    const int64_t n = (int64_t)p->N * p->N * p->N;
    hipStream_t st = p->stream;
    const int nb = ublocks(n);
    const Slots sl{k};
    float* rs = ws;                 // r_0 .. r_{k-1}
    float* x = ws + (int64_t)k * n;
    float* pv = x + n;
    float* q = pv + n;              // products (and u = T e)
    float* s = q + n;               // preconditioned residual / P Sbar
    float* rn = s + n;              // r_k, then Rbar
    float* pb = rn + n;             // Pbar
    float* acc = pb + n;            // gradient accumulator, centred grid
    float* junk = p->tmp;           // |F Sbar|^2 of the accumulation, unused
    double* part = p->partials3;
#define UCK(call)                            \
    do {                                     \
        hipError_t e_ = (call);              \
        if (e_ != hipSuccess) return e_;     \
    } while (0)
    auto dot = [&](const float* a, const float* b, int slot) -> hipError_t {
        hipLaunchKernelGGL(k_udot, dim3(nb), dim3(UT), 0, st, a, b, n, part);
        hipLaunchKernelGGL(k_ufinish, dim3(1), dim3(UT), 0, st, part, nb, sc, slot);
        return hipGetLastError();
    };
    UCK(precond_set(p, d));
    UCK(fill_zero(acc, n * sizeof(float), st));
    double total = 0.0;
    for (int pr = 0; pr < nprobes; ++pr) {
        const float* z = probes + (int64_t)pr * n;
        // forward: b = T z, PCG from x0 = 0
        UCK(fft_apply_AtA(p, z, rs, lam));
        UCK(dot(z, rs, sl.nz()));
        UCK(fill_zero(x, n * sizeof(float), st));
        UCK(fft_precond(p, p->dhalf, rs, s));
        UCK(hipMemcpyAsync(pv, s, n * sizeof(float), hipMemcpyDeviceToDevice, st));
        UCK(dot(rs, s, sl.rho(0)));
        for (int i = 0; i < k; ++i) {
            const float* ri = rs + (int64_t)i * n;
            float* rnext = i + 1 < k ? rs + (int64_t)(i + 1) * n : rn;
            UCK(fft_apply_AtA(p, pv, q, lam));
            UCK(dot(pv, q, sl.pi(i)));
            hipLaunchKernelGGL(k_ualpha, dim3(1), dim3(1), 0, st, sc, sl, i);
            hipLaunchKernelGGL(k_ustep, dim3(nb), dim3(UT), 0, st, x, pv, ri, q, rnext, sc, sl.alpha(i), n);
            UCK(fft_precond(p, p->dhalf, rnext, s));
            UCK(dot(rnext, s, sl.rho(i + 1)));
            hipLaunchKernelGGL(k_ubeta, dim3(1), dim3(1), 0, st, sc, sl, i);
            hipLaunchKernelGGL(k_udir, dim3(nb), dim3(UT), 0, st, pv, s, sc, sl.beta(i), n);
            UCK(hipGetLastError());
        }
        // loss: e = z - x_k, u = T e
        hipLaunchKernelGGL(k_usub, dim3(nb), dim3(UT), 0, st, pv, z, x, n);
        UCK(fft_apply_AtA(p, pv, q, lam));
        UCK(dot(pv, q, sl.num()));
        double h2[2];
        UCK(hipMemcpyAsync(h2, sc + sl.num(), 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        UCK(hipStreamSynchronize(st));
        total += h2[0] / h2[1];
        if (!grad) continue;
        // reverse pass; xbar overwrites x (x_k is no longer needed), Rbar lives in rn
        hipLaunchKernelGGL(k_uxbar, dim3(nb), dim3(UT), 0, st, x, q, sc, sl.nz(), n);
        UCK(fill_zero(junk, n * sizeof(float), st));
        for (int i = k - 1; i >= 0; --i) {
            const int last = i == k - 1;
            if (!last) UCK(fft_apply_AtA(p, rn, q, lam));  // u = T Rbar_{i+1}
            hipLaunchKernelGGL(k_upbar, dim3(nb), dim3(UT), 0, st, pb, x, q, sc, sl, i, last, n);
            // dL/dd += Re(conj(F Sbar_i) F r_i) (Sbar_i = Pbar_i), accumulated on the centred grid
            UCK(fft_forward_r2c(p, pb, p->S1));
            UCK(fft_forward_r2c(p, rs + (int64_t)i * n, p->S2));
            UCK(probe_accumulate(p, p->S2, p->S1, junk, acc, part, 1024));
            if (i > 0) {  // Rbar_i = Rbar_{i+1} + P Sbar_i (Rbar_0 is not needed)
                if (last) UCK(fill_zero(rn, n * sizeof(float), st));
                UCK(fft_precond(p, p->dhalf, pb, s));
                hipLaunchKernelGGL(k_uadd, dim3(nb), dim3(UT), 0, st, rn, s, n);
            }
            UCK(hipGetLastError());
        }
    }
    if (grad) {
        const float c = (float)(1.0 / ((double)n * nprobes));
        hipLaunchKernelGGL(k_ugrad, dim3(nb), dim3(UT), 0, st, grad, acc, d, c, n);
        UCK(hipGetLastError());
    }
    *loss_host = total / nprobes;
    return hipStreamSynchronize(st);
#undef UCK
}
