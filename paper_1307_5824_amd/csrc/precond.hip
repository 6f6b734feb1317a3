// Kernels that serve the Fourier-diagonal preconditioners: the network's input features (pooled
// kernel spectrum), the probe statistics of the probe-loss objective, and T. Chan's optimal
// circulant spectrum (the Fourier diagonal of A*A + lambda; circulant diagonalisation, eq. circ1).
#include <algorithm>

#include "firm_internal.h"

namespace {

// feat[f] (centred R^3) = log(mean of |K^| over the (2N/R)^3 block / Ker(0) + lam_rel); K^ is read
// from the blocked half spectrum, the other half by K^(-q) = K^(q).
__global__ void k_features(const float* __restrict__ kh, int N, int C, int R, float inv_ker0, float lam_rel,
                           float* __restrict__ feat) {
    const int L = 2 * N, s = L / R, ng = (N + 1 + C - 1) / C;
    const int64_t RV = (int64_t)R * R * R;
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < RV; f += (int64_t)gridDim.x * blockDim.x) {
        const int f1 = (int)(f / ((int64_t)R * R)), f2 = (int)((f / R) % R), f3 = (int)(f % R);
        double acc = 0.0;
        for (int a = 0; a < s; ++a)
            for (int b = 0; b < s; ++b)
                for (int c = 0; c < s; ++c) {
                    int k1 = ((f1 * s + a) - N + L) % L, k2 = ((f2 * s + b) - N + L) % L, k3 = ((f3 * s + c) - N + L) % L;
                    if (k3 > N) { k1 = (L - k1) % L; k2 = (L - k2) % L; k3 = L - k3; }
                    acc += fabsf(kh[(((int64_t)k2 * ng + k3 / C) * L + k1) * C + k3 % C]);
                }
        feat[f] = logf((float)(acc / ((double)s * s * s)) * inv_ker0 + lam_rel);
    }
}

// A[q] += |u^(q)|^2, B[q] += Re(conj u^ z^), partial sums of |z^|^2, on the centred N^3 grid from the
// half spectra (the other half by conjugate symmetry, which leaves these real quantities unchanged).
__global__ void __launch_bounds__(256) k_probe_accum(const float2* __restrict__ zh, const float2* __restrict__ uh,
                                                     int N, int QPn, float* __restrict__ A, float* __restrict__ B,
                                                     double* partials) {
    __shared__ double red[4];
    const int64_t n = (int64_t)N * N * N;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int q1 = (int)(i / ((int64_t)N * N)), q2 = (int)((i / N) % N), q3 = (int)(i % N);
        int k1 = (q1 + N / 2) % N, k2 = (q2 + N / 2) % N, k3 = (q3 + N / 2) % N;
        if (k3 > N / 2) { k1 = (N - k1) % N; k2 = (N - k2) % N; k3 = N - k3; }
        const int64_t h = ((int64_t)k1 * N + k2) * QPn + k3;
        const float2 z = zh[h], u = uh[h];
        A[i] += u.x * u.x + u.y * u.y;
        B[i] += u.x * z.x + u.y * z.y;
        acc += (double)z.x * z.x + (double)z.y * z.y;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

}  // namespace

hipError_t kernel_features(firm_plan p, float lam_rel, int res, float* feat) {
    // the stored spectrum carries the 1 / (2N)^3 of the inverse transform; the features use the
    // Fourier multiplier itself
    const double L3 = 8.0 * p->N * p->N * p->N;
    const int64_t RV = (int64_t)res * res * res;
    hipLaunchKernelGGL(k_features, dim3((unsigned)std::min<int64_t>((RV + 255) / 256, 4096)), dim3(256), 0, p->stream,
                       p->khat, p->N, fft_cols_per_block(2 * p->N, false), res, (float)(L3 / p->ker0), lam_rel, feat);
    return hipGetLastError();
}

namespace {

// T. Chan's optimal circulant of the N^3 Toeplitz operator, first column:
// c(j) = sum over o_d in {j_d, j_d - N} (o_d != -N) of prod_d (1 - |o_d| / N) Ker(o).
__global__ void k_chan_fold(const float* __restrict__ kerc, int N, float* __restrict__ c) {
    const int N2 = 2 * N;
    const int64_t n = (int64_t)N * N * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int j[3] = {(int)(i / ((int64_t)N * N)), (int)((i / N) % N), (int)(i % N)};
        double acc = 0.0;
        for (int m = 0; m < 8; ++m) {
            double w = 1.0;
            int pos[3];
            bool ok = true;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int o = (m >> d) & 1 ? j[d] - N : j[d];
                if (o == -N) ok = false;
                w *= 1.0 - (double)(o < 0 ? -o : o) / N;
                pos[d] = (o + N2) % N2;  // circulant position of offset o
            }
            if (ok) acc += w * (double)kerc[((int64_t)pos[0] * N2 + pos[1]) * N2 + pos[2]];
        }
        c[i] = (float)acc;
    }
}

// real spectrum on the centred N^3 grid (+ lam) from the half spectrum [N][N][QPn] in FFT order
__global__ void k_half_to_centred(const float2* __restrict__ h, int N, int QPn, float lam, float* __restrict__ out) {
    const int64_t n = (int64_t)N * N * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int q1 = (int)(i / ((int64_t)N * N)), q2 = (int)((i / N) % N), q3 = (int)(i % N);
        int k1 = (q1 + N / 2) % N, k2 = (q2 + N / 2) % N, k3 = (q3 + N / 2) % N;
        if (k3 > N / 2) { k1 = (N - k1) % N; k2 = (N - k2) % N; k3 = N - k3; }
        out[i] = h[((int64_t)k1 * N + k2) * QPn + k3].x + lam;
    }
}

// T. Chan's spectrum of the damping term mu L_p on the centred N^3 grid, added to out.  The symbol
// w^p = (sum_d a(theta_d))^p, a = 2 - 2 cos, expands by the multinomial theorem into products of
// per-axis powers a^i, whose kernels (2 - S - S^-1)^i have the taps (-1)^o C(2i, i + o), |o| <= i;
// Chan's Fejer-weighted fold of a product kernel is the product of the per-axis folds
// sum_o (1 - |o| / N) (-1)^o C(2i, i + o) cos(2 pi q o / N).
__device__ double chan_axis(int i, int q, int N) {
    double s = 0.0, binom = 1.0;  // C(2i, i + o) for o = i down to -i
    for (int o = i; o >= -i; --o) {
        const double tap = ((o & 1) ? -1.0 : 1.0) * binom;
        s += (1.0 - fabs((double)o) / N) * tap * cos(2.0 * M_PI * (double)q * o / N);
        const int k = i - o;  // binom = C(2i, k); next C(2i, k + 1)
        binom = binom * (2 * i - k) / (k + 1);
    }
    return s;
}

__global__ void k_chan_reg(float* __restrict__ out, int N, double mu, int order) {
    const int64_t n = (int64_t)N * N * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int q[3] = {(int)(i / ((int64_t)N * N)) - N / 2, (int)((i / N) % N) - N / 2, (int)(i % N) - N / 2};
        double acc = 0.0, fact[8] = {1, 1, 2, 6, 24, 120, 720, 5040};
        for (int a = 0; a <= order; ++a)
            for (int b = 0; a + b <= order; ++b) {
                const int c = order - a - b;
                acc += fact[order] / (fact[a] * fact[b] * fact[c]) * chan_axis(a, q[0], N) * chan_axis(b, q[1], N) *
                       chan_axis(c, q[2], N);
            }
        out[i] = (float)((double)out[i] + mu * acc);
    }
}

}  // namespace

hipError_t chan_spectrum(firm_plan p, double lam, float* out) {
    const int64_t n = (int64_t)p->N * p->N * p->N;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_chan_fold, dim3(blocks), dim3(256), 0, p->stream, p->kerc, p->N, p->tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = fft_forward_r2c(p, p->tmp, p->S1);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_half_to_centred, dim3(blocks), dim3(256), 0, p->stream, p->S1, p->N, p->QPn, (float)lam, out);
    if (p->reg_order > 0 && p->reg_mu_eff > 0.0)
        hipLaunchKernelGGL(k_chan_reg, dim3(blocks), dim3(256), 0, p->stream, out, p->N, p->reg_mu_eff, p->reg_order);
    return hipGetLastError();
}

hipError_t probe_accumulate(firm_plan p, const float2* zh, const float2* uh, float* A, float* B, double* partials,
                            int nblocks) {
    hipLaunchKernelGGL(k_probe_accum, dim3(nblocks), dim3(256), 0, p->stream, zh, uh, p->N, p->QPn, A, B, partials);
    return hipGetLastError();
}

