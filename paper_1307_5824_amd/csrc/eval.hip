// Reconstruction accuracy (section 4): the Fourier shell correlation of two volumes,
//   FSC(i) = sum_{j in Shell_i} F(V1)(j) conj F(V2)(j) / sqrt(sum |F(V1)|^2 sum |F(V2)|^2),
// Shell_i = {j : 0.5 + (i-1) + eps <= ||j|| < 0.5 + i + eps}, eps = 1e-4, i = 1 .. N/2 - 1, and the
// modified form restricted to the frequencies outside or inside a missing cone about the third
// axis (the cone a random conical tilt series leaves unsampled: half-angle 90 degrees minus the
// tilt).  Against the true volume the FSC is the Fourier cross-resolution.
//
// Both volumes are transformed by the N^3 real-to-half-spectrum FFT; the half spectrum holds q3 in
// [0, N/2], and the other half follows from F(-j) = conj F(j), whose terms equal those of j (and lie
// in the same shell and cone region), so the columns q3 in (0, N/2) count twice.  The centring
// phase (-1)^(q1+q2+q3) of the uncentred transform cancels in every term.
#include <algorithm>
#include <cmath>

#include "firm_internal.h"

namespace {

constexpr int FSC_SHELLS = 128;  // N / 2 at N = 256

// per (region, shell) sums of Re(F1 conj F2), |F1|^2, |F2|^2; regions: all, outside, inside
__global__ void __launch_bounds__(256) k_fsc_sums(const float2* __restrict__ h1, const float2* __restrict__ h2, int N,
                                                  int QPn, double cos_cone, double* __restrict__ sums) {
    __shared__ double acc[3 * 3 * FSC_SHELLS];
    for (int i = threadIdx.x; i < 9 * FSC_SHELLS; i += 256) acc[i] = 0.0;
    __syncthreads();
    const int H = N / 2 + 1;
    const int64_t n = (int64_t)N * N * H;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int q1 = (int)(e / ((int64_t)N * H)), q2 = (int)((e / H) % N), q3 = (int)(e % H);
        const int j1 = q1 < N / 2 ? q1 : q1 - N, j2 = q2 < N / 2 ? q2 : q2 - N, j3 = q3;
        const double r = sqrt((double)j1 * j1 + (double)j2 * j2 + (double)j3 * j3);
        const int shell = (int)floor(r - 0.5 - 1e-4) + 1;
        if (r < 0.5 + 1e-4 || shell < 1 || shell > N / 2 - 1) continue;
        const float2 a = h1[((int64_t)q1 * N + q2) * QPn + q3], b = h2[((int64_t)q1 * N + q2) * QPn + q3];
        const double w = (q3 == 0 || q3 == N / 2) ? 1.0 : 2.0;
        const double x = w * ((double)a.x * b.x + (double)a.y * b.y);
        const double p1 = w * ((double)a.x * a.x + (double)a.y * a.y), p2 = w * ((double)b.x * b.x + (double)b.y * b.y);
        const int region = fabs((double)j3) > r * cos_cone ? 2 : 1;  // inside the cone: angle to the axis < half-angle
        for (int k = 0; k < 2; ++k) {
            double* s = acc + 3 * (k == 0 ? 0 : region) * FSC_SHELLS + shell;
            atomicAdd(s, x);
            atomicAdd(s + FSC_SHELLS, p1);
            atomicAdd(s + 2 * FSC_SHELLS, p2);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 9 * FSC_SHELLS; i += 256)
        if (acc[i] != 0.0) atomicAdd(&sums[i], acc[i]);
}

}  // namespace

hipError_t fsc_sums(firm_plan p, const float* V1, const float* V2, double cone_deg, double* sums_dev) {
    if (p->N / 2 > FSC_SHELLS) return hipErrorInvalidValue;
    hipError_t e = fill_zero(sums_dev, 9 * FSC_SHELLS * sizeof(double), p->stream);
    if (e != hipSuccess) return e;
    e = fft_forward_r2c(p, V1, p->S1);
    if (e != hipSuccess) return e;
    e = fft_forward_r2c(p, V2, p->S2);
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)p->N * p->N * (p->N / 2 + 1);
    const double cos_cone = cos(cone_deg * M_PI / 180.0);
    hipLaunchKernelGGL(k_fsc_sums, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 2048)), dim3(256), 0, p->stream,
                       p->S1, p->S2, p->N, p->QPn, cos_cone, sums_dev);
    return hipGetLastError();
}

int fsc_max_shells() { return FSC_SHELLS; }
