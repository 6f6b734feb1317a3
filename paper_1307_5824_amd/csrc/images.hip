// Step 1 of the algorithm (section 3.4): Fourier slices from real-space images, and a
// real-space image generator for synthetic data.
//
// Slices.  An image J_m on the pixel grid x in [-N/2, N/2)^2 (pixel i at x = i - N/2) gives
// b(k, m) = sum_x J_m(x) exp(-2 pi i <k, x> / N) (the centred DFT of section 2.2) at the disk
// points ||k|| <= N/2.  The FFT passes transform the array index i, so b(k) = (-1)^(k1 + k2)
// X(k mod N); the real rows keep q2 in [0, N/2] and X(-q) = conj X(q) supplies the rest.  The
// disk's boundary points k_d = +N/2 take the periodic value X(N/2), equal to X(-N/2).
//
// Images.  A Gaussian blob a exp(-||x - c||^2 / (2 s^2)) projects along the viewing direction
// (third row of R_m) to the 2D Gaussian a sqrt(2 pi) s exp(-||x - p||^2 / (2 s^2)) centred at
// p = ((R_m c)_1, (R_m c)_2); an image of a particle off-centre by s_m is J(x - s_m), so p moves
// by s_m (the back-projection undoes this by its re-centring phase).  Blobs farther than
// PROJ_CUT sigmas from a pixel row are skipped (their weight is below exp(-PROJ_CUT^2 / 2)).
// Pixel noise: N(0, sigma^2) per pixel from Philox4x32-10 keyed by the seed, counter
// (m, pixel, 0, 2), sigma^2 = mean clean pixel power / SNR.
#include <cmath>

#include "firm_internal.h"
#include "philox.h"

#define IMG_THREADS 256
#define IMG_MAXB 320
#define PROJ_CUT 9.0f

namespace {

// One image row of one disk row per block: block (g, r) writes the points (k1, k2) of row
// r = k1 + N/2 of image g of the batch.
__global__ void __launch_bounds__(IMG_THREADS) k_img_gather(const float2* __restrict__ spec, int N, int QPn, int P,
                                                           const int* __restrict__ rowstart, int m0,
                                                           float2* __restrict__ b) {
    const int r = blockIdx.x % (N + 1), g = blockIdx.x / (N + 1);
    const int k1 = r - N / 2;
    const int kmax = (int)floor(sqrt((double)(N * N / 4 - k1 * k1)) + 1e-9);
    const float2* X = spec + (int64_t)g * N * QPn;
    const int q1 = (k1 + N) % N, q1m = (N - q1) % N;
    float2* out = b + (int64_t)(m0 + g) * P + rowstart[r];
    for (int k2 = -kmax + (int)threadIdx.x; k2 <= kmax; k2 += IMG_THREADS) {
        float2 v = k2 >= 0 ? X[(int64_t)q1 * QPn + k2] : X[(int64_t)q1m * QPn - k2];
        if (k2 < 0) v.y = -v.y;
        if ((k1 + k2) & 1) { v.x = -v.x; v.y = -v.y; }
        out[k2] = v;
    }
}

struct ImgArgs {
    int N, M, B;
    const double* c12;     // rows 1 and 2 of R_m
    const double* shifts;  // M x 2 or null
    const double* blobs;   // B x 5: c (3), sigma, a sqrt(2 pi) sigma
    float* img;
    double* partials;      // per-block clean power
    double snr;
    uint64_t seed;
};

// Clean images: block (m, row band); the blob list of each row is rebuilt in LDS with the
// row factor w exp(-(x1 - p1)^2 / (2 s^2)) folded in.
constexpr int IMG_ROWS = 8;

__global__ void __launch_bounds__(IMG_THREADS) k_synth_images(ImgArgs a) {
    __shared__ float bp1[IMG_MAXB], bp2[IMG_MAXB], binv[IMG_MAXB], bw[IMG_MAXB], bcut[IMG_MAXB];
    __shared__ float lp2[IMG_MAXB], linv[IMG_MAXB], lw[IMG_MAXB], lcut[IMG_MAXB];
    __shared__ int ln;
    __shared__ double red[IMG_THREADS / 64];
    const int N = a.N;
    const int bands = (N + IMG_ROWS - 1) / IMG_ROWS;
    const int m = blockIdx.x / bands, band = blockIdx.x % bands;
    const double* c = a.c12 + 6 * (int64_t)m;
    const double s1 = a.shifts ? a.shifts[2 * (int64_t)m] : 0.0, s2 = a.shifts ? a.shifts[2 * (int64_t)m + 1] : 0.0;
    for (int i = threadIdx.x; i < a.B; i += IMG_THREADS) {
        const double* q = a.blobs + 5 * i;
        const double s = q[3];
        bp1[i] = (float)(c[0] * q[0] + c[1] * q[1] + c[2] * q[2] + s1);
        bp2[i] = (float)(c[3] * q[0] + c[4] * q[1] + c[5] * q[2] + s2);
        binv[i] = (float)(0.5 / (s * s));
        bw[i] = (float)q[4];
        bcut[i] = PROJ_CUT * (float)s;
    }
    double acc = 0.0;
    for (int rr = 0; rr < IMG_ROWS; ++rr) {
        const int i1 = band * IMG_ROWS + rr;
        if (i1 >= N) break;  // uniform
        __syncthreads();
        if (threadIdx.x == 0) ln = 0;
        __syncthreads();
        const float x1 = (float)(i1 - N / 2);
        for (int i = threadIdx.x; i < a.B; i += IMG_THREADS) {
            const float d = x1 - bp1[i];
            if (fabsf(d) <= bcut[i]) {
                const int k = atomicAdd(&ln, 1);
                lp2[k] = bp2[i];
                linv[k] = binv[i];
                lw[k] = bw[i] * expf(-d * d * binv[i]);
                lcut[k] = bcut[i];
            }
        }
        __syncthreads();
        const int n = ln;
        float* row = a.img + ((int64_t)m * N + i1) * N;
        for (int i2 = threadIdx.x; i2 < N; i2 += IMG_THREADS) {
            const float x2 = (float)(i2 - N / 2);
            float v = 0.f;
            for (int k = 0; k < n; ++k) {
                const float d = x2 - lp2[k];
                if (fabsf(d) <= lcut[k]) v = fmaf(lw[k], expf(-d * d * linv[k]), v);
            }
            row[i2] = v;
            acc += (double)v * v;
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) a.partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Per-block sums of the block partials (grid-stride over the partials), then one block totals.
__global__ void __launch_bounds__(256) k_sum(const double* __restrict__ in, int64_t n, double* __restrict__ out) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) acc += in[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(256) k_img_noise(ImgArgs a, const double* __restrict__ power) {
    const int N = a.N;
    const int64_t per = (int64_t)N * N, total = (int64_t)a.M * per;
    const float sigma = (float)sqrt(power[0] / (double)total / a.snr);
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int m = (int)(i / per);
        const uint32_t pix = (uint32_t)(i - (int64_t)m * per);
        const Philox4 r = philox4x32_10(Philox4{{(uint32_t)m, pix, 0u, 2u}}, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
        a.img[i] += sigma * philox_normal(r);
    }
}

}  // namespace

int64_t synth_images_scratch(int N, int M) { return (int64_t)M * ((N + IMG_ROWS - 1) / IMG_ROWS) + 1025; }

// b rows m0 .. m0 + G - 1 from the half spectra of G images.
hipError_t images_gather(firm_plan p, const float2* spec, int G, int m0, float2* b) {
    const int64_t blocks = (int64_t)G * (p->N + 1);
    hipLaunchKernelGGL(k_img_gather, dim3((unsigned)blocks), dim3(IMG_THREADS), 0, p->stream, spec, p->N, p->QPn, p->P,
                       p->rowstart, m0, b);
    return hipGetLastError();
}

// blobs_dev: B x 5 doubles (c, sigma, a sqrt(2 pi) sigma); partials: npart >= synth_images_scratch
// doubles of device scratch.
hipError_t synth_images(firm_plan p, int B, const double* blobs_dev, double snr, uint64_t seed, float* img,
                        double* partials, int64_t npart) {
    const int N = p->N;
    const int64_t blocks = (int64_t)p->M * ((N + IMG_ROWS - 1) / IMG_ROWS);
    if (B > IMG_MAXB || blocks + 1025 > npart) return hipErrorInvalidValue;
    ImgArgs a;
    a.N = N; a.M = p->M; a.B = B; a.c12 = p->c12; a.shifts = p->shifts; a.blobs = blobs_dev; a.img = img;
    a.partials = partials; a.snr = snr; a.seed = seed;
    hipLaunchKernelGGL(k_synth_images, dim3((unsigned)blocks), dim3(IMG_THREADS), 0, p->stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !(snr > 0) || !std::isfinite(snr)) return e;
    double* mid = partials + blocks;
    hipLaunchKernelGGL(k_sum, dim3(1024), dim3(256), 0, p->stream, partials, blocks, mid);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, p->stream, mid, (int64_t)1024, mid + 1024);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_img_noise, dim3(4096), dim3(256), 0, p->stream, a, (const double*)(mid + 1024));
    return hipGetLastError();
}
