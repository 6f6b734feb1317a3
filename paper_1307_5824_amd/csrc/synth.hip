// Synthetic slices for benchmarks: translated, CTF-filtered Fourier slices of a
// sum of Gaussian blobs (closed form through the projection-slice theorem,
// eq. continuous_fps, with the paper's Fourier convention of section 2.2) plus
// complex white noise with the symmetry of a real image's DFT.
//
// phi(x) = sum_b a_b exp(-||x - c_b||^2 / (2 s_b^2)) has the transform
// sum_b a_b (2 pi s_b^2)^{3/2} exp(-s_b^2 ||w||^2 / 2) exp(-i <c_b, w>); at
// w = xi_{k,m} (||xi|| = ||omega_k||) the slice value is multiplied by
// h_m(||omega_k||) and by exp(-i <omega_k, s_m>) for an image shifted by s_m.
// Noise draws come from Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC 2011)
// keyed by the seed with counter (m, j, 0, 0), j the half-disk index.
#include <algorithm>
#include <cmath>

#include "firm_internal.h"
#include "philox.h"

extern "C" void firm_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    Philox4 c{{ctr[0], ctr[1], ctr[2], ctr[3]}};
    const Philox4 r = philox4x32_10(c, key[0], key[1]);
    for (int i = 0; i < 4; ++i) out[i] = r.v[i];
}

namespace {

constexpr int ST = 256;

struct SynthArgs {
    int N, M, P, B;
    const double* c12;
    const int32_t* group;
    const float* table;
    int Q;
    const double* shifts;
    const double* blobs;  // B x 5: c (3), sigma, a (2 pi sigma^2)^{3/2} (a for a point source)
    const int* rowstart;
    float2* b;
    double* partials;
    double snr_sigma;     // noise std per sample (pass 2)
    uint64_t seed;
};

__device__ __forceinline__ int find_row(const int* rowoff_lds, int N, int j) {
    // rows k1 = -N/2 .. N/2; rowoff_lds[r] = first disk index of row r
    int lo = 0, hi = N;  // answer in [0, N]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rowoff_lds[mid] <= j) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(ST) k_synth_clean(SynthArgs a) {
    __shared__ double bl[5 * 320];
    __shared__ int rowoff[260];
    __shared__ double red[ST / 64];
    const int N = a.N;
    for (int i = threadIdx.x; i < 5 * a.B; i += ST) bl[i] = a.blobs[i];
    for (int r = threadIdx.x; r <= N; r += ST) {
        const int k1 = r - N / 2;
        const int k2lo = -(int)floor(sqrt((double)(N * N / 4 - k1 * k1)) + 1e-9);
        rowoff[r] = a.rowstart[r] + k2lo;
    }
    __syncthreads();
    const int64_t total = (int64_t)a.M * a.P;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)ST + threadIdx.x; i < total; i += (int64_t)gridDim.x * ST) {
        const int m = (int)(i / a.P), j = (int)(i - (int64_t)m * a.P);
        const int r = find_row(rowoff, N, j);
        const int k1 = r - N / 2;
        const int k2 = j - a.rowstart[r];
        const double* c = a.c12 + 6 * (int64_t)m;
        const double w1 = 6.283185307179586 * k1 / N, w2 = 6.283185307179586 * k2 / N;
        const double xi0 = w1 * c[0] + w2 * c[3], xi1 = w1 * c[1] + w2 * c[4], xi2 = w1 * c[2] + w2 * c[5];
        const float om2 = (float)(w1 * w1 + w2 * w2);
        float re = 0.f, im = 0.f;
        for (int bb = 0; bb < a.B; ++bb) {
            const double* q = bl + 5 * bb;
            const float s = (float)q[3];
            const float amp = s > 0.f ? (float)q[4] * expf(-0.5f * s * s * om2) : (float)q[4];
            double th = -(q[0] * xi0 + q[1] * xi1 + q[2] * xi2);
            th -= 6.283185307179586 * rint(th * 0.15915494309189535);
            float sn, cs;
            sincosf((float)th, &sn, &cs);
            re += amp * cs;
            im += amp * sn;
        }
        const int g = a.group ? a.group[m] : 0;
        const float h = a.table ? a.table[(int64_t)g * a.Q + k1 * k1 + k2 * k2] : 1.f;
        float cs = 1.f, sn = 0.f;
        if (a.shifts) {
            double th = -(w1 * a.shifts[2 * (int64_t)m] + w2 * a.shifts[2 * (int64_t)m + 1]);
            th -= 6.283185307179586 * rint(th * 0.15915494309189535);
            sincosf((float)th, &sn, &cs);
        }
        const float br = h * (cs * re - sn * im), bi = h * (cs * im + sn * re);
        a.b[i] = make_float2(br, bi);
        acc += (double)br * br + (double)bi * bi;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) a.partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_synth_noise(SynthArgs a, const double* power, int nparts) {
    __shared__ double sig;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nparts; ++i) s += power[i];
        sig = sqrt(s / ((double)a.M * a.P) / a.snr_sigma);  // snr passed in snr_sigma
    }
    __syncthreads();
    const float sigma = (float)sig;
    const int64_t total = (int64_t)a.M * a.P;
    const int half = a.P / 2;  // centre index
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(i / a.P), j = (int)(i - (int64_t)m * a.P);
        const int jj = j < half ? j : a.P - 1 - j;
        Philox4 c{{(uint32_t)m, (uint32_t)jj, 0u, 0u}};
        const Philox4 r = philox4x32_10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
        const float u1 = ((float)r.v[0] + 0.5f) * 2.3283064365386963e-10f;
        const float u2 = ((float)r.v[1] + 0.5f) * 2.3283064365386963e-10f;
        const float rad = sqrtf(-2.f * logf(u1));
        float sn, cs;
        sincosf(6.283185307179586f * u2, &sn, &cs);
        float nr, ni;
        if (j == half) { nr = sigma * rad * cs; ni = 0.f; }
        else {
            nr = sigma * 0.70710678f * rad * cs;
            ni = sigma * 0.70710678f * rad * sn;
            if (j > half) ni = -ni;
        }
        float2 v = a.b[i];
        a.b[i] = make_float2(v.x + nr, v.y + ni);
    }
}

// standard normals: out[i] from Philox4x32-10 with counter (i mod 2^32, i / 2^32, offset, 1), Box-Muller
__global__ void k_normals(uint64_t seed, uint64_t offset, int64_t n, float* out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        Philox4 c{{(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)offset, 1u}};
        const Philox4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const float u1 = ((float)r.v[0] + 0.5f) * 2.3283064365386963e-10f;
        const float u2 = ((float)r.v[1] + 0.5f) * 2.3283064365386963e-10f;
        out[i] = sqrtf(-2.f * logf(u1)) * cosf(6.283185307179586f * u2);
    }
}

}  // namespace

hipError_t synth_normals(firm_plan p, uint64_t seed, uint64_t offset, int64_t n, float* out) {
    hipLaunchKernelGGL(k_normals, dim3(4096), dim3(256), 0, p->stream, seed, offset, n, out);
    return hipGetLastError();
}

hipError_t synth_slices(firm_plan p, int B, const double* blobs_dev, double snr, uint64_t seed, float2* b,
                        double* power_dev) {
    SynthArgs a;
    a.N = p->N; a.M = p->M; a.P = p->P; a.B = B;
    a.c12 = p->c12; a.group = p->group; a.table = p->table; a.Q = p->Q; a.shifts = p->shifts;
    a.blobs = blobs_dev; a.rowstart = p->rowstart; a.b = b; a.partials = power_dev;
    a.snr_sigma = snr; a.seed = seed;
    const int nblk = 2048;
    hipLaunchKernelGGL(k_synth_clean, dim3(nblk), dim3(ST), 0, p->stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (snr > 0 && std::isfinite(snr)) {
        hipLaunchKernelGGL(k_synth_noise, dim3(4096), dim3(256), 0, p->stream, a, (const double*)power_dev, nblk);
        e = hipGetLastError();
    }
    return e;
}

namespace {

// V(n) = sum_b a_b exp(-||n - c_b||^2 / (2 s_b^2)) on the N^3 grid, n = i - N/2 (section 3.1's volume
// sampling of the blob potential); blobs B x 5 as (c, s, a).
__global__ void __launch_bounds__(256) k_blob_volume(const double* __restrict__ blobs, int B, int N,
                                                     float* __restrict__ V) {
    __shared__ double bl[5 * 320];
    for (int i = threadIdx.x; i < 5 * B; i += 256) bl[i] = blobs[i];
    __syncthreads();
    const int64_t n = (int64_t)N * N * N;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double x = (double)(i / ((int64_t)N * N)) - N / 2, y = (double)((i / N) % N) - N / 2,
                     z = (double)(i % N) - N / 2;
        double v = 0.0;
        for (int b = 0; b < B; ++b) {
            const double dx = x - bl[5 * b], dy = y - bl[5 * b + 1], dz = z - bl[5 * b + 2], s = bl[5 * b + 3];
            v += bl[5 * b + 4] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * s * s));
        }
        V[i] = (float)v;
    }
}

}  // namespace

hipError_t synth_volume(firm_plan p, int B, const double* blobs_dev, float* V) {
    const int64_t n = (int64_t)p->N * p->N * p->N;
    hipLaunchKernelGGL(k_blob_volume, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0,
                       p->stream, blobs_dev, B, p->N, V);
    return hipGetLastError();
}
