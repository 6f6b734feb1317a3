// Learned Fourier-diagonal preconditioner: a 3D conv net on the g^3 pooled log kernel
// spectrum (g a power of two >= 32; 32 in training, larger grids at inference: the network is
// fully convolutional), its training, and the kernels that turn its output into the diagonal d
// of z = F^{-1}(d . F r) (circulant diagonalisation, section 2.3, eq. circ1).
//
// Network (C channels, circular padding, cross-correlation with 3^3 filters):
//   o = c4(relu(c3(relu(c2(relu(c1(f)))))))
// The diagonal is d = 1 / (t + Ker(0) exp(U sym(o))) with t the Fourier diagonal of A*A + lambda
// (T. Chan's circulant spectrum): the network learns a floor under the analytic spectrum.
// Layers c2, c3 (C -> C) are implicit GEMMs on the matrix cores: one wavefront computes a
// 32-voxel row segment x 32 output channels tile with v_mfma_f32_32x32x16_bf16 (BF16 operands, FP32
// accumulation), K = 27 taps x C input channels; forward and backward-data share the kernel
// (the backward uses the transposed weights and the mirrored taps); their weight gradients are
// GEMMs over the voxels on the same instruction.  c1, c4, their weight gradients and Adam run on
// the vector ALUs in FP32.  Activations are channel-last
// [batch][voxel][C], stored in FP32 and as BF16 copies for the matrix cores.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "firm_internal.h"

// Scratch of firm_precond_from_output_noalloc: the symmetrised network output on grids up to
// 128^3 (8 MiB on every GPU the library runs on, held until the process ends).  In host code this
// name is a host-side stand-in: kernels receive the device address from hipGetSymbolAddress.
constexpr int NOALLOC_MAX_RES = 128;
static __device__ __align__(256) float scratch[NOALLOC_MAX_RES * NOALLOC_MAX_RES * NOALLOC_MAX_RES];

namespace {

constexpr int CH = 32;           // channels
constexpr int G0 = 32;           // coarse grid of training (and the smallest)

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef float f16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int wrapg(int i, int g) { return i & (g - 1); }
__device__ __forceinline__ int vox(int a, int b, int c, int g) {
    return (wrapg(a, g) * g + wrapg(b, g)) * g + wrapg(c, g);
}

// ------------------------------------------------------------------ weights --

// masters w[co][ci][27] (tap = 9 a + 3 b + c, offset (a-1, b-1, c-1)) -> BF16 layouts
// fwd[tap][co][ci] and bwd[tap][ci][co]
__global__ void k_pack_weights(const float* __restrict__ w, __bf16* __restrict__ fwd, __bf16* __restrict__ bwd) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 27 * CH * CH; i += gridDim.x * blockDim.x) {
        const int tap = i % 27, ci = (i / 27) % CH, co = i / (27 * CH);
        const __bf16 v = (__bf16)w[i];
        fwd[(tap * CH + co) * CH + ci] = v;
        bwd[(tap * CH + ci) * CH + co] = v;
    }
}

// ------------------------------------------------------------------ layer 1 --

// h1[b][v][co] = relu(b1[co] + sum_tap w1[co][tap] f[b][v + off(tap)])
__global__ void __launch_bounds__(256) k_conv_first(const float* __restrict__ f, const float* __restrict__ w1,
                                                    const float* __restrict__ b1, float* __restrict__ h,
                                                    __bf16* __restrict__ hb, int B, int g) {
    __shared__ float ws[CH * 27], bs[CH];
    for (int i = threadIdx.x; i < CH * 27; i += 256) ws[i] = w1[i];
    if (threadIdx.x < CH) bs[threadIdx.x] = b1[threadIdx.x];
    __syncthreads();
    const int64_t GV = (int64_t)g * g * g, n = (int64_t)B * GV;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int b = (int)(i / GV), v = (int)(i % GV);
        const int v1 = v / (g * g), v2 = (v / g) % g, v3 = v % g;
        float nb[27];
#pragma unroll
        for (int t = 0; t < 27; ++t)
            nb[t] = f[(int64_t)b * GV + vox(v1 + t / 9 - 1, v2 + (t / 3) % 3 - 1, v3 + t % 3 - 1, g)];
        for (int co = 0; co < CH; ++co) {
            float z = bs[co];
#pragma unroll
            for (int t = 0; t < 27; ++t) z = fmaf(ws[co * 27 + t], nb[t], z);
            z = fmaxf(z, 0.f);
            h[i * CH + co] = z;
            hb[i * CH + co] = (__bf16)z;
        }
    }
}

// ------------------------------------------------------------- MFMA layers --

// One wavefront: 32 voxels of a row (b, v1, v2, 32 s .. 32 s + 31) x 32 output channels.
//   out[v][n] = sum_tap sum_k x[v + sgn * off(tap)][k] W[tap][n][k]
// FWD: + bias, relu, store FP32 and BF16.   BWD: multiply by (hprev > 0), store FP32 and BF16.
// Operand layout of v_mfma_f32_32x32x16_bf16 (lane l, element t):
//   A[i][k]: i = l % 32, k = 8 (l / 32) + t;  B[k][j]: j = l % 32, k = 8 (l / 32) + t;
//   D[i][j] (16 values): j = l % 32, i = 8 (t / 4) + 4 (l / 32) + t % 4.
template <bool FWD>
__global__ void __launch_bounds__(256) k_conv_mfma(const __bf16* __restrict__ x, const __bf16* __restrict__ W,
                                                   const float* __restrict__ bias, const float* __restrict__ hprev,
                                                   float* __restrict__ out, __bf16* __restrict__ outb, int B,
                                                   int g) {
    __shared__ bf8_t wl[27 * CH * CH / 8];  // 55,296 B
    const bf8_t* W8 = reinterpret_cast<const bf8_t*>(W);
    for (int i = threadIdx.x; i < 27 * CH * CH / 8; i += 256) wl[i] = W8[i];
    __syncthreads();
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int segs = g / 32;
    const int row = blockIdx.x * 4 + wave;  // (b, v1, v2, segment)
    if (row >= B * g * g * segs) return;
    const int seg = row % segs, r2 = row / segs;
    const int b = r2 / (g * g), v1 = (r2 / g) % g, v2 = r2 % g, s0 = 32 * seg;
    const int i = l & 31, kb = l >> 5;
    const int sgn = FWD ? 1 : -1;
    f16_t acc = {};
    const int64_t GV = (int64_t)g * g * g;
    const __bf16* xb = x + (int64_t)b * GV * CH;
#pragma unroll 1
    for (int tap = 0; tap < 27; ++tap) {
        const int da = sgn * (tap / 9 - 1), db = sgn * ((tap / 3) % 3 - 1), dc = sgn * (tap % 3 - 1);
        const int src = vox(v1 + da, v2 + db, s0 + i + dc, g);
#pragma unroll
        for (int c0 = 0; c0 < CH; c0 += 16) {
            const bf8_t a = *reinterpret_cast<const bf8_t*>(xb + (int64_t)src * CH + c0 + 8 * kb);
            const bf8_t w = wl[((tap * CH + i) * CH + c0 + 8 * kb) / 8];
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, w, acc, 0, 0, 0);
        }
    }
    const int j = l & 31;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int vi = 8 * (t / 4) + 4 * kb + (t % 4);
        const int64_t o = ((int64_t)b * GV + ((int64_t)v1 * g + v2) * g + s0 + vi) * CH + j;
        float z = acc[t];
        if (FWD) z = fmaxf(z + bias[j], 0.f);
        else z = hprev[o] > 0.f ? z : 0.f;
        out[o] = z;
        outb[o] = (__bf16)z;
    }
}

// ------------------------------------------------------------------ layer 4 --

// o[b][v] = b4 + sum_tap sum_ci w4[ci][tap] h3[b][v + off][ci]
__global__ void __launch_bounds__(256) k_conv_last(const float* __restrict__ h, const float* __restrict__ w4,
                                                   const float* __restrict__ b4, float* __restrict__ o, int B,
                                                   int g) {
    __shared__ float ws[CH * 27];
    for (int i = threadIdx.x; i < CH * 27; i += 256) ws[i] = w4[i];
    __syncthreads();
    const int64_t GV = (int64_t)g * g * g, n = (int64_t)B * GV;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int b = (int)(i / GV), v = (int)(i % GV);
        const int v1 = v / (g * g), v2 = (v / g) % g, v3 = v % g;
        float z = b4[0];
        for (int t = 0; t < 27; ++t) {
            const float* hn =
                h + ((int64_t)b * GV + vox(v1 + t / 9 - 1, v2 + (t / 3) % 3 - 1, v3 + t % 3 - 1, g)) * CH;
#pragma unroll 8
            for (int ci = 0; ci < CH; ++ci) z = fmaf(ws[ci * 27 + t], hn[ci], z);
        }
        o[i] = z;
    }
}

// gz3[b][v][ci] = (h3 > 0) sum_tap w4[ci][tap] go[b][v - off(tap)]
__global__ void __launch_bounds__(256) k_conv_last_bwd(const float* __restrict__ go, const float* __restrict__ w4,
                                                       const float* __restrict__ h3, float* __restrict__ gz,
                                                       __bf16* __restrict__ gzb, int B, int g) {
    __shared__ float ws[CH * 27];
    for (int i = threadIdx.x; i < CH * 27; i += 256) ws[i] = w4[i];
    __syncthreads();
    const int64_t GV = (int64_t)g * g * g, n = (int64_t)B * GV;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int b = (int)(i / GV), v = (int)(i % GV);
        const int v1 = v / (g * g), v2 = (v / g) % g, v3 = v % g;
        float gt[27];
#pragma unroll
        for (int t = 0; t < 27; ++t)
            gt[t] = go[(int64_t)b * GV + vox(v1 - (t / 9 - 1), v2 - ((t / 3) % 3 - 1), v3 - (t % 3 - 1), g)];
        for (int ci = 0; ci < CH; ++ci) {
            float s = 0.f;
#pragma unroll
            for (int t = 0; t < 27; ++t) s = fmaf(ws[ci * 27 + t], gt[t], s);
            const float r = h3[i * CH + ci] > 0.f ? s : 0.f;
            gz[i * CH + ci] = r;
            gzb[i * CH + ci] = (__bf16)r;
        }
    }
}

// ---------------------------------------------------------------- gradients --

// dW[co][ci][tap] += sum_{b,v in chunk} gz[b][v][co] x[b][v + off(tap)][ci] (x channel-last, CI channels),
// db[co] += sum gz (tap 0 blocks only).  Block: one tap, one chunk of voxels; thread = (co, ci).
template <int CI>
__global__ void __launch_bounds__(CH * CI) k_wgrad(const float* __restrict__ gz, const float* __restrict__ x,
                                                   float* __restrict__ dw, float* __restrict__ db, int B,
                                                   int chunk, int g) {
    const int tap = blockIdx.y;
    const int co = threadIdx.x / CI, ci = threadIdx.x % CI;
    const int64_t v0 = (int64_t)blockIdx.x * chunk;
    const int64_t GV = (int64_t)g * g * g, n = (int64_t)B * GV;
    const int da = tap / 9 - 1, dbb = (tap / 3) % 3 - 1, dc = tap % 3 - 1;
    float acc = 0.f, accb = 0.f;
    for (int64_t i = v0; i < v0 + chunk && i < n; ++i) {
        const int b = (int)(i / GV), v = (int)(i % GV);
        const int v1 = v / (g * g), v2 = (v / g) % g, v3 = v % g;
        const float gv = gz[i * CH + co];
        acc = fmaf(gv, x[((int64_t)b * GV + vox(v1 + da, v2 + dbb, v3 + dc, g)) * CI + ci], acc);
        accb += gv;
    }
    unsafeAtomicAdd(&dw[(co * CI + ci) * 27 + tap], acc);
    if (tap == 0 && ci == 0) unsafeAtomicAdd(&db[co], accb);
}

// Weight gradients of the C -> C layers on the matrix cores: for every tap a GEMM over the voxels,
//   dW[co][ci][tap] += sum_v gz[b][v][co] x[b][v + off(tap)][ci],   db[co] += sum_v gz[b][v][co],
// with the BF16 copies of gz and x that the layers' MFMA passes use (FP32 accumulation).
// Block: 9 wavefronts; wavefront w takes the neighbour row (da, db) = (w / 3 - 1, w % 3 - 1) and
// its three taps 3 w + c (dc = c - 1), one 32 x 32 accumulator each (A[i][k] = gz[k][co = i],
// B[k][j] = x[k + off][ci = j], K = voxels, 16 per instruction).  The block walks its rows
// (b, v1, v2, 32-voxel segment); per row, gz's 32 voxels and each wavefront's neighbour row with
// one voxel of halo at either end (periodic) are staged in LDS in their global [voxel][channel]
// layout, and the operands gather 8 voxels of one channel.  The next row's global loads are
// issued before the current row's products, so that their latency overlaps them.
constexpr int WG_WAVES = 9;
constexpr int WG_XCH = 34 * CH / 8;  // 16-byte chunks of a neighbour row with its halo

__global__ void __launch_bounds__(64 * WG_WAVES) k_wgrad_mfma(const __bf16* __restrict__ gz,
                                                             const __bf16* __restrict__ x, float* __restrict__ dw,
                                                             float* __restrict__ db, int B, int g,
                                                             int rows_per_block) {
    __shared__ bf8_t gzs[32 * CH / 8];             // [voxel][channel], 2 KB
    __shared__ bf8_t xs[WG_WAVES][WG_XCH];         // [wave][halo voxel p][channel], 19.1 KB
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int da = wave / 3 - 1, dbb = wave % 3 - 1;
    const int segs = g / 32;
    const int64_t rows = (int64_t)B * g * g * segs;
    const int64_t GV = (int64_t)g * g * g;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
    // this thread's staging chunks of a row: gz chunk threadIdx.x (< 128), halo chunks l + 64 q
    bf8_t pg = {}, px[3] = {};
    auto fetch = [&](int64_t row) {
        const int seg = (int)(row % segs);
        const int64_t r2 = row / segs;
        const int b = (int)(r2 / ((int64_t)g * g)), v1 = (int)((r2 / g) % g), v2 = (int)(r2 % g), s0 = 32 * seg;
        const __bf16* xb = x + (int64_t)b * GV * CH;
        if (threadIdx.x < 32 * CH / 8) {
            const int v = threadIdx.x / (CH / 8), c8 = threadIdx.x % (CH / 8);
            pg = *reinterpret_cast<const bf8_t*>(gz + ((int64_t)b * GV + ((int64_t)v1 * g + v2) * g + s0 + v) * CH +
                                                 8 * c8);
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int c = l + 64 * q;
            if (c < WG_XCH) {
                const int p = c / (CH / 8), c8 = c % (CH / 8);
                px[q] = *reinterpret_cast<const bf8_t*>(xb + (int64_t)vox(v1 + da, v2 + dbb, s0 - 1 + p, g) * CH +
                                                        8 * c8);
            }
        }
    };
    f16_t acc0 = {}, acc1 = {}, acc2 = {};
    float accb = 0.f;
    const int i = l & 31, kb = l >> 5;
    const __bf16* gzl = reinterpret_cast<const __bf16*>(gzs);
    const __bf16* xl = reinterpret_cast<const __bf16*>(xs[wave]);
    if (r0 < r1) fetch(r0);
    for (int64_t row = r0; row < r1; ++row) {
        __syncthreads();  // every wavefront has read the previous row's operands
        if (threadIdx.x < 32 * CH / 8) gzs[threadIdx.x] = pg;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if (l + 64 * q < WG_XCH) xs[wave][l + 64 * q] = px[q];
        __syncthreads();
        if (row + 1 < r1) fetch(row + 1);
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int k0 = 16 * kk + 8 * kb;
            bf8_t a;
            __bf16 xv[10];  // voxels k0 .. k0 + 9 of the halo row: the three taps' operands overlap
#pragma unroll
            for (int t = 0; t < 8; ++t) a[t] = gzl[(k0 + t) * CH + i];
#pragma unroll
            for (int t = 0; t < 10; ++t) xv[t] = xl[(k0 + t) * CH + i];
            bf8_t b0, b1, b2;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                b0[t] = xv[t];
                b1[t] = xv[t + 1];
                b2[t] = xv[t + 2];
            }
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc1, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b2, acc2, 0, 0, 0);
        }
        if (wave == 0 && l < CH)
            for (int v = 0; v < 32; ++v) accb += (float)gzl[v * CH + l];
    }
    // D[i][j]: j = l % 32 (ci), i = 8 (t / 4) + 4 (l / 32) + t % 4 (co)
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int co = 8 * (t / 4) + 4 * kb + (t % 4);
        float* d = dw + (co * CH + i) * 27 + 3 * wave;
        unsafeAtomicAdd(d, acc0[t]);
        unsafeAtomicAdd(d + 1, acc1[t]);
        unsafeAtomicAdd(d + 2, acc2[t]);
    }
    if (wave == 0 && l < CH) unsafeAtomicAdd(&db[l], accb);
}

// dW4[ci][tap] = sum go[b][v] h3[b][v + off][ci]; db4 = sum go.  Block: one tap, chunk; thread = ci.
__global__ void __launch_bounds__(256) k_wgrad_last(const float* __restrict__ go, const float* __restrict__ h3,
                                                    float* __restrict__ dw, float* __restrict__ db, int B,
                                                    int chunk, int g) {
    const int tap = blockIdx.y;
    const int ci = threadIdx.x % CH, part = threadIdx.x / CH;  // 8 parts of the chunk
    const int64_t GV = (int64_t)g * g * g, n = (int64_t)B * GV;
    const int da = tap / 9 - 1, dbb = (tap / 3) % 3 - 1, dc = tap % 3 - 1;
    float acc = 0.f, accb = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * chunk + part; i < (int64_t)(blockIdx.x + 1) * chunk && i < n; i += 8) {
        const int b = (int)(i / GV), v = (int)(i % GV);
        const int v1 = v / (g * g), v2 = (v / g) % g, v3 = v % g;
        const float gv = go[i];
        acc = fmaf(gv, h3[((int64_t)b * GV + vox(v1 + da, v2 + dbb, v3 + dc, g)) * CH + ci], acc);
        accb += gv;
    }
    unsafeAtomicAdd(&dw[ci * 27 + tap], acc);
    if (tap == 0 && ci == 0) unsafeAtomicAdd(&db[0], accb);
}

// Adam on FP32 masters (Kingma & Ba 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr mhat / (sqrt(vhat) + eps); gradients scaled by gscale.  The last parameter (the output
// bias: the log of the floor's level) steps at lr_last.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float lr_last, float b1, float b2, float eps, float c1,
                       float c2, float gscale) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float rate = i == n - 1 ? lr_last : lr;
        const float gi = g[i] * gscale;
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= rate * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// ------------------------------------------------------- diagonal and loss --

__device__ __forceinline__ int flipg(int u, int g) { return (g - u) & (g - 1); }  // centred index of -u

// s = (o(u) + o(-u)) / 2 on the centred g^3 grid (index u + g/2 -> flipped (g - idx) % g)
__global__ void k_symmetrise(const float* __restrict__ o, float* __restrict__ s, int B, int g) {
    const int64_t GV = (int64_t)g * g * g, n = (int64_t)B * GV;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i / GV), v = (int)(i % GV);
        const int v1 = v / (g * g), v2 = (v / g) % g, v3 = v % g;
        s[i] = 0.5f * (o[i] + o[(int64_t)b * GV + ((int64_t)flipg(v1, g) * g + flipg(v2, g)) * g + flipg(v3, g)]);
    }
}

// periodic linear interpolation weights of fine centred index q on the coarse grid
__device__ __forceinline__ void interp(int i, int N, int g, int& c0, int& c1, float& t) {
    const float u = (float)(i - N / 2) * ((float)g / (float)N);
    const float fl = floorf(u);
    t = u - fl;
    const int lo = (int)fl;
    c0 = wrapg(lo + g / 2, g);
    c1 = wrapg(lo + 1 + g / 2, g);
}

__device__ __forceinline__ float upsample_at(const float* s, int i1, int i2, int i3, int N, int g) {
    int a0, a1, b0, b1, e0, e1;
    float ta, tb, te;
    interp(i1, N, g, a0, a1, ta);
    interp(i2, N, g, b0, b1, tb);
    interp(i3, N, g, e0, e1, te);
    auto S = [&](int a, int b, int e) { return s[((int64_t)a * g + b) * g + e]; };
    const float x00 = S(a0, b0, e0) * (1 - te) + S(a0, b0, e1) * te;
    const float x01 = S(a0, b1, e0) * (1 - te) + S(a0, b1, e1) * te;
    const float x10 = S(a1, b0, e0) * (1 - te) + S(a1, b0, e1) * te;
    const float x11 = S(a1, b1, e0) * (1 - te) + S(a1, b1, e1) * te;
    return (x00 * (1 - tb) + x01 * tb) * (1 - ta) + (x10 * (1 - tb) + x11 * tb) * ta;
}

// floor mu = exp(U s) and diagonal d = 1 / (t + ker0 mu) at fine index (i1, i2, i3)
__device__ __forceinline__ float floor_diag(const float* s, const float* t, int64_t i, int N, int g, float ker0,
                                            float& mu) {
    const int i1 = (int)(i / ((int64_t)N * N)), i2 = (int)((i / N) % N), i3 = (int)(i % N);
    mu = expf(upsample_at(s, i1, i2, i3, N, g));
    return 1.f / (t[i] + ker0 * mu);
}

// d = 1 / (t + ker0 exp(U s)) on the centred N^3 grid
__global__ void k_diag_from_s(const float* __restrict__ s, const float* __restrict__ t, float* __restrict__ d, int N,
                              int g, float ker0) {
    const int64_t n = (int64_t)N * N * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float mu;
        d[i] = floor_diag(s, t, i, N, g, ker0, mu);
    }
}

// Every objective's gradient with respect to log d is mapped to U s by
// d log d / d (U s) = -ker0 mu d (log d = -log(t + ker0 exp(U s))).

// probe objective: loss partial sums (d^2 A - 2 d B) (+ C added on the host) and
// gr = dL/d(U s), with dL/dlog d = (2 d A - 2 B) d / sumC
__global__ void __launch_bounds__(256) k_loss_grad(const float* __restrict__ s, const float* __restrict__ t,
                                                   const float* __restrict__ A, const float* __restrict__ Bs,
                                                   float* __restrict__ gr, int N, int g, float ker0, float inv_sumc,
                                                   double* partials) {
    __shared__ double red[4];
    const int64_t n = (int64_t)N * N * N;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float mu;
        const float d = floor_diag(s, t, i, N, g, ker0, mu);
        const float a = A[i], bb = Bs[i];
        acc += (double)d * d * a - 2.0 * (double)d * bb;
        gr[i] = (2.f * d * a - 2.f * bb) * d * inv_sumc * (-ker0 * mu * d);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Kaporin objective, pass 1: block partials of sum d t and sum log(d t)
__global__ void __launch_bounds__(256) k_kap_sums(const float* __restrict__ s, const float* __restrict__ t, int N,
                                                  int g, float ker0, double* partials, int nblk) {
    __shared__ double red[8];
    const int64_t n = (int64_t)N * N * N;
    double a1 = 0.0, a2 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float mu;
        const double dt = (double)floor_diag(s, t, i, N, g, ker0, mu) * t[i];
        a1 += dt;
        a2 += log(dt);
    }
    for (int o = 32; o > 0; o >>= 1) {
        a1 += __shfl_down(a1, o, 64);
        a2 += __shfl_down(a2, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = a1;
        red[4 + (threadIdx.x >> 6)] = a2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
        partials[nblk + blockIdx.x] = red[4] + red[5] + red[6] + red[7];
    }
}

// Kaporin objective, pass 2: dL/dlog d = d t / sum(d t) - 1 / n, mapped to U s
__global__ void k_kap_grad(const float* __restrict__ s, const float* __restrict__ t, float* __restrict__ gr, int N,
                           int g, float ker0, double inv_sum, double inv_n) {
    const int64_t n = (int64_t)N * N * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float mu;
        const float d = floor_diag(s, t, i, N, g, ker0, mu);
        const double dt = (double)d * t[i];
        gr[i] = (float)(dt * inv_sum - inv_n) * (-ker0 * mu * d);
    }
}

// a given gradient with respect to log d, mapped to U s
__global__ void k_logd_grad(const float* __restrict__ s, const float* __restrict__ t, const float* __restrict__ gl,
                            float* __restrict__ gr, int N, int g, float ker0) {
    const int64_t n = (int64_t)N * N * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float mu;
        const float d = floor_diag(s, t, i, N, g, ker0, mu);
        gr[i] = gl[i] * (-ker0 * mu * d);
    }
}

// gs = U^T g: each coarse point gathers, per axis, the fine indices whose interpolation reads it
// (those within one coarse cell of it) with their weights.
__device__ __forceinline__ int adj_axis(int uc, int N, int g, int* fi, float* wi) {
    const int centre = ((uc - g / 2) * N) / g + N / 2;  // a fine index near the coarse point
    const int rad = N / g + 1;                          // N <= 8 g: at most 19 candidates
    int cnt = 0;
    for (int q = centre - rad; q <= centre + rad; ++q) {
        const int qi = ((q % N) + N) % N;
        int c0, c1;
        float t;
        interp(qi, N, g, c0, c1, t);
        float w = 0.f;
        if (c0 == uc) w += 1.f - t;
        if (c1 == uc) w += t;
        if (w != 0.f) { fi[cnt] = qi; wi[cnt] = w; ++cnt; }
    }
    return cnt;
}

__global__ void k_upsample_adj(const float* __restrict__ gr, float* __restrict__ gs, int N, int g) {
    const int GV = g * g * g;
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < GV; u += gridDim.x * blockDim.x) {
        int f1[24], f2[24], f3[24];
        float w1[24], w2[24], w3[24];
        const int n1 = adj_axis(u / (g * g), N, g, f1, w1);
        const int n2 = adj_axis((u / g) % g, N, g, f2, w2);
        const int n3 = adj_axis(u % g, N, g, f3, w3);
        float acc = 0.f;
        for (int a = 0; a < n1; ++a)
            for (int b = 0; b < n2; ++b) {
                const float wab = w1[a] * w2[b];
                const float* gl = gr + ((int64_t)f1[a] * N + f2[b]) * N;
                for (int c = 0; c < n3; ++c) acc += wab * w3[c] * gl[f3[c]];
            }
        gs[u] = acc;
    }
}

}  // namespace

// ------------------------------------------------------------------- host --

struct firm_pcnet_s {
    int bmax = 0;
    hipStream_t stream = nullptr;
    std::string err;
    float* prm = nullptr;   // FP32 masters, oracle order: w1 b1 w2 b2 w3 b3 w4 b4
    float* grad = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    int step = 0;
    __bf16 *w2f = nullptr, *w2b = nullptr, *w3f = nullptr, *w3b = nullptr;
    int64_t cap = 0;        // voxels (batch x g^3) the activation buffers hold
    float *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *o = nullptr, *s = nullptr;
    __bf16 *h1b = nullptr, *h2b = nullptr, *h3b = nullptr;
    float *go = nullptr, *gz = nullptr, *gz2 = nullptr, *gtmp = nullptr, *gs = nullptr;
    __bf16 *gzb = nullptr, *gz2b = nullptr;
    double* part = nullptr;
    double* hpart = nullptr;  // pinned
    int gN = 0;
};

namespace {

constexpr int64_t OFF_W1 = 0, OFF_B1 = OFF_W1 + CH * 27, OFF_W2 = OFF_B1 + CH, OFF_B2 = OFF_W2 + CH * CH * 27,
                  OFF_W3 = OFF_B2 + CH, OFF_B3 = OFF_W3 + CH * CH * 27, OFF_W4 = OFF_B3 + CH,
                  OFF_B4 = OFF_W4 + CH * 27, NPARAM = OFF_B4 + 1;

firm_status net_fail(firm_pcnet n, firm_status s, const std::string& msg) {
    if (n) n->err = msg;
    return firm_fail(nullptr, s, msg);
}

#define NHIP(n, call)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return net_fail((n), FIRM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int nblk(int64_t n, int t = 256) { return (int)std::min<int64_t>((n + t - 1) / t, 65536); }

bool valid_res(int g) { return g >= G0 && g <= 256 && (g & (g - 1)) == 0; }

hipError_t pack(firm_pcnet n) {
    hipLaunchKernelGGL(k_pack_weights, dim3(64), dim3(256), 0, n->stream, n->prm + OFF_W2, n->w2f, n->w2b);
    hipLaunchKernelGGL(k_pack_weights, dim3(64), dim3(256), 0, n->stream, n->prm + OFF_W3, n->w3f, n->w3b);
    return hipGetLastError();
}

void free_acts(firm_pcnet n) {
    void* d[] = {n->h1, n->h2, n->h3, n->o, n->s, n->h1b, n->h2b, n->h3b, n->go, n->gz, n->gz2, n->gs, n->gzb,
                 n->gz2b};
    for (void* p : d)
        if (p) (void)hipFree(p);
    n->h1 = n->h2 = n->h3 = n->o = n->s = n->go = n->gz = n->gz2 = n->gs = nullptr;
    n->h1b = n->h2b = n->h3b = n->gzb = n->gz2b = nullptr;
    n->cap = 0;
}

// Activation and gradient buffers for nv voxels (batch x g^3); reallocated only to grow.
hipError_t ensure_cap(firm_pcnet n, int64_t nv) {
    if (nv <= n->cap) return hipSuccess;
    (void)hipStreamSynchronize(n->stream);
    free_acts(n);
    hipError_t e = hipSuccess;
    auto al = [&](auto** p, int64_t cnt) {
        if (e == hipSuccess) e = hipMalloc((void**)p, cnt * sizeof(**p));
    };
    al(&n->h1, nv * CH); al(&n->h2, nv * CH); al(&n->h3, nv * CH);
    al(&n->h1b, nv * CH); al(&n->h2b, nv * CH); al(&n->h3b, nv * CH);
    al(&n->o, nv); al(&n->s, nv); al(&n->go, nv); al(&n->gs, nv);
    al(&n->gz, nv * CH); al(&n->gz2, nv * CH); al(&n->gzb, nv * CH); al(&n->gz2b, nv * CH);
    if (e != hipSuccess) {
        free_acts(n);
        return e;
    }
    n->cap = nv;
    return hipSuccess;
}

hipError_t forward(firm_pcnet n, const float* feat, int B, int g) {
    const int64_t nv = (int64_t)B * g * g * g;
    hipLaunchKernelGGL(k_conv_first, dim3(nblk(nv)), dim3(256), 0, n->stream, feat, n->prm + OFF_W1, n->prm + OFF_B1,
                       n->h1, n->h1b, B, g);
    const int64_t rows = (int64_t)B * g * g * (g / 32);
    hipLaunchKernelGGL((k_conv_mfma<true>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, n->stream, n->h1b,
                       n->w2f, n->prm + OFF_B2, nullptr, n->h2, n->h2b, B, g);
    hipLaunchKernelGGL((k_conv_mfma<true>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, n->stream, n->h2b,
                       n->w3f, n->prm + OFF_B3, nullptr, n->h3, n->h3b, B, g);
    hipLaunchKernelGGL(k_conv_last, dim3(nblk(nv)), dim3(256), 0, n->stream, n->h3, n->prm + OFF_W4,
                       n->prm + OFF_B4, n->o, B, g);
    return hipGetLastError();
}

}  // namespace

extern "C" {

int64_t firm_pcnet_num_params(void) { return NPARAM; }

void firm_pcnet_destroy(firm_pcnet n) {
    if (!n) return;
    free_acts(n);
    void* d[] = {n->prm, n->grad, n->m, n->v, n->w2f, n->w2b, n->w3f, n->w3b, n->gtmp, n->part};
    for (void* p : d)
        if (p) (void)hipFree(p);
    if (n->hpart) (void)hipHostFree(n->hpart);
    delete n;
}

firm_status firm_pcnet_create(firm_pcnet* out, int max_batch, void* stream) {
    if (!out || max_batch < 1 || max_batch > 64) return firm_fail(nullptr, FIRM_ERR_ARG, "max_batch must be in [1, 64]");
    *out = nullptr;
    firm_pcnet n = new firm_pcnet_s();
    n->bmax = max_batch;
    n->stream = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    auto al = [&](auto** p, int64_t cnt) {
        if (e == hipSuccess) e = hipMalloc((void**)p, cnt * sizeof(**p));
    };
    al(&n->prm, NPARAM); al(&n->grad, NPARAM); al(&n->m, NPARAM); al(&n->v, NPARAM);
    al(&n->w2f, 27 * CH * CH); al(&n->w2b, 27 * CH * CH); al(&n->w3f, 27 * CH * CH); al(&n->w3b, 27 * CH * CH);
    al(&n->part, 4096);
    if (e == hipSuccess) e = ensure_cap(n, (int64_t)max_batch * G0 * G0 * G0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&n->hpart, 4096 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemset(n->prm, 0, NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMemset(n->m, 0, NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMemset(n->v, 0, NPARAM * sizeof(float));
    if (e != hipSuccess) {
        firm_pcnet_destroy(n);
        return firm_fail(nullptr, FIRM_ERR_ALLOC, std::string("pcnet allocation: ") + hipGetErrorString(e));
    }
    *out = n;
    return FIRM_OK;
}

firm_status firm_pcnet_set_params(firm_pcnet n, const float* host) {
    if (!n || !host) return firm_fail(nullptr, FIRM_ERR_ARG, "null argument");
    for (int64_t i = 0; i < NPARAM; ++i)
        if (!std::isfinite(host[i])) return net_fail(n, FIRM_ERR_ARG, "parameters must be finite");
    NHIP(n, hipMemcpyAsync(n->prm, host, NPARAM * sizeof(float), hipMemcpyHostToDevice, n->stream));
    NHIP(n, fill_zero(n->m, NPARAM * sizeof(float), n->stream));
    NHIP(n, fill_zero(n->v, NPARAM * sizeof(float), n->stream));
    NHIP(n, pack(n));
    NHIP(n, hipStreamSynchronize(n->stream));
    n->step = 0;
    return FIRM_OK;
}

firm_status firm_pcnet_get_params(firm_pcnet n, float* host) {
    if (!n || !host) return firm_fail(nullptr, FIRM_ERR_ARG, "null argument");
    NHIP(n, hipMemcpyAsync(host, n->prm, NPARAM * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    return FIRM_OK;
}

firm_status firm_pcnet_forward(firm_pcnet n, const float* feat, int res, float* out, int B) {
    if (!n || !feat || !out) return firm_fail(nullptr, FIRM_ERR_ARG, "null argument");
    if (B < 1 || B > n->bmax) return net_fail(n, FIRM_ERR_ARG, "batch out of range");
    if (!valid_res(res)) return net_fail(n, FIRM_ERR_ARG, "res must be a power of two in [32, 256]");
    const int64_t nv = (int64_t)B * res * res * res;
    NHIP(n, ensure_cap(n, nv));
    NHIP(n, forward(n, feat, B, res));
    NHIP(n, hipMemcpyAsync(out, n->o, (size_t)nv * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    return FIRM_OK;
}

// Loss (mean over the batch) and parameter gradients for B samples at size N.  t, A and Bs are
// [B][N^3] device arrays on the centred grid; sumc and ker0 are host arrays of B values.
firm_status firm_pcnet_loss_grad(firm_pcnet n, const float* feat, int res, int B, int N, int objective,
                                 const float* t, const float* A, const float* Bs, const double* sumc,
                                 const double* ker0, double* loss, float* grad_host) {
    if (!n) return firm_fail(nullptr, FIRM_ERR_ARG, "null network");
    if (objective < 0 || objective > 2)
        return net_fail(n, FIRM_ERR_ARG, "objective must be 0 (probe), 1 (Kaporin) or 2 (given log-d gradient)");
    if (!feat || !t || !ker0 || (objective != 2 && !loss) || (objective != 1 && !A) ||
        (objective == 0 && (!Bs || !sumc)))
        return net_fail(n, FIRM_ERR_ARG, "null argument");
    if (B < 1 || B > n->bmax) return net_fail(n, FIRM_ERR_ARG, "batch out of range");
    if (N < 8 || N > 256 || (N & (N - 1))) return net_fail(n, FIRM_ERR_ARG, "N must be a power of two in [8, 256]");
    if (!valid_res(res) || N > 8 * res) return net_fail(n, FIRM_ERR_ARG, "res must be a power of two in [32, 256], N <= 8 res");
    const int g = res;
    const int64_t GV = (int64_t)g * g * g;
    const int64_t n3 = (int64_t)N * N * N;
    if (n->gN < N) {
        if (n->gtmp) (void)hipFree(n->gtmp);
        n->gtmp = nullptr;
        NHIP(n, hipMalloc((void**)&n->gtmp, n3 * sizeof(float)));
        n->gN = N;
    }
    for (int b = 0; b < B; ++b)
        if ((objective == 0 && !(sumc[b] > 0)) || !(ker0[b] > 0))
            return net_fail(n, FIRM_ERR_ARG, "sumc and ker0 must be > 0");
    NHIP(n, ensure_cap(n, (int64_t)B * GV));
    hipStream_t st = n->stream;
    NHIP(n, forward(n, feat, B, g));
    hipLaunchKernelGGL(k_symmetrise, dim3(nblk((int64_t)B * GV)), dim3(256), 0, st, n->o, n->s, B, g);
    const int lb = nblk(n3);
    const int lblocks = std::min(lb, 1024);
    double total = 0.0;
    for (int b = 0; b < B; ++b) {
        const float* sb = n->s + (int64_t)b * GV;
        const float* tb = t + b * n3;
        const float k0 = (float)ker0[b];
        if (objective == 0) {
            hipLaunchKernelGGL(k_loss_grad, dim3(lblocks), dim3(256), 0, st, sb, tb, A + b * n3, Bs + b * n3, n->gtmp,
                               N, g, k0, (float)(1.0 / sumc[b]), n->part);
            NHIP(n, hipMemcpyAsync(n->hpart, n->part, lblocks * sizeof(double), hipMemcpyDeviceToHost, st));
            NHIP(n, hipStreamSynchronize(st));
            double sp = 0.0;
            for (int i = 0; i < lblocks; ++i) sp += n->hpart[i];
            total += sp / sumc[b] + 1.0;
        } else if (objective == 1) {
            hipLaunchKernelGGL(k_kap_sums, dim3(lblocks), dim3(256), 0, st, sb, tb, N, g, k0, n->part, lblocks);
            NHIP(n, hipMemcpyAsync(n->hpart, n->part, 2 * lblocks * sizeof(double), hipMemcpyDeviceToHost, st));
            NHIP(n, hipStreamSynchronize(st));
            double sdt = 0.0, slog = 0.0;
            for (int i = 0; i < lblocks; ++i) {
                sdt += n->hpart[i];
                slog += n->hpart[lblocks + i];
            }
            if (!(sdt > 0) || !std::isfinite(sdt) || !std::isfinite(slog))
                return net_fail(n, FIRM_ERR_ARG, "Kaporin objective needs t > 0 and a finite diagonal");
            total += std::log(sdt / (double)n3) - slog / (double)n3;
            hipLaunchKernelGGL(k_kap_grad, dim3(nblk(n3)), dim3(256), 0, st, sb, tb, n->gtmp, N, g, k0, 1.0 / sdt,
                               1.0 / (double)n3);
        } else {
            hipLaunchKernelGGL(k_logd_grad, dim3(nblk(n3)), dim3(256), 0, st, sb, tb, A + b * n3, n->gtmp, N, g, k0);
        }
        hipLaunchKernelGGL(k_upsample_adj, dim3(nblk(GV)), dim3(256), 0, st, n->gtmp, n->gs + (int64_t)b * GV, N, g);
    }
    if (loss) *loss = objective == 2 ? 0.0 : total / B;
    hipLaunchKernelGGL(k_symmetrise, dim3(nblk((int64_t)B * GV)), dim3(256), 0, st, n->gs, n->go, B, g);
    // backward
    NHIP(n, fill_zero(n->grad, NPARAM * sizeof(float), st));
    const int chunks = (int)(((int64_t)B * GV + 255) / 256);
    hipLaunchKernelGGL(k_wgrad_last, dim3(chunks, 27), dim3(256), 0, st, n->go, n->h3, n->grad + OFF_W4,
                       n->grad + OFF_B4, B, 256, g);
    hipLaunchKernelGGL(k_conv_last_bwd, dim3(nblk((int64_t)B * GV)), dim3(256), 0, st, n->go, n->prm + OFF_W4,
                       n->h3, n->gz, n->gzb, B, g);
    const int64_t rows = (int64_t)B * g * g * (g / 32);
    // weight gradients of the C -> C layers: about 512 workgroups (two per CU), each over a run of rows
    const int rpb = (int)((rows + 511) / 512);
    const unsigned wblocks = (unsigned)((rows + rpb - 1) / rpb);
    hipLaunchKernelGGL(k_wgrad_mfma, dim3(wblocks), dim3(64 * WG_WAVES), 0, st, n->gzb, n->h2b, n->grad + OFF_W3,
                       n->grad + OFF_B3, B, g, rpb);
    hipLaunchKernelGGL((k_conv_mfma<false>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, n->gzb, n->w3b,
                       nullptr, n->h2, n->gz2, n->gz2b, B, g);
    hipLaunchKernelGGL(k_wgrad_mfma, dim3(wblocks), dim3(64 * WG_WAVES), 0, st, n->gz2b, n->h1b, n->grad + OFF_W2,
                       n->grad + OFF_B2, B, g, rpb);
    hipLaunchKernelGGL((k_conv_mfma<false>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, n->gz2b, n->w2b,
                       nullptr, n->h1, n->gz, n->gzb, B, g);
    hipLaunchKernelGGL((k_wgrad<1>), dim3(chunks, 27), dim3(CH), 0, st, n->gz, feat, n->grad + OFF_W1,
                       n->grad + OFF_B1, B, 256, g);
    NHIP(n, hipGetLastError());
    if (grad_host) {
        NHIP(n, hipMemcpyAsync(grad_host, n->grad, NPARAM * sizeof(float), hipMemcpyDeviceToHost, st));
        NHIP(n, hipStreamSynchronize(st));
        for (int64_t i = 0; i < NPARAM; ++i) grad_host[i] /= (float)B;
    }
    return FIRM_OK;
}

firm_status firm_pcnet_train_step(firm_pcnet n, const float* feat, int res, int B, int N, int objective,
                                  const float* t, const float* A, const float* Bs, const double* sumc,
                                  const double* ker0, double lr, double lr_floor, double* loss) {
    if (!n) return firm_fail(nullptr, FIRM_ERR_ARG, "null network");
    if (!(lr > 0.0) || !std::isfinite(lr) || !(lr_floor >= 0.0) || !std::isfinite(lr_floor))
        return net_fail(n, FIRM_ERR_ARG, "lr must be finite and > 0, lr_floor finite and >= 0");
    firm_status s = firm_pcnet_loss_grad(n, feat, res, B, N, objective, t, A, Bs, sumc, ker0, loss, nullptr);
    if (s != FIRM_OK) return s;
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)n->step), c2 = 1.f - std::pow(b2, (float)n->step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(NPARAM)), dim3(256), 0, n->stream, n->prm, n->grad, n->m, n->v,
                       (int)NPARAM, (float)lr, (float)lr_floor, b1, b2, 1e-8f, c1, c2, 1.f / (float)B);
    NHIP(n, pack(n));
    return FIRM_OK;
}

}  // extern "C"

namespace {

// symmetrise the network output into s (res^3 floats) and form d on the plan's grid
firm_status diag_from_output(firm_plan p, const float* out, int res, const float* t, float* d, float* s) {
    const int64_t GV = (int64_t)res * res * res;
    hipLaunchKernelGGL(k_symmetrise, dim3(nblk(GV)), dim3(256), 0, p->stream, out, s, 1, res);
    const int64_t n3 = (int64_t)p->N * p->N * p->N;
    hipLaunchKernelGGL(k_diag_from_s, dim3(nblk(n3)), dim3(256), 0, p->stream, s, t, d, p->N, res, (float)p->ker0);
    return FIRM_OK;
}

firm_status precond_args(firm_plan p, const float* out, int res, const float* t, float* d) {
    if (!p || !out || !t || !d) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (!valid_res(res) || p->N > 8 * res)
        return firm_fail(p, FIRM_ERR_ARG, "res must be a power of two in [32, 256], N <= 8 res");
    if (!p->have_kernel) return firm_fail(p, FIRM_ERR_STATE, "no kernel");
    return FIRM_OK;
}

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[MAX_DEVICES] = {};  // device address of `scratch`, per device

// Device address of `scratch` on the current device, looked up once per device.
hipError_t scratch_address(float** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<float*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

// Set-up of the no-allocation entry point on the current device (called by firm_plan_create).
hipError_t noalloc_scratch_setup() {
    float* s = nullptr;
    return scratch_address(&s);
}

extern "C" {

// d (centred N^3) = 1 / (t + Ker(0) exp(U sym(out))) for the plan's kernel, out on the res^3 grid
firm_status firm_precond_from_output(firm_plan p, const float* out, int res, const float* t, float* d) {
    firm_status st = precond_args(p, out, res, t, d);
    if (st != FIRM_OK) return st;
    const int64_t GV = (int64_t)res * res * res;
    float* s = nullptr;
    FIRM_HIP(p, hipMalloc((void**)&s, GV * sizeof(float)));
    diag_from_output(p, out, res, t, d, s);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    (void)hipFree(s);
    if (e != hipSuccess) return firm_fail(p, FIRM_ERR_HIP, std::string("precond_from_output: ") + hipGetErrorString(e));
    return FIRM_OK;
}

// firm_precond_from_output with the symmetrised output in the static scratch (res <= 128): no
// allocation, enqueued on the plan stream without synchronising.  Nothing needs clearing: the
// symmetrisation writes every entry the diagonal kernel reads.
firm_status firm_precond_from_output_noalloc(firm_plan p, const float* out, int res, const float* t, float* d) {
    firm_status st = precond_args(p, out, res, t, d);
    if (st != FIRM_OK) return st;
    if (res > NOALLOC_MAX_RES)
        return firm_fail(p, FIRM_ERR_ARG, "res must be <= 128: the no-allocation scratch holds 128^3 floats");
    float* s = nullptr;
    FIRM_HIP(p, scratch_address(&s));
    diag_from_output(p, out, res, t, d, s);
    FIRM_HIP(p, hipGetLastError());
    return FIRM_OK;
}

const char* firm_pcnet_last_error(firm_pcnet n) { return n ? n->err.c_str() : ""; }

}  // extern "C"
