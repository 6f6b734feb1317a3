// 3D FFT passes of libfirm: the A*A product through the 2N circulant embedding
// (section 3.2, eq. embedding_circulant with eq. circ1 in three dimensions), the
// kernel spectrum, the gridding transforms and the Fourier-diagonal
// preconditioner.  Every pass transforms one axis of a 3D array with the
// LDS-staged pencils of fft_core.h; zero padding, cropping, mode selection, the
// kernel multiply and the CG vector work are fused into the loads and stores.
#include "fft_core.h"
#include "firm_internal.h"

namespace {

template <class S> struct VecOf;
template <> struct VecOf<float> { using V = float2; };
template <> struct VecOf<double> { using V = double2; };

// threads of a pencil workgroup keyed by one integer (L * 16 + sizeof(scalar)), so that the
// launch-bounds argument carries no comma
template <int LS>
struct FftThr {
    static constexpr int value = (LS % 16 == 8) ? FftCfg<LS / 16, double2>::THREADS : FftCfg<LS / 16, float2>::THREADS;
};

enum MapKind { MAP_FIRST = 0, MAP_CIRC = 1, MAP_CENTER = 2 };
enum EpiKind { EPI_STORE = 0, EPI_REAL = 1, EPI_KER = 2, EPI_ATB = 3 };

struct EpiArgs {
    double scale = 1.0;
    const float* dec_e = nullptr;   // per output index along the transformed axis
    const float* dec_o = nullptr;   // per outer index
    const float* dec_c = nullptr;   // per column
    int wrap_o = -1;                // outer index whose plane is zero (circulant wrap)
    float k0 = 0.f;                 // constant added (EPI_KER)
    const double* k0dev = nullptr;  // constant added, device scalar (EPI_ATB)
};

// bin of output index t for a mode map; -1 means "store zero"
template <int MAP>
__device__ __forceinline__ int out_bin(int t, int L, int n_out) {
    if constexpr (MAP == MAP_FIRST) {
        return t;
    } else if constexpr (MAP == MAP_CIRC) {  // offsets (-N, N) from L bins, n_out = 2N
        const int N = n_out >> 1;
        return t < N ? t : (t == N ? -1 : t - n_out + L);
    } else {  // centred modes -n_out/2 .. n_out/2 - 1
        const int n = t - (n_out >> 1);
        return n < 0 ? n + L : n;
    }
}

__device__ __forceinline__ bool cg_inactive(const int* active) { return active && *active == 0; }

// Block sum of a double; result valid in thread 0.
template <int THREADS>
__device__ __forceinline__ double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < THREADS / 64; ++i) s += red[i];
    return s;
}

// ---------------------------------------------------------------------------
// Real rows -> half spectra.  Rows 2i and 2i+1 form one complex pencil
// z = x_a + i x_b (zero-padded from n_in to L); X_a(q) = (Z(q) + conj Z(L-q)) / 2,
// X_b(q) = (Z(q) - conj Z(L-q)) / 2i; modes q < n_keep are stored.
// PRO: the rows are p = src + beta * pvec (CG direction update), written back to pvec.
template <int L, bool PRO, class S = float>
__global__ void __launch_bounds__(FftThr<L * 16 + (int)sizeof(S)>::value)
k_r2c_rows(const S* __restrict__ src, int nrows, int in_pitch, int n_in, typename VecOf<S>::V* __restrict__ dst,
           int out_pitch, int n_keep, S sg, const typename VecOf<S>::V* __restrict__ tw, S* pvec,
           const double* beta_dev, const int* active) {
    using V = typename VecOf<S>::V;
    using Cfg = FftCfg<L, V>;
    constexpr int C = Cfg::C, CP = Cfg::CP, NT = Cfg::THREADS;
    __shared__ V buf[L * CP];
    if (cg_inactive(active)) return;
    const int tid = threadIdx.x;
    const int pair0 = blockIdx.x * C;
    const int npairs = nrows >> 1;
    S beta = 0;
    if (PRO) beta = (S)(*beta_dev);
    for (int idx = tid; idx < C * (L - n_in); idx += NT) {
        const int c = idx % C, e = n_in + idx / C;
        buf[e * CP + c] = mkv<V>(0, 0);
    }
    S* bf = reinterpret_cast<S*>(buf);
    for (int idx = tid; idx < C * 2 * n_in; idx += NT) {
        const int e = idx % n_in, t = idx / n_in, rr = t & 1, c = t >> 1;
        const int pr = pair0 + c;
        S v = 0;
        if (pr < npairs) {
            const int64_t g = (int64_t)(2 * pr + rr) * in_pitch + e;
            v = src[g];
            if (PRO) {
                v = v + beta * pvec[g];
                pvec[g] = v;
            }
        }
        bf[2 * (e * CP + c) + rr] = v;
    }
    __syncthreads();
    fft_lds<L, C>(buf, tw, sg);
    for (int idx = tid; idx < C * n_keep; idx += NT) {
        const int q = idx % n_keep, c = idx / n_keep;
        const int pr = pair0 + c;
        if (pr >= npairs) continue;
        const V Z = buf[q * CP + c];
        const V Zm = buf[((L - q) & (L - 1)) * CP + c];
        const V Sp = mkv<V>((S)0.5 * (Z.x + Zm.x), (S)0.5 * (Z.y - Zm.y));   // (Z + conj Zm)/2
        const V D = mkv<V>((S)0.5 * (Z.x - Zm.x), (S)0.5 * (Z.y + Zm.y));    // (Z - conj Zm)/2
        dst[(int64_t)(2 * pr) * out_pitch + q] = Sp;
        dst[(int64_t)(2 * pr + 1) * out_pitch + q] = mkv<V>(D.y, -D.x);       // D / i
    }
}

// Half spectra (modes 0..L/2 of two real rows) -> real rows, first n_out samples.
// y = scale * x + lam * xadd.  CG: also a block partial of sum(xadd * y) in FP64.
template <int L, bool DOT, class S = float>
__global__ void __launch_bounds__(FftThr<L * 16 + (int)sizeof(S)>::value)
k_c2r_rows(const typename VecOf<S>::V* __restrict__ src, int nrows, int in_pitch, S* __restrict__ dst, int out_pitch,
           int n_out, S sg, S scale, S lam, const S* __restrict__ xadd,
           const typename VecOf<S>::V* __restrict__ tw, double* partials, const int* active) {
    using V = typename VecOf<S>::V;
    using Cfg = FftCfg<L, V>;
    constexpr int C = Cfg::C, CP = Cfg::CP, NT = Cfg::THREADS;
    constexpr int H = L / 2 + 1;
    __shared__ V buf[L * CP];
    __shared__ double red[NT / 64];
    if (cg_inactive(active)) return;
    const int tid = threadIdx.x;
    const int pair0 = blockIdx.x * C;
    const int npairs = nrows >> 1;
    for (int idx = tid; idx < C * H; idx += NT) {
        const int q = idx % H, c = idx / H;
        const int pr = pair0 + c;
        V Ya = mkv<V>(0, 0), Yb = Ya;
        if (pr < npairs) {
            Ya = src[(int64_t)(2 * pr) * in_pitch + q];
            Yb = src[(int64_t)(2 * pr + 1) * in_pitch + q];
        }
        buf[q * CP + c] = mkv<V>(Ya.x - Yb.y, Ya.y + Yb.x);                 // Ya + i Yb
        if (q > 0 && q < L / 2) buf[(L - q) * CP + c] = mkv<V>(Ya.x + Yb.y, Yb.x - Ya.y);  // conj Ya + i conj Yb
    }
    __syncthreads();
    fft_lds<L, C>(buf, tw, sg);
    double acc = 0.0;
    for (int idx = tid; idx < C * 2 * n_out; idx += NT) {
        const int e = idx % n_out, t = idx / n_out, rr = t & 1, c = t >> 1;
        const int pr = pair0 + c;
        if (pr >= npairs) continue;
        const V v = buf[e * CP + c];
        const int64_t g = (int64_t)(2 * pr + rr) * out_pitch + e;
        S y = scale * (rr ? v.y : v.x);
        if (xadd) {
            const S xv = xadd[g];
            y += lam * xv;
            if (DOT) acc += (double)xv * (double)y;
        }
        dst[g] = y;
    }
    if (DOT) {
        const double s = block_sum<NT>(acc, red);
        if (tid == 0) partials[blockIdx.x] = s;
    }
}

// Complex pencils along one axis.  Block -> (outer o, column group); CONTIG means the
// transformed axis is contiguous (elements adjacent), otherwise columns are adjacent.
template <int L, bool CONTIG, int MAP, int EPI, class S = float>
__global__ void __launch_bounds__(FftThr<L * 16 + (int)sizeof(S)>::value)
k_c2c(const typename VecOf<S>::V* __restrict__ src, void* __restrict__ dstv, int ncols, int64_t s_outer, int64_t s_col,
      int64_t s_elem, int64_t d_outer, int64_t d_col, int64_t d_elem, int n_in, int n_out, S sg,
      const typename VecOf<S>::V* __restrict__ tw, EpiArgs ep, const int* active) {
    using V = typename VecOf<S>::V;
    using Cfg = FftCfg<L, V>;
    constexpr int C = Cfg::C, CP = Cfg::CP, NT = Cfg::THREADS;
    __shared__ V buf[L * CP];
    if (cg_inactive(active)) return;
    const int tid = threadIdx.x;
    const int ng = (ncols + C - 1) / C;
    const int o = blockIdx.x / ng;
    const int c0 = (blockIdx.x - o * ng) * C;
    const int nc = min(C, ncols - c0);
    for (int idx = tid; idx < C * (L - n_in); idx += NT) {
        const int c = idx % C, e = n_in + idx / C;
        buf[e * CP + c] = mkv<V>(0, 0);
    }
    const V* s0 = src + o * s_outer + c0 * s_col;
    for (int idx = tid; idx < C * n_in; idx += NT) {
        int c, e;
        if (CONTIG) { e = idx % n_in; c = idx / n_in; }
        else { c = idx % C; e = idx / C; }
        if (c < nc) buf[e * CP + c] = s0[c * s_col + e * s_elem];
    }
    __syncthreads();
    fft_lds<L, C>(buf, tw, sg);
    for (int idx = tid; idx < C * n_out; idx += NT) {
        int c, t;
        if (CONTIG) { t = idx % n_out; c = idx / n_out; }
        else { c = idx % C; t = idx / C; }
        if (c >= nc) continue;
        const int bin = out_bin<MAP>(t, L, n_out);
        const V v = bin < 0 ? mkv<V>(0, 0) : buf[bin * CP + c];
        const int64_t g = o * d_outer + (int64_t)(c0 + c) * d_col + (int64_t)t * d_elem;
        if constexpr (EPI == EPI_STORE) {
            reinterpret_cast<V*>(dstv)[g] = v;
        } else if constexpr (EPI == EPI_REAL) {
            reinterpret_cast<S*>(dstv)[g] = v.x * (S)ep.scale;
        } else if constexpr (EPI == EPI_KER) {
            float r = 0.f;
            if (bin >= 0 && o != ep.wrap_o)
                r = v.x * ep.dec_e[t] * ep.dec_o[o] * ep.dec_c[c0 + c] + ep.k0;
            reinterpret_cast<float*>(dstv)[g] = r;
        } else {  // EPI_ATB
            reinterpret_cast<float*>(dstv)[g] =
                v.x * ep.dec_e[t] * ep.dec_o[o] * ep.dec_c[c0 + c] + (float)(*ep.k0dev);
        }
    }
}

// Middle pass of the product: along axis 1, zero-pad the first n_in entries, forward
// transform, multiply by the real spectrum, inverse transform, keep the first n_in.
template <int L, class S = float>
__global__ void __launch_bounds__(FftThr<L * 16 + (int)sizeof(S)>::value)
k_conv_mid(typename VecOf<S>::V* __restrict__ data, const S* __restrict__ spec, int ncols, int64_t s_outer,
           int64_t s_elem, int64_t k_outer, int64_t k_elem, int n_in, const typename VecOf<S>::V* __restrict__ tw,
           const int* active) {
    using V = typename VecOf<S>::V;
    using Cfg = FftCfg<L, V>;
    constexpr int C = Cfg::C, CP = Cfg::CP, NT = Cfg::THREADS;
    __shared__ V buf[L * CP];
    if (cg_inactive(active)) return;
    const int tid = threadIdx.x;
    const int ng = (ncols + C - 1) / C;
    const int o = blockIdx.x / ng;
    const int c0 = (blockIdx.x - o * ng) * C;
    const int nc = min(C, ncols - c0);
    V* d0 = data + o * s_outer + c0;
    const S* k0 = spec + o * k_outer + c0;
    for (int idx = tid; idx < C * (L - n_in); idx += NT) {
        const int c = idx % C, e = n_in + idx / C;
        buf[e * CP + c] = mkv<V>(0, 0);
    }
    for (int idx = tid; idx < C * n_in; idx += NT) {
        const int c = idx % C, e = idx / C;
        if (c < nc) buf[e * CP + c] = d0[c + e * s_elem];
    }
    __syncthreads();
    fft_lds<L, C>(buf, tw, (S)-1);
    for (int idx = tid; idx < C * L; idx += NT) {
        const int c = idx % C, e = idx / C;
        if (c < nc) {
            const S k = k0[c + e * k_elem];
            V v = buf[e * CP + c];
            buf[e * CP + c] = mkv<V>(v.x * k, v.y * k);
        }
    }
    __syncthreads();
    fft_lds<L, C>(buf, tw, (S)1);
    for (int idx = tid; idx < C * n_in; idx += NT) {
        const int c = idx % C, e = idx / C;
        if (c < nc) d0[c + e * s_elem] = buf[e * CP + c];
    }
}

// ----------------------------------------------------------------- launchers
template <int L, bool PRO, class S = float>
hipError_t launch_r2c(hipStream_t st, const S* src, int nrows, int in_pitch, int n_in, typename VecOf<S>::V* dst,
                      int out_pitch, int n_keep, S sg, const typename VecOf<S>::V* tw, S* pvec = nullptr,
                      const double* beta = nullptr, const int* active = nullptr) {
    using Cfg = FftCfg<L, typename VecOf<S>::V>;
    const int blocks = ceil_div(nrows / 2, Cfg::C);
    hipLaunchKernelGGL((k_r2c_rows<L, PRO, S>), dim3(blocks), dim3(Cfg::THREADS), 0, st, src, nrows,
                       in_pitch, n_in, dst, out_pitch, n_keep, sg, tw, pvec, beta, active);
    return hipGetLastError();
}

template <int L, bool DOT, class S = float>
hipError_t launch_c2r(hipStream_t st, const typename VecOf<S>::V* src, int nrows, int in_pitch, S* dst, int out_pitch,
                      int n_out, S sg, S scale, S lam, const S* xadd, const typename VecOf<S>::V* tw,
                      double* partials = nullptr, const int* active = nullptr) {
    using Cfg = FftCfg<L, typename VecOf<S>::V>;
    const int blocks = ceil_div(nrows / 2, Cfg::C);
    hipLaunchKernelGGL((k_c2r_rows<L, DOT, S>), dim3(blocks), dim3(Cfg::THREADS), 0, st, src, nrows,
                       in_pitch, dst, out_pitch, n_out, sg, scale, lam, xadd, tw, partials, active);
    return hipGetLastError();
}

template <int L, bool CONTIG, int MAP, int EPI, class S = float>
hipError_t launch_c2c(hipStream_t st, const typename VecOf<S>::V* src, void* dst, int nouter, int ncols,
                      int64_t s_outer, int64_t s_col, int64_t s_elem, int64_t d_outer, int64_t d_col,
                      int64_t d_elem, int n_in, int n_out, S sg, const typename VecOf<S>::V* tw,
                      EpiArgs ep = EpiArgs(), const int* active = nullptr) {
    using Cfg = FftCfg<L, typename VecOf<S>::V>;
    const int blocks = nouter * ceil_div(ncols, Cfg::C);
    hipLaunchKernelGGL((k_c2c<L, CONTIG, MAP, EPI, S>), dim3(blocks), dim3(Cfg::THREADS), 0, st, src, dst,
                       ncols, s_outer, s_col, s_elem, d_outer, d_col, d_elem, n_in, n_out, sg, tw, ep, active);
    return hipGetLastError();
}

template <int L, class S = float>
hipError_t launch_mid(hipStream_t st, typename VecOf<S>::V* data, const S* spec, int nouter, int ncols,
                      int64_t s_outer, int64_t s_elem, int64_t k_outer, int64_t k_elem, int n_in,
                      const typename VecOf<S>::V* tw, const int* active = nullptr) {
    using Cfg = FftCfg<L, typename VecOf<S>::V>;
    const int blocks = nouter * ceil_div(ncols, Cfg::C);
    hipLaunchKernelGGL((k_conv_mid<L, S>), dim3(blocks), dim3(Cfg::THREADS), 0, st, data, spec, ncols,
                       s_outer, s_elem, k_outer, k_elem, n_in, tw, active);
    return hipGetLastError();
}

#define RET_IF(e)                       \
    do {                                \
        hipError_t e__ = (e);           \
        if (e__ != hipSuccess) return e__; \
    } while (0)

// The five passes of y = crop(IFFT(K^ . FFT(pad x))) + lam x for one N (L = 2N).
// CG form: the first pass forms p = src + beta p and the last q = . + lam p with <p, q>.
template <int L>
hipError_t apply_passes(firm_plan p, const float* src, float* pvec, float* y, float lam, const double* beta,
                        const int* active, double* partials) {
    const int N = L / 2, QP = p->QP;
    hipStream_t st = p->stream;
    const bool cg = (beta != nullptr);
    // A: rows along i3, N real -> padded 2N transform, modes 0..N kept
    if (cg)
        RET_IF((launch_r2c<L, true>(st, src, N * N, N, N, p->T1, QP, N + 1, -1.f, p->tw, pvec, beta, active)));
    else
        RET_IF((launch_r2c<L, false>(st, src, N * N, N, N, p->T1, QP, N + 1, -1.f, p->tw)));
    // B: along i2 for every (i1, q3): T1[i1][i2][q3] (N) -> T2[i1][q2][q3] (2N)
    RET_IF((launch_c2c<L, false, MAP_FIRST, EPI_STORE>(st, p->T1, p->T2, N, N + 1, (int64_t)N * QP, 1, QP,
                                                         (int64_t)L * QP, 1, QP, N, L, -1.f, p->tw, EpiArgs(),
                                                         active)));
    // C: along i1 for every (q2, q3): forward, times K^, inverse, keep i1 < N
    RET_IF((launch_mid<L>(st, p->T2, p->khat, L, N + 1, QP, (int64_t)L * QP, QP, (int64_t)L * QP, N, p->tw,
                          active)));
    // D: inverse along q2, keep i2 < N: T2[i1][q2][q3] -> T1[i1][i2][q3]
    RET_IF((launch_c2c<L, false, MAP_FIRST, EPI_STORE>(st, p->T2, p->T1, N, N + 1, (int64_t)L * QP, 1, QP,
                                                         (int64_t)N * QP, 1, QP, L, N, 1.f, p->tw, EpiArgs(),
                                                         active)));
    // E: inverse along q3 (half spectrum -> real), crop, + lam x
    if (cg)
        return launch_c2r<L, true>(st, p->T1, N * N, QP, y, N, N, 1.f, 1.f, lam, pvec, p->tw, partials, active);
    return launch_c2r<L, false>(st, p->T1, N * N, QP, y, N, N, 1.f, 1.f, lam, src, p->tw);
}

// FP64 form of the product, for true residuals and the FP64 solver modes: the same
// five passes in double with the double spectrum khat64.
template <int L>
hipError_t apply_passes64(firm_plan p, const double* x, double* y, double lam) {
    const int N = L / 2, QP = p->QP;
    hipStream_t st = p->stream;
    RET_IF((launch_r2c<L, false, double>(st, x, N * N, N, N, p->T1d, QP, N + 1, -1.0, p->tw64)));
    RET_IF((launch_c2c<L, false, MAP_FIRST, EPI_STORE, double>(st, p->T1d, p->T2d, N, N + 1, (int64_t)N * QP, 1,
                                                                 QP, (int64_t)L * QP, 1, QP, N, L, -1.0, p->tw64)));
    RET_IF((launch_mid<L, double>(st, p->T2d, p->khat64, L, N + 1, QP, (int64_t)L * QP, QP, (int64_t)L * QP, N,
                                  p->tw64)));
    RET_IF((launch_c2c<L, false, MAP_FIRST, EPI_STORE, double>(st, p->T2d, p->T1d, N, N + 1, (int64_t)L * QP, 1,
                                                                 QP, (int64_t)N * QP, 1, QP, L, N, 1.0, p->tw64)));
    return launch_c2r<L, false, double>(st, p->T1d, N * N, QP, y, N, N, 1.0, 1.0, lam, x, p->tw64);
}

// khat64 = Re DFT_{2N}(kerc) / (2N)^3 in FP64 from the circulant column held as double.
template <int L>
hipError_t khat64_passes(firm_plan p, const double* kerc64, double2* w1) {
    const int N = L / 2, QP = p->QP;
    hipStream_t st = p->stream;
    RET_IF((launch_r2c<L, false, double>(st, kerc64, L * L, L, L, w1, QP, N + 1, -1.0, p->tw64)));
    RET_IF((launch_c2c<L, false, MAP_FIRST, EPI_STORE, double>(st, w1, w1, L, N + 1, (int64_t)L * QP, 1, QP,
                                                                 (int64_t)L * QP, 1, QP, L, L, -1.0, p->tw64)));
    EpiArgs ep;
    ep.scale = 1.0 / ((double)L * (double)L * (double)L);
    return launch_c2c<L, false, MAP_FIRST, EPI_REAL, double>(st, w1, p->khat64, L, N + 1, QP, 1, (int64_t)L * QP,
                                                             QP, 1, (int64_t)L * QP, L, L, -1.0, p->tw64, ep);
}

template <int L>
hipError_t khat_passes(firm_plan p, float2* w1) {
    const int N = L / 2, QP = p->QP;
    hipStream_t st = p->stream;
    // rows along p3 (2N real, no padding) -> modes 0..N
    RET_IF((launch_r2c<L, false>(st, p->kerc, L * L, L, L, w1, QP, N + 1, -1.f, p->tw)));
    // along p2, in place
    RET_IF((launch_c2c<L, false, MAP_FIRST, EPI_STORE>(st, w1, w1, L, N + 1, (int64_t)L * QP, 1, QP,
                                                         (int64_t)L * QP, 1, QP, L, L, -1.f, p->tw)));
    // along p1, real part / (2N)^3 -> khat
    EpiArgs ep;
    ep.scale = 1.0 / ((double)L * (double)L * (double)L);
    return launch_c2c<L, false, MAP_FIRST, EPI_REAL>(st, w1, p->khat, L, N + 1, QP, 1, (int64_t)L * QP, QP, 1,
                                                     (int64_t)L * QP, L, L, -1.f, p->tw, ep);
}

// Kernel gridding transform, L = 4N: real grid g (index = position mod L) -> Ker on
// offsets (-N, N), circulant positions p1, p2 in [0, 2N), n3 in [0, N): chalf[p1][p2][n3].
template <int L>
hipError_t kergrid_passes(firm_plan p, const float* grid, float2* h1, float2* h2, float* chalf) {
    const int N = L / 4, N2 = 2 * N;
    hipStream_t st = p->stream;
    // axis 3: real rows of L -> modes n3 in [0, N), exp(+i) sign
    RET_IF((launch_r2c<L, false>(st, grid, L * L, L, L, h1, N, N, 1.f, p->tw)));
    // axis 2: h1[l1][l2][n3] -> h2[l1][p2][n3]
    RET_IF((launch_c2c<L, false, MAP_CIRC, EPI_STORE>(st, h1, h2, L, N, (int64_t)L * N, 1, N, (int64_t)N2 * N,
                                                        1, N, L, N2, 1.f, p->tw)));
    // axis 1: h2[l1][p2][n3] -> chalf[p1][p2][n3] = Re / phihat^3 + k0 term, wrap planes zero
    EpiArgs ep;
    ep.dec_e = p->deconv_ker;
    ep.dec_o = p->deconv_ker;
    ep.dec_c = p->deconv_ker;
    ep.wrap_o = N;
    ep.k0 = (float)p->ker_k0;
    return launch_c2c<L, false, MAP_CIRC, EPI_KER>(st, h2, chalf, N2, N, N, 1, (int64_t)N2 * N, N, 1,
                                                   (int64_t)N2 * N, L, N2, 1.f, p->tw, ep);
}

// Back-projection transform, L = 2N: complex grid (index = position mod L) -> N^3 centred
// modes, Re / phihat^3 + k = 0 term.
template <int L>
hipError_t atbgrid_passes(firm_plan p, const float2* grid, float2* j1, float2* j2, float* atb,
                          const double* k0dev) {
    const int N = L / 2;
    hipStream_t st = p->stream;
    // axis 3 (contiguous): rows of L -> centred N modes
    RET_IF((launch_c2c<L, true, MAP_CENTER, EPI_STORE>(st, grid, j1, 1, L * L, 0, L, 1, 0, N, 1, L, N, 1.f,
                                                         p->tw)));
    // axis 2: j1[l1][l2][i3] -> j2[l1][i2][i3]
    RET_IF((launch_c2c<L, false, MAP_CENTER, EPI_STORE>(st, j1, j2, L, N, (int64_t)L * N, 1, N,
                                                          (int64_t)N * N, 1, N, L, N, 1.f, p->tw)));
    // axis 1: j2[l1][i2][i3] -> atb[i1][i2][i3]
    EpiArgs ep;
    ep.dec_e = p->deconv_atb;
    ep.dec_o = p->deconv_atb;
    ep.dec_c = p->deconv_atb;
    ep.k0dev = k0dev;
    return launch_c2c<L, false, MAP_CENTER, EPI_ATB>(st, j2, atb, N, N, N, 1, (int64_t)N * N, N, 1,
                                                     (int64_t)N * N, L, N, 1.f, p->tw, ep);
}

// z = IFFT_N(d . FFT_N(r)) with dhalf = d / N^3 in [N][N][QPn] FFT order (q3 in [0, N/2]).
template <int L>
hipError_t precond_passes(firm_plan p, const float* dhalf, const float* r, float* z, const int* active,
                          double* partials) {
    const int N = L, H = N / 2 + 1, QPn = p->QPn;
    hipStream_t st = p->stream;
    RET_IF((launch_r2c<L, false, float>(st, r, N * N, N, N, p->S1, QPn, H, -1.f, p->tw, nullptr, nullptr, active)));
    RET_IF((launch_c2c<L, false, MAP_FIRST, EPI_STORE>(st, p->S1, p->S1, N, H, (int64_t)N * QPn, 1, QPn,
                                                         (int64_t)N * QPn, 1, QPn, N, N, -1.f, p->tw, EpiArgs(),
                                                         active)));
    RET_IF((launch_mid<L>(st, p->S1, dhalf, N, H, QPn, (int64_t)N * QPn, QPn, (int64_t)N * QPn, N, p->tw,
                          active)));
    RET_IF((launch_c2c<L, false, MAP_FIRST, EPI_STORE>(st, p->S1, p->S1, N, H, (int64_t)N * QPn, 1, QPn,
                                                         (int64_t)N * QPn, 1, QPn, N, N, 1.f, p->tw, EpiArgs(),
                                                         active)));
    if (partials)  // z and the block partials of <r, z>
        return launch_c2r<L, true, float>(st, p->S1, N * N, QPn, z, N, N, 1.f, 1.f, 0.f, r, p->tw, partials, active);
    return launch_c2r<L, false, float>(st, p->S1, N * N, QPn, z, N, N, 1.f, 1.f, 0.f, nullptr, p->tw);
}

}  // namespace

#define DISPATCH_L(Lval, call_tmpl, ...)                  \
    switch (Lval) {                                       \
        case 8: return call_tmpl<8>(__VA_ARGS__);         \
        case 16: return call_tmpl<16>(__VA_ARGS__);       \
        case 32: return call_tmpl<32>(__VA_ARGS__);       \
        case 64: return call_tmpl<64>(__VA_ARGS__);       \
        case 128: return call_tmpl<128>(__VA_ARGS__);     \
        case 256: return call_tmpl<256>(__VA_ARGS__);     \
        case 512: return call_tmpl<512>(__VA_ARGS__);     \
        case 1024: return call_tmpl<1024>(__VA_ARGS__);   \
        default: return hipErrorInvalidValue;             \
    }

hipError_t fft_apply_AtA(firm_plan p, const float* x, float* y, float lam) {
    DISPATCH_L(2 * p->N, apply_passes, p, x, nullptr, y, lam, nullptr, nullptr, nullptr);
}

hipError_t fft_apply_cg(firm_plan p, const float* r, float* pvec, float* q, float lam, const double* beta_dev,
                        const int* active, double* partials) {
    DISPATCH_L(2 * p->N, apply_passes, p, r, pvec, q, lam, beta_dev, active, partials);
}

hipError_t fft_khat_from_kerc(firm_plan p, float2* w1) { DISPATCH_L(2 * p->N, khat_passes, p, w1); }

hipError_t fft_apply_AtA64(firm_plan p, const double* x, double* y, double lam) {
    DISPATCH_L(2 * p->N, apply_passes64, p, x, y, lam);
}

hipError_t fft_khat64_from_kerc64(firm_plan p, const double* kerc64, double2* w1) {
    DISPATCH_L(2 * p->N, khat64_passes, p, kerc64, w1);
}

hipError_t fft_ker_grid(firm_plan p, const float* grid, float2* h1, float2* h2, float* chalf) {
    DISPATCH_L(4 * p->N, kergrid_passes, p, grid, h1, h2, chalf);
}

hipError_t fft_atb_grid(firm_plan p, const float2* grid, float2* j1, float2* j2, float* atb,
                        const double* k0term) {
    DISPATCH_L(2 * p->N, atbgrid_passes, p, grid, j1, j2, atb, k0term);
}

hipError_t fft_precond(firm_plan p, const float* dhalf, const float* r, float* z, const int* active,
                       double* partials) {
    DISPATCH_L(p->N, precond_passes, p, dhalf, r, z, active, partials);
}
