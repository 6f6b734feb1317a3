// 3D FFT passes of libfirm: the A*A product through the 2N circulant embedding
// (section 3.2, eq. embedding_circulant with eq. circ1 in three dimensions), the
// kernel spectrum, the gridding transforms and the Fourier-diagonal
// preconditioner.  Every pass transforms one axis of a 3D array with the
// register-resident pencil FFT of fft_core.h: each thread loads its 8 elements
// straight from HBM and stores its 8 results straight back, so zero padding,
// cropping, mode selection, the kernel multiply and the CG vector work sit in
// the loads and stores.
#include <hip/hip_ext.h>

#include <algorithm>

#include "fft_core.h"
#include "firm_internal.h"

namespace {

// Kernel-attached timing of the product's passes: when the calling thread has armed a pair of
// events, the next pass launch carries them in its dispatch (hipExtLaunchKernelGGL), so they
// hold that kernel's own start and end, without the gaps between launches that events
// recorded on the stream between passes would add.
thread_local hipEvent_t tl_pass_ev[2] = {nullptr, nullptr};

#define FIRM_PASS_LAUNCH(K, G, B, ST, ...)                                              \
    do {                                                                                \
        if (tl_pass_ev[0]) {                                                            \
            hipExtLaunchKernelGGL(K, G, B, 0, ST, tl_pass_ev[0], tl_pass_ev[1], 0, __VA_ARGS__); \
            tl_pass_ev[0] = tl_pass_ev[1] = nullptr;                                    \
        } else {                                                                        \
            hipLaunchKernelGGL(K, G, B, 0, ST, __VA_ARGS__);                            \
        }                                                                               \
    } while (0)

// arm the timing events of the next pass launch (no-op for ev == nullptr)
inline void arm_pass_events(hipEvent_t* ev, int pass) {
    if (!ev) return;
    tl_pass_ev[0] = ev[2 * pass];
    tl_pass_ev[1] = ev[2 * pass + 1];
}

template <class S> struct VecOf;
template <> struct VecOf<float> { using V = float2; };
template <> struct VecOf<double> { using V = double2; };

// Twiddle table copy to LDS in two halves: fetch() loads the thread's share into registers as
// the kernel's first global load, store() writes it to LDS after the kernel has issued its data
// loads, so that the table's L2 latency overlaps the loads from HBM instead of preceding them
// (a copy loop waits for its load before it can store).  The data loads between the two halves
// must carry no condition: the wait before the store counts outstanding loads, and across a
// conditional load the compiler can only wait for the data as well, which puts the store and
// barrier after the data instead of under it.
template <int NT, class V>
struct TwCopy {
    static constexpr int R = (FIRM_TWN + NT - 1) / NT;
    V r[R];
    __device__ __forceinline__ void fetch(const V* __restrict__ tw) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = (int)threadIdx.x + k * NT;
            if (i < FIRM_TWN) r[k] = tw[i];
        }
    }
    __device__ __forceinline__ void store(V* twl) const {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = (int)threadIdx.x + k * NT;
            if (i < FIRM_TWN) twl[i] = r[k];
        }
    }
};

// threads of a pencil workgroup keyed by one integer (L * 16 + sizeof(scalar)), so that the
// launch-bounds argument carries no comma
template <int LS>
struct FftThr {
    static constexpr int value = (LS % 16 == 8) ? FftCfg<LS / 16, double2>::THREADS : FftCfg<LS / 16, float2>::THREADS;
};

// Pencils per workgroup of the row passes (contiguous rows; the exchange buffer is pencil-major,
// so the pencil count changes no access pattern).  At L = 512 four pencils (256 threads, 26 KB of
// LDS with the twiddle table) let six workgroups share a CU where sixteen allowed two: their load,
// transform and store phases then overlap, and the two row passes of the N = 256 product run 7-8%
// faster (44.1 -> 40.8 and 47.7 -> 43.8 us, bit-identical results); two pencils are slower again.
#ifndef FIRM_ROWC512
#define FIRM_ROWC512 4
#endif
template <int L, class V>
struct RowCfg {
    static constexpr int C = (L == 512 && sizeof(V) == 8) ? FIRM_ROWC512 : FftCfg<L, V>::C;
    static constexpr int THREADS = C * L / 8;
};
template <int LS>
struct RowThr {
    static constexpr int value = (LS % 16 == 8) ? RowCfg<LS / 16, double2>::THREADS : RowCfg<LS / 16, float2>::THREADS;
};

// waves per SIMD that two workgroups of that size need (the VGPR budget of the middle pass)
template <int LS>
struct FftTwoBlocks {
    static constexpr int value = FftThr<LS>::value / 128;
};

enum MapKind { MAP_FIRST = 0, MAP_CIRC = 1, MAP_CENTER = 2 };
enum EpiKind { EPI_STORE = 0, EPI_REAL_BLOCKED = 1, EPI_KER = 2, EPI_ATB = 3 };

struct EpiArgs {
    double scale = 1.0;
    const float* dec_e = nullptr;   // per output index along the transformed axis
    const float* dec_o = nullptr;   // per outer index
    const float* dec_c = nullptr;   // per column
    int wrap_o = -1;                // outer index whose plane is zero (circulant wrap)
    float k0 = 0.f;                 // constant added (EPI_KER)
    const double* k0dev = nullptr;  // constant added, device scalar (EPI_ATB)
};

// Output index of transform bin e for a mode map; -1 drops the bin.  MAP_CIRC keeps the
// offsets (-N, N) of an L-point transform (n_out = 2N) in circulant order; its wrap slot N
// is written as zero by the thread that holds bin N.
template <int MAP>
__device__ __forceinline__ int out_index(int e, int L, int n_out, bool& zero) {
    zero = false;
    if constexpr (MAP == MAP_FIRST) {
        return e < n_out ? e : -1;
    } else if constexpr (MAP == MAP_CIRC) {
        const int N = n_out >> 1;
        if (e < N) return e;
        if (e == N) { zero = true; return N; }
        return e > L - N ? e - L + n_out : -1;
    } else {  // centred modes -n_out/2 .. n_out/2 - 1
        const int h = n_out >> 1;
        if (e < h) return e + h;
        return e >= L - h ? e - L + h : -1;
    }
}

__device__ __forceinline__ bool cg_inactive(const int* active) { return active && *active == 0; }

// Non-temporal (streaming) loads of 2-, 4- and 8-byte values and stores of 4- and 8-byte values;
// wider ones are plain.  Every
// pass of the product reads its input and writes its output once, so none of it is worth
// caching: at N = 256 the five passes take 397 instead of 433 us per product with these.
template <class T>
__device__ __forceinline__ T ld_nt(const T* p) {
    if constexpr (sizeof(T) == 8) {
        const long long b = __builtin_nontemporal_load(reinterpret_cast<const long long*>(p));
        return *reinterpret_cast<const T*>(&b);
    } else if constexpr (sizeof(T) == 4) {
        const int b = __builtin_nontemporal_load(reinterpret_cast<const int*>(p));
        return *reinterpret_cast<const T*>(&b);
    } else if constexpr (sizeof(T) == 2) {
        const short b = __builtin_nontemporal_load(reinterpret_cast<const short*>(p));
        return *reinterpret_cast<const T*>(&b);
    } else {
        return *p;
    }
}
template <class T>
__device__ __forceinline__ void st_nt(const T& v, T* p) {
    if constexpr (sizeof(T) == 8)
        __builtin_nontemporal_store(*reinterpret_cast<const long long*>(&v), reinterpret_cast<long long*>(p));
    else if constexpr (sizeof(T) == 4)
        __builtin_nontemporal_store(*reinterpret_cast<const int*>(&v), reinterpret_cast<int*>(p));
    else
        *p = v;
}

// Block sum of a double; result valid in thread 0.
template <int THREADS>
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
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
template <int L, bool PRO, class S, bool HIN>
__global__ void __launch_bounds__(RowThr<L * 16 + (int)sizeof(S)>::value)
k_rows_r2c(const S* __restrict__ src, int nrows, int in_pitch, int n_in, typename VecOf<S>::V* __restrict__ dst,
           int out_pitch, int n_keep, S sg, const typename VecOf<S>::V* __restrict__ tw, S* pvec,
           const double* beta_dev, const int* active) {
    // HIN: rows zero-padded from L/2 (known at compile time: the first stage's zero inputs fold)
    using V = typename VecOf<S>::V;
    constexpr int C = RowCfg<L, V>::C, T = L / 8;
    using P = Pen<L, C, true>;
    constexpr bool TWL = sizeof(S) == 4;
    __shared__ V lds[P::LDS];
    __shared__ V twl[TWL ? FIRM_TWN : 1];
    if (cg_inactive(active)) return;
    TwCopy<P::NT, V> twc;
    if constexpr (TWL) twc.fetch(tw);
    const V* twp = TWL ? twl : tw;
    if (HIN) n_in = L / 2;
    const int c = P::c(), j = P::j();
    const int pr = blockIdx.x * C + c;
    const bool valid = pr < (nrows >> 1);
    S beta = 0;
    if (PRO) beta = (S)(*beta_dev);
    V v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int e = j + t * T;
        S a = 0, b = 0;
        if (!(HIN && t >= 4) && valid && e < n_in) {
            const int64_t g = (int64_t)(2 * pr) * in_pitch + e;
            a = ld_nt(src + g);
            b = ld_nt(src + g + in_pitch);
            if (PRO) {
                a += beta * pvec[g];
                b += beta * pvec[g + in_pitch];
                pvec[g] = a;
                pvec[g + in_pitch] = b;
            }
        }
        v[t] = mkv<V>(a, b);
    }
    if constexpr (TWL) {
        twc.store(twl);
        __syncthreads();  // the twiddle table is in place
    }
    fft_reg<L, C, true>(v, lds, twp, sg);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 8; ++t) lds[P::idx(j + t * T, c)] = v[t];
    __syncthreads();
    if (!valid) return;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int q = j + t * T;
        if (q < n_keep) {
            const V Z = lds[P::idx(q, c)];
            const V Zm = lds[P::idx((L - q) & (L - 1), c)];
            const V D = mkv<V>((S)0.5 * (Z.x - Zm.x), (S)0.5 * (Z.y + Zm.y));   // (Z - conj Zm)/2
            // plain stores: the half spectra of a product's first pass (135 MB at N = 256) stay in
            // the memory-side cache for the next pass, which reads them 5 us sooner than after
            // streaming stores; the larger arrays of the other passes do not fit it
            dst[(int64_t)(2 * pr) * out_pitch + q] = mkv<V>((S)0.5 * (Z.x + Zm.x), (S)0.5 * (Z.y - Zm.y));
            dst[(int64_t)(2 * pr + 1) * out_pitch + q] = mkv<V>(D.y, -D.x);       // D / i
        }
    }
}

// CG step fused into the last pass of the product q = (A*A + lam) p: with alpha already formed,
// x += alpha p and r -= alpha q (FP64 arithmetic, FP32 storage), and the block partials of
// ||r||^2; q itself is not stored.
struct CgStep {
    float* x;
    const float* p;
    float* r;
    const double* alpha;
};

// Half spectra (modes 0..L/2 of two real rows) -> real rows, first n_out samples.
// y = scale * x + lam * xadd.  DOT: also a block partial of sum(xadd * y) in FP64.
// STEP: y is the CG product q, consumed by the CG step (dst unused), partials of ||r||^2.
template <int L, bool DOT, class S, bool HOUT, bool STEP = false>
__global__ void __launch_bounds__(RowThr<L * 16 + (int)sizeof(S)>::value)
k_rows_c2r(const typename VecOf<S>::V* __restrict__ src, int nrows, int in_pitch, S* __restrict__ dst, int out_pitch,
           int n_out, S sg, S scale, S lam, const S* __restrict__ xadd, const typename VecOf<S>::V* __restrict__ tw,
           double* partials, const int* active, CgStep step) {
    using V = typename VecOf<S>::V;
    constexpr int C = RowCfg<L, V>::C, T = L / 8, NT = RowCfg<L, V>::THREADS;
    using P = Pen<L, C, true>;
    constexpr bool TWL = sizeof(S) == 4;
    static_assert(P::LDS * sizeof(V) >= (NT / 64) * sizeof(double), "reduction scratch");
    __shared__ V lds[P::LDS];  // exchange buffer; after the transform, the DOT reduction's scratch
    __shared__ V twl[TWL ? FIRM_TWN : 1];
    if (cg_inactive(active)) return;
    TwCopy<NT, V> twc;
    if constexpr (TWL) twc.fetch(tw);
    const V* twp = TWL ? twl : tw;
    const int c = P::c(), j = P::j();
    const int pr = blockIdx.x * C + c;
    const bool valid = pr < (nrows >> 1);
    const int prl = valid ? pr : (nrows >> 1) - 1;  // a pencil that does not exist loads the last one
    V v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int e = j + t * T;
        const int m = e <= L / 2 ? e : L - e;
        const V Ya = src[(int64_t)(2 * prl) * in_pitch + m];
        const V Yb = src[(int64_t)(2 * prl + 1) * in_pitch + m];
        const V z = e <= L / 2 ? mkv<V>(Ya.x - Yb.y, Ya.y + Yb.x)     // Ya + i Yb
                               : mkv<V>(Ya.x + Yb.y, Yb.x - Ya.y);    // conj Ya + i conj Yb
        v[t] = valid ? z : mkv<V>(0, 0);
    }
    if constexpr (TWL) {
        twc.store(twl);
        __syncthreads();  // the twiddle table is in place
    }
    fft_reg<L, C, true>(v, lds, twp, sg);
    double acc = 0.0;
    double alpha = 0.0;
    if constexpr (STEP) alpha = *step.alpha;
    if (valid) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = j + t * T;
            if (HOUT ? t < 4 : e < n_out) {  // HOUT: the first L/2 samples (n_out = L/2)
#pragma unroll
                for (int rr = 0; rr < 2; ++rr) {
                    const int64_t g = (int64_t)(2 * pr + rr) * out_pitch + e;
                    S y = scale * (rr ? v[t].y : v[t].x);
                    if constexpr (STEP) {
                        const float pv = ld_nt(step.p + g), xv = ld_nt(step.x + g), rv0 = ld_nt(step.r + g);
                        st_nt((float)((double)xv + alpha * (double)pv), step.x + g);
                        const float rv = (float)((double)rv0 - alpha * (double)y);
                        st_nt(rv, step.r + g);
                        acc += (double)rv * (double)rv;
                        continue;
                    }
                    if (xadd) {
                        const S xv = xadd[g];
                        y += lam * xv;
                        if (DOT) acc += (double)xv * (double)y;
                    }
                    st_nt(y, dst + g);
                }
            }
        }
    }
    if (DOT || STEP) {
        __syncthreads();  // every wavefront has finished reading the exchange buffer
        const double s = block_sum<NT>(acc, reinterpret_cast<double*>(lds));
        if (threadIdx.x == 0) partials[blockIdx.x] = s;
    }
}


// First pass of a preconditioned CG iteration with the preconditioner's last pass fused in.
// In: the half spectra of z = F^{-1}(d . F r) along i3 (the preconditioner's output before its
// inverse row transform, S1 [row][q3 <= N/2], pitch qpn).  Per pencil (rows 2 pr and 2 pr + 1 of
// the N^2 rows along i3, packed as one complex sequence): the N-point inverse transform gives z;
// then p = z + beta p (stored); then the 2N-point forward transform of p's rows zero-padded from N,
// as two N-point transforms: its even outputs X(2m) are the N-point DFT of p, its odd outputs
// X(2m+1) that of p(e) exp(-2 pi i e / 2N); their half spectra go to dst (pitch out_pitch, modes
// 0..N), as the product's first pass writes them.  z is never stored.
constexpr int PZC = 8;  // pencils per workgroup
template <int N>
__global__ void __launch_bounds__(PZC * N / 8) k_rows_pz(const float2* __restrict__ S1, int qpn, float* pvec,
                                                      const double* __restrict__ beta_dev, float2* __restrict__ dst,
                                                      int out_pitch, const float2* __restrict__ tw, const int* active) {
    using V = float2;
    constexpr int C = PZC, T = N / 8, NT = C * T, L = 2 * N;
    using P = Pen<N, C, true>;
    static_assert(FIRM_TWN % L == 0, "twist from the twiddle table");
    __shared__ V lds[2 * P::LDS];  // the transforms' exchange buffer (first half), then both spectra
    __shared__ V twl[FIRM_TWN];
    if (cg_inactive(active)) return;
    TwCopy<NT, V> twc;
    twc.fetch(tw);
    const int c = P::c(), j = P::j();
    const int pr = blockIdx.x * C + c;  // the grid covers the N^2 / 2 pencils exactly
    const float beta = (float)(*beta_dev);
    V v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int e = j + t * T;
        const int m = e <= N / 2 ? e : N - e;
        const V Ya = S1[(int64_t)(2 * pr) * qpn + m];
        const V Yb = S1[(int64_t)(2 * pr + 1) * qpn + m];
        v[t] = e <= N / 2 ? mkv<V>(Ya.x - Yb.y, Ya.y + Yb.x)    // Ya + i Yb
                          : mkv<V>(Ya.x + Yb.y, Yb.x - Ya.y);   // conj Ya + i conj Yb
    }
    twc.store(twl);
    __syncthreads();  // the twiddle table is in place
    fft_reg<N, C, true>(v, lds, twl, 1.f);  // z of row 2 pr (real part) and 2 pr + 1 (imaginary part)
    V w[8], u[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int e = j + t * T;
        const int64_t g = (int64_t)(2 * pr) * N + e;
        const float a = v[t].x + beta * pvec[g], b = v[t].y + beta * pvec[g + N];
        pvec[g] = a;
        pvec[g + N] = b;
        w[t] = mkv<V>(a, b);
        u[t] = c_mul(w[t], twl[e * (FIRM_TWN / L)]);  // times exp(-2 pi i e / 2N)
    }
    fft_reg<N, C, true>(w, lds, twl, -1.f);  // X(2m), m = j + T t
    fft_reg<N, C, true>(u, lds, twl, -1.f);  // X(2m + 1)
    __syncthreads();  // every wavefront has read the exchange buffer
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int m = j + t * T;
        lds[P::idx(m, c)] = w[t];
        lds[P::LDS + P::idx(m, c)] = u[t];
    }
    __syncthreads();
    // half spectra of the two rows, modes q in [0, N]: from X(q) and X(2N - q), both of q's parity
#pragma unroll
    for (int t = 0; t <= 8; ++t) {
        const int q = j + t * T;
        if (q <= N) {
            const int h = q & 1;
            const int mq = q >> 1, mm = (N - ((q + h) >> 1)) & (N - 1);
            const V Z = lds[h * P::LDS + P::idx(mq, c)];
            const V Zm = lds[h * P::LDS + P::idx(mm, c)];
            const V D = mkv<V>(0.5f * (Z.x - Zm.x), 0.5f * (Z.y + Zm.y));  // (Z - conj Zm) / 2
            // plain stores, as the product's first pass: the next pass finds them in the memory-side cache
            dst[(int64_t)(2 * pr) * out_pitch + q] = mkv<V>(0.5f * (Z.x + Zm.x), 0.5f * (Z.y - Zm.y));
            dst[(int64_t)(2 * pr + 1) * out_pitch + q] = mkv<V>(D.y, -D.x);  // D / i
        }
    }
}

// The Fourier-diagonal preconditioner's outer passes for N <= 64, one workgroup per i1 slab
// (the N x N slab and its N x (N/2 + 1) half spectrum fit LDS).  FWD: rows along i3 real to
// half spectrum (two real rows per complex pencil, as k_rows_r2c), then columns along i2
// forward (as k_cols), written to S1[i1][q2][q3]; !FWD: columns along q2 inverse, then rows
// half spectrum to real (as k_rows_c2r), written to z[i1][i2][i3].  Two launches instead of
// four: at these sizes a launch costs its few microseconds whatever it moves.
template <int L, bool FWD>
__global__ void __launch_bounds__(FftThr<L * 16 + 4>::value)
k_precond_slab(const float* __restrict__ r, float2* __restrict__ S1, float* __restrict__ z, int QPn,
               const float2* __restrict__ tw, const int* active) {
    using V = float2;
    constexpr int N = L, H = N / 2 + 1, C = FftCfg<L, V>::C, T = L / 8, NT = FftCfg<L, V>::THREADS;
    static_assert(N / 2 <= C, "the row pencils of a slab are one chunk");
    using PR = Pen<L, C, true>;   // rows: lanes along elements
    using PC = Pen<L, C, false>;  // columns: lanes along columns
    constexpr int XL = PR::LDS > PC::LDS ? PR::LDS : PC::LDS;
    __shared__ V lds[XL];
    __shared__ V sl[N * H];  // the slab's half spectrum [i2 or q2][q3]
    __shared__ V twl[FIRM_TWN];
    if (cg_inactive(active)) return;
    for (int i = threadIdx.x; i < FIRM_TWN; i += NT) twl[i] = tw[i];
    const int64_t i1 = blockIdx.x;
    const int c = PR::c(), j = PR::j();  // row pencil c = rows (2c, 2c + 1)
    const bool rv = c < N / 2;
    const int cc = PC::c(), jj = PC::j();
    V v[8];
    if constexpr (FWD) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = j + t * T;
            v[t] = rv ? mkv<V>(r[(i1 * N + 2 * c) * N + e], r[(i1 * N + 2 * c + 1) * N + e]) : mkv<V>(0, 0);
        }
        __syncthreads();  // the twiddle table is in place
        fft_reg<L, C, true>(v, lds, twl, -1.f);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 8; ++t) lds[PR::idx(j + t * T, c)] = v[t];
        __syncthreads();
        if (rv) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int q = j + t * T;
                if (q < H) {
                    const V Z = lds[PR::idx(q, c)];
                    const V Zm = lds[PR::idx((L - q) & (L - 1), c)];
                    const V D = mkv<V>(0.5f * (Z.x - Zm.x), 0.5f * (Z.y + Zm.y));     // (Z - conj Zm)/2
                    sl[(2 * c) * H + q] = mkv<V>(0.5f * (Z.x + Zm.x), 0.5f * (Z.y - Zm.y));
                    sl[(2 * c + 1) * H + q] = mkv<V>(D.y, -D.x);                        // D / i
                }
            }
        }
        __syncthreads();
        for (int c0 = 0; c0 < H; c0 += C) {
            const int col = c0 + cc;
            const bool cv = col < H;
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = cv ? sl[(jj + t * T) * H + col] : mkv<V>(0, 0);
            fft_reg<L, C, false>(v, lds, twl, -1.f);
            if (cv) {
#pragma unroll
                for (int t = 0; t < 8; ++t) S1[(i1 * N + jj + t * T) * QPn + col] = v[t];
            }
            __syncthreads();
        }
    } else {
        __syncthreads();  // the twiddle table is in place
        for (int c0 = 0; c0 < H; c0 += C) {
            const int col = c0 + cc;
            const bool cv = col < H;
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = cv ? S1[(i1 * N + jj + t * T) * QPn + col] : mkv<V>(0, 0);
            fft_reg<L, C, false>(v, lds, twl, 1.f);
            if (cv) {
#pragma unroll
                for (int t = 0; t < 8; ++t) sl[(jj + t * T) * H + col] = v[t];
            }
            __syncthreads();
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = j + t * T;
            const int m = e <= L / 2 ? e : L - e;
            const V Ya = rv ? sl[(2 * c) * H + m] : mkv<V>(0, 0);
            const V Yb = rv ? sl[(2 * c + 1) * H + m] : mkv<V>(0, 0);
            v[t] = e <= L / 2 ? mkv<V>(Ya.x - Yb.y, Ya.y + Yb.x)     // Ya + i Yb
                              : mkv<V>(Ya.x + Yb.y, Yb.x - Ya.y);    // conj Ya + i conj Yb
        }
        fft_reg<L, C, true>(v, lds, twl, 1.f);
        if (rv) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int e = j + t * T;
                z[(i1 * N + 2 * c) * N + e] = v[t].x;
                z[(i1 * N + 2 * c + 1) * N + e] = v[t].y;
            }
        }
    }
}

// Pencil of the middle pass over nouter rows of ncols columns, C pencils per block.  When C
// does not divide ncols, the ncols % C columns of every row's last, partial group are packed C
// to a block (pencils of consecutive rows), in the first blocks of the grid (started first:
// their accesses do not coalesce); every later block takes one full group (o, g).  Without
// this, each row's last block would run both transforms for a few pencils.  (The one-transform
// column passes keep one block per group: there the uncoalesced tail accesses cost more than
// the idle pencils.)  Out: the row o, the column group g, the column cc within it, and whether
// the pencil exists (o is clamped to a valid row when it does not).
template <int C>
__device__ __forceinline__ void tail_packed_pencil(int nouter, int ncols, int c, int& o, int& g, int& cc, bool& valid) {
    const int rtail = ncols % C, ngm = ncols / C;
    const int ntail = (nouter * rtail + C - 1) / C;
    if ((int)blockIdx.x >= ntail) {
        const int b = blockIdx.x - ntail;
        o = b / ngm;
        g = b - o * ngm;
        cc = c;
        valid = true;
    } else {
        const int pi = blockIdx.x * C + c;
        o = pi / rtail;
        cc = pi - o * rtail;
        g = ngm;
        valid = o < nouter;
        if (!valid) o = nouter - 1;
    }
}

// blocks of the middle pass: full groups plus the packed tail columns
template <int C>
inline int tail_packed_blocks(int nouter, int ncols) {
    return nouter * (ncols / C) + (nouter * (ncols % C) + C - 1) / C;
}
// Complex pencils along one axis.  Block -> (outer o, column group); CONTIG means the
// transformed axis is contiguous (lanes along elements), otherwise lanes run along columns.
template <int L, bool CONTIG, int MAP, int EPI, class S, int PADK>
__global__ void __launch_bounds__(FftThr<L * 16 + (int)sizeof(S)>::value)
k_cols(const typename VecOf<S>::V* __restrict__ src, void* __restrict__ dstv, int ncols, int64_t s_outer,
       int64_t s_col, int64_t s_elem, int64_t d_outer, int64_t d_col, int64_t d_elem, int64_t s_group,
       int64_t d_group, int n_in, int n_out, S sg, const typename VecOf<S>::V* __restrict__ tw, EpiArgs ep,
       const int* active) {
    // PADK 1: input zero-padded from L/2; 2: only the first L/2 outputs kept (MAP_FIRST); known at
    // compile time so that the first / last stage folds
    using V = typename VecOf<S>::V;
    constexpr int C = FftCfg<L, V>::C, T = L / 8;
    using P = Pen<L, C, CONTIG>;
    constexpr bool TWL = sizeof(S) == 4 && !CONTIG;
    __shared__ V lds[P::LDS];
    __shared__ V twl[TWL ? FIRM_TWN : 1];
    if (cg_inactive(active)) return;
    TwCopy<P::NT, V> twc;
    if constexpr (TWL) twc.fetch(tw);
    const V* twp = TWL ? twl : tw;
    if (PADK == 1) n_in = L / 2;
    if (PADK == 2) n_out = L / 2;
    const int ng = (ncols + C - 1) / C;
    const int c = P::c(), j = P::j();
    const int o = blockIdx.x / ng;
    const int g = blockIdx.x - o * ng;
    const int col = g * C + c;
    const bool valid = col < ncols;
    const V* s0 = src + o * s_outer + (int64_t)g * s_group + (int64_t)c * s_col;
    V v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int e = j + t * T;
        v[t] = (!(PADK == 1 && t >= 4) && valid && e < n_in) ? ld_nt(s0 + e * s_elem) : mkv<V>(0, 0);
    }
    if constexpr (TWL) {
        twc.store(twl);
        __syncthreads();  // the twiddle table is in place
    }
    fft_reg<L, C, CONTIG>(v, lds, twp, sg);
    if (!valid) return;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        if (PADK == 2 && t >= 4) continue;
        bool zero;
        const int u = out_index<MAP>(j + t * T, L, n_out, zero);
        if (u < 0) continue;
        const V val = zero ? mkv<V>(0, 0) : v[t];
        const int64_t gi = o * d_outer + (int64_t)g * d_group + (int64_t)c * d_col + (int64_t)u * d_elem;
        if constexpr (EPI == EPI_STORE) {
            st_nt(val, reinterpret_cast<V*>(dstv) + gi);
        } else if constexpr (EPI == EPI_REAL_BLOCKED) {
            // spectrum in the layout read by k_mid: [outer][column group][element][C]
            reinterpret_cast<S*>(dstv)[(((int64_t)o * ng + g) * L + u) * C + c] = val.x * (S)ep.scale;
        } else if constexpr (EPI == EPI_KER) {
            float r = 0.f;
            if (!zero && o != ep.wrap_o) r = (float)val.x * ep.dec_e[u] * ep.dec_o[o] * ep.dec_c[col] + ep.k0;
            reinterpret_cast<float*>(dstv)[gi] = r;
        } else {  // EPI_ATB
            reinterpret_cast<float*>(dstv)[gi] =
                (float)val.x * ep.dec_e[u] * ep.dec_o[o] * ep.dec_c[col] + (float)(*ep.k0dev);
        }
    }
}

// ---- 16-bit spectrum (option khat_bf16) ----------------------------------------------
// Shell of a frequency of the blocked half spectrum: the rounded radius of the signed
// frequency (q1, q2 in [0, L), q3 in [0, L/2]).  Encoder and product evaluate the same
// integer expression, so both see the same shell.
__device__ __forceinline__ int khat_shell(int q1, int q2, int q3, int L) {
    const int a = q1 < L / 2 ? q1 : q1 - L, b = q2 < L / 2 ? q2 : q2 - L;
    return (int)floorf(sqrtf((float)(a * a + b * b + q3 * q3)) + 0.5f);
}

constexpr int KSH_MAX = 448;  // shells at N <= 256: round(sqrt(3) N) + 1 <= 445

// blocked element i -> (q1, q2, q3); false for the padding columns q3 > N
__device__ __forceinline__ bool khat_blocked_q(int64_t i, int L, int C, int ng, int& q1, int& q2, int& q3) {
    const int c = (int)(i % C);
    q1 = (int)((i / C) % L);
    const int g = (int)((i / ((int64_t)C * L)) % ng);
    q2 = (int)(i / ((int64_t)C * L * ng));
    q3 = g * C + c;
    return q3 <= L / 2;
}

// Fourier-space damping term of the multiplier: kh(q) += coef w(q)^order, with
// w(q) = sum_d 4 sin^2(pi q_d / L) the symbol of the 7-point negative Laplacian on the L-periodic
// grid (q in FFT order; the symbol is even, so the axis order of the blocked layout is immaterial).
template <class S>
__global__ void __launch_bounds__(256) k_khat_reg(S* __restrict__ kh, int L, int C, int ng, double coef, int order) {
    const int64_t n = (int64_t)L * ng * L * C;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        int q1, q2, q3;
        if (!khat_blocked_q(i, L, C, ng, q1, q2, q3)) continue;
        const double s1 = sin(M_PI * q1 / L), s2 = sin(M_PI * q2 / L), s3 = sin(M_PI * q3 / L);
        const double w = 4.0 * (s1 * s1 + s2 * s2 + s3 * s3);
        double wp = 1.0;
        for (int k = 0; k < order; ++k) wp *= w;
        kh[i] = (S)((double)kh[i] + coef * wp);
    }
}

// pass 1: per-shell sum and count (block-private in LDS, then added to the global totals)
__global__ void __launch_bounds__(256) k_khat_shell_sum(const float* __restrict__ kh, int L, int C, int ng,
                                                        double* __restrict__ gsum, unsigned* __restrict__ gcnt) {
    __shared__ double ssum[KSH_MAX];
    __shared__ unsigned scnt[KSH_MAX];
    for (int i = threadIdx.x; i < KSH_MAX; i += 256) { ssum[i] = 0.0; scnt[i] = 0u; }
    __syncthreads();
    const int64_t n = (int64_t)L * ng * L * C;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        int q1, q2, q3;
        if (!khat_blocked_q(i, L, C, ng, q1, q2, q3)) continue;
        const int sh = khat_shell(q1, q2, q3, L);
        atomicAdd(&ssum[sh], (double)kh[i]);
        atomicAdd(&scnt[sh], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < KSH_MAX; i += 256)
        if (scnt[i]) {
            atomicAdd(&gsum[i], ssum[i]);
            atomicAdd(&gcnt[i], scnt[i]);
        }
}

// pass 2: per-shell largest deviation from the shell mean (non-negative floats compare as
// their bit patterns)
__global__ void __launch_bounds__(256) k_khat_shell_dev(const float* __restrict__ kh, int L, int C, int ng,
                                                        const double* __restrict__ gsum,
                                                        const unsigned* __restrict__ gcnt,
                                                        unsigned* __restrict__ gdev) {
    __shared__ float smu[KSH_MAX];
    __shared__ unsigned sdev[KSH_MAX];
    for (int i = threadIdx.x; i < KSH_MAX; i += 256) {
        smu[i] = gcnt[i] ? (float)(gsum[i] / gcnt[i]) : 0.f;
        sdev[i] = 0u;
    }
    __syncthreads();
    const int64_t n = (int64_t)L * ng * L * C;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        int q1, q2, q3;
        if (!khat_blocked_q(i, L, C, ng, q1, q2, q3)) continue;
        const int sh = khat_shell(q1, q2, q3, L);
        atomicMax(&sdev[sh], __float_as_uint(fabsf(kh[i] - smu[sh])));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < KSH_MAX; i += 256)
        if (sdev[i]) atomicMax(&gdev[i], sdev[i]);
}

// pass 3: the per-shell (offset, scale) pairs
__global__ void k_khat_shell_tab(const double* __restrict__ gsum, const unsigned* __restrict__ gcnt,
                                 const unsigned* __restrict__ gdev, float2* __restrict__ tab) {
    for (int i = threadIdx.x; i < KSH_MAX; i += blockDim.x) {
        const float dev = __uint_as_float(gdev[i]);
        tab[i] = make_float2(gcnt[i] ? (float)(gsum[i] / gcnt[i]) : 0.f, dev > 0.f ? dev : 1.f);
    }
}

// pass 4: BF16 codes of (K^ - offset) / scale (or of K^ itself, tab null), rounded to nearest
// even; padding columns 0
__global__ void __launch_bounds__(256) k_khat_encode16(const float* __restrict__ kh, int L, int C, int ng,
                                                       const float2* __restrict__ tab, uint16_t* __restrict__ k16) {
    const int64_t n = (int64_t)L * ng * L * C;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        int q1, q2, q3;
        uint16_t code = 0;
        if (khat_blocked_q(i, L, C, ng, q1, q2, q3)) {
            const float2 ms = tab ? tab[khat_shell(q1, q2, q3, L)] : make_float2(0.f, 1.f);
            const uint32_t u = __float_as_uint((kh[i] - ms.x) / ms.y);
            code = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
        }
        k16[i] = code;
    }
}

// Middle pass of the product: along axis 1, zero-pad the first n_in entries, forward
// transform, multiply by the real spectrum (blocked layout [outer][group][element][C]),
// inverse transform, keep the first n_in.
// K16: the spectrum is the 16-bit form of the option khat_bf16 (BF16 codes b, value
// mu(shell) + sc(shell) b with the per-shell pairs in shtab, or b itself when shtab is null).
// DOT (a half spectrum, columns q3 in [0, ncols - 1]): also a block partial of
// <x, y> = sum over the full spectrum of (K^ + kadd) |X^|^2 (Parseval, unnormalised transforms),
// the first and last columns once and the others twice (X^(-q) = conj X^(q)).
template <int L, class S, bool HALF, bool K16, bool DOT>
__global__ void __launch_bounds__(FftThr<L * 16 + (int)sizeof(S)>::value)
k_mid(typename VecOf<S>::V* __restrict__ data, const void* __restrict__ specv, const float2* __restrict__ shtab,
      S kadd, int nouter, int ncols, int64_t s_outer, int64_t s_elem, int64_t s_group, int n_in,
      const typename VecOf<S>::V* __restrict__ tw, const int* active, double* __restrict__ dotp) {
    // HALF: the pencils are zero-padded (n_in = L / 2) and only their first half is kept, which
    // the compiler folds into the first and last stages
    using V = typename VecOf<S>::V;
    constexpr int C = FftCfg<L, V>::C, T = L / 8;
    using P = Pen<L, C, false>;
    // FP32: the twiddle table is copied to LDS (short-latency reads, fewer live registers); the
    // FP64 form keeps it in global memory (its registers already bound the occupancy)
    constexpr bool TWL = sizeof(S) == 4;
    __shared__ V lds[P::LDS];
    __shared__ V twl[TWL ? FIRM_TWN : 1];
    __shared__ double red[DOT ? P::NT / 64 : 1];
    if (cg_inactive(active)) return;
    // ULD: HALF with a 32-bit spectrum loads its data without a condition, so the FP32 table
    // copy can be split around the loads (the 16-bit form keeps both: its shell-table lookups
    // are conditional, and the branch-free loads cost it the registers of its second workgroup)
    constexpr bool ULD = HALF && !K16;
    constexpr bool TWS = TWL && ULD;
    if (TWL && !TWS)
        for (int i = threadIdx.x; i < FIRM_TWN; i += P::NT) twl[i] = tw[i];
    TwCopy<P::NT, V> twc;
    if constexpr (TWS) twc.fetch(tw);
    const V* twp = TWL ? twl : tw;
    const int nin = HALF ? L / 2 : n_in;
    const int ng = (ncols + C - 1) / C;  // column groups of the data and spectrum layouts
    const int c = P::c(), j = P::j();
    int o, g, cc;
    bool valid;
    tail_packed_pencil<C>(nouter, ncols, c, o, g, cc, valid);
    const int col = g * C + cc;
    V* d0 = data + o * s_outer + (int64_t)g * s_group + cc;
    const int64_t kofs = ((int64_t)o * ng + g) * L * C + cc;
    V v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int e = j + t * T;
        if (HALF && t >= 4) {
            v[t] = mkv<V>(0, 0);  // e >= L / 2
        } else if (ULD) {
            // e < L / 2 = nin, and a pencil that does not exist has the address of one that
            // does (tail_packed_pencil), so the load needs no branch
            const V w = ld_nt(d0 + e * s_elem);
            v[t] = valid ? w : mkv<V>(0, 0);
        } else {
            v[t] = (valid && e < nin) ? ld_nt(d0 + e * s_elem) : mkv<V>(0, 0);
        }
    }
    // the spectrum values are loaded before the forward transform, which hides their latency
    S kv[8];
    if constexpr (!K16) {
        const S* k0 = reinterpret_cast<const S*>(specv) + kofs;
#pragma unroll
        for (int t = 0; t < 8; ++t) kv[t] = ld_nt(k0 + (j + t * T) * C);
    } else {
        const uint16_t* k0 = reinterpret_cast<const uint16_t*>(specv) + kofs;
        uint16_t raw[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) raw[t] = ld_nt(k0 + (j + t * T) * C);
        if (shtab) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const float2 ms = shtab[valid ? khat_shell(j + t * T, o, col, L) : 0];
                kv[t] = (S)(ms.x + ms.y * __uint_as_float((uint32_t)raw[t] << 16));
            }
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) kv[t] = (S)__uint_as_float((uint32_t)raw[t] << 16);
        }
    }
    if constexpr (TWS) twc.store(twl);
    if (TWL) __syncthreads();  // the twiddle table is in place
    fft_reg<L, C, false>(v, lds, twp, (S)-1);
    // the thread's 8 terms in FP32 (as the product itself), the block sum in FP64
    S acc8 = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const S k = kv[t] + kadd;
        if (DOT) acc8 += k * (v[t].x * v[t].x + v[t].y * v[t].y);
        v[t] = mkv<V>(v[t].x * k, v[t].y * k);
    }
    if constexpr (DOT) {  // pencils that do not exist hold zeros
        double acc = (double)acc8 * ((col == 0 || col == ncols - 1) ? 1.0 : 2.0);
        acc = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    }
    fft_reg<L, C, false>(v, lds, twp, (S)1);
    if constexpr (DOT) {
        // the inverse transform's LDS exchanges (lengths of 16 and more) put barriers between
        // every wave's partial and this read, so the block sum needs no barrier of its own
        if constexpr (L < 16) __syncthreads();
        if (threadIdx.x == 0) {
            double sum = 0.0;
            for (int w = 0; w < P::NT / 64; ++w) sum += red[w];
            dotp[blockIdx.x] = sum;
        }
    }
    if (!valid) return;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int e = j + t * T;
        if (HALF ? t < 4 : e < nin) st_nt(v[t], d0 + e * s_elem);
    }
}

// blocked spectrum [outer][group][element][C] -> dense [element][outer][n_cols]
template <class S>
__global__ void k_unblock(const S* __restrict__ blk, float* __restrict__ out, int L, int nouter, int ncols, int C) {
    const int ng = (ncols + C - 1) / C;
    const int64_t tot = (int64_t)L * nouter * ncols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int col = (int)(i % ncols), o = (int)((i / ncols) % nouter), e = (int)(i / ((int64_t)ncols * nouter));
        out[i] = (float)blk[(((int64_t)o * ng + col / C) * L + e) * C + col % C];
    }
}

// ----------------------------------------------------------------- launchers
template <int L, bool PRO, class S = float>
hipError_t launch_r2c(hipStream_t st, const S* src, int nrows, int in_pitch, int n_in, typename VecOf<S>::V* dst,
                      int out_pitch, int n_keep, S sg, const typename VecOf<S>::V* tw, S* pvec = nullptr,
                      const double* beta = nullptr, const int* active = nullptr) {
    using Cfg = RowCfg<L, typename VecOf<S>::V>;
    const int blocks = ceil_div(nrows / 2, Cfg::C);
    if (2 * n_in == L)
        FIRM_PASS_LAUNCH((k_rows_r2c<L, PRO, S, true>), dim3(blocks), dim3(Cfg::THREADS), st, src, nrows, in_pitch,
                           n_in, dst, out_pitch, n_keep, sg, tw, pvec, beta, active);
    else
        FIRM_PASS_LAUNCH((k_rows_r2c<L, PRO, S, false>), dim3(blocks), dim3(Cfg::THREADS), st, src, nrows,
                           in_pitch, n_in, dst, out_pitch, n_keep, sg, tw, pvec, beta, active);
    return hipGetLastError();
}

template <int L, bool DOT, class S = float>
hipError_t launch_c2r(hipStream_t st, const typename VecOf<S>::V* src, int nrows, int in_pitch, S* dst, int out_pitch,
                      int n_out, S sg, S scale, S lam, const S* xadd, const typename VecOf<S>::V* tw,
                      double* partials = nullptr, const int* active = nullptr) {
    using Cfg = RowCfg<L, typename VecOf<S>::V>;
    if (nrows < 2 || nrows % 2) return hipErrorInvalidValue;  // whole row pairs (the kernel loads the last one)
    const int blocks = ceil_div(nrows / 2, Cfg::C);
    if (2 * n_out == L)
        FIRM_PASS_LAUNCH((k_rows_c2r<L, DOT, S, true>), dim3(blocks), dim3(Cfg::THREADS), st, src, nrows, in_pitch,
                           dst, out_pitch, n_out, sg, scale, lam, xadd, tw, partials, active, CgStep{});
    else
        FIRM_PASS_LAUNCH((k_rows_c2r<L, DOT, S, false>), dim3(blocks), dim3(Cfg::THREADS), st, src, nrows,
                           in_pitch, dst, out_pitch, n_out, sg, scale, lam, xadd, tw, partials, active, CgStep{});
    return hipGetLastError();
}

// the last pass of the CG product with the CG step (n_out = L / 2)
template <int L>
hipError_t launch_c2r_step(hipStream_t st, const float2* src, int nrows, int in_pitch, int out_pitch, const float2* tw,
                           double* partials, const int* active, CgStep step) {
    using Cfg = RowCfg<L, float2>;
    if (nrows < 2 || nrows % 2) return hipErrorInvalidValue;  // whole row pairs (the kernel loads the last one)
    const int blocks = ceil_div(nrows / 2, Cfg::C);
    FIRM_PASS_LAUNCH((k_rows_c2r<L, false, float, true, true>), dim3(blocks), dim3(Cfg::THREADS), st, src, nrows,
                       in_pitch, (float*)nullptr, out_pitch, L / 2, 1.f, 1.f, 0.f, (const float*)nullptr, tw, partials,
                       active, step);
    return hipGetLastError();
}

template <int L, bool CONTIG, int MAP, int EPI, class S = float>
hipError_t launch_cols(hipStream_t st, const typename VecOf<S>::V* src, void* dst, int nouter, int ncols,
                       int64_t s_outer, int64_t s_col, int64_t s_elem, int64_t d_outer, int64_t d_col,
                       int64_t d_elem, int n_in, int n_out, S sg, const typename VecOf<S>::V* tw,
                       EpiArgs ep = EpiArgs(), const int* active = nullptr, int64_t s_group = -1,
                       int64_t d_group = -1) {
    using Cfg = FftCfg<L, typename VecOf<S>::V>;
    const int blocks = nouter * ceil_div(ncols, Cfg::C);
    // column group strides: by default the columns are one strided sequence (group = C columns)
    if (s_group < 0) s_group = (int64_t)Cfg::C * s_col;
    if (d_group < 0) d_group = (int64_t)Cfg::C * d_col;
    if (MAP == MAP_FIRST && EPI == EPI_STORE && 2 * n_in == L)
        FIRM_PASS_LAUNCH((k_cols<L, CONTIG, MAP, EPI, S, 1>), dim3(blocks), dim3(Cfg::THREADS), st, src, dst,
                           ncols, s_outer, s_col, s_elem, d_outer, d_col, d_elem, s_group, d_group, n_in, n_out, sg,
                           tw, ep, active);
    else if (MAP == MAP_FIRST && EPI == EPI_STORE && 2 * n_out == L)
        FIRM_PASS_LAUNCH((k_cols<L, CONTIG, MAP, EPI, S, 2>), dim3(blocks), dim3(Cfg::THREADS), st, src, dst,
                           ncols, s_outer, s_col, s_elem, d_outer, d_col, d_elem, s_group, d_group, n_in, n_out, sg,
                           tw, ep, active);
    else
        FIRM_PASS_LAUNCH((k_cols<L, CONTIG, MAP, EPI, S, 0>), dim3(blocks), dim3(Cfg::THREADS), st, src, dst,
                           ncols, s_outer, s_col, s_elem, d_outer, d_col, d_elem, s_group, d_group, n_in, n_out, sg,
                           tw, ep, active);
    return hipGetLastError();
}

// spec16 / shtab: the 16-bit spectrum of the option khat_bf16 (FP32 only), used instead of spec
template <int L, class S = float>
hipError_t launch_mid(hipStream_t st, typename VecOf<S>::V* data, const S* spec, int nouter, int ncols,
                      int64_t s_outer, int64_t s_elem, int n_in, const typename VecOf<S>::V* tw,
                      const int* active = nullptr, int64_t s_group = -1, S kadd = 0,
                      const uint16_t* spec16 = nullptr, const float2* shtab = nullptr, double* dotp = nullptr) {
    using Cfg = FftCfg<L, typename VecOf<S>::V>;
    constexpr int C = Cfg::C;
    if (s_group < 0) s_group = C;
    const void* sp = spec16 ? (const void*)spec16 : (const void*)spec;
    const int blocks = tail_packed_blocks<C>(nouter, ncols);
    bool k16 = false;
    if constexpr (sizeof(S) == 4) k16 = spec16 != nullptr;
    const bool half = 2 * n_in == L, dot = dotp != nullptr;
#define FIRM_MID(H, K, D)                                                                                      \
    FIRM_PASS_LAUNCH((k_mid<L, S, H, K, D>), dim3(blocks), dim3(Cfg::THREADS), st, data, sp, shtab, kadd, \
                       nouter, ncols, s_outer, s_elem, s_group, n_in, tw, active, dotp)
    if (k16) {
        if constexpr (sizeof(S) == 4) {
            if (half) {
                if (dot) FIRM_MID(true, true, true);
                else FIRM_MID(true, true, false);
            } else {
                if (dot) FIRM_MID(false, true, true);
                else FIRM_MID(false, true, false);
            }
        }
    } else if (half) {
        if (dot) FIRM_MID(true, false, true);
        else FIRM_MID(true, false, false);
    } else {
        if (dot) FIRM_MID(false, false, true);
        else FIRM_MID(false, false, false);
    }
#undef FIRM_MID
    return hipGetLastError();
}

#define RET_IF(e)                          \
    do {                                   \
        hipError_t e__ = (e);              \
        if (e__ != hipSuccess) return e__; \
    } while (0)

// The five passes of y = crop(IFFT(K^ . FFT(pad x))) + lam x for one N (L = 2N), as a front
// (passes A-C) and a back (passes D-E).
// CG form: the front's first pass forms p = src + beta p and its middle pass the block
// partials of <p, q> from the spectrum (fft_apply_cg_partials of them); the back's last pass
// takes the CG step with the alpha formed from them in between (fft_apply_cg_step_partials
// partials of ||r||^2).
template <int L>
hipError_t apply_front_bc(firm_plan p, float lam, const int* active, double* dotp, hipEvent_t* ev);

template <int L>
hipError_t apply_front(firm_plan p, const float* src, float* pvec, float lam, const double* beta, const int* active,
                       double* dotp, hipEvent_t* ev) {
    const int N = L / 2, QP = p->QP;
    hipStream_t st = p->stream;
    // A: rows along i3, N real -> padded 2N transform, modes 0..N kept
    arm_pass_events(ev, 0);
    if (beta)
        RET_IF((launch_r2c<L, true>(st, src, N * N, N, N, p->T1, QP, N + 1, -1.f, p->tw, pvec, beta, active)));
    else
        RET_IF((launch_r2c<L, false>(st, src, N * N, N, N, p->T1, QP, N + 1, -1.f, p->tw)));
    return apply_front_bc<L>(p, lam, active, dotp, ev);
}

// the front of the preconditioned CG product with the preconditioner's last pass fused into its
// first (k_rows_pz): z's half spectra in S1 -> p = z + beta p -> T1
template <int L>
hipError_t apply_front_pz(firm_plan p, float* pvec, float lam, const double* beta, const int* active, double* dotp) {
    if constexpr (L >= 256 && L <= 1024) {
        constexpr int N = L / 2;
        hipLaunchKernelGGL((k_rows_pz<N>), dim3(N * N / 2 / PZC), dim3(PZC * N / 8), 0, p->stream, p->S1, p->QPn,
                           pvec, beta, p->T1, p->QP, p->tw, active);
        RET_IF(hipGetLastError());
        return apply_front_bc<L>(p, lam, active, dotp, nullptr);
    } else {
        return hipErrorInvalidValue;
    }
}

template <int L>
hipError_t apply_front_bc(firm_plan p, float lam, const int* active, double* dotp, hipEvent_t* ev) {
    const int N = L / 2, QP = p->QP;
    hipStream_t st = p->stream;
    // T2 is blocked [q2][q3 group][i1][C] (C = the pencils per workgroup), so that every pencil
    // group of the middle pass is one contiguous block
    constexpr int C = FftCfg<L, float2>::C;
    const int64_t ng = (N + 1 + C - 1) / C, sg_ = (int64_t)N * C, se_ = ng * (int64_t)N * C;
    // B: along i2 for every (i1, q3): T1[i1][i2][q3] (N) -> T2[q2][g][i1][c] (2N)
    arm_pass_events(ev, 1);
    RET_IF((launch_cols<L, false, MAP_FIRST, EPI_STORE>(st, p->T1, p->T2, N, N + 1, (int64_t)N * QP, 1, QP, C, 1,
                                                          se_, N, L, -1.f, p->tw, EpiArgs(), active, -1, sg_)));
    // C: along i1 for every (q2, q3): forward, times K^ + lam / L^3, inverse, keep i1 < N.
    // With the unnormalised inverse the lam term adds exactly lam x to the cropped output, so
    // that pass E need not read x
    const float kadd = lam / ((float)L * L * L);
    arm_pass_events(ev, 2);
    RET_IF((launch_mid<L>(st, p->T2, p->khat, L, N + 1, se_, C, N, p->tw, active, sg_, kadd,
                          p->khat_bf16 ? p->khat16 : nullptr, p->khat_bf16 == 1 ? p->shtab : nullptr, dotp)));
    return hipSuccess;
}

template <int L>
hipError_t apply_back(firm_plan p, float* y, const int* active, const CgStep* step, double* partials,
                      hipEvent_t* ev) {
    const int N = L / 2, QP = p->QP;
    hipStream_t st = p->stream;
    constexpr int C = FftCfg<L, float2>::C;
    const int64_t ng = (N + 1 + C - 1) / C, sg_ = (int64_t)N * C, se_ = ng * (int64_t)N * C;
    // D: inverse along q2, keep i2 < N: T2[q2][g][i1][c] -> T1[i1][i2][q3]
    arm_pass_events(ev, 3);
    RET_IF((launch_cols<L, false, MAP_FIRST, EPI_STORE>(st, p->T2, p->T1, N, N + 1, C, 1, se_, (int64_t)N * QP, 1,
                                                          QP, L, N, 1.f, p->tw, EpiArgs(), active, sg_, -1)));
    // E: inverse along q3 (half spectrum -> real), crop; CG form: the CG step instead of a store
    arm_pass_events(ev, 4);
    if (step)
        RET_IF(launch_c2r_step<L>(st, p->T1, N * N, QP, N, p->tw, partials, active, *step));
    else
        RET_IF((launch_c2r<L, false>(st, p->T1, N * N, QP, y, N, N, 1.f, 1.f, 0.f, (const float*)nullptr, p->tw,
                                     nullptr, active)));
    return hipSuccess;
}

template <int L>
hipError_t apply_passes(firm_plan p, const float* x, float* y, float lam, hipEvent_t* ev = nullptr) {
    RET_IF(apply_front<L>(p, x, nullptr, lam, nullptr, nullptr, nullptr, ev));
    return apply_back<L>(p, y, nullptr, nullptr, nullptr, ev);
}

// FP64 form of the product, for true residuals and the FP64 solver modes: the same
// five passes in double with the double spectrum khat64.
template <int L>
hipError_t apply_passes64(firm_plan p, const double* x, double* y, double lam) {
    const int N = L / 2, QP = p->QP;
    hipStream_t st = p->stream;
    RET_IF((launch_r2c<L, false, double>(st, x, N * N, N, N, p->T1d, QP, N + 1, -1.0, p->tw64)));
    constexpr int C = FftCfg<L, double2>::C;  // T2d blocked like T2, with the FP64 pencil count
    const int64_t ng = (N + 1 + C - 1) / C, sg_ = (int64_t)N * C, se_ = ng * (int64_t)N * C;
    RET_IF((launch_cols<L, false, MAP_FIRST, EPI_STORE, double>(st, p->T1d, p->T2d, N, N + 1, (int64_t)N * QP, 1,
                                                                  QP, C, 1, se_, N, L, -1.0, p->tw64, EpiArgs(),
                                                                  nullptr, -1, sg_)));
    RET_IF((launch_mid<L, double>(st, p->T2d, p->khat64, L, N + 1, se_, C, N, p->tw64, nullptr, sg_)));
    RET_IF((launch_cols<L, false, MAP_FIRST, EPI_STORE, double>(st, p->T2d, p->T1d, N, N + 1, C, 1, se_,
                                                                  (int64_t)N * QP, 1, QP, L, N, 1.0, p->tw64,
                                                                  EpiArgs(), nullptr, sg_, -1)));
    return launch_c2r<L, false, double>(st, p->T1d, N * N, QP, y, N, N, 1.0, 1.0, lam, x, p->tw64);
}

// Spectrum of the circulant column: Re DFT_{2N}(kerc) / (2N)^3 for q3 in [0, N], written in the
// blocked layout of k_mid.  S is the arithmetic (float for khat, double for khat64).
template <int L, class S>
hipError_t khat_passes(firm_plan p, const S* kerc, typename VecOf<S>::V* w1, S* out,
                       const typename VecOf<S>::V* tw) {
    const int N = L / 2, QP = p->QP;
    hipStream_t st = p->stream;
    RET_IF((launch_r2c<L, false, S>(st, kerc, L * L, L, L, w1, QP, N + 1, (S)-1, tw)));
    RET_IF((launch_cols<L, false, MAP_FIRST, EPI_STORE, S>(st, w1, w1, L, N + 1, (int64_t)L * QP, 1, QP,
                                                             (int64_t)L * QP, 1, QP, L, L, (S)-1, tw)));
    EpiArgs ep;
    ep.scale = 1.0 / ((double)L * (double)L * (double)L);
    return launch_cols<L, false, MAP_FIRST, EPI_REAL_BLOCKED, S>(st, w1, out, L, N + 1, QP, 1, (int64_t)L * QP, 0,
                                                                 0, 0, L, L, (S)-1, tw, ep);
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
    RET_IF((launch_cols<L, false, MAP_CIRC, EPI_STORE>(st, h1, h2, L, N, (int64_t)L * N, 1, N, (int64_t)N2 * N, 1,
                                                         N, L, N2, 1.f, p->tw)));
    // axis 1: h2[l1][p2][n3] -> chalf[p1][p2][n3] = Re / phihat^3 + k0 term, wrap planes zero
    EpiArgs ep;
    ep.dec_e = p->deconv_ker;
    ep.dec_o = p->deconv_ker;
    ep.dec_c = p->deconv_ker;
    ep.wrap_o = N;
    ep.k0 = (float)p->ker_k0;
    return launch_cols<L, false, MAP_CIRC, EPI_KER>(st, h2, chalf, N2, N, N, 1, (int64_t)N2 * N, N, 1,
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
    RET_IF((launch_cols<L, true, MAP_CENTER, EPI_STORE>(st, grid, j1, 1, L * L, 0, L, 1, 0, N, 1, L, N, 1.f,
                                                          p->tw)));
    // axis 2: j1[l1][l2][i3] -> j2[l1][i2][i3]
    RET_IF((launch_cols<L, false, MAP_CENTER, EPI_STORE>(st, j1, j2, L, N, (int64_t)L * N, 1, N, (int64_t)N * N, 1,
                                                           N, L, N, 1.f, p->tw)));
    // axis 1: j2[l1][i2][i3] -> atb[i1][i2][i3]
    EpiArgs ep;
    ep.dec_e = p->deconv_atb;
    ep.dec_o = p->deconv_atb;
    ep.dec_c = p->deconv_atb;
    ep.k0dev = k0dev;
    return launch_cols<L, false, MAP_CENTER, EPI_ATB>(st, j2, atb, N, N, N, 1, (int64_t)N * N, N, 1,
                                                      (int64_t)N * N, L, N, 1.f, p->tw, ep);
}

// z = IFFT_N(d . FFT_N(r)) with dhalf = d / N^3 in the blocked layout (q3 in [0, N/2]).
template <int L>
hipError_t precond_passes(firm_plan p, const float* dhalf, const float* r, float* z, const int* active,
                          double* partials) {
    const int N = L, H = N / 2 + 1, QPn = p->QPn;
    hipStream_t st = p->stream;
    if constexpr (L <= 64) {  // slab kernels around the middle pass: 3 launches instead of 5
        if (!z) return hipErrorInvalidValue;
        constexpr int NT = FftCfg<L, float2>::THREADS;
        hipLaunchKernelGGL((k_precond_slab<L, true>), dim3(N), dim3(NT), 0, st, r, p->S1, (float*)nullptr, QPn,
                           p->tw, active);
        RET_IF(hipGetLastError());
        RET_IF((launch_mid<L>(st, p->S1, dhalf, N, H, QPn, (int64_t)N * QPn, N, p->tw, active, -1, 0.f, nullptr,
                              nullptr, partials)));
        hipLaunchKernelGGL((k_precond_slab<L, false>), dim3(N), dim3(NT), 0, st, (const float*)nullptr, p->S1, z,
                           QPn, p->tw, active);
        return hipGetLastError();
    }
    RET_IF((launch_r2c<L, false, float>(st, r, N * N, N, N, p->S1, QPn, H, -1.f, p->tw, nullptr, nullptr, active)));
    RET_IF((launch_cols<L, false, MAP_FIRST, EPI_STORE>(st, p->S1, p->S1, N, H, (int64_t)N * QPn, 1, QPn,
                                                          (int64_t)N * QPn, 1, QPn, N, N, -1.f, p->tw, EpiArgs(),
                                                          active)));
    // partials: <r, z> = sum of dhalf |R^|^2 over the spectrum (Parseval, unnormalised
    // transforms), fft_precond_partials(p) block partials from the middle pass
    RET_IF((launch_mid<L>(st, p->S1, dhalf, N, H, QPn, (int64_t)N * QPn, N, p->tw, active, -1, 0.f, nullptr,
                          nullptr, partials)));
    RET_IF((launch_cols<L, false, MAP_FIRST, EPI_STORE>(st, p->S1, p->S1, N, H, (int64_t)N * QPn, 1, QPn,
                                                          (int64_t)N * QPn, 1, QPn, N, N, 1.f, p->tw, EpiArgs(),
                                                          active)));
    if (!z) return hipSuccess;  // the row half spectra of z stay in S1 (for k_rows_pz)
    return launch_c2r<L, false, float>(st, p->S1, N * N, QPn, z, N, N, 1.f, 1.f, 0.f, nullptr, p->tw, nullptr, active);
}

template <int L>
hipError_t khat_f32(firm_plan p, float2* w1) { return khat_passes<L, float>(p, p->kerc, w1, p->khat, p->tw); }
// adds the plan's damping term (if any) to a blocked spectrum of L-point pencils
template <int L, class S>
hipError_t khat_add_reg(firm_plan p, S* kh) {
    if (p->reg_order <= 0 || !(p->reg_mu_eff > 0.0)) return hipSuccess;
    constexpr int C = FftCfg<L, typename VecOf<S>::V>::C;
    const int N = L / 2, ng = (N + 1 + C - 1) / C;
    const int64_t n = (int64_t)L * ng * L * C;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    const double coef = p->reg_mu_eff / ((double)L * L * L);  // the spectrum carries 1 / L^3
    hipLaunchKernelGGL(k_khat_reg<S>, dim3(blocks), dim3(256), 0, p->stream, kh, L, C, ng, coef, p->reg_order);
    return hipGetLastError();
}

template <int L>
hipError_t khat_f64(firm_plan p, const double* k64, double2* w1) {
    RET_IF((khat_passes<L, double>(p, k64, w1, p->khat64, p->tw64)));
    return khat_add_reg<L, double>(p, p->khat64);
}

// Forward N^3 real-to-half-spectrum transform: out [N][N][QPn] complex, FFT order, q3 in [0, N/2].
template <int L>
hipError_t fwd_r2c_passes(firm_plan p, const float* x, float2* out) {
    const int N = L, H = N / 2 + 1, QPn = p->QPn;
    hipStream_t st = p->stream;
    RET_IF((launch_r2c<L, false, float>(st, x, N * N, N, N, out, QPn, H, -1.f, p->tw)));
    RET_IF((launch_cols<L, false, MAP_FIRST, EPI_STORE>(st, out, out, N, H, (int64_t)N * QPn, 1, QPn,
                                                          (int64_t)N * QPn, 1, QPn, N, N, -1.f, p->tw)));
    return launch_cols<L, false, MAP_FIRST, EPI_STORE>(st, out, out, N, H, QPn, 1, (int64_t)N * QPn, QPn, 1,
                                                       (int64_t)N * QPn, N, N, -1.f, p->tw);
}

// Forward-projection grid, L = 2N: N^3 real u (array index i, zero-padded to L per axis) ->
// X[q1][q2][q3] = sum_i u_i exp(-2 pi i <i, q> / L) for q1, q2 in [0, L), q3 in [0, N] (pitch QP).
template <int L>
hipError_t projgrid_passes(firm_plan p, const float* u, float2* t1, float2* w, float2* X) {
    const int N = L / 2, QP = p->QP;
    hipStream_t st = p->stream;
    // axis 3: rows of N real -> modes 0..N of the padded transform, t1[i1][i2][q3]
    RET_IF((launch_r2c<L, false, float>(st, u, N * N, N, N, t1, QP, N + 1, -1.f, p->tw)));
    // axis 2: t1[i1][i2][q3] -> w[i1][q2][q3]
    RET_IF((launch_cols<L, false, MAP_FIRST, EPI_STORE>(st, t1, w, N, N + 1, (int64_t)N * QP, 1, QP,
                                                          (int64_t)L * QP, 1, QP, N, L, -1.f, p->tw)));
    // axis 1: w[i1][q2][q3] -> X[q1][q2][q3]
    return launch_cols<L, false, MAP_FIRST, EPI_STORE>(st, w, X, L, N + 1, QP, 1, (int64_t)L * QP, QP, 1,
                                                       (int64_t)L * QP, N, L, -1.f, p->tw);
}

// G real N x N images (L = N, row pitch N) -> half spectra out[g][q1][q2], q2 in [0, N/2]
// (pitch QPn): rows, then columns, both forward.
template <int L>
hipError_t img_r2c_passes(firm_plan p, const float* img, int G, float2* out) {
    const int N = L, H = N / 2 + 1, QPn = p->QPn;
    hipStream_t st = p->stream;
    RET_IF((launch_r2c<L, false, float>(st, img, G * N, N, N, out, QPn, H, -1.f, p->tw)));
    return launch_cols<L, false, MAP_FIRST, EPI_STORE>(st, out, out, G, H, (int64_t)N * QPn, 1, QPn,
                                                       (int64_t)N * QPn, 1, QPn, N, N, -1.f, p->tw);
}

template <int L>
int cols_per_block_t(bool dbl) { return dbl ? FftCfg<L, double2>::C : FftCfg<L, float2>::C; }

}  // namespace

#define DISPATCH_L(Lval, call_tmpl, ...)                \
    switch (Lval) {                                     \
        case 8: return call_tmpl<8>(__VA_ARGS__);       \
        case 16: return call_tmpl<16>(__VA_ARGS__);     \
        case 32: return call_tmpl<32>(__VA_ARGS__);     \
        case 64: return call_tmpl<64>(__VA_ARGS__);     \
        case 128: return call_tmpl<128>(__VA_ARGS__);   \
        case 256: return call_tmpl<256>(__VA_ARGS__);   \
        case 512: return call_tmpl<512>(__VA_ARGS__);   \
        case 1024: return call_tmpl<1024>(__VA_ARGS__); \
        default: break;                                 \
    }

int fft_cols_per_block(int L, bool dbl) {
    DISPATCH_L(L, cols_per_block_t, dbl);
    return 0;
}

namespace {
template <int L>
int apply_mid_blocks_t() { return tail_packed_blocks<FftCfg<L, float2>::C>(L, L / 2 + 1); }
}  // namespace

int fft_apply_cg_partials(firm_plan p) {
    DISPATCH_L(2 * p->N, apply_mid_blocks_t);
    return 0;
}

namespace {
template <int L>
int c2r_blocks_t(int N) { return ceil_div(N * N / 2, RowCfg<L, float2>::C); }
}  // namespace

int fft_apply_cg_step_partials(firm_plan p) {
    DISPATCH_L(2 * p->N, c2r_blocks_t, p->N);
    return 0;
}

namespace {
template <int L>
int precond_mid_blocks_t() { return tail_packed_blocks<FftCfg<L, float2>::C>(L, L / 2 + 1); }
}  // namespace

int fft_precond_partials(firm_plan p) {
    DISPATCH_L(p->N, precond_mid_blocks_t);
    return 0;
}

int64_t fft_t2_elems(int N, bool dbl) {
    const int C = fft_cols_per_block(2 * N, dbl);
    return (int64_t)2 * N * N * (((N + 1 + C - 1) / C) * C);
}

size_t blocked_spectrum_elems(int L, int nouter, int ncols, bool dbl) {
    const int C = fft_cols_per_block(L, dbl);
    return (size_t)nouter * (size_t)((ncols + C - 1) / C) * C * (size_t)L;
}

hipError_t fft_apply_AtA(firm_plan p, const float* x, float* y, float lam) {
    DISPATCH_L(2 * p->N, apply_passes, p, x, y, lam);
    return hipErrorInvalidValue;
}

namespace {
hipError_t apply_events_dispatch(firm_plan p, const float* x, float* y, float lam, hipEvent_t* ev) {
    DISPATCH_L(2 * p->N, apply_passes, p, x, y, lam, ev);
    return hipErrorInvalidValue;
}
}  // namespace

hipError_t fft_apply_AtA_events(firm_plan p, const float* x, float* y, float lam, hipEvent_t* ev) {
    const hipError_t e = apply_events_dispatch(p, x, y, lam, ev);
    tl_pass_ev[0] = tl_pass_ev[1] = nullptr;  // a pass that failed before its launch leaves none armed
    return e;
}

hipError_t fft_apply_cg_front(firm_plan p, const float* src, float* pvec, float lam, const double* beta_dev,
                              const int* active, double* dotp) {
    DISPATCH_L(2 * p->N, apply_front, p, src, pvec, lam, beta_dev, active, dotp, nullptr);
    return hipErrorInvalidValue;
}

hipError_t fft_apply_cg_front_pz(firm_plan p, float* pvec, float lam, const double* beta_dev, const int* active,
                                 double* dotp) {
    DISPATCH_L(2 * p->N, apply_front_pz, p, pvec, lam, beta_dev, active, dotp);
    return hipErrorInvalidValue;
}

hipError_t fft_apply_cg_step(firm_plan p, float* x, const float* pvec, float* r, const double* alpha_dev,
                             const int* active, double* partials) {
    const CgStep step{x, pvec, r, alpha_dev};
    DISPATCH_L(2 * p->N, apply_back, p, nullptr, active, &step, partials, nullptr);
    return hipErrorInvalidValue;
}

hipError_t fft_apply_AtA64(firm_plan p, const double* x, double* y, double lam) {
    DISPATCH_L(2 * p->N, apply_passes64, p, x, y, lam);
    return hipErrorInvalidValue;
}

namespace {
template <int L>
hipError_t khat_f32_all(firm_plan p, float2* w1) {
    RET_IF(khat_f32<L>(p, w1));
    RET_IF((khat_add_reg<L, float>(p, p->khat)));
    if (!p->khat_bf16) return hipSuccess;
    constexpr int C = FftCfg<L, float2>::C;
    const int N = L / 2, ng = (N + 1 + C - 1) / C;
    const int64_t n = (int64_t)L * ng * L * C;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    if (p->khat_bf16 == 2) {  // plain BF16 codes
        hipLaunchKernelGGL(k_khat_encode16, dim3(blocks), dim3(256), 0, p->stream, p->khat, L, C, ng,
                           (const float2*)nullptr, p->khat16);
        return hipGetLastError();
    }
    // 16-bit copy with per-shell offset and scale; the statistics live in w1 (free again)
    double* gsum = reinterpret_cast<double*>(w1);
    unsigned* gcnt = reinterpret_cast<unsigned*>(gsum + KSH_MAX);
    unsigned* gdev = gcnt + KSH_MAX;
    RET_IF(fill_zero(gsum, KSH_MAX * (sizeof(double) + 2 * sizeof(unsigned)), p->stream));
    hipLaunchKernelGGL(k_khat_shell_sum, dim3(blocks), dim3(256), 0, p->stream, p->khat, L, C, ng, gsum, gcnt);
    hipLaunchKernelGGL(k_khat_shell_dev, dim3(blocks), dim3(256), 0, p->stream, p->khat, L, C, ng, gsum, gcnt, gdev);
    hipLaunchKernelGGL(k_khat_shell_tab, dim3(1), dim3(256), 0, p->stream, gsum, gcnt, gdev, p->shtab);
    hipLaunchKernelGGL(k_khat_encode16, dim3(blocks), dim3(256), 0, p->stream, p->khat, L, C, ng, p->shtab, p->khat16);
    return hipGetLastError();
}
}  // namespace

hipError_t fft_khat_from_kerc(firm_plan p, float2* w1) {
    DISPATCH_L(2 * p->N, khat_f32_all, p, w1);
    return hipErrorInvalidValue;
}

hipError_t fft_khat64_from_kerc64(firm_plan p, const double* kerc64, double2* w1) {
    DISPATCH_L(2 * p->N, khat_f64, p, kerc64, w1);
    return hipErrorInvalidValue;
}

hipError_t fft_ker_grid(firm_plan p, const float* grid, float2* h1, float2* h2, float* chalf) {
    DISPATCH_L(4 * p->N, kergrid_passes, p, grid, h1, h2, chalf);
    return hipErrorInvalidValue;
}

hipError_t fft_atb_grid(firm_plan p, const float2* grid, float2* j1, float2* j2, float* atb,
                        const double* k0term) {
    DISPATCH_L(2 * p->N, atbgrid_passes, p, grid, j1, j2, atb, k0term);
    return hipErrorInvalidValue;
}

hipError_t fft_precond(firm_plan p, const float* dhalf, const float* r, float* z, const int* active,
                       double* partials) {
    DISPATCH_L(p->N, precond_passes, p, dhalf, r, z, active, partials);
    return hipErrorInvalidValue;
}

hipError_t fft_forward_r2c(firm_plan p, const float* x, float2* out) {
    DISPATCH_L(p->N, fwd_r2c_passes, p, x, out);
    return hipErrorInvalidValue;
}

hipError_t fft_images_r2c(firm_plan p, const float* img, int G, float2* out) {
    DISPATCH_L(p->N, img_r2c_passes, p, img, G, out);
    return hipErrorInvalidValue;
}

hipError_t fft_project_grid(firm_plan p, const float* u, float2* t1, float2* w, float2* X) {
    DISPATCH_L(2 * p->N, projgrid_passes, p, u, t1, w, X);
    return hipErrorInvalidValue;
}

hipError_t fft_khat_unblock(firm_plan p, float* out) {
    const int L = 2 * p->N;
    const int64_t n = (int64_t)L * L * (p->N + 1);
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_unblock<float>, dim3(blocks), dim3(256), 0, p->stream, p->khat, out, L, L, p->N + 1,
                       fft_cols_per_block(L, false));
    return hipGetLastError();
}
