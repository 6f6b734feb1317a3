// Batched 1D FFTs of power-of-two length L (8..1024) on pencils staged in LDS.
//
// A workgroup holds C pencils in LDS as buf[e * (C + 1) + c] (element e of
// pencil c; the +1 pitch keeps strided rows off one bank).  It runs C * L / 8
// threads; thread t owns pencil c = t % C and butterfly row j = t / C, and
// keeps up to 8 complex values in registers per stage.
//
// The transform is a self-sorting (Stockham) decomposition of the DFT
// X_k = sum_n x_n exp(sg * 2 pi i k n / L) into radix-8 stages with one final
// radix-4 or radix-2 stage: with Ns the product of the radices already applied,
// butterfly u in [0, L/r) reads x[u + s L/r] (s < r), multiplies element s by
// exp(sg 2 pi i s k / (Ns r)) with k = u mod Ns, takes an r-point DFT and writes
// it to (u - k) r + k + s Ns.  Twiddles come from a 1024-entry table of
// exp(-2 pi i m / 1024) computed in double on the host.
#pragma once

#include <hip/hip_runtime.h>

#ifndef FIRM_TWN
#define FIRM_TWN 1024
#endif

// complex helpers for float2 and double2
template <class V> struct CxT;
template <> struct CxT<float2> { using S = float; };
template <> struct CxT<double2> { using S = double; };
template <class V>
__device__ __forceinline__ V mkv(typename CxT<V>::S a, typename CxT<V>::S b) { V v; v.x = a; v.y = b; return v; }

template <class V>
__device__ __forceinline__ V c_mul(V a, V b) { return mkv<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
template <class V>
__device__ __forceinline__ V c_add(V a, V b) { return mkv<V>(a.x + b.x, a.y + b.y); }
template <class V>
__device__ __forceinline__ V c_sub(V a, V b) { return mkv<V>(a.x - b.x, a.y - b.y); }
// multiply by sg * i
template <class V>
__device__ __forceinline__ V c_mul_si(V a, typename CxT<V>::S sg) { return mkv<V>(-sg * a.y, sg * a.x); }

template <int R, class V>
struct DftSmall;

template <class V>
struct DftSmall<2, V> {
    static __device__ __forceinline__ void run(V* v, typename CxT<V>::S) {
        V a = v[0], b = v[1];
        v[0] = c_add(a, b);
        v[1] = c_sub(a, b);
    }
};

template <class V>
struct DftSmall<4, V> {
    static __device__ __forceinline__ void run(V* v, typename CxT<V>::S sg) {
        V t0 = c_add(v[0], v[2]), t1 = c_sub(v[0], v[2]);
        V t2 = c_add(v[1], v[3]), t3 = c_mul_si(c_sub(v[1], v[3]), sg);
        v[0] = c_add(t0, t2);
        v[2] = c_sub(t0, t2);
        v[1] = c_add(t1, t3);
        v[3] = c_sub(t1, t3);
    }
};

template <class V>
struct DftSmall<8, V> {
    static __device__ __forceinline__ void run(V* v, typename CxT<V>::S sg) {
        using S = typename CxT<V>::S;
        // even / odd halves, then combine with W8^k = exp(sg i pi k / 4)
        V e[4] = {v[0], v[2], v[4], v[6]};
        V o[4] = {v[1], v[3], v[5], v[7]};
        DftSmall<4, V>::run(e, sg);
        DftSmall<4, V>::run(o, sg);
        const S h = (S)0.70710678118654752440;
        V w1 = mkv<V>(h * (o[1].x - sg * o[1].y), h * (o[1].y + sg * o[1].x));
        V w2 = c_mul_si(o[2], sg);
        V w3 = mkv<V>(h * (-o[3].x - sg * o[3].y), h * (-o[3].y + sg * o[3].x));
        v[0] = c_add(e[0], o[0]);
        v[4] = c_sub(e[0], o[0]);
        v[1] = c_add(e[1], w1);
        v[5] = c_sub(e[1], w1);
        v[2] = c_add(e[2], w2);
        v[6] = c_sub(e[2], w2);
        v[3] = c_add(e[3], w3);
        v[7] = c_sub(e[3], w3);
    }
};

template <int L, int C, int R, int NS, class V>
__device__ __forceinline__ void fft_stage(V* buf, const V* __restrict__ tw, typename CxT<V>::S sg, int c, int j) {
    constexpr int NB = 8 / R;
    constexpr int CP = C + 1;
    V v[8];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int u = j + b * (L / 8);
#pragma unroll
        for (int s = 0; s < R; ++s) v[b * R + s] = buf[(u + s * (L / R)) * CP + c];
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int u = j + b * (L / 8);
        const int k = u & (NS - 1);
        if (NS > 1) {
#pragma unroll
            for (int s = 1; s < R; ++s) {
                V w = tw[(s * k) * (FIRM_TWN / (NS * R))];
                w.y *= -sg;  // table holds exp(-2 pi i m / T); sg = -1 keeps it, sg = +1 conjugates
                v[b * R + s] = c_mul(v[b * R + s], w);
            }
        }
        DftSmall<R, V>::run(&v[b * R], sg);
        const int base = (u - k) * R + k;
#pragma unroll
        for (int s = 0; s < R; ++s) buf[(base + s * NS) * CP + c] = v[b * R + s];
    }
    __syncthreads();
}

template <int L, int C, int NS, class V>
__device__ __forceinline__ void fft_stages(V* buf, const V* __restrict__ tw, typename CxT<V>::S sg, int c, int j) {
    if constexpr (NS < L) {
        constexpr int REM = L / NS;
        constexpr int R = REM >= 8 ? 8 : REM;
        fft_stage<L, C, R, NS, V>(buf, tw, sg, c, j);
        fft_stages<L, C, NS * R, V>(buf, tw, sg, c, j);
    }
}

// In-place transform of the C pencils in buf; must be entered after a barrier
// that publishes buf, and leaves after one.
template <int L, int C, class V>
__device__ __forceinline__ void fft_lds(V* buf, const V* __restrict__ tw, typename CxT<V>::S sg) {
    const int t = threadIdx.x;
    fft_stages<L, C, 1, V>(buf, tw, sg, t % C, t / C);
}

// pencils per workgroup for each length (threads = C * L / 8)
template <int L, class V = float2>
struct FftCfg {
    static constexpr bool DBL = sizeof(V) == 16;
    static constexpr int C = DBL ? (L >= 256 ? 8 : (L >= 128 ? 16 : 2048 / L))
                                 : (L >= 1024 ? 8 : (L >= 128 ? 16 : 2048 / L));
    static constexpr int THREADS = C * L / 8;
    static constexpr int CP = C + 1;
};
