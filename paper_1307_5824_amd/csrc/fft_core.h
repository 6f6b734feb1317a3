// Batched 1D FFTs of power-of-two length L (8..1024); a workgroup transforms C
// pencils with C * L / 8 threads, 8 complex values per thread.
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

// Sum of a double over the 64 lanes of a wavefront (all lanes active), returned in every
// lane.  The lanes are combined with DPP moves, which run on the vector ALU, instead of LDS
// permutes: pairs and quads by quad permutes, the four quads of each 16-lane row by two row
// rotations (every lane then holds its row's sum), the four rows by reading one lane of each.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_f64(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x124>(v);  // row_ror:4
    v += dpp_f64<0x128>(v);  // row_ror:8
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

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

// ---------------------------------------------------------------------------
// Register-resident transform.  Thread (c, j), j in [0, L/8), holds in v[t] the
// element e = j + t L/8 of pencil c.  Every Stockham stage reads exactly these
// elements: butterfly b (of 8/R per thread) of radix R takes u = j + b L/8 and its
// inputs u + s L/R, i.e. slot t = b + s (8/R).  Intermediate outputs go to LDS at
// their self-sorting positions and are read back in the same slot pattern; the
// last stage leaves X[j + t L/8] in v[t] (natural order), so global loads and
// stores need no LDS staging.
//
// Layouts of the exchange buffer: JF (lanes run along j, for contiguous rows)
// keeps pencils apart, element e of pencil c at c (L + L/8) + e + e/8; otherwise
// (lanes run along c, for strided columns) element-major at e (C + 1) + c.
template <int L, int C, bool JF>
struct Pen {
    static constexpr int T = L / 8;                        // threads per pencil
    static constexpr int NT = C * T;                       // threads per workgroup
    static constexpr int LDS = JF ? C * (L + L / 8) : L * (C + 1);
    static __device__ __forceinline__ int c() { return JF ? (int)threadIdx.x / T : (int)threadIdx.x % C; }
    static __device__ __forceinline__ int j() { return JF ? (int)threadIdx.x % T : (int)threadIdx.x / C; }
    static __device__ __forceinline__ int idx(int e, int cc) {
        return JF ? cc * (L + L / 8) + e + (e >> 3) : e * (C + 1) + cc;
    }
};

template <int L, int C, bool JF, int R, int NS, class V>
__device__ __forceinline__ void reg_stage(V (&v)[8], V* lds, const V* __restrict__ tw, typename CxT<V>::S sg,
                                          int c, int j) {
    using P = Pen<L, C, JF>;
    constexpr int NB = 8 / R;
    constexpr bool FIRST = (NS == 1);
    constexpr bool LAST = (NS * R == L);
    if (!FIRST) {  // gather this stage's inputs (written by the previous stage)
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = lds[P::idx(j + t * (L / 8), c)];
    }
    V y[8];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int u = j + b * (L / 8);
        const int k = u & (NS - 1);
        V w[R];
#pragma unroll
        for (int s = 0; s < R; ++s) w[s] = v[b + s * NB];
        if (NS > 1) {
#pragma unroll
            for (int s = 1; s < R; ++s) {
                V t = tw[(s * k) * (FIRM_TWN / (NS * R))];
                t.y *= -sg;  // table holds exp(-2 pi i m / T); sg = +1 conjugates
                w[s] = c_mul(w[s], t);
            }
        }
        DftSmall<R, V>::run(w, sg);
#pragma unroll
        for (int s = 0; s < R; ++s) y[b + s * NB] = w[s];
    }
    if (LAST) {
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = y[t];
    } else {
        __syncthreads();  // every thread has read the buffer's previous contents
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int u = j + b * (L / 8);
            const int k = u & (NS - 1);
#pragma unroll
            for (int s = 0; s < R; ++s) lds[P::idx((u - k) * R + k + s * NS, c)] = y[b + s * NB];
        }
        __syncthreads();
    }
}

constexpr int first_radix(int L) {
    int r = L;
    while (r > 8) r /= 8;
    return r;
}

template <int L, int C, bool JF, int NS, class V>
__device__ __forceinline__ void reg_stages(V (&v)[8], V* lds, const V* __restrict__ tw, typename CxT<V>::S sg,
                                           int c, int j) {
    if constexpr (NS < L) {
        // the radix-2 or radix-4 stage (lengths not a power of 8) goes first
        constexpr int R = NS == 1 ? first_radix(L) : 8;
        reg_stage<L, C, JF, R, NS, V>(v, lds, tw, sg, c, j);
        reg_stages<L, C, JF, NS * R, V>(v, lds, tw, sg, c, j);
    }
}

// In-register transform of the thread's 8 slots (see above).  The exchange buffer may
// hold anything on entry; it is free again after the call returns (no pending reads).
template <int L, int C, bool JF, class V>
__device__ __forceinline__ void fft_reg(V (&v)[8], V* lds, const V* __restrict__ tw, typename CxT<V>::S sg) {
    using P = Pen<L, C, JF>;
    reg_stages<L, C, JF, 1, V>(v, lds, tw, sg, P::c(), P::j());
}

// pencils per workgroup for each length (threads = C * L / 8)
template <int L, class V = float2>
struct FftCfg {
    static constexpr bool DBL = sizeof(V) == 16;
    static constexpr int C = DBL ? (L >= 1024 ? 4 : (L >= 256 ? 8 : (L >= 128 ? 16 : 2048 / L)))
                                 : (L >= 1024 ? 8 : (L >= 128 ? 16 : 2048 / L));
    static constexpr int THREADS = C * L / 8;
};
