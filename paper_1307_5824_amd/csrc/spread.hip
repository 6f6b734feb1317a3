// Type-1 non-uniform FFT gridding of libfirm (section 3.4, steps 2 and 3).
//
// Ker (eq. kernel) and A*b (eq. backprojection) are sums over the sample points
// xi_{k,m} = R_m^{-1}(omega_k, 0).  In fine-grid units (grid size L = s N) the
// point is t = s (k1 c1_m + k2 c2_m), c1, c2 the first two columns of R_m^{-1}.
// Each point is spread with a separable Kaiser-Bessel window of width W onto a
// periodic grid; a grid FFT divided by the window's transform gives the sums.
//
// Work decomposition: the grid is cut into T^3 tiles.  A workgroup owns one
// tile (or one tile and a range of images): it tests every image plane of its
// range against the tile's circumscribed sphere, enumerates the disk points of
// the surviving images whose cell floor(t + L/2) lies in the tile, and
// accumulates their full W^3 stencils into a (T + W)^3 LDS tile; the tile is
// then added to the global grid with one atomic per cell.  Each point is spread
// exactly once.
//
// The LDS accumulation uses no atomics (LDS float atomics run at a fraction of
// the plain read/write rate on this chip).  Each wavefront owns a slab of rows
// (first tile axis) of the padded tile.  The per-point window weights are
// computed once, one thread per point, and staged in LDS; then every wavefront
// walks the staged points whose W rows meet its slab, with its lanes on the
// W x W footprint of the other two axes: all W rows are read, updated and
// written back inside the slab.  Within one instruction the lanes' cells are
// distinct and no two wavefronts write the same row, so the plain
// read-modify-write is race-free.  Only the half disk (k1 > 0, or k1 = 0 and
// k2 > 0) is spread: its partner -k is folded in (Ker is real and even; for A*b
// the pair (k, -k) gives the real part exactly), and k = 0 is added afterwards
// in closed form.
#include <algorithm>
#include <cmath>
#include <vector>

#include "firm_internal.h"

#define KB_DEG 10
#define SP_QCAP 1024

namespace {

struct SpreadArgs {
    int N, M, L, nt;
    double s;
    const double* c12;
    const float* nrm;
    const int32_t* group;
    const float* table;
    int Q;
    const float* poly;
    const int4* work;
    void* grid;
    const float2* b;
    const double* shifts;
    const int* rowstart;  // index of (k1, 0) shifted: idx(k1, k2) = rowstart[k1 + N/2] + k2
    int P;
};

template <int W>
__device__ __forceinline__ void kb_weights(const float* __restrict__ poly, float x, float* out) {
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const float* c = poly + j * (KB_DEG + 1);
        float v = c[KB_DEG];
#pragma unroll
        for (int d = KB_DEG - 1; d >= 0; --d) v = fmaf(v, x, c[d]);
        out[j] = v;
    }
}

// Smallest LDS row pitch >= PT at which the W x W footprint cells j2 * pitch + j3 of one
// instruction fall in distinct banks (64 banks of 4 bytes).
constexpr int row_pitch(int PT, int W) {
    for (int rp = PT; rp < PT + 32; ++rp) {
        bool ok = true;
        for (int a = 0; a < W * W && ok; ++a)
            for (int b = a + 1; b < W * W && ok; ++b)
                if (((a / W) * rp + a % W) % 64 == ((b / W) * rp + b % W) % 64) ok = false;
        if (ok) return rp;
    }
    return PT;
}

template <int T, int W, bool CPLX, int NTH>
__global__ void __launch_bounds__(NTH, NTH / 128) k_spread(SpreadArgs a) {
    constexpr int SP_THREADS = NTH, SP_WAVES = NTH / 64;
    constexpr int PT = T + W;
    constexpr int PADLO = (W + 1) / 2 - 1;
    constexpr int NCELL = PT * PT * PT;
    constexpr int H = (PT + SP_WAVES - 1) / SP_WAVES;  // rows per wavefront slab
    constexpr int RP = row_pitch(PT, W);               // LDS pitch of a tile row (bank-conflict free)
    constexpr int PP = PT * RP;                        // LDS pitch of a tile plane
    constexpr int NR = SP_WAVES * H;                   // planes, padded to whole slabs
    constexpr int NV = CPLX ? 2 : 1;                   // real and imaginary parts in separate tiles
    // staged point: for each wavefront its H slab-row weights (0 outside the window), then the
    // window weights of axes 1 and 2; stride in floats
    constexpr int PSTR = ((SP_WAVES * H + 2 * W) + 3) / 4 * 4;
    static_assert(W <= 8, "window width");
    constexpr int SP_PB = 96;                          // points staged per batch (two tiles per CU)
    __shared__ __align__(16) float tile[NV * NR * PP];
    __shared__ __align__(16) float pt_w[SP_PB * PSTR];
    __shared__ int pt_lo[SP_PB];
    __shared__ float2 pt_v[CPLX ? SP_PB : 1];
    constexpr int NK = PT - W + 1;                     // possible first rows of a window
    __shared__ int pt_key[SP_PB], pt_slot[SP_PB], bstart[NK + 1];
    __shared__ int img_m[SP_THREADS];
    __shared__ int img_k1[SP_THREADS];
    __shared__ int queue[SP_QCAP];
    __shared__ int nimg, qn, qfail, any;

    const int tid = threadIdx.x;
    const int4 wk = a.work[blockIdx.x];
    const int nt = a.nt;
    const int tt[3] = {wk.x / (nt * nt), (wk.x / nt) % nt, wk.x % nt};
    const int L = a.L, N = a.N;
    const double halfL = 0.5 * L;

    for (int i = tid; i < NV * NR * PP; i += SP_THREADS) tile[i] = 0.f;
    if (tid == 0) any = 0;

    const double tc[3] = {tt[0] * T + 0.5 * T - halfL, tt[1] * T + 0.5 * T - halfL, tt[2] * T + 0.5 * T - halfL};
    const double Rt = T * 0.8660254037844386 + 1e-3;
    const double rk = Rt / a.s;
    const int S = (int)floor(2.0 * rk) + 3;
    const int N2 = N * N;

    // points of the queue [0, nq) staged and accumulated in batches of SP_PB
    auto process = [&](int nq) {
        if (tid == 0 && nq > 0) any = 1;
        const int wv = tid >> 6, lane = tid & 63;
        const int r0 = wv * H;                                   // this wave's rows [r0, r0 + H)
        for (int pb = 0; pb < nq; pb += SP_PB) {
            const int nb = min(SP_PB, nq - pb);
            // stage the batch: each of its threads computes one point's tile-relative window
            // start and weights; wave 0 ranks the points by their first row (counting sort
            // with ballots); each point is then written to its rank, so that the points
            // meeting a wavefront's slab form one contiguous range
            float ph[3][W];
            int lo[3] = {0, 0, 0};
            float scale = 1.f;
            float2 pval = make_float2(0.f, 0.f);
            if (tid < nb) {
                const int e = queue[pb + tid];
                const int sl = e >> 18, k1 = ((e >> 9) & 511) - 256, k2 = (e & 511) - 256;
                const int m = img_m[sl];
                const double* c = a.c12 + 6 * (int64_t)m;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    // |t_d| <= L/2 in exact arithmetic; clamp the rounding excess so the
                    // stencil stays inside the padded tile for every width
                    const double tau = fmin(fmax(a.s * (k1 * c[d] + k2 * c[3 + d]) + halfL, 0.0), (double)L);
                    const double left = tau - 0.5 * W;
                    const int b0 = (int)floor(left) + 1;
                    const float f = (float)((double)b0 - left);  // in (0, 1]
                    kb_weights<W>(a.poly, 2.f * f - 1.f, ph[d]);
                    // in [0, PT - W] for every point of the tile (clamped position); the bound
                    // also keeps the LDS accesses inside the tile should rounding ever differ
                    lo[d] = min(max(b0 - (tt[d] * T - PADLO), 0), PT - W);
                }
                const int g = a.group ? a.group[m] : 0;
                const float h = a.table ? a.table[(int64_t)g * a.Q + k1 * k1 + k2 * k2] : 1.f;
                if constexpr (!CPLX) {
                    scale = 2.f * h * h;
                } else {
                    // h exp(i theta) (b(k) + conj b(-k)), theta = 2 pi <k, s_m> / N (re-centring)
                    const int idx = a.rowstart[k1 + N / 2] + k2;
                    const float2 bp = a.b[(int64_t)m * a.P + idx];
                    const float2 bm = a.b[(int64_t)m * a.P + (a.P - 1 - idx)];
                    const float sr = bp.x + bm.x, si = bp.y - bm.y;
                    float cs = 1.f, sn = 0.f;
                    if (a.shifts) {
                        const double th = 6.283185307179586 * (k1 * a.shifts[2 * (int64_t)m] +
                                                              k2 * a.shifts[2 * (int64_t)m + 1]) / N;
                        cs = (float)cos(th);
                        sn = (float)sin(th);
                    }
                    pval = make_float2(h * (cs * sr - sn * si), h * (cs * si + sn * sr));
                }
                pt_key[tid] = lo[0];
            }
            __syncthreads();
            if (tid < 64) {
                constexpr int NCH = (SP_PB + 63) / 64;
                const int ln = tid;
                const uint64_t lt = (1ull << ln) - 1ull;
                int key[NCH];
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) key[ch] = ch * 64 + ln < nb ? pt_key[ch * 64 + ln] : -1;
                int run = 0;
                for (int v = 0; v < NK; ++v) {
                    if (ln == 0) bstart[v] = run;
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) {
                        const uint64_t msk = __ballot(key[ch] == v);
                        if (key[ch] == v) pt_slot[ch * 64 + ln] = run + __popcll(msk & lt);
                        run += __popcll(msk);
                    }
                }
                if (ln == 0) bstart[NK] = run;
            }
            __syncthreads();
            if (tid < nb) {
                const int d = pt_slot[tid];
                float* q = pt_w + d * PSTR;
#pragma unroll
                for (int r = 0; r < SP_WAVES * H; ++r) {  // row r of the padded tile
                    const int j1 = r - lo[0];
                    float w = 0.f;
#pragma unroll
                    for (int j = 0; j < W; ++j) w = (j1 == j) ? ph[0][j] : w;
                    q[r] = scale * w;
                }
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    q[SP_WAVES * H + j] = ph[1][j];
                    q[SP_WAVES * H + W + j] = ph[2][j];
                }
                pt_lo[d] = lo[0] | (lo[1] << 8) | (lo[2] << 16);
                if constexpr (CPLX) pt_v[d] = pval;
            }
            __syncthreads();
            // this wavefront's points: first row in [r0 - W + 1, r0 + H - 1], taken two at a time;
            // when the two footprints are disjoint both points' rows are read before either is
            // written back (two independent read-modify-write chains in flight)
            const int vlo = max(0, r0 - W + 1), vhi = min(NK - 1, r0 + H - 1);
            const int pbeg = vlo <= vhi ? bstart[vlo] : 0, pend = vlo <= vhi ? bstart[vhi + 1] : 0;
            constexpr int A2 = SP_WAVES * H, A3 = SP_WAVES * H + W;
            const int jl = lane < W * W ? lane : 0;
            const int j2 = jl / W, j3 = jl - (jl / W) * W;  // footprint cell of this lane
            const bool act = lane < W * W;
            struct Pt {
                int cb, l1, l2;
                float rw[H];
                float w23;
                float2 v;
            };
            auto load = [&](int pi, Pt& q) {
                const float* w = pt_w + pi * PSTR;
                const int lw = pt_lo[pi];
                q.l1 = (lw >> 8) & 255;
                q.l2 = lw >> 16;
                q.cb = r0 * PP + (q.l1 + j2) * RP + q.l2 + j3;
#pragma unroll
                for (int k = 0; k < H; ++k) q.rw[k] = w[r0 + k];
                q.w23 = w[A2 + j2] * w[A3 + j3];
                q.v = CPLX ? pt_v[pi] : make_float2(0.f, 0.f);
            };
            // rows of the slab: read, then add weight * value (weight 0 outside the window)
            auto rd = [&](const Pt& q, float (&vr)[H], float (&vi)[H]) {
#pragma unroll
                for (int k = 0; k < H; ++k) {
                    vr[k] = tile[q.cb + k * PP];
                    if (CPLX) vi[k] = tile[NR * PP + q.cb + k * PP];
                }
            };
            auto wr = [&](const Pt& q, const float (&vr)[H], const float (&vi)[H]) {
                if constexpr (!CPLX) {
#pragma unroll
                    for (int k = 0; k < H; ++k) tile[q.cb + k * PP] = fmaf(q.rw[k], q.w23, vr[k]);
                } else {
                    const float sr = q.w23 * q.v.x, si = q.w23 * q.v.y;
#pragma unroll
                    for (int k = 0; k < H; ++k) {
                        tile[q.cb + k * PP] = fmaf(q.rw[k], sr, vr[k]);
                        tile[NR * PP + q.cb + k * PP] = fmaf(q.rw[k], si, vi[k]);
                    }
                }
            };
            for (int pi = pbeg; pi < pend; pi += 2) {
                const bool two = pi + 1 < pend;
                Pt a, b;
                load(pi, a);
                load(two ? pi + 1 : pi, b);
                const bool apart = two && (abs(a.l1 - b.l1) >= W || abs(a.l2 - b.l2) >= W);
                float ar[H], ai[H], br[H], bi[H];
                if (act) {
                    if (apart) {
                        rd(a, ar, ai);
                        rd(b, br, bi);
                        wr(a, ar, ai);
                        wr(b, br, bi);
                    } else {
                        rd(a, ar, ai);
                        wr(a, ar, ai);
                        if (two) {
                            rd(b, br, bi);
                            wr(b, br, bi);
                        }
                    }
                }
            }
            __syncthreads();
        }
    };

    // positions tau whose (clamped) cell lies in the tile, widened by a margin far above the
    // rounding of the row intervals; the edge tiles also own the clamped cells beyond the grid
    constexpr double MARGIN = 1e-3, FAR = 1e30;
    double blo[3], bhi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        blo[d] = tt[d] == 0 ? -FAR : tt[d] * T - MARGIN;
        bhi[d] = (tt[d] + 1) * T >= L ? FAR : (tt[d] + 1) * T + MARGIN;
    }
    if (tid == 0) { qn = 0; qfail = SP_QCAP; }

    for (int mb = wk.y; mb < wk.z; mb += SP_THREADS) {
        __syncthreads();
        if (tid == 0) nimg = 0;
        __syncthreads();
        const int m = mb + tid;
        if (m < wk.z) {
            const float* n = a.nrm + 4 * (int64_t)m;
            const double dist = fabs(tc[0] * n[0] + tc[1] * n[1] + tc[2] * n[2]);
            if (dist <= Rt + 1e-3) {
                const double* c = a.c12 + 6 * (int64_t)m;
                const double u1 = (tc[0] * c[0] + tc[1] * c[1] + tc[2] * c[2]) / a.s;
                const int sl = atomicAdd(&nimg, 1);
                img_m[sl] = m;
                img_k1[sl] = (int)ceil(u1 - rk) - 1;  // first candidate row
            }
        }
        __syncthreads();
        // one (view, row k1) per thread: the k2 interval whose cells lie in the tile (three slabs,
        // plus the disk and half-disk bounds), the exact cell test per point (a bit mask), then
        // the points are queued.  A reservation that does not fit waits for the queue to be
        // processed; the reservations that fitted form the prefix up to the first that did not.
        const int units = nimg * S;
        for (int ub = 0; ub < units; ub += SP_THREADS) {
            const int u = ub + tid;
            int sl = 0, k1 = 0, klo = 0;
            uint32_t mask = 0u;
            if (u < units) {
                sl = u / S;
                k1 = img_k1[sl] + (u - sl * S);
                if (k1 >= 0 && 4 * k1 * k1 <= N2) {
                    const double* c = a.c12 + 6 * (int64_t)img_m[sl];
                    const int kd = (int)sqrt((double)(N2 / 4 - k1 * k1)) + 1;  // >= the disk's |k2|
                    double lo = -kd, hi = kd;
                    bool ok = true;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const double al = a.s * k1 * c[d] + halfL, be = a.s * c[3 + d];
                        if (fabs(be) < 1e-9) {
                            ok = ok && al >= blo[d] && al <= bhi[d];
                        } else {
                            const double t1 = (blo[d] - al) / be, t2 = (bhi[d] - al) / be;
                            lo = fmax(lo, fmin(t1, t2));
                            hi = fmin(hi, fmax(t1, t2));
                        }
                    }
                    klo = (int)ceil(lo);
                    if (k1 == 0) klo = max(klo, 1);
                    // a row crosses a tile in at most T sqrt(3) / s + 1 points
                    const int cnt = ok && hi >= klo ? min((int)floor(hi) - klo + 1, 32) : 0;
                    for (int j = 0; j < cnt; ++j) {
                        const int k2 = klo + j;
                        bool in = 4 * (k1 * k1 + k2 * k2) <= N2;
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const double tau = a.s * (k1 * c[d] + k2 * c[3 + d]) + halfL;
                            int cell = (int)floor(tau);
                            cell = cell < 0 ? 0 : (cell > L - 1 ? L - 1 : cell);
                            in = in && (cell / T == tt[d]);
                        }
                        if (in) mask |= 1u << j;
                    }
                }
            }
            const int c = __popc(mask);
            bool pend = c > 0;
            while (true) {
                if (pend) {
                    const int pos = atomicAdd(&qn, c);
                    if (pos + c <= SP_QCAP) {
                        uint32_t mk = mask;
                        for (int w = pos; mk; ++w) {
                            const int j = __ffs(mk) - 1;
                            mk &= mk - 1u;
                            queue[w] = (sl << 18) | ((k1 + 256) << 9) | (klo + j + 256);
                        }
                        pend = false;
                    } else {
                        atomicMin(&qfail, pos);
                    }
                }
                if (!__syncthreads_or(pend)) break;
                process(min(qfail, qn));  // the queue is full
                __syncthreads();
                if (tid == 0) { qn = 0; qfail = SP_QCAP; }
                __syncthreads();
            }
        }
        // the view slots are refilled next round: process what is queued
        process(qn);
        __syncthreads();
        if (tid == 0) { qn = 0; qfail = SP_QCAP; }
    }
    __syncthreads();
    if (!any) return;
    const int o0 = tt[0] * T - PADLO, o1 = tt[1] * T - PADLO, o2 = tt[2] * T - PADLO;
    for (int i = tid; i < NCELL; i += SP_THREADS) {
        const int l0 = i / (PT * PT), l1 = (i / PT) % PT, l2 = i % PT;
        const int li = l0 * PP + l1 * RP + l2;
        // grid index = position mod L, position = cell - L/2
        const int g0 = ((o0 + l0 - L / 2) % L + L) % L;
        const int g1 = ((o1 + l1 - L / 2) % L + L) % L;
        const int g2 = ((o2 + l2 - L / 2) % L + L) % L;
        const int64_t gi = ((int64_t)g0 * L + g1) * L + g2;
        if (!CPLX) {
            const float v = tile[li];
            if (v != 0.f) unsafeAtomicAdd(reinterpret_cast<float*>(a.grid) + gi, v);
        } else {
            const float vr = tile[li], vi = tile[NR * PP + li];
            float* gp = reinterpret_cast<float*>(a.grid) + 2 * gi;
            if (vr != 0.f) unsafeAtomicAdd(gp, vr);
            if (vi != 0.f) unsafeAtomicAdd(gp + 1, vi);
        }
    }
}

__global__ void k_fill_zero(float4* p, size_t n4) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Re sum_m h_m(0) b(0, m): the k = 0 term of Re A*b (its exponential is 1 for all n).
__global__ void k_atb_k0(const float2* __restrict__ b, const int32_t* group, const float* table, int Q, int M,
                         int P, double* out) {
    __shared__ double red[4];
    double acc = 0.0;
    const int c = (P - 1) / 2;
    for (int m = threadIdx.x; m < M; m += 256) {
        const int g = group ? group[m] : 0;
        const float h = table ? table[(int64_t)g * Q] : 1.f;
        acc += (double)h * (double)b[(int64_t)m * P + c].x;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = red[0] + red[1] + red[2] + red[3];
}

// chalf[p1][p2][n3] (n3 in [0, N)) -> kerc[p1][p2][p3] using Ker(-n) = Ker(n); p3 = N is 0.
__global__ void k_kerc_from_half(const float* __restrict__ chalf, float* __restrict__ kerc, int N) {
    const int N2 = 2 * N;
    const int64_t tot = (int64_t)N2 * N2 * N2;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int p3 = (int)(i % N2), p2 = (int)((i / N2) % N2), p1 = (int)(i / ((int64_t)N2 * N2));
        float v;
        if (p3 < N) v = chalf[((int64_t)p1 * N2 + p2) * N + p3];
        else if (p3 == N) v = 0.f;
        else v = chalf[((int64_t)((N2 - p1) % N2) * N2 + (N2 - p2) % N2) * N + (N2 - p3)];
        kerc[i] = v;
    }
}

// circulant order c[p] (offset o(p)) <-> centred order ker[j] (offset j - N)
__global__ void k_kerc_centred(const float* __restrict__ src, float* __restrict__ dst, int N, int to_centred) {
    const int N2 = 2 * N;
    const int64_t tot = (int64_t)N2 * N2 * N2;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int a3 = (int)(i % N2), a2 = (int)((i / N2) % N2), a1 = (int)(i / ((int64_t)N2 * N2));
        // index a in the destination order; map to the source order
        int s1, s2, s3;
        if (to_centred) {  // dst centred j -> offset j - N -> circulant p = offset mod 2N
            s1 = (a1 - N + N2) % N2; s2 = (a2 - N + N2) % N2; s3 = (a3 - N + N2) % N2;
            const bool wrap = (a1 == 0) || (a2 == 0) || (a3 == 0);
            dst[i] = wrap ? 0.f : src[((int64_t)s1 * N2 + s2) * N2 + s3];
        } else {           // dst circulant p -> offset o(p) -> centred j = o + N; p = N is the wrap
            const bool wrap = (a1 == N) || (a2 == N) || (a3 == N);
            s1 = (a1 + N) % N2; s2 = (a2 + N) % N2; s3 = (a3 + N) % N2;
            dst[i] = wrap ? 0.f : src[((int64_t)s1 * N2 + s2) * N2 + s3];
        }
    }
}

__global__ void k_f2d(const float* __restrict__ a, double* __restrict__ o, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        o[i] = a[i];
}

int grid_blocks(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 65536); }

// Ker (real tile): 8 wavefronts with 3-row slabs; A*b (two tiles, re and im): 4 with 5-row slabs,
// so that two workgroups fit the LDS of a compute unit in both cases.
template <int T, bool CPLX, int NTH = CPLX ? 256 : 512>
hipError_t launch_spread(firm_plan p, int L, const int* work, int nwork, void* grid, const float2* b) {
    SpreadArgs a;
    a.N = p->N; a.M = p->M; a.L = L; a.nt = (L + T - 1) / T;
    a.s = (double)L / p->N;
    a.c12 = p->c12; a.nrm = p->nrm; a.group = p->group; a.table = p->table; a.Q = p->Q;
    a.poly = p->kb_poly; a.work = reinterpret_cast<const int4*>(work); a.grid = grid;
    a.b = b; a.shifts = p->shifts; a.rowstart = p->rowstart; a.P = p->P;
    if (nwork == 0) return hipSuccess;
    switch (p->kbw) {
        case 4: hipLaunchKernelGGL((k_spread<T, 4, CPLX, NTH>), dim3(nwork), dim3(NTH), 0, p->stream, a); break;
        case 5: hipLaunchKernelGGL((k_spread<T, 5, CPLX, NTH>), dim3(nwork), dim3(NTH), 0, p->stream, a); break;
        case 6: hipLaunchKernelGGL((k_spread<T, 6, CPLX, NTH>), dim3(nwork), dim3(NTH), 0, p->stream, a); break;
        case 7: hipLaunchKernelGGL((k_spread<T, 7, CPLX, NTH>), dim3(nwork), dim3(NTH), 0, p->stream, a); break;
        case 8: hipLaunchKernelGGL((k_spread<T, 8, CPLX, NTH>), dim3(nwork), dim3(NTH), 0, p->stream, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

#define SP_TILE_REAL 16
#define SP_TILE_CPLX 12

// Host work list: tiles of an L^3 grid that can hold points (|centre| - R <= L/2), each
// split into image ranges of about `chunk` images for the most loaded tiles, ordered by
// expected work (tiles near the origin meet every image plane) so that the heavy ones start first.
std::vector<int> spread_worklist(int L, int T, int M, double s) {
    const int nt = (L + T - 1) / T;
    const double Rt = T * 0.8660254037844386;
    struct Item { double w; int t, m0, m1; };
    std::vector<Item> items;
    const int chunk = 16384;
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b)
            for (int c = 0; c < nt; ++c) {
                const double x = a * T + 0.5 * T - 0.5 * L, y = b * T + 0.5 * T - 0.5 * L,
                             z = c * T + 0.5 * T - 0.5 * L;
                const double rho = std::sqrt(x * x + y * y + z * z);
                if (rho - Rt > 0.5 * L + 1.0) continue;
                const double frac = rho <= Rt ? 1.0 : Rt / rho;
                const double expect = frac * M;
                const int nch = std::max(1, (int)std::ceil(expect / chunk));
                const int per = (M + nch - 1) / nch;
                for (int k = 0; k < nch; ++k) {
                    const int m0 = k * per, m1 = std::min(M, m0 + per);
                    if (m0 < m1) items.push_back({expect / nch, (a * nt + b) * nt + c, m0, m1});
                }
            }
    std::stable_sort(items.begin(), items.end(), [](const Item& u, const Item& v) { return u.w > v.w; });
    std::vector<int> out;
    out.reserve(items.size() * 4);
    for (auto& it : items) { out.push_back(it.t); out.push_back(it.m0); out.push_back(it.m1); out.push_back(0); }
    (void)s;
    return out;
}

int spread_tile_real() { return SP_TILE_REAL; }
int spread_tile_cplx() { return SP_TILE_CPLX; }

hipError_t fill_zero(void* ptr, size_t bytes, hipStream_t s) {
    const size_t n4 = bytes / 16;
    if (n4) hipLaunchKernelGGL(k_fill_zero, dim3(grid_blocks(n4)), dim3(256), 0, s, (float4*)ptr, n4);
    const size_t rem = bytes - n4 * 16;
    if (rem) {
        hipError_t e = hipMemsetAsync((char*)ptr + n4 * 16, 0, rem, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t spread_ker(firm_plan p, float* grid) {
    return launch_spread<SP_TILE_REAL, false>(p, 4 * p->N, p->tiles_ker, p->ntiles_ker, grid, nullptr);
}

hipError_t spread_atb(firm_plan p, const float2* b, float2* grid) {
    return launch_spread<SP_TILE_CPLX, true>(p, 2 * p->N, p->tiles_atb, p->ntiles_atb, grid, b);
}

hipError_t atb_k0_term(firm_plan p, const float2* b, double* out) {
    hipLaunchKernelGGL(k_atb_k0, dim3(1), dim3(256), 0, p->stream, b, p->group, p->table, p->Q, p->M, p->P, out);
    return hipGetLastError();
}

hipError_t kerc_from_half(firm_plan p, const float* chalf) {
    const int64_t n = 8LL * p->N * p->N * p->N;
    hipLaunchKernelGGL(k_kerc_from_half, dim3(grid_blocks(n)), dim3(256), 0, p->stream, chalf, p->kerc, p->N);
    return hipGetLastError();
}

hipError_t kerc_to_centred(firm_plan p, float* out) {
    const int64_t n = 8LL * p->N * p->N * p->N;
    hipLaunchKernelGGL(k_kerc_centred, dim3(grid_blocks(n)), dim3(256), 0, p->stream, p->kerc, out, p->N, 1);
    return hipGetLastError();
}

hipError_t kerc_from_centred(firm_plan p, const float* in) {
    const int64_t n = 8LL * p->N * p->N * p->N;
    hipLaunchKernelGGL(k_kerc_centred, dim3(grid_blocks(n)), dim3(256), 0, p->stream, in, p->kerc, p->N, 0);
    return hipGetLastError();
}

hipError_t kerc_to_double(firm_plan p, double* out) {
    const int64_t n = 8LL * p->N * p->N * p->N;
    hipLaunchKernelGGL(k_f2d, dim3(grid_blocks(n)), dim3(256), 0, p->stream, p->kerc, out, n);
    return hipGetLastError();
}
