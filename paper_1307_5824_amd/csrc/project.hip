// Forward projector of libfirm (eq. forward-projector): slices of a volume at the sample
// points xi_{k,m} = R_m^{-1}(omega_k, 0), with the CTF and the image shift applied,
//
//   b(k, m) = h_m(|k|) exp(-i <omega_k, s_m>) sum_n V(n) exp(-i <n, xi_{k,m}>).
//
// This is the adjoint of the back-projection (spread.hip; it re-centres by
// exp(+i <omega_k, s_m>)), evaluated as a type-2 non-uniform FFT on the same grid (L = 2N),
// with the same Kaiser-Bessel window and the same cell convention:
//   1. u(n) = V(n) / phihat(n1) phihat(n2) phihat(n3)      (the window's transform)
//   2. G(g) = sum_n u(n) exp(-2 pi i <n, g> / L), g in [0, L)^3 (three FFT passes; real u,
//      so only q3 in [0, N] is formed, the rest is conj G(-g))
//   3. b = sum over the W^3 window cells of weight * G(cell), one thread per sample point.
// Step 3 walks the grid in T^3 tiles, the transpose of the gridding spread: a workgroup loads
// its (T + W)^3 padded tile of G into LDS once, finds the sample points whose cell lies in
// the tile (plane test, then the disk points near the plane), and each thread gathers one
// point's W^3 window from LDS.  Every point belongs to exactly one tile, so every output is
// written once, with no atomics.  The half disk (k1 > 0, or k1 = 0 and k2 > 0) is gathered;
// b(-k) = conj b(k) for real V, and b(0) = h(0) sum V is formed exactly.
#include <algorithm>
#include <cmath>

#include "firm_internal.h"

#define KB_DEG 10
#define PJ_TILE 12
#define PJ_QCAP 2048
#define PJ_THREADS 512
#define PJ_PREP_BLOCKS 1024
#define PJ_VPT 2

namespace {

struct ProjArgs {
    int N, M, L, nt, P, Q, QP;
    double s;
    // per-view arrays in the order of the views' normals (blocks of 512 views with the box of
    // their normals in vbox), and the map from that order to the caller's
    const double* c12;
    const float* nrm;
    const int32_t* group;
    const int* vorder;
    const float4* vbox;
    const float* table;
    const float* poly;
    const int4* work;
    const float2* X;       // [q1][q2][q3], q3 in [0, N], pitch QP
    const double* shifts;
    const int* rowstart;
    float2* b;
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

// u = V / (phihat(n1) phihat(n2) phihat(n3)) and per-block FP64 partial sums of V.
__global__ void __launch_bounds__(256) k_fp_prep(const float* __restrict__ V, const float* __restrict__ dec, int N,
                                                 float* __restrict__ u, double* __restrict__ partials) {
    __shared__ double red[4];
    const int64_t n3 = (int64_t)N * N * N;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n3; i += (int64_t)gridDim.x * 256) {
        const int i3 = (int)(i % N), i2 = (int)((i / N) % N), i1 = (int)(i / ((int64_t)N * N));
        const float v = V[i];
        acc += (double)v;
        u[i] = v * dec[i1] * dec[i2] * dec[i3];
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// b(0, m) = h_m(0) sum V; every block forms the same sum of the partials in the same order.
__global__ void __launch_bounds__(256) k_fp_k0(const double* __restrict__ partials, int nblk,
                                               const int32_t* __restrict__ group, const float* __restrict__ table,
                                               int Q, int M, int P, float2* __restrict__ b) {
    __shared__ double red[4];
    __shared__ float total;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) acc += partials[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) total = (float)((red[0] + red[1]) + (red[2] + red[3]));
    __syncthreads();
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= M) return;
    const int g = group ? group[m] : 0;
    const float h = table ? table[(int64_t)g * Q] : 1.f;
    b[(int64_t)m * P + (P - 1) / 2] = make_float2(h * total, 0.f);
}

// G at grid index q from the half spectrum X of the array-index transform: the volume sits at
// n = i - N/2, so G(q) = i^(q1 + q2 + q3) X(q) (L is a multiple of 4), and X(q) = conj X(-q).
__device__ __forceinline__ float2 grid_value(const float2* __restrict__ X, int L, int N, int QP, int q0, int q1,
                                             int q2) {
    float2 v;
    if (q2 <= N) {
        v = X[((int64_t)q0 * L + q1) * QP + q2];
    } else {
        const int r0 = q0 == 0 ? 0 : L - q0, r1 = q1 == 0 ? 0 : L - q1;
        v = X[((int64_t)r0 * L + r1) * QP + (L - q2)];
        v.y = -v.y;
    }
    switch ((q0 + q1 + q2) & 3) {
        case 1: return make_float2(-v.y, v.x);
        case 2: return make_float2(-v.x, -v.y);
        case 3: return make_float2(v.y, -v.x);
        default: return v;
    }
}

// Fine-grid position of the disk point (k1, k2) of a view along axis d, in the form the
// gridding spread uses: the point enumeration (which tile owns a point) and the gather (where
// its window starts) evaluate this one expression, so the two agree to the last bit.
__device__ __forceinline__ double tau_of(double s, int k1, int k2, double cd, double c3d, double halfL) {
    return fma(s, fma((double)k2, c3d, (double)k1 * cd), halfL);
}

// One queued point: view m and disk point (k1, k2) of the half disk.
template <int T, int W>
__device__ __forceinline__ void gather_point(const ProjArgs& a, const float2* __restrict__ tile, const int* tt, int m,
                                             int k1, int k2) {
    constexpr int PT = T + W;
    constexpr int PADLO = (W + 1) / 2 - 1;
    const int N = a.N;
    const double halfL = 0.5 * a.L;
    const double* c = a.c12 + 6 * (int64_t)m;
    float ph[3][W];
    int lo[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // window start and weights exactly as the gridding spread forms them
        const double tau = fmin(fmax(tau_of(a.s, k1, k2, c[d], c[3 + d], halfL), 0.0), (double)a.L);
        const double left = tau - 0.5 * W;
        const int b0 = (int)floor(left) + 1;
        const float f = (float)((double)b0 - left);  // in (0, 1]
        kb_weights<W>(a.poly, 2.f * f - 1.f, ph[d]);
        lo[d] = min(max(b0 - (tt[d] * T - PADLO), 0), PT - W);
    }
    // one window plane per iteration (W^2 LDS loads in flight); the plane weight rotates
    // through w0 so that no register array is indexed at run time
    float ar = 0.f, ai = 0.f;
    float w0[W];
#pragma unroll
    for (int t = 0; t < W; ++t) w0[t] = ph[0][t];
    const float2* pl = tile + (lo[0] * PT + lo[1]) * PT + lo[2];
#pragma unroll 1
    for (int j0 = 0; j0 < W; ++j0, pl += PT * PT) {
        const float wp = w0[0];
#pragma unroll
        for (int t = 0; t < W - 1; ++t) w0[t] = w0[t + 1];
#pragma unroll
        for (int j1 = 0; j1 < W; ++j1) {
            const float2* row = pl + j1 * PT;
            float sr = 0.f, si = 0.f;
#pragma unroll
            for (int j2 = 0; j2 < W; ++j2) {
                const float2 g = row[j2];
                sr = fmaf(ph[2][j2], g.x, sr);
                si = fmaf(ph[2][j2], g.y, si);
            }
            const float w = wp * ph[1][j1];
            ar = fmaf(w, sr, ar);
            ai = fmaf(w, si, ai);
            // at most half a plane of loads in flight: keeps the gather within 128 registers
            if (j1 == W / 2) __builtin_amdgcn_sched_barrier(0);
        }
    }
    const int g = a.group ? a.group[m] : 0;
    const float h = a.table ? a.table[(int64_t)g * a.Q + k1 * k1 + k2 * k2] : 1.f;
    float cs = 1.f, sn = 0.f;
    if (a.shifts) {
        // theta = 2 pi x, x = <k, s_m> / N reduced to [-1/2, 1/2] in FP64, then an FP32 sincospi
        const double x = (k1 * a.shifts[2 * (int64_t)m] + k2 * a.shifts[2 * (int64_t)m + 1]) / N;
        sincospif(2.f * (float)(x - rint(x)), &sn, &cs);
    }
    // h exp(-i theta) (ar + i ai), and its conjugate at -k
    const float2 v = make_float2(h * (ar * cs + ai * sn), h * (ai * cs - ar * sn));
    const int idx = a.rowstart[k1 + N / 2] + k2;
    const int64_t mo = a.vorder[m];  // the caller's view index
    a.b[mo * a.P + idx] = v;
    a.b[mo * a.P + (a.P - 1 - idx)] = make_float2(v.x, -v.y);
}

// Four waves per SIMD (two 512-thread workgroups per CU) up to W = 7; the W = 8 gather needs
// more than 128 registers and runs at two.
template <int T, int W, int NTH>
__global__ void __launch_bounds__(NTH, (W <= 7 ? 4 : 2)) k_project(ProjArgs a) {
    constexpr int PT = T + W;                  // padded tile edge (window starts in [0, T])
    constexpr int PADLO = (W + 1) / 2 - 1;
    constexpr int NCELL = PT * PT * PT;
    constexpr int IMGCAP = (PJ_VPT + 1) * NTH;
    __shared__ float2 tile[NCELL];
    __shared__ int img_m[IMGCAP], img_r[IMGCAP];  // surviving views and their first candidate row
    // queued points (view slot, k1, k2), -1 for an unused entry
    __shared__ int queue[PJ_QCAP];
    __shared__ int nimg, qn;

    const int tid = threadIdx.x;
    const int4 wk = a.work[blockIdx.x];
    const int nt = a.nt;
    const int tt[3] = {wk.x / (nt * nt), (wk.x / nt) % nt, wk.x % nt};
    const int L = a.L, N = a.N;
    const double halfL = 0.5 * L;

    // the padded tile of G: LDS cell l holds grid index (tt * T - PADLO + l - L/2) mod L
    const int o0 = tt[0] * T - PADLO - L / 2, o1 = tt[1] * T - PADLO - L / 2, o2 = tt[2] * T - PADLO - L / 2;
    for (int i = tid; i < NCELL; i += NTH) {
        const int l0 = i / (PT * PT), l1 = (i / PT) % PT, l2 = i % PT;
        const int q0 = ((o0 + l0) % L + L) % L, q1 = ((o1 + l1) % L + L) % L, q2 = ((o2 + l2) % L + L) % L;
        tile[i] = grid_value(a.X, L, N, a.QP, q0, q1, q2);
    }
    // The tile's constants, the same in every lane, kept in LDS and read where they are used
    // (vector registers holding them across the loops below would spill): its centre relative to
    // the grid's centre in FP32 (the plane test's margin of 2e-3 and the candidate rows' slack
    // of one row are far above its rounding), the row radius rk, and the slab bounds: positions
    // tau whose (clamped) cell lies in the tile, widened by a margin far above the rounding of the
    // FP32 row intervals; the edge tiles also own the clamped cells beyond the grid.  Each
    // interval is then trimmed to the exact one with the FP64 cell test.
    __shared__ float tcl[3], blo[3], bhi[3], rkl;
    if (tid == 0) {
        qn = 0;
        nimg = 0;
        constexpr float MARGIN = 1e-2f, FAR = 1e30f;
        for (int d = 0; d < 3; ++d) {
            tcl[d] = tt[d] * T + 0.5f * T - 0.5f * L;
            blo[d] = tt[d] == 0 ? -FAR : tt[d] * T - MARGIN;
            bhi[d] = (tt[d] + 1) * T >= L ? FAR : (tt[d] + 1) * T + MARGIN;
        }
        rkl = (T * 0.8660254f + 1e-3f) / (float)a.s;
    }
    const int S = (int)floorf(2.f * ((T * 0.8660254f + 1e-3f) / (float)a.s)) + 3;  // candidate rows per view
    const int N2 = N * N;
    // the point (k1, k2) of the view with columns c lies in the tile: inside the disk and its
    // clamped cell in the tile per axis
    auto in_tile = [&](const double* c, int k1, int k2) {
        if (4 * (k1 * k1 + k2 * k2) > N2) return false;
        bool in = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int cell = (int)floor(tau_of(a.s, k1, k2, c[d], c[3 + d], halfL));
            cell = cell < 0 ? 0 : (cell > L - 1 ? L - 1 : cell);
            in = in && (cell / T == tt[d]);
        }
        return in;
    };

    auto flush = [&](int n) {
        for (int qi = tid; qi < n; qi += NTH) {
            const int e = queue[qi];
            if (e >= 0) gather_point<T, W>(a, tile, tt, img_m[e >> 17], (e >> 9) & 255, (e & 511) - 256);
        }
    };

    // blocks of NTH views (the work range starts on a block), up to NTH of them at a time: their
    // boxes of normals are tested first, into a bit mask, and the rounds below visit the live
    // blocks only, PJ_VPT at a time (a block whose box of normals n gives no |n . c| within the
    // bound below for the tile's centre c holds no view that meets the tile)
    __shared__ unsigned bmask[NTH / 32];
    __shared__ int lblk[PJ_VPT + 2];  // a round's live blocks (in the group), their count, the cursor
    const int blk0 = wk.y / NTH, blk1 = (wk.z + NTH - 1) / NTH;
    for (int gb = blk0; gb < blk1; gb += NTH) {
        if (tid < NTH / 32) bmask[tid] = 0u;
        __syncthreads();
        if (gb + tid < blk1) {
            const float4 lo = a.vbox[2 * (gb + tid)], hi = a.vbox[2 * (gb + tid) + 1];
            const float p0 = tcl[0] * lo.x, q0 = tcl[0] * hi.x, p1 = tcl[1] * lo.y, q1 = tcl[1] * hi.y;
            const float p2 = tcl[2] * lo.z, q2 = tcl[2] * hi.z;
            const float dmin = fminf(p0, q0) + fminf(p1, q1) + fminf(p2, q2);
            const float dmax = fmaxf(p0, q0) + fmaxf(p1, q1) + fmaxf(p2, q2);
            const float lim = 0.5f * T * lo.w + 3e-3f;
            if (dmin <= lim && dmax >= -lim) atomicOr(&bmask[tid >> 5], 1u << (tid & 31));
        }
        if (tid == 0) lblk[PJ_VPT + 1] = 0;
        bool more = true;  // uniform
        while (more) {
            __syncthreads();  // the counters are reset, the tile and the block mask are in place
            // 1. views whose plane meets the tile, at least NTH of them (or all that remain),
            //    PJ_VPT live blocks per round, one view per thread and block, so that the loads
            //    of a round overlap
            int ni = 0;
            while (true) {
                if (tid == 0) {
                    int n = 0, cur = lblk[PJ_VPT + 1];
                    while (n < PJ_VPT && cur < NTH) {
                        const unsigned w = bmask[cur >> 5] & (~0u << (cur & 31));
                        if (w == 0u) {
                            cur = (cur | 31) + 1;
                            continue;
                        }
                        const int b = (cur & ~31) + __builtin_ctz(w);
                        lblk[n++] = b;
                        cur = b + 1;
                    }
                    lblk[PJ_VPT] = n;
                    lblk[PJ_VPT + 1] = cur;
                }
                __syncthreads();
                const int nl = lblk[PJ_VPT];
                if (nl == 0) {
                    more = false;
                    ni = nimg;
                    break;
                }
                float4 nv[PJ_VPT];
                unsigned livev = 0u;
#pragma unroll
                for (int v = 0; v < PJ_VPT; ++v) {
                    const int m = v < nl ? (gb + lblk[v]) * NTH + tid : wk.z;
                    const bool live = m < wk.z;
                    nv[v] = live ? *reinterpret_cast<const float4*>(a.nrm + 4 * (int64_t)m) : make_float4(0.f, 0.f, 0.f, 0.f);
                    livev |= (unsigned)live << v;
                }
#pragma unroll
                for (int v = 0; v < PJ_VPT; ++v) {
                    const int m = v < nl ? (gb + lblk[v]) * NTH + tid : wk.z;
                    // the plane meets the tile's cube: distance of the centre at most the cube's
                    // half extent along the normal
                    const float dist = fabsf(tcl[0] * nv[v].x + tcl[1] * nv[v].y + tcl[2] * nv[v].z);
                    if (((livev >> v) & 1u) && dist <= 0.5f * T * (fabsf(nv[v].x) + fabsf(nv[v].y) + fabsf(nv[v].z)) + 2e-3f) {
                        const double* c = a.c12 + 6 * (int64_t)m;
                        const float u1 = (tcl[0] * (float)c[0] + tcl[1] * (float)c[1] + tcl[2] * (float)c[2]) / (float)a.s;
                        const int sl = atomicAdd(&nimg, 1);
                        img_m[sl] = m;
                        img_r[sl] = (int)ceilf(u1 - rkl) - 1;
                    }
                }
                __syncthreads();
                ni = nimg;
                __syncthreads();  // read by every thread before the next round adds to it
                if (ni >= NTH) break;
            }
            // 2. one (view, row k1) per thread: the k2 interval whose cells lie in the tile (three
            //    slabs, plus the disk and half-disk bounds), trimmed to the exact cell test at both
            //    ends (the cell along a row is monotone in k2, so the points that pass form an
            //    interval).  Queue space is reserved per thread; a reservation that does not fit
            //    is retried after the full queue has been gathered.
            const int units = ni * S;
            for (int base = 0; base < units; base += NTH) {
                const int u = base + tid;
                int sl = 0, k1 = 0, klo = 0, cnt = 0;
                if (u < units) {
                    sl = u / S;
                    k1 = img_r[sl] + (u - sl * S);
                    if (k1 >= 0 && 4 * k1 * k1 <= N2) {
                        const double* c = a.c12 + 6 * (int64_t)img_m[sl];
                        const int kd = (int)sqrtf((float)(N2 / 4 - k1 * k1)) + 1;  // >= the disk's |k2|
                        float lo = (float)-kd, hi = (float)kd;
                        bool ok = true;
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const float al = (float)(a.s * k1 * c[d] + halfL), be = (float)(a.s * c[3 + d]);
                            if (fabsf(be) < 1e-6f) {
                                ok = ok && al >= blo[d] && al <= bhi[d];
                            } else {
                                // reciprocal to about 1 ulp: far inside the bounds' margin
                                const float rb = __builtin_amdgcn_rcpf(be);
                                const float t1 = (blo[d] - al) * rb, t2 = (bhi[d] - al) * rb;
                                lo = fmaxf(lo, fminf(t1, t2));
                                hi = fminf(hi, fmaxf(t1, t2));
                            }
                        }
                        klo = (int)ceilf(lo);
                        if (k1 == 0) klo = max(klo, 1);
                        int khi = (int)floorf(hi);
                        if (ok) {
                            while (klo <= khi && !in_tile(c, k1, klo)) ++klo;
                            while (khi >= klo && !in_tile(c, k1, khi)) --khi;
                            // a row crosses a tile in at most T sqrt(3) / s + 1 points
                            cnt = min(khi - klo + 1, 32);
                        }
                    }
                }
                bool pend = cnt > 0;
                while (true) {
                    if (pend) {
                        const int pos = atomicAdd(&qn, cnt);
                        if (pos + cnt <= PJ_QCAP) {
                            for (int j = 0; j < cnt; ++j) queue[pos + j] = (sl << 17) | (k1 << 9) | (klo + j + 256);
                            pend = false;
                        } else {
                            for (int j = pos; j < PJ_QCAP; ++j) queue[j] = -1;
                        }
                    }
                    if (!__syncthreads_or(pend)) break;
                    flush(PJ_QCAP);  // the queue is full
                    __syncthreads();
                    if (tid == 0) qn = 0;
                    __syncthreads();
                }
            }
            // 3. the view slots are refilled next round: gather what is queued
            const int nq = qn;  // every reservation of the last chunk fitted (read after its barrier)
            flush(nq);
            __syncthreads();
            if (tid == 0) { qn = 0; nimg = 0; }
        }
    }
}

}  // namespace

// b (M x P complex64, disk order) = forward projection of V (N^3, centred order).
// Workspaces: p->tmp (u), p->T1, p->ws1, p->grid (the caller has sized the gridding workspaces).
hipError_t forward_project(firm_plan p, const float* V, float2* b) {
    const int N = p->N, L = 2 * N;
    if (spread_tile_cplx() != PJ_TILE) return hipErrorInvalidValue;
    hipStream_t st = p->stream;
    const int nblk = std::min<int>(PJ_PREP_BLOCKS, p->npart);
    hipLaunchKernelGGL(k_fp_prep, dim3(nblk), dim3(256), 0, st, V, p->deconv_atb, N, p->tmp, p->partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fp_k0, dim3((p->M + 255) / 256), dim3(256), 0, st, p->partials, nblk, p->group, p->table,
                       p->Q, p->M, p->P, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    float2* X = reinterpret_cast<float2*>(p->grid);
    if ((e = fft_project_grid(p, p->tmp, p->T1, reinterpret_cast<float2*>(p->ws1), X)) != hipSuccess) return e;
    if (p->ntiles_atb == 0) return hipSuccess;
    ProjArgs a;
    a.N = N; a.M = p->M; a.L = L; a.nt = (L + PJ_TILE - 1) / PJ_TILE; a.P = p->P; a.Q = p->Q; a.QP = p->QP;
    a.s = 2.0;
    // the views in the order of their normals (blocks of SP_VBLK views, one per round and thread)
    static_assert(PJ_THREADS == SP_VBLK, "a block of views per round and thread");
    a.c12 = p->c12s; a.nrm = p->nrms; a.group = p->groups; a.table = p->table; a.poly = p->kb_poly;
    a.vorder = p->vorder; a.vbox = p->vbox;
    a.work = reinterpret_cast<const int4*>(p->tiles_atb);
    a.X = X; a.shifts = p->shiftss; a.rowstart = p->rowstart; a.b = b;
    const dim3 grid(p->ntiles_atb), blk(PJ_THREADS);
    switch (p->kbw) {
        case 4: hipLaunchKernelGGL((k_project<PJ_TILE, 4, PJ_THREADS>), grid, blk, 0, st, a); break;
        case 5: hipLaunchKernelGGL((k_project<PJ_TILE, 5, PJ_THREADS>), grid, blk, 0, st, a); break;
        case 6: hipLaunchKernelGGL((k_project<PJ_TILE, 6, PJ_THREADS>), grid, blk, 0, st, a); break;
        case 7: hipLaunchKernelGGL((k_project<PJ_TILE, 7, PJ_THREADS>), grid, blk, 0, st, a); break;
        case 8: hipLaunchKernelGGL((k_project<PJ_TILE, 8, PJ_THREADS>), grid, blk, 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
