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
// range against the tile's cube, enumerates the disk points of the surviving
// images whose cell floor(t + L/2) lies in the tile (an exact k2 interval per
// row), and accumulates their full W^3 stencils into a (T + W)^3 LDS tile; the
// tile is then added to the global grid with one atomic per cell.  Each point is
// spread exactly once.
//
// LDS float atomics run at a small fraction of the plain read/write rate on this
// chip, 64-bit integer atomics at about the plain rate.  The tile is therefore
// accumulated in fixed point: 64-bit integer cells, each term the FP32 product
// rounded to an integer in units of 1/fxs (a power of 2 with |term| < 2^31),
// added with one integer atomic per cell.  Integer sums are exact and independent
// of the order of the adds, so every wavefront takes any staged point.  The
// per-point window weights are computed once, one thread per point and axis, and
// staged in LDS; the lanes of a wavefront sit on the W x W footprint of the last
// two axes and add the point's W rows.  Ker's terms are non-negative; A*b is
// spread one component (re, then im) per launch, with signed terms and a unit
// that follows from the largest |component| of the data.  Only the half disk (k1 > 0, or k1 = 0 and
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
    float fxs;      // fixed-point accumulation: integer units per unit of grid value (a power of 2)
    double fx_inv;  // 1 / fxs
    // when set, fxs is the largest power of 2 not above fx_coef / bmax, bmax the float whose bits
    // are at fx_bmax (the largest |component| of the data), found on the device before the launch
    const unsigned* fx_bmax;
    float fx_coef;
    int comp;  // complex data spread one component at a time: the component (0 re, 1 im)
    // the per-view arrays above are in the gridding's view order; vorder maps a position to the
    // caller's view index (for b), vbox holds per block of SP_VBLK views the box of the normals
    const int* vorder;
    const float4* vbox;
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

// LDS bank layout of the footprint accesses.  LDS has 32 banks of 4 bytes and serves a wave's
// access in groups of lanes: two groups of 32 for 4-byte elements, four groups of 16 for
// 8-byte elements (G groups of 64 / G lanes, whose elements must fall in 64 / G distinct
// element slots modulo 128 bytes).  The W x W footprint cells j2 * pitch + j3 (in elements) are
// split by rows among the G groups so that each group's cells are conflict-free.
// place_rows: assign rows r.. to groups (grp[]), by backtracking.
constexpr bool place_rows(int r, int W, int rp, int G, int* grp) {
    if (r == W) return true;
    const int cap = 64 / G;
    for (int g = 0; g < G; ++g) {
        int n = 0;
        for (int q = 0; q < r; ++q) n += grp[q] == g;
        if ((n + 1) * W > cap) continue;
        bool ok = true;
        for (int q = 0; q < r && ok; ++q) {
            if (grp[q] != g) continue;
            for (int i = 0; i < W && ok; ++i)
                for (int j = 0; j < W && ok; ++j)
                    if ((q * rp + i) % cap == (r * rp + j) % cap) ok = false;
        }
        if (!ok) continue;
        grp[r] = g;
        if (place_rows(r + 1, W, rp, G, grp)) return true;
    }
    return false;
}

// group of every footprint row (two bits per row) for row pitch rp, or -1 if none is
// conflict-free
constexpr int row_groups(int rp, int W, int G) {
    int grp[8] = {};
    if (!place_rows(0, W, rp, G, grp)) return -1;
    int code = 0;
    for (int r = 0; r < W; ++r) code |= grp[r] << (2 * r);
    return code;
}

// smallest LDS row pitch >= PT that admits a conflict-free split
constexpr int row_pitch(int PT, int W, int G) {
    for (int rp = PT; rp < PT + 32; ++rp)
        if (row_groups(rp, W, G) >= 0) return rp;
    return PT;
}

// Fine-grid position of the disk point (k1, k2) of a view along axis d: the one expression
// that both the point enumeration (which tile owns the point) and the staging (where its
// window starts) evaluate, so that the two agree to the last bit.
__device__ __forceinline__ double tau_of(double s, int k1, int k2, double cd, double c3d, double halfL) {
    return fma(s, fma((double)k2, c3d, (double)k1 * cd), halfL);
}

// Points staged per batch: the most, in whole rounds (a round gives every wavefront FQ points),
// that keep one staging item (point, axis) per thread and the workgroup's LDS within its budget.
constexpr int sp_batch(int nth, int fixed_bytes, int per_point, int budget, int round) {
    int pb = nth / 3 / round * round;
    while (pb > round && fixed_bytes + pb * per_point > budget) pb -= round;
    return pb;
}

// One tile plane of 64-bit integer cells.  Complex data (A*b) is spread one component per
// launch (a.comp), so that its tile is as small as the kernel's: two workgroups per CU up to
// W = 7, one for W = 8.
template <int T, int W, bool CPLX, int NTH>
__global__ void __launch_bounds__(NTH, (W >= 8 ? NTH / 256 : NTH / 128)) k_spread(SpreadArgs a) {
    constexpr int SP_THREADS = NTH, SP_WAVES = NTH / 64;
    constexpr int PT = T + W;
    constexpr int PADLO = (W + 1) / 2 - 1;
    constexpr int NCELL = PT * PT * PT;
    constexpr int G = 4;                               // lane groups of an 8-byte LDS access
    constexpr int RP = row_pitch(PT, W, G);            // LDS pitch of a tile row, in cells (conflict-free)
    constexpr int GROUPS = row_groups(RP, W, G);       // lane group of every footprint row
    constexpr int PP = PT * RP;                        // LDS pitch of a tile plane
    // staged point: the W window weights of axes 0, 1, 2 at 0, W, 2W (axis 0 times the point's
    // value in fixed-point units); stride in floats
    constexpr int PSTR = 3 * W;
    static_assert(W >= 3 && W <= 8, "window width");
    constexpr int FQ = 4;  // points a wavefront accumulates at a time (see the accumulation)
    // LDS besides the staged points: the tile, the view slots (and for complex data their views,
    // groups and the disk's row starts), the queue, and 512 bytes for the counters, the tile
    // constants, the lane map, the flush's partial sums and alignment.  The batch is as large as
    // the rest allows: two workgroups share a CU up to W = 7 (80 KB each), one at W = 8.
    // the queue: the A*b tile leaves room for 256 more entries (fewer stops of the enumeration);
    // the kernel's tile 32 fewer, for the block mask of the culling
    constexpr int QCAP = CPLX ? SP_QCAP + 256 : SP_QCAP - 32;
    constexpr int LDS_FIXED = PT * PP * 8 + NTH * 4 * (CPLX ? 3 : 1) + (CPLX ? 264 * 4 : 0) + QCAP * 4 + 512;
    constexpr int SP_PB = sp_batch(NTH, LDS_FIXED, PSTR * 4 + 4, W >= 8 ? 160 * 1024 : 80 * 1024, FQ * SP_WAVES);
    static_assert(SP_PB >= FQ * SP_WAVES && 3 * SP_PB <= NTH, "staging batch");
    constexpr int NIT = (3 * SP_PB + NTH - 1) / NTH;   // staging items (point, axis) per thread
    __shared__ __align__(16) unsigned long long tile64[PT * PP];
    __shared__ __align__(16) float pt_w[SP_PB * PSTR];
    __shared__ int pt_lo[SP_PB];                       // window starts of axes 0, 1, 2 in bytes 0, 1, 2
    __shared__ int img_m[SP_THREADS];
    __shared__ int img_o[CPLX ? SP_THREADS : 1];  // complex data: the slot's view in the caller's order
    __shared__ int img_g[CPLX ? SP_THREADS : 1];  // complex data: the slot's CTF group
    __shared__ int rs_l[CPLX ? 264 : 1];              // row starts of the disk order (N <= 256)
    __shared__ int queue[QCAP];
    __shared__ int nimg, qn, qfail, any;
    __shared__ float geo[12];  // the tile's constants (see below)
    __shared__ unsigned short lmap[64];  // footprint cell of each lane (see below)

    const int tid = threadIdx.x;
    const int4 wk = a.work[blockIdx.x];
    float fxs = a.fxs;
    double fx_inv = a.fx_inv;
    if (a.fx_bmax) {
        const float bm = __uint_as_float(*a.fx_bmax);
        int e = 0;
        if (bm > 0.f) e = (int)fmin(fmax(floor(log2((double)a.fx_coef / (double)bm)), -100.0), 100.0);
        fxs = ldexpf(1.f, e);
        fx_inv = ldexp(1.0, -e);
    }
    const int nt = a.nt;
    const int tt0 = wk.x / (nt * nt), tt1 = (wk.x / nt) % nt, tt2 = wk.x % nt;
    const int L = a.L, N = a.N;
    const double halfL = 0.5 * L;

    for (int i = tid; i < PT * PP; i += SP_THREADS) tile64[i] = 0ull;
    if (tid == 0) { any = 0; nimg = 0; qn = 0; qfail = QCAP; }
    if constexpr (CPLX)
        for (int i = tid; i <= a.N; i += SP_THREADS) rs_l[i] = a.rowstart[i];

    // the tile's centre (relative to the grid's centre) in FP32: the plane tests carry margins of
    // 2e-3 and more against its rounding (< 3e-5 at |c| <= 512), and the candidate rows one row.
    // These tile constants are the same in every lane; they are kept in LDS (geo) and read where
    // they are used, since vector registers holding them across the loops below would spill.
    enum { G_TC0, G_TC1, G_TC2, G_BLO0, G_BLO1, G_BLO2, G_BHI0, G_BHI1, G_BHI2, G_RK, G_INVS, G_N };
    // candidate rows of a view: the k1 within rk of the projection u1 of the tile's centre onto the
    // plane (rk: the circumscribed sphere's radius in lattice units), widened by 1e-3 for the
    // rounding of u1: S = floor(2 rk + 2e-3) + 2 rows from ceil(u1 - rk - 1e-3)
    const int S = (int)floorf(2.f * ((T * 0.8660254f + 1e-3f) / (float)a.s) + 2e-3f) + 2;
    if (tid == 0) {
        // positions tau whose (clamped) cell lies in the tile, widened by a margin far above the
        // rounding of the FP32 row intervals; the edge tiles also own the clamped cells beyond the
        // grid.  Each interval is then trimmed to the exact one with the FP64 cell test.
        constexpr float MARGIN = 1e-2f, FAR = 1e30f;
        const int tt[3] = {tt0, tt1, tt2};
        for (int d = 0; d < 3; ++d) {
            geo[G_TC0 + d] = tt[d] * T + 0.5f * T - 0.5f * L;
            geo[G_BLO0 + d] = tt[d] == 0 ? -FAR : tt[d] * T - MARGIN;
            geo[G_BHI0 + d] = (tt[d] + 1) * T >= L ? FAR : (tt[d] + 1) * T + MARGIN;
        }
        geo[G_RK] = (T * 0.8660254f + 1e-3f) / (float)a.s;
        geo[G_INVS] = 1.f / (float)a.s;
    }
    if (tid < 64) {
        // footprint cell (j2, j3) of each lane: lane group g holds the rows assigned to it, W lanes
        // per row; kept in LDS and read where the adds need it (registers holding it across the
        // staging would spill)
        const int lane = tid;
        int j2 = 0, j3 = 0;
        bool act = false;
        if constexpr (GROUPS >= 0) {
            const int g = lane / (64 / G), idx = lane % (64 / G), rank = idx / W;
            int seen = 0;
#pragma unroll
            for (int r = 0; r < W; ++r) {
                if (((GROUPS >> (2 * r)) & 3) != g) continue;
                if (seen == rank) {
                    j2 = r;
                    j3 = idx - rank * W;
                    act = true;
                }
                ++seen;
            }
        } else {
            act = lane < W * W;
            const int jl = act ? lane : 0;
            j2 = jl / W;
            j3 = jl - j2 * W;
        }
        lmap[lane] = (unsigned short)(j2 | (j3 << 4) | ((int)act << 8));
    }
    __syncthreads();  // the counters, the tile constants, the lane map and the row starts are in place
    const int N2 = N * N;

    // points of the queue [0, nq) staged and accumulated in batches of SP_PB
    auto process = [&](int nq) {
        if (tid == 0 && nq > 0) any = 1;
        // tile coordinates as values: a select between the captured references would be a
        // select between addresses, which puts them in scratch memory
        const int tv0 = tt0, tv1 = tt1, tv2 = tt2;
        const int wv = tid >> 6, lane = tid & 63;
        for (int pb = 0; pb < nq; pb += SP_PB) {
            const int nb = min(SP_PB, nq - pb);
            // stage the batch: one item per (point, axis), spread over all threads, computes the
            // window start and weights along that axis; the axis-0 item also computes the point's
            // value and folds it, in fixed-point units, into its weights.  The point keeps its
            // batch position.
            float ph[NIT][W];
            int lod[NIT], pp[NIT], dd[NIT];
            float scale = 1.f;
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int i = tid + it * SP_THREADS;
                dd[it] = -1;
                pp[it] = 0;
                lod[it] = 0;
                if (i < 3 * nb) {
                    const int d = i / nb, p = i - d * nb;
                    dd[it] = d;
                    pp[it] = p;
                    const int e = queue[pb + p];
                    const int sl = e >> 18, k1 = ((e >> 9) & 511) - 256, k2 = (e & 511) - 256;
                    const int m = img_m[sl];
                    const double* c = a.c12 + 6 * (int64_t)m;
                    const int ttd = d == 0 ? tv0 : (d == 1 ? tv1 : tv2);
                    // |t_d| <= L/2 in exact arithmetic; clamp the rounding excess so the
                    // stencil stays inside the padded tile for every width
                    const double tau = fmin(fmax(tau_of(a.s, k1, k2, c[d], c[3 + d], halfL), 0.0), (double)L);
                    const double left = tau - 0.5 * W;
                    const int b0 = (int)floor(left) + 1;
                    const float f = (float)((double)b0 - left);  // in (0, 1]
                    kb_weights<W>(a.poly, 2.f * f - 1.f, ph[it]);
                    // in [0, PT - W] for every point of the tile (clamped position); the bound
                    // also keeps the LDS accesses inside the tile should rounding ever differ
                    lod[it] = min(max(b0 - (ttd * T - PADLO), 0), PT - W);
                    if (d == 0) {
                        const int g = CPLX ? img_g[sl] : a.group[m];
                        const float h = a.table ? a.table[(int64_t)g * a.Q + k1 * k1 + k2 * k2] : 1.f;
                        if constexpr (!CPLX) {
                            scale = 2.f * h * h * fxs;
                        } else {
                            // h exp(i theta) (b(k) + conj b(-k)), theta = 2 pi <k, s_m> / N (re-centring)
                            const int idx = rs_l[k1 + N / 2] + k2;
                            const int64_t mo = img_o[sl];  // the caller's view index
                            const float2 bp = a.b[mo * a.P + idx];
                            const float2 bm = a.b[mo * a.P + (a.P - 1 - idx)];
                            const float sr = bp.x + bm.x, si = bp.y - bm.y;
                            float cs = 1.f, sn = 0.f;
                            if (a.shifts) {
                                // theta / 2 pi reduced to [-1/2, 1/2] in FP64, then the FP32 sine and
                                // cosine of pi times twice that
                                const double f = (k1 * a.shifts[2 * (int64_t)m] + k2 * a.shifts[2 * (int64_t)m + 1]) / N;
                                sincospif((float)(2.0 * (f - rint(f))), &sn, &cs);
                            }
                            scale = fxs * h * (a.comp ? cs * si + sn * sr : cs * sr - sn * si);
                        }
                    }
                }
            }
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int d = dd[it];
                if (d < 0) continue;
                // weights of axis d at W d, window starts in the bytes of pt_lo
                float* q = pt_w + pp[it] * PSTR + W * d;
#pragma unroll
                for (int j = 0; j < W; ++j) q[j] = d == 0 ? scale * ph[it][j] : ph[it][j];
                reinterpret_cast<unsigned char*>(pt_lo)[4 * pp[it] + d] = (unsigned char)lod[it];
            }
            __syncthreads();
            // The wavefronts take the batch's points in turn, the lanes on the W x W footprint of
            // axes 1 and 2, one 64-bit integer atomic add per cell and window row.  Integer
            // addition is associative, so the tile is exact and independent of the order of the
            // adds; each term is the FP32 product rounded to an integer (|term| < 2^31 by the
            // choice of fxs).  A wavefront takes FQ of its points at a time: their window words and
            // axis-0 weights (the same for every lane) arrive in one LDS read spread over the
            // lanes and are then broadcast from registers (readlane); each footprint lane reads
            // its own axis-1 and axis-2 weights.  All reads of the FQ points come before their
            // adds, so the wavefront waits once per FQ points (LDS completes in order, so a read
            // issued after adds waits for them).  The lanes off the footprint take part in the
            // reads only.
            const int lm = lmap[lane];
            const int j2 = lm & 15, j3 = (lm >> 4) & 15;
            const bool act = (lm >> 8) != 0;
            static_assert(FQ == 4, "the register list of the asm statement below names 4");
            static_assert(FQ * 8 + FQ <= 64, "one read for the uniform data");
            const int wvu = __builtin_amdgcn_readfirstlane(wv);
            // lane roles of the uniform read: 8 q + k -> weight k of point q (k < 8); 32 + q -> window
            // word of point q; the other lanes repeat point q's window word
            const int uq = lane < 32 ? (lane >> 3) : (lane - 32) % FQ;
            // the adds at a raised wavefront priority: where the two workgroups of a CU are in
            // different phases, the issue of the LDS-bound adds goes first and the staging or
            // enumeration of the other, bound by load latency, fills the gaps
            __builtin_amdgcn_s_setprio(2);
            for (int p0 = wvu; p0 < nb; p0 += FQ * SP_WAVES) {
                int pq[FQ];
#pragma unroll
                for (int q = 0; q < FQ; ++q) pq[q] = min(p0 + q * SP_WAVES, nb - 1);
                int pl = pq[0];
#pragma unroll
                for (int q = 1; q < FQ; ++q) pl = uq == q ? pq[q] : pl;
                const float* src = lane < 32 ? pt_w + pl * PSTR + (lane & 7) : reinterpret_cast<const float*>(pt_lo + pl);
                float w2[FQ], w3[FQ];
#pragma unroll
                for (int q = 0; q < FQ; ++q) {
                    w2[q] = pt_w[pq[q] * PSTR + W + j2];
                    w3[q] = pt_w[pq[q] * PSTR + 2 * W + j3];
                }
                float u = *src;
                // all the reads are issued here, before any register of theirs is used
                asm volatile("" : "+v"(u), "+v"(w2[0]), "+v"(w3[0]), "+v"(w2[1]), "+v"(w3[1]),
                             "+v"(w2[2]), "+v"(w3[2]), "+v"(w2[3]), "+v"(w3[3]));
                if (!act) continue;
#pragma unroll
                for (int q = 0; q < FQ; ++q) {
                    if (p0 + q * SP_WAVES >= nb) break;
                    const float w23 = w2[q] * w3[q];
                    const int lw = __builtin_amdgcn_readlane(__float_as_int(u), 32 + q);
                    const int cb = (lw & 255) * PP + (((lw >> 8) & 255) + j2) * RP + ((lw >> 16) & 255) + j3;
#pragma unroll
                    for (int r = 0; r < W; ++r) {
                        const float wxr = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(u), 8 * q + r));
                        // Ker: non-negative terms; a component of complex data: signed terms
                        const unsigned long long t = CPLX ? (unsigned long long)(long long)(int)rintf(wxr * w23)
                                                          : (unsigned long long)(unsigned)fmaf(wxr, w23, 0.5f);
                        __hip_atomic_fetch_add(&tile64[cb + r * PP], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
            }
            __builtin_amdgcn_s_setprio(0);
            __syncthreads();
        }
    };


    // the point (k1, k2) of the view with columns c lies in the tile (the test that decides
    // which tile spreads a point): inside the disk and its clamped cell in the tile per axis
    auto in_tile = [&](const double* c, int k1, int k2) {
        if (4 * (k1 * k1 + k2 * k2) > N2) return false;
        bool in = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int cell = (int)floor(tau_of(a.s, k1, k2, c[d], c[3 + d], halfL));
            cell = cell < 0 ? 0 : (cell > L - 1 ? L - 1 : cell);
            in = in && (cell / T == (d == 0 ? tt0 : (d == 1 ? tt1 : tt2)));
        }
        return in;
    };

    // the view slots and the queue persist across the image chunks, so that batches are full:
    // queued points name their view by slot, and the slots are reused only after the queue has
    // been processed.  A chunk is VPT views per thread (the fixed cost of a chunk, barriers and
    // the latency of the view data, is paid once for all of them).
    constexpr int VPT = 8;
    __shared__ unsigned bmask[SP_THREADS / 32];  // the live blocks of the current group of blocks
    // a chunk's live blocks (in the group), their count, and the next block of the group to look at
    __shared__ int lblk[VPT + 2];
    int base = 0;  // first slot whose rows are not yet enumerated
    // blocks of SP_THREADS views (the work range starts on a block)
    const int blk0 = wk.y / SP_THREADS, blk1 = (wk.z + SP_THREADS - 1) / SP_THREADS;
    for (int gb = blk0; gb < blk1; gb += SP_THREADS) {
        // block tests, one block per thread, up to SP_THREADS blocks at a time: a block whose box
        // of normals n gives no |n . c| within the bound below for the tile's centre c holds no
        // view that meets the tile.  The chunks below visit the live blocks only.
        if (tid < SP_THREADS / 32) bmask[tid] = 0u;
        __syncthreads();
        if (gb + tid < blk1) {
            const float tc0 = geo[G_TC0], tc1 = geo[G_TC1], tc2 = geo[G_TC2];
            const float4 lo = a.vbox[2 * (gb + tid)], hi = a.vbox[2 * (gb + tid) + 1];
            const float p0 = tc0 * lo.x, q0 = tc0 * hi.x, p1 = tc1 * lo.y, q1 = tc1 * hi.y;
            const float p2 = tc2 * lo.z, q2 = tc2 * hi.z;
            const float dmin = fminf(p0, q0) + fminf(p1, q1) + fminf(p2, q2);
            const float dmax = fmaxf(p0, q0) + fmaxf(p1, q1) + fmaxf(p2, q2);
            const float lim = 0.5f * T * lo.w + 3e-3f;
            if (dmin <= lim && dmax >= -lim) atomicOr(&bmask[tid >> 5], 1u << (tid & 31));
        }
        if (tid == 0) lblk[VPT + 1] = 0;
        while (true) {
            __syncthreads();  // the mask is complete, and the last chunk's blocks are no longer read
            if (tid == 0) {
                int n = 0, cur = lblk[VPT + 1];
                while (n < VPT && cur < SP_THREADS) {
                    const unsigned w = bmask[cur >> 5] & (~0u << (cur & 31));
                    if (w == 0u) {
                        cur = (cur | 31) + 1;
                        continue;
                    }
                    const int b = (cur & ~31) + __builtin_ctz(w);
                    lblk[n++] = b;
                    cur = b + 1;
                }
                lblk[VPT] = n;
                lblk[VPT + 1] = cur;
            }
            __syncthreads();
            const int nl = lblk[VPT];
            if (nl == 0) break;
            // a chunk: the views of up to VPT live blocks, one per thread and block
            unsigned pendv = 0u;  // this thread's views of the chunk that meet the tile, not yet in a slot
            {
                float4 nv[VPT];
                unsigned livev = 0u;
#pragma unroll
                for (int v = 0; v < VPT; ++v) {
                    const int m = v < nl ? (gb + lblk[v]) * SP_THREADS + tid : wk.z;
                    const bool live = m < wk.z;
                    nv[v] = live ? *reinterpret_cast<const float4*>(a.nrm + 4 * (int64_t)m) : make_float4(0.f, 0.f, 0.f, 0.f);
                    livev |= (unsigned)live << v;
                }
    #pragma unroll
                for (int v = 0; v < VPT; ++v) {
                    // the plane meets the tile's cube: distance of the centre at most the cube's half
                    // extent along the normal
                    if (((livev >> v) & 1u) && fabsf(geo[G_TC0] * nv[v].x + geo[G_TC1] * nv[v].y + geo[G_TC2] * nv[v].z) <=
                                                    0.5f * T * (fabsf(nv[v].x) + fabsf(nv[v].y) + fabsf(nv[v].z)) + 2e-3f)
                        pendv |= 1u << v;
                }
            }
            while (true) {
                // slots for the surviving views while free ones last
                for (int v = 0; v < VPT; ++v) {
                    if (!((pendv >> v) & 1u)) continue;
                    const int sl = atomicAdd(&nimg, 1);
                    if (sl < SP_THREADS) {
                        img_m[sl] = (gb + lblk[v]) * SP_THREADS + tid;
                        pendv &= ~(1u << v);
                    }
                }
                __syncthreads();
                const int top = min(nimg, SP_THREADS);
                if constexpr (CPLX) {
                    // the new slots' CTF groups and views in the caller's order, read once per slot
                    // here (in parallel) rather than by the staging of every point
                    if (tid >= base && tid < top) {
                        const int m = img_m[tid];
                        img_o[tid] = a.vorder[m];
                        img_g[tid] = a.group[m];
                    }
                    __syncthreads();
                }
                // one (view, row k1) per thread: the k2 interval whose cells lie in the tile (three slabs,
                // plus the disk and half-disk bounds), trimmed to the exact test at both ends (the cell
                // along a row is monotone in k2, so the points that pass form an interval), then the
                // points are queued.  A reservation that does not fit waits for the queue's whole
                // batches to be processed; the reservations that fitted form the prefix up to the
                // first that did not.
                const int units = (top - base) * S;
                for (int ub = 0; ub < units; ub += SP_THREADS) {
                    const int u = ub + tid;
                    int sl = 0, k1 = 0, klo = 0, cnt = 0;
                    if (u < units) {
                        const int v = u / S;
                        sl = base + v;
                        const double* c = a.c12 + 6 * (int64_t)img_m[sl];
                        const float u1 = (geo[G_TC0] * (float)c[0] + geo[G_TC1] * (float)c[1] + geo[G_TC2] * (float)c[2]) *
                                         geo[G_INVS];
                        k1 = (int)ceilf(u1 - geo[G_RK] - 1e-3f) + (u - v * S);
                        if (k1 >= 0 && 4 * k1 * k1 <= N2) {
                            const int kd = (int)sqrtf((float)(N2 / 4 - k1 * k1)) + 1;  // >= the disk's |k2|
                            float lo = (float)-kd, hi = (float)kd;
                            bool ok = true;
    #pragma unroll
                            for (int d = 0; d < 3; ++d) {
                                const float bl = geo[G_BLO0 + d], bh = geo[G_BHI0 + d];
                                const float al = (float)(a.s * k1 * c[d] + halfL), be = (float)(a.s * c[3 + d]);
                                if (fabsf(be) < 1e-6f) {
                                    ok = ok && al >= bl && al <= bh;
                                } else {
                                    // reciprocal to about 1 ulp: far inside the bounds' margin
                                    const float rb = __builtin_amdgcn_rcpf(be);
                                    const float t1 = (bl - al) * rb, t2 = (bh - al) * rb;
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
                            if (pos + cnt <= QCAP) {
                                for (int j = 0; j < cnt; ++j) queue[pos + j] = (sl << 18) | ((k1 + 256) << 9) | (klo + j + 256);
                                pend = false;
                            } else {
                                atomicMin(&qfail, pos);
                            }
                        }
                        if (!__syncthreads_or(pend)) break;
                        // the queue is full: process its whole batches and keep the rest at its front
                        const int nv = min(qfail, qn);
                        const int nfull = nv / SP_PB * SP_PB;
                        process(nfull);
                        const int rest = nv - nfull;
                        const int keep = tid < rest ? queue[nfull + tid] : 0;
                        __syncthreads();
                        if (tid < rest) queue[tid] = keep;
                        if (tid == 0) { qn = rest; qfail = QCAP; }
                        __syncthreads();
                    }
                }
                base = top;
                if (!__syncthreads_or(pendv != 0u)) break;
                // the slots ran out: process everything queued, then reuse them
                process(qn);
                __syncthreads();
                if (tid == 0) { qn = 0; qfail = QCAP; nimg = 0; }
                __syncthreads();
                base = 0;
            }
        }
    }
    __syncthreads();
    process(qn);
    __syncthreads();
    if (!any) return;
    const int o0 = tt0 * T - PADLO, o1 = tt1 * T - PADLO, o2 = tt2 * T - PADLO;
    for (int i = tid; i < NCELL; i += SP_THREADS) {
        const int l0 = i / (PT * PT), l1 = (i / PT) % PT, l2 = i % PT;
        const int li = l0 * PP + l1 * RP + l2;
        // grid index = position mod L, position = cell - L/2
        const int g0 = ((o0 + l0 - L / 2) % L + L) % L;
        const int g1 = ((o1 + l1 - L / 2) % L + L) % L;
        const int g2 = ((o2 + l2 - L / 2) % L + L) % L;
        const int64_t gi = ((int64_t)g0 * L + g1) * L + g2;
        // the exact integer sum, rounded once to FP32; complex data: component a.comp
        if constexpr (!CPLX) {
            const unsigned long long v = tile64[li];
            if (v) unsafeAtomicAdd(reinterpret_cast<float*>(a.grid) + gi, (float)((double)v * fx_inv));
        } else {
            const long long v = (long long)tile64[li];
            if (v) unsafeAtomicAdd(reinterpret_cast<float*>(a.grid) + 2 * gi + a.comp, (float)((double)v * fx_inv));
        }
    }
}

// bits of the largest |component| of n complex values (atomic max on the bits of non-negative
// floats, which order like the floats); *out starts at 0
__global__ void k_absmax(const float4* __restrict__ b, int64_t n2, const float2* __restrict__ tail, int ntail,
                         unsigned* out) {
    float m = 0.f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
        const float4 v = b[i];
        m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) m = fmaxf(m, fmaxf(fabsf(tail[threadIdx.x].x), fabsf(tail[threadIdx.x].y)));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

__global__ void k_set_u32(unsigned* p, unsigned v) { *p = v; }

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

// 8 wavefronts per workgroup; the tile and the staging fit two workgroups in the LDS of a compute
// unit (one for W = 8).
template <int T, bool CPLX, int NTH = 512>
hipError_t launch_spread(firm_plan p, int L, const int* work, int nwork, void* grid, const float2* b, float fxs,
                         const unsigned* fx_bmax = nullptr, float fx_coef = 0.f, int comp = 0) {
    SpreadArgs a;
    a.N = p->N; a.M = p->M; a.L = L; a.nt = (L + T - 1) / T;
    a.s = (double)L / p->N;
    a.c12 = p->c12s; a.nrm = p->nrms; a.group = p->groups; a.table = p->table; a.Q = p->Q;
    a.poly = p->kb_poly; a.work = reinterpret_cast<const int4*>(work); a.grid = grid;
    a.b = b; a.shifts = p->shiftss; a.rowstart = p->rowstart; a.P = p->P;
    a.vorder = p->vorder; a.vbox = p->vbox;
    static_assert(NTH == SP_VBLK, "a culling round's view blocks are the host's normal-box blocks");
    a.fxs = fxs; a.fx_inv = 1.0 / (double)fxs;
    a.fx_bmax = fx_bmax; a.fx_coef = fx_coef; a.comp = comp;
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

#define SP_TILE_REAL 13
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
                // ranges start on multiples of SP_VBLK: the spread's culling rounds read the normal
                // boxes of whole blocks
                const int per = ((M + nch - 1) / nch + SP_VBLK - 1) / SP_VBLK * SP_VBLK;
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
    return launch_spread<SP_TILE_REAL, false>(p, 4 * p->N, p->tiles_ker, p->ntiles_ker, grid, nullptr, p->fx_ker);
}

hipError_t spread_atb(firm_plan p, const float2* b, float2* grid) {
    // the fixed-point unit follows from the largest |component| of b, found first
    const int64_t n = (int64_t)p->M * p->P;
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, p->stream, p->fx_bmax, 0u);
    hipLaunchKernelGGL(k_absmax, dim3(grid_blocks(n / 2)), dim3(256), 0, p->stream,
                       reinterpret_cast<const float4*>(b), n / 2, b + (n / 2) * 2, (int)(n % 2), p->fx_bmax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // one component per launch: a one-plane tile leaves room for two workgroups per CU
    for (int comp = 0; comp < 2; ++comp) {
        e = launch_spread<SP_TILE_CPLX, true>(p, 2 * p->N, p->tiles_atb, p->ntiles_atb, grid, b, 1.f,
                                                         p->fx_bmax, p->fx_atb_coef, comp);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
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
