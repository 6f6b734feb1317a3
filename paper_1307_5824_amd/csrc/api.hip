// C ABI of libfirm: plan creation and validation, workspaces, and the calls that
// chain the HIP kernels of the other translation units.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "firm_internal.h"

#define KB_DEG 10

namespace {

std::mutex g_err_mu;
std::string g_err;  // last error raised without a plan

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

template <class T>
hipError_t dalloc(T** ptr, size_t count) {
    *ptr = nullptr;
    if (count == 0) return hipSuccess;
    return hipMalloc((void**)ptr, count * sizeof(T));
}

// Modified Bessel function I0 by its power series sum_k ((x/2)^2)^k / (k!)^2.
double bessel_i0(double x) {
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 200; ++k) {
        term *= q / ((double)k * k);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

// Kaiser-Bessel window phi(u) = I0(beta sqrt(1 - (2u/W)^2)) / I0(beta) on |u| <= W/2 and its
// Fourier transform W sinh(sqrt(beta^2 - (W nu / 2)^2)) / sqrt(...) / I0(beta) (sin form past the
// zero of the root).  beta follows Beatty, Nishimura & Pauly (2005) for oversampling 2.
double kb_phi(double u, int W, double beta) {
    const double t = 2.0 * u / W;
    if (std::fabs(t) > 1.0) return 0.0;
    return bessel_i0(beta * std::sqrt(std::max(0.0, 1.0 - t * t))) / bessel_i0(beta);
}

double kb_phihat(double nu, int W, double beta) {
    const double z2 = beta * beta - 0.25 * W * W * nu * nu;
    double v;
    if (z2 > 1e-12) { const double z = std::sqrt(z2); v = W * std::sinh(z) / z; }
    else if (z2 < -1e-12) { const double z = std::sqrt(-z2); v = W * std::sin(z) / z; }
    else v = W;
    return v / bessel_i0(beta);
}

// Solve the (n x n) system A c = y by Gaussian elimination with partial pivoting.
void solve_dense(std::vector<double>& A, std::vector<double>& y, int n) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
            std::swap(y[c], y[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            y[r] -= f * y[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        double s = y[c];
        for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * y[k];
        y[c] = s / A[c * n + c];
    }
}

}  // namespace

// Window tables: per window cell j a degree-KB_DEG polynomial in x = 2 f - 1 (f in [0, 1],
// the cell offset is u = f - W/2 + j) interpolating phi at Chebyshev nodes; reciprocal
// transforms for the deconvolution of the kernel (L = 4N, circulant positions) and of
// A*b (L = 2N, centred indices).
void kb_tables(firm_plan p, std::vector<float>& poly, std::vector<float>& dker, std::vector<float>& datb) {
    const int W = p->kbw, D = KB_DEG, N = p->N;
    const double beta = p->beta;
    poly.assign((size_t)W * (D + 1), 0.f);
    for (int j = 0; j < W; ++j) {
        std::vector<double> A((D + 1) * (D + 1)), y(D + 1);
        for (int i = 0; i <= D; ++i) {
            const double x = std::cos(M_PI * (i + 0.5) / (D + 1));
            const double u = 0.5 * (x + 1.0) - 0.5 * W + j;
            double xp = 1.0;
            for (int k = 0; k <= D; ++k) { A[i * (D + 1) + k] = xp; xp *= x; }
            y[i] = kb_phi(u, W, beta);
        }
        solve_dense(A, y, D + 1);
        for (int k = 0; k <= D; ++k) poly[j * (D + 1) + k] = (float)y[k];
    }
    dker.assign(2 * N, 0.f);
    const double Lk = 4.0 * N;
    for (int pp = 0; pp < 2 * N; ++pp) {
        if (pp == N) continue;
        const int n = pp < N ? pp : pp - 2 * N;
        dker[pp] = (float)(1.0 / kb_phihat(2.0 * M_PI * n / Lk, W, beta));
    }
    datb.assign(N, 0.f);
    const double La = 2.0 * N;
    for (int i = 0; i < N; ++i) {
        const int n = i - N / 2;
        datb[i] = (float)(1.0 / kb_phihat(2.0 * M_PI * n / La, W, beta));
    }
}

firm_status firm_fail(firm_plan p, firm_status s, const std::string& msg) {
    if (p) p->err = msg;
    else { std::lock_guard<std::mutex> lk(g_err_mu); g_err = msg; }
    return s;
}

extern "C" {

int64_t firm_slice_points(int N) {
    if (N <= 0 || N > 4096) return -1;
    int64_t P = 0;
    for (int k1 = -N / 2; k1 <= N / 2; ++k1)
        for (int k2 = -N / 2; k2 <= N / 2; ++k2)
            if (4LL * (k1 * k1 + k2 * k2) <= (int64_t)N * N) ++P;
    return P;
}

const char* firm_last_error(firm_plan p) {
    if (p) return p->err.c_str();
    std::lock_guard<std::mutex> lk(g_err_mu);
    return g_err.c_str();
}

void firm_plan_destroy(firm_plan p) {
    if (!p) return;
    void* dev[] = {p->S2, p->c12, p->nrm, p->group, p->table, p->shifts, p->kb_poly, p->deconv_ker, p->deconv_atb,
                   p->tw, p->kerc, p->khat, p->T1, p->T2, p->r, p->p, p->z, p->tmp, p->partials,
                   p->partials2, p->partials3, p->scal, p->dhalf, p->S1, p->grid, p->ws1, p->ws2,
                   p->tiles_ker, p->tiles_atb, p->dscal, p->rowstart, p->flags, p->khat64, p->T1d,
                   p->T2d, p->tw64, p->x64, p->r64, p->p64, p->q64, p->y64, p->atb64, p->rhs, p->dvec,
                   p->img_ws, p->khat16, p->shtab, p->uws, p->usc, p->c12s, p->nrms, p->groups, p->shiftss,
                   p->vorder, p->vbox};
    for (void* d : dev)
        if (d) (void)hipFree(d);
    if (p->host_scal) (void)hipHostFree(p->host_scal);
    if (p->host_flags) (void)hipHostFree(p->host_flags);
    delete p;
}

firm_status firm_plan_set_stream(firm_plan p, void* stream) {
    if (!p) return firm_fail(nullptr, FIRM_ERR_ARG, "null plan");
    p->stream = (hipStream_t)stream;
    return FIRM_OK;
}

firm_status firm_plan_create(firm_plan* out, int N, int M, const double* rot, const double* shifts,
                             const int32_t* ctf_group, int G, const float* ctf_table, const firm_options* opt) {
    if (!out) return firm_fail(nullptr, FIRM_ERR_ARG, "out is null");
    *out = nullptr;
    if (!is_pow2(N) || N < 8 || N > 256) return firm_fail(nullptr, FIRM_ERR_ARG, "N must be a power of two in [8, 256]");
    if (M < 1 || M > (1 << 24)) return firm_fail(nullptr, FIRM_ERR_ARG, "M must be in [1, 2^24]");
    if (!rot) return firm_fail(nullptr, FIRM_ERR_ARG, "rotations is null");
    if (ctf_table && G < 1) return firm_fail(nullptr, FIRM_ERR_ARG, "G must be >= 1 with a CTF table");
    const int Q = N * N / 4 + 1;
    const int Geff = ctf_table ? G : 1;
    for (int m = 0; m < M; ++m) {
        const double* R = rot + 9 * (int64_t)m;
        for (int i = 0; i < 9; ++i)
            if (!std::isfinite(R[i])) return firm_fail(nullptr, FIRM_ERR_ARG, "rotation " + std::to_string(m) + " not finite");
        double dev = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k) s += R[3 * k + i] * R[3 * k + j];
                dev = std::max(dev, std::fabs(s - (i == j ? 1.0 : 0.0)));
            }
        const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                           R[2] * (R[3] * R[7] - R[4] * R[6]);
        if (dev > 1e-6 || det <= 0)
            return firm_fail(nullptr, FIRM_ERR_ARG, "rotation " + std::to_string(m) + " is not in SO(3)");
        if (shifts && (!std::isfinite(shifts[2 * (int64_t)m]) || !std::isfinite(shifts[2 * (int64_t)m + 1])))
            return firm_fail(nullptr, FIRM_ERR_ARG, "shift " + std::to_string(m) + " not finite");
        if (ctf_group && (ctf_group[m] < 0 || ctf_group[m] >= Geff))
            return firm_fail(nullptr, FIRM_ERR_ARG, "ctf_group[" + std::to_string(m) + "] out of [0, G)");
    }
    if (ctf_table)
        for (int64_t i = 0; i < (int64_t)G * Q; ++i)
            if (!std::isfinite(ctf_table[i])) return firm_fail(nullptr, FIRM_ERR_ARG, "ctf_table not finite");
    firm_options o{};
    if (opt) o = *opt;
    if (o.kb_width == 0) o.kb_width = 7;
    if (o.kb_width < 4 || o.kb_width > 8) return firm_fail(nullptr, FIRM_ERR_ARG, "kb_width must be in [4, 8]");
    if (o.khat_bf16 < 0 || o.khat_bf16 > 2) return firm_fail(nullptr, FIRM_ERR_ARG, "khat_bf16 must be 0, 1 or 2");
    if (o.check_every < 0) return firm_fail(nullptr, FIRM_ERR_ARG, "check_every must be >= 0");
    if (o.precision < 0 || o.precision > 2) return firm_fail(nullptr, FIRM_ERR_ARG, "precision must be 0, 1 or 2");
    if (o.lambda_relative != 0 && o.lambda_relative != 1)
        return firm_fail(nullptr, FIRM_ERR_ARG, "lambda_relative must be 0 or 1");
    if (!(o.inner_tol >= 0.0) || o.inner_tol >= 1.0) return firm_fail(nullptr, FIRM_ERR_ARG, "inner_tol must be in [0, 1)");

    firm_plan p = new firm_plan_s();
    p->N = N; p->M = M; p->G = Geff; p->Q = Q;
    p->P = (int)firm_slice_points(N);
    p->QP = ((N + 1) + 15) / 16 * 16;
    p->QPn = ((N / 2 + 1) + 15) / 16 * 16;
    p->kbw = o.kb_width;
    const double sig = 2.0;
    p->beta = M_PI * std::sqrt((o.kb_width / sig) * (o.kb_width / sig) * (sig - 0.5) * (sig - 0.5) - 0.8);
    p->refine_every = o.refine_every == 0 ? 50 : o.refine_every;
    p->check_every = o.check_every == 0 ? 10 : o.check_every;
    p->stagnation_iters = o.stagnation_iters == 0 ? 300 : o.stagnation_iters;
    p->stream = (hipStream_t)o.stream;
    p->precision = o.precision;
    p->lambda_relative = o.lambda_relative;
    p->inner_tol = o.inner_tol;  // 0: chosen per solve from its tolerance
    p->khat_bf16 = o.khat_bf16;

    // geometry: columns 1 and 2 of R^{-1} = R^T are rows 1 and 2 of R; normal = c1 x c2
    std::vector<double> c12((size_t)M * 6);
    std::vector<float> nrm((size_t)M * 4);
    std::vector<int32_t> grp(M, 0);
    double k0 = 0.0;
    for (int m = 0; m < M; ++m) {
        const double* R = rot + 9 * (int64_t)m;
        double* c = &c12[6 * (size_t)m];
        for (int d = 0; d < 3; ++d) { c[d] = R[d]; c[3 + d] = R[3 + d]; }
        const double n0 = c[1] * c[5] - c[2] * c[4], n1 = c[2] * c[3] - c[0] * c[5], n2 = c[0] * c[4] - c[1] * c[3];
        nrm[4 * m] = (float)n0; nrm[4 * m + 1] = (float)n1; nrm[4 * m + 2] = (float)n2; nrm[4 * m + 3] = 0.f;
        if (ctf_group) grp[m] = ctf_group[m];
        const double h0 = ctf_table ? (double)ctf_table[(int64_t)grp[m] * Q] : 1.0;
        k0 += h0 * h0;
    }
    p->ker_k0 = k0;
    // The gridding visits the views in the order of their planes' normals: each normal folded to
    // the hemisphere where its largest component is positive, keyed by that axis and a Morton
    // code of the other two components over it, so that a block of SP_VBLK consecutive views
    // spans a small cone and the box of its normals lets a tile skip the whole block.
    std::vector<int32_t> vord(M);
    std::vector<double> c12s((size_t)M * 6);
    std::vector<float> nrms((size_t)M * 4);
    std::vector<int32_t> grps(M);
    std::vector<double> shs(shifts ? (size_t)M * 2 : 0);
    const int nvblk = (M + SP_VBLK - 1) / SP_VBLK;
    std::vector<float4> vbox((size_t)nvblk * 2);
    {
        std::vector<std::pair<uint64_t, int32_t>> key(M);
        for (int m = 0; m < M; ++m) {
            const float* n = &nrm[4 * (size_t)m];
            int ax = 0;
            for (int d = 1; d < 3; ++d)
                if (std::fabs(n[d]) > std::fabs(n[ax])) ax = d;
            const double inv = 1.0 / (double)n[ax];  // |n[ax]| >= 1/sqrt(3)
            const double u = n[(ax + 1) % 3] * inv, v = n[(ax + 2) % 3] * inv;  // in [-1, 1]
            const uint32_t qu = (uint32_t)std::min(1023.0, std::max(0.0, (u + 1.0) * 511.5));
            const uint32_t qv = (uint32_t)std::min(1023.0, std::max(0.0, (v + 1.0) * 511.5));
            uint64_t mort = 0;
            for (int b = 0; b < 10; ++b) mort |= (uint64_t)((qu >> b) & 1u) << (2 * b) | (uint64_t)((qv >> b) & 1u) << (2 * b + 1);
            key[m] = {((uint64_t)ax << 20) | mort, m};
        }
        std::stable_sort(key.begin(), key.end());
        for (int j = 0; j < M; ++j) {
            const int m = key[j].second;
            vord[j] = m;
            for (int d = 0; d < 6; ++d) c12s[6 * (size_t)j + d] = c12[6 * (size_t)m + d];
            const float* n = &nrm[4 * (size_t)m];
            int ax = 0;
            for (int d = 1; d < 3; ++d)
                if (std::fabs(n[d]) > std::fabs(n[ax])) ax = d;
            const float sg = n[ax] < 0.f ? -1.f : 1.f;  // the same plane; the tests use |n . x|
            for (int d = 0; d < 3; ++d) nrms[4 * (size_t)j + d] = sg * n[d];
            nrms[4 * (size_t)j + 3] = 0.f;
            grps[j] = grp[m];
            if (shifts) { shs[2 * (size_t)j] = shifts[2 * (size_t)m]; shs[2 * (size_t)j + 1] = shifts[2 * (size_t)m + 1]; }
        }
        for (int bk = 0; bk < nvblk; ++bk) {
            float lo[3] = {1e30f, 1e30f, 1e30f}, hi[3] = {-1e30f, -1e30f, -1e30f};
            double l1 = 0.0;
            for (int j = bk * SP_VBLK; j < std::min(M, (bk + 1) * SP_VBLK); ++j) {
                const float* n = &nrms[4 * (size_t)j];
                for (int d = 0; d < 3; ++d) { lo[d] = std::min(lo[d], n[d]); hi[d] = std::max(hi[d], n[d]); }
                l1 = std::max(l1, (double)std::fabs(n[0]) + std::fabs(n[1]) + std::fabs(n[2]));
            }
            vbox[2 * (size_t)bk] = make_float4(lo[0], lo[1], lo[2], (float)(l1 * (1.0 + 1e-6)));
            vbox[2 * (size_t)bk + 1] = make_float4(hi[0], hi[1], hi[2], 0.f);
        }
    }
    std::vector<int> rowstart(N + 1);
    {
        int off = 0;
        for (int k1 = -N / 2; k1 <= N / 2; ++k1) {
            int lo = 1, cnt = 0;
            for (int k2 = -N / 2; k2 <= N / 2; ++k2)
                if (4 * (k1 * k1 + k2 * k2) <= N * N) { if (cnt == 0) lo = k2; ++cnt; }
            rowstart[k1 + N / 2] = off - lo;
            off += cnt;
        }
    }
    std::vector<float2> tw(FIRM_TWN);
    for (int m = 0; m < FIRM_TWN; ++m) {
        const double a = -2.0 * M_PI * m / FIRM_TWN;
        tw[m] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    std::vector<float> poly, dker, datb;
    kb_tables(p, poly, dker, datb);
    {
        // fixed-point unit of the kernel gridding: every term 2 h^2 w1 w2 w3 stays below 2^31 units
        double wmax = 0.0;
        for (int j = 0; j < p->kbw; ++j)
            for (int i = 0; i <= 4000; ++i) {
                const double x = -1.0 + i / 2000.0;
                double v = 0.0;
                for (int k = KB_DEG; k >= 0; --k) v = v * x + (double)poly[j * (KB_DEG + 1) + k];
                wmax = std::max(wmax, std::fabs(v));
            }
        double hmax = ctf_table ? 0.0 : 1.0;
        if (ctf_table)
            for (int64_t i = 0; i < (int64_t)Geff * Q; ++i) hmax = std::max(hmax, std::fabs((double)ctf_table[i]));
        // A*b: a term is w1 w2 w3 h e^{i theta} (b(k) + conj b(-k)) per component, at most
        // 2 sqrt(2) hmax bmax wmax^3 in magnitude; the unit is fixed per call from bmax
        p->fx_atb_coef = (float)std::min(1e30, 2147483648.0 / (2.0 * std::sqrt(2.0) * std::max(hmax, 1e-30) * wmax * wmax * wmax * 1.05));
        const double bound = 2.0 * hmax * hmax * wmax * wmax * wmax * 1.05;
        int e = bound > 0.0 ? (int)std::floor(std::log2(2147483648.0 / bound)) : 0;
        e = std::min(std::max(e, -100), 100);
        p->fx_ker = std::ldexp(1.0f, e);
    }
    std::vector<int> wk = spread_worklist(4 * N, spread_tile_real(), M, 4.0);
    std::vector<int> wa = spread_worklist(2 * N, spread_tile_cplx(), M, 2.0);
    p->ntiles_ker = (int)(wk.size() / 4);
    p->ntiles_atb = (int)(wa.size() / 4);

    const int64_t n3 = (int64_t)N * N * N;
    const int64_t N2 = 2 * N;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(dalloc(&p->c12, c12.size()));
    chk(dalloc(&p->nrm, nrm.size()));
    chk(dalloc(&p->group, (size_t)M));
    if (ctf_table) chk(dalloc(&p->table, (size_t)G * Q));
    if (shifts) chk(dalloc(&p->shifts, (size_t)M * 2));
    chk(dalloc(&p->c12s, c12s.size()));
    chk(dalloc(&p->nrms, nrms.size()));
    chk(dalloc(&p->groups, (size_t)M));
    if (shifts) chk(dalloc(&p->shiftss, (size_t)M * 2));
    chk(dalloc(&p->vorder, (size_t)M));
    chk(dalloc(&p->vbox, vbox.size()));
    chk(dalloc(&p->kb_poly, poly.size()));
    chk(dalloc(&p->deconv_ker, dker.size()));
    chk(dalloc(&p->deconv_atb, datb.size()));
    chk(dalloc(&p->tw, (size_t)FIRM_TWN));
    chk(dalloc(&p->kerc, (size_t)(N2 * N2 * N2)));
    chk(dalloc(&p->khat, blocked_spectrum_elems(2 * N, 2 * N, N + 1, false)));
    if (p->khat_bf16) {
        chk(dalloc(&p->khat16, blocked_spectrum_elems(2 * N, 2 * N, N + 1, false)));
        chk(dalloc(&p->shtab, (size_t)448));
    }
    chk(dalloc(&p->T1, (size_t)((int64_t)N * N * p->QP)));
    chk(dalloc(&p->T2, (size_t)fft_t2_elems(N, false)));
    chk(dalloc(&p->r, (size_t)n3));
    chk(dalloc(&p->p, (size_t)n3));
    chk(dalloc(&p->z, (size_t)n3));
    chk(dalloc(&p->tmp, (size_t)n3));
    p->npart = 16384;
    chk(dalloc(&p->partials, (size_t)p->npart));
    chk(dalloc(&p->partials2, (size_t)p->npart));
    chk(dalloc(&p->partials3, (size_t)p->npart));
    chk(dalloc(&p->scal, 32));
    chk(dalloc(&p->flags, 8));
    chk(dalloc(&p->dhalf, blocked_spectrum_elems(N, N, N / 2 + 1, false)));
    chk(dalloc(&p->S1, (size_t)((int64_t)N * N * p->QPn)));
    chk(dalloc(&p->dscal, 8));
    p->fx_bmax = reinterpret_cast<unsigned*>(p->dscal + 1);
    chk(dalloc(&p->rowstart, (size_t)(N + 1)));
    chk(dalloc(&p->tiles_ker, wk.size()));
    chk(dalloc(&p->tiles_atb, wa.size()));
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->host_scal, 32 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->host_flags, 8 * sizeof(int), hipHostMallocDefault);
    if (e != hipSuccess) {
        firm_plan_destroy(p);
        return firm_fail(nullptr, e == hipErrorOutOfMemory ? FIRM_ERR_ALLOC : FIRM_ERR_HIP,
                         std::string("plan allocation: ") + hipGetErrorString(e));
    }
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    up(p->c12, c12.data(), c12.size() * sizeof(double));
    up(p->nrm, nrm.data(), nrm.size() * sizeof(float));
    up(p->group, grp.data(), grp.size() * sizeof(int32_t));
    if (ctf_table) up(p->table, ctf_table, (size_t)G * Q * sizeof(float));
    if (shifts) up(p->shifts, shifts, (size_t)M * 2 * sizeof(double));
    up(p->c12s, c12s.data(), c12s.size() * sizeof(double));
    up(p->nrms, nrms.data(), nrms.size() * sizeof(float));
    up(p->groups, grps.data(), grps.size() * sizeof(int32_t));
    if (shifts) up(p->shiftss, shs.data(), shs.size() * sizeof(double));
    up(p->vorder, vord.data(), vord.size() * sizeof(int32_t));
    up(p->vbox, vbox.data(), vbox.size() * sizeof(float4));
    up(p->kb_poly, poly.data(), poly.size() * sizeof(float));
    up(p->deconv_ker, dker.data(), dker.size() * sizeof(float));
    up(p->deconv_atb, datb.data(), datb.size() * sizeof(float));
    up(p->tw, tw.data(), tw.size() * sizeof(float2));
    up(p->rowstart, rowstart.data(), rowstart.size() * sizeof(int));
    up(p->tiles_ker, wk.data(), wk.size() * sizeof(int));
    up(p->tiles_atb, wa.data(), wa.size() * sizeof(int));
    if (e == hipSuccess) e = noalloc_scratch_setup();
    if (e != hipSuccess) {
        firm_plan_destroy(p);
        return firm_fail(nullptr, FIRM_ERR_HIP, std::string("plan upload: ") + hipGetErrorString(e));
    }
    *out = p;
    return FIRM_OK;
}

}  // extern "C"

namespace {

firm_status ensure_ws(firm_plan p, void** ptr, size_t* have, size_t need) {
    if (*have >= need) return FIRM_OK;
    if (*ptr) { (void)hipFree(*ptr); *ptr = nullptr; *have = 0; }
    hipError_t e = hipMalloc(ptr, need);
    if (e != hipSuccess) {
        *ptr = nullptr;
        return firm_fail(p, FIRM_ERR_ALLOC, std::string("workspace allocation: ") + hipGetErrorString(e));
    }
    *have = need;
    return FIRM_OK;
}

// Workspaces for both gridding pipelines (sized for the larger, the kernel's).
firm_status ensure_grid_ws(firm_plan p) {
    const size_t N = p->N, L = 4 * N, N2 = 2 * N;
    const size_t grid = std::max(L * L * L * sizeof(float), N2 * N2 * N2 * sizeof(float2));
    const size_t w1 = std::max({L * L * N * sizeof(float2), N2 * N2 * N * sizeof(float2),
                                N2 * N2 * (size_t)p->QP * sizeof(float2)});
    const size_t w2 = std::max(L * N2 * N * sizeof(float2) + N2 * N2 * N * sizeof(float),
                               N2 * N * N * sizeof(float2));
    firm_status s;
    if ((s = ensure_ws(p, &p->grid, &p->grid_bytes, grid)) != FIRM_OK) return s;
    if ((s = ensure_ws(p, &p->ws1, &p->ws1_bytes, w1)) != FIRM_OK) return s;
    return ensure_ws(p, &p->ws2, &p->ws2_bytes, w2);
}

// Ker(0) of the current kernel (circulant position 0), for the relative lambda reading.
firm_status read_ker0(firm_plan p) {
    float v = 0.f;
    FIRM_HIP(p, hipMemcpyAsync(&v, p->kerc, sizeof(float), hipMemcpyDeviceToHost, p->stream));
    FIRM_HIP(p, hipStreamSynchronize(p->stream));
    p->ker0 = v;
    return FIRM_OK;
}

double lambda_eff(firm_plan p, double lam) { return p->lambda_relative ? lam * p->ker0 : lam; }

// The product's spectrum from the circulant column kerc (in the plan): Ker(0), then the spectrum
// with the damping term of the plan's regularizer (its weight read like lambda) and its 16-bit copy.
firm_status spectrum_from_kerc(firm_plan p) {
    firm_status s = read_ker0(p);
    if (s != FIRM_OK) return s;
    p->reg_mu_eff = lambda_eff(p, p->reg_mu);
    FIRM_HIP(p, fft_khat_from_kerc(p, (float2*)p->ws1));
    p->have_kernel = true;
    p->khat64_valid = false;
    return FIRM_OK;
}

}  // namespace

firm_status ensure_fp64(firm_plan p) {
    const size_t N = p->N, N2 = 2 * N, n3 = N * N * N;
    hipError_t e = hipSuccess;
    auto al = [&](auto** ptr, size_t count) {
        if (e == hipSuccess && *ptr == nullptr) e = hipMalloc((void**)ptr, count * sizeof(**ptr));
    };
    al(&p->khat64, blocked_spectrum_elems(2 * N, 2 * N, N + 1, true));
    al(&p->T1d, N * N * p->QP);
    al(&p->T2d, (size_t)fft_t2_elems((int)N, true));
    al(&p->tw64, (size_t)FIRM_TWN);
    al(&p->x64, n3);
    al(&p->r64, n3);
    al(&p->p64, n3);
    al(&p->q64, n3);
    al(&p->y64, n3);
    al(&p->atb64, n3);
    al(&p->rhs, n3);
    al(&p->dvec, n3);
    if (e != hipSuccess) return firm_fail(p, FIRM_ERR_ALLOC, std::string("FP64 buffers: ") + hipGetErrorString(e));
    if (!p->khat64_valid) {
        std::vector<double2> tw(FIRM_TWN);
        for (int m = 0; m < FIRM_TWN; ++m) {
            const double a = -2.0 * M_PI * m / FIRM_TWN;
            tw[m] = make_double2(std::cos(a), std::sin(a));
        }
        FIRM_HIP(p, hipMemcpy(p->tw64, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice));
        double* k64 = nullptr;
        double2* w1 = nullptr;
        FIRM_HIP(p, hipMalloc((void**)&k64, N2 * N2 * N2 * sizeof(double)));
        e = hipMalloc((void**)&w1, N2 * N2 * p->QP * sizeof(double2));
        if (e == hipSuccess) e = kerc_to_double(p, k64);
        if (e == hipSuccess) e = fft_khat64_from_kerc64(p, k64, w1);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        (void)hipFree(k64);
        if (w1) (void)hipFree(w1);
        if (e != hipSuccess) return firm_fail(p, FIRM_ERR_HIP, std::string("FP64 spectrum: ") + hipGetErrorString(e));
        p->khat64_valid = true;
    }
    return FIRM_OK;
}

extern "C" {

firm_status firm_kernel_precompute(firm_plan p) {
    if (!p) return firm_fail(nullptr, FIRM_ERR_ARG, "null plan");
    firm_status s = ensure_grid_ws(p);
    if (s != FIRM_OK) return s;
    const size_t N = p->N, L = 4 * N, N2 = 2 * N;
    float* grid = (float*)p->grid;
    float2* h1 = (float2*)p->ws1;
    float2* h2 = (float2*)p->ws2;
    float* chalf = (float*)((char*)p->ws2 + L * N2 * N * sizeof(float2));
    FIRM_HIP(p, fill_zero(grid, L * L * L * sizeof(float), p->stream));
    FIRM_HIP(p, spread_ker(p, grid));
    FIRM_HIP(p, fft_ker_grid(p, grid, h1, h2, chalf));
    FIRM_HIP(p, kerc_from_half(p, chalf));
    return spectrum_from_kerc(p);
}

firm_status firm_kernel_get(firm_plan p, float* ker) {
    if (!p || !ker) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (!p->have_kernel) return firm_fail(p, FIRM_ERR_STATE, "no kernel: call firm_kernel_precompute or firm_kernel_set");
    FIRM_HIP(p, kerc_to_centred(p, ker));
    return FIRM_OK;
}

firm_status firm_kernel_set(firm_plan p, const float* ker) {
    if (!p || !ker) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    const size_t N2 = 2 * p->N;
    firm_status s = ensure_ws(p, &p->ws1, &p->ws1_bytes, N2 * N2 * (size_t)p->QP * sizeof(float2));
    if (s != FIRM_OK) return s;
    FIRM_HIP(p, kerc_from_centred(p, ker));
    return spectrum_from_kerc(p);
}

firm_status firm_set_regularizer(firm_plan p, int order, double mu) {
    if (!p) return firm_fail(nullptr, FIRM_ERR_ARG, "null plan");
    if (order < 0 || order > 3) return firm_fail(p, FIRM_ERR_ARG, "order must be in [0, 3]");
    if (!(mu >= 0.0) || !std::isfinite(mu)) return firm_fail(p, FIRM_ERR_ARG, "mu must be finite and >= 0");
    p->reg_order = mu > 0.0 ? order : 0;
    p->reg_mu = order > 0 ? mu : 0.0;
    if (!p->have_kernel) return FIRM_OK;  // applied when the kernel's spectrum is built
    const size_t N2 = 2 * p->N;
    firm_status s = ensure_ws(p, &p->ws1, &p->ws1_bytes, N2 * N2 * (size_t)p->QP * sizeof(float2));
    if (s != FIRM_OK) return s;
    return spectrum_from_kerc(p);
}

firm_status firm_kernel_spectrum(firm_plan p, float* khat) {
    if (!p || !khat) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (!p->have_kernel) return firm_fail(p, FIRM_ERR_STATE, "no kernel");
    FIRM_HIP(p, fft_khat_unblock(p, khat));
    return FIRM_OK;
}

firm_status firm_backproject(firm_plan p, const void* b, float* atb) {
    if (!p || !b || !atb) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    firm_status s = ensure_grid_ws(p);
    if (s != FIRM_OK) return s;
    const size_t N = p->N, L = 2 * N;
    float2* grid = (float2*)p->grid;
    float2* j1 = (float2*)p->ws1;
    float2* j2 = (float2*)p->ws2;
    FIRM_HIP(p, fill_zero(grid, L * L * L * sizeof(float2), p->stream));
    FIRM_HIP(p, spread_atb(p, (const float2*)b, grid));
    FIRM_HIP(p, atb_k0_term(p, (const float2*)b, p->dscal));
    FIRM_HIP(p, fft_atb_grid(p, grid, j1, j2, atb, p->dscal));
    return FIRM_OK;
}

firm_status firm_forward_project(firm_plan p, const float* V, void* b) {
    if (!p || !V || !b) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    firm_status s = ensure_grid_ws(p);
    if (s != FIRM_OK) return s;
    FIRM_HIP(p, forward_project(p, V, (float2*)b));
    return FIRM_OK;
}

firm_status firm_apply_AtA(firm_plan p, const float* x, float* y, double lambda) {
    if (!p || !x || !y) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (x == y) return firm_fail(p, FIRM_ERR_ARG, "x and y must not alias");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return firm_fail(p, FIRM_ERR_ARG, "lambda must be finite and >= 0");
    if (!p->have_kernel) return firm_fail(p, FIRM_ERR_STATE, "no kernel: call firm_kernel_precompute or firm_kernel_set");
    FIRM_HIP(p, fft_apply_AtA(p, x, y, (float)lambda_eff(p, lambda)));
    return FIRM_OK;
}

firm_status firm_apply_AtA_timed(firm_plan p, const float* x, float* y, double lambda, int reps,
                                 float* pass_ms) {
    if (!p || !x || !y || !pass_ms) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (x == y) return firm_fail(p, FIRM_ERR_ARG, "x and y must not alias");
    if (reps < 1) return firm_fail(p, FIRM_ERR_ARG, "reps must be >= 1");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return firm_fail(p, FIRM_ERR_ARG, "lambda must be finite and >= 0");
    if (!p->have_kernel) return firm_fail(p, FIRM_ERR_STATE, "no kernel: call firm_kernel_precompute or firm_kernel_set");
    hipEvent_t ev[10];
    for (int i = 0; i < 10; ++i) FIRM_HIP(p, hipEventCreate(&ev[i]));
    double acc[5] = {0, 0, 0, 0, 0};
    hipError_t e = hipSuccess;
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        e = fft_apply_AtA_events(p, x, y, (float)lambda_eff(p, lambda), ev);
        if (e == hipSuccess) e = hipEventSynchronize(ev[9]);
        for (int i = 0; i < 5 && e == hipSuccess; ++i) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
            acc[i] += ms;
        }
    }
    for (int i = 0; i < 10; ++i) (void)hipEventDestroy(ev[i]);
    if (e != hipSuccess) return firm_fail(p, FIRM_ERR_HIP, std::string("timed apply: ") + hipGetErrorString(e));
    for (int i = 0; i < 5; ++i) pass_ms[i] = (float)(acc[i] / reps);
    return FIRM_OK;
}

firm_status firm_apply_AtA_f64(firm_plan p, const double* x, double* y, double lambda) {
    if (!p || !x || !y) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (x == y) return firm_fail(p, FIRM_ERR_ARG, "x and y must not alias");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return firm_fail(p, FIRM_ERR_ARG, "lambda must be finite and >= 0");
    if (!p->have_kernel) return firm_fail(p, FIRM_ERR_STATE, "no kernel: call firm_kernel_precompute or firm_kernel_set");
    firm_status s = ensure_fp64(p);
    if (s != FIRM_OK) return s;
    FIRM_HIP(p, fft_apply_AtA64(p, x, y, lambda_eff(p, lambda)));
    return FIRM_OK;
}

static firm_status cg_args(firm_plan p, const void* atb, const void* x, double lambda, double tol, int max_iter,
                           const float* d, firm_cg_report* rep) {
    if (!p || !atb || !x) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return firm_fail(p, FIRM_ERR_ARG, "lambda must be finite and >= 0");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return firm_fail(p, FIRM_ERR_ARG, "tol must be finite and >= 0");
    if (max_iter < 0) return firm_fail(p, FIRM_ERR_ARG, "max_iter must be >= 0");
    if (d && p->precision == 2) return firm_fail(p, FIRM_ERR_ARG, "precision 2 runs plain CG: pass no preconditioner");
    if (!p->have_kernel) return firm_fail(p, FIRM_ERR_STATE, "no kernel: call firm_kernel_precompute or firm_kernel_set");
    if (rep) std::memset(rep, 0, sizeof(*rep));
    return FIRM_OK;
}

firm_status firm_cg_solve(firm_plan p, const float* atb, float* x, double lambda, double tol, int max_iter,
                          const float* d, firm_cg_report* rep) {
    firm_status s = cg_args(p, atb, x, lambda, tol, max_iter, d, rep);
    if (s != FIRM_OK) return s;
    return cg_solve(p, atb, x, lambda_eff(p, lambda), tol, max_iter, d, rep);
}

firm_status firm_cg_solve_f64(firm_plan p, const double* atb, double* x, double lambda, double tol, int max_iter,
                              const float* d, firm_cg_report* rep) {
    firm_status s = cg_args(p, atb, x, lambda, tol, max_iter, d, rep);
    if (s != FIRM_OK) return s;
    if (p->precision == 0) return firm_fail(p, FIRM_ERR_STATE, "precision 0 solves in FP32: use firm_cg_solve");
    return cg_solve64(p, atb, x, lambda_eff(p, lambda), tol, max_iter, d, rep);
}

firm_status firm_precond_apply(firm_plan p, const float* d, const float* r, float* z) {
    if (!p || !d || !r || !z) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    FIRM_HIP(p, precond_set(p, d));
    FIRM_HIP(p, fft_precond(p, p->dhalf, r, z));
    return FIRM_OK;
}

firm_status firm_images_to_slices(firm_plan p, const float* images, void* b) {
    if (!p || !images || !b) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    const size_t per = (size_t)p->N * p->QPn * sizeof(float2);
    const int G = (int)std::max<size_t>(1, std::min<size_t>((size_t)p->M, (size_t(1) << 30) / per));
    firm_status s = ensure_ws(p, &p->img_ws, &p->img_ws_bytes, (size_t)G * per);
    if (s != FIRM_OK) return s;
    float2* ws = (float2*)p->img_ws;
    const int64_t npix = (int64_t)p->N * p->N;
    for (int m0 = 0; m0 < p->M; m0 += G) {
        const int g = std::min(G, p->M - m0);
        FIRM_HIP(p, fft_images_r2c(p, images + (int64_t)m0 * npix, g, ws));
        FIRM_HIP(p, images_gather(p, ws, g, m0, (float2*)b));
    }
    return FIRM_OK;
}

firm_status firm_synth_images(firm_plan p, int B, const double* centers, const double* sigmas, const double* amps,
                              double snr, uint64_t seed, float* images) {
    if (!p || !images || (B > 0 && (!centers || !sigmas || !amps))) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (B < 1 || B > 320) return firm_fail(p, FIRM_ERR_ARG, "B must be in [1, 320]");
    std::vector<double> bl((size_t)B * 5);
    for (int i = 0; i < B; ++i) {
        if (!(sigmas[i] > 0.0) || !std::isfinite(sigmas[i]))
            return firm_fail(p, FIRM_ERR_ARG, "image blobs need sigma > 0");
        for (int d = 0; d < 3; ++d) bl[5 * i + d] = centers[3 * i + d];
        bl[5 * i + 3] = sigmas[i];
        bl[5 * i + 4] = amps[i] * std::sqrt(2.0 * M_PI) * sigmas[i];
    }
    const int64_t nscr = synth_images_scratch(p->N, p->M);
    double* dbl = nullptr;
    FIRM_HIP(p, hipMalloc((void**)&dbl, (bl.size() + (size_t)nscr) * sizeof(double)));
    hipError_t e = hipMemcpyAsync(dbl, bl.data(), bl.size() * sizeof(double), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = synth_images(p, B, dbl, snr, seed, images, dbl + bl.size(), nscr);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    (void)hipFree(dbl);
    if (e != hipSuccess) return firm_fail(p, FIRM_ERR_HIP, std::string("synth images: ") + hipGetErrorString(e));
    return FIRM_OK;
}

firm_status firm_synth_slices(firm_plan p, int B, const double* centers, const double* sigmas, const double* amps,
                              double snr, uint64_t seed, void* b) {
    if (!p || !b || (B > 0 && (!centers || !sigmas || !amps))) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (B < 1 || B > 320) return firm_fail(p, FIRM_ERR_ARG, "B must be in [1, 320]");
    std::vector<double> bl((size_t)B * 5);
    for (int i = 0; i < B; ++i) {
        if (!(sigmas[i] >= 0.0)) return firm_fail(p, FIRM_ERR_ARG, "sigma must be >= 0");
        for (int d = 0; d < 3; ++d) bl[5 * i + d] = centers[3 * i + d];
        bl[5 * i + 3] = sigmas[i];
        bl[5 * i + 4] = sigmas[i] > 0 ? amps[i] * std::pow(2.0 * M_PI * sigmas[i] * sigmas[i], 1.5) : amps[i];
    }
    double* dbl = nullptr;
    FIRM_HIP(p, hipMalloc((void**)&dbl, bl.size() * sizeof(double)));
    hipError_t e = hipMemcpyAsync(dbl, bl.data(), bl.size() * sizeof(double), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = synth_slices(p, B, dbl, snr, seed, (float2*)b, p->partials);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    (void)hipFree(dbl);
    if (e != hipSuccess) return firm_fail(p, FIRM_ERR_HIP, std::string("synth: ") + hipGetErrorString(e));
    return FIRM_OK;
}

firm_status firm_synth_volume(firm_plan p, int B, const double* centers, const double* sigmas, const double* amps,
                              float* V) {
    if (!p || !V || (B > 0 && (!centers || !sigmas || !amps))) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (B < 1 || B > 320) return firm_fail(p, FIRM_ERR_ARG, "B must be in [1, 320]");
    std::vector<double> bl((size_t)B * 5);
    for (int i = 0; i < B; ++i) {
        if (!(sigmas[i] > 0.0) || !std::isfinite(sigmas[i])) return firm_fail(p, FIRM_ERR_ARG, "volume blobs need sigma > 0");
        for (int d = 0; d < 3; ++d) bl[5 * i + d] = centers[3 * i + d];
        bl[5 * i + 3] = sigmas[i];
        bl[5 * i + 4] = amps[i];
    }
    double* dbl = nullptr;
    FIRM_HIP(p, hipMalloc((void**)&dbl, bl.size() * sizeof(double)));
    hipError_t e = hipMemcpyAsync(dbl, bl.data(), bl.size() * sizeof(double), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = synth_volume(p, B, dbl, V);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    (void)hipFree(dbl);
    if (e != hipSuccess) return firm_fail(p, FIRM_ERR_HIP, std::string("synth volume: ") + hipGetErrorString(e));
    return FIRM_OK;
}

firm_status firm_fsc(firm_plan p, const float* V1, const float* V2, double cone_deg, double* out) {
    if (!p || !V1 || !V2 || !out) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (!(cone_deg >= 0.0 && cone_deg <= 90.0)) return firm_fail(p, FIRM_ERR_ARG, "cone_deg must be in [0, 90]");
    const int64_t N = p->N;
    const int S = fsc_max_shells();
    if (N / 2 > S) return firm_fail(p, FIRM_ERR_ARG, "N too large for the shell table");
    if (!p->S2) {
        firm_status s = ensure_ws(p, (void**)&p->S2, &p->s2_bytes, (size_t)(N * N * p->QPn) * sizeof(float2));
        if (s != FIRM_OK) return s;
    }
    FIRM_HIP(p, fsc_sums(p, V1, V2, cone_deg, p->partials3));
    std::vector<double> h((size_t)9 * S);
    FIRM_HIP(p, hipMemcpyAsync(h.data(), p->partials3, h.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    FIRM_HIP(p, hipStreamSynchronize(p->stream));
    const int nsh = (int)(N / 2 - 1);
    for (int r = 0; r < 3; ++r)
        for (int i = 1; i <= nsh; ++i) {
            const double num = h[(3 * r) * S + i], d1 = h[(3 * r + 1) * S + i], d2 = h[(3 * r + 2) * S + i];
            out[r * nsh + i - 1] = d1 > 0.0 && d2 > 0.0 ? num / std::sqrt(d1 * d2) : std::nan("");
        }
    return FIRM_OK;
}

}  // extern "C"

extern "C" {

firm_status firm_kernel_features(firm_plan p, double lam_rel, int res, float* feat) {
    if (!p || !feat) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (res < 32 || res > 256 || (res & (res - 1)) || res > 2 * p->N)
        return firm_fail(p, FIRM_ERR_ARG, "res must be a power of two in [32, min(256, 2N)]");
    if (!(lam_rel >= 0.0) || !std::isfinite(lam_rel)) return firm_fail(p, FIRM_ERR_ARG, "lam_rel must be >= 0");
    if (!p->have_kernel) return firm_fail(p, FIRM_ERR_STATE, "no kernel");
    FIRM_HIP(p, kernel_features(p, (float)lam_rel, res, feat));
    return FIRM_OK;
}

firm_status firm_probe_stats(firm_plan p, const float* probes, int nprobes, double lambda, float* A, float* B,
                             double* sumc) {
    if (!p || !probes || !A || !B || !sumc) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (nprobes < 1) return firm_fail(p, FIRM_ERR_ARG, "nprobes must be >= 1");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return firm_fail(p, FIRM_ERR_ARG, "lambda must be finite and >= 0");
    if (!p->have_kernel) return firm_fail(p, FIRM_ERR_STATE, "no kernel");
    const int64_t N = p->N, n3 = N * N * N;
    if (!p->S2) {
        firm_status s = ensure_ws(p, (void**)&p->S2, &p->s2_bytes, (size_t)(N * N * p->QPn) * sizeof(float2));
        if (s != FIRM_OK) return s;
    }
    hipStream_t st = p->stream;
    FIRM_HIP(p, fill_zero(A, n3 * sizeof(float), st));
    FIRM_HIP(p, fill_zero(B, n3 * sizeof(float), st));
    const int nb = 1024;
    double total = 0.0;
    for (int k = 0; k < nprobes; ++k) {
        const float* z = probes + k * n3;
        FIRM_HIP(p, fft_apply_AtA(p, z, p->tmp, (float)lambda_eff(p, lambda)));
        FIRM_HIP(p, fft_forward_r2c(p, p->tmp, p->S2));
        FIRM_HIP(p, fft_forward_r2c(p, z, p->S1));
        FIRM_HIP(p, probe_accumulate(p, p->S1, p->S2, A, B, p->partials3, nb));
        FIRM_HIP(p, hipMemcpyAsync(p->host_scal + 16, p->partials3, 16 * sizeof(double), hipMemcpyDeviceToHost, st));
        std::vector<double> part(nb);
        FIRM_HIP(p, hipMemcpyAsync(part.data(), p->partials3, nb * sizeof(double), hipMemcpyDeviceToHost, st));
        FIRM_HIP(p, hipStreamSynchronize(st));
        for (double v : part) total += v;
    }
    *sumc = total;
    return FIRM_OK;
}

firm_status firm_chan_spectrum(firm_plan p, double lambda, float* t) {
    if (!p || !t) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return firm_fail(p, FIRM_ERR_ARG, "lambda must be finite and >= 0");
    if (!p->have_kernel) return firm_fail(p, FIRM_ERR_STATE, "no kernel");
    FIRM_HIP(p, chan_spectrum(p, lambda_eff(p, lambda), t));
    return FIRM_OK;
}

firm_status firm_pcg_unrolled(firm_plan p, const float* d, const float* probes, int nprobes, int k, double lambda,
                              double* loss, float* grad) {
    if (!p || !d || !probes || !loss) return firm_fail(p, FIRM_ERR_ARG, "null argument");
    if (nprobes < 1) return firm_fail(p, FIRM_ERR_ARG, "nprobes must be >= 1");
    if (k < 1 || k > 1000) return firm_fail(p, FIRM_ERR_ARG, "k must be in [1, 1000]");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return firm_fail(p, FIRM_ERR_ARG, "lambda must be finite and >= 0");
    if (!p->have_kernel) return firm_fail(p, FIRM_ERR_STATE, "no kernel");
    const int64_t N = p->N;
    firm_status s = ensure_ws(p, (void**)&p->uws, &p->uws_bytes,
                              (size_t)unrolled_workspace_floats((int)N, k) * sizeof(float));
    if (s == FIRM_OK)
        s = ensure_ws(p, (void**)&p->usc, &p->usc_bytes, (size_t)unrolled_scalar_count(k) * sizeof(double));
    if (s == FIRM_OK && !p->S2)
        s = ensure_ws(p, (void**)&p->S2, &p->s2_bytes, (size_t)(N * N * p->QPn) * sizeof(float2));
    if (s != FIRM_OK) return s;
    FIRM_HIP(p, pcg_unrolled(p, d, probes, nprobes, k, (float)lambda_eff(p, lambda), p->uws, p->usc, loss, grad));
    if (!std::isfinite(*loss)) return firm_fail(p, FIRM_ERR_BREAKDOWN, "unrolled PCG: non-finite loss");
    return FIRM_OK;
}

firm_status firm_synth_normals(firm_plan p, uint64_t seed, uint64_t offset, int64_t n, float* out) {
    if (!p || !out || n < 0) return firm_fail(p, FIRM_ERR_ARG, "bad argument");
    FIRM_HIP(p, synth_normals(p, seed, offset, n, out));
    return FIRM_OK;
}

}  // extern "C"
